// Batched correction and serving: many fields advance together.
//
// Every field keeps its own state (Algorithm 1 run per field: own target
// set, own critical-point order, own convergence flag and counters); what is
// shared is the launch.  One iteration over the whole batch is four launches
// of persistent kernels that walk a device-resident list of work items:
//   check   (field, box) items of every unconverged field (one launch per
//           value type and dimensionality),
//   apply   (field, vertex range) items,
//   finalize one wave per field.
// Items are laid out field after field with a prefix array, so a block finds
// its field by binary search; blocks of converged fields never get items
// because the host rebuilds the lists (a few hundred bytes) between polls.
// The iterations between two polls are replayed from a captured hipGraph:
// the kernels read their item counts from device memory, so the lists can
// change between replays without a new capture.
#include <algorithm>
#include <cstring>
#include <vector>

#include "exz_host.h"
#include "loop_box.h"

namespace exz {

struct ItemList {
  uint32_t nfields;           // active fields
  uint32_t total;             // items over all active fields
  const uint32_t *field;      // [nfields] index into the FieldDev array
  const uint32_t *base;       // [nfields + 1] item prefix
};


// Check passes over the boxes of fields of one value type T.
template <class T, int TY, int TZ>
__global__ void __launch_bounds__(64 * TY)
    k_check_batch(const FieldDev *__restrict__ fields, const uint32_t *__restrict__ lists,
                  const uint32_t *__restrict__ conn) {
  __shared__ CheckLds<T, TY, TZ> L;
  load_conn(L, conn);
  const uint32_t nf = lists[0], total = lists[1];
  const uint32_t *field = lists + 2, *base = lists + 2 + nf;
  uint32_t k = 0;
  for (uint32_t it = blockIdx.x; it < total; it += gridDim.x) {
    k = next_field_uniform(base, nf, it, k);
    const FieldDev &fd = fields[__builtin_amdgcn_readfirstlane(field[k])];
    const uint32_t tile = it - base[k];
    const State *st = fd.st;
    // frontier passes skip boxes the last apply did not touch (and clear
    // the flag of those they take); every thread reads the same flag
    bool take = !st->done;
    if (take && fd.frontier && !st->dense) take = fd.bdirty[tile] != 0;
    if (take) {
      if (fd.frontier) {
        __syncthreads();  // every thread has read the flag (frontier pass)
        if (threadIdx.x == 0 && threadIdx.y == 0) fd.bdirty[tile] = 0;
      }
      // (a frontier pass tags the chunks of its marks, for the apply after it)
      if (chunk_pass(fd))
        check_box<T, TY, TZ, true>(fd, box_of(fd, tile, TY, TZ), L);
      else
        check_box<T, TY, TZ>(fd, box_of(fd, tile, TY, TZ), L);
    }
    __syncthreads();
  }
}

// Vertices of one batched apply item: item_quads quads (by default sixteen
// per thread), so the item's set-up (finding its field, reading its
// descriptor) is amortised.
constexpr uint32_t APPLY_ITEM_QUADS = 16 * APPLY_BLOCK;

// ApplyBoundedEdits: field k owns items [base[k], base[k+1]), one per
// 4 * item_quads vertices.
__global__ void __launch_bounds__(APPLY_BLOCK) k_apply_batch(const FieldDev *__restrict__ fields,
                                                             const uint32_t *__restrict__ lists,
                                                             uint32_t item_quads) {
  const uint32_t nf = lists[0], total = lists[1];
  const uint32_t *field = lists + 2, *base = lists + 2 + nf;
  // counts are added to a field's shards when the block moves on to the
  // next field (items of one field are consecutive)
  uint32_t k = 0, kc = 0;
  EditCount ec = {{0, 0, 0, 0, 0}};
  for (uint32_t it = blockIdx.x; it < total; it += gridDim.x) {
    k = next_field_uniform(base, nf, it, k);
    if (k != kc) {
      flush_counts<APPLY_BLOCK / 64>(fields[field[kc]].st, ec, blockIdx.x);
      ec = EditCount{{0, 0, 0, 0, 0}};
      kc = k;
    }
    const FieldDev &fd = fields[__builtin_amdgcn_readfirstlane(field[k])];
    if (!fd.st->done) {
      const uint32_t q0 = (it - base[k]) * item_quads;
      const uint32_t nq = min(((uint32_t)fd.n + 3) / 4, q0 + item_quads);
      if (fd.dtype == 0)
        apply_quads<float, true>(fd, q0 + threadIdx.x, APPLY_BLOCK, nq, ec);
      else
        apply_quads<double, true>(fd, q0 + threadIdx.x, APPLY_BLOCK, nq, ec);
    }
  }
  if (nf) flush_counts<APPLY_BLOCK / 64>(fields[field[kc]].st, ec, blockIdx.x);
}

// Order passes (reformulated event constraints): field k owns items
// [base[k], base[k+1]), one per ORD_ITEM ranks of its critical points.
constexpr uint32_t ORD_ITEM = 16 * 256;
__global__ void __launch_bounds__(256) k_order_batch(const FieldDev *__restrict__ fields,
                                                     const uint32_t *__restrict__ lists) {
  const uint32_t nf = lists[0], total = lists[1];
  const uint32_t *field = lists + 2, *base = lists + 2 + nf;
  uint32_t k = 0;
  for (uint32_t it = blockIdx.x; it < total; it += gridDim.x) {
    k = next_field_uniform(base, nf, it, k);
    const FieldDev &fd = fields[__builtin_amdgcn_readfirstlane(field[k])];
    if (fd.st->done) continue;
    const uint32_t r0 = (it - base[k]) * ORD_ITEM;
    const uint32_t lim = min((uint32_t)fd.K, r0 + ORD_ITEM + 1);  // the item's pairs only
    const uint32_t tag = fd.st->tag;
    // a frontier pass tests only the wave's 256 ranks whose tag is the last
    // pass's (as the single-field check does), and tags the chunks it marks
    const bool front = chunk_pass(fd);
    const uint32_t prev = tag == 1 ? MARK_TAGS : tag - 1;
    for (uint32_t j = 0; j < ORD_ITEM && r0 + j + 1 < lim; j += 1024) {
      const uint32_t rw = r0 + j + 256u * (threadIdx.x >> 6);  // this wave's first rank
      if (front && !(rw + 1 < lim && glob(fd.oflag)[rw >> 8] == prev)) continue;
      const uint32_t r = r0 + j + 4 * threadIdx.x;
      if (fd.dtype == 0) {
        if (front) order_quad<float, true>(fd, r, lim, __lane_id() != 63, tag);
        else order_quad<float>(fd, r, lim, __lane_id() != 63, tag);
      } else {
        if (front) order_quad<double, true>(fd, r, lim, __lane_id() != 63, tag);
        else order_quad<double>(fd, r, lim, __lane_id() != 63, tag);
      }
    }
  }
}

__global__ void __launch_bounds__(64) k_finalize_batch(const FieldDev *fields, const uint32_t *lists) {
  const uint32_t nf = lists[0];
  if (blockIdx.x < nf) finalize_field(fields[lists[2 + blockIdx.x]]);
}

// Gathers per-field setup results: err flags and K.
__global__ void k_gather_setup(const FieldDev *fields, uint32_t nfields, uint32_t *out) {
  const uint32_t k = blockIdx.x * 64 + threadIdx.x;
  if (k >= nfields) return;
  const FieldDev &fd = fields[k];
  out[2 * k] = fd.st->err;
  out[2 * k + 1] = fd.cpoff[fd.nchunk];
}

}  // namespace exz

// ---------------------------------------------------------------------------
// host side

using namespace exz;

namespace {

exz_status fail_b(exz_ctx *ctx, exz_status st, const char *msg) {
  if (ctx) ctx->last_error = msg;
  return st;
}

#define HIP_OR_FAIL_B(call)                                                                 \
  do {                                                                                      \
    hipError_t _e = (call);                                                                 \
    if (_e != hipSuccess) {                                                                 \
      if (ctx) ctx->last_error = std::string(#call " failed: ") + hipGetErrorString(_e);     \
      return EXZ_E_HIP;                                                                     \
    }                                                                                       \
  } while (0)

// Per-field host bookkeeping of a batch.
struct Member {
  FieldDev fd;
  int index;          // position in the caller's array
  exz_status status;  // setup errors
  bool active;
  size_t offA, offB;
  int64_t max_iters;
  bool certify;
};

}  // namespace

namespace exz {

// Launch geometry shared by all members of a batch (context options
// "btile3", "btile2", "bgrid_box", "bgrid_apply", "bitem"; 0 = default).
struct BatchShape {
  int ty3 = 4, tz3 = 8;  // boxes for 3D fields
  int ty2 = 16, tz2 = 1; // boxes for 1D/2D fields
  int grid_box = 0;      // persistent check grid cap (0: 8 work-groups per CU)
  int grid_apply = 0;    // persistent apply grid cap (0: 16 work-groups per CU)
  uint32_t item_quads = APPLY_ITEM_QUADS;  // quads per apply item
};

BatchShape batch_shape(const exz_ctx *ctx) {
  BatchShape b;
  if (ctx->btile3) {
    b.ty3 = ctx->btile3 / 100;
    b.tz3 = ctx->btile3 % 100;
  } else if (ctx->tile_y && ctx->tile_z) {  // an explicit "tile" applies to 3D members
    b.ty3 = ctx->tile_y;
    b.tz3 = ctx->tile_z;
  }
  if (ctx->btile2) {
    b.ty2 = ctx->btile2 / 100;
    b.tz2 = ctx->btile2 % 100;
  }
  b.grid_box = ctx->bgrid_box;
  b.grid_apply = ctx->bgrid_apply;
  if (ctx->bitem) b.item_quads = (uint32_t)ctx->bitem * APPLY_BLOCK;
  return b;
}

// Box geometry of a member for the batch's shape.
void batch_geometry(const BatchShape &b, FieldDev &fd) {
  const bool three = fd.nz > 1;
  fd.tile_y = three ? b.ty3 : b.ty2;
  fd.tile_z = three ? b.tz3 : b.tz2;
  fd.ty_shift = __builtin_ctz((unsigned)fd.tile_y);
  fd.tz_shift = __builtin_ctz((unsigned)fd.tile_z);
  fd.tiles_y = (fd.ny + fd.tile_y - 1) / fd.tile_y;
  fd.tiles_z = (fd.nz + fd.tile_z - 1) / fd.tile_z;
  fd.ntiles = fd.tiles_x * fd.tiles_y * fd.tiles_z;
}

// Persistent grids: enough work-groups to fill the chip, never more than
// there are items.
int batch_grid(uint64_t items, int cap, int per_cu) {
  const uint64_t c = cap > 0 ? (uint64_t)cap : (uint64_t)256 * per_cu;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(items, c));
}

// Host-built item lists for one phase, in pinned memory.
struct Lists {
  std::vector<uint32_t> v;  // [nf, total, field[nf], base[nf+1]]
  void build(const std::vector<int> &fields, const std::vector<uint32_t> &items) {
    const uint32_t nf = (uint32_t)fields.size();
    v.assign(2 + nf + nf + 1, 0);
    v[0] = nf;
    uint32_t acc = 0;
    for (uint32_t k = 0; k < nf; ++k) {
      v[2 + k] = (uint32_t)fields[k];
      v[2 + nf + k] = acc;
      acc += items[k];
    }
    v[2 + nf + nf] = acc;
    v[1] = acc;
  }
};

// Runs the batched loop over `members` (already set up, fd.st valid) until
// every member is done.  dev_fields holds the FieldDev array on the device.
exz_status run_batch_loop(exz_ctx *ctx, std::vector<Member> &members, FieldDev *dev_fields,
                          const BatchShape &shape, int max_chunks, hipStream_t s);

}  // namespace exz

// Device list buffers, capacity per list 2 + 2*nf + 1 words: boxes of 3D
// float32 / 3D float64 / 2D-1D float32 / 2D-1D float64 fields, finalize (one
// item per field), apply chunks.
enum { L_BOX3F, L_BOX3D, L_BOX2F, L_BOX2D, L_FIN, L_APPLY, L_ORD, L_EVT, NLISTS };
static size_t list_words(size_t nf) { return 2 + 2 * nf + 1; }

namespace exz {

template <class T>
static void box_launch_check(int ty, int tz, const FieldDev *fields, const uint32_t *list,
                             const uint32_t *conn, int grid, hipStream_t s) {
#define EXZ_BOX_CHECK_B(a, b)                                                                 \
  if (ty == a && tz == b)                                                                     \
    hipLaunchKernelGGL((k_check_batch<T, a, b>), dim3(grid), dim3(64, a), 0, s, fields, list, \
                       conn);
  EXZ_BOX_SHAPES(EXZ_BOX_CHECK_B)
#undef EXZ_BOX_CHECK_B
}

// Issue `iters` batched iterations.
static void issue_iterations(exz_ctx *ctx, const FieldDev *fields, uint32_t *dlists, size_t lw,
                             const BatchShape &shape, int iters, int grid_box,
                             int grid_fin, int grid_apply, int grid_ord, int grid_evt,
                             hipStream_t s) {
  const uint32_t item_quads = shape.item_quads;
  auto list = [&](int q) { return dlists + q * lw; };
  uint32_t *lf = list(L_FIN), *la = list(L_APPLY), *lo = list(L_ORD);
  for (int it = 0; it < iters; ++it) {
    box_launch_check<float>(shape.ty3, shape.tz3, fields, list(L_BOX3F), ctx->d_conn, grid_box, s);
    box_launch_check<double>(shape.ty3, shape.tz3, fields, list(L_BOX3D), ctx->d_conn, grid_box, s);
    box_launch_check<float>(shape.ty2, shape.tz2, fields, list(L_BOX2F), ctx->d_conn, grid_box, s);
    box_launch_check<double>(shape.ty2, shape.tz2, fields, list(L_BOX2D), ctx->d_conn, grid_box, s);
    // original-mode members: their event constraints on the pointers the
    // check just wrote
    if (grid_evt > 0) (void)launch_events_batch(fields, list(L_EVT), ctx->d_comp, grid_evt, s);
    hipLaunchKernelGGL(k_order_batch, dim3(grid_ord), dim3(256), 0, s, fields, lo);
    hipLaunchKernelGGL(k_apply_batch, dim3(grid_apply), dim3(APPLY_BLOCK), 0, s, fields, la,
                       item_quads);
    hipLaunchKernelGGL(k_finalize_batch, dim3(grid_fin), dim3(64), 0, s, fields, lf);
  }
}

static uint32_t apply_items(const FieldDev &fd, uint32_t item_quads);

// Host item lists of one batched iteration over the fields fds[k] with
// active[k], written into the pinned buffer hl (NLISTS lists of lw words).
static void build_lists(const std::vector<const FieldDev *> &fds, const std::vector<bool> &active,
                        uint32_t item_quads, uint32_t *hl, size_t lw) {
  std::vector<int> f[NLISTS];
  std::vector<uint32_t> n[NLISTS];
  for (size_t k = 0; k < fds.size(); ++k) {
    if (!active[k]) continue;
    const FieldDev &fd = *fds[k];
    const int idx = (int)k;
    const int box = fd.nz > 1 ? (fd.dtype == 0 ? L_BOX3F : L_BOX3D)
                              : (fd.dtype == 0 ? L_BOX2F : L_BOX2D);
    f[box].push_back(idx);
    n[box].push_back((uint32_t)fd.ntiles);
    f[L_FIN].push_back(idx);
    n[L_FIN].push_back(1);
    f[L_APPLY].push_back(idx);
    n[L_APPLY].push_back(apply_items(fd, item_quads));
    if (fd.mode != 1 && fd.K > 1) {
      f[L_ORD].push_back(idx);
      n[L_ORD].push_back(((uint32_t)fd.K - 1 + ORD_ITEM - 1) / ORD_ITEM);
    }
    if (fd.mode == 1 && fd.K > 0) {
      f[L_EVT].push_back(idx);
      n[L_EVT].push_back(((uint32_t)fd.K + EVENT_ITEM - 1) / EVENT_ITEM);
    }
  }
  for (int q = 0; q < NLISTS; ++q) {
    Lists L;
    L.build(f[q], n[q]);
    std::memcpy(hl + q * lw, L.v.data(), L.v.size() * 4);
  }
}

// Items of the apply pass of one field: 4 * item_quads vertices each.
static uint32_t apply_items(const FieldDev &fd, uint32_t item_quads) {
  const uint32_t nq = ((uint32_t)fd.n + 3) / 4;
  return (nq + item_quads - 1) / item_quads;
}

exz_status run_batch_loop(exz_ctx *ctx, std::vector<Member> &members, FieldDev *dev_fields,
                          const BatchShape &shape, int max_chunks, hipStream_t s) {
  const size_t nf = members.size();
  const size_t lw = list_words(nf);
  // device + pinned list buffers
  std::vector<uint32_t> host(NLISTS * lw, 0);
  uint32_t *dlists = nullptr, *hl = nullptr;
  State *hstates = nullptr;
  HIP_OR_FAIL_B(hipMalloc(&dlists, NLISTS * lw * sizeof(uint32_t)));
  struct Free {
    uint32_t *&d;
    uint32_t *&h;
    State *&st;
    ~Free() {
      if (d) (void)hipFree(d);
      if (h) (void)hipHostFree(h);
      if (st) (void)hipHostFree(st);
    }
  } guard{dlists, hl, hstates};
  HIP_OR_FAIL_B(hipHostMalloc((void **)&hl, NLISTS * lw * sizeof(uint32_t), hipHostMallocDefault));
  HIP_OR_FAIL_B(hipHostMalloc((void **)&hstates, std::max<size_t>(nf, 1) * sizeof(State),
                              hipHostMallocDefault));
  // persistent grids: enough blocks to fill the chip, never more than items
  uint64_t max_boxes = 0, max_apply = 0, max_ord = 0, max_evt = 0;
  for (auto &m : members) {
    max_boxes += (uint64_t)m.fd.ntiles;
    max_apply += apply_items(m.fd, shape.item_quads);
    max_ord += ((uint64_t)m.fd.K + ORD_ITEM - 1) / ORD_ITEM;
    if (m.fd.mode == 1) max_evt += ((uint64_t)m.fd.K + EVENT_ITEM - 1) / EVENT_ITEM;
  }
  const int grid_box = batch_grid(max_boxes, shape.grid_box, 8);
  const int grid_apply = batch_grid(max_apply, shape.grid_apply, 16);
  const int grid_ord = batch_grid(max_ord, 0, 8);
  const int grid_evt = max_evt ? batch_grid(max_evt, 0, 8) : 0;
  int chunk = ctx->poll > 0 ? ctx->poll : 4;
  hipGraphExec_t exec = nullptr;
  int exec_chunk = 0;
  int grid_fin = (int)nf;
  for (int round = 0; round < max_chunks; ++round) {
    // item lists over the active members
    std::vector<const FieldDev *> fds(nf);
    std::vector<bool> act(nf);
    bool any = false;
    for (size_t k = 0; k < nf; ++k) {
      fds[k] = &members[k].fd;
      act[k] = members[k].active;
      any |= act[k];
    }
    if (!any) break;
    build_lists(fds, act, shape.item_quads, hl, lw);
    HIP_OR_FAIL_B(hipMemcpyAsync(dlists, hl, NLISTS * lw * sizeof(uint32_t),
                                 hipMemcpyHostToDevice, s));
    if (ctx->graph) {
      if (!exec || exec_chunk != chunk) {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        hipGraph_t graph = nullptr;
        HIP_OR_FAIL_B(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        issue_iterations(ctx, dev_fields, dlists, lw, shape, chunk, grid_box, grid_fin,
                         grid_apply, grid_ord, grid_evt, s);
        const hipError_t ce = hipStreamEndCapture(s, &graph);  // always ends the capture
        HIP_OR_FAIL_B(ce);
        const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIP_OR_FAIL_B(e);
        exec_chunk = chunk;
      }
      HIP_OR_FAIL_B(hipGraphLaunch(exec, s));
    } else {
      issue_iterations(ctx, dev_fields, dlists, lw, shape, chunk, grid_box, grid_fin,
                         grid_apply, grid_ord, grid_evt, s);
      HIP_OR_FAIL_B(hipGetLastError());
    }
    // the members' states are consecutive (one array, slot k = member k)
    HIP_OR_FAIL_B(hipMemcpyAsync(hstates, members[0].fd.st, nf * sizeof(State),
                                 hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL_B(hipStreamSynchronize(s));
    for (size_t k = 0; k < nf; ++k) {
      if (!members[k].active) continue;
      if (hstates[k].done != RUNNING) {
        members[k].active = false;
        continue;
      }
      // every changing iteration lowers a value and a vertex moves at most
      // N + 1 times; two more passes may change nothing (frontier, then dense)
      const int64_t cap = (int64_t)(members[k].fd.N + 1) * members[k].fd.n + 4;
      if (hstates[k].passes > cap) {
        if (exec) (void)hipGraphExecDestroy(exec);
        return fail_b(ctx, EXZ_E_HIP, "batched loop did not terminate");
      }
    }
    if (ctx->poll == 0) chunk = std::min(chunk * 2, 32);
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  return EXZ_OK;
}

}  // namespace exz

namespace exz {

hipError_t ensure_work_stream(exz_ctx *ctx) {
  if (ctx->work) return hipSuccess;
  hipError_t e = hipStreamCreateWithFlags(&ctx->work, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  e = hipEventCreateWithFlags(&ctx->order_in, hipEventDisableTiming);
  if (e != hipSuccess) return e;
  return hipEventCreateWithFlags(&ctx->order_out, hipEventDisableTiming);
}

// The side streams start after everything issued so far on s ...
static hipError_t side_fork(exz_ctx *ctx, hipStream_t s) {
  for (int j = 0; j < exz_ctx::NSIDE; ++j) {
    if (!ctx->side[j]) {
      const hipError_t e = hipStreamCreateWithFlags(&ctx->side[j], hipStreamNonBlocking);
      if (e != hipSuccess) return e;
    }
  }
  for (int j = 0; j <= exz_ctx::NSIDE; ++j) {
    if (!ctx->side_ev[j]) {
      const hipError_t e = hipEventCreateWithFlags(&ctx->side_ev[j], hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
  }
  hipError_t e = hipEventRecord(ctx->side_ev[exz_ctx::NSIDE], s);
  for (int j = 0; j < exz_ctx::NSIDE && e == hipSuccess; ++j)
    e = hipStreamWaitEvent(ctx->side[j], ctx->side_ev[exz_ctx::NSIDE], 0);
  return e;
}

// ... and s continues after everything issued on them.
static hipError_t side_join(exz_ctx *ctx, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (int j = 0; j < exz_ctx::NSIDE && e == hipSuccess; ++j) {
    e = hipEventRecord(ctx->side_ev[j], ctx->side[j]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, ctx->side_ev[j], 0);
  }
  return e;
}

}  // namespace exz

extern "C" {

exz_status exz_correct_batch(exz_ctx *ctx, const exz_field *fields, int32_t nfields,
                             exz_result *results, void *stream) {
  if (!ctx || nfields < 0 || (nfields > 0 && (!fields || !results))) return EXZ_E_INVALID;
  if (ctx->busy) return fail_b(ctx, EXZ_E_BUSY, "context busy");
  ctx->busy = true;
  struct Unbusy {
    exz_ctx *c;
    ~Unbusy() { c->busy = false; }
  } unbusy{ctx};
  ctx->last_error.clear();
  HIP_OR_FAIL_B(hipSetDevice(ctx->device));
  // The iterations are captured into a graph, which HIP does not allow on the
  // legacy default stream: run on the context's own stream, ordered after the
  // caller's stream (the call returns only when the work is done).
  HIP_OR_FAIL_B(ensure_work_stream(ctx));
  HIP_OR_FAIL_B(hipEventRecord(ctx->order_in, (hipStream_t)stream));
  HIP_OR_FAIL_B(hipStreamWaitEvent(ctx->work, ctx->order_in, 0));
  hipStream_t s = ctx->work;
  exz_status first_err = EXZ_OK;
  for (int k = 0; k < nfields; ++k) {
    std::memset(&results[k], 0, sizeof(exz_result));
    results[k].certified = -1;
  }
  std::vector<Member> mem;
  const BatchShape shape = batch_shape(ctx);
  for (int k = 0; k < nfields; ++k) {
    const exz_field &fl = fields[k];
    Member m;
    m.index = k;
    m.status = prepare_field(ctx, &fl.params, m.fd);
    if (m.status == EXZ_OK && (!fl.f || !fl.g_hat || !fl.g_out))
      m.status = fail_b(ctx, EXZ_E_INVALID, "null field pointer");
    if (m.status == EXZ_OK && fl.params.resume && !fl.cnt_io)
      m.status = fail_b(ctx, EXZ_E_INVALID, "resume needs cnt_io");
    if (m.status != EXZ_OK) {
      results[k].status = m.status;
      if (first_err == EXZ_OK) first_err = m.status;
      continue;
    }
    // box shape of the batch for this field's dimensionality
    batch_geometry(shape, m.fd);
    m.fd.f = fl.f;
    m.fd.g_hat = fl.g_hat;
    m.fd.g = fl.g_out;
    m.max_iters = fl.params.max_iters;
    m.certify = fl.params.certify != 0;
    m.active = true;
    mem.push_back(m);
  }
  const size_t nb = mem.size();
  if (nb) {
    hipEvent_t e0, e1, e2;
    HIP_OR_FAIL_B(hipEventCreate(&e0));
    HIP_OR_FAIL_B(hipEventCreate(&e1));
    HIP_OR_FAIL_B(hipEventCreate(&e2));
    HIP_OR_FAIL_B(hipEventRecord(e0, s));
    // phase A workspaces and states, one allocation
    Layout LA;
    std::vector<size_t[9]> oa(nb);
    std::vector<size_t> baseA(nb);
    for (size_t k = 0; k < nb; ++k) {
      Layout L;
      layout_a(mem[k].fd, fields[mem[k].index].cnt_io == nullptr, 0, false, L, oa[k]);
      baseA[k] = LA.add(L.total);
    }
    const size_t st_off = LA.add(nb * sizeof(State));
    const size_t fd_off = LA.add(nb * sizeof(FieldDev));
    const size_t gather_off = LA.add(nb * 2 * sizeof(uint32_t));
    HIP_OR_FAIL_B(ctx->BA.reserve(LA.total));
    char *A = (char *)ctx->BA.take(LA.total);
    State *states = (State *)(A + st_off);
    FieldDev *dev_fields = (FieldDev *)(A + fd_off);
    uint32_t *gather = (uint32_t *)(A + gather_off);
    // fields are set up independently (own workspace), spread over the
    // side streams so that their many small kernels overlap
    HIP_OR_FAIL_B(side_fork(ctx, s));
    for (size_t k = 0; k < nb; ++k) {
      hipStream_t sk = ctx->side[k % exz_ctx::NSIDE];
      FieldDev &fd = mem[k].fd;
      char *b = A + baseA[k];
      fd.st = states + k;
      fd.low = (uint16_t *)(b + oa[k][1]);
      fd.code = (uint8_t *)(b + oa[k][1] + 2 * (size_t)fd.n);
      fd.cpbits = (unsigned long long *)(b + oa[k][2]);
      fd.cpoff = (uint32_t *)(b + oa[k][3]);
      fd.tmark = (uint8_t *)(b + oa[k][4]);
      fd.mchunk = fd.tmark + mark_pad_bytes(fd);
      fd.fe = (uint8_t *)(b + oa[k][5]);
      fd.bdirty = (uint8_t *)(b + oa[k][8]);
      fd.blist = box_list_of(fd, b + oa[k][8]);
      uint8_t *cnt_io = fields[mem[k].index].cnt_io;
      fd.cnt = cnt_io ? cnt_io : (uint8_t *)(b + oa[k][6]);
      fd.vec = quad_aligned(fd);
      uint32_t *scan_tmp = (uint32_t *)(b + oa[k][7]);
      HIP_OR_FAIL_B(launch_state_reset(fd, mem[k].max_iters, sk));
      HIP_OR_FAIL_B(launch_setup(fd, ctx->d_conn, sk));
      HIP_OR_FAIL_B(launch_scan_u32(fd.cpoff, fd.cpoff, (uint32_t)fd.nchunk, scan_tmp,
                                    scan_tmp_words((uint32_t)fd.nchunk), sk));
    }
    HIP_OR_FAIL_B(side_join(ctx, s));
    std::vector<FieldDev> host_fd(nb);
    for (size_t k = 0; k < nb; ++k) host_fd[k] = mem[k].fd;
    HIP_OR_FAIL_B(hipMemcpyAsync(dev_fields, host_fd.data(), nb * sizeof(FieldDev),
                                 hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_gather_setup, dim3((unsigned)((nb + 63) / 64)), dim3(64), 0, s, dev_fields,
                       (uint32_t)nb, gather);
    std::vector<uint32_t> hg(2 * nb);
    HIP_OR_FAIL_B(hipMemcpyAsync(hg.data(), gather, 2 * nb * sizeof(uint32_t),
                                 hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL_B(hipStreamSynchronize(s));
    // phase B
    Layout LB;
    std::vector<size_t[12]> ob(nb);
    std::vector<size_t> baseB(nb);
    for (size_t k = 0; k < nb; ++k) {
      Member &m = mem[k];
      const uint32_t err = hg[2 * k];
      if (err & ERR_NONFINITE) m.status = EXZ_E_NONFINITE;
      else if (err & ERR_BOUND) m.status = EXZ_E_BOUND;
      if (m.status != EXZ_OK) {
        m.active = false;
        results[m.index].status = m.status;
        if (first_err == EXZ_OK) {
          first_err = m.status;
          ctx->last_error = exz_status_string(m.status);
        }
        continue;
      }
      m.fd.K = (int32_t)hg[2 * k + 1];
      Layout L;
      layout_b(m.fd, (uint32_t)m.fd.K, L, ob[k]);
      baseB[k] = LB.add(L.total);
    }
    // The critical points of all members with keys of one width are sorted
    // together (see SortTile): a few launches per pass for the whole batch
    // instead of twenty per member.  A group whose counts would not fit 32
    // bits sorts member by member.
    struct SortGroup {
      uint64_t total = 0, tiles = 0;
      std::vector<SortTile> desc;
      size_t keys = 0, keys_tmp = 0, vals = 0, vals_tmp = 0, hist = 0, scan = 0, tdesc = 0;
      bool on = false;
    } grp[2];
    std::vector<uint32_t> start(nb, 0);
    for (size_t k = 0; k < nb; ++k) {
      const Member &m = mem[k];
      if (!m.active || m.fd.K <= 0) continue;
      SortGroup &g = grp[m.fd.dtype == 0 ? 0 : 1];
      const uint32_t K = (uint32_t)m.fd.K, nt = (K + SORT_TILE - 1) / SORT_TILE;
      start[k] = (uint32_t)g.total;
      for (uint32_t t = 0; t < nt; ++t)
        g.desc.push_back(SortTile{(uint32_t)g.total + t * SORT_TILE,
                                  std::min(SORT_TILE, K - t * SORT_TILE),
                                  (uint32_t)(256 * g.tiles), nt, t});
      g.total += K;
      g.tiles += nt;
    }
    for (int gi = 0; gi < 2; ++gi) {
      SortGroup &g = grp[gi];
      const size_t kb = gi == 0 ? 4 : 8;
      g.on = g.total > 0 && g.total < (1ull << 31) && 256 * g.tiles < (1ull << 31);
      if (!g.on) continue;
      g.keys = LB.add(kb * g.total);
      g.keys_tmp = LB.add(kb * g.total);
      g.vals = LB.add(4 * g.total);
      g.vals_tmp = LB.add(4 * g.total);
      g.hist = LB.add(4 * (256 * g.tiles + 1));
      g.scan = LB.add(4 * scan_tmp_words((uint32_t)(256 * g.tiles)));
      g.tdesc = LB.add(sizeof(SortTile) * g.tiles);
    }
    HIP_OR_FAIL_B(ctx->BB.reserve(LB.total ? LB.total : 256));
    char *Bm = (char *)ctx->BB.take(LB.total);
    HIP_OR_FAIL_B(side_fork(ctx, s));
    for (size_t k = 0; k < nb; ++k) {
      Member &m = mem[k];
      hipStream_t sk = ctx->side[k % exz_ctx::NSIDE];
      if (!m.active) continue;
      FieldDev &fd = m.fd;
      char *b = Bm + baseB[k];
      const uint32_t K = (uint32_t)fd.K;
      fd.cp_rank = (uint32_t *)(b + ob[k][0]);
      fd.cp_below = fd.cp_rank + (K ? K : 1);
      fd.oflag = (uint8_t *)(fd.cp_below + ((K ? K : 1) + 31) / 32);
      fd.cp_vtx = (uint32_t *)(b + ob[k][1]);
      fd.cp_idx = (uint32_t *)(b + ob[k][3]);
      fd.cpr = b + ob[k][4];
      if (K == 0) continue;
      const SortGroup &g = grp[fd.dtype == 0 ? 0 : 1];
      if (g.on) {  // into the group's arrays; sorted below
        const size_t kb = fd.dtype == 0 ? 4 : 8;
        HIP_OR_FAIL_B(launch_cp_compact(fd, ctx->d_comp, Bm + g.keys + kb * start[k],
                                        (uint32_t *)(Bm + g.vals) + start[k], sk));
      } else {
        const size_t hw = radix_hist_words(K);
        HIP_OR_FAIL_B(launch_cp_compact(fd, ctx->d_comp, b + ob[k][5], (uint32_t *)(b + ob[k][7]), sk));
        HIP_OR_FAIL_B(launch_radix_sort(fd.dtype == 0 ? 4 : 8, b + ob[k][5], (uint32_t *)(b + ob[k][7]),
                                        b + ob[k][6], (uint32_t *)(b + ob[k][8]), K,
                                        (uint32_t *)(b + ob[k][9]), (uint32_t *)(b + ob[k][10]),
                                        scan_tmp_words((uint32_t)(hw - 1)), sk));
        HIP_OR_FAIL_B(launch_cp_init(fd, (uint32_t *)(b + ob[k][7]), sk));
      }
    }
    if (grp[0].on || grp[1].on) {
      HIP_OR_FAIL_B(side_join(ctx, s));
      for (int gi = 0; gi < 2; ++gi) {
        const SortGroup &g = grp[gi];
        if (!g.on) continue;
        HIP_OR_FAIL_B(hipMemcpyAsync(Bm + g.tdesc, g.desc.data(), sizeof(SortTile) * g.tiles,
                                     hipMemcpyHostToDevice, s));
        HIP_OR_FAIL_B(launch_radix_sort_tiles(
            gi == 0 ? 4 : 8, Bm + g.keys, (uint32_t *)(Bm + g.vals), Bm + g.keys_tmp,
            (uint32_t *)(Bm + g.vals_tmp), (uint32_t)g.total, (const SortTile *)(Bm + g.tdesc),
            (uint32_t)g.tiles, (uint32_t *)(Bm + g.hist), (uint32_t *)(Bm + g.scan),
            scan_tmp_words((uint32_t)(256 * g.tiles)), s));
      }
      HIP_OR_FAIL_B(side_fork(ctx, s));
      for (size_t k = 0; k < nb; ++k) {
        const Member &m = mem[k];
        if (!m.active || m.fd.K <= 0) continue;
        const SortGroup &g = grp[m.fd.dtype == 0 ? 0 : 1];
        if (g.on)
          HIP_OR_FAIL_B(launch_cp_init(m.fd, (uint32_t *)(Bm + g.vals) + start[k],
                                       ctx->side[k % exz_ctx::NSIDE]));
      }
    }
    for (size_t k = 0; k < nb; ++k)
      if (mem[k].active) host_fd[k] = mem[k].fd;
    // original-mode members: path workspace (f's and g's labels, saddle
    // order, f's selections; the certificate's labels too) and its set-up,
    // on the member's side stream after its critical points
    Layout LP;
    std::vector<size_t[6]> op(nb);
    std::vector<size_t> baseP(nb, 0);
    for (size_t k = 0; k < nb; ++k) {
      if (!mem[k].active || mem[k].fd.mode != 1) continue;
      Layout L;
      layout_c(mem[k].fd, true, mem[k].certify, L, op[k]);
      baseP[k] = LP.add(L.total);
    }
    if (LP.total) {
      HIP_OR_FAIL_B(ctx->BC.reserve(LP.total));
      char *Pm = (char *)ctx->BC.take(LP.total);
      for (size_t k = 0; k < nb; ++k) {
        Member &m = mem[k];
        if (!m.active || m.fd.mode != 1) continue;
        hipStream_t sk = ctx->side[k % exz_ctx::NSIDE];
        FieldDev &fd = m.fd;
        char *cb = Pm + baseP[k];
        fd.lab_f = (uint32_t *)(cb + op[k][0]);
        fd.lab = (uint32_t *)(cb + op[k][1]);
        fd.sad_rank = (uint32_t *)(cb + op[k][2]);
        fd.sel_f = (uint32_t *)(cb + op[k][3]);
        HIP_OR_FAIL_B(launch_original_setup(fd, ctx->d_comp, (uint32_t *)(cb + op[k][4]),
                                            (uint32_t *)(cb + op[k][5]),
                                            scan_tmp_words((uint32_t)(fd.K ? fd.K : 1)), sk));
        host_fd[k] = fd;
      }
    }
    HIP_OR_FAIL_B(side_join(ctx, s));
    HIP_OR_FAIL_B(hipMemcpyAsync(dev_fields, host_fd.data(), nb * sizeof(FieldDev),
                                 hipMemcpyHostToDevice, s));
    HIP_OR_FAIL_B(hipEventRecord(e1, s));
    std::vector<Member> run;
    for (auto &m : mem)
      if (m.active) run.push_back(m);
    // run only the live members, but index the device array by batch slot
    for (auto &m : mem) m.active = m.active;  // (kept for clarity)
    {
      std::vector<Member> all = mem;  // slot k == device index k
      const exz_status ls = run_batch_loop(ctx, all, dev_fields, shape, 1 << 30, s);
      // (the loop stops each member at its own pass cap)
      if (ls != EXZ_OK) return ls;
    }
    // certificates, then results
    for (size_t k = 0; k < nb; ++k) {
      Member &m = mem[k];
      if (m.status != EXZ_OK || !m.certify) continue;
      uint32_t *lab_g = nullptr;
      FieldDev fd = m.fd;
      if (fd.mode == 1) {
        lab_g = fd.lab;  // its path workspace holds the certificate's labels
      } else {
        const exz_status cs = setup_paths(ctx, fd, false, true, ctx->C, &lab_g, s);
        if (cs != EXZ_OK) return cs;
      }
      HIP_OR_FAIL_B(launch_certify(fd, ctx->d_comp, lab_g, s));
      HIP_OR_FAIL_B(hipStreamSynchronize(s));
    }
    HIP_OR_FAIL_B(hipEventRecord(e2, s));
    std::vector<State> hs(nb);
    HIP_OR_FAIL_B(hipMemcpyAsync(hs.data(), states, nb * sizeof(State), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL_B(hipStreamSynchronize(s));
    float setup_ms = 0, loop_ms = 0;
    (void)hipEventElapsedTime(&setup_ms, e0, e1);
    (void)hipEventElapsedTime(&loop_ms, e1, e2);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    for (size_t k = 0; k < nb; ++k) {
      Member &m = mem[k];
      if (m.status != EXZ_OK) continue;
      exz_result &r = results[m.index];
      const State &st = hs[k];
      r.iterations = st.iterations;
      r.edited_vertices = st.edited_total;
      r.targets_total = st.targets_total;
      r.edit_ops = st.edit_ops;
      r.lossless_vertices = st.lossless_total;
      r.floor_vertices = st.floor_total;
      r.residual_violations = st.residual;
      r.num_critical = m.fd.K;
      r.status = st.done == STUCK ? EXZ_W_STUCK : st.done == MAXITERS ? EXZ_W_MAX_ITERS : EXZ_OK;
      if (m.certify) r.certified = st.cert_bad == 0 ? 1 : 0;
      r.setup_ms = setup_ms;  // batch-wide device times
      r.loop_ms = loop_ms;
    }
  }
  return first_err;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// serving primitives: jobs advanced together by exz_step

extern "C" {

size_t exz_job_bytes(const exz_params *params) {
  if (!params || params->event_mode != EXZ_EVENT_REFORMULATED) return 0;
  return exz_workspace_bytes(params);
}

}  // extern "C"

namespace {

bool event_ended(hipEvent_t e) { return !e || hipEventQuery(e) != hipErrorNotReady; }

// Every event recorded for the job has completed: no device work of it is
// left (a step's state copy follows that step's kernels).
bool job_quiet(const exz_job *job) {
  if (!event_ended(job->a_done) || !event_ended(job->ready)) return false;
  for (int s = 0; s < exz_job::NSTATE; ++s)
    if (job->recorded[s] && !event_ended(job->polled[s])) return false;
  return true;
}

// (the job's work has ended: its events and pinned block go to the
// context's spares, its arenas to the pool)
void free_job(exz_job *job) {
  exz_ctx *ctx = job->ctx;
  auto spare_event = [&](hipEvent_t e) {
    if (!e) return;
    if (ctx->spare_events.size() < exz_ctx::SPARE_JOBS * (2 + exz_job::NSTATE))
      ctx->spare_events.push_back(e);
    else
      (void)hipEventDestroy(e);
  };
  for (hipEvent_t e : {job->ready, job->a_done}) spare_event(e);
  for (hipEvent_t e : job->polled) spare_event(e);
  job->A.release();
  job->B.release();
  if (job->pinned) {
    if (ctx->spare_pinned.size() < exz_ctx::SPARE_JOBS)
      ctx->spare_pinned.push_back(job->pinned);
    else
      (void)hipHostFree(job->pinned);
  }
  delete job;
}

// Frees the released jobs whose device work has ended.
void reap(exz_ctx *ctx) {
  auto &g = ctx->graveyard;
  for (size_t k = 0; k < g.size();) {
    if (job_quiet(g[k])) {
      free_job(g[k]);
      g[k] = g.back();
      g.pop_back();
    } else {
      ++k;
    }
  }
}

// A submitted job whose phase A has ended: check the validation flags and
// issue phase B on its creation stream (or mark the job failed).  Nothing
// happens while phase A runs.
exz_status job_advance(exz_job *job) {
  if (job->phase != 0) return EXZ_OK;
  const hipError_t q = hipEventQuery(job->a_done);
  if (q == hipErrorNotReady) return EXZ_OK;
  exz_ctx *ctx = job->ctx;
  exz_status st = EXZ_OK;
  const exz::State &hs = job->pinned->st[0];
  if (q != hipSuccess) {
    st = fail_b(ctx, EXZ_E_HIP, "job set-up failed on the device");
  } else if (hs.err & ERR_NONFINITE) {
    st = fail_b(ctx, EXZ_E_NONFINITE, "NaN or Inf in f or g_hat");
  } else if (hs.err & ERR_BOUND) {
    st = fail_b(ctx, EXZ_E_BOUND, "g_hat outside [f - xi, f + xi]");
  } else {
    st = setup_phase_b(ctx, job->fd, job->pinned->k, job->B, job->create_stream);
    if (st == EXZ_OK && hipEventRecord(job->ready, job->create_stream) != hipSuccess)
      st = fail_b(ctx, EXZ_E_HIP, "hipEventRecord failed");
  }
  if (st != EXZ_OK) {
    job->phase = 2;
    job->failed = st;
    job->failed_msg = ctx->last_error;
    return st;
  }
  job->result.num_critical = job->fd.K;
  job->phase = 1;
  return EXZ_OK;
}

// Phase A of a new job on `stream` (validation, reference topology, the
// critical-point bitmask); *out gets a job in phase 0.
exz_status job_begin(exz_ctx *ctx, const exz_field *field, void *stream, exz_job **out) {
  if (!ctx || !field || !out) return EXZ_E_INVALID;
  *out = nullptr;
  if (field->params.event_mode != EXZ_EVENT_REFORMULATED)
    return fail_b(ctx, EXZ_E_INVALID, "jobs run the reformulated event constraints only");
  if (!field->f || !field->g_hat || !field->g_out)
    return fail_b(ctx, EXZ_E_INVALID, "null field pointer");
  if (field->params.resume && !field->cnt_io)
    return fail_b(ctx, EXZ_E_INVALID, "resume needs cnt_io");
  HIP_OR_FAIL_B(hipSetDevice(ctx->device));
  reap(ctx);
  exz_job *job = new exz_job();
  job->ctx = ctx;
  job->A.budget = job->B.budget = &ctx->budget;  // the job's workspace counts against the budget
  job->A.exact = job->B.exact = true;             // exact sizes, handed to the pool when freed
  job->A.pool = job->B.pool = &ctx->job_pool;
  job->params = field->params;
  std::memset(&job->result, 0, sizeof job->result);
  job->result.certified = -1;
  job->create_stream = (hipStream_t)stream;
  job->last = (hipStream_t)stream;
  job->phase = 0;
  exz_status st = EXZ_OK;
  if (!ctx->spare_pinned.empty()) {  // a freed job's block (its work has ended)
    job->pinned = (exz_job::Pinned *)ctx->spare_pinned.back();
    ctx->spare_pinned.pop_back();
  } else if (hipHostMalloc((void **)&job->pinned, sizeof(exz_job::Pinned), hipHostMallocDefault) !=
             hipSuccess) {
    job->pinned = nullptr;
    st = fail_b(ctx, EXZ_E_NOMEM, "hipHostMalloc failed");
  }
  std::vector<hipEvent_t *> evs = {&job->a_done, &job->ready};
  for (hipEvent_t &e : job->polled) evs.push_back(&e);
  for (hipEvent_t *e : evs) {
    if (st != EXZ_OK) break;
    if (!ctx->spare_events.empty()) {  // completed events of freed jobs
      *e = ctx->spare_events.back();
      ctx->spare_events.pop_back();
    } else if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
      *e = nullptr;
      st = fail_b(ctx, EXZ_E_HIP, "hipEventCreateWithFlags failed");
    }
  }
  if (st == EXZ_OK) st = prepare_field(ctx, &field->params, job->fd);
  if (st == EXZ_OK) {
    FieldDev &fd = job->fd;
    batch_geometry(batch_shape(ctx), fd);  // the boxes of the batched launches
    st = setup_phase_a(ctx, fd, field->f, field->g_hat, field->g_out, field->cnt_io,
                       field->params.max_iters, job->A, (hipStream_t)stream, &job->pinned->st[0],
                       &job->pinned->k);
  }
  if (st == EXZ_OK && hipEventRecord(job->a_done, (hipStream_t)stream) != hipSuccess)
    st = fail_b(ctx, EXZ_E_HIP, "hipEventRecord failed");
  if (st != EXZ_OK) {
    (void)hipStreamSynchronize((hipStream_t)stream);  // work issued before the failure
    free_job(job);
    return st;
  }
  *out = job;
  return EXZ_OK;
}

}  // namespace

void free_graveyard(exz_ctx *ctx) {
  for (exz_job *j : ctx->graveyard) free_job(j);
  ctx->graveyard.clear();
  for (void *p : ctx->spare_pinned) (void)hipHostFree(p);
  ctx->spare_pinned.clear();
  for (hipEvent_t e : ctx->spare_events) (void)hipEventDestroy(e);
  ctx->spare_events.clear();
}

extern "C" {

exz_status exz_job_create(exz_ctx *ctx, const exz_field *field, void *stream, exz_job **out) {
  exz_job *job = nullptr;
  exz_status st = job_begin(ctx, field, stream, &job);
  if (st != EXZ_OK) return st;
  // wait for phase A: validation errors are returned here
  if (hipEventSynchronize(job->a_done) != hipSuccess) {
    free_job(job);
    return fail_b(ctx, EXZ_E_HIP, "hipEventSynchronize failed");
  }
  st = job_advance(job);
  if (st != EXZ_OK) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    free_job(job);
    return st;
  }
  *out = job;
  return EXZ_OK;
}

exz_status exz_job_submit(exz_ctx *ctx, const exz_field *field, void *stream, exz_job **out) {
  return job_begin(ctx, field, stream, out);
}

exz_status exz_step(exz_ctx *ctx, exz_job *const *jobs, int32_t njobs, int32_t iters,
                    void *stream) {
  if (!ctx || njobs < 0 || iters < 1 || (njobs > 0 && !jobs)) return EXZ_E_INVALID;
  if (njobs == 0) return EXZ_OK;
  hipStream_t s = (hipStream_t)stream;
  HIP_OR_FAIL_B(hipSetDevice(ctx->device));
  reap(ctx);
  // the jobs that are set up take part; a submitted job whose phase A has
  // ended gets its phase B issued now (failed ones and those still in phase
  // A sit this step out)
  std::vector<exz_job *> in;
  in.reserve((size_t)njobs);
  for (int32_t k = 0; k < njobs; ++k) {
    if (!jobs[k]) return fail_b(ctx, EXZ_E_INVALID, "null job");
    (void)job_advance(jobs[k]);
    if (jobs[k]->phase == 1) in.push_back(jobs[k]);
  }
  if (in.empty()) return EXZ_OK;
  const size_t nf = in.size();
  const size_t lw = list_words(nf);
  const size_t bytes = nf * sizeof(FieldDev) + NLISTS * lw * sizeof(uint32_t);
  // staging of the previous step must have been consumed before reuse
  if (ctx->step_copied) HIP_OR_FAIL_B(hipEventSynchronize(ctx->step_copied));
  else HIP_OR_FAIL_B(hipEventCreateWithFlags(&ctx->step_copied, hipEventDisableTiming));
  if (bytes > ctx->step_cap) {
    if (ctx->step_host) (void)hipHostFree(ctx->step_host);
    if (ctx->step_dev) (void)hipFree(ctx->step_dev);
    ctx->step_host = nullptr;
    ctx->step_dev = nullptr;
    ctx->step_cap = 0;
    HIP_OR_FAIL_B(hipHostMalloc(&ctx->step_host, bytes * 2, hipHostMallocDefault));
    HIP_OR_FAIL_B(hipMalloc(&ctx->step_dev, bytes * 2));
    ctx->step_cap = bytes * 2;
  }
  FieldDev *hf = (FieldDev *)ctx->step_host;
  uint32_t *hl = (uint32_t *)(hf + nf);
  // launch geometry: the jobs' own boxes (fixed when they were created), the
  // context's grid caps and apply item size
  BatchShape shape = batch_shape(ctx);
  bool have3 = false, have2 = false;
  for (size_t k = 0; k < nf; ++k) {
    const FieldDev &fd = in[k]->fd;
    int &ty = fd.nz > 1 ? shape.ty3 : shape.ty2, &tz = fd.nz > 1 ? shape.tz3 : shape.tz2;
    bool &have = fd.nz > 1 ? have3 : have2;
    if (!have) {
      ty = fd.tile_y;
      tz = fd.tile_z;
      have = true;
    } else if (ty != fd.tile_y || tz != fd.tile_z) {
      return fail_b(ctx, EXZ_E_INVALID, "jobs of one step must share their box shape");
    }
  }
  uint64_t boxes = 0, words = 0, ords = 0;
  std::vector<const FieldDev *> fds(nf);
  std::vector<bool> act(nf, true);
  // Stream order: this step starts after the previous step (which read the
  // device copy of the descriptors that is rewritten below, maybe on another
  // stream) and after the set-up of every job it takes for the first time.
  if (ctx->step_done) HIP_OR_FAIL_B(hipStreamWaitEvent(s, ctx->step_done, 0));
  else HIP_OR_FAIL_B(hipEventCreateWithFlags(&ctx->step_done, hipEventDisableTiming));
  for (size_t k = 0; k < nf; ++k) {
    exz_job *job = in[k];
    if (!job->joined) {
      HIP_OR_FAIL_B(hipStreamWaitEvent(s, job->ready, 0));
      job->joined = true;
    }
    hf[k] = job->fd;
    const FieldDev &fd = hf[k];
    fds[k] = &hf[k];
    words += apply_items(fd, shape.item_quads);
    boxes += (uint64_t)fd.ntiles;
    ords += ((uint64_t)fd.K + ORD_ITEM - 1) / ORD_ITEM;
    job->last = s;
  }
  build_lists(fds, act, shape.item_quads, hl, lw);
  FieldDev *df = (FieldDev *)ctx->step_dev;
  uint32_t *dl = (uint32_t *)(df + nf);
  HIP_OR_FAIL_B(hipMemcpyAsync(df, hf, bytes, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL_B(hipEventRecord(ctx->step_copied, s));
  const int grid_box = batch_grid(boxes, shape.grid_box, 8);
  const int grid_apply = batch_grid(words, shape.grid_apply, 16);
  const int grid_ord = batch_grid(ords, 0, 8);
  issue_iterations(ctx, df, dl, lw, shape, iters, grid_box, (int)nf, grid_apply, grid_ord, 0, s);
  HIP_OR_FAIL_B(hipGetLastError());
  // each job's state after the step, into the next of its host slots, for
  // exz_job_query (which reads the latest slot whose copy has ended)
  for (exz_job *job : in) {
    const int slot = (job->slot + 1) % exz_job::NSTATE;
    HIP_OR_FAIL_B(hipMemcpyAsync(&job->pinned->st[slot], job->fd.st, sizeof(exz::State),
                                 hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL_B(hipEventRecord(job->polled[slot], s));
    job->recorded[slot] = true;
    job->slot = slot;
  }
  HIP_OR_FAIL_B(hipEventRecord(ctx->step_done, s));
  return EXZ_OK;
}

}  // extern "C"

namespace {

// The result fields of a job from a copy of its device state.
void fill_result(exz_job *job, const exz::State &hs, int32_t *done, exz_result *result) {
  *done = hs.done != RUNNING;
  exz_result &r = job->result;
  r.iterations = hs.iterations;
  r.edited_vertices = hs.edited_total;
  r.targets_total = hs.targets_total;
  r.edit_ops = hs.edit_ops;
  r.lossless_vertices = hs.lossless_total;
  r.floor_vertices = hs.floor_total;
  r.residual_violations = hs.residual;
  r.status = hs.done == STUCK ? EXZ_W_STUCK : hs.done == MAXITERS ? EXZ_W_MAX_ITERS : EXZ_OK;
  if (result) *result = r;
}

exz_status job_failure(exz_job *job, int32_t *done) {
  *done = 1;
  job->ctx->last_error = job->failed_msg;
  return job->failed;
}

}  // namespace

extern "C" {

exz_status exz_job_poll(exz_job *job, int32_t *done, exz_result *result) {
  if (!job || !done) return EXZ_E_INVALID;
  exz_ctx *ctx = job->ctx;
  HIP_OR_FAIL_B(hipSetDevice(ctx->device));
  if (job->phase == 0) {  // a submitted job: finish its set-up first
    HIP_OR_FAIL_B(hipEventSynchronize(job->a_done));
    (void)job_advance(job);
  }
  if (job->phase == 2) return job_failure(job, done);
  State hs;
  HIP_OR_FAIL_B(hipMemcpyAsync(&hs, job->fd.st, sizeof(State), hipMemcpyDeviceToHost, job->last));
  HIP_OR_FAIL_B(hipStreamSynchronize(job->last));
  fill_result(job, hs, done, result);
  return EXZ_OK;
}

exz_status exz_job_query(exz_job *job, int32_t *done, exz_result *result) {
  if (!job || !done) return EXZ_E_INVALID;
  *done = 0;
  exz_ctx *ctx = job->ctx;
  HIP_OR_FAIL_B(hipSetDevice(ctx->device));
  (void)job_advance(job);
  if (job->phase == 2) return job_failure(job, done);
  if (job->phase == 0 || job->slot < 0) return EXZ_OK;  // not stepped yet
  for (int t = 0, s = job->slot; t < exz_job::NSTATE;
       ++t, s = (s + exz_job::NSTATE - 1) % exz_job::NSTATE) {
    if (!job->recorded[s]) continue;
    const hipError_t q = hipEventQuery(job->polled[s]);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return fail_b(ctx, EXZ_E_HIP, "hipEventQuery failed");
    fill_result(job, job->pinned->st[s], done, result);
    return EXZ_OK;
  }
  return EXZ_OK;
}

exz_status exz_job_release(exz_job *job) {
  if (!job) return EXZ_OK;
  exz_ctx *ctx = job->ctx;
  (void)hipSetDevice(ctx->device);
  // the workspace goes back once the device is done with it
  if (job_quiet(job)) free_job(job);
  else ctx->graveyard.push_back(job);
  reap(ctx);
  return EXZ_OK;
}

}  // extern "C"
