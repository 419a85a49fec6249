// One iteration of the correction loop (Algorithm 1) on the device:
//   check     CheckConstraints (Sec. 4.2): steepest ascent and descent
//             neighbours of g against f, link order of saddles (and of
//             regular vertices of f that g turned into saddles), and the
//             reformulated event constraints (Sec. 4.3): each critical point
//             of f against the next one in f's order, whose value is
//             gathered from g.  Each vertex marks the vertices it asks to
//             decrease (its neighbours or itself) in a byte per vertex, the
//             target set S;
//   apply     ApplyBoundedEdits (Sec. 3.3): every marked vertex is edited in
//             place and its mark cleared;
//   finalize  convergence / stuck / iteration-cap decision, counter reset.
// A mark is a plain store of 1: many checks may mark the same vertex, and
// every such store leaves the same byte, so no atomics are needed.  All
// checks of an iteration read the same g, and the edits run in a later
// launch (synchronous, Jacobi-style rounds).  Every kernel returns at once
// when the field is already done, so a host may issue more iterations than
// needed and poll rarely.
//
// check is a stencil over the 14-neighbour Freudenthal mesh.  A work-group
// owns a 64 x TY x TZ box of vertices; it stages the box plus a one-cell
// halo row by row (coalesced loads, many in flight per thread) into LDS, and
// each thread evaluates TZ vertices of one (x, y) column from LDS.  Halo
// re-reads are served by L2: consecutive boxes run on the same XCD.  With
// frontier passes, apply flags the boxes whose check reads a value it
// changed: the boxes around the vertex, and the box of the previous critical
// point in f's order, which compares itself with the vertex.  The next check
// visits only flagged boxes; a pass that changes nothing is followed by one
// dense pass before the loop may stop, so the decision always rests on a
// check of every vertex.
#include <algorithm>

#include "loop_box.h"

namespace exz {


// Persistent grids.  Blocks are dispatched round-robin over the 8 XCDs;
// XCD x owns one contiguous range of boxes and its blocks walk that range
// interleaved (stride = blocks on the XCD), so the boxes in flight on an XCD
// at any moment are adjacent and their halos meet in its L2.  A launch after
// convergence costs only its (small) grid.
struct BoxWalk {
  uint32_t first, end, stride;
};

__device__ __forceinline__ BoxWalk box_walk(const FieldDev &fd) {
  const uint32_t G = gridDim.x, b = blockIdx.x, xcd = b & 7u;
  const uint32_t nx = G < 8 ? G : 8;                   // XCDs with blocks
  const uint32_t mine = (G - xcd + 7) / 8;             // blocks on this XCD
  const uint32_t per = ((uint32_t)fd.ntiles + nx - 1) / nx;
  BoxWalk w;
  w.first = xcd * per + (b >> 3);
  w.end = min((uint32_t)fd.ntiles, (xcd + 1) * per);
  w.stride = mine;
  return w;
}

template <class T, int TY, int TZ>
__global__ void __launch_bounds__(64 * TY) k_check(FieldDev fd, const uint32_t *__restrict__ conn) {
  State *st = fd.st;
  if (st->done) return;
  __shared__ CheckLds<T, TY, TZ> L;
  __shared__ unsigned long long pick;
  load_conn(L, conn);
  const BoxWalk w = box_walk(fd);
  const bool lead = threadIdx.x == 0 && threadIdx.y == 0;
  uint32_t done_v = 0;  // vertices checked by this work-group (lead thread)
  // The reformulated event constraints over all ranks, in items of four
  // ranks per thread (the order test does not depend on this pass's
  // check): a work-group takes one item after each box of a dense pass, so
  // that the streaming of the critical-point values overlaps the other
  // work-groups' arithmetic, and the rest after its boxes.
  const bool order = fd.mode != 1 && fd.K > 1;
  const uint32_t K = (uint32_t)fd.K, tag = st->tag;
  const uint32_t tid = threadIdx.y * 64 + threadIdx.x, per = 4u * 64u * TY;
  uint32_t ob = blockIdx.x * per;  // this work-group's next item
  if (!fd.frontier || st->dense) {
    // a dense pass consumes every box flag: clear them, so none is stale
    for (uint32_t tile = w.first; tile < w.end; tile += w.stride) {
      const BoxOrigin o = box_of(fd, tile, TY, TZ);
      check_box<T, TY, TZ>(fd, o, L);
      if (lead) {
        done_v += box_vertices(fd, o, TY, TZ);
        if (fd.frontier) fd.bdirty[tile] = 0;
      }
      __syncthreads();
      if (order && ob + 1 < K) {
        order_quad<T>(fd, ob + 4u * tid, K, threadIdx.x != 63, tag);
        ob += gridDim.x * per;
      }
    }
  } else {
    // Frontier pass: a box none of whose cells (halo included) changed in
    // the last apply would name the same targets as at its last check, and
    // those were all blocked then and still are, so only dirty boxes are
    // checked.  The first wave reads (and clears) the flags of the block's
    // next 64 boxes.
    for (uint32_t t0 = w.first; t0 < w.end; t0 += 64u * w.stride) {
      if (threadIdx.y == 0) {
        const uint32_t tile = t0 + threadIdx.x * w.stride;
        bool d = false;
        if (tile < w.end) {
          d = fd.bdirty[tile] != 0;
          if (d) fd.bdirty[tile] = 0;
        }
        const unsigned long long b = __ballot(d);
        if (threadIdx.x == 0) pick = b;
      }
      __syncthreads();
      unsigned long long b = pick;
      __syncthreads();  // pick is rewritten for the next 64 boxes
      while (b) {
        const uint32_t k = (uint32_t)(__ffsll(b) - 1);
        b &= b - 1;
        const BoxOrigin o = box_of(fd, t0 + k * w.stride, TY, TZ);
        check_box<T, TY, TZ>(fd, o, L);
        if (lead) done_v += box_vertices(fd, o, TY, TZ);
        __syncthreads();
      }
    }
  }
  if (lead && done_v) atomicAdd(&st->checked, (unsigned long long)done_v);
  if (order)
    for (; ob + 1 < K; ob += gridDim.x * per) order_quad<T>(fd, ob + 4u * tid, K, threadIdx.x != 63, tag);
}

// Reference topology of f, box by box over the same persistent walk.
template <class T, int TY, int TZ>
__global__ void __launch_bounds__(64 * TY) k_ref(FieldDev fd, const uint32_t *__restrict__ conn) {
  __shared__ RefLds<T, TY, TZ> L;
  copy_conn<TY>(L.conn, conn);
  const BoxWalk w = box_walk(fd);
  for (uint32_t tile = w.first; tile < w.end; tile += w.stride) {
    ref_box<T, TY, TZ>(fd, box_of(fd, tile, TY, TZ), L);
    __syncthreads();
  }
}

// ApplyBoundedEdits over the target marks.
template <class T>
__global__ void __launch_bounds__(APPLY_BLOCK) k_apply(FieldDev fd) {
  if (fd.st->done) return;
  const uint32_t nq = ((uint32_t)fd.n + 3) / 4;
  EditCount ec = {{0, 0, 0, 0, 0}};
  apply_quads<T>(fd, blockIdx.x * APPLY_BLOCK + threadIdx.x, gridDim.x * APPLY_BLOCK, nq, ec);
  flush_counts<APPLY_BLOCK / 64>(fd.st, ec, blockIdx.x);
}

__global__ void __launch_bounds__(64) k_finalize(FieldDev fd) { finalize_field(fd); }

__global__ void __launch_bounds__(64) k_state_reset(State *st, int64_t max_iters) {
  const int lane = threadIdx.x;
#pragma unroll
  for (int k = 0; k < 5; ++k) st->shard[k][lane] = 0;
  if (lane != 0) return;
  st->done = RUNNING;
  st->err = 0;
  st->ntargets = st->changed = st->lossless = st->floored = st->first = 0;
  st->cert_bad = 0;
  st->nsaddle = 0;
  st->dense = 1;
  st->noflag = 1;  // the first iterations change values in nearly every box
  st->busy = 1;
  st->tag = 1;
  st->iterations = st->edit_ops = st->lossless_total = st->floor_total = st->edited_total = 0;
  st->targets_total = 0;
  st->residual = 0;
  st->max_iters = max_iters;
  st->passes = 0;
  st->checked = 0;
}

hipError_t launch_state_reset(const FieldDev &fd, int64_t max_iters, hipStream_t s) {
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, fd.st, max_iters);
  return hipGetLastError();
}

bool box_supported(int ty, int tz) {
#define EXZ_BOX_MATCH(a, b) if (ty == a && tz == b) return true;
  EXZ_BOX_SHAPES(EXZ_BOX_MATCH)
#undef EXZ_BOX_MATCH
  return false;
}

// Enough work-groups of 64 x tile_y threads to fill 256 CUs (2048 waves of
// 64 per XCD share), never more than there are boxes.
// fd.grid_blocks = 0 launches one work-group per box instead.
static int persistent_grid(const FieldDev &fd) {
  const int per_cu = fd.tile_y >= 16 ? 2 : fd.tile_y >= 8 ? 4 : 8;
  const int g = fd.grid_blocks > 0 ? fd.grid_blocks : fd.grid_blocks == 0 ? fd.ntiles : 256 * per_cu;
  return fd.ntiles < g ? fd.ntiles : g;
}

// The check pass (with the critical-point order test of the reformulated
// constraints), then, in original mode, the per-saddle event kernels.
template <class T>
static void launch_check_events(const FieldDev &fd, const uint32_t *conn, const uint8_t *comp,
                                hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0) (void)hipEventRecord(ev0, s);
#define EXZ_BOX_CHECK(a, b)                                                                \
  if (fd.tile_y == a && fd.tile_z == b)                                                    \
    hipLaunchKernelGGL((k_check<T, a, b>), dim3(persistent_grid(fd)), dim3(64, a), 0, s, fd, conn);
  EXZ_BOX_SHAPES(EXZ_BOX_CHECK)
#undef EXZ_BOX_CHECK
  if (ev1) (void)hipEventRecord(ev1, s);
  // (the reformulated mode's order test runs inside the check kernel)
  if (fd.mode == 1) (void)launch_original_events(fd, comp, s);
}

template <class T>
static void launch_ref_t(const FieldDev &fd, const uint32_t *conn, hipStream_t s) {
#define EXZ_BOX_REF(a, b)                                                                  \
  if (fd.tile_y == a && fd.tile_z == b)                                                    \
    hipLaunchKernelGGL((k_ref<T, a, b>), dim3(persistent_grid(fd)), dim3(64, a), 0, s, fd, conn);
  EXZ_BOX_SHAPES(EXZ_BOX_REF)
#undef EXZ_BOX_REF
}

hipError_t launch_ref(const FieldDev &fd, const uint32_t *conn, hipStream_t s) {
  if (fd.dtype == 0)
    launch_ref_t<float>(fd, conn, s);
  else
    launch_ref_t<double>(fd, conn, s);
  return hipGetLastError();
}

template <class T>
static void launch_apply(const FieldDev &fd, hipStream_t s) {
  const int chunks = (int)(((uint32_t)fd.n + APPLY_CHUNK - 1) / APPLY_CHUNK);
  hipLaunchKernelGGL(k_apply<T>, dim3(std::min(chunks, 8192)), dim3(APPLY_BLOCK), 0, s, fd);
}

template <class T>
static void launch_phases(const FieldDev &fd, const uint32_t *conn, const uint8_t *comp,
                          hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  launch_check_events<T>(fd, conn, comp, s, ev0, ev1);
  launch_apply<T>(fd, s);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, fd);
}

hipError_t launch_iteration(const FieldDev &fd, const uint32_t *conn, const uint8_t *comp,
                            hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (fd.dtype == 0)
    launch_phases<float>(fd, conn, comp, s, ev0, ev1);
  else
    launch_phases<double>(fd, conn, comp, s, ev0, ev1);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// diagnostics: one check pass, target flags as bytes

hipError_t launch_debug_check(const FieldDev &fd, const uint32_t *conn, hipStream_t s) {
  if (fd.dtype == 0)
    launch_check_events<float>(fd, conn, nullptr, s, nullptr, nullptr);
  else
    launch_check_events<double>(fd, conn, nullptr, s, nullptr, nullptr);
  return hipGetLastError();
}

__global__ void k_targets_to_bytes(FieldDev fd, uint8_t *out) {
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  bool hit = false;
  if (t < (uint32_t)fd.n) {
    hit = fd.tmark[t] == fd.st->tag;
    out[t] = hit;
  }
  const uint32_t c = wave_sum((uint32_t)hit);
  if (__lane_id() == 0 && c) atomicAdd(&fd.st->ntargets, c);
}

hipError_t launch_targets_to_bytes(const FieldDev &fd, uint8_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_targets_to_bytes, dim3((fd.n + 255) / 256), dim3(256), 0, s, fd, out);
  return hipGetLastError();
}

}  // namespace exz
