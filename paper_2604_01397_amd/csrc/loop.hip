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
// changed (the boxes around the vertex), finalize lists the flagged boxes,
// and the next check visits only those, spread evenly over its work-groups
// (the flagged boxes cluster where the field still moves, so a fixed share
// of the boxes per work-group would leave most of them idle); a pass that
// changes nothing is followed by one dense pass before the loop may stop, so
// the decision always rests on a check of every vertex.
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
  // this work-group's next item (64-bit: a grid of one work-group per box
  // can step past 2^32 ranks)
  unsigned long long ob = (unsigned long long)blockIdx.x * per;
  const unsigned long long ostep = (unsigned long long)gridDim.x * per;
  const bool dense = !fd.frontier || st->dense;
  if (dense) {
    for (uint32_t tile = w.first; tile < w.end; tile += w.stride) {
      const BoxOrigin o = box_of(fd, tile, TY, TZ);
      check_box<T, TY, TZ>(fd, o, L);
      if (lead) done_v += box_vertices(fd, o, TY, TZ);
      __syncthreads();
      if (order && ob + 1 < K) {
        order_quad<T>(fd, (uint32_t)ob + 4u * tid, K, threadIdx.x != 63, tag);
        ob += ostep;
      }
    }
  } else {
    // Frontier pass: a box none of whose cells (halo included) changed in
    // the last apply would name the same targets as at its last check, and
    // those were all blocked then and still are, so only the listed (dirty)
    // boxes are checked.  XCD x takes the x-th eighth of the list and its
    // work-groups interleave over it, so every work-group checks the same
    // number of boxes (to one) and boxes adjacent in the list, which are
    // near in the field, share an L2.
    const uint32_t M = st->nfront, G = gridDim.x, x = blockIdx.x & 7u;
    const uint32_t nx = G < 8 ? G : 8;
    const uint32_t lo = (uint32_t)((unsigned long long)M * x / nx);
    const uint32_t hi = (uint32_t)((unsigned long long)M * (x + 1) / nx);
    const uint32_t mine = (G - x + 7) / 8;
    for (uint32_t j = lo + (blockIdx.x >> 3); j < hi; j += mine) {
      const BoxOrigin o = box_of(fd, glob(fd.blist)[j], TY, TZ);
      check_box<T, TY, TZ, true>(fd, o, L);
      if (lead) done_v += box_vertices(fd, o, TY, TZ);
      __syncthreads();
    }
  }
  if (lead && done_v) atomicAdd(&st->checked, (unsigned long long)done_v);
  if (order && dense) {
    for (; ob + 1 < K; ob += ostep) order_quad<T>(fd, (uint32_t)ob + 4u * tid, K, threadIdx.x != 63, tag);
  } else if (order) {
    // A frontier pass tests only the pairs a value of which the last apply
    // changed (the others are as at their last test, and so are the targets
    // they named): each wave's 256 ranks of an item carry the tag of the
    // last apply that moved one of them or the first rank after them.  Each
    // lane reads the tag of one of its wave's items; the wave tests the
    // items whose tag is the last pass's (and tags the chunks of its marks,
    // for the apply after it).
    // (rank positions in 64 bits: with one work-group per box, 64 steps of
    // the grid exceed 2^32 ranks)
    const uint32_t prev = tag == 1 ? MARK_TAGS : tag - 1;
    const uint32_t lane = threadIdx.x, wb = 256u * threadIdx.y;
    const unsigned long long step = ostep;
    for (unsigned long long k0 = 0; ob + k0 * step + 1 < K; k0 += 64) {
      const unsigned long long rb = ob + (k0 + lane) * step + wb;
      unsigned long long live = __ballot(rb + 1 < K && glob(fd.oflag)[rb >> 8] == prev);
      while (live) {
        const unsigned long long k = k0 + (unsigned long long)(__ffsll(live) - 1);
        live &= live - 1;
        order_quad<T, true>(fd, (uint32_t)(ob + k * step + wb) + 4u * lane, K, lane != 63, tag);
      }
    }
  }
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
  // the list of the last frontier check has been read: finalize refills it
  if (blockIdx.x == 0 && threadIdx.x == 0) fd.st->nfront = 0;
  const uint32_t nq = ((uint32_t)fd.n + 3) / 4;
  EditCount ec = {{0, 0, 0, 0, 0}};
  apply_quads<T, true>(fd, blockIdx.x * APPLY_BLOCK + threadIdx.x, gridDim.x * APPLY_BLOCK, nq, ec);
  flush_counts<APPLY_BLOCK / 64>(fd.st, ec, blockIdx.x);
}

// Frontier list: work-group b >= 1 of finalize takes LIST_TILES box flags,
// 16 per thread, lists the flagged boxes (block-wide prefix sum, one atomic
// per work-group for its place in the list) and clears their flags.  The
// list's order does not matter to the check; each work-group's part of it is
// in box order.
constexpr int LIST_BLOCK = 256;
constexpr uint32_t LIST_TILES = 16u * LIST_BLOCK;

__device__ __forceinline__ void list_dirty_boxes(const FieldDev &fd, uint32_t part) {
  __shared__ uint32_t wsum[LIST_BLOCK / 64];
  __shared__ uint32_t base;
  const uint32_t nt = (uint32_t)fd.ntiles, tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const uint32_t t0 = part * LIST_TILES + 16u * tid;
  uint8_t *F = fd.bdirty;
  uint32_t bits = 0;  // bit k: box t0 + k is flagged
  const bool whole = t0 + 16 <= nt;  // 16-byte aligned: the flags start 256-aligned
  if (whole) {
    const u32x4 v = *glob(reinterpret_cast<const u32x4 *>(F + t0));
    const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int c = 0; c < 16; ++c) bits |= (((wd[c >> 2] >> (8 * (c & 3))) & 255u) != 0) << c;
  } else {
    for (uint32_t c = 0; t0 + c < nt && c < 16; ++c) bits |= (uint32_t)(glob(F)[t0 + c] != 0) << c;
  }
  const uint32_t cnt = (uint32_t)__popc(bits);
  uint32_t incl = cnt;  // inclusive prefix over the wave
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(incl, d);
    if (lane >= (uint32_t)d) incl += o;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t woff = 0, total = 0;
#pragma unroll
  for (int k = 0; k < LIST_BLOCK / 64; ++k) {
    woff += (uint32_t)k < w ? wsum[k] : 0u;
    total += wsum[k];
  }
  if (tid == 0) base = total ? atomicAdd(&fd.st->nfront, total) : 0u;
  __syncthreads();
  if (!bits) return;
  uint32_t pos = base + woff + incl - cnt;
  for (uint32_t b = bits; b; b &= b - 1) glob(fd.blist)[pos++] = t0 + (uint32_t)(__ffs(b) - 1);
  if (whole)
    *glob(reinterpret_cast<u32x4 *>(F + t0)) = u32x4{0u, 0u, 0u, 0u};
  else
    for (uint32_t b = bits; b; b &= b - 1) glob(F)[t0 + (uint32_t)(__ffs(b) - 1)] = 0;
}

// Work-group 0: the loop decision; the others (frontier passes only): the
// frontier list of the boxes the apply just flagged.
__global__ void __launch_bounds__(LIST_BLOCK) k_finalize(FieldDev fd) {
  if (blockIdx.x == 0) {
    if (threadIdx.x < 64) finalize_field(fd);
    return;
  }
  if (fd.st->done) return;  // (set by work-group 0 meanwhile: the list goes unused)
  list_dirty_boxes(fd, blockIdx.x - 1);
}

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
  st->nfront = 0;
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
  const uint32_t lists = fd.frontier ? ((uint32_t)fd.ntiles + LIST_TILES - 1) / LIST_TILES : 0u;
  hipLaunchKernelGGL(k_finalize, dim3(1 + lists), dim3(LIST_BLOCK), 0, s, fd);
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
