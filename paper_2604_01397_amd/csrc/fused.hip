// Fused passes of the correction loop (reformulated event constraints, one
// field): pass p applies the targets named in pass p-1 (ApplyBoundedEdits,
// Sec. 3.3) and checks the resulting field (CheckConstraints, Sec. 4.2) in
// one sweep over the boxes, so the field, the marks and the counts are staged
// once per iteration instead of being read by two kernels.
//
// An edit depends only on the vertex's own value, f, count and mark, so a
// work-group can apply the edits of every cell it stages -- its box and the
// one-cell halo -- and obtain exactly the values the owners of the halo
// cells write (Jacobi rounds, Alg. 1).  For that every block must read the
// state before the pass, so g and the counts are double-buffered (pass p
// reads buffer p % 2 and writes buffer (p+1) % 2), the marks rotate over three
// buffers (read the previous pass's, write this pass's, clear the next one),
// and the dirty-box flags over two.
//
// Frontier rule: box B is processed in pass p when its cells plus halo hold
// a mark of pass p-1 or changed in pass p-1 (the first pass and fixpoint
// confirmations process every box).  An unprocessed box did not change in the
// last two passes, so the buffer it did not write still holds its current
// values; its check would name the targets of its last check, which were
// blocked then and still are.  Results are those of dense passes, bit for bit.
#include <algorithm>

#include "loop_box.h"

namespace exz {

// Buffers of one fused pass.
struct PassBufs {
  const void *gin;      // field before the pass
  void *gout;           // field after the pass (written for processed boxes)
  const uint8_t *cin;   // edit counts before / after
  uint8_t *cout;
  const uint8_t *min;   // targets named by the previous pass
  uint8_t *din;         // boxes to process in this pass (read and cleared)
  // fd.tmark = targets named now, fd.bdirty = boxes for the next pass
};

// Per staged cell: bit 7 marked (a target of the previous pass), bit 6 its
// value or count moved, bit 5 it landed on its lower bound, bits 0..4 the
// new count.
constexpr uint32_t CN_MARK = 128u, CN_MOVED = 64u, CN_FLOOR = 32u, CN_COUNT = 31u;

template <class T, int TY, int TZ>
struct StepLds {
  T S[Box<TY, TZ>::NE];        // values after this pass's edits
  uint8_t CN[Box<TY, TZ>::NE];  // edit flags (above)
  uint32_t ref[TZ][64 * TY];   // own vertices: code | lower mask << 8 | count << 24
  uint32_t dirs;               // boxes to mark for the next pass (axis masks)
};

// The bounded edit of one staged cell (Sec. 3.3): returns its new value and
// sets its flags.
template <class T>
__device__ __forceinline__ T edit_cell(T g0, T fv, uint32_t c0, T xiT, T delta, int N,
                                       uint32_t &flags) {
  const T L = lower_bound(fv, xiT);
  flags = CN_MARK | (c0 & CN_COUNT);
  if (g0 == L) return g0;  // blocked at the floor
  const uint32_t c = c0 + 1;
  const T v = c > (uint32_t)N ? L : (g0 - delta < L ? L : g0 - delta);
  flags = CN_MARK | CN_MOVED | (v == L ? CN_FLOOR : 0u) | c;
  return v;
}

// Stages the field of the box plus its halo with this pass's edits applied.
// First the values and marks, row by row as in stage_rows(), straight into
// LDS (a thread keeps only the field index of its cells and a bit mask of
// the marked ones); then f and the count of the marked cells, and their
// edits overwrite the staged values (a thread rewrites only cells it wrote).
template <class T, int TY, int TZ>
__device__ __forceinline__ void stage_apply(const FieldDev &fd, const PassBufs &pb,
                                            StepLds<T, TY, TZ> &L, BoxOrigin o) {
  using B = Box<TY, TZ>;
  constexpr int NR = B::H * B::D;
  constexpr int RPW = (NR + TY - 1) / TY;
  constexpr int NEDGE = (2 * NR + 64 * TY - 1) / (64 * TY);
  constexpr int NC = RPW + NEDGE;  // cells per thread
  static_assert(NC <= 32, "marked-cell mask is 32 bits");
  const int lane = threadIdx.x, w = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int tid = w * 64 + lane;
  const int nx = fd.nx, ny = fd.ny, nz = fd.nz;
  const T *gin = (const T *)pb.gin;
  uint32_t idx[NC];  // field index of each cell (0 where outside)
  uint32_t inside = 0;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    int gx, gy, gz;
    bool ok;
    if (k < RPW) {
      const int row = w + k * TY;
      gy = o.y0 - 1 + row % B::H;
      gz = o.z0 - 1 + row / B::H;
      gx = o.x0 - 1 + lane;
      ok = row < NR;
    } else {
      const int t = tid + (k - RPW) * 64 * TY, row = t >> 1;
      gy = o.y0 - 1 + row % B::H;
      gz = o.z0 - 1 + row / B::H;
      gx = o.x0 + 63 + (t & 1);
      ok = t < 2 * NR;
    }
    const bool in = ok && gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
    inside |= (uint32_t)in << k;
    idx[k] = in ? ((uint32_t)gz * (uint32_t)ny + (uint32_t)gy) * (uint32_t)nx + (uint32_t)gx : 0u;
  }
  // LDS cell of cell k of this thread, -1 where none
  auto slot = [&](int k) -> int {
    if (k < RPW) {
      const int row = w + k * TY;
      return row < NR ? row * B::W + lane : -1;
    }
    const int t = tid + (k - RPW) * 64 * TY;
    return t < 2 * NR ? (t >> 1) * B::W + 64 + (t & 1) : -1;
  };
  // one round of loads: value, mark, f and count of every cell (in dense
  // passes nearly every line of f and of the counts is needed anyway)
  const T *F = (const T *)fd.f;
  const T xiT = (T)fd.xiT, delta = (T)fd.delta;
#pragma unroll
  for (int k0 = 0; k0 < NC; k0 += 4) {
    T v[4], fv[4];
    uint32_t mk[4], c0[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (k0 + j >= NC) break;
      const uint32_t id = idx[k0 + j];
      v[j] = glob(gin)[id];
      mk[j] = glob(pb.min)[id];
      fv[j] = glob(F)[id];
      c0[j] = glob(pb.cin)[id];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + j;
      if (k >= NC) break;
      const int e = slot(k);
      if (e < 0) continue;
      const bool in = (inside >> k) & 1u;
      uint32_t flags = 0;
      T val = in ? v[j] : outside_value<T>();
      if (in && mk[j]) val = edit_cell<T>(v[j], fv[j], c0[j], xiT, delta, fd.N, flags);
      L.S[e] = val;
      L.CN[e] = (uint8_t)flags;
    }
  }
}

// Axis mask of a coordinate c relative to a box of extent W along that
// axis (c in -1 .. W): bit 1 the box itself, bit 0 the box below when c is
// on or past the low face, bit 2 the box above when on or past the high face.
__device__ __forceinline__ uint32_t axis_bits(int c, int W) {
  return 2u | (c <= 0 ? 1u : 0u) | (c >= W - 1 ? 4u : 0u);
}

// Boxes whose cells plus halo contain local point (lx, ly, lz) of box B:
// three 3-bit axis masks (x bits 0-2, y bits 3-5, z bits 6-8).
template <int TY, int TZ>
__device__ __forceinline__ uint32_t point_dirs(int lx, int ly, int lz) {
  return axis_bits(lx, 64) | (axis_bits(ly, TY) << 3) | (axis_bits(lz, TZ) << 6);
}

// One box of a fused pass.
template <class T, int TY, int TZ>
__device__ __forceinline__ uint32_t step_box(const FieldDev &fd, const PassBufs &pb,
                                             const uint32_t *__restrict__ conn, uint32_t tile,
                                             StepLds<T, TY, TZ> &L, EditCount &ec) {
  using B = Box<TY, TZ>;
  const BoxOrigin o = box_of(fd, tile, TY, TZ);
  const int lx = threadIdx.x, ly = threadIdx.y, tid = ly * 64 + lx;
  const int x = o.x0 + lx, y = o.y0 + ly;
  const bool col = x < fd.nx && y < fd.ny;
  const uint32_t plane = (uint32_t)fd.nx * (uint32_t)fd.ny;
  const uint32_t i0 = (uint32_t)x + (uint32_t)fd.nx * ((uint32_t)y + (uint32_t)fd.ny * (uint32_t)o.z0);
  uint32_t refs[TZ];
#pragma unroll
  for (int k = 0; k < TZ; ++k) {
    const bool in = col && o.z0 + k < fd.nz;
    const uint32_t id = in ? i0 + k * plane : 0u;
    refs[k] = glob(fd.code)[id] | ((uint32_t)glob(fd.low)[id] << 8) | ((uint32_t)glob(pb.cin)[id] << 24);
  }
  if (tid == 0) L.dirs = 0;
  stage_apply<T, TY, TZ>(fd, pb, L, o);
#pragma unroll
  for (int k = 0; k < TZ; ++k) L.ref[k][tid] = refs[k];
  const bool interior = o.x0 >= 1 && o.x0 + 64 <= fd.nx - 1 && o.y0 >= 1 &&
                        o.y0 + TY <= fd.ny - 1 && o.z0 >= 1 && o.z0 + TZ <= fd.nz - 1;
  __syncthreads();
  T *gout = (T *)pb.gout;
  uint32_t dirs = 0, done_v = 0;
#pragma unroll 1
  for (int k = 0; k < TZ; ++k) {
    const int z = o.z0 + k;
    if (!(col && z < fd.nz)) continue;
    const uint32_t i = i0 + k * plane;
    const int e = (k + 1) * B::PLANE + (ly + 1) * B::W + lx + 1;
    const T val = L.S[e];
    const uint32_t flags = L.CN[e];
    const uint32_t rf = L.ref[k][tid];
    const uint32_t c_own = rf >> 24;
    const uint32_t c_new = (flags & CN_MOVED) ? (flags & CN_COUNT) : c_own;
    glob(gout)[i] = val;
    glob(pb.cout)[i] = (uint8_t)c_new;
    if (flags & CN_MARK) ++ec.v[0];
    if (flags & CN_MOVED) {
      ++ec.v[1];
      ec.v[2] += c_new > (uint32_t)fd.N;
      ec.v[3] += (flags & CN_FLOOR) != 0;
      ec.v[4] += c_new == 1;
      const uint32_t rk = glob(fd.rank_of)[i];
      if (rk != 0xFFFFFFFFu) glob((T *)fd.cp_val)[rk] = val;
      dirs |= point_dirs<TY, TZ>(lx, ly, k);
    }
    uint32_t av = 0, dv = 0;
    uint32_t r = check_vertex<T>(fd, conn, L.S + e, -B::PLANE, B::PLANE, x, y, z, i, rf & 255u,
                                 (rf >> 8) & 0xFFFFu, av, dv, interior);
    if (r) {
      post_targets(fd, i, r);
      if ((r >> SELF) & 1u) dirs |= point_dirs<TY, TZ>(lx, ly, k);
      r &= LOW_MASK;
      while (r) {
        const int s = __ffs(r) - 1;
        r &= r - 1;
        dirs |= point_dirs<TY, TZ>(lx + DXS[s], ly + DYS[s], k + DZS[s]);
      }
    }
    ++done_v;
  }
  if (dirs) atomicOr(&L.dirs, dirs);
  __syncthreads();
  if (tid == 0 && L.dirs) {  // this pass's targets and changes: boxes for the next pass
    const uint32_t d = L.dirs;
    const int bx = (int)(tile % (uint32_t)fd.tiles_x), r2 = (int)(tile / (uint32_t)fd.tiles_x);
    const int by = r2 % fd.tiles_y, bz = r2 / fd.tiles_y;
    for (int dz = -1; dz <= 1; ++dz) {
      if (!((d >> (7 + dz)) & 1u) || bz + dz < 0 || bz + dz >= fd.tiles_z) continue;
      for (int dy = -1; dy <= 1; ++dy) {
        if (!((d >> (4 + dy)) & 1u) || by + dy < 0 || by + dy >= fd.tiles_y) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          if (!((d >> (1 + dx)) & 1u) || bx + dx < 0 || bx + dx >= fd.tiles_x) continue;
          glob(fd.bdirty)[(bx + dx) + fd.tiles_x * ((by + dy) + fd.tiles_y * (bz + dz))] = 1;
        }
      }
    }
  }
  return done_v;
}

// A fused pass over the boxes of the field (persistent, XCD-interleaved walk
// as in k_check).  Frontier passes read the flags of 64 boxes at a time.
template <class T, int TY, int TZ>
__global__ void __launch_bounds__(64 * TY) k_step(FieldDev fd, PassBufs pb,
                                                  const uint32_t *__restrict__ conn) {
  State *st = fd.st;
  if (st->done) return;
  __shared__ StepLds<T, TY, TZ> L;
  __shared__ unsigned long long pick;
  const uint32_t G = gridDim.x, b = blockIdx.x, xcd = b & 7u;
  const uint32_t nxcd = G < 8 ? G : 8, mine = (G - xcd + 7) / 8;
  const uint32_t per = ((uint32_t)fd.ntiles + nxcd - 1) / nxcd;
  const uint32_t first = xcd * per + (b >> 3), end = min((uint32_t)fd.ntiles, (xcd + 1) * per);
  const bool lead = threadIdx.x == 0 && threadIdx.y == 0;
  const bool all = !fd.frontier || st->dense;
  EditCount ec = {{0, 0, 0, 0, 0}};
  uint32_t count = 0;
  for (uint32_t t0 = first; t0 < end; t0 += 64u * mine) {
    if (threadIdx.y == 0) {  // flags of the next 64 boxes (read and cleared)
      const uint32_t tile = t0 + threadIdx.x * mine;
      bool d = false;
      if (tile < end) {
        d = glob(pb.din)[tile] != 0;
        if (d) glob(pb.din)[tile] = 0;
      }
      const unsigned long long m = __ballot(all ? tile < end : d);
      if (threadIdx.x == 0) pick = m;
    }
    __syncthreads();
    unsigned long long m = pick;
    __syncthreads();
    while (m) {
      const uint32_t k = (uint32_t)(__ffsll(m) - 1);
      m &= m - 1;
      count += step_box<T, TY, TZ>(fd, pb, conn, t0 + k * mine, L, ec);
      __syncthreads();
    }
  }
  const uint32_t checked = wave_sum(count);
  __shared__ uint32_t part[TY];
  if (threadIdx.x == 0) part[threadIdx.y] = checked;
  flush_counts<TY>(st, ec, blockIdx.x);  // synchronises the block
  if (lead) {
    uint32_t c = 0;
    for (int k = 0; k < TY; ++k) c += part[k];
    if (c) atomicAdd(&st->checked, (unsigned long long)c);
  }
}

__global__ void k_zero_bytes(const State *st, uint8_t *p, uint32_t nwords) {
  if (st->done) return;
  for (uint32_t k = blockIdx.x * 256 + threadIdx.x; k < nwords; k += gridDim.x * 256)
    glob(reinterpret_cast<u32x4 *>(p))[k] = u32x4{0u, 0u, 0u, 0u};
}

template <class T>
static void launch_step(const FieldDev &fd, const PassBufs &pb, const uint32_t *conn, int grid,
                        hipStream_t s) {
#define EXZ_BOX_STEP(a, b)                                                                   \
  if (fd.tile_y == a && fd.tile_z == b)                                                      \
    hipLaunchKernelGGL((k_step<T, a, b>), dim3(grid), dim3(64, a), 0, s, fd, pb, conn);
  EXZ_BOX_SHAPES(EXZ_BOX_STEP)
#undef EXZ_BOX_STEP
}

// Marks of one buffer: n + 64 bytes rounded up to 16-byte words.
uint32_t fused_mark_words(const FieldDev &fd) { return ((uint32_t)fd.n + 64 + 15) / 16; }

// One fused pass p: clear the marks of pass p+1, apply + check, the
// critical-point compare (its targets and boxes go to this pass's buffers),
// finalize.  bufs: g[2], cnt[2], marks[3], dirty[2].
hipError_t launch_fused_pass(FieldDev fd, const FusedBufs &fb, int64_t p, const uint32_t *conn,
                             const uint8_t *comp, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  (void)comp;
  const int a = (int)(p % 2), bn = (int)((p + 1) % 2);
  PassBufs pb;
  pb.gin = fb.g[a];
  pb.gout = fb.g[bn];
  pb.cin = fb.cnt[a];
  pb.cout = fb.cnt[bn];
  pb.min = fb.marks[(p + 2) % 3];  // pass p-1
  pb.din = fb.dirty[a];
  fd.tmark = fb.marks[p % 3];
  fd.bdirty = fb.dirty[bn];
  const uint32_t nw = fused_mark_words(fd);
  hipLaunchKernelGGL(k_zero_bytes, dim3(std::min<uint32_t>((nw + 255) / 256, 4096)), dim3(256), 0,
                     s, fd.st, fb.marks[(p + 1) % 3], nw);
  const int per_cu = fd.tile_y >= 16 ? 2 : fd.tile_y >= 8 ? 4 : 8;
  const int g = fd.grid_blocks > 0 ? fd.grid_blocks : 256 * per_cu;
  const int grid = std::min(fd.ntiles, g);
  if (ev0) (void)hipEventRecord(ev0, s);
  if (fd.dtype == 0)
    launch_step<float>(fd, pb, conn, grid, s);
  else
    launch_step<double>(fd, pb, conn, grid, s);
  if (ev1) (void)hipEventRecord(ev1, s);
  (void)launch_cpcmp_only(fd, s);
  (void)launch_finalize(fd, s);
  return hipGetLastError();
}

}  // namespace exz
