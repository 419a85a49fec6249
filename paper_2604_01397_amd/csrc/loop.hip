// One iteration of the correction loop (Algorithm 1) on the device:
//   check     CheckConstraints on every vertex (Sec. 4.2): steepest ascent and
//             descent neighbours of g against f, link order of saddles
//             (and of regular vertices of f that g turned into saddles).
//             Each vertex writes the set of vertices it asks to decrease as
//             a 15-bit slot mask (its neighbours and itself);
//   cpcmp     reformulated event constraints (Sec. 4.3): each critical point
//             of f against its successor in f's sorted order; an inverted
//             pair sets the request bit of the lower one on itself;
//   apply     ApplyBoundedEdits (Sec. 3.3): a vertex is a target when it or
//             a neighbour requested it; targets are edited in place;
//   finalize  convergence / stuck / iteration-cap decision, counter reset.
// The set S of Algorithm 1 is never materialised as a list: requests are
// gathered (pulled) by their target, so no two threads write the same word
// and no atomics are needed per target.  All checks of an iteration read the
// same g, and the edits run in a later launch (synchronous, Jacobi-style
// rounds).  Every kernel returns at once when the field is already done, so
// a host may issue more iterations than needed and poll rarely.
//
// check and apply are stencils over the 14-neighbour Freudenthal mesh.  Both
// run as 2.5D tiles: a work-group owns a 64 x tile_y column of tile_z planes
// and marches it along z, keeping planes z-1, z, z+1 (with a one-cell halo
// in x and y) in LDS, so each step reads one new plane from HBM with
// coalesced row loads instead of 15 scattered loads per vertex.
#include "exz_internal.h"

namespace exz {

constexpr int HALO_W = 66;  // 64 columns + halo on both sides

struct TileGeom {
  int x0, y0, zb, ze;
};

__device__ __forceinline__ TileGeom tile_of(const FieldDev &fd) {
  const uint32_t tile = xcd_swizzle(blockIdx.x, gridDim.x);
  const uint32_t tx = tile % (uint32_t)fd.tiles_x;
  const uint32_t r = tile / (uint32_t)fd.tiles_x;
  const uint32_t ty = r % (uint32_t)fd.tiles_y;
  const uint32_t tz = r / (uint32_t)fd.tiles_y;
  TileGeom t;
  t.x0 = (int)tx * 64;
  t.y0 = (int)ty * fd.tile_y;
  t.zb = (int)tz * fd.tile_z;
  t.ze = min(fd.nz, t.zb + fd.tile_z);
  return t;
}

// A plane of a field staged through registers into LDS: (tile_y + 2) rows of
// HALO_W values starting at (x0 - 1, y0 - 1), zero outside the domain.  The
// fetch for plane z + 2 is issued one step ahead of its store, so its HBM
// latency overlaps the compute of the current plane.  At most 4 values per
// thread (tile_y >= 1 means 64 * tile_y threads for 66 * (tile_y + 2) values).
constexpr int STAGE_REGS = 4;

template <class V>
__device__ __forceinline__ void fetch_plane(const FieldDev &fd, const V *src, V (&r)[STAGE_REGS],
                                            int x0, int y0, int zz, int tid, int nthr) {
  const int PS = HALO_W * (fd.tile_y + 2);
  const bool zin = zz >= 0 && zz < fd.nz;
#pragma unroll
  for (int k = 0; k < STAGE_REGS; ++k) {
    const int e = tid + k * nthr;
    const int yy = e / HALO_W, xx = e - yy * HALO_W;
    const int gx = x0 - 1 + xx, gy = y0 - 1 + yy;
    V v = V(0);
    if (e < PS && zin && gx >= 0 && gx < fd.nx && gy >= 0 && gy < fd.ny)
      v = src[gx + fd.nx * (gy + fd.ny * zz)];
    r[k] = v;
  }
}

template <class V>
__device__ __forceinline__ void store_plane(const FieldDev &fd, V *dst, const V (&r)[STAGE_REGS],
                                            int tid, int nthr) {
  const int PS = HALO_W * (fd.tile_y + 2);
#pragma unroll
  for (int k = 0; k < STAGE_REGS; ++k) {
    const int e = tid + k * nthr;
    if (e < PS) dst[e] = r[k];
  }
}

// Requests of one vertex as a slot mask (bit SELF = the vertex itself).
// P points at the LDS centre value of the vertex; pm / pp are the offsets
// of the planes below / above relative to the centre plane.
template <class T>
__device__ __forceinline__ uint32_t check_vertex(const FieldDev &fd, const uint32_t *__restrict__ conn,
                                                 const T *P, int pm, int pp, int x, int y, int z,
                                                 uint32_t i, uint32_t codeb, uint32_t lowf) {
  const int nx = fd.nx, nxy = fd.nx * fd.ny;
  const uint32_t vm = valid_slots(x, y, z, fd.nx, fd.ny, fd.nz);
  const T gi = P[0];
  T gn[NSLOT];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int po = DZS[s] < 0 ? pm : DZS[s] > 0 ? pp : 0;
    gn[s] = P[po + DYS[s] * HALO_W + DXS[s]];
  }
  T amax = gi, amin = gi;
  uint32_t ia = i, id = i, lower = 0;
  int asc = SELF, desc = SELF;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const T gj = gn[s];
    const bool ok = (vm >> s) & 1u;
    const uint32_t j = (uint32_t)((int)i + slot_delta(s, nx, nxy));
    lower |= (uint32_t)(ok & sos_lt(gj, j, gi, i)) << s;
    const bool up = ok & sos_lt(amax, ia, gj, j);
    amax = up ? gj : amax;
    ia = up ? j : ia;
    asc = up ? s : asc;
    const bool dn = ok & sos_lt(gj, j, amin, id);
    amin = dn ? gj : amin;
    id = dn ? j : id;
    desc = dn ? s : desc;
  }
  const uint32_t code = codeb;
  const int asc_f = (int)(code & 15u), desc_f = (int)(code >> 4);
  const uint32_t lower_f = lowf & LOW_MASK;
  // link order applies to saddles of f, and to regular vertices of f that g
  // turned into saddles (critical-point consistency)
  bool link_rule = (lowf & LOW_SADDLE) != 0;
  if (!link_rule && lower != lower_f && asc_f != SELF && desc_f != SELF && lower != 0 &&
      lower != vm) {
    const uint32_t up = vm & ~lower;
    const bool regular_g = ((conn[lower >> 5] >> (lower & 31u)) & 1u) &&
                           ((conn[up >> 5] >> (up & 31u)) & 1u);
    link_rule = !regular_g;
  }
  uint32_t req = 0;
  // ascent side: the neighbour g wrongly takes as highest goes down
  if (asc != asc_f) req |= 1u << asc;
  // descent side: f's lowest neighbour goes down until it is lowest again
  if (desc != desc_f) req |= 1u << desc_f;
  // link order: a flipped pair goes down at its lower end in f
  if (link_rule) {
    const uint32_t diff = lower ^ lower_f;
    req |= diff & lower_f;
    if (diff & ~lower_f) req |= 1u << SELF;
  }
  return req;
}

template <class T>
__global__ void __launch_bounds__(1024) k_check(FieldDev fd, const uint32_t *__restrict__ conn) {
  if (fd.st->done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *P = (T *)smem_raw;
  const TileGeom tg = tile_of(fd);
  const int PS = HALO_W * (fd.tile_y + 2);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int tid = ly * 64 + lx, nthr = 64 * fd.tile_y;
  const T *G = (const T *)fd.g;
  const int x = tg.x0 + lx, y = tg.y0 + ly;
  const bool inside = x < fd.nx && y < fd.ny;
  const int cofs = (ly + 1) * HALO_W + lx + 1;
  const uint32_t plane = (uint32_t)fd.nx * (uint32_t)fd.ny;
  T r[STAGE_REGS];
  fetch_plane(fd, G, r, tg.x0, tg.y0, tg.zb - 1, tid, nthr);
  store_plane(fd, P + ((tg.zb + 2) % 3) * PS, r, tid, nthr);
  fetch_plane(fd, G, r, tg.x0, tg.y0, tg.zb, tid, nthr);
  store_plane(fd, P + (tg.zb % 3) * PS, r, tid, nthr);
  fetch_plane(fd, G, r, tg.x0, tg.y0, tg.zb + 1, tid, nthr);
  uint32_t i = inside ? (uint32_t)(x + fd.nx * (y + fd.ny * tg.zb)) : 0u;
  uint32_t codeb = inside ? fd.code[i] : 0u, lowf = inside ? fd.low[i] : 0u;
  for (int z = tg.zb; z < tg.ze; ++z) {
    const int s0 = z % 3, sp = (z + 1) % 3, sm = (z + 2) % 3;
    store_plane(fd, P + sp * PS, r, tid, nthr);  // plane z + 1
    if (z + 1 < tg.ze) fetch_plane(fd, G, r, tg.x0, tg.y0, z + 2, tid, nthr);
    const bool more = inside && z + 1 < tg.ze;
    const uint32_t codeb_n = more ? fd.code[i + plane] : 0u;
    const uint32_t lowf_n = more ? fd.low[i + plane] : 0u;
    __syncthreads();
    if (inside) {
      const T *c = P + s0 * PS + cofs;
      fd.req[i] = (uint16_t)check_vertex<T>(fd, conn, c, (sm - s0) * PS, (sp - s0) * PS, x, y,
                                             z, i, codeb, lowf);
    }
    i += plane;
    codeb = codeb_n;
    lowf = lowf_n;
    __syncthreads();
  }
}

// Reformulated event constraints: consecutive critical points in f's order
// must keep their order in g; an inverted pair decreases the lower one.
// Rank k maps to a distinct vertex, so the read-modify-write of its request
// word races with nothing.
template <class T>
__global__ void __launch_bounds__(256) k_cpcmp(FieldDev fd) {
  if (fd.st->done) return;
  const T *V = (const T *)fd.cp_val;
  const uint32_t k = blockIdx.x * 256 + threadIdx.x;
  if (k + 1 < (uint32_t)fd.K) {
    const T a = V[k], b = V[k + 1];
    const uint32_t ia = fd.cp_idx[k], ib = fd.cp_idx[k + 1];
    if (sos_lt(b, ib, a, ia)) fd.req[ia] = (uint16_t)(fd.req[ia] | (1u << SELF));
  }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  return v;
}

// Is the vertex whose LDS request word is Q[0] requested by itself or by a
// neighbour?  Neighbour i = t - d(s) asks for t when bit s of its mask is
// set; i lies in the domain exactly when the opposite slot s^1 is valid at t.
__device__ __forceinline__ bool requested(const uint16_t *Q, int qm, int qp, uint32_t vm) {
  uint32_t hit = (Q[0] >> SELF) & 1u;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int po = DZS[s] > 0 ? qm : DZS[s] < 0 ? qp : 0;  // plane of z - dz
    const uint32_t w = Q[po - DYS[s] * HALO_W - DXS[s]];
    hit |= ((vm >> (s ^ 1)) & (w >> s)) & 1u;
  }
  return hit != 0;
}

// ApplyBoundedEdits: each target moves once, from its own value, by one step
// of Delta (never below L); its (N+1)-th edit stores L itself; a target that
// already sits on L cannot move.  Counters are reduced per work-group and
// added to one of 64 shards.
template <class T>
__global__ void __launch_bounds__(1024) k_apply(FieldDev fd) {
  State *st = fd.st;
  if (st->done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  uint16_t *Q = (uint16_t *)smem_raw;
  const TileGeom tg = tile_of(fd);
  const int PS = HALO_W * (fd.tile_y + 2);
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int tid = ly * 64 + lx, nthr = 64 * fd.tile_y;
  const int x = tg.x0 + lx, y = tg.y0 + ly;
  const bool inside = x < fd.nx && y < fd.ny;
  const int cofs = (ly + 1) * HALO_W + lx + 1;
  T *G = (T *)fd.g;
  const T *F = (const T *)fd.f;
  const T xiT = (T)fd.xiT, delta = (T)fd.delta;
  uint32_t targets = 0, changed = 0, lossless = 0, floored = 0, first = 0;
  uint16_t r[STAGE_REGS];
  fetch_plane(fd, (const uint16_t *)fd.req, r, tg.x0, tg.y0, tg.zb - 1, tid, nthr);
  store_plane(fd, Q + ((tg.zb + 2) % 3) * PS, r, tid, nthr);
  fetch_plane(fd, (const uint16_t *)fd.req, r, tg.x0, tg.y0, tg.zb, tid, nthr);
  store_plane(fd, Q + (tg.zb % 3) * PS, r, tid, nthr);
  fetch_plane(fd, (const uint16_t *)fd.req, r, tg.x0, tg.y0, tg.zb + 1, tid, nthr);
  for (int z = tg.zb; z < tg.ze; ++z) {
    const int s0 = z % 3, sp = (z + 1) % 3, sm = (z + 2) % 3;
    store_plane(fd, Q + sp * PS, r, tid, nthr);
    if (z + 1 < tg.ze) fetch_plane(fd, (const uint16_t *)fd.req, r, tg.x0, tg.y0, z + 2, tid, nthr);
    __syncthreads();
    if (inside) {
      const uint32_t vm = valid_slots(x, y, z, fd.nx, fd.ny, fd.nz);
      if (requested(Q + s0 * PS + cofs, (sm - s0) * PS, (sp - s0) * PS, vm)) {
        const uint32_t t = (uint32_t)(x + fd.nx * (y + fd.ny * z));
        ++targets;
        const T g0 = G[t];
        const T L = lower_bound(F[t], xiT);
        if (g0 != L) {
          const int c = fd.cnt[t] + 1;
          fd.cnt[t] = (uint8_t)c;
          T v;
          if (c > fd.N) {
            v = L;
            ++lossless;
          } else {
            const T cand = g0 - delta;
            v = cand < L ? L : cand;
          }
          G[t] = v;
          if (is_cp(fd.cpbits, t))
            ((T *)fd.cp_val)[fd.vo2rank[cp_order(fd.cpbits, fd.cpoff, t)]] = v;
          ++changed;
          floored += v == L;
          first += c == 1;
        }
      }
    }
    __syncthreads();
  }
  __shared__ uint32_t part[5][16];
  const int w = tid >> 6, lane = tid & 63;
  targets = wave_sum(targets);
  changed = wave_sum(changed);
  lossless = wave_sum(lossless);
  floored = wave_sum(floored);
  first = wave_sum(first);
  if (lane == 0) {
    part[0][w] = targets;
    part[1][w] = changed;
    part[2][w] = lossless;
    part[3][w] = floored;
    part[4][w] = first;
  }
  __syncthreads();
  if (tid < 5) {
    uint32_t v = 0;
    for (int k = 0; k < fd.tile_y; ++k) v += part[tid][k];
    if (v) atomicAdd(&st->shard[tid][blockIdx.x & 63], v);
  }
}

// Sums the shards of the apply pass and decides how the loop goes on.
__global__ void __launch_bounds__(64) k_finalize(FieldDev fd) {
  State *st = fd.st;
  if (st->done) return;
  const int lane = threadIdx.x;
  uint32_t v[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    v[k] = wave_sum(st->shard[k][lane]);
    st->shard[k][lane] = 0;
  }
  if (lane != 0) return;
  const uint32_t nt = v[0], ch = v[1];
  if (fd.trace && st->iterations < fd.trace_cap) {
    fd.trace[2 * st->iterations] = nt;
    fd.trace[2 * st->iterations + 1] = ch;
  }
  if (nt == 0) {
    st->done = CONVERGED;
  } else if (ch == 0) {
    st->done = STUCK;
    st->residual = nt;
  } else {
    st->iterations += 1;
    st->edit_ops += ch;
    st->lossless_total += v[2];
    st->floor_total += v[3];
    st->edited_total += v[4];
    if (st->max_iters > 0 && st->iterations >= st->max_iters) st->done = MAXITERS;
  }
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
  st->iterations = st->edit_ops = st->lossless_total = st->floor_total = st->edited_total = 0;
  st->residual = 0;
  st->max_iters = max_iters;
}

hipError_t launch_state_reset(const FieldDev &fd, int64_t max_iters, hipStream_t s) {
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, fd.st, max_iters);
  return hipGetLastError();
}

static size_t plane_bytes(const FieldDev &fd, size_t elem) {
  return 3 * (size_t)HALO_W * (fd.tile_y + 2) * elem;
}

template <class T>
static void launch_check_cpcmp(const FieldDev &fd, const uint32_t *conn, hipStream_t s,
                               hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0) (void)hipEventRecord(ev0, s);
  hipLaunchKernelGGL(k_check<T>, dim3(fd.ntiles), dim3(64, fd.tile_y), plane_bytes(fd, sizeof(T)),
                     s, fd, conn);
  if (ev1) (void)hipEventRecord(ev1, s);
  if (fd.K > 1) hipLaunchKernelGGL(k_cpcmp<T>, dim3((fd.K + 254) / 256), dim3(256), 0, s, fd);
}

template <class T>
static void launch_phases(const FieldDev &fd, const uint32_t *conn, hipStream_t s, hipEvent_t ev0,
                          hipEvent_t ev1) {
  launch_check_cpcmp<T>(fd, conn, s, ev0, ev1);
  hipLaunchKernelGGL(k_apply<T>, dim3(fd.ntiles), dim3(64, fd.tile_y), plane_bytes(fd, 2), s, fd);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, fd);
}

hipError_t launch_iteration(const FieldDev &fd, const uint32_t *conn, hipStream_t s,
                            hipEvent_t ev0, hipEvent_t ev1) {
  if (fd.dtype == 0)
    launch_phases<float>(fd, conn, s, ev0, ev1);
  else
    launch_phases<double>(fd, conn, s, ev0, ev1);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// diagnostics: one check pass, target flags as bytes

hipError_t launch_debug_check(const FieldDev &fd, const uint32_t *conn, hipStream_t s) {
  if (fd.dtype == 0)
    launch_check_cpcmp<float>(fd, conn, s, nullptr, nullptr);
  else
    launch_check_cpcmp<double>(fd, conn, s, nullptr, nullptr);
  return hipGetLastError();
}

__global__ void k_targets_to_bytes(FieldDev fd, uint8_t *out) {
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  bool hit = false;
  if (t < (uint32_t)fd.n) {
    const int x = (int)(t % (uint32_t)fd.nx);
    const uint32_t r = t / (uint32_t)fd.nx;
    const int y = (int)(r % (uint32_t)fd.ny);
    const int z = (int)(r / (uint32_t)fd.ny);
    const uint32_t vm = valid_slots(x, y, z, fd.nx, fd.ny, fd.nz);
    uint32_t h = (fd.req[t] >> SELF) & 1u;
    for (int s = 0; s < NSLOT; ++s)
      if ((vm >> (s ^ 1)) & 1u) h |= (fd.req[t - fd.dlt[s]] >> s) & 1u;
    hit = h != 0;
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
