// Device building blocks of one correction iteration on the 14-neighbour
// Freudenthal mesh, shared by the single-field kernels (loop.hip) and the
// batched ones (batch.hip): box staging, the per-vertex check, the
// critical-point pair compare, the per-box apply and counter reduction.
#pragma once

#include "exz_internal.h"

namespace exz {

constexpr int HALO_W = 66;  // 64 columns + a halo cell on both sides

template <int TY, int TZ>
struct Box {
  static constexpr int W = HALO_W, H = TY + 2, D = TZ + 2;
  static constexpr int PLANE = W * H, NE = W * H * D, NT = 64 * TY;
  static constexpr int R = (NE + NT - 1) / NT;  // staged values per thread
};

struct BoxOrigin {
  int x0, y0, z0;
};

__device__ __forceinline__ BoxOrigin box_of(const FieldDev &fd, uint32_t tile, int TY, int TZ) {
  const uint32_t tx = tile % (uint32_t)fd.tiles_x;
  const uint32_t r = tile / (uint32_t)fd.tiles_x;
  const uint32_t ty = r % (uint32_t)fd.tiles_y;
  const uint32_t tz = r / (uint32_t)fd.tiles_y;
  return BoxOrigin{(int)tx * 64, (int)ty * TY, (int)tz * TZ};
}

// Value staged for cells outside the domain: NaN for field values (every
// IEEE comparison with it is false, so an absent neighbour is never lower,
// higher, the maximum or the minimum), 0 for request masks (no request).
template <class V> __device__ __forceinline__ V outside_value() { return V(0); }
template <> __device__ __forceinline__ float outside_value<float>() { return __int_as_float(0x7FC00000); }
template <> __device__ __forceinline__ double outside_value<double>() {
  return __longlong_as_double(0x7FF8000000000000ll);
}

// Staging of a box plus its one-cell halo into LDS.  Each thread's element
// offsets (relative to the halo's first cell) are the same for every box,
// so they are computed once per kernel.  A box whose halo lies inside the
// domain -- most of them -- loads with one add per element; a box at the
// domain boundary clamps coordinates so every load stays valid and then
// overwrites the cells outside the domain with outside_value().  Loads are
// unconditional and their values always stored, so all of a thread's loads
// are in flight at once (a value used on one path only invites the compiler
// to move its load under that branch, one round trip per element).
template <int TY, int TZ>
struct StageMap {
  using B = Box<TY, TZ>;
  uint32_t off[B::R];  // element offset from the halo origin, in the field
  uint32_t cell[B::R]; // (xx, yy, zz) of the element, packed 8:8:8
};

template <int TY, int TZ>
__device__ __forceinline__ void stage_map(const FieldDev &fd, int tid, StageMap<TY, TZ> &m) {
  using B = Box<TY, TZ>;
#pragma unroll
  for (int k = 0; k < B::R; ++k) {
    const int e = min(tid + k * B::NT, B::NE - 1);
    const int zz = e / B::PLANE, rem = e - zz * B::PLANE;
    const int yy = rem / B::W, xx = rem - yy * B::W;
    m.off[k] = (uint32_t)xx + (uint32_t)fd.nx * ((uint32_t)yy + (uint32_t)fd.ny * (uint32_t)zz);
    m.cell[k] = (uint32_t)xx | ((uint32_t)yy << 8) | ((uint32_t)zz << 16);
  }
}

template <int TY, int TZ, class V>
__device__ __forceinline__ void stage_box(const FieldDev &fd, const V *src, V *S, BoxOrigin o,
                                          int tid, const StageMap<TY, TZ> &m) {
  using B = Box<TY, TZ>;
  V r[B::R];
  const bool interior = o.x0 >= 1 && o.x0 + 64 <= fd.nx - 1 && o.y0 >= 1 &&
                        o.y0 + TY <= fd.ny - 1 && o.z0 >= 1 && o.z0 + TZ <= fd.nz - 1;
  uint32_t outside = 0;
  if (interior) {
    const V *base = src + ((uint32_t)(o.x0 - 1) +
                           (uint32_t)fd.nx * ((uint32_t)(o.y0 - 1) + (uint32_t)fd.ny * (uint32_t)(o.z0 - 1)));
#pragma unroll
    for (int k = 0; k < B::R; ++k) r[k] = base[m.off[k]];
  } else {
#pragma unroll
    for (int k = 0; k < B::R; ++k) {
      const int gx = o.x0 - 1 + (int)(m.cell[k] & 255u);
      const int gy = o.y0 - 1 + (int)((m.cell[k] >> 8) & 255u);
      const int gz = o.z0 - 1 + (int)(m.cell[k] >> 16);
      const bool in = (gx >= 0) & (gx < fd.nx) & (gy >= 0) & (gy < fd.ny) & (gz >= 0) & (gz < fd.nz);
      outside |= (uint32_t)!in << k;
      const uint32_t cx = (uint32_t)min(max(gx, 0), fd.nx - 1);
      const uint32_t cy = (uint32_t)min(max(gy, 0), fd.ny - 1);
      const uint32_t cz = (uint32_t)min(max(gz, 0), fd.nz - 1);
      r[k] = src[cx + (uint32_t)fd.nx * (cy + (uint32_t)fd.ny * cz)];
    }
  }
#pragma unroll
  for (int k = 0; k < B::R; ++k) {
    const int e = tid + k * B::NT;
    if (e < B::NE) S[e] = r[k];
  }
  if (outside) {
#pragma unroll
    for (int k = 0; k < B::R; ++k) {
      const int e = tid + k * B::NT;
      if (e < B::NE && ((outside >> k) & 1u)) S[e] = outside_value<V>();
    }
  }
}

// Requests of one vertex as a slot mask (bit SELF = the vertex itself).
// P points at the LDS centre value of the vertex; pm / pp are the offsets
// of the planes below / above relative to the centre plane.
template <class T>
__device__ __forceinline__ uint32_t check_vertex(const FieldDev &fd, const uint32_t *__restrict__ conn,
                                                 const T *P, int pm, int pp, int x, int y, int z,
                                                 uint32_t i, uint32_t codeb, uint32_t lowf,
                                                 uint32_t &asc_v, uint32_t &desc_v, bool interior) {
  // Vertex indices of the neighbours, ascending: the slots with a negative
  // offset (odd), the vertex itself, the slots with a positive offset (even).
  // Offsets are dx + nx*dy + nx*ny*dz, ordered lexicographically by
  // (dz, dy, dx) on any grid where the slot is in the domain.
  constexpr int ORDER[NSLOT + 1] = {13, 11, 9, 7, 5, 3, 1, SELF, 0, 2, 4, 6, 8, 10, 12};
  const uint32_t vm = interior ? 0x3FFFu : slots_in_domain(x, y, z, fd.nx, fd.ny, fd.nz);
  const T gi = P[0];
  T gn[NSLOT];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int po = DZS[s] < 0 ? pm : DZS[s] > 0 ? pp : 0;
    gn[s] = P[po + DYS[s] * HALO_W + DXS[s]];
  }
  // One pass in index order: with ">=" a later (higher-index) candidate wins
  // a tie, which is the SoS maximum; with "<" the earlier (lower-index) one
  // keeps it, which is the SoS minimum.  A neighbour with a lower index is
  // below i when its value is <= g_i, one with a higher index when it is
  // < g_i.  NaN (outside the domain) never compares true.
  T bmax = -INFINITY, bmin = INFINITY;
  int asc = SELF, desc = SELF;
  uint32_t lower = 0;
#pragma unroll
  for (int q = 0; q <= NSLOT; ++q) {
    const int s = ORDER[q];
    const T v = s == SELF ? gi : gn[s];
    if (s != SELF) lower |= (uint32_t)(q < 7 ? v <= gi : v < gi) << s;
    const bool up = v >= bmax;
    bmax = up ? v : bmax;
    asc = up ? s : asc;
    const bool dn = v < bmin;
    bmin = dn ? v : bmin;
    desc = dn ? s : desc;
  }
  if (fd.mode == 1) {  // vertex indices are needed for path tracing only
    asc_v = (uint32_t)((int)i + fd.dlt[asc]);
    desc_v = (uint32_t)((int)i + fd.dlt[desc]);
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

// Adds the targets named by vertex i's request mask r (bit s: the neighbour
// in slot s, bit SELF: i itself).
__device__ __forceinline__ void post_targets(const FieldDev &fd, uint32_t i, uint32_t r) {
  if ((r >> SELF) & 1u) mark_target(fd.tbits, i);
  r &= LOW_MASK;
  while (r) {
    const int s = __ffs(r) - 1;
    r &= r - 1;
    mark_target(fd.tbits, (uint32_t)((int)i + fd.dlt[s]));
  }
}

// Vertices of the box inside the domain.
__device__ __forceinline__ uint32_t box_vertices(const FieldDev &fd, BoxOrigin o, int TY, int TZ) {
  return (uint32_t)(min(64, fd.nx - o.x0) * min(TY, fd.ny - o.y0) * min(TZ, fd.nz - o.z0));
}

// CheckConstraints on one box: stage g, add the targets every vertex names
// to the target set (and, in original mode, write g's descent / ascent
// pointers).
template <class T, int TY, int TZ>
__device__ __forceinline__ void check_box(const FieldDev &fd, const uint32_t *__restrict__ conn,
                                          BoxOrigin o, T *S, const StageMap<TY, TZ> &m) {
  using B = Box<TY, TZ>;
  const int lx = threadIdx.x, ly = threadIdx.y, tid = ly * 64 + lx;
  const int x = o.x0 + lx, y = o.y0 + ly;
  const bool col = x < fd.nx && y < fd.ny;
  const uint32_t plane = (uint32_t)fd.nx * (uint32_t)fd.ny;
  const uint32_t i0 = (uint32_t)x + (uint32_t)fd.nx * ((uint32_t)y + (uint32_t)fd.ny * (uint32_t)o.z0);
  uint32_t codes[TZ], lows[TZ];
#pragma unroll
  for (int k = 0; k < TZ; ++k) {  // issued with the staging loads, unconditionally
    const bool in = col && o.z0 + k < fd.nz;
    const uint32_t idx = in ? i0 + k * plane : 0u;
    const uint32_t cb = fd.code[idx], lb = fd.low[idx];
    codes[k] = in ? cb : 0u;
    lows[k] = in ? lb : 0u;
  }
  stage_box<TY, TZ>(fd, (const T *)fd.g, S, o, tid, m);
  const bool interior = o.x0 >= 1 && o.x0 + 64 <= fd.nx - 1 && o.y0 >= 1 &&
                        o.y0 + TY <= fd.ny - 1 && o.z0 >= 1 && o.z0 + TZ <= fd.nz - 1;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < TZ; ++k) {
    const int z = o.z0 + k;
    if (col && z < fd.nz) {
      const uint32_t i = i0 + k * plane;
      const T *c = S + (k + 1) * B::PLANE + (ly + 1) * B::W + lx + 1;
      uint32_t av = 0, dv = 0;
      const uint32_t r = check_vertex<T>(fd, conn, c, -B::PLANE, B::PLANE, x, y, z, i, codes[k],
                                         lows[k], av, dv, interior);
      if (r) post_targets(fd, i, r);
      if (fd.mode == 1) {  // original event constraints trace g's integral paths
        fd.lab[i] = dv;
        fd.lab[fd.n + i] = (uint32_t)fd.n + av;
      }
    }
  }
}

// Reformulated event constraints: consecutive critical points in f's order
// must keep their order in g; an inverted pair decreases the lower one.
// Values are finite, so b > a settles most pairs without the vertex indices.
template <class T>
__device__ __forceinline__ void cp_pair(const FieldDev &fd, uint32_t r) {
  const T *V = (const T *)fd.cp_val;
  const T a = V[r], b = V[r + 1];
  if (b > a) return;
  const uint32_t ia = fd.cp_idx[r], ib = fd.cp_idx[r + 1];
  if (sos_lt(b, ib, a, ia)) mark_target(fd.tbits, ia);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  return v;
}

// ApplyBoundedEdits: each target moves once, from its own value, by one step
// of Delta (never below L); its (N+1)-th edit stores L itself; a target that
// already sits on L cannot move.  Counters are reduced per work-group and
// added to one of 64 shards.
struct EditCount {
  uint32_t v[5];  // targets, changed, lossless, floored, first edits
};

// Marks every box whose check reads vertex t (the box plus its one-cell
// halo contains t), so the next frontier check visits it.
__device__ __forceinline__ void mark_boxes(const FieldDev &fd, uint32_t t) {
  const uint32_t x = t % (uint32_t)fd.nx, r = t / (uint32_t)fd.nx;
  const uint32_t y = r % (uint32_t)fd.ny, z = r / (uint32_t)fd.ny;
  const uint32_t ty = (uint32_t)fd.tile_y, tz = (uint32_t)fd.tile_z;
  const uint32_t bx0 = x ? (x - 1) >> 6 : 0, bx1 = min((x + 1) >> 6, (uint32_t)fd.tiles_x - 1);
  const uint32_t by0 = y ? (y - 1) / ty : 0, by1 = min((y + 1) / ty, (uint32_t)fd.tiles_y - 1);
  const uint32_t bz0 = z ? (z - 1) / tz : 0, bz1 = min((z + 1) / tz, (uint32_t)fd.tiles_z - 1);
  for (uint32_t bz = bz0; bz <= bz1; ++bz)
    for (uint32_t by = by0; by <= by1; ++by)
      for (uint32_t bx = bx0; bx <= bx1; ++bx)
        fd.bdirty[bx + (uint32_t)fd.tiles_x * (by + (uint32_t)fd.tiles_y * bz)] = 1;
}

// ApplyBoundedEdits on the 32 vertices of target word w; clears the word
// and adds this thread's counts to ec.  In frontier mode every vertex whose
// value or count moved marks the boxes that read it.
template <class T>
__device__ __forceinline__ void apply_word(const FieldDev &fd, uint32_t w, EditCount &ec) {
  uint32_t bits = fd.tbits[w];
  if (!bits) return;
  fd.tbits[w] = 0;
  ec.v[0] += (uint32_t)__popc(bits);
  T *G = (T *)fd.g;
  const T *F = (const T *)fd.f;
  const T xiT = (T)fd.xiT, delta = (T)fd.delta;
  while (bits) {
    const uint32_t t = w * 32u + (uint32_t)(__ffs(bits) - 1);
    bits &= bits - 1;
    const T g0 = G[t], fv = F[t];
    const uint32_t c0 = fd.cnt[t], rk = fd.rank_of[t];
    const T L = lower_bound(fv, xiT);
    if (g0 == L) continue;  // at the floor: blocked
    const uint32_t c = c0 + 1;
    fd.cnt[t] = (uint8_t)c;
    T v;
    if (c > (uint32_t)fd.N) {
      v = L;  // (N+1)-th edit: store the lower bound itself
      ++ec.v[2];
    } else {
      const T cand = g0 - delta;
      v = cand < L ? L : cand;
    }
    G[t] = v;
    if (rk != 0xFFFFFFFFu) ((T *)fd.cp_val)[rk] = v;
    ++ec.v[1];
    ec.v[3] += v == L;
    ec.v[4] += c == 1;
    if (fd.frontier) mark_boxes(fd, t);
  }
}

// Work-group size of the apply passes (threads, one target word each).
constexpr int APPLY_BLOCK = 256;

// Block reduction of the edit counts, added to one of the field's 64 shards.
template <int TY>
__device__ __forceinline__ void flush_counts(State *st, EditCount ec, uint32_t shard) {
  __shared__ uint32_t part[5][TY];
  const int tid = threadIdx.y * 64 + threadIdx.x, w = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const uint32_t v = wave_sum(ec.v[k]);
    if (lane == 0) part[k][w] = v;
  }
  __syncthreads();
  if (tid < 5) {
    uint32_t v = 0;
    for (int k = 0; k < TY; ++k) v += part[tid][k];
    if (v) atomicAdd(&st->shard[tid][shard & 63u], v);
  }
}

// Sums the shards of the apply pass and decides how the loop goes on.
__device__ __forceinline__ void finalize_field(const FieldDev &fd) {
  State *st = fd.st;
  if (st->done) return;
  const int lane = threadIdx.x;
  if (lane == 0) st->passes += 1;
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
  if (ch == 0 && fd.frontier && !st->dense) {
    // A frontier pass skips boxes whose requests were all blocked, so it
    // cannot tell a fixpoint from convergence (or count the residual): one
    // dense pass over the unchanged field settles it.
    st->dense = 1;
  } else if (nt == 0) {
    st->done = CONVERGED;
  } else if (ch == 0) {
    st->done = STUCK;
    st->residual = nt;
  } else {
    st->dense = 0;
    st->iterations += 1;
    st->edit_ops += ch;
    st->lossless_total += v[2];
    st->floor_total += v[3];
    st->edited_total += v[4];
    if (st->max_iters > 0 && st->iterations >= st->max_iters) st->done = MAXITERS;
  }
}


// Box shapes (TY, TZ) with compiled kernels; the tile_y / tile_z options
// pick one of them.
#define EXZ_BOX_SHAPES(X) \
  X(1, 1) X(2, 2) X(4, 1) X(4, 2) X(4, 4) X(8, 1) X(8, 2) X(8, 4) X(4, 8) X(16, 1) X(16, 2)

}  // namespace exz
