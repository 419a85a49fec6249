// Setup of one correction: validation of the band, the critical-point
// bitmask (from f's reference topology, which k_ref in loop.hip computes
// box by box with the check's box walk, staging and closed-neighbourhood
// order), the prefix counts that index
// it, the critical-point list and its sorted order.
//
// Paper: steepest ascent/descent neighbours and critical types from local
// comparisons (Sec. 3.1-3.2); the error band |f - g| <= xi (Sec. 4.1); the
// sorted order of the critical points of f (Sec. 4.3).
#include <algorithm>
#include <vector>

#include "exz_host.h"

namespace exz {

// ---------------------------------------------------------------------------
// link component table (host)

void build_component_table(uint8_t *out) {
  // Two slots are joined in the link when their offset difference is itself
  // an offset of the mesh (they span a triangle with the centre vertex).
  uint32_t adj[NSLOT] = {0};
  for (int a = 0; a < NSLOT; ++a)
    for (int b = 0; b < NSLOT; ++b) {
      const int dx = DXS[b] - DXS[a], dy = DYS[b] - DYS[a], dz = DZS[b] - DZS[a];
      for (int s = 0; s < NSLOT; ++s)
        if (DXS[s] == dx && DYS[s] == dy && DZS[s] == dz) adj[a] |= 1u << b;
    }
  for (uint32_t m = 0; m < (1u << NSLOT); ++m) {
    uint32_t left = m;
    int comps = 0;
    while (left) {
      uint32_t comp = left & (~left + 1u);
      for (;;) {
        uint32_t grow = comp;
        for (int s = 0; s < NSLOT; ++s)
          if (comp >> s & 1u) grow |= adj[s];
        grow &= m;
        if (grow == comp) break;
        comp = grow;
      }
      left &= ~comp;
      ++comps;
    }
    out[m] = (uint8_t)comps;
  }
}

void build_connected_bits(const uint8_t *comp, uint32_t *out) {
  for (int w = 0; w < 512; ++w) out[w] = 0;
  for (uint32_t m = 0; m < (1u << NSLOT); ++m)
    if (comp[m] == 1) out[m >> 5] |= 1u << (m & 31);
}

// ---------------------------------------------------------------------------
// setup kernel

constexpr int SETUP_BLOCK = 256;

template <class T>
__global__ void __launch_bounds__(SETUP_BLOCK) k_setup(FieldDev fd) {
  const uint32_t i = blockIdx.x * SETUP_BLOCK + threadIdx.x;
  const bool active = i < (uint32_t)fd.n;
  bool cp = false;
  if (active) {
    const T *F = (const T *)fd.f;
    const T *Gh = (const T *)fd.g_hat;
    const T fi = F[i], gi = Gh[i];
    const T xiT = (T)fd.xiT;
    const T L = lower_bound(fi, xiT);
    if (!isfinite(fi) || !isfinite(gi)) {
      atomicOr(&fd.st->err, ERR_NONFINITE);
    } else {
      if (gi < L || gi > upper_bound(fi, xiT)) atomicOr(&fd.st->err, ERR_BOUND);
    }
    // The edits of a vertex follow one fixed sequence (Sec. 3.3): steps of
    // delta while they stay above L, then one edit that stores L (a clamped
    // step, or the (N+1)-th edit), after which the vertex is blocked.  Its
    // count at that edit is fixed by the value and count it starts from, so
    // apply needs f (for L) only there.
    {
      const uint32_t c0 = fd.resume ? fd.cnt[i] : 0u;
      const T delta = (T)fd.delta;
      uint32_t e = c0;
      if (!(gi == L)) {
        T g = gi;
        for (e = c0 + 1; e <= (uint32_t)fd.N; ++e) {
          const T cand = g - delta;
          if (cand < L || cand == L) break;
          g = cand;
        }
      }
      fd.fe[i] = (uint8_t)min(e, 255u);
    }
    // a maximum is its own steepest ascent, a minimum its own steepest
    // descent (a lone vertex counts as a minimum)
    const uint32_t code = fd.code[i];
    cp = (code & 15u) == SELF || (code >> 4) == SELF || (fd.low[i] & LOW_SADDLE);
    if (fd.g != fd.g_hat) ((T *)fd.g)[i] = gi;
    if (!fd.resume) fd.cnt[i] = 0;
  }
  if (active) fd.tmark[i] = 0;
  if (active && (i & 255u) == 0) fd.mchunk[i >> MARK_CHUNK_SHIFT] = 0;
  if (i < 64) fd.tmark[(uint32_t)fd.n + i] = 0;  // padding
  if (i < (uint32_t)fd.ntiles) fd.bdirty[i] = 0;  // ntiles <= n
  // one 64-bit word of the CP bitmask per wave (waves cover aligned chunks)
  const unsigned long long b = __ballot(cp);
  if ((threadIdx.x & 63) == 0 && active) {
    fd.cpbits[i >> 6] = b;
    fd.cpoff[i >> 6] = (uint32_t)__popcll(b);
  }
}

// The same set-up four vertices per thread, for fields of 4k vertices whose
// buffers allow vector accesses: values by 16-byte loads and stores, the
// byte arrays a 32-bit word at a time.  Each bitmask word (64 vertices, 16
// lanes of quads) is assembled from four ballots, one per position in the
// quad.
typedef float s_f32x4 __attribute__((ext_vector_type(4)));
typedef double s_f64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void load4(const float *p, float *o) {
  const s_f32x4 v = *glob(reinterpret_cast<const s_f32x4 *>(p));
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void load4(const double *p, double *o) {
  const s_f64x2 a = glob(reinterpret_cast<const s_f64x2 *>(p))[0];
  const s_f64x2 b = glob(reinterpret_cast<const s_f64x2 *>(p))[1];
  o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}
__device__ __forceinline__ void store4(float *p, const float *o) {
  s_f32x4 v;
  v.x = o[0]; v.y = o[1]; v.z = o[2]; v.w = o[3];
  *glob(reinterpret_cast<s_f32x4 *>(p)) = v;
}
__device__ __forceinline__ void store4(double *p, const double *o) {
  s_f64x2 a, b;
  a.x = o[0]; a.y = o[1]; b.x = o[2]; b.y = o[3];
  glob(reinterpret_cast<s_f64x2 *>(p))[0] = a;
  glob(reinterpret_cast<s_f64x2 *>(p))[1] = b;
}

// Bit k of the low 16 bits of x moved to bit 4k.
__device__ __forceinline__ unsigned long long spread4(unsigned long long x) {
  x = (x | (x << 24)) & 0x000000FF000000FFull;
  x = (x | (x << 12)) & 0x000F000F000F000Full;
  x = (x | (x << 6)) & 0x0303030303030303ull;
  x = (x | (x << 3)) & 0x1111111111111111ull;
  return x;
}

template <class T>
__global__ void __launch_bounds__(SETUP_BLOCK) k_setup_quad(FieldDev fd) {
  const uint32_t q = blockIdx.x * SETUP_BLOCK + threadIdx.x;
  const uint32_t n = (uint32_t)fd.n, nq = n / 4;
  uint32_t cpn = 0;  // bit c: vertex 4q + c is a critical point of f
  if (q < nq) {
    const uint32_t v = 4u * q;
    T f4[4], g4[4];
    load4((const T *)fd.f + v, f4);
    load4((const T *)fd.g_hat + v, g4);
    const uint32_t code4 = *glob(reinterpret_cast<const uint32_t *>(fd.code + v));
    const uint32_t low01 = *glob(reinterpret_cast<const uint32_t *>(fd.low + v));
    const uint32_t low23 = *glob(reinterpret_cast<const uint32_t *>(fd.low + v + 2));
    const uint32_t c04 = fd.resume ? *glob(reinterpret_cast<const uint32_t *>(fd.cnt + v)) : 0u;
    const T xiT = (T)fd.xiT, delta = (T)fd.delta;
    uint32_t err = 0, fe4 = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const T fi = f4[c], gi = g4[c];
      const T L = lower_bound(fi, xiT);
      if (!isfinite(fi) || !isfinite(gi))
        err |= ERR_NONFINITE;
      else if (gi < L || gi > upper_bound(fi, xiT))
        err |= ERR_BOUND;
      // the count of the edit that stores L (as in k_setup)
      const uint32_t c0 = (c04 >> (8 * c)) & 255u;
      uint32_t e = c0;
      if (!(gi == L)) {
        T g = gi;
        for (e = c0 + 1; e <= (uint32_t)fd.N; ++e) {
          const T cand = g - delta;
          if (cand < L || cand == L) break;
          g = cand;
        }
      }
      fe4 |= min(e, 255u) << (8 * c);
      const uint32_t code = (code4 >> (8 * c)) & 255u;
      const uint32_t lw = ((c < 2 ? low01 : low23) >> (16 * (c & 1))) & 0xFFFFu;
      const bool cp = (code & 15u) == SELF || (code >> 4) == SELF || (lw & LOW_SADDLE);
      cpn |= (uint32_t)cp << c;
    }
    if (err) atomicOr(&fd.st->err, err);
    *glob(reinterpret_cast<uint32_t *>(fd.fe + v)) = fe4;
    if (fd.g != fd.g_hat) store4((T *)fd.g + v, g4);
    if (!fd.resume) *glob(reinterpret_cast<uint32_t *>(fd.cnt + v)) = 0u;
    *glob(reinterpret_cast<uint32_t *>(fd.tmark + v)) = 0u;
    if ((v & 255u) == 0) fd.mchunk[v >> MARK_CHUNK_SHIFT] = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (v + c < (uint32_t)fd.ntiles) fd.bdirty[v + c] = 0;  // ntiles <= n
  }
  if (q < 16) *glob(reinterpret_cast<uint32_t *>(fd.tmark + n + 4u * q)) = 0u;  // padding
  unsigned long long b[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) b[c] = __ballot((cpn >> c) & 1u);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t j = (q - lane) / 16u + lane;  // this lane's word (lanes 0..3)
  if (lane < 4 && (unsigned long long)j * 64u < (unsigned long long)n) {
    const uint32_t sh = 16u * lane;
    unsigned long long word = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) word |= spread4((b[c] >> sh) & 0xFFFFull) << c;
    fd.cpbits[j] = word;
    fd.cpoff[j] = (uint32_t)__popcll(word);
  }
}

// The reference topology box by box (staged through LDS), then validation,
// copies and the critical-point bitmask from its codes (four vertices per
// thread when the field allows it).
hipError_t launch_setup(const FieldDev &fd, const uint32_t *conn, hipStream_t s) {
  const hipError_t e = launch_ref(fd, conn, s);
  if (e != hipSuccess) return e;
  const bool quads = fd.vec && fd.n % 4 == 0 && (uintptr_t)fd.g_hat % 16 == 0;
  if (quads) {
    const int grid = (fd.n / 4 + SETUP_BLOCK - 1) / SETUP_BLOCK;
    if (fd.dtype == 0)
      hipLaunchKernelGGL(k_setup_quad<float>, dim3(grid), dim3(SETUP_BLOCK), 0, s, fd);
    else
      hipLaunchKernelGGL(k_setup_quad<double>, dim3(grid), dim3(SETUP_BLOCK), 0, s, fd);
    return hipGetLastError();
  }
  const int grid = (fd.n + SETUP_BLOCK - 1) / SETUP_BLOCK;
  if (fd.dtype == 0)
    hipLaunchKernelGGL(k_setup<float>, dim3(grid), dim3(SETUP_BLOCK), 0, s, fd);
  else
    hipLaunchKernelGGL(k_setup<double>, dim3(grid), dim3(SETUP_BLOCK), 0, s, fd);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exclusive scan of uint32 (three phases: block sums, scan of the sums,
// block-local scans plus offsets).  out may alias in.  out[count] = total.

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  const int lane = __lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(v, d);
    if (lane >= d) v += t;
  }
  return v;
}

// Exclusive scan across a block of SCAN_BLOCK threads; returns the prefix of
// this thread and the block total in *total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *total) {
  __shared__ uint32_t wsum[SCAN_BLOCK / 64];
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < SCAN_BLOCK / 64; ++k) {
    if (k < w) off += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_sums(const uint32_t *in, uint32_t count,
                                                          uint32_t *sums) {
  const uint32_t base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  uint32_t v = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < count) v += in[base + k];
  uint32_t tot;
  block_exclusive_scan(v, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_top(uint32_t *sums, uint32_t nb) {
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nb; base += SCAN_BLOCK) {
    const uint32_t k = base + threadIdx.x;
    const uint32_t v = k < nb ? sums[k] : 0;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, &tot);
    if (k < nb) sums[k] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_apply(const uint32_t *in, uint32_t *out,
                                                           uint32_t count, const uint32_t *sums,
                                                           uint32_t nb) {
  const uint32_t base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = base + k < count ? in[base + k] : 0;
    sum += v[k];
  }
  uint32_t tot;
  uint32_t run = block_exclusive_scan(sum, &tot) + sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < count) out[base + k] = run;
    run += v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[count] = sums[nb];
}

size_t scan_tmp_words(uint32_t count) {
  return (size_t)(count + SCAN_TILE - 1) / SCAN_TILE + 1;
}

hipError_t launch_scan_u32(const uint32_t *in, uint32_t *out, uint32_t count, uint32_t *tmp,
                           size_t tmp_words, hipStream_t s) {
  const uint32_t nb = (count + SCAN_TILE - 1) / SCAN_TILE;
  if (tmp_words < (size_t)nb + 1) return hipErrorInvalidValue;
  if (nb == 0) {
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_BLOCK), 0, s, tmp, 0u);
    hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(SCAN_BLOCK), 0, s, in, out, 0u, tmp, 0u);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(SCAN_BLOCK), 0, s, in, count, tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_BLOCK), 0, s, tmp, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(SCAN_BLOCK), 0, s, in, out, count, tmp, nb);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// critical-point list in vertex order: sort keys, side table

// Order-preserving unsigned key of a value; -0 and +0 share the key of +0
// because the SoS order compares values with IEEE equality.
__device__ __forceinline__ uint32_t sort_key(float v) {
  uint32_t u = __float_as_uint(v == 0.0f ? 0.0f : v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ unsigned long long sort_key(double v) {
  unsigned long long u = (unsigned long long)__double_as_longlong(v == 0.0 ? 0.0 : v);
  return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}

// The critical points in vertex order (slot vo): their vertex, and the sort
// key of f with the slot as payload.
template <class T>
__global__ void __launch_bounds__(SETUP_BLOCK) k_cp_compact(FieldDev fd, void *keys_,
                                                            uint32_t *vals) {
  const uint32_t i = blockIdx.x * SETUP_BLOCK + threadIdx.x;
  if (i >= (uint32_t)fd.n || !is_cp(fd.cpbits, i)) return;
  const T *F = (const T *)fd.f;
  const uint32_t vo = cp_order(fd.cpbits, fd.cpoff, i);
  fd.cp_vtx[vo] = i;
  vals[vo] = vo;
  using K = decltype(sort_key(T(0)));
  ((K *)keys_)[vo] = sort_key(F[i]);
}

// The same four vertices per thread (quads of a field of 4k vertices with
// 16-byte aligned f): the quad's values in one load when it holds a
// critical point.
template <class T>
__global__ void __launch_bounds__(SETUP_BLOCK) k_cp_compact_quad(FieldDev fd, void *keys_,
                                                                 uint32_t *vals) {
  const uint32_t q = blockIdx.x * SETUP_BLOCK + threadIdx.x;
  if (q >= (uint32_t)fd.n / 4) return;
  const uint32_t v = 4u * q, sh = v & 63u;
  const unsigned long long bits = fd.cpbits[v >> 6];
  const uint32_t m = (uint32_t)(bits >> sh) & 15u;
  if (!m) return;
  uint32_t vo = fd.cpoff[v >> 6] + (uint32_t)__popcll(bits & ((1ull << sh) - 1ull));
  T f4[4];
  load4((const T *)fd.f + v, f4);
  using K = decltype(sort_key(T(0)));
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (!((m >> c) & 1u)) continue;
    fd.cp_vtx[vo] = v + c;
    vals[vo] = vo;
    ((K *)keys_)[vo] = sort_key(f4[c]);
    ++vo;
  }
}

hipError_t launch_cp_compact(const FieldDev &fd, const uint8_t *, void *keys, uint32_t *vals,
                             hipStream_t s) {
  if (fd.vec && fd.n % 4 == 0) {
    const int grid = (fd.n / 4 + SETUP_BLOCK - 1) / SETUP_BLOCK;
    if (fd.dtype == 0)
      hipLaunchKernelGGL(k_cp_compact_quad<float>, dim3(grid), dim3(SETUP_BLOCK), 0, s, fd, keys, vals);
    else
      hipLaunchKernelGGL(k_cp_compact_quad<double>, dim3(grid), dim3(SETUP_BLOCK), 0, s, fd, keys, vals);
    return hipGetLastError();
  }
  const int grid = (fd.n + SETUP_BLOCK - 1) / SETUP_BLOCK;
  if (fd.dtype == 0)
    hipLaunchKernelGGL(k_cp_compact<float>, dim3(grid), dim3(SETUP_BLOCK), 0, s, fd, keys, vals);
  else
    hipLaunchKernelGGL(k_cp_compact<double>, dim3(grid), dim3(SETUP_BLOCK), 0, s, fd, keys, vals);
  return hipGetLastError();
}

// After the stable sort of the keys (payload = vertex-order slot), in two
// passes that read nothing at random (scattered stores cost less here than
// gathers).  In rank order: per slot its rank (a scattered store), and per
// rank whether the next critical point has the lower vertex index (slots
// follow vertex order, so the slots decide; one bit per rank, a word per 32
// ranks from a wave's ballot).  Then in slot order: per rank in f's order
// the vertex and its current value (scattered stores; g is read nearly in
// order).
__global__ void __launch_bounds__(SETUP_BLOCK) k_cp_rank(FieldDev fd, const uint32_t *sorted_vo) {
  const uint32_t r = blockIdx.x * SETUP_BLOCK + threadIdx.x;
  const uint32_t K = (uint32_t)fd.K;
  bool below = false;
  if (r < K) {
    const uint32_t vo = sorted_vo[r];
    fd.cp_rank[vo] = r;
    below = r + 1 < K && sorted_vo[r + 1] < vo;
    if ((r & 255u) == 0) fd.oflag[r >> 8] = 0;
  }
  const unsigned long long b = __ballot(below);
  const uint32_t lane = threadIdx.x & 63u;
  if (lane == 0 && r < K) fd.cp_below[r >> 5] = (uint32_t)b;
  if (lane == 32 && r < K) fd.cp_below[r >> 5] = (uint32_t)(b >> 32);
}

template <class T>
__global__ void __launch_bounds__(SETUP_BLOCK) k_cp_init(FieldDev fd) {
  const uint32_t vo = blockIdx.x * SETUP_BLOCK + threadIdx.x;
  if (vo >= (uint32_t)fd.K) return;
  const uint32_t v = fd.cp_vtx[vo], r = fd.cp_rank[vo];
  fd.cp_idx[r] = v;
  ((T *)fd.cpr)[r] = ((const T *)fd.g)[v];
}

hipError_t launch_cp_init(const FieldDev &fd, const uint32_t *sorted_vo, hipStream_t s) {
  if (fd.K == 0) return hipSuccess;
  const int grid = (fd.K + SETUP_BLOCK - 1) / SETUP_BLOCK;
  hipLaunchKernelGGL(k_cp_rank, dim3(grid), dim3(SETUP_BLOCK), 0, s, fd, sorted_vo);
  if (fd.dtype == 0)
    hipLaunchKernelGGL(k_cp_init<float>, dim3(grid), dim3(SETUP_BLOCK), 0, s, fd);
  else
    hipLaunchKernelGGL(k_cp_init<double>, dim3(grid), dim3(SETUP_BLOCK), 0, s, fd);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// diagnostics: the band bounds as the device computes them

template <class T>
__global__ void k_debug_bounds(const T *f, int64_t n, T xiT, T *L, T *U) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  L[i] = lower_bound(f[i], xiT);
  U[i] = upper_bound(f[i], xiT);
}

hipError_t launch_debug_bounds(int dtype, const void *f, int64_t n, double xiT, void *L, void *U,
                               hipStream_t s) {
  const int grid = (int)((n + 255) / 256);
  if (grid == 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(k_debug_bounds<float>, dim3(grid), dim3(256), 0, s, (const float *)f, n,
                       (float)xiT, (float *)L, (float *)U);
  else
    hipLaunchKernelGGL(k_debug_bounds<double>, dim3(grid), dim3(256), 0, s, (const double *)f, n,
                       xiT, (double *)L, (double *)U);
  return hipGetLastError();
}

}  // namespace exz
