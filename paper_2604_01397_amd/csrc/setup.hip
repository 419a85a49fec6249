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

// The reference topology box by box (staged through LDS), then validation,
// copies and the critical-point bitmask from its codes.
hipError_t launch_setup(const FieldDev &fd, const uint32_t *conn, hipStream_t s) {
  const hipError_t e = launch_ref(fd, conn, s);
  if (e != hipSuccess) return e;
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

hipError_t launch_cp_compact(const FieldDev &fd, const uint8_t *, void *keys, uint32_t *vals,
                             hipStream_t s) {
  const int grid = (fd.n + SETUP_BLOCK - 1) / SETUP_BLOCK;
  if (fd.dtype == 0)
    hipLaunchKernelGGL(k_cp_compact<float>, dim3(grid), dim3(SETUP_BLOCK), 0, s, fd, keys, vals);
  else
    hipLaunchKernelGGL(k_cp_compact<double>, dim3(grid), dim3(SETUP_BLOCK), 0, s, fd, keys, vals);
  return hipGetLastError();
}

// After the stable sort of the keys (payload = vertex-order slot): per rank
// in f's order the vertex and the current value (read in rank order, the
// slot's vertex and value gathered), per slot its rank (a scattered store),
// and per rank whether the next critical point has the lower vertex index
// (slots follow vertex order, so the slots decide; one bit per rank, a word
// per 32 ranks from a wave's ballot).
template <class T>
__global__ void __launch_bounds__(SETUP_BLOCK) k_cp_init(FieldDev fd, const uint32_t *sorted_vo) {
  const uint32_t r = blockIdx.x * SETUP_BLOCK + threadIdx.x;
  const uint32_t K = (uint32_t)fd.K;
  bool below = false;
  if (r < K) {
    const uint32_t vo = sorted_vo[r];
    const uint32_t v = fd.cp_vtx[vo];
    fd.cp_idx[r] = v;
    fd.cp_rank[vo] = r;
    ((T *)fd.cpr)[r] = ((const T *)fd.g)[v];
    below = r + 1 < K && sorted_vo[r + 1] < vo;
    if ((r & 255u) == 0) fd.oflag[r >> 8] = 0;
  }
  const unsigned long long b = __ballot(below);
  const uint32_t lane = threadIdx.x & 63u;
  if (lane == 0 && r < K) fd.cp_below[r >> 5] = (uint32_t)b;
  if (lane == 32 && r < K) fd.cp_below[r >> 5] = (uint32_t)(b >> 32);
}

hipError_t launch_cp_init(const FieldDev &fd, const uint32_t *sorted_vo, hipStream_t s) {
  if (fd.K == 0) return hipSuccess;
  const int grid = (fd.K + SETUP_BLOCK - 1) / SETUP_BLOCK;
  if (fd.dtype == 0)
    hipLaunchKernelGGL(k_cp_init<float>, dim3(grid), dim3(SETUP_BLOCK), 0, s, fd, sorted_vo);
  else
    hipLaunchKernelGGL(k_cp_init<double>, dim3(grid), dim3(SETUP_BLOCK), 0, s, fd, sorted_vo);
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
