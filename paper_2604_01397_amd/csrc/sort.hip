// Stable LSD radix sort of (key, uint32 payload) pairs, 8-bit digits.
//
// Sorts the critical points of f by value; the payload is their index in
// vertex order, and because the input is in vertex order a stable sort
// yields the Simulation-of-Simplicity order (equal values ascend by index,
// Sec. 3.3 footnote) that the reformulated event constraints compare
// against (Sec. 4.3).
//
// One pass = per-block digit histograms (digit-major), an exclusive scan of
// the histograms, and a stable scatter that orders each tile by digit in LDS
// before writing it out in coalesced runs.
#include "exz_host.h"

namespace exz {

constexpr int RS_BLOCK = 256;
constexpr int RS_WAVES = RS_BLOCK / 64;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_BLOCK * RS_ITEMS;

static_assert(RS_TILE == SORT_TILE, "sort tiles");

// A work-group's tile: its keys [e0, e0 + n) and where its count of digit d
// goes in the digit-major histogram (hist[h0 + d * stride]): one sort over
// all blocks (tiles == nullptr), or the tiles of several fields.
struct TileOf {
  uint32_t e0, n, h0, stride;
};
__device__ __forceinline__ TileOf tile_of(const SortTile *tiles, uint32_t count, uint32_t nblocks) {
  TileOf t;
  if (tiles) {
    const SortTile d = tiles[blockIdx.x];
    t.e0 = d.start;
    t.n = d.count;
    t.h0 = d.hbase + d.t;
    t.stride = d.ntiles;
  } else {
    t.e0 = blockIdx.x * RS_TILE;
    t.n = min((uint32_t)RS_TILE, count - t.e0);
    t.h0 = blockIdx.x;
    t.stride = nblocks;
  }
  return t;
}

template <class K>
__global__ void __launch_bounds__(RS_BLOCK) k_rs_hist(const K *keys, uint32_t count, int shift,
                                                      uint32_t *hist, uint32_t nblocks,
                                                      const SortTile *tiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const TileOf tl = tile_of(tiles, count, nblocks);
  for (int r = 0; r < RS_ITEMS; ++r) {
    const uint32_t i = r * RS_BLOCK + threadIdx.x;
    if (i < tl.n) atomicAdd(&h[(uint32_t)(keys[tl.e0 + i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * tl.stride + tl.h0] = h[threadIdx.x];
}

// Stable scatter of one tile of RS_TILE elements.  Wave w owns the tile's
// elements w * 64 * RS_ITEMS .. (w + 1) * 64 * RS_ITEMS - 1 and ranks them in
// order, round by round, against digit counters of its own in LDS (lanes
// holding the same digit are found with eight ballots; the lowest of them
// advances the counter after all have read it, so no barrier is needed
// inside the wave's loop).  One barrier later the counters become each
// wave's offset within each digit of the tile, the tile's digits are laid
// out in LDS in digit order (an exclusive scan of the tile's counts), the
// elements are placed there, and the tile is written out run by run:
// consecutive threads write consecutive positions of one digit's output
// range, so the stores coalesce.  offs is the scanned digit-major
// histogram; the tile's own count of digit d is the difference of two
// neighbouring entries.
template <class K>
__global__ void __launch_bounds__(RS_BLOCK) k_rs_scatter(const K *kin, const uint32_t *vin, K *kout,
                                                         uint32_t *vout, uint32_t count, int shift,
                                                         const uint32_t *offs, uint32_t nblocks,
                                                         const SortTile *tiles) {
  __shared__ K sk[RS_TILE];
  __shared__ uint32_t sv[RS_TILE];
  __shared__ uint32_t gbase[256];   // output position of the tile's first element of digit d
  __shared__ uint32_t lstart[256];  // first LDS slot of digit d
  __shared__ uint32_t wcnt[RS_WAVES][256];
  __shared__ uint32_t wtot[RS_WAVES];
  const int lane = __lane_id(), w = threadIdx.x >> 6, t = threadIdx.x;
  const TileOf tl = tile_of(tiles, count, nblocks);
  const uint32_t hidx = (uint32_t)t * tl.stride + tl.h0;
  const uint32_t g0 = offs[hidx];
  const uint32_t c = offs[hidx + 1] - g0;  // this tile's count of digit t
  gbase[t] = g0;
#pragma unroll
  for (int k = 0; k < RS_WAVES; ++k) wcnt[k][t] = 0;
  __syncthreads();
  const unsigned long long below = (1ull << lane) - 1ull;
  const uint32_t wbase = (uint32_t)w * (64u * RS_ITEMS);  // the wave's first key in the tile
  K key[RS_ITEMS];
  uint32_t val[RS_ITEMS], rk[RS_ITEMS];  // rank within the wave's digit | digit << 16
#pragma unroll
  for (int r = 0; r < RS_ITEMS; ++r) {
    const uint32_t e = wbase + (uint32_t)r * 64u + (uint32_t)lane;
    const bool valid = e < tl.n;
    key[r] = 0;
    val[r] = 0;
    uint32_t d = 0;
    if (valid) {
      key[r] = kin[tl.e0 + e];
      val[r] = vin[tl.e0 + e];
      d = (uint32_t)(key[r] >> shift) & 255u;
    }
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const unsigned long long bb = __ballot(valid && on);
      m &= on ? bb : ~bb;
    }
    const uint32_t before = wcnt[w][d];
    rk[r] = (before + (uint32_t)__popcll(m & below)) | (d << 16);
    // the wave's LDS accesses complete in order: every lane has read the
    // counter before its lowest lane advances it
    if (valid && lane == __ffsll((long long)m) - 1) wcnt[w][d] = before + (uint32_t)__popcll(m);
  }
  __syncthreads();
  // per digit (thread t): each wave's offset within the tile's digit t
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < RS_WAVES; ++k) {
    const uint32_t x = wcnt[k][t];
    wcnt[k][t] = acc;
    acc += x;
  }
  // exclusive scan of the tile's digit counts: waves, then across waves
  uint32_t inc = c;
#pragma unroll
  for (int dd = 1; dd < 64; dd <<= 1) {
    const uint32_t o = __shfl_up(inc, dd);
    if (lane >= dd) inc += o;
  }
  if (lane == 63) wtot[w] = inc;
  __syncthreads();
  uint32_t woff = 0;
#pragma unroll
  for (int k = 0; k < RS_WAVES; ++k) woff += k < w ? wtot[k] : 0u;
  lstart[t] = woff + inc - c;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RS_ITEMS; ++r) {
    const uint32_t e = wbase + (uint32_t)r * 64u + (uint32_t)lane;
    if (e < tl.n) {
      const uint32_t d = rk[r] >> 16;
      const uint32_t pos = lstart[d] + wcnt[w][d] + (rk[r] & 0xFFFFu);
      sk[pos] = key[r];
      sv[pos] = val[r];
    }
  }
  __syncthreads();
  for (uint32_t j = t; j < tl.n; j += RS_BLOCK) {
    const K k = sk[j];
    const uint32_t d = (uint32_t)(k >> shift) & 255u;
    const uint32_t pos = gbase[d] + (j - lstart[d]);
    kout[pos] = k;
    vout[pos] = sv[j];
  }
}

size_t radix_hist_words(uint32_t count) {
  const uint32_t nblocks = (count + RS_TILE - 1) / RS_TILE;
  return (size_t)256 * (nblocks ? nblocks : 1) + 1;
}

template <class K>
static hipError_t sort_impl(K *keys, uint32_t *vals, K *ktmp, uint32_t *vtmp, uint32_t count,
                            uint32_t *hist, uint32_t *scan_tmp, size_t scan_words, hipStream_t s) {
  if (count <= 1) return hipSuccess;
  const uint32_t nblocks = (count + RS_TILE - 1) / RS_TILE;
  K *ka = keys, *kb = ktmp;
  uint32_t *va = vals, *vb = vtmp;
  for (int shift = 0; shift < (int)(8 * sizeof(K)); shift += 8) {
    hipLaunchKernelGGL(k_rs_hist<K>, dim3(nblocks), dim3(RS_BLOCK), 0, s, ka, count, shift, hist,
                       nblocks, (const SortTile *)nullptr);
    hipError_t e = launch_scan_u32(hist, hist, 256u * nblocks, scan_tmp, scan_words, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rs_scatter<K>, dim3(nblocks), dim3(RS_BLOCK), 0, s, ka, va, kb, vb, count,
                       shift, hist, nblocks, (const SortTile *)nullptr);
    K *kt = ka; ka = kb; kb = kt;
    uint32_t *vt = va; va = vb; vb = vt;
  }
  // an even number of passes leaves the result in (keys, vals)
  return hipGetLastError();
}

// The same passes over the tiles of several fields' keys (see SortTile): one
// histogram and one scatter launch per pass for all of them.
template <class K>
static hipError_t sort_tiles_impl(K *keys, uint32_t *vals, K *ktmp, uint32_t *vtmp, uint32_t count,
                                  const SortTile *tiles, uint32_t ntiles, uint32_t *hist,
                                  uint32_t *scan_tmp, size_t scan_words, hipStream_t s) {
  if (ntiles == 0) return hipSuccess;
  K *ka = keys, *kb = ktmp;
  uint32_t *va = vals, *vb = vtmp;
  for (int shift = 0; shift < (int)(8 * sizeof(K)); shift += 8) {
    hipLaunchKernelGGL(k_rs_hist<K>, dim3(ntiles), dim3(RS_BLOCK), 0, s, ka, count, shift, hist,
                       ntiles, tiles);
    hipError_t e = launch_scan_u32(hist, hist, 256u * ntiles, scan_tmp, scan_words, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rs_scatter<K>, dim3(ntiles), dim3(RS_BLOCK), 0, s, ka, va, kb, vb, count,
                       shift, hist, ntiles, tiles);
    K *kt = ka; ka = kb; kb = kt;
    uint32_t *vt = va; va = vb; vb = vt;
  }
  // an even number of passes leaves the result in (keys, vals)
  return hipGetLastError();
}

hipError_t launch_radix_sort_tiles(int key_bytes, void *keys, uint32_t *vals, void *keys_tmp,
                                   uint32_t *vals_tmp, uint32_t count, const SortTile *tiles,
                                   uint32_t ntiles, uint32_t *hist, uint32_t *scan_tmp,
                                   size_t scan_words, hipStream_t s) {
  if (key_bytes == 4)
    return sort_tiles_impl<uint32_t>((uint32_t *)keys, vals, (uint32_t *)keys_tmp, vals_tmp, count,
                                     tiles, ntiles, hist, scan_tmp, scan_words, s);
  if (key_bytes == 8)
    return sort_tiles_impl<unsigned long long>((unsigned long long *)keys, vals,
                                               (unsigned long long *)keys_tmp, vals_tmp, count,
                                               tiles, ntiles, hist, scan_tmp, scan_words, s);
  return hipErrorInvalidValue;
}

hipError_t launch_radix_sort(int key_bytes, void *keys, uint32_t *vals, void *keys_tmp,
                             uint32_t *vals_tmp, uint32_t count, uint32_t *hist, uint32_t *scan_tmp,
                             size_t scan_words, hipStream_t s) {
  if (key_bytes == 4)
    return sort_impl<uint32_t>((uint32_t *)keys, vals, (uint32_t *)keys_tmp, vals_tmp, count, hist,
                               scan_tmp, scan_words, s);
  if (key_bytes == 8)
    return sort_impl<unsigned long long>((unsigned long long *)keys, vals,
                                         (unsigned long long *)keys_tmp, vals_tmp, count, hist,
                                         scan_tmp, scan_words, s);
  return hipErrorInvalidValue;
}

}  // namespace exz
