// Internal declarations of the gfx950 EXaCTz library: the per-field device
// descriptor, the loop state, device helpers shared by the kernels and the
// host-side launch wrappers.  Not part of the public ABI (include/exactz.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace exz {

// ---------------------------------------------------------------------------
// Mesh: the Freudenthal triangulation of the grid.  Slot s is the neighbour
// at offset (DX[s], DY[s], DZ[s]); slot 14 stands for the vertex itself.
// Slots 0..5 are the in-plane offsets, so a 2D field (nz = 1) and a 1D field
// (ny = nz = 1) use the same tables with the out-of-domain slots masked off.
constexpr int NSLOT = 14;
constexpr int SELF = 14;
constexpr int DXS[NSLOT] = {+1, -1, 0, 0, +1, -1, 0, 0, +1, -1, 0, 0, +1, -1};
constexpr int DYS[NSLOT] = {0, 0, +1, -1, +1, -1, 0, 0, 0, 0, +1, -1, +1, -1};
constexpr int DZS[NSLOT] = {0, 0, 0, 0, 0, 0, +1, -1, +1, -1, +1, -1, +1, -1};

// Reference topology of f, per vertex, in two dense arrays:
//   code  (1 byte)  ascent slot in the low nibble, descent slot in the high
//                   nibble (SELF for a maximum / minimum);
//   low   (2 bytes) lower-link slot mask in bits 0..13, LOW_SADDLE if the
//                   vertex is a saddle of f.
// Both are read with coalesced loads by the check pass.
constexpr uint32_t LOW_SADDLE = 1u << 15;
constexpr uint32_t LOW_MASK = 0x3FFFu;
constexpr uint32_t NONE = 0xFFFFFFFFu;  // no vertex / no box

enum Done : int32_t { RUNNING = 0, CONVERGED = 1, STUCK = 2, MAXITERS = 3 };
constexpr int MAX_JUMP_ROUNDS = 34;  // pointer jumping over < 2^32 labels
enum SetupErr : uint32_t { ERR_NONFINITE = 1u, ERR_BOUND = 2u };

// Device-resident loop state of one field.  Per-iteration counters are
// reset by the finalize step; totals accumulate over the call.
struct State {
  int32_t done;
  uint32_t err;
  uint32_t ntargets;   // |S| of the current iteration (worklist length)
  uint32_t changed;    // values changed by the current iteration
  uint32_t lossless;   // (N+1)-th edits in the current iteration
  uint32_t floored;    // edits that landed on L in the current iteration
  uint32_t first;      // edits that took a count from 0 to 1
  uint32_t cert_bad;   // certificate mismatches
  uint32_t shard[5][64];  // per-iteration counters of the apply pass, sharded by block
  uint32_t nsaddle;       // saddles of f (original mode)
  int32_t dense;          // the next check covers every box (first pass, fixpoint confirmation)
  int32_t noflag;         // this iteration's apply sets no box flags (the next check is dense)
  int32_t busy;           // the last apply changed many values (> n / 64): the next apply
                          // fetches every quad's counts ahead
  uint32_t tag;           // mark byte of this pass's targets (1 .. MARK_TAGS)
  uint32_t nfront;        // boxes in the frontier list (single-field loop)
  uint32_t jump[MAX_JUMP_ROUNDS];  // pointer-jumping round flags
  int64_t iterations;
  int64_t edit_ops;
  int64_t lossless_total;
  int64_t floor_total;
  int64_t edited_total;
  int64_t targets_total;          // sum of |S| over the iterations that changed a value
  int64_t residual;
  int64_t max_iters;
  int64_t passes;                 // check passes that ran (profiling)
  unsigned long long checked;     // vertices those passes checked (profiling)
};

// Everything a kernel needs to work on one field.  Passed by value to the
// single-field kernels and stored in a device array for the batched ones.
struct FieldDev {
  int32_t nx, ny, nz, n;
  int32_t nchunk;       // ceil(n / 64): 64-vertex chunks of the CP bitmask
  int32_t dtype;        // 0 float32, 1 float64
  int32_t N;            // n_steps
  int32_t mode;         // event mode
  int32_t K;            // number of critical points of f
  int32_t Ks;           // number of saddles of f
  int32_t resume;
  int32_t tile_y, tile_z;    // stencil boxes of 64 x tile_y x tile_z vertices
  int32_t tiles_x, tiles_y, tiles_z;
  int32_t ntiles;            // tiles_x * tiles_y * tiles_z
  int32_t grid_blocks;       // stencil grid: 0 one block per box, < 0 persistent default, > 0 fixed
  int32_t trace_cap;
  int32_t frontier;     // 1: re-check only boxes whose closed neighbourhood changed
  int32_t ty_shift, tz_shift;  // log2 of tile_y / tile_z
  int32_t vec;          // f, g 16-byte and cnt 4-byte aligned: apply reads four vertices at once
  int32_t dlt[16];      // linear index offset of each slot (dlt[SELF] = 0)
  double xiT, delta;    // in the field type, widened exactly to double
  const void *f;
  const void *g_hat;
  void *g;              // the field being corrected (g_out)
  uint8_t *cnt;
  uint8_t *fe;          // n: the edit count at which the vertex's value reaches its lower
                        // bound (the edits before it are plain steps of delta)
  uint8_t *code;
  uint16_t *low;
  unsigned long long *cpbits;
  uint32_t *cpoff;      // nchunk + 1 exclusive prefix counts
  uint32_t *cp_vtx;     // K, vertex order -> vertex
  uint32_t *cp_rank;    // K, vertex order: rank in f's order
  uint32_t *cp_below;   // (K + 31) / 32 words, bit r: the critical point of rank r + 1 has the
                        // lower vertex index of the pair (r, r + 1)
  uint8_t *oflag;       // (K + 255) / 256: the tag of the last single-field apply that moved
                        // a critical point of these 256 ranks (or the first of the next)
  void *cpr;            // K: current value of every critical point of f, in f's order
  uint32_t *cp_idx;     // K, rank -> vertex
  uint32_t *sad_rank;   // saddle order -> rank in the CP order (K capacity)
  uint32_t *sel_f;      // 2 per critical point, in vertex order: selections in f (join,
                        // split) or ~0
  uint32_t *lab;        // 2n: g's descent / ascent labels (original mode)
  uint32_t *lab_f;      // 2n: f's resolved path termini (original mode, certificate)
  uint8_t *tmark;       // n: the target set of the iteration (1 = decrease this vertex)
  uint8_t *mchunk;      // n / 256: the tag of the last pass that marked a vertex of the
                        // 256-vertex chunk (apply passes over chunks without marks)
  uint8_t *bdirty;      // ntiles: boxes whose check reads a value the last apply changed
  uint32_t *blist;      // ntiles: the flagged boxes, listed (and their flags cleared) after
                        // each single-field apply for the next frontier check
  int64_t *trace;       // 2 * trace_cap (|S|, changed) per iteration, nullable
  State *st;
};

// ---------------------------------------------------------------------------
// device helpers

// Device pointers read out of a descriptor in memory (the batched kernels)
// have no address space, so accesses through them compile to flat
// instructions, which also hold the LDS wait counter.  glob() states that a
// pointer is global memory; for kernel arguments it changes nothing.
template <class P>
__device__ __forceinline__ __attribute__((address_space(1))) P *glob(P *p) {
  return (__attribute__((address_space(1))) P *)p;
}

// Adds vertex t to the target set: a plain byte store (every writer stores
// the same value, so concurrent marks of one target need no atomics; the
// cache keeps per-byte dirty masks, so neighbouring marks do not clash).
// Batched item lists ([nf, total, field[nf], base[nf + 1]]): the field slot
// of item `it` (largest k with base[k] <= it), found by walking forward from
// slot k: a block (or thread) visits its items in increasing order, so the
// walk is short and reads a few cached words.
__device__ __forceinline__ uint32_t next_field(const uint32_t *base, uint32_t nf, uint32_t it,
                                               uint32_t k) {
  while (k + 1 < nf && base[k + 1] <= it) ++k;
  return k;
}

// The same for a whole work-group (it is the same on every lane): the slot
// is made explicitly wave-uniform so the field's descriptor is read with
// scalar loads.
__device__ __forceinline__ uint32_t next_field_uniform(const uint32_t *base, uint32_t nf,
                                                       uint32_t it, uint32_t k) {
  return __builtin_amdgcn_readfirstlane(next_field(base, nf, it, k));
}

// Target marks carry the pass that made them: a mark is the pass's tag byte
// (1 .. MARK_TAGS, in turn; 0 = none), so apply takes the bytes equal to the
// current tag and need not clear them.  The apply of a pass with the last
// tag zeroes the whole array, so no mark outlives the cycle of tags.  The
// 256-vertex chunk of a mark gets the tag too; a chunk tag left over from an
// earlier cycle only makes apply visit a chunk without marks.
// Chunks are tagged (CH) only in frontier passes, which mark few vertices;
// the apply after such a pass skips untagged chunks.
constexpr uint32_t MARK_TAGS = 254;
constexpr uint32_t MARK_CHUNK_SHIFT = 8;
__device__ __forceinline__ bool chunk_pass(const FieldDev &fd) {
  return fd.frontier && !fd.st->dense;
}
template <bool CH = false>
__device__ __forceinline__ void mark_target(const FieldDev &fd, uint32_t t, uint32_t tag) {
  glob(fd.tmark)[t] = (uint8_t)tag;
  if (CH) glob(fd.mchunk)[t >> MARK_CHUNK_SHIFT] = (uint8_t)tag;
}

// Simulation of Simplicity: (a, ia) < (b, ib).  Bitwise, not short-circuit,
// so that the compiler emits straight-line compares instead of branches.
template <class T>
__device__ __forceinline__ bool sos_lt(T a, uint32_t ia, T b, uint32_t ib) {
  return (a < b) | ((a == b) & (ia < ib));
}

template <class T> struct Bits;
template <> struct Bits<float> {
  using U = uint32_t;
  static __device__ __forceinline__ U to(float v) { return __float_as_uint(v); }
  static __device__ __forceinline__ float from(U u) { return __uint_as_float(u); }
  static constexpr U SIGN = 0x80000000u;
  static constexpr U MAXF = 0x7F7FFFFFu;
};
template <> struct Bits<double> {
  using U = unsigned long long;
  static __device__ __forceinline__ U to(double v) { return (U)__double_as_longlong(v); }
  static __device__ __forceinline__ double from(U u) { return __longlong_as_double((long long)u); }
  static constexpr U SIGN = 0x8000000000000000ull;
  static constexpr U MAXF = 0x7FEFFFFFFFFFFFFFull;
};

// Next representable value towards +inf / -inf of a finite x.
template <class T>
__device__ __forceinline__ T next_up(T x) {
  using B = Bits<T>;
  typename B::U u = B::to(x);
  if ((u & ~B::SIGN) == 0) return B::from(1);  // +-0 -> smallest subnormal
  return B::from((u & B::SIGN) ? u - 1 : u + 1);
}
template <class T>
__device__ __forceinline__ T next_down(T x) {
  using B = Bits<T>;
  typename B::U u = B::to(x);
  if ((u & ~B::SIGN) == 0) return B::from(B::SIGN | 1);
  return B::from((u & B::SIGN) ? u + 1 : u - 1);
}

// Knuth's TwoSum: s = RN(a + b) and the exact error e = (a + b) - s.
template <class T>
__device__ __forceinline__ T two_sum(T a, T b, T &e) {
  T s = a + b;
  T bb = s - a;
  e = (a - (s - bb)) + (b - bb);
  return s;
}

// Lower bound L = RU(f - xiT): the smallest T not below f - xiT.
template <class T>
__device__ __forceinline__ T lower_bound(T f, T xiT) {
  T e;
  T s = two_sum(f, -xiT, e);
  if (isinf(s)) return -Bits<T>::from(Bits<T>::MAXF);
  return e > T(0) ? next_up(s) : s;
}
// Upper bound U = RD(f + xiT): the largest T not above f + xiT.
template <class T>
__device__ __forceinline__ T upper_bound(T f, T xiT) {
  T e;
  T s = two_sum(f, xiT, e);
  if (isinf(s)) return Bits<T>::from(Bits<T>::MAXF);
  return e < T(0) ? next_down(s) : s;
}

// In-domain neighbour slots of (x, y, z).
__device__ __forceinline__ uint32_t valid_slots(int x, int y, int z, int nx, int ny, int nz) {
  const bool xm = x > 0, xp = x < nx - 1, ym = y > 0, yp = y < ny - 1, zm = z > 0,
             zp = z < nz - 1;
  uint32_t v = 0;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    bool ok = (DXS[s] < 0 ? xm : DXS[s] > 0 ? xp : true) &&
              (DYS[s] < 0 ? ym : DYS[s] > 0 ? yp : true) &&
              (DZS[s] < 0 ? zm : DZS[s] > 0 ? zp : true);
    v |= (uint32_t)ok << s;
  }
  return v;
}

// The same set as valid_slots, from six boundary tests instead of per-slot
// logic (slot groups with a -1 / +1 component along each axis).
__device__ __forceinline__ uint32_t slots_in_domain(int x, int y, int z, int nx, int ny, int nz) {
  constexpr uint32_t XN = (1u << 1) | (1u << 5) | (1u << 9) | (1u << 13);
  constexpr uint32_t XP = (1u << 0) | (1u << 4) | (1u << 8) | (1u << 12);
  constexpr uint32_t YN = (1u << 3) | (1u << 5) | (1u << 11) | (1u << 13);
  constexpr uint32_t YP = (1u << 2) | (1u << 4) | (1u << 10) | (1u << 12);
  constexpr uint32_t ZN = (1u << 7) | (1u << 9) | (1u << 11) | (1u << 13);
  constexpr uint32_t ZP = (1u << 6) | (1u << 8) | (1u << 10) | (1u << 12);
  uint32_t out = 0;
  out |= x == 0 ? XN : 0u;
  out |= x == nx - 1 ? XP : 0u;
  out |= y == 0 ? YN : 0u;
  out |= y == ny - 1 ? YP : 0u;
  out |= z == 0 ? ZN : 0u;
  out |= z == nz - 1 ? ZP : 0u;
  return 0x3FFFu & ~out;
}

__device__ __forceinline__ int slot_delta(int s, int nx, int nxy) {
  return DXS[s] + nx * DYS[s] + nxy * DZS[s];
}

// Block index -> logical work index such that consecutive logical indices
// run on the same XCD (blocks are dispatched round-robin over the 8 XCDs,
// each with its own L2): XCD k gets one contiguous range of the work.
__device__ __forceinline__ uint32_t xcd_swizzle(uint32_t b, uint32_t nb) {
  const uint32_t q = nb >> 3, r = nb & 7u, x = b & 7u, k = b >> 3;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Index of critical point i in vertex order, from the chunk bitmask and the
// chunk prefix counts.
__device__ __forceinline__ uint32_t cp_order(const unsigned long long *cpbits, const uint32_t *cpoff,
                                             uint32_t i) {
  const uint32_t c = i >> 6;
  const unsigned long long below = (1ull << (i & 63)) - 1ull;
  return cpoff[c] + (uint32_t)__popcll(cpbits[c] & below);
}
__device__ __forceinline__ bool is_cp(const unsigned long long *cpbits, uint32_t i) {
  return (cpbits[i >> 6] >> (i & 63)) & 1ull;
}

// ---------------------------------------------------------------------------
// host side

// Component counts of the link subgraph induced by every 14-bit slot mask
// (2^14 bytes), built on the host from the offset table.
void build_component_table(uint8_t *out16k);
// One bit per slot mask: set when the mask induces exactly one connected
// component of the link (2^14 bits = 512 words).
void build_connected_bits(const uint8_t *comp16k, uint32_t *out512);

// Launch wrappers (kernels live in setup.hip / loop.hip / sort.hip).
// Reference topology of f (code, low) box by box; conn = one-component bits.
hipError_t launch_ref(const FieldDev &fd, const uint32_t *conn, hipStream_t s);
// launch_ref, then validation, copies and the critical-point bitmask.
hipError_t launch_setup(const FieldDev &fd, const uint32_t *conn, hipStream_t s);
hipError_t launch_scan_u32(const uint32_t *in, uint32_t *out, uint32_t count, uint32_t *tmp,
                           size_t tmp_words, hipStream_t s);
size_t scan_tmp_words(uint32_t count);
hipError_t launch_cp_compact(const FieldDev &fd, const uint8_t *comp, void *keys, uint32_t *vals,
                             hipStream_t s);
hipError_t launch_radix_sort(int key_bytes, void *keys, uint32_t *vals, void *keys_tmp,
                             uint32_t *vals_tmp, uint32_t count, uint32_t *hist, uint32_t *scan_tmp,
                             size_t scan_words, hipStream_t s);
size_t radix_hist_words(uint32_t count);
hipError_t launch_cp_init(const FieldDev &fd, const uint32_t *sorted_vo, hipStream_t s);
bool box_supported(int tile_y, int tile_z);
hipError_t launch_state_reset(const FieldDev &fd, int64_t max_iters, hipStream_t s);
hipError_t launch_iteration(const FieldDev &fd, const uint32_t *conn, const uint8_t *comp,
                            hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_finalize(const FieldDev &fd, hipStream_t s);
hipError_t launch_certify(const FieldDev &fd, const uint8_t *comp, uint32_t *lab_g, hipStream_t s);
// The original-mode event kernel over the original-mode fields of a batch:
// item lists as the other batched passes, 256 critical points per item.
constexpr uint32_t EVENT_ITEM = 256;
hipError_t launch_events_batch(const FieldDev *fields, const uint32_t *lists, const uint8_t *comp,
                               int grid, hipStream_t s);
hipError_t launch_original_setup(const FieldDev &fd, const uint8_t *comp, uint32_t *tmp,
                                 uint32_t *scan_tmp, size_t scan_words, hipStream_t s);
hipError_t launch_original_events(const FieldDev &fd, const uint8_t *comp, hipStream_t s);
int jump_rounds(uint32_t count);
hipError_t launch_debug_bounds(int dtype, const void *f, int64_t n, double xiT, void *L, void *U,
                               hipStream_t s);
hipError_t launch_debug_check(const FieldDev &fd, const uint32_t *conn, hipStream_t s);
hipError_t launch_targets_to_bytes(const FieldDev &fd, uint8_t *out, hipStream_t s);

// Batched launches over a device array of FieldDev (see batch.hip).
struct BatchDev {
  const FieldDev *fields;    // device array
  const int32_t *tile_base;  // nfields + 1 prefix of check tiles
  const int32_t *cp_base;    // nfields + 1 prefix of CP compare items
  int32_t nfields;
  int32_t total_tiles;
  int32_t total_cp;
};
hipError_t launch_batch_iteration(const BatchDev &b, const uint8_t *comp, int grid, hipStream_t s);

}  // namespace exz
