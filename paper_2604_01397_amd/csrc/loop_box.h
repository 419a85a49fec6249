// Device building blocks of one correction iteration on the 14-neighbour
// Freudenthal mesh, shared by the single-field kernels (loop.hip) and the
// batched ones (batch.hip): box staging, the per-vertex check (with the
// critical-point order test), the apply and counter reduction.
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

// Staging of a box plus its one-cell halo into LDS, row by row: a row is
// the 66 cells x0-1 .. x0+64 at one (y, z).  Wave w stages rows w, w + TY,
// ... (cells x0-1 .. x0+62, one per lane, from a row address the whole wave
// shares); the last two cells of every row come in one extra pass over all
// rows.  Rows outside the domain, and cells left or right of it, are
// staged as outside_value().  All loads of a thread are issued before the
// first LDS write.
// Conversion of a staged cell: the value itself ...
struct AsIs {
  template <class V> static __device__ __forceinline__ V conv(V v, uint32_t) { return v; }
};

// ... or, for float fields, a key that orders the cells the way the
// simulated order of Sec. 3.3 (footnote) orders the vertices, with no ties:
// the value widened exactly to double (-0 becomes +0 first, as IEEE equality
// treats them alike), its 29 unused low mantissa bits carrying the cell's
// position in the staged box.  Cells are numbered in the order of their
// global indices, so between equal values the later cell wins; for negative
// values a larger magnitude is a smaller value, so the position is stored
// reversed there.  Distinct floats stay ordered (they differ by at least
// 2^29 units of the double's last place), and every pair of keys differs, so
// one double max / min or one subtraction decides an SoS comparison.  The
// outside value (a quiet NaN) stays a quiet NaN.
struct TagKey {
  static __device__ __forceinline__ double conv(float v, uint32_t cell) {
    const double d = (double)(v + 0.0f);
    const unsigned long long b = (unsigned long long)__double_as_longlong(d);
    const uint32_t neg = (uint32_t)((long long)b >> 63);
    return __longlong_as_double((long long)(b | ((cell ^ neg) & 0xFFFFu)));
  }
  // staged-box position of a key
  static __device__ __forceinline__ uint32_t cell(double k) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(k);
    const uint32_t neg = (uint32_t)((long long)b >> 63);
    return ((uint32_t)b ^ neg) & 0xFFFFu;
  }
};

template <int TY, int TZ, class V, class Conv = AsIs, class O = V>
__device__ __forceinline__ void stage_rows(const FieldDev &fd, const V *__restrict__ src, O *S,
                                           BoxOrigin o) {
  using B = Box<TY, TZ>;
  constexpr int NR = B::H * B::D;             // rows of the halo box
  constexpr int RPW = (NR + TY - 1) / TY;     // rows per wave
  constexpr int NEDGE = (2 * NR + 64 * TY - 1) / (64 * TY);  // edge cells per thread
  // blocks are 64 wide, so threadIdx.y is the same on every lane of a wave
  const int lane = threadIdx.x, w = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int tid = w * 64 + lane;
  const int nx = fd.nx, ny = fd.ny, nz = fd.nz;
  const bool inner_x = o.x0 >= 1 && o.x0 + 64 <= nx - 1;
  const int xl = o.x0 - 1 + lane;                      // this lane's cell of a row
  const bool in_x = xl >= 0 && xl < nx;
  const uint32_t cxl = (uint32_t)min(max(xl, 0), nx - 1);
  V r[RPW];
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int row = w + k * TY;
    const int yy = row % B::H, zz = row / B::H;
    const int gy = o.y0 - 1 + yy, gz = o.z0 - 1 + zz;
    const bool row_in = row < NR && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
    r[k] = outside_value<V>();
    if (row_in) {  // uniform across the wave
      const V *rp = src + ((uint32_t)gz * (uint32_t)ny + (uint32_t)gy) * (uint32_t)nx;
      const V v = glob(rp)[inner_x ? (uint32_t)xl : cxl];
      r[k] = (inner_x || in_x) ? v : outside_value<V>();
    }
  }
  V e[NEDGE];
#pragma unroll
  for (int k = 0; k < NEDGE; ++k) {
    const int t = tid + k * 64 * TY;
    const int row = t >> 1, side = t & 1;
    const int yy = row % B::H, zz = row / B::H;
    const int gy = o.y0 - 1 + yy, gz = o.z0 - 1 + zz, gx = o.x0 + 63 + side;
    const bool in = t < 2 * NR && gy >= 0 && gy < ny && gz >= 0 && gz < nz && gx < nx;
    const uint32_t cy = (uint32_t)min(max(gy, 0), ny - 1), cz = (uint32_t)min(max(gz, 0), nz - 1);
    const uint32_t cx = (uint32_t)min(gx, nx - 1);
    const V v = glob(src)[(cz * (uint32_t)ny + cy) * (uint32_t)nx + cx];
    e[k] = in ? v : outside_value<V>();
  }
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int row = w + k * TY;
    const uint32_t c = (uint32_t)(row * B::W + lane);
    if (row < NR) S[c] = Conv::conv(r[k], c);
  }
#pragma unroll
  for (int k = 0; k < NEDGE; ++k) {
    const int t = tid + k * 64 * TY;
    const uint32_t c = (uint32_t)((t >> 1) * B::W + 64 + (t & 1));
    if (t < 2 * NR) S[c] = Conv::conv(e[k], c);
  }
}

// Order of a vertex within its closed neighbourhood, from staged values
// (cells outside the domain are NaN): the slots of the SoS maximum and
// minimum (SELF for the vertex itself) and the mask of lower neighbours.
// P points at the LDS centre value of the vertex; pm / pp are the offsets
// of the planes below / above relative to the centre plane.
template <class T>
__device__ __forceinline__ void closed_order(const T *P, int pm, int pp, int &asc, int &desc,
                                             uint32_t &lower) {
  // Vertex indices of the neighbours, ascending: the slots with a negative
  // offset (odd), the vertex itself, the slots with a positive offset (even).
  // Offsets are dx + nx*dy + nx*ny*dz, ordered lexicographically by
  // (dz, dy, dx) on any grid where the slot is in the domain.
  constexpr int ORDER[NSLOT + 1] = {13, 11, 9, 7, 5, 3, 1, SELF, 0, 2, 4, 6, 8, 10, 12};
  T v[NSLOT + 1];  // closed neighbourhood in index order
#pragma unroll
  for (int q = 0; q <= NSLOT; ++q) {
    const int s = ORDER[q];
    const int po = s == SELF ? 0 : DZS[s] < 0 ? pm : DZS[s] > 0 ? pp : 0;
    v[q] = s == SELF ? P[0] : P[po + DYS[s] * HALO_W + DXS[s]];
  }
  const T gi = v[7];
  // Extreme values first (NaN, outside the domain, is ignored by fmax /
  // fmin), then the slot: the SoS maximum is the highest-index vertex
  // holding the largest value, the SoS minimum the lowest-index vertex
  // holding the smallest.
  T hi = gi, lo = gi;
#pragma unroll
  for (int q = 0; q <= NSLOT; ++q) {
    if (q == 7) continue;
    hi = fmax(hi, v[q]);
    lo = fmin(lo, v[q]);
  }
  asc = SELF;
  desc = SELF;
#pragma unroll
  for (int q = 0; q <= NSLOT; ++q) {
    asc = v[q] == hi ? ORDER[q] : asc;
    desc = v[NSLOT - q] == lo ? ORDER[NSLOT - q] : desc;
  }
  // A neighbour with a lower index is below i when its value is <= g_i,
  // one with a higher index when it is < g_i; NaN never compares true.
  lower = 0;
#pragma unroll
  for (int q = 0; q <= NSLOT; ++q) {
    if (q == 7) continue;
    lower |= (uint32_t)(q < 7 ? v[q] <= gi : v[q] < gi) << ORDER[q];
  }
}

// Requests of one vertex as a slot mask (bit SELF = the vertex itself).
// P points at the LDS centre value of the vertex; pm / pp are the offsets
// of the planes below / above relative to the centre plane; dlt holds the
// linear offset of every slot.
template <class T>
__device__ __forceinline__ uint32_t check_vertex(const FieldDev &fd, const uint32_t *__restrict__ conn,
                                                 const int32_t *dlt, const T *P, int pm, int pp,
                                                 int x, int y, int z,
                                                 uint32_t i, uint32_t codeb, uint32_t lowf,
                                                 uint32_t &asc_v, uint32_t &desc_v, bool interior) {
  const uint32_t vm = interior ? 0x3FFFu : slots_in_domain(x, y, z, fd.nx, fd.ny, fd.nz);
  int asc, desc;
  uint32_t lower;
  closed_order<T>(P, pm, pp, asc, desc, lower);
  if (fd.mode == 1) {  // vertex indices are needed for path tracing only
    asc_v = (uint32_t)((int)i + dlt[asc]);
    desc_v = (uint32_t)((int)i + dlt[desc]);
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

// Vertices of the box inside the domain.
__device__ __forceinline__ uint32_t box_vertices(const FieldDev &fd, BoxOrigin o, int TY, int TZ) {
  return (uint32_t)(min(64, fd.nx - o.x0) * min(TY, fd.ny - o.y0) * min(TZ, fd.nz - o.z0));
}

// Adds the targets named by vertex i's request mask r (bit s: the neighbour
// in slot s, at offset dlt[s]; bit SELF: i itself).
template <bool CH>
__device__ __forceinline__ void post_targets(const FieldDev &fd, const int32_t *dlt, uint32_t i,
                                             uint32_t r, uint32_t tag) {
  if ((r >> SELF) & 1u) mark_target<CH>(fd, i, tag);
  r &= LOW_MASK;
  while (r) {
    const int s = __ffs(r) - 1;
    r &= r - 1;
    mark_target<CH>(fd, (uint32_t)((int)i + dlt[s]), tag);
  }
}

// LDS of one check work-group: the staged box (float fields as tie-free
// keys, double fields as values), the reference codes of its own vertices
// (code byte | lower mask << 8), the link connectivity bits, the field's
// slot offsets and, for the keyed boxes, the slot of every cell offset a
// neighbour can have (offset + SLOT_BIAS; other entries unused).  With the
// tables in LDS the vertex loop issues no global load.
constexpr int CONN_WORDS = 512;  // one bit per 14-bit slot mask
template <int TY, int TZ>
struct CellSlots {
  static constexpr int B = Box<TY, TZ>::PLANE + Box<TY, TZ>::W + 1;  // SLOT_BIAS
  static constexpr int N = 2 * B + 1;
};
template <class T, int TY, int TZ>
struct CheckLds {
  double S[Box<TY, TZ>::NE];
  uint32_t ref[sizeof(T) == 4 ? 1 : TZ][64 * TY];  // keyed boxes keep the codes in registers
  uint32_t conn[CONN_WORDS];
  int32_t dlt[16];
  uint8_t slot_of[CellSlots<TY, TZ>::N];
};

// Maximum / minimum of two keys with v_max_f64 / v_min_f64 as they are: a
// quiet NaN operand yields the other one.  (fmax would first quiet each
// operand with a separate instruction, since a value loaded from memory
// could be a signalling NaN; staged keys never are.)
__device__ __forceinline__ double key_max(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double key_min(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// check_vertex on tie-free keys (float fields, see TagKey): one double
// max / min each over the closed neighbourhood gives the steepest ascent /
// descent, whose slots come from their cells through L.slot_of; the lower
// mask is the sign of key(neighbour) - key(i), one subtraction and one
// funnel shift per slot.  Same requests as check_vertex.
// closed_order on tie-free keys: P points at the key of the vertex (cell cc
// of the staged box), vm is its mask of in-domain slots.
template <int TY, int TZ>
__device__ __forceinline__ void key_order(const double *P, uint32_t cc, const uint8_t *slot_of,
                                          uint32_t vm, int &asc, int &desc, uint32_t &lower) {
  using B = Box<TY, TZ>;
  double v[NSLOT];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) v[s] = P[DZS[s] * B::PLANE + DYS[s] * B::W + DXS[s]];
  const double c = P[0];
  double hi = c, lo = c;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    hi = key_max(hi, v[s]);  // a quiet NaN (outside the domain) is ignored
    lo = key_min(lo, v[s]);
  }
  lower = 0;
#pragma unroll
  for (int s = NSLOT - 1; s >= 0; --s) {
    const double d = v[s] - c;  // never zero: keys are distinct
    const uint32_t dh = (uint32_t)((unsigned long long)__double_as_longlong(d) >> 32);
    lower = __builtin_amdgcn_alignbit(lower, dh, 31);  // lower << 1 | sign(d)
  }
  lower &= vm;
  asc = slot_of[TagKey::cell(hi) - cc + CellSlots<TY, TZ>::B];
  desc = slot_of[TagKey::cell(lo) - cc + CellSlots<TY, TZ>::B];
}

// Fills the cell-offset -> slot table of a keyed box (threads 0..14).
template <int TY, int TZ>
__device__ __forceinline__ void fill_slot_of(uint8_t *slot_of, int tid) {
  using B = Box<TY, TZ>;
  if (tid < NSLOT + 1) {
    const int s = tid;
    const int off = s == SELF ? 0 : DZS[s] * B::PLANE + DYS[s] * B::W + DXS[s];
    slot_of[off + CellSlots<TY, TZ>::B] = (uint8_t)s;
  }
}

// Copies the connectivity bits into LDS; the barrier of the first box
// orders it before any use.
template <int TY>
__device__ __forceinline__ void copy_conn(uint32_t *dst, const uint32_t *__restrict__ conn) {
  for (int k = threadIdx.y * 64 + threadIdx.x; k < CONN_WORDS; k += 64 * TY) dst[k] = conn[k];
}
template <class T, int TY, int TZ>
__device__ __forceinline__ void load_conn(CheckLds<T, TY, TZ> &L, const uint32_t *__restrict__ conn) {
  copy_conn<TY>(L.conn, conn);
}

__device__ __forceinline__ bool one_component(const uint32_t *conn, uint32_t m) {
  return (conn[m >> 5] >> (m & 31u)) & 1u;
}

// LDS of one reference-topology work-group: the staged box of f (keys for
// float fields, values for double fields), the link connectivity bits and
// the cell-offset -> slot table.
template <class T, int TY, int TZ>
struct RefLds {
  double S[Box<TY, TZ>::NE];
  uint32_t conn[CONN_WORDS];
  uint8_t slot_of[CellSlots<TY, TZ>::N];
};

// Reference topology of f on one box (Sec. 3.1-3.2): per vertex the code
// byte (steepest ascent slot | steepest descent slot << 4, SELF at a maximum
// / minimum) and the lower mask, with LOW_SADDLE when the lower or the upper
// link is not one connected piece.  The caller synchronises the block after
// it.
template <class T, int TY, int TZ>
__device__ __forceinline__ void ref_box(const FieldDev &fd, BoxOrigin o, RefLds<T, TY, TZ> &L) {
  using B = Box<TY, TZ>;
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int x = o.x0 + lx, y = o.y0 + ly;
  const bool col = x < fd.nx && y < fd.ny;
  const uint32_t plane = (uint32_t)fd.nx * (uint32_t)fd.ny;
  const uint32_t i0 = (uint32_t)x + (uint32_t)fd.nx * ((uint32_t)y + (uint32_t)fd.ny * (uint32_t)o.z0);
  constexpr bool keyed = sizeof(T) == 4;
  if (keyed) {
    fill_slot_of<TY, TZ>(L.slot_of, ly * 64 + lx);
    stage_rows<TY, TZ, float, TagKey, double>(fd, (const float *)fd.f, L.S, o);
  } else {
    stage_rows<TY, TZ, double, AsIs, double>(fd, (const double *)fd.f, L.S, o);
  }
  const bool interior = o.x0 >= 1 && o.x0 + 64 <= fd.nx - 1 && o.y0 >= 1 &&
                        o.y0 + TY <= fd.ny - 1 && o.z0 >= 1 && o.z0 + TZ <= fd.nz - 1;
  __syncthreads();
#pragma unroll 1
  for (int k = 0; k < TZ; ++k) {
    const int z = o.z0 + k;
    if (col && z < fd.nz) {
      const uint32_t i = i0 + k * plane;
      const uint32_t cc = (uint32_t)((k + 1) * B::PLANE + (ly + 1) * B::W + lx + 1);
      const double *c = L.S + cc;
      const uint32_t vm = interior ? 0x3FFFu : slots_in_domain(x, y, z, fd.nx, fd.ny, fd.nz);
      int asc, desc;
      uint32_t lower;
      if (keyed)
        key_order<TY, TZ>(c, cc, L.slot_of, vm, asc, desc, lower);
      else
        closed_order<double>(c, -B::PLANE, B::PLANE, asc, desc, lower);
      uint32_t low = lower;
      if (lower != 0 && lower != vm &&
          !(one_component(L.conn, lower) && one_component(L.conn, vm & ~lower)))
        low |= LOW_SADDLE;
      glob(fd.code)[i] = (uint8_t)(asc | (desc << 4));
      glob(fd.low)[i] = (uint16_t)low;
    }
  }
}

// Requests of a vertex (as check_vertex) once its steepest slots in g and
// its lower mask in g are known.
__device__ __forceinline__ uint32_t requests_of(const uint32_t *conn, uint32_t vm, int asc, int desc,
                                                uint32_t lower, uint32_t codeb, uint32_t lowf) {
  const int asc_f = (int)(codeb & 15u), desc_f = (int)(codeb >> 4);
  const uint32_t lower_f = lowf & LOW_MASK;
  bool link_rule = (lowf & LOW_SADDLE) != 0;
  if (!link_rule && lower != lower_f && asc_f != SELF && desc_f != SELF && lower != 0 &&
      lower != vm) {
    const uint32_t up = vm & ~lower;
    const bool regular_g = ((conn[lower >> 5] >> (lower & 31u)) & 1u) &&
                           ((conn[up >> 5] >> (up & 31u)) & 1u);
    link_rule = !regular_g;
  }
  uint32_t req = 0;
  if (asc != asc_f) req |= 1u << asc;
  if (desc != desc_f) req |= 1u << desc_f;
  if (link_rule) {
    const uint32_t diff = lower ^ lower_f;
    req |= diff & lower_f;
    if (diff & ~lower_f) req |= 1u << SELF;
  }
  return req;
}

// Keys of one plane of a thread's column walk: the vertex's cell and its six
// in-plane neighbours (slots 0..5), read from the staged box.
struct PlaneKeys {
  double c, xp, xm, yp, ym, xyp, xym;
};

// The keyed check of the TZ vertices of one (x, y) column of a box, walked
// upwards in z.  A vertex's closed neighbourhood is the 2 x 2 square of cells
// at and above-right of it in its own plane and the plane above, plus the
// square at and below-left of it in its own plane and the plane below (the
// two cubes of the Freudenthal star).  Walking up, each plane's cells are
// read once (7 reads per vertex instead of 15) and the maxima / minima of
// the squares are kept, so the steepest neighbours cost 9 max and 9 min
// operations per vertex.  Requests and, in original mode, g's pointers are
// those of check_vertex.
template <int TY, int TZ, bool CH>
__device__ __forceinline__ void check_column_keys(const FieldDev &fd, CheckLds<float, TY, TZ> &L,
                                                  BoxOrigin o, const uint32_t *refs, bool interior,
                                                  uint32_t tag) {
  using B = Box<TY, TZ>;
  constexpr int W = B::W;
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int x = o.x0 + lx, y = o.y0 + ly;
  const bool col = x < fd.nx && y < fd.ny;
  const uint32_t plane = (uint32_t)fd.nx * (uint32_t)fd.ny;
  const uint32_t i0 = (uint32_t)x + (uint32_t)fd.nx * ((uint32_t)y + (uint32_t)fd.ny * (uint32_t)o.z0);
  const uint32_t cell0 = (uint32_t)((ly + 1) * W + lx + 1);  // this column's cell in plane 0
  const double *S = L.S;
  // plane 0 (below the box): the lower-left square; plane 1: the upper-right square
  double m_c = S[cell0], m_xm = S[cell0 - 1], m_ym = S[cell0 - W], m_xym = S[cell0 - W - 1];
  double m_max = key_max(key_max(m_c, m_xm), key_max(m_ym, m_xym));
  double m_min = key_min(key_min(m_c, m_xm), key_min(m_ym, m_xym));
  PlaneKeys c;
  {
    const uint32_t b = cell0 + B::PLANE;
    c.c = S[b];
    c.xp = S[b + 1];
    c.yp = S[b + W];
    c.xyp = S[b + W + 1];
  }
  double cp_max = key_max(key_max(c.c, c.xp), key_max(c.yp, c.xyp));
  double cp_min = key_min(key_min(c.c, c.xp), key_min(c.yp, c.xyp));
#pragma unroll
  for (int k = 0; k < TZ; ++k) {
    // this vertex's plane (k + 1): the lower-left cells; the plane above: the
    // upper-right square
    const uint32_t b = cell0 + (uint32_t)(k + 1) * B::PLANE, bu = b + B::PLANE;
    c.xm = S[b - 1];
    c.ym = S[b - W];
    c.xym = S[b - W - 1];
    const double u_c = S[bu], u_xp = S[bu + 1], u_yp = S[bu + W], u_xyp = S[bu + W + 1];
    const double cm_max = key_max(key_max(c.c, c.xm), key_max(c.ym, c.xym));
    const double cm_min = key_min(key_min(c.c, c.xm), key_min(c.ym, c.xym));
    const double up_max = key_max(key_max(u_c, u_xp), key_max(u_yp, u_xyp));
    const double up_min = key_min(key_min(u_c, u_xp), key_min(u_yp, u_xyp));
    const double hi = key_max(key_max(m_max, cm_max), key_max(cp_max, up_max));
    const double lo = key_min(key_min(m_min, cm_min), key_min(cp_min, up_min));
    const int z = o.z0 + k;
    const uint32_t vm = interior ? 0x3FFFu : slots_in_domain(x, y, z, fd.nx, fd.ny, fd.nz);
    // lower mask, slot 13 first so that slot s ends at bit s
    const double nb[NSLOT] = {c.xp, c.xm, c.yp, c.ym, c.xyp, c.xym, u_c,
                              m_c, u_xp, m_xm, u_yp, m_ym, u_xyp, m_xym};
    uint32_t lower = 0;
#pragma unroll
    for (int s = NSLOT - 1; s >= 0; --s) {
      const double d = nb[s] - c.c;  // never zero: keys are distinct
      const uint32_t dh = (uint32_t)((unsigned long long)__double_as_longlong(d) >> 32);
      lower = __builtin_amdgcn_alignbit(lower, dh, 31);
    }
    lower &= vm;
    const uint32_t cc = b;
    const int asc = L.slot_of[TagKey::cell(hi) - cc + CellSlots<TY, TZ>::B];
    const int desc = L.slot_of[TagKey::cell(lo) - cc + CellSlots<TY, TZ>::B];
    if (col && z < fd.nz) {
      const uint32_t i = i0 + (uint32_t)k * plane;
      const uint32_t r = requests_of(L.conn, vm, asc, desc, lower, refs[k] & 255u, refs[k] >> 8);
      if (r) post_targets<CH>(fd, L.dlt, i, r, tag);
      if (fd.mode == 1) {  // original event constraints trace g's integral paths
        glob(fd.lab)[i] = (uint32_t)((int)i + L.dlt[desc]);
        glob(fd.lab)[fd.n + i] = (uint32_t)fd.n + (uint32_t)((int)i + L.dlt[asc]);
      }
    }
    // move up one plane
    m_c = c.c;
    m_xm = c.xm;
    m_ym = c.ym;
    m_xym = c.xym;
    m_max = cm_max;
    m_min = cm_min;
    c.c = u_c;
    c.xp = u_xp;
    c.yp = u_yp;
    c.xyp = u_xyp;
    cp_max = up_max;
    cp_min = up_min;
  }
}

// The plain (double field) check of one box's columns, vertex by vertex.
template <int TY, int TZ, bool CH>
__device__ __forceinline__ void check_column_plain(const FieldDev &fd, CheckLds<double, TY, TZ> &L,
                                                   BoxOrigin o, bool interior, uint32_t tag) {
  using B = Box<TY, TZ>;
  const int lx = threadIdx.x, ly = threadIdx.y, tid = ly * 64 + lx;
  const int x = o.x0 + lx, y = o.y0 + ly;
  const bool col = x < fd.nx && y < fd.ny;
  const uint32_t plane = (uint32_t)fd.nx * (uint32_t)fd.ny;
  const uint32_t i0 = (uint32_t)x + (uint32_t)fd.nx * ((uint32_t)y + (uint32_t)fd.ny * (uint32_t)o.z0);
#pragma unroll 1
  for (int k = 0; k < TZ; ++k) {
    const int z = o.z0 + k;
    if (col && z < fd.nz) {
      const uint32_t i = i0 + k * plane;
      const uint32_t cc = (uint32_t)((k + 1) * B::PLANE + (ly + 1) * B::W + lx + 1);
      const double *c = L.S + cc;
      const uint32_t rf = L.ref[k][tid];
      uint32_t av = 0, dv = 0;
      const uint32_t r = check_vertex<double>(fd, L.conn, L.dlt, c, -B::PLANE, B::PLANE, x, y, z, i,
                                              rf & 255u, rf >> 8, av, dv, interior);
      if (r) post_targets<CH>(fd, L.dlt, i, r, tag);
      if (fd.mode == 1) {  // original event constraints trace g's integral paths
        glob(fd.lab)[i] = dv;
        glob(fd.lab)[fd.n + i] = (uint32_t)fd.n + av;
      }
    }
  }
}

// CheckConstraints on one box (Sec. 4.2): stage g (and the box's reference
// codes), add the targets every vertex names to the target set (and, in
// original mode, write g's descent / ascent pointers).  The order of the
// critical points of f (Sec. 4.3) is tested by its own pass (order_quad).
// The caller synchronises the block after it.
template <class T, int TY, int TZ, bool CH = false>
__device__ __forceinline__ void check_box(const FieldDev &fd, BoxOrigin o, CheckLds<T, TY, TZ> &L) {
  constexpr bool keyed = sizeof(T) == 4;  // float fields: tie-free keys
  const uint32_t tag = __builtin_amdgcn_readfirstlane(fd.st->tag);
  const int lx = threadIdx.x, ly = threadIdx.y, tid = ly * 64 + lx;
  const int x = o.x0 + lx, y = o.y0 + ly;
  const bool col = x < fd.nx && y < fd.ny;
  const uint32_t plane = (uint32_t)fd.nx * (uint32_t)fd.ny;
  const uint32_t i0 = (uint32_t)x + (uint32_t)fd.nx * ((uint32_t)y + (uint32_t)fd.ny * (uint32_t)o.z0);
  uint32_t refs[TZ];
#pragma unroll
  for (int k = 0; k < TZ; ++k) {  // issued with the staging loads, unconditionally
    const bool in = col && o.z0 + k < fd.nz;
    const uint32_t idx = in ? i0 + k * plane : 0u;
    const uint32_t cb = glob(fd.code)[idx], lb = glob(fd.low)[idx];
    refs[k] = cb | (lb << 8);
  }
  if (tid == 0) {  // constant indices: scalar loads, ordered by the barrier below
#pragma unroll
    for (int q = 0; q < 16; ++q) L.dlt[q] = fd.dlt[q];
  }
  if (keyed) fill_slot_of<TY, TZ>(L.slot_of, tid);
  const bool interior = o.x0 >= 1 && o.x0 + 64 <= fd.nx - 1 && o.y0 >= 1 &&
                        o.y0 + TY <= fd.ny - 1 && o.z0 >= 1 && o.z0 + TZ <= fd.nz - 1;
  if constexpr (keyed) {
    stage_rows<TY, TZ, float, TagKey, double>(fd, (const float *)fd.g, L.S, o);
    __syncthreads();
    check_column_keys<TY, TZ, CH>(fd, L, o, refs, interior, tag);
  } else {
    stage_rows<TY, TZ, double, AsIs, double>(fd, (const double *)fd.g, L.S, o);
#pragma unroll
    for (int k = 0; k < TZ; ++k) L.ref[k][tid] = refs[k];
    __syncthreads();
    check_column_plain<TY, TZ, CH>(fd, L, o, interior, tag);
  }
}

// Four values from an aligned block (vector loads and stores).
template <class T> struct Vec4;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <> struct Vec4<float> {
  static __device__ __forceinline__ void load(const float *p, float *o) {
    const f32x4 v = *glob(reinterpret_cast<const f32x4 *>(p));
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
  static __device__ __forceinline__ void store(float *p, const float *o) {
    f32x4 v;
    v.x = o[0]; v.y = o[1]; v.z = o[2]; v.w = o[3];
    *glob(reinterpret_cast<f32x4 *>(p)) = v;
  }
};
template <> struct Vec4<double> {
  static __device__ __forceinline__ void load(const double *p, double *o) {
    const f64x2 a = glob(reinterpret_cast<const f64x2 *>(p))[0];
    const f64x2 b = glob(reinterpret_cast<const f64x2 *>(p))[1];
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
  }
  static __device__ __forceinline__ void store(double *p, const double *o) {
    f64x2 a, b;
    a.x = o[0]; a.y = o[1]; b.x = o[2]; b.y = o[3];
    glob(reinterpret_cast<f64x2 *>(p))[0] = a;
    glob(reinterpret_cast<f64x2 *>(p))[1] = b;
  }
};

// Reformulated event constraints (Sec. 4.3) on the ranks r .. r+3 of the
// critical points in f's order: for each pair (r', r' + 1) with r' + 1 < K,
// when g puts the one of rank r' + 1 below the one of rank r', the latter
// (the lower one in f) goes down.  The values come from cpr, which apply
// keeps current in f's order, so a pass streams it (one vector load per
// lane; the value after the lane's four comes from the next lane when that
// lane holds the next four, else from one more load).  Ties in g are broken
// by the vertex index: cp_below holds, per rank, whether the next critical
// point's index is the lower one.  Every lane of the wave calls this (the
// shuffle); lanes with r >= K test nothing.  K may cut the ranks short of
// the field's count (a batched item stops there).
template <class T, bool CH = false>
__device__ __forceinline__ void order_quad(const FieldDev &fd, uint32_t r, uint32_t K,
                                           bool next_in_lane, uint32_t tag) {
  const T *V = (const T *)fd.cpr;
  T a[4];
  if (r + 4 <= K) {
    Vec4<T>::load(V + r, a);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = r + c < K ? glob(V)[r + c] : (T)0;
  }
  const uint32_t bw = r < K ? glob(fd.cp_below)[r >> 5] >> (r & 31u) : 0u;
  T nx = __shfl_down(a[0], 1);
  if (!next_in_lane && r + 4 < K) nx = glob(V)[r + 4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const T lo = a[c], hi = c < 3 ? a[c + 1] : nx;
    const bool below = (bw >> c) & 1u;
    if (r + c + 1 < K && (hi < lo || (hi == lo && below)))
      mark_target<CH>(fd, glob(fd.cp_idx)[r + c], tag);
  }
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

// Marks every box whose check reads a vertex of the row segment
// x0 .. x1 at (y, z): the boxes whose cells plus one-cell halo contain it,
// so the next frontier check visits them.
__device__ __forceinline__ void mark_box_range(const FieldDev &fd, uint32_t x0, uint32_t x1,
                                               uint32_t y, uint32_t z) {
  const uint32_t bx0 = x0 ? (x0 - 1) >> 6 : 0, bx1 = min((x1 + 1) >> 6, (uint32_t)fd.tiles_x - 1);
  const uint32_t by0 = y ? (y - 1) >> fd.ty_shift : 0;
  const uint32_t by1 = min((y + 1) >> fd.ty_shift, (uint32_t)fd.tiles_y - 1);
  const uint32_t bz0 = z ? (z - 1) >> fd.tz_shift : 0;
  const uint32_t bz1 = min((z + 1) >> fd.tz_shift, (uint32_t)fd.tiles_z - 1);
  for (uint32_t bz = bz0; bz <= bz1; ++bz)
    for (uint32_t by = by0; by <= by1; ++by)
      for (uint32_t bx = bx0; bx <= bx1; ++bx)
        glob(fd.bdirty)[bx + (uint32_t)fd.tiles_x * (by + (uint32_t)fd.tiles_y * bz)] = 1;
}

// Work-group size of the apply passes.  A thread takes four consecutive
// vertices (their marks are one 32-bit word), so a wave covers 256
// consecutive vertices and a work-group APPLY_CHUNK.
constexpr int APPLY_BLOCK = 256;
constexpr uint32_t APPLY_CHUNK = 4 * APPLY_BLOCK;

// The bytes of w equal to tag, as 1 (others 0).
__device__ __forceinline__ uint32_t marks_of(uint32_t w, uint32_t tag) {
  const uint32_t x = w ^ (tag * 0x01010101u);  // a marked byte is 0 here
  const uint32_t t = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;  // bit 7: byte nonzero
  return (~t & 0x80808080u) >> 7;
}

// Raw mark bytes of vertices 4q .. 4q+3 (the mark array is padded).
__device__ __forceinline__ uint32_t quad_marks(const FieldDev &fd, uint32_t q) {
  return *glob(reinterpret_cast<const uint32_t *>(fd.tmark + 4u * q));
}

// What apply fetches one quad ahead: the quad's marks and, with the
// reformulated constraints, the critical-point bitmask word and prefix count
// of its 64-vertex chunk (raw: decoded only once they are needed, so the
// loads stay in flight while the current quad is edited).
// When the last pass changed many values (busy), also the quad's edit counts
// and final-edit counts (whole aligned quads only; ce = 0 otherwise), so
// that the loads of f a final edit needs go out with the value loads.
struct QuadHead {
  uint32_t m;
  unsigned long long bits;
  uint32_t off;
  uint32_t c4, e4;
  bool ce;
};

__device__ __forceinline__ QuadHead quad_head(const FieldDev &fd, uint32_t q, uint32_t nq,
                                              bool busy) {
  QuadHead h = {0u, 0ull, 0u, 0u, 0u, false};
  if (q < nq) {
    h.m = quad_marks(fd, q);
    if (fd.mode != 1) {  // a quad lies in one 64-vertex chunk of the bitmask
      h.bits = glob(fd.cpbits)[q >> 4];
      h.off = glob(fd.cpoff)[q >> 4];
    }
    if (busy && fd.vec && 4u * q + 3 < (uint32_t)fd.n) {
      h.c4 = *glob(reinterpret_cast<const uint32_t *>(fd.cnt + 4u * q));
      h.e4 = *glob(reinterpret_cast<const uint32_t *>(fd.fe + 4u * q));
      h.ce = true;
    }
  }
  return h;
}

// Inputs of one quad v .. v+3 of apply: value, f and edit count; with the
// reformulated constraints also which of them are critical points of f
// (bits 0..3) and, for the marked ones, their ranks in f's order.
template <class T>
struct QuadIn {
  T g[4];
  uint32_t c[4], e[4];  // edit counts, and the counts at which each reaches its floor
  T fl[4];              // f of the marked vertices whose next edit stores L
  uint32_t cpm;
  uint32_t rank[4];
};

// Loads the inputs of the quad at v whose mark bytes are m (m != 0): vector
// loads when the whole quad is in the field and aligned, else one load per
// vertex (unmarked ones read vertex v, which is valid).
template <class T>
__device__ __forceinline__ void load_quad(const FieldDev &fd, uint32_t v, const QuadHead &h,
                                          QuadIn<T> &d) {
  const uint32_t m = h.m;
  d.cpm = 0;
  if (fd.mode != 1) {  // ranks first: issued together with the value loads
    const uint32_t sh = v & 63u;
    d.cpm = (uint32_t)(h.bits >> sh) & 15u;
    const uint32_t vo0 = h.off + (uint32_t)__popcll(h.bits & ((1ull << sh) - 1ull));
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (((d.cpm >> c) & 1u) && ((m >> (8 * c)) & 255u))
        d.rank[c] = glob(fd.cp_rank)[vo0 + (uint32_t)__popc(d.cpm & ((1u << c) - 1u))];
  }
  const T *G = (const T *)fd.g;
  if (h.ce) {  // counts fetched ahead: f goes out with the values
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      d.c[c] = (h.c4 >> (8 * c)) & 255u;
      d.e[c] = (h.e4 >> (8 * c)) & 255u;
    }
    Vec4<T>::load(G + v, d.g);
  } else if (fd.vec && v + 3 < (uint32_t)fd.n) {
    Vec4<T>::load(G + v, d.g);
    const uint32_t c4 = *glob(reinterpret_cast<const uint32_t *>(fd.cnt + v));
    const uint32_t e4 = *glob(reinterpret_cast<const uint32_t *>(fd.fe + v));
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      d.c[c] = (c4 >> (8 * c)) & 255u;
      d.e[c] = (e4 >> (8 * c)) & 255u;
    }
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t t = ((m >> (8 * c)) & 255u) ? v + c : v;
      d.g[c] = glob(G)[t];
      d.c[c] = glob(fd.cnt)[t];
      d.e[c] = glob(fd.fe)[t];
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (((m >> (8 * c)) & 255u) && d.c[c] + 1 == d.e[c]) d.fl[c] = glob((const T *)fd.f)[v + c];
}

// ApplyBoundedEdits on the vertices v .. v+3 whose mark bytes in m are set,
// from the inputs d; clears the marks and adds this thread's counts to ec.
// A vertex's value is a plain step of delta below the last one until its
// count reaches fe, where it becomes L (f is read for those edits only), and
// blocked after that (its value is L).
// A whole aligned quad is written back with one vector store of its values
// and one 32-bit store of its counts (unmarked vertices keep theirs).
// Returns the vertices whose value or count moved, as bits 0..3.
template <class T>
__device__ __forceinline__ uint32_t edit_quad(const FieldDev &fd, uint32_t v, uint32_t m,
                                              const QuadIn<T> &d, EditCount &ec, uint32_t otag) {
  T *G = (T *)fd.g;
  const T xiT = (T)fd.xiT, delta = (T)fd.delta;
  uint32_t moved = 0, cw = 0;
  T gn[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    gn[c] = d.g[c];
    cw |= d.c[c] << (8 * c);
    if (!((m >> (8 * c)) & 255u)) continue;
    ++ec.v[0];
    if (d.c[c] >= d.e[c]) continue;  // at the floor: blocked
    const uint32_t cn = d.c[c] + 1;
    cw = (cw & ~(255u << (8 * c))) | (cn << (8 * c));
    T nv;
    if (cn == d.e[c]) {
      nv = lower_bound(d.fl[c], xiT);  // a clamped step or the (N+1)-th edit
      ++ec.v[3];
      ec.v[2] += cn > (uint32_t)fd.N;
    } else {
      nv = d.g[c] - delta;
    }
    gn[c] = nv;
    // a critical point of f: the copy of its value, in f's order, that the
    // order pass streams, and (otag != 0) the tags of the rank groups whose
    // pairs it belongs to, for the next frontier check
    if ((d.cpm >> c) & 1u) {
      const uint32_t r = d.rank[c];
      glob((T *)fd.cpr)[r] = nv;
      if (otag) {
        glob(fd.oflag)[r >> 8] = (uint8_t)otag;
        if ((r & 255u) == 0 && r) glob(fd.oflag)[(r - 1) >> 8] = (uint8_t)otag;
      }
    }
    moved |= 1u << c;
    ++ec.v[1];
    ec.v[4] += cn == 1;
  }
  if (moved) {
    if (fd.vec && v + 3 < (uint32_t)fd.n) {
      Vec4<T>::store(G + v, gn);
      *glob(reinterpret_cast<uint32_t *>(fd.cnt + v)) = cw;
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (!((moved >> c) & 1u)) continue;
        glob(G)[v + c] = gn[c];
        glob(fd.cnt)[v + c] = (uint8_t)(cw >> (8 * c));
      }
    }
  }
  return moved;
}

// Box marks for the vertices that moved in one wave (lane l moved the
// vertices v + bits of `moved`; the wave's vertices are consecutive): one
// range when they lie on one grid row (marked by one lane), else every
// lane marks its own.  All lanes of the wave take part.
__device__ __forceinline__ void mark_moved_boxes(const FieldDev &fd, uint32_t v, uint32_t moved) {
  const unsigned long long b = __ballot(moved != 0);
  if (!b) return;
  const uint32_t first = v + (moved ? (uint32_t)(__ffs(moved) - 1) : 0u);
  const uint32_t last = v + (moved ? 31u - (uint32_t)__clz(moved) : 0u);
  const uint32_t lo = __shfl(first, __ffsll(b) - 1), hi = __shfl(last, 63 - __clzll(b));
  const uint32_t nx = (uint32_t)fd.nx, ny = (uint32_t)fd.ny;
  const uint32_t x = lo % nx, r = lo / nx;
  if (x + (hi - lo) < nx) {
    if (__lane_id() == (uint32_t)(__ffsll(b) - 1)) mark_box_range(fd, x, x + (hi - lo), r % ny, r / ny);
    return;
  }
  while (moved) {
    const uint32_t t = v + (uint32_t)(__ffs(moved) - 1);
    moved &= moved - 1;
    const uint32_t tx = t % nx, tr = t / nx;
    mark_box_range(fd, tx, tx, tr % ny, tr / ny);
  }
}

// ApplyBoundedEdits over quads q = q0, q0 + stride, ... (< nq): the marks
// (and critical-point words) of the next quad are fetched before the current
// one is edited.  One quad
// per thread at a time keeps the register count, and so the number of waves
// in flight, high.  Box flags for the next frontier pass are set unless the
// last pass changed so many values that the next check covers every box
// anyway (State::noflag).
//
// With SKIP (a wave's lanes hold 64 consecutive quads from a multiple of 64,
// and stride is a multiple of 64), after a frontier check that changed few
// values, only the 256-vertex chunks tagged by this pass are visited: each
// lane reads the chunk tag of one of the wave's steps, and the wave walks the
// steps whose tag matches.
template <class T>
__device__ __forceinline__ void apply_quad(const FieldDev &fd, uint32_t q, QuadHead h, uint32_t tag,
                                           bool wipe, bool flag, EditCount &ec) {
  uint32_t moved = 0;
  h.m = marks_of(h.m, tag);
  if (wipe) *glob(reinterpret_cast<uint32_t *>(fd.tmark + 4u * q)) = 0;
  if (h.m) {
    QuadIn<T> d;
    load_quad<T>(fd, 4u * q, h, d);
    moved = edit_quad<T>(fd, 4u * q, h.m, d, ec, flag ? tag : 0u);
  }
  if (flag) mark_moved_boxes(fd, 4u * q, moved);
}

template <class T, bool SKIP = false>
__device__ __forceinline__ void apply_quads(const FieldDev &fd, uint32_t q0, uint32_t stride,
                                            uint32_t nq, EditCount &ec) {
  const bool flag = fd.frontier && !fd.st->noflag;
  const bool busy = fd.st->busy != 0;
  const uint32_t tag = fd.st->tag;
  const bool wipe = tag == MARK_TAGS;  // the last tag of the cycle: zero every mark
  if (SKIP && !busy && !wipe && chunk_pass(fd)) {
    // (chunk and quad positions in 64 bits, whatever the grid)
    const unsigned long long c0 = __builtin_amdgcn_readfirstlane(q0 >> 6), cs = stride >> 6;
    const unsigned long long nc = (nq + 63) >> 6;
    const uint32_t lane = __lane_id();
    for (unsigned long long s0 = 0; c0 + s0 * cs < nc; s0 += 64) {
      const unsigned long long c = c0 + (s0 + lane) * cs;
      unsigned long long live = __ballot(c < nc && glob(fd.mchunk)[c] == tag);
      if (!live) continue;
      uint32_t q = (uint32_t)(q0 + (s0 + (unsigned long long)(__ffsll(live) - 1)) * stride);
      live &= live - 1;
      QuadHead h = quad_head(fd, q, nq, busy);
      for (;;) {
        const uint32_t qn =
            live ? (uint32_t)(q0 + (s0 + (unsigned long long)(__ffsll(live) - 1)) * stride) : nq;
        live &= live - 1;
        const QuadHead hn = quad_head(fd, qn, nq, busy);
        apply_quad<T>(fd, q, h, tag, false, flag, ec);
        if (qn >= nq) break;
        q = qn;
        h = hn;
      }
    }
    return;
  }
  QuadHead h = quad_head(fd, q0, nq, busy);
  for (uint32_t q = q0; q < nq; q += stride) {
    const QuadHead hn = quad_head(fd, q + stride, nq, busy);
    apply_quad<T>(fd, q, h, tag, wipe, flag, ec);
    h = hn;
  }
}

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
  // a work-group may flush again (the batched apply does, once per field it
  // moves on from): part must not be rewritten before it has been summed
  __syncthreads();
}

constexpr uint32_t NOFLAG_PER_BOX = 4;

// Sums the shards of the apply pass and decides how the loop goes on.
__device__ __forceinline__ void finalize_field(const FieldDev &fd) {
  State *st = fd.st;
  if (st->done) return;
  const int lane = threadIdx.x;
  if (lane == 0) {
    st->passes += 1;
    st->tag = st->tag % MARK_TAGS + 1;
  }
  uint32_t v[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    v[k] = wave_sum(st->shard[k][lane]);
    st->shard[k][lane] = 0;
  }
  if (lane != 0) return;
  const uint32_t nt = v[0], ch = v[1];
  st->ntargets = nt;
  st->changed = ch;
  if (fd.trace && st->iterations < fd.trace_cap) {
    fd.trace[2 * st->iterations] = nt;
    fd.trace[2 * st->iterations + 1] = ch;
  }
  // Were the targets just applied named by a check that covered every box?
  if (ch == 0 && fd.frontier && !st->dense) {
    // A frontier pass skips boxes whose requests were all blocked, so it
    // cannot tell a fixpoint from convergence (or count the residual): a
    // dense pass over the unchanged field settles it.
    st->dense = 1;
    st->noflag = 0;
  } else if (nt == 0) {
    st->done = CONVERGED;
  } else if (ch == 0) {
    st->done = STUCK;
    st->residual = nt;
  } else {
    // an apply that set no box flags is followed by a check of every box;
    // after many changes (more than NOFLAG_PER_BOX per box) nearly every box
    // would be flagged, so the next apply skips the flags
    st->dense = st->noflag;
    st->noflag = fd.frontier && ch > NOFLAG_PER_BOX * (uint32_t)fd.ntiles;
    st->busy = ch > (uint32_t)fd.n / 64;
    st->iterations += 1;
    st->edit_ops += ch;
    st->lossless_total += v[2];
    st->floor_total += v[3];
    st->edited_total += v[4];
    st->targets_total += nt;
    if (st->max_iters > 0 && st->iterations >= st->max_iters) st->done = MAXITERS;
  }
}


// Box shapes (TY, TZ) with compiled kernels; the tile_y / tile_z options
// pick one of them.
#define EXZ_BOX_SHAPES(X) \
  X(1, 1) X(2, 2) X(4, 1) X(4, 2) X(4, 4) X(8, 1) X(8, 2) X(8, 4) X(4, 8) X(16, 1) X(16, 2)

}  // namespace exz
