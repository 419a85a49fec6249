// TEST INFRASTRUCTURE ONLY -- the CPU oracle of the EXaCTz correction loop.
//
// A plain, slow, sequential reference of what the GPU library computes.  Only
// the test suite, the smoke check and the CPU-baseline leg of the benchmark
// load it; the product path never does.  It shares no code, header or table
// with the GPU library.
//
// What it follows (EXaCTz, arXiv 2604.01397):
//  * PL scalar field on vertices, ties broken by Simulation of Simplicity: on
//    equal values the vertex with the larger global index is larger
//    (Sec. 3.3, footnote).
//  * Integral paths step to the highest / lowest neighbour (Sec. 3.1);
//    critical types from the lower / upper link (Sec. 3.2).
//  * Algorithm 1: g <- g_hat; repeat { S <- CheckConstraints(g, f); stop if
//    S is empty; g <- ApplyBoundedEdits(g, S, xi) }.
//  * CheckConstraints (Sec. 4.2): steepest-ascent / steepest-descent
//    neighbours must match f; a saddle keeps its order with every neighbour;
//    event constraints either in their original form (saddle order + per
//    saddle extremum selection by integral-path tracing, Sec. 4.2) or in the
//    reformulated form (order of all critical points of f, Sec. 4.3).
//  * ApplyBoundedEdits (Sec. 3.3): decrease by Delta = xi/N per iteration,
//    never below the lower bound f - xi; more than N edits store the lower
//    bound itself.
//
// Readings where the paper is silent (mesh, tie index, which vertex each rule
// decreases, spurious saddles, edit schedule, float floor) are the ones listed
// in the project's design notes; each is restated where it is used below.
//
// Floating point: every value operation is done in the field type T with
// round-to-nearest-even, except the band bounds, which are computed with the
// hardware rounding mode switched to upward / downward (fesetround).  Build
// with -frounding-math -ffp-contract=off.

#include <algorithm>
#include <array>
#include <cfenv>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <random>
#include <vector>

#pragma STDC FENV_ACCESS ON

namespace {

enum { TYPE_REGULAR = 0, TYPE_MIN = 1, TYPE_MAX = 2, TYPE_SADDLE = 3 };
enum { MODE_REFORMULATED = 0, MODE_ORIGINAL = 1 };
enum {
  ST_OK = 0, ST_STUCK = 1, ST_MAX_ITERS = 2,
  ST_INVALID = -1, ST_NONFINITE = -2, ST_BOUND = -3
};

// ---------------------------------------------------------------------------
// mesh

struct Mesh {
  int64_t nx = 1, ny = 1, nz = 1, n = 0;
  std::vector<std::array<int, 3>> offs;  // neighbour offsets (dx, dy, dz)
  std::vector<std::vector<char>> adj;    // adj[a][b]: link edge between offsets a, b
};

bool link_edge(const Mesh &m, int a, int b);

// 3D: the Freudenthal (Kuhn) triangulation of the cube grid -- every nonzero
// v in {-1,0,1}^3 whose nonzero entries share one sign (14 neighbours).
// 2D: the same rule in the plane, i.e. (+-1,0), (0,+-1), +(1,1), -(1,1).
// 1D: +-1.
bool make_mesh(int ndim, const int64_t *dims, Mesh &m) {
  if (ndim < 1 || ndim > 3) return false;
  int64_t d[3] = {1, 1, 1};
  for (int k = 0; k < ndim; ++k) {
    if (dims[k] < 1) return false;
    d[k] = dims[k];
  }
  m.nx = d[0]; m.ny = d[1]; m.nz = d[2];
  m.n = m.nx * m.ny * m.nz;
  m.offs.clear();
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int v[3] = {dx, dy, dz};
        bool pos = false, neg = false, zero = true;
        for (int k = 0; k < 3; ++k) {
          if (v[k] > 0) pos = true;
          if (v[k] < 0) neg = true;
          if (v[k] != 0) zero = false;
        }
        if (zero || (pos && neg)) continue;
        if (ndim < 3 && dz != 0) continue;
        if (ndim < 2 && dy != 0) continue;
        m.offs.push_back({dx, dy, dz});
      }
  const int k = (int)m.offs.size();
  m.adj.assign(k, std::vector<char>(k, 0));
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) m.adj[a][b] = link_edge(m, a, b);
  return true;
}

// In-domain neighbours of i: pairs (offset index, vertex index).
void neighbours(const Mesh &m, int64_t i, std::vector<std::pair<int, int64_t>> &out) {
  out.clear();
  const int64_t x = i % m.nx, y = (i / m.nx) % m.ny, z = i / (m.nx * m.ny);
  for (int s = 0; s < (int)m.offs.size(); ++s) {
    const int64_t X = x + m.offs[s][0], Y = y + m.offs[s][1], Z = z + m.offs[s][2];
    if (X < 0 || Y < 0 || Z < 0 || X >= m.nx || Y >= m.ny || Z >= m.nz) continue;
    out.push_back({s, X + m.nx * (Y + m.ny * Z)});
  }
}

// Two neighbours a, b of a vertex span a triangle with it (a link edge) iff
// their difference is itself a mesh offset.
bool link_edge(const Mesh &m, int a, int b) {
  int d[3];
  for (int k = 0; k < 3; ++k) d[k] = m.offs[b][k] - m.offs[a][k];
  for (auto &o : m.offs)
    if (o[0] == d[0] && o[1] == d[1] && o[2] == d[2]) return true;
  return false;
}

// ---------------------------------------------------------------------------
// order and local topology of a field h

// SoS order: h_i < h_j, or equal values and i < j.  IEEE comparison, so
// -0 == +0 and the tie goes to the index.
template <class T>
inline bool lt(const T *h, int64_t i, int64_t j) {
  return h[i] < h[j] || (h[i] == h[j] && i < j);
}

struct Local {
  int64_t asc, desc;   // SoS argmax / argmin over the closed neighbourhood
  uint32_t lower;      // bit s set: neighbour at offset s is lower than i
  int lc, uc;          // components of the lower / upper link
  int type;
};

// Connected components of the link vertices selected by `sel` (offset bits),
// joined by link edges.  Plain breadth-first search.
int components(const Mesh &m, const std::vector<std::pair<int, int64_t>> &nb,
               uint32_t sel) {
  std::vector<int> nodes;
  for (auto &p : nb)
    if (sel >> p.first & 1u) nodes.push_back(p.first);
  std::vector<char> seen(nodes.size(), 0);
  int comps = 0;
  for (size_t s = 0; s < nodes.size(); ++s) {
    if (seen[s]) continue;
    ++comps;
    std::vector<size_t> stack{s};
    seen[s] = 1;
    while (!stack.empty()) {
      size_t a = stack.back();
      stack.pop_back();
      for (size_t b = 0; b < nodes.size(); ++b)
        if (!seen[b] && m.adj[nodes[a]][nodes[b]]) {
          seen[b] = 1;
          stack.push_back(b);
        }
    }
  }
  return comps;
}

// Steepest neighbours and lower-link mask only (fills nb).
template <class T>
Local pointers(const Mesh &m, const T *h, int64_t i,
               std::vector<std::pair<int, int64_t>> &nb) {
  neighbours(m, i, nb);
  Local L;
  L.asc = i;
  L.desc = i;
  L.lower = 0;
  L.lc = L.uc = -1;
  L.type = -1;
  for (auto &p : nb) {
    const int64_t j = p.second;
    if (lt(h, j, i)) L.lower |= 1u << p.first;
    if (lt(h, L.asc, j)) L.asc = j;
    if (lt(h, j, L.desc)) L.desc = j;
  }
  return L;
}

// Link component counts and critical type from the lower-link mask.
void classify(const Mesh &m, const std::vector<std::pair<int, int64_t>> &nb,
              Local &L) {
  uint32_t all = 0;
  for (auto &p : nb) all |= 1u << p.first;
  L.lc = components(m, nb, L.lower);
  L.uc = components(m, nb, all & ~L.lower);
  if (L.lower == 0)
    L.type = TYPE_MIN;
  else if (L.lower == all)
    L.type = TYPE_MAX;
  else if (L.lc == 1 && L.uc == 1)
    L.type = TYPE_REGULAR;
  else
    L.type = TYPE_SADDLE;
}

template <class T>
Local local_topology(const Mesh &m, const T *h, int64_t i,
                     std::vector<std::pair<int, int64_t>> &nb) {
  Local L = pointers(m, h, i, nb);
  classify(m, nb, L);
  return L;
}

// Vertex reached by following pointers p from v until a fixed point.
int64_t terminus(const std::vector<int64_t> &p, int64_t v) {
  while (p[v] != v) v = p[v];
  return v;
}

// ---------------------------------------------------------------------------
// bounds

// xi_T: the largest T not above xi.  L_i: the smallest T not below f_i - xi_T.
// U_i: the largest T not above f_i + xi_T.  Computed by switching the FPU
// rounding direction; volatile keeps the compiler from folding across it.
template <class T>
T round_down_xi(double xi) {
  const int old = fegetround();
  fesetround(FE_DOWNWARD);
  volatile double v = xi;
  volatile T r = (T)v;
  fesetround(old);
  return r;
}

template <class T>
void bounds(T f, T xiT, T &L, T &U) {
  const int old = fegetround();
  volatile T a = f, b = xiT;
  fesetround(FE_UPWARD);
  volatile T lo = a - b;
  fesetround(FE_DOWNWARD);
  volatile T hi = a + b;
  fesetround(old);
  L = lo;
  U = hi;
}

template <class T>
T step_size(T xiT, int N) {
  volatile T a = xiT, b = (T)N;
  volatile T d = a / b;  // default rounding: to nearest, ties to even
  return d;
}

// ---------------------------------------------------------------------------
// reference topology of f and the check pass

struct Reference {
  Mesh mesh;
  std::vector<int64_t> asc, desc;
  std::vector<uint32_t> lower;
  std::vector<int8_t> type;
  std::vector<int8_t> lc, uc;
  std::vector<int64_t> cps;       // critical points of f, ascending in SoS(f)
  std::vector<int64_t> saddles;   // saddles of f, ascending in SoS(f)
  std::vector<int64_t> mf;        // per saddle (original mode): join selection
  std::vector<int64_t> Mf;        // per saddle (original mode): split selection
};

template <class T>
void build_reference(const Mesh &m, const T *f, int mode, Reference &R) {
  const int64_t n = m.n;
  R.mesh = m;
  R.asc.resize(n); R.desc.resize(n); R.lower.resize(n);
  R.type.resize(n); R.lc.resize(n); R.uc.resize(n);
  std::vector<std::pair<int, int64_t>> nb;
  for (int64_t i = 0; i < n; ++i) {
    Local L = local_topology(m, f, i, nb);
    R.asc[i] = L.asc; R.desc[i] = L.desc; R.lower[i] = L.lower;
    R.type[i] = (int8_t)L.type; R.lc[i] = (int8_t)L.lc; R.uc[i] = (int8_t)L.uc;
  }
  R.cps.clear();
  for (int64_t i = 0; i < n; ++i)
    if (R.type[i] != TYPE_REGULAR) R.cps.push_back(i);
  std::sort(R.cps.begin(), R.cps.end(),
            [&](int64_t a, int64_t b) { return lt(f, a, b); });
  R.saddles.clear();
  for (int64_t c : R.cps)
    if (R.type[c] == TYPE_SADDLE) R.saddles.push_back(c);
  R.mf.assign(R.saddles.size(), -1);
  R.Mf.assign(R.saddles.size(), -1);
  if (mode == MODE_ORIGINAL) {
    // Extremum selected by each saddle in f (Sec. 4.2, event constraints):
    // join saddle -> the highest minimum reached by descending from its lower
    // link; split saddle -> the lowest maximum reached by ascending from its
    // upper link.
    for (size_t k = 0; k < R.saddles.size(); ++k) {
      const int64_t s = R.saddles[k];
      neighbours(m, s, nb);
      if (R.lc[s] >= 2)
        for (auto &p : nb)
          if (R.lower[s] >> p.first & 1u) {
            const int64_t t = terminus(R.desc, p.second);
            if (R.mf[k] < 0 || lt(f, R.mf[k], t)) R.mf[k] = t;
          }
      if (R.uc[s] >= 2)
        for (auto &p : nb)
          if (!(R.lower[s] >> p.first & 1u)) {
            const int64_t t = terminus(R.asc, p.second);
            if (R.Mf[k] < 0 || lt(f, t, R.Mf[k])) R.Mf[k] = t;
          }
    }
  }
}

// One CheckConstraints pass on g: sets mark[t] = 1 for every vertex t the
// rules ask to decrease.  Returns the number of marked vertices.
template <class T>
int64_t check(const Reference &R, const T *f, const T *g, int mode,
              std::vector<uint8_t> &mark, const std::vector<int64_t> &order) {
  const Mesh &m = R.mesh;
  std::fill(mark.begin(), mark.end(), 0);
  std::vector<std::pair<int, int64_t>> nb;
  std::vector<int64_t> gasc, gdesc;
  if (mode == MODE_ORIGINAL) {
    gasc.resize(m.n);
    gdesc.resize(m.n);
  }
  for (int64_t i : order) {
    Local G = pointers(m, g, i, nb);
    // The type only matters below for a regular vertex of f; with the same
    // lower link as in f it is regular in g as well.
    if (R.type[i] == TYPE_REGULAR) {
      if (G.lower == R.lower[i])
        G.type = TYPE_REGULAR;
      else
        classify(m, nb, G);
    }
    if (mode == MODE_ORIGINAL) {
      gasc[i] = G.asc;
      gdesc[i] = G.desc;
    }
    // EG constraints, ascending side: the neighbour g now takes as steepest
    // ascent is wrongly high -- decrease it.
    if (G.asc != R.asc[i]) mark[G.asc] = 1;
    // EG constraints, descending side: decrease the neighbour f takes as
    // steepest descent, so it becomes the lowest again.
    if (G.desc != R.desc[i]) mark[R.desc[i]] = 1;
    // Saddle link order (and critical-point consistency for a regular vertex
    // of f that g turned into a saddle): every flipped pair with a neighbour
    // is repaired by decreasing whichever of the two is lower in f.
    if (R.type[i] == TYPE_SADDLE ||
        (R.type[i] == TYPE_REGULAR && G.type == TYPE_SADDLE)) {
      for (auto &p : nb) {
        const bool lower_f = R.lower[i] >> p.first & 1u;
        const bool lower_g = G.lower >> p.first & 1u;
        if (lower_f != lower_g) mark[lower_f ? p.second : i] = 1;
      }
    }
  }
  if (mode == MODE_REFORMULATED) {
    // Reformulated event constraints: every critical point of f keeps its
    // place among all critical points; an inverted consecutive pair
    // decreases the one that is lower in f.
    for (size_t k = 0; k + 1 < R.cps.size(); ++k)
      if (lt(g, R.cps[k + 1], R.cps[k])) mark[R.cps[k]] = 1;
  } else {
    // Saddle ordering constraints (C2): consecutive saddles of f.
    for (size_t k = 0; k + 1 < R.saddles.size(); ++k)
      if (lt(g, R.saddles[k + 1], R.saddles[k])) mark[R.saddles[k]] = 1;
    // Event constraints (C3) by integral-path tracing in g.  When the
    // extremum a saddle selects in g differs from its selection in f, the
    // edit goes where Sec. 4.2 puts it: a join saddle lowers the minimum g
    // selects until it sits below f's choice; a split saddle, by the same
    // argument with decreasing edits only, lowers f's choice of maximum until
    // it sits below the one g selects.
    for (size_t k = 0; k < R.saddles.size(); ++k) {
      const int64_t s = R.saddles[k];
      neighbours(m, s, nb);
      uint32_t glower = 0;
      for (auto &p : nb)
        if (lt(g, p.second, s)) glower |= 1u << p.first;
      if (R.lc[s] >= 2) {
        int64_t sel = -1;
        for (auto &p : nb)
          if (glower >> p.first & 1u) {
            const int64_t t = terminus(gdesc, p.second);
            if (sel < 0 || lt(g, sel, t)) sel = t;
          }
        if (sel >= 0 && sel != R.mf[k]) mark[sel] = 1;
      }
      if (R.uc[s] >= 2) {
        int64_t sel = -1;
        for (auto &p : nb)
          if (!(glower >> p.first & 1u)) {
            const int64_t t = terminus(gasc, p.second);
            if (sel < 0 || lt(g, t, sel)) sel = t;
          }
        if (sel >= 0 && sel != R.Mf[k]) mark[R.Mf[k]] = 1;
      }
    }
  }
  int64_t cnt = 0;
  for (int64_t i = 0; i < m.n; ++i) cnt += mark[i];
  return cnt;
}

// ---------------------------------------------------------------------------
// the loop

struct Stats {
  int64_t iterations, edited_vertices, edit_ops, lossless_vertices,
      floor_vertices, residual_violations, num_critical, status;
};

template <class T>
int correct(int ndim, const int64_t *dims, const T *f, const T *g_hat, T *g_out,
            uint8_t *cnt_io, int resume, double xi, int N, int mode,
            int64_t max_iters, uint64_t shuffle_seed, int64_t *trace,
            int64_t trace_cap, Stats &st) {
  std::memset(&st, 0, sizeof st);
  Mesh m;
  if (!make_mesh(ndim, dims, m) || !(xi > 0) || !std::isfinite(xi) || N < 1 ||
      N > 14 || (mode != MODE_REFORMULATED && mode != MODE_ORIGINAL))
    return st.status = ST_INVALID;
  const int64_t n = m.n;
  const T xiT = round_down_xi<T>(xi);
  if (!(xiT > 0)) return st.status = ST_INVALID;
  const T delta = step_size(xiT, N);

  // Validation: finite inputs and g_hat inside [L_i, U_i].
  std::vector<T> Lb(n), Ub(n);
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(f[i]) || !std::isfinite(g_hat[i])) return st.status = ST_NONFINITE;
  }
  for (int64_t i = 0; i < n; ++i) {
    bounds(f[i], xiT, Lb[i], Ub[i]);
    if (g_hat[i] < Lb[i] || g_hat[i] > Ub[i]) return st.status = ST_BOUND;
  }

  Reference R;
  build_reference(m, f, mode, R);
  st.num_critical = (int64_t)R.cps.size();

  std::vector<T> g(g_hat, g_hat + n);
  std::vector<uint8_t> cnt(n, 0);
  if (resume && cnt_io) std::copy(cnt_io, cnt_io + n, cnt.begin());

  std::vector<int64_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = i;
  if (shuffle_seed) {
    std::mt19937_64 rng(shuffle_seed);
    std::shuffle(order.begin(), order.end(), rng);
  }

  std::vector<uint8_t> mark(n, 0);
  int status = ST_OK;
  for (;;) {
    const int64_t nt = check(R, f, g.data(), mode, mark, order);
    if (nt == 0) break;  // converged
    // ApplyBoundedEdits on a snapshot: each target moves once, from its own
    // value in g^t.  A target already at its lower bound cannot move.
    std::vector<T> next(g);
    int64_t changed = 0;
    for (int64_t t : order) {
      if (!mark[t]) continue;
      const T g0 = g[t];
      if (g0 == Lb[t]) continue;  // blocked at the floor
      const int c = cnt[t] + 1;
      cnt[t] = (uint8_t)c;
      T v;
      if (c > N) {
        v = Lb[t];  // lossless: store the lower bound itself
        ++st.lossless_vertices;
      } else {
        const T cand = g0 - delta;
        v = cand < Lb[t] ? Lb[t] : cand;
      }
      next[t] = v;
      if (v == Lb[t]) ++st.floor_vertices;
      if (c == 1) ++st.edited_vertices;
      ++changed;
    }
    if (trace && st.iterations < trace_cap) {
      trace[2 * st.iterations] = nt;
      trace[2 * st.iterations + 1] = changed;
    }
    if (changed == 0) {  // nothing can move: fixpoint with violations left
      st.residual_violations = nt;
      status = ST_STUCK;
      break;
    }
    g.swap(next);
    st.edit_ops += changed;
    ++st.iterations;
    if (max_iters > 0 && st.iterations >= max_iters) {
      status = ST_MAX_ITERS;
      break;
    }
  }
  std::copy(g.begin(), g.end(), g_out);
  if (cnt_io) std::copy(cnt.begin(), cnt.end(), cnt_io);
  return st.status = status;
}

}  // namespace

// ---------------------------------------------------------------------------
// C entry points (ctypes).  dtype: 0 = float32, 1 = float64.

extern "C" {

// Full correction.  stats[8] = {iterations, edited_vertices, edit_ops,
// lossless_vertices, floor_vertices, residual_violations, num_critical,
// status}.  trace (nullable) receives (|T^t|, changed^t) pairs.
int oref_correct(int ndim, const int64_t *dims, int dtype, const void *f,
                 const void *g_hat, void *g_out, uint8_t *cnt_io, int resume,
                 double xi, int n_steps, int mode, int64_t max_iters,
                 uint64_t shuffle_seed, int64_t *trace, int64_t trace_cap,
                 int64_t *stats) {
  Stats st;
  int r;
  if (dtype == 0)
    r = correct<float>(ndim, dims, (const float *)f, (const float *)g_hat,
                       (float *)g_out, cnt_io, resume, xi, n_steps, mode,
                       max_iters, shuffle_seed, trace, trace_cap, st);
  else if (dtype == 1)
    r = correct<double>(ndim, dims, (const double *)f, (const double *)g_hat,
                        (double *)g_out, cnt_io, resume, xi, n_steps, mode,
                        max_iters, shuffle_seed, trace, trace_cap, st);
  else
    return ST_INVALID;
  if (stats) {
    const int64_t v[8] = {st.iterations, st.edited_vertices, st.edit_ops,
                          st.lossless_vertices, st.floor_vertices,
                          st.residual_violations, st.num_critical, st.status};
    std::memcpy(stats, v, sizeof v);
  }
  return r;
}

// One CheckConstraints pass of field g against reference f (no validation).
// mark_out[n] receives 0/1.  Returns |T|, or -1 on bad arguments.
int64_t oref_targets(int ndim, const int64_t *dims, int dtype, const void *f,
                     const void *g, int mode, uint8_t *mark_out) {
  Mesh m;
  if (!make_mesh(ndim, dims, m)) return -1;
  std::vector<int64_t> order(m.n);
  for (int64_t i = 0; i < m.n; ++i) order[i] = i;
  std::vector<uint8_t> mark(m.n, 0);
  Reference R;
  int64_t c;
  if (dtype == 0) {
    build_reference(m, (const float *)f, mode, R);
    c = check(R, (const float *)f, (const float *)g, mode, mark, order);
  } else if (dtype == 1) {
    build_reference(m, (const double *)f, mode, R);
    c = check(R, (const double *)f, (const double *)g, mode, mark, order);
  } else {
    return -1;
  }
  std::copy(mark.begin(), mark.end(), mark_out);
  return c;
}

// Local topology of every vertex of h: asc/desc vertex, lower-link offset
// mask, lower/upper link component counts and type (0 regular, 1 min, 2 max,
// 3 saddle).  Any output pointer may be null.
int oref_topology(int ndim, const int64_t *dims, int dtype, const void *h,
                  int64_t *asc, int64_t *desc, uint32_t *lower, int8_t *lc,
                  int8_t *uc, int8_t *type) {
  Mesh m;
  if (!make_mesh(ndim, dims, m)) return -1;
  std::vector<std::pair<int, int64_t>> nb;
  for (int64_t i = 0; i < m.n; ++i) {
    Local L = dtype == 0 ? local_topology(m, (const float *)h, i, nb)
                         : local_topology(m, (const double *)h, i, nb);
    if (asc) asc[i] = L.asc;
    if (desc) desc[i] = L.desc;
    if (lower) lower[i] = L.lower;
    if (lc) lc[i] = (int8_t)L.lc;
    if (uc) uc[i] = (int8_t)L.uc;
    if (type) type[i] = (int8_t)L.type;
  }
  return 0;
}

// Critical points of h in ascending SoS order; returns K (fills at most cap).
int64_t oref_critical_order(int ndim, const int64_t *dims, int dtype,
                            const void *h, int64_t *out, int64_t cap) {
  Mesh m;
  if (!make_mesh(ndim, dims, m)) return -1;
  Reference R;
  if (dtype == 0)
    build_reference(m, (const float *)h, MODE_REFORMULATED, R);
  else
    build_reference(m, (const double *)h, MODE_REFORMULATED, R);
  for (int64_t k = 0; k < (int64_t)R.cps.size() && k < cap; ++k) out[k] = R.cps[k];
  return (int64_t)R.cps.size();
}

// Mesh offsets (3 ints each); returns their count.
int oref_offsets(int ndim, int *out) {
  Mesh m;
  const int64_t dims[3] = {3, 3, 3};
  if (!make_mesh(ndim, dims, m)) return -1;
  for (size_t s = 0; s < m.offs.size(); ++s)
    for (int k = 0; k < 3; ++k) out[3 * s + k] = m.offs[s][k];
  return (int)m.offs.size();
}

// Band bounds, xi_T and Delta for n values of f.
int oref_bounds(int dtype, int64_t n, const void *f, double xi, int n_steps,
                void *L, void *U, double *xiT_out, double *delta_out) {
  if (dtype == 0) {
    const float xiT = round_down_xi<float>(xi);
    for (int64_t i = 0; i < n; ++i)
      bounds(((const float *)f)[i], xiT, ((float *)L)[i], ((float *)U)[i]);
    *xiT_out = xiT;
    *delta_out = step_size(xiT, n_steps);
  } else if (dtype == 1) {
    const double xiT = round_down_xi<double>(xi);
    for (int64_t i = 0; i < n; ++i)
      bounds(((const double *)f)[i], xiT, ((double *)L)[i], ((double *)U)[i]);
    *xiT_out = xiT;
    *delta_out = step_size(xiT, n_steps);
  } else {
    return -1;
  }
  return 0;
}

}  // extern "C"
