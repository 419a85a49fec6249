// Original event constraints (Sec. 4.2) and the extremum-graph certificate.
//
// The original form of the event constraints needs, per saddle of f, the
// extremum its integral paths select: a join saddle (its lower link has two
// or more components) selects the highest minimum reached by steepest descent
// from its lower neighbours, a split saddle the lowest maximum reached by
// steepest ascent from its upper neighbours (Sec. 3.1-3.2, 4.1 C3).  For f
// (once, at set-up) and for the certificate the paths of every vertex are
// resolved at once by pointer jumping over the steepest descent / ascent
// pointers: lab[v] <- lab[lab[v]] until nothing changes, a logarithmic
// number of rounds in the longest path.  Descent labels occupy lab[0, n),
// ascent labels lab[n, 2n) (stored as n + vertex).
//
// Per iteration (original mode) only the paths from the link neighbours of
// f's saddles are needed: the check pass writes g's pointers and one kernel
// follows those paths on them (setting each start's pointer to its path's
// end, so shared paths are walked once) and applies (C2 with a thread per
// saddle in f's order, C3 with a thread per critical point in vertex order)
//   C2  consecutive saddles of f keep their order in g (the lower one in f
//       goes down when inverted), and
//   C3  the selection in g equals the selection in f; otherwise a join
//       saddle lowers the minimum g selects (below f's choice) and a split
//       saddle lowers f's choice of maximum (below g's), the edits Sec. 4.2
//       prescribes with decreasing edits only.
// The certificate compares the path termini of f and g' for every vertex and
// all critical types: the extremum-graph identity of Sec. 4.1, C1.
#include "exz_host.h"

namespace exz {

// --- saddle order: ranks (in the CP order) of the saddles of f -------------

__global__ void k_saddle_flags(FieldDev fd, uint32_t *flags) {
  const uint32_t r = blockIdx.x * 256 + threadIdx.x;
  if (r < (uint32_t)fd.K) flags[r] = (fd.low[fd.cp_idx[r]] & LOW_SADDLE) ? 1u : 0u;
}

__global__ void k_saddle_scatter(FieldDev fd, const uint32_t *pre) {
  const uint32_t r = blockIdx.x * 256 + threadIdx.x;
  if (r >= (uint32_t)fd.K) return;
  if (pre[r + 1] != pre[r]) fd.sad_rank[pre[r]] = r;
  if (r == 0) fd.st->nsaddle = pre[fd.K];
}

// --- pointers and jumping --------------------------------------------------

// f's steepest descent / ascent pointers from the reference code byte.
__global__ void k_ptr_f(FieldDev fd, uint32_t *lab) {
  const uint32_t v = blockIdx.x * 256 + threadIdx.x;
  if (v >= (uint32_t)fd.n) return;
  const uint32_t code = fd.code[v];
  const uint32_t a = code & 15u, d = code >> 4;
  lab[v] = d == SELF ? v : (uint32_t)((int)v + fd.dlt[d]);
  lab[fd.n + v] = (uint32_t)fd.n + (a == SELF ? v : (uint32_t)((int)v + fd.dlt[a]));
}

// One pointer-jumping round over count labels; flag[round] records whether
// anything moved.  A round after an unchanged one returns at once.  A label
// whose target points at itself has reached its chain's end and never
// changes again: bit v of conv records that, so later rounds read one
// 32-bit word per 32 such labels instead of the labels.  Each wave takes 64
// consecutive labels, i.e. two whole words of conv, and is their only
// writer.
__global__ void k_jump(uint32_t *lab, uint32_t count, uint32_t *conv, State *st, int round,
                       int honour_done) {
  if (honour_done && st->done) return;
  if (round > 0 && st->jump[round - 1] == 0) return;
  const uint32_t lane = threadIdx.x & 63u;
  const unsigned long long wave = (blockIdx.x * 256ull + threadIdx.x) >> 6;
  const unsigned long long waves = gridDim.x * 4ull;
  bool moved = false;
  for (unsigned long long base = wave * 64; base < count; base += waves * 64) {
    const uint32_t v = (uint32_t)base + lane;
    const uint32_t w = (uint32_t)(base >> 5) + (lane >> 5);
    const uint32_t old = conv[w];
    bool fin = (unsigned long long)v >= count || ((old >> (lane & 31u)) & 1u);
    if (!fin) {
      const uint32_t p = lab[v];
      const uint32_t q = lab[p];
      if (q != p) {
        lab[v] = q;
        moved = true;
      } else {
        fin = true;
      }
    }
    const unsigned long long b = __ballot(fin);
    const uint32_t nw = lane < 32 ? (uint32_t)b : (uint32_t)(b >> 32);
    if ((lane & 31u) == 0 && nw != old) conv[w] = nw;
  }
  if (__any(moved) && __lane_id() == 0) st->jump[round] = 1u;
}

__global__ void k_jump_reset(State *st, uint32_t *conv, uint32_t words) {
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  if (t < MAX_JUMP_ROUNDS) st->jump[t] = 0;
  for (uint32_t k = t; k < words; k += gridDim.x * 256) conv[k] = 0;
}

int jump_rounds(uint32_t count) {
  int r = 1;
  while ((1ull << (r - 1)) < (unsigned long long)count && r < MAX_JUMP_ROUNDS) ++r;
  return r;
}

// Words of the convergence bitmask of count labels: two per 64 labels.
size_t jump_conv_words(uint64_t count) { return (size_t)((count + 63) / 64) * 2; }

// Resolves count labels.  The convergence bitmask lives right after the
// 2n labels of fd.lab (the caller's layout reserves it there); the labels
// resolved here may be fd.lab's own or another array of 2n labels.
static hipError_t jump_all(const FieldDev &fd, uint32_t *lab, uint32_t count, int honour_done,
                           hipStream_t s) {
  uint32_t *conv = fd.lab + 2 * (size_t)fd.n;
  const uint32_t words = (uint32_t)jump_conv_words(count);
  const uint32_t gw = (words + 255) / 256;
  hipLaunchKernelGGL(k_jump_reset, dim3(gw < 1024 ? (gw ? gw : 1) : 1024), dim3(256), 0, s, fd.st,
                     conv, words);
  const uint32_t g = (count + 255) / 256;
  const int grid = (int)(g < 4096 ? (g ? g : 1) : 4096);
  const int rounds = jump_rounds(count);
  for (int r = 0; r < rounds; ++r)
    hipLaunchKernelGGL(k_jump, dim3(grid), dim3(256), 0, s, lab, count, conv, fd.st, r,
                       honour_done);
  return hipGetLastError();
}

// --- per-saddle selections -------------------------------------------------

__device__ __forceinline__ void coords(const FieldDev &fd, uint32_t v, int &x, int &y, int &z) {
  x = (int)(v % (uint32_t)fd.nx);
  const uint32_t r = v / (uint32_t)fd.nx;
  y = (int)(r % (uint32_t)fd.ny);
  z = (int)(r / (uint32_t)fd.ny);
}

// Extremum selected by saddle s of field h over the neighbours in `sel`:
// join: SoS-highest descent terminus; split: SoS-lowest ascent terminus.
template <class T>
__device__ __forceinline__ uint32_t select_extremum(const FieldDev &fd, const T *h,
                                                    const uint32_t *lab, uint32_t s, uint32_t sel,
                                                    bool join) {
  uint32_t best = NONE;
  T bv = T(0);
  for (int k = 0; k < NSLOT; ++k) {
    if (!((sel >> k) & 1u)) continue;
    const uint32_t j = (uint32_t)((int)s + fd.dlt[k]);
    const uint32_t t = join ? lab[j] : lab[fd.n + j] - (uint32_t)fd.n;
    const T tv = h[t];
    const bool better = best == NONE || (join ? sos_lt(bv, best, tv, t) : sos_lt(tv, t, bv, best));
    if (better) {
      best = t;
      bv = tv;
    }
  }
  return best;
}

// Selections of f, per critical point in vertex order (slot vo of cp_vtx):
// neighbouring threads then read neighbouring vertices.  Critical points
// that are not saddles select nothing.
template <class T>
__global__ void k_select_f(FieldDev fd, const uint8_t *comp) {
  const uint32_t k = blockIdx.x * 256 + threadIdx.x;
  if (k >= (uint32_t)fd.K) return;
  const T *F = (const T *)fd.f;
  const uint32_t s = fd.cp_vtx[k];
  if (!(fd.low[s] & LOW_SADDLE)) {
    fd.sel_f[2 * k] = NONE;
    fd.sel_f[2 * k + 1] = NONE;
    return;
  }
  int x, y, z;
  coords(fd, s, x, y, z);
  const uint32_t vm = valid_slots(x, y, z, fd.nx, fd.ny, fd.nz);
  const uint32_t lower = fd.low[s] & LOW_MASK, upper = vm & ~lower;
  fd.sel_f[2 * k] = comp[lower] >= 2 ? select_extremum(fd, F, fd.lab_f, s, lower, true) : NONE;
  fd.sel_f[2 * k + 1] = comp[upper] >= 2 ? select_extremum(fd, F, fd.lab_f, s, upper, false) : NONE;
}

// End of the steepest descent (join) / ascent (split) path of g from v,
// followed on g's pointers in lab (each pointer goes strictly down / up in
// the simulated order, so a path has fewer than n steps; the bound only
// guards the loop).  The start's pointer is then set to the end, which is
// the end of its path too: later walks through it jump there at once, and a
// walk that reads the old pointer reaches the same end.  (Halving every path
// it walks, as union-find does, measured no faster: the walks are short and
// the cost is the scattered loads of the saddles' neighbourhoods.)
__device__ __forceinline__ uint32_t path_end(const FieldDev &fd, uint32_t *lab, uint32_t v,
                                             bool join) {
  uint32_t *P = join ? lab : lab + fd.n;
  const uint32_t off = join ? 0u : (uint32_t)fd.n;
  uint32_t u = v;
  for (uint32_t step = 0; step < (uint32_t)fd.n; ++step) {
    const uint32_t p = P[u] - off;
    if (p == u) break;
    u = p;
  }
  if (u != v) P[v] = u + off;
  return u;
}

// select_extremum on g's pointers (the path ends followed on the fly).
template <class T>
__device__ __forceinline__ uint32_t select_extremum_g(const FieldDev &fd, const T *h, uint32_t *lab,
                                                      uint32_t s, uint32_t sel, bool join) {
  uint32_t best = NONE;
  T bv = T(0);
  for (int k = 0; k < NSLOT; ++k) {
    if (!((sel >> k) & 1u)) continue;
    const uint32_t t = path_end(fd, lab, (uint32_t)((int)s + fd.dlt[k]), join);
    const T tv = h[t];
    const bool better = best == NONE || (join ? sos_lt(bv, best, tv, t) : sos_lt(tv, t, bv, best));
    if (better) {
      best = t;
      bv = tv;
    }
  }
  return best;
}

// The event constraints of thread k: C2 for the k-th saddle in f's order,
// C3 for the critical point in vertex-order slot k.
template <class T>
__device__ __forceinline__ void events_one(const FieldDev &fd, const uint8_t *comp, uint32_t k) {
  const State *st = fd.st;
  const uint32_t ns = st->nsaddle;
  const uint32_t tag = st->tag;
  const T *G = (const T *)fd.g;
  // C2: saddle order (thread k takes the k-th saddle in f's order)
  if (k + 1 < ns) {
    const uint32_t s = fd.cp_idx[fd.sad_rank[k]];
    const uint32_t sn = fd.cp_idx[fd.sad_rank[k + 1]];
    if (sos_lt(G[sn], sn, G[s], s)) mark_target(fd, s, tag);
  }
  // C3: selected extrema along the integral paths of g (thread k takes the
  // critical point in vertex-order slot k)
  if (k >= (uint32_t)fd.K) return;
  const uint32_t s = fd.cp_vtx[k];
  const uint32_t mf = fd.sel_f[2 * k], Mf = fd.sel_f[2 * k + 1];
  if (mf == NONE && Mf == NONE) return;
  int x, y, z;
  coords(fd, s, x, y, z);
  const uint32_t vm = valid_slots(x, y, z, fd.nx, fd.ny, fd.nz);
  const T gs = G[s];
  uint32_t glower = 0;
  for (int q = 0; q < NSLOT; ++q) {
    if (!((vm >> q) & 1u)) continue;
    const uint32_t j = (uint32_t)((int)s + fd.dlt[q]);
    glower |= (uint32_t)sos_lt(G[j], j, gs, s) << q;
  }
  if (mf != NONE && glower) {
    const uint32_t mg = select_extremum_g(fd, G, fd.lab, s, glower, true);
    if (mg != mf) mark_target(fd, mg, tag);
  }
  const uint32_t gupper = vm & ~glower;
  if (Mf != NONE && gupper) {
    const uint32_t Mg = select_extremum_g(fd, G, fd.lab, s, gupper, false);
    if (Mg != Mf) mark_target(fd, Mf, tag);
  }
}

template <class T>
__global__ void k_events(FieldDev fd, const uint8_t *comp) {
  if (fd.st->done) return;
  events_one<T>(fd, comp, blockIdx.x * 256 + threadIdx.x);
}

__global__ void __launch_bounds__(EVENT_ITEM) k_events_batch(const FieldDev *__restrict__ fields,
                                                             const uint32_t *__restrict__ lists,
                                                             const uint8_t *comp) {
  const uint32_t nf = lists[0], total = lists[1];
  const uint32_t *field = lists + 2, *base = lists + 2 + nf;
  uint32_t k = 0;
  for (uint32_t it = blockIdx.x; it < total; it += gridDim.x) {
    k = next_field_uniform(base, nf, it, k);
    const FieldDev &fd = fields[__builtin_amdgcn_readfirstlane(field[k])];
    if (fd.st->done) continue;
    const uint32_t c = (it - base[k]) * EVENT_ITEM + threadIdx.x;
    if (fd.dtype == 0)
      events_one<float>(fd, comp, c);
    else
      events_one<double>(fd, comp, c);
  }
}

// --- certificate -----------------------------------------------------------

template <class T>
__global__ void k_ptr_g(FieldDev fd, uint32_t *lab) {
  const uint32_t v = blockIdx.x * 256 + threadIdx.x;
  if (v >= (uint32_t)fd.n) return;
  const T *G = (const T *)fd.g;
  int x, y, z;
  coords(fd, v, x, y, z);
  const uint32_t vm = valid_slots(x, y, z, fd.nx, fd.ny, fd.nz);
  const T gv = G[v];
  T amax = gv, amin = gv;
  uint32_t ia = v, id = v;
  for (int q = 0; q < NSLOT; ++q) {
    if (!((vm >> q) & 1u)) continue;
    const uint32_t j = (uint32_t)((int)v + fd.dlt[q]);
    const T gj = G[j];
    if (sos_lt(amax, ia, gj, j)) {
      amax = gj;
      ia = j;
    }
    if (sos_lt(gj, j, amin, id)) {
      amin = gj;
      id = j;
    }
  }
  lab[v] = id;
  lab[fd.n + v] = (uint32_t)fd.n + ia;
}

// Counts vertices whose path termini or critical type differ between f and g.
template <class T>
__global__ void k_cert_compare(FieldDev fd, const uint8_t *comp, const uint32_t *lab_g) {
  const uint32_t v = blockIdx.x * 256 + threadIdx.x;
  bool bad = false;
  if (v < (uint32_t)fd.n) {
    const T *G = (const T *)fd.g;
    bad = lab_g[v] != fd.lab_f[v] || lab_g[fd.n + v] != fd.lab_f[fd.n + v];
    int x, y, z;
    coords(fd, v, x, y, z);
    const uint32_t vm = valid_slots(x, y, z, fd.nx, fd.ny, fd.nz);
    const T gv = G[v];
    uint32_t lower = 0;
    for (int q = 0; q < NSLOT; ++q) {
      if (!((vm >> q) & 1u)) continue;
      const uint32_t j = (uint32_t)((int)v + fd.dlt[q]);
      lower |= (uint32_t)sos_lt(G[j], j, gv, v) << q;
    }
    const uint32_t lf = fd.low[v] & LOW_MASK;
    const bool saddle_f = (fd.low[v] & LOW_SADDLE) != 0;
    const bool ext_g = lower == 0 || lower == vm;
    const bool saddle_g = !ext_g && !(comp[lower] == 1 && comp[vm & ~lower] == 1);
    const bool ext_f = lf == 0 || lf == vm;
    // minima / maxima agree through the path termini (a vertex is its own
    // terminus exactly when it is an extremum); saddles and regular
    // vertices must agree as well
    bad |= saddle_g != saddle_f || ext_g != ext_f;
  }
  if (__any(bad) && __lane_id() == 0) atomicAdd(&fd.st->cert_bad, 1u);
}

// --- launch wrappers -------------------------------------------------------

hipError_t launch_original_setup(const FieldDev &fd, const uint8_t *comp, uint32_t *tmp,
                                 uint32_t *scan_tmp, size_t scan_words, hipStream_t s) {
  const int gk = (fd.K + 255) / 256 ? (fd.K + 255) / 256 : 1;
  hipLaunchKernelGGL(k_saddle_flags, dim3(gk), dim3(256), 0, s, fd, tmp);
  hipError_t e = launch_scan_u32(tmp, tmp, (uint32_t)fd.K, scan_tmp, scan_words, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_saddle_scatter, dim3(gk), dim3(256), 0, s, fd, tmp);
  const int gn = (fd.n + 255) / 256;
  hipLaunchKernelGGL(k_ptr_f, dim3(gn), dim3(256), 0, s, fd, fd.lab_f);
  e = jump_all(fd, fd.lab_f, 2u * (uint32_t)fd.n, 0, s);
  if (e != hipSuccess) return e;
  if (fd.dtype == 0)
    hipLaunchKernelGGL(k_select_f<float>, dim3(gk), dim3(256), 0, s, fd, comp);
  else
    hipLaunchKernelGGL(k_select_f<double>, dim3(gk), dim3(256), 0, s, fd, comp);
  return hipGetLastError();
}

// The check has just written g's pointers into fd.lab; the events follow
// the paths they need from there (no labels of all 2n pointers resolved).
hipError_t launch_original_events(const FieldDev &fd, const uint8_t *comp, hipStream_t s) {
  const int gk = (fd.K + 255) / 256 ? (fd.K + 255) / 256 : 1;
  if (fd.dtype == 0)
    hipLaunchKernelGGL(k_events<float>, dim3(gk), dim3(256), 0, s, fd, comp);
  else
    hipLaunchKernelGGL(k_events<double>, dim3(gk), dim3(256), 0, s, fd, comp);
  return hipGetLastError();
}

hipError_t launch_events_batch(const FieldDev *fields, const uint32_t *lists, const uint8_t *comp,
                               int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_events_batch, dim3(grid), dim3(EVENT_ITEM), 0, s, fields, lists, comp);
  return hipGetLastError();
}

hipError_t launch_certify(const FieldDev &fd, const uint8_t *comp, uint32_t *lab_g,
                          hipStream_t s) {
  const int gn = (fd.n + 255) / 256;
  if (fd.mode != EXZ_EVENT_ORIGINAL) {  // f's resolved labels are built on demand
    hipLaunchKernelGGL(k_ptr_f, dim3(gn), dim3(256), 0, s, fd, fd.lab_f);
    hipError_t e = jump_all(fd, fd.lab_f, 2u * (uint32_t)fd.n, 0, s);
    if (e != hipSuccess) return e;
  }
  if (fd.dtype == 0)
    hipLaunchKernelGGL(k_ptr_g<float>, dim3(gn), dim3(256), 0, s, fd, lab_g);
  else
    hipLaunchKernelGGL(k_ptr_g<double>, dim3(gn), dim3(256), 0, s, fd, lab_g);
  hipError_t e = jump_all(fd, lab_g, 2u * (uint32_t)fd.n, 0, s);
  if (e != hipSuccess) return e;
  if (fd.dtype == 0)
    hipLaunchKernelGGL(k_cert_compare<float>, dim3(gn), dim3(256), 0, s, fd, comp, lab_g);
  else
    hipLaunchKernelGGL(k_cert_compare<double>, dim3(gn), dim3(256), 0, s, fd, comp, lab_g);
  return hipGetLastError();
}

}  // namespace exz
