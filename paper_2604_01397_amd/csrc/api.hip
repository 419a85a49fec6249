// Host side of the C ABI declared in include/exactz.h: contexts, workspace,
// the single-field correction driver and the diagnostics entry points.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/exactz.h"
#include "exz_internal.h"
#include "exz_host.h"

using namespace exz;

// ---------------------------------------------------------------------------
// helpers

namespace exz {

void Arena::release() {
  if (fixed) {
    base = end = nullptr;
    after = nullptr;
    cap = off = 0;
    fixed = false;
    return;
  }
  if (base && pool) {
    pool->give(base, cap);  // stays charged to the budget while pooled
  } else {
    if (base) (void)hipFree(base);
    if (budget) budget->used -= cap;
  }
  base = nullptr;
  cap = off = 0;
}

char *Pool::take(size_t need, size_t &got) {
  size_t best = blocks.size();
  for (size_t k = 0; k < blocks.size(); ++k) {
    const size_t b = blocks[k].bytes;
    if (b >= need && b <= need + need / 4 + ((size_t)1 << 20) &&
        (best == blocks.size() || b < blocks[best].bytes))
      best = k;
  }
  if (best == blocks.size()) return nullptr;
  char *p = blocks[best].p;
  got = blocks[best].bytes;
  bytes -= got;
  blocks[best] = blocks.back();
  blocks.pop_back();
  return p;
}

void Pool::give(char *p, size_t n) {
  blocks.push_back(Block{p, n});
  bytes += n;
  while (bytes > cap && !blocks.empty()) {  // past the cap: free the largest
    size_t big = 0;
    for (size_t k = 1; k < blocks.size(); ++k)
      if (blocks[k].bytes > blocks[big].bytes) big = k;
    (void)hipFree(blocks[big].p);
    bytes -= blocks[big].bytes;
    if (budget) budget->used -= blocks[big].bytes;
    blocks[big] = blocks.back();
    blocks.pop_back();
  }
}

void Pool::trim() {
  for (const Block &b : blocks) {
    (void)hipFree(b.p);
    if (budget) budget->used -= b.bytes;
  }
  blocks.clear();
  bytes = 0;
}

hipError_t Arena::reserve(size_t bytes) {
  off = 0;
  if (fixed) {
    if (after) {
      const uintptr_t a = ((uintptr_t)after->base + after->off + 255) & ~(uintptr_t)255;
      base = (char *)a;
      cap = base < end ? (size_t)(end - base) : 0;
    }
    return bytes <= cap ? hipSuccess : hipErrorOutOfMemory;
  }
  if (bytes <= cap) return hipSuccess;
  release();
  if (pool) {  // a pooled block is already charged to the budget
    size_t got = 0;
    if (char *p = pool->take(bytes, got)) {
      base = p;
      cap = got;
      return hipSuccess;
    }
  }
  const size_t want = exact ? bytes : bytes + bytes / 8 + 4096;
  if (pool && pool->bytes && budget && budget->limit && budget->used + bytes > budget->limit)
    pool->trim();  // pooled memory gives way to a job that needs it
  if (budget && budget->limit && budget->used + want > budget->limit) {
    // the slack is a convenience: fall back to the exact size before failing
    if (budget->used + bytes > budget->limit) return hipErrorOutOfMemory;
  }
  const size_t got = (budget && budget->limit && budget->used + want > budget->limit) ? bytes : want;
  hipError_t e = hipMalloc(&base, got);
  if (e != hipSuccess && pool && pool->bytes) {  // the device is full: free the pool, try again
    (void)hipGetLastError();
    pool->trim();
    e = hipMalloc(&base, got);
  }
  if (e != hipSuccess) {
    base = nullptr;
    (void)hipGetLastError();
    return e;
  }
  cap = got;
  if (budget) budget->used += got;
  return hipSuccess;
}

void *Arena::take(size_t bytes) {
  off = (off + 255) & ~(size_t)255;
  void *p = base + off;
  off += bytes;
  return p;
}

size_t Layout::add(size_t bytes) {
  total = (total + 255) & ~(size_t)255;
  const size_t at = total;
  total += bytes;
  return at;
}

}  // namespace exz

static exz_status fail(exz_ctx *ctx, exz_status st, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->last_error = buf;
  }
  return st;
}

#define HIP_OR_FAIL(call)                                                               \
  do {                                                                                  \
    hipError_t _e = (call);                                                             \
    if (_e != hipSuccess)                                                               \
      return fail(ctx, EXZ_E_HIP, "%s failed: %s", #call, hipGetErrorString(_e));        \
  } while (0)

namespace {

struct Busy {
  exz_ctx *c;
  bool ok;
  explicit Busy(exz_ctx *ctx) : c(ctx), ok(!ctx->busy) {
    if (ok) c->busy = true;
  }
  ~Busy() {
    if (ok) c->busy = false;
  }
};

}  // namespace

namespace exz {

// Box shape when none is set: 64 x 4 x 8 for volumes, 64 x 16 rows for
// planes, single rows for lines (taller boxes would leave threads idle).
void default_box(int ny, int nz, int &ty, int &tz) {
  if (nz > 1) {
    ty = 4;
    tz = 8;
  } else if (ny > 1) {
    ty = 16;
    tz = 1;
  } else {
    ty = 1;
    tz = 1;
  }
}

// Validates params and fills geometry, bounds and step of fd.
exz_status prepare_field(exz_ctx *ctx, const exz_params *p, FieldDev &fd) {
  std::memset(&fd, 0, sizeof fd);
  if (!p) return fail(ctx, EXZ_E_INVALID, "params is null");
  if (p->ndim < 1 || p->ndim > 3) return fail(ctx, EXZ_E_INVALID, "ndim must be 1..3");
  if (p->dtype != EXZ_F32 && p->dtype != EXZ_F64) return fail(ctx, EXZ_E_INVALID, "bad dtype");
  int64_t d[3] = {1, 1, 1};
  for (int k = 0; k < p->ndim; ++k) d[k] = p->dims[k];
  for (int k = p->ndim; k < 3; ++k)
    if (p->dims[k] != 1 && p->dims[k] != 0)
      return fail(ctx, EXZ_E_INVALID, "unused dims must be 1");
  for (int k = 0; k < 3; ++k)
    if (d[k] < 1) return fail(ctx, EXZ_E_INVALID, "dims must be >= 1");
  const int64_t n = d[0] * d[1] * d[2];
  if (d[0] >= (1ll << 31) || d[1] >= (1ll << 31) || d[2] >= (1ll << 31) || n >= (1ll << 31))
    return fail(ctx, EXZ_E_INVALID, "field has 2^31 or more vertices");
  if (!(std::isfinite(p->xi) && p->xi > 0)) return fail(ctx, EXZ_E_INVALID, "xi must be finite and > 0");
  if (p->n_steps < 1 || p->n_steps > 14) return fail(ctx, EXZ_E_INVALID, "n_steps must be 1..14");
  if (p->event_mode != EXZ_EVENT_REFORMULATED && p->event_mode != EXZ_EVENT_ORIGINAL)
    return fail(ctx, EXZ_E_INVALID, "bad event_mode");
  if (p->max_iters < 0) return fail(ctx, EXZ_E_INVALID, "max_iters must be >= 0");
  fd.nx = (int32_t)d[0];
  fd.ny = (int32_t)d[1];
  fd.nz = (int32_t)d[2];
  fd.n = (int32_t)n;
  fd.nchunk = (int32_t)((n + 63) / 64);
  fd.dtype = p->dtype;
  fd.N = p->n_steps;
  fd.mode = p->event_mode;
  fd.resume = p->resume ? 1 : 0;
  int ty = ctx ? ctx->tile_y : 0, tz = ctx ? ctx->tile_z : 0;
  if (ty == 0) default_box(fd.ny, fd.nz, ty, tz);
  fd.tile_y = ty;
  fd.tile_z = tz;
  fd.ty_shift = __builtin_ctz((unsigned)ty);  // compiled box sides are powers of two
  fd.tz_shift = __builtin_ctz((unsigned)tz);
  fd.tiles_x = (fd.nx + 63) / 64;
  fd.tiles_y = (fd.ny + ty - 1) / ty;
  fd.tiles_z = (fd.nz + fd.tile_z - 1) / fd.tile_z;
  const int64_t ntiles = (int64_t)fd.tiles_x * fd.tiles_y * fd.tiles_z;
  if (ntiles >= (1ll << 31)) return fail(ctx, EXZ_E_INVALID, "too many tiles");
  fd.ntiles = (int32_t)ntiles;
  fd.grid_blocks = ctx ? ctx->grid_blocks : -1;
  // original mode rewrites g's pointer labels by pointer jumping every
  // iteration, so its check pass always covers every box
  fd.frontier = (ctx ? ctx->frontier : true) && p->event_mode == EXZ_EVENT_REFORMULATED;
  const int nxy = fd.nx * fd.ny;
  for (int s = 0; s < NSLOT; ++s) fd.dlt[s] = DXS[s] + fd.nx * DYS[s] + nxy * DZS[s];
  fd.dlt[SELF] = 0;
  // xi_T: largest value of the field type not above xi; Delta = RN(xi_T / N)
  if (p->dtype == EXZ_F32) {
    float x = (float)p->xi;
    if ((double)x > p->xi) x = std::nextafter(x, -INFINITY);
    if (!(x > 0.0f)) return fail(ctx, EXZ_E_INVALID, "xi rounds to 0 in float32");
    const volatile float nn = (float)p->n_steps;
    const volatile float dl = x / nn;
    fd.xiT = x;
    fd.delta = dl;
  } else {
    const volatile double nn = (double)p->n_steps;
    const volatile double dl = p->xi / nn;
    fd.xiT = p->xi;
    fd.delta = dl;
  }
  return EXZ_OK;
}

// Per-vertex workspace (phase A).
void layout_a(const FieldDev &fd, bool own_cnt, int trace_cap, bool need_lab, Layout &L,
              size_t off[9]) {
  const size_t n = (size_t)fd.n;
  off[0] = L.add(sizeof(State));
  off[1] = L.add(3 * n);                                     // code, low
  off[2] = L.add(8 * (size_t)fd.nchunk);                     // cpbits
  off[3] = L.add(4 * ((size_t)fd.nchunk + 1));               // cpoff
  off[4] = L.add(mark_bytes(fd));                            // target marks + zero padding
  off[5] = L.add(n);                                         // fe
  off[6] = own_cnt ? L.add(n) : 0;                           // cnt
  off[7] = L.add(4 * scan_tmp_words((uint32_t)fd.nchunk));   // scan tmp
  // dirty box flags and their list, sized for the smallest box (64 x 1 x 1)
  // so the footprint does not depend on the box shape
  off[8] = L.add(box_flag_bytes(fd));
  (void)trace_cap;
  (void)need_lab;
}

// Per-critical-point workspace (phase B) for K critical points.
void layout_b(const FieldDev &fd, uint32_t K, Layout &L, size_t off[12]) {
  const size_t b = fd.dtype == 0 ? 4 : 8;
  const size_t kb = b;  // sort key bytes
  const uint32_t Kc = K ? K : 1;
  off[0] = L.add(4 * (size_t)Kc + 4 * (((size_t)Kc + 31) / 32) + ((size_t)Kc + 255) / 256);  // cp_rank, cp_below, oflag
  off[1] = L.add(4 * (size_t)Kc);  // cp_vtx
  off[2] = 0;
  off[3] = L.add(4 * (size_t)Kc);  // cp_idx
  off[4] = L.add(b * Kc);          // cpr
  off[5] = L.add(kb * Kc);         // keys
  off[6] = L.add(kb * Kc);         // keys tmp
  off[7] = L.add(4 * (size_t)Kc);  // vals
  off[8] = L.add(4 * (size_t)Kc);  // vals tmp
  const size_t hw = radix_hist_words(Kc);
  off[9] = L.add(4 * hw);          // histograms
  off[10] = L.add(4 * scan_tmp_words((uint32_t)(hw - 1)));
  off[11] = 0;
}

exz_status setup_phase_a(exz_ctx *ctx, FieldDev &fd, const void *f, const void *g_hat,
                         void *g_out, uint8_t *cnt_io, int64_t max_iters, Arena &A, hipStream_t s,
                         State *h_state, uint32_t *h_k) {
  fd.f = f;
  fd.g_hat = g_hat;
  fd.g = g_out;
  Layout LA;
  size_t oa[9];
  layout_a(fd, cnt_io == nullptr, 0, false, LA, oa);
  if (A.reserve(LA.total) != hipSuccess)
    return fail(ctx, EXZ_E_NOMEM, "%zu bytes of per-vertex workspace do not fit (%s)", LA.total,
                A.fixed ? "static buffer" : "device memory or context budget");
  char *base = (char *)A.take(LA.total);
  fd.st = (State *)(base + oa[0]);
  fd.low = (uint16_t *)(base + oa[1]);
  fd.code = (uint8_t *)(base + oa[1] + 2 * (size_t)fd.n);
  fd.cpbits = (unsigned long long *)(base + oa[2]);
  fd.cpoff = (uint32_t *)(base + oa[3]);
  fd.tmark = (uint8_t *)(base + oa[4]);
  fd.mchunk = fd.tmark + mark_pad_bytes(fd);
  fd.fe = (uint8_t *)(base + oa[5]);
  fd.bdirty = (uint8_t *)(base + oa[8]);
  fd.blist = box_list_of(fd, base + oa[8]);
  fd.cnt = cnt_io ? cnt_io : (uint8_t *)(base + oa[6]);
  fd.vec = quad_aligned(fd);
  uint32_t *scan_tmp = (uint32_t *)(base + oa[7]);

  HIP_OR_FAIL(launch_state_reset(fd, max_iters, s));
  HIP_OR_FAIL(launch_setup(fd, ctx->d_conn, s));
  HIP_OR_FAIL(launch_scan_u32(fd.cpoff, fd.cpoff, (uint32_t)fd.nchunk, scan_tmp,
                              scan_tmp_words((uint32_t)fd.nchunk), s));
  HIP_OR_FAIL(hipMemcpyAsync(h_state, fd.st, sizeof(State), hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(hipMemcpyAsync(h_k, fd.cpoff + fd.nchunk, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  return EXZ_OK;
}

exz_status setup_phase_b(exz_ctx *ctx, FieldDev &fd, uint32_t K, Arena &B, hipStream_t s) {
  fd.K = (int32_t)K;
  Layout LB;
  size_t ob[12];
  layout_b(fd, K, LB, ob);
  if (B.reserve(LB.total) != hipSuccess)
    return fail(ctx, EXZ_E_NOMEM, "%zu bytes of critical-point workspace do not fit (%s)",
                LB.total, B.fixed ? "static buffer" : "device memory or context budget");
  char *bb = (char *)B.take(LB.total);
  fd.cp_rank = (uint32_t *)(bb + ob[0]);
  fd.cp_below = fd.cp_rank + (K ? K : 1);
  fd.oflag = (uint8_t *)(fd.cp_below + ((K ? K : 1) + 31) / 32);
  fd.cp_vtx = (uint32_t *)(bb + ob[1]);
  fd.cp_idx = (uint32_t *)(bb + ob[3]);
  fd.cpr = bb + ob[4];
  void *keys = bb + ob[5];
  void *keys_tmp = bb + ob[6];
  uint32_t *vals = (uint32_t *)(bb + ob[7]);
  uint32_t *vals_tmp = (uint32_t *)(bb + ob[8]);
  uint32_t *hist = (uint32_t *)(bb + ob[9]);
  uint32_t *stmp = (uint32_t *)(bb + ob[10]);
  const size_t hw = radix_hist_words(K ? K : 1);
  if (K > 0) {
    HIP_OR_FAIL(launch_cp_compact(fd, ctx->d_comp, keys, vals, s));
    HIP_OR_FAIL(launch_radix_sort(fd.dtype == 0 ? 4 : 8, keys, vals, keys_tmp, vals_tmp, K, hist,
                                  stmp, scan_tmp_words((uint32_t)(hw - 1)), s));
    HIP_OR_FAIL(launch_cp_init(fd, vals, s));
  }
  return EXZ_OK;
}

// Validation, reference topology, CP order (phases A and B).  On success fd
// is ready for iterations and ctx->h_state holds the setup flags.
exz_status setup_field(exz_ctx *ctx, FieldDev &fd, const void *f, const void *g_hat, void *g_out,
                       uint8_t *cnt_io, int64_t max_iters, Arena &A, Arena &B, hipStream_t s) {
  exz_status st = setup_phase_a(ctx, fd, f, g_hat, g_out, cnt_io, max_iters, A, s, ctx->h_state,
                                ctx->h_k);
  if (st != EXZ_OK) return st;
  HIP_OR_FAIL(hipStreamSynchronize(s));
  if (ctx->h_state->err & ERR_NONFINITE) return fail(ctx, EXZ_E_NONFINITE, "NaN or Inf in f or g_hat");
  if (ctx->h_state->err & ERR_BOUND) return fail(ctx, EXZ_E_BOUND, "g_hat outside [f - xi, f + xi]");
  return setup_phase_b(ctx, fd, *ctx->h_k, B, s);
}

// Path-tracing workspace: original event mode (g labels, f termini, saddle
// order, f's selections) and/or the certificate (f termini, g labels).
void layout_c(const FieldDev &fd, bool original, bool certify, Layout &L, size_t off[6]) {
  const size_t n = (size_t)fd.n, K = (size_t)(fd.K ? fd.K : 1);
  off[0] = (original || certify) ? L.add(8 * n) : 0;  // lab_f
  // lab (g) / certificate labels, then the convergence bitmask of 2n labels
  off[1] = (original || certify) ? L.add(8 * n + 4 * jump_conv_words(2 * (uint64_t)n)) : 0;
  off[2] = original ? L.add(4 * K) : 0;               // sad_rank
  off[3] = original ? L.add(8 * K) : 0;               // sel_f
  off[4] = original ? L.add(4 * (K + 1)) : 0;         // saddle flags / prefix
  off[5] = original ? L.add(4 * scan_tmp_words((uint32_t)K)) : 0;
}

exz_status setup_paths(exz_ctx *ctx, FieldDev &fd, bool original, bool certify, Arena &C,
                       uint32_t **lab_g, hipStream_t s) {
  if (!original && !certify) return EXZ_OK;
  Layout LC;
  size_t oc[6];
  layout_c(fd, original, certify, LC, oc);
  if (C.reserve(LC.total) != hipSuccess)
    return fail(ctx, EXZ_E_NOMEM, "%zu bytes of path workspace do not fit (%s)", LC.total,
                C.fixed ? "static buffer" : "device memory or context budget");
  char *cb = (char *)C.take(LC.total);
  fd.lab_f = (uint32_t *)(cb + oc[0]);
  fd.lab = (uint32_t *)(cb + oc[1]);
  *lab_g = fd.lab;
  if (original) {
    fd.sad_rank = (uint32_t *)(cb + oc[2]);
    fd.sel_f = (uint32_t *)(cb + oc[3]);
    HIP_OR_FAIL(launch_original_setup(fd, ctx->d_comp, (uint32_t *)(cb + oc[4]),
                                      (uint32_t *)(cb + oc[5]),
                                      scan_tmp_words((uint32_t)(fd.K ? fd.K : 1)), s));
  }
  return EXZ_OK;
}

}  // namespace exz

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char *exz_status_string(int status) {
  switch (status) {
    case EXZ_OK: return "ok";
    case EXZ_W_STUCK: return "stuck at a fixpoint with residual violations";
    case EXZ_W_MAX_ITERS: return "stopped at max_iters";
    case EXZ_E_INVALID: return "invalid argument";
    case EXZ_E_NONFINITE: return "non-finite input";
    case EXZ_E_BOUND: return "decompressed field outside the error band";
    case EXZ_E_NOMEM: return "out of memory";
    case EXZ_E_HIP: return "HIP runtime error";
    case EXZ_E_BUSY: return "context busy";
    default: return "unknown status";
  }
}

const char *exz_last_error(const exz_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

exz_status exz_ctx_create(int device, size_t hbm_budget_bytes, exz_ctx **out) {
  if (!out) return EXZ_E_INVALID;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return EXZ_E_INVALID;
  if (hipSetDevice(device) != hipSuccess) return EXZ_E_HIP;
  exz_ctx *ctx = new exz_ctx();
  ctx->device = device;
  ctx->budget.limit = hbm_budget_bytes;
  for (Arena *a : {&ctx->A, &ctx->B, &ctx->C, &ctx->BA, &ctx->BB, &ctx->BC, &ctx->H})
    a->budget = &ctx->budget;
  ctx->job_pool.budget = &ctx->budget;
  // events of the single-field driver, created here so that a correction
  // call creates nothing
  if (hipEventCreate(&ctx->ev_start) != hipSuccess || hipEventCreate(&ctx->ev_setup) != hipSuccess ||
      hipEventCreate(&ctx->ev_end) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->poll_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->poll_ev[1], hipEventDisableTiming) != hipSuccess ||
      scratch_lookup(device, &ctx->scratch, &ctx->scratch_bytes) != hipSuccess) {
    exz_ctx_destroy(ctx);
    return EXZ_E_HIP;
  }
  std::vector<uint8_t> comp(1u << NSLOT);
  build_component_table(comp.data());
  std::vector<uint32_t> conn(512);
  build_connected_bits(comp.data(), conn.data());
  if (hipMalloc(&ctx->d_comp, comp.size()) != hipSuccess ||
      hipMemcpy(ctx->d_comp, comp.data(), comp.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMalloc(&ctx->d_conn, 512 * sizeof(uint32_t)) != hipSuccess ||
      hipMemcpy(ctx->d_conn, conn.data(), 512 * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipHostMalloc((void **)&ctx->h_state, sizeof(State) * 2, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&ctx->h_k, 64, hipHostMallocDefault) != hipSuccess) {
    exz_ctx_destroy(ctx);
    return EXZ_E_NOMEM;
  }
  *out = ctx;
  return EXZ_OK;
}

exz_status exz_ctx_destroy(exz_ctx *ctx) {
  if (!ctx) return EXZ_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  free_graveyard(ctx);  // (their arenas go to the pool, freed next)
  ctx->job_pool.trim();
  ctx->A.release();
  ctx->B.release();
  ctx->C.release();
  ctx->BA.release();
  ctx->BB.release();
  ctx->BC.release();
  ctx->H.release();
  if (ctx->step_host) (void)hipHostFree(ctx->step_host);
  if (ctx->step_dev) (void)hipFree(ctx->step_dev);
  if (ctx->step_copied) (void)hipEventDestroy(ctx->step_copied);
  if (ctx->step_done) (void)hipEventDestroy(ctx->step_done);
  if (ctx->order_in) (void)hipEventDestroy(ctx->order_in);
  if (ctx->order_out) (void)hipEventDestroy(ctx->order_out);
  if (ctx->work) (void)hipStreamDestroy(ctx->work);
  for (int j = 0; j < exz_ctx::NSIDE; ++j)
    if (ctx->side[j]) (void)hipStreamDestroy(ctx->side[j]);
  for (int j = 0; j <= exz_ctx::NSIDE; ++j)
    if (ctx->side_ev[j]) (void)hipEventDestroy(ctx->side_ev[j]);
  for (auto &e : ctx->events) (void)hipEventDestroy(e);
  if (ctx->ev_start) (void)hipEventDestroy(ctx->ev_start);
  if (ctx->ev_setup) (void)hipEventDestroy(ctx->ev_setup);
  if (ctx->ev_end) (void)hipEventDestroy(ctx->ev_end);
  if (ctx->poll_ev[0]) (void)hipEventDestroy(ctx->poll_ev[0]);
  if (ctx->poll_ev[1]) (void)hipEventDestroy(ctx->poll_ev[1]);
  if (ctx->d_comp) (void)hipFree(ctx->d_comp);
  if (ctx->d_conn) (void)hipFree(ctx->d_conn);
  if (ctx->h_state) (void)hipHostFree(ctx->h_state);
  if (ctx->h_k) (void)hipHostFree(ctx->h_k);
  delete ctx;
  return EXZ_OK;
}

exz_status exz_ctx_set_option(exz_ctx *ctx, const char *key, int64_t value) {
  if (!ctx || !key) return EXZ_E_INVALID;
  const std::string k(key);
  if (k == "profile") {
    ctx->profile = value != 0;
  } else if (k == "poll") {
    if (value < 0 || value > 256) return fail(ctx, EXZ_E_INVALID, "poll must be 0..256");
    ctx->poll = (int)value;
  } else if (k == "graph") {
    ctx->graph = value != 0;
  } else if (k == "tile_z") {
    const int ty = ctx->tile_y ? ctx->tile_y : 4;
    if (!box_supported(ty, (int)value))
      return fail(ctx, EXZ_E_INVALID, "no compiled box %d x %d", ty, (int)value);
    ctx->tile_y = ty;
    ctx->tile_z = (int)value;
  } else if (k == "tile_y") {
    const int tz = ctx->tile_z ? ctx->tile_z : 1;
    if (!box_supported((int)value, tz))
      return fail(ctx, EXZ_E_INVALID, "no compiled box %d x %d", (int)value, tz);
    ctx->tile_y = (int)value;
    ctx->tile_z = tz;
  } else if (k == "frontier") {  // 1: re-check only changed boxes (reformulated mode)
    ctx->frontier = value != 0;
  } else if (k == "job_pool") {  // bytes of freed job arenas kept for later jobs
    if (value < 0) return fail(ctx, EXZ_E_INVALID, "job_pool must be >= 0");
    ctx->job_pool.cap = (size_t)value;
    if (ctx->job_pool.bytes > ctx->job_pool.cap) ctx->job_pool.trim();
  } else if (k == "trim") {  // free the pooled job arenas now (waits for the device)
    ctx->job_pool.trim();
  } else if (k == "grid") {  // stencil work-groups: -1 persistent (default), 0 one per box
    if (value < -1 || value > (1 << 24)) return fail(ctx, EXZ_E_INVALID, "grid must be -1..2^24");
    ctx->grid_blocks = (int)value;
  } else if (k == "tile") {  // tile_y * 100 + tile_z, set together; 0 = by dimensionality
    const int ty = (int)(value / 100), tz = (int)(value % 100);
    if (value != 0 && !box_supported(ty, tz))
      return fail(ctx, EXZ_E_INVALID, "no compiled box %d x %d", ty, tz);
    ctx->tile_y = ty;
    ctx->tile_z = tz;
  } else if (k == "btile3" || k == "btile2") {  // batched / job boxes, 0 = default
    const int ty = (int)(value / 100), tz = (int)(value % 100);
    if (value != 0 && (!box_supported(ty, tz) || (k == "btile2" && tz != 1)))
      return fail(ctx, EXZ_E_INVALID, "no compiled box %d x %d for %s", ty, tz, key);
    (k == "btile3" ? ctx->btile3 : ctx->btile2) = (int)value;
  } else if (k == "bgrid_box" || k == "bgrid_apply") {  // batched grid caps, 0 = default
    if (value < 0 || value > (1 << 20)) return fail(ctx, EXZ_E_INVALID, "%s must be 0..2^20", key);
    (k == "bgrid_box" ? ctx->bgrid_box : ctx->bgrid_apply) = (int)value;
  } else if (k == "bitem") {  // batched apply item: quads per thread, 0 = default (16)
    if (value < 0 || value > 256) return fail(ctx, EXZ_E_INVALID, "bitem must be 0..256");
    ctx->bitem = (int)value;
  } else {
    return fail(ctx, EXZ_E_INVALID, "unknown option '%s'", key);
  }
  return EXZ_OK;
}

size_t exz_workspace_bytes_k(const exz_params *p, int64_t num_critical) {
  FieldDev fd;
  if (prepare_field(nullptr, p, fd) != EXZ_OK) return 0;
  if (num_critical < 0 || num_critical > fd.n) return 0;
  Layout LA, LB;
  size_t oa[9], ob[12];
  layout_a(fd, true, 0, p->event_mode == EXZ_EVENT_ORIGINAL || p->certify, LA, oa);
  layout_b(fd, (uint32_t)num_critical, LB, ob);
  Layout LC;
  size_t oc[6];
  fd.K = (int32_t)num_critical;
  layout_c(fd, p->event_mode == EXZ_EVENT_ORIGINAL, p->certify != 0, LC, oc);
  return LA.total + LB.total + LC.total;
}

size_t exz_workspace_bytes(const exz_params *p) {
  FieldDev fd;
  if (!p || prepare_field(nullptr, p, fd) != EXZ_OK) return 0;
  return exz_workspace_bytes_k(p, fd.n);
}

static void fill_result(exz_result *r, const State &st, int status) {
  r->iterations = st.iterations;
  r->edited_vertices = st.edited_total;
  r->targets_total = st.targets_total;
  r->edit_ops = st.edit_ops;
  r->lossless_vertices = st.lossless_total;
  r->floor_vertices = st.floor_total;
  r->residual_violations = st.residual;
  r->status = status;
}

exz_status exz_correct(exz_ctx *ctx, const void *f, const void *g_hat, void *g_out,
                       uint8_t *cnt_io, const exz_params *params, exz_result *result,
                       void *stream) {
  exz_result dummy;
  exz_result *res = result ? result : &dummy;
  std::memset(res, 0, sizeof *res);
  res->certified = -1;
  if (!ctx) return (exz_status)(res->status = EXZ_E_INVALID);
  Busy busy(ctx);
  if (!busy.ok) return (exz_status)(res->status = fail(ctx, EXZ_E_BUSY, "context busy"));
  ctx->last_error.clear();
  exz_status st = exz_correct_impl(ctx, f, g_hat, g_out, cnt_io, params, res, (hipStream_t)stream,
                                   ctx->A, ctx->B, ctx->C, ctx->profile);
  res->status = st;
  return st;
}

exz_status exz_correct_host(exz_ctx *ctx, const void *f, const void *g_hat, void *g_out,
                            uint8_t *cnt_io, const exz_params *params, exz_result *result) {
  exz_result dummy;
  exz_result *res = result ? result : &dummy;
  std::memset(res, 0, sizeof *res);
  res->certified = -1;
  if (!ctx) return (exz_status)(res->status = EXZ_E_INVALID);
  Busy busy(ctx);
  if (!busy.ok) return (exz_status)(res->status = fail(ctx, EXZ_E_BUSY, "context busy"));
  ctx->last_error.clear();
  if (!f || !g_hat || !g_out)
    return (exz_status)(res->status = fail(ctx, EXZ_E_INVALID, "null field pointer"));
  FieldDev fd;
  exz_status st = prepare_field(ctx, params, fd);
  if (st != EXZ_OK) return (exz_status)(res->status = st);
  if (params->resume && !cnt_io)
    return (exz_status)(res->status = fail(ctx, EXZ_E_INVALID, "resume needs cnt_io"));
  if (hipSetDevice(ctx->device) != hipSuccess)
    return (exz_status)(res->status = fail(ctx, EXZ_E_HIP, "hipSetDevice failed"));
  // device copies: f, g (g_hat in, g' out, corrected in place), counts
  const size_t n = (size_t)fd.n, vb = n * (fd.dtype == EXZ_F32 ? 4 : 8);
  Layout L;
  const size_t of = L.add(vb), og = L.add(vb), oc = L.add(n);
  if (ctx->H.reserve(L.total) != hipSuccess)
    return (exz_status)(res->status = fail(ctx, EXZ_E_NOMEM, "%zu bytes for the device copies "
                                           "do not fit", L.total));
  char *base = (char *)ctx->H.take(L.total);
  void *df = base + of, *dg = base + og;
  uint8_t *dc = (uint8_t *)(base + oc);
  hipStream_t s = nullptr;
  hipError_t e = hipMemcpy(df, f, vb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dg, g_hat, vb, hipMemcpyHostToDevice);
  if (e == hipSuccess && params->resume) e = hipMemcpy(dc, cnt_io, n, hipMemcpyHostToDevice);
  if (e != hipSuccess)
    return (exz_status)(res->status = fail(ctx, EXZ_E_HIP, "copy in: %s", hipGetErrorString(e)));
  st = exz_correct_impl(ctx, df, dg, dg, dc, params, res, s, ctx->A, ctx->B, ctx->C, ctx->profile);
  res->status = st;
  if (st < 0) return st;
  e = hipMemcpy(g_out, dg, vb, hipMemcpyDeviceToHost);
  if (e == hipSuccess && cnt_io) e = hipMemcpy(cnt_io, dc, n, hipMemcpyDeviceToHost);
  if (e != hipSuccess)
    return (exz_status)(res->status = fail(ctx, EXZ_E_HIP, "copy out: %s", hipGetErrorString(e)));
  return st;
}

size_t exz_ctx_bytes_in_use(const exz_ctx *ctx) { return ctx ? ctx->budget.used : 0; }

exz_status exz_debug_bounds(exz_ctx *ctx, int32_t dtype, const void *f, int64_t n, double xi,
                            void *L_out, void *U_out, void *stream) {
  if (!ctx || !f || !L_out || !U_out || n < 0) return EXZ_E_INVALID;
  exz_params p;
  std::memset(&p, 0, sizeof p);
  p.ndim = 1;
  p.dtype = dtype;
  p.dims[0] = n > 0 ? n : 1;
  p.dims[1] = p.dims[2] = 1;
  p.xi = xi;
  p.n_steps = 5;
  FieldDev fd;
  exz_status st = prepare_field(ctx, &p, fd);
  if (st != EXZ_OK) return st;
  HIP_OR_FAIL(hipSetDevice(ctx->device));
  HIP_OR_FAIL(launch_debug_bounds(dtype, f, n, fd.xiT, L_out, U_out, (hipStream_t)stream));
  HIP_OR_FAIL(hipStreamSynchronize((hipStream_t)stream));
  return EXZ_OK;
}

exz_status exz_debug_targets(exz_ctx *ctx, const void *f, const void *g, const exz_params *params,
                             uint8_t *mark_out, int64_t *count, void *stream) {
  if (!ctx || !f || !g || !mark_out || !count) return EXZ_E_INVALID;
  Busy busy(ctx);
  if (!busy.ok) return fail(ctx, EXZ_E_BUSY, "context busy");
  hipStream_t s = (hipStream_t)stream;
  HIP_OR_FAIL(hipSetDevice(ctx->device));
  FieldDev fd;
  exz_status st = prepare_field(ctx, params, fd);
  if (st != EXZ_OK) return st;
  if (params->event_mode != EXZ_EVENT_REFORMULATED)
    return fail(ctx, EXZ_E_INVALID, "diagnostic check supports the reformulated mode only");
  // g plays g_hat and g_out at once (no copy); the band check still applies.
  st = setup_field(ctx, fd, f, g, const_cast<void *>(g), nullptr, 0, ctx->A, ctx->B, s);
  if (st != EXZ_OK) return st;
  HIP_OR_FAIL(launch_debug_check(fd, ctx->d_conn, s));
  HIP_OR_FAIL(launch_targets_to_bytes(fd, mark_out, s));
  HIP_OR_FAIL(hipMemcpyAsync(ctx->h_state, fd.st, sizeof(State), hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(hipStreamSynchronize(s));
  *count = ctx->h_state->ntargets;
  return EXZ_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// the single-field driver

namespace exz {

exz_status exz_correct_impl(exz_ctx *ctx, const void *f, const void *g_hat, void *g_out,
                            uint8_t *cnt_io, const exz_params *params, exz_result *res,
                            hipStream_t s, Arena &A, Arena &B, Arena &C, bool profile) {
  if (!f || !g_hat || !g_out) return fail(ctx, EXZ_E_INVALID, "null field pointer");
  FieldDev fd;
  exz_status st = prepare_field(ctx, params, fd);
  if (st != EXZ_OK) return st;
  if (params->resume && !cnt_io) return fail(ctx, EXZ_E_INVALID, "resume needs cnt_io");
  HIP_OR_FAIL(hipSetDevice(ctx->device));
  HIP_OR_FAIL(hipEventRecord(ctx->ev_start, s));
  st = setup_field(ctx, fd, f, g_hat, g_out, cnt_io, params->max_iters, A, B, s);
  if (st != EXZ_OK) return st;
  res->num_critical = fd.K;
  uint32_t *lab_g = nullptr;
  st = setup_paths(ctx, fd, params->event_mode == EXZ_EVENT_ORIGINAL, params->certify != 0,
                   C, &lab_g, s);
  if (st != EXZ_OK) return st;
  HIP_OR_FAIL(hipEventRecord(ctx->ev_setup, s));

  // Iterations are issued in chunks; each chunk ends with an asynchronous
  // copy of the device state into one of two pinned slots.  The host keeps
  // one chunk in flight while it reads the previous chunk's state, so the
  // GPU never waits for the host; after convergence the kernels return at
  // once, so the chunk issued past the end costs only its launches.
  // every changing iteration moves a value down and a vertex moves at most
  // N + 1 times; at most two more passes (the frontier pass that finds the
  // fixpoint and the dense one that confirms it) change nothing
  const int64_t cap = (int64_t)(fd.N + 1) * fd.n + 4;
  int chunk = ctx->poll > 0 ? ctx->poll : 4;
  int64_t issued = 0;
  size_t ev_used = 0;
  auto issue_chunk = [&](int slot) -> exz_status {
    for (int k = 0; k < chunk; ++k) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (profile) {
        while (ctx->events.size() < ev_used + 2) {
          hipEvent_t e;
          HIP_OR_FAIL(hipEventCreate(&e));
          ctx->events.push_back(e);
        }
        e0 = ctx->events[ev_used];
        e1 = ctx->events[ev_used + 1];
        ev_used += 2;
      }
      HIP_OR_FAIL(launch_iteration(fd, ctx->d_conn, ctx->d_comp, s, e0, e1));
    }
    issued += chunk;
    HIP_OR_FAIL(hipMemcpyAsync(ctx->h_state + slot, fd.st, sizeof(State), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipEventRecord(ctx->poll_ev[slot], s));
    return EXZ_OK;
  };
  // Adaptive chunks.  The host learns a pass's state a chunk late, so each
  // chunk should end where the field can end at the earliest.  Once most
  // values have settled, the number a pass changes falls by a factor of
  // about 2.5 or more per pass, so a field whose last known pass changed c
  // values needs at least log_2.5(c) more passes, then the frontier pass
  // that finds the fixpoint and the dense one that confirms it: chunks reach
  // that far (4 to 16 passes; 8 before any state is known).
  int slot = 0;
  const State *known = nullptr;
  st = issue_chunk(slot);
  if (st != EXZ_OK) return st;
  for (;;) {
    if (ctx->poll == 0) {
      if (!known) {
        chunk = 8;
      } else {
        const double c = known->changed > 1 ? (double)known->changed : 1.0;
        const int64_t end = known->passes + (int64_t)std::ceil(std::log(c) / std::log(2.5)) + 2;
        chunk = (int)std::min<int64_t>(16, std::max<int64_t>(4, end - issued));
      }
    }
    st = issue_chunk(1 - slot);
    if (st != EXZ_OK) return st;
    HIP_OR_FAIL(hipEventSynchronize(ctx->poll_ev[slot]));
    if (ctx->h_state[slot].done != RUNNING) break;
    if (ctx->h_state[slot].passes > cap) return fail(ctx, EXZ_E_HIP, "loop did not terminate");
    known = &ctx->h_state[slot];
    slot = 1 - slot;
  }
  // the chunk still in flight ran past the fixpoint; its copy holds the final state
  HIP_OR_FAIL(hipEventSynchronize(ctx->poll_ev[1 - slot]));
  ctx->h_state[0] = ctx->h_state[1 - slot];
  if (params->certify) {
    HIP_OR_FAIL(launch_certify(fd, ctx->d_comp, lab_g, s));
    HIP_OR_FAIL(hipMemcpyAsync(ctx->h_state, fd.st, sizeof(State), hipMemcpyDeviceToHost, s));
  }
  HIP_OR_FAIL(hipEventRecord(ctx->ev_end, s));
  HIP_OR_FAIL(hipEventSynchronize(ctx->ev_end));
  const State hs = *ctx->h_state;
  if (params->certify) res->certified = hs.cert_bad == 0 ? 1 : 0;
  float ms = 0;
  HIP_OR_FAIL(hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_setup));
  res->setup_ms = ms;
  HIP_OR_FAIL(hipEventElapsedTime(&ms, ctx->ev_setup, ctx->ev_end));
  res->loop_ms = ms;
  int status = EXZ_OK;
  if (hs.done == STUCK) status = EXZ_W_STUCK;
  if (hs.done == MAXITERS) status = EXZ_W_MAX_ITERS;
  fill_result(res, hs, status);
  if (profile) {
    // every check launch issued, those past the fixpoint included (they
    // return at once), so the average matches a kernel trace of the call
    const int64_t launched = (int64_t)(ev_used / 2);
    double tot = 0;
    for (int64_t k = 0; k < launched; ++k) {
      HIP_OR_FAIL(hipEventElapsedTime(&ms, ctx->events[2 * k], ctx->events[2 * k + 1]));
      tot += ms;
    }
    res->check_launches = launched;
    res->check_ms = tot;
    res->check_vertices = (int64_t)hs.checked;
  }
  return (exz_status)status;
}

}  // namespace exz
