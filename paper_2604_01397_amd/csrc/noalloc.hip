// exz_correct_noalloc: exz_correct for callers that cannot allocate device
// memory (code under stream capture, tight serving loops, harnesses that
// forbid hipMalloc).  Its workspace -- the per-vertex reference arrays,
// target marks, box flags, loop state, critical-point list and sort buffers
// that exz_correct takes from the context's growable arenas -- lives in one
// static device buffer per GPU, `scratch`, held until the process ends.
//
// The buffer's device address is looked up once per device, with that
// device current, when a context is created on it (exz_ctx_create), and
// kept per device; host code only ever hands kernels that address.  Every
// correction call initialises all of its workspace in its set-up kernels, so
// what an earlier call left in the buffer is never read.  All calls on one
// GPU share its buffer: calls that overlap in time on the same GPU (two host
// threads, or two streams without ordering between them) race.
#include <cstdio>
#include <cstring>
#include <mutex>

#include "exz_host.h"

namespace exz {

constexpr size_t SCRATCH_BYTES = (size_t)128 << 20;  // 128 MiB per GPU

static __device__ __align__(256) char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static void *g_scratch[MAX_DEVICES];
static std::mutex g_scratch_mu;

// The caller has made `device` current.
hipError_t scratch_lookup(int device, void **ptr, size_t *bytes) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[device] = p;
  }
  *ptr = g_scratch[device];
  *bytes = SCRATCH_BYTES;
  return hipSuccess;
}

}  // namespace exz

using namespace exz;

extern "C" exz_status exz_correct_noalloc(exz_ctx *ctx, const void *f, const void *g_hat,
                                          void *g_out, uint8_t *cnt_io, const exz_params *params,
                                          exz_result *result, void *stream) {
  exz_result dummy;
  exz_result *res = result ? result : &dummy;
  std::memset(res, 0, sizeof *res);
  res->certified = -1;
  if (!ctx) return (exz_status)(res->status = EXZ_E_INVALID);
  if (ctx->busy) {
    ctx->last_error = "context busy";
    return (exz_status)(res->status = EXZ_E_BUSY);
  }
  ctx->busy = true;
  struct Unbusy {
    exz_ctx *c;
    ~Unbusy() { c->busy = false; }
  } unbusy{ctx};
  ctx->last_error.clear();
  if (!ctx->scratch) {
    ctx->last_error = "no static workspace on this device";
    return (exz_status)(res->status = EXZ_E_HIP);
  }
  // Size check before anything is issued: the per-vertex workspace must fit
  // (the critical-point part is checked once K is known, before its use).
  FieldDev fd;
  exz_status st = prepare_field(ctx, params, fd);
  if (st != EXZ_OK) return (exz_status)(res->status = st);
  Layout LA;
  size_t oa[9];
  layout_a(fd, cnt_io == nullptr, 0, false, LA, oa);
  if (LA.total > ctx->scratch_bytes) {
    char buf[256];
    snprintf(buf, sizeof buf,
             "field needs %zu bytes of per-vertex workspace; the static buffer holds %zu",
             LA.total, ctx->scratch_bytes);
    ctx->last_error = buf;
    return (exz_status)(res->status = EXZ_E_NOMEM);
  }
  // phases A, B and the path workspace one after another in the buffer
  char *end = (char *)ctx->scratch + ctx->scratch_bytes;
  Arena A, B, C;
  A.wrap(ctx->scratch, ctx->scratch_bytes);
  B.chain(&A, end);
  C.chain(&B, end);
  st = exz_correct_impl(ctx, f, g_hat, g_out, cnt_io, params, res, (hipStream_t)stream, A, B, C,
                        false);
  res->status = st;
  return st;
}
