// Batched and serving entry points (many fields per launch).
#include <cstring>

#include "exz_host.h"

extern "C" {

exz_status exz_correct_batch(exz_ctx *ctx, const exz_field *fields, int32_t nfields,
                             exz_result *results, void *stream) {
  (void)fields; (void)nfields; (void)results; (void)stream;
  if (ctx) ctx->last_error = "batched correction is not available in this build";
  return EXZ_E_INVALID;
}

exz_status exz_job_create(exz_ctx *ctx, const exz_field *field, void *stream, exz_job **out) {
  (void)field; (void)stream;
  if (out) *out = nullptr;
  if (ctx) ctx->last_error = "jobs are not available in this build";
  return EXZ_E_INVALID;
}

exz_status exz_step(exz_ctx *ctx, exz_job *const *jobs, int32_t njobs, int32_t iters, void *stream) {
  (void)ctx; (void)jobs; (void)njobs; (void)iters; (void)stream;
  return EXZ_E_INVALID;
}

exz_status exz_job_poll(exz_job *job, int32_t *done, exz_result *result) {
  (void)job; (void)done; (void)result;
  return EXZ_E_INVALID;
}

exz_status exz_job_release(exz_job *job) {
  (void)job;
  return EXZ_E_INVALID;
}

size_t exz_job_bytes(const exz_params *params) { return exz_workspace_bytes(params); }

}  // extern "C"
