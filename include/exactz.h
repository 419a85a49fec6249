/* exactz.h -- C ABI of the MI355X (gfx950) EXaCTz correction library.
 *
 * The library corrects a decompressed scalar field g_hat against its
 * original f so that the extremum graph and the contour tree of the result
 * equal those of f, while every value stays within the absolute error bound
 * xi (EXaCTz, arXiv 2604.01397).  It implements Algorithm 1 of the paper:
 *   g <- g_hat; repeat { S <- CheckConstraints(g, f); stop if S is empty;
 *                        g <- ApplyBoundedEdits(g, S, xi) }
 * with the checks of Sec. 4.2 (steepest ascent / descent neighbours, saddle
 * link order) and the event constraints either in the reformulated form of
 * Sec. 4.3 (the order of all critical points of f) or in the original form
 * of Sec. 4.2 (saddle order and per-saddle extremum selection traced along
 * integral paths).  Edits follow Sec. 3.3: each round a flagged vertex drops
 * by Delta = xi_T / N; the (N+1)-th edit stores the lower bound itself.
 *
 * Conventions shared by every entry point:
 *  - Fields are dense arrays of float32 or float64 with x the fastest index:
 *    vertex (x, y, z) is element x + nx*(y + ny*z).  dims[] holds
 *    (nx, ny, nz); unused trailing dims are 1.  1D, 2D and 3D fields live on
 *    the Freudenthal triangulation of the grid (14 neighbours in 3D, 6 in
 *    2D, 2 in 1D).  Ties are broken by the linear index (Sec. 3.3, footnote).
 *  - All field pointers are DEVICE pointers owned by the caller; the library
 *    never frees caller memory.  f and g_hat are read-only; g_out may alias
 *    g_hat (in-place correction).
 *  - xi_T, the largest value of the field type not above xi, is the bound
 *    actually enforced; L_i / U_i are the exact round-up of f_i - xi_T and
 *    round-down of f_i + xi_T.  g_hat must satisfy L_i <= g_hat_i <= U_i.
 *  - Work is issued on the given HIP stream (hipStream_t passed as void*;
 *    NULL = the default stream).  Calls return after that stream has
 *    finished the correction (the loop polls a device flag), so results are
 *    valid on return.
 *  - One context serves one host thread at a time; a reentrant call on a
 *    busy context returns EXZ_E_BUSY.
 *  - The result depends only on (f, g_hat, params): not on tile shapes,
 *    batch composition, other jobs or the number of iterations per poll.
 */
#ifndef EXACTZ_H
#define EXACTZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { EXZ_F32 = 0, EXZ_F64 = 1 } exz_dtype;

typedef enum {
  EXZ_EVENT_REFORMULATED = 0, /* order of all critical points (Sec. 4.3) */
  EXZ_EVENT_ORIGINAL = 1      /* saddle order + path-traced selection (Sec. 4.2) */
} exz_event_mode;

typedef enum {
  EXZ_OK = 0,
  EXZ_W_STUCK = 1,      /* fixpoint with violations left: every target sits at
                           its lower bound (float rounding made two distinct
                           f values share one bound); residual_violations > 0 */
  EXZ_W_MAX_ITERS = 2,  /* stopped after params.max_iters changing rounds */
  EXZ_E_INVALID = -1,   /* null pointer, ndim not in 1..3, a dim < 1,
                           n >= 2^31, xi not finite or xi_T <= 0, n_steps
                           outside 1..14, unknown mode or dtype */
  EXZ_E_NONFINITE = -2, /* NaN or Inf in f or g_hat */
  EXZ_E_BOUND = -3,     /* some g_hat_i outside [L_i, U_i] */
  EXZ_E_NOMEM = -4,     /* device or pinned allocation failed / over budget */
  EXZ_E_HIP = -5,       /* a HIP runtime call failed (see exz_last_error) */
  EXZ_E_BUSY = -6       /* context already in use */
} exz_status;

/* Problem description (Algorithm 1 inputs besides the two fields). */
typedef struct {
  int32_t ndim;        /* 1, 2 or 3 */
  int32_t dtype;       /* exz_dtype */
  int64_t dims[3];     /* nx, ny, nz; unused = 1 */
  double xi;           /* absolute error bound, > 0 */
  int32_t n_steps;     /* N of Sec. 3.3; 5 in the paper; 1..14 */
  int32_t event_mode;  /* exz_event_mode */
  int64_t max_iters;   /* 0 = run to the fixpoint */
  int32_t certify;     /* 1 = after the loop, verify on the device that every
                          vertex's steepest-descent and steepest-ascent path
                          ends where it ends in f and that all critical types
                          agree (the extremum-graph identity of Sec. 4.1) */
  int32_t resume;      /* 1 = cnt_io holds edit counts of an earlier call on
                          the same f (g_hat is then the state it left) */
} exz_params;

/* Outcome of one correction. */
typedef struct {
  int64_t iterations;          /* rounds that changed at least one value */
  int64_t edited_vertices;     /* vertices whose count went 0 -> 1 in this call */
  int64_t edit_ops;            /* value changes in this call (|E| increments) */
  int64_t lossless_vertices;   /* vertices given the lower bound by the
                                  (N+1)-th edit in this call */
  int64_t floor_vertices;      /* vertices that reached L_i in this call */
  int64_t residual_violations; /* |S| at a stuck fixpoint, else 0 */
  int64_t num_critical;        /* critical points of f */
  int32_t status;              /* exz_status of the call */
  int32_t certified;           /* -1 not run, 0 mismatch, 1 identical */
  double setup_ms;             /* device time of validation + reference topology */
  double loop_ms;              /* device time of the correction loop */
  int64_t check_launches;      /* profiling: check launches issued (those
                                  past the fixpoint return at once) */
  double check_ms;             /* profiling: their summed device time */
  int64_t check_vertices;      /* profiling: vertices they checked (a
                                  frontier pass checks changed boxes only) */
  int64_t targets_total;       /* sum over the iterations that changed a
                                  value of |S| (targets named, blocked ones
                                  included) */
} exz_result;

typedef struct exz_ctx exz_ctx;

/* Create a context on HIP device `device` (makes it current on this
 * thread).  The context owns a device workspace that grows on demand and is
 * reused across calls; hbm_budget_bytes caps the device memory the context
 * and its jobs hold at any time (0 = no cap).  A call whose workspace would
 * exceed the cap returns EXZ_E_NOMEM and leaves earlier state intact, so a
 * scheduler can admit work by the budget.  *out is set on success. */
exz_status exz_ctx_create(int device, size_t hbm_budget_bytes, exz_ctx **out);

/* Device bytes the context and its live jobs hold now (what the budget
 * counts). */
size_t exz_ctx_bytes_in_use(const exz_ctx *ctx);

/* Release the context and its workspace.  NULL is accepted. */
exz_status exz_ctx_destroy(exz_ctx *ctx);

/* Tuning and diagnostics.  None of them changes a result.  Keys:
 *   "profile"  0/1: record device events around every check pass and
 *              report check_launches / check_ms / check_vertices;
 *   "poll"     iterations issued between two host polls (1..256; default:
 *              adaptive: 4, then 8, then chunks of 4..16 that reach the
 *              earliest pass the field can end at, from the last pass the
 *              host saw and the values it changed);
 *   "graph"    0/1: replay the iterations between polls from a captured
 *              hipGraph (batched calls; default 1);
 *   "tile"     check box 64 x tile_y x tile_z given as tile_y * 100 + tile_z;
 *              compiled boxes (y, z): (1,1) (2,2) (4,1) (4,2) (4,4) (8,1)
 *              (8,2) (8,4) (4,8) (16,1) (16,2); 0 (default) picks 4 x 8 for
 *              volumes, 16 x 1 for planes and 1 x 1 for lines.  "tile_y" and
 *              "tile_z" set one side;
 *   "grid"     check work-groups: -1 persistent (default), 0 one per box,
 *              > 0 that many (persistent);
 *   "frontier" 0/1: after the first pass, re-check only boxes whose check
 *              reads a value the last apply changed (a vertex of the box or
 *              its halo), and test the order of the critical points only
 *              for the ranks next to a moved one (reformulated mode;
 *              default 1).  A pass that changes nothing is followed by a
 *              check of every box;
 *   "btile3" / "btile2"  boxes of the 3D / 1D-2D members of batched calls
 *              and of jobs created afterwards (tile_y * 100 + tile_z; 2D
 *              boxes need tile_z = 1; 0 = 4 x 8 and 16 x 1).  A plain
 *              "tile" also sets the 3D box of batches when "btile3" is 0;
 *   "bgrid_box" / "bgrid_apply"  work-group caps of the batched check and
 *              apply passes (0 = 8 resp. 16 per compute unit);
 *   "bitem"    batched apply item size in quads per thread (1..256; 0 = 16);
 *   "job_pool" bytes of released jobs' workspace the context keeps for
 *              later jobs (default 32 GiB; 0 frees each at once).  Taking
 *              pooled memory needs no allocation and freeing into the pool
 *              no wait for the device; pooled bytes count as in use.  A
 *              job whose workspace would pass the context's budget, or whose
 *              allocation fails, frees the pool first (then tries again);
 *   "trim"     frees the pooled job workspace now (value ignored).
 * Returns EXZ_E_INVALID for an unknown key or value. */
exz_status exz_ctx_set_option(exz_ctx *ctx, const char *key, int64_t value);

/* Device workspace the library needs for one field, in bytes, beyond the
 * caller's f, g_hat, g_out and cnt_io.  Sizes the per-critical-point arrays
 * for the worst case (every vertex critical).  0 for invalid params.
 * exz_workspace_bytes_k: the same for a field with num_critical critical
 * points (a count a job's result reports once its set-up has run; a
 * scheduler may admit with an estimate and correct it then). */
size_t exz_workspace_bytes(const exz_params *params);
size_t exz_workspace_bytes_k(const exz_params *params, int64_t num_critical);

/* Correct one field (Algorithm 1).
 *   f       device, n values of params->dtype, read-only
 *   g_hat   device, n values, read-only unless aliased by g_out
 *   g_out   device, n values, receives g'
 *   cnt_io  device, n bytes, nullable: receives the per-vertex edit count
 *           (the edit set E of Algorithm 1: 0..N+1); read first if
 *           params->resume
 *   result  host, filled on every return (status mirrors the return value)
 *   stream  hipStream_t or NULL
 * Errors: see exz_status.  On an error status g_out is unspecified. */
exz_status exz_correct(exz_ctx *ctx, const void *f, const void *g_hat, void *g_out,
                       uint8_t *cnt_io, const exz_params *params, exz_result *result,
                       void *stream);

/* exz_correct for HOST pointers (tests, small tools): f, g_hat and the
 * counts are copied to device buffers the context owns (they count against
 * its budget), corrected on the default stream, and g' (and the counts if
 * cnt_io is not NULL) copied back into g_out / cnt_io, which may alias
 * g_hat.  The same statuses as exz_correct; on an error status g_out is
 * left unchanged.  Timings in *result exclude the copies. */
exz_status exz_correct_host(exz_ctx *ctx, const void *f, const void *g_hat, void *g_out,
                            uint8_t *cnt_io, const exz_params *params, exz_result *result);

/* exz_correct for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, statuses and results as exz_correct (bit for bit), but the
 * call allocates nothing: its workspace is one static device buffer of
 * 128 MiB per GPU, held until the process ends, that every call on that GPU
 * shares.  A field whose workspace does not fit (about 7 bytes per vertex
 * plus 32 (float32) or 44 (float64) bytes per critical point, path
 * workspace for the original mode or the certificate on top) returns
 * EXZ_E_NOMEM with a message; the per-vertex part is checked before any work
 * is issued.  The caller passes f, g_hat, g_out (and cnt_io) as for
 * exz_correct.  Calls that overlap in time on the same GPU race on the
 * buffer: serialise them.  Profiling counters are not recorded. */
exz_status exz_correct_noalloc(exz_ctx *ctx, const void *f, const void *g_hat, void *g_out,
                               uint8_t *cnt_io, const exz_params *params, exz_result *result,
                               void *stream);

/* One field of a batch. */
typedef struct {
  exz_params params;
  const void *f;      /* device */
  const void *g_hat;  /* device */
  void *g_out;        /* device, may alias g_hat */
  uint8_t *cnt_io;    /* device, nullable */
} exz_field;

/* Correct many fields of mixed size, dimension and dtype together: each
 * phase of an iteration is one launch over the (field, tile) items of all
 * fields that have not converged, with per-field worklists, counters and
 * convergence flags (Algorithm 1 run independently per field).  results[k]
 * is what exz_correct would return for fields[k], bit for bit.  Returns the
 * first error status among the fields, else EXZ_OK (warnings are per
 * field).  The fields' set-up runs on streams owned by the context (so the
 * small kernels of different fields overlap) and the iterations on the
 * context's own stream; all of it starts after the work already issued on
 * `stream` and completes before anything issued on `stream` afterwards. */
exz_status exz_correct_batch(exz_ctx *ctx, const exz_field *fields, int32_t nfields,
                             exz_result *results, void *stream);

/* Serving primitives: a job keeps its correction state resident on the
 * device between calls, so a host scheduler can admit new jobs while others
 * iterate (continuous batching).  exz_job_create validates the field and
 * builds the reference topology of f (it allocates the job's workspace; it
 * waits for the validation, so a bad field is reported here);
 * exz_step advances every listed unfinished job by up to `iters` rounds in
 * shared batched launches; exz_job_poll reports completion (it waits for
 * the work issued for the job); exz_job_release returns the job's workspace
 * to the context (not the caller's buffers) once the device is done with
 * it, without waiting.  A job's final state equals exz_correct on the same
 * field (Algorithm 1 per field).
 *
 * For a scheduler that must never wait on the device:
 *   exz_job_submit   as exz_job_create, but returns once the first half of
 *                    the set-up (validation, reference topology, counts of
 *                    critical points) is issued on `stream`; the second
 *                    half (the critical points in f's order) is issued on
 *                    the same stream by the first exz_step, exz_job_query or
 *                    exz_job_poll that finds the first half ended, and a
 *                    step skips the job until then.  `stream` must stay
 *                    valid until then.  A validation error (EXZ_E_BOUND,
 *                    EXZ_E_NONFINITE) is reported by exz_job_query /
 *                    exz_job_poll with *done = 1; the job must still be
 *                    released.
 *   exz_job_query    as exz_job_poll, but never waits: *done and *result
 *                    reflect the job's state after its latest step whose
 *                    work has ended (*done = 0 while no step of it has). */
typedef struct exz_job exz_job;
exz_status exz_job_create(exz_ctx *ctx, const exz_field *field, void *stream, exz_job **out);
exz_status exz_job_submit(exz_ctx *ctx, const exz_field *field, void *stream, exz_job **out);
exz_status exz_step(exz_ctx *ctx, exz_job *const *jobs, int32_t njobs, int32_t iters,
                    void *stream);
exz_status exz_job_poll(exz_job *job, int32_t *done, exz_result *result);
exz_status exz_job_query(exz_job *job, int32_t *done, exz_result *result);
exz_status exz_job_release(exz_job *job);
size_t exz_job_bytes(const exz_params *params);

/* Human-readable text of a status; last error message of a context. */
const char *exz_status_string(int status);
const char *exz_last_error(const exz_ctx *ctx);

/* Diagnostics used by the tests (not needed for correction):
 * the band bounds L_i, U_i exactly as the device computes them
 * (TwoSum-based directed rounding), for n values of f (device pointers). */
exz_status exz_debug_bounds(exz_ctx *ctx, int32_t dtype, const void *f, int64_t n, double xi,
                            void *L_out, void *U_out, void *stream);

/* Diagnostics: one CheckConstraints pass of g against f, no edit.  Writes
 * mark_out[i] = 1 for every vertex the rules would decrease (device, n
 * bytes) and returns |S| in *count. */
exz_status exz_debug_targets(exz_ctx *ctx, const void *f, const void *g, const exz_params *params,
                             uint8_t *mark_out, int64_t *count, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* EXACTZ_H */
