/*
 * km.h -- C ABI of libkmaa: Anderson-accelerated Lloyd K-Means on AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Zhang, Yao, Peng, Yu, Deng, "Fast K-Means Clustering with Anderson
 * Acceleration" (arXiv 1805.10638).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array arguments named X, C, C0, C_out, rho, rho_prev, rho_out are
 *    DEVICE pointers (memory from hipMalloc or a framework allocator on the
 *    context's device), row-major and contiguous.  The caller owns them; the
 *    library never frees or retains them after the call returns.  X, C, C0
 *    and C_out start on a 16-byte boundary (allocator base pointers do);
 *    otherwise the call returns KM_EINVAL.
 *  - Scalar outputs (E, iters) and statistics structs are HOST pointers.
 *  - X is N x d, stored as float32 (KM_X_F32) or as bfloat16 bit patterns
 *    (KM_X_BF16, uint16 per element).  C, C0 and C_out are K x d float32.
 *    Labels are int32 in [0, K).
 *  - Limits: 1 <= K <= N, 1 <= d <= 256, K <= 4096, N < 2^31.  Violations
 *    return KM_EINVAL (bad value) or KM_EUNSUPPORTED (beyond a limit).
 *  - Every call is stream-ordered on the context's HIP stream and returns
 *    after the results are complete (it synchronises that stream).
 *  - Errors are reported by status code only; km_last_error() gives a
 *    message for the last failing call on that context.  On error, outputs
 *    are unspecified.  A context is not thread-safe.
 */
#ifndef KM_H
#define KM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KM_OK = 0,               /* converged (exactly, or by the energy tolerance) */
  KM_NOT_CONVERGED = 1,    /* max_iter reached; outputs hold the last accepted iterate */
  KM_EINVAL = -1,          /* invalid argument */
  KM_ENOMEM = -2,          /* device allocation failed */
  KM_EDEVICE = -3,         /* HIP runtime error */
  KM_EUNSUPPORTED = -4,    /* argument beyond a documented limit */
  KM_ENONFINITE = -5       /* an energy evaluated to Inf/NaN */
} km_status;

typedef enum { KM_X_F32 = 0, KM_X_BF16 = 1 } km_xtype;

/* Precision of the distance GEMM inside the assignment step.  Labels are the
 * exact float64 argmin either way: rows whose best/second-best gap is within
 * a rigorous rounding bound of the GEMM are re-checked with float64 direct
 * differences. */
typedef enum { KM_GEMM_F32 = 0, KM_GEMM_BF16 = 1 } km_prec;

/* Solver flags (km_opts.flags). */
#define KM_FLAG_FIXED_M        1u  /* keep m at m_init (classical fixed-m Anderson, Sec. 2.2) */
#define KM_FLAG_LITERAL_RETURN 2u  /* return as soon as an assignment repeats, even for an
                                      accelerated iterate (Algorithm 1 read literally) */
#define KM_FLAG_BOUNDS         4u  /* kmeans_solve: keep per-row lower bounds of the distance to
                                      the second-nearest centroid (Hamerly's bound, as the paper's
                                      assignment step does, Sec. 3) and skip the distance GEMM for
                                      rows whose bound proves their label; float32 GEMM with the
                                      K x d centroids fitting the kernel's LDS budget only (ignored
                                      otherwise and by the engine).  Labels and decisions are those
                                      of the full assignment; E may differ in its last bits. */

#define KM_M_MAX_LIMIT 64          /* largest supported m_max */
#define KM_TRACE_REC 80            /* doubles per trace record (see km_opts) */

typedef struct km_ctx km_ctx;

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; NULL selects the device's null stream).  The context owns
 * a workspace that grows on demand and is freed by km_destroy. */
km_status km_create(int device, void *hip_stream, km_ctx **out);
void km_destroy(km_ctx *ctx);

/* Change the stream of an existing context. */
km_status km_set_stream(km_ctx *ctx, void *hip_stream);

/* Static string for a status code. */
const char *km_status_str(int status);

/* Message describing the last failure on `ctx` ("" if none). */
const char *km_last_error(const km_ctx *ctx);

/* Library version as 10000*major + 100*minor + patch. */
int km_version(void);

/* Time every candidate-assignment launch of kmeans_solve (1) or not (0,
 * default), with HIP start and end events taken by the kernel's own dispatch.
 * Results appear in km_solve_stats.assign_ms, and for kmeans_g in
 * km_g_stats.assign_ms / update_ms. */
km_status km_set_timing(km_ctx *ctx, int enable);

/* Tile shape of the assignment kernel for later calls on this context whose
 * precision, X type, padded width (from d) and K bucket (the power of two
 * at or above K, at least 16) match (prec, xt, d, K).  shape 0 is the
 * built-in default; 1 .. KM_TILE_SHAPES-1 select alternatives of the kernel
 * family (rows per workgroup, waves, LDS chunk).  Labels and centroids do
 * not depend on the shape; E may differ in its last bits (summation order
 * of per-workgroup partials).  This is the hook of the autotuner.  Returns
 * KM_EINVAL for a shape or size outside the supported range. */
#define KM_TILE_SHAPES 4
km_status km_set_tile_shape(km_ctx *ctx, km_prec prec, km_xtype xt, int32_t d, int32_t K, int32_t shape);
/* Current shape for (prec, xt, d, K); -1 for invalid arguments. */
int32_t km_get_tile_shape(const km_ctx *ctx, km_prec prec, km_xtype xt, int32_t d, int32_t K);

typedef struct {
  int64_t changed;         /* rows whose label differs from rho_prev (0 if rho_prev NULL) */
  int64_t recheck_rows;    /* rows whose label was re-checked with float64 differences (the
                              GEMM's rounding bound could not separate the two best scores) */
  int64_t near_tie_rows;   /* rows whose two smallest float64 squared distances d1 <= d2
                              satisfy (d2 - d1) < 1e-6 d2 (or d2 = 0): the near ties of the
                              parity definition; every such row is among the re-checked rows */
  int32_t empty_clusters;  /* clusters with no sample (centroid kept, reading R9) */
  float assign_ms;         /* device time of the assignment kernel, -1 unless timing is on */
  float update_ms;         /* device time of the update step (cluster sums and sizes,
                              means), -1 unless timing is on; the one pass over X that
                              bounds |x| for the fixed-point sums is not included */
} km_g_stats;

/*
 * kmeans_g -- one application of the fixed-point map G of Sec. 2.1, Eq. (6).
 *   rho   = Assignment-Step(X, C)            (Sec. 1, Eq. (3); lowest index on ties)
 *   C_out = Update-Step(X, rho)              (Sec. 1, Eq. (4)); an empty cluster keeps C_j
 *   *E    = sum_i ||x_i - c_{rho_i}||^2      (Sec. 1, Eq. (1)), energy of the INPUT C
 * Cluster sums: when K*d + K <= 10240, int64 fixed-point sums of the
 * coordinates rounded to multiples of 2^-e, 2^e the largest power of two with
 * N * max|x| * 2^e < 2^62 and max|x| * 2^e < 2^51 (each mean within
 * N * max|x| * 2^-61 of the exact mean of the float32 values, max|x| * 2^-51
 * below 2048 rows); otherwise float64 sums in a fixed order.  Both
 * are bitwise reproducible; kmeans_solve and the engine use the same sums.
 * Arguments:
 *   X [N x d] (xt), C [K x d] float32, rho_prev [N] int32 or NULL (only used
 *   to count changed labels), rho [N] int32 out, C_out [K x d] float32 out
 *   (must not alias C or X), E host double out, st host stats out or NULL.
 */
km_status kmeans_g(km_ctx *ctx, const void *X, km_xtype xt, int64_t N, int32_t d, int32_t K,
                   const float *C, km_prec prec, const int32_t *rho_prev,
                   int32_t *rho, float *C_out, double *E, km_g_stats *st);

/*
 * kmeans_g_noalloc -- kmeans_g for callers that cannot allocate device memory
 * (code being recorded into a HIP graph, tight serving loops, hosts that
 * forbid allocation after start-up).  Same arguments, checks, kernels and
 * results as kmeans_g (labels, C_out and E bitwise equal for the same
 * inputs and tile shape), but the call allocates nothing: every buffer
 * beyond the caller's inputs and outputs comes from one fixed device array
 * of KM_NOALLOC_SCRATCH_BYTES per device, which the library holds from
 * km_create until the process ends.
 *   Limit: a shape whose scratch (control block, prepared centroids, energy
 *   partials, N flagged-row slots and the update's buffers; roughly
 *   4 N + 8 (K d + K) * 256 bytes on the fixed-point path, 12 N + 8 d (N/512
 *   + K) on the sorting path) exceeds the array returns KM_EUNSUPPORTED with
 *   the bytes it would need in km_last_error.
 *   Every call on a device shares that device's array, and the array keeps
 *   the last call's contents: calls that overlap in time on one device (two
 *   host threads, or two contexts on different streams) race and must be
 *   serialised by the caller.
 */
#define KM_NOALLOC_SCRATCH_BYTES (64u << 20)
km_status kmeans_g_noalloc(km_ctx *ctx, const void *X, km_xtype xt, int64_t N, int32_t d, int32_t K,
                           const float *C, km_prec prec, const int32_t *rho_prev,
                           int32_t *rho, float *C_out, double *E, km_g_stats *st);

typedef struct {
  double eps1;          /* dynamic-m shrink threshold (Sec. 3 default 0.02) */
  double eps2;          /* dynamic-m grow threshold (Sec. 3 default 0.5) */
  double ridge;         /* Tikhonov term of the normalised normal equations (1e-10) */
  int32_t m_init;       /* initial m, clipped to m_max (Sec. 3 default 2) */
  int32_t max_iter;     /* iteration cap (default 500) */
  km_prec prec;         /* distance-GEMM precision (default KM_GEMM_F32) */
  uint32_t flags;       /* KM_FLAG_* */
  /* Optional step-by-step trace, device pointers, both may be NULL:
   *   trace_C   [(max_iter + 1) x K x d] float32: candidate C^t at slot t.
   *   trace_rec [(max_iter + 1) x KM_TRACE_REC] double, slot t holds
   *     0 t, 1 E(candidate), 2 changed labels of candidate, 3 m after the
   *     m-rule, 4 decision (0 Lloyd candidate kept, 1 accelerated kept,
   *     2 rejected, 3 converged, 4 stopped by tol, 5 max_iter),
   *     5 E(fall-back), 6 changed labels of fall-back, 7 accepted energy,
   *     8 m_t, 9 columns used, 10 re-checked rows, 11 stop code, 12 near-tie rows,
   *     16.. theta_1..theta_{m_t}. */
  float *trace_C;
  double *trace_rec;
  /* Optional HOST pointer, NULL or (max_iter + 1) ints: entry 0 is the initial m,
   * entry t (1 <= t <= iters) the m after the dynamic-m rule of iteration t
   * (Sec. 2.2); entries past iters are not written. */
  int32_t *m_traj;
} km_opts;

/* Fill `opt` with the defaults listed above. */
void km_opts_default(km_opts *opt);

typedef struct {
  int32_t iters;           /* value of t at return */
  int32_t accepted;        /* iterations that kept an accelerated candidate */
  int32_t rejected;        /* iterations that fell back to the Lloyd iterate */
  int32_t assign_passes;   /* assignment passes incl. the one of G(C0) */
  int32_t m_final;         /* m at return */
  int32_t assign_launches; /* timed candidate assignment launches (timing on) */
  int64_t recheck_rows;    /* rows re-checked in float64, summed over passes */
  int64_t near_tie_rows;   /* near-tie rows (see km_g_stats), summed over passes */
  int64_t gemm_rows;       /* rows that went through the distance GEMM, summed over passes
                              (N per pass unless KM_FLAG_BOUNDS skipped rows) */
  int32_t bounds;          /* 1 if row bounds were in use */
  double device_ms;        /* wall time of the call measured with HIP events */
  double assign_ms;        /* summed duration of the timed assignment launches */
} km_solve_stats;

/*
 * kmeans_solve -- Anderson-accelerated Lloyd iteration with dynamic m and
 * the energy-decrease safeguard (Sec. 2.1, Sec. 2.2, Algorithm 1).
 *   Starts from C0 [K x d] float32.  m_max (0..KM_M_MAX_LIMIT) bounds the
 *   number of previous iterates; m_max = 0 is plain Lloyd.  tol >= 0 stops
 *   when the accepted energy's relative decrease is at most tol (0 = run to
 *   an exact fixed point).  opt may be NULL (defaults).
 * Outputs: C_out [K x d] float32 (may alias C0), rho_out [N] int32, *E the
 *   energy of C_out, *iters, *st (host, may be NULL).
 * Returns KM_OK on convergence, KM_NOT_CONVERGED after max_iter iterations
 * (outputs hold the last accepted iterate), or an error.
 */
km_status kmeans_solve(km_ctx *ctx, const void *X, km_xtype xt, int64_t N, int32_t d, int32_t K,
                       const float *C0, int32_t m_max, double tol, const km_opts *opt,
                       float *C_out, int32_t *rho_out, double *E, int32_t *iters,
                       km_solve_stats *st);

/* ---------------------------------------------------------------------
 * Many instances at once (batched and served solving).
 *
 * A job is one kmeans_solve problem with its own X, sizes, C0 and outputs.
 * An engine advances all its active jobs together, one iteration of
 * Algorithm 1 each per step: every step of the method (assignment per tile
 * shape, controller, update, finalisation, Anderson combination) is one
 * batched launch over the active jobs, and while the set of jobs does not
 * change the launches of an iteration are replayed from a HIP graph.
 * A job gets the labels, iteration count and decisions of kmeans_solve on
 * it alone; E and C may differ in the last bits where a different split of
 * the per-workgroup energy partials rounds differently.
 * ------------------------------------------------------------------- */
typedef struct {
  const void *X;         /* N x d, device */
  km_xtype xt;
  int64_t N;
  int32_t d, K;
  const float *C0;       /* K x d float32, device */
  float *C_out;          /* K x d float32, device, written when the job finishes */
  int32_t *rho_out;      /* N int32, device, written when the job finishes */
  km_prec prec;          /* distance-GEMM precision of this job */
} km_job;

typedef struct {
  int64_t ticket;        /* from km_engine_submit; the job index for kmeans_solve_batch */
  int32_t status;        /* KM_OK, KM_NOT_CONVERGED or KM_ENONFINITE */
  int32_t iters;
  double E;
  int32_t accepted, rejected, assign_passes, m_final;
  int64_t recheck_rows, near_tie_rows;
  double latency_ms;     /* host time from submission to the result being ready */
} km_job_result;

typedef struct km_engine km_engine;

/* Engine on ctx's device (its own internal stream, ordered after ctx's
 * stream at creation).  Jobs share m_max, tol and opt (opt may be NULL; its
 * trace and m_traj pointers must be NULL).  hbm_budget bounds the device bytes
 * of the admitted jobs at once (0: no bound): each job counts its workspace
 * plus its X, C0, C_out and rho_out; queued jobs are admitted
 * in submission order when they fit.  graphs = 1 replays iterations from a
 * HIP graph while the job set is unchanged.  Each job's GEMM precision is
 * its own (km_job.prec; opt->prec is not used). */
km_status km_engine_create(km_ctx *ctx, int32_t m_max, double tol, const km_opts *opt,
                           int64_t hbm_budget, int32_t graphs, km_engine **out);
/* Waits for the device and releases everything; unfinished jobs are dropped. */
void km_engine_destroy(km_engine *e);

/* Device workspace bytes of a job (what the budget counts), or -1. */
int64_t km_job_workspace_bytes(const km_job *job, int32_t m_max);

/* Queue a job (checked like kmeans_solve); *ticket names its result.  Its
 * buffers must stay valid until km_engine_poll has returned the result.
 * KM_ENOMEM if its device memory alone (workspace, X, C0, C_out, rho_out)
 * exceeds the budget. */
km_status km_engine_submit(km_engine *e, const km_job *job, int64_t *ticket);

/* Admit queued jobs that fit (at iteration boundaries), launch one
 * iteration of every active job when fewer than three are in flight, and
 * collect the iterations that have completed.  wait = 1: if nothing could
 * be launched or collected, block until the oldest iteration in flight
 * completes; wait = 0 never blocks except while the job set changes (the
 * engine then drains its own stream).  Any count pointer may be NULL: jobs
 * on the device, waiting for admission, results ready. */
km_status km_engine_step(km_engine *e, int32_t wait, int32_t *n_active, int32_t *n_queued, int32_t *n_ready);

/* Fraction (0, 1] of the device's resident assignment workgroups this
 * engine's launches may take (1: all, and twice as many for balance).
 * Below 1 the rest of the device stays free for work on other streams,
 * e.g. a second engine serving small jobs while this one serves large ones. */
km_status km_engine_set_share(km_engine *e, double frac);

/* 1 and *res filled if a finished job's result was taken (oldest first), 0 if none. */
int32_t km_engine_poll(km_engine *e, km_job_result *res);

/* Solve n jobs as one batch (an engine without budget, graphs on) and wait;
 * res[i] is job i's result.  KM_OK when every job ran (each job's status is
 * in res[i]). */
km_status kmeans_solve_batch(km_ctx *ctx, const km_job *jobs, int32_t n, int32_t m_max, double tol,
                             const km_opts *opt, km_job_result *res);

#ifdef __cplusplus
}
#endif

#endif /* KM_H */
