/*
 * fkconv -- FK-table convolution on MI355X (gfx950), C ABI.
 *
 * The operation (Section 3, Eq. (1) of the paper): observables are
 * contractions of a PDF sampled on an x-grid, f_a(x_alpha), with a
 * precomputed FK ("fast kernel") table, one table per dataset:
 *
 *   DIS (linear):       T[i,r]     = sum_{a, alpha} FK[i,a,alpha] f_r[a,alpha]
 *   hadronic (Eq. (1)): sigma[i,r] = sum_{a,b,alpha,beta}
 *                                      FK[i,a,b,alpha,beta] f_r[a,alpha] f_r[b,beta]
 *
 * with i a datapoint, a, b flavours, alpha, beta grid points and r a PDF
 * replica; all replicas share the table and are computed in one pass
 * (Section 3 suggests parallelising over replicas).  The paper's Eq. (1)
 * names grid indices (i, j) and flavour indices (alpha, beta); this header
 * uses i for datapoints instead.
 *
 * Conventions for every entry point
 *  - Return value: FK_OK (0) or a negative FK_E_* code.  No exception and no
 *    abort crosses the ABI; fk_last_error() returns a message for the last
 *    failing call on the context.
 *  - Host pointers (const double*, const uint8_t*, const int32_t*) are read
 *    during the call only; the library copies what it keeps.
 *  - Device pointers (float*, double* documented as "device") belong to the
 *    caller and must stay valid until the work queued on ``stream`` is done.
 *  - ``stream`` is a hipStream_t (NULL = the legacy default stream).  Calls
 *    that take a stream are asynchronous: they enqueue kernels and return.
 *  - Layouts are row-major with the replica index fastest:
 *      PDF f       [nflav][nx][nrep]   float32, device
 *      observables [ndata][nrep]       float32, device
 *  - Calls on one table/group handle use that handle's scratch memory, so
 *    they must be ordered on one stream.  The serving loop gives each of its
 *    streams private scratch per table, so direct calls and served requests
 *    on the same table may overlap.
 */
#ifndef FKCONV_H
#define FKCONV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fk_ctx fk_ctx;
typedef int32_t fk_status;
typedef int64_t fk_table;   /* a loaded table or a group of tables */
typedef int64_t fk_cov;     /* a loaded block-diagonal covariance */
typedef int64_t fk_ticket;  /* a serving request */
typedef int64_t fk_mlp;     /* a network PDF parametrisation */

enum {
  FK_OK = 0,
  FK_E_ARG = -1,        /* null pointer, bad enum, non-positive size */
  FK_E_SHAPE = -2,      /* sizes inconsistent with the table */
  FK_E_GRID = -3,       /* x-grid differs from the table's */
  FK_E_HANDLE = -4,     /* unknown or unloaded handle */
  FK_E_BUDGET = -5,     /* device-memory budget exhausted */
  FK_E_TOO_LARGE = -6,  /* request can never fit its limits */
  FK_E_HIP = -7,        /* HIP runtime error (context may be unusable) */
  FK_E_NOTPD = -8,      /* covariance block not positive definite */
  FK_E_STATE = -9,      /* call not valid in the current state */
  FK_E_QUEUE_FULL = -10 /* serving queue full, retry later */
};

enum { FK_DIS = 1, FK_HAD = 2 };                      /* table kinds */
enum { FK_F32 = 0, FK_BF16 = 1, FK_FP8E4M3 = 2 };     /* storage dtypes */
enum { FK_QUEUED = 0, FK_RUNNING = 1, FK_DONE = 2, FK_FAILED = 3 };

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device ``device``.  All device memory the library
 * allocates (tables, covariances, per-handle scratch, serving buffers) is
 * charged against ``hbm_budget_bytes`` (0 = 90% of the free device memory);
 * an allocation beyond it fails with FK_E_BUDGET.  *out is set on success. */
fk_status fk_create(fk_ctx **out, int32_t device, uint64_t hbm_budget_bytes);

/* Stop the serving loop if running, wait for the device, free everything.
 * Handles of this context become invalid. */
fk_status fk_destroy(fk_ctx *ctx);

/* Message of the last failing call on ``ctx`` (or of a failed fk_create when
 * ctx is NULL).  Valid until the next call on the context. */
const char *fk_last_error(const fk_ctx *ctx);

/* Bytes currently charged to the budget, and the budget itself. */
fk_status fk_memory(const fk_ctx *ctx, uint64_t *used_bytes, uint64_t *budget_bytes);

/* Context options.
 *  FK_OPT_KERNELS  FK_KERNELS_STREAM (default): the streaming hadronic
 *                  forward/adjoint and DIS forward kernels where a plan has
 *                  them; FK_KERNELS_ITEM: the persistent / per-item kernels
 *                  (for comparisons: the two families sum in different
 *                  orders, so results agree to rounding, not bitwise).
 * Takes effect for calls issued after it returns.  FK_E_ARG for an unknown
 * option or value. */
enum { FK_OPT_KERNELS = 1 };
enum { FK_KERNELS_STREAM = 0, FK_KERNELS_ITEM = 1 };
fk_status fk_set_option(fk_ctx *ctx, int32_t option, int64_t value);

/* ---- tables (Section 3: one FK table per dataset) --------------------- */

/* Load one dataset's FK table and keep it resident on the device.
 *  kind        FK_DIS or FK_HAD.
 *  ndata       datapoints N >= 1.   nflav  flavours F (1..64).
 *  nx          grid points X (2..128).
 *  xgrid       host [nx], the x-grid the table is defined on (kept for the
 *              grid check of the conv calls).
 *  mask        host; DIS: [nflav], hadronic: [nflav][nflav] row-major; a
 *              nonzero entry marks an active flavour (pair).  Only active
 *              blocks are stored, as in the paper's base table with 49 flavour
 *              combinations (Table 3 caption).
 *  fk          host float64, active blocks only:
 *                DIS      [ndata][nact][nx]        active flavours ascending
 *                hadronic [ndata][npairs][nx][nx]  active (a,b) row-major,
 *                         element [i,c,alpha,beta] multiplies f_a(x_alpha) f_b(x_beta)
 *              General (non-symmetric) hadronic tables and masks are accepted.
 *  store_dtype FK_F32, FK_BF16 or FK_FP8E4M3: the format the table is stored
 *              and multiplied in (FP32 accumulation in every case).  Each
 *              datapoint row is scaled by a power of two s_i so its largest
 *              entry fits the format; the scale is applied exactly afterwards.
 * The table is packed on the host (only active blocks, per-datapoint scale,
 * round-to-nearest-even) and copied to the device once.  The device keeps
 * two copies of each table: DIS, the table and its transpose (for the
 * adjoint); hadronic, the symmetric part S = FK + FK^T over unordered flavour
 * pairs (blocks b > a, and S_aa / 2 on the diagonal) for the forward, since
 * Eq. (1) only sees S, and S over the whole symmetric pattern for the
 * adjoint. */
fk_status fk_load_table(fk_ctx *ctx, int32_t kind, int32_t ndata, int32_t nflav,
                        int32_t nx, const double *xgrid, const uint8_t *mask,
                        const double *fk, int32_t store_dtype, fk_table *out);

/* Free a table (or a group; tables in a group stay loaded). */
fk_status fk_unload_table(fk_ctx *ctx, fk_table table);

/* Build a group of tables of one kind, dtype and x-grid that later calls
 * treat as one table whose datapoints are the concatenation of the members'
 * (in the given order).  One call then convolves every dataset of a fit in
 * one set of launches.  The member tables must outlive the group. */
fk_status fk_group_create(fk_ctx *ctx, int32_t ntables, const fk_table *tables,
                          fk_table *out);

/* Describe a table or group (any output pointer may be NULL). */
fk_status fk_table_info(fk_ctx *ctx, fk_table table, int32_t *kind, int32_t *ndata,
                        int32_t *nflav, int32_t *nx, int32_t *store_dtype,
                        uint64_t *device_bytes);

/* ---- convolutions (asynchronous on ``stream``) ------------------------- */

/* DIS observables T [ndata][nrep] (device float32) of a DIS table/group.
 *  pdf_xgrid  host [nx] or NULL: when given it must equal the table's grid
 *             (relative 1e-12), else FK_E_GRID.
 *  pdf        device float32 [nflav][nx][nrep].
 *  nrep       replicas R >= 1 (any size; processed in chunks of 128). */
fk_status fk_conv_dis(fk_ctx *ctx, fk_table table, const double *pdf_xgrid,
                      const float *pdf, int32_t nrep, float *out, void *stream);

/* fk_conv_dis for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same kernels and the same results, bitwise, but the staged PDF operand
 * lives in a static device array of 4 MiB per GPU (held until the process
 * ends) instead of the table's scratch, and the call allocates nothing.
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (on different streams, or from different contexts) race and must be
 * ordered by the caller.  FK_E_TOO_LARGE when the table's staged operand
 * exceeds 4 MiB (it takes about 120 KiB per distinct flavour pattern of 9
 * flavours on 50 x-points in BF16, 240 KiB in FP32),
 * FK_E_STATE when the table does not use the streaming DIS kernel; other
 * arguments and errors as fk_conv_dis. */
fk_status fk_conv_dis_static(fk_ctx *ctx, fk_table table, const double *pdf_xgrid,
                             const float *pdf, int32_t nrep, float *out, void *stream);

/* Hadronic observables sigma [ndata][nrep], Eq. (1), of a hadronic
 * table/group.  Same arguments as fk_conv_dis. */
fk_status fk_conv_had(fk_ctx *ctx, fk_table table, const double *pdf_xgrid,
                      const float *pdf, int32_t nrep, float *out, void *stream);

/* Adjoint (vector-Jacobian product) of the convolution with respect to the
 * PDF, the gradient the paper's custom operator returns beside the
 * convolution (Section 3, Table 1):
 *   DIS:      g[a,alpha,r] = sum_i gbar[i,r] FK[i,a,alpha]
 *   hadronic: g[p,r] = sum_i gbar[i,r] (sum_q FK[i,p,q] f[q,r] + sum_q FK[i,q,p] f[q,r]),
 *             p = (a,alpha), q = (b,beta)
 *  pdf        device float32 [nflav][nx][nrep] (ignored for DIS, may be NULL).
 *  grad_out   device float32 [ndata][nrep], gbar.
 *  grad_pdf   device float32 [nflav][nx][nrep]; overwritten, or added to when
 *             ``accumulate`` is nonzero.  Rows of inactive flavours get 0. */
fk_status fk_conv_backward(fk_ctx *ctx, fk_table table, const float *pdf,
                           const float *grad_out, int32_t nrep, float *grad_pdf,
                           int32_t accumulate, void *stream);

/* ---- the flattened form of Table 3 ----------------------------------------
 * Table 3 of the paper times the hadronic convolution as a product of an FK
 * table N x K with a "PDF" matrix K x R, K = 49 flavour combinations x 27^2
 * grid points: the PDF enters through the luminosity
 *   L[(c, alpha, beta)][r] = f[a_c][alpha][r] f[b_c][beta][r]
 * over the active pairs c = (a_c, b_c), and out = FK L.  These calls
 * compute that form (for comparison with Table 3; the conv calls above
 * never form L). */

/* Luminosity of the nonzero entries of ``mask`` (host [nflav][nflav],
 * taken in row-major (a, b) order, at most 1024):
 *  pdf  device float32 [nflav][nx][nrep]
 *  lum  device float32 [npairs * nx * nx][nrep], row (c * nx + alpha) * nx + beta. */
fk_status fk_luminosity(fk_ctx *ctx, int32_t nflav, int32_t nx, const uint8_t *mask,
                        const float *pdf, int32_t nrep, float *lum, void *stream);

/* Device bytes of the workspace fk_flat_conv needs for this shape (0 when
 * it needs none). */
fk_status fk_flat_conv_workspace(fk_ctx *ctx, int64_t n, int64_t k, int64_t r, uint64_t *bytes);

/* out[n][r] = sum_k fk[n][k] lum[k][r]: FP32 inputs, FP32 accumulation in a
 * fixed order (so results are reproducible), device row-major arrays
 *  fk [n][k], lum [k][r], out [n][r];
 * ``work`` (device, ``work_bytes``) holds the partial sums when K is split
 * over workgroups (fk_flat_conv_workspace).  n <= 1048560, r <= 4194240.  Few rows or
 * columns (n <= 16 or r <= 16) stream through the vector units (bound by
 * HBM), larger products run on the FP32 matrix cores. */
fk_status fk_flat_conv(fk_ctx *ctx, int64_t n, int64_t k, int64_t r, const float *fk,
                       const float *lum, float *out, void *work, uint64_t work_bytes,
                       void *stream);

/* ---- network PDF and gradient descent -------------------------------------
 * The steps either side of the convolution in a fit: Section 2 describes
 * fits that parametrise the PDF with a neural network trained by gradient
 * descent, and Section 3 a network that generates the PDF on the x-grid the
 * FK tables are convolved with.  The paper gives no architecture; this one
 * is: inputs (x, ln x), a tanh layer of h1 units, a tanh layer of h2 units,
 * a linear output per flavour, times x^alpha_a (1 - x)^beta_a:
 *   f_r[a][alpha] = x^alpha_a (1-x)^beta_a (W3 tanh(W2 tanh(W1 in + b1) + b2) + b3)_a
 * with one network per replica r.  Parameters of replica r are the row
 * params[r][P], P = 3 h1 + h2 h1 + h2 + nflav h2 + nflav, in the order
 * W1 [h1][2], b1 [h1], W2 [h2][h1], b2 [h2], W3 [nflav][h2], b3 [nflav]
 * (row-major).  FP32 arithmetic; one workgroup per replica. */

/* Describe a network on ``xgrid`` (host [nx], values in (0, 1]) with the
 * preprocessing exponents pre_alpha, pre_beta (host [nflav]); the grid
 * features are kept on the device.  *nparams = P (may be NULL).
 * FK_E_SHAPE unless 1 <= nflav, h1, h2 <= 64, nx <= 256 and one replica's
 * parameters and activations fit 64 KiB of LDS. */
fk_status fk_mlp_create(fk_ctx *ctx, int32_t nflav, int32_t nx, const double *xgrid, int32_t h1,
                        int32_t h2, const double *pre_alpha, const double *pre_beta, fk_mlp *out,
                        int32_t *nparams);
fk_status fk_mlp_destroy(fk_ctx *ctx, fk_mlp mlp);

/* pdf (device [nflav][nx][nrep]) = the networks of params (device [nrep][P]). */
fk_status fk_mlp_forward(fk_ctx *ctx, fk_mlp mlp, const float *params, int32_t nrep, float *pdf,
                         void *stream);

/* grad_params (device [nrep][P]) = gradient of sum_{a,alpha,r}
 * grad_pdf[a][alpha][r] f_r[a][alpha] with respect to params: the
 * reverse pass through the network, e.g. after fk_conv_backward turned
 * d chi2 / d sigma into grad_pdf.  Each parameter's gradient is summed over
 * the grid points in order (reproducible). */
fk_status fk_mlp_backward(fk_ctx *ctx, fk_mlp mlp, const float *params, const float *grad_pdf,
                          int32_t nrep, float *grad_params, void *stream);

/* Gradient-descent step params[i] -= lr * grad[i] for i < n (device arrays). */
fk_status fk_sgd_update(fk_ctx *ctx, float *params, const float *grad, int64_t n, float lr,
                        void *stream);

/* ---- chi2 in FP64 ---------------------------------------------------------
 * chi2_r = (sigma_r - D)^T C^{-1} (sigma_r - D) with C block-diagonal (one
 * block per dataset).  The fit's loss; the paper does not write it out.  */

/* Load a covariance: ``nblocks`` SPD blocks of sizes block_n[k], given as
 * host float64 row-major blocks one after the other.  The blocks are copied
 * to the device and Cholesky-factored there in FP64 (C = L L^T); the
 * triangular inverse of L is kept for the per-call solves.  FK_E_NOTPD if a
 * block is not positive definite. */
fk_status fk_load_covariance(fk_ctx *ctx, int32_t nblocks, const int32_t *block_n,
                             const double *cov, fk_cov *out);
fk_status fk_unload_covariance(fk_ctx *ctx, fk_cov cov);

/* sigma      device float32 [ntot][nrep] (ntot = sum block_n).
 * data       device float64 [ntot].
 * chi2       device float64 [nrep].
 * dchi2_dsigma device float32 [ntot][nrep] = 2 C^{-1} (sigma - D), or NULL.
 * All arithmetic is FP64. */
fk_status fk_chi2(fk_ctx *ctx, fk_cov cov, const float *sigma, const double *data,
                  int32_t nrep, double *chi2, float *dchi2_dsigma, void *stream);

/* ---- kernel timing --------------------------------------------------------
 * When enabled, every launch of the library's kernels on the caller's stream
 * is bracketed by a pair of HIP events on that stream, so the durations are
 * those of the kernels alone.  Kernel kinds index the arrays below. */
enum {
  FK_K_STAGE = 0,       /* B-operand staging (PDF or adjoint weights) */
  FK_K_HAD_FWD = 1,     /* hadronic forward MFMA kernel, persistent form */
  FK_K_DIS_FWD = 2,     /* DIS forward MFMA kernel, partial-sum form */
  FK_K_FWD_REDUCE = 3,  /* forward partial-sum reduction */
  FK_K_HAD_ADJ = 4,     /* hadronic adjoint MFMA kernel, per-item form */
  FK_K_DIS_ADJ = 5,     /* DIS adjoint MFMA kernel */
  FK_K_ADJ_REDUCE = 6,  /* adjoint partial-sum reduction */
  FK_K_CHI2 = 7,        /* FP64 chi2 kernels of one call, together */
  FK_K_HAD_STREAM = 8,  /* hadronic forward MFMA kernel, stream form */
  FK_K_DIS_STREAM = 9,  /* DIS forward MFMA kernel, stream form (no reduction) */
  FK_K_HAD_ADJ_STREAM = 10, /* hadronic adjoint MFMA kernel, stream form */
  FK_K_COUNT = 11
};
fk_status fk_timing_enable(fk_ctx *ctx, int32_t enable);

/* Wait for the recorded events and return, per kernel kind, the summed
 * duration in milliseconds and the number of launches since the previous
 * read (host arrays of FK_K_COUNT entries); then reset. */
fk_status fk_timing_read(fk_ctx *ctx, double *total_ms, int64_t *launches);

/* Measured ceiling of the matrix cores: a kernel of independent
 * v_mfma_f32_16x16x32_bf16 chains on register operands (no memory traffic),
 * 32 waves per compute unit, ``iters`` rounds of eight MFMAs per wave; the
 * best of three timed runs (after one warm-up) in dense BF16 TFLOP/s.  Runs
 * on the legacy default stream and waits for it.  The denominator of the
 * roofline fractions is the datasheet peak; this is the achievable one. */
fk_status fk_measure_mfma_peak(fk_ctx *ctx, int32_t iters, double *tflops);

/* ---- serving: continuous batching of convolution requests --------------
 * Requests name a resident table, carry their own PDF batch and output,
 * and are admitted as request slots and the request-buffer budget allow.
 * Requests on the same table that are admitted together share one pass over
 * the table (their replicas are concatenated); passes of different tables
 * run concurrently on several streams.  A request's result does not depend
 * on which other requests share its pass. */
typedef struct {
  fk_table table;     /* a table (not a group) */
  int32_t nrep;       /* replicas of this request, >= 1 */
  int32_t precision;  /* FK_BF16: the table as loaded, or its FP32 fallback
                         when fk_table_probe found its error above the
                         tolerance; FK_F32: its FP32 fallback table if one
                         is linked (else as loaded) */
  const float *pdf;   /* device [nflav][nx][nrep], valid until DONE/FAILED */
  float *out;         /* device [ndata][nrep], written when DONE */
  uint64_t tag;       /* caller data, unused by the library */
  void *ready;        /* hipEvent_t or NULL: the pass reads ``pdf`` only
                         after this event has completed (record it on the
                         stream that produces the PDF); it must stay valid
                         until the request is DONE or FAILED.  With NULL the
                         PDF must be complete when fk_submit is called. */
} fk_request;

/* Start the serving loop: ``nslots`` requests may be in flight at once,
 * ``nstreams`` device streams run passes concurrently, and staging and
 * scratch memory for in-flight requests is limited to ``request_budget_bytes``
 * (charged to the context budget up front). */
fk_status fk_serve_start(fk_ctx *ctx, int32_t nslots, int32_t nstreams,
                         uint64_t request_budget_bytes);
fk_status fk_serve_stop(fk_ctx *ctx);

/* Link an FP32 copy of a table, used for requests with precision FK_F32. */
fk_status fk_table_set_fallback(fk_ctx *ctx, fk_table table, fk_table fallback);

/* Probe a reduced-precision table (BF16 or FP8) against its linked FP32
 * fallback on a caller PDF batch: both are convolved on ``stream`` and the
 * normwise error max_r ||y_r - y32_r||_2 / ||y32_r||_2 is computed on the
 * device (FP64 sums) and returned in *err (the call waits for the stream).
 * When *err > tol, served requests that ask for the table's own format run
 * on the fallback from then on (FP32 differs from the FP64 definition by
 * about 1e-7, far below any tolerance this is used with); otherwise they
 * run on the table.  The tolerance the paper's setting suggests for BF16 is
 * 5e-3.  The call allocates its two outputs and frees them before it
 * returns.  FK_E_STATE when no fallback is linked. */
fk_status fk_table_probe(fk_ctx *ctx, fk_table table, const float *pdf, int32_t nrep,
                         double tol, double *err, void *stream);

/* Queue a request; never blocks.  FK_E_QUEUE_FULL when the queue is full,
 * FK_E_TOO_LARGE when the request could never fit the request budget. */
fk_status fk_submit(fk_ctx *ctx, const fk_request *req, fk_ticket *out);

/* State of a ticket: FK_QUEUED, FK_RUNNING, FK_DONE or FK_FAILED.  The
 * record of a finished ticket is kept until 65536 later requests have
 * finished (then FK_E_HANDLE), or until fk_serve_stop. */
fk_status fk_poll(fk_ctx *ctx, fk_ticket ticket, int32_t *state);

/* Timing of a finished ticket in nanoseconds of the host steady clock:
 * submission, admission and completion (completion = when fk_poll could
 * first report DONE). */
fk_status fk_ticket_times(fk_ctx *ctx, fk_ticket ticket, uint64_t *t_submit,
                          uint64_t *t_admit, uint64_t *t_done);

#ifdef __cplusplus
}
#endif

#endif /* FKCONV_H */
