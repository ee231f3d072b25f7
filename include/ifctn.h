/*
 * ifctn.h -- C ABI of the iFCTN tensor-completion hot path for MI355X (gfx950).
 *
 * The library solves the iFCTN tensor-completion model (paper: "iFCTN: an
 * intra-block Fully-Connected Tensor Network Decomposition for Tensor
 * Completion", arXiv 2511.16358, eq. (iFCTN-TC)) by proximal alternating
 * minimisation (Algorithm 1): per sweep, every cherry factor G_{k,i} is
 * updated column by column by the proximal least-squares closed form of
 * eq. (updateG), in the order k ascending, i ascending, and then the filled
 * tensor X is updated by eq. (updateX).  All steps run in HIP kernels on the
 * device; the header uses only plain C types.
 *
 * Conventions
 *  - Modes are 0-based.  Tensors are dense, row-major (the last mode is the
 *    fastest), element (i_0,...,i_{N-1}) at offset sum_m i_m * prod_{n>m} I_n.
 *    (The paper numbers modes from 1 and unfolds with mode 1 fastest; the
 *    method itself does not depend on the storage order.)
 *  - The rank matrix R is symmetric, R[a][b] = R[b][a] >= 1 for a != b; the
 *    diagonal is ignored (Def. 2).
 *  - Cherry factor G_{k,i} (Def. 1, eq. (3)) has shape R[k][i] x I_k.  A
 *    "packed factor array" holds all N(N-1) factors as float64 in the order k
 *    ascending, then i ascending (i != k), each one row-major.
 *  - Pointers named *_dev are device pointers (hipMalloc / torch tensors on
 *    the GPU); pointers named *_host are host pointers.  The caller keeps
 *    ownership of every pointer it passes; the library copies what it needs.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued asynchronously on it; calls that return host values
 *    (statistics, factors) synchronise it.
 *  - Every call returns an ifctn_status; no exception crosses the boundary.
 *    On failure ifctn_last_error() gives a message (thread-local).
 *  - A job is not thread-safe; different jobs are independent.
 */
#ifndef IFCTN_H
#define IFCTN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IFCTN_MAX_ORDER 5 /* tensor order N: 2..5 */
/* every R[a][b] in 1..36.  A job with all ranks <= 8 runs the fused kernels
 * (routes 0-2 of ifctn_plan_blocks); a job with any rank above 8 runs every
 * block by the large-rank route (route 3: X o D_{-k} and its mode products
 * into U_k, the per-column Gram rows as a GEMM, one Cholesky per column, all
 * in float64, and a separate X step), in FP32 or FP64 precision only
 * (BF16_REFINE: IFCTN_E_UNSUPPORTED). */
#define IFCTN_MAX_RANK 36
#define IFCTN_MAX_ENTRIES 2147483647LL /* prod(dims) above this: IFCTN_E_UNSUPPORTED */

typedef enum {
  IFCTN_OK = 0,
  IFCTN_E_INVAL = -1,       /* invalid argument (shape, rank, rho, pointer, ...)      */
  IFCTN_E_NOMEM = -2,       /* device allocation failed                                */
  IFCTN_E_HIP = -3,         /* HIP runtime error (message kept)                        */
  IFCTN_E_STATE = -4,       /* call not valid in the job's state                       */
  IFCTN_E_UNSUPPORTED = -5  /* valid in the paper's model, not supported by this build */
} ifctn_status;

typedef enum {
  IFCTN_FP32 = 0,        /* X and the streaming passes in float32; Gram, Cholesky,
                            factors and reductions in float64                      */
  IFCTN_BF16_REFINE = 1, /* X stored and streamed as bfloat16 (round to nearest even)
                            with float32 arithmetic, until ifctn_promote (or the last
                            refine_sweeps sweeps of ifctn_complete) switches the job to
                            the FP32 path; O, outputs and Xhat are float32            */
  IFCTN_FP64 = 2         /* every step in float64                                   */
} ifctn_precision;

typedef struct {
  int32_t order;                                    /* N                               */
  int64_t dims[IFCTN_MAX_ORDER];                    /* I_0 .. I_{N-1}, each >= 1       */
  int32_t ranks[IFCTN_MAX_ORDER][IFCTN_MAX_ORDER];  /* symmetric iFCTN ranks           */
  double rho;    /* proximal weight of the factor blocks, > 0 (Sec. 4.2; 0.1 in Sec. 5) */
  double rho_x;  /* proximal weight of the X step, > 0 (eq. (updateX)); 0 => rho      */
  int32_t precision;     /* ifctn_precision                                          */
  int32_t refine_sweeps; /* BF16_REFINE: float32 sweeps that end ifctn_complete (>= 0);
                            other precisions: must be 0                             */
} ifctn_params;

typedef struct {
  double rel_change;  /* ||X^{s+1} - X^s||_F / ||X^s||_F of the last sweep (Algorithm 1 stop test) */
  double objective;   /* F = f(G^{s+1}, X^{s+1}) = 1/2 ||X^{s+1} - iFCTN(G^{s+1})||_F^2 (eq. (iFCTN-TC)) */
  double x_norm2;     /* ||X^s||_F^2                                                  */
  double dx_norm2;    /* ||X^{s+1} - X^s||_F^2                                         */
  double dg_norm2;    /* sum over blocks of ||G_{k,i}^{s+1} - G_{k,i}^s||_F^2 (Lemma 2)  */
  int32_t sweeps_done;/* sweeps run on this job since ifctn_init                         */
  int32_t converged;  /* 1 if the last sweep met rel_change < eps (ifctn_complete only)  */
} ifctn_stats;

typedef struct ifctn_job ifctn_job;

/* Number of float64 entries of a packed factor array: sum over k and i != k of
 * R[k][i] * I_k (the storage count of Sec. 4.3).  Returns 0 for invalid params. */
size_t ifctn_num_factor_entries(const ifctn_params* params);

/* Device bytes a job with these params allocates (for admission by HBM
 * budget).  Returns 0 for invalid params. */
size_t ifctn_workspace_bytes(const ifctn_params* params);

/* Create a job: validates params, allocates device memory, sets
 * X^0 = P_Omega(O) (O on Omega, 0 elsewhere; Algorithm 1 initialisation)
 * and G^0 from G0_host.
 *   O_dev:    observed tensor, prod(dims) elements, float32 (FP32 and BF16_REFINE
 *             precision) or float64 (FP64 precision).  Entries off Omega are ignored.
 *   mask_dev: prod(dims) bytes, nonzero = observed (the sample set Omega).
 *   G0_host:  packed initial factors (float64); NULL = the seeded default of
 *             ifctn_default_factors with seed 0 (Algorithm 1 takes G^0 as an
 *             input without fixing how it is drawn).
 * Fails with IFCTN_E_INVAL when an observed entry is not finite.  Synchronises
 * the stream.  On success *out owns all device memory until ifctn_destroy. */
ifctn_status ifctn_init(const ifctn_params* params, const void* O_dev, const uint8_t* mask_dev,
                        const double* G0_host, void* stream, ifctn_job** out);

/* Seeded default initial factors for Algorithm 1 (which takes G^0 as an
 * input): writes ifctn_num_factor_entries(params) float64 values to G_host in
 * the packed order.  Entry n is s * u_n, where u_n in [0, 1) is the top 53 bits
 * of output n of SplitMix64 started from seed (the state after n + 1 steps,
 * seed + (n + 1) * 0x9E3779B97F4A7C15, mixed as in Steele, Lea and Flood,
 * OOPSLA 2014), and s = 2 (m / prod_{a<b} R_ab)^(1/(2e)) over the e = N(N-1)/2
 * edges, so that the expected value of every entry of iFCTN(G^0) equals m, the
 * root mean square of the observed entries of O (m = 1 when none is observed
 * or all are 0; m is reduced on the device in a fixed order).  O_dev and
 * mask_dev are as for ifctn_init.  Takes a small stream-ordered device buffer
 * (hipMallocAsync / hipFreeAsync on stream) and synchronises the stream.  IFCTN_E_INVAL for invalid params or NULL pointers. */
ifctn_status ifctn_default_factors(const ifctn_params* params, const void* O_dev, const uint8_t* mask_dev,
                                   uint64_t seed, void* stream, double* G_host);

/* Run nsweeps >= 0 full PAM sweeps (every factor block by eq. (updateG), then
 * eq. (updateX)).  Asynchronous when stats is NULL; otherwise synchronises
 * and fills *stats for the last sweep run. */
ifctn_status ifctn_sweep(ifctn_job* job, int32_t nsweeps, ifctn_stats* stats);

/* Write a dense tensor to out_dev (float32 for FP32 and BF16_REFINE jobs,
 * float64 for FP64): which = 0: iFCTN(G) of the current factors (eq. (iFCTN));
 * which = 1: X (during the bfloat16 phase: O on Omega, the widened bfloat16
 * values elsewhere). */
ifctn_status ifctn_reconstruct(ifctn_job* job, void* out_dev, int32_t which);

/* Copy the current factors to a packed float64 host array.  Synchronises. */
ifctn_status ifctn_get_factors(ifctn_job* job, double* G_host);

/* End the bfloat16 phase of a BF16_REFINE job (precision pattern: cheap
 * bfloat16 sweeps, then float32 refinement sweeps of the same PAM iteration,
 * Algorithm 1): X becomes float32, exactly O on Omega and the widened
 * bfloat16 values elsewhere, and every later sweep runs the FP32 path.
 * Idempotent; IFCTN_E_STATE for jobs of other precisions.  Asynchronous. */
ifctn_status ifctn_promote(ifctn_job* job);

/* Release a job and its device memory (NULL is accepted). */
ifctn_status ifctn_destroy(ifctn_job* job);

/* Algorithm 1 end to end (G0_host as for ifctn_init: NULL = the seeded default
 * of seed 0): init, sweeps until rel_change < eps or t_max sweeps
 * (eps = 0 runs exactly t_max), write X to X_out_dev (same dtype as O_dev),
 * fill *stats (nullable), destroy.  Synchronises.  BF16_REFINE: the first
 * t_max - refine_sweeps sweeps (or fewer, when the stop test is met) stream
 * bfloat16, then the job is promoted and min(refine_sweeps, t_max) float32
 * sweeps follow; converged reports the stop test of the bfloat16 phase. */
ifctn_status ifctn_complete(const ifctn_params* params, const void* O_dev, const uint8_t* mask_dev,
                            const double* G0_host, int32_t t_max, double eps, void* X_out_dev,
                            ifctn_stats* stats, void* stream);

/* Materialise iFCTN(G) (eq. (iFCTN)) for packed factors G_host into out_dev
 * (float32 for FP32 params, float64 for FP64), without a job.  Synchronises. */
ifctn_status ifctn_assemble(const ifctn_params* params, const double* G_host, void* out_dev,
                            void* stream);

/* ifctn_assemble without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  The packed factors and every edge matrix W_ab are
 * staged in a fixed device array of IFCTN_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends; its address
 * on the current device is looked up on the first call there.  The
 * arguments, result and synchronisation are those of ifctn_assemble.  A
 * problem whose factors and edge matrices need more than that array
 * (256-aligned sizes: 8 bytes per factor entry, 8 + element size per W_ab
 * entry) returns IFCTN_E_UNSUPPORTED before touching the device.  Every call
 * on one GPU shares the one array and leaves its contents behind (nothing in
 * it has to start at zero): calls that overlap on the same GPU, from
 * different threads or streams, race and must be serialised by the caller. */
#define IFCTN_NOALLOC_SCRATCH_BYTES (16ull << 20)
ifctn_status ifctn_assemble_noalloc(const ifctn_params* params, const double* G_host, void* out_dev,
                                    void* stream);

/* Per-kernel timing with HIP events stamped with the start and end of every
 * launch of the given kernel class, on the stream it runs on (0 = mode-k
 * contraction, 1 = factor-block solve, 2 = X update, 3 = Gram weights or the
 * Gamma_k build, 4 = the U-row reduction of a Gamma-route block when Gamma_k
 * is built on the job's second stream).  enable = 1 starts a fresh tally,
 * 0 stops.  The query synchronises and returns the total milliseconds and
 * launch count since the tally started; an unknown class: IFCTN_E_INVAL. */
ifctn_status ifctn_timing_enable(ifctn_job* job, int32_t enable);
ifctn_status ifctn_timing_query(ifctn_job* job, int32_t kernel_class, double* total_ms,
                                int64_t* launches);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of completion requests on one GPU.
 *
 * A server owns a device pool of hbm_budget_bytes (allocated once at create)
 * and a scheduler thread.  Submitted requests wait in a FIFO queue and are
 * admitted when one of max_active slots is free and the pool has room for the
 * job's workspace (ifctn_workspace_bytes); a request needing more than the
 * whole budget is refused at submit.  Each resident job runs Algorithm 1
 * (t_max, eps, and for BF16_REFINE the float32 refinement sweeps, as in
 * ifctn_complete) in rounds of sweeps_per_round sweeps on one of num_streams
 * HIP streams, with the stop test on the device; jobs admitted while others
 * run overlap with them on the device.  A job runs the same kernels in the
 * same order as ifctn_complete, so its result does not depend on the mix.
 * ------------------------------------------------------------------------- */
typedef struct ifctn_server ifctn_server;

typedef struct {
  size_t hbm_budget_bytes;  /* device pool for resident jobs, allocated at create     */
  int32_t max_active;       /* jobs resident at once (slots), 1..1024                  */
  int32_t num_streams;      /* HIP streams the resident jobs are spread over, 1..16    */
  int32_t sweeps_per_round; /* sweeps issued per job between two looks at its flags, >= 1 */
  int32_t device;           /* HIP device ordinal the server runs on                   */
} ifctn_server_config;

typedef struct {
  ifctn_params params;
  const void* O_dev;        /* device, as for ifctn_init; complete before submit (the server's
                               streams do not wait for the caller's); the caller keeps it valid
                               until the request's completion has been polled                */
  const uint8_t* mask_dev;  /* device, same rules                                            */
  const double* G0_host;    /* packed initial factors; copied at submit                      */
  int32_t t_max;            /* sweeps (>= 0)                                                 */
  double eps;               /* stop tolerance (>= 0; 0 = exactly t_max sweeps)               */
  void* X_out_dev;          /* device, prod(dims) elements of the job's output dtype; written
                               before the completion is reported                             */
  uint64_t tag;             /* returned in the completion                                    */
} ifctn_request;

typedef struct {
  uint64_t tag;
  int32_t status;           /* ifctn_status of the request                                   */
  ifctn_stats stats;        /* as ifctn_complete's (valid when status == IFCTN_OK)          */
  double t_submit;          /* seconds since the server was created (steady clock)           */
  double t_admit;
  double t_done;
} ifctn_completion;

/* Create a server (allocates the pool and pinned host memory, starts the
 * scheduler thread).  IFCTN_E_NOMEM when the pool does not fit. */
ifctn_status ifctn_server_create(const ifctn_server_config* config, ifctn_server** out);

/* Queue a request.  Invalid params or pointers: IFCTN_E_INVAL; a workspace
 * larger than the whole budget: IFCTN_E_NOMEM (nothing is queued then). */
ifctn_status ifctn_server_submit(ifctn_server* server, const ifctn_request* request);

/* Move up to max finished requests into out (completion order); *n = count.
 * wait_ms > 0 waits up to that long for the first one. */
ifctn_status ifctn_server_poll(ifctn_server* server, ifctn_completion* out, int32_t max, int32_t* n,
                               int32_t wait_ms);

/* Requests still queued (not admitted) and finished ones not yet polled. */
ifctn_status ifctn_server_queued(ifctn_server* server, int32_t* queued, int32_t* completed_unpolled);

/* Stop admitting, drop queued requests, wait for resident jobs to finish and
 * release everything (NULL is accepted). */
ifctn_status ifctn_server_destroy(ifctn_server* server);

/* Image-quality metrics of Sec. 5 for an H x W x B tensor (row-major, bands
 * the last mode) against a reference of the same shape, both on the device in
 * float32 (precision = IFCTN_FP32) or float64 (IFCTN_FP64):
 *   PSNR_b = 10 log10(peak^2 / MSE_b) over all pixels of band b (+inf when
 *   the band is exact), MPSNR = mean over bands;
 *   SSIM_b = mean over the positions where an 11 x 11 Gaussian window
 *   (standard deviation 1.5, normalised) fits of
 *   ((2 mu_x mu_y + C1)(2 s_xy + C2)) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)),
 *   C1 = (0.01 peak)^2, C2 = (0.03 peak)^2 (Wang et al. 2004), MSSIM = mean over bands.
 * psnr_host / ssim_host (nullable) receive the B per-band values.  H and W must
 * be at least 11.  Allocates a small scratch buffer; synchronises the stream. */
ifctn_status ifctn_image_metrics(const void* X_dev, const void* ref_dev, int64_t H, int64_t W, int64_t B,
                                 int32_t precision, double peak, double* psnr_host, double* ssim_host,
                                 double* mpsnr, double* mssim, void* stream);

/* How each factor block of a job with these params would run (with the
 * options as they stand), one entry per mode k in out[0 .. order-1]:
 *   route: 0 = per-column solves with the Gram weights of eq. (updateG)
 *          computed in the contraction launch; 1 = the same in the phased
 *          form; 2 = the Gamma route (Gamma_k = Z_k^T Z_k of Prop. 1 built in
 *          a launch of its own, per-column H_j from it); 3 = the large-rank
 *          route (every block of a job with an edge rank above 8);
 *   gamma_fma: route 2 only, multiply-adds of building Gamma_k.
 * IFCTN_E_INVAL for invalid params or a NULL out. */
typedef struct {
  int32_t route;
  int32_t reserved;
  double gamma_fma;
} ifctn_block_plan;
ifctn_status ifctn_plan_blocks(const ifctn_params* params, ifctn_block_plan* out);

/* Process-wide tuning option, read when a job is created:
 *   "phased_min": a factor block uses the phased form (partial Gram matrices
 *   over ranges of the Gram weight set on many workgroups, then one
 *   workgroup per column for the solve) when one of its Gram weight sets
 *   holds at least this many entries; the one-workgroup-per-column form
 *   otherwise.  Both give the same solution of eq. (updateG) up to rounding.
 *   value < 0 restores the default (16384).
 *   "phased_onelaunch": 1 runs each sub-block of a phased block as one launch
 *   (the last workgroup of a column tile to finish its partial sums solves
 *   the tile's columns); default (value <= 0): two launches per sub-block.
 *   "merge_gram": 0 computes the Gram weights in a launch of their own
 *   instead of as extra workgroups of the contraction launch (default).
 *   "contract_div", "contract_emin": a contraction workgroup covers about
 *   max(contract_emin, nX / contract_div) tensor entries (defaults 1280 and
 *   4096; values <= 0 restore them).
 *   "contract_jmax": a contraction workgroup whose fibre or own mode is the
 *   contiguous one spans at most this many indices of mode k, and at most as
 *   many as eight accumulator slots per thread allow (default 8; values
 *   <= 0 restore it).
 * Unknown names: IFCTN_E_INVAL. */
ifctn_status ifctn_set_option(const char* name, int64_t value);
/*   "gamma": factor-block route -- 1 (default): the Gamma route for blocks
 *   that would otherwise take the phased form, 0: never, 2: wherever it fits.
 *   "overlap": 1 (default): in a job with Gamma-route blocks the mode-k
 *   contraction runs on a second stream of the job's own (default
 *   priority), concurrently with the Gamma_k build on the job's stream, and
 *   is joined by an event before the solve; 0: everything in line on the
 *   job's stream.  Jobs of a server always run in line.
 *   "ugroup": the contraction's partial slots are summed in groups of this
 *   many by the last workgroup of each group (default 0: off).
 *   "inject_admit_failures": the next `value` server admissions fail with
 *   IFCTN_E_NOMEM (fault injection for tests). */

/* Message of the last failed call on this thread ("" if none). */
const char* ifctn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* IFCTN_H */
