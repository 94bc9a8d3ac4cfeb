/*
 * cesmlmc -- MLMC level sampler with (smoothed) circulant embedding on
 * MI355X (gfx950).  C ABI.
 *
 * The operations follow Istratuca & Teckentrup, "Smoothed Circulant
 * Embedding with Applications to Multilevel Monte Carlo Methods for PDEs
 * with Random Coefficients":
 *   covariance model          Section 2.1, eqs. (matern-cov-function),
 *                             (p-norm-cov-function)
 *   embedding + eigenvalues   Section 2.1.2; Algorithm 1 steps 1-3
 *   padding / periodisation   Section 2.2, eq. (periodic-cov-fun)
 *   smoothing (tau dropped)   Section 2.4, eq. (tau-definition); Algorithm 2
 *   field sample              Algorithm 1 step 4(a)-(f)
 *   PDE and its discretisation Section 3.1 eq. (pde-model), Section 3.2
 *   level difference Y        Section 3.4 (Y_l = Q_{h_l} - Q_{h_{l-1}}),
 *                             eq. (mlmc-estimator-smoothed)
 *
 * Conventions
 *   - Every function returns an int status: CES_OK (0) or a negative
 *     CES_ERR_* code; ces_last_error() gives a message (thread-local).
 *   - No C++ types or exceptions cross this boundary.
 *   - "dev" pointers are device (HBM) pointers owned by the caller;
 *     "host" pointers are ordinary host memory owned by the caller.
 *   - hip_stream is a hipStream_t (NULL = the null stream).  Calls that
 *     take a stream only enqueue work unless stated otherwise.
 *   - Contexts and plans are created and destroyed by the library.  A
 *     context is used by one host thread at a time.  A plan is immutable
 *     after creation, apart from the lattice ces_plan_set_lattice attaches,
 *     and belongs to its context.
 *   - Nodal arrays are (m+1) x (m+1) with the x index fastest
 *     (p = i1 + (m+1) i2), the lexicographic order of Section 2.1.2.
 *   - Determinism: sample i of a plan is a pure function of
 *     (plan, seed, i); it does not depend on count, first_sample or
 *     batching.
 */
#ifndef CESMLMC_H
#define CESMLMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CES_OK = 0,
    CES_ERR_ARG = -1,     /* invalid argument (message says which)          */
    CES_ERR_NOT_PSD = -2, /* no nonnegative embedding within max_pad_factor */
    CES_ERR_NOMEM = -3,   /* device memory budget or allocation exhausted   */
    CES_ERR_NOCONV = -4,  /* a solve hit cg_max_iter (per-sample status)    */
    CES_ERR_DEVICE = -5,  /* HIP runtime error                              */
    CES_ERR_BUSY = -6
};

enum { CES_COV_MATERN = 0, CES_COV_SEPEXP = 1 };
/* SINGLE: Y = Q_f on mesh h = 1/m_fine.  PAIR: Y = Q_f - Q_c with the
 * coarse mesh 2h, both from one field sample (Algorithm 1 step 4(e)). */
enum { CES_LEVEL_SINGLE = 0, CES_LEVEL_PAIR = 1 };
/* Nonnegativity policy of Algorithm 1 step 3(a)-(b).  Accept iff
 * min Lambda >= -1e-13 max Lambda.  GROW pads J = 0, m/2, m while
 * 2(m+J) <= max_pad_factor m; CLAMP keeps J = 0 and zeroes negatives;
 * FAIL returns CES_ERR_NOT_PSD. */
enum { CES_PSD_GROW = 0, CES_PSD_CLAMP = 1, CES_PSD_FAIL = 2 };
/* Cutoff norm of the smooth periodisation (Section 2.2): EUCLID uses the
 * 2-norm with plateau sqrt(2) and kappa = 2 ell - sqrt(2); INF uses the
 * max-norm with plateau 1 and kappa = 2 ell - 1. */
enum { CES_PERIOD_EUCLID = 0, CES_PERIOD_INF = 1 };
/* PAIR: complex xi, one DFT gives samples 2q (real part) and 2q+1
 * (imaginary part).  HARTLEY: real xi, Z = Re v + Im v (Algorithm 1
 * step 4(d)), one DFT per sample. */
enum { CES_FIELD_PAIR = 0, CES_FIELD_HARTLEY = 1 };
/* FP64: field and multigrid in double.  MIXED: field and multigrid in
 * float, conjugate-gradient iterates, residual and QoI in double. */
enum { CES_PREC_FP64 = 0, CES_PREC_MIXED = 1 };
/* DIRICHLET0: u = 0 on the boundary.  FLOWCELL: u = 1 at x1 = 0, u = 0 at
 * x1 = 1, zero flux at x2 = 0 and x2 = 1 (Section 3.1). */
enum { CES_BC_DIRICHLET0 = 0, CES_BC_FLOWCELL = 1 };
/* QoIs of Sections 3.1 and 4 on the P1 solution: integral of u,
 * u(qoi_x, qoi_y), L2 norm, outward flux through x1 = 1. */
enum { CES_QOI_INTEGRAL = 0, CES_QOI_POINT = 1, CES_QOI_L2 = 2, CES_QOI_OUTFLUX = 3 };
/* Coarse field of a PAIR level.  RESTRICT: the fine embedding's field (with
 * tau_coarse) at the even nodes (Algorithm 1 step 4(e)).  EMBED: the
 * coarse mesh's own embedding, as a SINGLE plan of mesh 2h with tau_fine =
 * tau_coarse would set it up, driven by the fine normals of the nearest
 * signed frequencies: per axis, coarse index j (signed k = j or j - n_c,
 * period n_c 2h) takes the fine xi at round(k n_f / (2 n_c)) mod n_f (fine
 * period n_f h; ties upwards; the identity on signed frequencies when
 * n_f = 2 n_c).  The selection is injective when n_f >= 2 n_c, so the
 * coarse term has exactly the law of the next coarser level's fine term
 * and the smoothed estimator (eq. (mlmc-estimator-smoothed)) telescopes
 * exactly; plan creation fails with CES_ERR_ARG when n_f < 2 n_c (the
 * coarse mesh padded relatively more than the fine one). */
enum { CES_COUPLE_RESTRICT = 0, CES_COUPLE_EMBED = 1 };
/* Multigrid cycle of the CG preconditioner (the library's own solver for
 * Algorithm 1 step 4(g); the paper uses GMRES with ILU).  V: V(2,2) cycle.
 * W1: level 1 visited twice per cycle (two coarse corrections, the same
 * symmetric operator), fewer CG iterations for a few more launches per
 * iteration: faster where a call carries many samples, slower for one
 * sample per call.  AUTO: W1 for SINGLE levels whose length scale (lambda /
 * sqrt(2 nu) for Matern, lambda for SEPEXP) spans at least 8 fine cells, V
 * otherwise.  Meshes with m <= 16, and with m <= 32 for a QoI linear in
 * u, are solved directly (banded L D L^T in double); other meshes with
 * m = 32 solve with their own small-mesh cycle. */
enum { CES_CYCLE_AUTO = 0, CES_CYCLE_V = 1, CES_CYCLE_W1 = 2 };

typedef struct ces_context_s* ces_context;
typedef struct ces_plan_s* ces_plan;

/* One level of the estimator (problem statement of Sections 2.1, 3.1 and
 * 3.5).  Initialise with ces_level_desc_default(). */
typedef struct {
    int32_t struct_size;   /* sizeof(ces_level_desc) */
    int32_t cov_kind;      /* CES_COV_* */
    double nu;             /* Matern smoothness nu > 0 (ignored for SEPEXP) */
    double lambda;         /* length scale lambda > 0 */
    double sigma2;         /* marginal variance sigma^2 > 0 */
    int32_t m_fine;        /* intervals per side, h = 1/m_fine; power of two, 4..4096 */
    int32_t level_kind;    /* CES_LEVEL_*; PAIR needs m_fine >= 8 */
    int64_t tau_fine;      /* eigenvalues dropped for the fine-mesh field; -1 = n (sqrt(s)) */
    int64_t tau_coarse;    /* eigenvalues dropped for the coarse-mesh field; -1 = n.  A PAIR
                              level with tau_fine != tau_coarse draws two fields from one xi
                              and needs n <= 4096 (CES_ERR_ARG otherwise) */
    int32_t psd_policy;    /* CES_PSD_* */
    int32_t periodization; /* CES_PERIOD_* */
    int32_t max_pad_factor;/* cap on n / m_fine for GROW (2..4) */
    int32_t field_mode;    /* CES_FIELD_* */
    int32_t precision;     /* CES_PREC_* */
    int32_t bc;            /* CES_BC_* */
    int32_t qoi;           /* CES_QOI_* */
    int32_t coupling;      /* CES_COUPLE_* (PAIR levels; 0 otherwise) */
    double qoi_x, qoi_y;   /* point of CES_QOI_POINT */
    double f_value;        /* constant source term f */
    double cg_rtol;        /* stop when ||r||_2 <= cg_rtol ||r_0||_2 */
    int32_t cg_max_iter;   /* iteration cap per solve */
    uint32_t stream;       /* level tag: fourth Philox counter word */
    int32_t mg_cycle;      /* CES_CYCLE_* */
    int32_t reserved;      /* 0 */
} ces_level_desc;

typedef struct {
    int32_t n;             /* embedding size per axis, n = 2(m + J) */
    int32_t J;             /* padding */
    double lam_min;        /* min / max eigenvalue before clamping */
    double lam_max;
    int64_t n_clamped;     /* eigenvalues set to zero by the policy */
    int64_t tau_fine;      /* resolved drop counts */
    int64_t tau_coarse;
    double boundary_gap;   /* relative gap between the last kept and the first
                              dropped eigenvalue of the coarse mask (0 if tie) */
    int32_t mg_levels;     /* multigrid levels of the fine solve */
    int32_t n_coarse;      /* embedding size per axis of the coarse field (n unless EMBED) */
    size_t bytes_per_sample; /* device workspace per in-flight sample */
} ces_plan_info;

/* Fill *d with defaults: Matern nu=1/2, lambda=0.1, sigma2=1, m=32, SINGLE,
 * tau 0/0, GROW, EUCLID, pad 4, PAIR field, MIXED, DIRICHLET0, INTEGRAL at
 * (7/15, 7/15), f=1, rtol 1e-10, 500 iterations, stream 0. */
void ces_level_desc_default(ces_level_desc* d);

/* Bind to HIP device `device`.  mem_budget_bytes caps the library's own
 * workspace (0 = 90% of free device memory).  A plan's sample workspace,
 * allocated on its first sampling call, holds as many samples as fit in
 * 9 GiB or 64 samples, whichever is more (at most 8192; 65536 for
 * m <= 32), or in the size in MiB given by the environment variable
 * CESMLMC_WORKSPACE_MB, and within the budget.  A
 * request larger than the workspace runs in the fewest chunks that fit,
 * all of (nearly) equal size. */
int ces_context_create(int device, size_t mem_budget_bytes, ces_context* out);
int ces_context_destroy(ces_context ctx);

/* Algorithm 1 steps 1-3 (+ Algorithm 2 masks): covariance column, FP64 2-D
 * DFT on the device, nonnegativity policy, orbit symmetrisation, masks,
 * amplitudes sqrt(Lambda)/n.  Synchronous.  CES_ERR_NOT_PSD possible. */
int ces_plan_create(ces_context ctx, const ces_level_desc* desc, ces_plan* out);
int ces_plan_info_get(ces_plan plan, ces_plan_info* info);
int ces_plan_destroy(ces_plan plan);

/* Level samples i = first_sample .. first_sample+count-1 (Algorithm 1
 * step 4 per sample, Section 3.4 difference).  y_dev[t] = Y of sample
 * first_sample+t.  q_fine_dev, q_coarse_dev (Q_f, Q_c; Q_c = 0 for SINGLE),
 * iters_dev (CG iterations of the fine solve; meshes with m <= 16, and
 * with m <= 32 for a QoI linear in u (every QoI but L2), are solved
 * directly and report 1) and status_dev (0, or CES_ERR_NOCONV if
 * either solve hit cg_max_iter) may be NULL.
 * Asynchronous on hip_stream; the call returns once the work is enqueued
 * except for a bounded number of convergence polls. */
int ces_sample(ces_plan plan, uint64_t seed, uint64_t first_sample, int64_t count,
               double* y_dev, double* q_fine_dev, double* q_coarse_dev,
               int32_t* iters_dev, int32_t* status_dev, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ces_sample with every workspace buffer taken from one static device array
 * of 256 MiB per device (held from the library's load until the process
 * ends).  Arguments and outputs as for ces_sample, bit for bit the same
 * results.  Allocates nothing: the call zeroes the plan's part of the array
 * with a kernel, then enqueues the field, solve and finalize kernels on
 * hip_stream chunk by chunk (fine and coarse solves one after the other)
 * and returns once every solve's convergence has been read back.  All
 * calls on a device share the array, which keeps the last call's contents:
 * calls that overlap on one device (other streams or threads) race.
 * CES_ERR_ARG when one sample unit of the plan (two samples in PAIR field
 * mode) needs more workspace than the array holds (the message gives the
 * bytes; 2049^2 meshes do not fit); CES_ERR_BUSY when the plan is in use. */
int ces_sample_noalloc(ces_plan plan, uint64_t seed, uint64_t first_sample, int64_t count,
                       double* y_dev, double* q_fine_dev, double* q_coarse_dev,
                       int32_t* iters_dev, int32_t* status_dev, void* hip_stream);

/* ---- batches of levels of uneven size (MLMC rounds, served work) ------ */

/* One request: samples first_sample .. first_sample+count-1 of `plan`
 * with the outputs of ces_sample (device pointers; all but y may be NULL). */
typedef struct {
    ces_plan plan;
    uint64_t seed;
    uint64_t first_sample;
    int64_t count;
    double* y;
    double* q_fine;
    double* q_coarse;
    int32_t* iters;
    int32_t* status;
} ces_request;

/* Schedule of ces_sample and ces_sample_batch.  No field changes any
 * result (each sample's arithmetic is fixed by its plan); only the speed.
 *   depth          CG iterations of a solve enqueued ahead of its
 *                  convergence read-back, 1..4 (default 2)
 *   max_lanes      plans worked on concurrently, 0 = all (default 0)
 *   chunk_samples  samples per solver launch, 0 = the plan's workspace
 *                  capacity (default 0)
 *   graphs         1: each CG iteration of a tiled solve is replayed from a
 *                  captured HIP graph (one launch instead of about twelve);
 *                  0: launched kernel by kernel (default 0) */
typedef struct {
    int32_t depth;
    int32_t max_lanes;
    int64_t chunk_samples;
    int32_t graphs;
    int32_t reserved;
} ces_schedule;

/* Samples of every request, in one scheduled pass (the levels of an MLMC
 * estimator, Section 3.4, have meshes h_0 .. h_L and sample counts N_l of
 * very different sizes).  Each distinct plan is a lane with its own
 * streams, forked from hip_stream and joined back into it; a plan's
 * requests run one after another in its lane, lanes run concurrently, and
 * meshes with m <= 32 are solved in a single launch per chunk.  Every
 * output equals what ces_sample gives for that request alone, bit for bit.
 * A plan may appear in several requests but not in two concurrent calls
 * (CES_ERR_BUSY).  Returns once every solve's convergence has been seen;
 * the outputs are complete when hip_stream reaches the join. */
int ces_sample_batch(ces_context ctx, const ces_request* reqs, int32_t nreq, void* hip_stream);

int ces_schedule_get(ces_context ctx, ces_schedule* out);
/* Unset (zero) depth means 2. */
int ces_schedule_set(ces_context ctx, const ces_schedule* sched);

/* Autotuner: runs ces_sample_batch(reqs) under candidate schedules (each
 * run recomputes the same samples into the requests' outputs), keeps the
 * fastest as the context's schedule and returns it in *chosen and its
 * time in *best_ms (either may be NULL).  Synchronous.  When the
 * environment variable CESMLMC_AUTOTUNE_CACHE names a file, the choice is
 * appended to it under a key of the device architecture and, per distinct
 * plan, its descriptor and sample count in the batch; a later call with the
 * same key applies the stored choice and runs the batch once (its outputs
 * computed, *best_ms the stored time) instead of tuning again. */
int ces_autotune(ces_context ctx, const ces_request* reqs, int32_t nreq, void* hip_stream,
                 ces_schedule* chosen, double* best_ms);

/* ---- adaptive MLMC estimator on top of the sampler -------------------- */

/* Options of ces_mlmc_run.  Initialise with ces_mlmc_opts_default(). */
typedef struct {
    int32_t struct_size;   /* sizeof(ces_mlmc_opts) */
    double eps;            /* target root mean squared error */
    int32_t l_start;       /* levels 0..l_start are used from the start (>= 0) */
    int32_t reserved0;
    int64_t n_pilot;       /* first samples of a level newly added (>= 2) */
    double theta;          /* share of eps^2 for the estimator variance; the
                              paper's sample-size rule uses 1/2 */
    double alpha;          /* weak order for the bias estimate; <= 0: fitted */
    int32_t cost_model;    /* 0: cost of a level sample = unknowns of its
                              meshes; 1: measured device time per sample */
    int32_t max_rounds;    /* bound on sampling rounds */
    uint64_t seed;
} ces_mlmc_opts;

#define CES_MLMC_MAX_LEVELS 16

typedef struct {
    double estimate;       /* sum over levels of the sample mean of Y_l */
    double variance;       /* sum of V_l / N_l (estimator variance) */
    double bias;           /* |E[Y_L]| / (2^alpha - 1) (Richardson) */
    double alpha, beta, gamma;  /* fitted rates of |E[Y_l]|, V_l, C_l in h_l */
    int32_t levels;        /* L + 1 */
    int32_t converged;     /* 1: variance <= theta eps^2 and bias^2 <= (1-theta) eps^2 */
    int32_t rounds;
    int32_t reserved;
    int64_t n[CES_MLMC_MAX_LEVELS];      /* samples per level */
    double mean[CES_MLMC_MAX_LEVELS];    /* sample mean of Y_l */
    double var[CES_MLMC_MAX_LEVELS];     /* sample variance of Y_l */
    double cost[CES_MLMC_MAX_LEVELS];    /* cost per sample (model or seconds) */
} ces_mlmc_result;

void ces_mlmc_opts_default(ces_mlmc_opts* o);

/* Adaptive MLMC (Section 3.3, eq. (mlmc-estimator); smoothed form eq.
 * (mlmc-estimator-smoothed)).  levels[l] is the plan of level l: level 0 a
 * SINGLE plan on mesh h_0, level l >= 1 a PAIR plan on mesh h_0 / 2^l (its
 * coarse mesh is level l-1's).  finest (may be NULL) gives, per level, the
 * plan to use while that level is the finest one (the smoothed estimator
 * keeps the finest fine field unsmoothed); when a level stops being the
 * finest its samples are discarded and it is sampled again with
 * levels[l].  Each round samples, for every level in use,
 * the missing samples (sample indices continue per level, seed opts.seed)
 * in one ces_sample_batch call, updates the level means and variances, and
 * sets N_l = ceil(eps^-2 / theta * sqrt(V_l / C_l) * sum_k sqrt(V_k C_k))
 * (eq. (optimal-nl) with theta = 1/2).  When no level needs samples, the
 * bias |E[Q_h - Q]| is estimated by Richardson extrapolation with
 * extrapolant Q_2h, |E[Y_L]| / (2^alpha - 1) (Section 4); if its square
 * exceeds (1 - theta) eps^2 the next level is added (up to nlevels), else
 * the run has converged.  alpha, beta, gamma are least-squares slopes of
 * log2 |mean_l|, log2 V_l, log2 C_l against l over levels 1..L.
 * Levels must be independent: every level samples indices from 0 under
 * the one seed, so the level tags (desc.stream) of level l (levels[l] and
 * finest[l], which may share a tag) must differ from every other level's
 * (CES_ERR_ARG otherwise).  Synchronous; hip_stream orders the sampling. */
int ces_mlmc_run(ces_context ctx, const ces_plan* levels, const ces_plan* finest, int32_t nlevels,
                 const ces_mlmc_opts* opts, void* hip_stream, ces_mlmc_result* out);

/* ces_mlmc_run with a checkpoint (host file `path`, may be NULL): the run's
 * state after every round -- the level in use, per level the sample count,
 * Welford mean and sum of squared deviations, planned count, next sample
 * index and cost, the fitted rates and the stop flags -- is written as JSON
 * (17 significant digits, written to path.tmp and renamed).  If `path`
 * exists when the call starts, the run continues from it; a file written
 * for other options or plans is refused (CES_ERR_ARG).  max_new_rounds > 0
 * stops the call after that many rounds of its own (0: no limit), leaving
 * the state in the file.  Since every level sample is a pure function of
 * (plan, seed, index), a run resumed any number of times gives results bit
 * for bit those of an uninterrupted one (with cost_model 0: measured costs
 * are the resumed calls' own). */
int ces_mlmc_run_checkpointed(ces_context ctx, const ces_plan* levels, const ces_plan* finest, int32_t nlevels,
                              const ces_mlmc_opts* opts, const char* path, int32_t max_new_rounds,
                              void* hip_stream, ces_mlmc_result* out);

/* Coarsest mesh rule of Section 3.5, eq. (mlmc-h0-bound-matern-covariance)
 * and eq. (mlmc-h0-bound-exp-covariance): the largest h_0 = 2^-k with
 * h_0 <= sqrt(8 nu) lambda (Matern) or h_0 <= lambda (separable
 * exponential); returns m_0 = 1/h_0 in *m0. */
int ces_mlmc_coarsest_mesh(const ces_level_desc* desc, int32_t* m0);

/* ---- smoothing parameter and smoothing error -------------------------- */

/* Number of eigenvalues to drop on a mesh h = 1/m (Section 3.5): the
 * smoothing error bound of the covariance's corollary (separable
 * exponential: C_s tau / (s - tau + 1); Matern: eq. (tau-values-matern))
 * set equal to the discretisation error C_alpha h^alpha, with s = n^2 =
 * 4 (m + J)^2.  Separable exponential: closed form, eq.
 * (k-values-p-norm-cov) (needs J = 0: its classical embedding is
 * nonnegative).  Matern: the root of eq. (tau-values-matern) in [0, s] by
 * bisection (the left side increases strictly in tau); s when the right
 * side is at least s.  cs_over_calpha = C_s / C_alpha > 0 (constants of the
 * two bounds, from pilot runs), alpha > 0.  *tau = the root rounded to the
 * nearest integer; *tau_real (may be NULL) = the root.  Host only;
 * CES_ERR_ARG on invalid arguments. */
int ces_tau_rule(int32_t cov_kind, double nu, int32_t m, int32_t J, double alpha, double cs_over_calpha,
                 int64_t* tau, double* tau_real);

typedef struct {
    int32_t struct_size;   /* sizeof(ces_smoothing_stats), set by the caller */
    int32_t reserved;
    int64_t n;             /* samples */
    double mean;           /* sample mean of Q_h - Q~_h */
    double mean_abs;       /* sample mean of |Q_h - Q~_h| */
    double var;            /* sample variance of Q_h - Q~_h (n - 1 denominator) */
    double mean_q;         /* sample mean of Q_h */
    double mean_q_smoothed;/* sample mean of Q~_h */
} ces_smoothing_stats;

/* Smoothing error of one mesh (Section 4.1, the quantities E[Q_h - Q~_h]
 * and V[Q_h - Q~_h]; Corollaries (error-1-norm-cov), (error-matern-cov)):
 * `full` and `smoothed` are SINGLE plans that differ only in tau_fine
 * (same mesh, covariance, field mode, precision, PDE data and stream), so
 * sample i of `seed` draws the same normals in both and Q_h^(i) - Q~_h^(i)
 * is taken on one realisation of the field.  Samples first .. first+count-1
 * (count >= 2) of both plans run in one ces_sample_batch call; the
 * statistics are accumulated on the host in sample order.  Synchronous;
 * hip_stream orders the sampling. */
int ces_smoothing_error(ces_context ctx, ces_plan full, ces_plan smoothed, uint64_t seed, uint64_t first,
                        int64_t count, void* hip_stream, ces_smoothing_stats* out);

/* ---- randomised quasi-Monte Carlo (extension named in Section 5) ------ */

/* QMC drives the real (Hartley) factorisation of Sections 2.1.1-2.1.2 with
 * a randomly shifted rank-1 lattice rule instead of Philox normals on the s
 * eigen indices it is given; the other normals stay Philox ones.
 *   point i (radical-inverse order: the first 2^k points are the lattice
 *   rule with N = 2^k for every k) of shift r, coordinate j:
 *     U = (bitreverse64(i) * z_j + D_rj) mod 2^64,
 *     u = (floor(U / 2^12) + 1/2) 2^-52,    xi_{dims[j]} = Phi^-1(u),
 *   D_rj = x0 + 2^32 x1 of Philox4x32-10 with counter (j, r, 2^32-1,
 *   stream), key = the sampling seed.
 * Sample index g of a lattice plan is point g / R of shift g mod R, so the
 * first N R samples are N points of every shift. */

/* Generating vector by the component-by-component construction (Sloan,
 * Kuo and Joe, 2002) for N = 2^log2_points points: coordinate j takes the
 * odd z <= N/2 (z = 1 for N <= 2) minimising the shift-averaged worst-case
 * error of the weighted unanchored Sobolev space with product weights,
 *   e^2 = -1 + (1/N) sum_k prod_j (1 + gamma_j B2({k z_j / N})),
 *   B2(x) = x (x - 1) + 1/6,
 * given z_0..z_{j-1}; each candidate's sum takes every term truncated to a
 * multiple of 2^-40 and adds them exactly (result independent of the
 * summation order), ties to the smaller z.  gamma: s host doubles >= 0 with
 * sum <= 64; z: s host uint32 (out).  0 <= log2_points <= 20, s >= 1.
 * Host only (threads; O(s N^2 / 2)).  CES_ERR_ARG on invalid arguments. */
int ces_lattice_cbc(int32_t log2_points, int32_t s, const double* gamma, uint32_t* z);

/* The s eigen indices of the plan's fine embedding with the largest
 * eigenvalues (value descending, index ascending; clamped eigenvalues)
 * into dims (s host int64) and their values into lam (s host doubles, may
 * be NULL).  Needs the plan's eigenvalues (every plan made by
 * ces_plan_create keeps them). */
int ces_plan_lattice_order(ces_plan plan, int32_t s, int64_t* dims, double* lam);

/* Attach a lattice to a HARTLEY plan: s coordinates with generating vector
 * z (s host uint32, odd for every coordinate to be a permutation of the
 * points) on eigen indices dims (s distinct host int64 in [0, n^2); NULL =
 * ces_plan_lattice_order's), `shifts` >= 2 random shifts.  s = 0 detaches
 * (plain Monte Carlo again).  Every later sampling call on the plan (and
 * the coarse field of an EMBED pair) uses it; sample indices must stay
 * below 2^63.  Not concurrent with sampling on the plan (CES_ERR_BUSY).
 * CES_ERR_ARG: not HARTLEY, s out of [0, n^2], repeated or out-of-range
 * dims, shifts < 2. */
int ces_plan_set_lattice(ces_plan plan, int32_t s, const uint32_t* z, const int64_t* dims, int32_t shifts);

/* ces_plan_lattice_order + weights gamma_j = lam_j / sum lam (the
 * eigenvalues of the chosen indices, scaled to sum 1) + ces_lattice_cbc +
 * ces_plan_set_lattice. */
int ces_plan_set_lattice_default(ces_plan plan, int32_t s, int32_t log2_points, int32_t shifts);

typedef struct {
    int32_t struct_size;   /* sizeof(ces_mlqmc_opts) */
    int32_t l_start;       /* levels 0..l_start are used from the start (>= 0) */
    double eps;            /* target root mean squared error */
    int64_t n_pilot;       /* points per shift of a level newly added (>= 1) */
    double theta;          /* share of eps^2 for the estimator variance */
    double alpha;          /* weak order for the bias estimate; <= 0: fitted */
    int32_t cost_model;    /* 0: unknowns of the level's solves, 1: measured */
    int32_t max_rounds;    /* bound on sampling rounds */
    uint64_t seed;
} ces_mlqmc_opts;

void ces_mlqmc_opts_default(ces_mlqmc_opts* o);

/* Multilevel QMC (Giles and Waterhouse, 2009) over lattice plans (every
 * plan in levels and finest has a lattice; all share one shift count R).
 * Level l holds N_l points of each of the R shifts (samples 0 .. N_l R - 1);
 * its estimate is the mean of the R shift averages and V_l their sample
 * variance / R.  Each round samples what is missing on every level in use
 * in one ces_sample_batch call (per-shift sums add samples in index
 * order), then, while sum_l V_l > theta eps^2 with V_l halved per planned
 * doubling, doubles N_l of the level with the largest V_l / (C_l N_l)
 * (ties: the lower level).  When nothing is to be sampled the bias and the
 * addition of levels follow ces_mlmc_run (Richardson, alpha fitted over
 * levels 1..L when L >= 2, else 1).  out: n[l] = N_l R, mean[l] the level
 * estimate, var[l] the variance of the shift averages (R - 1 denominator),
 * variance = sum var[l] / R.  Level tags as for ces_mlmc_run.
 * Synchronous. */
int ces_mlqmc_run(ces_context ctx, const ces_plan* levels, const ces_plan* finest, int32_t nlevels,
                  const ces_mlqmc_opts* opts, void* hip_stream, ces_mlmc_result* out);

/* ---- serving: continuous batching with memory admission -------------- */

/* A server owns a host thread that plans, admits and runs requests as they
 * arrive.  Each request is one level descriptor (its own covariance, mesh,
 * precision ...) with a seed and a sample range; its results are written
 * to caller-owned host memory.  Requests with identical descriptors share
 * one plan.  Set-up (ces_plan_create's work) runs on a planner thread; a
 * planned request is admitted when its device memory (workspace sized for
 * its sample count, plus outputs) fits within mem_budget_bytes next to the
 * admitted ones and fewer than max_inflight are admitted; admitted
 * requests join the running batch at once (no waiting for a round to end)
 * and leave it as they complete.  Y of a request equals what ces_sample
 * returns for the same descriptor, seed and range, bit for bit.  Device
 * memory comes from a caching pool owned by the server. */
typedef struct ces_server_s* ces_server;

typedef struct {
    int64_t submitted;     /* requests accepted by ces_server_submit */
    int64_t completed;     /* requests whose results are in host memory */
    int64_t failed;        /* requests that ended with an error */
    int64_t queued;        /* submitted, not yet admitted */
    int64_t admitted;      /* admitted, not yet complete */
    int64_t samples_done;  /* level samples of completed requests */
    size_t mem_in_use;     /* device bytes of the server's pool in use */
    size_t mem_peak;       /* largest mem_in_use seen */
    int32_t plans_cached;  /* plans alive (shared by identical descriptors) */
    int32_t reserved;
} ces_server_stats;

/* mem_budget_bytes = 0: 90% of the context's budget.  max_inflight <= 0:
 * 64.  The context must outlive the server and may be used by its owner
 * thread meanwhile (the server has its own streams and memory pool). */
int ces_server_create(ces_context ctx, size_t mem_budget_bytes, int32_t max_inflight, ces_server* out);

/* Queue a request; returns at once.  y_host (count doubles) and status_host
 * (count int32, may be NULL) must stay valid until the request is done.
 * The descriptor is copied; invalid descriptors fail here (CES_ERR_ARG). */
int ces_server_submit(ces_server srv, const ces_level_desc* desc, uint64_t seed, uint64_t first_sample,
                      int64_t count, double* y_host, int32_t* status_host, int64_t* request_id);

/* *state: 0 queued, 1 admitted, 2 done (results in host memory), or a
 * negative CES_ERR_* code.  *latency_s (may be NULL): submit to completion
 * for done requests, time since submit otherwise. */
int ces_server_poll(ces_server srv, int64_t request_id, int32_t* state, double* latency_s);

/* Block until every request submitted so far is done or failed. */
int ces_server_drain(ces_server srv);

int ces_server_get_stats(ces_server srv, ces_server_stats* out);

/* Drain, stop the threads, free the plans and the memory pool. */
int ces_server_destroy(ces_server srv);

/* ---- parity hooks (same kernels as ces_sample) ------------------------ */

/* Box-Muller normals of Philox counter (e, q mod 2^32, q >> 32, stream),
 * key = seed, for e = first_e .. first_e+count-1: out_dev[2t] = g0,
 * out_dev[2t+1] = g1. */
int ces_normals(uint64_t seed, uint64_t q, uint32_t stream, uint64_t first_e, int64_t count,
                double* out_dev, void* hip_stream);

/* Symmetrised eigenvalues (n*n doubles, after clamping) into host memory. */
int ces_plan_eigenvalues(ces_plan plan, double* host_out);

/* Masks (1 = kept) of the fine field (n*n bytes) and of the coarse field
 * (n*n bytes of the fine embedding; for EMBED pairs n_coarse*n_coarse bytes
 * of the coarse embedding, see ces_plan_info); either may be NULL. */
int ces_plan_mask(ces_plan plan, uint8_t* host_fine, uint8_t* host_coarse);

/* Gaussian fields Z (before exp) of sample `sample`: z_fine_dev gets
 * (m+1)^2 doubles, z_coarse_dev (m/2+1)^2 doubles (PAIR plans; may be NULL). */
int ces_field(ces_plan plan, uint64_t seed, uint64_t sample, double* z_fine_dev,
              double* z_coarse_dev, void* hip_stream);

/* Solve -div(k grad u) = f with the plan's boundary condition on the fine
 * (grid = 0, m = m_fine) or coarse (grid = 1, m = m_fine/2) mesh for
 * `count` coefficient arrays k_dev (count x (m+1)^2 doubles, k > 0).
 * u_dev receives count x (m+1)^2 doubles (boundary values included);
 * iters_dev (may be NULL) the CG iterations, negative if not converged. */
int ces_solve(ces_plan plan, int32_t grid, int64_t count, const double* k_dev, double* u_dev,
              int32_t* iters_dev, void* hip_stream);

/* ---- launch profiler (bench and roofline reporting) ------------------ */

/* Per-kernel aggregate since the last read: HIP-event time summed over
 * launches, and the algorithmic bytes those launches move (inputs read
 * once, outputs written once; samples already converged are not counted). */
typedef struct {
    char name[48];
    int64_t launches;
    double total_ms;
    double bytes;
} ces_profile_entry;

/* Process-wide.  on != 0 starts recording HIP events around every library
 * kernel launch (clearing earlier records); on == 0 stops. */
int ces_profile_enable(int32_t on);

/* Process-wide.  Restricts the recording to launches of the kernel with
 * this profile name (as ces_profile_read reports it, e.g. "pcg_dir"), so
 * that a timed region pays the HIP events of that kernel's launches only;
 * NULL or "" records every kernel again.  The name is copied.  Kept across
 * ces_profile_enable calls. */
int ces_profile_only(const char* name);

/* Synchronises with the recorded launches, writes up to max_entries
 * entries (largest total time first) to host memory and the number of
 * kernels to *n_entries, then clears the records. */
int ces_profile_read(ces_profile_entry* out, int32_t max_entries, int32_t* n_entries);

const char* ces_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CESMLMC_H */
