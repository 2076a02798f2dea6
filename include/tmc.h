/*
 * tmc.h -- C ABI of libtmc, the MI355X (gfx950) Tensor Monte Carlo chain estimator.
 *
 * Paper: L. Aitchison, "Tensor Monte Carlo: Particle Methods for the GPU Era",
 * arXiv 1806.08593.
 *
 * What the library computes.  For each of n_chains independent chains of latent
 * layers 0..L-1 (layer 0 is adjacent to the data, layer L-1 is the top), with K_l
 * samples z_l^k of layer l drawn from a proposal, the TMC estimate of eq. (is)
 * (Sec. "TMC for factorised proposals"):
 *
 *   log P_TMC = log [ 1/prod_l K_l * sum_{k_0..k_{L-1}}
 *                     exp( sum_l u_l[k_l] + sum_{l<L-1} f_l[k_l, k_{l+1}] ) ]
 *
 * where the importance ratio has been factorised as in eq. (fac) and the Appendix
 * "Typical choice of factors":
 *   u_l[k]       unary log-terms supplied by the caller: -log Q(z_l^k), plus the
 *                log-likelihood log P(x | z_0^k) on layer 0 and the log-prior of the
 *                top layer on layer L-1 (a non-factorised proposal of Sec.
 *                "Non-factorised proposals" also enters here: it is indexed by k_l only);
 *   f_l[i, j]    the pairwise log-factor log P(z_l^i | z_{l+1}^j).
 * The sum is evaluated by summing out one index at a time (Sec. "Efficient
 * averaging"), each step a log-domain matrix-vector product (Appendix "Numerically
 * stable matrix (tensor) products in the log-domain").
 *
 * Three families of entry points:
 *   tmc_gauss_*      the chained diagonal-Gaussian model of Sec. "Computational costs
 *                    for TMC and IWAE": f_l[i,j] = log N(z_l^i; mu_l^j, diag exp(2 s_l)),
 *                    where mu_l^j (the conditional mean produced by the caller's network
 *                    from parent sample z_{l+1}^j) and s_l (log standard deviation,
 *                    shared by all parent samples) are inputs.  Gradients with respect
 *                    to z, mu, s and u are returned for reparameterised training.
 *   tmc_logfactor_*  any chain whose log-factors f_l are supplied as dense matrices
 *                    (e.g. the exact discrete marginalisation of the Appendix).
 *   tmc_star_*       not a chain: one global latent shared by many local latents (the
 *                    latent-variable model of Sec. "Efficient averaging"), below.
 * and the log-domain matrix product itself (tmc_logmmexp).
 *
 * Memory.  Every data pointer is DEVICE memory on the plan's device unless marked
 * (host).  The caller allocates and owns every buffer, including the workspace; the
 * library owns only its plans (descriptor tables, tuned tile choices, graphs).
 * Execute calls never allocate and never synchronise, so they may be captured into
 * a hipGraph by the caller.  Inputs are never written.  Outputs are overwritten.
 *
 * Layout.  Buffers are flat arrays; the problem descriptor gives the element
 * offset of each layer's block.  Row-major:
 *   z  : z_l    [K_l][D_l]        at layers[l].z_off
 *   mu : mu_l   [K_{l+1}][D_l]    at layers[l].mu_off  (row j = mean given z_{l+1}^j)
 *   s  : s_l    [D_l]             at layers[l].s_off   (several layers may share one;
 *                                 [K_{l+1}][D_l] with TMC_FLAG_PARENT_SCALE)
 *   u  : u_l    [K_l]             at layers[l].u_off
 *   f  : f_l    [K_l][K_{l+1}]    at layers[l].f_off
 * Gradient buffers use the same offsets as the matching input.  Element type is
 * double in TMC_FP64 mode and float otherwise; log P and its upstream gradient
 * are always double, one per chain.
 *
 * Errors.  Every call returns a status synchronously (validation and enqueue
 * failures); tmc_last_error() gives the calling thread's last message.  No C++
 * exception crosses this interface.  NaN inputs give NaN outputs; a chain whose
 * weights are all zero (every term -inf) gives log P = -inf, never NaN.
 *
 * Threads.  Distinct plans may be used concurrently; one plan must not be used by
 * two threads or two streams at the same time (its workspace layout and device
 * tables are shared by its calls).
 */
#ifndef TMC_H_
#define TMC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TMC_ABI_VERSION 6

typedef enum tmc_status {
  TMC_OK = 0,
  TMC_ERR_INVALID_ARG = 1,   /* null pointer, bad enum, inconsistent descriptor */
  TMC_ERR_SHAPE = 2,         /* K or D out of the supported range */
  TMC_ERR_WORKSPACE = 3,     /* workspace missing or misaligned */
  TMC_ERR_UNSUPPORTED = 4,   /* valid request the chosen engine cannot run */
  TMC_ERR_HIP = 5,           /* a HIP runtime call failed (message has the HIP error) */
  TMC_ERR_NUMERIC = 6,       /* device flagged a non-finite log P (tmc_plan_check) */
  TMC_ERR_STATE = 7          /* call order violated (e.g. backward without forward) */
} tmc_status;

/* Arithmetic of the O(K^2) per-entry work.  The O(K) per-row and per-layer
 * bookkeeping (row/column constants, message offsets, log P) is FP64 in all modes. */
typedef enum tmc_precision {
  TMC_FP64 = 0,     /* all per-entry arithmetic in double */
  TMC_FP32 = 1,     /* factor GEMM on FP32 MFMA, log-sum-exp in float */
  TMC_BF16X3 = 2    /* factor GEMM on BF16 MFMA with FP32 accumulation, operands split
                       into bf16 hi+lo parts and summed as hi*hi + hi*lo + lo*hi;
                       log-sum-exp in float */
} tmc_precision;

typedef enum tmc_engine {
  TMC_ENGINE_AUTO = 0,    /* fused for FP32/BF16X3, plain for FP64 */
  TMC_ENGINE_FUSED = 1,   /* factors recomputed on MFMA inside the message kernels,
                             never stored (FP32, BF16X3) */
  TMC_ENGINE_PLAIN = 2    /* factors materialised in the workspace, then streamed by
                             the log-sum-exp kernels (FP64, FP32) */
} tmc_engine;

/* Problem flags. */
#define TMC_FLAG_FORWARD_ONLY 1  /* no backward will follow: the fused forward skips
                                    the work it does only for gradients */
#define TMC_FLAG_PERSISTENT 2    /* fused engine: run each pass as one persistent
                                    launch per width bucket over a queue of whole
                                    chains instead of one launch per chain depth */
#define TMC_FLAG_PARENT_SCALE 4  /* parent-dependent scales: the general conditional of
                                    Sec. "Computational costs for TMC and IWAE",
                                    N(z_l; mu(z_{l+1}), diag sigma(z_{l+1})^2), whose
                                    standard deviation, like its mean, is produced from
                                    the parent sample.  Every s_l block is then
                                    [K_{l+1}][D_l] (row j: log standard deviation given
                                    parent sample j, the layout of mu_l), blocks of
                                    different layers may not overlap, and ds has the same
                                    layout.  Plain engine (TMC_FP64, TMC_FP32); the auto
                                    engine picks it, TMC_ENGINE_FUSED is rejected. */

/* One latent layer of one chain (host struct). */
typedef struct tmc_layer {
  int32_t K;       /* samples of this layer, >= 1 */
  int32_t D;       /* dimension of z_l (and of mu_l, s_l), >= 1 (gauss entry points) */
  int64_t z_off;   /* element offset of z_l [K][D]; not read for the top layer */
  int64_t u_off;   /* element offset of u_l [K] */
  int64_t mu_off;  /* element offset of mu_l [K_{l+1}][D]; ignored for the top layer */
  int64_t s_off;   /* element offset of s_l [D] ([K_{l+1}][D] with TMC_FLAG_PARENT_SCALE);
                      ignored for the top layer.  Layers (of any chains) may share a [D]
                      block; their ds is then summed. */
  int64_t f_off;   /* element offset of f_l [K][K_{l+1}] (logfactor entry points);
                      ignored for the top layer */
} tmc_layer;

/* One chain (host struct): layers[first_layer .. first_layer + n_layers - 1],
 * ordered from the layer next to the data (0) to the top. */
typedef struct tmc_chain {
  int32_t n_layers;
  int32_t first_layer;
} tmc_chain;

typedef struct tmc_problem {
  int32_t n_chains;
  int32_t n_layers;             /* length of layers[] */
  const tmc_chain* chains;      /* (host) n_chains entries */
  const tmc_layer* layers;      /* (host) n_layers entries */
  int32_t precision;            /* tmc_precision */
  int32_t engine;               /* tmc_engine */
  int32_t flags;                /* TMC_FLAG_* */
  int32_t reserved;             /* must be 0 */
  double exponent;              /* kappa: every importance weight enters raised to the power
                                   kappa, i.e. log P = log [1/prod_l K_l sum exp(kappa (sum u +
                                   sum f))] and its gradients; 2 gives the squared weights of
                                   the DReGs surrogate (Appendix "Combining DReGs and TMC").
                                   0 (a zero-initialised struct) means 1; otherwise finite
                                   and > 0.  Applies to every execute call of the plan
                                   (tmc_gauss_factors writes the unscaled factors). */
} tmc_problem;

typedef struct tmc_plan* tmc_plan_t;

/* Summary of a plan (host struct filled by tmc_plan_info). */
typedef struct tmc_plan_info {
  int64_t factor_entries;       /* sum over chains and layer pairs of K_l * K_{l+1} */
  int64_t workspace_bytes;
  int32_t engine;               /* engine actually used */
  int32_t precision;
  int32_t max_depth;            /* max chain length L */
  int32_t tile_rows;            /* fused engine: rows per workgroup tile */
  int32_t tile_cols;            /* fused engine: columns per inner tile */
  int32_t waves_per_group;      /* fused engine: waves of the widest per-depth workgroup (4, 8) */
  int32_t persistent;           /* fused engine: passes run as persistent launches */
  int32_t tuned;                /* launch shape chosen by tmc_plan_autotune or its cache */
  int32_t wide_fwd;             /* fused per-depth forward: 8-wave groups where eligible */
  int32_t wide_bwd;             /* fused per-depth backward: 8-wave groups where eligible */
} tmc_plan_info;

/* ---- library ---- */
int tmc_abi_version(void);
const char* tmc_status_string(tmc_status status);
/* Last error message of the calling thread ("" if none).  Valid until the next call
 * on this thread. */
const char* tmc_last_error(void);

/* ---- plans ---- */
/* Validates the problem, lays out the workspace, picks tile shapes (tuned table or
 * defaults) and uploads the descriptor tables to `device`.  Allocates device memory
 * for those tables (the only allocation the library makes).  Errors:
 * TMC_ERR_INVALID_ARG (null/bad descriptor, overlapping output ranges, partially
 * overlapping s blocks), TMC_ERR_SHAPE (K or D outside the engine's limits),
 * TMC_ERR_UNSUPPORTED (engine/precision combination not provided),
 * TMC_ERR_HIP. */
tmc_status tmc_plan_create(const tmc_problem* problem, int device, tmc_plan_t* out);
tmc_status tmc_plan_destroy(tmc_plan_t plan);
/* Bytes of device workspace every execute call of this plan needs (256-byte
 * aligned pointer required).  The forward leaves in it what the backward reads, so
 * a backward must use the workspace of the forward it differentiates. */
tmc_status tmc_plan_workspace_size(tmc_plan_t plan, size_t* bytes);
tmc_status tmc_plan_info_get(tmc_plan_t plan, tmc_plan_info* out);
/* Synchronises `stream` (a hipStream_t, NULL = default stream) and reports device
 * flags raised since the last check: TMC_ERR_NUMERIC if some log P was NaN or +inf. */
tmc_status tmc_plan_check(tmc_plan_t plan, void* stream);

/* ---- Gaussian chain (Sec. "Computational costs for TMC and IWAE") ---- */
/* Forward: logp[c] (double, n_chains) = log P_TMC of chain c.  Enqueued on `stream`
 * (hipStream_t).  Workspace receives the messages the backward needs. */
tmc_status tmc_gauss_fwd(tmc_plan_t plan, const void* z, const void* mu, const void* s,
                         const void* u, double* logp, void* workspace, void* stream);
/* Backward: given dlogp[c] (double, upstream gradient of each chain's log P), writes
 * dz (dz of every top layer is 0), dmu, ds (summed over layers sharing an s block)
 * and du.  Reads the workspace left by the matching tmc_gauss_fwd; z, mu, s, u must
 * be unchanged since that forward.  Any gradient pointer may be NULL to skip it. */
tmc_status tmc_gauss_bwd(tmc_plan_t plan, const void* z, const void* mu, const void* s,
                         const void* u, const double* dlogp, void* workspace,
                         void* dz, void* dmu, void* ds, void* du, void* stream);
/* Allocation-free forward, for callers that cannot allocate device memory (code
 * under hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * tmc_gauss_fwd with the workspace taken from a device array the library holds for
 * the life of the process, TMC_NOALLOC_WORKSPACE_MAX bytes on each GPU it runs on
 * (looked up once per device when the first plan on that device is created).  The
 * caller still passes inputs and the logp output; the call allocates and frees
 * nothing and does not synchronise.  Same results as tmc_gauss_fwd (the same
 * kernels).  Errors: TMC_ERR_WORKSPACE if the plan needs a larger workspace than
 * TMC_NOALLOC_WORKSPACE_MAX (tmc_plan_workspace_size; forward-only plans need the
 * least), TMC_ERR_HIP if the array's address could not be obtained, otherwise as
 * tmc_gauss_fwd.  Every call on one GPU shares that GPU's array, which keeps the last
 * call's contents (nothing in it has to start at zero: the forward initialises what it
 * reads): calls that overlap on one GPU -- on different streams or from different
 * threads -- race, and a tmc_gauss_bwd cannot use the state this call leaves. */
#define TMC_NOALLOC_WORKSPACE_MAX ((size_t)64 << 20)
tmc_status tmc_gauss_fwd_noalloc(tmc_plan_t plan, const void* z, const void* mu, const void* s,
                                 const void* u, double* logp, void* stream);
/* Writes the pairwise log-factors f_l [K_l][K_{l+1}] (at layers[l].f_off of `f`) by
 * direct difference in the plan's precision (FP64 or FP32).  For inspection and for
 * feeding tmc_logfactor_*; the fused engine never materialises them. */
tmc_status tmc_gauss_factors(tmc_plan_t plan, const void* z, const void* mu, const void* s,
                             void* f, void* stream);

/* ---- Chains with caller-supplied log-factors ---- */
tmc_status tmc_logfactor_fwd(tmc_plan_t plan, const void* f, const void* u, double* logp,
                             void* workspace, void* stream);
/* df_l[i,j] = dlogp * d log P / d f_l[i,j] (the pairwise posterior marginal over sample
 * indices), du_l[k] = dlogp * d log P / d u_l[k].  df or du may be NULL. */
tmc_status tmc_logfactor_bwd(tmc_plan_t plan, const void* f, const void* u,
                             const double* dlogp, void* workspace, void* df, void* du,
                             void* stream);

/* ---- Star model: a global latent shared by N local latents ---- */
/* The latent-variable model of Sec. "Efficient averaging" (its factor graph figure):
 * a global latent theta with K_theta samples and, for each of N data points, a local
 * latent z_i with K samples whose conditional depends on theta,
 *
 *   log P_TMC = log [ 1/(K_theta K^N) sum_{kt, k_1..k_N}
 *                     exp( uth[kt] + sum_i (u_i[k_i] + f_i[kt, k_i]) ) ]
 *             = logsumexp_kt( uth[kt] + sum_i m_i[kt] ) - ln K_theta,
 *   m_i[kt]   = logsumexp_k( u_i[k] + f_i[kt, k] ) - ln K,
 *
 * with f_i[kt, k] = log N(z_i^k; mth^kt, diag exp(2 s)): mth^kt is the mean of every
 * local latent given global sample kt (produced by the caller from theta^kt), s the log
 * standard deviation.  uth[kt] holds log P(theta^kt) - log Q(theta^kt); u_i[k] holds
 * log P(x_i | z_i^k) - log Q(z_i^k).  The Gaussian example of Sec. "Comparing TMC, SMC
 * and IWAE" is D = 1, mth^kt = theta^kt, s = 0.
 * n_instances independent models of the same shape are evaluated together.
 * Layout (row-major, element type double for TMC_FP64 and float for TMC_FP32):
 *   mth [S][K_theta][D], s [S][D], z [S][N][K][D], u [S][N][K], uth [S][K_theta],
 * S = n_instances; logp and dlogp are double [S].  The plan is a tmc_plan_t: destroy,
 * workspace size, info (factor_entries = S N K_theta K), check and timing calls apply;
 * the chain entry points reject it, and the star entry points reject chain plans. */
typedef struct tmc_star_problem {
  int32_t n_instances;  /* S >= 1 */
  int32_t N;            /* data points (local latents) per instance, >= 1 */
  int32_t K_theta;      /* samples of the global latent, 1 .. 4194304 */
  int32_t K;            /* samples of each local latent, 1 .. 4194304 */
  int32_t D;            /* dimension of each local latent, 1 .. 32 */
  int32_t precision;    /* TMC_FP64 or TMC_FP32 (per-entry arithmetic; sums over rows,
                           messages and log P are double) */
  int32_t flags;        /* 0 or TMC_FLAG_FORWARD_ONLY (smaller workspace, no backward) */
  int32_t reserved;     /* must be 0 */
} tmc_star_problem;

/* Errors: TMC_ERR_INVALID_ARG (null, bad flags or precision, S N or S K_theta D too
 * large for one launch grid), TMC_ERR_SHAPE (N, K, K_theta or D out of range),
 * TMC_ERR_UNSUPPORTED (TMC_BF16X3: the factors of such low-dimensional latents are not
 * a contraction worth the matrix cores), TMC_ERR_HIP. */
tmc_status tmc_star_plan_create(const tmc_star_problem* problem, int device, tmc_plan_t* out);
/* Forward: logp[S].  The workspace receives the messages and weights the backward reads. */
tmc_status tmc_star_gauss_fwd(tmc_plan_t plan, const void* mth, const void* s, const void* z,
                              const void* u, const void* uth, double* logp, void* workspace,
                              void* stream);
/* Backward: given dlogp[S], writes dmth [S][K_theta][D], ds [S][D], dz [S][N][K][D],
 * du [S][N][K] and duth [S][K_theta] (each dlogp times the derivative of log P; any may
 * be NULL to skip it).  Reads the workspace of the matching forward; mth, s, z, u must be
 * unchanged since.  Sums over points and samples run in a fixed order (deterministic). */
tmc_status tmc_star_gauss_bwd(tmc_plan_t plan, const void* mth, const void* s, const void* z,
                              const void* u, const double* dlogp, void* workspace, void* dmth,
                              void* ds, void* dz, void* du, void* duth, void* stream);

/* ---- Log-domain matrix product ---- */
/* The Appendix "Numerically stable matrix (tensor) products in the log-domain" in its
 * matrix-matrix form (what loopy graphs, and the messages of several chains at once,
 * contract: Sec. "Efficient averaging"): for b < batch,
 *   Z_b[i,k] = log sum_j exp(X_b[i,j] + Y_b[j,k]),
 * X [batch][M][K], Y [batch][K][N], Z [batch][M][N], row-major device buffers of double
 * (TMC_FP64) or float (TMC_FP32, TMC_BF16X3).  The Appendix's shift by the row maxima of X
 * and the column maxima of Y, the shifted exponentials multiplied on the matrix cores
 * (FP64 MFMA, FP32 MFMA, or BF16 hi/lo products as for the Gaussian factors), then every
 * entry whose shifted product fell below e^-600 (TMC_FP64) or e^-60 (the others) --
 * where the shift underflows: the maxima of X's row and Y's column at indices j far
 * apart -- recomputed exactly, with its own maximum over j, on the vector ALU.  All -inf
 * rows or columns give -inf; NaN propagates; +inf inputs give NaN.  The workspace holds
 * the shifts and the prepared operands: tmc_logmmexp_workspace_size bytes (every
 * precision), 256-byte aligned.  No plan: the call validates, enqueues on `stream` and
 * returns.  Errors: TMC_ERR_SHAPE (batch or M outside [1, 65535], K or N outside
 * [1, 2^24]), TMC_ERR_INVALID_ARG (NULL pointer, unknown precision), TMC_ERR_WORKSPACE,
 * TMC_ERR_HIP. */
tmc_status tmc_logmmexp_workspace_size(int32_t batch, int32_t M, int32_t K, int32_t N,
                                       int32_t precision, size_t* bytes);
tmc_status tmc_logmmexp(int32_t batch, int32_t M, int32_t K, int32_t N, int32_t precision,
                        const void* X, const void* Y, void* Z, void* workspace, void* stream);

/* ---- graphs ---- */
/* Record the enqueue of one execute call (same arguments as the call) into a hipGraph
 * owned by the plan; which = 0 forward, 1 backward.  The pointers are baked into the
 * graph.  Replay with tmc_plan_graph_launch. */
tmc_status tmc_plan_graph_capture_gauss(tmc_plan_t plan, int which, const void* z,
                                        const void* mu, const void* s, const void* u,
                                        double* logp, const double* dlogp, void* workspace,
                                        void* dz, void* dmu, void* ds, void* du,
                                        void* stream);
tmc_status tmc_plan_graph_launch(tmc_plan_t plan, int which, void* stream);

/* ---- launch shape ---- */
/* Batching of many chains of uneven depth and width (fused engine).  By default each
 * pass launches one kernel per chain depth and width bucket, over all chains at that
 * depth (a workgroup of 4 waves per block of 128 samples of one layer pair; in the
 * forward of gradient plans, 8 waves per 256 samples for widths d = 97..128).  With
 * TMC_FLAG_PERSISTENT (or when the tuner picks it) each pass is one persistent launch
 * per width bucket: its workgroups take whole chains from a queue in the workspace,
 * most expensive chain (sum of K_l K_{l+1} D_l) first, and each runs every layer pair
 * of its chain in order (top-down in the forward, bottom-up in the backward), so no
 * launch boundary separates the depths and no workgroup waits for another. */

/* Launch-shape tuner: runs every candidate launch shape of a fused plan (per-depth
 * launches, for gradient plans with or without 8-wave workgroups of 256 rows / columns
 * in each direction where the width allows; persistent launches with 1x or 2x the
 * resident workgroup capacity; for forward-only plans, 1 or 2 staged 32-sample subtiles
 * per LDS stage) `reps` times
 * (reps >= 1) on the caller's buffers -- a forward, plus a backward unless the plan is
 * forward-only -- times each with HIP events on `stream`, and keeps the fastest for
 * later calls.  Output buffers are overwritten; dz, dmu, ds, du, dlogp may be NULL for a
 * forward-only plan.  Synchronises the stream.  If the environment variable
 * TMC_TUNE_CACHE names a file, the choice is appended to it as a line
 * "<shape signature> <persist> <grid factor> <stages> <wide forward> <wide backward>" and
 * plans created later with the
 * same signature start from it.  Not for use during graph capture.  Plain-engine plans:
 * returns TMC_OK without doing anything. */
tmc_status tmc_plan_autotune(tmc_plan_t plan, const void* z, const void* mu, const void* s,
                             const void* u, const double* dlogp, void* workspace, void* dz,
                             void* dmu, void* ds, void* du, int reps, void* stream);

/* ---- measurement ---- */
/* Kernel classes timed by the plan's optional event timer. */
typedef enum tmc_kernel_class {
  TMC_KC_PLAIN_FACTOR = 0,   /* plain: materialise f_l */
  TMC_KC_PLAIN_LSE_FWD = 1,  /* plain: streaming row log-sum-exp (forward messages) */
  TMC_KC_PLAIN_LSE_BWD = 2,  /* plain: column-strip marginals (backward messages) */
  TMC_KC_PLAIN_GRAD = 3,     /* plain: Gaussian gradients from the marginals */
  TMC_KC_FUSED_PREP = 4,     /* fused: operand packing and row/column constants */
  TMC_KC_FUSED_FWD = 5,      /* fused: factor GEMM + forward message */
  TMC_KC_FUSED_BWD = 6,      /* fused: factor GEMM + marginals + gradient GEMM */
  TMC_KC_OTHER = 7,          /* initialisation, log-normaliser, reductions */
  TMC_KC_STAR_MSG = 8,       /* star model: local messages m_i (forward) */
  TMC_KC_STAR_BWD = 9,       /* star model: local and global gradient passes */
  TMC_KC_COUNT = 10
} tmc_kernel_class;

/* enable != 0: every later execute call on this plan records a hipEvent pair around
 * each kernel launch, on the stream the kernel runs on (up to a fixed pool of
 * events; launches beyond it are not timed).  Clears accumulated times.  Not for use
 * inside graph capture.  enable == 0 turns it off. */
tmc_status tmc_plan_set_timing(tmc_plan_t plan, int enable);
/* Synchronises the recorded events and returns, for kernel class `kc`, the summed
 * device time of its timed launches (ms) and their count. */
tmc_status tmc_plan_timing(tmc_plan_t plan, int kc, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* TMC_H_ */
