/*
 * ksgcmi.h - C ABI of the MI355X (gfx950) nearest-neighbour conditional mutual
 * information library.
 *
 * What is computed.  The paper (IDTxl, Summary) describes greedy multivariate
 * transfer-entropy network inference: for every target a parent set is built by
 * repeatedly adding the candidate past variable that maximises a conditional
 * mutual information (CMI) criterion, each inclusion gated by a test against
 * null distributions from surrogate data (network-inference paragraph), with the
 * nonlinear KSG nearest-neighbour estimator (Kraskov, Stoegbauer & Grassberger
 * 2004) as the accurate continuous estimator and direct estimator access for
 * (conditional) MI (estimator paragraph).  The paper prints no formula; the
 * estimator is KSG algorithm 1 in the CMI form of Frenzel & Pompe (2007):
 *
 *   d_ij^S  = max over the coordinates a of subspace S of |fl32(p_ja - p_ia)|
 *   eps_i   = k-th smallest of { d_ij^XYZ : j != i }          (multiset order statistic)
 *   n_S(i)  = #{ j != i : d_ij^S < eps_i },  S in {XZ, YZ, Z}  (strict; d^Z = 0 if Z empty)
 *   I       = psi(k) - <psi(n_XZ+1) + psi(n_YZ+1) - psi(n_Z+1)>
 *           = H_{k-1} - (1/N) sum_i [H_{n_XZ(i)} + H_{n_YZ(i)} - H_{n_Z(i)}]   (nats)
 *
 * with every coordinate difference one IEEE FP32 round-to-nearest-even
 * subtraction and FP64 harmonic numbers H_n.  Results are not clipped at 0.
 *
 * Conventions.
 *  - Every function returns a ksg_status; nothing throws or aborts across the ABI.
 *  - Pointers are DEVICE pointers unless a comment says "host".  The caller owns
 *    every buffer it passes; the library never frees or retains caller memory
 *    beyond the call (device work is stream-ordered on the context's stream).
 *  - Point sets are structure-of-arrays: a d-dimensional variable of N points is
 *    d columns of N floats, column c at ptr[c*N + i].
 *  - Arguments are validated on the host before any device work.  Non-finite
 *    data are rejected with KSG_ENONFINITE by a device-side check (one stream
 *    synchronisation) unless KSG_OPT_CHECK_FINITE is switched off.
 *  - A context is not thread-safe: use one context per host thread.  Contexts on
 *    one device share nothing.
 *  - ksg_last_error(ctx) describes the last failure on that context.
 *
 * Limits: 1 <= k <= 16, N > k, N <= 2^31 - 1024, d_x >= 1, d_y >= 1, d_z >= 0,
 * d_x + d_y + d_z <= 32 (<= 16 under KSG algorithm 2).  Problems of up to 16 columns run
 * kernels compiled per column count; 17..32 columns run one brute-force kernel compiled for 32
 * columns, or the grouped kernels when d_x = d_y = 1 and several problems share Y and Z.
 */
#ifndef KSGCMI_H
#define KSGCMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ksg_status {
  KSG_OK = 0,
  KSG_EINVAL = 1,      /* bad argument (null pointer, dims, k, sizes, options) */
  KSG_ETOOFEW = 2,     /* N <= k: the k-th neighbour does not exist */
  KSG_ENONFINITE = 3,  /* NaN or infinity in the input data */
  KSG_ENOMEM = 4,      /* device or pinned-host allocation failed */
  KSG_EDEVICE = 5,     /* a HIP runtime call failed (message in ksg_last_error) */
  KSG_ENODEV = 6,      /* no usable HIP device */
  KSG_EBUFSMALL = 7    /* caller-provided output capacity too small (needed size reported) */
} ksg_status;

#define KSG_MAX_DIMS 32
#define KSG_MAX_K 16

typedef struct ksg_ctx ksg_ctx;

/* Library version as 10000*major + 100*minor + patch. */
int ksg_version(void);

/* Human-readable name of a status code (static string). */
const char* ksg_status_string(int status);

/* Number of visible HIP devices (0 when none); never fails. */
int ksg_device_count(void);

/* What the HIP runtime reports for a device (the figures the roofline's peaks derive from). */
typedef struct ksg_device_props {
  char name[128];
  char arch[64];         /* gcnArchName, e.g. "gfx950:sramecc+:xnack-" */
  int32_t cus;           /* compute units */
  int32_t clock_khz;     /* peak engine clock */
  int32_t mem_clock_khz; /* peak memory clock */
  int32_t mem_bus_bits;  /* memory bus width */
  int64_t total_mem;     /* bytes */
  int32_t l2_bytes;
  int32_t lds_per_cu;    /* bytes of LDS per compute unit */
  int32_t lds_per_block; /* bytes of LDS one work-group may use */
  int32_t wave_size;
} ksg_device_props;

/* Fill *out for HIP device `device` (host call; no context needed).
 * Errors: KSG_EINVAL (out NULL), KSG_ENODEV (no such device). */
int ksg_device_props_get(int32_t device, ksg_device_props* out);

/* Host utility (no device needed): harmonic numbers H_0..H_nmax (H_n = sum_{m<=n} 1/m, so
 * psi(n+1) = H_n - Euler's gamma) into the host array out[nmax+1], FP64, from a
 * double-double running sum.  These are the digamma values the estimator uses.
 * Errors: KSG_EINVAL (nmax < 0, out NULL). */
int ksg_harmonic_table(int64_t nmax, double* out);

/* Create a context on HIP device `device`, issuing all work on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the context.
 * Errors: KSG_EINVAL (out == NULL, device out of range), KSG_ENODEV. */
int ksg_ctx_create(ksg_ctx** out, int device, void* hip_stream);

/* Release a context and its workspace (waits for its pending work). NULL is a no-op. */
void ksg_ctx_destroy(ksg_ctx* ctx);

/* Text of the last error on this context; valid until the next call on it. */
const char* ksg_last_error(const ksg_ctx* ctx);

/* Options. */
typedef enum ksg_option {
  KSG_OPT_CHECK_FINITE = 1, /* 1 (default): reject non-finite data; 0: trust inputs */
  KSG_OPT_GROUP_SIZE = 2,   /* problems searched together when they share Y, Z, N and k and
                               have 1-D X: -1 (default) = autotuned per conditioning dimension,
                               0 = off, 8 or 16 = forced */
  KSG_OPT_USE_GRAPH = 3,    /* 1: capture the launches of a batch into a HIP graph (with private
                             * copies of its descriptors) and replay the graph when the same batch
                             * (same problems, columns, gathers, output and options) comes again,
                             * skipping the host planning, the upload and the per-launch overhead;
                             * at most 32 graphs per context (least recently used dropped); the
                             * graphs that write a work buffer are freed when it grows.  Used only
                             * with KSG_OPT_TIMING = 0 and
                             * KSG_OPT_CHECK_FINITE = 0 (select_parents checks its data once and
                             * runs its steps without the check).  0 (default): direct launches */
  KSG_OPT_TIMING = 4,       /* 1: time every search-kernel launch with HIP events (default 0) */
  KSG_OPT_ALGORITHM = 5,    /* KSG algorithm of every later estimate (default 1):
                             * 1: eps_i = joint k-th neighbour distance, strict counts in XZ, YZ, Z,
                             *    I = H_{k-1} - <H_{n_xz} + H_{n_yz} - H_{n_z}>;
                             * 2: the k nearest neighbours (ties by the lower index) span a
                             *    rectangle with one side per space (the largest X, Y and Z distance
                             *    to them), counts with <= inside it,
                             *    I = psi(k) - 2/k + <psi(n_z) - psi(n_xz) - psi(n_yz) + 1/n_xz + 1/n_yz>,
                             *    without Z I = psi(k) - 1/k + psi(N) - <psi(n_x) + psi(n_y)>.
                             *    counts_out then holds these counts (n_z = N-1 without Z), eps_out
                             *    the k-th neighbour's joint distance, local_out the pointwise values.
                             *    Problems are searched one by one (no grouping). */
  KSG_OPT_GROUP_CHUNK = 7,  /* grouped problems run in chunks whose radii (FP32) and Y/Z terms
                             * (FP64) hold at most this many elements: 0 (default) = 2^27, i.e.
                             * 1.5 GiB of workspace; smaller values bound the workspace (more
                             * launches, same results) */
  KSG_OPT_MEM_LIMIT = 9,    /* bytes of device workspace the context may hold (columns pool,
                             * radii, terms, descriptors, graphs...): 0 (default) = no limit; a
                             * batch that needs more fails with KSG_ENOMEM and leaves the context
                             * usable */
  KSG_OPT_TILE_Q = 8,       /* queries per work-group of the brute-force kernels: 0 (default) =
                             * the autotuner's choice for the launch's size (256 before tuning),
                             * or 64, 128, 256 forced; same results up to the order of the FP64
                             * sum */
  KSG_OPT_WINDOWS = 6       /* 1 (default): single problems (not grouped) with k <= 4, N at or
                             * above the window threshold of their column count (2048 before
                             * ksg_autotune; the tuner's per-D choice after it; 2: 2048 always),
                             * an unpermuted Z column and, under algorithm 2, no per-point
                             * outputs are searched with
                             * their rows in the order of that column, each tile scanning only the
                             * rows its radii, rectangle sides and counts can reach (same results
                             * up to the order of the FP64 sum; either KSG algorithm; under
                             * algorithm 2 neighbours tied at the k-th distance are still taken
                             * by the lower row index); 0: brute force over all rows */
} ksg_option;
int ksg_ctx_set_option(ksg_ctx* ctx, int option, int64_t value);

/* KSG_OPT_USE_GRAPH bookkeeping (host int64 outputs): batches captured into graphs, graph
 * replays, and graphs held now.  Errors: KSG_EINVAL. */
int ksg_graph_stats(ksg_ctx* ctx, int64_t* captures, int64_t* replays, int64_t* held);

/* Autotuner of the launch shapes, from timings of synthetic batches on the context's device:
 * (1) the group size (8 or 16) of the grouped kernels for k <= 4 and k <= 8 and every
 * conditioning dimension m = 0..14 (32 problems of n points sharing Y and Z; m > 14 always use
 * 8); (2) the tile height (64, 128 or 256 queries per work-group) of the brute-force kernels,
 * for launches of fewer than 4 x (compute units) tiles of 256 and for larger ones; (3) for
 * single problems of D = 3..16 columns with an unpermuted Z column, the smallest N in
 * {2048, 8192, 32768} at which the key-ordered window search beats the brute-force kernel
 * (never: INT32_MAX).  Later batches on the context use these choices (KSG_OPT_GROUP_SIZE = -1,
 * KSG_OPT_TILE_Q = 0, KSG_OPT_WINDOWS = 1).  cache_path (host string or NULL): a text file of
 * per-device results (keyed by architecture, compute units and library version); an existing
 * entry is used instead of timing, a new one is appended.  tuned_out (host int32 [46] or NULL):
 * the 15 group sizes for k <= 4, the 15 for k <= 8, the two tile heights, the 14 window
 * thresholds for D = 3..16.  Synchronises.
 * Errors: KSG_EINVAL (n outside [256, 2^20]), KSG_ENOMEM, KSG_EDEVICE. */
int ksg_autotune(ksg_ctx* ctx, int64_t n, const char* cache_path, int32_t* tuned_out);

/* With KSG_OPT_TIMING on: device time of the search kernels (radius, counts and per-tile
 * digamma sums, finalisation excluded) summed over all search phases since the last call, in
 * milliseconds, with their count and algorithmic operation count.  Problems searched alone
 * count N(N-1)(4D+2) (per ordered pair D subtractions, D-1 maxima and 1 compare for the
 * radius, the same plus 3 compares for the counts); with KSG_OPT_WINDOWS, the same per pair
 * over the pairs that each wave's scan visits (padding lanes included).  Problems searched
 * in groups that share Y and Z are counted on the device over the work executed (key
 * windows and exact skips decide which reference steps run): the shared Y/Z distances once
 * per pair of an executed
 * step (2m+2 for the radius, 2m for the X counts), 3 operations per pair for each problem's
 * radius and X count steps, and for the Y/Z counts, per visited reference, its d^Z and d^YZ
 * (2m+1) plus one compare per binary-search level for each of the two ranks.
 * Synchronises the stream; resets the accumulators.  Outputs are host pointers. */
int ksg_take_timing(ksg_ctx* ctx, double* ms, int64_t* launches, double* ops);

/* The grouped kernels' device work counters behind the last ksg_take_timing (host
 * uint64[5]): problem-steps of the radius kernel, problem-steps of the X count kernel, the
 * radius kernel's shared-part operations / 256 (a step is 4 references x 64 query lanes), the
 * Y/Z count kernel's operations, the X count kernel's shared-part operations / 256.
 * Errors: KSG_EINVAL. */
int ksg_last_work(ksg_ctx* ctx, uint64_t* counters);

/* Per-kernel split of the last ksg_take_timing (host arrays of 4, in the order: grouped
 * radius kernel, Y/Z count kernel, X count kernel, single-problem search kernels (brute force
 * and key-ordered windows together)): device milliseconds (each launch timed by its own pair
 * of events), algorithmic operations (as counted for ksg_take_timing) and launch counts.
 * Errors: KSG_EINVAL. */
int ksg_last_kernels(ksg_ctx* ctx, double* ms, double* ops, int64_t* launches);

/* ---------------------------------------------------------------------------
 * Single estimate (direct estimator access, Summary estimator paragraph).
 * x, y, z: SoA columns, dims[0], dims[1], dims[2] columns of N floats (z may be
 * NULL iff dims[2] == 0).  k: neighbour rank.  *out_nats (host): the estimate.
 * Synchronises the context's stream.
 * Errors: KSG_EINVAL, KSG_ETOOFEW, KSG_ENONFINITE, KSG_ENOMEM, KSG_EDEVICE. */
int cmi_ksg(ksg_ctx* ctx, const float* x, const float* y, const float* z, int64_t N,
            const int32_t dims[3], int32_t k, double* out_nats);

/* ---------------------------------------------------------------------------
 * The estimate of cmi_ksg without any allocation, for callers that cannot allocate: code under
 * HIP stream capture, tight serving loops, harnesses that forbid hipMalloc.  Arguments as for
 * cmi_ksg, except out_nats: a DEVICE pointer to one double, written in stream order (the call
 * returns once the work is queued on the context's stream; nothing synchronises).
 * Everything beyond the caller's inputs and output lives in one static device array of the
 * library (under 5 MiB per device, held until the process ends; located when a context is
 * created on the device), so the call allocates nothing and calls no hipMalloc, hipFree or
 * hipMemset.  Limits: N <= KSG_NOALLOC_MAX_N, d_x + d_y + d_z <= 16.  Data holding NaN or
 * infinity give a NaN estimate (no status: that would need a synchronisation).  Every call on
 * one device shares that array: calls that overlap on one GPU (several streams or threads)
 * race and must be ordered by the caller.  The search is the brute-force kernel of the batched
 * path, so the estimate equals cmi_ksg's up to the order of the FP64 sum.
 * Errors (host-side checks only): KSG_EINVAL (null pointers, dims, k, N above the limit),
 * KSG_ETOOFEW, KSG_EDEVICE (the array could not be set up on this device, or a launch failed). */
#define KSG_NOALLOC_MAX_N 65536
int cmi_ksg_noalloc(ksg_ctx* ctx, const float* x, const float* y, const float* z, int64_t N,
                    const int32_t dims[3], int32_t k, double* out_nats);

/* ---------------------------------------------------------------------------
 * Batched estimates: all problems of the batch are searched by one set of launches on the
 * context's stream, one work-group per work item (a 256-query tile of a problem or of a group
 * of problems), longest work first, so that the hardware dispatcher hands the work out as
 * compute units free up.  The set: the column pack (with the surrogate gathers); for problems
 * that share Y and Z and have 1-D X (the candidates x surrogates of a greedy step) the key
 * order, block interleave and three search launches per chunk of groups (radius, Y/Z counts,
 * X counts with the digamma partial sums); for the other problems one launch per column
 * count or shape (brute force or key-ordered windows), run side by side on three auxiliary
 * streams joined back by events; then one finalisation launch.  With KSG_OPT_USE_GRAPH the
 * set is captured once into a HIP graph and replayed when the same batch comes again.
 *
 * perm_x: NULL, or an int32 row gather of length n applied to X only
 * (X'[i] = X[perm_x[i]]: a permutation surrogate, Summary network-inference
 * paragraph); Y and Z are never permuted.
 * eps_out / counts_out / local_out: NULL or per-point outputs: eps_i (FP32 [n]),
 * counts (int32 [3][n]: n_XZ, n_YZ, n_Z) and the local (pointwise) CMI values
 * psi(k) - psi(n_XZ+1) - psi(n_YZ+1) + psi(n_Z+1) (FP64 [n]).
 */
typedef struct ksg_problem {
  int64_t n;
  int32_t dx, dy, dz, k;
  const float* x;
  const float* y;
  const float* z;
  const int32_t* perm_x;
  float* eps_out;
  int32_t* counts_out;
  double* local_out;
} ksg_problem;

/* probs: host array of n_probs problems.  out_nats: device FP64 [n_probs].
 * Stream-ordered: returns once the work is queued (after the optional finite
 * check, which synchronises).  Inputs must stay valid until the stream reaches
 * the end of the batch.
 * Errors: KSG_EINVAL (with the index of the first bad problem in ksg_last_error),
 * KSG_ETOOFEW, KSG_ENONFINITE, KSG_ENOMEM, KSG_EDEVICE. */
int cmi_ksg_batch(ksg_ctx* ctx, const ksg_problem* probs, int32_t n_probs, double* out_nats);

/* ---------------------------------------------------------------------------
 * Max-statistic surrogate test (Summary, network-inference paragraph: surrogate
 * null distributions gate each inclusion; problem paragraph: errors from testing
 * many sources are controlled).  cmi: device FP64 [c][P+1]; column 0 holds the
 * c original estimates, columns 1..P the surrogate rounds (round p applies the
 * same permutation to every candidate).
 *   c_star = argmax_c cmi[c][0] (lowest index wins ties), t_obs = cmi[c_star][0]
 *   T_p    = max_c cmi[c][p],  count = #{p : T_p >= t_obs},  pval = count / P
 *   significant = pval < alpha;  tau05 / tau01 = ceil(0.05 P)-th / ceil(0.01 P)-th
 *   largest T_p (so that p < alpha  <=>  t_obs > tau_alpha).
 * out: host.  Synchronises.  Errors: KSG_EINVAL, KSG_EDEVICE. */
typedef struct ksg_maxstat_result {
  int32_t c_star;
  int32_t count;
  int32_t significant;
  int32_t n_perm;
  double t_obs;
  double pval;
  double tau05;
  double tau01;
} ksg_maxstat_result;
int ksg_maxstat(ksg_ctx* ctx, const double* cmi, int32_t c, int32_t n_perm, double alpha,
                ksg_maxstat_result* out);

/* ---------------------------------------------------------------------------
 * Lagged embedding (Summary, network-inference paragraph: the conditioning
 * builds a non-uniform embedding of candidate past variables and optimises
 * source-target delays).  data: device FP32 [n_trials][n_vars][T] (the generic
 * multivariate time-series format, Summary last paragraph).  Embedded points are
 * t = max_lag .. T-1 of every trial, pooled trial-major: N = n_trials*(T-max_lag).
 * cand_out: device FP32 [n_vars*max_lag][N]; candidate v*max_lag + (l-1) holds
 * x_v(t - l).  y_out: device FP32 [N], x_target(t).  Stream-ordered.
 * Errors: KSG_EINVAL. */
int ksg_embed(ksg_ctx* ctx, const float* data, int32_t n_vars, int64_t T, int32_t n_trials,
              int32_t target, int32_t max_lag, float* cand_out, float* y_out);

/* ---------------------------------------------------------------------------
 * One greedy step on embedded columns (the unit that select_parents repeats): for
 * every candidate c in pool and every round p = 0..n_perm (0 = original data,
 * p >= 1 = X rows gathered through perms[p-1], the same gather for every candidate)
 * estimate I(X_c ; Y | Z) with Z = the cond columns, all in one batched launch, then
 * apply the max-statistic test.
 * cand: device FP32 [C][N] columns (layout of ksg_embed); y: device FP32 [N];
 * pool, cond: host int32 candidate indices (< C, not checked against C: the caller
 * guarantees they address columns of cand); perms: device int32 [n_perm][N];
 * cmi_out: device FP64 [n_pool][n_perm+1]; result: host.  Synchronises.
 * Errors: KSG_EINVAL, KSG_ETOOFEW, KSG_ENONFINITE, KSG_ENOMEM, KSG_EDEVICE. */
int ksg_greedy_step(ksg_ctx* ctx, const float* cand, const float* y, int64_t N, const int32_t* pool,
                    int32_t n_pool, const int32_t* cond, int32_t n_cond, const int32_t* perms,
                    int32_t n_perm, int32_t k, double alpha, double* cmi_out,
                    ksg_maxstat_result* result);

/* ---------------------------------------------------------------------------
 * Greedy parent selection for one target (Summary, network-inference paragraph).
 * Candidates (mode KSG_MODE_MULTIVARIATE_TE): every variable's past (the target's own
 * included) at lags 1..max_lag, index v*max_lag + (lag-1), one pool.  Each step estimates the CMI
 * of every remaining candidate and its n_perm surrogates given the selected set
 * in one batched launch, applies the max-statistic test and either includes the
 * argmax (significant) or stops.  perms: device int32 [n_perm][N] row
 * permutations, N = n_trials*(T-max_lag); surrogate round p uses perms[p-1] for
 * every candidate.  With omnibus = 1 the final source set is tested jointly:
 * I(selected sources ; Y | selected target past), surrogates permuting the
 * source block rows.
 *
 * The conditioning set holds at most max_cond columns (0: the column limit less X and Y, i.e.
 * 30, or 14 under KSG algorithm 2).  When a step includes a candidate and the next step would
 * need more conditioning columns than that, the selection ends with truncated = 1: the paper's
 * statistical stop (a non-significant test or an empty pool) was not reached.  max_steps, when
 * it ends the loop, does not set truncated.
 *
 * Variants named beside multivariate TE in the same paragraph (readings, the paper defines
 * neither): KSG_MODE_MULTIVARIATE_MI: the pool without the target's own past;
 * KSG_MODE_BIVARIATE_TE: first the target's own past alone, then each source in index order
 * on its own, its lags conditioned only on the selected target past and its own selected lags.
 *
 * Post-selection pruning (prune = 1; the problem paragraph's control of errors over many
 * sources): each selected source c gets I(c ; Y | every other selected candidate) and its
 * surrogates (c's rows permuted by perms, shared by all c); with T_min the smallest (lowest
 * index on ties) and T_p the per-round minima, p = #{p : T_p >= T_min}/n_perm; if p >= alpha
 * the minimising source is removed and the test repeats, else the rest are kept.  The
 * omnibus test, when asked for, runs on the pruned set.
 *
 * Sequential max-statistic test (sequential = 1), after pruning and, when the omnibus test was
 * asked for, only if it is significant: each kept source c gets I(c ; Y | every other kept
 * candidate) and its surrogates as for pruning, and the table goes through
 * ksg_maxstat_sequential; sources it does not find significant are removed from the parents
 * (seq_removed) and the kept sources' p-values are reported (seq_pval).
 *
 * Every estimate uses the context's KSG algorithm (KSG_OPT_ALGORITHM).
 *
 * Learned null: learned != NULL gates each step first with the threshold
 * network (ksg_mlp) evaluated on the step's feature vector; only steps whose
 * t_obs lies within [tau05_hat - margin_lo*s, tau05_hat + margin_hi*s],
 * s = |tau01_hat - tau05_hat|, run the surrogates.  judge = 1 also runs the
 * plain test on every step, uses ITS decision, and counts disagreements.
 */
typedef struct ksg_mlp ksg_mlp;

typedef struct ksg_select_opts {
  int32_t k;
  int32_t max_lag;
  int32_t n_perm;
  int32_t omnibus;
  double alpha;
  const int32_t* perms;
  const ksg_mlp* learned;
  double margin_lo;
  double margin_hi;
  int32_t judge;
  int32_t max_steps; /* 0 = until the test stops or the pool is empty */
  int32_t mode;      /* KSG_MODE_* */
  int32_t prune;     /* 1: min-statistic pruning of the selected sources */
  int32_t sequential; /* 1: sequential max-statistic test of the kept sources (after pruning;
                       * skipped when the omnibus test ran and was not significant) */
  int32_t max_cond;   /* 0 = the library's limit; else at most this many conditioning columns */
  /* Resume (checkpoint of a run cut short): host int32 [n_resume] candidate indices
   * (v*max_lag + lag-1) included by an earlier run of the same target, data, permutations and
   * options, in inclusion order.  They start the conditioning set, leave the pool and head the
   * parent list (cmi and pval NaN: their tests are not re-run); n_steps counts the new tests
   * only.  Multivariate modes only.  n_resume = 0: a fresh selection. */
  const int32_t* resume;
  int32_t n_resume;
  int32_t verify_stop; /* learned null: 1 = a step the gate would stop on runs the plain test,
                        * whose decision is taken (a wrong stop loses every later parent, a wrong
                        * inclusion adds one); 0 = the gate decides both ways */
  int32_t deep_dz;     /* learned null: 0 = margin_lo/margin_hi on every step; > 0 = steps that
                        * condition on at least deep_dz columns use margin_lo_deep/margin_hi_deep
                        * (the thresholds' spread narrows with depth while the network's error
                        * does not, so deep steps need margins of their own) */
  double margin_lo_deep;
  double margin_hi_deep;
} ksg_select_opts;

enum { KSG_MODE_MULTIVARIATE_TE = 0, KSG_MODE_BIVARIATE_TE = 1, KSG_MODE_MULTIVARIATE_MI = 2 };

/* Per-step record (host arrays of `capacity` entries, caller-allocated; any may be NULL). */
typedef struct ksg_parent_set {
  int32_t capacity;
  int32_t n;            /* parents selected (inclusion order) */
  int32_t* var;         /* [capacity] variable of each parent */
  int32_t* lag;         /* [capacity] lag of each parent */
  double* cmi;          /* [capacity] t_obs of the step that included it */
  double* pval;         /* [capacity] its p-value (-1 when decided by the learned gate) */
  int32_t n_steps;      /* tests run, including the final non-significant one */
  int32_t n_fallback;   /* learned path: steps that ran the full surrogate test */
  int32_t n_disagree;   /* judge mode: steps where gate and plain test disagreed */
  int32_t n_gate_decided; /* learned path: steps decided by the gate alone */
  int32_t omnibus_tested;
  int32_t omnibus_significant;
  double omnibus_cmi;
  double omnibus_pval;
  int64_t n_cmi;        /* CMI estimates computed (originals + surrogates) */
  /* Optional per-step log (host arrays of step_capacity entries, any may be NULL; steps beyond
   * step_capacity are not logged): t_obs; the gate's predictions sqrt(N)*(tau_0.05, tau_0.01)
   * ([step_capacity][2], NaN when no gate ran); the gate's verdict (+1 include, -1 stop,
   * 0 borderline, 2 no gate); the plain test's decision (1 significant, 0 not, -1 not run). */
  int32_t step_capacity;
  double* step_tobs;
  float* step_pred;
  int32_t* step_verdict;
  int32_t* step_plain;
  /* Pruning: candidates removed (v*max_lag + lag-1, removal order; host array of capacity
   * entries or NULL) and how many; var/lag/cmi/pval above hold the kept parents. */
  int32_t n_pruned;
  int32_t* pruned;
  /* Sequential test: sources removed (candidate indices in rank order; host array of capacity
   * entries or NULL) and how many; seq_pval (host [capacity] or NULL): the test's p-value of
   * each kept parent in the order of var/lag (-1 for the target's own past or when the test did
   * not run). */
  int32_t n_seq_removed;
  int32_t* seq_removed;
  double* seq_pval;
  /* 1: the inclusion loop ended at the conditioning limit (max_cond) after a significant step,
   * not at a non-significant test or an empty pool; 0 otherwise. */
  int32_t truncated;
} ksg_parent_set;

/* data: device FP32 [n_trials][n_vars][T].  out: host struct.
 * Errors: KSG_EINVAL, KSG_ETOOFEW, KSG_ENONFINITE, KSG_ENOMEM, KSG_EDEVICE,
 * KSG_EBUFSMALL (more parents than capacity; out->n holds the number needed). */
int select_parents(ksg_ctx* ctx, const float* data, int32_t n_vars, int64_t T, int32_t n_trials,
                   int32_t target, const ksg_select_opts* opts, ksg_parent_set* out);

/* False discovery rate across targets (network-inference paragraph; reading: Benjamini-
 * Hochberg at level alpha on the targets' omnibus p-values): reject[i] = 1 for the r smallest
 * p-values, r the largest rank with p_(r) <= r * alpha / n (ties in index order), else 0.
 * Host arrays of n entries.  Errors: KSG_EINVAL (null pointers, n < 0, alpha outside (0,1)). */
int ksg_fdr_bh(const double* pvals, int32_t n, double alpha, int32_t* reject);

/* Sequential max-statistic test (reading of the post-selection statistics named in the
 * network-inference paragraph): table host FP64 [rows][n_perm+1], column 0 the observed CMI of
 * each tested variable, column 1+p its surrogate of round p.  The observed values are ranked in
 * descending order (lower row first on ties); the r-th ranked one gets p_r = #{p : r-th largest
 * surrogate value of round p >= its value} / n_perm and is significant when p_r < alpha; the
 * first rank that is not significant ends the test (it and every later rank: significant = 0,
 * later ranks keep pval = 1).  Outputs host int32 significant[rows], FP64 pval[rows] in row
 * order.  Host code, no device work.  Errors: KSG_EINVAL (null pointers, rows < 0, n_perm < 1,
 * alpha outside (0,1)). */
int ksg_maxstat_sequential(const double* table, int32_t rows, int32_t n_perm, double alpha,
                           int32_t* significant, double* pval);

/* ---------------------------------------------------------------------------
 * Learned null: a 16-64-64-2 perceptron (ReLU hidden layers, BF16 parameters,
 * FP32 accumulation) predicting the step's tau_0.05 and tau_0.01 thresholds
 * scaled by sqrt(N).  The paper has no learned null; this is the library's own gate
 * in front of the surrogate test of the network-inference paragraph, which stays
 * as the fallback and the judge.
 *
 * Parameter layout (5378 floats): W1[64][16] b1[64] W2[64][64] b2[64] W3[2][64] b3[2].
 * Features (16 per step, raw, standardised inside the network with mu/sd):
 *   log N, d_x, d_y, d_z, k, log c, log P, sqrt(N)*(largest, second largest,
 *   mean, sd of the c original CMIs), skewness and excess kurtosis of Y, mean
 *   skewness, mean excess kurtosis and mean |lag-1 autocorrelation| of the
 *   candidate columns.
 */
#define KSG_MLP_NPARAMS 5378
#define KSG_MLP_NFEAT 16

/* init: host FP32 [5378] initial master parameters.  */
int ksg_mlp_create(ksg_ctx* ctx, ksg_mlp** out, const float* init);
void ksg_mlp_destroy(ksg_mlp* m);
/* mu, sd: host FP32 [16] feature standardisation (sd > 0). */
int ksg_mlp_set_norm(ksg_mlp* m, const float* mu, const float* sd);
/* Copy FP32 master parameters to host [5378] (bf16 = 1: the BF16-rounded values in use). */
int ksg_mlp_get_params(const ksg_mlp* m, float* out, int32_t bf16);
int ksg_mlp_set_params(ksg_mlp* m, const float* params);
/* Forward: feats device FP32 [B][16] raw features -> out device FP32 [B][2].  ksg_mlp_predict is
 * the same call under the name of the survey's boundary. */
int ksg_mlp_forward(ksg_ctx* ctx, const ksg_mlp* m, const float* feats, int64_t B, float* out);
int ksg_mlp_predict(ksg_ctx* ctx, const ksg_mlp* m, const float* feats, int64_t B, float* out);
/* Loss and gradient of L = (1/B) sum_b 0.5 |out_b - t_b|^2 with respect to the
 * BF16 parameters: grad device FP32 [5378], loss device FP32 [1]. */
int ksg_mlp_grad(ksg_ctx* ctx, const ksg_mlp* m, const float* feats, const float* targets,
                 int64_t B, float* grad, float* loss);
/* Adam training (beta1 0.9, beta2 0.999, eps 1e-8) on device data, minibatches of
 * `batch` rows taken in order; loss_hist (host [epochs] or NULL) gets the mean
 * minibatch loss of every epoch. */
int ksg_mlp_train(ksg_ctx* ctx, ksg_mlp* m, const float* feats, const float* targets, int64_t B,
                  int32_t epochs, int32_t batch, float lr, float* loss_hist);
int ksg_mlp_save(const ksg_mlp* m, const char* path);
int ksg_mlp_load(ksg_ctx* ctx, ksg_mlp** out, const char* path);

/* Step features on the device: orig_cmi device FP64 [c]; y device FP32 [N];
 * cand device FP32 columns, cand_idx host int32 [c] (which candidate columns of
 * the pool are in the step); out device FP32 [16].  Used by select_parents; exposed
 * for parity tests. */
int ksg_step_features(ksg_ctx* ctx, const double* orig_cmi, int32_t c, const float* y,
                      const float* cand, int64_t N, const int32_t* cand_idx, int32_t dx,
                      int32_t dy, int32_t dz, int32_t k, int32_t n_perm, float* out);

/* Training examples for the threshold network from one greedy step's surrogate table:
 * every candidate subset of the step (rows of `table`) has its own max-statistic null
 * distribution (the same round permutations act on every candidate), so each subset gives
 * one example.  table: device FP64 [rows][n_perm+1] (column 0 = originals; the layout of
 * ksg_greedy_step); row_cand: host int32 [rows], candidate column of each row; subsets in
 * CSR form: sub_off host int32 [n_sub+1] (sub_off[0] = 0, strictly increasing), sub_rows
 * host int32 [sub_off[n_sub]].  cand: device FP32 [C][N]; y: device FP32 [N]; dz: the
 * step's conditioning dimension.  Outputs (device): feats FP32 [n_sub][16] (the step
 * features of the subset), targets FP32 [n_sub][2] = sqrt(N) * (tau_0.05, tau_0.01), obs
 * FP64 [n_sub][2] = (sqrt(N) * t_obs, 1.0 if the plain test is significant at 0.05 else 0.0).
 * Synchronises.  Errors: KSG_EINVAL, KSG_ENOMEM, KSG_EDEVICE. */
int ksg_null_examples(ksg_ctx* ctx, const double* table, int32_t rows, int32_t n_perm,
                      const int32_t* row_cand, const int32_t* sub_off, const int32_t* sub_rows,
                      int32_t n_sub, const float* cand, int32_t C, const float* y, int64_t N,
                      int32_t dz, int32_t k, float* feats, float* targets, double* obs);

/* Set the network's feature standardisation to the per-feature mean and population
 * standard deviation of feats (device FP32 [B][16]).  Synchronises. */
int ksg_mlp_fit_norm(ksg_ctx* ctx, ksg_mlp* m, const float* feats, int64_t B);

/* Calibrate the gate margins on held-out examples (feats [B][16] and obs [B][2] as written by
 * ksg_null_examples, device): with u = (sqrt(N) t_obs - pred_0.05) / |pred_0.01 - pred_0.05|,
 * the gate includes when u > margin_hi and stops when u < -margin_lo; each margin is the
 * smallest value >= 0 that leaves at most floor(rate/2 * B) examples decided against the
 * plain test on its side.  Outputs (host): margins, the fraction of examples left to the
 * surrogate test (fallback) and the number decided wrongly (wrong).  Synchronises. */
int ksg_gate_calibrate(ksg_ctx* ctx, const ksg_mlp* m, const float* feats, const double* obs,
                       int64_t B, double rate, double* margin_lo, double* margin_hi,
                       double* fallback, int64_t* wrong);

/* The same calibration with a separate allowance per side: margin_lo leaves at most
 * floor(rate_stop * B) significant examples decided as stops, margin_hi at most
 * floor(rate_include * B) non-significant examples decided as inclusions
 * (ksg_gate_calibrate(rate) = this with rate/2 on both sides).  A wrong inclusion at the step
 * where the plain test would stop lets the selection run on, so a caller that confirms every
 * predicted stop with the surrogates (verify_stop) may want rate_include < rate_stop.  Both
 * rates in [0, 1); outputs as above.  Synchronises. */
int ksg_gate_calibrate_sides(ksg_ctx* ctx, const ksg_mlp* m, const float* feats, const double* obs,
                             int64_t B, double rate_stop, double rate_include, double* margin_lo,
                             double* margin_hi, double* fallback, int64_t* wrong);

#ifdef __cplusplus
}
#endif

#endif /* KSGCMI_H */
