/*
 * hq.h — C ABI of the MI355X hypercube queueing solver (libhq.so).
 *
 * The library computes the stationary distribution P of the 2^N-state
 * busy/idle loss CTMC of the spatial hypercube model with heterogeneous
 * service rates (Section 2.1: N units, J demand nodes, each node dispatches
 * to its first idle preferred unit, calls finding every unit busy are lost),
 * by the Conditional Probability Update iteration (Algorithm 1) over the
 * birth-death reformulation (Proposition 1, eqs. (8)-(10)).
 *
 * Conventions shared by every entry point:
 *   - State m is a bitmask: bit u set <=> unit u busy (the index y(B_m) of
 *     Section 3.2 with unit i = bit i-1).  Exported P is in this order.
 *   - Rates are in any consistent time unit; P is invariant under scaling
 *     all rates together.
 *   - Inputs are copied during the call; the caller may free them on return.
 *     Output arrays are caller-allocated host memory unless stated.
 *   - Every failure returns a status code (never aborts or throws across the
 *     ABI) and sets a thread-local message readable with hq_last_error().
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Errors from the HIP runtime are reported as HQ_ERR_DEVICE.
 */
#ifndef HQ_H
#define HQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HQ_BUFFER_UNLIMITED (-1)
#define HQ_BUFFER_MAX 65536 /* largest finite waiting room */
#define HQ_MAX_N 30 /* 2^30 states; colex ranks and layer offsets fit in uint32 */

typedef struct hq_ctx hq_ctx; /* opaque; owns its host and device memory */
typedef struct hq_mlp hq_mlp; /* opaque; the warm-start network (see below) */

#define HQ_MLP_IN 32      /* feature slots per unit (19 used, the rest zero) */
#define HQ_MLP_HIDDEN 256 /* width of both hidden layers */
#define HQ_MLP_PARAMS (HQ_MLP_IN * HQ_MLP_HIDDEN + HQ_MLP_HIDDEN + HQ_MLP_HIDDEN * HQ_MLP_HIDDEN + \
                       HQ_MLP_HIDDEN + HQ_MLP_HIDDEN + 1)

typedef enum {
    HQ_OK = 0,
    HQ_ERR_INVALID_ARG = 1,  /* bad size, rate, preference row, tolerance, option */
    HQ_ERR_OUT_OF_MEMORY = 2,/* host or device allocation failed */
    HQ_ERR_DEVICE = 3,       /* HIP runtime error, or no usable GPU */
    HQ_ERR_NOT_CONVERGED = 4,/* max_iters reached; the last iterate stays readable */
    HQ_ERR_NUMERIC = 5,      /* NaN/Inf or a zero denominator in a layer reduction */
    HQ_ERR_STATE = 6         /* results requested before any solve/iterate */
} hq_status;

/* storage precision of the conditional-probability vector */
enum {
    HQ_FP64 = 0,          /* FP64 state, FP64 arithmetic (default) */
    HQ_FP32 = 1,          /* FP32 state with per-layer scale, FP64 reductions and residual */
    HQ_FP32_POLISH64 = 2  /* FP32 sweeps to the FP32 floor, then FP64 sweeps to tol */
};

/* reading of Algorithm 1's inner mu(n) loop (delta is never stated) */
enum {
    HQ_INNER_CLOSED = 0,  /* the delta -> 0 limit: mu(n) = B / (1 - A) each layer (one pass with
                             look-ahead sums at the default tile shape up to N = 26, else two) */
    HQ_INNER_ONE = 1,     /* one update per layer (delta = infinity); same fixed point */
    HQ_INNER_LITERAL = 2  /* the inner loop of Algorithm 1 as written, tolerance opts.delta
                             (two passes; the loop itself runs on the layer's sums) */
};

/* initial iterate */
enum {
    HQ_INIT_UNIFORM = 0, /* p_n(m) = 1 / C(N, n), as Algorithm 1 step 2 */
    HQ_INIT_PRODUCT = 1, /* p_n(m) proportional to prod_{u in m} x_u, with x fitted on the host so that the
                            start's busy probabilities (layer law from (10) with the start's own mu(n))
                            equal init_rho; targets no start can meet give the closest one found */
    HQ_INIT_STATE = 2,   /* resume: conditional probabilities p_n(m) from init_state (bitmask order) */
    HQ_INIT_LEARNED = 3  /* product form with rho predicted by opts.mlp (falls back to uniform) */
};

/* stopping rule */
enum {
    HQ_STOP_RESIDUAL = 0, /* relative L1 balance residual of (1) <= tol (default) */
    HQ_STOP_DELTA = 1     /* the paper's max_{n,m} |p^k - p^(k-1)| <= tol (Algorithm 1 step 3) */
};

typedef struct {
    int precision;            /* HQ_FP64 | HQ_FP32 | HQ_FP32_POLISH64 */
    int inner;                /* HQ_INNER_CLOSED | HQ_INNER_ONE | HQ_INNER_LITERAL */
    int init;                 /* HQ_INIT_* */
    int stop;                 /* HQ_STOP_* */
    int max_iters;            /* <= 0: default 100000 */
    int check_every;          /* residual cadence; <= 0: adaptive (predicts the crossing) */
    int tile_bits;            /* low bits per tile b (4..12); <= 0: choose */
    int device;               /* HIP device ordinal; < 0: current device */
    int stored_layers;        /* top layers whose dispatch coefficients are precomputed and
                                 stored (FP64, N values per state): 0 = choose (from the top
                                 down, the layers whose per-tile dispatch programs average
                                 >= 32 terms per state, within 16 GiB and a quarter
                                 of the free device memory), < 0 = none,
                                 k > 0 = layers N-k..N-1 */
    const double* init_rho;   /* [N] per-unit utilisations for HQ_INIT_PRODUCT (copied) */
    const double* init_state; /* [2^N] conditional probabilities for HQ_INIT_STATE (copied) */
    void* stream;             /* hipStream_t to run on (e.g. torch's current stream); NULL = own stream */
    const hq_mlp* mlp;        /* network for HQ_INIT_LEARNED (evaluated during hq_create) */
    int buffer;               /* waiting room for calls that find every unit busy (Section 2.2,
                                 Proposition 2): 0 = none (loss system), 0 < C <= HQ_BUFFER_MAX =
                                 at most C waiting calls, HQ_BUFFER_UNLIMITED = no limit (needs
                                 Lambda < sum mu_i) */
    double delta;             /* tolerance of the inner loop for HQ_INNER_LITERAL (finite, > 0;
                                 the loop stops when max_m |p^{r} - p^{r-1}| <= delta) */
} hq_options;

typedef struct {
    int status;                  /* hq_status of the solve */
    int iterations;              /* outer iterations (full layer sweeps) performed */
    int checks;                  /* residual evaluations performed */
    int fp64_iterations;         /* of which in FP64 (HQ_FP32_POLISH64) */
    double residual;             /* last relative L1 balance residual (FP64) */
    double seconds;              /* wall time of the solve (init + sweeps + checks) */
    double sweep_seconds;        /* device time of the sweeps alone (HIP events) */
    double state_updates_per_s;  /* (2^N - 2) * iterations / sweep_seconds */
    double mass_error;           /* sum(P) - 1 before the final renormalisation */
    double max_layer_drift;      /* max_n |sum_{C_n} p_n - 1| at the end */
    int warm_used;               /* 1 if a product-form / learned initial iterate was kept, 0 if
                                    the uniform start was used (no warm start, or fallback) */
} hq_info;

/* Fill *opts with the defaults (FP64, one inner update per layer, uniform
 * init, residual stop, adaptive checks, no waiting room). */
void hq_default_options(hq_options* opts);

/*
 * Create a solver for one instance (Section 2.1; Algorithm 1 inputs).
 *   N          number of units, 1..HQ_MAX_N
 *   J          number of demand nodes, >= 1
 *   lambda_j   [J] arrival rate of node j (lambda f_j), finite, >= 0, sum may be 0
 *   mu_i       [N] service rate of unit i (the paper's nu_i), finite, > 0
 *   pref_lists [J*N] row j = units 0..N-1 in node j's order of preference,
 *              most preferred first; each row must be a permutation
 *   opts       nullable; NULL = defaults
 *   out        receives the context (NULL on failure)
 * Preprocessing (unit relabelling, merged dispatch terms, per-tile dispatch
 * tables) and device allocation happen here.  Errors: HQ_ERR_INVALID_ARG,
 * HQ_ERR_OUT_OF_MEMORY, HQ_ERR_DEVICE.
 */
hq_status hq_create(int N, int J, const double* lambda_j, const double* mu_i,
                    const int32_t* pref_lists, const hq_options* opts, hq_ctx** out);

/*
 * Run Algorithm 1 from the configured initial iterate until the stopping
 * rule holds (tol > 0) or max_iters.  info (nullable) receives the
 * statistics.  A solve whose residual has stopped falling (six checks in a
 * row with less than a 0.01 % decrease per iteration: the rounding floor of
 * FP64 above tol, or divergence) ends early with HQ_ERR_NOT_CONVERGED and
 * the residual reached.  Returns HQ_OK, HQ_ERR_NOT_CONVERGED (iterate still readable),
 * HQ_ERR_NUMERIC, HQ_ERR_DEVICE or HQ_ERR_INVALID_ARG (tol <= 0 or NaN).
 * With Lambda = 0 the result is P(empty) = 1 and HQ_OK.
 */
hq_status hq_solve(hq_ctx* ctx, double tol, hq_info* info);

/*
 * Marginals of the last iterate (Proposition 1: P(m) = p(|m|) p_|m|(m)):
 *   rho_u [N]   (nullable) busy probability of each unit, sum_{m containing u} P(m)
 *   p_n   [N+1] (nullable) number-busy distribution p(n) of (10); with a
 *               waiting room p_n[N] includes the states with calls waiting
 * P is renormalised to sum 1 first.  HQ_ERR_STATE before any solve.
 */
hq_status hq_marginals(const hq_ctx* ctx, double* rho_u, double* p_n);

/*
 * Waiting-room measures of the last iterate (Section 2.2, Proposition 2 and
 * the remark after it).  A waiting room changes only the birth-death
 * marginal: the layers p_n(m) are those of the loss system, and the states
 * with every unit busy and c calls waiting have P~{c} = p(N) rho^c with
 * rho = Lambda / sum mu_i.
 *   summary [4] (nullable) P(every unit busy, waiting calls included),
 *               P(at least one call waits), mean number of waiting calls,
 *               P(an arriving call is lost) (P(full) without a room, the
 *               room-full probability with C > 0, 0 when unlimited)
 *   tail    [len] (nullable) P~{c} for c = 1..len; entries beyond C are 0
 * With buffer = 0 every waiting quantity is 0.  hq_state and hq_marginals
 * already include the room: P over the 2^N unit states sums to
 * 1 - P(at least one call waits), and rho_u and p_n(N) count the waiting
 * states as all units busy.  HQ_ERR_STATE before any solve.
 */
hq_status hq_queue(const hq_ctx* ctx, double* summary, double* tail, int len);

/*
 * Dispatch measures of the last iterate: unit workloads and response times,
 * the performance measures the stationary law serves (Section 1).  A call
 * from node j is sent to the first unit of its list that is idle (eq. (3)),
 * so with G(S) = sum over states m containing S of P(m),
 *   q[j * N + i] = G(units ranked before i by j) - G(those and i),
 * the probability that a call from node j is sent to unit i on arrival.
 * Computed on the device: P in bitmask order, an in-place superset-sum
 * transform over all N bits, one pass of reads per node.
 *   travel      [J*N] (nullable) travel time to node j from unit i at
 *               [j * N + i], finite; unit labels as in pref_lists
 *   q           [J*N] (nullable) out, as above; sum_i q[j * N + i] is the
 *               probability that some unit is idle (1 - P(full) without a
 *               waiting room; calls that wait are not counted)
 *   mean_travel (nullable) out: mean travel time of the calls sent on
 *               arrival, sum_j lambda_j sum_i q t / sum_j lambda_j sum_i q
 *               (needs travel)
 * Allocates 2^N doubles of device memory on the first call (kept until
 * hq_destroy).  Errors: HQ_ERR_INVALID_ARG, HQ_ERR_STATE before any solve,
 * HQ_ERR_OUT_OF_MEMORY, HQ_ERR_DEVICE.
 */
hq_status hq_dispatch(const hq_ctx* ctx, const double* travel, double* q, double* mean_travel);

/*
 * Export the stationary distribution of the last iterate, assembled as in
 * Proposition 1 (Section 2.2): P(m) = p(|m|) p_|m|(m), with the number-busy
 * marginal p(n) of (10) and the conditional layer probabilities p_n(m) of
 * (8).  The final step of Algorithm 1.
 *   P [2^N] caller-allocated host memory, bitmask order (bit u = unit u of
 *     the caller's labels busy); renormalised so that the whole system sums
 *     to 1 (with a waiting room the unit states sum to 1 - P(a call waits)).
 * Stages the vector in a device buffer of 2^N doubles that the context
 * allocates on the first export and keeps until hq_destroy (the buffer
 * hq_dispatch uses).  Errors: HQ_ERR_INVALID_ARG (NULL), HQ_ERR_STATE
 * before any solve, HQ_ERR_OUT_OF_MEMORY, HQ_ERR_DEVICE.
 */
hq_status hq_state(const hq_ctx* ctx, double* P);

/*
 * Solve several instances (an uneven batch of candidate deployments) to tol
 * in one persistent launch: Algorithm 1 (initial iterate, Gauss-Seidel
 * layer sweeps with the update (12)-(14), balance-residual stop on (1)) for
 * every instance, the instances independent of each other.  Every context
 * must be on the same device and must have been created with HQ_FP64 or
 * HQ_FP32 storage, the residual stopping rule and the closed or one-update
 * inner form (HQ_ERR_INVALID_ARG otherwise).  infos (nullable) [count].
 * A large instance is shared by up to 16 work-groups that meet at a barrier
 * after every layer; the results agree with hq_solve to rounding, and a
 * repeated batch gives bitwise the same results.  A barrier wait that runs
 * out (a device fault) ends that instance with HQ_ERR_DEVICE.
 * Returns HQ_OK only if every instance converged; per-instance statuses are
 * in infos.
 */
hq_status hq_solve_batch(hq_ctx* const* ctxs, int count, double tol, hq_info* infos);

/*
 * hq_solve_batch for callers that cannot allocate device memory during the
 * call: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results and errors as hq_solve_batch
 * (the contexts are created beforehand and own their state vectors); the
 * work queue, per-instance descriptors and results and the group-barrier
 * counters and partials live in a static device array of about 0.8 MB that
 * every GPU the library runs on holds until the process ends.  The call
 * makes no device allocation: no hipMalloc or hipFree, no captured graph,
 * no event; it runs on the first context's stream, uses the work-group
 * size tuned by an earlier hq_solve_batch of the same batch signature (256
 * otherwise), and returns after the batch has finished.
 *   count  at most HQ_NOALLOC_MAX_BATCH (256); more is HQ_ERR_INVALID_ARG.
 * Every call on one GPU shares that GPU's array and keeps the last call's
 * contents in it (the counters are cleared by the launch itself).  Calls on
 * one GPU must not overlap: the library serialises its own calls within a
 * process, and each call finishes its device work before it returns.
 */
#define HQ_NOALLOC_MAX_BATCH 256
hq_status hq_solve_batch_noalloc(hq_ctx* const* ctxs, int count, double tol, hq_info* infos);

/*
 * Shape of the most recent batched solve in this process, for reports:
 * the work-group size (threads) it ran with, 0 before any batched solve.
 * The batch kernel sweeps with 10 low bits per tile; the work-group size
 * is timed over 256, 512 and 1024 threads on the first hq_solve_batch of
 * each batch signature (precision, count, sorted unit counts) and reused
 * for that signature afterwards.
 */
int hq_batch_last_block(void);

/* Release a context (NULL-safe). */
void hq_destroy(hq_ctx* ctx);

/* Message for the last non-OK status on this thread ("" if none). */
const char* hq_last_error(void);

/* ---------------------------------------------------------------------
 * Inspection entry points (used for parity checks and resumption).
 * ------------------------------------------------------------------- */

/* Run exactly `iters` outer iterations from the current iterate (the
 * initial one if none has run), with no residual check.  Lets a caller stop
 * the GPU at the same iteration count as a reference. */
hq_status hq_iterate(hq_ctx* ctx, int iters);

/* Reset the iterate to the configured initial one. */
hq_status hq_reset(hq_ctx* ctx);

/* Relative L1 balance residual of the current iterate, in FP64. */
hq_status hq_residual(hq_ctx* ctx, double* residual);

/* Conditional layer probabilities p_n(m) of (8) [2^N] in bitmask order
 * (unnormalised values as iterated; the resume format of HQ_INIT_STATE).
 * Stages through the same context-owned device buffer as hq_state. */
hq_status hq_conditional(const hq_ctx* ctx, double* pcond);

/* Layer scalars [4*(N+1)]: for n = 0..N, lambda(n), mu(n), p(n), and
 * alpha_n = mu(n)/lambda(n-1) as last used in the update (12). */
hq_status hq_layer_scalars(const hq_ctx* ctx, double* out);

/* Export P [2^N] (bitmask order, sum 1) into device memory `dev_P` of the
 * context's device, on `stream` (NULL = the context's stream). */
hq_status hq_state_device(const hq_ctx* ctx, double* dev_P, void* stream);

/* Number of units of a context. */
int hq_num_units(const hq_ctx* ctx);

/* ---------------------------------------------------------------------
 * Learned warm start: an MLP (HQ_MLP_IN -> 256 -> 256 -> 1, ReLU, sigmoid
 * output) that predicts each unit's busy probability from scale-free
 * features of the instance.  Its prediction seeds the product-form initial
 * iterate p_n(m) proportional to prod_{u in m} rho/(1-rho), normalised per
 * layer with elementary symmetric polynomials (a uniform rho gives the
 * 1/C(N,n) start of Algorithm 1).  Products run on the matrix cores with
 * BF16 operands and FP32 accumulation; master weights and Adam state are
 * FP32.  Parameters are packed as W1[IN*256] (row = feature), b1[256],
 * W2[256*256] (row = input), b2[256], w3[256], b3[1].
 * ------------------------------------------------------------------- */

/* Per-unit features [N * HQ_MLP_IN] of an instance (host computation; same
 * arguments as hq_create): relative service rate, shares of demand that
 * rank the unit at positions 0..7 and 8+, offered load, load-discounted
 * exposure, N/32, rate relative to the fastest unit, first-choice share
 * times N, a constant 1, and the independence approximation of the unit's
 * utilisation (units busy independently; a call reaches a unit when every
 * unit its node ranks earlier is busy): the approximate utilisation, the
 * share of calls that reach the unit, and the clipped log-odds / 8. */
hq_status hq_mlp_features(int N, int J, const double* lambda_j, const double* mu_i,
                          const int32_t* pref_lists, float* features);

/* New network on `device` (< 0: current) with Glorot-uniform weights from `seed`. */
hq_status hq_mlp_create(int device, unsigned long long seed, hq_mlp** out);
void hq_mlp_destroy(hq_mlp* mlp); /* NULL-safe */

/* Copy the FP32 parameters out of / into the network ([HQ_MLP_PARAMS]). */
hq_status hq_mlp_get_params(const hq_mlp* mlp, float* params);
hq_status hq_mlp_set_params(hq_mlp* mlp, const float* params);

/* Predictions y[rows] for features X[rows * HQ_MLP_IN]. */
hq_status hq_mlp_forward(hq_mlp* mlp, const float* X, int rows, float* y);

/* One forward + backward pass of the mean squared error of rows (X, t):
 * gradient of the loss w.r.t. the packed parameters into grad
 * [HQ_MLP_PARAMS], the loss into *loss (nullable). */
hq_status hq_mlp_gradient(hq_mlp* mlp, const float* X, const float* t, int rows, float* grad,
                          float* loss);

/* Adam training (lr, beta 0.9/0.999) of the mean squared error over
 * `epochs` shuffled passes (seeded) with minibatches of `batch` rows
 * (a multiple of 32); epoch_loss [epochs] (nullable) gets the mean loss. */
hq_status hq_mlp_train(hq_mlp* mlp, const float* X, const float* t, int rows, int epochs, int batch,
                       float lr, unsigned long long seed, float* epoch_loss);

#ifdef __cplusplus
}
#endif

#endif /* HQ_H */
