/*
 * CPU FP64 oracle of the Conditional Probability Update (CPU) iteration.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and
 * the benchmark's CPU-baseline leg load it; the library never does, and the
 * two share no code, header, table or helper.
 *
 * What it computes (paper, Section 2 and Section 3.1):
 *   - the loss system of Section 2.1 (buffer C = 0): N units, J demand nodes
 *     with arrival rates lam[j] (= lambda f_j), one preference list per node,
 *     service rate nu[u] per unit; state m is the busy set, unit u = bit u;
 *   - transition rates, eq. (3): arrival-driven rate into m from m\{u}
 *     (u in m) is the summed rate of the nodes all of whose units ranked
 *     before u are busy in m (the product in (3) read with upper limit
 *     eta_j(u) - 1); service-driven rate into m from m+{u} is nu[u];
 *   - the coefficients are generated per target state exactly as
 *     Algorithm 3 does: walk each node's list over the busy units of m and
 *     credit lam[j] to every busy unit met before the first idle one;
 *   - Algorithm 1: initial p_n = 1/C(N,n), then outer iterations that sweep
 *     layers n = 1..N-1 in ascending order with the update (12), the inner
 *     mu(n) loop (12)+(14) and lambda(n) by (13); p(n) by (10) and
 *     P(m) = p(|m|) p_|m|(m) (Proposition 1);
 *   - the global balance residual of (1): sum_m |inflow - outflow| over
 *     sum_m P(m)(lambda_m + mu_m).
 *
 * Inner-loop modes for the mu(n) loop of Algorithm 1:
 *   ORC_INNER_CLOSED  : the limit of the inner loop.  With layers n-1 and n+1
 *                       held fixed, (12)+(14) make mu an affine map
 *                       mu -> A mu + B; the loop converges to B / (1 - A).
 *   ORC_INNER_LITERAL : repeat (12) then (14) until max |change| <= delta
 *                       (at least one update, starting from the previous
 *                       iteration's mu(n)).
 *   ORC_INNER_ONE     : exactly one update per layer (delta = infinity).
 *
 * Parity of the iteration path with the paper's own runs is unpinned: the
 * paper prints no per-iteration values.  The final distribution is pinned
 * (by the tests) against dense and sparse direct solves, closed forms and
 * invariants.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC hq_oracle.c -o libhq_oracle.so -lm
 * Per-state loops run under OpenMP; every sum is taken sequentially in
 * increasing state index, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_INNER_CLOSED = 0, ORC_INNER_LITERAL = 1, ORC_INNER_ONE = 2 };
enum { ORC_STOP_RESIDUAL = 0, ORC_STOP_DELTA = 1 };

/* number of OpenMP threads the oracle will use (1 without OpenMP) */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int popcount32(uint32_t x) { return __builtin_popcount(x); }

static double binom(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return floor(r + 0.5);
}

/* Algorithm 3 for one target state m: a[u] = arrival-driven rate from
 * m\{u} into m, for every u (0 for idle u).  For each node j, walk its list
 * from the most preferred unit; every busy unit met before the first idle
 * unit receives lam[j]. */
void orc_up_coefficients(int N, int J, const double* lam, const int32_t* pref,
                         uint32_t m, double* a) {
    for (int u = 0; u < N; ++u) a[u] = 0.0;
    for (int j = 0; j < J; ++j) {
        const int32_t* z = pref + (size_t)j * N;
        for (int h = 0; h < N; ++h) {
            int u = z[h];
            if (!((m >> u) & 1u)) break; /* first idle unit ends the walk */
            a[u] += lam[j];
        }
    }
}

/* total service rate mu_m = sum of nu over busy units */
static double state_mu(int N, const double* nu, uint32_t m) {
    double s = 0.0;
    for (int u = 0; u < N; ++u)
        if ((m >> u) & 1u) s += nu[u];
    return s;
}

/* Relative L1 global-balance residual of an unnormalised-or-normalised P
 * (bitmask order), eq. (1): inflow(m) = sum_{u in m} a(m,u) P(m\u)
 * + sum_{u notin m} nu_u P(m+u), outflow(m) = P(m)(lambda_m + mu_m), with
 * lambda_m = Lambda except for the all-busy state (0).  Coefficients come
 * from Algorithm 3 for each state; returns sum|in-out| / sum outflow.
 * If `terms` is non-NULL it receives (in - out) per state. */
double orc_residual(int N, int J, const double* lam, const double* nu,
                    const int32_t* pref, const double* P, double* terms) {
    const uint32_t S = 1u << N, full = S - 1u;
    double Lam = 0.0;
    for (int j = 0; j < J; ++j) Lam += lam[j];
    double* diff = (double*)malloc(sizeof(double) * S);
    double* outf = (double*)malloc(sizeof(double) * S);
#pragma omp parallel
    {
        double* a = (double*)malloc(sizeof(double) * (N > 0 ? N : 1));
#pragma omp for schedule(dynamic, 256)
        for (long long mm = 0; mm < (long long)S; ++mm) {
            uint32_t m = (uint32_t)mm;
            orc_up_coefficients(N, J, lam, pref, m, a);
            double in = 0.0;
            for (int u = 0; u < N; ++u) {
                uint32_t bit = 1u << u;
                if (m & bit) in += a[u] * P[m ^ bit];
                else in += nu[u] * P[m | bit];
            }
            double lm = (m == full) ? 0.0 : Lam;
            double out = P[m] * (lm + state_mu(N, nu, m));
            diff[m] = in - out;
            outf[m] = out;
        }
        free(a);
    }
    double num = 0.0, den = 0.0;
    for (uint32_t m = 0; m < S; ++m) {
        num += fabs(diff[m]);
        den += outf[m];
        if (terms) terms[m] = diff[m];
    }
    free(diff);
    free(outf);
    return den > 0.0 ? num / den : 0.0;
}

/* Layer lists: states of each popcount class in increasing index order. */
typedef struct {
    uint32_t* states; /* all 2^N states grouped by layer */
    size_t* start;    /* start[n] .. start[n+1] */
} layers_t;

static void build_layers(int N, layers_t* L) {
    const uint32_t S = 1u << N;
    L->states = (uint32_t*)malloc(sizeof(uint32_t) * S);
    L->start = (size_t*)calloc((size_t)N + 2, sizeof(size_t));
    for (uint32_t m = 0; m < S; ++m) L->start[popcount32(m) + 1]++;
    for (int n = 0; n <= N; ++n) L->start[n + 1] += L->start[n];
    size_t* fill = (size_t*)malloc(sizeof(size_t) * ((size_t)N + 1));
    for (int n = 0; n <= N; ++n) fill[n] = L->start[n];
    for (uint32_t m = 0; m < S; ++m) L->states[fill[popcount32(m)]++] = m;
    free(fill);
}

static void free_layers(layers_t* L) {
    free(L->states);
    free(L->start);
}

/*
 * Pieces of Algorithm 1 shared by orc_solve and the timing sample below.
 *
 * step2_coefficients: step 2 of Algorithm 1 (every coefficient once, by
 * Algorithm 3) for `count` states (states[i], or i when states is NULL):
 * mu[m] = mu_m and coef[m*N + u] = a(m, u).
 */
static void step2_coefficients(int N, int J, const double* lam, const double* nu, const int32_t* pref,
                               const uint32_t* states, long long count, double* mu, double* coef) {
#pragma omp parallel for schedule(dynamic, 256)
    for (long long i = 0; i < count; ++i) {
        uint32_t m = states ? states[i] : (uint32_t)i;
        mu[m] = state_mu(N, nu, m);
        orc_up_coefficients(N, J, lam, pref, m, coef + (size_t)m * N);
    }
}

/* The two parts of (12) that do not depend on the inner iterate, for the
 * states states[b..e) of one layer: U(m) = sum_{u in m} a(m,u) p(m\u) /
 * (Lambda + mu_m) and D(m) = sum_{u notin m} nu_u p(m+u) / (Lambda + mu_m). */
static void layer_parts(int N, const double* nu, double Lam, const double* coef, const double* mu,
                        const double* p, const uint32_t* states, size_t b, size_t e, double* U, double* D) {
#pragma omp parallel for schedule(dynamic, 256)
    for (long long ii = (long long)b; ii < (long long)e; ++ii) {
        uint32_t m = states[ii];
        const double* a = coef + (size_t)m * N;
        double up = 0.0, dn = 0.0;
        for (int u = 0; u < N; ++u) {
            uint32_t bit = 1u << u;
            if (m & bit) up += a[u] * p[m ^ bit]; /* from layer n-1, lambda_lm */
            else dn += nu[u] * p[m | bit];        /* from layer n+1, mu_lm = nu_u */
        }
        double den = Lam + mu[m]; /* lambda_m + mu_m, lambda_m = Lambda for n < N */
        U[m] = up / den;
        D[m] = dn / den;
    }
}

/* One step of the inner loop: pnew(m) = ratio U(m) + beta D(m) over the
 * layer; *change = max |pnew - previous pnew|; returns mu = sum mu_m pnew(m)
 * (eq. (14)). */
static double inner_step(const uint32_t* states, size_t b, size_t e, const double* U, const double* D,
                         const double* mu, double ratio, double beta, double* pnew, double* change) {
    double ch = 0.0, smu = 0.0;
    for (size_t i = b; i < e; ++i) {
        uint32_t m = states[i];
        double v = ratio * U[m] + beta * D[m];
        double d = fabs(v - pnew[m]);
        if (d > ch) ch = d;
        pnew[m] = v;
        smu += mu[m] * v;
    }
    *change = ch;
    return smu;
}

/* Commit a layer: p = pnew, the largest change, and the sums behind
 * lambda(n) (13) and mu(n) (14). */
static void commit_layer(const uint32_t* states, size_t b, size_t e, const double* pnew, const double* mu,
                         double* p, double* maxdelta, double* sp, double* smu) {
    double a = 0.0, c = 0.0, md = *maxdelta;
    for (size_t i = b; i < e; ++i) {
        uint32_t m = states[i];
        double d = fabs(pnew[m] - p[m]);
        if (d > md) md = d;
        p[m] = pnew[m];
        a += p[m];
        c += mu[m] * p[m];
    }
    *maxdelta = md;
    *sp = a;
    *smu = c;
}

/*
 * Full Algorithm 1.
 *
 * Inputs: N (1..26), J >= 1, lam[J] >= 0 with sum > 0, nu[N] > 0,
 * pref[J*N] (row j: units, most preferred first), inner mode and delta
 * (LITERAL only), stop mode and tol, max_iters, check_every (residual mode
 * checks every check_every iterations, and always at max_iters), init_p
 * (NULL = uniform 1/C(N,n), else conditional probabilities in bitmask order).
 *
 * Outputs (caller-allocated):
 *   P[2^N]     stationary distribution, bitmask order, renormalised to sum 1
 *   pcond[2^N] conditional layer probabilities p_n(m), bitmask order
 *   layer[3*(N+1)]  lambda(n), mu(n), p(n) for n = 0..N
 *   stats[8]   iterations, final residual, sum(P)-1 before renormalising,
 *              max layer normalisation drift max_n |sum p_n - 1| at the end,
 *              last max |p^k - p^(k-1)|, coefficient seconds, iteration
 *              seconds, threads
 *   trace[max_iters] (nullable): residual after each checked iteration (or
 *              -1 for unchecked ones)
 *   layer_trace (nullable): [max_iters * (N+1)] sum p_n after each iteration
 * Returns 0 on convergence, 1 if max_iters was reached, -1 on bad input.
 */
int orc_solve(int N, int J, const double* lam, const double* nu, const int32_t* pref,
              int inner_mode, double delta, int stop_mode, double tol, int max_iters,
              int check_every, const double* init_p, double* P, double* pcond,
              double* layer, double* stats, double* trace, double* layer_trace) {
    if (N < 1 || N > 26 || J < 1 || max_iters < 1) return -1;
    if (check_every < 1) check_every = 1;
    const uint32_t S = 1u << N, full = S - 1u;
    double Lam = 0.0;
    for (int j = 0; j < J; ++j) Lam += lam[j];
    struct timespec t0, t1, t2;
    clock_gettime(CLOCK_MONOTONIC, &t0);

    /* degenerate: no arrivals, the chain sits in the empty state */
    if (!(Lam > 0.0)) {
        for (uint32_t m = 0; m < S; ++m) {
            P[m] = (m == 0) ? 1.0 : 0.0;
            pcond[m] = 0.0;
        }
        for (int n = 0; n <= N; ++n) {
            layer[3 * n + 0] = 0.0;
            layer[3 * n + 1] = 0.0;
            layer[3 * n + 2] = (n == 0) ? 1.0 : 0.0;
        }
        pcond[0] = 1.0;
        memset(stats, 0, sizeof(double) * 8);
        stats[7] = orc_threads();
        return 0;
    }

    layers_t LY;
    build_layers(N, &LY);

    /* per-state service rate and the Algorithm-3 coefficient table
     * (step 2 of Algorithm 1 precomputes every coefficient once) */
    double* mu = (double*)malloc(sizeof(double) * S);
    double* coef = (double*)malloc(sizeof(double) * (size_t)S * N);
    step2_coefficients(N, J, lam, nu, pref, NULL, (long long)S, mu, coef);
    clock_gettime(CLOCK_MONOTONIC, &t1);

    double* p = pcond;
    double* U = (double*)malloc(sizeof(double) * S);
    double* D = (double*)malloc(sizeof(double) * S);
    double* pnew = (double*)malloc(sizeof(double) * S);
    double* lamn = (double*)malloc(sizeof(double) * (N + 1));
    double* mun = (double*)malloc(sizeof(double) * (N + 1));

    /* initialisation (Algorithm 1, step 2) */
    for (int n = 0; n <= N; ++n) {
        double c = 1.0 / binom(N, n);
        for (size_t i = LY.start[n]; i < LY.start[n + 1]; ++i) {
            uint32_t m = LY.states[i];
            p[m] = init_p ? init_p[m] : c;
        }
    }
    p[0] = 1.0;    /* p_0(empty) = 1 */
    p[full] = 1.0; /* p_N(full) = 1 */
    /* initial layer scalars from (13)-(14) */
    for (int n = 0; n <= N; ++n) {
        double sl = 0.0, sm = 0.0;
        for (size_t i = LY.start[n]; i < LY.start[n + 1]; ++i) {
            uint32_t m = LY.states[i];
            sl += p[m] * ((m == full) ? 0.0 : Lam);
            sm += p[m] * mu[m];
        }
        lamn[n] = sl;
        mun[n] = sm;
    }

    int k = 0, converged = 0;
    double res = -1.0, maxdelta = 0.0;
    while (k < max_iters) {
        ++k;
        maxdelta = 0.0;
        for (int n = 1; n <= N - 1; ++n) {
            const size_t b = LY.start[n], e = LY.start[n + 1];
            const double Lprev = lamn[n - 1];            /* lambda^k(n-1), already updated */
            const double beta = lamn[n] / mun[n + 1];    /* lambda^{k-1}(n) / mu^{k-1}(n+1) */
            /* the two r-independent parts of (12) for every state of the layer */
            layer_parts(N, nu, Lam, coef, mu, p, LY.states, b, e, U, D);
            double mu_star;
            if (inner_mode == ORC_INNER_CLOSED) {
                /* p(m) = (mu/Lprev) U(m) + beta D(m);  mu' = sum mu_m p(m) = A mu + B */
                double sA = 0.0, sB = 0.0;
                for (size_t i = b; i < e; ++i) {
                    uint32_t m = LY.states[i];
                    sA += mu[m] * U[m];
                    sB += mu[m] * D[m];
                }
                double A = sA / Lprev, B = beta * sB;
                mu_star = B / (1.0 - A);
                for (size_t i = b; i < e; ++i) {
                    uint32_t m = LY.states[i];
                    pnew[m] = (mu_star / Lprev) * U[m] + beta * D[m];
                }
            } else {
                /* literal inner loop, starting from mu^{k-1}(n) and the previous
                 * iteration's layer values */
                double mu_cur = mun[n];
                for (size_t i = b; i < e; ++i) pnew[LY.states[i]] = p[LY.states[i]];
                for (int r = 0;; ++r) {
                    double change = 0.0;
                    mu_cur = inner_step(LY.states, b, e, U, D, mu, mu_cur / Lprev, beta, pnew, &change);
                    if (inner_mode == ORC_INNER_ONE) break;
                    if (change <= delta || r > 1000000) break;
                }
                mu_star = mu_cur;
            }
            (void)mu_star;
            /* commit the layer and its scalars (13)-(14) */
            double sp = 0.0, smu = 0.0;
            commit_layer(LY.states, b, e, pnew, mu, p, &maxdelta, &sp, &smu);
            lamn[n] = Lam * sp;
            mun[n] = smu;
        }
        if (layer_trace) {
            for (int n = 0; n <= N; ++n) {
                double s = 0.0;
                for (size_t i = LY.start[n]; i < LY.start[n + 1]; ++i) s += p[LY.states[i]];
                layer_trace[(size_t)(k - 1) * (N + 1) + n] = s;
            }
        }
        int check = (stop_mode == ORC_STOP_RESIDUAL) && ((k % check_every) == 0 || k == max_iters);
        if (trace) trace[k - 1] = -1.0;
        if (stop_mode == ORC_STOP_DELTA) {
            if (maxdelta <= tol) {
                converged = 1;
                break;
            }
        } else if (check) {
            /* assemble P (10) and measure the balance residual (1) */
            double g = 1.0, G = 1.0;
            for (int n = 1; n <= N; ++n) {
                g = g * lamn[n - 1] / mun[n];
                G += g;
            }
            g = 1.0;
            for (int n = 0; n <= N; ++n) {
                if (n > 0) g = g * lamn[n - 1] / mun[n];
                double pn = g / G;
                for (size_t i = LY.start[n]; i < LY.start[n + 1]; ++i) {
                    uint32_t m = LY.states[i];
                    P[m] = pn * p[m];
                }
            }
            /* residual with the precomputed coefficients */
            double num = 0.0, den = 0.0;
            for (uint32_t m = 0; m < S; ++m) {
                const double* a = coef + (size_t)m * N;
                double in = 0.0;
                for (int u = 0; u < N; ++u) {
                    uint32_t bit = 1u << u;
                    if (m & bit) in += a[u] * P[m ^ bit];
                    else in += nu[u] * P[m | bit];
                }
                double out = P[m] * (((m == full) ? 0.0 : Lam) + mu[m]);
                num += fabs(in - out);
                den += out;
            }
            res = num / den;
            if (trace) trace[k - 1] = res;
            if (res <= tol) {
                converged = 1;
                break;
            }
        }
    }
    clock_gettime(CLOCK_MONOTONIC, &t2);

    /* Algorithm 1 steps 16-17: p(n) by (10), P = p(|m|) p_|m|(m) */
    double g = 1.0, G = 1.0;
    for (int n = 1; n <= N; ++n) {
        g = g * lamn[n - 1] / mun[n];
        G += g;
    }
    g = 1.0;
    double total = 0.0, drift = 0.0;
    for (int n = 0; n <= N; ++n) {
        if (n > 0) g = g * lamn[n - 1] / mun[n];
        double pn = g / G;
        layer[3 * n + 0] = lamn[n];
        layer[3 * n + 1] = mun[n];
        layer[3 * n + 2] = pn;
        double s = 0.0;
        for (size_t i = LY.start[n]; i < LY.start[n + 1]; ++i) {
            uint32_t m = LY.states[i];
            P[m] = pn * p[m];
            s += p[m];
        }
        if (fabs(s - 1.0) > drift) drift = fabs(s - 1.0);
    }
    for (uint32_t m = 0; m < S; ++m) total += P[m];
    for (uint32_t m = 0; m < S; ++m) P[m] /= total;
    if (stop_mode == ORC_STOP_DELTA || res < 0.0 || !converged)
        res = orc_residual(N, J, lam, nu, pref, P, NULL);

    stats[0] = k;
    stats[1] = res;
    stats[2] = total - 1.0;
    stats[3] = drift;
    stats[4] = maxdelta;
    stats[5] = (t1.tv_sec - t0.tv_sec) + 1e-9 * (t1.tv_nsec - t0.tv_nsec);
    stats[6] = (t2.tv_sec - t1.tv_sec) + 1e-9 * (t2.tv_nsec - t1.tv_nsec);
    stats[7] = orc_threads();

    free(mu);
    free(coef);
    free(U);
    free(D);
    free(pnew);
    free(lamn);
    free(mun);
    free_layers(&LY);
    return converged ? 0 : 1;
}

/*
 * Timing sample of Algorithm 1 (the CPU baseline of the benchmark), built
 * from the same pieces as orc_solve: step 2's coefficients (Algorithm 3)
 * for `count` consecutive states of layer n (colex order, starting at
 * position `first`), then `reps` outer-iteration updates of those states
 * with one inner step ((12), (14)) and the commit of (13)-(14), reading
 * neighbours from full-size layers held at 1/C(N, n -+ 1).  `threads` > 0
 * sets the OpenMP thread count for the call.
 *   out[4]: seconds of the coefficient step, seconds per update rep,
 *           threads used, a checksum of the updated values.
 * Returns 0, or -1 on bad input or allocation failure.
 */
int orc_time_sample(int N, int J, const double* lam, const double* nu, const int32_t* pref, int n,
                    long long first, long long count, int reps, int threads, double* out) {
    if (N < 2 || N > 26 || n < 1 || n > N - 1 || first < 0 || count < 1 || reps < 1) return -1;
    const uint32_t S = 1u << N;
    const double layer_n = binom(N, n);
    if ((double)(first + count) > layer_n) return -1;
#ifdef _OPENMP
    const int saved = omp_get_max_threads();
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    double Lam = 0.0;
    for (int j = 0; j < J; ++j) Lam += lam[j];
    /* the sample's states, in the order orc_solve visits layer n */
    uint32_t* st = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)count);
    double* mu = (double*)malloc(sizeof(double) * S);
    double* coef = (double*)malloc(sizeof(double) * (size_t)S * N); /* only the sample's rows are touched */
    double* p = (double*)malloc(sizeof(double) * S);
    double* U = (double*)malloc(sizeof(double) * S);
    double* D = (double*)malloc(sizeof(double) * S);
    double* pnew = (double*)malloc(sizeof(double) * S);
    int rc = 0;
    if (!st || !mu || !coef || !p || !U || !D || !pnew) {
        rc = -1;
    } else {
        long long pos = 0, k = 0;
        for (uint32_t m = 0; m < S && k < count; ++m)
            if (popcount32(m) == n) {
                if (pos >= first) st[k++] = m;
                ++pos;
            }
        double inv_c[33];
        for (int i = 0; i <= N; ++i) inv_c[i] = 1.0 / binom(N, i);
        for (uint32_t m = 0; m < S; ++m) p[m] = inv_c[popcount32(m)];
        struct timespec t0, t1, t2;
        clock_gettime(CLOCK_MONOTONIC, &t0);
        step2_coefficients(N, J, lam, nu, pref, st, count, mu, coef);
        clock_gettime(CLOCK_MONOTONIC, &t1);
        /* any positive layer scalars: the cost does not depend on them */
        const double ratio = 1.0 / Lam, beta = 1.0;
        double maxdelta = 0.0, sp = 0.0, smu = 0.0;
        for (int r = 0; r < reps; ++r) {
            double change = 0.0;
            layer_parts(N, nu, Lam, coef, mu, p, st, 0, (size_t)count, U, D);
            for (long long i = 0; i < count; ++i) pnew[st[i]] = p[st[i]];
            (void)inner_step(st, 0, (size_t)count, U, D, mu, ratio, beta, pnew, &change);
            commit_layer(st, 0, (size_t)count, pnew, mu, p, &maxdelta, &sp, &smu);
        }
        clock_gettime(CLOCK_MONOTONIC, &t2);
        out[0] = (t1.tv_sec - t0.tv_sec) + 1e-9 * (t1.tv_nsec - t0.tv_nsec);
        out[1] = ((t2.tv_sec - t1.tv_sec) + 1e-9 * (t2.tv_nsec - t1.tv_nsec)) / reps;
        out[2] = orc_threads();
        out[3] = sp + smu;
    }
    free(st);
    free(mu);
    free(coef);
    free(p);
    free(U);
    free(D);
    free(pnew);
#ifdef _OPENMP
    omp_set_num_threads(saved);
#endif
    return rc;
}

/*
 * One layer update of (12) for a sample of states, from caller-supplied
 * neighbour layers, with Algorithm-3 coefficients generated on demand for
 * each state (no table).  pl and pu are conditional probabilities in
 * bitmask order (only entries of layers n-1 and n+1 are read).  For each
 * states[i] (all in layer n, 1 <= n <= N-1): out[i] = alpha*U + beta*D,
 * U = sum_{u in m} a(m,u) pl(m\u) / (Lambda+mu_m),
 * D = sum_{u notin m} nu_u pu(m+u) / (Lambda+mu_m).
 * If outU/outD are non-NULL they receive U and D.
 */
void orc_update_states(int N, int J, const double* lam, const double* nu,
                       const int32_t* pref, long long count, const uint32_t* states,
                       const double* pl, const double* pu, double alpha, double beta,
                       double* out, double* outU, double* outD) {
    double Lam = 0.0;
    for (int j = 0; j < J; ++j) Lam += lam[j];
#pragma omp parallel
    {
        double* a = (double*)malloc(sizeof(double) * N);
#pragma omp for schedule(dynamic, 64)
        for (long long i = 0; i < count; ++i) {
            uint32_t m = states[i];
            orc_up_coefficients(N, J, lam, pref, m, a);
            double up = 0.0, dn = 0.0;
            for (int u = 0; u < N; ++u) {
                uint32_t bit = 1u << u;
                if (m & bit) up += a[u] * pl[m ^ bit];
                else dn += nu[u] * pu[m | bit];
            }
            double den = Lam + state_mu(N, nu, m);
            double Uv = up / den, Dv = dn / den;
            out[i] = alpha * Uv + beta * Dv;
            if (outU) outU[i] = Uv;
            if (outD) outD[i] = Dv;
        }
        free(a);
    }
}

/* Sums over a whole layer n of U(m), mu_m U(m), D(m), mu_m D(m) (U, D as in
 * orc_update_states), taken in increasing state order.  out[4]. */
void orc_layer_sums(int N, int J, const double* lam, const double* nu, const int32_t* pref,
                    int n, const double* pl, const double* pu, double* out) {
    const uint32_t S = 1u << N;
    long long cnt = 0;
    for (uint32_t m = 0; m < S; ++m)
        if (popcount32(m) == n) ++cnt;
    uint32_t* st = (uint32_t*)malloc(sizeof(uint32_t) * (cnt > 0 ? cnt : 1));
    long long c = 0;
    for (uint32_t m = 0; m < S; ++m)
        if (popcount32(m) == n) st[c++] = m;
    double* o = (double*)malloc(sizeof(double) * (cnt > 0 ? cnt : 1));
    double* U = (double*)malloc(sizeof(double) * (cnt > 0 ? cnt : 1));
    double* D = (double*)malloc(sizeof(double) * (cnt > 0 ? cnt : 1));
    orc_update_states(N, J, lam, nu, pref, cnt, st, pl, pu, 0.0, 0.0, o, U, D);
    double s[4] = {0, 0, 0, 0};
    for (long long i = 0; i < cnt; ++i) {
        double mum = state_mu(N, nu, st[i]);
        s[0] += U[i];
        s[1] += mum * U[i];
        s[2] += D[i];
        s[3] += mum * D[i];
    }
    for (int i = 0; i < 4; ++i) out[i] = s[i];
    free(st);
    free(o);
    free(U);
    free(D);
}

/* Per-unit busy probabilities rho_u = sum_{m containing u} P(m), and the
 * number-busy marginal pn[n] = sum_{|m| = n} P(m), from P in bitmask order. */
void orc_marginals(int N, const double* P, double* rho, double* pn) {
    const uint32_t S = 1u << N;
    for (int u = 0; u < N; ++u) rho[u] = 0.0;
    for (int n = 0; n <= N; ++n) pn[n] = 0.0;
    for (uint32_t m = 0; m < S; ++m) {
        pn[popcount32(m)] += P[m];
        for (int u = 0; u < N; ++u)
            if ((m >> u) & 1u) rho[u] += P[m];
    }
}

/* Balance terms of (1) for sampled states: out[i] = inflow - outflow at
 * states[i], and outflow[i] = P(m)(lambda_m + mu_m), with P in bitmask order
 * and Algorithm-3 coefficients generated per state. */
void orc_balance_terms(int N, int J, const double* lam, const double* nu, const int32_t* pref,
                       long long count, const uint32_t* states, const double* P, double* out,
                       double* outflow) {
    const uint32_t full = (N >= 32) ? 0xffffffffu : ((1u << N) - 1u);
    double Lam = 0.0;
    for (int j = 0; j < J; ++j) Lam += lam[j];
#pragma omp parallel
    {
        double* a = (double*)malloc(sizeof(double) * N);
#pragma omp for schedule(dynamic, 64)
        for (long long i = 0; i < count; ++i) {
            uint32_t m = states[i];
            orc_up_coefficients(N, J, lam, pref, m, a);
            double in = 0.0;
            for (int u = 0; u < N; ++u) {
                uint32_t bit = 1u << u;
                if (m & bit) in += a[u] * P[m ^ bit];
                else in += nu[u] * P[m | bit];
            }
            double o = P[m] * (((m == full) ? 0.0 : Lam) + state_mu(N, nu, m));
            out[i] = in - o;
            outflow[i] = o;
        }
        free(a);
    }
}

/*
 * Birth-death marginal of the buffered system, Proposition 2 and the remark
 * after it (Section 2.2).  With a waiting room of C calls the conditional
 * layer probabilities p_n are those of the loss system; only the marginal
 * changes: lambda(N) = Lambda (an arrival at the full state waits),
 * lambda(n) = Lambda for N < n < N + C, lambda(N + C) = 0, and
 * mu(n) = sum_i nu_i for n > N.  G(n) is the running product of
 * lambda(n-1) / mu(n); p(n) = G(n) p(0) with p(0) = 1 / sum_n G(n).
 *   lamn, mun: lambda(n), mu(n) for n = 0..N of a loss-system solve
 *              (lamn[N] is not used);
 *   C: waiting room (C >= 0); C < 0 means unlimited, which needs
 *      Lambda < sum_i nu_i (the geometric series of the remark);
 *   p: [N + 1] out, p(n) for n = 0..N (all units busy and nobody waiting
 *      for n = N);
 *   tail: [C] out (nullable; finite C only), P~{c} = p(N + c);
 *   summary: [4] out: P(all units busy), P(at least one call waits),
 *      mean number waiting, P(an arrival is lost).
 * Returns 0, or -1 for an unlimited room that is not stable.
 */
int orc_birth_death(int N, const double* lamn, const double* mun, double Lam, double sum_nu, int C,
                    double* p, double* tail, double* summary) {
    const double rho = Lam / sum_nu;
    if (C < 0 && !(rho < 1.0)) return -1;
    /* G(n) for n <= N by the product of the ratios */
    double* g = (double*)malloc(sizeof(double) * (N + 1));
    g[0] = 1.0;
    for (int n = 1; n <= N; ++n) g[n] = g[n - 1] * lamn[n - 1] / mun[n];
    double Z = 0.0;
    for (int n = 0; n <= N; ++n) Z += g[n];
    /* G(N + c) = G(N) rho^c, c = 1..C, summed term by term (finite) or as
     * the geometric series rho / (1 - rho) (unlimited) */
    double wait = 0.0, wait_mean = 0.0;
    if (C > 0) {
        double r = 1.0;
        for (int c = 1; c <= C; ++c) {
            r *= rho;
            wait += g[N] * r;
            wait_mean += c * g[N] * r;
        }
    } else if (C < 0) {
        wait = g[N] * rho / (1.0 - rho);
        wait_mean = g[N] * rho / ((1.0 - rho) * (1.0 - rho));
    }
    Z += wait;
    for (int n = 0; n <= N; ++n) p[n] = g[n] / Z;
    if (tail && C > 0) {
        double r = 1.0;
        for (int c = 1; c <= C; ++c) {
            r *= rho;
            tail[c - 1] = g[N] * r / Z;
        }
    }
    summary[0] = p[N] + wait / Z;
    summary[1] = wait / Z;
    summary[2] = wait_mean / Z;
    /* arrivals see time averages: lost at the full state (C = 0) or with
     * the waiting room full (C > 0); never with unlimited room */
    if (C == 0) summary[3] = p[N];
    else if (C > 0) summary[3] = g[N] * pow(rho, C) / Z;
    else summary[3] = 0.0;
    free(g);
    return 0;
}

/*
 * Dispatch probabilities of the loss system (the performance measures named
 * in Section 1: unit workloads and response times): for a call from node j,
 * the probability that unit u is the one sent, i.e. that u is the first
 * unit of node j's list that is idle.  Arrivals see time averages, so
 *   q[j * N + u] = sum_m P(m) [first idle unit of pref row j in m is u].
 * Brute force over every state and node, O(2^N J N).  sum_u q[j * N + u] is
 * 1 - P(all busy).
 */
void orc_dispatch(int N, int J, const int32_t* pref, const double* P, double* q) {
    const uint32_t S = 1u << N;
    memset(q, 0, sizeof(double) * (size_t)J * N);
#pragma omp parallel for schedule(dynamic, 4)
    for (int j = 0; j < J; ++j) {
        const int32_t* row = pref + (size_t)j * N;
        double* qj = q + (size_t)j * N;
        for (uint32_t m = 0; m < S; ++m) {
            for (int h = 0; h < N; ++h) {
                const int u = row[h];
                if (!((m >> u) & 1u)) {
                    qj[u] += P[m];
                    break;
                }
            }
        }
    }
}
