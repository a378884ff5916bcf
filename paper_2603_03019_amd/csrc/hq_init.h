// Host-side weights of the product-form starting iterate (no HIP; also built
// by a CPU checker).
//
// The start is p_n(m) = prod_{u in m} x_u / e_n(x) inside each layer n,
// with e_n the elementary symmetric polynomials of x. The solver derives the
// layer law p(n) of the start from its own lambda(n), mu(n) by the
// birth-death product (10) (Proposition 1). The busy probabilities of the
// assembled start are therefore not the odds x_u / (1 + x_u) but
//   rho_u(x) = sum_n p(n) x_u e_{n-1}(x without u) / e_n(x)  (+ waiting mass).
// calibrate() looks for x with rho(x) equal to given target utilisations, so
// a predicted utilisation is also the utilisation of the start it seeds.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

namespace hqinit {

// e[0..n] of the values v[0..n-1] (v may hold any positive weights).
inline void elementary(const double* v, int n, double* e) {
    e[0] = 1.0;
    for (int k = 1; k <= n; ++k) e[k] = 0.0;
    for (int i = 0; i < n; ++i)
        for (int k = i + 1; k >= 1; --k) e[k] += v[i] * e[k - 1];
}

// Busy probability of each unit under the start with weights x[N]: layer
// laws from the product form, layer weights from the birth-death law with
// lambda(n) = Lam for n < N, mu(n) = sum_u nu_u P(u busy | layer n), and
// with a waiting room (C > 0 places, C < 0 unlimited, C = 0 none) the
// states above layer N, in which every unit is busy, at rates Lam and
// sum nu. Returns false if a value is not finite.
inline bool start_utilisation(int N, const double* x, const double* nu, double Lam, int C, double* rho) {
    std::vector<double> e(N + 1), eu(N + 1), rest(N > 0 ? N - 1 : 0);
    std::vector<double> cond((size_t)N * (N + 1), 0.0), mu_n(N + 1, 0.0);
    elementary(x, N, e.data());
    for (int u = 0; u < N; ++u) {
        int j = 0;
        for (int v = 0; v < N; ++v)
            if (v != u) rest[j++] = x[v];
        elementary(rest.data(), N - 1, eu.data());
        for (int n = 1; n <= N; ++n) {
            const double c = x[u] * eu[n - 1] / e[n];  // P(u busy | layer n)
            cond[(size_t)u * (N + 1) + n] = c;
            mu_n[n] += nu[u] * c;
        }
    }
    // log g(n) = sum_{k <= n} log(Lam / mu(k))
    std::vector<double> lg(N + 1, 0.0);
    for (int n = 1; n <= N; ++n) lg[n] = lg[n - 1] + std::log(Lam / mu_n[n]);
    double sum_nu = 0.0;
    for (int u = 0; u < N; ++u) sum_nu += nu[u];
    const double a = Lam / sum_nu;
    double tail = 0.0;  // waiting states relative to g(N)
    if (C > 0) {
        double t = 1.0;
        for (int c = 1; c <= C; ++c) tail += (t *= a);
    } else if (C < 0) {
        tail = a / (1.0 - a);
    }
    const double top = *std::max_element(lg.begin(), lg.end());
    std::vector<double> p(N + 1);
    double tot = 0.0;
    for (int n = 0; n <= N; ++n) tot += (p[n] = std::exp(lg[n] - top));
    const double wait = p[N] * tail;
    tot += wait;
    bool ok = std::isfinite(tot) && tot > 0.0;
    for (int u = 0; u < N; ++u) {
        double r = wait;
        for (int n = 1; n <= N; ++n) r += p[n] * cond[(size_t)u * (N + 1) + n];
        rho[u] = r / tot;
        ok = ok && std::isfinite(rho[u]);
    }
    return ok;
}

// Weights x[N] whose start has the target utilisations, by the odds-ratio
// fixed point x_u <- x_u * odds(target_u) / odds(rho_u(x)), started from
// x_u = odds(target_u) (targets clamped to [1e-6, 1 - 1e-6]). Targets that
// no start can meet (they need not balance flows) leave the closest iterate
// found, in max |rho(x) - target|, which is returned.
inline double calibrate(int N, const double* target, const double* nu, double Lam, int C, double* x,
                        int max_steps = 200, double tol = 1e-12) {
    std::vector<double> t(N), r(N), best(N);
    for (int u = 0; u < N; ++u) {
        t[u] = std::min(std::max(target[u], 1e-6), 1.0 - 1e-6);
        x[u] = t[u] / (1.0 - t[u]);
    }
    double best_err = INFINITY;
    for (int step = 0; step <= max_steps; ++step) {
        if (!start_utilisation(N, x, nu, Lam, C, r.data())) break;
        double err = 0.0;
        for (int u = 0; u < N; ++u) err = std::max(err, std::fabs(r[u] - t[u]));
        if (err < best_err) {
            best_err = err;
            best.assign(x, x + N);
        }
        if (err <= tol || step == max_steps) break;
        for (int u = 0; u < N; ++u) {
            const double ru = std::min(std::max(r[u], 1e-300), 1.0 - 1e-16);
            const double f = (t[u] / (1.0 - t[u])) * ((1.0 - ru) / ru);
            x[u] = std::min(std::max(x[u] * f, 1e-9), 1e9);  // e_n stays finite for N <= 30
        }
    }
    if (std::isfinite(best_err)) std::copy(best.begin(), best.end(), x);
    return best_err;
}

}  // namespace hqinit
