// The layer scalars of the previous layer formed at the start of the next
// layer's launch.  In an outer iteration every layer launch writes one
// partial per work-group (Σ p_n, Σ mu_m p_n, max change, -, Σ p_n w,
// Σ p_n z).  Instead of a one-work-group finalize launch after each layer,
// every work-group of the next layer's launch adds the previous layer's
// partials in the finalize kernel's fixed order (so all of them, and the
// unfused path, hold bitwise the same totals), uses lambda^k(n-1) = Lambda
// Σ p_{n-1} (13) and, for the look-ahead closed form, alpha_n, and work-group
// 0 records the previous layer's scalars the way the finalize launch does.
// Only small layers are fused this way (few partials to read per
// work-group), where the launch of a one-work-group kernel costs as much as
// the layer itself.  Consecutive layers write their partials to alternating
// halves of the partials buffer.  Included by the kernel sources only.
#pragma once

#include "hq_internal.h"

namespace hqfuse {

// the previous layer's partials to reduce first, or prev == nullptr
struct FuseArgs {
    const double* prev;
    uint32_t prev_count;
};

__device__ __forceinline__ double fsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ __forceinline__ double fmx(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}

// Fixed-order reduction of `count` partials, the result in every thread
// (the same arithmetic as the finalize kernel's reduction).  Uses `red`
// (HQ_NPART x waves doubles of LDS) and one work-group barrier pair.
template <int WG>
__device__ __forceinline__ void sum_partials_all(const double* partials, uint32_t count, double out[HQ_NPART],
                                                 double (*red)[WG / 64]) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double c[HQ_NPART] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (uint32_t i = tid; i < count; i += WG) {
        const double* pp = partials + (size_t)i * HQ_NPART;
        c[0] += pp[0];
        c[1] += pp[1];
        c[2] = fmax(c[2], pp[2]);
        c[3] = fmax(c[3], pp[3]);
        c[4] += pp[4];
        c[5] += pp[5];
    }
    c[0] = fsum(c[0]);
    c[1] = fsum(c[1]);
    c[2] = fmx(c[2]);
    c[3] = fmx(c[3]);
    c[4] = fsum(c[4]);
    c[5] = fsum(c[5]);
    if (lane == 0)
        for (int j = 0; j < HQ_NPART; ++j) red[j][w] = c[j];
    __syncthreads();
    double d[HQ_NPART] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < WG / 64; ++i) {
        d[0] += red[0][i];
        d[1] += red[1][i];
        d[2] = fmax(d[2], red[2][i]);
        d[3] = fmax(d[3], red[3][i]);
        d[4] += red[4][i];
        d[5] += red[5][i];
    }
    for (int j = 0; j < HQ_NPART; ++j) out[j] = d[j];
    __syncthreads();  // red may be reused
}

// The scalars of layer n's sweep that the previous layer's write changes.
struct Prev {
    double lam_prev;  // lambda^k(n-1)
    double alpha_la;  // look-ahead closed form: alpha_n (else unused)
};

// Reduce layer n-1's partials and form lambda^k(n-1) (and alpha_n with the
// look-ahead); work-group 0 records layer n-1's scalars as the finalize
// launch of an M_WRITE would (inner_one: 0 closed, 1 one update).
template <int WG>
__device__ __forceinline__ Prev prologue(const SweepParams& P, int n, int inner_one, const FuseArgs& F,
                                         double (*red)[WG / 64]) {
    double tot[HQ_NPART];
    sum_partials_all<WG>(F.prev, F.prev_count, tot, red);
    Prev r;
    r.lam_prev = P.Lam * tot[0];
    r.alpha_la = 0.0;
    const int m = n - 1;
    if (P.la) {
        // alpha_n = beta_n S_muD(n) / (Lambda S_U(n)), S_U(n) = Σ p_{n-1} w
        const double beta = P.sc.lam[n] / P.sc.mu[n + 1];
        r.alpha_la = beta * P.sc.zsum[n + 1] / (P.Lam * tot[4]);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const double used = inner_one == 1 ? P.sc.mu[m] / P.sc.lam[m - 1] : P.sc.alpha[m];
        const double mu = tot[1];
        if (!isfinite(r.lam_prev) || !(mu > 0.0) || !isfinite(mu)) P.sc.misc[2] = 1.0;
        P.sc.lam[m] = r.lam_prev;
        P.sc.mu[m] = mu;
        P.sc.alpha[m] = used;
        P.sc.delta[m] = tot[2];
        if (P.la) {
            P.sc.wsum[m] = tot[4];
            P.sc.zsum[m] = tot[5];
            if (!(tot[4] > 0.0) || !isfinite(r.alpha_la)) P.sc.misc[2] = 1.0;
            P.sc.alpha[n] = r.alpha_la;
        }
    }
    return r;
}

}  // namespace hqfuse
