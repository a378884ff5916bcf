// HIP kernels of the layer sweep (gfx950).
//
// State layout.  The conditional probabilities p_n(m) of all layers are one
// vector, layer after layer (layer n = states with n busy units, Section
// 2.2), each layer in colexicographic order (increasing bitmask).  A state
// m splits into a high part T (bits b..N-1, the "tile") and a low part L
// (bits 0..b-1) with q = |L|.  Inside a layer the states of one tile and
// one q form a contiguous "segment" of C(b, q) entries, ordered by the
// colex rank of L.  Flipping a high bit keeps L, so the neighbour sits at
// the SAME offset inside segment (T xor u, q) of layer n +- 1: a work-group
// that owns segment (T, q) reads its high-bit neighbours as contiguous,
// coalesced runs.  Low-bit neighbours stay in the small segments (T, q +- 1)
// and are found through a 2^b rank table held in LDS.
//
// Dispatch.  The arrival coefficient a(m, u) of eq. (3) / Algorithm 3 is
// evaluated on the fly from a merged preference trie.  Units are relabelled
// on the host so that the low (per-lane) bits are the units that demand
// nodes rank late; the part of the trie walk that depends only on T is
// precomputed per tile (tcoef), and only the remainder below a low unit is
// walked here, wave-uniformly, with per-lane subset tests.
//
// Each kernel ends with a deterministic two-level FP64 reduction: wave
// shuffles, one partial per work-group, and a fixed-order sum by the last
// work-group to finish, which also derives the layer scalars.
#include "hq_internal.h"

#include <math.h>

namespace hq {

enum Mode { M_PASS1 = 0, M_WRITE = 1, M_RESID = 2 };

__device__ __forceinline__ uint32_t C(const uint32_t* tb, int n, int k) {
    return (k < 0 || k > n) ? 0u : tb[n * 32 + k];
}

// Colex rank offset of the high part of a state: the sum over the i-th set
// bit of T (i = 1, 2, ...), at absolute position b + k, of C(b + k, q + i).
// Adding the colex rank of the low part gives the rank inside the layer.
__device__ __forceinline__ uint32_t tile_off(const uint32_t* tb, int b, uint32_t Tb, int q) {
    uint32_t off = 0;
    int i = 0;
    while (Tb) {
        const int k = __ffs(Tb) - 1;
        Tb &= Tb - 1;
        ++i;
        off += C(tb, b + k, q + i);
    }
    return off;
}

// Work-group -> (q, T): segments are ordered by q, then by the colex rank of
// T among the (n - q)-subsets of the H high bits.
__device__ __forceinline__ void decode_segment(const SweepParams& P, const LayerArgs& A, uint32_t g,
                                               int& q, uint32_t& Tb) {
    int qi = 0;
    while (A.qlo + qi < A.qhi && g >= A.seg_start[qi + 1]) ++qi;
    q = A.qlo + qi;
    uint32_t r = g - A.seg_start[qi];
    const int h = A.n - q;
    Tb = 0;
    int top = P.H;
    for (int i = h; i >= 1; --i) {
        int c = top - 1;
        while (C(P.binom, c, i) > r) --c;
        Tb |= 1u << c;
        r -= C(P.binom, c, i);
        top = c;
    }
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}

__device__ __forceinline__ void store_partial(double* p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), __double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_partial(const double* p) {
    return __longlong_as_double(__hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Reduce three per-thread values over the work-group, publish one partial,
// and return true in the last work-group of the grid with the grid totals
// in out[0..2] (sum, sum, max), summed in a fixed order.
__device__ bool grid_reduce3(double a0, double a1, double a2, double* partials,
                             unsigned int* counter, double out[3]) {
    __shared__ double s_red[3][HQ_WG / 64];
    __shared__ unsigned s_last;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_max(a2);
    if (lane == 0) {
        s_red[0][w] = a0;
        s_red[1][w] = a1;
        s_red[2][w] = a2;
    }
    __syncthreads();
    if (tid == 0) {
        double b0 = 0.0, b1 = 0.0, b2 = 0.0;
        for (int i = 0; i < HQ_WG / 64; ++i) {
            b0 += s_red[0][i];
            b1 += s_red[1][i];
            b2 = fmax(b2, s_red[2][i]);
        }
        double* pp = partials + (size_t)blockIdx.x * HQ_NPART;
        store_partial(pp + 0, b0);
        store_partial(pp + 1, b1);
        store_partial(pp + 2, b2);
        const unsigned t = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (t == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return false;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double c0 = 0.0, c1 = 0.0, c2 = 0.0;
    for (uint32_t i = tid; i < gridDim.x; i += HQ_WG) {
        const double* pp = partials + (size_t)i * HQ_NPART;
        c0 += load_partial(pp + 0);
        c1 += load_partial(pp + 1);
        c2 = fmax(c2, load_partial(pp + 2));
    }
    c0 = wave_sum(c0);
    c1 = wave_sum(c1);
    c2 = wave_max(c2);
    __syncthreads();
    if (lane == 0) {
        s_red[0][w] = c0;
        s_red[1][w] = c1;
        s_red[2][w] = c2;
    }
    __syncthreads();
    if (tid == 0) {
        double d0 = 0.0, d1 = 0.0, d2 = 0.0;
        for (int i = 0; i < HQ_WG / 64; ++i) {
            d0 += s_red[0][i];
            d1 += s_red[1][i];
            d2 = fmax(d2, s_red[2][i]);
        }
        out[0] = d0;
        out[1] = d1;
        out[2] = d2;
        __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return true;
}

// ---------------------------------------------------------------------------
// The layer kernel.  MODE:
//   M_PASS1  closed inner form, first pass: reduce S_U = sum U~(m) and
//            S_muD = sum mu_m D~(m) over the layer, then alpha_n.
//   M_WRITE  update (12): p_n(m) = alpha_n U~(m) + beta_n D~(m), write it,
//            reduce lambda(n) = Lambda sum p_n and mu(n) = sum mu_m p_n.
//   M_RESID  balance residual of (1) for the states of layer n.
// with U~(m) = sum_{u in m} a(m,u) p_{n-1}(m\u) / (Lambda + mu_m) and
//      D~(m) = sum_{u notin m} nu_u p_{n+1}(m+u) / (Lambda + mu_m).
// ---------------------------------------------------------------------------
template <typename T, int MODE, bool TRACK_DELTA>
__global__ __launch_bounds__(HQ_WG) void layer_kernel(SweepParams P, LayerArgs A, T* __restrict__ x,
                                                      int inner_one) {
    __shared__ uint32_t s_offD[HQ_MAXH], s_offU[HQ_MAXH];
    __shared__ uint32_t s_seg[4];
    __shared__ uint16_t s_rank[1 << HQ_MAXB];

    const int tid = threadIdx.x;
    const int n = A.n, b = P.b, H = P.H, N = P.N;
    int q;
    uint32_t Tb;
    decode_segment(P, A, blockIdx.x, q, Tb);

    if (tid < H) {
        const uint32_t bit = 1u << tid;
        if (Tb & bit)
            s_offD[tid] = P.layer_off[n - 1] + tile_off(P.binom, b, Tb ^ bit, q);
        else if (n < N)
            s_offU[tid] = P.layer_off[n + 1] + tile_off(P.binom, b, Tb | bit, q);
    } else if (tid == H) {
        s_seg[0] = (q >= 1) ? P.layer_off[n - 1] + tile_off(P.binom, b, Tb, q - 1) : 0u;
    } else if (tid == H + 1) {
        s_seg[1] = (q < b && n < N) ? P.layer_off[n + 1] + tile_off(P.binom, b, Tb, q + 1) : 0u;
    } else if (tid == H + 2) {
        s_seg[2] = P.layer_off[n] + tile_off(P.binom, b, Tb, q);
    }
    for (int i = tid; i < (1 << b); i += HQ_WG) s_rank[i] = P.lo_rank[i];
    __syncthreads();

    const uint32_t Tabs = Tb << b;
    double mu_hi = 0.0;
    for (int k = 0; k < H; ++k)
        if ((Tb >> k) & 1u) mu_hi += P.nu[b + k];
    const uint32_t cnt = C(P.binom, b, q);
    const double* tc = P.tcoef + (size_t)Tb * N;
    const uint32_t r0 = P.root_off[Tb], r1 = P.root_off[Tb + 1];
    const double is_dn = (n >= 1) ? P.inv_scale[n - 1] : 0.0;
    const double is_up = (n < N) ? P.inv_scale[n + 1] : 0.0;
    const double s_self = P.scale[n], is_self = P.inv_scale[n];
    const uint32_t offDlo = s_seg[0], offUlo = s_seg[1], offSelf = s_seg[2];

    double alpha = 0.0, beta = 0.0, pdn = 0.0, pself = 0.0, pup = 0.0;
    if (MODE == M_PASS1 || MODE == M_WRITE) {
        beta = P.sc.lam[n] / P.sc.mu[n + 1];  // lambda^{k-1}(n) / mu^{k-1}(n+1)
        if (MODE == M_WRITE)
            alpha = inner_one ? P.sc.mu[n] / P.sc.lam[n - 1]  // mu^{k-1}(n) / lambda^k(n-1)
                              : P.sc.alpha[n];                // closed-form limit (first pass)
    } else {
        pdn = (n >= 1) ? P.sc.pn[n - 1] : 0.0;
        pself = P.sc.pn[n];
        pup = (n < N) ? P.sc.pn[n + 1] : 0.0;
    }
    const uint32_t full = (N >= 32) ? 0xffffffffu : ((1u << N) - 1u);

    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    for (uint32_t t = tid; t < cnt; t += HQ_WG) {
        const uint32_t L = P.lo_unrank[P.lo_qstart[q] + t];
        const uint32_t m = Tabs | L;
        double U = 0.0, D = 0.0;
        // high units: segment-aligned, coalesced neighbours
        for (int k = 0; k < H; ++k) {
            if ((Tb >> k) & 1u)
                U += tc[b + k] * (double)x[s_offD[k] + t];
            else
                D += P.nu[b + k] * (double)x[s_offU[k] + t];
        }
        // low units: neighbours in segments (T, q -+ 1)
        for (int l = 0; l < b; ++l) {
            const uint32_t bit = 1u << l;
            const bool busy = (L & bit) != 0u;
            const uint32_t idx = (busy ? offDlo : offUlo) + s_rank[L ^ bit];
            const double v = (double)x[idx];
            if (busy)
                U += tc[l] * v;
            else
                D += P.nu[l] * v;
        }
        // per-lane remainder of the dispatch walk (subtrees below low units)
        for (uint32_t r = r0; r < r1; ++r) {
            uint32_t i = P.root_list[r];
            const uint32_t end = P.nodes[i].skip_unit >> 5;
            while (i < end) {
                const TrieNode nd = P.nodes[i];
                const bool c = (m & nd.need) == nd.need;
                if (!__any(c)) {
                    i = nd.skip_unit >> 5;
                    continue;
                }
                if (c) {
                    const int u = (int)(nd.skip_unit & 31u);
                    const uint32_t idx = (u >= b) ? s_offD[u - b] + t : offDlo + s_rank[L ^ (1u << u)];
                    U += nd.rate * (double)x[idx];
                }
                ++i;
            }
        }
        U *= is_dn;
        D *= is_up;
        const double mu_m = mu_hi + P.mu_lo[L];
        if (MODE == M_RESID) {
            const double lm = (m == full) ? 0.0 : P.Lam;
            const double self = (double)x[offSelf + t] * is_self;
            const double in = pdn * U + pup * D;
            const double out = pself * self * (lm + mu_m);
            acc0 += fabs(in - out);
            acc1 += out;
        } else {
            const double inv = 1.0 / (P.Lam + mu_m);
            const double Ut = U * inv, Dt = D * inv;
            if (MODE == M_PASS1) {
                acc0 += Ut;
                acc1 += mu_m * Dt;
            } else {
                const double p = alpha * Ut + beta * Dt;
                const uint32_t o = offSelf + t;
                if (TRACK_DELTA) acc2 = fmax(acc2, fabs(p - (double)x[o] * is_self));
                const T stored = (T)(p * s_self);
                x[o] = stored;
                const double ps = (double)stored * is_self;
                acc0 += ps;
                acc1 += mu_m * ps;
            }
        }
    }

    double tot[3];
    if (grid_reduce3(acc0, acc1, acc2, P.partials, P.counters + n, tot) && tid == 0) {
        double* misc = P.sc.misc;
        if (MODE == M_PASS1) {
            // mu* = B / (1 - A) with A = sum mu U~ / lambda(n-1) = 1 - Lambda S_U / lambda(n-1)
            // (since sum (Lambda + mu_m) U~ = lambda(n-1)), so alpha = mu*/lambda(n-1)
            // = beta S_muD / (Lambda S_U).
            const double a = beta * tot[1] / (P.Lam * tot[0]);
            if (!(tot[0] > 0.0) || !isfinite(a)) misc[2] = 1.0;
            P.sc.alpha[n] = a;
        } else if (MODE == M_WRITE) {
            const double lam = P.Lam * tot[0], mu = tot[1];
            if (!isfinite(lam) || !(mu > 0.0) || !isfinite(mu)) misc[2] = 1.0;
            P.sc.lam[n] = lam;
            P.sc.mu[n] = mu;
            P.sc.alpha[n] = alpha;
            P.sc.delta[n] = tot[2];
        } else {
            P.sc.rnum[n] = tot[0];
            P.sc.rden[n] = tot[1];
            if (!isfinite(tot[0]) || !isfinite(tot[1])) misc[2] = 1.0;
        }
    }
}

// Initial iterate of one layer: uniform 1/C(N,n) (Algorithm 1 step 2),
// product form prod_{u in m} x_u / e_n(x), or a given state (bitmask order,
// original unit labels mapped through `orig`).  Reduces lambda(n), mu(n).
template <typename T>
__global__ __launch_bounds__(HQ_WG) void init_kernel(SweepParams P, LayerArgs A, T* __restrict__ x,
                                                     const double* __restrict__ xu,
                                                     const double* __restrict__ given,
                                                     const uint32_t* __restrict__ orig_bit) {
    __shared__ uint32_t s_off;
    const int tid = threadIdx.x;
    const int n = A.n, b = P.b, H = P.H, N = P.N;
    int q;
    uint32_t Tb;
    decode_segment(P, A, blockIdx.x, q, Tb);
    if (tid == 0) s_off = P.layer_off[n] + tile_off(P.binom, b, Tb, q);
    __syncthreads();
    const uint32_t Tabs = Tb << b;
    double mu_hi = 0.0;
    for (int k = 0; k < H; ++k)
        if ((Tb >> k) & 1u) mu_hi += P.nu[b + k];
    const uint32_t cnt = C(P.binom, b, q);
    const double sc_self = P.scale[n], is_self = P.inv_scale[n];
    double acc0 = 0.0, acc1 = 0.0;
    for (uint32_t t = tid; t < cnt; t += HQ_WG) {
        const uint32_t L = P.lo_unrank[P.lo_qstart[q] + t];
        const uint32_t m = Tabs | L;
        double p;
        if (n == 0 || n == N) {
            p = 1.0;
        } else if (A.init_mode == 1) {
            double pr = 1.0;
            for (int u = 0; u < N; ++u)
                if ((m >> u) & 1u) pr *= xu[u];
            p = pr / A.e_n;
        } else if (A.init_mode == 2) {
            uint32_t mo = 0;
            for (int u = 0; u < N; ++u)
                if ((m >> u) & 1u) mo |= orig_bit[u];
            p = given[mo];
        } else {
            p = 1.0 / (double)C(P.binom, N, n);
        }
        const T stored = (T)(p * sc_self);
        x[s_off + t] = stored;
        const double ps = (double)stored * is_self;
        acc0 += ps;
        acc1 += (mu_hi + P.mu_lo[L]) * ps;
    }
    double tot[3];
    if (grid_reduce3(acc0, acc1, 0.0, P.partials, P.counters + n, tot) && tid == 0) {
        P.sc.lam[n] = (n == N) ? 0.0 : P.Lam * tot[0];
        P.sc.mu[n] = tot[1];
        P.sc.alpha[n] = 0.0;
        P.sc.delta[n] = 0.0;
    }
}

// p(n) of (10) from lambda(n), mu(n); total mass sum_m P(m); residual ratio.
__global__ void scalars_kernel(SweepParams P, int want_residual) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int N = P.N;
    double g = 1.0, G = 1.0;
    for (int n = 1; n <= N; ++n) {
        g = g * P.sc.lam[n - 1] / P.sc.mu[n];
        G += g;
    }
    g = 1.0;
    double mass = 0.0;
    for (int n = 0; n <= N; ++n) {
        if (n > 0) g = g * P.sc.lam[n - 1] / P.sc.mu[n];
        const double pn = g / G;
        P.sc.pn[n] = pn;
        // sum_{C_n} p_n = lambda(n) / Lambda for n < N; the full layer is fixed to 1
        mass += pn * ((n == N) ? 1.0 : P.sc.lam[n] / P.Lam);
    }
    P.sc.misc[1] = mass;
    if (!isfinite(G)) P.sc.misc[2] = 1.0;
    if (want_residual) {
        double num = 0.0, den = 0.0;
        for (int n = 0; n <= N; ++n) {
            num += P.sc.rnum[n];
            den += P.sc.rden[n];
        }
        P.sc.misc[0] = den > 0.0 ? num / den : 0.0;
    }
}

// P(m) (or p_n(m) when `conditional`) of one layer, scattered to bitmask
// order with original unit labels: out[orig(m)].
template <typename T>
__global__ __launch_bounds__(HQ_WG) void export_kernel(SweepParams P, LayerArgs A, const T* __restrict__ x,
                                                       double* __restrict__ out,
                                                       const uint32_t* __restrict__ orig_bit,
                                                       int conditional) {
    __shared__ uint32_t s_self;
    const int tid = threadIdx.x;
    const int n = A.n, b = P.b, N = P.N;
    int q;
    uint32_t Tb;
    decode_segment(P, A, blockIdx.x, q, Tb);
    if (tid == 0) s_self = P.layer_off[n] + tile_off(P.binom, b, Tb, q);
    __syncthreads();
    const uint32_t Tabs = Tb << b;
    uint32_t hi = 0;
    for (int u = b; u < N; ++u)
        if ((Tabs >> u) & 1u) hi |= orig_bit[u];
    const uint32_t cnt = C(P.binom, b, q);
    const double f = conditional ? P.inv_scale[n] : P.sc.pn[n] * P.inv_scale[n] / P.sc.misc[1];
    for (uint32_t t = tid; t < cnt; t += HQ_WG) {
        const uint32_t L = P.lo_unrank[P.lo_qstart[q] + t];
        uint32_t lo = 0;
        for (int u = 0; u < b; ++u)
            if ((L >> u) & 1u) lo |= orig_bit[u];
        out[hi | lo] = (double)x[s_self + t] * f;
    }
}

// Per-unit busy probabilities: partial sums of P(m) over the states of one
// layer, for every (relabelled) unit; the last work-group sums the
// partials in fixed order and adds them into rho[0..N-1].
template <typename T>
__global__ __launch_bounds__(HQ_WG) void marginal_kernel(SweepParams P, LayerArgs A, const T* __restrict__ x,
                                                         double* __restrict__ part, double* __restrict__ rho) {
    __shared__ uint32_t s_self;
    __shared__ double s_w[HQ_WG / 64][32];
    __shared__ unsigned s_last;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int n = A.n, b = P.b, H = P.H, N = P.N;
    int q;
    uint32_t Tb;
    decode_segment(P, A, blockIdx.x, q, Tb);
    if (tid == 0) s_self = P.layer_off[n] + tile_off(P.binom, b, Tb, q);
    __syncthreads();
    const uint32_t cnt = C(P.binom, b, q);
    const double f = P.sc.pn[n] * P.inv_scale[n] / P.sc.misc[1];
    double acc[HQ_MAXB + 1];
    for (int i = 0; i <= HQ_MAXB; ++i) acc[i] = 0.0;
    for (uint32_t t = tid; t < cnt; t += HQ_WG) {
        const uint32_t L = P.lo_unrank[P.lo_qstart[q] + t];
        const double v = (double)x[s_self + t] * f;
        acc[HQ_MAXB] += v;
        for (int l = 0; l < HQ_MAXB; ++l)
            if (l < b && ((L >> l) & 1u)) acc[l] += v;
    }
    for (int i = 0; i <= HQ_MAXB; ++i) {
        const double s = wave_sum(acc[i]);
        if (lane == 0) s_w[w][i] = s;
    }
    __syncthreads();
    if (tid < 32) {
        double s = 0.0;
        if (tid <= HQ_MAXB)
            for (int i = 0; i < HQ_WG / 64; ++i) s += s_w[i][tid];
        s_w[0][tid] = s;
    }
    __syncthreads();
    // partial vector of this work-group: low units, then high units (all get the segment mass)
    double* pp = part + (size_t)blockIdx.x * 32;
    if (tid < N) {
        double v;
        if (tid < b)
            v = s_w[0][tid];
        else
            v = ((Tb >> (tid - b)) & 1u) ? s_w[0][HQ_MAXB] : 0.0;
        store_partial(pp + tid, v);
    }
    __syncthreads();
    if (tid == 0) {
        const unsigned t = __hip_atomic_fetch_add(P.counters + n, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (t == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (tid < N) {
        double s = 0.0;
        for (uint32_t i = 0; i < gridDim.x; ++i) s += load_partial(part + (size_t)i * 32 + tid);
        rho[tid] += s;
    }
    if (tid == 0) __hip_atomic_store(P.counters + n, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// FP32 -> FP64 conversion of one layer (precision switch of the polish form).
__global__ void widen_kernel(const float* __restrict__ src, double* __restrict__ dst, uint32_t begin,
                             uint32_t count, double factor) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[begin + i] = (double)src[begin + i] * factor;
}

}  // namespace hq

// ---------------------------------------------------------------------------
// Launch wrappers with C++ linkage, called from the host code.
// ---------------------------------------------------------------------------
namespace hqk {

using namespace hq;

template <typename T>
static hipError_t launch_layer_t(int mode, bool track_delta, const SweepParams& P, const LayerArgs& A, T* x,
                                 int inner_one, hipStream_t s) {
    dim3 grid(A.groups), block(HQ_WG);
    if (mode == M_PASS1)
        hipLaunchKernelGGL((layer_kernel<T, M_PASS1, false>), grid, block, 0, s, P, A, x, inner_one);
    else if (mode == M_WRITE && track_delta)
        hipLaunchKernelGGL((layer_kernel<T, M_WRITE, true>), grid, block, 0, s, P, A, x, inner_one);
    else if (mode == M_WRITE)
        hipLaunchKernelGGL((layer_kernel<T, M_WRITE, false>), grid, block, 0, s, P, A, x, inner_one);
    else
        hipLaunchKernelGGL((layer_kernel<T, M_RESID, false>), grid, block, 0, s, P, A, x, inner_one);
    return hipGetLastError();
}

hipError_t launch_layer(int mode, bool track_delta, bool fp32, const SweepParams& P, const LayerArgs& A,
                        void* x, int inner_one, hipStream_t s) {
    return fp32 ? launch_layer_t<float>(mode, track_delta, P, A, (float*)x, inner_one, s)
                : launch_layer_t<double>(mode, track_delta, P, A, (double*)x, inner_one, s);
}

hipError_t launch_init(bool fp32, const SweepParams& P, const LayerArgs& A, void* x, const double* xu,
                       const double* given, const uint32_t* orig_bit, hipStream_t s) {
    dim3 grid(A.groups), block(HQ_WG);
    if (fp32)
        hipLaunchKernelGGL((init_kernel<float>), grid, block, 0, s, P, A, (float*)x, xu, given, orig_bit);
    else
        hipLaunchKernelGGL((init_kernel<double>), grid, block, 0, s, P, A, (double*)x, xu, given, orig_bit);
    return hipGetLastError();
}

hipError_t launch_scalars(const SweepParams& P, int want_residual, hipStream_t s) {
    hipLaunchKernelGGL(scalars_kernel, dim3(1), dim3(64), 0, s, P, want_residual);
    return hipGetLastError();
}

hipError_t launch_export(bool fp32, const SweepParams& P, const LayerArgs& A, const void* x, double* out,
                         const uint32_t* orig_bit, int conditional, hipStream_t s) {
    dim3 grid(A.groups), block(HQ_WG);
    if (fp32)
        hipLaunchKernelGGL((export_kernel<float>), grid, block, 0, s, P, A, (const float*)x, out, orig_bit,
                           conditional);
    else
        hipLaunchKernelGGL((export_kernel<double>), grid, block, 0, s, P, A, (const double*)x, out, orig_bit,
                           conditional);
    return hipGetLastError();
}

hipError_t launch_marginal(bool fp32, const SweepParams& P, const LayerArgs& A, const void* x, double* part,
                           double* rho, hipStream_t s) {
    dim3 grid(A.groups), block(HQ_WG);
    if (fp32)
        hipLaunchKernelGGL((marginal_kernel<float>), grid, block, 0, s, P, A, (const float*)x, part, rho);
    else
        hipLaunchKernelGGL((marginal_kernel<double>), grid, block, 0, s, P, A, (const double*)x, part, rho);
    return hipGetLastError();
}

hipError_t launch_widen(const float* src, double* dst, uint32_t begin, uint32_t count, double factor,
                        hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(widen_kernel, dim3((count + 255) / 256), dim3(256), 0, s, src, dst, begin, count, factor);
    return hipGetLastError();
}

}  // namespace hqk
