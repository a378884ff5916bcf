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
// evaluated on the fly.  The host merges the credits of all demand nodes
// into terms (units ranked before u, u, rate) and, per tile T, splits them:
// terms whose condition involves no low unit are uniform over the tile
// (tcoef), the rest form a short per-tile program of (low mask, rate)
// pairs grouped by unit.  Units are relabelled so that the low (per-lane)
// bits go to the units that demand nodes rank late, which keeps those
// programs short.  Per state the coefficient of a busy unit is then a few
// predicated adds, with no data-dependent memory access.
//
// Each kernel ends with a deterministic two-level FP64 reduction: wave
// shuffles, one partial per work-group, and a fixed-order sum by the last
// work-group to finish, which also derives the layer scalars.
#include "hq_fuse.h"
#include "hq_internal.h"
#include "hq_layout.h"
#include "hq_schedule.h"

#include <math.h>

#include <mutex>

namespace hq {

#define HQ_ERR_DEVICE_CODE 3
#define HQ_ERR_NOT_CONVERGED_CODE 4
#define HQ_ERR_NUMERIC_CODE 5

// Read-only tables are read through the constant address space: uniform
// indices then become scalar loads (they are never written while a kernel
// that reads them runs).
#define HQ_CONST __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const HQ_CONST T* ro(const T* p) {
    return (const HQ_CONST T*)p;
}

enum Mode { M_PASS1 = 0, M_WRITE = 1, M_RESID = 2 };

__device__ __forceinline__ uint32_t C(const uint32_t* tb, int n, int k) {
    return (k < 0 || k > n) ? 0u : tb[n * 32 + k];
}

// Work-groups are persistent: a fixed grid walks the layer's segment list.
// The hardware deals work-groups to the 8 XCDs round-robin; segment j of
// work-group w is chosen so that each XCD sweeps one contiguous eighth of
// the list (memory order), which keeps neighbouring tiles in one L2.
struct SegIter {
    uint32_t begin, end, step;
};
__device__ __forceinline__ SegIter seg_iter(uint32_t groups) {
    const uint32_t G = gridDim.x, w = blockIdx.x;
    if (G < 64 || (G & 7u)) return SegIter{w, groups, G};
    const uint32_t x = w & 7u, per = (groups + 7u) >> 3;
    const uint32_t lo = x * per, hi = min(groups, lo + per);
    return SegIter{lo + (w >> 3), hi, G >> 3};
}

// Segment: popcount class q of the low bits and tile T.
struct Seg {
    int q;
    uint32_t Tb;
};
__device__ __forceinline__ Seg seg_at(const SweepParams& P, const LayerArgs& A, uint32_t s) {
    const uint32_t d = ro(P.seg_desc)[A.desc_base + s];
    return Seg{(int)(d & 15u), d >> 4};
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}

// Reduce six per-thread values over the work-group (sum, sum, max, max,
// sum, sum) and store them as this work-group's partial.  No fence: the
// finalize kernel (or, after a small layer, the next layer's launch) that
// reads the partials runs after this kernel on the same stream.
__device__ void block_partial(double a0, double a1, double a2, double a3, double* partials, double a4 = 0.0,
                              double a5 = 0.0) {
    __shared__ double s_red[HQ_NPART][HQ_WG / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_max(a2);
    a3 = wave_max(a3);
    a4 = wave_sum(a4);
    a5 = wave_sum(a5);
    if (lane == 0) {
        s_red[0][w] = a0;
        s_red[1][w] = a1;
        s_red[2][w] = a2;
        s_red[3][w] = a3;
        s_red[4][w] = a4;
        s_red[5][w] = a5;
    }
    __syncthreads();
    if (tid == 0) {
        double b[HQ_NPART] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int i = 0; i < HQ_WG / 64; ++i) {
            b[0] += s_red[0][i];
            b[1] += s_red[1][i];
            b[2] = fmax(b[2], s_red[2][i]);
            b[3] = fmax(b[3], s_red[3][i]);
            b[4] += s_red[4][i];
            b[5] += s_red[5][i];
        }
        double* pp = partials + (size_t)blockIdx.x * HQ_NPART;
        for (int j = 0; j < HQ_NPART; ++j) pp[j] = b[j];
    }
}

// Fixed-order reduction of `count` partials by one work-group.
__device__ void sum_partials(const double* partials, uint32_t count, double out[HQ_NPART]) {
    __shared__ double s_red[HQ_NPART][HQ_WG / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double c[HQ_NPART] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (uint32_t i = tid; i < count; i += HQ_WG) {
        const double* pp = partials + (size_t)i * HQ_NPART;
        c[0] += pp[0];
        c[1] += pp[1];
        c[2] = fmax(c[2], pp[2]);
        c[3] = fmax(c[3], pp[3]);
        c[4] += pp[4];
        c[5] += pp[5];
    }
    c[0] = wave_sum(c[0]);
    c[1] = wave_sum(c[1]);
    c[2] = wave_max(c[2]);
    c[3] = wave_max(c[3]);
    c[4] = wave_sum(c[4]);
    c[5] = wave_sum(c[5]);
    if (lane == 0)
        for (int j = 0; j < HQ_NPART; ++j) s_red[j][w] = c[j];
    __syncthreads();
    if (tid == 0) {
        double d[HQ_NPART] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int i = 0; i < HQ_WG / 64; ++i) {
            d[0] += s_red[0][i];
            d[1] += s_red[1][i];
            d[2] = fmax(d[2], s_red[2][i]);
            d[3] = fmax(d[3], s_red[3][i]);
            d[4] += s_red[4][i];
            d[5] += s_red[5][i];
        }
        for (int j = 0; j < HQ_NPART; ++j) out[j] = d[j];
    }
}

// ---------------------------------------------------------------------------
// The layer kernel.  MODE:
//   M_PASS1  first pass of the closed and literal inner forms: reduce
//            S_U = sum U~(m) (closed) or sum mu_m U~(m) (literal, with
//            TRACK_DELTA: also max U~ and the first step's change) and
//            S_muD = sum mu_m D~(m) over the layer; the finalize step then
//            derives alpha_n.
//   M_WRITE  update (12): p_n(m) = alpha_n U~(m) + beta_n D~(m), write it,
//            reduce lambda(n) = Lambda sum p_n and mu(n) = sum mu_m p_n.
//   M_RESID  balance residual of (1) for the states of layer n.
// with U~(m) = sum_{u in m} a(m,u) p_{n-1}(m\u) / (Lambda + mu_m) and
//      D~(m) = sum_{u notin m} nu_u p_{n+1}(m+u) / (Lambda + mu_m).
// STORED: the layer's coefficients a(m, u) are read from `coefs` instead
// of being evaluated from the per-tile uniform coefficients and programs.
// ---------------------------------------------------------------------------
// Wave-granular segment iteration for the layer kernels: each 64-lane wave
// owns one segment at a time and walks its own share of the segment list,
// XCD-chunked like seg_iter.  No block-wide barrier inside the loop.
struct WaveIter {
    uint32_t begin, end, step;
};
__device__ __forceinline__ WaveIter wave_iter(uint32_t groups) {
    const uint32_t WPG = HQ_WG / 64;
    const uint32_t G = gridDim.x, w = blockIdx.x;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (G < 64 || (G & 7u)) return WaveIter{w * WPG + wv, groups, G * WPG};
    const uint32_t x = w & 7u, per = (groups + 7u) >> 3;
    const uint32_t lo = x * per, hi = min(groups, lo + per);
    return WaveIter{lo + (w >> 3) * WPG + wv, hi, (G >> 3) * WPG};
}

// Scalars of one layer update, fixed for the whole layer.
struct ModeScalars {
    double alpha, beta;       // coefficients of U~ and D~ in (12)
    double alpha0;            // mu^{k-1}(n) / lambda^k(n-1): first inner step (literal form)
    double pdn, pself, pup;   // p(n-1), p(n), p(n+1) (residual)
    double is_dn, is_up;      // inverse storage scales of layers n-1, n+1
    double s_self, is_self;   // storage scale of layer n and its inverse
};

template <int MODE>
__device__ __forceinline__ ModeScalars mode_scalars(const SweepParams& P, int n, int inner_one, const double* lam,
                                                    const double* mu, const double* alpha_closed,
                                                    const double* pn) {
    const int N = P.N;
    ModeScalars ms{};
    ms.is_dn = (n >= 1) ? P.inv_scale[n - 1] : 0.0;
    ms.is_up = (n < N) ? P.inv_scale[n + 1] : 0.0;
    ms.s_self = P.scale[n];
    ms.is_self = P.inv_scale[n];
    if (MODE == M_PASS1 || MODE == M_WRITE) {
        ms.beta = lam[n] / mu[n + 1];  // lambda^{k-1}(n) / mu^{k-1}(n+1)
        ms.alpha0 = mu[n] / lam[n - 1];  // mu^{k-1}(n) / lambda^k(n-1)
        if (MODE == M_WRITE)
            ms.alpha = inner_one == 1 ? ms.alpha0        // one inner update
                                      : alpha_closed[n];  // from the first pass (closed or literal)
    } else {
        ms.pdn = (n >= 1) ? pn[n - 1] : 0.0;
        ms.pself = pn[n];
        ms.pup = (n < N) ? pn[n + 1] : 0.0;
    }
    return ms;
}

// Wave-uniform values are fetched lane-parallel (lane i loads entry i of a
// small per-segment record with one vector load) and broadcast with
// readlane where they are used.  This keeps them out of scalar registers
// and costs one memory round trip per record instead of a chain of scalar
// loads.
__device__ __forceinline__ uint32_t bcast(uint32_t v, uint32_t i) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)i);
}
__device__ __forceinline__ double bcast(double v, uint32_t i) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const uint32_t lo = bcast((uint32_t)b, i), hi = bcast((uint32_t)(b >> 32), i);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The first 64 program terms of a tile are held in registers (lane i holds
// term i), the rest are read as scalar loads, four terms per batch (the
// program array ends in inert padding terms, so a batch never leaves it).
#define HQ_PROG_REG 64

// Wave-uniform part of a segment's record: descriptor and the position of
// its tile's program.  Fetched two segments ahead.
struct SegScal {
    uint32_t desc;    // (T << 4) | q
    uint32_t pstart;  // first program term of the tile
    uint32_t pcount;  // number of program terms
};

// Lane-parallel part, fetched one segment ahead so that its loads overlap
// the previous segment's work.
struct SegVec {
    uint32_t seg;  // lane k < H: start of segment (T xor e_k, q); lanes H, H+1, H+2: (T, q-1), (T, q+1), (T, q)
    uint32_t po;   // lane u <= N: prog_off[T][u] relative to the tile's first term
    double tc;     // lane u < N: tcoef[T][u]
    uint32_t pm;   // lane i: mask of program term i
    double pr;     //         and its rate
};

__device__ __forceinline__ SegScal fetch_scal(const SweepParams& P, const LayerArgs& A, uint32_t si) {
    SegScal r;
    r.desc = ro(P.seg_desc)[A.desc_base + si];
    const HQ_CONST uint32_t* sp = ro(reinterpret_cast<const uint32_t*>(P.seg_prog)) + 2 * (size_t)(A.desc_base + si);
    r.pstart = sp[0];
    r.pcount = sp[1];
    return r;
}

__device__ __forceinline__ SegVec fetch_vec(const SweepParams& P, int b, int H, const SegScal& sc, bool stored) {
    const int lane = threadIdx.x & 63;
    const int N = P.N;
    const uint32_t tiles = 1u << H;
    const int q = (int)(sc.desc & 15u);
    const uint32_t Tb = sc.desc >> 4;
    SegVec r;
    r.seg = 0u;
    if (lane < H)
        r.seg = P.segoff[hqlayout::seg_index(q, Tb ^ (1u << lane), tiles)];
    else if (lane == H)
        r.seg = hqlayout::low_down_segment(P.segoff, tiles, q, Tb);
    else if (lane == H + 1)
        r.seg = hqlayout::low_up_segment(P.segoff, tiles, q, b, Tb);
    else if (lane == H + 2)
        r.seg = P.segoff[hqlayout::seg_index(q, Tb, tiles)];
    r.po = 0u;
    r.tc = 0.0;
    r.pm = 0u;
    r.pr = 0.0;
    if (stored) return r;
    if (lane <= N) r.po = P.prog_off[(size_t)Tb * (N + 1) + lane] - sc.pstart;
    if (lane < N) r.tc = P.tcoef[(size_t)Tb * N + lane];
    if ((uint32_t)lane < sc.pcount) {
        const ProgTerm t = P.prog[sc.pstart + lane];
        r.pm = t.mask;
        r.pr = t.rate;
    }
    return r;
}

// Arrival coefficient of busy unit u for the lane's low pattern L: the
// tile-uniform part plus the unit's program terms whose mask lies in L.
// A term applies iff its mask has no bit outside L; the select keeps the
// sum bit-identical to adding 0.0 for the terms that do not apply.
__device__ __forceinline__ double unit_coef(const SweepParams& P, const SegScal& sc, const SegVec& r, int u,
                                            uint32_t L) {
    double c = bcast(r.tc, (uint32_t)u);
    const uint32_t i0 = bcast(r.po, (uint32_t)u), i1 = bcast(r.po, (uint32_t)u + 1u);
    const uint32_t nL = ~L;
    const uint32_t ireg = i1 < HQ_PROG_REG ? i1 : HQ_PROG_REG;
    for (uint32_t i = i0; i < ireg; ++i) {
        const uint32_t mk = bcast(r.pm, i);
        const double cn = c + bcast(r.pr, i);
        c = (nL & mk) == 0u ? cn : c;
    }
    const HQ_CONST ProgTerm* tp = ro(P.prog) + sc.pstart;
    for (uint32_t i = i0 > ireg ? i0 : ireg; i < i1; i += 4) {
        uint32_t mk4[4];
        double rt4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            mk4[k] = tp[i + k].mask;
            rt4[k] = tp[i + k].rate;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double cn = c + rt4[k];
            c = (i + k < i1 && (nL & mk4[k]) == 0u) ? cn : c;
        }
    }
    return c;
}

// One wave updates (or, for M_RESID / M_PASS1, evaluates) the states of one
// segment of layer A.n from its fetched record; accumulates the layer sums
// in acc0..acc2.  Every state reads its N neighbours once, all loads issued
// together; the arrival coefficient of busy unit u is tcoef[T][u] plus the
// lane's terms of the tile program of u (or, with STORED, the stored
// a(m, u)).  BF, HF: the tile shape (low bits b, high bits H) fixed at
// compile time, or 0 to take it from P.  With a fixed shape the unrolled
// per-unit code needs no run-time guards, which keeps the register budget
// at 4 waves per SIMD.
template <typename T, int MODE, bool TRACK_DELTA, bool STORED, int BF = 0, int HF = 0>
__device__ __forceinline__ void segment_compute(const SweepParams& P, const LayerArgs& A, T* __restrict__ x,
                                                const SegScal& sc, const SegVec& r, const uint16_t* s_rank,
                                                const uint16_t* s_unrank, const uint32_t* s_qstart,
                                                const ModeScalars& ms, double& acc0, double& acc1, double& acc2,
                                                double& acc3, double& acc4, double& acc5) {
    constexpr int MAXB = BF ? BF : HQ_MAXB, MAXH = HF ? HF : HQ_MAXH;
    const int lane = threadIdx.x & 63;
    const int n = A.n, N = P.N;
    const int b = BF ? BF : P.b, H = HF ? HF : P.H;
    const uint32_t full = (N >= 32) ? 0xffffffffu : ((1u << N) - 1u);
    const HQ_CONST double* nuc = ro(P.nu);
    const double alpha = ms.alpha, beta = ms.beta, pdn = ms.pdn, pself = ms.pself, pup = ms.pup;
    const double is_dn = ms.is_dn, is_up = ms.is_up, s_self = ms.s_self, is_self = ms.is_self;
    const int q = (int)(sc.desc & 15u);
    const uint32_t Tb = sc.desc >> 4;
    const uint32_t offDlo = bcast(r.seg, (uint32_t)H), offUlo = bcast(r.seg, (uint32_t)H + 1u);
    const uint32_t offSelf = bcast(r.seg, (uint32_t)H + 2u);
    double mu_hi = 0.0;
    for (int k = 0; k < H; ++k)
        if ((Tb >> k) & 1u) mu_hi += nuc[b + k];
    const uint32_t cnt = ro(P.binom)[b * 32 + q];
    const double* cs = P.coefs + A.coef_base + (offSelf - ro(P.layer_off)[n]);
    const uint32_t qs = s_qstart[q];
    const uint32_t Tabs = Tb << b;

    for (uint32_t t = lane; t < cnt; t += 64) {
        const uint32_t L = s_unrank[qs + t];
        const uint32_t m = Tabs | L;
        // every neighbour value first: low units in the small segments
        // (T, q -+ 1), high units segment-aligned and coalesced
        // with a run-time shape the high units go in chunks of HQ_HCHUNK
        // (a bounded register budget); with a fixed shape all at once
        constexpr int HB = HF ? MAXH : HQ_HCHUNK;
        double vl[MAXB], vh[HB], cl[MAXB];
#pragma unroll
        for (int l = 0; l < MAXB; ++l)
            if (l < b) vl[l] = (double)x[hqlayout::low_neighbour(L, l, offDlo, offUlo, s_rank)];
        // stored coefficients (zero for idle units): every load issued before any use
        if (STORED) {
#pragma unroll
            for (int l = 0; l < MAXB; ++l)
                if (l < b) cl[l] = cs[(size_t)l * A.count + t];
        }
        if (HF) {
#pragma unroll
            for (int k = 0; k < HB; ++k)
                if (k < H) vh[k] = (double)x[bcast(r.seg, (uint32_t)k) + t];
        }
        double U = 0.0, D = 0.0, mu_lo = 0.0;
#pragma unroll
        for (int l = 0; l < MAXB; ++l) {
            if (l < b) {
                const double nl = nuc[l];
                if ((L >> l) & 1u) {
                    const double c = STORED ? cl[l] : unit_coef(P, sc, r, l, L);
                    U += c * vl[l];
                    mu_lo += nl;
                } else {
                    D += nl * vl[l];
                }
            }
        }
        if (HF) {
            double ch[HB];
            if (STORED) {
#pragma unroll
                for (int k = 0; k < HB; ++k)
                    if (k < H && ((Tb >> k) & 1u)) ch[k] = cs[(size_t)(b + k) * A.count + t];
            }
#pragma unroll
            for (int k = 0; k < HB; ++k) {
                if (k < H) {
                    if ((Tb >> k) & 1u) {
                        const double c = STORED ? ch[k] : unit_coef(P, sc, r, b + k, L);
                        U += c * vh[k];
                    } else {
                        D += nuc[b + k] * vh[k];
                    }
                }
            }
        } else {
            for (int k0 = 0; k0 < H; k0 += HB) {
#pragma unroll
                for (int j = 0; j < HB; ++j)
                    if (k0 + j < H) vh[j] = (double)x[bcast(r.seg, (uint32_t)(k0 + j)) + t];
                double ch[HB];
                if (STORED) {
#pragma unroll
                    for (int j = 0; j < HB; ++j)
                        if (k0 + j < H && ((Tb >> (k0 + j)) & 1u)) ch[j] = cs[(size_t)(b + k0 + j) * A.count + t];
                }
#pragma unroll
                for (int j = 0; j < HB; ++j) {
                    const int k = k0 + j;
                    if (k < H) {
                        if ((Tb >> k) & 1u) {
                            const double c = STORED ? ch[j] : unit_coef(P, sc, r, b + k, L);
                            U += c * vh[j];
                        } else {
                            D += nuc[b + k] * vh[j];
                        }
                    }
                }
            }
        }
        U *= is_dn;
        D *= is_up;
        const double mu_m = mu_hi + mu_lo;
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
                if (TRACK_DELTA) {
                    // literal inner loop: sum mu U~, sum mu D~, max U~ and the
                    // first step's change against the previous iterate
                    acc0 += mu_m * Ut;
                    acc1 += mu_m * Dt;
                    acc2 = fmax(acc2, Ut);
                    const double v0 = ms.alpha0 * Ut + beta * Dt;
                    acc3 = fmax(acc3, fabs(v0 - (double)x[offSelf + t] * is_self));
                } else {
                    acc0 += Ut;
                    acc1 += mu_m * Dt;
                }
            } else {
                const double p = alpha * Ut + beta * Dt;
                const uint32_t o = offSelf + t;
                if (TRACK_DELTA) acc2 = fmax(acc2, fabs(p - (double)x[o] * is_self));
                const T stored = (T)(p * s_self);
                x[o] = stored;
                const double ps = (double)stored * is_self;
                acc0 += ps;
                acc1 += mu_m * ps;
                if (P.la) {
                    acc4 += ps * P.la[2 * (size_t)o];
                    acc5 += ps * P.la[2 * (size_t)o + 1];
                }
            }
        }
    }
}

// Fetch and process one segment (no look-ahead; used by the batch kernel).
template <typename T, int MODE, bool TRACK_DELTA, bool STORED>
__device__ __forceinline__ void segment_update(const SweepParams& P, const LayerArgs& A, T* __restrict__ x,
                                               uint32_t si, const uint16_t* s_rank, const uint16_t* s_unrank,
                                               const uint32_t* s_qstart, const ModeScalars& ms, double& acc0,
                                               double& acc1, double& acc2) {
    const SegScal sc = fetch_scal(P, A, si);
    const SegVec r = fetch_vec(P, P.b, P.H, sc, STORED);
    double unused = 0.0, unused4 = 0.0, unused5 = 0.0;
    segment_compute<T, MODE, TRACK_DELTA, STORED>(P, A, x, sc, r, s_rank, s_unrank, s_qstart, ms, acc0, acc1, acc2,
                                                  unused, unused4, unused5);
}

// Occupancy floors (waves per SIMD) that the register allocation must keep:
// 4 with computed coefficients, 3 with stored ones from H = 14 (the counts
// the kernel reaches without the fused prologue of hq_fuse.h).
template <typename T, int MODE, bool TRACK_DELTA, bool STORED, int BF = 0, int HF = 0>
__global__ __launch_bounds__(HQ_WG) __attribute__((amdgpu_waves_per_eu(STORED ? (HF >= 14 ? 3 : 2) : 4, 8))) void
layer_kernel(SweepParams P, LayerArgs A, T* __restrict__ x, int inner_one, hqfuse::FuseArgs F) {
    __shared__ double s_fred[HQ_NPART][HQ_WG / 64];
    __shared__ uint16_t s_rank[1 << HQ_MAXB];    // colex rank of a low pattern inside its class
    __shared__ uint16_t s_unrank[1 << HQ_MAXB];  // low patterns by (popcount, value)
    __shared__ uint32_t s_qstart[HQ_MAXB + 2];

    const int tid = threadIdx.x;
    const int b = BF ? BF : P.b, H = HF ? HF : P.H;
    for (int i = tid; i < (1 << b); i += HQ_WG) {
        s_rank[i] = P.lo_rank[i];
        s_unrank[i] = P.lo_unrank[i];
    }
    if (tid <= b + 1) s_qstart[tid] = P.lo_qstart[tid];
    __syncthreads();
    // the previous layer's scalars, when its finalize launch is fused into this one
    hqfuse::Prev pv{0.0, 0.0};
    const bool fused = MODE == M_WRITE && F.prev != nullptr;
    if (fused) pv = hqfuse::prologue<HQ_WG>(P, A.n, inner_one, F, s_fred);
    ModeScalars ms = mode_scalars<MODE>(P, A.n, inner_one, P.sc.lam, P.sc.mu, P.sc.alpha, P.sc.pn);
    if (fused) {
        ms.alpha0 = P.sc.mu[A.n] / pv.lam_prev;
        ms.alpha = inner_one == 1 ? ms.alpha0 : (P.la ? pv.alpha_la : ms.alpha);
    }
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0, acc4 = 0.0, acc5 = 0.0;
    // Software pipeline over this wave's segments: the scalar record of
    // segment i+2 and the lane-parallel record of segment i+1 are in flight
    // while segment i is processed.
    const WaveIter it = wave_iter(A.groups);
    SegScal s0{}, s1{};
    SegVec v0{};
    if (it.begin < it.end) {
        s0 = fetch_scal(P, A, it.begin);
        v0 = fetch_vec(P, b, H, s0, STORED);
    }
    if (it.begin + it.step < it.end) s1 = fetch_scal(P, A, it.begin + it.step);
    for (uint32_t si = it.begin; si < it.end; si += it.step) {
        SegVec v1{};
        SegScal s2{};
        if (si + it.step < it.end) v1 = fetch_vec(P, b, H, s1, STORED);
        if (si + 2 * it.step < it.end) s2 = fetch_scal(P, A, si + 2 * it.step);
        segment_compute<T, MODE, TRACK_DELTA, STORED, BF, HF>(P, A, x, s0, v0, s_rank, s_unrank, s_qstart, ms, acc0,
                                                              acc1, acc2, acc3, acc4, acc5);
        s0 = s1;
        v0 = v1;
        s1 = s2;
    }
    block_partial(acc0, acc1, acc2, acc3, P.partials, acc4, acc5);
}

// Layer scalars from the work-group partials of the kernel just run on the
// same stream (one work-group, fixed summation order).
// inner: 0 closed form, 1 one update, 2 literal loop with tolerance P.delta.
// With the look-ahead closed form (P.la set): the write of layer n also
// yields sum p_n w and sum p_n z, from which the closed-form alpha of layer
// n + 1 follows before that layer is swept:
//   alpha_{n+1} = beta_{n+1} S_muD(n+1) / (Lambda S_U(n+1)),
//   S_U(n+1) = sum_{C_n} p_n w (this iteration), S_muD(n+1) = sum_{C_{n+2}}
//   p_{n+2} z (the last write of layer n + 2, i.e. the previous iteration),
// the same sums the first pass forms, re-indexed over the neighbour layers.
__device__ __forceinline__ void lookahead_alpha(const SweepParams& P, int m) {
    // alpha of layer m from the stored sums; m in 1..N-1
    const double beta = P.sc.lam[m] / P.sc.mu[m + 1];
    const double su = P.sc.wsum[m - 1], smud = P.sc.zsum[m + 1];
    const double a = beta * smud / (P.Lam * su);
    if (!(su > 0.0) || !isfinite(a)) P.sc.misc[2] = 1.0;
    P.sc.alpha[m] = a;
}

__global__ __launch_bounds__(HQ_WG) void finalize_kernel(SweepParams P, int mode, int n, uint32_t count,
                                                         int inner_one) {
    double tot[HQ_NPART];
    sum_partials(P.partials, count, tot);
    if (threadIdx.x != 0) return;
    double* misc = P.sc.misc;
    const int N = P.N;
    if (mode == M_PASS1 && inner_one == 2) {
        // the inner loop of Algorithm 1 as written: p^r = (mu_r / L) U~ +
        // beta D~ with mu_0 = mu^{k-1}(n) and mu_{r+1} = sum mu_m p^r; it
        // stops at the first step whose max change is <= delta.  The first
        // change (against the previous iterate) came from the pass; after
        // that p^{r+1} - p^r = ((mu_{r+1} - mu_r) / L) U~.
        const double L = P.sc.lam[n - 1], beta = P.sc.lam[n] / P.sc.mu[n + 1];
        const double s_muU = tot[0], s_muD = tot[1], maxU = tot[2];
        double mu_r = P.sc.mu[n], change = tot[3];
        for (int r = 0; r < 1000000 && !(change <= P.delta); ++r) {
            const double mu_next = (mu_r / L) * s_muU + beta * s_muD;
            change = fabs(mu_next - mu_r) / L * maxU;
            mu_r = mu_next;
        }
        const double a = mu_r / L;
        if (!isfinite(a)) misc[2] = 1.0;
        P.sc.alpha[n] = a;
    } else if (mode == M_PASS1) {
        // mu* = B / (1 - A) with A = sum mu U~ / lambda(n-1) = 1 - Lambda S_U / lambda(n-1)
        // (since sum (Lambda + mu_m) U~ = lambda(n-1)), so alpha = mu*/lambda(n-1)
        // = beta S_muD / (Lambda S_U).
        const double beta = P.sc.lam[n] / P.sc.mu[n + 1];
        const double a = beta * tot[1] / (P.Lam * tot[0]);
        if (!(tot[0] > 0.0) || !isfinite(a)) misc[2] = 1.0;
        P.sc.alpha[n] = a;
    } else if (mode == M_WRITE) {
        const double used = inner_one == 1 ? P.sc.mu[n] / P.sc.lam[n - 1] : P.sc.alpha[n];
        const double lam = P.Lam * tot[0], mu = tot[1];
        if (!isfinite(lam) || !(mu > 0.0) || !isfinite(mu)) misc[2] = 1.0;
        P.sc.lam[n] = lam;
        P.sc.mu[n] = mu;
        P.sc.alpha[n] = used;
        P.sc.delta[n] = tot[2];
        if (P.la) {
            P.sc.wsum[n] = tot[4];
            P.sc.zsum[n] = tot[5];
            // the next layer of this iteration, or layer 1 of the next one
            lookahead_alpha(P, n + 1 <= N - 1 ? n + 1 : 1);
        }
    } else if (mode == M_RESID) {
        P.sc.rnum[n] = tot[0];
        P.sc.rden[n] = tot[1];
        if (!isfinite(tot[0]) || !isfinite(tot[1])) misc[2] = 1.0;
    } else {  // initial iterate
        P.sc.lam[n] = (n == N) ? 0.0 : P.Lam * tot[0];
        P.sc.mu[n] = tot[1];
        P.sc.alpha[n] = 0.0;
        P.sc.delta[n] = 0.0;
        if (P.la) {
            P.sc.wsum[n] = tot[4];
            P.sc.zsum[n] = tot[5];
            if (n == N && N >= 2) lookahead_alpha(P, 1);  // every layer's sums are in
        }
    }
}

// Coefficients a(m, u) of every state of one layer, stored unit-major
// (coefs[coef_base + u * count + rank]), by the plain trie walk of
// Algorithm 3's rule: a node credits its rate to its unit iff every unit on
// its path (itself included) is busy in m.  Run once per instance for the
// top layers (nearly full states), where the per-tile programs are longest.
__global__ __launch_bounds__(HQ_WG) void coef_kernel(SweepParams P, LayerArgs A, double* __restrict__ coefs,
                                                     uint32_t nnodes) {
    const int tid = threadIdx.x;
    const int n = A.n, b = P.b, H = P.H, N = P.N;
    const uint32_t tiles = 1u << H;
    const SegIter it = seg_iter(A.groups);
    for (uint32_t si = it.begin; si < it.end; si += it.step) {
        const Seg sg = seg_at(P, A, si);
        const uint32_t rank0 = P.segoff[sg.q * tiles + sg.Tb] - P.layer_off[n];
        const uint32_t cnt = C(P.binom, b, sg.q);
        for (uint32_t t = tid; t < cnt; t += HQ_WG) {
            const uint32_t m = (sg.Tb << b) | P.lo_unrank[P.lo_qstart[sg.q] + t];
            double* out = coefs + A.coef_base + rank0 + t;
            for (int u = 0; u < N; ++u) out[(size_t)u * A.count] = 0.0;
            uint32_t i = 0;
            while (i < nnodes) {
                const TrieNode nd = P.nodes[i];
                if ((m & nd.need) == nd.need) {
                    out[(size_t)(nd.skip_unit & 31u) * A.count] += nd.rate;
                    ++i;
                } else {
                    i = nd.skip_unit >> 5;
                }
            }
        }
    }
}

// Per-state constants of the look-ahead closed form, for every state l of
// one layer, at its position in the state vector:
//   w(l) = sum_{u notin l} r(l, u) / (Lambda + mu_l + nu_u),
//   z(l) = sum_{u in l} nu_u (mu_l - nu_u) / (Lambda + mu_l - nu_u),
// with r(l, u) the arrival rate that l sends to its idle unit u (the demand
// nodes whose first idle unit in l is u, eq. (3)).  r comes from the merged
// preference trie: a node on a busy path whose own unit is idle passes its
// whole rate to that unit.
__global__ __launch_bounds__(HQ_WG) void lookahead_kernel(SweepParams P, LayerArgs A, double* __restrict__ wz,
                                                          uint32_t nnodes) {
    const int tid = threadIdx.x;
    const int n = A.n, b = P.b, N = P.N;
    const uint32_t tiles = 1u << P.H;
    const SegIter it = seg_iter(A.groups);
    for (uint32_t si = it.begin; si < it.end; si += it.step) {
        const Seg sg = seg_at(P, A, si);
        const uint32_t off = P.segoff[sg.q * tiles + sg.Tb];
        const uint32_t cnt = C(P.binom, b, sg.q);
        for (uint32_t t = tid; t < cnt; t += HQ_WG) {
            const uint32_t m = (sg.Tb << b) | P.lo_unrank[P.lo_qstart[sg.q] + t];
            double mu_m = 0.0;
            for (int u = 0; u < N; ++u)
                if ((m >> u) & 1u) mu_m += P.nu[u];
            double wv = 0.0, zv = 0.0;
            uint32_t i = 0;
            while (i < nnodes) {
                const TrieNode nd = P.nodes[i];
                if ((m & nd.need) == nd.need) {
                    ++i;  // unit busy: the calls go on down the list
                } else {
                    const int u = (int)(nd.skip_unit & 31u);  // first idle unit of these calls
                    wv += nd.rate / (P.Lam + mu_m + P.nu[u]);
                    i = nd.skip_unit >> 5;
                }
            }
            for (int u = 0; u < N; ++u)
                if ((m >> u) & 1u) zv += P.nu[u] * (mu_m - P.nu[u]) / (P.Lam + mu_m - P.nu[u]);
            wz[2 * (size_t)(off + t)] = wv;
            wz[2 * (size_t)(off + t) + 1] = zv;
        }
    }
    (void)n;
}

// Initial iterate of one layer: uniform 1/C(N,n) (Algorithm 1 step 2),
// product form prod_{u in m} x_u / e_n(x), or a given state (bitmask order,
// original unit labels mapped through `orig_bit`).  Partials for lambda(n), mu(n).
// Initial values of one segment (wave-level): uniform 1/C(N,n)
// (Algorithm 1 step 2), product form prod_{u in m} x_u / e_n(x), or a given
// state (bitmask order, original labels through `orig_bit`).
template <typename T>
__device__ __forceinline__ void init_segment(const SweepParams& P, const LayerArgs& A, T* __restrict__ x,
                                             uint32_t si, int init_mode, const double* __restrict__ xu,
                                             const double* __restrict__ given,
                                             const uint32_t* __restrict__ orig_bit, double& acc0, double& acc1,
                                             double& acc4, double& acc5) {
    const int lane = threadIdx.x & 63;
    const int n = A.n, b = P.b, H = P.H, N = P.N;
    const uint32_t tiles = 1u << H;
    const double sc_self = P.scale[n], is_self = P.inv_scale[n];
    const uint32_t d = ro(P.seg_desc)[A.desc_base + si];
    const int q = (int)(d & 15u);
    const uint32_t Tb = d >> 4;
    const uint32_t off = ro(P.segoff)[hqlayout::seg_index(q, Tb, tiles)];
    const uint32_t Tabs = Tb << b;
    double mu_hi = 0.0;
    for (int k = 0; k < H; ++k)
        if ((Tb >> k) & 1u) mu_hi += ro(P.nu)[b + k];
    const uint32_t cnt = ro(P.binom)[b * 32 + q];
    const uint32_t qs = P.lo_qstart[q];
    for (uint32_t t = lane; t < cnt; t += 64) {
        const uint32_t L = P.lo_unrank[qs + t];
        const uint32_t m = Tabs | L;
        double p;
        if (n == 0 || n == N) {
            p = 1.0;
        } else if (init_mode == 1) {
            double pr = 1.0;
            for (int u = 0; u < N; ++u)
                if ((m >> u) & 1u) pr *= xu[u];
            p = pr / A.e_n;
        } else if (init_mode == 2) {
            uint32_t mo = 0;
            for (int u = 0; u < N; ++u)
                if ((m >> u) & 1u) mo |= orig_bit[u];
            p = given[mo];
        } else {
            p = 1.0 / (double)A.count;
        }
        const T stored = (T)(p * sc_self);
        x[off + t] = stored;
        const double ps = (double)stored * is_self;
        double mu_lo = 0.0;
        for (int l = 0; l < b; ++l)
            if ((L >> l) & 1u) mu_lo += ro(P.nu)[l];
        acc0 += ps;
        acc1 += (mu_hi + mu_lo) * ps;
        if (P.la) {
            acc4 += ps * P.la[2 * (size_t)(off + t)];
            acc5 += ps * P.la[2 * (size_t)(off + t) + 1];
        }
    }
}

// Initial iterate of one layer; partials for lambda(n), mu(n).  Same
// wave-granular traversal (and so the same summation order of the layer
// sums) as the layer kernels: a resumed iterate reproduces the
// uninterrupted run bit for bit.
template <typename T>
__global__ __launch_bounds__(HQ_WG) void init_kernel(SweepParams P, LayerArgs A, T* __restrict__ x,
                                                     const double* __restrict__ xu,
                                                     const double* __restrict__ given,
                                                     const uint32_t* __restrict__ orig_bit) {
    double acc0 = 0.0, acc1 = 0.0, acc4 = 0.0, acc5 = 0.0;
    const WaveIter it = wave_iter(A.groups);
    for (uint32_t si = it.begin; si < it.end; si += it.step)
        init_segment<T>(P, A, x, si, A.init_mode, xu, given, orig_bit, acc0, acc1, acc4, acc5);
    block_partial(acc0, acc1, 0.0, 0.0, P.partials, acc4, acc5);
}

// Birth-death marginal p(n), n = 0..N, of (10) from lambda(n), mu(n), with
// the waiting room of Proposition 2: the states with every unit busy and c
// calls waiting carry p(N) rho^c, rho = Lambda / sum nu, for c = 1..C (or
// every c >= 1 when unlimited).  Returns the mass of those waiting states
// and writes their mean number of waiting calls to *wait_mean.
__device__ double birth_death(const SweepParams& P, const double* lam, const double* mu, double* pn,
                              double* wait_mean) {
    const int N = P.N;
    double g = 1.0, Z = 1.0;
    for (int n = 1; n <= N; ++n) {
        g = g * lam[n - 1] / mu[n];
        Z += g;
    }
    const double gN = g;
    // sum_c rho^c and sum_c c rho^c over the room
    double s0 = 0.0, s1 = 0.0;
    if (P.buffer != 0) {
        const double rho = P.Lam / P.sum_nu;
        if (P.buffer < 0) {
            s0 = rho / (1.0 - rho);
            s1 = rho / ((1.0 - rho) * (1.0 - rho));
        } else {
            double r = 1.0;
            for (int c = 1; c <= P.buffer; ++c) {
                r *= rho;
                s0 += r;
                s1 += c * r;
            }
        }
    }
    Z += gN * s0;
    g = 1.0;
    for (int n = 0; n <= N; ++n) {
        if (n > 0) g = g * lam[n - 1] / mu[n];
        pn[n] = g / Z;
    }
    *wait_mean = gN * s1 / Z;
    return gN * s0 / Z;
}

// p(n) of (10) from lambda(n), mu(n); total mass (unit states and waiting
// states); residual ratio.  misc: [0] residual, [1] mass, [2] numeric
// flag, [3] waiting-state mass, [4] mean number waiting.
__global__ void scalars_kernel(SweepParams P, int want_residual) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int N = P.N;
    double wmean = 0.0;
    const double wmass = birth_death(P, P.sc.lam, P.sc.mu, P.sc.pn, &wmean);
    double mass = wmass;
    for (int n = 0; n <= N; ++n) {
        // sum_{C_n} p_n = lambda(n) / Lambda for n < N; the full layer is fixed to 1
        mass += P.sc.pn[n] * ((n == N) ? 1.0 : P.sc.lam[n] / P.Lam);
    }
    P.sc.misc[1] = mass;
    P.sc.misc[3] = wmass;
    P.sc.misc[4] = wmean;
    if (!isfinite(mass)) P.sc.misc[2] = 1.0;
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
    const int tid = threadIdx.x;
    const int n = A.n, b = P.b, N = P.N;
    const double f = conditional ? P.inv_scale[n] : P.sc.pn[n] * P.inv_scale[n] / P.sc.misc[1];
    const SegIter it = seg_iter(A.groups);
    for (uint32_t si = it.begin; si < it.end; si += it.step) {
        const Seg sg = seg_at(P, A, si);
        const uint32_t off = P.segoff[sg.q * (1u << P.H) + sg.Tb];
        const uint32_t Tabs = sg.Tb << b;
        uint32_t hi = 0;
        for (int u = b; u < N; ++u)
            if ((Tabs >> u) & 1u) hi |= orig_bit[u];
        const uint32_t cnt = C(P.binom, b, sg.q);
        for (uint32_t t = tid; t < cnt; t += HQ_WG) {
            const uint32_t L = P.lo_unrank[P.lo_qstart[sg.q] + t];
            uint32_t lo = 0;
            for (int u = 0; u < b; ++u)
                if ((L >> u) & 1u) lo |= orig_bit[u];
            out[hi | lo] = (double)x[off + t] * f;
        }
    }
}

// Per-unit busy probabilities: each work-group writes the sums of P(m) over
// its segments for every (relabelled) unit as one partial row of 32.
template <typename T>
__global__ __launch_bounds__(HQ_WG) void marginal_kernel(SweepParams P, LayerArgs A, const T* __restrict__ x,
                                                         double* __restrict__ part) {
    __shared__ double s_w[HQ_WG / 64][HQ_MAXB + 1];
    __shared__ double s_hi[HQ_MAXH];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int n = A.n, b = P.b, H = P.H, N = P.N;
    const double f = P.sc.pn[n] * P.inv_scale[n] / P.sc.misc[1];
    if (tid < HQ_MAXH) s_hi[tid] = 0.0;
    double lo[HQ_MAXB];
    for (int l = 0; l < HQ_MAXB; ++l) lo[l] = 0.0;
    const SegIter it = seg_iter(A.groups);
    for (uint32_t si = it.begin; si < it.end; si += it.step) {
        const Seg sg = seg_at(P, A, si);
        const uint32_t off = P.segoff[sg.q * (1u << H) + sg.Tb];
        const uint32_t cnt = C(P.binom, b, sg.q);
        double mass = 0.0;
        for (uint32_t t = tid; t < cnt; t += HQ_WG) {
            const uint32_t L = P.lo_unrank[P.lo_qstart[sg.q] + t];
            const double v = (double)x[off + t] * f;
            mass += v;
            for (int l = 0; l < HQ_MAXB; ++l)
                if (l < b && ((L >> l) & 1u)) lo[l] += v;
        }
        mass = wave_sum(mass);
        __syncthreads();
        if (lane == 0) s_w[w][HQ_MAXB] = mass;
        __syncthreads();
        if (tid == 0) {
            double sm = 0.0;
            for (int i = 0; i < HQ_WG / 64; ++i) sm += s_w[i][HQ_MAXB];
            for (int k = 0; k < H; ++k)
                if ((sg.Tb >> k) & 1u) s_hi[k] += sm;
        }
    }
    for (int l = 0; l < HQ_MAXB; ++l) {
        const double s = wave_sum(lo[l]);
        if (lane == 0) s_w[w][l] = s;
    }
    __syncthreads();
    double* pp = part + (size_t)blockIdx.x * 32;
    if (tid < N) {
        double v = 0.0;
        if (tid < b)
            for (int i = 0; i < HQ_WG / 64; ++i) v += s_w[i][tid];
        else
            v = s_hi[tid - b];
        pp[tid] = v;
    }
}

// Adds the fixed-order sum of `count` marginal partial rows into rho[0..N-1].
__global__ void marginal_finalize_kernel(SweepParams P, const double* __restrict__ part, uint32_t count,
                                         double* __restrict__ rho) {
    const int u = threadIdx.x;
    if (u >= P.N) return;
    double s = 0.0;
    for (uint32_t i = 0; i < count; ++i) s += part[(size_t)i * 32 + u];
    rho[u] += s;
}

// FP32 -> FP64 conversion of one layer (precision switch of the polish form).
__global__ void widen_kernel(const float* __restrict__ src, double* __restrict__ dst, uint32_t begin,
                             uint32_t count, double factor) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[begin + i] = (double)src[begin + i] * factor;
}

// ---------------------------------------------------------------------------
// Batched solve: a persistent grid; each work-group takes the next instance
// from a work queue (largest first, as the host orders them) and runs all
// of Algorithm 1 on it — initial iterate, Gauss-Seidel layer sweeps, inner
// form, residual checks with the same adaptive schedule as the single
// solver — with work-group barriers between layers and no other
// synchronisation.  Waves of the group share each layer's segments.
// ---------------------------------------------------------------------------
template <int BS>
__device__ __forceinline__ void block_sum3(double& a0, double& a1, double& a2, double (*s_red)[BS / 64]) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_max(a2);
    __syncthreads();
    if (lane == 0) {
        s_red[0][w] = a0;
        s_red[1][w] = a1;
        s_red[2][w] = a2;
    }
    __syncthreads();
    double b0 = 0.0, b1 = 0.0, b2 = 0.0;
    for (int i = 0; i < BS / 64; ++i) {
        b0 += s_red[0][i];
        b1 += s_red[1][i];
        b2 = fmax(b2, s_red[2][i]);
    }
    a0 = b0;
    a1 = b1;
    a2 = b2;
}

// One layer of one instance inside the batch kernel: the waves of the
// work-groups sharing the instance take its segments round-robin, wave w of
// rank r starting at segment r * waves + w.
template <typename T, int MODE>
__device__ __forceinline__ void batch_layer(const SweepParams& P, const LayerArgs& A, T* x, const uint16_t* s_rank,
                                            const uint16_t* s_unrank, const uint32_t* s_qstart,
                                            const ModeScalars& ms, uint32_t first, uint32_t stride, double& a0,
                                            double& a1, double& a2) {
    if (A.stored) {
        for (uint32_t si = first; si < A.groups; si += stride)
            segment_update<T, MODE, false, true>(P, A, x, si, s_rank, s_unrank, s_qstart, ms, a0, a1, a2);
    } else {
        for (uint32_t si = first; si < A.groups; si += stride)
            segment_update<T, MODE, false, false>(P, A, x, si, s_rank, s_unrank, s_qstart, ms, a0, a1, a2);
    }
}

// The k work-groups that share one batch instance.  `epoch` counts the
// barriers this work-group has passed; the group's counter only grows, so
// barrier e is passed once it reaches e * k.
struct GroupCtx {
    unsigned int* count;
    double* part;
    int k, rank;
    unsigned int epoch;
    int ok;  // 0 once a barrier wait ran out (the instance then stops)
};

// Barrier of the work-groups of one instance: the usual device-wide
// pattern (work-group barrier, agent-scope release, arrival, bounded wait,
// agent-scope acquire, work-group barrier), so the state-vector writes and
// partials of every member are visible to all of them afterwards.  A wait
// that runs out of spins marks the group failed instead of hanging.
#define HQ_GROUP_SPINS (1u << 22)
__device__ __forceinline__ void group_barrier(GroupCtx& g, int* s_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int target = (g.epoch + 1u) * (unsigned int)g.k;
        int ok = g.ok;
        __threadfence();
        __hip_atomic_fetch_add(g.count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned int spins = 0;
        while (ok && __hip_atomic_load(g.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > HQ_GROUP_SPINS) ok = 0;
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
        *s_flag = ok;
    }
    __syncthreads();
    g.ok = *s_flag;
    g.epoch += 1u;
}

// Block totals of (sum, sum, max), then, for a group, the totals over its
// work-groups: each writes its totals to its slot of the current buffer,
// and after the barrier every member adds the k slots in rank order, so all
// members hold bitwise the same totals.
template <int BS>
__device__ __forceinline__ void group_sum3(double& a0, double& a1, double& a2, double (*s_red)[BS / 64],
                                          GroupCtx& g, int* s_flag) {
    block_sum3<BS>(a0, a1, a2, s_red);
    if (g.k == 1) return;
    double* buf = g.part + (size_t)(g.epoch & 1u) * (HQ_GROUP_MAX * 3);
    if (threadIdx.x == 0) {
        buf[g.rank * 3 + 0] = a0;
        buf[g.rank * 3 + 1] = a1;
        buf[g.rank * 3 + 2] = a2;
    }
    group_barrier(g, s_flag);
    double b0 = 0.0, b1 = 0.0, b2 = 0.0;
    for (int r = 0; r < g.k; ++r) {
        b0 += __hip_atomic_load(buf + r * 3 + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        b1 += __hip_atomic_load(buf + r * 3 + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        b2 = fmax(b2, __hip_atomic_load(buf + r * 3 + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    a0 = b0;
    a1 = b1;
    a2 = b2;
}

template <typename T, int BS>
__global__ __launch_bounds__(BS) void batch_kernel(const BatchItem* __restrict__ items,
                                                   const BatchEntry* __restrict__ entries, BatchOut* __restrict__ outs,
                                                   int count, unsigned int* __restrict__ next) {
    __shared__ uint16_t s_rank[1 << HQ_MAXB];
    __shared__ uint16_t s_unrank[1 << HQ_MAXB];
    __shared__ uint32_t s_qstart[HQ_MAXB + 2];
    __shared__ double s_lam[32], s_mu[32], s_alpha[32], s_pn[32];
    __shared__ double s_red[3][BS / 64];
    __shared__ int s_item, s_go, s_next, s_flag;
    const int tid = threadIdx.x;
    const uint32_t NW = BS / 64, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = (int)__hip_atomic_fetch_add(next, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int ei = __builtin_amdgcn_readfirstlane(s_item);
        if (ei >= count) break;
        const BatchEntry E = entries[ei];
        const int ii = E.item;
        const BatchItem& B = items[ii];
        GroupCtx g{B.group_count, B.group_part, E.k, E.rank, 0u, 1};
        const uint32_t first = (uint32_t)E.rank * NW + wv, stride = (uint32_t)E.k * NW;
        const SweepParams& P = B.P;
        T* x = (T*)B.x;
        const int N = P.N, b = P.b;
        for (int i = tid; i < (1 << b); i += BS) {
            s_rank[i] = P.lo_rank[i];
            s_unrank[i] = P.lo_unrank[i];
        }
        if (tid <= b + 1) s_qstart[tid] = P.lo_qstart[tid];
        __syncthreads();
        // initial iterate and its layer scalars (13)-(14)
        for (int n = 0; n <= N; ++n) {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, la4 = 0.0, la5 = 0.0;  // (look-ahead sums unused here)
            for (uint32_t si = first; si < B.layers[n].groups; si += stride)
                init_segment<T>(P, B.layers[n], x, si, B.init_mode, B.xu, B.given, B.orig_bit, a0, a1, la4, la5);
            group_sum3<BS>(a0, a1, a2, s_red, g, &s_flag);
            if (tid == 0) {
                s_lam[n] = (n == N) ? 0.0 : P.Lam * a0;
                s_mu[n] = a1;
                s_alpha[n] = 0.0;
            }
        }
        __syncthreads();
        int k = 0, checks = 0, status = HQ_ERR_NOT_CONVERGED_CODE;
        int next_check = B.check_every > 0 ? B.check_every : hqsched::kFirstCheck;
        double res = -1.0;
        hqsched::Tracker tr = hqsched::start();  // used by thread 0 only
        int stall32 = 0;
        if (next_check > B.max_iters) next_check = B.max_iters;
        while (k < B.max_iters) {
            for (int n = 1; n <= N - 1; ++n) {
                const LayerArgs& A = B.layers[n];
                if (!B.inner_one) {
                    const ModeScalars ms = mode_scalars<M_PASS1>(P, n, 0, s_lam, s_mu, s_alpha, s_pn);
                    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
                    batch_layer<T, M_PASS1>(P, A, x, s_rank, s_unrank, s_qstart, ms, first, stride, a0, a1, a2);
                    group_sum3<BS>(a0, a1, a2, s_red, g, &s_flag);
                    if (tid == 0) s_alpha[n] = ms.beta * a1 / (P.Lam * a0);
                    __syncthreads();
                }
                const ModeScalars ms = mode_scalars<M_WRITE>(P, n, B.inner_one, s_lam, s_mu, s_alpha, s_pn);
                double a0 = 0.0, a1 = 0.0, a2 = 0.0;
                batch_layer<T, M_WRITE>(P, A, x, s_rank, s_unrank, s_qstart, ms, first, stride, a0, a1, a2);
                group_sum3<BS>(a0, a1, a2, s_red, g, &s_flag);
                if (tid == 0) {
                    s_alpha[n] = ms.alpha;
                    s_lam[n] = P.Lam * a0;
                    s_mu[n] = a1;
                }
                __syncthreads();
            }
            ++k;
            if (k < next_check && k < B.max_iters) continue;
            // residual of (1): p(n) of (10), then every layer
            if (tid == 0) {
                double wmean;
                (void)birth_death(P, s_lam, s_mu, s_pn, &wmean);
            }
            __syncthreads();
            double a0 = 0.0, a1 = 0.0, a2 = 0.0;
            for (int n = 0; n <= N; ++n) {
                const ModeScalars ms = mode_scalars<M_RESID>(P, n, 0, s_lam, s_mu, s_alpha, s_pn);
                batch_layer<T, M_RESID>(P, B.layers[n], x, s_rank, s_unrank, s_qstart, ms, first, stride, a0, a1,
                                        a2);
            }
            group_sum3<BS>(a0, a1, a2, s_red, g, &s_flag);
            ++checks;
            if (tid == 0) {
                res = a1 > 0.0 ? a0 / a1 : 0.0;
                int go = 1;
                if (!g.ok) {
                    status = HQ_ERR_DEVICE_CODE;
                    go = 0;
                } else if (!isfinite(res)) {
                    status = HQ_ERR_NUMERIC_CODE;
                    go = 0;
                } else if (res <= B.tol) {
                    status = 0;
                    go = 0;
                } else {
                    // FP32 storage floor, or an FP64 residual that stopped falling
                    if (sizeof(T) == 4 && tr.prev_res > 0.0 && res > 0.8 * tr.prev_res && ++stall32 >= 3) go = 0;
                    next_check = hqsched::next_check(tr, k, res, B.tol, B.check_every);
                    if (hqsched::record(tr, k, res) && sizeof(T) == 8) go = 0;
                    if (next_check > B.max_iters) next_check = B.max_iters;
                }
                s_go = go;
                s_next = next_check;
            }
            __syncthreads();
            next_check = s_next;  // every thread takes thread 0's schedule
            if (!s_go) break;
        }
        // publish the instance's scalars where the single-instance entry points read them
        if (tid == 0 && E.rank == 0) {
            double wmean = 0.0;
            const double wmass = birth_death(P, s_lam, s_mu, s_pn, &wmean);
            double mass = wmass;
            for (int n = 0; n <= N; ++n) {
                const double pn = s_pn[n];
                P.sc.pn[n] = pn;
                P.sc.lam[n] = s_lam[n];
                P.sc.mu[n] = s_mu[n];
                P.sc.alpha[n] = s_alpha[n];
                mass += pn * ((n == N) ? 1.0 : s_lam[n] / P.Lam);
            }
            P.sc.misc[0] = res;
            P.sc.misc[1] = mass;
            P.sc.misc[3] = wmass;
            P.sc.misc[4] = wmean;
            P.sc.misc[2] = (status == HQ_ERR_NUMERIC_CODE) ? 1.0 : 0.0;
            BatchOut o;
            o.iterations = k;
            o.checks = checks;
            o.status = status;
            o.pad = 0;
            o.residual = res;
            outs[ii] = o;
        }
    }
}

// ---------------------------------------------------------------------------
// Dispatch probabilities (unit workloads and response times).  A call from
// node j goes to unit pi_j[h] iff pi_j[0..h-1] are busy and pi_j[h] is
// idle, so with G(S) = sum_{m superset of S} P(m) (superset sums of P),
//   q_j(pi_j[h]) = G(prefix of length h) - G(prefix of length h + 1).
// G comes from an in-place superset-sum transform of P over all N bits, a
// few bits per pass.
// ---------------------------------------------------------------------------
// One pass over bits [L, L + M): thread (hi, lo) holds the 2^M entries
// hi * 2^(L+M) + mid * 2^L + lo in registers; consecutive threads take
// consecutive lo, so loads coalesce once 2^L >= 64.
template <int M>
__global__ __launch_bounds__(256) void zeta_kernel(double* __restrict__ G, int N, int L) {
    const unsigned long long total = 1ull << (N - M);
    const unsigned long long t = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const unsigned long long lo = t & ((1ull << L) - 1ull), hi = t >> L;
    const unsigned long long base = (hi << (L + M)) + lo, stride = 1ull << L;
    double v[1 << M];
#pragma unroll
    for (int k = 0; k < (1 << M); ++k) v[k] = G[base + (unsigned long long)k * stride];
#pragma unroll
    for (int bit = 0; bit < M; ++bit)
#pragma unroll
        for (int k = 0; k < (1 << M); ++k)
            if (!((k >> bit) & 1)) v[k] += v[k | (1 << bit)];
#pragma unroll
    for (int k = 0; k < (1 << M); ++k) G[base + (unsigned long long)k * stride] = v[k];
}

// q[j * N + u] for every node j (one thread each), from the superset sums.
__global__ __launch_bounds__(256) void dispatch_kernel(const double* __restrict__ G, int N, int J,
                                                       const int32_t* __restrict__ pref, double* __restrict__ q) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J) return;
    const int32_t* row = pref + (size_t)j * N;
    double* qj = q + (size_t)j * N;
    uint32_t S = 0u;
    double gs = G[0];
    for (int h = 0; h < N; ++h) {
        const int u = row[h];
        const uint32_t S2 = S | (1u << u);
        const double g2 = G[S2];
        qj[u] = gs - g2;
        S = S2;
        gs = g2;
    }
}

// sums[0] = sum_j lambda_j sum_u q_ju t_ju, sums[1] = sum_j lambda_j sum_u
// q_ju, in a fixed order (one work-group).
__global__ __launch_bounds__(256) void travel_kernel(const double* __restrict__ q, const double* __restrict__ lam,
                                                     const double* __restrict__ travel, int N, int J,
                                                     double* __restrict__ sums) {
    __shared__ double s_a[4], s_b[4];
    double a = 0.0, b = 0.0;
    const size_t total = (size_t)J * N;
    for (size_t i = threadIdx.x; i < total; i += blockDim.x) {
        const double w = lam[i / N] * q[i];
        a += w * travel[i];
        b += w;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        s_a[w] = a;
        s_b[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
        for (int i = 0; i < 4; ++i) {
            x += s_a[i];
            y += s_b[i];
        }
        sums[0] = x;
        sums[1] = y;
    }
}

__global__ void reset_counter_kernel(unsigned int* c) {
    if (threadIdx.x == 0) *c = 0u;
}

__global__ void zero_counters_kernel(unsigned int* c, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) c[i] = 0u;
}

}  // namespace hq

// ---------------------------------------------------------------------------
// Launch wrappers with C++ linkage, called from the host code.
// ---------------------------------------------------------------------------
namespace hqk {

using namespace hq;

// Persistent grid: at most HQ_GRID work-groups, a multiple of 8 when large.
static uint32_t grid_for(uint32_t groups) {
    if (groups < 64) return groups;
    uint32_t g = groups < HQ_GRID ? groups : HQ_GRID;
    return g & ~7u;
}

// Fixed-shape kernels for the default tiles of the larger instances (b = 10
// for N = 16..30) and for b = 12 at N = 28..30: the sweep (with computed
// or stored coefficients) and the residual.  Other shapes and modes use the
// run-time-shaped kernels.
template <typename T, int BF, int HF>
static void launch_fixed(int mode, bool stored, bool track, const SweepParams& P, const LayerArgs& A, T* x,
                         int inner_one, const hqfuse::FuseArgs& F, hipStream_t s) {
    dim3 grid(grid_for(A.groups)), block(HQ_WG);
    if (mode == M_WRITE && stored)
        hipLaunchKernelGGL((layer_kernel<T, M_WRITE, false, true, BF, HF>), grid, block, 0, s, P, A, x, inner_one, F);
    else if (mode == M_WRITE)
        hipLaunchKernelGGL((layer_kernel<T, M_WRITE, false, false, BF, HF>), grid, block, 0, s, P, A, x, inner_one, F);
    else if (mode == M_PASS1 && track)
        hipLaunchKernelGGL((layer_kernel<T, M_PASS1, true, false, BF, HF>), grid, block, 0, s, P, A, x, inner_one, F);
    else if (mode == M_PASS1)
        hipLaunchKernelGGL((layer_kernel<T, M_PASS1, false, false, BF, HF>), grid, block, 0, s, P, A, x, inner_one, F);
    else
        hipLaunchKernelGGL((layer_kernel<T, M_RESID, false, false, BF, HF>), grid, block, 0, s, P, A, x, inner_one, F);
}

// The sweep (computed or stored coefficients, without the delta tracking of
// the paper's stopping rule), the first pass of the closed and literal inner
// forms and the residual, for computed coefficients.
template <typename T>
static bool launch_layer_fixed(int mode, bool stored, bool track, const SweepParams& P, const LayerArgs& A,
                               T* x, int inner_one, const hqfuse::FuseArgs& F, hipStream_t s) {
    if (mode == M_WRITE && track) return false;
    if (mode != M_WRITE && stored) return false;
#define HQ_FIXED(BV, HV)                                                      \
    if (P.b == BV && P.H == HV) {                                             \
        launch_fixed<T, BV, HV>(mode, stored, track, P, A, x, inner_one, F, s); \
        return true;                                                          \
    }
    HQ_FIXED(10, 6) HQ_FIXED(10, 7) HQ_FIXED(10, 8) HQ_FIXED(10, 9) HQ_FIXED(10, 10) HQ_FIXED(10, 11)
    HQ_FIXED(10, 12) HQ_FIXED(10, 13) HQ_FIXED(10, 14) HQ_FIXED(10, 15) HQ_FIXED(10, 16) HQ_FIXED(10, 17)
    HQ_FIXED(10, 18) HQ_FIXED(10, 19) HQ_FIXED(10, 20) HQ_FIXED(12, 16) HQ_FIXED(12, 17) HQ_FIXED(12, 18)
#undef HQ_FIXED
    return false;
}

template <typename T, bool STORED>
static void launch_layer_s(int mode, bool track_delta, const SweepParams& P, const LayerArgs& A, T* x,
                           int inner_one, const hqfuse::FuseArgs& F, hipStream_t s) {
    dim3 grid(grid_for(A.groups)), block(HQ_WG);
    if (launch_layer_fixed<T>(mode, STORED, track_delta, P, A, x, inner_one, F, s)) return;
    if (mode == M_PASS1 && track_delta)
        hipLaunchKernelGGL((layer_kernel<T, M_PASS1, true, STORED>), grid, block, 0, s, P, A, x, inner_one, F);
    else if (mode == M_PASS1)
        hipLaunchKernelGGL((layer_kernel<T, M_PASS1, false, STORED>), grid, block, 0, s, P, A, x, inner_one, F);
    else if (mode == M_WRITE && track_delta)
        hipLaunchKernelGGL((layer_kernel<T, M_WRITE, true, STORED>), grid, block, 0, s, P, A, x, inner_one, F);
    else if (mode == M_WRITE)
        hipLaunchKernelGGL((layer_kernel<T, M_WRITE, false, STORED>), grid, block, 0, s, P, A, x, inner_one, F);
    else
        hipLaunchKernelGGL((layer_kernel<T, M_RESID, false, STORED>), grid, block, 0, s, P, A, x, inner_one, F);
}

uint32_t launch_sweep(int mode, bool track, bool fp32, const SweepParams& P, const LayerArgs& A, void* x,
                      int inner_one, const hqfuse::FuseArgs& F, hipStream_t s);

// One layer launch without its finalize; returns the number of work-group
// partials it writes (at P.partials).
static uint32_t launch_layer_only(int mode, bool track_delta, bool fp32, const SweepParams& P, const LayerArgs& A,
                                  void* x, int inner_one, const hqfuse::FuseArgs& F, hipStream_t s) {
    // the default tile shape runs on the sweep kernels of hq_sweep.hip
    const uint32_t parts = launch_sweep(mode, track_delta, fp32, P, A, x, inner_one, F, s);
    if (parts) return parts;
    if (fp32) {
        if (A.stored)
            launch_layer_s<float, true>(mode, track_delta, P, A, (float*)x, inner_one, F, s);
        else
            launch_layer_s<float, false>(mode, track_delta, P, A, (float*)x, inner_one, F, s);
    } else {
        if (A.stored)
            launch_layer_s<double, true>(mode, track_delta, P, A, (double*)x, inner_one, F, s);
        else
            launch_layer_s<double, false>(mode, track_delta, P, A, (double*)x, inner_one, F, s);
    }
    return grid_for(A.groups);
}

hipError_t launch_layer(int mode, bool track_delta, bool fp32, const SweepParams& P, const LayerArgs& A,
                        void* x, int inner_one, hipStream_t s) {
    const hqfuse::FuseArgs none{nullptr, 0u};
    const uint32_t parts = launch_layer_only(mode, track_delta, fp32, P, A, x, inner_one, none, s);
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(HQ_WG), 0, s, P, mode, A.n, parts, inner_one);
    return hipGetLastError();
}

// The sweeps of layers 1..N-1 of one outer iteration (one update, or the
// look-ahead closed form).  A layer launch forms the previous layer's
// scalars itself (hq_fuse.h) when that layer wrote at most HQ_FUSE_PARTS
// partials; after a larger layer, where every work-group reading all the
// partials would cost more than the one-work-group launch, the finalize
// launch stays.  Layer n writes its partials to half[n & 1].
#define HQ_FUSE_PARTS 1024
hipError_t launch_write_chain(bool track_delta, bool fp32, const SweepParams& P, const LayerArgs* layers, int N,
                              void* x, int inner_one, double* half0, double* half1, bool fuse, hipStream_t s) {
    hqfuse::FuseArgs F{nullptr, 0u};
    SweepParams Pn = P;
    for (int n = 1; n <= N - 1; ++n) {
        Pn.partials = (n & 1) ? half1 : half0;
        const uint32_t parts = launch_layer_only(M_WRITE, track_delta, fp32, Pn, layers[n], x, inner_one, F, s);
        F = hqfuse::FuseArgs{Pn.partials, parts};
        if (!fuse || parts > HQ_FUSE_PARTS || n == N - 1) {
            hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(HQ_WG), 0, s, Pn, (int)M_WRITE, n, parts, inner_one);
            F = hqfuse::FuseArgs{nullptr, 0u};
        }
    }
    return hipGetLastError();
}

hipError_t launch_lookahead(const SweepParams& P, const LayerArgs& A, double* wz, uint32_t nnodes,
                            hipStream_t s) {
    hipLaunchKernelGGL(lookahead_kernel, dim3(grid_for(A.groups)), dim3(HQ_WG), 0, s, P, A, wz, nnodes);
    return hipGetLastError();
}

hipError_t launch_coef(const SweepParams& P, const LayerArgs& A, double* coefs, uint32_t nnodes, hipStream_t s) {
    hipLaunchKernelGGL(coef_kernel, dim3(grid_for(A.groups)), dim3(HQ_WG), 0, s, P, A, coefs, nnodes);
    return hipGetLastError();
}

hipError_t launch_init(bool fp32, const SweepParams& P, const LayerArgs& A, void* x, const double* xu,
                       const double* given, const uint32_t* orig_bit, hipStream_t s) {
    dim3 grid(grid_for(A.groups)), block(HQ_WG);
    if (fp32)
        hipLaunchKernelGGL((init_kernel<float>), grid, block, 0, s, P, A, (float*)x, xu, given, orig_bit);
    else
        hipLaunchKernelGGL((init_kernel<double>), grid, block, 0, s, P, A, (double*)x, xu, given, orig_bit);
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(HQ_WG), 0, s, P, 3, A.n, grid_for(A.groups), 0);
    return hipGetLastError();
}

hipError_t launch_scalars(const SweepParams& P, int want_residual, hipStream_t s) {
    hipLaunchKernelGGL(scalars_kernel, dim3(1), dim3(64), 0, s, P, want_residual);
    return hipGetLastError();
}

hipError_t launch_export(bool fp32, const SweepParams& P, const LayerArgs& A, const void* x, double* out,
                         const uint32_t* orig_bit, int conditional, hipStream_t s) {
    dim3 grid(grid_for(A.groups)), block(HQ_WG);
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
    dim3 grid(grid_for(A.groups)), block(HQ_WG);
    if (fp32)
        hipLaunchKernelGGL((marginal_kernel<float>), grid, block, 0, s, P, A, (const float*)x, part);
    else
        hipLaunchKernelGGL((marginal_kernel<double>), grid, block, 0, s, P, A, (const double*)x, part);
    hipLaunchKernelGGL(marginal_finalize_kernel, dim3(1), dim3(32), 0, s, P, (const double*)part,
                       grid_for(A.groups), rho);
    return hipGetLastError();
}

hipError_t launch_batch(bool fp32, int block, const BatchItem* items, const BatchEntry* entries, BatchOut* outs,
                        int count, unsigned int* next, unsigned int* group_counts, int n_items, int grid,
                        hipStream_t s) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, next);
    hipLaunchKernelGGL(zero_counters_kernel, dim3(n_items > 0 ? (n_items + 255) / 256 : 1), dim3(256), 0, s,
                       group_counts, n_items);
#define HQ_BATCH_CASE(BSZ)                                                                                    \
    case BSZ:                                                                                               \
        if (fp32)                                                                                           \
            hipLaunchKernelGGL((batch_kernel<float, BSZ>), dim3(grid), dim3(BSZ), 0, s, items, entries, outs, count, next); \
        else                                                                                                \
            hipLaunchKernelGGL((batch_kernel<double, BSZ>), dim3(grid), dim3(BSZ), 0, s, items, entries, outs, count, next); \
        break;
    switch (block) {
        HQ_BATCH_CASE(256)
        HQ_BATCH_CASE(512)
        HQ_BATCH_CASE(1024)
        default:
            return hipErrorInvalidValue;
    }
#undef HQ_BATCH_CASE
    return hipGetLastError();
}

// Scratch of the allocation-free batched solve: one copy of this array on
// every GPU the library runs on, held until the process ends.  Host code
// never passes `scratch` itself to a kernel (on the host it only names the
// symbol); it uses the device address hipGetSymbolAddress returns for the
// current device, looked up once per device.
static __device__ __align__(256) unsigned char scratch[sizeof(BatchScratch)];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[HQ_MAX_DEVICES] = {};

hipError_t noalloc_scratch(int device, BatchScratch** out) {
    *out = nullptr;
    if (device < 0 || device >= HQ_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
        void* ptr = nullptr;
        e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = ptr;
    }
    *out = static_cast<BatchScratch*>(g_scratch_ptr[device]);
    return hipSuccess;
}

hipError_t launch_dispatch(double* G, int N, int J, const int32_t* pref, double* q, const double* lam,
                           const double* travel, double* sums, hipStream_t s) {
    for (int L = 0; L < N;) {
        const int M = N - L < 5 ? N - L : 5;
        const unsigned long long threads = 1ull << (N - M);
        const dim3 grid((unsigned)((threads + 255) / 256)), block(256);
        switch (M) {
            case 1: hipLaunchKernelGGL(zeta_kernel<1>, grid, block, 0, s, G, N, L); break;
            case 2: hipLaunchKernelGGL(zeta_kernel<2>, grid, block, 0, s, G, N, L); break;
            case 3: hipLaunchKernelGGL(zeta_kernel<3>, grid, block, 0, s, G, N, L); break;
            case 4: hipLaunchKernelGGL(zeta_kernel<4>, grid, block, 0, s, G, N, L); break;
            default: hipLaunchKernelGGL(zeta_kernel<5>, grid, block, 0, s, G, N, L); break;
        }
        L += M;
    }
    hipLaunchKernelGGL(dispatch_kernel, dim3((J + 255) / 256), dim3(256), 0, s, (const double*)G, N, J, pref, q);
    if (travel) hipLaunchKernelGGL(travel_kernel, dim3(1), dim3(256), 0, s, (const double*)q, lam, travel, N, J, sums);
    return hipGetLastError();
}

hipError_t launch_widen(const float* src, double* dst, uint32_t begin, uint32_t count, double factor,
                        hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(widen_kernel, dim3((count + 255) / 256), dim3(256), 0, s, src, dst, begin, count, factor);
    return hipGetLastError();
}

}  // namespace hqk
