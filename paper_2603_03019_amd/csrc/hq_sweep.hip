// The layer sweep for the default tile shape (b = 10 low bits per tile,
// H = N - 10 high bits, N = 16..26): one kernel per layer launch that
// evaluates, for every state m of layer n, the two gathers of the update
// (12) of Algorithm 1,
//     U~(m) = sum_{u in m}    a(m, u) p_{n-1}(m \ u) / (Lambda + mu_m),
//     D~(m) = sum_{u notin m} nu_u    p_{n+1}(m + u) / (Lambda + mu_m),
// and then writes p_n(m) = alpha_n U~ + beta_n D~ (sweep), reduces the
// layer sums of the inner mu(n) loop (first pass of the closed and literal
// forms), or evaluates the balance residual of (1) (check).
//
// Mapping.  A 64-lane wave owns one segment (tile T, low class q) at a time:
// the C(10, q) states that share their high bits, lane t taking states t,
// t + 64, ...  What is uniform over the segment comes from a precomputed
// 128-byte record (neighbour segment starts, the tile's program position,
// the service-rate sum of the busy high units), fetched lane-parallel two
// segments ahead.  What depends on the low pattern comes from a 40-byte row
// per (q, t), read coalesced: for the pattern's q set bits (increasing) the
// offset of the neighbour L minus that bit inside segment (T, q - 1) of layer
// n - 1, then for its 10 - q clear bits the offset of L plus that bit inside
// (T, q + 1) of layer n + 1, each with the LDS slot of its weight, and the
// service-rate sum of the pattern's units.  So entry i is a down-neighbour
// for every lane iff i < q: no per-lane branch.  High-bit neighbours sit at
// the same offset t of segment (T xor 2^k, q) and are read as contiguous
// runs.  Every load and store goes through one buffer resource spanning
// layers n - 1 .. n + 1, with the segment starts as scalar offsets.
//
// Weights.  Per segment, lane u forms the weight of unit u in the combined
// sum: alpha-side (tile coefficient of a busy unit, eq. (3) / Algorithm 3)
// or beta-side (service rate of an idle unit), with the layer scalars and
// storage scales folded in.  All weights go to a per-wave LDS slot: a
// high unit's is read as a broadcast, a low unit's by the lane's entry.
// Per-tile program terms (busy units whose coefficient depends on low
// bits) are added for the units the record marks, each unit's terms summed
// first and multiplied once by its neighbour value: a high unit's value is
// still in registers (the first two such units get a second copy loaded
// next to the others, the rest are selected from the loaded set), a low
// unit's is read again from the staging area.
//
// Arithmetic is FP64 throughout; with FP32 storage the neighbour values are
// widened on load and the written value rounded once.
#include "hq_fuse.h"
#include "hq_internal.h"

#include <math.h>

namespace hqsweep {

#define HQ_CONST __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const HQ_CONST T* cro(const T* p) {
    return (const HQ_CONST T*)p;
}

constexpr int B = HQ_SWEEP_B;  // low bits per tile
constexpr int WAVES = HQ_WG / 64;
constexpr int RSRC_W3 = 0x00020000;  // buffer resource word 3 on gfx9 (32-bit data format, raw)
constexpr int HQ_AUX_NT = 2;         // cache-policy operand of a buffer load: non-temporal

// S_WRITE_LA: the sweep of the closed inner form, which also accumulates
// the look-ahead sums of the next layers' alpha
enum { S_WRITE = 0, S_PASS1 = 1, S_RESID = 2, S_WRITE_LA = 3 };

__device__ __forceinline__ uint32_t rl(uint32_t v, int i) { return (uint32_t)__builtin_amdgcn_readlane((int)v, i); }
__device__ __forceinline__ double rld(double v, int i) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const uint32_t lo = rl((uint32_t)b, i), hi = rl((uint32_t)(b >> 32), i);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The lane index, as a value the compiler cannot hoist out of a loop (the
// empty volatile asm): offsets derived from it are formed where a load
// needs them instead of being held in registers across the state loop.
__device__ __forceinline__ uint32_t lane_now() {
    uint32_t l = threadIdx.x & 63u;
    asm volatile("" : "+v"(l));
    return l;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}

// 1 / d for d > 0: the hardware reciprocal refined by two Newton steps.
__device__ __forceinline__ double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

template <typename T>
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
        return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, T v, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, 0);
}

// Layer scalars of one launch.  wa/wb: factors of the alpha-side (busy
// unit, tile coefficient) and beta-side (idle unit, service rate) weights.
struct Scal {
    double wa, wb;            // S_WRITE: alpha s_self / s_dn, beta s_self / s_up; S_RESID: p(n-1) / s_dn,
                              // p(n+1) / s_up; S_PASS1: 1 / s_dn, 1 / s_up (two sums)
    double alpha0, beta0;     // literal loop: first inner step
    double is_self, pself;    // inverse storage scale of layer n; p(n) (residual)
};

// fused: lambda^k(n-1) (and with the look-ahead alpha_n) come from the
// launch's own reduction of the previous layer's partials (hq_fuse.h)
template <int MODE>
__device__ __forceinline__ Scal load_scal(const SweepParams& P, int n, int inner_one, bool fused,
                                          const hqfuse::Prev& pv) {
    Scal s{};
    const int N = P.N;
    const double is_dn = P.inv_scale[n - 1], is_up = P.inv_scale[n + 1];
    s.is_self = P.inv_scale[n];
    if (MODE == S_RESID) {
        s.wa = P.sc.pn[n - 1] * is_dn;
        s.wb = P.sc.pn[n + 1] * is_up;
        s.pself = P.sc.pn[n];
    } else {
        const double beta = P.sc.lam[n] / P.sc.mu[n + 1];    // lambda^{k-1}(n) / mu^{k-1}(n+1)
        const double lam_prev = fused ? pv.lam_prev : P.sc.lam[n - 1];
        const double alpha0 = P.sc.mu[n] / lam_prev;  // mu^{k-1}(n) / lambda^k(n-1)
        s.alpha0 = alpha0;
        s.beta0 = beta;
        if (MODE == S_WRITE || MODE == S_WRITE_LA) {
            const double alpha = inner_one == 1 ? alpha0 : (fused && P.la ? pv.alpha_la : P.sc.alpha[n]);
            const double s_self = P.scale[n];
            s.wa = alpha * is_dn * s_self;
            s.wb = beta * is_up * s_self;
        } else {
            s.wa = is_dn;
            s.wb = is_up;
        }
    }
    (void)N;
    return s;
}

// Sum of the rates of unit u's program terms whose low mask lies in L (nL
// = ~L).  The tile's first 64 terms are held lane-parallel (mask in tmk,
// rate in trt); terms past 64 are read as scalar loads.  pov: lane u holds
// the absolute index of unit u's first term, pstart that of the tile's.
__device__ __forceinline__ double unit_terms(const HQ_CONST ProgTerm* pg, uint32_t pov, uint32_t pstart, uint32_t tmk,
                                             double trt, int u, uint32_t nL) {
    const uint32_t i0 = rl(pov, u) - pstart, i1 = rl(pov, u + 1) - pstart;
    const uint32_t ir = i1 < 64u ? i1 : 64u;
    double c = 0.0;
    for (uint32_t i = i0; i < ir; ++i) {
        const uint32_t mk = rl(tmk, (int)i);
        const double rt = rld(trt, (int)i);
        c += (mk & nL) == 0u ? rt : 0.0;
    }
    for (uint32_t i = i0 > 64u ? i0 : 64u; i < i1; ++i) {
        const uint32_t mk = pg[i].mask;
        const double rt = pg[i].rate;
        c += (mk & nL) == 0u ? rt : 0.0;
    }
    return c;
}

// vh[k] for a wave-uniform k, by a chain of selects (the values stay in
// registers; no indexed private array, no memory round trip).
template <int HF>
__device__ __forceinline__ double pick(const double (&vh)[HF], int k) {
    double v = vh[0];
#pragma unroll
    for (int j = 1; j < HF; ++j) {
        v = k == j ? vh[j] : v;
        // keeps the chain a chain of selects (not an indexed private array)
        asm volatile("" : "+v"(v));
    }
    return v;
}

// One wave, one segment.  HF = H (high bits), fixed at compile time.
template <typename T, int MODE, bool TRACK, int HF>
__device__ __forceinline__ void segment(const SweepParams& P, __amdgpu_buffer_rsrc_t xr,
                                        __amdgpu_buffer_rsrc_t rowr, const uint32_t base, const uint32_t rec,
                                        const double tcv, const uint32_t pov, const uint32_t tmk, const double trt,
                                        const Scal& s, double* wlds, T* stage, const uint16_t* s_rank,
                                        double& acc0, double& acc1, double& acc2, double& acc3, double& acc4,
                                        double& acc5, __amdgpu_buffer_rsrc_t lar, const uint32_t lbase,
                                        const double* s_nu) {
    constexpr uint32_t SZ = sizeof(T);
    const int lane = threadIdx.x & 63;
    const uint32_t desc = rl(rec, HQ_REC_DESC);
    const int q = (int)(desc & 15u);
    const uint32_t Tb = desc >> 4;
    // scalar byte offsets inside the window (layers n-1 .. n+1); a segment
    // without down- or up-neighbour segment gets 0, which nothing then reads
    const uint32_t o_self = (rl(rec, HQ_REC_SELF) - base) * SZ;
    const uint32_t o_dn = q > 0 ? (rl(rec, HQ_REC_DN) - base) * SZ : 0u;
    const uint32_t o_up = q < B ? (rl(rec, HQ_REC_UP) - base) * SZ : 0u;
    uint32_t o_hi[HF];
#pragma unroll
    for (int k = 0; k < HF; ++k) o_hi[k] = (rl(rec, HQ_REC_HI + k) - base) * SZ;
    const double mu_hi = __longlong_as_double(
        (long long)(((unsigned long long)rl(rec, HQ_REC_MUHI + 1) << 32) | rl(rec, HQ_REC_MUHI)));
    const double den_hi = P.Lam + mu_hi;
    const uint32_t cnt = cro(P.binom)[B * 32 + q];
    const uint32_t cnt_dn = q > 0 ? cro(P.binom)[B * 32 + q - 1] : 0u;
    const uint32_t cnt_up = q < B ? cro(P.binom)[B * 32 + q + 1] : 0u;
    const uint32_t qs = cro(P.lo_qstart)[q];
    const uint32_t pmask = rl(rec, HQ_REC_PMASK);
    // the first two high units with program terms: their neighbour values
    // are loaded a second time, next to the others, for the term step
    const uint32_t hm = pmask >> B;
    const int k0 = hm ? __builtin_ctz(hm) : -1;
    const uint32_t hm1 = hm & (hm - 1u);
    const int k1 = hm1 ? __builtin_ctz(hm1) : -1;
    const uint32_t o_t0 = k0 >= 0 ? (rl(rec, HQ_REC_HI + k0) - base) * SZ : o_self;
    const uint32_t o_t1 = k1 >= 0 ? (rl(rec, HQ_REC_HI + k1) - base) * SZ : o_self;
    const uint32_t pstart = rl(rec, HQ_REC_PSTART);
    const HQ_CONST ProgTerm* pg = cro(P.prog) + pstart;
    // weights: lane u < N holds unit u's; alpha-side for busy units (tile
    // coefficient), beta-side for idle ones (service rate)
    const double nu_l = s_nu[lane];
    const bool busy_hi = lane >= B && lane < P.N && ((Tb >> (lane - B)) & 1u);
    // (PASS1 keeps the two sides apart, side factors applied at the end)
    const double wA = MODE == S_PASS1 ? (busy_hi ? tcv : nu_l) : (busy_hi ? s.wa * tcv : s.wb * nu_l);
    // The previous segment's LDS reads of this wave are done (a wave's LDS
    // operations complete in order).  Then the weights go to this wave's
    // slots: low unit l busy at [l], idle at [16 + l]; high unit B + k at
    // [32 + k]; and the low-neighbour segments (T, q - 1) of layer n - 1 and
    // (T, q + 1) of layer n + 1 go to this wave's staging area, one after the
    // other.  (Issuing all of a segment's staging loads before the first LDS
    // write needs up to 16 more registers here, which spill in the look-ahead
    // instantiation and made it slower.)
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane < B) {
        wlds[lane] = MODE == S_PASS1 ? tcv : s.wa * tcv;
        wlds[16 + lane] = MODE == S_PASS1 ? nu_l : s.wb * nu_l;
    } else if (lane < P.N) {
        wlds[32 + lane - B] = wA;
    }
    const uint32_t la_o = (rl(rec, HQ_REC_SELF) - lbase) * 16u;
    for (uint32_t i = lane; i < cnt_dn; i += 64) stage[i] = (T)bload<T>(xr, i * SZ, o_dn);
    for (uint32_t i = lane; i < cnt_up; i += 64) stage[cnt_dn + i] = (T)bload<T>(xr, i * SZ, o_up);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();

    for (uint32_t t = lane; t < cnt; t += 64) {
        // weights are read from LDS in every pass (kept out of registers)
        asm volatile("" ::: "memory");
        const uint32_t ro = (qs + t) * (uint32_t)sizeof(LowRow);
        // row: L | off[10] | slot[10] | mu_lo
        const auto r0 = __builtin_amdgcn_raw_buffer_load_b128(rowr, ro, 0, 0);
        const auto r1 = __builtin_amdgcn_raw_buffer_load_b128(rowr, ro + 16, 0, 0);
        const double mu_lo = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rowr, ro + 32, 0, 0));
        const uint32_t w[8] = {r0[0], r0[1], r0[2], r0[3], r1[0], r1[1], r1[2], r1[3]};
        const uint32_t L = w[0] & 0xffffu;
        const uint32_t t8 = t * SZ;
        // every neighbour value first: high-bit neighbours from memory, the
        // low-bit ones from the staged segments
        double vl[B], vh[HF];
#pragma unroll
        for (int k = 0; k < HF; ++k) vh[k] = bload<T>(xr, t8, o_hi[k]);
        const double vt0 = bload<T>(xr, t8, o_t0), vt1 = bload<T>(xr, t8, o_t1);
        // closed form: the look-ahead pair (w, z) of this state, one 16-byte
        // load in flight with the neighbours; the pairs are read once per
        // sweep, so the load is marked non-temporal (they should not push
        // neighbour values out of the L2)
        double lw = 0.0, lz = 0.0;
        if (MODE == S_WRITE_LA) {
            const u32x4 wz = __builtin_amdgcn_raw_buffer_load_b128(lar, la_o + t * 16u, 0, HQ_AUX_NT);
            lw = __builtin_bit_cast(double, (unsigned long long)wz[0] | ((unsigned long long)wz[1] << 32));
            lz = __builtin_bit_cast(double, (unsigned long long)wz[2] | ((unsigned long long)wz[3] << 32));
        }
#pragma unroll
        for (int i = 0; i < B; ++i) {
            // off[i] is the 16-bit field at byte 2 + 2 i: byte offset in the staging area
            const uint32_t word = w[(2 + 2 * i) >> 2];
            const uint32_t off = ((2 + 2 * i) & 3) ? (word >> 16) : (word & 0xffffu);
            vl[i] = (double)*(const T*)((const char*)stage + off);
        }
        double A = 0.0, Bs = 0.0;
#pragma unroll
        for (int i = 0; i < B; ++i) {
            // slot[i] is the byte at 22 + i
            const uint32_t word = w[(22 + i) >> 2];
            const uint32_t slot = (word >> (8 * ((22 + i) & 3))) & 0xffu;
            const double wl = *(const double*)((const char*)wlds + slot);
            if (MODE == S_PASS1) {
                if (i < q)
                    A = fma(wl, vl[i], A);
                else
                    Bs = fma(wl, vl[i], Bs);
            } else {
                A = fma(wl, vl[i], A);
            }
        }
#pragma unroll
        for (int k = 0; k < HF; ++k) {
            if (MODE == S_PASS1 && !((Tb >> k) & 1u))
                Bs = fma(wlds[32 + k], vh[k], Bs);
            else
                A = fma(wlds[32 + k], vh[k], A);
        }
        // per-tile program terms: a busy unit u gains `rate` in the states
        // whose low bits contain the term's mask.  The unit's terms are summed
        // first, then multiplied once by its neighbour value: a high unit's
        // from registers (the second copy of the first two such units, a
        // select over the loaded set for the others), a low unit's read
        // again from the staging area and kept only where the unit is busy.
        const uint32_t nL = ~L;
        uint32_t um = pmask;
        while (um) {
            const int u = __builtin_ctz(um);
            um &= um - 1u;
            double c = unit_terms(pg, pov, pstart, tmk, trt, u, nL);
            double v;
            if (u < B) {
                const bool bz = (L >> u) & 1u;
                const uint32_t rk = bz ? (uint32_t)s_rank[L ^ (1u << u)] : 0u;
                v = (double)stage[rk];
                c = bz ? c : 0.0;
            } else if (u - B == k0) {
                v = vt0;
            } else if (u - B == k1) {
                v = vt1;
            } else {
                v = pick<HF>(vh, u - B);
            }
            A = fma(MODE == S_PASS1 ? c : s.wa * c, v, A);
        }
        const double mu_m = mu_hi + mu_lo;
        const double inv = recip(den_hi + mu_lo);
        if (MODE == S_RESID) {
            // in = p(n-1) U + p(n+1) D (weights), out = p(n) p_n(m) (Lambda + mu_m)
            const double self_v = bload<T>(xr, t8, o_self) * s.is_self;
            const double out = s.pself * self_v * (P.Lam + mu_m);
            acc0 += fabs(A - out);
            acc1 += out;
        } else if (MODE == S_PASS1) {
            const double Ut = A * s.wa * inv, Dt = Bs * s.wb * inv;
            if (TRACK) {
                acc0 = fma(mu_m, Ut, acc0);
                acc1 = fma(mu_m, Dt, acc1);
                acc2 = fmax(acc2, Ut);
                const double v0 = s.alpha0 * Ut + s.beta0 * Dt;
                acc3 = fmax(acc3, fabs(v0 - bload<T>(xr, t8, o_self) * s.is_self));
            } else {
                acc0 += Ut;
                acc1 = fma(mu_m, Dt, acc1);
            }
        } else {
            const T stored = (T)(A * inv);  // already scaled for storage
            if (TRACK) acc2 = fmax(acc2, fabs((double)stored - bload<T>(xr, t8, o_self)) * s.is_self);
            bstore<T>(xr, stored, t8, o_self);
            const double ps = (double)stored * s.is_self;
            acc0 += ps;
            acc1 = fma(mu_m, ps, acc1);
            if (MODE == S_WRITE_LA) {
                // look-ahead closed form: the sums the next layers' alpha needs
                acc4 = fma(ps, lw, acc4);
                acc5 = fma(ps, lz, acc5);
            }
        }
    }
}

template <typename T, int MODE, bool TRACK, int HF>
__global__ __launch_bounds__(HQ_WG) __attribute__((amdgpu_waves_per_eu(MODE == S_PASS1 ? 4 : 5, 8))) void sweep_kernel(SweepParams P, LayerArgs A, T* __restrict__ x,
                                                      int inner_one, hqfuse::FuseArgs F) {
    __shared__ double s_w[WAVES * 64];
    __shared__ T s_stage[WAVES][HQ_SWEEP_STAGE];  // per wave: segments (T, q - 1) and (T, q + 1)
    __shared__ uint16_t s_rank[1 << B];
    __shared__ double s_red[HQ_NPART][WAVES];
    __shared__ double s_nu[64];  // service rates, 0 past N
    const int tid = threadIdx.x, lane = tid & 63;
    for (int i = tid; i < (1 << B); i += HQ_WG) s_rank[i] = P.lo_rank[i];
    if (tid < 64) s_nu[tid] = tid < P.N ? P.nu[tid] : 0.0;
    __syncthreads();
    const int n = A.n;
    // the previous layer's scalars, when its finalize launch is fused into this one
    const bool fused = (MODE == S_WRITE || MODE == S_WRITE_LA) && F.prev != nullptr;
    hqfuse::Prev pv{0.0, 0.0};
    if (fused) pv = hqfuse::prologue<HQ_WG>(P, n, inner_one, F, s_red);
    const Scal s = load_scal<MODE>(P, n, inner_one, fused, pv);
    // the window of layers n - 1 .. n + 1 (offsets fit 32 bits up to N = 30)
    const uint32_t base = cro(P.layer_off)[n - 1];
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(x + base, 0, -1, RSRC_W3);
    const LowRow* rows = sizeof(T) == 8 ? P.lrow : P.lrow32;
    const __amdgpu_buffer_rsrc_t rowr = __builtin_amdgcn_make_buffer_rsrc(const_cast<LowRow*>(rows), 0,
                                                                          (1 << B) * (int)sizeof(LowRow), RSRC_W3);
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0, acc4 = 0.0, acc5 = 0.0;
    // look-ahead pairs (w, z) of layer n, 16 bytes per state
    const uint32_t lbase = cro(P.layer_off)[n];
    const __amdgpu_buffer_rsrc_t lar = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double*>(MODE == S_WRITE_LA ? P.la + 2 * (size_t)lbase : P.partials), 0, -1, RSRC_W3);
    // wave-granular segments; the eight XCDs sweep contiguous eighths
    const uint32_t G = gridDim.x, wg = blockIdx.x;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    uint32_t begin, end, step;
    if (G < 64 || (G & 7u)) {
        begin = wg * WAVES + wv;
        end = A.groups;
        step = G * WAVES;
    } else {
        const uint32_t xcd = wg & 7u, per = (A.groups + 7u) >> 3;
        const uint32_t lo = xcd * per;
        begin = lo + (wg >> 3) * WAVES + wv;
        end = min(A.groups, lo + per);
        step = (G >> 3) * WAVES;
    }
    double* wlds = s_w + wv * 64;
    // The record of segment i + 2 and the tile coefficients and program
    // offsets of segment i + 1 are in flight while segment i is processed.
    // They are read through buffer resources at clamped offsets (always
    // inside the arrays): no lane-masked branch around a load, and no
    // per-lane 64-bit address held across the state loop (such addresses
    // were spilled to scratch and reloaded, with a full wait, per segment).
    // A segment index past the wave's share reads the share's last record,
    // which nothing then uses.
    const __amdgpu_buffer_rsrc_t recr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t*>(P.srec + (size_t)A.desc_base * HQ_REC_WORDS), 0, -1, RSRC_W3);
    const __amdgpu_buffer_rsrc_t tcr = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(P.tcoef), 0, -1, RSRC_W3);
    const __amdgpu_buffer_rsrc_t por =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(P.prog_off), 0, -1, RSRC_W3);
    const __amdgpu_buffer_rsrc_t pgr = __builtin_amdgcn_make_buffer_rsrc(const_cast<ProgTerm*>(P.prog), 0, -1, RSRC_W3);
    const uint32_t last = end > 0u ? end - 1u : 0u;
    const uint32_t Nu = (uint32_t)P.N;
    auto load_rec = [&](uint32_t si) -> uint32_t {
        const uint32_t l = lane_now();
        return __builtin_amdgcn_raw_buffer_load_b32(recr, min(l, (uint32_t)HQ_REC_WORDS - 1u) * 4u,
                                                    min(si, last) * (uint32_t)(HQ_REC_WORDS * 4), 0);
    };
    // tile data of a segment, lane-parallel: lane u its tile coefficient and
    // the absolute index of its first program term, lane i the mask and rate
    // of program term i < 64 (lanes past the counts hold copies of the last
    // entry, which nothing reads)
    struct Tile {
        double tcv, trt;
        uint32_t pov, tmk;
    };
    auto load_tile = [&](uint32_t rec) -> Tile {
        Tile tl{0.0, 0.0, 0u, 0u};
        const uint32_t l = lane_now();
        const uint32_t Tb = rl(rec, HQ_REC_DESC) >> 4;
        tl.tcv = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(tcr, min(l, Nu - 1u) * 8u,
                                                                                 Tb * Nu * 8u, 0));
        if (rl(rec, HQ_REC_PMASK) != 0u) {
            const uint32_t pstart = rl(rec, HQ_REC_PSTART), pcount = rl(rec, HQ_REC_PCOUNT);
            tl.pov = __builtin_amdgcn_raw_buffer_load_b32(por, min(l, Nu) * 4u, Tb * (Nu + 1u) * 4u, 0);
            const u32x4 tm = __builtin_amdgcn_raw_buffer_load_b128(pgr, min(l, pcount - 1u) * 16u, pstart * 16u, 0);
            tl.tmk = tm[0];
            tl.trt = __builtin_bit_cast(double, (unsigned long long)tm[2] | ((unsigned long long)tm[3] << 32));
        }
        return tl;
    };
    T* stage = s_stage[wv];
    uint32_t rec0 = load_rec(begin), rec1 = load_rec(begin + step);
    Tile t0 = load_tile(rec0);
    for (uint32_t si = begin; si < end; si += step) {
        const uint32_t rec2 = load_rec(si + 2 * step);
        const Tile t1 = load_tile(rec1);
        segment<T, MODE, TRACK, HF>(P, xr, rowr, base, rec0, t0.tcv, t0.pov, t0.tmk, t0.trt, s, wlds, stage, s_rank,
                                    acc0, acc1, acc2, acc3, acc4, acc5, lar, lbase, s_nu);
        rec0 = rec1;
        rec1 = rec2;
        t0 = t1;
    }
    // work-group partials (sum, sum, max, max); the finalize launch adds
    // them in a fixed order
    acc0 = wave_sum(acc0);
    acc1 = wave_sum(acc1);
    acc2 = wave_max(acc2);
    acc3 = wave_max(acc3);
    acc4 = wave_sum(acc4);
    acc5 = wave_sum(acc5);
    if (lane == 0) {
        s_red[0][wv] = acc0;
        s_red[1][wv] = acc1;
        s_red[2][wv] = acc2;
        s_red[3][wv] = acc3;
        s_red[4][wv] = acc4;
        s_red[5][wv] = acc5;
    }
    __syncthreads();
    if (tid == 0) {
        double b[HQ_NPART] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int i = 0; i < WAVES; ++i) {
            b[0] += s_red[0][i];
            b[1] += s_red[1][i];
            b[2] = fmax(b[2], s_red[2][i]);
            b[3] = fmax(b[3], s_red[3][i]);
            b[4] += s_red[4][i];
            b[5] += s_red[5][i];
        }
        double* pp = P.partials + (size_t)blockIdx.x * HQ_NPART;
        for (int j = 0; j < HQ_NPART; ++j) pp[j] = b[j];
    }
}

}  // namespace hqsweep

namespace hqk {

using namespace hqsweep;

// Work-groups of one launch: every wave owns whole segments, and the grid
// never exceeds what the device holds at once (the kernel's occupancy times
// the compute units), so no work-group waits for another to finish before
// it starts its share; a multiple of 8 when large (XCD-chunked order).
template <typename T, int MODE, bool TRACK, int HF>
static uint32_t resident_groups() {
    static const uint32_t r = [] {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sweep_kernel<T, MODE, TRACK, HF>, HQ_WG, 0) !=
                hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        (void)hipGetLastError();
        return (uint32_t)(per_cu * cus);
    }();
    return r;
}

template <typename T, int MODE, bool TRACK, int HF>
static uint32_t sweep_grid(uint32_t groups) {
    const uint32_t wgs = (groups + WAVES - 1) / WAVES;
    if (wgs < 64) return wgs > 0 ? wgs : 1;
    const uint32_t cap = resident_groups<T, MODE, TRACK, HF>();
    uint32_t g = wgs < cap ? wgs : cap;
    return g >= 8 ? g & ~7u : g;
}

template <typename T, int MODE, bool TRACK, int HF>
static uint32_t launch_one(const SweepParams& P, const LayerArgs& A, T* x, int inner_one, const hqfuse::FuseArgs& F,
                           hipStream_t s) {
    const uint32_t g = sweep_grid<T, MODE, TRACK, HF>(A.groups);
    hipLaunchKernelGGL((sweep_kernel<T, MODE, TRACK, HF>), dim3(g), dim3(HQ_WG), 0, s, P, A, x, inner_one, F);
    return g;
}

template <typename T, int HF>
static uint32_t launch_h(int mode, bool track, const SweepParams& P, const LayerArgs& A, T* x, int inner_one,
                         const hqfuse::FuseArgs& F, hipStream_t s) {
    if (mode == 1 /* M_WRITE */ && P.la)
        return track ? 0u : launch_one<T, S_WRITE_LA, false, HF>(P, A, x, inner_one, F, s);
    if (mode == 1 && !track) return launch_one<T, S_WRITE, false, HF>(P, A, x, inner_one, F, s);
    if (mode == 1) return launch_one<T, S_WRITE, true, HF>(P, A, x, inner_one, F, s);
    const hqfuse::FuseArgs none{nullptr, 0u};
    if (mode == 0 /* M_PASS1 */ && track) return launch_one<T, S_PASS1, true, HF>(P, A, x, inner_one, none, s);
    if (mode == 0) return launch_one<T, S_PASS1, false, HF>(P, A, x, inner_one, none, s);
    return launch_one<T, S_RESID, false, HF>(P, A, x, inner_one, none, s);
}

// Launch the sweep kernel of layer A.n for the default tile shape; returns
// the number of work-groups (whose partials the finalize launch reads), or
// 0 when this shape or layer is not covered (stored coefficients, long
// tile programs, another tile width, the end layers of the residual, the
// closed form's sweep with the paper's delta tracking).
uint32_t launch_sweep(int mode, bool track, bool fp32, const SweepParams& P, const LayerArgs& A, void* x,
                      int inner_one, const hqfuse::FuseArgs& F, hipStream_t s) {
    if (P.b != B || A.stored || A.general || !P.srec || !P.lrow || A.n < 1 || A.n >= P.N) return 0;
#define HQ_SW(HV)                                                                     \
    case HV:                                                                          \
        return fp32 ? launch_h<float, HV>(mode, track, P, A, (float*)x, inner_one, F, s) \
                    : launch_h<double, HV>(mode, track, P, A, (double*)x, inner_one, F, s);
    switch (P.H) {
        HQ_SW(6) HQ_SW(7) HQ_SW(8) HQ_SW(9) HQ_SW(10) HQ_SW(11) HQ_SW(12) HQ_SW(13) HQ_SW(14) HQ_SW(15)
        HQ_SW(16)
        default:
            return 0;
    }
#undef HQ_SW
}

}  // namespace hqk
