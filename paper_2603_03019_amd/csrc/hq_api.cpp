// Host side of libhq: the C ABI of include/hq.h, instance preprocessing and
// the orchestration of Algorithm 1 on one GPU.
#include <hip/hip_runtime.h>

#include <atomic>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hq.h"
#include "hq_internal.h"
#include "hq_batchplan.h"
#include "hq_init.h"
#include "hq_layout.h"
#include "hq_schedule.h"
#include "hq_sweeptab.h"

namespace hqk {
hipError_t launch_layer(int mode, bool track_delta, bool fp32, const SweepParams& P, const LayerArgs& A, void* x,
                        int inner_one, hipStream_t s);
hipError_t launch_write_chain(bool track_delta, bool fp32, const SweepParams& P, const LayerArgs* layers, int N,
                              void* x, int inner_one, double* half0, double* half1, bool fuse, hipStream_t s);
hipError_t launch_init(bool fp32, const SweepParams& P, const LayerArgs& A, void* x, const double* xu,
                       const double* given, const uint32_t* orig_bit, hipStream_t s);
hipError_t launch_scalars(const SweepParams& P, int want_residual, hipStream_t s);
hipError_t launch_export(bool fp32, const SweepParams& P, const LayerArgs& A, const void* x, double* out,
                         const uint32_t* orig_bit, int conditional, hipStream_t s);
hipError_t launch_marginal(bool fp32, const SweepParams& P, const LayerArgs& A, const void* x, double* part,
                           double* rho, hipStream_t s);
hipError_t launch_dispatch(double* G, int N, int J, const int32_t* pref, double* q, const double* lam,
                           const double* travel, double* sums, hipStream_t s);
hipError_t launch_widen(const float* src, double* dst, uint32_t begin, uint32_t count, double factor,
                        hipStream_t s);
hipError_t launch_coef(const SweepParams& P, const LayerArgs& A, double* coefs, uint32_t nnodes, hipStream_t s);
hipError_t launch_lookahead(const SweepParams& P, const LayerArgs& A, double* wz, uint32_t nnodes,
                            hipStream_t s);
hipError_t launch_batch(bool fp32, int block, const BatchItem* items, const BatchEntry* entries, BatchOut* outs,
                        int count, unsigned int* next, unsigned int* group_counts, int n_items, int grid,
                        hipStream_t s);
hipError_t noalloc_scratch(int device, BatchScratch** out);
}  // namespace hqk

// automatic choice of stored-coefficient layers (see hq_create)
#define HQ_STORE_TERMS 32.0
// layers of at least this many program terms per state go to the general
// layer kernel rather than the default-shape sweep
#define HQ_GENERAL_TERMS 10.0
#define HQ_STORE_BYTES (16ull << 30)

namespace {

enum { M_PASS1 = 0, M_WRITE = 1, M_RESID = 2 };

thread_local std::string g_err;

hq_status fail(hq_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

}  // namespace

void hq_set_error(const std::string& msg) { g_err = msg; }
hq_status hq_mlp_predict_instance(const hq_mlp* mc, int N, int J, const double* lam, const double* mu,
                                  const int32_t* pref, std::vector<double>& rho);

namespace {

struct HipError {
    hipError_t e;
    const char* what;
};

#define HQ_HIP(call)                                   \
    do {                                               \
        hipError_t _e = (call);                        \
        if (_e != hipSuccess) throw HipError{_e, #call}; \
    } while (0)

template <typename T>
T* dalloc(size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) throw std::bad_alloc();
    return static_cast<T*>(p);
}

template <typename T>
void h2d(T* d, const std::vector<T>& h, hipStream_t s) {
    if (!h.empty()) HQ_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

double binom_d(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return std::floor(r + 0.5);
}

}  // namespace

struct hq_ctx {
    int N = 0, J = 0, b = 0, H = 0, device = 0;
    double Lam = 0.0;
    bool lam_zero = false;
    hq_options opts{};
    std::vector<double> rho_init;    // relabelled
    std::vector<double> x_init;      // product-form weights calibrated to rho_init
    std::vector<double> state_init;  // original bitmask order
    std::vector<int> orig;           // new label -> original unit
    std::vector<double> nu;          // relabelled service rates
    std::vector<double> lam_in;      // lambda_j as given
    std::vector<int32_t> pref_in;    // preference lists as given (original unit labels)
    std::vector<TrieNode> nodes;
    size_t max_groups = 0;
    std::vector<LayerArgs> layers;   // per layer n = 0..N
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // device memory
    double* x64 = nullptr;
    float* x32 = nullptr;
    double *d_nu = nullptr, *d_tcoef = nullptr, *d_scal = nullptr, *d_part = nullptr;
    double *d_scale64 = nullptr, *d_scale32 = nullptr, *d_rho = nullptr, *d_xu = nullptr, *d_given = nullptr;
    uint32_t *d_binom = nullptr, *d_layer_off = nullptr, *d_lo_qstart = nullptr, *d_prog_off = nullptr,
             *d_orig_bit = nullptr, *d_seg_desc = nullptr, *d_segoff = nullptr, *d_seg_prog = nullptr;
    ProgTerm* d_prog = nullptr;
    size_t prog_terms = 0;
    // dispatch measures (allocated on first use)
    double *d_G = nullptr, *d_q = nullptr, *d_lam_in = nullptr, *d_travel = nullptr, *d_tsum = nullptr;
    int32_t* d_pref_in = nullptr;
    bool dispatch_ready = false;
    double* d_coefs = nullptr;
    int stored_from = -1;  // first layer with stored coefficients (-1: none)
    uint16_t *d_lo_unrank = nullptr, *d_lo_rank = nullptr;
    TrieNode* d_nodes = nullptr;
    unsigned int* d_counters = nullptr;
    double* d_la = nullptr;      // look-ahead closed form: (w(l), z(l)) per state, interleaved (2 * 2^N)
    uint32_t* d_srec = nullptr;  // segment records of the default-shape sweep
    LowRow* d_lrow = nullptr;    // its low-pattern rows (FP64 offsets)
    LowRow* d_lrow32 = nullptr;  // and with FP32 offsets
    SweepParams P64{}, P32{};
    bool use_graphs = true;  // replay captured iterations (HQ_NO_GRAPH=1: launch eagerly)
    bool fuse = true;        // small layers form the previous layer's scalars (HQ_NO_FUSE=1: never)
    hipGraphExec_t iter_exec[2][2] = {};  // [FP32 storage][delta tracking]
    bool have_iterate = false;
    bool learned = false;      // product-form weights came from the network
    bool active_fp32 = false;  // storage of the current iterate
    int iterations_done = 0;

    ~hq_ctx() { release(); }
    void release() {
        void* ptrs[] = {x64,       x32,        d_nu,       d_tcoef,     d_scal,     d_part,
                        d_scale64, d_scale32,  d_rho,      d_xu,       d_given,     d_binom,    d_layer_off,
                        d_lo_qstart, d_prog_off, d_prog, d_orig_bit, d_lo_unrank, d_lo_rank, d_nodes,
                        d_counters, d_seg_desc, d_segoff,   d_coefs,     d_seg_prog, d_G,
                        d_q,       d_lam_in,   d_travel,   d_tsum,     d_pref_in,  d_srec,      d_lrow,     d_la,
                        d_lrow32};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
        x64 = nullptr;
        x32 = nullptr;
        for (auto& row : iter_exec)
            for (auto& e : row) {
                if (e) (void)hipGraphExecDestroy(e);
                e = nullptr;
            }
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        ev0 = ev1 = nullptr;
        if (own_stream && stream) (void)hipStreamDestroy(stream);
        stream = nullptr;
    }
    uint64_t states() const { return 1ull << N; }
    const SweepParams& params(bool fp32) const { return fp32 ? P32 : P64; }
    void* xbuf(bool fp32) const { return fp32 ? (void*)x32 : (void*)x64; }
};

namespace {

// ----------------------------------------------------------------------------
// preprocessing
// ----------------------------------------------------------------------------

hq_status validate(int N, int J, const double* lam, const double* mu, const int32_t* pref) {
    if (N < 1 || N > HQ_MAX_N) return fail(HQ_ERR_INVALID_ARG, "N must be in [1, " + std::to_string(HQ_MAX_N) + "]");
    if (J < 1) return fail(HQ_ERR_INVALID_ARG, "J must be >= 1");
    if (!lam || !mu || !pref) return fail(HQ_ERR_INVALID_ARG, "null input array");
    for (int j = 0; j < J; ++j)
        if (!std::isfinite(lam[j]) || lam[j] < 0.0)
            return fail(HQ_ERR_INVALID_ARG, "lambda_j must be finite and >= 0 (node " + std::to_string(j) + ")");
    for (int u = 0; u < N; ++u)
        if (!std::isfinite(mu[u]) || !(mu[u] > 0.0))
            return fail(HQ_ERR_INVALID_ARG, "mu_i must be finite and > 0 (unit " + std::to_string(u) + ")");
    std::vector<char> seen(N);
    for (int j = 0; j < J; ++j) {
        std::fill(seen.begin(), seen.end(), 0);
        for (int h = 0; h < N; ++h) {
            int32_t u = pref[(size_t)j * N + h];
            if (u < 0 || u >= N || seen[u])
                return fail(HQ_ERR_INVALID_ARG,
                            "preference row " + std::to_string(j) + " is not a permutation of 0..N-1");
            seen[u] = 1;
        }
    }
    return HQ_OK;
}

// Merged preference trie in preorder (node = shared prefix, rate = summed
// arrival rate of the nodes through it), over relabelled units.
std::vector<TrieNode> build_trie(int N, int J, const double* lam, const std::vector<int32_t>& rp) {
    std::vector<int> ids;
    for (int j = 0; j < J; ++j)
        if (lam[j] > 0.0) ids.push_back(j);
    std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) {
        return std::lexicographical_compare(rp.begin() + (size_t)a * N, rp.begin() + (size_t)(a + 1) * N,
                                            rp.begin() + (size_t)b * N, rp.begin() + (size_t)(b + 1) * N);
    });
    std::vector<TrieNode> nodes;
    std::vector<uint32_t> path(N, 0);
    std::vector<uint32_t> skip;
    int prev = -1;
    for (int a : ids) {
        const int32_t* row = rp.data() + (size_t)a * N;
        int cp = 0;
        if (prev >= 0) {
            const int32_t* pr = rp.data() + (size_t)prev * N;
            while (cp < N && pr[cp] == row[cp]) ++cp;
            for (int d = cp; d < N; ++d) skip[path[d]] = (uint32_t)nodes.size();
        }
        for (int d = cp; d < N; ++d) {
            TrieNode nd;
            nd.need = (d > 0 ? nodes[path[d - 1]].need : 0u) | (1u << row[d]);
            nd.skip_unit = (uint32_t)row[d];
            nd.rate = 0.0;
            path[d] = (uint32_t)nodes.size();
            nodes.push_back(nd);
            skip.push_back(0);
        }
        for (int d = 0; d < N; ++d) nodes[path[d]].rate += lam[a];
        prev = a;
    }
    if (prev >= 0)
        for (int d = 0; d < N; ++d) skip[path[d]] = (uint32_t)nodes.size();
    for (size_t i = 0; i < nodes.size(); ++i) nodes[i].skip_unit |= skip[i] << 5;
    return nodes;
}

void setup_params(hq_ctx* c) {
    SweepParams P{};
    P.N = c->N;
    P.b = c->b;
    P.H = c->H;
    P.buffer = c->opts.buffer;
    P.delta = c->opts.delta;
    P.Lam = c->Lam;
    P.sum_nu = 0.0;
    for (int u = 0; u < c->N; ++u) P.sum_nu += c->nu[u];
    P.nu = c->d_nu;
    P.binom = c->d_binom;
    P.layer_off = c->d_layer_off;
    P.lo_unrank = c->d_lo_unrank;
    P.lo_rank = c->d_lo_rank;
    P.lo_qstart = c->d_lo_qstart;
    P.tcoef = c->d_tcoef;
    P.seg_desc = c->d_seg_desc;
    P.seg_prog = reinterpret_cast<const uint2*>(c->d_seg_prog);
    P.segoff = c->d_segoff;
    P.prog_off = c->d_prog_off;
    P.prog = c->d_prog;
    P.nodes = c->d_nodes;
    P.coefs = c->d_coefs;
    const int L = c->N + 1;
    P.sc.lam = c->d_scal + 0 * L;
    P.sc.mu = c->d_scal + 1 * L;
    P.sc.alpha = c->d_scal + 2 * L;
    P.sc.pn = c->d_scal + 3 * L;
    P.sc.rnum = c->d_scal + 4 * L;
    P.sc.rden = c->d_scal + 5 * L;
    P.sc.delta = c->d_scal + 6 * L;
    P.sc.misc = c->d_scal + 7 * L;
    P.sc.wsum = c->d_scal + 8 * L + 8;
    P.sc.zsum = c->d_scal + 9 * L + 8;
    P.la = c->d_la;
    P.srec = c->d_srec;
    P.lrow = c->d_lrow;
    P.lrow32 = c->d_lrow32;
    P.partials = c->d_part;
    P.counters = c->d_counters;
    c->P64 = P;
    c->P32 = P;
    c->P64.scale = c->d_scale64;
    c->P64.inv_scale = c->d_scale64 + L;
    c->P32.scale = c->d_scale32;
    c->P32.inv_scale = c->d_scale32 + L;
}

hq_status create_impl(int N, int J, const double* lam, const double* mu, const int32_t* pref,
                      const hq_options* opts, hq_ctx** out) {
    hq_status st = validate(N, J, lam, mu, pref);
    if (st != HQ_OK) return st;
    hq_options o;
    hq_default_options(&o);
    if (opts) o = *opts;
    if (o.precision < HQ_FP64 || o.precision > HQ_FP32_POLISH64)
        return fail(HQ_ERR_INVALID_ARG, "unknown precision");
    if (o.inner != HQ_INNER_CLOSED && o.inner != HQ_INNER_ONE && o.inner != HQ_INNER_LITERAL)
        return fail(HQ_ERR_INVALID_ARG, "unknown inner mode");
    if (o.inner == HQ_INNER_LITERAL && !(o.delta > 0.0 && std::isfinite(o.delta)))
        return fail(HQ_ERR_INVALID_ARG, "HQ_INNER_LITERAL needs a finite delta > 0");
    if (o.init < HQ_INIT_UNIFORM || o.init > HQ_INIT_LEARNED) return fail(HQ_ERR_INVALID_ARG, "unknown init mode");
    if (o.init == HQ_INIT_LEARNED && !o.mlp) return fail(HQ_ERR_INVALID_ARG, "HQ_INIT_LEARNED needs opts.mlp");
    if (o.stop != HQ_STOP_RESIDUAL && o.stop != HQ_STOP_DELTA) return fail(HQ_ERR_INVALID_ARG, "unknown stop rule");
    if (o.init == HQ_INIT_PRODUCT && !o.init_rho) return fail(HQ_ERR_INVALID_ARG, "HQ_INIT_PRODUCT needs init_rho");
    if (o.init == HQ_INIT_STATE && !o.init_state) return fail(HQ_ERR_INVALID_ARG, "HQ_INIT_STATE needs init_state");
    if (o.buffer < HQ_BUFFER_UNLIMITED || o.buffer > HQ_BUFFER_MAX)
        return fail(HQ_ERR_INVALID_ARG, "buffer must be in [0, HQ_BUFFER_MAX] or HQ_BUFFER_UNLIMITED");
    if (o.buffer == HQ_BUFFER_UNLIMITED) {
        double L = 0.0, M = 0.0;
        for (int j = 0; j < J; ++j) L += lam[j];
        for (int u = 0; u < N; ++u) M += mu[u];
        if (!(L < M)) return fail(HQ_ERR_INVALID_ARG, "an unlimited waiting room needs sum lambda_j < sum mu_i");
    }
    if (o.tile_bits > 0 && (o.tile_bits < 1 || o.tile_bits > HQ_MAXB))
        return fail(HQ_ERR_INVALID_ARG, "tile_bits must be in [1, 12]");
    if (o.init == HQ_INIT_PRODUCT)
        for (int u = 0; u < N; ++u)
            if (!std::isfinite(o.init_rho[u]) || o.init_rho[u] < 0.0 || o.init_rho[u] > 1.0)
                return fail(HQ_ERR_INVALID_ARG, "init_rho values must be in [0, 1]");

    std::unique_ptr<hq_ctx> c(new (std::nothrow) hq_ctx());
    if (!c) return fail(HQ_ERR_OUT_OF_MEMORY, "host allocation failed");
    c->N = N;
    c->J = J;
    c->opts = o;
    double Lam = 0.0;
    for (int j = 0; j < J; ++j) Lam += lam[j];
    c->Lam = Lam;
    c->lam_zero = !(Lam > 0.0);
    int b = o.tile_bits > 0 ? o.tile_bits : 10;  // measured fastest from N = 16 to 30
    if (b > N) b = N;
    c->b = b;
    c->H = N - b;
    if (c->H > HQ_MAXH) return fail(HQ_ERR_INVALID_ARG, "tile_bits too small for this N");

    // relabel units (new label u <-> original unit orig[u])
    c->lam_in.assign(lam, lam + J);
    c->pref_in.assign(pref, pref + (size_t)J * N);
    c->orig = hqtables::relabel(N, J, lam, mu, pref);
    std::vector<int> newlab(N);
    for (int u = 0; u < N; ++u) newlab[c->orig[u]] = u;
    c->nu.resize(N);
    for (int u = 0; u < N; ++u) c->nu[u] = mu[c->orig[u]];
    std::vector<int32_t> rp((size_t)J * N);
    for (size_t i = 0; i < rp.size(); ++i) rp[i] = newlab[pref[i]];
    if (o.init == HQ_INIT_PRODUCT) {
        c->rho_init.resize(N);
        for (int u = 0; u < N; ++u) c->rho_init[u] = o.init_rho[c->orig[u]];
    }
    if (o.init == HQ_INIT_LEARNED) {
        // predicted utilisations seed the product form; the network runs on its own device
        std::vector<double> rho;
        hq_status ps = hq_mlp_predict_instance(o.mlp, N, J, lam, mu, pref, rho);
        if (ps != HQ_OK) return ps;
        c->rho_init.resize(N);
        for (int u = 0; u < N; ++u) c->rho_init[u] = rho[c->orig[u]];
        c->opts.init = HQ_INIT_PRODUCT;
        c->learned = true;
    }
    c->opts.mlp = nullptr;
    if (!c->rho_init.empty()) {
        c->x_init.resize(N);
        hqinit::calibrate(N, c->rho_init.data(), c->nu.data(), Lam, o.buffer, c->x_init.data());
    }
    if (o.init == HQ_INIT_STATE) c->state_init.assign(o.init_state, o.init_state + (1ull << N));
    c->opts.init_rho = nullptr;
    c->opts.init_state = nullptr;

    c->nodes = build_trie(N, J, lam, rp);
    std::vector<double> tcoef;
    std::vector<uint32_t> prog_off;
    std::vector<ProgTerm> prog;
    hqtables::build_programs(N, b, hqtables::build_terms(N, J, lam, rp), tcoef, prog_off, prog);
    c->prog_terms = prog.size();

    // layout tables (hq_layout.h)
    hqlayout::Layout lay;
    hqlayout::build_layout(N, b, lay);
    std::vector<uint32_t> tb(32 * 32, 0);
    for (int n = 0; n < 32; ++n)
        for (int k = 0; k <= n; ++k) tb[n * 32 + k] = (uint32_t)binom_d(n, k);
    const std::vector<uint32_t>& layer_off = lay.layer_off;
    const std::vector<uint16_t>& lo_unrank = lay.lo_unrank;
    const std::vector<uint16_t>& lo_rank = lay.lo_rank;
    const std::vector<uint32_t>& lo_qstart = lay.lo_qstart;
    const std::vector<uint32_t>& segoff = lay.segoff;
    const std::vector<uint32_t>& seg_desc = lay.seg_desc;
    // per segment: where its tile's program starts and how many terms it has
    std::vector<uint32_t> seg_prog(2 * seg_desc.size());
    for (size_t i = 0; i < seg_desc.size(); ++i) {
        const size_t T = seg_desc[i] >> 4;
        seg_prog[2 * i] = prog_off[T * (N + 1)];
        seg_prog[2 * i + 1] = prog_off[T * (N + 1) + N] - prog_off[T * (N + 1)];
    }
    // segment records and low-pattern rows of the default-shape sweep
    // (hq_sweep.hip); HQ_LEGACY_SWEEP=1 in the environment keeps every
    // layer on the general kernels instead
    std::vector<uint32_t> srec;
    std::vector<LowRow> lrow, lrow32;
    const char* legacy = std::getenv("HQ_LEGACY_SWEEP");
    const char* nograph = std::getenv("HQ_NO_GRAPH");
    const char* nola = std::getenv("HQ_NO_LOOKAHEAD");
    c->use_graphs = !(nograph && nograph[0] == '1');
    // HQ_NO_FUSE=1: a finalize launch after every layer (for comparisons)
    const char* nofuse = std::getenv("HQ_NO_FUSE");
    c->fuse = !(nofuse && nofuse[0] == '1');
    // the default-shape sweep kernels serve H = 6..16 (N = 16..26); from
    // H = 17 the general layer kernel measured faster (N = 27: 7.07 against
    // 7.59 ms per outer iteration, N = 30: 52.0 against 56.6 ms).  They
    // address the programs with 32-bit byte offsets.
    if (b == HQ_SWEEP_B && c->H >= 6 && c->H <= 16 && prog.size() < (1ull << 27) && !(legacy && legacy[0] == '1')) {
        lrow = hqsweeptab::low_rows(lay, c->nu, 8);
        lrow32 = hqsweeptab::low_rows(lay, c->nu, 4);
        srec = hqsweeptab::seg_records(lay, prog_off, c->nu);
    }
    c->layers.resize(N + 1);
    size_t max_groups = 1;
    for (int n = 0; n <= N; ++n) {
        LayerArgs A{};
        A.n = n;
        A.desc_base = lay.desc_base[n];
        A.groups = lay.desc_base[n + 1] - lay.desc_base[n];
        A.count = (uint32_t)binom_d(N, n);
        max_groups = std::max(max_groups, (size_t)A.groups);
        c->layers[n] = A;
    }
    c->max_groups = max_groups;
    // Layers near the top (nearly all units busy) have the longest per-tile
    // programs; their coefficients can be computed once and stored
    // (unit-major, N doubles per state).  Auto: from layer N-1 down, every
    // layer whose tiles average at least HQ_STORE_TERMS program terms per
    // state, within HQ_STORE_BYTES of coefficients and a quarter of the
    // device's free memory.  Reading N stored values per state costs about
    // as much as evaluating ~30 program terms; below ~20 terms storing is
    // measurably slower.
    // program terms per state of each layer (tile program lengths weighted
    // by the tiles' states in the layer)
    std::vector<double> num(N + 1, 0.0), den(N + 1, 0.0);
    {
        const uint64_t ntiles = 1ull << (N - b);
        for (uint64_t T = 0; T < ntiles; ++T) {
            const double len = (double)(prog_off[T * (N + 1) + N] - prog_off[T * (N + 1)]);
            const int h = __builtin_popcountll(T);
            for (int q = 0; q <= b; ++q) {
                const double w = binom_d(b, q);
                num[h + q] += w * len;
                den[h + q] += w;
            }
        }
    }
    // the look-ahead closed form (one pass per layer) needs the default-shape
    // sweep, which accumulates its sums while it writes
    const bool lookahead = o.inner == HQ_INNER_CLOSED && !srec.empty() && !(nola && nola[0] == '1');
    int top = o.stored_layers;
    if (top == 0) {
        uint64_t budget = HQ_STORE_BYTES;
        size_t free_b = 0, total_b = 0;
        if ((o.device < 0 || hipSetDevice(o.device) == hipSuccess) && hipMemGetInfo(&free_b, &total_b) == hipSuccess)
            budget = std::min<uint64_t>(budget, free_b / 4);
        else
            (void)hipGetLastError();
        uint64_t bytes = 0;
        for (int n = N - 1; n >= 1; --n) {
            const uint64_t add = (uint64_t)N * (uint64_t)binom_d(N, n) * sizeof(double);
            if (num[n] < HQ_STORE_TERMS * den[n] || bytes + add > budget) break;
            bytes += add;
            ++top;
        }
    } else if (top < 0) {
        top = 0;
    }
    top = std::min(top, std::max(N - 1, 0));
    unsigned long long coef_total = 0;
    c->stored_from = top > 0 ? N - top : -1;
    for (int n = 1; n <= N - 1; ++n) {
        if (top > 0 && n >= N - top) {
            c->layers[n].stored = 1;
            c->layers[n].coef_base = coef_total;
            coef_total += (unsigned long long)N * c->layers[n].count;
        } else if (num[n] >= HQ_GENERAL_TERMS * den[n] && !lookahead) {
            // long programs: the general kernel, which forms each busy unit's
            // coefficient next to its neighbour value, measured faster there
            // (N = 26 clustered, layers 16..19: 252, 213, 163, 133 against
            // 259, 228, 174, 144 us).  The look-ahead closed form keeps the
            // sweep, whose look-ahead pairs arrive as one 16-byte load per
            // state (N = 26: 1.146 against 1.152 s to 1e-8).
            c->layers[n].general = 1;
        }
    }
    // storage scales: 1 for FP64; for FP32 the power of two nearest C(N, n)
    std::vector<double> s64(2 * (N + 1), 1.0), s32(2 * (N + 1));
    for (int n = 0; n <= N; ++n) {
        int e = (int)std::lround(std::log2(binom_d(N, n)));
        s32[n] = std::ldexp(1.0, e);
        s32[N + 1 + n] = std::ldexp(1.0, -e);
    }
    std::vector<uint32_t> orig_bit(N);
    for (int u = 0; u < N; ++u) orig_bit[u] = 1u << c->orig[u];

    try {
        if (o.device >= 0) HQ_HIP(hipSetDevice(o.device));
        HQ_HIP(hipGetDevice(&c->device));
        if (o.stream) {
            c->stream = (hipStream_t)o.stream;
        } else {
            HQ_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
        HQ_HIP(hipEventCreate(&c->ev0));
        HQ_HIP(hipEventCreate(&c->ev1));
        const uint64_t S = c->states();
        if (o.precision != HQ_FP32) c->x64 = dalloc<double>(S);
        if (o.precision != HQ_FP64) c->x32 = dalloc<float>(S);
        c->d_nu = dalloc<double>(N);
        c->d_tcoef = dalloc<double>(tcoef.size());
        c->d_scal = dalloc<double>(10 * (N + 1) + 8);
        // two halves of max_groups partials each (consecutive layer launches of an
        // outer iteration alternate between them; a launch writes at most one
        // partial per segment of its layer)
        c->d_part = dalloc<double>(max_groups * 32);
        c->d_scale64 = dalloc<double>(s64.size());
        c->d_scale32 = dalloc<double>(s32.size());
        c->d_rho = dalloc<double>(32);
        c->d_xu = dalloc<double>(N);
        c->d_binom = dalloc<uint32_t>(tb.size());
        c->d_layer_off = dalloc<uint32_t>(layer_off.size());
        c->d_lo_qstart = dalloc<uint32_t>(lo_qstart.size());
        c->d_prog_off = dalloc<uint32_t>(prog_off.size());
        c->d_prog = dalloc<ProgTerm>(std::max<size_t>(prog.size(), 1));
        c->d_seg_desc = dalloc<uint32_t>(seg_desc.size());
        c->d_seg_prog = dalloc<uint32_t>(seg_prog.size());
        c->d_segoff = dalloc<uint32_t>(segoff.size());
        c->d_coefs = dalloc<double>(coef_total);
        c->d_orig_bit = dalloc<uint32_t>(N);
        c->d_lo_unrank = dalloc<uint16_t>(lo_unrank.size());
        c->d_lo_rank = dalloc<uint16_t>(lo_rank.size());
        c->d_nodes = dalloc<TrieNode>(c->nodes.size());
        c->d_counters = dalloc<unsigned int>(N + 1);
        // the look-ahead closed form (one pass per layer) needs the default-shape
        // sweep, which accumulates its sums while it writes
        if (lookahead) c->d_la = dalloc<double>(2 * S);
        if (!srec.empty()) {
            c->d_srec = dalloc<uint32_t>(srec.size());
            c->d_lrow = dalloc<LowRow>(lrow.size());
            c->d_lrow32 = dalloc<LowRow>(lrow32.size());
        }
        hipStream_t s = c->stream;
        h2d(c->d_nu, c->nu, s);
        h2d(c->d_tcoef, tcoef, s);
        h2d(c->d_scale64, s64, s);
        h2d(c->d_scale32, s32, s);
        h2d(c->d_binom, tb, s);
        h2d(c->d_layer_off, layer_off, s);
        h2d(c->d_lo_qstart, lo_qstart, s);
        h2d(c->d_prog_off, prog_off, s);
        if (!prog.empty()) h2d(c->d_prog, prog, s);
        h2d(c->d_seg_desc, seg_desc, s);
        h2d(c->d_seg_prog, seg_prog, s);
        h2d(c->d_segoff, segoff, s);
        h2d(c->d_orig_bit, orig_bit, s);
        h2d(c->d_lo_unrank, lo_unrank, s);
        h2d(c->d_lo_rank, lo_rank, s);
        h2d(c->d_nodes, c->nodes, s);
        if (!srec.empty()) {
            h2d(c->d_srec, srec, s);
            h2d(c->d_lrow, lrow, s);
            h2d(c->d_lrow32, lrow32, s);
        }
        HQ_HIP(hipMemsetAsync(c->d_counters, 0, sizeof(unsigned int) * (N + 1), s));
        HQ_HIP(hipMemsetAsync(c->d_scal, 0, sizeof(double) * (10 * (N + 1) + 8), s));
        if (!c->state_init.empty()) {
            c->d_given = dalloc<double>(S);
            HQ_HIP(hipMemcpyAsync(c->d_given, c->state_init.data(), S * sizeof(double), hipMemcpyHostToDevice, s));
        }
        setup_params(c.get());
        if (c->d_la)
            for (int n = 0; n <= N; ++n)
                HQ_HIP(hqk::launch_lookahead(c->P64, c->layers[n], c->d_la, (uint32_t)c->nodes.size(), s));
        for (int n = 1; n <= N - 1; ++n)
            if (c->layers[n].stored)
                HQ_HIP(hqk::launch_coef(c->P64, c->layers[n], c->d_coefs, (uint32_t)c->nodes.size(), s));
        HQ_HIP(hipStreamSynchronize(s));
    } catch (const std::bad_alloc&) {
        return fail(HQ_ERR_OUT_OF_MEMORY, "device allocation failed");
    } catch (const HipError& e) {
        return fail(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    *out = c.release();
    return HQ_OK;
}

// ----------------------------------------------------------------------------
// iteration
// ----------------------------------------------------------------------------

// Host part of the initial iterate: the product-form weights calibrated at
// create time (uploaded) and the elementary symmetric polynomials e_n(x) in
// FP64.
// Returns the init mode of the kernels (0 uniform, 1 product, 2 given).
int prepare_init(hq_ctx* c, std::vector<double>& e) {
    const int N = c->N;
    e.assign(N + 1, 0.0);
    if (c->opts.init == HQ_INIT_PRODUCT) {
        const std::vector<double>& xu = c->x_init;
        hqinit::elementary(xu.data(), N, e.data());
        HQ_HIP(hipMemcpyAsync(c->d_xu, xu.data(), N * sizeof(double), hipMemcpyHostToDevice, c->stream));
        return 1;
    }
    return c->opts.init == HQ_INIT_STATE ? 2 : 0;
}

void run_init(hq_ctx* c, bool fp32) {
    std::vector<double> e;
    const int mode = prepare_init(c, e);
    for (int n = 0; n <= c->N; ++n) {
        LayerArgs A = c->layers[n];
        A.init_mode = mode;
        A.e_n = e[n];
        HQ_HIP(hqk::launch_init(fp32, c->params(fp32), A, c->xbuf(fp32), c->d_xu, c->d_given, c->d_orig_bit,
                                c->stream));
    }
    c->active_fp32 = fp32;
    c->have_iterate = true;
    c->iterations_done = 0;
}

// The launches of one outer iteration: for n = 1..N-1 in order, the layer
// kernel (and for the closed and literal inner forms its first pass) with
// the finalize launch that forms the layer's scalars.  With one update or
// the look-ahead closed form each layer launch forms the previous layer's
// scalars itself, and only the last layer has a finalize launch.
void launch_iteration(hq_ctx* c, bool track_delta) {
    const bool fp32 = c->active_fp32;
    const int inner = c->opts.inner;  // 0 closed, 1 one update, 2 literal loop
    if (inner == HQ_INNER_ONE || (inner == HQ_INNER_CLOSED && c->d_la)) {
        HQ_HIP(hqk::launch_write_chain(track_delta, fp32, c->params(fp32), c->layers.data(), c->N, c->xbuf(fp32),
                                       inner, c->d_part, c->d_part + c->max_groups * HQ_NPART, c->fuse, c->stream));
        return;
    }
    for (int n = 1; n <= c->N - 1; ++n) {
        const LayerArgs& A = c->layers[n];
        // the closed form's first pass is not needed when its sums come from
        // the look-ahead (alpha_n is then already on the device)
        if (inner == HQ_INNER_LITERAL || (inner == HQ_INNER_CLOSED && !c->d_la))
            HQ_HIP(hqk::launch_layer(M_PASS1, inner == HQ_INNER_LITERAL, fp32, c->params(fp32), A, c->xbuf(fp32),
                                     inner, c->stream));
        HQ_HIP(hqk::launch_layer(M_WRITE, track_delta, fp32, c->params(fp32), A, c->xbuf(fp32), inner, c->stream));
    }
}

// One outer iteration.  Its 2(N-1) (or 4(N-1)) launches depend only on
// device memory, so they are captured once per storage precision and
// stopping rule as a graph of kernel nodes and replayed.
void run_sweep(hq_ctx* c, bool track_delta) {
    if (c->use_graphs) {
        hipGraphExec_t& ex = c->iter_exec[c->active_fp32 ? 1 : 0][track_delta ? 1 : 0];
        if (!ex) {
            hipGraph_t g = nullptr;
            HQ_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            hipError_t le = hipSuccess;
            try {
                launch_iteration(c, track_delta);
            } catch (const HipError& e) {
                le = e.e;
            }
            const hipError_t ce = hipStreamEndCapture(c->stream, &g);
            HQ_HIP(le);
            HQ_HIP(ce);
            const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) ex = nullptr;
            HQ_HIP(ie);
        }
        HQ_HIP(hipGraphLaunch(ex, c->stream));
    } else {
        launch_iteration(c, track_delta);
    }
    c->iterations_done++;
}

// residual of the current iterate; also refreshes p(n) and the mass.
void run_residual(hq_ctx* c, double misc[3]) {
    const bool fp32 = c->active_fp32;
    HQ_HIP(hqk::launch_scalars(c->params(fp32), 0, c->stream));
    for (int n = 0; n <= c->N; ++n)
        HQ_HIP(hqk::launch_layer(M_RESID, false, fp32, c->params(fp32), c->layers[n], c->xbuf(fp32), 0, c->stream));
    HQ_HIP(hqk::launch_scalars(c->params(fp32), 1, c->stream));
    HQ_HIP(hipMemcpyAsync(misc, c->P64.sc.misc, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HQ_HIP(hipStreamSynchronize(c->stream));
}

void widen(hq_ctx* c) {
    std::vector<double> s32(2 * (c->N + 1));
    // inverse FP32 scales, recomputed on the host
    for (int n = 0; n <= c->N; ++n) {
        int e = (int)std::lround(std::log2(binom_d(c->N, n)));
        s32[n] = std::ldexp(1.0, -e);
    }
    uint32_t begin = 0;
    for (int n = 0; n <= c->N; ++n) {
        const uint32_t cnt = (uint32_t)binom_d(c->N, n);
        HQ_HIP(hqk::launch_widen(c->x32, c->x64, begin, cnt, s32[n], c->stream));
        begin += cnt;
    }
    c->active_fp32 = false;
}

double max_delta(hq_ctx* c) {
    std::vector<double> d(c->N + 1);
    HQ_HIP(hipMemcpyAsync(d.data(), c->P64.sc.delta, (c->N + 1) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HQ_HIP(hipStreamSynchronize(c->stream));
    double m = 0.0;
    for (int n = 1; n < c->N; ++n) m = std::max(m, d[n]);
    return m;
}

hq_status solve_impl(hq_ctx* c, double tol, hq_info* info) {
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(HQ_ERR_INVALID_ARG, "tol must be finite and > 0");
    hq_info inf{};
    auto t0 = std::chrono::steady_clock::now();
    if (c->lam_zero) {
        c->have_iterate = true;
        inf.status = HQ_OK;
        if (info) *info = inf;
        return HQ_OK;
    }
    const int max_iters = c->opts.max_iters > 0 ? c->opts.max_iters : 100000;
    const int fixed = c->opts.check_every;
    const bool delta_stop = c->opts.stop == HQ_STOP_DELTA;
    const int prec = c->opts.precision;
    hq_status status = HQ_ERR_NOT_CONVERGED;
    bool stalled64 = false;
    double sweep_ms = 0.0;
    try {
        run_init(c, prec != HQ_FP64);
        inf.warm_used = 0;
        if (c->opts.init == HQ_INIT_PRODUCT) {
            // cold start as fallback: keep the warm iterate only if its balance
            // residual is below the uniform start's
            double mw[3], mc[3];
            run_residual(c, mw);
            const int saved = c->opts.init;
            c->opts.init = HQ_INIT_UNIFORM;
            run_init(c, prec != HQ_FP64);
            run_residual(c, mc);
            c->opts.init = saved;
            inf.checks += 2;
            if (std::isfinite(mw[0]) && mw[0] < mc[0]) {
                run_init(c, prec != HQ_FP64);
                inf.warm_used = 1;
            }
        }
        // residual-check schedule and stall detection (hq_schedule.h)
        hqsched::Tracker tr = hqsched::start();
        int k = 0, next = fixed > 0 ? fixed : std::min(hqsched::kFirstCheck, max_iters);
        double last_res = -1.0;
        int stall32 = 0, fp64_from = prec == HQ_FP64 ? 0 : -1;
        double misc[3] = {0, 0, 0};
        while (k < max_iters) {
            HQ_HIP(hipEventRecord(c->ev0, c->stream));
            const int todo = delta_stop ? 1 : std::max(1, std::min(next, max_iters) - k);
            for (int i = 0; i < todo; ++i) run_sweep(c, delta_stop);
            HQ_HIP(hipEventRecord(c->ev1, c->stream));
            k += todo;
            if (delta_stop) {
                HQ_HIP(hipEventSynchronize(c->ev1));
                float ms = 0.f;
                HQ_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
                sweep_ms += ms;
                const double d = max_delta(c);
                if (d <= tol || k >= max_iters) {
                    run_residual(c, misc);
                    inf.checks++;
                    last_res = misc[0];
                    if (misc[2] != 0.0) status = HQ_ERR_NUMERIC;
                    else status = (d <= tol) ? HQ_OK : HQ_ERR_NOT_CONVERGED;
                    break;
                }
                continue;
            }
            run_residual(c, misc);
            float ms = 0.f;
            HQ_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
            sweep_ms += ms;
            inf.checks++;
            const double res = misc[0];
            if (misc[2] != 0.0 || !std::isfinite(res)) {
                status = HQ_ERR_NUMERIC;
                last_res = res;
                break;
            }
            const double prev_res = tr.prev_res;
            last_res = res;
            if (res <= tol) {
                status = HQ_OK;
                break;
            }
            // FP32 storage floor: hand over to FP64 (polish form) or stop
            if (c->active_fp32) {
                const bool stalled = prev_res > 0.0 && res > 0.8 * prev_res;
                if (res <= 1e-6 || stalled) {
                    if (prec == HQ_FP32_POLISH64) {
                        widen(c);
                        fp64_from = k;
                        tr = hqsched::start();
                        tr.prev_k = k;
                        next = k + (fixed > 0 ? fixed : 4);
                        continue;
                    }
                    if (stalled && ++stall32 >= 3) {
                        status = HQ_ERR_NOT_CONVERGED;
                        break;
                    }
                }
            }
            // schedule the next check (extrapolated decay); an FP64 iterate
            // whose residual has stopped falling ends the solve
            next = hqsched::next_check(tr, k, res, tol, fixed);
            if (hqsched::record(tr, k, res) && !c->active_fp32) {
                status = HQ_ERR_NOT_CONVERGED;
                stalled64 = true;
                break;
            }
        }
        inf.iterations = k;
        inf.fp64_iterations = fp64_from >= 0 ? k - fp64_from : 0;
        inf.residual = last_res;
        HQ_HIP(hqk::launch_scalars(c->params(c->active_fp32), 0, c->stream));
        std::vector<double> scal(8 * (c->N + 1) + 8);
        HQ_HIP(hipMemcpyAsync(scal.data(), c->d_scal, scal.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HQ_HIP(hipStreamSynchronize(c->stream));
        const int L = c->N + 1;
        inf.mass_error = scal[7 * L + 1] - 1.0;
        double drift = 0.0;
        for (int n = 0; n < c->N; ++n) drift = std::max(drift, std::fabs(scal[n] / c->Lam - 1.0));
        inf.max_layer_drift = drift;
    } catch (const HipError& e) {
        return fail(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    auto t1 = std::chrono::steady_clock::now();
    inf.seconds = std::chrono::duration<double>(t1 - t0).count();
    inf.sweep_seconds = sweep_ms * 1e-3;
    inf.state_updates_per_s = inf.sweep_seconds > 0 ? (double)(c->states() - 2) * inf.iterations / inf.sweep_seconds : 0.0;
    inf.status = status;
    if (info) *info = inf;
    if (status == HQ_ERR_NOT_CONVERGED)
        g_err = stalled64 ? "the residual stopped decreasing before tol (rounding floor or divergence)"
                          : "max_iters reached (or FP32 floor) before tol";
    if (status == HQ_ERR_NUMERIC) g_err = "non-finite value or zero denominator in a layer reduction";
    return status;
}

// ----------------------------------------------------------------------------
// batched solve
// ----------------------------------------------------------------------------

// Device buffers and captured graphs of the batch launch, per device.
struct BatchRes {
    BatchItem* items = nullptr;
    BatchOut* outs = nullptr;
    unsigned int* next = nullptr;
    BatchEntry* entries = nullptr;      // work queue, up to HQ_GROUP_MAX entries per instance
    unsigned int* group_counts = nullptr;  // one barrier counter per instance
    double* group_parts = nullptr;      // [cap][2][HQ_GROUP_MAX][3]
    int cap = 0;
    hipStream_t stream = nullptr;
    struct Graph {
        bool fp32;
        int block, count, items, grid;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
};
std::mutex g_batch_mu;
std::map<int, BatchRes> g_batch;
std::map<std::string, int> g_batch_tuned;  // batch signature -> work-group size
std::atomic<int> g_batch_last_block{0};    // work-group size of the last batched solve

BatchRes& batch_res(int device, int count) {
    BatchRes& r = g_batch[device];
    if (!r.stream) HQ_HIP(hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking));
    if (r.cap < count) {
        for (auto& g : r.graphs) (void)hipGraphExecDestroy(g.exec);
        r.graphs.clear();
        if (r.items) (void)hipFree(r.items);
        if (r.outs) (void)hipFree(r.outs);
        if (r.entries) (void)hipFree(r.entries);
        if (r.group_counts) (void)hipFree(r.group_counts);
        if (r.group_parts) (void)hipFree(r.group_parts);
        if (!r.next) r.next = dalloc<unsigned int>(1);
        r.cap = std::max(count, 64);
        r.items = dalloc<BatchItem>(r.cap);
        r.outs = dalloc<BatchOut>(r.cap);
        r.entries = dalloc<BatchEntry>((size_t)r.cap * HQ_GROUP_MAX);
        r.group_counts = dalloc<unsigned int>(r.cap);
        r.group_parts = dalloc<double>((size_t)r.cap * 2 * HQ_GROUP_MAX * 3);
    }
    return r;
}

// One launch of the batch kernel (reset of the work counter and of the
// group barrier counters, then the persistent kernel) as a captured
// hipGraph, reused for equal shapes.  `count` is the number of queue entries.
void batch_launch(BatchRes& r, bool fp32, int block, int count, int n_items, int grid) {
    for (auto& g : r.graphs)
        if (g.fp32 == fp32 && g.block == block && g.count == count && g.items == n_items && g.grid == grid) {
            HQ_HIP(hipGraphLaunch(g.exec, r.stream));
            return;
        }
    hipGraph_t graph = nullptr;
    HQ_HIP(hipStreamBeginCapture(r.stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = hqk::launch_batch(fp32, block, r.items, r.entries, r.outs, count, r.next, r.group_counts,
                                      n_items, grid, r.stream);
    hipError_t ce = hipStreamEndCapture(r.stream, &graph);
    HQ_HIP(le);
    HQ_HIP(ce);
    hipGraphExec_t exec = nullptr;
    HQ_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    r.graphs.push_back({fp32, block, count, n_items, grid, exec});
    HQ_HIP(hipGraphLaunch(exec, r.stream));
}

int device_cus() {
    int cus = 256;
    hipDeviceProp_t prop;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        cus = prop.multiProcessorCount;
    return std::max(1, cus);
}

// One batched launch over contexts of one storage precision.  fixed ==
// nullptr: the device's batch resources (allocated and grown on demand), a
// work-group size autotuned per batch signature, and a captured graph.
// fixed != nullptr: the static scratch of the allocation-free entry point,
// no device allocation, no graph, no event; the work-group size is the
// tuned one if this batch signature was tuned before, else 256.
hq_status batch_group(const std::vector<hq_ctx*>& cs, const std::vector<int>& pos, bool fp32, double tol,
                      hq_info* infos, int device, BatchScratch* fixed) {
    const int count = (int)cs.size();
    std::vector<BatchItem> items(count);
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    // largest instances first: the work queue then balances the tail
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cs[a]->N > cs[b]->N; });
    for (int j = 0; j < count; ++j) {
        hq_ctx* c = cs[order[j]];
        std::vector<double> e;
        const int mode = prepare_init(c, e);
        BatchItem& it = items[j];
        std::memset(&it, 0, sizeof(it));
        it.P = c->params(fp32);
        for (int n = 0; n <= c->N; ++n) {
            it.layers[n] = c->layers[n];
            it.layers[n].init_mode = mode;
            it.layers[n].e_n = e[n];
        }
        it.x = c->xbuf(fp32);
        it.inner_one = c->opts.inner == HQ_INNER_ONE ? 1 : 0;
        it.max_iters = c->opts.max_iters > 0 ? c->opts.max_iters : 100000;
        it.check_every = c->opts.check_every;
        it.tol = tol;
        it.init_mode = mode;
        it.xu = c->d_xu;
        it.given = c->d_given;
        it.orig_bit = c->d_orig_bit;
    }
    std::lock_guard<std::mutex> lock(g_batch_mu);
    BatchRes* r = nullptr;
    BatchItem* d_items;
    BatchEntry* d_entries;
    BatchOut* d_outs;
    unsigned int *d_next, *d_counts;
    double* d_parts;
    hipStream_t stream;
    if (fixed) {
        d_items = fixed->items;
        d_entries = fixed->entries;
        d_outs = fixed->outs;
        d_next = fixed->next;
        d_counts = fixed->group_counts;
        d_parts = fixed->group_parts;
        stream = cs[0]->stream;
    } else {
        r = &batch_res(device, count);
        d_items = r->items;
        d_entries = r->entries;
        d_outs = r->outs;
        d_next = r->next;
        d_counts = r->group_counts;
        d_parts = r->group_parts;
        stream = r->stream;
    }
    const int cus = device_cus();
    // Work sharing (hq_batchplan.h): an instance gets k work-groups, so that
    // the largest instances do not leave the rest of the device idle.
    std::vector<BatchEntry> entries;
    {
        std::vector<double> sizes(count);
        for (int j = 0; j < count; ++j) {
            sizes[j] = std::ldexp(1.0, cs[order[j]]->N);
            items[j].group_count = d_counts + j;
            items[j].group_part = d_parts + (size_t)j * 2 * HQ_GROUP_MAX * 3;
        }
        for (const hqplan::Entry& e : hqplan::plan(sizes, cus, HQ_GROUP_MAX))
            entries.push_back(BatchEntry{e.item, e.rank, e.k, 0});
    }
    const int n_entries = (int)entries.size();
    if (fixed && n_entries > HQ_NOALLOC_MAX_BATCH * HQ_GROUP_MAX)
        return fail(HQ_ERR_INVALID_ARG, "batch work plan exceeds the static scratch");
    const int grid = std::max(1, std::min(n_entries, 2 * cus));
    HQ_HIP(hipMemcpyAsync(d_entries, entries.data(), sizeof(BatchEntry) * n_entries, hipMemcpyHostToDevice,
                          stream));
    // autotuner: time each work-group size on this batch (a few iterations)
    std::string sig = std::string(fp32 ? "f32" : "f64") + ":" + std::to_string(count);
    {
        std::vector<int> ns;
        for (auto* c : cs) ns.push_back(c->N);
        std::sort(ns.begin(), ns.end());
        for (int n : ns) sig += "," + std::to_string(n);
    }
    int block = 0;
    auto tuned = g_batch_tuned.find(sig);
    if (tuned != g_batch_tuned.end()) {
        block = tuned->second;
    } else if (fixed) {
        block = 256;
    } else {
        std::vector<BatchItem> probe = items;
        for (auto& it : probe) {
            it.max_iters = std::min(it.max_iters, 6);
            it.check_every = 6;
        }
        HQ_HIP(hipMemcpyAsync(d_items, probe.data(), sizeof(BatchItem) * count, hipMemcpyHostToDevice, stream));
        hipEvent_t e0, e1;
        HQ_HIP(hipEventCreate(&e0));
        HQ_HIP(hipEventCreate(&e1));
        float best = 1e30f;
        for (int bs : {256, 512, 1024}) {
            batch_launch(*r, fp32, bs, n_entries, count, grid);  // warm-up (graph build)
            HQ_HIP(hipEventRecord(e0, stream));
            batch_launch(*r, fp32, bs, n_entries, count, grid);
            HQ_HIP(hipEventRecord(e1, stream));
            HQ_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            HQ_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                block = bs;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        g_batch_tuned[sig] = block;
    }
    g_batch_last_block.store(block);
    auto t0 = std::chrono::steady_clock::now();
    HQ_HIP(hipMemcpyAsync(d_items, items.data(), sizeof(BatchItem) * count, hipMemcpyHostToDevice, stream));
    std::vector<BatchOut> outs(count);
    float kms = 0.f;
    if (fixed) {
        HQ_HIP(hqk::launch_batch(fp32, block, d_items, d_entries, d_outs, n_entries, d_next, d_counts, count, grid,
                                 stream));
        HQ_HIP(hipMemcpyAsync(outs.data(), d_outs, sizeof(BatchOut) * count, hipMemcpyDeviceToHost, stream));
        HQ_HIP(hipStreamSynchronize(stream));
    } else {
        hipEvent_t k0, k1;
        HQ_HIP(hipEventCreate(&k0));
        HQ_HIP(hipEventCreate(&k1));
        HQ_HIP(hipEventRecord(k0, stream));
        batch_launch(*r, fp32, block, n_entries, count, grid);
        HQ_HIP(hipEventRecord(k1, stream));
        HQ_HIP(hipMemcpyAsync(outs.data(), d_outs, sizeof(BatchOut) * count, hipMemcpyDeviceToHost, stream));
        HQ_HIP(hipStreamSynchronize(stream));
        HQ_HIP(hipEventElapsedTime(&kms, k0, k1));
        (void)hipEventDestroy(k0);
        (void)hipEventDestroy(k1);
    }
    const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (fixed) kms = (float)(wall * 1e3);  // no events in this form: the host clock around the launch
    hq_status worst = HQ_OK;
    for (int j = 0; j < count; ++j) {
        hq_ctx* c = cs[order[j]];
        c->have_iterate = true;
        c->active_fp32 = fp32;
        c->iterations_done = outs[j].iterations;
        const hq_status st = (hq_status)outs[j].status;
        if (st != HQ_OK && worst == HQ_OK) worst = st;
        if (infos) {
            hq_info& inf = infos[pos[order[j]]];
            std::memset(&inf, 0, sizeof(inf));
            inf.status = st;
            inf.iterations = outs[j].iterations;
            inf.checks = outs[j].checks;
            inf.residual = outs[j].residual;
            inf.seconds = wall;
            inf.sweep_seconds = kms * 1e-3;
            inf.state_updates_per_s =
                kms > 0.f ? (double)(c->states() - 2) * outs[j].iterations / (kms * 1e-3) : 0.0;
        }
    }
    return worst;
}

hq_status batch_impl(hq_ctx* const* ctxs, int count, double tol, hq_info* infos, bool noalloc) {
    if (count < 0 || (count > 0 && !ctxs)) return fail(HQ_ERR_INVALID_ARG, "bad batch arguments");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(HQ_ERR_INVALID_ARG, "tol must be finite and > 0");
    std::vector<hq_ctx*> g64, g32;
    std::vector<int> p64, p32;
    int device = -1;
    for (int i = 0; i < count; ++i) {
        hq_ctx* c = ctxs[i];
        if (!c) return fail(HQ_ERR_INVALID_ARG, "null context in batch");
        if (device < 0) device = c->device;
        if (c->device != device) return fail(HQ_ERR_INVALID_ARG, "batch contexts must share one device");
        if (c->opts.precision == HQ_FP32_POLISH64)
            return fail(HQ_ERR_INVALID_ARG, "batched solves take HQ_FP64 or HQ_FP32 contexts");
        if (c->opts.stop != HQ_STOP_RESIDUAL)
            return fail(HQ_ERR_INVALID_ARG, "batched solves use the residual stopping rule");
        if (c->opts.inner == HQ_INNER_LITERAL)
            return fail(HQ_ERR_INVALID_ARG, "batched solves take the closed or one-update inner form");
    }
    hq_status worst = HQ_OK;
    for (int i = 0; i < count; ++i) {
        hq_ctx* c = ctxs[i];
        if (c->lam_zero) {
            c->have_iterate = true;
            if (infos) {
                std::memset(&infos[i], 0, sizeof(hq_info));
                infos[i].status = HQ_OK;
            }
            continue;
        }
        HQ_HIP(hipStreamSynchronize(c->stream));
        if (c->opts.precision == HQ_FP32) {
            g32.push_back(c);
            p32.push_back(i);
        } else {
            g64.push_back(c);
            p64.push_back(i);
        }
    }
    if (device >= 0) HQ_HIP(hipSetDevice(device));
    BatchScratch* fixed = nullptr;
    if (noalloc && device >= 0) {
        // the per-device address of the static scratch (looked up once per device)
        HQ_HIP(hqk::noalloc_scratch(device, &fixed));
    }
    if (!g64.empty()) {
        hq_status s = batch_group(g64, p64, false, tol, infos, device, fixed);
        if (s != HQ_OK && worst == HQ_OK) worst = s;
    }
    if (!g32.empty()) {
        hq_status s = batch_group(g32, p32, true, tol, infos, device, fixed);
        if (s != HQ_OK && worst == HQ_OK) worst = s;
    }
    if (worst == HQ_ERR_NOT_CONVERGED) g_err = "some instances reached max_iters before tol";
    if (worst == HQ_ERR_NUMERIC) g_err = "non-finite value in a batched instance";
    return worst;
}

}  // namespace

// ----------------------------------------------------------------------------
// C ABI
// ----------------------------------------------------------------------------
extern "C" {

void hq_default_options(hq_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = HQ_FP64;
    o->inner = HQ_INNER_ONE;
    o->init = HQ_INIT_UNIFORM;
    o->stop = HQ_STOP_RESIDUAL;
    o->max_iters = 100000;
    o->check_every = 0;
    o->tile_bits = 0;
    o->device = -1;
}

const char* hq_last_error(void) { return g_err.c_str(); }

hq_status hq_create(int N, int J, const double* lambda_j, const double* mu_i, const int32_t* pref_lists,
                    const hq_options* opts, hq_ctx** out) {
    if (!out) return fail(HQ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    try {
        return create_impl(N, J, lambda_j, mu_i, pref_lists, opts, out);
    } catch (const std::bad_alloc&) {
        return fail(HQ_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (const std::length_error&) {
        return fail(HQ_ERR_OUT_OF_MEMORY, "per-tile dispatch programs exceed 2^32 terms");
    } catch (const HipError& e) {
        return fail(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    } catch (...) {
        return fail(HQ_ERR_DEVICE, "unexpected failure in hq_create");
    }
}

void hq_destroy(hq_ctx* ctx) { delete ctx; }

hq_status hq_solve(hq_ctx* ctx, double tol, hq_info* info) {
    if (!ctx) return fail(HQ_ERR_INVALID_ARG, "ctx is NULL");
    try {
        return solve_impl(ctx, tol, info);
    } catch (const std::bad_alloc&) {
        return fail(HQ_ERR_OUT_OF_MEMORY, "allocation failed");
    } catch (...) {
        return fail(HQ_ERR_DEVICE, "unexpected failure in hq_solve");
    }
}

hq_status hq_iterate(hq_ctx* ctx, int iters) {
    if (!ctx) return fail(HQ_ERR_INVALID_ARG, "ctx is NULL");
    if (iters < 0) return fail(HQ_ERR_INVALID_ARG, "iters must be >= 0");
    if (ctx->lam_zero) {
        ctx->have_iterate = true;
        return HQ_OK;
    }
    try {
        if (!ctx->have_iterate) run_init(ctx, ctx->opts.precision != HQ_FP64);
        for (int i = 0; i < iters; ++i) run_sweep(ctx, false);
        HQ_HIP(hipStreamSynchronize(ctx->stream));
    } catch (const HipError& e) {
        return fail(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    return HQ_OK;
}

hq_status hq_reset(hq_ctx* ctx) {
    if (!ctx) return fail(HQ_ERR_INVALID_ARG, "ctx is NULL");
    if (ctx->lam_zero) return HQ_OK;
    try {
        run_init(ctx, ctx->opts.precision != HQ_FP64);
        HQ_HIP(hipStreamSynchronize(ctx->stream));
    } catch (const HipError& e) {
        return fail(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    return HQ_OK;
}

hq_status hq_residual(hq_ctx* ctx, double* residual) {
    if (!ctx || !residual) return fail(HQ_ERR_INVALID_ARG, "null argument");
    if (!ctx->have_iterate) return fail(HQ_ERR_STATE, "no iterate yet");
    if (ctx->lam_zero) {
        *residual = 0.0;
        return HQ_OK;
    }
    try {
        double misc[3];
        run_residual(ctx, misc);
        *residual = misc[0];
    } catch (const HipError& e) {
        return fail(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    return HQ_OK;
}

static hq_status export_impl(const hq_ctx* cc, double* dev_out, int conditional, hipStream_t s) {
    hq_ctx* c = const_cast<hq_ctx*>(cc);
    const bool fp32 = c->active_fp32;
    HQ_HIP(hqk::launch_scalars(c->params(fp32), 0, s));
    for (int n = 0; n <= c->N; ++n)
        HQ_HIP(hqk::launch_export(fp32, c->params(fp32), c->layers[n], c->xbuf(fp32), dev_out, c->d_orig_bit,
                                  conditional, s));
    return HQ_OK;
}

static hq_status host_export(const hq_ctx* c, double* out, int conditional) {
    if (!c || !out) return fail(HQ_ERR_INVALID_ARG, "null argument");
    if (!c->have_iterate) return fail(HQ_ERR_STATE, "no solve has run");
    const uint64_t S = c->states();
    if (c->lam_zero) {
        std::fill(out, out + S, 0.0);
        out[0] = 1.0;
        return HQ_OK;
    }
    hq_ctx* cm = const_cast<hq_ctx*>(c);
    try {
        // the staging vector in bitmask order is the context's (the same
        // buffer as the dispatch transform's), allocated on first use and
        // kept until hq_destroy
        if (!cm->d_G) cm->d_G = dalloc<double>(S);
        export_impl(c, cm->d_G, conditional, c->stream);
        HQ_HIP(hipMemcpyAsync(out, cm->d_G, S * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HQ_HIP(hipStreamSynchronize(c->stream));
    } catch (const std::bad_alloc&) {
        return fail(HQ_ERR_OUT_OF_MEMORY, "device allocation failed");
    } catch (const HipError& e) {
        return fail(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    return HQ_OK;
}

hq_status hq_state(const hq_ctx* ctx, double* P) { return host_export(ctx, P, 0); }
hq_status hq_conditional(const hq_ctx* ctx, double* pcond) { return host_export(ctx, pcond, 1); }

hq_status hq_state_device(const hq_ctx* ctx, double* dev_P, void* stream) {
    if (!ctx || !dev_P) return fail(HQ_ERR_INVALID_ARG, "null argument");
    if (!ctx->have_iterate) return fail(HQ_ERR_STATE, "no solve has run");
    hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
    try {
        if (ctx->lam_zero) {
            HQ_HIP(hipMemsetAsync(dev_P, 0, ctx->states() * sizeof(double), s));
            const double one = 1.0;
            HQ_HIP(hipMemcpyAsync(dev_P, &one, sizeof(double), hipMemcpyHostToDevice, s));
            HQ_HIP(hipStreamSynchronize(s));
            return HQ_OK;
        }
        if (s != ctx->stream) HQ_HIP(hipStreamSynchronize(ctx->stream));
        export_impl(ctx, dev_P, 0, s);
        // on the library's own stream the caller cannot order after it: finish here
        if (!stream) HQ_HIP(hipStreamSynchronize(s));
    } catch (const HipError& e) {
        return fail(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    return HQ_OK;
}

hq_status hq_marginals(const hq_ctx* cc, double* rho_u, double* p_n) {
    if (!cc) return fail(HQ_ERR_INVALID_ARG, "ctx is NULL");
    if (!cc->have_iterate) return fail(HQ_ERR_STATE, "no solve has run");
    hq_ctx* c = const_cast<hq_ctx*>(cc);
    const int N = c->N;
    if (c->lam_zero) {
        if (rho_u) std::fill(rho_u, rho_u + N, 0.0);
        if (p_n) {
            std::fill(p_n, p_n + N + 1, 0.0);
            p_n[0] = 1.0;
        }
        return HQ_OK;
    }
    try {
        const bool fp32 = c->active_fp32;
        HQ_HIP(hqk::launch_scalars(c->params(fp32), 0, c->stream));
        HQ_HIP(hipMemsetAsync(c->d_rho, 0, 32 * sizeof(double), c->stream));
        for (int n = 0; n <= N; ++n)
            HQ_HIP(hqk::launch_marginal(fp32, c->params(fp32), c->layers[n], c->xbuf(fp32), c->d_part, c->d_rho,
                                        c->stream));
        std::vector<double> rho(32), scal(8 * (N + 1) + 8);
        HQ_HIP(hipMemcpyAsync(rho.data(), c->d_rho, 32 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HQ_HIP(hipMemcpyAsync(scal.data(), c->d_scal, scal.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HQ_HIP(hipStreamSynchronize(c->stream));
        const int L = N + 1;
        const double mass = scal[7 * L + 1];
        const double wait = scal[7 * L + 3] / mass;  // states with calls waiting: every unit busy
        if (rho_u)
            for (int u = 0; u < N; ++u) rho_u[c->orig[u]] = rho[u] + wait;
        if (p_n) {
            for (int n = 0; n <= N; ++n) {
                const double layer_sum = (n == N) ? 1.0 : scal[n] / c->Lam;
                p_n[n] = scal[3 * L + n] * layer_sum / mass;
            }
            p_n[N] += wait;
        }
    } catch (const HipError& e) {
        return fail(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    return HQ_OK;
}

hq_status hq_dispatch(const hq_ctx* cc, const double* travel, double* q, double* mean_travel) {
    if (!cc) return fail(HQ_ERR_INVALID_ARG, "ctx is NULL");
    if (mean_travel && !travel) return fail(HQ_ERR_INVALID_ARG, "mean_travel needs travel");
    if (!cc->have_iterate) return fail(HQ_ERR_STATE, "no solve has run");
    hq_ctx* c = const_cast<hq_ctx*>(cc);
    const int N = c->N, J = c->J;
    const size_t JN = (size_t)J * N;
    if (travel)
        for (size_t i = 0; i < JN; ++i)
            if (!std::isfinite(travel[i])) return fail(HQ_ERR_INVALID_ARG, "travel times must be finite");
    if (c->lam_zero) {
        // every unit idle: each call goes to its first choice (no call has a rate)
        std::vector<double> q0(JN, 0.0);
        for (int j = 0; j < J; ++j) q0[(size_t)j * N + c->pref_in[(size_t)j * N]] = 1.0;
        if (q) std::copy(q0.begin(), q0.end(), q);
        if (mean_travel) *mean_travel = 0.0;
        return HQ_OK;
    }
    try {
        if (!c->dispatch_ready) {
            if (!c->d_G) c->d_G = dalloc<double>(c->states());
            if (!c->d_q) c->d_q = dalloc<double>(JN);
            if (!c->d_lam_in) c->d_lam_in = dalloc<double>(J);
            if (!c->d_travel) c->d_travel = dalloc<double>(JN);
            if (!c->d_tsum) c->d_tsum = dalloc<double>(2);
            if (!c->d_pref_in) c->d_pref_in = dalloc<int32_t>(JN);
            h2d(c->d_lam_in, c->lam_in, c->stream);
            h2d(c->d_pref_in, c->pref_in, c->stream);
            c->dispatch_ready = true;
        }
        if (travel) HQ_HIP(hipMemcpyAsync(c->d_travel, travel, JN * sizeof(double), hipMemcpyHostToDevice, c->stream));
        export_impl(c, c->d_G, 0, c->stream);
        HQ_HIP(hqk::launch_dispatch(c->d_G, N, J, c->d_pref_in, c->d_q, c->d_lam_in, travel ? c->d_travel : nullptr,
                                    c->d_tsum, c->stream));
        double sums[2] = {0.0, 0.0};
        if (q) HQ_HIP(hipMemcpyAsync(q, c->d_q, JN * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        if (mean_travel) HQ_HIP(hipMemcpyAsync(sums, c->d_tsum, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HQ_HIP(hipStreamSynchronize(c->stream));
        if (mean_travel) *mean_travel = sums[1] > 0.0 ? sums[0] / sums[1] : 0.0;
    } catch (const std::bad_alloc&) {
        return fail(HQ_ERR_OUT_OF_MEMORY, "device allocation failed");
    } catch (const HipError& e) {
        return fail(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    return HQ_OK;
}

hq_status hq_queue(const hq_ctx* cc, double* summary, double* tail, int len) {
    if (!cc) return fail(HQ_ERR_INVALID_ARG, "ctx is NULL");
    if (tail && len < 0) return fail(HQ_ERR_INVALID_ARG, "len must be >= 0");
    if (!cc->have_iterate) return fail(HQ_ERR_STATE, "no solve has run");
    hq_ctx* c = const_cast<hq_ctx*>(cc);
    const int N = c->N, C = c->opts.buffer;
    double pfull = 0.0, wait = 0.0, wmean = 0.0;
    if (!c->lam_zero) {
        try {
            HQ_HIP(hqk::launch_scalars(c->params(c->active_fp32), 0, c->stream));
            std::vector<double> scal(8 * (N + 1) + 8);
            HQ_HIP(hipMemcpyAsync(scal.data(), c->d_scal, scal.size() * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
            HQ_HIP(hipStreamSynchronize(c->stream));
            const int L = N + 1;
            const double mass = scal[7 * L + 1];
            pfull = scal[3 * L + N] / mass;  // p(N): the full layer has the single state
            wait = scal[7 * L + 3] / mass;
            wmean = scal[7 * L + 4] / mass;
        } catch (const HipError& e) {
            return fail(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
        }
    }
    const double rho = c->Lam / c->P64.sum_nu;
    if (summary) {
        summary[0] = pfull + wait;
        summary[1] = wait;
        summary[2] = wmean;
        summary[3] = C == 0 ? pfull : (C > 0 ? pfull * std::pow(rho, C) : 0.0);
    }
    if (tail) {
        double r = pfull;
        for (int k = 0; k < len; ++k) {
            r *= rho;
            tail[k] = (C < 0 || k < C) ? r : 0.0;
        }
    }
    return HQ_OK;
}

hq_status hq_layer_scalars(const hq_ctx* cc, double* out) {
    if (!cc || !out) return fail(HQ_ERR_INVALID_ARG, "null argument");
    if (!cc->have_iterate) return fail(HQ_ERR_STATE, "no iterate yet");
    hq_ctx* c = const_cast<hq_ctx*>(cc);
    const int N = c->N, L = N + 1;
    if (c->lam_zero) {
        std::fill(out, out + 4 * L, 0.0);
        out[2] = 1.0;
        return HQ_OK;
    }
    try {
        HQ_HIP(hqk::launch_scalars(c->params(c->active_fp32), 0, c->stream));
        std::vector<double> scal(8 * L + 8);
        HQ_HIP(hipMemcpyAsync(scal.data(), c->d_scal, scal.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HQ_HIP(hipStreamSynchronize(c->stream));
        for (int n = 0; n <= N; ++n) {
            out[4 * n + 0] = scal[0 * L + n];
            out[4 * n + 1] = scal[1 * L + n];
            out[4 * n + 2] = scal[3 * L + n];
            out[4 * n + 3] = scal[2 * L + n];
        }
    } catch (const HipError& e) {
        return fail(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    return HQ_OK;
}

int hq_num_units(const hq_ctx* ctx) { return ctx ? ctx->N : 0; }

hq_status hq_solve_batch(hq_ctx* const* ctxs, int count, double tol, hq_info* infos) {
    try {
        return batch_impl(ctxs, count, tol, infos, false);
    } catch (const std::bad_alloc&) {
        return fail(HQ_ERR_OUT_OF_MEMORY, "allocation failed in hq_solve_batch");
    } catch (const HipError& e) {
        return fail(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
}

int hq_batch_last_block(void) { return g_batch_last_block.load(); }

hq_status hq_solve_batch_noalloc(hq_ctx* const* ctxs, int count, double tol, hq_info* infos) {
    if (count > HQ_NOALLOC_MAX_BATCH)
        return fail(HQ_ERR_INVALID_ARG, "hq_solve_batch_noalloc takes at most " +
                                            std::to_string(HQ_NOALLOC_MAX_BATCH) + " contexts");
    try {
        return batch_impl(ctxs, count, tol, infos, true);
    } catch (const std::bad_alloc&) {
        return fail(HQ_ERR_OUT_OF_MEMORY, "host allocation failed in hq_solve_batch_noalloc");
    } catch (const HipError& e) {
        return fail(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
}

}  // extern "C"
