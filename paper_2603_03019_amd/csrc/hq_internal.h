// Internal definitions shared by the HIP translation units of libhq.
// Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define HQ_MAXB 12          // largest low-bit tile width b
#define HQ_MAXH 26          // largest high-bit count H = N - b
#define HQ_WG 256           // threads per work-group of the layer kernels
#define HQ_NPART 3          // partial sums per work-group

// One node of the merged preference trie, in preorder.  A node stands for
// a preference prefix shared by one or more demand nodes; `rate` is the
// summed arrival rate of those demand nodes.  `need` is the set of units on
// the path from the root to this node inclusive: a state m credits `rate`
// to the node's unit iff need is a subset of m (every unit up to and
// including this one is busy).  Descendants of a node live in
// [index + 1, skip).
struct TrieNode {
    uint32_t need;
    uint32_t skip_unit;  // (skip << 5) | unit
    double rate;
};

// Layer-scalar block kept on the device, indexed by layer n = 0..N.
// lam[n], mu[n]: lambda(n), mu(n) of (13)-(14) for the current iterate;
// alpha[n]: mu(n)/lambda(n-1) factor used in the last update of layer n;
// pn[n]: birth-death marginal p(n) of (10); rnum/rden: residual partial
// sums per layer; delta[n]: max |p^k - p^(k-1)| of the last sweep.
struct DevScalars {
    double* lam;
    double* mu;
    double* alpha;
    double* pn;
    double* rnum;
    double* rden;
    double* delta;
    double* misc;  // [0] residual, [1] total mass, [2] error flag (non-finite seen)
};

// Everything a layer kernel needs about the instance and the layout.
struct SweepParams {
    int N, b, H;
    double Lam;                  // total arrival rate
    const double* nu;            // [N] service rates (relabelled units)
    const uint32_t* binom;       // [32*32] C(n, k) at n*32 + k
    const uint32_t* layer_off;   // [N+2] first index of layer n in the state vector
    const uint16_t* lo_unrank;   // [2^b] low patterns ordered by (popcount, value)
    const uint16_t* lo_rank;     // [2^b] rank of a low pattern inside its popcount class
    const uint32_t* lo_qstart;   // [b+2] start of popcount class q in lo_unrank
    const double* mu_lo;         // [2^b] service-rate sum of a low pattern
    const double* tcoef;         // [2^H * N] per-tile dispatch coefficients
    const uint32_t* root_off;    // [2^H + 1] per-tile list of per-lane trie roots
    const uint32_t* root_list;
    const TrieNode* nodes;
    const double* scale;         // [N+1] storage scale of each layer (x = scale * p)
    const double* inv_scale;     // [N+1]
    DevScalars sc;
    double* partials;            // [max_groups * HQ_NPART]
    unsigned int* counters;      // [N+1]
};

// Segments of one layer: popcount class q of the low bits and the rank of
// the high-bit tile among tiles with n - q set bits.
struct LayerArgs {
    int n;
    int qlo, qhi;
    uint32_t seg_start[HQ_MAXB + 2];  // prefix over q = qlo..qhi of C(H, n - q)
    uint32_t groups;                  // total work-groups
    double beta;                      // unused placeholder (computed on device)
    double e_n;                       // product-form normaliser for init
    int init_mode;
};
