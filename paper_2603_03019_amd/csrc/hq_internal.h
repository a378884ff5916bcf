// Internal definitions shared by the HIP translation units of libhq.
// Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hq_sweeptab.h"  // LowRow, segment record layout
#include "hq_tables.h"    // ProgTerm

#define HQ_MAXB 12          // largest low-bit tile width b
#define HQ_MAXH 26          // largest high-bit count H = N - b
#define HQ_WG 256           // threads per work-group of the layer kernels
#define HQ_NPART 6          // partials per work-group of the layer kernels (sum, sum, max, max, sum, sum)
#ifndef HQ_HCHUNK
#define HQ_HCHUNK 8         // high-unit neighbour loads issued together by the run-time-shape sweep
#endif
#define HQ_GRID 2048        // persistent work-groups per layer launch (8 per CU)

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
    double* wsum;  // look-ahead closed form: sum_{C_n} p_n(l) w(l) of the last write of layer n
    double* zsum;  //   and sum_{C_n} p_n(l) z(l)
};

// Everything a layer kernel needs about the instance and the layout.
struct SweepParams {
    int N, b, H;
    int buffer;                  // waiting room: 0 none, C > 0, -1 unlimited (Proposition 2)
    double Lam;                  // total arrival rate
    double sum_nu;               // sum of the service rates (mu(n) for n > N)
    double delta;                // tolerance of the literal inner loop
    const double* nu;            // [N] service rates (relabelled units)
    const uint32_t* binom;       // [32*32] C(n, k) at n*32 + k
    const uint32_t* layer_off;   // [N+2] first index of layer n in the state vector
    const uint16_t* lo_unrank;   // [2^b] low patterns ordered by (popcount, value)
    const uint16_t* lo_rank;     // [2^b] rank of a low pattern inside its popcount class
    const uint32_t* lo_qstart;   // [b+2] start of popcount class q in lo_unrank
    const double* tcoef;         // [2^H * N] per-tile dispatch coefficients
    const uint32_t* seg_desc;    // per layer and work-group: (T << 4) | q
    const uint32_t* segoff;      // [(b+1) * 2^H] absolute start of segment (T, q)
    const uint32_t* prog_off;    // [2^H * (N+1)] per tile: first program term of unit u, and the end
    const ProgTerm* prog;        // per-tile dispatch programs, grouped by unit
    const uint2* seg_prog;       // per seg_desc entry: (first program term, term count) of its tile
    const TrieNode* nodes;
    const double* coefs;         // stored coefficients of the top layers (unit-major per layer)
    const double* la;            // look-ahead closed form: (w(l), z(l)) per state, interleaved
                                 // (layout order), or null
    const double* scale;         // [N+1] storage scale of each layer (x = scale * p)
    const double* inv_scale;     // [N+1]
    DevScalars sc;
    const uint32_t* srec;        // segment records (HQ_REC_WORDS each), seg_desc order; b = HQ_SWEEP_B only
    const LowRow* lrow;          // [2^b] low-pattern rows, FP64 offsets; b = HQ_SWEEP_B only
    const LowRow* lrow32;        // the same with FP32 offsets
    double* partials;            // [max_groups * 32]
    unsigned int* counters;      // [N+1]
};

// Per-layer launch arguments.
struct LayerArgs {
    int n;
    uint32_t groups;       // work-groups (segments) of the layer
    uint32_t desc_base;    // first entry of this layer in seg_desc
    uint32_t count;        // C(N, n)
    int stored;            // coefficients of this layer are stored in coefs
    int general;           // swept by the general layer kernel (long tile programs)
    unsigned long long coef_base;  // offset of this layer in coefs (unit-major, count per unit)
    double e_n;            // product-form normaliser for init
    int init_mode;
};

// Largest number of work-groups that share one instance of a batch.
#define HQ_GROUP_MAX 16

// One instance of a batched solve: everything the persistent batch kernel
// needs to run Algorithm 1 on it, in one work-group or in a group of them.
struct BatchItem {
    SweepParams P;
    LayerArgs layers[31];     // n = 0..N
    void* x;                  // state vector (FP64 or FP32, as the launch)
    int inner_one;
    int max_iters;
    int check_every;          // <= 0: adaptive
    double tol;
    int init_mode;            // 0 uniform, 1 product form, 2 given state
    const double* xu;         // product-form x_u (relabelled)
    const double* given;      // given state (original bitmask order)
    const uint32_t* orig_bit; // relabelled unit -> original bit
    unsigned int* group_count; // arrivals at the group's barriers (zeroed per launch)
    double* group_part;        // [2][HQ_GROUP_MAX][3] per-work-group partial sums, double-buffered
};

// One entry of the batch work queue: rank `rank` of the `k` work-groups
// that share instance `item` (k = 1: the instance runs in one work-group).
// The ranks of an instance are consecutive entries.
struct BatchEntry {
    int item, rank, k, pad;
};

// Per-instance results of a batched solve.
struct BatchOut {
    int iterations, checks, status, pad;
    double residual;
};

// Largest batch of the allocation-free batched solve, and the layout of its
// scratch: the work queue, per-instance descriptors and results, the work
// counter and the group barriers' counters and partial sums, all in one
// static device array per GPU (hq_kernels.hip).
#define HQ_NOALLOC_MAX_BATCH 256
#define HQ_MAX_DEVICES 64  // device ordinals the per-device scratch addresses are kept for
struct BatchScratch {
    BatchItem items[HQ_NOALLOC_MAX_BATCH];
    BatchEntry entries[HQ_NOALLOC_MAX_BATCH * HQ_GROUP_MAX];
    BatchOut outs[HQ_NOALLOC_MAX_BATCH];
    unsigned int group_counts[HQ_NOALLOC_MAX_BATCH];
    unsigned int next[64];
    double group_parts[HQ_NOALLOC_MAX_BATCH * 2 * HQ_GROUP_MAX * 3];
};

