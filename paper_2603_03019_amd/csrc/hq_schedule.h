// When to evaluate the balance residual of (1) during the outer iteration of
// Algorithm 1, and when a solve has stopped making progress.  Shared by the
// host loop of hq_solve and the batched kernel; plain C++ (no HIP types), so
// the CPU tests run it as it is.
//
// The residual of the iteration decays geometrically once the transient is
// over, so after two checks the next one is placed where the measured decay
// rate predicts the tolerance will be met (at most 64 iterations ahead).  A
// check that shows no decrease is followed by one 8 iterations later.
//
// A solve has stalled when several checks in a row fail to improve on the
// best residual seen so far by at least a factor 0.9999 per outer iteration
// since that best.  That happens at the rounding floor of the arithmetic (a
// tolerance below what FP64 can reach), where the residual only fluctuates,
// or when the iterate diverges; the caller then returns
// HQ_ERR_NOT_CONVERGED with the residual reached instead of running to
// max_iters.
#pragma once

#include <math.h>

#ifdef __HIPCC__
#define HQ_SD __host__ __device__ __forceinline__
#else
#define HQ_SD inline
#endif

namespace hqsched {

constexpr int kMaxStep = 64;          // longest gap between two residual checks
constexpr int kRetryStep = 8;         // gap after a check that showed no decrease
constexpr int kFirstCheck = 8;        // first check of an adaptive schedule
constexpr double kProgress = 0.9999;  // least decrease per iteration that counts as progress
constexpr int kStallChecks = 6;       // checks in a row without progress that end a solve

struct Tracker {
    double prev_res;  // residual at the previous check (< 0: none yet)
    int prev_k;       // iteration of the previous check
    double best;      // best residual that counted as progress (< 0: none yet)
    int best_k;       // its iteration
    int stall;        // checks in a row without progress
};

HQ_SD Tracker start() { return Tracker{-1.0, 0, -1.0, 0, 0}; }

// Whether the check at iteration k (residual res) fell short of progress:
// not below the best residual so far by kProgress per iteration since it.
// A NaN residual counts as no progress.
HQ_SD bool no_progress(const Tracker& t, int k, double res) {
    if (!(t.best > 0.0)) return false;
    const int dk = k - t.best_k > 1 ? k - t.best_k : 1;
    return !(res <= t.best * pow(kProgress, (double)dk));
}

// Iteration of the next check after the one at iteration k.  fixed > 0: a
// fixed cadence; otherwise extrapolate the decay since the previous check.
HQ_SD int next_check(const Tracker& t, int k, double res, double tol, int fixed) {
    if (fixed > 0) return k + fixed;
    if (t.prev_res > 0.0 && res < t.prev_res && res > 0.0 && tol > 0.0) {
        const int dk = k - t.prev_k > 1 ? k - t.prev_k : 1;
        const double rate = pow(res / t.prev_res, 1.0 / (double)dk);
        double need = (double)kMaxStep;
        if (rate > 0.0 && rate < 1.0) {
            need = log(tol / res) / log(rate);
            if (!(need < (double)kMaxStep)) need = (double)kMaxStep;  // also catches NaN
            if (need < 1.0) need = 1.0;
        }
        return k + (int)ceil(need);
    }
    return k + kRetryStep;
}

// Record the check at iteration k; true once kStallChecks checks in a row
// have shown no progress.
HQ_SD bool record(Tracker& t, int k, double res) {
    if (no_progress(t, k, res)) {
        t.stall += 1;
    } else {
        t.stall = 0;
        t.best = res;
        t.best_k = k;
    }
    t.prev_res = res;
    t.prev_k = k;
    return t.stall >= kStallChecks;
}

}  // namespace hqsched
