// CPU driver of the residual-check schedule (csrc/hq_schedule.h): runs the
// outer loop of an FP64 solve against a model residual r(k) read from stdin
//     tol max_iters fixed r0 rate floor noise
// with r(k) = max(floor, r0 * rate^k) * (1 + noise * z_k), z_k uniform in
// [-1, 1) from a fixed linear congruential sequence, and prints
//     <outcome> <iterations> <checks>
// with outcome "ok" (res <= tol), "stalled" or "max_iters".
#include <cmath>
#include <cstdio>

#include "hq_schedule.h"

int main() {
    double tol, r0, rate, floor_, noise;
    int max_iters, fixed;
    if (std::scanf("%lf %d %d %lf %lf %lf %lf", &tol, &max_iters, &fixed, &r0, &rate, &floor_, &noise) != 7)
        return 2;
    unsigned long long lcg = 12345;
    hqsched::Tracker tr = hqsched::start();
    int k = 0, checks = 0;
    int next = fixed > 0 ? fixed : (hqsched::kFirstCheck < max_iters ? hqsched::kFirstCheck : max_iters);
    while (k < max_iters) {
        k = next < max_iters ? (next > k ? next : k + 1) : max_iters;
        lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
        const double z = (double)(lcg >> 11) / 9007199254740992.0 * 2.0 - 1.0;
        const double res = std::fmax(floor_, r0 * std::pow(rate, (double)k)) * (1.0 + noise * z);
        ++checks;
        if (res <= tol) {
            std::printf("ok %d %d\n", k, checks);
            return 0;
        }
        next = hqsched::next_check(tr, k, res, tol, fixed);
        if (hqsched::record(tr, k, res)) {
            std::printf("stalled %d %d\n", k, checks);
            return 0;
        }
    }
    std::printf("max_iters %d %d\n", k, checks);
    return 0;
}
