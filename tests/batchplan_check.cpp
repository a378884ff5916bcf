// CPU driver of the batch work plan (hq_batchplan.h).
// Reads from stdin: count cus kmax, then count instance sizes (states);
// writes one line "item rank k" per queue entry.
#include <cstdio>
#include <vector>

#include "hq_batchplan.h"

int main() {
    int count = 0, cus = 0, kmax = 0;
    if (std::scanf("%d %d %d", &count, &cus, &kmax) != 3 || count < 0) return 2;
    std::vector<double> sizes(count);
    for (int j = 0; j < count; ++j)
        if (std::scanf("%lf", &sizes[j]) != 1) return 2;
    for (const hqplan::Entry& e : hqplan::plan(sizes, cus, kmax)) std::printf("%d %d %d\n", e.item, e.rank, e.k);
    return 0;
}
