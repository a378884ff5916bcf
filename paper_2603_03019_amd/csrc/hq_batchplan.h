// Work plan of a batched solve (no HIP; also built by a CPU checker).
//
// Instance j of the batch (in the order the queue serves them, largest
// first) gets k_j work-groups: about its share of all states times the
// number of compute units, at least 1 and at most `kmax`.  The plan lists
// one queue entry per (instance, rank), the ranks of an instance
// consecutive, so that a rank is only ever taken by a running work-group
// and only the instance at the head of the queue can be partly taken.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

namespace hqplan {

struct Entry {
    int item, rank, k;
};

// sizes[j] = number of states of instance j (2^N_j), in queue order.
inline std::vector<Entry> plan(const std::vector<double>& sizes, int cus, int kmax) {
    double total = 0.0;
    for (double w : sizes) total += w;
    const double share = total / std::max(1, cus);
    std::vector<Entry> out;
    for (int j = 0; j < (int)sizes.size(); ++j) {
        const double want = share > 0.0 ? std::round(sizes[j] / share) : 1.0;
        const int k = (int)std::min<double>(kmax, std::max(1.0, want));
        for (int r = 0; r < k; ++r) out.push_back(Entry{j, r, k});
    }
    return out;
}

}  // namespace hqplan
