// Host-side dispatch tables of the sweep (no HIP): unit relabelling, the
// merged dispatch terms of Algorithm 3 and the per-tile programs.  Shared by
// the library and by a CPU checker built with a plain C++ compiler.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <stdexcept>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

// One term of a tile's dispatch program: unit u (given by the group the
// term sits in) gains `rate` in every state of the tile whose low bits
// contain `mask` (the low units ranked before u by the demand nodes summed
// into the term).
struct ProgTerm {
    uint32_t mask;
    uint32_t pad;
    double rate;
};

namespace hqtables {

// Relabel units so that the low label bits (per-lane inside a tile) go to the
// units demand nodes reach last: weight of unit u = sum_j lambda_j r^h over
// the rank h of u in node j's list, r = offered load clipped to [0.3, 0.95].
inline std::vector<int> relabel(int N, int J, const double* lam, const double* mu, const int32_t* pref) {
    double L = 0.0, M = 0.0;
    for (int j = 0; j < J; ++j) L += lam[j];
    for (int u = 0; u < N; ++u) M += mu[u];
    const double r = std::min(0.95, std::max(0.3, L / M));
    std::vector<double> w(N, 0.0);
    for (int j = 0; j < J; ++j) {
        double f = lam[j];
        for (int h = 0; h < N; ++h) {
            w[pref[(size_t)j * N + h]] += f;
            f *= r;
        }
    }
    std::vector<int> order(N);
    for (int u = 0; u < N; ++u) order[u] = u;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return w[a] < w[b]; });
    return order;  // order[new label] = original unit
}

// Dispatch credits of Algorithm 3 as merged terms.  Node j credits
// lambda_j to its h-th unit iff that unit and every unit ranked before it
// are busy; with u in m already required by the up-sum of (12), the term
// is (cond = units ranked before u, u, lambda_j).  Terms with the same
// (cond, u) are summed.
struct Term {
    uint32_t cond;
    int unit;
    double rate;
};

inline std::vector<Term> build_terms(int N, int J, const double* lam, const std::vector<int32_t>& rp) {
    std::unordered_map<uint64_t, size_t> index;
    std::vector<Term> terms;
    for (int j = 0; j < J; ++j) {
        if (!(lam[j] > 0.0)) continue;
        uint32_t cond = 0;
        for (int h = 0; h < N; ++h) {
            const int u = rp[(size_t)j * N + h];
            const uint64_t key = ((uint64_t)u << 32) | cond;
            auto it = index.find(key);
            if (it == index.end()) {
                index.emplace(key, terms.size());
                terms.push_back(Term{cond, u, lam[j]});
            } else {
                terms[it->second].rate += lam[j];
            }
            cond |= 1u << u;
        }
    }
    // deterministic order: by unit, then condition
    std::sort(terms.begin(), terms.end(), [](const Term& a, const Term& b) {
        return a.unit != b.unit ? a.unit < b.unit : a.cond < b.cond;
    });
    return terms;
}

// Per-tile dispatch tables.  For tile T (high units busy iff their bit is
// set) a term applies to the tile's states iff its high condition bits lie
// in T.  Terms with no low condition bits are uniform over the tile and are
// summed into tcoef[T][u]; the others are merged by (low mask, unit) into
// the tile's program, grouped by unit: prog_off[T * (N+1) + u] is the first
// term of unit u, prog_off[T * (N+1) + N] the end.  A high unit that is idle
// in T never needs its coefficient and gets no terms.
inline void build_programs(int N, int b, const std::vector<Term>& terms, std::vector<double>& tcoef,
                    std::vector<uint32_t>& prog_off, std::vector<ProgTerm>& prog) {
    const int H = N - b;
    const uint32_t tiles = 1u << H;
    const uint32_t lomask = (1u << b) - 1u;
    tcoef.assign((size_t)tiles * N, 0.0);
    prog_off.assign((size_t)tiles * (N + 1), 0);
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (tiles < 64) nth = 1;
    std::vector<std::vector<ProgTerm>> part(nth);
    std::vector<std::vector<uint32_t>> counts(nth);  // per tile and unit, within the part
    auto work = [&](unsigned w) {
        const uint32_t t0 = (uint32_t)((uint64_t)tiles * w / nth), t1 = (uint32_t)((uint64_t)tiles * (w + 1) / nth);
        std::vector<ProgTerm>& out = part[w];
        std::vector<uint32_t>& cnt = counts[w];
        cnt.assign((size_t)(t1 - t0) * N, 0);
        std::vector<std::pair<uint32_t, double>> cur;  // (low mask, rate) of one unit
        for (uint32_t T = t0; T < t1; ++T) {
            double* tc = tcoef.data() + (size_t)T * N;
            size_t i = 0;
            while (i < terms.size()) {
                const int u = terms[i].unit;
                size_t e = i;
                while (e < terms.size() && terms[e].unit == u) ++e;
                const bool needed = u < b || ((T >> (u - b)) & 1u);
                cur.clear();
                for (size_t k = i; k < e && needed; ++k) {
                    const uint32_t hi = terms[k].cond >> b, lo = terms[k].cond & lomask;
                    if (hi & ~T) continue;
                    if (lo == 0) {
                        tc[u] += terms[k].rate;
                    } else {
                        cur.emplace_back(lo, terms[k].rate);
                    }
                }
                if (!cur.empty()) {
                    std::stable_sort(cur.begin(), cur.end(),
                                     [](const std::pair<uint32_t, double>& a, const std::pair<uint32_t, double>& b) {
                                         return a.first < b.first;
                                     });
                    uint32_t c = 0;
                    for (size_t k = 0; k < cur.size(); ++k) {
                        if (k > 0 && cur[k].first == cur[k - 1].first) {
                            out.back().rate += cur[k].second;
                        } else {
                            out.push_back(ProgTerm{cur[k].first, 0u, cur[k].second});
                            ++c;
                        }
                    }
                    cnt[(size_t)(T - t0) * N + u] = c;
                }
                i = e;
            }
        }
    };
    if (nth == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        for (unsigned w = 0; w < nth; ++w) th.emplace_back(work, w);
        for (auto& t : th) t.join();
    }
    size_t total = 0;
    for (auto& v : part) total += v.size();
    if (total + 3 >= 0xffffffffull) throw std::length_error("dispatch program too large");
    prog.clear();
    prog.reserve(total);
    uint32_t pos = 0;
    for (unsigned w = 0; w < nth; ++w) {
        const uint32_t t0 = (uint32_t)((uint64_t)tiles * w / nth), t1 = (uint32_t)((uint64_t)tiles * (w + 1) / nth);
        for (uint32_t T = t0; T < t1; ++T) {
            for (int u = 0; u < N; ++u) {
                prog_off[(size_t)T * (N + 1) + u] = pos;
                pos += counts[w][(size_t)(T - t0) * N + u];
            }
            prog_off[(size_t)T * (N + 1) + N] = pos;
        }
        prog.insert(prog.end(), part[w].begin(), part[w].end());
        std::vector<ProgTerm>().swap(part[w]);
    }
    // the sweep reads terms in batches of four; inert terms past the end
    // keep a batch that starts at the last term inside the array
    for (int k = 0; k < 3; ++k) prog.push_back(ProgTerm{0xffffffffu, 0u, 0.0});
}

}  // namespace hqtables
