// CPU driver of the product-form start calibration (hq_init.h).
// Reads from stdin: N C Lam, then nu[N], then target[N]; writes the
// calibrated weights x[N] and the returned max |rho(x) - target| to stdout.
#include <cstdio>
#include <vector>

#include "hq_init.h"

int main() {
    int N = 0, C = 0;
    double Lam = 0.0;
    if (std::scanf("%d %d %lf", &N, &C, &Lam) != 3 || N < 1 || N > 30) return 2;
    std::vector<double> nu(N), t(N), x(N);
    for (int u = 0; u < N; ++u)
        if (std::scanf("%lf", &nu[u]) != 1) return 2;
    for (int u = 0; u < N; ++u)
        if (std::scanf("%lf", &t[u]) != 1) return 2;
    const double err = hqinit::calibrate(N, t.data(), nu.data(), Lam, C, x.data());
    for (int u = 0; u < N; ++u) std::printf("%.17g\n", x[u]);
    std::printf("%.17g\n", err);
    return 0;
}
