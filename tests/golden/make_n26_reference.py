"""Write the oracle's converged answer for the N = 26 benchmark deployment.

    python tests/golden/make_n26_reference.py [out.txt]

The full stationary distribution at 2^26 states (512 MiB) is too large to
keep, and the oracle needs about an hour for it on 8 host cores, so this
script runs the CPU oracle's Algorithm 1 once (FP64, balance residual of
(1) <= 1e-12) and keeps what a GPU test can compare against:

* the number-busy marginal p(n) of (10) and the per-unit busy
  probabilities rho_u (sums of P over the states where unit u is busy);
* P(m) at 4096 states drawn with probability P(m) (the states that carry
  the mass, so that the mean of |dP| / P over them estimates the L1
  distance) and at 4096 states drawn uniformly (where P is tiny and the
  relative error is hardest to keep).

It calls only the oracle and the seeded instance generator.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import cpu  # noqa: E402
from paper_2603_03019_amd.instances import config_instance  # noqa: E402

TOL = 1e-12
SAMPLES = 4096


def main(out_path: str) -> None:
    inst = config_instance(3, 0)  # N = 26, J = 1000 in 4 clusters, load 0.7
    N = inst.N
    t0 = time.time()
    r = cpu.solve(inst, tol=TOL, inner="one", check_every=10)
    wall = time.time() - t0
    if not r.converged:
        raise SystemExit(f"oracle did not reach {TOL}: residual {r.residual}")
    rho, pn = cpu.marginals(N, r.P)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([3, 0, 26])))
    w = r.P / r.P.sum()
    heavy = np.sort(rng.choice(1 << N, size=SAMPLES, replace=True, p=w))
    flat = np.sort(rng.integers(0, 1 << N, size=SAMPLES))
    with open(out_path, "w") as f:
        f.write("# Oracle answer for the N = 26 benchmark deployment (instance generator config 3,\n")
        f.write("# index 0: J = 1000 demand nodes in 4 clusters, load 0.7).  Algorithm 1 in FP64\n")
        f.write("# (one inner update per layer; the fixed point is the stationary law of\n")
        f.write("# (1)-(3)), stopped at a relative L1 balance residual of (1) <= 1e-12.\n")
        f.write(f"# iterations {r.iterations} residual {r.residual:.6e} mass_error {r.mass_error:.3e}\n")
        f.write(f"# coefficient seconds {r.coef_seconds:.1f} iteration seconds {r.iter_seconds:.1f} "
                f"threads {r.threads} wall {wall:.1f}\n")
        f.write("# rows: 'pn n p(n)' (eq. (10)), 'rho u rho_u', 'heavy m P(m)' (m drawn with\n")
        f.write("# probability P(m)), 'flat m P(m)' (m drawn uniformly).  Units as in the input.\n")
        f.write(f"N {N}\n")
        f.write(f"iterations {r.iterations}\n")
        f.write(f"residual {r.residual:.17e}\n")
        for n in range(N + 1):
            f.write(f"pn {n} {pn[n]:.17e}\n")
        for u in range(N):
            f.write(f"rho {u} {rho[u]:.17e}\n")
        for m in heavy:
            f.write(f"heavy {int(m)} {r.P[m]:.17e}\n")
        for m in flat:
            f.write(f"flat {int(m)} {r.P[m]:.17e}\n")
    print(f"wrote {out_path}: {r.iterations} iterations, residual {r.residual:.3e}, {wall:.0f} s", flush=True)


if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(here, "n26_oracle.txt"))
