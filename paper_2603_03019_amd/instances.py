"""Seeded synthetic deployments of the spatial hypercube loss model.

This module only draws inputs: unit and demand-node positions, demand weights,
service rates and the distance-sorted preference lists that the model of
Section 2.1 takes (N units, J demand nodes with arrival rates, one preference
list per node, one service rate per unit).  It holds none of the solver's
arithmetic, so both the CPU oracle and the GPU library can consume the same
instances without sharing any solver code.

Every instance is a pure function of (config id, instance index):
``numpy.random.Generator(PCG64(SeedSequence([config, index])))`` with a fixed
draw order:

1. (batched / training configs only) the unit count N;
2. unit positions, uniform in the unit square, shape (N, 2);
3. demand-node positions: uniform in the unit square, or (clustered
   configurations) 4 cluster centres uniform in the unit square, a uniform
   cluster label per node, and an isotropic normal offset of std ``sigma``;
4. demand weights w ~ Dirichlet(1, ..., 1);
5. service rates nu_u ~ U[lo, hi) (skipped for the homogeneous variant,
   where nu_u = 1);
6. (training / warm-start configs only) the load Lambda / sum(nu) ~ U[0.5, 0.9).

Derived: Lambda = load * sum(nu); lambda_j = Lambda * w_j; pref[j] = stable
argsort of the squared Euclidean distances from node j to every unit, so ties
go to the lower unit index.
"""
from __future__ import annotations

import dataclasses
import struct
from typing import Optional

import numpy as np

__all__ = [
    "Instance",
    "make_instance",
    "config_instance",
    "CONFIGS",
    "write_instance",
    "read_instance",
]


@dataclasses.dataclass
class Instance:
    """One deployment: everything the solver needs plus the geometry."""

    N: int
    J: int
    lam: np.ndarray  # float64 [J], per-node arrival rate lambda_j = Lambda f_j
    nu: np.ndarray  # float64 [N], per-unit service rate
    pref: np.ndarray  # int32 [J, N], row j = units, most preferred first
    unit_xy: np.ndarray  # float64 [N, 2]
    atom_xy: np.ndarray  # float64 [J, 2]
    load: float  # Lambda / sum(nu)
    config: int = 0
    index: int = 0

    @property
    def Lambda(self) -> float:
        return float(self.lam.sum())

    def copy(self) -> "Instance":
        return dataclasses.replace(
            self,
            lam=self.lam.copy(),
            nu=self.nu.copy(),
            pref=self.pref.copy(),
            unit_xy=self.unit_xy.copy(),
            atom_xy=self.atom_xy.copy(),
        )


def _rng(config: int, index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(config), int(index)])))


def make_instance(
    N: Optional[int],
    J: int,
    *,
    config: int,
    index: int,
    load: Optional[float],
    nu_range=(0.8, 1.2),
    homogeneous: bool = False,
    clusters: int = 0,
    sigma: float = 0.1,
    n_range=None,
    load_range=None,
) -> Instance:
    """Draw one instance in the fixed order described in the module docstring.

    Pass ``N=None`` with ``n_range=(lo, hi)`` to draw N ~ U{lo..hi} first, and
    ``load=None`` with ``load_range=(lo, hi)`` to draw the load last.
    """
    rng = _rng(config, index)
    if N is None:
        lo, hi = n_range
        N = int(rng.integers(lo, hi + 1))
    if N < 1:
        raise ValueError("N must be >= 1")
    unit_xy = rng.random((N, 2))
    if clusters > 0:
        centres = rng.random((clusters, 2))
        labels = rng.integers(0, clusters, size=J)
        atom_xy = centres[labels] + sigma * rng.standard_normal((J, 2))
    else:
        atom_xy = rng.random((J, 2))
    w = rng.dirichlet(np.ones(J))
    if homogeneous:
        nu = np.ones(N)
    else:
        nu = rng.uniform(nu_range[0], nu_range[1], size=N)
    if load is None:
        load = float(rng.uniform(load_range[0], load_range[1]))
    Lam = float(load) * float(nu.sum())
    lam = Lam * w
    d2 = ((atom_xy[:, None, :] - unit_xy[None, :, :]) ** 2).sum(axis=2)
    pref = np.argsort(d2, axis=1, kind="stable").astype(np.int32)
    return Instance(
        N=N,
        J=J,
        lam=np.ascontiguousarray(lam, dtype=np.float64),
        nu=np.ascontiguousarray(nu, dtype=np.float64),
        pref=np.ascontiguousarray(pref, dtype=np.int32),
        unit_xy=unit_xy,
        atom_xy=atom_xy,
        load=float(load),
        config=int(config),
        index=int(index),
    )


# The five workload families.  Each entry maps to make_instance keyword
# arguments; "variants" select the load (config 2) or the homogeneous case.
CONFIGS = {
    # small plain FP64 system: N=10, J=40, uniform geometry, load 0.5
    1: dict(N=10, J=40, load=0.5, nu_range=(0.8, 1.2)),
    # N=20, J=200, loads {0.3, 0.6, 0.9} and a homogeneous (nu=1) variant
    2: dict(N=20, J=200, load=0.6, nu_range=(0.8, 1.2)),
    # N=26, J=1000, 4 Gaussian demand clusters (sigma 0.1), load 0.7
    3: dict(N=26, J=1000, load=0.7, nu_range=(0.5, 1.5), clusters=4, sigma=0.1),
    # batch of candidate deployments: N ~ U{12..18}, J=100, load 0.6
    4: dict(N=None, n_range=(12, 18), J=100, load=0.6, nu_range=(0.8, 1.2)),
    # warm-start training pool: N ~ U{16..20}, J=500, load ~ U[0.5, 0.9)
    5: dict(N=None, n_range=(16, 20), J=500, load=None, load_range=(0.5, 0.9), nu_range=(0.8, 1.2)),
    # warm-start evaluation pool: N=24, J=500, load ~ U[0.5, 0.9)
    6: dict(N=24, J=500, load=None, load_range=(0.5, 0.9), nu_range=(0.8, 1.2)),
}


def config_instance(config: int, index: int, **overrides) -> Instance:
    """Instance ``index`` of workload family ``config`` (keys of CONFIGS).

    ``overrides`` replace any keyword of the family (e.g. ``load=0.9``,
    ``homogeneous=True`` or a smaller ``N`` for a scaled-down case).
    """
    kw = dict(CONFIGS[config])
    kw.update(overrides)
    return make_instance(config=config, index=index, **kw)


_MAGIC = b"HQI1"


def write_instance(path: str, inst: Instance) -> None:
    """Little-endian file: magic, N, J, config, index (int32), load (f64),
    lambda f64[J], nu f64[N], pref i32[J*N], unit_xy f64[N*2], atom_xy f64[J*2]."""
    with open(path, "wb") as f:
        f.write(_MAGIC)
        f.write(struct.pack("<iiiid", inst.N, inst.J, inst.config, inst.index, inst.load))
        f.write(inst.lam.astype("<f8").tobytes())
        f.write(inst.nu.astype("<f8").tobytes())
        f.write(inst.pref.astype("<i4").tobytes())
        f.write(inst.unit_xy.astype("<f8").tobytes())
        f.write(inst.atom_xy.astype("<f8").tobytes())


def read_instance(path: str) -> Instance:
    with open(path, "rb") as f:
        if f.read(4) != _MAGIC:
            raise ValueError(f"{path}: not an instance file")
        N, J, config, index, load = struct.unpack("<iiiid", f.read(24))
        lam = np.frombuffer(f.read(8 * J), dtype="<f8").astype(np.float64)
        nu = np.frombuffer(f.read(8 * N), dtype="<f8").astype(np.float64)
        pref = np.frombuffer(f.read(4 * J * N), dtype="<i4").astype(np.int32).reshape(J, N)
        unit_xy = np.frombuffer(f.read(16 * N), dtype="<f8").reshape(N, 2).copy()
        atom_xy = np.frombuffer(f.read(16 * J), dtype="<f8").reshape(J, 2).copy()
    return Instance(N, J, lam, nu, pref, unit_xy, atom_xy, load, config, index)
