"""Seeded synthetic NMPC instances (problem data only).

This module is shared by the CPU oracle and by the HIP path's tests and
benchmark. It builds the numbers that *define* a problem -- grid sizes, time
step, cost weights, the factors of the input operator, the initial state and
the reference -- and holds none of the solution method's arithmetic.

Problem class (Sec. 2 and Sec. 3 of the paper; readings listed in the design doc):
first-order nonlinear heat equation w_t = k(w) Lap(w) + B u on the unit
interval or square with zero Dirichlet values on the boundary, discretized by
central differences on ``nsy x nsx`` interior nodes (``dx = 1/(nsx+1)``,
``dy = 1/(nsy+1)``), conductivity ``k(w) = k0 (1 + k1 w)``, stage cost
``0.5 q |x - xref|^2 + 0.5 r |u|^2``, horizon ``N`` backward-Euler stages of
length ``h``.

The input operator is stored in Kronecker form: input ``m = b*lx + a``
(``0 <= a < lx``, ``0 <= b < ly``) acts on node ``(iy, ix)`` with weight
``gy[b, iy] * gx[a, ix]``. A Gaussian actuator lattice is exactly of this form
(the 2D Gaussian factors into x and y parts); 1D point sources use ``ly = 1``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

__all__ = [
    "Problem",
    "gaussian_factors",
    "point_source_factors",
    "make_problem",
    "make_instance",
    "make_batch",
    "ragged_specs",
    "CONFIG_NAMES",
]


@dataclasses.dataclass
class Problem:
    """All data that defines one discretized NMPC problem (shape + physics)."""

    dim: int            # 1 or 2
    nsx: int            # interior nodes along x
    nsy: int            # interior nodes along y (1 for dim == 1)
    N: int              # horizon stages
    lx: int             # input lattice size along x
    ly: int             # input lattice size along y (1 for dim == 1)
    gx: np.ndarray      # [lx, nsx] float64
    gy: np.ndarray      # [ly, nsy] float64
    h: float            # stage length
    k0: float = 0.5     # conductivity k(w) = k0 (1 + k1 w)
    k1: float = 0.5
    q: float = 1.0      # state weight (Q = q I)
    r: float = 0.01     # input weight (R = r I)
    gamma: float = 0.0  # regularization weight
    tau: float = 0.0    # barrier weight of the input box u_lo <= u <= u_hi (0: no box)
    u_lo: float = 0.0
    u_hi: float = 0.0
    name: str = ""

    @property
    def n(self) -> int:
        return self.nsx * self.nsy

    @property
    def m(self) -> int:
        return self.lx * self.ly

    @property
    def dx(self) -> float:
        return 1.0 / (self.nsx + 1)

    @property
    def dy(self) -> float:
        return 1.0 / (self.nsy + 1) if self.dim == 2 else 1.0

    def dense_B(self) -> np.ndarray:
        """Input matrix B [n, m] with B[iy*nsx+ix, b*lx+a] = gy[b,iy] gx[a,ix]."""
        return np.kron(self.gy.T, self.gx.T)

    def with_(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def gaussian_factors(ns: int, L: int, sigma: float) -> np.ndarray:
    """Factor g[a, i] = exp(-(p_i - c_a)^2 / (2 sigma^2)) of a Gaussian lattice.

    Nodes sit at ``p_i = (i+1)/(ns+1)``; lattice centres at ``c_a = (a+1/2)/L``.
    The product of an x factor and a y factor is the untruncated,
    unnormalized 2D Gaussian patch.
    """
    p = (np.arange(ns) + 1.0) / (ns + 1.0)
    c = (np.arange(L) + 0.5) / L
    return np.exp(-((p[None, :] - c[:, None]) ** 2) / (2.0 * sigma * sigma))


def point_source_factors(ns: int, nodes_1based: List[int]) -> np.ndarray:
    """Unit point sources: g[a, i] = 1 if node i (0-based) is source a."""
    g = np.zeros((len(nodes_1based), ns))
    for a, j in enumerate(nodes_1based):
        g[a, j - 1] = 1.0
    return g


KMAX = 0.75  # k(1) = 0.5 (1 + 0.5): fixed conductivity bound in the time-step rule


def grid_h(ns: int) -> float:
    """Stage length h = 0.2 dx^2 / kmax for an ``ns``-interior-node axis."""
    dx = 1.0 / (ns + 1)
    return 0.2 * dx * dx / KMAX


def make_problem(name: str, *, ns: Optional[int] = None, N: Optional[int] = None,
                 gamma_rel: float = 1.0, lattice: Optional[int] = None) -> Problem:
    """Problem of a named workload.

    ``c0``: 1D, 16 interior nodes, N=20, h=1e-3, point sources at nodes 4 and 12.
    ``c1``: 2D 64x64, N=40, 4x4 Gaussian lattice (sigma 0.05).
    ``c2``: 2D 256x256, N=100, 8x8 lattice.
    ``grid``: 2D with explicit ``ns``/``N`` (ragged batches use it).
    ``gamma = gamma_rel * h * r``.
    """
    r = 0.01
    if name == "c0":
        nsx = 16
        h = 1e-3
        N_ = 20 if N is None else N
        p = Problem(dim=1, nsx=nsx, nsy=1, N=N_, lx=2, ly=1,
                    gx=point_source_factors(nsx, [4, 12]), gy=np.ones((1, 1)),
                    h=h, r=r, name="c0")
    elif name in ("c1", "c2", "grid"):
        defaults = {"c1": (64, 40, 4), "c2": (256, 100, 8), "grid": (ns, N, 4)}
        ns_, N_, L_ = defaults[name]
        if ns is not None:
            ns_ = ns
        if N is not None:
            N_ = N
        if lattice is not None:
            L_ = lattice
        if ns_ is None or N_ is None:
            raise ValueError("grid workload needs ns and N")
        g = gaussian_factors(ns_, L_, 0.05)
        p = Problem(dim=2, nsx=ns_, nsy=ns_, N=N_, lx=L_, ly=L_, gx=g, gy=g.copy(),
                    h=grid_h(ns_), r=r, name=name if name != "grid" else f"g{ns_}n{N_}")
    else:
        raise KeyError(name)
    p.gamma = gamma_rel * p.h * p.r
    return p


def _xref_field(prob: Problem, rng: np.random.Generator) -> np.ndarray:
    """Smooth reference: 0.3 * s / max|s|, s = sum of 8 seeded sine products."""
    a = rng.integers(1, 5, size=8)
    b = rng.integers(1, 5, size=8)
    c = rng.uniform(-1.0, 1.0, size=8)
    xs = (np.arange(prob.nsx) + 1.0) * prob.dx
    ys = (np.arange(prob.nsy) + 1.0) * prob.dy
    s = np.zeros((prob.nsy, prob.nsx))
    for q in range(8):
        s += c[q] * np.sin(np.pi * b[q] * ys)[:, None] * np.sin(np.pi * a[q] * xs)[None, :]
    mx = np.max(np.abs(s))
    return (0.3 * s / mx).reshape(-1)


def make_instance(prob: Problem, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """(x0, xref) for one seed: x0 ~ U[0, 0.2]^n drawn first, then the reference."""
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(0.0, 0.2, size=prob.n)
    if prob.dim == 1:
        j = np.arange(1, prob.nsx + 1)
        xref = 0.3 * np.sin(np.pi * j / (prob.nsx + 1))
    else:
        xref = _xref_field(prob, rng)
    return x0, xref


def make_batch(prob: Problem, seeds) -> Tuple[np.ndarray, np.ndarray]:
    """Stacked (x0 [B, n], xref [B, n]) for a list of seeds."""
    xs, rs = zip(*(make_instance(prob, int(s)) for s in seeds))
    return np.stack(xs), np.stack(rs)


def ragged_specs(count: int, seed: int = 0,
                 grids=(32, 48, 64, 96), horizons=(20, 40, 60)) -> List[Tuple[int, int, int]]:
    """(ns, N, instance_seed) per instance of a ragged batch, drawn from one seed."""
    rng = np.random.default_rng(seed)
    g = rng.choice(np.asarray(grids), size=count)
    hz = rng.choice(np.asarray(horizons), size=count)
    sd = rng.integers(0, 2**31 - 1, size=count)
    return [(int(a), int(b), int(c)) for a, b, c in zip(g, hz, sd)]


CONFIG_NAMES: Dict[str, str] = {
    "c0": "1D heat, 16 nodes, N=20, 2 point sources",
    "c1": "2D heat 64x64, N=40, 4x4 Gaussian lattice",
    "c2": "2D heat 256x256, N=100, 8x8 Gaussian lattice",
}
