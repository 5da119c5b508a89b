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
    "ModelProblem",
    "make_plate_problem",
    "make_plate_instance",
    "make_wave_problem",
    "make_wave_instance",
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
    B: Optional[np.ndarray] = None   # explicit dense input matrix [n, m] (overrides gx, gy)

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
        """Input matrix B [n, m] with B[iy*nsx+ix, b*lx+a] = gy[b,iy] gx[a,ix],
        or the explicit matrix when one is given."""
        if self.B is not None:
            return np.asarray(self.B, dtype=np.float64)
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


# ----------------------------------------------------------------------------
# Further workloads of the paper's PDE class (Sec. 2): problem data only.

@dataclasses.dataclass
class ModelProblem:
    """One discretized NMPC problem of the model engine (data only).

    Grid: ``nsy x nsx`` nodes, node ``p = iy * nsx + ix``. ``boundary``:
    ``"neumann"`` -- the nodes include the boundary of the unit square
    (``dx = 1/(nsx-1)``) and the normal derivative is zero there (Sec. 2.1,
    fictitious points); ``"dirichlet"`` -- interior nodes (``dx = 1/(nsx+1)``),
    zero values outside.

    Models (``model``):
      ``"plate"`` -- thin plate, ``w_t = alpha Lap w - beta (w - t_amb) -
      rad (w^4 - t_amb^4)`` (Sec. 5); the inputs are the temperatures of the
      actuator nodes ``act`` (those nodes are not states);
      ``"wave"`` -- second order in time (Sec. 2, a = 1):
      ``W_tt + damp W_t = k0 (1 + k1 W) Lap W + B u``, state ``(W, W_t)``;
      ``"heat"`` -- ``w_t = k0 (1 + k1 w) Lap w + B u`` with a dense B.
    Stage cost ``0.5 q |w - wref|^2 + 0.5 qv |W_t|^2 + 0.5 r |u - uref|^2``
    (qv: wave only), regularization ``gamma``, optional input box ``[u_lo,
    u_hi]`` by the log barrier ``tau`` (eq. nlp_relaxed).
    """

    model: str
    nsx: int
    nsy: int
    N: int
    h: float
    boundary: str = "dirichlet"
    act: Optional[List[int]] = None      # plate: actuator node indices
    B: Optional[np.ndarray] = None       # wave / heat: [nsx*nsy, m]
    q: float = 1.0
    qv: float = 0.0
    r: float = 0.01
    gamma: float = 0.0
    tau: float = 0.0
    u_lo: float = 0.0
    u_hi: float = 0.0
    u_cold: float = 0.0                  # inputs of the cold start
    alpha: float = 0.0                   # plate physics
    beta: float = 0.0
    rad: float = 0.0
    t_amb: float = 0.0
    k0: float = 0.0                      # wave / heat physics
    k1: float = 0.0
    damp: float = 0.0
    name: str = ""

    @property
    def nodes(self) -> int:
        return self.nsx * self.nsy

    @property
    def m(self) -> int:
        return len(self.act) if self.model == "plate" else int(self.B.shape[1])

    @property
    def dx(self) -> float:
        return 1.0 / (self.nsx - 1) if self.boundary == "neumann" else 1.0 / (self.nsx + 1)

    @property
    def dy(self) -> float:
        if self.nsy == 1:
            return 1.0
        return 1.0 / (self.nsy - 1) if self.boundary == "neumann" else 1.0 / (self.nsy + 1)

    def with_(self, **kw) -> "ModelProblem":
        return dataclasses.replace(self, **kw)


# Copper plate of Sec. 5 (Table of process parameters)
PLATE_RHO, PLATE_CP, PLATE_TZ, PLATE_K = 8960.0, 386.0, 0.01, 400.0
PLATE_HC, PLATE_TA, PLATE_EPS, PLATE_SB = 1.0, 300.0, 0.5, 5.67e-8
PLATE_ACT_AXIS = (2, 5, 7, 10)   # actuator rows/columns on the 13 x 13 grid (reading)


def make_plate_problem(N: int = 20, T: float = 100.0, ns: int = 13,
                       tau: float = 100.0, gamma: float = 0.5, r: float = 0.1) -> ModelProblem:
    """The paper's copper-plate NMPC problem: 13 x 13 nodes, zero Neumann
    boundary, 16 actuator nodes (a 4 x 4 lattice at rows/columns 2, 5, 7, 10:
    the figure with their positions is not available), inputs boxed to
    [T_a, T_a + 400] with tau = 100, gamma = 0.5, Q = I, R = 0.1 I, T = 100 s,
    N = 20. The PDE rho C_p t_z w_t = k t_z Lap w - 2 Q_c - 2 Q_r divided by
    rho C_p t_z."""
    if ns != 13:
        axis = tuple(int(round(v * (ns - 1) / 12.0)) for v in PLATE_ACT_AXIS)
    else:
        axis = PLATE_ACT_AXIS
    act = [iy * ns + ix for iy in axis for ix in axis]
    c = PLATE_RHO * PLATE_CP * PLATE_TZ
    return ModelProblem(model="plate", nsx=ns, nsy=ns, N=N, h=T / N, boundary="neumann",
                        act=act, q=1.0, r=r, gamma=gamma, tau=tau, u_lo=PLATE_TA,
                        u_hi=PLATE_TA + 400.0, u_cold=PLATE_TA + 200.0,
                        alpha=PLATE_K / (PLATE_RHO * PLATE_CP), beta=2.0 * PLATE_HC / c,
                        rad=2.0 * PLATE_EPS * PLATE_SB / c, t_amb=PLATE_TA, name="plate")


def plate_reference(P: ModelProblem, kind: str, rng: np.random.Generator) -> np.ndarray:
    """Temperature reference over all nodes [nsy*nsx]: a slope or a V shape
    (the paper's two reference shapes, drawn from the seed: direction, level
    and amplitude), inside [T_a + 50, T_a + 350]."""
    xs = np.linspace(0.0, 1.0, P.nsx)
    ys = np.linspace(0.0, 1.0, P.nsy)
    X, Y = np.meshgrid(xs, ys)
    th = rng.uniform(0.0, 2.0 * np.pi)
    s = np.cos(th) * (X - 0.5) + np.sin(th) * (Y - 0.5)
    if kind == "v":
        s = np.abs(s - rng.uniform(-0.2, 0.2))
    s = (s - s.min()) / max(s.max() - s.min(), 1e-12)
    lo = rng.uniform(50.0, 120.0)
    amp = rng.uniform(120.0, 230.0)
    return (P.t_amb + lo + amp * s).reshape(-1)


def make_plate_instance(P: ModelProblem, seed: int, kind: Optional[str] = None):
    """(x0 [nodes], xref [nodes]) for one seed. x0: the ambient temperature
    plus a seeded disturbance U[0, 20] K (seed 0 with kind given: exactly the
    ambient temperature, the paper's start); the actuator nodes' entries are
    not states and are ignored by the solvers (the reference's values there
    are the input references u_ref)."""
    rng = np.random.default_rng(seed)
    k = kind if kind is not None else ("slope" if rng.uniform() < 0.5 else "v")
    dist = rng.uniform(0.0, 20.0, size=P.nodes)
    x0 = np.full(P.nodes, P.t_amb) + (0.0 if (kind is not None and seed == 0) else dist)
    return x0, plate_reference(P, k, rng)


def make_wave_problem(ns: int = 24, N: int = 30, lattice: int = 4, sigma: float = 0.1,
                      k0: float = 1.0, k1: float = 0.5, damp: float = 2.0, rho: float = 0.3,
                      q: float = 1.0, qv: float = 0.1, r: float = 0.01,
                      gamma_rel: float = 1.0) -> ModelProblem:
    """Nonlinear damped membrane, second order in time, on ns x ns interior
    nodes (zero Dirichlet values), Gaussian actuator lattice as a dense B.
    The stage length is chosen from the sweep contraction of the reduced
    system (eq. jaco2_sys): 4 h^2 kmax / dx^2 = rho with kmax = k0 (1 + k1)."""
    dx = 1.0 / (ns + 1)
    g = gaussian_factors(ns, lattice, sigma)
    B = np.kron(g.T, g.T)
    kmax = k0 * (1.0 + k1)
    h = dx * np.sqrt(rho / (4.0 * kmax))
    return ModelProblem(model="wave", nsx=ns, nsy=ns, N=N, h=float(h), boundary="dirichlet",
                        B=B, q=q, qv=qv, r=r, gamma=gamma_rel * h * r, k0=k0, k1=k1,
                        damp=damp, name=f"wave{ns}n{N}")


def make_wave_instance(P: ModelProblem, seed: int):
    """(x0 [2 nodes]: W0 ~ U[0, 0.2] then W_t = 0; xref [nodes]: W reference,
    the smooth field of the heat workloads)."""
    rng = np.random.default_rng(seed)
    W0 = rng.uniform(0.0, 0.2, size=P.nodes)
    a = rng.integers(1, 5, size=8)
    b = rng.integers(1, 5, size=8)
    c = rng.uniform(-1.0, 1.0, size=8)
    xs = (np.arange(P.nsx) + 1.0) * P.dx
    ys = (np.arange(P.nsy) + 1.0) * P.dy
    s = np.zeros((P.nsy, P.nsx))
    for k in range(8):
        s += c[k] * np.sin(np.pi * b[k] * ys)[:, None] * np.sin(np.pi * a[k] * xs)[None, :]
    wref = (0.3 * s / np.max(np.abs(s))).reshape(-1)
    return np.concatenate([W0, np.zeros(P.nodes)]), wref
