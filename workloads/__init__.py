"""Seeded synthetic workloads for the backward Feynman-Kac exit-probability scheme.

This module only *describes* problems: grids (node coordinate arrays), drift
and diffusion parameters, exit regions, quadrature order, time step and step
count.  It holds none of the scheme's arithmetic, so the CPU reference
(``oracle/``) and the GPU library (``paper_2104_14561_amd``) can both take
their inputs from here without sharing any computation.

Problem statement (paper, Section 2, Eq. (e1)-(e2)): an SDE
dX = b(t,X) dt + sigma(t,X) dW on a box, exit probability P(t,x).  All
workloads here use an isotropic constant diffusion sigma = sqrt(2 D) I, as in
dX = sqrt(2D) dW.

Workloads (the paper's flows are analytic, so these stand in for them exactly;
there is no dataset):

* ``bm1d``        1D Brownian motion, D = 0.5, exit from (-1, 1), 201 nodes,
                  T = 1, dt = 0.01, 16-node Gauss-Hermite rule (Section 4.1).
* ``cell2d``      time-periodic cellular flow, stream function
                  psi = A sin(pi (x + eps sin(omega t))) sin(pi y) on
                  [0,2]x[0,1], 513x257 nodes, exit region = complement of the
                  disc of radius 0.3 centred at (0.5, 0.5), 8x8 nodes
                  (a cellular flow as in Section 4.2, with a disc target).
* ``cell2d_batch64`` 64 seeded cellular-flow instances on uneven grids.
* ``cell2d_adj``  ``cell2d`` with dt = 5e-4 and 2000 steps.
* ``abc3d``       time-modulated ABC flow on a 129^3 grid, periodic in x, y,
                  exit at |z| >= pi/2, 6x6x6 nodes; ``abc3d_batch8`` draws D.
* ``paper2d``     the paper's own 2D example (Section 4.2): Pe = 10 roll flow,
                  periodic in x_1, exit through x_2 in {0, 1}.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

COEF_CONST = "const"            # p = (b_0, .., b_{d-1}); constant drift
COEF_CELLULAR2D = "cellular2d"  # p = (A, eps, omega)
COEF_ABC3D = "abc3d"            # p = (A, B, C, amp)
COEF_ROLLS2D = "rolls2d"        # p = (Pe, eps, omega, n): the flow of Section 4.2

REGION_BOX = "box"    # exit when a non-periodic coordinate leaves the open box
REGION_BALL = "ball"  # exit also when |z - c| >= r

N_DRIFT_PARAMS = {COEF_CONST: None, COEF_CELLULAR2D: 3, COEF_ABC3D: 4, COEF_ROLLS2D: 3}


@dataclasses.dataclass
class Axis:
    """One axis of the Cartesian mesh S = S^1 x ... x S^d (paper Section 3.1.2).

    ``nodes`` are strictly increasing coordinates.  On a periodic axis the last
    node is the image of the first one (x[n-1] = x[0] + period) and carries the
    same value.
    """

    nodes: np.ndarray
    periodic: bool = False

    def __post_init__(self):
        self.nodes = np.ascontiguousarray(self.nodes, dtype=np.float64)

    @property
    def n(self) -> int:
        return int(self.nodes.shape[0])


@dataclasses.dataclass
class Problem:
    """One instance of the exit-probability problem.

    Attributes follow the paper's problem statement: the grid, the drift b
    (``coef_kind`` + ``coef``), the diffusion D (sigma = sqrt(2D) I), the
    exit region, the Gauss-Hermite order Q* (``gh_q`` nodes per Brownian
    dimension), the time step ``dt``, the step count ``n_steps`` and the start
    time ``t0`` (step n uses coefficients at t0 + n dt).
    """

    axes: List[Axis]
    coef_kind: str
    coef: Tuple[float, ...]
    D: float
    region_kind: str = REGION_BOX
    center: Tuple[float, ...] = (0.0, 0.0, 0.0)
    radius: float = 0.0
    gh_q: int = 3
    dt: float = 1e-2
    n_steps: int = 1
    t0: float = 0.0
    name: str = ""
    hermite: str = "r1"   # "r1": values and first derivatives; "r2": also the mixed ones
    # per axis (low face, high face) of the box: "exit1" (a point on or beyond
    # it exits with value 1, the default), "exit0" (exits with value 0) or
    # "reflect"; None: every face "exit1"
    faces: Optional[Tuple[Tuple[str, str], ...]] = None

    @property
    def d(self) -> int:
        return len(self.axes)

    @property
    def shape(self) -> Tuple[int, ...]:
        return tuple(a.n for a in self.axes)

    @property
    def n_nodes(self) -> int:
        return int(np.prod(self.shape))

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def uniform_axis(lo: float, hi: float, n: int, periodic: bool = False) -> Axis:
    return Axis(np.linspace(lo, hi, n), periodic)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def bm1d(n: int = 201, dt: float = 0.01, n_steps: int = 100, gh_q: int = 16,
         D: float = 0.5) -> Problem:
    """1D Brownian motion dX = sqrt(2D) dW, exit from (-1, 1)."""
    return Problem(axes=[uniform_axis(-1.0, 1.0, n)], coef_kind=COEF_CONST,
                   coef=(0.0,), D=D, region_kind=REGION_BOX, gh_q=gh_q,
                   dt=dt, n_steps=n_steps, name="bm1d")


def cell2d(nx: int = 513, ny: int = 257, A: float = 1.0, eps: float = 0.1,
           omega: float = 2.0 * math.pi, D: float = 1e-3, dt: float = 1e-3,
           n_steps: int = 1000, gh_q: int = 8, radius: float = 0.3,
           center=(0.5, 0.5), name: str = "cell2d") -> Problem:
    """Cellular flow psi = A sin(pi(x + eps sin(omega t))) sin(pi y), disc target."""
    return Problem(axes=[uniform_axis(0.0, 2.0, nx), uniform_axis(0.0, 1.0, ny)],
                   coef_kind=COEF_CELLULAR2D, coef=(A, eps, omega), D=D,
                   region_kind=REGION_BALL, center=tuple(center) + (0.0,),
                   radius=radius, gh_q=gh_q, dt=dt, n_steps=n_steps, name=name)


def cell2d_adj(**kw) -> Problem:
    kw.setdefault("dt", 5e-4)
    kw.setdefault("n_steps", 2000)
    kw.setdefault("name", "cell2d_adj")
    return cell2d(**kw)


BATCH64_SEED = 210414561
ABC8_SEED = 210414562


def cell2d_batch(n_inst: int = 64, seed: int = BATCH64_SEED, n_steps: int = 1000,
                 dt: float = 1e-3, gh_q: int = 8, max_m: int = 8) -> List[Problem]:
    """Seeded cellular-flow instances on uneven grids (128m+1) x (64m+1).

    Per instance, in order: m ~ U{1..max_m}, A ~ U[0.5, 1.5], eps ~ U[0, 0.3],
    omega ~ U[pi, 4 pi], log10 D ~ U[-4, -2].
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_inst):
        m = int(rng.integers(1, max_m + 1))
        A = float(rng.uniform(0.5, 1.5))
        eps = float(rng.uniform(0.0, 0.3))
        omega = float(rng.uniform(math.pi, 4.0 * math.pi))
        D = float(10.0 ** rng.uniform(-4.0, -2.0))
        out.append(cell2d(nx=128 * m + 1, ny=64 * m + 1, A=A, eps=eps, omega=omega,
                          D=D, dt=dt, n_steps=n_steps, gh_q=gh_q,
                          name=f"cell2d_batch[{i}]"))
    return out


def abc3d(n: int = 129, D: float = 5e-4, A: float = 1.0, B: float = 0.8,
          C: float = 0.6, amp: float = 0.1, dt: float = 2e-3, n_steps: int = 500,
          gh_q: int = 6, name: str = "abc3d") -> Problem:
    """ABC flow (A sin z + C cos y, B sin x + A cos z, C sin y + B cos x),
    each amplitude times (1 + amp sin t); periodic in x, y; exit at |z| >= pi/2."""
    two_pi = 2.0 * math.pi
    return Problem(axes=[uniform_axis(0.0, two_pi, n, periodic=True),
                         uniform_axis(0.0, two_pi, n, periodic=True),
                         uniform_axis(-0.5 * math.pi, 0.5 * math.pi, n)],
                   coef_kind=COEF_ABC3D, coef=(A, B, C, amp), D=D,
                   region_kind=REGION_BOX, gh_q=gh_q, dt=dt, n_steps=n_steps,
                   name=name)


def abc3d_batch(n_inst: int = 8, seed: int = ABC8_SEED, **kw) -> List[Problem]:
    """ABC instances with log10 D ~ U[-4, -3] (seeded)."""
    rng = np.random.default_rng(seed)
    Ds = [float(10.0 ** rng.uniform(-4.0, -3.0)) for _ in range(n_inst)]
    return [abc3d(D=D, name=f"abc3d_batch[{i}]", **kw) for i, D in enumerate(Ds)]


def paper2d(n1: int = 129, n2: int = 33, Pe: float = 10.0, eps: float = 0.15,
            omega: float = 2.0 * math.pi / 10.0, n: int = 2, T: float = 0.05,
            dt: float = 5e-4, gh_q: int = 6) -> Problem:
    """The paper's own 2D example (Section 4.2, Eq. (ex2model)-(ex3)):
    dX = Pe v(X, t) dt + dW on [-pi, pi] x [0, 1], periodic in x_1, exit
    through x_2 = 0 and x_2 = 1, with the cellular (Rayleigh-Benard roll)
    velocity v of 2n cells perturbed by eps cos(omega t); Pe = 10,
    eps = 0.15, omega = 2 pi / 10, n = 2, T_max = 0.05.  dW has unit
    variance rate, so D = 1/2.  The grid, dt and Q* are not given in the
    paper: 128 cells on the periodic axis, 32 across, dt = 5e-4 (100 steps)
    and a 6-node rule."""
    return Problem(axes=[uniform_axis(-math.pi, math.pi, n1, periodic=True),
                         uniform_axis(0.0, 1.0, n2)],
                   coef_kind=COEF_ROLLS2D, coef=(Pe, eps, omega, float(n)), D=0.5,
                   region_kind=REGION_BOX, gh_q=gh_q, dt=dt,
                   n_steps=int(round(T / dt)), name="paper2d")


COEF_RUNAWAY3D = "runaway3d"

# Section 4.3, Eq. (parameters): the time-independent runaway-electron model
RE_PARAMS = dict(E=0.3, tau=1e5, Z=1.0, delta=0.042, nu_ee=1.0, v_T=1.0, r_D=0.7, W=1e-2,
                 Delta_p=20.0, V0=0.003, D0=1e-4)


def remark2_axis(lo: float, mid: float, hi: float, h_coarse: float, h_fine: float) -> Axis:
    """Piecewise-uniform axis: spacing h_coarse on [lo, mid], h_fine on
    [mid, hi] (the non-uniform radial grid of Section 4.3)."""
    a = np.linspace(lo, mid, int(round((mid - lo) / h_coarse)) + 1)
    b = np.linspace(mid, hi, int(round((hi - mid) / h_fine)) + 1)
    return Axis(np.concatenate([a, b[1:]]))


def runaway3d(n_p: int = 49, n_xi: int = 41, r_axis: Optional[Axis] = None,
              p_min: float = 2.0, p_max: float = 50.0, dt: float = 0.5, T: float = 120.0,
              gh_q: int = 4, t_star: float = 0.0, name: str = "runaway3d", **params) -> Problem:
    """The runaway-electron model of Section 4.3 (Eq. (ex32d)): state (p, xi,
    r), xi = cos(theta); p in (p_min, p_max), xi in [-1, 1], r in [0, 1].
    Runaway means leaving through p = p_max (value 1); leaving through p_min
    (thermalised) or the wall r = 1 counts 0; xi = +-1 and the axis r = 0
    reflect.  Default r grid: the paper's non-uniform one, spacing 0.1 on
    [0, r_D] and 0.0025 on [r_D, 1].  The p and xi grids, dt and Q* are not
    given in the paper (49 x 41 nodes, dt = 0.5, Q* = 4).  t_star > 0 gives
    the thermal-quench model (then pass E0, That0, Thatf, Ttilde)."""
    q = dict(RE_PARAMS)
    q.update(params)
    if r_axis is None:
        r_axis = remark2_axis(0.0, q["r_D"], 1.0, 0.1, 0.0025)
    coef = (q["E"] if t_star <= 0 else q.get("E0", 1e-3), q["tau"], q["Z"], q["delta"], q["nu_ee"],
            q["v_T"], q["r_D"], q["W"], q["Delta_p"], q["V0"], q["D0"], t_star,
            q.get("That0", 3.0), q.get("Thatf", 0.005), q.get("Ttilde", 3.0), q.get("mc2", 511.0))
    return Problem(axes=[uniform_axis(p_min, p_max, n_p), uniform_axis(-1.0, 1.0, n_xi), r_axis],
                   coef_kind=COEF_RUNAWAY3D, coef=coef, D=0.0, region_kind=REGION_BOX,
                   gh_q=gh_q, dt=dt, n_steps=int(round(T / dt)), name=name,
                   faces=(("exit0", "exit1"), ("reflect", "reflect"), ("reflect", "exit0")))


def region_mean_weights(prob: "Problem") -> np.ndarray:
    """Objective weights for J = mean of u^0 over the target region: 1/m on
    the m nodes strictly inside the disc/ball (squared distance below r^2),
    0 elsewhere; for a box region, on every node off the non-periodic faces.
    Shape prob.shape.  This is an input (dJ/du^0), not part of the scheme."""
    grids = np.meshgrid(*[ax.nodes for ax in prob.axes], indexing="ij")
    if prob.region_kind == "ball":
        d2 = np.zeros(prob.shape)
        for a, g in enumerate(grids):
            d2 = d2 + (g - prob.center[a]) ** 2
        mask = d2 < prob.radius ** 2
    else:
        mask = np.ones(prob.shape, dtype=bool)
        for a, ax in enumerate(prob.axes):
            if not ax.periodic:
                idx = [slice(None)] * prob.d
                for end in (0, -1):
                    idx[a] = end
                    mask[tuple(idx)] = False
    m = mask.astype(np.float64)
    return m / max(m.sum(), 1.0)


def random_field(shape: Sequence[int], seed: int, lo: float = 0.0,
                 hi: float = 1.0) -> np.ndarray:
    """Seeded uniform random field (test states for single-step checks)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=tuple(shape)).astype(np.float64)


def by_name(name: str):
    table = {
        "bm1d": lambda: [bm1d()],
        "cell2d": lambda: [cell2d()],
        "cell2d_batch64": lambda: cell2d_batch(),
        "cell2d_adj": lambda: [cell2d_adj()],
        "abc3d_batch8": lambda: abc3d_batch(),
    }
    return table[name]()
