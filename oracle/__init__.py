"""CPU reference ("oracle") for the backward Feynman-Kac exit-probability scheme.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the GPU library never does.  It shares no code
with the GPU path.  The arithmetic lives in ``fkoracle.c`` (plain FP64 C99)
and ``gauss_hermite.py`` (Golub-Welsch); this file only marshals arguments.

Pins (see ``tests/test_oracle_*.py``): Gauss-Hermite nodes against
numpy.polynomial.hermite.hermgauss and the Gaussian moments; Hermite
exactness on cubics; PCHIP exactness on affine data and shape preservation;
pure translation; conservation of constants; the closed-form exit probability
of 1D Brownian motion (paper Section 4.1, Eq. (e45), odd terms only); a Monte
Carlo run of the same discrete chain; convergence orders in dt and dx; finite
differences for the adjoint.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

from .gauss_hermite import gh_rule, tensor_rule  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fkoracle.c")
_LIB = os.path.join(_HERE, "libfkoracle.so")

COEF = {"const": 0, "cellular2d": 1, "abc3d": 2, "rolls2d": 3, "runaway3d": 4}
FACE = {"exit1": 0, "exit0": 1, "reflect": 2}
REGION = {"box": 0, "ball": 1}


def build(force: bool = True) -> str:
    """Compile fkoracle.c into libfkoracle.so (gcc, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=gnu99", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("x", ctypes.POINTER(ctypes.c_double) * 3),
        ("periodic", ctypes.c_int * 3),
        ("coef_kind", ctypes.c_int),
        ("p", ctypes.c_double * 16),
        ("D", ctypes.c_double),
        ("region_kind", ctypes.c_int),
        ("c", ctypes.c_double * 3),
        ("r", ctypes.c_double),
        ("gh_n", ctypes.c_int),
        ("gh_a", ctypes.POINTER(ctypes.c_double)),
        ("gh_w", ctypes.POINTER(ctypes.c_double)),
        ("dt", ctypes.c_double),
        ("n_steps", ctypes.c_int),
        ("t0", ctypes.c_double),
        ("hermite", ctypes.c_int),
        ("face", (ctypes.c_int * 2) * 3),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Problem)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_long)
        up = ctypes.POINTER(ctypes.c_ubyte)
        sig = {
            "fko_num_nodes": (ctypes.c_long, [P]),
            "fko_is_exit_point": (ctypes.c_int, [P, dp]),
            "fko_node_class": (ctypes.c_int, [P, ctypes.c_long]),
            "fko_active_nodes": (ctypes.c_long, [P, lp]),
            "fko_drift": (None, [P, ctypes.c_double, dp, dp]),
            "fko_sigma": (None, [P, ctypes.c_double, dp, dp]),
            "fko_re_coeffs": (None, [P, ctypes.c_double, ctypes.c_double, dp]),
            "fko_exit_value": (ctypes.c_int, [P, dp]),
            "fko_num_theta": (ctypes.c_int, [P]),
            "fko_landing": (None, [P, ctypes.c_int, ctypes.c_long, ctypes.c_int, dp]),
            "fko_cell": (ctypes.c_int, [dp, ctypes.c_int, ctypes.c_double]),
            "fko_slopes": (None, [P, dp, dp]),
            "fko_num_fields": (ctypes.c_int, [P]),
            "fko_interp": (ctypes.c_double, [P, dp, dp, dp]),
            "fko_interp_grad": (None, [P, dp, dp, dp, dp]),
            "fko_step": (ctypes.c_int, [P, ctypes.c_int, dp, dp]),
            "fko_step_cells": (ctypes.c_int, [P, ctypes.c_int, dp, ip, up]),
            "fko_chi": (None, [P, dp]),
            "fko_solve": (ctypes.c_int, [P, ip, ctypes.c_int, dp, up, up]),
            "fko_solve_horizons": (ctypes.c_int, [P, ip, ctypes.c_int, dp]),
            "fko_assemble_row": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_long, dp, dp]),
            "fko_adjoint": (ctypes.c_int, [P, dp, dp, dp, up]),
            "fko_solve_all": (ctypes.c_int, [P, dp, up]),
            "fko_adjoint_states": (ctypes.c_int, [P, dp, dp, dp, dp, up]),
            "fko_set_flat_rel": (None, [ctypes.c_double]),
            "fko_get_flat_rel": (ctypes.c_double, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _up(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))


class OracleProblem:
    """A workloads.Problem marshalled for the C oracle (keeps arrays alive)."""

    def __init__(self, prob, gh_q: Optional[int] = None, D: Optional[float] = None,
                 coef: Optional[Sequence[float]] = None):
        self.prob = prob
        q = prob.gh_q if gh_q is None else gh_q
        a, w = gh_rule(q)
        self.gh_a = np.ascontiguousarray(a, dtype=np.float64)
        self.gh_w = np.ascontiguousarray(w, dtype=np.float64)
        self.nodes = [np.ascontiguousarray(ax.nodes, dtype=np.float64) for ax in prob.axes]
        s = _Problem()
        s.d = prob.d
        for i in range(3):
            s.n[i] = prob.axes[i].n if i < prob.d else 1
            s.periodic[i] = int(prob.axes[i].periodic) if i < prob.d else 0
            s.x[i] = _dp(self.nodes[i]) if i < prob.d else None
        s.coef_kind = COEF[prob.coef_kind]
        cf = list(prob.coef if coef is None else coef)
        for i in range(16):
            s.p[i] = float(cf[i]) if i < len(cf) else 0.0
        s.D = float(prob.D if D is None else D)
        s.region_kind = REGION[prob.region_kind]
        for i in range(3):
            s.c[i] = float(prob.center[i]) if i < len(prob.center) else 0.0
        s.r = float(prob.radius)
        s.gh_n = q
        s.gh_a = _dp(self.gh_a)
        s.gh_w = _dp(self.gh_w)
        s.dt = float(prob.dt)
        s.n_steps = int(prob.n_steps)
        s.t0 = float(prob.t0)
        s.hermite = 2 if getattr(prob, "hermite", "r1") == "r2" else 1
        faces = getattr(prob, "faces", None)
        for a in range(3):
            for side in range(2):
                s.face[a][side] = FACE[faces[a][side]] if faces and a < len(faces) else 0
        self.s = s
        self.Q = q ** prob.d
        self.J = int(np.prod(prob.shape))
        self.shape = prob.shape

    @property
    def ptr(self):
        return ctypes.byref(self.s)


def _op(prob, **kw) -> OracleProblem:
    return prob if isinstance(prob, OracleProblem) else OracleProblem(prob, **kw)


def node_class(prob) -> np.ndarray:
    """0 active, 1 exit, 2 periodic image; shape = grid shape."""
    op = _op(prob)
    lib = _load()
    return np.array([lib.fko_node_class(op.ptr, j) for j in range(op.J)],
                    dtype=np.int8).reshape(op.shape)


def active_nodes(prob) -> np.ndarray:
    op = _op(prob)
    lib = _load()
    m = lib.fko_active_nodes(op.ptr, None)
    out = np.zeros(max(m, 1), dtype=np.int64)
    lib.fko_active_nodes(op.ptr, out.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))
    return out[:m]


def chi(prob) -> np.ndarray:
    op = _op(prob)
    u = np.zeros(op.J)
    _load().fko_chi(op.ptr, _dp(u))
    return u.reshape(op.shape)


def drift(prob, t: float, x: Sequence[float]) -> np.ndarray:
    op = _op(prob)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    b = np.zeros(3)
    _load().fko_drift(op.ptr, float(t), _dp(xx), _dp(b))
    return b[: op.prob.d]


def sigma(prob, t: float, x: Sequence[float]) -> np.ndarray:
    """Diffusion coefficient of each axis (the SDE's dW factor) at (t, x)."""
    op = _op(prob)
    xx = np.zeros(3)
    xx[: len(x)] = x
    sg = np.zeros(3)
    _load().fko_sigma(op.ptr, float(t), _dp(xx), _dp(sg))
    return sg[: op.prob.d]


def re_coeffs(prob, t: float, p: float) -> np.ndarray:
    """Runaway-electron collision functions (C_A, C_B, C_F, dC_A/dp) at
    momentum p and time t."""
    op = _op(prob)
    out = np.zeros(4)
    _load().fko_re_coeffs(op.ptr, float(t), float(p), _dp(out))
    return out


def exit_value(prob, z) -> int:
    """-1 if z does not exit, else the value it takes (1 or 0)."""
    op = _op(prob)
    zz = np.zeros(3)
    zz[: len(z)] = z
    return int(_load().fko_exit_value(op.ptr, _dp(zz)))


def cell(nodes: np.ndarray, z: float) -> int:
    x = np.ascontiguousarray(nodes, dtype=np.float64)
    return int(_load().fko_cell(_dp(x), x.shape[0], float(z)))


def landing(prob, n: int, j: int, q: int) -> np.ndarray:
    op = _op(prob)
    z = np.zeros(3)
    _load().fko_landing(op.ptr, int(n), int(j), int(q), _dp(z))
    return z[: op.prob.d]


def is_exit_point(prob, z) -> bool:
    op = _op(prob)
    zz = np.zeros(3)
    zz[: len(z)] = z
    return bool(_load().fko_is_exit_point(op.ptr, _dp(zz)))


def slopes(prob, u: np.ndarray) -> np.ndarray:
    """Derivative fields: the PCHIP slopes along every axis and, for the R2
    interpolant, the twist fields ({0,1}, {0,2}, {1,2}, {0,1,2});
    shape (fields,) + grid shape."""
    op = _op(prob)
    lib = _load()
    nf = int(lib.fko_num_fields(op.ptr))
    uu = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    g = np.zeros(op.J * nf)
    lib.fko_slopes(op.ptr, _dp(uu), _dp(g))
    return g.reshape((nf,) + tuple(op.shape))


def interp(prob, u: np.ndarray, g: np.ndarray, z, grad: bool = False):
    op = _op(prob)
    uu = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    gg = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
    zz = np.zeros(3)
    zz[: len(z)] = z
    lib = _load()
    if grad:
        out = np.zeros(3)
        lib.fko_interp_grad(op.ptr, _dp(uu), _dp(gg), _dp(zz), _dp(out))
        return out[: op.prob.d]
    return float(lib.fko_interp(op.ptr, _dp(uu), _dp(gg), _dp(zz)))


def step(prob, n: int, u_next: np.ndarray) -> np.ndarray:
    """One backward step u^{n+1} -> u^n from an arbitrary state."""
    op = _op(prob)
    uu = np.ascontiguousarray(u_next, dtype=np.float64).reshape(-1)
    out = np.zeros(op.J)
    if _load().fko_step(op.ptr, int(n), _dp(uu), _dp(out)) != 0:
        raise MemoryError("oracle step failed")
    return out.reshape(op.shape)


def step_cells(prob, n: int, u_next: np.ndarray):
    """Landing cells [Ja, Q, d] (-1 where the point exits) and exit flags [Ja, Q]."""
    op = _op(prob)
    Ja = active_nodes(op).shape[0]
    uu = np.ascontiguousarray(u_next, dtype=np.float64).reshape(-1)
    cells = np.zeros((max(Ja, 1), op.Q, op.prob.d), dtype=np.int32)
    exitf = np.zeros((max(Ja, 1), op.Q), dtype=np.uint8)
    if _load().fko_step_cells(op.ptr, int(n), _dp(uu), _ip(cells), _up(exitf)) != 0:
        raise MemoryError("oracle step_cells failed")
    return cells[:Ja], exitf[:Ja]


def exit_bits_size(prob) -> int:
    op = _op(prob)
    Ja = active_nodes(op).shape[0]
    return (op.prob.n_steps * Ja * op.Q + 7) // 8


def solve(prob, snaps: Sequence[int] = (0,), record_exits: bool = False,
          frozen_exits: Optional[np.ndarray] = None, **kw):
    """Whole backward pass; returns array [len(snaps)] + grid shape (and the
    exit-bit record when ``record_exits``)."""
    op = _op(prob, **kw)
    sn = np.ascontiguousarray(snaps, dtype=np.int32)
    out = np.zeros((len(sn), op.J))
    rec = np.zeros(exit_bits_size(op), dtype=np.uint8) if record_exits else None
    use = None if frozen_exits is None else np.ascontiguousarray(frozen_exits, dtype=np.uint8)
    rc = _load().fko_solve(op.ptr, _ip(sn), len(sn), _dp(out), _up(rec), _up(use))
    if rc != 0:
        raise MemoryError("oracle solve failed")
    out = out.reshape((len(sn),) + tuple(op.shape))
    return (out, rec) if record_exits else out


def solve_horizons(prob, horizons: Sequence[int]) -> np.ndarray:
    """Algorithm 1 (Section 3.2): p^m of Eq. (e37) for every horizon m (in
    steps, from the problem's t0) in one backward sweep; array
    [len(horizons)] + grid shape."""
    op = _op(prob)
    m = np.ascontiguousarray(horizons, dtype=np.int32)
    out = np.zeros((len(m), op.J))
    rc = _load().fko_solve_horizons(op.ptr, _ip(m), len(m), _dp(out))
    if rc == -2:
        raise ValueError("horizons must be >= 1")
    if rc != 0:
        raise MemoryError("oracle solve_horizons failed")
    return out.reshape((len(m),) + tuple(op.shape))


def assemble_row(prob, n: int, j: int):
    """Dense row of A_n: (coefficients [(d+1), J], exit mass)."""
    op = _op(prob)
    row = np.zeros(op.J * (op.prob.d + 1))
    em = np.zeros(1)
    _load().fko_assemble_row(op.ptr, int(n), int(j), _dp(row), _dp(em))
    return row.reshape(op.prob.d + 1, op.J), float(em[0])


def num_theta(prob) -> int:
    return int(_load().fko_num_theta(_op(prob).ptr))


def adjoint(prob, lam0: np.ndarray, frozen_exits: Optional[np.ndarray] = None, **kw):
    """Gradient of <lam0, u^0> w.r.t. theta = (drift params..., D), and lam^N."""
    op = _op(prob, **kw)
    lam = np.ascontiguousarray(lam0, dtype=np.float64).reshape(-1)
    grad = np.zeros(8)
    lamN = np.zeros(op.J)
    use = None if frozen_exits is None else np.ascontiguousarray(frozen_exits, dtype=np.uint8)
    rc = _load().fko_adjoint(op.ptr, _dp(lam), _dp(grad), _dp(lamN), _up(use))
    if rc != 0:
        raise MemoryError("oracle adjoint failed")
    return grad[: num_theta(op)], lamN.reshape(op.shape)


def solve_all(prob, frozen_exits: Optional[np.ndarray] = None, **kw) -> np.ndarray:
    """Every state of the backward pass: array [N + 1] + grid shape, entry n = u^n."""
    op = _op(prob, **kw)
    N = int(op.prob.n_steps)
    U = np.zeros((N + 1) * op.J)
    use = None if frozen_exits is None else np.ascontiguousarray(frozen_exits, dtype=np.uint8)
    if _load().fko_solve_all(op.ptr, _dp(U), _up(use)) != 0:
        raise MemoryError("oracle solve_all failed")
    return U.reshape((N + 1,) + tuple(op.shape))


def adjoint_states(prob, U: np.ndarray, lam0: np.ndarray,
                   frozen_exits: Optional[np.ndarray] = None, **kw):
    """Reverse sweep of the adjoint from caller-supplied states U[n] = u^n
    (n = 0..N); returns (grad, lam^N) like ``adjoint``."""
    op = _op(prob, **kw)
    UU = np.ascontiguousarray(U, dtype=np.float64).reshape(-1)
    assert UU.shape[0] == (op.prob.n_steps + 1) * op.J
    lam = np.ascontiguousarray(lam0, dtype=np.float64).reshape(-1)
    grad = np.zeros(8)
    lamN = np.zeros(op.J)
    use = None if frozen_exits is None else np.ascontiguousarray(frozen_exits, dtype=np.uint8)
    rc = _load().fko_adjoint_states(op.ptr, _dp(UU), _dp(lam), _dp(grad), _dp(lamN), _up(use))
    if rc != 0:
        raise MemoryError("oracle adjoint_states failed")
    return grad[: num_theta(op)], lamN.reshape(op.shape)


class flat_rel:
    """Context manager setting the oracle's flat-stretch threshold of the PCHIP
    linearisation (relative; default 2^-30, 0 = exact equality only)."""

    def __init__(self, r: float):
        self.r = float(r)

    def __enter__(self):
        lib = _load()
        self.old = lib.fko_get_flat_rel()
        lib.fko_set_flat_rel(self.r)
        return self

    def __exit__(self, *exc):
        _load().fko_set_flat_rel(self.old)
        return False
