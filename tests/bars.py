"""Test bars derived from the oracle's own sensitivity (test infrastructure).

Where the scheme amplifies rounding, two correct FP64 implementations that
round differently disagree by more than their rounding; the bar of a GPU
comparison is then the oracle's response to perturbations of the size of
that rounding difference, measured on the CPU."""
from __future__ import annotations

import numpy as np

import oracle

# relative difference of the GPU's and the oracle's FP64 states: 2^-44
# (256 ulps of 1), above the 1e-13 absolute the single-step FP64 parity
# tests allow on values of at most 1
STATE_REL_DIFF = 2.0 ** -44


def lamN_sensitivity(prob, lam0, rel=2.0 ** -44, trials=3, seed=7):
    """Largest relative change of the oracle's dJ/du^N per unit relative
    perturbation of its stored states (used to set the dJ/du^N bar of the GPU
    comparison from the rounding difference of the two state sequences)."""
    U = oracle.solve_all(prob)
    _, l0 = oracle.adjoint_states(prob, U, lam0)
    rng = np.random.default_rng(seed)
    inner = (U > 0) & (U < 1)
    worst = 0.0
    for _ in range(trials):
        Up = np.where(inner, U * (1 + rel * rng.uniform(-1, 1, size=U.shape)), U)
        _, l = oracle.adjoint_states(prob, Up, lam0)
        worst = max(worst, float(np.abs(l - l0).max() / np.abs(l0).max()) / rel)
    return worst


def lamN_fp32_emulation(prob, lam0):
    """The oracle's dJ/du^N over its own states as an FP32 implementation
    holds them: every state rounded to FP32, and values whose divided
    differences' product underflows FP32's normal range in the PCHIP slope
    (|u| below sqrt(FLT_MIN) times the smallest spacing) set to zero -- the two
    ways FP32 flips the PCHIP Jacobian to its flat branch at the edge of the
    spreading solution.  Returns (relative l1 norm of the difference from the
    exact FP64 dJ/du^N, relative difference of the two l1 norms)."""
    U = oracle.solve_all(prob)
    _, l_ref = oracle.adjoint_states(prob, U, lam0)
    h = min(float(np.diff(ax.nodes).min()) for ax in prob.axes)
    tau = float(np.sqrt(np.finfo(np.float32).tiny)) * h
    U32 = U.astype(np.float32).astype(np.float64)
    U32[np.abs(U32) < tau] = 0.0
    del U
    _, l32 = oracle.adjoint_states(prob, U32, lam0)
    n_ref = float(np.abs(l_ref).sum())
    return (float(np.abs(l32 - l_ref).sum()) / n_ref,
            abs(float(np.abs(l32).sum()) - n_ref) / n_ref)
