"""Gauss-Hermite rule for the oracle (test infrastructure only).

The expectation in the scheme is an integral against the Gaussian density
rho(xi) = pi^{-m/2} exp(-|xi|^2) (paper Section 3.1.3, Eq. (expec)), evaluated
with the tensor-product Gauss-Hermite rule of Eq. (quad)/(e31).  The 1D rule is
obtained here by the Golub-Welsch method: the nodes are the eigenvalues of the
symmetric tridiagonal Jacobi matrix of the physicists' Hermite polynomials
(zero diagonal, off-diagonal sqrt(k/2), k = 1..Q*-1), and each weight is the
squared first component of the matching unit eigenvector times mu_0 = sqrt(pi).
Dividing by sqrt(pi) (the density's normalisation) leaves the squared first
components, so the weights sum to one.

Reading (the paper is silent): the exact rule is symmetric about 0, so the
computed nodes and weights are symmetrised and the middle node of an odd rule is
set to exactly 0.
"""
from __future__ import annotations

import numpy as np


def gh_rule(q: int):
    """Return (nodes a_k, weights w_k), k = 0..q-1, nodes ascending, sum(w) = 1."""
    if q < 1:
        raise ValueError("q must be >= 1")
    if q == 1:
        return np.zeros(1), np.ones(1)
    k = np.arange(1, q, dtype=np.float64)
    off = np.sqrt(k / 2.0)
    jac = np.diag(off, 1) + np.diag(off, -1)
    vals, vecs = np.linalg.eigh(jac)          # library eigen-solver as one step
    w = vecs[0, :] ** 2
    a = 0.5 * (vals - vals[::-1])
    w = 0.5 * (w + w[::-1])
    if q % 2 == 1:
        a[q // 2] = 0.0
    return np.ascontiguousarray(a), np.ascontiguousarray(w)


def tensor_rule(q: int, m: int):
    """Tensor rule in m dimensions: nodes (Q, m) and weights (Q,), Q = q**m.

    Index order is lexicographic with the last dimension fastest; the weight of
    a tensor node is the product of its 1D weights taken from dimension 0 up.
    """
    a, w = gh_rule(q)
    grids = np.meshgrid(*([np.arange(q)] * m), indexing="ij")
    idx = np.stack([g.reshape(-1) for g in grids], axis=1)
    nodes = a[idx]
    weights = np.ones(idx.shape[0])
    for i in range(m):
        weights = weights * w[idx[:, i]]
    return nodes, weights
