"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names the passage of the paper (or the mathematical fact) it pins.
A plausible slip in the oracle -- a dropped slope term, a wrong sign of the
drift, a transposed axis, the wrong time level, an unnormalised weight, a wrong
end-node rule -- fails at least one of them.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
from numpy.polynomial.hermite import hermgauss
from scipy.interpolate import PchipInterpolator

import oracle
import workloads as W
from analytic import p_exit_images, p_exit_series

# ---------------------------------------------------------------------------
# Gauss-Hermite rule (Section 3.1.3, Eq. (expec)-(quad); Remark 2)
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("q", list(range(1, 33)))
def test_gh_matches_library(q):
    a, w = oracle.gh_rule(q)
    ha, hw = hermgauss(q)
    np.testing.assert_allclose(a, ha, rtol=0, atol=2e-13 * max(1.0, np.abs(ha).max()))
    np.testing.assert_allclose(w, hw / math.sqrt(math.pi), rtol=1e-11, atol=1e-15)
    assert abs(w.sum() - 1.0) < 1e-14


@pytest.mark.parametrize("q", [1, 2, 3, 6, 8, 16])
def test_gh_gaussian_moments(q):
    """E[xi^k] under rho = pi^{-1/2} e^{-xi^2}: 0 for odd k, (k-1)!!/2^{k/2} for
    even k; the q-point rule is exact up to degree 2q-1 (Remark 2)."""
    a, w = oracle.gh_rule(q)
    for k in range(0, 2 * q):
        got = float(np.sum(w * a ** k))
        if k % 2:
            exact = 0.0
        else:
            exact = float(np.prod(np.arange(k - 1, 0, -2))) / 2 ** (k // 2) if k else 1.0
        scale = float(np.sum(w * np.abs(a) ** k))     # rounding scale of the sum
        assert abs(got - exact) <= 1e-13 * max(1.0, scale), (q, k, got, exact)


def test_gh_symmetric_and_max_nodes():
    for q, amax in [(3, 1.224745), (6, 2.350605), (8, 2.930637), (16, 4.688739)]:
        a, w = oracle.gh_rule(q)
        assert np.all(a == -a[::-1]) and np.all(w == w[::-1])
        assert abs(a.max() - amax) < 1e-6


def test_tensor_rule_weights():
    nodes, weights = oracle.tensor_rule(4, 2)
    assert nodes.shape == (16, 2)
    assert abs(weights.sum() - 1.0) < 1e-14
    # E[xi_0^2 xi_1^2] = 1/4 for the product density
    assert abs(np.sum(weights * nodes[:, 0] ** 2 * nodes[:, 1] ** 2) - 0.25) < 1e-14
    # last dimension fastest
    a, _ = oracle.gh_rule(4)
    assert nodes[1, 1] == a[1] and nodes[1, 0] == a[0]


# ---------------------------------------------------------------------------
# Cell location
# ---------------------------------------------------------------------------


def test_cell_matches_searchsorted():
    rng = np.random.default_rng(1)
    x = np.sort(rng.uniform(-1, 3, size=37))
    zs = np.concatenate([rng.uniform(-2, 4, size=2000), x, [x[0], x[-1], -5.0, 9.0]])
    for z in zs:
        ref = int(np.clip(np.searchsorted(x, z, side="right") - 1, 0, len(x) - 2))
        assert oracle.cell(x, z) == ref, z


# ---------------------------------------------------------------------------
# Cubic Hermite interpolant (Section 3.1.2) and PCHIP slopes (Eq. (e300))
# ---------------------------------------------------------------------------


def _problem_on(nodes_list, periodic=None):
    periodic = periodic or [False] * len(nodes_list)
    axes = [W.Axis(np.asarray(x), p) for x, p in zip(nodes_list, periodic)]
    return W.Problem(axes=axes, coef_kind="const", coef=(0.0,) * len(axes), D=0.1,
                     region_kind="box", gh_q=3, dt=0.01, n_steps=1)


def test_hermite_exact_on_cubics_1d():
    rng = np.random.default_rng(2)
    x = np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1, 20)]))
    p = np.polynomial.Polynomial([0.3, -1.2, 2.5, -0.7])
    prob = _problem_on([x])
    u, g = p(x), p.deriv()(x)[None, :]
    for z in rng.uniform(0, 1, 200):
        assert abs(oracle.interp(prob, u, g, [z]) - p(z)) < 1e-13
        dz = oracle.interp(prob, u, g, [z], grad=True)[0]
        assert abs(dz - p.deriv()(z)) < 1e-11


@pytest.mark.parametrize("d", [2, 3])
def test_hermite_tensor_exact_on_separable_cubics(d):
    """Values + first partials, no mixed terms: exact on sum_i p_i(x_i)."""
    rng = np.random.default_rng(3 + d)
    xs = [np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1, 6 + i)])) for i in range(d)]
    polys = [np.polynomial.Polynomial(rng.normal(size=4)) for _ in range(d)]
    prob = _problem_on(xs)
    grids = np.meshgrid(*xs, indexing="ij")
    u = sum(polys[i](grids[i]) for i in range(d))
    g = np.stack([polys[i].deriv()(grids[i]) for i in range(d)])
    for _ in range(100):
        z = rng.uniform(0, 1, d)
        exact = sum(polys[i](z[i]) for i in range(d))
        assert abs(oracle.interp(prob, u, g, z) - exact) < 1e-12
        grad = oracle.interp(prob, u, g, z, grad=True)
        for i in range(d):
            assert abs(grad[i] - polys[i].deriv()(z[i])) < 1e-10


def test_hermite_partition_and_continuity():
    """H00 + H01 = 1: constants reproduced with zero slopes; C1 across a face."""
    x = np.linspace(0, 1, 9)
    prob = _problem_on([x])
    rng = np.random.default_rng(5)
    u = rng.uniform(size=9)
    g = rng.normal(size=(1, 9))
    for k in range(1, 8):
        xl = x[k] - 1e-9
        xr = x[k] + 1e-9
        assert abs(oracle.interp(prob, u, g, [xl]) - oracle.interp(prob, u, g, [xr])) < 1e-7
        gl = oracle.interp(prob, u, g, [xl], grad=True)[0]
        gr = oracle.interp(prob, u, g, [xr], grad=True)[0]
        assert abs(gl - g[0, k]) < 1e-6 and abs(gr - g[0, k]) < 1e-6
    assert abs(oracle.interp(prob, np.full(9, 0.7), np.zeros((1, 9)), [0.33]) - 0.7) < 1e-15


def test_pchip_interior_matches_library_on_uniform_axis():
    """On a uniform axis the library PCHIP slope formula reduces to Eq. (e300)
    (harmonic mean, zero when the differences differ in sign or vanish)."""
    rng = np.random.default_rng(6)
    x = np.linspace(-1, 2, 41)
    u = np.cumsum(rng.normal(size=41)) * 0.1
    u[10:14] = u[10]          # flat run: zero differences
    prob = _problem_on([x])
    g = oracle.slopes(prob, u)[0]
    ref = PchipInterpolator(x, u).derivative()(x)
    np.testing.assert_allclose(g[1:-1], ref[1:-1], rtol=1e-12, atol=1e-14)


def test_pchip_end_nodes_follow_paper_rule():
    """End slopes substitute (delta_1, delta_2) and (delta_{J-1}, delta_{J-2})."""
    x = np.array([0.0, 0.5, 1.5, 3.0, 3.5])
    u = np.array([0.0, 1.0, 1.5, 2.5, 2.0])
    prob = _problem_on([x])
    g = oracle.slopes(prob, u)[0]
    d = np.diff(u) / np.diff(x)
    hm = lambda a, b: 0.0 if a * b <= 0 else 2.0 / (1.0 / a + 1.0 / b)
    assert abs(g[0] - hm(d[0], d[1])) < 1e-15
    assert abs(g[-1] - hm(d[-1], d[-2])) < 1e-15
    assert g[-1] == 0.0 and g[3] == 0.0      # sign change at node 3


def test_pchip_affine_exact_and_periodic_constant():
    x = np.linspace(0, 1, 11)
    y = np.linspace(-1, 1, 7)
    prob = _problem_on([x, y])
    X, Y = np.meshgrid(x, y, indexing="ij")
    g = oracle.slopes(prob, 2.0 * X - 3.0 * Y + 1.0)
    np.testing.assert_allclose(g[0], 2.0, rtol=1e-13)
    np.testing.assert_allclose(g[1], -3.0, rtol=1e-13)
    # periodic axis: sin(2 pi x) sampled with node n-1 = node 0
    xp = np.linspace(0, 1, 65)
    probp = _problem_on([xp], [True])
    u = np.sin(2 * np.pi * xp)
    gp = oracle.slopes(probp, u)[0]
    assert gp[0] == gp[-1]
    # equal one-sided differences across the seam: slope = sin(2 pi h) / h,
    # and the mirror node x = 1/2 carries the opposite slope
    hp = xp[1] - xp[0]
    assert abs(gp[0] - np.sin(2 * np.pi * hp) / hp) < 1e-12
    assert abs(gp[0] + gp[32]) < 1e-12


def test_pchip_shape_preserving():
    """Monotone data -> monotone interpolant within the data range (the paper
    relies on this to keep 0 <= u <= 1, Section 1 and 3.1.2)."""
    rng = np.random.default_rng(7)
    x = np.sort(np.concatenate([[0, 1], rng.uniform(0, 1, 30)]))
    u = np.sort(rng.uniform(size=x.size))
    prob = _problem_on([x])
    g = oracle.slopes(prob, u)
    zz = np.linspace(0, 1, 3001)
    vals = np.array([oracle.interp(prob, u, g, [z]) for z in zz])
    assert np.all(np.diff(vals) >= -1e-14)
    assert vals.min() >= u.min() - 1e-14 and vals.max() <= u.max() + 1e-14


# ---------------------------------------------------------------------------
# Whole step: translation, constants, affine fields, drift conventions
# ---------------------------------------------------------------------------


def test_translation_1d_and_2d():
    """sigma = 0 and b = (k h)/dt: the scheme shifts chi by k cells per step.
    Pins the sign of the drift, the axis order and the exit rule."""
    n0, n1, dt, N = 21, 17, 0.01, 6
    x = np.linspace(0.0, 2.0, n0)
    y = np.linspace(0.0, 1.0, n1)
    h0, h1 = x[1] - x[0], y[1] - y[0]
    k0, k1 = 1, -2
    prob = W.Problem(axes=[W.Axis(x), W.Axis(y)], coef_kind="const",
                     coef=(k0 * h0 / dt, k1 * h1 / dt), D=0.0, region_kind="box",
                     gh_q=2, dt=dt, n_steps=N)
    out = oracle.solve(prob, snaps=list(range(N + 1)))
    I0, I1 = np.meshgrid(np.arange(n0), np.arange(n1), indexing="ij")
    for n in range(N + 1):
        m = N - n
        # the walk is monotone per axis: it has exited iff it starts on a face
        # or ends on or beyond one
        start = (I0 == 0) | (I0 == n0 - 1) | (I1 == 0) | (I1 == n1 - 1)
        hit = start | (I0 + m * k0 >= n0 - 1) | (I0 + m * k0 <= 0) | \
            (I1 + m * k1 >= n1 - 1) | (I1 + m * k1 <= 0)
        np.testing.assert_allclose(out[n], hit.astype(float), atol=1e-12, err_msg=f"n={n}")
    # 1D
    p1 = W.Problem(axes=[W.Axis(x)], coef_kind="const", coef=(-h0 / dt,), D=0.0,
                   region_kind="box", gh_q=3, dt=dt, n_steps=N)
    o1 = oracle.solve(p1, snaps=[0])[0]
    i0 = np.arange(n0)
    np.testing.assert_allclose(o1, ((i0 - N <= 0) | (i0 == n0 - 1)).astype(float), atol=1e-12)


@pytest.mark.parametrize("which", ["cell", "abc"])
def test_constant_one_preserved(which):
    if which == "cell":
        prob = W.cell2d(nx=41, ny=21, n_steps=3)
    else:
        prob = W.abc3d(n=13, n_steps=3, D=2e-3)
    u = oracle.step(prob, 1, np.ones(prob.shape))
    np.testing.assert_allclose(u, 1.0, atol=1e-14)


def test_affine_field_moves_with_drift_only():
    """Symmetric GH nodes + exact PCHIP on affine data: one step maps
    u = alpha + beta.x to alpha + beta.(x + b dt) at nodes whose landing points
    stay inside the box (Eq. (e31) with E[xi] = 0)."""
    x = np.linspace(0, 4, 41)
    y = np.linspace(0, 2, 21)
    b = (0.7, -0.4)
    dt = 0.02
    prob = W.Problem(axes=[W.Axis(x), W.Axis(y)], coef_kind="const", coef=b, D=0.05,
                     region_kind="box", gh_q=4, dt=dt, n_steps=1)
    X, Y = np.meshgrid(x, y, indexing="ij")
    u1 = 0.2 + 0.1 * X - 0.3 * Y
    u0 = oracle.step(prob, 0, u1)
    inner = (slice(8, -8), slice(6, -6))
    expect = 0.2 + 0.1 * (X + b[0] * dt) - 0.3 * (Y + b[1] * dt)
    np.testing.assert_allclose(u0[inner], expect[inner], atol=1e-14)


def _psi_cell(x, y, t, A, eps, om):
    return A * np.sin(np.pi * (x + eps * np.sin(om * t))) * np.sin(np.pi * y)


def test_cellular_drift_is_rotated_stream_gradient_at_t_n():
    """Affine state => u^n - u^{n+1} = dt * beta . b(t_n, x_j).  b is obtained
    here by central differences of the stream function psi of the workload,
    with b = (-dpsi/dy, dpsi/dx) (the paper's sign convention, Section 4.2),
    evaluated at the left end t_n of the step."""
    A, eps, om = 1.3, 0.25, 9.0
    dt, n = 0.01, 7
    prob = W.cell2d(nx=81, ny=41, A=A, eps=eps, omega=om, D=1e-4, dt=dt,
                    n_steps=10, radius=0.45)
    x, y = prob.axes[0].nodes, prob.axes[1].nodes
    X, Y = np.meshgrid(x, y, indexing="ij")
    beta = (0.6, -0.9)
    u1 = beta[0] * X + beta[1] * Y
    u0 = oracle.step(prob, n, u1)
    t = n * dt
    hh = 1e-6
    bx = -(_psi_cell(X, Y + hh, t, A, eps, om) - _psi_cell(X, Y - hh, t, A, eps, om)) / (2 * hh)
    by = (_psi_cell(X + hh, Y, t, A, eps, om) - _psi_cell(X - hh, Y, t, A, eps, om)) / (2 * hh)
    cls = oracle.node_class(prob)
    # nodes well inside the disc (no landing point exits)
    r = np.hypot(X - 0.5, Y - 0.5)
    sel = (cls == 0) & (r < 0.35)
    got = (u0 - u1)[sel] / dt
    want = beta[0] * bx[sel] + beta[1] * by[sel]
    np.testing.assert_allclose(got, want, atol=1e-6)
    # a one-step shift of the time level would be visible at this omega
    t1 = (n + 1) * dt
    bx1 = -(_psi_cell(X, Y + hh, t1, A, eps, om) - _psi_cell(X, Y - hh, t1, A, eps, om)) / (2 * hh)
    assert np.abs(beta[0] * (bx1 - bx)[sel]).max() > 1e-3


def _psi_rolls(x1, x2, t, eps, om, n):
    return np.sin(np.pi * x2) * (np.sin(n * x1) + eps * np.cos(om * t) * np.cos(n * x1))


def test_paper2d_drift_is_roll_flow_of_stream_function():
    """Section 4.2: Pe v with v = (-dpsi/dx2, dpsi/dx1) for the roll stream
    function psi = sin(pi x2) (sin(n x1) + eps cos(omega t) cos(n x1)) (the
    printed v_1, v_2 are its derivatives, so v is divergence-free); at
    eps = 0 the elliptic points (+-pi/4, 1/2), (+-3pi/4, 1/2) and the hyperbolic
    points (0, 0), (+-pi/2, 0), (pi, 1) are stagnation points."""
    Pe, eps, om, n = 10.0, 0.15, 2 * math.pi / 10, 2
    prob = W.paper2d(Pe=Pe, eps=eps, omega=om, n=n)
    rng = np.random.default_rng(9)
    hh = 1e-6
    for _ in range(25):
        x1, x2 = float(rng.uniform(-math.pi, math.pi)), float(rng.uniform(0, 1))
        t = float(rng.uniform(0, 10))
        b = oracle.drift(prob, t, [x1, x2])
        d1 = (_psi_rolls(x1 + hh, x2, t, eps, om, n) - _psi_rolls(x1 - hh, x2, t, eps, om, n)) / (2 * hh)
        d2 = (_psi_rolls(x1, x2 + hh, t, eps, om, n) - _psi_rolls(x1, x2 - hh, t, eps, om, n)) / (2 * hh)
        np.testing.assert_allclose(b, [-Pe * d2, Pe * d1], atol=1e-7)
    still = W.paper2d(eps=0.0)
    for pt in [(math.pi / 4, 0.5), (-math.pi / 4, 0.5), (3 * math.pi / 4, 0.5),
               (-3 * math.pi / 4, 0.5), (0.0, 0.0), (math.pi / 2, 0.0), (-math.pi / 2, 0.0),
               (math.pi, 1.0)]:
        assert np.abs(oracle.drift(still, 1.0, list(pt))).max() < 1e-12, pt
    assert oracle.num_theta(prob) == 4


def test_paper2d_exit_probability_low_in_roll_cores():
    """The result stated for Fig. ex2:f1: with the time-dependent perturbation
    the exit probability at T_max is small at the elliptic points (the roll
    cores) and large near the separatrices, where the flow carries tracers
    to the walls x2 = 0, 1.  Bounds hold (box exit: exit nodes at 1)."""
    prob = W.paper2d()
    u0 = oracle.solve(prob, snaps=[0])[0]
    x1, x2 = prob.axes[0].nodes, prob.axes[1].nodes
    mid = int(np.argmin(np.abs(x2 - 0.5)))
    def at(v):
        return u0[int(np.argmin(np.abs(x1 - v))), mid]
    cores = [at(v) for v in (-3 * math.pi / 4, -math.pi / 4, math.pi / 4, 3 * math.pi / 4)]
    seps = [at(v) for v in (-math.pi / 2, 0.0, math.pi / 2)]
    assert max(cores) < 0.5 * min(seps), (cores, seps)
    assert u0.min() >= -1e-3 and u0.max() <= 1 + 1e-12
    assert np.all(u0[:, 0] == 1.0) and np.all(u0[:, -1] == 1.0)
    # periodic in x1: the image column equals the first
    assert np.array_equal(u0[0], u0[-1])


def test_abc_drift_is_beltrami_and_modulated():
    """The ABC field satisfies curl v = v and div v = 0; the modulation
    multiplies it by 1 + amp sin t."""
    prob = W.abc3d(n=9, A=1.0, B=0.8, C=0.6, amp=0.1)
    rng = np.random.default_rng(8)
    hh = 1e-5
    for _ in range(20):
        p = rng.uniform(-3, 3, 3)
        t = float(rng.uniform(0, 5))
        f = 1.0 + 0.1 * math.sin(t)
        v = oracle.drift(prob, t, p)
        J = np.zeros((3, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = hh
            J[:, k] = (oracle.drift(prob, t, p + e) - oracle.drift(prob, t, p - e)) / (2 * hh)
        curl = np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])
        np.testing.assert_allclose(curl, v, atol=1e-8)
        assert abs(np.trace(J)) < 1e-8
        v0 = oracle.drift(prob, 0.0, p)
        np.testing.assert_allclose(v, f * v0, rtol=1e-13, atol=1e-15)


def test_diffusion_scale_from_quadratic():
    """For u = x^2 on an interior window the expectation adds
    E[(S a)^2] = S^2/2 with S = sqrt(2D) sqrt(2 dt), i.e. 2 D dt: pins the
    sqrt(2 dt) factor of Eq. (e31) and sigma = sqrt(2D).  PCHIP slopes are
    not exact on x^2, so a fine grid and a loose tolerance are used."""
    x = np.linspace(-1, 1, 4001)
    D, dt = 0.3, 1e-3
    prob = W.Problem(axes=[W.Axis(x)], coef_kind="const", coef=(0.0,), D=D,
                     region_kind="box", gh_q=4, dt=dt, n_steps=1)
    u1 = x ** 2
    u0 = oracle.step(prob, 0, u1)
    mid = slice(1500, 2500)
    np.testing.assert_allclose((u0 - u1)[mid], 2 * D * dt, rtol=2e-3)


def test_periodic_axis_wraps():
    """Pure translation across a periodic seam: a bump moves around the
    circle and comes back."""
    n, dt = 33, 0.01
    x = np.linspace(0, 1, n)
    h = x[1] - x[0]
    z = np.linspace(-1, 1, 9)
    prob = W.Problem(axes=[W.Axis(x, True), W.Axis(z)], coef_kind="const",
                     coef=(3 * h / dt, 0.0), D=0.0, region_kind="box", gh_q=2,
                     dt=dt, n_steps=1)
    rng = np.random.default_rng(9)
    u = rng.uniform(size=(n, 9))
    u[-1] = u[0]
    u1 = oracle.step(prob, 0, u)
    inner = slice(1, -1)
    for i in range(n - 1):
        np.testing.assert_allclose(u1[i, inner], u[(i + 3) % (n - 1), inner], atol=1e-12)
    np.testing.assert_allclose(u1[-1], u1[0], atol=0)


# ---------------------------------------------------------------------------
# Whole scheme against the closed form (Section 4.1)
# ---------------------------------------------------------------------------


def test_series_forms_agree():
    xs = np.linspace(0.05, 1.95, 39)
    for T in (0.01, 0.1, 0.5, 1.0, 3.0):
        np.testing.assert_allclose(p_exit_series(T, xs, 2.0), p_exit_images(T, xs, 2.0),
                                   atol=1e-12)
    # survey-quoted reference values at the centre of (-1, 1)
    assert abs(p_exit_series(1.0, 1.0, 2.0) - 0.629222570200) < 1e-11


def remark2_grid(L, h, dt, sigma, q):
    """Uniform interior spacing h; first and last cells of width
    sigma sqrt(2 dt) max|a| so that every landing point of an interior node
    stays in the closed domain (Remark 2, with b = 0)."""
    a, _ = oracle.gh_rule(q)
    hb = sigma * math.sqrt(2 * dt) * np.abs(a).max()
    m = max(1, int(round((L - 2 * hb) / h)))
    inner = np.linspace(hb, L - hb, m + 1)
    return np.concatenate([[0.0], inner, [L]])


def test_bm_first_order_in_dt_on_remark2_grid():
    """Paper Fig. ex3:f2 setting: X = X0 + W on [0, 10], T = 3, 3-point rule,
    PCHIP, Assumption 1 enforced: error O(dt)."""
    L, T, q = 10.0, 3.0, 3
    errs, dts = [], [0.2, 0.1, 0.05, 0.025]
    for dt in dts:
        x = remark2_grid(L, 0.02, dt, 1.0, q)
        prob = W.Problem(axes=[W.Axis(x)], coef_kind="const", coef=(0.0,), D=0.5,
                         region_kind="box", gh_q=q, dt=dt, n_steps=int(round(T / dt)))
        u0 = oracle.solve(prob, snaps=[0])[0]
        errs.append(np.abs(u0 - p_exit_series(T, x, L)).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 0.8), (errs, rates)
    assert errs[-1] < 0.01


def test_bm1d_workload_vs_series_and_bounds():
    """bm1d violates Assumption 1 (a landing point reaches 66 cells), so the
    discrete-monitoring bias is visible; loose gate on u^0, strict bounds."""
    prob = W.bm1d()
    snaps = list(range(0, 101, 10))
    out = oracle.solve(prob, snaps=snaps)
    x = prob.axes[0].nodes
    u0 = out[0]
    ser = p_exit_series(1.0, x + 1.0, 2.0)
    assert np.abs(u0 - ser).max() < 0.1
    assert out.min() >= -1e-14 and out.max() <= 1 + 1e-14
    # horizon monotonicity (autonomous): u^n >= u^{n+1}
    for a, b in zip(out[:-1], out[1:]):
        assert np.all(a >= b - 1e-12)


def test_bm1d_matches_discrete_chain_monte_carlo():
    """The scheme computes E over one Euler step per time step with exit checked
    at step ends; a Monte Carlo run of that chain must agree within sampling
    error plus the quadrature/interpolation error of the scheme."""
    prob = W.bm1d()
    u0 = oracle.solve(prob, snaps=[0])[0]
    x = prob.axes[0].nodes
    rng = np.random.default_rng(10)
    sig_sqdt = math.sqrt(2 * prob.D * prob.dt)
    for j in (100, 150, 190):
        n_paths = 400_000
        pos = np.full(n_paths, x[j])
        alive = np.ones(n_paths, dtype=bool)
        for _ in range(prob.n_steps):
            pos[alive] += sig_sqdt * rng.standard_normal(alive.sum())
            alive &= (pos > -1.0) & (pos < 1.0)
        p_mc = 1.0 - alive.mean()
        se = math.sqrt(max(p_mc * (1 - p_mc), 1e-12) / n_paths)
        assert abs(u0[j] - p_mc) < 5 * se + 4e-3, (j, u0[j], p_mc, se)


def _one_step_error(m, f):
    """RMS error of one step on smooth data f against the exact Gauss-Hermite
    expectation of f itself (library rule), at nodes whose landing points stay
    inside the disc: isolates the interpolation error of Section 3.1.2.  The
    drift is the cellular flow, taken from central differences of its stream
    function, so that the in-cell positions of landing points spread."""
    prob = W.cell2d(nx=32 * m + 1, ny=16 * m + 1, D=2e-3, dt=5e-3, n_steps=4,
                    radius=0.45, gh_q=4)
    x, y = prob.axes[0].nodes, prob.axes[1].nodes
    X, Y = np.meshgrid(x, y, indexing="ij")
    n = 2
    u0 = oracle.step(prob, n, f(X, Y))
    a, w = hermgauss(4)
    w = w / math.sqrt(math.pi)
    S = math.sqrt(2 * prob.D) * math.sqrt(2 * prob.dt)
    A, eps, om = prob.coef
    t, hh = n * prob.dt, 1e-6
    bx = -(_psi_cell(X, Y + hh, t, A, eps, om) - _psi_cell(X, Y - hh, t, A, eps, om)) / (2 * hh)
    by = (_psi_cell(X + hh, Y, t, A, eps, om) - _psi_cell(X - hh, Y, t, A, eps, om)) / (2 * hh)
    ex = np.zeros_like(X)
    for i in range(4):
        for k in range(4):
            ex += w[i] * w[k] * f(X + bx * prob.dt + S * a[i], Y + by * prob.dt + S * a[k])
    sel = np.hypot(X - 0.5, Y - 0.5) < 0.35
    return math.sqrt(np.mean((u0 - ex)[sel] ** 2))


@pytest.mark.parametrize("name", ["exp", "separable", "trig"])
def test_second_order_in_space_one_step(name):
    """Second order in dx (Section 3.1.4, Eq. (e_err)): the one-step error on
    smooth data falls at least like h^2.  The tensor interpolant without mixed
    (twist) terms has an h_x h_y f_xy error with zero cell mean, so the
    constant oscillates; the gates are the overall order and a bound on
    err / h^2."""
    f = {"exp": lambda X, Y: np.exp(0.5 * X + 0.3 * Y),
         "separable": lambda X, Y: np.exp(0.5 * X) + np.sin(3 * Y),
         "trig": lambda X, Y: np.sin(3 * X) * np.cos(2 * Y) + 0.5 * X * Y}[name]
    ms = [1, 2, 4, 8]
    errs = [_one_step_error(m, f) for m in ms]
    for m, e in zip(ms[1:], errs[1:]):
        assert e * m * m <= 2.0 * errs[0], errs
    assert math.log2(errs[0] / errs[-1]) / 3 >= 1.8, errs


def test_stability_large_dt():
    """Unconditional stability (Section 3.1.4): dt far beyond any CFL limit
    keeps u bounded in 1D."""
    prob = W.bm1d(dt=0.5, n_steps=40)
    out = oracle.solve(prob, snaps=[0, 20, 40])
    assert np.isfinite(out).all()
    assert out.min() >= -1e-12 and out.max() <= 1 + 1e-12


# ---------------------------------------------------------------------------
# Matrix form (Eq. (e34)-(e36)) and adjoint
# ---------------------------------------------------------------------------


def test_dense_row_reproduces_step():
    prob = W.cell2d(nx=33, ny=17, n_steps=4, D=5e-3, radius=0.4)
    rng = np.random.default_rng(11)
    u = rng.uniform(size=prob.shape)
    u0 = oracle.step(prob, 2, u)
    g = oracle.slopes(prob, u)
    vec = np.concatenate([u.reshape(1, -1), g.reshape(2, -1)])
    act = oracle.active_nodes(prob)
    for j in act[:: max(1, len(act) // 25)]:
        row, em = oracle.assemble_row(prob, 2, int(j))
        assert abs(em + np.sum(row * vec) - u0.reshape(-1)[j]) < 1e-13


def _fd_grad(prob, k, h, rec, lam):
    """Central difference of <lam, u^0> in theta_k = (differentiable drift
    parameters..., D), exit classification frozen."""
    coef = list(prob.coef)
    n_drift = W.N_DRIFT_PARAMS[prob.coef_kind] or prob.d
    D = prob.D
    vals = []
    for sgn in (+1, -1):
        c2, D2 = list(coef), D
        if k < n_drift:
            c2[k] = coef[k] + sgn * h * max(1.0, abs(coef[k]))
        else:
            D2 = D + sgn * h * D
        u0 = oracle.solve(prob, snaps=[0], frozen_exits=rec, coef=c2, D=D2)[0]
        vals.append(float(np.sum(lam * u0)))
    step = h * (max(1.0, abs(coef[k])) if k < n_drift else D)
    return (vals[0] - vals[1]) / (2 * step)


@pytest.mark.parametrize("which", ["cell", "const1d", "abc", "rolls"])
def test_adjoint_matches_central_differences(which):
    """Frozen exit classification, central differences with h = 1e-6."""
    if which == "cell":
        prob = W.cell2d(nx=49, ny=25, n_steps=12, dt=2e-3, D=2e-3, A=1.1, eps=0.2, omega=5.0)
    elif which == "rolls":
        prob = W.paper2d(n1=41, n2=17, dt=2e-3, T=0.024, eps=0.4, omega=30.0, gh_q=4)
    elif which == "const1d":
        prob = W.Problem(axes=[W.uniform_axis(-1, 1, 41)], coef_kind="const", coef=(0.3,),
                         D=0.2, region_kind="box", gh_q=5, dt=0.01, n_steps=15)
    else:
        prob = W.abc3d(n=11, n_steps=4, dt=0.05, D=3e-3)
    _, rec = oracle.solve(prob, snaps=[0], record_exits=True)
    rng = np.random.default_rng(12)
    lam = rng.uniform(size=prob.shape)
    grad, _ = oracle.adjoint(prob, lam, frozen_exits=rec)
    for k in range(len(grad)):
        fd = _fd_grad(prob, k, 1e-6, rec, lam)
        scale = max(abs(fd), 1e-8 * np.abs(lam).sum())
        assert abs(grad[k] - fd) <= 1e-5 * scale + 1e-9, (k, grad[k], fd)


def _amplification(prob, n_from, n_to, eps=1e-9, seed=0):
    base = oracle.solve(prob, snaps=[n_from, n_to])
    cls = oracle.node_class(prob)
    rng = np.random.default_rng(seed)
    u = base[0] + eps * rng.standard_normal(prob.shape) * (cls == 0)
    for n in range(n_from - 1, n_to - 1, -1):
        u = oracle.step(prob, n, u)
    return float(np.abs(u - base[1]).max()) / eps


def test_conditioning_depends_on_resolution():
    """The scheme (tensor Hermite interpolant with PCHIP slopes) amplifies a
    perturbation of the state strongly when diffusion is far below the grid
    scale (seeded batch instance 16: 129x65, D = 1.25e-4), and damps it on the
    resolved 513x257 workload.  Any rounding (FP32 apply: ~6e-8) is amplified the
    same way, which bounds the attainable FP32 accuracy on such instances."""
    coarse = W.cell2d_batch()[16].replace(n_steps=1000)
    assert coarse.shape == (129, 65)
    a_coarse = _amplification(coarse, 1000, 900)
    fine = W.cell2d(n_steps=100)
    a_fine = _amplification(fine, 100, 0)
    print(a_coarse, a_fine)
    assert a_coarse > 1e3
    assert a_fine < 1.0


def test_adjoint_translation_equivariant_in_flat_rows():
    """Box exit, constant drift: away from the x faces every row of u^n along x
    is the same function of y, so the adjoint of a point source shifted by one
    row along x is the shifted adjoint.  Rows that are equal up to rounding
    make the PCHIP slope's divided differences vanish; the linearisation must
    treat them as flat (derivative 0) whatever their last bits, else a spurious
    O(1) jump appears between neighbouring rows."""
    prob = W.Problem(axes=[W.uniform_axis(0, 1, 37), W.uniform_axis(0, 2, 71)],
                     coef_kind="const", coef=(0.4, -0.7), D=0.01, region_kind="box",
                     gh_q=5, dt=0.01, n_steps=3)
    outs = []
    for i in (12, 13):
        lam0 = np.zeros(prob.shape)
        lam0[i, 2] = 1.0
        outs.append(oracle.adjoint(prob, lam0)[1])
    a, b = outs
    assert np.abs(a[8:26, :] - b[9:27, :]).max() <= 1e-12 * np.abs(a).max()


def test_full_size_cell2d_adjoint_fixture_matches_frozen_central_differences():
    """The stored 2000-step oracle adjoint of the 513x257 cellular flow
    (tests/golden/make_cell2d_adj.py) against the stored central differences
    with the exit classification frozen (relative step 1e-6): the adjoint is
    the derivative of the scheme with exits held fixed.  The differences with
    exits recomputed are stored beside them; a landing point that changes side
    within +-h switches its value to 1, so they need not agree."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "cell2d_adj_oracle.json")
    with open(path) as f:
        ref = json.load(f)
    prob = W.cell2d_adj()
    assert tuple(ref["problem"][k] for k in ("nx", "ny")) == prob.shape
    assert ref["problem"]["dt"] == prob.dt and ref["problem"]["n_steps"] == prob.n_steps
    assert ref["problem"]["coef"] == list(prob.coef) and ref["problem"]["D"] == prob.D
    g, fd = np.array(ref["grad"]), np.array(ref["fd_frozen_exits"])
    assert np.all(np.abs(g - fd) <= 1e-5 * np.abs(fd) + 1e-12), (g, fd)
    assert 0.0 < ref["J0"] < 1.0


def test_adjoint_taylor_remainder_is_second_order():
    """With the exit classification frozen, J(theta + h e) - J(theta) - h <grad, e>
    falls like h^2 along a mixed direction of all four parameters: a wrong or
    dropped gradient term leaves an O(h) remainder (a factor 10 per decade)."""
    prob = W.cell2d(nx=49, ny=25, n_steps=12, dt=2e-3, D=2e-3, A=1.1, eps=0.2, omega=5.0)
    _, rec = oracle.solve(prob, snaps=[0], record_exits=True)
    lam = np.random.default_rng(13).uniform(size=prob.shape)
    grad, _ = oracle.adjoint(prob, lam, frozen_exits=rec)
    theta = np.array(list(prob.coef) + [prob.D])
    e = np.array([0.3, -0.5, 0.7, 0.4]) * theta

    def J(t):
        u0 = oracle.solve(prob, snaps=[0], frozen_exits=rec, coef=list(t[:3]), D=t[3])[0]
        return float(np.sum(lam * u0))

    J0 = J(theta)
    R = [abs(J(theta + h * e) - J0 - h * float(np.dot(grad, e))) for h in (1e-2, 1e-3, 1e-4)]
    assert 70 < R[0] / R[1] < 130 and 70 < R[1] / R[2] < 130, R


# ---------------------------------------------------------------------------
# Disc (ball) exit region (Section 2: exit region and exit time; a disc target
# inside the grid box)
# ---------------------------------------------------------------------------

# an off-centre disc (centre not on the diagonal, so that swapped centre
# coordinates change the region) on a rectangular grid
DISC_C = (0.63, 0.41)
DISC_R = 0.29


def _disc_problem(n0=61, n1=37, **kw):
    base = dict(axes=[W.uniform_axis(0.0, 2.0, n0), W.uniform_axis(0.0, 1.0, n1)],
                coef_kind="const", coef=(0.0, 0.0), D=0.0, region_kind="ball",
                center=DISC_C + (0.0,), radius=DISC_R, gh_q=2, dt=0.01, n_steps=1)
    base.update(kw)
    return W.Problem(**base)


def _disc_exit_mask(X, Y, c, r, box):
    """Exit region from numpy's hypot (a different formula from the squared
    distance the scheme compares) and the box faces."""
    (x0, x1), (y0, y1) = box
    return (np.hypot(X - c[0], Y - c[1]) >= r) | (X <= x0) | (X >= x1) | (Y <= y0) | (Y >= y1)


def test_disc_node_classes_match_hypot_mask():
    """Exit nodes of a disc target are the nodes at distance >= r from the
    centre (or on a face of the box); no node of this grid lies within 1e-6 of
    the circle, so the two formulas must agree exactly."""
    prob = _disc_problem()
    x, y = prob.axes[0].nodes, prob.axes[1].nodes
    X, Y = np.meshgrid(x, y, indexing="ij")
    dist = np.hypot(X - DISC_C[0], Y - DISC_C[1])
    assert np.abs(dist - DISC_R).min() > 1e-6
    expect = _disc_exit_mask(X, Y, DISC_C, DISC_R, ((0.0, 2.0), (0.0, 1.0)))
    cls = oracle.node_class(prob)
    assert np.array_equal(cls == 1, expect)
    assert np.array_equal(cls == 0, ~expect)
    # chi is 1 exactly on the exit nodes
    assert np.array_equal(oracle.chi(prob), expect.astype(float))
    # the point test on off-grid points around the circle
    rng = np.random.default_rng(3)
    ang = rng.uniform(0, 2 * np.pi, 400)
    rad = DISC_R * (1.0 + rng.choice([-1, 1], 400) * rng.uniform(1e-6, 0.2, 400))
    for a, rr in zip(ang, rad):
        z = (DISC_C[0] + rr * np.cos(a), DISC_C[1] + rr * np.sin(a))
        assert oracle.is_exit_point(prob, z) == (rr >= DISC_R), (z, rr)


def test_disc_translation_exits_exactly():
    """sigma = 0 and b = (k0 h0, k1 h1)/dt: every landing point is a grid node,
    shifted by (k0, k1) nodes per step, so u^n_j = 1 exactly when the walk
    j + m (k0, k1), m = 0 .. N - n, meets an exit node (of the disc or of the
    box) -- with the exit region taken from numpy's hypot, not the scheme."""
    n0, n1, dt, N = 61, 37, 0.01, 7
    x = np.linspace(0.0, 2.0, n0)
    y = np.linspace(0.0, 1.0, n1)
    h0, h1 = x[1] - x[0], y[1] - y[0]
    for k0, k1 in ((1, 0), (0, -1), (2, 1), (-1, 2)):
        prob = _disc_problem(coef=(k0 * h0 / dt, k1 * h1 / dt), dt=dt, n_steps=N, gh_q=3)
        out = oracle.solve(prob, snaps=list(range(N + 1)))
        I0, I1 = np.meshgrid(np.arange(n0), np.arange(n1), indexing="ij")
        for n in range(N + 1):
            hit = np.zeros((n0, n1), dtype=bool)
            for m in range(N - n + 1):
                J0, J1 = I0 + m * k0, I1 + m * k1
                off = (J0 <= 0) | (J0 >= n0 - 1) | (J1 <= 0) | (J1 >= n1 - 1)
                Jc0, Jc1 = np.clip(J0, 0, n0 - 1), np.clip(J1, 0, n1 - 1)
                inside_exit = _disc_exit_mask(x[Jc0], y[Jc1], DISC_C, DISC_R,
                                              ((0.0, 2.0), (0.0, 1.0)))
                hit |= off | inside_exit
            np.testing.assert_allclose(out[n], hit.astype(float), atol=1e-12,
                                       err_msg=f"shift ({k0},{k1}) n={n}")


def _disc_survival_bessel(T, D, R, K=200):
    """Probability that sqrt(2 D) W started at the centre of a disc of radius
    R has not left it by T: sum_k 2 / (j_k J1(j_k)) exp(-j_k^2 D T / R^2), j_k
    the zeros of J0 (heat equation in the disc, radial eigenfunctions)."""
    from scipy.special import j1, jn_zeros
    j = jn_zeros(0, K)
    return float(np.sum(2.0 / (j * j1(j)) * np.exp(-j * j * D * T / R ** 2)))


def test_disc_exit_from_centre_vs_bessel_series():
    """Zero drift, exit from a disc (r = 0.3) of the unit square, started at
    the centre: the scheme against the closed-form exit probability.  The
    scheme monitors exits at step ends only, which biases it low by about the
    Broadie-Glasserman-Kou shift of the boundary, 0.5826 sigma sqrt(dt); with
    the radius shifted by that amount the series agrees to a few 1e-3, and the
    plain-series gap shrinks with dt."""
    R, D, T = 0.3, 0.02, 0.4
    sig = math.sqrt(2 * D)
    gaps, gaps_bgk = [], []
    for dt in (0.004, 0.001):
        N = int(round(T / dt))
        prob = W.Problem(axes=[W.uniform_axis(0, 1, 129), W.uniform_axis(0, 1, 129)],
                         coef_kind="const", coef=(0.0, 0.0), D=D, region_kind="ball",
                         center=(0.5, 0.5, 0.0), radius=R, gh_q=8, dt=dt, n_steps=N)
        u0 = oracle.solve(prob, snaps=[0])[0]
        pc = u0[64, 64]
        gaps.append(pc - (1.0 - _disc_survival_bessel(T, D, R)))
        gaps_bgk.append(pc - (1.0 - _disc_survival_bessel(T, D, R + 0.5826 * sig * math.sqrt(dt))))
    print("plain", gaps, "shifted", gaps_bgk)
    assert -0.015 < gaps[0] < 0 and -0.008 < gaps[1] < 0 and abs(gaps[1]) < 0.6 * abs(gaps[0])
    assert all(abs(g) < 0.006 for g in gaps_bgk)


def test_disc_exit_matches_discrete_chain_monte_carlo():
    """Zero drift, off-centre disc: Monte Carlo of the chain the scheme
    discretises (Gaussian steps, exit checked at step ends) from four nodes
    near the circle.  The interpolant of u^{n+1} in cells cut by the circle
    mixes inside values with the exit nodes' 1, an O(h) effect that shrinks
    under refinement; at h = 1/200 the gap is within 0.015."""
    c, r = (0.46, 0.55), 0.31
    D, dt, N = 0.01, 0.004, 50
    pts = [(0.62, 0.54), (0.46, 0.80), (0.24, 0.52), (0.46, 0.28)]
    rng = np.random.default_rng(11)
    s = math.sqrt(2 * D * dt)
    mc = []
    for px, py in pts:
        npth = 300_000
        pos = np.empty((npth, 2))
        pos[:, 0], pos[:, 1] = px, py
        alive = np.ones(npth, dtype=bool)
        for _ in range(N):
            pos[alive] += s * rng.standard_normal((int(alive.sum()), 2))
            alive &= np.hypot(pos[:, 0] - c[0], pos[:, 1] - c[1]) < r
        p = 1.0 - alive.mean()
        mc.append((p, math.sqrt(max(p * (1 - p), 1e-12) / npth)))
    worst = {}
    for n in (51, 201):
        prob = W.Problem(axes=[W.uniform_axis(0, 1, n), W.uniform_axis(0, 1, n)],
                         coef_kind="const", coef=(0.0, 0.0), D=D, region_kind="ball",
                         center=c + (0.0,), radius=r, gh_q=8, dt=dt, n_steps=N)
        u0 = oracle.solve(prob, snaps=[0])[0]
        errs = []
        for (px, py), (p, se) in zip(pts, mc):
            i, j = int(round(px * (n - 1))), int(round(py * (n - 1)))
            errs.append(abs(u0[i, j] - p) - 5 * se)
        worst[n] = max(errs)
    print(worst)
    assert worst[201] < 0.015 and worst[201] < worst[51] / 3


# ---------------------------------------------------------------------------
# Linearisation of the PCHIP slope at its kinks (adjoint)
# ---------------------------------------------------------------------------


def _box2d_adjoint_case():
    prob = W.Problem(axes=[W.uniform_axis(0, 1, 37), W.uniform_axis(0, 2, 71)],
                     coef_kind="const", coef=(0.4, -0.7), D=0.01, region_kind="box",
                     gh_q=5, dt=0.01, n_steps=9)
    lam0 = np.random.default_rng(21).uniform(size=prob.shape)
    return prob, lam0


def test_flat_rule_theta_gradient_independent_of_threshold():
    """The slope 2ab/(a+b) has a kink where a divided difference vanishes; the
    adjoint takes derivative 0 at differences below a relative threshold of
    the values (2^-30).  On the box case, whose rows along x are equal up to
    a factor that decays continuously away from the x faces (relative
    differences of neighbours at every scale from 2^-52 up), the parameter
    gradient does not depend on the threshold: 2^-20 .. 2^-44 and exact
    equality give the same gradient within 1e-7."""
    prob, lam0 = _box2d_adjoint_case()
    U = oracle.solve_all(prob)
    g0, _ = oracle.adjoint_states(prob, U, lam0)
    for e in (20, 24, 28, 34, 40, 44, None):
        with oracle.flat_rel(0.0 if e is None else 2.0 ** -e):
            g, _ = oracle.adjoint_states(prob, U, lam0)
        assert np.abs(g - g0).max() <= 1e-7 * np.abs(g0).max(), (e, g, g0)


def test_flat_rule_makes_lamN_a_smooth_function_of_the_states():
    """With the rule, dJ/du^N responds linearly to a perturbation of the
    stored states (relative size 2^-52 .. 2^-40, slope below 2e5); without it
    (exact equality only), a 1-ulp perturbation flips Jacobian branches of
    rows that are flat up to rounding and moves dJ/du^N by more than 1e-3 of
    its size.  The slope bounds the dJ/du^N difference between two correct
    implementations whose states differ by their rounding."""
    prob, lam0 = _box2d_adjoint_case()
    U = oracle.solve_all(prob)
    _, l0 = oracle.adjoint_states(prob, U, lam0)
    rng = np.random.default_rng(7)
    inner = (U > 0) & (U < 1)
    for rel in (2.0 ** -52, 2.0 ** -46, 2.0 ** -40):
        Up = np.where(inner, U * (1 + rel * rng.uniform(-1, 1, size=U.shape)), U)
        _, l = oracle.adjoint_states(prob, Up, lam0)
        assert np.abs(l - l0).max() <= 2e5 * rel * np.abs(l0).max(), rel
    with oracle.flat_rel(0.0):
        _, lr = oracle.adjoint_states(prob, U, lam0)
        worst = 0.0
        for _ in range(3):
            up = rng.integers(0, 2, size=U.shape) == 1
            Up = np.where(inner, np.where(up, np.nextafter(U, 2.0), np.nextafter(U, -1.0)), U)
            _, l = oracle.adjoint_states(prob, Up, lam0)
            worst = max(worst, float(np.abs(l - lr).max() / np.abs(lr).max()))
    assert worst > 1e-3, worst


# ---------------------------------------------------------------------------
# Algorithm 1 (Section 3.2): several horizons in one backward sweep
# ---------------------------------------------------------------------------

def test_algorithm1_columns_are_the_products_of_eq_e37():
    """Column m of Algorithm 1 is p^m of Eq. (e37): the product of the step
    operators with coefficients at t0 + (m-1) dt, .., t0 applied to chi.  Two
    other routes to the same product: a Scheme-1 pass of N = m steps (same
    arithmetic, bitwise), and one pass of N = M steps started at
    t0 - (M - m) dt, whose state u^{M-m} has met the same coefficient times
    (up to the rounding of the shifted times).  For this time-dependent flow
    u^{M-m} of an unshifted pass is a different quantity (reading 12)."""
    prob = W.cell2d(nx=49, ny=25, n_steps=30, D=2e-3, omega=7.0, eps=0.25)
    hz = [7, 30, 18, 1, 18]
    cols = oracle.solve_horizons(prob, hz)
    M = max(hz)
    one = oracle.solve(prob.replace(n_steps=M), snaps=[M - m for m in hz])
    for h, m in enumerate(hz):
        sep = oracle.solve(prob.replace(n_steps=m), snaps=[0])[0]
        assert np.array_equal(cols[h], sep), m
        shifted = prob.replace(n_steps=M, t0=prob.t0 - (M - m) * prob.dt)
        s = oracle.solve(shifted, snaps=[M - m])[0]
        assert np.abs(cols[h] - s).max() <= 1e-13, m
        if m < M:
            assert np.abs(cols[h] - one[h]).max() > 1e-3, m
    assert np.array_equal(cols[2], cols[4])
    with pytest.raises(ValueError):
        oracle.solve_horizons(prob, [3, 0])


def test_algorithm1_brownian_columns_vs_series():
    """1D Brownian motion (Section 4.1, autonomous): every column is the
    Scheme-1 state u^{M-m} of one pass, and approaches the closed form
    Eq. (e45) at its own horizon on a Remark-2 grid (first order in dt:
    halving dt roughly halves the error at every horizon); bounds [0, 1] and
    monotone in the horizon."""
    L, q = 10.0, 3
    errs = []
    for dt in (0.1, 0.05):
        x = remark2_grid(L, 0.05, dt, 1.0, q)
        hz = [int(round(T / dt)) for T in (0.5, 1.0, 2.0, 3.0)]
        prob = W.Problem(axes=[W.Axis(x)], coef_kind="const", coef=(0.0,), D=0.5,
                         region_kind="box", gh_q=q, dt=dt, n_steps=max(hz))
        cols = oracle.solve_horizons(prob, hz)
        one = oracle.solve(prob, snaps=[max(hz) - m for m in hz])
        assert np.abs(cols - one).max() <= 1e-14
        assert cols.min() >= -1e-14 and cols.max() <= 1 + 1e-14
        assert np.all(np.diff(cols, axis=0) >= -1e-12)
        errs.append([np.abs(c - p_exit_series(m * dt, x, L)).max() for c, m in zip(cols, hz)])
    errs = np.array(errs)
    assert np.all(errs[1] < 0.6 * errs[0]), errs
    assert errs[1].max() < 0.04, errs


def test_algorithm1_exit_probability_grows_with_horizon():
    """Exiting by a later horizon is at least as likely (the events are
    nested).  In 2D the scheme keeps this only approximately: the tensor
    interpolant without twist terms (reading 8) can overshoot where the disc's
    exit value 1 meets the interior, so a node next to the circle may lose a
    little between horizons, and the scheme carries a trace of that inward.
    Gates: the disc mean grows at every horizon; away from the circle (more
    than two cells) no node decreases by more than 1e-4; next to it the
    decrease stays below 1e-2 (observed: 1.7e-5 and 6.8e-3)."""
    prob = W.cell2d(nx=65, ny=33, n_steps=60, D=3e-3, dt=2e-3, A=1.2, eps=0.2, omega=9.0)
    hz = [5, 10, 20, 35, 60]
    cols = oracle.solve_horizons(prob, hz)
    w = W.region_mean_weights(prob)
    means = [float((w * c).sum()) for c in cols]
    assert np.all(np.diff(means) > 1e-3), means
    inc = np.diff(cols, axis=0)
    X, Y = np.meshgrid(prob.axes[0].nodes, prob.axes[1].nodes, indexing="ij")
    near = np.abs(np.hypot(X - 0.5, Y - 0.5) - prob.radius) <= 2.0 / 32
    assert inc[:, ~near].min() >= -1e-4, inc[:, ~near].min()
    assert inc.min() >= -1e-2, inc.min()


# ---------------------------------------------------------------------------
# The R2 interpolant: full tensor cubic Hermite with PCHIP-composed twist
# fields (Section 3.1.2, "tensor product"; the mixed derivatives the R1
# reading leaves out)
# ---------------------------------------------------------------------------


def _grid2d(r2=True):
    prob = W.Problem(axes=[W.uniform_axis(0.0, 1.0, 9), W.uniform_axis(-1.0, 0.6, 7)],
                     coef_kind="const", coef=(0.0, 0.0), D=0.0, region_kind="box",
                     gh_q=1, dt=0.01, n_steps=1, hermite="r2" if r2 else "r1")
    X, Y = np.meshgrid(prob.axes[0].nodes, prob.axes[1].nodes, indexing="ij")
    return prob, X, Y


def test_r2_exact_on_tensor_products_of_cubics():
    """With exact value, slope and twist fields the R2 interpolant reproduces
    p(x) q(y) (2D) and p(x) q(y) r(z) (3D) for cubics p, q, r to rounding."""
    p = np.polynomial.Polynomial([0.3, -1.2, 0.7, 2.1])
    q = np.polynomial.Polynomial([1.1, 0.4, -0.9, 0.5])
    r = np.polynomial.Polynomial([-0.2, 0.8, 0.3, -0.6])
    prob, X, Y = _grid2d()
    u = p(X) * q(Y)
    g = np.stack([p.deriv()(X) * q(Y), p(X) * q.deriv()(Y), p.deriv()(X) * q.deriv()(Y)])
    rng = np.random.default_rng(31)
    for _ in range(40):
        z = [rng.uniform(0, 1), rng.uniform(-1, 0.6)]
        assert abs(oracle.interp(prob, u, g, z) - p(z[0]) * q(z[1])) <= 1e-13
    prob3 = W.Problem(axes=[W.uniform_axis(0, 1, 6), W.uniform_axis(0, 2, 5), W.uniform_axis(-1, 1, 7)],
                      coef_kind="const", coef=(0.0, 0.0, 0.0), D=0.0, region_kind="box",
                      gh_q=1, dt=0.01, n_steps=1, hermite="r2")
    A, B, C = np.meshgrid(*[ax.nodes for ax in prob3.axes], indexing="ij")
    P0, P1 = p(A), p.deriv()(A)
    Q0, Q1 = q(B), q.deriv()(B)
    R0, R1 = r(C), r.deriv()(C)
    u3 = P0 * Q0 * R0
    # fields: d/dx, d/dy, d/dz, then {x,y}, {x,z}, {y,z}, {x,y,z}
    g3 = np.stack([P1 * Q0 * R0, P0 * Q1 * R0, P0 * Q0 * R1,
                   P1 * Q1 * R0, P1 * Q0 * R1, P0 * Q1 * R1, P1 * Q1 * R1])
    for _ in range(40):
        z = [rng.uniform(0, 1), rng.uniform(0, 2), rng.uniform(-1, 1)]
        assert abs(oracle.interp(prob3, u3, g3, z) - p(z[0]) * q(z[1]) * r(z[2])) <= 1e-12


def test_r1_misses_exactly_the_twist_term_on_bilinear_data():
    """u = a + b x + c y + d x y: the PCHIP slopes and the composed twist are
    exact on bilinear data, so R2 reproduces u exactly, while R1 misses
    d h_x h_y s(1-s)(1-2s) t(1-t)(1-2t) -- the closed form of the dropped
    twist term (its sign and scale)."""
    a, b, c, d = 0.2, -0.7, 0.4, 1.3
    prob, X, Y = _grid2d()
    u = a + b * X + c * Y + d * X * Y
    g2 = oracle.slopes(prob, u)
    assert g2.shape[0] == 3
    np.testing.assert_allclose(g2[2], d, atol=1e-13)
    prob1 = prob.replace(hermite="r1")
    g1 = oracle.slopes(prob1, u)
    assert g1.shape[0] == 2
    hx = prob.axes[0].nodes[1] - prob.axes[0].nodes[0]
    hy = prob.axes[1].nodes[1] - prob.axes[1].nodes[0]
    rng = np.random.default_rng(32)
    for _ in range(30):
        z = [rng.uniform(0, 1), rng.uniform(-1, 0.6)]
        exact = a + b * z[0] + c * z[1] + d * z[0] * z[1]
        assert abs(oracle.interp(prob, u, g2, z) - exact) <= 1e-13
        k0 = oracle.cell(prob.axes[0].nodes, z[0])
        k1 = oracle.cell(prob.axes[1].nodes, z[1])
        s = (z[0] - prob.axes[0].nodes[k0]) / hx
        t = (z[1] - prob.axes[1].nodes[k1]) / hy
        miss = d * hx * hy * s * (1 - s) * (1 - 2 * s) * t * (1 - t) * (1 - 2 * t)
        assert abs((exact - oracle.interp(prob1, u, g1, z)) - miss) <= 1e-13


def test_r2_step_translates_bilinear_data_exactly():
    """sigma = 0, constant drift, no exit reachable: one step moves bilinear
    data by b dt exactly with R2 (rounding), not with R1."""
    a, b, c, d = 0.1, 0.5, -0.3, 0.9
    axes = [W.uniform_axis(0.0, 1.0, 21), W.uniform_axis(0.0, 1.0, 17)]
    prob = W.Problem(axes=axes, coef_kind="const", coef=(0.37, -0.21), D=0.0,
                     region_kind="box", gh_q=1, dt=0.03, n_steps=1, hermite="r2")
    X, Y = np.meshgrid(axes[0].nodes, axes[1].nodes, indexing="ij")
    u = a + b * X + c * Y + d * X * Y
    inner = (X > 0.2) & (X < 0.8) & (Y > 0.2) & (Y < 0.8)
    Xs, Ys = X + 0.37 * 0.03, Y - 0.21 * 0.03
    want = a + b * Xs + c * Ys + d * Xs * Ys
    got2 = oracle.step(prob, 0, u)
    got1 = oracle.step(prob.replace(hermite="r1"), 0, u)
    assert np.abs(got2 - want)[inner].max() <= 1e-13
    assert np.abs(got1 - want)[inner].max() > 1e-7


def test_r2_twist_field_is_pchip_composed_x_then_y():
    """The twist field is the PCHIP slope along y of the PCHIP slope along x
    (reading: the one-dimensional rule composed in increasing axis order).
    Pinned against scipy's PchipInterpolator, whose interior slopes on a
    uniform axis are the paper's harmonic mean: at interior nodes whose
    stencils stay interior, on data where the limiter acts (the two orders of
    composition differ there)."""
    from scipy.interpolate import PchipInterpolator
    prob, X, Y = _grid2d()
    rng = np.random.default_rng(33)
    u = np.sin(2.5 * X) * np.cos(1.7 * Y) + 0.3 * rng.uniform(-1, 1, size=X.shape)
    g = oracle.slopes(prob, u)
    x, y = prob.axes[0].nodes, prob.axes[1].nodes
    gx = np.stack([PchipInterpolator(x, u[:, j]).derivative()(x) for j in range(len(y))], axis=1)
    gxy = np.stack([PchipInterpolator(y, gx[i, :]).derivative()(y) for i in range(len(x))], axis=0)
    gy = np.stack([PchipInterpolator(y, u[i, :]).derivative()(y) for i in range(len(x))], axis=0)
    gyx = np.stack([PchipInterpolator(x, gy[:, j]).derivative()(x) for j in range(len(y))], axis=1)
    sl = (slice(2, -2), slice(2, -2))    # stencils of stencils stay interior
    np.testing.assert_allclose(g[2][sl], gxy[sl], atol=1e-12)
    assert np.abs(gxy - gyx)[sl].max() > 1e-3


# ---------------------------------------------------------------------------
# Boundary faces: exit with value 1, exit with value 0, reflecting (the
# runaway-electron model of Section 4.3 leaves through p_max with value 1,
# through p_min and the wall r = 1 with value 0, and reflects at xi = +-1 and
# on the axis r = 0)
# ---------------------------------------------------------------------------


def _bm_faces(faces, n=201, D=0.1, dt=1e-4, T=0.4, gh_q=8):
    return W.Problem(axes=[W.uniform_axis(0.0, 1.0, n)], coef_kind="const", coef=(0.0,), D=D,
                     region_kind="box", gh_q=gh_q, dt=dt, n_steps=int(round(T / dt)),
                     faces=(faces,))


def _series_exit0_exit1(x, D, T, K=200):
    k = np.arange(1, K + 1)[:, None]
    return x + np.sum(2 * (-1.0) ** k / (k * np.pi) * np.sin(k * np.pi * x) *
                      np.exp(-D * (k * np.pi) ** 2 * T), axis=0)


def _series_reflect_exit1(x, D, T, K=200):
    k = np.arange(0, K)[:, None]
    lam = (k + 0.5) * np.pi
    return 1 - np.sum(2 * (-1.0) ** k / lam * np.cos(lam * x) * np.exp(-D * lam ** 2 * T), axis=0)


@pytest.mark.parametrize("faces", [("exit0", "exit1"), ("reflect", "exit1")])
def test_faces_brownian_exit_through_one_face_vs_series(faces):
    """Brownian motion on (0, 1) with D = 0.1 up to T = 0.4: the probability of
    leaving through x = 1 when x = 0 counts 0 (Dirichlet 0) or reflects
    (Neumann), against the closed-form sine / cosine series of the heat
    equation; the discrete monitoring of the chain biases the result by
    about 0.58 sigma sqrt(dt) near the faces (0.003 here)."""
    prob = _bm_faces(faces)
    u0 = oracle.solve(prob, snaps=[0])[0]
    x = prob.axes[0].nodes
    ref = (_series_exit0_exit1 if faces[0] == "exit0" else _series_reflect_exit1)(x, 0.1, 0.4)
    err = np.abs(u0 - ref)
    print(faces, "max err", err.max())
    assert err.max() <= 6e-3
    assert u0[-1] == 1.0
    if faces[0] == "exit0":
        assert u0[0] == 0.0
    else:
        assert oracle.node_class(prob)[0] == 0   # the reflecting face is an active node


def test_reflecting_face_translates_linear_data_exactly():
    """sigma = 0, drift toward a reflecting face: a landing point beyond it is
    mirrored, so one step maps linear data u = a + b x to a + b z with
    z = lo + (lo - (x + b_drift dt)) near the face."""
    axes = [W.uniform_axis(0.0, 1.0, 41)]
    prob = W.Problem(axes=axes, coef_kind="const", coef=(-2.0,), D=0.0, region_kind="box",
                     gh_q=1, dt=0.01, n_steps=1, faces=(("reflect", "exit1"),))
    x = axes[0].nodes
    u = 0.3 + 0.5 * x
    got = oracle.step(prob, 0, u)
    z = x - 0.02
    z = np.where(z < 0.0, 0.0 + (0.0 - z), z)
    want = 0.3 + 0.5 * z
    assert np.abs(got[:-1] - want[:-1]).max() <= 1e-14
    assert got[-1] == 1.0


def _re(**kw):
    kw.setdefault("n_p", 13)
    kw.setdefault("n_xi", 9)
    kw.setdefault("r_axis", W.remark2_axis(0.0, 0.7, 1.0, 0.1, 0.05))
    return W.runaway3d(**kw)


def test_runaway_collision_functions_from_their_definitions():
    """Section 4.3: psi(y) = (phi - y phi') / (2 y^2) with phi(y) =
    2/sqrt(pi) int_0^y exp(-s^2) ds, evaluated here by quadrature (scipy),
    gives C_A, C_B, C_F; the small- and large-y limits psi ~ 2y/(3 sqrt(pi))
    and psi ~ 1/(2 y^2) hold; dC_A/dp equals central differences of C_A."""
    from scipy.integrate import quad
    prob = _re()
    delta, Z = 0.042, 1.0
    for pm in (2.0, 5.5, 13.0, 31.0, 50.0):
        gam = math.sqrt(1 + (delta * pm) ** 2)
        y = pm / gam
        phi = 2 / math.sqrt(math.pi) * quad(lambda s: math.exp(-s * s), 0, y)[0]
        dphi = 2 / math.sqrt(math.pi) * math.exp(-y * y)
        psi = (phi - y * dphi) / (2 * y * y)
        CA, CB, CF, dCA = oracle.re_coeffs(prob, 0.0, pm)
        np.testing.assert_allclose([CA, CB, CF],
                                   [psi / y, 0.5 / y * (Z + phi - psi + 0.5 * y * y * delta ** 4),
                                    2 * psi], rtol=1e-10)
        h = 1e-5 * pm
        fd = (oracle.re_coeffs(prob, 0.0, pm + h)[0] - oracle.re_coeffs(prob, 0.0, pm - h)[0]) / (2 * h)
        assert abs(dCA - fd) <= 1e-7 * abs(fd) + 1e-12
    # limits of psi through C_A = psi / y (nu = v_T = 1)
    tiny = W.runaway3d(delta=0.0, p_min=1e-3, n_p=4, n_xi=4, r_axis=W.uniform_axis(0, 1, 4))
    y = 1e-3
    assert abs(oracle.re_coeffs(tiny, 0.0, y)[0] * y / (2 * y / (3 * math.sqrt(math.pi))) - 1) < 1e-5
    y = 30.0
    assert abs(oracle.re_coeffs(tiny, 0.0, y)[0] * y / (1 / (2 * y * y)) - 1) < 1e-12


def test_runaway_drift_and_diffusion_follow_eq_ex32d():
    """The p drift holds (1/p^2) d(p^2 C_A)/dp (checked by central differences
    of p^2 C_A), the xi drift and the diffusion coefficients follow
    Eq. (ex32d), the r drift is V(r) + dD/dr (central differences of D)."""
    prob = _re()
    E, tau, delta = 0.3, 1e5, 0.042
    rng = np.random.default_rng(41)
    for _ in range(12):
        pm, xi, r = rng.uniform(2.5, 49), rng.uniform(-0.99, 0.99), rng.uniform(0.01, 0.99)
        CA, CB, CF, _ = oracle.re_coeffs(prob, 0.0, pm)
        gam = math.sqrt(1 + (delta * pm) ** 2)
        h = 1e-5 * pm
        dp2CA = ((pm + h) ** 2 * oracle.re_coeffs(prob, 0.0, pm + h)[0]
                 - (pm - h) ** 2 * oracle.re_coeffs(prob, 0.0, pm - h)[0]) / (2 * h)
        b = oracle.drift(prob, 0.0, [pm, xi, r])
        bp = E * xi - gam * pm / tau * (1 - xi * xi) - CF + dp2CA / (pm * pm)
        bxi = E * (1 - xi * xi) / pm - xi * (1 - xi * xi) / (tau * gam) - 2 * xi * CB / (pm * pm)
        Dr = lambda rr: 0.5e-4 * (1 + math.tanh((rr - 0.7) / 1e-2)) * math.exp(-(pm / 20) ** 2)  # noqa: E731
        hr = 1e-7
        br = (0.003 if r > 0.7 else 0.0) + (Dr(r + hr) - Dr(r - hr)) / (2 * hr)
        np.testing.assert_allclose(b, [bp, bxi, br], rtol=1e-6, atol=1e-12)
        sg = oracle.sigma(prob, 0.0, [pm, xi, r])
        np.testing.assert_allclose(sg, [math.sqrt(2 * CA), math.sqrt(2 * CB) / pm * math.sqrt(1 - xi * xi),
                                        math.sqrt(2 * Dr(r))], rtol=1e-12)


def test_runaway_probability_faces_and_monotone_in_field():
    """On the runaway model: nodes on p = p_max hold 1, on p_min and the
    wall r = 1 hold 0 (exit faces), xi = +-1 and r = 0 are active (reflecting);
    0 <= P_RE <= 1 up to the interpolant's overshoot; without electric field
    hardly anything runs away, and P_RE grows with E (its mean, and at nearly
    every node where the electron moves along the field)."""
    base = _re(dt=1.0, T=20.0)
    cls = oracle.node_class(base)
    assert np.all(cls[-1] == 1) and np.all(cls[0] == 1) and np.all(cls[:, :, -1] == 1)
    assert np.all(cls[1:-1, :, :-1] == 0)
    u = {E: oracle.solve(_re(dt=1.0, T=20.0, E=E), snaps=[0])[0] for E in (0.0, 0.15, 0.3)}
    for v in u.values():
        # the corner of p_max and the wall belongs to p_max (the lowest axis decides)
        assert np.all(v[-1] == 1.0) and np.all(v[0] == 0.0) and np.all(v[:-1, :, -1] == 0.0)
        assert v.min() >= -1e-3 and v.max() <= 1 + 1e-3
    inner = (slice(1, -1), slice(None), slice(0, -1))
    assert u[0.0][inner].mean() < 0.1 * u[0.3][inner].mean()
    assert u[0.0][inner].mean() < u[0.15][inner].mean() < u[0.3][inner].mean()
    # the field accelerates electrons moving along it (dp = E xi dt): where
    # xi >= 1/2 the runaway probability grows with E at nearly every node
    # (pointwise order is not a theorem of the discrete scheme: the PCHIP
    # interpolant does not preserve order in the data); where xi < 0 the
    # field decelerates and no order is expected
    xi = base.axes[1].nodes
    fwd = (slice(1, -1), xi >= 0.5, slice(0, -1))
    for lo, hi in ((0.0, 0.15), (0.15, 0.3)):
        assert np.mean(u[lo][fwd] <= u[hi][fwd] + 1e-9) >= 0.99, (lo, hi)


def test_runaway_thermal_quench_parameters():
    """t_* > 0: That(0) = That_0 gives v_T = 1 (That_0 = Ttilde), nu = 1 and
    E = E_0 at t = 0; as the plasma cools, E grows like That^(-3/2)."""
    tq = W.runaway3d(n_p=5, n_xi=5, r_axis=W.uniform_axis(0, 1, 5), t_star=10.0, E0=1e-3,
                     That0=3.0, Thatf=0.005, Ttilde=3.0, tau=6000.0, r_D=0.0, W=1e-4,
                     Delta_p=2.0, V0=0.0)
    c0 = oracle.re_coeffs(tq, 0.0, 10.0)
    ref = _re()
    cr = oracle.re_coeffs(ref.replace(coef=(1e-3, 6000.0, 1.0, math.sqrt(6 / 511.0), 1.0, 1.0) +
                                      ref.coef[6:]), 0.0, 10.0)
    np.testing.assert_allclose(c0, cr, rtol=1e-12)
    b0 = oracle.drift(tq, 0.0, [10.0, 1.0, 0.5])
    b1 = oracle.drift(tq, 30.0, [10.0, 1.0, 0.5])
    Th = 0.005 + (3.0 - 0.005) * math.exp(-3.0)
    assert b1[1] < 0 and b0[0] != b1[0]
    # at xi = 1 the p drift is E - C_F + (1/p^2) d(p^2 C_A)/dp: its E part scales
    c1 = oracle.re_coeffs(tq, 30.0, 10.0)
    e_part0 = b0[0] - (-c0[2] + 2 * c0[0] / 10.0 + c0[3])
    e_part1 = b1[0] - (-c1[2] + 2 * c1[0] / 10.0 + c1[3])
    np.testing.assert_allclose([e_part0, e_part1], [1e-3, 1e-3 * (3.0 / Th) ** 1.5], rtol=1e-9)
