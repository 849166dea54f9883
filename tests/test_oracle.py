"""Pins of the FP64 oracle against things other than itself.

Every check here uses an independent source: scipy's B-spline and Bernstein
evaluators, closed-form projections, polynomial root finding, brute force,
matrices printed in the paper, or first-order optimality checked numerically.
"""
import numpy as np
import pytest
from scipy.interpolate import BPoly, BSpline, PPoly
from scipy.spatial import cKDTree

import oracle
from conftest import load_golden
from paper_2504_11498_amd import gen


def random_curve(rng, p, n_cp, dup=0):
    P = rng.uniform(0, 1, (n_cp, 3))
    n_int = n_cp - p - 1
    base = np.sort(rng.uniform(0.02, 0.98, n_int - dup))
    if dup:
        base = np.sort(np.concatenate([base, rng.choice(base, dup, replace=False)]))
    U = np.concatenate([np.zeros(p + 1), base, np.ones(p + 1)])
    return P, U


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build(force=False)


# --------------------------------------------------------------------------- basis / evaluation
@pytest.mark.parametrize("p", [1, 2, 3, 5, 7, 9])
def test_basis_partition_of_unity_and_sum(p):
    rng = np.random.default_rng(10 + p)
    P, U = random_curve(rng, p, p + 9, dup=1 if p >= 2 else 0)
    spl = BSpline(U, P, p)
    for t in np.concatenate([rng.uniform(0, 1, 40), [0.0, 1.0], U[p + 1 : -p - 1]]):
        N = oracle.basis(p, U, t)
        assert np.all(N >= -1e-15)
        assert abs(N.sum() - 1.0) <= 1e-14
        np.testing.assert_allclose(N @ P, spl(t), atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6, 7, 9])
def test_deboor_matches_scipy_with_derivatives(p):
    rng = np.random.default_rng(100 + p)
    P, U = random_curve(rng, p, 3 * p + 5, dup=1 if p >= 3 else 0)
    t = np.concatenate([rng.uniform(0, 1, 300), [0.0, 1.0]])
    X, D1, D2 = oracle.eval_curve(p, P, U, t, derivs=True)
    spl = BSpline(U, P, p)
    np.testing.assert_allclose(X, spl(t), atol=1e-13)
    np.testing.assert_allclose(D1, spl.derivative(1)(t), atol=1e-9 * np.abs(D1).max())
    if p >= 2:
        np.testing.assert_allclose(D2, spl.derivative(2)(t), atol=1e-8 * np.abs(D2).max())


def test_deboor_right_end_uses_last_span():
    rng = np.random.default_rng(3)
    P, U = random_curve(rng, 3, 10)
    X = oracle.eval_curve(3, P, U, [1.0])
    np.testing.assert_allclose(X[0], P[-1], atol=1e-15)  # clamped end interpolates the last point


# --------------------------------------------------------------------------- Boehm spans
@pytest.mark.parametrize("p,dup", [(2, 1), (3, 0), (4, 2), (5, 1), (7, 0)])
def test_boehm_spans_match_bernstein_form(p, dup):
    rng = np.random.default_rng(200 + p)
    P, U = random_curve(rng, p, 4 * p + 3, dup=dup)
    bz, tab = oracle.bezier_spans(p, P, U)
    distinct = np.unique(U)
    assert bz.shape[0] == distinct.shape[0] - 1
    np.testing.assert_array_equal(tab[:, 0], distinct[:-1])
    x = np.concatenate([tab[:, 0], tab[-1:, 1]])
    bp = BPoly(np.transpose(bz, (1, 0, 2)), x)
    t = np.linspace(0, 1, 2001)
    np.testing.assert_allclose(bp(t), BSpline(U, P, p)(t), atol=1e-13)


# --------------------------------------------------------------------------- paper-printed matrices
def test_printed_rebasement_matrix_converts_power_to_bernstein():
    """b = T a with the paper's printed T (Sec. 5.3): the Bernstein form evaluated by the
    oracle's de Casteljau must equal the power polynomial evaluated by numpy."""
    T = np.array([[float(v) for v in r.split()] for r in load_golden("power_to_bernstein_deg5.txt")])
    assert T.shape == (6, 6)
    rng = np.random.default_rng(5)
    a = rng.normal(size=(6, 3))
    b = T @ a
    u = np.linspace(0, 1, 33)
    ref = np.stack([np.polynomial.polynomial.polyval(u, a[:, c]) for c in range(3)], -1)
    np.testing.assert_allclose(oracle.bez_eval(b, u), ref, atol=1e-13)


def _printed_S(z):
    rows = load_golden("subdivision_matrix_Sz.txt")
    env = {"__builtins__": {}, "z": z}
    return np.array([[eval(e, env) for e in r.split(";")] for r in rows], dtype=np.float64)  # noqa: S307


@pytest.mark.parametrize("z", [0.125, 0.3, 0.5, 0.77])
def test_printed_subdivision_matrix_matches_de_casteljau(z):
    rng = np.random.default_rng(int(z * 1000))
    P = rng.uniform(0, 1, (4, 3))
    S = _printed_S(z)
    L, R = oracle.bez_split(P, z)
    np.testing.assert_allclose(S[:4] @ P, L, atol=1e-15)
    np.testing.assert_allclose(S[4:] @ P, R, atol=1e-15)
    # and the halves reproduce the curve on their sub-ranges
    u = np.linspace(0, 1, 17)
    np.testing.assert_allclose(oracle.bez_eval(L, u), oracle.bez_eval(P, z * u), atol=1e-14)
    np.testing.assert_allclose(oracle.bez_eval(R, u), oracle.bez_eval(P, z + (1 - z) * u), atol=1e-14)


@pytest.mark.parametrize("p", [4, 6, 9])
def test_degree_p_split_reproduces_curve(p):
    rng = np.random.default_rng(p)
    Q = rng.uniform(0, 1, (p + 1, 3))
    L, R = oracle.bez_split(Q, 0.37)
    u = np.linspace(0, 1, 9)
    ref = BPoly(Q[:, None, :], [0, 1])
    np.testing.assert_allclose(oracle.bez_eval(L, u), ref(0.37 * u), atol=1e-14)
    np.testing.assert_allclose(oracle.bez_eval(R, u), ref(0.37 + 0.63 * u), atol=1e-14)


# --------------------------------------------------------------------------- reduction
def _elevate_np(Q, times):
    for _ in range(times):
        p = Q.shape[0] - 1
        i = np.arange(p + 2)[:, None] / (p + 1)
        lo = np.vstack([np.zeros((1, 3)), Q])
        hi = np.vstack([Q, np.zeros((1, 3))])
        Q = i * lo + (1 - i) * hi
    return Q


@pytest.mark.parametrize("p", [4, 5, 6, 7, 9])
def test_reduction_of_elevated_cubic_is_exact(p):
    """A cubic written at degree p must come back unchanged with delta = (1, 1)."""
    rng = np.random.default_rng(300 + p)
    R0 = rng.uniform(0, 1, (4, 3))
    Q = _elevate_np(R0, p - 3)
    # the elevated piece is the same curve (checked with scipy's Bernstein evaluator)
    u = np.linspace(0, 1, 11)
    np.testing.assert_allclose(BPoly(Q[:, None, :], [0, 1])(u), BPoly(R0[:, None, :], [0, 1])(u), atol=1e-14)
    R, dl = oracle.g1_reduce(Q)
    np.testing.assert_allclose(dl, [1.0, 1.0], atol=1e-11)
    np.testing.assert_allclose(R, R0, atol=1e-12)


@pytest.mark.parametrize("p", [4, 5, 7])
def test_reduction_is_g1_and_l2_optimal(p):
    rng = np.random.default_rng(400 + p)
    Q = rng.uniform(0, 1, (p + 1, 3))
    R, dl = oracle.g1_reduce(Q)
    # G1 conditions of Sec. 5.2.2 (eq. G1-condition)
    np.testing.assert_allclose(R[0], Q[0], atol=0)
    np.testing.assert_allclose(R[3], Q[p], atol=0)
    np.testing.assert_allclose(R[1], Q[0] + p / 3 * (Q[1] - Q[0]) * dl[0], atol=1e-14)
    np.testing.assert_allclose(R[2], Q[p] - p / 3 * (Q[p] - Q[p - 1]) * dl[1], atol=1e-14)

    # L2 error (eq. epsl) by 40-point Gauss-Legendre (numpy) as a function of (d0, d1)
    x, w = np.polynomial.legendre.leggauss(40)
    u, w = 0.5 * (x + 1), 0.5 * w
    Qu = BPoly(Q[:, None, :], [0, 1])(u)

    def eps(d0, d1):
        Rr = np.array([Q[0], Q[0] + p / 3 * (Q[1] - Q[0]) * d0, Q[p] - p / 3 * (Q[p] - Q[p - 1]) * d1, Q[p]])
        diff = Qu - BPoly(Rr[:, None, :], [0, 1])(u)
        return float(np.sum(w * np.sum(diff * diff, -1)))

    e0 = eps(*dl)
    h = 1e-4
    g0 = (eps(dl[0] + h, dl[1]) - eps(dl[0] - h, dl[1])) / (2 * h)
    g1 = (eps(dl[0], dl[1] + h) - eps(dl[0], dl[1] - h)) / (2 * h)
    assert abs(g0) < 1e-7 and abs(g1) < 1e-7
    for d0, d1 in [(0.02, 0), (-0.02, 0), (0, 0.02), (0, -0.02), (0.01, 0.01)]:
        assert eps(dl[0] + d0, dl[1] + d1) > e0


def test_gram_closed_form_matches_quadrature():
    """Eq. gram: g_ij = C(m,i)C(n,j) / ((m+n+1) C(m+n,i+j)) equals the integral of B_i^m B_j^n."""
    from math import comb

    x, w = np.polynomial.legendre.leggauss(30)
    u, w = 0.5 * (x + 1), 0.5 * w
    for m, n in [(3, 3), (3, 5), (3, 7)]:
        for i in range(m + 1):
            for j in range(n + 1):
                bi = comb(m, i) * u**i * (1 - u) ** (m - i)
                bj = comb(n, j) * u**j * (1 - u) ** (n - j)
                g = comb(m, i) * comb(n, j) / ((m + n + 1) * comb(m + n, i + j))
                assert abs(np.sum(w * bi * bj) - g) < 4e-15
    # G_{3,3} in FP64 is 16 doubles = 128 bytes (Sec. 5.1)
    assert np.zeros((4, 4)).nbytes == 128


# --------------------------------------------------------------------------- decomposition
def _pieces_vs_spline(curves, dec, tol):
    """Every cubic piece stays within tol of the original spline (4097 samples, scipy evaluation)."""
    off = 0
    worst = 0.0
    for c in range(curves.n):
        p, P, U = curves.curve(c)
        spl = BSpline(U, P, p)
        k = int(dec["counts"][c])
        for s in range(off, off + k):
            ta, tb = dec["tab"][s]
            u = np.linspace(0, 1, 4097)
            R = dec["R"][s]
            err = np.linalg.norm(BPoly(R[:, None, :], [0, 1])(u) - spl(ta + u * (tb - ta)), axis=1).max()
            worst = max(worst, err / tol[c])
        # pieces tile the domain in order
        tab = dec["tab"][off : off + k]
        assert tab[0, 0] == 0.0 and tab[-1, 1] == 1.0
        assert np.all(tab[1:, 0] == tab[:-1, 1])
        off += k
    return worst


def test_decomposition_low_degree_is_exact():
    rng = np.random.default_rng(11)
    degs, cps, kts = [], [], []
    for p in [1, 2, 2, 3, 3]:
        P, U = random_curve(rng, p, 12, dup=1 if p == 3 else 0)
        degs.append(p), cps.append(P), kts.append(U)
    curves = gen._pack(degs, cps, kts)
    tol = np.full(curves.n, 1e-6)
    dec = oracle.decompose(curves, tol)
    assert _pieces_vs_spline(curves, dec, tol) * 1e-6 < 1e-13
    for c in range(curves.n):  # one cubic per non-degenerate span
        assert dec["counts"][c] == len(np.unique(curves.curve(c)[2])) - 1


def test_decomposition_high_degree_within_tolerance():
    curves = gen.curves_batched_geometry(seed=21, n_curves=12, deg_lo=4, deg_hi=7, cp_lo=8, cp_hi=40)
    tol = 1e-6 * curves.bbox_diag()
    dec = oracle.decompose(curves, tol)
    assert dec["R"].shape[0] > 2 * sum(len(np.unique(curves.curve(c)[2])) - 1 for c in range(curves.n))
    assert _pieces_vs_spline(curves, dec, tol) <= 1.0


# --------------------------------------------------------------------------- projection
def _single(p, P, U):
    return gen._pack([p], [np.asarray(P, float)], [np.asarray(U, float)])


def test_projection_straight_line_closed_form():
    """Equally spaced collinear Bezier control points give C(t) = P0 + t (Pp - P0)."""
    rng = np.random.default_rng(1)
    for p in [2, 3, 5]:
        A, B = rng.uniform(0, 1, 3), rng.uniform(0, 1, 3)
        P = A + np.linspace(0, 1, p + 1)[:, None] * (B - A)
        U = np.concatenate([np.zeros(p + 1), np.ones(p + 1)])
        q = rng.uniform(-0.5, 1.5, (400, 3))
        r = oracle.project(_single(p, P, U), np.zeros(400, np.int32), q)
        d = B - A
        ts = np.clip((q - A) @ d / (d @ d), 0, 1)
        ds = np.linalg.norm(q - (A + ts[:, None] * d), axis=1)
        np.testing.assert_allclose(r["dist"], ds, atol=1e-14)
        inner = (ts > 1e-6) & (ts < 1 - 1e-6)
        np.testing.assert_allclose(r["t"][inner], ts[inner], atol=1e-12)


def _roots_reference(p, P, U, q):
    """Global minimum by all real roots of dD/dt per polynomial piece (scipy PPoly + numpy roots)."""
    pps = [PPoly.from_spline((U, P[:, c], p)) for c in range(3)]
    x = pps[0].x
    best = (np.inf, 0.0)
    for k in range(len(x) - 1):
        a, b = x[k], x[k + 1]
        if not b > a:
            continue
        # local power form in s = t - a, highest power first
        polys = [np.poly1d(pp.c[:, k]) for pp in pps]
        D = sum((pc - qc) ** 2 for pc, qc in zip(polys, q))
        cand = [0.0, b - a]
        for r in D.deriv().roots:
            if abs(r.imag) < 1e-9 and -1e-12 <= r.real <= b - a + 1e-12:
                cand.append(min(max(r.real, 0.0), b - a))
        for s in cand:
            d = np.sqrt(max(D(s), 0.0))
            if d < best[0]:
                best = (d, a + s)
    return best


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_projection_tiny_exhaustive_roots(p):
    rng = np.random.default_rng(500 + p)
    for trial in range(6):
        P, U = random_curve(rng, p, p + 3, dup=0)
        curves = _single(p, P, U)
        q = rng.uniform(-0.2, 1.2, (25, 3))
        r = oracle.project(curves, np.zeros(25, np.int32), q)
        for i in range(25):
            d, t = _roots_reference(p, P, U, q[i])
            assert abs(r["dist"][i] - d) <= 1e-11, (trial, i, r["dist"][i], d)
            if r["runner"][i] > r["dist"][i] + 1e-6 and r["kappa"][i] > 1e-3:
                assert abs(r["t"][i] - t) <= 1e-7


def test_projection_quadratic_bezier_cubic_equation():
    rng = np.random.default_rng(9)
    P = rng.uniform(0, 1, (3, 3))
    U = np.array([0, 0, 0, 1, 1, 1.0])
    q = rng.uniform(-0.3, 1.3, (200, 3))
    r = oracle.project(_single(2, P, U), np.zeros(200, np.int32), q)
    a0, a1, a2 = P[0], 2 * (P[1] - P[0]), P[0] - 2 * P[1] + P[2]
    for i in range(200):
        # (C - q).C' = 0 is a cubic: (a0-q + a1 t + a2 t^2).(a1 + 2 a2 t)
        r0 = a0 - q[i]
        coeffs = [2 * a2 @ a2, 3 * a1 @ a2, a1 @ a1 + 2 * r0 @ a2, r0 @ a1]
        cands = [0.0, 1.0] + [x.real for x in np.roots(coeffs) if abs(x.imag) < 1e-12 and 0 <= x.real <= 1]
        ds = [np.linalg.norm(a0 + a1 * t + a2 * t * t - q[i]) for t in cands]
        assert abs(min(ds) - r["dist"][i]) < 1e-13


def test_projection_inversion_of_on_curve_points():
    curves = gen.curves_batched_geometry(seed=31, n_curves=20, deg_lo=2, deg_hi=7, cp_lo=8, cp_hi=40)
    rng = np.random.default_rng(2)
    cid = np.repeat(np.arange(curves.n, dtype=np.int32), 30)
    t0 = rng.uniform(0, 1, cid.shape[0])
    q = oracle.eval_batch(curves, cid, t0)
    r = oracle.project(curves, cid, q)
    assert r["dist"].max() < 1e-13
    ok = r["runner"] > 1e-9
    np.testing.assert_allclose(r["t"][ok], t0[ok], atol=1e-9)


def test_projection_never_worse_than_dense_sampling():
    curves, qs = gen.curve_single(1, n_queries=3000)
    p, P, U = curves.curve(0)
    tt = np.linspace(0, 1, 1_000_001)
    X = BSpline(U, P, p)(tt)
    dd, ii = cKDTree(X).query(qs.point)
    r = oracle.project(curves, qs.curve_id, qs.point)
    assert np.all(r["dist"] <= dd + 1e-15)
    # and within the sampling resolution of it
    assert np.all(dd - r["dist"] <= 5e-6)
    # where the minimum is unique the dense argmin agrees in t to the sampling step
    u = r["runner"] > r["dist"] + 1e-3
    assert np.all(np.abs(tt[ii[u]] - r["t"][u]) <= 2e-5)


# --------------------------------------------------------------------------- seeding network (MLP)
from scipy.special import ndtr  # noqa: E402  standard normal CDF: GELU(z) = z * Phi(z)

NIN, NH, NOUT = 15, 128, 2


def _blocks(params):
    o = 0
    out = []
    for shape in [(NH, NIN), (NH,), (NH, NH), (NH,), (NOUT, NH), (NOUT,)]:
        n = int(np.prod(shape))
        out.append(params[o : o + n].reshape(shape))
        o += n
    return out


def test_mlp_param_count():
    assert oracle.mlp_param_count() == 18818


def test_mlp_linear_network_via_gelu_odd_part():
    """GELU(z) - GELU(-z) = z exactly, so a network whose hidden units come in
    (+z, -z) pairs and whose next layer takes their difference is linear:
    y = w . x + c in closed form.  A transposed weight layout or a wrong
    activation fails this."""
    rng = np.random.default_rng(7)
    p = np.zeros(oracle.mlp_param_count())
    W1, b1, W2, b2, W3, b3 = _blocks(p)
    for k in range(NIN):
        W1[2 * k, k] = 1.0
        W1[2 * k + 1, k] = -1.0
        W2[2 * k, 2 * k], W2[2 * k, 2 * k + 1] = 1.0, -1.0
        W2[2 * k + 1, 2 * k], W2[2 * k + 1, 2 * k + 1] = -1.0, 1.0
    w0, w1 = rng.normal(size=NIN), rng.normal(size=NIN)
    for k in range(NIN):
        W3[0, 2 * k], W3[0, 2 * k + 1] = w0[k], -w0[k]
        W3[1, 2 * k], W3[1, 2 * k + 1] = w1[k], -w1[k]
    b3[:] = [0.25, -0.5]
    x = rng.normal(size=(33, NIN))
    _, y, _ = oracle.mlp_loss(p, x)
    np.testing.assert_allclose(y[:, 0], x @ w0 + 0.25, rtol=0, atol=1e-12)
    np.testing.assert_allclose(y[:, 1], x @ w1 - 0.5, rtol=0, atol=1e-12)


def test_mlp_single_path_matches_normal_cdf():
    """One active unit per layer: y0 = g(a * g(x_3 + 0.5) - 0.2) + 0.1 with
    g(z) = z * Phi(z), Phi from scipy's ndtr."""
    p = np.zeros(oracle.mlp_param_count())
    W1, b1, W2, b2, W3, b3 = _blocks(p)
    W1[5, 3], b1[5] = 1.0, 0.5
    W2[9, 5], b2[9] = 1.7, -0.2
    W3[0, 9], b3[0] = 1.0, 0.1
    x = np.linspace(-3, 3, 13)[:, None] * np.eye(NIN)[3][None, :]
    _, y, _ = oracle.mlp_loss(p, x)
    g = lambda z: z * ndtr(z)  # noqa: E731
    want = g(1.7 * g(x[:, 3] + 0.5) - 0.2) + 0.1
    np.testing.assert_allclose(y[:, 0], want, rtol=0, atol=1e-14)
    np.testing.assert_allclose(y[:, 1], 0.0, atol=0)


def test_mlp_loss_terms():
    """Loss with a zero network (outputs = biases): MSE masked by accept plus
    binary cross-entropy log(1 + exp(-z)) for a = 1 and log(1 + exp(z)) for a = 0."""
    p = np.zeros(oracle.mlp_param_count())
    b3 = _blocks(p)[5]
    b3[:] = [0.3, 1.25]
    us = np.array([0.1, 0.9, 0.5, 0.0])
    ac = np.array([1.0, 0.0, 1.0, 0.0])
    loss, _, _ = oracle.mlp_loss(p, np.zeros((4, NIN)), us, ac)
    z = 1.25
    terms = ac * (0.3 - us) ** 2 + np.where(ac > 0, np.logaddexp(0, -z), np.logaddexp(0, z))
    assert loss == pytest.approx(terms.mean(), rel=0, abs=1e-15)


def test_mlp_gradient_central_differences():
    """Backward pass against central differences of the loss, on entries of
    every parameter block."""
    rng = np.random.default_rng(11)
    npar = oracle.mlp_param_count()
    p = rng.normal(0, 0.3, npar)
    x = rng.normal(size=(24, NIN))
    us = rng.uniform(0, 1, 24)
    ac = (rng.uniform(size=24) < 0.5).astype(float)
    loss, _, g = oracle.mlp_loss(p, x, us, ac, grad=True)
    offs = np.cumsum([0, NH * NIN, NH, NH * NH, NH, NOUT * NH, NOUT])
    idx = np.concatenate([rng.integers(offs[b], offs[b + 1], 6) for b in range(6)])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        num = (oracle.mlp_loss(pp, x, us, ac)[0] - oracle.mlp_loss(pm, x, us, ac)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-7 * max(1.0, abs(num)), (i, num, g[i])


# --------------------------------------------------------------------------- surfaces (tensor product)
from scipy.interpolate import NdBSpline  # noqa: E402
from scipy.optimize import minimize  # noqa: E402


def _one_surface(p, q, nu, nv, rng, height=True):
    x = np.linspace(0, 1, nu)
    y = np.linspace(0, 1, nv)
    X, Y = np.meshgrid(x, y, indexing="ij")
    Z = rng.uniform(-0.3, 0.3, X.shape) if height else rng.uniform(0, 1, X.shape)
    P = np.stack([X, Y, Z], -1).reshape(-1, 3)
    U = np.r_[np.zeros(p + 1), np.sort(rng.uniform(0.05, 0.95, nu - p - 1)), np.ones(p + 1)]
    V = np.r_[np.zeros(q + 1), np.sort(rng.uniform(0.05, 0.95, nv - q - 1)), np.ones(q + 1)]
    return gen.SurfaceSet(np.array([p], np.int32), np.array([q], np.int32), np.array([nu], np.int32),
                          np.array([nv], np.int32), np.array([0, nu * nv], np.int64), P, np.array([0, len(U)], np.int64),
                          U, np.array([0, len(V)], np.int64), V)


def _ndb(S):
    p, q, nu, nv, P, U, V = oracle.surf_surface(S, 0)
    return NdBSpline((U, V), P.reshape(nu, nv, 3), (p, q))


@pytest.mark.parametrize("p,q", [(3, 3), (5, 5), (2, 4), (1, 3)])
def test_surface_eval_matches_scipy(p, q):
    rng = np.random.default_rng(100 + 10 * p + q)
    S = _one_surface(p, q, p + 6, q + 5, rng, height=False)
    uv = np.concatenate([rng.uniform(0, 1, (300, 2)), [[0, 0], [1, 1], [0, 1], [1, 0]]])
    got = oracle.surf_eval(S, np.zeros(len(uv), np.int32), uv)
    np.testing.assert_allclose(got, _ndb(S)(uv), atol=1e-14)


@pytest.mark.parametrize("p,q", [(3, 3), (5, 5), (2, 3)])
def test_surface_bezier_patches_reproduce_surface(p, q):
    """Boehm patches: each patch net evaluated by Bernstein sums equals the surface on its rectangle."""
    from math import comb

    rng = np.random.default_rng(7 + p + q)
    S = _one_surface(p, q, p + 5, q + 4, rng)
    nets, rects = oracle.surf_patches(S, 0)
    assert len(nets) == (p + 5 - p) * (q + 4 - q)
    spl = _ndb(S)
    st = rng.uniform(0, 1, (40, 2))
    for net, rc in zip(nets, rects):
        Bu = np.array([[comb(p, i) * s ** i * (1 - s) ** (p - i) for i in range(p + 1)] for s in st[:, 0]])
        Bv = np.array([[comb(q, j) * t ** j * (1 - t) ** (q - j) for j in range(q + 1)] for t in st[:, 1]])
        val = np.einsum("ni,nj,ijc->nc", Bu, Bv, net)
        uv = np.stack([rc[0] + st[:, 0] * (rc[1] - rc[0]), rc[2] + st[:, 1] * (rc[3] - rc[2])], 1)
        np.testing.assert_allclose(val, spl(uv), atol=1e-13)
    # exact bicubic patches have zero deviation; a shifted net deviates by the shift
    if p == 3 and q == 3:
        assert oracle.surf_patch_deviation(S, 0, nets[5], rects[5]) <= 1e-14
        assert abs(oracle.surf_patch_deviation(S, 0, nets[5] + [0, 0, 1e-3], rects[5]) - 1e-3) <= 1e-14


def test_surface_projection_plane_closed_form():
    """Control points at the Greville abscissae reproduce S(u, v) = (u, v, 0) (linear precision), so the
    projection of (x, y, z) is (clamp(x), clamp(y)) with the matching distance."""
    rng = np.random.default_rng(3)
    p = q = 3
    n = 9
    U = np.r_[np.zeros(p + 1), np.sort(rng.uniform(0.1, 0.9, n - p - 1)), np.ones(p + 1)]
    V = np.r_[np.zeros(q + 1), np.sort(rng.uniform(0.1, 0.9, n - q - 1)), np.ones(q + 1)]
    gu = np.array([U[i + 1:i + p + 1].mean() for i in range(n)])
    gv = np.array([V[j + 1:j + q + 1].mean() for j in range(n)])
    X, Y = np.meshgrid(gu, gv, indexing="ij")
    P = np.stack([X, Y, np.zeros_like(X)], -1).reshape(-1, 3)
    S = gen.SurfaceSet(np.array([p], np.int32), np.array([q], np.int32), np.array([n], np.int32),
                       np.array([n], np.int32), np.array([0, n * n], np.int64), P, np.array([0, len(U)], np.int64),
                       U, np.array([0, len(V)], np.int64), V)
    x = rng.uniform(-0.4, 1.4, (200, 3))
    r = oracle.surf_project(S, np.zeros(200, np.int32), x)
    cu, cv = np.clip(x[:, 0], 0, 1), np.clip(x[:, 1], 0, 1)
    np.testing.assert_allclose(r["uv"][:, 0], cu, atol=1e-9)
    np.testing.assert_allclose(r["uv"][:, 1], cv, atol=1e-9)
    np.testing.assert_allclose(r["dist"], np.linalg.norm(x - np.stack([cu, cv, 0 * cu], 1), axis=1), atol=1e-12)


@pytest.mark.parametrize("p", [3, 5])
def test_surface_inversion_of_on_surface_points(p):
    """Height fields over a monotone grid: a point on the surface has a unique foot point, its own (u0, v0)."""
    rng = np.random.default_rng(50 + p)
    S = _one_surface(p, p, 12, 11, rng)
    uv0 = rng.uniform(0, 1, (300, 2))
    x = oracle.surf_eval(S, np.zeros(300, np.int32), uv0)
    r = oracle.surf_project(S, np.zeros(300, np.int32), x)
    assert r["dist"].max() <= 1e-12
    np.testing.assert_allclose(r["uv"], uv0, atol=1e-9)


def test_surface_projection_brute_force():
    """Dense 401 x 401 sampling of scipy's surface, then a bounded quasi-Newton polish from the 5 best
    samples: the oracle is never worse and agrees to 1e-9."""
    rng = np.random.default_rng(77)
    S = _one_surface(3, 3, 7, 6, rng)
    spl = _ndb(S)
    g = np.linspace(0, 1, 401)
    G = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    pts = spl(G)
    x = rng.uniform(-0.2, 1.2, (40, 3))
    x[:, 2] = rng.uniform(-0.6, 0.6, 40)
    r = oracle.surf_project(S, np.zeros(40, np.int32), x)
    for k in range(40):
        d = np.linalg.norm(pts - x[k], axis=1)
        best = np.inf
        for i in np.argsort(d)[:5]:
            res = minimize(lambda w: float(np.sum((spl(w[None])[0] - x[k]) ** 2)), G[i], method="L-BFGS-B",
                           bounds=[(0, 1), (0, 1)], options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 500})
            best = min(best, np.sqrt(res.fun), d[i])
        assert r["dist"][k] <= best + 1e-12
        assert abs(r["dist"][k] - best) <= 1e-9


def test_mlp_surface_variant_loss_and_gradient():
    """The patch variant (51 inputs, outputs u, v, logit): loss terms with a zero network and central
    differences of the gradient."""
    nin, nout = 51, 3
    npar = oracle.mlp_param_count(n_in=nin, n_out=nout)
    assert npar == 23555
    p = np.zeros(npar)
    p[-3:] = [0.2, 0.7, -0.4]
    tgt = np.array([[0.1, 0.5], [0.9, 0.3], [0.6, 0.6]])
    ac = np.array([1.0, 0.0, 1.0])
    loss, y, _ = oracle.mlp_loss(p, np.zeros((3, nin)), tgt, ac, n_in=nin, n_out=nout)
    terms = ac * ((0.2 - tgt[:, 0]) ** 2 + (0.7 - tgt[:, 1]) ** 2) + np.where(ac > 0, np.logaddexp(0, 0.4),
                                                                              np.logaddexp(0, -0.4))
    assert loss == pytest.approx(terms.mean(), rel=0, abs=1e-15)
    rng = np.random.default_rng(12)
    p = rng.normal(0, 0.2, npar)
    x = rng.normal(size=(16, nin))
    tgt = rng.uniform(0, 1, (16, 2))
    ac = (rng.uniform(size=16) < 0.5).astype(float)
    _, _, g = oracle.mlp_loss(p, x, tgt, ac, n_in=nin, n_out=nout, grad=True)
    h = 1e-6
    for i in rng.choice(npar, 24, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        num = (oracle.mlp_loss(pp, x, tgt, ac, n_in=nin, n_out=nout)[0] -
               oracle.mlp_loss(pm, x, tgt, ac, n_in=nin, n_out=nout)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-7 * max(1.0, abs(num)), (i, num, g[i])
