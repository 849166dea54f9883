"""Pins of the rational (NURBS) oracle against things other than itself.

The paper's method is stated for non-rational curves (Sec. 6, discussion and
limitations; Sec. 7).  Independent sources here: the rational curve as the
quotient of two scipy B-splines (numerator with the points w_i P_i, denominator
with the weights), with the quotient rule for its derivatives; exact circles
(a quadratic NURBS reproduces a circle, so distances and foot points have closed
forms); equal weights (the curve is then the non-rational one, projected by the
polynomial oracle); and dense brute force.
"""
import numpy as np
import pytest
from scipy.interpolate import BSpline

import oracle
from paper_2504_11498_amd import gen


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build(force=False)


def _random_nurbs(rng, p, n_cp):
    P = rng.uniform(0, 1, (n_cp, 3))
    w = np.exp(rng.uniform(np.log(0.25), np.log(4.0), n_cp))
    U = np.concatenate([np.zeros(p + 1), np.sort(rng.uniform(0.02, 0.98, n_cp - p - 1)), np.ones(p + 1)])
    return P, w, U


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8])
def test_rational_eval_is_the_quotient_of_scipy_bsplines(p):
    rng = np.random.default_rng(500 + p)
    P, w, U = _random_nurbs(rng, p, p + 10)
    num, den = BSpline(U, w[:, None] * P, p), BSpline(U, w, p)
    t = np.concatenate([rng.uniform(0, 1, 300), [0.0, 1.0]])
    X, D1, D2 = oracle.nurbs_eval_curve(p, P, w, U, t, derivs=True)
    N, W = num(t), den(t)[:, None]
    C = N / W
    np.testing.assert_allclose(X, C, atol=1e-13)
    N1, W1 = num.derivative(1)(t), den.derivative(1)(t)[:, None]
    C1 = (N1 - C * W1) / W
    np.testing.assert_allclose(D1, C1, atol=1e-9 * np.abs(C1).max())
    if p >= 2:
        N2, W2 = num.derivative(2)(t), den.derivative(2)(t)[:, None]
        C2 = (N2 - 2 * C1 * W1 - C * W2) / W
        np.testing.assert_allclose(D2, C2, atol=1e-8 * np.abs(C2).max())


def test_circle_closed_forms():
    """A full circle as a quadratic NURBS: every point at the radius; the distance from q is
    sqrt((rho - R)^2 + h^2) (rho the distance of q's projection onto the circle's plane from the centre, h its
    height above the plane), and the foot point is centre + R (q_plane - centre)/rho."""
    curves, _, circles = gen.curves_rational(13, n_random=0, n_circles=8, per_curve=4)
    rng = np.random.default_rng(1)
    for k, (c, R, nrm) in enumerate(circles):
        p, P, U = curves.curve(k)
        w = curves.weights[curves.cp_off[k]:curves.cp_off[k + 1]]
        X = oracle.nurbs_eval_curve(p, P, w, U, np.linspace(0, 1, 1001))
        np.testing.assert_allclose(np.linalg.norm(X - c, axis=1), R, atol=1e-14)
        q = c + rng.uniform(-0.6, 0.6, (200, 3))
        h = (q - c) @ nrm
        qp = q - h[:, None] * nrm
        rho = np.linalg.norm(qp - c, axis=1)
        keep = rho > 1e-3  # away from the axis, where every circle point is a minimum
        q, h, qp, rho = q[keep], h[keep], qp[keep], rho[keep]
        r = oracle.nurbs_project(curves.subset([k]), curves.weights[curves.cp_off[k]:curves.cp_off[k + 1]],
                                 np.zeros(len(q), np.int32), q)
        np.testing.assert_allclose(r["dist"], np.sqrt((rho - R) ** 2 + h ** 2), atol=1e-13)
        foot = c + R * (qp - c) / rho[:, None]
        Xt = oracle.nurbs_eval_curve(p, P, w, U, r["t"])
        ok = r["kappa"] > 1e-3
        np.testing.assert_allclose(Xt[ok], foot[ok], atol=1e-7)


def test_equal_weights_project_like_the_polynomial_curve():
    rng = np.random.default_rng(21)
    curves = gen.curves_batched_geometry(seed=21, n_curves=12, deg_lo=2, deg_hi=6, cp_lo=8, cp_hi=40)
    s = rng.uniform(0.5, 3.0, curves.n)  # one weight per curve: the rational curve is the polynomial one
    w = np.concatenate([np.full(curves.cp_off[i + 1] - curves.cp_off[i], s[i]) for i in range(curves.n)])
    cid = np.repeat(np.arange(curves.n, dtype=np.int32), 60)
    q = rng.uniform(-0.1, 1.1, (cid.shape[0], 3))
    ra, rp = oracle.nurbs_project(curves, w, cid, q), oracle.project(curves, cid, q)
    np.testing.assert_allclose(ra["dist"], rp["dist"], atol=1e-13)
    diag = curves.bbox_diag()[cid]
    ok = ((rp["runner"] - rp["dist"]) > 2e-6 * diag) & (rp["kappa"] > 1e-3)
    assert ok.mean() > 0.9
    np.testing.assert_allclose(ra["t"][ok], rp["t"][ok], atol=1e-9)
    np.testing.assert_allclose(ra["kappa"][ok], rp["kappa"][ok], rtol=1e-6, atol=1e-9)
    both_unique = ok & ((ra["runner"] - ra["dist"]) > 2e-6 * diag)
    assert both_unique.sum() >= 0.99 * ok.sum()


def test_rational_projection_against_dense_sampling():
    """Random NURBS: the oracle's distance lies between the densely sampled minimum (scipy quotient, 200k
    samples) and that minimum less half a sample step times the largest sampled speed times 1.5."""
    rng = np.random.default_rng(31)
    for p in (2, 3, 5):
        P, w, U = _random_nurbs(rng, p, p + 14)
        curves = gen._pack([p], [P], [U])
        q = rng.uniform(-0.1, 1.1, (60, 3))
        r = oracle.nurbs_project(curves, w, np.zeros(len(q), np.int32), q)
        num, den = BSpline(U, w[:, None] * P, p), BSpline(U, w, p)
        ts = np.linspace(0, 1, 200_001)
        X = num(ts) / den(ts)[:, None]
        sp = np.linalg.norm(np.diff(X, axis=0), axis=1).max()  # largest distance between neighbouring samples
        for i in range(len(q)):
            dmin = np.sqrt(((X - q[i]) ** 2).sum(1)).min()
            assert r["dist"][i] <= dmin + 1e-13
            assert r["dist"][i] >= dmin - sp - 1e-13


def test_weights_are_validated():
    P = np.random.default_rng(0).uniform(0, 1, (6, 3))
    U = np.array([0, 0, 0, 0, 0.4, 0.6, 1, 1, 1, 1.0])
    with pytest.raises(ValueError):
        oracle.nurbs_eval_curve(3, P, np.r_[np.ones(5), 0.0], U, [0.5])
    with pytest.raises(ValueError):
        oracle.nurbs_eval_curve(3, P, np.r_[np.ones(5), np.nan], U, [0.5])
