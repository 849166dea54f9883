"""Pins of the FP64 oracle at degrees 16..32, beyond the power form's reach.

The paper's GPU design stops at degree 31 (Sec. 6, discussion and limitations;
Sec. 7); the oracle and the library go to 32.  Independent sources: scipy's
B-spline and Bernstein evaluators, exact degree elevation (a degree-32 Bezier
curve that IS a cubic must project like the cubic), and dense brute force.
"""
import numpy as np
import pytest
from scipy.interpolate import BPoly, BSpline

import oracle
from paper_2504_11498_amd import gen


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build(force=False)


def _curve(rng, p, n_cp):
    P = rng.uniform(0, 1, (n_cp, 3))
    U = np.concatenate([np.zeros(p + 1), np.sort(rng.uniform(0.02, 0.98, n_cp - p - 1)), np.ones(p + 1)])
    return P, U


@pytest.mark.parametrize("p", [16, 24, 32])
def test_deboor_matches_scipy_high_degree(p):
    rng = np.random.default_rng(300 + p)
    P, U = _curve(rng, p, p + 12)
    t = np.concatenate([rng.uniform(0, 1, 200), [0.0, 1.0], U[p + 1:-p - 1]])
    X, D1, D2 = oracle.eval_curve(p, P, U, t, derivs=True)
    spl = BSpline(U, P, p)
    np.testing.assert_allclose(X, spl(t), atol=1e-12)
    np.testing.assert_allclose(D1, spl.derivative(1)(t), atol=1e-8 * np.abs(D1).max())
    np.testing.assert_allclose(D2, spl.derivative(2)(t), atol=1e-7 * np.abs(D2).max())
    for tt in t[:40]:
        N = oracle.basis(p, U, tt)
        assert np.all(N >= -1e-15) and abs(N.sum() - 1.0) <= 1e-13


@pytest.mark.parametrize("p", [20, 32])
def test_boehm_spans_high_degree(p):
    rng = np.random.default_rng(400 + p)
    P, U = _curve(rng, p, p + 9)
    bz, tab = oracle.bezier_spans(p, P, U)
    x = np.concatenate([tab[:, 0], tab[-1:, 1]])
    bp = BPoly(np.transpose(bz, (1, 0, 2)), x)
    t = np.linspace(0, 1, 2001)
    np.testing.assert_allclose(bp(t), BSpline(U, P, p)(t), atol=1e-12)


def _elevate(Q, to):
    """Exact Bezier degree elevation (each step a convex combination of neighbours), repeated up to degree ``to``."""
    while Q.shape[0] - 1 < to:
        p = Q.shape[0] - 1
        a = np.arange(p + 2)[:, None] / (p + 1)
        lo = np.vstack([np.zeros((1, 3)), Q])
        hi = np.vstack([Q, np.zeros((1, 3))])
        Q = a * lo + (1 - a) * hi
    return Q


def test_elevated_cubic_projects_like_the_cubic():
    """A degree-32 single-span curve obtained by elevating a cubic is the cubic: same projections."""
    rng = np.random.default_rng(7)
    Q3 = rng.uniform(0, 1, (4, 3))
    Q32 = _elevate(Q3.copy(), 32)
    c3 = gen._pack([3], [Q3], [np.r_[np.zeros(4), np.ones(4)]])
    c32 = gen._pack([32], [Q32], [np.r_[np.zeros(33), np.ones(33)]])
    q = rng.uniform(-0.2, 1.2, (400, 3))
    cid = np.zeros(400, np.int32)
    r3, r32 = oracle.project(c3, cid, q), oracle.project(c32, cid, q)
    np.testing.assert_allclose(r32["dist"], r3["dist"], atol=1e-13)
    diag = c3.bbox_diag()[0]
    ok = ((r3["runner"] - r3["dist"]) > 2e-6 * diag) & (r3["kappa"] > 1e-3)
    assert ok.mean() > 0.9
    np.testing.assert_allclose(r32["t"][ok], r3["t"][ok], atol=1e-9)
    # the elevated curve evaluates to the cubic (scipy, both degrees)
    t = np.linspace(0, 1, 101)
    np.testing.assert_allclose(BSpline(np.r_[np.zeros(33), np.ones(33)], Q32, 32)(t),
                               BSpline(np.r_[np.zeros(4), np.ones(4)], Q3, 3)(t), atol=1e-13)


def test_high_degree_projection_against_dense_sampling():
    """p = 24: the oracle's distance lies between the densely sampled minimum and that minimum less half a
    sample step times the largest speed (scipy evaluation, 400k samples)."""
    rng = np.random.default_rng(11)
    p = 24
    P, U = _curve(rng, p, p + 16)
    curves = gen._pack([p], [P], [U])
    q = rng.uniform(-0.1, 1.1, (120, 3))
    r = oracle.project(curves, np.zeros(len(q), np.int32), q)
    spl = BSpline(U, P, p)
    ts = np.linspace(0, 1, 400_001)
    X = spl(ts)
    vmax = np.linalg.norm(spl.derivative(1)(ts), axis=1).max()
    h = ts[1] - ts[0]
    for i in range(len(q)):
        d = np.sqrt(((X - q[i]) ** 2).sum(1))
        dmin = d.min()
        assert r["dist"][i] <= dmin + 1e-13
        assert r["dist"][i] >= dmin - 0.5 * h * vmax - 1e-13
