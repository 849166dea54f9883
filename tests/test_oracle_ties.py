"""Pins of the oracle's runner-up distance and conditioning (kappa) outputs.

These outputs decide where the parity tests demand parameter and piece-index
equality (a unique, well-conditioned minimiser), so they are pinned here
against closed forms, not against the oracle itself:

* the parabola y = x^2 as a quadratic Bezier curve, x = 2t - 1: a query
  (0, h) with 1/2 < h < 3/2 has two mirror minima x = +-sqrt(h - 1/2) at distance
  sqrt(h - 1/4) (runner = distance), kappa = (4h - 2)/(4h - 1); with h < 1/2
  the vertex is the only minimum (kappa = 1 - 2h); h = 1/2 is the vertex's
  centre of curvature (kappa = 0);
* a query off the mirror line: both minima from the real roots of the cubic
  g'(x) = 2x^3 + (1 - 2h)x - delta (numpy.roots, a textbook routine);
* a W-shaped polyline (degree 1, and the same W as a C0 quadratic with doubled
  knots): corner minima without a stationary point, distances in closed form;
* domain ends that are local minima (the parabola seen from far above);
* surfaces: the parabolic cylinder (2u - 1, v, (2u - 1)^2) with the same closed
  forms, the same cylinder split into two patches by an exact knot insertion
  (a point held on the shared patch side is not a second minimum), and a
  W-shaped crease surface whose corner lines are minima.

The global-minimiser definition with several correct answers is Sec. 4, eq.
projections; corner and end candidates are Sec. 5.3, Properties 1-2.
"""
import numpy as np
import pytest

import oracle
from paper_2504_11498_amd import gen


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build(force=False)


def _curve(p, P, U):
    return gen._pack([p], [np.asarray(P, float)], [np.asarray(U, float)])


PARABOLA = _curve(2, [[-1, 1, 0], [0, -1, 0], [1, 1, 0]], [0, 0, 0, 1, 1, 1])


def _proj(curves, q):
    q = np.atleast_2d(np.asarray(q, float))
    return oracle.project(curves, np.zeros(len(q), np.int32), q)


@pytest.mark.parametrize("h", [0.75, 1.0, 1.25, 1.45])
def test_mirror_parabola_runner_equals_distance(h):
    r = _proj(PARABOLA, [0.0, h, 0.0])
    d = np.sqrt(h - 0.25)
    x = np.sqrt(h - 0.5)
    assert abs(r["dist"][0] - d) <= 1e-14
    assert abs(r["runner"][0] - d) <= 1e-14  # the mirror minimum is an exact tie
    assert abs(r["t"][0] - (1 - x) / 2) <= 1e-12  # ties go to the smaller parameter
    assert abs(r["kappa"][0] - (4 * h - 2) / (4 * h - 1)) <= 1e-9


@pytest.mark.parametrize("h", [0.1, 0.3, 0.45])
def test_vertex_minimum_is_unique(h):
    r = _proj(PARABOLA, [0.0, h, 0.0])
    assert abs(r["dist"][0] - h) <= 1e-14
    assert abs(r["t"][0] - 0.5) <= 1e-12
    assert np.isinf(r["runner"][0])
    assert abs(r["kappa"][0] - (1 - 2 * h)) <= 1e-9


def test_centre_of_curvature_is_ill_conditioned():
    """q at the vertex's centre of curvature (0, 1/2): distance^2 - 1/4 = x^4, kappa = 0."""
    r = _proj(PARABOLA, [0.0, 0.5, 0.0])
    assert abs(r["dist"][0] - 0.5) <= 1e-14
    assert r["kappa"][0] < 1e-3
    assert abs(r["t"][0] - 0.5) <= 1e-3
    assert r["runner"][0] >= r["dist"][0] - 1e-15  # no other minimum, or the same flat valley


@pytest.mark.parametrize("delta,h", [(0.01, 1.0), (-0.02, 1.2), (0.001, 0.8), (0.05, 1.4)])
def test_off_mirror_runner_from_cubic_roots(delta, h):
    r = _proj(PARABOLA, [delta, h, 0.0])
    xs = [z.real for z in np.roots([2.0, 0.0, 1 - 2 * h, -delta]) if abs(z.imag) < 1e-12 and abs(z.real) <= 1]
    g2 = lambda x: 6 * x * x + 1 - 2 * h  # noqa: E731  (second derivative of g)
    mins = sorted(np.hypot(x - delta, x * x - h) for x in xs if g2(x) > 0)
    assert len(mins) == 2
    assert abs(r["dist"][0] - mins[0]) <= 1e-13
    assert abs(r["runner"][0] - mins[1]) <= 1e-12


def test_domain_ends_are_runner_candidates():
    """From (0, 3) the parabola's ends x = +-1 are the two minima on [-1, 1] (g' = x(2x^2 - 5) < 0 on (0, 1])."""
    r = _proj(PARABOLA, [0.0, 3.0, 0.0])
    assert abs(r["dist"][0] - np.sqrt(5.0)) <= 1e-14
    assert r["t"][0] == 0.0
    assert abs(r["runner"][0] - np.sqrt(5.0)) <= 1e-14
    assert r["kappa"][0] == 1.0


W_PTS = [[-2, 3, 0], [-1, 0, 0], [0, 3, 0], [1, 0, 0], [2, 3, 0]]


def _w_curves():
    """The W polyline (degree 1) and the same W as a quadratic with C0 joints (doubled knots, each leg a
    quadratic with equally spaced collinear control points, i.e. the linear parametrisation)."""
    lin = _curve(1, W_PTS, [0, 0, 0.25, 0.5, 0.75, 1, 1])
    P = np.asarray(W_PTS, float)
    Q = [P[0]]
    for k in range(4):
        Q += [(P[k] + P[k + 1]) / 2, P[k + 1]]
    quad = _curve(2, Q, [0, 0, 0, 0.25, 0.25, 0.5, 0.5, 0.75, 0.75, 1, 1, 1])
    return lin, quad


@pytest.mark.parametrize("delta", [0.0, 0.1, -0.25, 0.5])
def test_c0_corners_are_minima_and_runners(delta):
    """Below the W, both lower corners are minima: each leg leaves its corner uphill (the query lies in the
    corner's cone |x| < 3 |y|), and no leg has an interior foot point."""
    d_left = np.hypot(1 + delta, 1.0)   # corner (-1, 0) at t = 1/4
    d_right = np.hypot(1 - delta, 1.0)  # corner (1, 0) at t = 3/4
    for curves in _w_curves():
        r = _proj(curves, [delta, -1.0, 0.0])
        assert abs(r["dist"][0] - min(d_left, d_right)) <= 1e-14
        assert abs(r["t"][0] - (0.25 if d_left <= d_right else 0.75)) <= 1e-12
        assert abs(r["runner"][0] - max(d_left, d_right)) <= 1e-14
        assert r["kappa"][0] == 1.0


def test_c0_corner_with_interior_runner():
    """Query (0.3, 2) near the middle peak: every leg has an interior foot point (closed-form segment
    projection); the nearest is the minimum, the second nearest the runner-up, and no corner or end is a
    minimum from there."""
    q = np.array([0.3, 2.0, 0.0])

    def seg_foot(a, b):
        a, b = np.asarray(a, float), np.asarray(b, float)
        s = np.clip((q - a) @ (b - a) / ((b - a) @ (b - a)), 0, 1)
        return np.linalg.norm(a + s * (b - a) - q), s

    feet = [seg_foot(W_PTS[k], W_PTS[k + 1]) for k in range(4)]
    interior = sorted(d for d, s in feet if 0 < s < 1)
    for curves in _w_curves():
        r = _proj(curves, q)
        assert abs(r["dist"][0] - interior[0]) <= 1e-14
        assert abs(r["runner"][0] - interior[1]) <= 1e-13


# --------------------------------------------------------------------------- surfaces
def _surface(p, q, nu, nv, P, U, V):
    P = np.asarray(P, float).reshape(-1, 3)
    return gen.SurfaceSet(np.array([p], np.int32), np.array([q], np.int32), np.array([nu], np.int32),
                          np.array([nv], np.int32), np.array([0, nu * nv], np.int64), P,
                          np.array([0, len(U)], np.int64), np.asarray(U, float), np.array([0, len(V)], np.int64),
                          np.asarray(V, float))


def _cylinder(split):
    """(2u - 1, v, (2u - 1)^2) on [0,1]^2, quadratic in both directions (linear in v by linear precision).
    split: the u knot 1/2 inserted (exact), giving two patches."""
    xz = np.array([[-1, 1], [0, -1], [1, 1]], float)
    U = [0, 0, 0, 1, 1, 1]
    if split:
        xz = np.array([xz[0], (xz[0] + xz[1]) / 2, (xz[1] + xz[2]) / 2, xz[2]])
        U = [0, 0, 0, 0.5, 1, 1, 1]
    ys = [0.0, 0.5, 1.0]
    P = [[x, y, z] for x, z in xz for y in ys]
    return _surface(2, 2, len(xz), 3, P, U, [0, 0, 0, 1, 1, 1])


def _sproj(S, x):
    x = np.atleast_2d(np.asarray(x, float))
    return oracle.surf_project(S, np.zeros(len(x), np.int32), x)


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("h", [0.75, 1.25])
def test_surface_mirror_runner_equals_distance(split, h):
    S = _cylinder(split)
    r = _sproj(S, [0.0, 0.4, h])
    d = np.sqrt(h - 0.25)
    x = np.sqrt(h - 0.5)
    assert abs(r["dist"][0] - d) <= 1e-13
    assert abs(r["runner"][0] - d) <= 1e-12
    # either mirror point (the two distances agree to rounding, which decides between the patches)
    u = r["uv"][0][0]
    assert min(abs(u - (1 - x) / 2), abs(u - (1 + x) / 2)) <= 1e-9 and abs(r["uv"][0][1] - 0.4) <= 1e-9
    assert abs(r["kappa"][0] - (4 * h - 2) / (4 * h - 1)) <= 1e-8


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("delta", [0.0, 0.001, -0.003])
def test_surface_unique_near_patch_side(split, delta):
    """h = 0.3 < 1/2: a single minimum near x = delta / 0.4, next to the split's shared side at u = 1/2. The
    other patch stops on that side with the gradient pointing across (distance only ~4e-6 larger): it is not a
    second minimum of the surface."""
    h = 0.3
    S = _cylinder(split)
    r = _sproj(S, [delta, 0.6, h])
    xs = [z.real for z in np.roots([2.0, 0.0, 1 - 2 * h, -delta]) if abs(z.imag) < 1e-12 and abs(z.real) <= 1]
    assert len(xs) == 1
    assert abs(r["dist"][0] - np.hypot(xs[0] - delta, xs[0] ** 2 - h)) <= 1e-13
    assert np.isinf(r["runner"][0])


def test_surface_crease_minima():
    """The W polyline of the curve tests extruded along y (degree 1 x 1): both lower creases are minima. The
    surface oracle reports a runner-up within its uniqueness margin (3e-6 of the box diagonal) exactly and
    may report inf beyond it."""
    P = [[x, y, z] for x, z, _ in W_PTS for y in (0.0, 1.0)]
    S = _surface(1, 1, 5, 2, P, [0, 0, 0.25, 0.5, 0.75, 1, 1], [0, 0, 1, 1])
    margin = 3e-6 * np.linalg.norm(np.ptp(np.asarray(P, float), axis=0))
    for delta in (0.0, 1e-7, -3e-7, 0.1, -0.2):
        r = _sproj(S, [delta, 0.5, -1.0])
        dl, dr = np.hypot(1 + delta, 1.0), np.hypot(1 - delta, 1.0)
        assert abs(r["dist"][0] - min(dl, dr)) <= 1e-13
        if max(dl, dr) - min(dl, dr) < margin:
            assert abs(r["runner"][0] - max(dl, dr)) <= 1e-12
        else:
            assert np.isinf(r["runner"][0]) or abs(r["runner"][0] - max(dl, dr)) <= 1e-12


# --------------------------------------------------------------------------- C0 quadratics, every minimum by roots
def _quadratic_minima(P, U, q):
    """Every local minimum of |C(t) - q| on a quadratic B-spline, from closed forms per span.

    On a span the curve is C(x) = A x^2 + B x + D (x in [0, 1], taken exactly through three points
    of scipy's evaluation), so f(x) = (C - q).C' = 2|A|^2 x^3 + 3 A.B x^2 + (|B|^2 + 2 A.(D - q)) x
    + B.(D - q) is a cubic whose real roots (numpy.roots) with f' > 0 are the stationary minima.
    A C0 joint is a minimum when the left span's f at its end is negative and the right span's f at
    its start positive; a domain end when f points into the domain.  Returns [(t, dist)]."""
    from scipy.interpolate import BSpline

    bs = BSpline(np.asarray(U, float), np.asarray(P, float), 2)
    ks = [k for k in range(2, len(U) - 3) if U[k] < U[k + 1]]
    mins, ends = [], []
    for k in ks:
        a, b = U[k], U[k + 1]
        x = np.array([a, 0.5 * (a + b), b])
        X = np.stack([bs(t) for t in x])
        # the span's own polynomial through C(a), C(mid), C(b) (continuous at the ends)
        P0, Pm, P2 = X[0], X[1], X[2]
        P1 = 2.0 * Pm - 0.5 * (P0 + P2)
        A, B, D = P0 - 2 * P1 + P2, 2 * (P1 - P0), P0
        r = D - q
        coef = [2 * (A @ A), 3 * (A @ B), B @ B + 2 * (A @ r), B @ r]
        f = lambda s: np.polyval(coef, s)  # noqa: E731
        fp = lambda s: 6 * (A @ A) * s * s + 6 * (A @ B) * s + B @ B + 2 * (A @ r)  # noqa: E731
        for z in np.roots(coef):
            if abs(z.imag) < 1e-9 and 0.0 < z.real < 1.0 and fp(z.real) > 0:
                s = z.real
                mins.append((a + s * (b - a), np.linalg.norm(A * s * s + B * s + r)))
        ends.append((a, b, f(0.0), f(1.0), np.linalg.norm(r), np.linalg.norm(A + B + r)))
    for (a0, b0, f00, f01, d00, d01), (a1, b1, f10, f11, d10, d11) in zip(ends[:-1], ends[1:]):
        if f01 < 0.0 and f10 > 0.0:
            mins.append((b0, d01))
    if ends[0][2] >= 0.0:
        mins.append((ends[0][0], ends[0][4]))
    if ends[-1][3] <= 0.0:
        mins.append((ends[-1][1], ends[-1][5]))
    return mins


def test_c0_quadratic_runner_from_cubic_roots():
    """The corner family of the adversarial workload (C0 quadratics, queries next to the joints):
    the oracle's distance and runner-up equal the best and the best distinct (|t - t*| > 1e-6) of all
    closed-form local minima.  This includes minima inside a span a few 1e-6 from a C0 joint, where
    the one-sided derivatives of the two spans differ."""
    from scipy.interpolate import BSpline

    curves, o = gen.curves_adversarial()
    cids = np.asarray(o["corner_cid"])
    q = np.empty((len(cids), 3))
    for i, (c, t0, off) in enumerate(zip(cids, o["corner_t0"], o["corner_offset"])):
        p, P, U = curves.curve(c)
        q[i] = BSpline(np.asarray(U, float), np.asarray(P, float), p)(t0) + off
    r = oracle.project(curves, cids.astype(np.int32), q)
    checked_close = 0
    for i, c in enumerate(cids):
        p, P, U = curves.curve(c)
        assert p == 2
        mins = _quadratic_minima(P, U, q[i])
        t_best, d_best = min(mins, key=lambda m: m[1])
        others = [d for t, d in mins if abs(t - t_best) > 1e-6]
        runner = min(others) if others else np.inf
        diag = curves.bbox_diag()[c]
        assert abs(r["dist"][i] - d_best) <= 1e-12 * diag, i
        if np.isfinite(runner):
            assert abs(r["runner"][i] - runner) <= 1e-11 * diag, (i, r["runner"][i], runner)
            checked_close += runner - d_best <= 4e-6 * diag
        else:
            assert np.isinf(r["runner"][i])
    assert checked_close >= 1  # at least one runner-up within the tie margin (next to a joint)
