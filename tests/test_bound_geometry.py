"""The geometric facts the sphere-list bounds rest on, checked by brute force on seeded random cubic Bezier pieces
(numpy only, no GPU).  For a piece with control points P0..P3 and a query q:

- every point of the piece lies within rho of the chord P0P3, rho = the larger of P1's and P2's distances to the
  chord (the piece lies in the convex hull of its control points, which lies in that capsule), so
  dist(q, chord) - rho <= dist(q, piece);
- the sphere around any centre c with radius max |Pi - c| holds the piece, so |q - c| - r <= dist(q, piece) <= |q - c| + r;
- the distance to any point of the piece (B(0), B(1/3), B(2/3), B(1)) is an upper bound of dist(q, piece), and
  the best of the four lies within a sixth of the parameter range (times the largest speed) of the minimum.

dist(q, piece) is the minimum over 20,001 parameter samples refined by a golden-section search, which is within
1e-9 of the true minimum for these sizes."""
import numpy as np


def _bezier(P, t):
    t = np.asarray(t)[..., None]
    s = 1.0 - t
    return s**3 * P[0] + 3 * t * s * s * P[1] + 3 * t * t * s * P[2] + t**3 * P[3]


def _dist_piece(P, q, n=20001):
    t = np.linspace(0.0, 1.0, n)
    d = np.linalg.norm(_bezier(P, t) - q, axis=1)
    i = int(np.argmin(d))
    # golden-section refinement around the best sample
    a, b = t[max(i - 1, 0)], t[min(i + 1, n - 1)]
    f = lambda x: float(np.linalg.norm(_bezier(P, x) - q))
    g = (np.sqrt(5.0) - 1.0) / 2.0
    for _ in range(60):
        c, e = b - g * (b - a), a + g * (b - a)
        if f(c) < f(e):
            b = e
        else:
            a = c
    return min(d[i], f(0.5 * (a + b)))


def _seg_dist(v, a):
    aa = float(a @ a)
    t = 0.0 if aa == 0.0 else min(max(float(v @ a) / aa, 0.0), 1.0)
    return float(np.linalg.norm(v - t * a))


def _pieces(rng, n):
    out = []
    for k in range(n):
        kind = k % 4
        if kind == 0:  # generic
            P = rng.normal(size=(4, 3))
        elif kind == 1:  # nearly straight, long (the pieces beside a strut's nearest one)
            d = rng.normal(size=3)
            P = np.outer([0.0, 1.0, 2.0, 3.0], d) + 1e-3 * rng.normal(size=(4, 3))
        elif kind == 2:  # closed loop: P0 == P3, a zero chord
            P = rng.normal(size=(4, 3))
            P[3] = P[0]
        else:  # degenerate to a point
            P = np.repeat(rng.normal(size=(1, 3)), 4, axis=0)
        out.append(P)
    return out


def test_capsule_sphere_and_point_bounds():
    rng = np.random.default_rng(2504)
    worst_cap = worst_sph = -np.inf
    for P in _pieces(rng, 64):
        a = P[3] - P[0]
        rho = max(_seg_dist(P[1] - P[0], a), _seg_dist(P[2] - P[0], a))
        c = P.mean(axis=0) + 0.1 * rng.normal(size=3)
        r = float(np.max(np.linalg.norm(P - c, axis=1)))
        for q in rng.normal(size=(8, 3)) * rng.choice([0.1, 1.0, 10.0], size=(8, 1)):
            d = _dist_piece(P, q)
            cap = _seg_dist(q - P[0], a) - rho
            worst_cap = max(worst_cap, cap - d)
            sq = float(np.linalg.norm(q - c))
            worst_sph = max(worst_sph, sq - r - d, d - (sq + r))
            pts = _bezier(P, np.array([0.0, 1.0 / 3.0, 2.0 / 3.0, 1.0]))
            ub = float(np.min(np.linalg.norm(pts - q, axis=1)))
            assert ub >= d - 1e-12
            # within a sixth of the parameter range of the minimiser: |B'| <= 3 max |Pi+1 - Pi|
            speed = 3.0 * float(np.max(np.linalg.norm(np.diff(P, axis=0), axis=1)))
            assert ub <= d + speed / 6.0 + 1e-12
    assert worst_cap <= 1e-9, worst_cap
    assert worst_sph <= 1e-9, worst_sph


def test_capsule_is_tight_for_straight_pieces():
    """Beside the nearest piece of a straight run, the capsule bound is far above the sphere bound: the reason the
    list filter uses it (a query ten units off a straight run, two units along it from the piece: the sphere bound
    gives away nearly the whole radius, the capsule nothing)."""
    P = np.array([[2.0, 0, 0], [3.0, 0, 0], [4.0, 0, 0], [5.0, 0, 0]])  # the piece two to the right
    q = np.array([0.0, 10.0, 0.0])
    d = _dist_piece(P, q)
    a = P[3] - P[0]
    cap = _seg_dist(q - P[0], a) - 0.0
    c = P.mean(axis=0)
    sph = float(np.linalg.norm(q - c)) - float(np.max(np.linalg.norm(P - c, axis=1)))
    assert abs(cap - d) < 1e-9 and cap > sph + 1.0
