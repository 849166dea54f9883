"""Seeded synthetic workloads for B-spline point projection and inversion.

This module only draws random geometry and random query *recipes*.  It holds
none of the projection method's arithmetic: it never evaluates a curve or a
surface.  Where a query is "a point on the curve plus an offset", the generator
returns the drawn parameter and the drawn offset; whoever consumes the workload
evaluates the geometry with its own evaluator and adds the offset.  Both the
CPU oracle and the GPU path consume the same draws.

Workloads (the paper's problem statement, Sec. 4, fixes the inputs: a degree,
control points, a clamped knot vector and a set of query points):

* ``curve_single``   -- one clamped cubic curve, 16 control points uniform in
  [0,1]^3, clamped uniform knots (13 spans); 10,000 queries uniform in the
  control-point box scaled by 1.1 about its centre.
* ``curves_batched`` -- 4,096 curves of degree U{2..7}, control-point count
  log-uniform in [8, 256], non-uniform clamped knots from normalised cumulative
  Exp(1) increments with 10% of the interior knots doubled; 256 queries per
  curve, each a Gaussian offset (sigma = 0.05 * box diagonal) from a
  parameter-uniform point on the curve.
* ``surfaces``       -- 256 height-field surfaces, degree 3x3 or 5x5 on a 32x32
  net (sum of four random sinusoids plus N(0, 0.02)), non-uniform clamped knots
  in u and v; queries half on-surface, half offset.
* ``curves_lattice`` -- 65,536 random-walk strut curves of degree U{3..9} with
  U{64..1024} control points; queries split in proportion to a caller-supplied
  weight per curve (the cubic segment count).

All draws use numpy's PCG64 generator.  Parameters are on the normalised knot
domain [0, 1].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class CurveSet:
    """CSR batch of clamped B-spline curves (FP64, xyz interleaved)."""

    degree: np.ndarray  # int32 [n]
    cp_off: np.ndarray  # int64 [n+1]
    cp: np.ndarray  # float64 [cp_off[-1], 3]
    knot_off: np.ndarray  # int64 [n+1]
    knots: np.ndarray  # float64 [knot_off[-1]]
    weights: np.ndarray | None = None  # float64 [cp_off[-1]]: rational curves (NURBS), else None

    @property
    def n(self) -> int:
        return int(self.degree.shape[0])

    def curve(self, i: int):
        p = int(self.degree[i])
        P = self.cp[self.cp_off[i] : self.cp_off[i + 1]]
        U = self.knots[self.knot_off[i] : self.knot_off[i + 1]]
        return p, P, U

    def bbox_diag(self) -> np.ndarray:
        """Diagonal length of each curve's control-point box (per curve)."""
        out = np.empty(self.n)
        for i in range(self.n):
            P = self.cp[self.cp_off[i] : self.cp_off[i + 1]]
            out[i] = float(np.linalg.norm(P.max(0) - P.min(0)))
        return out

    def subset(self, ids) -> "CurveSet":
        ids = np.asarray(ids, dtype=np.int64)
        deg = self.degree[ids].astype(np.int32)
        cps = [self.cp[self.cp_off[i] : self.cp_off[i + 1]] for i in ids]
        kts = [self.knots[self.knot_off[i] : self.knot_off[i + 1]] for i in ids]
        cp_off = np.zeros(len(ids) + 1, np.int64)
        cp_off[1:] = np.cumsum([len(c) for c in cps])
        k_off = np.zeros(len(ids) + 1, np.int64)
        k_off[1:] = np.cumsum([len(k) for k in kts])
        w = None
        if self.weights is not None:
            w = np.concatenate([self.weights[self.cp_off[i] : self.cp_off[i + 1]] for i in ids])
        return CurveSet(deg, cp_off, np.concatenate(cps).reshape(-1, 3), k_off, np.concatenate(kts), w)


@dataclass
class CurveQueries:
    """Query recipe: q = C_{curve_id}(t0) + offset when ``on_curve_base`` else q = point."""

    curve_id: np.ndarray  # int32 [N]
    t0: np.ndarray | None = None  # float64 [N] parameter on the normalised domain
    offset: np.ndarray | None = None  # float64 [N,3]
    point: np.ndarray | None = None  # float64 [N,3] absolute query points (box-uniform workloads)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.curve_id.shape[0])

    def materialise(self, eval_fn) -> np.ndarray:
        """Return q [N,3] float64, evaluating base points with the caller's ``eval_fn(curve_id, t) -> [N,3]``."""
        if self.point is not None:
            return np.ascontiguousarray(self.point, dtype=np.float64)
        base = eval_fn(self.curve_id, self.t0)
        return np.ascontiguousarray(base + self.offset, dtype=np.float64)


def _clamped(interior: np.ndarray, p: int) -> np.ndarray:
    return np.concatenate([np.zeros(p + 1), np.sort(interior), np.ones(p + 1)])


def _exp_interior(rng: np.random.Generator, n_distinct: int) -> np.ndarray:
    """n_distinct interior knots in (0,1): normalised cumulative sums of Exp(1) increments."""
    if n_distinct <= 0:
        return np.zeros(0)
    inc = rng.exponential(1.0, n_distinct + 1)
    cs = np.cumsum(inc)
    return cs[:-1] / cs[-1]


def _pack(degrees, cps, knots) -> CurveSet:
    n = len(degrees)
    cp_off = np.zeros(n + 1, np.int64)
    cp_off[1:] = np.cumsum([len(c) for c in cps])
    k_off = np.zeros(n + 1, np.int64)
    k_off[1:] = np.cumsum([len(k) for k in knots])
    return CurveSet(
        np.asarray(degrees, np.int32),
        cp_off,
        np.ascontiguousarray(np.concatenate(cps).reshape(-1, 3), dtype=np.float64),
        k_off,
        np.ascontiguousarray(np.concatenate(knots), dtype=np.float64),
    )


# ---------------------------------------------------------------------------
# One cubic curve, box-uniform queries
# ---------------------------------------------------------------------------
def curve_single(seed: int = 1, n_queries: int = 10_000, n_cp: int = 16, degree: int = 3):
    rng = np.random.default_rng(seed)
    P = rng.uniform(0.0, 1.0, (n_cp, 3))
    n_spans = n_cp - degree
    interior = np.arange(1, n_spans) / n_spans
    U = _clamped(interior, degree)
    curves = _pack([degree], [P], [U])
    lo, hi = P.min(0), P.max(0)
    c, h = 0.5 * (lo + hi), 0.5 * (hi - lo) * 1.1
    q = rng.uniform(c - h, c + h, (n_queries, 3))
    return curves, CurveQueries(np.zeros(n_queries, np.int32), point=q, meta={"kind": "box"})


# ---------------------------------------------------------------------------
# Thousands of curves of uneven degree and length
# ---------------------------------------------------------------------------
def curves_batched_geometry(seed: int = 2, n_curves: int = 4096, deg_lo: int = 2, deg_hi: int = 7,
                            cp_lo: int = 8, cp_hi: int = 256, dup_frac: float = 0.1) -> CurveSet:
    rng = np.random.default_rng(seed)
    degs, cps, kts = [], [], []
    for _ in range(n_curves):
        p = int(rng.integers(deg_lo, deg_hi + 1))
        n_cp = int(round(float(np.exp(rng.uniform(np.log(cp_lo), np.log(cp_hi))))))
        n_cp = max(n_cp, p + 1)
        P = rng.uniform(0.0, 1.0, (n_cp, 3))
        n_int = n_cp - p - 1
        n_dup = int(round(dup_frac * n_int))
        # doubling a knot keeps the total count: n_int - n_dup distinct values, n_dup of them doubled
        n_dup = min(n_dup, max(n_int - n_dup, 0))
        n_dist = n_int - n_dup
        base = _exp_interior(rng, n_dist)
        if n_dup > 0:
            dup = rng.choice(n_dist, size=n_dup, replace=False)
            interior = np.concatenate([base, base[dup]])
        else:
            interior = base
        degs.append(p)
        cps.append(P)
        kts.append(_clamped(interior, p))
    return _pack(degs, cps, kts)


def offset_queries(seed: int, curves: CurveSet, per_curve=None, counts=None, sigma_rel: float = 0.05,
                   on_curve_frac: float = 0.0) -> CurveQueries:
    """Queries q = C(t0) + N(0, (sigma_rel*bbox)^2 I3), t0 ~ U(0,1), grouped by curve.

    ``counts`` (per curve) overrides ``per_curve``.  A fraction ``on_curve_frac`` of each curve's
    queries get a zero offset (inversion queries).
    """
    rng = np.random.default_rng(seed)
    if counts is None:
        counts = np.full(curves.n, int(per_curve), np.int64)
    counts = np.asarray(counts, np.int64)
    cid = np.repeat(np.arange(curves.n, dtype=np.int32), counts)
    n = cid.shape[0]
    t0 = rng.uniform(0.0, 1.0, n)
    diag = curves.bbox_diag()
    off = rng.standard_normal((n, 3)) * (sigma_rel * diag[cid])[:, None]
    on = np.zeros(n, bool)
    if on_curve_frac > 0:
        on = rng.uniform(0.0, 1.0, n) < on_curve_frac
        off[on] = 0.0
    return CurveQueries(cid, t0=t0, offset=off, meta={"kind": "offset", "sigma_rel": sigma_rel, "on_curve": on})


def curves_batched(seed: int = 2, n_curves: int = 4096, per_curve: int = 256):
    curves = curves_batched_geometry(seed, n_curves)
    return curves, offset_queries(seed + 100, curves, per_curve=per_curve)


# ---------------------------------------------------------------------------
# Lattice struts: long random-walk curves of high degree
# ---------------------------------------------------------------------------
def curves_lattice_geometry(seed: int = 5, n_curves: int = 65_536, deg_lo: int = 3, deg_hi: int = 9,
                            cp_lo: int = 64, cp_hi: int = 1024, step: float = 0.01) -> CurveSet:
    rng = np.random.default_rng(seed)
    degs, cps, kts = [], [], []
    for _ in range(n_curves):
        p = int(rng.integers(deg_lo, deg_hi + 1))
        n_cp = int(rng.integers(cp_lo, cp_hi + 1))
        P0 = rng.uniform(0.0, 1.0, 3)
        P = P0 + np.concatenate([np.zeros((1, 3)), np.cumsum(rng.standard_normal((n_cp - 1, 3)) * step, 0)])
        degs.append(p)
        cps.append(P)
        kts.append(_clamped(_exp_interior(rng, n_cp - p - 1), p))
    return _pack(degs, cps, kts)


def proportional_counts(weights, total: int) -> np.ndarray:
    """Split ``total`` queries in proportion to ``weights`` (largest remainder)."""
    w = np.asarray(weights, np.float64)
    share = w / w.sum() * total
    base = np.floor(share).astype(np.int64)
    rem = total - int(base.sum())
    order = np.argsort(-(share - base), kind="stable")
    base[order[:rem]] += 1
    return base


# ---------------------------------------------------------------------------
# Height-field surfaces
# ---------------------------------------------------------------------------
@dataclass
class SurfaceSet:
    deg_u: np.ndarray  # int32 [n]
    deg_v: np.ndarray  # int32 [n]
    n_u: np.ndarray  # int32 [n] control points along u
    n_v: np.ndarray  # int32 [n]
    cp_off: np.ndarray  # int64 [n+1] offset in points; net stored u-major: P[i*n_v + j]
    cp: np.ndarray  # float64 [.., 3]
    ku_off: np.ndarray
    ku: np.ndarray
    kv_off: np.ndarray
    kv: np.ndarray

    @property
    def n(self) -> int:
        return int(self.deg_u.shape[0])


def surfaces(seed: int = 3, n_surf: int = 256, net: int = 32, per_surface: int = 16_384):
    rng = np.random.default_rng(seed)
    du, dv, nu, nv, cps, kus, kvs = [], [], [], [], [], [], []
    x = np.arange(net) / (net - 1)
    X, Y = np.meshgrid(x, x, indexing="ij")
    for s in range(n_surf):
        p = 3 if s % 2 == 0 else 5
        a = rng.uniform(0.05, 0.25, 4)
        f = rng.uniform(0.5, 3.0, (4, 2))
        ph = rng.uniform(0.0, 2 * np.pi, 4)
        Z = sum(a[k] * np.sin(2 * np.pi * (f[k, 0] * X + f[k, 1] * Y) + ph[k]) for k in range(4))
        Z = Z + rng.normal(0.0, 0.02, Z.shape)
        P = np.stack([X, Y, Z], -1).reshape(-1, 3)
        du.append(p)
        dv.append(p)
        nu.append(net)
        nv.append(net)
        cps.append(P)
        kus.append(_clamped(_exp_interior(rng, net - p - 1), p))
        kvs.append(_clamped(_exp_interior(rng, net - p - 1), p))
    n = n_surf
    cp_off = np.zeros(n + 1, np.int64)
    cp_off[1:] = np.cumsum([len(c) for c in cps])
    ku_off = np.zeros(n + 1, np.int64)
    ku_off[1:] = np.cumsum([len(k) for k in kus])
    kv_off = np.zeros(n + 1, np.int64)
    kv_off[1:] = np.cumsum([len(k) for k in kvs])
    surf = SurfaceSet(np.array(du, np.int32), np.array(dv, np.int32), np.array(nu, np.int32),
                      np.array(nv, np.int32), cp_off, np.concatenate(cps), ku_off, np.concatenate(kus),
                      kv_off, np.concatenate(kvs))
    sid = np.repeat(np.arange(n, dtype=np.int32), per_surface)
    m = sid.shape[0]
    uv0 = rng.uniform(0.0, 1.0, (m, 2))
    on = (np.arange(m) % per_surface) < per_surface // 2
    diag = np.array([np.linalg.norm(c.max(0) - c.min(0)) for c in cps])
    off = rng.standard_normal((m, 3)) * (0.05 * diag[sid])[:, None]
    off[on] = 0.0
    return surf, {"surface_id": sid, "uv0": uv0, "offset": off, "on_surface": on}


# ---------------------------------------------------------------------------
# Adversarial workloads: several correct answers, corners, poor conditioning
# ---------------------------------------------------------------------------
def _mirror_x(P: np.ndarray) -> np.ndarray:
    """Mirror points in the plane x = 1/2."""
    M = P.copy()
    M[:, 0] = 1.0 - M[:, 0]
    return M


def _mirror_net(half: np.ndarray, mid: np.ndarray | None) -> np.ndarray:
    """Control polygon symmetric about x = 1/2: half, the optional middle point, the mirrored half reversed."""
    parts = [half] + ([mid[None, :]] if mid is not None else []) + [_mirror_x(half)[::-1]]
    return np.concatenate(parts)


def _mirror_knots(rng: np.random.Generator, n_int: int, double: bool = False) -> np.ndarray:
    """n_int interior knot slots symmetric about 1/2 (each value twice when double)."""
    per = 2 if double else 1
    k = n_int // per
    h = _exp_interior(rng, k // 2) * 0.5 * (1.0 - 0.1 * rng.uniform())  # strictly inside (0, 1/2)
    vals = np.concatenate([h, [0.5] if k % 2 else [], 1.0 - h[::-1]])
    return np.repeat(vals, per)


def curves_adversarial(seed: int = 9):
    """Curves and query recipes where the projection has several correct answers or a poorly
    conditioned one (the global-minimiser definition with ties, Sec. 4 eq. projections; corner and
    end candidates, Sec. 5.3 Properties 1-2).  Families (curve ids in ``fam``):

    * ``mirror``  -- 48 curves symmetric about the plane x = 1/2 (degree 2, 3, 4, 5 or 7, 8..40
      control points, symmetric non-uniform knots); 24 queries each uniform on that plane within the
      control box scaled by 1.1: the distance is even about t = 1/2, so the minimum is either at
      t = 1/2 or one of a mirror pair (an exact tie);
    * ``corner``  -- 24 mirror-symmetric quadratics with every interior knot doubled (only C0 at
      each joint); 16 queries each: a joint parameter plus an N(0, (0.03 diag)^2) offset, so many
      minima sit on a corner with no stationary point;
    * ``hairpin`` -- 8 cubic hairpins (two legs 0.4 apart joined by a bend, symmetric about
      x = 1/2); 32 queries each on the mirror plane between the legs: equidistant from both legs;
    * ``centre``  -- near centres of curvature, q = C(t0) + s R N (R the radius of curvature, N the
      principal normal): on 32 mirror curves at t0 = 1/2 (two queries with s ~ U[0.9985, 0.9995], six
      with s ~ U[0.97, 0.999]) and on 32 random cubic curves at random t0 (s ~ U[0.9, 1.0]); 8 queries
      each.  The caller places q with its own evaluator (``centre_cid``, ``centre_t0``, ``centre_s``).

    Returns (CurveSet, dict): ``point``/``point_cid`` for the absolute queries (mirror, hairpin),
    ``corner_cid``/``corner_t0``/``corner_offset`` and the ``centre_*`` recipes, and ``fam``."""
    rng = np.random.default_rng(seed)
    degs, cps, kts, fam = [], [], [], {"mirror": [], "corner": [], "hairpin": [], "centre_sym": [], "centre": []}

    def add(name, p, P, U):
        fam[name].append(len(degs))
        degs.append(p)
        cps.append(P)
        kts.append(U)

    def mirror_curve(p, n):
        half = rng.uniform(0.0, 1.0, (n // 2, 3))
        half[:, 0] = rng.uniform(0.0, 0.45, n // 2)
        mid = np.array([0.5, rng.uniform(), rng.uniform()]) if n % 2 else None
        P = _mirror_net(half, mid)
        U = _clamped(_mirror_knots(rng, n - p - 1), p)
        return P, U

    for i in range(48):
        p = [2, 3, 4, 5, 7][i % 5]
        n = int(rng.integers(max(p + 1, 8), 41))
        add("mirror", p, *mirror_curve(p, n))
    for i in range(24):
        k = int(rng.integers(3, 10))  # distinct interior knots, each doubled
        n = 3 + 2 * k
        half = rng.uniform(0.0, 1.0, (n // 2, 3))
        half[:, 0] = rng.uniform(0.0, 0.45, n // 2)
        mid = np.array([0.5, rng.uniform(), rng.uniform()])
        add("corner", 2, _mirror_net(half, mid), _clamped(_mirror_knots(rng, n - 3, double=True), 2))
    for i in range(8):
        ys = np.array([0.0, 0.2, 0.4, 0.6, 0.8, 0.95])
        half = np.stack([0.3 + np.array([0, 0, 0, 0, 0, 0.06]), ys, np.full(6, 0.5)], 1)
        half[:, 1:] += rng.normal(0.0, 0.01, (6, 2))
        half[-1, 0] += rng.uniform(0.0, 0.04)
        P = _mirror_net(half, None)
        add("hairpin", 3, P, _clamped(np.arange(1, 9) / 9.0, 3))
    for i in range(32):
        p = [3, 4, 5][i % 3]
        add("centre_sym", p, *mirror_curve(p, int(rng.integers(9, 30))))
    for i in range(32):
        n = int(rng.integers(8, 24))
        add("centre", 3, rng.uniform(0.0, 1.0, (n, 3)), _clamped(_exp_interior(rng, n - 4), 3))

    curves = _pack(degs, cps, kts)
    diag = curves.bbox_diag()
    out = {"fam": {k: np.array(v, np.int32) for k, v in fam.items()}}
    pts, pcid = [], []
    for c in fam["mirror"]:
        P = cps[c]
        lo, hi = P.min(0), P.max(0)
        ctr, half = 0.5 * (lo + hi), 0.55 * (hi - lo)
        q = rng.uniform(ctr - half, ctr + half, (24, 3))
        q[:, 0] = 0.5
        pts.append(q)
        pcid.append(np.full(24, c, np.int32))
    for c in fam["hairpin"]:
        q = np.stack([np.full(32, 0.5), rng.uniform(0.05, 0.75, 32), 0.5 + rng.uniform(-0.05, 0.05, 32)], 1)
        pts.append(q)
        pcid.append(np.full(32, c, np.int32))
    out["point"] = np.concatenate(pts)
    out["point_cid"] = np.concatenate(pcid)
    ccid, ct0, coff = [], [], []
    for c in fam["corner"]:
        U = kts[c]
        joints = np.unique(U[3:-3])
        ccid.append(np.full(16, c, np.int32))
        ct0.append(rng.choice(joints, 16))
        coff.append(rng.normal(0.0, 0.03 * diag[c], (16, 3)))
    out["corner_cid"], out["corner_t0"], out["corner_offset"] = np.concatenate(ccid), np.concatenate(ct0), np.concatenate(coff)
    zcid, zt0, zs = [], [], []
    for c in fam["centre_sym"]:
        zcid.append(np.full(8, c, np.int32))
        zt0.append(np.full(8, 0.5))
        zs.append(np.concatenate([rng.uniform(0.9985, 0.9995, 2), rng.uniform(0.97, 0.999, 6)]))
    for c in fam["centre"]:
        zcid.append(np.full(8, c, np.int32))
        zt0.append(rng.uniform(0.1, 0.9, 8))
        zs.append(rng.uniform(0.9, 1.0, 8))
    out["centre_cid"], out["centre_t0"], out["centre_s"] = np.concatenate(zcid), np.concatenate(zt0), np.concatenate(zs)
    return curves, out


def surfaces_mirror(seed: int = 10, n_surf: int = 8, net: int = 32, per_surface: int = 160):
    """Height fields symmetric about the plane x = 1/2 (z(x, y) = g(x, y) + g(1 - x, y) with g four random
    sinusoids; knots in u symmetric about 1/2, in v from Exp(1) increments; degree 3x3 and 5x5 alternating)
    and queries on that plane: (1/2, y, z) with y ~ U[0, 1] and z uniform over the net's z range widened by
    half of it on each side.  The distance is even about u = 1/2, so the minimum is on the mirror or one of a
    mirror pair (an exact tie).  Returns (SurfaceSet, sid, q)."""
    rng = np.random.default_rng(seed)
    du, dv, nu, nv, cps, kus, kvs = [], [], [], [], [], [], []
    x = np.arange(net) / (net - 1)
    X, Y = np.meshgrid(x, x, indexing="ij")
    qs, sids = [], []
    for s in range(n_surf):
        p = 3 if s % 2 == 0 else 5
        a = rng.uniform(0.05, 0.2, 4)
        f = rng.uniform(0.5, 2.5, (4, 2))
        ph = rng.uniform(0.0, 2 * np.pi, 4)

        def g(Xa, Ya):
            return sum(a[k] * np.sin(2 * np.pi * (f[k, 0] * Xa + f[k, 1] * Ya) + ph[k]) for k in range(4))

        Z = g(X, Y) + g(X[::-1, :], Y)  # X[::-1] holds 1 - x exactly on this grid
        P = np.stack([X, Y, Z], -1).reshape(-1, 3)
        du.append(p)
        dv.append(p)
        nu.append(net)
        nv.append(net)
        cps.append(P)
        kus.append(_clamped(_mirror_knots(rng, net - p - 1), p))
        kvs.append(_clamped(_exp_interior(rng, net - p - 1), p))
        zlo, zhi = Z.min(), Z.max()
        w = zhi - zlo
        q = np.stack([np.full(per_surface, 0.5), rng.uniform(0.0, 1.0, per_surface),
                      rng.uniform(zlo - 0.5 * w, zhi + 0.5 * w, per_surface)], 1)
        qs.append(q)
        sids.append(np.full(per_surface, s, np.int32))
    n = n_surf
    cp_off = np.zeros(n + 1, np.int64)
    cp_off[1:] = np.cumsum([len(c) for c in cps])
    ku_off = np.zeros(n + 1, np.int64)
    ku_off[1:] = np.cumsum([len(k) for k in kus])
    kv_off = np.zeros(n + 1, np.int64)
    kv_off[1:] = np.cumsum([len(k) for k in kvs])
    surf = SurfaceSet(np.array(du, np.int32), np.array(dv, np.int32), np.array(nu, np.int32),
                      np.array(nv, np.int32), cp_off, np.concatenate(cps), ku_off, np.concatenate(kus),
                      kv_off, np.concatenate(kvs))
    return surf, np.concatenate(sids), np.concatenate(qs)


def curves_high_degree(seed: int = 11, degrees=(16, 20, 24, 28, 32), per_degree: int = 4, cp_extra=(1, 24),
                       per_curve: int = 128):
    """Curves of degree 16..32 (beyond the power form's reach): per degree, ``per_degree`` curves with
    p + 1 + U{cp_extra} control points uniform in [0,1]^3 and Exp(1) knots (the first curve of each degree a
    single Bezier span), and ``per_curve`` offset queries each (sigma = 0.05 * diag, a quarter on the curve)."""
    rng = np.random.default_rng(seed)
    degs, cps, kts = [], [], []
    for p in degrees:
        for k in range(per_degree):
            n_cp = p + 1 + (0 if k == 0 else int(rng.integers(cp_extra[0], cp_extra[1] + 1)))
            degs.append(int(p))
            cps.append(rng.uniform(0.0, 1.0, (n_cp, 3)))
            kts.append(_clamped(_exp_interior(rng, n_cp - p - 1), int(p)))
    curves = _pack(degs, cps, kts)
    return curves, offset_queries(seed + 100, curves, per_curve=per_curve, on_curve_frac=0.25)


# ---------------------------------------------------------------------------
# Rational curves (NURBS)
# ---------------------------------------------------------------------------
def _circle_net(rng: np.random.Generator):
    """Full circle as a quadratic NURBS: 9 control points on a square around the centre, weights 1 and
    sqrt(1/2) alternating, knots {0^3, 1/4^2, 1/2^2, 3/4^2, 1^3}; random centre, radius and plane."""
    sq = np.array([[1, 0], [1, 1], [0, 1], [-1, 1], [-1, 0], [-1, -1], [0, -1], [1, -1], [1, 0]], float)
    w = np.array([1.0, np.sqrt(0.5)] * 4 + [1.0])
    A = np.linalg.qr(rng.standard_normal((3, 3)))[0]  # random orthonormal frame
    r = rng.uniform(0.2, 0.5)
    c = rng.uniform(0.3, 0.7, 3)
    P = c + r * (sq[:, :1] * A[:, 0] + sq[:, 1:] * A[:, 1])
    U = np.array([0, 0, 0, 0.25, 0.25, 0.5, 0.5, 0.75, 0.75, 1, 1, 1.0])
    return P, w, U, c, r, A[:, 2]


def curves_rational(seed: int = 13, n_random: int = 56, n_circles: int = 8, per_curve: int = 128):
    """Rational B-spline curves: ``n_circles`` exact full circles (quadratic NURBS) and ``n_random`` curves of
    degree U{2..5} with U{8..40} control points uniform in [0,1]^3, weights log-uniform in [1/4, 4] and Exp(1)
    knots with 10% doubled.  Queries as the batched curves: ``per_curve`` offsets of N(0, (0.05 diag)^2) from
    parameter-uniform curve points, a quarter of them on the curve.  Returns (CurveSet with weights, queries,
    circles) where circles = list of (centre, radius, normal) of the first ``n_circles`` curves."""
    rng = np.random.default_rng(seed)
    degs, cps, kts, ws, circles = [], [], [], [], []
    for _ in range(n_circles):
        P, w, U, c, r, nrm = _circle_net(rng)
        degs.append(2)
        cps.append(P)
        ws.append(w)
        kts.append(U)
        circles.append((c, r, nrm))
    for _ in range(n_random):
        p = int(rng.integers(2, 6))
        n_cp = int(rng.integers(max(8, p + 1), 41))
        n_int = n_cp - p - 1
        n_dup = min(int(round(0.1 * n_int)), n_int // 2)
        base = _exp_interior(rng, n_int - n_dup)
        interior = np.concatenate([base, base[rng.choice(n_int - n_dup, n_dup, replace=False)]]) if n_dup else base
        degs.append(p)
        cps.append(rng.uniform(0.0, 1.0, (n_cp, 3)))
        ws.append(np.exp(rng.uniform(np.log(0.25), np.log(4.0), n_cp)))
        kts.append(_clamped(interior, p))
    curves = _pack(degs, cps, kts)
    curves.weights = np.concatenate(ws)
    return curves, offset_queries(seed + 100, curves, per_curve=per_curve, on_curve_frac=0.25), circles
