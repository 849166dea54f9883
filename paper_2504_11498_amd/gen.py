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
        return CurveSet(deg, cp_off, np.concatenate(cps).reshape(-1, 3), k_off, np.concatenate(kts))


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
