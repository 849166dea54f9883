"""FP64 CPU oracle for batched B-spline point projection and inversion.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product library never imports this
package.  The arithmetic lives in ``mrep_oracle.c`` (plain C, OpenMP over
queries and curves); this module builds it with gcc and marshals numpy arrays.

Each wrapper names the passage of the paper its C function follows; see the
header of ``mrep_oracle.c`` for the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mrep_oracle.c")
_SRC_MLP = os.path.join(_HERE, "mlp_oracle.c")
_SRC_SURF = os.path.join(_HERE, "surf_oracle.c")
_SRC_CLIP = os.path.join(_HERE, "clip_oracle.c")
_SRC_NURBS = os.path.join(_HERE, "nurbs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", "-o", tmp, _SRC, _SRC_MLP, _SRC_SURF, _SRC_CLIP, _SRC_NURBS, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in (_SRC, _SRC_MLP, _SRC_SURF, _SRC_CLIP, _SRC_NURBS)):
        build(force=True)
    lib = C.CDLL(_LIB)
    dp, ip, lp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    lib.orc_basis.argtypes = [C.c_int, C.c_int, dp, C.c_double, dp]
    lib.orc_eval.argtypes = [C.c_int, C.c_int, dp, dp, C.c_int64, dp, dp, dp, dp]
    lib.orc_eval_batch.argtypes = [C.c_int, ip, lp, dp, lp, dp, C.c_int64, ip, dp, dp]
    lib.orc_bezier_spans.argtypes = [C.c_int, C.c_int, dp, dp, C.c_int, dp, dp]
    lib.orc_bez_split.argtypes = [C.c_int, dp, C.c_double, dp, dp]
    lib.orc_bez_split.restype = None
    lib.orc_bez_eval.argtypes = [C.c_int, dp, C.c_double, dp]
    lib.orc_bez_eval.restype = None
    lib.orc_g1_reduce.argtypes = [C.c_int, dp, dp, dp]
    lib.orc_piece_deviation.argtypes = [C.c_int, dp, dp, C.c_int]
    lib.orc_piece_deviation.restype = C.c_double
    lib.orc_decompose_batch.argtypes = [C.c_int, ip, lp, dp, lp, dp, dp, C.c_int]
    lib.orc_decompose_batch.restype = C.c_void_p
    lib.orc_dec_status.argtypes = [C.c_void_p]
    lib.orc_dec_counts.argtypes = [C.c_void_p, lp]
    lib.orc_dec_counts.restype = C.c_int64
    lib.orc_dec_fetch.argtypes = [C.c_void_p, dp, dp, ip]
    lib.orc_dec_fetch.restype = None
    lib.orc_dec_free.argtypes = [C.c_void_p]
    lib.orc_dec_free.restype = None
    lib.orc_project_batch.argtypes = [C.c_int, ip, lp, dp, lp, dp, C.c_int64, ip, dp, dp, dp, ip, dp, dp,
                                      C.c_int]
    lib.orc_max_threads.restype = C.c_int
    lib.orc_mlp_loss.argtypes = [C.c_int, C.c_int, C.c_int, dp, C.c_int64, dp, dp, dp, dp, dp]
    lib.orc_mlp_loss.restype = C.c_double
    sargs = [C.c_int, ip, ip, ip, ip, lp, dp, lp, dp, lp, dp]
    lib.orc_surf_eval_batch.argtypes = sargs + [C.c_int64, ip, dp, dp]
    lib.orc_surf_project_batch.argtypes = sargs + [C.c_int64, ip, dp, dp, dp, dp, dp, C.c_int]
    lib.orc_surf_patches.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, dp, dp, dp, C.c_int, dp, dp]
    lib.orc_surf_patch_deviation.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, dp, dp, dp, dp, dp, C.c_int]
    lib.orc_surf_patch_deviation.restype = C.c_double
    lib.orc_clip_e_poly.argtypes = [dp, dp, dp]
    lib.orc_clip_e_poly.restype = None
    lib.orc_ferrari.argtypes = [dp, dp]
    lib.orc_ferrari_01.argtypes = [dp, dp]
    lib.orc_rebase.argtypes = [C.c_int, dp, dp]
    lib.orc_rebase.restype = None
    lib.orc_sub_left.argtypes = [C.c_int, C.c_double, dp]
    lib.orc_sub_left.restype = None
    lib.orc_sub_right.argtypes = [C.c_int, C.c_double, dp]
    lib.orc_sub_right.restype = None
    lib.orc_hull_axis.argtypes = [C.c_int, dp, dp, dp]
    lib.orc_clip_apply.argtypes = [C.c_int, dp, C.c_double, C.c_double, dp]
    lib.orc_clip_apply.restype = None
    lib.orc_clip_piece.argtypes = [dp, dp, C.c_int, dp, dp, dp]
    lib.orc_clip_pairs.argtypes = [C.c_int64, dp, dp, C.c_int, C.c_int, C.c_double, dp, dp, dp]
    lib.orc_clip_pairs.restype = None
    lib.onc_eval.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.c_int64, dp, dp, dp, dp]
    lib.onc_eval_batch.argtypes = [C.c_int, ip, lp, dp, dp, lp, dp, C.c_int64, ip, dp, dp]
    lib.onc_project_batch.argtypes = [C.c_int, ip, lp, dp, dp, lp, dp, C.c_int64, ip, dp, dp, dp, dp, dp, C.c_int]
    lib.onc_piece_deviation.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.c_double, C.c_double, dp, C.c_int]
    lib.onc_piece_deviation.restype = C.c_double
    _lib = lib
    return lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def basis(p: int, U, t: float) -> np.ndarray:
    """All N_{i,p}(t) by the Cox-de Boor recursion (Sec. 4, eq. bsplinebasis)."""
    U = _d(U)
    n = U.shape[0] - p - 1
    N = np.zeros(n)
    if _load().orc_basis(p, n, _ptr(U, C.c_double), float(t), _ptr(N, C.c_double)) != 0:
        raise RuntimeError("orc_basis failed")
    return N


def eval_curve(p: int, P, U, t, derivs: bool = False):
    """C(t) (and C', C'') by de Boor's algorithm on the B-spline of Sec. 4."""
    P, U, t = _d(P), _d(U), np.atleast_1d(_d(t))
    m = t.shape[0]
    X, D1, D2 = np.zeros((m, 3)), np.zeros((m, 3)), np.zeros((m, 3))
    rc = _load().orc_eval(p, P.shape[0], _ptr(P, C.c_double), _ptr(U, C.c_double), m, _ptr(t, C.c_double),
                          _ptr(X, C.c_double), _ptr(D1, C.c_double), _ptr(D2, C.c_double))
    if rc != 0:
        raise ValueError("bad curve")
    return (X, D1, D2) if derivs else X


def eval_batch(curves, cid, t) -> np.ndarray:
    """X[i] = C_{cid[i]}(t[i]) over a CSR curve set (de Boor)."""
    cid = np.ascontiguousarray(cid, dtype=np.int32)
    t = _d(t)
    X = np.zeros((t.shape[0], 3))
    rc = _load().orc_eval_batch(curves.n, _ptr(curves.degree, C.c_int32), _ptr(curves.cp_off, C.c_int64),
                                _ptr(_d(curves.cp), C.c_double), _ptr(curves.knot_off, C.c_int64),
                                _ptr(_d(curves.knots), C.c_double), t.shape[0], _ptr(cid, C.c_int32),
                                _ptr(t, C.c_double), _ptr(X, C.c_double))
    if rc != 0:
        raise ValueError("bad curve id")
    return X


def bezier_spans(p: int, P, U):
    """Bezier control points of every non-degenerate span by Boehm knot insertion (Sec. 5.2.1)."""
    P, U = _d(P), _d(U)
    n = P.shape[0]
    bz = np.zeros((n, p + 1, 3))
    tab = np.zeros((n, 2))
    ns = _load().orc_bezier_spans(p, n, _ptr(P, C.c_double), _ptr(U, C.c_double), n, _ptr(bz, C.c_double),
                                  _ptr(tab, C.c_double))
    if ns < 0:
        raise ValueError("bad curve")
    return bz[:ns].copy(), tab[:ns].copy()


def bez_eval(Q, u) -> np.ndarray:
    """de Casteljau evaluation of a Bezier piece with control points Q[p+1,3] at each u."""
    Q = _d(Q)
    u = np.atleast_1d(_d(u))
    out = np.zeros((u.shape[0], 3))
    lib = _load()
    for i, x in enumerate(u):
        lib.orc_bez_eval(Q.shape[0] - 1, _ptr(Q, C.c_double), float(x), out[i].ctypes.data_as(C.POINTER(C.c_double)))
    return out


def bez_split(Q, z: float):
    """de Casteljau split of a Bezier piece at z (Sec. 5.2.2, eq. submatrix)."""
    Q = _d(Q)
    p = Q.shape[0] - 1
    L, R = np.zeros_like(Q), np.zeros_like(Q)
    _load().orc_bez_split(p, _ptr(Q, C.c_double), float(z), _ptr(L, C.c_double), _ptr(R, C.c_double))
    return L, R


def g1_reduce(Q):
    """G1-continuous L2-optimal cubic of a degree-p Bezier piece (Sec. 5.2.2); returns (R[4,3], (d0,d1))."""
    Q = _d(Q)
    p = Q.shape[0] - 1
    R = np.zeros((4, 3))
    dl = np.zeros(2)
    if _load().orc_g1_reduce(p, _ptr(Q, C.c_double), _ptr(R, C.c_double), _ptr(dl, C.c_double)) != 0:
        raise ValueError("bad degree")
    return R, dl


def piece_deviation(Q, R, ns: int = 4097) -> float:
    """max over ns uniform samples of |Q(u) - R(u)| (same-parameter deviation)."""
    Q, R = _d(Q), _d(R)
    return float(_load().orc_piece_deviation(Q.shape[0] - 1, _ptr(Q, C.c_double), _ptr(R, C.c_double), ns))


def decompose(curves, tol_abs, nthreads: int = 0):
    """Cubic pieces of every curve: Boehm spans, elevation / G1-L2 reduction, error-controlled splits.

    Returns dict(counts[n], R[S,4,3], tab[S,2] (t_a, t_b), span[S]).
    """
    tol = np.broadcast_to(_d(tol_abs), (curves.n,)).copy()
    lib = _load()
    h = lib.orc_decompose_batch(curves.n, _ptr(curves.degree, C.c_int32), _ptr(curves.cp_off, C.c_int64),
                                _ptr(_d(curves.cp), C.c_double), _ptr(curves.knot_off, C.c_int64),
                                _ptr(_d(curves.knots), C.c_double), _ptr(tol, C.c_double), int(nthreads))
    try:
        if lib.orc_dec_status(h) != 0:
            raise ValueError("decomposition failed (bad curve or piece cap exceeded)")
        counts = np.zeros(curves.n, np.int64)
        tot = lib.orc_dec_counts(h, _ptr(counts, C.c_int64))
        R = np.zeros((tot, 4, 3))
        tab = np.zeros((tot, 2))
        span = np.zeros(tot, np.int32)
        lib.orc_dec_fetch(h, _ptr(R, C.c_double), _ptr(tab, C.c_double), _ptr(span, C.c_int32))
    finally:
        lib.orc_dec_free(h)
    return {"counts": counts, "R": R, "tab": tab, "span": span}


def project(curves, cid, q, nthreads: int = 0):
    """Global minimiser of |q - C(t)| over each query's own curve (Sec. 4, eq. projections).

    Returns dict(t, dist, span, kappa, runner): runner is the distance of the best other local
    minimum (inf if none), kappa = f'(t*)/|C'(t*)|^2 at a stationary minimiser (1 at a boundary one).
    """
    cid = np.ascontiguousarray(cid, dtype=np.int32)
    q = _d(q).reshape(-1, 3)
    m = q.shape[0]
    t, d, kap, run = np.zeros(m), np.zeros(m), np.zeros(m), np.zeros(m)
    span = np.zeros(m, np.int32)
    rc = _load().orc_project_batch(curves.n, _ptr(curves.degree, C.c_int32), _ptr(curves.cp_off, C.c_int64),
                                   _ptr(_d(curves.cp), C.c_double), _ptr(curves.knot_off, C.c_int64),
                                   _ptr(_d(curves.knots), C.c_double), m, _ptr(cid, C.c_int32),
                                   _ptr(q, C.c_double), _ptr(t, C.c_double), _ptr(d, C.c_double),
                                   _ptr(span, C.c_int32), _ptr(kap, C.c_double), _ptr(run, C.c_double),
                                   int(nthreads))
    if rc != 0:
        raise ValueError("bad curve or id")
    return {"t": t, "dist": d, "span": span, "kappa": kap, "runner": run}


def max_threads() -> int:
    return int(_load().orc_max_threads())


def mlp_loss(params, x, u_star=None, accept=None, n_in=15, hidden=128, n_out=2, grad=False):
    """FP64 seeding-network forward (and backward) on a batch (see mlp_oracle.c).

    u_star: targets [B, n_out - 1] (or [B] for n_out = 2).  Returns (loss, y[B, n_out], grad or None)."""
    params = _d(params)
    x = _d(x).reshape(-1, n_in)
    B = x.shape[0]
    y = np.zeros((B, n_out))
    g = np.zeros_like(params) if grad else None
    us = _d(u_star).reshape(B, n_out - 1) if u_star is not None else None
    ac = _d(accept) if accept is not None else None
    loss = _load().orc_mlp_loss(n_in, hidden, n_out, _ptr(params, C.c_double), B, _ptr(x, C.c_double),
                                _ptr(us, C.c_double) if us is not None else None,
                                _ptr(ac, C.c_double) if ac is not None else None, _ptr(y, C.c_double),
                                _ptr(g, C.c_double) if g is not None else None)
    return float(loss), y, g


def mlp_param_count(n_in=15, hidden=128, n_out=2):
    return hidden * n_in + hidden + hidden * hidden + hidden + n_out * hidden + n_out


# --------------------------------------------------------------------------- surfaces (surf_oracle.c)
def _surf_args(S):
    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)  # noqa: E731
    i64 = lambda a: np.ascontiguousarray(a, dtype=np.int64)  # noqa: E731
    keep = [i32(S.deg_u), i32(S.deg_v), i32(S.n_u), i32(S.n_v), i64(S.cp_off), _d(S.cp), i64(S.ku_off), _d(S.ku),
            i64(S.kv_off), _d(S.kv)]
    ptrs = [_ptr(keep[0], C.c_int32), _ptr(keep[1], C.c_int32), _ptr(keep[2], C.c_int32), _ptr(keep[3], C.c_int32),
            _ptr(keep[4], C.c_int64), _ptr(keep[5], C.c_double), _ptr(keep[6], C.c_int64), _ptr(keep[7], C.c_double),
            _ptr(keep[8], C.c_int64), _ptr(keep[9], C.c_double)]
    return keep, [int(S.n)] + ptrs


def surf_eval(S, sid, uv):
    """S_{sid[k]}(u_k, v_k) by tensor-product de Boor (FP64)."""
    sid = np.ascontiguousarray(sid, dtype=np.int32)
    uv = _d(uv).reshape(-1, 2)
    out = np.zeros((sid.shape[0], 3))
    keep, args = _surf_args(S)
    _load().orc_surf_eval_batch(*args, sid.shape[0], _ptr(sid, C.c_int32), _ptr(uv, C.c_double), _ptr(out, C.c_double))
    return out


def surf_surface(S, k):
    """(p, q, nu, nv, P[nu*nv,3], U, V) of surface k."""
    return (int(S.deg_u[k]), int(S.deg_v[k]), int(S.n_u[k]), int(S.n_v[k]),
            np.ascontiguousarray(S.cp[S.cp_off[k]:S.cp_off[k + 1]], dtype=np.float64),
            np.ascontiguousarray(S.ku[S.ku_off[k]:S.ku_off[k + 1]], dtype=np.float64),
            np.ascontiguousarray(S.kv[S.kv_off[k]:S.kv_off[k + 1]], dtype=np.float64))


def surf_patches(S, k):
    """Exact Bezier patches of surface k by Boehm insertion: nets[np, p+1, q+1, 3], rects[np, 4]."""
    p, q, nu, nv, P, U, V = surf_surface(S, k)
    cap = nu * nv
    nets = np.zeros((cap, p + 1, q + 1, 3))
    rects = np.zeros((cap, 4))
    n = _load().orc_surf_patches(p, q, nu, nv, _ptr(P, C.c_double), _ptr(U, C.c_double), _ptr(V, C.c_double), cap,
                                 _ptr(nets, C.c_double), _ptr(rects, C.c_double))
    if n < 0:
        raise ValueError("orc_surf_patches failed")
    return nets[:n], rects[:n]


def surf_patch_deviation(S, k, R, rect, ns=33):
    """Largest |R(s,t) - S(u,v)| of a bicubic patch R[4,4,3] on rect over an ns x ns grid."""
    p, q, nu, nv, P, U, V = surf_surface(S, k)
    R = _d(R).reshape(4, 4, 3)
    rect = _d(rect)
    return float(_load().orc_surf_patch_deviation(p, q, nu, nv, _ptr(P, C.c_double), _ptr(U, C.c_double),
                                                  _ptr(V, C.c_double), _ptr(R, C.c_double), _ptr(rect, C.c_double),
                                                  int(ns)))


def surf_project(S, sid, q, nthreads: int = 0):
    """Global minimiser (u, v) of |q - S(u, v)| over each query's own surface.

    Returns dict(uv[n,2], dist, runner, kappa): runner = distance of the best other local minimum farther than
    1e-6 in parameter (inf if none within 3e-6 * diag), kappa = smallest eigenvalue of the distance Hessian
    relative to the first fundamental form at an interior minimiser (1 on the boundary)."""
    sid = np.ascontiguousarray(sid, dtype=np.int32)
    q = _d(q).reshape(-1, 3)
    n = sid.shape[0]
    uv = np.zeros((n, 2))
    dist, runner, kappa = np.zeros(n), np.zeros(n), np.zeros(n)
    keep, args = _surf_args(S)
    rc = _load().orc_surf_project_batch(*args, n, _ptr(sid, C.c_int32), _ptr(q, C.c_double), _ptr(uv, C.c_double),
                                        _ptr(dist, C.c_double), _ptr(runner, C.c_double), _ptr(kappa, C.c_double),
                                        int(nthreads))
    if rc != 0:
        raise ValueError("orc_surf_project_batch failed")
    return {"uv": uv, "dist": dist, "runner": runner, "kappa": kappa}


# ---------------------------------------------------------------------------
# The paper's refinement path for one cubic piece (clip_oracle.c): monotonic
# decomposition (Sec. 5.2.3), elimination (Sec. 5.3, Properties 1-2),
# rebasement (Sec. 5.3, matrix T) and Bezier clipping (Sec. 5.4.1).
# ---------------------------------------------------------------------------
def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def clip_e_poly(Q, q) -> np.ndarray:
    """Power coefficients a[0..5] of E(t) = 2 (C(t) - q) . C'(t) (eq. Et) for a cubic Bezier Q[4,3]."""
    Q, q = _d(Q), _d(q)
    a = np.zeros(6)
    _load().orc_clip_e_poly(_dp(Q), _dp(q), _dp(a))
    return a


def ferrari(c) -> np.ndarray:
    """Sorted real roots of c[0] + c[1] x + ... + c[4] x^4 by Ferrari's method (Sec. 5.2.3)."""
    c = _d(c)
    r = np.zeros(4)
    n = _load().orc_ferrari(_dp(c), _dp(r))
    return r[:n].copy()


def ferrari_01(c) -> np.ndarray:
    """The split points of the refinement path: Ferrari's roots within [-0.5, 1.5], each polished by three Newton
    steps on the full quartic (the reading for leading coefficients at rounding level), sorted."""
    c = _d(c)
    r = np.zeros(4)
    n = _load().orc_ferrari_01(_dp(c), _dp(r))
    return r[:n].copy()


def rebase(a) -> np.ndarray:
    """Bernstein coefficients b = T a of a power-form polynomial (Sec. 5.3)."""
    a = _d(a)
    b = np.zeros_like(a)
    _load().orc_rebase(a.shape[0] - 1, _dp(a), _dp(b))
    return b


def sub_matrices(n: int, z: float):
    """(S_L(z), S_R(z)) of a degree-n Bezier (Sec. 5.2.2)."""
    L, R = np.zeros((n + 1, n + 1)), np.zeros((n + 1, n + 1))
    lib = _load()
    lib.orc_sub_left(n, float(z), _dp(L))
    lib.orc_sub_right(n, float(z), _dp(R))
    return L, R


def hull_axis(b):
    """[z1, z2] = the convex hull of (i/n, b_i) intersected with the t axis, or None (Sec. 5.4.1)."""
    b = _d(b)
    z1, z2 = C.c_double(), C.c_double()
    ok = _load().orc_hull_axis(b.shape[0] - 1, _dp(b), C.byref(z1), C.byref(z2))
    return (z1.value, z2.value) if ok else None


def clip_apply(b, z1: float, z2: float) -> np.ndarray:
    """S_[z1,z2] b = S_L((z2 - z1)/(1 - z1)) S_R(z1) b (eq. subdivisionmatrix)."""
    b = _d(b)
    out = np.zeros_like(b)
    _load().orc_clip_apply(b.shape[0] - 1, _dp(b), float(z1), float(z2), _dp(out))
    return out


def clip_piece(Q, q, iters: int = 3):
    """The paper's refinement of one (query, cubic piece) pair; returns (t, d2, info) with info = (monotonic
    intervals, kept intervals, largest remaining clip width, roots of E' in (0, 1))."""
    Q, q = _d(Q), _d(q)
    t, d2 = C.c_double(), C.c_double()
    info = np.zeros(4)
    _load().orc_clip_piece(_dp(Q), _dp(q), int(iters), C.byref(t), C.byref(d2), _dp(info))
    return t.value, d2.value, info


def clip_pairs(Q, q, iters: int = 3, safeguard: bool = False, tol_t: float = 0.0):
    """clip_piece over pairs Q[n,4,3], q[n,3] (OpenMP); returns (t[n], d2[n], info[n,4]).  With safeguard, a
    clipping that keeps more than half of the interval is followed by a halving on the sign of E, and clipping
    stops once the interval is below tol_t (or after iters)."""
    Q = _d(Q).reshape(-1, 12)
    q = _d(q).reshape(-1, 3)
    n = Q.shape[0]
    t, d2, info = np.zeros(n), np.zeros(n), np.zeros((n, 4))
    _load().orc_clip_pairs(n, _dp(Q), _dp(q), int(iters), int(bool(safeguard)), float(tol_t), _dp(t), _dp(d2),
                           _dp(info))
    return t, d2, info


# ---------------------------------------------------------------------------
# Rational B-spline (NURBS) curves (nurbs_oracle.c): the paper's method is
# stated for non-rational curves (Sec. 6, discussion and limitations; Sec. 7);
# these compute the plain definitions on C = sum N w P / sum N w.
# ---------------------------------------------------------------------------
def nurbs_eval_curve(p: int, P, w, U, t, derivs: bool = False):
    """C(t) (and C', C'') of one rational curve: de Boor on the homogeneous points, then the quotient rule."""
    P, w, U, t = _d(P), _d(w), _d(U), np.atleast_1d(_d(t))
    m = t.shape[0]
    X, D1, D2 = np.zeros((m, 3)), np.zeros((m, 3)), np.zeros((m, 3))
    rc = _load().onc_eval(p, P.shape[0], _ptr(P, C.c_double), _ptr(w, C.c_double), _ptr(U, C.c_double), m,
                          _ptr(t, C.c_double), _ptr(X, C.c_double), _ptr(D1, C.c_double), _ptr(D2, C.c_double))
    if rc != 0:
        raise ValueError("bad rational curve")
    return (X, D1, D2) if derivs else X


def nurbs_eval_batch(curves, weights, cid, t) -> np.ndarray:
    """X[i] = C_{cid[i]}(t[i]) over a CSR set of rational curves (weights per control point)."""
    cid = np.ascontiguousarray(cid, dtype=np.int32)
    t, w = _d(t), _d(weights)
    X = np.zeros((t.shape[0], 3))
    rc = _load().onc_eval_batch(curves.n, _ptr(curves.degree, C.c_int32), _ptr(curves.cp_off, C.c_int64),
                                _ptr(_d(curves.cp), C.c_double), _ptr(w, C.c_double), _ptr(curves.knot_off, C.c_int64),
                                _ptr(_d(curves.knots), C.c_double), t.shape[0], _ptr(cid, C.c_int32),
                                _ptr(t, C.c_double), _ptr(X, C.c_double))
    if rc != 0:
        raise ValueError("bad rational curve or id")
    return X


def nurbs_project(curves, weights, cid, q, nthreads: int = 0):
    """Global minimiser of |q - C(t)| over each query's own rational curve (Sec. 4, eq. projections).

    Returns dict(t, dist, kappa, runner) with the meanings of project()."""
    cid = np.ascontiguousarray(cid, dtype=np.int32)
    q, w = _d(q).reshape(-1, 3), _d(weights)
    m = q.shape[0]
    t, d, kap, run = np.zeros(m), np.zeros(m), np.zeros(m), np.zeros(m)
    rc = _load().onc_project_batch(curves.n, _ptr(curves.degree, C.c_int32), _ptr(curves.cp_off, C.c_int64),
                                   _ptr(_d(curves.cp), C.c_double), _ptr(w, C.c_double),
                                   _ptr(curves.knot_off, C.c_int64), _ptr(_d(curves.knots), C.c_double), m,
                                   _ptr(cid, C.c_int32), _ptr(q, C.c_double), _ptr(t, C.c_double),
                                   _ptr(d, C.c_double), _ptr(kap, C.c_double), _ptr(run, C.c_double), int(nthreads))
    if rc != 0:
        raise ValueError("bad rational curve or id")
    return {"t": t, "dist": d, "kappa": kap, "runner": run}


def nurbs_piece_deviation(p: int, P, w, U, ta: float, tb: float, R, ns: int = 2049) -> float:
    """Largest sampled |C(t) - R(u)|, t = ta + u (tb - ta), of a cubic Bezier piece R against the rational curve."""
    P, w, U, R = _d(P), _d(w), _d(U), _d(R).reshape(4, 3)
    return float(_load().onc_piece_deviation(p, P.shape[0], _ptr(P, C.c_double), _ptr(w, C.c_double),
                                             _ptr(U, C.c_double), float(ta), float(tb), _ptr(R, C.c_double), int(ns)))
