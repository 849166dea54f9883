"""CPU tests of libmrep's host side: exported symbols, constant matrices against
the paper's printed values, the FP64 M-rep decomposition against the oracle's
independent Boehm-based decomposition, and every host-forceable error code."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from conftest import ROOT, load_golden
from paper_2504_11498_amd import gen

mrep = pytest.importorskip("paper_2504_11498_amd.mrep", reason="libmrep.so not built")


def test_every_declared_symbol_is_exported():
    hdr = open(os.path.join(ROOT, "include", "mrep.h")).read()
    declared = set(re.findall(r"\b(mrep_[a-z_0-9]+)\s*\(", hdr))
    assert declared == set(mrep.EXPORTS)
    lib = C.CDLL(mrep.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name
    assert mrep.abi_version() == 10


def test_rebasement_matrix_matches_printed_T5():
    T = np.array([[float(v) for v in r.split()] for r in load_golden("power_to_bernstein_deg5.txt")])
    np.testing.assert_allclose(mrep.bernstein_matrix(5, inverse=True), T, atol=1e-15)
    for p in range(1, 10):
        B, Bi = mrep.bernstein_matrix(p), mrep.bernstein_matrix(p, inverse=True)
        np.testing.assert_allclose(B @ Bi, np.eye(p + 1), atol=1e-12)


def test_bernstein_matrix_reproduces_bernstein_basis():
    from math import comb

    u = np.linspace(0, 1, 11)
    for p in [2, 3, 6]:
        U = np.vander(u, p + 1, increasing=True)
        ref = np.stack([comb(p, i) * u**i * (1 - u) ** (p - i) for i in range(p + 1)], -1)
        np.testing.assert_allclose(U @ mrep.bernstein_matrix(p), ref, atol=1e-13)


@pytest.mark.parametrize("z", [0.2, 0.5, 0.9])
def test_subdivision_matrix_matches_printed_Sz(z):
    rows = load_golden("subdivision_matrix_Sz.txt")
    env = {"__builtins__": {}, "z": z}
    S = np.array([[eval(e, env) for e in r.split(";")] for r in rows])  # noqa: S307
    np.testing.assert_allclose(mrep.subdivision_matrix(3, z), S, atol=1e-15)


def test_degree_p_subdivision_agrees_with_oracle_de_casteljau():
    rng = np.random.default_rng(4)
    for p in [4, 7]:
        Q = rng.uniform(0, 1, (p + 1, 3))
        S = mrep.subdivision_matrix(p, 0.3)
        L, R = oracle.bez_split(Q, 0.3)
        np.testing.assert_allclose(S[: p + 1] @ Q, L, atol=1e-14)
        np.testing.assert_allclose(S[p + 1 :] @ Q, R, atol=1e-14)


def test_gram_matrix_closed_form():
    x, w = np.polynomial.legendre.leggauss(30)
    u, w = 0.5 * (x + 1), 0.5 * w
    from math import comb

    for m, n in [(3, 3), (3, 6)]:
        G = mrep.gram_matrix(m, n)
        for i in range(m + 1):
            for j in range(n + 1):
                bi = comb(m, i) * u**i * (1 - u) ** (m - i)
                bj = comb(n, j) * u**j * (1 - u) ** (n - j)
                assert abs(G[i, j] - np.sum(w * bi * bj)) < 4e-15
        np.testing.assert_allclose(G.sum(1), 1.0 / (m + 1), atol=1e-15)  # rows sum to 1/(m+1)


def _compare_with_oracle(curves, tol_rel):
    plan = mrep.decompose_curves(curves, tol_rel)
    ex = plan.export()
    diag = curves.bbox_diag()
    ref = oracle.decompose(curves, tol_rel * diag)
    counts = np.diff(ex["seg_off"])
    mismatch = np.nonzero(counts != ref["counts"])[0]
    return plan, ex, ref, counts, mismatch, diag


def test_decomposition_low_degree_matches_boehm():
    curves, _ = gen.curve_single(1)
    plan, ex, ref, counts, mismatch, diag = _compare_with_oracle(curves, 1e-6)
    assert plan.n_segments == 13 and mismatch.size == 0
    np.testing.assert_array_equal(ex["seg_t"], ref["tab"])
    assert np.abs(ex["seg_cp"] - ref["R"]).max() <= 1e-13 * diag[0]
    # p = 2 (elevated) and doubled knots
    c2 = gen.curves_batched_geometry(seed=8, n_curves=30, deg_lo=2, deg_hi=3, cp_lo=8, cp_hi=60)
    plan, ex, ref, counts, mismatch, diag = _compare_with_oracle(c2, 1e-6)
    assert mismatch.size == 0
    np.testing.assert_array_equal(ex["seg_t"], ref["tab"])
    assert np.abs(ex["seg_cp"] - ref["R"]).max() <= 1e-12


@pytest.mark.parametrize("which", ["deg4-7", "deg16-32"])
def test_decomposition_high_degree_matches_oracle_breakpoints(which):
    """Degrees 4..7, and 16..32 where the library takes each span's Bezier points from blossoms instead of the
    power form (the oracle always from Boehm's knot insertion)."""
    if which == "deg4-7":
        curves = gen.curves_batched_geometry(seed=9, n_curves=48, deg_lo=4, deg_hi=7, cp_lo=8, cp_hi=120)
    else:
        curves, _ = gen.curves_high_degree(per_degree=2, cp_extra=(1, 12))
    plan, ex, ref, counts, mismatch, diag = _compare_with_oracle(curves, 1e-6)
    assert mismatch.size == 0, mismatch
    np.testing.assert_allclose(ex["seg_t"], ref["tab"], atol=1e-14)
    # the G1/L2-optimal cubic is unique: both derivations agree to rounding
    assert np.abs(ex["seg_cp"] - ref["R"]).max() <= 1e-10
    # every piece within tolerance of the exact curve (oracle's dense check)
    worst = 0.0
    for c in range(curves.n):
        p, P, U = curves.curve(c)
        bz, tab = oracle.bezier_spans(p, P, U)
        for s in range(ex["seg_off"][c], ex["seg_off"][c + 1]):
            ta, tb = ex["seg_t"][s]
            k = int(np.searchsorted(tab[:, 0], ta, side="right") - 1)
            h = tab[k, 1] - tab[k, 0]
            # exact piece: split the span's Bezier at the piece's local range
            a, b = (ta - tab[k, 0]) / h, (tb - tab[k, 0]) / h
            _, right = oracle.bez_split(bz[k], a)
            piece, _ = oracle.bez_split(right, (b - a) / (1 - a) if a < 1 else 1.0)
            worst = max(worst, oracle.piece_deviation(piece, ex["seg_cp"][s], 2049) / (1e-6 * diag[c]))
    assert worst <= 1.0


def _curveset(p, P, U):
    return gen._pack([p], [np.asarray(P, float)], [np.asarray(U, float)])


def test_error_codes():
    P = np.random.default_rng(0).uniform(0, 1, (6, 3))
    U = np.array([0, 0, 0, 0, 0.4, 0.6, 1, 1, 1, 1.0])
    mrep.decompose_curves(_curveset(3, P, U), 1e-6)  # valid
    cases = [
        (_curveset(0, P, np.concatenate([[0], U[3:7], [1, 1]])), 1e-6, mrep.E_BAD_DEGREE),
        (_curveset(33, np.zeros((40, 3)), np.linspace(0, 1, 74)), 1e-6, mrep.E_BAD_DEGREE),
        (_curveset(3, P, U[::-1]), 1e-6, mrep.E_BAD_KNOTS),
        (_curveset(3, P, np.array([0, 0, 0, 0.1, 0.4, 0.6, 1, 1, 1, 1.0])), 1e-6, mrep.E_BAD_KNOTS),
        (_curveset(3, P, np.array([0, 0, 0, 0, 0.5, 0.5, 0.5, 0.5, 1, 1, 1, 1.0])[:10]), 1e-6, mrep.E_BAD_KNOTS),
        (_curveset(3, P, U[:-1]), 1e-6, mrep.E_BAD_KNOTS),
        (_curveset(3, P, np.where(U == 0.4, np.nan, U)), 1e-6, mrep.E_BAD_KNOTS),
        (_curveset(3, P, U), 0.0, mrep.E_TOL),
        (_curveset(3, P, U), -1.0, mrep.E_TOL),
        (_curveset(2, P[:3], np.array([0, 0, 0, 1, 1, 1.0])), float("nan"), mrep.E_TOL),
    ]
    for curves, tol, code in cases:
        with pytest.raises(mrep.MrepError) as ei:
            mrep.decompose_curves(curves, tol)
        assert ei.value.code == code, (ei.value, code)
    # interior multiplicity p+1
    U2 = np.array([0, 0, 0, 0, 0.5, 0.5, 0.5, 0.5, 1, 1, 1, 1.0])
    with pytest.raises(mrep.MrepError) as ei:
        mrep.decompose_curves(_curveset(3, np.zeros((8, 3)), U2), 1e-6)
    assert ei.value.code == mrep.E_BAD_KNOTS
    # null pointers and bad option structs at the C level
    assert mrep._decompose(1, None, None, None, None, None, 1e-6, 0, None) == mrep.E_INVALID_ARG
    o = mrep.Opts()
    assert mrep._opts_default(C.byref(o)) == mrep.OK and o.max_candidates == 32 and o.precision == mrep.PREC_BF16
    assert mrep.default_opts().max_candidates == 32
    assert mrep._opts_default(None) == mrep.E_INVALID_ARG
    o = mrep.default_opts()
    o.struct_size = 3
    b = C.c_int64()
    assert mrep._ws_bytes(None, 10, C.byref(o), C.byref(b)) == mrep.E_INVALID_ARG
    assert mrep._project(None, C.byref(o), 10, None, None, None, 0, None, None, None, None, None) == mrep.E_INVALID_ARG
    assert mrep._upload(None, None, 0, None, None) == mrep.E_INVALID_ARG


def test_span_layout_offsets_and_errors():
    """mrep_span_layout: one interval per q = p .. n - 1 and p + 1 points per interval; bad counts are rejected; the
    device call rejects null pointers before it launches anything."""
    curves = gen.curves_batched_geometry(2, n_curves=64)
    iv, pt = mrep.span_layout(curves)
    n_cp = np.diff(curves.cp_off)
    np.testing.assert_array_equal(np.diff(iv), n_cp - curves.degree)
    np.testing.assert_array_equal(np.diff(pt), (n_cp - curves.degree) * (curves.degree + 1))
    assert iv[0] == 0 and pt[0] == 0
    P = np.random.default_rng(0).uniform(0, 1, (6, 3))
    U = np.array([0, 0, 0, 0, 0.4, 0.6, 1, 1, 1, 1.0])
    cases = [
        (_curveset(0, P, U[2:-2]), mrep.E_BAD_DEGREE),
        (_curveset(16, np.zeros((20, 3)), np.linspace(0, 1, 37)), mrep.E_BAD_DEGREE),
        (_curveset(3, P[:3], np.array([0, 0, 0, 0, 1, 1, 1.0])), mrep.E_BAD_DEGREE),
        (_curveset(3, P, U[:-1]), mrep.E_BAD_KNOTS),
    ]
    for cv, code in cases:
        with pytest.raises(mrep.MrepError) as ei:
            mrep.span_layout(cv)
        assert ei.value.code == code, (ei.value, code)
    assert mrep._span_layout(-1, None, None, None, None, None) == mrep.E_INVALID_ARG
    nul = (None,) * 10
    assert mrep._span_bezier(1, 5, 3, *nul) == mrep.E_INVALID_ARG
    assert mrep._span_bezier(0, -1, 3, *nul) == mrep.E_INVALID_ARG
    assert mrep._span_bezier(0, 0, 0, *nul) == mrep.E_INVALID_ARG
    assert mrep._span_bezier(0, 0, 16, *nul) == mrep.E_INVALID_ARG
    assert mrep._span_bezier(0, 0, 15, *nul) == mrep.OK


def test_piece_cap_is_reported():
    # an absurd tolerance forces more than the per-span piece cap
    rng = np.random.default_rng(1)
    P = rng.uniform(0, 1, (8, 3))
    U = np.concatenate([np.zeros(8), np.ones(8)])
    with pytest.raises(mrep.MrepError) as ei:
        mrep.decompose_curves(_curveset(7, P, U), 1e-17)
    assert ei.value.code == mrep.E_TOL


def test_seeding_network_sizes_and_host_errors():
    """Parameter counts equal the oracle networks'; sizes and argument errors need no device."""
    assert mrep.nn_param_count() == mrep.nn_param_count(mrep.NN_CURVE) == oracle.mlp_param_count() == 18818
    assert mrep.nn_param_count(mrep.NN_SURFACE) == oracle.mlp_param_count(51, 128, 3) == 23555
    assert mrep._nn_param_count(7) == -1
    for kind, n_in, n_out in ((mrep.NN_CURVE, 15, 2), (mrep.NN_SURFACE, 51, 3)):
        sb, wb = C.c_int64(), C.c_int64()
        assert mrep._nn_bytes(kind, 4096, C.byref(sb), C.byref(wb)) == mrep.OK
        assert sb.value >= 4 * 4 * mrep.nn_param_count(kind) and sb.value % 256 == 0
        assert wb.value >= 4096 * (4 * 128 + n_in + 2 * n_out) * 4
        assert mrep._nn_bytes(kind, -1, C.byref(sb), None) == mrep.E_INVALID_ARG
        assert mrep._nn_bytes(kind, 1, None, None) == mrep.E_INVALID_ARG
        h = mrep._vp()
        assert mrep._nn_bind(kind, None, sb.value, C.byref(h)) == mrep.E_INVALID_ARG
        assert mrep._nn_bind(kind, mrep._vp(256), 16, C.byref(h)) == mrep.E_SMALL_BUFFER
        assert mrep._nn_bind(kind, mrep._vp(257), sb.value, C.byref(h)) == mrep.E_INVALID_ARG
    sb = C.c_int64()
    assert mrep._nn_bytes(2, 1, C.byref(sb), None) == mrep.E_INVALID_ARG
    assert mrep._nn_bind(2, mrep._vp(256), 1 << 20, C.byref(mrep._vp())) == mrep.E_INVALID_ARG
    assert mrep._nn_train(None, 10, None, None, None, 10, None, 1e-3, None, None, None, 0, None) == mrep.E_INVALID_ARG
    assert mrep._nn_forward(None, 10, None, None, None, 0, None) == mrep.E_INVALID_ARG
    assert mrep._nn_infer(None, 10, None, None, None) == mrep.E_INVALID_ARG
    assert mrep._project_seeded(None, None, None, 10, None, None, None, 0, None, None, None, None,
                                None) == mrep.E_INVALID_ARG
    assert mrep._project_s_seeded(None, None, None, 10, None, None, None, 0, None, None, None, None,
                                  None) == mrep.E_INVALID_ARG
    assert mrep._nn_surf_features(None, 10, None, None, None, None, None, 0, None) == mrep.E_INVALID_ARG
    assert mrep._tune(None, None, 10, None, None, None, 0, None, None, None, None, None, None,
                      None) == mrep.E_INVALID_ARG
    assert mrep._set_strategy(None, 0) == mrep.E_INVALID_ARG
    assert mrep._split(None, 1, None, None, None, mrep.ROOTS_FERRARI, None, None, None) == mrep.E_INVALID_ARG


# --------------------------------------------------------------------------- surfaces
def _surf(p, q, nu, nv, seed, height=True):
    rng = np.random.default_rng(seed)
    x, y = np.linspace(0, 1, nu), np.linspace(0, 1, nv)
    X, Y = np.meshgrid(x, y, indexing="ij")
    Z = 0.1 * np.sin(4 * X + 3 * Y) + rng.normal(0, 0.02, X.shape) if height else rng.uniform(0, 1, X.shape)
    P = np.stack([X, Y, Z], -1).reshape(-1, 3)
    iu = np.cumsum(rng.exponential(1, nu - p))
    iv = np.cumsum(rng.exponential(1, nv - q))
    U = np.r_[np.zeros(p + 1), iu[:-1] / iu[-1], np.ones(p + 1)]
    V = np.r_[np.zeros(q + 1), iv[:-1] / iv[-1], np.ones(q + 1)]
    return gen.SurfaceSet(np.array([p], np.int32), np.array([q], np.int32), np.array([nu], np.int32),
                          np.array([nv], np.int32), np.array([0, nu * nv], np.int64), P, np.array([0, len(U)], np.int64),
                          U, np.array([0, len(V)], np.int64), V)


def test_surface_bicubic_patches_equal_boehm():
    S = _surf(3, 3, 9, 8, 1)
    ex = mrep.decompose_surfaces(S, 1e-6).export_surfaces()
    nets, rects = oracle.surf_patches(S, 0)
    assert ex["patch_cp"].shape[0] == len(nets) == 6 * 5
    np.testing.assert_allclose(ex["patch_cp"], nets, atol=1e-13)
    np.testing.assert_allclose(ex["patch_uv"], rects, atol=0)
    np.testing.assert_array_equal(ex["patch_span"], np.arange(30))


@pytest.mark.parametrize("p,q", [(5, 5), (4, 3), (2, 5)])
def test_surface_reduced_patches_within_tolerance(p, q):
    S = _surf(p, q, 12, 11, 2 + p + q)
    tol_rel = 1e-6
    ex = mrep.decompose_surfaces(S, tol_rel).export_surfaces()
    diag = np.linalg.norm(S.cp.max(0) - S.cp.min(0))
    nets, rects = oracle.surf_patches(S, 0)
    # the pieces of every span patch tile its rectangle
    for sp, rc in enumerate(rects):
        mine = ex["patch_uv"][ex["patch_span"] == sp]
        area = np.sum((mine[:, 1] - mine[:, 0]) * (mine[:, 3] - mine[:, 2]))
        assert abs(area - (rc[1] - rc[0]) * (rc[3] - rc[2])) <= 1e-12
        assert np.all(mine[:, 0] >= rc[0]) and np.all(mine[:, 1] <= rc[1])
        assert np.all(mine[:, 2] >= rc[2]) and np.all(mine[:, 3] <= rc[3])
    rng = np.random.default_rng(0)
    pick = rng.choice(len(ex["patch_uv"]), min(60, len(ex["patch_uv"])), replace=False)
    for k in pick:
        dev = oracle.surf_patch_deviation(S, 0, ex["patch_cp"][k], ex["patch_uv"][k], ns=33)
        assert dev <= tol_rel * diag * (1 + 1e-9), (k, dev / diag)


def test_surface_elevated_bicubic_recovered_exactly():
    """A single bicubic Bezier patch written at degree (5, 4) reduces back to itself with no split."""
    rng = np.random.default_rng(9)
    R = rng.uniform(0, 1, (4, 4, 3))

    def elev(n, d):  # (d+1) x (n+1) matrix writing degree n at degree d
        M = np.eye(n + 1)
        for e in range(n, d):
            E = np.zeros((e + 2, e + 1))
            for i in range(e + 2):
                if i > 0:
                    E[i, i - 1] = i / (e + 1)
                if i <= e:
                    E[i, i] = 1 - i / (e + 1)
            M = E @ M
        return M

    N = np.einsum("ia,abc,jb->ijc", elev(3, 5), R, elev(3, 4))
    S = gen.SurfaceSet(np.array([5], np.int32), np.array([4], np.int32), np.array([6], np.int32),
                       np.array([5], np.int32), np.array([0, 30], np.int64), N.reshape(-1, 3),
                       np.array([0, 12], np.int64), np.r_[np.zeros(6), np.ones(6)], np.array([0, 10], np.int64),
                       np.r_[np.zeros(5), np.ones(5)])
    ex = mrep.decompose_surfaces(S, 1e-9).export_surfaces()
    assert ex["patch_cp"].shape[0] == 1
    np.testing.assert_allclose(ex["patch_cp"][0], R, atol=1e-12)


def test_surface_decomposition_errors():
    S = _surf(3, 3, 6, 6, 4)
    bad = gen.SurfaceSet(S.deg_u, S.deg_v, S.n_u, S.n_v, S.cp_off, S.cp, S.ku_off, S.ku.copy(), S.kv_off, S.kv)
    bad.ku[1] = 0.5  # not clamped / decreasing
    with pytest.raises(mrep.MrepError) as e:
        mrep.decompose_surfaces(bad, 1e-6)
    assert e.value.code == mrep.E_BAD_KNOTS
    bad2 = gen.SurfaceSet(np.array([9], np.int32), S.deg_v, S.n_u, S.n_v, S.cp_off, S.cp, S.ku_off, S.ku, S.kv_off,
                          S.kv)
    with pytest.raises(mrep.MrepError) as e:
        mrep.decompose_surfaces(bad2, 1e-6)
    assert e.value.code == mrep.E_BAD_DEGREE
    with pytest.raises(mrep.MrepError) as e:
        mrep.decompose_surfaces(S, -1.0)
    assert e.value.code == mrep.E_TOL
    plan = mrep.decompose_surfaces(S, 1e-6)
    assert plan.is_surfaces and plan.n_segments == 9
    with pytest.raises(mrep.MrepError):
        plan.export()


def test_rational_decomposition_pieces_within_tolerance():
    """NURBS: every exported polynomial cubic piece lies within tol of the rational curve (the rational oracle's
    dense check), pieces tile each curve's domain in order, and bad weights are refused."""
    curves, _, circles = gen.curves_rational(13, n_random=24, n_circles=4, per_curve=1)
    plan = mrep.decompose_curves(curves, 1e-6)
    ex = plan.export()
    diag = curves.bbox_diag()
    worst = 0.0
    for k in range(curves.n):
        p, P, U = curves.curve(k)
        w = curves.weights[curves.cp_off[k]:curves.cp_off[k + 1]]
        tab = ex["seg_t"][ex["seg_off"][k]:ex["seg_off"][k + 1]]
        assert tab[0, 0] == U[p] and tab[-1, 1] == U[-p - 1]
        np.testing.assert_array_equal(tab[1:, 0], tab[:-1, 1])
        for s in range(ex["seg_off"][k], ex["seg_off"][k + 1]):
            ta, tb = ex["seg_t"][s]
            worst = max(worst, oracle.nurbs_piece_deviation(p, P, w, U, ta, tb, ex["seg_cp"][s], 513) / (1e-6 * diag[k]))
    assert worst <= 1.0
    bad = gen.CurveSet(curves.degree, curves.cp_off, curves.cp, curves.knot_off, curves.knots, curves.weights.copy())
    bad.weights[3] = -1.0
    with pytest.raises(mrep.MrepError) as e:
        mrep.decompose_curves(bad, 1e-6)
    assert e.value.code == mrep.E_INVALID_ARG
    assert mrep._decompose_rational(1, None, None, None, None, None, None, 1e-6, 0, None) == mrep.E_INVALID_ARG
