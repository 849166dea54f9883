"""GPU parity on adversarial queries: ties, C0 corners and poor conditioning.

The global-minimiser definition (Sec. 4, eq. projections) admits several correct
answers when two local minima are (nearly) equally far, and corner and end
candidates (Sec. 5.3, Properties 1-2) hold minima with no stationary point.  The
workloads (``gen.curves_adversarial``, ``gen.surfaces_mirror``) put queries on mirror
planes of symmetric curves and surfaces (exact mirror ties), between the legs of
hairpins (equidistant from two parallel legs), next to C0 joints, and near centres
of curvature (kappa -> 0).  For every query: the distance within 1e-6 * diag of the
oracle's, realised by the returned parameter on the exact geometry (the oracle's
evaluator), the returned piece holding the returned parameter, NEAR_TIE where the
oracle's runner-up lies within the tie margin (and not where it lies clearly beyond),
ILL_COND where the oracle's kappa is small; the parameter itself where the oracle's
minimum is unique and well conditioned.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2504_11498_amd import gen
from parity import compare, compare_surf, oracle_pieces

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _materialise(curves, o):
    """Absolute queries, corner queries (joint point + offset) and curvature-centre queries."""
    q_pts, c_pts = o["point"], o["point_cid"]
    q_cor = oracle.eval_batch(curves, o["corner_cid"], o["corner_t0"]) + o["corner_offset"]
    qc = []
    for cid, t0, s in zip(o["centre_cid"], o["centre_t0"], o["centre_s"]):
        p, P, U = curves.curve(cid)
        X, D1, D2 = oracle.eval_curve(p, P, U, [t0], derivs=True)
        X, D1, D2 = X[0], D1[0], D2[0]
        sp = D1 @ D1
        n = D2 - (D2 @ D1) / sp * D1  # principal normal direction times the curvature |C'|^2
        qc.append(X + s * sp / (n @ n) * n)
    q = np.concatenate([q_pts, q_cor, np.array(qc)])
    cid = np.concatenate([c_pts, o["corner_cid"], o["centre_cid"]]).astype(np.int32)
    return np.ascontiguousarray(q), cid


@pytest.fixture(scope="module")
def adv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_11498_amd import mrep

    curves, o = gen.curves_adversarial()
    q, cid = _materialise(curves, o)
    _say(f"[setup] adversarial curves: {curves.n} curves, {q.shape[0]} queries; oracle")
    ref = oracle.project(curves, cid, q)
    geom = mrep.decompose_curves(curves, 1e-6).upload()
    return mrep, curves, o, q, cid, ref, geom, oracle_pieces(curves, 1e-6)


def _np(out):
    t, d, s, f = out
    torch.cuda.synchronize()
    return {"t": t.cpu().numpy(), "dist": d.cpu().numpy(), "seg": s.cpu().numpy(),
            "flags": f.cpu().numpy().view(np.uint32)}


@pytest.mark.parametrize("mode", ["bf16", "fp64", "clip", "spheres"])
def test_curve_ties_corners_and_centres(adv, mode):
    mrep, curves, o, q, cid, ref, geom, dec = adv
    _say(f"[case] adversarial curves, {q.shape[0]} queries, {mode}")
    qt = torch.from_numpy(q).cuda()
    ct = torch.from_numpy(cid).cuda()
    if mode == "spheres":
        out = _np(geom.project_seeded(qt, ct, None, mrep.default_opts("bf16")))
    else:
        opts = mrep.default_opts("fp64" if mode == "fp64" else "bf16", clip=(mode == "clip"))
        out = _np(geom.project(qt, ct, opts))
    st = compare(curves, cid, q, out, ref, dec, label=f"adversarial/{mode}", flags=True)
    _say(f"[ok] {st}")
    # the workload is adversarial: a large share of exact ties, and ill-conditioned unique minima
    assert st["ties"] >= 0.3 * q.shape[0] and st["ill"] >= 20
    # per family: the mirror and hairpin queries hold the ties, the corner queries corner minima
    fam = o["fam"]
    hair = np.isin(cid, fam["hairpin"])
    assert np.mean((out["flags"][hair] & mrep.F_NEAR_TIE) != 0) > 0.9


def test_curve_ties_seeded(adv):
    """The seeded call's certificate path (untrained network: the walk and certificate decide)."""
    mrep, curves, o, q, cid, ref, geom, dec = adv
    nn = mrep.Network(seed=5, kind=mrep.NN_CURVE)
    _say(f"[case] adversarial curves, seeded (untrained network), {q.shape[0]} queries")
    out = _np(geom.project_seeded(torch.from_numpy(q).cuda(), torch.from_numpy(cid).cuda(), nn, mrep.default_opts("bf16")))
    st = compare(curves, cid, q, out, ref, dec, label="adversarial/seeded", flags=True)
    _say(f"[ok] {st}")


def test_corner_minima_sit_on_joints(adv):
    """Where the oracle's minimum is a C0 corner (t* at a doubled knot, unique), the GPU returns that joint."""
    mrep, curves, o, q, cid, ref, geom, dec = adv
    out = _np(geom.project(torch.from_numpy(q).cuda(), torch.from_numpy(cid).cuda(), mrep.default_opts("bf16")))
    corner = np.isin(cid, o["fam"]["corner"])
    on_joint = np.zeros(q.shape[0], bool)
    for i in np.nonzero(corner)[0]:
        p, P, U = curves.curve(cid[i])
        on_joint[i] = np.min(np.abs(np.unique(U[3:-3]) - ref["t"][i])) <= 1e-12
    diag = curves.bbox_diag()[cid]
    sel = on_joint & ((ref["runner"] - ref["dist"]) > 4e-6 * diag)
    _say(f"[case] corner minima: {int(sel.sum())} unique minima on a C0 joint")
    assert sel.sum() >= 50
    np.testing.assert_allclose(out["t"][sel], ref["t"][sel], atol=1e-12, rtol=0)


@pytest.fixture(scope="module")
def mirror_surf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_11498_amd import mrep

    S, sid, q = gen.surfaces_mirror()
    _say(f"[setup] mirror surfaces: {S.n} surfaces, {q.shape[0]} queries on the mirror plane; oracle")
    ref = oracle.surf_project(S, sid, q)
    plan = mrep.decompose_surfaces(S, 1e-6)
    return mrep, S, sid, q, ref, plan, plan.upload()


@pytest.mark.parametrize("mode", ["plain", "seeded"])
def test_surface_mirror_ties(mirror_surf, mode):
    mrep, S, sid, q, ref, plan, geom = mirror_surf
    _say(f"[case] mirror surfaces, {q.shape[0]} queries, {mode}")
    qt = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    st_ = torch.from_numpy(np.ascontiguousarray(sid, dtype=np.int32)).cuda()
    if mode == "plain":
        uv, d, p, f = geom.project_surfaces(qt, st_, mrep.default_opts())
    else:
        nn = mrep.Network(seed=3, kind=mrep.NN_SURFACE)
        uv, d, p, f = geom.project_surfaces_seeded(qt, st_, nn, mrep.default_opts())
    torch.cuda.synchronize()
    out = {"uv": uv.cpu().numpy(), "dist": d.cpu().numpy(), "patch": p.cpu().numpy(),
           "flags": f.cpu().numpy().view(np.uint32)}
    st = compare_surf(S, sid, q, out, ref, plan.export_surfaces(), label=f"mirror-surf/{mode}", flags=True)
    _say(f"[ok] {st}")
    assert st["ties"] >= 0.2 * q.shape[0]
