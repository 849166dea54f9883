"""GPU parity of the paper's refinement path (MREP_OPT_CLIP: Ferrari split, elimination, rebasement, Bezier
clipping on every candidate pair) against the FP64 oracle, on the same seeded inputs as the plain path: the single
cubic, a batched-curve subset, the full batched size sampled, inversion, lattice struts and the sphere strategy."""
import sys

import numpy as np
import pytest

import oracle
from paper_2504_11498_amd import gen
from parity import compare, oracle_pieces

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mrep():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_11498_amd import mrep as m

    return m


def _run(m, geom, q, cid, invert=False, **kw):
    opts = m.default_opts("bf16", clip=True, **kw)
    qt = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    ct = torch.from_numpy(np.ascontiguousarray(cid, dtype=np.int32)).cuda()
    t, d, s, f = geom.project(qt, ct, opts, invert=invert)
    torch.cuda.synchronize()
    return {"t": t.cpu().numpy(), "dist": d.cpu().numpy(), "seg": s.cpu().numpy(), "flags": f.cpu().numpy().view(np.uint32)}


def test_clip_single_cubic_all_queries(mrep):
    curves, qs = gen.curve_single(1)
    geom = mrep.decompose_curves(curves, 1e-6).upload()
    ref = oracle.project(curves, qs.curve_id, qs.point)
    _say("[case] clip refiner, single cubic, 10000 box queries")
    out = _run(mrep, geom, qs.point, qs.curve_id)
    st = compare(curves, qs.curve_id, qs.point, out, ref, oracle_pieces(curves, 1e-6), label="clip/single")
    _say(f"[ok] {st}")


@pytest.fixture(scope="module")
def batched(mrep):
    curves, qs = gen.curves_batched(2)
    q = qs.materialise(lambda cid, t: oracle.eval_batch(curves, cid, t))
    _say("[setup] batched curves: decomposing 4096 curves on the host")
    geom = mrep.decompose_curves(curves, 1e-6).upload()
    rng = np.random.default_rng(7)
    sub = np.sort(rng.choice(qs.n, 20_000, replace=False))
    ref = oracle.project(curves, qs.curve_id[sub], q[sub])
    return curves, qs, q, geom, sub, ref, oracle_pieces(curves, 1e-6)


def test_clip_batched_subset(mrep, batched):
    curves, qs, q, geom, sub, ref, dec = batched
    _say("[case] clip refiner, batched curves, 20000-query subset")
    out = _run(mrep, geom, q[sub], qs.curve_id[sub])
    st = compare(curves, qs.curve_id[sub], q[sub], out, ref, dec, label="clip/batched")
    _say(f"[ok] {st} fullscan={np.mean((out['flags'] & mrep.F_FULLSCAN) != 0):.4f}")


def test_clip_full_size_sampled_and_agrees_with_newton_refiner(mrep, batched):
    """All 1,048,576 queries in the bench configuration: 2000 sampled outputs against the oracle, and every query's
    distance within the parity bar of the Newton refiner's."""
    curves, qs, q, geom, sub, ref, dec = batched
    _say("[case] clip refiner, full 1M queries")
    out = _run(mrep, geom, q, qs.curve_id)
    assert np.all(np.isfinite(out["dist"])) and np.all(out["seg"] >= 0)
    pick = np.sort(np.random.default_rng(11).choice(qs.n, 2000, replace=False))
    r = oracle.project(curves, qs.curve_id[pick], q[pick])
    st = compare(curves, qs.curve_id[pick], q[pick], {k: v[pick] for k, v in out.items()}, r, dec, label="clip/full")
    qt = torch.from_numpy(q).cuda()
    ct = torch.from_numpy(qs.curve_id).cuda()
    t, d, s, f = geom.project(qt, ct, mrep.default_opts("bf16"))
    torch.cuda.synchronize()
    diag = curves.bbox_diag()[qs.curve_id]
    assert np.max(np.abs(d.cpu().numpy() - out["dist"]) / diag) <= 1e-6
    _say(f"[ok] {st}")


def test_clip_inversion_of_on_curve_points(mrep, batched):
    curves, qs, q, geom, sub, ref, dec = batched
    _say("[case] clip refiner, inversion of on-curve points")
    rng = np.random.default_rng(3)
    cid = rng.integers(0, curves.n, 5000).astype(np.int32)
    t0 = rng.uniform(0, 1, 5000)
    pts = oracle.eval_batch(curves, cid, t0)
    out = _run(mrep, geom, pts, cid, invert=True)
    diag = curves.bbox_diag()[cid]
    assert np.all(out["dist"] <= 1e-6 * diag)
    assert not np.any(out["flags"] & mrep.F_OFFCURVE)
    r = oracle.project(curves, cid, pts)
    ok = (r["runner"] - r["dist"]) > 2e-6 * diag
    assert np.all(np.abs(out["t"][ok] - t0[ok]) <= 1e-7)


@pytest.mark.parametrize("strategy", ["screen", "spheres"])
def test_clip_lattice_struts(mrep, strategy):
    """Lattice struts (degree 3..9 random walks) through the screen and through the sphere strategy."""
    curves = gen.curves_lattice_geometry(55, n_curves=128)
    plan = mrep.decompose_curves(curves, 1e-6)
    n_seg = np.diff(plan.export()["seg_off"])
    qs = gen.offset_queries(155, curves, counts=gen.proportional_counts(n_seg, 128 * 128))
    q = qs.materialise(lambda cid, t: oracle.eval_batch(curves, cid, t))
    geom = plan.upload()
    sub = np.sort(np.random.default_rng(17).choice(qs.n, 3000, replace=False))
    ref = oracle.project(curves, qs.curve_id[sub], q[sub])
    _say(f"[case] clip refiner, lattice struts, {strategy}, 3000 queries")
    if strategy == "spheres":
        geom.set_strategy(mrep.STRATEGY_SPHERES)
    out = _run(mrep, geom, q[sub], qs.curve_id[sub], tuned=strategy == "spheres")
    st = compare(curves, qs.curve_id[sub], q[sub], out, ref, oracle_pieces(curves, 1e-6), label=f"clip/lattice/{strategy}")
    _say(f"[ok] {st}")
