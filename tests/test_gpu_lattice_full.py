"""GPU parity at the full lattice-strut size: 65,536 random-walk B-splines (degree 3..9, 64..1024 control
points), 16,777,216 queries in proportion to each curve's cubic pieces, decomposed on the device and projected
in the launch configuration the benchmark times (the autotuned sphere strategy), and with the plain BF16
screen.  The FP64 oracle checks a random sample of 512 queries one by one; properties that hold at any size
check all 16,777,216: every answer is a valid piece of its curve, no farther than the query's own base point
C(t0) (the query is that point plus an offset), and the two strategies agree on every distance."""
import sys

import numpy as np
import pytest

import oracle
from paper_2504_11498_amd import gen
from parity import compare, oracle_pieces

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N_CURVES = 65_536
SAMPLE = 512


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mrep():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_11498_amd import mrep as m

    return m


@pytest.fixture(scope="module")
def full(mrep):
    dev = torch.device("cuda", 0)
    _say(f"[setup] full lattice: generating {N_CURVES} struts")
    curves = gen.curves_lattice_geometry(5, n_curves=N_CURVES)
    cp = torch.from_numpy(np.ascontiguousarray(curves.cp)).to(dev)
    kn = torch.from_numpy(np.ascontiguousarray(curves.knots)).to(dev)
    _say("[setup] device decomposition")
    plan = mrep.decompose_curves_device(curves, 1e-6, dev, cp_dev=cp, knots_dev=kn)
    n_seg = np.diff(plan.seg_off())
    geom = plan.upload(dev)
    plan.close()
    del cp, kn
    qs = gen.offset_queries(105, curves, counts=gen.proportional_counts(n_seg, 256 * N_CURVES))
    _say(f"[setup] {int(n_seg.sum())} pieces, {qs.n} queries; evaluating base points (oracle)")
    q = qs.materialise(lambda cid, t: oracle.eval_batch(curves, cid, t))
    rng = np.random.default_rng(23)
    sub = np.sort(rng.choice(qs.n, SAMPLE, replace=False))
    # the sampled queries' curves as a set of their own (the oracle decomposes only these)
    ids, local = np.unique(qs.curve_id[sub], return_inverse=True)
    sc = curves.subset(ids)
    _say(f"[setup] oracle on {SAMPLE} sampled queries over {ids.size} curves")
    ref = oracle.project(sc, local.astype(np.int32), q[sub])
    dec = oracle_pieces(sc, 1e-6)
    yield curves, qs, q, n_seg, geom, sub, sc, local.astype(np.int32), ref, dec
    del geom
    torch.cuda.empty_cache()


def _out(t, d, s, f):
    torch.cuda.synchronize()
    return {"t": t.cpu().numpy(), "dist": d.cpu().numpy(), "seg": s.cpu().numpy(), "flags": f.cpu().numpy().view(np.uint32)}


def _all_queries(out, qs, n_seg, diag, label):
    """Properties of every answer: finite, a piece of its curve, t in [0, 1], and no farther than the base
    point C(t0) at distance |offset| (up to the distance tolerance)."""
    assert np.all(np.isfinite(out["dist"])), label
    seg_ok = (out["seg"] >= 0) & (out["seg"] < n_seg[qs.curve_id])
    assert seg_ok.all(), f"{label}: {np.count_nonzero(~seg_ok)} invalid piece indices"
    assert np.all((out["t"] >= 0.0) & (out["t"] <= 1.0)), label
    bound = np.linalg.norm(qs.offset, axis=1) + 1e-6 * diag
    far = np.nonzero(out["dist"] > bound)[0]
    assert far.size == 0, f"{label}: {far.size} answers farther than the base point, e.g. {far[:5]}"


def test_full_lattice_tuned_and_screen(mrep, full):
    curves, qs, q, n_seg, geom, sub, sc, local, ref, dec = full
    qt = torch.from_numpy(q).cuda()
    ct = torch.from_numpy(qs.curve_id).cuda()
    strat, ms_screen, ms_spheres, outs = geom.tune(qt, ct)
    _say(f"[case] full lattice tuned: strategy {strat}, screen {ms_screen:.1f} ms, spheres {ms_spheres:.1f} ms")
    assert strat == mrep.STRATEGY_SPHERES
    del outs
    tuned = _out(*geom.project(qt, ct, mrep.default_opts("bf16", tuned=True)))
    diag = curves.bbox_diag()[qs.curve_id]
    _all_queries(tuned, qs, n_seg, diag, "full/tuned")
    st = compare(sc, local, q[sub], {k: v[sub] for k, v in tuned.items()}, ref, dec, label="full/tuned", flags=True)
    _say(f"[ok] tuned {st}")
    _say("[case] full lattice plain BF16 screen")
    screen = _out(*geom.project(qt, ct, mrep.default_opts("bf16")))
    _all_queries(screen, qs, n_seg, diag, "full/screen")
    st = compare(sc, local, q[sub], {k: v[sub] for k, v in screen.items()}, ref, dec, label="full/screen", flags=True)
    _say(f"[ok] screen {st}")
    # both strategies certify the global minimum: every distance agrees within the tolerance
    gap = np.abs(tuned["dist"] - screen["dist"]) / diag
    assert gap.max() <= 2e-6, f"strategies disagree by {gap.max():.3e} of the diagonal"
    same = np.mean(tuned["seg"] == screen["seg"])
    _say(f"[ok] strategies agree: max gap {gap.max():.3e}, same piece {same:.6f}, "
         f"fullscan {np.mean((tuned['flags'] & mrep.F_FULLSCAN) != 0):.5f}")
