"""GPU parity at degrees 16..32: the exact spans are Bezier points (de Casteljau in
the FP64 polish and in evaluation) instead of the power form, which has no digits
left at these degrees.  The paper's own GPU design stops at degree 31 (Sec. 6,
discussion and limitations); here each span is one host loop and each query one
thread, so no block size caps the degree."""
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
def hd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_11498_amd import mrep

    curves, qs = gen.curves_high_degree()
    q = qs.materialise(lambda cid, t: oracle.eval_batch(curves, cid, t))
    _say(f"[setup] degree 16..32: {curves.n} curves, {qs.n} queries; decompose, oracle")
    geom = mrep.decompose_curves(curves, 1e-6).upload()
    ref = oracle.project(curves, qs.curve_id, q)
    return mrep, curves, qs, q, geom, ref, oracle_pieces(curves, 1e-6)


def _np(out):
    t, d, s, f = out
    torch.cuda.synchronize()
    return {"t": t.cpu().numpy(), "dist": d.cpu().numpy(), "seg": s.cpu().numpy(),
            "flags": f.cpu().numpy().view(np.uint32)}


@pytest.mark.parametrize("mode", ["bf16", "fp64", "clip", "spheres"])
def test_high_degree_projection_parity(hd, mode):
    mrep, curves, qs, q, geom, ref, dec = hd
    _say(f"[case] degree 16..32 projection, {qs.n} queries, {mode}")
    qt = torch.from_numpy(q).cuda()
    ct = torch.from_numpy(qs.curve_id).cuda()
    if mode == "spheres":
        out = _np(geom.project_seeded(qt, ct, None, mrep.default_opts("bf16")))
    else:
        out = _np(geom.project(qt, ct, mrep.default_opts("fp64" if mode == "fp64" else "bf16", clip=(mode == "clip"))))
    st = compare(curves, qs.curve_id, q, out, ref, dec, label=f"highdeg/{mode}")
    _say(f"[ok] {st}")
    assert st["wc_frac"] > 0.8
    # every answer was decided by the FP64 polish on the exact (Bezier) span
    assert np.all((out["flags"] & mrep.F_POLISHED) != 0)


def test_high_degree_inversion_and_eval(hd):
    mrep, curves, qs, q, geom, ref, dec = hd
    on = qs.meta["on_curve"]
    _say(f"[case] degree 16..32 inversion of {int(on.sum())} on-curve points, evaluation")
    out = _np(geom.project(torch.from_numpy(q[on]).cuda(), torch.from_numpy(qs.curve_id[on]).cuda(),
                           mrep.default_opts("bf16"), invert=True))
    diag = curves.bbox_diag()[qs.curve_id[on]]
    assert np.all(out["dist"] <= 1e-12 * diag)
    assert np.all((out["flags"] & mrep.F_OFFCURVE) == 0)
    # unique on-curve points invert to their own parameter
    uni = (ref["runner"][on] - ref["dist"][on]) > 2e-6 * diag
    np.testing.assert_allclose(out["t"][uni], qs.t0[on][uni], atol=1e-9)
    # evaluation on the Bezier spans against the oracle's de Boor
    t = np.random.default_rng(3).uniform(0, 1, qs.n)
    X = geom.eval(torch.from_numpy(qs.curve_id).cuda(), torch.from_numpy(t).cuda()).cpu().numpy()
    ref_x = oracle.eval_batch(curves, qs.curve_id, t)
    err = np.abs(X - ref_x).max(1) / curves.bbox_diag()[qs.curve_id]
    assert err.max() <= 1e-13, err.max()
