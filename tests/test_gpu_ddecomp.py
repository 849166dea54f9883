"""GPU parity of the device decomposition (Sec. 5.2.1-5.2.2 run by kernels).

mrep_decompose_curves_device must give the host decomposition's pieces,
breakpoints and tables bit for bit: both run the same arithmetic without
contraction.  For each workload: the plan summaries agree, the exported pieces
(offsets, breakpoints, control points, span indices) are equal, and the two
uploaded geometry buffers are byte-equal.  The breakpoints themselves are
pinned to the oracle's decomposition in the host tests; a projection through
the device-built geometry is checked against the oracle here as well.  Bad
input gets the host decomposition's error codes.
"""
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


def _workloads():
    return {
        "batched_512": lambda: gen.curves_batched_geometry(n_curves=512),
        "lattice_256": lambda: gen.curves_lattice_geometry(n_curves=256),
        "degree_10_15": lambda: gen.curves_high_degree(degrees=(10, 12, 15), per_degree=4),
        "c0_corners": lambda: gen.curves_adversarial()[0],
    }


def _curves(make):
    c = make()
    return c[0] if isinstance(c, tuple) else c


@pytest.mark.parametrize("name", list(_workloads()))
def test_device_plan_equals_host_plan(mrep, name):
    curves = _curves(_workloads()[name])
    if int(np.max(curves.degree)) > 15:
        curves = curves.subset(np.nonzero(np.asarray(curves.degree) <= 15)[0])
    _say(f"[case] device decomposition {name}: {curves.n} curves")
    host = mrep.decompose_curves(curves, 1e-6)
    dev = mrep.decompose_curves_device(curves, 1e-6)
    for k in ("n_curves", "n_spans", "n_segments", "device_bytes", "max_degree"):
        assert getattr(dev.info, k) == getattr(host.info, k), k
    eh, ed = host.export(), dev.export()
    for k in eh:
        assert np.array_equal(eh[k], ed[k]), k
    gh, gd = host.upload(zero=True), dev.upload(zero=True)
    torch.cuda.synchronize()
    bh, bd = gh.buf.cpu().numpy(), gd.buf.cpu().numpy()
    assert bh.shape == bd.shape
    diff = np.nonzero(bh != bd)[0]
    assert diff.size == 0, f"{diff.size} bytes differ, first at {diff[:8]}"
    _say(f"[ok] {name}: {dev.n_segments} pieces, {dev.device_bytes} bytes equal")


def test_projection_through_device_geometry(mrep):
    curves, qs = gen.curves_batched(2, n_curves=256, per_curve=16)
    q = qs.materialise(lambda cid, t: oracle.eval_batch(curves, cid, t))
    geom = mrep.decompose_curves_device(curves, 1e-6).upload()
    out = geom.project(torch.from_numpy(q).cuda(), torch.from_numpy(qs.curve_id).cuda(), mrep.default_opts("bf16"))
    t, d, s, f = out
    torch.cuda.synchronize()
    res = {"t": t.cpu().numpy(), "dist": d.cpu().numpy(), "seg": s.cpu().numpy(), "flags": f.cpu().numpy().view(np.uint32)}
    ref = oracle.project(curves, qs.curve_id, q)
    st = compare(curves, qs.curve_id, q, res, ref, oracle_pieces(curves, 1e-6), label="device-decomposed")
    _say(f"[ok] {st}")


def test_device_decomposition_errors(mrep):
    curves = gen.curves_batched_geometry(n_curves=8)
    kn = np.array(curves.knots, copy=True)
    k0 = int(curves.knot_off[3])
    kn[k0 + 5], kn[k0 + 6] = kn[k0 + 6] + 0.1, kn[k0 + 5]  # knots of curve 3 out of order
    bad = gen.CurveSet(curves.degree, curves.cp_off, curves.cp, curves.knot_off, kn)
    with pytest.raises(mrep.MrepError) as e:
        mrep.decompose_curves_device(bad, 1e-6)
    assert e.value.code == mrep.E_BAD_KNOTS and "curve 3" in str(e.value)
    hi = gen.curves_high_degree(degrees=(16,), per_degree=1)[0]
    with pytest.raises(mrep.MrepError) as e:
        mrep.decompose_curves_device(hi, 1e-6)
    assert e.value.code == mrep.E_BAD_DEGREE
