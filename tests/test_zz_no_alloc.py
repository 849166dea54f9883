"""GPU: the allocation-free projection (mrep_project_curves_noalloc, fixed per-GPU
scratch) against the workspace entry point (mrep_project_curves) through the C ABI,
on two calls in a row, the second with a smaller batch, and against the FP64 oracle."""
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
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_11498_amd import mrep

    curves, qs = gen.curves_batched(2, n_curves=512, per_curve=256)
    q = qs.materialise(lambda cid, t: oracle.eval_batch(curves, cid, t))
    geom = mrep.decompose_curves(curves, 1e-6).upload()
    return mrep, curves, qs, q, geom


def _np(out):
    t, d, s, f = out
    torch.cuda.synchronize()
    return {"t": t.cpu().numpy(), "dist": d.cpu().numpy(), "seg": s.cpu().numpy(),
            "flags": f.cpu().numpy().view(np.uint32)}


def _same(a, b, label):
    for k in ("t", "dist", "seg", "flags"):
        assert np.array_equal(a[k], b[k]), f"{label}: {k} differs at {np.nonzero(a[k] != b[k])[0][:5]}"


@pytest.mark.parametrize("precision", ["bf16", "fp64"])
def test_noalloc_equals_workspace_call_twice(setup, precision):
    mrep, curves, qs, q, geom = setup
    opts = mrep.default_opts(precision)
    rng = np.random.default_rng(11)
    # first call: every query; second: a smaller, reordered subset (the scratch keeps the first call's contents)
    sizes = [qs.n, 20_000]
    for k, n in enumerate(sizes):
        idx = np.arange(qs.n) if k == 0 else np.sort(rng.choice(qs.n, n, replace=False))[::-1].copy()
        _say(f"[case] noalloc {precision} call {k + 1}: {n} queries")
        qt = torch.from_numpy(np.ascontiguousarray(q[idx])).cuda()
        ct = torch.from_numpy(np.ascontiguousarray(qs.curve_id[idx], dtype=np.int32)).cuda()
        a = _np(geom.project_noalloc(qt, ct, opts))
        b = _np(geom.project(qt, ct, opts))
        _same(a, b, f"{precision}/call{k + 1}")
        if k == 1:
            ref = oracle.project(curves, qs.curve_id[idx], q[idx])
            st = compare(curves, qs.curve_id[idx], q[idx], a, ref, oracle_pieces(curves, 1e-6),
                         label=f"noalloc/{precision}")
            _say(f"[ok] {st}")


def test_noalloc_rejects_batches_beyond_the_scratch(setup):
    mrep, curves, qs, q, geom = setup
    opts = mrep.default_opts("bf16")
    n = 1
    while geom.workspace_bytes(n, opts) <= mrep.NOALLOC_SCRATCH_BYTES:
        n *= 2
    _say(f"[case] noalloc over the limit: {n} queries ({geom.workspace_bytes(n, opts)} bytes)")
    # the size check runs before any device work: the arrays are never read
    qt = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    ct = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(mrep.MrepError) as e:
        geom.project_noalloc(qt, ct, opts)
    assert e.value.code == mrep.E_SMALL_BUFFER
    # a timed call is refused (its events would be created)
    with pytest.raises(mrep.MrepError):
        geom.project_noalloc(qt[:16], ct[:16], mrep.default_opts("bf16", time_stages=True))
    # the entry point still works after the refusals
    out = _np(geom.project_noalloc(torch.from_numpy(np.ascontiguousarray(q[:64])).cuda(),
                                   torch.from_numpy(np.ascontiguousarray(qs.curve_id[:64], dtype=np.int32)).cuda(), opts))
    ref = oracle.project(curves, qs.curve_id[:64], q[:64])
    compare(curves, qs.curve_id[:64], q[:64], out, ref, label="noalloc/after-refusal")
