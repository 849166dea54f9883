"""GPU tests of the seeding network (forward, backward, Adam, training) and of the
seeded and sphere-pruned projections, against the FP64 oracle on the same seeded inputs."""
import sys

import numpy as np
import pytest

import oracle
from paper_2504_11498_amd import gen
from parity import compare, oracle_pieces

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NIN, NH, NOUT = 15, 128, 2


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mrep():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_11498_amd import mrep as m

    return m


def _params(seed):
    """Seeded parameters (numpy): weights uniform in +-1/sqrt(fan_in), biases uniform in +-0.1."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in [(NH, NIN), (NH, NH), (NOUT, NH)]:
        a = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-a, a, fan_out * fan_in))
        parts.append(rng.uniform(-0.1, 0.1, fan_out))
    return np.concatenate(parts).astype(np.float32)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _blocks(v):
    offs = np.cumsum([0, NH * NIN, NH, NH * NH, NH, NOUT * NH, NOUT])
    return [v[offs[i]:offs[i + 1]] for i in range(6)]


def test_forward_and_fused_inference_match_oracle(mrep):
    _say("[case] network forward: training kernels and fused kernel vs oracle, 1000 rows")
    p = _params(1)
    rng = np.random.default_rng(2)
    x = (rng.normal(size=(1000, NIN)) * 2.0).astype(np.float32)
    net = mrep.Network(seed=None)
    net.set_params(p)
    xt = torch.from_numpy(x).cuda()
    y_f = net.forward(xt).cpu().numpy()
    y_i = net.infer(xt).cpu().numpy()
    _, y_ref, _ = oracle.mlp_loss(p.astype(np.float64), x.astype(np.float64))
    for k in range(NOUT):
        assert _rel(y_f[:, k], y_ref[:, k]) <= 2e-2, ("forward", k, _rel(y_f[:, k], y_ref[:, k]))
        assert _rel(y_i[:, k], y_ref[:, k]) <= 2e-2, ("infer", k, _rel(y_i[:, k], y_ref[:, k]))
    # both paths round the same operands to BF16; only the FP32 summation order differs
    assert _rel(y_i, y_f) <= 2e-3
    # empty and single-row calls
    assert net.infer(xt[:0]).shape == (0, 2)
    one = net.infer(xt[7:8].contiguous()).cpu().numpy()
    np.testing.assert_allclose(one[0], y_i[7], rtol=0, atol=1e-6)


def test_gradient_matches_oracle(mrep):
    _say("[case] network loss and gradient vs oracle, 777 rows")
    p = _params(3)
    rng = np.random.default_rng(4)
    B = 777
    x = rng.normal(size=(B, NIN)).astype(np.float32)
    us = rng.uniform(0, 1, B).astype(np.float32)
    ac = (rng.uniform(size=B) < 0.5).astype(np.float32)
    net = mrep.Network(seed=None)
    net.set_params(p)
    loss = torch.zeros(1, device="cuda")
    grad = torch.zeros(mrep.nn_param_count(), device="cuda")
    xt, ut, at = (torch.from_numpy(v).cuda() for v in (x, us, ac))
    net.train_step(xt, ut, at, lr=0.0, loss=loss, grad=grad)
    torch.cuda.synchronize()
    l_ref, _, g_ref = oracle.mlp_loss(p.astype(np.float64), x.astype(np.float64), us.astype(np.float64),
                                      ac.astype(np.float64), grad=True)
    assert abs(float(loss.item()) - l_ref) <= 1e-2 * abs(l_ref)
    g = grad.cpu().numpy()
    rels = [_rel(a, b) for a, b in zip(_blocks(g), _blocks(g_ref))]
    _say(f"[ok] BF16 gradient relative L2 per block {[f'{r:.2e}' for r in rels]}")
    assert max(rels) <= 2e-2, rels
    # lr = 0 leaves the parameters unchanged
    np.testing.assert_array_equal(net.get_params(), p)
    # FP32-compute debug mode: the same step without BF16 rounding, to 1e-5 of the FP64 reference
    net.set_compute(mrep.NN_COMPUTE_FP32)
    grad.zero_()
    net.train_step(xt, ut, at, lr=0.0, loss=loss, grad=grad)
    torch.cuda.synchronize()
    net.set_compute(mrep.NN_COMPUTE_BF16)
    g32 = grad.cpu().numpy()
    rels32 = [_rel(a, b) for a, b in zip(_blocks(g32), _blocks(g_ref))]
    _say(f"[ok] FP32 gradient relative L2 per block {[f'{r:.2e}' for r in rels32]}")
    assert max(rels32) <= 1e-5, rels32
    assert abs(float(loss.item()) - l_ref) <= 1e-5 * abs(l_ref)


def test_adam_first_step_and_row_gather(mrep):
    """Adam's first bias-corrected step is -lr g / (|g| + eps); a gathered batch equals the materialised one."""
    _say("[case] Adam first step, minibatch gather")
    p = _params(5)
    rng = np.random.default_rng(6)
    N, B = 3000, 512
    x = rng.normal(size=(N, NIN)).astype(np.float32)
    us = rng.uniform(0, 1, N).astype(np.float32)
    ac = (rng.uniform(size=N) < 0.5).astype(np.float32)
    rows = np.sort(rng.choice(N, B, replace=False)).astype(np.int32)
    xt, ut, at = (torch.from_numpy(v).cuda() for v in (x, us, ac))
    net = mrep.Network(seed=None)
    net.set_params(p)
    g1 = torch.zeros(mrep.nn_param_count(), device="cuda")
    net.train_step(xt, ut, at, rows=torch.from_numpy(rows).cuda(), lr=1e-3, grad=g1)
    torch.cuda.synchronize()
    g = g1.cpu().numpy()
    step = net.get_params().astype(np.float64) - p
    want = -1e-3 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(step, want, rtol=0, atol=2e-6)
    # the same batch passed materialised gives the same gradient bit for bit
    net2 = mrep.Network(seed=None)
    net2.set_params(p)
    g2 = torch.zeros_like(g1)
    net2.train_step(xt[rows].contiguous(), ut[rows].contiguous(), at[rows].contiguous(), lr=0.0, grad=g2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(g2.cpu().numpy(), g)


# --------------------------------------------------------------------------- seeded projection
@pytest.fixture(scope="module")
def trained(mrep):
    """A network trained on held-out geometry (other seeds than the evaluation set)."""
    from paper_2504_11498_amd import seeding

    _say("[setup] training set: 128 held-out curves x 400 queries")
    curves = gen.curves_batched_geometry(31, n_curves=128)
    qs = gen.offset_queries(131, curves, per_curve=400)
    q = qs.materialise(lambda cid, t: oracle.eval_batch(curves, cid, t))
    plan = mrep.decompose_curves(curves, 1e-6)
    geom = plan.upload()
    x, u, a, stats = seeding.training_pairs(plan, geom, q, qs.curve_id, seed=0)
    _say(f"[setup] {stats}")
    net = mrep.Network(seed=7)
    losses = seeding.train(net, x, u, a, epochs=16, batch=1024, lr=1e-3, seed=0)
    _say(f"[setup] loss first {losses[:20].mean():.4f} last {losses[-20:].mean():.4f} ({len(losses)} steps)")
    return net, losses, stats


def test_training_reduces_loss(trained):
    net, losses, stats = trained
    assert stats["label_in_candidates"] > 0.5
    assert losses[-20:].mean() < 0.7 * losses[:20].mean()


@pytest.fixture(scope="module")
def evalset(mrep):
    curves = gen.curves_batched_geometry(2, n_curves=256)
    qs = gen.offset_queries(102, curves, per_curve=61)
    q = qs.materialise(lambda cid, t: oracle.eval_batch(curves, cid, t))
    _say("[setup] evaluation set: 256 curves x 61 queries, oracle projection")
    plan = mrep.decompose_curves(curves, 1e-6)
    geom = plan.upload()
    ref = oracle.project(curves, qs.curve_id, q)
    return curves, qs.curve_id, q, geom, ref, oracle_pieces(curves, 1e-6)


def _seeded(geom, q, cid, net):
    m = sys.modules["paper_2504_11498_amd.mrep"]
    qt = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    ct = torch.from_numpy(np.ascontiguousarray(cid, dtype=np.int32)).cuda()
    t, d, s, f = geom.project_seeded(qt, ct, net, m.default_opts("bf16"))
    torch.cuda.synchronize()
    return {"t": t.cpu().numpy(), "dist": d.cpu().numpy(), "seg": s.cpu().numpy(), "flags": f.cpu().numpy().view(np.uint32)}


@pytest.mark.parametrize("which", ["trained", "untrained", "pruned"])
def test_seeded_projection_parity(mrep, trained, evalset, which):
    curves, cid, q, geom, ref, dec = evalset
    net = {"trained": trained[0], "untrained": None, "pruned": None}[which]
    if which == "untrained":
        net = mrep.Network(seed=99)
    _say(f"[case] seeded projection ({which}), {cid.shape[0]} queries")
    out = _seeded(geom, q, cid, net)
    st = compare(curves, cid, q, out, ref, dec, label=f"seeded/{which}")
    fb = float(np.mean((out["flags"] & mrep.F_NN_FALLBACK) != 0))
    _say(f"[ok] {st} fallback={fb:.4f}")
    if which == "pruned":
        assert fb == 0.0
    if which == "trained":
        assert fb < 0.5


def test_seeded_edge_cases(mrep, trained):
    _say("[case] seeded edge cases: empty, single query, bad ids, endpoints, one-span curves")
    net = trained[0]
    rng = np.random.default_rng(12)
    degs, cps, kts = [], [], []
    for p in [1, 2, 3, 5, 7]:
        degs.append(p), cps.append(rng.uniform(0, 1, (p + 1, 3))), kts.append(np.r_[np.zeros(p + 1), np.ones(p + 1)])
    curves = gen._pack(degs, cps, kts)
    geom = mrep.decompose_curves(curves, 1e-6).upload()
    e = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    geom.project_seeded(e, torch.empty(0, dtype=torch.int32, device="cuda"), net)
    cid = np.repeat(np.arange(curves.n, dtype=np.int32), 100)
    q = rng.uniform(-0.5, 1.5, (cid.shape[0], 3))
    for c in range(curves.n):
        p, P, U = curves.curve(c)
        q[c * 100] = P[0]
        q[c * 100 + 1] = P[-1]
        q[c * 100 + 2] = P[0] + 100.0
    ref = oracle.project(curves, cid, q)
    for which in (net, None):
        out = _seeded(geom, q, cid, which)
        compare(curves, cid, q, out, ref, oracle_pieces(curves, 1e-6), label="seeded-edge")
        for c in range(curves.n):
            assert abs(out["t"][c * 100]) <= 1e-12 and abs(out["t"][c * 100 + 1] - 1.0) <= 1e-12
        one = _seeded(geom, q[5:6], cid[5:6], which)
        assert one["t"][0] == out["t"][5] and one["dist"][0] == out["dist"][5]
    bad = cid.copy()
    bad[::7] = curves.n + 3
    bad[3] = -1
    out = _seeded(geom, q, bad, net)
    isbad = (bad < 0) | (bad >= curves.n)
    assert np.all((out["flags"][isbad] & 0x40) != 0) and np.all(np.isnan(out["dist"][isbad]))
    assert np.all(np.isfinite(out["dist"][~isbad]))


def test_features_candidates_are_nearest_spheres(mrep, evalset):
    """The exported candidates are valid curve-local pieces, distinct, and the label piece is usually among them."""
    curves, cid, q, geom, ref, dec = evalset
    qt = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    ct = torch.from_numpy(np.ascontiguousarray(cid, dtype=np.int32)).cuda()
    seg, x = geom.features(qt, ct)
    torch.cuda.synchronize()
    seg, x = seg.cpu().numpy(), x.cpu().numpy()
    n_seg = np.diff(dec[1])[cid]
    assert np.all((seg >= 0) & (seg < n_seg[:, None]) | (seg == -1))
    srt = np.sort(seg, axis=1)
    assert not np.any((srt[:, 1:] == srt[:, :-1]) & (srt[:, 1:] >= 0))
    assert np.all(np.isfinite(x))
    # features are centred control points: the four points' mean is zero
    cps = x[:, :, :12].reshape(-1, 4, 4, 3)
    assert np.abs(cps.mean(axis=2)).max() <= 1e-5
