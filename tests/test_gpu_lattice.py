"""GPU parity on lattice-strut curves (random walks of degree 3..9 with 64..1024 control points, queries in
proportion to each curve's cubic pieces): plain BF16 and FP64 projection, the seeded and sphere-pruned
projections, against the FP64 oracle on the same seeded inputs."""
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


@pytest.fixture(scope="module")
def lattice(mrep):
    curves = gen.curves_lattice_geometry(55, n_curves=256)
    _say("[setup] lattice: decomposing 256 strut curves on the host")
    plan = mrep.decompose_curves(curves, 1e-6)
    n_seg = np.diff(plan.export()["seg_off"])
    counts = gen.proportional_counts(n_seg, 256 * 256)
    qs = gen.offset_queries(155, curves, counts=counts)
    q = qs.materialise(lambda cid, t: oracle.eval_batch(curves, cid, t))
    geom = plan.upload()
    rng = np.random.default_rng(17)
    sub = np.sort(rng.choice(qs.n, 3000, replace=False))
    _say(f"[setup] {plan.n_segments} pieces, {qs.n} queries; oracle on a 3000-query sample")
    ref = oracle.project(curves, qs.curve_id[sub], q[sub])
    return curves, qs, q, geom, sub, ref, oracle_pieces(curves, 1e-6)


def _out(t, d, s, f):
    torch.cuda.synchronize()
    return {"t": t.cpu().numpy(), "dist": d.cpu().numpy(), "seg": s.cpu().numpy(), "flags": f.cpu().numpy().view(np.uint32)}


def test_lattice_plain_all_queries_sampled(mrep, lattice):
    curves, qs, q, geom, sub, ref, dec = lattice
    _say(f"[case] lattice plain bf16, all {qs.n} queries, 3000 sampled")
    qt = torch.from_numpy(q).cuda()
    ct = torch.from_numpy(qs.curve_id).cuda()
    out = _out(*geom.project(qt, ct, mrep.default_opts("bf16")))
    assert np.all(np.isfinite(out["dist"])) and np.all(out["seg"] >= 0)
    st = compare(curves, qs.curve_id[sub], q[sub], {k: v[sub] for k, v in out.items()}, ref, dec, label="lattice/bf16")
    _say(f"[ok] {st} fullscan={np.mean((out['flags'] & mrep.F_FULLSCAN) != 0):.4f}")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lattice_exhaustive_subset(mrep, lattice, precision):
    """Every piece examined (FP64, or the FP32 tier) on the sample; the FP32 tier also lands on the BF16
    screen's parameter where the oracle's minimum is unique and well conditioned."""
    curves, qs, q, geom, sub, ref, dec = lattice
    _say(f"[case] lattice {precision}, 3000-query sample")
    qt = torch.from_numpy(np.ascontiguousarray(q[sub])).cuda()
    ct = torch.from_numpy(np.ascontiguousarray(qs.curve_id[sub])).cuda()
    out = _out(*geom.project(qt, ct, mrep.default_opts(precision)))
    st = compare(curves, qs.curve_id[sub], q[sub], out, ref, dec, label=f"lattice/{precision}")
    if precision == "fp32":
        bf = _out(*geom.project(qt, ct, mrep.default_opts("bf16")))
        diag = curves.bbox_diag()[qs.curve_id[sub]]
        wc = ((ref["runner"] - ref["dist"]) > 2e-6 * diag) & (ref["kappa"] >= 1e-3)
        assert np.abs(bf["t"] - out["t"])[wc].max() <= 1e-10
    _say(f"[ok] {st}")


@pytest.mark.parametrize("which", ["seeded", "pruned"])
def test_lattice_seeded_and_pruned(mrep, lattice, which):
    """The seeded call with an untrained network (the certificate decides, whatever the network says) and the
    sphere-pruned call: same answers as the oracle on the sample."""
    curves, qs, q, geom, sub, ref, dec = lattice
    _say(f"[case] lattice {which}, 3000-query sample")
    net = mrep.Network(seed=3) if which == "seeded" else None
    qt = torch.from_numpy(np.ascontiguousarray(q[sub])).cuda()
    ct = torch.from_numpy(np.ascontiguousarray(qs.curve_id[sub])).cuda()
    out = _out(*geom.project_seeded(qt, ct, net, mrep.default_opts("bf16")))
    st = compare(curves, qs.curve_id[sub], q[sub], out, ref, dec, label=f"lattice/{which}")
    _say(f"[ok] {st} fallback={np.mean((out['flags'] & mrep.F_NN_FALLBACK) != 0):.4f}")


@pytest.fixture(scope="module")
def trained_struts(mrep):
    """A curve network trained on 128 held-out struts (other seeds than the evaluation set)."""
    from paper_2504_11498_amd import seeding

    _say("[setup] training set: 128 held-out struts x 512 queries")
    tc = gen.curves_lattice_geometry(65, n_curves=128)
    tq = gen.offset_queries(165, tc, per_curve=512)
    q = tq.materialise(lambda cid, t: oracle.eval_batch(tc, cid, t))
    plan = mrep.decompose_curves(tc, 1e-6)
    geom = plan.upload()
    x, u, a, stats = seeding.training_pairs(plan, geom, q, tq.curve_id, seed=0)
    _say(f"[setup] {stats}")
    net = mrep.Network(seed=7)
    losses = seeding.train(net, x, u, a, epochs=10, batch=1024, lr=1e-3, seed=0)
    _say(f"[setup] loss first {losses[:20].mean():.4f} last {losses[-20:].mean():.4f} ({len(losses)} steps)")
    return net, losses, stats


def test_lattice_seeded_trained(mrep, lattice, trained_struts):
    """The network trained on held-out struts: its loss falls, the seeded call gives the oracle's answers on
    the sample, and its seeds are accepted more often than an untrained network's (what the seed gains)."""
    curves, qs, q, geom, sub, ref, dec = lattice
    net, losses, stats = trained_struts
    assert stats["label_in_candidates"] > 0.5
    assert losses[-20:].mean() < 0.8 * losses[:20].mean()
    qt = torch.from_numpy(np.ascontiguousarray(q[sub])).cuda()
    ct = torch.from_numpy(np.ascontiguousarray(qs.curve_id[sub])).cuda()
    fb = {}
    for name, nn in (("trained", net), ("untrained", mrep.Network(seed=3))):
        _say(f"[case] lattice seeded, {name} network, 3000-query sample")
        out = _out(*geom.project_seeded(qt, ct, nn, mrep.default_opts("bf16")))
        st = compare(curves, qs.curve_id[sub], q[sub], out, ref, dec, label=f"lattice/{name}")
        fb[name] = float(np.mean((out["flags"] & mrep.F_NN_FALLBACK) != 0))
        _say(f"[ok] {st} fallback={fb[name]:.4f}")
    assert fb["trained"] < fb["untrained"], fb


def test_box_schedules_identical(mrep, lattice):
    """The sphere-list kernel's schedules (4, 8, 16 lanes per query; tile map or persistent per-XCD queues) give
    bit-identical answers: the sphere strategy on all queries, the seeded call (which also exports the network's
    candidate pieces) on the sample, and the exported features."""
    curves, qs, q, geom, sub, ref, dec = lattice
    qt = torch.from_numpy(q).cuda()
    ct = torch.from_numpy(qs.curve_id).cuda()
    qs_t = torch.from_numpy(np.ascontiguousarray(q[sub])).cuda()
    cs_t = torch.from_numpy(np.ascontiguousarray(qs.curve_id[sub])).cuda()
    net = mrep.Network(seed=3)
    geom.set_strategy(mrep.STRATEGY_SPHERES)
    first = None
    try:
        for lanes in (4, 8, 16):
            for pers in (0, 1):
                _say(f"[case] box schedule lanes={lanes} persistent={pers}")
                geom.set_schedule(lanes, pers)
                assert geom.schedule()[:2] == (lanes, pers)
                plain = _out(*geom.project(qt, ct, mrep.default_opts("bf16", tuned=True)))
                seeded = _out(*geom.project_seeded(qs_t, cs_t, net, mrep.default_opts("bf16")))
                seg, x = geom.features(qs_t, cs_t)
                torch.cuda.synchronize()
                got = (plain, seeded, seg.cpu().numpy(), x.cpu().numpy())
                if first is None:
                    first = got
                    compare(curves, qs.curve_id[sub], q[sub], {k: v[sub] for k, v in plain.items()}, ref, dec,
                            label="lattice/schedule")
                    continue
                for a, b in ((first[0], got[0]), (first[1], got[1])):
                    for k in ("t", "dist", "seg", "flags"):
                        np.testing.assert_array_equal(a[k], b[k], err_msg=f"lanes={lanes} persistent={pers} {k}")
                np.testing.assert_array_equal(first[2], got[2])
                np.testing.assert_array_equal(first[3], got[3])
        with pytest.raises(mrep.MrepError):
            geom.set_schedule(5, 0)
    finally:
        geom.set_schedule(8, 0)
        geom.set_strategy(mrep.STRATEGY_SCREEN)


def test_lattice_autotuner(mrep, lattice):
    """mrep_tune_curves times both strategies on the batch; on these compact struts the sphere strategy is the
    faster one.  The tuned projection and inversion then run it, with the oracle's answers on the sample."""
    curves, qs, q, geom, sub, ref, dec = lattice
    _say("[case] lattice autotuner")
    qt = torch.from_numpy(q).cuda()
    ct = torch.from_numpy(qs.curve_id).cuda()
    strat, ms_screen, ms_spheres, outs = geom.tune(qt, ct)
    lanes, pers, sched_ms = geom.schedule()
    _say(f"[info] strategy {strat}, screen {ms_screen:.3f} ms, spheres {ms_spheres:.3f} ms; box schedule "
         f"lanes={lanes} persistent={pers}, per schedule {sched_ms}")
    assert strat == mrep.STRATEGY_SPHERES and ms_spheres < ms_screen
    assert lanes in (4, 8, 16) and pers in (0, 1) and all(m > 0 for m in sched_ms)
    assert ms_spheres == min(sched_ms)
    tuned = _out(*outs)
    compare(curves, qs.curve_id[sub], q[sub], {k: v[sub] for k, v in tuned.items()}, ref, dec, label="lattice/tuned")
    again = _out(*geom.project(qt, ct, mrep.default_opts("bf16", tuned=True)))
    for k in ("t", "dist", "seg", "flags"):
        np.testing.assert_array_equal(again[k], tuned[k])
    # inversion through the tuned strategy: on-curve points, and offset points reported off the curve
    rng = np.random.default_rng(4)
    cid = rng.integers(0, curves.n, 4000).astype(np.int32)
    t0 = rng.uniform(0, 1, 4000)
    pts = oracle.eval_batch(curves, cid, t0)
    diag = curves.bbox_diag()[cid]
    inv = _out(*geom.project(torch.from_numpy(pts).cuda(), torch.from_numpy(cid).cuda(),
                             mrep.default_opts("bf16", tuned=True), invert=True))
    assert np.all(inv["dist"] <= 1e-6 * diag) and not np.any(inv["flags"] & mrep.F_OFFCURVE)
    off = pts + rng.normal(size=pts.shape) * (0.01 * diag)[:, None]
    inv2 = _out(*geom.project(torch.from_numpy(off).cuda(), torch.from_numpy(cid).cuda(),
                              mrep.default_opts("bf16", tuned=True), invert=True))
    assert np.all(((inv2["flags"] & mrep.F_OFFCURVE) != 0) == (inv2["dist"] > 1e-6 * diag))
