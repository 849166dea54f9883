"""GPU parity of the device span decomposition (mrep_span_bezier_curves, Sec. 5.2.1) against the oracle's Boehm knot
insertion: every non-degenerate knot interval of the batched-curve workload, of lattice struts, and of random curves of
every degree 1..15 with repeated interior knots (zero-length intervals come back as NaN points)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2504_11498_amd import gen

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


def _random_curves(seed, degrees):
    """Random clamped curves; interior knots get multiplicity 1 .. p (p gives a C0 joint)."""
    rng = np.random.default_rng(seed)
    deg, cps, kns = [], [], []
    for p in degrees:
        n_cp = int(rng.integers(p + 1, p + 12))
        P = rng.uniform(-1, 1, (n_cp, 3)) * rng.uniform(0.1, 100)
        n_int = n_cp - p - 1
        mult = []
        while sum(mult) < n_int:
            m = int(rng.integers(1, p + 1)) if rng.random() < 0.3 else 1
            mult.append(min(m, n_int - sum(mult)))
        base = np.repeat(np.sort(rng.uniform(0.01, 0.99, len(mult))), mult)
        deg.append(p)
        cps.append(P)
        kns.append(np.concatenate([np.zeros(p + 1), base, np.ones(p + 1)]))
    cp_off = np.concatenate([[0], np.cumsum([len(c) for c in cps])]).astype(np.int64)
    k_off = np.concatenate([[0], np.cumsum([len(k) for k in kns])]).astype(np.int64)
    return gen.CurveSet(np.asarray(deg, np.int32), cp_off, np.concatenate(cps), k_off, np.concatenate(kns))


def _check(m, curves, label):
    dc = m.DeviceCurves(curves)
    bz, t = dc.span_bezier()
    torch.cuda.synchronize()
    bz, t = bz.cpu().numpy(), t.cpu().numpy()
    worst, n_spans = 0.0, 0
    for c in range(curves.n):
        p = int(curves.degree[c])
        P = curves.cp[curves.cp_off[c] : curves.cp_off[c + 1]]
        U = curves.knots[curves.knot_off[c] : curves.knot_off[c + 1]]
        ref_bz, ref_t = oracle.bezier_spans(p, P, U)
        i0, i1 = int(dc.iv_off[c]), int(dc.iv_off[c + 1])
        tt = t[i0:i1]
        np.testing.assert_array_equal(tt[:, 0], U[p : len(U) - p - 1])  # [U_q, U_q+1], q = p .. n - 1
        np.testing.assert_array_equal(tt[:, 1], U[p + 1 : len(U) - p])
        live = tt[:, 0] < tt[:, 1]
        got = bz[dc.pt_off[c] : dc.pt_off[c + 1]].reshape(i1 - i0, p + 1, 3)
        assert np.all(np.isnan(got[~live]))
        assert int(live.sum()) == ref_bz.shape[0]
        np.testing.assert_array_equal(tt[live], ref_t)
        scale = np.max(np.abs(P))
        err = np.max(np.abs(got[live] - ref_bz)) / scale if ref_bz.size else 0.0
        assert err <= 1e-13 * p, (label, c, p, err)
        worst = max(worst, err)
        n_spans += ref_bz.shape[0]
    _say(f"[ok] {label}: {curves.n} curves, {n_spans} spans, max |dQ| / max |P| = {worst:.2e}")


def test_spans_batched_curves(mrep):
    _say("[case] device spans, batched curves (4096 curves, degree 2..7)")
    curves = gen.curves_batched_geometry(2)
    _check(mrep, curves, "batched")


def test_spans_lattice_struts(mrep):
    _say("[case] device spans, lattice struts (2048 curves, degree 3..9)")
    curves = gen.curves_lattice_geometry(5, n_curves=2048)
    _check(mrep, curves, "lattice")


@pytest.mark.parametrize("lo,hi", [(1, 3), (4, 5), (6, 7), (8, 9), (1, 15)])
def test_spans_every_degree_with_repeated_knots(mrep, lo, hi):
    """Each kernel instance (largest degree 3, 5, 7, 9, 15) on random curves with repeated interior knots."""
    _say(f"[case] device spans, random curves of degree {lo}..{hi} with repeated interior knots")
    degrees = [p for p in range(lo, hi + 1) for _ in range(12)]
    curves = _random_curves(40 + hi, degrees)
    _check(mrep, curves, f"degrees {lo}..{hi}")


def test_spans_max_degree_below_a_curve_degree(mrep):
    """max_degree smaller than a curve's degree: that curve's intervals get NaN ends, the others are exact."""
    _say("[case] device spans, max_degree 3 on a batch of degrees 2..6")
    curves = _random_curves(77, [2, 3, 6, 3, 5, 2])
    dc = mrep.DeviceCurves(curves)
    dc.max_degree = 3
    bz, t = dc.span_bezier()
    torch.cuda.synchronize()
    bz, t = bz.cpu().numpy(), t.cpu().numpy()
    for c in range(curves.n):
        p, P, U = curves.curve(c)
        tt = t[dc.iv_off[c] : dc.iv_off[c + 1]]
        if p > 3:
            assert np.all(np.isnan(tt))
            continue
        ref_bz, _ = oracle.bezier_spans(p, P, U)
        live = tt[:, 0] < tt[:, 1]
        got = bz[dc.pt_off[c] : dc.pt_off[c + 1]].reshape(-1, p + 1, 3)[live]
        np.testing.assert_allclose(got, ref_bz, rtol=0, atol=1e-13 * np.max(np.abs(P)))


def test_spans_minimal_curves_and_empty_batch(mrep):
    """Curves with exactly p + 1 points (one Bezier span each); and a call with no intervals."""
    _say("[case] device spans, minimal curves and empty batch")
    rng = np.random.default_rng(5)
    deg = list(range(1, 16))
    cps = [rng.uniform(-1, 1, (p + 1, 3)) for p in deg]
    kns = [np.concatenate([np.zeros(p + 1), np.ones(p + 1)]) for p in deg]
    cp_off = np.concatenate([[0], np.cumsum([p + 1 for p in deg])]).astype(np.int64)
    k_off = np.concatenate([[0], np.cumsum([2 * p + 2 for p in deg])]).astype(np.int64)
    curves = gen.CurveSet(np.asarray(deg, np.int32), cp_off, np.concatenate(cps), k_off, np.concatenate(kns))
    dc = mrep.DeviceCurves(curves)
    bz, t = dc.span_bezier()
    torch.cuda.synchronize()
    # a single span of a clamped curve with p + 1 points is the control polygon itself
    np.testing.assert_allclose(bz.cpu().numpy(), curves.cp, rtol=0, atol=1e-14)
    np.testing.assert_array_equal(t.cpu().numpy(), np.tile([0.0, 1.0], (len(deg), 1)))
    empty = gen.CurveSet(np.zeros(0, np.int32), np.zeros(1, np.int64), np.zeros((0, 3)), np.zeros(1, np.int64),
                         np.zeros(0))
    d0 = mrep.DeviceCurves(empty)
    b0, t0 = d0.span_bezier()
    torch.cuda.synchronize()
    assert b0.numel() == 0 and t0.numel() == 0


def test_spans_full_size_lattice_sampled(mrep):
    """All 65,536 lattice struts (35.2M intervals, the size the benchmark times): every interval end checked against the
    knots, and 60 sampled curves' Bezier points against the oracle, gathered on the device."""
    _say("[case] device spans, 65,536 lattice struts, 60 sampled curves")
    curves = gen.curves_lattice_geometry(5, n_curves=65_536)
    dc = mrep.DeviceCurves(curves)
    bz, t = dc.span_bezier()
    torch.cuda.synchronize()
    assert dc.n_intervals == int(np.sum(np.diff(curves.cp_off) - curves.degree))
    # interval ends: [U_q, U_q+1] for q = p .. n - 1 of every curve (built on the host from the knots)
    q0 = np.concatenate([curves.knot_off[c] + curves.degree[c] + np.arange(curves.cp_off[c + 1] - curves.cp_off[c]
                                                                            - curves.degree[c])
                         for c in range(0, curves.n, 97)])
    ivs = np.concatenate([dc.iv_off[c] + np.arange(dc.iv_off[c + 1] - dc.iv_off[c]) for c in range(0, curves.n, 97)])
    tt = t[torch.from_numpy(ivs).cuda()].cpu().numpy()
    np.testing.assert_array_equal(tt[:, 0], curves.knots[q0])
    np.testing.assert_array_equal(tt[:, 1], curves.knots[q0 + 1])
    pick = np.sort(np.random.default_rng(23).choice(curves.n, 60, replace=False))
    for c in pick:
        p, P, U = curves.curve(c)
        ref_bz, _ = oracle.bezier_spans(p, P, U)
        rows = torch.arange(int(dc.pt_off[c]), int(dc.pt_off[c + 1]), device=bz.device)
        got = bz[rows].cpu().numpy().reshape(-1, p + 1, 3)
        tc = t[int(dc.iv_off[c]) : int(dc.iv_off[c + 1])].cpu().numpy()
        live = tc[:, 0] < tc[:, 1]
        assert int(live.sum()) == ref_bz.shape[0]
        err = np.max(np.abs(got[live] - ref_bz)) / np.max(np.abs(P))
        assert err <= 1e-13 * p, (c, p, err)
    _say(f"[ok] full-size lattice: {dc.n_intervals} intervals, {dc.n_points} Bezier points, 60 curves sampled")
