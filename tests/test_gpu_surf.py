"""GPU parity of surface projection / inversion / evaluation against the FP64 oracle."""
import sys

import numpy as np
import pytest

import oracle
from paper_2504_11498_amd import gen
from parity import T_ABS as UV_ABS, compare_surf, surf_diag as _diag

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


def _run(geom, q, sid, invert=False):
    m = sys.modules["paper_2504_11498_amd.mrep"]
    qt = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    st = torch.from_numpy(np.ascontiguousarray(sid, dtype=np.int32)).cuda()
    uv, d, p, f = geom.project_surfaces(qt, st, m.default_opts(), invert=invert)
    torch.cuda.synchronize()
    return {"uv": uv.cpu().numpy(), "dist": d.cpu().numpy(), "patch": p.cpu().numpy(),
            "flags": f.cpu().numpy().view(np.uint32)}


@pytest.fixture(scope="module")
def c3small(mrep):
    S, Q = gen.surfaces(3, n_surf=8, per_surface=600)
    sid = Q["surface_id"]
    q = oracle.surf_eval(S, sid, Q["uv0"]) + Q["offset"]
    _say("[setup] 8 surfaces (4 bicubic, 4 quintic), 4800 queries: decompose, upload, oracle")
    plan = mrep.decompose_surfaces(S, 1e-6)
    geom = plan.upload()
    ref = oracle.surf_project(S, sid, q)
    return S, Q, sid, q, plan, geom, ref


def test_surface_projection_parity(c3small):
    S, Q, sid, q, plan, geom, ref = c3small
    _say("[case] surface projection, 4800 queries (half on the surface)")
    out = _run(geom, q, sid)
    st = compare_surf(S, sid, q, out, ref, plan.export_surfaces(), label="surf")
    _say(f"[ok] {st} fullscan={np.mean((out['flags'] & 0x20) != 0):.4f}")


def test_surface_inversion(c3small):
    S, Q, sid, q, plan, geom, ref = c3small
    on = Q["on_surface"]
    _say("[case] surface inversion of on-surface points")
    x = oracle.surf_eval(S, sid[on], Q["uv0"][on])
    out = _run(geom, x, sid[on], invert=True)
    diag = _diag(S)[sid[on]]
    assert np.all(out["dist"] <= 1e-6 * diag)
    assert not np.any(out["flags"] & 0x10)
    np.testing.assert_allclose(out["uv"], Q["uv0"][on], atol=UV_ABS)
    off = x + np.random.default_rng(1).normal(size=x.shape) * (0.01 * diag)[:, None]
    out2 = _run(geom, off, sid[on], invert=True)
    assert np.all(((out2["flags"] & 0x10) != 0) == (out2["dist"] > 1e-6 * diag))


def test_surface_eval(c3small, mrep):
    S, Q, sid, q, plan, geom, ref = c3small
    rng = np.random.default_rng(4)
    s = rng.integers(0, S.n, 5000).astype(np.int32)
    uv = np.concatenate([rng.uniform(0, 1, (4996, 2)), [[0, 0], [1, 1], [0, 1], [1, 0]]])
    xyz = geom.eval_surfaces(torch.from_numpy(s).cuda(), torch.from_numpy(uv).cuda())
    torch.cuda.synchronize()
    np.testing.assert_allclose(xyz.cpu().numpy(), oracle.surf_eval(S, s, uv), atol=1e-12)


def test_surface_edge_cases(c3small, mrep):
    S, Q, sid, q, plan, geom, ref = c3small
    _say("[case] surfaces: empty, single query, bad ids, far points, deterministic order")
    e = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    geom.project_surfaces(e, torch.empty(0, dtype=torch.int32, device="cuda"))
    out = _run(geom, q, sid)
    one = _run(geom, q[7:8], sid[7:8])
    assert one["dist"][0] == out["dist"][7] and np.all(one["uv"][0] == out["uv"][7])
    rev = _run(geom, q[::-1], sid[::-1])
    np.testing.assert_array_equal(rev["uv"][::-1], out["uv"])
    np.testing.assert_array_equal(rev["dist"][::-1], out["dist"])
    bad = sid.copy()
    bad[::5] = S.n + 2
    bad[1] = -1
    ob = _run(geom, q, bad)
    isbad = (bad < 0) | (bad >= S.n)
    assert np.all(ob["flags"][isbad] & 0x40) and np.all(np.isnan(ob["dist"][isbad]))
    assert np.all(ob["patch"][isbad] == -1)
    np.testing.assert_array_equal(ob["dist"][~isbad], out["dist"][~isbad])
    # far points: projections land on the boundary or a corner, flagged
    far = np.tile(np.array([[5.0, 5.0, 0.0], [-5.0, 0.5, 0.0]]), (S.n, 1))
    fs = np.repeat(np.arange(S.n, dtype=np.int32), 2)
    of = _run(geom, far, fs)
    rf = oracle.surf_project(S, fs, far)
    compare_surf(S, fs, far, of, rf, label="far")
    assert np.all(of["flags"] & 0x8)


def test_batched_surfaces_full_size_sampled(mrep):
    """All 256 surfaces and 4,194,304 queries in the launch configuration the benchmark times; 800 sampled
    outputs checked against the oracle."""
    S, Q = gen.surfaces(3)
    _say("[setup] batched surfaces: decomposing 256 surfaces on the host")
    plan = mrep.decompose_surfaces(S, 1e-6)
    geom = plan.upload()
    sid = Q["surface_id"]
    st = torch.from_numpy(sid).cuda()
    q = (geom.eval_surfaces(st, torch.from_numpy(Q["uv0"]).cuda()) + torch.from_numpy(Q["offset"]).cuda()).contiguous()
    _say("[case] batched surfaces, 4,194,304 queries")
    uv, d, p, f = geom.project_surfaces(q, st, mrep.default_opts())
    torch.cuda.synchronize()
    out = {"uv": uv.cpu().numpy(), "dist": d.cpu().numpy(), "patch": p.cpu().numpy(), "flags": f.cpu().numpy().view(np.uint32)}
    assert np.all(np.isfinite(out["dist"])) and np.all(out["patch"] >= 0)
    rng = np.random.default_rng(21)
    pick = np.sort(rng.choice(len(sid), 800, replace=False))
    qn = q.cpu().numpy()[pick]
    ref = oracle.surf_project(S, sid[pick], qn)
    st_ = compare_surf(S, sid[pick], qn, {k: v[pick] for k, v in out.items()}, ref, plan.export_surfaces(), label="c3")
    _say(f"[ok] {st_}")
