"""GPU monotonic decomposition (mrep_monotonic_split, Sec. 5.2.3): the roots of E' in (0, 1) for (query, piece)
pairs by Ferrari's method and by Newton's iteration, against the oracle's Ferrari roots on its own pieces (cubic
curves: the library's pieces equal the oracle's Boehm pieces) and against a sign scan of E' (brute force)."""
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


@pytest.fixture(scope="module")
def pairs(mrep):
    """Cubic curves of the batched distribution; each query against every piece of its curve."""
    curves = gen.curves_batched_geometry(31, n_curves=24, deg_lo=3, deg_hi=3)
    qs = gen.offset_queries(131, curves, per_curve=24)
    q = qs.materialise(lambda cid, t: oracle.eval_batch(curves, cid, t))
    plan = mrep.decompose_curves(curves, 1e-6)
    dec = oracle.decompose(curves, 1e-6 * curves.bbox_diag())
    off = np.concatenate([[0], np.cumsum(dec["counts"])])
    assert np.array_equal(np.diff(plan.export()["seg_off"]), dec["counts"])
    cid, pc, qq, R = [], [], [], []
    for i in range(qs.n):
        c = qs.curve_id[i]
        for k in range(off[c + 1] - off[c]):
            cid.append(c)
            pc.append(k)
            qq.append(q[i])
            R.append(dec["R"][off[c] + k])
    return plan.upload(), np.array(cid, np.int32), np.array(pc, np.int32), np.array(qq), np.array(R)


def _gpu(m, geom, cid, pc, q, method):
    r, c = geom.monotonic_split(torch.from_numpy(cid).cuda(), torch.from_numpy(pc).cuda(), torch.from_numpy(q).cuda(),
                                method)
    torch.cuda.synchronize()
    return r.cpu().numpy(), c.cpu().numpy()


def test_ferrari_split_matches_oracle(mrep, pairs):
    geom, cid, pc, q, R = pairs
    _say(f"[case] monotonic split, Ferrari, {cid.size} pairs")
    roots, count = _gpu(mrep, geom, cid, pc, q, mrep.ROOTS_FERRARI)
    checked = 0
    for i in range(cid.size):
        a = oracle.clip_e_poly(R[i], q[i])
        ep = np.array([(m + 1) * a[m + 1] for m in range(5)])
        ref = np.sort([x for x in oracle.ferrari_01(ep) if 0.0 < x < 1.0])
        # skip roots within 1e-6 of each other or of an end (ill-conditioned: either side may drop them)
        if ref.size and (np.min(np.concatenate([ref, 1 - ref])) < 1e-6 or (ref.size > 1 and np.min(np.diff(ref)) < 1e-4)):
            continue
        assert count[i] == ref.size, (i, roots[i], ref)
        np.testing.assert_allclose(roots[i, : count[i]], ref, rtol=0, atol=1e-9)
        checked += 1
    assert checked > 0.99 * cid.size
    _say(f"[ok] {checked} pairs, mean roots {count.mean():.3f}")


def test_roots_are_the_sign_changes_of_eprime(mrep, pairs):
    """Brute force: E' sampled on a fine grid changes sign exactly where the Ferrari roots lie."""
    geom, cid, pc, q, R = pairs
    roots, count = _gpu(mrep, geom, cid, pc, q, mrep.ROOTS_FERRARI)
    grid = np.linspace(0, 1, 4001)
    rng = np.random.default_rng(0)
    for i in rng.choice(cid.size, 400, replace=False):
        a = oracle.clip_e_poly(R[i], q[i])
        ep = np.array([(m + 1) * a[m + 1] for m in range(5)])
        v = np.polyval(ep[::-1], grid)
        ch = np.nonzero(np.sign(v[:-1]) * np.sign(v[1:]) < 0)[0]
        r = roots[i, : count[i]]
        # every grid sign change holds a root, and every root lies at a sign change (or touches zero)
        for k in ch:
            assert np.any((r >= grid[k] - 1e-12) & (r <= grid[k + 1] + 1e-12)), (i, r, grid[k])
        assert count[i] >= ch.size


def test_newton_roots_are_ferrari_roots(mrep, pairs):
    geom, cid, pc, q, R = pairs
    _say("[case] monotonic split, Newton from 8 starts")
    rf, cf = _gpu(mrep, geom, cid, pc, q, mrep.ROOTS_FERRARI)
    rn, cn = _gpu(mrep, geom, cid, pc, q, mrep.ROOTS_NEWTON)
    missed = 0
    for i in range(cid.size):
        for x in rn[i, : cn[i]]:
            assert np.min(np.abs(rf[i, : cf[i]] - x), initial=1.0) <= 1e-8, (i, rn[i], rf[i])
        missed += cf[i] - cn[i]
    _say(f"[ok] Newton roots are Ferrari roots; Ferrari found {missed} more over {cid.size} pairs")


def test_split_edge_cases(mrep, pairs):
    geom, cid, pc, q, R = pairs
    bad_c = np.array([-1, 10_000, 0, 0], np.int32)
    bad_p = np.array([0, 0, -1, 1_000_000], np.int32)
    _, c = _gpu(mrep, geom, bad_c, bad_p, q[:4], mrep.ROOTS_FERRARI)
    assert np.all(c == -1)
    with pytest.raises(mrep.MrepError):
        _gpu(mrep, geom, cid[:4], pc[:4], q[:4], 7)
    r, c = _gpu(mrep, geom, cid[:0], pc[:0], q[:0], mrep.ROOTS_NEWTON)
    assert r.shape == (0, 4) and c.shape == (0,)
