"""HIP graph capture of a projection call: a captured mrep_project_curves replays with the same answers as the
eager call, replay after replay, with other eager work and new inputs in between (every kernel of the call
clears its own counters; nothing in it is a memset or a host synchronisation)."""
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


@pytest.mark.parametrize("mode", ["screen", "spheres", "fp64"])
def test_graph_replay_matches_eager(mrep, mode):
    _say(f"[case] graph capture and replay, {mode}")
    curves = gen.curves_batched_geometry(21, n_curves=64) if mode != "spheres" else \
        gen.curves_lattice_geometry(25, n_curves=64)
    geom = mrep.decompose_curves(curves, 1e-6).upload()
    n = 4096
    batches = []
    for b in range(4):
        qs = gen.offset_queries(300 + b, curves, per_curve=n // curves.n)
        batches.append((torch.from_numpy(qs.materialise(lambda c, t: oracle.eval_batch(curves, c, t))).cuda(),
                        torch.from_numpy(qs.curve_id).cuda()))
    opts = mrep.default_opts("fp64" if mode == "fp64" else "bf16", tuned=mode == "spheres")
    if mode == "spheres":
        geom.set_strategy(mrep.STRATEGY_SPHERES)
    ws = torch.empty(geom.workspace_bytes(n, opts), dtype=torch.uint8, device="cuda")
    q_in = batches[0][0].clone()
    c_in = batches[0][1].clone()
    outs = (torch.empty(n, dtype=torch.float64, device="cuda"), torch.empty(n, dtype=torch.float64, device="cuda"),
            torch.empty(n, dtype=torch.int32, device="cuda"), torch.empty(n, dtype=torch.int32, device="cuda"))
    # warm up on a side stream, then capture
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        geom.project(q_in, c_in, opts, workspace=ws, out=outs)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        geom.project(q_in, c_in, opts, workspace=ws, out=outs)
    torch.cuda.synchronize()
    for b in (1, 2, 3, 0, 2):
        q, c = batches[b]
        ref = [x.clone() for x in geom.project(q, c, opts)]  # eager, its own workspace
        q_in.copy_(q)
        c_in.copy_(c)
        g.replay()
        torch.cuda.synchronize()
        for x, y in zip(outs, ref):
            assert torch.equal(x, y), f"replay of batch {b} differs from the eager call"
    _say("[ok] 5 replays equal to the eager calls")
