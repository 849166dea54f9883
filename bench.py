"""Throughput of batched point projection onto B-spline curves on one MI355X.

Headline workload: lattice struts at full size -- 65,536 clamped random-walk
B-splines (degree U{3..9}, 64..1024 control points, non-uniform knots),
decomposed to cubic Bezier pieces at 1e-6 of each curve's box diagonal;
16,777,216 queries split across the curves in proportion to their cubic pieces,
each a Gaussian offset (0.05 * diagonal) from a parameter-uniform curve point.
One step is one projection call on all queries with the plain method in the
strategy the autotuner picks for this batch; the plain MFMA screen, the
NN-seeded call and the sphere-pruned call are timed beside it.

Prints one JSON line: the headline with its roofline and the CPU oracle
baseline, plus blocks for the batched curves, a single cubic (latency),
surfaces and the device span decomposition.  ``--gpus`` above 1 is refused:
the library runs on one GPU per process.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "point projections/s (err≤1e-6·bbox), plain vs NN-seeded, curves+surfaces"
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 MFMA
HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector
FLOPS_PER_SAMPLE_METHOD = 2 * 19  # the monomial-form distance of one (query, piece, sample): 19 multiply-adds
FLOPS_PER_SAMPLE_PADDED = 2 * 32  # one 16x16x32 MFMA output element per (query, piece, sample)
FLOPS_PER_PAIR = 32 * 2 * 12  # refine of one (query, piece) pair: 32 sampled distances of 12 FP32 FMA
FLOPS_PER_SPHERE_TEST = 10  # |q - c| - r against a bound: 3 sub, 3 mul, 2 add, sqrt, sub
MLP_CURVE_FLOPS = 2 * (15 * 128 + 128 * 128 + 128 * 2)  # curve network forward per row


def _kernel_source_hash():
    with open(os.path.join(ROOT, "paper_2504_11498_amd", "csrc", "mrep_screen.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic():
    """HBM bytes per screen launch from committed rocprofv3 counter runs, if still current."""
    path = os.path.join(ROOT, "profiles", "screen_bf16_batched_curves_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256_16") != _kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def _span_traffic():
    """HBM bytes per span-decomposition launch, per workload, from committed rocprofv3 counter runs, if still current."""
    path = os.path.join(ROOT, "profiles", "span_bezier_curves_traffic.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, "paper_2504_11498_amd", "csrc", "mrep_spans.hip"), "rb") as f:
        if rec.get("kernel_source_sha256_16") != hashlib.sha256(f.read()).hexdigest()[:16]:
            return {}
    return {k: v.get("hbm_bytes_per_launch") for k, v in rec.get("workloads", {}).items()}


# the sources each headline kernel is built from (its file and the headers it includes)
KERNEL_SOURCES = {
    "k_box": ["mrep_nn.hip", "mrep_refine.h", "mrep_dev.h", "mrep_internal.h", "mrep.h"],
    "k_pairs": ["mrep_device.hip", "mrep_refine.h", "mrep_dev.h", "mrep_internal.h", "mrep.h"],
    "k_finish": ["mrep_device.hip", "mrep_refine.h", "mrep_dev.h", "mrep_internal.h", "mrep.h"],
}


def sources_hash(names):
    h = hashlib.sha256()
    for name in names:
        d = "include" if name == "mrep.h" else os.path.join("paper_2504_11498_amd", "csrc")
        h.update(name.encode())
        with open(os.path.join(ROOT, d, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _lattice_traffic():
    """HBM bytes per launch of the lattice headline's kernels (k_box, k_pairs, k_finish of the sphere-strategy
    call) from committed rocprofv3 counter runs, for each kernel whose sources have not changed since."""
    path = os.path.join(ROOT, "profiles", "lattice_struts_traffic.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        rec = json.load(f)
    return {k: v.get("hbm_bytes_per_launch") for k, v in rec.get("kernels", {}).items()
            if k in KERNEL_SOURCES and v.get("sources_sha256_16") == sources_hash(KERNEL_SOURCES[k])}


def nn_training_block(dev, batch=4096, steps=200):
    """One training step (gather, forward, loss, backward, Adam) of each network kind at a fixed batch on
    synthetic rows, timed over `steps` steps; flops of the three layers' products (forward, input gradients
    of layers 2 and 3, weight gradients) against the BF16 MFMA peak."""
    import torch

    from paper_2504_11498_amd import mrep

    out = {"batch": batch, "steps": steps}
    g = torch.Generator(device="cpu").manual_seed(0)
    for kind, name in ((mrep.NN_CURVE, "curve"), (mrep.NN_SURFACE, "surface")):
        n_in, n_out = mrep.NN_DIMS[kind]
        h = 128
        n = 16 * batch
        x = torch.randn(n, n_in, generator=g).to(dev)
        u = torch.rand(n * (n_out - 1), generator=g).to(dev)
        a = (torch.rand(n, generator=g) > 0.5).float().to(dev)
        rows = torch.randperm(n, generator=g).to(torch.int32).to(dev)
        net = mrep.Network(dev, seed=1, kind=kind)
        for i in range(5):
            net.train_step(x, u, a, rows=rows[:batch], lr=1e-3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            net.train_step(x, u, a, rows=rows[(i % 16) * batch:(i % 16 + 1) * batch], lr=1e-3)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        flop = 2 * batch * ((n_in * h + h * h + h * n_out) + (h * n_out + h * h) + (n_in * h + h * h + h * n_out))
        tf = flop / (ms * 1e-3) / 1e12
        out[name] = {"ms_per_step": ms, "flop_per_step": flop, "achieved_tflops": tf, "frac_bf16_peak": tf / 2500.0,
                     "layers": f"{n_in}-{h}-{h}-{n_out}"}
    return out


def summarize_rocprof(path):
    """Per-kernel duration summary (calls, mean/min/max microseconds, total ms) of a rocprofv3 SQLite result."""
    import sqlite3

    con = sqlite3.connect(path)
    rows = con.execute(
        "select name, count(*), avg(end-start), min(end-start), max(end-start), sum(end-start) "
        "from kernels group by name order by sum(end-start) desc").fetchall()
    print(f"{'kernel':70s} {'calls':>5s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'total_ms':>10s}")
    for name, n, avg, lo, hi, tot in rows:
        print(f"{name[:70]:70s} {n:5d} {avg / 1e3:10.1f} {lo / 1e3:10.1f} {hi / 1e3:10.1f} {tot / 1e6:10.3f}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-seeded", action="store_true", help="skip the learned-seeding and sphere-pruned variants")
    ap.add_argument("--no-surfaces", action="store_true", help="skip the batched-surfaces workload")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-curves workload block")
    ap.add_argument("--no-single", action="store_true", help="skip the single-cubic latency block")
    ap.add_argument("--no-spans", action="store_true", help="skip the device span decomposition block")
    ap.add_argument("--no-host-decompose", action="store_true",
                    help="lattice: skip the host decomposition that the device decomposition is timed and compared "
                         "against (profiling runs)")
    ap.add_argument("--no-clip", action="store_true",
                    help="skip the batched curves with the paper's refinement path (MREP_OPT_CLIP)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the autotuner and small-batch graph measurements on the batched curves")
    ap.add_argument("--lattice-curves", type=int, default=65_536,
                    help="strut curves of the headline lattice workload (65536 = the full microstructure "
                         "configuration; queries = 256 per curve)")
    ap.add_argument("--summarize-rocprof", metavar="RESULTS_DB", help="print a kernel summary of a rocprofv3 result and exit")
    ap.add_argument("--train-step", action="store_true",
                    help="time network training steps (batch 4096, both network kinds), print one JSON line and exit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run three 512 MiB device-to-device copies and exit (scales the HBM byte counters)")
    args = ap.parse_args()
    if args.summarize_rocprof:
        summarize_rocprof(args.summarize_rocprof)
        return
    if args.calibrate_copy:
        import torch

        x = torch.ones(512 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print("copied 3 x 512 MiB", flush=True)
        return
    if args.train_step:
        import torch

        print(json.dumps(nn_training_block(torch.device("cuda", 0))), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    result = lattice_headline(args, dev)
    torch.cuda.empty_cache()
    if not args.no_batched:
        result["batched_curves"] = batched_curves_block(args, dev)
        torch.cuda.empty_cache()
    if not args.no_single:
        result["single_cubic"] = single_cubic_block(args, dev)
        result["nn_training"] = nn_training_block(dev)
    if not args.no_surfaces:
        torch.cuda.empty_cache()
        result["surfaces"] = surfaces_bench(args, dev)
    if not args.no_spans:
        torch.cuda.empty_cache()
        from paper_2504_11498_amd import gen

        result["span_decomposition"] = span_decomposition(gen.curves_batched_geometry(2), args, dev)
    print(json.dumps(result), flush=True)


def _say(tag, msg):
    print(f"[{tag} {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def host_points(curves, qs):
    """The query points C(t0) + offset on the host, evaluated by scipy's B-spline routine (neither the oracle nor
    the library under test), so that the GPU and the oracle's sample see the same inputs."""
    from scipy.interpolate import BSpline

    cid = np.asarray(qs.curve_id)
    order = np.argsort(cid, kind="stable")
    bounds = np.searchsorted(cid[order], np.arange(curves.n + 1))
    out = np.empty((cid.shape[0], 3))
    for c in np.nonzero(np.diff(bounds))[0]:
        idx = order[bounds[c]:bounds[c + 1]]
        p, P, U = curves.curve(int(c))
        out[idx] = BSpline(U, P, p)(qs.t0[idx])
    return np.ascontiguousarray(out + qs.offset)


def host_surface_points(S, Q):
    """Surface query points S(u0, v0) + offset on the host, by scipy's tensor-product B-spline routine."""
    from scipy.interpolate import NdBSpline

    sid = np.asarray(Q["surface_id"])
    out = np.empty((sid.shape[0], 3))
    for k in range(S.n):
        idx = np.nonzero(sid == k)[0]
        if idx.size == 0:
            continue
        P = S.cp[S.cp_off[k]:S.cp_off[k + 1]].reshape(int(S.n_u[k]), int(S.n_v[k]), 3)
        ku = S.ku[S.ku_off[k]:S.ku_off[k + 1]]
        kv = S.kv[S.kv_off[k]:S.kv_off[k + 1]]
        out[idx] = NdBSpline((ku, kv), P, (int(S.deg_u[k]), int(S.deg_v[k])))(Q["uv0"][idx])
    return np.ascontiguousarray(out + Q["offset"])


def device_decomposition(args, dev, curves):
    """Decompose the batch on the device (Sec. 5.2.1-5.2.2 by kernels) and, unless --no-host-decompose, on the
    host too: the host time, the device time (decomposition, then the table build of mrep_upload; inputs already
    resident), and whether the two geometry buffers are byte-equal.  Returns the device geometry."""
    import torch

    from paper_2504_11498_amd import mrep

    out = {}
    geom_h = None
    if not args.no_host_decompose:
        t0 = time.perf_counter()
        plan_h = mrep.decompose_curves(curves, 1e-6)
        out["host_s"] = time.perf_counter() - t0
        _say("decompose", f"host: {plan_h.n_segments} pieces in {out['host_s']:.1f} s; uploading")
        t0 = time.perf_counter()
        geom_h = plan_h.upload(dev, zero=True)
        torch.cuda.synchronize()
        out["host_upload_s"] = time.perf_counter() - t0  # PCIe copy of the host tables
        del plan_h
    cp = torch.from_numpy(np.ascontiguousarray(curves.cp, dtype=np.float64)).to(dev)
    kn = torch.from_numpy(np.ascontiguousarray(curves.knots, dtype=np.float64)).to(dev)
    mrep.decompose_curves_device(curves, 1e-6, dev, cp_dev=cp, knots_dev=kn).close()  # first launch of each kernel
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = mrep.decompose_curves_device(curves, 1e-6, dev, cp_dev=cp, knots_dev=kn)
    torch.cuda.synchronize()
    out["device_s"] = time.perf_counter() - t0
    buf = torch.zeros(max(plan.device_bytes, 256), dtype=torch.uint8, device=dev)  # allocation not timed
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    geom = plan.upload(dev, buf=buf)
    torch.cuda.synchronize()
    out["device_tables_s"] = time.perf_counter() - t0
    out["pieces"] = int(plan.n_segments)
    out["spans"] = int(plan.info.n_spans)
    out["geometry_bytes"] = int(plan.device_bytes)
    if geom_h is not None:
        out["device_equals_host"] = bool(geom_h.buf.numel() == geom.buf.numel() and torch.equal(geom_h.buf, geom.buf))
        out["speedup_vs_host"] = out["host_s"] / (out["device_s"] + out["device_tables_s"])
        del geom_h
    _say("decompose", f"device: {plan.n_segments} pieces in {out['device_s']:.3f} s + tables "
                      f"{out['device_tables_s']:.3f} s; equal to host: {out.get('device_equals_host')}")
    n_seg = np.diff(plan.seg_off())
    n_pieces = int(plan.n_segments)
    plan.close()
    torch.cuda.empty_cache()
    out.update(geom=geom, n_seg=n_seg, n_pieces=n_pieces)
    return out


def lattice_headline(args, dev):
    """The headline: lattice struts at full size -- 65,536 random-walk B-splines (degree U{3..9}, 64..1024 control
    points, steps N(0, 0.01^2)), 16,777,216 queries in proportion to each curve's cubic pieces, offset by
    N(0, (0.05 diag)^2) from parameter-uniform curve points.  A step = one projection call on all queries with the
    plain method in the strategy the autotuner picks on this batch (MFMA screen or sphere lists); beside it the
    plain screen, the NN-seeded call (curve network trained on held-out struts) and the sphere-pruned call."""
    import torch

    from paper_2504_11498_amd import gen, mrep, seeding

    n_curves = int(args.lattice_curves)
    _say("lattice", f"generating {n_curves} struts")
    curves = gen.curves_lattice_geometry(5, n_curves=n_curves)
    dec = device_decomposition(args, dev, curves)
    geom, n_seg, n_pieces = dec.pop("geom"), dec.pop("n_seg"), dec.pop("n_pieces")
    qs = gen.offset_queries(105, curves, counts=gen.proportional_counts(n_seg, 256 * n_curves))
    cid = torch.from_numpy(qs.curve_id).to(dev)
    q_host = host_points(curves, qs)
    q = torch.from_numpy(q_host).to(dev)
    n = q.shape[0]
    # work units of the screen: every (query, piece of its curve, sample)
    samples = 32 * int(np.sum(n_seg[qs.curve_id].astype(np.int64)))

    def outs_like():
        return (torch.empty(n, dtype=torch.float64, device=dev), torch.empty(n, dtype=torch.float64, device=dev),
                torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev))

    # the plain method: the autotuner's strategy on this batch
    strat, ms_screen, ms_spheres, _ = geom.tune(q, cid)
    lanes, persistent, sched_ms = geom.schedule()
    _say("lattice", f"{n} queries; tuner: screen {ms_screen:.2f} ms, spheres {ms_spheres:.2f} ms (box kernel "
                    f"{lanes} lanes per query, {'persistent' if persistent else 'tile map'})")
    topts = mrep.default_opts("bf16", time_stages=True, tuned=True)
    tws = torch.empty(geom.workspace_bytes(n, topts), dtype=torch.uint8, device=dev)
    outs = outs_like()

    def tuned():
        geom.project(q, cid, topts, workspace=tws, out=outs)

    for _ in range(max(1, args.warmup)):
        tuned()
        mrep.last_stage_times()
    torch.cuda.synchronize()
    stage = np.zeros(mrep.N_STAGES)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        tuned()
        st = mrep.last_stage_times()
        stage[:len(st)] += st
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = e0.elapsed_time(e1) / args.steps
    stage /= args.steps
    ovf, pairs, tests = geom.workspace_counts(tws, tests=True)
    del tws
    value = n / (ms / 1e3)
    _say("lattice", f"plain ({['screen', 'spheres'][strat]}) {ms:.2f} ms per call")
    strategy = ["screen", "spheres"][strat]
    if strat == mrep.STRATEGY_SPHERES:
        stage_ms = {"group": float(stage[0]), "candidates_k_box": float(stage[1]), "pair_refine": float(stage[4]),
                    "finish": float(stage[5])}
    else:
        stage_ms = {"group": float(stage[0]), "screen": float(stage[1]), "pair_refine": float(stage[2]),
                    "finish": float(stage[3])}
    flags = outs[3].cpu().numpy().view(np.uint32)

    # the plain MFMA screen on the same batch (its roofline on this workload)
    sopts = mrep.default_opts("bf16", time_stages=True)
    sws = torch.empty(geom.workspace_bytes(n, sopts), dtype=torch.uint8, device=dev)
    souts = outs_like()

    def screen():
        geom.project(q, cid, sopts, workspace=sws, out=souts)

    screen()
    ms_s, st_s = _timed(screen, max(1, min(args.steps, 5)))
    del sws
    screen_block = {
        "value": n / (ms_s / 1e3), "unit": "projections/s", "ms_per_step": ms_s,
        "stage_ms": {"group": float(st_s[0]), "screen": float(st_s[1]), "pair_refine": float(st_s[2]),
                     "finish": float(st_s[3])},
        "screened_samples_per_step": samples,
        "roofline": screen_roofline(samples, float(st_s[1]), ms_s),
    }
    _say("lattice", f"screen {ms_s:.2f} ms per call")

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "projections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": f"lattice struts: {n_curves} random-walk B-splines (degree U{{3..9}}, 64..1024 control "
                        f"points), {n:,} offset queries in proportion to cubic pieces; plain method (autotuned "
                        f"strategy: {strategy}; FP32 refine, FP64 polish)",
            "n_curves": n_curves,
            "queries": int(n),
            "cubic_pieces": n_pieces,
            "tol_rel": 1e-6,
            "strategy": strategy,
            "tune_ms": {"screen": ms_screen, "spheres": ms_spheres},
            "box_schedule": {"lanes_per_query": lanes, "persistent": bool(persistent),
                             "tune_ms": {f"{4 << (k % 3)} lanes, {'persistent' if k >= 3 else 'tile map'}": m
                                         for k, m in enumerate(sched_ms)}},
            "decomposition": dec,
            "stage_ms": stage_ms,
            "candidate_pairs": pairs,
            "fullscan_queries": ovf,
            "wall_s_timed": wall,
            "polished_frac": float(np.mean((flags & mrep.F_POLISHED) != 0)),
            "near_tie_frac": float(np.mean((flags & mrep.F_NEAR_TIE) != 0)),
        },
        "screen": screen_block,
    }
    # the roofline of the call's dominant kernel (largest stage), the others beside it
    coef_bytes = int(np.sum(24 * (np.asarray(curves.degree, np.int64)[qs.curve_id] + 1)))
    roofs = {"k_pairs": pairs_roofline(pairs, stage_ms["pair_refine"]),
             "k_finish": finish_roofline(n, pairs, coef_bytes, stage_ms["finish"])}
    if strat == mrep.STRATEGY_SPHERES:
        roofs["k_box"] = box_roofline(tests, stage_ms["candidates_k_box"])
        result["config"]["sphere_tests"] = tests
    else:
        roofs["k_screen_bf16"] = screen_block["roofline"]
    traffic = _lattice_traffic() if strat == mrep.STRATEGY_SPHERES else {}
    for k, r in roofs.items():
        if k in traffic and r is not None:
            r["traffic"] = traffic[k]
    kernel_ms = {k: (r or {}).get("time_ms", 0.0) for k, r in roofs.items()}
    dominant = max(kernel_ms, key=kernel_ms.get)
    result["roofline"] = roofs.pop(dominant)
    result["rooflines_other_kernels"] = roofs

    # NN-seeded (curve network trained on held-out struts) and sphere-pruned, same queries
    seeded_outs = None
    if not args.no_seeded:
        t0 = time.perf_counter()
        tr_curves = gen.curves_lattice_geometry(15, n_curves=max(64, n_curves // 8))
        tr_plan = mrep.decompose_curves(tr_curves, 1e-6)
        tr_qs = gen.offset_queries(115, tr_curves, per_curve=256)
        tr_geom = tr_plan.upload(dev)
        tr_cid = torch.from_numpy(tr_qs.curve_id).to(dev)
        tr_q = (tr_geom.eval(tr_cid, torch.from_numpy(tr_qs.t0).to(dev)) +
                torch.from_numpy(tr_qs.offset).to(dev)).contiguous()
        x, u, a, tstats = seeding.training_pairs(tr_plan, tr_geom, tr_q, tr_cid, seed=0)
        net = mrep.Network(dev, seed=7)
        t1 = time.perf_counter()
        losses = seeding.train(net, x, u, a, epochs=10, batch=4096, lr=1e-3, seed=0)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t1
        prep_s = t1 - t0
        del x, u, a, tr_geom, tr_plan
        untrained = mrep.Network(dev, seed=7)
        eopts = mrep.default_opts("bf16", time_stages=True)
        ews = torch.empty(geom.seeded_workspace_bytes(n, eopts), dtype=torch.uint8, device=dev)
        diag = torch.from_numpy(curves.bbox_diag()).to(dev)[cid.long()]
        res = {}
        for name, nn in (("nn", net), ("nn_untrained", untrained), ("sphere_pruned", None)):
            so = outs_like()

            def step():
                geom.project_seeded(q, cid, nn, eopts, workspace=ews, out=so)

            for _ in range(max(1, args.warmup)):
                step()
            ms2, st2 = _timed(step, max(1, min(args.steps, 10)))
            f2 = so[3].cpu().numpy().view(np.uint32)
            res[name] = {
                "value": n / (ms2 / 1e3), "unit": "projections/s", "ms_per_step": ms2,
                "vs_plain_value": ms / ms2,
                "stage_ms": {"group": float(st2[0]), "candidates": float(st2[1]), "network": float(st2[2]),
                             "seed_certify": float(st2[3]), "pair_refine": float(st2[4]), "finish": float(st2[5])},
                "fallback_frac": float(np.mean((f2 & mrep.F_NN_FALLBACK) != 0)),
                "vs_plain_max_dist_rel": float(((so[1] - outs[1]).abs() / diag).max().item()),
            }
            if name == "nn":
                seeded_outs = so
                res[name]["roofline_mlp"] = mlp_roofline(4 * n, float(st2[2]))
            _say("lattice", f"seeded {name}: {ms2:.2f} ms per call, fallback {res[name]['fallback_frac']:.3f}")
        del ews
        res["training"] = {"curves": int(tr_curves.n), **tstats, "epochs": 10, "batch": 4096,
                           "steps": int(len(losses)), "loss_first": float(losses[:50].mean()),
                           "loss_last": float(losses[-50:].mean()), "prep_s": prep_s, "train_s": train_s,
                           "ms_per_train_step": 1e3 * train_s / max(1, len(losses))}
        res["nn_speedup_vs_plain"] = res["nn"]["vs_plain_value"]
        res["nn_speedup_vs_sphere_pruned"] = res["sphere_pruned"]["ms_per_step"] / res["nn"]["ms_per_step"]
        result["seeded"] = res

    if not args.no_cpu_baseline:
        result["cpu_baseline"], result["parity_on_sample"] = lattice_cpu_baseline(
            curves, qs, q_host, outs, seeded_outs, souts, args.cpu_seconds)
    return result


def screen_roofline(samples, screen_ms, call_ms):
    """k_screen_bf16 against the dense BF16 MFMA peak.  Method work: one distance per (query, piece, sample) in
    the monomial form, 19 multiply-adds (38 flop); beside it the padded-K figure (one 16x16x32 MFMA output
    element, 64 flop, what the matrix cores execute) and the whole-call fraction."""
    method = samples * FLOPS_PER_SAMPLE_METHOD / (screen_ms / 1e3) / 1e12
    padded = samples * FLOPS_PER_SAMPLE_PADDED / (screen_ms / 1e3) / 1e12
    whole = samples * FLOPS_PER_SAMPLE_METHOD / (call_ms / 1e3) / 1e12
    return {"bound": "mfma", "kernel": "k_screen_bf16", "achieved": method, "peak": BF16_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": method / BF16_PEAK_TFLOPS,
            "per_unit": "38 flop (19 MAC, the monomial-form distance) per screened (query, piece, sample)",
            "frac_padded_k": padded / BF16_PEAK_TFLOPS,
            "per_unit_padded_k": "64 flop per screened sample: one 16x16x32 BF16 MFMA output element (K padded to 32)",
            "frac_whole_call": whole / BF16_PEAK_TFLOPS, "time_ms": screen_ms}


def pairs_roofline(pairs, pair_ms):
    """k_pairs<float> (the refine of every listed (query, piece) pair) against the FP32 vector peak: per pair the
    certified piece minimum, 32 sampled distances of 12 FP32 multiply-adds each (cubic in Horner form per
    coordinate, squared norm), 768 flop; the Newton steps that follow are not counted."""
    achieved = pairs * FLOPS_PER_PAIR / (pair_ms / 1e3) / 1e12 if pair_ms > 0 else None
    return {"bound": "alu", "kernel": "k_pairs<float>", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS if achieved else None,
            "traffic": None, "units": int(pairs), "time_ms": pair_ms,
            "per_unit": "768 flop per listed (query, piece) pair: 32 samples x 12 FP32 FMA"}


def box_roofline(tests, box_ms):
    """k_box (sphere lists) against the FP32 vector peak: per sphere test |q - c| - r against a bound, 10 flop
    (3 sub, 3 mul, 2 add, sqrt, sub); the tests are counted by the kernel (mrep_workspace_counts)."""
    achieved = tests * FLOPS_PER_SPHERE_TEST / (box_ms / 1e3) / 1e12 if box_ms > 0 else None
    return {"bound": "alu", "kernel": "k_box", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS if achieved else None,
            "traffic": None, "units": int(tests), "time_ms": box_ms,
            "per_unit": "10 flop per sphere test |q - c| - r against a bound (cluster and piece spheres)"}


def finish_roofline(n, pairs, coef_bytes, finish_ms):
    """k_finish (top-2 of each query's pair records, FP64 polish on the exact span, write) against HBM: per
    query 4 index words, the query, the polished span's (p+1) x 3 FP64 coefficients, its interval and piece
    bounds, and the 24-byte result; per pair its 32-byte record and 4-byte piece index."""
    byts = n * (16 + 24 + 16 + 4 + 16 + 24) + pairs * 36 + coef_bytes
    achieved = byts / (finish_ms / 1e3) / 1e9 if finish_ms > 0 else None
    return {"bound": "hbm", "kernel": "k_finish", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS if achieved else None, "traffic": None, "units": int(n),
            "algorithmic_bytes": int(byts), "time_ms": finish_ms,
            "per_unit": "100 B per query + 36 B per pair + 24 (p+1) B of span coefficients per query"}


def mlp_roofline(rows, ms):
    """k_mlp against the dense BF16 MFMA peak: 2 x (15x128 + 128x128 + 128x2) = 37,120 flop per curve row."""
    if not ms > 0:
        return None
    a = rows * MLP_CURVE_FLOPS / (ms / 1e3) / 1e12
    return {"bound": "mfma", "kernel": "k_mlp", "achieved": a, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": a / BF16_PEAK_TFLOPS, "rows": int(rows), "per_unit": "37,120 flop per (query, candidate) row"}


def lattice_cpu_baseline(curves, qs, q_all, outs, seeded_outs, screen_outs, seconds):
    """The FP64 oracle on a bounded random sample of the headline queries (its throughput on this host), and
    the parity of the benchmarked outputs (plain, seeded, screen) on that sample."""
    sys.path.insert(0, ROOT)
    import oracle

    oracle.build(force=False)
    rng = np.random.default_rng(7)
    n = qs.n
    order = rng.permutation(n)
    pilot = np.sort(order[:256])
    t0 = time.perf_counter()
    oracle.project(curves, qs.curve_id[pilot], q_all[pilot])
    rate = 256 / max(time.perf_counter() - t0, 1e-6)
    m = int(min(max(rate * seconds, 1024), 100_000))
    idx = np.sort(order[:m])
    t0 = time.perf_counter()
    r = oracle.project(curves, qs.curve_id[idx], q_all[idx])
    dt = time.perf_counter() - t0
    diag = curves.bbox_diag()[qs.curve_id[idx]]
    unique = (r["runner"] - r["dist"]) > 2e-6 * diag
    wc = unique & (r["kappa"] >= 1e-3)

    def parity(o):
        d = o[1].cpu().numpy()[idx]
        t = o[0].cpu().numpy()[idx]
        err = np.abs(d - r["dist"]) / diag
        terr = np.abs(t - r["t"])[wc]
        return {"max_dist_err_rel_bbox": float(err.max()), "max_t_err_unique_wellcond": float(terr.max()) if wc.any() else None,
                "pass": bool(err.max() <= 1e-6 and (not wc.any() or terr.max() <= 1e-7))}

    par = {"queries": int(m), "unique_wellcond_frac": float(wc.mean()), "plain": parity(outs),
           "screen": parity(screen_outs)}
    if seeded_outs is not None:
        par["nn_seeded"] = parity(seeded_outs)
    cpu = {"value": m / dt, "unit": "projections/s", "cores": oracle.max_threads(), "kind": "oracle",
           "sample": f"{m} of the {n} headline queries (uniform random, seed 7): certified FP64 projection on the "
                     f"original B-splines, {dt:.1f} s"}
    return cpu, par


def batched_curves_block(args, dev):
    """Batched curves: 4,096 clamped B-splines (degree U{2..7}, 8..256 control points, 10% doubled knots), 1,048,576
    offset queries (256 per curve).  One call = BF16 MFMA screen, FP32 Newton, FP64 polish."""
    import torch

    from paper_2504_11498_amd import gen, mrep

    curves, qs = gen.curves_batched(2)
    t0 = time.perf_counter()
    plan = mrep.decompose_curves(curves, 1e-6)
    decompose_s = time.perf_counter() - t0
    geom = plan.upload(dev)
    seg_counts = np.diff(plan.seg_off())
    cid = torch.from_numpy(qs.curve_id).to(dev)
    q_host = host_points(curves, qs)
    q = torch.from_numpy(q_host).to(dev)
    n = qs.n
    opts = mrep.default_opts("bf16", time_stages=True)
    outs = (torch.empty(n, dtype=torch.float64, device=dev), torch.empty(n, dtype=torch.float64, device=dev),
            torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev))
    ws = torch.empty(geom.workspace_bytes(n, opts), dtype=torch.uint8, device=dev)

    def step():
        geom.project(q, cid, opts, workspace=ws, out=outs)

    for _ in range(args.warmup):
        step()
    ms, stage = _timed(step, args.steps)
    samples = 32 * int(np.sum(seg_counts[qs.curve_id].astype(np.int64)))
    flags = outs[3].cpu().numpy().view(np.uint32)
    ovf, pairs = geom.workspace_counts(ws)
    roof = screen_roofline(samples, float(stage[1]), ms)
    roof["traffic"] = _traffic()
    res = {
        "workload": "batched curves: 4096 clamped B-splines, degree U{2..7}, 8-256 control points, 1,048,576 "
                    "offset queries; plain method (BF16 MFMA screen, FP32 Newton, FP64 polish)",
        "value": n / (ms / 1e3), "unit": "projections/s", "ms_per_step": ms, "queries": int(n),
        "cubic_pieces": int(plan.n_segments), "decompose_s_host": decompose_s,
        "screened_samples_per_step": samples, "candidate_pairs": pairs, "fullscan_queries": ovf,
        "stage_ms": {"group": float(stage[0]), "screen": float(stage[1]), "pair_refine": float(stage[2]),
                     "finish": float(stage[3])},
        "polished_frac": float(np.mean((flags & mrep.F_POLISHED) != 0)),
        "roofline": roof,
        "roofline_pairs": pairs_roofline(pairs, float(stage[2])),
    }
    _say("batched", f"{ms:.3f} ms per call")
    if not args.no_extras:
        strat, ms_screen, ms_spheres, _ = geom.tune(q, cid, out=tuple(torch.empty_like(o) for o in outs))
        res["autotune"] = {"strategy": ["screen", "spheres"][strat], "ms": {"screen": ms_screen, "spheres": ms_spheres}}
        res["graph_small_batches"] = graph_small_batches(geom, q, cid)
        res["precision_tiers"] = precision_tiers(geom, q, cid, outs, curves, qs)
    if not args.no_clip:
        res["clip_refiner"] = clip_refiner(geom, q, cid, outs, curves, res["value"], stage, ws, args)
    if not args.no_seeded:
        res["seeded"] = seeded_variants(geom, q, cid, outs, curves, res["value"], args)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(curves, qs, q_host, outs, min(args.cpu_seconds, 8.0))
    return res


def precision_tiers(geom, q, cid, bf_outs, curves, qs):
    """The same batch in the FP32 and FP64 tiers (every piece examined in that precision, FP64 polish): time
    per call and the largest differences from the BF16 screen's answers."""
    import torch

    from paper_2504_11498_amd import mrep

    n = q.shape[0]
    diag = torch.from_numpy(curves.bbox_diag()).to(q.device)[cid.long()]
    res = {}
    for name in ("fp32", "fp64"):
        opts = mrep.default_opts(name)
        ws = torch.empty(geom.workspace_bytes(n, opts), dtype=torch.uint8, device=q.device)
        outs = tuple(torch.empty_like(o) for o in bf_outs)

        def step():
            geom.project(q, cid, opts, workspace=ws, out=outs)

        step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        res[name] = {"ms_per_call": ms, "value": n / (ms / 1e3),
                     "vs_bf16_max_dist_rel": float(((outs[1] - bf_outs[1]).abs() / diag).max().item()),
                     "vs_bf16_same_piece_frac": float((outs[2] == bf_outs[2]).double().mean().item())}
        _say("batched", f"{name} tier {ms:.2f} ms per call")
    return res


def single_cubic_block(args, dev):
    """One cubic curve (16 control points, 13 spans), 10,000 queries uniform in its box x1.1: far too small to
    fill the GPU, so its absolute latency per call (median of 10 after 3 warm-ups), FP64 and BF16 modes."""
    import torch

    from paper_2504_11498_amd import gen, mrep

    curves, qs = gen.curve_single(1)
    geom = mrep.decompose_curves(curves, 1e-6).upload(dev)
    q = torch.from_numpy(qs.point).to(dev)
    cid = torch.from_numpy(qs.curve_id).to(dev)
    res = {"workload": "single cubic: 16 control points, 13 spans, 10,000 box queries", "queries": int(qs.n)}
    for prec in ("fp64", "bf16"):
        opts = mrep.default_opts(prec)
        outs = (torch.empty(qs.n, dtype=torch.float64, device=dev), torch.empty(qs.n, dtype=torch.float64, device=dev),
                torch.empty(qs.n, dtype=torch.int32, device=dev), torch.empty(qs.n, dtype=torch.int32, device=dev))
        ws = torch.empty(geom.workspace_bytes(qs.n, opts), dtype=torch.uint8, device=dev)
        for _ in range(3):
            geom.project(q, cid, opts, workspace=ws, out=outs)
        times = []
        for _ in range(10):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            geom.project(q, cid, opts, workspace=ws, out=outs)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        res[prec] = {"latency_ms_median": float(np.median(times)), "latency_ms_min": float(np.min(times))}
    return res


def _timed(fn, steps):
    import torch

    from paper_2504_11498_amd import mrep

    stage = None
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
        st = mrep.last_stage_times()
        stage = st if stage is None else stage + st
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, stage / steps


def graph_small_batches(geom, q, cid, batch: int = 4096, calls: int = 200):
    """Small batches are launch-bound: per-call time of `calls` projections of `batch` queries, eager and as
    replays of one captured HIP graph (new queries copied into its input buffer before each replay)."""
    import torch

    from paper_2504_11498_amd import mrep

    dev = q.device
    opts = mrep.default_opts("bf16")
    qb, cb = q[:batch].clone(), cid[:batch].clone()
    ws = torch.empty(geom.workspace_bytes(batch, opts), dtype=torch.uint8, device=dev)
    outs = (torch.empty(batch, dtype=torch.float64, device=dev), torch.empty(batch, dtype=torch.float64, device=dev),
            torch.empty(batch, dtype=torch.int32, device=dev), torch.empty(batch, dtype=torch.int32, device=dev))
    src = [(q[i * batch:(i + 1) * batch], cid[i * batch:(i + 1) * batch]) for i in range(8)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        geom.project(qb, cb, opts, workspace=ws, out=outs)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        geom.project(qb, cb, opts, workspace=ws, out=outs)

    def eager():
        for i in range(calls):
            qi, ci = src[i % 8]
            qb.copy_(qi)
            cb.copy_(ci)
            geom.project(qb, cb, opts, workspace=ws, out=outs)

    def replay():
        for i in range(calls):
            qi, ci = src[i % 8]
            qb.copy_(qi)
            cb.copy_(ci)
            g.replay()

    res = {"batch": batch, "calls": calls}
    for name, fn in (("eager", eager), ("graph", replay)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        res[name + "_us_per_call"] = (time.perf_counter() - t0) / calls * 1e6
    res["graph_projections_per_s"] = batch / (res["graph_us_per_call"] / 1e6)
    return res


def clip_refiner(geom, q, cid, plain_outs, curves, plain_value, plain_stage, ws, args):
    """The same batch with the paper's refinement path on every candidate pair (Ferrari split of E', elimination,
    rebasement, Bezier clipping; MREP_OPT_CLIP) in place of the sampled minimum + Newton; compared with the plain
    method's answers."""
    import torch

    from paper_2504_11498_amd import mrep

    n = q.shape[0]
    opts = mrep.default_opts("bf16", time_stages=True, clip=True)
    outs = tuple(torch.empty_like(o) for o in plain_outs)

    def step():
        geom.project(q, cid, opts, workspace=ws, out=outs)

    for _ in range(args.warmup):
        step()
    ms, stage = _timed(step, args.steps)
    diag = torch.from_numpy(curves.bbox_diag()).to(q.device)[cid.long()]
    dd = ((outs[1] - plain_outs[1]).abs() / diag).max().item()
    dt = (outs[0] - plain_outs[0]).abs()
    # the monotonic split alone (roots of E'), Ferrari against Newton's iteration, on every query paired with the
    # piece holding its projection (the paper's comparison of the analytic and the numerical root finders)
    piece = plain_outs[2]
    split = {}
    for name, method in (("ferrari", mrep.ROOTS_FERRARI), ("newton", mrep.ROOTS_NEWTON)):
        for _ in range(args.warmup):
            geom.monotonic_split(cid, piece, q, method)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            roots, count = geom.monotonic_split(cid, piece, q, method)
        e1.record()
        torch.cuda.synchronize()
        split[name] = {"us_per_call": e0.elapsed_time(e1) * 1e3 / args.steps,
                       "mean_roots": float(count.float().mean().item())}
    split["pairs"] = int(n)
    split["newton_over_ferrari"] = split["newton"]["us_per_call"] / split["ferrari"]["us_per_call"]
    return {
        "monotonic_split": split,
        "value": n / (ms / 1e3),
        "ms_per_step": ms,
        "vs_plain_value": (n / (ms / 1e3)) / plain_value,
        "stage_ms": {"group": float(stage[0]), "screen": float(stage[1]), "pair_refine": float(stage[2]),
                     "finish": float(stage[3])},
        "plain_pair_refine_ms": float(plain_stage[2]),
        "vs_plain_max_dist_rel": dd,
        "vs_plain_t_over_1e-7": int((dt > 1e-7).sum().item()),
    }


def span_decomposition(curves, args, dev):
    """The exact Bezier form of every knot interval on the device (mrep_span_bezier_curves), for the batched curves
    and for 65,536 lattice struts.  Algorithmic bytes per launch: every control point, knot and per-curve offset
    read once, every Bezier point and interval end written once."""
    import torch

    from paper_2504_11498_amd import gen, mrep

    out = {}
    traffic = _span_traffic()
    for name, make in (("batched_curves", lambda: curves),
                       ("lattice_struts_65536", lambda: gen.curves_lattice_geometry(5, n_curves=65_536))):
        cv = make()
        dc = mrep.DeviceCurves(cv, dev)
        bz, t = dc.span_bezier()
        for _ in range(args.warmup):
            dc.span_bezier(bz, t)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            dc.span_bezier(bz, t)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / args.steps
        n_c = cv.n
        alg = (cv.cp.size * 8 + cv.knots.size * 8 + n_c * 4 + 4 * (n_c + 1) * 8 +
               dc.n_points * 24 + dc.n_intervals * 16)
        out[name] = {"curves": int(n_c), "intervals": dc.n_intervals, "bezier_points": dc.n_points,
                     "us_per_launch": us, "intervals_per_s": dc.n_intervals / (us * 1e-6),
                     "algorithmic_bytes": int(alg), "achieved_GBps": alg / (us * 1e-6) / 1e9,
                     "hbm_frac": alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBPS, "traffic": traffic.get(name)}
        print(f"[bench] span decomposition {name}: {us:.1f} us", file=sys.stderr, flush=True)
        del dc, bz, t
        torch.cuda.empty_cache()
    return out


def seeded_variants(geom, q, cid, plain_outs, curves, plain_value, args):
    """Learned seeding: train on held-out curves, then time the seeded and the sphere-pruned projection
    of the same queries; both are compared with the plain method's answers."""
    import torch

    from paper_2504_11498_amd import gen, mrep, seeding

    dev = q.device
    t0 = time.perf_counter()
    tr_curves = gen.curves_batched_geometry(12, n_curves=1024)
    tr_qs = gen.offset_queries(112, tr_curves, per_curve=1000)
    tr_plan = mrep.decompose_curves(tr_curves, 1e-6)
    tr_geom = tr_plan.upload(dev)
    tr_cid = torch.from_numpy(tr_qs.curve_id).to(dev)
    tr_q = (tr_geom.eval(tr_cid, torch.from_numpy(tr_qs.t0).to(dev)) + torch.from_numpy(tr_qs.offset).to(dev)).contiguous()
    x, u, a, stats = seeding.training_pairs(tr_plan, tr_geom, tr_q, tr_cid, seed=0)
    prep_s = time.perf_counter() - t0
    net = mrep.Network(dev, seed=7)
    t0 = time.perf_counter()
    losses = seeding.train(net, x, u, a, epochs=10, batch=4096, lr=1e-3, seed=0)
    train_s = time.perf_counter() - t0
    del x, u, a, tr_geom

    n = q.shape[0]
    opts = mrep.default_opts("bf16", time_stages=True)
    outs = tuple(torch.empty_like(o) for o in plain_outs)
    ws = torch.empty(geom.seeded_workspace_bytes(n, opts), dtype=torch.uint8, device=dev)
    res = {}
    for name, nn in (("nn", net), ("sphere_pruned", None)):
        def step():
            geom.project_seeded(q, cid, nn, opts, workspace=ws, out=outs)

        for _ in range(args.warmup):
            step()
        ms, stage = _timed(step, args.steps)
        flags = outs[3].cpu().numpy().view(np.uint32)
        diag = torch.from_numpy(curves.bbox_diag()).to(dev)[cid.long()]
        dd = ((outs[1] - plain_outs[1]).abs() / diag).max().item()
        dt = (outs[0] - plain_outs[0]).abs()
        res[name] = {
            "value": n / (ms / 1e3),
            "ms_per_step": ms,
            "speedup_vs_plain": (n / (ms / 1e3)) / plain_value,
            "stage_ms": {"group": float(stage[0]), "candidates": float(stage[1]), "network": float(stage[2]),
                         "seed_certify": float(stage[3]), "pair_refine": float(stage[4]), "finish": float(stage[5])},
            "fallback_frac": float(np.mean((flags & mrep.F_NN_FALLBACK) != 0)),
            "vs_plain_max_dist_rel": dd,
            "vs_plain_t_over_1e-7": int((dt > 1e-7).sum().item()),
        }
    res["training"] = {"geometry": "1024 held-out curves (seed 12), 1000 offset queries each (seed 112)",
                       **stats, "epochs": 10, "batch": 4096, "lr": 1e-3, "steps": int(len(losses)),
                       "loss_first": float(losses[:50].mean()), "loss_last": float(losses[-50:].mean()),
                       "prep_s": prep_s, "train_s": train_s}
    return res


def surfaces_bench(args, dev):
    """Batched surfaces: 256 tensor-product B-spline height fields (bicubic and quintic, 32 x 32 nets),
    16,384 queries each (half on the surface, half offset by N(0, (0.05 diag)^2)), decomposed into bicubic
    patches at 1e-6 of the net's box diagonal.  A step = one mrep_project_surfaces call on all 4,194,304."""
    import torch

    from paper_2504_11498_amd import gen, mrep

    S, Q = gen.surfaces(3)
    t0 = time.perf_counter()
    plan = mrep.decompose_surfaces(S, 1e-6)
    decompose_s = time.perf_counter() - t0
    geom = plan.upload(dev)
    sid = torch.from_numpy(Q["surface_id"]).to(dev)
    q_host = host_surface_points(S, Q)
    q = torch.from_numpy(q_host).to(dev)
    n = q.shape[0]
    opts = mrep.default_opts(time_stages=True)
    outs = (torch.empty((n, 2), dtype=torch.float64, device=dev), torch.empty(n, dtype=torch.float64, device=dev),
            torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev))
    ws = torch.empty(geom.surface_workspace_bytes(n, opts), dtype=torch.uint8, device=dev)

    def step():
        geom.project_surfaces(q, sid, opts, workspace=ws, out=outs)

    for _ in range(max(1, args.warmup)):
        step()
    steps = max(1, min(args.steps, 5))
    ms, stage = _timed(step, steps)
    flags = outs[3].cpu().numpy().view(np.uint32)
    res = {
        "workload": "batched surfaces: 256 B-spline height fields (degree 3x3 and 5x5, 32x32 nets), "
                    "4,194,304 queries (half on the surface)",
        "value": n / (ms / 1e3),
        "unit": "projections/s",
        "ms_per_step": ms,
        "steps": steps,
        "queries": int(n),
        "patches": int(plan.n_segments),
        "decompose_s_host": decompose_s,
        "stage_ms": {"group_spheres": float(stage[0]), "patch_minima": float(stage[1]),
                     "polish_write": float(stage[2])},
        "fullscan_frac": float(np.mean((flags & mrep.F_FULLSCAN) != 0)),
    }
    seeded_outs = None
    if not args.no_seeded:
        from paper_2504_11498_amd import seeding

        # the surface network, trained outside the timed region on about 2M pairs from 64 held-out surfaces
        # (other seeds), labels from the library's certified projection
        S2, Q2 = gen.surfaces(31, n_surf=64, per_surface=19_500)
        plan2 = mrep.decompose_surfaces(S2, 1e-6)
        geom2 = plan2.upload(dev)
        sid2 = torch.from_numpy(Q2["surface_id"]).to(dev)
        q2 = (geom2.eval_surfaces(sid2, torch.from_numpy(Q2["uv0"]).to(dev))
              + torch.from_numpy(Q2["offset"]).to(dev)).contiguous()
        t0 = time.perf_counter()
        x, tgt, acc, tstats = seeding.surface_training_pairs(plan2, geom2, q2, sid2, seed=0)
        net = mrep.Network(dev, seed=7, kind=mrep.NN_SURFACE)
        losses = seeding.train(net, x, tgt, acc, epochs=4, batch=4096, lr=1e-3, seed=0)
        train_s = time.perf_counter() - t0
        seeded_outs = tuple(torch.empty_like(o) for o in outs)
        ws2 = torch.empty(geom.surface_seeded_workspace_bytes(n, opts), dtype=torch.uint8, device=dev)

        def sstep():
            geom.project_surfaces_seeded(q, sid, net, opts, workspace=ws2, out=seeded_outs)

        for _ in range(max(1, args.warmup)):
            sstep()
        ms2, stage2 = _timed(sstep, steps)
        f2 = seeded_outs[3].cpu().numpy().view(np.uint32)
        res["seeded"] = {
            "value": n / (ms2 / 1e3),
            "unit": "projections/s",
            "ms_per_step": ms2,
            "stage_ms": {"group_spheres_candidates": float(stage2[0]), "network": float(stage2[1]),
                         "seed_patch_minima": float(stage2[2]), "polish_write": float(stage2[3])},
            "nn_fallback_frac": float(np.mean((f2 & mrep.F_NN_FALLBACK) != 0)),
            "fullscan_frac": float(np.mean((f2 & mrep.F_FULLSCAN) != 0)),
            "training": {"surfaces": 64, "queries": int(q2.shape[0]), **tstats, "steps": int(len(losses)),
                         "loss_first": float(losses[:20].mean()), "loss_last": float(losses[-20:].mean()),
                         "seconds": train_s},
        }
    if not args.no_cpu_baseline:
        sys.path.insert(0, ROOT)
        import oracle

        oracle.build(force=False)
        rng = np.random.default_rng(8)
        pick = np.sort(rng.choice(n, 2000, replace=False))
        qs = q_host[pick]
        t0 = time.perf_counter()
        r = oracle.surf_project(S, Q["surface_id"][pick], qs)
        dt = time.perf_counter() - t0
        diag = np.array([np.linalg.norm(S.cp[S.cp_off[k]:S.cp_off[k + 1]].max(0) - S.cp[S.cp_off[k]:S.cp_off[k + 1]].min(0))
                         for k in range(S.n)])[Q["surface_id"][pick]]
        d_g = outs[1].cpu().numpy()[pick]
        uv_g = outs[0].cpu().numpy()[pick]
        unique = (r["runner"] - r["dist"]) > 2e-6 * diag
        wc = unique & (r["kappa"] >= 1e-3)
        res["cpu_baseline"] = {"value": 2000 / dt, "unit": "projections/s", "cores": oracle.max_threads(),
                               "kind": "oracle", "sample": "2000 random queries of the same workload"}
        res["parity_on_sample"] = {"max_dist_rel": float(np.max(np.abs(d_g - r["dist"]) / diag)),
                                   "max_uv_err_unique": float(np.max(np.abs(uv_g - r["uv"]).max(1)[wc])) if wc.any() else 0.0}
        if seeded_outs is not None:
            d2 = seeded_outs[1].cpu().numpy()[pick]
            uv2 = seeded_outs[0].cpu().numpy()[pick]
            res["seeded"]["parity_on_sample"] = {
                "max_dist_rel": float(np.max(np.abs(d2 - r["dist"]) / diag)),
                "max_uv_err_unique": float(np.max(np.abs(uv2 - r["uv"]).max(1)[wc])) if wc.any() else 0.0}
    return res


def cpu_baseline(curves, qs, q_all, outs, seconds):
    """The FP64 oracle timed on this host on a bounded random sample of the same queries."""
    sys.path.insert(0, ROOT)
    import oracle

    oracle.build(force=False)
    rng = np.random.default_rng(7)
    order = rng.permutation(qs.n)

    def run(idx):
        t0 = time.perf_counter()
        r = oracle.project(curves, qs.curve_id[idx], q_all[idx])
        return r, time.perf_counter() - t0

    pilot = np.sort(order[:1024])
    _, dt = run(pilot)
    rate = 1024 / max(dt, 1e-6)
    m = int(min(max(rate * seconds, 2048), 200_000))
    idx = np.sort(order[:m])
    r, dt = run(idx)
    # parity of the benchmarked GPU outputs on the same sample
    t_g = outs[0].cpu().numpy()[idx]
    d_g = outs[1].cpu().numpy()[idx]
    diag = curves.bbox_diag()[qs.curve_id[idx]]
    unique = (r["runner"] - r["dist"]) > 2e-6 * diag
    wc = unique & (r["kappa"] >= 1e-3)
    return {
        "value": m / dt,
        "unit": "projections/s",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "sample": f"{m} of the {qs.n} benchmark queries (uniform random, seed 7), certified FP64 projection "
                  f"on the original B-splines, {dt:.1f} s",
        "parity_on_sample": {
            "max_dist_err_rel_bbox": float(np.max(np.abs(d_g - r["dist"]) / diag)),
            "max_t_err_unique_wellcond": float(np.max(np.abs(t_g[wc] - r["t"][wc]))) if wc.any() else None,
            "unique_wellcond_frac": float(wc.mean()),
        },
    }


if __name__ == "__main__":
    main()
