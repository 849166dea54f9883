"""Shared helpers for GPU-vs-oracle parity checks (test infrastructure).

Parity bar (from the method's accuracy target):
  - distance within 1e-6 * box diagonal of the curve, never below the oracle's
    global minimum by more than rounding;
  - parameter within 1e-7 where the oracle's minimum is unique (runner-up local
    minimum farther than 2e-6 * diag) and well conditioned (kappa >= 1e-3);
  - piece index identical where unique and the oracle's t* is not within 1e-7
    of a piece boundary of the oracle's own decomposition.
"""
import numpy as np

import oracle

DIST_REL = 1e-6
T_ABS = 1e-7
UNIQUE_REL = 2e-6
KAPPA_MIN = 1e-3


def oracle_pieces(curves, tol_rel):
    ref = oracle.decompose(curves, tol_rel * curves.bbox_diag())
    off = np.zeros(curves.n + 1, np.int64)
    off[1:] = np.cumsum(ref["counts"])
    return ref, off


def oracle_seg_index(ref, off, cid, t):
    seg = np.zeros(t.shape[0], np.int64)
    near = np.zeros(t.shape[0], bool)
    for i in range(t.shape[0]):
        c = cid[i]
        ta = ref["tab"][off[c] : off[c + 1], 0]
        tb = ref["tab"][off[c] : off[c + 1], 1]
        k = int(np.searchsorted(ta, t[i], side="right") - 1)
        k = min(max(k, 0), ta.shape[0] - 1)
        seg[i] = k
        bps = np.concatenate([ta[1:], tb[:-1]])
        near[i] = bps.size > 0 and np.min(np.abs(bps - t[i])) <= T_ABS
    return seg, near


def compare(curves, cid, q, gpu, ref_proj, ref_dec=None, tol_rel=1e-6, label=""):
    """gpu: dict of numpy t, dist, seg, flags.  Returns a dict of stats; asserts the bar."""
    diag = curves.bbox_diag()[cid]
    d_ref, t_ref = ref_proj["dist"], ref_proj["t"]
    err_d = np.abs(gpu["dist"] - d_ref) / diag
    below = (d_ref - gpu["dist"]) / diag
    unique = (ref_proj["runner"] - d_ref) > UNIQUE_REL * diag
    wc = unique & (ref_proj["kappa"] >= KAPPA_MIN)
    err_t = np.abs(gpu["t"] - t_ref)
    stats = {"n": int(cid.shape[0]), "max_dist_rel": float(err_d.max()), "max_t_err_wc": float(err_t[wc].max()) if wc.any() else 0.0,
             "unique_frac": float(unique.mean()), "wc_frac": float(wc.mean())}
    bad_d = np.nonzero(err_d > DIST_REL)[0]
    assert bad_d.size == 0, f"{label}: {bad_d.size} distances off, worst {err_d.max():.3e} at {bad_d[:5]}"
    assert below.max() <= 1e-12, f"{label}: GPU distance below the global minimum by {below.max():.3e}"
    bad_t = np.nonzero(wc & (err_t > T_ABS))[0]
    assert bad_t.size == 0, f"{label}: {bad_t.size} parameters off, worst {err_t[wc].max():.3e} at {bad_t[:5]}"
    if ref_dec is not None:
        ref, off = ref_dec
        seg_ref, near = oracle_seg_index(ref, off, cid, t_ref)
        chk = unique & ~near
        bad_s = np.nonzero(chk & (gpu["seg"] != seg_ref))[0]
        stats["seg_checked"] = int(chk.sum())
        assert bad_s.size == 0, f"{label}: {bad_s.size} piece indices differ, e.g. {bad_s[:5]}"
    return stats


# --------------------------------------------------------------------------- surfaces
def surf_diag(S):
    return np.array([np.linalg.norm(S.cp[S.cp_off[k]:S.cp_off[k + 1]].max(0) - S.cp[S.cp_off[k]:S.cp_off[k + 1]].min(0))
                     for k in range(S.n)])


def compare_surf(S, sid, q, out, ref, ex=None, label=""):
    """Parity bar: distance within 1e-6 * diag and never below the oracle; (u, v) within 1e-7 where the
    oracle's minimum is unique and well conditioned; the patch index equals the exported patch holding the
    oracle's (u, v) where unique and not within 1e-7 of a patch side."""
    diag = surf_diag(S)[sid]
    err = np.abs(out["dist"] - ref["dist"]) / diag
    below = (ref["dist"] - out["dist"]) / diag
    unique = (ref["runner"] - ref["dist"]) > UNIQUE_REL * diag
    wc = unique & (ref["kappa"] >= KAPPA_MIN)
    duv = np.abs(out["uv"] - ref["uv"]).max(1)
    st = {"n": int(len(sid)), "max_dist_rel": float(err.max()), "max_uv_err_wc": float(duv[wc].max()) if wc.any() else 0.0,
          "wc_frac": float(wc.mean())}
    bad = np.nonzero(err > DIST_REL)[0]
    assert bad.size == 0, f"{label}: {bad.size} distances off, worst {err.max():.3e} at {bad[:5]}"
    assert below.max() <= 1e-12, f"{label}: below the oracle by {below.max():.3e}"
    bad = np.nonzero(wc & (duv > T_ABS))[0]
    if bad.size:
        for i in bad[:6]:
            print(f"  q{i} gpu uv={out['uv'][i]} d={out['dist'][i]:.15g} f={out['flags'][i]:#x} | oracle uv={ref['uv'][i]} "
                  f"d={ref['dist'][i]:.15g} kappa={ref['kappa'][i]:.3g} runner={ref['runner'][i]:.6g}", flush=True)
    assert bad.size == 0, f"{label}: {bad.size} (u,v) off, worst {duv[wc].max():.3e} at {bad[:5]}"
    if ex is not None:
        checked = 0
        for i in np.nonzero(unique)[0]:
            o0, o1 = ex["patch_off"][sid[i]], ex["patch_off"][sid[i] + 1]
            r = ex["patch_uv"][o0:o1]
            u, v = ref["uv"][i]
            inside = (r[:, 0] <= u) & (u <= r[:, 1]) & (r[:, 2] <= v) & (v <= r[:, 3])
            near = np.min(np.abs(np.concatenate([r[inside, 0] - u, r[inside, 1] - u, r[inside, 2] - v,
                                                 r[inside, 3] - v]))) if inside.any() else 0.0
            if near <= 1e-7:
                continue
            k = int(np.nonzero(inside)[0][0])
            assert out["patch"][i] == k, f"{label}: query {i} patch {out['patch'][i]} != {k}"
            checked += 1
        st["patch_checked"] = checked
    return st
