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


# the reported distance must be realised by the reported parameter: |C(t) - q|
# (the oracle's de Boor evaluation) within this of dist, relative to the diagonal
REAL_REL = 1e-12
# flag bands (the oracle's runner-up gap and kappa; between the bands either answer is right)
TIE_SET, TIE_CLEAR = 1e-6, 4e-6
ILL_SET, ILL_CLEAR = 3e-3, 3e-2
F_NEAR_TIE, F_ILL_COND = 0x2, 0x4


def check_flags(gpu, ref_proj, diag, label=""):
    """NEAR_TIE set where the oracle's runner-up is within TIE_SET * diag of the minimum and clear where it
    is beyond TIE_CLEAR * diag; where unique, ILL_COND set where the oracle's kappa < ILL_SET and clear where
    kappa > ILL_CLEAR (interior stationary minima: the oracle reports kappa = 1 at ends and corners)."""
    gap = (ref_proj["runner"] - ref_proj["dist"]) / diag
    tie_flag = (gpu["flags"] & F_NEAR_TIE) != 0
    ill_flag = (gpu["flags"] & F_ILL_COND) != 0
    must_tie, must_not = gap <= TIE_SET, gap > TIE_CLEAR
    bad = np.nonzero((must_tie & ~tie_flag) | (must_not & tie_flag))[0]
    st = {"ties": int(must_tie.sum()), "unique": int(must_not.sum()), "near_tie_set": int(tie_flag.sum())}
    tkey = "t" if "t" in gpu else "uv"
    for i in bad[:6]:
        print(f"  q{i} gpu {tkey}={gpu[tkey][i]} d={gpu['dist'][i]:.15g} flags={int(gpu['flags'][i]):#x} | oracle "
              f"{tkey}={ref_proj[tkey][i]} d={ref_proj['dist'][i]:.15g} runner={ref_proj['runner'][i]:.15g} "
              f"kappa={ref_proj['kappa'][i]:.4g}", flush=True)
    assert bad.size == 0, (f"{label}: NEAR_TIE disagrees with the oracle on {bad.size} queries, e.g. {bad[:5]} "
                           f"gap {gap[bad[:5]]} flag {tie_flag[bad[:5]]}")
    kap = ref_proj["kappa"]
    ill, well = must_not & (kap < ILL_SET), must_not & (kap > ILL_CLEAR)
    bad = np.nonzero((ill & ~ill_flag) | (well & ill_flag))[0]
    st["ill"] = int(ill.sum())
    assert bad.size == 0, (f"{label}: ILL_COND disagrees with the oracle on {bad.size} queries, e.g. {bad[:5]} "
                           f"kappa {kap[bad[:5]]} flag {ill_flag[bad[:5]]}")
    return st


def compare(curves, cid, q, gpu, ref_proj, ref_dec=None, tol_rel=1e-6, label="", flags=False):
    """gpu: dict of numpy t, dist, seg, flags.  Returns a dict of stats; asserts the bar.

    Every query: distance parity; the distance realised by the returned parameter on the exact curve
    (oracle evaluation, rational when the curve set has weights); the returned piece holds the returned
    parameter (with ref_dec: (dict with "tab", offsets) -- the oracle's decomposition, or the library's exported
    pieces for rational curves, whose pieces the oracle validates instead of reproducing).  flags: the
    NEAR_TIE / ILL_COND bits against the oracle's runner-up and kappa (check_flags)."""
    diag = curves.bbox_diag()[cid]
    if getattr(curves, "weights", None) is not None:
        X = oracle.nurbs_eval_batch(curves, curves.weights, cid, gpu["t"])
    else:
        X = oracle.eval_batch(curves, cid, gpu["t"])
    real = np.abs(np.linalg.norm(X - q, axis=1) - gpu["dist"]) / diag
    bad_r = np.nonzero(~(real <= REAL_REL))[0]
    assert bad_r.size == 0, (f"{label}: {bad_r.size} distances not realised by their parameter, worst "
                             f"{np.nanmax(real):.3e} at {bad_r[:5]}")
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
    stats["max_realised_rel"] = float(real.max()) if real.size else 0.0
    if flags:
        stats.update(check_flags(gpu, ref_proj, diag, label))
    if ref_dec is not None:
        ref, off = ref_dec
        # the returned piece holds the returned parameter (the oracle's pieces have the library's breakpoints)
        g = off[cid] + gpu["seg"]
        inside = (gpu["seg"] >= 0) & (off[cid] + gpu["seg"] < off[cid + 1])
        g = np.where(inside, g, 0)
        slack = 1e-12
        holds = inside & (ref["tab"][g, 0] - slack <= gpu["t"]) & (gpu["t"] <= ref["tab"][g, 1] + slack)
        bad_h = np.nonzero(~holds)[0]
        assert bad_h.size == 0, f"{label}: {bad_h.size} returned pieces do not hold the returned t, e.g. {bad_h[:5]}"
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


def compare_surf(S, sid, q, out, ref, ex=None, label="", flags=False):
    """Parity bar: distance within 1e-6 * diag and never below the oracle; (u, v) within 1e-7 where the
    oracle's minimum is unique and well conditioned; the patch index equals the exported patch holding the
    oracle's (u, v) where unique and not within 1e-7 of a patch side."""
    diag = surf_diag(S)[sid]
    X = oracle.surf_eval(S, sid, out["uv"])
    real = np.abs(np.linalg.norm(X - q, axis=1) - out["dist"]) / diag
    bad = np.nonzero(~(real <= REAL_REL))[0]
    assert bad.size == 0, (f"{label}: {bad.size} distances not realised by their (u, v), worst {np.nanmax(real):.3e} "
                           f"at {bad[:5]}")
    err = np.abs(out["dist"] - ref["dist"]) / diag
    below = (ref["dist"] - out["dist"]) / diag
    unique = (ref["runner"] - ref["dist"]) > UNIQUE_REL * diag
    wc = unique & (ref["kappa"] >= KAPPA_MIN)
    duv = np.abs(out["uv"] - ref["uv"]).max(1)
    st = {"n": int(len(sid)), "max_dist_rel": float(err.max()), "max_uv_err_wc": float(duv[wc].max()) if wc.any() else 0.0,
          "wc_frac": float(wc.mean()), "max_realised_rel": float(real.max())}
    if flags:
        st.update(check_flags(out, ref, diag, label))
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
