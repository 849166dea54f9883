"""Training data and training loop of the seeding networks.

Argument marshalling around libmrep: the candidate pieces and the network
inputs come from ``mrep_nn_features`` (curves) or ``mrep_nn_surface_features``
(surfaces), the labels from the library's certified projection
(``mrep_project_curves`` in FP64 mode, ``mrep_project_surfaces``), and every
forward, backward and Adam step runs in ``mrep_nn_train_step``.  Host code only
turns the projected parameter into the label of each candidate piece and
shuffles.

Label of a (query, candidate piece) pair: accept = 1 when the projection lies
on that piece (the piece holding the minimising parameter), with u* its local
parameter; accept = 0 otherwise, with the parameter loss masked.  The set is
balanced to equal numbers of positive and negative pairs.
"""
from __future__ import annotations

import numpy as np

from . import mrep


def training_pairs(plan, geom, q, curve_id, seed: int = 0, balance: bool = True):
    """(x[N,15], u[N], a[N]) device float32 tensors and a stats dict for queries q[n,3] on curve_id[n]
    (numpy arrays or device tensors)."""
    import torch

    if isinstance(q, torch.Tensor):
        qt, ct = q.contiguous(), curve_id.contiguous()
        curve_id = curve_id.cpu().numpy()
    else:
        qt = torch.from_numpy(np.ascontiguousarray(q, dtype=np.float64)).cuda()
        ct = torch.from_numpy(np.ascontiguousarray(curve_id, dtype=np.int32)).cuda()
    seg, x = geom.features(qt, ct)
    t, _, s, _ = geom.project(qt, ct, mrep.default_opts("fp64"))
    torch.cuda.synchronize()
    seg_h = seg.cpu().numpy()
    t_h, s_h = t.cpu().numpy(), s.cpu().numpy()
    ex = plan.export()
    seg_off, seg_t = ex["seg_off"], ex["seg_t"]
    cid = np.asarray(curve_id, np.int64)
    valid = seg_h >= 0
    gidx = np.where(valid, seg_off[cid][:, None] + seg_h, 0)
    accept = valid & (seg_h == s_h[:, None])
    ta, tb = seg_t[gidx, 0], seg_t[gidx, 1]
    u = np.where(accept, np.clip((t_h[:, None] - ta) / np.where(tb > ta, tb - ta, 1.0), 0.0, 1.0), 0.0)
    flat = np.flatnonzero(valid.ravel())
    pos = flat[accept.ravel()[flat]]
    neg = flat[~accept.ravel()[flat]]
    rng = np.random.default_rng(seed)
    if balance and len(neg) > len(pos):
        neg = rng.choice(neg, len(pos), replace=False)
    rows = np.sort(np.concatenate([pos, neg]))
    stats = {"queries": int(len(cid)), "pairs": int(len(rows)), "positives": int(len(pos)),
             "label_in_candidates": float(np.mean(accept.any(axis=1)))}
    r = torch.from_numpy(rows).cuda()
    xs = x.reshape(-1, mrep.NN_IN)[r].contiguous()
    us = torch.from_numpy(u.ravel()[rows].astype(np.float32)).cuda()
    ac = torch.from_numpy(accept.ravel()[rows].astype(np.float32)).cuda()
    return xs, us, ac, stats


def train(nn, x, u, a, epochs: int = 10, batch: int = 4096, lr: float = 1e-3, seed: int = 0):
    """Adam over shuffled minibatches; returns the per-step batch losses (numpy).  u: the targets (u[N] for
    curves, st[N, 2] for surfaces)."""
    import torch

    n = int(x.shape[0])
    batch = max(1, min(batch, n))
    steps = max(1, n // batch)
    loss = torch.zeros(epochs * steps, dtype=torch.float32, device=x.device)
    rng = np.random.default_rng(seed)
    k = 0
    for _ in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)[: steps * batch].astype(np.int32)).to(x.device)
        for i in range(steps):
            nn.train_step(x, u, a, rows=perm[i * batch:(i + 1) * batch], lr=lr, loss=loss[k:k + 1])
            k += 1
    torch.cuda.synchronize()
    return loss.cpu().numpy()


def surface_training_pairs(plan, geom, q, surface_id, seed: int = 0, balance: bool = True):
    """(x[N,51], st[N,2], a[N]) device float32 tensors and a stats dict for queries q[n,3] on surface_id[n].

    Labels come from the library's certified surface projection: a candidate patch is accepted when the projected
    (u, v) lies in its closed parameter rectangle, with (s, t) the local coordinates there."""
    import torch

    if isinstance(q, torch.Tensor):
        qt, ct = q.contiguous(), surface_id.contiguous()
        surface_id = surface_id.cpu().numpy()
    else:
        qt = torch.from_numpy(np.ascontiguousarray(q, dtype=np.float64)).cuda()
        ct = torch.from_numpy(np.ascontiguousarray(surface_id, dtype=np.int32)).cuda()
    patch, x = geom.surface_features(qt, ct)
    uv, _, _, _ = geom.project_surfaces(qt, ct)
    torch.cuda.synchronize()
    patch_h, uv_h = patch.cpu().numpy(), uv.cpu().numpy()
    ex = plan.export_surfaces()
    off, rect = ex["patch_off"], ex["patch_uv"]
    sid = np.asarray(surface_id, np.int64)
    valid = patch_h >= 0
    g = np.where(valid, off[sid][:, None] + patch_h, 0)
    r = rect[g]  # [n, 4, 4] (u0, u1, v0, v1)
    u, v = uv_h[:, 0][:, None], uv_h[:, 1][:, None]
    su = np.where(r[..., 1] > r[..., 0], r[..., 1] - r[..., 0], 1.0)
    sv = np.where(r[..., 3] > r[..., 2], r[..., 3] - r[..., 2], 1.0)
    s = (u - r[..., 0]) / su
    t = (v - r[..., 2]) / sv
    eps = 1e-9
    accept = valid & (s >= -eps) & (s <= 1 + eps) & (t >= -eps) & (t <= 1 + eps)
    st = np.stack([np.clip(s, 0.0, 1.0), np.clip(t, 0.0, 1.0)], axis=-1)
    st = np.where(accept[..., None], st, 0.0)
    flat = np.flatnonzero(valid.ravel())
    pos = flat[accept.ravel()[flat]]
    neg = flat[~accept.ravel()[flat]]
    rng = np.random.default_rng(seed)
    if balance and len(neg) > len(pos):
        neg = rng.choice(neg, len(pos), replace=False)
    rows = np.sort(np.concatenate([pos, neg]))
    stats = {"queries": int(len(sid)), "pairs": int(len(rows)), "positives": int(len(pos)),
             "label_in_candidates": float(np.mean(accept.any(axis=1)))}
    rr = torch.from_numpy(rows).cuda()
    xs = x.reshape(-1, x.shape[-1])[rr].contiguous()
    ts = torch.from_numpy(st.reshape(-1, 2)[rows].astype(np.float32)).cuda()
    ac = torch.from_numpy(accept.ravel()[rows].astype(np.float32)).cuda()
    return xs, ts, ac, stats
