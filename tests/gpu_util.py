"""Helpers shared by the GPU parity tests (argument plumbing only)."""
import numpy as np
import torch

import workloads as W


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def csr_to_dev(rp, ci, v, vdtype):
    return dev(rp, torch.int64), dev(ci, torch.int32), dev(v, vdtype)


def normwise(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def star_plus_er(n, avg_deg, seed, hub_frac=1.0):
    """ER pattern plus a hub row connected to a fraction of all other rows
    (a row far longer than any tile or team), values in [0, 1]."""
    rng = np.random.default_rng(seed)
    wl = W.er_planted(n, 4, avg_deg, 0.05, seed, val_dtype=torch.float64)
    rp, ci, v, _ = wl.numpy()
    rows = [list(zip(ci[rp[i]:rp[i + 1]], v[rp[i]:rp[i + 1]])) for i in range(n)]
    hub = 0
    others = rng.choice(np.arange(1, n), size=int((n - 1) * hub_frac), replace=False)
    have = {int(j) for j, _ in rows[hub]}
    for j in others:
        j = int(j)
        if j in have:
            continue
        s = float(rng.random())
        rows[hub].append((j, s))
        rows[j].append((hub, s))
    rp2 = [0]
    ci2, v2 = [], []
    for i in range(n):
        ent = sorted(rows[i])
        ci2 += [int(j) for j, _ in ent]
        v2 += [float(s) for _, s in ent]
        rp2.append(len(ci2))
    return (np.array(rp2, dtype=np.int64), np.array(ci2, dtype=np.int32),
            np.array(v2, dtype=np.float64))
