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


def sample_rows(row_ptr, seed, k=2000):
    """Random articles plus the 8 largest rows and rows of each length class
    (at most 64, 65-2,048, more than 2,048 nonzeros); sorted, distinct."""
    deg = (row_ptr[1:] - row_ptr[:-1]).cpu().numpy()
    rng = np.random.default_rng(seed)
    rows = [rng.integers(0, deg.shape[0], k), np.argsort(deg)[-8:]]
    for lo, hi in ((0, 0), (1, 64), (65, 2048), (2049, 1 << 40)):
        cand = np.flatnonzero((deg >= lo) & (deg <= hi))
        if cand.size:
            rows.append(rng.choice(cand, min(64, cand.size), replace=False))
    return np.unique(np.concatenate(rows)).astype(np.int64)


def sub_csr(row_ptr, col_idx, val, rows):
    """Rows `rows` of the device CSR, copied to the host."""
    r = torch.from_numpy(rows).to(row_ptr.device)
    beg, lens = row_ptr[r], row_ptr[r + 1] - row_ptr[r]
    sub_rp = torch.zeros(rows.shape[0] + 1, dtype=torch.int64, device=row_ptr.device)
    torch.cumsum(lens, 0, out=sub_rp[1:])
    total = int(sub_rp[-1])
    owner = torch.repeat_interleave(torch.arange(rows.shape[0], device=row_ptr.device), lens)
    idx = beg[owner] + (torch.arange(total, device=row_ptr.device) - sub_rp[owner])
    return (sub_rp.cpu().numpy(), col_idx[idx].cpu().numpy(),
            val[idx].double().cpu().numpy())
