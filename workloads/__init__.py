"""Seeded synthetic inputs for the fuzzy-clustering solver and its oracle.

This module only draws inputs: similarity matrices S (symmetric CSR, no
diagonal stored), planted memberships and start points U0.  It holds none of
the method's arithmetic and is shared by the tests, the smoke check and the
benchmark, which feed the same arrays to the HIP path and to the oracle.

Every draw comes from a ``torch.Generator`` seeded from (seed, stream), so a
workload is a pure function of its parameters and the device it is drawn on
(CPU and GPU generators produce different streams; tests draw on the CPU).

Recipes (the five benchmark configurations built from them are in configs.json):

* ``er_planted``   -- Erdos-Renyi pattern with m distinct unordered pairs
  (i != j) drawn uniformly; values s_ij = clip(u*_i . u*_j + N(0, sigma^2), 0, 1),
  one draw per unordered pair, mirrored; stored zeros stay stored.
* ``chung_lu_planted`` -- power-law pattern: weights w_i i.i.d. from a
  continuous Pareto density proportional to w^-gamma on [w_min, w_max] with
  w_min chosen for the requested mean degree; pair endpoints drawn
  proportional to w (inverse CDF), self pairs dropped, duplicates removed,
  topped up to m distinct pairs; values as above.
* planted memberships: either Dirichlet(alpha) rows over all c clusters, or
  overlapping communities where node i joins k_i ~ U{1..kmax} of the c
  communities (without replacement) with Dirichlet(alpha) weights.
* start points: Dirichlet(1) rows (uniform on the simplex), or the constant
  1/c matrix.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np
import torch

# Stream identifiers keep independent draws apart for a given seed.
_STREAM_PATTERN, _STREAM_WEIGHTS, _STREAM_PLANT, _STREAM_NOISE, _STREAM_U0 = 1, 2, 3, 4, 5


def _gen(seed: int, stream: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed((int(seed) * 1_000_003 + stream * 7_919) & 0x7FFF_FFFF_FFFF_FFFF)
    return g


@dataclass
class Workload:
    """A symmetric CSR similarity (no diagonal stored) and a start point."""
    n: int
    c: int
    row_ptr: torch.Tensor   # int64 [n+1]
    col_idx: torch.Tensor   # int32 [nnz], sorted within each row
    val: torch.Tensor       # float32 or float64 [nnz]
    U0: torch.Tensor        # [n, c], rows on the unit simplex
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    def to(self, device) -> "Workload":
        return Workload(self.n, self.c, self.row_ptr.to(device), self.col_idx.to(device),
                        self.val.to(device), self.U0.to(device), dict(self.meta))

    def numpy(self):
        """(row_ptr int64, col_idx int32, val float64, U0 float64) host arrays."""
        return (self.row_ptr.cpu().numpy().astype(np.int64),
                self.col_idx.cpu().numpy().astype(np.int32),
                self.val.cpu().double().numpy(),
                self.U0.cpu().double().numpy())


# ----------------------------------------------------------------------------
# random variates
# ----------------------------------------------------------------------------

def _gamma(shape: torch.Tensor, g: torch.Generator) -> torch.Tensor:
    """Gamma(shape, 1) variates by Marsaglia and Tsang's squeeze method, with
    the boost Gamma(a) = Gamma(a + 1) * U^(1/a) for a < 1."""
    a = shape.to(torch.float64)
    small = a < 1.0
    a1 = torch.where(small, a + 1.0, a)
    d = a1 - 1.0 / 3.0
    cc = 1.0 / torch.sqrt(9.0 * d)
    out = torch.empty_like(a)
    todo = torch.arange(a.numel(), device=a.device)
    while todo.numel() > 0:
        x = torch.randn(todo.numel(), generator=g, device=a.device, dtype=torch.float64)
        u = torch.rand(todo.numel(), generator=g, device=a.device, dtype=torch.float64)
        dd, c_ = d[todo], cc[todo]
        v = (1.0 + c_ * x) ** 3
        ok = (v > 0) & (torch.log(u.clamp_min(1e-300)) <
                        0.5 * x * x + dd - dd * v + dd * torch.log(v.clamp_min(1e-300)))
        out[todo[ok]] = (dd * v)[ok]
        todo = todo[~ok]
    if bool(small.any()):
        u = torch.rand(a.numel(), generator=g, device=a.device, dtype=torch.float64)
        boost = u.clamp_min(1e-300) ** (1.0 / a)
        out = torch.where(small, out * boost, out)
    return out


def dirichlet_rows(n: int, c: int, alpha: float, seed: int, stream: int = _STREAM_U0,
                   device="cpu", dtype=torch.float64) -> torch.Tensor:
    """n rows, each Dirichlet(alpha * 1_c) (normalised Gamma draws)."""
    g = _gen(seed, stream, device)
    if alpha == 1.0:
        u = torch.rand(n, c, generator=g, device=device, dtype=torch.float64)
        x = -torch.log1p(-u)
    else:
        x = _gamma(torch.full((n * c,), float(alpha), device=device), g).view(n, c)
    x = x / x.sum(dim=1, keepdim=True)
    return x.to(dtype)


def uniform_start(n: int, c: int, device="cpu", dtype=torch.float64) -> torch.Tensor:
    return torch.full((n, c), 1.0 / c, device=device, dtype=dtype)


@dataclass
class Communities:
    """Overlapping planted memberships: node i has weights w[i, s] on
    communities ids[i, s] (unused slots carry weight 0)."""
    ids: torch.Tensor   # int64 [n, kmax]
    w: torch.Tensor     # float64 [n, kmax]


def planted_communities(n: int, c: int, kmax: int, alpha: float, seed: int,
                        device="cpu") -> Communities:
    g = _gen(seed, _STREAM_PLANT, device)
    kmax = min(kmax, c)
    k = torch.randint(1, kmax + 1, (n,), generator=g, device=device)
    # kmax distinct communities per node: the first kmax of a random permutation
    # (argsort of uniform keys); only the first k_i are used.
    keys = torch.rand(n, c, generator=g, device=device)
    ids = torch.argsort(keys, dim=1)[:, :kmax].contiguous()
    del keys
    gam = _gamma(torch.full((n * kmax,), float(alpha), device=device), g).view(n, kmax)
    used = torch.arange(kmax, device=device).view(1, -1) < k.view(-1, 1)
    gam = torch.where(used, gam, torch.zeros_like(gam))
    w = gam / gam.sum(dim=1, keepdim=True)
    return Communities(ids, w)


def communities_dense(cm: Communities, c: int) -> torch.Tensor:
    n = cm.ids.shape[0]
    U = torch.zeros(n, c, dtype=torch.float64, device=cm.ids.device)
    U.scatter_add_(1, cm.ids, cm.w)
    return U


def _planted_dot(cm_or_dense, a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    if isinstance(cm_or_dense, Communities):
        ia, wa = cm_or_dense.ids[a], cm_or_dense.w[a]
        ib, wb = cm_or_dense.ids[b], cm_or_dense.w[b]
        eq = ia.unsqueeze(2) == ib.unsqueeze(1)
        return (wa.unsqueeze(2) * wb.unsqueeze(1) * eq).sum(dim=(1, 2))
    U = cm_or_dense
    return (U[a] * U[b]).sum(dim=1)


# ----------------------------------------------------------------------------
# sparsity patterns
# ----------------------------------------------------------------------------

def _distinct_pairs(draw, m: int, n: int, device, batch: int):
    """Draw unordered pairs with ``draw(k) -> (a, b)`` until m distinct pairs
    with a != b exist; keep the first m distinct pairs in draw order.  Returns
    (a, b) with a < b, ordered by the key a*n + b."""
    keys = torch.empty(0, dtype=torch.int64, device=device)
    order_base = 0
    first_idx = torch.empty(0, dtype=torch.int64, device=device)
    while True:
        a, b = draw(batch)
        keep = a != b
        a, b = a[keep], b[keep]
        lo, hi = torch.minimum(a, b), torch.maximum(a, b)
        new_keys = lo * n + hi
        new_idx = torch.arange(order_base, order_base + new_keys.numel(), device=device)
        order_base += int(batch)
        keys = torch.cat([keys, new_keys])
        first_idx = torch.cat([first_idx, new_idx])
        skeys, perm = torch.sort(keys, stable=True)
        head = torch.ones_like(skeys, dtype=torch.bool)
        head[1:] = skeys[1:] != skeys[:-1]
        keys, first_idx = skeys[head], first_idx[perm[head]]
        if keys.numel() >= m:
            sel = torch.sort(first_idx).indices[:m]
            kept = torch.sort(keys[sel]).values
            return kept // n, kept % n
        batch = max(1024, int((m - keys.numel()) * 1.2) + 1024)


def er_pairs(n: int, m: int, seed: int, device="cpu"):
    g = _gen(seed, _STREAM_PATTERN, device)

    def draw(k):
        a = torch.randint(0, n, (k,), generator=g, device=device)
        b = torch.randint(0, n, (k,), generator=g, device=device)
        return a, b
    return _distinct_pairs(draw, m, n, device, batch=int(m * 1.02) + 1024)


def pareto_wmin_for_mean(mean: float, gamma: float, wmax: float) -> float:
    """w_min such that the Pareto density proportional to w^-gamma on
    [w_min, wmax] has the given mean (bisection)."""
    a = gamma - 1.0

    def mean_of(wmin):
        r = (wmin / wmax) ** a
        if abs(a - 1.0) < 1e-12:
            tail = math.log(wmax / wmin)
        else:
            tail = (wmax ** (1.0 - a) - wmin ** (1.0 - a)) / (1.0 - a)
        return a * wmin ** a / (1.0 - r) * tail
    lo, hi = 1e-6, mean
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mean_of(mid) < mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def chung_lu_pairs(n: int, m: int, gamma: float, mean_deg: float, wmax: float, seed: int,
                   device="cpu"):
    """Power-law pairs: endpoints drawn proportional to Pareto weights."""
    gw = _gen(seed, _STREAM_WEIGHTS, device)
    wmin = pareto_wmin_for_mean(mean_deg, gamma, wmax)
    a = gamma - 1.0
    u = torch.rand(n, generator=gw, device=device, dtype=torch.float64)
    lo, hi = wmin ** (-a), wmax ** (-a)
    w = (lo - u * (lo - hi)) ** (-1.0 / a)
    cdf = torch.cumsum(w, 0)
    total = float(cdf[-1])
    g = _gen(seed, _STREAM_PATTERN, device)
    chunk = 1 << 26

    def draw(k):
        outs = []
        for s in range(0, k, chunk):
            kk = min(chunk, k - s)
            q = torch.rand(2, kk, generator=g, device=device, dtype=torch.float64) * total
            idx = torch.searchsorted(cdf, q).clamp_max(n - 1)
            outs.append(idx)
        idx = torch.cat(outs, dim=1)
        return idx[0], idx[1]
    return _distinct_pairs(draw, m, n, device, batch=int(m * 1.08) + 1024), wmin


def symmetric_csr(n: int, a: torch.Tensor, b: torch.Tensor, v: torch.Tensor):
    """CSR of the symmetric matrix with entries v at (a, b) and (b, a), a < b,
    input sorted by (a, b).  Columns come out sorted within each row: the
    lower part (b, a) entries precede the upper part (a, b) entries."""
    device = a.device
    m = a.numel()
    cnt_up = torch.bincount(a, minlength=n)
    cnt_lo = torch.bincount(b, minlength=n)
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    row_ptr[1:] = torch.cumsum(cnt_up + cnt_lo, 0)
    nnz = int(row_ptr[-1])
    col = torch.empty(nnz, dtype=torch.int32, device=device)
    val = torch.empty(nnz, dtype=v.dtype, device=device)
    up_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    up_ptr[1:] = torch.cumsum(cnt_up, 0)
    lo_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    lo_ptr[1:] = torch.cumsum(cnt_lo, 0)
    k = torch.arange(m, device=device)
    # upper entries (row a, column b): already sorted by (a, b)
    pos = row_ptr[a] + cnt_lo[a] + (k - up_ptr[a])
    col[pos] = b.to(torch.int32)
    val[pos] = v
    # lower entries (row b, column a): sort by (b, a)
    perm = torch.sort(b * n + a).indices
    bs, as_ = b[perm], a[perm]
    pos = row_ptr[bs] + (k - lo_ptr[bs])
    col[pos] = as_.to(torch.int32)
    val[pos] = v[perm]
    return row_ptr, col, val


def _values(planted, a, b, sigma, seed, device, dtype, chunk=1 << 24):
    g = _gen(seed, _STREAM_NOISE, device)
    out = torch.empty(a.numel(), dtype=dtype, device=device)
    for s in range(0, a.numel(), chunk):
        e = min(a.numel(), s + chunk)
        dot = _planted_dot(planted, a[s:e], b[s:e])
        noise = torch.randn(e - s, generator=g, device=device, dtype=torch.float64) * sigma
        out[s:e] = (dot + noise).clamp(0.0, 1.0).to(dtype)
    return out


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def er_planted(n: int, c: int, avg_deg: float, sigma: float, seed: int, *,
               plant: str = "communities", alpha: float = 0.2, kmax: int = 3,
               u0: str = "dirichlet", device="cpu", val_dtype=torch.float32,
               u_dtype=torch.float32) -> Workload:
    """ER pattern with m = round(n * avg_deg / 2) pairs and planted values."""
    m = int(round(n * avg_deg / 2.0))
    if plant == "dirichlet":
        planted = dirichlet_rows(n, c, alpha, seed, stream=_STREAM_PLANT, device=device)
    else:
        planted = planted_communities(n, c, kmax, alpha, seed, device=device)
    a, b = er_pairs(n, m, seed, device=device)
    v = _values(planted, a, b, sigma, seed, device, val_dtype)
    row_ptr, col, val = symmetric_csr(n, a, b, v)
    U0 = (dirichlet_rows(n, c, 1.0, seed, device=device, dtype=u_dtype) if u0 == "dirichlet"
          else uniform_start(n, c, device=device, dtype=u_dtype))
    return Workload(n, c, row_ptr, col, val, U0,
                    dict(pattern="er", pairs=m, avg_deg=avg_deg, sigma=sigma, seed=seed,
                         plant=plant, alpha=alpha, kmax=kmax, u0=u0))


def chung_lu_planted(n: int, c: int, mean_deg: float, gamma: float, wmax: float,
                     sigma: float, seed: int, *, alpha: float = 0.2, kmax: int = 3,
                     device="cpu", val_dtype=torch.float32,
                     u_dtype=torch.float32) -> Workload:
    m = int(round(n * mean_deg / 2.0))
    planted = planted_communities(n, c, kmax, alpha, seed, device=device)
    (a, b), wmin = chung_lu_pairs(n, m, gamma, mean_deg, wmax, seed, device=device)
    v = _values(planted, a, b, sigma, seed, device, val_dtype)
    del planted
    row_ptr, col, val = symmetric_csr(n, a, b, v)
    del a, b, v
    U0 = dirichlet_rows(n, c, 1.0, seed, device=device, dtype=u_dtype)
    deg = row_ptr[1:] - row_ptr[:-1]
    return Workload(n, c, row_ptr, col, val, U0,
                    dict(pattern="chung-lu", pairs=m, mean_deg=mean_deg, gamma=gamma,
                         wmax=wmax, wmin=wmin, sigma=sigma, seed=seed,
                         realised_mean_deg=float(deg.double().mean()),
                         realised_max_deg=int(deg.max())))


# The five configurations of the fuzzy-clustering workload family, as stored
# in configs.json (generator, parameters, seed and how each is run).
CONFIGS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs.json")
_DT = {"fp64": torch.float64, "fp32": torch.float32}


def configs() -> dict:
    """The configuration records of configs.json, by name (C1..C5)."""
    with open(CONFIGS_PATH) as fh:
        return {k: v for k, v in json.load(fh).items() if not k.startswith("_")}


def from_config(name: str, seed: int | None = None, device="cpu", n: int | None = None,
                **overrides) -> Workload:
    """The workload of configuration `name` (C1..C4), with its stored seed
    unless one is given; n (and any generator keyword) may be overridden to
    build a smaller instance of the same family."""
    rec = configs()[name]
    p = dict(rec["params"])
    p.update(overrides)
    seed = rec["seed"] if seed is None else seed
    n_stored = p.pop("n")
    n = n_stored if n is None else n
    vdt, udt = _DT[p.pop("values")], _DT[p.pop("iterates")]
    if rec["generator"] == "er_planted":
        return er_planted(n, p.pop("c"), p.pop("avg_deg"), p.pop("sigma"), seed, device=device,
                          val_dtype=vdt, u_dtype=udt, **p)
    if rec["generator"] == "chung_lu_planted":
        return chung_lu_planted(n, p.pop("c"), p.pop("mean_deg"), p.pop("gamma"), p.pop("wmax"),
                                p.pop("sigma"), seed, device=device, val_dtype=vdt, u_dtype=udt, **p)
    raise ValueError(f"{name}: no single-instance generator ({rec['generator']})")


def config_small_fp64(seed: int = 0, device="cpu", u0: str = "dirichlet") -> Workload:
    """C1: n=2,000, c=8: Dirichlet(0.3) planted rows over 8 clusters, ER pattern
    of average degree 20 (40,000 stored nnz), sigma=0.02, FP64 values."""
    return from_config("C1", seed, device, u0=u0)


def config_medium(seed: int = 0, device="cpu", n: int = 1_000_000) -> Workload:
    """C2: n=1e6, c=32: 32 overlapping communities (1-3 per node,
    Dirichlet(0.2)), ER pattern of average degree 30 (~3e7 stored nnz),
    sigma=0.05, FP32."""
    return from_config("C2", seed, device, n)


def config_full_power_law(seed: int = 0, device="cpu", n: int = 70_000_000) -> Workload:
    """C3: n=7e7, c=32: power-law degrees (gamma 2.1, mean 20, max 50,000),
    ~1.4e9 stored nnz, planted values as in the medium config, FP32."""
    return from_config("C3", seed, device, n)


def config_mixed_full(seed: int = 0, device="cpu", n: int = 70_000_000) -> Workload:
    """C4: the medium generator at n=7e7: ER pattern of average degree 30
    (~2.1e9 stored nnz), 32 overlapping communities, sigma=0.05, FP32 values
    (the mixed-precision solver keeps its own FP16 copy)."""
    return from_config("C4", seed, device, n)


def two_cluster_er(seed: int = 0, device="cpu", n1: int = 500_000, n2: int = 250_000,
                   deg1: float = 1200.0, deg2: float = 1600.0, bridges: int = 200) -> Workload:
    """The artificial graph of the paper's experiments (section 5): two
    Erdos-Renyi clusters of n1 and n2 nodes with edge probabilities
    deg1/(n1-1) and deg2/(n2-1), here as the expected number of edges drawn as
    distinct pairs, plus `bridges` distinct edges between the clusters.
    Similarities are the adjacency (S = A + I through the unit diagonal), the
    start puts every node fully in the second cluster, and
    meta["labels"] holds the ground truth (0 for the first n1 nodes)."""
    n = n1 + n2
    m1 = int(round(deg1 * n1 / 2.0))
    m2 = int(round(deg2 * n2 / 2.0))
    a1, b1 = er_pairs(n1, m1, seed, device=device)
    a2, b2 = er_pairs(n2, m2, seed + 1, device=device)
    g = _gen(seed, _STREAM_PLANT, device)
    ka = torch.empty(0, dtype=torch.int64, device=device)
    while ka.numel() < bridges:           # distinct inter-cluster pairs, first in draw order
        x = torch.randint(0, n1, (2 * bridges,), generator=g, device=device)
        y = torch.randint(n1, n, (2 * bridges,), generator=g, device=device)
        cand = torch.cat([ka, x * n + y])
        uniq, inv = torch.unique(cand, return_inverse=True)
        first = torch.full((uniq.numel(),), cand.numel(), dtype=torch.int64, device=device)
        first.scatter_reduce_(0, inv, torch.arange(cand.numel(), device=device), reduce="amin")
        ka = cand[torch.sort(first).values]
    ka = ka[:bridges]
    keys = torch.cat([a1 * n + b1, (a2 + n1) * n + (b2 + n1), ka])
    del a1, b1, a2, b2
    keys = torch.sort(keys).values
    a, b = keys // n, keys % n
    del keys
    v = torch.ones(a.numel(), dtype=torch.float32, device=device)
    row_ptr, col, val = symmetric_csr(n, a, b, v)
    del a, b, v
    U0 = torch.zeros(n, 2, dtype=torch.float32, device=device)
    U0[:, 1] = 1.0
    labels = torch.cat([torch.zeros(n1, dtype=torch.int8), torch.ones(n2, dtype=torch.int8)])
    return Workload(n, 2, row_ptr, col, val, U0,
                    dict(pattern="two-cluster ER", n1=n1, n2=n2, deg1=deg1, deg2=deg2,
                         bridges=bridges, labels=labels))


def serving_request(req_id: int, device="cpu", base_seed: int = 0) -> Workload:
    """One request of C5: n log-uniform in [500, 2e5], c in {4,8,16,32,64},
    average degree U(10, 40), planted communities, ER pattern (the ranges as
    stored in configs.json)."""
    p = configs()["C5"]["params"]
    g = _gen(base_seed + req_id, 6, "cpu")
    u = torch.rand(3, generator=g, dtype=torch.float64)
    lo, hi = (math.log(x) for x in p["n_loguniform"])
    n = int(round(math.exp(lo + float(u[0]) * (hi - lo))))
    choices = p["c_choices"]
    c = choices[min(len(choices) - 1, int(float(u[1]) * len(choices)))]
    d0, d1 = p["avg_deg_uniform"]
    d = d0 + (d1 - d0) * float(u[2])
    return er_planted(n, c, d, p["sigma"], base_seed + req_id, alpha=p["alpha"], kmax=p["kmax"],
                      device=device)
