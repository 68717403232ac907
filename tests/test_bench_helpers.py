"""The measurement helpers of bench.py whose output is reported: the
renumbered column sequences the gather probe walks, the Cuthill-McKee order
and the count of columns repeated inside row blocks.  Checked on small graphs
against scipy's breadth-first search and against brute force."""

import numpy as np
import pytest
import scipy.sparse as sp
import torch
from scipy.sparse.csgraph import breadth_first_order

import bench
import workloads as W


@pytest.fixture(scope="module")
def graph():
    wl = W.chung_lu_planted(3000, 8, 12.0, 2.1, 400.0, 0.05, 4)
    deg = np.diff(wl.row_ptr.numpy())
    assert (deg == 0).any()      # rows the search cannot reach
    return wl


def _brute_relabel(rp, ci, perm):
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    out = []
    for old in perm:
        out.extend(inv[ci[rp[old]:rp[old + 1]]])
    return np.asarray(out), inv


def test_relabelled_columns_brute_force(graph):
    rp, ci = graph.row_ptr.numpy(), graph.col_idx.numpy()
    perm = np.random.default_rng(1).permutation(graph.n)
    col, inv = bench.relabelled_columns(graph.row_ptr, graph.col_idx, torch.from_numpy(perm),
                                        chunk_rows=257)
    ref, ref_inv = _brute_relabel(rp, ci, perm)
    assert np.array_equal(col.numpy(), ref) and np.array_equal(inv.numpy(), ref_inv)


def test_degree_relabelling_is_descending_degree_ties_by_index(graph):
    rp, ci = graph.row_ptr.numpy(), graph.col_idx.numpy()
    deg = np.diff(rp)
    perm = np.array(sorted(range(graph.n), key=lambda i: (-deg[i], i)))
    col, _ = bench.degree_relabelled_columns(graph.row_ptr, graph.col_idx, chunk_rows=100)
    assert np.array_equal(col.numpy(), _brute_relabel(rp, ci, perm)[0])


def test_cuthill_mckee_levels_and_parent_order(graph):
    rp, ci = graph.row_ptr.numpy(), graph.col_idx.numpy()
    deg = np.diff(rp)
    perm_t, reached = bench.cuthill_mckee_order(graph.row_ptr, graph.col_idx, edge_chunk=500)
    perm = perm_t.numpy()
    assert np.array_equal(np.sort(perm), np.arange(graph.n))
    assert deg[perm[0]] == deg.max()
    A = sp.csr_matrix((np.ones(ci.size), ci, rp), shape=(graph.n, graph.n))
    bfs, pred = breadth_first_order(A, int(perm[0]), directed=False, return_predecessors=True)
    assert reached == bfs.size and set(perm[:reached]) == set(bfs)
    dist = np.full(graph.n, -1)
    dist[perm[0]] = 0
    for v in bfs[1:]:
        dist[v] = dist[pred[v]] + 1
    lev = dist[perm[:reached]]
    assert (np.diff(lev) >= 0).all()          # levels contiguous, in order
    pos = np.empty(graph.n, np.int64)
    pos[perm] = np.arange(graph.n)
    keys = []
    for v in perm[1:reached]:                  # first-placed neighbour one level up, then degree
        nb = ci[rp[v]:rp[v + 1]]
        keys.append((pos[nb[dist[nb] == dist[v] - 1]].min(), deg[v]))
    assert keys == sorted(keys)
    rest = perm[reached:]                      # unreached rows by descending degree
    assert (np.diff(deg[rest]) <= 0).all()


@pytest.mark.parametrize("use_perm", [False, True])
def test_block_column_reuse_brute_force(graph, use_perm):
    rp, ci = graph.row_ptr.numpy(), graph.col_idx.numpy()
    deg = np.diff(rp)
    if use_perm:
        perm = np.random.default_rng(7).permutation(graph.n)
    else:
        perm = np.array(sorted(range(graph.n), key=lambda i: (-deg[i], i)))
    col, _ = bench.relabelled_columns(graph.row_ptr, graph.col_idx, torch.from_numpy(perm))
    col = col.numpy()
    rp_new = np.concatenate([[0], np.cumsum(deg[perm])])
    B = 64
    nblk = (graph.n + B - 1) // B
    total = repeats = hot = 0
    for b in range(nblk):                      # every block sampled
        cols = col[rp_new[b * B]:rp_new[min((b + 1) * B, graph.n)]]
        seen = set()
        for j in cols:
            if j in seen:
                repeats += 1
                hot += j < 32768
            seen.add(j)
        total += cols.size
    got = bench.block_column_reuse(graph.row_ptr, torch.from_numpy(col), sample_blocks=nblk,
                                   perm=torch.from_numpy(perm) if use_perm else None)
    assert got["nonzeros_sampled"] == total
    assert got["repeated_columns_share"] == pytest.approx(repeats / total, abs=0)
    assert got["repeats_on_32768_hottest_rows_share"] == pytest.approx(hot / repeats, abs=0)


def test_community_order_groups_by_dominant_planted_community(graph):
    perm = bench.community_order(graph, 4, 8).numpy()
    assert np.array_equal(np.sort(perm), np.arange(graph.n))
    cm = W.planted_communities(graph.n, 8, 3, 0.2, 4)
    dom = cm.ids.gather(1, torch.argmax(cm.w, dim=1, keepdim=True)).flatten().numpy()
    deg = np.diff(graph.row_ptr.numpy())
    key = list(zip(dom[perm], -deg[perm]))
    assert key == sorted(key)


def test_bench_refuses_more_than_one_gpu():
    """--gpus above 1 exits with a message before anything touches a GPU."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120, cwd=root)
    assert out.returncode == 2 and "one GPU" in out.stderr


def test_solver_order_for_each_leg():
    """The library's orders pass by name; a built order reaches the power-law
    legs as its array and the other workloads as degree order."""
    import argparse
    perm = np.arange(5, dtype=np.int32)[::-1].copy()
    for name in ("none", "degree"):
        a = argparse.Namespace(reorder=name)
        assert bench.solver_order(a) == name and bench.solver_order(a, power_law=False) == name
    for name in ("cm", "community"):
        a = argparse.Namespace(reorder=name, given_order=perm)
        assert bench.solver_order(a) is perm
        assert bench.solver_order(a, power_law=False) == "degree"
