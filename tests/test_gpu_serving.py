"""Serving: continuous batching of many solves on one GPU (fc_server_*).

Every served request must give exactly the result of the same solve run
alone through fc_create + fc_solve (same options): the batched kernels do,
per instance, the work of the single-instance kernels.  Admission respects
the memory budget, a request larger than the budget fails alone, and a
request that goes non-finite does not disturb the others.
"""
import time

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

SOLVE = dict(backtrack=True, tol_pgrad=1e-4, max_iter=150, norm_estimate="frobenius",
             check_every=8)


@pytest.fixture(scope="module")
def fc():
    import paper_2506_04045_amd as fc
    fc.library_path()
    return fc


def _requests(k, seed0=100, nmax=6000):
    out = []
    for i in range(k):
        g = np.random.default_rng(seed0 + i)
        n = int(np.exp(g.uniform(np.log(300), np.log(nmax))))
        c = [4, 8, 16, 32, 64, 3, 20][i % 7]
        d = float(g.uniform(6, 20))
        out.append(W.er_planted(n, c, d, 0.05, seed0 + i).to("cuda"))
    return out


def _alone(fc, wl, **kw):
    opts = dict(SOLVE)
    opts.update(kw)
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, wl.c, wl.U0, **opts) as s:
        info = s.solve()
        return info, s.get_u().cpu().numpy()


def _serve(fc, reqs, server_kw=None, stagger=None, **kw):
    opts = dict(SOLVE)
    opts.update(kw)
    done = {}
    with fc.Server(**(server_kw or {})) as sv:
        order = list(range(len(reqs)))
        submitted = 0
        t0 = time.time()
        while len(done) < len(reqs):
            limit = len(reqs) if stagger is None else min(len(reqs), stagger + len(done))
            while submitted < limit:
                wl = reqs[order[submitted]]
                sv.submit(order[submitted], wl.row_ptr, wl.col_idx, wl.val, wl.c, wl.U0, **opts)
                submitted += 1
            for r in sv.poll(64, timeout_us=20000):
                U = sv.get_u(r.req_id).cpu().numpy() if r.status == 0 else None
                done[r.req_id] = (r, U)
                sv.release(r.req_id)
            assert time.time() - t0 < 120, "serving did not finish"
    return done


@pytest.mark.parametrize("solo_max", [0, 4])
@pytest.mark.parametrize("use_graph", [True, False])
def test_results_are_the_same_alone_and_in_the_mix(fc, use_graph, solo_max):
    """solo_max = 0: every request batched; 4: the first ones run in the solo
    lane while few are active, the others join the batched kernels."""
    reqs = _requests(14)
    alone = [_alone(fc, wl) for wl in reqs]
    served = _serve(fc, reqs, dict(use_graph=use_graph, ticks_per_poll=4, solo_max=solo_max))
    for i, wl in enumerate(reqs):
        r, U = served[i]
        info, U_ref = alone[i]
        assert r.status == 0
        assert r.iter == info.iter and r.stop_reason == info.stop_reason
        assert r.f == info.f, (i, r.f, info.f)
        assert np.array_equal(U, U_ref), i


def test_staggered_arrivals_join_running_batches(fc):
    reqs = _requests(10, seed0=300)
    alone = [_alone(fc, wl) for wl in reqs]
    served = _serve(fc, reqs, dict(max_active=3, ticks_per_poll=2), stagger=3)
    for i in range(len(reqs)):
        r, U = served[i]
        assert r.status == 0 and r.f == alone[i][0].f and np.array_equal(U, alone[i][1])
        assert r.t_submit <= r.t_setup <= r.t_admit <= r.t_start <= r.t_finish


def test_admission_respects_the_memory_budget(fc):
    reqs = _requests(8, seed0=500, nmax=3000)
    with fc.Server(max_active=64, hbm_budget=64 * 2**20, ticks_per_poll=2) as sv:
        for i, wl in enumerate(reqs):
            sv.submit(i, wl.row_ptr, wl.col_idx, wl.val, wl.c, wl.U0, **SOLVE)
        seen, peak = {}, 0.0
        t0 = time.time()
        while len(seen) < len(reqs):
            st = sv.stats()
            peak = max(peak, st["bytes_in_use"])
            for r in sv.poll(16, timeout_us=5000):
                seen[r.req_id] = r
                sv.release(r.req_id)
            assert time.time() - t0 < 120
        assert all(r.status == 0 for r in seen.values())
        assert 0 < peak <= 64 * 2**20


def test_request_larger_than_the_budget_fails_alone(fc):
    big = W.er_planted(50_000, 64, 10.0, 0.05, 700).to("cuda")   # ~77 MB of iterates
    with fc.Server(hbm_budget=2 * 2**20) as sv:
        sv.submit(1, big.row_ptr, big.col_idx, big.val, big.c, big.U0, **SOLVE)
        res = []
        t0 = time.time()
        while not res:
            res = sv.poll(4, timeout_us=20000)
            assert time.time() - t0 < 30
        from paper_2506_04045_amd import _native
        assert res[0].status == _native.FC_ERR_OUT_OF_MEMORY


def test_nonfinite_request_is_isolated(fc):
    reqs = _requests(5, seed0=900)
    bad = reqs[2]
    U0 = bad.U0.clone()
    U0[0, 0] = float("nan")
    bad_wl = W.Workload(bad.n, bad.c, bad.row_ptr, bad.col_idx, bad.val, U0)
    alone = {i: _alone(fc, wl) for i, wl in enumerate(reqs) if i != 2}
    mixed = reqs[:2] + [bad_wl] + reqs[3:]
    served = _serve(fc, mixed)
    from paper_2506_04045_amd import _native
    assert served[2][0].status == _native.FC_ERR_NONFINITE
    for i, (info, U_ref) in alone.items():
        r, U = served[i]
        assert r.status == 0 and r.f == info.f and np.array_equal(U, U_ref)


def test_a_served_solve_follows_the_oracle(fc):
    wl = W.er_planted(4000, 16, 15.0, 0.05, 17)
    rp, ci, v, U0 = wl.numpy()
    served = _serve(fc, [wl.to("cuda")], backtrack=True, tol_pgrad=0.0, max_iter=40,
                    norm_estimate="frobenius", L0=50.0)
    r, U = served[0]
    ref = oracle.solve(rp, ci, v, True, U0, accelerate=True, max_iter=40, backtrack=True, L0=50.0)
    assert r.iter == 40
    assert abs(r.f - ref.f[-1]) <= 1e-4 * abs(ref.f[-1])
    assert np.abs(U - ref.X).max() <= 1e-4


def test_relabelled_requests_match_their_solo_runs(fc):
    reqs = _requests(6, seed0=1100)
    alone = [_alone(fc, wl, reorder="degree") for wl in reqs]
    served = _serve(fc, reqs, dict(ticks_per_poll=2), reorder="degree")
    for i in range(len(reqs)):
        r, U = served[i]
        assert r.status == 0 and r.f == alone[i][0].f and np.array_equal(U, alone[i][1])


def test_tuned_schedule_keeps_every_result(fc):
    """The autotuner runs the sample under many schedules (graph replay,
    ticks per poll, launch-table entries per padded width), checks that none
    changes a result, and returns a valid schedule; a server built from it
    still gives every request its solo result."""
    reqs = _requests(10, seed0=300, nmax=4000)
    sample = [dict(row_ptr=wl.row_ptr, col_idx=wl.col_idx, val=wl.val, c=wl.c, U0=wl.U0, **SOLVE)
              for wl in reqs]
    t = fc.tune_server(sample, use_graph=False, ticks_per_poll=8)
    print(f"tuned schedule {t}")
    assert t["ticks_per_poll"] in (4, 8, 16, 32)
    widths = {max(4, 1 << (wl.c - 1).bit_length()) for wl in reqs}
    for k, cp in enumerate((4, 8, 16, 32, 64)):
        if cp in widths:
            assert t["grid_fused"][k] in (1, 2, 4) and t["grid_spmm"][k] in (4, 8, 16, 32)
        else:
            assert t["grid_fused"][k] == 0 and t["grid_spmm"][k] == 0
    assert t["solves_per_s"] > 0 and t["runs"] >= 9
    served = _serve(fc, reqs, dict(ticks_per_poll=t["ticks_per_poll"], use_graph=t["use_graph"],
                                   grid_fused=t["grid_fused"], grid_spmm=t["grid_spmm"]))
    for i, wl in enumerate(reqs):
        r, U = served[i]
        info, U_ref = _alone(fc, wl)
        assert r.status == 0
        assert r.f == info.f and r.iter == info.iter
        assert np.array_equal(U, U_ref)


def test_large_request_sums_as_it_does_alone(fc):
    """An instance above two fused workgroups per CU of 64-row tiles with
    eight tiles each (n > 2 * CUs * 512) gets more fused workgroups; served
    and solo solves use the same count, so the result stays bitwise equal."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    n = 2 * cus * 512 + 40_000
    big = W.er_planted(n, 4, 6.0, 0.05, 1300).to("cuda")
    small = _requests(3, seed0=1400)
    kw = dict(max_iter=30)
    alone = [_alone(fc, wl, **kw) for wl in [big] + small]
    served = _serve(fc, [big] + small, dict(ticks_per_poll=4), **kw)
    for i in range(4):
        r, U = served[i]
        info, U_ref = alone[i]
        assert r.status == 0 and r.iter == info.iter
        assert r.f == info.f, (i, r.f, info.f)
        assert np.array_equal(U, U_ref), i


def test_cancel_queued_and_running_requests(fc):
    """fc_server_cancel: a running request stops with its last accepted
    iterate (rows on the simplex, fewer iterations than its budget), a queued
    one leaves the queue without running, the others finish exactly as they
    do alone, and unknown ids are rejected."""
    from paper_2506_04045_amd import _native as N
    cancelled = N.STATUS_CODES["FC_ERR_CANCELLED"]
    big = W.er_planted(200_000, 32, 20.0, 0.05, 901).to("cuda")
    small = _requests(3, seed0=910)
    alone = [_alone(fc, wl) for wl in small]
    budget = 20_000
    long_solve = dict(SOLVE, max_iter=budget, tol_pgrad=0.0)
    seen = {}

    def collect(timeout_us=20000):
        for r in sv.poll(16, timeout_us=timeout_us):
            seen[r.req_id] = r
            if r.req_id in (10, 12):
                k = r.req_id - 10
                assert r.status == 0 and r.f == alone[k][0].f
                assert np.array_equal(sv.get_u(r.req_id).cpu().numpy(), alone[k][1])

    with fc.Server(max_active=2, ticks_per_poll=2) as sv:
        sv.submit(0, big.row_ptr, big.col_idx, big.val, big.c, big.U0, **long_solve)
        sv.submit(1, big.row_ptr, big.col_idx, big.val, big.c, big.U0, **long_solve)
        for i, wl in enumerate(small):       # queued behind the two big ones
            sv.submit(10 + i, wl.row_ptr, wl.col_idx, wl.val, wl.c, wl.U0, **SOLVE)
        time.sleep(0.3)
        sv.cancel(0)                         # running
        sv.cancel(11)                        # queued (both slots are taken)
        with pytest.raises(N.FcError):
            sv.cancel(12345)
        t0 = time.time()
        while 0 not in seen or 11 not in seen:
            collect()
            assert time.time() - t0 < 60
        r0, r11 = seen[0], seen[11]
        assert r0.status == cancelled and 0 < r0.iter < budget
        U0c = sv.get_u(0).double()
        assert (U0c >= 0).all() and float((U0c.sum(1) - 1).abs().max()) <= 1e-5
        assert r11.status == cancelled and r11.iter == 0
        sv.cancel(1)
        sv.release(0)
        sv.release(11)
        t0 = time.time()
        while len(seen) < 5:
            collect()
            assert time.time() - t0 < 60
        assert seen[1].status == cancelled and seen[1].iter < budget
        sv.cancel(10)                        # already finished: left as it is
        assert sv.poll(16, timeout_us=0) == []


@pytest.mark.parametrize("depths", [[2, 8, 2, 8, 2], [8, 2, 8, 2, 8]])
def test_spmm_tile_shape_changes_no_result(fc, depths):
    """The tuned tile shape of the batched sparse product (gathers in flight
    per slot) changes speed only: every request, all batched, bitwise equals
    its solo run."""
    reqs = _requests(10, seed0=1300)
    alone = [_alone(fc, wl) for wl in reqs]
    served = _serve(fc, reqs, dict(ticks_per_poll=4, solo_max=0, spmm_depth=depths))
    for i in range(len(reqs)):
        r, U = served[i]
        assert r.status == 0 and r.f == alone[i][0].f and np.array_equal(U, alone[i][1]), i
