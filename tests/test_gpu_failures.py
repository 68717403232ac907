"""Out-of-memory handling, forced from the host with the library's
allocation-failure hook (fc_debug_fail_allocations): each allocation a
solver's set-up, a stateless call or the serving worker makes is failed in
turn; the call must report FC_ERR_OUT_OF_MEMORY and release what it held,
and later calls must work and give the results of an undisturbed run (for a
served request: its solo result, bit for bit).  No kernel sees a failed
buffer: every failure returns before the first launch that would use it."""

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

OOM = 3   # FC_ERR_OUT_OF_MEMORY


@pytest.fixture(scope="module")
def fc():
    import paper_2506_04045_amd as fc
    fc.library_path()
    yield fc
    fc.debug_fail_allocations(-1)


@pytest.fixture(autouse=True)
def _injection_off(fc):
    fc.debug_fail_allocations(-1)
    yield
    fc.debug_fail_allocations(-1)


@pytest.fixture(scope="module")
def power_law():
    """Hub rows (chunked), medium rows and empty rows: every allocation site
    of the set-up is reached, with degree relabelling and validation on."""
    wl = W.chung_lu_planted(6000, 8, 20.0, 2.1, 20_000.0, 0.05, 22).to("cuda")
    deg = (wl.row_ptr[1:] - wl.row_ptr[:-1]).cpu()
    assert (deg > 2048).any() and ((deg > 64) & (deg <= 2048)).any()
    return wl


def _free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("kw", [dict(reorder="degree", validate=True),
                                dict(backtrack=True, precision="mixed"),
                                dict(single_pass=True, step=1e-4)],
                         ids=["relabelled", "mixed_backtracking", "single_pass"])
def test_solver_setup_fails_cleanly_at_every_allocation(fc, power_law, kw):
    from paper_2506_04045_amd import _native
    wl = power_law
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, wl.U0, **kw) as ref:
        ref.step(12)
        U_ref, f_ref = ref.get_u().cpu().numpy(), ref.info().f
    free0 = _free_bytes()
    failures = 0
    for after in range(400):
        fc.debug_fail_allocations(after)
        try:
            s = fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, wl.U0, **kw)
        except _native.FcError as e:
            assert e.status == OOM, (after, str(e))
            failures += 1
            continue
        fc.debug_fail_allocations(-1)
        with s:
            s.step(12)
            assert np.array_equal(s.get_u().cpu().numpy(), U_ref) and s.info().f == f_ref
        break
    else:
        pytest.fail("the set-up did not succeed within 400 allocations")
    free1 = _free_bytes()
    print(f"{kw}: {failures} allocation points failed cleanly; free memory "
          f"{(free1 - free0) / 2**20:+.1f} MiB")
    assert failures >= 10
    assert free1 >= free0 - (64 << 20)   # nothing the failed set-ups held is kept


def test_stateless_calls_report_out_of_memory(fc, power_law):
    from paper_2506_04045_amd import _native
    wl = power_law
    U = wl.U0
    f_ref = fc.objective(wl.row_ptr, wl.col_idx, wl.val, U)
    G_ref = fc.gram(U)
    fc.debug_fail_allocations(0)
    for call in (lambda: fc.objective(wl.row_ptr, wl.col_idx, wl.val, U),
                 lambda: fc.gram(U),
                 lambda: fc.spectral_norm(wl.row_ptr, wl.col_idx, wl.val)):
        with pytest.raises(_native.FcError) as e:
            call()
        assert e.value.status == OOM
    P = fc.project(U.double() * 2.0)   # allocates nothing
    fc.debug_fail_allocations(-1)
    assert np.abs(P.sum(1).cpu().numpy() - 1.0).max() <= 1e-12
    assert fc.objective(wl.row_ptr, wl.col_idx, wl.val, U) == f_ref
    assert np.array_equal(fc.gram(U), G_ref)


def _poll_for(sv, req_id, timeout_s=60.0):
    import time
    t_end = time.time() + timeout_s
    while time.time() < t_end:
        for r in sv.poll(timeout_us=20_000):
            if r.req_id == req_id:
                return r
    pytest.fail(f"request {req_id} did not finish")


def test_server_isolates_an_allocation_failure(fc):
    a = W.er_planted(3000, 8, 12.0, 0.05, 41).to("cuda")
    b = W.er_planted(4000, 16, 15.0, 0.05, 42).to("cuda")
    opts = dict(backtrack=True, max_iter=60, tol_pgrad=1e-4)
    with fc.Solver(b.row_ptr, b.col_idx, b.val, 16, b.U0, **opts) as solo:
        solo.solve()
        U_solo, f_solo = solo.get_u().cpu().numpy(), solo.info().f
    for solo_max in (4, 0):   # the solo lane and the batched tables
        with fc.Server(solo_max=solo_max) as sv:
            fc.debug_fail_allocations(0)
            sv.submit(1, a.row_ptr, a.col_idx, a.val, 8, a.U0, **opts)
            r1 = _poll_for(sv, 1)
            fc.debug_fail_allocations(-1)
            assert r1.status == OOM
            sv.submit(2, b.row_ptr, b.col_idx, b.val, 16, b.U0, **opts)
            r2 = _poll_for(sv, 2)
            assert r2.status == 0 and r2.f == f_solo
            assert np.array_equal(sv.get_u(2).cpu().numpy(), U_solo)
            sv.release(2)
            assert sv.stats()["bytes_in_use"] == 0
