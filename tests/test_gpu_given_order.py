"""A caller-given article order (FC_REORDER_GIVEN, `reorder=<array>` in the
binding).  Problem (P) is invariant under renumbering the articles, so any
order gives the natural order's iterates up to the order of the
cross-article sums.  The descending-degree order handed over by the caller
is the library's own relabelling, so it must reproduce FC_REORDER_DEGREE bit
for bit.  Invalid orders are rejected on the host before any device work,
a checkpoint resumes only under the order it was taken with, and a served
request under a given order runs exactly as it does alone."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fc():
    import paper_2506_04045_amd as fc
    fc.library_path()
    return fc


def _degree_order(row_ptr):
    deg = np.diff(row_ptr.cpu().numpy())
    return np.argsort(-deg, kind="stable").astype(np.int32)


@pytest.mark.parametrize("mode", [dict(), dict(defer_loss=True), dict(single_pass=True)],
                         ids=["default", "deferred", "single_pass"])
def test_given_degree_order_is_the_degree_relabelling_bit_for_bit(fc, mode):
    wl = W.chung_lu_planted(20000, 16, 20.0, 2.1, 20_000.0, 0.05, 9).to("cuda")
    perm = _degree_order(wl.row_ptr)
    assert not np.array_equal(perm, np.arange(wl.n))
    out = []
    for reorder in ("degree", perm):
        with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 16, wl.U0, step=1e-4, reorder=reorder,
                       **mode) as s:
            info = s.step(30)
            out.append((s.get_u().cpu().numpy(), info.f, s.history()["f"]))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]
    assert np.array_equal(out[0][2], out[1][2], equal_nan=True)


@pytest.mark.parametrize("single", [False, True])
def test_random_order_matches_the_natural_order_and_the_oracle(fc, single):
    wl = W.chung_lu_planted(6000, 8, 20.0, 2.1, 20_000.0, 0.05, 22, val_dtype=torch.float64,
                            u_dtype=torch.float64)
    rp, ci, v, U0 = wl.numpy()
    perm = np.random.default_rng(5).permutation(wl.n).astype(np.int32)
    ref = oracle.solve(rp, ci, v, True, U0, accelerate=True, max_iter=25, step=2e-4)
    d = wl.to("cuda")
    res = {}
    for name, reorder in (("none", "none"), ("given", perm)):
        with fc.Solver(d.row_ptr, d.col_idx, d.val, 8, d.U0, precision="fp64", step=2e-4,
                       reorder=reorder, single_pass=single) as s:
            info = s.step(25)
            res[name] = (s.get_u(torch.float64).cpu().numpy(), info.f)
    U, f = res["given"]
    assert np.abs(U - res["none"][0]).max() <= 1e-12
    assert abs(f - res["none"][1]) <= 1e-12 * abs(res["none"][1])
    assert np.abs(U - ref.X).max() <= 1e-9
    assert abs(f - ref.f[-1]) <= 1e-9 * abs(ref.f[0])


def test_invalid_orders_are_rejected(fc):
    from paper_2506_04045_amd import _native as N
    wl = W.er_planted(3000, 8, 10.0, 0.05, 3).to("cuda")
    good = np.random.default_rng(1).permutation(wl.n).astype(np.int32)
    cases = {}
    rep = good.copy()
    rep[17] = rep[4]
    cases["repeat"] = (rep, "entry 17 repeats")
    out = good.copy()
    out[9] = wl.n
    cases["range"] = (out, "entry 9 is outside")
    for name, (perm, msg) in cases.items():
        with pytest.raises(N.FcError) as e:
            fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, wl.U0, reorder=perm)
        assert e.value.status == N.FC_ERR_INVALID_ARG and msg in str(e.value), name
    with pytest.raises(ValueError):       # the binding checks the length
        fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, wl.U0, reorder=good[:-1])
    # FC_REORDER_GIVEN with no array, through the C ABI
    lib = N.load()
    opt = fc._options(8)
    opt.reorder = N.FC_REORDER_GIVEN
    csr = fc._CsrView(wl.row_ptr, wl.col_idx, wl.val)
    h = ctypes.c_void_p()
    st = lib.fc_create(ctypes.byref(csr.c), ctypes.byref(opt), None, N.FC_F32, None, ctypes.byref(h))
    assert st == N.FC_ERR_INVALID_ARG and not h.value
    assert b"perm" in lib.fc_last_error()
    # the library still works afterwards
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, wl.U0, reorder=good) as s:
        s.step(3)


def test_checkpoint_resumes_only_under_its_order(fc):
    from paper_2506_04045_amd import _native as N
    wl = W.er_planted(5000, 8, 12.0, 0.05, 31).to("cuda")
    rng = np.random.default_rng(2)
    P, Q = (rng.permutation(wl.n).astype(np.int32) for _ in range(2))
    kw = dict(step=1e-3)
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, wl.U0, reorder=P, **kw) as a:
        a.step(21)
        U_ref, f_ref = a.get_u().cpu().numpy(), a.info().f
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, wl.U0, reorder=P, **kw) as b:
        b.step(8)
        state = b.get_state()
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, None, reorder=P, **kw) as c:
        c.set_state(state)
        c.step(13)
        assert np.array_equal(c.get_u().cpu().numpy(), U_ref) and c.info().f == f_ref
    for other in (Q, "degree", "none"):
        with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, None, reorder=other, **kw) as d:
            with pytest.raises(N.FcError):
                d.set_state(state)


def _poll_for(sv, req_id, timeout_s=60.0):
    import time
    t_end = time.time() + timeout_s
    while time.time() < t_end:
        for r in sv.poll(timeout_us=20_000):
            if r.req_id == req_id:
                return r
    pytest.fail(f"request {req_id} did not finish")


@pytest.mark.parametrize("solo_max", [4, 0], ids=["solo_lane", "batched"])
def test_served_request_under_a_given_order_is_its_solo_run(fc, solo_max):
    from paper_2506_04045_amd import _native as N
    wl = W.er_planted(4000, 16, 15.0, 0.05, 42).to("cuda")
    perm = np.random.default_rng(8).permutation(wl.n).astype(np.int32)
    opts = dict(backtrack=True, max_iter=60, tol_pgrad=1e-4)
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 16, wl.U0, reorder=perm, **opts) as solo:
        solo.solve()
        U_solo, f_solo = solo.get_u().cpu().numpy(), solo.info().f
    with fc.Server(solo_max=solo_max) as sv:
        bad = perm.copy()
        bad[3] = bad[0]
        with pytest.raises(N.FcError) as e:
            sv.submit(1, wl.row_ptr, wl.col_idx, wl.val, 16, wl.U0, reorder=bad, **opts)
        assert e.value.status == N.FC_ERR_INVALID_ARG
        # the binding's int32 copy of the order is released when submit
        # returns; the request runs from the server's own copy
        sv.submit(2, wl.row_ptr, wl.col_idx, wl.val, 16, wl.U0, reorder=perm, **opts)
        r = _poll_for(sv, 2)
        assert r.status == 0 and r.f == f_solo
        assert np.array_equal(sv.get_u(2).cpu().numpy(), U_solo)
        sv.release(2)
        assert sv.stats()["bytes_in_use"] == 0
