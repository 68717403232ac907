"""Solver-level parity of the HIP path against the FP64 oracle (Alg. 2-4),
called through the C ABI.

Tolerances (stated in the fuzzy-clustering workload's parity bar):
* FP64 on the GPU follows the oracle to rounding: per-iteration losses within
  1e-9 relative, iterates within 1e-9.
* FP32 on the GPU against the FP64 oracle: final loss within 1e-4 relative,
  the loss decrease f(U0) - f(U_K) within 1e-5 relative (the loss is
  dominated by ||G||^2 ~ n^2/c^2, which hides the decrease, so the decrease is
  checked on its own), iterates within 1e-4, rows summing to 1 within 1e-6.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests import pins
from tests.gpu_util import csr_to_dev, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fc():
    import paper_2506_04045_amd as fc
    fc.library_path()
    return fc


@pytest.fixture(scope="module")
def small():
    """The n = 2,000, c = 8 workload (Dirichlet(0.3) planted rows, ER
    degree 20, sigma 0.02) with a Dirichlet(1) start."""
    wl = W.config_small_fp64(seed=0)
    rp, ci, v, U0 = wl.numpy()
    spec, _ = oracle.spectral_norm(rp, ci, v, True)
    return dict(rp=rp, ci=ci, v=v, U0=U0, n=wl.n, c=wl.c,
                tau=1.0 / oracle.lipschitz_bound(spec, wl.n))


def _solve_gpu(fc, rp, ci, v, U0, c, prec, iters, **kw):
    vd = torch.float64 if prec == "fp64" else torch.float32
    ud = torch.float64 if prec == "fp64" else torch.float32
    S = csr_to_dev(rp, ci, v, vd)
    with fc.Solver(*S, c, dev(U0, ud), precision=prec, **kw) as s:
        info = s.step(iters)
        U = s.get_u(torch.float64).cpu().numpy()
        hist = s.history()
    return info, U, hist


@pytest.mark.parametrize("defer", [False, True])
def test_small_fp64_trajectory(fc, small, defer):
    d = small
    ref = oracle.solve(d["rp"], d["ci"], d["v"], True, d["U0"], accelerate=True, max_iter=200,
                       step=d["tau"])
    info, U, hist = _solve_gpu(fc, d["rp"], d["ci"], d["v"], d["U0"], d["c"], "fp64", 200,
                               defer_loss=defer)
    assert info.iter == 200
    # the device computed tau = 1/L_thm by its own power iteration
    assert hist["tau"][1] == pytest.approx(d["tau"], rel=1e-10)
    assert np.abs(hist["f"] - ref.f).max() <= 1e-9 * abs(ref.f[0])
    assert np.abs(U - ref.X).max() <= 1e-9


@pytest.mark.parametrize("defer", [False, True])
def test_small_fp32_against_fp64_oracle(fc, small, defer):
    d = small
    U0 = d["U0"].astype(np.float32).astype(np.float64)
    v = d["v"].astype(np.float32).astype(np.float64)
    ref = oracle.solve(d["rp"], d["ci"], v, True, U0, accelerate=True, max_iter=200,
                       step=d["tau"])
    info, U, hist = _solve_gpu(fc, d["rp"], d["ci"], v, U0, d["c"], "fp32", 200, step=d["tau"],
                               defer_loss=defer)
    f_rel = abs(info.f - ref.f[-1]) / abs(ref.f[-1])
    df_ref = ref.f[0] - ref.f[-1]
    df_rel = abs((hist["f"][0] - info.f) - df_ref) / abs(df_ref)
    print(f"fp32 small: f_rel={f_rel:.2e} df_rel={df_rel:.2e} "
          f"max|dU|={np.abs(U - ref.X).max():.2e}")
    assert f_rel <= 1e-4
    assert df_rel <= 1e-5
    assert np.abs(U - ref.X).max() <= 1e-4
    assert np.abs(U.sum(1) - 1).max() <= 1e-6
    assert (U >= 0).all()


def test_uniform_start_is_a_fixed_point(fc, small):
    d = small
    U0 = np.full((d["n"], d["c"]), 1.0 / d["c"])
    info, U, hist = _solve_gpu(fc, d["rp"], d["ci"], d["v"], U0, d["c"], "fp64", 200)
    assert np.abs(U - U0).max() <= 1e-12
    assert np.ptp(hist["f"]) <= 1e-12 * abs(hist["f"][0])
    # U0 = NULL means the same constant start
    S = csr_to_dev(d["rp"], d["ci"], d["v"], torch.float64)
    with fc.Solver(*S, d["c"], None, precision="fp64") as s:
        s.step(5)
        assert np.abs(s.get_u(torch.float64).cpu().numpy() - U0).max() <= 1e-12


@pytest.mark.parametrize("diag", ["stored", "unit"])
@pytest.mark.parametrize("accelerate", [False, True])
@pytest.mark.parametrize("c", [1, 3, 17, 33, 64])
def test_fp64_parity_shapes(fc, diag, accelerate, c):
    defer = (c + accelerate + (diag == "unit")) % 2 == 1   # half the cases deferred
    n = 1000 + 41
    wl = W.er_planted(n, c, 8.0, 0.05, c, val_dtype=torch.float64, u_dtype=torch.float64)
    rp, ci, v, U0 = wl.numpy()
    if diag == "stored":   # store a diagonal to exercise that mode
        A = pins.dense_similarity(rp, ci, v, False, n) + np.diag(np.linspace(0.2, 0.9, n))
        rp, ci, v = pins.csr_from_dense(A)
    tau = 2e-4
    ref = oracle.solve(rp, ci, v, diag == "unit", U0, accelerate=accelerate, max_iter=25, step=tau)
    info, U, hist = _solve_gpu(fc, rp, ci, v, U0, c, "fp64", 25, step=tau, diag=diag,
                               accelerate=accelerate, defer_loss=defer)
    assert np.abs(hist["f"] - ref.f).max() <= 1e-9 * abs(ref.f[0])
    assert np.abs(U - ref.X).max() <= 1e-9


def test_backtracking_fp64_follows_the_oracle(fc):
    wl = W.er_planted(20000, 16, 20.0, 0.05, 4, val_dtype=torch.float64, u_dtype=torch.float64)
    rp, ci, v, U0 = wl.numpy()
    ref = oracle.solve(rp, ci, v, True, U0, accelerate=True, max_iter=40, backtrack=True, L0=10.0)
    info, U, hist = _solve_gpu(fc, rp, ci, v, U0, 16, "fp64", 40, backtrack=True, L0=10.0)
    assert (hist["trials"][1:] == ref.trials[1:]).all()
    assert np.array_equal(hist["tau"][1:], ref.tau[1:])
    assert np.abs(hist["f"] - ref.f).max() <= 1e-9 * abs(ref.f[0])
    assert np.abs(U - ref.X).max() <= 1e-8
    assert info.trials == int(ref.trials[1:].sum())


def test_fp32_replays_the_oracle_step_sequence(fc):
    wl = W.er_planted(20000, 32, 30.0, 0.05, 5)
    rp, ci, v, U0 = wl.numpy()
    ref = oracle.solve(rp, ci, v, True, U0, accelerate=True, max_iter=60, backtrack=True, L0=10.0)
    info, U, hist = _solve_gpu(fc, rp, ci, v, U0, 32, "fp32", 60, step_schedule=ref.tau[1:])
    f_rel = abs(info.f - ref.f[-1]) / abs(ref.f[-1])
    print(f"replay fp32: f_rel={f_rel:.2e} max|dU|={np.abs(U - ref.X).max():.2e}")
    assert f_rel <= 1e-4
    assert np.abs(U - ref.X).max() <= 1e-4
    assert np.abs(U.sum(1) - 1).max() <= 1e-6
    # free-running FP32 backtracking takes (nearly) the same decisions
    info2, U2, hist2 = _solve_gpu(fc, rp, ci, v, U0, 32, "fp32", 60, backtrack=True, L0=10.0)
    agree = np.mean(hist2["tau"][1:] == ref.tau[1:])
    print(f"free-running fp32 backtracking: step agreement {agree:.3f}")
    assert agree >= 0.9


@pytest.mark.parametrize("defer", [False, True])
def test_gpa_loss_stop_example41(fc, defer):
    ex = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "example41.json")))
    S = np.array(ex["S"], dtype=float)
    rp, ci, v = pins.csr_from_dense(S)
    X0 = np.zeros((7, 2))
    X0[:, 0] = 1.0
    ref = oracle.solve(rp, ci, v, False, X0, accelerate=False, max_iter=5000, step=0.1,
                       tol_loss=0.0)
    Sd = csr_to_dev(rp, ci, v, torch.float64)
    with fc.Solver(*Sd, 2, dev(X0, torch.float64), precision="fp64", diag="stored",
                   accelerate=False, step=0.1, tol_loss=0.0, max_iter=5000,
                   defer_loss=defer) as s:
        info = s.solve()
        U = s.get_u(torch.float64).cpu().numpy()
        hist = s.history()
    assert info.stop_reason == 2  # FC_STOP_LOSS
    assert info.iter == ref.iters and info.trials == ref.iters
    assert np.abs(hist["f"] - ref.f).max() <= 1e-12 * abs(ref.f[0])
    assert round(info.f, 2) == ex["scenario2"]["loss"]
    assert np.abs(U - ref.X).max() <= 1e-12
    # scenario 3: the uniform start stops after one iteration, unchanged
    X3 = np.full((7, 2), 0.5)
    with fc.Solver(*Sd, 2, dev(X3, torch.float64), precision="fp64", diag="stored",
                   accelerate=False, step=0.1, tol_loss=0.0, max_iter=50, defer_loss=defer) as s:
        info = s.solve()
        assert info.iter == 1 and info.f == pytest.approx(12.25, abs=1e-12)
        assert np.abs(s.get_u(torch.float64).cpu().numpy() - 0.5).max() == 0.0


def test_pgrad_stop_matches_the_oracle(fc):
    wl = W.er_planted(3000, 8, 10.0, 0.05, 6, val_dtype=torch.float64, u_dtype=torch.float64)
    rp, ci, v, U0 = wl.numpy()
    ref = oracle.solve(rp, ci, v, True, U0, accelerate=True, max_iter=300, backtrack=True,
                       L0=1.0, tol_pgrad=1e-2)
    Sd = csr_to_dev(rp, ci, v, torch.float64)
    with fc.Solver(*Sd, 8, dev(U0, torch.float64), precision="fp64", backtrack=True, L0=1.0,
                   tol_pgrad=1e-2, max_iter=300, check_every=7) as s:
        info = s.solve()
        hist = s.history()
    assert ref.stop_reason == oracle.STOP_PGRAD and info.stop_reason == 3
    assert info.iter == ref.iters
    assert np.allclose(hist["r"][1:], ref.r[1:], rtol=1e-9)


@pytest.mark.parametrize("defer", [False, True])
def test_step_calls_compose_and_are_deterministic(fc, defer):
    wl = W.er_planted(5000, 32, 15.0, 0.05, 7)
    S = wl.to("cuda")
    outs = []
    for split in ([7], [3, 4], [1, 1, 5]):
        with fc.Solver(S.row_ptr, S.col_idx, S.val, 32, S.U0, step=1e-3, defer_loss=defer) as s:
            for k in split:
                s.step(k)
            outs.append((s.get_u().cpu().numpy(), s.info().f, s.history()["f"]))
    for U, f, hf in outs[1:]:
        assert np.array_equal(U, outs[0][0]) and f == outs[0][1]
        assert np.array_equal(hf, outs[0][2])


def test_solve_budget_and_info(fc):
    wl = W.er_planted(3000, 8, 10.0, 0.05, 8)
    S = wl.to("cuda")
    with fc.Solver(S.row_ptr, S.col_idx, S.val, 8, S.U0, step=1e-3, max_iter=13) as s:
        info = s.solve()
        assert info.iter == 13 and info.stop_reason == 1
        again = s.solve()
        assert again.iter == 13
        more = s.step(2)          # fc_step ignores the solve budget
        assert more.iter == 15
        t = [1.0]
        for _ in range(16):
            t.append((1 + math.sqrt(1 + 4 * t[-1] ** 2)) / 2)
        assert more.t == pytest.approx(t[15], rel=1e-14)


@pytest.mark.parametrize("backtrack", [False, True])
def test_history_records_match_the_device_state(fc, tmp_path, backtrack):
    """The JSONL log's inertial weight for iteration K is the weight the
    device reported, after K - 1 iterations, for forming Y_K; its steps and
    losses are the history's."""
    wl = W.er_planted(3000, 8, 10.0, 0.05, 9)
    S = wl.to("cuda")
    kw = dict(backtrack=True) if backtrack else dict(step=1e-3)
    with fc.Solver(S.row_ptr, S.col_idx, S.val, 8, S.U0, **kw) as s:
        betas = []
        for _ in range(12):
            betas.append(s.info().beta)
            s.step(1)
        path = tmp_path / "hist.jsonl"
        assert s.write_history_jsonl(str(path)) == 13
        hist = s.history()
    recs = [json.loads(line) for line in path.read_text().splitlines()]
    for k in range(1, 13):
        assert recs[k]["beta"] == pytest.approx(betas[k - 1], rel=1e-14, abs=1e-300)
        assert recs[k]["tau"] == hist["tau"][k] and recs[k]["f"] == hist["f"][k]
        assert recs[k]["trials"] == hist["trials"][k]


def test_single_row_and_single_cluster(fc):
    rp = np.array([0, 0], dtype=np.int64)
    ci = np.zeros(0, dtype=np.int32)
    v = np.zeros(0)
    U0 = np.array([[0.2, 0.3, 0.5]])
    info, U, hist = _solve_gpu(fc, rp, ci, v, U0, 3, "fp64", 3, step=0.1)
    ref = oracle.solve(rp, ci, v, True, U0, accelerate=True, max_iter=3, step=0.1)
    assert np.abs(U - ref.X).max() <= 1e-14
    wl = W.er_planted(500, 1, 6.0, 0.05, 9, val_dtype=torch.float64, u_dtype=torch.float64)
    rp, ci, v, U0 = wl.numpy()
    info, U, hist = _solve_gpu(fc, rp, ci, v, U0, 1, "fp64", 3, step=0.1)
    assert np.array_equal(U, np.ones_like(U))


def test_nonfinite_start_is_reported(fc):
    wl = W.er_planted(300, 4, 6.0, 0.05, 10)
    U0 = wl.U0.clone()
    U0[3, 1] = float("nan")
    S = wl.to("cuda")
    from paper_2506_04045_amd import _native
    with pytest.raises(_native.FcError) as e:
        fc.Solver(S.row_ptr, S.col_idx, S.val, 4, U0.cuda(), step=1e-3)
    assert e.value.status == _native.FC_ERR_NONFINITE


def test_validation_rejects_bad_matrices(fc):
    from paper_2506_04045_amd import _native
    A = np.array([[0, 1, 0], [0.5, 0, 1], [0, 1, 0]], dtype=float)   # not symmetric
    rp, ci, v = pins.csr_from_dense(A)
    Sd = csr_to_dev(rp, ci, v, torch.float32)
    with pytest.raises(_native.FcError) as e:
        fc.Solver(*Sd, 2, None, validate=True, step=0.1)
    assert e.value.status == _native.FC_ERR_NOT_SYMMETRIC
    B = np.array([[1, 1, 0], [1, 0, 1], [0, 1, 0]], dtype=float)     # stored diagonal
    rp, ci, v = pins.csr_from_dense(B)
    with pytest.raises(_native.FcError) as e:
        fc.Solver(*csr_to_dev(rp, ci, v, torch.float32), 2, None, validate=True, step=0.1)
    assert e.value.status == _native.FC_ERR_INVALID_ARG
    with fc.Solver(*csr_to_dev(rp, ci, v, torch.float32), 2, None, validate=True, diag="stored",
                   step=0.1) as s:
        assert s.step(2).iter == 2
    # malformed structure: row_ptr is checked on the host before any entry is
    # read, so none of these reaches the device's entry checks
    C = np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=float)
    rp, ci, v = pins.csr_from_dense(C)
    for bad_rp in ([0, 2, 1_000_000_000, 6], [0, 3, 2, 6], [1, 2, 4, 6], [0, 2, 4, 5]):
        Sd = csr_to_dev(np.array(bad_rp, dtype=np.int64), ci, v, torch.float32)
        with pytest.raises(_native.FcError) as e:
            fc.Solver(*Sd, 2, None, validate=True, step=0.1)
        assert e.value.status == _native.FC_ERR_NOT_SYMMETRIC, bad_rp
        assert "row_ptr" in str(e.value)
    bad_ci = ci.copy()
    bad_ci[3] = 7                                                      # column out of range
    with pytest.raises(_native.FcError) as e:
        fc.Solver(*csr_to_dev(rp, bad_ci, v, torch.float32), 2, None, validate=True, step=0.1)
    assert e.value.status == _native.FC_ERR_NOT_SYMMETRIC and "col_idx" in str(e.value)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_hub_rows_take_the_chunked_path(fc, prec):
    """Rows longer than the chunk threshold (2,048 nonzeros) are summed in
    chunks and combined per row; the solve must still follow the oracle."""
    from tests.gpu_util import star_plus_er
    rp, ci, v = star_plus_er(6000, 4.0, 12)
    assert np.diff(rp).max() > 2 * 2048
    n, c = 6000, 16
    U0 = pins.random_simplex_rows(n, c, np.random.default_rng(12))
    if prec == "fp32":
        v = v.astype(np.float32).astype(np.float64)
        U0 = U0.astype(np.float32).astype(np.float64)
    ref = oracle.solve(rp, ci, v, True, U0, accelerate=True, max_iter=30, step=2e-4)
    info, U, hist = _solve_gpu(fc, rp, ci, v, U0, c, prec, 30, step=2e-4)
    tol = 1e-9 if prec == "fp64" else 1e-4
    assert np.abs(U - ref.X).max() <= tol
    assert abs(info.f - ref.f[-1]) <= tol * abs(ref.f[-1])


@pytest.mark.parametrize("backtrack", [False, True])
def test_checkpoint_resume_is_bitwise(fc, backtrack):
    wl = W.er_planted(4000, 16, 12.0, 0.05, 13)
    S = wl.to("cuda")
    kw = dict(backtrack=True, L0=10.0) if backtrack else dict(step=1e-3)
    with fc.Solver(S.row_ptr, S.col_idx, S.val, 16, S.U0, **kw) as a:
        a.step(25)
        U_ref, f_ref = a.get_u().cpu().numpy(), a.info().f
        h_ref = a.history()
    with fc.Solver(S.row_ptr, S.col_idx, S.val, 16, S.U0, **kw) as b:
        b.step(11)
        state = b.get_state()
    with fc.Solver(S.row_ptr, S.col_idx, S.val, 16, None, **kw) as c:
        c.set_state(state)
        assert c.info().iter == 11
        c.step(14)
        assert np.array_equal(c.get_u().cpu().numpy(), U_ref) and c.info().f == f_ref
        assert np.array_equal(c.history()["f"], h_ref["f"])
    from paper_2506_04045_amd import _native
    with fc.Solver(S.row_ptr, S.col_idx, S.val, 8, None, step=1e-3) as d:
        with pytest.raises(_native.FcError):
            d.set_state(state)


@pytest.mark.parametrize("kw", [dict(step=1e-3), dict(backtrack=True), dict(defer_loss=True, step=1e-3),
                                dict(single_pass=True, step=1e-3), dict(precision="mixed", step=1e-3)],
                         ids=["fixed", "backtracking", "deferred", "single_pass", "mixed"])
def test_checkpoint_bytes_depend_only_on_the_inputs(fc, kw):
    """Two solvers of the same instance, on buffers that held other data
    before, give byte-identical checkpoints: at the start (slots not yet
    written) and after some iterations (padded columns: c = 3, or 6 in mixed
    precision)."""
    c = 6 if kw.get("precision") == "mixed" else 3   # mixed precision needs c >= 5
    wl = W.chung_lu_planted(3000, c, 15.0, 2.1, 2_000.0, 0.05, 17).to("cuda")
    junk = torch.full((1 << 22,), float("nan"), device="cuda")   # recycled memory
    del junk
    states = []
    for _ in range(2):
        with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, c, wl.U0, reorder="degree", **kw) as s:
            first = s.get_state()
            s.step(6)
            states.append((first, s.get_state()))
        filler = torch.randn(1 << 22, device="cuda")   # the next solver reuses dirty memory
        del filler
    assert states[0][0] == states[1][0]
    assert states[0][1] == states[1][1]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_power_law_instance_follows_the_oracle(fc, prec):
    wl = W.chung_lu_planted(20000, 16, 20.0, 2.1, 50_000.0, 0.05, 5,
                            val_dtype=torch.float64, u_dtype=torch.float64)
    rp, ci, v, U0 = wl.numpy()
    if prec == "fp32":
        v = v.astype(np.float32).astype(np.float64)
        U0 = U0.astype(np.float32).astype(np.float64)
    spec, _ = oracle.spectral_norm(rp, ci, v, True)
    tau = 20.0 / oracle.lipschitz_bound(spec, wl.n)
    ref = oracle.solve(rp, ci, v, True, U0, accelerate=True, max_iter=40, step=tau)
    info, U, hist = _solve_gpu(fc, rp, ci, v, U0, 16, prec, 40, step=tau)
    tol = 1e-9 if prec == "fp64" else 1e-4
    print(f"power-law {prec}: f_rel={abs(info.f - ref.f[-1]) / abs(ref.f[-1]):.2e} "
          f"max|dU|={np.abs(U - ref.X).max():.2e}")
    assert np.abs(U - ref.X).max() <= tol
    assert abs(info.f - ref.f[-1]) <= tol * abs(ref.f[-1])


# --------------------------------------------------------------------------
# degree relabelling (internal renumbering of the articles)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_degree_relabelling_follows_the_oracle(fc, prec):
    """With the articles renumbered by degree inside the solver, the iterate
    handed back (in the caller's order) still follows the oracle run on the
    caller's numbering, and agrees with the solver run without renumbering."""
    wl = W.chung_lu_planted(20000, 16, 20.0, 2.1, 50_000.0, 0.05, 7,
                            val_dtype=torch.float64, u_dtype=torch.float64)
    rp, ci, v, U0 = wl.numpy()
    if prec != "fp64":
        v = v.astype(np.float32).astype(np.float64)
        U0 = U0.astype(np.float32).astype(np.float64)
    v_ref = v.astype(np.float16).astype(np.float64) if prec == "mixed" else v
    spec, _ = oracle.spectral_norm(rp, ci, v_ref, True)
    tau = 20.0 / oracle.lipschitz_bound(spec, wl.n)
    ref = oracle.solve(rp, ci, v_ref, True, U0, accelerate=True, max_iter=40, step=tau)
    info, U, hist = _solve_gpu(fc, rp, ci, v, U0, 16, prec, 40, step=tau, reorder="degree")
    info0, U_plain, _ = _solve_gpu(fc, rp, ci, v, U0, 16, prec, 40, step=tau)
    tol = {"fp64": 1e-9, "fp32": 1e-4, "mixed": 5e-3}[prec]
    du = np.abs(U - ref.X).max()
    print(f"relabelled {prec}: f_rel={abs(info.f - ref.f[-1]) / abs(ref.f[-1]):.2e} "
          f"max|dU|={du:.2e} max|dU| vs unrelabelled={np.abs(U - U_plain).max():.2e}")
    assert du <= tol
    assert abs(info.f - ref.f[-1]) <= (1e-9 if prec == "fp64" else 1e-4) * abs(ref.f[-1])
    assert np.abs(U - U_plain).max() <= {"fp64": 1e-12, "fp32": 1e-5, "mixed": 1e-3}[prec]
    assert np.abs(U.sum(1) - 1).max() <= 1e-6


def test_degree_relabelling_checkpoints(fc):
    wl = W.chung_lu_planted(6000, 8, 20.0, 2.1, 5_000.0, 0.05, 8).to("cuda")
    kw = dict(step=1e-4, reorder="degree")
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, wl.U0, **kw) as a:
        a.step(20)
        U_ref, f_ref = a.get_u().cpu().numpy(), a.info().f
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, wl.U0, **kw) as b:
        b.step(9)
        state = b.get_state()
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, None, **kw) as c:
        c.set_state(state)
        c.step(11)
        assert np.array_equal(c.get_u().cpu().numpy(), U_ref) and c.info().f == f_ref
    from paper_2506_04045_amd import _native
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, None, step=1e-4) as d:
        with pytest.raises(_native.FcError):
            d.set_state(state)


def test_degree_relabelling_with_hub_rows_and_empty_rows(fc):
    from tests.gpu_util import star_plus_er
    rp, ci, v = star_plus_er(6000, 3.0, 21, hub_frac=0.9)
    deg = np.diff(rp)
    assert deg.max() > 2 * 2048 and (deg == 0).any()
    n, c = 6000, 8
    U0 = pins.random_simplex_rows(n, c, np.random.default_rng(21))
    ref = oracle.solve(rp, ci, v, True, U0, accelerate=True, max_iter=20, step=2e-4)
    info, U, _ = _solve_gpu(fc, rp, ci, v, U0, c, "fp64", 20, step=2e-4, reorder="degree",
                            validate=True)
    assert np.abs(U - ref.X).max() <= 1e-9
    assert abs(info.f - ref.f[-1]) <= 1e-9 * abs(ref.f[-1])


def test_medium_config_replays_500_backtracking_iterations_fp32(fc):
    """The n = 1e6, c = 32 configuration (ER degree 30, 3e7 nonzeros) over its
    500 iterations: the FP64 oracle's run of backtracking FISTA (stored by
    tests/golden/make_medium_replay.py, which calls only the oracle and the
    workload generator) replayed by the FP32 solver through its accepted
    steps.  The whole loss history, the decrease, Xbar_500 at the stored
    sample rows and the row sums are compared."""
    from tests.golden.make_medium_replay import OUT, fingerprint
    gold = json.load(open(OUT))
    wl = W.config_medium(seed=0)
    rp, ci, v, U0 = wl.numpy()
    assert fingerprint(rp, ci, v, U0) == gold["instance"], "the seeded instance changed"
    K = gold["iters"]
    tau = np.asarray(gold["tau"])
    f_ref = np.asarray(gold["f"])
    assert K == 500 and sum(gold["trials"]) > K      # rejected trials happened
    info, U, hist = _solve_gpu(fc, rp, ci, v, U0, 32, "fp32", K, step_schedule=tau)
    assert info.iter == K
    rows = np.asarray(gold["rows"])
    X_ref = np.asarray(gold["X_rows"])
    f_hist_rel = np.abs(hist["f"] - f_ref).max() / abs(f_ref[-1])
    df = f_ref[0] - f_ref[-1]
    df_rel = abs((hist["f"][0] - info.f) - df) / abs(df)
    du = np.abs(U[rows] - X_ref).max()
    print(f"medium replay fp32, {K} iterations: f history rel {f_hist_rel:.2e} "
          f"df_rel={df_rel:.2e} (df={df:.6e}) max|dU| on {rows.size} rows {du:.2e}")
    assert f_hist_rel <= 1e-4
    assert df_rel <= 1e-5
    assert du <= 1e-4
    assert np.abs(U.sum(1) - 1).max() <= 1e-6 and (U >= 0).all()


def test_medium_config_backtracking_decisions_fp64(fc):
    """The same instance in FP64, free-running: the device's backtracking takes
    the oracle's decisions (trials and accepted steps) over the first 40 stored
    iterations."""
    from tests.golden.make_medium_replay import OUT
    gold = json.load(open(OUT))
    wl = W.config_medium(seed=0)
    rp, ci, v, U0 = wl.numpy()
    K = 40
    info, U, hist = _solve_gpu(fc, rp, ci, v, U0, 32, "fp64", K, backtrack=True,
                               L0=gold["L0"])
    assert (hist["trials"][1:] == np.asarray(gold["trials"][:K])).all()
    assert np.array_equal(hist["tau"][1:], np.asarray(gold["tau"][:K]))
    f_ref = np.asarray(gold["f"][:K + 1])
    assert np.abs(hist["f"] - f_ref).max() <= 1e-9 * abs(f_ref[0])


# --------------------------------------------------------------------------
# deferred loss evaluation
# --------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_deferred_loss_follows_the_oracle_and_the_default_mode(fc, prec):
    wl = W.chung_lu_planted(20000, 16, 20.0, 2.1, 50_000.0, 0.05, 9,
                            val_dtype=torch.float64, u_dtype=torch.float64)
    rp, ci, v, U0 = wl.numpy()
    if prec != "fp64":
        v = v.astype(np.float32).astype(np.float64)
        U0 = U0.astype(np.float32).astype(np.float64)
    v_ref = v.astype(np.float16).astype(np.float64) if prec == "mixed" else v
    spec, _ = oracle.spectral_norm(rp, ci, v_ref, True)
    tau = 20.0 / oracle.lipschitz_bound(spec, wl.n)
    ref = oracle.solve(rp, ci, v_ref, True, U0, accelerate=True, max_iter=30, step=tau)
    info, U, hist = _solve_gpu(fc, rp, ci, v, U0, 16, prec, 30, step=tau, defer_loss=True,
                               reorder="degree")
    info0, U0g, hist0 = _solve_gpu(fc, rp, ci, v, U0, 16, prec, 30, step=tau, reorder="degree")
    tol = {"fp64": 1e-9, "fp32": 1e-4, "mixed": 1e-4}[prec]
    f_err = np.abs(hist["f"] - ref.f).max() / abs(ref.f[-1])
    print(f"deferred {prec}: history f_rel {f_err:.2e} max|dU| {np.abs(U - ref.X).max():.2e} "
          f"vs default mode {np.abs(U - U0g).max():.2e}")
    assert info.iter == 30 and len(hist["f"]) == 31
    assert f_err <= tol
    assert np.abs(U - ref.X).max() <= {"fp64": 1e-9, "fp32": 1e-4, "mixed": 5e-3}[prec]
    assert np.abs(U - U0g).max() <= {"fp64": 1e-12, "fp32": 1e-5, "mixed": 1e-3}[prec]
    assert np.abs(hist["f"] - hist0["f"]).max() <= {"fp64": 1e-12, "fp32": 1e-6,
                                                    "mixed": 1e-6}[prec] * abs(ref.f[0])
    assert info.f == hist["f"][-1] and info.f_prev == hist["f"][-2]


def test_deferred_loss_checkpoints_and_rules(fc):
    wl = W.er_planted(4000, 16, 12.0, 0.05, 13).to("cuda")
    kw = dict(step=1e-3, defer_loss=True)
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 16, wl.U0, **kw) as a:
        a.step(21)
        U_ref, f_ref, h_ref = a.get_u().cpu().numpy(), a.info().f, a.history()["f"]
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 16, wl.U0, **kw) as b:
        b.step(8)
        state = b.get_state()
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 16, None, **kw) as c:
        c.set_state(state)
        c.step(13)
        assert np.array_equal(c.get_u().cpu().numpy(), U_ref) and c.info().f == f_ref
        assert np.array_equal(c.history()["f"], h_ref)
    from paper_2506_04045_amd import _native
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 16, None, step=1e-3) as d:
        with pytest.raises(_native.FcError):
            d.set_state(state)
    with pytest.raises(_native.FcError):   # backtracking needs each trial's loss
        fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 16, None, backtrack=True, defer_loss=True)
    with fc.Server() as sv:                # the server evaluates every loss in its tick
        with pytest.raises(_native.FcError):
            sv.submit(1, wl.row_ptr, wl.col_idx, wl.val, 16, wl.U0, defer_loss=True)
