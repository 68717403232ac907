"""Single-pass iteration (fc_options.single_pass) against the FP64 oracle.

The mode computes the same iteration as Alg. 4 (and Alg. 2/3 for GPA) --
the projected gradient step at the extrapolated point Y_n, the next
extrapolated point -- with S applied once per iteration to the stored Y_n,
and evaluates the structured loss of Alg. 3 only when the iterate is read
out at the end of an fc_step call.  So iterates and read-out losses are
compared with the oracle's, at the tolerances of the default mode:
* FP64: losses within 1e-9 relative, iterates within 1e-9;
* FP32 against the FP64 oracle: loss within 1e-4 relative, the decrease
  within 1e-5 relative, iterates within 1e-4, rows summing to 1 within 1e-6.
"""

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests import pins
from tests.gpu_util import csr_to_dev, dev, star_plus_er

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fc():
    import paper_2506_04045_amd as fc
    fc.library_path()
    return fc


@pytest.fixture(scope="module")
def small():
    wl = W.config_small_fp64(seed=0)
    rp, ci, v, U0 = wl.numpy()
    spec, _ = oracle.spectral_norm(rp, ci, v, True)
    return dict(rp=rp, ci=ci, v=v, U0=U0, n=wl.n, c=wl.c,
                tau=1.0 / oracle.lipschitz_bound(spec, wl.n))


def _solver(fc, rp, ci, v, U0, c, prec, **kw):
    vd = torch.float64 if prec == "fp64" else torch.float32
    S = csr_to_dev(rp, ci, v, vd)
    return fc.Solver(*S, c, dev(U0, vd), precision=prec, **kw), S


def test_fp64_trajectory_and_read_outs(fc, small):
    """200 FISTA iterations at tau = 1/L_thm in three fc_step calls: the
    iterate and the loss at every read-out follow the oracle."""
    d = small
    ref = oracle.solve(d["rp"], d["ci"], d["v"], True, d["U0"], accelerate=True, max_iter=200,
                       step=d["tau"])
    s, _ = _solver(fc, d["rp"], d["ci"], d["v"], d["U0"], d["c"], "fp64", single_pass=True)
    with s:
        for upto in (37, 100, 200):
            info = s.step(upto - s.info().iter)
            assert info.iter == upto
            assert abs(info.f - ref.f[upto]) <= 1e-9 * abs(ref.f[0])
        U = s.get_u(torch.float64).cpu().numpy()
        hist = s.history()
    assert np.abs(U - ref.X).max() <= 1e-9
    # losses only at read-outs; steps and gradient-mapping norms everywhere
    known = np.flatnonzero(np.isfinite(hist["f"]))
    assert list(known) == [0, 37, 100, 200]
    # the device formed tau = 1/L_thm by its own power iteration
    assert np.allclose(hist["tau"][1:], ref.tau[1:], rtol=1e-10, atol=0)
    assert np.abs(hist["r"][1:] - ref.r[1:]).max() <= 1e-8 * ref.r[1:].max()


def test_fp32_against_fp64_oracle(fc, small):
    d = small
    U0 = d["U0"].astype(np.float32).astype(np.float64)
    v = d["v"].astype(np.float32).astype(np.float64)
    ref = oracle.solve(d["rp"], d["ci"], v, True, U0, accelerate=True, max_iter=200,
                       step=d["tau"])
    s, _ = _solver(fc, d["rp"], d["ci"], v, U0, d["c"], "fp32", single_pass=True,
                   step=d["tau"])
    with s:
        f0 = s.info().f
        info = s.step(200)
        U = s.get_u(torch.float64).cpu().numpy()
    f_rel = abs(info.f - ref.f[-1]) / abs(ref.f[-1])
    df_ref = ref.f[0] - ref.f[-1]
    df_rel = abs((f0 - info.f) - df_ref) / abs(df_ref)
    du = np.abs(U - ref.X).max()
    print(f"single-pass fp32 small: f_rel={f_rel:.2e} df_rel={df_rel:.2e} max|dU|={du:.2e}")
    assert f_rel <= 1e-4 and df_rel <= 1e-5 and du <= 1e-4
    assert np.abs(U.sum(1) - 1).max() <= 1e-6 and (U >= 0).all()


@pytest.mark.parametrize("diag", ["stored", "unit"])
@pytest.mark.parametrize("accelerate", [False, True])
@pytest.mark.parametrize("c", [1, 3, 17, 33, 64])
def test_fp64_parity_shapes(fc, diag, accelerate, c):
    n = 1000 + 41
    wl = W.er_planted(n, c, 8.0, 0.05, c, val_dtype=torch.float64, u_dtype=torch.float64)
    rp, ci, v, U0 = wl.numpy()
    if diag == "stored":
        A = pins.dense_similarity(rp, ci, v, False, n) + np.diag(np.linspace(0.2, 0.9, n))
        rp, ci, v = pins.csr_from_dense(A)
    tau = 2e-4
    ref = oracle.solve(rp, ci, v, diag == "unit", U0, accelerate=accelerate, max_iter=25, step=tau)
    s, _ = _solver(fc, rp, ci, v, U0, c, "fp64", step=tau, diag=diag, accelerate=accelerate,
                   single_pass=True)
    with s:
        info = s.step(25)
        U = s.get_u(torch.float64).cpu().numpy()
    assert abs(info.f - ref.f[-1]) <= 1e-9 * abs(ref.f[0])
    assert np.abs(U - ref.X).max() <= 1e-9


def _star_or_power_law(kind):
    if kind == "star":     # one hub row of 0.9 n entries, empty rows
        rp, ci, v = star_plus_er(6000, 3.0, 21, hub_frac=0.9)
        deg = np.diff(rp)
        assert deg.max() > 2 * 2048 and (deg == 0).any()
        return rp, ci, v
    wl = W.chung_lu_planted(6000, 8, 20.0, 2.1, 20_000.0, 0.05, 22, val_dtype=torch.float64)
    rp, ci, v, _ = wl.numpy()
    deg = np.diff(rp)      # medium rows (65..2048 entries) and chunked heavy rows
    assert ((deg > 64) & (deg <= 2048)).sum() > 10 and (deg > 2048).any()
    return rp, ci, v


@pytest.mark.parametrize("kind", ["star", "power_law"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_long_rows_empty_rows_and_relabelling(fc, prec, kind):
    """Rows longer than the light limit come from the pre-pass (medium rows
    whole, hub rows in chunks); empty rows; degree relabelling."""
    rp, ci, v = _star_or_power_law(kind)
    n, c = 6000, 8
    U0 = pins.random_simplex_rows(n, c, np.random.default_rng(21))
    if prec == "fp32":
        v = v.astype(np.float32).astype(np.float64)
        U0 = U0.astype(np.float32).astype(np.float64)
    ref = oracle.solve(rp, ci, v, True, U0, accelerate=True, max_iter=20, step=2e-4)
    tol_u, tol_f = (1e-9, 1e-9) if prec == "fp64" else (1e-5, 1e-6)
    for reorder in ("none", "degree"):
        s, _ = _solver(fc, rp, ci, v, U0, c, prec, step=2e-4, reorder=reorder, single_pass=True)
        with s:
            info = s.step(20)
            U = s.get_u(torch.float64).cpu().numpy()
        assert np.abs(U - ref.X).max() <= tol_u, reorder
        assert abs(info.f - ref.f[-1]) <= tol_f * abs(ref.f[-1]), reorder


def test_matches_the_default_mode_on_a_power_law_instance(fc):
    wl = W.chung_lu_planted(20000, 16, 20.0, 2.1, 50_000.0, 0.05, 9,
                            val_dtype=torch.float64, u_dtype=torch.float64)
    rp, ci, v, U0 = wl.numpy()
    spec, _ = oracle.spectral_norm(rp, ci, v, True)
    tau = 20.0 / oracle.lipschitz_bound(spec, wl.n)
    ref = oracle.solve(rp, ci, v, True, U0, accelerate=True, max_iter=30, step=tau)
    out = {}
    for single in (False, True):
        s, _ = _solver(fc, rp, ci, v, U0, 16, "fp64", step=tau, reorder="degree",
                       single_pass=single)
        with s:
            out[single] = (s.step(30).f, s.get_u(torch.float64).cpu().numpy())
    assert np.abs(out[True][1] - out[False][1]).max() <= 1e-12
    assert abs(out[True][0] - ref.f[-1]) <= 1e-9 * abs(ref.f[0])
    assert np.abs(out[True][1] - ref.X).max() <= 1e-9


def test_gradient_mapping_stop(fc, small):
    d = small
    ref = oracle.solve(d["rp"], d["ci"], d["v"], True, d["U0"], accelerate=True, max_iter=400,
                       step=d["tau"], tol_pgrad=0.5)
    assert ref.stop_reason == oracle.STOP_PGRAD and ref.iters < 400
    s, _ = _solver(fc, d["rp"], d["ci"], d["v"], d["U0"], d["c"], "fp64", tol_pgrad=0.5,
                   max_iter=400, step=d["tau"], single_pass=True)
    with s:
        info = s.solve()
        U = s.get_u(torch.float64).cpu().numpy()
    assert info.iter == ref.iters and info.stop_reason == 3   # FC_STOP_PGRAD
    assert abs(info.f - ref.f[-1]) <= 1e-9 * abs(ref.f[0])
    assert np.abs(U - ref.X).max() <= 1e-9


def test_checkpoint_resume_is_bitwise(fc):
    wl = W.er_planted(5000, 8, 12.0, 0.05, 31).to("cuda")
    kw = dict(step=1e-3, single_pass=True)
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, wl.U0, **kw) as a:
        a.step(21)
        U_ref, f_ref = a.get_u().cpu().numpy(), a.info().f
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, wl.U0, **kw) as b:
        b.step(8)
        state = b.get_state()
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, None, **kw) as c:
        c.set_state(state)
        c.step(13)
        assert np.array_equal(c.get_u().cpu().numpy(), U_ref) and c.info().f == f_ref
    from paper_2506_04045_amd import _native
    with fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, None, step=1e-3) as d:
        with pytest.raises(_native.FcError):
            d.set_state(state)


def test_unsupported_combinations_are_rejected(fc):
    from paper_2506_04045_amd import _native
    wl = W.er_planted(2000, 8, 10.0, 0.05, 3).to("cuda")
    for kw in (dict(backtrack=True), dict(precision="mixed"), dict(tol_loss=0.0)):
        with pytest.raises(_native.FcError):
            fc.Solver(wl.row_ptr, wl.col_idx, wl.val, 8, wl.U0, single_pass=True, **kw)
    with fc.Server() as sv:
        with pytest.raises(_native.FcError):
            sv.submit(1, wl.row_ptr, wl.col_idx, wl.val, 8, wl.U0, single_pass=True)
