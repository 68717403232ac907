"""Kernel-level parity of the HIP path against the FP64 oracle, called through
the C ABI: simplex projection, sparse product, Gram matrix, structured
objective and power iteration.

Tolerances: FP64 kernels agree to rounding (1e-12 relative); FP32 kernels
to a normwise relative error of 1e-5, computed against the oracle run in
double on the same FP32-representable inputs.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests import pins
from tests.gpu_util import csr_to_dev, dev, normwise, star_plus_er

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fc():
    import paper_2506_04045_amd as fc
    fc.library_path()
    return fc


# --------------------------------------------------------------------------
# projection onto the simplex
# --------------------------------------------------------------------------

@pytest.mark.parametrize("c", [1, 2, 3, 5, 8, 13, 16, 17, 31, 32, 33, 63, 64])
def test_project_fp64_matches_duchi(fc, c):
    rng = np.random.default_rng(c)
    rows = 1000 + 37   # several tiles and a ragged tail
    V = rng.normal(size=(rows, c)) * np.where(rng.random((rows, 1)) < 0.3, 10.0, 1.0)
    V[::7, :] = V[::7, :1]                 # rows of ties
    ref = oracle.project_columns(V)
    out = fc.project(dev(V, torch.float64)).cpu().numpy()
    assert np.abs(out - ref).max() <= 1e-13 * max(1.0, np.abs(V).max())
    assert np.abs(out.sum(1) - 1).max() <= 1e-13 * c


@pytest.mark.parametrize("c", [1, 3, 8, 32, 64])
def test_project_fp32_and_leading_dimension(fc, c):
    rng = np.random.default_rng(100 + c)
    rows, ld = 777, c + 5
    V = rng.normal(size=(rows, ld)).astype(np.float32)
    Vt = dev(V)
    out = fc.project(Vt, c=c).cpu().numpy()
    ref = oracle.project_columns(V[:, :c].astype(np.float64))
    assert np.abs(out[:, :c] - ref).max() <= 1e-6
    assert np.abs(out[:, :c].sum(1) - 1).max() <= 1e-6
    # untouched columns beyond c keep their (uninitialised) slot: compare
    # in-place use instead, which must leave them alone
    Vi = dev(V)
    fc.project(Vi, out=Vi, c=c)
    got = Vi.cpu().numpy()
    assert np.array_equal(got[:, c:], V[:, c:])
    assert np.abs(got[:, :c] - ref).max() <= 1e-6


def test_project_kkt_on_simplex_points_and_empty(fc):
    rng = np.random.default_rng(5)
    X = pins.random_simplex_rows(300, 7, rng)
    out = fc.project(dev(X, torch.float64)).cpu().numpy()
    assert np.abs(out - X).max() <= 1e-15
    empty = torch.empty(0, 4, dtype=torch.float32, device="cuda")
    assert fc.project(empty).numel() == 0


# --------------------------------------------------------------------------
# sparse product, Gram, objective
# --------------------------------------------------------------------------

def _instance(n=3001, c=8, seed=0):
    wl = W.er_planted(n, c, 12.0, 0.05, seed, val_dtype=torch.float64, u_dtype=torch.float64)
    return wl.numpy()


@pytest.mark.parametrize("diag", ["unit", "stored"])
@pytest.mark.parametrize("c", [1, 3, 8, 16, 32, 64])
def test_spmm_fp64_and_fp32(fc, diag, c):
    rp, ci, v, _ = _instance(2003, 4, seed=c)
    rng = np.random.default_rng(c)
    U = rng.random((rp.shape[0] - 1, c))
    ref = oracle.x_s(rp, ci, v, diag == "unit", U)
    z64 = fc.spmm(*csr_to_dev(rp, ci, v, torch.float64), dev(U, torch.float64), diag=diag)
    assert normwise(z64.cpu().numpy(), ref) <= 1e-13
    U32 = U.astype(np.float32)
    v32 = v.astype(np.float32)
    ref32 = oracle.x_s(rp, ci, v32.astype(np.float64), diag == "unit", U32.astype(np.float64))
    z32 = fc.spmm(*csr_to_dev(rp, ci, v32, torch.float32), dev(U32), diag=diag)
    assert normwise(z32.cpu().numpy(), ref32) <= 1e-5


def test_spmm_heavy_row_and_empty_rows(fc):
    rp, ci, v = star_plus_er(5000, 3.0, 1, hub_frac=0.9)
    deg = np.diff(rp)
    assert deg.max() >= 4000 and (deg == 0).sum() > 0
    U = np.random.default_rng(2).random((5000, 32))
    ref = oracle.x_s(rp, ci, v, True, U)
    z = fc.spmm(*csr_to_dev(rp, ci, v, torch.float64), dev(U, torch.float64)).cpu().numpy()
    assert normwise(z, ref) <= 1e-13
    z32 = fc.spmm(*csr_to_dev(rp, ci, v.astype(np.float32), torch.float32),
                  dev(U.astype(np.float32))).cpu().numpy()
    ref32 = oracle.x_s(rp, ci, v.astype(np.float32).astype(np.float64), True,
                       U.astype(np.float32).astype(np.float64))
    assert normwise(z32, ref32) <= 1e-5
    # the hub row on its own
    assert np.abs(z32[0] - ref32[0]).max() <= 1e-5 * np.abs(ref32[0]).max()


def test_spmm_without_nonzeros(fc):
    n, c = 100, 8
    rp = np.zeros(n + 1, dtype=np.int64)
    ci = np.zeros(0, dtype=np.int32)
    v = np.zeros(0)
    U = np.random.default_rng(0).random((n, c))
    z = fc.spmm(dev(rp), dev(ci, torch.int32), dev(v, torch.float64), dev(U, torch.float64))
    assert np.array_equal(z.cpu().numpy(), U)
    z0 = fc.spmm(dev(rp), dev(ci, torch.int32), dev(v, torch.float64), dev(U, torch.float64),
                 diag="stored")
    assert np.array_equal(z0.cpu().numpy(), np.zeros_like(U))


@pytest.mark.parametrize("c", [1, 2, 8, 16, 20, 32, 64])
@pytest.mark.parametrize("n", [1, 15, 1000, 4099])
def test_gram(fc, c, n):
    rng = np.random.default_rng(n + c)
    U = pins.random_simplex_rows(n, c, rng)
    ref = oracle.share(U)
    G = fc.gram(dev(U, torch.float64))
    assert normwise(G, ref) <= 1e-14
    U32 = U.astype(np.float32)
    G32 = fc.gram(dev(U32))
    assert normwise(G32, oracle.share(U32.astype(np.float64))) <= 1e-6
    assert np.allclose(G32, G32.T, rtol=0, atol=0)


@pytest.mark.parametrize("diag", ["unit", "stored"])
def test_objective(fc, diag):
    rp, ci, v, U0 = _instance(3001, 8, seed=3)
    unit = diag == "unit"
    ref = oracle.loss(rp, ci, v, unit, U0)
    f64 = fc.objective(*csr_to_dev(rp, ci, v, torch.float64), dev(U0, torch.float64), diag=diag)
    assert abs(f64 - ref) <= 1e-12 * abs(ref)
    U32 = U0.astype(np.float32)
    v32 = v.astype(np.float32)
    ref32 = oracle.loss(rp, ci, v32.astype(np.float64), unit, U32.astype(np.float64))
    f32 = fc.objective(*csr_to_dev(rp, ci, v32, torch.float32), dev(U32), diag=diag)
    assert abs(f32 - ref32) <= 1e-6 * abs(ref32)


def test_objective_example41(fc):
    import json
    import os
    ex = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "example41.json")))
    S = np.array(ex["S"], dtype=float)
    rp, ci, v = pins.csr_from_dense(S)
    X3 = np.ascontiguousarray(np.array(ex["scenario3"]["X"]).T)
    f = fc.objective(*csr_to_dev(rp, ci, v, torch.float64), dev(X3, torch.float64), diag="stored")
    assert f == pytest.approx(12.25, abs=1e-12)
    rpu, ciu, vu = pins.csr_from_dense(S, drop_diag=True)
    X1 = np.ascontiguousarray(np.array(ex["scenario1"]["X"]).T)
    fu = fc.objective(*csr_to_dev(rpu, ciu, vu, torch.float64), dev(X1, torch.float64), diag="unit")
    assert round(fu, 2) == ex["scenario1"]["loss"]


@pytest.mark.parametrize("diag", ["unit", "stored"])
def test_spectral_norm(fc, diag):
    rp, ci, v, _ = W.config_small_fp64().numpy()
    ref, _ = oracle.spectral_norm(rp, ci, v, diag == "unit")
    got, it = fc.spectral_norm(*csr_to_dev(rp, ci, v, torch.float64), diag=diag)
    assert got == pytest.approx(ref, rel=1e-9)
    got32, _ = fc.spectral_norm(*csr_to_dev(rp, ci, v.astype(np.float32), torch.float32), diag=diag)
    assert got32 == pytest.approx(ref, rel=1e-6)


def test_spmm_power_law_rows_of_every_class(fc):
    """A power-law pattern has short rows (two-slot teams), medium rows
    (65-2,048 nonzeros, whole-wave teams) and hub rows (chunked)."""
    wl = W.chung_lu_planted(20000, 16, 20.0, 2.1, 50_000.0, 0.05, 3, val_dtype=torch.float64)
    rp, ci, v, _ = wl.numpy()
    deg = np.diff(rp)
    assert (deg <= 64).any() and ((deg > 64) & (deg <= 2048)).any() and (deg > 2048).any()
    U = np.random.default_rng(4).random((wl.n, 16))
    ref = oracle.x_s(rp, ci, v, True, U)
    z = fc.spmm(*csr_to_dev(rp, ci, v, torch.float64), dev(U, torch.float64)).cpu().numpy()
    assert normwise(z, ref) <= 1e-13
    v32, U32 = v.astype(np.float32), U.astype(np.float32)
    ref32 = oracle.x_s(rp, ci, v32.astype(np.float64), True, U32.astype(np.float64))
    z32 = fc.spmm(*csr_to_dev(rp, ci, v32, torch.float32), dev(U32)).cpu().numpy()
    assert normwise(z32, ref32) <= 1e-5


def test_gather_probe_runs_and_checks_its_arguments(fc):
    """fc_gather_probe (a memory-system measurement, not a step of the
    method): it times a flat pass of row gathers and rejects bad sizes."""
    from paper_2506_04045_amd import _native as N
    n = 50_000
    U = torch.rand(n, 32, device="cuda")
    col = torch.randint(0, n, (400_000,), device="cuda", dtype=torch.int32)
    ms = fc.gather_probe(col, U, wg_per_cu=4, reps=3)
    assert 0.0 < ms < 1000.0
    ms_bf16 = fc.gather_probe(col, U.to(torch.bfloat16), wg_per_cu=4, reps=3)
    assert 0.0 < ms_bf16 < 1000.0
    lib = N.load()
    out = ctypes.c_double(0.0)
    for nnz, rows, rb, w, reps in ((0, n, 128, 4, 1), (10, 0, 128, 4, 1), (10, n, 96, 4, 1),
                                   (10, n, 128, 0, 1), (10, n, 128, 65, 1), (10, n, 128, 4, 0)):
        st = lib.fc_gather_probe(col.data_ptr(), nnz, U.data_ptr(), rows, rb, w, reps, None,
                                 ctypes.byref(out))
        assert st == 1, (nnz, rows, rb, w, reps)
