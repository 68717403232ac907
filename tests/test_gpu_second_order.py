"""Second-order check of Theorem 4.1 on the GPU against the FP64 oracle:
the Hessian applied to a direction (eq. hessian), and the Lanczos search
for the smallest curvature over the face directions at a point.

Bars: FP64 Hessian-vector products within 1e-12 normwise of the oracle's,
FP32 within 1e-5; the smallest curvature within 1e-9 (FP64) of the dense
eigenvalue of the oracle's restricted Hessian when the Krylov space spans
the face, and its Ritz direction a unit face direction whose Rayleigh
quotient is that value.
"""
import json
import os

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


@pytest.mark.parametrize("diag", ["unit", "stored"])
@pytest.mark.parametrize("c", [1, 3, 8, 32, 64])
def test_hessian_vector_matches_the_oracle(fc, diag, c):
    wl = W.er_planted(3001, max(c, 2), 12.0, 0.05, c, val_dtype=torch.float64,
                      u_dtype=torch.float64)
    rp, ci, v, _ = wl.numpy()
    rng = np.random.default_rng(c)
    U = pins.random_simplex_rows(wl.n, c, rng)
    V = rng.normal(size=(wl.n, c))
    ref = oracle.hvp(rp, ci, v, diag == "unit", U, V)
    hv = fc.hessian_vector(*csr_to_dev(rp, ci, v, torch.float64), dev(U, torch.float64),
                           dev(V, torch.float64), diag=diag).cpu().numpy()
    assert normwise(hv, ref) <= 1e-12
    U32, V32, v32 = U.astype(np.float32), V.astype(np.float32), v.astype(np.float32)
    ref32 = oracle.hvp(rp, ci, v32.astype(np.float64), diag == "unit", U32.astype(np.float64),
                       V32.astype(np.float64))
    hv32 = fc.hessian_vector(*csr_to_dev(rp, ci, v32, torch.float32), dev(U32), dev(V32),
                             diag=diag).cpu().numpy()
    assert normwise(hv32, ref32) <= 1e-5


def test_hessian_vector_with_hub_rows(fc):
    rp, ci, v = star_plus_er(5000, 3.0, 4, hub_frac=0.9)
    rng = np.random.default_rng(4)
    U = pins.random_simplex_rows(5000, 16, rng)
    V = rng.normal(size=(5000, 16))
    ref = oracle.hvp(rp, ci, v, True, U, V)
    hv = fc.hessian_vector(*csr_to_dev(rp, ci, v, torch.float64), dev(U, torch.float64),
                           dev(V, torch.float64)).cpu().numpy()
    assert normwise(hv, ref) <= 1e-12


def test_example41_saddle_is_certified(fc):
    ex = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "example41.json")))
    S = np.array(ex["S"], dtype=float)
    rp, ci, v = pins.csr_from_dense(S)
    X3 = np.ascontiguousarray(np.array(ex["scenario3"]["X"]).T)
    Vbar = np.ascontiguousarray(np.array(ex["hessian_check"]["V"], dtype=float).T)
    Sd = csr_to_dev(rp, ci, v, torch.float64)
    hv = fc.hessian_vector(*Sd, dev(X3, torch.float64), dev(Vbar, torch.float64),
                           diag="stored").cpu().numpy()
    assert float((hv * Vbar).sum()) == pytest.approx(-4.0, abs=1e-12)
    lam_ref, _ = oracle.curvature_dense(rp, ci, v, False, X3)
    V0 = np.random.default_rng(0).normal(size=X3.shape)
    lam, D, steps = fc.curvature(*Sd, dev(X3, torch.float64), dev(V0, torch.float64),
                                 krylov=20, diag="stored")
    D = D.cpu().numpy()
    assert lam < 0 and lam == pytest.approx(lam_ref, abs=1e-10)
    assert steps <= 7                      # the face has dimension 7
    assert np.abs(D.sum(1)).max() <= 1e-12 and abs(np.linalg.norm(D) - 1) <= 1e-10
    assert float((D * oracle.hvp(rp, ci, v, False, X3, D)).sum()) == pytest.approx(lam, abs=1e-9)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_curvature_at_a_solver_iterate(fc, prec):
    """At an iterate of the solver (some components driven to zero), the
    Lanczos value matches the dense restricted eigenvalue when the Krylov
    space can span the face."""
    wl = W.er_planted(120, 4, 10.0, 0.05, 21, val_dtype=torch.float64, u_dtype=torch.float64)
    rp, ci, v, U0 = wl.numpy()
    ref = oracle.solve(rp, ci, v, True, U0, accelerate=False, max_iter=60, step=2e-3)
    X = ref.X
    assert (X == 0).sum() > 0
    lam_ref, _ = oracle.curvature_dense(rp, ci, v, True, X)
    dim = int(sum(max(0, (X[i] > 0).sum() - 1) for i in range(wl.n)))
    dt = torch.float64 if prec == "fp64" else torch.float32
    Xd = X if prec == "fp64" else X.astype(np.float32).astype(np.float64)
    vd = v if prec == "fp64" else v.astype(np.float32).astype(np.float64)
    if prec == "fp32":
        lam_ref, _ = oracle.curvature_dense(rp, ci, vd, True, Xd)
    V0 = np.random.default_rng(1).normal(size=X.shape)
    lam, D, steps = fc.curvature(*csr_to_dev(rp, ci, vd, dt), dev(Xd, dt), dev(V0, dt),
                                 krylov=min(512, dim + 5))
    D = D.double().cpu().numpy()
    tol = 1e-9 if prec == "fp64" else 1e-4
    print(f"curvature {prec}: lambda {lam:.10e} dense {lam_ref:.10e} steps {steps} dim {dim}")
    assert abs(lam - lam_ref) <= tol * max(1.0, abs(lam_ref))
    assert np.abs(D[Xd == 0]).max() == 0.0
    assert np.abs(D.sum(1)).max() <= (1e-12 if prec == "fp64" else 1e-6)


def test_curvature_rules(fc):
    wl = W.er_planted(200, 4, 8.0, 0.05, 2)
    rp, ci, v, U0 = wl.numpy()
    from paper_2506_04045_amd import _native
    Sd = csr_to_dev(rp, ci, v.astype(np.float32), torch.float32)
    U = dev(U0.astype(np.float32))
    with pytest.raises(_native.FcError):   # start direction off the face
        fc.curvature(*Sd, U, torch.ones_like(U), krylov=5)
    with pytest.raises(_native.FcError):
        fc.curvature(*Sd, U, U.clone(), krylov=0)
