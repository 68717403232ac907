"""Mixed precision (S values in FP16, a bfloat16 copy of the iterate for the
sparse product, FP32 accumulation, FP64 reductions and threshold sums)
against the FP64 oracle, on an instance of the medium ER generator.

Two references separate quantisation from arithmetic: the oracle on the
original S, and the oracle on S rounded to FP16.  Bar: final loss within
1e-4 relative of the oracle on the FP16-rounded S, rows summing to 1 within
1e-6; the iterate error is reported and bounded by the bfloat16 rounding of
the gathered rows (5e-3).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_util import csr_to_dev, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fc():
    import paper_2506_04045_amd as fc
    fc.library_path()
    return fc


@pytest.mark.parametrize("c", [8, 32, 64])
def test_mixed_against_fp64_oracle(fc, c):
    wl = W.er_planted(50_000, c, 30.0, 0.05, 11)
    rp, ci, v, U0 = wl.numpy()
    v32 = v.astype(np.float32)
    v16 = v32.astype(np.float16).astype(np.float64)
    spec, _ = oracle.spectral_norm(rp, ci, v16, True)
    tau = 10.0 / oracle.lipschitz_bound(spec, wl.n)
    iters = 100
    ref16 = oracle.solve(rp, ci, v16, True, U0, accelerate=True, max_iter=iters, step=tau)
    ref = oracle.solve(rp, ci, v32.astype(np.float64), True, U0, accelerate=True,
                       max_iter=iters, step=tau)
    S = csr_to_dev(rp, ci, v32, torch.float32)
    with fc.Solver(*S, c, dev(U0.astype(np.float32)), precision="mixed", step=tau) as s:
        info = s.step(iters)
        U = s.get_u(torch.float64).cpu().numpy()
        hist = s.history()
    f_rel16 = abs(info.f - ref16.f[-1]) / abs(ref16.f[-1])
    f_rel = abs(info.f - ref.f[-1]) / abs(ref.f[-1])
    df16 = ref16.f[0] - ref16.f[-1]
    df_rel16 = abs((hist["f"][0] - info.f) - df16) / abs(df16)
    du16 = np.abs(U - ref16.X).max()
    du = np.abs(U - ref.X).max()
    print(f"mixed c={c}: f_rel(fp16 S)={f_rel16:.2e} f_rel(S)={f_rel:.2e} "
          f"df_rel(fp16 S)={df_rel16:.2e} max|dU|(fp16 S)={du16:.2e} max|dU|(S)={du:.2e}")
    assert f_rel16 <= 1e-4
    assert np.abs(U.sum(1) - 1).max() <= 1e-6
    assert (U >= 0).all()
    assert du16 <= 5e-3


def test_mixed_on_the_medium_config_twin(fc):
    """The n = 1e6, c = 32 instance (ER degree 30): mixed precision against
    the oracle on S and on S rounded to FP16, 10 iterations."""
    wl = W.config_medium(seed=0)
    rp, ci, v, U0 = wl.numpy()
    v32 = v.astype(np.float32)
    v16 = v32.astype(np.float16).astype(np.float64)
    tau = 20.0 / oracle.lipschitz_bound(np.sqrt((v16 ** 2).sum() + wl.n), wl.n)
    iters = 10
    ref16 = oracle.solve(rp, ci, v16, True, U0, accelerate=True, max_iter=iters, step=tau)
    ref = oracle.solve(rp, ci, v32.astype(np.float64), True, U0, accelerate=True,
                       max_iter=iters, step=tau)
    S = csr_to_dev(rp, ci, v32, torch.float32)
    with fc.Solver(*S, 32, dev(U0.astype(np.float32)), precision="mixed", step=tau,
                   reorder="degree") as s:
        info = s.step(iters)
        U = s.get_u(torch.float64).cpu().numpy()
    f_rel16 = abs(info.f - ref16.f[-1]) / abs(ref16.f[-1])
    f_rel = abs(info.f - ref.f[-1]) / abs(ref.f[-1])
    du16, du = np.abs(U - ref16.X).max(), np.abs(U - ref.X).max()
    print(f"mixed medium: f_rel(fp16 S)={f_rel16:.2e} f_rel(S)={f_rel:.2e} "
          f"max|dU|(fp16 S)={du16:.2e} max|dU|(S)={du:.2e}")
    assert f_rel16 <= 1e-4
    assert np.abs(U.sum(1) - 1).max() <= 1e-6 and (U >= 0).all()
    assert du16 <= 5e-3
