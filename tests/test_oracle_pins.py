"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself: the
objective by its double-sum definition (problem (P)), finite differences,
the KKT conditions and a support enumeration for the simplex projection,
values printed in Example 4.1, Theorem 3.1's monotonicity and Lipschitz
bound, a planted exact factorisation, a dense eigen-solver for ||S||_2, and
an independent dense re-implementation of the iterations.
"""
import json
import math
import os

import numpy as np
import pytest

from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "example41.json")


@pytest.fixture(scope="module")
def ex41():
    with open(GOLDEN) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def ex41_csr(ex, mode):
    S = np.array(ex["S"], dtype=float)
    if mode == "stored":
        return pins.csr_from_dense(S), S
    return pins.csr_from_dense(S, drop_diag=True), S


# --------------------------------------------------------------------------
# objective and gradient
# --------------------------------------------------------------------------

@pytest.mark.parametrize("diag_unit", [False, True])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_structured_loss_equals_definition(O, diag_unit, seed):
    rng = np.random.default_rng(seed)
    n, c = 9, 4
    (rp, ci, v), A = pins.random_symmetric_csr(n, 0.4, rng, with_diag=not diag_unit)
    U = pins.random_simplex_rows(n, c, rng)
    S = pins.dense_similarity(rp, ci, v, diag_unit, n)
    f_def = pins.objective_by_definition(S, U)
    f = O.loss(rp, ci, v, diag_unit, U)
    assert abs(f - f_def) <= 1e-12 * max(1.0, abs(f_def))


@pytest.mark.parametrize("diag_unit", [False, True])
def test_gradient_matches_finite_differences(O, diag_unit):
    rng = np.random.default_rng(7)
    n, c = 7, 3
    (rp, ci, v), _ = pins.random_symmetric_csr(n, 0.5, rng, with_diag=not diag_unit)
    U = pins.random_simplex_rows(n, c, rng)
    S = pins.dense_similarity(rp, ci, v, diag_unit, n)
    g_fd = pins.central_difference_gradient(S, U)
    g = O.gradient(rp, ci, v, diag_unit, U)
    assert np.abs(g - g_fd).max() <= 1e-6 * max(1.0, np.abs(g_fd).max())


def test_x_s_is_the_sparse_product(O):
    rng = np.random.default_rng(3)
    n, c = 12, 5
    (rp, ci, v), A = pins.random_symmetric_csr(n, 0.3, rng)
    U = rng.random((n, c))
    for diag_unit in (False, True):
        S = A + (np.eye(n) if diag_unit else 0)
        assert np.allclose(O.x_s(rp, ci, v, diag_unit, U), S @ U, rtol=0, atol=1e-13)


def test_share_is_the_gram_matrix_across_blocks(O):
    """share = sum of outer products; the blocked sum spans several blocks and a
    ragged tail (65,536 columns per block)."""
    rng = np.random.default_rng(11)
    U = rng.random((3 * 65536 + 77, 3))
    G = O.share(U)
    ref = np.zeros((3, 3))
    for k in range(3):
        for l in range(3):
            ref[k, l] = math.fsum(U[:, k] * U[:, l])
    assert np.abs(G - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(G, G.T)


def _sub_csr(rp, ci, v, rows):
    sub_rp = [0]
    sub_ci, sub_v = [], []
    for r in rows:
        sub_ci += list(ci[rp[r]:rp[r + 1]])
        sub_v += list(v[rp[r]:rp[r + 1]])
        sub_rp.append(len(sub_ci))
    return np.array(sub_rp), np.array(sub_ci, dtype=np.int32), np.array(sub_v)


@pytest.mark.parametrize("diag_unit", [False, True])
def test_rows_subset_product_and_step_match_dense_definitions(O, diag_unit):
    """x_s_rows is the product at a list of articles; step_rows is one
    projected gradient step there (Alg. 2), checked against the dense
    gradient by finite differences and the support-enumeration projection."""
    rng = np.random.default_rng(12)
    n, c = 10, 4
    (rp, ci, v), A = pins.random_symmetric_csr(n, 0.4, rng)
    S = A + (np.eye(n) if diag_unit else 0)
    U = pins.random_simplex_rows(n, c, rng)
    rows = np.array([7, 0, 3, 3, 9])
    sub = _sub_csr(rp, ci, v, rows)
    assert np.allclose(O.x_s_rows(rows, *sub, diag_unit, U), (S @ U)[rows], rtol=0, atol=1e-13)
    tau = 0.05
    grad = pins.central_difference_gradient(S, U)
    for r, x in zip(rows, O.step_rows(rows, *sub, diag_unit, U, tau)):
        y = pins.project_simplex_bruteforce(U[r] - tau * grad[r])
        assert np.abs(x - y).max() <= 1e-7


# --------------------------------------------------------------------------
# projection onto the simplex (section 2; Alg. 1 computes the same point)
# --------------------------------------------------------------------------

def _kkt_ok(v, y, tol=1e-12):
    if (y < 0).any() or abs(y.sum() - 1.0) > tol:
        return False
    pos = y > 0
    if not pos.any():
        return False
    tau = (v - y)[pos].mean()
    return (np.abs((v - y)[pos] - tau) <= tol).all() and (v[~pos] <= tau + tol).all()


@pytest.mark.parametrize("c", [1, 2, 3, 5, 8])
def test_projection_kkt_and_bruteforce(O, c):
    rng = np.random.default_rng(c)
    for trial in range(200):
        scale = [0.1, 1.0, 10.0][trial % 3]
        v = rng.normal(size=c) * scale
        if trial % 7 == 0 and c > 1:
            v[1] = v[0]               # ties
        y = O.project_simplex(v)
        assert _kkt_ok(v, y), (v, y)
        assert np.abs(y - pins.project_simplex_bruteforce(v)).max() <= 1e-13


def test_projection_special_cases(O):
    rng = np.random.default_rng(11)
    # a point of the simplex is its own projection
    x = pins.random_simplex_rows(1, 6, rng)[0]
    assert np.abs(O.project_simplex(x) - x).max() <= 1e-15
    # invariance under adding a constant to every component
    v = rng.normal(size=6)
    assert np.abs(O.project_simplex(v + 3.7) - O.project_simplex(v)).max() <= 1e-14
    # C = 1: the simplex is the single point 1
    assert O.project_simplex(np.array([-4.2]))[0] == 1.0
    # C = 2: closed form y1 = clip((v1 - v2 + 1)/2, 0, 1)
    for _ in range(50):
        v = rng.normal(size=2) * 2
        y1 = min(1.0, max(0.0, (v[0] - v[1] + 1.0) / 2.0))
        assert np.allclose(O.project_simplex(v), [y1, 1.0 - y1], atol=1e-15)
    # row-wise application
    V = rng.normal(size=(20, 5))
    P = O.project_columns(V)
    for i in range(20):
        assert np.abs(P[i] - pins.project_simplex_bruteforce(V[i])).max() <= 1e-13


def test_projection_extreme_scales_and_wide_rows(O):
    """Offsets far from zero, tiny spreads, exact simplex points with zero
    components and rows up to 64 wide: the KKT conditions hold, and the
    result is unchanged by a constant shift (section 2: the projection
    ignores multiples of the ones vector)."""
    rng = np.random.default_rng(41)
    for c in (4, 17, 32, 64):
        for trial in range(60):
            v = rng.normal(size=c) * [1e-9, 1e-3, 1.0, 1e3][trial % 4]
            shift = [0.0, 1e6, -1e6, 0.25][(trial // 4) % 4]
            y = O.project_simplex(v + shift)
            tol = 1e-12 * max(1.0, abs(shift))
            assert _kkt_ok(v + shift, y, tol=tol), (c, trial)
            if shift == 0.0:
                y0 = O.project_simplex(v)
                assert np.abs(y0 - O.project_simplex(v + 0.375)).max() <= 1e-13
    # an exact point of the simplex with zero components is its own projection
    x = np.zeros(8)
    x[[1, 4, 6]] = [0.5, 0.25, 0.25]
    assert np.array_equal(O.project_simplex(x), x)
    # equal components share the mass equally
    assert np.allclose(O.project_simplex(np.full(5, 3.0)), 0.2, rtol=0, atol=1e-15)


# --------------------------------------------------------------------------
# planted exact factorisation
# --------------------------------------------------------------------------

@pytest.mark.parametrize("accelerate", [False, True])
def test_planted_factorisation_is_a_zero_fixed_point(O, accelerate):
    rng = np.random.default_rng(5)
    n, c = 12, 3
    Ustar = pins.random_simplex_rows(n, c, rng)
    S = Ustar @ Ustar.T                       # diagonal included, stored
    rp, ci, v = pins.csr_from_dense(S)
    assert abs(O.loss(rp, ci, v, False, Ustar)) <= 1e-12 * n * n
    assert np.abs(O.gradient(rp, ci, v, False, Ustar)).max() <= 1e-12 * n
    res = O.solve(rp, ci, v, False, Ustar, accelerate=accelerate, max_iter=20, step=0.01)
    assert np.abs(res.X - Ustar).max() <= 1e-12
    assert np.abs(res.f).max() <= 1e-12 * n * n


# --------------------------------------------------------------------------
# Example 4.1
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["stored", "unit"])
def test_example41_printed_losses(O, ex41, mode):
    (rp, ci, v), S = ex41_csr(ex41, mode)
    unit = mode == "unit"
    X3 = np.array(ex41["scenario3"]["X"]).T
    assert O.loss(rp, ci, v, unit, X3) == pytest.approx(12.25, abs=1e-12)
    for key in ("scenario1", "scenario2"):
        X = np.array(ex41[key]["X"]).T
        assert round(O.loss(rp, ci, v, unit, X), 2) == ex41[key]["loss"]


def test_example41_diagonal_modes_agree(O, ex41):
    (rp_s, ci_s, v_s), S = ex41_csr(ex41, "stored")
    (rp_u, ci_u, v_u), _ = ex41_csr(ex41, "unit")
    rng = np.random.default_rng(0)
    X = pins.random_simplex_rows(7, 2, rng)
    assert O.loss(rp_s, ci_s, v_s, False, X) == pytest.approx(O.loss(rp_u, ci_u, v_u, True, X),
                                                              rel=1e-15)
    assert np.allclose(O.gradient(rp_s, ci_s, v_s, False, X),
                       O.gradient(rp_u, ci_u, v_u, True, X), atol=1e-14)
    # the adjacency in the fixture's edge list is the printed S minus I
    n = 7
    A = np.zeros((n, n))
    for a, b in ex41["edges"]:
        A[a - 1, b - 1] = A[b - 1, a - 1] = 1
    assert np.array_equal(A + np.eye(n), S)


def test_example41_scenario3_is_a_fixed_point_with_negative_curvature(O, ex41):
    (rp, ci, v), _ = ex41_csr(ex41, "stored")
    X3 = np.array(ex41["scenario3"]["X"]).T
    res = O.solve(rp, ci, v, False, X3, accelerate=False, max_iter=50, step=ex41["step"],
                  tol_loss=0.0)
    assert res.iters == 1 and res.stop_reason == O.STOP_LOSS
    assert np.abs(res.X - X3).max() == 0.0
    V = np.array(ex41["hessian_check"]["V"], dtype=float).T
    g = O.gradient(rp, ci, v, False, X3)
    assert float((g * V).sum()) == pytest.approx(ex41["hessian_check"]["grad_dot_V"], abs=1e-13)
    h = 1e-4
    gp = O.gradient(rp, ci, v, False, X3 + h * V)
    gm = O.gradient(rp, ci, v, False, X3 - h * V)
    quad = float(((gp - gm) * V).sum()) / (2 * h)
    assert quad == pytest.approx(ex41["hessian_check"]["hessian_quadratic_form"], abs=1e-6)


def test_example41_scenario2_biased_start(O, ex41):
    (rp, ci, v), _ = ex41_csr(ex41, "stored")
    X0 = np.zeros((7, 2))
    X0[:, 0] = 1.0
    res = O.solve(rp, ci, v, False, X0, accelerate=False, max_iter=5000, step=ex41["step"],
                  tol_loss=0.0)
    assert res.stop_reason == O.STOP_LOSS
    assert round(res.f[-1], 2) == ex41["scenario2"]["loss"]
    X2 = np.array(ex41["scenario2"]["X"]).T
    assert np.abs(res.X - X2).max() <= 1e-2
    # every accepted step before the stop decreased the loss
    assert (np.diff(res.f[:-1]) < 0).all()


def test_example41_global_optimum(O, ex41):
    (rp, ci, v), _ = ex41_csr(ex41, "stored")
    rng = np.random.default_rng(41)
    best_f, best_X = np.inf, None
    for _ in range(40):
        X0 = pins.random_simplex_rows(7, 2, rng)
        res = O.solve(rp, ci, v, False, X0, accelerate=False, max_iter=3000,
                      step=ex41["step"], tol_loss=0.0)
        if res.f[-1] < best_f:
            best_f, best_X = res.f[-1], res.X
    assert round(best_f, 2) == ex41["scenario1"]["loss"]
    X1 = np.array(ex41["scenario1"]["X"]).T
    # the optimum has the printed structure up to the label swap
    k = 0 if best_X[1, 0] > 0.5 else 1
    Xl = best_X[:, [k, 1 - k]]
    assert Xl[1, 0] == pytest.approx(1.0, abs=1e-9) and Xl[5, 1] == pytest.approx(1.0, abs=1e-9)
    assert np.abs(Xl - X1).max() <= 0.03


# --------------------------------------------------------------------------
# Theorem 3.1: Lipschitz bound and monotone GPA
# --------------------------------------------------------------------------

def test_spectral_norm_matches_dense_eigensolver(O):
    import workloads as W
    wl = W.config_small_fp64()
    rp, ci, v, _ = wl.numpy()
    for diag_unit in (False, True):
        S = pins.dense_similarity(rp, ci, v, diag_unit, wl.n)
        ref = np.abs(np.linalg.eigvalsh(S)).max()
        est, it = O.spectral_norm(rp, ci, v, diag_unit)
        assert est == pytest.approx(ref, rel=1e-9), it


def test_gradient_lipschitz_bound(O):
    rng = np.random.default_rng(17)
    n, c = 30, 4
    (rp, ci, v), A = pins.random_symmetric_csr(n, 0.3, rng)
    spec = np.abs(np.linalg.eigvalsh(A)).max()
    L = O.lipschitz_bound(spec, n)
    worst = 0.0
    for _ in range(50):
        X = pins.random_simplex_rows(n, c, rng)
        Y = pins.random_simplex_rows(n, c, rng)
        num = np.linalg.norm(O.gradient(rp, ci, v, False, X) - O.gradient(rp, ci, v, False, Y))
        worst = max(worst, num / np.linalg.norm(X - Y))
    assert worst <= L


def test_gpa_monotone_below_the_theorem_step(O):
    rp, ci, v, U0 = _small_instance(seed=3, n=300, c=4)
    wl_n = U0.shape[0]
    spec, _ = O.spectral_norm(rp, ci, v, True)
    tau = 0.99 / O.lipschitz_bound(spec, wl_n)
    res = O.solve(rp, ci, v, True, U0, accelerate=False, max_iter=60, step=tau)
    d = np.diff(res.f)
    assert (d <= 1e-13 * np.abs(res.f[1:])).all()
    assert (d < 0).sum() >= 55


# --------------------------------------------------------------------------
# the iterations, against an independent dense implementation
# --------------------------------------------------------------------------

def _dense_grad(S, Y):
    """Dense gradient -4 Y (S - Y^T Y) in the paper's C x N orientation."""
    return -4.0 * Y @ (S - Y.T @ Y)


def _dense_project(V):
    return np.stack([pins.project_simplex_bruteforce(V[:, i]) for i in range(V.shape[1])],
                    axis=1)


def _dense_iterations(S, X0, tau, iters, accelerate, points=None):
    """GPA / FISTA written from the dense formulas: gradient -4 X (S - X^T X)
    in the paper's C x N orientation, objective by definition, projection by
    support enumeration, inertial parameter t_{n+1} = (1 + sqrt(1 + 4 t_n^2))/2.
    ``tau`` is a constant or a sequence tau_1..tau_iters; ``points`` collects
    the extrapolated points Y_n (C x N) if given."""
    taus = np.broadcast_to(np.asarray(tau, dtype=float), (iters,))
    Xbar_prev = X0.T.copy()          # C x N
    Y = X0.T.copy()
    t = 1.0
    fs = [pins.objective_by_definition(S, X0)]
    Xbar = Xbar_prev
    for it in range(iters):
        if points is not None:
            points.append(Y.copy())
        grad = _dense_grad(S, Y)
        V = Y - taus[it] * grad
        Xbar = _dense_project(V)
        fs.append(pins.objective_by_definition(S, Xbar.T))
        t_next = (1 + math.sqrt(1 + 4 * t * t)) / 2
        beta = (t - 1) / t_next if accelerate else 0.0
        Y = Xbar + beta * (Xbar - Xbar_prev)
        Xbar_prev, t = Xbar, t_next
    return Xbar.T, np.array(fs)


@pytest.mark.parametrize("accelerate", [False, True])
@pytest.mark.parametrize("diag_unit", [False, True])
def test_iterations_match_dense_implementation(O, accelerate, diag_unit):
    rng = np.random.default_rng(23)
    n, c = 9, 3
    (rp, ci, v), _ = pins.random_symmetric_csr(n, 0.5, rng, with_diag=not diag_unit)
    S = pins.dense_similarity(rp, ci, v, diag_unit, n)
    X0 = pins.random_simplex_rows(n, c, rng)
    tau = 0.02
    res = O.solve(rp, ci, v, diag_unit, X0, accelerate=accelerate, max_iter=12, step=tau)
    Xd, fd = _dense_iterations(S, X0, tau, 12, accelerate)
    assert np.abs(res.X - Xd).max() <= 1e-12
    assert np.abs(res.f - fd).max() <= 1e-11 * np.abs(fd).max()
    # first FISTA step has zero inertia: it equals the first GPA step
    one = O.solve(rp, ci, v, diag_unit, X0, accelerate=True, max_iter=1, step=tau)
    one_gpa = O.solve(rp, ci, v, diag_unit, X0, accelerate=False, max_iter=1, step=tau)
    assert np.array_equal(one.X, one_gpa.X)


def test_fista_differs_from_gpa_from_the_second_step(O):
    rng = np.random.default_rng(29)
    n, c = 9, 3
    (rp, ci, v), _ = pins.random_symmetric_csr(n, 0.5, rng)
    X0 = pins.random_simplex_rows(n, c, rng)
    a = O.solve(rp, ci, v, True, X0, accelerate=True, max_iter=2, step=0.02)
    b = O.solve(rp, ci, v, True, X0, accelerate=False, max_iter=2, step=0.02)
    # t_2 = (1 + sqrt 5)/2 gives beta_1 = 0, so the second steps still agree
    assert np.abs(a.X - b.X).max() <= 1e-15
    a3 = O.solve(rp, ci, v, True, X0, accelerate=True, max_iter=3, step=0.02)
    b3 = O.solve(rp, ci, v, True, X0, accelerate=False, max_iter=3, step=0.02)
    assert np.abs(a3.X - b3.X).max() > 1e-6


# --------------------------------------------------------------------------
# step-size rules
# --------------------------------------------------------------------------

def _small_instance(seed=2, n=200, c=4):
    import torch
    import workloads as W
    wl = W.er_planted(n, c, 10.0, 0.05, seed, val_dtype=torch.float64, u_dtype=torch.float64)
    return wl.numpy()


def test_backtracking_no_rejection_above_lipschitz(O):
    rp, ci, v, U0 = _small_instance()
    n = U0.shape[0]
    spec, _ = O.spectral_norm(rp, ci, v, True)
    L = O.lipschitz_bound(spec, n)
    res = O.solve(rp, ci, v, True, U0, accelerate=True, max_iter=15, backtrack=True, L0=L)
    assert (res.trials[1:] == 1).all()
    assert np.allclose(res.tau[1:], 1.0 / L, rtol=0)


def test_backtracking_gpa_is_monotone_and_l_grows_geometrically(O):
    rp, ci, v, U0 = _small_instance()
    res = O.solve(rp, ci, v, True, U0, accelerate=False, max_iter=30, backtrack=True,
                  L0=1e-3, eta=2.0)
    assert (np.diff(res.f) <= 1e-12 * np.abs(res.f[1:])).all()
    L = 1.0 / res.tau[1:]
    assert (np.diff(L) >= 0).all()
    k = np.log2(L / 1e-3)
    assert np.allclose(k, np.round(k), atol=1e-9)
    assert res.trials[1] > 1


@pytest.mark.parametrize("accelerate", [False, True])
def test_backtracking_accepts_the_first_l_with_sufficient_decrease(O, accelerate):
    """At every iteration the accepted L satisfies
    f(p) <= f(Y) + <grad f(Y), p - Y> + (L/2) ||p - Y||^2 and, when the trial
    was not the first, L/eta violates it (checked with dense definitions)."""
    rng = np.random.default_rng(37)
    n, c, eta = 9, 3, 2.0
    (rp, ci, v), _ = pins.random_symmetric_csr(n, 0.5, rng)
    S = pins.dense_similarity(rp, ci, v, True, n)
    X0 = pins.random_simplex_rows(n, c, rng)
    res = O.solve(rp, ci, v, True, X0, accelerate=accelerate, max_iter=8, backtrack=True,
                  L0=0.05, eta=eta)
    Ys = []
    _dense_iterations(S, X0, res.tau[1:], 8, accelerate, points=Ys)

    def model_gap(Y, L):
        g = _dense_grad(S, Y)
        p = _dense_project(Y - g / L)
        fy = pins.objective_by_definition(S, Y.T)
        fp = pins.objective_by_definition(S, p.T)
        return fp - (fy + (g * (p - Y)).sum() + 0.5 * L * ((p - Y) ** 2).sum())

    rejected_seen = False
    for it in range(1, 9):
        L = 1.0 / res.tau[it]
        assert model_gap(Ys[it - 1], L) <= 1e-10
        if res.trials[it] > 1:
            rejected_seen = True
            assert model_gap(Ys[it - 1], L / eta) > 0
    assert rejected_seen


def test_step_schedule_replays_backtracking(O):
    rp, ci, v, U0 = _small_instance()
    bt = O.solve(rp, ci, v, True, U0, accelerate=True, max_iter=25, backtrack=True, L0=1e-2)
    rp_ = O.solve(rp, ci, v, True, U0, accelerate=True, max_iter=25,
                  step_schedule=bt.tau[1:])
    assert np.array_equal(bt.X, rp_.X)
    assert np.array_equal(bt.f, rp_.f)


def test_pgrad_stop_rule(O):
    rp, ci, v, U0 = _small_instance()
    res = O.solve(rp, ci, v, True, U0, accelerate=True, max_iter=500, backtrack=True,
                  L0=1e-2, tol_pgrad=1e-2)
    assert res.stop_reason == O.STOP_PGRAD
    assert res.r[-1] <= 1e-2 * res.r[1]
    assert (res.r[1:-1] > 1e-2 * res.r[1]).all()


# --------------------------------------------------------------------------
# the gradient-mapping norm r_n (the paper defines no such measure; it is read
# as the length of the projected-gradient step taken at Y_n, over tau_n)
# --------------------------------------------------------------------------

def _fd_gradient_cn(S, Y):
    """Gradient of f at Y (C x N) by central differences of the double-sum
    objective, in the C x N orientation."""
    return pins.central_difference_gradient(S, Y.T.copy(), h=1e-5).T


def test_pgrad_interior_step_has_the_tangent_gradient_norm(O):
    """Closed form.  When the step from Y stays inside the simplex, the
    projection only removes each row's mean, so Y - P(Y - tau grad) =
    tau (grad - row means) and r_1 = ||grad f(Y) (I - 11^T/c)||_F for every
    small tau.  The gradient here comes from central differences of the
    objective's definition, not from any formula of the oracle."""
    rng = np.random.default_rng(43)
    n, c = 8, 3
    (rp, ci, v), _ = pins.random_symmetric_csr(n, 0.5, rng)
    S = pins.dense_similarity(rp, ci, v, True, n)
    X0 = 0.25 / c + 0.75 * pins.random_simplex_rows(n, c, rng)   # entries >= 1/(4c)
    g = pins.central_difference_gradient(S, X0, h=1e-5)          # N x C rows
    tangent = g - g.mean(axis=1, keepdims=True)
    want = float(np.sqrt((tangent ** 2).sum()))
    for tau in (1e-5, 3e-5):
        assert (X0 - tau * g).min() > 0        # the step stays interior
        for accelerate in (False, True):
            res = O.solve(rp, ci, v, True, X0, accelerate=accelerate, max_iter=1, step=tau)
            assert res.r[1] == pytest.approx(want, rel=1e-7), (tau, accelerate)


@pytest.mark.parametrize("mode", ["gpa", "fista", "backtrack"])
def test_pgrad_norm_follows_its_definition_along_the_run(O, mode):
    """r_n = ||Y_n - P_Omega(Y_n - tau_n grad f(Y_n))||_F / tau_n at every
    iteration, with Y_n, the gradient (finite differences of the objective's
    definition) and the projection (support enumeration) all formed
    independently of the oracle; and the relative stop fires at the first n
    with r_n <= tol r_1."""
    rng = np.random.default_rng(47)
    n, c = 9, 3
    (rp, ci, v), _ = pins.random_symmetric_csr(n, 0.5, rng)
    S = pins.dense_similarity(rp, ci, v, True, n)
    X0 = pins.random_simplex_rows(n, c, rng)
    kw = dict(max_iter=10)
    if mode == "backtrack":
        kw.update(backtrack=True, L0=0.05)
    else:
        kw.update(step=0.02)
    res = O.solve(rp, ci, v, True, X0, accelerate=mode != "gpa", **kw)
    Ys = []
    _dense_iterations(S, X0, res.tau[1:], 10, mode != "gpa", points=Ys)
    for it in range(1, 11):
        Y, tau = Ys[it - 1], res.tau[it]
        Xbar = _dense_project(Y - tau * _fd_gradient_cn(S, Y))
        r_def = float(np.sqrt(((Y - Xbar) ** 2).sum())) / tau
        assert res.r[it] == pytest.approx(r_def, rel=1e-6), it
    # the stop fires at the first iteration that meets the relative test
    tol = float(res.r[6] / res.r[1]) * 1.0000001
    first = next(k for k in range(1, 11) if res.r[k] <= tol * res.r[1])
    stopped = O.solve(rp, ci, v, True, X0, accelerate=mode != "gpa", tol_pgrad=tol, **kw)
    assert stopped.stop_reason == O.STOP_PGRAD
    assert stopped.iters == first


# --------------------------------------------------------------------------
# equivariance
# --------------------------------------------------------------------------

def test_node_and_label_permutation_equivariance(O):
    rng = np.random.default_rng(31)
    n, c = 40, 4
    (rp, ci, v), A = pins.random_symmetric_csr(n, 0.2, rng)
    X0 = pins.random_simplex_rows(n, c, rng)
    base = O.solve(rp, ci, v, True, X0, accelerate=True, max_iter=30, step=1e-3)
    p = rng.permutation(n)
    rp2, ci2, v2 = pins.csr_from_dense(A[np.ix_(p, p)])
    perm_nodes = O.solve(rp2, ci2, v2, True, X0[p], accelerate=True, max_iter=30, step=1e-3)
    assert np.abs(perm_nodes.X - base.X[p]).max() <= 1e-12
    q = rng.permutation(c)
    perm_labels = O.solve(rp, ci, v, True, X0[:, q], accelerate=True, max_iter=30, step=1e-3)
    assert np.abs(perm_labels.X - base.X[:, q]).max() <= 1e-12


# --------------------------------------------------------------------------
# second order (Theorem 4.1): Hessian-vector products and curvature on the face
# --------------------------------------------------------------------------

def _quadratic_form_by_definition(S, X, V, h=0.25):
    """<V, Hess f(X) V> = 2 a2, where f(X + eps V) = a0 + ... + a4 eps^4 is a
    quartic in eps: five samples of the double-sum objective fix it exactly."""
    eps = np.array([-2.0, -1.0, 0.0, 1.0, 2.0]) * h
    vals = [pins.objective_by_definition(S, X + e * V) for e in eps]
    coef = np.linalg.solve(np.vander(eps, 5, increasing=True), vals)
    return 2.0 * coef[2]


@pytest.mark.parametrize("diag_unit", [False, True])
def test_hvp_matches_the_objective_by_definition(O, diag_unit):
    rng = np.random.default_rng(31)
    n, c = 8, 3
    (rp, ci, v), A = pins.random_symmetric_csr(n, 0.5, rng)
    S = A + (np.eye(n) if diag_unit else 0)
    X = pins.random_simplex_rows(n, c, rng)
    V = rng.normal(size=(n, c))
    HV = O.hvp(rp, ci, v, diag_unit, X, V)
    q = _quadratic_form_by_definition(S, X, V)
    assert float((V * HV).sum()) == pytest.approx(q, rel=1e-9)
    for _ in range(3):     # every component, through polarization
        W = rng.normal(size=(n, c))
        pol = 0.25 * (_quadratic_form_by_definition(S, X, V + W)
                       - _quadratic_form_by_definition(S, X, V - W))
        assert float((W * HV).sum()) == pytest.approx(pol, rel=1e-8, abs=1e-9)
        HW = O.hvp(rp, ci, v, diag_unit, X, W)
        assert float((W * HV).sum()) == pytest.approx(float((V * HW).sum()), rel=1e-12)


def test_example41_hessian_form_and_negative_curvature(O, ex41):
    (rp, ci, v), _ = ex41_csr(ex41, "stored")
    X3 = np.array(ex41["scenario3"]["X"]).T
    V = np.array(ex41["hessian_check"]["V"], dtype=float).T
    HV = O.hvp(rp, ci, v, False, X3, V)
    assert float((V * HV).sum()) == pytest.approx(ex41["hessian_check"]["hessian_quadratic_form"],
                                                  abs=1e-12)
    lam, D = O.curvature_dense(rp, ci, v, False, X3)
    assert lam <= -4.0 / float((V * V).sum()) + 1e-12     # Rayleigh quotient bound
    assert np.abs(D.sum(1)).max() <= 1e-12 and abs(np.linalg.norm(D) - 1) <= 1e-12
    assert float((D * O.hvp(rp, ci, v, False, X3, D)).sum()) == pytest.approx(lam, abs=1e-10)


def test_planted_minimizer_has_no_negative_curvature(O):
    rng = np.random.default_rng(5)
    n, c = 12, 3
    Ustar = pins.random_simplex_rows(n, c, rng)
    S = Ustar @ Ustar.T
    rp, ci, v = pins.csr_from_dense(S)
    lam, _ = O.curvature_dense(rp, ci, v, False, Ustar)
    assert lam >= -1e-10
    # a face point with zero components: the basis keeps them at zero
    Z = Ustar.copy()
    Z[0] = [1.0, 0.0, 0.0]
    B = O.face_basis(Z)
    assert B.shape[1] == n * (c - 1) - 2
    assert np.abs(B.T @ B - np.eye(B.shape[1])).max() <= 1e-12
    assert np.abs(B[1:3, :]).max() == 0.0
