"""Dense, definition-level helpers used to pin the oracle on tiny inputs.

These are written from the problem statement itself (section 2): the
objective as the double sum over all (i, j), the projection as the minimiser
of the distance over the simplex found by enumerating supports.  They share
nothing with the oracle's structured formulas, which is what makes them pins.
"""
import itertools

import numpy as np


def dense_similarity(row_ptr, col_idx, val, diag_unit, n):
    S = np.zeros((n, n))
    for i in range(n):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            S[i, col_idx[e]] += val[e]
    if diag_unit:
        S += np.eye(n)
    return S


def objective_by_definition(S, U):
    """f = sum_i sum_j (s_ij - sum_k x_ki x_kj)^2 with x_i = U[i] (problem (P))."""
    n = S.shape[0]
    total = 0.0
    for i in range(n):
        for j in range(n):
            y = 0.0
            for k in range(U.shape[1]):
                y += U[i, k] * U[j, k]
            total += (S[i, j] - y) ** 2
    return total


def central_difference_gradient(S, U, h=1e-6):
    G = np.zeros_like(U)
    for i in range(U.shape[0]):
        for k in range(U.shape[1]):
            Up, Um = U.copy(), U.copy()
            Up[i, k] += h
            Um[i, k] -= h
            G[i, k] = (objective_by_definition(S, Up) - objective_by_definition(S, Um)) / (2 * h)
    return G


def project_simplex_bruteforce(v):
    """argmin ||y - v|| over the unit simplex by trying every support set:
    on a support A the minimiser is v_A - t with t = (sum v_A - 1)/|A|; keep
    the feasible candidate (all entries >= 0) of smallest distance."""
    c = len(v)
    best, best_d = None, np.inf
    for r in range(1, c + 1):
        for A in itertools.combinations(range(c), r):
            A = list(A)
            t = (v[A].sum() - 1.0) / len(A)
            y = np.zeros(c)
            y[A] = v[A] - t
            if (y >= -1e-15).all():
                d = ((y - v) ** 2).sum()
                if d < best_d:
                    best, best_d = np.maximum(y, 0.0), d
    return best


def csr_from_dense(S, drop_diag=False):
    n = S.shape[0]
    row_ptr = [0]
    cols, vals = [], []
    for i in range(n):
        for j in range(n):
            if drop_diag and i == j:
                continue
            if S[i, j] != 0:
                cols.append(j)
                vals.append(S[i, j])
        row_ptr.append(len(cols))
    return (np.array(row_ptr, dtype=np.int64), np.array(cols, dtype=np.int32),
            np.array(vals, dtype=np.float64))


def random_symmetric_csr(n, density, rng, with_diag=False):
    A = rng.random((n, n)) * (rng.random((n, n)) < density)
    A = np.triu(A, 1)
    A = A + A.T
    if with_diag:
        A += np.diag(rng.random(n))
    return csr_from_dense(A), A


def random_simplex_rows(n, c, rng):
    X = rng.exponential(size=(n, c))
    return X / X.sum(axis=1, keepdims=True)
