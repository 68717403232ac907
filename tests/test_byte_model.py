"""The algorithmic bytes bench.py divides by kernel time (the roofline's
numerator), checked against an inventory of the arrays each launch must
touch once, and at the n = 7e7, c = 32, 1.4e9-nonzero power-law workload
against the figures the measurement reports (GB = 1e9 bytes)."""

import pytest

import bench

N, C, NNZ = 70_000_000, 32, 1_400_000_000
N_LONG, NNZ_LONG = 2_360_000, 798_000_000     # rows longer than 64 nonzeros, ~57 % of them


def _total(arrays):
    return sum(count * width for count, width in arrays)


def _single_pass_inventory(n, c, nnz, n_long, nnz_long):
    """(element count, bytes per element) of what one launch reads or writes."""
    light = nnz - nnz_long
    single = [(n + 1, 8),              # row_ptr
              (light, 4), (light, 4),  # the light rows' column indices and values
              (n * c, 4),              # Y_n: its own rows, and each gathered row once
              (n * c, 4),              # Xbar_{n-1}
              (n_long * c, 4),         # the long rows' products from the pre-pass
              (n * c, 4),              # Xbar_n written
              (n * c, 4)]              # Y_{n+1} written
    prepass = [(n_long + 1, 8),        # the long rows' pointers
               (nnz_long, 4), (nnz_long, 4),
               (n_long * c, 4)]        # their products written
    minimum = [(n + 1, 8), (nnz, 4), (nnz, 4), (n * c, 4), (n * c, 4), (n * c, 4), (n * c, 4)]
    return _total(single), _total(prepass), _total(minimum)


def _two_pass_inventory(n, c, nnz, b_val, b_u, b_x, b_z, b_shadow):
    spmm = [(n + 1, 8), (nnz, 4), (nnz, b_val),
            (n * c, b_u),              # each gathered row once
            (n * c, b_z)]              # S Xbar written
    fused = [(n * c, b_x), (n * c, b_x),   # Xbar_n, Xbar_{n-1}
             (n * c, b_z), (n * c, b_z),   # S Xbar_n, S Xbar_{n-1}
             (n * c, b_x),                 # Xbar_{n+1} written
             (n * c, b_shadow)]            # its bfloat16 copy for the next gathers (mixed)
    return _total(spmm), _total(fused)


@pytest.mark.parametrize("shape", [(N, C, NNZ, N_LONG, NNZ_LONG), (1000, 3, 7000, 0, 0),
                                   (12_345, 64, 400_000, 17, 9_000)])
def test_single_pass_bytes_match_the_inventory(shape):
    n, c, nnz, n_long, nnz_long = shape
    got = bench.single_pass_bytes(n, c, nnz, n_long, nnz_long)
    single, prepass, minimum = _single_pass_inventory(n, c, nnz, n_long, nnz_long)
    assert (got["fused"], got["spmm"], got["iteration_minimum"]) == (single, prepass, minimum)


@pytest.mark.parametrize("prec,widths", [("fp32", (4, 4, 4, 4, 0)), ("fp64", (8, 8, 8, 8, 0)),
                                         ("mixed", (2, 2, 4, 4, 2))])
def test_two_pass_bytes_match_the_inventory(prec, widths):
    got = bench.algorithmic_bytes(N, C, NNZ, prec)
    spmm, fused = _two_pass_inventory(N, C, NNZ, *widths)
    assert got["spmm"] == spmm and got["fused"] == fused
    b_val, b_x = widths[0], widths[2]
    minimum = _total([(N + 1, 8), (NNZ, 4), (NNZ, b_val)] + [(N * C, b_x)] * 4)   # Y_n, Xbar_{n-1} read; Xbar_n, Y_{n+1} written
    assert got["iteration_minimum"] == minimum


def test_headline_figures():
    sp = bench.single_pass_bytes(N, C, NNZ, N_LONG, NNZ_LONG)
    tp = bench.algorithmic_bytes(N, C, NNZ, "fp32")
    assert round(sp["iteration_minimum"] / 1e9, 1) == 47.6
    assert round(sp["fused"] / 1e9, 1) == 41.5
    assert round(tp["spmm"] / 1e9, 1) == 29.7
    assert round((tp["spmm"] + tp["fused"]) / 1e9, 1) == 74.5
