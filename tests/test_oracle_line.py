"""Pins of the oracle's ordered line iteration spaces (Section 3: do_i_inc ...
do_k_dec process a line cell by cell in a fixed order, lines independent).

* A constant recurrence u(c) = u(c-1)/2 + 1 from seed 0 is 2 - 2^-c at cell
  c, exactly (every value is a dyadic rational).
* The dec order equals the inc order on the reversed line; any axis equals
  axis 2 on the transposed array (so the index bookkeeping is pinned).
* Forward elimination + back substitution solve every line's tridiagonal
  system: compared with numpy.linalg.solve on the dense matrix of each line
  (this pins tridiag_fwd and tridiag_back, which tridiag_solve composes).
"""
import numpy as np
import pytest

import oracle


def test_constant_recurrence_closed_form():
    shape = (7, 3, 4)
    out = oracle.line_recur(np.full(shape, 0.5), np.ones(shape), axis=2, direction=1, seed=0.0)
    n = np.arange(shape[0])
    expect = 2.0 - 2.0 ** -n
    for j in range(3):
        for i in range(4):
            assert np.array_equal(out[:, j, i], expect)
    # seed enters as the value before the first cell
    out = oracle.line_recur(np.full(shape, 0.5), np.zeros(shape), axis=2, direction=1, seed=8.0)
    assert np.array_equal(out[:, 0, 0], 8.0 * 0.5 ** (n + 1))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_dec_is_inc_on_reversed_line(axis):
    g = np.random.default_rng(axis)
    shape = (5, 6, 7)
    a = g.uniform(-0.9, 0.9, shape)
    b = g.standard_normal(shape)
    ax = 2 - axis  # numpy axis of grid axis (i, j, k) in the [k][j][i] layout
    inc = oracle.line_recur(np.flip(a, ax), np.flip(b, ax), axis, 1, seed=0.3)
    dec = oracle.line_recur(a, b, axis, -1, seed=0.3)
    assert np.array_equal(np.flip(inc, ax), dec)


@pytest.mark.parametrize("axis", [0, 1])
def test_axis_is_k_on_transposed_grid(axis):
    g = np.random.default_rng(10 + axis)
    shape = (4, 5, 6)
    a = g.uniform(-0.9, 0.9, shape)
    b = g.standard_normal(shape)
    got = oracle.line_recur(a, b, axis, 1, seed=-1.0)
    ax = 2 - axis
    perm = [ax] + [d for d in range(3) if d != ax]  # line axis first
    ref = oracle.line_recur(np.ascontiguousarray(a.transpose(perm)), np.ascontiguousarray(b.transpose(perm)),
                            2, 1, seed=-1.0)
    inv = np.argsort(perm)
    assert np.array_equal(got, ref.transpose(inv))


@pytest.mark.parametrize("axis,direction", [(2, 1), (2, -1), (1, 1), (0, -1)])
def test_thomas_solves_each_line(axis, direction):
    g = np.random.default_rng(20 + axis)
    shape = (9, 6, 11)
    lo = g.uniform(-1, 1, shape)
    up = g.uniform(-1, 1, shape)
    di = 2.5 + g.uniform(0, 1, shape)  # diagonally dominant
    rhs = g.standard_normal(shape)
    x = oracle.tridiag_solve(lo, di, up, rhs, axis, direction)
    ax = 2 - axis
    L = shape[ax]
    moved = [np.moveaxis(v, ax, -1).reshape(-1, L) for v in (lo, di, up, rhs, x)]
    for lo_l, di_l, up_l, r_l, x_l in zip(*moved):
        # the line in its processing order: lo couples to the previous cell
        order = np.arange(L) if direction > 0 else np.arange(L)[::-1]
        M = np.zeros((L, L))
        for s, c in enumerate(order):
            M[s, s] = di_l[c]
            if s > 0:
                M[s, s - 1] = lo_l[c]
            if s + 1 < L:
                M[s, s + 1] = up_l[c]
        ref = np.linalg.solve(M, r_l[order])
        np.testing.assert_allclose(x_l[order], ref, rtol=0, atol=1e-13 * max(1.0, np.abs(ref).max()))
