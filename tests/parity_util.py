"""Comparison helpers shared by the GPU parity tests (no GPU code here).

assert_close bounds the error two ways: rel-L2 over all entries, and the
largest entry error relative to the largest reference entry, so that one target
far off cannot hide inside a norm over thousands.  solve_residual checks the
solved expansions of the triangular solves (What = M^{-1} W, lhat = M^{-T} l)
through the products they must reproduce, which are well conditioned although
M = K(X, Y) is not (cond ~ 2e9 at tau = 1e-6 for 1/r).
"""
import numpy as np


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def assert_close(a, b, tol, what="", max_tol=None):
    """rel-L2 <= tol and max |a - b| <= max_tol * max |b| (max_tol = tol by default)."""
    a, b = np.asarray(a), np.asarray(b)
    e2, ei = rel(a, b), max_rel(a, b)
    mt = tol if max_tol is None else max_tol
    assert e2 <= tol and ei <= mt, f"{what}: rel-L2 {e2:.3e} (<= {tol:.0e}), max {ei:.3e} (<= {mt:.0e})"
    return e2, ei


def kernel_matrix(oracle_lib, kernel, param, A, B):
    """K(a_i, b_j) through the oracle's point kernel (rows A, columns B)."""
    z = (A[:, None, :] - B[None, :, :]).reshape(-1, 3)
    return oracle_lib.kernel_eval(kernel, param, z).reshape(A.shape[0], B.shape[0])


def solve_residual(M, solved, rhs, transpose=False):
    """Residual of solved rows (one box each): ||M x - b|| / ||b|| over all boxes,
    and the largest per-box value (boxes with b = 0 skipped).  transpose: the
    rows solve M^T x = b."""
    prod = solved @ M if transpose else solved @ M.T
    nb = np.linalg.norm(rhs, axis=1)
    per = np.linalg.norm(prod - rhs, axis=1)
    live = nb > 0
    return float(np.linalg.norm(prod - rhs) / np.linalg.norm(rhs)), float((per[live] / nb[live]).max())
