"""Comparison helpers of the GPU parity tests.

Solutions are [S][N] arrays, one right-hand side per row.  They are compared
column by column (column = right-hand side): the relative 2-norm error
||x_s - x_s^or|| / ||x_s^or|| of every column, and its element-wise form
max_k |x_sk - x_sk^or| / max_k |x_sk^or|.  The worst column is reported.  One
relative norm over all columns at once could hide a bad column among many;
the element-wise form catches an error confined to a few nodes.
"""
import numpy as np


def col_errors(X, Xo):
    """(2-norm errors, max-norm errors) per column of X against Xo."""
    X = np.atleast_2d(np.asarray(X))
    Xo = np.atleast_2d(np.asarray(Xo))
    assert X.shape == Xo.shape, (X.shape, Xo.shape)
    d = X - Xo
    e2 = np.linalg.norm(d, axis=1) / np.linalg.norm(Xo, axis=1)
    einf = np.abs(d).max(axis=1) / np.abs(Xo).max(axis=1)
    return e2, einf


def assert_cols(X, Xo, tol, tol_inf=None, what=""):
    """Every column within tol (2-norm) and tol_inf (max-norm, default tol).
    Returns the worst errors (2-norm, max-norm)."""
    e2, einf = col_errors(X, Xo)
    tol_inf = tol if tol_inf is None else tol_inf
    s2, si = int(np.argmax(e2)), int(np.argmax(einf))
    assert e2[s2] <= tol and einf[si] <= tol_inf, (
        f"{what}: column {s2} has relative 2-norm error {e2[s2]:.3e} (bound {tol:.0e}); "
        f"column {si} has max-norm error {einf[si]:.3e} (bound {tol_inf:.0e})")
    return float(e2[s2]), float(einf[si])


def rel(a, b):
    """Relative 2-norm error of one vector (a gradient, a model)."""
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
