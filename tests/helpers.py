"""Shared test helpers: oracle runs and the relative-error measure of macros.

Relative error of macroparameters: n and T relative to themselves, u
relative to the thermal speed sqrt(2 R_g T), q relative to p sqrt(2 R_g T)
with p = m n R_g T; the maximum over cells and components is reported.
"""

import numpy as np


def macro_rel_err(a, b, Rg=0.5, m=1.0):
    """a, b: [n_cells, 8] arrays (n, u1, u2, u3, T, q1, q2, q3); b is the reference."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n, T = b[:, 0], b[:, 4]
    c = np.sqrt(2.0 * Rg * T)
    p = m * n * Rg * T
    e = np.zeros((b.shape[0], 4))
    e[:, 0] = np.abs(a[:, 0] - n) / np.abs(n)
    e[:, 1] = np.abs(a[:, 1:4] - b[:, 1:4]).max(1) / c
    e[:, 2] = np.abs(a[:, 4] - T) / np.abs(T)
    e[:, 3] = np.abs(a[:, 5:8] - b[:, 5:8]).max(1) / (p * c)
    return float(e.max()), e


def tucker_full(G, U):
    A = np.einsum("abc,ia,jb,kc->ijk", G, U[0], U[1], U[2], optimize=True)
    return A
