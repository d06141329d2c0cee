"""O1: brute-force full-tensor step followed by truncated HOSVD (oracle).

TEST INFRASTRUCTURE ONLY.

The plain definition of one step: expand every needed cell to its N^3
tensor, evaluate Alg. 2 (macroparameters, f_S, J) and the face fluxes of
eq. exact-flux literally, form f* = f + dt R (eq. expl-scheme-final, Alg. 1),
then round f* with Op1 (LAPACK SVD of the three unfoldings).  One rounding
per cell per step, applied to the exact full update, is the reading of the
paper's "round after operations that grow the ranks".

With exact=True the face fluxes use the exact |xi_n| on every face instead
of the estimate (on faces off the coordinate axes; on axis faces the two
coincide): the paper's standard, full-tensor discrete velocity method, the
baseline of its Table 1.
"""

import numpy as np

from . import kinetic as kin
from . import tucker as tk
from .fv import BC_INFLOW, BC_OUTFLOW, BC_SYM, BC_WALL, axis_of


def ghost_full(S, j, Fi):
    """Boundary value on the far side of boundary face j (cell value Fi)."""
    bc = S.bc(j)
    kind = bc["kind"]
    if kind == BC_INFLOW:
        return kin.maxwell_full(bc["n"], np.array(bc["u"]), bc["T"], S.xi, S.Rg)
    if kind == BC_OUTFLOW:
        return Fi
    if kind == BC_SYM:
        a = axis_of(S.mesh["face_normal"][j])
        if a < 0:
            raise ValueError("symmetry boundary needs an axis-aligned face")
        return np.flip(Fi, axis=a)
    if kind == BC_WALL:
        fw1 = kin.maxwell_full(1.0, np.zeros(3), bc["Tw"], S.xi, S.Rg)
        xn = S.xin_full(j)
        est = S.estimate_full(j)
        pout = 0.5 * (xn + est)
        pin = 0.5 * (xn - est)
        nw = -(pout * Fi).sum() / (pin * fw1).sum()
        return nw * fw1
    raise ValueError(f"unknown boundary kind {kind}")


def update_full(S, i, get, exact=False):
    """f* of cell i from the full tensors returned by get(cell)."""
    mesh = S.mesh
    Fi = get(i)
    n, u, T, q = kin.macros_full(Fi, S.xi, S.dxi, S.Rg, S.m)
    nu = kin.collision_freq(n, T, S.Kn, S.omega, S.Rg, S.m)
    R = nu * (kin.fs_full(n, u, T, q, S.xi, S.Pr, S.Rg, S.m) - Fi)
    V = mesh["cell_volume"][i]
    for j, s in S.cell_faces[i]:
        L, Rc = mesh["face_left"][j], mesh["face_right"][j]
        fL = get(L)
        fR = get(Rc) if Rc >= 0 else ghost_full(S, j, fL)
        xn = S.xin_full(j)
        est = np.abs(xn) if exact else S.estimate_full(j)
        Fj = 0.5 * xn * (fL + fR) - 0.5 * est * (fR - fL)
        R = R - s * (mesh["face_area"][j] / V) * Fj
    return Fi + S.dt * R


def step_full(S, F, cells=None, round_result=True, exact=False):
    """One O1 step.  F: dict or array cell -> full tensor.

    Returns dict cell -> (rounded Tucker tensor, or f* when round_result is
    False) for `cells` (default: all cells).
    """
    get = (lambda c: F[c])
    if cells is None:
        cells = range(S.mesh["n_cells"])
    out = {}
    for i in cells:
        X = update_full(S, i, get, exact)
        out[i] = tk.hosvd(X, S.tol, S.cap) if round_result else X
    return out


def initial_full(S, macros0, cells=None):
    if cells is None:
        cells = range(S.mesh["n_cells"])
    return {i: kin.maxwell_full(macros0[i, 0], macros0[i, 1:4], macros0[i, 4], S.xi, S.Rg)
            for i in cells}


def run_full(S, macros0, steps):
    """O1 for every cell of a (small) mesh; returns the list of states."""
    F = initial_full(S, macros0)
    for _ in range(steps):
        st = step_full(S, F)
        F = {i: tk.full(t) for i, t in st.items()}
    return F
