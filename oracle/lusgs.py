"""LU-SGS implicit iteration, full-tensor and Tucker forms (oracle).

TEST INFRASTRUCTURE ONLY.

Section "Tensorized discrete velocity method", implicit scheme: the
right-hand side of eq. expl-scheme-final is taken at the new level and
linearised (eq. linear-system).  Multiplied through by dt:

    [I - dt dR/df] df = dt R(f^n),      f^{n+1} = f^n + df.

Readings (the paper lists only the diagonal term and its rank-1 division):

* Jacobian.  f_S is held fixed (its dependence on f is dropped, as the
  paper does for the diagonal).  The block coupling cell i to the far cell
  m of its face l is the derivative of the face flux of eq. exact-flux with
  the explicit step's P_out / P_in:  B_im = (dt A_l / V_i) P_in,l, with
  P_in <= 0.  Boundary ghosts are held fixed: no implicit coupling through
  boundary faces.
* Diagonal.  Eq. diagonal_term times dt, with |xi_n| replaced by the bound
  of eq. xin-one-rank-approx:
      D_i = (1 + dt nu_i) 1 + (dt / (2 V_i)) (sum_l A_l) |xi|,
      |xi|(i1,i2,i3) = sqrt(xi_i1^2 + xi_i2^2 + xi_i3^2),
  summed over every face of the cell (boundary faces included), nu_i from
  the macroparameters of f_i^n.  D_est is the rank-1 truncated HOSVD of
  D_i (our reading of "approximated by a tensor with ranks 1"), and the
  division by it is exact (eq. one_rank_division).
* Sweep order.  A greedy colouring of the face graph: cells in index
  order, each takes the smallest colour no already coloured neighbour has.
  L (U) holds the blocks whose far cell has a smaller (larger) colour;
  cells of one colour share no face, so each colour is one parallel stage.
      forward:  df*_i = D_i^-1 (dt R_i - sum_{m lower} B_im df*_m)
      backward: df_i  = df*_i - D_i^-1 sum_{m upper} B_im df_m
  which solves (D + L) D^-1 (D + U) df = dt R.
* Tucker form.  Each stage's tensor is one Op2 sum of Tucker terms divided
  by D_est term by term, then one Op4 rounding (tolerance eps relative to
  that tensor, rank cap): df*_i for every cell, df_i for every cell with a
  later neighbour (the others keep df*_i), and f_i + df_i.
"""

import numpy as np

from . import kinetic as kin
from . import tucker as tk
from . import tucker_dvm as td


def colouring(mesh):
    """Greedy colouring of the face graph in cell-index order."""
    nc = mesh["n_cells"]
    nbrs = [set() for _ in range(nc)]
    for L, R in zip(mesh["face_left"], mesh["face_right"]):
        if R >= 0 and R != L:
            nbrs[L].add(int(R))
            nbrs[R].add(int(L))
    col = np.full(nc, -1, dtype=np.int64)
    for i in range(nc):
        taken = {col[m] for m in nbrs[i] if col[m] >= 0}
        c = 0
        while c in taken:
            c += 1
        col[i] = c
    return col


def speed(xi):
    """|xi| on the velocity grid (eq. xin-one-rank-approx's bound)."""
    return np.sqrt(xi[:, None, None] ** 2 + xi[None, :, None] ** 2 + xi[None, None, :] ** 2)


def diag_full(S, i, nu):
    """D_i of eq. diagonal_term with the bound, times dt, as a full tensor."""
    mesh = S.mesh
    area = sum(mesh["face_area"][j] for j, _ in S.cell_faces[i])
    return (1.0 + S.dt * nu) + (S.dt / (2.0 * mesh["cell_volume"][i])) * area * speed(S.xi)


def diag_est(S, i, nu):
    """Rank-1 truncated HOSVD of D_i (Tucker, core 1x1x1)."""
    return tk.hosvd(diag_full(S, i, nu), 0.0, 1)


def rank1_vectors(d):
    """(sigma u1, u2, u3) of a rank-1 Tucker tensor, for divide_rank1."""
    return d.G[0, 0, 0] * d.U[0][:, 0], d.U[1][:, 0], d.U[2][:, 0]


def far_blocks(S, i):
    """(far cell, B_im as a Tucker tensor) for the interior faces of cell i."""
    mesh = S.mesh
    V = mesh["cell_volume"][i]
    out = []
    for j, s in S.cell_faces[i]:
        m = mesh["face_right"][j] if s > 0 else mesh["face_left"][j]
        if m < 0:
            continue
        _, pin = S.p_terms(j, s)
        out.append((int(m), pin.scaled(S.dt * mesh["face_area"][j] / V)))
    return out


# ---- full tensors (no rounding) -------------------------------------------

def sweeps_full(S, col, D, rhs):
    """LU-SGS sweeps on full tensors: D, rhs dicts cell -> N^3 arrays."""
    nc = S.mesh["n_cells"]
    order = sorted(range(nc), key=lambda c: (col[c], c))
    B = {i: [(m, tk.full(b)) for m, b in far_blocks(S, i)] for i in range(nc)}
    dfs = {}
    for i in order:
        acc = rhs[i].copy()
        for m, b in B[i]:
            if col[m] < col[i]:
                acc = acc - b * dfs[m]
        dfs[i] = acc / D[i]
    df = {}
    for i in reversed(order):
        acc = np.zeros_like(rhs[i])
        for m, b in B[i]:
            if col[m] > col[i]:
                acc = acc + b * df[m]
        df[i] = dfs[i] - acc / D[i]
    return df


def rhs_full(S, F):
    """dt R_i = f*_i - f_i from the full-tensor explicit update (O1)."""
    from . import dvm
    get = (lambda c: F[c])
    return {i: dvm.update_full(S, i, get) - F[i] for i in range(S.mesh["n_cells"])}


def step_full(S, F, col=None):
    """One LU-SGS iteration on full tensors with the rank-1 diagonal."""
    if col is None:
        col = colouring(S.mesh)
    D = {}
    for i in range(S.mesh["n_cells"]):
        n, u, T, q = kin.macros_full(F[i], S.xi, S.dxi, S.Rg, S.m)
        nu = kin.collision_freq(n, T, S.Kn, S.omega, S.Rg, S.m)
        D[i] = tk.full(diag_est(S, i, nu))
    df = sweeps_full(S, col, D, rhs_full(S, F))
    return {i: F[i] + df[i] for i in F}


# ---- Tucker form -----------------------------------------------------------

def rhs_terms(S, i, get):
    """The Tucker terms of dt R_i (the explicit update's terms with the
    cell's own coefficient 1 - dt nu replaced by -dt nu), and nu_i."""
    terms, (n, u, T, q) = td.update_terms(S, i, get)
    nu = kin.collision_freq(n, T, S.Kn, S.omega, S.Rg, S.m)
    terms[0] = get(i).scaled(-S.dt * nu)
    return terms, nu


def step(S, states, col=None):
    """One LU-SGS iteration in Tucker form; states: dict cell -> Tucker.

    Returns (new states, df*, df) as dicts."""
    mesh = S.mesh
    nc = mesh["n_cells"]
    if col is None:
        col = colouring(mesh)
    get = (lambda c: states[c])
    order = sorted(range(nc), key=lambda c: (col[c], c))
    rhs, dinv = {}, {}
    for i in range(nc):
        terms, nu = rhs_terms(S, i, get)
        rhs[i] = terms
        dinv[i] = rank1_vectors(diag_est(S, i, nu))
    blocks = {i: far_blocks(S, i) for i in range(nc)}
    dfs = {}
    for i in order:
        terms = list(rhs[i])
        for m, b in blocks[i]:
            if col[m] < col[i]:
                terms.append(tk.hadamard(b, dfs[m]).scaled(-1.0))
        dfs[i] = tk.round_sum([tk.divide_rank1(t, *dinv[i]) for t in terms], S.tol, S.cap)
    df = {}
    for i in reversed(order):
        upper = [(m, b) for m, b in blocks[i] if col[m] > col[i]]
        if not upper:
            df[i] = dfs[i]
            continue
        terms = [dfs[i]]
        for m, b in upper:
            terms.append(tk.divide_rank1(tk.hadamard(b, df[m]).scaled(-1.0), *dinv[i]))
        df[i] = tk.round_sum(terms, S.tol, S.cap)
    new = {i: tk.round_sum([states[i], df[i]], S.tol, S.cap) for i in range(nc)}
    return new, dfs, df


def run(S, macros0, iters):
    states = td.initial_states(S, macros0)
    col = colouring(S.mesh)
    for _ in range(iters):
        states, _, _ = step(S, states, col)
    return states
