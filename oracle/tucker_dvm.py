"""O2: the step computed in Tucker form (oracle; timed CPU baseline).

TEST INFRASTRUCTURE ONLY.

Per cell, following the tensorised method (Section "Tensorized discrete
velocity method"):
  1. macroparameters by Op5 convolutions (Alg. 2, its moment part);
  2. f_S directly in Tucker form (rank 4 per mode);
  3. boundary ghosts in Tucker form (rank-1 Maxwellians, the cell itself,
     the cell with one factor's rows reversed, the scaled wall Maxwellian);
  4. the update f + dt R as a sum of terms: (1 - dt nu) f, dt nu f_S and,
     per face, -(dt A/V) P_out o f and -(dt A/V) P_in o g (Op3 products);
  5. one Op4 rounding of the Op2 sum of those terms.
In exact arithmetic this equals O1 (the same tensor is rounded).  step_faces
is the variant with the paper's intermediate roundings: each face's pair of
terms rounded on its own before the final sum.
"""

import numpy as np

from . import kinetic as kin
from . import tucker as tk
from .fv import BC_INFLOW, BC_OUTFLOW, BC_SYM, BC_WALL, axis_of


def ghost_tucker(S, j, f):
    bc = S.bc(j)
    kind = bc["kind"]
    if kind == BC_INFLOW:
        return kin.maxwell_rank1(bc["n"], np.array(bc["u"]), bc["T"], S.xi, S.Rg)
    if kind == BC_OUTFLOW:
        return f
    if kind == BC_SYM:
        a = axis_of(S.mesh["face_normal"][j])
        if a < 0:
            raise ValueError("symmetry boundary needs an axis-aligned face")
        U = [u.copy() for u in f.U]
        U[a] = U[a][::-1].copy()
        return tk.Tucker(f.G.copy(), U)
    if kind == BC_WALL:
        fw1 = kin.maxwell_rank1(1.0, np.zeros(3), bc["Tw"], S.xi, S.Rg)
        pout, pin = S.p_terms(j, 1.0)
        one = np.ones(S.N)
        num = tk.convolve(tk.hadamard(pout, f), one, one, one)
        den = tk.convolve(tk.hadamard(pin, fw1), one, one, one)
        return fw1.scaled(-num / den)
    raise ValueError(f"unknown boundary kind {kind}")


def grouped_terms(S, i, get):
    """The terms of f* for cell i grouped by origin: the cell's own terms
    [(1 - dt nu) f, dt nu f_S], then per face the pair
    [-(dt A/V) P_out o f, -(dt A/V) P_in o g]; and the macros of f_i."""
    mesh = S.mesh
    f = get(i)
    n, u, T, q = kin.macros_tucker(f, S.xi, S.dxi, S.Rg, S.m)
    nu = kin.collision_freq(n, T, S.Kn, S.omega, S.Rg, S.m)
    fs = kin.fs_tucker(n, u, T, q, S.xi, S.Pr, S.Rg, S.m)
    dt = S.dt
    own = [f.scaled(1.0 - dt * nu), fs.scaled(dt * nu)]
    faces = []
    V = mesh["cell_volume"][i]
    for j, s in S.cell_faces[i]:
        c = -dt * mesh["face_area"][j] / V
        pout, pin = S.p_terms(j, s)
        nb = mesh["face_right"][j] if s > 0 else mesh["face_left"][j]
        g = get(nb) if nb >= 0 else ghost_tucker(S, j, f)
        faces.append([tk.hadamard(pout, f).scaled(c), tk.hadamard(pin, g).scaled(c)])
    return own, faces, (n, u, T, q)


def update_terms(S, i, get):
    """The Tucker terms whose sum is f* for cell i, and the macros of f_i."""
    own, faces, mac = grouped_terms(S, i, get)
    return own + [t for pair in faces for t in pair], mac


def step(S, states, cells=None):
    """One O2 step; states: dict/array cell -> Tucker.  Returns dict."""
    get = (lambda c: states[c])
    if cells is None:
        cells = range(S.mesh["n_cells"])
    out = {}
    for i in cells:
        terms, _ = update_terms(S, i, get)
        out[i] = tk.round_sum(terms, S.tol, S.cap)
    return out


def step_faces(S, states, cells=None):
    """The step with the paper's intermediate rounding placement (Section
    "Tensorized discrete velocity method": a rounding after each operation
    that can raise the ranks a lot): each face's flux term, the Op2 sum of
    its two Op3 products (ranks of P_out, P_in times those of f, g), is
    rounded to the relative accuracy eps and the cap on its own; the
    rounded face terms are then summed with the cell's own terms and the sum
    rounded once more.  With eps -> 0 it is the step above."""
    get = (lambda c: states[c])
    if cells is None:
        cells = range(S.mesh["n_cells"])
    out = {}
    for i in cells:
        own, faces, _ = grouped_terms(S, i, get)
        rounded = [tk.round_sum(pair, S.tol, S.cap) for pair in faces]
        out[i] = tk.round_sum(own + rounded, S.tol, S.cap)
    return out


def initial_states(S, macros0, cells=None):
    if cells is None:
        cells = range(S.mesh["n_cells"])
    return {i: kin.maxwell_rank1(macros0[i, 0], macros0[i, 1:4], macros0[i, 4], S.xi, S.Rg)
            for i in cells}


def run(S, macros0, steps):
    st = initial_states(S, macros0)
    for _ in range(steps):
        st = step(S, st)
    return st


def cone(S, targets, steps):
    """Cells needed at each level to advance `targets` by `steps` steps.

    Level s (0..steps) holds every cell within graph distance steps - s of a
    target; advancing level s-1 -> s only reads cells of level s-1.
    """
    levels = [set(int(t) for t in targets)]
    for _ in range(steps):
        cur = set(levels[0])
        for c in levels[0]:
            cur.update(S.neighbours(c))
        levels.insert(0, cur)
    return [sorted(l) for l in levels]


def run_cone(S, macros0, targets, steps, full_path=False, faces=False):
    """Advance only the dependency cone of `targets`; O2 (or O1) states
    (faces: the intermediate-rounding step, step_faces)."""
    from . import dvm
    levels = cone(S, targets, steps)
    if full_path:
        F = dvm.initial_full(S, macros0, levels[0])
        for s in range(1, steps + 1):
            st = dvm.step_full(S, F, levels[s])
            F = {i: tk.full(t) for i, t in st.items()}
            last = st
        return last if steps else {i: tk.hosvd(F[i], 0.0, S.N) for i in levels[0]}
    st = initial_states(S, macros0, levels[0])
    adv = step_faces if faces else step
    for s in range(1, steps + 1):
        st = adv(S, st, levels[s])
    return st


def macros_of(S, t):
    """(n, u1, u2, u3, T, q1, q2, q3) of a Tucker state."""
    n, u, T, q = kin.macros_tucker(t, S.xi, S.dxi, S.Rg, S.m)
    return np.array([n, u[0], u[1], u[2], T, q[0], q[1], q[2]])
