"""Finite-volume setup shared by the two oracle levels (oracle).

TEST INFRASTRUCTURE ONLY.

Semi-discrete scheme (eq. ode_system) with the first-order flux of
eq. exact-flux, where |xi_n| may be replaced by an estimate (the paper's
Rusanov-type remark).  Readings used here:

* |xi_n| estimate: on faces whose normal is a coordinate axis, the exact
  |xi_a| (rank 1).  On other faces, the truncated HOSVD of the exact tensor
  |xi . e| with mode ranks capped at 6 (the paper's rank) and singular
  values <= 1e-14 sigma_1 dropped.  P+ = (xi_n + est)/2, P- = (xi_n - est)/2.
* Gather form: for cell i and face l with outward normal s e_j,
  -(A/V) sign F_j = -(A/V) (P_out f_i + P_in f_nb) with
  P_out = (s xi.e + est)/2, P_in = (s xi.e - est)/2; identical to Alg. 1.
* Boundary ghosts (Section "Mathematical model", boundary conditions):
  free stream -> Maxwellian of the given macroparameters; zero-gradient
  outflow -> the cell's own f; symmetry plane (axis-aligned only) -> f
  with the normal velocity index reversed; diffuse wall -> n_w f_w1 with
  f_w1 the unit-density wall Maxwellian and n_w = -<P_out, f>/<P_in, f_w1>
  (impermeability with the same P as the flux, so the wall mass flux is 0).
* Time step: dt = CFL / max_i (D_i + nu_i^0), D_i = xi_max/(2 V_i)
  sum_l A_l ||e_l||_1 (the explicit scheme's positivity bound), nu^0 from
  the input macroparameters; fixed for the run.
* Everything in a step is computed from f^n (explicit Euler, eq.
  expl-scheme-final).
"""

import numpy as np

from . import kinetic as kin
from . import tucker as tk

BC_SYM, BC_INFLOW, BC_OUTFLOW, BC_WALL = 0, 1, 2, 3


def axis_of(e):
    """Index of the coordinate axis e lies on, or -1 for an oblique normal."""
    nz = np.nonzero(np.asarray(e) != 0.0)[0]
    return int(nz[0]) if nz.shape[0] == 1 else -1


class Setup:
    """Mesh, velocity grid, physics and per-face data for one instance."""

    def __init__(self, mesh, cfg, macros0):
        self.mesh = mesh
        self.cfg = cfg
        self.N = int(cfg["N"])
        self.xi_max = float(cfg["xi_max"])
        self.xi, self.dxi = kin.grid(self.N, self.xi_max)
        self.Pr, self.omega, self.Kn = cfg["Pr"], cfg["omega"], cfg["Kn"]
        self.Rg, self.m = cfg.get("Rg", 0.5), cfg.get("m", 1.0)
        self.tol, self.cap = float(cfg["tol"]), int(cfg["cap"])
        nc = mesh["n_cells"]
        fl, fr = mesh["face_left"], mesh["face_right"]
        # per-cell face lists (face id, sign): sign +1 when the face normal
        # points out of the cell
        order = [[] for _ in range(nc)]
        for j in range(mesh["n_faces"]):
            order[fl[j]].append((j, 1.0))
            if fr[j] >= 0:
                order[fr[j]].append((j, -1.0))
        self.cell_faces = order
        self._est = {}
        self.dt = self._time_step(macros0, float(cfg["cfl"]))

    # ---- geometry / time step -------------------------------------------
    def _time_step(self, macros0, cfl):
        mesh = self.mesh
        D = np.zeros(mesh["n_cells"])
        l1 = np.abs(mesh["face_normal"]).sum(1) * mesh["face_area"]
        np.add.at(D, mesh["face_left"], l1)
        inner = mesh["face_right"] >= 0
        np.add.at(D, mesh["face_right"][inner], l1[inner])
        D *= self.xi_max / (2.0 * mesh["cell_volume"])
        nu0 = np.array([kin.collision_freq(m[0], m[4], self.Kn, self.omega, self.Rg, self.m)
                        for m in macros0])
        return cfl / float((D + nu0).max())

    def neighbours(self, i):
        fl, fr = self.mesh["face_left"], self.mesh["face_right"]
        out = []
        for j, s in self.cell_faces[i]:
            c = fr[j] if s > 0 else fl[j]
            if c >= 0:
                out.append(int(c))
        return out

    # ---- |xi_n| estimate ------------------------------------------------
    def estimate(self, j):
        """Tucker form of the |xi . e_j| estimate for face j."""
        if j in self._est:
            return self._est[j]
        e = self.mesh["face_normal"][j]
        a = axis_of(e)
        xi = self.xi
        if a >= 0:
            U = [np.ones(self.N) for _ in range(3)]
            U[a] = np.abs(xi)
            t = tk.tucker_rank1(*U)
        else:
            X = e[0] * xi[:, None, None] + e[1] * xi[None, :, None] + e[2] * xi[None, None, :]
            t = tk.hosvd(np.abs(X), 0.0, 6, drop_rel=1e-14)
        self._est[j] = t
        return t

    def estimate_full(self, j):
        return tk.full(self.estimate(j))

    def xin_full(self, j):
        e = self.mesh["face_normal"][j]
        xi = self.xi
        return e[0] * xi[:, None, None] + e[1] * xi[None, :, None] + e[2] * xi[None, None, :]

    def p_terms(self, j, s):
        """(P_out, P_in) of face j seen from the cell with orientation s."""
        e = self.mesh["face_normal"][j]
        a = axis_of(e)
        xi = self.xi
        if a >= 0:
            sig = s * e[a]
            Uo = [np.ones(self.N) for _ in range(3)]
            Ui = [np.ones(self.N) for _ in range(3)]
            Uo[a] = np.maximum(sig * xi, 0.0)
            Ui[a] = np.minimum(sig * xi, 0.0)
            return tk.tucker_rank1(*Uo), tk.tucker_rank1(*Ui)
        xn = tk.lemma1(s * e[0] * xi, s * e[1] * xi, s * e[2] * xi)
        est = self.estimate(j)
        return (tk.add(xn.scaled(0.5), est.scaled(0.5)),
                tk.add(xn.scaled(0.5), est.scaled(-0.5)))

    def bc(self, j):
        return self.mesh["bc"][-int(self.mesh["face_right"][j]) - 1]
