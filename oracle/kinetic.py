"""Velocity grid, macroparameters and the S-model operator (oracle).

TEST INFRASTRUCTURE ONLY.

Velocity grid (Section "Discrete velocity method"): uniform nodes
xi_i = -xi_max + i dxi, i = 0..N-1, dxi = 2 xi_max / (N-1), the same in all
three axes; quadrature weight dxi^3 at every node (no end-point halving).

Macroparameters (model equations; Alg. 2): n, u, T from the raw moments
(T = (int xi^2 f - n u^2) / (3 n R_g)), q = m/2 int v v^2 f with v = xi - u.

S-model (eq. shakhov_integral).  The printed coefficient of the heat-flux
correction is dimensionally inconsistent; the reading used here is
A_s = 2 (1 - Pr) / (5 m n (R_g T)^2), the standard Shakhov form, chosen so
that the heat flux of f_S equals (1 - Pr) q (checked in the tests).

Collision frequency nu = p / mu(T) with p = m n R_g T and the power law
mu(T) = mu_ref T^omega; the nondimensional reading mu_ref = Kn / 2 (with
R_g = 1/2, m = 1) gives nu = n T^(1-omega) / Kn.
"""

import numpy as np

from . import tucker as tk


def grid(N, xi_max):
    dxi = 2.0 * xi_max / (N - 1)
    return -xi_max + np.arange(N) * dxi, dxi


def _axes(xi):
    return xi[:, None, None], xi[None, :, None], xi[None, None, :]


def macros_full(F, xi, dxi, Rg=0.5, m=1.0):
    """Alg. 2 on a full N^3 tensor: returns (n, u[3], T, q[3])."""
    w = dxi ** 3
    X = _axes(xi)
    n = w * F.sum()
    u = np.array([w * (X[a] * F).sum() / n for a in range(3)])
    u2 = float((u * u).sum())
    xi2 = X[0] ** 2 + X[1] ** 2 + X[2] ** 2
    T = (w * (xi2 * F).sum() - n * u2) / (3.0 * n * Rg)
    v = [X[a] - u[a] for a in range(3)]
    v2 = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
    q = np.array([0.5 * m * w * (v[a] * v2 * F).sum() for a in range(3)])
    return float(n), u, float(T), q


def maxwell_full(n, u, T, xi, Rg=0.5):
    X = _axes(xi)
    v2 = sum((X[a] - u[a]) ** 2 for a in range(3))
    return n / (2.0 * np.pi * Rg * T) ** 1.5 * np.exp(-v2 / (2.0 * Rg * T))


def shakhov_coef(n, T, Pr, Rg=0.5, m=1.0):
    return 2.0 * (1.0 - Pr) / (5.0 * m * n * (Rg * T) ** 2)


def fs_full(n, u, T, q, xi, Pr, Rg=0.5, m=1.0):
    """f_S = f_M [1 + A_s (q.v) (v^2/(2 R_g T) - 5/2)] on the full grid."""
    X = _axes(xi)
    v = [X[a] - u[a] for a in range(3)]
    v2 = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
    qv = q[0] * v[0] + q[1] * v[1] + q[2] * v[2]
    fm = maxwell_full(n, u, T, xi, Rg)
    return fm * (1.0 + shakhov_coef(n, T, Pr, Rg, m) * qv * (v2 / (2.0 * Rg * T) - 2.5))


def collision_freq(n, T, Kn, omega, Rg=0.5, m=1.0):
    p = m * n * Rg * T
    mu = 0.5 * Kn * T ** omega
    return p / mu


def maxwell_rank1(n, u, T, xi, Rg=0.5):
    """Rank-1 Maxwellian: U_a(i) = n^(1/3) (2 pi R_g T)^(-1/2) exp(-(xi_i-u_a)^2/(2 R_g T))."""
    c = n ** (1.0 / 3.0) / np.sqrt(2.0 * np.pi * Rg * T)
    U = [c * np.exp(-(xi - u[a]) ** 2 / (2.0 * Rg * T)) for a in range(3)]
    return tk.tucker_rank1(U[0], U[1], U[2])


def macros_tucker(t, xi, dxi, Rg=0.5, m=1.0):
    """Macroparameters of a Tucker tensor by Op5 convolutions (Alg. 2)."""
    w = dxi ** 3
    one = np.ones_like(xi)
    W = lambda a, v: [v if b == a else one for b in range(3)]  # noqa: E731
    n = w * tk.convolve(t, one, one, one)
    u = np.array([w * tk.convolve(t, *W(a, xi)) / n for a in range(3)])
    E = sum(w * tk.convolve(t, *W(a, xi * xi)) for a in range(3))
    T = (E - n * float((u * u).sum())) / (3.0 * n * Rg)
    q = np.zeros(3)
    for a in range(3):
        va = xi - u[a]
        acc = tk.convolve(t, *W(a, va ** 3))
        for b in range(3):
            if b == a:
                continue
            vb = xi - u[b]
            ws = [one, one, one]
            ws[a] = va
            ws[b] = vb * vb
            acc += tk.convolve(t, *ws)
        q[a] = 0.5 * m * w * acc
    return float(n), u, float(T), q


def fs_tucker(n, u, T, q, xi, Pr, Rg=0.5, m=1.0):
    """f_S in Tucker form with mode ranks 4.

    Factors: column k of mode a is f_M's 1-D factor times v_a^k (k = 0..3).
    Expanding f_M [1 + A_s sum_a q_a v_a (beta v^2 - 5/2)], beta = 1/(2 R_g T),
    gives the monomials 1, v_a, v_a^3 and v_a v_c^2 (c != a), i.e. a core
    with 13 non-zeros.  (Proposition 1 bounds the ranks by 5.)
    """
    fm = maxwell_rank1(n, u, T, xi, Rg)
    A = shakhov_coef(n, T, Pr, Rg, m)
    beta = 1.0 / (2.0 * Rg * T)
    U = []
    for a in range(3):
        v = xi - u[a]
        base = fm.U[a][:, 0]
        U.append(np.stack([base, base * v, base * v ** 2, base * v ** 3], 1))
    G = np.zeros((4, 4, 4))
    G[0, 0, 0] = 1.0
    for a in range(3):
        idx = [0, 0, 0]
        idx[a] = 1
        G[tuple(idx)] += -2.5 * A * q[a]
        idx = [0, 0, 0]
        idx[a] = 3
        G[tuple(idx)] += A * beta * q[a]
        for c in range(3):
            if c == a:
                continue
            idx = [0, 0, 0]
            idx[a] = 1
            idx[c] = 2
            G[tuple(idx)] += A * beta * q[a]
    return tk.Tucker(G, U)
