"""Pins of the oracle's velocity grid, macroparameters and S-model."""

import numpy as np
import pytest

from oracle import kinetic as kin
from oracle import tucker as tk

RG, M = 0.5, 1.0


def mixture(xi, comps):
    return sum(kin.maxwell_full(n, np.array(u), T, xi, RG) for n, u, T in comps)


def mixture_closed_form(comps):
    """n, u, T, q of a sum of Maxwellians (exact Gaussian moments).

    For a component with density n_k, mean w_k, temperature T_k and
    d = w_k - u: int v v^2 f_k = n_k d (5 R T_k + |d|^2); the energy is
    sum n_k (3 R T_k + |d|^2) = 3 n R T.
    """
    n = sum(c[0] for c in comps)
    u = sum(c[0] * np.array(c[1]) for c in comps) / n
    e = sum(c[0] * (3 * RG * c[2] + ((np.array(c[1]) - u) ** 2).sum()) for c in comps)
    T = e / (3 * n * RG)
    q = 0.5 * M * sum(c[0] * (np.array(c[1]) - u) * (5 * RG * c[2] + ((np.array(c[1]) - u) ** 2).sum())
                      for c in comps)
    return n, u, T, q


def test_grid_nodes():
    xi, dxi = kin.grid(16, 4.5)
    assert xi[0] == -4.5 and abs(xi[-1] - 4.5) < 1e-14
    assert abs(dxi - 9.0 / 15) < 1e-15
    np.testing.assert_allclose(xi + xi[::-1], 0.0, atol=1e-14)


@pytest.mark.parametrize("N,xmax,tol", [(96, 9.0, 1e-11), (16, 4.5, 3e-7), (32, 6.0, 1e-8)])
def test_maxwellian_moments_closed_form(N, xmax, tol):
    xi, dxi = kin.grid(N, xmax)
    n, u, T = 1.2, np.array([0.3, -0.1, 0.05]), 1.1
    F = kin.maxwell_full(n, u, T, xi, RG)
    n2, u2, T2, q2 = kin.macros_full(F, xi, dxi, RG, M)
    assert abs(n2 - n) / n < tol
    assert np.abs(u2 - u).max() / np.sqrt(2 * RG * T) < tol
    assert abs(T2 - T) / T < tol * 20
    assert np.abs(q2).max() / (n * RG * T * np.sqrt(2 * RG * T)) < tol * 20


def test_zero_mean_maxwellian_has_exactly_zero_flux():
    xi, dxi = kin.grid(16, 4.5)
    F = kin.maxwell_full(1.0, np.zeros(3), 1.0, xi, RG)
    n, u, T, q = kin.macros_full(F, xi, dxi, RG, M)
    assert np.abs(u).max() < 1e-15 and np.abs(q).max() < 1e-15


def test_heat_flux_closed_form_mixture():
    xi, dxi = kin.grid(96, 9.0)
    comps = [(0.7, (0.4, -0.2, 0.1), 0.9), (0.5, (-0.3, 0.25, 0.0), 1.3)]
    F = mixture(xi, comps)
    n, u, T, q = kin.macros_full(F, xi, dxi, RG, M)
    n0, u0, T0, q0 = mixture_closed_form(comps)
    assert abs(n - n0) < 1e-11 and np.abs(u - u0).max() < 1e-11
    assert abs(T - T0) < 1e-10 and np.abs(q - q0).max() < 1e-10
    assert np.abs(q0).max() > 1e-2  # non-trivial heat flux


def test_rank1_maxwellian_pointwise():
    xi, dxi = kin.grid(16, 4.5)
    n, u, T = 0.9, np.array([0.2, 0.0, -0.3]), 1.05
    np.testing.assert_allclose(tk.full(kin.maxwell_rank1(n, u, T, xi, RG)),
                               kin.maxwell_full(n, u, T, xi, RG), rtol=1e-13, atol=1e-17)


def test_macros_tucker_equal_full():
    xi, dxi = kin.grid(20, 5.0)
    comps = [(0.7, (0.4, -0.2, 0.1), 0.9), (0.5, (-0.3, 0.25, 0.0), 1.3)]
    F = mixture(xi, comps)
    t = tk.hosvd(F, 0.0, 20)
    a = kin.macros_full(F, xi, dxi, RG, M)
    b = kin.macros_tucker(t, xi, dxi, RG, M)
    assert abs(a[0] - b[0]) < 1e-13 and abs(a[2] - b[2]) < 1e-12
    np.testing.assert_allclose(a[1], b[1], atol=1e-13)
    np.testing.assert_allclose(a[3], b[3], atol=1e-12)


def test_fs_tucker_pointwise_and_rank():
    xi, dxi = kin.grid(16, 4.5)
    n, u, T, q = 1.1, np.array([0.1, -0.2, 0.05]), 0.95, np.array([0.03, -0.02, 0.01])
    t = kin.fs_tucker(n, u, T, q, xi, 2 / 3, RG, M)
    assert t.ranks == (4, 4, 4) and int((t.G != 0).sum()) == 13
    np.testing.assert_allclose(tk.full(t), kin.fs_full(n, u, T, q, xi, 2 / 3, RG, M),
                               rtol=1e-12, atol=1e-16)
    # Proposition 1 bound: mode ranks <= 5 (here numerically 4)
    assert max(tk.hosvd(tk.full(t), 1e-13, 16).ranks) <= 5


def test_shakhov_coefficient_reading():
    # heat flux of f_S equals (1 - Pr) q and n, u, T are preserved; the
    # printed coefficient would give 0.375 instead of 1/3 at n = 1.5
    xi, dxi = kin.grid(96, 9.0)
    n, u, T, q = 1.5, np.array([0.2, -0.1, 0.3]), 1.2, np.array([0.05, -0.03, 0.02])
    Pr = 2.0 / 3.0
    F = kin.fs_full(n, u, T, q, xi, Pr, RG, M)
    n2, u2, T2, q2 = kin.macros_full(F, xi, dxi, RG, M)
    np.testing.assert_allclose(q2 / q, 1 - Pr, rtol=1e-8)
    assert abs(n2 - n) < 1e-11 and np.abs(u2 - u).max() < 1e-11 and abs(T2 - T) < 1e-10


def test_collision_conserves():
    xi, dxi = kin.grid(16, 4.5)
    comps = [(0.7, (0.4, -0.2, 0.1), 0.9), (0.5, (-0.3, 0.25, 0.0), 1.3)]
    F = mixture(xi, comps)
    n, u, T, q = kin.macros_full(F, xi, dxi, RG, M)
    nu = kin.collision_freq(n, T, 0.1, 0.5, RG, M)
    J = nu * (kin.fs_full(n, u, T, q, xi, 2 / 3, RG, M) - F)
    w = dxi ** 3
    X = np.meshgrid(xi, xi, xi, indexing="ij")
    scale = nu * n
    assert abs(w * J.sum()) / scale < 1e-8
    for a in range(3):
        assert abs(w * (X[a] * J).sum()) / scale < 1e-8
    assert abs(w * ((X[0] ** 2 + X[1] ** 2 + X[2] ** 2) * J).sum()) / scale < 1e-8


def test_collision_frequency_reading():
    assert abs(kin.collision_freq(1.2, 1.1, 0.1, 0.5) - 1.2 * 1.1 ** 0.5 / 0.1) < 1e-12
    assert kin.collision_freq(1.0, 1.0, np.inf, 0.5) == 0.0
