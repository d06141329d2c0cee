"""Pins of the oracle's finite-volume step (O1 brute force, O2 Tucker form)."""

import numpy as np
import pytest

import synth
from oracle import dvm, fv, kinetic as kin, tucker as tk, tucker_dvm as td


def small_cfg(**kw):
    cfg = dict(N=8, xi_max=4.0, cap=4, tol=1e-6, cfl=0.5, Pr=2 / 3, omega=0.5, Kn=0.1,
               Rg=0.5, m=1.0, seed=0, init="random")
    cfg.update(kw)
    return cfg


def closed_channel():
    m = synth.channel_with_obstacle(nx=6, ny=4, nz=4, h=0.25,
                                    obstacle=((2, 3), (1, 2), (1, 3)))
    return m


def open_channel():
    return synth.channel_with_obstacle(nx=6, ny=4, nz=4, h=0.25,
                                       obstacle=((2, 3), (1, 2), (1, 3)),
                                       inflow=(1.0, (0.8, 0.0, 0.0), 1.0), Tw=1.3)


def total_mass(S, F):
    w = S.dxi ** 3
    return sum(S.mesh["cell_volume"][i] * w * F[i].sum() for i in F)


def test_axis_upwind_split_is_exact():
    S = fv.Setup(synth.periodic_box(4), small_cfg(), synth.initial_macros(small_cfg(), synth.periodic_box(4)))
    for j in (0, 70, 150):
        for s in (1.0, -1.0):
            po, pi = S.p_terms(j, s)
            a = fv.axis_of(S.mesh["face_normal"][j])
            sig = s * S.mesh["face_normal"][j][a]
            X = S.xin_full(j) * s
            np.testing.assert_array_equal(tk.full(po), np.maximum(X, 0.0))
            np.testing.assert_array_equal(tk.full(pi), np.minimum(X, 0.0))
            assert po.ranks == (1, 1, 1) and sig in (1.0, -1.0)


def test_estimate_axis_rank1_and_oblique_bound():
    xi, _ = kin.grid(16, 4.5)
    A = np.abs(xi)[None, :, None] * np.ones((16, 1, 16))
    t = tk.hosvd(A, 0.0, 6, drop_rel=1e-14)
    assert t.ranks == (1, 1, 1)
    np.testing.assert_allclose(tk.full(t), A, atol=1e-13)
    rng = np.random.default_rng(0)
    e = rng.standard_normal(3)
    e /= np.linalg.norm(e)
    X = np.abs(e[0] * xi[:, None, None] + e[1] * xi[None, :, None] + e[2] * xi[None, None, :])
    t, sig = tk.hosvd(X, 0.0, 6, drop_rel=1e-14, return_sigma=True)
    assert t.ranks == (6, 6, 6)
    err2 = np.linalg.norm(tk.full(t) - X) ** 2
    assert err2 <= sum((s[6:] ** 2).sum() for s in sig) * (1 + 1e-10)
    assert np.sqrt(err2) / np.linalg.norm(X) < 0.05


def test_flux_consistency_any_estimate():
    # F(f, f) = xi_n f whatever estimate replaces |xi_n|
    mesh = synth.jittered_box(3, 3, 3, 1 / 3, seed=1)
    cfg = small_cfg()
    S = fv.Setup(mesh, cfg, synth.initial_macros(cfg, mesh))
    xi = S.xi
    f = kin.maxwell_full(1.0, np.array([0.2, 0.1, 0.0]), 1.0, xi)
    j = int(np.nonzero(mesh["face_right"] >= 0)[0][0])
    xn, est = S.xin_full(j), S.estimate_full(j)
    Fj = 0.5 * xn * (f + f) - 0.5 * est * (f - f)
    np.testing.assert_allclose(Fj, xn * f, rtol=1e-15, atol=0)


def test_one_dimensional_upwind_textbook():
    # fields varying along x only, no collisions: the step is the textbook
    # first-order upwind scheme along x (y and z fluxes cancel)
    n = 4
    mesh = synth.periodic_box(n)
    cfg = small_cfg(Kn=np.inf)
    m0 = np.zeros((n ** 3, 5))
    ii = np.arange(n ** 3) % n
    m0[:, 0] = 1.0 + 0.2 * np.sin(2 * np.pi * ii / n)
    m0[:, 1] = 0.3 * np.cos(2 * np.pi * ii / n)
    m0[:, 4] = 1.0 + 0.1 * ii
    S = fv.Setup(mesh, cfg, m0)
    F = dvm.initial_full(S, m0)
    h = 1.0 / n
    lam = S.dt / h
    ap = np.maximum(S.xi, 0.0)[:, None, None]
    am = np.minimum(S.xi, 0.0)[:, None, None]
    for i in (0, 5, 22):
        X = dvm.update_full(S, i, lambda c: F[c])
        il, ir = (i // n) * n + (i - 1) % n, (i // n) * n + (i + 1) % n
        ref = F[i] - lam * (ap * (F[i] - F[il]) + am * (F[ir] - F[i]))
        np.testing.assert_allclose(X, ref, rtol=0, atol=1e-14 * np.abs(F[i]).max())


@pytest.mark.parametrize("kind", ["periodic", "jittered", "walls"])
def test_transport_conserves_mass(kind):
    if kind == "periodic":
        mesh = synth.periodic_box(3)
    elif kind == "jittered":
        mesh = synth.jittered_box(3, 3, 3, 1 / 3, seed=5)
    else:
        mesh = closed_channel()
        mesh["bc"][0] = dict(mesh["bc"][2])
        mesh["bc"][1] = dict(mesh["bc"][2])
    cfg = small_cfg(Kn=np.inf, tol=0.0, cap=8)
    m0 = synth.initial_macros(cfg, mesh)
    S = fv.Setup(mesh, cfg, m0)
    F = dvm.initial_full(S, m0)
    M0 = total_mass(S, F)
    X = {i: dvm.update_full(S, i, lambda c: F[c]) for i in F}
    assert abs(total_mass(S, X) - M0) / M0 < 1e-13


def test_wall_and_symmetry_carry_no_mass():
    mesh = open_channel()
    cfg = small_cfg()
    m0 = synth.initial_macros(dict(cfg, init="random"), mesh)
    S = fv.Setup(mesh, cfg, m0)
    F = dvm.initial_full(S, m0)
    w = S.dxi ** 3
    seen = set()
    for j in np.nonzero(mesh["face_right"] < 0)[0]:
        kind = S.bc(j)["kind"]
        if kind not in (fv.BC_WALL, fv.BC_SYM):
            continue
        fL = F[mesh["face_left"][j]]
        g = dvm.ghost_full(S, j, fL)
        Fj = 0.5 * S.xin_full(j) * (fL + g) - 0.5 * S.estimate_full(j) * (g - fL)
        assert abs(w * Fj.sum()) < 1e-14
        if kind == fv.BC_WALL:
            n, u, T, q = kin.macros_full(g, S.xi, S.dxi)
            assert abs(T - 1.3) < 1e-2 and np.abs(u).max() < 1e-12
        seen.add(kind)
    assert seen == {fv.BC_WALL, fv.BC_SYM}


def test_uniform_maxwellian_is_steady():
    # the cfg0 grid and cell size on a 3^3 periodic box (every cell of a
    # uniform state sees the same update whatever the box size)
    cfg = synth.make_config("cfg0", init="uniform")
    mesh = synth.periodic_box(3, length=3.0 / 8.0)
    m0 = synth.initial_macros(cfg, mesh)
    S = fv.Setup(mesh, cfg, m0)
    st = td.initial_states(S, m0)
    ref = td.macros_of(S, st[0])
    for _ in range(20):
        st = td.step(S, st)
    for i in (0, 13, 26):
        assert st[i].ranks == (1, 1, 1)
        m = td.macros_of(S, st[i])
        assert abs(m[0] - ref[0]) / ref[0] < 1e-9
        assert abs(m[4] - ref[4]) / ref[4] < 1e-9
        # u relative to the thermal speed, q to p sqrt(2 R_g T)
        assert np.abs(m[1:4]).max() < 1e-14 and np.abs(m[5:]).max() / 0.5 < 1e-14


def test_full_rank_tucker_step_equals_full_step():
    mesh = open_channel()
    cfg = small_cfg(tol=0.0, cap=8)
    m0 = synth.initial_macros(dict(cfg, init="random"), mesh)
    S = fv.Setup(mesh, cfg, m0)
    F = dvm.initial_full(S, m0)
    st = td.initial_states(S, m0)
    out = td.step(S, st)
    for i in range(mesh["n_cells"]):
        X = dvm.update_full(S, i, lambda c: F[c])
        np.testing.assert_allclose(tk.full(out[i]), X, rtol=0, atol=1e-12 * np.abs(X).max())


@pytest.mark.parametrize("meshkind", ["periodic", "channel", "jittered"])
def test_truncated_tucker_step_equals_hosvd_of_full_step(meshkind):
    if meshkind == "periodic":
        mesh = synth.periodic_box(4)
    elif meshkind == "channel":
        mesh = open_channel()
    else:
        mesh = synth.jittered_box(3, 3, 3, 1 / 3, seed=3)
    cfg = small_cfg(N=10, cap=4, tol=1e-6)
    m0 = synth.initial_macros(cfg, mesh)
    S = fv.Setup(mesh, cfg, m0)
    st = td.initial_states(S, m0)
    F = dvm.initial_full(S, m0)
    for _ in range(2):
        o2 = td.step(S, st)
        o1 = dvm.step_full(S, F)
        for i in range(mesh["n_cells"]):
            assert o1[i].ranks == o2[i].ranks
            a, b = tk.full(o1[i]), tk.full(o2[i])
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-11 * np.abs(a).max())
        st = o2
        F = {i: tk.full(t) for i, t in o1.items()}


def test_cone_matches_full_run():
    mesh = open_channel()
    cfg = small_cfg(N=8, cap=3)
    m0 = synth.initial_macros(cfg, mesh)
    S = fv.Setup(mesh, cfg, m0)
    ref = td.run(S, m0, 2)
    got = td.run_cone(S, m0, [0, 17, mesh["n_cells"] - 1], 2)
    for i in got:
        np.testing.assert_allclose(tk.full(got[i]), tk.full(ref[i]), rtol=0, atol=1e-14)


def test_time_step_reading():
    cfg = synth.make_config("cfg0")
    mesh = synth.configs.make_mesh(cfg)
    m0 = synth.initial_macros(cfg, mesh)
    S = fv.Setup(mesh, cfg, m0)
    nu0 = (m0[:, 0] * m0[:, 4] ** 0.5 / 0.1).max()
    assert abs(S.dt - 0.5 / (3 * 4.5 * 8 + nu0)) < 1e-15


def _mixture_box():
    """A spatially uniform periodic box whose f is a two-Maxwellian mixture.

    Transport cancels exactly on a uniform periodic state, so one step is
    f' = f + dt J(f) in every cell.  With J = nu (f_S - f) (eq.
    shakhov_integral) and the heat flux of f_S equal to (1 - Pr) q, the
    step keeps n, u, T and scales the heat flux by 1 - dt nu Pr.  The grid
    (N = 48 on [-7, 7]) integrates these Gaussians to about 1e-15.
    """
    comps = [(0.7, (0.4, -0.2, 0.1), 0.9), (0.5, (-0.3, 0.25, 0.0), 1.3)]
    cfg = small_cfg(N=48, xi_max=7.0, Kn=0.05, tol=0.0, cap=8)
    mesh = synth.periodic_box(3, length=6.0)
    xi, dxi = kin.grid(48, 7.0)
    full = sum(kin.maxwell_full(n, np.array(u), T, xi) for n, u, T in comps)
    parts = [kin.maxwell_rank1(n, np.array(u), T, xi) for n, u, T in comps]
    tuck = tk.add(parts[0], parts[1])
    n, u, T, q = kin.macros_full(full, xi, dxi)
    m0 = np.tile(np.array([n, *u, T]), (mesh["n_cells"], 1))
    S = fv.Setup(mesh, cfg, m0)
    # nu = p / mu with p = m n R_g T and mu = (Kn / 2) T^omega (a reading:
    # the paper is dimensional; parity unpinned beyond its role as the rate)
    nu = n * 0.5 * T / (0.5 * cfg["Kn"] * T ** cfg["omega"])
    return S, full, tuck, (n, u, T, q), nu


def _check_collision_step(S, macros_after, before, nu):
    n, u, T, q = before
    n1, u1, T1, q1 = macros_after
    c = np.sqrt(T)
    assert abs(n1 - n) / n < 1e-13
    assert np.abs(u1 - u).max() / c < 1e-13
    assert abs(T1 - T) / T < 1e-13
    expect = (1.0 - S.dt * nu * S.Pr) * q
    assert 0.2 < S.dt * nu < 0.6  # the collision term moves q well beyond the tolerance
    np.testing.assert_allclose(q1, expect, rtol=1e-12, atol=1e-12 * np.abs(q).max())


def test_collision_step_direction_and_rate_full():
    """O1: f' = f + dt nu (f_S - f) on a uniform mixture: n, u, T kept, q' = (1 - dt nu Pr) q."""
    S, full, _, before, nu = _mixture_box()
    F = {i: full for i in range(S.mesh["n_cells"])}
    for i in (0, 5):
        X = dvm.update_full(S, i, lambda c: F[c])
        _check_collision_step(S, kin.macros_full(X, S.xi, S.dxi), before, nu)
    out = dvm.step_full(S, F, cells=[3])
    _check_collision_step(S, kin.macros_tucker(out[3], S.xi, S.dxi), before, nu)


def test_collision_step_direction_and_rate_tucker():
    """O2: the same step in Tucker form (exact rounding, tol 0)."""
    S, _, tuck, before, nu = _mixture_box()
    st = {i: tuck for i in range(S.mesh["n_cells"])}
    out = td.step(S, st, cells=[0, 13])
    for i in (0, 13):
        _check_collision_step(S, kin.macros_tucker(out[i], S.xi, S.dxi), before, nu)


def test_exact_flux_is_the_upwind_choice_per_node():
    """dvm with exact=True (the standard DVM baseline): on a jittered mesh
    each face takes, per velocity node, xi_n f_L where xi_n > 0 and xi_n f_R
    otherwise (written out with a branch per node); mass is conserved in
    the closed box; on an axis mesh the result equals the estimate path."""
    mesh = synth.jittered_box(3, 3, 3, 1 / 3, seed=4)
    cfg = small_cfg(Kn=0.2)
    m0 = synth.initial_macros(cfg, mesh)
    S = fv.Setup(mesh, cfg, m0)
    F = dvm.initial_full(S, m0)
    get = (lambda c: F[c])
    xi = S.xi
    for i in (0, 13, 26):
        X = dvm.update_full(S, i, get, exact=True)
        n, u, T, q = kin.macros_full(F[i], xi, S.dxi, S.Rg, S.m)
        nu = kin.collision_freq(n, T, S.Kn, S.omega, S.Rg, S.m)
        ref = F[i] + S.dt * nu * (kin.fs_full(n, u, T, q, xi, S.Pr, S.Rg, S.m) - F[i])
        V = mesh["cell_volume"][i]
        for j, s in S.cell_faces[i]:
            L, R = mesh["face_left"][j], mesh["face_right"][j]
            e = mesh["face_normal"][j]
            fL = F[L]
            fR = F[R] if R >= 0 else dvm.ghost_full(S, j, fL)
            Fj = np.empty_like(fL)
            for p in np.ndindex(fL.shape):
                x = e[0] * xi[p[0]] + e[1] * xi[p[1]] + e[2] * xi[p[2]]
                Fj[p] = x * (fL[p] if x > 0 else fR[p])
            ref = ref - S.dt * s * mesh["face_area"][j] / V * Fj
        np.testing.assert_allclose(X, ref, rtol=0, atol=1e-14 * np.abs(F[i]).max())
    cfg0 = small_cfg(Kn=np.inf)
    S0 = fv.Setup(mesh, cfg0, m0)
    M0 = total_mass(S0, F)
    X = {i: dvm.update_full(S0, i, get, exact=True) for i in F}
    assert abs(total_mass(S0, X) - M0) / M0 < 1e-13
    pm = synth.periodic_box(3)
    Sp = fv.Setup(pm, cfg, synth.initial_macros(cfg, pm))
    Fp = dvm.initial_full(Sp, synth.initial_macros(cfg, pm))
    for i in (0, 7):
        a = dvm.update_full(Sp, i, lambda c: Fp[c], exact=True)
        b = dvm.update_full(Sp, i, lambda c: Fp[c])
        assert np.array_equal(a, b)
