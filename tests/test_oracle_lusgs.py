"""Pins of the LU-SGS oracle (implicit scheme of the tensorised method:
eq. linear-system, eq. diagonal_term, eq. xin-one-rank-approx,
eq. one_rank_division), checked against the algebra they must satisfy,
not against the oracle's own formulas."""

import numpy as np
import pytest

import synth
from oracle import dvm, fv, kinetic as kin, lusgs, tucker as tk, tucker_dvm as td


def cfg_of(**kw):
    cfg = dict(N=6, xi_max=4.0, cap=6, tol=1e-6, cfl=4.0, Pr=2 / 3, omega=0.5, Kn=0.3,
               Rg=0.5, m=1.0, seed=3, init="random")
    cfg.update(kw)
    return cfg


def channel():
    return synth.channel_with_obstacle(nx=4, ny=3, nz=2, h=0.25, obstacle=((1, 2), (1, 2), (0, 1)),
                                       inflow=(1.0, (0.6, 0.0, 0.0), 1.0), Tw=1.4)


def setup(mesh, **kw):
    cfg = cfg_of(**kw)
    m0 = synth.initial_macros(cfg, mesh)
    return fv.Setup(mesh, cfg, m0), m0


def neighbours(mesh):
    nb = [set() for _ in range(mesh["n_cells"])]
    for L, R in zip(mesh["face_left"], mesh["face_right"]):
        if R >= 0 and R != L:
            nb[L].add(int(R))
            nb[R].add(int(L))
    return nb


@pytest.mark.parametrize("mesh,ncol", [(synth.periodic_box(4), 2), (synth.periodic_box(3), None),
                                       (channel(), None)])
def test_colouring_is_a_proper_colouring(mesh, ncol):
    col = lusgs.colouring(mesh)
    for i, nb in enumerate(neighbours(mesh)):
        assert all(col[m] != col[i] for m in nb)
    if ncol is not None:  # an even periodic box is bipartite: the greedy order finds 2 colours
        assert col.max() + 1 == ncol


def node_block(S, i, m, p):
    """B_im at velocity node p from the face list: (dt A / V) min(s xi_a, 0)
    summed over the faces between i and m (axis-aligned faces)."""
    mesh = S.mesh
    xi = S.xi
    tot = 0.0
    for j in range(mesh["n_faces"]):
        L, R = mesh["face_left"][j], mesh["face_right"][j]
        if R < 0:
            continue
        if L == i and R == m:
            s = 1.0
        elif R == i and L == m:
            s = -1.0
        else:
            continue
        e = mesh["face_normal"][j]
        a = int(np.nonzero(e)[0][0])
        tot += S.dt * mesh["face_area"][j] / mesh["cell_volume"][i] * min(s * e[a] * xi[p[a]], 0.0)
    return tot


@pytest.mark.parametrize("mesh", [synth.periodic_box(3), synth.periodic_box(4), channel()])
def test_sweeps_solve_the_factored_system(mesh):
    """(D + L) D^-1 (D + U) df = rhs per velocity node, with D, L, U built
    from the face list as dense matrices over the cells."""
    S, _ = setup(mesh, N=4)
    nc = mesh["n_cells"]
    rng = np.random.default_rng(5)
    D = {i: 1.0 + rng.random((4, 4, 4)) for i in range(nc)}
    rhs = {i: rng.standard_normal((4, 4, 4)) for i in range(nc)}
    col = lusgs.colouring(mesh)
    df = lusgs.sweeps_full(S, col, D, rhs)
    nb = neighbours(mesh)
    for p in [(0, 0, 0), (3, 1, 2), (1, 3, 0), (2, 2, 3)]:
        Md = np.diag([D[i][p] for i in range(nc)])
        Ml = np.zeros((nc, nc))
        Mu = np.zeros((nc, nc))
        for i in range(nc):
            for m in nb[i]:
                b = node_block(S, i, m, p)
                if col[m] < col[i]:
                    Ml[i, m] = b
                else:
                    Mu[i, m] = b
        x = np.array([df[i][p] for i in range(nc)])
        lhs = (Md + Ml) @ np.linalg.solve(Md, (Md + Mu) @ x)
        r = np.array([rhs[i][p] for i in range(nc)])
        assert np.allclose(lhs, r, rtol=0, atol=1e-12 * np.abs(r).max()), p


def test_rank1_division_is_exact():
    """Eq. one_rank_division: dividing the factors' rows equals the
    element-wise quotient of the full tensors."""
    S, m0 = setup(channel())
    rng = np.random.default_rng(1)
    A = tk.Tucker(rng.standard_normal((3, 2, 4)), [rng.standard_normal((6, r)) for r in (3, 2, 4)])
    for i in (0, 5):
        d = lusgs.diag_est(S, i, 0.7)
        got = tk.full(tk.divide_rank1(A, *lusgs.rank1_vectors(d)))
        ref = tk.full(A) / tk.full(d)
        assert np.allclose(got, ref, rtol=1e-13, atol=0)


def test_rank1_diagonal_is_the_hosvd_of_the_bound():
    """D_est's factor is the leading eigenvector of the mode-1 Gram of
    D = a 1 + b |xi|, written out as a^2 N^2 11^T + a b (1 p^T + p 1^T)
    + b^2 Q with p, Q from |xi| alone; its core is D x u x u x u; every
    entry is positive (so the division is defined) and D dominates the
    exact diagonal of eq. diagonal_term (|xi_n| <= |xi|)."""
    mesh = channel()
    S, _ = setup(mesh)
    N = S.N
    Sx = np.sqrt(S.xi[:, None, None] ** 2 + S.xi[None, :, None] ** 2 + S.xi[None, None, :] ** 2)
    S1 = Sx.reshape(N, N * N)
    p, Q = S1.sum(1), S1 @ S1.T
    one = np.ones(N)
    for i, nu in ((0, 0.4), (7, 2.5)):
        faces = S.cell_faces[i]
        V = mesh["cell_volume"][i]
        a = 1.0 + S.dt * nu
        b = S.dt * sum(mesh["face_area"][j] for j, _ in faces) / (2.0 * V)
        M = a * a * N * N * np.outer(one, one) + a * b * (np.outer(one, p) + np.outer(p, one)) + b * b * Q
        w, v = np.linalg.eigh(M)
        u = np.abs(v[:, -1])
        d = lusgs.diag_est(S, i, nu)
        for k in range(3):
            assert np.allclose(d.U[k][:, 0], u, rtol=1e-12, atol=0)
        sig = a * u.sum() ** 3 + b * np.einsum("abc,a,b,c->", Sx, u, u, u)
        assert abs(d.G[0, 0, 0] - sig) <= 1e-12 * sig
        assert (tk.full(d) > 0).all()
        exact = np.full((N, N, N), a)
        for j, s in faces:
            e = mesh["face_normal"][j]
            xn = e[0] * S.xi[:, None, None] + e[1] * S.xi[None, :, None] + e[2] * S.xi[None, None, :]
            exact = exact + S.dt * mesh["face_area"][j] / (2.0 * V) * np.abs(xn)
        assert (lusgs.diag_full(S, i, nu) >= exact - 1e-14).all()


def test_uniform_equilibrium_is_a_fixed_point():
    """A uniform state in a periodic box without collisions (Kn infinite)
    has R = 0: one LU-SGS iteration leaves it unchanged, in full and in
    Tucker form."""
    mesh = synth.periodic_box(3)
    cfg = cfg_of(init="uniform", Kn=np.inf)
    m0 = np.tile([1.1, 0.2, -0.1, 0.05, 0.9], (mesh["n_cells"], 1))
    S = fv.Setup(mesh, cfg, m0)
    F = dvm.initial_full(S, m0)
    G = lusgs.step_full(S, F)
    for i in F:
        assert np.allclose(G[i], F[i], rtol=0, atol=1e-11 * np.abs(F[i]).max())
    st = td.initial_states(S, m0)
    new, _, df = lusgs.step(S, st)
    for i in st:
        assert np.abs(tk.full(df[i])).max() <= 1e-11 * np.abs(tk.full(st[i])).max()
        assert np.allclose(tk.full(new[i]), tk.full(st[i]), rtol=0, atol=1e-11 * np.abs(tk.full(st[i])).max())


def explicit_residual(S, F):
    get = (lambda c: F[c])
    num = sum(np.sum((dvm.update_full(S, i, get) - F[i]) ** 2) for i in F)
    return np.sqrt(num / sum(np.sum(F[i] ** 2) for i in F)) / S.dt


def test_implicit_iteration_reduces_the_residual_faster():
    """The point of the implicit scheme: at CFL 8 (the explicit step's
    positivity bound is CFL 1) LU-SGS lowers the explicit residual |R(f)|
    monotonically and, per iteration, faster than explicit steps at CFL
    0.9 from the same random start."""
    mesh = synth.periodic_box(3)
    S, m0 = setup(mesh, cfl=8.0, Kn=0.3, N=8)
    Se, _ = setup(mesh, cfl=0.9, Kn=0.3, N=8)
    F = dvm.initial_full(S, m0)
    E = dvm.initial_full(Se, m0)
    r0 = explicit_residual(S, F)
    prev = r0
    for _ in range(10):
        F = lusgs.step_full(S, F)
        E = dvm.step_full(Se, E, round_result=False)
        r = explicit_residual(S, F)
        assert r < prev
        prev = r
    re = explicit_residual(S, E)
    print(f"after 10 iterations: LU-SGS {prev / r0:.3f}, explicit {re / r0:.3f} of the initial residual")
    assert prev < 0.7 * re


def test_tucker_iteration_matches_full_at_tight_tolerance():
    """With tolerance 1e-13 and no rank cap below N, the Tucker-form
    iteration (rounded df*, df and f + df) equals the full-tensor one."""
    S, m0 = setup(channel(), tol=1e-13, cap=6)
    F = dvm.initial_full(S, m0)
    st = td.initial_states(S, m0)
    for _ in range(2):
        F = lusgs.step_full(S, F)
        st, _, _ = lusgs.step(S, st)
    scale = max(np.abs(F[i]).max() for i in F)
    err = max(np.abs(tk.full(st[i]) - F[i]).max() for i in F) / scale
    assert err < 1e-11, err


def test_tucker_iteration_rounds_to_the_tolerance():
    """At tolerance 1e-4 the Tucker iteration stays within a few eps of the
    full-tensor iteration after three iterations and keeps lower ranks."""
    S, m0 = setup(channel(), tol=1e-4, cap=6)
    F = dvm.initial_full(S, m0)
    st = td.initial_states(S, m0)
    for _ in range(3):
        F = lusgs.step_full(S, F)
        st, _, _ = lusgs.step(S, st)
    scale = max(np.linalg.norm(F[i]) for i in F)
    err = max(np.linalg.norm(tk.full(st[i]) - F[i]) for i in F) / scale
    assert err < 1e-3, err
    assert max(max(st[i].ranks) for i in st) < 6
