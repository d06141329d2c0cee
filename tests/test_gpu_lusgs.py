"""LU-SGS implicit iterations on the GPU (tk_lusgs) against the Tucker-form
LU-SGS oracle: the same colouring, rank-1 diagonal, sweeps and roundings."""

import numpy as np
import pytest

import synth
from helpers import macro_rel_err
from oracle import fv, lusgs, tucker_dvm as td
from paper_1912_04582_amd import tk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tk.Context(0)
    yield c
    c.close()


def channel_case(N, cap, tol, init, cfl, seed=21, Kn=0.1, precision="fp64"):
    m = synth.channel_with_obstacle(nx=8, ny=4, nz=4, h=0.25, obstacle=((3, 5), (1, 3), (1, 3)),
                                    inflow=(1.0, (0.9, 0.0, 0.0), 1.0), Tw=1.4)
    cfg = dict(N=N, xi_max=4.5, cap=cap, tol=tol, cfl=cfl, Pr=2 / 3, omega=0.5, Kn=Kn, Rg=0.5, m=1.0,
               seed=seed, init=init, precision=precision)
    return m, cfg, synth.initial_macros(cfg, m)


def oracle_run(m, cfg, m0, iters):
    S = fv.Setup(m, cfg, m0)
    st = lusgs.run(S, m0, iters)
    mac = np.array([td.macros_of(S, st[i]) for i in range(m["n_cells"])])
    ranks = np.array([st[i].ranks for i in range(m["n_cells"])])
    return mac, ranks


CASES = [
    # N, cap, tol, init, CFL, iterations, precision, bar
    (16, 6, 1e-6, "random", 4.0, 3, "fp64", 1e-10),
    (24, 8, 1e-6, "freestream", 8.0, 3, "fp64", 1e-10),
    (32, 12, 1e-5, "random", 4.0, 2, "fp64", 1e-10),
    (32, 12, 1e-5, "random", 4.0, 2, "mixed", 1e-5),
    (24, 8, 1e-6, "freestream", 8.0, 3, "mixed", 1e-5),
]


@pytest.mark.parametrize("N,cap,tol,init,cfl,iters,precision,bar", CASES)
def test_lusgs_matches_oracle(ctx, N, cap, tol, init, cfl, iters, precision, bar):
    m, cfg, m0 = channel_case(N, cap, tol, init, cfl, precision=precision)
    mesh = tk.Mesh(ctx, m)
    st = tk.State(ctx, mesh, cfg, m0)
    res = st.lusgs(iters, residual=True)
    got = st.moments()
    ranks = st.ranks()[0]
    st.close()
    mesh.close()
    ref, oranks = oracle_run(m, cfg, m0, iters)
    err, _ = macro_rel_err(got, ref)
    print(f"LU-SGS N={N} {precision} CFL {cfl} {iters} iterations: max rel macro err {err:.3e}, "
          f"residual {res[0]:.3e}, rank mismatches {(ranks != oranks).any(1).sum()}")
    assert np.isfinite(res).all() and res[0] > 0
    assert err < bar, err
    if precision == "fp64":
        assert (ranks == oranks).all()


def test_lusgs_batch_matches_oracle(ctx):
    """Two instances with different N-independent parameters in one state."""
    items = [channel_case(16, 6, 1e-6, "random", 4.0, seed=5, Kn=0.05),
             channel_case(16, 5, 1e-5, "freestream", 6.0, seed=6, Kn=0.5)]
    meshes = [tk.Mesh(ctx, m) for m, _, _ in items]
    st = tk.State(ctx, meshes, [c for _, c, _ in items], [m0 for _, _, m0 in items])
    st.lusgs(2)
    got = st.moments()
    st.close()
    for mm in meshes:
        mm.close()
    off = 0
    for m, cfg, m0 in items:
        ref, _ = oracle_run(m, cfg, m0, 2)
        n = m["n_cells"]
        err, _ = macro_rel_err(got[off:off + n], ref)
        assert err < 1e-10, err
        off += n


def test_lusgs_keeps_an_equilibrium(ctx):
    """A uniform state in a periodic box without collisions has R = 0: the
    iteration leaves it unchanged."""
    m = synth.periodic_box(4)
    cfg = dict(N=16, xi_max=4.5, cap=4, tol=1e-6, cfl=8.0, Pr=2 / 3, omega=0.5, Kn=np.inf, Rg=0.5, m=1.0,
               seed=1, init="uniform", precision="fp64")
    m0 = np.tile([1.1, 0.2, -0.1, 0.05, 0.9], (m["n_cells"], 1))
    mesh = tk.Mesh(ctx, m)
    st = tk.State(ctx, mesh, cfg, m0)
    a = st.moments()
    st.lusgs(3)
    b = st.moments()
    st.close()
    mesh.close()
    err, _ = macro_rel_err(b, a)
    assert err < 1e-12, err


def test_lusgs_refuses_unsupported_states(ctx):
    m, cfg, m0 = channel_case(16, 6, 1e-6, "random", 4.0)
    mesh = tk.Mesh(ctx, m)
    st = tk.State(ctx, mesh, cfg, m0, plain=True)
    with pytest.raises(tk.TkError) as e:
        st.lusgs(1)
    assert e.value.status == tk.TK_EINVAL
    st.close()
    mesh.close()
    jm = synth.jittered_box(3, 3, 3, 1 / 3, seed=2)
    mesh = tk.Mesh(ctx, jm)
    st = tk.State(ctx, mesh, cfg, synth.initial_macros(cfg, jm))
    with pytest.raises(tk.TkError) as e:
        st.lusgs(1)
    assert e.value.status == tk.TK_EINVAL
    st.close()
    mesh.close()
