"""The step with intermediate rounding of each face's flux term
(tk_state_face_rounding) against the oracle's step_faces: the same face
terms, rounded on their own, summed with the cell's own terms and rounded
again."""

import numpy as np
import pytest

import synth
from helpers import macro_rel_err
from oracle import fv, tucker_dvm as td
from paper_1912_04582_amd import tk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tk.Context(0)
    yield c
    c.close()


def channel():
    return synth.channel_with_obstacle(nx=8, ny=4, nz=4, h=0.25, obstacle=((3, 5), (1, 3), (1, 3)),
                                       inflow=(1.0, (0.9, 0.0, 0.0), 1.0), Tw=1.4)


def jittered():
    return synth.jittered_box(4, 3, 3, 0.25, seed=7)


def case(mesh, N, cap, tol, precision, seed=3):
    cfg = dict(N=N, xi_max=4.5, cap=cap, tol=tol, cfl=0.5, Pr=2 / 3, omega=0.5, Kn=0.1, Rg=0.5, m=1.0,
               seed=seed, init="random", precision=precision)
    return cfg, synth.initial_macros(cfg, mesh)


def oracle_run(mesh, cfg, m0, plan):
    S = fv.Setup(mesh, cfg, m0)
    st = td.initial_states(S, m0)
    for faces in plan:
        st = td.step_faces(S, st) if faces else td.step(S, st)
    mac = np.array([td.macros_of(S, st[i]) for i in range(mesh["n_cells"])])
    ranks = np.array([st[i].ranks for i in range(mesh["n_cells"])])
    return mac, ranks


def gpu_run(ctx, mesh, cfg, m0, plan, chunk=None):
    tm = tk.Mesh(ctx, mesh)
    st = tk.State(ctx, tm, cfg, m0)
    if chunk:
        st.set_chunk(chunk)
    for faces in plan:
        st.face_rounding(faces)
        st.step(1)
    got, ranks = st.moments(), st.ranks()[0]
    st.close()
    tm.close()
    return got, ranks


CASES = [
    # mesh, N, cap, tol, precision, steps, pass size, bar
    ("channel", 16, 6, 1e-4, "fp64", 3, None, 1e-10),
    ("channel", 32, 8, 1e-4, "fp64", 2, 37, 1e-10),
    ("jittered", 16, 6, 1e-4, "fp64", 2, None, 1e-10),
    ("jittered", 24, 6, 1e-4, "fp64", 2, 11, 1e-10),
    ("channel", 24, 8, 1e-4, "mixed", 2, None, 1e-5),
    ("jittered", 16, 6, 1e-4, "mixed", 2, None, 1e-5),
    ("jittered", 48, 6, 1e-4, "fp64", 1, None, 1e-10),
]


@pytest.mark.parametrize("kind,N,cap,tol,precision,steps,chunk,bar", CASES)
def test_face_rounding_matches_oracle(ctx, kind, N, cap, tol, precision, steps, chunk, bar):
    mesh = channel() if kind == "channel" else jittered()
    cfg, m0 = case(mesh, N, cap, tol, precision)
    plan = [True] * steps
    got, ranks = gpu_run(ctx, mesh, cfg, m0, plan, chunk)
    ref, oranks = oracle_run(mesh, cfg, m0, plan)
    err, _ = macro_rel_err(got, ref)
    print(f"face rounding {kind} N={N} {precision} {steps} steps: max rel macro err {err:.3e}, "
          f"rank mismatches {(ranks != oranks).any(1).sum()}", flush=True)
    assert err < bar, err
    if precision == "fp64":
        assert (ranks == oranks).all()


def test_face_rounding_toggles_per_step(ctx):
    # on, off, on: each step follows the placement in force
    mesh = jittered()
    cfg, m0 = case(mesh, 16, 6, 1e-4, "fp64", seed=9)
    plan = [True, False, True]
    got, ranks = gpu_run(ctx, mesh, cfg, m0, plan)
    ref, oranks = oracle_run(mesh, cfg, m0, plan)
    err, _ = macro_rel_err(got, ref)
    assert err < 1e-10, err
    assert (ranks == oranks).all()


def test_face_rounding_is_a_different_result(ctx):
    # at a loose tolerance the intermediate roundings move the result, by no
    # more than the roundings' bound allows
    mesh = jittered()
    cfg, m0 = case(mesh, 16, 6, 1e-3, "fp64", seed=4)
    a, _ = gpu_run(ctx, mesh, cfg, m0, [True, True])
    b, _ = gpu_run(ctx, mesh, cfg, m0, [False, False])
    d, _ = macro_rel_err(a, b)
    assert 1e-12 < d < 1e-1, d


def test_face_rounding_refuses_plain_states(ctx):
    mesh = channel()
    cfg, m0 = case(mesh, 16, 6, 1e-4, "fp64")
    tm = tk.Mesh(ctx, mesh)
    pl = tk.State(ctx, tm, cfg, m0, plain=True)
    with pytest.raises(tk.TkError):
        pl.face_rounding(True)
    pl.close()
    tm.close()


def test_face_rounding_batch_matches_oracle(ctx):
    # two instances of one state with their own tolerance and cap: every
    # face-term rounding takes its instance's
    items = []
    for k, (mesh, cap, tol) in enumerate([(channel(), 6, 1e-4), (jittered(), 5, 1e-3)]):
        cfg, m0 = case(mesh, 16, cap, tol, "fp64", seed=20 + k)
        items.append((mesh, cfg, m0))
    meshes = [tk.Mesh(ctx, m) for m, _, _ in items]
    st = tk.State(ctx, meshes, [c for _, c, _ in items], [m0 for _, _, m0 in items])
    st.face_rounding(True)
    st.step(2)
    got, ranks = st.moments(), st.ranks()[0]
    st.close()
    for mm in meshes:
        mm.close()
    off = 0
    for mesh, cfg, m0 in items:
        n = mesh["n_cells"]
        ref, oranks = oracle_run(mesh, cfg, m0, [True, True])
        err, _ = macro_rel_err(got[off:off + n], ref)
        assert err < 1e-10, err
        assert (ranks[off:off + n] == oranks).all()
        off += n
