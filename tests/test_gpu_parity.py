"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: the FP64 path matches the oracle to 1e-10 relative on n, u, T
and q (u against the thermal speed, q against p sqrt(2 R_g T)); the mixed
path (FP32 term assembly, FP64 Gram/eigen/projection/moments) to 1e-5.
Rank decisions must agree; where they cannot (a tail sum within rounding
of the threshold) the oracle's decision margin is reported.
"""

import numpy as np
import pytest

import synth
from helpers import macro_rel_err, tucker_full
from oracle import dvm, fv, kinetic as kin, tucker as otk, tucker_dvm as td
from paper_1912_04582_amd import tk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tk.Context(0)
    yield c
    c.close()


def small_channel(N=16, cap=6, tol=1e-6, precision="fp64", Kn=0.1, nx=6):
    m = synth.channel_with_obstacle(nx=nx, ny=4, nz=4, h=0.25, obstacle=((2, 3), (1, 2), (1, 3)),
                                    inflow=(1.0, (0.8, 0.0, 0.0), 1.0), Tw=1.3)
    cfg = dict(N=N, xi_max=4.5, cap=cap, tol=tol, cfl=0.5, Pr=2 / 3, omega=0.5, Kn=Kn, Rg=0.5, m=1.0,
               seed=11, init="random", precision=precision)
    return m, cfg


def oracle_macros(S, states):
    return np.array([td.macros_of(S, states[i]) for i in range(S.mesh["n_cells"])])


def gpu_state(ctx, m, cfg, macros):
    mesh = tk.Mesh(ctx, m)
    st = tk.State(ctx, mesh, cfg, macros)
    return mesh, st


@pytest.mark.parametrize("N", [16, 24, 32])
def test_round_tucker_matches_oracle_hosvd(ctx, N):
    rng = np.random.default_rng(N)
    x = np.linspace(-3, 3, N)
    tensors, refs = [], []
    for t in range(6):
        # smooth low-rank part plus a decaying random part: ranks above and
        # below the cap, tails above and below the threshold
        terms = [otk.hosvd(np.exp(-(x[:, None, None] - c) ** 2 - (x[None, :, None] + c) ** 2 / (1 + c)
                                  - x[None, None, :] ** 2 * (1 + 0.5 * c)), 0.0, 4) for c in (0.2, 0.7)]
        r = (3 + t, 5, 2 + t)
        G = rng.standard_normal(r) * (10.0 ** -np.arange(r[0]))[:, None, None]
        U = [np.linalg.qr(rng.standard_normal((N, r[a])))[0] for a in range(3)]
        terms.append(otk.Tucker(1e-3 * G, U))
        s = terms[0]
        for q in terms[1:]:
            s = otk.add(s, q)
        tensors.append((s.G, s.U))
        refs.append(otk.full(s))
    for tol, cap in ((1e-6, 12), (1e-3, 16), (1e-9, 5)):
        out = ctx.round_tucker(tensors, tol, cap)
        for (G, U), A in zip(out, refs):
            ref = otk.hosvd(A, tol, cap)
            assert tuple(G.shape) == ref.ranks, (G.shape, ref.ranks)
            B = tucker_full(G, U)
            err = np.abs(B - otk.full(ref)).max() / np.abs(A).max()
            assert err < 1e-11, err
            for a in range(3):
                np.testing.assert_allclose(U[a].T @ U[a], np.eye(U[a].shape[1]), atol=1e-12)


@pytest.mark.parametrize("name", ["cfg0"])
def test_initial_moments(ctx, name):
    cfg = synth.make_config(name)
    m = synth.configs.make_mesh(cfg)
    m0 = synth.initial_macros(cfg, m)
    mesh, st = gpu_state(ctx, m, cfg, m0)
    got = st.moments()
    S = fv.Setup(m, cfg, m0)
    ref = oracle_macros(S, td.initial_states(S, m0))
    err, _ = macro_rel_err(got, ref)
    assert err < 1e-13, err
    assert abs(st.dt() - S.dt) <= 1e-15 * S.dt
    st.close(); mesh.close()


def compare_states(st, S, ref_states, N, cells, tol_rel):
    worst = 0.0
    for i in cells:
        G, U = st.export(i, N)
        ref = ref_states[i]
        assert tuple(G.shape) == ref.ranks, (i, G.shape, ref.ranks)
        A = otk.full(ref)
        err = np.abs(tucker_full(G, U) - A).max() / np.abs(A).max()
        worst = max(worst, err)
    assert worst < tol_rel, worst
    return worst


def test_cfg0_one_step_per_cell(ctx):
    cfg = synth.make_config("cfg0")
    m = synth.configs.make_mesh(cfg)
    m0 = synth.initial_macros(cfg, m)
    mesh, st = gpu_state(ctx, m, cfg, m0)
    S = fv.Setup(m, cfg, m0)
    st.step(1)
    cells = [0, 1, 63, 200, 511]
    ref = td.step(S, td.initial_states(S, m0), cells)
    # one-step states from the plain definition as well
    ref1 = dvm.step_full(S, dvm.initial_full(S, m0), cells)
    compare_states(st, S, ref, 16, cells, 1e-11)
    compare_states(st, S, ref1, 16, cells, 1e-11)
    st.close(); mesh.close()


def test_cfg0_full_run_fp64(ctx):
    """The small workload end to end: 512 cells, N = 16, cap 6, 20 steps."""
    cfg = synth.make_config("cfg0")
    m = synth.configs.make_mesh(cfg)
    m0 = synth.initial_macros(cfg, m)
    mesh, st = gpu_state(ctx, m, cfg, m0)
    st.step(cfg["steps"])
    got = st.moments()
    S = fv.Setup(m, cfg, m0)
    ref_states = td.run(S, m0, cfg["steps"])
    ref = oracle_macros(S, ref_states)
    err, _ = macro_rel_err(got, ref)
    print(f"cfg0 20 steps FP64 max rel macro err {err:.3e}")
    assert err < 1e-10, err
    ranks, C = st.ranks()
    oranks = np.array([ref_states[i].ranks for i in range(m["n_cells"])])
    assert (ranks == oranks).all()
    st.close(); mesh.close()


def test_channel_boundaries_fp64(ctx):
    m, cfg = small_channel()
    m0 = synth.initial_macros(cfg, m)
    mesh, st = gpu_state(ctx, m, cfg, m0)
    S = fv.Setup(m, cfg, m0)
    ref_states = td.run(S, m0, 4)
    st.step(4)
    err, _ = macro_rel_err(st.moments(), oracle_macros(S, ref_states))
    print(f"channel FP64 4 steps max rel macro err {err:.3e}")
    assert err < 1e-10, err
    compare_states(st, S, ref_states, cfg["N"], range(m["n_cells"]), 1e-10)
    st.close(); mesh.close()


def test_channel_mixed_precision(ctx):
    m, cfg = small_channel(N=32, cap=12, tol=1e-5, precision="mixed")
    m0 = synth.initial_macros(cfg, m)
    mesh, st = gpu_state(ctx, m, cfg, m0)
    S = fv.Setup(m, cfg, m0)
    ref_states = td.run(S, m0, 3)
    st.step(3)
    err, _ = macro_rel_err(st.moments(), oracle_macros(S, ref_states))
    print(f"channel mixed N=32 3 steps max rel macro err {err:.3e}")
    assert err < 1e-5, err
    st.close(); mesh.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_plain_step_matches_full_update(ctx, precision, tol):
    m, cfg = small_channel(precision=precision)
    m0 = synth.initial_macros(cfg, m)
    mesh = tk.Mesh(ctx, m)
    st = tk.State(ctx, mesh, cfg, m0, plain=True)
    st.step(1)
    got = st.moments()
    S = fv.Setup(m, cfg, m0)
    F = dvm.initial_full(S, m0)
    ref = []
    for i in range(m["n_cells"]):
        X = dvm.update_full(S, i, lambda c: F[c])
        n, u, T, q = kin.macros_full(X, S.xi, S.dxi)
        ref.append([n, *u, T, *q])
    err, _ = macro_rel_err(got, np.array(ref))
    print(f"plain {precision} 1 step max rel macro err {err:.3e}")
    assert err < tol, err
    st.close(); mesh.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_plain_step_on_oblique_faces_matches_exact_flux(ctx, precision, tol):
    """The plain comparator on a jittered mesh (faces off the axes): the
    standard DVM step with the exact |xi_n| per node, against the oracle's
    exact-flux update."""
    m = synth.jittered_box(4, 3, 3, 0.25, seed=9)
    cfg = dict(N=16, xi_max=4.5, cap=6, tol=1e-6, cfl=0.5, Pr=2 / 3, omega=0.5, Kn=0.2, Rg=0.5, m=1.0,
               seed=9, init="random", precision=precision)
    m0 = synth.initial_macros(cfg, m)
    mesh = tk.Mesh(ctx, m)
    st = tk.State(ctx, mesh, cfg, m0, plain=True)
    st.step(2)
    got = st.moments()
    st.close(); mesh.close()
    S = fv.Setup(m, cfg, m0)
    F = dvm.initial_full(S, m0)
    for _ in range(2):
        F = dvm.step_full(S, F, round_result=False, exact=True)
    ref = []
    for i in range(m["n_cells"]):
        n, u, T, q = kin.macros_full(F[i], S.xi, S.dxi)
        ref.append([n, *u, T, *q])
    err, _ = macro_rel_err(got, np.array(ref))
    print(f"plain {precision} jittered 2 steps max rel macro err {err:.3e}")
    assert err < tol, err


def test_mixed_drift_monitor_against_fp64(ctx):
    """A drift monitor, not parity evidence (the parity of the mixed path
    is the oracle tests' 1e-5 over a few steps): after 80 warm-started
    steps with rank growth near the walls the mixed path stays within 1e-3
    of the GPU FP64 path.  Rank decisions may differ at the truncation
    threshold and compound (on the full channel 4.6e-5 after 200 steps,
    against 3e-7 for the FP64 path's spread under a 1e-7 input
    perturbation), so this bar only catches a broken mixed path."""
    m, cfg = small_channel(N=24, cap=8, tol=1e-5, precision="mixed", nx=8)
    m0 = synth.initial_macros(cfg, m)
    mesh = tk.Mesh(ctx, m)
    a = tk.State(ctx, mesh, cfg, m0)
    b = tk.State(ctx, mesh, dict(cfg, precision="fp64"), m0)
    for _ in range(4):
        a.step(20)
        b.step(20)
    err, _ = macro_rel_err(a.moments(), b.moments())
    print(f"mixed vs FP64, 80 steps: max rel macro err {err:.3e}")
    assert err < 1e-3, err
    a.close(); b.close(); mesh.close()


def test_batch_equals_alone_and_oracle(ctx):
    """Instances advanced together give the same result as each alone."""
    specs = []
    m1, c1 = small_channel(N=16, cap=5, tol=1e-6)
    specs.append((m1, c1))
    m2 = synth.periodic_box(3)
    c2 = dict(c1, cap=4, tol=1e-5, Kn=0.3, seed=21)
    specs.append((m2, c2))
    m3 = synth.periodic_box(4, length=0.5)
    c3 = dict(c1, cap=6, tol=1e-7, Kn=0.05, seed=22, xi_max=5.0)
    specs.append((m3, c3))
    macros = [synth.initial_macros(c, m) for m, c in specs]
    meshes = [tk.Mesh(ctx, m) for m, _ in specs]
    batch = tk.State(ctx, meshes, [c for _, c in specs], macros)
    res = batch.step(4, residual=True)
    got = batch.moments()
    batch.close()
    off = 0
    for (m, c), mesh, m0 in zip(specs, meshes, macros):
        alone = tk.State(ctx, mesh, c, m0)
        alone.step(4)
        a = alone.moments()
        alone.close()
        part = got[off:off + m["n_cells"]]
        assert np.array_equal(part, a), np.abs(part - a).max()
        off += m["n_cells"]
    # the second instance against the oracle
    S = fv.Setup(m2, c2, macros[1])
    ref = oracle_macros(S, td.run(S, macros[1], 4))
    err, _ = macro_rel_err(got[specs[0][0]["n_cells"]:specs[0][0]["n_cells"] + m2["n_cells"]], ref)
    assert err < 1e-10, err
    assert res.shape == (3,) and np.all(res > 0)
    for mesh in meshes:
        mesh.close()


def test_uniform_state_stays_rank1_on_gpu(ctx):
    cfg = synth.make_config("cfg0", init="uniform")
    m = synth.configs.make_mesh(cfg)
    m0 = synth.initial_macros(cfg, m)
    mesh, st = gpu_state(ctx, m, cfg, m0)
    first = st.moments()
    st.step(20)
    last = st.moments()
    r, C = st.ranks()
    assert (r == 1).all()
    assert np.abs(last[:, 0] / first[:, 0] - 1).max() < 1e-9
    assert np.abs(last[:, 4] / first[:, 4] - 1).max() < 1e-9
    assert np.abs(last[:, 1:4]).max() < 1e-13 and np.abs(last[:, 5:]).max() < 1e-13
    st.close(); mesh.close()


def test_invalid_arguments_rejected(ctx):
    m, cfg = small_channel()
    m0 = synth.initial_macros(cfg, m)
    mesh = tk.Mesh(ctx, m)
    for bad in (dict(N=20), dict(cap=17), dict(cap=0), dict(tol=-1.0), dict(N=64)):
        with pytest.raises(tk.TkError) as ei:
            tk.State(ctx, mesh, dict(cfg, **bad), m0)
        assert ei.value.status == tk.TK_EINVAL
    neg = m0.copy()
    neg[3, 4] = -1.0
    with pytest.raises(tk.TkError) as ei:
        tk.State(ctx, mesh, cfg, neg)
    assert ei.value.status == tk.TK_ENUMERIC
    mesh.close()


def full_macros(S, F):
    out = []
    for i in range(S.mesh["n_cells"]):
        n, u, T, q = kin.macros_full(F[i], S.xi, S.dxi, S.Rg, S.m)
        out.append([n, *u, T, *q])
    return np.array(out)


@pytest.mark.parametrize("precision,N,cap,tol,steps,bar", [("fp64", 16, 6, 1e-6, 3, 1e-10),
                                                          ("mixed", 24, 6, 1e-5, 2, 1e-5),
                                                          ("fp64", 32, 6, 1e-6, 2, 1e-10)])
def test_jittered_mesh_oblique_faces(ctx, precision, N, cap, tol, steps, bar):
    """Faces off the coordinate axes: rank-6 |xi.e| estimates and Hadamard flux terms.
    N = 16 and 24 run the one-stage expansion; FP64 at N = 32 exceeds its LDS
    budget, so every cell takes the general (restaging) expansion."""
    m = synth.jittered_box(3, 3, 3, 1 / 3, seed=7)
    cfg = dict(N=N, xi_max=4.5, cap=cap, tol=tol, cfl=0.5, Pr=2 / 3, omega=0.5, Kn=0.2, Rg=0.5, m=1.0,
               seed=31, init="random", precision=precision)
    m0 = synth.initial_macros(cfg, m)
    mesh, st = gpu_state(ctx, m, cfg, m0)
    st.step(steps)
    got = st.moments()
    S = fv.Setup(m, cfg, m0)
    F = dvm.run_full(S, m0, steps)
    err, _ = macro_rel_err(got, full_macros(S, F))
    print(f"jittered {precision} N={N} {steps} steps max rel macro err {err:.3e}")
    assert err < bar, err
    st.close(); mesh.close()


def test_serving_alone_equals_mix(ctx):
    """Served requests: results equal to the same request served alone; the
    two N = 16 requests on axis-aligned meshes, submitted together, share
    one batched state (with different rank caps and tolerances)."""
    import time
    reqs = []
    for k, (mk, N, cap, tol) in enumerate([(lambda: synth.periodic_box(3), 16, 4, 1e-5),
                                           (lambda: synth.jittered_box(3, 3, 3, 1 / 3, seed=3), 16, 5, 1e-6),
                                           (lambda: synth.periodic_box(4, length=0.5), 24, 6, 1e-5),
                                           (lambda: synth.periodic_box(3, length=0.7), 16, 6, 1e-6)]):
        m = mk()
        cfg = dict(N=N, xi_max=4.5, cap=cap, tol=tol, cfl=0.5, Pr=2 / 3, omega=0.5, Kn=0.2, Rg=0.5, m=1.0,
                   seed=40 + k, init="random", precision="mixed")
        reqs.append((m, cfg, synth.initial_macros(cfg, m)))

    def serve(items):
        srv = tk.Server(ctx)
        tickets = [srv.submit(m, c, m0, 12, 1e-9) for m, c, m0 in items]
        out = {}
        t0 = time.time()
        while len(out) < len(tickets) and time.time() - t0 < 120:
            for t in tickets:
                if t in out:
                    continue
                r = srv.poll(t)
                if r["status"] != tk.TK_PENDING:
                    out[t] = r
            time.sleep(0.01)
        stats = srv.stats()
        srv.close()
        return [out[t] for t in tickets], stats

    mix, stats = serve(reqs)
    assert stats["largest_cohort"] == 2 and stats["cohorts"] == 3, stats
    assert stats["request_steps"] == 4 * 12 and stats["cohort_steps"] == 3 * 12, stats
    for k, item in enumerate(reqs):
        alone = serve([item])[0][0]
        assert mix[k]["status"] == tk.TK_OK and alone["status"] == tk.TK_OK
        assert mix[k]["steps"] == alone["steps"] == 12
        assert np.array_equal(mix[k]["macros"], alone["macros"])
        assert mix[k]["t_arrive"] <= mix[k]["t_admit"] <= mix[k]["t_done"]
    # the served result equals a plain state run
    m, c, m0 = reqs[0]
    mesh, st = gpu_state(ctx, m, c, m0)
    st.step(12)
    assert np.array_equal(st.moments(), mix[0]["macros"])
    st.close(); mesh.close()


@pytest.mark.parametrize("faces", ["axis", "oblique"])
def test_serving_late_request_joins_the_running_cohort(ctx, faces):
    """A request admitted while another of its kind runs joins that cohort
    at its next step boundary (the cohort's state rebuilt, the running
    request's state, kept bases and face estimates copied over on the
    device); both results equal the requests served alone, bit for bit, and
    the late steps are shared."""
    import time
    reqs = []
    for k, (n, cap, tol) in enumerate([(4, 6, 1e-6), (3, 4, 1e-5)]):
        if faces == "axis":
            m = synth.periodic_box(n, length=0.5 + 0.1 * k)
        else:
            m = synth.jittered_box(n, n, 3, 1.0 / n, seed=80 + k)
        cfg = dict(N=16, xi_max=4.5, cap=cap, tol=tol, cfl=0.5, Pr=2 / 3, omega=0.5, Kn=0.2, Rg=0.5, m=1.0,
                   seed=70 + k, init="random", precision="mixed")
        reqs.append((m, cfg, synth.initial_macros(cfg, m)))
    steps = (200, 12)

    def wait(srv, t):
        t0 = time.time()
        while time.time() - t0 < 120:
            r = srv.poll(t)
            if r["status"] != tk.TK_PENDING:
                return r
            time.sleep(0.005)
        raise TimeoutError

    srv = tk.Server(ctx)
    ta = srv.submit(*reqs[0], steps[0], 1e-12)
    t0 = time.time()
    while srv.poll(ta, want_macros=False)["steps"] < 3 and time.time() - t0 < 60:
        time.sleep(0.001)
    assert srv.poll(ta, want_macros=False)["status"] == tk.TK_PENDING
    tb = srv.submit(*reqs[1], steps[1], 1e-12)
    rb, ra = wait(srv, tb), wait(srv, ta)
    stats = srv.stats()
    srv.close()
    assert ra["status"] == rb["status"] == tk.TK_OK and ra["steps"] == steps[0] and rb["steps"] == steps[1]
    assert stats["cohorts"] == 2 and stats["largest_cohort"] == 2, stats
    assert stats["request_steps"] == sum(steps) and stats["cohort_steps"] == steps[0], stats
    for item, n, got in zip(reqs, steps, (ra, rb)):
        alone = tk.Server(ctx)
        t = alone.submit(*item, n, 1e-12)
        r = wait(alone, t)
        alone.close()
        assert np.array_equal(got["macros"], r["macros"])


def test_serving_refuses_requests_that_never_fit(ctx):
    srv = tk.Server(ctx, budget=1 << 20)
    m = synth.periodic_box(3)
    cfg = dict(N=16, xi_max=4.5, cap=4, tol=1e-5, cfl=0.5, Pr=2 / 3, omega=0.5, Kn=0.2, Rg=0.5, m=1.0,
               seed=1, init="random", precision="mixed")
    with pytest.raises(tk.TkError) as ei:
        srv.submit(m, cfg, synth.initial_macros(cfg, m), 5, 1e-5)
    assert ei.value.status == tk.TK_ENOMEM
    srv.close()
