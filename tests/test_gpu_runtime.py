"""Runtime features on the GPU, through the C ABI: rounding-pass sizes,
the pass-size choice by timed trial steps, graph replay of a step, and
parity at the full sizes of the channel and jittered-box workloads on
sampled cells (their dependency cones advanced by the FP64 oracle)."""

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


def box_case(n=16, N=16, precision="fp64", cap=6, tol=1e-6):
    cfg = dict(synth.make_config("cfg0"), N=N, cap=cap, tol=tol, precision=precision)
    m = synth.periodic_box(n)
    return m, cfg, synth.initial_macros(cfg, m)


def test_pass_sizes_give_identical_bits(ctx):
    m, cfg, m0 = box_case(8)
    mesh = tk.Mesh(ctx, m)
    a = tk.State(ctx, mesh, cfg, m0)
    b = tk.State(ctx, mesh, cfg, m0)
    _, cmax = a.chunk()
    a.set_chunk(cmax)
    b.set_chunk(37)  # 13 full passes and a ragged one of 31 cells
    assert b.chunk() == (37, cmax)
    a.step(3)
    b.step(3)
    assert np.array_equal(a.moments(), b.moments())
    assert np.array_equal(a.ranks()[0], b.ranks()[0])
    for c in (0, 100, 511):
        ga, ua = a.export(c, cfg["N"])
        gb, ub = b.export(c, cfg["N"])
        assert np.array_equal(ga, gb) and all(np.array_equal(x, y) for x, y in zip(ua, ub))
    with pytest.raises(tk.TkError) as ei:
        b.set_chunk(cmax + 1)
    assert ei.value.status == tk.TK_EINVAL
    a.close(); b.close(); mesh.close()


def handoff_channel():
    """N = 32 mixed, cap 12, tol 1e-8 from rough fields: most cells exceed
    the small expansion layout's rank 8 after two steps (the list hand-off
    of k_expand_pipe), the rest round in factor space or stay small."""
    m = synth.channel_with_obstacle(nx=8, ny=4, nz=4, h=0.25, obstacle=((3, 5), (1, 3), (1, 3)),
                                    inflow=(1.0, (0.9, 0.0, 0.0), 1.0), Tw=1.4)
    cfg = dict(N=32, xi_max=6.0, cap=12, tol=1e-8, cfl=0.5, Pr=2 / 3, omega=0.5, Kn=0.1, Rg=0.5, m=1.0,
               seed=8, init="random", precision="mixed")
    return m, cfg, synth.initial_macros(cfg, m)


def jittered_case(precision):
    m = synth.jittered_box(5, 4, 4, 0.2, seed=12)
    cfg = dict(synth.make_config("cfg0"), N=16, cap=6, tol=1e-6, precision=precision)
    return m, cfg, synth.initial_macros(cfg, m)


TWO_STREAM_CASES = {
    "box-fp64": lambda: box_case(8, N=16, precision="fp64"),
    "box-mixed": lambda: box_case(8, N=16, precision="mixed"),
    "channel-N32-handoff": handoff_channel,
    "jittered-fp64": lambda: jittered_case("fp64"),
    "jittered-mixed": lambda: jittered_case("mixed"),
}


@pytest.mark.parametrize("case", list(TWO_STREAM_CASES))
def test_two_stream_passes_give_identical_bits(case):
    """Rounding passes alternating between two streams with two workspaces
    (kernel timing on, events on each pass's stream), all passes on one
    stream, and one pass over every cell must give the same bits: periodic
    boxes, the N = 32 channel whose expansion hands most cells to the
    full-layout launch (per-workspace hand-off lists), and a jittered mesh
    (oblique-face expansion and its per-workspace lists)."""
    c = tk.Context(0)
    try:
        m, cfg, m0 = TWO_STREAM_CASES[case]()
        mesh = tk.Mesh(c, m)
        out = []
        for chunk, two in ((None, True), (37, True), (37, False)):  # several passes, the last ragged
            st = tk.State(c, mesh, cfg, m0)
            assert st.streams(two)
            st.set_chunk(chunk or st.chunk()[1])
            c.prof_enable(True)
            st.step(3)
            c.prof_enable(False)
            out.append((st.moments(), st.ranks()[0], st.export(77 % m["n_cells"], cfg["N"])))
            st.close()
        ma, ra, (ga, ua) = out[0]
        for mb, rb, (gb, ub) in out[1:]:
            assert np.array_equal(ma, mb) and np.array_equal(ra, rb)
            assert np.array_equal(ga, gb) and all(np.array_equal(x, y) for x, y in zip(ua, ub))
        mesh.close()
    finally:
        c.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_equals_eager(ctx, precision):
    m, cfg, m0 = box_case(8, N=16, precision=precision)
    mesh = tk.Mesh(ctx, m)
    eager = tk.State(ctx, mesh, cfg, m0)
    graph = tk.State(ctx, mesh, cfg, m0)
    for s in (eager, graph):
        s.set_chunk(200)
    graph.use_graph(True)
    # replays of both parities, eager work (moments) between them, and a
    # pass-size change that forces a new capture
    for k in range(5):
        if k == 3:
            eager.set_chunk(128)
            graph.set_chunk(128)
        eager.step(2)
        graph.step(2)
        ma, mb = eager.moments(), graph.moments()
        assert np.array_equal(ma, mb), (k, np.abs(ma - mb).max())
        assert np.array_equal(eager.ranks()[0], graph.ranks()[0])
    eager.close(); graph.close(); mesh.close()


def test_pass_size_choice_is_kept_per_shape():
    c = tk.Context(0)
    try:
        m, cfg, m0 = box_case(16)  # 4096 cells: several candidate sizes
        mesh = tk.Mesh(c, m)
        a = tk.State(c, mesh, cfg, m0)
        _, cmax = a.chunk()
        trials = a.tune()
        # 16 untimed steps, then 4 timed steps per candidate size
        assert trials >= 16 + 4 * 2 and (trials - 16) % 4 == 0
        chosen, _ = a.chunk()
        assert 256 <= chosen <= cmax
        assert a.tune() == 0
        # a second state of the same shape starts with the chosen size
        b = tk.State(c, mesh, cfg, m0)
        assert b.chunk()[0] == chosen
        assert b.tune() == 0
        # the trial steps computed the same bits as fixed-size steps
        ref = tk.State(c, mesh, cfg, m0)
        ref.set_chunk(cmax)
        ref.step(trials)
        assert np.array_equal(a.moments(), ref.moments())
        for s in (a, b, ref):
            s.close()
        mesh.close()
    finally:
        c.close()


def sampled_parity(name, steps, count, bar):
    cfg = synth.make_config(name)
    mesh = synth.configs.make_mesh(cfg)
    m0 = synth.initial_macros(cfg, mesh)
    fl, fr = mesh["face_left"], mesh["face_right"]
    picks = []
    for b in range(len(mesh["bc"])):
        cand = fl[fr == -(b + 1)]
        picks.append(int(cand[len(cand) // 3]))
    rng = np.random.default_rng(5)
    while len(picks) < count:
        picks.append(int(rng.integers(mesh["n_cells"])))
    picks = sorted(set(picks))
    print(f"{name}: {mesh['n_cells']} cells, cells {picks}, {steps} steps", flush=True)
    c = tk.Context(0)
    try:
        tm = tk.Mesh(c, mesh)
        st = tk.State(c, tm, cfg, m0)
        st.step(steps)
        got = st.moments()[picks]
        st.close()
        tm.close()
    finally:
        c.close()
    S = fv.Setup(mesh, cfg, m0)
    ref = td.run_cone(S, m0, picks, steps)
    ref = np.array([td.macros_of(S, ref[i]) for i in picks])
    err, _ = macro_rel_err(got, ref)
    print(f"{name}: max rel macro err {err:.3e} (bar {bar})")
    assert err < bar, err


def test_channel_full_size_sampled_cells():
    sampled_parity("cfg1", 3, 8, 1e-5)


def test_jittered_box_full_size_sampled_cells():
    sampled_parity("cfg2", 2, 3, 1e-5)


def small_channel_case(precision="mixed", N=16):
    m = synth.channel_with_obstacle(nx=6, ny=4, nz=4, h=0.25, obstacle=((2, 3), (1, 2), (1, 3)),
                                    inflow=(1.0, (0.8, 0.0, 0.0), 1.0), Tw=1.3)
    cfg = dict(N=N, xi_max=4.5, cap=6, tol=1e-6, cfl=0.5, Pr=2 / 3, omega=0.5, Kn=0.1, Rg=0.5, m=1.0,
               seed=11, init="random", precision=precision)
    return m, cfg, synth.initial_macros(cfg, m)


def test_expansion_rank_handoff_matches_oracle(ctx):
    """N = 32, mixed, cap 12 from rough initial fields at tolerance 1e-8:
    after two steps most cells have ranks above 8, so the third step's
    expansion runs both launches (sources within the small LDS layout, then
    the handed-over cells through the full layout); every cell is checked
    against the FP64 oracle."""
    m, cfg, m0 = small_channel_case(N=32)
    cfg = dict(cfg, cap=12, tol=1e-8)
    mesh = tk.Mesh(ctx, m)
    st = tk.State(ctx, mesh, cfg, m0)
    st.step(2)
    r, _ = st.ranks()
    print(f"max rank after 2 steps {r.max()}, cells above 8: {(r.max(1) > 8).sum()}", flush=True)
    assert (r.max(1) > 8).sum() > 10
    st.step(1)
    got = st.moments()
    st.close()
    mesh.close()
    S = fv.Setup(m, cfg, m0)
    n = m["n_cells"]
    ref = td.run(S, m0, 3)
    ref = np.array([td.macros_of(S, ref[i]) for i in range(n)])
    err, _ = macro_rel_err(got, ref)
    print(f"rank hand-off: max rel macro err {err:.3e}")
    assert err < 1e-5, err


@pytest.mark.parametrize("plain", [False, True])
def test_checkpoint_restore_continues_bit_for_bit(ctx, plain):
    m, cfg, m0 = small_channel_case()
    mesh = tk.Mesh(ctx, m)
    a = tk.State(ctx, mesh, cfg, m0, plain=plain)
    a.step(5)
    ck = a.checkpoint()
    a.step(5)
    # a state built from other initial fields (so another dt) takes the
    # checkpoint's state and step parameters
    other = m0.copy()
    other[:, 4] *= 1.7
    b = tk.State(ctx, mesh, cfg, other, plain=plain)
    b.restore(ck)
    b.step(5)
    assert np.array_equal(a.moments(), b.moments())
    if not plain:
        assert np.array_equal(a.ranks()[0], b.ranks()[0])
    # a checkpoint only fits a state of the same shape
    m2, cfg2, m02 = small_channel_case(N=24)
    c = tk.State(ctx, mesh, cfg2, m02, plain=plain)
    with pytest.raises(tk.TkError) as ei:
        c.restore(ck)
    assert ei.value.status == tk.TK_EINVAL
    with pytest.raises(tk.TkError):
        c.restore(ck[:100])
    if not plain:
        # ranks outside 1..CS in the buffer are refused before they reach
        # the device, and the state still takes the intact checkpoint
        rb = a.ranks()[0]
        b2 = tk.State(ctx, mesh, cfg, m0)
        b2.step(5)
        ck5 = b2.checkpoint()
        pat = b2.ranks()[0].astype(np.int32).tobytes()
        raw = ck5.tobytes()
        off = raw.find(pat)  # the rank section precedes the other int sections
        assert off > 0
        bad = ck5.copy()
        bad[off:off + 4] = np.frombuffer(np.int32(99).tobytes(), dtype=np.uint8)
        with pytest.raises(tk.TkError) as ei:
            b2.restore(bad)
        assert ei.value.status == tk.TK_EINVAL
        b2.restore(ck5)
        b2.step(5)
        assert np.array_equal(b2.ranks()[0], rb)
        b2.close()
    for s in (a, b, c):
        s.close()
    mesh.close()
