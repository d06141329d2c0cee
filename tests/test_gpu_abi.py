"""C-ABI calls on the GPU beyond the step: tk_round on a resident state
against the oracle's truncated HOSVD of each cell's tensor, and contexts
whose device memory comes from the caller's allocator."""

import ctypes as C

import numpy as np
import pytest

import synth
from helpers import macro_rel_err, tucker_full
from oracle import tucker as otk
from paper_1912_04582_amd import tk

pytestmark = pytest.mark.gpu


def small_state(ctx, precision="fp64", N=16, steps=3):
    cfg = dict(synth.make_config("cfg0"), N=N, cap=6, tol=1e-6, precision=precision)
    m = synth.periodic_box(4)
    m0 = synth.initial_macros(cfg, m)
    mesh = tk.Mesh(ctx, m)
    st = tk.State(ctx, mesh, cfg, m0)
    st.step(steps)
    return mesh, st, cfg, m, m0


@pytest.mark.parametrize("precision,N", [("fp64", 16), ("mixed", 32)])
def test_state_round_matches_oracle_hosvd(precision, N):
    ctx = tk.Context(0)
    try:
        mesh, st, cfg, m, _ = small_state(ctx, precision, N)
        cells = range(m["n_cells"])
        full = {c: tucker_full(*st.export(c, N)) for c in cells}
        tol, cap = 1e-3, 4
        st.round(tol, cap)
        worst = 0.0
        for c in cells:
            G, U = st.export(c, N)
            ref = otk.hosvd(full[c], tol, cap)
            assert tuple(G.shape) == ref.ranks, (c, G.shape, ref.ranks)
            err = np.abs(tucker_full(G, U) - otk.full(ref)).max() / np.abs(full[c]).max()
            worst = max(worst, err)
        print(f"tk_round {precision} N={N}: max rel err vs LAPACK HOSVD {worst:.3e}")
        assert worst < 1e-11, worst
        for bad in ((-1.0, 4), (1e-3, 0), (1e-3, cfg["cap"] + 1)):
            with pytest.raises(tk.TkError) as e:
                st.round(*bad)
            assert e.value.status == tk.TK_EINVAL
        st.close(); mesh.close()
    finally:
        ctx.close()


def test_caller_allocator_serves_every_buffer():
    hip = C.CDLL("libamdhip64.so.7")
    hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    hip.hipFree.argtypes = [C.c_void_p]
    live = {}
    calls = {"alloc": 0, "free": 0}

    def alloc(n):
        p = C.c_void_p()
        if hip.hipMalloc(C.byref(p), n) != 0:
            return None
        live[p.value] = n
        calls["alloc"] += 1
        return p.value

    def free(p):
        assert p in live, "free of an address the allocator did not return"
        del live[p]
        calls["free"] += 1
        hip.hipFree(p)

    results = []
    for hooked in (False, True):
        ctx = tk.Context(0, alloc=(alloc, free)) if hooked else tk.Context(0)
        try:
            mesh, st, *_ = small_state(ctx, "fp64", 16, steps=2)
            results.append((st.moments(), st.ranks()[0]))
            if hooked:
                assert calls["alloc"] > 10 and live
            st.close(); mesh.close()
        finally:
            ctx.close()
    assert not live and calls["alloc"] == calls["free"]
    assert np.array_equal(results[0][0], results[1][0]) and np.array_equal(results[0][1], results[1][1])
