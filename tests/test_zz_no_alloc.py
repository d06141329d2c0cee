"""tk_round_tucker_noalloc (device buffers, no device allocation, work space
in the library's fixed scratch array) against tk_round_tucker on the same
Tucker tensors: the same kernels, so the same bits.  Two calls in a row, the
first over more tensors than one pass of the scratch array holds, the second
over fewer."""

import ctypes as C

import numpy as np
import pytest

from paper_1912_04582_amd import tk

pytestmark = pytest.mark.gpu


class DeviceBuffers:
    """Device memory for the test through the HIP runtime the library itself
    loads (libamdhip64.so.7): the test allocates, the entry point does not."""

    def __init__(self):
        tk.lib()
        self.hip = C.CDLL("libamdhip64.so.7")
        self.hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        self.hip.hipFree.argtypes = [C.c_void_p]
        self.hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        self.ptrs = []

    def _ok(self, e, what):
        assert e == 0, f"{what} failed with HIP error {e}"

    def put(self, a):
        a = np.ascontiguousarray(a)
        p = C.c_void_p()
        self._ok(self.hip.hipMalloc(C.byref(p), max(a.nbytes, 8)), "hipMalloc")
        self.ptrs.append(p.value)
        self._ok(self.hip.hipMemcpy(p.value, a.ctypes.data, a.nbytes, 1), "hipMemcpy H2D")
        return p.value

    def get(self, ptr, like):
        out = np.empty_like(like)
        self._ok(self.hip.hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2), "hipMemcpy D2H")
        return out

    def free(self):
        for p in self.ptrs:
            self.hip.hipFree(p)
        self.ptrs = []


def random_tuckers(rng, N, count, rmax):
    out = []
    x = np.linspace(-3.0, 3.0, N)
    for t in range(count):
        r = tuple(int(v) for v in rng.integers(1, rmax + 1, 3))
        G = rng.standard_normal(r)
        G *= np.exp(-np.add.outer(np.add.outer(np.arange(r[0]), np.arange(r[1])), np.arange(r[2])))
        U = []
        for a in range(3):
            base = np.exp(-(x[:, None] - rng.uniform(-1, 1, r[a])[None, :]) ** 2)
            U.append(base + 1e-3 * rng.standard_normal((N, r[a])))
        out.append((G, U))
    return out


def pack(tensors, N, cap):
    n = len(tensors)
    core = np.zeros((n, cap, cap, cap))  # [t][k3][k2][k1]
    fac = np.zeros((n, 3, cap, N))
    rank = np.zeros((n, 3), dtype=np.int32)
    for t, (G, U) in enumerate(tensors):
        r = G.shape
        rank[t] = r
        core[t, :r[2], :r[1], :r[0]] = np.transpose(G, (2, 1, 0))
        for a in range(3):
            fac[t, a, :r[a], :] = U[a].T
    return core, fac, rank


def run_noalloc(ctx, dev, tensors, N, in_cap, tol, cap):
    core, fac, rank = pack(tensors, N, in_cap)
    n = len(tensors)
    ci, fi, ri = dev.put(core), dev.put(fac), dev.put(rank)
    co_h = np.full((n, cap, cap, cap), np.nan)
    fo_h = np.full((n, 3, cap, N), np.nan)
    ro_h = np.full((n, 3), -7, dtype=np.int32)
    co, fo, ro = dev.put(co_h), dev.put(fo_h), dev.put(ro_h)
    ctx.round_tucker_noalloc(N, n, in_cap, ci, fi, ri, tol, cap, co, fo, ro)
    ctx.sync()
    co, fo, ro = dev.get(co, co_h), dev.get(fo, fo_h), dev.get(ro, ro_h)
    out = []
    for t in range(n):
        r = tuple(int(v) for v in ro[t])
        assert all(1 <= v <= cap for v in r), r
        # padding beyond the ranks is written as zeros
        assert np.all(np.isfinite(co[t])) and np.all(np.isfinite(fo[t]))
        G = np.transpose(co[t, :r[2], :r[1], :r[0]], (2, 1, 0))
        U = [fo[t, a, :r[a], :].T for a in range(3)]
        out.append((G, U))
    return out


@pytest.mark.parametrize("N", [32, 16])
def test_noalloc_rounding_equals_allocating_rounding(N):
    rng = np.random.default_rng(100 + N)
    ctx = tk.Context(0)
    dev = DeviceBuffers()
    try:
        # one pass of the 32 MiB array holds 107 tensors at N = 32 and 699 at
        # N = 16: the first call spans two passes at N = 32
        for count, tol, cap in ((130, 1e-6, 8), (5, 1e-4, 12)):
            tensors = random_tuckers(rng, N, count, 10)
            in_cap = max(max(G.shape) for G, _ in tensors)
            ref = ctx.round_tucker(tensors, tol, cap)
            got = run_noalloc(ctx, dev, tensors, N, in_cap, tol, cap)
            for (Gr, Ur), (Gg, Ug) in zip(ref, got):
                assert Gr.shape == Gg.shape
                assert np.array_equal(Gr, Gg)
                for a in range(3):
                    assert np.array_equal(Ur[a], Ug[a])
    finally:
        dev.free()
        ctx.close()


def test_noalloc_rejects_bad_shapes():
    ctx = tk.Context(0)
    try:
        for N, in_cap, cap in ((48, 4, 4), (32, 17, 4), (16, 4, 17), (16, 20, 4)):
            with pytest.raises(tk.TkError) as e:
                ctx.round_tucker_noalloc(N, 1, in_cap, 1, 1, 1, 1e-6, cap, 1, 1, 1)
            assert e.value.status == tk.TK_EINVAL
    finally:
        ctx.close()
