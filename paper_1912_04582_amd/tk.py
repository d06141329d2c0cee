"""ctypes binding of libtk.so (include/tk.h): argument marshalling only.

Functions keep the C names (tk_ctx_create, tk_mesh_load, tk_state_init,
tk_moments, tk_step, tk_round_tucker, ...); the small classes below wrap
the handles.  Every computation runs in the HIP library; this module never
falls back to a CPU path and raises if the library is missing.
"""

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtk.so")

TK_OK, TK_PENDING = 0, 1
TK_EINVAL, TK_ENOMEM, TK_ENUMERIC, TK_EDEVICE, TK_EBUSY, TK_ENOTFOUND = -1, -2, -3, -4, -5, -6
TK_BC_SYM, TK_BC_INFLOW, TK_BC_OUTFLOW, TK_BC_WALL = 0, 1, 2, 3
TK_FP64, TK_MIXED = 0, 1

STATUS_NAMES = {0: "TK_OK", 1: "TK_PENDING", -1: "TK_EINVAL", -2: "TK_ENOMEM", -3: "TK_ENUMERIC",
                -4: "TK_EDEVICE", -5: "TK_EBUSY", -6: "TK_ENOTFOUND"}

EXPORTED = [
    "tk_ctx_create", "tk_ctx_destroy", "tk_last_error", "tk_sync", "tk_prof_enable", "tk_prof_get",
    "tk_prof_reset", "tk_prof_eig", "tk_mesh_load", "tk_mesh_destroy", "tk_state_init", "tk_state_init_batch",
    "tk_state_destroy", "tk_state_info", "tk_state_dt", "tk_state_set_chunk", "tk_state_chunk",
    "tk_state_tune", "tk_state_use_graph", "tk_state_streams", "tk_state_rounding", "tk_state_checkpoint", "tk_state_restore", "tk_moments", "tk_step", "tk_step_async", "tk_lusgs", "tk_state_face_rounding",
    "tk_state_ranks", "tk_state_export", "tk_round", "tk_round_tucker", "tk_round_tucker_noalloc",
    "tk_plain_init", "tk_ctx_create_ex",
    "tk_serve_create",
    "tk_serve_submit", "tk_serve_poll", "tk_serve_stats", "tk_serve_destroy",
]


class TkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class tk_bc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_double), ("u", C.c_double * 3), ("T", C.c_double),
                ("T_w", C.c_double)]


class tk_mesh_desc(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("n_faces", C.c_int32),
                ("face_left", C.POINTER(C.c_int32)), ("face_right", C.POINTER(C.c_int32)),
                ("face_normal", C.POINTER(C.c_double)), ("face_area", C.POINTER(C.c_double)),
                ("cell_volume", C.POINTER(C.c_double)), ("cell_center", C.POINTER(C.c_double)),
                ("n_bc", C.c_int32), ("bc", C.POINTER(tk_bc))]


class tk_params(C.Structure):
    _fields_ = [("N", C.c_int32), ("xi_max", C.c_double), ("R_g", C.c_double), ("m", C.c_double),
                ("Pr", C.c_double), ("omega", C.c_double), ("Kn", C.c_double), ("tol", C.c_double),
                ("rank_cap", C.c_int32), ("cfl", C.c_double), ("precision", C.c_int32)]


class tk_tucker(C.Structure):
    _fields_ = [("N", C.c_int32), ("r", C.c_int32 * 3), ("core", C.POINTER(C.c_double)),
                ("U", C.POINTER(C.c_double) * 3)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class tk_alloc_fns(C.Structure):
    _fields_ = [("user", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN)]


class tk_request(C.Structure):
    _fields_ = [("mesh", tk_mesh_desc), ("params", tk_params), ("macro", C.POINTER(C.c_double)),
                ("max_steps", C.c_int32), ("residual_tol", C.c_double)]


class tk_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("steps", C.c_int32), ("residual", C.c_double),
                ("t_arrive", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("macro_out", C.POINTER(C.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1912_04582_amd.build`")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        st = C.c_int32
        sig = {
            "tk_ctx_create": [C.c_int32, C.c_size_t, P, C.POINTER(P)],
            "tk_ctx_destroy": [P],
            "tk_sync": [P],
            "tk_prof_enable": [P, C.c_int32],
            "tk_prof_get": [P, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)],
            "tk_prof_reset": [P],
            "tk_prof_eig": [P, C.POINTER(C.c_int64), C.c_int32],
            "tk_mesh_load": [P, C.POINTER(tk_mesh_desc), C.POINTER(P)],
            "tk_mesh_destroy": [P],
            "tk_state_init": [P, P, C.POINTER(tk_params), C.POINTER(C.c_double), C.POINTER(P)],
            "tk_state_init_batch": [P, C.c_int32, C.POINTER(P), C.POINTER(tk_params),
                                    C.POINTER(C.POINTER(C.c_double)), C.POINTER(P)],
            "tk_plain_init": [P, P, C.POINTER(tk_params), C.POINTER(C.c_double), C.POINTER(P)],
            "tk_state_destroy": [P],
            "tk_state_info": [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
            "tk_state_dt": [P, C.c_int32, C.POINTER(C.c_double)],
            "tk_state_set_chunk": [P, C.c_int32],
            "tk_state_chunk": [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
            "tk_state_tune": [P, C.POINTER(C.c_int32)],
            "tk_state_use_graph": [P, C.c_int32],
            "tk_state_streams": [P, C.c_int32, C.POINTER(C.c_int32)],
            "tk_state_rounding": [P, C.c_int32, C.POINTER(C.c_int64)],
            "tk_state_checkpoint": [P, C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t)],
            "tk_state_restore": [P, C.c_void_p, C.c_size_t],
            "tk_moments": [P, C.POINTER(C.c_double)],
            "tk_step": [P, C.c_int32, C.POINTER(C.c_double)],
            "tk_lusgs": [P, C.c_int32, C.POINTER(C.c_double)],
            "tk_state_face_rounding": [P, C.c_int32],
            "tk_step_async": [P, C.c_int32],
            "tk_state_ranks": [P, C.POINTER(C.c_int32), C.POINTER(C.c_double)],
            "tk_state_export": [P, C.c_int32, C.POINTER(tk_tucker)],
            "tk_round_tucker": [P, C.c_int32, C.POINTER(tk_tucker), C.c_double, C.c_int32,
                                C.POINTER(tk_tucker)],
            "tk_round": [P, C.c_double, C.c_int32],
            "tk_ctx_create_ex": [C.c_int32, C.c_size_t, P, C.POINTER(tk_alloc_fns), C.POINTER(P)],
            "tk_round_tucker_noalloc": [P, C.c_int32, C.c_int32, C.c_int32, P, P, P, C.c_double, C.c_int32,
                                        P, P, P],
            "tk_serve_create": [P, C.c_size_t, C.POINTER(P)],
            "tk_serve_submit": [P, C.POINTER(tk_request), C.POINTER(C.c_uint64)],
            "tk_serve_poll": [P, C.c_uint64, C.POINTER(tk_result)],
            "tk_serve_stats": [P, C.POINTER(C.c_int64)],
            "tk_serve_destroy": [P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = st
        L.tk_last_error.argtypes = [P]
        L.tk_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _check(status, ctx=None):
    if status < 0:
        msg = lib().tk_last_error(ctx).decode() if ctx else ""
        raise TkError(status, msg)
    return status


def make_params(cfg):
    """tk_params from a config dict (N, xi_max, Rg, m, Pr, omega, Kn, tol, cap, cfl, precision)."""
    prec = cfg.get("precision", "fp64")
    return tk_params(int(cfg["N"]), float(cfg["xi_max"]), float(cfg.get("Rg", 0.5)),
                     float(cfg.get("m", 1.0)), float(cfg["Pr"]), float(cfg["omega"]),
                     float(cfg["Kn"]), float(cfg["tol"]), int(cfg["cap"]), float(cfg["cfl"]),
                     TK_MIXED if prec == "mixed" else TK_FP64)


class _MeshArrays:
    """Keeps the numpy arrays of a tk_mesh_desc alive."""

    def __init__(self, m):
        self.fl = np.ascontiguousarray(m["face_left"], dtype=np.int32)
        self.fr = np.ascontiguousarray(m["face_right"], dtype=np.int32)
        self.fn = np.ascontiguousarray(m["face_normal"], dtype=np.float64)
        self.fa = np.ascontiguousarray(m["face_area"], dtype=np.float64)
        self.vol = np.ascontiguousarray(m["cell_volume"], dtype=np.float64)
        self.ctr = np.ascontiguousarray(m["cell_center"], dtype=np.float64)
        bcs = m.get("bc", [])
        self.bc = (tk_bc * max(1, len(bcs)))()
        for i, b in enumerate(bcs):
            self.bc[i] = tk_bc(int(b["kind"]), float(b.get("n", 0.0)),
                               (C.c_double * 3)(*[float(x) for x in b.get("u", (0.0, 0.0, 0.0))]),
                               float(b.get("T", 0.0)), float(b.get("Tw", 0.0)))
        self.desc = tk_mesh_desc(int(m["n_cells"]), int(m["n_faces"]), _iptr(self.fl), _iptr(self.fr),
                                 _dptr(self.fn), _dptr(self.fa), _dptr(self.vol), _dptr(self.ctr),
                                 len(bcs), self.bc)


class Context:
    def __init__(self, device=0, budget=0, stream=None, alloc=None):
        """alloc: optional (alloc(nbytes) -> device address, free(address))
        pair of Python callables used for every device buffer (tk_ctx_create_ex)."""
        h = C.c_void_p()
        if alloc is None:
            _check(lib().tk_ctx_create(int(device), int(budget), stream, C.byref(h)))
        else:
            fa, ff = alloc
            self._alloc = tk_alloc_fns(None, ALLOC_FN(lambda user, n: fa(n) or None),
                                       FREE_FN(lambda user, p: ff(p)))
            _check(lib().tk_ctx_create_ex(int(device), int(budget), stream, C.byref(self._alloc), C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().tk_ctx_destroy(self.h)
            self.h = None

    def sync(self):
        _check(lib().tk_sync(self.h), self.h)

    def prof_enable(self, on=True):
        _check(lib().tk_prof_enable(self.h, 1 if on else 0), self.h)

    def prof_reset(self):
        _check(lib().tk_prof_reset(self.h), self.h)

    def prof_get(self, kernel):
        ms, n = C.c_double(), C.c_int64()
        _check(lib().tk_prof_get(self.h, kernel.encode(), C.byref(ms), C.byref(n)), self.h)
        return ms.value, n.value

    def eig_stats(self, reset=False):
        v = (C.c_int64 * 4)()
        _check(lib().tk_prof_eig(self.h, v, 1 if reset else 0), self.h)
        return {"lead": v[0], "full": v[1], "sweeps": v[2], "fallback": v[3]}

    def round_tucker(self, tensors, tol, cap):
        """tk_round_tucker on a list of (core, [U1, U2, U3]) numpy Tucker tensors."""
        n = len(tensors)
        ins = (tk_tucker * n)()
        outs = (tk_tucker * n)()
        keep, obufs = [], []
        N = tensors[0][1][0].shape[0]
        for i, (G, U) in enumerate(tensors):
            Gf = np.asfortranarray(G, dtype=np.float64)
            Us = [np.asfortranarray(u, dtype=np.float64) for u in U]
            keep += [Gf] + Us
            ins[i].N = N
            ins[i].r = (C.c_int32 * 3)(*G.shape)
            ins[i].core = _dptr(Gf)
            for a in range(3):
                ins[i].U[a] = _dptr(Us[a])
            oc = np.zeros(cap ** 3)
            ou = [np.zeros(N * cap) for _ in range(3)]
            obufs.append((oc, ou))
            outs[i].core = _dptr(oc)
            for a in range(3):
                outs[i].U[a] = _dptr(ou[a])
        _check(lib().tk_round_tucker(self.h, n, ins, float(tol), int(cap), outs), self.h)
        res = []
        for i in range(n):
            r = tuple(outs[i].r)
            oc, ou = obufs[i]
            G = oc[:r[0] * r[1] * r[2]].reshape(r, order="F").copy()
            U = [ou[a][:N * r[a]].reshape((N, r[a]), order="F").copy() for a in range(3)]
            res.append((G, U))
        return res

    def round_tucker_noalloc(self, N, count, in_cap, core_in, fac_in, rank_in, tol, cap, core_out, fac_out,
                             rank_out):
        """tk_round_tucker_noalloc on caller-owned device buffers given as raw
        device addresses (ints), enqueued on the context stream; call sync()
        before reading the outputs."""
        _check(lib().tk_round_tucker_noalloc(self.h, int(N), int(count), int(in_cap), C.c_void_p(core_in),
                                             C.c_void_p(fac_in), C.c_void_p(rank_in), float(tol), int(cap),
                                             C.c_void_p(core_out), C.c_void_p(fac_out), C.c_void_p(rank_out)),
               self.h)


class Mesh:
    def __init__(self, ctx, mesh):
        self.ctx = ctx
        self.arrays = _MeshArrays(mesh)
        h = C.c_void_p()
        _check(lib().tk_mesh_load(ctx.h, C.byref(self.arrays.desc), C.byref(h)), ctx.h)
        self.h = h
        self.n_cells = int(mesh["n_cells"])

    def close(self):
        if self.h:
            lib().tk_mesh_destroy(self.h)
            self.h = None


class State:
    """A Tucker (or, with plain=True, full-tensor) state of one or more instances."""

    def __init__(self, ctx, meshes, cfgs, macros, plain=False):
        self.ctx = ctx
        if isinstance(meshes, Mesh):
            meshes, cfgs, macros = [meshes], [cfgs], [macros]
        self.meshes = meshes
        self.macros_in = [np.ascontiguousarray(m, dtype=np.float64) for m in macros]
        h = C.c_void_p()
        if plain:
            if len(meshes) != 1:
                raise ValueError("plain state takes one mesh")
            p = make_params(cfgs[0])
            _check(lib().tk_plain_init(ctx.h, meshes[0].h, C.byref(p), _dptr(self.macros_in[0]),
                                       C.byref(h)), ctx.h)
        elif len(meshes) == 1:
            p = make_params(cfgs[0])
            _check(lib().tk_state_init(ctx.h, meshes[0].h, C.byref(p), _dptr(self.macros_in[0]),
                                       C.byref(h)), ctx.h)
        else:
            n = len(meshes)
            ps = (tk_params * n)(*[make_params(c) for c in cfgs])
            mh = (C.c_void_p * n)(*[m.h.value for m in meshes])
            mp = (C.POINTER(C.c_double) * n)(*[_dptr(m) for m in self.macros_in])
            _check(lib().tk_state_init_batch(ctx.h, n, mh, ps, mp, C.byref(h)), ctx.h)
        self.h = h
        nc, ni = C.c_int32(), C.c_int32()
        _check(lib().tk_state_info(h, C.byref(nc), C.byref(ni)), ctx.h)
        self.n_cells, self.n_instances = nc.value, ni.value
        self.plain = plain

    def close(self):
        if self.h:
            lib().tk_state_destroy(self.h)
            self.h = None

    def dt(self, inst=0):
        v = C.c_double()
        _check(lib().tk_state_dt(self.h, int(inst), C.byref(v)), self.ctx.h)
        return v.value

    def set_chunk(self, cells):
        """Cells per rounding pass; 0 = chosen by timing trial steps."""
        _check(lib().tk_state_set_chunk(self.h, int(cells)), self.ctx.h)

    def chunk(self):
        c, m = C.c_int32(), C.c_int32()
        _check(lib().tk_state_chunk(self.h, C.byref(c), C.byref(m)), self.ctx.h)
        return c.value, m.value

    def tune(self):
        """Run the pass-size trial steps now (they advance the state);
        returns how many were run."""
        n = C.c_int32()
        _check(lib().tk_state_tune(self.h, C.byref(n)), self.ctx.h)
        return n.value

    def checkpoint(self):
        """The whole state as a host byte array (tk_state_checkpoint)."""
        n = C.c_size_t()
        _check(lib().tk_state_checkpoint(self.h, None, 0, C.byref(n)), self.ctx.h)
        buf = np.zeros(n.value, dtype=np.uint8)
        _check(lib().tk_state_checkpoint(self.h, buf.ctypes.data_as(C.c_void_p), buf.nbytes, C.byref(n)),
               self.ctx.h)
        return buf

    def restore(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib().tk_state_restore(self.h, buf.ctypes.data_as(C.c_void_p), buf.nbytes), self.ctx.h)

    def use_graph(self, on=True):
        _check(lib().tk_state_use_graph(self.h, 1 if on else 0), self.ctx.h)

    def streams(self, two=None):
        """Set alternate passes on a second stream (two=True) or all on one
        (False); None leaves it.  Returns whether a second stream exists."""
        av = C.c_int32()
        _check(lib().tk_state_streams(self.h, -1 if two is None else (1 if two else 0), C.byref(av)), self.ctx.h)
        return bool(av.value)

    def rounding(self, factor_space=None):
        """tk_state_rounding: factor_space True/False selects the rounding
        path, None leaves it.  Returns (and resets) the counters: cells rounded
        in factor space, cells rounded in the N-basis by eager steps, Jacobi
        sweeps and FP64 operations in factor space."""
        v = (C.c_int64 * 4)()
        fs = -1 if factor_space is None else (1 if factor_space else 0)
        _check(lib().tk_state_rounding(self.h, fs, v), self.ctx.h)
        return {"factor": v[0], "nbasis": v[1], "sweeps": v[2], "flops": v[3]}

    def round(self, tol, cap):
        """tk_round: round every cell of the state again (FP64, N-basis)."""
        _check(lib().tk_round(self.h, float(tol), int(cap)), self.ctx.h)

    def moments(self):
        out = np.zeros((self.n_cells, 8))
        _check(lib().tk_moments(self.h, _dptr(out)), self.ctx.h)
        return out

    def step(self, n=1, residual=False):
        res = np.zeros(self.n_instances) if residual else None
        _check(lib().tk_step(self.h, int(n), _dptr(res) if residual else None), self.ctx.h)
        return res

    def lusgs(self, n=1, residual=False):
        """tk_lusgs: n LU-SGS implicit iterations."""
        res = np.zeros(self.n_instances) if residual else None
        _check(lib().tk_lusgs(self.h, int(n), _dptr(res) if residual else None), self.ctx.h)
        return res

    def face_rounding(self, on=True):
        """tk_state_face_rounding: round each face's flux term before the sum."""
        _check(lib().tk_state_face_rounding(self.h, 1 if on else 0), self.ctx.h)

    def step_async(self, n=1):
        _check(lib().tk_step_async(self.h, int(n)), self.ctx.h)

    def ranks(self):
        r = np.zeros((self.n_cells, 3), dtype=np.int32)
        mc = C.c_double()
        _check(lib().tk_state_ranks(self.h, _iptr(r), C.byref(mc)), self.ctx.h)
        return r, mc.value

    def export(self, cell, N, cap=16):
        core = np.zeros(cap ** 3)
        U = [np.zeros(N * cap) for _ in range(3)]
        t = tk_tucker()
        t.core = _dptr(core)
        for a in range(3):
            t.U[a] = _dptr(U[a])
        _check(lib().tk_state_export(self.h, int(cell), C.byref(t)), self.ctx.h)
        r = tuple(t.r)
        G = core[:r[0] * r[1] * r[2]].reshape(r, order="F").copy()
        Us = [U[a][:N * r[a]].reshape((N, r[a]), order="F").copy() for a in range(3)]
        return G, Us


class Server:
    """tk_serve_*: continuous batching of independent solves on one device
    (requests admitted together with the same N and precision share one
    batched state and its launches)."""

    def __init__(self, ctx, budget=0):
        self.ctx = ctx
        h = C.c_void_p()
        _check(lib().tk_serve_create(ctx.h, int(budget), C.byref(h)), ctx.h)
        self.h = h
        self._keep = {}
        self._ncells = {}

    def submit(self, mesh, cfg, macros, max_steps, residual_tol):
        arrays = _MeshArrays(mesh)
        mac = np.ascontiguousarray(macros, dtype=np.float64)
        req = tk_request(arrays.desc, make_params(cfg), _dptr(mac), int(max_steps), float(residual_tol))
        t = C.c_uint64()
        _check(lib().tk_serve_submit(self.h, C.byref(req), C.byref(t)), self.ctx.h)
        self._ncells[t.value] = int(mesh["n_cells"])
        return t.value

    def poll(self, ticket, want_macros=True):
        res = tk_result()
        out = np.zeros((self._ncells.get(ticket, 0), 8)) if want_macros else None
        res.macro_out = _dptr(out) if want_macros else None
        st = lib().tk_serve_poll(self.h, C.c_uint64(ticket), C.byref(res))
        if st == TK_ENOTFOUND:
            raise TkError(st, "unknown ticket")
        return {"status": res.status, "steps": res.steps, "residual": res.residual,
                "t_arrive": res.t_arrive, "t_admit": res.t_admit, "t_done": res.t_done,
                "macros": out if res.status != TK_PENDING else None}

    def stats(self):
        """Cohorts formed, cohort steps (shared launch sets), request steps,
        requests in the largest cohort."""
        v = (C.c_int64 * 4)()
        _check(lib().tk_serve_stats(self.h, v), self.ctx.h)
        return {"cohorts": v[0], "cohort_steps": v[1], "request_steps": v[2], "largest_cohort": v[3]}

    def close(self):
        if self.h:
            lib().tk_serve_destroy(self.h)
            self.h = None
