"""C-ABI library checks that need no GPU: loading, exported symbols, host-side
mesh validation through a host-only context."""

import os
import re

import numpy as np
import pytest

import synth
from paper_1912_04582_amd import tk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "tk.h")).read()
    return sorted(set(re.findall(r"^\s*(?:tk_status|const char\*)\s+(tk_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    L = tk.lib()
    names = declared_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(tk.EXPORTED) == names


def host_ctx():
    return tk.Context(device=-1)


def test_host_context_validates_meshes():
    ctx = host_ctx()
    try:
        for m in (synth.periodic_box(4), synth.channel_with_obstacle(8, 4, 4, 0.25, ((2, 3), (1, 2), (1, 2)))):
            mesh = tk.Mesh(ctx, m)
            mesh.close()
    finally:
        ctx.close()


def _expect_einval(mesh_dict, needle):
    ctx = host_ctx()
    try:
        with pytest.raises(tk.TkError) as ei:
            tk.Mesh(ctx, mesh_dict)
        assert ei.value.status == tk.TK_EINVAL
        assert needle in str(ei.value)
    finally:
        ctx.close()


def test_open_cell_rejected():
    m = synth.periodic_box(4)
    keep = np.ones(m["n_faces"], dtype=bool)
    keep[5] = False
    for k in ("face_left", "face_right", "face_normal", "face_area"):
        m[k] = m[k][keep]
    m["n_faces"] -= 1
    _expect_einval(m, "not closed")


def test_bad_indices_rejected():
    m = synth.periodic_box(4)
    m["face_right"] = m["face_right"].copy()
    m["face_right"][3] = m["n_cells"] + 7
    _expect_einval(m, "out of range")
    m = synth.periodic_box(4)
    m["face_right"] = m["face_right"].copy()
    m["face_right"][3] = -5  # boundary index 4 with an empty bc table
    _expect_einval(m, "boundary index")


def test_oblique_faces_accepted():
    ctx = host_ctx()
    try:
        tk.Mesh(ctx, synth.jittered_box(3, 3, 3, 1 / 3, seed=0)).close()
    finally:
        ctx.close()


def test_oblique_symmetry_face_rejected():
    # one closed cube cell whose x faces are tilted symmetry planes
    c, s = np.cos(0.3), np.sin(0.3)
    nrm = np.array([[c, s, 0.0], [-c, -s, 0.0], [0, 1.0, 0], [0, -1.0, 0], [0, 0, 1.0], [0, 0, -1.0]])
    m = {"n_cells": 1, "n_faces": 6, "face_left": np.zeros(6, dtype=np.int32),
         "face_right": -np.ones(6, dtype=np.int32), "face_normal": nrm, "face_area": np.ones(6),
         "cell_volume": np.ones(1), "cell_center": np.zeros((1, 3)),
         "bc": [{"kind": synth.BC_SYM}]}
    _expect_einval(m, "coordinate-axis planes")


def test_too_many_faces_rejected():
    m = synth.periodic_box(4)
    for k in ("face_left", "face_right", "face_normal", "face_area"):
        m[k] = np.concatenate([m[k], m[k][:1]])
    m["n_faces"] += 1
    _expect_einval(m, "more than 6 faces")


def test_state_on_host_context_is_edevice():
    ctx = host_ctx()
    try:
        cfg = synth.make_config("cfg0")
        m = synth.periodic_box(4)
        mesh = tk.Mesh(ctx, m)
        with pytest.raises(tk.TkError) as ei:
            tk.State(ctx, mesh, cfg, synth.initial_macros(cfg, m))
        assert ei.value.status == tk.TK_EDEVICE
        mesh.close()
    finally:
        ctx.close()
