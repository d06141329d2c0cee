"""Pins of the oracle's intermediate-rounding step (each face's flux term
rounded before the sum; Section "Tensorized discrete velocity method")."""

import numpy as np
import pytest

import synth
from oracle import dvm, fv, tucker as tk, tucker_dvm as td


def small_cfg(**kw):
    cfg = dict(N=8, xi_max=4.0, cap=8, tol=0.0, cfl=0.5, Pr=2 / 3, omega=0.5, Kn=0.1,
               Rg=0.5, m=1.0, seed=0, init="random")
    cfg.update(kw)
    return cfg


def meshes():
    return {
        "channel": synth.channel_with_obstacle(nx=5, ny=3, nz=3, h=0.25, obstacle=((2, 3), (1, 2), (1, 2)),
                                               inflow=(1.0, (0.8, 0.0, 0.0), 1.0), Tw=1.3),
        "jittered": synth.jittered_box(3, 3, 2, 1 / 3, seed=5),
    }


def face_terms_full(S, i, F):
    """Per face of cell i, its contribution to f* on the full grid (the O1
    flux of the face times -dt s A / V)."""
    mesh = S.mesh
    V = mesh["cell_volume"][i]
    out = []
    for j, s in S.cell_faces[i]:
        L, Rc = mesh["face_left"][j], mesh["face_right"][j]
        fL = F[L]
        fR = F[Rc] if Rc >= 0 else dvm.ghost_full(S, j, fL)
        xn = S.xin_full(j)
        est = S.estimate_full(j)
        Fj = 0.5 * xn * (fL + fR) - 0.5 * est * (fR - fL)
        out.append(-S.dt * s * (mesh["face_area"][j] / V) * Fj)
    return out


@pytest.mark.parametrize("kind", ["channel", "jittered"])
def test_face_rounding_without_truncation_is_the_full_step(kind):
    mesh = meshes()[kind]
    cfg = small_cfg()
    m0 = synth.initial_macros(cfg, mesh)
    S = fv.Setup(mesh, cfg, m0)
    F = dvm.initial_full(S, m0)
    out = td.step_faces(S, td.initial_states(S, m0))
    for i in range(mesh["n_cells"]):
        X = dvm.update_full(S, i, lambda c: F[c])
        np.testing.assert_allclose(tk.full(out[i]), X, rtol=0, atol=1e-12 * np.abs(X).max())


@pytest.mark.parametrize("kind", ["channel", "jittered"])
def test_face_rounding_error_within_the_roundings_bound(kind):
    # each T-HOSVD keeps tail <= eps^2 |A|^2 / 3 per mode, so it moves its
    # tensor by at most eps |A|; the variant's error against the exact update
    # is at most eps (sum_l |E_l| + |sum|) with |sum| <= |f*| + sum_l eps |E_l|
    mesh = meshes()[kind]
    eps = 1e-3
    cfg = small_cfg(N=10, cap=10, tol=eps)
    m0 = synth.initial_macros(cfg, mesh)
    S = fv.Setup(mesh, cfg, m0)
    # from states of rank > 1 (one ordinary step), so that the face terms
    # have something to drop on axis-aligned faces too
    st = td.step(S, td.initial_states(S, m0))
    F = {i: tk.full(t) for i, t in st.items()}
    var = td.step_faces(S, st)
    one = td.step(S, st)
    moved = 0.0
    for i in range(mesh["n_cells"]):
        X = dvm.update_full(S, i, lambda c: F[c])
        E = [np.linalg.norm(e) for e in face_terms_full(S, i, F)]
        bound = eps * (sum(E) + np.linalg.norm(X) + eps * sum(E))
        err = np.linalg.norm(tk.full(var[i]) - X)
        assert err <= bound * (1 + 1e-9), (i, err, bound)
        moved = max(moved, np.linalg.norm(tk.full(var[i]) - tk.full(one[i])) / np.linalg.norm(X))
    # a real variant: the intermediate roundings change the result
    assert moved > 1e-12


def test_face_rounding_matches_full_tensor_hosvd_placement():
    # the same placement through LAPACK's SVD of full tensors: each face term
    # (from O1's flux) rounded by Op1, the sum with the cell's own terms
    # rounded again; the oracle reaches it through the concatenated factors
    mesh = meshes()["jittered"]
    eps = 1e-4
    cfg = small_cfg(N=10, cap=10, tol=eps)
    m0 = synth.initial_macros(cfg, mesh)
    S = fv.Setup(mesh, cfg, m0)
    F = dvm.initial_full(S, m0)
    var = td.step_faces(S, td.initial_states(S, m0))
    for i in range(mesh["n_cells"]):
        X = dvm.update_full(S, i, lambda c: F[c])
        E = face_terms_full(S, i, F)
        own = X - sum(E)
        Er = [tk.full(tk.hosvd(e, eps, cfg["cap"])) for e in E]
        ref = tk.hosvd(own + sum(Er), eps, cfg["cap"])
        assert ref.ranks == var[i].ranks
        a = tk.full(ref)
        np.testing.assert_allclose(tk.full(var[i]), a, rtol=0, atol=1e-10 * np.abs(a).max())
