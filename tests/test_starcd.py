"""STAR-CD ASCII mesh files: a jittered lattice written in that format and
read back gives the generator's mesh (volumes, face areas, closure, boundary
faces), and the C ABI accepts it."""

import numpy as np
import pytest

import synth
from paper_1912_04582_amd import starcd, tk


def lattice_files(tmp_path, nx, ny, nz, h, seed, jitter=0.2):
    # the node field of synth.jittered_box for the same arguments
    rng = np.random.default_rng(seed)
    X = np.stack(np.meshgrid(np.arange(nx + 1) * h, np.arange(ny + 1) * h, np.arange(nz + 1) * h,
                             indexing="ij"), -1)
    inner = np.zeros((nx + 1, ny + 1, nz + 1), dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    X = X + rng.uniform(-jitter * h, jitter * h, size=X.shape) * inner[..., None]
    vid = np.arange((nx + 1) * (ny + 1) * (nz + 1)).reshape(nx + 1, ny + 1, nz + 1)
    cells = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                cells.append([vid[i, j, k], vid[i + 1, j, k], vid[i + 1, j + 1, k], vid[i, j + 1, k],
                              vid[i, j, k + 1], vid[i + 1, j, k + 1], vid[i + 1, j + 1, k + 1], vid[i, j + 1, k + 1]])
    bnd, reg = [], []
    for j in range(ny):
        for k in range(nz):
            bnd += [[vid[0, j, k], vid[0, j + 1, k], vid[0, j + 1, k + 1], vid[0, j, k + 1]],
                    [vid[nx, j, k], vid[nx, j + 1, k], vid[nx, j + 1, k + 1], vid[nx, j, k + 1]]]
            reg += [1, 2]
    for i in range(nx):
        for k in range(nz):
            bnd += [[vid[i, 0, k], vid[i + 1, 0, k], vid[i + 1, 0, k + 1], vid[i, 0, k + 1]],
                    [vid[i, ny, k], vid[i + 1, ny, k], vid[i + 1, ny, k + 1], vid[i, ny, k + 1]]]
            reg += [3, 3]
    for i in range(nx):
        for j in range(ny):
            bnd += [[vid[i, j, 0], vid[i + 1, j, 0], vid[i + 1, j + 1, 0], vid[i, j + 1, 0]],
                    [vid[i, j, nz], vid[i + 1, j, nz], vid[i + 1, j + 1, nz], vid[i, j + 1, nz]]]
            reg += [3, 3]
    prefix = str(tmp_path / "box")
    starcd.write_starcd(prefix, X.reshape(-1, 3), np.array(cells), np.array(bnd), np.array(reg))
    return prefix


BCS = {1: {"kind": synth.BC_INFLOW, "n": 1.0, "u": (0.5, 0.0, 0.0), "T": 1.0, "Tw": 0.0},
       2: {"kind": synth.BC_OUTFLOW, "n": 0.0, "u": (0.0, 0.0, 0.0), "T": 0.0, "Tw": 0.0},
       3: {"kind": synth.BC_SYM, "n": 0.0, "u": (0.0, 0.0, 0.0), "T": 0.0, "Tw": 0.0}}


def test_read_back_matches_generator(tmp_path):
    nx, ny, nz, h = 4, 3, 2, 0.25
    m = starcd.read_starcd(lattice_files(tmp_path, nx, ny, nz, h, seed=9), BCS)
    ref = synth.jittered_box(nx, ny, nz, h, seed=9, permute=False)
    assert m["n_cells"] == ref["n_cells"] == nx * ny * nz
    assert m["n_faces"] == ref["n_faces"]
    np.testing.assert_allclose(m["cell_volume"], ref["cell_volume"], rtol=1e-13)
    np.testing.assert_allclose(m["cell_center"], ref["cell_center"], rtol=0, atol=1e-15)
    assert abs(m["cell_volume"].sum() - nx * ny * nz * h ** 3) < 1e-14
    np.testing.assert_allclose(np.sort(m["face_area"]), np.sort(ref["face_area"]), rtol=1e-13)
    assert synth.meshes.check_closed(m) < 1e-13
    # boundary faces: x-min inflow, x-max outflow, the rest symmetry
    fr, fn = m["face_right"], m["face_normal"]
    for b, want in ((0, (-1, 0, 0)), (1, (1, 0, 0))):
        sel = fr == -(b + 1)
        assert sel.sum() == ny * nz
        np.testing.assert_allclose(fn[sel], np.tile(want, (sel.sum(), 1)), atol=1e-15)
    assert (fr == -3).sum() == 2 * (nx * nz + nx * ny)


def test_loads_through_the_c_abi(tmp_path):
    m = starcd.read_starcd(lattice_files(tmp_path, 3, 3, 3, 1 / 3, seed=2), BCS)
    ctx = tk.Context(device=-1)
    try:
        tk.Mesh(ctx, m).close()
    finally:
        ctx.close()


def test_errors(tmp_path):
    prefix = lattice_files(tmp_path, 2, 2, 2, 0.5, seed=1)
    with pytest.raises(ValueError, match="no condition"):
        starcd.read_starcd(prefix, {1: BCS[1], 2: BCS[2]})
    # drop one boundary record: an open face
    lines = open(prefix + ".bnd").read().splitlines()
    open(prefix + ".bnd", "w").write("\n".join(lines[1:]) + "\n")
    with pytest.raises(ValueError, match="open face"):
        starcd.read_starcd(prefix, BCS)
