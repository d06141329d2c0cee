"""STAR-CD ASCII hexahedral meshes (the mesh input of the paper's program,
Sec. "The program") to and from the mesh description that `tk_mesh_load`
takes.

Files, whitespace separated, one record per line:

* ``<prefix>.vrt``: ``vertex_id x y z``
* ``<prefix>.cel``: ``cell_id v1 v2 v3 v4 v5 v6 v7 v8 [further integers]``
  (v1-v4 one end face in cyclic order, v5-v8 the opposite face, v(k+4)
  joined to vk)
* ``<prefix>.bnd``: ``face_id v1 v2 v3 v4 region [further fields]``

Vertex ids may be any positive integers.  Geometry of each (possibly
non-planar) quadrilateral face: the vector area S = (x3 - x1) x (x4 - x2) / 2,
exact for a bilinear face, so the faces of a closed hexahedron sum to zero;
cell volume V = sum over its faces of S . xbar / 3 with S outward and xbar
the mean of the face's four vertices; cell centre: mean of its eight
vertices.  Faces are oriented from their left cell to the right cell (or out
of the mesh on boundary faces).
"""

import numpy as np

# the six faces of a hexahedron, as positions in its vertex list
_HEX_FACES = ((0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7))


def _ints(line, n):
    parts = line.split()
    return [int(p) for p in parts[:n]], parts[n:]


def read_starcd(prefix, bc_by_region):
    """Mesh description (dict of arrays, the layout of `tk_mesh_desc`) of the
    STAR-CD files `prefix`.vrt/.cel/.bnd.

    bc_by_region: {region id of the .bnd file: boundary condition dict with
    'kind', 'n', 'u', 'T', 'Tw'}.  Raises ValueError on a face shared by more
    than two cells, a cell face neither shared nor listed in the .bnd file,
    or a boundary face of a region without a condition.
    """
    vid, xyz = [], []
    with open(prefix + ".vrt") as fh:
        for line in fh:
            if not line.strip():
                continue
            p = line.split()
            vid.append(int(p[0]))
            xyz.append([float(p[1]), float(p[2]), float(p[3])])
    index = {v: i for i, v in enumerate(vid)}
    X = np.array(xyz, dtype=np.float64)
    cells = []
    with open(prefix + ".cel") as fh:
        for line in fh:
            if not line.strip():
                continue
            ids, _ = _ints(line, 9)
            cells.append([index[v] for v in ids[1:9]])
    cells = np.array(cells, dtype=np.int64)
    regions = sorted(bc_by_region)
    bc_index = {r: i for i, r in enumerate(regions)}
    bnd = {}
    with open(prefix + ".bnd") as fh:
        for line in fh:
            if not line.strip():
                continue
            ids, _ = _ints(line, 6)
            key = tuple(sorted(index[v] for v in ids[1:5]))
            if ids[5] not in bc_index:
                raise ValueError(f"boundary region {ids[5]} has no condition")
            bnd[key] = bc_index[ids[5]]
    nc = cells.shape[0]
    ctr = X[cells].mean(axis=1)
    owner = {}
    fl, fr, S, xb = [], [], [], []
    for c in range(nc):
        for f in _HEX_FACES:
            q = [int(cells[c, i]) for i in f]
            key = tuple(sorted(q))
            x0, x1, x2, x3 = X[q[0]], X[q[1]], X[q[2]], X[q[3]]
            s = 0.5 * np.cross(x2 - x0, x3 - x1)
            mid = 0.25 * (x0 + x1 + x2 + x3)
            if np.dot(s, mid - ctr[c]) < 0.0:
                s = -s  # outward from c
            if key in owner:
                j = owner.pop(key)
                if j < 0:
                    raise ValueError("face shared by more than two cells")
                fr[j] = c
                owner[key] = -1
            else:
                owner[key] = len(fl)
                fl.append(c)
                fr.append(None)
                S.append(s)
                xb.append(mid)
    for key, j in owner.items():
        if j >= 0:
            if key not in bnd:
                raise ValueError(f"open face {key} is not a boundary face")
            fr[j] = -(bnd[key] + 1)
    fl = np.array(fl, dtype=np.int64)
    fr = np.array(fr, dtype=np.int64)
    S = np.array(S)
    xb = np.array(xb)
    vol = np.zeros(nc)
    np.add.at(vol, fl, (S * xb).sum(1) / 3.0)
    inner = fr >= 0
    np.add.at(vol, fr[inner], -(S[inner] * xb[inner]).sum(1) / 3.0)
    A = np.sqrt((S * S).sum(1))
    return {
        "n_cells": nc, "n_faces": int(fl.shape[0]),
        "face_left": fl.astype(np.int32), "face_right": fr.astype(np.int32),
        "face_normal": S / A[:, None], "face_area": A, "cell_volume": vol, "cell_center": ctr,
        "bc": [dict(bc_by_region[r]) for r in regions],
    }


def write_starcd(prefix, nodes, cells, bnd_faces, bnd_regions):
    """Write STAR-CD ASCII files: nodes [V,3], cells [C,8] (0-based vertex
    positions in STAR-CD order), boundary faces [B,4] (0-based) with their
    region ids [B].  Vertex, cell and face ids are written 1-based."""
    with open(prefix + ".vrt", "w") as fh:
        for i, x in enumerate(np.asarray(nodes, dtype=np.float64)):
            fh.write(f"{i + 1:9d} {x[0]:.17g} {x[1]:.17g} {x[2]:.17g}\n")
    with open(prefix + ".cel", "w") as fh:
        for i, c in enumerate(np.asarray(cells)):
            fh.write(f"{i + 1:9d} " + " ".join(f"{int(v) + 1:9d}" for v in c) + "        1        1\n")
    with open(prefix + ".bnd", "w") as fh:
        for i, (f, r) in enumerate(zip(np.asarray(bnd_faces), np.asarray(bnd_regions))):
            fh.write(f"{i + 1:9d} " + " ".join(f"{int(v) + 1:9d}" for v in f) + f" {int(r):9d}        1  WALL\n")
