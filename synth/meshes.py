"""Hexahedral mesh generators (seeded, synthetic).

A mesh is a plain dict of numpy arrays, the same content the paper's mesh
reader stores for the solver (cell volumes, face normals and areas, face to
cell connectivity; Section "Implementation"):

  n_cells, n_faces           ints
  face_left   int32[n_f]     cell on the side the normal points away from
  face_right  int32[n_f]     cell the normal points into, or -(bc+1) for a
                             boundary face (the left cell is then the
                             interior cell and the normal points out of the
                             domain)
  face_normal float64[n_f,3] unit normal, left -> right
  face_area   float64[n_f]
  cell_volume float64[n_c]
  cell_center float64[n_c,3]
  bc          list of dicts  {"kind": BC_*, "n", "u", "T", "Tw"}

Periodic boundaries are expressed as interior faces.  Geometry of
non-planar faces uses the bilinear-face vector area S = (x2-x0) x (x3-x1)/2,
which makes every closed hexahedron's vector areas sum to zero; the volume
is sum_f S_f . xbar_f / 3 over the outward face vectors.
"""

import numpy as np

BC_SYM, BC_INFLOW, BC_OUTFLOW, BC_WALL = 0, 1, 2, 3


def _bc(kind, n=0.0, u=(0.0, 0.0, 0.0), T=0.0, Tw=0.0):
    return {"kind": int(kind), "n": float(n), "u": tuple(float(x) for x in u),
            "T": float(T), "Tw": float(Tw)}


def _finish(fl, fr, fn, fa, vol, ctr, bcs):
    return {
        "n_cells": int(vol.shape[0]),
        "n_faces": int(fl.shape[0]),
        "face_left": np.ascontiguousarray(fl, dtype=np.int32),
        "face_right": np.ascontiguousarray(fr, dtype=np.int32),
        "face_normal": np.ascontiguousarray(fn, dtype=np.float64),
        "face_area": np.ascontiguousarray(fa, dtype=np.float64),
        "cell_volume": np.ascontiguousarray(vol, dtype=np.float64),
        "cell_center": np.ascontiguousarray(ctr, dtype=np.float64),
        "bc": list(bcs),
    }


def periodic_box(n, length=1.0):
    """n^3 cubic cells on [0,length]^3 with periodic wrap in every axis.

    Cell (i,j,k) has index i + n*(j + n*k).  Every cell owns its +x, +y and
    +z faces (normal +e_axis), so there are 3 n^3 faces, all interior.
    """
    n = int(n)
    if n < 3:
        raise ValueError("periodic box needs at least 3 cells per axis")
    h = length / n
    idx = np.arange(n ** 3).reshape(n, n, n)  # [k, j, i]
    fl, fr, fn = [], [], []
    for ax in range(3):
        nb = np.roll(idx, -1, axis=2 - ax)  # +1 along axis ax (i is last)
        fl.append(idx.ravel())
        fr.append(nb.ravel())
        e = np.zeros((n ** 3, 3))
        e[:, ax] = 1.0
        fn.append(e)
    fl = np.concatenate(fl)
    fr = np.concatenate(fr)
    fn = np.concatenate(fn)
    fa = np.full(fl.shape[0], h * h)
    vol = np.full(n ** 3, h ** 3)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ctr = np.stack([(i.ravel() + 0.5) * h, (j.ravel() + 0.5) * h, (k.ravel() + 0.5) * h], 1)
    return _finish(fl, fr, fn, fa, vol, ctr, [])


def channel_with_obstacle(nx=64, ny=32, nz=32, h=1.0 / 32,
                          obstacle=((16, 24), (12, 20), (12, 20)),
                          inflow=(1.0, (2.0 * np.sqrt(5.0 / 6.0), 0.0, 0.0), 1.0),
                          Tw=1.0):
    """Cartesian channel with a removed box of cells (a solid obstacle).

    x-min faces: free-stream inflow (n, u, T from `inflow`); x-max faces:
    zero-gradient outflow; y and z side planes: symmetry; faces between a
    fluid cell and an obstacle cell: diffuse wall at temperature Tw.
    The default inflow speed 2*sqrt(5/6) is Mach 2 for a monatomic gas with
    R_g = 1/2 and T = 1 (sound speed sqrt(gamma R_g T), gamma = 5/3).
    Boundary-condition ids: 0 inflow, 1 outflow, 2 symmetry, 3 wall.
    """
    present = np.ones((nz, ny, nx), dtype=bool)  # [k, j, i]
    if obstacle is not None:
        (i0, i1), (j0, j1), (k0, k1) = obstacle
        present[k0:k1, j0:j1, i0:i1] = False
    cid = -np.ones((nz, ny, nx), dtype=np.int64)
    cid[present] = np.arange(int(present.sum()))
    bcs = [_bc(BC_INFLOW, inflow[0], inflow[1], inflow[2]), _bc(BC_OUTFLOW),
           _bc(BC_SYM), _bc(BC_WALL, Tw=Tw)]
    B_IN, B_OUT, B_SYM, B_WALL = 0, 1, 2, 3
    fl, fr, fn = [], [], []

    def add(l, r, ax, sgn):
        fl.append(l)
        fr.append(r)
        e = np.zeros((l.shape[0], 3))
        e[:, ax] = sgn
        fn.append(e)

    dims = (nx, ny, nz)
    for ax in range(3):
        npax = 2 - ax  # numpy axis of lattice axis ax
        n_ax = dims[ax]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[npax] = slice(0, n_ax - 1)
        hi[npax] = slice(1, n_ax)
        cl, ch = cid[tuple(lo)], cid[tuple(hi)]
        both = (cl >= 0) & (ch >= 0)
        add(cl[both], ch[both], ax, 1.0)
        wall_up = (cl >= 0) & (ch < 0)  # fluid below, obstacle above
        add(cl[wall_up], np.full(int(wall_up.sum()), -(B_WALL + 1)), ax, 1.0)
        wall_dn = (cl < 0) & (ch >= 0)
        add(ch[wall_dn], np.full(int(wall_dn.sum()), -(B_WALL + 1)), ax, -1.0)
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[npax] = 0
        last[npax] = n_ax - 1
        cf, cz = cid[tuple(first)].ravel(), cid[tuple(last)].ravel()
        cf, cz = cf[cf >= 0], cz[cz >= 0]
        b_lo = B_IN if ax == 0 else B_SYM
        b_hi = B_OUT if ax == 0 else B_SYM
        add(cf, np.full(cf.shape[0], -(b_lo + 1)), ax, -1.0)
        add(cz, np.full(cz.shape[0], -(b_hi + 1)), ax, 1.0)
    fl = np.concatenate(fl)
    fr = np.concatenate(fr)
    fn = np.concatenate(fn)
    fa = np.full(fl.shape[0], h * h)
    nc = int(present.sum())
    vol = np.full(nc, h ** 3)
    k, j, i = np.nonzero(present)
    ctr = np.stack([(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h], 1)
    return _finish(fl, fr, fn, fa, vol, ctr, bcs)


def _face_vector(x0, x1, x2, x3):
    return 0.5 * np.cross(x2 - x0, x3 - x1)


def jittered_box(nx, ny, nz, h, seed, jitter=0.2, permute=True):
    """Hex mesh of an nx*ny*nz lattice with interior nodes displaced.

    Every interior node coordinate is moved by U(-jitter*h, jitter*h);
    boundary nodes stay on the box, so boundary faces remain exact
    axis-aligned planes.  The box is closed by symmetry planes (bc id 0).
    With `permute`, faces are randomly reordered and each interior face has
    its left/right cells swapped (normal flipped) with probability 1/2.
    """
    rng = np.random.default_rng(seed)
    X = np.stack(np.meshgrid(np.arange(nx + 1) * h, np.arange(ny + 1) * h,
                             np.arange(nz + 1) * h, indexing="ij"), -1)  # [i,j,k,3]
    inner = np.zeros((nx + 1, ny + 1, nz + 1), dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    d = rng.uniform(-jitter * h, jitter * h, size=X.shape)
    X = X + d * inner[..., None]
    cid = np.arange(nx * ny * nz).reshape(nz, ny, nx).transpose(2, 1, 0)  # [i,j,k]
    bcs = [_bc(BC_SYM)]
    fl, fr, S, xb = [], [], [], []

    def faces(ax):
        # face nodes ordered so that S points along +axis
        if ax == 0:
            I = np.arange(nx + 1)[:, None, None]
            J = np.arange(ny)[None, :, None]
            K = np.arange(nz)[None, None, :]
            I, J, K = np.broadcast_arrays(I, J, K)
            n0, n1, n2, n3 = X[I, J, K], X[I, J + 1, K], X[I, J + 1, K + 1], X[I, J, K + 1]
            lo_ok, hi_ok = I > 0, I < nx
            lo_c = cid[np.maximum(I - 1, 0), J, K]
            hi_c = cid[np.minimum(I, nx - 1), J, K]
        elif ax == 1:
            I = np.arange(nx)[:, None, None]
            J = np.arange(ny + 1)[None, :, None]
            K = np.arange(nz)[None, None, :]
            I, J, K = np.broadcast_arrays(I, J, K)
            n0, n1, n2, n3 = X[I, J, K], X[I, J, K + 1], X[I + 1, J, K + 1], X[I + 1, J, K]
            lo_ok, hi_ok = J > 0, J < ny
            lo_c = cid[I, np.maximum(J - 1, 0), K]
            hi_c = cid[I, np.minimum(J, ny - 1), K]
        else:
            I = np.arange(nx)[:, None, None]
            J = np.arange(ny)[None, :, None]
            K = np.arange(nz + 1)[None, None, :]
            I, J, K = np.broadcast_arrays(I, J, K)
            n0, n1, n2, n3 = X[I, J, K], X[I + 1, J, K], X[I + 1, J + 1, K], X[I, J + 1, K]
            lo_ok, hi_ok = K > 0, K < nz
            lo_c = cid[I, J, np.maximum(K - 1, 0)]
            hi_c = cid[I, J, np.minimum(K, nz - 1)]
        s = _face_vector(n0, n1, n2, n3).reshape(-1, 3)
        c = (0.25 * (n0 + n1 + n2 + n3)).reshape(-1, 3)
        lo_ok, hi_ok = lo_ok.ravel(), hi_ok.ravel()
        lo_c, hi_c = lo_c.ravel(), hi_c.ravel()
        inter = lo_ok & hi_ok
        fl.append(lo_c[inter]); fr.append(hi_c[inter]); S.append(s[inter]); xb.append(c[inter])
        lo_b = ~lo_ok  # face on the low boundary plane: cell above, normal -axis
        fl.append(hi_c[lo_b]); fr.append(np.full(int(lo_b.sum()), -1)); S.append(-s[lo_b]); xb.append(c[lo_b])
        hi_b = ~hi_ok
        fl.append(lo_c[hi_b]); fr.append(np.full(int(hi_b.sum()), -1)); S.append(s[hi_b]); xb.append(c[hi_b])

    for ax in range(3):
        faces(ax)
    fl = np.concatenate(fl).astype(np.int64)
    fr = np.concatenate(fr).astype(np.int64)
    S = np.concatenate(S)
    xb = np.concatenate(xb)
    nc = nx * ny * nz
    # volumes from outward face vectors
    vol = np.zeros(nc)
    np.add.at(vol, fl, (S * xb).sum(1) / 3.0)
    interior = fr >= 0
    np.add.at(vol, fr[interior], -(S[interior] * xb[interior]).sum(1) / 3.0)
    ctr = np.zeros((nc, 3))
    # cell centre: mean of the 8 corner nodes
    for di in (0, 1):
        for dj in (0, 1):
            for dk in (0, 1):
                ctr += X[di:nx + di, dj:ny + dj, dk:nz + dk].transpose(2, 1, 0, 3).reshape(-1, 3)
    ctr /= 8.0
    if permute:
        perm = rng.permutation(fl.shape[0])
        fl, fr, S = fl[perm], fr[perm], S[perm]
        swap = (rng.random(fl.shape[0]) < 0.5) & (fr >= 0)
        fl_new = np.where(swap, fr, fl)
        fr_new = np.where(swap, fl, fr)
        S = np.where(swap[:, None], -S, S)
        fl, fr = fl_new, fr_new
    A = np.sqrt((S * S).sum(1))
    e = S / A[:, None]
    return _finish(fl, fr, e, A, vol, ctr, bcs)


def merge_meshes(meshes):
    """Disjoint union of meshes (cell and face ids offset, bc tables joined).

    Returns the merged mesh and the cell offset of each input mesh.
    """
    fl, fr, fn, fa, vol, ctr, bcs, offs = [], [], [], [], [], [], [], []
    c0 = 0
    for m in meshes:
        b0 = len(bcs)
        l = m["face_left"].astype(np.int64) + c0
        r = m["face_right"].astype(np.int64)
        r = np.where(r >= 0, r + c0, r - b0)
        fl.append(l); fr.append(r); fn.append(m["face_normal"]); fa.append(m["face_area"])
        vol.append(m["cell_volume"]); ctr.append(m["cell_center"])
        bcs.extend(m["bc"])
        offs.append(c0)
        c0 += m["n_cells"]
    out = _finish(np.concatenate(fl), np.concatenate(fr), np.concatenate(fn),
                  np.concatenate(fa), np.concatenate(vol), np.concatenate(ctr), bcs)
    return out, np.array(offs, dtype=np.int64)


def check_closed(mesh, rel=1e-12):
    """Max over cells of |sum_l sign A e| / sum_l A (0 for closed cells)."""
    nc = mesh["n_cells"]
    fl, fr = mesh["face_left"], mesh["face_right"]
    Se = mesh["face_normal"] * mesh["face_area"][:, None]
    acc = np.zeros((nc, 3))
    asum = np.zeros(nc)
    np.add.at(acc, fl, Se)
    np.add.at(asum, fl, mesh["face_area"])
    m = fr >= 0
    np.add.at(acc, fr[m], -Se[m])
    np.add.at(asum, fr[m], mesh["face_area"][m])
    return float((np.sqrt((acc ** 2).sum(1)) / asum).max())
