"""Named synthetic workloads and their seeded initial macroparameters.

The paper's only workload (flow past a cylinder on a private unstructured
mesh, N = 64) is not reproducible here; these synthetic flows stand in for
it.  Physical units follow the nondimensionalisation R_g = 1/2, m = 1 (so
2 R_g T = T and speeds are in units of sqrt(2 R_g T0)).

Each config is a dict with the mesh builder, velocity grid, physics and run
parameters.  `initial_macros(cfg, mesh)` returns float64[n_cells, 5] rows
(n, u1, u2, u3, T).
"""

import numpy as np

from . import meshes

PHYS = {"Pr": 2.0 / 3.0, "omega": 0.5, "Kn": 0.1, "Rg": 0.5, "m": 1.0}

CONFIGS = {
    # periodic 8^3 box, random Maxwellian per cell, FP64 path
    "cfg0": dict(name="periodic-8^3-N16", mesh=("periodic_box", dict(n=8)),
                 N=16, xi_max=4.5, cap=6, tol=1e-6, cfl=0.5, steps=20,
                 seed=0, init="random", precision="fp64", **PHYS),
    # channel 64x32x32 with an 8^3 obstacle, Mach-2 free stream
    "cfg1": dict(name="channel-64x32x32-obstacle-N32", mesh=("channel_with_obstacle", {}),
                 N=32, xi_max=6.0, cap=12, tol=1e-5, cfl=0.5, steps=200,
                 seed=1, init="freestream", precision="mixed", **PHYS),
    # jittered 80x50x50 box, density bump + temperature jump
    "cfg2": dict(name="jittered-80x50x50-N48",
                 mesh=("jittered_box", dict(nx=80, ny=50, nz=50, h=1.0 / 80, seed=2)),
                 N=48, xi_max=7.0, cap=16, tol=1e-5, cfl=0.5, steps=100,
                 seed=2, init="bump", precision="mixed", **PHYS),
}


def make_mesh(cfg):
    kind, kw = cfg["mesh"]
    return getattr(meshes, kind)(**kw)


def make_config(name, **override):
    cfg = dict(CONFIGS[name])
    cfg.update(override)
    return cfg


def initial_macros(cfg, mesh):
    nc = mesh["n_cells"]
    init = cfg["init"]
    out = np.zeros((nc, 5))
    if init == "random":
        rng = np.random.default_rng(cfg["seed"])
        out[:, 0] = rng.uniform(0.8, 1.2, nc)
        out[:, 1:4] = rng.normal(0.0, 0.1, (nc, 3))
        out[:, 4] = rng.uniform(0.9, 1.1, nc)
    elif init == "freestream":
        bc = mesh["bc"][0]
        out[:, 0] = bc["n"]
        out[:, 1:4] = np.array(bc["u"])[None, :]
        out[:, 4] = bc["T"]
    elif init == "bump":
        c = mesh["cell_center"]
        lo = c.min(0)
        hi = c.max(0)
        xc = 0.5 * (lo + hi)
        r2 = ((c - xc) ** 2).sum(1)
        out[:, 0] = 1.0 + 0.5 * np.exp(-r2 / (2 * 0.1 ** 2))
        out[:, 4] = np.where(c[:, 0] < 0.5, 1.0, 2.0)
    elif init == "uniform":
        out[:, 0] = 1.0
        out[:, 4] = 1.0
    else:
        raise ValueError(init)
    return out


def batch_instances(seed=3, count=256, k_range=(1e3, 3.2e4), Ns=(16, 24, 32),
                    caps=(4, 16)):
    """Instance list for the batched workload: periodic boxes of k^3 cells.

    k^3 is log-uniform in k_range, N uniform over Ns, rank cap uniform in
    the inclusive range `caps`; each instance carries its own init seed.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        c3 = np.exp(rng.uniform(np.log(k_range[0]), np.log(k_range[1])))
        k = int(round(c3 ** (1.0 / 3.0)))
        N = int(rng.choice(Ns))
        cap = int(rng.integers(caps[0], caps[1] + 1))
        out.append(dict(name=f"inst{i}", mesh=("periodic_box", dict(n=k)), N=N,
                        xi_max=4.5, cap=cap, tol=1e-6, cfl=0.5, steps=50,
                        seed=int(rng.integers(1 << 30)), init="random",
                        precision="mixed", **PHYS))
    return out


def serve_requests(seed=4, count=200, cells=(1e3, 1e5), Ns=(16, 24, 32),
                   tols=(1e-4, 1e-5, 1e-6), kn=(0.01, 1.0)):
    """Request list for the served workload (jittered closed boxes)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        c = np.exp(rng.uniform(np.log(cells[0]), np.log(cells[1])))
        k = max(3, int(round(c ** (1.0 / 3.0))))
        N = int(rng.choice(Ns))
        tol = float(rng.choice(tols))
        Kn = float(np.exp(rng.uniform(np.log(kn[0]), np.log(kn[1]))))
        phys = dict(PHYS)
        phys["Kn"] = Kn
        out.append(dict(name=f"req{i}",
                        mesh=("jittered_box", dict(nx=k, ny=k, nz=k, h=1.0 / k,
                                                   seed=int(rng.integers(1 << 30)))),
                        N=N, xi_max=4.5, cap=16, tol=tol, cfl=0.5, steps=500,
                        residual_tol=1e-5, seed=int(rng.integers(1 << 30)),
                        init="random", precision="mixed", **phys))
    return out
