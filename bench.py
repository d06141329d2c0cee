"""Throughput of the Tucker S-model step on one MI355X.

Workload (default): the channel flow with an obstacle -- 64x32x32 lattice
minus an 8^3 obstacle (65,024 hex cells), Mach-2 inflow, zero-gradient
outflow, symmetry sides, diffuse walls at T_w = 1; velocity grid 32^3 on
[-6, 6]^3; rank cap 12, rounding tolerance 1e-5; mixed precision (FP32
N-basis term assembly; FP64 factor-space rounding, Grams, eigensolves,
projection and moments); 200 steps.  A step is one pass of the whole hot
path over every cell: moments, f_S, boundary ghosts, flux terms,
truncated-HOSVD rounding.  Inputs are resident in HBM before the timed
region.  The state advances the workload's 200 steps; the timed region is
the last `--steps` of them (default all, after `--warmup` steps), with no
per-kernel events; `--steps 20` times steps 180-200, where the ranks are
highest.

One JSON line on stdout: metric/value (cell-updates/s over the timed
window); per-kernel times, the roofline of the dominant kernel family and
of every other family (with its HBM rate) from five further steps with every pass on one stream and HIP events around
each launch; the plain full-tensor GPU step on the same workload; the FP64
path timed on the same window and the mixed path's end-of-run macro error
against it, beside the FP64 path's own spread under a 1e-7 input
perturbation; LU-SGS iterations against explicit FP64 steps; the step with
intermediate rounding of each face's flux term against the one-rounding
step (`face_rounding`, a few steps after a short ordinary run); a sampled
parity check against the FP64 oracle and the oracle's own CPU throughput
(`cpu_baseline`, one single-thread process per host core).
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from paper_1912_04582_amd import tk  # noqa: E402

PEAK = {"fp64_mfma": 78.6e12, "fp32_mfma": 157.3e12, "fp32_vec_nopk": 78.6e12, "fp64_vec": 78.6e12,
        "hbm": 8.0e12}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    cfg = synth.make_config(name)
    mesh = synth.configs.make_mesh(cfg)
    return cfg, mesh, synth.initial_macros(cfg, mesh)


def gram_flops(N, cells):
    # symmetric mode Grams: 3 modes x N(N+1)/2 entries x N^2 products x 2
    return cells * 3.0 * N * (N + 1) / 2 * N * N * 2


def expand_flops(N, ranks, nb_ranks):
    """Mode-product flops of the term assembly for cells with the given ranks.

    Per source (the cell, its six far sides) 2 (r1 r2 r3 N + r1 r2 N^2 + r1 N^3),
    plus the rank-4 f_S; boundary sides count as the cell's own ranks.
    """
    def src(r):
        r = np.asarray(r, dtype=np.float64)
        return 2 * (r[..., 0] * r[..., 1] * r[..., 2] * N + r[..., 0] * r[..., 1] * N * N + r[..., 0] * N ** 3)
    return float(src(ranks).sum() + src(nb_ranks).sum() + ranks.shape[0] * src(np.array([4, 4, 4])))


def neighbour_ranks(mesh, ranks):
    fl, fr = mesh["face_left"], mesh["face_right"]
    out = []
    inner = fr >= 0
    out.append(ranks[fr[inner]])      # far side of the left cells
    out.append(ranks[fl[inner]])      # far side of the right cells
    out.append(ranks[fl[~inner]])     # boundary ghosts: the cell's own ranks (upper bound)
    return np.concatenate(out)


def eig_flops(N, matrices, sweeps):
    """The eigensolver's own work: per matrix the warm-start rotation V^T G V
    (4 N^3), per Jacobi sweep N (N - 1) / 2 rotations of 10 N flops each (two
    rows and two columns of the matrix, two columns of the vectors), and the
    sorted basis written out (the counted sweeps come from the library)."""
    return matrices * 4.0 * N ** 3 + sweeps * 5.0 * N * N * (N - 1)


def project_flops(N, ranks):
    r = np.asarray(ranks, dtype=np.float64)
    r1, r2, r3 = r[:, 0], r[:, 1], r[:, 2]
    return float((2 * (r1 * N ** 3 + r1 * r2 * N * N + r1 * r2 * r3 * N)).sum())


FAMILIES = {"rround": "k_rround", "moments": "k_moments", "expand": "k_expand", "gram": "k_gram",
            "eig": "k_eig", "project": "k_project"}
SOURCES = {"rround": "k_rround.hip", "moments": "k_moments.hip", "expand": "k_expand.hip", "gram": "k_gram.hip",
           "eig": "k_eig.hip", "project": "k_project.hip"}


def family_of(kernel_name):
    """Kernel family of a demangled kernel name (k_expand_pipe<...> -> expand)."""
    import re
    m = re.search(r"\b(k_[a-z0-9_]+)\s*[<(]", kernel_name)
    base = m.group(1) if m else kernel_name
    for fam, stem in FAMILIES.items():
        if base == stem or (base.startswith(stem + "_") and base != "k_expand_plain"):
            return fam
    return None


def source_sha(fam):
    import hashlib
    path = os.path.join(ROOT, "paper_1912_04582_amd", "csrc", SOURCES[fam])
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(workload_name, fam):
    """HBM bytes per step of a kernel family in the timed window, from the
    committed counter summary (FETCH_SIZE and WRITE_SIZE runs of the same
    command, copy-calibrated), or None when there is none for this workload
    or the kernel's source has changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload_name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    k = d.get("kernels", {}).get(fam)
    if not k or k.get("sha256") != source_sha(fam):
        return None
    return k["fetch_bytes_per_step"] + k["write_bytes_per_step"]


def window_rows(rows, window, tail=0):
    """Dispatches of the timed window: `window` steps, each opened by a
    factor-space (or, without it, moments) launch, ending `tail` steps before
    the last (the per-kernel steps that follow the timed window); rows sorted
    by start."""
    rows = sorted(rows, key=lambda r: r["start"])
    marks = [r for r in rows if family_of(r["name"]) == "rround"] or \
        [r for r in rows if family_of(r["name"]) == "moments"]
    t0 = marks[-(window + tail)]["start"] if len(marks) >= window + tail else rows[0]["start"]
    t1 = marks[-tail]["start"] if tail and len(marks) >= tail else float("inf")
    return [r for r in rows if t0 <= r["start"] < t1]


def trace_summary(trace_csv, window, bench_json=None, tail=5):
    """Markdown tables of kernel-family times of a rocprofv3 --kernel-trace
    CSV of this script: the timed window (two streams), and the `tail`
    per-kernel steps after it (one stream) beside the HIP-event times of the
    bench line, launch by launch the same kernels."""
    import csv
    rows = []
    with open(trace_csv) as fh:
        for r in csv.DictReader(fh):
            rows.append({"name": r["Kernel_Name"], "start": int(r["Start_Timestamp"]),
                         "end": int(r["End_Timestamp"])})
    def families(win):
        fam = {}
        for r in win:
            f = family_of(r["name"])
            if f:
                t = fam.setdefault(f, [0.0, 0])
                t[0] += (r["end"] - r["start"]) / 1e6
                t[1] += 1
        return fam
    hip, hip_launch = {}, {}
    if bench_json:
        with open(bench_json) as fh:
            b = json.loads(fh.read().strip().splitlines()[-1])
        for f, ms in b.get("kernel_ms_per_step_one_stream", b.get("kernel_ms_per_step", {})).items():
            hip[f] = ms
        roof = b.get("roofline") or {}
        if roof.get("kernel"):
            hip_launch[roof["kernel"]] = roof.get("avg_launch_ms")
    win = window_rows(rows, window, tail)
    out = [f"Timed window (the {window} steps, two streams):", "",
           "| family | launches | total (ms) | per step (ms) | average per launch (ms) |", "|---|---|---|---|---|"]
    for f, (ms, n) in sorted(families(win).items(), key=lambda kv: -kv[1][0]):
        out.append(f"| {f} | {n} | {ms:.2f} | {ms / window:.3f} | {ms / n:.4f} |")
    span = (win[-1]["end"] - win[0]["start"]) / 1e6
    out += ["", f"{len(win)} launches over {span:.1f} ms ({span / window:.2f} ms per step of device time span).", ""]
    if tail:
        pw = window_rows(rows, tail, 0)
        out += [f"Per-kernel window (the {tail} steps after it, one stream) against the bench line's HIP events:", "",
                "| family | launches | per step (ms) | average per launch (ms) | HIP events, per step (ms) | "
                "HIP events, average per launch (ms) |", "|---|---|---|---|---|---|"]
        for f, (ms, n) in sorted(families(pw).items(), key=lambda kv: -kv[1][0]):
            he = f"{hip[f]:.3f}" if f in hip else "-"
            hl = f"{hip_launch[f]:.4f}" if hip_launch.get(f) else "-"
            out.append(f"| {f} | {n} | {ms / tail:.3f} | {ms / n:.4f} | {he} | {hl} |")
    return "\n".join(out)


def counter_rows(csv_path, counter):
    import csv
    rows = []
    with open(csv_path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            rows.append({"name": r["Kernel_Name"], "id": int(r["Dispatch_Id"]), "value": float(r["Counter_Value"])})
    # one value per dispatch (the counter summed over its instances)
    agg = {}
    for r in rows:
        a = agg.setdefault(r["id"], {"name": r["name"], "id": r["id"], "value": 0.0})
        a["value"] += r["value"]
    return sorted(agg.values(), key=lambda r: r["id"])


def traffic_summary(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, window, workload_name, tail=5):
    """Bytes per step of each kernel family in the timed window (the sum over
    its launches there, divided by the window's steps: independent of how the
    step splits its cells into launches): FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) scaled so that the 1 GiB elementwise copy reads and writes
    1 GiB."""
    def calib(path, counter):
        rows = [r for r in counter_rows(path, counter) if "elementwise" in r["name"] or "mul" in r["name"]]
        v = sorted(r["value"] for r in rows)[len(rows) // 2]  # median of the copy launches
        return (1 << 30) / (v * 1024.0)
    fr, fw = calib(copy_fetch_csv, "FETCH_SIZE"), calib(copy_write_csv, "WRITE_SIZE")
    out = {"workload": workload_name, "window_steps": window,
           "note": f"HBM bytes per step in the timed window: FETCH_SIZE x {fr:.3f} + WRITE_SIZE x {fw:.3f} "
                   "(KiB per dispatch, scaled so the 1 GiB copy kernel reads and writes 1 GiB); valid while "
                   "the kernel source is unchanged",
           "fetch_scale": fr, "write_scale": fw, "kernels": {}}
    for counter, scale, key in (("FETCH_SIZE", fr, "fetch_bytes_per_step"), ("WRITE_SIZE", fw, "write_bytes_per_step")):
        rows = counter_rows(fetch_csv if counter == "FETCH_SIZE" else write_csv, counter)
        marks = [r for r in rows if family_of(r["name"]) == "rround"] or \
            [r for r in rows if family_of(r["name"]) == "moments"]
        i0 = marks[-(window + tail)]["id"] if len(marks) >= window + tail else rows[0]["id"]
        i1 = marks[-tail]["id"] if tail and len(marks) >= tail else float("inf")
        fam = {}
        for r in rows:
            f = family_of(r["name"])
            if f and i0 <= r["id"] < i1:
                t = fam.setdefault(f, [0.0, 0, set()])
                t[0] += r["value"] * 1024.0 * scale
                t[1] += 1
                t[2].add(r["name"].replace("void tk::(anonymous namespace)::", "").split("(")[0])
        for f, (b, n, names) in fam.items():
            k = out["kernels"].setdefault(f, {"kernels": sorted(names),
                                              "source": f"paper_1912_04582_amd/csrc/{SOURCES[f]}",
                                              "sha256": source_sha(f), "launches": n})
            k[key] = b / window
    return out


def roofline(fam, cfg, mesh, res, steps):
    """Achieved rate of one kernel family against its bound, per launch.

    rround: the FP64 operations the factor-space kernels count for the cells
    they round (Gram-Schmidt, core assembly, Grams, Jacobi, rotations,
    outputs; 2 per multiply-add), FP64 vector peak.  N-basis families: the
    per-cell models above times the cells that took that path in the window."""
    N, nc = cfg["N"], mesh["n_cells"]
    ms, launches = res["prof"][fam]
    if not launches:
        return None
    per_launch_s = ms / 1e3 / launches
    launches_per_step = launches / steps
    rp = res.get("prof_paths") or {}
    nb = rp.get("nbasis", nc * steps) / steps  # N-basis cells per step
    r_avg = 0.5 * (res["ranks0"].astype(np.float64) + res["ranks1"].astype(np.float64))
    frac_nb = nb / nc
    if fam == "rround":
        work, bound, peak, unit = rp.get("flops", 0) / steps, "alu", PEAK["fp64_vec"], "TFLOP/s"
    elif fam == "gram":
        work, bound, peak, unit = gram_flops(N, nb), "mfma", PEAK["fp64_mfma"], "TFLOP/s"
    elif fam == "eig":
        ek = res.get("eig_stats") or {}
        mats = ek.get("full", 3 * nb * steps) / steps
        work, bound, peak, unit = eig_flops(N, mats, ek.get("sweeps", 0) / steps), "alu", PEAK["fp64_vec"], "TFLOP/s"
    elif fam == "expand":
        work = frac_nb * expand_flops(N, r_avg, neighbour_ranks(mesh, r_avg))
        bound, peak, unit = "alu", PEAK["fp32_vec_nopk"], "TFLOP/s"
    elif fam == "project":
        work, bound, peak, unit = frac_nb * project_flops(N, r_avg), "alu", PEAK["fp64_vec"], "TFLOP/s"
    else:
        return None
    achieved = work / launches_per_step / per_launch_s / 1e12
    per_step = measured_traffic(cfg["name"], fam)
    traffic = per_step / launches_per_step if per_step is not None else None
    return {"bound": bound, "achieved": achieved, "peak": peak / 1e12, "unit": unit,
            "frac": achieved / (peak / 1e12), "traffic": traffic, "kernel": fam,
            "avg_launch_ms": per_launch_s * 1e3, "launches_per_step": launches_per_step,
            "work_per_launch": work / launches_per_step}


def has_oblique_faces(mesh):
    e = np.abs(np.asarray(mesh["face_normal"]))
    return bool(((e > 1e-12).sum(1) > 1).any())


def sample_targets(mesh, count=12, seed=0):
    """Cells next to each boundary kind plus random interior cells."""
    fr, fl = mesh["face_right"], mesh["face_left"]
    picks = []
    for b in range(len(mesh["bc"])):
        cand = fl[fr == -(b + 1)]
        if cand.shape[0]:
            picks.append(int(cand[cand.shape[0] // 2]))
    rng = np.random.default_rng(seed)
    while len(picks) < count:
        picks.append(int(rng.integers(mesh["n_cells"])))
    return sorted(set(picks))[:count]


def cpu_leg(name, targets, steps):
    """Oracle (O2) dependency cones of `targets` advanced `steps` steps; prints JSON."""
    from oracle import fv, tucker_dvm as td
    cfg, mesh, m0 = workload(name)
    S = fv.Setup(mesh, cfg, m0)  # mesh tables and dt: set-up, not timed (as on the GPU)
    t0 = time.perf_counter()
    levels = td.cone(S, targets, steps)
    st = td.run_cone(S, m0, targets, steps)
    t1 = time.perf_counter()
    updates = sum(len(l) for l in levels[1:])
    macros = {int(i): td.macros_of(S, st[i]).tolist() for i in targets}
    print(json.dumps({"seconds": t1 - t0, "updates": updates, "macros": macros,
                      "levels": [len(l) for l in levels]}))


def run_cpu_leg(name, targets, steps, workers):
    """The oracle's cones of `targets`, split round-robin over `workers`
    processes run at the same time (one thread each)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    groups = [targets[i::workers] for i in range(workers)]
    groups = [g for g in groups if g]
    procs = []
    for g in groups:
        cmd = [sys.executable, os.path.abspath(__file__), "--cpu-leg", "--workload", name,
               "--targets", ",".join(map(str, g)), "--leg-steps", str(steps)]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env))
    out = {"seconds": 0.0, "updates": 0, "macros": {}, "workers": len(procs)}
    for pr in procs:
        so, se = pr.communicate(timeout=900)
        if pr.returncode != 0:
            raise RuntimeError(se[-2000:])
        r = json.loads(so.strip().splitlines()[-1])
        out["seconds"] = max(out["seconds"], r["seconds"])
        out["updates"] += r["updates"]
        out["macros"].update(r["macros"])
    return out


def host_cores():
    """CPU threads this process may use, at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def advance(st, steps, label):
    """st.step(steps) in calls of at most 10 steps, with a progress line at
    most every 30 s (long untimed runs)."""
    done, t_last = 0, time.perf_counter()
    while done < steps:
        k = min(10, steps - done)
        st.step(k)
        done += k
        if time.perf_counter() - t_last > 30 and done < steps:
            log(f"    {label}: {done}/{steps} steps")
            t_last = time.perf_counter()


def gpu_macros_after(cfg, mesh, m0, steps):
    ctx = tk.Context(0)
    try:
        tm = tk.Mesh(ctx, mesh)
        st = tk.State(ctx, tm, cfg, m0)
        advance(st, steps, f"{cfg['precision']} run")
        out = st.moments()
        st.close()
        tm.close()
    finally:
        ctx.close()
    return out


def macro_rel_err(a, b, Rg=0.5, m=1.0):
    a, b = np.asarray(a), np.asarray(b)
    n, T = b[:, 0], b[:, 4]
    c = np.sqrt(2 * Rg * T)
    p = m * n * Rg * T
    e = max(np.abs(a[:, 0] / n - 1).max(), np.abs(a[:, 4] / T - 1).max(),
            (np.abs(a[:, 1:4] - b[:, 1:4]).max(1) / c).max(),
            (np.abs(a[:, 5:8] - b[:, 5:8]).max(1) / (p * c)).max())
    return float(e)


def run_gpu(cfg, mesh, m0, total, window, warmup, plain=False, prof=True, one_stream=False, tune=True,
            prof_steps=5):
    """Advance a state `total` steps from the initial fields and time the
    last `window` of them (after at least `warmup` untimed steps on the same
    state), with no per-kernel events in the timed region.  Pass-size trials
    run first on a throw-away state.  With `prof`, `prof_steps` further steps
    follow with every rounding pass on the context stream and HIP events
    around every launch: the per-kernel times, rounding-path counts,
    eigensolver counters and ranks of that window feed the roofline (one
    kernel at a time, so no launch shares the device with another pass)."""
    window = min(window, total)
    pre = max(warmup, total - window)
    ctx = tk.Context(0)
    try:
        tm = tk.Mesh(ctx, mesh)
        if tune and not plain:
            # untimed: the pass-size trial steps (the choice is kept on the
            # context for the timed state of the same shape)
            w = tk.State(ctx, tm, cfg, m0)
            if one_stream:
                w.streams(False)
            trials = w.tune()
            log(f"  rounding pass: {w.chunk()[0]} cells (of {w.chunk()[1]}), chosen over {trials} steps")
            w.close()
        st = tk.State(ctx, tm, cfg, m0, plain=plain)
        two = None
        if not plain:
            if one_stream:
                st.streams(False)
                two = False
            else:
                two = st.streams(None)  # the second stream is used when it exists
        if pre:
            advance(st, pre, "untimed steps")
        ctx.sync()
        ctx.prof_enable(False)
        if not plain:
            st.rounding()
        t0 = time.perf_counter()
        st.step(window)  # waits for completion
        t1 = time.perf_counter()
        rcount = None
        if not plain:
            rcount = st.rounding()
            log(f"  rounding paths over the window (cell-updates): {rcount}")
        rmain, C = (None, None) if plain else st.ranks()
        final = st.moments()
        prof_ms, eig, pcount, r0, r1, pw = {}, None, None, None, None, 0
        if prof:
            pw = prof_steps
            if not plain:
                st.streams(False)
                st.rounding()
                r0 = st.ranks()[0]
            ctx.eig_stats(reset=True)
            ctx.prof_reset()
            ctx.prof_enable(True)
            st.step(pw)
            ctx.prof_enable(False)
            fams = ["moments", "rround", "expand", "gram", "eig", "project"] if not plain else \
                ["plain_moments", "plain_step"]
            prof_ms = {f: ctx.prof_get(f) for f in fams}
            eig = ctx.eig_stats(reset=True)
            if not plain:
                pcount = st.rounding()
                r1 = st.ranks()[0]
                log(f"  per-kernel window ({pw} steps, one stream): eigensolver {eig}, rounding paths {pcount}")
        st.close()
        tm.close()
    finally:
        ctx.close()
    return dict(seconds=t1 - t0, prof=prof_ms, prof_steps=pw, ranks0=r0, ranks1=r1, ranks_end=rmain,
                compression=C, rounding_paths=rcount, prof_paths=pcount, final=final, pre=pre, window=window,
                two_streams=two, eig_stats=eig)


def run_batch(steps, warmup, count, prof_steps=3):
    """The batched workload: independent periodic boxes grouped by N into
    one state per N; every state advances `steps` steps."""
    insts = synth.configs.batch_instances(count=count)
    groups = {}
    for c in insts:
        m = synth.configs.make_mesh(c)
        groups.setdefault(c["N"], []).append((c, m, synth.initial_macros(c, m)))
    ctx = tk.Context(0)
    try:
        states, meshes = [], []
        for N, items in sorted(groups.items()):
            ms = [tk.Mesh(ctx, m) for _, m, _ in items]
            meshes += ms
            # untimed: pass-size trials on a throw-away state of the group
            # (kept on the context for the timed state of the same shape)
            w = tk.State(ctx, ms, [c for c, _, _ in items], [m0 for _, _, m0 in items])
            w.tune()
            if warmup:
                w.step(warmup)
            w.close()
            st = tk.State(ctx, ms, [c for c, _, _ in items], [m0 for _, _, m0 in items])
            st.use_graph(True)
            states.append(st)
        cells = sum(s.n_cells for s in states)
        ctx.sync()
        t0 = time.perf_counter()
        for st in states:
            st.step_async(steps)
        ctx.sync()
        t1 = time.perf_counter()
        # kernel-family times from a few further eager steps with HIP events
        ctx.prof_reset()
        ctx.prof_enable(True)
        for st in states:
            st.step_async(prof_steps)
        ctx.sync()
        ctx.prof_enable(False)
        prof = {f: ctx.prof_get(f) for f in ["moments", "expand", "gram", "eig", "project"]}
        chunks = {st.n_cells: st.chunk()[0] for st in states}
        for st in states:
            st.close()
        for m in meshes:
            m.close()
    finally:
        ctx.close()
    return dict(seconds=t1 - t0, cells=cells, prof=prof, prof_steps=prof_steps, chunks=chunks,
                groups={N: (len(v), sum(m["n_cells"] for _, m, _ in v)) for N, v in groups.items()})


def run_lusgs(cfg, mesh, m0, iters, cfl):
    """LU-SGS iterations (CFL `cfl`) against explicit steps (the workload's
    CFL) from the same initial state, FP64 and mixed: time per iteration,
    the kernel families of one more iteration, and the residual per
    iteration."""
    c64 = dict(cfg, precision="fp64")
    cmx = dict(cfg, precision="mixed")
    out = {}
    ctx = tk.Context(0)
    try:
        tm = tk.Mesh(ctx, mesh)
        for kind, c in (("lusgs", dict(c64, cfl=cfl)), ("explicit", c64), ("lusgs_mixed", dict(cmx, cfl=cfl)),
                        ("explicit_mixed", cmx)):
            st = tk.State(ctx, tm, c, m0)
            st.streams(False)
            go = st.lusgs if kind.startswith("lusgs") else st.step
            go(1)  # untimed: set-up (colouring, buffers) and first rounding
            res = []
            t0 = time.perf_counter()
            for _ in range(iters):
                res.append(float(go(1, residual=True)[0]))
            t1 = time.perf_counter()
            ctx.prof_reset()
            ctx.prof_enable(True)
            go(1)
            ctx.prof_enable(False)
            fams = ["moments", "lusgs", "expand", "gram", "eig", "project", "rround"]
            out[kind] = {"ms_per_iteration": 1e3 * (t1 - t0) / iters, "iterations": iters, "cfl": c["cfl"],
                         "residual_per_iteration": res,
                         "kernel_ms_one_iteration": {f: ctx.prof_get(f)[0] for f in fams if ctx.prof_get(f)[1]}}
            log(f"{kind}: {out[kind]['ms_per_iteration']:.2f} ms per iteration at CFL {c['cfl']}, "
                f"residuals {['%.2e' % r for r in res]}")
            st.close()
        tm.close()
    finally:
        ctx.close()
    out["cost_ratio"] = out["lusgs"]["ms_per_iteration"] / out["explicit"]["ms_per_iteration"]
    out["cost_ratio_mixed"] = out["lusgs_mixed"]["ms_per_iteration"] / out["explicit_mixed"]["ms_per_iteration"]
    return out


def run_faces(cfg, mesh, m0, pre, steps):
    """The intermediate-rounding step (each face's flux term rounded before
    the sum) against the one-rounding step: two states advanced `pre`
    ordinary steps, then `steps` timed steps each way; time per step, the
    kernel families of one more step and the macro difference between the
    two results."""
    ctx = tk.Context(0)
    out = {"pre_steps": pre, "steps": steps}
    try:
        tm = tk.Mesh(ctx, mesh)
        finals = {}
        for kind in ("one_rounding", "face_rounding"):
            st = tk.State(ctx, tm, cfg, m0)
            st.step(pre)
            ctx.sync()
            if kind == "face_rounding":
                st.face_rounding(True)
            t0 = time.perf_counter()
            st.step(steps)
            ctx.sync()
            t1 = time.perf_counter()
            finals[kind] = st.moments()
            ctx.prof_reset()
            ctx.prof_enable(True)
            st.step(1)
            ctx.prof_enable(False)
            fams = ["moments", "expand", "gram", "eig", "project", "rround"]
            out[kind] = {"ms_per_step": 1e3 * (t1 - t0) / steps,
                         "kernel_ms_one_step": {f: ctx.prof_get(f)[0] for f in fams if ctx.prof_get(f)[1]}}
            log(f"{kind}: {out[kind]['ms_per_step']:.2f} ms/step over steps {pre}..{pre + steps}")
            st.close()
        tm.close()
    finally:
        ctx.close()
    out["cost_ratio"] = out["face_rounding"]["ms_per_step"] / out["one_rounding"]["ms_per_step"]
    out["max_rel_macro_diff"] = macro_rel_err(finals["face_rounding"], finals["one_rounding"])
    log(f"face rounding / one rounding: {out['cost_ratio']:.2f}x per step, macro difference "
        f"{out['max_rel_macro_diff']:.3e} after {steps} steps (tol {cfg['tol']})")
    return out


def serve_run(reqs, rate, seed=5):
    """Submit requests (arrivals at t = 0 when rate is None, else Poisson with
    `rate` per second), wait for all; latency = t_done - t_arrive."""
    ctx = tk.Context(0)
    srv = tk.Server(ctx)
    rng = np.random.default_rng(seed)
    t_next = 0.0
    tickets = []
    t0 = time.perf_counter()
    for m, c, m0, steps, rtol in reqs:
        if rate:
            t_next += rng.exponential(1.0 / rate)
            while time.perf_counter() - t0 < t_next:
                time.sleep(0.001)
        tickets.append(srv.submit(m, c, m0, steps, rtol))
        log(f"    submitted request {len(tickets) - 1} at {time.perf_counter() - t0:.2f} s")
    done = {}
    while len(done) < len(tickets):
        for i, t in enumerate(tickets):
            if t not in done:
                r = srv.poll(t, want_macros=False)
                if r["status"] != tk.TK_PENDING:
                    done[t] = r
                    log(f"    request {i}: {reqs[i][0]['n_cells']} cells, {r['steps']} steps, "
                        f"latency {r['t_done'] - r['t_arrive']:.2f} s ({len(done)}/{len(tickets)} done)")
        time.sleep(0.002)
    t1 = time.perf_counter()
    stats = srv.stats()
    srv.close()
    ctx.close()
    res = [done[t] for t in tickets]
    lat = np.array([r["t_done"] - r["t_arrive"] for r in res])
    updates = sum(r["steps"] * q[0]["n_cells"] for r, q in zip(res, reqs))
    return dict(seconds=t1 - t0, latency=lat, updates=updates, stats=stats,
                status=[r["status"] for r in res], steps=[r["steps"] for r in res])


def run_serve(count, max_steps, seed=4, rate=None):
    specs = synth.configs.serve_requests(seed=seed, count=count)
    reqs = []
    for c in specs:
        m = synth.configs.make_mesh(c)
        reqs.append((m, c, synth.initial_macros(c, m), min(max_steps, c["steps"]), c["residual_tol"]))
    if rate:
        log(f"serving {count} requests: Poisson at {rate} per second")
        return dict(paced=serve_run(reqs, rate), rate=rate, cells=[q[0]["n_cells"] for q in reqs])
    log(f"serving {count} requests: saturated, then Poisson at 0.7x and 0.35x the saturated rate")
    sat = serve_run(reqs, None)
    rate = 0.7 * count / sat["seconds"]
    paced = serve_run(reqs, rate)
    half = serve_run(reqs, 0.5 * rate, seed=6)
    return dict(saturated=sat, paced=paced, paced_half=half, rate=rate, cells=[q[0]["n_cells"] for q in reqs])


def table1_oblique_workload():
    """The jittered-box recipe (density bump, temperature jump, N = 48 on
    [-7, 7]) on a 40x25x25 box: faces off the coordinate axes, where the
    Tucker step uses the rank-6 |xi_n| estimate and the standard DVM the
    exact |xi_n|."""
    cfg = dict(synth.make_config("cfg2"), name="jittered-40x25x25-N48",
               mesh=("jittered_box", dict(nx=40, ny=25, nz=25, h=1.0 / 40, seed=2)))
    mesh = synth.configs.make_mesh(cfg)
    return cfg, mesh, synth.initial_macros(cfg, mesh)


def run_table1(steps, eps_list=(1e-3, 1e-4, 1e-5), oblique=False):
    """The paper's Table 1 on a synthetic flow: mean compression ratio
    C = mean over cells of (r1 r2 r3 + N (r1 + r2 + r3)) / N^3 and the
    relative 2-norm difference of the temperature field from the standard
    (full-tensor) DVM after the same number of steps, for several rounding
    tolerances.  The channel's faces are axis-aligned (both steps use the
    exact |xi_n|); on the jittered box the Tucker step uses the estimate."""
    cfg, mesh, m0 = table1_oblique_workload() if oblique else workload("cfg1")
    ctx = tk.Context(0)
    rows = []
    try:
        tm = tk.Mesh(ctx, mesh)
        p = tk.State(ctx, tm, cfg, m0, plain=True)
        t0 = time.perf_counter()
        p.step(steps)
        tp = time.perf_counter() - t0
        Tp = p.moments()[:, 4]
        p.close()
        log(f"table1: standard DVM {steps} steps, {1e3 * tp / steps:.2f} ms/step")
        for eps in eps_list:
            st = tk.State(ctx, tm, dict(cfg, tol=eps), m0)
            st.tune()
            st.close()
            st = tk.State(ctx, tm, dict(cfg, tol=eps), m0)
            t0 = time.perf_counter()
            st.step(steps)
            tt = time.perf_counter() - t0
            T = st.moments()[:, 4]
            _, C = st.ranks()
            st.close()
            dT = float(np.linalg.norm(T - Tp) / np.linalg.norm(Tp))
            rows.append({"eps": eps, "mean_C": C, "dT_rel_2norm": dT, "ms_per_step": 1e3 * tt / steps})
            log(f"table1: eps {eps:g}: C {C:.4g}, dT {dT:.3e}, {1e3 * tt / steps:.2f} ms/step")
        tm.close()
    finally:
        ctx.close()
    return {"standard_ms_per_step": 1e3 * tp / steps, "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's own step count)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg1")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--one-stream", action="store_true",
                    help="run every rounding pass on one stream (per-kernel times without the concurrent pass)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=50)
    ap.add_argument("--parity-steps", type=int, default=None,
                    help="oracle cone depth (default 6 on the channel, 2 on the jittered box)")
    ap.add_argument("--parity-cells", type=int, default=None)
    ap.add_argument("--no-fp64-check", action="store_true",
                    help="skip the FP64 GPU run used for the end-of-run mixed-precision error")
    ap.add_argument("--no-lusgs", action="store_true", help="skip the LU-SGS iteration timing")
    ap.add_argument("--no-faces", action="store_true", help="skip the intermediate-rounding step timing")
    ap.add_argument("--faces-pre", type=int, default=20)
    ap.add_argument("--faces-steps", type=int, default=3)
    ap.add_argument("--lusgs-iters", type=int, default=4)
    ap.add_argument("--lusgs-cfl", type=float, default=4.0)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--serve-count", type=int, default=12)
    ap.add_argument("--serve-max-steps", type=int, default=100)
    ap.add_argument("--serve-rate", type=float, default=None,
                    help="only the Poisson run, at this many requests per second")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a 1 GiB read + 1 GiB write elementwise copy, five times (the "
                         "reference kernel for scaling HBM byte counters)")
    ap.add_argument("--trace-summary", nargs="+", metavar=("KERNEL_TRACE_CSV", "BENCH_JSON"),
                    help="print the timed window's kernel-family times of a rocprofv3 kernel trace of this "
                         "script (and the bench line's HIP-event times) as markdown, then exit")
    ap.add_argument("--traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write profiles/traffic_<workload>.json from FETCH_SIZE / WRITE_SIZE counter runs of "
                         "this script and of --calibrate-copy, then exit")
    ap.add_argument("--cpu-leg", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--targets", default="", help=argparse.SUPPRESS)
    ap.add_argument("--leg-steps", type=int, default=2, help=argparse.SUPPRESS)
    a = ap.parse_args()
    if a.cpu_leg:
        cpu_leg(a.workload, [int(x) for x in a.targets.split(",")], a.leg_steps)
        return
    if a.trace_summary:
        print(trace_summary(a.trace_summary[0], a.steps or 20, a.trace_summary[1] if len(a.trace_summary) > 1 else None))
        return
    if a.traffic:
        name = synth.make_config(a.workload)["name"]
        out = traffic_summary(*a.traffic, a.steps or 20, name)
        with open(os.path.join(ROOT, "profiles", f"traffic_{name}.json"), "w") as fh:
            json.dump(out, fh, indent=1)
        print(json.dumps(out, indent=1))
        return
    if a.calibrate_copy:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4, "launches": 5}))
        return
    if a.gpus != 1:
        print(json.dumps({"error": "one GPU per process: the step runs on a single device; --gpus must be 1"}))
        sys.exit(2)
    if a.workload == "serve":
        r = run_serve(a.serve_count, a.serve_max_steps, rate=a.serve_rate)
        out = {"metric": "served Tucker S-model cell-updates/s; p50/p99 request latency",
               "unit": "cell-updates/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "f32 terms + f64 rounding", "data": "synthetic",
               "config": {"workload": f"serving {a.serve_count} jittered-box requests",
                          "max_steps": a.serve_max_steps, "cells": r["cells"]}}
        for key in [k for k in ("saturated", "paced", "paced_half") if k in r]:
            q = r[key]
            out[key] = {"value": q["updates"] / q["seconds"], "seconds": q["seconds"],
                        "p50_latency_s": float(np.percentile(q["latency"], 50)),
                        "p99_latency_s": float(np.percentile(q["latency"], 99)),
                        "statuses": sorted(set(q["status"])), "steps": q["steps"],
                        "shared_launches": q["stats"]}
            log(f"serve {key}: {out[key]['value']:.4g} cell-updates/s, p50 {out[key]['p50_latency_s']:.2f} s, "
                f"p99 {out[key]['p99_latency_s']:.2f} s over {q['seconds']:.1f} s")
        out["arrival_rate_per_s"] = r["rate"]
        if "paced_half" in r:
            out["arrival_rate_half_per_s"] = 0.5 * r["rate"]
        out["value"] = out["paced"]["value"]
        print(json.dumps(out), flush=True)
        return
    if a.workload in ("table1", "table1-oblique"):
        oblique = a.workload == "table1-oblique"
        steps = a.steps or (50 if oblique else 200)
        r = run_table1(steps, oblique=oblique)
        cfg_t = table1_oblique_workload()[0] if oblique else synth.make_config("cfg1")
        print(json.dumps({
            "metric": "mean compression ratio and temperature difference vs the standard DVM (Table 1 style)",
            "unit": "ratio", "n_gpus": 1, "steps": steps, "data": "synthetic",
            "config": {"workload": cfg_t["name"], "precision": "mixed", "cap": cfg_t["cap"],
                       "faces": "oblique (rank-6 estimate in the Tucker step)" if oblique else "axis-aligned"},
            "standard_dvm_ms_per_step": r["standard_ms_per_step"], "rows": r["rows"]}), flush=True)
        return
    if a.workload == "batch":
        steps = a.steps or 50
        r = run_batch(steps, a.warmup, a.batch_count)
        value = r["cells"] * steps / r["seconds"]
        log(f"batch: {r['cells']} cells in {a.batch_count} instances {r['groups']}, "
            f"{1e3 * r['seconds'] / steps:.2f} ms/step, {value:.4g} cell-updates/s")
        for f, (ms, n) in r["prof"].items():
            log(f"  {f:10s} {ms:10.2f} ms total over {n} launches ({r['prof_steps']} eager profiled steps)")
        print(json.dumps({
            "metric": "batched Tucker S-model cell-updates/s", "value": value,
            "unit": "cell-updates/s", "n_gpus": 1, "steps": steps, "warmup": a.warmup,
            "ms_per_step": 1e3 * r["seconds"] / steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32 terms + f64 rounding", "data": "synthetic",
            "config": {"workload": f"batch of {a.batch_count} periodic boxes", "cells": r["cells"],
                       "groups_by_N": {str(k): v for k, v in r["groups"].items()}},
            "graph_replay": True, "rounding_pass_cells": {str(k): v for k, v in r["chunks"].items()},
            "kernel_ms_per_step_eager": {f: ms / r["prof_steps"] for f, (ms, n) in r["prof"].items()}}),
            flush=True)
        return
    cfg, mesh, m0 = workload(a.workload)
    nc = mesh["n_cells"]
    N = cfg["N"]
    oblique = has_oblique_faces(mesh)
    total = int(cfg["steps"])
    window = min(a.steps or total, total)
    if a.parity_steps is None:
        a.parity_steps = 2 if oblique else 6
    if a.parity_cells is None:
        a.parity_cells = 4 if oblique else 48
    log(f"workload {cfg['name']}: {nc} cells, N={N}, cap {cfg['cap']}, tol {cfg['tol']}, {cfg['precision']}; "
        f"{total} steps, the last {window} timed")
    res = run_gpu(cfg, mesh, m0, total, window, a.warmup, one_stream=a.one_stream)
    ms_step = 1e3 * res["seconds"] / window
    value = nc * window / res["seconds"]
    log(f"tucker: {ms_step:.2f} ms/step over steps {res['pre']}..{res['pre'] + window}, {value:.4g} cell-updates/s, "
        f"mean compression {res['compression']:.4g}")
    for f, (ms, n) in res["prof"].items():
        log(f"  {f:10s} {ms / res['prof_steps']:8.3f} ms/step over {n} launches (one stream, events)")
    r1 = res["ranks_end"]
    rmax = r1.max(1)
    log("  final max-rank histogram:", np.bincount(rmax, minlength=cfg["cap"] + 1).tolist())
    log(f"  mean rank {r1.mean():.2f}")
    fam, (fms, fn) = max(res["prof"].items(), key=lambda kv: kv[1][0])
    roof = roofline(fam, cfg, mesh, res, res["prof_steps"])
    log(f"  roofline ({fam}): {roof}")
    # every family against its own bound, with the HBM rate its counted
    # bytes (copy-calibrated counters, null once its source changed) give
    kernel_roofs = {}
    for f in res["prof"]:
        r = roofline(f, cfg, mesh, res, res["prof_steps"])
        if r is None:
            continue
        if r["traffic"] is not None:
            r["hbm_gbps"] = r["traffic"] / (r["avg_launch_ms"] / 1e3) / 1e9
            r["hbm_frac"] = r["hbm_gbps"] * 1e9 / PEAK["hbm"]
        kernel_roofs[f] = r
        log(f"  {f:10s} {r['achieved']:.3g} {r['unit']} ({r['frac']:.3f} of {r['peak']:.4g}, {r['bound']})"
            + (f", HBM {r['hbm_gbps']:.0f} GB/s ({r['hbm_frac']:.3f})" if "hbm_gbps" in r else ""))
    plain = None
    if not a.no_plain:
        pres = run_gpu(cfg, mesh, m0, a.plain_steps, a.plain_steps, 1, plain=True)
        pv = nc * a.plain_steps / pres["seconds"]
        plain = {"value": pv, "unit": "cell-updates/s", "ms_per_step": 1e3 * pres["seconds"] / a.plain_steps,
                 "steps": a.plain_steps, "storage": "N^3 values per cell",
                 "kernel_ms_per_step": {f: ms / pres["prof_steps"] for f, (ms, n) in pres["prof"].items()}}
        log(f"plain: {plain['ms_per_step']:.2f} ms/step, {pv:.4g} cell-updates/s")
    cpu = parity = None
    if not a.no_cpu:
        targets = sample_targets(mesh, a.parity_cells)
        workers = host_cores()
        leg = run_cpu_leg(a.workload, targets, a.parity_steps, workers)
        cpu = {"value": leg["updates"] / leg["seconds"], "unit": "cell-updates/s", "cores": leg["workers"],
               "kind": "oracle",
               "sample": f"Tucker-form oracle, dependency cones of {len(targets)} cells advanced "
                         f"{a.parity_steps} steps from the initial state, split over {leg['workers']} "
                         f"single-thread processes ({leg['updates']} cell-updates, {leg['seconds']:.1f} s "
                         f"for the slowest process)"}
        g = gpu_macros_after(cfg, mesh, m0, a.parity_steps)
        ref = np.array([leg["macros"][str(t)] for t in targets])
        err = macro_rel_err(g[targets], ref)
        bar = 1e-5 if cfg["precision"] == "mixed" else 1e-10
        parity = {"max_rel_err": err, "bar": bar, "pass": bool(err <= bar), "cells": targets,
                  "steps": a.parity_steps}
        log(f"cpu oracle: {cpu['value']:.4g} cell-updates/s on {leg['workers']} processes; "
            f"parity after {a.parity_steps} steps: {err:.3e}")
    end = fp64 = None
    if cfg["precision"] == "mixed" and not a.no_fp64_check:
        # The FP64 path on the same window (timed), the mixed path against it
        # at the end of the run, and the FP64 path's own spread when its
        # inputs move by 1e-7 relative (the oracle's noise floor under an
        # FP32-sized perturbation)
        c64 = dict(cfg, precision="fp64")
        # (no pass-size trials at N = 48, where an FP64 step takes seconds)
        r64 = run_gpu(c64, mesh, m0, total, window, a.warmup, prof=False, one_stream=a.one_stream, tune=N <= 32)
        fp64 = {"value": nc * window / r64["seconds"], "unit": "cell-updates/s",
                "ms_per_step": 1e3 * r64["seconds"] / window, "steps": window}
        log(f"fp64 path: {fp64['ms_per_step']:.2f} ms/step, {fp64['value']:.4g} cell-updates/s")
        rng = np.random.default_rng(7)
        mp = m0.copy()
        mp[:, 0] *= 1.0 + 1e-7 * rng.standard_normal(nc)
        mp[:, 1:4] += 1e-7 * np.sqrt(mp[:, 4:5]) * rng.standard_normal((nc, 3))
        mp[:, 4] *= 1.0 + 1e-7 * rng.standard_normal(nc)
        # as many steps as the timed runs took (their warm-up steps come on
        # top of the run when the whole run is timed)
        ran = r64["pre"] + r64["window"]
        assert ran == res["pre"] + res["window"]
        g64p = gpu_macros_after(c64, mesh, mp, ran)
        e_end = macro_rel_err(res["final"], r64["final"])
        floor = macro_rel_err(g64p, r64["final"])
        end = {"steps": ran, "max_rel_err_mixed_vs_fp64": e_end,
               "fp64_input_perturbation_1e-7_spread": floor, "bar": 1e-5, "within_bar": bool(e_end <= 1e-5)}
        log(f"end of run: mixed vs FP64 path after {ran} steps: {e_end:.3e} "
            f"(FP64 with inputs perturbed by 1e-7: {floor:.3e})")
    lu = None
    if not a.no_lusgs and N <= 32 and not oblique:
        lu = run_lusgs(cfg, mesh, m0, a.lusgs_iters, a.lusgs_cfl)
    faces = None
    if not a.no_faces:
        faces = run_faces(cfg, mesh, m0, a.faces_pre, a.faces_steps)
    out = {
        "metric": "Tucker S-model cell-updates/s vs plain GPU step; macro error vs the FP64 path stated",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": window, "warmup": res["pre"],
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 factor-space rounding, f32 N-basis terms" if cfg["precision"] == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "cells": nc, "N": N, "rank_cap": cfg["cap"], "tol": cfg["tol"],
                   "precision": cfg["precision"], "run_steps": res["pre"] + window,
                   "timed_window": [res["pre"], res["pre"] + window],
                   "rounding_streams": 2 if res["two_streams"] else 1},
        "dominant_kernel": fam,
        "kernel_ms_per_step_one_stream": {f: ms / res["prof_steps"] for f, (ms, n) in res["prof"].items()},
        "per_kernel_window": {"steps": res["prof_steps"], "after_step": res["pre"] + window,
                              "how": "every rounding pass on one stream, HIP events around each launch"},
        "rounding_paths_per_step": {k: v / window for k, v in (res["rounding_paths"] or {}).items()},
        "mean_compression": res["compression"],
        "roofline": roof,
        "kernel_rooflines": kernel_roofs,
        "plain_gpu": plain,
        "fp64_path": fp64,
        "cpu_baseline": cpu,
        "parity": parity,
        "end_of_run": end,
        "lusgs": lu,
        "face_rounding": faces,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
