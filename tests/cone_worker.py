"""Oracle dependency cones of a few target cells of a named workload, run as
a separate single-thread process so that several can run at once: prints
one JSON line {cell: macros}.  Test infrastructure (calls only the oracle)."""

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--targets", required=True)
    ap.add_argument("--steps", type=int, required=True)
    a = ap.parse_args()
    import synth
    from oracle import fv, tucker_dvm as td
    cfg = synth.make_config(a.workload)
    mesh = synth.configs.make_mesh(cfg)
    m0 = synth.initial_macros(cfg, mesh)
    S = fv.Setup(mesh, cfg, m0)
    targets = [int(x) for x in a.targets.split(",")]
    st = td.run_cone(S, m0, targets, a.steps)
    print(json.dumps({str(t): td.macros_of(S, st[t]).tolist() for t in targets}))


if __name__ == "__main__":
    main()
