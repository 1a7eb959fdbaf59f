"""Writes pair_counts.json: exact (sample, voxel) pair counts of the named
synthetic workloads, computed by the FP64 oracle's scatter loop only.

U counts every pair of a disk sample and a voxel within the blob radius over
the full box; U_half counts those whose voxel has x >= 0 (the half box the
GPU kernels accumulate).  The benchmark divides these counts by its measured
times to report updates per second.

Run:  python tests/golden/pair_counts.py [name ...]   (default: small paper precision)
Entries for names not given are kept.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pair_counts.json")


def main(names=("small", "paper", "precision")):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        w = synth.make_workload(name)
        _, _, U, Uh = oracle.insert(w.n, w.slices, w.quats, with_half=True,
                                    nthreads=os.cpu_count() or 1)
        data[name] = {"n": w.n, "S": w.S, "U": U, "U_half": Uh, "blob": "a=1.9 alpha=15 m=0 N=10000 lerp",
                      "seeds": [w.meta["seed_phantom"], w.meta["seed_orient"]]}
        print(name, data[name], flush=True)
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(tuple(sys.argv[1:]) or ("small", "paper", "precision"))
