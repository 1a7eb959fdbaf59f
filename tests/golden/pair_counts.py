"""Writes pair_counts.json: exact (sample, voxel) pair counts of the named
synthetic workloads, computed by the FP64 oracle's scatter loop only.

U counts every pair of a disk sample and a voxel within the blob radius over
the full box; U_half counts those whose voxel has x >= 0 (the half box the
GPU kernels accumulate).  The benchmark divides these counts by its measured
times to report updates per second.

Named batches (synth.BATCHES) get one entry per reconstruction.

Run:  python tests/golden/pair_counts.py [name ...]   (default: small paper precision)
Entries for names not given are kept.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pair_counts.json")


def batch_counts(name):
    """Per-job pair counts of a named batch (orientations only: the counts do
    not depend on the sample values, so the oracle runs on zero slices, a few
    thousand at a time)."""
    jobs = []
    for spec in synth.batch_specs(name):
        n, S = spec[0], spec[1]
        q = synth.batch_quaternions(spec)
        U = Uh = 0
        for s0 in range(0, S, 2000):
            s1 = min(S, s0 + 2000)
            zero = np.zeros((s1 - s0, n, n // 2 + 1), dtype=np.complex64)
            _, _, u, uh = oracle.insert(n, zero, q[s0:s1], with_half=True, nthreads=os.cpu_count() or 1)
            U, Uh = U + u, Uh + uh
        jobs.append({"n": n, "S": S, "U": U, "U_half": Uh, "seeds": [spec[3], spec[4]]})
        print(name, jobs[-1], flush=True)
    return {"jobs": jobs, "U": sum(j["U"] for j in jobs), "U_half": sum(j["U_half"] for j in jobs),
            "blob": "a=1.9 alpha=15 m=0 N=10000 lerp"}


def main(names=("small", "paper", "precision")):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        if name in synth.BATCHES:
            data[name] = batch_counts(name)
            continue
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
