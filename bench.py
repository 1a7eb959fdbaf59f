"""Benchmark of the Fourier-slice insertion path on one MI355X.

A step is one pass of the whole path over the workload's slices, all inputs
already resident in HBM: zero G and W, insert every slice in batches of
1,500 (orientation prep, tile-binned gather, partial-sum reduction), and
finalize (Hermitian mirror, V = G / W).  The default workload is the
paper-scale case: 10,000 slices of 128 x 128 (half plane 128 x 65 complex64)
into a 129^3 volume with a Kaiser-Bessel blob a = 1.9, alpha = 15, order 0
and a 10,000-entry table.

The headline value is slice-sample x voxel updates per second: the exact
number of (disk sample, voxel within the blob) pairs of the workload, counted
by the FP64 oracle and stored in tests/golden/pair_counts.json, divided by
the measured time per step.  Printed as one JSON line, which also carries
the roofline of the insertion kernel, the same step with the plain per-voxel
gather ("plain", and "default_over_plain"), the step with the configuration
the library's dynamic tuner selects on this workload ("tuned", and
"tuned_over_plain"), the step with the interpolation weights evaluated on
the fly instead of read from the table ("on_the_fly"), the FP64 oracle timed
on a sample of the workload
("cpu_baseline"), and the error of the measured configuration against that
oracle on the same sample ("error_vs_oracle").  The headline value is the
library's default configuration, untuned.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X vector FP32 (published)
PEAK_HBM_GBPS = 8000.0        # MI355X HBM3E (published)
FLOPS_PER_UPDATE = 10         # essential: 5 for d^2, 2 FMA + 1 add for G.re, G.im, W
KERNEL_SRCS = [os.path.join(ROOT, "paper_1910_08498_amd", "csrc", f)
               for f in ("kernels.hip", "slab.hip", "recon_api.cpp")]   # kernels and their work plan
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "insert_slab_paper_traffic.json")

WORKLOAD_TEXT = {
    "paper": "paper-scale insertion: 10,000 Fourier slices of 128x128 (half plane 128x65 complex64) "
             "into a 129^3 complex64 G + float32 W, KB blob a=1.9 alpha=15 m=0, 10,000-entry table (lerp), "
             "batches of 1,500 slices",
    "small": "small insertion: 500 Fourier slices of 64x64 (half plane 64x33 complex64) into a 65^3 "
             "complex64 G + float32 W, KB blob a=1.9 alpha=15 m=0, 10,000-entry table (lerp)",
    "precision": "large insertion with 16-bit slice storage: 50,000 Fourier slices of 256x256 (half plane "
                 "256x129, 45,000 Haar-uniform + 5,000 clustered views) into a 257^3 complex64 G + float32 W, "
                 "KB blob a=1.9 alpha=15 m=0, 10,000-entry table (lerp), batches of 1,500 slices",
    "batch8": "batched insertion: 8 reconstructions, boxes 64,96,128,160,192,224,256,256, slice counts "
              "uniform in 2,000-20,000 (seed 5), complex64 slices, FP32, one persistent slab launch per round "
              "of batches of up to 1,500 slices per reconstruction, configuration from the library's tuner",
}


def kernel_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def load_traffic(launch_count_per_step):
    """HBM bytes per insertion launch from committed rocprofv3 PMC runs, if
    they were taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256") != kernel_sha():
        return None
    return t.get("bytes_per_launch")


def cpu_model() -> str:
    """The host CPU's model name (as lscpu prints it)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workload, n_slices: int, slices=None, n_single: int = 0):
    """The FP64 oracle on a bounded sample of the same workload, on all the
    host cores this process may use (at most 16, the host share of one GPU)
    and, on a smaller sample, on one thread; returns the timing record and
    the oracle's G and W for the all-core sample."""
    import oracle
    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = nproc
    threads = max(1, min(avail, 16))
    sl = (workload.slices if slices is None else slices)[:n_slices]
    q = workload.quats[:n_slices]
    oracle.insert(workload.n, sl[:8], q[:8], nthreads=threads)      # load / warm
    t0 = time.perf_counter()
    G, W, U = oracle.insert(workload.n, sl, q, nthreads=threads)
    dt = time.perf_counter() - t0
    rec = {"value": U / dt, "unit": "updates/s", "cores": threads, "kind": "oracle",
           "sample": f"first {n_slices} of {workload.S} slices of the same workload "
                     f"({U} pairs, FP64 scatter, table lerp), {dt:.2f} s wall",
           "nproc": nproc, "cpu_model": cpu_model()}
    if n_single > 0:
        k = min(n_single, n_slices)
        t0 = time.perf_counter()
        _, _, U1 = oracle.insert(workload.n, sl[:k], q[:k], nthreads=1)
        dt1 = time.perf_counter() - t0
        rec["single_thread"] = {"value": U1 / dt1, "unit": "updates/s", "cores": 1,
                                "sample": f"first {k} slices ({U1} pairs), {dt1:.2f} s wall"}
    return rec, G, W


def error_vs_oracle(rec, torch, slices, quats, scales, k: int, batch: int, V, G_o, W_o):
    """Relative L2 error of the measured configuration against the oracle on
    the CPU-baseline sample: the first k slices inserted into a cleared
    volume, whole volume compared."""
    import oracle
    from paper_1910_08498_amd import recon
    rec.reset()
    for s0 in range(0, k, batch):
        s1 = min(k, s0 + batch)
        recon.recon_insert_batch(rec.ctx, slices[s0:s1], None if scales is None else scales[s0:s1],
                                 quats[s0:s1], s1 - s0)
    rec.finalize(out=V)
    torch.cuda.synchronize()
    G, W, Vg = rec.G.cpu().numpy(), rec.W.cpu().numpy(), V.cpu().numpy()
    return {"G": oracle.rel_l2(G, G_o), "W": oracle.rel_l2(W, W_o), "V": oracle.rel_l2(Vg, oracle.finalize(G_o, W_o)),
            "bound": 1e-5, "sample": f"first {k} slices, whole volume, FP64 oracle on the values the kernels read"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="paper", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--variant", default="slab", choices=["slab", "binned", "naive"])
    ap.add_argument("--batch", type=int, default=1500)
    ap.add_argument("--dtype", default="c64", choices=["c64", "f16", "bf16"],
                    help="slice storage: complex64, half pairs with a per-slice scale, or bfloat16 pairs")
    ap.add_argument("--cpu-slices", type=int, default=2500,
                    help="slices in the CPU-oracle sample (0 disables the CPU baseline)")
    ap.add_argument("--cpu-single-slices", type=int, default=400,
                    help="slices in the one-thread CPU-oracle sample (0 disables it)")
    ap.add_argument("--plain-steps", type=int, default=1,
                    help="steps timed with the naive (plain) kernel for comparison (0 disables)")
    ap.add_argument("--tune-steps", type=int, default=50,
                    help="random-search steps of the library's tuner before the tuned leg (0 disables it)")
    ap.add_argument("--otf-steps", type=int, default=2,
                    help="steps timed with interpolation weights evaluated on the fly instead of the table "
                         "(0 disables)")
    ap.add_argument("--h2d-steps", type=int, default=2,
                    help="steps timed with the slices uploaded from pinned host memory (0 disables)")
    ap.add_argument("--traversal", type=int, default=0, choices=[0, 1, 2, 3],
                    help="recon_config.traversal of the measured configuration (slab: lanes' column order, "
                         "bit 0; spatial work queue, bit 1)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB after timing (HBM counter calibration)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {args.gpus} is not supported (the insertion would "
              f"shard by slices: each GPU inserts its share into its own G and W, then one sum-reduction)",
              file=sys.stderr)
        return 2
    if args.workload == "batch8":
        return bench_batch8(args)

    import numpy as np
    import torch

    import synth
    from paper_1910_08498_amd import recon

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"bench: generating workload '{args.workload}'", file=sys.stderr, flush=True)
    w = synth.make_workload(args.workload)
    with open(os.path.join(ROOT, "tests", "golden", "pair_counts.json")) as f:
        counts = json.load(f)[args.workload]
    assert counts["n"] == w.n and counts["S"] == w.S
    U, U_half = int(counts["U"]), int(counts["U_half"])

    quats = torch.from_numpy(w.quats).to(dev)
    scales = None
    cpu_slices = w.slices
    if args.dtype == "c64":
        slices = torch.from_numpy(w.slices).to(dev)
        slice_bytes = w.slices.nbytes + w.quats.nbytes
        sdt = recon.RECON_SLICE_C64
    else:
        from synth.phantom import dequantize_slices, quantize_slices
        bits, sc = quantize_slices(w.slices, args.dtype)
        tdt = torch.float16 if args.dtype == "f16" else torch.bfloat16
        slices = torch.from_numpy(bits.view(np.int16)).to(dev).view(tdt)
        sdt = recon.RECON_SLICE_F16 if args.dtype == "f16" else recon.RECON_SLICE_BF16
        slice_bytes = bits.nbytes + w.quats.nbytes
        if args.dtype == "f16":
            scales = torch.from_numpy(sc).to(dev)
            slice_bytes += sc.nbytes
        if args.cpu_slices > 0:        # the oracle gets the values the kernels read
            k = min(args.cpu_slices, w.S)
            cpu_slices = dequantize_slices(bits[:k], sc[:k], args.dtype)
        del bits
    rec = recon.Reconstruction(w.n, device=dev, max_batch=args.batch, slice_dtype=sdt)
    variant_ids = {"slab": recon.RECON_VARIANT_SLAB, "binned": recon.RECON_VARIANT_BINNED,
                   "naive": recon.RECON_VARIANT_NAIVE}

    def set_default(**extra):
        # the measured configuration: the library's defaults for the variant
        # (every knob a leg may have changed), with the requested traversal
        cfg = dict(variant=variant_ids[args.variant], waves_per_block=0, slab_flags=0, inner_chunk=0, split=0,
                   weights=0, traversal=args.traversal)
        cfg.update(extra)
        rec.set_config(**cfg)

    set_default()
    V = torch.empty_like(rec.G)
    nb = (w.S + args.batch - 1) // args.batch
    stream = torch.cuda.current_stream()

    def step(events=None):
        rec.reset()
        for b in range(nb):
            s0, s1 = b * args.batch, min(w.S, (b + 1) * args.batch)
            if events is not None:
                recon.recon_set_timing_events(rec.ctx, *events[b])
            recon.recon_insert_batch(rec.ctx, slices[s0:s1], None if scales is None else scales[s0:s1],
                                     quats[s0:s1], s1 - s0)
        if events is not None:
            recon.recon_set_timing_events(rec.ctx, None, None)
        rec.finalize(out=V)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"bench: timing {args.steps} steps", file=sys.stderr, flush=True)

    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nb)]
          for _ in range(args.steps)]
    for row in ev:                 # torch creates the HIP events on first record
        for a, b in row:
            a.record(stream)
            b.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(ev[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    kernel_ms = np.array([[a.elapsed_time(b) for a, b in row] for row in ev])     # [steps, nb]
    kernel_ms_per_step = float(kernel_ms.sum(axis=1).mean())
    avg_launch_ms = float(kernel_ms.mean())

    value = U / (ms_per_step / 1e3)
    # roofline of the dominant kernel (the insertion kernel), per launch
    flops_per_step = FLOPS_PER_UPDATE * U_half
    achieved_tflops = flops_per_step / (kernel_ms_per_step / 1e3) / 1e12
    half_vox = (w.n // 2 + 1) * (w.n + 1) ** 2
    gw_rmw = 2 * 12 * half_vox * nb          # G (8 B) + W (4 B) read and written per launch
    alg_bytes_step = slice_bytes + gw_rmw
    # the stored counter run covers the default configuration only
    traffic = load_traffic(nb) if (args.workload, args.variant, args.dtype, args.batch) == \
        ("paper", "slab", "c64", 1500) else None

    h2d = None
    if args.h2d_steps > 0:
        h2d = h2d_inclusive(args, torch, recon, rec, slices, quats, scales, nb, w.S, U, V)

    tuned = None
    if args.tune_steps > 0:
        tuned = tuned_leg(args, torch, recon, rec, step, nb, w.S, slices, quats, scales, U, ms_per_step)
        set_default()

    plain = None
    if args.plain_steps > 0 and args.variant != "naive":
        set_default(variant=recon.RECON_VARIANT_NAIVE, traversal=0)
        step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.plain_steps):
            step()
        torch.cuda.synchronize()
        plain_ms = 1e3 * (time.perf_counter() - t1) / args.plain_steps
        plain = {"value": U / (plain_ms / 1e3), "ms_per_step": plain_ms, "variant": "naive"}
        set_default()

    otf = None
    if args.otf_steps > 0 and args.workload != "batch8":
        # the same step with the blob evaluated on the fly (Horner's rule on its
        # power series) instead of read from the table; the library's default
        # configuration for that weight source
        set_default(weights=recon.RECON_WEIGHTS_OTF)
        otf_cfg = rec.config()
        step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.otf_steps):
            step()
        torch.cuda.synchronize()
        otf_ms = 1e3 * (time.perf_counter() - t1) / args.otf_steps
        otf = {"value": U / (otf_ms / 1e3), "ms_per_step": otf_ms, "config": otf_cfg,
               "note": "interpolation weights evaluated on the fly (the table leg is value)"}
        set_default()

    if args.calib_copy_mb > 0:
        nbytes = args.calib_copy_mb << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = err = None
    if args.cpu_slices > 0:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        k = min(args.cpu_slices, w.S)
        cpu, G_o, W_o = cpu_baseline(w, k, cpu_slices, args.cpu_single_slices)
        err = error_vs_oracle(rec, torch, slices, quats, scales, k, args.batch, V, G_o, W_o)
        del G_o, W_o

    result = {
        "metric": "slice-sample×voxel updates/s",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded 40-Gaussian phantom projections (exact line integrals) and their centered "
                "DFTs, Haar-uniform orientations; stands in for EMPIAR-10010",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "n": w.n, "slices": w.S, "batch": args.batch,
                   "variant": args.variant, "slice_storage": args.dtype, "traversal": args.traversal,
                   "pairs_U": U, "pairs_half_box": U_half},
        "roofline": {
            "bound": "alu",
            "kernel": {"slab": "k_insert_slab", "binned": "k_insert_binned", "naive": "k_insert_naive"}[args.variant],
            "achieved": achieved_tflops,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / PEAK_FP32_TFLOPS,
            "traffic": traffic,
            "avg_launch_ms": avg_launch_ms,
            "launches_per_step": nb,
            "flops_per_update": FLOPS_PER_UPDATE,
            "hbm_alg_GBps": alg_bytes_step / (kernel_ms_per_step / 1e3) / 1e9,
            "hbm_alg_frac": alg_bytes_step / (kernel_ms_per_step / 1e3) / 1e9 / PEAK_HBM_GBPS,
        },
        "h2d_inclusive": h2d,
        "plain": plain,
        "default_over_plain": None if plain is None else value / plain["value"],
        "on_the_fly": otf,
        "tuned": tuned,
        "tuned_over_plain": None if plain is None or tuned is None else tuned["value"] / plain["value"],
        "error_vs_oracle": err,
        "cpu_baseline": cpu,
    }
    print(json.dumps(result), flush=True)
    rec.close()
    return 0


def tuned_leg(args, torch, recon, rec, step, nb, S, slices, quats, scales, U, default_ms):
    """The library's dynamic tuner on this workload: a seeded random search of
    --tune-steps configurations, each step one real insertion call of the
    workload's batches (non-blocking tuning), then the step timed with the
    configuration it selected."""
    recon.recon_tune_begin(rec.ctx, max_steps=args.tune_steps, seed=2024)
    k = 0
    while recon.recon_tune_get_info(rec.ctx).active:
        b = k % nb
        s0, s1 = b * args.batch, min(S, (b + 1) * args.batch)
        recon.recon_insert_batch(rec.ctx, slices[s0:s1], None if scales is None else scales[s0:s1],
                                 quats[s0:s1], s1 - s0)
        k += 1
    recon.recon_tune_end(rec.ctx)
    info = recon.recon_tune_get_info(rec.ctx)
    cfg = rec.config()
    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    return {"value": U / (ms / 1e3), "ms_per_step": ms, "over_default": default_ms / ms,
            "search": f"random search, {int(info.steps_done)} of {int(info.space_size)} configurations, "
                      f"one insertion call each", "config": cfg}


def h2d_inclusive(args, torch, recon, rec, slices, quats, scales, nb, S, U, V):
    """The same step with the slices starting in pinned host memory: each
    batch is copied to one of two device buffers on a second stream while the
    previous batch is inserted (events order the two streams).  Reported
    beside the main figure, never as it."""
    dev = slices.device
    host = torch.empty(slices.shape, dtype=slices.dtype, pin_memory=True)
    host.copy_(slices.cpu())
    per = args.batch
    bufs = [torch.empty((per,) + tuple(slices.shape[1:]), dtype=slices.dtype, device=dev) for _ in range(2)]
    comp = torch.cuda.current_stream()
    copy = torch.cuda.Stream(device=dev)           # default priority
    copied = [torch.cuda.Event() for _ in range(2)]
    used = [torch.cuda.Event() for _ in range(2)]
    for e in used:
        e.record(comp)

    def step():
        rec.reset()
        for b in range(nb):
            s0, s1 = b * per, min(S, (b + 1) * per)
            k = b % 2
            with torch.cuda.stream(copy):
                copy.wait_event(used[k])
                bufs[k][: s1 - s0].copy_(host[s0:s1], non_blocking=True)
                copied[k].record(copy)
            comp.wait_event(copied[k])
            recon.recon_insert_batch(rec.ctx, bufs[k][: s1 - s0], None if scales is None else scales[s0:s1],
                                     quats[s0:s1], s1 - s0)
            used[k].record(comp)
        rec.finalize(out=V)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.h2d_steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.h2d_steps
    nbytes = slices.numel() * slices.element_size()
    del host, bufs
    return {"value": U / (ms / 1e3), "unit": "updates/s", "ms_per_step": ms,
            "host_to_device_GBps": nbytes / (ms / 1e3) / 1e9,
            "note": "slices uploaded from pinned host memory per batch, overlapped with insertion"}


def bench_batch8(args) -> int:
    """Eight reconstructions of different box sizes inserted by one persistent
    launch per round (recon_batch_insert), each round up to --batch slices
    per reconstruction.  The launch configuration is the one the library's
    tuner selects on the largest box (a random search over real insertion
    calls), given to the batch through its first context.  The step (zero,
    every round, finalize) is captured once in a HIP graph and replayed; the
    same rounds with one launch per reconstruction, eager, are timed beside
    it.  Slices are phantom projections (synth), pair counts exact
    (tests/golden/pair_counts.json), and each reconstruction's first slices
    are checked against the FP64 oracle."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_1910_08498_amd import recon

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    with open(os.path.join(ROOT, "tests", "golden", "pair_counts.json")) as f:
        counts = json.load(f)["batch8"]
    specs = synth.batch_specs("batch8")
    assert [(j["n"], j["S"]) for j in counts["jobs"]] == [(sp[0], sp[1]) for sp in specs]
    side = torch.cuda.Stream(device=dev)          # default priority; graphs are captured on it
    jobs = []
    with torch.cuda.stream(side):
        for spec in specs:
            n, S, K, sp, so = spec
            print(f"bench: job n={n} S={S}", file=sys.stderr, flush=True)
            w = synth.make_workload("small", n=n, S=S, K=K, seed_phantom=sp, seed_orient=so)
            rec = recon.Reconstruction(n, device=dev, stream=side, max_batch=args.batch)
            jobs.append({"w": w, "rec": rec, "sl": torch.from_numpy(w.slices).to(dev),
                         "q": torch.from_numpy(w.quats).to(dev)})
    side.synchronize()
    rounds = max((j["w"].S + args.batch - 1) // args.batch for j in jobs)

    # tune on the largest box, hand the configuration to the batch's first context
    big = max(jobs, key=lambda j: j["w"].n * j["w"].n * j["w"].S)
    tuned_cfg = None
    if args.tune_steps > 0:
        rb = big["rec"]
        recon.recon_tune_begin(rb.ctx, max_steps=args.tune_steps, seed=2024)
        k = 0
        while recon.recon_tune_get_info(rb.ctx).active:
            s0 = (k * args.batch) % max(1, big["w"].S - args.batch)
            recon.recon_insert_batch(rb.ctx, big["sl"][s0:s0 + args.batch], None, big["q"][s0:s0 + args.batch],
                                     args.batch)
            k += 1
        recon.recon_tune_end(rb.ctx)
        tuned_cfg = recon.recon_get_config(rb.ctx)
        if tuned_cfg.variant == recon.RECON_VARIANT_SLAB:
            recon.recon_set_config(jobs[0]["rec"].ctx, tuned_cfg)
        side.synchronize()
    ctxs = [j["rec"].ctx for j in jobs]
    ws = torch.empty(recon.recon_batch_query_size(ctxs), dtype=torch.uint8, device=dev)
    b = recon.recon_batch_create(ctxs, ws)

    def round_args(r):
        sls, qts, cnt = [], [], []
        for j in jobs:
            S = j["w"].S
            s0, s1 = min(S, r * args.batch), min(S, (r + 1) * args.batch)
            sls.append(j["sl"][s0:s1] if s1 > s0 else None)
            qts.append(j["q"][s0:s1] if s1 > s0 else None)
            cnt.append(s1 - s0)
        return sls, qts, cnt

    prepared = [round_args(r) for r in range(rounds)]

    def step():
        for j in jobs:
            j["rec"].reset()
        for sls, qts, cnt in prepared:
            recon.recon_batch_insert(b, sls, None, qts, cnt)
        for j in jobs:
            j["rec"].finalize()

    def step_separate():
        for j in jobs:
            j["rec"].reset()
        for sls, qts, cnt in prepared:
            for j, sl, q, c in zip(jobs, sls, qts, cnt):
                if c:
                    recon.recon_insert_batch(j["rec"].ctx, sl, None, q, c)
        for j in jobs:
            j["rec"].finalize()

    def timed(fn):
        with torch.cuda.stream(side):
            for _ in range(args.warmup):
                fn()
            side.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fn()
            side.synchronize()
        return 1e3 * (time.perf_counter() - t0) / args.steps

    ms_eager = timed(step)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        step()                                     # warm state before capture
        side.synchronize()
        with torch.cuda.graph(graph, stream=side):
            step()
    side.synchronize()
    ms = timed(graph.replay)
    ms_sep = timed(step_separate)
    U, U_half = int(counts["U"]), int(counts["U_half"])

    # the batched insertion kernel's own duration, per launch: events on the
    # launch stream around the kernel alone (the first context's timing
    # events), over eager runs of the step's rounds
    kev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(rounds)]
           for _ in range(max(1, args.steps))]
    c0 = jobs[0]["rec"].ctx
    with torch.cuda.stream(side):
        for row in kev:                           # torch creates the HIP events on first record
            for e0, e1 in row:
                e0.record(side)
                e1.record(side)
        side.synchronize()
        for row in kev:
            for j in jobs:
                j["rec"].reset()
            for (sls, qts, cnt), (e0, e1) in zip(prepared, row):
                recon.recon_set_timing_events(c0, e0, e1)
                recon.recon_batch_insert(b, sls, None, qts, cnt)
            recon.recon_set_timing_events(c0, None, None)
        side.synchronize()
    kernel_ms = np.array([[e0.elapsed_time(e1) for e0, e1 in row] for row in kev])     # [steps, rounds]
    kernel_ms_per_step = float(kernel_ms.sum(axis=1).mean())
    achieved_tflops = FLOPS_PER_UPDATE * U_half / (kernel_ms_per_step / 1e3) / 1e12
    # algorithmic bytes: every slice read once; every launch reads and writes
    # each box's half of G (8 B) and W (4 B)
    slice_bytes = sum(j["w"].S * j["w"].n * (j["w"].n // 2 + 1) * 8 for j in jobs)
    gw_rmw = sum(2 * 12 * (j["w"].n // 2 + 1) * (j["w"].n + 1) ** 2 for j in jobs) * rounds
    hbm_gbps = (slice_bytes + gw_rmw) / (kernel_ms_per_step / 1e3) / 1e9

    # each reconstruction's first slices, through the same batched launch, against the oracle
    k = 120
    errs = []
    with torch.cuda.stream(side):
        for j in jobs:
            j["rec"].reset()
        sls, qts, cnt = [], [], []
        for j in jobs:
            sls.append(j["sl"][:k])
            qts.append(j["q"][:k])
            cnt.append(min(k, j["w"].S))
        recon.recon_batch_insert(b, sls, None, qts, cnt)
        Vs = [j["rec"].finalize() for j in jobs]
        side.synchronize()
    for j, V in zip(jobs, Vs):
        w = j["w"]
        Go, Wo, _ = oracle.insert(w.n, w.slices[:k], w.quats[:k], nthreads=16)
        errs.append({"n": w.n, "G": oracle.rel_l2(j["rec"].G.cpu().numpy(), Go),
                     "W": oracle.rel_l2(j["rec"].W.cpu().numpy(), Wo),
                     "V": oracle.rel_l2(V.cpu().numpy(), oracle.finalize(Go, Wo))})
    result = {
        "metric": "slice-sample×voxel updates/s", "value": U / (ms / 1e3), "unit": "updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic: seeded phantom projections (exact line integrals) and their centered DFTs, "
                "Haar-uniform orientations, per reconstruction",
        "config": {"workload": WORKLOAD_TEXT["batch8"], "boxes": [j["w"].n for j in jobs],
                   "slices": [j["w"].S for j in jobs], "rounds_per_step": rounds, "pairs_U": U,
                   "launch": "one captured HIP graph per step, replayed",
                   "batch_config": None if tuned_cfg is None else
                   {k2: getattr(tuned_cfg, k2) for k2, _ in recon.recon_config._fields_ if k2 != "reserved"},
                   "tuned_on": f"n={big['w'].n}, {args.tune_steps} random-search steps"},
        "eager": {"value": U / (ms_eager / 1e3), "ms_per_step": ms_eager},
        "separate_launches": {"value": U / (ms_sep / 1e3), "ms_per_step": ms_sep,
                              "launches_per_round": len(jobs)},
        "error_vs_oracle": {"per_job": errs, "bound": 1e-5,
                            "sample": f"first {k} slices of each reconstruction, one batched launch, whole volumes"},
        "roofline": {
            "bound": "alu",
            "kernel": "k_insert_slab",
            "achieved": achieved_tflops,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / PEAK_FP32_TFLOPS,
            "traffic": None,
            "avg_launch_ms": float(kernel_ms.mean()),
            "launches_per_step": rounds,
            "flops_per_update": FLOPS_PER_UPDATE,
            "pairs_half_box": U_half,
            "hbm_alg_GBps": hbm_gbps,
            "hbm_alg_frac": hbm_gbps / PEAK_HBM_GBPS,
        },
        "cpu_baseline": None,
    }
    print(json.dumps(result), flush=True)
    recon.recon_batch_destroy(b)
    for j in jobs:
        j["rec"].close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
