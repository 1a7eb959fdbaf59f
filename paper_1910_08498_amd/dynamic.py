"""Dynamic autotuning of a whole reconstruction (host-side driver).

The paper tunes the insertion kernel while the reconstruction runs
(Sect. 3.2, dynamic tuning; Sect. 5.3.2 and its table of dynamically tuned
3D Fourier reconstruction): every tuning step is one real kernel call with
a new configuration, random search stops after 50 steps (or after the whole
space), and the result is the whole run's time relative to the oraculum, a
run that uses the best configuration from the first call on.  This module
reproduces that protocol on one MI355X with the library's own tuner
(recon_tune_begin: non-blocking search, each step one recon_insert_batch
call, steps timed with events over the insertion and its partial-sum
reduction) on synthetic data of the paper's shape: boxes of 156, the
paper's 1,826,160 samples inserted in calls of 1,500 (1,218 calls, the last
one partial), cycling through a resident set of phantom slices.

Policies (each a whole run: zero G and W, all calls, finalize):
  oraculum      the fastest configuration, found beforehand by timing every
                configuration of the space (median of a few calls each);
  default       the library's default configuration, no tuning;
  random        random search of `steps` steps (seeded), repeated;
  whole_space   every configuration once, then the fastest;
  guided        a trained predictor's top 3 plus the default configuration
                (when a predictor file is given), else nothing.
Printed as one JSON line.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np
import torch

from . import recon

PAPER_SAMPLES = 1_826_160      # images of the paper's data set (Sect. 5.3.2)
CALL_SLICES = 1500             # samples per kernel call (Sect. 5.3.2)


def calls_for(samples: int, per_call: int = CALL_SLICES) -> list:
    """Slice counts of the calls that insert `samples` samples."""
    full, rest = divmod(samples, per_call)
    return [per_call] * full + ([rest] if rest else [])


class Run:
    """A reconstruction context over a resident set of slices, cycled."""

    def __init__(self, n: int, resident: int, seed: int, device="cuda:0"):
        import synth
        self.dev = torch.device(device)
        w = synth.make_workload("paper", n=n, S=resident, K=40, seed_phantom=seed, seed_orient=seed + 1)
        self.n, self.R = n, resident
        self.slices = torch.from_numpy(w.slices).to(self.dev)
        self.quats = torch.from_numpy(w.quats).to(self.dev)
        self.rec = recon.Reconstruction(n, device=self.dev)
        self.V = torch.empty_like(self.rec.G)
        self.default = recon.recon_get_config(self.rec.ctx)
        self.pos = 0

    def call(self, count: int):
        """One kernel call: the next `count` resident slices (wrapping)."""
        if self.pos + count > self.R:
            self.pos = 0
        s0 = self.pos
        recon.recon_insert_batch(self.rec.ctx, self.slices[s0:s0 + count], None, self.quats[s0:s0 + count], count)
        self.pos += count

    def whole(self, calls: list, before=None) -> float:
        """Wall time of a whole run (s): reset, `before` (e.g. start a tuning
        search), every call, finalize, synchronise."""
        torch.cuda.synchronize(self.dev)
        t0 = time.perf_counter()
        self.rec.reset()
        self.pos = 0
        if before is not None:
            before()
        for c in calls:
            self.call(c)
        self.rec.finalize(out=self.V)
        torch.cuda.synchronize(self.dev)
        return time.perf_counter() - t0

    def restore_default(self):
        recon.recon_tune_end(self.rec.ctx)
        recon.recon_set_config(self.rec.ctx, self.default)


def time_configs(run: Run, repeats: int = 3) -> np.ndarray:
    """Median time of one full call (s) of every configuration of the space
    (prep, insertion and reduction, events on the stream), after a warm-up."""
    size = recon.recon_tune_space_size(run.rec.ctx)
    out = np.zeros(size)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for i in range(size):
        recon.recon_set_config(run.rec.ctx, recon.recon_tune_space_config(run.rec.ctx, i))
        run.call(CALL_SLICES)
        t = []
        for _ in range(repeats):
            e0.record()
            run.call(CALL_SLICES)
            e1.record()
            e1.synchronize()
            t.append(e0.elapsed_time(e1) * 1e-3)
        out[i] = float(np.median(t))
    recon.recon_set_config(run.rec.ctx, run.default)
    return out


def guided_order(run: Run, model_file: str, k: int = 3) -> list:
    """Tuning-space indices to try: a trained predictor's top k runnable
    configurations for this workload, then the default if not among them."""
    from . import learned
    model, keys = learned.load_predictor(model_file, device=run.dev)
    size = recon.recon_tune_space_size(run.rec.ctx)
    space_keys = [learned.config_key(recon.recon_tune_space_config(run.rec.ctx, i)) for i in range(size)]
    total = torch.cuda.get_device_properties(run.dev).multi_processor_count
    feats = learned.features(run.n, CALL_SLICES, float(run.rec.params.blob_radius), 1.0)
    prob = model.predict(feats.reshape(1, -1))[0]
    col = {kk: i for i, kk in enumerate(keys)}
    p_space = np.array([prob[col[kk]] if kk in col else -np.inf for kk in space_keys])
    order = [int(i) for i in learned.ranked_candidates(p_space, np.isfinite(p_space), k)]
    d = space_keys.index(learned.config_key(run.default)) if learned.config_key(run.default) in space_keys else -1
    if d >= 0 and d not in order:
        order.append(d)
    del total
    return order


def protocol(n: int = 156, samples: int = PAPER_SAMPLES, resident: int = 6000, steps: int = 50,
             repeats: int = 100, seed: int = 11, model_file: str | None = None, device="cuda:0") -> dict:
    calls = calls_for(samples)
    run = Run(n, resident, seed, device)
    log = lambda m: print(f"dynamic: {m}", file=sys.stderr, flush=True)   # noqa: E731
    log(f"n={n}, {len(calls)} calls of up to {CALL_SLICES} slices, resident set {resident}")
    run.whole(calls[:20])                                      # warm-up
    t_cfg = time_configs(run)
    best = int(np.argmin(t_cfg))
    size = t_cfg.size
    log(f"space of {size} configurations timed; fastest {t_cfg[best] * 1e3:.3f} ms per call (index {best})")

    def fixed(idx):
        recon.recon_set_config(run.rec.ctx, recon.recon_tune_space_config(run.rec.ctx, idx))
        t = run.whole(calls)
        run.restore_default()
        return t

    t_orc = min(fixed(best) for _ in range(3))
    t_def = min(run.whole(calls) for _ in range(3))
    log(f"oraculum {t_orc:.3f} s, default {t_def:.3f} s")
    rand = []
    for r in range(repeats):
        t = run.whole(calls, before=lambda: recon.recon_tune_begin(run.rec.ctx, max_steps=steps, seed=seed * 1000 + r))
        info = recon.recon_tune_get_info(run.rec.ctx)
        rand.append((t, int(info.best_index)))
        run.restore_default()
        if (r + 1) % 10 == 0:
            log(f"random search {r + 1}/{repeats}: mean {np.mean([x[0] for x in rand]):.3f} s")
    t_whole = run.whole(calls, before=lambda: recon.recon_tune_begin(run.rec.ctx, max_steps=0, seed=seed))
    run.restore_default()
    rp = np.array([t_orc / t for t, _ in rand])
    out = {
        "workload": f"{samples} samples of {n}x{n} (half plane {n}x{n // 2 + 1} complex64) in {len(calls)} calls "
                    f"of up to {CALL_SLICES}, cycling {resident} resident phantom slices; KB blob a=1.9 alpha=15 "
                    f"m=0, 10,000-entry table",
        "space_size": size,
        "config_time_ms": {"best": float(t_cfg[best] * 1e3), "mean": float(t_cfg.mean() * 1e3),
                           "average_over_best": float(t_cfg.mean() / t_cfg[best])},
        "best_config": {k: getattr(recon.recon_tune_space_config(run.rec.ctx, best), k)
                        for k, _ in recon.recon_config._fields_ if k != "reserved"},
        "oraculum_s": t_orc,
        "default": {"s": t_def, "pct_of_oraculum": 100.0 * t_orc / t_def},
        "random": {"steps": steps, "repeats": repeats, "mean_s": float(np.mean([t for t, _ in rand])),
                   "pct_of_oraculum_mean": float(100.0 * rp.mean()), "pct_of_oraculum_sd": float(100.0 * rp.std()),
                   "found_within_5pct": float(np.mean([t_cfg[b] <= 1.05 * t_cfg[best] for _, b in rand]))},
        "whole_space": {"steps": size, "s": t_whole, "pct_of_oraculum": 100.0 * t_orc / t_whole},
    }
    if model_file:
        order = guided_order(run, model_file)
        tg = []
        for r in range(5):
            tg.append(run.whole(calls, before=lambda: recon.recon_tune_begin(run.rec.ctx, order=order)))
            info = recon.recon_tune_get_info(run.rec.ctx)
            picked = int(info.best_index)
            run.restore_default()
        t_g = min(tg)
        out["guided"] = {"steps": len(order), "order": order, "picked": picked, "s": t_g,
                         "pct_of_oraculum": 100.0 * t_orc / t_g,
                         "picked_over_best_call": float(t_cfg[picked] / t_cfg[best])}
    run.rec.close()
    return out


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="the paper's dynamic-tuning protocol on a whole reconstruction")
    ap.add_argument("--n", type=int, default=156)
    ap.add_argument("--samples", type=int, default=PAPER_SAMPLES)
    ap.add_argument("--resident", type=int, default=6000)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--repeats", type=int, default=100)
    ap.add_argument("--predictor", default=None, help="predictor file written by learned --save-model")
    args = ap.parse_args(argv)
    res = protocol(args.n, args.samples, args.resident, args.steps, args.repeats, model_file=args.predictor)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
