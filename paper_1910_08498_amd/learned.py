"""Learned configuration predictor on top of the autotuner (host-side driver).

Everything numeric runs in the library's HIP kernels: the timings come from
the insertion kernels timed with events, and the predictor is trained and
evaluated with recon_mlp_train_step / recon_mlp_forward.  This module only
marshals data: it builds seeded synthetic workloads, collects the time of
every configuration of the tuning space on each of them, turns timings into
target distributions, and measures the regret of the predicted configuration
against the fastest measured one (exhaustive search).

Features of a workload: log2(n), log2 of the slices per kernel call (the
library inserts batches of up to 1,500 slices, so only workloads of fewer
slices differ), blob radius a, and the fraction of the device's compute
units the reconstruction may use.  The last one is varied on the one device
available by running the timings on a CU-masked stream
(hipExtStreamCreateWithCUMask) with the library's cu_count set to match.

Each configuration is timed as the median of several calls, each call a
whole recon_insert_batch (orientation prep, insertion and the partial-sum
reduction of split tiles, whose cost the split knob changes), at the batch
size the library runs.  The predictor's classes are the slab-kernel
configurations with table weights and the default traversal: the other
variants and weights on the fly never win on this device, the traversal
settings change a call's time by a few per cent at most, and leaving them
out keeps the timing collection short (the run-time search still covers
the traversal knob).

The predictor ranks the configurations; at run time the library's tuner
then measures its top candidates, and the library's default configuration,
on real work (recon_tune_begin with a candidate order) and keeps the
fastest, which also measures how far the top-1 prediction was from the best
candidate.  With the default among the candidates the guided search is never
worse than running the default, up to timing noise.  When the predictor is not
confident (top probability below a threshold) the tuner falls back to its
random search.

Configurations are identified by their knob values (variant, waves per
work-group, inner chunk, split, slab flags, weight source, traversal).  The runnable set depends on the
workload (some kernel instances exist only for some blob windows), so the
predictor scores the union of the configurations seen in training and only
runnable ones are chosen for a workload.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import recon

N_HIDDEN = 64
CU_CHOICES = (64, 128, 192, 256)
CALL_SLICES = 1500          # the library's default batch (slices per kernel call)


def features(n: int, slices: int, a: float, cu_frac: float) -> np.ndarray:
    """Workload features: log2 n, log2 slices per call, blob radius, CU fraction."""
    return np.array([math.log2(n), math.log2(min(slices, CALL_SLICES)), a, cu_frac], dtype=np.float64)


def config_key(c) -> tuple:
    return (int(c.variant), int(c.waves_per_block), int(c.inner_chunk), int(c.split), int(c.slab_flags),
            int(c.weights), int(c.traversal))


KEY_LEN = 7


def _key(values) -> tuple:
    """A stored key as a tuple; keys written before the traversal knob existed
    (six values) take the default traversal 0."""
    k = tuple(int(v) for v in values)
    return k + (0,) * (KEY_LEN - len(k)) if k else k


@dataclass
class TuneRecord:
    n: int
    slices: int
    a: float
    ns_per_slice: np.ndarray            # [C] insertion-kernel time per slice of each configuration
    keys: list = field(default_factory=list)     # [C] configuration keys, aligned with ns_per_slice
    default_key: tuple | None = None    # the library's default configuration for this workload
    meta: dict = field(default_factory=dict)
    cus: int = 256                      # compute units the insertion may use
    cus_total: int = 256                # compute units of the device

    def features(self) -> np.ndarray:
        return features(self.n, self.slices, self.a, self.cus / self.cus_total)

    def save(self, path: str):
        np.savez(path, n=self.n, slices=self.slices, a=self.a, ns_per_slice=self.ns_per_slice,
                 keys=np.array(self.keys, dtype=np.int64).reshape(len(self.keys), -1),
                 default_key=np.array(self.default_key if self.default_key is not None else [], dtype=np.int64),
                 cus=self.cus, cus_total=self.cus_total)

    @staticmethod
    def load(path: str) -> "TuneRecord":
        z = np.load(path)
        dk = _key(z["default_key"]) or None
        return TuneRecord(n=int(z["n"]), slices=int(z["slices"]), a=float(z["a"]),
                          ns_per_slice=np.asarray(z["ns_per_slice"], dtype=np.float64),
                          keys=[_key(k) for k in z["keys"]], default_key=dk,
                          cus=int(z["cus"]), cus_total=int(z["cus_total"]))


def union_keys(records) -> list:
    """Configuration keys of all records, in first-seen order."""
    seen, out = set(), []
    for r in records:
        for k in r.keys:
            if k not in seen:
                seen.add(k)
                out.append(k)
    return out


def time_matrix(records, keys) -> np.ndarray:
    """[W, C] time per slice; +inf where a configuration does not run on a workload."""
    col = {k: i for i, k in enumerate(keys)}
    ns = np.full((len(records), len(keys)), np.inf)
    for w, r in enumerate(records):
        for k, t in zip(r.keys, r.ns_per_slice):
            if k in col:
                ns[w, col[k]] = t
    return ns


def sample_workloads(seed: int, count: int, n_range=(48, 384), s_range=(1000, 50000), a_range=(1.5, 2.5),
                     cu_choices=CU_CHOICES):
    """Seeded workload parameters (n, slices, a, CUs): n even (uniform), slices
    log-uniform, a uniform, CUs uniform over cu_choices."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(n_range[0] // 2, n_range[1] // 2 + 1)) * 2
        s = int(round(math.exp(rng.uniform(math.log(s_range[0]), math.log(s_range[1])))))
        a = float(rng.uniform(*a_range))
        cus = int(cu_choices[int(rng.integers(0, len(cu_choices)))])
        out.append((n, s, a, cus))
    return out


def cu_mask_words(cus: int, total: int, groups: int = 8) -> list:
    """CU mask (32 bits per word) selecting `cus` of `total` compute units
    spread evenly: the first cus/groups units of each of `groups` equal
    blocks of the CU numbering.  Whether the numbering runs block by block
    over the XCDs or round-robin across them, every XCD gets the same share."""
    if total % groups or cus % groups or not 0 < cus <= total:
        raise ValueError(f"cus ({cus}) and total ({total}) must be positive multiples of {groups}, cus <= total")
    per, take = total // groups, cus // groups
    words = [0] * ((total + 31) // 32)
    for g in range(groups):
        for j in range(take):
            b = g * per + j
            words[b // 32] |= 1 << (b % 32)
    return words


class CUMaskedStream:
    """A HIP stream restricted to `cus` compute units (default priority), as a
    torch external stream; destroyed on close()."""

    def __init__(self, cus: int, device="cuda:0"):
        self.dev = torch.device(device)
        total = torch.cuda.get_device_properties(self.dev).multi_processor_count
        words = cu_mask_words(cus, total)
        hip = ctypes.CDLL("libamdhip64.so")
        self._destroy = hip.hipStreamDestroy
        self._destroy.argtypes = [ctypes.c_void_p]
        create = hip.hipExtStreamCreateWithCUMask
        create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
        handle = ctypes.c_void_p()
        arr = (ctypes.c_uint32 * len(words))(*words)
        with torch.cuda.device(self.dev):
            rc = create(ctypes.byref(handle), len(words), arr)
        if rc != 0:
            raise RuntimeError(f"hipExtStreamCreateWithCUMask failed ({rc})")
        self.handle = handle.value
        self.stream = torch.cuda.ExternalStream(self.handle, device=self.dev)
        self.cus, self.total = cus, total

    def close(self):
        if self.handle:
            torch.cuda.synchronize(self.dev)
            self._destroy(ctypes.c_void_p(self.handle))
            self.handle = None


def slab_table(cfg) -> bool:
    """The predictor's classes: slab-kernel configurations with table weights
    and the default traversal."""
    return (int(cfg.variant) == recon.RECON_VARIANT_SLAB and int(cfg.weights) == recon.RECON_WEIGHTS_TABLE
            and int(cfg.traversal) == 0)


def time_space(n: int, slices: int, a: float, seed: int, batch_cap: int = CALL_SLICES, device="cuda:0",
               repeats: int = 3, cus: int | None = None, keep=slab_table) -> TuneRecord:
    """Times the configurations of the tuning space that `keep` accepts on one
    call of min(slices, batch_cap) synthetic slices (random complex samples,
    uniform orientations: the cost depends on the geometry, not the values),
    with the library's default batch size (so the work plan is the one it
    runs).  Each configuration: one warm-up call, then the median of
    `repeats` calls, each timed with events around the whole
    recon_insert_batch.  With `cus` below the device's CU count the insertion
    runs on a CU-masked stream with the library's cu_count set to match."""
    dev = torch.device(device)
    total = torch.cuda.get_device_properties(dev).multi_processor_count
    cus = total if cus is None else int(cus)
    masked = CUMaskedStream(cus, dev) if cus < total else None
    count = min(slices, batch_cap)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    h = n // 2
    sl = torch.randn((count, n, h + 1, 2), generator=g, device=dev, dtype=torch.float32)
    sl = torch.view_as_complex(sl).contiguous()
    q = torch.randn((count, 4), generator=g, device=dev, dtype=torch.float32)
    torch.cuda.synchronize(dev)
    stream = masked.stream if masked else torch.cuda.current_stream(dev)
    rec = recon.Reconstruction(n, device=dev, max_batch=max(count, CALL_SLICES), blob_radius=float(np.float32(a)),
                               stream=stream)
    if masked:
        rec.set_config(cu_count=cus)
    default_key = config_key(recon.recon_get_config(rec.ctx))
    size = recon.recon_tune_space_size(rec.ctx)
    ns, keys = [], []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for i in range(size):
        cfg = recon.recon_tune_space_config(rec.ctx, i)
        if keep is not None and not keep(cfg):
            continue
        keys.append(config_key(cfg))
        recon.recon_set_config(rec.ctx, cfg)
        recon.recon_insert_batch(rec.ctx, sl, None, q, count)       # warm-up
        t = []
        for _ in range(repeats):
            e0.record(stream)
            recon.recon_insert_batch(rec.ctx, sl, None, q, count)
            e1.record(stream)
            e1.synchronize()
            t.append(e0.elapsed_time(e1))
        ns.append(float(np.median(t)) * 1e6 / count)
    rec.close()
    if masked:
        masked.close()
    return TuneRecord(n=n, slices=slices, a=a, ns_per_slice=np.array(ns), keys=keys, default_key=default_key,
                      cus=cus, cus_total=total)


def soft_targets(ns: np.ndarray, temperature: float = 0.02) -> np.ndarray:
    """Target distribution over configurations: softmax of -(t / t_best) / T
    (configurations that do not run, t = +inf, get zero mass)."""
    r = -(ns / ns.min(axis=1, keepdims=True)) / temperature
    r -= r.max(axis=1, keepdims=True)
    e = np.exp(r)
    return e / e.sum(axis=1, keepdims=True)


class Normalizer:
    def __init__(self, X: np.ndarray):
        self.mu = X.mean(axis=0)
        self.sd = X.std(axis=0) + 1e-9

    def __call__(self, X: np.ndarray) -> np.ndarray:
        return (X - self.mu) / self.sd


class Predictor:
    """MLP features -> configuration scores, trained with the library's kernels."""

    def __init__(self, n_out: int, seed: int = 0, device="cuda:0", n_in: int = 4):
        self.dev = torch.device(device)
        self.n_in, self.H, self.C = n_in, N_HIDDEN, n_out
        rng = np.random.default_rng(seed)
        shapes = [(self.n_in, self.H), (self.H,), (self.H, self.H), (self.H,), (self.H, self.C), (self.C,)]
        parts = []
        for shp in shapes:
            if len(shp) == 2:
                lim = math.sqrt(6.0 / shp[0])
                parts.append(rng.uniform(-lim, lim, shp).ravel())
            else:
                parts.append(np.zeros(shp))
        self.params = torch.tensor(np.concatenate(parts), dtype=torch.float32, device=self.dev)
        self.norm = None

    def fit(self, X: np.ndarray, Y: np.ndarray, steps: int = 3000, lr: float = 0.1) -> list:
        self.norm = Normalizer(X)
        B = X.shape[0]
        x = torch.tensor(self.norm(X), dtype=torch.float32, device=self.dev)
        y = torch.tensor(Y, dtype=torch.float32, device=self.dev)
        _, wsb = recon.recon_mlp_sizes(self.n_in, self.H, self.C, B)
        ws = torch.empty(wsb, dtype=torch.uint8, device=self.dev)
        loss = torch.empty(steps, dtype=torch.float32, device=self.dev)
        for i in range(steps):
            recon.recon_mlp_train_step(self.params, self.n_in, self.H, self.C, x, y, B, lr, ws, loss[i:i + 1])
        return loss.cpu().numpy().tolist()

    def save(self, path: str, keys: list):
        """Parameters, feature normalisation and class keys, in one .npz."""
        np.savez(path, params=self.params.cpu().numpy(), mu=self.norm.mu, sd=self.norm.sd,
                 keys=np.array(keys, dtype=np.int64), n_in=self.n_in, n_out=self.C)

    def predict(self, X: np.ndarray) -> np.ndarray:
        B = X.shape[0]
        x = torch.tensor(self.norm(X), dtype=torch.float32, device=self.dev)
        _, wsb = recon.recon_mlp_sizes(self.n_in, self.H, self.C, B)
        ws = torch.empty(wsb, dtype=torch.uint8, device=self.dev)
        p = torch.empty((B, self.C), dtype=torch.float32, device=self.dev)
        recon.recon_mlp_forward(self.params, self.n_in, self.H, self.C, x, B, ws, p)
        return p.cpu().numpy()


def load_predictor(path: str, device="cuda:0"):
    """A predictor written by Predictor.save, and its class keys."""
    z = np.load(path)
    model = Predictor(int(z["n_out"]), device=device, n_in=int(z["n_in"]))
    model.params = torch.tensor(z["params"], dtype=torch.float32, device=model.dev)
    norm = Normalizer(np.zeros((1, model.n_in)))
    norm.mu, norm.sd = z["mu"], z["sd"]
    model.norm = norm
    return model, [_key(k) for k in z["keys"]]


def regret(ns: np.ndarray, choice: np.ndarray) -> np.ndarray:
    """Time of the chosen configuration over the fastest, minus one, per workload."""
    return ns[np.arange(ns.shape[0]), choice] / ns.min(axis=1) - 1.0


def random_search_regret(ns: np.ndarray, steps: int, trials: int = 200, seed: int = 0) -> np.ndarray:
    """Expected regret of the best of `steps` random runnable configurations
    (the paper's random search with a fixed budget), averaged over trials."""
    rng = np.random.default_rng(seed)
    W, _ = ns.shape
    out = np.zeros(W)
    for w in range(W):
        ok = np.flatnonzero(np.isfinite(ns[w]))
        for _ in range(trials):
            picks = rng.choice(ok, size=min(steps, ok.size), replace=False)
            out[w] += ns[w, picks].min() / ns[w, ok].min() - 1.0
    return out / trials


def ranked_candidates(prob: np.ndarray, runnable: np.ndarray, k: int) -> np.ndarray:
    """Indices of the k most probable runnable configurations, best first."""
    p = np.where(runnable, prob, -np.inf)
    order = np.argsort(-p, kind="stable")
    return order[:min(k, int(runnable.sum()))]


def guided_regret(ns: np.ndarray, prob: np.ndarray, k: int, default=None) -> np.ndarray:
    """Regret of measuring the predictor's top-k runnable configurations (and
    the default configuration default[w], when given) and keeping the
    fastest (k or k + 1 tuning steps)."""
    out = np.zeros(ns.shape[0])
    for w in range(ns.shape[0]):
        ok = np.isfinite(ns[w])
        cand = list(ranked_candidates(prob[w], ok, k))
        if default is not None and default[w] >= 0 and ok[default[w]]:
            cand.append(int(default[w]))
        out[w] = ns[w, cand].min() / ns[w, ok].min() - 1.0
    return out


def policy_regret(ns: np.ndarray, prob: np.ndarray, k: int, tau: float, budget: int, trials: int = 200,
                  seed: int = 0):
    """The run-time policy: if the top probability is at least tau, measure
    the top-k predicted configurations; otherwise fall back to a random search
    of `budget` steps.  Returns (regret per workload, steps per workload,
    fallback mask)."""
    conf = np.where(np.isfinite(ns), prob, -np.inf).max(axis=1)
    fallback = conf < tau
    reg = guided_regret(ns, prob, k)
    if fallback.any():
        reg[fallback] = random_search_regret(ns[fallback], budget, trials=trials, seed=seed)
    steps = np.where(fallback, budget, k)
    return reg, steps, fallback


def tune_with_predictor(rec, model, keys: list, features: np.ndarray, k: int = 3, tau: float = 0.05,
                        budget: int = 10, seed: int = 0, with_default: bool = True) -> dict:
    """Starts the library's tuner on a live reconstruction: the predictor's
    top-k runnable configurations in rank order, then the context's current
    (default) configuration if it is not among them, when the predictor is
    confident; else a random search of `budget` steps.  The caller then
    performs its recon_insert_batch calls (each tuning step is real work);
    `judge` reads the outcome afterwards."""
    size = recon.recon_tune_space_size(rec.ctx)
    space_keys = [config_key(recon.recon_tune_space_config(rec.ctx, i)) for i in range(size)]
    col = {kk: i for i, kk in enumerate(keys)}
    prob = model.predict(features.reshape(1, -1))[0]
    runnable = np.array([kk in col for kk in space_keys])
    p_space = np.array([prob[col[kk]] if kk in col else -np.inf for kk in space_keys])
    conf = float(p_space[runnable].max()) if runnable.any() else 0.0
    if conf >= tau:
        order = [int(i) for i in ranked_candidates(p_space, runnable, k)]
        dkey = config_key(recon.recon_get_config(rec.ctx))
        if with_default and dkey in space_keys and space_keys.index(dkey) not in order:
            order.append(space_keys.index(dkey))
        recon.recon_tune_begin(rec.ctx, order=order)
        return {"policy": "predicted", "order": order, "confidence": conf}
    recon.recon_tune_begin(rec.ctx, max_steps=budget, seed=seed)
    return {"policy": "random_search", "order": None, "confidence": conf}


def judge(rec, plan: dict) -> dict:
    """Outcome of a tuning run started by tune_with_predictor: the selected
    configuration and, for a predicted order, the measured regret of the
    top-1 prediction against the fastest measured candidate."""
    info = recon.recon_tune_get_info(rec.ctx)
    out = dict(plan, steps=int(info.steps_done), best_index=int(info.best_index),
               best_ns_per_slice=float(info.best_ns_per_slice), active=bool(info.active))
    if plan["order"] and info.steps_done >= 1:
        out["top1_is_best"] = plan["order"][0] == info.best_index
    return out


def evaluate(train: list, test: list, steps: int = 3000, lr: float = 0.1, temperature: float = 0.02,
             seed: int = 0, search_budget: int = 10) -> dict:
    """Trains on `train` records and reports regrets on `test` records."""
    keys = union_keys(train)
    Xtr = np.stack([r.features() for r in train])
    Ytr = soft_targets(time_matrix(train, keys), temperature)
    Xte = np.stack([r.features() for r in test])
    NSte = time_matrix(test, keys)
    model = Predictor(Ytr.shape[1], seed=seed, n_in=Xtr.shape[1])
    losses = model.fit(Xtr, Ytr, steps=steps, lr=lr)
    prob = model.predict(Xte)
    scores = np.where(np.isfinite(NSte), prob, -np.inf)    # only runnable choices
    pred = scores.argmax(axis=1)
    fin = np.where(np.isfinite(NSte), NSte, np.nan)
    col = {k: i for i, k in enumerate(keys)}
    dflt = np.array([col.get(r.default_key, -1) for r in test])
    out = {
        "train_workloads": len(train), "test_workloads": len(test), "configs": int(Ytr.shape[1]),
        "loss_first": losses[0], "loss_last": losses[-1],
        "regret_learned_mean": float(regret(NSte, pred).mean()),
        "regret_learned_max": float(regret(NSte, pred).max()),
        "regret_random_search_mean": float(random_search_regret(NSte, search_budget, seed=seed).mean()),
        "random_search_budget": search_budget,
        "mean_config_over_best": float((np.nanmean(fin, axis=1) / NSte.min(axis=1)).mean()),
        "regret_top3_mean": float(guided_regret(NSte, prob, 3).mean()),
        "regret_guided_mean": float(guided_regret(NSte, prob, 3, dflt).mean()),
        "regret_guided_max": float(guided_regret(NSte, prob, 3, dflt).max()),
        "regret_random_search3_mean": float(random_search_regret(NSte, 3, seed=seed).mean()),
        "regret_random_search4_mean": float(random_search_regret(NSte, 4, seed=seed).mean()),
    }
    conf = np.where(np.isfinite(NSte), prob, -np.inf).max(axis=1)
    out["confidence_quartiles"] = [float(x) for x in np.quantile(conf, [0.25, 0.5, 0.75])]
    out["policy"] = []
    for tau in (0.02, 0.05, 0.1, 0.2):
        reg, st, fb = policy_regret(NSte, prob, 3, tau, search_budget, seed=seed)
        out["policy"].append({"k": 3, "tau": tau, "fallback_budget": search_budget,
                              "regret_mean": float(reg.mean()), "regret_max": float(reg.max()),
                              "steps_mean": float(st.mean()), "fallback_fraction": float(fb.mean())})
    if all(d >= 0 and np.isfinite(NSte[w, d]) for w, d in enumerate(dflt)):
        out["regret_default_mean"] = float(regret(NSte, dflt).mean())
        out["regret_default_max"] = float(regret(NSte, dflt).max())
    return out, model, keys


def portability_matrix(records) -> np.ndarray:
    """Performance portability of tuned configurations: entry [x, y] is the
    fastest time on workload y over the time, on y, of the configuration
    tuned (fastest) on workload x (1 on the diagonal; nan where x's best does
    not run on y)."""
    keys = union_keys(records)
    ns = time_matrix(records, keys)
    best = ns.argmin(axis=1)
    out = np.empty((len(records), len(records)))
    for x in range(len(records)):
        for y in range(len(records)):
            t = ns[y, best[x]]
            out[x, y] = ns[y].min() / t if np.isfinite(t) else np.nan
    return out


def main(argv=None):
    import argparse
    import json
    import sys
    import time
    ap = argparse.ArgumentParser(description="collect tuning data, train and evaluate the learned predictor")
    ap.add_argument("--train", type=int, default=200)
    ap.add_argument("--test", type=int, default=50)
    ap.add_argument("--batch-cap", type=int, default=CALL_SLICES)
    ap.add_argument("--repeats", type=int, default=3, help="timed calls per configuration (median)")
    ap.add_argument("--save-model", default=None, help="write the trained predictor (.npz)")
    ap.add_argument("--n-max", type=int, default=384)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--out", default=None)
    ap.add_argument("--portability", action="store_true",
                    help="instead: tune at one box size (or CU count), run at another")
    ap.add_argument("--records-dir", default=None,
                    help="keep each workload's timings here (rec_<k>.npz) and reuse the ones present")
    ap.add_argument("--time-limit", type=float, default=0.0,
                    help="stop collecting after this many seconds (0: no limit); with --records-dir a "
                         "later run resumes")
    args = ap.parse_args(argv)
    t0 = time.time()
    if args.portability:
        res = {}
        boxes = (32, 50, 64, 90, 128)
        recs = [time_space(n, 1500, 1.9, seed=n, batch_cap=1500) for n in boxes]
        res["boxes"] = {"labels": list(boxes), "slices": 1500, "a": 1.9,
                        "matrix": np.round(portability_matrix(recs), 4).tolist()}
        cus = CU_CHOICES
        recs = [time_space(128, 1500, 1.9, seed=7, batch_cap=1500, cus=c) for c in cus]
        res["cus"] = {"labels": list(cus), "n": 128, "slices": 1500, "a": 1.9,
                      "matrix": np.round(portability_matrix(recs), 4).tolist()}
        res["collection_s"] = time.time() - t0
        print(json.dumps(res), flush=True)
        return 0
    records = []
    params = sample_workloads(1000, args.train, n_range=(48, args.n_max)) + \
        sample_workloads(2000, args.test, n_range=(48, args.n_max))
    import os
    if args.records_dir:
        os.makedirs(args.records_dir, exist_ok=True)
    for k, (n, s, a, cus) in enumerate(params):
        path = os.path.join(args.records_dir, f"rec_{k}.npz") if args.records_dir else None
        if path and os.path.exists(path):
            records.append(TuneRecord.load(path))
            continue
        if args.time_limit > 0 and time.time() - t0 > args.time_limit:
            print(f"learned: time limit reached after {k} workloads; run again to resume", file=sys.stderr,
                  flush=True)
            return 3
        records.append(time_space(n, s, a, seed=k, batch_cap=args.batch_cap, cus=cus, repeats=args.repeats))
        if path:
            records[-1].save(path)
        print(f"learned: workload {k + 1}/{len(params)} n={n} S={s} a={a:.2f} CUs={cus} "
              f"best {records[-1].ns_per_slice.min():.1f} ns/slice ({time.time() - t0:.0f} s)",
              file=sys.stderr, flush=True)
    res, model, keys = evaluate(records[:args.train], records[args.train:], steps=args.steps)
    res["collection_s"] = time.time() - t0
    res["batch_cap"] = args.batch_cap
    res["repeats"] = args.repeats
    if args.save_model:
        model.save(args.save_model, keys)
    print(json.dumps(res), flush=True)
    if args.out:
        keys = union_keys(records)
        col = {k: i for i, k in enumerate(keys)}
        np.savez(args.out, features=np.stack([r.features() for r in records]),
                 ns=time_matrix(records, keys), keys=np.array(keys), n_train=args.train,
                 default_index=np.array([col.get(r.default_key, -1) for r in records]))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
