"""Batched insertion: several reconstructions of different box sizes in one
persistent launch must equal their FP64 oracles, and the batch insert must
replay correctly from a captured HIP graph."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_08498_amd import recon
    return torch, torch.device("cuda:0"), recon


def make_jobs(torch, dev, recon, specs, stream):
    jobs = []
    for k, (n, S) in enumerate(specs):
        w = synth.make_workload("small", n=n, S=S, K=6, seed_phantom=50 + k, seed_orient=60 + k)
        rec = recon.Reconstruction(n, device=dev, stream=stream, max_batch=max(S, 1))
        jobs.append((w, rec, torch.from_numpy(w.slices).to(dev), torch.from_numpy(w.quats).to(dev)))
    return jobs


# the second case puts a box above 256 in the launch, so every box of it is
# inserted with the slab kernel's exact geometry
@pytest.mark.parametrize("specs", [[(32, 70), (48, 40), (20, 90), (64, 25), (34, 0)],
                                   [(32, 70), (272, 30), (48, 40)]], ids=["small", "with_large_box"])
def test_batch_matches_oracle_per_reconstruction(env, specs):
    torch, dev, recon = env
    stream = torch.cuda.current_stream()
    jobs = make_jobs(torch, dev, recon, specs, stream)
    ctxs = [j[1].ctx for j in jobs]
    ws = torch.empty(recon.recon_batch_query_size(ctxs), dtype=torch.uint8, device=dev)
    b = recon.recon_batch_create(ctxs, ws)
    print(f"[gpu] batch of {len(jobs)} reconstructions {specs}", flush=True)
    recon.recon_batch_insert(b, [j[2] for j in jobs], None, [j[3] for j in jobs], [S for _, S in specs])
    for w, rec, _, _ in jobs:
        V = rec.finalize()
        torch.cuda.synchronize()
        if w.S == 0:
            assert float(rec.W.abs().sum()) == 0.0
            continue
        G, W, U = oracle.insert(w.n, w.slices, w.quats)
        eg = oracle.rel_l2(rec.G.cpu().numpy(), G)
        ew = oracle.rel_l2(rec.W.cpu().numpy(), W)
        ev = oracle.rel_l2(V.cpu().numpy(), oracle.finalize(G, W))
        print(f"   n={w.n} S={w.S}: G={eg:.2e} W={ew:.2e} V={ev:.2e}", flush=True)
        assert max(eg, ew, ev) <= 1e-5
        assert rec.stats() == (w.S, 0)
    recon.recon_batch_destroy(b)
    for j in jobs:
        j[1].close()


def test_batch_rejects_mismatched_blobs(env):
    torch, dev, recon = env
    a = recon.Reconstruction(16, device=dev)
    c = recon.Reconstruction(16, device=dev, blob_radius=1.5)
    with pytest.raises(recon.ReconError):
        recon.recon_batch_query_size([a.ctx, c.ctx])
    with pytest.raises(recon.ReconError):
        recon.recon_batch_query_size([a.ctx, a.ctx])
    a.close()
    c.close()


def test_batch_insert_replays_from_graph(env):
    torch, dev, recon = env
    specs = [(32, 30), (24, 50)]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        jobs = make_jobs(torch, dev, recon, specs, side)
    torch.cuda.synchronize()
    ctxs = [j[1].ctx for j in jobs]
    ws = torch.empty(recon.recon_batch_query_size(ctxs), dtype=torch.uint8, device=dev)
    b = recon.recon_batch_create(ctxs, ws)
    args = ([j[2] for j in jobs], None, [j[3] for j in jobs], [S for _, S in specs])
    # eager reference: one batch insert
    recon.recon_batch_insert(b, *args)
    side.synchronize()
    ref = [(j[1].G.clone(), j[1].W.clone()) for j in jobs]
    for j in jobs:
        j[1].reset()
    side.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        recon.recon_batch_insert(b, *args)
    side.synchronize()
    for r in range(1, 4):
        graph.replay()
        torch.cuda.synchronize()
        for (G0, W0), j in zip(ref, jobs):
            # r replays accumulate r copies of the batch (same order of sums up to rounding)
            assert float((j[1].W - r * W0).abs().max()) <= 1e-4 * r * float(W0.abs().max())
            assert float((j[1].G - r * G0).abs().max()) <= 1e-4 * r * float(G0.abs().max())
        _ = torch.ones(1000, device=dev).sum().item()   # eager work between replays
    recon.recon_batch_destroy(b)
    for j in jobs:
        j[1].close()


def test_batch_rounds_with_reconstructions_that_run_out(env):
    """Several batched rounds where the reconstructions run out of slices at
    different rounds: a job with no slices in a round is skipped by the
    launch (its items and partial sums), and what it already holds must
    stay, so each reconstruction still equals its oracle."""
    torch, dev, recon = env
    stream = torch.cuda.current_stream()
    specs = [(40, 120), (32, 30), (48, 75)]
    per = 50
    jobs = []
    for k, (n, S) in enumerate(specs):
        w = synth.make_workload("small", n=n, S=S, K=6, seed_phantom=110 + k, seed_orient=120 + k)
        rec = recon.Reconstruction(n, device=dev, stream=stream, max_batch=per)
        rec.set_config(split=64)      # many split tiles, so partial sums are in play
        jobs.append((w, rec, torch.from_numpy(w.slices).to(dev), torch.from_numpy(w.quats).to(dev)))
    ctxs = [j[1].ctx for j in jobs]
    ws = torch.empty(recon.recon_batch_query_size(ctxs), dtype=torch.uint8, device=dev)
    b = recon.recon_batch_create(ctxs, ws)
    rounds = max((S + per - 1) // per for _, S in specs)
    print(f"[gpu] batch rounds {rounds} over {specs}, {per} slices per round", flush=True)
    for r in range(rounds):
        sls, qts, cnt = [], [], []
        for w, _, sl, q in jobs:
            s0, s1 = min(w.S, r * per), min(w.S, (r + 1) * per)
            sls.append(sl[s0:s1] if s1 > s0 else None)
            qts.append(q[s0:s1] if s1 > s0 else None)
            cnt.append(s1 - s0)
        recon.recon_batch_insert(b, sls, None, qts, cnt)
    for w, rec, _, _ in jobs:
        V = rec.finalize()
        torch.cuda.synchronize()
        G, W, U = oracle.insert(w.n, w.slices, w.quats)
        eg = oracle.rel_l2(rec.G.cpu().numpy(), G)
        ew = oracle.rel_l2(rec.W.cpu().numpy(), W)
        ev = oracle.rel_l2(V.cpu().numpy(), oracle.finalize(G, W))
        print(f"   n={w.n} S={w.S}: G={eg:.2e} W={ew:.2e} V={ev:.2e}", flush=True)
        assert max(eg, ew, ev) <= 1e-5
        assert rec.stats() == (w.S, 0)
    recon.recon_batch_destroy(b)
    for j in jobs:
        j[1].close()
