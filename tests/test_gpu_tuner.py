"""Dynamic (non-blocking) autotuning on the GPU: every tuning step inserts
real slices with a different kernel configuration, so the reconstruction
must still match the FP64 oracle; the search then keeps the fastest."""
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


def test_tuning_space_is_runnable(env):
    torch, dev, recon = env
    rec = recon.Reconstruction(32, device=dev)
    n = recon.recon_tune_space_size(rec.ctx)
    assert n >= 100
    seen = set()
    for i in range(n):
        c = recon.recon_tune_space_config(rec.ctx, i)
        recon.recon_set_config(rec.ctx, c)      # every member is accepted
        seen.add((c.variant, c.waves_per_block, c.inner_chunk, c.split, c.slab_flags, c.weights, c.traversal))
    assert len(seen) == n
    with pytest.raises(recon.ReconError):
        recon.recon_tune_space_config(rec.ctx, n)
    rec.close()


def test_full_search_keeps_parity_and_selects_best(env):
    torch, dev, recon = env
    rec = recon.Reconstruction(32, device=dev, max_batch=2)
    size = recon.recon_tune_space_size(rec.ctx)
    # one tuning step per call of 2 slices: enough calls to visit the whole space
    w = synth.make_workload("small", n=32, S=2 * (size + 12), K=6, seed_phantom=31, seed_orient=32)
    print(f"[gpu] tuner: space {size}, {w.S} slices in batches of 2", flush=True)
    recon.recon_tune_begin(rec.ctx, max_steps=0, seed=7)
    rec.insert(torch.from_numpy(w.slices).to(dev), torch.from_numpy(w.quats).to(dev))
    V = rec.finalize()
    info = recon.recon_tune_get_info(rec.ctx)
    torch.cuda.synchronize()
    assert info.active == 0 and info.steps_done == size
    assert 0 <= info.best_index < size
    assert 0 < info.best_ns_per_slice <= info.mean_ns_per_slice
    cur = recon.recon_get_config(rec.ctx)
    key = ("variant", "waves_per_block", "inner_chunk", "split", "slab_flags", "weights", "traversal")
    assert [getattr(cur, k) for k in key] == [getattr(info.best, k) for k in key]
    G, W, U = oracle.insert(w.n, w.slices, w.quats)
    Vo = oracle.finalize(G, W)
    eg = oracle.rel_l2(rec.G.cpu().numpy(), G)
    ew = oracle.rel_l2(rec.W.cpu().numpy(), W)
    ev = oracle.rel_l2(V.cpu().numpy(), Vo)
    print(f"   rel-L2 G={eg:.2e} W={ew:.2e} V={ev:.2e}", flush=True)
    assert max(eg, ew, ev) <= 1e-5
    rec.close()


def test_bounded_search_and_early_end(env):
    torch, dev, recon = env
    w = synth.make_workload("small", n=32, S=40, K=4, seed_phantom=33, seed_orient=34)
    rec = recon.Reconstruction(w.n, device=dev, max_batch=4)
    recon.recon_tune_begin(rec.ctx, max_steps=5, seed=1)
    sl, qt = torch.from_numpy(w.slices).to(dev), torch.from_numpy(w.quats).to(dev)
    rec.insert(sl[:12], qt[:12])       # three steps
    info = recon.recon_tune_get_info(rec.ctx)
    assert info.active == 1 and info.steps_done == 3
    recon.recon_tune_end(rec.ctx)
    info = recon.recon_tune_get_info(rec.ctx)
    assert info.active == 0 and info.steps_done == 3
    rec.insert(sl[12:], qt[12:])
    rec.finalize()                     # fills the x < 0 half of G and W
    torch.cuda.synchronize()
    G, W, U = oracle.insert(w.n, w.slices, w.quats)
    assert oracle.rel_l2(rec.G.cpu().numpy(), G) <= 1e-5
    assert oracle.rel_l2(rec.W.cpu().numpy(), W) <= 1e-5
    rec.close()
