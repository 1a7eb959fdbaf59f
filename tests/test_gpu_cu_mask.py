"""Insertion on a stream restricted to a subset of the compute units
(hipExtStreamCreateWithCUMask) with the library's cu_count set to match:
the persistent kernels run one work-group per allowed CU, and the result is
bitwise the same as on the whole device (every voxel has one writer and the
partial sums are reduced in a fixed order).  Also the tuner's candidate
order: exactly the given configurations are measured, in that order, and the
fastest of them is kept."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_08498_amd import learned, recon
    return torch, torch.device("cuda:0"), recon, learned


@pytest.fixture(scope="module")
def workload():
    return synth.make_workload("small", n=64, S=300, K=10, seed_phantom=31, seed_orient=32)


def run(torch, dev, recon, w, stream=None, **cfg):
    rec = recon.Reconstruction(w.n, device=dev, stream=stream)
    if cfg:
        rec.set_config(**cfg)
    sl = torch.from_numpy(w.slices).to(dev)
    qt = torch.from_numpy(w.quats).to(dev)
    torch.cuda.synchronize()
    rec.insert(sl, qt)
    V = rec.finalize()
    torch.cuda.synchronize()
    out = (rec.G.cpu().numpy(), rec.W.cpu().numpy(), V.cpu().numpy(), rec.stats())
    rec.close()
    return out


@pytest.mark.parametrize("cus", [64, 128])
@pytest.mark.parametrize("variant", ["slab", "binned"])
def test_cu_masked_stream_gives_identical_volumes(env, workload, cus, variant):
    torch, dev, recon, learned = env
    v = {"slab": recon.RECON_VARIANT_SLAB, "binned": recon.RECON_VARIANT_BINNED}[variant]
    print(f"[gpu] cu mask: {cus} CUs, variant {variant}", flush=True)
    ref = run(torch, dev, recon, workload, variant=v, waves_per_block=0, slab_flags=0)
    ms = learned.CUMaskedStream(cus, dev)
    try:
        got = run(torch, dev, recon, workload, stream=ms.stream, variant=v, waves_per_block=0, slab_flags=0,
                  cu_count=cus)
    finally:
        ms.close()
    for a, b in zip(ref[:3], got[:3]):
        assert np.array_equal(a, b)
    assert got[3] == (workload.S, 0)


def test_cu_count_out_of_range_rejected(env):
    torch, dev, recon, learned = env
    rec = recon.Reconstruction(16, device=dev)
    total = torch.cuda.get_device_properties(dev).multi_processor_count
    for bad in (-1, total + 1):
        with pytest.raises(recon.ReconError) as ei:
            rec.set_config(cu_count=bad)
        assert ei.value.status == recon.RECON_ECONFIG
    rec.close()


def test_tuner_follows_a_candidate_order(env, workload):
    torch, dev, recon, learned = env
    w = workload
    rec = recon.Reconstruction(w.n, device=dev, max_batch=100)
    size = recon.recon_tune_space_size(rec.ctx)
    order = [size - 1, 0, size // 2]
    keys = [learned.config_key(recon.recon_tune_space_config(rec.ctx, i)) for i in order]
    recon.recon_tune_begin(rec.ctx, order=order)
    sl = torch.from_numpy(w.slices).to(dev)
    qt = torch.from_numpy(w.quats).to(dev)
    seen = []
    for b in range(3):
        # each call runs (and times) the next candidate
        recon.recon_insert_batch(rec.ctx, sl[100 * b:100 * b + 100], None, qt[100 * b:100 * b + 100], 100)
        seen.append(learned.config_key(recon.recon_get_config(rec.ctx)))
    info = recon.recon_tune_get_info(rec.ctx)
    assert info.steps_done == 3
    recon.recon_tune_end(rec.ctx)               # selects the fastest of the three
    info = recon.recon_tune_get_info(rec.ctx)
    assert not info.active and info.steps_done == 3
    assert info.best_index in order
    assert learned.config_key(recon.recon_get_config(rec.ctx)) == keys[order.index(info.best_index)]
    assert seen == keys                        # measured exactly these, in this order
    for bad in ([size], [0, 0], []):
        with pytest.raises(recon.ReconError):
            recon.recon_tune_begin(rec.ctx, order=bad)
    rec.close()
