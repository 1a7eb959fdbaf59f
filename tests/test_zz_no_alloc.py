"""The allocation-free entry point recon_init_static (the workspace in the
library's static device array) against recon_init with a caller workspace:
the same kernels on the same inputs give bit-identical G, W and V, on two
contexts in a row (the second with a smaller box and fewer slices, so the
array still holds the first's contents), and the array belongs to one live
context per device at a time."""
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


def run(env, w, static, **params):
    torch, dev, recon = env
    print(f"[gpu] n={w.n} S={w.S} static_workspace={static} params={params}", flush=True)
    rec = recon.Reconstruction(w.n, device=dev, static_workspace=static, **params)
    assert (rec.ws is None) == static
    rec.insert(torch.from_numpy(w.slices).to(dev), torch.from_numpy(w.quats).to(dev))
    V = rec.finalize()
    torch.cuda.synchronize()
    out = rec.G.cpu().numpy(), rec.W.cpu().numpy(), V.cpu().numpy(), rec.stats(), rec.config()
    rec.close()
    return out


def check_same(a, b):
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
    assert a[3] == b[3] and a[4] == b[4]


def test_static_workspace_matches_caller_workspace_twice(env):
    big = synth.make_workload("small", n=64, S=700, K=10, seed_phantom=61, seed_orient=62)
    small = synth.make_workload("small", n=24, S=90, K=5, seed_phantom=63, seed_orient=64)
    for w, params in ((big, dict(max_batch=256)), (small, dict(max_batch=64))):
        s = run(env, w, True, **params)
        c = run(env, w, False, **params)
        check_same(s, c)
        Go, Wo, _ = oracle.insert(w.n, w.slices, w.quats)
        Vo = oracle.finalize(Go, Wo)
        e = [oracle.rel_l2(s[0], Go), oracle.rel_l2(s[1], Wo), oracle.rel_l2(s[2], Vo)]
        print(f"   rel-L2 vs FP64 oracle G={e[0]:.2e} W={e[1]:.2e} V={e[2]:.2e}", flush=True)
        assert max(e) <= 1e-5


def test_static_workspace_has_one_owner_per_device(env):
    torch, dev, recon = env
    a = recon.Reconstruction(16, device=dev, static_workspace=True)
    with pytest.raises(recon.ReconError) as ei:
        recon.Reconstruction(16, device=dev, static_workspace=True)
    assert ei.value.status == recon.RECON_EINVAL
    a.close()
    b = recon.Reconstruction(16, device=dev, static_workspace=True)   # released by the destroy
    b.close()
