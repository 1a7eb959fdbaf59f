"""Interpolation weights evaluated on the fly (the paper's alternative to
precomputed weights, Sect. 4.2 "3D Fourier Reconstruction"): every variant
against the FP64 oracle's exact blob (power series of I_m, no table), for
several blobs, with no table at all (table_size = 0) and as a configuration
of a context that also has a table; the exact-geometry path of large boxes;
and the benchmark workload on sampled voxels."""
import numpy as np
import pytest

import oracle
import synth
from parity_util import cutoff_flips, errors, flip_limit, fmt

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_08498_amd import recon
    return torch, torch.device("cuda:0"), recon


def run(env, w, variant, weights, **params):
    torch, dev, recon = env
    print(f"[gpu] on-the-fly n={w.n} S={w.S} variant={variant} weights={weights} params={params}", flush=True)
    rec = recon.Reconstruction(w.n, device=dev, **params)
    # 0: the library's default for the variant and weight source (set_config
    # starts from the current configuration, which follows the table)
    rec.set_config(variant={"naive": 1, "binned": 2, "slab": 3}[variant], waves_per_block=0, slab_flags=0,
                   inner_chunk=0, split=0, weights=weights)
    rec.insert(torch.from_numpy(w.slices).to(dev), torch.from_numpy(w.quats).to(dev))
    V = rec.finalize()
    torch.cuda.synchronize()
    cfg = rec.config()
    out = rec.G.cpu().numpy(), rec.W.cpu().numpy(), V.cpu().numpy()
    rec.close()
    assert cfg["weights"] == 2
    return out


def check(gpu, w, blob, r_max=None):
    Go, Wo, U = oracle.insert(w.n, w.slices, w.quats, blob=blob, r_max=r_max)
    Vo = oracle.finalize(Go, Wo)
    G, W, V = gpu
    flip = cutoff_flips(W, Wo, oracle.blob_values([blob.a ** 2], blob)[0])
    assert flip.sum() <= flip_limit(U, w.n, blob.a)
    k = ~flip
    e = errors(G[k], W[k], V[k], Go[k], Wo[k], Vo[k])
    print(f"   {int(flip.sum())} cut-off flips; " + fmt(e), flush=True)
    assert e["G"] <= TOL and e["W"] <= TOL and e["V"] <= TOL


@pytest.mark.parametrize("variant", ["naive", "binned", "slab"])
@pytest.mark.parametrize("a,alpha,m,r_max", [
    (1.9, 15.0, 0, None), (2.5, 40.0, 2, None), (1.2, 8.0, 1, None), (2.95, 0.0, 0, None),
    (1.6, 10.0, 0, 13.0), (2.2, 60.0, 4, None),
])
def test_on_the_fly_without_table(env, variant, a, alpha, m, r_max):
    w = synth.make_workload("small", n=32, S=90, K=6, seed_phantom=51, seed_orient=52)
    params = dict(blob_radius=a, blob_alpha=alpha, blob_order=m, table_size=0, max_batch=64)
    if r_max is not None:
        params["r_max"] = r_max
    gpu = run(env, w, variant, 0, **params)
    check(gpu, w, oracle.Blob(a=float(np.float32(a)), alpha=alpha, m=m, N=0), r_max)


def test_on_the_fly_as_a_configuration_of_a_table_context(env):
    # a context with the default table, switched to on-the-fly weights, gives
    # bit for bit what a context without a table gives, and both stay within
    # the table's own error (6e-8 per weight) of the table result
    torch, dev, recon = env
    w = synth.make_workload("small", n=48, S=200, K=8, seed_phantom=53, seed_orient=54)
    a = run(env, w, "slab", 2)
    b = run(env, w, "slab", 0, table_size=0)
    assert all(np.array_equal(x.view(np.uint32), y.view(np.uint32)) for x, y in zip(a, b))
    check(a, w, oracle.Blob(N=0))
    rec = recon.Reconstruction(w.n, device=dev)
    rec.insert(torch.from_numpy(w.slices).to(dev), torch.from_numpy(w.quats).to(dev))
    rec.finalize()          # the x < 0 half, as in the runs above
    torch.cuda.synchronize()
    Wt = rec.W.cpu().numpy()
    rec.close()
    assert oracle.rel_l2(a[1], Wt) <= 2e-6


def test_on_the_fly_exact_geometry_box(env):
    # h = 150 > 67.4 a: the slab kernel's exact window geometry
    w = synth.make_workload("small", n=300, S=24, K=6, seed_phantom=55, seed_orient=56)
    gpu = run(env, w, "slab", 0, table_size=0, max_batch=16)
    check(gpu, w, oracle.Blob(N=0))


def test_on_the_fly_paper_scale_sampled(env):
    torch, dev, recon = env
    w = synth.make_workload("paper")
    G, W, V = run(env, w, "slab", 0, table_size=0)
    h = w.n // 2
    rng = np.random.default_rng(57)
    vox = np.concatenate([rng.integers(-h, h + 1, size=(1200, 3)), rng.integers(-4, 5, size=(100, 3))])
    Gv, Wv, _ = oracle.voxels(w.n, w.slices, w.quats, vox, blob=oracle.Blob(N=0), nthreads=16)
    idx = (vox[:, 2] + h, vox[:, 1] + h, vox[:, 0] + h)
    e = [oracle.rel_l2(G[idx], Gv), oracle.rel_l2(W[idx], Wv), oracle.rel_l2(V[idx], oracle.finalize(Gv, Wv))]
    print(f"   sampled rel-L2 G={e[0]:.2e} W={e[1]:.2e} V={e[2]:.2e}", flush=True)
    assert max(e) <= TOL
