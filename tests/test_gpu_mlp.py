"""The learned predictor's HIP kernels against the FP64 reference (oracle/mlp.py):
probabilities, loss and every gradient, and a training trajectory."""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_08498_amd import recon
    return torch, torch.device("cuda:0"), recon


def flat(params):
    return np.concatenate([params[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def unflat(v, n_in, H, C):
    out, o = {}, 0
    for k, shp in (("W1", (n_in, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, C)), ("b3", (C,))):
        n = int(np.prod(shp))
        out[k] = v[o:o + n].reshape(shp)
        o += n
    return out


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("B,n_in,H,C", [(1, 4, 64, 2), (37, 4, 64, 129), (200, 4, 64, 129), (5, 7, 33, 17)])
def test_forward_loss_and_gradients_match_reference(env, B, n_in, H, C):
    torch, dev, recon = env
    rng = np.random.default_rng(B + C)
    params = mlp.init_params(rng, n_in, H, C)
    for k in ("b1", "b2", "b3"):
        params[k] = rng.normal(0, 0.1, params[k].shape)
    x = rng.normal(size=(B, n_in))
    y = rng.dirichlet(np.ones(C), size=B)
    npar, wsb = recon.recon_mlp_sizes(n_in, H, C, B)
    assert npar == flat(params).size
    tp = torch.tensor(flat(params), dtype=torch.float32, device=dev)
    tx = torch.tensor(x, dtype=torch.float32, device=dev)
    ty = torch.tensor(y, dtype=torch.float32, device=dev)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    probs = torch.empty((B, C), dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    grads = torch.empty(npar, dtype=torch.float32, device=dev)
    print(f"[gpu] mlp B={B} n_in={n_in} H={H} C={C}", flush=True)
    recon.recon_mlp_forward(tp, n_in, H, C, tx, B, ws, probs)
    recon.recon_mlp_train_step(tp, n_in, H, C, tx, ty, B, 0.0, ws, loss, grads)
    torch.cuda.synchronize()
    # the reference runs on the same FP32-rounded inputs
    p32 = {k: v.astype(np.float32).astype(np.float64) for k, v in params.items()}
    x32 = x.astype(np.float32).astype(np.float64)
    y32 = y.astype(np.float32).astype(np.float64)
    p_ref, _ = mlp.forward(p32, x32)
    g_ref = mlp.backward(p32, x32, y32)
    assert rel(probs.cpu().numpy(), p_ref) < 1e-5
    assert abs(float(loss.cpu()[0]) - mlp.loss(p32, x32, y32)) < 1e-5 * max(1.0, mlp.loss(p32, x32, y32))
    g = unflat(grads.cpu().numpy().astype(np.float64), n_in, H, C)
    for k in g:
        assert rel(g[k], g_ref[k]) < 1e-4, k
    # lr = 0 leaves the parameters unchanged
    assert np.array_equal(tp.cpu().numpy(), flat(params).astype(np.float32))


def test_training_follows_reference_trajectory(env):
    torch, dev, recon = env
    rng = np.random.default_rng(9)
    B, n_in, H, C = 64, 4, 64, 12
    params = mlp.init_params(rng, n_in, H, C)
    x = rng.normal(size=(B, n_in))
    y = np.eye(C)[rng.integers(0, C, B)]
    npar, wsb = recon.recon_mlp_sizes(n_in, H, C, B)
    tp = torch.tensor(flat(params), dtype=torch.float32, device=dev)
    tx = torch.tensor(x, dtype=torch.float32, device=dev)
    ty = torch.tensor(y, dtype=torch.float32, device=dev)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ref = {k: v.astype(np.float32).astype(np.float64) for k, v in params.items()}
    xr, losses = x.astype(np.float32).astype(np.float64), []
    for step in range(60):
        recon.recon_mlp_train_step(tp, n_in, H, C, tx, ty, B, 0.2, ws, loss)
        losses.append(float(loss.cpu()[0]))
        ref = mlp.sgd_step(ref, mlp.backward(ref, xr, y), 0.2)
    torch.cuda.synchronize()
    assert losses[-1] < 0.5 * losses[0]
    assert rel(tp.cpu().numpy().astype(np.float64), flat(ref)) < 1e-3
