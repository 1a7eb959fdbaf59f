"""Comparison helpers shared by the GPU parity tests (no GPU code here).

rel_l2 over the whole box (the parity metric) and the per-voxel diagnostic:
over the voxels that received a sizeable weight (W_o >= 1e-3 max W_o), the
largest relative error of W and of V = G / W.  V's relative error is taken
only where |V_o| is not tiny against the largest |V_o| of that set, since V
passes through zero (the transform of the phantom does) and a relative error
there says nothing about the arithmetic.
"""
from __future__ import annotations

import numpy as np

import oracle

W_FRAC = 1e-3       # voxels with W_o >= W_FRAC * max W_o
V_FRAC = 1e-3       # ... and, for V, |V_o| >= V_FRAC * max |V_o| over them


def errors(G, W, V, Go, Wo, Vo) -> dict:
    """rel-L2 of G, W, V and the per-voxel maxima (see module text)."""
    out = {"G": oracle.rel_l2(G, Go), "W": oracle.rel_l2(W, Wo), "V": oracle.rel_l2(V, Vo)}
    Wo = np.asarray(Wo, dtype=np.float64)
    sel = Wo >= W_FRAC * Wo.max() if Wo.size and Wo.max() > 0 else np.zeros(Wo.shape, bool)
    if sel.any():
        w_rel = np.abs(np.asarray(W, np.float64)[sel] - Wo[sel]) / Wo[sel]
        vo = np.asarray(Vo, np.complex128)[sel]
        dv = np.abs(np.asarray(V, np.complex128)[sel] - vo)
        big = np.abs(vo) >= V_FRAC * np.abs(vo).max()
        out["W_max_rel"] = float(w_rel.max())
        out["V_max_rel"] = float((dv[big] / np.abs(vo[big])).max()) if big.any() else 0.0
        out["voxels"] = int(sel.sum())
    else:
        out["W_max_rel"] = out["V_max_rel"] = 0.0
        out["voxels"] = 0
    return out


def fmt(e: dict) -> str:
    return (f"rel-L2 G={e['G']:.2e} W={e['W']:.2e} V={e['V']:.2e}; per voxel (W >= 1e-3 max W, "
            f"{e['voxels']} voxels) max |dW|/W={e['W_max_rel']:.2e} max |dV|/|V|={e['V_max_rel']:.2e}")


def cutoff_flips(W, Wo, edge: float):
    """Voxels whose W differs from the oracle by whole blob-edge samples.

    A sample within FP32 rounding of the inclusive cut-off d^2 = a^2 may be
    taken or left out unlike the FP64 oracle; it then moves W at one voxel by
    b(a^2) (and G by b(a^2) F).  Returns the boolean mask of the voxels whose
    difference is an integer number k >= 1 of edge weights, up to 1 % of an
    edge weight plus the FP32 accumulation error allowed at that voxel
    (1e-5 W); every other voxel stays in the comparison.  With an edge weight
    too small to see (<= 1e-4) no voxel is masked."""
    W = np.asarray(W, np.float64)
    Wo = np.asarray(Wo, np.float64)
    if edge <= 1e-4:
        return np.zeros(W.shape, bool)
    dW = np.abs(W - Wo)
    noise = 1e-5 * np.abs(Wo)
    k = np.rint(dW / edge)
    return (k >= 1) & (dW > 0.5 * edge + noise) & (np.abs(dW - k * edge) <= 0.01 * edge + noise)


def flip_limit(U: int, n: int, a: float) -> float:
    """Most cut-off flips consistent with FP32 geometry, for U pairs in a box n.

    A voxel position relative to a rotated sample carries an FP32 error of a
    few units in the last place of the largest coordinate h = n/2 (taken as 8
    ulp), so d^2 near a^2 is uncertain by delta = 2 a * 8 h 2^-23.  With the
    pair offsets spread uniformly over the blob's ball, P(d^2 <= x) =
    (x / a^2)^(3/2), so a share of about 3 delta / a^2 of the pairs lies within
    delta of the cut-off; each flipped voxel needs at least one such pair.
    The limit is four times that expectation (and at least one voxel)."""
    delta = 2.0 * a * 8.0 * max(n // 2, 1) * 2.0 ** -23
    return max(1.0, 4.0 * 3.0 * delta / (a * a) * U)


def progress(request, msg: str) -> None:
    """Prints past pytest's output capture, so a long CPU step (the oracle
    over a large workload) reports as it goes."""
    capman = request.config.pluginmanager.getplugin("capturemanager")
    if capman is None:
        print(msg, flush=True)
        return
    with capman.global_and_fixture_disabled():
        print(msg, flush=True)


def oracle_insert_chunked(request, n, slices, quats, chunk=2500, **kw):
    """oracle.insert over the slices in chunks, summed (G and W are sums over
    slices), with a progress line per chunk."""
    G = W = None
    U = 0
    S = len(quats)
    for s0 in range(0, S, chunk):
        g, w, u = oracle.insert(n, slices[s0:s0 + chunk], quats[s0:s0 + chunk], **kw)
        if G is None:
            G, W = g, w
        else:
            G += g
            W += w
        U += u
        progress(request, f"[cpu] oracle: {min(s0 + chunk, S)} of {S} slices")
    return G, W, U
