"""fp64 reference of the surrogate network (test infrastructure only).

The learned surrogate maps the parameters of one ring walk (SU(2) coin
angles, start coin state, T/N) to its position distribution in 512 symmetric
bins.  This module is the plain, slow definition of that network in float64
numpy, used to check the GPU forward pass, loss and gradients; it shares no
code with the HIP path.  The parameters are passed in as a dict of arrays (the
GPU's bf16-rounded weights when comparing with it).

Network (input F = 32 features, zero-padded; T = steps of the walk):
    h1 = relu(x W1^T + b1)          W1: 512 x 32
    h2 = relu(h1 W2^T + b2)         W2: 1024 x 512
    h3 = relu(h2 W3^T + b3)         W3: 1024 x 1024
    z4 = h3 W4^T + b4               W4: 1024 x 1024, read as 2 channels x 512 positions
    l[i] = cb + sum_c sum_j cw[c, j] z4[c, i + j - 4]   (1D conv, 9 taps, zero padding)
    q = softmax(l)                  a density over 512 cells of the scaled coordinate
    p = R(T) q                      the 512 position bins
The walk after T steps lives on the sites x0 - T + 2k, k = 0..T.  Cell j of q
covers k in [j (T+1)/512, (j+1)(T+1)/512) (site k is the unit interval
[k, k+1)), its mass spread uniformly over that interval; R(T) hands each site's
share to the bin that holds it (the binning of the ring distributions: bins of
w = 8 sites, the start site half to each of the two middle bins).
Loss: mean over the batch of KL(y || p) = sum_b y_b (log y_b - log p_b), with
0 log 0 = 0.

bf16=True rounds, as a bf16 matrix-core pipeline with fp32 accumulation must,
the operands of every matrix product to bfloat16 (round to nearest even of
their fp32 value): the hidden activations h1, h2, h3 that feed the next layer,
and in the backward pass each layer's dZ where it enters the two products
dZ^T H and dZ W (the bias gradients sum the unrounded dZ).  The inputs and the
weights are rounded by the caller.  Everything else stays float64.
"""
from __future__ import annotations

import numpy as np

NBINS = 512
NCELLS = 512
BIN_SITES = 8           # sites per bin of the N = 4097 rings (floor((N - 1) / 2 / 256))
CONV_TAPS = 9
CONV_PAD = 4
SHAPES = {
    "W1": (512, 32), "b1": (512,),
    "W2": (1024, 512), "b2": (1024,),
    "W3": (1024, 1024), "b3": (1024,),
    "W4": (1024, 1024), "b4": (1024,),
    "cw": (2, CONV_TAPS), "cb": (1,),
}
ORDER = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4", "cw", "cb")


def n_params() -> int:
    return int(sum(np.prod(s) for s in SHAPES.values()))


def unflatten(flat: np.ndarray) -> dict:
    out, o = {}, 0
    for k in ORDER:
        n = int(np.prod(SHAPES[k]))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(SHAPES[k])
        o += n
    return out


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in ORDER])


def _conv(z4, cw, cb):
    """l[b, i] = cb + sum_c sum_j cw[c, j] z4[b, c, i + j - 4] with zero padding."""
    B = z4.shape[0]
    zp = np.zeros((B, 2, NBINS + 2 * CONV_PAD))
    zp[:, :, CONV_PAD:CONV_PAD + NBINS] = z4
    out = np.full((B, NBINS), cb[0])
    for c in range(2):
        for j in range(CONV_TAPS):
            out += cw[c, j] * zp[:, c, j:j + NBINS]
    return out


def site_bin(dx: int, w: int = BIN_SITES, nbins: int = NBINS):
    """[(bin, share)] of the site at offset dx from the start (symmetric binning)."""
    h = nbins // 2
    if dx == 0:
        return [(h - 1, 0.5), (h, 0.5)]
    if dx < 0:
        k = (-dx - 1) // w
        return [(h - 1 - k, 1.0)] if k < h else []
    k = (dx - 1) // w
    return [(h + k, 1.0)] if k < h else []


def resample_matrix(T: int, w: int = BIN_SITES) -> np.ndarray:
    """R(T): NBINS x NCELLS, column j = how cell j's mass lands in the bins."""
    R = np.zeros((NBINS, NCELLS))
    clen = (T + 1) / NCELLS
    for j in range(NCELLS):
        a, b = j * clen, (j + 1) * clen
        for k in range(int(np.floor(a)), int(np.ceil(b))):
            ov = min(b, k + 1) - max(a, k)
            if ov <= 0:
                continue
            for bi, sh in site_bin(-T + 2 * k, w):
                R[bi, j] += sh * ov / clen
    return R


def bf16_round(v: np.ndarray) -> np.ndarray:
    """v rounded to bfloat16 (nearest, ties to even) through its fp32 value, as float64."""
    u = np.ascontiguousarray(np.asarray(v, dtype=np.float64).astype(np.float32)).view(np.uint32)
    r = (u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))) & np.uint32(0xFFFF0000)
    return r.view(np.float32).astype(np.float64)


def forward(p: dict, x: np.ndarray, T, bf16: bool = False) -> dict:
    x = np.asarray(x, dtype=np.float64)
    rnd = bf16_round if bf16 else (lambda v: v)
    a = {"x": x}
    a["z1"] = x @ p["W1"].T + p["b1"]
    a["h1"] = rnd(np.maximum(a["z1"], 0.0))
    a["z2"] = a["h1"] @ p["W2"].T + p["b2"]
    a["h2"] = rnd(np.maximum(a["z2"], 0.0))
    a["z3"] = a["h2"] @ p["W3"].T + p["b3"]
    a["h3"] = rnd(np.maximum(a["z3"], 0.0))
    a["z4"] = a["h3"] @ p["W4"].T + p["b4"]
    a["l"] = _conv(a["z4"].reshape(-1, 2, NBINS), p["cw"], p["cb"])
    m = a["l"].max(axis=1, keepdims=True)
    e = np.exp(a["l"] - m)
    a["q"] = e / e.sum(axis=1, keepdims=True)
    T = np.broadcast_to(np.asarray(T, dtype=np.int64), (x.shape[0],))
    a["R"] = [resample_matrix(int(t)) for t in T]
    a["p"] = np.stack([R @ q for R, q in zip(a["R"], a["q"])])
    return a


def _kl_rows(y, pb):
    y = np.asarray(y, dtype=np.float64)
    safe = np.where(y > 0, y, 1.0)
    return np.sum(np.where(y > 0, y * (np.log(safe) - np.log(np.where(y > 0, pb, 1.0))), 0.0), axis=1)


def loss(p: dict, x: np.ndarray, y: np.ndarray, T, bf16: bool = False) -> float:
    a = forward(p, x, T, bf16)
    return float(np.mean(_kl_rows(y, a["p"])))


def backward(p: dict, x: np.ndarray, y: np.ndarray, T, bf16: bool = False) -> dict:
    """Gradients of loss() with respect to every parameter (chain rule written out)."""
    a = forward(p, x, T, bf16)
    rnd = bf16_round if bf16 else (lambda v: v)
    y = np.asarray(y, dtype=np.float64)
    B = x.shape[0]
    # dL/dp_b = -y_b / p_b; dL/dq = R^T dL/dp; softmax: dl = q (dq - <q, dq>)
    gp = np.where(y > 0, -y / np.where(y > 0, a["p"], 1.0), 0.0) / B
    dq = np.stack([R.T @ g for R, g in zip(a["R"], gp)])
    dl = a["q"] * (dq - np.sum(a["q"] * dq, axis=1, keepdims=True))
    g = {}
    g["cb"] = np.array([dl.sum()])
    z4 = a["z4"].reshape(B, 2, NBINS)
    zp = np.zeros((B, 2, NBINS + 2 * CONV_PAD))
    zp[:, :, CONV_PAD:CONV_PAD + NBINS] = z4
    g["cw"] = np.zeros((2, CONV_TAPS))
    dzp = np.zeros_like(zp)
    for c in range(2):
        for j in range(CONV_TAPS):
            g["cw"][c, j] = np.sum(dl * zp[:, c, j:j + NBINS])
            dzp[:, c, j:j + NBINS] += p["cw"][c, j] * dl
    dz4 = dzp[:, :, CONV_PAD:CONV_PAD + NBINS].reshape(B, 2 * NBINS)
    g["W4"] = rnd(dz4).T @ a["h3"]
    g["b4"] = dz4.sum(axis=0)
    dh3 = rnd(dz4) @ p["W4"]
    dz3 = dh3 * (a["z3"] > 0)
    g["W3"] = rnd(dz3).T @ a["h2"]
    g["b3"] = dz3.sum(axis=0)
    dh2 = rnd(dz3) @ p["W3"]
    dz2 = dh2 * (a["z2"] > 0)
    g["W2"] = rnd(dz2).T @ a["h1"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = rnd(dz2) @ p["W2"]
    dz1 = dh1 * (a["z1"] > 0)
    g["W1"] = rnd(dz1).T @ a["x"]
    g["b1"] = dz1.sum(axis=0)
    return g


def tvd(p: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Total-variation distance 1/2 sum_b |p_b - q_b| per row."""
    return 0.5 * np.sum(np.abs(np.asarray(p, np.float64) - np.asarray(q, np.float64)), axis=-1)


def features(N, T, angles, psi0) -> np.ndarray:
    """The 32 input features of each walk (fp64): sin/cos of (theta, phi, chi);
    |a|, Re b', Im b' with b' = b e^{-i arg a}; T/N; cos and sin of
    delta = arg b - arg a + chi - phi; zeros."""
    N = np.asarray(N, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    ang = np.asarray(angles, dtype=np.float64).reshape(-1, 3)
    p = np.asarray(psi0, dtype=np.complex128).reshape(-1, 2)
    th, ph, ch = ang[:, 0], ang[:, 1], ang[:, 2]
    a, b = p[:, 0], p[:, 1]
    arga, argb = np.angle(a), np.angle(b)
    bp = b * np.exp(-1j * arga)
    dl = argb - arga + ch - ph
    X = np.zeros((p.shape[0], 32))
    X[:, 0], X[:, 1] = np.sin(th), np.cos(th)
    X[:, 2], X[:, 3] = np.sin(ph), np.cos(ph)
    X[:, 4], X[:, 5] = np.sin(ch), np.cos(ch)
    X[:, 6], X[:, 7], X[:, 8] = np.abs(a), bp.real, bp.imag
    X[:, 9] = T / N
    X[:, 10], X[:, 11] = np.cos(dl), np.sin(dl)
    return X
