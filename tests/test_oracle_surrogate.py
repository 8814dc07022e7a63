"""Pins of the fp64 surrogate-network oracle: finite differences of its loss
against its backward pass, and properties of its forward pass."""
import numpy as np
import pytest

from oracle import surrogate as S


def _small_params(rng, scale=0.05):
    p = {}
    for k in S.ORDER:
        p[k] = rng.normal(size=S.SHAPES[k]) * scale
    p["cw"] = rng.normal(size=S.SHAPES["cw"]) * 0.5
    return p


def _batch(rng, B=3, T=(300, 2048, 1001)):
    x = np.zeros((B, 32))
    x[:, :12] = rng.normal(size=(B, 12))
    T = np.array(T[:B])
    y = np.zeros((B, S.NBINS))
    for i, t in enumerate(T):                          # support of a walk of t steps
        half = int(np.ceil(t / S.BIN_SITES))
        y[i, 256 - half:256 + half] = rng.random(2 * half) ** 4 + 1e-3
        y[i, 256 - half] = 0.0                         # exact zeros exercise 0 log 0
    y /= y.sum(axis=1, keepdims=True)
    return x, y, T


def test_forward_is_a_distribution_on_the_cone():
    rng = np.random.default_rng(0)
    p = _small_params(rng)
    x, _, T = _batch(rng)
    a = S.forward(p, x, T)
    assert np.all(a["q"] > 0) and np.allclose(a["q"].sum(axis=1), 1.0, atol=1e-13)
    assert np.allclose(a["p"].sum(axis=1), 1.0, atol=1e-12)
    for i, t in enumerate(T):                          # no mass beyond the light cone
        half = int(np.ceil(t / S.BIN_SITES))
        assert np.all(a["p"][i, :256 - half] == 0) and np.all(a["p"][i, 256 + half:] == 0)


def test_resample_matrix_geometry():
    """Columns sum to 1; a uniform cell density gives each bin its share of sites."""
    for T in (256, 257, 1000, 2048):
        R = S.resample_matrix(T)
        assert np.allclose(R.sum(axis=0), 1.0, atol=1e-12)
        p = R @ np.full(S.NCELLS, 1.0 / S.NCELLS)      # uniform over the T + 1 sites
        counts = np.zeros(S.NBINS)
        for k in range(T + 1):
            for b, sh in S.site_bin(-T + 2 * k):
                counts[b] += sh
        assert np.allclose(p, counts / (T + 1), atol=1e-12)


def test_loss_is_kl_and_zero_at_match():
    rng = np.random.default_rng(1)
    p = _small_params(rng)
    x, _, T = _batch(rng)
    pb = S.forward(p, x, T)["p"]
    assert abs(S.loss(p, x, pb, T)) <= 1e-13        # KL(p || p) = 0
    _, y, _ = _batch(rng)
    assert S.loss(p, x, y, T) > 0.0


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    p = _small_params(rng)
    x, y, T = _batch(rng)
    g = S.backward(p, x, y, T)
    h = 1e-6
    for k in S.ORDER:
        flat = p[k].ravel()
        for _ in range(3):
            i = int(rng.integers(0, flat.size))
            old = flat[i]
            flat[i] = old + h
            lp = S.loss(p, x, y, T)
            flat[i] = old - h
            lm = S.loss(p, x, y, T)
            flat[i] = old
            num = (lp - lm) / (2 * h)
            ana = g[k].ravel()[i]
            assert abs(num - ana) <= 1e-7 + 1e-5 * abs(num), (k, i, num, ana)


def test_flatten_roundtrip():
    rng = np.random.default_rng(3)
    p = _small_params(rng)
    q = S.unflatten(S.flatten(p))
    for k in S.ORDER:
        assert np.array_equal(p[k], q[k])
    assert S.n_params() == S.flatten(p).size


def test_features_invariants():
    """Features depend on the start state only through its global-phase class."""
    rng = np.random.default_rng(4)
    psi = rng.normal(size=(5, 2)) + 1j * rng.normal(size=(5, 2))
    psi /= np.linalg.norm(psi, axis=1, keepdims=True)
    ang = rng.uniform(0, 3, size=(5, 3))
    X1 = S.features(np.full(5, 4097), np.full(5, 300), ang, psi)
    X2 = S.features(np.full(5, 4097), np.full(5, 300), ang, psi * np.exp(1j * 0.7))
    assert np.allclose(X1, X2, atol=1e-12)
    assert np.allclose(X1[:, 6] ** 2 + X1[:, 7] ** 2 + X1[:, 8] ** 2, 1.0)


def test_bf16_round_matches_torch_and_ties_to_even():
    """The oracle's bf16 rounding (round to nearest, ties to even, through fp32)
    against torch's CPU conversion on random and on tie values."""
    import torch
    rng = np.random.default_rng(2)
    v = np.concatenate([rng.normal(size=4096) * 10.0 ** rng.integers(-20, 20, size=4096),
                        [0.0, -0.0, 1.0, -2.5, 3.0e38, 1e-39]])
    want = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16_round(v), want)
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: to the even mantissa, 1;
    # 1 + 3 * 2^-8 halfway between 1 + 2^-7 and 1 + 2^-6: to 1 + 2^-6
    assert S.bf16_round(np.array([1 + 2.0 ** -8]))[0] == 1.0
    assert S.bf16_round(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6
    assert S.bf16_round(np.array([1 + 2.0 ** -8 + 2.0 ** -20]))[0] == 1 + 2.0 ** -7


def test_bf16_option_changes_only_the_rounding():
    """With bf16 operands the fp64 network moves by the rounding only: loss and
    gradients stay within a few 1e-3 relative of the unrounded network's, and
    differ from them."""
    rng = np.random.default_rng(8)
    p = {k: rng.normal(size=v) * 0.05 for k, v in S.SHAPES.items()}
    x = S.bf16_round(rng.normal(size=(6, 32)))
    T = rng.integers(256, 2048, size=6)
    y = S.forward(p, rng.normal(size=(6, 32)), T)["p"]      # targets on the walks' support
    l0, l1 = S.loss(p, x, y, T), S.loss(p, x, y, T, bf16=True)
    assert l0 != l1 and abs(l0 - l1) <= 1e-2 * abs(l0)
    g0, g1 = S.backward(p, x, y, T), S.backward(p, x, y, T, bf16=True)
    for k in S.ORDER:
        if k == "cb":                    # exactly zero (softmax is shift invariant)
            assert abs(g0[k][0]) <= 1e-12 and abs(g1[k][0]) <= 1e-12
            continue
        rel = np.linalg.norm(g1[k] - g0[k]) / max(np.linalg.norm(g0[k]), 1e-30)
        assert 0.0 < rel <= 5e-2, k
