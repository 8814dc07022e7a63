"""The learned surrogate on the GPU: forward pass and gradients against the
fp64 network oracle (on the GPU's bf16-rounded weights), training, and the
fallback semantics of surr_predict against the plain batched walk."""
import numpy as np
import pytest

from oracle import surrogate as S
from paper_1003_3779_amd import inputs, qwalk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    qwalk.load()
    yield


def _walk_params(seed, n, N=4097, tmin=256, tmax=2048):
    rng = np.random.Generator(np.random.PCG64(seed))
    T = rng.integers(tmin, tmax, size=n, endpoint=True)
    ang = inputs.su2_angles(rng, n)
    psi0 = np.stack([inputs.haar_state(rng, 2) for _ in range(n)])
    return np.full(n, N, dtype=np.int64), T.astype(np.int64), ang, psi0


def _plain_bins(N, T, ang, psi0):
    b = qwalk.Batch(N, T, ang, psi0, prec=qwalk.QW_C64, nbins=512)
    b.run()
    out = b.binned()
    b.destroy()
    return out


def test_features_match_oracle():
    N, T, ang, psi0 = _walk_params(1, 300)
    s = qwalk.Surrogate(seed=1)
    X = s.features(N, T, ang, psi0)
    s.destroy()
    assert np.max(np.abs(X - S.features(N, T, ang, psi0))) <= 2e-6


def test_forward_matches_oracle():
    N, T, ang, psi0 = _walk_params(2, 256)
    s = qwalk.Surrogate(seed=7)
    X = s.features(N, T, ang, psi0)
    q = s.forward(X, T)
    p = S.unflatten(s.params(bf16_rounded=True).astype(np.float64))
    s.destroy()
    xr = S.bf16_round(X)                                # the GPU feeds bf16 inputs
    assert np.all(np.abs(q.sum(axis=1) - 1.0) <= 1e-4)
    # on the same bf16-rounded operands (inputs, weights, hidden activations)
    # only the fp32 accumulation and the fp32 head differ from the fp64 oracle
    qb = S.forward(p, xr, T, bf16=True)["p"]
    assert np.max(S.tvd(q, qb)) <= 5e-3
    # the fp64 network without the rounding of the activations is farther away
    qr = S.forward(p, xr, T)["p"]
    assert np.max(S.tvd(q, qr)) <= 2e-2


def test_gradients_match_oracle():
    N, T, ang, psi0 = _walk_params(3, 256)
    y = _plain_bins(N, T, ang, psi0).astype(np.float64)
    y /= y.sum(axis=1, keepdims=True)
    s = qwalk.Surrogate(seed=11)
    X = s.features(N, T, ang, psi0)
    loss, g = s.loss_grad(X, y.astype(np.float32), T)
    p = S.unflatten(s.params(bf16_rounded=True).astype(np.float64))
    s.destroy()
    xr = S.bf16_round(X)
    # the oracle on the GPU's bf16 operands: inputs, weights, hidden activations
    # and each layer's dZ where it enters a matrix product
    lref = S.loss(p, xr, y, T, bf16=True)
    assert abs(loss - lref) <= 5e-3 * abs(lref)
    gr = S.backward(p, xr, y, T, bf16=True)
    gg = S.unflatten(g.astype(np.float64))
    for k in S.ORDER:
        if k == "cb":
            # softmax is invariant under a common shift of the logits: the exact
            # gradient of the output bias is zero, so compare absolutely
            assert abs(gr[k][0]) <= 1e-12 and abs(gg[k][0]) <= 1e-4, (gr[k], gg[k])
            continue
        rel = np.linalg.norm(gg[k] - gr[k]) / max(np.linalg.norm(gr[k]), 1e-30)
        print(f"# gradient {k}: relative error {rel:.2e}", flush=True)
        assert rel <= 1e-2, (k, rel)


def test_training_reduces_loss_and_save_load(tmp_path):
    torch = pytest.importorskip("torch")
    n = 4096
    N, T, ang, psi0 = _walk_params(4, n)
    y = _plain_bins(N, T, ang, psi0)
    s = qwalk.Surrogate(seed=3)
    X = s.features(N, T, ang, psi0)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.from_numpy(y).cuda()
    Td = torch.from_numpy(T.astype(np.int32)).cuda()
    hist = s.train(Xd, Yd, Td, n, batch=512, epochs=6, lr=1e-3, seed=5)
    assert np.all(np.isfinite(hist))
    assert hist[-1] < 0.7 * hist[0]
    q1 = s.forward(X[:64], T[:64])
    path = str(tmp_path / "s.qws")
    s.save(path)
    s.destroy()
    s2 = qwalk.Surrogate.load_file(path)
    assert np.array_equal(s2.forward(X[:64], T[:64]), q1)
    s2.destroy()


def test_predict_fallback_semantics():
    """Out-of-range walks and chunks whose re-check fails return exactly the
    plain walk's bins; the untouched chunks return the network's."""
    n = 2048
    N, T, ang, psi0 = _walk_params(5, n)
    N[:10] = 3001                                     # outside the training range
    T[10:20] = 4000
    plain = _plain_bins(N, T, ang, psi0)
    s = qwalk.Surrogate(seed=9)                       # untrained: every re-check fails
    out, fb, st = s.predict(N, T, ang, psi0, chunk=512)
    assert st.out_of_range == 20 and fb.all() and st.failed_chunks == 4
    assert np.array_equal(out, plain)
    # an impossible tolerance keeps the network's answer except where re-checked/out of range
    out2, fb2, st2 = s.predict(N, T, ang, psi0, chunk=512, tvd_tol=2.0)
    assert st2.failed_chunks == 0 and st2.fallback == 20 and fb2.sum() == 20
    net = s.forward(s.features(N, T, ang, psi0), T)
    keep = ~fb2
    rechecked = np.all(out2 == plain, axis=1) & keep
    assert rechecked.sum() >= st2.rechecked - 1     # re-checked walks carry the plain result
    assert np.array_equal(out2[keep & ~rechecked], net[keep & ~rechecked])
    s.destroy()


def test_predict_device_output_matches_host_output():
    """The bins written to device memory equal the host-output call bit for
    bit, including the re-checked and fallback rows."""
    torch = pytest.importorskip("torch")
    n = 1500                                           # ragged last chunk and padded network rows
    N, T, ang, psi0 = _walk_params(6, n)
    N[:3] = 2001                                       # out of range: plain walk
    s = qwalk.Surrogate(seed=13)
    for tol in (1e-3, 2.0):                            # every chunk falls back / none does
        host, fb_h, st_h = s.predict(N, T, ang, psi0, chunk=512, tvd_tol=tol)
        dev = torch.empty((n, 512), dtype=torch.float32, device="cuda")
        out, fb_d, st_d = s.predict(N, T, ang, psi0, chunk=512, tvd_tol=tol, out=dev)
        assert out is dev
        assert np.array_equal(dev.cpu().numpy(), host)
        assert np.array_equal(fb_h, fb_d) and st_h.failed_chunks == st_d.failed_chunks
    s.destroy()


def test_trained_network_gain_over_the_plain_walk():
    """What the trained network adds, on held-out walks: its binned answers are
    far closer to the plain walk's than the best answer that ignores the coin
    and the start state (the mean training distribution of the same T range),
    and its pass costs a small fraction of the plain batch's time; at a loose
    tolerance (TVD 0.3) surr_predict answers most walks with the network.  At
    1e-3 every chunk falls back (the floor: tests/test_oracle_surrogate_floor.py)."""
    torch = pytest.importorskip("torch")
    n_tr, n_ev = 1 << 16, 8192
    N, T, ang, psi0 = _walk_params(21, n_tr)
    b = qwalk.Batch(N, T, ang, psi0, prec=qwalk.QW_C64, nbins=512)
    b.run()
    Y = b.binned()
    b.destroy()
    s = qwalk.Surrogate(seed=21)
    X = s.features(N, T, ang, psi0)
    Xd, Yd, Td = (torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(),
                  torch.from_numpy(T.astype(np.int32)).cuda())
    hist = s.train(Xd, Yd, Td, n_tr, batch=1024, epochs=12, lr=1e-3, seed=21)
    assert np.all(np.isfinite(hist)) and hist[-1] < 0.5 * hist[0]
    Ne, Te, Ae, Pe = _walk_params(22, n_ev)
    b = qwalk.Batch(Ne, Te, Ae, Pe, prec=qwalk.QW_C64, nbins=512)
    b.run()
    Ye = b.binned().astype(np.float64)
    plain_ms = b.info().last_run_ms
    b.destroy()
    net = s.forward(s.features(Ne, Te, Ae, Pe), Te).astype(np.float64)
    tvd_net = 0.5 * np.abs(net - Ye).sum(axis=1)
    tvd_mean = 0.5 * np.abs(Y.astype(np.float64).mean(axis=0)[None, :] - Ye).sum(axis=1)
    print(f"# held-out TVD median: network {np.median(tvd_net):.3f}, mean distribution "
          f"{np.median(tvd_mean):.3f}", flush=True)
    assert np.median(tvd_net) < 0.5 * np.median(tvd_mean)
    out, fb, st = s.predict(Ne, Te, Ae, Pe, tvd_tol=0.3)
    print(f"# tol 0.3: fallback {fb.mean():.3f}, network {st.ms_network:.2f} ms, plain batch {plain_ms:.2f} ms",
          flush=True)
    assert fb.mean() < 0.5
    assert st.ms_network < 0.2 * plain_ms
    _, fb3, st3 = s.predict(Ne, Te, Ae, Pe, tvd_tol=1e-3)
    assert fb3.all() and st3.failed_chunks == (n_ev + 1023) // 1024
    s.destroy()
