"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances: complex128 runs must match the oracle to 1e-12 max-abs on
amplitudes and P(x); complex64 runs to 2e-5 max-abs on P(x) (the walk's fp32
budget after 2048 steps).  Every input is seeded; expected values come from
the oracle only.
"""
import math
import zlib

import numpy as np
import pytest

import oracle
from paper_1003_3779_amd import inputs, qwalk

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32_P = 2e-5


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    qwalk.load()
    yield


def _oracle_coin(kind, d, ang=(0.0, 0.0, 0.0), dense=None):
    return oracle.coin(kind, d, *ang, dense=dense)


def _run_gpu(extent, disp, kind, psi0, x0, T, prec, ang=(0.0, 0.0, 0.0), dense=None, **opts):
    w = qwalk.Walk(extent, disp, kind, psi0, x0, prec=prec, theta=ang[0], phi=ang[1], chi=ang[2], dense=dense)
    if opts:
        w.set_options(**opts)
    w.step(T)
    P = w.probabilities()
    psi = w.get_state()
    n = w.norm()
    st = w.stats()
    w.destroy()
    return P, psi, n, st


def _oracle_run(extent, disp, C, psi0, x0, T):
    Lx = extent[0]
    Ly = extent[1] if len(extent) > 1 else 1
    psi = oracle.walk(Lx, Ly, disp, C, (x0[0], x0[1] if len(x0) > 1 else 0), psi0, T)
    return oracle.prob(psi), psi


def _as_oracle_layout(psi_gpu):
    # GPU: (d, Ly, Lx) -> oracle: (Ly, Lx, d)
    return np.transpose(psi_gpu, (1, 2, 0))


# ---------------------------------------------------------------- 1D ring
def test_ring1d_hadamard_full_config():
    cfg = inputs.config("ring1d")
    N = cfg["extent"][0]
    P, psi, n, st = _run_gpu((N,), cfg["disp"], qwalk.HADAMARD, cfg["psi0"], cfg["x0"], cfg["T"], qwalk.QW_C128)
    Pr, psir = _oracle_run((N,), cfg["disp"], _oracle_coin(oracle.HADAMARD, 2), cfg["psi0"], cfg["x0"], cfg["T"])
    assert np.max(np.abs(P - Pr)) <= TOL64
    assert np.max(np.abs(_as_oracle_layout(psi) - psir)) <= TOL64
    assert abs(n - 1.0) <= TOL64
    assert st.t == cfg["T"]


RING_CASES = [
    # N, T, depth, prec
    (1, 5, 0, qwalk.QW_C128), (2, 7, 0, qwalk.QW_C128), (3, 9, 1, qwalk.QW_C128), (7, 30, 0, qwalk.QW_C128),
    (64, 100, 0, qwalk.QW_C128), (513, 600, 0, qwalk.QW_C128), (1000, 333, 1, qwalk.QW_C128),
    (4095, 700, 0, qwalk.QW_C128), (4097, 300, 0, qwalk.QW_C128),           # whole ring / tiles boundary
    (5001, 1200, 16, qwalk.QW_C128), (20011, 150, 4, qwalk.QW_C128), (9999, 203, 8, qwalk.QW_C128),
    (8192, 500, 0, qwalk.QW_C64), (8193, 500, 0, qwalk.QW_C64), (777, 2048, 0, qwalk.QW_C64),
    (30001, 257, 16, qwalk.QW_C64), (5000, 301, 1, qwalk.QW_C64),
]


@pytest.mark.parametrize("N,T,depth,prec", RING_CASES)
def test_ring_random_unitary(N, T, depth, prec):
    rng = np.random.default_rng(N * 7 + T)
    U = inputs.haar_unitary(rng, 2)
    psi0 = inputs.haar_state(rng, 2)
    x0 = (int(rng.integers(0, N)), 0)
    P, psi, n, _ = _run_gpu((N,), inputs.RING, qwalk.DENSE, psi0, x0, T, prec, dense=U, block_depth=depth)
    Pr, psir = _oracle_run((N,), inputs.RING, U, psi0, x0, T)
    if prec == qwalk.QW_C128:
        assert np.max(np.abs(P - Pr)) <= TOL64
        assert np.max(np.abs(_as_oracle_layout(psi) - psir)) <= TOL64
        assert abs(n - 1.0) <= TOL64
    else:
        assert np.max(np.abs(P - Pr)) <= TOL32_P


@pytest.mark.parametrize("theta", [0.3, 1.2, 2.9])
def test_ring_su2(theta):
    rng = np.random.default_rng(int(theta * 100))
    phi, chi = rng.uniform(0, 2 * math.pi, 2)
    psi0 = inputs.haar_state(rng, 2)
    N, T = 2049, 1024
    P, psi, n, _ = _run_gpu((N,), inputs.RING, qwalk.SU2, psi0, (1024, 0), T, qwalk.QW_C128, ang=(theta, phi, chi))
    Pr, psir = _oracle_run((N,), inputs.RING, _oracle_coin(oracle.SU2, 2, (theta, phi, chi)), psi0, (1024, 0), T)
    assert np.max(np.abs(P - Pr)) <= TOL64
    assert np.max(np.abs(_as_oracle_layout(psi) - psir)) <= TOL64


def test_ring_c64_2048_steps_budget():
    """complex64 Hadamard walk after 2048 steps, with and without renormalisation."""
    N, T = 4097, 2048
    Pr, _ = _oracle_run((N,), inputs.RING, _oracle_coin(oracle.HADAMARD, 2), inputs.PSI0_LR, (2048, 0), T)
    P, _, n, st = _run_gpu((N,), inputs.RING, qwalk.HADAMARD, inputs.PSI0_LR, (2048, 0), T, qwalk.QW_C64)
    assert np.max(np.abs(P - Pr)) <= TOL32_P
    assert st.renorm_checks == T // 64 and st.renorms >= 1
    assert abs(n - 1.0) <= 1e-5
    P2, _, n2, st2 = _run_gpu((N,), inputs.RING, qwalk.HADAMARD, inputs.PSI0_LR, (2048, 0), T, qwalk.QW_C64,
                              renorm_every=0)
    assert st2.renorms == 0
    assert np.max(np.abs(P2 - Pr)) <= TOL32_P


def test_ring_window_and_depth_are_bitwise_identical():
    rng = np.random.default_rng(5)
    U = inputs.haar_unitary(rng, 2)
    psi0 = inputs.haar_state(rng, 2)
    N, T, x0 = 12289, 400, (6000, 0)
    res = []
    for depth, window in ((1, 1), (1, 0), (4, 1), (8, 1), (16, 1), (16, 0)):
        P, psi, _, _ = _run_gpu((N,), inputs.RING, qwalk.DENSE, psi0, x0, T, qwalk.QW_C128, dense=U,
                                block_depth=depth, window=window)
        res.append(psi)
    for r in res[1:]:
        assert np.array_equal(r, res[0])


# ---------------------------------------------------------------- 2D torus
TORUS_COINS = [
    ("grover", qwalk.GROVER, oracle.GROVER),
    ("hh", qwalk.HADAMARD2, oracle.HADAMARD2),
    ("fourier", qwalk.FOURIER, oracle.FOURIER),
    ("haar", qwalk.DENSE, None),
]


@pytest.mark.parametrize("table", ["PAIR", "EQ8", "DIAG"])
@pytest.mark.parametrize("coin_name,kind,okind", TORUS_COINS)
@pytest.mark.parametrize("depth", [1, 4, 8])
def test_torus_c128(table, coin_name, kind, okind, depth):
    disp = getattr(inputs, table)
    # a seed fixed by the case's name (str hashes are salted per process)
    rng = np.random.default_rng(zlib.crc32(f"{table}-{coin_name}-{depth}".encode()))
    dense = inputs.haar_unitary(rng, 4) if kind == qwalk.DENSE else None
    C = dense if dense is not None else _oracle_coin(okind, 4)
    psi0 = inputs.haar_state(rng, 4)
    ext = (97, 70)
    x0 = (int(rng.integers(0, 97)), int(rng.integers(0, 70)))
    T = 61
    P, psi, n, _ = _run_gpu(ext, disp, kind, psi0, x0, T, qwalk.QW_C128, dense=dense, block_depth=depth)
    Pr, psir = _oracle_run(ext, disp, C, psi0, x0, T)
    assert np.max(np.abs(P - Pr)) <= TOL64
    assert np.max(np.abs(_as_oracle_layout(psi) - psir)) <= TOL64
    assert abs(n - 1.0) <= TOL64


@pytest.mark.parametrize("depth", [1, 4, 8, 12, 16])
@pytest.mark.parametrize("coin_name,kind,okind", TORUS_COINS)
def test_torus_c64(coin_name, kind, okind, depth):
    rng = np.random.default_rng(depth * 31 + kind)
    dense = inputs.haar_unitary(rng, 4) if kind == qwalk.DENSE else None
    C = dense if dense is not None else _oracle_coin(okind, 4)
    psi0 = inputs.haar_state(rng, 4)
    ext, x0, T = (130, 67), (64, 33), 150
    P, _, n, _ = _run_gpu(ext, inputs.PAIR, kind, psi0, x0, T, qwalk.QW_C64, dense=dense, block_depth=depth)
    Pr, _ = _oracle_run(ext, inputs.PAIR, C, psi0, x0, T)
    assert np.max(np.abs(P - Pr)) <= TOL32_P
    assert abs(n - 1.0) <= 1e-5


def test_torus_small_and_degenerate():
    """Lattices narrower than a wave and 1-wide tori use the one-step kernel."""
    for ext in ((1, 1), (1, 5), (5, 1), (3, 2), (33, 17), (63, 64)):
        rng = np.random.default_rng(ext[0] * 100 + ext[1])
        U = inputs.haar_unitary(rng, 4)
        psi0 = inputs.haar_state(rng, 4)
        x0 = (0, ext[1] - 1)
        for depth in (0, 1):
            P, psi, n, _ = _run_gpu(ext, inputs.PAIR, qwalk.DENSE, psi0, x0, 13, qwalk.QW_C128, dense=U,
                                    block_depth=depth)
            Pr, psir = _oracle_run(ext, inputs.PAIR, U, psi0, x0, 13)
            assert np.max(np.abs(_as_oracle_layout(psi) - psir)) <= TOL64, ext


def test_torus_blocked_equals_unblocked_bitwise():
    """Every block depth (with remainders run at the largest smaller depth) and
    both window modes give the same amplitudes bit for bit."""
    rng = np.random.default_rng(77)
    psi0 = inputs.haar_state(rng, 4)
    for prec, depths in ((qwalk.QW_C128, (4, 8)), (qwalk.QW_C64, (4, 8, 12, 16))):
        for kind in (qwalk.GROVER, qwalk.HADAMARD2):
            res = []
            for depth, window in ((1, 1), (1, 0)) + tuple((k, 1) for k in depths) + ((depths[-1], 0),):
                # 83 steps: at K = 12 six blocks, one of 8 and three single steps; the c64
                # norm check every 64 steps splits them further
                _, psi, _, _ = _run_gpu((200, 150), inputs.PAIR, kind, psi0, (10, 140), 83, prec,
                                        block_depth=depth, window=window)
                res.append(psi)
            for r in res[1:]:
                assert np.array_equal(r, res[0])


@pytest.mark.parametrize("prec", [qwalk.QW_C128, qwalk.QW_C64])
@pytest.mark.parametrize("table", ["PAIR", "EQ8", "DIAG"])
def test_torus_prefetch_depth_is_bitwise_neutral(prec, table):
    """The torus kernel's read-ahead (1 or 3 rows), its segment length (waves
    per launch) and its block order (XCD-aware or linear) change only when loads
    are issued and which wave takes which strip: every block depth gives the same
    amplitudes bit for bit."""
    disp = getattr(inputs, table)
    rng = np.random.default_rng(len(table) * 10 + prec)
    U = inputs.haar_unitary(rng, 4)
    psi0 = inputs.haar_state(rng, 4)
    ext, x0, T = (211, 90), (100, 7), 97          # ragged strips and segments, wraps in y
    depths = (4, 8) if prec == qwalk.QW_C128 else (4, 8, 12, 16)
    for depth in depths:
        res = []
        for pd, waves, order in ((1, 0, 0), (3, 0, 2), (3, 37, 1), (1, 5000, 2), (3, 5000, 1), (3, 9, 2)):
            _, psi, _, _ = _run_gpu(ext, disp, qwalk.DENSE, psi0, x0, T, prec, dense=U, block_depth=depth,
                                    prefetch_rows=pd, stream_waves=waves, block_order=order, renorm_every=0)
            res.append(psi)
        for r in res[1:]:
            assert np.array_equal(res[0], r), depth
        if prec == qwalk.QW_C128:
            Pr, psir = _oracle_run(ext, disp, U, psi0, x0, T)
            assert np.max(np.abs(_as_oracle_layout(res[1]) - psir)) <= TOL64


def test_torus_wraps_around():
    """Cone larger than the torus: the walk wraps through the periodic boundary."""
    rng = np.random.default_rng(8)
    U = inputs.haar_unitary(rng, 4)
    psi0 = inputs.haar_state(rng, 4)
    ext, x0, T = (70, 66), (3, 60), 150
    for depth in (1, 8):
        P, psi, _, _ = _run_gpu(ext, inputs.DIAG, qwalk.DENSE, psi0, x0, T, qwalk.QW_C128, dense=U, block_depth=depth)
        Pr, psir = _oracle_run(ext, inputs.DIAG, U, psi0, x0, T)
        assert np.max(np.abs(_as_oracle_layout(psi) - psir)) <= TOL64


# ---------------------------------------------------------------- state API
def test_reversal():
    rng = np.random.default_rng(3)
    psi0 = inputs.haar_state(rng, 4)
    U = inputs.haar_unitary(rng, 4)
    for prec, tol in ((qwalk.QW_C128, 1e-12), (qwalk.QW_C64, 1e-5)):
        w = qwalk.Walk((80, 90), inputs.PAIR, qwalk.DENSE, psi0, (40, 45), prec=prec, dense=U)
        w.set_options(renorm_every=0)
        start = w.get_state()
        w.step(100)
        assert np.max(np.abs(w.get_state() - start)) > 1e-3
        w.step_inverse(100)
        back = w.get_state()
        assert w.time() == 0
        w.destroy()
        assert np.max(np.abs(back - start)) <= tol


def test_set_state_and_resume():
    rng = np.random.default_rng(4)
    U = inputs.haar_unitary(rng, 2)
    N = 3001
    z = rng.normal(size=(2, 1, N)) + 1j * rng.normal(size=(2, 1, N))
    z /= np.linalg.norm(z)
    w = qwalk.Walk((N,), inputs.RING, qwalk.DENSE, inputs.PSI0_LR, (0, 0), dense=U)
    w.set_state(z)
    assert np.max(np.abs(w.get_state() - z)) == 0.0
    w.step(200)
    got = w.get_state()
    want = oracle.evolve(_as_oracle_layout(z), inputs.RING, U, 200)
    assert np.max(np.abs(_as_oracle_layout(got) - want)) <= TOL64
    # resume: step T, save, restore into a fresh walk, step T == step 2T
    w2 = qwalk.Walk((N,), inputs.RING, qwalk.DENSE, inputs.PSI0_LR, (0, 0), dense=U)
    w2.set_state(got)
    w2.step(150)
    w.step(150)
    assert np.array_equal(w.get_state(), w2.get_state())
    # an unnormalised state is refused and leaves the walk unchanged
    before = w.get_state()
    with pytest.raises(qwalk.QWError) as e:
        w.set_state(z * 1.001)
    assert e.value.code == qwalk.QW_ENOTNORM
    assert np.array_equal(w.get_state(), before)
    w.destroy()
    w2.destroy()


def test_device_outputs_and_ext_buffers():
    torch = pytest.importorskip("torch")
    N, T = 6000, 500
    nb = qwalk.state_bytes((N,), inputs.RING, qwalk.QW_C128)
    a = torch.empty(nb, dtype=torch.uint8, device="cuda")
    b = torch.empty(nb, dtype=torch.uint8, device="cuda")
    scr = torch.empty(qwalk.scratch_bytes(), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    Pr, _ = _oracle_run((N,), inputs.RING, _oracle_coin(oracle.HADAMARD, 2), inputs.PSI0_LR, (3000, 0), T)
    for scratch in (None, scr):       # the library's own scratch area, then the caller's
        w = qwalk.Walk((N,), inputs.RING, qwalk.HADAMARD, inputs.PSI0_LR, (3000, 0), stream=stream,
                       state_buffers=(a, b), scratch=scratch)
        w.step(T)
        P = torch.empty(N, dtype=torch.float64, device="cuda")
        w.probabilities(out=P)
        n = w.norm()
        stream.synchronize()
        assert np.max(np.abs(P.cpu().numpy() - Pr[0])) <= TOL64
        assert abs(n - 1.0) <= TOL64
        w.destroy()


# ---------------------------------------------------------------- full-size 2D runs
def test_grover_4096_full_lattice_vs_oracle_t256():
    """The 4096^2 torus in the benchmarked launch configuration, compared with
    the light-cone oracle at T = 256."""
    cfg = inputs.config("grover2d")
    Lx, Ly = cfg["extent"]
    T = 256
    for prec, tol in ((qwalk.QW_C128, TOL64), (qwalk.QW_C64, TOL32_P)):
        w = qwalk.Walk(cfg["extent"], cfg["disp"], qwalk.GROVER, cfg["psi0"], cfg["x0"], prec=prec)
        w.step(T)
        P = w.probabilities()
        w.destroy()
        Pr, _ = _oracle_run(cfg["extent"], cfg["disp"], _oracle_coin(oracle.GROVER, 4), cfg["psi0"], cfg["x0"], T)
        assert np.max(np.abs(P - Pr)) <= tol


@pytest.mark.parametrize("prec", [qwalk.QW_C128, qwalk.QW_C64])
def test_grover_4096_t2048_properties(prec):
    """Full benchmark workload: properties that hold at any size."""
    cfg = inputs.config("grover2d")
    x0 = cfg["x0"]
    w = qwalk.Walk(cfg["extent"], cfg["disp"], qwalk.GROVER, cfg["psi0"], x0, prec=prec)
    w.step(cfg["T"])
    P = w.probabilities()
    n = w.norm()
    w.destroy()
    tol = TOL64 if prec == qwalk.QW_C128 else 1e-5
    assert abs(n - 1.0) <= tol
    lim = 4.0 / math.pi ** 2
    assert abs(P[x0[1], x0[0]] - lim) <= (1e-5 if prec == qwalk.QW_C128 else 3e-5)
    yy, xx = np.meshgrid(np.arange(P.shape[0]) - x0[1], np.arange(P.shape[1]) - x0[0], indexing="ij")
    assert np.all(P[(xx + yy - cfg["T"]) % 2 != 0] == 0.0)


def test_hh_16384_diagonal_factorises_full_size():
    """The 16384^2, T = 4096, complex64 H(x)H configuration on the diagonal table:
    there a product start a (x) b stays a product of two 1D Hadamard walks (c = 2j + k,
    j moving x by (-1)^j and k moving y by (-1)^k), so every P(x, y) is P_a(x) P_b(y)
    of two oracle ring walks; compared on all 2^28 sites."""
    import torch
    cfg = inputs.config("hh2d")
    ext, T, x0 = cfg["extent"], cfg["T"], cfg["x0"]
    rng = np.random.Generator(np.random.PCG64(33))
    a, b = inputs.haar_state(rng, 2), inputs.haar_state(rng, 2)
    w = qwalk.Walk(ext, inputs.DIAG, qwalk.HADAMARD2, np.kron(a, b), x0, prec=qwalk.QW_C64)
    w.step(T)
    P = torch.empty((ext[1], ext[0]), dtype=torch.float64, device="cuda")
    w.probabilities(out=P)
    n = w.norm()
    w.destroy()
    H = oracle.coin(oracle.HADAMARD, 2)
    px = oracle.prob(oracle.walk(ext[0], 1, inputs.RING, H, (x0[0], 0), a, T))[0]
    py = oracle.prob(oracle.walk(ext[1], 1, inputs.RING, H, (x0[1], 0), b, T))[0]
    ref = torch.outer(torch.from_numpy(py).cuda(), torch.from_numpy(px).cuda())
    assert torch.max(torch.abs(P - ref)).item() <= TOL32_P
    assert abs(n - 1.0) <= 1e-5


def test_hh_16384_properties():
    """The benchmark's 16384^2 H(x)H walk (pair table, Haar start, complex64):
    norm, nothing outside the light-cone box, and the site parity of a walk that
    moves one coordinate by one every step."""
    import torch
    cfg = inputs.config("hh2d")
    ext, T, x0 = cfg["extent"], cfg["T"], cfg["x0"]
    w = qwalk.Walk(ext, cfg["disp"], qwalk.HADAMARD2, cfg["psi0"], x0, prec=qwalk.QW_C64)
    w.step(T)
    P = torch.empty((ext[1], ext[0]), dtype=torch.float64, device="cuda")
    w.probabilities(out=P)
    n = w.norm()
    w.destroy()
    assert abs(n - 1.0) <= 1e-5
    yy = torch.arange(ext[1], device="cuda").view(-1, 1) - x0[1]
    xx = torch.arange(ext[0], device="cuda").view(1, -1) - x0[0]
    outside = (torch.abs(xx) + torch.abs(yy) > T) | ((xx + yy - T) % 2 != 0)
    assert torch.count_nonzero(P[outside]).item() == 0
    assert abs(torch.sum(P[~outside]).item() - 1.0) <= 1e-5


@pytest.mark.parametrize("name", ["fourier2d_diag", "fourier2d_natural"])
def test_fourier_workloads_full_size(name):
    """The paper's 2D workload shape (Fourier coin, diagonal and natural
    lattices, Size 500) at full size against the oracle."""
    cfg = inputs.config(name)
    ext, T, x0 = cfg["extent"], cfg["T"], cfg["x0"]
    P, psi, n, _ = _run_gpu(ext, cfg["disp"], cfg["coin"], cfg["psi0"], x0, T, qwalk.QW_C128)
    Pr, psir = _oracle_run(ext, cfg["disp"], _oracle_coin(oracle.FOURIER, 4), cfg["psi0"], x0, T)
    assert np.max(np.abs(P - Pr)) <= TOL64
    assert np.max(np.abs(_as_oracle_layout(psi) - psir)) <= TOL64
    assert abs(n - 1.0) <= TOL64
    # the diagonal lattice moves both coordinates every step: site parity (x + y) even
    if cfg["disp"] == inputs.DIAG:
        yy, xx = np.indices(P.shape)
        assert np.all(P[((xx - x0[0]) + (yy - x0[1])) % 2 == 1] == 0.0)


@pytest.mark.parametrize("prec", [qwalk.QW_C128, qwalk.QW_C64])
@pytest.mark.parametrize("real", [True, False])
def test_small_ring_halo_kernel_bitwise(prec, real):
    """Rings of up to 2048 (c128) / 4096 (c64) sites run in four waves with
    32-site halos, exchanging through LDS every 32 steps: bit for bit the one-step
    kernel's amplitudes, for rings shorter than a wave's window (repeated in it),
    block boundaries inside and between the pieces a walk is stepped in, and
    both coin paths; c128 also against the oracle."""
    sizes = [1, 2, 3, 5, 63, 64, 65, 255, 256, 257, 600, 1000, 2001, 2048]
    if prec == qwalk.QW_C64:
        sizes += [2049, 3000, 4096]
    for N in sizes:
        rng = np.random.default_rng(N + 3 * real + 7 * prec)
        if real:
            th = float(rng.uniform(0, np.pi))
            U = np.array([[np.cos(th), np.sin(th)], [-np.sin(th), np.cos(th)]], dtype=np.complex128)
        else:
            U = inputs.haar_unitary(rng, 2)
        psi0 = inputs.haar_state(rng, 2)
        x0 = (int(rng.integers(0, N)), 0)
        res = []
        for depth in (1, 0):
            w = qwalk.Walk((N,), inputs.RING, qwalk.DENSE, psi0, x0, prec=prec, dense=U)
            w.set_options(block_depth=depth, renorm_every=0)
            for n in (7, 1, 25, 0, 64, 33):
                w.step(n)
            res.append(w.get_state())
            w.destroy()
        assert np.array_equal(res[0], res[1]), N
        if prec == qwalk.QW_C128:
            _, psir = _oracle_run((N,), inputs.RING, U, psi0, x0, 130)
            assert np.max(np.abs(_as_oracle_layout(res[1]) - psir)) <= TOL64, N


@pytest.mark.parametrize("prec", [qwalk.QW_C128, qwalk.QW_C64])
def test_ring_live_sublattice_bitwise(prec):
    """A ring walk from one site whose support stays clear of itself runs on its
    live parity only (half the sites per step): bit for bit the one-step kernel's
    amplitudes, stepped in pieces (odd and even start times), up to t = (N - 1) / 2
    and past it (the full-lattice kernel takes over), after walk_set_state (no
    longer from one site: the full lattice; complex128) and for odd and even
    rings; the updates counted are the live ones."""
    rng = np.random.default_rng(40 + prec)
    for N in (7, 64, 101, 1000, 2001, 2048) + ((3001, 4095) if prec == qwalk.QW_C64 else ()):
        U = inputs.haar_unitary(rng, 2)
        psi0 = inputs.haar_state(rng, 2)
        x0 = (int(rng.integers(0, N)), 0)
        half = (N - 1) // 2
        pieces = (1, 2, 13, 32, 33, half // 3, half - (81 + half // 3)) if half > 120 else (1, 2, max(half - 3, 0))
        pieces = tuple(p for p in pieces if p > 0) + (5, 64)  # the last two cross t = (N - 1) / 2
        res, upd = [], []
        for depth in (1, 0):
            w = qwalk.Walk((N,), inputs.RING, qwalk.DENSE, psi0, x0, prec=prec, dense=U)
            w.set_options(block_depth=depth, renorm_every=0)
            states = []
            for k, n in enumerate(pieces):
                w.step(n)
                states.append(w.get_state())
                if k == 2:
                    upd.append(w.stats().updates)
            w.destroy()
            res.append(states)
        for k, (a, b) in enumerate(zip(res[0], res[1])):
            assert np.array_equal(a, b), (N, k)
        if N >= 64:  # live slots only while t <= (N - 1) / 2: about half the ring per step
            assert upd[1] <= 0.55 * N * 2 * sum(pieces[:3]), (N, upd)
        if prec != qwalk.QW_C128:  # (set_state wants a state normalised to fp64 accuracy)
            continue
        # a state set from outside runs on the full lattice
        w = qwalk.Walk((N,), inputs.RING, qwalk.DENSE, psi0, x0, prec=prec, dense=U)
        w.set_options(renorm_every=0)
        w.step(3)
        st = w.get_state()
        w.set_state(st)
        u0 = w.stats().updates
        w.step(4)
        assert w.stats().updates - u0 == N * 2 * 4
        got = w.get_state()
        w.destroy()
        w = qwalk.Walk((N,), inputs.RING, qwalk.DENSE, psi0, x0, prec=prec, dense=U)
        w.set_options(block_depth=1, renorm_every=0)
        w.step(7)
        assert np.array_equal(got, w.get_state()), N
        w.destroy()
        _, psir = _oracle_run((N,), inputs.RING, U, psi0, x0, sum(pieces))
        assert np.max(np.abs(_as_oracle_layout(res[1][-1]) - psir)) <= TOL64, N


@pytest.mark.parametrize("prec", [qwalk.QW_C128, qwalk.QW_C64])
def test_ring_real_coin_bitwise(prec):
    """Real coins (Hadamard, real rotations) take a real-arithmetic path in the
    whole-ring kernel: the same amplitudes as one step per launch (complex
    arithmetic with zero imaginary parts), and the oracle's in c128."""
    th = 0.83
    Rot = np.array([[np.cos(th), np.sin(th)], [-np.sin(th), np.cos(th)]], dtype=np.complex128)
    rng = np.random.default_rng(12)
    psi0 = inputs.haar_state(rng, 2)
    for kind, dense, oc in ((qwalk.HADAMARD, None, oracle.coin(oracle.HADAMARD, 2)), (qwalk.DENSE, Rot, Rot)):
        N, T, x0 = 3001, 700, (1500, 0)
        res = []
        for depth in (1, 0):
            _, psi, _, _ = _run_gpu((N,), inputs.RING, kind, psi0, x0, T, prec, dense=dense, block_depth=depth,
                                    renorm_every=0)
            res.append(psi)
        assert np.array_equal(res[0], res[1])
        if prec == qwalk.QW_C128:
            Pr, psir = _oracle_run((N,), inputs.RING, oc, psi0, x0, T)
            assert np.max(np.abs(_as_oracle_layout(res[1]) - psir)) <= TOL64


def test_live_kernel_timing_leaves_results_and_counts_every_launch():
    """With the profile option on, large stream launches stamp their own timing
    events and small ones are bracketed by recorded events: the amplitudes are
    those of the untimed walk bit for bit, every launch is counted once, and
    every timed kernel reports a positive time."""
    import time
    import torch
    L, T = 1024, 300                                    # boxes grow past 2^18 sites
    psi0 = inputs.haar_state(np.random.default_rng(21), 4)
    res, profs = [], []
    for prof in (0, 1):
        w = qwalk.Walk((L, L), inputs.PAIR, qwalk.GROVER, psi0, (L // 2, L // 2), prec=qwalk.QW_C128)
        w.set_options(profile=prof)
        w.profile(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w.step(T)
        torch.cuda.synchronize()
        wall_ms = 1e3 * (time.perf_counter() - t0)
        p = w.profile(reset=True)
        st = w.stats()
        res.append(w.get_state())
        profs.append((p, st, wall_ms))
        w.destroy()
    assert np.array_equal(res[0], res[1])
    p, st, wall_ms = profs[1]
    assert sum(k["launches"] for k in p.values()) == st.launches
    assert p["stream2d"]["launches"] > 0
    for name, k in p.items():
        if k["launches"]:
            assert k["ms"] > 0.0, name
    assert sum(k["ms"] for k in p.values()) <= wall_ms
    assert sum(k["launches"] for k in profs[0][0].values()) == 0     # profile off: nothing timed
