"""The torus streaming kernel with workgroup-wide strips (waves side by side
on 256 columns, edge columns exchanged through LDS; with real coins each
complex number split over two lanes) against the one-wave strips, the
one-step kernel and the oracle.

Every stored amplitude is the same expression in the same order whichever
kernel computes it, so the variants must agree bit for bit; complex128 runs
must also match the oracle to 1e-12 max-abs, complex64 runs to 2e-5 on P.
Tori are at least 256 sites wide (the variant's minimum), with ragged strips
and segments, and cones that cross both seams.  Inputs are seeded; expected
values come from the oracle only.
"""
import numpy as np
import pytest

import oracle
from paper_1003_3779_amd import inputs, qwalk

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32_P = 2e-5
# stream_kernel: one-wave strips; workgroup strips (real coins: each complex
# number split over two lanes); workgroup strips with complex lanes
WAVE, WG, WGC = 1, 2, 3


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    qwalk.load()
    yield


def _run(extent, disp, kind, psi0, x0, T, prec, dense=None, **opts):
    w = qwalk.Walk(extent, disp, kind, psi0, x0, prec=prec, dense=dense)
    w.set_options(**opts)
    w.step(T)
    P = w.probabilities()
    psi = w.get_state()
    n = w.norm()
    w.destroy()
    return P, psi, n


def _oracle(extent, disp, C, psi0, x0, T):
    psi = oracle.walk(extent[0], extent[1], disp, C, x0, psi0, T)
    return oracle.prob(psi), np.transpose(psi, (2, 0, 1))


COINS = [("grover", qwalk.GROVER, oracle.GROVER), ("hh", qwalk.HADAMARD2, oracle.HADAMARD2),
         ("haar", qwalk.DENSE, None)]


@pytest.mark.parametrize("prec", [qwalk.QW_C128, qwalk.QW_C64])
@pytest.mark.parametrize("table", ["PAIR", "EQ8"])
@pytest.mark.parametrize("coin_name,kind,okind", COINS)
def test_wg_strips_bitwise_and_vs_oracle(prec, table, coin_name, kind, okind):
    """Depths 4, 8, 12, 16 on workgroup strips equal the one-step kernel bit
    for bit (and the one-wave strips where they have the depth); the cone
    crosses the x and y seams of a 301 x 90 torus (two strips, the second
    ragged; rows wrap)."""
    disp = getattr(inputs, table)
    rng = np.random.default_rng(1000 + 10 * prec + len(table) + kind)
    dense = inputs.haar_unitary(rng, 4) if kind == qwalk.DENSE else None
    C = dense if dense is not None else oracle.coin(okind, 4)
    psi0 = inputs.haar_state(rng, 4)
    ext, x0, T = (301, 90), (17, 80), 101
    print(f"# wg: prec={prec} table={table} coin={coin_name}", flush=True)
    _, ref, _ = _run(ext, disp, kind, psi0, x0, T, prec, dense=dense, block_depth=1, renorm_every=0)
    for depth in (4, 8, 12, 16):
        for variant in (WG, WGC):
            _, psi, _ = _run(ext, disp, kind, psi0, x0, T, prec, dense=dense, block_depth=depth,
                             stream_kernel=variant, renorm_every=0)
            assert np.array_equal(psi, ref), (depth, variant)
        if prec == qwalk.QW_C64 or depth <= 8:
            _, psi_w, _ = _run(ext, disp, kind, psi0, x0, T, prec, dense=dense, block_depth=depth,
                               stream_kernel=WAVE, renorm_every=0)
            assert np.array_equal(psi_w, ref), depth
    Pr, psir = _oracle(ext, disp, C, psi0, x0, T)
    P, psi, n = _run(ext, disp, kind, psi0, x0, T, prec, dense=dense, stream_kernel=WG)
    if prec == qwalk.QW_C128:
        assert np.max(np.abs(psi - psir)) <= TOL64
        assert np.max(np.abs(P - Pr)) <= TOL64
        assert abs(n - 1.0) <= TOL64
    else:
        assert np.max(np.abs(P - Pr)) <= TOL32_P
        assert abs(n - 1.0) <= 1e-5


@pytest.mark.parametrize("prec", [qwalk.QW_C128, qwalk.QW_C64])
def test_wg_launch_shape_is_bitwise_neutral(prec):
    """Segment length (target waves), read-ahead rows and block order change only
    which workgroup computes which rows and when loads are issued (complex lanes
    for a Haar coin, split lanes for the Grover coin)."""
    rng = np.random.default_rng(2024 + prec)
    U = inputs.haar_unitary(rng, 4)
    psi0 = inputs.haar_state(rng, 4)
    ext, x0, T = (517, 263), (250, 5), 120   # three strips (the last ragged), rows wrap
    for kind, dense, C in ((qwalk.DENSE, U, U), (qwalk.GROVER, None, oracle.coin(oracle.GROVER, 4))):
        for depth in (8, 12):
            res = []
            for pd, waves, order in ((3, 0, 0), (1, 0, 2), (3, 4, 1), (3, 37, 2), (1, 5000, 1), (3, 100000, 2)):
                _, psi, _ = _run(ext, inputs.PAIR, kind, psi0, x0, T, prec, dense=dense, block_depth=depth,
                                 stream_kernel=WG, prefetch_rows=pd, stream_waves=waves, block_order=order,
                                 renorm_every=0)
                res.append(psi)
            for r in res[1:]:
                assert np.array_equal(res[0], r), (kind, depth)
        if prec == qwalk.QW_C128:
            Pr, psir = _oracle(ext, inputs.PAIR, C, psi0, x0, T)
            assert np.max(np.abs(res[0] - psir)) <= TOL64


def test_wg_cone_wraps_whole_torus():
    """A cone wider than the torus in both axes (every site updated, strips
    overlapping the seam): workgroup strips against the oracle."""
    rng = np.random.default_rng(99)
    U = inputs.haar_unitary(rng, 4)
    psi0 = inputs.haar_state(rng, 4)
    ext, x0, T = (258, 40), (255, 1), 170
    for table in ("PAIR", "EQ8"):
        disp = getattr(inputs, table)
        for kind, dense, C in ((qwalk.DENSE, U, U), (qwalk.HADAMARD2, None, oracle.coin(oracle.HADAMARD2, 4))):
            P, psi, n = _run(ext, disp, kind, psi0, x0, T, qwalk.QW_C128, dense=dense, block_depth=8,
                             stream_kernel=WG)
            Pr, psir = _oracle(ext, disp, C, psi0, x0, T)
            assert np.max(np.abs(psi - psir)) <= TOL64, (table, kind)
            assert abs(n - 1.0) <= TOL64


def test_wg_preference_falls_back():
    """Asking for workgroup strips on a walk they cannot take (diagonal table,
    a torus narrower than 256 sites) runs the one-wave strips: same result."""
    rng = np.random.default_rng(5)
    U = inputs.haar_unitary(rng, 4)
    psi0 = inputs.haar_state(rng, 4)
    for ext, table in (((300, 64), "DIAG"), ((200, 100), "PAIR")):
        disp = getattr(inputs, table)
        _, a, _ = _run(ext, disp, qwalk.DENSE, psi0, (100, 30), 40, qwalk.QW_C128, dense=U, block_depth=8,
                       stream_kernel=WG)
        _, b, _ = _run(ext, disp, qwalk.DENSE, psi0, (100, 30), 40, qwalk.QW_C128, dense=U, block_depth=1)
        assert np.array_equal(a, b), table


@pytest.mark.parametrize("Ly", [1, 2, 3, 5, 31])
def test_wg_short_tori(Ly):
    """Tori of 1 to 31 rows (every row wraps onto itself within a launch) on
    workgroup strips, both lane layouts, against the one-step kernel bit for bit
    and the oracle."""
    rng = np.random.default_rng(700 + Ly)
    psi0 = inputs.haar_state(rng, 4)
    ext, x0, T = (300, Ly), (290, Ly // 2), 37
    _, ref, _ = _run(ext, inputs.PAIR, qwalk.GROVER, psi0, x0, T, qwalk.QW_C128, block_depth=1)
    for depth in (4, 12):
        for variant in (WG, WGC):
            _, psi, _ = _run(ext, inputs.PAIR, qwalk.GROVER, psi0, x0, T, qwalk.QW_C128, block_depth=depth,
                             stream_kernel=variant)
            assert np.array_equal(psi, ref), (depth, variant)
    _, psir = _oracle(ext, inputs.PAIR, oracle.coin(oracle.GROVER, 4), psi0, x0, T)
    assert np.max(np.abs(ref - psir)) <= TOL64
