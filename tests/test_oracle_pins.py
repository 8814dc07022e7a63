"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's gather loop: each check comes from an
independent formulation (explicit matrix of U built from the scatter form of
the shift, path sums, exact arithmetic), a closed form, an invariant or a
special case that reduces to a textbook result.  They run on the CPU only.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from paper_1003_3779_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden", "limits.txt")


def _limits():
    out = {}
    with open(GOLD) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, val = line.split()[:2]
            out[name] = float(val)
    return out


LIMITS = _limits()


# ---------------------------------------------------------------------------
# independent formulation 1: the operator U = S (I (x) C) as an explicit matrix
# (Eqs. (2)-(3)): S|x, c> = |x + e_c, c>, the coin acts on the coin register
# ---------------------------------------------------------------------------
def dense_U(Lx, Ly, disp, C):
    d = C.shape[0]
    V = Lx * Ly
    n = V * d

    def idx(x, y, c):
        return ((y % Ly) * Lx + (x % Lx)) * d + c

    coin_part = np.kron(np.eye(V), C)            # I (x) C in the (position, coin) basis
    S = np.zeros((n, n), dtype=np.complex128)
    for y in range(Ly):
        for x in range(Lx):
            for c in range(d):
                ex, ey = disp[c]
                S[idx(x + ex, y + ey, c), idx(x, y, c)] += 1.0
    return S @ coin_part


def random_state(rng, Lx, Ly, d):
    z = rng.normal(size=(Ly, Lx, d)) + 1j * rng.normal(size=(Ly, Lx, d))
    return z / np.linalg.norm(z)


COIN_CASES_1D = [
    ("hadamard", lambda rng: oracle.coin(oracle.HADAMARD, 2)),
    ("su2", lambda rng: oracle.coin(oracle.SU2, 2, *inputs.su2_angles(rng, 1)[0])),
    ("grover2", lambda rng: oracle.coin(oracle.GROVER, 2)),
    ("fourier2", lambda rng: oracle.coin(oracle.FOURIER, 2)),
    ("haar", lambda rng: inputs.haar_unitary(rng, 2)),
]
COIN_CASES_2D = [
    ("grover", lambda rng: oracle.coin(oracle.GROVER, 4)),
    ("hh", lambda rng: oracle.coin(oracle.HADAMARD2, 4)),
    ("fourier", lambda rng: oracle.coin(oracle.FOURIER, 4)),
    ("haar", lambda rng: inputs.haar_unitary(rng, 4)),
]


@pytest.mark.parametrize("N", [1, 2, 3, 5, 8, 9])
@pytest.mark.parametrize("coin_name,coin_fn", COIN_CASES_1D)
def test_dense_matrix_power_ring(N, coin_name, coin_fn):
    rng = np.random.default_rng(100 + N)
    C = coin_fn(rng)
    U = dense_U(N, 1, inputs.RING, C)
    psi = random_state(rng, N, 1, 2)
    for T in (1, 2, 7):
        want = (np.linalg.matrix_power(U, T) @ psi.ravel()).reshape(psi.shape)
        got = oracle.evolve(psi, inputs.RING, C, T)
        assert np.max(np.abs(got - want)) <= 1e-13


@pytest.mark.parametrize("shape", [(3, 3), (4, 5), (6, 4), (5, 6)])
@pytest.mark.parametrize("table", ["PAIR", "EQ8", "DIAG"])
@pytest.mark.parametrize("coin_name,coin_fn", COIN_CASES_2D)
def test_dense_matrix_power_torus(shape, table, coin_name, coin_fn):
    Lx, Ly = shape
    disp = getattr(inputs, table)
    rng = np.random.default_rng(Lx * 10 + Ly)
    C = coin_fn(rng)
    U = dense_U(Lx, Ly, disp, C)
    psi = random_state(rng, Lx, Ly, 4)
    for T in (1, 3, 6):
        want = (np.linalg.matrix_power(U, T) @ psi.ravel()).reshape(psi.shape)
        got = oracle.evolve(psi, disp, C, T)
        assert np.max(np.abs(got - want)) <= 1e-13


def test_dense_matrix_power_windowed_start():
    """The windowed sweep from a single-site start equals the matrix power."""
    rng = np.random.default_rng(7)
    for disp in (inputs.PAIR, inputs.DIAG):
        C = inputs.haar_unitary(rng, 4)
        U = dense_U(7, 6, disp, C)
        psi0 = inputs.haar_state(rng, 4)
        x0 = (3, 2)
        start = oracle.initial_state(7, 6, 4, x0, psi0)
        for T in (1, 2, 5, 9):
            want = (np.linalg.matrix_power(U, T) @ start.ravel()).reshape(start.shape)
            got = oracle.walk(7, 6, disp, C, x0, psi0, T, windowed=True)
            assert np.max(np.abs(got - want)) <= 1e-13


# ---------------------------------------------------------------------------
# independent formulation 2: path sums over all coin sequences
# ---------------------------------------------------------------------------
def path_sum(Lx, Ly, disp, C, x0, psi0, T):
    """psi_T(x, c) = sum over component sequences (c_1..c_T) of
    C[c_T][c_{T-1}] ... C[c_1][c_0] psi0[c_0], landing at x0 + sum_t e_{c_t}."""
    d = C.shape[0]
    out = np.zeros((Ly, Lx, d), dtype=np.complex128)
    for seq in itertools.product(range(d), repeat=T):
        amp_vec = psi0.copy()                    # amplitude per c_0
        x, y = x0
        prev = None
        amp = None
        # amplitude of the path = sum_{c_0} prod C[c_t][c_{t-1}] psi0[c_0]
        for t, c in enumerate(seq):
            if t == 0:
                amp = np.dot(C[c, :], amp_vec)
            else:
                amp = C[c, prev] * amp
            prev = c
            x += disp[c][0]
            y += disp[c][1]
        out[y % Ly, x % Lx, seq[-1]] += amp
    return out


@pytest.mark.parametrize("T", [1, 2, 5, 9])
def test_path_sum_ring(T):
    rng = np.random.default_rng(T)
    C = inputs.haar_unitary(rng, 2)
    psi0 = inputs.haar_state(rng, 2)
    N = 2 * T + 3
    want = path_sum(N, 1, inputs.RING, C, (T + 1, 0), psi0, T)
    got = oracle.walk(N, 1, inputs.RING, C, (T + 1, 0), psi0, T)
    assert np.max(np.abs(got - want)) <= 1e-13


@pytest.mark.parametrize("table", ["PAIR", "EQ8", "DIAG"])
def test_path_sum_torus(table):
    disp = getattr(inputs, table)
    rng = np.random.default_rng(11)
    C = inputs.haar_unitary(rng, 4)
    psi0 = inputs.haar_state(rng, 4)
    T = 5
    want = path_sum(13, 12, disp, C, (6, 5), psi0, T)
    got = oracle.walk(13, 12, disp, C, (6, 5), psi0, T)
    assert np.max(np.abs(got - want)) <= 1e-13


def test_hadamard_exact_rational():
    """Exact P_t(x) of the Hadamard walk in Q(sqrt 2, i) (sympy path sum) vs the oracle."""
    sympy = pytest.importorskip("sympy")
    s = sympy.sqrt(2) / 2
    H = [[s, s], [s, -s]]
    psi0 = [sympy.I * s, s]
    T = 8
    amps = {}
    for seq in itertools.product(range(2), repeat=T):
        a = H[seq[0]][0] * psi0[0] + H[seq[0]][1] * psi0[1]
        for t in range(1, T):
            a = H[seq[t]][seq[t - 1]] * a
        x = sum(1 if c == 0 else -1 for c in seq)
        key = (x, seq[-1])
        amps[key] = amps.get(key, 0) + a
    P = {}
    for (x, c), a in amps.items():
        P[x] = P.get(x, 0) + sympy.nsimplify(sympy.expand(a * sympy.conjugate(a)))
    N = 2 * T + 1
    x0 = T
    got = oracle.prob(oracle.walk(N, 1, inputs.RING, oracle.coin(oracle.HADAMARD, 2), (x0, 0), inputs.PSI0_LR, T))
    for x, p in P.items():
        assert p.is_rational
        assert abs(got[0, x0 + x] - float(p)) <= 1e-15
    assert sum(P.values()) == 1


# ---------------------------------------------------------------------------
# invariants and special cases
# ---------------------------------------------------------------------------
def test_norm_conserved_ring1d():
    cfg = inputs.config("ring1d")
    N = cfg["extent"][0]
    C = oracle.coin(oracle.HADAMARD, 2)
    psi = oracle.walk(N, 1, cfg["disp"], C, cfg["x0"], cfg["psi0"], cfg["T"])
    assert abs(oracle.norm(oracle.prob(psi)) - 1.0) <= 1e-12


def test_norm_conserved_torus():
    rng = np.random.default_rng(5)
    C = inputs.haar_unitary(rng, 4)
    psi = oracle.walk(64, 48, inputs.PAIR, C, (31, 17), inputs.haar_state(rng, 4), 200, windowed=False)
    assert abs(oracle.norm(oracle.prob(psi)) - 1.0) <= 1e-12


def test_mirror_symmetry_hadamard():
    """The Hadamard walk from (|L> + i|R>)/sqrt 2 is mirror symmetric about x0."""
    cfg = inputs.config("ring1d")
    N, x0 = cfg["extent"][0], cfg["x0"][0]
    P = oracle.prob(oracle.walk(N, 1, cfg["disp"], oracle.coin(oracle.HADAMARD, 2), cfg["x0"], cfg["psi0"], cfg["T"]))[0]
    x = np.arange(1, 1001)
    assert np.max(np.abs(P[x0 + x] - P[x0 - x])) <= 1e-15
    # and it is genuinely spread (not trivially symmetric): the peaks sit near |x| = T/sqrt 2
    assert np.argmax(P[x0:]) > 600


def test_asymmetric_start_is_not_symmetric():
    """Control for the mirror pin: the start |R> alone drifts to one side."""
    P = oracle.prob(oracle.walk(401, 1, inputs.RING, oracle.coin(oracle.HADAMARD, 2), (200, 0),
                                np.array([1, 0], dtype=complex), 200))[0]
    x = np.arange(-200, 201)
    assert np.sum(P * x) > 20.0


@pytest.mark.parametrize("table", ["RING", "PAIR", "EQ8", "DIAG"])
def test_site_parity_and_light_cone(table):
    disp = getattr(inputs, table)
    d = len(disp)
    rng = np.random.default_rng(3)
    C = inputs.haar_unitary(rng, d)
    if d == 2:
        Lx, Ly, x0 = 61, 1, (30, 0)
    else:
        Lx, Ly, x0 = 41, 39, (20, 19)
    psi0 = inputs.haar_state(rng, d)
    for T in (0, 1, 4, 13):
        full = oracle.walk(Lx, Ly, disp, C, x0, psi0, T, windowed=False)
        win = oracle.walk(Lx, Ly, disp, C, x0, psi0, T, windowed=True)
        assert np.array_equal(full, win)                 # windowed sweep == full sweep (value-exact)
        P = oracle.prob(full)
        yy, xx = np.meshgrid(np.arange(Ly) - x0[1], np.arange(Lx) - x0[0], indexing="ij")
        outside = np.maximum(np.abs(xx), np.abs(yy)) > T
        assert np.all(P[outside] == 0.0)
        if table == "DIAG":
            wrong = ((xx - T) % 2 != 0) | ((yy - T) % 2 != 0)
        else:
            wrong = (xx + yy - T) % 2 != 0
        assert np.all(P[wrong] == 0.0)
        assert np.any(P[~wrong] > 0.0)


def _moments(P, x0):
    x = np.arange(P.size) - x0
    return float(np.sum(P * x)), float(np.sum(P * x * x))


def test_hadamard_variance_limit():
    cfg = inputs.config("ring1d")
    N, x0, T = cfg["extent"][0], cfg["x0"][0], cfg["T"]
    P = oracle.prob(oracle.walk(N, 1, cfg["disp"], oracle.coin(oracle.HADAMARD, 2), cfg["x0"], cfg["psi0"], T))[0]
    m1, m2 = _moments(P, x0)
    var = m2 - m1 * m1
    assert abs(m1) <= 1e-10
    assert abs(var / T ** 2 - LIMITS["hadamard_var_limit"]) <= 1e-5


@pytest.mark.parametrize("theta", [0.3, 0.9, 2.0])
def test_su2_second_moment_limit(theta):
    """E[X_t^2]/t^2 -> 1 - |b| for a 2x2 coin whose off-diagonal modulus is |b| = |sin theta|."""
    rng = np.random.default_rng(int(theta * 10))
    phi, chi = rng.uniform(0, 2 * math.pi, 2)
    C = oracle.coin(oracle.SU2, 2, theta, phi, chi)
    T = 600
    N = 2 * T + 1
    P = oracle.prob(oracle.walk(N, 1, inputs.RING, C, (T, 0), inputs.haar_state(rng, 2), T))[0]
    _, m2 = _moments(P, T)
    assert abs(m2 / T ** 2 - (1 - abs(math.sin(theta)))) <= 1e-4


def test_su2_is_unitary_and_special():
    rng = np.random.default_rng(1)
    for th, ph, ch in inputs.su2_angles(rng, 20):
        C = oracle.coin(oracle.SU2, 2, th, ph, ch)
        assert np.max(np.abs(C.conj().T @ C - np.eye(2))) <= 1e-15
        assert abs(np.linalg.det(C) - 1.0) <= 1e-15


def test_hadamard_equals_su2_up_to_phase():
    """H = i C(pi/4, -pi/2, -pi/2): amplitudes agree up to i^T, P agrees."""
    Csu2 = oracle.coin(oracle.SU2, 2, math.pi / 4, -math.pi / 2, -math.pi / 2)
    H = oracle.coin(oracle.HADAMARD, 2)
    assert np.max(np.abs(1j * Csu2 - H)) <= 1e-15
    T = 300
    a = oracle.walk(2 * T + 1, 1, inputs.RING, H, (T, 0), inputs.PSI0_LR, T)
    b = oracle.walk(2 * T + 1, 1, inputs.RING, Csu2, (T, 0), inputs.PSI0_LR, T)
    assert np.max(np.abs(a - (1j ** T) * b)) <= 1e-13
    assert np.max(np.abs(oracle.prob(a) - oracle.prob(b))) <= 1e-14


def test_su2_gauge_invariance():
    """P is unchanged under (phi, chi) -> (phi + a, chi + a) for a single-site start."""
    rng = np.random.default_rng(9)
    psi0 = inputs.haar_state(rng, 2)
    T = 250
    P1 = oracle.prob(oracle.walk(2 * T + 1, 1, inputs.RING, oracle.coin(oracle.SU2, 2, 0.7, 0.4, 1.9), (T, 0), psi0, T))
    P2 = oracle.prob(oracle.walk(2 * T + 1, 1, inputs.RING, oracle.coin(oracle.SU2, 2, 0.7, 0.4 + 1.1, 1.9 + 1.1), (T, 0), psi0, T))
    assert np.max(np.abs(P1 - P2)) <= 1e-14
    # control: changing phi alone does change P
    P3 = oracle.prob(oracle.walk(2 * T + 1, 1, inputs.RING, oracle.coin(oracle.SU2, 2, 0.7, 0.4 + 1.1, 1.9), (T, 0), psi0, T))
    assert np.max(np.abs(P1 - P3)) > 1e-4


def test_su2_reduces_to_real_rotation():
    """For P alone, the SU(2) walk C(theta, phi, chi) from psi0 equals the walk with
    the real rotation [[cos t, sin t], [-sin t, cos t]] from (psi0_0, e^{i(chi-phi)} psi0_1):
    the gauge (phi, chi) -> (phi - phi, chi - phi) plus conjugation by diag(1, e^{i(chi-phi)}),
    which commutes with the shift.  (Used by the batched walks, whose outputs are P only.)"""
    rng = np.random.default_rng(31)
    for th, ph, ch in inputs.su2_angles(rng, 6):
        psi0 = inputs.haar_state(rng, 2)
        N, T, x0 = 301, 150, (150, 0)
        P = oracle.prob(oracle.walk(N, 1, inputs.RING, oracle.coin(oracle.SU2, 2, th, ph, ch), x0, psi0, T))
        R = np.array([[math.cos(th), math.sin(th)], [-math.sin(th), math.cos(th)]], dtype=complex)
        psi0r = np.array([psi0[0], np.exp(1j * (ch - ph)) * psi0[1]])
        Pr = oracle.prob(oracle.walk(N, 1, inputs.RING, R, x0, psi0r, T))
        assert np.max(np.abs(P - Pr)) <= 1e-14
        # control: without the phase on the second component the distributions differ
        Pw = oracle.prob(oracle.walk(N, 1, inputs.RING, R, x0, psi0, T))
        if abs(math.sin(ch - ph)) > 0.1 and abs(psi0[0] * psi0[1]) > 0.05:
            assert np.max(np.abs(P - Pw)) > 1e-6


@pytest.mark.parametrize("table", ["RING", "PAIR", "DIAG"])
def test_exact_reversal(table):
    disp = getattr(inputs, table)
    d = len(disp)
    rng = np.random.default_rng(21)
    C = inputs.haar_unitary(rng, d)
    Lx, Ly = (37, 1) if d == 2 else (17, 14)
    psi = random_state(rng, Lx, Ly, d)
    fwd = oracle.evolve(psi, disp, C, 25)
    back = oracle.evolve_inverse(fwd, disp, C, 25)
    assert np.max(np.abs(back - psi)) <= 1e-12
    assert np.max(np.abs(fwd - psi)) > 1e-3


def test_inverse_matches_matrix_inverse():
    rng = np.random.default_rng(4)
    C = inputs.haar_unitary(rng, 4)
    U = dense_U(4, 5, inputs.EQ8, C)
    psi = random_state(rng, 4, 5, 4)
    want = (np.linalg.inv(U) @ psi.ravel()).reshape(psi.shape)
    got = oracle.evolve_inverse(psi, inputs.EQ8, C, 1)
    assert np.max(np.abs(got - want)) <= 1e-13


def _origin_prob(disp, psi0, T, L):
    G = oracle.coin(oracle.GROVER, 4)
    x0 = (L // 2, L // 2)
    P = oracle.prob(oracle.walk(L, L, disp, G, x0, psi0, T))
    return P[x0[1], x0[0]]


def test_grover_localisation_pair_ordering():
    """With opposite directions paired, the start (1,-1,-1,1)/2 localises:
    P(origin, t) -> 4/pi^2 for even t, with an error that falls ~ 1/t^2."""
    lim = LIMITS["grover_loc_origin_limit"]
    p64 = _origin_prob(inputs.PAIR, inputs.PSI0_GROVER_LOC, 64, 131)
    p128 = _origin_prob(inputs.PAIR, inputs.PSI0_GROVER_LOC, 128, 259)
    e64, e128 = abs(p64 - lim), abs(p128 - lim)
    assert e128 <= 1e-4
    assert 2.5 <= e64 / e128 <= 6.0


def test_grover_no_localisation_eq8_ordering():
    """Same amplitudes in the order of Eq. (8) pair opposite directions with equal
    signs: the walker leaves the origin."""
    p = _origin_prob(inputs.EQ8, inputs.PSI0_GROVER_LOC, 128, 259)
    assert p <= 1e-3


def test_grover_uniform_start_keeps_origin_weight():
    p = _origin_prob(inputs.PAIR, inputs.PSI0_GROVER_UNI, 128, 259)
    assert p >= 0.5


def test_diagonal_hh_factorises():
    """Diagonal lattice + H(x)H + product start u (x) w = product of two 1D Hadamard walks."""
    rng = np.random.default_rng(12)
    u, w = inputs.haar_state(rng, 2), inputs.haar_state(rng, 2)
    T, L = 40, 83
    psi0 = np.kron(u, w)                          # c = 2j + k, j the first factor
    HH = oracle.coin(oracle.HADAMARD2, 4)
    H = oracle.coin(oracle.HADAMARD, 2)
    P2 = oracle.prob(oracle.walk(L, L, inputs.DIAG, HH, (41, 41), psi0, T))
    Pu = oracle.prob(oracle.walk(L, 1, inputs.RING, H, (41, 0), u, T))[0]
    Pw = oracle.prob(oracle.walk(L, 1, inputs.RING, H, (41, 0), w, T))[0]
    assert np.max(np.abs(P2 - np.outer(Pw, Pu))) <= 1e-15


def test_hh_is_kron():
    H = oracle.coin(oracle.HADAMARD, 2)
    assert np.max(np.abs(oracle.coin(oracle.HADAMARD2, 4) - np.kron(H, H))) <= 1e-15
    F = oracle.coin(oracle.FOURIER, 4)
    assert np.max(np.abs(F - np.array([[1j ** (a * b) for b in range(4)] for a in range(4)]) / 2)) <= 1e-15
    G = oracle.coin(oracle.GROVER, 4)
    assert np.max(np.abs(G @ G - np.eye(4))) <= 1e-15


def test_1d_embedded_in_2d():
    """Natural lattice, coin H on the +-x pair (+) H on the +-y pair, start in the
    +-x pair: the 2D walk stays on the row y0 and reproduces the 1D walk."""
    H = oracle.coin(oracle.HADAMARD, 2)
    C = np.zeros((4, 4), dtype=complex)
    C[:2, :2] = H
    C[2:, 2:] = H
    T, L = 60, 125
    psi0 = np.concatenate([inputs.PSI0_LR, [0, 0]])
    P2 = oracle.prob(oracle.walk(L, 9, inputs.PAIR, C, (62, 4), psi0, T))
    P1 = oracle.prob(oracle.walk(L, 1, inputs.RING, H, (62, 0), inputs.PSI0_LR, T))[0]
    assert np.max(np.abs(P2[4] - P1)) <= 1e-15
    assert np.all(np.delete(P2, 4, axis=0) == 0.0)


def test_shift_tables_follow_eq8():
    """EQ8 is Eq. (8): (j,k) moves (m,n) by ((-1)^j (1 - delta_jk), (-1)^j delta_jk)."""
    for j in (0, 1):
        for k in (0, 1):
            dl = 1 if j == k else 0
            assert inputs.EQ8[2 * j + k] == ((-1) ** j * (1 - dl), (-1) ** j * dl)
            assert inputs.DIAG[2 * j + k] == ((-1) ** j, (-1) ** k)


def test_binning_symmetric_and_complete():
    cfg_T = 600
    N = 4097
    x0 = 2048
    P = oracle.prob(oracle.walk(N, 1, inputs.RING, oracle.coin(oracle.HADAMARD, 2), (x0, 0), inputs.PSI0_LR, cfg_T))[0]
    b = oracle.bin_ring(P, x0, 512)
    assert abs(b.sum() - P.sum()) <= 1e-13
    assert np.max(np.abs(b - b[::-1])) <= 1e-14
    # bin 256 + j covers offsets 8j+1 .. 8j+8 (plus half the start site for j = 0)
    j = 20
    assert abs(b[256 + j] - P[x0 + 8 * j + 1: x0 + 8 * j + 9].sum()) <= 1e-15
    assert abs(b[255 - j] - P[x0 - 8 * j - 8: x0 - 8 * j].sum()) <= 1e-15
