"""Pins of the spectral ring oracle (CPU only).

The spectral oracle evaluates psi_T = U^T psi_0 through the lattice Fourier
transform; the gather oracle steps the walk site by site.  They share no
code, so agreement on many rings, coins and step counts (wrapping ones
included) pins the spectral formulation, and closed forms pin it where only
it can go (T up to 5e5).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import spectral
from paper_1003_3779_amd import inputs


@pytest.mark.parametrize("N,T", [(1, 5), (2, 7), (3, 9), (7, 30), (64, 100), (513, 600), (1000, 333),
                                 (4097, 2048), (1001, 3001), (20011, 150)])
def test_equals_gather_oracle(N, T):
    rng = np.random.default_rng(N * 13 + T)
    U = inputs.haar_unitary(rng, 2)
    psi0 = inputs.haar_state(rng, 2)
    x0 = int(rng.integers(0, N))
    ref = oracle.walk(N, 1, inputs.RING, U, (x0, 0), psi0, T, windowed=False)[0]
    got = spectral.ring_walk(N, U, x0, psi0, T)
    assert np.max(np.abs(got - ref)) <= 1e-12
    Pg = spectral.ring_prob(N, U, x0, psi0, T)
    assert np.max(np.abs(Pg - oracle.prob(ref[None])[0])) <= 1e-12


def test_other_table_and_su2():
    """The table enters through the phases of D(k): the swapped ring table and
    the SU(2) family agree with the gather oracle too."""
    rng = np.random.default_rng(5)
    swapped = ((-1, 0), (1, 0))
    for th in (0.2, 1.3, 2.8):
        C = oracle.coin(oracle.SU2, 2, th, *rng.uniform(0, 2 * math.pi, 2))
        psi0 = inputs.haar_state(rng, 2)
        for disp in (inputs.RING, swapped):
            ref = oracle.walk(301, 1, disp, C, (150, 0), psi0, 140)[0]
            got = spectral.ring_walk(301, C, 150, psi0, 140, disp)
            assert np.max(np.abs(got - ref)) <= 1e-12


def test_planted_mistakes_are_caught():
    """A wrong phase sign, a transposed coin and a dropped step each move the
    result far from the gather oracle."""
    rng = np.random.default_rng(9)
    U = inputs.haar_unitary(rng, 2)
    psi0 = inputs.haar_state(rng, 2)
    N, T, x0 = 257, 90, 100
    ref = oracle.walk(N, 1, inputs.RING, U, (x0, 0), psi0, T)[0]
    assert np.max(np.abs(spectral.ring_walk(N, U, x0, psi0, T, ((-1, 0), (1, 0))) - ref)) > 1e-3
    assert np.max(np.abs(spectral.ring_walk(N, U.T, x0, psi0, T) - ref)) > 1e-3
    assert np.max(np.abs(spectral.ring_walk(N, U, x0, psi0, T - 1) - ref)) > 1e-3


def test_norm_and_mirror_symmetry_long():
    """The Hadamard walk from (|L> + i|R>)/sqrt 2 after 10^5 steps: norm 1 within
    the powering's rounding (T eps) and P symmetric about the start."""
    N, T = 200003, 100000
    x0 = N // 2
    P = spectral.ring_prob(N, oracle.coin(oracle.HADAMARD, 2), x0, inputs.PSI0_LR, T)
    assert abs(P.sum() - 1.0) <= 1e-10
    off = np.arange(1, T + 1)
    assert np.max(np.abs(P[x0 + off] - P[x0 - off])) <= 1e-12
    # site parity: only offsets with the parity of T are occupied
    assert np.max(P[x0 + np.arange(-T + 1, T, 2)]) <= 1e-20


@pytest.mark.parametrize("theta", [0.4, 1.1, 2.5])
def test_su2_second_moment_limit_long(theta):
    """E[(x - x0)^2] / T^2 -> 1 - |sin theta| for the SU(2) walk (a closed form of
    the asymptotic spreading; the finite-T correction is O(1/T)), at T = 2e5."""
    rng = np.random.default_rng(int(theta * 10))
    phi, chi = rng.uniform(0, 2 * math.pi, 2)
    C = oracle.coin(oracle.SU2, 2, theta, phi, chi)
    N, T = 400003, 200000
    x0 = N // 2
    P = spectral.ring_prob(N, C, x0, inputs.haar_state(rng, 2), T)
    dx = np.arange(N) - x0
    m2 = float(np.sum(P * dx.astype(np.float64) ** 2)) / T ** 2
    assert abs(m2 - (1.0 - abs(math.sin(theta)))) <= 1e-3
