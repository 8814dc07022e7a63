"""Why the learned surrogate cannot answer at total-variation distance 1e-3:
the floor, measured on the oracle (CPU only, no network involved).

The surrogate maps (theta, phi, chi, start state, T) of a ring walk of
N = 4097 sites to its 512 binned probabilities.  Two properties of the exact
map, computed here with the oracle on seeded coins and start states, bound
how close any smooth approximation of it can come:

* the step count: the binned distribution after T and after T + 2 steps
  differs by TVD >= 2e-2 (the interference between the two branches of the
  walk's dispersion relation oscillates with T at every binned position), so
  a network must resolve T exactly and follow a function that oscillates
  through hundreds of periods over T in [256, 2048];
* the coin angle: moving theta by 1e-3 rad moves the bins by TVD >= 1e-2
  (after 300 steps; more the longer the walk), so a TVD of 1e-3 needs theta
  to about 1e-4 rad.  bf16 features carry sin and cos of theta to a relative
  2^-9: rounding only the coin angle to what bf16 features can represent
  moves the exact bins by more than 1e-3 for most coins.

The re-check and fallback therefore answer every walk at 1e-3 with the plain
walk; the surrogate's speed is reported at looser tolerances.  Expected
values come from the oracle only.
"""
import numpy as np
import pytest

import oracle
from paper_1003_3779_amd import inputs

N = 4097
X0 = N // 2


def _bins(theta, phi, chi, psi0, T):
    C = oracle.coin(oracle.SU2, 2, theta, phi, chi)
    P = oracle.prob(oracle.walk(N, 1, inputs.RING, C, (X0, 0), psi0, T))[0]
    return oracle.bin_ring(P, X0, 512)


def _tvd(a, b):
    return 0.5 * float(np.abs(a - b).sum())


def _draws(seed, n):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        th = rng.uniform(0.0, np.pi)
        ph, ch = rng.uniform(0.0, 2 * np.pi, 2)
        out.append((th, ph, ch, inputs.haar_state(rng, 2)))
    return out


@pytest.fixture(scope="module", autouse=True)
def threads():
    oracle.set_threads(0)
    yield


@pytest.mark.parametrize("T", [300, 1000, 2000])
def test_bins_change_by_far_more_than_1e3_from_T_to_T_plus_2(T):
    for th, ph, ch, psi0 in _draws(123, 4):
        a, b = _bins(th, ph, ch, psi0, T), _bins(th, ph, ch, psi0, T + 2)
        assert abs(a.sum() - 1.0) < 1e-12 and abs(b.sum() - 1.0) < 1e-12
        assert _tvd(a, b) >= 2e-2, (th, T)


@pytest.mark.parametrize("T", [300, 2000])
def test_bins_move_by_far_more_than_1e3_when_theta_moves_by_1e3(T):
    for th, ph, ch, psi0 in _draws(124, 4):
        assert _tvd(_bins(th, ph, ch, psi0, T), _bins(th + 1e-3, ph, ch, psi0, T)) >= 1e-2, (th, T)


def _bf16(v):
    """Round float64 values to bfloat16 (nearest even), returned as float64."""
    f = np.asarray(v, dtype=np.float32).view(np.uint32).astype(np.uint64)
    f = (f + 0x7FFF + ((f >> 16) & 1)) & 0xFFFF0000
    return f.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_features_cannot_pin_theta_to_1e3_tvd():
    """The coin angle a bf16 feature pair (sin theta, cos theta) can name is
    up to about 2^-9 rad away from the true one; at T = 2000 that alone moves
    the exact bins by more than TVD 1e-3 for most coins."""
    over = 0
    draws = _draws(125, 8)
    for th, ph, ch, psi0 in draws:
        thq = float(np.arctan2(_bf16(np.sin(th)), _bf16(np.cos(th))))
        if _tvd(_bins(th, ph, ch, psi0, 2000), _bins(thq, ph, ch, psi0, 2000)) > 1e-3:
            over += 1
    assert over >= len(draws) // 2
