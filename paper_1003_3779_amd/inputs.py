"""Seeded synthetic inputs for the coined-walk workloads.

This module holds data and random draws only -- no step of the walk itself --
so that the CPU oracle and the HIP path can be fed the very same arrays.

Displacement tables (the vector e_c that coin component c moves along) are
literal data:
  RING   1D ring, c = 0 -> right (+1), c = 1 -> left (-1): the coin space is
         |R> (+) |L> (Sec. 2.2, Eq. (4)); the listing of the segment kernel
         (Fig. 2) gathers component 0 from the left neighbour and component 1
         from the right one, i.e. component 0 moves right.
  PAIR   2D natural lattice, c = (+x, -x, +y, -y): opposite directions are
         the pairs {0,1} and {2,3}.
  EQ8    2D natural lattice in the order of the shift of Eq. (8) with
         c = 2j + k: (0,+1), (+1,0), (-1,0), (0,-1) in (x, y) = (m, n).
  DIAG   2D diagonal lattice (Fig. 1c, Tables 2-3): e_{2j+k} = ((-1)^j, (-1)^k).
"""
from __future__ import annotations

import math

import numpy as np

RING = ((1, 0), (-1, 0))
PAIR = ((1, 0), (-1, 0), (0, 1), (0, -1))
EQ8 = ((0, 1), (1, 0), (-1, 0), (0, -1))
DIAG = ((1, 1), (1, -1), (-1, 1), (-1, -1))

# coin kinds (same numbering as the C ABI and the oracle)
HADAMARD, SU2, GROVER, HADAMARD2, FOURIER, DENSE = range(6)

SQRT1_2 = 1.0 / math.sqrt(2.0)

# 1D start coin state (|L> + i|R>)/sqrt(2) in (R, L) component order
PSI0_LR = np.array([1j * SQRT1_2, SQRT1_2], dtype=np.complex128)
# 2D Grover start states in the PAIR ordering
PSI0_GROVER_LOC = np.array([0.5, -0.5, -0.5, 0.5], dtype=np.complex128)
PSI0_GROVER_UNI = np.array([0.5, 0.5, 0.5, 0.5], dtype=np.complex128)
# the "Fourier initial state" of the Fourier-coin walks (Fig. 4): read as the
# Fourier coin applied to |0>, i.e. the uniform coin state
PSI0_FOURIER = np.array([0.5, 0.5, 0.5, 0.5], dtype=np.complex128)


def haar_state(rng: np.random.Generator, d: int) -> np.ndarray:
    """A Haar-random unit vector in C^d: a complex Gaussian, normalised."""
    z = rng.normal(size=d) + 1j * rng.normal(size=d)
    return (z / np.linalg.norm(z)).astype(np.complex128)


def haar_unitary(rng: np.random.Generator, d: int) -> np.ndarray:
    """A Haar-random d x d unitary (QR of a complex Gaussian, phases fixed)."""
    z = (rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return (q * ph[None, :]).astype(np.complex128)


def su2_angles(rng: np.random.Generator, n: int) -> np.ndarray:
    """n SU(2) coin angle triples: theta ~ U(0, pi), phi, chi ~ U(0, 2 pi)."""
    out = np.empty((n, 3), dtype=np.float64)
    out[:, 0] = rng.uniform(0.0, math.pi, size=n)
    out[:, 1] = rng.uniform(0.0, 2 * math.pi, size=n)
    out[:, 2] = rng.uniform(0.0, 2 * math.pi, size=n)
    return out


def ragged_ring_batch(seed: int, n: int, nmin: int = 1001, nmax: int = 999999,
                      tmin: int = 256) -> dict:
    """Parameters of n independent rings: N odd in [nmin, nmax], T in [tmin, N//2],
    SU(2) angles and Haar start coin states, drawn in that order from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N = 2 * rng.integers(nmin // 2, nmax // 2, size=n, endpoint=True) + 1
    T = np.array([rng.integers(tmin, max(tmin, int(k) // 2), endpoint=True) for k in N], dtype=np.int64)
    ang = su2_angles(rng, n)
    psi0 = np.stack([haar_state(rng, 2) for _ in range(n)])
    return {"N": N.astype(np.int64), "T": T, "angles": ang, "psi0": psi0}


def config(name: str) -> dict:
    """The fixed workloads (sizes, coins, start states) used by tests and bench."""
    if name == "ring1d":        # 1D Hadamard ring, N = 2001, T = 1000, complex128
        return dict(dim=1, extent=(2001, 1), disp=RING, coin=HADAMARD, x0=(1000, 0),
                    psi0=PSI0_LR, T=1000, prec="c128")
    if name == "grover2d":      # 2D Grover torus 4096^2, T = 2048, localising start
        return dict(dim=2, extent=(4096, 4096), disp=PAIR, coin=GROVER, x0=(2048, 2048),
                    psi0=PSI0_GROVER_LOC, T=2048, prec="c128")
    if name == "grover2d_uniform":
        return dict(dim=2, extent=(4096, 4096), disp=PAIR, coin=GROVER, x0=(2048, 2048),
                    psi0=PSI0_GROVER_UNI, T=2048, prec="c128")
    if name == "fourier2d_diag":     # the paper's 2D workload shape (Fig. 4, Tables 2-3): diagonal
        return dict(dim=2, extent=(500, 500), disp=DIAG, coin=FOURIER, x0=(250, 250),   # lattice,
                    psi0=PSI0_FOURIER, T=250, prec="c128")                              # Size 500
    if name == "fourier2d_natural":  # the same walk on the natural lattice of Eq. (8)
        return dict(dim=2, extent=(500, 500), disp=EQ8, coin=FOURIER, x0=(250, 250),
                    psi0=PSI0_FOURIER, T=250, prec="c128")
    if name == "fourier2d_diag_4096":  # the diagonal Fourier walk at the benchmark torus size
        return dict(dim=2, extent=(4096, 4096), disp=DIAG, coin=FOURIER, x0=(2048, 2048),
                    psi0=PSI0_FOURIER, T=2048, prec="c128")
    if name == "hh2d":          # 2D H(x)H torus 16384^2, T = 4096, complex64, Haar start (seed 3)
        rng = np.random.Generator(np.random.PCG64(3))
        return dict(dim=2, extent=(16384, 16384), disp=PAIR, coin=HADAMARD2, x0=(8192, 8192),
                    psi0=haar_state(rng, 4), T=4096, prec="c64")
    raise KeyError(name)
