"""Spectral oracle of the ring walk (test infrastructure only).

TEST INFRASTRUCTURE ONLY: used by ``tests/`` to check long ring walks whose
step-by-step oracle (``qw_oracle.c``) would run for hours.  It shares no code
with the HIP path and none with the gather loops of ``qw_oracle.c``.

What it computes.  The walk on a ring of N sites is psi_T = U^T psi_0 with
U = S (I (x) C) (Sec. 2.1, Eq. (2)); the shift S moves component c by e_c
(Eq. (3); on the ring e_0 = +1, e_1 = -1).  U commutes with translations, so
the lattice Fourier transform
    psi^(k, c) = sum_x exp(-2 pi i k x / N) psi(x, c),   k = 0 .. N-1,
block-diagonalises it: one step is psi^'(k) = M(k) psi^(k) with the d x d
matrix
    M(k) = D(k) C,   D(k) = diag_c exp(-2 pi i k e_c / N),
because psi'(x, c) = sum_c' C[c][c'] psi(x - e_c, c') turns the translation by
e_c into the phase exp(-2 pi i k e_c / N).  Hence psi^_T(k) = M(k)^T psi^_0(k)
and psi_T is the inverse transform.  This is U^T psi_0 exactly (up to
rounding), evaluated in another basis: M(k)^T by binary powering (about
2 log2 T small matrix products per k), the transforms by numpy's FFT.

Rounding: binary powering multiplies the relative error of M^T by about T
(T * 1.1e-16 = 5.5e-11 at T = 5e5); the transforms add O(eps log N).  Far
below the 2e-5 budget of complex64 walks it checks; against the gather oracle
it agrees to 1e-12 on the rings the tests pin it with.
"""
from __future__ import annotations

import numpy as np


def _phase(num: np.ndarray, N: int) -> np.ndarray:
    """exp(-2 pi i num / N) for integer num, reduced modulo N first (exact)."""
    r = np.mod(num, N).astype(np.float64)
    return np.exp(-2j * np.pi * r / N)


def step_matrices(N: int, C: np.ndarray, disp) -> np.ndarray:
    """M(k) = D(k) C for k = 0 .. N-1, shape (N, d, d)."""
    C = np.asarray(C, dtype=np.complex128)
    d = C.shape[0]
    e = [int(np.asarray(disp[c]).reshape(-1)[0]) for c in range(d)]
    k = np.arange(N, dtype=np.int64)
    M = np.empty((N, d, d), dtype=np.complex128)
    for c in range(d):
        M[:, c, :] = _phase(k * e[c], N)[:, None] * C[c, :][None, :]
    return M


def matrix_power_apply(M: np.ndarray, v: np.ndarray, T: int) -> np.ndarray:
    """M^T v per k (M: (N, d, d), v: (N, d)) by binary powering of T."""
    if T < 0:
        raise ValueError("T must be >= 0")
    v = np.array(v, dtype=np.complex128)
    P = np.array(M, dtype=np.complex128)
    t = int(T)
    while t > 0:
        if t & 1:
            v = np.einsum("kab,kb->ka", P, v)
        t >>= 1
        if t:
            P = np.matmul(P, P)
    return v


def ring_walk(N: int, C: np.ndarray, x0: int, psi0, T: int, disp=((1, 0), (-1, 0))) -> np.ndarray:
    """psi_T of the ring walk started at |x0> (x) psi0, shape (N, d) complex128."""
    C = np.asarray(C, dtype=np.complex128)
    d = C.shape[0]
    k = np.arange(N, dtype=np.int64)
    v0 = _phase(k * int(x0), N)[:, None] * np.asarray(psi0, dtype=np.complex128).reshape(1, d)
    vT = matrix_power_apply(step_matrices(N, C, disp), v0, T)
    return np.fft.ifft(vT, axis=0)


def ring_prob(N: int, C: np.ndarray, x0: int, psi0, T: int, disp=((1, 0), (-1, 0))) -> np.ndarray:
    """P(x) = sum_c |psi_T(x, c)|^2 (c ascending) of ring_walk."""
    psi = ring_walk(N, C, x0, psi0, T, disp)
    P = np.zeros(N, dtype=np.float64)
    for c in range(psi.shape[1]):
        P += psi[:, c].real ** 2 + psi[:, c].imag ** 2
    return P
