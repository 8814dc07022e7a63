"""CPU oracle for the coined quantum walk (arXiv:1003.3779).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``, never by the product package.
It shares no code with the HIP path.

The arithmetic lives in ``qw_oracle.c`` (plain complex128 loops, built with
``-O2 -ffp-contract=off``); this module only marshals numpy arrays through
ctypes.  State arrays here are complex128 of shape (Ly, Lx, d): position-major
with the coin index innermost.  A ring of N sites is the torus (1, N).

Functions and the passages they follow (see ``qw_oracle.c`` for the details):
  coin(kind, d, ...)        coin families named in Sec. 3 after Eq. (7)
  evolve(psi, ...)          T steps of U = S (I (x) C), Eqs. (2)-(3), (8), (10)
  evolve_inverse(psi, ...)  T steps of U^-1, unitarity of Eq. (2)
  prob(psi)                 P(x) = sum_c |psi(x,c)|^2, Eqs. (4)-(6)
  norm(P)                   sum_x P(x)
  bin_ring(P, x0, nbins)    symmetric binning of a ring distribution
  philox(ctr, key)          Philox4x32-10 (the random source of the broken links)
  rbl_threshold(p)          floor(p * 2^32): a link is broken when its Philox output word
                            (word 2 (y & 1) + pair of the call of its row pair) is below it
  evolve_rbl(psi, ...)      T steps with random broken links, Sec. 3 Eqs. (9)-(10), and
                            the finite segment / box with reflecting walls (Fig. 3)
  graph_reverse(off, tgt)   the other end of every arc's edge (general graphs)
  graph_evolve(off, tgt, kind, psi, T)  T steps of U = S (I (x) C) on a general graph,
                            Sec. 2.1 Eqs. (1)-(3) (one amplitude per arc)
  graph_prob(off, psi)      P(v) = sum over v's arcs of |psi|^2
  set_threads(n)            threads of the site loops (OpenMP; results are bitwise
                            independent of the count)

The spectral ring walk (psi_T through the diagonalisation of U by the lattice
Fourier transform) is in ``oracle.spectral``; the fp64 network of the learned
surrogate in ``oracle.surrogate``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qw_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

HADAMARD, SU2, GROVER, HADAMARD2, FOURIER, DENSE = range(6)

_lib = None


def build(force: bool = True) -> str:
    """Compile qw_oracle.c into liboracle.so with gcc (plain C, fp64)."""
    stale = not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    if force or stale:
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-std=c99", "-D_GNU_SOURCE", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
            _SRC, "-o", tmp, "-lm",
        ])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _open(path: str):
    """Open an oracle library and declare its signatures."""
    lib = ctypes.CDLL(path)
    i64, i32, dp, ip = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p
    lib.orc_coin.argtypes = [i32, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
    lib.orc_coin.restype = i32
    lib.orc_evolve.argtypes = [i64, i64, i32, ip, dp, dp, i64, i32, i64, i64, i64]
    lib.orc_evolve.restype = i32
    lib.orc_evolve_inverse.argtypes = [i64, i64, i32, ip, dp, dp, i64]
    lib.orc_evolve_inverse.restype = i32
    lib.orc_prob.argtypes = [i64, i32, dp, dp]
    lib.orc_prob.restype = None
    lib.orc_norm.argtypes = [i64, dp]
    lib.orc_norm.restype = ctypes.c_double
    lib.orc_bin.argtypes = [i64, i64, dp, i32, dp]
    lib.orc_bin.restype = i32
    lib.orc_philox.argtypes = [dp, dp, dp]
    lib.orc_philox.restype = None
    u64 = ctypes.c_uint64
    lib.orc_evolve_rbl.argtypes = [i64, i64, i32, ip, dp, dp, i64, i64, u64, u64, u64, i32]
    lib.orc_evolve_rbl.restype = i32
    lib.orc_graph_reverse.argtypes = [i64, dp, dp, dp]
    lib.orc_graph_reverse.restype = i32
    lib.orc_graph_evolve.argtypes = [i64, dp, dp, i32, i32, dp, dp, i64]
    lib.orc_graph_evolve.restype = i32
    lib.orc_graph_prob.argtypes = [i64, dp, dp, dp]
    lib.orc_graph_prob.restype = None
    lib.orc_set_threads.argtypes = [i32]
    lib.orc_set_threads.restype = i32
    return lib


def _load():
    global _lib
    if _lib is None:
        build(force=False)                      # compiles when missing or older than the source
        _lib = _open(_LIB_PATH)
    return _lib


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's site loops; n <= 0 keeps the current setting
    (the OpenMP default follows OMP_NUM_THREADS).  Returns the count in use."""
    return int(_load().orc_set_threads(int(n)))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def coin(kind: int, d: int, theta: float = 0.0, phi: float = 0.0, chi: float = 0.0,
         dense: np.ndarray | None = None) -> np.ndarray:
    """The d x d coin matrix of the given family (complex128)."""
    lib = _load()
    out = np.zeros((d, d), dtype=np.complex128)
    dn = None
    if dense is not None:
        dn = np.ascontiguousarray(dense, dtype=np.complex128)
        if dn.shape != (d, d):
            raise ValueError("dense coin must be d x d")
    rc = lib.orc_coin(kind, d, theta, phi, chi, _ptr(dn) if dn is not None else None, _ptr(out))
    if rc != 0:
        raise ValueError(f"orc_coin: bad coin kind={kind} d={d}")
    return out


def _disp_array(disp, d):
    a = np.ascontiguousarray(np.asarray(disp, dtype=np.int32).reshape(d, 2))
    return a


def initial_state(Lx: int, Ly: int, d: int, x0, psi0) -> np.ndarray:
    """psi_0 = |x0> (x) psi0 as a (Ly, Lx, d) complex128 array."""
    psi = np.zeros((Ly, Lx, d), dtype=np.complex128)
    psi[x0[1] % Ly, x0[0] % Lx, :] = np.asarray(psi0, dtype=np.complex128)
    return psi


def evolve(psi: np.ndarray, disp, C: np.ndarray, T: int, windowed: bool = False,
           x0=(0, 0), t0: int = 0) -> np.ndarray:
    """T steps of U = S (I (x) C) on a copy of psi (shape (Ly, Lx, d)).

    windowed=True asserts that psi vanishes outside the box of radius t0 about
    x0 and updates only the light-cone box at each step.
    """
    lib = _load()
    Ly, Lx, d = psi.shape
    out = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    da = _disp_array(disp, d)
    Cc = np.ascontiguousarray(C, dtype=np.complex128)
    rc = lib.orc_evolve(Lx, Ly, d, _ptr(da), _ptr(Cc), _ptr(out), int(T), int(bool(windowed)),
                        int(x0[0]), int(x0[1]), int(t0))
    if rc != 0:
        raise RuntimeError("orc_evolve failed")
    return out


def evolve_inverse(psi: np.ndarray, disp, C: np.ndarray, T: int) -> np.ndarray:
    """T steps of U^-1 = (I (x) C^dagger) S^-1 on a copy of psi."""
    lib = _load()
    Ly, Lx, d = psi.shape
    out = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    da = _disp_array(disp, d)
    Cc = np.ascontiguousarray(C, dtype=np.complex128)
    rc = lib.orc_evolve_inverse(Lx, Ly, d, _ptr(da), _ptr(Cc), _ptr(out), int(T))
    if rc != 0:
        raise RuntimeError("orc_evolve_inverse failed")
    return out


def prob(psi: np.ndarray) -> np.ndarray:
    """P(x) = sum_c |psi(x,c)|^2 as a (Ly, Lx) float64 array."""
    lib = _load()
    Ly, Lx, d = psi.shape
    p = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.empty((Ly, Lx), dtype=np.float64)
    lib.orc_prob(Lx * Ly, d, _ptr(p), _ptr(out))
    return out


def norm(P: np.ndarray) -> float:
    """sum_x P(x), pairwise summation."""
    lib = _load()
    p = np.ascontiguousarray(P, dtype=np.float64).ravel()
    return float(lib.orc_norm(p.size, _ptr(p)))


def bin_ring(P: np.ndarray, x0: int, nbins: int = 512) -> np.ndarray:
    """Symmetric binning of a ring distribution P (length N) about x0."""
    lib = _load()
    p = np.ascontiguousarray(P, dtype=np.float64).ravel()
    out = np.zeros(nbins, dtype=np.float64)
    rc = lib.orc_bin(p.size, int(x0), _ptr(p), int(nbins), _ptr(out))
    if rc != 0:
        raise ValueError("orc_bin: bad arguments")
    return out


def walk(Lx: int, Ly: int, disp, C: np.ndarray, x0, psi0, T: int, windowed: bool = True) -> np.ndarray:
    """psi_T for a walk started at |x0> (x) psi0 (light-cone windowed by default)."""
    d = C.shape[0]
    psi = initial_state(Lx, Ly, d, x0, psi0)
    return evolve(psi, disp, C, T, windowed=windowed, x0=x0, t0=0)


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 of a 4-word counter and a 2-word key (uint32 words)."""
    lib = _load()
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint64).astype(np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64).astype(np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def rbl_threshold(p: float) -> int:
    """floor(p * 2^32), the integer threshold of a link breaking with probability p."""
    if not (0.0 <= p <= 1.0):
        raise ValueError("p must lie in [0, 1]")
    return int(math.floor(p * 4294967296.0))


def evolve_rbl(psi: np.ndarray, disp, C: np.ndarray, T: int, p: float, seed: int = 0,
               realization: int = 0, step0: int = 0, walls: bool = False) -> np.ndarray:
    """T steps with random broken links (probability p per link and step) on a
    copy of psi; step s draws its links with step index step0 + s.  walls: the
    links across the lattice edge are always broken (segment / box)."""
    lib = _load()
    Ly, Lx, d = psi.shape
    out = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    da = _disp_array(disp, d)
    Cc = np.ascontiguousarray(C, dtype=np.complex128)
    rc = lib.orc_evolve_rbl(Lx, Ly, d, _ptr(da), _ptr(Cc), _ptr(out), int(T), int(step0),
                            rbl_threshold(p), int(seed), int(realization), int(bool(walls)))
    if rc != 0:
        raise ValueError("orc_evolve_rbl: bad arguments (every component needs an opposite)")
    return out


def _graph_arrays(off, tgt):
    o = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    t = np.ascontiguousarray(np.asarray(tgt, dtype=np.int64))
    if o.ndim != 1 or o.size < 2 or o[0] != 0 or o[-1] != t.size:
        raise ValueError("offsets must start at 0 and end at the number of arcs")
    return o, t


def graph_reverse(off, tgt) -> np.ndarray:
    """rev[k]: the arc at the other end of arc k's edge (a self-loop is its own)."""
    lib = _load()
    o, t = _graph_arrays(off, tgt)
    rev = np.zeros(t.size, dtype=np.int64)
    if lib.orc_graph_reverse(o.size - 1, _ptr(o), _ptr(t), _ptr(rev)) != 0:
        raise ValueError("arcs do not pair into undirected edges")
    return rev


def graph_evolve(off, tgt, kind: int, psi, T: int, dense=None) -> np.ndarray:
    """T steps of the coined walk on a general graph (one amplitude per arc).
    kind: GROVER, FOURIER or DENSE (dense: list of d x d matrices for d = 1 .. dmax)."""
    lib = _load()
    o, t = _graph_arrays(off, tgt)
    out = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128)).copy()
    if out.size != t.size:
        raise ValueError("one amplitude per arc")
    table, dmax = None, 0
    if dense is not None:
        dmax = len(dense)
        table = np.ascontiguousarray(np.concatenate([np.asarray(m, dtype=np.complex128).reshape(-1)
                                                     for m in dense]))
    rc = lib.orc_graph_evolve(o.size - 1, _ptr(o), _ptr(t), int(kind), int(dmax),
                              _ptr(table) if table is not None else None, _ptr(out), int(T))
    if rc != 0:
        raise ValueError("orc_graph_evolve: bad graph or coin")
    return out


def graph_prob(off, psi) -> np.ndarray:
    lib = _load()
    o = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    p = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
    P = np.empty(o.size - 1, dtype=np.float64)
    lib.orc_graph_prob(o.size - 1, _ptr(o), _ptr(p), _ptr(P))
    return P
