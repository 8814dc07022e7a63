"""ctypes binding of libqwalk.so (C ABI in include/qwalk.h).

Argument marshalling only: every step of the walk runs in the library's HIP
kernels.  Names follow the C entry points.  Device buffers may be given as
torch tensors (their ``data_ptr()`` is passed) and streams as
``torch.cuda.Stream`` objects (their ``cuda_stream`` handle is passed); torch
is plumbing here, never compute.

There is no fallback: if ``libqwalk.so`` is missing or cannot be loaded, every
entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

QW_OK, QW_EINVAL, QW_ENOMEM, QW_EHIP, QW_ERANGE, QW_ENOTNORM = 0, -1, -2, -3, -4, -5
QW_C128, QW_C64 = 0, 1
HADAMARD, SU2, GROVER, HADAMARD2, FOURIER, DENSE = range(6)

_STATUS_NAMES = {0: "QW_OK", -1: "QW_EINVAL", -2: "QW_ENOMEM", -3: "QW_EHIP", -4: "QW_ERANGE", -5: "QW_ENOTNORM"}

# every symbol the header declares (checked by the tests)
ABI_SYMBOLS = (
    "walk_create", "walk_create_ext", "walk_scratch_bytes", "walk_state_bytes", "walk_step", "walk_step_inverse",
    "walk_probabilities", "walk_norm", "walk_get_state", "walk_set_state", "walk_set_options",
    "walk_get_options", "walk_time", "walk_stats", "walk_destroy", "walk_last_error",
    "walk_reset", "walk_profile", "walk_set_broken_links", "walk_set_reflecting_walls", "walk_run_noalloc",
    "walk_batch_create", "walk_batch_run", "walk_batch_moments", "walk_batch_binned",
    "walk_batch_probabilities", "walk_batch_info", "walk_batch_tune", "walk_batch_destroy",
    "walk_batch_last_error",
    "surr_num_params", "surr_create", "surr_get_params", "surr_set_params", "surr_features", "surr_forward",
    "surr_loss_grad", "surr_train", "surr_set_range", "surr_predict", "surr_save", "surr_load",
    "surr_destroy", "surr_last_error",
    "graph_walk_create", "graph_walk_reset", "graph_walk_step", "graph_walk_probabilities", "graph_walk_norm",
    "graph_walk_get_state", "graph_walk_info", "graph_walk_destroy", "graph_walk_last_error",
)
KERNEL_NAMES = ("step", "ring_whole", "ring_tiles", "stream2d")


class GraphInfo(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64), ("narcs", ctypes.c_int64), ("max_degree", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("t", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("step_ms", ctypes.c_double), ("bytes_per_step", ctypes.c_double)]


class QWError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Lattice(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("d", ctypes.c_int32), ("extent", ctypes.c_int64 * 2),
                ("disp", (ctypes.c_int32 * 2) * 4)]


class Coin(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("theta", ctypes.c_double), ("phi", ctypes.c_double),
                ("chi", ctypes.c_double), ("dense", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("block_depth", ctypes.c_int32), ("window", ctypes.c_int32),
                ("renorm_every", ctypes.c_int64), ("renorm_tol", ctypes.c_double),
                ("profile", ctypes.c_int32), ("prefetch_rows", ctypes.c_int32),
                ("stream_waves", ctypes.c_int32), ("block_order", ctypes.c_int32),
                ("stream_kernel", ctypes.c_int32)]


class KernelProfile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("bytes_read", ctypes.c_double),
                ("bytes_written", ctypes.c_double), ("updates", ctypes.c_double), ("min_bytes", ctypes.c_double)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("nbins", ctypes.c_int32), ("keep_probabilities", ctypes.c_int32),
                ("tiled_variant", ctypes.c_int32), ("no_graph", ctypes.c_int32),
                ("renorm_every", ctypes.c_int32), ("whole_max_sites", ctypes.c_int32),
                ("walls", ctypes.c_int32), ("full_lattice", ctypes.c_int32),
                ("link_p", ctypes.c_double), ("link_seed", ctypes.c_uint64),
                ("realization0", ctypes.c_uint64)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("grid", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("whole_ring_walks", ctypes.c_int64), ("est_updates", ctypes.c_double),
                ("last_run_ms", ctypes.c_double), ("bucket_cfg", ctypes.c_int32 * 3),
                ("bucket_tile_sites", ctypes.c_int32 * 3), ("bucket_depth", ctypes.c_int32 * 3),
                ("reserved", ctypes.c_int32), ("est_cone_updates", ctypes.c_double)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("epochs", ctypes.c_int32), ("lr", ctypes.c_float),
                ("lr_floor", ctypes.c_float), ("weight_decay", ctypes.c_float), ("epoch_offset", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("schedule_epochs", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PredictOpts(ctypes.Structure):
    _fields_ = [("recheck_frac", ctypes.c_double), ("tvd_tol", ctypes.c_double), ("chunk", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("out_on_device", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PredictStats(ctypes.Structure):
    _fields_ = [("out_of_range", ctypes.c_int64), ("rechecked", ctypes.c_int64), ("failed_chunks", ctypes.c_int64),
                ("fallback", ctypes.c_int64), ("max_tvd_sampled", ctypes.c_double), ("ms_network", ctypes.c_double),
                ("ms_recheck", ctypes.c_double), ("ms_fallback", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("renorm_checks", ctypes.c_int64), ("renorms", ctypes.c_int64),
                ("last_norm", ctypes.c_double), ("launches", ctypes.c_int64), ("updates", ctypes.c_int64)]


_lib = None


def load():
    """Open libqwalk.so (built in-tree by ``build.build_library``)."""
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"libqwalk.so is not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "walk_create": [P, P, P, P, I32, P, P],
        "walk_create_ext": [P, P, P, P, I32, P, P, P, P, P],
        "walk_run_noalloc": [P, P, P, P, I32, P, P, P, P, I64, P, P],
        "walk_scratch_bytes": [P],
        "walk_state_bytes": [P, I32, P],
        "walk_step": [P, I64],
        "walk_step_inverse": [P, I64],
        "walk_probabilities": [P, P, I32],
        "walk_norm": [P, P],
        "walk_get_state": [P, P, I32],
        "walk_set_state": [P, P, I32],
        "walk_set_options": [P, P],
        "walk_get_options": [P, P],
        "walk_time": [P, P],
        "walk_stats": [P, P],
        "walk_destroy": [P],
        "walk_reset": [P, P, P],
        "walk_profile": [P, P, I32],
        "walk_set_broken_links": [P, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64],
        "walk_set_reflecting_walls": [P, I32],
        "walk_batch_create": [I64, P, P, P, P, P, I32, P, P, P],
        "walk_batch_run": [P],
        "walk_batch_moments": [P, P, I32],
        "walk_batch_binned": [P, P, I32],
        "walk_batch_probabilities": [P, P, P, I32],
        "walk_batch_info": [P, P],
        "walk_batch_tune": [P, I32, I32],
        "walk_batch_destroy": [P],
        "surr_create": [ctypes.c_uint64, P, P],
        "surr_get_params": [P, P, I32],
        "surr_set_params": [P, P],
        "surr_features": [P, I64, P, P, P, P, P],
        "surr_forward": [P, I64, P, P, P],
        "surr_loss_grad": [P, I64, P, P, P, P, P],
        "surr_train": [P, I64, P, P, P, P, P],
        "surr_set_range": [P, I64, I32, I32],
        "surr_predict": [P, I64, P, P, P, P, P, P, P, P],
        "surr_save": [P, ctypes.c_char_p],
        "surr_load": [ctypes.c_char_p, P, P],
        "surr_destroy": [P],
        "graph_walk_create": [I64, P, P, I32, P, I32, P, I32, P, P],
        "graph_walk_reset": [P, P],
        "graph_walk_step": [P, I64],
        "graph_walk_probabilities": [P, P, I32],
        "graph_walk_norm": [P, P],
        "graph_walk_get_state": [P, P, I32],
        "graph_walk_info": [P, P],
        "graph_walk_destroy": [P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.surr_num_params.argtypes = []
    lib.surr_num_params.restype = ctypes.c_int64
    for name in ("walk_last_error", "walk_batch_last_error", "surr_last_error", "graph_walk_last_error"):
        f = getattr(lib, name)
        f.argtypes = []
        f.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int):
    if rc != QW_OK:
        msg = load().walk_last_error().decode(errors="replace")
        raise QWError(rc, msg)


def _ptr_of(buf):
    """Device pointer of a torch tensor, or an int address."""
    if buf is None:
        return None
    if hasattr(buf, "data_ptr"):
        return ctypes.c_void_p(buf.data_ptr())
    return ctypes.c_void_p(int(buf))


def _stream_of(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def make_lattice(extent, disp) -> Lattice:
    disp = [tuple(int(v) for v in e) for e in disp]
    d = len(disp)
    lat = Lattice()
    lat.dim = 1 if d == 2 else 2
    lat.d = d
    lat.extent[0] = int(extent[0])
    lat.extent[1] = int(extent[1]) if len(extent) > 1 else 1
    for c, (dx, dy) in enumerate(disp):
        lat.disp[c][0] = dx
        lat.disp[c][1] = dy
    return lat


class Walk:
    """One walk: ``walk_create`` ... ``walk_destroy`` on a handle."""

    def __init__(self, extent, disp, coin_kind: int, psi0, x0, prec: int = QW_C128,
                 theta: float = 0.0, phi: float = 0.0, chi: float = 0.0, dense=None,
                 stream=None, state_buffers=None, scratch=None, dim: int | None = None):
        lib = load()
        self._lib = lib
        self.lattice = make_lattice(extent, disp)
        if dim is not None:
            self.lattice.dim = dim
        self.d = self.lattice.d
        self.V = int(self.lattice.extent[0]) * (int(self.lattice.extent[1]) if self.lattice.dim == 2 else 1)
        self.Lx = int(self.lattice.extent[0])
        self.Ly = int(self.lattice.extent[1]) if self.lattice.dim == 2 else 1
        self.prec = prec
        self._dense = None
        coin = Coin()
        coin.kind = coin_kind
        coin.theta, coin.phi, coin.chi = theta, phi, chi
        if dense is not None:
            dn = np.ascontiguousarray(np.asarray(dense, dtype=np.complex128))
            self._dense = dn
            coin.dense = dn.ctypes.data
        p0 = np.ascontiguousarray(np.asarray(psi0, dtype=np.complex128))
        x0a = (ctypes.c_int64 * 2)(int(x0[0]), int(x0[1]) if len(x0) > 1 else 0)
        h = ctypes.c_void_p()
        self._keep = (state_buffers, scratch)
        if state_buffers is None:
            rc = lib.walk_create(ctypes.byref(self.lattice), ctypes.byref(coin), p0.ctypes.data, x0a, prec,
                                 _stream_of(stream), ctypes.byref(h))
        else:
            a, b = state_buffers
            rc = lib.walk_create_ext(ctypes.byref(self.lattice), ctypes.byref(coin), p0.ctypes.data, x0a, prec,
                                     _stream_of(stream), _ptr_of(a), _ptr_of(b),
                                     _ptr_of(scratch) if scratch is not None else None, ctypes.byref(h))
        _check(rc)
        self.h = h

    # -- ABI calls --
    def step(self, T: int):
        _check(self._lib.walk_step(self.h, int(T)))

    def step_inverse(self, T: int):
        _check(self._lib.walk_step_inverse(self.h, int(T)))

    def probabilities(self, out=None) -> np.ndarray | None:
        """P(x) as a (Ly, Lx) float64 host array, or into a device tensor ``out``."""
        if out is not None:
            _check(self._lib.walk_probabilities(self.h, _ptr_of(out), 1))
            return None
        P = np.empty((self.Ly, self.Lx), dtype=np.float64)
        _check(self._lib.walk_probabilities(self.h, P.ctypes.data, 0))
        return P

    def norm(self) -> float:
        v = ctypes.c_double()
        _check(self._lib.walk_norm(self.h, ctypes.byref(v)))
        return v.value

    def get_state(self, out=None) -> np.ndarray | None:
        """psi as a (d, Ly, Lx) complex128 host array (or into a device tensor)."""
        if out is not None:
            _check(self._lib.walk_get_state(self.h, _ptr_of(out), 1))
            return None
        s = np.empty((self.d, self.Ly, self.Lx), dtype=np.complex128)
        _check(self._lib.walk_get_state(self.h, s.ctypes.data, 0))
        return s

    def set_state(self, psi):
        """psi: (d, Ly, Lx) complex128 host array, or a device tensor of the same bytes."""
        if hasattr(psi, "data_ptr"):
            _check(self._lib.walk_set_state(self.h, _ptr_of(psi), 1))
            return
        s = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
        if s.size != self.d * self.V:
            raise ValueError("state has the wrong size")
        _check(self._lib.walk_set_state(self.h, s.ctypes.data, 0))

    def reset(self, psi0, x0):
        p0 = np.ascontiguousarray(np.asarray(psi0, dtype=np.complex128))
        x0a = (ctypes.c_int64 * 2)(int(x0[0]), int(x0[1]) if len(x0) > 1 else 0)
        _check(self._lib.walk_reset(self.h, p0.ctypes.data, x0a))

    def set_broken_links(self, p: float, seed: int = 0, realization: int = 0):
        """Random broken links (probability p per link and step; p = 0: intact).
        Only at t = 0; walk_reset keeps the setting."""
        _check(self._lib.walk_set_broken_links(self.h, float(p), int(seed), int(realization)))

    def set_reflecting_walls(self, on: bool = True):
        """Finite segment / box: the links across the lattice edge always broken.
        Only at t = 0; walk_reset keeps the setting."""
        _check(self._lib.walk_set_reflecting_walls(self.h, int(bool(on))))

    def profile(self, reset: bool = False) -> dict:
        """Per-kernel totals of the launches timed while the profile option was on."""
        arr = (KernelProfile * len(KERNEL_NAMES))()
        _check(self._lib.walk_profile(self.h, arr, int(bool(reset))))
        out = {}
        for name, k in zip(KERNEL_NAMES, arr):
            out[name] = {"launches": k.launches, "ms": k.ms, "bytes_read": k.bytes_read,
                         "bytes_written": k.bytes_written, "updates": k.updates, "min_bytes": k.min_bytes}
        return out

    def set_options(self, block_depth: int | None = None, window: int | None = None,
                    renorm_every: int | None = None, renorm_tol: float | None = None,
                    profile: int | None = None, prefetch_rows: int | None = None,
                    stream_waves: int | None = None, block_order: int | None = None,
                    stream_kernel: int | None = None):
        o = self.get_options()
        if stream_kernel is not None:
            o.stream_kernel = int(stream_kernel)
        if block_order is not None:
            o.block_order = int(block_order)
        if stream_waves is not None:
            o.stream_waves = int(stream_waves)
        if prefetch_rows is not None:
            o.prefetch_rows = int(prefetch_rows)
        if profile is not None:
            o.profile = int(profile)
        if block_depth is not None:
            o.block_depth = block_depth
        if window is not None:
            o.window = window
        if renorm_every is not None:
            o.renorm_every = renorm_every
        if renorm_tol is not None:
            o.renorm_tol = renorm_tol
        _check(self._lib.walk_set_options(self.h, ctypes.byref(o)))

    def get_options(self) -> Options:
        o = Options()
        _check(self._lib.walk_get_options(self.h, ctypes.byref(o)))
        return o

    def time(self) -> int:
        t = ctypes.c_int64()
        _check(self._lib.walk_time(self.h, ctypes.byref(t)))
        return t.value

    def stats(self) -> Stats:
        s = Stats()
        _check(self._lib.walk_stats(self.h, ctypes.byref(s)))
        return s

    def destroy(self):
        if getattr(self, "h", None) is not None and self.h.value is not None:
            rc = self._lib.walk_destroy(self.h)
            self.h = ctypes.c_void_p()
            _check(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def state_bytes(extent, disp, prec: int) -> int:
    lat = make_lattice(extent, disp)
    n = ctypes.c_size_t()
    _check(load().walk_state_bytes(ctypes.byref(lat), prec, ctypes.byref(n)))
    return n.value


def run_noalloc(extent, disp, coin_kind: int, psi0, x0, T: int, state_buffers, prec: int = QW_C128,
                P_out=None, want_norm: bool = True, options: "Options | None" = None, stream=None,
                theta: float = 0.0, phi: float = 0.0, chi: float = 0.0, dense=None):
    """One whole walk through walk_run_noalloc (no device allocation inside the
    call): the caller's two state buffers, P into the device tensor P_out (or
    none); returns the norm (host float) when want_norm, else None."""
    lib = load()
    lat = make_lattice(extent, disp)
    coin = Coin()
    coin.kind = coin_kind
    coin.theta, coin.phi, coin.chi = theta, phi, chi
    dn = None
    if dense is not None:
        dn = np.ascontiguousarray(np.asarray(dense, dtype=np.complex128))
        coin.dense = dn.ctypes.data
    p0 = np.ascontiguousarray(np.asarray(psi0, dtype=np.complex128))
    x0a = (ctypes.c_int64 * 2)(int(x0[0]), int(x0[1]) if len(x0) > 1 else 0)
    a, b = state_buffers
    nrm = ctypes.c_double()
    _check(lib.walk_run_noalloc(ctypes.byref(lat), ctypes.byref(coin), p0.ctypes.data, x0a, prec,
                                ctypes.byref(options) if options is not None else None, _stream_of(stream),
                                _ptr_of(a), _ptr_of(b), int(T), _ptr_of(P_out) if P_out is not None else None,
                                ctypes.byref(nrm) if want_norm else None))
    return nrm.value if want_norm else None


def scratch_bytes() -> int:
    """Bytes of the scratch buffer walk_create_ext takes."""
    n = ctypes.c_size_t()
    _check(load().walk_scratch_bytes(ctypes.byref(n)))
    return n.value


def _bcheck(rc: int):
    if rc != QW_OK:
        msg = load().walk_batch_last_error().decode(errors="replace")
        raise QWError(rc, msg)


class Batch:
    """Independent ring walks in one persistent launch (walk_batch_*).  The options
    are those of qw_batch_opts; full_lattice=True makes the tiled rings update both
    parities of their light cone (by default a ring whose cone never wraps keeps
    only the live parity: the same results, half the work)."""

    def __init__(self, N, T, angles, psi0, x0=None, prec: int = QW_C64, nbins: int = 0,
                 keep_probabilities: bool = False, tiled_variant: int = 0, no_graph: bool = False,
                 renorm_every: int = 0, stream=None, whole_max_sites: int = 0, walls: bool = False,
                 link_p: float = 0.0, link_seed: int = 0, realization0: int = 0, full_lattice: bool = False):
        lib = load()
        self._lib = lib
        self.N = np.ascontiguousarray(np.asarray(N, dtype=np.int64))
        self.T = np.ascontiguousarray(np.asarray(T, dtype=np.int64))
        n = self.N.size
        ang = np.ascontiguousarray(np.asarray(angles, dtype=np.float64).reshape(n, 3))
        p0 = np.ascontiguousarray(np.asarray(psi0, dtype=np.complex128).reshape(n, 2))
        xa = None if x0 is None else np.ascontiguousarray(np.asarray(x0, dtype=np.int64))
        self.n, self.nbins, self.keep = n, nbins, keep_probabilities
        o = BatchOpts(nbins, int(bool(keep_probabilities)), int(tiled_variant), int(bool(no_graph)),
                      int(renorm_every), int(whole_max_sites), int(bool(walls)), int(bool(full_lattice)),
                      float(link_p),
                      int(link_seed), int(realization0))
        h = ctypes.c_void_p()
        _bcheck(lib.walk_batch_create(n, self.N.ctypes.data, self.T.ctypes.data, ang.ctypes.data, p0.ctypes.data,
                                      None if xa is None else xa.ctypes.data, prec, ctypes.byref(o),
                                      _stream_of(stream), ctypes.byref(h)))
        self.h = h

    def run(self):
        _bcheck(self._lib.walk_batch_run(self.h))

    def moments(self) -> np.ndarray:
        out = np.empty((self.n, 3), dtype=np.float64)
        _bcheck(self._lib.walk_batch_moments(self.h, out.ctypes.data, 0))
        return out

    def binned(self, out=None):
        if out is not None:
            _bcheck(self._lib.walk_batch_binned(self.h, _ptr_of(out), 1))
            return None
        b = np.empty((self.n, self.nbins), dtype=np.float32)
        _bcheck(self._lib.walk_batch_binned(self.h, b.ctypes.data, 0))
        return b

    def probabilities(self, out=None) -> list | None:
        """Every walk's P(x), walk after walk: a list of host arrays, or into
        `out` (a device tensor of sum(N) float64)."""
        if out is not None:
            _bcheck(self._lib.walk_batch_probabilities(self.h, _ptr_of(out), None, 1))
            return None
        flat = np.empty(int(self.N.sum()), dtype=np.float64)
        off = np.empty(self.n + 1, dtype=np.int64)
        _bcheck(self._lib.walk_batch_probabilities(self.h, flat.ctypes.data, off.ctypes.data, 0))
        return [flat[off[i]:off[i + 1]] for i in range(self.n)]

    def info(self) -> BatchInfo:
        i = BatchInfo()
        _bcheck(self._lib.walk_batch_info(self.h, ctypes.byref(i)))
        return i

    def tune(self, samples: int = 8, save: bool = False):
        _bcheck(self._lib.walk_batch_tune(self.h, int(samples), int(bool(save))))

    def destroy(self):
        if getattr(self, "h", None) is not None and self.h.value is not None:
            rc = self._lib.walk_batch_destroy(self.h)
            self.h = ctypes.c_void_p()
            _bcheck(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _scheck(rc: int):
    if rc != QW_OK:
        msg = load().surr_last_error().decode(errors="replace")
        raise QWError(rc, msg)


def _walk_arrays(N, T, angles, psi0):
    N = np.ascontiguousarray(np.asarray(N, dtype=np.int64))
    T = np.ascontiguousarray(np.asarray(T, dtype=np.int64))
    n = N.size
    ang = np.ascontiguousarray(np.asarray(angles, dtype=np.float64).reshape(n, 3))
    p0 = np.ascontiguousarray(np.asarray(psi0, dtype=np.complex128).reshape(n, 2))
    return n, N, T, ang, p0


class Surrogate:
    """The learned surrogate (surr_*): features -> network -> 512 bins, with
    the plain walk as fallback and arbiter."""

    NBINS = 512
    NFEAT = 32

    def __init__(self, seed: int = 0, stream=None, _handle=None):
        lib = load()
        self._lib = lib
        if _handle is not None:
            self.h = _handle
            return
        h = ctypes.c_void_p()
        _scheck(lib.surr_create(int(seed), _stream_of(stream), ctypes.byref(h)))
        self.h = h

    @classmethod
    def load_file(cls, path: str, stream=None) -> "Surrogate":
        lib = load()
        h = ctypes.c_void_p()
        _scheck(lib.surr_load(path.encode(), _stream_of(stream), ctypes.byref(h)))
        return cls(_handle=h)

    @staticmethod
    def num_params() -> int:
        return int(load().surr_num_params())

    def params(self, bf16_rounded: bool = False) -> np.ndarray:
        out = np.empty(self.num_params(), dtype=np.float32)
        _scheck(self._lib.surr_get_params(self.h, out.ctypes.data, int(bool(bf16_rounded))))
        return out

    def set_params(self, flat):
        a = np.ascontiguousarray(np.asarray(flat, dtype=np.float32))
        if a.size != self.num_params():
            raise ValueError("wrong parameter count")
        _scheck(self._lib.surr_set_params(self.h, a.ctypes.data))

    def features(self, N, T, angles, psi0) -> np.ndarray:
        n, N, T, ang, p0 = _walk_arrays(N, T, angles, psi0)
        out = np.empty((n, self.NFEAT), dtype=np.float32)
        _scheck(self._lib.surr_features(self.h, n, N.ctypes.data, T.ctypes.data, ang.ctypes.data, p0.ctypes.data,
                                        out.ctypes.data))
        return out

    def forward(self, X, T) -> np.ndarray:
        X = np.ascontiguousarray(np.asarray(X, dtype=np.float32))
        T = np.ascontiguousarray(np.asarray(T, dtype=np.int32))
        out = np.empty((X.shape[0], self.NBINS), dtype=np.float32)
        _scheck(self._lib.surr_forward(self.h, X.shape[0], X.ctypes.data, T.ctypes.data, out.ctypes.data))
        return out

    def loss_grad(self, X, Y, T):
        X = np.ascontiguousarray(np.asarray(X, dtype=np.float32))
        Y = np.ascontiguousarray(np.asarray(Y, dtype=np.float32))
        T = np.ascontiguousarray(np.asarray(T, dtype=np.int32))
        loss = ctypes.c_double()
        g = np.empty(self.num_params(), dtype=np.float32)
        _scheck(self._lib.surr_loss_grad(self.h, X.shape[0], X.ctypes.data, Y.ctypes.data, T.ctypes.data,
                                         ctypes.byref(loss), g.ctypes.data))
        return loss.value, g

    def train(self, X_dev, Y_dev, T_dev, n: int, batch: int = 1024, epochs: int = 10, lr: float = 1e-3,
              lr_floor: float = 0.05, weight_decay: float = 0.0, seed: int = 0, epoch_offset: int = 0,
              schedule_epochs: int = 0) -> np.ndarray:
        """X_dev (n x 32 float32), Y_dev (n x 512 float32), T_dev (n int32): device tensors."""
        o = TrainOpts(batch, epochs, lr, lr_floor, weight_decay, epoch_offset, seed, schedule_epochs, 0)
        hist = np.zeros(epochs, dtype=np.float32)
        _scheck(self._lib.surr_train(self.h, int(n), _ptr_of(X_dev), _ptr_of(Y_dev), _ptr_of(T_dev),
                                     ctypes.byref(o), hist.ctypes.data))
        return hist

    def set_range(self, N: int, tmin: int, tmax: int):
        _scheck(self._lib.surr_set_range(self.h, int(N), int(tmin), int(tmax)))

    def predict(self, N, T, angles, psi0, recheck_frac: float = 0.01, tvd_tol: float = 1e-3, chunk: int = 1024,
                seed: int = 1, out=None):
        """Binned P of the walks; out: None (a new host array) or a contiguous
        float32 CUDA tensor of n x 512 that receives the bins on the device."""
        n, N, T, ang, p0 = _walk_arrays(N, T, angles, psi0)
        on_dev = out is not None
        if on_dev:
            if (not out.is_cuda or str(out.dtype) != "torch.float32" or not out.is_contiguous()
                    or tuple(out.shape) != (n, self.NBINS)):
                raise ValueError("out must be a contiguous float32 CUDA tensor of shape (n, 512)")
            ptr = out.data_ptr()
        else:
            out = np.empty((n, self.NBINS), dtype=np.float32)
            ptr = out.ctypes.data
        fb = np.zeros(n, dtype=np.uint8)
        st = PredictStats()
        o = PredictOpts(recheck_frac, tvd_tol, chunk, seed, 1 if on_dev else 0, 0)
        _scheck(self._lib.surr_predict(self.h, n, N.ctypes.data, T.ctypes.data, ang.ctypes.data, p0.ctypes.data,
                                       ctypes.byref(o), ptr, fb.ctypes.data, ctypes.byref(st)))
        return out, fb.astype(bool), st

    def save(self, path: str):
        _scheck(self._lib.surr_save(self.h, path.encode()))

    def destroy(self):
        if getattr(self, "h", None) is not None and self.h.value is not None:
            rc = self._lib.surr_destroy(self.h)
            self.h = ctypes.c_void_p()
            _scheck(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _gcheck(rc: int):
    if rc != QW_OK:
        msg = load().graph_walk_last_error().decode(errors="replace")
        raise QWError(rc, msg)


class GraphWalk:
    """Coined walk on a general graph (graph_walk_*): arcs in compressed rows,
    one amplitude per arc; coins by degree (GROVER, FOURIER or DENSE)."""

    def __init__(self, offsets, targets, coin_kind: int, psi0, prec: int = QW_C128, dense=None, stream=None):
        lib = load()
        self._lib = lib
        self.off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.tgt = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
        self.nv = self.off.size - 1
        p0 = np.ascontiguousarray(np.asarray(psi0, dtype=np.complex128))
        table, dmax = None, 0
        if dense is not None:
            dmax = len(dense)
            table = np.ascontiguousarray(np.concatenate([np.asarray(m, dtype=np.complex128).ravel() for m in dense]))
        self._table = table
        h = ctypes.c_void_p()
        _gcheck(lib.graph_walk_create(self.nv, self.off.ctypes.data, self.tgt.ctypes.data if self.tgt.size else None,
                                      int(coin_kind), table.ctypes.data if table is not None else None, dmax,
                                      p0.ctypes.data, int(prec), _stream_of(stream), ctypes.byref(h)))
        self.h = h

    def reset(self, psi0):
        p0 = np.ascontiguousarray(np.asarray(psi0, dtype=np.complex128))
        _gcheck(self._lib.graph_walk_reset(self.h, p0.ctypes.data))

    def step(self, T: int):
        _gcheck(self._lib.graph_walk_step(self.h, int(T)))

    def probabilities(self, out=None):
        if out is not None:
            _gcheck(self._lib.graph_walk_probabilities(self.h, _ptr_of(out), 1))
            return out
        P = np.empty(self.nv, dtype=np.float64)
        _gcheck(self._lib.graph_walk_probabilities(self.h, P.ctypes.data, 0))
        return P

    def norm(self) -> float:
        n = ctypes.c_double()
        _gcheck(self._lib.graph_walk_norm(self.h, ctypes.byref(n)))
        return n.value

    def get_state(self) -> np.ndarray:
        psi = np.empty(self.tgt.size, dtype=np.complex128)
        _gcheck(self._lib.graph_walk_get_state(self.h, psi.ctypes.data, 0))
        return psi

    def info(self) -> GraphInfo:
        i = GraphInfo()
        _gcheck(self._lib.graph_walk_info(self.h, ctypes.byref(i)))
        return i

    def destroy(self):
        if getattr(self, "h", None) is not None and self.h.value is not None:
            rc = self._lib.graph_walk_destroy(self.h)
            self.h = ctypes.c_void_p()
            _gcheck(rc)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
