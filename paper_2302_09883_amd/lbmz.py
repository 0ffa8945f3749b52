"""ctypes binding of liblbmz (include/lbmz.h): argument marshalling only.

Every computation runs in the HIP library; this module converts arguments
(NumPy arrays on the host, PyTorch tensors on the device), passes the current
PyTorch stream, and turns status codes into exceptions.  If the library has
not been built the import of :func:`library` raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmz.so")

LBMZ_OK, LBMZ_EINVAL, LBMZ_ENOMEM, LBMZ_EDEVICE, LBMZ_EOVERFLOW, LBMZ_ENAN, LBMZ_ESTATE = 0, -1, -2, -3, -4, -5, -6
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EOVERFLOW", -5: "ENAN", -6: "ESTATE"}

SCHEMES = {"fv_upwind": 0, "d2q9_bgk": 1, "euler_rusanov": 2, "d3q19_bgk": 3}
WAVELETS = {"haar": 0, "bl53": 1}
RULES = {"capped": 0, "constant": 1, "accum": 2}
DTYPES = {"f32": 0, "f64": 1}
VALUES = {"f32": 0, "f16": 1, "e4m3": 2, "e4m3b": 3}
NP_DTYPES = {"f32": np.float32, "f64": np.float64}
MASK_BIT = 1 << 31


class LbmzError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbmz {_STATUS.get(code, code)}: {msg}")
        self.code = code


class Grid(ct.Structure):
    _fields_ = [("dim", ct.c_int), ("n", ct.c_int64 * 3), ("periodic", ct.c_int), ("h", ct.c_double)]


class Scheme(ct.Structure):
    _fields_ = [("kind", ct.c_int), ("dtype", ct.c_int), ("vel", ct.c_double * 3), ("cfl", ct.c_double),
                ("tau", ct.c_double), ("gamma", ct.c_double)]


class Patch(ct.Structure):
    _fields_ = [("p", ct.c_int * 3), ("wavelet", ct.c_int), ("rule", ct.c_int), ("values", ct.c_int)]


class Stats(ct.Structure):
    _fields_ = [("steps", ct.c_int64), ("nnz_total", ct.c_int64), ("store_bytes", ct.c_int64),
                ("capacity_bytes", ct.c_int64), ("dense_bytes", ct.c_int64), ("ratio", ct.c_double),
                ("nfields", ct.c_int32), ("npatch", ct.c_int32), ("totals", ct.c_double * 16),
                ("regrows", ct.c_int64), ("mask_records", ct.c_int64), ("list_records", ct.c_int64),
                ("ms_last_call", ct.c_double)]


_ALLOC = ct.CFUNCTYPE(ct.c_void_p, ct.c_size_t, ct.c_void_p)
_FREE = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_void_p)

_lib = None


def library() -> ct.CDLL:
    """Load liblbmz.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or python -m paper_2302_09883_amd.build")
    # PyTorch (the device-memory and stream plumbing) ships its own HIP
    # runtime; loading it first makes the library bind to that same runtime,
    # so that both share one device context in this process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ct.CDLL(LIB_PATH)
    P = ct.POINTER
    vp = ct.c_void_p
    sig = {
        "lbmz_create": ([P(Grid), P(Scheme), P(Patch), ct.c_int, ct.c_double, P(vp)], ct.c_int),
        "lbmz_create_reference": ([P(Grid), P(Scheme), P(vp)], ct.c_int),
        "lbmz_set_allocator": ([vp, _ALLOC, _FREE, vp], ct.c_int),
        "lbmz_set_stream": ([vp, vp], ct.c_int),
        "lbmz_set_pool_capacity": ([vp, ct.c_int64], ct.c_int),
        "lbmz_set_field": ([vp, ct.c_int, vp, ct.c_size_t, ct.c_int], ct.c_int),
        "lbmz_set_macroscopic": ([vp, vp, vp, vp, ct.c_size_t, ct.c_int], ct.c_int),
        "lbmz_set_macroscopic3": ([vp, vp, vp, vp, vp, ct.c_size_t, ct.c_int], ct.c_int),
        "lbmz_get_totals": ([vp, vp, ct.c_int], ct.c_int),
        "lbmz_step": ([vp, ct.c_int], ct.c_int),
        "lbmz_decompress_field": ([vp, ct.c_int, vp, ct.c_size_t, ct.c_int], ct.c_int),
        "lbmz_stats": ([vp, P(Stats)], ct.c_int),
        "lbmz_store_size": ([vp, P(ct.c_int64), P(ct.c_int64)], ct.c_int),
        "lbmz_get_store": ([vp, vp, vp, ct.c_size_t], ct.c_int),
        "lbmz_put_store": ([vp, vp, vp, ct.c_size_t], ct.c_int),
        "lbmz_set_coefficients": ([vp, vp, ct.c_size_t, ct.c_int], ct.c_int),
        "lbmz_set_execution": ([vp, ct.c_int, ct.c_int], ct.c_int),
        "lbmz_get_execution": ([vp, P(ct.c_int), P(ct.c_int)], ct.c_int),
        "lbmz_autotune": ([vp, ct.c_int, vp], ct.c_int),
        "lbmz_set_patch_eps": ([vp, vp, ct.c_size_t, ct.c_int], ct.c_int),
        "lbmz_set_patch_levels": ([vp, vp, ct.c_size_t], ct.c_int),
        "lbmz_enable_features": ([vp, ct.c_int], ct.c_int),
        "lbmz_get_features": ([vp, vp, ct.c_size_t, ct.c_int], ct.c_int),
        "lbmz_last_error": ([vp], ct.c_char_p),
        "lbmz_net_create": ([ct.c_int, P(vp)], ct.c_int),
        "lbmz_net_param_count": ([vp], ct.c_int),
        "lbmz_net_set_stream": ([vp, vp], ct.c_int),
        "lbmz_net_set_params": ([vp, vp, ct.c_size_t], ct.c_int),
        "lbmz_net_get_params": ([vp, vp, ct.c_size_t], ct.c_int),
        "lbmz_net_forward": ([vp, vp, ct.c_int, vp, ct.c_int], ct.c_int),
        "lbmz_net_gradients": ([vp, vp, vp, ct.c_int, vp, P(ct.c_float), ct.c_int], ct.c_int),
        "lbmz_net_train_step": ([vp, vp, vp, ct.c_int, ct.c_float, P(ct.c_float), ct.c_int], ct.c_int),
        "lbmz_net_gradients_noalloc": ([vp, vp, vp, ct.c_int, vp, vp], ct.c_int),
        "lbmz_net_last_error": ([vp], ct.c_char_p),
        "lbmz_net_destroy": ([vp], None),
        "lbmz_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _buffer(x, dtype):
    """(pointer, nbytes, on_device, keepalive) of a NumPy array or a CUDA tensor."""
    if _is_torch(x):
        if not x.is_cuda:
            x = x.numpy()
        else:
            if not x.is_contiguous():
                raise ValueError("device tensors must be contiguous")
            return ct.c_void_p(x.data_ptr()), x.numel() * x.element_size(), 1, x
    a = np.ascontiguousarray(x, dtype=dtype)
    return ct.c_void_p(a.ctypes.data), a.nbytes, 0, a


class Context:
    """One compressed (or, with ``reference=True``, uncompressed) simulation."""

    def __init__(self, n: int, scheme: str = "d2q9_bgk", dtype: str = "f32", p: int = 64,
                 wavelet: str = "bl53", levels: int = 5, eps: float = 1e-4, rule: str = "capped",
                 vel=(1.0, 0.5), cfl: float = 0.5, tau: float = 0.6, reference: bool = False,
                 stream=None, torch_allocator: bool = False, pool_capacity: int | None = None,
                 values: str = "f32", gamma: float = 1.4):
        self._lib = library()
        self.n, self.scheme, self.dtype, self.p = n, scheme, dtype, p
        self.values = values
        self.wavelet, self.levels, self.eps, self.rule = wavelet, levels, eps, rule
        self.reference = reference
        self.np_dtype = NP_DTYPES[dtype]
        self.nfields = {"d2q9_bgk": 9, "euler_rusanov": 4, "d3q19_bgk": 19}.get(scheme, 1)
        self.dim = 3 if scheme == "d3q19_bgk" else 2
        self.s = (p + 1 if wavelet == "bl53" else p) if not reference else n
        g = Grid(self.dim, (ct.c_int64 * 3)(n, n, n if self.dim == 3 else 1), 1, 1.0 / n)
        sc = Scheme(SCHEMES[scheme], DTYPES[dtype], (ct.c_double * 3)(vel[0], vel[1], 0.0), cfl, tau, gamma)
        h = ct.c_void_p()
        if reference:
            rc = self._lib.lbmz_create_reference(ct.byref(g), ct.byref(sc), ct.byref(h))
        else:
            pt = Patch((ct.c_int * 3)(p, p, p if self.dim == 3 else 1), WAVELETS[wavelet], RULES[rule], VALUES[values])
            rc = self._lib.lbmz_create(ct.byref(g), ct.byref(sc), ct.byref(pt), levels, eps, ct.byref(h))
        if rc != LBMZ_OK:
            raise LbmzError(rc, "create failed (invalid geometry, levels, scheme or no kernel for the key)")
        self._h = h
        self._cb = None
        if torch_allocator:
            self._use_torch_allocator()
        if stream is None:
            stream = _current_stream()
        self._check(self._lib.lbmz_set_stream(self._h, ct.c_void_p(stream)))
        if pool_capacity is not None:
            self.set_pool_capacity(pool_capacity)

    # -- plumbing -------------------------------------------------------------
    def _check(self, rc):
        if rc != LBMZ_OK:
            msg = self._lib.lbmz_last_error(self._h)
            raise LbmzError(rc, msg.decode() if msg else "")

    def _use_torch_allocator(self):
        import torch

        dev = torch.cuda.current_device()

        def _alloc(nbytes, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev)
            except Exception:   # noqa: BLE001 - reported to the library as NULL
                return None

        def _free(ptr, user):
            torch.cuda.caching_allocator_delete(ptr)

        self._cb = (_ALLOC(_alloc), _FREE(_free))
        self._check(self._lib.lbmz_set_allocator(self._h, self._cb[0], self._cb[1], None))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lbmz_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # noqa: BLE001
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- state ----------------------------------------------------------------
    def set_pool_capacity(self, nbytes: int):
        self._check(self._lib.lbmz_set_pool_capacity(self._h, int(nbytes)))

    def set_field(self, field: int, data):
        ptr, nb, dev, keep = _buffer(data, self.np_dtype)
        self._check(self._lib.lbmz_set_field(self._h, field, ptr, nb, dev))
        del keep

    def set_macroscopic(self, rho, ux, uy, uz=None):
        """Equilibrium populations of the given density and velocity (``uz`` for D3Q19)."""
        arrs = (rho, ux, uy) if self.dim == 2 else (rho, ux, uy, uz)
        if any(x is None for x in arrs):
            raise ValueError("the D3Q19 scheme needs uz")
        bufs = [_buffer(x, self.np_dtype) for x in arrs]
        if len({b[1] for b in bufs}) != 1 or len({b[2] for b in bufs}) != 1:
            raise ValueError("the fields must have the same size and location")
        ptrs = [b[0] for b in bufs]
        if self.dim == 3:
            self._check(self._lib.lbmz_set_macroscopic3(self._h, *ptrs, bufs[0][1], bufs[0][2]))
        else:
            self._check(self._lib.lbmz_set_macroscopic(self._h, *ptrs, bufs[0][1], bufs[0][2]))

    def set_coefficients(self, coef):
        ptr, nb, dev, keep = _buffer(coef, self.np_dtype)
        self._check(self._lib.lbmz_set_coefficients(self._h, ptr, nb, dev))
        del keep

    def set_execution(self, persistent: bool = False, graph: bool = False):
        self._check(self._lib.lbmz_set_execution(self._h, int(bool(persistent)), int(bool(graph))))

    def execution(self):
        p, g = ct.c_int(), ct.c_int()
        self._check(self._lib.lbmz_get_execution(self._h, ct.byref(p), ct.byref(g)))
        return bool(p.value), bool(g.value)

    def autotune(self, steps_per_variant: int = 5):
        """Pick the fastest execution mode on the current state (advances 8 x steps_per_variant steps);
        returns the four measured ms per step, index 2 * persistent + graph."""
        ms = np.zeros(4, dtype=np.float32)
        self._check(self._lib.lbmz_autotune(self._h, int(steps_per_variant), ct.c_void_p(ms.ctypes.data)))
        return ms

    def set_patch_eps(self, eps=None):
        """Per-patch thresholds ``[npatch]`` (float64, host or device), or None for the single eps."""
        if eps is None:
            self._check(self._lib.lbmz_set_patch_eps(self._h, None, 0, 0))
            return
        ptr, nb, dev, keep = _buffer(eps, np.float64)
        self._check(self._lib.lbmz_set_patch_eps(self._h, ptr, nb // 8, dev))
        del keep

    def set_patch_levels(self, levels=None):
        """One level count per patch (the learned control), or None for the context's single count."""
        if levels is None:
            self._check(self._lib.lbmz_set_patch_levels(self._h, None, 0))
            return
        a = np.ascontiguousarray(levels, dtype=np.int32)
        self._check(self._lib.lbmz_set_patch_levels(self._h, ct.c_void_p(a.ctypes.data), a.size))

    def enable_features(self, on: bool = True):
        self._check(self._lib.lbmz_enable_features(self._h, int(bool(on))))

    def features(self, out=None):
        """Network inputs of the last step, ``float32 [npatch, 4 nfields, 8, 8]`` (host unless ``out``
        is a device tensor): the stride-8 coefficients, then per field the level 1, 2, 3 energies."""
        npatch = (self.n // self.p) ** 2
        if out is None:
            out = np.empty((npatch, 4 * self.nfields, 8, 8), dtype=np.float32)
        ptr, nb, dev, keep = _buffer(out, np.float32)
        self._check(self._lib.lbmz_get_features(self._h, ptr, nb, dev))
        return out

    def step(self, n: int = 1):
        self._check(self._lib.lbmz_step(self._h, int(n)))

    def decompress_field(self, field: int, out=None):
        if out is None:
            out = np.empty((self.n,) * self.dim, dtype=self.np_dtype)
        ptr, nb, dev, keep = _buffer(out, self.np_dtype)
        if not dev and keep is not out:
            raise ValueError("host output must be a contiguous array of the context dtype")
        self._check(self._lib.lbmz_decompress_field(self._h, field, ptr, nb, dev))
        return out

    def fields(self) -> np.ndarray:
        """All fields on the host, ``[nfields, n, n]`` (``[nfields, n, n, n]`` in 3-D)."""
        return np.stack([self.decompress_field(f) for f in range(self.nfields)])

    def stats(self) -> dict:
        st = Stats()
        self._check(self._lib.lbmz_stats(self._h, ct.byref(st)))
        d = {k: getattr(st, k) for k, _ in Stats._fields_}
        d["totals"] = self.totals().tolist()
        return d

    def totals(self) -> np.ndarray:
        """FP64 per-field (trapezoid-weighted) sums of the decompressed state, ``[nfields]``."""
        out = np.zeros(self.nfields, dtype=np.float64)
        self._check(self._lib.lbmz_get_totals(self._h, ct.c_void_p(out.ctypes.data), self.nfields))
        return out

    # -- compressed store -------------------------------------------------------
    def store(self):
        """``(table uint32 [npatch, nfields, 2], pool bytes)`` of the current state."""
        pb, te = ct.c_int64(), ct.c_int64()
        self._check(self._lib.lbmz_store_size(self._h, ct.byref(pb), ct.byref(te)))
        table = np.empty(2 * te.value, dtype=np.uint32)
        pool = np.empty(pb.value, dtype=np.uint8)
        self._check(self._lib.lbmz_get_store(self._h, ct.c_void_p(table.ctypes.data),
                                             ct.c_void_p(pool.ctypes.data), pool.nbytes))
        npatch = te.value // self.nfields
        return table.reshape(npatch, self.nfields, 2), pool.tobytes()

    def put_store(self, table, pool: bytes):
        t = np.ascontiguousarray(table, dtype=np.uint32)
        buf = np.frombuffer(pool, dtype=np.uint8)
        self._check(self._lib.lbmz_put_store(self._h, ct.c_void_p(t.ctypes.data),
                                             ct.c_void_p(buf.ctypes.data), buf.nbytes))


class Net:
    """The learned threshold predictor of include/lbmz.h (bfloat16 weights, float32 accumulation)."""

    def __init__(self, k: int, stream=None):
        self._lib = library()
        h = ct.c_void_p()
        rc = self._lib.lbmz_net_create(int(k), ct.byref(h))
        if rc != LBMZ_OK:
            raise LbmzError(rc, "network creation failed")
        self._h = h
        self.k = int(k)
        self.nparams = int(self._lib.lbmz_net_param_count(h))
        if stream is None:
            stream = _current_stream()
        self._check(self._lib.lbmz_net_set_stream(h, ct.c_void_p(stream)))

    def _check(self, rc):
        if rc != LBMZ_OK:
            msg = self._lib.lbmz_net_last_error(self._h)
            raise LbmzError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lbmz_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # noqa: BLE001
            pass

    def set_params(self, params):
        a = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self._lib.lbmz_net_set_params(self._h, ct.c_void_p(a.ctypes.data), a.size))

    def params(self) -> np.ndarray:
        a = np.empty(self.nparams, dtype=np.float32)
        self._check(self._lib.lbmz_net_get_params(self._h, ct.c_void_p(a.ctypes.data), a.size))
        return a

    def forward(self, x, out=None):
        ptr, nb, dev, keep = _buffer(x, np.float32)
        batch = nb // (36 * 64 * 4)
        if out is None:
            out = np.empty((batch, self.k), dtype=np.float32)
        optr, _, odev, okeep = _buffer(out, np.float32)
        if odev != dev:
            raise ValueError("inputs and outputs must live on the same side")
        self._check(self._lib.lbmz_net_forward(self._h, ptr, batch, optr, dev))
        return out

    def gradients(self, x, t):
        xa = np.ascontiguousarray(x, dtype=np.float32)
        ta = np.ascontiguousarray(t, dtype=np.float32)
        g = np.empty(self.nparams, dtype=np.float32)
        loss = ct.c_float()
        self._check(self._lib.lbmz_net_gradients(self._h, ct.c_void_p(xa.ctypes.data), ct.c_void_p(ta.ctypes.data),
                                                 xa.shape[0], ct.c_void_p(g.ctypes.data), ct.byref(loss), 0))
        return g, float(loss.value)

    def gradients_noalloc(self, x, t, grad, loss):
        """lbmz_net_gradients_noalloc: x, t, grad and loss are contiguous float32
        device tensors ([B][9][8][8], [B][K], [nparams], [1]); asynchronous on
        the network's stream."""
        for a in (x, t, grad, loss):
            if not (_is_torch(a) and a.is_cuda and a.is_contiguous()):
                raise ValueError("device tensors expected")
        self._check(self._lib.lbmz_net_gradients_noalloc(self._h, ct.c_void_p(x.data_ptr()), ct.c_void_p(t.data_ptr()),
                                                         int(x.shape[0]), ct.c_void_p(grad.data_ptr()),
                                                         ct.c_void_p(loss.data_ptr())))

    def train_step(self, x, t, lr: float) -> float:
        xp, xb, xdev, xk = _buffer(x, np.float32)
        tp, tb, tdev, tk = _buffer(t, np.float32)
        loss = ct.c_float()
        self._check(self._lib.lbmz_net_train_step(self._h, xp, tp, xb // (36 * 64 * 4), ct.c_float(lr),
                                                  ct.byref(loss), xdev))
        return float(loss.value)


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:   # noqa: BLE001
        pass
    return None
