"""CPU oracle of LOPC (arXiv 2603.26968) -- TEST INFRASTRUCTURE ONLY.

A thin ctypes wrapper around ``lopc_ref.c``, the plain single-threaded C
implementation of the compressor written from the paper.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark use it; the
GPU library and its Python binding never import it.

Every function takes and returns numpy arrays / bytes and raises
:class:`OracleError` with the C status code on failure.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lopc_ref.c")
_LIB_PATH = os.path.join(_HERE, "liblopc_ref.so")

OK, E_ARG, E_NONFINITE, E_BOUND, E_RANGE, E_CAPACITY, E_FORMAT, E_NOMEM = (
    0, -1, -2, -3, -4, -5, -6, -8)

ABS, NOA = 0, 1
CHUNK_BYTES = 16384


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile lopc_ref.c with gcc into liblopc_ref.so (IEEE-exact flags)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        c_i64p = ctypes.POINTER(ctypes.c_int64)
        c_u64p = ctypes.POINTER(ctypes.c_uint64)
        c_szp = ctypes.POINTER(ctypes.c_size_t)
        c_dp = ctypes.POINTER(ctypes.c_double)
        vp, sz, ci, cd = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
        sig = {
            "lopc_ref_error_params": (ci, [vp, ci, sz, cd, ci, c_dp, c_dp]),
            "lopc_ref_quantize": (ci, [cd, cd, ci, c_i64p]),
            "lopc_ref_bins": (ci, [vp, ci, sz, cd, vp]),
            "lopc_ref_subbins": (ci, [vp, ci, ci, c_i64p, vp, vp]),
            "lopc_ref_bin_floor": (ci, [ctypes.c_int64, cd, ci, c_dp]),
            "lopc_ref_reconstruct": (ci, [ctypes.c_int64, ctypes.c_uint64, cd, ci, c_dp]),
            "lopc_ref_diffnb": (None, [vp, sz, ci]),
            "lopc_ref_undiffnb": (None, [vp, sz, ci]),
            "lopc_ref_bit": (ci, [vp, sz, ci, vp]),
            "lopc_ref_unbit": (ci, [vp, sz, ci, vp]),
            "lopc_ref_rze": (sz, [vp, sz, ci, vp, ctypes.POINTER(ci)]),
            "lopc_ref_unrze": (ci, [vp, sz, sz, ci, vp]),
            "lopc_ref_compress_bound": (ci, [ci, ci, c_i64p, c_szp]),
            "lopc_ref_compress": (ci, [vp, ci, ci, c_i64p, cd, ci, vp, sz, c_szp]),
            "lopc_ref_stream_info": (ci, [vp, sz, ctypes.POINTER(ci), ctypes.POINTER(ci),
                                          c_i64p, c_dp, c_dp]),
            "lopc_ref_decompress": (ci, [vp, sz, vp, sz]),
            "lopc_ref_decode_codes": (ci, [vp, sz, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code: int, what: str) -> None:
    if code != OK:
        raise OracleError(code, what)


def _dtype_code(a: np.ndarray) -> int:
    if a.dtype == np.float32:
        return 0
    if a.dtype == np.float64:
        return 1
    raise TypeError("field must be float32 or float64")


def _dims(shape) -> ctypes.Array:
    d = (ctypes.c_int64 * 3)(1, 1, 1)
    for i, s in enumerate(shape):
        d[i] = int(s)
    return d


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


# ---------------------------------------------------------------- parameters
def error_params(x: np.ndarray, eb: float, mode: int = NOA):
    x = np.ascontiguousarray(x)
    eps, inv = ctypes.c_double(), ctypes.c_double()
    _check(lib().lopc_ref_error_params(_ptr(x), _dtype_code(x), x.size, float(eb),
                                       int(mode), ctypes.byref(eps), ctypes.byref(inv)),
           "error_params")
    return eps.value, inv.value


def quantize(y: float, inv: float, dtype_code: int = 1) -> int:
    b = ctypes.c_int64()
    _check(lib().lopc_ref_quantize(float(y), float(inv), dtype_code, ctypes.byref(b)),
           "quantize")
    return b.value


def bins(x: np.ndarray, inv: float) -> np.ndarray:
    x = np.ascontiguousarray(x)
    out = np.empty(x.shape, np.int64)
    _check(lib().lopc_ref_bins(_ptr(x), _dtype_code(x), x.size, float(inv), _ptr(out)),
           "bins")
    return out


def subbins(x: np.ndarray, b: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x)
    b = np.ascontiguousarray(b, dtype=np.int64)
    if x.ndim not in (2, 3) or b.shape != x.shape:
        raise ValueError("subbins needs a 2D/3D field and bins of the same shape")
    out = np.empty(x.shape, np.uint64)
    _check(lib().lopc_ref_subbins(_ptr(x), _dtype_code(x), x.ndim, _dims(x.shape),
                                  _ptr(b), _ptr(out)), "subbins")
    return out


def bin_floor(b: int, inv: float, dtype_code: int) -> float:
    v = ctypes.c_double()
    _check(lib().lopc_ref_bin_floor(int(b), float(inv), dtype_code, ctypes.byref(v)),
           "bin_floor")
    return v.value


def reconstruct(b: int, s: int, inv: float, dtype_code: int) -> float:
    v = ctypes.c_double()
    _check(lib().lopc_ref_reconstruct(int(b), int(s), float(inv), dtype_code,
                                      ctypes.byref(v)), "reconstruct")
    return v.value


# ---------------------------------------------------------------- stages
def diffnb(words: np.ndarray, k: int) -> np.ndarray:
    w = np.array(words, dtype=np.int64, copy=True)
    lib().lopc_ref_diffnb(_ptr(w), w.size, k)
    return w


def undiffnb(words: np.ndarray, k: int) -> np.ndarray:
    w = np.array(words, dtype=np.int64, copy=True)
    lib().lopc_ref_undiffnb(_ptr(w), w.size, k)
    return w


def bit(data: bytes, k: int) -> bytes:
    a = np.frombuffer(bytes(data), np.uint8).copy()
    m = a.size // k
    out = np.zeros(a.size, np.uint8)
    _check(lib().lopc_ref_bit(_ptr(a), m, k, _ptr(out)), "bit")
    return out.tobytes()


def unbit(data: bytes, k: int) -> bytes:
    a = np.frombuffer(bytes(data), np.uint8).copy()
    m = a.size // k
    out = np.zeros(a.size, np.uint8)
    _check(lib().lopc_ref_unbit(_ptr(a), m, k, _ptr(out)), "unbit")
    return out.tobytes()


def rze(data: bytes, w: int):
    """Returns (encoded bytes, passthrough flag)."""
    a = np.frombuffer(bytes(data), np.uint8).copy()
    out = np.zeros(max(a.size, 1), np.uint8)
    pt = ctypes.c_int()
    n = lib().lopc_ref_rze(_ptr(a), a.size, w, _ptr(out), ctypes.byref(pt))
    return out[:n].tobytes(), bool(pt.value)


def unrze(data: bytes, length: int, w: int) -> bytes:
    a = np.frombuffer(bytes(data), np.uint8).copy()
    if a.size == 0:
        a = np.zeros(1, np.uint8)
        n_in = 0
    else:
        n_in = a.size
    out = np.zeros(max(length, 1), np.uint8)
    _check(lib().lopc_ref_unrze(_ptr(a), n_in, length, w, _ptr(out)), "unrze")
    return out[:length].tobytes()


# ---------------------------------------------------------------- streams
def compress_bound(shape, dtype) -> int:
    code = 0 if np.dtype(dtype) == np.float32 else 1
    n = ctypes.c_size_t()
    _check(lib().lopc_ref_compress_bound(code, len(shape), _dims(shape), ctypes.byref(n)),
           "compress_bound")
    return n.value


def compress(x: np.ndarray, eb: float, mode: int = NOA) -> bytes:
    x = np.ascontiguousarray(x)
    cap = compress_bound(x.shape, x.dtype)
    out = np.empty(cap, np.uint8)
    size = ctypes.c_size_t()
    _check(lib().lopc_ref_compress(_ptr(x), _dtype_code(x), x.ndim, _dims(x.shape),
                                   float(eb), int(mode), _ptr(out), cap,
                                   ctypes.byref(size)), "compress")
    return out[:size.value].tobytes()


def stream_info(stream: bytes) -> dict:
    a = np.frombuffer(bytes(stream), np.uint8)
    dt, nd = ctypes.c_int(), ctypes.c_int()
    d = (ctypes.c_int64 * 3)()
    eps, inv = ctypes.c_double(), ctypes.c_double()
    _check(lib().lopc_ref_stream_info(_ptr(a) if a.size else None, a.size, ctypes.byref(dt),
                                      ctypes.byref(nd), d, ctypes.byref(eps),
                                      ctypes.byref(inv)), "stream_info")
    shape = tuple(int(d[i]) for i in range(nd.value))
    return {"dtype": np.float32 if dt.value == 0 else np.float64, "shape": shape,
            "eps": eps.value, "inv": inv.value}


def decompress(stream: bytes) -> np.ndarray:
    info = stream_info(stream)
    a = np.frombuffer(bytes(stream), np.uint8)
    out = np.empty(info["shape"], info["dtype"])
    _check(lib().lopc_ref_decompress(_ptr(a), a.size, _ptr(out), out.nbytes),
           "decompress")
    return out


def decode_codes(stream: bytes):
    """Bins (int64) and subbins (uint64) stored in a stream."""
    info = stream_info(stream)
    a = np.frombuffer(bytes(stream), np.uint8)
    b = np.empty(info["shape"], np.int64)
    s = np.empty(info["shape"], np.uint64)
    _check(lib().lopc_ref_decode_codes(_ptr(a), a.size, _ptr(b), _ptr(s)), "decode_codes")
    return b, s
