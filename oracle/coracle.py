"""ctypes wrapper of the plain C oracle (``coracle.c``) — test infrastructure only.

``build()`` compiles ``libcoracle.so`` next to this file with gcc.  ``load()``
builds on first use when the library is missing or older than its source.
"""

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "coracle.c")
LIB = os.path.join(HERE, "libcoracle.so")

_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        U32, U64, I = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        lib.co_fermat_dft_sampled.argtypes = [U32, U32, U64, U64, P, P, U64, P, P, P, I]
        lib.co_fermat_dft_sampled.restype = I
        lib.co_fermat_mul2exp.argtypes = [U32, P, U32, U64, P, P]
        lib.co_fermat_mul2exp.restype = I
        lib.co_nega_dft_sampled.argtypes = [U32, U64, U32, U64, U64, P, U64, P, P, I]
        lib.co_nega_dft_sampled.restype = I
        lib.co_prime_dft_sampled.argtypes = [U64, U64, U64, U32, U64, U64, P, U64, P, P, I]
        lib.co_prime_dft_sampled.restype = I
        lib.co_zx_coeffs.argtypes = [P, U64, U32, P, U64, U32, P, U64, P, U32, I]
        lib.co_zx_coeffs.restype = I
        lib.co_zmx_coeffs.argtypes = [P, U64, P, U64, U64, P, U64, P, I]
        lib.co_zmx_coeffs.restype = I
        lib.co_fingerprint.argtypes = [P, U64, U32, U64, U64]
        lib.co_fingerprint.restype = U64
        lib.co_fingerprint64.argtypes = [P, U64, U64, U64]
        lib.co_fingerprint64.restype = U64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _threads(n):
    if n is None:
        n = min(16, os.cpu_count() or 1)
    return int(n)


def fermat_dft_sampled(N, L, s, limbs, tops, js, nthreads=None):
    """Eq. (1) in Z/(2^N+1) at indices js; limbs (z, N/32) uint32, tops (z,) uint32."""
    lib = load()
    limbs = np.ascontiguousarray(limbs, dtype=np.uint32)
    tops = np.ascontiguousarray(tops, dtype=np.uint32)
    js = np.ascontiguousarray(js, dtype=np.uint64)
    W = N // 32
    z = limbs.shape[0]
    out_l = np.zeros((len(js), W), dtype=np.uint32)
    out_t = np.zeros(len(js), dtype=np.uint32)
    rc = lib.co_fermat_dft_sampled(N, L, s, z, _ptr(limbs), _ptr(tops), len(js), _ptr(js), _ptr(out_l),
                                   _ptr(out_t), _threads(nthreads))
    if rc:
        raise ValueError("co_fermat_dft_sampled: bad arguments")
    return out_l, out_t


def prime_dft_sampled(ring, L, s, a, js, nthreads=None):
    """Eq. (1) in Z/pZ (ring: tft_oracle.PrimeRing) at indices js; a: uint32 values."""
    lib = load()
    a = np.ascontiguousarray(a, dtype=np.uint32)
    js = np.ascontiguousarray(js, dtype=np.uint64)
    out = np.zeros(len(js), dtype=np.uint32)
    rc = lib.co_prime_dft_sampled(ring.p, ring.theta, ring.ord, L, s, len(a), _ptr(a), len(js), _ptr(js),
                                  _ptr(out), _threads(nthreads))
    if rc:
        raise ValueError("co_prime_dft_sampled: bad arguments")
    return out


def fermat_mul2exp(N, limbs, top, e):
    lib = load()
    limbs = np.ascontiguousarray(limbs, dtype=np.uint32)
    out = np.zeros(N // 32, dtype=np.uint32)
    t = ctypes.c_uint32(0)
    lib.co_fermat_mul2exp(N, _ptr(limbs), int(top), int(e), _ptr(out), ctypes.byref(t))
    return out, t.value


def nega_dft_sampled(K, m, L, s, a, js, nthreads=None):
    """Eq. (1) in (Z/mZ)[y]/(y^K+1) at indices js; a (z, K) uint64."""
    lib = load()
    a = np.ascontiguousarray(a, dtype=np.uint64)
    js = np.ascontiguousarray(js, dtype=np.uint64)
    out = np.zeros((len(js), K), dtype=np.uint64)
    rc = lib.co_nega_dft_sampled(K, m, L, s, a.shape[0], _ptr(a), len(js), _ptr(js), _ptr(out),
                                 _threads(nthreads))
    if rc:
        raise ValueError("co_nega_dft_sampled: bad arguments")
    return out


def zx_coeffs(g, h, ks, ow, nthreads=None):
    """Exact Z[x] product coefficients at ks as (len(ks), ow) uint32 limbs."""
    lib = load()
    g = np.ascontiguousarray(g, dtype=np.uint32)
    h = np.ascontiguousarray(h, dtype=np.uint32)
    ks = np.ascontiguousarray(ks, dtype=np.uint64)
    out = np.zeros((len(ks), ow), dtype=np.uint32)
    rc = lib.co_zx_coeffs(_ptr(g), g.shape[0], g.shape[1], _ptr(h), h.shape[0], h.shape[1], _ptr(ks), len(ks),
                          _ptr(out), ow, _threads(nthreads))
    if rc:
        raise ValueError("co_zx_coeffs: coefficient does not fit in %d limbs" % ow)
    return out


def zmx_coeffs(g, h, m, ks, nthreads=None):
    lib = load()
    g = np.ascontiguousarray(g, dtype=np.uint64)
    h = np.ascontiguousarray(h, dtype=np.uint64)
    ks = np.ascontiguousarray(ks, dtype=np.uint64)
    out = np.zeros(len(ks), dtype=np.uint64)
    rc = lib.co_zmx_coeffs(_ptr(g), len(g), _ptr(h), len(h), m, _ptr(ks), len(ks), _ptr(out), _threads(nthreads))
    if rc:
        raise ValueError("co_zmx_coeffs: bad modulus")
    return out


def fingerprint(limbs, P, r):
    lib = load()
    limbs = np.ascontiguousarray(limbs, dtype=np.uint32)
    return lib.co_fingerprint(_ptr(limbs), limbs.shape[0], limbs.shape[1], P, r)


def fingerprint64(vals, P, r):
    lib = load()
    vals = np.ascontiguousarray(vals, dtype=np.uint64)
    return lib.co_fingerprint64(_ptr(vals), len(vals), P, r)
