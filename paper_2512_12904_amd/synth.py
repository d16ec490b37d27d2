"""Seeded synthetic inputs (ctypes binding of csrc/hqc_synth.c).

Only random draws live here -- dense uniform vectors, uniform bytes and
uniform fixed-weight supports -- shaped like the HQC parameter sets of
Table I.  No HQC arithmetic: whoever consumes the draws (the GPU library, or
the CPU checker in the tests) computes keys and ciphertexts from them.

Sizes are passed in explicitly (a dict with n, n1, n2, k, delta, w, wr, we),
so this module carries no parameter table of its own.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "hqc_synth.c")
_SO = os.path.join(_HERE, "libhqc_synth.so")
_lib = None

U8P = ctypes.POINTER(ctypes.c_uint8)
U32P = ctypes.POINTER(ctypes.c_uint32)
U64P = ctypes.POINTER(ctypes.c_uint64)
I64P = ctypes.POINTER(ctypes.c_int64)


class _Sizes(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in (
        "param_id", "n", "n1", "n2", "k", "delta", "w", "wr", "we", "rho")]


def build():
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-Wall", "-fPIC", "-shared",
                           "-o", _SO, _SRC, "-lpthread"])


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        L.synth_splitmix64_next.restype = ctypes.c_uint64
        L.synth_splitmix64_next.argtypes = [U64P]
        L.synth_seed.restype = ctypes.c_uint64
        L.synth_seed.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.synth_fixed_weight.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, U32P]
        L.synth_dense.argtypes = [ctypes.c_uint64, ctypes.c_int, U64P]
        L.synth_keys.restype = ctypes.c_int
        L.synth_keys.argtypes = [ctypes.c_uint64, ctypes.POINTER(_Sizes), ctypes.c_size_t,
                                 ctypes.c_uint64, U64P, U32P, U32P, ctypes.c_int]
        L.synth_encryptions.restype = ctypes.c_int
        L.synth_encryptions.argtypes = [ctypes.c_uint64, ctypes.POINTER(_Sizes), ctypes.c_size_t,
                                        I64P, ctypes.c_uint64, U8P, U32P, U32P, U32P,
                                        ctypes.c_int]
        L.synth_stress.restype = ctypes.c_int
        L.synth_stress.argtypes = [ctypes.c_uint64, ctypes.POINTER(_Sizes), ctypes.c_size_t,
                                   ctypes.c_uint64, U8P, U32P, U8P, U64P, ctypes.c_int]
        L.synth_fill_words.argtypes = [ctypes.c_uint64, ctypes.c_size_t, U64P]
        _lib = L
    return _lib


def threads():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(16, os.cpu_count() or 1))


def _sizes(pid, sz):
    # rho (largest noise weight drawn for a clean block) only matters for stress words
    return _Sizes(pid, sz["n"], sz["n1"], sz["n2"], sz["k"], sz["delta"], sz["w"], sz["wr"],
                  sz["we"], sz.get("rho", 0))


def _p(a, t):
    return None if a is None else a.ctypes.data_as(t)


def splitmix64(state, count):
    """count outputs of the SplitMix64 stream started at state."""
    st = ctypes.c_uint64(state)
    return np.array([lib().synth_splitmix64_next(ctypes.byref(st)) for _ in range(count)],
                    np.uint64)


def seed(parent, salt):
    return lib().synth_seed(parent, salt)


def fixed_weight(seed_value, bound, w):
    out = np.zeros(w, np.uint32)
    lib().synth_fixed_weight(seed_value, bound, w, _p(out, U32P))
    return out


def keys(master, pid, sz, count, key_id0=0):
    """h (count x ceil(n/64) uint64), x, y (count x w uint32)."""
    nwords = (sz["n"] + 63) // 64
    h = np.zeros((count, nwords), np.uint64)
    x = np.zeros((count, sz["w"]), np.uint32)
    y = np.zeros((count, sz["w"]), np.uint32)
    s = _sizes(pid, sz)
    rc = lib().synth_keys(master, ctypes.byref(s), count, key_id0, _p(h, U64P), _p(x, U32P),
                          _p(y, U32P), threads())
    assert rc == 0
    return h, x, y


def encryptions(master, pid, sz, count, key_of=None, ct_id0=0):
    """m (count x k uint8), r1, r2 (count x wr), e (count x we)."""
    m = np.zeros((count, sz["k"]), np.uint8)
    r1 = np.zeros((count, sz["wr"]), np.uint32)
    r2 = np.zeros((count, sz["wr"]), np.uint32)
    e = np.zeros((count, sz["we"]), np.uint32)
    ko = None if key_of is None else np.ascontiguousarray(key_of, dtype=np.int64)
    s = _sizes(pid, sz)
    rc = lib().synth_encryptions(master, ctypes.byref(s), count, _p(ko, I64P), ct_id0,
                                 _p(m, U8P), _p(r1, U32P), _p(r2, U32P), _p(e, U32P), threads())
    assert rc == 0
    return m, r1, r2, e


def stress(master, pid, sz, count, word_id0=0):
    """m (count x k), bad (count x delta), dval (count x delta), noise (count x n1*n2/64).

    sz["rho"] bounds the noise weight of each block that is not drawn as bad."""
    vwords = sz["n1"] * sz["n2"] // 64
    m = np.zeros((count, sz["k"]), np.uint8)
    bad = np.zeros((count, sz["delta"]), np.uint32)
    dval = np.zeros((count, sz["delta"]), np.uint8)
    noise = np.zeros((count, vwords), np.uint64)
    s = _sizes(pid, sz)
    rc = lib().synth_stress(master, ctypes.byref(s), count, word_id0, _p(m, U8P),
                            _p(bad, U32P), _p(dval, U8P), _p(noise, U64P), threads())
    assert rc == 0
    return m, bad, dval, noise


def words(seed_value, shape):
    """Uniform uint64 words (content-free filler)."""
    out = np.zeros(shape, np.uint64)
    lib().synth_fill_words(seed_value, out.size, _p(out, U64P))
    return out
