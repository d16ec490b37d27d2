"""ctypes binding of the plain C oracle (hqc_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the product package.  See
hqc_oracle.h for the paper passages each function follows and what pins it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hqc_oracle.c")
_SOURCES = [_SRC, os.path.join(_HERE, "kem_oracle.c"), os.path.join(_HERE, "ring_oracle.c")]
_HEADERS = [os.path.join(_HERE, "hqc_oracle.h"), os.path.join(_HERE, "kem_oracle.h"),
            os.path.join(_HERE, "ring_oracle.h")]
_SO = os.path.join(_HERE, "libhqc_oracle.so")
_lib = None

U8P = ctypes.POINTER(ctypes.c_uint8)
U32P = ctypes.POINTER(ctypes.c_uint32)
U64P = ctypes.POINTER(ctypes.c_uint64)
I32P = ctypes.POINTER(ctypes.c_int32)
I64P = ctypes.POINTER(ctypes.c_int64)


def build():
    """Compile the oracle with gcc into oracle/libhqc_oracle.so."""
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-Wall", "-fPIC", "-shared",
                           "-o", _SO] + _SOURCES + ["-lpthread"])


class _Param(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in (
        "id", "n", "n1", "k", "rs_d", "delta", "n2", "rm_d", "mult", "w", "wr",
        "we", "nwords", "vwords")]


class _Trace(ctypes.Structure):
    _fields_ = [("S", ctypes.c_uint8 * 64), ("lambda_", ctypes.c_uint8 * 65),
                ("L", ctypes.c_int32), ("omega", ctypes.c_uint8 * 64),
                ("located", ctypes.c_uint8 * 256), ("err", ctypes.c_uint8 * 256)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or any(os.path.getmtime(_SO) < os.path.getmtime(f)
                                          for f in _SOURCES + _HEADERS):
            build()
        L = ctypes.CDLL(_SO)
        L.hqco_param.argtypes = [ctypes.c_int, ctypes.POINTER(_Param)]
        L.hqco_gf_mul.restype = ctypes.c_uint8
        L.hqco_gf_mul.argtypes = [ctypes.c_uint8, ctypes.c_uint8]
        L.hqco_gf_pow.restype = ctypes.c_uint8
        L.hqco_gf_pow.argtypes = [ctypes.c_uint8, ctypes.c_uint32]
        L.hqco_gf_inv.restype = ctypes.c_uint8
        L.hqco_gf_inv.argtypes = [ctypes.c_uint8]
        L.hqco_gf_tables.argtypes = [U8P, U8P]
        L.hqco_mul_sparse.argtypes = [ctypes.c_int, U64P, U32P, ctypes.c_int, U64P]
        L.hqco_rm_encode.argtypes = [ctypes.c_int, ctypes.c_uint8, U64P]
        L.hqco_fht128.argtypes = [I32P, I32P]
        L.hqco_rm_decode.restype = ctypes.c_uint8
        L.hqco_rm_decode.argtypes = [ctypes.c_int, U64P, I32P]
        L.hqco_rs_generator.argtypes = [ctypes.c_int, U8P]
        L.hqco_rs_encode.argtypes = [ctypes.c_int, ctypes.c_int, U8P, U8P]
        L.hqco_rs_syndromes.argtypes = [ctypes.c_int, ctypes.c_int, U8P, U8P]
        L.hqco_rs_berlekamp_massey.restype = ctypes.c_int
        L.hqco_rs_berlekamp_massey.argtypes = [ctypes.c_int, U8P, U8P]
        L.hqco_rs_decode.argtypes = [ctypes.c_int, ctypes.c_int, U8P, U8P,
                                     ctypes.POINTER(_Trace)]
        L.hqco_code_encode.argtypes = [ctypes.c_int, U8P, U64P]
        L.hqco_code_decode.argtypes = [ctypes.c_int, U64P, U8P, U8P, ctypes.POINTER(_Trace)]
        L.hqco_keygen.argtypes = [ctypes.c_int, U64P, U32P, U32P, U64P]
        L.hqco_encrypt.argtypes = [ctypes.c_int, U64P, U64P, U8P, U32P, U32P, U32P, U64P, U64P]
        L.hqco_decrypt.argtypes = [ctypes.c_int, U32P, U64P, U64P, U8P]
        L.hqco_stress_word.argtypes = [ctypes.c_int, U8P, ctypes.c_int, U32P, U8P, U64P, U64P]
        L.hqco_keygen_batch.argtypes = [ctypes.c_int, ctypes.c_size_t, U64P, U32P, U32P, U64P,
                                        ctypes.c_int]
        L.hqco_encrypt_batch.argtypes = [ctypes.c_int, ctypes.c_size_t, U64P, U64P, I64P, U8P,
                                         U32P, U32P, U32P, U64P, U64P, ctypes.c_int]
        L.hqco_decrypt_batch.argtypes = [ctypes.c_int, ctypes.c_size_t, U32P, I64P, U64P, U64P,
                                         U8P, ctypes.c_int]
        L.hqco_keccak_f1600.argtypes = [U64P]
        L.hqco_ring_levels.restype = ctypes.c_int
        L.hqco_ring_levels.argtypes = [ctypes.c_int]
        L.hqco_ring_mul_dense.argtypes = [ctypes.c_int, U64P, U64P, U64P]
        L.hqco_ring_mul_sparse.argtypes = [ctypes.c_int, U64P, U64P, U64P]
        L.hqco_ring_mul.restype = ctypes.c_int
        L.hqco_ring_mul.argtypes = [ctypes.c_int, U64P, U64P, U64P, ctypes.c_uint32]
        L.hqco_shake256.argtypes = [U8P, ctypes.c_size_t, U8P, ctypes.c_size_t]
        L.hqco_fixed_weight.argtypes = [ctypes.c_int, ctypes.c_int, U32P, U32P]
        L.hqco_kem_seed_words.argtypes = [ctypes.c_int, U8P, U32P]
        L.hqco_kem_encaps.argtypes = [ctypes.c_int, U64P, U64P, U8P, U64P, U64P, U8P]
        L.hqco_kem_decaps.restype = ctypes.c_int
        L.hqco_kem_decaps.argtypes = [ctypes.c_int, U64P, U64P, U32P, U8P, U64P, U64P, U8P]
        L.hqco_kem_encaps_batch.argtypes = [ctypes.c_int, ctypes.c_size_t, U64P, U64P, U8P,
                                            U64P, U64P, U8P, ctypes.c_int]
        L.hqco_kem_decaps_batch.argtypes = [ctypes.c_int, ctypes.c_size_t, U64P, U64P, U32P,
                                            U8P, U64P, U64P, U8P, I32P, ctypes.c_int]
        L.hqco_decode_batch.argtypes = [ctypes.c_int, ctypes.c_size_t, U64P, U8P, ctypes.c_int]
        L.hqco_stress_batch.argtypes = [ctypes.c_int, ctypes.c_size_t, U8P, U32P, U8P, U64P,
                                        U64P, ctypes.c_int]
        for f in ("hqco_keygen_batch", "hqco_encrypt_batch", "hqco_decrypt_batch",
                  "hqco_decode_batch", "hqco_stress_batch", "hqco_param",
                  "hqco_kem_encaps_batch", "hqco_kem_decaps_batch"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t):
    """Pointer to a C-contiguous numpy array (None passes NULL)."""
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(t)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def param(pid):
    """Table I parameters plus derived sizes, as a dict."""
    p = _Param()
    if lib().hqco_param(pid, ctypes.byref(p)) != 0:
        raise ValueError("unknown parameter id %r" % (pid,))
    return {f: getattr(p, f) for f, _ in _Param._fields_}


def default_threads():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(16, os.cpu_count() or 1))


# ---- GF(2^8) -------------------------------------------------------------
def gf_mul(a, b):
    return lib().hqco_gf_mul(a, b)


def gf_pow(a, e):
    return lib().hqco_gf_pow(a, e)


def gf_inv(a):
    return lib().hqco_gf_inv(a)


def gf_tables():
    e = np.zeros(255, np.uint8)
    lg = np.zeros(256, np.uint8)
    lib().hqco_gf_tables(_p(e, U8P), _p(lg, U8P))
    return e, lg


# ---- ring product ----------------------------------------------------------
def mul_sparse(n, a, supp):
    a = _u64(a)
    supp = _u32(supp)
    out = np.zeros((n + 63) // 64, np.uint64)
    lib().hqco_mul_sparse(n, _p(a, U64P), _p(supp, U32P), len(supp), _p(out, U64P))
    return out


# ---- RM --------------------------------------------------------------------
def rm_encode(mult, b):
    out = np.zeros(2 * mult, np.uint64)
    lib().hqco_rm_encode(mult, b, _p(out, U64P))
    return out


def fht128(x):
    x = np.ascontiguousarray(x, dtype=np.int32)
    out = np.zeros(128, np.int32)
    lib().hqco_fht128(_p(x, I32P), _p(out, I32P))
    return out


def rm_decode(mult, blk):
    blk = _u64(blk)
    T = np.zeros(128, np.int32)
    b = lib().hqco_rm_decode(mult, _p(blk, U64P), _p(T, I32P))
    return b, T


# ---- RS --------------------------------------------------------------------
def rs_generator(two_delta):
    g = np.zeros(two_delta + 1, np.uint8)
    lib().hqco_rs_generator(two_delta, _p(g, U8P))
    return g


def rs_encode(n1, k, m):
    m = _u8(m)
    c = np.zeros(n1, np.uint8)
    lib().hqco_rs_encode(n1, k, _p(m, U8P), _p(c, U8P))
    return c


def rs_syndromes(n1, two_delta, c):
    c = _u8(c)
    S = np.zeros(two_delta, np.uint8)
    lib().hqco_rs_syndromes(n1, two_delta, _p(c, U8P), _p(S, U8P))
    return S


def rs_berlekamp_massey(two_delta, S):
    S = _u8(S)
    lam = np.zeros(two_delta + 1, np.uint8)
    L = lib().hqco_rs_berlekamp_massey(two_delta, _p(S, U8P), _p(lam, U8P))
    return lam, L


def _trace_dict(t, n1, td):
    return {"S": np.array(t.S[:td], np.uint8), "lambda": np.array(t.lambda_[:td + 1], np.uint8),
            "L": t.L, "omega": np.array(t.omega[:td], np.uint8),
            "located": np.array(t.located[:n1], np.uint8), "err": np.array(t.err[:n1], np.uint8)}


def rs_decode(n1, k, c):
    c = _u8(c)
    m = np.zeros(k, np.uint8)
    t = _Trace()
    lib().hqco_rs_decode(n1, k, _p(c, U8P), _p(m, U8P), ctypes.byref(t))
    return m, _trace_dict(t, n1, n1 - k)


# ---- concatenated code -----------------------------------------------------
def code_encode(pid, m):
    p = param(pid)
    m = _u8(m)
    cw = np.zeros(p["vwords"], np.uint64)
    lib().hqco_code_encode(pid, _p(m, U8P), _p(cw, U64P))
    return cw


def code_decode(pid, r):
    p = param(pid)
    r = _u64(r)
    m = np.zeros(p["k"], np.uint8)
    sym = np.zeros(p["n1"], np.uint8)
    t = _Trace()
    lib().hqco_code_decode(pid, _p(r, U64P), _p(m, U8P), _p(sym, U8P), ctypes.byref(t))
    return m, sym, _trace_dict(t, p["n1"], 2 * p["delta"])


# ---- PKE -------------------------------------------------------------------
def keygen(pid, h, x, y):
    p = param(pid)
    s = np.zeros(p["nwords"], np.uint64)
    h, x, y = _u64(h), _u32(x), _u32(y)
    lib().hqco_keygen(pid, _p(h, U64P), _p(x, U32P), _p(y, U32P), _p(s, U64P))
    return s


def encrypt(pid, h, s, m, r1, r2, e):
    p = param(pid)
    u = np.zeros(p["nwords"], np.uint64)
    v = np.zeros(p["vwords"], np.uint64)
    h, s, m, r1, r2, e = _u64(h), _u64(s), _u8(m), _u32(r1), _u32(r2), _u32(e)
    lib().hqco_encrypt(pid, _p(h, U64P), _p(s, U64P), _p(m, U8P), _p(r1, U32P), _p(r2, U32P),
                       _p(e, U32P), _p(u, U64P), _p(v, U64P))
    return u, v


def decrypt(pid, y, u, v):
    p = param(pid)
    m = np.zeros(p["k"], np.uint8)
    y, u, v = _u32(y), _u64(u), _u64(v)
    lib().hqco_decrypt(pid, _p(y, U32P), _p(u, U64P), _p(v, U64P), _p(m, U8P))
    return m


def stress_word(pid, m, bad, dval, noise):
    p = param(pid)
    r = np.zeros(p["vwords"], np.uint64)
    m, bad, dval, noise = _u8(m), _u32(bad), _u8(dval), _u64(noise)
    lib().hqco_stress_word(pid, _p(m, U8P), len(bad), _p(bad, U32P), _p(dval, U8P),
                           _p(noise, U64P), _p(r, U64P))
    return r


# ---- batches ---------------------------------------------------------------
def _check(rc):
    if rc != 0:
        raise ValueError("oracle batch call failed (%d)" % rc)


def keygen_batch(pid, h, x, y, nthreads=None):
    p = param(pid)
    h, x, y = _u64(h), _u32(x), _u32(y)
    cnt = h.shape[0]
    s = np.zeros((cnt, p["nwords"]), np.uint64)
    _check(lib().hqco_keygen_batch(pid, cnt, _p(h, U64P), _p(x, U32P), _p(y, U32P),
                                   _p(s, U64P), nthreads or default_threads()))
    return s


def encrypt_batch(pid, h, s, m, r1, r2, e, key_of=None, nthreads=None):
    p = param(pid)
    h, s, m, r1, r2, e = _u64(h), _u64(s), _u8(m), _u32(r1), _u32(r2), _u32(e)
    cnt = m.shape[0]
    ko = None if key_of is None else np.ascontiguousarray(key_of, dtype=np.int64)
    u = np.zeros((cnt, p["nwords"]), np.uint64)
    v = np.zeros((cnt, p["vwords"]), np.uint64)
    _check(lib().hqco_encrypt_batch(pid, cnt, _p(h, U64P), _p(s, U64P), _p(ko, I64P),
                                    _p(m, U8P), _p(r1, U32P), _p(r2, U32P), _p(e, U32P),
                                    _p(u, U64P), _p(v, U64P), nthreads or default_threads()))
    return u, v


def decrypt_batch(pid, y, u, v, key_of=None, nthreads=None):
    p = param(pid)
    y, u, v = _u32(y), _u64(u), _u64(v)
    cnt = u.shape[0]
    ko = None if key_of is None else np.ascontiguousarray(key_of, dtype=np.int64)
    m = np.zeros((cnt, p["k"]), np.uint8)
    _check(lib().hqco_decrypt_batch(pid, cnt, _p(y, U32P), _p(ko, I64P), _p(u, U64P),
                                    _p(v, U64P), _p(m, U8P), nthreads or default_threads()))
    return m


def decode_batch(pid, r, nthreads=None):
    p = param(pid)
    r = _u64(r)
    cnt = r.shape[0]
    m = np.zeros((cnt, p["k"]), np.uint8)
    _check(lib().hqco_decode_batch(pid, cnt, _p(r, U64P), _p(m, U8P),
                                   nthreads or default_threads()))
    return m


def stress_batch(pid, m, bad, dval, noise, out=None, nthreads=None):
    """Stress words; out may be the noise array itself (filled in place)."""
    p = param(pid)
    m, bad, dval, noise = _u8(m), _u32(bad), _u8(dval), _u64(noise)
    cnt = m.shape[0]
    r = np.zeros((cnt, p["vwords"]), np.uint64) if out is None else out
    _check(lib().hqco_stress_batch(pid, cnt, _p(m, U8P), _p(bad, U32P), _p(dval, U8P),
                                   _p(noise, U64P), _p(r, U64P), nthreads or default_threads()))
    return r


# ---- KEM (kem_oracle.c) -------------------------------------------------------

KEM_KEY_BYTES = 32


def keccak_f1600(state):
    a = _u64(state).copy()
    assert a.shape == (25,)
    lib().hqco_keccak_f1600(_p(a, U64P))
    return a


def shake256(data, outlen):
    src = np.frombuffer(bytes(data) + b"\0", dtype=np.uint8).copy()
    out = np.zeros(outlen + 1, np.uint8)
    lib().hqco_shake256(_p(src, U8P), len(data), _p(out, U8P), outlen)
    return bytes(out[:outlen])


def fixed_weight(n, w, a):
    a = _u32(a)
    assert a.shape == (w,)
    out = np.zeros(w, np.uint32)
    lib().hqco_fixed_weight(n, w, _p(a, U32P), _p(out, U32P))
    return out


def kem_seed_words(pid, m):
    p = param(pid)
    m = _u8(m)
    out = np.zeros(2 * p["wr"] + p["we"], np.uint32)
    lib().hqco_kem_seed_words(pid, _p(m, U8P), _p(out, U32P))
    return out


def kem_encaps(pid, h, s, m):
    p = param(pid)
    h, s, m = _u64(h), _u64(s), _u8(m)
    u = np.zeros(p["nwords"], np.uint64)
    v = np.zeros(p["vwords"], np.uint64)
    key = np.zeros(KEM_KEY_BYTES, np.uint8)
    lib().hqco_kem_encaps(pid, _p(h, U64P), _p(s, U64P), _p(m, U8P), _p(u, U64P), _p(v, U64P),
                          _p(key, U8P))
    return u, v, key


def kem_decaps(pid, h, s, y, sigma, u, v):
    h, s, y, sigma, u, v = _u64(h), _u64(s), _u32(y), _u8(sigma), _u64(u), _u64(v)
    key = np.zeros(KEM_KEY_BYTES, np.uint8)
    ok = lib().hqco_kem_decaps(pid, _p(h, U64P), _p(s, U64P), _p(y, U32P), _p(sigma, U8P),
                               _p(u, U64P), _p(v, U64P), _p(key, U8P))
    return key, bool(ok)


def kem_encaps_batch(pid, h, s, m, nthreads=None):
    p = param(pid)
    h, s, m = _u64(h), _u64(s), _u8(m)
    count = m.shape[0]
    u = np.zeros((count, p["nwords"]), np.uint64)
    v = np.zeros((count, p["vwords"]), np.uint64)
    key = np.zeros((count, KEM_KEY_BYTES), np.uint8)
    _check(lib().hqco_kem_encaps_batch(pid, count, _p(h, U64P), _p(s, U64P), _p(m, U8P),
                                       _p(u, U64P), _p(v, U64P), _p(key, U8P),
                                       nthreads or default_threads()))
    return u, v, key


def kem_decaps_batch(pid, h, s, y, sigma, u, v, nthreads=None):
    h, s, y, sigma, u, v = _u64(h), _u64(s), _u32(y), _u8(sigma), _u64(u), _u64(v)
    count = u.shape[0]
    key = np.zeros((count, KEM_KEY_BYTES), np.uint8)
    ok = np.zeros(count, np.int32)
    _check(lib().hqco_kem_decaps_batch(pid, count, _p(h, U64P), _p(s, U64P), _p(y, U32P),
                                       _p(sigma, U8P), _p(u, U64P), _p(v, U64P), _p(key, U8P),
                                       _p(ok, I32P), nthreads or default_threads()))
    return key, ok.astype(bool)


# ---- adaptive ring multiplication (ring_oracle.c) ------------------------------

def ring_levels(uwords):
    return lib().hqco_ring_levels(uwords)


def _ring_args(n, a, b):
    U = (n + 63) // 64
    a, b = _u64(a), _u64(b)
    assert a.shape == (U,) and b.shape == (U,)
    return a, b, np.zeros(U, np.uint64)


def ring_mul_dense(n, a, b):
    a, b, out = _ring_args(n, a, b)
    lib().hqco_ring_mul_dense(n, _p(a, U64P), _p(b, U64P), _p(out, U64P))
    return out


def ring_mul_sparse(n, a, b):
    a, b, out = _ring_args(n, a, b)
    lib().hqco_ring_mul_sparse(n, _p(a, U64P), _p(b, U64P), _p(out, U64P))
    return out


def ring_mul(n, a, b, threshold):
    """(out, path): path 0 = sparse (weight(a) <= threshold), 1 = dense."""
    a, b, out = _ring_args(n, a, b)
    path = lib().hqco_ring_mul(n, _p(a, U64P), _p(b, U64P), _p(out, U64P), threshold)
    return out, path
