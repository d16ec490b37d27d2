"""Python binding of libhqc_gpu.so (include/hqc_gpu.h).

Argument marshalling only: torch device tensors in, their device pointers
and the current HIP stream out to the C ABI.  Every step of decryption runs
in the library's kernels; if the library cannot be loaded these functions
raise -- there is no fallback.

Tensor layouts (per item, row-major, on the GPU):
  u  int64 [count, u_words]   bit t of u is bit t % 64 of word t // 64
  v  int64 [count, v_words]   (or r for decode)
  y  int32 [count, w]         support indices of the secret key
  m  uint8 [count, k]
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "libhqc_gpu.so")

HQC_OK, HQC_EINVAL, HQC_ERANGE, HQC_EHIP, HQC_ENOMEM = 0, -1, -2, -3, -4
F_PER_ITEM_LAUNCH = 0x1
F_GRAPH = 0x2

# every function declared in include/hqc_gpu.h
EXPORTS = (
    "hqc_sizes", "hqc_decrypt_batch", "hqc_decode_batch", "hqc_decrypt_mixed",
    "hqc_decode_mixed", "hqc_keystore_create", "hqc_keystore_put", "hqc_keystore_put_many",
    "hqc_keystore_destroy", "hqc_keystore_bad_ids", "hqc_decrypt_batch_keyed",
    "hqc_decrypt_mixed_keyed", "hqc_strerror",
    "hqc_last_hip_error", "hqc_default_grid", "hqc_shutdown", "hqc_keygen_batch",
    "hqc_encrypt_batch", "hqc_code_encode_batch", "hqc_kem_workspace_bytes", "hqc_kem_encaps_batch",
    "hqc_kem_decaps_batch", "hqc_kem_decaps_batch_noalloc", "hqc_fixed_weight_batch", "hqc_ring_workspace_bytes", "hqc_ring_default_threshold",
    "hqc_ring_mul_batch", "hqc_autotune_decrypt", "hqc_tune_set", "hqc_tune_get",
    "hqc_tune_clear", "hqc_launch_config", "hqc_debug_bytes", "hqc_decrypt_debug",
)


class HqcError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        msg = "%s failed: %s (%d)" % (what, strerror(code), code)
        if code == HQC_EHIP:
            msg += ", hipError %d" % lib().hqc_last_hip_error()
        super().__init__(msg)


class Sizes(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in (
        "param_id", "n", "n1", "k", "delta", "n2", "mult", "w", "wr", "we", "u_words",
        "v_words")]


class Params(ctypes.Structure):
    _fields_ = [("param_id", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("stream", ctypes.c_void_p), ("grid", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("shape", ctypes.c_int32)]


class TuneReport(ctypes.Structure):
    _fields_ = [("param_id", ctypes.c_int32), ("tile", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("ms", ctypes.c_float), ("heuristic_tile", ctypes.c_int32),
                ("heuristic_grid", ctypes.c_int32), ("heuristic_ms", ctypes.c_float),
                ("candidates", ctypes.c_int32), ("identical", ctypes.c_int32),
                ("count", ctypes.c_uint64), ("shape", ctypes.c_int32),
                ("heuristic_shape", ctypes.c_int32)]


class Segment(ctypes.Structure):
    _fields_ = [("param_id", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("count", ctypes.c_size_t), ("u", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("y", ctypes.c_void_p), ("m_out", ctypes.c_void_p)]


_lib = None


def lib():
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError("libhqc_gpu.so is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(SO_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        L.hqc_sizes.argtypes = [ctypes.c_int, ctypes.POINTER(Sizes)]
        L.hqc_decrypt_batch.argtypes = [ctypes.POINTER(Params), vp, vp, vp, vp, sz]
        L.hqc_decode_batch.argtypes = [ctypes.POINTER(Params), vp, vp, sz]
        L.hqc_decrypt_mixed.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Segment), ctypes.c_int]
        L.hqc_decode_mixed.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Segment), ctypes.c_int]
        L.hqc_keystore_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(sz)]
        L.hqc_keystore_put.argtypes = [vp, ctypes.c_int, ctypes.c_uint32, vp]
        L.hqc_keystore_put_many.argtypes = [vp, ctypes.c_int, ctypes.c_uint32, sz, vp]
        L.hqc_keystore_destroy.argtypes = [vp]
        L.hqc_keystore_bad_ids.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
        L.hqc_decrypt_batch_keyed.argtypes = [ctypes.POINTER(Params), vp, vp, vp, vp, vp, sz]
        L.hqc_decrypt_mixed_keyed.argtypes = [ctypes.POINTER(Params), vp, ctypes.POINTER(Segment),
                                              ctypes.c_int]
        L.hqc_strerror.restype = ctypes.c_char_p
        L.hqc_strerror.argtypes = [ctypes.c_int]
        L.hqc_last_hip_error.argtypes = []
        L.hqc_default_grid.argtypes = [ctypes.c_int]
        L.hqc_keygen_batch.argtypes = [ctypes.POINTER(Params), vp, vp, vp, vp, sz]
        L.hqc_encrypt_batch.argtypes = [ctypes.POINTER(Params), vp, vp, vp, vp, vp, vp, vp, vp, sz]
        L.hqc_code_encode_batch.argtypes = [ctypes.POINTER(Params), vp, vp, vp, sz]
        L.hqc_kem_workspace_bytes.restype = ctypes.c_size_t
        L.hqc_kem_workspace_bytes.argtypes = [ctypes.c_int, sz]
        L.hqc_kem_encaps_batch.argtypes = [ctypes.POINTER(Params), vp, vp, vp, vp, vp, vp, vp, sz,
                                           sz]
        L.hqc_kem_decaps_batch.argtypes = [ctypes.POINTER(Params), vp, vp, vp, vp, vp, vp, vp, vp,
                                           sz, sz]
        L.hqc_kem_decaps_batch_noalloc.argtypes = [ctypes.POINTER(Params), vp, vp, vp, vp, vp, vp,
                                                   vp, sz]
        L.hqc_fixed_weight_batch.argtypes = [ctypes.POINTER(Params), vp, vp, sz]
        L.hqc_ring_workspace_bytes.restype = ctypes.c_size_t
        L.hqc_ring_workspace_bytes.argtypes = [ctypes.c_int, sz, sz]
        L.hqc_ring_default_threshold.restype = ctypes.c_uint32
        L.hqc_ring_default_threshold.argtypes = [ctypes.c_int]
        L.hqc_ring_mul_batch.argtypes = [ctypes.POINTER(Params), vp, vp, vp, vp, ctypes.c_uint32,
                                         vp, sz, sz]
        L.hqc_shutdown.restype = None
        L.hqc_shutdown.argtypes = []
        L.hqc_autotune_decrypt.argtypes = [ctypes.c_int, sz, ctypes.c_int, vp,
                                           ctypes.POINTER(TuneReport)]
        L.hqc_tune_set.argtypes = [ctypes.c_int, sz, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.hqc_tune_get.argtypes = [ctypes.c_int, sz, ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.hqc_tune_clear.restype = None
        L.hqc_launch_config.argtypes = [ctypes.POINTER(Params), sz, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.hqc_tune_clear.argtypes = []
        L.hqc_debug_bytes.restype = ctypes.c_size_t
        L.hqc_debug_bytes.argtypes = [ctypes.c_int]
        L.hqc_decrypt_debug.argtypes = [ctypes.POINTER(Params), vp, vp, vp, vp, vp, sz]
        _lib = L
    return _lib


def strerror(code):
    return lib().hqc_strerror(code).decode()


def _check(rc, what):
    if rc != HQC_OK:
        raise HqcError(rc, what)


def sizes(pid):
    s = Sizes()
    _check(lib().hqc_sizes(pid, ctypes.byref(s)), "hqc_sizes")
    return {f: getattr(s, f) for f, _ in Sizes._fields_}


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _params(pid, flags, grid, stream, tile=0, shape=0):
    return Params(pid, flags, _stream(stream), grid, tile, shape)


def _dev(t, dtype, name, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0)


def _out(out, count, k, device):
    if out is None:
        out = torch.empty((count, k), dtype=torch.uint8, device=device)
    return out


def decrypt_batch(pid, u, v, y, out=None, flags=0, grid=0, stream=None, tile=0, shape=0):
    """m[i] = HQC.PKE.Decrypt(y[i], (u[i], v[i])) for every row (Alg. 2)."""
    s = sizes(pid)
    count = u.shape[0]
    out = _out(out, count, s["k"], u.device)
    p = _params(pid, flags, grid, stream, tile, shape)
    rc = lib().hqc_decrypt_batch(
        ctypes.byref(p), _dev(u, torch.int64, "u", (count, s["u_words"])),
        _dev(v, torch.int64, "v", (count, s["v_words"])),
        _dev(y, torch.int32, "y", (count, s["w"])),
        _dev(out, torch.uint8, "out", (count, s["k"])), count)
    _check(rc, "hqc_decrypt_batch")
    return out


def decode_batch(pid, r, out=None, flags=0, grid=0, stream=None, tile=0, shape=0):
    """m[i] = C.Decode(r[i]) (the concatenated decoder alone)."""
    s = sizes(pid)
    count = r.shape[0]
    out = _out(out, count, s["k"], r.device)
    p = _params(pid, flags, grid, stream, tile, shape)
    rc = lib().hqc_decode_batch(ctypes.byref(p), _dev(r, torch.int64, "r", (count, s["v_words"])),
                                _dev(out, torch.uint8, "out", (count, s["k"])), count)
    _check(rc, "hqc_decode_batch")
    return out


def _segments(items, decode, keyed=False):
    segs = (Segment * len(items))()
    outs = []
    for i, it in enumerate(items):
        pid = it["pid"]
        s = sizes(pid)
        u = it["r"] if decode else it["u"]
        count = u.shape[0]
        out = _out(it.get("out"), count, s["k"], u.device)
        outs.append(out)
        segs[i].param_id = pid
        segs[i].count = count
        segs[i].u = _dev(u, torch.int64, "u/r", (count, s["v_words"] if decode else s["u_words"]))
        if not decode:
            segs[i].v = _dev(it["v"], torch.int64, "v", (count, s["v_words"]))
            if keyed:
                segs[i].y = _dev(it["key_ids"], torch.int32, "key_ids", (count,))
            else:
                segs[i].y = _dev(it["y"], torch.int32, "y", (count, s["w"]))
        segs[i].m_out = _dev(out, torch.uint8, "out", (count, s["k"]))
    return segs, outs


def decrypt_mixed(items, flags=0, grid=0, stream=None, tile=0):
    """One launch over several parameter sets.  items: list of dicts with
    pid, u, v, y (and optionally out); returns the list of outputs."""
    segs, outs = _segments(items, decode=False)
    p = _params(0, flags, grid, stream, tile)
    _check(lib().hqc_decrypt_mixed(ctypes.byref(p), segs, len(items)), "hqc_decrypt_mixed")
    return outs


def decode_mixed(items, flags=0, grid=0, stream=None, tile=0):
    """items: list of dicts with pid, r (and optionally out)."""
    segs, outs = _segments(items, decode=True)
    p = _params(0, flags, grid, stream, tile)
    _check(lib().hqc_decode_mixed(ctypes.byref(p), segs, len(items)), "hqc_decode_mixed")
    return outs


class KeyStore:
    """Device-resident secret keys y, capacity per parameter set."""

    def __init__(self, cap1, cap3, cap5):
        self._h = ctypes.c_void_p()
        cap = (ctypes.c_size_t * 3)(cap1, cap3, cap5)
        _check(lib().hqc_keystore_create(ctypes.byref(self._h), cap), "hqc_keystore_create")

    @property
    def handle(self):
        if not self._h:
            raise ValueError("keystore destroyed")
        return self._h

    def put(self, pid, key_id0, y_host):
        """y_host: numpy uint32 [count, w] (host memory)."""
        import numpy as np
        y_host = np.ascontiguousarray(y_host, dtype=np.uint32)
        if y_host.ndim == 1:
            y_host = y_host[None, :]
        rc = lib().hqc_keystore_put_many(self.handle, pid, key_id0, y_host.shape[0],
                                         y_host.ctypes.data_as(ctypes.c_void_p))
        _check(rc, "hqc_keystore_put_many")

    def bad_ids(self):
        v = ctypes.c_uint64()
        _check(lib().hqc_keystore_bad_ids(self.handle, ctypes.byref(v)), "hqc_keystore_bad_ids")
        return v.value

    def close(self):
        if self._h:
            lib().hqc_keystore_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decrypt_batch_keyed(pid, ks, u, v, key_ids, out=None, flags=0, grid=0, stream=None, tile=0, shape=0):
    """decrypt_batch with y[i] = slot key_ids[i] of the keystore."""
    s = sizes(pid)
    count = u.shape[0]
    out = _out(out, count, s["k"], u.device)
    p = _params(pid, flags, grid, stream, tile, shape)
    rc = lib().hqc_decrypt_batch_keyed(
        ctypes.byref(p), ks.handle, _dev(u, torch.int64, "u", (count, s["u_words"])),
        _dev(v, torch.int64, "v", (count, s["v_words"])),
        _dev(key_ids, torch.int32, "key_ids", (count,)),
        _dev(out, torch.uint8, "out", (count, s["k"])), count)
    _check(rc, "hqc_decrypt_batch_keyed")
    return out


def decrypt_mixed_keyed(ks, items, flags=0, grid=0, stream=None, tile=0):
    """One launch over several parameter sets with keys from the keystore.
    items: list of dicts with pid, u, v, key_ids (int32 [count]) and
    optionally out; returns the list of outputs."""
    segs, outs = _segments(items, decode=False, keyed=True)
    p = _params(0, flags, grid, stream, tile)
    _check(lib().hqc_decrypt_mixed_keyed(ctypes.byref(p), ks.handle, segs, len(items)),
           "hqc_decrypt_mixed_keyed")
    return outs


def keygen_batch(pid, h, x, y, out=None, grid=0, stream=None):
    """s[i] = x[i] + h[i]*y[i] (Alg. 3; the randomness h, x, y is an input)."""
    sz = sizes(pid)
    count = h.shape[0]
    if out is None:
        out = torch.empty((count, sz["u_words"]), dtype=torch.int64, device=h.device)
    p = _params(pid, 0, grid, stream)
    rc = lib().hqc_keygen_batch(
        ctypes.byref(p), _dev(h, torch.int64, "h", (count, sz["u_words"])),
        _dev(x, torch.int32, "x", (count, sz["w"])), _dev(y, torch.int32, "y", (count, sz["w"])),
        _dev(out, torch.int64, "out", (count, sz["u_words"])), count)
    _check(rc, "hqc_keygen_batch")
    return out


def encrypt_batch(pid, h, s, m, r1, r2, e, u_out=None, v_out=None, grid=0, stream=None):
    """(u, v) = HQC.PKE.Encrypt((h[i], s[i]), m[i]) with the randomness
    r1, r2, e as input (Alg. 1)."""
    sz = sizes(pid)
    count = h.shape[0]
    dev = h.device
    if u_out is None:
        u_out = torch.empty((count, sz["u_words"]), dtype=torch.int64, device=dev)
    if v_out is None:
        v_out = torch.empty((count, sz["v_words"]), dtype=torch.int64, device=dev)
    p = _params(pid, 0, grid, stream)
    rc = lib().hqc_encrypt_batch(
        ctypes.byref(p), _dev(h, torch.int64, "h", (count, sz["u_words"])),
        _dev(s, torch.int64, "s", (count, sz["u_words"])),
        _dev(m, torch.uint8, "m", (count, sz["k"])),
        _dev(r1, torch.int32, "r1", (count, sz["wr"])), _dev(r2, torch.int32, "r2", (count, sz["wr"])),
        _dev(e, torch.int32, "e", (count, sz["we"])),
        _dev(u_out, torch.int64, "u_out", (count, sz["u_words"])),
        _dev(v_out, torch.int64, "v_out", (count, sz["v_words"])), count)
    _check(rc, "hqc_encrypt_batch")
    return u_out, v_out


def code_encode_batch(pid, m, sym_err=None, out=None, grid=0, stream=None):
    """r[i] = the concatenated codeword (Sec. II-A) of the RS codeword of m[i]
    plus sym_err[i] (uint8 [count, n1], or None for C.Encode(m[i]))."""
    sz = sizes(pid)
    count = m.shape[0]
    if out is None:
        out = torch.empty((count, sz["v_words"]), dtype=torch.int64, device=m.device)
    p = _params(pid, 0, grid, stream)
    err = ctypes.c_void_p(0) if sym_err is None else _dev(sym_err, torch.uint8, "sym_err",
                                                         (count, sz["n1"]))
    rc = lib().hqc_code_encode_batch(ctypes.byref(p), _dev(m, torch.uint8, "m", (count, sz["k"])),
                                     err, _dev(out, torch.int64, "out", (count, sz["v_words"])),
                                     count)
    _check(rc, "hqc_code_encode_batch")
    return out


def default_grid(pid):
    g = lib().hqc_default_grid(pid)
    if g < 0:
        raise HqcError(g, "hqc_default_grid")
    return g


def shutdown():
    lib().hqc_shutdown()


KEM_KEY_BYTES = 32


def kem_workspace_bytes(pid, count):
    return lib().hqc_kem_workspace_bytes(pid, count)


def _workspace(pid, count, device, workspace):
    need = kem_workspace_bytes(pid, count)
    if workspace is None:
        workspace = torch.empty(max(need, 8), dtype=torch.uint8, device=device)
    if workspace.numel() < need:
        raise ValueError("workspace holds %d bytes, %d needed" % (workspace.numel(), need))
    return workspace


def kem_encaps_batch(pid, h, s, m, u_out=None, v_out=None, key_out=None, workspace=None,
                     grid=0, stream=None):
    """KEM encapsulation of the caller's messages m[i] under (h[i], s[i]):
    returns (u, v, key); the construction is documented in hqc_gpu.h."""
    sz = sizes(pid)
    count = h.shape[0]
    dev = h.device
    if u_out is None:
        u_out = torch.empty((count, sz["u_words"]), dtype=torch.int64, device=dev)
    if v_out is None:
        v_out = torch.empty((count, sz["v_words"]), dtype=torch.int64, device=dev)
    if key_out is None:
        key_out = torch.empty((count, KEM_KEY_BYTES), dtype=torch.uint8, device=dev)
    ws = _workspace(pid, count, dev, workspace)
    p = _params(pid, 0, grid, stream)
    rc = lib().hqc_kem_encaps_batch(
        ctypes.byref(p), _dev(h, torch.int64, "h", (count, sz["u_words"])),
        _dev(s, torch.int64, "s", (count, sz["u_words"])),
        _dev(m, torch.uint8, "m", (count, sz["k"])),
        _dev(u_out, torch.int64, "u_out", (count, sz["u_words"])),
        _dev(v_out, torch.int64, "v_out", (count, sz["v_words"])),
        _dev(key_out, torch.uint8, "key_out", (count, KEM_KEY_BYTES)),
        _dev(ws, torch.uint8, "workspace"), ws.numel(), count)
    _check(rc, "hqc_kem_encaps_batch")
    return u_out, v_out, key_out


def kem_decaps_batch(pid, h, s, y, sigma, u, v, key_out=None, workspace=None, grid=0,
                     stream=None, tile=0):
    """KEM decapsulation: key[i] from (u[i], v[i]) with the secret (y[i],
    sigma[i]) and public (h[i], s[i]); implicit rejection (no error output)."""
    sz = sizes(pid)
    count = u.shape[0]
    dev = u.device
    if key_out is None:
        key_out = torch.empty((count, KEM_KEY_BYTES), dtype=torch.uint8, device=dev)
    ws = _workspace(pid, count, dev, workspace)
    p = _params(pid, 0, grid, stream, tile)
    rc = lib().hqc_kem_decaps_batch(
        ctypes.byref(p), _dev(h, torch.int64, "h", (count, sz["u_words"])),
        _dev(s, torch.int64, "s", (count, sz["u_words"])),
        _dev(y, torch.int32, "y", (count, sz["w"])),
        _dev(sigma, torch.uint8, "sigma", (count, sz["k"])),
        _dev(u, torch.int64, "u", (count, sz["u_words"])),
        _dev(v, torch.int64, "v", (count, sz["v_words"])),
        _dev(key_out, torch.uint8, "key_out", (count, KEM_KEY_BYTES)),
        _dev(ws, torch.uint8, "workspace"), ws.numel(), count)
    _check(rc, "hqc_kem_decaps_batch")
    return key_out


NOALLOC_SCRATCH_BYTES = 64 << 20


def kem_decaps_batch_noalloc(pid, h, s, y, sigma, u, v, key_out, grid=0, stream=None):
    """kem_decaps_batch with the library's fixed scratch as workspace
    (hqc_kem_decaps_batch_noalloc): allocates nothing, key_out is required."""
    sz = sizes(pid)
    count = u.shape[0]
    p = _params(pid, 0, grid, stream)
    rc = lib().hqc_kem_decaps_batch_noalloc(
        ctypes.byref(p), _dev(h, torch.int64, "h", (count, sz["u_words"])),
        _dev(s, torch.int64, "s", (count, sz["u_words"])),
        _dev(y, torch.int32, "y", (count, sz["w"])),
        _dev(sigma, torch.uint8, "sigma", (count, sz["k"])),
        _dev(u, torch.int64, "u", (count, sz["u_words"])),
        _dev(v, torch.int64, "v", (count, sz["v_words"])),
        _dev(key_out, torch.uint8, "key_out", (count, KEM_KEY_BYTES)), count)
    _check(rc, "hqc_kem_decaps_batch_noalloc")
    return key_out


RING_SPARSE_MAX = 4096


def ring_workspace_bytes(pid, count, chunk_items=None):
    return lib().hqc_ring_workspace_bytes(pid, count, count if chunk_items is None else chunk_items)


def ring_default_threshold(pid):
    return lib().hqc_ring_default_threshold(pid)


def ring_mul_batch(pid, a, b, out=None, threshold=None, path_out=None, workspace=None,
                   chunk_items=None, grid=0, stream=None):
    """out[i] = a[i] * b[i] in GF(2)[X]/(X^n - 1) (Sec. III-B adaptive path:
    sparse Eq. (1) when weight(a[i]) <= threshold, else dense Karatsuba).
    Returns (out, path) with path[i] = 0 sparse / 1 dense."""
    sz = sizes(pid)
    count = a.shape[0]
    dev = a.device
    if out is None:
        out = torch.empty((count, sz["u_words"]), dtype=torch.int64, device=dev)
    if path_out is None:
        path_out = torch.empty(count, dtype=torch.uint8, device=dev)
    if threshold is None:
        threshold = ring_default_threshold(pid)
    if workspace is None:
        workspace = torch.empty(max(8, ring_workspace_bytes(pid, count, chunk_items)),
                                dtype=torch.uint8, device=dev)
    p = _params(pid, 0, grid, stream)
    rc = lib().hqc_ring_mul_batch(
        ctypes.byref(p), _dev(a, torch.int64, "a", (count, sz["u_words"])),
        _dev(b, torch.int64, "b", (count, sz["u_words"])),
        _dev(out, torch.int64, "out", (count, sz["u_words"])),
        _dev(path_out, torch.uint8, "path_out", (count,)), threshold,
        _dev(workspace, torch.uint8, "workspace"), workspace.numel(), count)
    _check(rc, "hqc_ring_mul_batch")
    return out, path_out


def fixed_weight_batch(pid, draws, out=None, grid=0, stream=None):
    """Floyd's sampling of the KEM: draws (count x (2 wr + we) int32) ->
    supports of r1, r2, e (same shape)."""
    sz = sizes(pid)
    nd = 2 * sz["wr"] + sz["we"]
    count = draws.shape[0]
    if out is None:
        out = torch.empty((count, nd), dtype=torch.int32, device=draws.device)
    p = _params(pid, 0, grid, stream)
    rc = lib().hqc_fixed_weight_batch(ctypes.byref(p), _dev(draws, torch.int32, "draws", (count, nd)),
                                      _dev(out, torch.int32, "out", (count, nd)), count)
    _check(rc, "hqc_fixed_weight_batch")
    return out


def autotune_decrypt(pid, count, reps=5, stream=None):
    """Time the decryption kernel's (tile, grid) candidates on count random
    ciphertexts and store the fastest in the library's table (see
    hqc_autotune_decrypt); returns the report as a dict."""
    r = TuneReport()
    _check(lib().hqc_autotune_decrypt(pid, count, reps, _stream(stream), ctypes.byref(r)),
           "hqc_autotune_decrypt")
    return {f: getattr(r, f) for f, _ in TuneReport._fields_}


def tune_set(pid, count, tile, grid, shape=1):
    """Table entry for count's bucket: tile, grid, shape (1 = A, 2 = B);
    tile = grid = shape = 0 removes it."""
    _check(lib().hqc_tune_set(pid, count, tile, grid, shape), "hqc_tune_set")


def tune_get(pid, count):
    """(tile, grid, shape) of count's bucket, or (0, 0, 0)."""
    t, g, sh = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().hqc_tune_get(pid, count, ctypes.byref(t), ctypes.byref(g), ctypes.byref(sh)),
           "hqc_tune_get")
    return t.value, g.value, sh.value


def tune_clear():
    lib().hqc_tune_clear()


def launch_config(pid, count, grid=0, tile=0, shape=0):
    """(shape, tile, grid) of the launch decrypt_batch makes for count items
    with these knobs (1 = shape A, 2 = shape B), on the current device."""
    p = _params(pid, 0, grid, None, tile, shape)
    sh, t, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().hqc_launch_config(ctypes.byref(p), count, ctypes.byref(sh), ctypes.byref(t),
                                   ctypes.byref(g)), "hqc_launch_config")
    return sh.value, t.value, g.value


def decrypt_debug(pid, u, v, y, flags=0, grid=0, stream=None, tile=0):
    """decrypt_batch plus each item's intermediates (hqc_decrypt_debug):
    returns (m, record) with record a dict of numpy arrays: "r" (received
    word, count x n1*n2/64 uint64), "sym" (RM symbols), "S" (syndromes),
    "lam" (the error locator Lambda, Lambda_0 = 1), "e" (error values at the
    message positions)."""
    sz = sizes(pid)
    count = u.shape[0]
    nb = lib().hqc_debug_bytes(pid)
    out = torch.empty((count, sz["k"]), dtype=torch.uint8, device=u.device)
    rec = torch.zeros((count, nb), dtype=torch.uint8, device=u.device)
    p = _params(pid, flags, grid, stream, tile)
    rc = lib().hqc_decrypt_debug(
        ctypes.byref(p), _dev(u, torch.int64, "u", (count, sz["u_words"])),
        _dev(v, torch.int64, "v", (count, sz["v_words"])), _dev(y, torch.int32, "y", (count, sz["w"])),
        _dev(out, torch.uint8, "m", (count, sz["k"])), _dev(rec, torch.uint8, "dbg", (count, nb)), count)
    _check(rc, "hqc_decrypt_debug")
    r = rec.cpu().numpy()
    n1, k, td = sz["n1"], sz["k"], 2 * sz["delta"]
    o_sym = 8 * sz["v_words"]
    o_s = o_sym + n1
    o_l = o_s + td
    o_e = o_l + td + 1
    fields = {"r": np.ascontiguousarray(r[:, :o_sym]).view(np.uint64), "sym": r[:, o_sym:o_s],
              "S": r[:, o_s:o_l], "lam": r[:, o_l:o_e], "e": r[:, o_e:o_e + k]}
    return out, fields
