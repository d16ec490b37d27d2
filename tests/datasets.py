"""Seeded test datasets: random draws from paper_2512_12904_amd.synth, keys and
ciphertexts computed by the CPU oracle (never by the GPU library)."""
import numpy as np

import oracle
from paper_2512_12904_amd import synth


def sizes(pid):
    p = oracle.param(pid)
    p["rho"] = (p["rm_d"] - 1) // 2
    return p


def pke(pid, count, master, shared_key=False):
    """count ciphertexts with their keys.  Own key per item (key id = item), or
    one key (id 0) for all.  Returns a dict of numpy arrays; m is the ground truth."""
    p = sizes(pid)
    nkeys = 1 if shared_key else count
    h, x, y = synth.keys(master, pid, p, nkeys)
    s = oracle.keygen_batch(pid, h, x, y)
    key_of = np.zeros(count, np.int64) if shared_key else np.arange(count, dtype=np.int64)
    m, r1, r2, e = synth.encryptions(master, pid, p, count, key_of=key_of)
    u, v = oracle.encrypt_batch(pid, h, s, m, r1, r2, e, key_of=key_of)
    y_items = y[key_of]
    return {"pid": pid, "h": h, "s": s, "y_keys": y, "key_of": key_of, "y": np.ascontiguousarray(y_items),
            "m": m, "u": u, "v": v}


def stress(pid, count, master, word_id0=0):
    """Decoder stress words: exactly delta symbol errors plus in-radius noise."""
    p = sizes(pid)
    m, bad, dval, noise = synth.stress(master, pid, p, count, word_id0=word_id0)
    r = oracle.stress_batch(pid, m, bad, dval, noise, out=noise)
    return {"pid": pid, "m": m, "r": r}
