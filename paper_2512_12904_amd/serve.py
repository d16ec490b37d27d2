"""Continuous-batching decryption server on one GPU.

Requests (parameter set, b ciphertexts, each with its key id) arrive over
time.  The server keeps the secret keys device-resident (a KeyStore), and
runs S slots, each a HIP stream with its own device buffers of `budget / S`
bytes.  While earlier batches are on the GPU, newly arrived requests are
admitted into any free slot, as many as fit in its bytes (u + v + m + key id
of every item); a request larger than a slot is split across batches.  A
slot's batch is one keyed decryption launch over every parameter set present
(hqc_decrypt_mixed_keyed), with the ciphertexts and key ids copied
host-to-device on the slot's stream and the messages copied back; a request
is complete when all of its items are back on the host.  Latency is
measured from the request's arrival time to that point.  When the pools
carry the expected messages, every served message is compared with them.

Everything numeric runs in libhqc_gpu.so; this module schedules copies and
launches (PyTorch supplies pinned memory, device memory and streams).
"""
import collections
import time

import numpy as np
import torch

from . import hqc

SETS = (1, 3, 5)


class Request:
    __slots__ = ("rid", "pid", "key", "b", "arrival", "src", "done_items", "t_done", "m")

    def __init__(self, rid, pid, key, b, arrival, src):
        self.rid, self.pid, self.key, self.b, self.arrival, self.src = rid, pid, key, b, arrival, src
        self.done_items = 0
        self.t_done = None
        self.m = None


class _Slot:
    """One stream with device buffers for up to `cap[pid]` items per set."""

    def __init__(self, device, budget, sizes):
        self.stream = torch.cuda.Stream(device=device)
        self.event = None
        self.parts = []  # (request, first item, count, pid, offset in slot buffers)
        per_item = {pid: 8 * (s["u_words"] + s["v_words"]) + s["k"] + 4 for pid, s in sizes.items()}
        # the budget is shared by the three sets in proportion to their item size
        self.cap = {pid: max(1, int(budget // per_item[pid] // 3)) for pid in sizes}
        self.u = {pid: torch.empty((self.cap[pid], s["u_words"]), dtype=torch.int64, device=device)
                  for pid, s in sizes.items()}
        self.v = {pid: torch.empty((self.cap[pid], s["v_words"]), dtype=torch.int64, device=device)
                  for pid, s in sizes.items()}
        self.m = {pid: torch.empty((self.cap[pid], s["k"]), dtype=torch.uint8, device=device)
                  for pid, s in sizes.items()}
        self.kid = {pid: torch.empty(self.cap[pid], dtype=torch.int32, device=device) for pid in sizes}
        self.m_host = {pid: torch.empty((self.cap[pid], s["k"]), dtype=torch.uint8, pin_memory=True)
                       for pid, s in sizes.items()}
        self.fill = {pid: 0 for pid in sizes}

    def busy(self):
        return self.event is not None


class Server:
    """pools[pid] = dict(u=..., v=..., key=..., m=...): pinned host tensors
    u (int64 [rows, u_words]), v (int64 [rows, v_words]) and key (int32
    [rows], the key id of each ciphertext) that requests refer to (request
    src = first row, rows src .. src+b-1), and optionally m (numpy uint8
    [rows, k]), the message of each row, against which every served message
    is checked (counted in `mismatches`)."""

    def __init__(self, keystore, pools, streams=4, budget_bytes=512 << 20, device="cuda:0",
                 tile=0):
        self.ks = keystore
        self.pools = pools
        self.device = torch.device(device)
        self.sizes = {pid: hqc.sizes(pid) for pid in SETS}
        self.slots = [_Slot(self.device, budget_bytes // streams, self.sizes) for _ in range(streams)]
        self.tile = tile
        self.launches = 0
        self.checked = 0
        self.mismatches = 0

    # -- one batch --------------------------------------------------------
    def _launch(self, slot, queue):
        for pid in SETS:
            slot.fill[pid] = 0
        slot.parts = []
        with torch.cuda.stream(slot.stream):
            while queue:
                req, first = queue[0]
                pid = req.pid
                room = slot.cap[pid] - slot.fill[pid]
                if room <= 0:
                    break
                cnt = min(room, req.b - first)
                off = slot.fill[pid]
                pool = self.pools[pid]
                src = req.src + first
                slot.u[pid][off:off + cnt].copy_(pool["u"][src:src + cnt], non_blocking=True)
                slot.v[pid][off:off + cnt].copy_(pool["v"][src:src + cnt], non_blocking=True)
                slot.kid[pid][off:off + cnt].copy_(pool["key"][src:src + cnt], non_blocking=True)
                slot.parts.append((req, first, cnt, pid, off))
                slot.fill[pid] += cnt
                if first + cnt == req.b:
                    queue.popleft()
                else:
                    queue[0] = (req, first + cnt)
                    break  # this slot is full for that set
            items = [{"pid": pid, "u": slot.u[pid][:slot.fill[pid]],
                      "v": slot.v[pid][:slot.fill[pid]], "key_ids": slot.kid[pid][:slot.fill[pid]],
                      "out": slot.m[pid][:slot.fill[pid]]} for pid in SETS if slot.fill[pid]]
            # one launch for the whole batch, whatever sets it holds
            hqc.decrypt_mixed_keyed(self.ks, items, stream=slot.stream, tile=self.tile)
            self.launches += 1
            for pid in SETS:
                f = slot.fill[pid]
                if f:
                    slot.m_host[pid][:f].copy_(slot.m[pid][:f], non_blocking=True)
            slot.event = torch.cuda.Event()
            slot.event.record(slot.stream)

    def _collect(self, slot, now, keep_results):
        """Hand the finished batch's messages to their requests; returns the
        number of requests that became complete."""
        finished = 0
        for req, first, cnt, pid, off in slot.parts:
            want = self.pools[pid].get("m")
            if want is not None:
                got = slot.m_host[pid][off:off + cnt].numpy()
                src = req.src + first
                self.mismatches += int(np.count_nonzero((got != want[src:src + cnt]).any(axis=1)))
                self.checked += cnt
            if keep_results:
                if req.m is None:
                    req.m = np.empty((req.b, self.sizes[pid]["k"]), np.uint8)
                req.m[first:first + cnt] = slot.m_host[pid][off:off + cnt].numpy()
            req.done_items += cnt
            if req.done_items == req.b:
                req.t_done = now
                finished += 1
        slot.parts = []
        slot.event = None
        return finished

    # -- the loop ---------------------------------------------------------
    def run(self, requests, keep_results=False, realtime=True):
        """Serve `requests` (sorted by arrival, times in seconds from start).
        With realtime=False all requests are available at once."""
        queue = collections.deque()
        nxt = 0
        n = len(requests)
        t0 = time.perf_counter()
        done = 0
        while done < n:
            now = time.perf_counter() - t0
            while nxt < n and (not realtime or requests[nxt].arrival <= now):
                queue.append((requests[nxt], 0))
                nxt += 1
            progressed = False
            for slot in self.slots:
                if slot.busy() and slot.event.query():
                    done += self._collect(slot, time.perf_counter() - t0, keep_results)
                    progressed = True
                if not slot.busy() and queue:
                    self._launch(slot, queue)
                    progressed = True
            if not progressed:
                if nxt < n and realtime and not queue and not any(s.busy() for s in self.slots):
                    wait = requests[nxt].arrival - (time.perf_counter() - t0)
                    if wait > 2e-4:
                        time.sleep(wait - 1e-4)
                else:
                    time.sleep(0)
        wall = time.perf_counter() - t0
        return wall


def poisson_requests(rate_decrypts, seconds, counts, seed, b_max=4096, mix=(0.5, 0.3, 0.2),
                     pool_rows=None):
    """Arrivals at `rate_decrypts` offered decryptions per second (requests
    per second = rate / E[b]), parameter set drawn with `mix`, b uniform in
    1..b_max, the first ciphertext row uniform in the set's pool (the rows
    carry their own key ids; `key` records a uniform key id for the
    record only)."""
    rng = np.random.default_rng(seed)
    mean_b = (1 + b_max) / 2.0
    lam = rate_decrypts / mean_b
    reqs = []
    t = 0.0
    rid = 0
    while True:
        t += rng.exponential(1.0 / lam)
        if t > seconds:
            break
        pid = SETS[int(rng.choice(3, p=mix))]
        b = int(rng.integers(1, b_max + 1))
        key = int(rng.integers(0, counts[pid]))
        rows = pool_rows[pid]
        src = int(rng.integers(0, rows - b + 1))
        reqs.append(Request(rid, pid, key, b, t, src))
        rid += 1
    return reqs


def latency_stats(reqs, wall):
    lat = np.array([r.t_done - r.arrival for r in reqs])
    items = sum(r.b for r in reqs)
    out = {"requests": len(reqs), "decrypts": items,
           "achieved_decrypts_per_s": items / wall if wall > 0 else 0.0,
           "p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
           "p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None}
    for pid in SETS:
        sub = np.array([r.t_done - r.arrival for r in reqs if r.pid == pid])
        if len(sub):
            out["HQC-%d_p99_ms" % pid] = float(np.percentile(sub, 99) * 1e3)
    return out
