"""Continuous-batching transcoding server over the C ABI (one GPU).

Requests arrive open-loop (each has an arrival time).  Output space comes
from one device-resident arena whose size is set from the device's free HBM
when the server starts: the free memory reported by the runtime, less a
reserve left for the library's workspaces and other users, capped by a
configurable budget.  The scheduler loop, on every pass:

* takes the requests that have arrived and admits them while their output
  fits in the arena (space is reserved per request for the worst case of
  any input: 4 bytes per input byte for UTF-8 -> UTF-16LE, since a byte
  >= F0 counts two words even in an invalid request and the offsets of the
  requests after it include them; 3 bytes per input unit for UTF-16LE ->
  UTF-8); requests that do not fit are held back until completions free
  space;
* launches the admitted requests of each direction as ONE batched call
  (their payloads lie back to back in device memory) on the next of
  ``nstreams`` streams, and queues a device-to-host copy of their results
  behind it;
* polls the events of the launches in flight, stamps the completion time of
  every finished one, and frees arena space in launch order (the arena is
  a ring).

Latency is completion time minus arrival time; throughput is input bytes
over the span from the first arrival to the last completion.  Every
conversion runs in the library's kernels; this module only schedules.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Deque, List, Optional, Tuple

import numpy as np
import torch

from . import convert_utf8_to_utf16le_batch_async, convert_utf16le_to_utf8_batch_async, load, results_tensor


@dataclass
class _Flight:
    event: torch.cuda.Event
    ids: np.ndarray           # request ids of this launch
    kind: int                 # 0: UTF-8 -> UTF-16LE, 1: the reverse
    held: int                 # arena bytes held until completion
    start: int = 0            # arena byte offset of the launch's output
    done: bool = False


@dataclass
class ServeResult:
    """Per request: status, count, output offset (bytes into the output
    arena) and latency (s); plus the run's totals: ``held_back`` requests
    arrived while the arena had no room for them and waited for
    completions (``held_passes`` scheduler passes refused a batch)."""
    status: np.ndarray
    count: np.ndarray
    out_off: np.ndarray
    latency: np.ndarray
    span_s: float
    input_bytes: int
    launches: int
    max_inflight: int
    held_back: int = 0
    held_passes: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def gbps(self) -> float:
        return self.input_bytes / self.span_s / 1e9 if self.span_s > 0 else 0.0

    def percentile_us(self, q: float) -> float:
        return float(np.percentile(self.latency, q) * 1e6)


class _Ring:
    """Byte ring over an output arena; frees in allocation order."""

    def __init__(self, size: int):
        self.size = size
        self.head = 0
        self.used = 0

    def alloc(self, nbytes: int) -> Optional[Tuple[int, int]]:
        """(start, bytes charged) or None when it does not fit now."""
        if nbytes > self.size:
            raise ValueError("request larger than the output arena")
        start, waste = self.head, 0
        if start + nbytes > self.size:   # does not fit before the end: start over at 0
            waste, start = self.size - start, 0
        if self.used + waste + nbytes > self.size:
            return None
        self.used += waste + nbytes
        self.head = start + nbytes
        return start, waste + nbytes

    def free(self, nbytes: int) -> None:
        self.used -= nbytes
        if self.used == 0:   # empty: the next allocation may use the whole ring
            self.head = 0


ALIGN = 256   # arena reservations start on 256-byte boundaries


def reservation(kind: int, units: int) -> int:
    """Arena bytes reserved for ``units`` input units of direction ``kind``
    (the worst-case output of any input, rounded up to ``ALIGN``)."""
    per_unit = 4 if kind == 0 else 3
    return -(-per_unit * int(units) // ALIGN) * ALIGN


def prewarm_windows(off: np.ndarray, kind: int, max_batch_bytes: int, pool_bytes: int) -> List[Tuple[int, int]]:
    """Queue windows [i, j) of one direction (``off``: its requests' unit
    offsets) with the most input units and with the most requests among
    the batches ``Server.run`` can form when every request has arrived:
    from any i, up to the batch limit in input bytes, at least one request,
    and an output reservation (4 bytes per UTF-8 byte, 3 per UTF-16LE unit)
    that fits the pool."""
    nq = int(off.size) - 1
    if nq <= 0:
        return []
    per_unit = 4 if kind == 0 else 3
    i = np.arange(nq)
    j = np.maximum(np.searchsorted(off, off[:-1] + max_batch_bytes // (1 + kind), side="right") - 1, i + 1)
    # a reservation that does not fit the pool is admitted shorter
    fit = np.searchsorted(off, off[:-1] + pool_bytes // per_unit, side="right") - 1
    j = np.where(per_unit * (off[j] - off[i]) <= pool_bytes, j, np.maximum(np.minimum(j, fit), i + 1))
    units = off[j] - off[i]
    ok = per_unit * units <= pool_bytes
    if not ok.any():
        return []
    picks = {int(np.argmax(np.where(ok, units, -1))), int(np.argmax(np.where(ok, j - i, -1)))}
    return [(a, int(j[a])) for a in sorted(picks)]


class Server:
    """Device-resident payload arenas, one output arena sized from free HBM
    and a stream pool.  ``reqs`` is a ``workloads.RequestSet``.

    The output arena takes ``min(hbm_budget, free HBM - hbm_reserve)`` bytes,
    the free HBM being read from the runtime after the payloads are on the
    device.  Its size is ``arena_bytes``; a request whose reservation alone
    exceeds it is refused at construction."""

    def __init__(self, reqs, nstreams: int = 4, hbm_budget: int = 8 << 30, hbm_reserve: int = 2 << 30,
                 max_inflight: int = 16, max_batch_bytes: int = 256 << 20, device: str = "cuda"):
        load()
        self.r = reqs
        self.dev = torch.device(device)
        self.n = int(reqs.arrival.size)
        self.d8 = torch.from_numpy(reqs.data8).to(self.dev)
        self.d16 = torch.from_numpy(reqs.data16.view(np.int16)).to(self.dev)
        self.off8_dev = torch.from_numpy(reqs.off8).to(self.dev)
        self.off16_dev = torch.from_numpy(reqs.off16).to(self.dev)
        torch.cuda.synchronize(self.dev)
        free, _ = torch.cuda.mem_get_info(self.dev)
        self.free_hbm_at_start = int(free)
        arena = min(int(hbm_budget), int(free) - int(hbm_reserve))
        self.arena_bytes = max(arena, 0) // ALIGN * ALIGN
        largest = max([reservation(0, int(d)) for d in np.diff(reqs.off8)] +
                      [reservation(1, int(d)) for d in np.diff(reqs.off16)] + [0])
        if largest > self.arena_bytes:
            raise ValueError(f"the output arena ({self.arena_bytes} bytes: budget {hbm_budget}, free HBM {free}, "
                             f"reserve {hbm_reserve}) cannot hold the largest request ({largest} bytes)")
        self.arena = torch.empty(max(self.arena_bytes, ALIGN), dtype=torch.uint8, device=self.dev)
        self.out16 = self.arena.view(torch.int16)   # UTF-16 words (reservations start on even bytes)
        self.out8 = self.arena
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(nstreams)]          # default priority
        self.max_inflight = max_inflight
        self.max_batch_bytes = max_batch_bytes
        n8, n16 = int(reqs.ids8.size), int(reqs.ids16.size)
        # results by position in each direction's queue (pinned host copies)
        self.res8_host = torch.zeros((max(n8, 1), 2), dtype=torch.int64).pin_memory()
        self.res16_host = torch.zeros((max(n16, 1), 2), dtype=torch.int64).pin_memory()
        torch.cuda.synchronize()

    def _launch(self, kind: int, i: int, j: int, start: int, s: torch.cuda.Stream):
        """One batched call on stream ``s`` over positions i..j-1 of the
        queue of direction ``kind`` (0: UTF-8 -> UTF-16LE), output from byte
        ``start`` of the arena (a multiple of ``ALIGN``); returns the device
        output offsets and results."""
        off_k, off_dev = (self.r.off8, self.off8_dev) if kind == 0 else (self.r.off16, self.off16_dev)
        k, nu = j - i, int(off_k[j] - off_k[i])
        with torch.cuda.stream(s):
            offs = off_dev[i:j + 1] - int(off_k[i])
            oo = torch.empty(k + 1, dtype=torch.int64, device=self.dev)
            res = results_tensor(k, device=self.dev)
            if kind == 0:
                out = self.out16[start // 2:start // 2 + 2 * nu] if nu else self.out16[:1]
                rc = convert_utf8_to_utf16le_batch_async(self.d8[int(off_k[i]):int(off_k[j])], offs, out,
                                                         oo, res, out_cap=2 * nu, stream=s)
            else:
                out = self.out8[start:start + 3 * nu] if nu else self.out8[:1]
                rc = convert_utf16le_to_utf8_batch_async(self.d16[int(off_k[i]):int(off_k[j])], offs, out,
                                                         oo, res, out_cap=3 * nu, stream=s)
        if rc != 0:
            raise RuntimeError(f"batched call failed: {rc}")
        return oo, res

    def prewarm(self) -> None:
        """Bring every stream's library workspace to the size the largest
        batch of this request set needs, so that no call made while requests
        are served has to grow one (growing drains the stream and frees
        device memory, which waits for the whole device).  Per direction
        and stream, one batched call over the window of queued requests
        with the most input and one over the window with the most requests,
        each as long as ``run`` may form a batch (the batch limit and the
        output arena).  Run it again after changing the geometry table."""
        r = self.r
        for kind, off in ((0, r.off8), (1, r.off16)):
            wins = prewarm_windows(off, kind, self.max_batch_bytes, self.arena_bytes)
            for s in self.streams:
                for i, j in wins:
                    self._launch(kind, i, j, 0, s)
                s.synchronize()   # the calls share the pool's first bytes

    def run(self, time_scale: float = 1.0, collect: bool = False) -> ServeResult:
        """Serve every request once, replaying arrivals in wall-clock time
        (``time_scale`` stretches the schedule).  With ``collect`` every
        launch's output is copied to the host as it completes, before its
        arena space can be reused, so that ``output_of`` returns any
        request's output after the run (for checking; it slows the loop)."""
        r = self.r
        n = self.n
        arr = r.arrival * time_scale
        arr8 = arr[r.ids8] if r.ids8.size else np.zeros(0)
        arr16 = arr[r.ids16] if r.ids16.size else np.zeros(0)
        out_off = np.full(n, -1, dtype=np.int64)
        done_t = np.zeros(n)
        ring = _Ring(self.arena_bytes)
        inflight: Deque[_Flight] = collections.deque()
        batch_offsets = []   # (ids, device out_offsets, arena byte base, kind) of the batched launches
        queue = [{"arr": arr8, "off": r.off8, "off_dev": self.off8_dev, "ids": r.ids8, "host": self.res8_host,
                  "next": 0},
                 {"arr": arr16, "off": r.off16, "off_dev": self.off16_dev, "ids": r.ids16, "host": self.res16_host,
                  "next": 0}]
        finished = launches = max_inflight = si = held_passes = 0
        held = np.zeros(n, dtype=bool)   # requests that arrived and had to wait for arena space
        blobs = []                       # collect: (arena start, host copy) per completed launch
        blob_of = np.full(n, -1, dtype=np.int64)
        t0 = time.perf_counter()
        while finished < n:
            now = time.perf_counter() - t0
            launched = False
            # each direction: the arrived requests (up to the batch limit) in one batched call
            for kind in (0, 1):
                q = queue[kind]
                arr_k, off_k = q["arr"], q["off"]
                i = q["next"]
                if i >= arr_k.size or arr_k[i] > now or len(inflight) >= self.max_inflight:
                    continue
                j = max(int(np.searchsorted(arr_k, now, side="right")), i + 1)
                lim = int(np.searchsorted(off_k, off_k[i] + self.max_batch_bytes // (1 + kind), side="right")) - 1
                j = min(j, max(lim, i + 1))
                got = ring.alloc(reservation(kind, int(off_k[j] - off_k[i])))
                while got is None and j > i + 1:   # admit a shorter prefix of the queue
                    j = i + (j - i) // 2
                    got = ring.alloc(reservation(kind, int(off_k[j] - off_k[i])))
                if got is None:   # held back until completions free arena space
                    if not inflight and ring.used == 0:
                        raise RuntimeError(f"request {int(q['ids'][i])} cannot be admitted into an empty arena")
                    held[q["ids"][i:max(int(np.searchsorted(arr_k, now, side="right")), i + 1)]] = True
                    held_passes += 1
                    continue
                start, charged = got
                k = j - i
                s = self.streams[si % len(self.streams)]
                si += 1
                with torch.cuda.stream(s):
                    oo, res = self._launch(kind, i, j, start, s)
                    q["host"][i:j].copy_(res[:k], non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(s)
                ids = q["ids"][i:j]
                batch_offsets.append((ids, oo, start, kind))
                inflight.append(_Flight(ev, ids, kind, charged, start))
                q["next"] = j
                launches += 1
                launched = True
            max_inflight = max(max_inflight, len(inflight))
            # completion stamps for every finished launch; space back in launch order
            t = time.perf_counter() - t0
            for f in inflight:
                if not f.done and f.event.query():
                    if collect:
                        blob_of[f.ids] = len(blobs)
                        blobs.append((f.start, self.arena[f.start:f.start + f.held].cpu().numpy()))
                    f.done = True
                    done_t[f.ids] = t
                    finished += f.ids.size
            freed = False
            while inflight and inflight[0].done:
                f = inflight.popleft()
                ring.free(f.held)
                freed = True
            if not launched and not freed:
                if inflight:
                    time.sleep(0)
                else:
                    nxt = min(q["arr"][q["next"]] if q["next"] < q["arr"].size else np.inf for q in queue)
                    wait = nxt - (time.perf_counter() - t0)
                    if wait > 0.0005:
                        time.sleep(wait - 0.0003)
        torch.cuda.synchronize()
        for ids, oo, base, kind in batch_offsets:   # arena byte offsets
            out_off[ids] = base + (2 if kind == 0 else 1) * oo[:-1].cpu().numpy()
        status = np.zeros(n, dtype=np.int32)
        count = np.zeros(n, dtype=np.int64)
        for ids, host, m in ((r.ids8, self.res8_host, r.ids8.size), (r.ids16, self.res16_host, r.ids16.size)):
            v = host[:m].numpy()
            st = (v[:, 0] & 0xFFFFFFFF).astype(np.int64)
            status[ids] = np.where(st >= 1 << 31, st - (1 << 32), st).astype(np.int32)
            count[ids] = v[:, 1]
        latency = done_t - arr
        span = float(done_t.max() - arr.min()) if n else 0.0
        return ServeResult(status=status, count=count, out_off=out_off, latency=latency, span_s=span,
                           input_bytes=int(r.size.sum()), launches=launches, max_inflight=max_inflight,
                           held_back=int(held.sum()), held_passes=held_passes,
                           extra={"blobs": blobs, "blob_of": blob_of} if collect else {})

    def output_of(self, res: ServeResult, rid: int) -> np.ndarray:
        """The output units of request ``rid`` after ``run`` (a valid
        request): from the host copy taken at its completion when the run
        collected outputs, else from the arena (valid only while later
        launches have not reused its space)."""
        cnt, o = int(res.count[rid]), int(res.out_off[rid])
        nbytes = 2 * cnt if self.r.kind[rid] == 0 else cnt
        if "blobs" in res.extra:
            start, blob = res.extra["blobs"][int(res.extra["blob_of"][rid])]
            b = blob[o - start:o - start + nbytes]
        else:
            b = self.arena[o:o + nbytes].cpu().numpy()
        return b.view(np.uint16) if self.r.kind[rid] == 0 else b
