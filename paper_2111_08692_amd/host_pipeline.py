"""Host-resident conversions: input and output in host memory, transferred
in chunks that overlap host-to-device copies, kernels and device-to-host
copies on a few streams (for data that comes from disk or the network).

The input is cut into chunks at character boundaries: a UTF-8 cut moves
forward over at most three continuation bytes, a UTF-16 cut moves past a
low surrogate.  Then every chunk is validated and converted on its own by
the single-buffer kernels, and the results compose exactly: the input is
valid iff every chunk is, its first error is the first error of the first
chunk that has one (offset by the chunk's start), and the output is the
chunks' outputs back to back.  (If a run of four or more continuation bytes
straddles a cut, an error lies at or before the cut's end of that run, so
the first failing chunk still reports the input's first error.)

Per chunk and stream: the host copies the chunk into a pinned staging
buffer, then the stream copies it to the device, converts it and copies
the result back.  When the stream is needed again the host reads that
result and queues the copy of exactly the chunk's output to a pinned
buffer; the host moves it into the caller's output array one round later,
so device-to-host copies overlap the staging of the next chunks.  Chunks
are collected in order, so each output lands at the running sum of the
counts before it.  Host copies are torch CPU copies (several threads).
The throughput of this path is bounded by PCIe and host copies, not by
HBM.
"""
from __future__ import annotations

import time
from typing import List, Tuple

import numpy as np
import torch

from . import (OK, convert_utf8_to_utf16le, convert_utf8_to_utf16le_async, convert_utf16le_to_utf8,
               convert_utf16le_to_utf8_async, decode_result, load, result_tensor)


def cuts_utf8(data: np.ndarray, chunk: int) -> List[int]:
    """Chunk boundaries (0 and n included) at non-continuation bytes."""
    n = int(data.size)
    cuts = [0]
    c = chunk
    while c < n:
        k = c
        while k < n and k < c + 3 and (int(data[k]) & 0xC0) == 0x80:
            k += 1
        if k > cuts[-1]:
            cuts.append(k)
        c = k + chunk
    if cuts[-1] != n:
        cuts.append(n)
    return cuts


def cuts_utf16(data: np.ndarray, chunk: int) -> List[int]:
    """Chunk boundaries (in units) that never separate a low surrogate from
    the unit before it."""
    m = int(data.size)
    cuts = [0]
    c = chunk
    while c < m:
        k = c + 1 if 0xDC00 <= int(data[c]) <= 0xDFFF else c
        if k > cuts[-1]:
            cuts.append(k)
        c = k + chunk
    if cuts[-1] != m:
        cuts.append(m)
    return cuts


class HostPipeline:
    """Pinned staging and device buffers for ``nstreams`` chunks in flight."""

    def __init__(self, chunk_bytes: int = 64 << 20, nstreams: int = 3, device: str = "cuda"):
        load()
        self.chunk = int(chunk_bytes)
        self.dev = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(nstreams)]   # default priority
        cap_in = self.chunk + 8   # a cut moves forward by at most 3 bytes / 1 unit
        self.h_in = [torch.empty(cap_in, dtype=torch.uint8).pin_memory() for _ in range(nstreams)]
        self.d_in = [torch.empty(cap_in, dtype=torch.uint8, device=self.dev) for _ in range(nstreams)]
        # worst-case outputs: 2 bytes per UTF-8 byte, 1.5 bytes per UTF-16 byte
        self.h_out = [torch.empty(2 * cap_in, dtype=torch.uint8).pin_memory() for _ in range(nstreams)]
        self.d_out = [torch.empty(2 * cap_in, dtype=torch.uint8, device=self.dev) for _ in range(nstreams)]
        self.d_res = [result_tensor(self.dev) for _ in range(nstreams)]
        self.h_res = [torch.zeros(2, dtype=torch.int64).pin_memory() for _ in range(nstreams)]
        self.events = [None] * nstreams
        self.last = {}

    def _run(self, data: np.ndarray, to16: bool) -> Tuple[int, int, np.ndarray]:
        unit = 1 if to16 else 2          # input bytes per unit
        out_unit = 2 if to16 else 1      # output bytes per unit
        raw = np.ascontiguousarray(data).view(np.uint8)
        raw_t = torch.from_numpy(raw)
        cuts = cuts_utf8(data, self.chunk) if to16 else cuts_utf16(data, self.chunk // 2)
        ns = len(self.streams)
        # at most 2 output bytes per UTF-8 byte, 3 per UTF-16 unit
        final = np.empty(2 * raw.size if to16 else 3 * (raw.size // 2), dtype=np.uint8)
        final_t = torch.from_numpy(final)
        written = 0
        first_err = None
        pend = [None] * ns       # (chunk index, start unit) per stream: converted, result not read
        out_pend = [None] * ns   # (event, output offset, bytes) per stream: copy to h_out queued
        t0 = time.perf_counter()
        nchunks = len(cuts) - 1

        def finish_out(si):
            # the stream's last output copy is done: move it into place
            if out_pend[si] is None:
                return
            ev, off, nb = out_pend[si]
            ev.synchronize()
            final_t[off:off + nb].copy_(self.h_out[si][:nb])
            out_pend[si] = None

        def collect(si):
            # the chunk's result, then queue the copy of exactly its output
            nonlocal first_err, written
            ci, start = pend[si]
            pend[si] = None
            self.events[si].synchronize()
            st, cnt = decode_result(self.h_res[si])
            if st != OK:
                if first_err is None or ci < first_err[0]:
                    first_err = (ci, st, start + cnt)
                return
            if first_err is not None:
                return
            finish_out(si)   # h_out[si] is free again
            nb = cnt * out_unit
            s = self.streams[si]
            with torch.cuda.stream(s):
                self.h_out[si][:nb].copy_(self.d_out[si][:nb], non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(s)
            out_pend[si] = (ev, written, nb)
            written += nb

        for ci in range(nchunks):
            if first_err is not None and first_err[0] < ci:
                break
            si = ci % ns
            if pend[si] is not None:
                collect(si)
                if first_err is not None and first_err[0] < ci:
                    break
            a, b = cuts[ci], cuts[ci + 1]
            nb = (b - a) * unit
            hb = self.h_in[si]
            hb[:nb].copy_(raw_t[a * unit:b * unit])
            s = self.streams[si]
            with torch.cuda.stream(s):
                self.d_in[si][:nb].copy_(hb[:nb], non_blocking=True)
                if to16:
                    d = self.d_in[si][:nb]
                    out = self.d_out[si].view(torch.int16)
                    rc = convert_utf8_to_utf16le_async(d, out, self.d_res[si], out_cap=out.numel(), stream=s)
                else:
                    d = self.d_in[si][:nb].view(torch.int16)
                    out = self.d_out[si]
                    rc = convert_utf16le_to_utf8_async(d, out, self.d_res[si], out_cap=out.numel(), stream=s)
                if rc != 0:
                    raise RuntimeError(f"call failed: {rc}")
                self.h_res[si].copy_(self.d_res[si], non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(s)
            self.events[si] = ev
            pend[si] = (ci, a)
        # the remaining chunks in order (ci, ci + 1, ... wrap around the streams)
        for k in range(ns):
            si = (nchunks + k) % ns
            if pend[si] is not None:
                collect(si)
        for k in range(ns):
            si = (nchunks + k) % ns
            if out_pend[si] is not None:
                finish_out(si)
        if first_err is not None:
            # the output of the valid prefix: the chunks before the failing
            # one (already in place) and the failing chunk's valid part,
            # converted again from its device input (its stream has run
            # nothing after it)
            ci, st, pos = first_err
            si = ci % ns
            k = pos - cuts[ci]   # valid units of the failing chunk
            if k > 0:
                s = self.streams[si]
                with torch.cuda.stream(s):
                    if to16:
                        st2, cnt2, o = convert_utf8_to_utf16le(self.d_in[si][:k], stream=s)
                    else:
                        st2, cnt2, o = convert_utf16le_to_utf8(self.d_in[si][:2 * k].view(torch.int16), stream=s)
                if st2 != OK:
                    raise RuntimeError(f"the valid prefix of chunk {ci} did not convert: {st2}")
                nb = cnt2 * out_unit
                final_t[written:written + nb].copy_(o.view(torch.uint8)[:nb])
                written += nb
        torch.cuda.synchronize(self.dev)
        self.last = {"seconds": time.perf_counter() - t0, "chunks": nchunks, "input_bytes": raw.size}
        out = final[:written]
        out = out.view(np.uint16) if to16 else out
        if first_err is not None:
            return first_err[1], first_err[2], out
        return OK, int(out.size), out

    def convert_utf8_to_utf16le(self, data: np.ndarray) -> Tuple[int, int, np.ndarray]:
        """Host uint8 array -> ``(status, count, uint16 array)``; on an error
        ``(kind, first error, the words of the valid prefix)``."""
        return self._run(np.asarray(data, dtype=np.uint8), True)

    def convert_utf16le_to_utf8(self, data: np.ndarray) -> Tuple[int, int, np.ndarray]:
        """Host uint16 array -> ``(status, count, uint8 array)``; on an error
        ``(kind, first error, the bytes of the valid prefix)``."""
        return self._run(np.asarray(data, dtype=np.uint16), False)
