"""Autotuning of the tile geometry and the scan schedule per operation and
input size class.

The library is compiled for several tile geometries (``geometries()``: waves
per workgroup, rows per wave, tile bytes) and runs the tile scan in one of
two schedules (``SCHEDULE_NAMES``: workgroups take tiles in block order, or
in the order they start, from a per-call ticket counter).  On every call it
looks up two process-wide tables (operation, size class) -> geometry and ->
schedule; the class of an input of b bytes is ceil(log2(b)).  Every choice
computes the same results; they differ in speed: large tiles amortise the
per-tile scan and look-back, small tiles put more workgroups on small
inputs, tickets cost a round trip per tile but keep look-back kernels on
concurrent streams from waiting on one another's unplaced workgroups.

``tune`` times every (geometry, schedule) pair on the caller's representative
text at a ladder of input sizes, for each operation asked for, with HIP
events.  With ``concurrency`` = N each timed round is N calls at once, one on
each of N streams (separate outputs, the same input), which is what a
server overlapping its calls sees: a geometry that wins alone can lose
there (the shipped table keeps 16 KiB tiles for large batched UTF-16LE calls
for that reason).  A measured class keeps the pair it had (the library's
shipped default, unless a table was installed) unless another is faster by
more than ``min_gain``; every other class takes the choice of the nearest
measured class.  The result is installed and returned as a JSON-ready dict;
``save`` and ``apply_file`` keep it in a JSON cache that records the library
version, the geometry list and the schedule names, so a cache from another
build is refused.

    python -m paper_2111_08692_amd.tune corpus.txt -o tune.json

All timed work is the library's own calls; this module only prepares inputs,
times and fills the table.
"""
from __future__ import annotations

import argparse
import json
import statistics
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import (OK, OP_BATCH_UTF8, OP_BATCH_UTF16LE, OP_CONVERT_UTF8, OP_CONVERT_UTF16LE, OP_VALIDATE_UTF8,
               OP_VALIDATE_UTF16LE, SCHEDULE_NAMES, SIZE_CLASSES, convert_utf8_to_utf16le,
               convert_utf8_to_utf16le_async, convert_utf8_to_utf16le_batch_async, convert_utf16le_to_utf8_async,
               convert_utf16le_to_utf8_batch_async, geometries, get_geometry, get_schedule, load, result_tensor,
               results_tensor, set_geometry, set_schedule, size_class, validate_utf8_async,
               validate_utf16le_async, version)

OPS = {
    "validate_utf8": OP_VALIDATE_UTF8,
    "convert_utf8_to_utf16le": OP_CONVERT_UTF8,
    "validate_utf16le": OP_VALIDATE_UTF16LE,
    "convert_utf16le_to_utf8": OP_CONVERT_UTF16LE,
    "convert_utf8_to_utf16le_batch": OP_BATCH_UTF8,
    "convert_utf16le_to_utf8_batch": OP_BATCH_UTF16LE,
}
DEFAULT_SIZES = tuple(1 << e for e in range(16, 29, 2))   # 64 KiB .. 256 MiB


def geometry_names() -> List[str]:
    return [f"{w}x{r}" for w, r, _ in geometries()]


def candidates(schedules: bool = True) -> List[Tuple[int, int]]:
    """The (geometry, schedule) pairs the tuner times: every geometry in
    block order, and with ``schedules`` every geometry in ticket order too."""
    ng = len(geometries())
    sched = range(len(SCHEDULE_NAMES)) if schedules else range(1)
    return [(g, s) for s in sched for g in range(ng)]


def candidate_name(g: int, s: int, names: Sequence[str]) -> str:
    return f"{names[g]}/{SCHEDULE_NAMES[s]}"


def nearest_fill(measured: Dict[int, int], nclasses: int = SIZE_CLASSES) -> List[int]:
    """Table row over every size class from the choices at the measured
    classes: each class takes the choice of the nearest measured class (the
    smaller one on a tie); no measurement leaves every class as it is (-1)."""
    if not measured:
        return [-1] * nclasses
    keys = sorted(measured)
    row = []
    for c in range(nclasses):
        best = min(keys, key=lambda m: (abs(m - c), m))
        row.append(measured[best])
    return row


def choose(times_us: Sequence[float], min_gain: float, current: int = 0) -> int:
    """Index of the geometry to use given per-geometry times: the fastest,
    unless it beats the ``current`` one by ``min_gain`` or less."""
    best = int(np.argmin(times_us))
    if best == current or times_us[best] * (1.0 + min_gain) >= times_us[current]:
        return current
    return best


def _cut_utf8(buf: np.ndarray, n: int) -> np.ndarray:
    """The first n bytes of buf, shortened to end before a character that
    would be split."""
    i = min(n, buf.size)
    while 0 < i < buf.size and (int(buf[i]) & 0xC0) == 0x80:
        i -= 1
    return buf[:i]


def _cut_utf16(buf: np.ndarray, m: int) -> np.ndarray:
    i = min(m, buf.size)
    if 0 < i < buf.size and 0xDC00 <= int(buf[i]) <= 0xDFFF:
        i -= 1
    return buf[:i]


def _string_offsets(units: np.ndarray, per_string: int, utf8: bool) -> np.ndarray:
    """Cuts every ``per_string`` units, moved back to character starts."""
    n = int(units.size)
    cuts = [0]
    c = per_string
    while c < n:
        k = c
        if utf8:
            while k > cuts[-1] and (int(units[k]) & 0xC0) == 0x80:
                k -= 1
        elif 0xDC00 <= int(units[k]) <= 0xDFFF:
            k -= 1
        if k > cuts[-1]:
            cuts.append(k)
        c += per_string
    cuts.append(n)
    return np.asarray(cuts, dtype=np.int64)


class _Inputs:
    """Device inputs of every ladder size, built from one valid UTF-8 sample."""

    def __init__(self, sample: np.ndarray, largest: int, device: torch.device):
        sample = np.ascontiguousarray(sample, dtype=np.uint8)
        if sample.size == 0:
            raise ValueError("empty sample")
        reps = -(-(largest + 4) // sample.size)
        self.u8 = np.tile(sample, reps)
        d = torch.from_numpy(self.u8).to(device)
        st, cnt, out = convert_utf8_to_utf16le(d)   # the library's own conversion
        if st != OK:
            raise ValueError(f"the sample is not valid UTF-8 (status {st} at {cnt})")
        self.u16 = out[:cnt].cpu().numpy().view(np.uint16)
        self.device = device
        del d, out

    def utf8(self, nbytes: int) -> torch.Tensor:
        return torch.from_numpy(np.ascontiguousarray(_cut_utf8(self.u8, nbytes))).to(self.device)

    def utf16(self, nbytes: int) -> torch.Tensor:
        w = np.ascontiguousarray(_cut_utf16(self.u16, nbytes // 2))
        return torch.from_numpy(w.view(np.int16)).to(self.device)


def _time_us(fn, min_ms: float, reps: int) -> float:
    """Median over ``reps`` runs of the mean time per call (us) of a loop
    of calls lasting at least ``min_ms``."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fn()
    e1.record()
    e1.synchronize()
    iters = max(1, int(min_ms / max(e0.elapsed_time(e1), 1e-3)))
    times = []
    for _ in range(reps):
        e0.record()
        for _ in range(iters):
            fn()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e3 / iters)
    return float(statistics.median(times))


def _call(op: int, data: torch.Tensor, per_string: int, stream=None):
    """A closure that enqueues one call of ``op`` on ``data`` on ``stream``
    (None: the current stream; outputs allocated once, outside the timed
    loop)."""
    dev = data.device
    res = result_tensor(dev)
    if op == OP_VALIDATE_UTF8:
        return lambda: _ok(validate_utf8_async(data, res, stream=stream))
    if op == OP_VALIDATE_UTF16LE:
        return lambda: _ok(validate_utf16le_async(data, res, stream=stream))
    if op == OP_CONVERT_UTF8:
        out = torch.empty(max(data.numel(), 1), dtype=torch.int16, device=dev)
        return lambda: _ok(convert_utf8_to_utf16le_async(data, out, res, stream=stream))
    if op == OP_CONVERT_UTF16LE:
        out = torch.empty(max(3 * data.numel(), 1), dtype=torch.uint8, device=dev)
        return lambda: _ok(convert_utf16le_to_utf8_async(data, out, res, stream=stream))
    host = data.cpu().numpy()
    if op == OP_BATCH_UTF8:
        offs = torch.from_numpy(_string_offsets(host, per_string, True)).to(dev)
        k = offs.numel() - 1
        out = torch.empty(max(2 * data.numel(), 1), dtype=torch.int16, device=dev)
        oo, rs = torch.empty(k + 1, dtype=torch.int64, device=dev), results_tensor(k, device=dev)
        return lambda: _ok(convert_utf8_to_utf16le_batch_async(data, offs, out, oo, rs, stream=stream))
    if op == OP_BATCH_UTF16LE:
        offs = torch.from_numpy(_string_offsets(host.view(np.uint16), per_string // 2, False)).to(dev)
        k = offs.numel() - 1
        out = torch.empty(max(3 * data.numel(), 1), dtype=torch.uint8, device=dev)
        oo, rs = torch.empty(k + 1, dtype=torch.int64, device=dev), results_tensor(k, device=dev)
        return lambda: _ok(convert_utf16le_to_utf8_batch_async(data, offs, out, oo, rs, stream=stream))
    raise ValueError(f"unknown operation {op}")


def _round(op: int, data: torch.Tensor, per_string: int, streams: Sequence[torch.cuda.Stream]):
    """A closure that enqueues one round: with one stream, one call on the
    current stream; with N streams, one call on each, forked from and joined
    back into the current stream, so that events on the current stream time
    the round."""
    if len(streams) <= 1:
        return _call(op, data, per_string)
    calls = [_call(op, data, per_string, stream=s) for s in streams]

    def run():
        cur = torch.cuda.current_stream()
        fork = torch.cuda.Event()
        fork.record(cur)
        for s, f in zip(streams, calls):
            s.wait_event(fork)
            f()
        for s in streams:
            join = torch.cuda.Event()
            join.record(s)
            cur.wait_event(join)
    return run


def _ok(rc: int) -> None:
    if rc != OK:
        raise RuntimeError(f"library call failed: {rc}")


def tune(sample: np.ndarray, ops: Sequence[str] = tuple(OPS), sizes: Sequence[int] = DEFAULT_SIZES,
         min_gain: float = 0.03, min_ms: float = 2.0, reps: int = 5, string_bytes: int = 4096,
         install: bool = True, device: str = "cuda", schedules: bool = True, concurrency: int = 1) -> dict:
    """Time every (geometry, schedule) pair (``candidates(schedules)``) for
    every operation in ``ops`` at every size in ``sizes`` (input bytes) on
    text cut from ``sample`` (valid UTF-8, host uint8, repeated as needed);
    batched operations cut their input into strings of about
    ``string_bytes``; each timed round is ``concurrency`` calls on as many
    streams.  Returns the tables and the measurements; with ``install`` the
    tables are also put in the library."""
    load()
    names = geometry_names()
    cands = candidates(schedules)
    cnames = [candidate_name(g, s, names) for g, s in cands]
    dev = torch.device(device)
    sizes = sorted(set(int(s) for s in sizes))
    concurrency = max(1, int(concurrency))
    streams = [torch.cuda.Stream(device=dev) for _ in range(concurrency)] if concurrency > 1 else []
    inputs = _Inputs(sample, max(sizes), dev)
    measured: Dict[str, list] = {}
    table: Dict[str, List[int]] = {}
    sched_table: Dict[str, List[int]] = {}
    saved_all = {op: [(get_geometry(OPS[op], c), get_schedule(OPS[op], c)) for c in range(SIZE_CLASSES)]
                 for op in OPS}
    saved = {op: saved_all[op] for op in ops}
    try:
        for name in ops:
            op = OPS[name]
            choices: Dict[int, int] = {}
            rows = []
            for nbytes in sizes:
                utf16 = op in (OP_VALIDATE_UTF16LE, OP_CONVERT_UTF16LE, OP_BATCH_UTF16LE)
                data = inputs.utf16(nbytes) if utf16 else inputs.utf8(nbytes)
                real = data.numel() * data.element_size()
                c = size_class(real)
                fn = _round(op, data, string_bytes, streams)
                before = saved_all[name][c]
                current = cands.index(before) if before in cands else 0
                times = []
                for g, s in cands:
                    _ok(set_geometry(op, c, g))
                    _ok(set_schedule(op, c, s))
                    if get_geometry(op, c) != g or get_schedule(op, c) != s:
                        raise RuntimeError("UTFGPU_GEOMETRY or UTFGPU_SCHEDULE is set: the table cannot be tuned")
                    times.append(_time_us(fn, min_ms, reps))
                pick = choose(times, min_gain, current)
                choices[c] = pick
                rows.append({"bytes": real, "class": c, "us": [round(t, 3) for t in times],
                             "before": cnames[current], "choice": cnames[pick]})
                del fn, data
            measured[name] = rows
            filled = nearest_fill(choices)
            table[name] = [cands[i][0] if i >= 0 else saved_all[name][c][0] for c, i in enumerate(filled)]
            sched_table[name] = [cands[i][1] if i >= 0 else saved_all[name][c][1] for c, i in enumerate(filled)]
    finally:
        for name, row in saved.items():   # restore, then install the result
            for c, (g, s) in enumerate(row):
                set_geometry(OPS[name], c, g)
                set_schedule(OPS[name], c, s)
        torch.cuda.synchronize()
    result = {"library": version(), "geometries": names, "schedules": list(SCHEDULE_NAMES),
              "candidates": cnames, "min_gain": min_gain, "string_bytes": string_bytes,
              "concurrency": concurrency, "measured": measured,
              "table": {op: [names[g] for g in row] for op, row in table.items()},
              "schedule": {op: [SCHEDULE_NAMES[s] for s in row] for op, row in sched_table.items()}}
    if install:
        apply(result)
    return result


def apply(result: dict) -> None:
    """Install the tables returned by ``tune`` (or read back from JSON)."""
    names = geometry_names()
    if result.get("geometries") != names:
        raise ValueError(f"tuning table for geometries {result.get('geometries')}, library has {names}")
    if result.get("schedules") != list(SCHEDULE_NAMES):
        raise ValueError(f"tuning table for schedules {result.get('schedules')}, library has {SCHEDULE_NAMES}")
    if result.get("library") != version():
        raise ValueError(f"tuning table for {result.get('library')!r}, library is {version()!r}")
    sched = result.get("schedule", {})
    if set(sched) != set(result["table"]):
        raise ValueError("the geometry and schedule tables cover different operations")
    for op, row in result["table"].items():   # check everything before installing anything
        if op not in OPS:
            raise ValueError(f"unknown operation {op!r}")
        if len(row) != SIZE_CLASSES or len(sched[op]) != SIZE_CLASSES:
            raise ValueError(f"{op}: {len(row)} / {len(sched[op])} size classes, expected {SIZE_CLASSES}")
        unknown = (set(row) - set(names)) | (set(sched[op]) - set(SCHEDULE_NAMES))
        if unknown:
            raise ValueError(f"{op}: unknown geometries or schedules {sorted(unknown)}")
    for op, row in result["table"].items():
        for c, gname in enumerate(row):
            _ok(set_geometry(OPS[op], c, names.index(gname)))
            _ok(set_schedule(OPS[op], c, SCHEDULE_NAMES.index(sched[op][c])))


def reset() -> None:
    """Every operation and class back to the library's shipped defaults."""
    for op in OPS.values():
        for c in range(SIZE_CLASSES):
            _ok(set_geometry(op, c, -1))
            _ok(set_schedule(op, c, -1))


def save(result: dict, path: str) -> None:
    with open(path, "w") as f:
        json.dump(result, f, indent=1)


def apply_file(path: str) -> dict:
    with open(path) as f:
        result = json.load(f)
    apply(result)
    return result


def main(argv: Optional[Sequence[str]] = None) -> int:
    ap = argparse.ArgumentParser(description="Tune the tile geometry and scan schedule on a UTF-8 text sample")
    ap.add_argument("sample", help="file of valid UTF-8 text (repeated to the largest size)")
    ap.add_argument("-o", "--out", required=True, help="JSON file to write")
    ap.add_argument("--ops", default=",".join(OPS), help="comma-separated operations")
    ap.add_argument("--sizes", default=",".join(str(s) for s in DEFAULT_SIZES), help="input bytes, comma-separated")
    ap.add_argument("--min-gain", type=float, default=0.03)
    ap.add_argument("--concurrency", type=int, default=1, help="calls timed at once, one per stream")
    ap.add_argument("--no-schedules", action="store_true", help="block order only")
    a = ap.parse_args(argv)
    sample = np.fromfile(a.sample, dtype=np.uint8)
    res = tune(sample, ops=a.ops.split(","), sizes=[int(s) for s in a.sizes.split(",")], min_gain=a.min_gain,
               schedules=not a.no_schedules, concurrency=a.concurrency)
    save(res, a.out)
    for op, rows in res["measured"].items():
        for r in rows:
            print(op, r["bytes"], r["choice"], r["us"], flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
