#!/usr/bin/env python3
"""Benchmark: validating UTF-8 <-> UTF-16LE transcoding on one MI355X.

One step converts, with validation, every buffer of the 1 GiB script-mix
workload in both directions:

* UTF-8 -> UTF-16LE: five 1 GiB UTF-8 buffers (ASCII, Latin, Cyrillic, CJK,
  emoji mixes) and their invalid variants (errors injected at a rate of
  1e-6 per byte);
* UTF-16LE -> UTF-8: five 1 GiB UTF-16LE buffers of the same mixes and their
  invalid variants (unpaired surrogates at a rate of 1e-6 per word).

Inputs and outputs are resident in HBM before timing starts; each step
enqueues the 20 conversions (asynchronous C-ABI calls) and copies their 20
results back to the host.  ``value`` is input bytes per second over the
timed steps.  Per-launch HIP events give every kernel's duration; the
roofline entry is the dominant kernel's algorithmic bytes (input read +
output written) per second against the 8 TB/s HBM peak.  The length and
validate-only kernels, the 1 MiB single-buffer latency, the batched and
served workloads (each beside plain single-buffer calls on the same bytes)
and the CPU oracle (on the host's cores, and on one core over a bounded
sample, with the CPU model) are reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--size-mib S]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import re
import multiprocessing as mp
import os
import statistics
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from workloads import (SCRIPT_MIXES, SEED_MIX1M, SEED_UTF8, SEED_UTF8_INVALID, SEED_UTF16,  # noqa: E402
                       SEED_UTF16_INVALID, make_buffer)

METRIC = "input GB/s validated+transcoded (UTF-8<->UTF-16LE) and % of HBM roofline, 1 GPU"
HBM_PEAK_GBS = 8000.0
ERROR_RATE = 1e-6
KERNEL_SOURCES = ["paper_2111_08692_amd/csrc/device_common.hpp", "paper_2111_08692_amd/csrc/utf8_kernels.hip",
                  "paper_2111_08692_amd/csrc/utf16_kernels.hip", "paper_2111_08692_amd/csrc/geometries.def"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the kernel sources' code (comments and blank lines left out,
    so the traffic figures stay attached to an unchanged kernel)."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
        for line in text.splitlines():
            code = re.sub(r"//.*", "", line).rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


# ---------------------------------------------------------------------------
# inputs
# ---------------------------------------------------------------------------

SERVE_REQUESTS = 10_000


def generate(size: int, serve: bool = True):
    """All buffers of the workload (host numpy), generated before any GPU
    work so the generator can fork worker processes."""
    ex = ProcessPoolExecutor(max_workers=16, mp_context=mp.get_context("fork"))
    bufs = []
    t0 = time.time()
    for mix in SCRIPT_MIXES:
        for enc, seed, eseed in (("utf-8", SEED_UTF8[mix], SEED_UTF8_INVALID[mix]),
                                 ("utf-16-le", SEED_UTF16[mix], SEED_UTF16_INVALID[mix])):
            valid = make_buffer(mix, size, seed, encoding=enc, executor=ex)
            bad = make_buffer(mix, size, seed, encoding=enc, error_rate=ERROR_RATE, error_seed=eseed, executor=ex)
            bufs.append((mix, enc, "valid", valid))
            bufs.append((mix, enc, "invalid", bad))
            log(f"generated {mix} {enc} ({time.time() - t0:.1f}s)")
    small = make_buffer("mix1m", 1 << 20, SEED_MIX1M)
    reqs = None
    if serve:
        from workloads import make_requests
        reqs = make_requests(SERVE_REQUESTS, executor=ex)
        log(f"generated {SERVE_REQUESTS} serving requests ({time.time() - t0:.1f}s)")
    ex.shutdown()
    return bufs, small, reqs


def cut_utf8(a: np.ndarray, n: int) -> np.ndarray:
    n = min(n, a.size)
    while 0 < n < a.size and (a[n] & 0xC0) == 0x80:
        n -= 1
    return a[:n]


def cut_utf16(a: np.ndarray, m: int) -> np.ndarray:
    m = min(m, a.size)
    if 0 < m < a.size and 0xD800 <= a[m - 1] <= 0xDBFF:
        m -= 1
    return a[:m]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _slices(a: np.ndarray, enc: str, parts: int):
    """``parts`` consecutive slices of ``a`` cut at character starts (a cut is
    moved forward past continuation bytes / low surrogates)."""
    cuts = [0]
    for k in range(1, parts):
        c = max(cuts[-1], a.size * k // parts)
        if enc == "utf-8":
            while c < a.size and (a[c] & 0xC0) == 0x80:
                c += 1
        elif c < a.size and 0xDC00 <= a[c] <= 0xDFFF:
            c += 1
        cuts.append(c)
    cuts.append(a.size)
    return [a[cuts[i]:cuts[i + 1]] for i in range(parts)]


def cpu_baseline(bufs, sample_bytes: int):
    """The oracle on the host: one thread on the first ``sample_bytes`` of
    every valid buffer, and all the host's cores on the whole valid buffers
    (each buffer cut at character starts into one slice per thread, every
    slice converted on its own; the oracle's C calls release the GIL, so
    the threads run in parallel)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle.build(force=False)
    total_in = 0
    total_t = 0.0
    for mix, enc, kind, b in bufs:
        if kind != "valid":
            continue
        if enc == "utf-8":
            s = cut_utf8(b.data, sample_bytes)
            t = time.perf_counter()
            st, cnt, _ = oracle.convert_utf8_to_utf16le(s)
            total_t += time.perf_counter() - t
            total_in += s.size
        else:
            s = cut_utf16(b.data, sample_bytes // 2)
            t = time.perf_counter()
            st, cnt, _ = oracle.convert_utf16le_to_utf8(s)
            total_t += time.perf_counter() - t
            total_in += 2 * s.size
        assert st == 0, (mix, enc, st)
    one_core = total_in / total_t / 1e9
    threads = len(os.sched_getaffinity(0))
    all_in, all_t = 0, 0.0
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for mix, enc, kind, b in bufs:
            if kind != "valid":
                continue
            conv = oracle.convert_utf8_to_utf16le if enc == "utf-8" else oracle.convert_utf16le_to_utf8
            parts = _slices(b.data, enc, threads)
            t = time.perf_counter()
            res = list(ex.map(conv, parts))
            all_t += time.perf_counter() - t
            all_in += b.data.nbytes
            assert all(r[0] == 0 for r in res), (mix, enc)
            del res
    return {"value": round(all_in / all_t / 1e9, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"all-core: the 10 valid buffers whole ({all_in / 2**30:.1f} GiB, {threads} threads, each "
                      f"buffer cut at character starts into one slice per thread), {all_t:.1f} s; one core: first "
                      f"{sample_bytes >> 20} MiB of each, {total_in / 2**30:.2f} GiB, {total_t:.1f} s",
            "single_core_GBps": round(one_core, 4), "cpu_model": cpu_model(), "host_threads": threads}


# ---------------------------------------------------------------------------
# main
# ---------------------------------------------------------------------------

def copy_reference(dev, stream, aux):
    """A plain 1 GiB device-to-device copy (the runtime's copy kernel): the
    HBM rate a streaming kernel can practically reach on this device, for
    reading the roofline fractions (bytes read + written per second)."""
    import torch
    a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
    for s_, e_ in ev:
        s_.record(stream)
        b.copy_(a)
        e_.record(stream)
    torch.cuda.synchronize()
    t = statistics.median(s_.elapsed_time(e_) for s_, e_ in ev) / 1e3
    aux["d2d_copy_1gib_GBps"] = round(2 * (1 << 30) / t / 1e9, 1)
    aux["d2d_copy_1gib_frac"] = round(2 * (1 << 30) / t / 1e9 / HBM_PEAK_GBS, 3)
    del a, b


def one_mib_latency(G, small, dev, stream, res, aux):
    """Latency of one synchronous 1 MiB call and the kernel time of one
    asynchronous call (the single-buffer 1 MiB case)."""
    import torch
    ds = torch.from_numpy(small.data).to(dev)
    o16 = torch.empty(small.data.size, dtype=torch.int16, device=dev)
    for _ in range(20):
        G.convert_utf8_to_utf16le(ds, out=o16)
    lat = []
    for _ in range(200):
        t = time.perf_counter()
        st, cnt, _ = G.convert_utf8_to_utf16le(ds, out=o16)
        lat.append(time.perf_counter() - t)
    assert st == 0
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(50)]
    for s_, e_ in ev:
        s_.record(stream)
        G.convert_utf8_to_utf16le_async(ds, o16, res[0])
        e_.record(stream)
    torch.cuda.synchronize()
    kt = statistics.median(s_.elapsed_time(e_) for s_, e_ in ev) / 1e3
    aux["mix1m_8to16_sync_call_us_p50"] = round(statistics.median(lat) * 1e6, 1)
    aux["mix1m_8to16_kernel_us"] = round(kt * 1e6, 1)
    aux["mix1m_8to16_kernel_input_GBps"] = round(small.data.size / kt / 1e9, 1)


def batch_leg(G, dev, stream, aux):
    """The batched workload: 100 000 independent UTF-8 strings (log-normal
    lengths, median 256 B, sigma 1.5, 16 B .. 1 MiB, one script mix each,
    1% with one injected error) converted by one batched call, against the
    same strings converted by one asynchronous single-buffer call each."""
    import torch
    from workloads.mixes import make_batch
    b = make_batch()
    k = b.offsets.size - 1
    d = torch.from_numpy(b.data).to(dev)
    offs = torch.from_numpy(b.offsets).to(dev)
    tot = torch.zeros(1, dtype=torch.int64, device=dev)
    G.utf16_length_from_utf8_async(d, tot)
    total = int(tot.item())
    out = torch.empty(max(total, 1), dtype=torch.int16, device=dev)
    oo = torch.empty(k + 1, dtype=torch.int64, device=dev)
    rs = G.results_tensor(k, device=dev)
    for _ in range(3):
        assert G.convert_utf8_to_utf16le_batch_async(d, offs, out, oo, rs) == 0
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
    for s_, e_ in ev:
        s_.record(stream)
        G.convert_utf8_to_utf16le_batch_async(d, offs, out, oo, rs)
        e_.record(stream)
    torch.cuda.synchronize()
    t = statistics.median(s_.elapsed_time(e_) for s_, e_ in ev) / 1e3
    st, cnt = G.decode_results(rs, k)
    ooff = oo.cpu().numpy()
    err = np.zeros(k, dtype=bool)
    err[list(b.errors)] = True
    assert np.all(st[~err] == 0) and np.array_equal(cnt[~err], np.diff(ooff)[~err]), "batch results"
    assert np.all((st[err] >= 1) & (st[err] <= 6)), "batch error kinds"
    assert np.array_equal(cnt[err], np.array([b.errors[i] for i in np.nonzero(err)[0]])), "batch error offsets"
    # the same strings, one asynchronous single-buffer call each
    res1 = torch.zeros((k, 2), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(k):
        a, e = int(b.offsets[i]), int(b.offsets[i + 1])
        G.convert_utf8_to_utf16le_async(d[a:e], out[int(ooff[i]):], res1[i], out_cap=int(ooff[i + 1] - ooff[i]))
    torch.cuda.synchronize()
    tloop = time.perf_counter() - t0
    # one plain single-buffer call over the same concatenated bytes (the
    # strings' boundaries ignored): the rate the batched call is compared with
    o1 = torch.empty(b.data.size, dtype=torch.int16, device=dev)
    r1 = G.result_tensor(device=dev)
    for _ in range(3):
        G.convert_utf8_to_utf16le_async(d, o1, r1)
    ev1 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
    for s_, e_ in ev1:
        s_.record(stream)
        G.convert_utf8_to_utf16le_async(d, o1, r1)
        e_.record(stream)
    torch.cuda.synchronize()
    t1 = statistics.median(s_.elapsed_time(e_) for s_, e_ in ev1) / 1e3
    del o1
    alg = b.data.size + 2 * total
    aux["batch100k_single_buffer_call_ms"] = round(t1 * 1e3, 3)
    aux["batch100k_time_vs_single_buffer"] = round(t / t1, 3)
    aux["batch100k_workload"] = (f"{k} UTF-8 strings, {b.data.size} bytes, log-normal lengths (median 256 B, "
                                 "sigma 1.5, 16 B..1 MiB), one script mix each, 1% with one error")
    aux["batch100k_call_ms"] = round(t * 1e3, 3)
    aux["batch100k_input_GBps"] = round(b.data.size / t / 1e9, 1)
    aux["batch100k_strings_per_s"] = round(k / t, 0)
    aux["batch100k_roofline_frac"] = round(alg / t / 1e9 / HBM_PEAK_GBS, 3)
    aux["batch100k_single_calls_ms"] = round(tloop * 1e3, 1)
    aux["batch100k_speedup_vs_single_calls"] = round(tloop / t, 1)


def serve_leg(reqs, small, aux):
    """The serving workload: open-loop Poisson arrivals at 50 000 requests/s,
    log-normal sizes (median 32 KiB, sigma ln(2^18)/6, 64 B..16 MiB), 50/50
    directions, 0.5% invalid; replayed in wall-clock time, then all at once
    (saturation); then both again with the tuner's geometry and schedule
    tables for the batched calls (tuned on the 1 MiB mixed-script text, four
    concurrent calls per timed round)."""
    from paper_2111_08692_amd.serve import Server
    import torch
    import paper_2111_08692_amd as G
    srv = Server(reqs, nstreams=4)
    srv.prewarm()             # every stream's workspace at its final size
    srv.run(time_scale=0.0)   # warm-up (allocator)
    # the same bytes as two plain single-buffer calls (each direction's
    # payloads back to back, request boundaries ignored): the rate the
    # served throughput is compared with
    o16 = torch.empty(srv.d8.numel(), dtype=torch.int16, device=srv.dev)
    o8 = torch.empty(3 * srv.d16.numel(), dtype=torch.uint8, device=srv.dev)
    rr = G.result_tensor(device=srv.dev)
    times = []
    for rep in range(4):
        torch.cuda.synchronize()
        t = time.perf_counter()
        G.convert_utf8_to_utf16le_async(srv.d8, o16, rr)
        G.convert_utf16le_to_utf8_async(srv.d16, o8, rr)
        torch.cuda.synchronize()
        if rep:
            times.append(time.perf_counter() - t)
    aux["serve_single_buffer_GBps"] = round(int(reqs.size.sum()) / min(times) / 1e9, 1)
    del o16, o8
    for tag, scale in (("50k_rps", 1.0), ("burst", 0.0)):
        res = srv.run(time_scale=scale)
        assert np.all(res.status[~reqs.invalid] == 0), "valid request failed"
        aux[f"serve_{tag}_p50_us"] = round(res.percentile_us(50), 1)
        aux[f"serve_{tag}_p99_us"] = round(res.percentile_us(99), 1)
        aux[f"serve_{tag}_GBps"] = round(res.gbps, 2)
        aux[f"serve_{tag}_launches"] = res.launches
    aux["serve_burst_vs_single_buffer"] = round(aux["serve_burst_GBps"] / aux["serve_single_buffer_GBps"], 3)
    # served outputs against single-buffer calls on the same payloads: a
    # seeded sample and the largest requests, from an extra all-at-once run
    # that copies each launch's output as it completes
    res = srv.run(time_scale=0.0, collect=True)
    rng = np.random.default_rng(604)
    ids = set(rng.choice(reqs.arrival.size, size=300, replace=False).tolist())
    ids |= set(np.argsort(reqs.size)[-20:].tolist())
    for rid in sorted(ids):
        kind = int(reqs.kind[rid])
        if kind == 0:
            j = int(np.searchsorted(reqs.ids8, rid))
            p = srv.d8[int(reqs.off8[j]):int(reqs.off8[j + 1])]
            st, cnt, out = G.convert_utf8_to_utf16le(p)
        else:
            j = int(np.searchsorted(reqs.ids16, rid))
            p = srv.d16[int(reqs.off16[j]):int(reqs.off16[j + 1])]
            st, cnt, out = G.convert_utf16le_to_utf8(p)
        assert (int(res.status[rid]), int(res.count[rid])) == (st, cnt), ("served result", rid)
        if st == 0:
            alone = out[:cnt].cpu().numpy()
            alone = alone.view(np.uint16) if kind == 0 else alone
            assert np.array_equal(srv.output_of(res, rid), alone), ("served output", rid)
    aux["serve_checked_requests"] = len(ids)
    aux["serve_workload"] = (f"{reqs.arrival.size} requests, {int(reqs.size.sum())} bytes, Poisson 50k/s "
                             "(open loop), log-normal sizes median 32 KiB sigma 2.08 in 64 B..16 MiB, 50/50 "
                             "directions, 0.5% invalid; each direction batched per pass, 4 streams, one output arena "
                             "sized from free HBM (8 GiB budget), every stream's workspace pre-sized before timing")
    # the same, with the batched calls' geometry and scan schedule tuned on
    # mixed-script text, four calls at a time on four streams as the server
    # runs them
    from paper_2111_08692_amd import tune
    try:
        tune.tune(small.data, ops=("convert_utf8_to_utf16le_batch", "convert_utf16le_to_utf8_batch"),
                  sizes=(1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22, 1 << 24), min_ms=1.0, reps=3,
                  string_bytes=32768, concurrency=4)
        srv.prewarm()
        srv.run(time_scale=0.0)
        res = srv.run(time_scale=1.0)
        assert np.all(res.status[~reqs.invalid] == 0), "valid request failed"
        aux["serve_50k_rps_tuned_p50_us"] = round(res.percentile_us(50), 1)
        aux["serve_50k_rps_tuned_p99_us"] = round(res.percentile_us(99), 1)
        res = srv.run(time_scale=0.0)
        assert np.all(res.status[~reqs.invalid] == 0), "valid request failed"
        aux["serve_burst_tuned_GBps"] = round(res.gbps, 2)
    finally:
        tune.reset()


def tune_leg(small, aux):
    """The tuner on the 1 MiB mixed-script text, at four input sizes: the
    (geometry, scan schedule) pair it picks, and its speed-up over geometry 0
    in block order and over the library's shipped table.  The result is not
    installed (the other legs run the shipped table)."""
    from paper_2111_08692_amd import tune
    t0 = time.time()
    res = tune.tune(small.data, ops=("convert_utf8_to_utf16le", "convert_utf16le_to_utf8",
                                     "convert_utf8_to_utf16le_batch", "convert_utf16le_to_utf8_batch"),
                    sizes=(1 << 16, 1 << 20, 1 << 24, 1 << 28), min_ms=2.0, reps=3, install=False)
    names = res["candidates"]   # "<geometry>/<schedule>", index 0 = geometry 0 in block order
    ops = {}
    for op, rows in res["measured"].items():
        ops[op] = {str(r["bytes"]): {"choice": r["choice"], "shipped": r["before"], "g0_us": r["us"][0],
                                     "speedup": round(r["us"][0] / r["us"][names.index(r["choice"])], 3),
                                     "speedup_vs_shipped": round(r["us"][names.index(r["before"])]
                                                                 / r["us"][names.index(r["choice"])], 3)}
                   for r in rows}
    aux["autotune"] = {"sample": "1 MiB mixed-script text, repeated; batched calls in strings of about 4 KiB",
                       "candidates": names, "seconds": round(time.time() - t0, 1), "ops": ops}


def host_leg(bufs, aux):
    """Host-resident input and output: one 1 GiB buffer per direction (CJK
    mix) through the chunked, pipelined host path (64 MiB chunks, 3
    streams).  Bounded by PCIe and host copies, reported apart from the HBM
    roofline, beside plain pinned copies over the same link."""
    import torch
    from paper_2111_08692_amd.host_pipeline import HostPipeline
    # the link alone: 1 GiB pinned host -> device and device -> pinned host
    n = 1 << 30
    hbuf = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    dbuf = torch.empty(n, dtype=torch.uint8, device="cuda")
    rate = {}
    for name, dst, src in (("h2d", dbuf, hbuf), ("d2h", hbuf, dbuf)):
        best = None
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            dst.copy_(src, non_blocking=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            best = dt if best is None else min(best, dt)
        rate[name] = n / best / 1e9
        aux[f"host_pcie_{name}_GBps"] = round(rate[name], 2)
    del hbuf, dbuf
    p = HostPipeline(chunk_bytes=64 << 20, nstreams=3)
    for mix, enc, kind, b in bufs:
        if mix != "cjk" or kind != "valid":
            continue
        conv = p.convert_utf8_to_utf16le if enc == "utf-8" else p.convert_utf16le_to_utf8
        conv(b.data[: 3 * (64 << 20) // b.data.itemsize])   # warm-up: one chunk on each stream
        st, cnt, out = conv(b.data)
        assert st == 0
        d = "8to16" if enc == "utf-8" else "16to8"
        aux[f"host_pipeline_cjk_{d}_GBps"] = round(b.data.nbytes / p.last["seconds"] / 1e9, 2)
        aux[f"host_pipeline_cjk_{d}_pcie_bytes"] = int(b.data.nbytes + out.nbytes)
        # the least time the link allows: input up and output down, overlapped
        link_s = max(b.data.nbytes / (rate["h2d"] * 1e9), out.nbytes / (rate["d2h"] * 1e9))
        aux[f"host_pipeline_cjk_{d}_frac_of_link"] = round(link_s / p.last["seconds"], 3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size-mib", type=int, default=1024, help="bytes per buffer (MiB); the workload is 1024")
    ap.add_argument("--cpu-sample-mib", type=int, default=768)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-aux", action="store_true",
                    help="skip the validate-only / length-only / 1 MiB latency figures (for profiled runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer three times (a plain copy kernel of known size, "
                         "the reference for the FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--batch-only", action="store_true",
                    help="only run the batched 100 000-string leg, print its figures and exit (for profiled runs)")
    ap.add_argument("--serve-only", action="store_true",
                    help="only run the serving leg, print its figures and exit (for profiled runs)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus above 1 is not supported "
                                   "(the transcoder is a single-GPU path, see DESIGN.md for how it would shard)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        src = torch.full((n,), 65, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": n, "launches": 3}), flush=True)
        return

    if args.batch_only:
        import torch
        import paper_2111_08692_amd as G
        G.load()
        aux = {}
        batch_leg(G, torch.device("cuda:0"), torch.cuda.current_stream(), aux)
        print(json.dumps(aux), flush=True)
        return

    if args.serve_only:
        from workloads import make_requests
        ex = ProcessPoolExecutor(max_workers=16, mp_context=mp.get_context("fork"))
        small = make_buffer("mix1m", 1 << 20, SEED_MIX1M)
        reqs = make_requests(SERVE_REQUESTS, executor=ex)
        ex.shutdown()
        import paper_2111_08692_amd as G
        G.load()
        aux = {}
        serve_leg(reqs, small, aux)
        print(json.dumps(aux), flush=True)
        reap_children()
        return

    size = args.size_mib << 20
    bufs, small, reqs = generate(size, serve=not args.no_aux)

    import torch
    import paper_2111_08692_amd as G

    assert torch.cuda.is_available(), "no GPU"
    G.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    # device-resident inputs
    dbufs = []
    for mix, enc, kind, b in bufs:
        host = torch.from_numpy(b.data.view(np.uint8) if enc == "utf-8" else b.data.view(np.int16))
        dbufs.append(host.to(dev))
    torch.cuda.synchronize()
    out16 = torch.empty(size, dtype=torch.int16, device=dev)          # >= n words for 8->16
    out8 = torch.empty(3 * (size // 2), dtype=torch.uint8, device=dev)  # >= 3m bytes for 16->8
    res = torch.zeros((len(bufs), 2), dtype=torch.int64, device=dev)
    lens = torch.zeros(len(bufs), dtype=torch.int64, device=dev)

    # output sizes (length queries) for the algorithmic byte counts
    for i, ((mix, enc, kind, b), d) in enumerate(zip(bufs, dbufs)):
        if enc == "utf-8":
            G.utf16_length_from_utf8_async(d, lens[i])
        else:
            G.utf8_length_from_utf16le_async(d, lens[i])
    out_units = lens.cpu().tolist()

    def enqueue(i, d, enc):
        if enc == "utf-8":
            rc = G.convert_utf8_to_utf16le_async(d, out16, res[i])
        else:
            rc = G.convert_utf16le_to_utf8_async(d, out8, res[i])
        assert rc == 0, rc

    def step(events=None):
        for i, ((mix, enc, kind, b), d) in enumerate(zip(bufs, dbufs)):
            if events is not None:
                events[i][0].record(stream)
            enqueue(i, d, enc)
            if events is not None:
                events[i][1].record(stream)
        return res.cpu()

    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    all_events = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in bufs] for _ in range(args.steps)]
    log("timed steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = step(all_events[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # results must match what the generator knows
    results = r.tolist()
    for (mix, enc, kind, b), (st, cnt), units in zip(bufs, results, out_units):
        st &= 0xFFFFFFFF
        if kind == "valid":
            assert st == 0 and cnt == units, (mix, enc, st, cnt, units)
        else:
            assert st in ((1, 2, 3, 4, 5, 6) if enc == "utf-8" else (7, 8)) and cnt == b.first_error, \
                (mix, enc, st, cnt, b.first_error)

    in_bytes = sum(int(b.data.nbytes) for _, _, _, b in bufs)
    value = in_bytes * args.steps / elapsed / 1e9

    # per-launch kernel durations
    dur = np.array([[s.elapsed_time(e) for s, e in row] for row in all_events]) / 1e3   # seconds
    per = {}
    kern_time = {"utf8_tile_kernel<convert>": 0.0, "utf16_tile_kernel<convert>": 0.0}
    kern_bytes = {"utf8_tile_kernel<convert>": 0, "utf16_tile_kernel<convert>": 0}
    for i, (mix, enc, kind, b) in enumerate(bufs):
        t = float(np.median(dur[:, i]))
        nin = int(b.data.nbytes)
        alg = nin + (2 * out_units[i] if enc == "utf-8" else out_units[i])
        name = "utf8_tile_kernel<convert>" if enc == "utf-8" else "utf16_tile_kernel<convert>"
        kern_time[name] += float(dur[:, i].sum())
        kern_bytes[name] += alg * args.steps
        key = f"{mix}/{'8to16' if enc == 'utf-8' else '16to8'}/{kind}"
        per[key] = {"input_GBps": round(nin / t / 1e9, 1), "hbm_GBps": round(alg / t / 1e9, 1),
                    "roofline_frac": round(alg / t / 1e9 / HBM_PEAK_GBS, 3), "ms": round(t * 1e3, 4),
                    "input_bytes": nin, "output_units": int(out_units[i])}
    dom = max(kern_time, key=kern_time.get)
    achieved = kern_bytes[dom] / kern_time[dom] / 1e9
    launches = args.steps * sum(1 for _, enc, _, _ in bufs if (enc == "utf-8") == dom.startswith("utf8"))

    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        with open(tpath) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == kernel_hash() and dom in tr.get("kernels", {}):
            traffic = tr["kernels"][dom]

    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom, "launches": launches,
                "algorithmic_bytes_per_launch": int(kern_bytes[dom] / launches),
                "avg_launch_ms": round(kern_time[dom] / launches * 1e3, 4)}

    # auxiliary kernels: validate-only and length-only on the valid buffers
    aux = None if args.no_aux else {}
    for name, fn in (() if args.no_aux else (("validate", None), ("length", None))):
        tt, nb = 0.0, 0
        for i, ((mix, enc, kind, b), d) in enumerate(zip(bufs, dbufs)):
            if kind != "valid":
                continue
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
            for s_, e_ in ev:
                s_.record(stream)
                if name == "validate":
                    (G.validate_utf8_async if enc == "utf-8" else G.validate_utf16le_async)(d, res[i])
                else:
                    (G.utf16_length_from_utf8_async if enc == "utf-8" else G.utf8_length_from_utf16le_async)(
                        d, lens[i])
                e_.record(stream)
            torch.cuda.synchronize()
            tt += statistics.median(s_.elapsed_time(e_) for s_, e_ in ev) / 1e3
            nb += int(b.data.nbytes)
        aux[f"{name}_only_input_GBps"] = round(nb / tt / 1e9, 1)
        aux[f"{name}_only_roofline_frac"] = round(nb / tt / 1e9 / HBM_PEAK_GBS, 3)

    # the 1 MiB single buffer: latency of one synchronous call
    if not args.no_aux:
        one_mib_latency(G, small, dev, stream, res, aux)
        copy_reference(dev, stream, aux)
        log("batched strings")
        batch_leg(G, dev, stream, aux)
        log("serving")
        serve_leg(reqs, small, aux)
        log("host-resident pipeline")
        host_leg(bufs, aux)
        log("geometry tuner")
        tune_leg(small, aux)

    cpu = None if args.no_cpu_baseline else cpu_baseline(bufs, args.cpu_sample_mib << 20)

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"five {args.size_mib} MiB script-mix buffers (ascii, latin, cyrillic, cjk, emoji) "
                               "plus invalid variants (error rate 1e-6), UTF-8->UTF-16LE and UTF-16LE->UTF-8, "
                               "validating",
                   "buffers_per_step": len(bufs), "input_bytes_per_step": in_bytes,
                   "buffer_bytes": size,
                   "tile_geometry": "shipped table: 8 waves x 4 rows (32 KiB tiles) at 1 GiB, both directions",
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {"per_buffer": per, "aux": aux, "kernel_hash": kernel_hash(),
                   "device": torch.cuda.get_device_name(0), "host_cores": os.cpu_count(),
                   "host_cores_usable": len(os.sched_getaffinity(0)), "cpu_model": cpu_model()},
    }
    print(json.dumps(line), flush=True)
    reap_children()


def reap_children():
    """Wait for (and report) any child process still alive at the end, so
    that the benchmark leaves none behind."""
    try:
        import psutil
    except ImportError:
        return
    kids = psutil.Process().children(recursive=True)
    if kids:
        log(f"{len(kids)} child process(es) left at the end: {[k.pid for k in kids]}; stopping them")
        for k in kids:
            try:
                k.terminate()
            except psutil.Error:
                pass
        psutil.wait_procs(kids, timeout=5)


if __name__ == "__main__":
    main()
