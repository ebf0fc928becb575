#!/usr/bin/env python3
"""Decompressed GB/s of the Gompresso/Bit decoder on one MI355X.

Headline workload (the plain single-stream configuration; `value`): 256 MiB
of seeded Zipf text, 1 MiB blocks each cut into 16 KiB sub-blocks (64 per
block), 32 KiB window, matches 3..258, code lengths <= 12.  The same data is
compressed twice, as an ordinary LZ77 stream (resolved by Multi-Round
Resolution) and as a Dependency-Elimination stream (resolved in one pass).
One step decodes both streams, each with one launch of the decoder (one
workgroup per block); inputs and outputs stay resident in HBM for the whole
timed region.

Beside it, on the same GPU and in the same run:
* batched: 4096 independent blocks of 4 KiB-4 MiB (half text, half CSV-like,
  ordinary or DE by a coin) in one graph-captured persistent launch, with the
  sub-block size picked by recompressing a sample and the launch shape by the
  library's autotuner, against the plain launch of the same blocks;
* serving: Poisson arrivals of requests of 64 KiB-64 MiB at 10-90 % of the
  batched peak through the library's request loop (64 GiB budget), with
  p50/p99 latency and admission wait per load level.

The CPU oracle's compressor generates the compressed inputs and its decoder,
run block-parallel over the host cores, is the CPU baseline.  Every decoded
byte is checked against the original data.

Prints one JSON line (see the field descriptions in the design doc).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "decompressed GB/s on 1 MI355X (MRR vs DE, % of HBM peak); p50/p99 request latency"
HBM_PEAK_GBPS = 8000.0
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1606_00519_amd", "csrc", f) for f in ("inflate.hip", "inflate.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "inflate_traffic_zipf256.json")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def params(de: int):
    import oracle
    return oracle.CompressParams(block_size=1 << 20, window=32768, max_match=258, lmax=12, sub_target_raw=16384,
                                 de=de, group=64)


# ----------------------------------------------------------------------------- oracle leg
def oracle_leg(size: int, threads: int, cpu_seconds: float):
    """Input generation with the oracle's compressor, and the oracle decoder
    timed block-parallel on the host cores (the paper's CPU method: a common
    queue of blocks; each thread takes the next block when it finishes)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    import synth
    t0 = time.time()
    data = synth.zipf_text(size, threads=threads).tobytes()
    log(f"generated {size} bytes of Zipf text in {time.time() - t0:.1f}s")
    streams = {}
    for mode, de in (("mrr", 0), ("de", 1)):
        t0 = time.time()
        streams[mode] = oracle.compress(data, params(de), threads=threads)
        log(f"compressed ({mode}) to {len(streams[mode])} bytes (ratio {size / len(streams[mode]):.3f}) "
            f"in {time.time() - t0:.1f}s")
    baseline = None
    if cpu_seconds > 0:
        baseline = cpu_baseline(streams, size, threads, cpu_seconds)
    return data, streams, baseline


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(streams: dict, size: int, threads: int, cpu_seconds: float) -> dict:
    """The oracle decoder (plain C, one block per call) on the host cores, on
    the headline data: all-core block-parallel (the paper's CPU method: a
    shared queue of blocks, each thread takes the next block when it
    finishes) over both streams, and single-threaded over a sample of blocks;
    median of 5 passes each, the sample sized to about cpu_seconds of CPU work."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    blocks = [blk for m in ("mrr", "de") for blk, _ in oracle.stream_blocks(streams[m])[0]]
    raw_all = 2 * size

    def one(b):
        rc, out = oracle.decompress_block(b)
        assert rc == 0
        return len(out)

    # a first pass sizes the sample
    t0 = time.perf_counter()
    n_probe = min(8, len(blocks))
    probe_raw = sum(one(b) for b in blocks[:n_probe])
    per_byte = (time.perf_counter() - t0) / probe_raw          # one core's seconds per byte
    # all-core: the whole of both streams per pass if that fits the budget, else a prefix
    share = min(1.0, cpu_seconds / 2 / 5 / (per_byte * raw_all))
    sample = blocks[:max(threads, int(len(blocks) * share))]
    times = []
    with ThreadPoolExecutor(threads) as ex:
        for _ in range(5):
            t0 = time.perf_counter()
            sample_raw = sum(ex.map(one, sample))
            times.append(time.perf_counter() - t0)
    allcore = sample_raw / float(np.median(times)) / 1e9
    # single thread: blocks of both modes, alternately
    n1 = max(2, int(cpu_seconds / 2 / 5 / (per_byte * (1 << 20))))
    half = len(blocks) // 2
    single = [blocks[i // 2 + (half if i % 2 else 0)] for i in range(min(n1, len(blocks)))]
    times1 = []
    for _ in range(5):
        t0 = time.perf_counter()
        raw1 = sum(one(b) for b in single)
        times1.append(time.perf_counter() - t0)
    st = raw1 / float(np.median(times1)) / 1e9
    res = {"value": round(allcore, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "single_thread_GBps": round(st, 4), "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "sample": f"all-core: {len(sample)} blocks of the headline MRR and DE streams "
                     f"({sample_raw >> 20} MiB decompressed per pass), block-parallel over {threads} threads "
                     f"with a shared block queue, median of 5 passes; single thread: {len(single)} blocks "
                     f"({raw1 >> 20} MiB) of both streams, median of 5 passes"}
    log(f"cpu baseline: {res['value']} GB/s on {threads} threads, {res['single_thread_GBps']} GB/s on one "
        f"({res['cpu_model']})")
    return res


def launch_shape(waves: int) -> str:
    if waves == 7:
        return ("one workgroup per block, 8 wavefronts: 7 decoders + fetcher (Huffman phase); "
                "6 resolvers + fetcher + flusher (LZ77 phase)")
    return f"one workgroup per block: {waves} decoder/resolver wavefront(s) + fetcher + flusher"


# ----------------------------------------------------------------------------- GPU leg
class StreamRun:
    """One compressed stream resident on the device, decoded as one batch (one
    job per block, the output contiguous): the launch bench.py times.  A second
    job table over the same buffers records per-block phase stamps, per-group
    rounds and per-block counters (GMP_FLAG_STATS) in an untimed run.  The job
    table is set up from the block headers by the library's own parser
    (gmp_block_info_parse)."""

    def __init__(self, ctx, s: bytes, raw: int):
        import struct

        import torch

        import paper_1606_00519_amd as gmp
        self.gmp = gmp
        nb, bs, total = gmp.stream_info(s)
        assert total == raw
        offs = struct.unpack_from(f"<{nb + 1}Q", s, 32)
        self.d_in = torch.frombuffer(bytearray(s), dtype=torch.uint8).cuda()
        self.out = torch.empty(raw, dtype=torch.uint8, device="cuda")
        self.status = torch.full((max(nb, 1),), 99, dtype=torch.int32, device="cuda")
        infos = [gmp.block_info(s[offs[b]:offs[b + 1]]) for b in range(nb)]
        self.n_groups = [(i["n_seq"] + 63) // 64 for i in infos]
        goff = np.concatenate([[0], np.cumsum(self.n_groups)]).astype(np.int64)
        self.goff = goff
        self.rounds = torch.zeros((max(int(goff[-1]), 1),), dtype=torch.uint8, device="cuda")
        self.times = torch.zeros((max(nb, 1), 4), dtype=torch.int64, device="cuda")
        self.stats = torch.zeros((max(nb, 1), gmp.STATS_WORDS), dtype=torch.int32, device="cuda")
        jobs, sjobs = [], []
        for b, i in enumerate(infos):
            args = (self.d_in.data_ptr() + offs[b], offs[b + 1] - offs[b], self.out.data_ptr() + b * bs,
                    i["raw_len"], i["n_seq"], i["n_lit"])
            jobs.append(gmp.Job(*args, None, None, None, i["format"]))
            sjobs.append(gmp.Job(*args, self.rounds.data_ptr() + int(goff[b]), self.times.data_ptr() + 32 * b,
                                 self.stats.data_ptr() + 4 * gmp.STATS_WORDS * b, i["format"]))
        self.batch = ctx.batch_create(jobs, self.status)
        self.sbatch = ctx.batch_create(sjobs, self.status)
        self.blocks, self.comp, self.raw = nb, len(s), raw

    def run(self, flags: int, waves: int, rounds_per_launch: int = 0) -> None:
        self.batch.run(flags, waves=waves, persistent=False, rounds_per_launch=rounds_per_launch)

    def check(self, data: bytes, what: str) -> None:
        st = self.status.cpu().numpy()
        if not np.all(st[:self.blocks] == 0):
            raise RuntimeError(f"{what}: device status {st[st != 0][:8]}")
        if not np.array_equal(self.out.cpu().numpy(), np.frombuffer(data, np.uint8)):
            raise RuntimeError(f"{what}: GPU output differs from the original data")

    def stats_run(self, flags: int, waves: int) -> dict:
        """Untimed run with GMP_FLAG_STATS: mean phase times (device clock),
        the rounds histogram over groups with back-references, and the
        paper's bytes per round (bytes copied in round r over all groups,
        divided by the number of groups)."""
        import torch
        self.sbatch.run(flags | self.gmp.FLAG_STATS, waves=waves, persistent=False)
        torch.cuda.synchronize()
        t = self.times.cpu().numpy().astype(np.int64)[:self.blocks]
        d = np.diff(t, axis=1) * 10 / 1e3  # microseconds: tables, sub-block decode, resolution
        span = (t[:, 3].max() - t[:, 0].min()) * 10 / 1e3
        r = self.rounds.cpu().numpy()[:int(self.goff[-1])] & 0x7F
        c = self.stats.cpu().numpy().astype(np.int64)[:self.blocks]
        groups = int(len(r))
        hist = np.bincount(r, minlength=65)
        rb = c[:, self.gmp.STAT_ROUND_BYTES:self.gmp.STAT_ROUND_BYTES + 64].sum(axis=0)
        last = int(np.max(np.nonzero(rb)[0])) + 1 if rb.any() else 0
        paths = np.bincount(c[:, self.gmp.STAT_A2_PATH], minlength=4)
        rej = {}
        for v in c[:, self.gmp.STAT_SEG_REJECT]:
            if v:
                rej[int(v)] = rej.get(int(v), 0) + 1
        return {"phases": {"tables_us": round(float(d[:, 0].mean()), 2),
                           "huffman_us": round(float(d[:, 1].mean()), 2),
                           "huffman_us_max": round(float(d[:, 1].max()), 2),
                           "lz_us": round(float(d[:, 2].mean()), 2), "lz_us_max": round(float(d[:, 2].max()), 2),
                           "launch_span_us": round(float(span), 2)},
                "groups": groups,
                "rounds_mean": round(float(r[r > 0].mean()), 3) if (r > 0).any() else 0.0,
                "rounds_hist": {int(k): int(v) for k, v in enumerate(hist) if v and k > 0},
                "groups_without_backrefs": int(hist[0]),
                "round_bytes": [int(x) for x in rb[:last]],
                "bytes_per_round": [round(float(x) / max(groups, 1), 3) for x in rb[:last]],
                "a2_paths": {"segmented": int(paths[1]), "per_sub_block": int(paths[2]), "byte_level": int(paths[3])},
                "segmented_rejections": rej,
                "segmented_further_attempts": int(c[:, self.gmp.STAT_SEG_RETRY].sum()),
                "repaired_lanes": int(c[:, self.gmp.STAT_REPAIRED].sum()),
                "split_groups": int(c[:, self.gmp.STAT_SPLIT].sum())}

    def close(self) -> None:
        self.batch.close()
        self.sbatch.close()


def time_modes(runs: dict, steps: int, warmup: int, waves: int) -> dict:
    """Each run alone: warm-up launches, then `steps` launches each bracketed
    by HIP events on the launch stream; mean and median kernel ms."""
    import torch
    stream = torch.cuda.current_stream()
    res = {}
    for name, (r, flags) in runs.items():
        for _ in range(warmup):
            r.run(flags, waves)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        for a, b in evs:
            a.record(stream)
            r.run(flags, waves)
            b.record(stream)
        torch.cuda.synchronize()
        ms = [a.elapsed_time(b) for a, b in evs]
        res[name] = {"mean": float(np.mean(ms)), "median": float(np.median(ms)), "min": float(np.min(ms))}
    return res


def mode_entry(raw: int, comp: int, ms: dict, stats: dict | None, copy_gbps: float | None) -> dict:
    t = ms["mean"] / 1e3
    alg = (raw + comp) / t / 1e9
    e = {"GBps": round(raw / t / 1e9, 3), "kernel_ms": round(ms["mean"], 4),
         "kernel_ms_median": round(ms["median"], 4), "kernel_ms_min": round(ms.get("min", ms["median"]), 4),
         "ratio": round(raw / comp, 4), "compressed_bytes": comp,
         "hbm_GBps": round(alg, 2), "hbm_frac": round(alg / HBM_PEAK_GBPS, 5)}
    if copy_gbps:
        e["copy_frac"] = round(alg / copy_gbps, 5)
    if stats:
        e.update(stats)
    return e


def copy_reference(size: int, steps: int) -> dict:
    """A plain device-to-device copy of `size` bytes (torch's copy kernel),
    timed like the decoder: the practical HBM bound the decoder's traffic is
    also reported against."""
    import torch
    src = torch.empty(size, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        dst.copy_(src)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in evs:
        a.record(stream)
        dst.copy_(src)
        b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.median([a.elapsed_time(b) for a, b in evs]))
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": size, "ms": round(ms, 4), "GBps": round(2 * size / (ms / 1e3) / 1e9, 2),
            "what": "torch device-to-device copy of the headline output size; GB/s counts bytes read + written"}


def gpu_leg(ctx, data: bytes, streams: dict, steps: int, warmup: int, waves: int):
    """The headline: one step decodes the MRR stream and then the DE stream of
    the same data, one launch each."""
    import torch

    import paper_1606_00519_amd as gmp
    size = len(data)
    runs = {m: (StreamRun(ctx, streams[m], size), gmp.MODE_MRR if m == "mrr" else gmp.MODE_DE)
            for m in ("mrr", "de")}
    stream = torch.cuda.current_stream()

    def step(evs=None):
        for mode, (r, flags) in runs.items():
            if evs is not None:
                evs[mode][0].record(stream)
            r.run(flags, waves)
            if evs is not None:
                evs[mode][1].record(stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev_list = [{m: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for m in runs} for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(ev_list[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = {m: {"mean": float(np.mean([e[m][0].elapsed_time(e[m][1]) for e in ev_list])),
                     "median": float(np.median([e[m][0].elapsed_time(e[m][1]) for e in ev_list])),
                     "min": float(np.min([e[m][0].elapsed_time(e[m][1]) for e in ev_list]))}
                 for m in runs}
    stats = {}
    for mode, (r, flags) in runs.items():
        r.check(data, mode)                      # what was timed
        stats[mode] = r.stats_run(flags, waves)  # untimed
        r.check(data, mode + " (stats run)")
    comp = {m: runs[m][0].comp for m in runs}
    n_blocks = runs["mrr"][0].blocks
    for r, _ in runs.values():
        r.close()
    return wall, kernel_ms, comp, n_blocks, stats


def side_leg(ctx, name: str, data: bytes, streams: dict, steps: int, warmup: int, waves: int,
             copy_gbps: float | None) -> dict:
    """Other configurations on the same GPU, each mode timed alone (`streams`:
    mode name -> (stream bytes, flags))."""
    size = len(data)
    runs = {m: (StreamRun(ctx, s, size), f) for m, (s, f) in streams.items()}
    ms = time_modes(runs, steps, warmup, waves)
    res = {}
    for m, (r, f) in runs.items():
        r.check(data, f"{name} {m}")
        st = r.stats_run(f, waves)
        r.check(data, f"{name} {m} (stats run)")
        res[m] = mode_entry(size, r.comp, ms[m], st, copy_gbps)
        r.close()
        log(f"{name} {m}: {res[m]['GBps']} GB/s ({res[m]['kernel_ms']} ms, ratio {res[m]['ratio']}, "
            f"{res[m]['rounds_mean']} rounds/group, phases {res[m]['phases']}, Huffman paths {res[m]['a2_paths']}, "
            f"rejections {res[m]['segmented_rejections']})")
    return res


def multilaunch_leg(ctx, data: bytes, stream: bytes, steps: int, warmup: int, waves: int) -> dict:
    """Multi-Round Resolution over several launches on the headline MRR
    stream: at most R rounds per group in the decoding launch, the pending
    back-references resolved by later launches (the paper's alternative MRR
    variant, section "Performance Impact of Nested back-references"), against
    every round in one launch."""
    import torch

    import paper_1606_00519_amd as gmp
    r = StreamRun(ctx, stream, len(data))
    stream_h = torch.cuda.current_stream()
    res = {}
    for R in (0, 16, 4, 1):
        for _ in range(warmup):
            r.run(gmp.MODE_MRR, waves, R)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        for a, b in evs:
            a.record(stream_h)
            r.run(gmp.MODE_MRR, waves, R)
            b.record(stream_h)
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        r.check(data, f"multi-launch R={R}")
        # back-references the decoding launch left to later launches
        r.sbatch.run(gmp.MODE_MRR | gmp.FLAG_STATS, waves=waves, persistent=False, rounds_per_launch=R)
        torch.cuda.synchronize()
        spilled = int(r.stats.cpu().numpy()[:r.blocks, gmp.STAT_SPILLED].astype(np.int64).sum())
        r.check(data, f"multi-launch R={R} (stats run)")
        launches = 1 if R == 0 else 1 + (64 + R - 1) // R
        res[f"R{R}" if R else "all_rounds"] = {"rounds_per_launch": R, "launches": launches, "ms": round(ms, 4),
                                               "GBps": round(len(data) / (ms / 1e3) / 1e9, 3),
                                               "spilled_backrefs": spilled}
        log(f"multi-launch R={R}: {res[f'R{R}' if R else 'all_rounds']}")
    r.close()
    return res


def compress_leg(ctx, data: bytes, cpu_sizes: dict, steps: int, warmup: int, waves: int) -> dict:
    """GPU compression of the headline text into byte-level blocks of 1 MiB
    (section "Parallel Compression"), ordinary and with Dependency
    Elimination: compressed GB/s (input bytes per second), ratio against the
    CPU compressor's, and the round trip through the GPU decoder; a sample of
    blocks also passes the CPU reference's format check."""
    import torch

    import oracle
    import paper_1606_00519_amd as gmp
    n = len(data)
    bs = 1 << 20
    nb = (n + bs - 1) // bs
    d_in = torch.frombuffer(bytearray(data), dtype=torch.uint8).cuda()
    cap = (gmp.compress_bound(bs) + 255) & ~255
    outs = torch.zeros(nb * cap, dtype=torch.uint8, device="cuda")
    lens = torch.zeros(nb, dtype=torch.int64, device="cuda")
    status = torch.full((nb,), 99, dtype=torch.int32, device="cuda")
    jobs = [gmp.CompressJob(d_in.data_ptr() + b * bs, min(bs, n - b * bs), outs.data_ptr() + b * cap, cap,
                            lens.data_ptr() + 8 * b, status.data_ptr() + 4 * b) for b in range(nb)]
    stream = torch.cuda.current_stream()
    res = {}
    for de in (0, 1):
        for _ in range(warmup):
            ctx.compress_batch(jobs, de=de)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        for a, b in evs:
            a.record(stream)
            ctx.compress_batch(jobs, de=de)
            b.record(stream)
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        if not np.all(status.cpu().numpy() == 0):
            raise RuntimeError("compress: a block failed")
        ln = lens.cpu().numpy().astype(np.int64)
        o = outs.cpu().numpy()
        blocks = [o[b * cap:b * cap + int(ln[b])].tobytes() for b in range(nb)]
        for b in (0, nb // 2, nb - 1):
            raw = data[b * bs:(b + 1) * bs]
            if oracle.validate_block(blocks[b]) != 0 or oracle.decompress_block(blocks[b]) != (0, raw):
                raise RuntimeError(f"compress: block {b} fails the CPU reference's check")
        s = oracle.assemble_stream(blocks, bs, n)
        r = StreamRun(ctx, s, n)
        r.run(gmp.MODE_AUTO, waves)
        torch.cuda.synchronize()
        r.check(data, f"compress de={de} round trip")
        r.close()
        comp = len(s)
        res["de" if de else "ordinary"] = {
            "ms": round(ms, 4), "GBps": round(n / (ms / 1e3) / 1e9, 3), "ratio": round(n / comp, 4),
            "cpu_compressor_ratio": round(n / cpu_sizes[de], 4),
            "hbm_GBps": round((n + comp) / (ms / 1e3) / 1e9, 2)}
        log(f"compress de={de}: {res['de' if de else 'ordinary']}")
    return res


def nesting_leg(ctx, steps: int, warmup: int, waves: int, mib: int = 64) -> dict:
    """Speed against back-reference nesting depth (section "Performance Impact
    of Nested back-references"): byte-level blocks of 1 MiB whose token
    streams hold k interleaved chains of 16-byte back-references, each copying
    the output of the one k sequences before it, so that every group of 64
    sequences takes 64/k rounds of Multi-Round Resolution by the paper's rule
    (ceil(64/k / 3) with sources moved through the group's own copies, the
    default); Sequential Copying of the same blocks beside them."""
    import oracle
    import synth
    import paper_1606_00519_amd as gmp
    res = {}
    for k in (64, 32, 16, 8, 4, 2, 1):
        n_seq = (1 << 20) // 17
        seqs, lits = synth.nesting_tokens(n_seq, k, str_len=16)
        # a record holds at most 255 literals: the initial literal run of
        # 1 + 17k bytes becomes literal-only records first (every group after
        # the first still holds 64 consecutive links of the chains)
        head, rest = divmod(int(seqs[0, 0]), 255)
        seqs = np.concatenate([np.tile(np.array([[255, 0, 0]], np.uint32), (head, 1)),
                               np.array([[rest, seqs[0, 1], seqs[0, 2]]], np.uint32), seqs[1:]])
        blk = oracle.encode_byte_block(seqs, lits, oracle.CompressParams(format=1))
        raw = len(lits) + int(seqs[:, 1].sum())
        rc, want = oracle.decompress_block(blk)
        assert rc == 0 and len(want) == raw
        # one stream of `mib` copies of the block (block size = its raw length)
        nb = max(1, (mib << 20) // raw)
        s = oracle.assemble_stream([blk] * nb, raw, raw * nb)
        data = want * nb
        runs = {"mrr": (StreamRun(ctx, s, len(data)), gmp.MODE_MRR),
                "mrr_plain": (StreamRun(ctx, s, len(data)), gmp.MODE_MRR | gmp.FLAG_PLAIN_MRR),
                "sc": (StreamRun(ctx, s, len(data)), gmp.MODE_SC)}
        ms = time_modes(runs, max(3, steps // 2), warmup, waves)
        e = {"depth": 64 // k, "blocks": nb, "raw_bytes": len(data)}
        for m, (r, f) in runs.items():
            r.check(data, f"nesting k={k} {m}")
            st = r.stats_run(f, waves)
            e[m] = {"GBps": round(len(data) / (ms[m]["mean"] / 1e3) / 1e9, 3), "kernel_ms": round(ms[m]["mean"], 4),
                    "rounds_mean": st["rounds_mean"], "lz_us": st["phases"]["lz_us"],
                    "bytes_per_round": st["bytes_per_round"][:4]}
            r.close()
        res[f"depth{64 // k}"] = e
        log(f"nesting depth {64 // k}: MRR {e['mrr']['GBps']} GB/s ({e['mrr']['rounds_mean']} rounds), "
            f"paper's rule {e['mrr_plain']['GBps']} GB/s ({e['mrr_plain']['rounds_mean']} rounds), "
            f"SC {e['sc']['GBps']} GB/s")
    return res


# ----------------------------------------------------------------------------- batched leg
def _compress_blocks(raws, subs, des, threads):
    """One oracle-compressed block per item (the item is the whole block)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    def one(k):
        p = oracle.CompressParams(block_size=max(len(raws[k]), 1), window=32768, max_match=258, lmax=12,
                                  sub_target_raw=subs[k], de=des[k], group=64)
        return oracle.compress_block(raws[k], p)

    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(one, range(len(raws))))


class _DeviceBatch:
    def __init__(self, ctx, blocks, raw_sizes):
        import torch

        import paper_1606_00519_amd as gmp
        offs, pos = [], 0
        for b in blocks:
            offs.append(pos)
            pos += (len(b) + 255) & ~255
        host = bytearray(max(pos, 16))
        for o, b in zip(offs, blocks):
            host[o:o + len(b)] = b
        self.d_in = torch.frombuffer(host, dtype=torch.uint8).cuda()
        self.o_offs = np.concatenate([[0], np.cumsum(raw_sizes)]).astype(np.int64)
        self.out = torch.empty(int(self.o_offs[-1]), dtype=torch.uint8, device="cuda")
        self.status = torch.full((len(blocks),), 99, dtype=torch.int32, device="cuda")
        jobs = []
        for k, b in enumerate(blocks):
            i = gmp.block_info(b)
            jobs.append(gmp.Job(self.d_in.data_ptr() + offs[k], len(b), self.out.data_ptr() + int(self.o_offs[k]),
                                i["raw_len"], i["n_seq"], i["n_lit"], None))
        self.batch = ctx.batch_create(jobs, self.status)
        self.comp = sum(len(b) for b in blocks)


def batched_leg(ctx, text: bytes, n_items: int, steps: int, warmup: int, threads: int):
    """Thousands of independent blocks of uneven sizes (text and CSV, ordinary
    and DE) in one graph-captured persistent launch: sub-block size chosen on
    a sample by recompressing it, launch shape by the library's autotuner;
    beside it the plain launch (one workgroup per block, one wavefront, no
    graph) of the same blocks."""
    import torch

    import paper_1606_00519_amd as gmp
    import synth
    t0 = time.time()
    csv = synth.csv_rows(1 << 30, threads=threads)
    txt = np.frombuffer(text, np.uint8)
    items = synth.batch_mix(n_items, text_corpus=len(txt), csv_corpus=len(csv))
    raws = [(txt if it["kind"] == "text" else csv)[it["off"]:it["off"] + it["size"]].tobytes() for it in items]
    des = [it["de"] for it in items]
    del csv
    total = sum(len(r) for r in raws)
    log(f"batched: {len(raws)} items, {total / 2**30:.2f} GiB raw, generated in {time.time() - t0:.1f}s")
    # sub-block size: recompress a sample at each candidate, autotune each
    n_s = min(384, len(raws))
    sub_res = {}
    for sub in (4096, 8192, 16384, 32768):
        blocks = _compress_blocks(raws[:n_s], [sub] * n_s, des[:n_s], threads)
        db = _DeviceBatch(ctx, blocks, [len(r) for r in raws[:n_s]])
        tun, ms = db.batch.autotune(gmp.MODE_AUTO, reps=3)
        sub_res[sub] = (ms, tun)
        db.batch.close()
        del db
        log(f"batched: sample sub-block {sub >> 10} KiB -> {ms:.3f} ms ({tun})")
    best_sub = min(sub_res, key=lambda k: sub_res[k][0])
    t0 = time.time()
    blocks = _compress_blocks(raws, [best_sub] * len(raws), des, threads)
    log(f"batched: compressed all items at {best_sub >> 10} KiB sub-blocks in {time.time() - t0:.1f}s")
    db = _DeviceBatch(ctx, blocks, [len(r) for r in raws])
    del blocks
    tun, tms = db.batch.autotune(gmp.MODE_AUTO, reps=3)
    db.batch.graph_create(gmp.MODE_AUTO, waves=tun["waves"], persistent=tun["persistent"],
                          workgroups=tun["workgroups"], rounds_per_launch=tun["rounds_per_launch"])
    stream = torch.cuda.current_stream()

    def timed(run):
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for a, b in evs:
            a.record(stream)
            run()
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in evs]))

    def check(what):
        st = db.status.cpu().numpy()
        if not np.all(st == 0):
            raise RuntimeError(f"batched ({what}): device status {st[st != 0][:8]}")
        got = db.out.cpu().numpy()
        for k, r in enumerate(raws):
            if got[db.o_offs[k]:db.o_offs[k + 1]].tobytes() != r:
                raise RuntimeError(f"batched ({what}): item {k} differs from its source bytes")

    graph_ms = timed(lambda: db.batch.graph_launch())
    check("graph")
    # the same launch shape without the graph and the device queue: one
    # workgroup per job at the tuned wavefront count, then at one wavefront
    db.out.zero_()
    same_ms = timed(lambda: db.batch.run(gmp.MODE_AUTO, waves=tun["waves"], persistent=False,
                                         rounds_per_launch=tun["rounds_per_launch"]))
    check("plain, tuned waves")
    db.out.zero_()
    plain_ms = timed(lambda: db.batch.run(gmp.MODE_AUTO, waves=1, persistent=False))
    check("plain")
    res = {"items": len(raws), "raw_bytes": total, "compressed_bytes": db.comp,
           "sub_block_kib": best_sub >> 10, "tuning": tun,
           "sample_ms_by_sub_block_kib": {k >> 10: round(v[0], 3) for k, v in sub_res.items()},
           "graph_ms": round(graph_ms, 3), "GBps": round(total / graph_ms / 1e6, 3),
           "plain_same_waves_ms": round(same_ms, 3), "plain_same_waves_GBps": round(total / same_ms / 1e6, 3),
           "plain_1wave_ms": round(plain_ms, 3), "plain_1wave_GBps": round(total / plain_ms / 1e6, 3)}
    db.batch.close()
    log(f"batched: graph {graph_ms:.2f} ms ({res['GBps']} GB/s), plain at {tun['waves']} waves {same_ms:.2f} ms, "
        f"plain at 1 wave {plain_ms:.2f} ms")
    return res


# ----------------------------------------------------------------------------- serving leg
def serve_leg(ctx, text: bytes, peak_gbps: float, n_pool: int, n_req: int, threads: int, waves: int,
              budget: int = 64 << 30, level_seconds: float = 5.0):
    """Poisson arrivals of requests (log-uniform 64 KiB-64 MiB, text or CSV,
    ordinary or DE) at offered loads of 10-90 % of the batched peak, admitted
    by the library's request loop within an HBM budget; the requests' buffers
    are resident on the device before the clock starts.  A request draws a
    pooled input; a pool entry whose previous copy is still in flight (or not
    yet checked) is not submitted again: the next free entry is taken.  Every
    completed request's output is compared on the device with its source
    bytes.  Reports achieved GB/s, p50/p99 latency (completion - arrival) and
    admission wait per load level."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    import oracle
    import paper_1606_00519_amd as gmp
    import synth
    t0 = time.time()
    csv = synth.csv_rows(1 << 30, threads=threads)
    txt = np.frombuffer(text, np.uint8)
    spec = synth.request_mix(n_pool, text_corpus=len(txt), csv_corpus=len(csv))
    raws = [(txt if r["kind"] == "text" else csv)[r["off"]:r["off"] + r["size"]].tobytes() for r in spec]
    del csv

    def comp(k):
        r = spec[k]
        p = (oracle.CompressParams(block_size=1 << 20, sub_target_raw=16384, de=r["de"]) if r["kind"] == "text"
             else oracle.CompressParams(block_size=2 << 20, sub_target_raw=32768, de=r["de"]))
        return oracle.compress(raws[k], p, threads=1)

    with ThreadPoolExecutor(threads) as ex:
        streams = list(ex.map(comp, range(n_pool)))
    log(f"serve: pool of {n_pool} requests ({sum(map(len, raws)) / 2**30:.2f} GiB raw) ready in "
        f"{time.time() - t0:.1f}s")
    pool = []
    for raw, s in zip(raws, streams):
        nb = gmp.stream_info(s)[0]
        pool.append({"d_in": torch.frombuffer(bytearray(s), dtype=torch.uint8).cuda(),
                     "h": np.frombuffer(s, np.uint8),   # host headers, passed without a copy
                     "ref": torch.frombuffer(bytearray(raw), dtype=torch.uint8).cuda(),
                     "out": torch.empty(len(raw), dtype=torch.uint8, device="cuda"),
                     "status": torch.full((nb,), 99, dtype=torch.int32, device="cuda"),
                     "busy": False, "checked": None})
    torch.cuda.synchronize()
    mean_u = float(np.mean([len(r) for r in raws]))
    srv = gmp.Server(ctx, budget_bytes=budget, slots=4, waves=waves)
    rng = np.random.default_rng(synth.SERVE_SEED + 100)
    stream = torch.cuda.current_stream()
    levels = []
    bad = []          # device flags: an output that differs from its source, or a block status != 0
    tag_entry = {}

    def completed(cs):
        for c in cs:
            e = pool[tag_entry.pop(c["tag"])]
            if c["status"] != 0:
                raise RuntimeError(f"serve: request {c['tag']} ended with status {c['status']}")
            bad.append(torch.ne(e["out"], e["ref"]).any() | torch.ne(e["status"], 0).any())
            ev = torch.cuda.Event()
            ev.record(stream)
            e["checked"] = ev
            e["busy"] = False
        return cs

    def free_entry(k):
        for j in range(n_pool):
            e = pool[(k + j) % n_pool]
            if not e["busy"] and (e["checked"] is None or e["checked"].query()):
                return (k + j) % n_pool
        return None

    for rho in [round(0.1 * i, 1) for i in range(1, 10)]:
        lam = rho * peak_gbps * 1e9 / mean_u
        n = int(min(n_req, max(200, level_seconds * lam)))
        arr = np.cumsum(rng.exponential(1.0 / lam, n))
        which = rng.integers(0, n_pool, n)
        done = []
        late = 0
        t_start = time.perf_counter()
        for i in range(n):
            while time.perf_counter() - t_start < arr[i]:
                pass
            k = free_entry(int(which[i]))
            while k is None:
                done += completed(srv.poll(4096))
                k = free_entry(int(which[i]))
            late += (time.perf_counter() - t_start - arr[i]) > 1e-3
            e = pool[k]
            e["busy"] = True
            tag_entry[i] = k
            srv.submit(e["d_in"], e["h"], e["out"], e["status"], gmp.MODE_AUTO, tag=i)
            if i % 16 == 0:
                done += completed(srv.poll(4096))
        srv.drain(600000)
        done += completed(srv.poll(1 << 16))
        if len(done) != n:
            raise RuntimeError(f"serve: {len(done)} of {n} requests completed")
        lat = np.array([(c["t_done_ns"] - c["t_submit_ns"]) / 1e6 for c in done])
        wait = np.array([(c["t_admit_ns"] - c["t_submit_ns"]) / 1e6 for c in done])
        span = (max(c["t_done_ns"] for c in done) - min(c["t_submit_ns"] for c in done)) / 1e9
        byt = sum(c["bytes"] for c in done)
        lv = {"rho": rho, "offered_GBps": round(lam * mean_u / 1e9, 3), "achieved_GBps": round(byt / span / 1e9, 3),
              "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
              "admit_wait_p50_ms": round(float(np.percentile(wait, 50)), 3),
              "admit_wait_p99_ms": round(float(np.percentile(wait, 99)), 3), "requests": n,
              "submitted_late_1ms": int(late)}
        levels.append(lv)
        log(f"serve: rho {rho}: {lv}")
    info = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    n_bad = int(torch.stack(bad).sum().item()) if bad else 0
    if n_bad:
        raise RuntimeError(f"serve: {n_bad} completed requests differ from their source bytes")
    return {"pool_requests": n_pool, "mean_request_bytes": int(mean_u), "budget_bytes": budget, "slots": 4,
            "launches": info["launches"], "peak_in_flight_bytes": info["peak_in_flight_bytes"],
            "peak_concurrent_launches": info["peak_slots"], "checked_requests": len(bad),
            "requests_per_level": f"min({n_req}, {level_seconds:g} s of arrivals)",
            "reference_peak_GBps": round(peak_gbps, 3), "levels": levels}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size-mib", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="CPU work for the oracle baseline, both of its legs together (0 = skip)")
    ap.add_argument("--threads", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--waves", type=int, default=7, choices=(1, 2, 4, 7),
                    help="decoder wavefronts per block (phase A); with 7, four of them resolve in phase B")
    ap.add_argument("--legs", default="paper_rule,byte,compress,csv,nesting,multilaunch,batched,serve",
                    help="side legs beside the headline (comma-separated; '' = headline only)")
    ap.add_argument("--csv-mib", type=int, default=1024, help="size of the low-entropy CSV configuration")
    ap.add_argument("--batch-items", type=int, default=4096, help="batched form: items")
    ap.add_argument("--serve-requests", type=int, default=4000, help="serving: requests per load level (at most)")
    ap.add_argument("--serve-pool", type=int, default=192, help="serving: distinct device-resident requests")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}); "
              f"blocks are independent, see DESIGN.md for how the decoder would shard.", file=sys.stderr)
        return 2
    legs = {x for x in args.legs.split(",") if x}
    size = args.size_mib << 20
    data, streams, baseline = oracle_leg(size, args.threads, args.cpu_seconds)
    import paper_1606_00519_amd as gmp
    import oracle
    import synth
    ctx = gmp.Context(0)
    copy_ref = copy_reference(size, args.steps)
    log(f"copy reference: {copy_ref['GBps']} GB/s")
    wall, kernel_ms, comp, n_blocks, stats = gpu_leg(ctx, data, streams, args.steps, args.warmup, args.waves)
    raw_step = 2 * size
    ms_per_step = wall / args.steps * 1e3
    value = raw_step / (wall / args.steps) / 1e9
    modes = {m: mode_entry(size, comp[m], kernel_ms[m], stats[m], copy_ref["GBps"]) for m in ("mrr", "de")}
    log(f"headline: {value:.2f} GB/s (MRR {modes['mrr']['GBps']}, DE {modes['de']['GBps']})")
    side = {}
    if "paper_rule" in legs:
        # the headline MRR stream resolved by the paper's round rule alone
        # (no source moved through the group's own copies): the rounds and
        # bytes per round the paper's figures are about
        side["paper_rule"] = side_leg(ctx, "paper-rule", data,
                                      {"mrr": (streams["mrr"], gmp.MODE_MRR | gmp.FLAG_PLAIN_MRR)},
                                      args.steps, args.warmup, args.waves, copy_ref["GBps"])
    if "byte" in legs:
        t0 = time.time()
        bs = {}
        for de in (0, 1):
            p = oracle.CompressParams(block_size=1 << 20, window=32768, max_match=258, de=de, group=64, format=1)
            bs[de] = oracle.compress(data, p, threads=args.threads)
        log(f"byte: compressed in {time.time() - t0:.1f}s")
        side["byte"] = side_leg(ctx, "byte", data, {"mrr": (bs[0], gmp.MODE_MRR), "de": (bs[1], gmp.MODE_DE),
                                                    "sc": (bs[0], gmp.MODE_SC)},
                                args.steps, args.warmup, args.waves, copy_ref["GBps"])
        if "compress" in legs:
            side["compress"] = compress_leg(ctx, data, {0: len(bs[0]), 1: len(bs[1])}, max(3, args.steps // 4),
                                            1, args.waves)
        del bs
    if "csv" in legs:
        t0 = time.time()
        n = args.csv_mib << 20
        csv = synth.csv_rows(n, threads=args.threads).tobytes()
        cs = {}
        for de in (0, 1):
            p = oracle.CompressParams(block_size=2 << 20, window=32768, max_match=258, lmax=12, sub_target_raw=32768,
                                      de=de, group=64)
            cs[de] = oracle.compress(csv, p, threads=args.threads)
        log(f"csv: {n >> 20} MiB generated and compressed in {time.time() - t0:.1f}s")
        side["csv"] = side_leg(ctx, "csv", csv, {"mrr": (cs[0], gmp.MODE_MRR), "de": (cs[1], gmp.MODE_DE)},
                               max(5, args.steps // 2), args.warmup, args.waves, copy_ref["GBps"])
        del csv, cs
    if "nesting" in legs:
        side["nesting"] = nesting_leg(ctx, args.steps, args.warmup, args.waves)
    if "multilaunch" in legs:
        side["multilaunch"] = multilaunch_leg(ctx, data, streams["mrr"], max(5, args.steps // 2), args.warmup,
                                              args.waves)
    batched = serving = None
    if "batched" in legs and args.batch_items > 0:
        batched = batched_leg(ctx, data, args.batch_items, min(args.steps, 5), 1, args.threads)
    if "serve" in legs and args.serve_requests > 0:
        peak = batched["GBps"] if batched else size / (kernel_ms["mrr"]["mean"] / 1e3) / 1e9
        serving = serve_leg(ctx, data, peak, args.serve_pool, args.serve_requests, args.threads, args.waves)
    ctx.close()
    dom = max(modes, key=lambda m: modes[m]["kernel_ms"])
    achieved = (size + comp[dom]) / (kernel_ms[dom]["mean"] / 1e3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_source_sha") == kernel_source_hash() and tr.get("mode") == dom and \
                tr.get("size_mib") == args.size_mib:
            traffic = tr.get("bytes_per_launch")
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic (seeded Zipf text, oracle-compressed)",
        "config": {"workload": f"zipf-text {args.size_mib} MiB, 1 MiB blocks x 64 sub-blocks of 16 KiB, "
                               f"window 32 KiB, matches 3-258, lmax 12; one MRR stream and one DE stream of "
                               f"the same data per step",
                   "raw_bytes_per_step": raw_step, "blocks_per_stream": n_blocks, "launch": launch_shape(args.waves)},
        "modes": modes,
        "roofline": {"bound": "hbm", "kernel": f"inflate_kernel ({dom})", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 5),
                     "traffic": traffic, "copy_kernel_GBps": copy_ref["GBps"],
                     "frac_of_copy": round(achieved / copy_ref["GBps"], 5)},
        "cpu_baseline": baseline,
        "copy_reference": copy_ref,
    }
    line.update(side)
    if batched:
        line["batched"] = batched
    if serving:
        line["serving"] = serving
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
