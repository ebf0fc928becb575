"""MI355X (gfx950) Gompresso decompressor (Bit and Byte formats) — Python binding of the C ABI.

Argument marshalling only: every decoding step runs in the HIP kernels of
``libgompresso_hip.so`` (built from ``csrc/`` by ``build.py``).  PyTorch
supplies device buffers and streams.  There is no CPU fallback: importing
this package raises if the HIP library is not built.

Entry points mirror ``include/gompresso.h``:
``Context.decompress_block``, ``Context.decompress_stream``,
``Context.batch_create`` / ``Batch.run``, ``block_info``, ``stream_info``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# torch first: its HIP runtime (libamdhip64.so.7) is then the one this
# library binds to, so device pointers and streams are shared with torch
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgompresso_hip.so")

OK, EINVAL, EFORMAT, ECODE, EDIST, ELEN, ESIZE, ESUB, EDEVICE, ENOMEM, EBUSY, ENOSYS, ESTALL, ERANGE = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10, -11, -12, -13)
NOALLOC_SCRATCH_BYTES = 32 << 20
MODE_AUTO, MODE_MRR, MODE_DE, MODE_SC = 0, 1, 2, 3
FLAG_STATS = 0x100
FLAG_VERIFY_DE = 0x200
FLAG_PLAIN_MRR = 0x400
# per-block counters (gmp_job.d_stats)
STATS_WORDS = 80
(STAT_A2_PATH, STAT_REPAIRED, STAT_GROUPS, STAT_SPLIT, STAT_DE_ROUNDS, STAT_STALL_SITE, STAT_SEG_REJECT,
 STAT_SEG_RETRY, STAT_SPILLED) = range(9)
STAT_ROUND_BYTES = 16

EXPORTS = ("gmp_ctx_create", "gmp_ctx_destroy", "gmp_strerror", "gmp_poll", "gmp_block_info_parse", "gmp_stream_info",
           "gmp_decompress_block", "gmp_decompress_stream", "gmp_batch_create", "gmp_batch_run",
           "gmp_batch_destroy", "gmp_batch_graph_create", "gmp_batch_graph_launch", "gmp_autotune",
           "gmp_server_create", "gmp_server_submit", "gmp_server_poll", "gmp_server_drain", "gmp_server_stats",
           "gmp_server_destroy", "gmp_workspace_bytes", "gmp_noalloc_init", "gmp_decompress_block_noalloc",
           "gmp_compress_bound", "gmp_compress_batch")


class GmpError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status} ({strerror(status)})")
        self.status = status


class BlockInfo(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in ("mode", "group", "lmax", "raw_len", "window", "max_match", "n_sub",
                                          "n_seq", "n_lit", "payload_bytes")] + [
        ("block_bytes", C.c_uint64), ("format", C.c_uint32), ("reserved", C.c_uint32)]


class Job(C.Structure):
    """gmp_job; `format` is the block's gmp_block_info format (1: byte-level, no token workspace)."""
    _fields_ = [("d_comp", C.c_void_p), ("comp_len", C.c_uint64), ("d_out", C.c_void_p), ("out_len", C.c_uint64),
                ("n_seq", C.c_uint32), ("n_lit", C.c_uint32), ("d_rounds", C.c_void_p), ("d_times", C.c_void_p),
                ("d_stats", C.c_void_p), ("format", C.c_uint32), ("reserved", C.c_uint32)]


class CompressParams(C.Structure):
    _fields_ = [("window", C.c_uint32), ("max_match", C.c_uint32), ("de", C.c_uint32), ("reserved", C.c_uint32)]


class CompressJob(C.Structure):
    _fields_ = [("d_in", C.c_void_p), ("in_len", C.c_uint64), ("d_out", C.c_void_p), ("out_cap", C.c_uint64),
                ("d_out_len", C.c_void_p), ("d_status", C.c_void_p)]


class Request(C.Structure):
    _fields_ = [("d_stream", C.c_void_p), ("h_stream", C.c_void_p), ("len", C.c_uint64), ("d_out", C.c_void_p),
                ("out_len", C.c_uint64), ("d_status", C.c_void_p), ("flags", C.c_uint32), ("reserved", C.c_uint32),
                ("tag", C.c_uint64)]


class Completion(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("status", C.c_int32), ("reserved", C.c_uint32), ("bytes", C.c_uint64),
                ("t_submit_ns", C.c_uint64), ("t_admit_ns", C.c_uint64), ("t_done_ns", C.c_uint64)]


class ServerInfo(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("finished", C.c_uint64), ("pending", C.c_uint64),
                ("in_flight_bytes", C.c_uint64), ("peak_in_flight_bytes", C.c_uint64), ("budget", C.c_uint64),
                ("launches", C.c_uint64), ("peak_slots", C.c_uint32), ("reserved", C.c_uint32)]


class Tuning(C.Structure):
    _fields_ = [("waves_per_block", C.c_uint32), ("persistent", C.c_uint32), ("workgroups", C.c_uint32),
                ("rounds_per_launch", C.c_uint32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc --offload-arch=gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, i32, u32, sz = C.c_void_p, C.c_int32, C.c_uint32, C.c_size_t
    L.gmp_ctx_create.argtypes = [C.c_int, C.POINTER(vp)]
    L.gmp_ctx_destroy.argtypes = [vp]
    L.gmp_ctx_destroy.restype = None
    L.gmp_strerror.argtypes = [i32]
    L.gmp_strerror.restype = C.c_char_p
    L.gmp_poll.argtypes = [vp, vp, C.POINTER(i32)]
    L.gmp_block_info_parse.argtypes = [vp, sz, C.POINTER(BlockInfo)]
    L.gmp_stream_info.argtypes = [vp, sz, C.POINTER(u32), C.POINTER(u32), C.POINTER(C.c_uint64)]
    L.gmp_decompress_block.argtypes = [vp, vp, sz, vp, sz, vp, sz, vp, u32, vp]
    L.gmp_decompress_stream.argtypes = [vp, vp, vp, sz, vp, sz, vp, u32, vp]
    L.gmp_batch_create.argtypes = [vp, C.POINTER(Job), u32, vp, C.POINTER(vp)]
    L.gmp_batch_run.argtypes = [vp, vp, u32, C.POINTER(Tuning), vp]
    L.gmp_batch_destroy.argtypes = [vp]
    L.gmp_batch_destroy.restype = None
    L.gmp_batch_graph_create.argtypes = [vp, vp, u32, C.POINTER(Tuning)]
    L.gmp_batch_graph_launch.argtypes = [vp, vp, vp]
    L.gmp_autotune.argtypes = [vp, vp, u32, u32, C.POINTER(Tuning), C.POINTER(C.c_float), vp]
    L.gmp_server_create.argtypes = [vp, C.c_uint64, C.c_uint64, u32, C.POINTER(Tuning), C.POINTER(vp)]
    L.gmp_server_submit.argtypes = [vp, C.POINTER(Request)]
    L.gmp_server_poll.argtypes = [vp, C.POINTER(Completion), u32]
    L.gmp_server_poll.restype = u32
    L.gmp_server_drain.argtypes = [vp, u32]
    L.gmp_server_stats.argtypes = [vp, C.POINTER(ServerInfo)]
    L.gmp_workspace_bytes.argtypes = [u32, u32, C.c_uint64]
    L.gmp_workspace_bytes.restype = C.c_uint64
    L.gmp_server_destroy.argtypes = [vp]
    L.gmp_server_destroy.restype = None
    L.gmp_noalloc_init.argtypes = []
    L.gmp_compress_bound.argtypes = [C.c_uint64]
    L.gmp_compress_bound.restype = C.c_uint64
    L.gmp_compress_batch.argtypes = [vp, C.POINTER(CompressJob), u32, C.POINTER(CompressParams), vp]
    L.gmp_decompress_block_noalloc.argtypes = [vp, sz, vp, sz, vp, sz, vp, u32, vp]
    for fn in ("gmp_ctx_create", "gmp_poll", "gmp_block_info_parse", "gmp_stream_info", "gmp_decompress_block",
               "gmp_decompress_stream", "gmp_batch_create", "gmp_batch_run", "gmp_batch_graph_create",
               "gmp_batch_graph_launch", "gmp_autotune", "gmp_server_create", "gmp_server_submit",
               "gmp_server_drain", "gmp_server_stats", "gmp_noalloc_init", "gmp_decompress_block_noalloc",
               "gmp_compress_batch"):
        getattr(L, fn).restype = i32
    return L


lib = _load()


def strerror(status: int) -> str:
    return lib.gmp_strerror(status).decode()


def _host(buf):
    """(pointer, length, keep-alive) of a host bytes-like or numpy array."""
    if isinstance(buf, np.ndarray):
        a = np.ascontiguousarray(buf)
        return a.ctypes.data, a.nbytes, a
    b = bytes(buf)
    cb = C.create_string_buffer(b, len(b))
    return C.addressof(cb), len(b), cb


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def block_info(h_block) -> dict:
    p, n, keep = _host(h_block)
    info = BlockInfo()
    st = lib.gmp_block_info_parse(p, n, C.byref(info))
    if st:
        raise GmpError(st, "gmp_block_info_parse")
    return {f: getattr(info, f) for f, _ in BlockInfo._fields_ if f != "reserved"}


def compress_bound(in_len: int) -> int:
    """Largest compressed size of a block (gmp_compress_bound)."""
    return int(lib.gmp_compress_bound(in_len))


def workspace_bytes(n_seq: int, n_lit: int, comp_len: int) -> int:
    """Device token workspace one block needs (gmp_workspace_bytes)."""
    return int(lib.gmp_workspace_bytes(n_seq, n_lit, comp_len))


def stream_info(h_stream) -> tuple[int, int, int]:
    if not isinstance(h_stream, np.ndarray):
        head = bytes(h_stream[:32])
        nb = int.from_bytes(head[12:16], "little") if len(head) >= 16 else 0
        h_stream = h_stream[:32 + 8 * (nb + 1)]  # header and block table only
    p, n, keep = _host(h_stream)
    nb, bs, tot = C.c_uint32(), C.c_uint32(), C.c_uint64()
    st = lib.gmp_stream_info(p, n, C.byref(nb), C.byref(bs), C.byref(tot))
    if st:
        raise GmpError(st, "gmp_stream_info")
    return nb.value, bs.value, tot.value


class Batch:
    """A device-resident job table (gmp_batch): decode many independent blocks per launch."""

    def __init__(self, ctx: "Context", jobs: list[Job], status):
        self.ctx = ctx
        self.n = len(jobs)
        self.status = status
        arr = (Job * max(self.n, 1))(*jobs)
        h = C.c_void_p()
        st = lib.gmp_batch_create(ctx.handle, arr, self.n, C.c_void_p(status.data_ptr()), C.byref(h))
        if st:
            raise GmpError(st, "gmp_batch_create")
        self.handle = h

    def run(self, flags: int = MODE_AUTO, waves: int = 1, persistent: bool = False, workgroups: int = 0,
            stream=None, rounds_per_launch: int = 0) -> None:
        t = Tuning(waves, int(persistent), workgroups, rounds_per_launch)
        st = lib.gmp_batch_run(self.ctx.handle, self.handle, flags, C.byref(t), _stream_handle(stream))
        if st:
            raise GmpError(st, "gmp_batch_run")

    def graph_create(self, flags: int = MODE_AUTO, waves: int = 1, persistent: bool = True,
                     workgroups: int = 0, rounds_per_launch: int = 0) -> None:
        """Capture this batch's launch as a HIP graph (gmp_batch_graph_create)."""
        t = Tuning(waves, int(persistent), workgroups, rounds_per_launch)
        st = lib.gmp_batch_graph_create(self.ctx.handle, self.handle, flags, C.byref(t))
        if st:
            raise GmpError(st, "gmp_batch_graph_create")

    def graph_launch(self, stream=None) -> None:
        st = lib.gmp_batch_graph_launch(self.ctx.handle, self.handle, _stream_handle(stream))
        if st:
            raise GmpError(st, "gmp_batch_graph_launch")

    def autotune(self, flags: int = MODE_AUTO, reps: int = 3, stream=None) -> tuple[dict, float]:
        """Time the launch candidates (gmp_autotune); returns (tuning, median ms)."""
        t, ms = Tuning(), C.c_float()
        st = lib.gmp_autotune(self.ctx.handle, self.handle, flags, reps, C.byref(t), C.byref(ms),
                              _stream_handle(stream))
        if st:
            raise GmpError(st, "gmp_autotune")
        return ({"waves": t.waves_per_block, "persistent": bool(t.persistent), "workgroups": t.workgroups,
                 "rounds_per_launch": t.rounds_per_launch}, float(ms.value))

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.gmp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """gmp_server: continuous batching of decompression requests on one GPU.

    submit() takes device-resident stream bytes (torch uint8 CUDA tensor), a host copy
    of the stream (for its headers), an output tensor and a per-block int32 status
    tensor; the caller keeps them alive until the request's completion is polled."""

    def __init__(self, ctx: "Context", budget_bytes: int, workspace_bytes: int = 0, slots: int = 4,
                 waves: int = 7):
        self.ctx = ctx
        t = Tuning(waves, 0, 0, 0)
        h = C.c_void_p()
        st = lib.gmp_server_create(ctx.handle, budget_bytes, workspace_bytes, slots, C.byref(t), C.byref(h))
        if st:
            raise GmpError(st, "gmp_server_create")
        self.handle = h
        self._keep = {}

    def submit(self, d_stream, h_stream, out, status, flags: int = MODE_AUTO, tag: int = 0) -> None:
        p, n, keep = _host(h_stream)
        r = Request(d_stream.data_ptr(), p, n, out.data_ptr(), out.numel(), status.data_ptr(), flags, 0, tag)
        st = lib.gmp_server_submit(self.handle, C.byref(r))
        if st:
            raise GmpError(st, "gmp_server_submit")
        self._keep[tag] = keep

    def poll(self, max_n: int = 256) -> list[dict]:
        arr = (Completion * max_n)()
        n = lib.gmp_server_poll(self.handle, arr, max_n)
        out = []
        for c in arr[:n]:
            self._keep.pop(c.tag, None)
            out.append({f: getattr(c, f) for f, _ in Completion._fields_ if f != "reserved"})
        return out

    def drain(self, timeout_ms: int = 60000) -> None:
        st = lib.gmp_server_drain(self.handle, timeout_ms)
        if st:
            raise GmpError(st, "gmp_server_drain")

    def stats(self) -> dict:
        i = ServerInfo()
        st = lib.gmp_server_stats(self.handle, C.byref(i))
        if st:
            raise GmpError(st, "gmp_server_stats")
        return {f: getattr(i, f) for f, _ in ServerInfo._fields_ if f != "reserved"}

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.gmp_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """gmp_ctx: token workspace, job tables and launch state on one GPU."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        st = lib.gmp_ctx_create(device, C.byref(h))
        if st:
            raise GmpError(st, "gmp_ctx_create")
        self.handle = h
        self.device = device

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.gmp_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def decompress_block(self, d_block, h_block, out, status, flags: int = MODE_AUTO, stream=None) -> None:
        """Decode one block (async).  d_block / out / status: torch uint8 / uint8 / int32 CUDA tensors;
        h_block: host copy of the block (header and index are read from it)."""
        p, n, keep = _host(h_block)
        st = lib.gmp_decompress_block(self.handle, C.c_void_p(d_block.data_ptr()), d_block.numel(), p, n,
                                      C.c_void_p(out.data_ptr()), out.numel(), C.c_void_p(status.data_ptr()),
                                      flags, _stream_handle(stream))
        if st:
            raise GmpError(st, "gmp_decompress_block")

    def decompress_stream(self, d_stream, h_stream, out, status, flags: int = MODE_AUTO, stream=None) -> None:
        """Decode every block of a stream (async); status holds one int32 per block."""
        p, n, keep = _host(h_stream)
        st = lib.gmp_decompress_stream(self.handle, C.c_void_p(d_stream.data_ptr()), p, n,
                                       C.c_void_p(out.data_ptr()), out.numel(), C.c_void_p(status.data_ptr()),
                                       flags, _stream_handle(stream))
        if st:
            raise GmpError(st, "gmp_decompress_stream")

    def compress_batch(self, jobs: list[CompressJob], window: int = 32768, max_match: int = 258, de: int = 0,
                       stream=None) -> None:
        """Compress blocks into byte-level blocks on the GPU (gmp_compress_batch, async)."""
        arr = (CompressJob * max(len(jobs), 1))(*jobs)
        prm = CompressParams(window, max_match, de, 0)
        st = lib.gmp_compress_batch(self.handle, arr, len(jobs), C.byref(prm), _stream_handle(stream))
        if st:
            raise GmpError(st, "gmp_compress_batch")

    def batch_create(self, jobs: list[Job], status) -> Batch:
        return Batch(self, jobs, status)

    def poll(self, stream=None) -> int:
        """First device-side error recorded by this context's launches since the last poll
        (gmp_poll; waits for the work queued on `stream`); 0 if none."""
        e = C.c_int32()
        st = lib.gmp_poll(self.handle, _stream_handle(stream), C.byref(e))
        if st:
            raise GmpError(st, "gmp_poll")
        return int(e.value)
