"""MI355X (gfx950) Gompresso/Bit decompressor — Python binding of the C ABI.

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

OK, EINVAL, EFORMAT, ECODE, EDIST, ELEN, ESIZE, ESUB, EDEVICE, ENOMEM, EBUSY, ENOSYS = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10, -11)
MODE_AUTO, MODE_MRR, MODE_DE = 0, 1, 2
FLAG_STATS = 0x100

EXPORTS = ("gmp_ctx_create", "gmp_ctx_destroy", "gmp_strerror", "gmp_block_info_parse", "gmp_stream_info",
           "gmp_decompress_block", "gmp_decompress_stream", "gmp_batch_create", "gmp_batch_run",
           "gmp_batch_destroy")


class GmpError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status} ({strerror(status)})")
        self.status = status


class BlockInfo(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in ("mode", "group", "lmax", "raw_len", "window", "max_match", "n_sub",
                                          "n_seq", "n_lit", "payload_bytes")] + [("block_bytes", C.c_uint64)]


class Job(C.Structure):
    _fields_ = [("d_comp", C.c_void_p), ("comp_len", C.c_uint64), ("d_out", C.c_void_p), ("out_len", C.c_uint64),
                ("n_seq", C.c_uint32), ("n_lit", C.c_uint32), ("d_rounds", C.c_void_p), ("d_times", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("waves_per_block", C.c_uint32), ("persistent", C.c_uint32), ("workgroups", C.c_uint32),
                ("reserved", C.c_uint32)]


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
    L.gmp_block_info_parse.argtypes = [vp, sz, C.POINTER(BlockInfo)]
    L.gmp_stream_info.argtypes = [vp, sz, C.POINTER(u32), C.POINTER(u32), C.POINTER(C.c_uint64)]
    L.gmp_decompress_block.argtypes = [vp, vp, sz, vp, sz, vp, sz, vp, u32, vp]
    L.gmp_decompress_stream.argtypes = [vp, vp, vp, sz, vp, sz, vp, u32, vp]
    L.gmp_batch_create.argtypes = [vp, C.POINTER(Job), u32, vp, C.POINTER(vp)]
    L.gmp_batch_run.argtypes = [vp, vp, u32, C.POINTER(Tuning), vp]
    L.gmp_batch_destroy.argtypes = [vp]
    L.gmp_batch_destroy.restype = None
    for fn in ("gmp_ctx_create", "gmp_block_info_parse", "gmp_stream_info", "gmp_decompress_block",
               "gmp_decompress_stream", "gmp_batch_create", "gmp_batch_run"):
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
    return {f: getattr(info, f) for f, _ in BlockInfo._fields_}


def stream_info(h_stream) -> tuple[int, int, int]:
    p, n, keep = _host(h_stream[:4096] if not isinstance(h_stream, np.ndarray) else h_stream)
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
            stream=None) -> None:
        t = Tuning(waves, int(persistent), workgroups, 0)
        st = lib.gmp_batch_run(self.ctx.handle, self.handle, flags, C.byref(t), _stream_handle(stream))
        if st:
            raise GmpError(st, "gmp_batch_run")

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.gmp_batch_destroy(self.handle)
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

    def batch_create(self, jobs: list[Job], status) -> Batch:
        return Batch(self, jobs, status)
