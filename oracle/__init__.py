"""CPU oracle for the Gompresso/Bit format (arXiv 1606.00519) — TEST INFRASTRUCTURE.

This package wraps ``gmpref.c``: the plain sequential decoder that defines
what the GPU path must produce, and the CPU compressor that produces every
compressed input (LZ77 hash-chain matcher with optional Dependency
Elimination, sub-block cutting, length-limited canonical Huffman coding).

Only the test suite, the smoke check and the benchmark's input-generation /
CPU-baseline leg may import it.  The GPU library never does; it shares no
code with this package.
"""
from __future__ import annotations

import ctypes as C
import os
import struct
import subprocess
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gmpref.c")
_LIB_PATH = os.path.join(_HERE, "libgmpref.so")

# status codes (gmpref.h)
OK, EINVAL, EFORMAT, ECODE, EDIST, ELEN, ESIZE, ESUB, ENOMEM = 0, -1, -2, -3, -4, -5, -6, -7, -9
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "EFORMAT", -3: "ECODE", -4: "EDIST", -5: "ELEN",
                -6: "ESIZE", -7: "ESUB", -9: "ENOMEM"}

BLOCK_HEADER_BYTES = 192
INDEX_ENTRY_BYTES = 16


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/libgmpref.so`` with the host C compiler."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Params(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in (
        "block_size", "window", "max_match", "lmax", "sub_target_raw", "sub_target_seq",
        "de", "group", "chain", "hash_mode", "staleness", "format")]


class BlockInfo(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in (
        "version", "mode", "group", "lmax", "raw_len", "window", "max_match",
        "n_sub", "n_seq", "n_lit", "payload_bytes")] + [("block_bytes", C.c_uint64), ("format", C.c_uint32),
                                                        ("reserved", C.c_uint32)]


@dataclass
class CompressParams:
    """Compressor parameters (defaults: 1 MiB blocks, 16 KiB sub-blocks, 32 KiB window)."""
    block_size: int = 1 << 20
    window: int = 32768
    max_match: int = 258
    lmax: int = 12
    sub_target_raw: int = 16384
    sub_target_seq: int = 0
    de: int = 0
    group: int = 64
    chain: int = 64
    hash_mode: int = 0
    staleness: int = 1024
    format: int = 0          # 0 Gompresso/Bit, 1 Gompresso/Byte

    def to_c(self) -> Params:
        return Params(*[getattr(self, f.name) for f in fields(self)])


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        u8p, szp = C.POINTER(C.c_uint8), C.POINTER(C.c_size_t)
        L.gmpref_compress.argtypes = [u8p, C.c_size_t, C.POINTER(Params), C.POINTER(u8p), szp]
        L.gmpref_compress_block.argtypes = [u8p, C.c_size_t, C.POINTER(Params), C.POINTER(u8p), szp]
        L.gmpref_parse_block.argtypes = [u8p, C.c_size_t, C.POINTER(Params), C.POINTER(C.c_void_p), szp,
                                         C.POINTER(u8p), szp, C.POINTER(C.c_void_p), szp]
        L.gmpref_encode_block.argtypes = [C.c_void_p, C.c_size_t, u8p, C.c_size_t, C.c_void_p, C.c_size_t,
                                          C.POINTER(Params), C.POINTER(u8p), szp]
        L.gmpref_encode_byte_block.argtypes = [C.c_void_p, C.c_size_t, u8p, C.c_size_t, C.POINTER(Params),
                                               C.POINTER(u8p), szp]
        L.gmpref_block_info_parse.argtypes = [u8p, C.c_size_t, C.POINTER(BlockInfo)]
        L.gmpref_decompress_block.argtypes = [u8p, C.c_size_t, u8p, C.c_size_t, szp]
        L.gmpref_decompress.argtypes = [u8p, C.c_size_t, u8p, C.c_size_t, szp]
        L.gmpref_block_tokens.argtypes = [u8p, C.c_size_t, C.POINTER(C.c_void_p), szp, C.POINTER(u8p), szp]
        L.gmpref_lz77_expand.argtypes = [C.c_void_p, C.c_size_t, u8p, C.c_size_t, C.c_uint32, C.c_uint32,
                                         u8p, C.c_size_t, szp]
        L.gmpref_validate_block.argtypes = [u8p, C.c_size_t]
        L.gmpref_de_holds.argtypes = [C.c_void_p, C.c_size_t, C.c_uint32]
        L.gmpref_mrr_rounds.argtypes = [C.c_void_p, C.c_size_t, C.c_uint32, C.c_void_p, C.c_void_p]
        L.gmpref_mrr_rounds_redirect.argtypes = [C.c_void_p, C.c_size_t, C.c_uint32, C.c_uint32, C.c_uint64,
                                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.gmpref_limited_lengths.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
        L.gmpref_canonical_codes.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        L.gmpref_length_table.argtypes = [C.c_void_p, C.c_void_p]
        L.gmpref_dist_table.argtypes = [C.c_void_p, C.c_void_p]
        L.gmpref_free.argtypes = [C.c_void_p]
        L.gmpref_default_params.argtypes = [C.POINTER(Params)]
        for fn in ("gmpref_compress", "gmpref_compress_block", "gmpref_parse_block", "gmpref_encode_block",
                   "gmpref_block_info_parse", "gmpref_decompress_block", "gmpref_decompress",
                   "gmpref_block_tokens", "gmpref_lz77_expand", "gmpref_validate_block", "gmpref_de_holds",
                   "gmpref_mrr_rounds", "gmpref_mrr_rounds_redirect", "gmpref_limited_lengths",
                   "gmpref_canonical_codes"):
            getattr(L, fn).restype = C.c_int
        L.gmpref_free.restype = None
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, rc: int, what: str):
        super().__init__(f"{what}: {STATUS_NAMES.get(rc, rc)}")
        self.rc = rc


def _u8(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(a), dtype=np.uint8)
    a = np.ascontiguousarray(a)
    return a.view(np.uint8).reshape(-1)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def _take(p, n: int) -> bytes:
    if not p:
        return b""
    data = C.string_at(p, n) if n else b""
    lib().gmpref_free(C.cast(p, C.c_void_p))
    return data


def _seq_array(seqs) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(seqs, dtype=np.uint32).reshape(-1, 3))
    return a


# --------------------------------------------------------------------------- compressor
def compress_block(data, params: CompressParams) -> bytes:
    a = _u8(data)
    out, n = C.POINTER(C.c_uint8)(), C.c_size_t()
    pc = params.to_c()
    rc = lib().gmpref_compress_block(_ptr(a), a.size, C.byref(pc), C.byref(out), C.byref(n))
    if rc:
        raise OracleError(rc, "compress_block")
    return _take(out, n.value)


def compress(data, params: CompressParams, threads: int = 1) -> bytes:
    """Compress a whole input into a stream.  With threads > 1 the blocks are
    compressed concurrently (each by the same single-threaded C code) and the
    stream is assembled here; the bytes equal the single-threaded C result."""
    a = _u8(data)
    if threads <= 1:
        out, n = C.POINTER(C.c_uint8)(), C.c_size_t()
        pc = params.to_c()
        rc = lib().gmpref_compress(_ptr(a), a.size, C.byref(pc), C.byref(out), C.byref(n))
        if rc:
            raise OracleError(rc, "compress")
        return _take(out, n.value)
    bs = params.block_size
    nb = (a.size + bs - 1) // bs
    with ThreadPoolExecutor(threads) as ex:
        blocks = list(ex.map(lambda i: compress_block(a[i * bs:(i + 1) * bs], params), range(nb)))
    return assemble_stream(blocks, bs, a.size)


def assemble_stream(blocks, block_size: int, raw_total: int) -> bytes:
    nb = len(blocks)
    head = 32 + 8 * (nb + 1)
    head = (head + 15) & ~15
    offs, pos = [], head
    for b in blocks:
        offs.append(pos)
        pos += (len(b) + 15) & ~15
    offs.append(pos)
    hdr = struct.pack("<IHHIIQQ", 0x46504D47, 1, 0, block_size, nb, raw_total, 0)
    hdr += struct.pack(f"<{nb + 1}Q", *offs)
    hdr += b"\0" * (head - len(hdr))
    parts = [hdr]
    for b in blocks:
        parts.append(b)
        parts.append(b"\0" * (((len(b) + 15) & ~15) - len(b)))
    return b"".join(parts)


def parse_block(data, params: CompressParams):
    """LZ77 parse of one block: (sequences (n,3) uint32, literal bytes, sequences per sub-block)."""
    a = _u8(data)
    sp, ns = C.c_void_p(), C.c_size_t()
    lp, nl = C.POINTER(C.c_uint8)(), C.c_size_t()
    up, nu = C.c_void_p(), C.c_size_t()
    pc = params.to_c()
    rc = lib().gmpref_parse_block(_ptr(a), a.size, C.byref(pc), C.byref(sp), C.byref(ns), C.byref(lp),
                                  C.byref(nl), C.byref(up), C.byref(nu))
    if rc:
        raise OracleError(rc, "parse_block")
    seqs = np.frombuffer(C.string_at(sp, 12 * ns.value), dtype=np.uint32).reshape(-1, 3).copy()
    subs = np.frombuffer(C.string_at(up, 4 * nu.value), dtype=np.uint32).copy()
    lib().gmpref_free(sp)
    lib().gmpref_free(up)
    return seqs, _take(lp, nl.value), subs


def encode_block(seqs, lits, sub_seqs, params: CompressParams) -> bytes:
    s = _seq_array(seqs)
    l = _u8(lits) if len(lits) else np.zeros(1, np.uint8)
    u = np.ascontiguousarray(np.asarray(sub_seqs, dtype=np.uint32))
    out, n = C.POINTER(C.c_uint8)(), C.c_size_t()
    pc = params.to_c()
    rc = lib().gmpref_encode_block(s.ctypes.data, s.shape[0], _ptr(l), len(lits), u.ctypes.data, u.size,
                                   C.byref(pc), C.byref(out), C.byref(n))
    if rc:
        raise OracleError(rc, "encode_block")
    return _take(out, n.value)


# --------------------------------------------------------------------------- decoder

def encode_byte_block(seqs, lits, params: CompressParams) -> bytes:
    """Gompresso/Byte block of a given token stream (literal runs <= 255 bytes)."""
    s = _seq_array(seqs)
    l = _u8(lits) if len(lits) else np.zeros(1, np.uint8)
    out, n = C.POINTER(C.c_uint8)(), C.c_size_t()
    pc = params.to_c()
    rc = lib().gmpref_encode_byte_block(s.ctypes.data, s.shape[0], _ptr(l), len(lits), C.byref(pc), C.byref(out),
                                        C.byref(n))
    if rc:
        raise OracleError(rc, "encode_byte_block")
    return _take(out, n.value)

def block_info(blk) -> dict:
    a = _u8(blk)
    info = BlockInfo()
    rc = lib().gmpref_block_info_parse(_ptr(a), a.size, C.byref(info))
    if rc:
        raise OracleError(rc, "block_info")
    return {f[0]: getattr(info, f[0]) for f in BlockInfo._fields_}


def decompress_block(blk, cap: int | None = None):
    """Returns (status, bytes).  cap defaults to the header's raw_len."""
    a = _u8(blk)
    if cap is None:
        try:
            cap = block_info(a)["raw_len"]
        except OracleError:
            cap = 0
    out = np.zeros(max(cap, 1), np.uint8)
    n = C.c_size_t()
    rc = lib().gmpref_decompress_block(_ptr(a), a.size, _ptr(out), cap, C.byref(n))
    return rc, (out[:n.value].tobytes() if rc == 0 else b"")


def stream_raw_total(stream) -> int:
    return struct.unpack_from("<Q", bytes(_u8(stream)[:32]), 16)[0]


def decompress(stream, cap: int | None = None):
    a = _u8(stream)
    if cap is None:
        cap = stream_raw_total(a)
    out = np.zeros(max(cap, 1), np.uint8)
    n = C.c_size_t()
    rc = lib().gmpref_decompress(_ptr(a), a.size, _ptr(out), cap, C.byref(n))
    return rc, (out[:n.value].tobytes() if rc == 0 else b"")


def block_tokens(blk):
    a = _u8(blk)
    sp, ns = C.c_void_p(), C.c_size_t()
    lp, nl = C.POINTER(C.c_uint8)(), C.c_size_t()
    rc = lib().gmpref_block_tokens(_ptr(a), a.size, C.byref(sp), C.byref(ns), C.byref(lp), C.byref(nl))
    if rc:
        return rc, None, None
    seqs = np.frombuffer(C.string_at(sp, 12 * ns.value), dtype=np.uint32).reshape(-1, 3).copy()
    lib().gmpref_free(sp)
    return rc, seqs, _take(lp, nl.value)


def lz77_expand(seqs, lits, window: int = 32768, max_match: int = 258, cap: int | None = None):
    s = _seq_array(seqs)
    if cap is None:
        cap = int(s[:, 0].sum() + s[:, 1].sum()) if s.size else 0
    l = _u8(lits) if len(lits) else np.zeros(1, np.uint8)
    out = np.zeros(max(cap, 1), np.uint8)
    n = C.c_size_t()
    rc = lib().gmpref_lz77_expand(s.ctypes.data, s.shape[0], _ptr(l), len(lits), window, max_match,
                                  _ptr(out), cap, C.byref(n))
    return rc, (out[:n.value].tobytes() if rc == 0 else b"")


def validate_block(blk) -> int:
    a = _u8(blk)
    return lib().gmpref_validate_block(_ptr(a), a.size)


def de_holds(seqs, group: int) -> bool:
    s = _seq_array(seqs)
    return bool(lib().gmpref_de_holds(s.ctypes.data, s.shape[0], group))


def mrr_rounds(seqs, group: int):
    """(rounds per group, bytes copied per round index 0..group-1)."""
    s = _seq_array(seqs)
    ng = (s.shape[0] + group - 1) // group
    rounds = np.zeros(max(ng, 1), np.uint32)
    bpr = np.zeros(group, np.uint64)
    rc = lib().gmpref_mrr_rounds(s.ctypes.data, s.shape[0], group, rounds.ctypes.data, bpr.ctypes.data)
    if rc:
        raise OracleError(rc, "mrr_rounds")
    return rounds[:ng], bpr


def mrr_rounds_redirect(seqs, group: int, jumps: int = 2, span_limit: int = 32768, per_seq: bool = False):
    """MRR rounds with sources moved through the group's own non-overlapping
    copies first (gmpref_mrr_rounds_redirect): (rounds per group, bytes per
    round), and with per_seq also (round of each sequence, distance it reads)."""
    s = _seq_array(seqs)
    ng = (s.shape[0] + group - 1) // group
    rounds = np.zeros(max(ng, 1), np.uint32)
    bpr = np.zeros(group, np.uint64)
    sr = np.zeros(max(s.shape[0], 1), np.uint32)
    sd = np.zeros(max(s.shape[0], 1), np.uint32)
    rc = lib().gmpref_mrr_rounds_redirect(s.ctypes.data, s.shape[0], group, jumps, C.c_uint64(span_limit),
                                          rounds.ctypes.data, bpr.ctypes.data, sr.ctypes.data, sd.ctypes.data)
    if rc:
        raise OracleError(rc, "mrr_rounds_redirect")
    if per_seq:
        return rounds[:ng], bpr, sr[:s.shape[0]], sd[:s.shape[0]]
    return rounds[:ng], bpr


def limited_lengths(weights, lmax: int) -> np.ndarray:
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.uint64))
    lens = np.zeros(w.size, np.uint8)
    rc = lib().gmpref_limited_lengths(w.ctypes.data, w.size, lmax, lens.ctypes.data)
    if rc:
        raise OracleError(rc, "limited_lengths")
    return lens


def canonical_codes(lens) -> np.ndarray:
    l = np.ascontiguousarray(np.asarray(lens, dtype=np.uint8))
    codes = np.zeros(l.size, np.uint32)
    rc = lib().gmpref_canonical_codes(l.ctypes.data, l.size, codes.ctypes.data)
    if rc:
        raise OracleError(rc, "canonical_codes")
    return codes


def length_table():
    b, e = np.zeros(29, np.uint16), np.zeros(29, np.uint8)
    lib().gmpref_length_table(b.ctypes.data, e.ctypes.data)
    return b, e


def dist_table():
    b, e = np.zeros(30, np.uint16), np.zeros(30, np.uint8)
    lib().gmpref_dist_table(b.ctypes.data, e.ctypes.data)
    return b, e


def stream_blocks(stream):
    """Split a stream into (block bytes, output offset) pairs."""
    a = bytes(_u8(stream))
    magic, ver, _flags, bs, nb, raw_total, _r = struct.unpack_from("<IHHIIQQ", a, 0)
    offs = struct.unpack_from(f"<{nb + 1}Q", a, 32)
    return [(a[offs[i]:offs[i + 1]], i * bs) for i in range(nb)], bs, raw_total
