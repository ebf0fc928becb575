"""Seeded synthetic inputs (no compression arithmetic lives here).

The paper measures on a 1 GB English-Wikipedia XML dump and on the
Hollywood-2009 sparse matrix stored as a Matrix Market CSV file (section
"Experimental Evaluation").  Neither is available; these generators stand in
for them with data of the same kind:

* ``zipf_text``  — natural-language-like text: a 10,000-word vocabulary of
  lowercase words (3-9 letters), words drawn i.i.d. with Zipf rank
  probabilities proportional to k^-1.1, separated by single spaces.
* ``csv_rows``   — low-entropy numeric CSV: 8 integer columns, each with its
  own 1,000 distinct values in [0, 10^6) drawn with Zipf(1.1) rank
  probabilities; 20 % of rows repeat one of the previous 256 rows exactly.

Corpora are concatenations of independent 1 MiB chunks, chunk ``c`` drawn
from ``numpy.random.default_rng([seed, c + 1])`` (PCG64), so any slice can
be produced without generating what precedes it and every prefix is stable.

Also here: token-stream generators (the random numbers a test draws are its
inputs): the nested-back-reference construction of the paper's section
"Performance Impact of Nested back-references" at the token level, random
valid token streams, and the batch / request size mixes.
"""
from __future__ import annotations

import hashlib
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK = 1 << 20
TEXT_SEED = 1
CSV_SEED = 2
BATCH_SEED = 3
SERVE_SEED = 4

# ----------------------------------------------------------------------------- helpers


def _zipf_cdf(n: int, s: float) -> np.ndarray:
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(w)
    return c / c[-1]


def _gather_tokens(table: np.ndarray, starts: np.ndarray, lens: np.ndarray, ids: np.ndarray,
                   n_bytes: int) -> np.ndarray:
    """Concatenate table entries ids[0], ids[1], ... and truncate to n_bytes."""
    tl = lens[ids].astype(np.int64)
    ends = np.cumsum(tl)
    k = int(np.searchsorted(ends, n_bytes, side="left")) + 1
    if k > ids.size or ends[-1] < n_bytes:
        raise ValueError("not enough tokens drawn")
    ids, tl = ids[:k], tl[:k]
    first = np.empty(k, np.int64)
    first[0] = 0
    np.cumsum(tl[:-1], out=first[1:])
    idx = np.repeat(starts[ids].astype(np.int64) - first, tl) + np.arange(int(tl.sum()), dtype=np.int64)
    return table[idx[:n_bytes]]


# ----------------------------------------------------------------------------- text

_text_vocab_cache: dict = {}


def _text_vocab(seed: int):
    if seed in _text_vocab_cache:
        return _text_vocab_cache[seed]
    rng = np.random.default_rng(seed)
    words, seen = [], set()
    while len(words) < 10_000:
        L = int(rng.integers(3, 10))
        w = bytes((rng.integers(0, 26, L) + ord("a")).astype(np.uint8))
        if w in seen:
            continue  # resample duplicates
        seen.add(w)
        words.append(w + b" ")
    lens = np.array([len(w) for w in words], np.int64)
    starts = np.zeros(len(words), np.int64)
    starts[1:] = np.cumsum(lens)[:-1]
    table = np.frombuffer(b"".join(words), np.uint8)
    v = (table, starts, lens, _zipf_cdf(10_000, 1.1))
    _text_vocab_cache[seed] = v
    return v


def text_chunk(c: int, seed: int = TEXT_SEED) -> np.ndarray:
    table, starts, lens, cdf = _text_vocab(seed)
    rng = np.random.default_rng([seed, c + 1])
    n_words = CHUNK // 5
    while True:
        ids = np.searchsorted(cdf, rng.random(n_words), side="right").clip(0, 9999)
        try:
            return _gather_tokens(table, starts, lens, ids, CHUNK)
        except ValueError:
            n_words *= 2


# ----------------------------------------------------------------------------- csv

_csv_table_cache: dict = {}


def _csv_tables(seed: int):
    if seed in _csv_table_cache:
        return _csv_table_cache[seed]
    rng = np.random.default_rng(seed)
    fields, cdfs = [], []
    for col in range(8):
        vals = rng.choice(1_000_000, size=1000, replace=False)
        sep = b"\n" if col == 7 else b","
        fields.extend(str(int(v)).encode() + sep for v in vals)
    lens = np.array([len(f) for f in fields], np.int64)
    starts = np.zeros(len(fields), np.int64)
    starts[1:] = np.cumsum(lens)[:-1]
    table = np.frombuffer(b"".join(fields), np.uint8)
    v = (table, starts, lens, _zipf_cdf(1000, 1.1))
    _csv_table_cache[seed] = v
    return v


def csv_chunk(c: int, seed: int = CSV_SEED) -> np.ndarray:
    table, starts, lens, cdf = _csv_tables(seed)
    rng = np.random.default_rng([seed, c + 1])
    n_rows = CHUNK // 40
    while True:
        vidx = np.searchsorted(cdf, rng.random((n_rows, 8)), side="right").clip(0, 999)
        i = np.arange(n_rows)
        rep = rng.random(n_rows) < 0.2
        back = np.minimum(i, 256)
        off = (rng.random(n_rows) * back).astype(np.int64)
        src = np.where(rep & (back > 0), i - 1 - off, i)
        # a repeated row may itself repeat an earlier row: follow to the origin
        while True:
            nxt = src[src]
            if np.array_equal(nxt, src):
                break
            src = nxt
        vidx = vidx[src]
        ids = (vidx + np.arange(8) * 1000).reshape(-1)
        try:
            return _gather_tokens(table, starts, lens, ids, CHUNK)
        except ValueError:
            n_rows *= 2


# ----------------------------------------------------------------------------- corpora

def _corpus(kind: str, off: int, n: int, seed: int | None, threads: int) -> np.ndarray:
    fn = text_chunk if kind == "text" else csv_chunk
    seed = (TEXT_SEED if kind == "text" else CSV_SEED) if seed is None else seed
    c0, c1 = off // CHUNK, (off + n + CHUNK - 1) // CHUNK
    if n == 0:
        return np.zeros(0, np.uint8)
    fn(c0, seed) if c0 == c1 - 1 else None  # warm the vocabulary/table cache before threading
    if threads > 1 and c1 - c0 > 1:
        with ThreadPoolExecutor(threads) as ex:
            parts = list(ex.map(lambda c: fn(c, seed), range(c0, c1)))
    else:
        parts = [fn(c, seed) for c in range(c0, c1)]
    buf = np.concatenate(parts) if len(parts) > 1 else parts[0]
    s = off - c0 * CHUNK
    return np.ascontiguousarray(buf[s:s + n])


def zipf_text(n: int, off: int = 0, seed: int | None = None, threads: int = 8) -> np.ndarray:
    """n bytes of Zipf text starting at byte ``off`` of the corpus."""
    _text_vocab(TEXT_SEED if seed is None else seed)
    return _corpus("text", off, n, seed, threads)


def csv_rows(n: int, off: int = 0, seed: int | None = None, threads: int = 8) -> np.ndarray:
    """n bytes of CSV-like rows starting at byte ``off`` of the corpus."""
    _csv_tables(CSV_SEED if seed is None else seed)
    return _corpus("csv", off, n, seed, threads)


def sha256(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# ----------------------------------------------------------------------------- token streams

def nesting_tokens(n_seq: int, k: int, str_len: int = 16, seed: int = 5):
    """Token stream whose back-references nest k-interleaved: sequence i copies
    the output of sequence i-k's back-reference (the first k copy from the
    initial literals), modelling the paper's repeated-string construction in
    which k alternating strings give nesting depth G/k per group of G.
    Returns (seqs (n,3) uint32, literal bytes)."""
    period = (str_len + 1) * k
    seqs = np.empty((n_seq, 3), np.uint32)
    seqs[:, 0] = 1
    seqs[:, 1] = str_len
    seqs[:, 2] = period
    seqs[0, 0] = 1 + period
    rng = np.random.default_rng(seed)
    n_lit = int(seqs[:, 0].sum())
    lits = rng.integers(0, 256, n_lit, dtype=np.uint8).tobytes()
    return seqs, lits


def random_tokens(n_seq: int, seed: int, window: int = 32768, max_match: int = 258,
                  mean_lit: float = 3.0, overlap_frac: float = 0.2, alphabet: int = 256,
                  first_lit: int = 1):
    """Random valid token stream: geometric literal runs, match lengths in
    [3, max_match] (short ones frequent), distances in [1, min(produced,
    window)], a fraction of them overlapping (distance < length).  Returns
    (seqs (n,3) uint32, literal bytes)."""
    rng = np.random.default_rng(seed)
    seqs = np.zeros((n_seq, 3), np.uint32)
    produced = 0
    n_lit = 0
    for i in range(n_seq):
        lit = int(rng.geometric(1.0 / (mean_lit + 1.0))) - 1
        if i == 0:
            lit = max(lit, first_lit)
        produced += lit
        n_lit += lit
        if produced == 0:
            lit = 1
            produced = 1
            n_lit += 1
        u = rng.random()
        if u < 0.7:
            mlen = int(rng.integers(3, min(16, max_match) + 1))
        elif u < 0.95:
            mlen = int(rng.integers(3, min(64, max_match) + 1))
        else:
            mlen = int(rng.integers(3, max_match + 1))
        hi = min(produced, window)
        if rng.random() < overlap_frac:
            d = int(rng.integers(1, min(hi, max(1, mlen - 1)) + 1))
        else:
            d = int(rng.integers(1, hi + 1))
        seqs[i] = (lit, mlen, d)
        produced += mlen
    lits = rng.integers(0, alphabet, n_lit, dtype=np.uint8).tobytes()
    return seqs, lits


# ----------------------------------------------------------------------------- mixes

def batch_mix(n_items: int = 4096, seed: int = BATCH_SEED, lo: int = 4096, hi: int = 4 << 20,
              text_corpus: int = 256 << 20, csv_corpus: int = 1 << 30):
    """Batched workload: sizes log-uniform in [lo, hi], exactly half text and
    half CSV (shuffled), resolution mode by a fair coin, each item a slice of
    its corpus at a uniform random offset.  Returns a list of dicts."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), n_items)).astype(np.int64)
    kinds = np.array(["text"] * (n_items // 2) + ["csv"] * (n_items - n_items // 2))
    rng.shuffle(kinds)
    modes = (rng.random(n_items) < 0.5).astype(np.int64)
    items = []
    for i in range(n_items):
        corpus = text_corpus if kinds[i] == "text" else csv_corpus
        off = int(rng.integers(0, corpus - sizes[i] + 1))
        items.append({"kind": str(kinds[i]), "size": int(sizes[i]), "off": off, "de": int(modes[i])})
    return items


def request_mix(n_req: int, seed: int = SERVE_SEED, lo: int = 64 << 10, hi: int = 64 << 20,
                text_corpus: int = 256 << 20, csv_corpus: int = 1 << 30):
    """Served workload: request sizes log-uniform in [lo, hi], generator and
    resolution mode each by a fair coin, content a slice at a random offset."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), n_req)).astype(np.int64)
    kinds = np.where(rng.random(n_req) < 0.5, "text", "csv")
    modes = (rng.random(n_req) < 0.5).astype(np.int64)
    reqs = []
    for i in range(n_req):
        corpus = text_corpus if kinds[i] == "text" else csv_corpus
        off = int(rng.integers(0, corpus - sizes[i] + 1))
        reqs.append({"kind": str(kinds[i]), "size": int(sizes[i]), "off": off, "de": int(modes[i])})
    return reqs


def slice_of(kind: str, off: int, n: int, threads: int = 1) -> np.ndarray:
    return zipf_text(n, off, threads=threads) if kind == "text" else csv_rows(n, off, threads=threads)
