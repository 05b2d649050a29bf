"""CPU oracle for the word counter. TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's ``cpu_baseline`` leg may import this
package. It wraps ``wc_oracle.cpp`` (plain single-threaded C++, std::unordered_map), which
follows the paper's definitions directly: Section 2 / Section 3.1 (lower-case, drop
punctuation, split into words), Section 3.1 / 3.2 (count per document in a dictionary, adding
while populating), Section 3.3 (group per-document counts and sum them) and Section 4.3
(per-corpus distinctive words, with the exact ranking stated in wc_oracle.cpp).

Pins (tests/test_oracle.py): brute force against Python's ``re`` on every short string over a
small alphabet and on random text; the paper's worked example of Section 2, its "Dog"/"dog."
remark, the grouped counts of Section 3.3 and the "(Applause)" marker of Section 4.3
(tests/golden/); the generator's rank histogram at workload scale; invariants; the top-k
ranking against a brute-force sort with exact fractions. Nothing here is "parity unpinned"
except the informational double score, which is recomputed from integers.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wc_oracle.cpp")
_PAR = os.path.join(_HERE, "cpu_parallel.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True, sanitize: bool = False, out: str | None = None) -> str:
    """Compile the oracle (single-threaded) and the paper's threaded CPU design (a timed
    baseline, cpu_parallel.cpp) with g++ -O2."""
    out = out or _LIB
    if not force and os.path.exists(out):
        return out
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", "-o", out, _SRC, _PAR]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g"]
    subprocess.run(cmd, check=True)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.oracle_count.restype = ctypes.c_void_p
        L.oracle_count.argtypes = [_u8p, ctypes.c_uint64, _u64p, ctypes.c_uint64, ctypes.c_int]
        L.oracle_count_utf8.restype = ctypes.c_void_p
        L.oracle_count_utf8.argtypes = [_u8p, ctypes.c_uint64, _u64p, ctypes.c_uint64,
                                        ctypes.c_int]
        L.oracle_merge.restype = ctypes.c_void_p
        L.oracle_merge.argtypes = [ctypes.c_uint32, ctypes.POINTER(_u8p), ctypes.POINTER(_u64p),
                                   ctypes.POINTER(_u64p), _u64p]
        for f in ("oracle_table_size", "oracle_table_total", "oracle_table_word_bytes"):
            getattr(L, f).restype = ctypes.c_uint64
            getattr(L, f).argtypes = [ctypes.c_void_p]
        L.oracle_table_export.restype = None
        L.oracle_table_export.argtypes = [ctypes.c_void_p, _u8p, _u64p, _u64p, _u64p]
        L.oracle_table_free.restype = None
        L.oracle_table_free.argtypes = [ctypes.c_void_p]
        L.oracle_topk_ratio.restype = ctypes.c_uint64
        L.oracle_topk_ratio.argtypes = [ctypes.c_uint32, ctypes.POINTER(_u8p),
                                        ctypes.POINTER(_u64p), ctypes.POINTER(_u64p), _u64p,
                                        ctypes.c_uint32, ctypes.c_uint64, _u64p, _u64p, _u64p,
                                        _dp, _u64p, _u64p, _u8p]
        L.cpu_parallel_count.restype = ctypes.c_void_p
        L.cpu_parallel_count.argtypes = [_u8p, ctypes.c_uint64, _u64p, ctypes.c_uint64,
                                         ctypes.c_uint32]
        for f in ("cpu_parallel_size", "cpu_parallel_total", "cpu_parallel_word_bytes"):
            getattr(L, f).restype = ctypes.c_uint64
            getattr(L, f).argtypes = [ctypes.c_void_p]
        L.cpu_parallel_seconds.restype = ctypes.c_double
        L.cpu_parallel_seconds.argtypes = [ctypes.c_void_p]
        L.cpu_parallel_export.restype = None
        L.cpu_parallel_export.argtypes = [ctypes.c_void_p, _u8p, _u64p, _u64p]
        L.cpu_parallel_free.restype = None
        L.cpu_parallel_free.argtypes = [ctypes.c_void_p]
        L.oracle_joint_word_bytes.restype = ctypes.c_uint64
        L.oracle_joint_word_bytes.argtypes = [ctypes.c_uint32, ctypes.POINTER(_u8p),
                                              ctypes.POINTER(_u64p), _u64p]
        _lib = L
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


@dataclass
class Table:
    """A word table in canonical order: entry e is words[word_offsets[e]:word_offsets[e+1]]."""
    words: np.ndarray         # uint8
    word_offsets: np.ndarray  # uint64[n+1]
    counts: np.ndarray        # uint64[n]
    docs: np.ndarray          # uint64[n] (zeros for a global table)
    total: int                # tokens
    per_doc: bool = False

    def __len__(self):
        return len(self.counts)

    def word(self, e: int) -> bytes:
        return self.words[self.word_offsets[e]:self.word_offsets[e + 1]].tobytes()

    def as_dict(self) -> dict:
        """{word: count} for a global table, {(doc, word): count} for a per-document one."""
        out = {}
        for e in range(len(self)):
            key = (int(self.docs[e]), self.word(e)) if self.per_doc else self.word(e)
            out[key] = int(self.counts[e])
        return out


def _export(h, per_doc=False) -> Table:
    L = lib()
    try:
        n = L.oracle_table_size(h)
        wb = L.oracle_table_word_bytes(h)
        words = np.zeros(max(wb, 1), dtype=np.uint8)
        offs = np.zeros(n + 1, dtype=np.uint64)
        cnts = np.zeros(max(n, 1), dtype=np.uint64)
        docs = np.zeros(max(n, 1), dtype=np.uint64)
        L.oracle_table_export(h, _p(words, _u8p), _p(offs, _u64p), _p(cnts, _u64p),
                              _p(docs, _u64p))
        return Table(words[:wb], offs, cnts[:n], docs[:n], L.oracle_table_total(h), per_doc)
    finally:
        L.oracle_table_free(h)


class OracleError(ValueError):
    pass


def count(text, offsets=None, per_doc: bool = False, utf8: bool = False) -> Table:
    """Count words of text (bytes / uint8 array) split into documents by offsets. utf8: the
    UTF-8 reading of wc_oracle.cpp (multi-byte word characters, ASCII-only folding)."""
    buf = np.frombuffer(bytes(text), dtype=np.uint8) if isinstance(text, (bytes, bytearray)) \
        else np.ascontiguousarray(text, dtype=np.uint8)
    if offsets is None:
        offsets = [0, len(buf)]
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    n_docs = len(off) - 1
    if n_docs < 0:
        raise OracleError("offsets must hold at least one value")
    keep = buf if len(buf) else np.zeros(1, dtype=np.uint8)
    fn = lib().oracle_count_utf8 if utf8 else lib().oracle_count
    h = fn(_p(keep, _u8p), len(buf), _p(off, _u64p), n_docs, int(per_doc))
    if not h:
        raise OracleError("invalid document offsets")
    return _export(h, per_doc)


def _table_arrays(tables):
    k = len(tables)
    words = [np.ascontiguousarray(t.words if len(t.words) else np.zeros(1, np.uint8), np.uint8)
             for t in tables]
    offs = [np.ascontiguousarray(t.word_offsets, np.uint64) for t in tables]
    cnts = [np.ascontiguousarray(t.counts if len(t.counts) else np.zeros(1, np.uint64), np.uint64)
            for t in tables]
    n = np.array([len(t.counts) for t in tables], dtype=np.uint64)
    W = (_u8p * k)(*[_p(w, _u8p) for w in words])
    O = (_u64p * k)(*[_p(o, _u64p) for o in offs])
    C = (_u64p * k)(*[_p(c, _u64p) for c in cnts])
    return (words, offs, cnts, n), W, O, C


def merge(tables) -> Table:
    """Pointwise sum of tables over the union of their words (Section 3.3)."""
    keep, W, O, C = _table_arrays(tables)
    h = lib().oracle_merge(len(tables), W, O, C, _p(keep[3], _u64p))
    return _export(h)


def table_from_dict(d: dict) -> Table:
    items = sorted(d.items())
    words = b"".join(w for w, _ in items)
    offs = np.zeros(len(items) + 1, dtype=np.uint64)
    np.cumsum([len(w) for w, _ in items], out=offs[1:])
    cnts = np.array([c for _, c in items], dtype=np.uint64)
    return Table(np.frombuffer(words, dtype=np.uint8).copy(), offs, cnts,
                 np.zeros(len(items), np.uint64), int(cnts.sum()) if len(items) else 0)


@dataclass
class TopK:
    words: list          # list (per corpus) of lists of bytes
    n_c: list            # list of uint64 arrays
    n_rest: list
    score: list          # list of float64 arrays
    vocab_size: int


def topk_ratio(tables, k: int, min_count: int = 1) -> TopK:
    """Per-corpus top-k distinctive words (Section 4.3; ranking as in wc_oracle.cpp)."""
    c = len(tables)
    keep, W, O, C = _table_arrays(tables)
    L = lib()
    jb = L.oracle_joint_word_bytes(c, W, O, _p(keep[3], _u64p))
    kk = max(k, 1)
    ow = np.zeros(c * kk, np.uint64)
    onc = np.zeros(c * kk, np.uint64)
    onr = np.zeros(c * kk, np.uint64)
    osc = np.zeros(c * kk, np.float64)
    nrows = np.zeros(c, np.uint64)
    # first call with no joint buffers to learn V, then fill them
    V = L.oracle_topk_ratio(c, W, O, C, _p(keep[3], _u64p), k, min_count, _p(ow, _u64p),
                            _p(onc, _u64p), _p(onr, _u64p), _p(osc, _dp), _p(nrows, _u64p),
                            None, None)
    joff = np.zeros(V + 1, np.uint64)
    jw = np.zeros(max(jb, 1), np.uint8)
    L.oracle_topk_ratio(c, W, O, C, _p(keep[3], _u64p), k, min_count, _p(ow, _u64p),
                        _p(onc, _u64p), _p(onr, _u64p), _p(osc, _dp), _p(nrows, _u64p),
                        _p(joff, _u64p), _p(jw, _u8p))
    words, ncs, nrs, scs = [], [], [], []
    for t in range(c):
        r = int(nrows[t])
        idx = ow[t * kk:t * kk + r]
        words.append([jw[joff[i]:joff[i + 1]].tobytes() for i in idx])
        ncs.append(onc[t * kk:t * kk + r].copy())
        nrs.append(onr[t * kk:t * kk + r].copy())
        scs.append(osc[t * kk:t * kk + r].copy())
    return TopK(words, ncs, nrs, scs, int(V))


def cpu_parallel(text, offsets=None, threads: int = 1):
    """The paper's CPU design (Section 3.1 threads each counting a share of the text, Section 3.2
    merging their dictionaries), for timing beside the GPU counter: (dict {word: count}, total
    tokens, seconds spent counting and merging)."""
    buf = np.frombuffer(bytes(text), dtype=np.uint8) if isinstance(text, (bytes, bytearray)) \
        else np.ascontiguousarray(text, dtype=np.uint8)
    if offsets is None:
        offsets = [0, len(buf)]
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    keep = buf if len(buf) else np.zeros(1, dtype=np.uint8)
    L = lib()
    h = L.cpu_parallel_count(_p(keep, _u8p), len(buf), _p(off, _u64p), len(off) - 1, threads)
    try:
        n = L.cpu_parallel_size(h)
        wb = L.cpu_parallel_word_bytes(h)
        words = np.zeros(max(wb, 1), dtype=np.uint8)
        offs = np.zeros(n + 1, dtype=np.uint64)
        cnts = np.zeros(max(n, 1), dtype=np.uint64)
        L.cpu_parallel_export(h, _p(words, _u8p), _p(offs, _u64p), _p(cnts, _u64p))
        wbytes = words.tobytes()
        d = {wbytes[offs[e]:offs[e + 1]]: int(cnts[e]) for e in range(n)}
        return d, int(L.cpu_parallel_total(h)), float(L.cpu_parallel_seconds(h))
    finally:
        L.cpu_parallel_free(h)
