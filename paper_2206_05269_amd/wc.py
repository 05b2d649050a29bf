"""ctypes binding of libwc (include/wc.h): argument marshalling only.

Every step of counting, merging and ranking runs in the HIP kernels of libwc.so; PyTorch
supplies device memory (the caller-owned workspace) and the stream. There is no CPU path:
when the library or a GPU is missing these functions raise.
"""
from __future__ import annotations

import ctypes
import json
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libwc.so")

WC_OK, WC_EINVAL, WC_ENOMEM, WC_ETABLEFULL, WC_EOVERFLOW, WC_EDEVICE, WC_EAGAIN = \
    0, -1, -2, -3, -4, -5, -6
WC_GLOBAL, WC_PER_DOC = 0, 1
WC_FLUSH_ALL, WC_FLUSH_BYPASS = 0, 1
WC_DIRECT_NEVER = 0xFFFFFFFF  # wc_tuning.direct_kib: no document skips the first count
WC_DEBUG_TIME, WC_DEBUG_NO_LDS, WC_DEBUG_DIRECT, WC_DEBUG_SPILL, WC_DEBUG_DOCS = 1, 2, 4, 8, 16
WC_FOLD_SQRT, WC_FOLD_ALT_HARMONIC = 0, 1
WC_TOKENIZE_ASCII, WC_TOKENIZE_UTF8 = 0, 1


class WcError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().wc_strerror(status).decode()
        if status == WC_EDEVICE:
            msg += f" (hipError {lib().wc_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{status}]")


class Tuning(ctypes.Structure):
    _fields_ = [("stage_bytes", ctypes.c_uint32), ("lds_entries", ctypes.c_uint32),
                ("flush_policy", ctypes.c_uint32), ("grid_blocks", ctypes.c_uint32),
                ("lds_load_pct", ctypes.c_uint32), ("chunk_bytes", ctypes.c_uint32),
                ("direct_kib", ctypes.c_uint32)]


class Opts(ctypes.Structure):
    _fields_ = [("count_bytes", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("table_slots", ctypes.c_uint64), ("tuning", ctypes.POINTER(Tuning)),
                ("debug_flags", ctypes.c_uint32), ("debug_hash_bits", ctypes.c_uint32),
                ("word_bytes_cap", ctypes.c_uint64), ("debug_count_bias", ctypes.c_uint64),
                ("tokenizer", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class Plan(ctypes.Structure):
    _fields_ = [("table_slots", ctypes.c_uint64), ("workspace_bytes", ctypes.c_uint64),
                ("max_entries", ctypes.c_uint64), ("word_bytes_cap", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("n_entries", ctypes.c_uint64), ("total_tokens", ctypes.c_uint64),
                ("word_bytes", ctypes.c_uint64), ("n_docs", ctypes.c_uint64),
                ("table_slots", ctypes.c_uint64), ("count_bytes", ctypes.c_uint32),
                ("mode", ctypes.c_uint32), ("d_word_offsets", ctypes.c_void_p),
                ("d_words", ctypes.c_void_p), ("d_counts", ctypes.c_void_p),
                ("d_doc_ptr", ctypes.c_void_p), ("d_doc_len", ctypes.c_void_p),
                ("d_docs", ctypes.c_void_p),
                ("kernel_ms", ctypes.c_float), ("total_ms", ctypes.c_float),
                ("stats", ctypes.c_uint64 * 5)]


class TopKStruct(ctypes.Structure):
    _fields_ = [("n_corpora", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("vocab_size", ctypes.c_uint64), ("d_word_offsets", ctypes.c_void_p),
                ("d_words", ctypes.c_void_p), ("d_n_c", ctypes.c_void_p),
                ("d_n_rest", ctypes.c_void_p), ("d_score", ctypes.c_void_p),
                ("n_rows", ctypes.c_uint64 * 64), ("word_bytes", ctypes.c_uint64)]


_lib = None


def lib():
    """Load libwc.so (building it first when it has never been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(_LIB_PATH)
        vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
        L.wc_strerror.restype = ctypes.c_char_p
        L.wc_strerror.argtypes = [ctypes.c_int32]
        L.wc_last_hip_error.restype = ctypes.c_int32
        L.wc_count_plan.argtypes = [u64, u64, ctypes.POINTER(Opts), ctypes.POINTER(Plan)]
        L.wc_count.argtypes = [vp, u64, vp, u64, ctypes.POINTER(Opts), vp, u64,
                               ctypes.POINTER(Result), vp]
        L.wc_count_static.argtypes = [vp, u64, vp, u64, ctypes.POINTER(Opts), vp, vp, u64, vp,
                                      u64, ctypes.POINTER(Result), vp]
        L.wc_count_host_plan.argtypes = [u64, u64, ctypes.POINTER(Opts), u64, ctypes.POINTER(Plan)]
        L.wc_count_host.argtypes = [vp, u64, vp, u64, ctypes.POINTER(Opts), u64, vp, vp, u64,
                                    ctypes.POINTER(Result), vp]
        L.wc_sort_canonical.argtypes = [u64, vp, vp, vp, vp]
        L.wc_sort_canonical.restype = ctypes.c_int32
        L.wc_merge_dense_plan.argtypes = [ctypes.POINTER(Result), ctypes.POINTER(Opts), u64,
                                          ctypes.POINTER(u64)]
        L.wc_merge_dense.argtypes = [ctypes.POINTER(Result), ctypes.POINTER(Opts), vp, u64,
                                     ctypes.POINTER(Result), vp]
        L.wc_merge_plan.argtypes = [ctypes.POINTER(ctypes.POINTER(Result)), u32,
                                    ctypes.POINTER(Opts), ctypes.POINTER(Plan)]
        L.wc_merge.argtypes = [ctypes.POINTER(ctypes.POINTER(Result)), u32, ctypes.POINTER(Opts),
                               vp, u64, ctypes.POINTER(Result), vp]
        L.wc_topk_ratio_plan.argtypes = [ctypes.POINTER(ctypes.POINTER(Result)), u32, u32,
                                         ctypes.POINTER(u64)]
        L.wc_topk_ratio.argtypes = [ctypes.POINTER(ctypes.POINTER(Result)), u32, u32, u64, vp,
                                    u64, ctypes.POINTER(TopKStruct), vp]
        L.wc_hash_words.argtypes = [vp, vp, u64, vp, vp]
        L.wc_table_to_host.argtypes = [ctypes.POINTER(Result), vp, vp, vp]
        L.wc_table_to_host.restype = ctypes.c_int32
        L.wc_server_create.argtypes = [ctypes.c_int, u64, u32, ctypes.POINTER(vp)]
        L.wc_server_submit.argtypes = [vp, vp, u64, vp, u64, ctypes.c_int, ctypes.POINTER(Opts),
                                       ctypes.POINTER(u64)]
        L.wc_server_poll.argtypes = [vp, u64, ctypes.POINTER(Result)]
        L.wc_server_wait.argtypes = [vp, u64, ctypes.POINTER(Result)]
        L.wc_server_times.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]
        L.wc_server_merge.argtypes = [vp, ctypes.POINTER(u64), u32, ctypes.POINTER(Opts),
                                      ctypes.POINTER(u64)]
        L.wc_server_release.argtypes = [vp, u64]
        L.wc_server_launches.argtypes = [vp]
        L.wc_server_launches.restype = u64
        L.wc_server_destroy.argtypes = [vp]
        for f in ("wc_server_create", "wc_server_submit", "wc_server_poll", "wc_server_wait",
                  "wc_server_times", "wc_server_merge", "wc_server_release", "wc_server_destroy"):
            getattr(L, f).restype = ctypes.c_int32
        L.wc_autotune_plan.argtypes = [u64, u64, ctypes.POINTER(Opts), ctypes.POINTER(u64)]
        L.wc_autotune.argtypes = [vp, u64, vp, u64, ctypes.POINTER(Opts), vp, u64,
                                  ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_float), vp]
        L.wc_autotune_plan.restype = ctypes.c_int32
        L.wc_autotune.restype = ctypes.c_int32
        L.wc_fold_sum_plan.argtypes = [u64, ctypes.POINTER(u64)]
        L.wc_fold_sum.argtypes = [u32, u64, vp, vp, u64, vp]
        L.wc_fold_sum_plan.restype = ctypes.c_int32
        L.wc_fold_sum.restype = ctypes.c_int32
        L.wc_batch_plan.argtypes = [ctypes.POINTER(Opts), u64, u64, ctypes.POINTER(u64)]
        L.wc_batch_create.argtypes = [ctypes.POINTER(Opts), u64, u64, vp, u64,
                                      ctypes.POINTER(vp)]
        L.wc_batch_run.argtypes = [vp, vp, u64, vp, u64, ctypes.POINTER(Result), vp]
        L.wc_batch_destroy.argtypes = [vp]
        for f in ("wc_batch_plan", "wc_batch_create", "wc_batch_run", "wc_batch_destroy"):
            getattr(L, f).restype = ctypes.c_int32
        for f in ("wc_count_plan", "wc_count", "wc_count_static", "wc_count_host_plan",
                  "wc_count_host", "wc_merge_dense_plan",
                  "wc_merge_dense", "wc_merge_plan", "wc_merge", "wc_topk_ratio_plan",
                  "wc_topk_ratio", "wc_hash_words"):
            getattr(L, f).restype = ctypes.c_int32
        _lib = L
    return _lib


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _require_cuda(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")


def _alloc(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class Table:
    """A word table in device memory (result of count or merge); owns its workspace."""

    def __init__(self, res: Result, workspace: torch.Tensor, keep: tuple = ()):
        self.res = res
        self.workspace = workspace
        self._keep = keep  # inputs that long-word references may point into

    # --- device views -------------------------------------------------------------------
    def _view(self, ptr: int, nbytes: int, dtype) -> torch.Tensor:
        base = self.workspace.data_ptr()
        off = int(ptr) - base
        if nbytes == 0:
            return torch.empty(0, dtype=dtype, device=self.workspace.device)
        assert 0 <= off and off + nbytes <= self.workspace.numel()
        return self.workspace[off:off + nbytes].view(dtype)

    @property
    def n_entries(self) -> int:
        return int(self.res.n_entries)

    @property
    def total_tokens(self) -> int:
        return int(self.res.total_tokens)

    @property
    def stats(self) -> dict:
        """Per-call statistics: the two-pass global count's spilled records, records sent
        straight to the global table, dictionary words and pass-2 overflow; the
        document-centric kernel's documents counted by its second pass (overflowed, or over the
        size limit; zero where a path has none)."""
        s = self.res.stats
        return {"spilled": int(s[0]), "arena_direct": int(s[1]), "dict_words": int(s[2]),
                "docs_recounted": int(s[3]), "reduce_overflow": int(s[4])}

    def word_offsets(self) -> torch.Tensor:
        return self._view(self.res.d_word_offsets, 8 * (self.n_entries + 1), torch.int64)

    def words(self) -> torch.Tensor:
        return self._view(self.res.d_words, int(self.res.word_bytes), torch.uint8)

    def counts(self) -> torch.Tensor:
        dt = torch.int32 if self.res.count_bytes == 4 else torch.int64
        return self._view(self.res.d_counts, self.res.count_bytes * self.n_entries, dt)

    def doc_ptr(self) -> Optional[torch.Tensor]:
        if not self.res.d_doc_ptr:
            return None
        return self._view(self.res.d_doc_ptr, 8 * int(self.res.n_docs), torch.int64)

    def doc_len(self) -> Optional[torch.Tensor]:
        if not self.res.d_doc_len:
            return None
        return self._view(self.res.d_doc_len, 8 * int(self.res.n_docs), torch.int64)

    def docs(self) -> Optional[torch.Tensor]:
        if not self.res.d_docs:
            return None
        return self._view(self.res.d_docs, 8 * self.n_entries, torch.int64)

    # --- host copies --------------------------------------------------------------------
    def to_host(self):
        """(words uint8, word_offsets int64[n+1], counts int64[n], docs int64[n] or None)."""
        w = self.words().cpu().numpy()
        o = self.word_offsets().cpu().numpy()
        c = self.counts().cpu().numpy().astype(np.int64)
        d = self.docs()
        return w, o, c, (d.cpu().numpy() if d is not None else None)

    def as_dict(self) -> dict:
        """{word: count}, or {(doc, word): count} for a per-document table."""
        w, o, c, d = self.to_host()
        wb = w.tobytes()
        if d is None:
            return {wb[o[e]:o[e + 1]]: int(c[e]) for e in range(len(c))}
        return {(int(d[e]), wb[o[e]:o[e + 1]]): int(c[e]) for e in range(len(c))}


def _opts(count_bytes, per_doc, table_slots, tuning, debug_flags, debug_hash_bits,
          word_bytes_cap, debug_count_bias=0, utf8=False):
    o = Opts()
    o.count_bytes = count_bytes
    o.mode = WC_PER_DOC if per_doc else WC_GLOBAL
    o.table_slots = table_slots
    o.tuning = ctypes.pointer(tuning) if tuning is not None else None
    o.debug_flags = debug_flags
    o.debug_hash_bits = debug_hash_bits
    o.word_bytes_cap = word_bytes_cap
    o.debug_count_bias = debug_count_bias
    o.tokenizer = WC_TOKENIZE_UTF8 if utf8 else WC_TOKENIZE_ASCII
    return o


def make_tuning(stage_bytes=0, lds_entries=0, flush_policy=WC_FLUSH_ALL, grid_blocks=0,
                lds_load_pct=0, chunk_bytes=0, direct_kib=0) -> Tuning:
    return Tuning(stage_bytes, lds_entries, flush_policy, grid_blocks, lds_load_pct, chunk_bytes,
                  direct_kib)


def count_plan(corpus_len: int, n_docs: int, *, count_bytes=8, per_doc=False, table_slots=0,
               tuning=None, word_bytes_cap=0) -> Plan:
    o = _opts(count_bytes, per_doc, table_slots, tuning, 0, 0, word_bytes_cap)
    p = Plan()
    st = lib().wc_count_plan(corpus_len, n_docs, ctypes.byref(o), ctypes.byref(p))
    if st != WC_OK:
        raise WcError(st, "wc_count_plan")
    return p


def count(corpus: torch.Tensor, offsets: Optional[torch.Tensor] = None, *, count_bytes: int = 8,
          per_doc: bool = False, table_slots: int = 0, tuning: Optional[Tuning] = None,
          debug_flags: int = 0, debug_hash_bits: int = 0, word_bytes_cap: int = 0,
          stream=None, regrow: bool = True, workspace: Optional[torch.Tensor] = None,
          debug_count_bias: int = 0, utf8: bool = False) -> Table:
    """Count the words of a device corpus (uint8) split into documents by offsets (int64).

    On a full table the call is repeated with twice the slots (regrow=True), and on an
    exported-word overflow with the reported byte count; other errors raise WcError.
    """
    _require_cuda(corpus, "corpus")
    if corpus.dtype != torch.uint8 or corpus.dim() != 1 or not corpus.is_contiguous():
        raise ValueError("corpus must be a contiguous 1-D uint8 tensor")
    n = corpus.numel()
    if offsets is None:
        offsets = torch.tensor([0, n], dtype=torch.int64, device=corpus.device)
    _require_cuda(offsets, "offsets")
    if offsets.dtype not in (torch.int64, torch.uint64) or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous int64 tensor")
    n_docs = offsets.numel() - 1
    if n_docs < 0:
        raise ValueError("offsets must hold at least one value")
    while True:
        o = _opts(count_bytes, per_doc, table_slots, tuning, debug_flags, debug_hash_bits,
                  word_bytes_cap, debug_count_bias, utf8)
        p = Plan()
        st = lib().wc_count_plan(n, n_docs, ctypes.byref(o), ctypes.byref(p))
        if st != WC_OK:
            raise WcError(st, "wc_count_plan")
        ws = workspace if (workspace is not None and workspace.numel() >= p.workspace_bytes) \
            else _alloc(p.workspace_bytes, corpus.device)
        res = Result()
        st = lib().wc_count(ctypes.c_void_p(corpus.data_ptr()), n,
                            ctypes.c_void_p(offsets.data_ptr()), n_docs, ctypes.byref(o),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(res),
                            _stream_handle(stream))
        if st == WC_ETABLEFULL and regrow:
            table_slots = 2 * int(p.table_slots)
            continue
        if st == WC_ENOMEM and regrow and per_doc:
            # per-document outputs or private tables ran out: grow what was short
            need_b = max(int(res.word_bytes), 3 * int(res.n_entries))
            grew = False
            if need_b > p.word_bytes_cap or int(res.n_entries) > p.max_entries:
                word_bytes_cap = need_b + need_b // 4 + 4096
                grew = True
            if int(res.table_slots) > p.table_slots:
                table_slots = 1 << (2 * int(res.table_slots) - 1).bit_length()
                grew = True
            if grew:
                continue
        if st == WC_ENOMEM and regrow and not per_doc and res.word_bytes > p.word_bytes_cap:
            word_bytes_cap = int(res.word_bytes)
            continue
        if st != WC_OK:
            raise WcError(st, "wc_count")
        return Table(res, ws)


def count_static(corpus: torch.Tensor, offsets: Optional[torch.Tensor] = None, *,
                 count_bytes: int = 8, table_slots: int = 0, tuning: Optional[Tuning] = None,
                 debug_flags: int = 0, debug_hash_bits: int = 0, word_bytes_cap: int = 0,
                 stream=None, regrow: bool = True) -> Table:
    """wc_count_static: count into one global table whose scratch is the library's static
    device array; only the output arrays are allocated here (one tensor). With regrow, a full
    table is counted again with twice the slots (up to the static limit of 2^20) and an
    exported-word overflow with the reported byte count; other errors raise WcError."""
    _require_cuda(corpus, "corpus")
    if corpus.dtype != torch.uint8 or corpus.dim() != 1 or not corpus.is_contiguous():
        raise ValueError("corpus must be a contiguous 1-D uint8 tensor")
    n = corpus.numel()
    if offsets is None:
        offsets = torch.tensor([0, n], dtype=torch.int64, device=corpus.device)
    _require_cuda(offsets, "offsets")
    n_docs = offsets.numel() - 1
    limit = 1 << 20  # the largest table the library's static scratch holds
    while True:
        o = _opts(count_bytes, False, table_slots, tuning, debug_flags, debug_hash_bits,
                  word_bytes_cap)
        p = Plan()
        st = lib().wc_count_plan(n, n_docs, ctypes.byref(o), ctypes.byref(p))
        if st != WC_OK:
            raise WcError(st, "wc_count_plan")
        max_e = min(int(p.table_slots), limit) if not table_slots else int(table_slots)
        wcap = int(p.word_bytes_cap)
        a = (8 * (max_e + 1) + 255) // 256 * 256
        b = (count_bytes * max_e + 255) // 256 * 256
        buf = _alloc(a + b + wcap, corpus.device)
        base = buf.data_ptr()
        res = Result()
        st = lib().wc_count_static(ctypes.c_void_p(corpus.data_ptr()), n,
                                   ctypes.c_void_p(offsets.data_ptr()), n_docs, ctypes.byref(o),
                                   ctypes.c_void_p(base), ctypes.c_void_p(base + a), max_e,
                                   ctypes.c_void_p(base + a + b), wcap, ctypes.byref(res),
                                   _stream_handle(stream))
        if st == WC_ETABLEFULL and regrow and max_e < limit:
            table_slots = min(2 * max_e, limit)
            continue
        if st == WC_ENOMEM and regrow and res.word_bytes > wcap:
            word_bytes_cap = int(res.word_bytes)
            continue
        if st != WC_OK:
            raise WcError(st, "wc_count_static")
        return Table(res, buf)


def count_host(text, offsets=None, *, piece_bytes: int = 256 << 20, count_bytes: int = 8,
               table_slots: int = 0, tuning: Optional[Tuning] = None, debug_flags: int = 0,
               utf8: bool = False, device="cuda", stream=None, regrow: bool = True,
               d_text: Optional[torch.Tensor] = None) -> Table:
    """Count a host corpus (numpy uint8 array, bytes, or a CPU uint8 tensor, ideally pinned)
    through wc_count_host: pieces are copied to the device while earlier pieces are counted.
    The device copy of the text (d_text, allocated when not given) is kept with the result."""
    if isinstance(text, torch.Tensor):
        if text.is_cuda or text.dtype != torch.uint8 or not text.is_contiguous():
            raise ValueError("text must be a contiguous host uint8 tensor")
        host_ptr, n, keep_host = text.data_ptr(), text.numel(), text
    else:
        buf = np.frombuffer(bytes(text), dtype=np.uint8) if isinstance(text, (bytes, bytearray)) \
            else np.ascontiguousarray(text, dtype=np.uint8)
        keep_host = buf if len(buf) else np.zeros(1, np.uint8)
        host_ptr, n = keep_host.ctypes.data, len(buf)
    off = np.ascontiguousarray([0, n] if offsets is None else offsets, dtype=np.uint64)
    n_docs = len(off) - 1
    if d_text is None:
        d_text = torch.empty(max(n, 1), dtype=torch.uint8, device=device)
    while True:
        o = _opts(count_bytes, False, table_slots, tuning, debug_flags, 0, 0, 0, utf8)
        p = Plan()
        st = lib().wc_count_host_plan(n, n_docs, ctypes.byref(o), piece_bytes, ctypes.byref(p))
        if st != WC_OK:
            raise WcError(st, "wc_count_host_plan")
        ws = _alloc(p.workspace_bytes, d_text.device)
        res = Result()
        st = lib().wc_count_host(ctypes.c_void_p(host_ptr), n, off.ctypes.data_as(ctypes.c_void_p),
                                 n_docs, ctypes.byref(o), piece_bytes,
                                 ctypes.c_void_p(d_text.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel(), ctypes.byref(res), _stream_handle(stream))
        if st == WC_ETABLEFULL and regrow:
            table_slots = 2 * int(p.table_slots)
            continue
        if st != WC_OK:
            raise WcError(st, "wc_count_host")
        return Table(res, ws, keep=(d_text, keep_host))


def sort_canonical(words: np.ndarray, word_offsets: np.ndarray, docs=None) -> np.ndarray:
    """wc_sort_canonical: the permutation that orders a host table by (document, word)."""
    o = np.ascontiguousarray(word_offsets, dtype=np.uint64)
    n = len(o) - 1
    w = np.ascontiguousarray(words, dtype=np.uint8)
    w = w if len(w) else np.zeros(1, np.uint8)
    d = None if docs is None else np.ascontiguousarray(docs, dtype=np.uint64)
    perm = np.zeros(max(n, 1), dtype=np.uint64)
    st = lib().wc_sort_canonical(n, o.ctypes.data, w.ctypes.data,
                                 d.ctypes.data if d is not None else None, perm.ctypes.data)
    if st != WC_OK:
        raise WcError(st, "wc_sort_canonical")
    return perm[:n].astype(np.int64)


def _result_array(tables: Sequence[Table]):
    arr = (ctypes.POINTER(Result) * len(tables))(*[ctypes.pointer(t.res) for t in tables])
    return arr


def merge(tables: Sequence[Table], *, count_bytes: int = 8, table_slots: int = 0, stream=None,
          debug_flags: int = 0) -> Table:
    """Pointwise sum of word tables over the union of their words (one global table)."""
    if not tables:
        raise ValueError("merge needs at least one table")
    dev = tables[0].workspace.device
    while True:
        o = _opts(count_bytes, False, table_slots, None, debug_flags, 0, 0)
        arr = _result_array(tables)
        p = Plan()
        st = lib().wc_merge_plan(arr, len(tables), ctypes.byref(o), ctypes.byref(p))
        if st != WC_OK:
            raise WcError(st, "wc_merge_plan")
        ws = _alloc(p.workspace_bytes, dev)
        res = Result()
        st = lib().wc_merge(arr, len(tables), ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()),
                            ws.numel(), ctypes.byref(res), _stream_handle(stream))
        if st == WC_ETABLEFULL:
            table_slots = 2 * int(p.table_slots)
            continue
        if st != WC_OK:
            raise WcError(st, "wc_merge")
        return Table(res, ws)


def merge_dense(per_doc: Table, *, count_bytes: int = 8, stream=None, debug_flags: int = 0,
                debug_count_bias: int = 0) -> Table:
    """The paper's reduce: per-document counts as a zero-padded words x documents matrix,
    summed by rows (wc_merge_dense). The result equals merge([per_doc])."""
    if per_doc.docs() is None:
        raise ValueError("merge_dense needs a per-document table")
    dev = per_doc.workspace.device
    n, d = per_doc.n_entries, max(int(per_doc.res.n_docs), 1)
    # plan for the upper bound when that matrix is small; else learn the rows first
    rows = n if n * d * 4 <= (1 << 30) else 1
    o = _opts(count_bytes, False, 0, None, debug_flags, 0, 0, debug_count_bias)
    for _ in range(2):
        need = ctypes.c_uint64()
        st = lib().wc_merge_dense_plan(ctypes.byref(per_doc.res), ctypes.byref(o), rows,
                                       ctypes.byref(need))
        if st != WC_OK:
            raise WcError(st, "wc_merge_dense_plan")
        ws = _alloc(need.value, dev)
        res = Result()
        st = lib().wc_merge_dense(ctypes.byref(per_doc.res), ctypes.byref(o),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(res),
                                  _stream_handle(stream))
        if st == WC_ENOMEM and res.n_entries > rows:
            rows = int(res.n_entries)
            continue
        if st != WC_OK:
            raise WcError(st, "wc_merge_dense")
        return Table(res, ws)
    raise WcError(WC_ENOMEM, "wc_merge_dense")


@dataclass
class TopK:
    words: list       # per corpus: list of bytes
    n_c: list         # per corpus: int64 arrays
    n_rest: list
    score: list       # per corpus: float64 arrays
    vocab_size: int


def topk_ratio(tables: Sequence[Table], k: int, min_count: int = 1, stream=None) -> TopK:
    """Per-corpus top-k distinctive words (see wc_topk in include/wc.h)."""
    C = len(tables)
    dev = tables[0].workspace.device
    arr = _result_array(tables)
    need = ctypes.c_uint64()
    st = lib().wc_topk_ratio_plan(arr, C, k, ctypes.byref(need))
    if st != WC_OK:
        raise WcError(st, "wc_topk_ratio_plan")
    ws = _alloc(need.value, dev)
    out = TopKStruct()
    st = lib().wc_topk_ratio(arr, C, k, min_count, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                             ctypes.byref(out), _stream_handle(stream))
    if st != WC_OK:
        raise WcError(st, "wc_topk_ratio")
    base = ws.data_ptr()

    def view(ptr, nbytes, dtype):
        off = int(ptr) - base
        return ws[off:off + nbytes].view(dtype) if nbytes else torch.empty(0, dtype=dtype)

    rows = C * k
    woff = view(out.d_word_offsets, 8 * (rows + 1), torch.int64).cpu().numpy()
    wbytes = view(out.d_words, int(out.word_bytes), torch.uint8).cpu().numpy().tobytes()
    nc = view(out.d_n_c, 8 * rows, torch.int64).cpu().numpy()
    nr = view(out.d_n_rest, 8 * rows, torch.int64).cpu().numpy()
    sc = view(out.d_score, 8 * rows, torch.float64).cpu().numpy()
    words, ncs, nrs, scs = [], [], [], []
    for c in range(C):
        r = int(out.n_rows[c])
        b = c * k
        words.append([wbytes[woff[b + j]:woff[b + j + 1]] for j in range(r)])
        ncs.append(nc[b:b + r].copy())
        nrs.append(nr[b:b + r].copy())
        scs.append(sc[b:b + r].copy())
    return TopK(words, ncs, nrs, scs, int(out.vocab_size))


def hash_words(words: Sequence[bytes], device="cuda") -> list:
    """FNV-1a 64 of each (folded) byte string, computed by the library's device function."""
    blob = b"".join(words)
    off = np.zeros(len(words) + 1, dtype=np.int64)
    np.cumsum([len(w) for w in words], out=off[1:])
    d_b = torch.tensor(list(blob) or [0], dtype=torch.uint8, device=device)
    d_o = torch.from_numpy(off).to(device)
    d_out = torch.zeros(max(len(words), 1), dtype=torch.int64, device=device)
    st = lib().wc_hash_words(ctypes.c_void_p(d_b.data_ptr()), ctypes.c_void_p(d_o.data_ptr()),
                             len(words), ctypes.c_void_p(d_out.data_ptr()),
                             _stream_handle(None))
    if st != WC_OK:
        raise WcError(st, "wc_hash_words")
    return [int(x) & 0xFFFFFFFFFFFFFFFF for x in d_out[:len(words)].cpu().tolist()]


class FoldSum:
    """Section 4.2's float map-reduce (wc_fold_sum) with its workspace and output held on the
    device, for repeated calls: run(n) enqueues the sum of terms 1..n on the stream and returns
    the one-element float64 device tensor it writes."""

    def __init__(self, kind: int, max_n: int, device="cuda"):
        need = ctypes.c_uint64()
        st = lib().wc_fold_sum_plan(max_n, ctypes.byref(need))
        if st != WC_OK:
            raise WcError(st, "wc_fold_sum_plan")
        self.kind = kind
        self.max_n = max_n
        self.workspace = _alloc(need.value, device)
        self.out = torch.zeros(1, dtype=torch.float64, device=device)

    def run(self, n: int, stream=None) -> torch.Tensor:
        if n > self.max_n:
            raise ValueError("n above max_n")
        st = lib().wc_fold_sum(self.kind, n, ctypes.c_void_p(self.out.data_ptr()),
                               ctypes.c_void_p(self.workspace.data_ptr()),
                               self.workspace.numel(), _stream_handle(stream))
        if st != WC_OK:
            raise WcError(st, "wc_fold_sum")
        return self.out


def fold_sum(kind: int, n: int, device="cuda") -> float:
    """Sum over i = 1..n of sqrt(i) (WC_FOLD_SQRT) or (-1)^(i+1)/i (WC_FOLD_ALT_HARMONIC)."""
    f = FoldSum(kind, n, device)
    out = f.run(n)
    torch.cuda.current_stream().synchronize()
    return float(out.cpu().item())


def output_sizes(corpus: torch.Tensor, offsets: torch.Tensor, *, per_doc: bool = True,
                 count_bytes: int = 4, stream=None) -> dict:
    """Output sizes (word_bytes_cap, table_slots) for fixed-capacity calls (Batch, autotune)
    on corpora like this one, from one count of it: the output words do not depend on the
    launch tuning and get a quarter of headroom; the private-table arena does, and gets twice
    what this count used (rounded up to a power of two)."""
    t = count(corpus, offsets, count_bytes=count_bytes, per_doc=per_doc, stream=stream)
    wb = int(t.res.word_bytes)
    slots = 1 << (2 * int(t.res.table_slots) - 1).bit_length() if per_doc else 0
    return {"word_bytes_cap": wb + wb // 4 + 4096, "table_slots": slots}


class Batch:
    """Per-document counting of whole corpora with one captured HIP graph (see wc_batch_*).

    Output capacity is fixed at creation: word_bytes_cap and table_slots (0 = defaults sized
    for natural text) bound the words and private tables of every run; a run beyond them
    raises WcError(WC_ENOMEM). output_sizes() derives both from a representative corpus."""

    def __init__(self, max_docs: int, max_bytes: int, *, count_bytes: int = 4,
                 tuning: Optional[Tuning] = None, word_bytes_cap: int = 0, table_slots: int = 0,
                 device="cuda", debug_hash_bits: int = 0):
        self._opts = _opts(count_bytes, True, table_slots, tuning, 0, debug_hash_bits,
                           word_bytes_cap)
        self._tuning = tuning  # keep the structure alive
        need = ctypes.c_uint64()
        st = lib().wc_batch_plan(ctypes.byref(self._opts), max_docs, max_bytes, ctypes.byref(need))
        if st != WC_OK:
            raise WcError(st, "wc_batch_plan")
        self.workspace = _alloc(need.value, device)
        h = ctypes.c_void_p()
        st = lib().wc_batch_create(ctypes.byref(self._opts), max_docs, max_bytes,
                                   ctypes.c_void_p(self.workspace.data_ptr()),
                                   self.workspace.numel(), ctypes.byref(h))
        if st != WC_OK:
            raise WcError(st, "wc_batch_create")
        self._h = h

    def run(self, corpus: torch.Tensor, offsets: torch.Tensor, stream=None) -> Table:
        _require_cuda(corpus, "corpus")
        _require_cuda(offsets, "offsets")
        res = Result()
        st = lib().wc_batch_run(self._h, ctypes.c_void_p(corpus.data_ptr()), corpus.numel(),
                                ctypes.c_void_p(offsets.data_ptr()), offsets.numel() - 1,
                                ctypes.byref(res), _stream_handle(stream))
        if st != WC_OK:
            raise WcError(st, "wc_batch_run")
        return Table(res, self.workspace)

    def close(self):
        if getattr(self, "_h", None):
            lib().wc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def result_to_dict(res: Result) -> dict:
    """{word: count} of a table anywhere in device memory (copied with wc_table_to_host)."""
    n = int(res.n_entries)
    off = np.zeros(n + 1, dtype=np.uint64)
    words = np.zeros(max(int(res.word_bytes), 1), dtype=np.uint8)
    cnt = np.zeros(max(n, 1), dtype=np.int32 if res.count_bytes == 4 else np.int64)
    st = lib().wc_table_to_host(ctypes.byref(res), off.ctypes.data_as(ctypes.c_void_p),
                                words.ctypes.data_as(ctypes.c_void_p),
                                cnt.ctypes.data_as(ctypes.c_void_p))
    if st != WC_OK:
        raise WcError(st, "wc_table_to_host")
    off = off - off[0]
    wb = words.tobytes()
    return {wb[int(off[e]):int(off[e + 1])]: int(cnt[e]) for e in range(n)}


class Server:
    """Request server (see wc_server_* in include/wc.h): counts submitted texts on several
    streams, keeps the tables resident, answers merge queries."""

    def __init__(self, mem_budget: int, max_streams: int = 4, device: int = 0):
        h = ctypes.c_void_p()
        st = lib().wc_server_create(device, mem_budget, max_streams, ctypes.byref(h))
        if st != WC_OK:
            raise WcError(st, "wc_server_create")
        self._h = h
        self._keep = {}  # texts the server reads in place, until their request is released

    def submit(self, text, offsets=None, *, count_bytes: int = 8, in_place: bool = False) -> int:
        """text: bytes / uint8 numpy array / CPU uint8 tensor (host: copied at submission, or
        with in_place=True read in place and kept alive here until released; a pinned tensor
        then goes to the device without staging), or a CUDA uint8 tensor (kept alive likewise)."""
        if isinstance(text, torch.Tensor) and text.is_cuda:
            n, ptr, keep, where = text.numel(), text.data_ptr(), text, 1
        elif isinstance(text, torch.Tensor):
            if text.dtype != torch.uint8 or not text.is_contiguous():
                raise ValueError("text must be a contiguous uint8 tensor")
            n, keep = text.numel(), text
            ptr = text.data_ptr() if n else np.zeros(1, np.uint8).ctypes.data
            where = 2 if in_place else 0
        else:
            buf = np.frombuffer(bytes(text), dtype=np.uint8) if isinstance(text, (bytes, bytearray)) \
                else np.ascontiguousarray(text, dtype=np.uint8)
            n = len(buf)
            keep = buf if n else np.zeros(1, np.uint8)
            ptr = keep.ctypes.data
            where = 2 if in_place else 0
        off = np.ascontiguousarray([0, n] if offsets is None else offsets, dtype=np.uint64)
        o = _opts(count_bytes, False, 0, None, 0, 0, 0)
        rid = ctypes.c_uint64()
        st = lib().wc_server_submit(self._h, ctypes.c_void_p(ptr), n,
                                    off.ctypes.data_as(ctypes.c_void_p), len(off) - 1, where,
                                    ctypes.byref(o), ctypes.byref(rid))
        if st != WC_OK:
            raise WcError(st, "wc_server_submit")
        if where:
            self._keep[int(rid.value)] = keep
        return int(rid.value)

    def poll(self, rid: int):
        res = Result()
        st = lib().wc_server_poll(self._h, rid, ctypes.byref(res))
        return st, res

    def wait(self, rid: int) -> Result:
        res = Result()
        st = lib().wc_server_wait(self._h, rid, ctypes.byref(res))
        if st != WC_OK:
            raise WcError(st, "wc_server_wait")
        return res

    def times(self, rid: int):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        lib().wc_server_times(self._h, rid, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return a.value, b.value, c.value

    def merge(self, ids, *, count_bytes: int = 8) -> int:
        arr = (ctypes.c_uint64 * len(ids))(*ids)
        o = _opts(count_bytes, False, 0, None, 0, 0, 0)
        rid = ctypes.c_uint64()
        st = lib().wc_server_merge(self._h, arr, len(ids), ctypes.byref(o), ctypes.byref(rid))
        if st != WC_OK:
            raise WcError(st, "wc_server_merge")
        return int(rid.value)

    def release(self, rid: int):
        lib().wc_server_release(self._h, rid)
        self._keep.pop(int(rid), None)

    def launches(self) -> int:
        return int(lib().wc_server_launches(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().wc_server_destroy(self._h)
            self._h = None
            self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _cache_file(path: Optional[str]) -> str:
    if path:
        return path
    env = os.environ.get("WC_AUTOTUNE_CACHE")
    if env:
        return env
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "wc_mi355x", "autotune.json")


def autotune(corpus: torch.Tensor, offsets: torch.Tensor, *, per_doc: bool = True,
             count_bytes: int = 4, cache_path: Optional[str] = None, use_cache: bool = True,
             stream=None) -> Tuning:
    """Pick a tuning for corpora like `corpus` by timing the library's candidate grid on it
    (wc_autotune), caching the choice in a JSON file keyed by device, mode and sample size."""
    _require_cuda(corpus, "corpus")
    props = torch.cuda.get_device_properties(corpus.device)
    size_class = int(corpus.numel()).bit_length()
    key = (f"{props.name}|{props.multi_processor_count}|{'doc' if per_doc else 'global'}|"
           f"{size_class}|direct")
    path = _cache_file(cache_path)
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return Tuning(*cache[key]["tuning"])
    n_docs = offsets.numel() - 1
    # grid points that still run out of room are skipped by the library
    sz = output_sizes(corpus, offsets, per_doc=per_doc, count_bytes=count_bytes, stream=stream)
    o = _opts(count_bytes, per_doc, sz["table_slots"] if per_doc else 0, None, 0, 0,
              sz["word_bytes_cap"])
    need = ctypes.c_uint64()
    st = lib().wc_autotune_plan(corpus.numel(), n_docs, ctypes.byref(o), ctypes.byref(need))
    if st != WC_OK:
        raise WcError(st, "wc_autotune_plan")
    ws = _alloc(need.value, corpus.device)
    best = Tuning()
    ms = ctypes.c_float()
    st = lib().wc_autotune(ctypes.c_void_p(corpus.data_ptr()), corpus.numel(),
                           ctypes.c_void_p(offsets.data_ptr()), n_docs, ctypes.byref(o),
                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(best),
                           ctypes.byref(ms), _stream_handle(stream))
    if st != WC_OK:
        raise WcError(st, "wc_autotune")
    if use_cache:
        cache[key] = {"tuning": [best.stage_bytes, best.lds_entries, best.flush_policy,
                                 best.grid_blocks, best.lds_load_pct, best.chunk_bytes,
                                 best.direct_kib],
                      "ms": ms.value}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return best
