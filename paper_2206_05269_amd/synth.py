"""Seeded synthetic corpora for the word counter.

This module draws text; it holds none of the counter's arithmetic (no tokenising, folding,
hashing or counting of text). Both the GPU path and the CPU oracle are fed the bytes it writes.

Recipe (the stand-in for the paper's presidential speeches, which are not redistributed with
the paper; Section 3 and Section 4.3 describe that data only in prose):

* Vocabulary: N distinct words; each word has a length drawn uniformly from 1..L and letters
  drawn uniformly from a-z. A word that repeats an earlier one is redrawn (length and letters),
  so the shortest lengths saturate (26 one-letter words, 676 two-letter words) and the length
  distribution is slightly non-uniform there. Rank = order of first draw, so rank and length are
  independent.
* Token ranks: finite Zipf, p_k proportional to k^-s for k = 1..N (optionally with some words
  re-weighted), drawn by inverse CDF.
* After every token one separator: space 0.8, newline 0.1, and each of , . ; ! ? " with 0.1/6.
* With probability 0.05 the first letter of a token is upper-cased.
* A document is filled token by token (a token is its word plus its separator) until the next
  token would not fit; the rest of the document is padded with spaces, so its last byte is
  always a delimiter.

Because vocabulary words are distinct runs of a-z and neither separators nor capitalisation
can join or split a word, the exact word table of a generated corpus is the histogram of the
ranks drawn (``expected``). That histogram is independent of any tokeniser.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

SEED_BASE = 2206052690

SEPARATORS = b" \n,.;!?\""
# cumulative probabilities of SEPARATORS above
_SEP_P = np.array([0.8, 0.1] + [0.1 / 6] * 6)

KiB = 1024
MiB = 1024 * 1024
GiB = 1024 * MiB


@dataclass
class Workload:
    """One named synthetic workload: vocabulary, Zipf law and document sizes."""
    name: str
    index: int
    vocab: int
    max_len: int
    zipf_s: float
    kind: str                      # "docs", "stream", "corpora"
    n_docs: int = 1
    doc_size: Optional[int] = None  # fixed size (docs / stream)
    lognormal: Optional[tuple] = None  # (median, sigma, lo, hi)
    n_corpora: int = 1
    reweight: int = 0              # words re-weighted per corpus
    reweight_factor: float = 1.0
    count_bytes: int = 4
    per_doc: bool = False
    table_slots: int = 0

    @property
    def seed(self) -> int:
        return SEED_BASE + self.index


WORKLOADS = {
    "plain-1MB": Workload("plain-1MB", 0, vocab=5000, max_len=12, zipf_s=1.1, kind="docs",
                          n_docs=4, doc_size=250_000, count_bytes=4),
    "corpora-4x2000": Workload("corpora-4x2000", 1, vocab=50_000, max_len=12, zipf_s=1.05,
                               kind="corpora", n_docs=2000, n_corpora=4,
                               lognormal=(8 * KiB, 1.0, 2 * KiB, 20 * KiB),
                               reweight=200, reweight_factor=5.0, count_bytes=4),
    "stream-8GiB": Workload("stream-8GiB", 2, vocab=1_000_000, max_len=16, zipf_s=1.0,
                            kind="stream", n_docs=1, doc_size=8 * GiB, count_bytes=8,
                            table_slots=1 << 22),
    "batched-100k": Workload("batched-100k", 3, vocab=200_000, max_len=12, zipf_s=1.1,
                             kind="docs", n_docs=100_000,
                             lognormal=(16 * KiB, 1.0, 200, 1 * MiB), count_bytes=4,
                             per_doc=True, table_slots=1 << 28),
    "serving": Workload("serving", 4, vocab=500_000, max_len=12, zipf_s=1.05, kind="docs",
                        n_docs=10_000, lognormal=(256 * KiB, 2.0, 1 * KiB, 64 * MiB),
                        count_bytes=8),
}


# ----------------------------------------------------------------------------------------
# vocabulary and distributions (numpy, host; deterministic per seed)
# ----------------------------------------------------------------------------------------

def make_vocab(n: int, max_len: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Return (words uint8[n, max_len] zero padded, lens int64[n]) of n distinct a-z words."""
    if n > sum(26 ** k for k in range(1, max_len + 1)):
        raise ValueError("vocabulary larger than the number of distinct words")
    rng = np.random.default_rng(seed)
    mats, lens_all = [], []
    have = 0
    seen_keys = None
    while have < n:
        m = int((n - have) * 1.25) + 64
        lens = rng.integers(1, max_len + 1, size=m)
        letters = rng.integers(ord("a"), ord("z") + 1, size=(m, max_len), dtype=np.uint8)
        letters[np.arange(max_len)[None, :] >= lens[:, None]] = 0
        mats.append(letters)
        lens_all.append(lens)
        allm = np.concatenate(mats)
        keys = np.ascontiguousarray(allm).view(np.dtype((np.void, max_len))).ravel()
        _, first = np.unique(keys, return_index=True)
        first.sort()
        have = len(first)
        seen_keys = first
    allm = np.concatenate(mats)
    alll = np.concatenate(lens_all)
    keep = seen_keys[:n]
    return np.ascontiguousarray(allm[keep]), alll[keep].astype(np.int64)


def zipf_probs(n: int, s: float, boost: Optional[np.ndarray] = None, factor: float = 1.0) -> np.ndarray:
    """p_k proportional to k^-s over k = 1..n, ranks in boost multiplied by factor."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    if boost is not None and len(boost):
        w[boost] *= factor
    return w / w.sum()


def lognormal_sizes(n: int, median: float, sigma: float, lo: int, hi: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = np.exp(rng.normal(math.log(median), sigma, size=n))
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


# ----------------------------------------------------------------------------------------
# token drawing and byte writing (torch; runs on CPU or GPU)
# ----------------------------------------------------------------------------------------

class _Drawer:
    def __init__(self, vocab: np.ndarray, lens: np.ndarray, probs: np.ndarray, device, gen):
        self.device = torch.device(device)
        self.gen = gen
        self.vocab = torch.from_numpy(vocab).to(self.device)             # [N, L] uint8
        self.vlens = torch.from_numpy(lens).to(self.device)              # [N] int64
        cdf = np.cumsum(probs)
        cdf[-1] = 1.0
        self.cdf = torch.from_numpy(cdf).to(self.device)
        self.n = len(lens)
        self.L = vocab.shape[1]
        sep_cdf = np.cumsum(_SEP_P)
        sep_cdf[-1] = 1.0
        self.sep_cdf = torch.from_numpy(sep_cdf).to(self.device)
        self.sep_bytes = torch.tensor(list(SEPARATORS), dtype=torch.uint8, device=self.device)

    def draw(self, m: int):
        u = torch.rand(m, generator=self.gen, device=self.device, dtype=torch.float64)
        r = torch.searchsorted(self.cdf, u, right=True).clamp_(max=self.n - 1)
        cu = torch.rand(m, generator=self.gen, device=self.device, dtype=torch.float64)
        su = torch.rand(m, generator=self.gen, device=self.device, dtype=torch.float64)
        sep = torch.searchsorted(self.sep_cdf, su, right=True).clamp_(max=len(SEPARATORS) - 1)
        return r, cu < 0.05, sep

    def write(self, out: torch.Tensor, pos: torch.Tensor, r: torch.Tensor, cap: torch.Tensor,
              sep: torch.Tensor):
        """Write tokens (word + separator) at absolute positions pos of out (uint8)."""
        lens = self.vlens[r]
        for i in range(self.L):
            m = lens > i
            if not bool(m.any()):
                break
            b = self.vocab[r[m], i]
            if i == 0:
                b = torch.where(cap[m], b - 32, b)
            out[pos[m] + i] = b
        out[pos + lens] = self.sep_bytes[sep]


def _device_gen(device, seed: int):
    g = torch.Generator(device=torch.device(device))
    g.manual_seed(seed)
    return g


@dataclass
class Corpus:
    text: torch.Tensor          # uint8[B]
    offsets: torch.Tensor       # int64[n_docs + 1]
    expected: torch.Tensor      # int64[N]: histogram of drawn ranks (all documents)
    vocab: np.ndarray           # uint8[N, L]
    vocab_lens: np.ndarray      # int64[N]
    n_tokens: int
    doc_expected: Optional[list] = None  # per-document histograms when asked for
    extra: dict = field(default_factory=dict)

    def expected_table(self) -> dict:
        """{word bytes: count} from the rank histogram."""
        cnt = self.expected.cpu().numpy()
        nz = np.nonzero(cnt)[0]
        return {bytes(self.vocab[k, :self.vocab_lens[k]]): int(cnt[k]) for k in nz}


def gen_docs(sizes, vocab, vlens, probs, seed: int, device="cpu", per_doc_truth=False,
             max_tokens_per_pass: int = 1 << 25, pair_truth=False) -> Corpus:
    """Documents of the given byte sizes, filled with Zipf tokens and padded with spaces.

    pair_truth: also return, in extra["pair_keys"] / extra["pair_counts"], the sorted distinct
    keys document * N + rank of the drawn tokens and how often each was drawn (the exact
    per-document tables, for corpora too large for one histogram per document)."""
    device = torch.device(device)
    sizes = np.asarray(sizes, dtype=np.int64)
    n_docs = len(sizes)
    offsets = np.zeros(n_docs + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    total = int(offsets[-1])
    text = torch.full((total,), 0x20, dtype=torch.uint8, device=device)
    gen = _device_gen(device, seed)
    dr = _Drawer(vocab, vlens, probs, device, gen)
    mean_tok = float((probs * (vlens + 1)).sum())
    budget = np.ceil(sizes / mean_tok * 1.5).astype(np.int64) + 32
    budget = np.minimum(budget, sizes // 2 + 1)
    expected = torch.zeros(dr.n, dtype=torch.int64, device=device)
    doc_truth = [] if per_doc_truth else None
    pair_keys, pair_counts = [], []
    n_tok = 0
    d0 = 0
    while d0 < n_docs:
        # group documents so that one pass draws at most max_tokens_per_pass tokens
        cum = np.cumsum(budget[d0:])
        d1 = d0 + max(1, int(np.searchsorted(cum, max_tokens_per_pass, side="right")))
        d1 = min(d1, n_docs)
        bud = budget[d0:d1]
        m = int(bud.sum())
        r, cap, sep = dr.draw(m)
        z = dr.vlens[r] + 1
        Z = torch.cumsum(z, 0)
        seg_start = np.zeros(d1 - d0, dtype=np.int64)
        np.cumsum(bud[:-1], out=seg_start[1:])
        seg_start_t = torch.from_numpy(seg_start).to(device)
        base = torch.where(seg_start_t > 0, Z[(seg_start_t - 1).clamp(min=0)],
                           torch.zeros_like(seg_start_t))
        lim = base + torch.from_numpy(sizes[d0:d1]).to(device)
        n_fit = torch.searchsorted(Z, lim, right=True) - seg_start_t
        n_fit = torch.minimum(n_fit, torch.from_numpy(bud).to(device))
        if bool((n_fit >= torch.from_numpy(bud).to(device)).any()):
            # a token is at least 2 bytes, so a budget of size//2+1 is never used up; any
            # other budget that is used up may have cut a document short
            raise RuntimeError("token budget exhausted; raise the budget factor")
        doc_of = torch.repeat_interleave(torch.arange(d1 - d0, device=device),
                                         torch.from_numpy(bud).to(device))
        idx_in = torch.arange(m, device=device) - seg_start_t[doc_of]
        keep = idx_in < n_fit[doc_of]
        pos = torch.from_numpy(offsets[d0:d1]).to(device)[doc_of] + (Z - z) - base[doc_of]
        rk, ck, sk, pk = r[keep], cap[keep], sep[keep], pos[keep]
        dr.write(text, pk, rk, ck, sk)
        expected += torch.bincount(rk, minlength=dr.n)
        if per_doc_truth:
            dk = doc_of[keep]
            for j in range(d1 - d0):
                doc_truth.append(torch.bincount(rk[dk == j], minlength=dr.n).cpu())
        if pair_truth:
            # documents of one pass never appear in another, so the keys stay sorted overall
            u, n_u = torch.unique((doc_of[keep] + d0) * dr.n + rk, return_counts=True)
            pair_keys.append(u)
            pair_counts.append(n_u)
        n_tok += int(keep.sum())
        d0 = d1
    cor = Corpus(text, torch.from_numpy(offsets).to(device), expected, vocab, vlens, n_tok,
                 doc_truth)
    if pair_truth:
        cor.extra["pair_keys"] = torch.cat(pair_keys) if pair_keys else \
            torch.empty(0, dtype=torch.int64, device=device)
        cor.extra["pair_counts"] = torch.cat(pair_counts) if pair_counts else \
            torch.empty(0, dtype=torch.int64, device=device)
    return cor


def gen_stream(size: int, vocab, vlens, probs, seed: int, device="cpu",
               piece_tokens: int = 1 << 26, progress=None) -> Corpus:
    """One document of `size` bytes, generated in pieces of piece_tokens tokens."""
    device = torch.device(device)
    text = torch.full((size,), 0x20, dtype=torch.uint8, device=device)
    gen = _device_gen(device, seed)
    dr = _Drawer(vocab, vlens, probs, device, gen)
    expected = torch.zeros(dr.n, dtype=torch.int64, device=device)
    cursor = 0
    n_tok = 0
    mean_tok = float((probs * (vlens + 1)).sum())
    while True:
        want = min(piece_tokens, int((size - cursor) / mean_tok * 1.1) + 4096)
        r, cap, sep = dr.draw(want)
        z = dr.vlens[r] + 1
        Z = torch.cumsum(z, 0) + cursor
        keep_n = int(torch.searchsorted(Z, torch.tensor([size], device=device), right=True)[0])
        done = keep_n < want
        r, cap, sep, Z, z = r[:keep_n], cap[:keep_n], sep[:keep_n], Z[:keep_n], z[:keep_n]
        dr.write(text, Z - z, r, cap, sep)
        expected += torch.bincount(r, minlength=dr.n)
        n_tok += keep_n
        if keep_n:
            cursor = int(Z[-1])
        if progress:
            progress(cursor, size)
        if done:
            break
    offsets = torch.tensor([0, size], dtype=torch.int64, device=device)
    return Corpus(text, offsets, expected, vocab, vlens, n_tok)


def doc_sizes(w: Workload, scale: float = 1.0) -> np.ndarray:
    n = max(1, int(round(w.n_docs * scale))) if w.kind != "stream" else 1
    if w.lognormal is not None:
        med, sig, lo, hi = w.lognormal
        return lognormal_sizes(n, med, sig, lo, hi, w.seed + 7919)
    size = w.doc_size if w.kind != "stream" else max(64, int(w.doc_size * scale))
    return np.full(n, size, dtype=np.int64)


def generate(name: str, device="cpu", scale: float = 1.0, per_doc_truth=False, progress=None,
             pair_truth=False):
    """Generate a named workload. scale < 1 shrinks the document count (or the stream size).

    Returns a Corpus, or for "corpora" workloads a list of one Corpus per corpus.
    """
    w = WORKLOADS[name]
    vocab, vlens = make_vocab(w.vocab, w.max_len, w.seed)
    if w.kind == "stream":
        size = max(64, int(w.doc_size * scale))
        probs = zipf_probs(w.vocab, w.zipf_s)
        return gen_stream(size, vocab, vlens, probs, w.seed + 1, device, progress=progress)
    if w.kind == "corpora":
        out = []
        rng = np.random.default_rng(w.seed + 104729)
        for c in range(w.n_corpora):
            boost = rng.choice(w.vocab, size=w.reweight, replace=False)
            probs = zipf_probs(w.vocab, w.zipf_s, boost, w.reweight_factor)
            n = max(1, int(round(w.n_docs * scale)))
            sizes = lognormal_sizes(n, *w.lognormal, seed=w.seed + 7919 + c)
            cor = gen_docs(sizes, vocab, vlens, probs, w.seed + 1 + c, device, per_doc_truth)
            cor.extra["boosted"] = np.sort(boost)
            out.append(cor)
        return out
    sizes = doc_sizes(w, scale)
    probs = zipf_probs(w.vocab, w.zipf_s)
    return gen_docs(sizes, vocab, vlens, probs, w.seed + 1, device, per_doc_truth,
                    pair_truth=pair_truth)


def random_text(n_bytes: int, seed: int, alphabet: bytes = b"aZ0' ,\x80\n") -> bytes:
    """Uniform random bytes over a small alphabet (for brute-force tokeniser checks)."""
    rng = np.random.default_rng(seed)
    a = np.frombuffer(alphabet, dtype=np.uint8)
    return a[rng.integers(0, len(a), size=n_bytes)].tobytes()


def random_splits(n_bytes: int, n_docs: int, seed: int) -> np.ndarray:
    """Nondecreasing offsets [0, ..., n_bytes] splitting n_bytes into n_docs documents."""
    rng = np.random.default_rng(seed)
    cuts = np.sort(rng.integers(0, n_bytes + 1, size=max(0, n_docs - 1)))
    return np.concatenate([[0], cuts, [n_bytes]]).astype(np.int64)
