"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit for bit.

Counts are integers, so the bar is exact equality of the (word, count) tables and of the token
totals. Inputs cover the paper's examples, brute-force alphabets, ragged stage and chunk
boundaries, misaligned buffers, long words, forced hash collisions, a table that must grow,
every tuning point, and the synthetic workloads (full size where the oracle's answer is known
from the generator's rank histogram).
"""
import collections
import itertools
import json
import os
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2206_05269_amd import synth
from paper_2206_05269_amd import wc

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(text: bytes | np.ndarray, offsets=None):
    a = np.frombuffer(text, dtype=np.uint8) if isinstance(text, (bytes, bytearray)) else text
    t = torch.from_numpy(np.ascontiguousarray(a).copy()).to(DEV) if len(a) else \
        torch.empty(0, dtype=torch.uint8, device=DEV)
    if offsets is None:
        offsets = [0, len(a)]
    o = torch.tensor(np.asarray(offsets, dtype=np.int64), device=DEV)
    return t, o


def gpu_count(text, offsets=None, **kw):
    t, o = to_dev(text, offsets)
    return wc.count(t, o, **kw)


def check(text, offsets=None, per_doc=False, **kw):
    """Count on the GPU and on the oracle; tables and totals must be identical."""
    want = oracle.count(text, offsets, per_doc=per_doc)
    got = gpu_count(text, offsets, per_doc=per_doc, **kw)
    assert got.total_tokens == want.total
    g = got.as_dict()
    w = want.as_dict()
    if g != w:
        missing = [k for k in w if k not in g][:5]
        extra = [k for k in g if k not in w][:5]
        wrong = [(k, g[k], w[k]) for k in w if k in g and g[k] != w[k]][:5]
        raise AssertionError(f"mismatch: missing {missing} extra {extra} wrong {wrong}")
    if per_doc:
        check_doc_layout(got, len(offsets) - 1)
    return got


def check_doc_layout(got, n_docs):
    """Each document's entries are the doc_len[d] entries from doc_ptr[d]; they tile the
    output exactly once; d_docs agrees; the word offsets are a CSR over the whole output."""
    dp = got.doc_ptr().cpu().numpy()
    dl = got.doc_len().cpu().numpy()
    docs = got.docs().cpu().numpy()
    n = got.n_entries
    assert len(dp) == n_docs and len(dl) == n_docs
    assert int(dl.sum()) == n
    cover = np.zeros(n + 1, dtype=np.int64)
    nz = dl > 0
    np.add.at(cover, dp[nz], 1)
    np.add.at(cover, dp[nz] + dl[nz], -1)
    assert (np.cumsum(cover)[:n] == 1).all()
    want_docs = np.repeat(np.arange(n_docs)[nz], dl[nz])
    order = np.repeat(dp[nz], dl[nz]) + (np.arange(n) - np.repeat(np.cumsum(dl[nz]) - dl[nz], dl[nz]))
    assert (docs[order] == want_docs).all()
    wo = got.word_offsets().cpu().numpy()
    assert wo[0] == 0 and (np.diff(wo) > 0).all() and wo[-1] == got.res.word_bytes


PATHS = {"direct": wc.WC_DEBUG_DIRECT, "spill": wc.WC_DEBUG_SPILL}


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def join_docs(docs):
    text = b"".join(docs)
    off = np.zeros(len(docs) + 1, dtype=np.int64)
    np.cumsum([len(d) for d in docs], out=off[1:])
    return text, off


# ------------------------------------------------------------------------------------------
# the paper's examples
# ------------------------------------------------------------------------------------------

def test_section2_worked_example():
    g = golden("section2_worked_example.json")
    text, off = join_docs([d.encode() for d in g["docs"]])
    got = check(text, off, count_bytes=4)
    assert {k.decode(): v for k, v in got.as_dict().items()} == g["reduced"]


def test_section2_case_and_punctuation():
    g = golden("section2_case_punct.json")
    got = check(g["text"].encode())
    assert {k.decode(): v for k, v in got.as_dict().items()} == g["expected"]


def test_section3_3_grouped_counts():
    g = golden("section3_3_grouping.json")
    w = g["word"].encode()
    text, off = join_docs([b" ".join([w] * n) + b"." for n in g["per_doc"]])
    per = check(text, off, per_doc=True)
    assert per.as_dict() == {(d, w): n for d, n in enumerate(g["per_doc"])}
    assert wc.merge([per]).as_dict() == {w: g["reduced"]}


def test_section4_3_applause():
    g = golden("section4_3_applause.json")
    check(g["text"].encode())


# ------------------------------------------------------------------------------------------
# brute force and edge cases
# ------------------------------------------------------------------------------------------

ALPHABET = [b"a", b"Z", b"0", b"'", b" ", b",", b"\x80", b"\n"]


def test_every_short_string_as_a_document():
    docs = [b"".join(p) for n in range(0, 6) for p in itertools.product(ALPHABET, repeat=n)]
    text, off = join_docs(docs)
    say("docs", len(docs), "bytes", len(text))
    check(text, off, per_doc=True)
    check(text, off)


@pytest.mark.parametrize("path", ["direct", "spill"])
def test_random_text_random_splits(path):
    for seed in range(4):
        text = synth.random_text(300_000, seed, alphabet=b"aAzZ09' ,.\x80\xff\n\t-\"bcY")
        off = synth.random_splits(len(text), 1 + seed * 97, seed + 100)
        say("seed", seed, path)
        check(text, off, debug_flags=PATHS[path])


def test_empty_inputs():
    g = gpu_count(b"")
    assert g.n_entries == 0 and g.total_tokens == 0
    g = gpu_count(b"   ,,. \n\x80")
    assert g.n_entries == 0 and g.total_tokens == 0
    check(b"a b", [0, 0, 0, 3, 3], per_doc=True)
    check(b"xxabcabcyy", [2, 5, 8])
    check(b"xxabcabcyy", [2, 4, 8])
    t, o = to_dev(b"abc", [0, 0])
    assert wc.count(t, o).n_entries == 0


def test_invalid_offsets_raise():
    with pytest.raises(wc.WcError) as e:
        gpu_count(b"abc def", [0, 5, 3])
    assert e.value.status == wc.WC_EINVAL
    with pytest.raises(wc.WcError) as e:
        gpu_count(b"abc", [0, 9])
    assert e.value.status == wc.WC_EINVAL


WORD_BYTES = np.frombuffer(b"abcXYZ019'", np.uint8)
SEP_BYTES = np.frombuffer(b" ,\n.", np.uint8)


def straddling_words(edge: int, n_edges: int, seed: int, max_len: int = 40) -> bytes:
    """Text in which, for every (length L in 1..max_len, offset k in 0..L), one word of L bytes
    covers the k bytes before some multiple of `edge` and the L - k bytes from it (k = 0: the
    word starts on the edge; k = L: it ends just before it). The gaps are filled with random
    short words and separators."""
    rng = np.random.default_rng(seed)
    cases = [(L, k) for L in range(1, max_len + 1) for k in range(L + 1)]
    order = rng.permutation(len(cases))
    out = bytearray()
    for i in range(n_edges):
        L, k = cases[order[i % len(cases)]]
        start = (i + 1) * edge - k
        # filler up to start - 1, then one separator before the word
        while len(out) < start - 1:
            room = start - 1 - len(out)
            fl = int(rng.integers(1, 8))
            if room > fl + 1:
                out += rng.choice(WORD_BYTES, fl).tobytes() + rng.choice(SEP_BYTES, 1).tobytes()
            else:
                out += b" " * room
        out += rng.choice(SEP_BYTES, 1).tobytes()
        assert len(out) == start
        out += rng.choice(WORD_BYTES, L).tobytes() + rng.choice(SEP_BYTES, 1).tobytes()
    return bytes(out)


def check_lengths_span(text: bytes, offsets, lo: int, hi: int):
    """The input really holds words of every length lo..hi (guards the test's own input)."""
    lens = {len(w) for w in oracle.count(text, offsets).as_dict()}
    missing = set(range(lo, hi + 1)) - lens
    assert not missing, f"input has no words of lengths {sorted(missing)}"


@pytest.mark.parametrize("stage,path", [(4096, "direct"), (8192, "direct"), (1024, "spill")])
def test_words_across_stage_boundaries(stage, path):
    """Words of every length 1..40 at every offset across stripe / stage edges: the one-pass
    kernel's stages (4 or 8 KiB) and the two-pass kernel's 1 KiB stripes (16 KiB stages; one
    stripe per wave), so words longer than 16 bytes and words carried into the next stripe both
    occur at edges."""
    n_edges = 861 if stage == 1024 else 200
    text = straddling_words(stage, n_edges, stage)
    check_lengths_span(text, None, 1, 40)
    tu = wc.make_tuning(stage_bytes=stage) if path == "direct" else None
    for shift in (0, 1, 7, 15):
        t = b"q" * shift + text
        say("stage", stage, path, "shift", shift, "bytes", len(t))
        check(t, tuning=tu, debug_flags=PATHS[path])
        check(t, [0, shift, len(t) // 3, len(t)], tuning=tu, debug_flags=PATHS[path])
    if path == "spill":
        # one workgroup over the whole text: the carried word crosses stages inside one range
        check(text, tuning=wc.make_tuning(grid_blocks=1), debug_flags=PATHS[path])
        check(text, tuning=wc.make_tuning(grid_blocks=3), debug_flags=PATHS[path])


def test_misaligned_corpus_pointer():
    c = synth.generate("plain-1MB")
    base = c.text.numpy()[:300_001]
    want = oracle.count(base).as_dict()
    for off in range(0, 17):
        # the view starts `off` bytes into an allocation, so its address is misaligned by
        # `off`; the byte before it is a word byte ('x') that must not join the first word
        big = torch.from_numpy(np.concatenate([np.frombuffer(b"x" * off, np.uint8), base]))
        view = big.to(DEV)[off:]
        assert view.numel() == len(base)
        got = wc.count(view, torch.tensor([0, len(base)], device=DEV))
        assert got.as_dict() == want, off
        assert got.total_tokens == sum(want.values())


@pytest.mark.parametrize("path", ["direct", "spill"])
def test_long_words(path):
    w1 = b"Ab" * 500_000             # 1 MB word, crosses many stages
    w16 = b"abcdefghijklmnop"
    w17 = w16 + b"Q"
    text = b" ".join([w1, w16, w17, w16.upper(), w17, w1.lower(), b"x", w1]) + b" "
    check(text, debug_flags=PATHS[path])
    check(text, [0, 1_000_001, len(text)], debug_flags=PATHS[path])
    check(text, per_doc=True, offsets=[0, 1_000_001, len(text)])  # large documents: one-pass
    check(text, per_doc=True, offsets=[0, 1_000_001, len(text)], debug_flags=wc.WC_DEBUG_DOCS)


@pytest.mark.parametrize("path", ["direct", "spill"])
def test_single_word_vocabulary_max_contention(path):
    text = b"the " * 400_000
    got = check(text, debug_flags=PATHS[path])
    assert got.as_dict() == {b"the": 400_000}


@pytest.mark.parametrize("path", ["direct", "spill"])
@pytest.mark.parametrize("bits", [1, 4, 8])
def test_forced_key_collisions(bits, path):
    c = synth.generate("plain-1MB")
    text = c.text.numpy()[:200_000]
    check(text, debug_hash_bits=bits, debug_flags=PATHS[path])
    check(np.frombuffer(b"ab abc abcd abcdefghijklmnopqrs abcdefghijklmnopqrt " * 50, np.uint8),
          debug_hash_bits=bits, debug_flags=PATHS[path])


def test_table_regrow():
    c = synth.generate("plain-1MB")
    text = c.text.numpy()
    got = check(text, table_slots=64)      # far too small: grows until it fits
    assert got.res.table_slots > 4096
    with pytest.raises(wc.WcError) as e:
        gpu_count(text, table_slots=64, regrow=False)
    assert e.value.status == wc.WC_ETABLEFULL


OVERFLOW_MODES = {
    "direct": dict(debug_flags=wc.WC_DEBUG_DIRECT),
    "spill": dict(debug_flags=wc.WC_DEBUG_SPILL),
    "docs": dict(per_doc=True, debug_flags=wc.WC_DEBUG_DOCS),
    "per_doc_direct": dict(per_doc=True, debug_flags=wc.WC_DEBUG_DIRECT),
}


@pytest.mark.parametrize("mode", list(OVERFLOW_MODES))
def test_count_width_overflow(mode):
    """A count above INT32_MAX exported at 4 bytes is WC_EOVERFLOW on every export path (the
    global one- and two-pass paths, both per-document kernels); at exactly INT32_MAX it is not;
    at 8 bytes the wide value is exported as is. The debug bias added to every exported count
    stands in for 2^31 tokens."""
    kw = OVERFLOW_MODES[mode]
    text = b"the cat The dog, the " * 2000
    off = [0, len(text) // 2, len(text)]
    want = oracle.count(text, off, per_doc=kw.get("per_doc", False)).as_dict()
    top = max(want.values())
    i32 = (1 << 31) - 1
    # the largest count lands exactly on INT32_MAX: still fits
    got = check_biased(text, off, i32 - top, 4, kw, want)
    assert max(got.values()) == i32
    with pytest.raises(wc.WcError) as e:
        gpu_count(text, off, count_bytes=4, debug_count_bias=i32 - top + 1, **kw)
    assert e.value.status == wc.WC_EOVERFLOW
    check_biased(text, off, 3 << 33, 8, kw, want)


def check_biased(text, off, bias, count_bytes, kw, want):
    got = gpu_count(text, off, count_bytes=count_bytes, debug_count_bias=bias, **kw)
    assert got.total_tokens == sum(want.values())
    d = got.as_dict()
    assert d == {k: v + bias for k, v in want.items()}
    return d


def test_merge_width_overflow():
    """Two wide tables whose sums pass INT32_MAX: merging them at 4 bytes is WC_EOVERFLOW, at 8
    bytes the exact sums."""
    text = b"alpha beta alpha gamma " * 500
    want = oracle.count(text).as_dict()
    big = 3 << 29  # 1.5 * 2^30: one table fits int32, the sum of two does not
    t = gpu_count(text, count_bytes=8, debug_count_bias=big)
    assert wc.merge([t, t], count_bytes=8).as_dict() == {k: 2 * (v + big) for k, v in want.items()}
    with pytest.raises(wc.WcError) as e:
        wc.merge([t, t], count_bytes=4)
    assert e.value.status == wc.WC_EOVERFLOW
    assert wc.merge([t], count_bytes=4).as_dict() == {k: v + big for k, v in want.items()}


def test_word_capacity_regrow():
    text = b" ".join(b"w%07d" % i for i in range(20_000))
    check(text, word_bytes_cap=16)


@pytest.mark.parametrize("stage,lds,policy,grid,no_lds", [
    (8192, 2048, wc.WC_FLUSH_ALL, 0, False),
    (4096, 256, wc.WC_FLUSH_ALL, 0, False),
    (8192, 4096, wc.WC_FLUSH_BYPASS, 0, False),
    (4096, 1024, wc.WC_FLUSH_BYPASS, 3, False),
    (8192, 2048, wc.WC_FLUSH_ALL, 1, False),
    (8192, 2048, wc.WC_FLUSH_ALL, 0, True),
])
def test_tuning_points_agree(stage, lds, policy, grid, no_lds):
    c = synth.generate("plain-1MB")
    tu = wc.make_tuning(stage_bytes=stage, lds_entries=lds, flush_policy=policy,
                        grid_blocks=grid)
    flags = wc.WC_DEBUG_NO_LDS if no_lds else 0
    check(c.text.numpy(), c.offsets.numpy(), tuning=tu, debug_flags=flags)


@pytest.mark.parametrize("lds,grid,pct", [(256, 0, 75), (256, 1, 50), (1024, 3, 90),
                                          (4096, 0, 75), (512, 7, 10)])
def test_spill_tuning_points(lds, grid, pct):
    """Small dictionaries send most tokens through the partitions; tiny grids give each
    pass-1 workgroup a long range; low loads send pass-2 overflow to the global table."""
    c = synth.generate("plain-1MB")
    tu = wc.make_tuning(lds_entries=lds, grid_blocks=grid, lds_load_pct=pct)
    check(c.text.numpy(), c.offsets.numpy(), tuning=tu, debug_flags=wc.WC_DEBUG_SPILL)
    cs = synth.generate("corpora-4x2000", scale=0.05)
    check(cs[0].text.numpy(), cs[0].offsets.numpy(), tuning=tu, debug_flags=wc.WC_DEBUG_SPILL)


@pytest.mark.parametrize("lds", [256, 1024, 4096])
def test_per_doc_relief_and_private_tables(lds):
    """Documents larger than the LDS table (emission of complete documents, moves to private
    tables), many tiny documents (several sub-windows per item), empty documents."""
    tu = wc.make_tuning(lds_entries=lds)
    c = synth.generate("plain-1MB")
    big = c.text.numpy()[:600_000]
    docs = wc.WC_DEBUG_DOCS  # the document-centric kernel, also for these large documents
    check(big, [0, 10, 10, 250_000, 250_001, 600_000], per_doc=True, tuning=tu, debug_flags=docs)
    tiny = synth.random_text(120_000, 9, alphabet=b"abcAB '. ")
    off = np.arange(0, 120_001, 7)
    off[-1] = 120_000
    check(tiny, off, per_doc=True, tuning=tu, debug_flags=docs)
    check(b"", [0, 0, 0], per_doc=True, tuning=tu, debug_flags=docs)


def test_per_doc_long_words_and_collisions():
    w = b"Z" * 40
    docs = [w + b" " + w.lower(), b"a" * 17 + b" x", b"", w + b" y " * 3000]
    text, off = join_docs(docs)
    for bits in (0, 3):
        check(text, off, per_doc=True, debug_hash_bits=bits)
        check(text, off, per_doc=True, debug_hash_bits=bits, tuning=wc.make_tuning(lds_entries=256))


@pytest.mark.parametrize("bits,direct", [(0, wc.WC_DIRECT_NEVER), (3, wc.WC_DIRECT_NEVER), (3, 0)])
def test_per_doc_private_table_collisions(bits, direct):
    """A document with more distinct words (9,000) than the second pass's LDS table holds: the
    rest go to its private table in device memory, claimed with a compare-and-swap first; with
    debug_hash_bits=3 every private key is one of eight values, so inserts probe far and tell
    words apart by their bytes. The document reaches the second pass by overflowing the first
    (WC_DIRECT_NEVER) or by its size (default limit)."""
    words = [b"w%05d" % i for i in range(9000)]
    rng = np.random.default_rng(5)
    doc = b" ".join(words + [words[i] for i in rng.integers(0, 9000, 6000)])
    text, off = join_docs([b"a b c", doc, b"tail words here a"])
    tu = wc.make_tuning(direct_kib=direct)
    check(text, off, per_doc=True, debug_hash_bits=bits, debug_flags=wc.WC_DEBUG_DOCS, tuning=tu)
    t, o = to_dev(text, off)
    got = wc.count(t, o, per_doc=True, count_bytes=4, debug_hash_bits=bits,
                   debug_flags=wc.WC_DEBUG_DOCS, tuning=tu)
    assert got.stats["docs_recounted"] >= 1


def test_per_doc_kernel_choice():
    """By default the document-centric kernel runs for documents averaging at most 64 KiB and
    the one-pass (document, word) table above that; both give the oracle's tables."""
    c = synth.generate("plain-1MB")
    text = c.text.numpy()[:800_000]
    for off in ([0, 65_536, 131_072], [0, 65_537, 131_073], [0, 300_000, 300_000, 800_000]):
        check(text[:off[-1]], off, per_doc=True)
        check(text[:off[-1]], off, per_doc=True, debug_flags=wc.WC_DEBUG_DOCS)
        check(text[:off[-1]], off, per_doc=True, debug_flags=wc.WC_DEBUG_DIRECT)


def test_per_doc_direct_path_agrees():
    c = synth.generate("batched-100k", scale=0.001)
    check(c.text.numpy(), c.offsets.numpy(), per_doc=True, debug_flags=wc.WC_DEBUG_DIRECT)


def test_per_doc_output_growth():
    c = synth.generate("batched-100k", scale=0.001)
    check(c.text.numpy(), c.offsets.numpy(), per_doc=True, word_bytes_cap=64, table_slots=4096,
          tuning=wc.make_tuning(lds_entries=256))


def test_spill_heavy_counts():
    """Dictionary words with large totals next to a Zipf tail that goes through the
    partitions; one pass-1 workgroup for the whole text."""
    rng = np.random.default_rng(5)
    words = [b"w%d" % i for i in range(3000)]
    idx = np.minimum(rng.zipf(1.3, size=300_000), 3000) - 1
    text = b" ".join(words[i] for i in idx) + b" " + b"the " * 100_000
    tu = wc.make_tuning(lds_entries=512, lds_load_pct=60)
    check(text, tuning=tu, debug_flags=wc.WC_DEBUG_SPILL)
    check(text, tuning=wc.make_tuning(grid_blocks=1), debug_flags=wc.WC_DEBUG_SPILL)


def _parts_of(words: np.ndarray) -> np.ndarray:
    """Partitions of words of at most 16 lower-case bytes (uint8[n, 16], zero padded) in the
    two-pass kernels: the low 8 bits of their 32-bit word hash (the packed word's dwords folded
    with rotations, then the MurmurHash3 finaliser). Used only to build inputs that crowd one
    partition; the test also checks the kernel's own statistics, so a change of the kernel's
    hash cannot leave it hollow."""
    d = np.ascontiguousarray(words).view("<u4").astype(np.uint64)
    a, b, c, e = d[:, 0], d[:, 1], d[:, 2], d[:, 3]
    m = np.uint64(0xffffffff)
    rotr = lambda x, r: ((x >> np.uint64(r)) | (x << np.uint64(32 - r))) & m
    h = ((a ^ rotr(b, 21)) + (c ^ rotr(e, 13))) & m
    h ^= h >> np.uint64(16)
    h = (h * np.uint64(0x85EBCA6B)) & m
    h ^= h >> np.uint64(13)
    h = (h * np.uint64(0xC2B2AE35)) & m
    h ^= h >> np.uint64(16)
    return (h & np.uint64(255)).astype(np.int64)


def test_two_pass_crowded_partition():
    """Thousands of distinct words of one partition: each pass-1 workgroup's share of the
    partition's arena blocks is used up, so the remaining records go straight to the global
    table (the kernel's own statistics must show it), with one, three or all workgroups."""
    rng = np.random.default_rng(11)
    cand = rng.integers(ord("a"), ord("z") + 1, size=(2_000_000, 16), dtype=np.uint8)
    lens = rng.integers(3, 13, size=len(cand))
    cand[np.arange(16)[None, :] >= lens[:, None]] = 0
    keep = cand[_parts_of(cand) == 0]
    words = sorted({bytes(r[r != 0]) for r in keep})[:6000]
    assert len(words) == 6000
    seq = [words[i] for i in rng.permutation(np.repeat(np.arange(len(words)), 3))]
    text = b" ".join(seq)
    assert len({len(w) for w in words}) == 10
    for lds in (256, 4096):
        got = check(text, tuning=wc.make_tuning(lds_entries=lds), debug_flags=wc.WC_DEBUG_SPILL)
        say("lds", lds, got.stats)
        assert got.stats["spilled"] > 0.9 * len(seq) - lds * 3
        assert got.stats["arena_direct"] > 0
    for grid in (1, 3):
        got = check(text, [0, len(text) // 2, len(text)], tuning=wc.make_tuning(grid_blocks=grid),
                    debug_flags=wc.WC_DEBUG_SPILL)
        say("grid", grid, got.stats)
        assert got.stats["arena_direct"] > 0


def test_two_pass_document_edges():
    """Documents that start on, just before and just after 8 KiB stage edges, and a stretch of
    5-byte documents (more document starts in a stage than threads in a workgroup)."""
    text = synth.random_text(200_000, 3, alphabet=b"abcdeXY' .,\n")
    n = len(text)
    off = {0, n}
    for k in range(1, 24):
        off |= {k * 8192 + d for d in (-17, -16, -15, -1, 0, 1, 15, 16, 17)}
    off |= set(range(100_000, 120_000, 5))
    offs = sorted(o for o in off if 0 <= o <= n)
    check(text, offs, debug_flags=wc.WC_DEBUG_SPILL)
    check(text, offs, tuning=wc.make_tuning(grid_blocks=3), debug_flags=wc.WC_DEBUG_SPILL)


def test_two_pass_one_byte_documents():
    """Every byte its own document over several stages: each byte of a word run starts a word,
    so a stage holds more starts than half its bytes."""
    text = b"ab" * 30_000 + b" x" * 5_000 + synth.random_text(50_000, 4)
    n = len(text)
    offs = list(range(0, 60_001)) + [70_000, n]
    check(text, offs, debug_flags=wc.WC_DEBUG_SPILL)
    check(text, offs, tuning=wc.make_tuning(lds_entries=256), debug_flags=wc.WC_DEBUG_SPILL)


# ------------------------------------------------------------------------------------------
# synthetic workloads
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("path", ["direct", "spill"])
def test_plain_1mb_int32(path):
    c = synth.generate("plain-1MB")
    got = check(c.text.numpy(), c.offsets.numpy(), count_bytes=4, debug_flags=PATHS[path])
    assert got.as_dict() == c.expected_table()
    assert got.counts().dtype == torch.int32


@pytest.mark.parametrize("path", ["direct", "spill"])
def test_corpora(path):
    for c in synth.generate("corpora-4x2000", scale=0.25):
        check(c.text.numpy(), c.offsets.numpy(), count_bytes=4, debug_flags=PATHS[path])


def test_per_doc_batched_sample():
    c = synth.generate("batched-100k", scale=0.003)
    say("docs", len(c.offsets) - 1, "bytes", len(c.text))
    check(c.text.numpy(), c.offsets.numpy(), per_doc=True, count_bytes=4)


@pytest.mark.parametrize("path", ["direct", "spill"])
def test_stream_piece(path):
    c = synth.generate("stream-8GiB", scale=1 / 256)
    got = check(c.text.numpy(), c.offsets.numpy(), debug_flags=PATHS[path])
    assert got.as_dict() == c.expected_table()


def test_stream_full_size_against_rank_histogram():
    """8 GiB single document, S = 2^22, int64: every count equals the generator's histogram."""
    say("generating 8 GiB on the GPU")
    c = synth.generate("stream-8GiB", device=DEV)
    say("generated", c.n_tokens, "tokens")
    got = wc.count(c.text, c.offsets, count_bytes=8, table_slots=1 << 22)
    assert got.total_tokens == c.n_tokens
    w, o, cnt, _ = got.to_host()
    # map each exported word to its vocabulary rank through a dictionary of the vocabulary
    vocab = {bytes(c.vocab[k, :c.vocab_lens[k]]): k for k in range(len(c.vocab_lens))}
    wb = w.tobytes()
    ranks = np.array([vocab[wb[o[e]:o[e + 1]]] for e in range(len(cnt))], dtype=np.int64)
    exp = c.expected.cpu().numpy()
    assert len(ranks) == int((exp > 0).sum())
    assert np.array_equal(cnt, exp[ranks])
    del c
    torch.cuda.empty_cache()


def vocab_keys(words: torch.Tensor, offsets: torch.Tensor, max_len: int) -> torch.Tensor:
    """Base-32 key of each word of at most max_len bytes over 'a'..'z' (a = 1, no byte = 0),
    from a word-bytes array and its offsets[n + 1] (torch, any device): distinct words have
    distinct keys, so a key identifies a vocabulary word."""
    lens = offsets[1:] - offsets[:-1]
    assert int(lens.max()) <= max_len and int(lens.min()) >= 1
    key = torch.zeros(lens.numel(), dtype=torch.int64, device=words.device)
    last = max(words.numel() - 1, 0)
    for j in range(max_len):
        b = words[(offsets[:-1] + j).clamp(max=last)].long() - 96
        key = key * 32 + torch.where(j < lens, b, torch.zeros_like(b))
    return key


def ranks_of(table_words, table_offsets, vocab: np.ndarray, vlens: np.ndarray, dev):
    """Vocabulary rank of each exported word (every word must be a vocabulary word)."""
    L = vocab.shape[1]
    vo = np.zeros(len(vlens) + 1, dtype=np.int64)
    np.cumsum(vlens, out=vo[1:])
    vw = np.concatenate([vocab[k, :vlens[k]] for k in range(len(vlens))])
    vk = vocab_keys(torch.from_numpy(vw).to(dev), torch.from_numpy(vo).to(dev), L)
    sk, perm = torch.sort(vk)
    tk = vocab_keys(table_words, table_offsets, L)
    i = torch.searchsorted(sk, tk).clamp(max=sk.numel() - 1)
    assert torch.equal(sk[i], tk), "an exported word is not a vocabulary word"
    return perm[i]


def test_batched_full_size_against_pair_histograms():
    """batched-100k at its full size (100,000 documents, 2.7 GB, 200,000-word vocabulary): one
    captured-graph run of the batch API gives every (document, word) count the generator drew,
    and its CSR layout is consistent."""
    say("generating batched-100k with per-(document, word) truth")
    c = synth.generate("batched-100k", device=DEV, pair_truth=True)
    n_docs = c.offsets.numel() - 1
    say("docs", n_docs, "bytes", c.text.numel(), "tokens", c.n_tokens)
    b = wc.Batch(max_docs=n_docs, max_bytes=c.text.numel(), count_bytes=4,
                 **wc.output_sizes(c.text, c.offsets, count_bytes=4))
    for rep in range(2):  # capture, then replay
        got = b.run(c.text, c.offsets)
        assert got.total_tokens == c.n_tokens
        n = got.n_entries
        assert n == c.extra["pair_keys"].numel()
        rank = ranks_of(got.words(), got.word_offsets(), c.vocab, c.vocab_lens, DEV)
        docs = got.docs()
        keys = docs * len(c.vocab_lens) + rank
        order = torch.argsort(keys)
        assert torch.equal(keys[order], c.extra["pair_keys"])
        assert torch.equal(got.counts().long()[order], c.extra["pair_counts"])
        # CSR: document d's entries are the doc_len[d] entries from doc_ptr[d]
        dp, dl = got.doc_ptr(), got.doc_len()
        assert int(dl.sum()) == n
        base = torch.repeat_interleave(dp, dl)
        first = torch.repeat_interleave(torch.cumsum(dl, 0) - dl, dl)
        pos = base + torch.arange(n, device=DEV) - first
        assert torch.equal(torch.sort(pos).values, torch.arange(n, device=DEV))
        assert torch.equal(docs[pos], torch.repeat_interleave(torch.arange(n_docs, device=DEV), dl))
        say("rep", rep, "entries", n, "ok")
        del rank, docs, keys, order, base, first, pos
    b.close()
    del c
    torch.cuda.empty_cache()


def test_corpora_full_size_counts_and_top50():
    """corpora-4x2000 at its full size (4 corpora x 2,000 documents, ~80 MB): each corpus's
    table and the top-50 distinctive words per corpus equal the oracle's."""
    cs = synth.generate("corpora-4x2000")
    tabs, otabs = [], []
    for i, c in enumerate(cs):
        say("corpus", i, "bytes", c.text.numel())
        got = check(c.text.numpy(), c.offsets.numpy(), count_bytes=4)
        assert got.as_dict() == c.expected_table()
        tabs.append(got)
        otabs.append(oracle.count(c.text.numpy(), c.offsets.numpy()))
    got = wc.topk_ratio(tabs, 50, 1)
    want = oracle.topk_ratio(otabs, 50, 1)
    assert got.vocab_size == want.vocab_size
    for i in range(len(cs)):
        assert got.words[i] == want.words[i]
        assert list(got.n_c[i]) == list(map(int, want.n_c[i]))
        assert list(got.n_rest[i]) == list(map(int, want.n_rest[i]))
        np.testing.assert_allclose(got.score[i], want.score[i], rtol=1e-12)


# ------------------------------------------------------------------------------------------
# merge, top-k, hash
# ------------------------------------------------------------------------------------------

def test_merge_matches_oracle():
    c = synth.generate("plain-1MB")
    text, off = c.text.numpy(), c.offsets.numpy()
    per = gpu_count(text, off, per_doc=True, count_bytes=4)
    whole = oracle.count(text, off).as_dict()
    assert wc.merge([per]).as_dict() == whole
    singles = [gpu_count(text[off[i]:off[i + 1]]) for i in range(len(off) - 1)]
    assert wc.merge(singles).as_dict() == whole
    a = wc.merge([wc.merge(singles[:2]), wc.merge(singles[2:])])
    assert a.as_dict() == whole
    g = golden("section2_worked_example.json")
    parts = []
    for p in g["partials"]:
        t = b" ".join(w.encode() for w, n in p.items() for _ in range(n))
        parts.append(gpu_count(t))
    assert {k.decode(): v for k, v in wc.merge(parts).as_dict().items()} == g["reduced"]


def test_dense_reduce_matches_merge_and_oracle():
    """The paper's zero-padded words x documents matrix summed by rows (Section 3.3) gives
    the oracle's reduced table, as the hash merge does: a few documents (one thread per row),
    hundreds of documents (one wave per row), empty documents, long words."""
    g = golden("section3_3_grouping.json")
    w = g["word"].encode()
    text, off = join_docs([b" ".join([w] * n) + b"." for n in g["per_doc"]])
    per = gpu_count(text, off, per_doc=True)
    assert wc.merge_dense(per).as_dict() == {w: g["reduced"]}
    c = synth.generate("plain-1MB")
    cs = synth.generate("corpora-4x2000", scale=0.1)
    long = b" ".join([b"Q" * 40, b"q" * 40, b"a" * 17, b"b"])
    cases = [(c.text.numpy(), c.offsets.numpy()),
             (cs[0].text.numpy(), cs[0].offsets.numpy()),
             (np.frombuffer(long * 3, np.uint8), [0, 0, len(long), len(long), 3 * len(long)])]
    for text, off in cases:
        per = gpu_count(text, off, per_doc=True, count_bytes=4)
        want = oracle.count(text, off).as_dict()
        for cb in (4, 8):
            got = wc.merge_dense(per, count_bytes=cb)
            assert got.as_dict() == want
            assert got.total_tokens == sum(want.values())
        assert wc.merge([per]).as_dict() == want
    # the row sums are checked against the count width
    per = gpu_count(cases[0][0], cases[0][1], per_doc=True, count_bytes=8,
                    debug_count_bias=1 << 30)
    with pytest.raises(wc.WcError) as e:
        wc.merge_dense(per, count_bytes=4)   # 4 documents of ~2^30 each
    assert e.value.status == wc.WC_EOVERFLOW


def test_merge_long_words_and_collisions():
    w = b"Q" * 40
    t1 = gpu_count(b" ".join([w, w.lower(), b"a" * 17, b"b"]))
    t2 = gpu_count(b" ".join([w, b"a" * 17, b"c"]))
    assert wc.merge([t1, t2]).as_dict() == {w.lower(): 3, b"a" * 17: 2, b"b": 1, b"c": 1}


def test_topk_matches_oracle():
    cs = synth.generate("corpora-4x2000", scale=0.1)
    tabs = [gpu_count(c.text.numpy(), c.offsets.numpy(), count_bytes=4) for c in cs]
    otabs = [oracle.count(c.text.numpy(), c.offsets.numpy()) for c in cs]
    for k, mc in ((50, 1), (7, 3), (300, 1)):
        got = wc.topk_ratio(tabs, k, mc)
        want = oracle.topk_ratio(otabs, k, mc)
        assert got.vocab_size == want.vocab_size
        for c in range(len(cs)):
            assert got.words[c] == want.words[c]
            assert list(got.n_c[c]) == list(map(int, want.n_c[c]))
            assert list(got.n_rest[c]) == list(map(int, want.n_rest[c]))
            np.testing.assert_allclose(got.score[c], want.score[c], rtol=1e-12)


def test_topk_ties_and_small_tables():
    tabs = [gpu_count(b"a b c a"), gpu_count(b"b c d"), gpu_count(b"a d d e")]
    otabs = [oracle.count(b"a b c a"), oracle.count(b"b c d"), oracle.count(b"a d d e")]
    for k in (1, 2, 5, 10):
        got = wc.topk_ratio(tabs, k)
        want = oracle.topk_ratio(otabs, k)
        assert got.words == want.words


def test_fnv1a_published_vectors():
    # FNV-1a 64 test vectors from the FNV reference (Fowler, Noll, Vo)
    h = wc.hash_words([b"", b"a", b"foobar"])
    assert h == [0xcbf29ce484222325, 0xaf63dc4c8601ec8c, 0x85944171f73967e8]
    # folding: the hash is taken over folded bytes
    assert wc.hash_words([b"FooBar"]) == [0x85944171f73967e8]


# ------------------------------------------------------------------------------------------
# batched (captured graph)
# ------------------------------------------------------------------------------------------

def test_batch_graph_replays_match_oracle():
    """One graph, replayed on corpora of different shapes, with eager work in between."""
    b = wc.Batch(max_docs=20_000, max_bytes=8 << 20, count_bytes=4)
    cases = []
    c = synth.generate("batched-100k", scale=0.002)
    cases.append((c.text.numpy(), c.offsets.numpy()))
    t2 = synth.random_text(200_000, 3, alphabet=b"abAB '.xyz")
    cases.append((np.frombuffer(t2, np.uint8), synth.random_splits(len(t2), 700, 4)))
    cases.append((c.text.numpy()[:100_000], np.array([0, 5, 5, 60_000, 100_000])))
    for rep in range(2):
        for text, off in cases:
            want = oracle.count(text, off, per_doc=True)
            t, o = to_dev(text, off)
            got = b.run(t, o)
            assert got.total_tokens == want.total
            assert got.as_dict() == want.as_dict()
            check_doc_layout(got, len(off) - 1)
            # unrelated eager work between replays
            torch.cuda.synchronize()
            _ = (t.float().sum() + 1).item()
    b.close()


def test_batch_rejects_oversize():
    b = wc.Batch(max_docs=10, max_bytes=1000)
    t, o = to_dev(b"x" * 2000, [0, 2000])
    with pytest.raises(wc.WcError) as e:
        b.run(t, o)
    assert e.value.status == wc.WC_EINVAL
    b.close()


# ------------------------------------------------------------------------------------------
# serving
# ------------------------------------------------------------------------------------------

def _requests(n, seed):
    rng = np.random.default_rng(seed)
    c = synth.generate("plain-1MB")
    base = c.text.numpy()
    out = []
    for i in range(n):
        size = int(min(len(base) - 1, np.exp(rng.normal(np.log(20_000), 1.5))))
        a = int(rng.integers(0, len(base) - size))
        out.append(base[a:a + size].tobytes())
    return out


def test_server_results_match_oracle_and_merge():
    srv = wc.Server(mem_budget=256 << 20, max_streams=3)
    texts = _requests(40, 1)
    ids = [srv.submit(t) for t in texts]
    for t, i in zip(texts, ids):
        got = wc.result_to_dict(srv.wait(i))
        assert got == oracle.count(t).as_dict()
    m = srv.merge(ids[:10])
    want = oracle.count(b"".join(texts[:10]), np.cumsum([0] + [len(t) for t in texts[:10]]))
    assert wc.result_to_dict(srv.wait(m)) == want.as_dict()
    assert srv.launches() < len(ids) + 1  # small requests were packed
    for i in ids + [m]:
        srv.release(i)
    srv.close()


def test_server_alone_and_in_the_mix_are_identical():
    texts = _requests(60, 2)
    probe = texts[17]
    alone = wc.Server(mem_budget=128 << 20, max_streams=1)
    a = wc.result_to_dict(alone.wait(alone.submit(probe)))
    alone.close()
    mix = wc.Server(mem_budget=64 << 20, max_streams=4)   # small budget: admission waits
    ids = [mix.submit(t) for t in texts]
    b = wc.result_to_dict(mix.wait(ids[17]))
    assert a == b == oracle.count(probe).as_dict()
    for t, i in zip(texts, ids):
        assert wc.result_to_dict(mix.wait(i)) == oracle.count(t).as_dict()
    mix.close()


def test_server_large_upload_and_packed_large_documents():
    """A 20 MiB request crosses the worker's two 8 MiB pinned upload buffers three times; the
    requests of a few hundred KB queued behind it are packed into one per-document launch whose
    documents average above 64 KiB (the one-pass (document, word) table)."""
    base = synth.generate("plain-1MB").text.numpy()
    big = np.tile(base, 21)[:(20 << 20) + 12_345].tobytes()
    mids = [base[a:a + n].tobytes() for a, n in ((0, 300_000), (100_000, 900_000),
                                                  (5, 700_001), (333, 500_000))]
    texts = [big] + mids
    srv = wc.Server(mem_budget=1 << 30, max_streams=2)
    ids = [srv.submit(t) for t in texts]
    for t, i in zip(texts, ids):
        assert wc.result_to_dict(srv.wait(i)) == oracle.count(t).as_dict()
    srv.close()


def test_server_serving_workload_requests():
    """Requests cut from the serving workload's text (500,000-word vocabulary, Zipf 1.05,
    lognormal sizes), among them one of 10 MiB and one just under the 64 MiB cap: each result is
    the oracle's table, and the large ones are the same alone and in the mix."""
    w = synth.WORKLOADS["serving"]
    vocab, vlens = synth.make_vocab(w.vocab, w.max_len, w.seed)
    sizes = [int(x) for x in np.minimum(
        synth.lognormal_sizes(48, *w.lognormal, seed=w.seed + 7919 + 5), 4 << 20)]
    big = {7: (10 << 20) + 333, 23: (64 << 20) - 1000}
    for i, n in big.items():
        sizes[i] = n
    total = sum(sizes)
    say("serving requests", len(sizes), "bytes", total)
    c = synth.gen_stream(total, vocab, vlens, synth.zipf_probs(w.vocab, w.zipf_s), w.seed + 11,
                         DEV)
    host = c.text.cpu().numpy()
    del c
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    texts = [host[a:a + n] for a, n in zip(starts, sizes)]
    want = {i: oracle.count(t).as_dict() for i, t in enumerate(texts)}
    alone = wc.Server(mem_budget=1 << 30, max_streams=1)
    a = {i: wc.result_to_dict(alone.wait(alone.submit(texts[i]))) for i in big}
    alone.close()
    mix = wc.Server(mem_budget=768 << 20, max_streams=4)
    ids = [mix.submit(t) for t in texts]
    for i, rid in enumerate(ids):
        got = wc.result_to_dict(mix.wait(rid))
        assert got == want[i], i
        if i in big:
            assert a[i] == got, i
    m = mix.merge([ids[i] for i in big])
    assert wc.result_to_dict(mix.wait(m)) == \
        oracle.count(b"".join(texts[i].tobytes() for i in big),
                     np.cumsum([0] + [sizes[i] for i in big])).as_dict()
    mix.close()


def test_server_release_during_merge():
    """Inputs released right after a merge is submitted stay readable until the merge has
    read them (their memory is freed afterwards), while new requests reuse the pool."""
    texts = _requests(24, 5)
    srv = wc.Server(mem_budget=32 << 20, max_streams=3)
    ids = [srv.submit(t) for t in texts[:8]]
    for i in ids:
        srv.wait(i)
    m = srv.merge(ids)
    for i in ids:
        srv.release(i)        # before the merge has necessarily run
    more = [srv.submit(t) for t in texts[8:]]   # reuse of the released memory
    want = oracle.count(b"".join(texts[:8]), np.cumsum([0] + [len(t) for t in texts[:8]]))
    assert wc.result_to_dict(srv.wait(m)) == want.as_dict()
    for t, i in zip(texts[8:], more):
        assert wc.result_to_dict(srv.wait(i)) == oracle.count(t).as_dict()
    with pytest.raises(wc.WcError) as e:
        srv.merge([ids[0]])   # released: no longer a request of the server
    assert e.value.status == wc.WC_EINVAL
    srv.close()


def test_server_budget_errors():
    srv = wc.Server(mem_budget=4 << 20, max_streams=1)
    with pytest.raises(wc.WcError) as e:
        srv.submit(b"word " * 2_000_000)   # 10 MB text: larger than the budget
    assert e.value.status == wc.WC_ENOMEM
    i = srv.submit(b"a b c a")
    assert wc.result_to_dict(srv.wait(i)) == {b"a": 2, b"b": 1, b"c": 1}
    srv.close()


def test_server_host_in_place_input():
    """Host text read in place (not copied at submission): pageable and pinned tensors and a
    numpy array, each request's table equals the oracle's."""
    texts = _requests(12, 8)
    srv = wc.Server(mem_budget=128 << 20, max_streams=3)
    ids = []
    for i, t in enumerate(texts):
        a = np.frombuffer(t, np.uint8)
        x = a if i % 3 == 0 else (torch.from_numpy(a.copy()) if i % 3 == 1
                                  else torch.from_numpy(a.copy()).pin_memory())
        ids.append(srv.submit(x, in_place=True))
    for t, i in zip(texts, ids):
        assert wc.result_to_dict(srv.wait(i)) == oracle.count(t).as_dict()
        srv.release(i)
    srv.close()


def test_server_device_input():
    c = synth.generate("plain-1MB")
    t = c.text.to(DEV)
    srv = wc.Server(mem_budget=256 << 20, max_streams=2)
    i = srv.submit(t, c.offsets.numpy())
    assert wc.result_to_dict(srv.wait(i)) == c.expected_table()
    srv.close()


def test_autotune_choice_is_exact_and_cached(tmp_path):
    c = synth.generate("batched-100k", scale=0.002)
    t, o = to_dev(c.text.numpy(), c.offsets.numpy())
    cache = str(tmp_path / "tune.json")
    tu = wc.autotune(t, o, per_doc=True, cache_path=cache)
    assert (tu.lds_entries, tu.chunk_bytes, tu.lds_load_pct) == (4096, 32 << 10, 85)
    assert os.path.exists(cache)
    tu2 = wc.autotune(t, o, per_doc=True, cache_path=cache)
    assert (tu2.lds_entries, tu2.chunk_bytes, tu2.lds_load_pct, tu2.direct_kib) == \
        (tu.lds_entries, tu.chunk_bytes, tu.lds_load_pct, tu.direct_kib)
    check(c.text.numpy(), c.offsets.numpy(), per_doc=True, tuning=tu)
    b = wc.Batch(max_docs=len(c.offsets), max_bytes=len(c.text), tuning=tu,
                 **wc.output_sizes(t, o))
    got = b.run(t, o)
    assert got.as_dict() == oracle.count(c.text.numpy(), c.offsets.numpy(), per_doc=True).as_dict()
    b.close()
    g = wc.autotune(t, o, per_doc=False, cache_path=cache)
    check(c.text.numpy(), c.offsets.numpy(), tuning=g, debug_flags=wc.WC_DEBUG_SPILL)


@pytest.mark.parametrize("direct_kib", [1, 32, wc.WC_DIRECT_NEVER])
def test_per_doc_direct_second_pass(direct_kib):
    """Documents longer than a 16 KiB work item and than direct_kib KiB skip the first count:
    counted once by the second pass (tokens included), the tables must not change."""
    c = synth.generate("batched-100k", scale=0.002)
    text, offs = c.text.numpy(), c.offsets.numpy()
    tu = wc.make_tuning(chunk_bytes=16 << 10, lds_entries=4096, lds_load_pct=85,
                        direct_kib=direct_kib)
    check(text, offs, per_doc=True, tuning=tu, debug_flags=wc.WC_DEBUG_DOCS)
    t, o = to_dev(text, offs)
    got = wc.count(t, o, per_doc=True, count_bytes=4, tuning=tu, debug_flags=wc.WC_DEBUG_DOCS,
                   **wc.output_sizes(t, o))
    sizes = np.diff(offs)
    if direct_kib != wc.WC_DIRECT_NEVER:
        big = int(((sizes > (16 << 10)) & (sizes > (direct_kib << 10))).sum())
        assert got.stats["docs_recounted"] >= big > 0
    want = oracle.count(text, offs, per_doc=True)
    b = wc.Batch(max_docs=len(offs), max_bytes=len(text), count_bytes=4, tuning=tu,
                 **wc.output_sizes(t, o))
    for _ in range(2):
        r = b.run(t, o)
        assert r.total_tokens == want.total and r.as_dict() == want.as_dict()
    b.close()


@pytest.mark.parametrize("chunk", [16 << 10, 32 << 10, 256 << 10, 1 << 20])
def test_per_doc_chunk_sizes(chunk):
    c = synth.generate("batched-100k", scale=0.002)
    check(c.text.numpy(), c.offsets.numpy(), per_doc=True,
          tuning=wc.make_tuning(chunk_bytes=chunk, lds_load_pct=50))


# ------------------------------------------------------------------------------------------
# UTF-8 tokeniser (Section 5.2's other languages)
# ------------------------------------------------------------------------------------------

UTF8_ALPHABET = [b"a", b"Z", b" ", b"\xc3", b"\xa9", b"\xe2", b"\x80", b"\x94", b"\xf0",
                 b"\x9f", b"\xed", b"\xa0"]


def check_utf8(text, offsets=None, per_doc=False, **kw):
    want = oracle.count(text, offsets, per_doc=per_doc, utf8=True)
    got = gpu_count(text, offsets, per_doc=per_doc, utf8=True, **kw)
    assert got.total_tokens == want.total
    g, w = got.as_dict(), want.as_dict()
    if g != w:
        missing = [k for k in w if k not in g][:5]
        extra = [k for k in g if k not in w][:5]
        wrong = [(k, g[k], w[k]) for k in w if k in g and g[k] != w[k]][:5]
        raise AssertionError(f"mismatch: missing {missing} extra {extra} wrong {wrong}")
    return got


def test_utf8_every_short_string_as_a_document():
    docs = [b"".join(p) for n in range(0, 5) for p in itertools.product(UTF8_ALPHABET, repeat=n)]
    text, off = join_docs(docs)
    say("docs", len(docs), "bytes", len(text))
    check_utf8(text, off)
    check_utf8(text, off, per_doc=True)


@pytest.mark.parametrize("stage", [4096, 8192])
def test_utf8_random_bytes_stage_edges_and_cuts(stage):
    """Mostly multi-byte text, sequences cut by stage edges (every shift of the corpus) and by
    document boundaries, words longer than 16 bytes, and 16-byte words with a byte >= 0x80 at
    positions 7 or 15 (stored as long words)."""
    rng = np.random.default_rng(stage)
    pieces = np.frombuffer(b"ab \xc3\xa9\xe2\x80\x94\xe6\x97\xa5\xf0\x9f\x98\x80\xce\xa9.", np.uint8)
    raw = rng.choice(pieces, 3 * stage).tobytes()
    special = ("aaaaaaaé" + "bbbbbbé" + " " + "ccccccccccccccé" + " " + "日本語のテキスト、"
               + "ddddddddddddddddddddddé ").encode()
    text = raw + special * 50 + raw[::-1]
    tu = wc.make_tuning(stage_bytes=stage)
    for shift in (0, 1, 3, 15):
        t = b"q" * shift + text
        say("stage", stage, "shift", shift)
        check_utf8(t, tuning=tu)
        off = synth.random_splits(len(t), 40 + shift, shift)
        check_utf8(t, off, tuning=tu)
        check_utf8(t, off, per_doc=True, tuning=tu)


def test_utf8_multilingual_and_ascii_agreement():
    text = ("Grüße aus Köln — naïve CAFÉ; Ωμέγα και άλφα… 日本語のテキスト、テスト。"
            "Привет, мир! ‘quoted’ “double” 5×3÷2 Zebra zebra\ufeffword ").encode() * 3000
    got = check_utf8(text)
    assert got.as_dict()["grüße".encode()] == 3000
    c = synth.generate("plain-1MB")
    a = gpu_count(c.text.numpy(), c.offsets.numpy(), utf8=True)
    assert a.as_dict() == c.expected_table()
    check_utf8(c.text.numpy(), c.offsets.numpy(), per_doc=True)
    # merging tables of UTF-8 words (16-byte words with high bytes take the long form)
    t1 = check_utf8(text[:len(text) // 2])
    t2 = check_utf8(text[len(text) // 2:])
    assert wc.merge([t1, t2]).as_dict() == oracle.count(
        text, [0, len(text) // 2, len(text)], utf8=True).as_dict()


# ------------------------------------------------------------------------------------------
# count from host memory, transfer pieces overlapped with counting
# ------------------------------------------------------------------------------------------

def test_count_host_pieces_match_oracle():
    """Pieces of 1 MiB cut at delimiters: the table equals the oracle's for a stream of several
    pieces, with documents of random sizes, a run of 3 MB without a delimiter across piece
    boundaries, pinned and pageable host input, and the UTF-8 reading."""
    c = synth.generate("stream-8GiB", scale=1 / 1024)          # 8 MiB, one document
    base = c.text.numpy()
    got = wc.count_host(base, piece_bytes=1 << 20)
    assert got.as_dict() == c.expected_table() and got.total_tokens == c.n_tokens
    pinned = torch.from_numpy(base.copy()).pin_memory()
    assert wc.count_host(pinned, piece_bytes=1 << 20).as_dict() == c.expected_table()
    text = np.concatenate([base[:2_500_000], np.frombuffer(b"x" * 3_000_000, np.uint8),
                           base[2_500_000:5_000_000]])
    off = synth.random_splits(len(text), 300, 9)
    want = oracle.count(text, off).as_dict()
    for piece in (1 << 20, 3 << 20):
        g = wc.count_host(text, off, piece_bytes=piece)
        assert g.as_dict() == want
    # one table from pieces equals the plain count of the same text on the device
    assert wc.count_host(text, off, piece_bytes=1 << 20, count_bytes=4).as_dict() == \
        gpu_count(text, off, count_bytes=4).as_dict()
    u = ("Grüße aus Köln — naïve CAFÉ; 日本語のテキスト、テスト。 ").encode() * 60_000
    assert wc.count_host(u, piece_bytes=1 << 20, utf8=True).as_dict() == \
        oracle.count(u, utf8=True).as_dict()
    e = wc.count_host(b"", [0, 0])
    assert e.n_entries == 0 and e.total_tokens == 0
