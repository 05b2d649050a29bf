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


@pytest.mark.parametrize("path", ["direct", "spill"])
@pytest.mark.parametrize("stage", [4096, 8192])
def test_words_across_stage_boundaries(stage, path):
    # words of every length 1..40 ending and starting at every position near stage edges
    rng = np.random.default_rng(stage)
    parts = []
    pos = 0
    while pos < 5 * stage:
        L = int(rng.integers(1, 41))
        w = bytes(rng.choice(list(b"abcXYZ019'"), L))
        sep = bytes(rng.choice(list(b" ,\n."), int(rng.integers(1, 3))))
        parts.append(w + sep)
        pos += L + len(sep)
    text = b"".join(parts)
    if path == "spill" and stage != 8192:
        pytest.skip("the two-pass kernel has one stage size (16 KiB, 1 KiB per wave)")
    for shift in (0, 1, 7, 15):
        t = b"q" * shift + text
        tu = wc.make_tuning(stage_bytes=stage)
        check(t, tuning=tu, debug_flags=PATHS[path])
        check(t, [0, shift, len(t) // 3, len(t)], tuning=tu, debug_flags=PATHS[path])


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


def _part_of(word: bytes) -> int:
    """Partition of a short word in the two-pass kernels (their 32-bit word hash, low 8 bits);
    used only to build inputs that crowd one partition."""
    b = word.lower().ljust(16, b"\0")
    a, b_, c, d = (int.from_bytes(b[i:i + 4], "little") for i in (0, 4, 8, 12))
    m = 0xffffffff
    h = ((a * 0x9E3779B1) ^ (b_ * 0x85EBCA77) ^ (c * 0xC2B2AE3D) ^ (d * 0x27D4EB2F)) & m
    h ^= h >> 15
    h = (h * 0x2C1B3C6D) & m
    h ^= h >> 13
    return h & 255


def test_two_pass_crowded_partition():
    """Thousands of distinct words of one partition in every stage: the LDS staging of that
    partition fills, the overflow list fills, and the rest goes to the global table."""
    rng = np.random.default_rng(11)
    words = set()
    while len(words) < 6000:
        w = bytes(rng.choice(list(b"abcdefghijklmnopqrstuvwxyz"), int(rng.integers(3, 9))))
        if _part_of(w) == 0:
            words.add(w)
    words = sorted(words)
    seq = [words[i] for i in rng.permutation(np.repeat(np.arange(len(words)), 2))]
    text = b" ".join(seq)
    for lds in (256, 4096):
        check(text, tuning=wc.make_tuning(lds_entries=lds), debug_flags=wc.WC_DEBUG_SPILL)
    check(text, [0, len(text) // 2, len(text)], tuning=wc.make_tuning(grid_blocks=1),
          debug_flags=wc.WC_DEBUG_SPILL)


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


def test_server_budget_errors():
    srv = wc.Server(mem_budget=4 << 20, max_streams=1)
    with pytest.raises(wc.WcError) as e:
        srv.submit(b"word " * 2_000_000)   # 10 MB text: larger than the budget
    assert e.value.status == wc.WC_ENOMEM
    i = srv.submit(b"a b c a")
    assert wc.result_to_dict(srv.wait(i)) == {b"a": 2, b"b": 1, b"c": 1}
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
    assert tu.lds_entries in (2048, 4096) and tu.chunk_bytes in (32 << 10, 64 << 10, 128 << 10)
    assert os.path.exists(cache)
    tu2 = wc.autotune(t, o, per_doc=True, cache_path=cache)
    assert (tu2.lds_entries, tu2.chunk_bytes, tu2.lds_load_pct) == \
        (tu.lds_entries, tu.chunk_bytes, tu.lds_load_pct)
    check(c.text.numpy(), c.offsets.numpy(), per_doc=True, tuning=tu)
    b = wc.Batch(max_docs=len(c.offsets), max_bytes=len(c.text), tuning=tu,
                 **wc.output_sizes(t, o))
    got = b.run(t, o)
    assert got.as_dict() == oracle.count(c.text.numpy(), c.offsets.numpy(), per_doc=True).as_dict()
    b.close()
    g = wc.autotune(t, o, per_doc=False, cache_path=cache)
    check(c.text.numpy(), c.offsets.numpy(), tuning=g, debug_flags=wc.WC_DEBUG_SPILL)


@pytest.mark.parametrize("chunk", [16 << 10, 32 << 10, 256 << 10, 1 << 20])
def test_per_doc_chunk_sizes(chunk):
    c = synth.generate("batched-100k", scale=0.002)
    check(c.text.numpy(), c.offsets.numpy(), per_doc=True,
          tuning=wc.make_tuning(chunk_bytes=chunk, lds_load_pct=50))
