"""The allocation-free entry point wc_count_static (scratch in the library's static device
array) against wc_count (scratch in a caller workspace), through the C ABI: identical tables
and totals on two calls in a row, the second with a smaller input (the array keeps the first
call's contents, so what must start at zero has to be cleared), and its limits rejected
before any device work."""
import numpy as np
import pytest
import torch

import oracle
from paper_2206_05269_amd import synth, wc

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _same(a: wc.Table, b: wc.Table):
    assert a.total_tokens == b.total_tokens
    assert a.n_entries == b.n_entries
    assert a.as_dict() == b.as_dict()


def test_static_matches_workspace_entry_point_twice():
    c = synth.generate("plain-1MB")
    big = c.text.to(DEV)
    big_off = c.offsets.to(DEV)
    small_txt = synth.random_text(120_000, 7, alphabet=b"abAB '.,xyz0\n")
    small = torch.from_numpy(np.frombuffer(small_txt, np.uint8).copy()).to(DEV)
    small_off = torch.tensor([0, 5, 5, 60_001, 120_000], dtype=torch.int64, device=DEV)
    for rep in range(2):
        for text, off, cb in ((big, big_off, 4), (small, small_off, 8)):
            print("rep", rep, "bytes", text.numel(), "count_bytes", cb, flush=True)
            got = wc.count_static(text, off, count_bytes=cb)
            ref = wc.count(text, off, count_bytes=cb, debug_flags=wc.WC_DEBUG_DIRECT)
            _same(got, ref)
            want = oracle.count(text.cpu().numpy(), off.cpu().numpy())
            assert got.as_dict() == want.as_dict()
            assert got.counts().dtype == (torch.int32 if cb == 4 else torch.int64)


def test_static_limits_and_errors():
    t = torch.from_numpy(np.frombuffer(b"a b c a " * 1000, np.uint8).copy()).to(DEV)
    with pytest.raises(wc.WcError) as e:
        wc.count_static(t, table_slots=1 << 21)       # beyond the static table
    assert e.value.status == wc.WC_ENOMEM
    many = b" ".join(b"w%05d" % i for i in range(2000))
    m = torch.from_numpy(np.frombuffer(many, np.uint8).copy()).to(DEV)
    with pytest.raises(wc.WcError) as e:
        wc.count_static(m, table_slots=64, regrow=False)   # 2000 words in 64 slots
    assert e.value.status == wc.WC_ETABLEFULL
    with pytest.raises(wc.WcError) as e:
        wc.count_static(m, word_bytes_cap=16, regrow=False)  # 12000 word bytes in 16
    assert e.value.status == wc.WC_ENOMEM
    with pytest.raises(wc.WcError) as e:
        wc.count_static(t, torch.tensor([0, 4, t.numel()], device=DEV), count_bytes=3)
    assert e.value.status == wc.WC_EINVAL
    got = wc.count_static(t, table_slots=1 << 20)
    assert got.as_dict() == {b"a": 2000, b"b": 1000, b"c": 1000}
