"""The C ABI without a GPU: libwc.so loads, exports every function include/*.h declares, and
the ctypes structures of the binding have the C layout (checked with a small gcc program)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2206_05269_amd import wc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    src = "".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*[\w\s\*]+?\b(wc_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    f = declared_functions()
    for name in ("wc_count", "wc_count_plan", "wc_merge", "wc_merge_plan", "wc_topk_ratio",
                 "wc_topk_ratio_plan", "wc_strerror", "wc_last_hip_error", "wc_hash_words",
                 "wc_fold_sum", "wc_fold_sum_plan"):
        assert name in f


def test_library_exports_every_declared_symbol():
    L = wc.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_strerror_without_gpu():
    L = wc.lib()
    assert L.wc_strerror(0) == b"ok"
    assert b"table" in L.wc_strerror(-3)


def test_plan_without_gpu():
    p = wc.count_plan(8 << 30, 1, count_bytes=8, table_slots=1 << 22)
    assert p.table_slots == 1 << 22 and p.workspace_bytes > (1 << 22) * 32
    with pytest.raises(wc.WcError):
        wc.count_plan(100, 1, count_bytes=3)
    with pytest.raises(wc.WcError):
        wc.count_plan(100, 1, table_slots=1000)


def test_struct_layouts_match_c(tmp_path):
    prog = tmp_path / "sizes.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "wc.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(wc_tuning),"
        " sizeof(wc_opts), sizeof(wc_plan), sizeof(wc_result), sizeof(wc_topk),"
        " offsetof(wc_result, d_word_offsets), offsetof(wc_result, kernel_ms),"
        " offsetof(wc_topk, n_rows));return 0;}\n")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o",
                    str(exe)], check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True,
                                       check=True).stdout.split()))
    want = [ctypes.sizeof(wc.Tuning), ctypes.sizeof(wc.Opts), ctypes.sizeof(wc.Plan),
            ctypes.sizeof(wc.Result), ctypes.sizeof(wc.TopKStruct),
            wc.Result.d_word_offsets.offset, wc.Result.kernel_ms.offset,
            wc.TopKStruct.n_rows.offset]
    assert got == want


def test_fold_sum_argument_errors_without_gpu():
    """Rejected before any device work: unknown kind, n above 2^53, small or missing workspace."""
    L = wc.lib()
    need = ctypes.c_uint64()
    assert L.wc_fold_sum_plan(10 ** 8, ctypes.byref(need)) == 0 and need.value == 2048 * 8
    assert L.wc_fold_sum_plan(1, ctypes.byref(need)) == 0 and need.value == 8
    p = ctypes.c_void_p(4096)  # never dereferenced: every call below fails its checks first
    assert L.wc_fold_sum(2, 10, p, p, 1 << 20, None) == wc.WC_EINVAL
    assert L.wc_fold_sum(0, (1 << 53) + 1, p, p, 1 << 20, None) == wc.WC_EINVAL
    assert L.wc_fold_sum(0, 10 ** 8, p, p, 8, None) == wc.WC_EINVAL
    assert L.wc_fold_sum(0, 10, None, p, 1 << 20, None) == wc.WC_EINVAL


def test_sort_canonical_without_gpu():
    """The host helper orders a table by (document, word bytes), a proper prefix first, for
    stored offsets that do not start at 0."""
    import numpy as np
    rng = np.random.default_rng(3)
    words = [bytes(rng.choice(np.frombuffer(b"ab'\xc3\xa9z", np.uint8), rng.integers(1, 5)))
             for _ in range(400)]
    docs = rng.integers(0, 5, size=len(words))
    blob = b"".join(words)
    off = np.concatenate([[0], np.cumsum([len(w) for w in words])]) + 1000
    perm = wc.sort_canonical(np.frombuffer(blob, np.uint8), off, docs)
    want = sorted(range(len(words)), key=lambda e: (int(docs[e]), words[e], e))
    assert list(perm) == want
    perm = wc.sort_canonical(np.frombuffer(blob, np.uint8), off)
    assert [words[e] for e in perm] == sorted(words)
    assert len(wc.sort_canonical(np.zeros(0, np.uint8), np.zeros(1, np.uint64))) == 0
