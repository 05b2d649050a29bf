"""GPU word-frequency counter for MI355X (gfx950): tokenise, hash and count words in HIP.

The compute path lives in the C-ABI library ``libwc.so`` built from ``csrc/``; ``wc`` is its
thin ctypes binding. ``synth`` writes seeded synthetic corpora. Importing the package does not
load the library; ``wc.lib()`` does, and fails loudly when it is missing.
"""
__all__ = ["wc", "synth"]
