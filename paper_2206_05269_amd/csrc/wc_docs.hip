// Per-document count (one table per document; the paper's per-document dictionaries of
// Section 3.1, before the grouping of Section 3.3).
//
// Work. The corpus is cut into 64 KiB windows; a work item is a window and owns the documents
// whose first byte lies in it (the last one may run past the window). Workgroups take items
// from a device-side queue (persistent grid), so documents of very different sizes balance.
// An item with many documents is processed kDocW documents at a time ("sub-window").
//
// Counting. A sub-window is scanned in 8 KiB stages like the single-stream kernels, with the
// documents' starts marked in the stage. Each token is counted in an LDS table keyed by
// (document, packed word). When a document is complete its entries leave LDS straight into
// the output: one 64-bit atomic add on a packed cursor (entries << 32 | bytes) reserves space
// for a group of documents, so every document's entries and word bytes are contiguous and the
// word offsets stay a valid CSR over the whole output.
//
// Large documents. When the LDS table cannot take a token, complete documents are emitted
// first; if that is not enough, the documents still open are moved to private open-addressing
// tables in device memory (one per document, cleared by the workgroup, sized from the
// document's length) and counted there; at the end of the sub-window each private table is
// compacted into the output. Words longer than 16 bytes always use the private table.
//
// Every size the kernels need is read from a device-side task description, so a whole call
// can be captured once in a HIP graph and replayed for other corpora.
#include "wc_internal.h"

namespace wc {

struct DocTable {
  uint64_t* lo;    // 0 = empty
  uint64_t* hi;    // | kTop, 0 until published
  uint32_t* doc1;  // document (sub-window relative) + 1, 0 until published
  uint32_t* cnt;
  uint32_t size;
};


// Count n occurrences of (doc1, word). Returns false when the table cannot take it (more
// than `cap` live entries, or no slot within `max_probe` slots). Linear probing over groups of
// 4 slots: the words of a group's four slots are read together (each a 64-bit atomic read, so
// a concurrent claim is never seen half written); the first empty slot ends the search (no
// deletions while counting). Wave-uniform probe loop.
WC_DEV bool doc_add(const DocTable& T, uint64_t lo, uint64_t hi, uint32_t doc1, uint32_t n,
                    uint32_t* live, uint32_t cap, uint32_t max_probe = 32) {
  const uint64_t hiw = hi | kTop;
  const uint32_t ng = T.size >> 2;  // groups of 4 slots (the size is a power of two >= 256)
  uint32_t g = __umulhi(lds_word_hash(lo, hi, doc1), ng);
  uint32_t probe = 0;
  bool active = true, ok = false;
  while (__any(active)) {
    bool won = false;
    if (active) {
      const uint32_t b = g * 4;
      uint64_t v[4];
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j)  // four 64-bit atomic reads, issued together
        v[j] = __hip_atomic_load(&T.lo[b + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      int state = 0;  // 0: all 4 taken by other words, 1: counted, 2: empty slot e, 3: look again
      uint32_t e = 0;
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j) {
        if (state != 0) continue;
        if (v[j] == 0) {
          state = 2;
          e = b + j;
        } else if (v[j] == lo) {
          const uint64_t sh = __hip_atomic_load(&T.hi[b + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          const uint32_t sd = __hip_atomic_load(&T.doc1[b + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (sh == 0 || sd == 0) {
            state = 3;  // claimed, not published yet
          } else if (sh == hiw && sd == doc1) {
            atomicAdd(&T.cnt[b + j], n);
            state = 1;
          }
        }
      }
      if (state == 1) {
        ok = true;
        active = false;
      } else if (state == 2) {
        if (__hip_atomic_load(live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < cap) {
          won = atomicCAS((unsigned long long*)&T.lo[e], 0ull, (unsigned long long)lo) == 0;
          if (won) {
            __hip_atomic_store(&T.doc1[e], doc1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_store(&T.hi[e], hiw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            atomicAdd(&T.cnt[e], n);
            ok = true;
            active = false;
          }  // else the slot was taken: look at this group again
        } else {
          active = false;  // table at its cap
        }
      } else if (state == 0) {
        g = g + 1 == ng ? 0 : g + 1;
        probe += 4;
        if (probe >= max_probe) active = false;
      }
    }
    {
      // the wave's new entries in one addition to the live count (one lane, not one per entry)
      const uint64_t wm = __ballot(won);
      if (wm && won && __builtin_amdgcn_mbcnt_hi((uint32_t)(wm >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)wm, 0u)) == 0)
        atomicAdd(live, (uint32_t)__popcll(wm));
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  return ok;
}

WC_DEV uint64_t slot_word_len(const Slot& sl) {
  if (sl.w0 & kTop) return sl.w1 & ~kTop;
  return packed_len(sl.w0, sl.w1 & ~kTop);
}

// word bytes of a packed short word
WC_DEV void put_packed(uint8_t* dst, uint64_t lo, uint64_t hi, uint32_t len) {
  for (uint32_t q = 0; q < len; ++q)
    dst[q] = (uint8_t)((q < 8 ? lo >> (8 * q) : hi >> (8 * (q - 8))) & 0xff);
}

template <int BLOCK>
WC_DEV uint32_t block_excl_scan32(uint32_t v, uint32_t* s_tmp, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = v;
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) s_tmp[wave] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int w = 0; w < BLOCK / 64; ++w) {
    uint32_t x = s_tmp[w];
    base += w < wave ? x : 0u;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void doc_kernel(DocParams P) {
  constexpr int STAGE = BLOCK * 16;
  constexpr int NWAVE = BLOCK / 64;
  constexpr int PER = 8;  // LDS entries per thread during emission / rebuild (E <= PER * BLOCK)
  __shared__ uint4 s_txt4[STAGE / 16 + 2];
  __shared__ uint16_t s_wm[BLOCK];
  __shared__ uint16_t s_last[BLOCK + 1];
  __shared__ uint32_t s_bnd[STAGE / 32 + 2];
  __shared__ uint16_t s_starts[STAGE / 2];  // token starts
  __shared__ uint32_t s_elen[PER * BLOCK];  // emission: word lengths, then byte offsets
  __shared__ uint32_t s_wsum[NWAVE];
  __shared__ uint64_t s_doff[kDocW + 1];
  __shared__ uint32_t s_dn[kDocW], s_db[kDocW], s_dfill[kDocW];
  __shared__ uint64_t s_pbase[kDocW];       // private table: first slot, or ~0
  __shared__ uint32_t s_pslots[kDocW];
  __shared__ uint32_t s_need[kDocW];        // a token of this document found no LDS slot
  __shared__ uint32_t s_live, s_carry[2], s_next_w;
  __shared__ uint64_t s_item, s_e0, s_b0, s_tokens, s_minpos;
  __shared__ uint32_t s_rlo, s_rhi;  // documents of the stage: [s_rlo, s_rhi)
  __shared__ uint32_t s_emitted, s_scan_tmp[NWAVE];
  extern __shared__ __align__(16) uint8_t s_dyn[];
  const uint8_t* s_txt = (const uint8_t*)s_txt4;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  Header* hdr = P.hdr;
  if (ld_relaxed32(&hdr->flags) & kFlagBadOffsets) return;

  const uint8_t* corpus = P.task->corpus;
  const uint64_t len = P.task->len;
  const uint64_t* offsets = P.task->offsets;
  const uint64_t n_docs = P.task->n_docs;
  const int64_t base_off = -(int64_t)((uintptr_t)corpus & 15);
  const uint64_t win = P.win_bytes;
  const uint64_t n_win = len / win + 1;

  const uint32_t E = P.lds_entries;
  DocTable T;
  T.lo = (uint64_t*)s_dyn;
  T.hi = T.lo + E;
  T.doc1 = (uint32_t*)(T.hi + E);
  T.cnt = T.doc1 + E;
  T.size = E;
  const uint32_t cap = P.lds_cap;
  for (uint32_t i = tid; i < E; i += BLOCK) {
    T.lo[i] = 0;
    T.hi[i] = 0;
    T.doc1[i] = 0;
    T.cnt[i] = 0;
  }
  if (tid == 0) {
    s_live = 0;
    s_tokens = 0;
  }

  auto load16 = [&](int64_t p) -> uint4 {
    if (p >= 0 && p + 16 <= (int64_t)len) return load_stream16(corpus + p);
    uint32_t w[4] = {0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u};
    for (int j = 0; j < 16; ++j) {
      int64_t q = p + j;
      if (q >= 0 && q < (int64_t)len) {
        uint32_t b = corpus[q];
        w[j >> 2] = (w[j >> 2] & ~(0xffu << ((j & 3) * 8))) | (b << ((j & 3) * 8));
      }
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
  };

  // ---- emission of LDS entries of documents [r0, r1) (sub-window relative), all threads ----
  // Entries of those documents leave LDS (the rest are reinserted); big documents are skipped.
  auto emit = [&](uint32_t r0, uint32_t r1, uint64_t d_first) {
    for (uint32_t r = tid; r < kDocW; r += BLOCK) {
      s_dn[r] = 0;
      s_db[r] = 0;
      s_dfill[r] = 0;
    }
    __syncthreads();
    uint64_t klo[PER], khi[PER];
    uint32_t kd[PER], kc[PER];
    for (int j = 0; j < PER; ++j) {
      uint32_t i = tid * PER + j;
      kc[j] = 0;
      kd[j] = 0;
      if (i < E && T.cnt[i]) {
        klo[j] = T.lo[i];
        khi[j] = T.hi[i] & ~kTop;
        kd[j] = T.doc1[i];
        kc[j] = T.cnt[i];
        uint32_t r = kd[j] - 1;
        if (r >= r0 && r < r1) {
          atomicAdd(&s_dn[r], 1u);
          atomicAdd(&s_db[r], packed_len(klo[j], khi[j]));
        }
      }
    }
    __syncthreads();
    // per-document bases (documents of the sub-window, at most kDocW <= BLOCK)
    uint32_t vn = tid < kDocW ? s_dn[tid] : 0u, vb = tid < kDocW ? s_db[tid] : 0u;
    uint32_t tn, tb;
    uint32_t bn = block_excl_scan32<BLOCK>(vn, s_scan_tmp, &tn);
    uint32_t bb = block_excl_scan32<BLOCK>(vb, s_scan_tmp, &tb);
    if (tid == 0) {
      uint64_t old = atomicAdd((unsigned long long*)&hdr->out_cursor,
                               (unsigned long long)(((uint64_t)tn << 32) | tb));
      s_e0 = old >> 32;
      s_b0 = old & 0xffffffffull;
      if (s_e0 + tn > P.cap_e || s_b0 + tb > P.cap_b) or32(&hdr->flags, kFlagWordCap);
    }
    __syncthreads();
    const uint64_t e0 = s_e0, b0 = s_b0;
    const bool room = e0 + tn <= P.cap_e && b0 + tb <= P.cap_b;
    if (tid < kDocW) {
      uint32_t r = tid;
      if (r >= r0 && r < r1 && s_pbase[r] == ~0ull) {
        P.doc_ptr[d_first + r] = e0 + bn;
        P.doc_len[d_first + r] = vn;
      }
      s_dn[tid] = bn;  // now: entry base of document r inside this emission
    }
    __syncthreads();
    // ranks inside each document, lengths in emission order
    uint32_t idx[PER];
    for (int j = 0; j < PER; ++j) {
      idx[j] = 0xffffffffu;
      if (kc[j]) {
        uint32_t r = kd[j] - 1;
        if (r >= r0 && r < r1) {
          idx[j] = s_dn[r] + atomicAdd(&s_dfill[r], 1u);
          s_elen[idx[j]] = packed_len(klo[j], khi[j]);
        }
      }
    }
    __syncthreads();
    // byte offsets: exclusive scan of s_elen[0 .. tn) in chunks of BLOCK
    {
      uint32_t carry = 0;
      for (uint32_t c0 = 0; c0 < tn; c0 += BLOCK) {
        uint32_t i = c0 + tid;
        uint32_t v = i < tn ? s_elen[i] : 0u;
        uint32_t t;
        uint32_t ex = block_excl_scan32<BLOCK>(v, s_scan_tmp, &t);
        if (i < tn) s_elen[i] = carry + ex;
        carry += t;
      }
    }
    __syncthreads();
    for (int j = 0; j < PER; ++j) {
      if (idx[j] == 0xffffffffu) continue;
      uint64_t e = e0 + idx[j];
      uint64_t bpos = b0 + s_elen[idx[j]];
      uint32_t wl = packed_len(klo[j], khi[j]);
      if (room) {
        P.word_offsets[e] = bpos;
        // a document has fewer than 2^31 tokens (the corpus is below 4 GiB), so only a
        // debug bias can take an LDS count past the 32-bit width
        const uint64_t c = (uint64_t)kc[j] + P.count_bias;
        if (P.count_bytes == 4) {
          if (c > 0x7fffffffull) or32(&hdr->flags, kFlagCountOverflow);
          ((int32_t*)P.counts)[e] = (int32_t)c;
        } else {
          ((int64_t*)P.counts)[e] = (int64_t)c;
        }
        P.docs[e] = d_first + kd[j] - 1;
        put_packed(P.words + bpos, klo[j], khi[j], wl);
      }
      kc[j] = 0;  // emitted
    }
    // rebuild the LDS table with what stays
    __syncthreads();
    for (int j = 0; j < PER; ++j) {
      uint32_t i = tid * PER + j;
      if (i < E) {
        T.lo[i] = 0;
        T.hi[i] = 0;
        T.doc1[i] = 0;
        T.cnt[i] = 0;
      }
    }
    if (tid == 0) s_live = 0;
    __syncthreads();
    for (int j = 0; j < PER; ++j)  // fewer live entries than slots: a full probe always lands
      if (kc[j]) doc_add(T, klo[j], khi[j], kd[j], kc[j], &s_live, E, E);
    __syncthreads();
  };

  // ---- move documents to private tables (all threads); their LDS entries go along ----------
  // Documents before `em` are already emitted: a flag left on one of them from a token that
  // later found an LDS slot is ignored.
  auto convert = [&](uint32_t em, uint32_t nd) {
    // allocate and clear private tables for flagged documents
    for (uint32_t r = em; r < nd; ++r) {
      if (!s_need[r] || s_pbase[r] != ~0ull) continue;
      if (tid == 0) {
        // a document of b bytes has at most b/2 + 1 distinct words: b + 2 slots keep a small
        // document's table at most half full; large documents get b/16 slots (natural text
        // has far fewer distinct words than tokens)
        uint64_t bytes = s_doff[r + 1] - s_doff[r];
        uint64_t want = bytes / 16 > 4096 ? bytes / 16 : 4096;
        if (bytes + 2 < want) want = bytes + 2;
        if (want < 64) want = 64;
        uint64_t slots = 1;
        while (slots < want) slots <<= 1;
        uint64_t base = atomicAdd((unsigned long long*)&hdr->arena_next, (unsigned long long)slots);
        if (base + slots > P.arena_slots) {
          or32(&hdr->flags, kFlagWordCap);
          base = ~0ull - 1;  // unusable: the call reports ENOMEM
        }
        s_pbase[r] = base;
        s_pslots[r] = (uint32_t)slots;
      }
      __syncthreads();
      if (s_pbase[r] != ~0ull - 1) {
        Slot* t = P.arena + s_pbase[r];
        for (uint32_t i = tid; i < s_pslots[r]; i += BLOCK) t[i] = Slot{0, 0, 0, 0};
      }
      __syncthreads();
    }
    // dump LDS entries of big documents into their tables; keep the others
    uint64_t klo[PER], khi[PER];
    uint32_t kd[PER], kc[PER];
    for (int j = 0; j < PER; ++j) {
      uint32_t i = tid * PER + j;
      kc[j] = 0;
      if (i < E && T.cnt[i]) {
        klo[j] = T.lo[i];
        khi[j] = T.hi[i] & ~kTop;
        kd[j] = T.doc1[i];
        kc[j] = T.cnt[i];
      }
    }
    __syncthreads();
    for (int j = 0; j < PER; ++j) {
      uint32_t i = tid * PER + j;
      if (i < E) {
        T.lo[i] = 0;
        T.hi[i] = 0;
        T.doc1[i] = 0;
        T.cnt[i] = 0;
      }
    }
    if (tid == 0) s_live = 0;
    __syncthreads();
    for (int j = 0; j < PER; ++j) {
      if (!kc[j]) continue;
      uint32_t r = kd[j] - 1;
      uint64_t pb = s_pbase[r];
      if (pb == ~0ull) {
        doc_add(T, klo[j], khi[j], kd[j], kc[j], &s_live, E, E);
      } else if (pb != ~0ull - 1) {
        uint64_t key = finish_key(fnv_packed(klo[j], khi[j], packed_len(klo[j], khi[j])), P.key_mask);
        table_insert<false>(P.arena + pb, s_pslots[r] - 1, key, short_id(klo[j], khi[j], 0),
                            kc[j], hdr, ~0ull);
      }
    }
    for (uint32_t r = tid; r < nd; r += BLOCK) s_need[r] = 0;
    __syncthreads();
  };

  // ---- compaction of one private table into the output (all threads) ----------------------
  auto compact_private = [&](uint32_t r, uint64_t d) {
    const Slot* t = P.arena + s_pbase[r];
    const uint32_t slots = s_pslots[r];
    uint32_t n = 0, b = 0;
    for (uint32_t i = tid; i < slots; i += BLOCK) {
      Slot sl = t[i];
      if (sl.key) {
        ++n;
        b += (uint32_t)slot_word_len(sl);
      }
    }
    uint32_t tn, tb;
    block_excl_scan32<BLOCK>(n, s_scan_tmp, &tn);
    block_excl_scan32<BLOCK>(b, s_scan_tmp, &tb);
    if (tid == 0) {
      uint64_t old = atomicAdd((unsigned long long*)&hdr->out_cursor,
                               (unsigned long long)(((uint64_t)tn << 32) | tb));
      s_e0 = old >> 32;
      s_b0 = old & 0xffffffffull;
      if (s_e0 + tn > P.cap_e || s_b0 + tb > P.cap_b) or32(&hdr->flags, kFlagWordCap);
      P.doc_ptr[d] = s_e0;
      P.doc_len[d] = tn;
    }
    __syncthreads();
    const bool room = s_e0 + tn <= P.cap_e && s_b0 + tb <= P.cap_b;
    uint64_t e_run = s_e0, b_run = s_b0;
    for (uint32_t c0 = 0; c0 < slots; c0 += BLOCK) {
      uint32_t i = c0 + tid;
      Slot sl;
      sl.key = 0;
      if (i < slots) sl = t[i];
      uint32_t wl = sl.key ? (uint32_t)slot_word_len(sl) : 0u;
      uint32_t cn, cb;
      uint32_t en = block_excl_scan32<BLOCK>(sl.key ? 1u : 0u, s_scan_tmp, &cn);
      uint32_t eb = block_excl_scan32<BLOCK>(wl, s_scan_tmp, &cb);
      if (sl.key && room) {
        uint64_t e = e_run + en, bp = b_run + eb;
        P.word_offsets[e] = bp;
        const uint64_t c = sl.cnt + P.count_bias;
        if (P.count_bytes == 4) {
          if (c > 0x7fffffffull) or32(&hdr->flags, kFlagCountOverflow);
          ((int32_t*)P.counts)[e] = (int32_t)c;
        } else {
          ((int64_t*)P.counts)[e] = (int64_t)c;
        }
        P.docs[e] = d;
        if (sl.w0 & kTop) {
          const uint8_t* src = (const uint8_t*)(uintptr_t)(sl.w0 & ~kTop);
          for (uint32_t q = 0; q < wl; ++q) P.words[bp + q] = (uint8_t)fold_byte(src[q]);
        } else {
          put_packed(P.words + bp, sl.w0, sl.w1 & ~kTop, wl);
        }
      }
      e_run += cn;
      b_run += cb;
    }
    __syncthreads();
  };

  while (true) {
    if (tid == 0) s_item = __hip_atomic_fetch_add(&hdr->work_next, 1ull, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint64_t w = s_item;
    __syncthreads();
    if (w >= n_win) break;
    const uint64_t da = P.win_doc[w];
    const uint64_t db = min(P.win_doc[w + 1], n_docs);
    for (uint64_t d0 = da; d0 < db; d0 += kDocW) {
      const uint32_t nd = (uint32_t)min((uint64_t)kDocW, db - d0);
      for (uint32_t i = tid; i <= nd; i += BLOCK) s_doff[i] = offsets[d0 + i];
      for (uint32_t i = tid; i < kDocW; i += BLOCK) {
        s_pbase[i] = ~0ull;
        s_need[i] = 0;
      }
      if (tid == 0) s_emitted = 0;
      __syncthreads();
      const int64_t A = (int64_t)s_doff[0], B = (int64_t)s_doff[nd];
      if (A < B) {
        const int64_t k0 = (A - base_off) / STAGE;
        const int64_t k1 = (B - base_off + STAGE - 1) / STAGE;
        if (tid == 0) s_carry[(k0 & 1) ^ 1] = 0;  // A is a document start
        for (int i = tid; i < STAGE / 32 + 2; i += BLOCK) s_bnd[i] = 0;
        __syncthreads();  // cleared before any thread marks the first stage's document starts
        uint4 cur = load16(base_off + k0 * STAGE + tid * 16);
        for (int64_t k = k0; k < k1; ++k) {
          const int64_t ls = base_off + k * STAGE, le = ls + STAGE;
          uint4 nxt = make_uint4(0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u);
          if (k + 1 < k1) nxt = load16(le + tid * 16);
          uint32_t f0, f1, f2, f3;
          uint32_t g0 = fold_classify4(cur.x, &f0), g1 = fold_classify4(cur.y, &f1);
          uint32_t g2 = fold_classify4(cur.z, &f2), g3 = fold_classify4(cur.w, &f3);
          uint32_t w16 = movemask4(f0) | (movemask4(f1) << 4) | (movemask4(f2) << 8) |
                         (movemask4(f3) << 12);
          const int64_t p = ls + tid * 16;
          if (p < A || p + 16 > B) {
            int64_t lo_cut = A - p, hi_cut = B - p;
            uint32_t m = 0xffffu;
            if (lo_cut > 0) m &= lo_cut >= 16 ? 0u : (0xffffu << lo_cut) & 0xffffu;
            if (hi_cut < 16) m &= hi_cut <= 0 ? 0u : (0xffffu >> (16 - hi_cut));
            w16 &= m;
          }
          s_txt4[tid] = make_uint4(g0, g1, g2, g3);
          s_wm[tid] = (uint16_t)w16;
          if (tid == 0) {
            uint32_t nw = 0;
            if (le >= A && le < B) {
              uint32_t byte = (k + 1 < k1) ? (nxt.x & 0xffu) : (uint32_t)corpus[le];
              nw = is_word_byte(byte) ? 1u : 0u;
            }
            s_next_w = nw;
          }
          for (uint32_t i = tid; i <= nd; i += BLOCK) {
            int64_t o = (int64_t)s_doff[i];
            if (o >= ls && o <= le) {
              uint64_t rel = (uint64_t)(o - ls);
              atomicOr(&s_bnd[rel >> 5], 1u << (rel & 31));
            }
          }
          if (tid == 0) {
            // the stage's tokens belong to documents [rlo, rhi): the last one starting at or
            // before the stage start, up to the last one starting inside the stage
            uint32_t a = 0, b = nd;
            while (b - a > 1) {
              const uint32_t m = (a + b) >> 1;
              if ((int64_t)s_doff[m] <= ls) a = m;
              else b = m;
            }
            uint32_t c = a + 1;
            while (c < nd && (int64_t)s_doff[c] < le) ++c;
            s_rlo = a;
            s_rhi = c;
          }
          __syncthreads();
          uint32_t prev = tid > 0 ? (s_wm[tid - 1] >> 15) : s_carry[(k & 1) ^ 1];
          uint32_t next = tid < BLOCK - 1 ? (s_wm[tid + 1] & 1u) : s_next_w;
          uint32_t bnd = (s_bnd[tid >> 1] >> ((tid & 1) * 16)) & 0xffffu;
          uint32_t bnext = (s_bnd[(tid + 1) >> 1] >> (((tid + 1) & 1) * 16)) & 1u;
          uint32_t wprev = ((w16 << 1) | prev) & 0xffffu;
          uint32_t start16 = w16 & (~wprev | bnd);
          uint32_t wnext = (w16 >> 1) | (next << 15);
          uint32_t bn16 = (bnd >> 1) | (bnext << 15);
          uint32_t last16 = w16 & (~wnext | bn16) & 0xffffu;
          s_last[tid] = (uint16_t)last16;
          if (tid == BLOCK - 1) {
            s_carry[k & 1] = w16 >> 15;
            s_last[BLOCK] = 0;
          }
          uint32_t cnt = __popc(start16);
          uint32_t incl = cnt;
          for (int dd = 1; dd < 64; dd <<= 1) {
            uint32_t y = __shfl_up(incl, dd, 64);
            if (lane >= dd) incl += y;
          }
          if (lane == 63) s_wsum[wave] = incl;
          __syncthreads();
          uint32_t base = 0, total = 0;
          for (int ww = 0; ww < NWAVE; ++ww) {
            uint32_t v = s_wsum[ww];
            base += ww < wave ? v : 0u;
            total += v;
          }
          uint32_t o = base + incl - cnt;
          uint32_t mm = start16;
          while (mm) {
            int j = __ffs(mm) - 1;
            s_starts[o++] = (uint16_t)(tid * 16 + j);
            mm &= mm - 1;
          }
          if (tid == 0) s_tokens += total;
          __syncthreads();
          for (int i = tid; i < STAGE / 32 + 2; i += BLOCK) s_bnd[i] = 0;

          // tokens, in rounds of BLOCK so that a full LDS table can be relieved in between
          for (uint32_t t0 = 0; t0 < total; t0 += BLOCK) {
            const uint32_t t = t0 + tid;
            bool pending = false, have = false, is_long = false;
            uint64_t lo = 0, hi = 0, h64 = 0, wstart = 0, wlen = 0;
            uint32_t r = 0;
            if (t < total) {
              have = true;
              const uint32_t s = s_starts[t];
              uint32_t q = s >> 4;
              uint32_t bits = (uint32_t)s_last[q] >> (s & 15);
              uint32_t e;
              bool crosses = false;
              if (bits) {
                e = s + __ffs(bits) - 1;
              } else {
                ++q;
                while (q < BLOCK && s_last[q] == 0) ++q;
                if (q < BLOCK) e = q * 16 + __ffs(s_last[q]) - 1;
                else { crosses = true; e = STAGE - 1; }
              }
              // document of the token: last i with s_doff[i] <= position
              const uint64_t pos = (uint64_t)(ls + s);
              uint32_t lo_i = s_rlo, hi_i = s_rhi;
              while (hi_i - lo_i > 1) {
                uint32_t mid = (lo_i + hi_i) >> 1;
                if (s_doff[mid] <= pos) lo_i = mid; else hi_i = mid;
              }
              r = lo_i;
              const uint32_t wl = e - s + 1;
              if (!crosses && wl <= 16) {
                const uint32_t* tw = (const uint32_t*)s_txt;
                uint32_t di = s >> 2, sh = s & 3;
                uint32_t d0w = tw[di], d1w = tw[di + 1], d2w = tw[di + 2], d3w = tw[di + 3], d4w = tw[di + 4];
                lo = (uint64_t)__builtin_amdgcn_alignbyte(d1w, d0w, sh) |
                     ((uint64_t)__builtin_amdgcn_alignbyte(d2w, d1w, sh) << 32);
                hi = (uint64_t)__builtin_amdgcn_alignbyte(d3w, d2w, sh) |
                     ((uint64_t)__builtin_amdgcn_alignbyte(d4w, d3w, sh) << 32);
                if (wl < 8) { lo &= (1ull << (8 * wl)) - 1; hi = 0; }
                else if (wl == 8) { hi = 0; }
                else if (wl < 16) { hi &= (1ull << (8 * (wl - 8))) - 1; }
                wlen = wl;
              } else {
                wstart = pos;
                uint64_t limit = crosses ? s_doff[r + 1] : pos + wl;
                wlen = scan_word(corpus, pos, limit, &lo, &hi, &h64);
                is_long = wlen > 16;
              }
            }
            // count it: private table, LDS, or wait for a relief round
            auto place = [&]() -> bool {
              const uint64_t pb = s_pbase[r];
              if (pb == ~0ull - 1) return true;  // no private table: the call reports ENOMEM
              if (pb != ~0ull) {
                uint64_t key;
                WordId id;
                if (is_long) {
                  key = finish_key(h64, P.key_mask);
                  id = long_id(corpus + wstart, wlen, 0);
                } else {
                  key = finish_key(fnv_packed(lo, hi, (uint32_t)wlen), P.key_mask);
                  id = short_id(lo, hi, 0);
                }
                table_insert<false>(P.arena + pb, s_pslots[r] - 1, key, id, 1, hdr, ~0ull);
                return true;
              }
              if (is_long) return false;
              return doc_add(T, lo, hi, r + 1, 1, &s_live, cap);
            };
            if (have && !place()) {
              pending = true;
              s_need[r] = 1;
            }
            // Relief: each pass either emits at least one complete document (documents that
            // end before this round's first token) or moves every open document that holds
            // LDS entries, and every document with a waiting token, to a private table; after
            // that every waiting token has a place, so the loop ends.
            while (__syncthreads_or(pending)) {
              // every token before the first waiting one is counted, so documents that end
              // at or before that token's position are complete
              if (tid == 0) s_minpos = ~0ull;
              __syncthreads();
              if (pending) atomicMin((unsigned long long*)&s_minpos,
                                     (unsigned long long)(ls + s_starts[t]));
              __syncthreads();
              const uint64_t first_pos = s_minpos;
              const uint32_t em = s_emitted;
              uint32_t done = em;
              while (done < nd && s_doff[done + 1] <= first_pos) ++done;
              __syncthreads();
              if (done > em) {
                emit(em, done, d0);
                if (tid == 0) s_emitted = done;
                __syncthreads();
              } else {
                for (uint32_t i = tid * PER; i < tid * PER + PER && i < E; ++i) {
                  if (T.cnt[i]) {
                    uint32_t rr = T.doc1[i] - 1;
                    if (rr >= em) s_need[rr] = 1;
                  }
                }
                __syncthreads();
                convert(em, nd);
              }
              if (pending && place()) pending = false;
            }
          }
          __syncthreads();
          cur = nxt;
        }
      }
      // sub-window end: every document is complete
      emit(s_emitted, nd, d0);
      for (uint32_t rr = 0; rr < nd; ++rr) {
        if (s_pbase[rr] != ~0ull && s_pbase[rr] != ~0ull - 1) compact_private(rr, d0 + rr);
      }
      __syncthreads();
    }
  }
  if (tid == 0) add64(&hdr->total_tokens, s_tokens);
}

// The number of output entries and word bytes; closes the word-offset CSR.
__global__ void doc_finish_kernel(DocParams P) {
  if (threadIdx.x || blockIdx.x) return;
  uint64_t c = P.hdr->out_cursor;
  uint64_t n = c >> 32, b = c & 0xffffffffull;
  P.hdr->n_entries = n;
  P.hdr->word_bytes = b;
  if (n <= P.cap_e) P.word_offsets[n] = b;
}

// first document that starts at or after each 64 KiB window (device-side sizes)
__global__ void doc_windows_kernel(DocParams P) {
  const uint64_t len = P.task->len, n_docs = P.task->n_docs;
  const uint64_t* offsets = P.task->offsets;
  const uint64_t n_win = len / P.win_bytes + 1;
  if (n_win + 1 > P.max_win + 1) {
    if (threadIdx.x == 0 && blockIdx.x == 0) or32(&P.hdr->flags, kFlagWordCap);
    return;
  }
  for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w <= n_win;
       w += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t x = w * P.win_bytes;
    uint64_t lo = 0, hi = n_docs + 1;
    while (lo < hi) {
      uint64_t mid = (lo + hi) >> 1;
      if (offsets[mid] < x) lo = mid + 1; else hi = mid;
    }
    P.win_doc[w] = lo;
  }
}

__global__ void doc_validate_kernel(DocParams P) {
  const uint64_t n_docs = P.task->n_docs, len = P.task->len;
  const uint64_t* off = P.task->offsets;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i <= n_docs;
       i += (uint64_t)gridDim.x * blockDim.x) {
    bool bad = (i < n_docs && off[i] > off[i + 1]) || (i == n_docs && off[i] > len);
    if (bad) or32(&P.hdr->flags, kFlagBadOffsets);
  }
}

hipError_t set_doc_smem(size_t dyn) {
  return hipFuncSetAttribute((const void*)doc_kernel<512>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
}

hipError_t launch_docs(const DocParams& P, uint32_t grid, size_t dyn, hipStream_t s) {
  hipLaunchKernelGGL(doc_validate_kernel, dim3(256), dim3(256), 0, s, P);
  hipLaunchKernelGGL(doc_windows_kernel, dim3(256), dim3(256), 0, s, P);
  hipLaunchKernelGGL(doc_kernel<512>, dim3(grid), dim3(512), dyn, s, P);
  hipLaunchKernelGGL(doc_finish_kernel, dim3(1), dim3(64), 0, s, P);
  return hipGetLastError();
}

}  // namespace wc
