// Per-document count (one table per document; the paper's per-document dictionaries of
// Section 3.1, before the grouping of Section 3.3).
//
// Work. The corpus is cut into windows of `win_bytes`; a work item is a window and owns the
// documents whose first byte lies in it (the last one may run past the window). Workgroups
// (1024 threads, one per CU) take items from a device-side queue (persistent grid), so
// documents of very different sizes balance. An item with many documents is processed kDocW
// documents at a time ("sub-window").
//
// Counting. A sub-window's text is scanned with the stripe scanner of the global count: each
// wave takes a contiguous run of 1 KiB stripes and runs on its own (no workgroup barrier
// inside the scan). A token's document is its sub-window index r, found from the document
// starts of its stripe; (word, r) is one 16-byte key (r sits in bit 7 of the bytes of the
// packed word's second half, bits that no word byte uses) in the LDS table shared with the
// global count's reduce. The scan is optimistic: a token that finds no room in the table, or a
// word longer than 16 bytes, marks its document as overflowed. After the scan every other
// document leaves LDS straight into the output: one 64-bit atomic add on a packed cursor
// (entries << 32 | bytes) reserves space for the sub-window, and one 64-bit LDS atomic per
// entry gives it its (entry, byte) place inside its document, so every document's entries
// and word bytes are contiguous and the word offsets stay a valid CSR over the whole output.
//
// A document longer than the window is always the last of its item; it is counted after the
// others, alone, with the whole LDS table to itself, unless it is also longer than the size
// limit (direct_kib): then it skips this pass. Such documents, and those that overflow, are
// queued for a second launch. Its queue is first sorted by size, largest first; then each
// document is counted by a whole workgroup: an LDS table with no overflow threshold (as many
// entries as the instance's LDS holds), then a private open-addressing table in device memory
// (taken from an arena, cleared by the workgroup, sized from the document's length) for the
// words that find no room. The entries of both tables are written out side by side with one
// reservation (a private word that also reached the LDS table is merged into its entry).
//
// Every size the kernels need is read from a device-side task description, so a whole call
// can be captured once in a HIP graph and replayed for other corpora.
#include "wc_internal.h"
#include "wc_stripe.h"

namespace wc {

namespace {

constexpr int kDocBlock = 1024;

// bits 0..3 of n -> bits 7, 15, 23, 31 (the top bits of four bytes)
WC_DEV uint32_t spread4(uint32_t n) {
  return (__umul24(n & 7u, 0x204080u) & 0x808080u) | ((n & 8u) << 28);
}
// bits 7, 15, 23, 31 -> bits 0..3
WC_DEV uint32_t gather4(uint32_t x) {
  return ((x >> 7) & 1u) | ((x >> 14) & 2u) | ((x >> 21) & 4u) | ((x >> 28) & 8u);
}
// The second half of a packed word with document r (< 256) in the top bits of its bytes.
WC_DEV uint64_t hi_with_doc(uint64_t hi, uint32_t r) {
  return hi | spread4(r & 15u) | ((uint64_t)spread4(r >> 4) << 32);
}
WC_DEV uint32_t key_doc(const uint4 k) { return gather4(k.z) | (gather4(k.w) << 4); }

// word bytes of a packed short word
WC_DEV void put_packed(uint8_t* dst, uint64_t lo, uint64_t hi, uint32_t len) {
  for (uint32_t q = 0; q < len; ++q)
    dst[q] = (uint8_t)((q < 8 ? lo >> (8 * q) : hi >> (8 * (q - 8))) & 0xff);
}

WC_DEV uint64_t slot_word_len(const Slot& sl) {
  if (sl.w0 & kTop) return sl.w1 & ~kTop;
  return packed_len(sl.w0, sl.w1 & ~kTop);
}

template <int BLOCK>
WC_DEV uint32_t block_excl_scan32(uint32_t v, uint32_t* s_tmp, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_scan(v);
  if (lane == 63) s_tmp[wave] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int w = 0; w < BLOCK / 64; ++w) {
    const uint32_t x = s_tmp[w];
    base += w < wave ? x : 0u;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

}  // namespace

size_t doc_dyn(uint32_t entries) { return (size_t)kRedSlots * 4 + (size_t)entries * 20; }

// kRecount = false: the optimistic pass over the work items; true: the overflowed documents,
// taken from the queue the first pass filled, one per workgroup at a time.
template <int BLOCK, bool kRecount>
__global__ __launch_bounds__(BLOCK) void doc_kernel(DocParams P) {
  constexpr int NW = BLOCK / 64;
  static_assert(kDocW <= BLOCK && kDocW <= 256, "a document index fits 8 bits");
  extern __shared__ __align__(16) uint8_t s_dyn[];
  __shared__ __align__(16) uint8_t s_txt[NW][kStripeText];
  __shared__ uint32_t s_list[NW][kWaveStarts];  // 16-bit starts, then the end bitmap
  __shared__ uint32_t s_bnd[NW][kBndWords];     // document starts of a stripe
  __shared__ uint64_t s_doff[kDocW + 1];
  __shared__ uint32_t s_over[kDocW];            // overflowed: counted again
  __shared__ unsigned long long s_dcur[kDocW];  // emission: (entries << 32 | bytes)
  __shared__ uint32_t s_nent, s_tmp[NW];
  __shared__ uint64_t s_item, s_e0, s_b0, s_pbase;
  __shared__ uint32_t s_pslots;
  __shared__ uint32_t s_pused;  // second pass: a word of the document went to its private table
  __shared__ unsigned long long s_tokens;
  __shared__ uint32_t s_direct;  // second pass: the document was queued without a first count
  static_assert(kWaveStarts / 2 + kEndWords <= kWaveStarts, "starts and ends fit a wave's list");

  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  Header* hdr = P.hdr;
  if (ld_relaxed32(&hdr->flags) & kFlagBadOffsets) return;

  const uint8_t* corpus = P.task->corpus;
  const uint64_t len = P.task->len;
  const uint64_t* offsets = P.task->offsets;
  const uint64_t n_docs = P.task->n_docs;
  const int64_t base_off = -(int64_t)((uintptr_t)corpus & 15);
  const uint64_t win = P.win_bytes;
  const uint64_t n_win = len / win + 1;

  // the second pass has no overflow threshold: its table fills all of its (more) entries,
  // and the words that find no room go to the document's private table
  const uint32_t E = kRecount ? P.rc_entries : P.lds_entries;
  RedTable T;
  T.slot = (uint32_t*)s_dyn;
  T.key = (uint4*)(T.slot + kRedSlots);
  T.cnt = (uint32_t*)(T.key + E);
  T.n = &s_nent;
  T.cap = kRecount ? E : min(P.lds_cap, E);
  T.stall = hdr;  // a word must never be both in the LDS table and in a private table
  for (uint32_t i = tid; i < kRedSlots; i += BLOCK) T.slot[i] = 0;
  for (uint32_t i = tid; i < E; i += BLOCK) {
    T.key[i] = make_uint4(0, 0, 0, 0);
    T.cnt[i] = 0;
  }
  for (uint32_t i = tid; i < NW * kWaveStarts; i += BLOCK) (&s_list[0][0])[i] = 0;
  for (uint32_t i = tid; i < NW * kBndWords; i += BLOCK) (&s_bnd[0][0])[i] = 0;
  if (tid == 0) {
    s_nent = 0;
    s_tokens = 0;
  }
  __syncthreads();

  uint8_t* const my_txt = s_txt[wv];
  uint16_t* const my_starts = (uint16_t*)s_list[wv];
  uint32_t* const my_ends = s_list[wv] + kWaveStarts / 2;
  uint32_t* const my_bnd = s_bnd[wv];

  // ---- the scan --------------------------------------------------------------------------
  // Tokens of [A, B). Optimistic: documents [0, nd) of the sub-window (starts in s_doff); a
  // token counts in the LDS table under its document, or marks the document as overflowed
  // (tokens of an overflowed document are not counted further). Recount: [A, B) is one
  // document; every token counts in the LDS table, else in the document's private table.
  // The first pass adds the tokens to the call's total.
  constexpr bool recount = kRecount;
  auto scan = [&](int64_t A, int64_t B, uint32_t nd) {
    const int64_t k0 = (A - base_off) / (int64_t)kStripe;
    const int64_t k1 = (B - base_off + (int64_t)kStripe - 1) / (int64_t)kStripe;
    const int64_t per = (k1 - k0 + NW - 1) / NW;
    const int64_t ka = k0 + (int64_t)wv * per;
    const int64_t kb = min(ka + per, k1);
    const int64_t nsw = kb > ka ? kb - ka : 0;
    auto stripe_pos = [&](int64_t i) -> int64_t { return base_off + (ka + i) * (int64_t)kStripe; };
    const bool pok = recount && s_pbase != ~0ull - 1;
    Slot* const priv = pok ? P.arena + s_pbase : nullptr;
    const uint64_t pmask = pok ? (uint64_t)s_pslots - 1 : 0;

    // a short word (lo, hi) of document r that found no room in the LDS table
    auto overflow = [&](uint64_t lo, uint64_t hi, uint32_t r) {
      if (!recount) {
        s_over[r] = 1;
      } else if (pok) {
        s_pused = 1;
        // (the key only places the word in this document's table, which the library alone
        // reads: a multiply-xorshift of the packed bytes instead of FNV-1a's byte loop)
        uint64_t k = (lo ^ ((hi << 29) | (hi >> 35))) * 0x9E3779B97F4A7C15ull;
        k ^= k >> 31;
        table_insert<false, true>(priv, pmask, finish_key(k, P.key_mask), short_id(lo, hi, 0), 1,
                                  hdr, ~0ull);
      }
    };
    // one short word (lo, hi) of document r, all lanes that call it together
    auto count_short = [&](uint64_t lo, uint64_t hi, uint32_t r) {
      if (!recount && s_over[r]) return;
      const uint64_t hr = recount ? hi : hi_with_doc(hi, r);
      const uint4 key = key4(lo, hr);
      const uint32_t h = red_hash(key);
      if (!red_hit(T, key, h) && !red_add(T, lo, hr, h)) overflow(lo, hi, r);
    };
    // a word whose end is not in the staged bytes, or longer than 16 bytes: from device memory
    // (limit: its end when known, else its document's end)
    auto long_word = [&](int64_t start, uint64_t limit, uint32_t r) {
      uint64_t lo, hi, h64;
      const uint64_t n = scan_word(corpus, (uint64_t)start, limit, &lo, &hi, &h64);
      if (n <= 16) {
        count_short(lo, hi, r);
      } else if (!recount) {
        s_over[r] = 1;
      } else if (pok) {
        s_pused = 1;
        table_insert<false, true>(priv, pmask, finish_key(h64, P.key_mask),
                                  long_id(corpus + start, n, 0), 1, hdr, ~0ull);
      }
    };
    auto doc_end = [&](uint32_t r) -> uint64_t { return recount ? (uint64_t)B : s_doff[r + 1]; };

    const uint4 blank = make_uint4(0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u);
    uint4 cur = blank, nx = blank;
    uint32_t carry = 0;
    int32_t rb = -1;  // last document starting before the stripe (optimistic scan)
    if (nsw > 0) {
      cur = load_text16(corpus, len, stripe_pos(0) + lane * 16);
      const int64_t q = stripe_pos(0) - 1;
      uint32_t f;
      fold_classify4(load_text4(corpus, len, q - 3), &f);
      carry = (q >= A && q < B) ? f >> 31 : 0u;
      if (!recount) {
        int32_t lo_i = -1, hi_i = (int32_t)nd;  // s_doff[lo_i] < p0 <= s_doff[hi_i]
        while (hi_i - lo_i > 1) {
          const int32_t m = (lo_i + hi_i) >> 1;
          if ((int64_t)s_doff[m] < stripe_pos(0)) lo_i = m;
          else hi_i = m;
        }
        rb = lo_i;
      }
    }
    if (nsw > 1) nx = load_text16(corpus, len, stripe_pos(1) + lane * 16);
    uint64_t tokens = 0;
    bool def = false;
    uint32_t def_s = 0, def_r = 0;

    for (int64_t i = 0; i < nsw; ++i) {
      const int64_t p0 = stripe_pos(i);
      // document starts in [p0, p0 + kStripe) (optimistic scan)
      uint32_t nb = 0;
      if (!recount) {
        while (rb + 1 < (int32_t)nd && (int64_t)s_doff[rb + 1] < p0) ++rb;
        for (int32_t j0 = rb + 1; j0 < (int32_t)nd; j0 += 64) {
          const int32_t j = j0 + lane;
          const int64_t o = j < (int32_t)nd ? (int64_t)s_doff[j] : INT64_MAX;
          const bool in = o < p0 + (int64_t)kStripe;
          if (in) atomicOr(&my_bnd[(uint32_t)(o - p0) >> 5], 1u << ((uint32_t)(o - p0) & 31));
          nb += (uint32_t)__popcll(__ballot(in));
          if (!__all(in)) break;
        }
      }
      const bool plain = nb == 0 && p0 >= A && p0 + (int64_t)kStripe <= B;

      // ---- classify ----------------------------------------------------------------------
      uint32_t w16;
      const uint4 g = classify16(cur, &w16);
      if (!plain) w16 = cut16(w16, p0 + lane * 16, A, B);
      ((uint4*)my_txt)[1 + lane] = g;
      cur = nx;
      if (i + 2 < nsw) nx = load_text16(corpus, len, stripe_pos(i + 2) + lane * 16);

      uint32_t bnd16 = 0, bnext = 0;
      if (nb) {
        wave_sync();
        bnd16 = (my_bnd[lane >> 1] >> ((lane & 1) * 16)) & 0xffffu;
        bnext = (my_bnd[(lane + 1) >> 1] >> (((lane + 1) & 1) * 16)) & 1u;  // lane 63: 0
      }

      // ---- word starts and ends ----------------------------------------------------------
      const uint32_t prev =
          (uint32_t)__builtin_amdgcn_update_dpp((int)carry, (int)(w16 >> 15), 0x138, 0xf, 0xf, false);
      const uint32_t nxt =
          (uint32_t)__builtin_amdgcn_update_dpp(1, (int)(w16 & 1u), 0x130, 0xf, 0xf, false);
      uint32_t start16 = w16 & (~((w16 << 1) | prev) | bnd16) & 0xffffu;
      const uint32_t last16 = w16 & (~((w16 >> 1) | (nxt << 15)) | (bnd16 >> 1) | (bnext << 15)) & 0xffffu;
      uint32_t ndef_j = 16;
      if (lane == 63 && start16) {
        const uint32_t j = 31 - __clz(start16);
        if ((last16 >> j) == 0) {
          ndef_j = j;
          start16 &= ~(1u << j);
        }
      }
      ((uint16_t*)my_ends)[1 + lane] = (uint16_t)last16;
      if (lane == 0) {
        const bool cont = (w16 & ~start16 & 1u) != 0;
        ((uint16_t*)my_ends)[0] = (uint16_t)(def && !cont ? 0x8000u : 0u);
      }
      // document of the token starting at staged position s (>= 16): the last document that
      // starts at or before it (empty documents share their start with the next one); only
      // the nb documents starting in this stripe can follow rb
      auto doc_at = [&](uint32_t s) -> uint32_t {
        if (recount) return 0u;
        if (nb == 0) return rb < 0 ? 0u : (uint32_t)rb;
        const int64_t pos = p0 - 16 + (int64_t)s;
        int32_t a = rb, b = rb + 1 + (int32_t)nb;  // s_doff[a] <= pos < s_doff[b]
        while (b - a > 1) {
          const int32_t m = (a + b) >> 1;
          if ((int64_t)s_doff[m] <= pos) a = m;
          else b = m;
        }
        return a < 0 ? 0u : (uint32_t)a;
      };

      // ---- compaction and tokens, kWaveStarts at a time -----------------------------------
      const uint32_t extra = (def && lane == 0) ? 1u : 0u;
      const uint32_t c = __popc(start16) + extra;
      const uint32_t incl = wave_incl_scan(c);
      const uint32_t n = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
      tokens += n;
      for (uint32_t w0 = 0; w0 < n; w0 += kWaveStarts) {
        if (extra && w0 == 0) my_starts[0] = (uint16_t)def_s;
        write_starts16(start16, incl - c + extra, w0, my_starts);
        wave_sync();
        const uint32_t nw = min(n - w0, kWaveStarts);
        // both tokens of the lane: start, length (0: no end within 32 bytes), document
        uint32_t s2[2], wl2[2], r2[2];
        bool sh2[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          s2[x] = my_starts[lane + 64 * x];
          const uint32_t q = s2[x] >> 5;
          wl2[x] = __ffs(__builtin_amdgcn_alignbit(my_ends[q + 1], my_ends[q], s2[x] & 31));
        }
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          const bool act = lane + 64 * x < nw;
          r2[x] = act ? (s2[x] < 16 ? def_r : doc_at(s2[x])) : 0u;
          sh2[x] = act && wl2[x] - 1 < 16u;
          if (act && !sh2[x]) {
            const int64_t start = p0 - 16 + (int64_t)s2[x];
            long_word(start, wl2[x] ? (uint64_t)(start + wl2[x]) : doc_end(r2[x]), r2[x]);
            wait_vmem();
          }
          if (!recount && sh2[x] && s_over[r2[x]]) sh2[x] = false;  // recounted later
        }
        // short words: packed, keyed and looked up together (the common case: the key has an
        // entry in its home group); the rest through the general insert, one at a time
        // (each LDS step reads for both tokens before either waits: pin)
        PackSrc ps[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) ps[x] = pack_read(my_txt, s2[x]);
#pragma unroll
        for (int x = 0; x < 2; ++x) pin(ps[x]);
        uint64_t lo2[2], hi2[2];
        uint4 key2[2];
        uint32_t h2[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          pack_join(ps[x], sh2[x] ? wl2[x] : 1u, &lo2[x], &hi2[x]);
          key2[x] = key4(lo2[x], recount ? hi2[x] : hi_with_doc(hi2[x], r2[x]));
          h2[x] = red_hash(key2[x]);
        }
        uint4 g2[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) g2[x] = ((const uint4*)T.slot)[red_group(h2[x])];
#pragma unroll
        for (int x = 0; x < 2; ++x) pin(g2[x]);
        uint32_t e2[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          // the first slot whose tag matches (selected from the last slot back, no branches)
          const uint32_t tag = red_tag(h2[x]);
          uint32_t m = 0u;
          m = (g2[x].w >> 13) == tag ? g2[x].w : m;
          m = (g2[x].z >> 13) == tag ? g2[x].z : m;
          m = (g2[x].y >> 13) == tag ? g2[x].y : m;
          m = (g2[x].x >> 13) == tag ? g2[x].x : m;
          e2[x] = m;
        }
        uint4 k2[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) k2[x] = T.key[e2[x] & 0x1fffu];
#pragma unroll
        for (int x = 0; x < 2; ++x) pin(k2[x]);
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          const bool eq = key_eq(k2[x], key2[x]);
          const bool hit = sh2[x] & (e2[x] != 0) & eq;
          if (hit) atomicAdd(&T.cnt[e2[x] & 0x1fffu], 1u);
          sh2[x] = sh2[x] && !hit;
        }
#pragma unroll 1
        for (int x = 0; x < 2; ++x) {
          if (sh2[x]) {
            const uint64_t hr = recount ? hi2[x] : hi_with_doc(hi2[x], r2[x]);
            if (!red_add(T, lo2[x], hr, h2[x])) {
              overflow(lo2[x], hi2[x], r2[x]);
              if (recount) wait_vmem();
            }
          }
        }
        wave_sync();
      }
      const uint32_t nj = (uint32_t)__builtin_amdgcn_readlane((int)ndef_j, 63);
      if (nj < 16) def_r = (uint32_t)__builtin_amdgcn_readfirstlane((int)doc_at(16 + 63 * 16 + nj));
      if (lane == 63) ((uint4*)my_txt)[0] = ((const uint4*)my_txt)[1 + 63];
      if (nb && lane < (int)kBndWords) my_bnd[lane] = 0;
      wave_sync();
      def = nj < 16;
      def_s = nj;
      carry = (uint32_t)__builtin_amdgcn_readlane((int)(w16 >> 15), 63);
    }
    if (def) {
      tokens += 1;
      if (lane == 0) long_word(stripe_pos(nsw) - 16 + (int64_t)def_s, doc_end(def_r), def_r);
    }
    if ((!recount || s_direct) && lane == 0 && tokens)
      atomicAdd(&s_tokens, (unsigned long long)tokens);
  };

  // ---- emission of the LDS entries of documents [0, nd) that did not overflow ------------
  auto emit = [&](uint32_t nd, uint64_t d0) {
    for (uint32_t r = tid; r < nd; r += BLOCK) s_dcur[r] = 0;
    __syncthreads();
    const uint32_t ne = min(s_nent, T.cap);
    for (uint32_t i = tid; i < ne; i += BLOCK) {
      if (!T.cnt[i]) continue;
      const uint4 k = T.key[i];
      const uint32_t r = key_doc(k);
      const uint64_t lo = (uint64_t)k.x | ((uint64_t)k.y << 32);
      const uint64_t hi = (uint64_t)(k.z & 0x7f7f7f7fu) | ((uint64_t)(k.w & 0x7f7f7f7fu) << 32);
      if (!s_over[r]) atomicAdd(&s_dcur[r], (1ull << 32) | packed_len(lo, hi));
    }
    __syncthreads();
    const uint64_t v = tid < (int)nd ? s_dcur[tid] : 0ull;
    uint32_t tn, tb;
    const uint32_t bn = block_excl_scan32<BLOCK>((uint32_t)(v >> 32), s_tmp, &tn);
    const uint32_t bb = block_excl_scan32<BLOCK>((uint32_t)v, s_tmp, &tb);
    if (tid == 0) {
      const uint64_t old = atomicAdd((unsigned long long*)&hdr->out_cursor,
                                     (unsigned long long)(((uint64_t)tn << 32) | tb));
      s_e0 = old >> 32;
      s_b0 = old & 0xffffffffull;
      if (s_e0 + tn > P.cap_e || s_b0 + tb > P.cap_b) or32(&hdr->flags, kFlagWordCap);
    }
    __syncthreads();
    const uint64_t e0 = s_e0, b0 = s_b0;
    const bool room = e0 + tn <= P.cap_e && b0 + tb <= P.cap_b;
    if (tid < (int)nd) {
      if (!s_over[tid]) {
        P.doc_ptr[d0 + tid] = e0 + bn;
        P.doc_len[d0 + tid] = v >> 32;
      }
      s_dcur[tid] = ((uint64_t)bn << 32) | bb;
    }
    __syncthreads();
    for (uint32_t i = tid; i < ne; i += BLOCK) {
      const uint32_t cnt = T.cnt[i];
      if (!cnt) continue;
      const uint4 k = T.key[i];
      const uint32_t r = key_doc(k);
      if (s_over[r]) continue;
      const uint64_t lo = (uint64_t)k.x | ((uint64_t)k.y << 32);
      const uint64_t hi = (uint64_t)(k.z & 0x7f7f7f7fu) | ((uint64_t)(k.w & 0x7f7f7f7fu) << 32);
      const uint32_t wl = packed_len(lo, hi);
      const uint64_t at = atomicAdd(&s_dcur[r], (1ull << 32) | wl);
      const uint64_t e = e0 + (at >> 32), bp = b0 + (at & 0xffffffffull);
      if (room) {
        P.word_offsets[e] = bp;
        // a document has fewer than 2^31 tokens (the corpus is below 4 GiB), so only a debug
        // bias can take an LDS count past the 32-bit width
        const uint64_t c = (uint64_t)cnt + P.count_bias;
        if (P.count_bytes == 4) {
          if (c > 0x7fffffffull) or32(&hdr->flags, kFlagCountOverflow);
          ((int32_t*)P.counts)[e] = (int32_t)c;
        } else {
          ((int64_t*)P.counts)[e] = (int64_t)c;
        }
        P.docs[e] = d0 + r;
        put_packed(P.words + bp, lo, hi, wl);
      }
    }
    __syncthreads();
  };

  // the LDS table back to empty (all threads)
  auto clear_table = [&]() {
    const uint32_t ne = min(s_nent, T.cap);
    __syncthreads();
    for (uint32_t i = tid; i < kRedSlots; i += BLOCK) T.slot[i] = 0;
    for (uint32_t i = tid; i < ne; i += BLOCK) {
      T.key[i] = make_uint4(0, 0, 0, 0);
      T.cnt[i] = 0;
    }
    __syncthreads();
    if (tid == 0) s_nent = 0;
    __syncthreads();
  };

  // ---- a document counted on its own: LDS table, then a private table ----------------------
  // Once the LDS table is full a word goes to the private table, but in the round that fills
  // it one lane may get the last entry for a word while another lane holding the same word is
  // refused: a short word of the private table can also sit in the LDS table. Its private
  // count is then added to the LDS entry and the private slot is left out of the output.
  auto recount_doc = [&](int64_t A, int64_t B, uint64_t d) {
    if (tid == 0) {
      // a document of b bytes has at most b/2 + 1 distinct words: b + 2 slots keep a small
      // document's table at most half full; large documents get b/16 slots (natural text has
      // far fewer distinct words than tokens)
      const uint64_t bytes = (uint64_t)(B - A);
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
      s_pbase = base;
      s_pslots = (uint32_t)slots;
      s_pused = 0;
      s_dcur[0] = 0;
    }
    __syncthreads();
    const bool usable = s_pbase != ~0ull - 1;
    const Slot* t = P.arena + (usable ? s_pbase : 0);
    const uint32_t slots = usable ? s_pslots : 0u;
    for (uint32_t i = tid; i < slots; i += BLOCK) P.arena[s_pbase + i] = Slot{0, 0, 0, 0};
    __syncthreads();
    if (A < B) scan(A, B, 1);
    __syncthreads();
    // the private table is read back only when a word went there (most documents fit the
    // LDS table; their cleared private table would be read twice for nothing)
    const uint32_t pslots = s_pused ? slots : 0u;
    // the document's entries and word bytes: LDS entries with a count, private slots in use
    const uint32_t ne = min(s_nent, T.cap);
    uint64_t part = 0;
    for (uint32_t i = tid; i < ne; i += BLOCK) {
      if (!T.cnt[i]) continue;
      const uint4 k = T.key[i];
      part += (1ull << 32) | packed_len((uint64_t)k.x | ((uint64_t)k.y << 32),
                                        (uint64_t)k.z | ((uint64_t)k.w << 32));
    }
    // LDS entry of a private slot's word, or -1
    auto in_lds = [&](const Slot& sl) -> int {
      if (sl.w0 & kTop) return -1;  // longer than 16 bytes: never in the LDS table
      const uint4 k = key4(sl.w0, sl.w1 & ~kTop);
      return red_find(T, k, red_hash(k));
    };
    for (uint32_t i = tid; i < pslots; i += BLOCK) {
      const Slot sl = t[i];
      if (!sl.key) continue;
      const int li = in_lds(sl);
      if (li >= 0) atomicAdd(&T.cnt[li], (uint32_t)sl.cnt);
      else part += (1ull << 32) | slot_word_len(sl);
    }
    if (part) atomicAdd(&s_dcur[0], (unsigned long long)part);
    __syncthreads();
    if (tid == 0) {
      const uint64_t tot = s_dcur[0];
      const uint64_t tn = tot >> 32, tb = tot & 0xffffffffull;
      const uint64_t old = atomicAdd((unsigned long long*)&hdr->out_cursor, (unsigned long long)tot);
      s_e0 = old >> 32;
      s_b0 = old & 0xffffffffull;
      if (s_e0 + tn > P.cap_e || s_b0 + tb > P.cap_b) or32(&hdr->flags, kFlagWordCap);
      if (usable) {
        P.doc_ptr[d] = s_e0;
        P.doc_len[d] = tn;
      }
      s_dcur[1] = tot;
      s_dcur[0] = 0;
    }
    __syncthreads();
    const uint64_t tot = s_dcur[1];
    const bool room = usable && s_e0 + (tot >> 32) <= P.cap_e && s_b0 + (tot & 0xffffffffull) <= P.cap_b;
    auto put = [&](uint64_t lo, uint64_t hi, uint32_t wl, uint64_t cnt, const uint8_t* src) {
      const uint64_t at = atomicAdd(&s_dcur[0], (1ull << 32) | wl);
      const uint64_t e = s_e0 + (at >> 32), bp = s_b0 + (at & 0xffffffffull);
      P.word_offsets[e] = bp;
      const uint64_t c = cnt + P.count_bias;
      if (P.count_bytes == 4) {
        if (c > 0x7fffffffull) or32(&hdr->flags, kFlagCountOverflow);
        ((int32_t*)P.counts)[e] = (int32_t)c;
      } else {
        ((int64_t*)P.counts)[e] = (int64_t)c;
      }
      P.docs[e] = d;
      if (src) {
        for (uint32_t q = 0; q < wl; ++q) P.words[bp + q] = (uint8_t)fold_byte(src[q]);
      } else {
        put_packed(P.words + bp, lo, hi, wl);
      }
    };
    if (room) {
      for (uint32_t i = tid; i < ne; i += BLOCK) {
        const uint32_t c = T.cnt[i];
        if (!c) continue;
        const uint4 k = T.key[i];
        const uint64_t lo = (uint64_t)k.x | ((uint64_t)k.y << 32);
        const uint64_t hi = (uint64_t)k.z | ((uint64_t)k.w << 32);
        put(lo, hi, packed_len(lo, hi), c, nullptr);
      }
      for (uint32_t i = tid; i < pslots; i += BLOCK) {
        const Slot sl = t[i];
        if (!sl.key || in_lds(sl) >= 0) continue;
        const bool lng = (sl.w0 & kTop) != 0;
        put(sl.w0, sl.w1 & ~kTop, (uint32_t)slot_word_len(sl), sl.cnt,
            lng ? (const uint8_t*)(uintptr_t)(sl.w0 & ~kTop) : nullptr);
      }
    }
    clear_table();
  };

  // documents of [d0, d0 + nd) that overflowed go to the second pass (their tokens are
  // already in the total)
  auto queue_over = [&](uint32_t nd, uint64_t d0) {
    for (uint32_t r = tid; r < nd; r += BLOCK) {
      if (s_over[r]) {
        const uint64_t q = atomicAdd((unsigned long long*)&hdr->over_n, 1ull);
        P.over_docs[q] = d0 + r;
      }
    }
    __syncthreads();
  };

  if constexpr (!kRecount) {
    // Thread 0 takes the next item as soon as it publishes the current one, so the atomic's
    // round trip overlaps the current item's work instead of starting the next item.
    uint64_t next = 0;
    if (tid == 0) next = __hip_atomic_fetch_add(&hdr->work_next, 1ull, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    while (true) {
      if (tid == 0) {
        s_item = next;
        if (next < n_win)
          next = __hip_atomic_fetch_add(&hdr->work_next, 1ull, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
      const uint64_t w = s_item;
      __syncthreads();
      if (w >= n_win) break;
      const uint64_t da = P.win_doc[w];
      const uint64_t db = min(P.win_doc[w + 1], n_docs);
      for (uint64_t d0 = da; d0 < db; d0 += kDocW) {
        const uint32_t nd = (uint32_t)min((uint64_t)kDocW, db - d0);
        for (uint32_t i = tid; i <= nd; i += BLOCK) s_doff[i] = offsets[d0 + i];
        for (uint32_t i = tid; i < nd; i += BLOCK) s_over[i] = 0;
        __syncthreads();
        // a document longer than the window is the last of its item: it is counted alone
        // after the others, with the whole LDS table to itself
        const uint64_t last_len = s_doff[nd] - s_doff[nd - 1];
        const bool big = last_len > win;
        const uint32_t ns = big ? nd - 1 : nd;
        if (ns > 0) {
          const int64_t A = (int64_t)s_doff[0], B = (int64_t)s_doff[ns];
          if (A < B) scan(A, B, ns);
          __syncthreads();
          emit(ns, d0);
          clear_table();
          queue_over(ns, d0);
        }
        if (big && P.direct_kib && last_len > ((uint64_t)P.direct_kib << 10)) {
          // large enough to overflow the LDS table: straight to the second pass, which also
          // counts its tokens
          if (tid == 0) {
            const uint64_t q = atomicAdd((unsigned long long*)&hdr->over_n, 1ull);
            P.over_docs[q] = (d0 + nd - 1) | kDirectDoc;
          }
          __syncthreads();
        } else if (big) {
          const uint64_t d = d0 + nd - 1;
          __syncthreads();
          if (tid == 0) {
            s_doff[0] = offsets[d];
            s_doff[1] = offsets[d + 1];
            s_over[0] = 0;
          }
          __syncthreads();
          scan((int64_t)s_doff[0], (int64_t)s_doff[1], 1);
          __syncthreads();
          emit(1, d);
          clear_table();
          queue_over(1, d);
        }
      }
    }
  } else {
    const uint64_t n_over = hdr->over_n;
    uint64_t next = 0;  // as in the first pass: the next queue position is taken early
    if (tid == 0) next = __hip_atomic_fetch_add(&hdr->over_next, 1ull, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    while (true) {
      if (tid == 0) {
        s_item = next;
        if (next < n_over)
          next = __hip_atomic_fetch_add(&hdr->over_next, 1ull, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
      const uint64_t q = s_item;
      __syncthreads();
      if (q >= n_over) break;
      const uint64_t e = P.over_sorted[q];
      const uint64_t d = e & kDocIdMask;
      if (tid == 0) s_direct = (e & kDirectDoc) != 0;
      recount_doc((int64_t)offsets[d], (int64_t)offsets[d + 1], d);
    }
  }
  if (tid == 0) add64(&hdr->total_tokens, s_tokens);
}

// The second pass's queue, largest document first: a counting sort over power-of-two size
// classes by one workgroup (each thread keeps the same entries in both passes). A workgroup
// that took a large document last would otherwise finish the pass alone.
__global__ __launch_bounds__(1024) void doc_order_kernel(DocParams P) {
  constexpr uint32_t kClasses = 48;  // floor(log2(bytes)), largest first
  __shared__ uint32_t s_cnt[kClasses], s_at[kClasses];
  const uint64_t n = P.hdr->over_n;
  const uint64_t* offsets = P.task->offsets;
  if (threadIdx.x < kClasses) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  for (uint64_t q = threadIdx.x; q < n; q += blockDim.x) {
    const uint64_t e = P.over_docs[q];
    const uint64_t d = e & kDocIdMask;
    const uint64_t b = offsets[d + 1] - offsets[d];
    const uint32_t c = b ? 63u - (uint32_t)__clzll((long long)b) : 0u;
    const uint32_t k = kClasses - 1 - min(c, kClasses - 1);
    P.over_docs[q] = (e & (kDirectDoc | kDocIdMask)) | ((uint64_t)k << 56);
    atomicAdd(&s_cnt[k], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = 0;
    for (uint32_t k = 0; k < kClasses; ++k) {
      s_at[k] = a;
      a += s_cnt[k];
    }
  }
  __syncthreads();
  for (uint64_t q = threadIdx.x; q < n; q += blockDim.x) {
    const uint64_t e = P.over_docs[q];
    const uint32_t k = (uint32_t)(e >> 56) & 0x7fu;
    P.over_sorted[atomicAdd(&s_at[k], 1u)] = e & (kDirectDoc | kDocIdMask);
  }
}

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

// The second pass's table takes what LDS its instance's static arrays leave (device limit per
// workgroup minus static size, less the slots), in whole multiples of 64 entries, at most
// what 13-bit entry indices reach; kDocLds when the attributes cannot be read.
uint32_t recount_entries() {
  static const uint32_t e = [] {
    int dev = 0, lim = 0;
    hipFuncAttributes a;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipFuncGetAttributes(&a, (const void*)doc_kernel<kDocBlock, true>) != hipSuccess)
      return kDocLds;
    const int64_t room = (int64_t)lim - (int64_t)a.sharedSizeBytes - (int64_t)kRedSlots * 4;
    int64_t n = room / 20 / 64 * 64;
    if (n > 8128) n = 8128;
    return n < (int64_t)kDocLds ? kDocLds : (uint32_t)n;
  }();
  return e;
}

hipError_t set_doc_smem(size_t dyn) {
  hipError_t e = hipFuncSetAttribute((const void*)doc_kernel<kDocBlock, false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)doc_kernel<kDocBlock, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)doc_dyn(recount_entries()));
  return e;
}

hipError_t launch_docs(const DocParams& P, uint32_t grid, size_t dyn, hipStream_t s) {
  hipLaunchKernelGGL(doc_validate_kernel, dim3(256), dim3(256), 0, s, P);
  hipLaunchKernelGGL(doc_windows_kernel, dim3(256), dim3(256), 0, s, P);
  hipLaunchKernelGGL((doc_kernel<kDocBlock, false>), dim3(grid), dim3(kDocBlock), dyn, s, P);
  hipLaunchKernelGGL(doc_order_kernel, dim3(1), dim3(1024), 0, s, P);
  hipLaunchKernelGGL((doc_kernel<kDocBlock, true>), dim3(grid), dim3(kDocBlock),
                     doc_dyn(P.rc_entries), s, P);
  hipLaunchKernelGGL(doc_finish_kernel, dim3(1), dim3(64), 0, s, P);
  return hipGetLastError();
}

}  // namespace wc
