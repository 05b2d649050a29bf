// Count kernel: the map (tokenise, hash) and the first level of the reduce (merge counts),
// fused. Section 3.1 counts each document's words in its own dictionary on CPU threads and
// Section 3.3 sums the grouped counts on the GPU; here one kernel scans the raw bytes, keeps
// a per-workgroup dictionary in LDS and merges it into one table in device memory, which is
// the GPU-resident dictionary that Section 5.2 proposes.
//
// Work split. The corpus is cut into stages of BLOCK*16 bytes at 16-byte aligned addresses;
// each workgroup scans a contiguous run of stages, 16 bytes per thread per stage (one
// 128-bit load), with the next stage's load in flight while the current one is processed.
// A word belongs to the stage holding its first byte; its owner reads past the stage end
// when the word continues (the result does not depend on where stages or workgroups cut).
//
// Per stage:
//   1. fold + classify 16 bytes per thread (SWAR), store folded bytes to LDS;
//   2. mark document starts that fall in the stage (from a precomputed per-stage cursor);
//   3. word-start / word-last bit masks from the byte classes of the thread and its
//      neighbours; block prefix sum of start counts compacts the starts into a list;
//   4. each thread takes tokens from the list: its length comes from the next word-last bit;
//      a word of <= 16 bytes is packed from LDS and counted in the LDS table; a longer word,
//      or one that runs past the stage, is read from device memory, hashed with FNV-1a 64
//      and inserted straight into the global table;
//   5. when the LDS table passes its load limit it is flushed: every entry is hashed with
//      FNV-1a 64 and added to the global table with one atomic add.
#include "wc_internal.h"

namespace wc {

struct LdsTable {
  uint64_t* lo;     // claim word: packed bytes 0..7 (0 = empty)
  uint64_t* hi;     // packed bytes 8..15 | kTop (0 until published)
  uint32_t* cnt;
  uint32_t* doc1;   // per-document mode: document + 1 (0 until published)
  uint32_t mask;
  uint32_t shift;   // 32 - log2(entries)
};


WC_DEV uint64_t lds_ld64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
WC_DEV uint32_t lds_ld32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Count one occurrence of a short word in the LDS table. Returns false when no slot was
// found within kMaxProbe probes (the caller then counts it in the global table).
//
// The probe loop is wave-uniform: it runs while any active lane of the wave still has work,
// so a lane that claims a slot publishes its identity inside the same iteration, before any
// lane of the wave reads it; a lane that finds a claimed but unpublished slot looks at it
// again in the next iteration instead of waiting. No lane ever waits on another lane.
template <bool kPerDoc>
WC_DEV bool lds_insert(const LdsTable& L, uint64_t lo, uint64_t hi, uint32_t doc1,
                       uint32_t* used) {
  constexpr int kMaxProbe = 32;
  const uint64_t hiw = hi | kTop;
  uint32_t i = lds_word_hash(lo, hi, doc1) >> L.shift;
  int probe = 0;
  bool active = true, ok = false;
  while (__any(active)) {
    uint64_t old = 1;
    if (active) old = atomicCAS((unsigned long long*)&L.lo[i], 0ull, (unsigned long long)lo);
    const bool won = active && old == 0;
    if (won) {
      if (kPerDoc) __hip_atomic_store(&L.doc1[i], doc1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __hip_atomic_store(&L.hi[i], hiw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      atomicAdd(&L.cnt[i], 1u);
      atomicAdd(used, 1u);
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);  // publication above stays before the reads below
    if (active) {
      bool advance = true;
      if (won) {
        ok = true;
        active = false;
        advance = false;
      } else if (old == lo) {
        uint64_t sh = lds_ld64(&L.hi[i]);
        uint32_t sd = kPerDoc ? lds_ld32(&L.doc1[i]) : 1u;
        if (sh == 0 || sd == 0) {
          advance = false;  // claimed, not yet published: look again next iteration
        } else if (sh == hiw && (!kPerDoc || sd == doc1)) {
          atomicAdd(&L.cnt[i], 1u);
          ok = true;
          active = false;
          advance = false;
        }
      }
      if (advance) {
        i = (i + 1) & L.mask;
        if (++probe >= kMaxProbe) active = false;
      }
    }
  }
  return ok;
}

template <bool kPerDoc>
WC_DEV uint64_t short_key(uint64_t lo, uint64_t hi, uint32_t doc1, uint64_t key_mask) {
  uint64_t h = fnv_packed(lo, hi, packed_len(lo, hi));
  if (kPerDoc) h = fnv_u32(h, doc1 - 1);
  return finish_key(h, key_mask);
}

// ---- UTF-8 tokeniser (the "other languages" of Section 5.2) ---------------------------------
// A byte is a word byte when it belongs to a well-formed UTF-8 sequence (Unicode Standard,
// Table 3-7) that lies inside one document and whose code point is a word character: the
// ASCII word bytes, or any code point from U+0080 up except U+0080..U+00BF, U+00D7, U+00F7,
// U+2000..U+206F, U+3000..U+303F and U+FEFF. Folding stays ASCII-only.
WC_DEV bool utf8_word_cp(uint32_t cp) {
  if (cp <= 0xBF || cp == 0xD7 || cp == 0xF7 || cp == 0xFEFF) return false;
  if (cp >= 0x2000 && cp <= 0x206F) return false;
  if (cp >= 0x3000 && cp <= 0x303F) return false;
  return true;
}

// Sequence length (2..4) of a lead byte c, the allowed range of the byte after it and the
// lead's code point bits; 0 when c does not start a multi-byte sequence.
WC_DEV uint32_t utf8_lead(uint32_t c, uint32_t* lo2, uint32_t* hi2, uint32_t* v) {
  *lo2 = 0x80u;
  *hi2 = 0xBFu;
  if (c >= 0xC2u && c <= 0xDFu) {
    *v = c & 0x1Fu;
    return 2;
  }
  if (c >= 0xE0u && c <= 0xEFu) {
    *v = c & 0x0Fu;
    if (c == 0xE0u) *lo2 = 0xA0u;
    if (c == 0xEDu) *hi2 = 0x9Fu;
    return 3;
  }
  if (c >= 0xF0u && c <= 0xF4u) {
    *v = c & 0x07u;
    if (c == 0xF0u) *lo2 = 0x90u;
    if (c == 0xF4u) *hi2 = 0x8Fu;
    return 4;
  }
  return 0;
}

// Word flag of the byte at logical position q under the UTF-8 reading. Bytes exist in
// [lo, hi); byte_at(x) reads one, starts_at(x) tells whether a document starts at x (a
// sequence never spans a document start).
template <class ByteAt, class StartsAt>
WC_DEV uint32_t utf8_word_byte(int64_t q, int64_t lo, int64_t hi, ByteAt byte_at,
                               StartsAt starts_at) {
  if (q < lo || q >= hi) return 0u;
  uint32_t c = byte_at(q);
  if (c < 0x80u) return is_word_byte(c) ? 1u : 0u;
  int64_t j = q;
  for (int k = 0; c >= 0x80u && c <= 0xBFu; ++k) {  // a continuation: step back to its lead
    if (k == 3 || j == lo || starts_at(j)) return 0u;
    c = byte_at(--j);
  }
  uint32_t lo2, hi2, v;
  const uint32_t n = utf8_lead(c, &lo2, &hi2, &v);
  if (n == 0 || j + (int64_t)n <= q) return 0u;
  for (uint32_t t = 1; t < n; ++t) {
    const int64_t x = j + t;
    if (x >= hi || starts_at(x)) return 0u;
    const uint32_t d = byte_at(x);
    if (d < (t == 1 ? lo2 : 0x80u) || d > (t == 1 ? hi2 : 0xBFu)) return 0u;
    v = (v << 6) | (d & 0x3Fu);
  }
  return utf8_word_cp(v) ? 1u : 0u;
}

// A document starts at logical position q (some offsets[d] == q, 1 <= d <= n_docs).
WC_DEV bool doc_starts_at(const uint64_t* offsets, uint64_t n_docs, int64_t q) {
  uint64_t a = 1, b = n_docs + 1;
  while (a < b) {
    const uint64_t m = (a + b) >> 1;
    if ((int64_t)offsets[m] < q) a = m + 1;
    else b = m;
  }
  return a <= n_docs && (int64_t)offsets[a] == q;
}

// A word starting at s that may run past the staged bytes, read from device memory under the
// UTF-8 reading (up to `limit`, the document end): length, packed bytes (<= 16), FNV-1a 64.
WC_DEV uint64_t scan_word_utf8(const uint8_t* corpus, uint64_t s, uint64_t limit, uint64_t* plo,
                               uint64_t* phi, uint64_t* pfnv) {
  auto byte_at = [&](int64_t x) -> uint32_t { return corpus[x]; };
  auto starts_at = [&](int64_t) -> bool { return false; };  // none inside [s, limit)
  uint64_t h = kFnvOffset, lo = 0, hi = 0, n = 0;
  for (uint64_t p = s; p < limit; ++p) {
    if (!utf8_word_byte((int64_t)p, (int64_t)s, (int64_t)limit, byte_at, starts_at)) break;
    const uint32_t f = fold_byte(corpus[p]);
    h = fnv_step(h, f);
    if (n < 8) lo |= (uint64_t)f << (8 * n);
    else if (n < 16) hi |= (uint64_t)f << (8 * (n - 8));
    ++n;
  }
  *plo = lo;
  *phi = hi;
  *pfnv = h;
  return n;
}

template <int BLOCK, bool kPerDoc, bool kUtf8>
__global__ __launch_bounds__(BLOCK) void count_kernel(CountParams P) {
  constexpr int STAGE = BLOCK * 16;
  constexpr int NWAVE = BLOCK / 64;
  constexpr int MAXB = 256;  // document starts kept per stage for per-document lookups
  __shared__ uint4 s_txt4[STAGE / 16 + 2];        // folded bytes of the stage (+32 B pad)
  __shared__ uint16_t s_wm[BLOCK];                // word-byte mask per thread
  __shared__ uint16_t s_last[BLOCK + 1];          // word-last mask per thread
  __shared__ uint32_t s_bnd[STAGE / 32 + 2];      // document start at byte i (0..STAGE)
  __shared__ uint16_t s_starts[STAGE];            // compacted token starts
  __shared__ uint32_t s_wsum[NWAVE];
  __shared__ uint16_t s_boff[kPerDoc ? MAXB : 1]; // stage-relative document starts
  __shared__ uint32_t s_used;
  __shared__ uint32_t s_carry[2];                 // word-byte flag of the previous stage's last byte
  __shared__ uint32_t s_next_w;                   // word-byte flag of the next stage's first byte
  __shared__ uint32_t s_ntok;
  extern __shared__ __align__(16) uint8_t s_dyn[];
  const uint8_t* s_txt = (const uint8_t*)s_txt4;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  Header* hdr = P.hdr;

  if (ld_relaxed32(&hdr->flags) & kFlagBadOffsets) return;

  LdsTable L;
  const uint32_t E = P.lds_entries;
  L.lo = (uint64_t*)s_dyn;
  L.hi = L.lo + E;
  L.cnt = (uint32_t*)(L.hi + E);
  L.doc1 = L.cnt + E;
  L.mask = E - 1;
  L.shift = 32 - (31 - __clz(E));
  const bool use_lds = !P.no_lds;

  for (uint32_t i = tid; i < E; i += BLOCK) {
    L.lo[i] = 0;
    L.hi[i] = 0;
    L.cnt[i] = 0;
    if (kPerDoc) L.doc1[i] = 0;
  }
  if (tid == 0) s_used = 0;

  const uint64_t st0 = (uint64_t)blockIdx.x * P.stages_per_wg;
  const uint64_t st1 = min(st0 + P.stages_per_wg, P.n_stages);
  if (st0 >= st1) return;

  const int64_t R0 = (int64_t)P.offsets[0], R1 = (int64_t)P.offsets[P.n_docs];
  const int64_t len = (int64_t)P.len;

  // logical position of byte j of thread t in stage k
  auto stage_pos = [&](uint64_t k) -> int64_t { return P.base_off + (int64_t)(k * STAGE); };

  auto load16 = [&](uint64_t k) -> uint4 {
    int64_t p = stage_pos(k) + tid * 16;
    uint4 v;
    if (p >= 0 && p + 16 <= len) {
      v = *(const uint4*)(P.corpus + p);
    } else {
      uint32_t w[4] = {0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u};
      for (int j = 0; j < 16; ++j) {
        int64_t q = p + j;
        if (q >= 0 && q < len) {
          uint32_t b = P.corpus[q];
          w[j >> 2] = (w[j >> 2] & ~(0xffu << ((j & 3) * 8))) | (b << ((j & 3) * 8));
        }
      }
      v = make_uint4(w[0], w[1], w[2], w[3]);
    }
    return v;
  };

  // word-byte flag of the byte at logical position q (0 outside the document range)
  auto wflag_at = [&](int64_t q) -> uint32_t {
    if (q < R0 || q >= R1 || q < 0 || q >= len) return 0u;
    return is_word_byte(P.corpus[q]) ? 1u : 0u;
  };

  // UTF-8 reading of a byte outside the staged stage: device memory, document starts by search
  auto g_byte = [&](int64_t x) -> uint32_t { return P.corpus[x]; };
  auto g_start = [&](int64_t x) -> bool { return doc_starts_at(P.offsets, P.n_docs, x); };
  if (tid == 0) {
    const int64_t q = stage_pos(st0) - 1;
    s_carry[(st0 & 1) ^ 1] = kUtf8 ? utf8_word_byte(q, R0, R1, g_byte, g_start) : wflag_at(q);
  }
  for (int i = tid; i < STAGE / 32 + 2; i += BLOCK) s_bnd[i] = 0;
  // the boundary bitmap is zero before any thread marks the first stage's document starts
  // (a slow wave could otherwise clear a word after another wave marked a bit in it)
  __syncthreads();

  uint4 cur = load16(st0);
  uint64_t tokens = 0;

  for (uint64_t k = st0; k < st1; ++k) {
    const int64_t ls = stage_pos(k);
    const int64_t le = ls + STAGE;
    uint4 nxt = make_uint4(0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u);
    if (k + 1 < st1) nxt = load16(k + 1);

    // ---- 1. fold + classify --------------------------------------------------------
    uint32_t f0, f1, f2, f3;
    uint32_t g0 = fold_classify4(cur.x, &f0), g1 = fold_classify4(cur.y, &f1);
    uint32_t g2 = fold_classify4(cur.z, &f2), g3 = fold_classify4(cur.w, &f3);
    uint32_t w16 = movemask4(f0) | (movemask4(f1) << 4) | (movemask4(f2) << 8) |
                   (movemask4(f3) << 12);
    const int64_t p = ls + tid * 16;
    if (!kUtf8 && (p < R0 || p + 16 > R1)) {
      int64_t lo_cut = R0 - p, hi_cut = R1 - p;
      uint32_t m = 0xffffu;
      if (lo_cut > 0) m &= lo_cut >= 16 ? 0u : (0xffffu << lo_cut) & 0xffffu;
      if (hi_cut < 16) m &= hi_cut <= 0 ? 0u : (0xffffu >> (16 - hi_cut));
      w16 &= m;
    }
    s_txt4[tid] = make_uint4(g0, g1, g2, g3);
    if (!kUtf8) s_wm[tid] = (uint16_t)w16;
    if (!kUtf8 && tid == 0) {
      // flag of the first byte of the next stage
      int64_t q = le;
      uint32_t nw;
      if (k + 1 < st1) {
        nw = (q >= R0 && q < R1 && q < len) ? (is_word_byte(nxt.x & 0xffu) ? 1u : 0u) : 0u;
      } else {
        nw = wflag_at(q);
      }
      s_next_w = nw;
    }

    // ---- 2. document starts in [ls, le] ----------------------------------------------
    const uint64_t c0 = P.stage_doc[k];       // first document start >= ls
    const uint64_t c1 = P.stage_doc[k + 1];   // first document start >= le
    const uint64_t nb = c1 - c0;
    for (uint64_t j = tid; j < nb; j += BLOCK) {
      uint64_t rel = P.offsets[c0 + j] - (uint64_t)ls;
      atomicOr(&s_bnd[rel >> 5], 1u << (rel & 31));
      if (kPerDoc && j < MAXB) s_boff[j] = (uint16_t)rel;
    }
    if (tid == 0 && c1 <= P.n_docs && (int64_t)P.offsets[c1] == le)
      atomicOr(&s_bnd[STAGE >> 5], 1u);
    __syncthreads();

    if (kUtf8) {
      // ---- 2b. UTF-8 word bytes: needs the staged bytes around each byte and the document
      // starts of the stage (a sequence never spans one)
      auto byte_at = [&](int64_t x) -> uint32_t {
        return (x >= ls && x < le) ? (uint32_t)s_txt[x - ls] : (uint32_t)P.corpus[x];
      };
      auto starts_at = [&](int64_t x) -> bool {
        if (x >= ls && x <= le) return (s_bnd[(x - ls) >> 5] >> ((x - ls) & 31)) & 1u;
        return doc_starts_at(P.offsets, P.n_docs, x);
      };
      w16 = 0;
      for (int j = 0; j < 16; ++j) w16 |= utf8_word_byte(p + j, R0, R1, byte_at, starts_at) << j;
      s_wm[tid] = (uint16_t)w16;
      if (tid == 0) s_next_w = utf8_word_byte(le, R0, R1, byte_at, starts_at);
      __syncthreads();
    }

    // ---- 3. start / last masks, compaction --------------------------------------------
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
    for (int d = 1; d < 64; d <<= 1) {
      uint32_t y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    uint32_t base = 0, total = 0;
    for (int w = 0; w < NWAVE; ++w) {
      uint32_t v = s_wsum[w];
      base += w < wave ? v : 0u;
      total += v;
    }
    uint32_t o = base + incl - cnt;
    uint32_t m = start16;
    while (m) {
      int j = __ffs(m) - 1;
      s_starts[o++] = (uint16_t)(tid * 16 + j);
      m &= m - 1;
    }
    tokens += (tid == 0) ? total : 0u;
    __syncthreads();
    // the boundary bitmap has been read (step 3): clear it for the next stage
    for (int i = tid; i < STAGE / 32 + 2; i += BLOCK) s_bnd[i] = 0;

    // ---- 4. tokens -------------------------------------------------------------------
    for (uint32_t t = tid; t < total; t += BLOCK) {
      const uint32_t s = s_starts[t];
      // next word-last bit at or after s
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
      uint32_t doc1 = 0;
      if (kPerDoc) {
        // document of position ls + s: (first start > ls + s) - 1
        uint64_t cnt_le;
        if (nb <= MAXB) {
          uint32_t lo_i = 0, hi_i = (uint32_t)nb;
          while (lo_i < hi_i) {
            uint32_t mid = (lo_i + hi_i) >> 1;
            if (s_boff[mid] <= s) lo_i = mid + 1; else hi_i = mid;
          }
          cnt_le = lo_i;
        } else {
          uint64_t lo_i = 0, hi_i = nb;
          while (lo_i < hi_i) {
            uint64_t mid = (lo_i + hi_i) >> 1;
            if (P.offsets[c0 + mid] <= (uint64_t)(ls + s)) lo_i = mid + 1; else hi_i = mid;
          }
          cnt_le = lo_i;
        }
        doc1 = (uint32_t)(c0 + cnt_le);  // (doc index) + 1
      }
      const uint32_t wl = e - s + 1;
      if (!crosses && wl <= 16) {
        // pack from LDS: 20 bytes starting at the aligned dword of s
        const uint32_t* tw = (const uint32_t*)s_txt;
        uint32_t di = s >> 2, sh = s & 3;
        uint32_t d0 = tw[di], d1 = tw[di + 1], d2 = tw[di + 2], d3 = tw[di + 3], d4 = tw[di + 4];
        uint32_t k0 = __builtin_amdgcn_alignbyte(d1, d0, sh);
        uint32_t k1 = __builtin_amdgcn_alignbyte(d2, d1, sh);
        uint32_t k2 = __builtin_amdgcn_alignbyte(d3, d2, sh);
        uint32_t k3 = __builtin_amdgcn_alignbyte(d4, d3, sh);
        uint64_t lo = (uint64_t)k0 | ((uint64_t)k1 << 32);
        uint64_t hi = (uint64_t)k2 | ((uint64_t)k3 << 32);
        if (wl < 8) { lo &= (1ull << (8 * wl)) - 1; hi = 0; }
        else if (wl == 8) { hi = 0; }
        else if (wl < 16) { hi &= (1ull << (8 * (wl - 8))) - 1; }
        if (kUtf8 && !packable(lo, hi)) {
          // a byte >= 0x80 where the packed form keeps its marks: stored as a long word
          uint64_t h = fnv_packed(lo, hi, wl);
          if (kPerDoc) h = fnv_u32(h, doc1 - 1);
          table_insert<kPerDoc>(P.table, P.mask, finish_key(h, P.key_mask),
                                long_id(P.corpus + (ls + s), wl, doc1), 1, hdr, P.occ_limit);
        } else {
          bool done = use_lds && lds_insert<kPerDoc>(L, lo, hi, doc1, &s_used);
          if (!done) {
            uint64_t key = short_key<kPerDoc>(lo, hi, doc1, P.key_mask);
            table_insert<kPerDoc>(P.table, P.mask, key, short_id(lo, hi, doc1), 1, hdr,
                                  P.occ_limit);
          }
        }
      } else {
        // long word, or a word that continues past the stage: read it from device memory
        uint64_t start = (uint64_t)(ls + s);
        uint64_t limit = (uint64_t)R1;
        if (crosses) {
          uint64_t nd = P.offsets[c1 <= P.n_docs ? c1 : P.n_docs];
          if (nd > (uint64_t)le && nd < limit) limit = nd;
        } else {
          limit = start + wl;
        }
        uint64_t lo, hi, h;
        uint64_t n = kUtf8 ? scan_word_utf8(P.corpus, start, limit, &lo, &hi, &h)
                           : scan_word(P.corpus, start, limit, &lo, &hi, &h);
        if (n <= 16 && (!kUtf8 || packable(lo, hi))) {
          bool done = use_lds && lds_insert<kPerDoc>(L, lo, hi, doc1, &s_used);
          if (!done) {
            uint64_t key = short_key<kPerDoc>(lo, hi, doc1, P.key_mask);
            table_insert<kPerDoc>(P.table, P.mask, key, short_id(lo, hi, doc1), 1, hdr, P.occ_limit);
          }
        } else {
          if (kPerDoc) h = fnv_u32(h, doc1 - 1);
          uint64_t key = finish_key(h, P.key_mask);
          table_insert<kPerDoc>(P.table, P.mask, key, long_id(P.corpus + start, n, doc1), 1, hdr,
                                P.occ_limit);
        }
      }
    }
    __syncthreads();

    // ---- 5. flush ---------------------------------------------------------------------
    const bool last_stage = (k + 1 == st1);
    if (use_lds && (last_stage || (P.policy == WC_FLUSH_ALL && s_used > P.lds_flush_at))) {
      for (uint32_t i = tid; i < E; i += BLOCK) {
        uint32_t c = L.cnt[i];
        if (c) {
          uint64_t lo = L.lo[i], hi = L.hi[i] & ~kTop;
          uint32_t d1 = kPerDoc ? L.doc1[i] : 0u;
          uint64_t key = short_key<kPerDoc>(lo, hi, d1, P.key_mask);
          table_insert<kPerDoc>(P.table, P.mask, key, short_id(lo, hi, d1), c, hdr, P.occ_limit);
          L.cnt[i] = 0;
        }
        L.lo[i] = 0;
        L.hi[i] = 0;
        if (kPerDoc) L.doc1[i] = 0;
      }
      __syncthreads();
      if (tid == 0) s_used = 0;
      __syncthreads();
    }
    cur = nxt;
  }
  if (tid == 0) add64(&hdr->total_tokens, tokens);
}

// First document start at or after the start of each stage (one binary search per stage).
__global__ void stage_doc_kernel(const uint64_t* __restrict__ offsets, uint64_t n_docs,
                                 int64_t base_off, uint32_t stage, uint64_t n_stages,
                                 uint64_t* __restrict__ out) {
  uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (k > n_stages) return;
  int64_t ls = base_off + (int64_t)(k * stage);
  uint64_t lo = 0, hi = n_docs + 1;  // search offsets[0..n_docs]
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    if ((int64_t)offsets[mid] < ls) lo = mid + 1; else hi = mid;
  }
  out[k] = lo;
}

// Offsets must be non-decreasing and end inside the corpus.
__global__ void validate_offsets_kernel(const uint64_t* __restrict__ offsets, uint64_t n_docs,
                                        uint64_t len, Header* hdr) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i > n_docs) return;
  bool bad = false;
  if (i < n_docs && offsets[i] > offsets[i + 1]) bad = true;
  if (i == n_docs && offsets[i] > len) bad = true;
  if (bad) or32(&hdr->flags, kFlagBadOffsets);
}

__global__ void read_range_kernel(const uint64_t* offsets, uint64_t n_docs, uint64_t* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    out[0] = offsets[0];
    out[1] = offsets[n_docs];
  }
}

template <bool kPerDoc, bool kUtf8>
static hipError_t launch_count_t(const CountParams& P, uint32_t grid, uint32_t block,
                                 size_t dyn, hipStream_t s) {
  if (block == 512) {
    hipLaunchKernelGGL((count_kernel<512, kPerDoc, kUtf8>), dim3(grid), dim3(512), dyn, s, P);
  } else {
    hipLaunchKernelGGL((count_kernel<256, kPerDoc, kUtf8>), dim3(grid), dim3(256), dyn, s, P);
  }
  return hipGetLastError();
}

hipError_t launch_count(const CountParams& P, bool per_doc, uint32_t grid, uint32_t block,
                        size_t dyn, hipStream_t s) {
  if (P.utf8)
    return per_doc ? launch_count_t<true, true>(P, grid, block, dyn, s)
                   : launch_count_t<false, true>(P, grid, block, dyn, s);
  return per_doc ? launch_count_t<true, false>(P, grid, block, dyn, s)
                 : launch_count_t<false, false>(P, grid, block, dyn, s);
}

hipError_t set_count_smem(uint32_t block, size_t dyn) {
  const void* k512[4] = {(const void*)count_kernel<512, false, false>,
                         (const void*)count_kernel<512, true, false>,
                         (const void*)count_kernel<512, false, true>,
                         (const void*)count_kernel<512, true, true>};
  const void* k256[4] = {(const void*)count_kernel<256, false, false>,
                         (const void*)count_kernel<256, true, false>,
                         (const void*)count_kernel<256, false, true>,
                         (const void*)count_kernel<256, true, true>};
  hipError_t e = hipSuccess;
  for (int i = 0; i < 4 && e == hipSuccess; ++i)
    e = hipFuncSetAttribute(block == 512 ? k512[i] : k256[i],
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
  return e;
}

hipError_t launch_stage_doc(const uint64_t* offsets, uint64_t n_docs, int64_t base_off,
                            uint32_t stage, uint64_t n_stages, uint64_t* out, hipStream_t s) {
  uint64_t n = n_stages + 1;
  uint32_t grid = (uint32_t)((n + 255) / 256);
  hipLaunchKernelGGL(stage_doc_kernel, dim3(grid), dim3(256), 0, s, offsets, n_docs, base_off,
                     stage, n_stages, out);
  return hipGetLastError();
}

hipError_t launch_validate(const uint64_t* offsets, uint64_t n_docs, uint64_t len, Header* hdr,
                           hipStream_t s) {
  uint64_t n = n_docs + 1;
  uint32_t grid = (uint32_t)((n + 255) / 256);
  hipLaunchKernelGGL(validate_offsets_kernel, dim3(grid), dim3(256), 0, s, offsets, n_docs, len,
                     hdr);
  return hipGetLastError();
}

}  // namespace wc
