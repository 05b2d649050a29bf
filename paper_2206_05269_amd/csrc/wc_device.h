// Device-side building blocks of the word counter (gfx950, wave64).
//
// Tokeniser (the paper's Section 2 / Section 3.1 normalisation, read as: ASCII case fold,
// word bytes [a-z0-9'], every other byte a delimiter, documents are hard delimiters):
// classify16() folds and classifies 16 bytes at a time in SWAR form.
//
// Word keys. A word of at most 16 bytes is carried as its folded bytes packed little-endian
// into two 64-bit values (lo, hi), zero padded; word bytes are never zero, so the packing is
// injective and the zero padding encodes the length. Longer words are carried as (pointer to
// their first byte, length).
//
// Global table. Open addressing with linear probing over S = 2^k slots of 32 bytes:
//   key  FNV-1a 64 of the folded word (continued over the document id in per-document mode);
//        0 = empty slot.
//   cnt  count (u64); per-document mode: low 32 bits count, high 32 bits document id + 1.
//   w0   short word: lo; long word: address of an occurrence | (1 << 63).
//   w1   short word: hi | (1 << 63); long word: length | (1 << 63).
// A new word claims a slot with a 64-bit CAS on key, then writes its identity fields. Each
// identity field is written exactly once, from 0 to a non-zero value, so a reader that sees
// the claimed key waits until the fields are non-zero and then compares them; no fence is
// needed and a slot never changes identity. Counts are then added with atomic adds. All
// accesses to a slot during counting are device-scope atomics (relaxed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define WC_DEV __device__ __forceinline__

namespace wc {

constexpr uint64_t kFnvOffset = 0xcbf29ce484222325ull;
constexpr uint64_t kFnvPrime = 0x100000001b3ull;
constexpr uint64_t kTop = 1ull << 63;

// error / status flags in the workspace header
constexpr uint32_t kFlagTableFull = 1u;
constexpr uint32_t kFlagBadOffsets = 2u;
constexpr uint32_t kFlagWordCap = 4u;
constexpr uint32_t kFlagCountOverflow = 8u;
constexpr uint32_t kFlagStall = 16u;  // a bounded wait inside a kernel gave up (internal error)

struct Slot {
  uint64_t key;
  uint64_t cnt;
  uint64_t w0;
  uint64_t w1;
};
static_assert(sizeof(Slot) == 32, "slot layout");

// Workspace header (device): flags and totals shared by the kernels of one call.
struct Header {
  uint32_t flags;
  uint32_t pad0;
  uint64_t total_tokens;
  uint64_t occupied;      // claimed slots
  uint64_t n_entries;
  uint64_t word_bytes;
  uint64_t max_count;
  uint64_t work_next;     // work-queue cursor (persistent launches)
  uint64_t out_cursor;    // per-document output: (entries << 32) | word bytes reserved
  uint64_t arena_next;    // per-document output: private-table slots taken
  // two-pass global count statistics: records written to the partitions, records pass 1
  // counted straight in the global table, dictionary words, (unused), records pass 2 could
  // not sum in LDS
  uint64_t stat[5];
  uint64_t over_n;        // per-document output: documents queued for the second pass
  uint64_t over_next;     // per-document output: second-pass queue cursor
};
static_assert(sizeof(Header) == 128, "header layout");

// ---------------------------------------------------------------------------------------
// atomics (device scope, relaxed)
// ---------------------------------------------------------------------------------------
WC_DEV uint64_t ld_relaxed(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
WC_DEV uint32_t ld_relaxed32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
WC_DEV void st_relaxed(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
WC_DEV void st_relaxed32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
WC_DEV uint64_t cas64(uint64_t* p, uint64_t expect, uint64_t desired) {
  __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return expect;  // the value seen before the operation
}
WC_DEV void add64(uint64_t* p, uint64_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
WC_DEV void add32(uint32_t* p, uint32_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
WC_DEV void or32(uint32_t* p, uint32_t v) {
  __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 16-byte load of streamed text (read once: non-temporal hint); p must be 16-byte aligned
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
WC_DEV uint4 load_stream16(const uint8_t* p) {
  u32x4_t v = __builtin_nontemporal_load((const u32x4_t*)p);
  return make_uint4(v.x, v.y, v.z, v.w);
}

// ---------------------------------------------------------------------------------------
// byte classes
// ---------------------------------------------------------------------------------------
WC_DEV uint32_t fold_byte(uint32_t x) { return (x - 'A' < 26u) ? x + 32u : x; }
WC_DEV bool is_word_byte(uint32_t x) {
  uint32_t f = fold_byte(x);
  return (f - 'a' < 26u) | (f - '0' < 10u) | (f == '\'');
}

// SWAR over one 32-bit word of 4 bytes: returns the folded bytes and, in *wflag, 0x80 in
// every byte position that holds a word byte.
WC_DEV uint32_t fold_classify4(uint32_t x, uint32_t* wflag) {
  const uint32_t H = 0x80808080u;
  uint32_t hi = x & H;                       // bytes >= 0x80 are never word bytes
  uint32_t l = x & 0x7f7f7f7fu;
  uint32_t lc = l | 0x20202020u;             // letters of both cases -> 0x61..0x7a
  uint32_t ge_a = lc + 0x1f1f1f1fu;          // bit7 set iff lc >= 0x61
  uint32_t gt_z = lc + 0x05050505u;          // bit7 set iff lc >= 0x7b
  uint32_t letter = ge_a & ~gt_z & ~hi & H;
  uint32_t ge_0 = l + 0x50505050u;           // bit7 iff l >= 0x30
  uint32_t gt_9 = l + 0x46464646u;           // bit7 iff l >= 0x3a
  uint32_t digit = ge_0 & ~gt_9;
  uint32_t ap = (l ^ 0x27272727u) + 0x7f7f7f7fu;  // bit7 iff l != 0x27
  uint32_t w = (letter | digit | ~ap) & ~hi & H;
  *wflag = w;
  return x | (letter >> 2);                   // set bit 5 of letters: fold A-Z
}

// 0x80-per-byte flags of 4 bytes -> 4-bit mask.
WC_DEV uint32_t movemask4(uint32_t f) {
  uint32_t s = (f >> 7) & 0x01010101u;
  s |= s >> 7;
  s |= s >> 14;
  return s & 0xfu;
}

// ---------------------------------------------------------------------------------------
// FNV-1a 64 (Fowler, Noll, Vo): h = offset basis; for each byte b: h = (h ^ b) * prime.
// The prime is 2^40 + 0x1b3.
// ---------------------------------------------------------------------------------------
WC_DEV uint64_t fnv_step(uint64_t h, uint32_t b) {
  h ^= b;
  return h * kFnvPrime;
}

// FNV-1a 64 over the n (<= 16) bytes of a packed short word.
WC_DEV uint64_t fnv_packed(uint64_t lo, uint64_t hi, uint32_t n) {
  uint64_t h = kFnvOffset;
  for (uint32_t i = 0; i < n; ++i) {
    uint64_t v = i < 8 ? lo : hi;
    h = fnv_step(h, (uint32_t)(v >> ((i & 7) * 8)) & 0xffu);
  }
  return h;
}

WC_DEV uint64_t fnv_u32(uint64_t h, uint32_t v) {
  for (int i = 0; i < 4; ++i) h = fnv_step(h, (v >> (8 * i)) & 0xffu);
  return h;
}

// Number of bytes of a packed short word.
WC_DEV uint32_t packed_len(uint64_t lo, uint64_t hi) {
  if (hi) return 8u + (uint32_t)((71 - __clzll(hi)) >> 3);
  return lo ? (uint32_t)((71 - __clzll(lo)) >> 3) : 0u;
}

// A word of <= 16 bytes can be stored packed (inline in a slot) when bytes 7 and 15 have
// their top bit clear: the top bits of the two packed halves mark long words and published
// slots. ASCII words always can; a UTF-8 word with a byte >= 0x80 there is stored as a long
// word (a reference to its bytes) instead.
WC_DEV bool packable(uint64_t lo, uint64_t hi) { return ((lo | hi) & kTop) == 0; }

// 32-bit placement hash of a packed short word and its document (+1; 0 for a global table)
// in per-workgroup LDS tables: multiply-xor of the four dwords and the document, then a
// finishing mix (constants from xxHash's primes). Only decides where an entry is probed
// first; counts never depend on it.
WC_DEV uint32_t lds_word_hash(uint64_t lo, uint64_t hi, uint32_t doc1) {
  const uint32_t a = (uint32_t)lo, b = (uint32_t)(lo >> 32), c = (uint32_t)hi,
                 d = (uint32_t)(hi >> 32);
  uint32_t h = a * 0x9E3779B1u ^ (b * 0x85EBCA77u) ^ (c * 0xC2B2AE3Du) ^ (d * 0x27D4EB2Fu) ^
               (doc1 * 0x165667B1u);
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 13;
  return h;
}

WC_DEV uint64_t finish_key(uint64_t h, uint64_t key_mask) {
  h &= key_mask;
  return h ? h : 1ull;
}

// ---------------------------------------------------------------------------------------
// folded byte compare of two long words in global memory
// ---------------------------------------------------------------------------------------
WC_DEV bool long_equal(const uint8_t* a, const uint8_t* b, uint64_t n) {
  for (uint64_t i = 0; i < n; ++i)
    if (fold_byte(a[i]) != fold_byte(b[i])) return false;
  return true;
}

// ---------------------------------------------------------------------------------------
// reading one word from device memory
// ---------------------------------------------------------------------------------------
// Scan a word from logical position s (its first byte) in device memory, up to `limit`
// (exclusive; the document end) or the first non-word byte. Returns the length, the packed
// bytes when the length is <= 16, and the FNV-1a 64 hash of the folded bytes.
WC_DEV uint64_t scan_word(const uint8_t* corpus, uint64_t s, uint64_t limit, uint64_t* plo,
                          uint64_t* phi, uint64_t* pfnv) {
  uint64_t h = kFnvOffset, lo = 0, hi = 0, n = 0;
  uint64_t p = s;
  bool done = false;
  while (!done && p < limit) {
    // the aligned 16-byte block containing p, when it lies inside [corpus, corpus + limit);
    // otherwise single bytes (limit <= corpus length, so no byte past the buffer is read)
    uintptr_t a = ((uintptr_t)(corpus + p)) & ~(uintptr_t)15;
    uint32_t first = (uint32_t)((uintptr_t)(corpus + p) - a);
    uint32_t wds[4];
    bool vec = a >= (uintptr_t)corpus && a + 16 <= (uintptr_t)(corpus + limit);
    if (vec) {
      uint4 v = *(const uint4*)a;
      wds[0] = v.x; wds[1] = v.y; wds[2] = v.z; wds[3] = v.w;
    }
    for (uint32_t j = first; j < 16; ++j) {
      if (p >= limit) { done = true; break; }
      uint32_t b = vec ? (wds[j >> 2] >> ((j & 3) * 8)) & 0xffu : (uint32_t)corpus[p];
      if (!is_word_byte(b)) { done = true; break; }
      uint32_t f = fold_byte(b);
      h = fnv_step(h, f);
      if (n < 8) lo |= (uint64_t)f << (8 * n);
      else if (n < 16) hi |= (uint64_t)f << (8 * (n - 8));
      ++n;
      ++p;
    }
  }
  *plo = lo;
  *phi = hi;
  *pfnv = h;
  return n;
}

// ---------------------------------------------------------------------------------------
// global table insert
// ---------------------------------------------------------------------------------------
// Identity of a word occurrence (plus the document in per-document mode).
struct WordId {
  uint64_t w0;    // short: lo; long: address | kTop
  uint64_t w1;    // short: hi | kTop; long: len | kTop
  uint32_t doc1;  // document + 1 (per-document mode), 0 otherwise
};

WC_DEV WordId short_id(uint64_t lo, uint64_t hi, uint32_t doc1) {
  WordId id;
  id.w0 = lo;
  id.w1 = hi | kTop;
  id.doc1 = doc1;
  return id;
}
WC_DEV WordId long_id(const uint8_t* p, uint64_t len, uint32_t doc1) {
  WordId id;
  id.w0 = (uint64_t)(uintptr_t)p | kTop;
  id.w1 = len | kTop;
  id.doc1 = doc1;
  return id;
}

// Compare a published slot against id. Slot fields must already be non-zero.
WC_DEV bool id_equal(const WordId& id, uint64_t s0, uint64_t s1, uint32_t sdoc1) {
  if (sdoc1 != id.doc1) return false;
  if (s1 != id.w1) return false;
  bool mine_long = (id.w0 & kTop) != 0;
  bool slot_long = (s0 & kTop) != 0;
  if (mine_long != slot_long) return false;
  if (!mine_long) return s0 == id.w0;
  const uint8_t* a = (const uint8_t*)(uintptr_t)(id.w0 & ~kTop);
  const uint8_t* b = (const uint8_t*)(uintptr_t)(s0 & ~kTop);
  return a == b || long_equal(a, b, id.w1 & ~kTop);
}

// Insert `n` occurrences of a word with key `key` into the table. Returns the slot index,
// or ~0 when no slot was found: after probing every slot (then the full flag is set), or
// once the full flag is set by any insert (the call then fails as full and its counts are
// discarded, so probing a crowded table further would only waste time).
// kPerDoc selects the 32-bit count layout.
//
// The probe loop is wave-uniform (it runs while any active lane has work), so a lane that
// claims a slot publishes the slot's identity inside that iteration, before any lane of its
// wave reads it; a lane that finds a claimed slot whose identity is not yet visible looks at
// the same slot again in the next iteration rather than waiting. No lane waits on a lane.
// kCasFirst claims with a compare-and-swap without reading the key first: one round trip for
// a new word, for tables where most inserts are new words and few lanes meet on one slot (a
// document's private table); shared tables read first, so that hot words do not turn every
// occurrence into an atomic on their slot.
template <bool kPerDoc, bool kCasFirst = false>
WC_DEV uint64_t table_insert(Slot* __restrict__ tab, uint64_t mask, uint64_t key,
                             const WordId& id, uint64_t n, Header* hdr, uint64_t occ_limit) {
  uint64_t i = key & mask;
  uint64_t probe = 0;
  uint64_t result = ~0ull;
  bool active = true;
  while (__any(active)) {
    Slot* s = tab + i;
    uint64_t k = 1;
    bool won = false;
    if (active) {
      k = kCasFirst ? 0 : ld_relaxed(&s->key);
      if (k == 0) {
        k = cas64(&s->key, 0, key);
        won = (k == 0);
      }
    }
    if (won) {
      // publish identity: each field goes from 0 to a non-zero value exactly once
      if (kPerDoc) st_relaxed32(((uint32_t*)&s->cnt) + 1, id.doc1);
      st_relaxed(&s->w1, id.w1);
      st_relaxed(&s->w0, id.w0);
      if (kPerDoc) add32((uint32_t*)&s->cnt, (uint32_t)n);
      else add64(&s->cnt, n);
    }
    if (occ_limit != ~0ull) {
      // claimed slots: one addition per wave (a single counter that every new word of every
      // workgroup would otherwise hit); no limit, no count
      const uint64_t wm = __ballot(won);
      if (won && __builtin_amdgcn_mbcnt_hi((uint32_t)(wm >> 32),
                                           __builtin_amdgcn_mbcnt_lo((uint32_t)wm, 0u)) == 0) {
        const uint64_t c = (uint64_t)__popcll(wm);
        uint64_t occ = __hip_atomic_fetch_add(&hdr->occupied, c, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        if (occ + c > occ_limit) or32(&hdr->flags, kFlagTableFull);
      }
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);  // publication above stays before the reads below
    if (active) {
      bool advance = true;
      if (won) {
        result = i;
        active = false;
        advance = false;
      } else if (k == key) {
        uint64_t s0 = ld_relaxed(&s->w0);
        uint64_t s1 = ld_relaxed(&s->w1);
        uint32_t sd = kPerDoc ? ld_relaxed32(((const uint32_t*)&s->cnt) + 1) : id.doc1;
        if (s0 == 0 || s1 == 0 || (kPerDoc && sd == 0)) {
          advance = false;  // claimed, identity not visible yet: look again next iteration
        } else if (id_equal(id, s0, s1, sd)) {
          if (kPerDoc) add32((uint32_t*)&s->cnt, (uint32_t)n);
          else add64(&s->cnt, n);
          result = i;
          active = false;
          advance = false;
        }
      }
      if (advance) {
        i = (i + 1) & mask;
        if (++probe > mask) {
          or32(&hdr->flags, kFlagTableFull);
          active = false;
        } else if ((probe & 63) == 0 && (ld_relaxed32(&hdr->flags) & kFlagTableFull)) {
          active = false;  // the call fails as full anyway: stop probing a crowded table
        }
      }
    }
  }
  return result;
}

}  // namespace wc
