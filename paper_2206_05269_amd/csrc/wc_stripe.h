// Pieces of the 1 KiB-stripe text scanner and of the LDS word table shared by the two-pass
// global count and the per-document count: staged text loads, SWAR classification, word
// packing from LDS, wave scans, the start list and the word-end bitmap of a stripe, and the
// tag-slot LDS table of 16-byte keys.
#pragma once

#include "wc_internal.h"

namespace wc {

constexpr uint32_t kLongEnd = 0x7ffu;                 // word end not within the staged bytes
constexpr uint32_t kBndWords = kStripeText / 32 + 1;  // document-start bits of a stripe

WC_DEV uint4 key4(uint64_t lo, uint64_t hi) {
  return make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
}

// 16 bytes of the logical text at p; bytes outside [0, len) read as spaces.
WC_DEV uint4 load_text16(const uint8_t* corpus, uint64_t len, int64_t p) {
  if (p >= 0 && p + 16 <= (int64_t)len) return load_stream16(corpus + p);
  uint32_t w[4] = {0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u};
#pragma unroll 1
  for (int j = 0; j < 16; ++j) {
    int64_t q = p + j;
    if (q >= 0 && q < (int64_t)len) {
      uint32_t b = corpus[q];
      w[j >> 2] = (w[j >> 2] & ~(0xffu << ((j & 3) * 8))) | (b << ((j & 3) * 8));
    }
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Folded bytes and 16-bit word mask of 16 text bytes.
WC_DEV uint4 classify16(uint4 v, uint32_t* w16) {
  uint32_t f0, f1, f2, f3;
  uint4 g;
  g.x = fold_classify4(v.x, &f0);
  g.y = fold_classify4(v.y, &f1);
  g.z = fold_classify4(v.z, &f2);
  g.w = fold_classify4(v.w, &f3);
  *w16 = movemask4(f0) | (movemask4(f1) << 4) | (movemask4(f2) << 8) | (movemask4(f3) << 12);
  return g;
}

// keep the bits of 16 bytes at logical position p that lie in [a, b)
WC_DEV uint32_t cut16(uint32_t w16, int64_t p, int64_t a, int64_t b) {
  if (p >= a && p + 16 <= b) return w16;
  int64_t lo_cut = a - p, hi_cut = b - p;
  uint32_t m = 0xffffu;
  if (lo_cut > 0) m &= lo_cut >= 16 ? 0u : (0xffffu << lo_cut) & 0xffffu;
  if (hi_cut < 16) m &= hi_cut <= 0 ? 0u : (0xffffu >> (16 - hi_cut));
  return w16 & m;
}

// Keeps a value in VGPRs at this point of the program: every load that produces it is issued
// before it, and the optimiser can neither split a wide LDS read into parts read one after
// another nor move the read into a branch. Pinning the results of several independent reads
// together makes a wave wait once for all of them.
WC_DEV void pin(uint32_t& v) { __asm__ volatile("" : "+v"(v)); }
WC_DEV void pin(uint4& v) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // one register quad
  u32x4 t = {v.x, v.y, v.z, v.w};
  __asm__ volatile("" : "+v"(t));
  v = make_uint4(t.x, t.y, t.z, t.w);
}

// a == b for two 16-byte keys, as one OR of XORs (pinned, so that it is not turned back into
// four compares and branches)
WC_DEV bool key_eq(const uint4 a, const uint4 b) {
  uint32_t d = (a.x ^ b.x) | (a.y ^ b.y) | (a.z ^ b.z) | (a.w ^ b.w);
  pin(d);
  return d == 0;
}

// Packing a word of the staged text in two steps, so that the LDS reads of several words can
// be issued together: pack_read takes the five dwords that hold the 16 bytes from byte s,
// pack_join aligns them and clears the bytes past the word (1 <= wl <= 16, all staged).
struct PackSrc {
  uint32_t d[5];
  uint32_t sh;
};
WC_DEV PackSrc pack_read(const uint8_t* s_txt, uint32_t s) {
  const uint32_t* tw = (const uint32_t*)s_txt;
  const uint32_t di = s >> 2;
  PackSrc r;
#pragma unroll
  for (int j = 0; j < 5; ++j) r.d[j] = tw[di + j];
  r.sh = s & 3;
  return r;
}
WC_DEV void pin(PackSrc& r) {
#pragma unroll
  for (int j = 0; j < 5; ++j) pin(r.d[j]);
}
// the bytes past the word cleared with computed shifts
WC_DEV void pack_join(const PackSrc& r, uint32_t wl, uint64_t* lo, uint64_t* hi) {
  uint64_t a = (uint64_t)__builtin_amdgcn_alignbyte(r.d[1], r.d[0], r.sh) |
               ((uint64_t)__builtin_amdgcn_alignbyte(r.d[2], r.d[1], r.sh) << 32);
  uint64_t b = (uint64_t)__builtin_amdgcn_alignbyte(r.d[3], r.d[2], r.sh) |
               ((uint64_t)__builtin_amdgcn_alignbyte(r.d[4], r.d[3], r.sh) << 32);
  const uint32_t ka = wl < 8 ? 64 - 8 * wl : 0u;    // bits of a past the word
  const uint32_t kb = wl < 16 ? 128 - 8 * wl : 0u;  // bits of b past the word (>= 64: all)
  a = (a << ka) >> ka;
  b = kb >= 64 ? 0ull : (b << kb) >> kb;
  *lo = a;
  *hi = b;
}
// the bytes past the word cleared with m, the word length's entry of the init_len_masks table
WC_DEV void pack_join(const PackSrc& r, const uint4 m, uint64_t* lo, uint64_t* hi) {
  const uint32_t a0 = __builtin_amdgcn_alignbyte(r.d[1], r.d[0], r.sh) & m.x;
  const uint32_t a1 = __builtin_amdgcn_alignbyte(r.d[2], r.d[1], r.sh) & m.y;
  const uint32_t a2 = __builtin_amdgcn_alignbyte(r.d[3], r.d[2], r.sh) & m.z;
  const uint32_t a3 = __builtin_amdgcn_alignbyte(r.d[4], r.d[3], r.sh) & m.w;
  *lo = (uint64_t)a0 | ((uint64_t)a1 << 32);
  *hi = (uint64_t)a2 | ((uint64_t)a3 << 32);
}

// Packed bytes of the word at byte s of the staged text (1 <= wl <= 16 bytes, all staged).
WC_DEV void pack_word(const uint8_t* s_txt, uint32_t s, uint32_t wl, uint64_t* lo, uint64_t* hi) {
  pack_join(pack_read(s_txt, s), wl, lo, hi);
}

// Byte masks of the first n of 16 bytes, n = 0..16 (one uint4 each), for pack_join.
WC_DEV void init_len_masks(uint4* m, uint32_t tid, uint32_t nthreads) {
  for (uint32_t n = tid; n <= 16; n += nthreads) {
    uint32_t w[4];
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
      const uint32_t nb = n > 4 * k ? min(n - 4 * k, 4u) : 0u;
      w[k] = nb >= 4 ? 0xffffffffu : (1u << (8 * nb)) - 1u;
    }
    m[n] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

// Inclusive prefix sum over the 64 lanes of a wave: shifts within each 16-lane row, then the
// row broadcasts of lanes 15 and 31 (lanes whose source is outside the row, and rows the mask
// leaves out, add 0).
WC_DEV uint32_t wave_incl_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  // opaque to the optimiser: a caller that subtracts its own term must not have the sum
  // rebuilt from the shifted partials (which keeps each shift a separate move)
  __asm__ volatile("" : "+v"(x));
  return x;
}

// Waits for every device-memory access of the wave (vmcnt 0; the other counters left alone).
// Ending a rarely taken branch with it keeps the compiler from waiting where the branch
// rejoins: it cannot tell which of the wave's loads are still in flight on the branch's path,
// and would otherwise make every wave, branch taken or not, wait there for all of them (the
// next stripe's text included).
WC_DEV void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Orders this wave's LDS accesses around the point in the compiler (the hardware keeps one
// wave's LDS operations in order).
WC_DEV void wave_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// 4 bytes of the logical text at p (p + base alignment keeps them in one aligned dword); bytes
// outside [0, len) read as spaces.
WC_DEV uint32_t load_text4(const uint8_t* corpus, uint64_t len, int64_t p) {
  if (p >= 0 && p + 4 <= (int64_t)len) return *(const uint32_t*)(corpus + p);
  uint32_t w = 0x20202020u;
  for (int j = 0; j < 4; ++j) {
    const int64_t q = p + j;
    if (q >= 0 && q < (int64_t)len)
      w = (w & ~(0xffu << (8 * j))) | ((uint32_t)corpus[q] << (8 * j));
  }
  return w;
}

// Positions of the word starts in this lane's 16 bytes (after the 16-byte prefix), in text
// order, for the ranks in [w0, w0 + kWaveStarts).
WC_DEV void write_starts16(uint32_t m, uint32_t rank, uint32_t w0, uint16_t* starts) {
  const uint32_t pos0 = 16 + (threadIdx.x & 63) * 16;
  while (m) {
    const uint32_t j = __ffs(m) - 1;
    if (rank - w0 < kWaveStarts) starts[rank - w0] = (uint16_t)(pos0 + j);
    ++rank;
    m &= m - 1;
  }
}

// Word-end bitmap of a wave's staged text: bit p set when byte p of the staged text (16-byte
// prefix, the stripe) is the last byte of a word; kEndWords words, the tail always zero.
constexpr uint32_t kEndWords = (kStripeText + 31) / 32 + 1;

// ---------------------------------------------------------------------------------------
// LDS table of 16-byte keys: kRedSlots slots of (19-bit tag << 13 | entry) probed in groups of
// 4 (one 16-byte read), and dense entries (key, count). A new key takes an entry, writes it,
// then claims the first empty slot of its group with a CAS; a reader that meets a claimed slot
// whose key is not visible yet looks again next iteration. Claimed slots of a group form a
// prefix and are never released, so a lane that loses a claim race finds the winner's key when
// it looks again: a key never holds two slots. The entry the loser had taken stays unused
// with count 0 (readers of the entries skip count 0). Keys are never all zero.
// ---------------------------------------------------------------------------------------
struct RedTable {
  uint32_t* slot;  // [kRedSlots], 0 = empty
  uint4* key;      // [cap]
  uint32_t* cnt;   // [cap]
  uint32_t* n;     // entries handed out
  uint32_t cap;
  Header* stall;   // when set: a give-up on a key that never became visible fails the call
};

// Hash of a key for the table (independent of the 32-bit word hash, whose low 8 bits choose the
// pass-2 partition): the dwords folded with rotations and one multiply; the group is the top 11
// bits, the tag 19 bits below them.
WC_DEV uint32_t red_hash(const uint4 v) {
  const uint32_t x = (v.x ^ __builtin_amdgcn_alignbit(v.y, v.y, 11)) +
                     (v.z ^ __builtin_amdgcn_alignbit(v.w, v.w, 23));
  return (x ^ (x >> 15)) * 0x9E3779B1u;
}
WC_DEV uint32_t red_tag(uint32_t h) { return ((h >> 2) & 0x7ffffu) | 1u; }
WC_DEV uint32_t red_group(uint32_t h) { return h >> 21; }

// The fast path of a lookup reads the first two groups of a key's probe sequence, its home
// group and the next: a key moves on to the next group only when its home group is full, so a
// key with an entry sits in one of them unless both were full when it was added. (With the
// home group alone, the keys of full groups, a few percent, missed the fast path on every
// occurrence, and a wave took the general insert whenever one of its lanes held such a key.)
WC_DEV uint32_t red_next_group(uint32_t g) { return (g + 1) & (kRedSlots / 4 - 1); }
// the first of the eight slots of groups a, b (in probe order) whose tag matches, or 0;
// selected from the last slot back, without branches
WC_DEV uint32_t red_pick8(const uint4 a, const uint4 b, uint32_t tag) {
  uint32_t m = 0u;
  m = (b.w >> 13) == tag ? b.w : m;
  m = (b.z >> 13) == tag ? b.z : m;
  m = (b.y >> 13) == tag ? b.y : m;
  m = (b.x >> 13) == tag ? b.x : m;
  m = (a.w >> 13) == tag ? a.w : m;
  m = (a.z >> 13) == tag ? a.z : m;
  m = (a.y >> 13) == tag ? a.y : m;
  m = (a.x >> 13) == tag ? a.x : m;
  return m;
}

// The common case: the word has an entry, found by the first tag match of its home group.
// Counts it and returns true; false sends the word to red_add.
WC_DEV bool red_hit(const RedTable& T, const uint4 want, uint32_t h) {
  const uint32_t tag = red_tag(h);
  const uint4 s4 = ((const uint4*)T.slot)[red_group(h)];
  const uint32_t e = (s4.x >> 13) == tag   ? s4.x
                     : (s4.y >> 13) == tag ? s4.y
                     : (s4.z >> 13) == tag ? s4.z
                     : (s4.w >> 13) == tag ? s4.w
                                           : 0u;
  if (e == 0) return false;
  const uint32_t idx = e & 0x1fffu;
  const uint4 k = T.key[idx];
  if (k.x != want.x || k.y != want.y || k.z != want.z || k.w != want.w) return false;
  atomicAdd(&T.cnt[idx], 1u);
  return true;
}

// Entry index of a key, or -1, in a table nobody is changing: the probe of red_add without
// its claims (a group with an empty slot ends it: claimed slots of a group form a prefix).
WC_DEV int red_find(const RedTable& T, const uint4 want, uint32_t h) {
  constexpr uint32_t kGroups = kRedSlots / 4;
  const uint32_t tag = red_tag(h);
  uint32_t g = red_group(h);
  for (int probe = 0; probe < 16; ++probe) {
    const uint4 s4 = ((const uint4*)T.slot)[g];
    const uint32_t e[4] = {s4.x, s4.y, s4.z, s4.w};
    bool empty = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if ((e[j] >> 13) == tag) {
        const uint32_t idx = e[j] & 0x1fffu;
        const uint4 k = T.key[idx];
        if (k.x == want.x && k.y == want.y && k.z == want.z && k.w == want.w) return (int)idx;
      } else if (e[j] == 0) {
        empty = true;
      }
    }
    if (empty) return -1;
    g = (g + 1) & (kGroups - 1);
  }
  return -1;
}

// Add one occurrence. Returns false when the word has no entry and none can be made (entries
// exhausted or 16 groups probed): the caller counts it elsewhere. New entries are handed out
// with one atomic per wave on the entry count.
WC_DEV bool red_add(const RedTable& T, uint64_t lo, uint64_t hi, uint32_t h) {
  constexpr uint32_t kGroups = kRedSlots / 4;
  constexpr uint32_t kNoEntry = 0xffffffffu;
  const uint32_t tag = red_tag(h);
  uint32_t g = red_group(h);
  static_assert(kGroups == 2048, "group index takes the hash's top 11 bits");
  const uint4 want = key4(lo, hi);
  const uint32_t lane = threadIdx.x & 63;
  uint32_t mine = kNoEntry, probe = 0, waits = 0;
  bool active = true, ok = false;
  while (__any(active)) {
    bool claim = false;
    int free_j = -1;
    if (active) {
      const uint4 s4 = ((const uint4*)T.slot)[g];
      const uint32_t e[4] = {s4.x, s4.y, s4.z, s4.w};
      bool found = false, wait = false;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (found) continue;
        if ((e[j] >> 13) == tag) {
          const uint32_t idx = e[j] & 0x1fffu;
          const uint4 k = T.key[idx];
          if (k.x == want.x && k.y == want.y && k.z == want.z && k.w == want.w) {
            atomicAdd(&T.cnt[idx], 1u);
            found = true;
          } else if ((k.x | k.y) == 0) {
            wait = true;  // claimed, key not visible yet
          }
        } else if (e[j] == 0 && free_j < 0) {
          free_j = j;
        }
      }
      if (found) {
        ok = true;
        active = false;
      } else if (wait) {
        // look at this group again. A key is written before its slot is claimed, so a claimed
        // slot shows a zero key only for a zero record, which no word makes: give up on it
        if (++waits >= 4096) {
          active = false;
          if (T.stall) or32(&T.stall->flags, kFlagStall);
        }
      } else if (free_j >= 0) {
        claim = true;
      } else {
        g = (g + 1) & (kGroups - 1);
        if (++probe >= 16) active = false;
      }
    }
    // entries for the lanes that claim a slot for the first time: one atomic per wave
    const bool need = claim && mine == kNoEntry;
    const uint64_t nm = __ballot(need);
    if (nm) {
      const uint32_t leader = (uint32_t)__ffsll((unsigned long long)nm) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(T.n, (uint32_t)__popcll(nm));
      base = (uint32_t)__builtin_amdgcn_readlane((int)base, (int)leader);
      if (need) {
        const uint32_t m =
            base + __builtin_amdgcn_mbcnt_hi((uint32_t)(nm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)nm, 0u));
        if (m < T.cap) {
          mine = m;
          T.key[m] = want;
        } else {
          claim = false;
          active = false;  // entries exhausted
        }
      }
    }
    if (claim) {
      const uint32_t prev = atomicCAS(&T.slot[g * 4 + free_j], 0u, (tag << 13) | mine);
      if (prev == 0) {
        atomicAdd(&T.cnt[mine], 1u);
        ok = true;
        active = false;
      }  // else the slot was taken: look at this group again
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  return ok;
}

}  // namespace wc
