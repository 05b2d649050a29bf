// Two-pass global count: the map of Section 3 (tokenise, key each word) with a workgroup-local
// dictionary of hot words, and the reduce (sum the counts of each word) over hash partitions.
//
// Why two passes. A word counted straight into the global table costs one device-scope
// atomic per token, and random atomics run at ~2.7e10/s chip-wide (measured), far below the
// byte rate of the scan. So:
//
//   dictionary: a sample of the text (kSampleStages stages of 8 KiB spread evenly over it) is
//     counted, and the most frequent words (up to kDictMax) become a read-only dictionary:
//     two-choice buckets of 4 tagged slots. A word is found in at most two 16-byte bucket
//     reads and one key read, with no insertion, eviction or probe loop.
//   pass 1 (global_map_kernel): scan the text; a dictionary word is counted in LDS; any other
//     token becomes a 16-byte record (its packed bytes) in one of 256 partitions chosen by a
//     hash of the word. Records wait in LDS (kStageSlots per partition) and leave in aligned
//     128-byte chunks into 4 KiB blocks of the partition's arena region, so the spill is
//     sequential full-line writes. The next block is requested half a block ahead, so its
//     atomic never stalls a flush.
//   pass 2 (global_reduce_kernel): one workgroup per partition reads that partition's
//     records, sums them in an LDS table and adds each distinct word once to the global
//     table; it also totals the dictionary hits of its share of dictionary words.
//
// Counts are exact whatever the dictionary holds: it only decides where a word is summed.
// Words longer than 16 bytes, and anything a bounded structure cannot take (a full overflow
// list, an exhausted arena region, a full pass-2 table), go to the global table directly.
#include "wc_internal.h"

namespace wc {

WC_DEV uint32_t word_hash32(uint64_t lo, uint64_t hi) {
  uint32_t a = (uint32_t)lo, b = (uint32_t)(lo >> 32), c = (uint32_t)hi, d = (uint32_t)(hi >> 32);
  uint32_t h = a * 0x9E3779B1u ^ (b * 0x85EBCA77u) ^ (c * 0xC2B2AE3Du) ^ (d * 0x27D4EB2Fu);
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 13;
  return h;
}

WC_DEV uint32_t part_of(uint32_t h) { return h & (kParts - 1); }

// dictionary placement: bucket 1 from the high bits of h; tag (low 20 bits) and bucket 2
// (high bits) from a second mix
WC_DEV uint32_t dict_h2(uint32_t h) {
  uint32_t x = h * 0x85EBCA77u;
  x ^= x >> 16;
  x *= 0xC2B2AE3Du;
  x ^= x >> 13;
  return x;
}
WC_DEV uint32_t dict_tag(uint32_t h2) { return (h2 & 0xFFFFFu) | 1u; }

WC_DEV uint4 key4(uint64_t lo, uint64_t hi) {
  return make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
}

template <bool kPerDoc>
WC_DEV uint64_t short_key_g(uint64_t lo, uint64_t hi, uint64_t key_mask) {
  return finish_key(fnv_packed(lo, hi, packed_len(lo, hi)), key_mask);
}

// Index of the word in the dictionary, or -1.
WC_DEV int dict_find(const uint4* tags4, const uint4* keys, uint32_t nb, uint64_t lo,
                     uint64_t hi, uint32_t h) {
  const uint32_t h2 = dict_h2(h);
  const uint32_t tag = dict_tag(h2);
  const uint4 want = key4(lo, hi);
  uint32_t b = __umulhi(h, nb);
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const uint4 t = tags4[b];
    const uint32_t e[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if ((e[j] >> 12) == tag) {
        const uint32_t idx = e[j] & 0xfffu;
        const uint4 k = keys[idx];
        if (k.x == want.x && k.y == want.y && k.z == want.z && k.w == want.w) return (int)idx;
      }
    }
    b = __umulhi(h2, nb);
  }
  return -1;
}

// ---------------------------------------------------------------------------------------
// LDS table of short words (lo, hi, count); no deletions while counting
// ---------------------------------------------------------------------------------------
struct LdsWords {
  uint64_t* lo;   // 0 = empty
  uint64_t* hi;   // packed bytes 8..15 | kTop; 0 until published
  uint32_t* cnt;
  uint32_t size;  // entries (any size; the home slot is the high half of h * size)
};

// Find the word and add n; insert it when absent and `may_insert`. Returns true when counted.
// A count never passes 2^31 - 1: an addition that would is undone and reported as not
// counted, so the caller counts it elsewhere and the kept sum stays exact.
// Wave-uniform loop: a lane that claims a slot publishes it inside the same iteration; a
// lane that meets a claimed, unpublished slot looks at it again next iteration.
WC_DEV bool lds_add(const LdsWords& T, uint64_t lo, uint64_t hi, uint32_t h, uint32_t n,
                    bool may_insert, uint32_t* live) {
  constexpr int kMaxProbe = 32;
  const uint64_t hiw = hi | kTop;
  uint32_t i = __umulhi(h, T.size);
  int probe = 0;
  bool active = true, ok = false;
  while (__any(active)) {
    uint64_t cur = 1;
    bool won = false;
    if (active) {
      cur = __hip_atomic_load(&T.lo[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (cur == 0 && may_insert) {
        cur = atomicCAS((unsigned long long*)&T.lo[i], 0ull, (unsigned long long)lo);
        won = cur == 0;
      }
    }
    if (won) {
      __hip_atomic_store(&T.hi[i], hiw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      atomicAdd(&T.cnt[i], n);
      atomicAdd(live, 1u);
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (active) {
      bool advance = true;
      if (won) {
        ok = true;
        active = false;
        advance = false;
      } else if (cur == 0) {
        active = false;  // absent and not inserting
        advance = false;
      } else if (cur == lo) {
        uint64_t sh = __hip_atomic_load(&T.hi[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (sh == 0) {
          advance = false;
        } else if (sh == hiw) {
          uint32_t old = atomicAdd(&T.cnt[i], n);
          if (old + (uint64_t)n > 0x7fffffffull) {
            atomicSub(&T.cnt[i], n);  // keep the entry below 2^31; caller counts n elsewhere
          } else {
            ok = true;
          }
          active = false;
          advance = false;
        }
      }
      if (advance) {
        i = (i + 1 == T.size) ? 0 : i + 1;
        if (++probe >= kMaxProbe) active = false;
      }
    }
  }
  return ok;
}

// Add n to a short word of the sample table (bounded probing: a sample may drop words).
WC_DEV void sample_insert(Slot* tab, uint64_t mask, uint64_t lo, uint64_t hi, uint32_t n) {
  const uint64_t key = finish_key(fnv_packed(lo, hi, packed_len(lo, hi)), ~0ull);
  const uint64_t w1 = hi | kTop;
  uint64_t i = key & mask;
  uint32_t probe = 0;
  bool active = true;
  while (__any(active)) {
    Slot* s = tab + i;
    uint64_t k = 1;
    bool won = false;
    if (active) {
      k = ld_relaxed(&s->key);
      if (k == 0) {
        k = cas64(&s->key, 0, key);
        won = k == 0;
      }
    }
    if (won) {
      st_relaxed(&s->w1, w1);
      st_relaxed(&s->w0, lo);
      add64(&s->cnt, n);
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (active) {
      bool advance = true;
      if (won) {
        active = false;
        advance = false;
      } else if (k == key) {
        uint64_t s0 = ld_relaxed(&s->w0), s1 = ld_relaxed(&s->w1);
        if (s0 == 0 || s1 == 0) {
          advance = false;
        } else if (s0 == lo && s1 == w1) {
          add64(&s->cnt, n);
          active = false;
          advance = false;
        }
      }
      if (advance) {
        i = (i + 1) & mask;
        if (++probe >= 64) active = false;
      }
    }
  }
}

// 16 bytes of the logical text at p; bytes outside [0, len) read as spaces.
WC_DEV uint4 load_text16(const uint8_t* corpus, uint64_t len, int64_t p) {
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

// Packed bytes of the word at byte s of the staged text (wl <= 16 bytes, all staged).
WC_DEV void pack_word(const uint8_t* s_txt, uint32_t s, uint32_t wl, uint64_t* lo, uint64_t* hi) {
  const uint32_t* tw = (const uint32_t*)s_txt;
  const uint32_t di = s >> 2, sh = s & 3;
  const uint32_t d0 = tw[di], d1 = tw[di + 1], d2 = tw[di + 2], d3 = tw[di + 3], d4 = tw[di + 4];
  uint64_t a = (uint64_t)__builtin_amdgcn_alignbyte(d1, d0, sh) |
               ((uint64_t)__builtin_amdgcn_alignbyte(d2, d1, sh) << 32);
  uint64_t b = (uint64_t)__builtin_amdgcn_alignbyte(d3, d2, sh) |
               ((uint64_t)__builtin_amdgcn_alignbyte(d4, d3, sh) << 32);
  if (wl < 8) {
    a &= (1ull << (8 * wl)) - 1;
    b = 0;
  } else if (wl == 8) {
    b = 0;
  } else if (wl < 16) {
    b &= (1ull << (8 * (wl - 8))) - 1;
  }
  *lo = a;
  *hi = b;
}

// Block-wide compaction of the word starts of a stage (one 16-bit mask per thread) into
// s_starts, in text order. Returns the number of starts. Contains two barriers.
template <int BLOCK>
WC_DEV uint32_t compact_starts(uint32_t start16, uint32_t* s_wsum, uint16_t* s_starts) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t cnt = __popc(start16);
  uint32_t incl = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) s_wsum[wave] = incl;
  __syncthreads();
  uint32_t base = 0, total = 0;
#pragma unroll
  for (int w = 0; w < BLOCK / 64; ++w) {
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
  __syncthreads();
  return total;
}

// ---------------------------------------------------------------------------------------
// dictionary: sample, threshold, placement
// ---------------------------------------------------------------------------------------
// One stage per workgroup, spread evenly over the text. Document boundaries are ignored and
// words cut at the stage edges count as they appear: the sample only ranks words.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void sample_kernel(GlobalParams P) {
  constexpr int STAGE = BLOCK * 16;
  __shared__ uint4 s_txt4[BLOCK + 2];
  __shared__ uint16_t s_wm[BLOCK];
  __shared__ uint16_t s_last[BLOCK + 1];
  __shared__ uint16_t s_starts[STAGE / 2];
  __shared__ uint32_t s_wsum[BLOCK / 64];
  __shared__ uint64_t s_lo[kSampleLds], s_hi[kSampleLds];
  __shared__ uint32_t s_cnt[kSampleLds];
  __shared__ uint32_t s_live;
  const int tid = threadIdx.x;
  if (ld_relaxed32(&P.hdr->flags) & kFlagBadOffsets) return;
  const int64_t R0 = (int64_t)P.offsets[0], R1 = (int64_t)P.offsets[P.n_docs];
  const uint64_t k = (uint64_t)blockIdx.x * P.n_stages / gridDim.x;
  const int64_t ls = P.base_off + (int64_t)(k * STAGE);
  uint32_t w16;
  uint4 g = classify16(load_text16(P.corpus, P.len, ls + tid * 16), &w16);
  w16 = cut16(w16, ls + tid * 16, R0, R1);
  s_txt4[tid] = g;
  s_wm[tid] = (uint16_t)w16;
  if (tid < 2) s_txt4[BLOCK + tid] = make_uint4(0, 0, 0, 0);
  if (tid == 0) {
    s_live = 0;
    s_last[BLOCK] = 0;
  }
  LdsWords T{s_lo, s_hi, s_cnt, kSampleLds};
  for (uint32_t i = tid; i < kSampleLds; i += BLOCK) {
    s_lo[i] = 0;
    s_hi[i] = 0;
    s_cnt[i] = 0;
  }
  __syncthreads();
  const uint32_t prev = tid > 0 ? (s_wm[tid - 1] >> 15) : 0u;
  const uint32_t next = tid < BLOCK - 1 ? (s_wm[tid + 1] & 1u) : 0u;
  const uint32_t start16 = w16 & ~((w16 << 1) | prev) & 0xffffu;
  const uint32_t last16 = w16 & ~((w16 >> 1) | (next << 15)) & 0xffffu;
  s_last[tid] = (uint16_t)last16;
  const uint32_t total = compact_starts<BLOCK>(start16, s_wsum, s_starts);
  const uint32_t cap = kSampleLds - kSampleLds / 4;
  for (uint32_t t = tid; t < total; t += BLOCK) {
    const uint32_t s = s_starts[t];
    uint32_t q = s >> 4;
    uint32_t bits = (uint32_t)s_last[q] >> (s & 15);
    uint32_t e;
    if (bits) {
      e = s + __ffs(bits) - 1;
    } else {
      ++q;
      while (q < BLOCK && s_last[q] == 0) ++q;  // the stage's last word byte ends a word
      if (q >= BLOCK) continue;
      e = q * 16 + __ffs(s_last[q]) - 1;
    }
    const uint32_t wl = e - s + 1;
    if (wl > 16) continue;
    uint64_t lo, hi;
    pack_word((const uint8_t*)s_txt4, s, wl, &lo, &hi);
    lds_add(T, lo, hi, word_hash32(lo, hi), 1, s_live < cap, &s_live);
  }
  __syncthreads();
  for (uint32_t i = tid; i < kSampleLds; i += BLOCK) {
    const uint32_t c = s_cnt[i];
    if (c) sample_insert(P.sample_table, kSampleSlots - 1, s_lo[i], s_hi[i] & ~kTop, c);
  }
}

// Count threshold of the selection: words with a sample count (clamped at 255) >= t fit the
// dictionary (acc of them); `room` more may come from count t - 1.
WC_DEV void dict_threshold(const uint32_t* hist, uint32_t cap, uint32_t* t, uint32_t* acc,
                           uint32_t* room) {
  uint32_t a = 0, th = 256;
  for (int c = 255; c >= 1; --c) {
    if (a + hist[c] > cap) break;
    a += hist[c];
    th = (uint32_t)c;
  }
  *t = th;
  *acc = a;
  *room = cap - a;
}

__global__ void dict_hist_kernel(GlobalParams P) {
  __shared__ uint32_t h[256];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < kSampleSlots;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const Slot& s = P.sample_table[i];
    if (s.key) atomicAdd(&h[s.cnt < 255 ? (uint32_t)s.cnt : 255u], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += blockDim.x)
    if (h[i]) atomicAdd(&P.dict->hist[i], h[i]);
}

__global__ void dict_select_kernel(GlobalParams P) {
  __shared__ uint32_t s_t, s_acc, s_room;
  if (threadIdx.x == 0) {
    uint32_t t, acc, room;
    dict_threshold(P.dict->hist, P.dict_cap, &t, &acc, &room);
    s_t = t;
    s_acc = acc;
    s_room = room;
  }
  __syncthreads();
  const uint32_t t = s_t, acc = s_acc, room = s_room;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < kSampleSlots;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const Slot s = P.sample_table[i];
    if (!s.key) continue;
    const uint32_t c = s.cnt < 255 ? (uint32_t)s.cnt : 255u;
    const uint4 k = key4(s.w0, s.w1 & ~kTop);
    if (c >= t) {
      uint32_t j = atomicAdd(&P.dict->n_high, 1u);
      if (j < acc) {
        P.dict->keys[j] = k;
        P.dict->cnt[j] = c;
      }
    } else if (c + 1 == t && room) {
      uint32_t j = atomicAdd(&P.dict->n_low, 1u);
      if (j < room) {
        P.dict->keys[acc + j] = k;
        P.dict->cnt[acc + j] = c;
      }
    }
  }
}

// One workgroup: place the selected words into buckets, hottest first (a counting sort on
// the sample counts), each into the emptier of its two buckets. A word that finds both
// buckets full is left out, so only the coldest words can be left out.
__global__ __launch_bounds__(1024) void dict_build_kernel(GlobalParams P) {
  __shared__ uint32_t s_fill[kDictBuckets];
  __shared__ uint32_t s_pos[256];
  __shared__ uint16_t s_order[kDictMax];
  __shared__ uint32_t s_n;
  const uint32_t tid = threadIdx.x;
  if (tid == 0) {
    uint32_t t, acc, room;
    dict_threshold(P.dict->hist, P.dict_cap, &t, &acc, &room);
    uint32_t low = P.dict->n_low;
    s_n = acc + (low < room ? low : room);
  }
  for (uint32_t i = tid; i < kDictBuckets; i += blockDim.x) s_fill[i] = 0;
  for (uint32_t i = tid; i < 256; i += blockDim.x) s_pos[i] = 0;
  __syncthreads();
  const uint32_t n = s_n;
  for (uint32_t i = tid; i < n; i += blockDim.x) atomicAdd(&s_pos[P.dict->cnt[i]], 1u);
  __syncthreads();
  if (tid == 0) {  // start of each count class, hottest class first
    uint32_t a = 0;
    for (int c = 255; c >= 0; --c) {
      uint32_t v = s_pos[c];
      s_pos[c] = a;
      a += v;
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < n; i += blockDim.x)
    s_order[atomicAdd(&s_pos[P.dict->cnt[i]], 1u)] = (uint16_t)i;
  __syncthreads();
  uint32_t nb = (P.dict_cap + 2) / 3;
  nb = nb < 16 ? 16 : (nb > kDictBuckets ? kDictBuckets : nb);
  for (uint32_t r0 = 0; r0 < n; r0 += blockDim.x) {
    const uint32_t r = r0 + tid;
    if (r < n) {
      const uint32_t i = s_order[r];
      const uint4 k = P.dict->keys[i];
      const uint64_t lo = (uint64_t)k.x | ((uint64_t)k.y << 32), hi = (uint64_t)k.z | ((uint64_t)k.w << 32);
      const uint32_t h = word_hash32(lo, hi), h2 = dict_h2(h);
      uint32_t b = __umulhi(h, nb), b2 = __umulhi(h2, nb);
      if (s_fill[b2] < s_fill[b]) {
        const uint32_t x = b;
        b = b2;
        b2 = x;
      }
      uint32_t slot = atomicAdd(&s_fill[b], 1u);
      if (slot >= 4) {
        b = b2;
        slot = atomicAdd(&s_fill[b], 1u);
      }
      if (slot < 4) P.dict->tags[b * 4 + slot] = (dict_tag(h2) << 12) | i;
    }
    __syncthreads();  // the next (colder) round sees these placements
  }
  if (tid == 0) {
    P.dict->n = n;
    P.dict->nb = nb;
    P.hdr->stat[2] = n;
  }
}

// ---------------------------------------------------------------------------------------
// pass 1
// ---------------------------------------------------------------------------------------
size_t global_map_dyn(uint32_t dict_cap) {
  constexpr int BLOCK = 512;
  return (size_t)kParts * kStageSlots * 16 + (size_t)(BLOCK + 2) * 16 + (size_t)kDictBuckets * 16 +
         (size_t)dict_cap * 20 + (size_t)BLOCK * 16;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void global_map_kernel(GlobalParams P) {
  constexpr int STAGE = BLOCK * 16;
  constexpr uint32_t kNone = 0xffffffffu;
  static_assert(BLOCK >= (int)kParts && BLOCK >= (int)kOverflow && BLOCK >= (int)kSdWin + 3,
                "one thread per partition, overflow entry and cached stage entry");
  extern __shared__ __align__(16) uint8_t s_dyn[];
  __shared__ uint16_t s_wm[BLOCK];
  __shared__ uint16_t s_last[BLOCK + 1];
  __shared__ uint32_t s_bnd[STAGE / 32 + 2];
  __shared__ uint32_t s_fill[kParts];
  __shared__ uint4 s_ovf[kOverflow];
  __shared__ uint16_t s_ovp[kOverflow];
  __shared__ uint64_t s_sd[kSdWin + 3];
  __shared__ uint32_t s_wsum[BLOCK / 64];
  __shared__ uint32_t s_novf, s_next_w, s_next_run;
  __shared__ uint32_t s_carry[2];
  __shared__ uint32_t s_stat[4];

  const uint32_t D = P.dict_cap;
  uint4* s_stage = (uint4*)s_dyn;                         // [kParts][kStageSlots]
  uint4* s_txt4 = s_stage + kParts * kStageSlots;         // [BLOCK + 2]
  uint4* s_tags4 = s_txt4 + (BLOCK + 2);                  // [kDictBuckets]
  uint4* s_keys = s_tags4 + kDictBuckets;                 // [D]
  uint32_t* s_cnt = (uint32_t*)(s_keys + D);              // [D]
  uint16_t* s_starts = (uint16_t*)(s_cnt + D);            // [STAGE / 2]
  const uint8_t* s_txt = (const uint8_t*)s_txt4;

  const int tid = threadIdx.x;
  Header* hdr = P.hdr;
  if (ld_relaxed32(&hdr->flags) & kFlagBadOffsets) return;
  const uint64_t st0 = (uint64_t)blockIdx.x * P.stages_per_wg;
  const uint64_t st1 = min(st0 + P.stages_per_wg, P.n_stages);
  const uint64_t n_stages = P.n_stages;
  const int64_t len = (int64_t)P.len;
  const int64_t R0 = (int64_t)P.offsets[0], R1 = (int64_t)P.offsets[P.n_docs];

  // dictionary into LDS
  const uint32_t nd = P.dict->n, nb = P.dict->nb;
  for (uint32_t i = tid; i < nb; i += BLOCK) s_tags4[i] = ((const uint4*)P.dict->tags)[i];
  for (uint32_t i = tid; i < nd; i += BLOCK) {
    s_keys[i] = P.dict->keys[i];
    s_cnt[i] = 0;
  }
  for (uint32_t p = tid; p < kParts; p += BLOCK) s_fill[p] = 0;
  if (tid == 0) s_novf = 0;
  if (tid < 4) s_stat[tid] = 0;
  for (int i = tid; i < STAGE / 32 + 2; i += BLOCK) s_bnd[i] = 0;

  // Thread p < kParts writes partition p: current block, records in it, next block.
  uint32_t blk = kNone, bpos = 0, nxt = kNone;
  bool nxt_req = false;
  if (tid < (int)kParts) blk = atomicAdd(&P.cursor[tid], 1u);

  // n (<= kChunkRec) staged records of partition p to the arena (thread p)
  auto put = [&](uint32_t p, uint32_t n) {
    const uint4* src = s_stage + p * kStageSlots;
    if (blk >= P.R) {
      // the partition's region is exhausted: count these in the global table
      atomicAdd(&s_stat[1], n);
      for (uint32_t j = 0; j < n; ++j) {
        const uint4 r = src[j];
        const uint64_t lo = (uint64_t)r.x | ((uint64_t)r.y << 32);
        const uint64_t hi = (uint64_t)r.z | ((uint64_t)r.w << 32);
        table_insert<false>(P.table, P.mask, short_key_g<false>(lo, hi, P.key_mask),
                            short_id(lo, hi, 0), 1, hdr, P.occ_limit);
      }
      return;
    }
    uint4* dst = P.arena + ((uint64_t)p * P.R + blk) * kBlockRec + bpos;
    for (uint32_t j = 0; j < n; ++j) dst[j] = src[j];
    bpos += n;
    if (bpos == kBlockRec) {
      P.fill[(uint64_t)p * P.R + blk] = (uint16_t)kBlockRec;
      blk = nxt_req ? nxt : atomicAdd(&P.cursor[p], 1u);
      nxt_req = false;
      bpos = 0;
    } else if (!nxt_req && bpos >= kBlockRec / 2) {
      nxt = atomicAdd(&P.cursor[p], 1u);  // used half a block from now
      nxt_req = true;
    }
  };
  // a full chunk of partition p leaves; the rest of its staging moves to the front (thread p)
  auto flush_part = [&](uint32_t p) {
    const uint32_t f = s_fill[p];
    uint32_t n = f < kStageSlots ? f : kStageSlots;  // reservations past the end overflowed
    if (n >= kChunkRec) {
      put(p, kChunkRec);
      uint4* st = s_stage + p * kStageSlots;
      for (uint32_t j = kChunkRec; j < n; ++j) st[j - kChunkRec] = st[j];
      n -= kChunkRec;
    }
    s_fill[p] = n;
  };
  auto stage_pos = [&](uint64_t k) -> int64_t { return P.base_off + (int64_t)(k * STAGE); };
  const uint4 blank = make_uint4(0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u);
  auto load16 = [&](uint64_t k) -> uint4 {
    return load_text16(P.corpus, P.len, stage_pos(k) + tid * 16);
  };

  // stage -> first document starting at or after it, cached kSdWin stages at a time
  uint64_t sd_base = st0;
  for (uint32_t i = tid; i < kSdWin + 3; i += BLOCK)
    s_sd[i] = P.stage_doc[min(st0 + i, n_stages)];
  if (tid == 0) {
    int64_t q = stage_pos(st0) - 1;
    s_carry[(st0 & 1) ^ 1] =
        (q >= R0 && q < R1 && q >= 0 && q < len && is_word_byte(P.corpus[q])) ? 1u : 0u;
  }
  __syncthreads();
  // document starts of stages st0 and st0 + 1 (thread i holds the i-th of its stage)
  auto doc_start = [&](uint64_t k) -> uint64_t {
    if (k >= n_stages) return ~0ull;
    const uint64_t c0 = s_sd[k - sd_base], c1 = s_sd[k + 1 - sd_base];
    return (uint64_t)tid < c1 - c0 ? P.offsets[c0 + tid] : ~0ull;
  };
  uint64_t bo1 = doc_start(st0), bo2 = doc_start(st0 + 1), bo0;

  // text: this stage and three ahead (one past the range: the next stage's first bytes close
  // a word that crosses the range end)
  uint4 cur = load16(st0), n1 = blank, n2 = blank, n3 = blank;
  if (st0 + 1 <= st1 && st0 + 1 < n_stages) n1 = load16(st0 + 1);
  if (st0 + 2 <= st1 && st0 + 2 < n_stages) n2 = load16(st0 + 2);
  if (st0 + 3 <= st1 && st0 + 3 < n_stages) n3 = load16(st0 + 3);
  uint64_t tokens = 0;
  uint32_t spilled = 0;  // records this thread sent to the partitions

  for (uint64_t k = st0; k < st1; ++k) {
    const int64_t ls = stage_pos(k);
    const int64_t le = ls + STAGE;
    if (k != st0 && (k - st0) % kSdWin == 0) {
      __syncthreads();  // every read of the previous window is done
      sd_base = k;
      for (uint32_t i = tid; i < kSdWin + 3; i += BLOCK)
        s_sd[i] = P.stage_doc[min(k + i, n_stages)];
      __syncthreads();
    }
    const uint64_t c0 = s_sd[k - sd_base], c1 = s_sd[k + 1 - sd_base];
    const uint64_t nb1 = k + 1 < n_stages ? s_sd[k + 2 - sd_base] - c1 : 0;
    bo0 = bo1;
    bo1 = bo2;
    bo2 = doc_start(k + 2);
    uint4 n4 = blank;
    if (k + 4 <= st1 && k + 4 < n_stages) n4 = load16(k + 4);

    // ---- 1. fold + classify; document starts in [ls, le] ---------------------------------
    uint32_t w16;
    const uint4 g = classify16(cur, &w16);
    const int64_t p = ls + tid * 16;
    w16 = cut16(w16, p, R0, R1);
    s_txt4[tid] = g;
    s_wm[tid] = (uint16_t)w16;
    const uint64_t nbk = c1 - c0;
    if ((uint64_t)tid < nbk) {
      const uint64_t rel = bo0 - (uint64_t)ls;
      atomicOr(&s_bnd[rel >> 5], 1u << (rel & 31));
    }
    for (uint64_t j = BLOCK + tid; j < nbk; j += BLOCK) {
      const uint64_t rel = P.offsets[c0 + j] - (uint64_t)ls;
      atomicOr(&s_bnd[rel >> 5], 1u << (rel & 31));
    }
    if (tid == 0) {
      // the next stage's first 16 bytes: a word running over the stage end finishes there
      uint32_t nw;
      s_txt4[BLOCK] = classify16(n1, &nw);
      int64_t cut_hi = R1;
      const bool doc_at_le = nb1 > 0 && (int64_t)bo1 == le;
      if (nb1 > 0 && (int64_t)bo1 < cut_hi) cut_hi = (int64_t)bo1;
      nw = cut16(nw, le, R0, cut_hi);
      if (doc_at_le) {
        atomicOr(&s_bnd[STAGE >> 5], 1u);
        nw = 0;
      }
      s_next_w = nw & 1u;
      s_next_run = (uint32_t)__builtin_ctz(~nw | 0x10000u);  // 16: runs past these bytes
    }
    __syncthreads();

    // ---- 2. start / last masks, compaction --------------------------------------------
    const uint32_t prev = tid > 0 ? (s_wm[tid - 1] >> 15) : s_carry[(k & 1) ^ 1];
    const uint32_t next = tid < BLOCK - 1 ? (s_wm[tid + 1] & 1u) : s_next_w;
    const uint32_t bnd = (s_bnd[tid >> 1] >> ((tid & 1) * 16)) & 0xffffu;
    const uint32_t bnext = (s_bnd[(tid + 1) >> 1] >> (((tid + 1) & 1) * 16)) & 1u;
    const uint32_t wprev = ((w16 << 1) | prev) & 0xffffu;
    const uint32_t start16 = w16 & (~wprev | bnd);
    const uint32_t wnext = (w16 >> 1) | (next << 15);
    const uint32_t bn16 = (bnd >> 1) | (bnext << 15);
    const uint32_t last16 = w16 & (~wnext | bn16) & 0xffffu;
    s_last[tid] = (uint16_t)last16;
    if (tid == BLOCK - 1) {
      s_carry[k & 1] = w16 >> 15;
      s_last[BLOCK] = 0;
    }
    const uint32_t total = compact_starts<BLOCK>(start16, s_wsum, s_starts);
    tokens += (tid == 0) ? total : 0u;
    for (int i = tid; i < STAGE / 32 + 2; i += BLOCK) s_bnd[i] = 0;
    const uint32_t next_run = s_next_run;

    // ---- 3. tokens ----------------------------------------------------------------------
    for (uint32_t t = tid; t < total; t += BLOCK) {
      const uint32_t s = s_starts[t];
      uint32_t q = s >> 4;
      const uint32_t bits = (uint32_t)s_last[q] >> (s & 15);
      uint32_t e;
      bool crosses = false;
      if (bits) {
        e = s + __ffs(bits) - 1;
      } else {
        ++q;
        while (q < BLOCK && s_last[q] == 0) ++q;
        if (q < BLOCK) {
          e = q * 16 + __ffs(s_last[q]) - 1;
        } else {
          crosses = true;
          e = STAGE + next_run - 1;
        }
      }
      const uint32_t wl = e - s + 1;
      uint64_t lo, hi;
      if (wl <= 16 && !(crosses && next_run >= 16)) {
        pack_word(s_txt, s, wl, &lo, &hi);
      } else {
        // longer than 16 bytes (or running past the bytes staged): from device memory
        const uint64_t start = (uint64_t)(ls + s);
        uint64_t limit = start + wl;
        if (crosses) {
          limit = (uint64_t)R1;
          if (c1 <= P.n_docs && P.offsets[c1] < limit) limit = P.offsets[c1];
        }
        uint64_t h64;
        const uint64_t n = scan_word(P.corpus, start, limit, &lo, &hi, &h64);
        if (n > 16) {
          table_insert<false>(P.table, P.mask, finish_key(h64, P.key_mask),
                              long_id(P.corpus + start, n, 0), 1, hdr, P.occ_limit);
          continue;
        }
      }
      const uint32_t h = word_hash32(lo, hi);
      const int idx = nd ? dict_find(s_tags4, s_keys, nb, lo, hi, h) : -1;
      if (idx >= 0) {
        atomicAdd(&s_cnt[idx], 1u);
        continue;
      }
      spilled += 1;
      const uint32_t pp = part_of(h);
      const uint32_t slot = atomicAdd(&s_fill[pp], 1u);
      if (slot < kStageSlots) {
        s_stage[pp * kStageSlots + slot] = key4(lo, hi);
      } else {
        const uint32_t o = atomicAdd(&s_novf, 1u);
        if (o < kOverflow) {
          s_ovf[o] = key4(lo, hi);
          s_ovp[o] = (uint16_t)pp;
        } else {
          atomicAdd(&s_stat[1], 1u);
          table_insert<false>(P.table, P.mask, short_key_g<false>(lo, hi, P.key_mask),
                              short_id(lo, hi, 0), 1, hdr, P.occ_limit);
        }
      }
    }
    __syncthreads();

    // ---- 4. full chunks leave; overflowed records are staged again ----------------------
    const uint32_t novf = s_novf < kOverflow ? s_novf : kOverflow;
    if (tid < (int)kParts) flush_part(tid);
    if (novf) {
      if (tid == 0) s_stat[2] += novf;
      bool pend = (uint32_t)tid < novf;
      uint4 rec = pend ? s_ovf[tid] : make_uint4(0, 0, 0, 0);
      uint32_t pp = pend ? s_ovp[tid] : 0u;
      __syncthreads();
      if (tid == 0) s_novf = 0;
      while (__syncthreads_or(pend)) {
        if (pend) {
          const uint32_t slot = atomicAdd(&s_fill[pp], 1u);
          if (slot < kStageSlots) {
            s_stage[pp * kStageSlots + slot] = rec;
            pend = false;
          }
        }
        __syncthreads();
        if (tid < (int)kParts) flush_part(tid);
      }
    }
    cur = n1;
    n1 = n2;
    n2 = n3;
    n3 = n4;
  }

  // ---- end of range: staged records leave, blocks close; dictionary hits go out ---------
  __syncthreads();
  if (tid < (int)kParts) {
    const uint32_t n = s_fill[tid];
    if (n) put(tid, n);
    if (blk < P.R) P.fill[(uint64_t)tid * P.R + blk] = (uint16_t)bpos;
    if (nxt_req && nxt < P.R) P.fill[(uint64_t)tid * P.R + nxt] = 0;
  }
  for (uint32_t i = tid; i < nd; i += BLOCK) P.dict_part[(uint64_t)blockIdx.x * D + i] = s_cnt[i];
  if (spilled) atomicAdd(&s_stat[0], spilled);
  __syncthreads();
  if (tid == 0) {
    if (s_stat[0]) add64(&hdr->stat[0], s_stat[0]);
    add64(&hdr->total_tokens, tokens);
    if (s_stat[1]) add64(&hdr->stat[1], s_stat[1]);
    if (s_stat[2]) add64(&hdr->stat[3], s_stat[2]);
  }
}

// ---------------------------------------------------------------------------------------
// pass 2: one workgroup per partition
// ---------------------------------------------------------------------------------------
size_t global_reduce_dyn(uint32_t entries) { return (size_t)entries * 20; }

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void global_reduce_kernel(GlobalParams P) {
  extern __shared__ __align__(16) uint8_t s_dyn[];
  __shared__ uint32_t s_live, s_miss;
  __shared__ unsigned long long s_dsum[kDictCols];
  const uint32_t p = blockIdx.x;
  const int tid = threadIdx.x;
  Header* hdr = P.hdr;
  if (ld_relaxed32(&hdr->flags) & kFlagBadOffsets) return;
  const uint32_t E = P.reduce_entries;
  LdsWords T;
  T.lo = (uint64_t*)s_dyn;
  T.hi = T.lo + E;
  T.cnt = (uint32_t*)(T.hi + E);
  T.size = E;
  for (uint32_t i = tid; i < E; i += BLOCK) {
    T.lo[i] = 0;
    T.hi[i] = 0;
    T.cnt[i] = 0;
  }
  for (uint32_t i = tid; i < kDictCols; i += BLOCK) s_dsum[i] = 0;
  if (tid == 0) {
    s_live = 0;
    s_miss = 0;
  }
  __syncthreads();

  // dictionary words [dc0, dc0 + ncol): hits summed over the pass-1 workgroups
  const uint32_t nd = P.dict->n;
  const uint32_t per = (nd + gridDim.x - 1) / gridDim.x;
  const uint32_t dc0 = p * per;
  const uint32_t ncol = dc0 < nd ? min(per, nd - dc0) : 0u;
  const uint32_t G1 = P.map_grid;
  for (uint32_t q = tid; q < ncol * G1; q += BLOCK) {
    const uint32_t c = q / G1, r = q - c * G1;
    const uint32_t v = P.dict_part[(uint64_t)r * P.dict_cap + dc0 + c];
    if (v) atomicAdd(&s_dsum[c], (unsigned long long)v);
  }

  // records of partition p
  const uint32_t nblk = min(P.cursor[p], P.R);
  const uint4* region = P.arena + (uint64_t)p * P.R * kBlockRec;
  const uint16_t* fills = P.fill + (uint64_t)p * P.R;
  constexpr uint32_t kPerIter = BLOCK / kBlockRec;  // blocks per iteration
  static_assert(BLOCK % kBlockRec == 0, "whole blocks per iteration");
  const uint32_t cap = P.reduce_cap;
  const uint32_t r_in = tid % kBlockRec, b_in = tid / kBlockRec;
  auto fetch = [&](uint32_t b0, uint32_t* n) -> uint4 {
    const uint32_t b = b0 + b_in;
    if (b >= nblk) {
      *n = 0;
      return make_uint4(0, 0, 0, 0);
    }
    *n = fills[b];  // issued with the record load; compared once both arrive
    return region[(uint64_t)b * kBlockRec + r_in];
  };
  uint32_t f0, f1, f2;
  uint4 v0 = fetch(0, &f0);
  uint4 v1 = fetch(kPerIter, &f1);
  uint4 v2 = fetch(2 * kPerIter, &f2);
  for (uint32_t b0 = 0; b0 < nblk; b0 += kPerIter) {
    uint32_t f3;
    const uint4 v3 = fetch(b0 + 3 * kPerIter, &f3);
    if (r_in < f0) {
      const uint64_t lo = (uint64_t)v0.x | ((uint64_t)v0.y << 32);
      const uint64_t hi = (uint64_t)v0.z | ((uint64_t)v0.w << 32);
      const bool ok = lds_add(T, lo, hi, word_hash32(lo, hi) * 0x9E3779B1u, 1,
                              s_live < cap, &s_live);
      if (!ok) {
        atomicAdd(&s_miss, 1u);
        table_insert<false>(P.table, P.mask, short_key_g<false>(lo, hi, P.key_mask),
                            short_id(lo, hi, 0), 1, hdr, P.occ_limit);
      }
    }
    v0 = v1;
    f0 = f1;
    v1 = v2;
    f1 = f2;
    v2 = v3;
    f2 = f3;
  }
  __syncthreads();
  for (uint32_t i = tid; i < E; i += BLOCK) {
    const uint32_t c = T.cnt[i];
    if (c) {
      const uint64_t lo = T.lo[i], hi = T.hi[i] & ~kTop;
      table_insert<false>(P.table, P.mask, short_key_g<false>(lo, hi, P.key_mask),
                          short_id(lo, hi, 0), c, hdr, P.occ_limit);
    }
  }
  for (uint32_t c = tid; c < ncol; c += BLOCK) {
    const uint64_t n = s_dsum[c];
    if (n) {
      const uint4 k = P.dict->keys[dc0 + c];
      const uint64_t lo = (uint64_t)k.x | ((uint64_t)k.y << 32);
      const uint64_t hi = (uint64_t)k.z | ((uint64_t)k.w << 32);
      table_insert<false>(P.table, P.mask, short_key_g<false>(lo, hi, P.key_mask),
                          short_id(lo, hi, 0), n, hdr, P.occ_limit);
    }
  }
  if (tid == 0 && s_miss) add64(&hdr->stat[4], s_miss);
}

hipError_t set_global_smem(uint32_t dict_cap, uint32_t reduce_entries) {
  hipError_t e = hipFuncSetAttribute((const void*)global_map_kernel<512>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)global_map_dyn(dict_cap));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)global_reduce_kernel<1024>,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)global_reduce_dyn(reduce_entries));
  return e;
}

hipError_t launch_global(const GlobalParams& P, hipEvent_t a, hipEvent_t b, hipStream_t s) {
  const uint32_t ns = (uint32_t)(P.n_stages < kSampleStages ? P.n_stages : kSampleStages);
  if (ns) hipLaunchKernelGGL(sample_kernel<512>, dim3(ns), dim3(512), 0, s, P);
  hipLaunchKernelGGL(dict_hist_kernel, dim3(256), dim3(256), 0, s, P);
  hipLaunchKernelGGL(dict_select_kernel, dim3(256), dim3(256), 0, s, P);
  hipLaunchKernelGGL(dict_build_kernel, dim3(1), dim3(1024), 0, s, P);
  if (a) {
    hipError_t e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(global_map_kernel<512>, dim3(P.map_grid), dim3(512),
                     global_map_dyn(P.dict_cap), s, P);
  if (b) {
    hipError_t e = hipEventRecord(b, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(global_reduce_kernel<1024>, dim3(kParts), dim3(1024),
                     global_reduce_dyn(P.reduce_entries), s, P);
  return hipGetLastError();
}

}  // namespace wc
