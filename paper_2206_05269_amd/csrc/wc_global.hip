// Two-pass global count: the map of Section 3 (tokenise, key each word) with a workgroup-local
// dictionary of hot words, and the reduce (sum the counts of each word) over hash partitions.
//
// Why two passes. A word counted straight into the global table costs one device-scope
// atomic per token, and random atomics run at ~2.7e10/s chip-wide (measured), far below the
// byte rate of the scan. So:
//
//   dictionary: a sample of the text (kSampleStages stages of 8 KiB spread evenly over it) is
//     counted, and the most frequent words (up to kDictMax) become a read-only perfect hash
//     (hash and displace): a word is found with one displacement read, one slot read and one
//     key compare, with no insertion, eviction or probe loop.
//   pass 1 (global_map_kernel): scan the text, each wave on its own 1 KiB stripes; a dictionary
//     word is counted in LDS; any other token becomes a 16-byte record (its packed bytes) in one
//     of 256 partitions chosen by a hash of the word, stored straight into the workgroup's
//     current 4 KiB block of that partition (an LDS ticket per partition gives its slot).
//   pass 2 (global_reduce_kernel): one workgroup per partition reads that partition's
//     records, sums them in an LDS table and adds each distinct word once to the global
//     table; it also totals the dictionary hits of its share of dictionary words.
//
// Counts are exact whatever the dictionary holds: it only decides where a word is summed.
// Words longer than 16 bytes, and anything a bounded structure cannot take (an exhausted arena
// region, a full pass-2 table), go to the global table directly.
#include "wc_internal.h"
#include "wc_stripe.h"

namespace wc {

// 32-bit hash of a packed word (16 bytes as four dwords): the dwords folded with rotations,
// then the 32-bit finaliser of MurmurHash3 (Appleby) for avalanche; two multiplies.
WC_DEV uint32_t word_hash32(uint64_t lo, uint64_t hi) {
  const uint32_t a = (uint32_t)lo, b = (uint32_t)(lo >> 32), c = (uint32_t)hi, d = (uint32_t)(hi >> 32);
  uint32_t h = (a ^ __builtin_amdgcn_alignbit(b, b, 21)) + (c ^ __builtin_amdgcn_alignbit(d, d, 13));
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

WC_DEV uint32_t part_of(uint32_t h) { return h & (kParts - 1); }

// The 32-bit word hash h serves the partition (bits 0-7) and the dictionary: group g = bits 0-8;
// the group's slots lie in region g mod 16 (256 slots); a word's slot in the region is an 8-bit
// field of h (bits 9-16, or bits 17-24 when bit 8 of the group's displacement is set) XOR the
// displacement's low 8 bits.
WC_DEV uint32_t dict_group(uint32_t h) { return h & (kDispBuckets - 1); }
WC_DEV uint32_t dict_field(uint32_t h, uint32_t sel) {
  return (h >> (__builtin_ctz(kDispBuckets) + 8 * sel)) & 0xffu;
}
WC_DEV uint32_t dict_slot(uint32_t h, uint32_t d) {
  const uint32_t g = dict_group(h);
  return ((g & (kDictRegions - 1)) << 8) | ((dict_field(h, (d >> 8) & 1u) ^ d) & 0xffu);
}

template <bool kPerDoc>
WC_DEV uint64_t short_key_g(uint64_t lo, uint64_t hi, uint64_t key_mask) {
  return finish_key(fnv_packed(lo, hi, packed_len(lo, hi)), key_mask);
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

// Positions (tid * 16 + bit) of the starts in mask m whose ranks, counted from `rank`, fall
// in [w0, w0 + cap), stored at s_starts[rank - w0].
WC_DEV void write_starts(uint32_t m, uint32_t rank, uint32_t w0, uint32_t cap,
                         uint16_t* s_starts) {
  const uint32_t pos0 = threadIdx.x * 16;
  while (m) {
    const int j = __ffs(m) - 1;
    if (rank - w0 < cap) s_starts[rank - w0] = (uint16_t)(pos0 + j);
    ++rank;
    m &= m - 1;
  }
}

// Block-wide compaction of the word starts of a stage (one 16-bit mask per thread), in text
// order: the starts of rank < cap go to s_starts; *rank0 = the rank of this thread's first
// start, for later windows. Returns the number of starts. Contains two barriers.
template <int BLOCK>
WC_DEV uint32_t compact_starts(uint32_t start16, uint32_t* s_wsum, uint16_t* s_starts,
                               uint32_t cap, uint32_t* rank0) {
  constexpr int NW = BLOCK / 64;
  static_assert(NW <= 16, "wave totals are scanned within one 16-lane row");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t cnt = __popc(start16);
  const uint32_t incl = wave_incl_scan(cnt);
  if (lane == 63) s_wsum[wave] = incl;
  __syncthreads();
  const uint32_t ws = lane < NW ? s_wsum[lane] : 0u;
  uint32_t wi = ws;
  wi += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)wi, 0x111, 0xf, 0xf, false);
  wi += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)wi, 0x112, 0xf, 0xf, false);
  wi += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)wi, 0x114, 0xf, 0xf, false);
  wi += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)wi, 0x118, 0xf, 0xf, false);
  const uint32_t base = (uint32_t)__builtin_amdgcn_readlane((int)(wi - ws), wave);
  const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)wi, NW - 1);
  const uint32_t o = base + incl - cnt;
  *rank0 = o;
  write_starts(start16, o, 0, cap, s_starts);
  __syncthreads();
  return total;
}

// ---------------------------------------------------------------------------------------
// dictionary: sample, threshold, placement
// ---------------------------------------------------------------------------------------
// kSamplePer stages per workgroup, all spread evenly over the text; the workgroup counts them
// in one LDS table and adds it to the sample table once (fewer workgroups adding the same hot
// words). Document boundaries are ignored and words cut at the stage edges count as they
// appear: the sample only ranks words.
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
  LdsWords T{s_lo, s_hi, s_cnt, kSampleLds};
  for (uint32_t i = tid; i < kSampleLds; i += BLOCK) {
    s_lo[i] = 0;
    s_hi[i] = 0;
    s_cnt[i] = 0;
  }
  if (tid < 2) s_txt4[BLOCK + tid] = make_uint4(0, 0, 0, 0);
  if (tid == 0) {
    s_live = 0;
    s_last[BLOCK] = 0;
  }
  const uint32_t cap = kSampleLds - kSampleLds / 4;
  const uint64_t n_sampled = (uint64_t)gridDim.x * kSamplePer;
  for (uint32_t it = 0; it < kSamplePer; ++it) {
    const uint64_t k = ((uint64_t)blockIdx.x * kSamplePer + it) * P.n_stages / n_sampled;
    const int64_t ls = P.base_off + (int64_t)(k * kGlobalStage);  // first STAGE bytes of it
    uint32_t w16;
    const uint4 g = classify16(load_text16(P.corpus, P.len, ls + tid * 16), &w16);
    w16 = cut16(w16, ls + tid * 16, R0, R1);
    __syncthreads();  // the previous stage's tokens are done with the staged text
    s_txt4[tid] = g;
    s_wm[tid] = (uint16_t)w16;
    __syncthreads();
    const uint32_t prev = tid > 0 ? (s_wm[tid - 1] >> 15) : 0u;
    const uint32_t next = tid < BLOCK - 1 ? (s_wm[tid + 1] & 1u) : 0u;
    const uint32_t start16 = w16 & ~((w16 << 1) | prev) & 0xffffu;
    const uint32_t last16 = w16 & ~((w16 >> 1) | (next << 15)) & 0xffffu;
    s_last[tid] = (uint16_t)last16;
    uint32_t rank0;
    // without document boundaries a start follows a delimiter, so a stage has <= STAGE / 2
    const uint32_t total = min(compact_starts<BLOCK>(start16, s_wsum, s_starts, STAGE / 2, &rank0),
                               (uint32_t)STAGE / 2);
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
  }
  __syncthreads();
  // Every workgroup's LDS table has the same layout (same hash, same size), so a hot word sits
  // at the same entry in all of them: walked in entry order, all workgroups would add to its
  // device slot at once. Each starts its walk at its own entry.
  const uint32_t rot = (blockIdx.x * 1031u) & (kSampleLds - 1);
  for (uint32_t j = tid; j < kSampleLds; j += BLOCK) {
    const uint32_t i = (j + rot) & (kSampleLds - 1);
    const uint32_t c = s_cnt[i];
    if (c) sample_insert(P.sample_table, kSampleSlots - 1, s_lo[i], s_hi[i] & ~kTop, c);
  }
}

// Count threshold of the selection: words with a sample count (clamped at 255) >= t fit the
// dictionary (acc of them); `room` more may come from count t - 1. hist is an LDS copy of the
// count histogram: from device memory, each step of the loop, which may stop at any count,
// would wait for its own load.
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

// The selected words of a workgroup's slots are listed in LDS and take their places in the
// dictionary with one device atomic per list (a word that finds the list full takes its own).
__global__ __launch_bounds__(256) void dict_select_kernel(GlobalParams P) {
  constexpr uint32_t kList = 256;
  __shared__ uint32_t s_t, s_acc, s_room, s_n[2], s_base[2];
  __shared__ uint4 s_key[2][kList];
  __shared__ uint32_t s_c[2][kList];
  __shared__ uint32_t s_hist[256];
  for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) s_hist[i] = P.dict->hist[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t, acc, room;
    dict_threshold(s_hist, P.dict_cap, &t, &acc, &room);
    s_t = t;
    s_acc = acc;
    s_room = room;
    s_n[0] = s_n[1] = 0;
  }
  __syncthreads();
  const uint32_t t = s_t, acc = s_acc, room = s_room;
  // list 0: count >= t (all fit, positions from 0); list 1: count t - 1 (the first `room` of
  // them fit, positions from acc)
  auto place = [&](uint32_t which, uint32_t j, const uint4 k, uint32_t c) {
    if (which == 0 ? j < acc : j < room) {
      P.dict->keys[(which == 0 ? 0u : acc) + j] = k;
      P.dict->cnt[(which == 0 ? 0u : acc) + j] = c;
    }
  };
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < kSampleSlots;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const Slot s = P.sample_table[i];
    if (!s.key) continue;
    const uint32_t c = s.cnt < 255 ? (uint32_t)s.cnt : 255u;
    const uint32_t which = c >= t ? 0u : (c + 1 == t && room) ? 1u : 2u;
    if (which == 2) continue;
    const uint4 k = key4(s.w0, s.w1 & ~kTop);
    const uint32_t l = atomicAdd(&s_n[which], 1u);
    if (l < kList) {
      s_key[which][l] = k;
      s_c[which][l] = c;
    } else {
      place(which, atomicAdd(which == 0 ? &P.dict->n_high : &P.dict->n_low, 1u), k, c);
    }
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const uint32_t n = min(s_n[threadIdx.x], kList);
    s_base[threadIdx.x] =
        n ? atomicAdd(threadIdx.x == 0 ? &P.dict->n_high : &P.dict->n_low, n) : 0u;
  }
  __syncthreads();
  for (uint32_t which = 0; which < 2; ++which) {
    const uint32_t n = min(s_n[which], kList);
    for (uint32_t l = threadIdx.x; l < n; l += blockDim.x)
      place(which, s_base[which] + l, s_key[which][l], s_c[which][l]);
  }
}

// kBuildGroups workgroups build the perfect hash of the selected words (hash and displace,
// after Belazzougui, Botelho and Dietzfelbinger): each groups all the words by the low bits of
// their hash, then its 16 waves fill its share of the 256-slot regions, one region per wave,
// each region with its 32 groups one after another, largest first (the placement was 135 of
// the 167 us of one workgroup filling two regions per wave); a group
// takes the first displacement that sends all of its words to free slots. Inside a group the
// hottest words come first; a word that cannot be placed with the others (the same slot field
// as a hotter word of its group in both fields, or no free displacement) is left out of the
// dictionary, which only moves its counting to the partitions.
constexpr uint32_t kBuildGroups = 2;
static_assert(kDictRegions % kBuildGroups == 0 && kDictRegions / kBuildGroups <= 16,
              "whole regions per workgroup, at most one per wave");
__global__ __launch_bounds__(1024) void dict_build_kernel(GlobalParams P) {
  constexpr uint32_t kMaxGroup = 64;  // words of one group placed at most (one per lane)
  constexpr uint32_t kRegionGroups = kDispBuckets / kDictRegions;
  static_assert(kDictSlots == kDictRegions * 256 && kRegionGroups <= 64, "256-slot regions");
  __shared__ uint32_t s_h[kDictMax];
  __shared__ uint8_t s_c8[kDictMax];      // sample counts (clamped at 255)
  __shared__ uint16_t s_gkeys[kDictMax];  // key indices grouped by group, hottest first
  __shared__ uint32_t s_gn[kDispBuckets], s_gstart[kDispBuckets];
  __shared__ uint8_t s_ord[kDictRegions][kRegionGroups];
  __shared__ uint32_t s_occ[kDictSlots / 32];
  __shared__ uint16_t s_slot[kDictSlots];
  __shared__ uint16_t s_disp[kDispBuckets];
  __shared__ uint32_t s_n, s_placed;
  __shared__ uint32_t s_hist[256];
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < 256; i += blockDim.x) s_hist[i] = P.dict->hist[i];
  __syncthreads();
  if (tid == 0) {
    uint32_t t, acc, room;
    dict_threshold(s_hist, P.dict_cap, &t, &acc, &room);
    const uint32_t low = P.dict->n_low;
    s_n = acc + (low < room ? low : room);
    s_placed = 0;
  }
  for (uint32_t i = tid; i < kDispBuckets; i += blockDim.x) {
    s_gn[i] = 0;
    s_disp[i] = 0;
  }
  for (uint32_t i = tid; i < kDictSlots / 32; i += blockDim.x) s_occ[i] = 0;
  __syncthreads();
  const uint32_t n = s_n;
  for (uint32_t i = tid; i < kDictSlots; i += blockDim.x) s_slot[i] = (uint16_t)n;
  for (uint32_t i = tid; i < n; i += blockDim.x) {
    const uint4 k = P.dict->keys[i];
    const uint32_t h = word_hash32((uint64_t)k.x | ((uint64_t)k.y << 32),
                                   (uint64_t)k.z | ((uint64_t)k.w << 32));
    s_h[i] = h;
    s_c8[i] = (uint8_t)P.dict->cnt[i];
    atomicAdd(&s_gn[dict_group(h)], 1u);
  }
  __syncthreads();
  if (tid < 64) {  // group starts: a scan over the groups, 8 per lane
    uint32_t v[kDispBuckets / 64], sum = 0;
    for (uint32_t j = 0; j < kDispBuckets / 64; ++j) {
      v[j] = sum;
      sum += s_gn[tid * (kDispBuckets / 64) + j];
    }
    const uint32_t incl = wave_incl_scan(sum);
    for (uint32_t j = 0; j < kDispBuckets / 64; ++j)
      s_gstart[tid * (kDispBuckets / 64) + j] = incl - sum + v[j];
  }
  __syncthreads();
  for (uint32_t g = tid; g < kDispBuckets; g += blockDim.x) s_gn[g] = 0;
  __syncthreads();
  for (uint32_t i = tid; i < n; i += blockDim.x) {
    const uint32_t g = dict_group(s_h[i]);
    s_gkeys[s_gstart[g] + atomicAdd(&s_gn[g], 1u)] = (uint16_t)i;
  }
  __syncthreads();
  for (uint32_t g = tid; g < kDispBuckets; g += blockDim.x) {  // hottest first in each group
    uint16_t* a = s_gkeys + s_gstart[g];
    const uint32_t m = s_gn[g];
    for (uint32_t x = 1; x < m; ++x) {
      const uint16_t v = a[x];
      const uint32_t cv = s_c8[v];
      uint32_t y = x;
      while (y > 0 && s_c8[a[y - 1]] < cv) {
        a[y] = a[y - 1];
        --y;
      }
      a[y] = v;
    }
  }
  __syncthreads();
  const uint32_t lane = tid & 63;
  // this workgroup's regions [r0, r1); wave v fills regions r0 + v, r0 + v + 16, ...
  const uint32_t per_wg = kDictRegions / gridDim.x;
  const uint32_t r0 = blockIdx.x * per_wg, r1 = r0 + per_wg;
  for (uint32_t r = r0 + (tid >> 6); r < r1; r += blockDim.x / 64) {
    // the region's groups g = r + 16 L, largest first
    const uint32_t my_n = lane < kRegionGroups ? s_gn[r + kDictRegions * lane] : 0u;
    uint32_t rank = 0;
    for (uint32_t x = 0; x < kRegionGroups; ++x) {
      const uint32_t nx = (uint32_t)__builtin_amdgcn_readlane((int)my_n, (int)x);
      rank += (nx > my_n || (nx == my_n && x < lane)) ? 1u : 0u;
    }
    if (lane < kRegionGroups) s_ord[r][rank] = (uint8_t)lane;
    wave_sync();
    uint32_t placed = 0;
    for (uint32_t o = 0; o < kRegionGroups; ++o) {
      const uint32_t g = r + kDictRegions * s_ord[r][o];
      const uint32_t m = min(s_gn[g], kMaxGroup);
      if (m == 0) break;  // the rest are empty
      const uint32_t ki = lane < m ? s_gkeys[s_gstart[g] + lane] : 0u;
      const uint32_t h = s_h[ki];
      // field select: the one that leaves fewer words out (a word whose field repeats a hotter
      // word's field is left out)
      const uint32_t f0 = dict_field(h, 0), f1 = dict_field(h, 1);
      bool k0 = lane < m, k1 = lane < m;
      for (uint32_t x = 0; x < m; ++x) {
        const uint32_t a0 = (uint32_t)__builtin_amdgcn_readlane((int)f0, (int)x);
        const uint32_t a1 = (uint32_t)__builtin_amdgcn_readlane((int)f1, (int)x);
        if (x < lane && a0 == f0) k0 = false;
        if (x < lane && a1 == f1) k1 = false;
      }
      const uint64_t km0 = __ballot(k0), km1 = __ballot(k1);
      const uint32_t sel = __popcll(km1) > __popcll(km0) ? 1u : 0u;
      uint64_t km = sel ? km1 : km0;
      const uint32_t f = sel ? f1 : f0;
      uint32_t d = 0;
      bool found = false;
      while (km && !found) {
        for (uint32_t base = 0; base < 256 && !found; base += 64) {
          const uint32_t cand = base + lane;
          bool ok = true;
          for (uint64_t rem = km; rem;) {
            uint32_t sl[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              sl[u] = 0xffffffffu;
              if (rem) {
                const uint32_t x = (uint32_t)__ffsll((unsigned long long)rem) - 1;
                rem &= rem - 1;
                sl[u] = (r << 8) | (((uint32_t)__builtin_amdgcn_readlane((int)f, (int)x) ^ cand) & 0xffu);
              }
            }
            uint32_t wv8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) wv8[u] = sl[u] != 0xffffffffu ? s_occ[sl[u] >> 5] : 0u;
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (sl[u] != 0xffffffffu && ((wv8[u] >> (sl[u] & 31)) & 1u)) ok = false;
          }
          const uint64_t okm = __ballot(ok);
          if (okm) {
            d = base + (uint32_t)__ffsll((unsigned long long)okm) - 1;
            found = true;
          }
        }
        if (!found) km &= ~(1ull << (63 - __clzll(km)));  // leave out the coldest and retry
      }
      if (found) {
        if ((km >> lane) & 1ull) {
          const uint32_t sl = (r << 8) | ((f ^ d) & 0xffu);
          atomicOr(&s_occ[sl >> 5], 1u << (sl & 31));
          s_slot[sl] = (uint16_t)ki;
        }
        if (lane == 0) s_disp[g] = (uint16_t)(d | (sel << 8));
        placed += (uint32_t)__popcll(km);
      }
      wave_sync();
    }
    if (lane == 0) atomicAdd(&s_placed, placed);
  }
  __syncthreads();
  // the displacements of this workgroup's groups (g mod kDictRegions in [r0, r1)) and the
  // slots of its regions; the placed counts add up (the image and the header start at zero)
  for (uint32_t i = tid; i < kDispBuckets; i += blockDim.x)
    if ((i & (kDictRegions - 1)) - r0 < per_wg) P.dict->disp[i] = s_disp[i];
  for (uint32_t i = r0 * 256 + tid; i < r1 * 256; i += blockDim.x) P.dict->slot[i] = s_slot[i];
  if (tid == 0) {
    if (blockIdx.x == 0) {
      P.dict->keys[n] = make_uint4(0, 0, 0, 0);
      P.dict->n = n;
    }
    atomicAdd(&P.dict->placed, s_placed);
    add64(&P.hdr->stat[2], s_placed);
  }
}

// ---------------------------------------------------------------------------------------
// pass 1
// ---------------------------------------------------------------------------------------
constexpr int kMapWaves = kMapBlock / 64;

size_t global_map_dyn(uint32_t dict_cap) {
  return (size_t)kMapWaves * kStripeText +
         (size_t)kDispBuckets * 4 + (size_t)kDictSlots * 2 + (size_t)(dict_cap + 1) * 16 +
         (size_t)dict_cap * 4 +
         (size_t)kMapWaves * kWaveStarts * 4;
}

// One workgroup of BLOCK threads scans a contiguous range of STAGE-byte stages; wave v takes
// a contiguous run of the range's 1 KiB stripes and runs on its own, with no workgroup barrier
// until the range ends. Per stripe: classify 16 bytes per lane (plus the byte before the
// stripe), word start / end masks, a wave-wide compaction of the word starts (with a bitmap of
// the word ends beside it), and up to two tokens per lane per round: counted in the
// dictionary, or written as a record to its partition, or (longer than 16 bytes) counted in the
// global table.
//
// Records. Each partition's records of this workgroup go to the workgroup's own blocks of that
// partition, in the order of a per-partition ticket taken with one LDS atomic: ticket t is
// slot t mod 256 of the workgroup's (t / 256)-th block. The arena is laid out workgroup-major:
// block k = w * J + j of partition p (workgroup w, its j-th block, J per workgroup) sits at
// arena block k * 256 + p, so the blocks a workgroup is filling lie side by side in one 1 MiB
// span instead of at a large power-of-two stride (which mapped them to few cache sets and had
// lines written back before they were full). Lanes store their records straight to the arena,
// one 16-byte store each. The lane holding a block's last slot sets its fill to full; the
// workgroup sets the fill of each partition's last, partial block when its range is done. A
// partition whose share of blocks is used up sends the rest of its records to the global
// table.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void global_map_kernel(GlobalParams P) {
  constexpr int NW = BLOCK / 64;
  constexpr int STAGE = BLOCK * 16;
  static_assert(STAGE == (int)kGlobalStage && NW * (int)kStripe == STAGE,
                "a stage is one stripe per wave");
  static_assert(NW == kMapWaves && BLOCK >= (int)kParts, "one thread per partition at the end");
  static_assert(kWaveStarts == 128, "a round takes two tokens per lane");
  extern __shared__ __align__(16) uint8_t s_dyn[];
  __shared__ uint32_t s_tick[kParts];  // records of each partition so far
  __shared__ uint4 s_lenmask[17];       // byte masks of word lengths 0..16
  __shared__ uint32_t s_bnd[NW][kBndWords];
  __shared__ uint32_t s_stat[4];

  const uint32_t D = P.dict_cap;
  uint8_t* s_txt = s_dyn;                                       // [NW][kStripeText]
  // group g's displacement d (8 bits and the field select) unpacked for the lookup: the byte
  // offset of its slot region in s_dslot (bits 16..31), the field's shift (bits 8..12), d's low
  // 8 bits (bits 0..7)
  uint32_t* s_disp = (uint32_t*)(s_txt + NW * kStripeText);    // [kDispBuckets]
  uint16_t* s_dslot = (uint16_t*)(s_disp + kDispBuckets);       // [kDictSlots]
  uint4* s_keys = (uint4*)(s_dslot + kDictSlots);               // [D + 1]
  uint32_t* s_cnt = (uint32_t*)(s_keys + D + 1);                // [D]
  uint32_t* s_pairs = s_cnt + D;                                // [NW][kWaveStarts]

  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  Header* hdr = P.hdr;
  if (ld_relaxed32(&hdr->flags) & kFlagBadOffsets) return;
  const uint64_t st0 = (uint64_t)blockIdx.x * P.stages_per_wg;
  const uint64_t st1 = min(st0 + P.stages_per_wg, P.n_stages);
  const uint64_t n_stages = P.n_stages;
  const int64_t R0 = (int64_t)P.offsets[0], R1 = (int64_t)P.offsets[P.n_docs];

  const uint32_t nd = P.dict->n;
  for (uint32_t i = tid; i < kDispBuckets; i += BLOCK) {
    const uint32_t d = P.dict->disp[i];
    s_disp[i] = ((i & (kDictRegions - 1)) << 25) |
                ((__builtin_ctz(kDispBuckets) + 8 * ((d >> 8) & 1u)) << 8) | (d & 0xffu);
  }
  for (uint32_t i = tid; i < kDictSlots; i += BLOCK) s_dslot[i] = P.dict->slot[i];
  for (uint32_t i = tid; i <= nd; i += BLOCK) s_keys[i] = P.dict->keys[i];
  for (uint32_t i = tid; i < nd; i += BLOCK) s_cnt[i] = 0;
  for (uint32_t p = tid; p < kParts; p += BLOCK) s_tick[p] = 0;
  init_len_masks(s_lenmask, tid, BLOCK);
  for (uint32_t i = tid; i < NW * kBndWords; i += BLOCK) (&s_bnd[0][0])[i] = 0;
  for (uint32_t i = tid; i < NW * kWaveStarts; i += BLOCK) s_pairs[i] = 0;
  if (tid < 4) s_stat[tid] = 0;
  __syncthreads();

  // This workgroup's j-th block of partition p is block k = w * J + j (J = S / G blocks each).
  const uint32_t G = gridDim.x, w = blockIdx.x;
  const uint32_t J = P.S / G;
  uint8_t* const my_txt = s_txt + wv * kStripeText;
  uint32_t* const my_bnd = s_bnd[wv];
  // per wave: kWaveStarts 16-bit starts, then the word-end bitmap
  uint16_t* const my_starts = (uint16_t*)(s_pairs + wv * kWaveStarts);
  uint32_t* const my_ends = s_pairs + wv * kWaveStarts + kWaveStarts / 2;
  static_assert(kWaveStarts / 2 + kEndWords <= kWaveStarts, "starts and ends fit a wave's list");

  auto insert_record = [&](const uint4 r) {
    const uint64_t lo = (uint64_t)r.x | ((uint64_t)r.y << 32);
    const uint64_t hi = (uint64_t)r.z | ((uint64_t)r.w << 32);
    table_insert<false>(P.table, P.mask, short_key_g<false>(lo, hi, P.key_mask),
                        short_id(lo, hi, 0), 1, hdr, P.occ_limit);
  };
  // first document start after pos (offsets[n_docs], the end of the range, is one)
  auto doc_limit = [&](uint64_t pos) -> uint64_t {
    uint64_t a = 1, b = P.n_docs;
    while (a < b) {
      const uint64_t m = (a + b) >> 1;
      if (P.offsets[m] > pos) b = m;
      else a = m + 1;
    }
    return P.offsets[a];
  };

  uint32_t spilled = 0, direct = 0;

  // a word longer than 16 bytes (or with its end beyond the staged bytes): from device memory,
  // into the global table
  auto long_token = [&](int64_t p0, uint32_t s, uint32_t e) {
    const uint64_t start = (uint64_t)(p0 + s);
    const uint64_t limit = e == kLongEnd ? doc_limit(start) : start + (e - s + 1);
    uint64_t lo, hi, h64;
    const uint64_t n = scan_word(P.corpus, start, limit, &lo, &hi, &h64);
    if (n > 16) {
      table_insert<false>(P.table, P.mask, finish_key(h64, P.key_mask),
                          long_id(P.corpus + start, n, 0), 1, hdr, P.occ_limit);
    } else {
      table_insert<false>(P.table, P.mask, short_key_g<false>(lo, hi, P.key_mask),
                          short_id(lo, hi, 0), 1, hdr, P.occ_limit);
    }
  };

  // One round: starts t and t + 64 of this wave's list (t = lane), for those below nw. A word's
  // end is the first set bit of the end bitmap at or after its start. Both tokens go through
  // each step together, so their LDS reads overlap. A token that misses the dictionary becomes
  // a record of its partition.
  auto token_round = [&](uint32_t nw, int64_t p0) {
    uint32_t s2[2], n2[2], e0[2], e1[2];
    bool f2[2];
    // (list entries past nw are stale starts of earlier rounds: in range, not counted)
#pragma unroll
    for (int x = 0; x < 2; ++x) s2[x] = my_starts[lane + 64 * x];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      e0[x] = my_ends[s2[x] >> 5];
      e1[x] = my_ends[(s2[x] >> 5) + 1];
    }
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      n2[x] = __ffs(__builtin_amdgcn_alignbit(e1[x], e0[x], s2[x] & 31));  // 0: no end in 32
      f2[x] = lane + 64 * x < nw && n2[x] - 1 < 16u;
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
      if (lane + 64 * x < nw && !f2[x]) {
        long_token(p0, s2[x], n2[x] ? s2[x] + n2[x] - 1 : kLongEnd);
        wait_vmem();
      }
    // each LDS step reads for both tokens before either waits (pin)
    PackSrc ps[2];
    uint4 lm[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      ps[x] = pack_read(my_txt, s2[x]);
      lm[x] = s_lenmask[f2[x] ? n2[x] : 1u];
    }
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      pin(ps[x]);
      pin(lm[x]);
    }
    uint64_t lo2[2], hi2[2];
    uint32_t h2[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      pack_join(ps[x], lm[x], &lo2[x], &hi2[x]);
      h2[x] = word_hash32(lo2[x], hi2[x]);
    }
    // the perfect hash's slot (dict_slot) from the unpacked displacement
    uint32_t d2[2], i2[2];
    uint4 k2[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) d2[x] = s_disp[dict_group(h2[x])];
#pragma unroll
    for (int x = 0; x < 2; ++x) pin(d2[x]);
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const uint32_t f = (h2[x] >> ((d2[x] >> 8) & 31u)) ^ d2[x];
      i2[x] = *(const uint16_t*)((const uint8_t*)s_dslot + (d2[x] >> 16) + ((f & 0xffu) << 1));
    }
#pragma unroll
    for (int x = 0; x < 2; ++x) pin(i2[x]);
#pragma unroll
    for (int x = 0; x < 2; ++x) k2[x] = s_keys[i2[x]];
#pragma unroll
    for (int x = 0; x < 2; ++x) pin(k2[x]);
    bool m2[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const bool hit = key_eq(k2[x], key4(lo2[x], hi2[x]));
      if (f2[x] && hit) atomicAdd(&s_cnt[i2[x]], 1u);
      m2[x] = f2[x] && !hit;
    }
    uint32_t t2[2] = {0u, 0u};
#pragma unroll
    for (int x = 0; x < 2; ++x)
      if (m2[x]) t2[x] = atomicAdd(&s_tick[part_of(h2[x])], 1u);
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      if (m2[x]) {
        const uint32_t p = part_of(h2[x]), j = t2[x] / kBlockRec, at = t2[x] % kBlockRec;
        const uint4 rec = key4(lo2[x], hi2[x]);
        if (j < J) {
          const uint64_t k = (uint64_t)w * J + j;
          P.arena[(k * kParts + p) * kBlockRec + at] = rec;
          if (at == kBlockRec - 1) P.fill[(uint64_t)p * P.S + k] = (uint16_t)kBlockRec;
        } else {
          ++direct;  // the partition's share of blocks is used up
          insert_record(rec);
        }
      }
    }
    spilled += (m2[0] ? 1u : 0u) + (m2[1] ? 1u : 0u);
  };

  // Wave wv scans its own contiguous run of nsw stripes of the workgroup's range. The word
  // byte before a stripe and the word that runs over a stripe's end come from the wave's
  // previous stripe: its last 16 bytes stay in LDS as the prefix of the next stripe's text
  // (my_txt: 16-byte prefix, the stripe, 16 bytes of padding), and such a word is finished by
  // the next stripe.
  const uint64_t nsw = st1 > st0 ? st1 - st0 : 0;
  const uint64_t sw0 = st0 * NW + (uint64_t)wv * nsw;
  auto stripe_pos = [&](uint64_t i) -> int64_t {
    return P.base_off + (int64_t)((sw0 + i) * kStripe);
  };
  // a stripe inside the text (the wave-uniform common case) is loaded without per-lane checks
  auto load_main = [&](uint64_t i) -> uint4 {
    const int64_t p = stripe_pos(i);
    if (p >= 0 && p + (int64_t)kStripe <= (int64_t)P.len) return load_stream16(P.corpus + p + lane * 16);
    return load_text16(P.corpus, P.len, p + lane * 16);
  };

  const uint4 blank = make_uint4(0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u);
  uint4 cur = blank, nx = blank;
  uint32_t carry = 0;  // the byte before the stripe is a word byte (wave-uniform)
  if (nsw > 0) {
    cur = load_main(0);
    const int64_t q = stripe_pos(0) - 1;
    uint32_t f;
    fold_classify4(load_text4(P.corpus, P.len, q - 3), &f);
    carry = (q >= R0 && q < R1) ? f >> 31 : 0u;
  }
  if (nsw > 1) nx = load_main(1);
  uint64_t tokens = 0;  // wave-uniform
  bool def = false;     // a word of the previous stripe runs over its end (wave-uniform) ...
  uint32_t def_s = 0;   // ... from prefix byte def_s
  // no document starts in the wave's whole run and it lies inside [R0, R1): every stripe is
  // plain, and the per-stripe cursor reads are skipped
  bool run_plain = false;
  if (nsw > 0) {
    const uint64_t sa = sw0 / NW, sb = min((sw0 + nsw - 1) / NW + 1, n_stages);
    run_plain = P.stage_doc[sa] == P.stage_doc[sb] && stripe_pos(0) >= R0 &&
                stripe_pos(nsw) <= R1;
  }

  for (uint64_t i = 0; i < nsw; ++i) {
    const int64_t p0 = stripe_pos(i);
    // documents starting in [p0, p0 + kStripe): the first at or after the stage start is
    // stage_doc[stage]
    uint64_t c0 = 0, c2 = 0;
    bool plain = run_plain;
    if (!run_plain) {
      const uint64_t stage = (sw0 + i) / NW;
      c0 = P.stage_doc[stage];
      c2 = P.stage_doc[min(stage + 1, n_stages)];
      plain = c2 == c0 && p0 >= R0 && p0 + (int64_t)kStripe <= R1;
    }

    // ---- classify ---------------------------------------------------------------------------
    uint32_t w16;
    const uint4 g = classify16(cur, &w16);
    if (!plain) w16 = cut16(w16, p0 + lane * 16, R0, R1);
    ((uint4*)my_txt)[1 + lane] = g;
    cur = nx;
    if (i + 2 < nsw) nx = load_main(i + 2);

    // ---- document starts of the stripe ---------------------------------------------------
    uint32_t bnd16 = 0, bnext = 0;
    if (!plain) {
      if (c2 > c0) {
        uint64_t j0 = c0, j1 = c2;
        while (j1 - j0 > 64) {  // first document starting at or after p0
          const uint64_t m = (j0 + j1) >> 1;
          if ((int64_t)P.offsets[m] < p0) j0 = m + 1;
          else j1 = m;
        }
        for (uint64_t jb = j0; jb < c2; jb += 64) {
          const uint64_t j = jb + lane;
          const int64_t o = j < c2 ? (int64_t)P.offsets[j] : INT64_MAX;
          if (o >= p0 && o < p0 + (int64_t)kStripe) {
            const uint32_t rel = (uint32_t)(o - p0);
            atomicOr(&my_bnd[rel >> 5], 1u << (rel & 31));
          }
          if (__all(o >= p0 + (int64_t)kStripe)) break;
        }
        wave_sync();
      }
      bnd16 = (my_bnd[lane >> 1] >> ((lane & 1) * 16)) & 0xffffu;
      bnext = (my_bnd[(lane + 1) >> 1] >> (((lane + 1) & 1) * 16)) & 1u;  // lane 63: 0
      wave_sync();
      if (lane < (int)kBndWords) my_bnd[lane] = 0;
    }

    // ---- word starts and ends --------------------------------------------------------------
    // previous lane's last byte (lane 0: the byte before the stripe); next lane's first byte
    // (lane 63: taken as a word byte: a word running to the stripe's end is finished by the
    // next stripe)
    const uint32_t prev =
        (uint32_t)__builtin_amdgcn_update_dpp((int)carry, (int)(w16 >> 15), 0x138, 0xf, 0xf, false);
    const uint32_t nxt =
        (uint32_t)__builtin_amdgcn_update_dpp(1, (int)(w16 & 1u), 0x130, 0xf, 0xf, false);
    uint32_t start16 = w16 & (~((w16 << 1) | prev) | bnd16) & 0xffffu;
    const uint32_t last16 = w16 & (~((w16 >> 1) | (nxt << 15)) | (bnd16 >> 1) | (bnext << 15)) & 0xffffu;
    // lane 63's last word, when it runs to the stripe's end, is left for the next stripe
    uint32_t ndef_j = 16;
    if (lane == 63 && start16) {
      const uint32_t j = 31 - __clz(start16);
      if ((last16 >> j) == 0) {
        ndef_j = j;
        start16 &= ~(1u << j);
      }
    }
    // end bitmap: lane l's ends at half-word 1 + l; half-word 0 (the prefix) holds one end, at
    // its last byte, when the previous stripe's last word stops there (lane 0's first byte does
    // not continue it)
    ((uint16_t*)my_ends)[1 + lane] = (uint16_t)last16;
    if (lane == 0) {
      const bool cont = (w16 & ~start16 & 1u) != 0;
      ((uint16_t*)my_ends)[0] = (uint16_t)(def && !cont ? 0x8000u : 0u);
    }

    // ---- compaction and tokens, kWaveStarts at a time -------------------------------------
    const uint32_t extra = (def && lane == 0) ? 1u : 0u;  // the carried word takes rank 0
    const uint32_t c = __popc(start16) + extra;
    const uint32_t incl = wave_incl_scan(c);
    const uint32_t n = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    tokens += n;
    for (uint32_t w0 = 0; w0 < n; w0 += kWaveStarts) {
      if (extra && w0 == 0) my_starts[0] = (uint16_t)def_s;
      write_starts16(start16, incl - c + extra, w0, my_starts);
      wave_sync();
      token_round(min(n - w0, kWaveStarts), p0 - 16);
      wave_sync();
    }
    // the stripe's last 16 bytes become the next stripe's prefix
    if (lane == 63) ((uint4*)my_txt)[0] = ((const uint4*)my_txt)[1 + 63];
    wave_sync();
    def = __builtin_amdgcn_readlane((int)ndef_j, 63) < 16;
    def_s = (uint32_t)__builtin_amdgcn_readlane((int)ndef_j, 63);
    carry = (uint32_t)__builtin_amdgcn_readlane((int)(w16 >> 15), 63);
  }
  // a word running over the range's end: from device memory
  if (def) {
    tokens += 1;
    if (lane == 0) long_token(stripe_pos(nsw) - 16, def_s, kLongEnd);
  }

  // ---- end of range: each partition's last block gets its fill; dictionary hits go out ----
  __syncthreads();
  if (tid < (int)kParts) {
    const uint32_t t = s_tick[tid], j = t / kBlockRec, at = t % kBlockRec;
    if (at && j < J) P.fill[(uint64_t)tid * P.S + (uint64_t)w * J + j] = (uint16_t)at;
  }
  for (uint32_t i = tid; i < nd; i += BLOCK) P.dict_part[(uint64_t)blockIdx.x * D + i] = s_cnt[i];
  if (spilled) atomicAdd(&s_stat[0], spilled);
  if (direct) atomicAdd(&s_stat[1], direct);
  if (lane == 0 && tokens) add64(&hdr->total_tokens, tokens);
  __syncthreads();
  if (tid == 0) {
    if (s_stat[0]) add64(&hdr->stat[0], s_stat[0]);
    if (s_stat[1]) add64(&hdr->stat[1], s_stat[1]);
  }
}

// ---------------------------------------------------------------------------------------
// pass 2: one workgroup per partition
// ---------------------------------------------------------------------------------------
size_t global_reduce_dyn(uint32_t entries) { return (size_t)kRedSlots * 4 + (size_t)entries * 20; }

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void global_reduce_kernel(GlobalParams P) {
  extern __shared__ __align__(16) uint8_t s_dyn[];
  __shared__ uint32_t s_nent, s_miss, s_nlist;
  __shared__ unsigned long long s_dsum[kDictCols];
  __shared__ uint16_t s_list[kWinBlocks], s_lfill[kWinBlocks];
  const uint32_t p = blockIdx.x;
  const int tid = threadIdx.x;
  Header* hdr = P.hdr;
  if (ld_relaxed32(&hdr->flags) & kFlagBadOffsets) return;
  const uint32_t E = P.reduce_entries;
  RedTable T;
  T.slot = (uint32_t*)s_dyn;
  T.key = (uint4*)(T.slot + kRedSlots);
  T.cnt = (uint32_t*)(T.key + E);
  T.n = &s_nent;
  T.cap = P.reduce_cap < E ? P.reduce_cap : E;
  T.stall = nullptr;  // a word the table gives up on is summed in the global table
  for (uint32_t i = tid; i < kRedSlots; i += BLOCK) T.slot[i] = 0;
  for (uint32_t i = tid; i < E; i += BLOCK) {
    T.key[i] = make_uint4(0, 0, 0, 0);
    T.cnt[i] = 0;
  }
  for (uint32_t i = tid; i < kDictCols; i += BLOCK) s_dsum[i] = 0;
  if (tid == 0) {
    s_nent = 0;
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

  // records of partition p: blocks k < S (every pass-1 workgroup's share); the non-empty ones
  // are listed kWinBlocks at a time and read whole. Block k is arena block k * 256 + p.
  const uint32_t nblk = P.S;
  const uint4* region = P.arena + (uint64_t)p * kBlockRec;
  const uint16_t* fills = P.fill + (uint64_t)p * P.S;
  constexpr uint32_t kPerIter = BLOCK / kBlockRec;  // blocks per iteration
  static_assert(BLOCK % kBlockRec == 0, "whole blocks per iteration");
  // b_in is the same for a whole wave (a block is 4 waves): list reads and block addresses
  // are scalar
  const uint32_t r_in = tid % kBlockRec;
  const uint32_t b_in = (uint32_t)__builtin_amdgcn_readfirstlane(tid / kBlockRec);
  static_assert(kBlockRec % 64 == 0, "a block spans whole waves");
  // kRec records per lane at once: the common case for all of them, then the rest one at a time
  constexpr int kRec = 4;
  // The common case (a word with an entry, found by the first tag match in the first two groups
  // of its probe sequence) is taken for all kRec records together: every pair of slot groups is
  // read, then every candidate key, so a wave waits for two LDS round trips per kRec records
  // instead of several per record.
  auto add_records = [&](const uint4* v, const bool* use) {
    uint32_t h[kRec], e[kRec];
    uint4 sa[kRec], sb[kRec], k4[kRec];
    bool d[kRec];
#pragma unroll
    for (int x = 0; x < kRec; ++x) h[x] = red_hash(v[x]);
#pragma unroll
    for (int x = 0; x < kRec; ++x) {
      sa[x] = ((const uint4*)T.slot)[red_group(h[x])];
      sb[x] = ((const uint4*)T.slot)[red_next_group(red_group(h[x]))];
    }
    // (pinned, each read stays whole: the optimiser would otherwise read the later slots of a
    // group only when the earlier ones miss, one round trip after another)
#pragma unroll
    for (int x = 0; x < kRec; ++x) {
      pin(sa[x]);
      pin(sb[x]);
    }
#pragma unroll
    for (int x = 0; x < kRec; ++x) e[x] = red_pick8(sa[x], sb[x], red_tag(h[x]));
    // (e = 0: entry 0 is read and not counted)
#pragma unroll
    for (int x = 0; x < kRec; ++x) k4[x] = T.key[e[x] & 0x1fffu];
#pragma unroll
    for (int x = 0; x < kRec; ++x) pin(k4[x]);
#pragma unroll
    for (int x = 0; x < kRec; ++x) {
      const bool eq = key_eq(k4[x], v[x]);
      const bool hit = use[x] & (e[x] != 0) & eq;
      if (hit) atomicAdd(&T.cnt[e[x] & 0x1fffu], 1u);
      d[x] = use[x] && !hit;
    }
#pragma unroll
    for (int x = 0; x < kRec; ++x) {
      if (__any(d[x])) {
        const uint64_t lo = (uint64_t)v[x].x | ((uint64_t)v[x].y << 32);
        const uint64_t hi = (uint64_t)v[x].z | ((uint64_t)v[x].w << 32);
        if (d[x] && !red_add(T, lo, hi, h[x])) {
          atomicAdd(&s_miss, 1u);
          table_insert<false>(P.table, P.mask, short_key_g<false>(lo, hi, P.key_mask),
                              short_id(lo, hi, 0), 1, hdr, P.occ_limit);
        }
      }
    }
  };
  for (uint32_t w0 = 0; w0 < nblk; w0 += kWinBlocks) {
    const uint32_t wn = min(kWinBlocks, nblk - w0);
    if (tid == 0) s_nlist = 0;
    __syncthreads();
    for (uint32_t k = tid; k < wn; k += BLOCK) {
      const uint32_t f = fills[w0 + k];
      if (f) {
        const uint32_t i = atomicAdd(&s_nlist, 1u);
        s_list[i] = (uint16_t)k;
        s_lfill[i] = (uint16_t)f;
      }
    }
    __syncthreads();
    const uint32_t nl = s_nlist;
    if (nl == 0) continue;
    // A thread takes record r_in of list entries e + x * kPerIter (x < kRec) per iteration.
    // Records arrive kDepth iterations ahead in register rings that are never rotated (a move
    // of a register with a load in flight would wait for it): the loop is unrolled by kDepth.
    // Loads never branch: past the list's end they read its first block and count nothing.
    constexpr int kDepth = 2;
    constexpr uint32_t kStep = kRec * kPerIter;
    uint4 v[kDepth][kRec];
    uint32_t f[kDepth][kRec];
    auto load = [&](uint32_t e, uint4& vv, uint32_t& ff) {
      const uint32_t ee = e < nl ? e : 0u;
      ff = e < nl ? s_lfill[ee] : 0u;
      vv = region[(uint64_t)(w0 + s_list[ee]) * (kParts * kBlockRec) + r_in];
    };
#pragma unroll
    for (int jj = 0; jj < kDepth; ++jj)
#pragma unroll
      for (int x = 0; x < kRec; ++x) load(jj * kStep + x * kPerIter + b_in, v[jj][x], f[jj][x]);
    for (uint32_t e0 = 0; e0 < nl; e0 += kDepth * kStep) {
#pragma unroll
      for (int jj = 0; jj < kDepth; ++jj) {
        bool use[kRec];
#pragma unroll
        for (int x = 0; x < kRec; ++x) use[x] = r_in < f[jj][x];
        add_records(v[jj], use);
        const uint32_t e = e0 + (jj + kDepth) * kStep + b_in;
#pragma unroll
        for (int x = 0; x < kRec; ++x) load(e + x * kPerIter, v[jj][x], f[jj][x]);
      }
    }
    __syncthreads();  // the list is rebuilt for the next window
  }
  __syncthreads();
  const uint32_t ne = min(s_nent, T.cap);
  for (uint32_t i = tid; i < ne; i += BLOCK) {
    const uint32_t c = T.cnt[i];
    if (c) {
      const uint4 k = T.key[i];
      const uint64_t lo = (uint64_t)k.x | ((uint64_t)k.y << 32);
      const uint64_t hi = (uint64_t)k.z | ((uint64_t)k.w << 32);
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
  hipError_t e = hipFuncSetAttribute((const void*)global_map_kernel<kMapBlock>,
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
  if (ns) hipLaunchKernelGGL(sample_kernel<512>, dim3((ns + kSamplePer - 1) / kSamplePer), dim3(512),
                             0, s, P);
  hipLaunchKernelGGL(dict_hist_kernel, dim3(256), dim3(256), 0, s, P);
  hipLaunchKernelGGL(dict_select_kernel, dim3(256), dim3(256), 0, s, P);
  hipLaunchKernelGGL(dict_build_kernel, dim3(kBuildGroups), dim3(1024), 0, s, P);
  if (a) {
    hipError_t e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(global_map_kernel<kMapBlock>, dim3(P.map_grid), dim3(kMapBlock),
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
