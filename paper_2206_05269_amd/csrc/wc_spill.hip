// Two-pass global count: the map (tokenise, hash) with a per-workgroup LDS table of hot
// words, and a partitioned reduce for everything else.
//
// Why two passes. Section 3.3 sums grouped counts of each word; on MI355X a word that is not
// in the workgroup's LDS table would cost one device-scope atomic per token, and random
// atomics run at ~2.7e10/s chip-wide (measured), far below the byte rate of the scan. So:
//
//   pass 1 (spill_count_kernel): scan the text as the direct kernel does; count words that
//     are in the LDS table there; write every other token as a 16-byte record (the packed
//     word, plus a count when it is not 1) to one of 256 partitions chosen by a hash of the
//     word. Records are staged per partition in LDS and leave in 128-byte pieces into 4 KiB
//     blocks of a partition arena, so the spill is sequential writes, not atomics. When the
//     LDS table fills, entries seen at most T times are moved out as records and the rest
//     stay (T adapts), which keeps the hottest words resident.
//   pass 2 (spill_reduce_kernel): one workgroup per partition reads that partition's records
//     (sequentially), sums them in an LDS table, and adds each distinct word once to the
//     global table, which the export step compacts.
//
// Words longer than 16 bytes (and anything that cannot be staged) go straight to the
// global table as in the direct kernel; counts stay exact on every path.
#include "wc_internal.h"

namespace wc {

// ---------------------------------------------------------------------------------------
// records
// ---------------------------------------------------------------------------------------
// A record is a packed short word (lo, hi). Word bytes are below 0x80, so the top bit of each
// of the 16 bytes is free: a record with count 1 leaves them clear; otherwise the top bit of
// byte 0 of lo is set and the count (1..32767) is spread over the other 15 top bits.
constexpr uint64_t kTopBits = 0x8080808080808080ull;
constexpr uint32_t kMaxRecordCount = 32767;

WC_DEV void record_encode(uint64_t lo, uint64_t hi, uint32_t c, uint64_t* rlo, uint64_t* rhi) {
  if (c == 1) {
    *rlo = lo;
    *rhi = hi;
    return;
  }
  uint64_t ml = 0x80, mh = 0;
  for (int i = 0; i < 7; ++i) ml |= (uint64_t)((c >> i) & 1u) << (8 * (i + 1) + 7);
  for (int i = 0; i < 8; ++i) mh |= (uint64_t)((c >> (7 + i)) & 1u) << (8 * i + 7);
  *rlo = lo | ml;
  *rhi = hi | mh;
}

WC_DEV uint32_t record_decode(uint64_t* lo, uint64_t* hi) {
  uint64_t a = *lo, b = *hi;
  *lo = a & ~kTopBits;
  *hi = b & ~kTopBits;
  if (!(a & 0x80)) return 1u;
  uint32_t c = 0;
  for (int i = 0; i < 7; ++i) c |= (uint32_t)((a >> (8 * (i + 1) + 7)) & 1u) << i;
  for (int i = 0; i < 8; ++i) c |= (uint32_t)((b >> (8 * i + 7)) & 1u) << (7 + i);
  return c;
}

WC_DEV uint32_t word_hash32(uint64_t lo, uint64_t hi) {
  uint32_t a = (uint32_t)lo, b = (uint32_t)(lo >> 32), c = (uint32_t)hi, d = (uint32_t)(hi >> 32);
  uint32_t h = a * 0x9E3779B1u ^ (b * 0x85EBCA77u) ^ (c * 0xC2B2AE3Du) ^ (d * 0x27D4EB2Fu);
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 13;
  return h;
}

WC_DEV uint32_t partition_of(uint32_t h) { return h & (kSpillParts - 1); }

// ---------------------------------------------------------------------------------------
// LDS table of short words (lo, hi, count); no deletions while tokens are being counted
// ---------------------------------------------------------------------------------------
struct HotTable {
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
WC_DEV bool hot_add(const HotTable& T, uint64_t lo, uint64_t hi, uint32_t h, uint32_t n,
                    bool may_insert, uint32_t* live) {
  constexpr int kMaxProbe = 24;
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

template <bool kPerDoc>
WC_DEV uint64_t short_key_g(uint64_t lo, uint64_t hi, uint64_t key_mask) {
  return finish_key(fnv_packed(lo, hi, packed_len(lo, hi)), key_mask);
}

// ---------------------------------------------------------------------------------------
// pass 1
// ---------------------------------------------------------------------------------------
// Partition staging in LDS and the block arena in device memory.
struct Spiller {
  uint4* stage;       // [kSpillParts][kStageRec] records
  uint32_t* fill;     // [kSpillParts] records staged
  uint32_t* blk;      // [kSpillParts] current arena block (0xffffffff = none)
  uint32_t* bpos;     // [kSpillParts] records written into the current block
};

// Write `n` staged records of partition p to the arena (one thread). Falls back to direct
// table inserts when the partition's region is exhausted.
WC_DEV void spill_flush(const SpillParams& P, const Spiller& S, uint32_t p, uint32_t n) {
  if (n == 0) return;
  uint32_t b = S.blk[p], pos = S.bpos[p];
  if (b == 0xffffffffu || pos + n > kBlockRec) {
    if (b != 0xffffffffu) P.fill[(uint64_t)p * P.R + b] = (uint16_t)pos;
    b = atomicAdd(&P.cursor[p], 1u);
    pos = 0;
    if (b >= P.R) {
      // region exhausted: count these records in the global table directly
      for (uint32_t j = 0; j < n; ++j) {
        uint4 r = S.stage[p * kStageRec + j];
        uint64_t lo = (uint64_t)r.x | ((uint64_t)r.y << 32), hi = (uint64_t)r.z | ((uint64_t)r.w << 32);
        uint32_t c = record_decode(&lo, &hi);
        table_insert<false>(P.table, P.mask, short_key_g<false>(lo, hi, P.key_mask),
                            short_id(lo, hi, 0), c, P.hdr, P.occ_limit);
      }
      S.blk[p] = 0xffffffffu;
      S.bpos[p] = 0;
      return;
    }
    S.blk[p] = b;
  }
  uint4* dst = P.arena + ((uint64_t)p * P.R + b) * kBlockRec + pos;
  for (uint32_t j = 0; j < n; ++j) dst[j] = S.stage[p * kStageRec + j];
  S.bpos[p] = pos + n;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void spill_count_kernel(SpillParams P) {
  constexpr int STAGE = BLOCK * 16;
  constexpr int NWAVE = BLOCK / 64;
  __shared__ uint4 s_txt4[STAGE / 16 + 2];
  __shared__ uint16_t s_wm[BLOCK];
  __shared__ uint16_t s_last[BLOCK + 1];
  __shared__ uint32_t s_bnd[STAGE / 32 + 2];
  __shared__ uint16_t s_starts[STAGE];
  __shared__ uint32_t s_wsum[NWAVE];
  __shared__ uint4 s_list[kSpillList];            // this stage's spill records
  __shared__ uint8_t s_lpart[kSpillList];
  __shared__ uint32_t s_nlist;
  __shared__ uint32_t s_live;
  __shared__ uint32_t s_thresh;
  __shared__ uint32_t s_carry[2];
  __shared__ uint32_t s_next_w;
  __shared__ uint32_t s_pending;
  extern __shared__ __align__(16) uint8_t s_dyn[];
  const uint8_t* s_txt = (const uint8_t*)s_txt4;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  Header* hdr = P.hdr;
  if (ld_relaxed32(&hdr->flags) & kFlagBadOffsets) return;

  // dynamic LDS: hot table, then partition staging
  const uint32_t E = P.lds_entries;
  HotTable T;
  T.lo = (uint64_t*)s_dyn;
  T.hi = T.lo + E;
  T.cnt = (uint32_t*)(T.hi + E);
  T.size = E;
  Spiller S;
  S.stage = (uint4*)(T.cnt + E);
  S.fill = (uint32_t*)(S.stage + kSpillParts * kStageRec);
  S.blk = S.fill + kSpillParts;
  S.bpos = S.blk + kSpillParts;

  for (uint32_t i = tid; i < E; i += BLOCK) {
    T.lo[i] = 0;
    T.hi[i] = 0;
    T.cnt[i] = 0;
  }
  for (uint32_t p = tid; p < kSpillParts; p += BLOCK) {
    S.fill[p] = 0;
    S.blk[p] = 0xffffffffu;
    S.bpos[p] = 0;
  }
  if (tid == 0) {
    s_live = 0;
    s_thresh = 1;
    s_nlist = 0;
  }

  const uint64_t st0 = (uint64_t)blockIdx.x * P.stages_per_wg;
  const uint64_t st1 = min(st0 + P.stages_per_wg, P.n_stages);
  if (st0 >= st1) return;
  const int64_t R0 = (int64_t)P.offsets[0], R1 = (int64_t)P.offsets[P.n_docs];
  const int64_t len = (int64_t)P.len;
  const uint32_t hot_cap = P.hot_cap;

  auto stage_pos = [&](uint64_t k) -> int64_t { return P.base_off + (int64_t)(k * STAGE); };
  auto load16 = [&](uint64_t k) -> uint4 {
    int64_t p = stage_pos(k) + tid * 16;
    uint4 v;
    if (p >= 0 && p + 16 <= len) {
      v = load_stream16(P.corpus + p);
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
  auto wflag_at = [&](int64_t q) -> uint32_t {
    if (q < R0 || q >= R1 || q < 0 || q >= len) return 0u;
    return is_word_byte(P.corpus[q]) ? 1u : 0u;
  };

  // add a record to this stage's spill list, or count it in the global table when full
  auto spill = [&](uint64_t lo, uint64_t hi, uint32_t h, uint32_t c) {
    uint32_t slot = atomicAdd(&s_nlist, 1u);
    if (slot < kSpillList) {
      uint64_t rlo, rhi;
      record_encode(lo, hi, c, &rlo, &rhi);
      s_list[slot] = make_uint4((uint32_t)rlo, (uint32_t)(rlo >> 32), (uint32_t)rhi,
                                (uint32_t)(rhi >> 32));
      s_lpart[slot] = (uint8_t)partition_of(h);
    } else {
      table_insert<false>(P.table, P.mask, short_key_g<false>(lo, hi, P.key_mask),
                          short_id(lo, hi, 0), c, hdr, P.occ_limit);
    }
  };

  // move this stage's spill list into partition staging, flushing full buffers (all threads)
  auto distribute = [&]() {
    const uint32_t m = min(s_nlist, (uint32_t)kSpillList);
    // each thread owns list entries tid, tid + BLOCK (kSpillList <= 2 * BLOCK)
    uint32_t pend = 0;
    for (int r = 0; r < 2; ++r)
      if (tid + r * BLOCK < (int)m) pend |= 1u << r;
    while (true) {
      for (int r = 0; r < 2; ++r) {
        if (!(pend & (1u << r))) continue;
        uint32_t i = tid + r * BLOCK;
        uint32_t p = s_lpart[i];
        uint32_t old = atomicAdd(&S.fill[p], 1u);
        if (old < kStageRec) {
          S.stage[p * kStageRec + old] = s_list[i];
          pend &= ~(1u << r);
        }
      }
      __syncthreads();
      for (uint32_t p = tid; p < kSpillParts; p += BLOCK) {
        uint32_t f = S.fill[p];
        if (f >= kStageRec) {
          spill_flush(P, S, p, kStageRec);
          S.fill[p] = 0;
        }
      }
      if (!__syncthreads_or(pend != 0)) break;
    }
    if (tid == 0) s_nlist = 0;
    __syncthreads();
  };

  if (tid == 0) s_carry[(st0 & 1) ^ 1] = wflag_at(stage_pos(st0) - 1);
  for (int i = tid; i < STAGE / 32 + 2; i += BLOCK) s_bnd[i] = 0;

  uint4 cur = load16(st0);
  uint4 nx1 = make_uint4(0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u);
  if (st0 + 1 < st1) nx1 = load16(st0 + 1);
  uint64_t tokens = 0;

  for (uint64_t k = st0; k < st1; ++k) {
    const int64_t ls = stage_pos(k);
    const int64_t le = ls + STAGE;
    uint4 nx2 = make_uint4(0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u);
    if (k + 2 < st1) nx2 = load16(k + 2);

    // ---- 1. fold + classify ----------------------------------------------------------
    uint32_t f0, f1, f2, f3;
    uint32_t g0 = fold_classify4(cur.x, &f0), g1 = fold_classify4(cur.y, &f1);
    uint32_t g2 = fold_classify4(cur.z, &f2), g3 = fold_classify4(cur.w, &f3);
    uint32_t w16 = movemask4(f0) | (movemask4(f1) << 4) | (movemask4(f2) << 8) |
                   (movemask4(f3) << 12);
    const int64_t p = ls + tid * 16;
    if (p < R0 || p + 16 > R1) {
      int64_t lo_cut = R0 - p, hi_cut = R1 - p;
      uint32_t m = 0xffffu;
      if (lo_cut > 0) m &= lo_cut >= 16 ? 0u : (0xffffu << lo_cut) & 0xffffu;
      if (hi_cut < 16) m &= hi_cut <= 0 ? 0u : (0xffffu >> (16 - hi_cut));
      w16 &= m;
    }
    s_txt4[tid] = make_uint4(g0, g1, g2, g3);
    s_wm[tid] = (uint16_t)w16;
    if (tid == 0) {
      int64_t q = le;
      uint32_t nw;
      if (k + 1 < st1) nw = (q >= R0 && q < R1 && q < len) ? (is_word_byte(nx1.x & 0xffu) ? 1u : 0u) : 0u;
      else nw = wflag_at(q);
      s_next_w = nw;
    }

    // ---- 2. document starts in [ls, le] ----------------------------------------------
    const uint64_t c0 = P.stage_doc[k];
    const uint64_t c1 = P.stage_doc[k + 1];
    const uint64_t nb = c1 - c0;
    for (uint64_t j = tid; j < nb; j += BLOCK) {
      uint64_t rel = P.offsets[c0 + j] - (uint64_t)ls;
      atomicOr(&s_bnd[rel >> 5], 1u << (rel & 31));
    }
    if (tid == 0 && c1 <= P.n_docs && (int64_t)P.offsets[c1] == le)
      atomicOr(&s_bnd[STAGE >> 5], 1u);
    __syncthreads();

    // ---- 3. start / last masks, compaction ---------------------------------------------
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
    const bool may_insert = s_live < hot_cap;
    __syncthreads();
    for (int i = tid; i < STAGE / 32 + 2; i += BLOCK) s_bnd[i] = 0;

    // ---- 4. tokens -------------------------------------------------------------------
    for (uint32_t t = tid; t < total; t += BLOCK) {
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
      const uint32_t wl = e - s + 1;
      uint64_t lo = 0, hi = 0;
      bool short_word = false;
      if (!crosses && wl <= 16) {
        const uint32_t* tw = (const uint32_t*)s_txt;
        uint32_t di = s >> 2, sh = s & 3;
        uint32_t d0 = tw[di], d1 = tw[di + 1], d2 = tw[di + 2], d3 = tw[di + 3], d4 = tw[di + 4];
        uint32_t k0 = __builtin_amdgcn_alignbyte(d1, d0, sh);
        uint32_t k1 = __builtin_amdgcn_alignbyte(d2, d1, sh);
        uint32_t k2 = __builtin_amdgcn_alignbyte(d3, d2, sh);
        uint32_t k3 = __builtin_amdgcn_alignbyte(d4, d3, sh);
        lo = (uint64_t)k0 | ((uint64_t)k1 << 32);
        hi = (uint64_t)k2 | ((uint64_t)k3 << 32);
        if (wl < 8) { lo &= (1ull << (8 * wl)) - 1; hi = 0; }
        else if (wl == 8) { hi = 0; }
        else if (wl < 16) { hi &= (1ull << (8 * (wl - 8))) - 1; }
        short_word = true;
      } else {
        uint64_t start = (uint64_t)(ls + s);
        uint64_t limit = (uint64_t)R1;
        if (crosses) {
          uint64_t nd = P.offsets[c1 <= P.n_docs ? c1 : P.n_docs];
          if (nd > (uint64_t)le && nd < limit) limit = nd;
        } else {
          limit = start + wl;
        }
        uint64_t h;
        uint64_t n = scan_word(P.corpus, start, limit, &lo, &hi, &h);
        if (n <= 16) {
          short_word = true;
        } else {
          table_insert<false>(P.table, P.mask, finish_key(h, P.key_mask),
                              long_id(P.corpus + start, n, 0), 1, hdr, P.occ_limit);
        }
      }
      if (short_word) {
        uint32_t h32 = word_hash32(lo, hi);
        if (!hot_add(T, lo, hi, h32, 1, may_insert, &s_live)) spill(lo, hi, h32, 1);
      }
    }
    __syncthreads();

    // ---- 5. evict cold words when the LDS table is full ---------------------------------
    if (s_live >= hot_cap) {
      // every entry seen at most s_thresh times leaves as a record; the rest are reinserted
      const uint32_t thr = s_thresh;
      constexpr int PER = 8;  // entries per thread (E <= PER * BLOCK)
      uint64_t klo[PER], khi[PER];
      uint32_t kc[PER];
      uint32_t kept = 0;
      for (int j = 0; j < PER; ++j) {
        uint32_t i = tid * PER + j;
        kc[j] = 0;
        if (i < E && T.cnt[i]) {
          klo[j] = T.lo[i];
          khi[j] = T.hi[i] & ~kTop;
          kc[j] = T.cnt[i];
        }
      }
      __syncthreads();
      for (int j = 0; j < PER; ++j) {
        uint32_t i = tid * PER + j;
        if (i < E) {
          T.lo[i] = 0;
          T.hi[i] = 0;
          T.cnt[i] = 0;
        }
      }
      if (tid == 0) s_live = 0;
      __syncthreads();
      // evicted entries go to the spill list in rounds (it holds kSpillList records)
      for (int j = 0; j < PER; ++j) {
        // survivors go back in; one that finds no slot leaves as records like the rest
        if (kc[j] > thr &&
            hot_add(T, klo[j], khi[j], word_hash32(klo[j], khi[j]), kc[j], true, &s_live)) {
          ++kept;
          kc[j] = 0;
        }
      }
      __syncthreads();
      for (int j = 0; j < PER; ++j) {
        bool have = kc[j] != 0;
        while (__syncthreads_or(have)) {
          if (have) {
            uint32_t c = kc[j];
            uint32_t piece = c > kMaxRecordCount ? kMaxRecordCount : c;
            uint32_t slot = atomicAdd(&s_nlist, 1u);
            if (slot < kSpillList) {
              uint64_t rlo, rhi;
              record_encode(klo[j], khi[j], piece, &rlo, &rhi);
              s_list[slot] = make_uint4((uint32_t)rlo, (uint32_t)(rlo >> 32), (uint32_t)rhi,
                                        (uint32_t)(rhi >> 32));
              s_lpart[slot] = (uint8_t)partition_of(word_hash32(klo[j], khi[j]));
              kc[j] -= piece;
              have = kc[j] != 0;
            }
          }
          __syncthreads();
          if (s_nlist >= kSpillList) distribute();
          else __syncthreads();
        }
      }
      // adapt the threshold: raise it when few entries left, lower it when most did
      const uint32_t live = s_live;
      __syncthreads();
      if (tid == 0) {
        if (live > hot_cap / 2) s_thresh = thr + 1;
        else if (live < hot_cap / 8 && thr > 1) s_thresh = thr - 1;
      }
      __syncthreads();
    }

    // ---- 6. stage the spill list ---------------------------------------------------------
    if (s_nlist) distribute();
    cur = nx1;
    nx1 = nx2;
  }

  // ---- end of range: every LDS entry leaves as records, then staging and blocks close -------
  {
    constexpr int PER = 8;
    for (int j = 0; j < PER; ++j) {
      uint32_t i = tid * PER + j;
      uint32_t c = (i < E) ? T.cnt[i] : 0u;
      uint64_t lo = c ? T.lo[i] : 0, hi = c ? (T.hi[i] & ~kTop) : 0;
      bool have = c != 0;
      while (__syncthreads_or(have)) {
        if (have) {
          uint32_t piece = c > kMaxRecordCount ? kMaxRecordCount : c;
          uint32_t slot = atomicAdd(&s_nlist, 1u);
          if (slot < kSpillList) {
            uint64_t rlo, rhi;
            record_encode(lo, hi, piece, &rlo, &rhi);
            s_list[slot] = make_uint4((uint32_t)rlo, (uint32_t)(rlo >> 32), (uint32_t)rhi,
                                      (uint32_t)(rhi >> 32));
            s_lpart[slot] = (uint8_t)partition_of(word_hash32(lo, hi));
            c -= piece;
            have = c != 0;
          }
        }
        __syncthreads();
        if (s_nlist >= kSpillList) distribute();
        else __syncthreads();
      }
    }
    if (s_nlist) distribute();
    for (uint32_t p = tid; p < kSpillParts; p += BLOCK) {
      spill_flush(P, S, p, S.fill[p]);
      S.fill[p] = 0;
      if (S.blk[p] != 0xffffffffu) P.fill[(uint64_t)p * P.R + S.blk[p]] = (uint16_t)S.bpos[p];
    }
  }
  if (tid == 0) add64(&hdr->total_tokens, tokens);
}

// ---------------------------------------------------------------------------------------
// pass 2: one workgroup per partition
// ---------------------------------------------------------------------------------------
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void spill_reduce_kernel(SpillParams P) {
  extern __shared__ __align__(16) uint8_t s_dyn[];
  __shared__ uint32_t s_live;
  const uint32_t p = blockIdx.x;
  const int tid = threadIdx.x;
  Header* hdr = P.hdr;
  if (ld_relaxed32(&hdr->flags) & kFlagBadOffsets) return;
  const uint32_t E = P.reduce_entries;
  HotTable T;
  T.lo = (uint64_t*)s_dyn;
  T.hi = T.lo + E;
  T.cnt = (uint32_t*)(T.hi + E);
  T.size = E;
  for (uint32_t i = tid; i < E; i += BLOCK) {
    T.lo[i] = 0;
    T.hi[i] = 0;
    T.cnt[i] = 0;
  }
  if (tid == 0) s_live = 0;
  __syncthreads();
  const uint32_t nblk = min(P.cursor[p], P.R);
  const uint4* region = P.arena + (uint64_t)p * P.R * kBlockRec;
  const uint16_t* fills = P.fill + (uint64_t)p * P.R;
  const uint32_t cap = E - E / 4;
  constexpr uint32_t kPerIter = BLOCK / kBlockRec;  // blocks per iteration
  auto fetch = [&](uint32_t b0, bool* valid) -> uint4 {
    const uint32_t b = b0 + tid / kBlockRec, r = tid % kBlockRec;
    *valid = b < nblk && r < fills[b];
    return *valid ? region[(uint64_t)b * kBlockRec + r] : make_uint4(0, 0, 0, 0);
  };
  bool v_ok, n_ok, n2_ok;
  uint4 v = fetch(0, &v_ok);
  uint4 nv = fetch(kPerIter, &n_ok);
  for (uint32_t b0 = 0; b0 < nblk; b0 += kPerIter) {
    uint4 nv2 = fetch(b0 + 2 * kPerIter, &n2_ok);
    if (v_ok) {
      uint64_t lo = (uint64_t)v.x | ((uint64_t)v.y << 32), hi = (uint64_t)v.z | ((uint64_t)v.w << 32);
      uint32_t c = record_decode(&lo, &hi);
      // the table word is a count of at most 2^31: larger sums go to the global table
      bool ok = hot_add(T, lo, hi, word_hash32(lo, hi) * 0x9E3779B1u, c,
                        s_live < cap, &s_live);
      if (!ok)
        table_insert<false>(P.table, P.mask, short_key_g<false>(lo, hi, P.key_mask),
                            short_id(lo, hi, 0), c, hdr, P.occ_limit);
    }
    v = nv;
    v_ok = n_ok;
    nv = nv2;
    n_ok = n2_ok;
  }
  __syncthreads();
  for (uint32_t i = tid; i < E; i += BLOCK) {
    uint32_t c = T.cnt[i];
    if (c) {
      uint64_t lo = T.lo[i], hi = T.hi[i] & ~kTop;
      table_insert<false>(P.table, P.mask, short_key_g<false>(lo, hi, P.key_mask),
                          short_id(lo, hi, 0), c, hdr, P.occ_limit);
    }
  }
}

hipError_t set_spill_smem(size_t count_dyn, size_t reduce_dyn) {
  hipError_t e = hipFuncSetAttribute((const void*)spill_count_kernel<512>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)count_dyn);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)spill_reduce_kernel<512>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)reduce_dyn);
  return e;
}

hipError_t launch_spill_count(const SpillParams& P, uint32_t grid, size_t dyn, hipStream_t s) {
  hipLaunchKernelGGL(spill_count_kernel<512>, dim3(grid), dim3(512), dyn, s, P);
  return hipGetLastError();
}

hipError_t launch_spill_reduce(const SpillParams& P, size_t dyn, hipStream_t s) {
  hipLaunchKernelGGL(spill_reduce_kernel<512>, dim3(kSpillParts), dim3(512), dyn, s, P);
  return hipGetLastError();
}

}  // namespace wc
