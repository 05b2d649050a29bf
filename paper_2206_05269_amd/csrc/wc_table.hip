// Table kernels: compaction of a hash table into dense arrays, per-document CSR grouping,
// merging word tables (Section 3.3: grouped counts of one word are summed), the per-corpus
// distinctive-word ranking (Section 4.3) and the FNV-1a 64 check entry point.

#include "wc_internal.h"

namespace wc {

// ------------------------------------------------------------------------------------------
// fill
// ------------------------------------------------------------------------------------------
__global__ void fill_zero_kernel(uint4* p, uint64_t n16, uint8_t* tail, uint32_t n_tail) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x < n_tail) tail[threadIdx.x] = 0;
}

hipError_t launch_fill_zero(void* p, uint64_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  // p is 16-byte aligned by construction (workspace regions are 256-byte aligned)
  uint64_t n16 = bytes / 16;
  uint32_t n_tail = (uint32_t)(bytes % 16);
  uint64_t blocks = (n16 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, (uint4*)p, n16,
                     (uint8_t*)p + n16 * 16, n_tail);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// export
// ------------------------------------------------------------------------------------------
WC_DEV uint64_t slot_len(const Slot& sl) {
  if (sl.w0 & kTop) return sl.w1 & ~kTop;
  return packed_len(sl.w0, sl.w1 & ~kTop);
}

template <int BLOCK>
WC_DEV uint64_t block_excl_scan(uint64_t v, uint64_t* s_tmp, uint64_t* total) {
  // s_tmp: BLOCK/64 entries
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t incl = v;
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) s_tmp[wave] = incl;
  __syncthreads();
  uint64_t base = 0, tot = 0;
  for (int w = 0; w < BLOCK / 64; ++w) {
    uint64_t x = s_tmp[w];
    base += w < wave ? x : 0;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

__global__ __launch_bounds__(kExportBlock) void export_count_kernel(ExportParams E) {
  __shared__ uint64_t s_a[kExportBlock / 64], s_b[kExportBlock / 64];
  const uint64_t b = blockIdx.x;
  // only the block's totals are needed here, so slots are read wave-contiguously (consecutive
  // lanes, consecutive slots) rather than in the write kernel's per-thread runs
  const uint64_t first = b * kExportSpan + threadIdx.x;
  uint64_t n = 0, bytes = 0;
  for (uint32_t j = 0; j < kExportItems; ++j) {
    uint64_t i = first + (uint64_t)j * kExportBlock;
    if (i < E.slots) {
      Slot sl = E.table[i];
      if (sl.key) {
        ++n;
        bytes += slot_len(sl);
      }
    }
  }
  uint64_t tn, tb;
  block_excl_scan<kExportBlock>(n, s_a, &tn);
  block_excl_scan<kExportBlock>(bytes, s_b, &tb);
  if (threadIdx.x == 0) {
    E.block_sums[2 * b] = tn;
    E.block_sums[2 * b + 1] = tb;
  }
}

__global__ __launch_bounds__(1024) void export_scan_kernel(ExportParams E) {
  __shared__ uint64_t s_a[16], s_b[16];
  __shared__ uint64_t s_carry[2];
  if (threadIdx.x == 0) s_carry[0] = s_carry[1] = 0;
  __syncthreads();
  for (uint64_t base = 0; base < E.n_blocks; base += 1024) {
    uint64_t i = base + threadIdx.x;
    uint64_t a = i < E.n_blocks ? E.block_sums[2 * i] : 0;
    uint64_t b = i < E.n_blocks ? E.block_sums[2 * i + 1] : 0;
    uint64_t ta, tb;
    uint64_t ea = block_excl_scan<1024>(a, s_a, &ta);
    uint64_t eb = block_excl_scan<1024>(b, s_b, &tb);
    if (i < E.n_blocks) {
      E.block_sums[2 * i] = ea + s_carry[0];
      E.block_sums[2 * i + 1] = eb + s_carry[1];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_carry[0] += ta;
      s_carry[1] += tb;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    E.hdr->n_entries = s_carry[0];
    E.hdr->word_bytes = s_carry[1];
    if (E.word_offsets) E.word_offsets[s_carry[0]] = s_carry[1];
    if (s_carry[1] > E.word_cap) E.hdr->flags |= kFlagWordCap;
  }
}

__global__ __launch_bounds__(kExportBlock) void export_write_kernel(ExportParams E) {
  __shared__ uint64_t s_a[kExportBlock / 64], s_b[kExportBlock / 64];
  const uint64_t b = blockIdx.x;
  const uint64_t first = b * kExportSpan + (uint64_t)threadIdx.x * kExportItems;
  Slot sl[kExportItems];
  uint64_t n = 0, bytes = 0;
  for (uint32_t j = 0; j < kExportItems; ++j) {
    uint64_t i = first + j;
    sl[j].key = 0;
    if (i < E.slots) {
      sl[j] = E.table[i];
      if (sl[j].key) {
        ++n;
        bytes += slot_len(sl[j]);
      }
    }
  }
  uint64_t tn, tb;
  uint64_t e = block_excl_scan<kExportBlock>(n, s_a, &tn) + E.block_sums[2 * b];
  uint64_t pos = block_excl_scan<kExportBlock>(bytes, s_b, &tb) + E.block_sums[2 * b + 1];
  const bool write_words = (E.hdr->flags & kFlagWordCap) == 0;
  for (uint32_t j = 0; j < kExportItems; ++j) {
    if (!sl[j].key) continue;
    const uint64_t i = first + j;
    uint64_t len = slot_len(sl[j]);
    uint64_t c = (E.per_doc ? (sl[j].cnt & 0xffffffffull) : sl[j].cnt) + E.count_bias;
    E.word_offsets[e] = pos;
    if (E.count_bytes == 4) {
      if (c > 0x7fffffffull) or32(&E.hdr->flags, kFlagCountOverflow);
      ((int32_t*)E.counts)[e] = (int32_t)c;
    } else {
      ((int64_t*)E.counts)[e] = (int64_t)c;
    }
    if (E.per_doc) E.docs[e] = (sl[j].cnt >> 32) - 1;
    if (E.slot_of_entry) E.slot_of_entry[e] = i;
    if (E.entry_of_slot) E.entry_of_slot[i] = e;
    if (write_words) {
      if (sl[j].w0 & kTop) {
        const uint8_t* src = (const uint8_t*)(uintptr_t)(sl[j].w0 & ~kTop);
        for (uint64_t q = 0; q < len; ++q) E.words[pos + q] = (uint8_t)fold_byte(src[q]);
      } else {
        uint64_t lo = sl[j].w0, hi = sl[j].w1 & ~kTop;
        for (uint64_t q = 0; q < len; ++q)
          E.words[pos + q] = (uint8_t)((q < 8 ? lo >> (8 * q) : hi >> (8 * (q - 8))) & 0xff);
      }
    }
    ++e;
    pos += len;
  }
}

// Dense list of the occupied slots with their documents (per-document export, first step).
__global__ __launch_bounds__(kExportBlock) void export_list_kernel(ExportParams E) {
  __shared__ uint64_t s_a[kExportBlock / 64];
  const uint64_t b = blockIdx.x;
  const uint64_t first = b * kExportSpan + (uint64_t)threadIdx.x * kExportItems;
  uint64_t keys[kExportItems], cnts[kExportItems];
  uint64_t n = 0;
  for (uint32_t j = 0; j < kExportItems; ++j) {
    uint64_t i = first + j;
    keys[j] = 0;
    if (i < E.slots) {
      keys[j] = E.table[i].key;
      cnts[j] = E.table[i].cnt;
      n += keys[j] != 0;
    }
  }
  uint64_t tn;
  uint64_t e = block_excl_scan<kExportBlock>(n, s_a, &tn) + E.block_sums[2 * b];
  for (uint32_t j = 0; j < kExportItems; ++j) {
    if (!keys[j]) continue;
    E.docs[e] = (cnts[j] >> 32) - 1;
    E.slot_of_entry[e] = first + j;
    ++e;
  }
}

hipError_t launch_export_list(const ExportParams& E, hipStream_t s) {
  uint32_t nb = (uint32_t)E.n_blocks;
  hipLaunchKernelGGL(export_count_kernel, dim3(nb), dim3(kExportBlock), 0, s, E);
  hipLaunchKernelGGL(export_scan_kernel, dim3(1), dim3(1024), 0, s, E);
  hipLaunchKernelGGL(export_list_kernel, dim3(nb), dim3(kExportBlock), 0, s, E);
  return hipGetLastError();
}

// Lengths of the words of slots listed in entry order (lens[n] = 0 closes the scan).
__global__ void slot_lens_kernel(const Slot* table, const uint64_t* slots, uint64_t n,
                                 uint64_t* lens) {
  uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (e > n) return;
  lens[e] = e < n ? slot_len(table[slots[e]]) : 0;
}

// Write entry e from slot slots[e]: count, document, word bytes at word_offsets[e].
__global__ void slot_write_kernel(const Slot* table, const uint64_t* slots, uint64_t n,
                                  const uint64_t* word_offsets, uint8_t* words, void* counts,
                                  uint32_t count_bytes, uint64_t count_bias, uint64_t* docs,
                                  Header* hdr) {
  uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  Slot sl = table[slots[e]];
  uint64_t c = (sl.cnt & 0xffffffffull) + count_bias;
  if (count_bytes == 4) {
    if (c > 0x7fffffffull) or32(&hdr->flags, kFlagCountOverflow);
    ((int32_t*)counts)[e] = (int32_t)c;
  } else {
    ((int64_t*)counts)[e] = (int64_t)c;
  }
  docs[e] = (sl.cnt >> 32) - 1;
  uint64_t pos = word_offsets[e], len = word_offsets[e + 1] - pos;
  if (sl.w0 & kTop) {
    const uint8_t* src = (const uint8_t*)(uintptr_t)(sl.w0 & ~kTop);
    for (uint64_t q = 0; q < len; ++q) words[pos + q] = (uint8_t)fold_byte(src[q]);
  } else {
    uint64_t lo = sl.w0, hi = sl.w1 & ~kTop;
    for (uint64_t q = 0; q < len; ++q)
      words[pos + q] = (uint8_t)((q < 8 ? lo >> (8 * q) : hi >> (8 * (q - 8))) & 0xff);
  }
}

hipError_t launch_slot_lens(const Slot* table, const uint64_t* slots, uint64_t n, uint64_t* lens,
                            hipStream_t s) {
  hipLaunchKernelGGL(slot_lens_kernel, dim3((uint32_t)((n + 1 + 255) / 256)), dim3(256), 0, s,
                     table, slots, n, lens);
  return hipGetLastError();
}

hipError_t launch_slot_write(const Slot* table, const uint64_t* slots, uint64_t n,
                             const uint64_t* word_offsets, uint8_t* words, void* counts,
                             uint32_t count_bytes, uint64_t count_bias, uint64_t* docs,
                             Header* hdr, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(slot_write_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s,
                     table, slots, n, word_offsets, words, counts, count_bytes, count_bias, docs,
                     hdr);
  return hipGetLastError();
}

hipError_t launch_export(const ExportParams& E, hipStream_t s) {
  uint32_t nb = (uint32_t)E.n_blocks;
  hipLaunchKernelGGL(export_count_kernel, dim3(nb), dim3(kExportBlock), 0, s, E);
  hipLaunchKernelGGL(export_scan_kernel, dim3(1), dim3(1024), 0, s, E);
  hipLaunchKernelGGL(export_write_kernel, dim3(nb), dim3(kExportBlock), 0, s, E);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// merge: insert the entries of one table
// ------------------------------------------------------------------------------------------
__global__ void merge_insert_kernel(MergeInput in, Slot* table, uint64_t mask,
                                    uint64_t occ_limit, uint64_t key_mask, Header* hdr,
                                    uint64_t* joint, uint32_t C) {
  uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (e >= in.n) return;
  uint64_t a = in.word_offsets[e], b = in.word_offsets[e + 1];
  uint64_t len = b - a;
  uint64_t c = in.count_bytes == 4 ? (uint64_t)(int64_t)((const int32_t*)in.counts)[e]
                                   : (uint64_t)((const int64_t*)in.counts)[e];
  if (len == 0 || c == 0) return;
  const uint8_t* w = in.words + a;
  uint64_t h = kFnvOffset, lo = 0, hi = 0;
  for (uint64_t q = 0; q < len; ++q) {
    uint32_t f = fold_byte(w[q]);
    h = fnv_step(h, f);
    if (q < 8) lo |= (uint64_t)f << (8 * q);
    else if (q < 16) hi |= (uint64_t)f << (8 * (q - 8));
  }
  uint64_t key = finish_key(h, key_mask);
  WordId id = len <= 16 && packable(lo, hi) ? short_id(lo, hi, 0) : long_id(w, len, 0);
  uint64_t slot = table_insert<false>(table, mask, key, id, c, hdr, occ_limit);
  if (joint && slot != ~0ull) add64(&joint[slot * C + in.column], c);
}

hipError_t launch_merge_insert(const MergeInput& in, Slot* table, uint64_t mask,
                               uint64_t occ_limit, uint64_t key_mask, Header* hdr,
                               uint64_t* joint_counts, uint32_t n_columns, hipStream_t s) {
  if (in.n == 0) return hipSuccess;
  uint32_t grid = (uint32_t)((in.n + 255) / 256);
  hipLaunchKernelGGL(merge_insert_kernel, dim3(grid), dim3(256), 0, s, in, table, mask,
                     occ_limit, key_mask, hdr, joint_counts, n_columns);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// FNV-1a 64 of strings (checked against published test vectors)
// ------------------------------------------------------------------------------------------
__global__ void hash_words_kernel(const uint8_t* bytes, const uint64_t* off, uint64_t n,
                                  uint64_t* out) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t h = kFnvOffset;
  for (uint64_t q = off[i]; q < off[i + 1]; ++q) h = fnv_step(h, fold_byte(bytes[q]));
  uint64_t lo = 0, hi = 0, len = off[i + 1] - off[i];
  if (len <= 16) {
    for (uint64_t q = 0; q < len; ++q) {
      uint64_t f = fold_byte(bytes[off[i] + q]);
      if (q < 8) lo |= f << (8 * q); else hi |= f << (8 * (q - 8));
    }
    // the packed path the counter takes must agree with the byte path
    if (fnv_packed(lo, hi, packed_len(lo, hi)) != h) h = 0;  // reported as 1: a mismatch shows
  }
  out[i] = finish_key(h, ~0ull);
}

hipError_t launch_hash_words(const uint8_t* bytes, const uint64_t* offsets, uint64_t n,
                             uint64_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(hash_words_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s,
                     bytes, offsets, n, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// top-k distinctive words
// ------------------------------------------------------------------------------------------
__global__ void column_totals_kernel(const uint64_t* joint, uint64_t V, uint32_t C,
                                     uint64_t* totals) {
  __shared__ uint64_t s_t[64];
  if (threadIdx.x < 64) s_t[threadIdx.x] = 0;
  __syncthreads();
  uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (e < V)
    for (uint32_t c = 0; c < C; ++c) atomicAdd((unsigned long long*)&s_t[c], (unsigned long long)joint[e * C + c]);
  __syncthreads();
  if (threadIdx.x < C && s_t[threadIdx.x]) add64(&totals[threadIdx.x], s_t[threadIdx.x]);
}

struct Ranker {
  const uint64_t* word_offsets;
  const uint8_t* words;
  const uint64_t* joint;
  const uint64_t* total;  // per entry: sum over corpora
  uint32_t C, c;

  WC_DEV uint64_t nc(uint32_t e) const { return joint[(uint64_t)e * C + c]; }
  WC_DEV uint64_t nr(uint32_t e) const { return total[e] - nc(e); }
  // true when entry a ranks before entry b
  WC_DEV bool better(uint32_t a, uint32_t b) const {
    uint64_t na = nc(a), nb = nc(b), ra = total[a] - na, rb = total[b] - nb;
    uint64_t x = na + 1, y = rb + 1, u = nb + 1, v = ra + 1;
    uint64_t lh = __umul64hi(x, y), ll = x * y, rh = __umul64hi(u, v), rl = u * v;
    if (lh != rh) return lh > rh;
    if (ll != rl) return ll > rl;
    if (na != nb) return na > nb;
    uint64_t pa = word_offsets[a], la = word_offsets[a + 1] - pa;
    uint64_t pb = word_offsets[b], lb = word_offsets[b + 1] - pb;
    uint64_t m = la < lb ? la : lb;
    for (uint64_t q = 0; q < m; ++q) {
      uint8_t ca = words[pa + q], cb = words[pb + q];
      if (ca != cb) return ca < cb;
    }
    return la < lb;
  }
};

// One workgroup per corpus: per-thread sorted lists of the best k, then a merge tree.
__global__ __launch_bounds__(kTopkThreads) void topk_kernel(TopkParams P, const uint64_t* total) {
  const uint32_t c = blockIdx.x;
  const uint32_t t = threadIdx.x;
  const uint32_t T = kTopkThreads;
  const uint32_t k = P.k;
  Ranker R{P.word_offsets, P.words, P.joint, total, P.C, c};
  uint32_t* buf[2] = {P.lists + ((uint64_t)c * 2 + 0) * T * k, P.lists + ((uint64_t)c * 2 + 1) * T * k};
  uint32_t* lens[2] = {P.list_len + ((uint64_t)c * 2 + 0) * T, P.list_len + ((uint64_t)c * 2 + 1) * T};
  const uint64_t minc = P.min_count > 0 ? P.min_count : 1;
  // phase 1: thread-local top-k
  uint32_t* my = buf[0] + (uint64_t)t * k;
  uint32_t n = 0;
  for (uint64_t e = t; e < P.V; e += T) {
    if (R.nc((uint32_t)e) < minc) continue;
    uint32_t ee = (uint32_t)e;
    if (n == k && !R.better(ee, my[k - 1])) continue;
    uint32_t pos = n < k ? n : k - 1;
    while (pos > 0 && R.better(ee, my[pos - 1])) {
      my[pos] = my[pos - 1];
      --pos;
    }
    my[pos] = ee;
    if (n < k) ++n;
  }
  lens[0][t] = n;
  __syncthreads();
  // phase 2: merge tree
  int src = 0;
  for (uint32_t step = 1; step < T; step <<= 1) {
    int dst = src ^ 1;
    if ((t % (2 * step)) == 0) {
      const uint32_t* a = buf[src] + (uint64_t)t * k;
      const uint32_t* b = buf[src] + (uint64_t)(t + step) * k;
      uint32_t na = lens[src][t], nb = lens[src][t + step];
      uint32_t* o = buf[dst] + (uint64_t)t * k;
      uint32_t i = 0, j = 0, m = 0;
      while (m < k && (i < na || j < nb)) {
        bool take_a = j >= nb || (i < na && R.better(a[i], b[j]));
        o[m++] = take_a ? a[i++] : b[j++];
      }
      lens[dst][t] = m;
    }
    __syncthreads();
    src = dst;
  }
  // phase 3: rows
  const uint32_t rows = lens[src][0];
  const uint32_t* best = buf[src];
  const double Nc = (double)P.totals[c];
  uint64_t all = 0;
  for (uint32_t q = 0; q < P.C; ++q) all += P.totals[q];
  const double Nr = (double)(all - P.totals[c]);
  const double Vd = (double)P.V;
  for (uint32_t r = t; r < rows; r += T) {
    uint32_t e = best[r];
    uint64_t nc = R.nc(e), nr = R.nr(e);
    uint64_t row = (uint64_t)c * k + r;
    P.out_entry[row] = e;
    P.out_nc[row] = nc;
    P.out_nr[row] = nr;
    P.out_score[row] = (((double)nc + 1.0) / (Nc + Vd)) / (((double)nr + 1.0) / (Nr + Vd));
  }
  if (t == 0) P.n_rows[c] = rows;
}

// Row word offsets (one workgroup) and row word bytes.
__global__ __launch_bounds__(1024) void topk_rows_kernel(TopkParams P) {
  __shared__ uint64_t s_tmp[16];
  __shared__ uint64_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  const uint64_t total_rows = (uint64_t)P.C * P.k;
  for (uint64_t base = 0; base < total_rows; base += 1024) {
    uint64_t r = base + threadIdx.x;
    uint64_t len = 0;
    if (r < total_rows) {
      uint32_t c = (uint32_t)(r / P.k), j = (uint32_t)(r % P.k);
      if (j < P.n_rows[c]) {
        uint64_t e = P.out_entry[r];
        len = P.word_offsets[e + 1] - P.word_offsets[e];
      }
    }
    uint64_t tot;
    uint64_t ex = block_excl_scan<1024>(len, s_tmp, &tot);
    uint64_t pos = ex + s_carry;
    if (r < total_rows) {
      P.out_word_offsets[r] = pos;
      if (len) {
        uint64_t e = P.out_entry[r];
        const uint8_t* src = P.words + P.word_offsets[e];
        for (uint64_t q = 0; q < len; ++q) P.out_words[pos + q] = src[q];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) s_carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) P.out_word_offsets[total_rows] = s_carry;
}

hipError_t launch_topk(const TopkParams& P, hipStream_t s) {
  // P.totals must be zeroed by the caller; per-entry totals are in P.totals + C
  uint32_t grid = (uint32_t)((P.V + 255) / 256);
  if (grid) hipLaunchKernelGGL(column_totals_kernel, dim3(grid), dim3(256), 0, s, P.joint, P.V, P.C, P.totals);
  hipLaunchKernelGGL(topk_kernel, dim3(P.C), dim3(kTopkThreads), 0, s, P, P.entry_total);
  hipLaunchKernelGGL(topk_rows_kernel, dim3(1), dim3(1024), 0, s, P);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// ------------------------------------------------------------------------------------------
// exclusive prefix sum of uint64 values: per-block scans, a scan of the block totals, and
// the block offsets added back
// ------------------------------------------------------------------------------------------
constexpr uint32_t kScanBlock = 256, kScanItems = 4, kScanSpan = kScanBlock * kScanItems;

uint64_t excl_scan_scratch(uint64_t n) { return ((n + kScanSpan - 1) / kScanSpan + 1) * 8; }

// out[i] = sum of in[b*span .. i) for the block b holding i; sums[b] = the block's total
__global__ __launch_bounds__(kScanBlock) void scan_local_kernel(const uint64_t* in, uint64_t* out,
                                                                uint64_t n, uint64_t* sums) {
  __shared__ uint64_t s_tmp[kScanBlock / 64];
  const uint64_t first = blockIdx.x * (uint64_t)kScanSpan + (uint64_t)threadIdx.x * kScanItems;
  uint64_t v[kScanItems], t = 0;
  for (uint32_t j = 0; j < kScanItems; ++j) {
    v[j] = first + j < n ? in[first + j] : 0;
    t += v[j];
  }
  uint64_t tot;
  uint64_t e = block_excl_scan<kScanBlock>(t, s_tmp, &tot);
  for (uint32_t j = 0; j < kScanItems; ++j) {
    if (first + j < n) out[first + j] = e;
    e += v[j];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// sums[0 .. nb) becomes its exclusive scan (one workgroup)
__global__ __launch_bounds__(1024) void scan_sums_kernel(uint64_t* sums, uint64_t nb) {
  __shared__ uint64_t s_tmp[16];
  __shared__ uint64_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (uint64_t base = 0; base < nb; base += 1024) {
    const uint64_t i = base + threadIdx.x;
    const uint64_t v = i < nb ? sums[i] : 0;
    uint64_t tot;
    const uint64_t e = block_excl_scan<1024>(v, s_tmp, &tot);
    if (i < nb) sums[i] = e + s_carry;
    __syncthreads();
    if (threadIdx.x == 0) s_carry += tot;
    __syncthreads();
  }
}

__global__ void scan_add_kernel(uint64_t* out, uint64_t n, const uint64_t* sums) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] += sums[i / kScanSpan];
}

hipError_t excl_scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* sums,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t nb = (n + kScanSpan - 1) / kScanSpan;
  hipLaunchKernelGGL(scan_local_kernel, dim3((uint32_t)nb), dim3(kScanBlock), 0, s, in, out, n,
                     sums);
  if (nb > 1) {
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, s, sums, nb);
    hipLaunchKernelGGL(scan_add_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, out,
                       n, sums);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// entries grouped by document: a counting sort (histogram, scan, scatter); the order inside a
// document is unspecified, as the result's entry order is
// ------------------------------------------------------------------------------------------
__global__ void doc_hist_kernel(const uint64_t* docs, uint64_t n, uint64_t* doc_len) {
  const uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (e < n) atomicAdd((unsigned long long*)&doc_len[docs[e]], 1ull);
}

__global__ void doc_scatter_kernel(const uint64_t* docs, const uint64_t* slots, uint64_t n,
                                   const uint64_t* doc_ptr, uint64_t* fill,
                                   uint64_t* sorted_docs, uint64_t* sorted_slots) {
  const uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const uint64_t d = docs[e];
  const uint64_t at = doc_ptr[d] + atomicAdd((unsigned long long*)&fill[d], 1ull);
  sorted_docs[at] = d;
  sorted_slots[at] = slots[e];
}

hipError_t group_by_doc(const uint64_t* docs, const uint64_t* slots, uint64_t n, uint64_t n_docs,
                        uint64_t* doc_ptr, uint64_t* doc_len, uint64_t* fill, uint64_t* sums,
                        uint64_t* sorted_docs, uint64_t* sorted_slots, hipStream_t s) {
  hipError_t e = launch_fill_zero(doc_len, n_docs * 8, s);
  if (e == hipSuccess) e = launch_fill_zero(fill, n_docs * 8, s);
  if (e != hipSuccess || n_docs == 0) return e;
  const uint32_t grid = (uint32_t)((n + 255) / 256);
  if (n) hipLaunchKernelGGL(doc_hist_kernel, dim3(grid), dim3(256), 0, s, docs, n, doc_len);
  e = excl_scan_u64(doc_len, doc_ptr, n_docs, sums, s);
  if (e == hipSuccess && n)
    hipLaunchKernelGGL(doc_scatter_kernel, dim3(grid), dim3(256), 0, s, docs, slots, n, doc_ptr,
                       fill, sorted_docs, sorted_slots);
  return e == hipSuccess ? hipGetLastError() : e;
}

}  // namespace wc
