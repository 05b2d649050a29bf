// The paper's own reduce (Section 3.3, timed in the Section 4.1 table): the per-document
// counts are laid out as a zero-padded matrix with one row per distinct word (key) and one
// column per document, and a kernel sums each row. Here the whole of it runs on the GPU:
//   1. keys: every (document, word) entry's word is inserted into a hash table without a
//      count, which gives each distinct word a slot; the table is compacted (export), so the
//      distinct words get dense row numbers and their bytes are written once;
//   2. the matrix (rows x documents, uint32, zero-filled) receives each entry's count at
//      (row of its word, its document);
//   3. the row-sum kernel adds each row and writes the word's total.
// The result is the same table wc_merge gives (a pointwise sum over documents); the point is
// the comparison with the hash merge, which never materialises the zeros.
#include "wc_internal.h"

namespace wc {

namespace {

// Insert the word of each entry (count 0) and note its slot.
__global__ void dense_key_kernel(MergeInput in, Slot* table, uint64_t mask, uint64_t occ_limit,
                                 uint64_t key_mask, Header* hdr, uint64_t* slot_of_input) {
  const uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (e >= in.n) return;
  const uint64_t a = in.word_offsets[e], len = in.word_offsets[e + 1] - a;
  const uint8_t* w = in.words + a;
  uint64_t h = kFnvOffset, lo = 0, hi = 0;
  for (uint64_t q = 0; q < len; ++q) {
    const uint32_t f = fold_byte(w[q]);
    h = fnv_step(h, f);
    if (q < 8) lo |= (uint64_t)f << (8 * q);
    else if (q < 16) hi |= (uint64_t)f << (8 * (q - 8));
  }
  const WordId id = len <= 16 && packable(lo, hi) ? short_id(lo, hi, 0) : long_id(w, len, 0);
  slot_of_input[e] = table_insert<false>(table, mask, finish_key(h, key_mask), id, 0, hdr,
                                         occ_limit);
}

// matrix[row(word of e) * n_docs + doc(e)] = count(e)
__global__ void dense_scatter_kernel(uint64_t n, const uint64_t* slot_of_input,
                                     const uint64_t* entry_of_slot, const uint64_t* docs,
                                     const void* counts, uint32_t count_bytes, uint64_t n_docs,
                                     uint32_t* matrix) {
  const uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const uint64_t slot = slot_of_input[e];
  if (slot == ~0ull) return;  // the table filled: the call fails as full
  const uint64_t c = count_bytes == 4 ? (uint64_t)((const int32_t*)counts)[e]
                                      : (uint64_t)((const int64_t*)counts)[e];
  matrix[entry_of_slot[slot] * n_docs + docs[e]] = (uint32_t)c;
}

// counts[r] = sum of row r; one wave per row (n_docs >= 64), else one thread per row.
__global__ __launch_bounds__(256) void dense_rowsum_kernel(const uint32_t* matrix, uint64_t rows,
                                                           uint64_t n_docs, void* counts,
                                                           uint32_t count_bytes, uint64_t bias,
                                                           Header* hdr) {
  auto put = [&](uint64_t r, uint64_t s) {
    s += bias;
    if (count_bytes == 4) {
      if (s > 0x7fffffffull) or32(&hdr->flags, kFlagCountOverflow);
      ((int32_t*)counts)[r] = (int32_t)s;
    } else {
      ((int64_t*)counts)[r] = (int64_t)s;
    }
  };
  if (n_docs >= 64) {
    const uint64_t lane = threadIdx.x & 63;
    const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t r = wave; r < rows; r += n_waves) {
      const uint32_t* row = matrix + r * n_docs;
      uint64_t s = 0;
      for (uint64_t d = lane; d < n_docs; d += 64) s += row[d];
      for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
      if (lane == 0) put(r, s);
    }
  } else {
    for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < rows;
         r += (uint64_t)gridDim.x * blockDim.x) {
      const uint32_t* row = matrix + r * n_docs;
      uint64_t s = 0;
      for (uint64_t d = 0; d < n_docs; ++d) s += row[d];
      put(r, s);
    }
  }
}

}  // namespace

hipError_t launch_dense_keys(const MergeInput& in, Slot* table, uint64_t mask,
                             uint64_t occ_limit, uint64_t key_mask, Header* hdr,
                             uint64_t* slot_of_input, hipStream_t s) {
  if (in.n == 0) return hipSuccess;
  hipLaunchKernelGGL(dense_key_kernel, dim3((uint32_t)((in.n + 255) / 256)), dim3(256), 0, s, in,
                     table, mask, occ_limit, key_mask, hdr, slot_of_input);
  return hipGetLastError();
}

hipError_t launch_dense_scatter(uint64_t n, const uint64_t* slot_of_input,
                                const uint64_t* entry_of_slot, const uint64_t* docs,
                                const void* counts, uint32_t count_bytes, uint64_t n_docs,
                                uint32_t* matrix, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(dense_scatter_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, n,
                     slot_of_input, entry_of_slot, docs, counts, count_bytes, n_docs, matrix);
  return hipGetLastError();
}

hipError_t launch_dense_rowsum(const uint32_t* matrix, uint64_t rows, uint64_t n_docs,
                               void* counts, uint32_t count_bytes, uint64_t bias, Header* hdr,
                               hipStream_t s) {
  if (rows == 0) return hipSuccess;
  const uint64_t per_block = n_docs >= 64 ? 4 : 256;  // rows a 256-thread block takes at once
  uint64_t blocks = (rows + per_block - 1) / per_block;
  blocks = blocks < 1 ? 1 : (blocks > 65536 ? 65536 : blocks);
  hipLaunchKernelGGL(dense_rowsum_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, matrix, rows,
                     n_docs, counts, count_bytes, bias, hdr);
  return hipGetLastError();
}

}  // namespace wc
