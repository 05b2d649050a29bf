// Internal interfaces between the host API (wc_api.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wc.h"
#include "wc_device.h"

namespace wc {

struct CountParams {
  const uint8_t* corpus;     // logical byte 0
  uint64_t len;
  const uint64_t* offsets;   // [n_docs + 1]
  uint64_t n_docs;
  uint64_t R0, R1;           // offsets[0], offsets[n_docs] (host copies)
  Slot* table;
  uint64_t mask;             // slots - 1
  uint64_t occ_limit;        // claimed slots above this set the full flag
  uint64_t key_mask;
  Header* hdr;
  const uint64_t* stage_doc; // [n_stages + 1]
  int64_t base_off;          // logical position of stage 0 (<= 0, > -16)
  uint64_t n_stages;
  uint64_t stages_per_wg;
  uint32_t lds_entries;
  uint32_t lds_flush_at;
  uint32_t policy;
  uint32_t no_lds;
  uint32_t utf8;             // WC_TOKENIZE_UTF8: the UTF-8 reading of word bytes
  uint32_t pad0;
};

// two-pass global count (wc_global.hip)
constexpr uint32_t kParts = 256;         // partitions of the spilled records
constexpr uint32_t kBlockRec = 256;      // records per arena block (4 KiB)
constexpr uint32_t kDictMax = 5120;      // hot-word dictionary capacity (words)
constexpr uint32_t kMapBlock = 1024;     // pass-1 workgroup
constexpr uint32_t kGlobalStage = kMapBlock * 16;  // bytes scanned per pass-1 stage
constexpr uint32_t kDispBuckets = 1024;   // dictionary: displacement buckets (low 9 hash bits)
constexpr uint32_t kDictSlots = 8192;    // dictionary: slots of the perfect hash
constexpr uint32_t kDictRegions = 32;    // dictionary: regions of 256 slots (group mod 32)
constexpr uint32_t kSampleStages = 512;  // pass-1 stages sampled (first 8 KiB of each)
constexpr uint32_t kSamplePer = 2;       // sampled stages per sample workgroup
constexpr uint32_t kSampleLds = 2048;    // LDS table of one sample workgroup
constexpr uint64_t kSampleSlots = 1ull << 19;  // device table of the sample
constexpr uint32_t kStripe = 1024;       // pass-1 bytes per wave per stage
constexpr uint32_t kStripeText = 16 + kStripe + 16;  // per wave: prefix, stripe, padding
constexpr uint32_t kWaveStarts = 128;    // (start, end) pairs of one wave listed at a time
constexpr uint32_t kDictCols = 64;       // dictionary words totalled per pass-2 workgroup
constexpr uint32_t kWinBlocks = 2048;    // pass 2 lists the non-empty blocks this many at a time
constexpr uint32_t kRedSlots = 8192;     // pass-2 LDS slots (13-bit entry indices)

// Dictionary of hot words, chosen from a sample and read-only while the text is scanned: a
// perfect hash by hash-and-displace. A word with hash h belongs to group h mod 512; the group's
// displacement picks its slot in region (h mod 16) (see dict_slot); the slot holds its key
// index; empty slots hold n, the index of an all-zero key that no word matches.
struct DictImage {
  uint32_t n;            // words (key entries) in the dictionary
  uint32_t placed;       // words placed in the perfect hash (the others are never looked up)
  uint32_t n_high;       // selection: words above the count threshold
  uint32_t n_low;        // selection: words at the threshold competing for the rest
  uint32_t hist[256];    // sample counts (clamped at 255) -> number of words
  uint16_t disp[kDispBuckets];
  uint16_t slot[kDictSlots];
  uint4 keys[kDictMax + 1];  // packed words (lo, hi); keys[n] = 0
  uint32_t cnt[kDictMax];    // their sample counts (clamped at 255)
};

struct GlobalParams {
  const uint8_t* corpus;
  uint64_t len;
  const uint64_t* offsets;
  uint64_t n_docs;
  Slot* table;
  uint64_t mask;
  uint64_t occ_limit;
  uint64_t key_mask;
  Header* hdr;
  const uint64_t* stage_doc;
  int64_t base_off;
  uint64_t n_stages;
  uint64_t stages_per_wg;
  uint32_t map_grid;         // pass-1 workgroups
  uint32_t dict_cap;         // dictionary capacity (<= kDictMax)
  DictImage* dict;
  uint32_t* dict_part;       // [map_grid][dict_cap] dictionary hits per pass-1 workgroup
  Slot* sample_table;        // [kSampleSlots]
  Header* sample_hdr;
  uint32_t reduce_entries;   // pass-2 LDS entries (distinct words of a partition, <= kRedSlots)
  uint32_t reduce_cap;       // entries used before further new words go to the global table
  uint32_t S;                // blocks per partition (kParts * S < 2^32): block k = w * J + j is
                             // the j-th of pass-1 workgroup w (J = S / map_grid)
  uint4* arena;              // [S][kParts][kBlockRec] records: block k of partition p at k * kParts + p
  uint16_t* fill;            // [kParts][S] records per block (zero before pass 1)
};
size_t global_map_dyn(uint32_t dict_cap);
size_t global_reduce_dyn(uint32_t entries);
hipError_t set_global_smem(uint32_t dict_cap, uint32_t reduce_entries);
// Sample, dictionary, pass 1 (between events a and b when given) and pass 2. The sample
// table, its header, the dictionary image and the block fills must be zero.
hipError_t launch_global(const GlobalParams& P, hipEvent_t a, hipEvent_t b, hipStream_t s);

// per-document count (wc_docs.hip)
constexpr uint64_t kWin = 32 * 1024;   // default bytes per work item window
constexpr uint64_t kMinWin = 16 * 1024;
constexpr uint32_t kDocW = 256;        // documents per sub-window
constexpr uint32_t kDocLds = 4096;     // LDS table entries (20 bytes each, beside 8192 slots)

struct DocTask {           // device-resident: every size the per-document kernels read
  const uint8_t* corpus;
  uint64_t len;
  const uint64_t* offsets;
  uint64_t n_docs;
};

struct DocParams {
  const DocTask* task;
  Header* hdr;
  uint64_t* win_doc;       // [max_win + 1]
  uint64_t max_win;
  uint64_t* word_offsets;  // [cap_e + 1]
  uint8_t* words;          // [cap_b]
  void* counts;
  uint32_t count_bytes;
  uint32_t lds_entries;
  uint32_t lds_cap;        // live LDS entries before relief
  uint32_t direct_kib;     // documents above this many KiB (0: none) skip the first pass
  uint64_t win_bytes;      // work item window
  uint64_t* docs;          // [cap_e]
  uint64_t* doc_ptr;       // [n_docs]
  uint64_t* doc_len;       // [n_docs]
  uint64_t cap_e, cap_b;
  Slot* arena;             // private tables of large documents
  uint64_t* over_docs;     // [n_docs] documents for the second pass, as queued
  uint64_t* over_sorted;   // [n_docs] the same, largest first
  uint64_t arena_slots;
  uint64_t key_mask;
  uint64_t count_bias;     // added to every exported count (debug; 0 normally)
  uint32_t rc_entries;     // second pass: LDS table entries (all of them usable)
  uint32_t pad1;
};
// second-pass queue entries: document index (bits 0-55), size class while the queue is sorted
// (bits 56-62), queued without a first count (bit 63)
constexpr uint64_t kDirectDoc = 1ull << 63;
constexpr uint64_t kDocIdMask = (1ull << 56) - 1;
size_t doc_dyn(uint32_t entries);  // dynamic LDS of the document kernel
uint32_t recount_entries();         // LDS entries of its second pass (the most that fit)
hipError_t set_doc_smem(size_t dyn);
hipError_t launch_docs(const DocParams& P, uint32_t grid, size_t dyn, hipStream_t s);

hipError_t launch_count(const CountParams& P, bool per_doc, uint32_t grid, uint32_t block,
                        size_t dyn, hipStream_t s);
hipError_t set_count_smem(uint32_t block, size_t dyn);
hipError_t launch_stage_doc(const uint64_t* offsets, uint64_t n_docs, int64_t base_off,
                            uint32_t stage, uint64_t n_stages, uint64_t* out, hipStream_t s);
hipError_t launch_validate(const uint64_t* offsets, uint64_t n_docs, uint64_t len, Header* hdr,
                           hipStream_t s);

// ---- export (compaction of a table into dense arrays) -----------------------------------
struct ExportParams {
  const Slot* table;
  uint64_t slots;
  Header* hdr;
  uint64_t* block_sums;      // [2 * n_blocks] (entries, bytes) per block, then scanned
  uint64_t n_blocks;
  uint64_t* word_offsets;    // [slots + 1]
  uint8_t* words;
  uint64_t word_cap;
  void* counts;
  uint32_t count_bytes;
  uint32_t per_doc;
  uint64_t* docs;            // per-document: entry document
  uint64_t* slot_of_entry;   // optional: entry -> slot (joint tables)
  uint64_t* entry_of_slot;   // optional: slot -> entry
  uint64_t count_bias;       // added to every exported count (debug; 0 normally)
};
constexpr uint32_t kExportBlock = 256;
constexpr uint32_t kExportItems = 4;  // slots per thread
constexpr uint64_t kExportSpan = kExportBlock * kExportItems;

hipError_t launch_export(const ExportParams& E, hipStream_t s);
hipError_t launch_export_list(const ExportParams& E, hipStream_t s);
hipError_t launch_slot_lens(const Slot* table, const uint64_t* slots, uint64_t n, uint64_t* lens,
                            hipStream_t s);
hipError_t launch_slot_write(const Slot* table, const uint64_t* slots, uint64_t n,
                             const uint64_t* word_offsets, uint8_t* words, void* counts,
                             uint32_t count_bytes, uint64_t count_bias, uint64_t* docs,
                             Header* hdr, hipStream_t s);
// exclusive prefix sum of n uint64 values (out may be in); sums: excl_scan_scratch(n) bytes
uint64_t excl_scan_scratch(uint64_t n);
hipError_t excl_scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* sums,
                         hipStream_t s);
// entries (docs[e], slots[e]) grouped by document into sorted_*; doc_ptr / doc_len per
// document; fill: n_docs scratch; sums: excl_scan_scratch(n_docs)
hipError_t group_by_doc(const uint64_t* docs, const uint64_t* slots, uint64_t n, uint64_t n_docs,
                        uint64_t* doc_ptr, uint64_t* doc_len, uint64_t* fill, uint64_t* sums,
                        uint64_t* sorted_docs, uint64_t* sorted_slots, hipStream_t s);

// ---- fills ---------------------------------------------------------------------------------
hipError_t launch_fill_zero(void* p, uint64_t bytes, hipStream_t s);

// ---- merge ---------------------------------------------------------------------------------
struct MergeInput {
  const uint64_t* word_offsets;
  const uint8_t* words;
  const void* counts;
  uint64_t n;
  uint32_t count_bytes;
  uint32_t column;           // joint tables: column of this input
};
hipError_t launch_merge_insert(const MergeInput& in, Slot* table, uint64_t mask,
                               uint64_t occ_limit, uint64_t key_mask, Header* hdr,
                               uint64_t* joint_counts, uint32_t n_columns, hipStream_t s);

// ---- dense reduce (the zero-padded keys x documents matrix) --------------------------------
hipError_t launch_dense_keys(const MergeInput& in, Slot* table, uint64_t mask,
                             uint64_t occ_limit, uint64_t key_mask, Header* hdr,
                             uint64_t* slot_of_input, hipStream_t s);
hipError_t launch_dense_scatter(uint64_t n, const uint64_t* slot_of_input,
                                const uint64_t* entry_of_slot, const uint64_t* docs,
                                const void* counts, uint32_t count_bytes, uint64_t n_docs,
                                uint32_t* matrix, hipStream_t s);
hipError_t launch_dense_rowsum(const uint32_t* matrix, uint64_t rows, uint64_t n_docs,
                               void* counts, uint32_t count_bytes, uint64_t bias, Header* hdr,
                               hipStream_t s);

// ---- top-k ---------------------------------------------------------------------------------
struct TopkParams {
  const uint64_t* word_offsets;  // joint vocabulary, V entries
  const uint8_t* words;
  const uint64_t* joint;         // [V * C] counts, entry-major
  uint64_t V;
  uint32_t C;
  uint32_t k;
  uint64_t min_count;
  uint64_t* totals;              // [C] token totals per corpus (computed by a kernel)
  uint32_t* lists;               // scratch: [C][2][T][k] entry indices
  uint32_t* list_len;            // scratch: [C][2][T]
  uint64_t* out_entry;           // [C * k] selected entries
  uint64_t* n_rows;              // [C]
  // outputs
  uint64_t* out_word_offsets;    // [C*k + 1]
  uint8_t* out_words;
  uint64_t* out_nc;
  uint64_t* out_nr;
  double* out_score;
  const uint64_t* entry_total;   // [V] sum over corpora
};
constexpr uint32_t kTopkThreads = 256;
hipError_t launch_topk(const TopkParams& P, hipStream_t s);

// ---- hashing (debug entry point) ------------------------------------------------------------
hipError_t launch_hash_words(const uint8_t* bytes, const uint64_t* offsets, uint64_t n,
                             uint64_t* out, hipStream_t s);

}  // namespace wc
