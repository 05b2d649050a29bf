/*
 * wc.h - C ABI of libwc, a word-frequency counter for AMD MI355X (gfx950).
 *
 * The operations follow "MapReduce for Counting Word Frequencies with MPI and GPUs":
 *   - map: lower-case the text, drop punctuation, split it into words and count each word
 *     per document (Section 2, Section 3.1);
 *   - reduce: sum the per-document counts of each word (Section 3.2, Section 3.3);
 *   - per-corpus comparison: find the words one corpus uses distinctly more often than the
 *     others (Section 4.3).
 * The whole map and reduce run on the GPU (the direction of Section 5.2): HIP kernels scan
 * the bytes, hash each word with FNV-1a 64, aggregate counts in per-workgroup LDS tables and
 * merge them into one open-addressing table in device memory.
 *
 * Tokeniser (the paper deletes punctuation before splitting; here every byte outside the
 * word alphabet is a delimiter, which agrees wherever punctuation only separates words):
 *   fold(x) = x + 32 for 'A'..'Z', else x (ASCII only);
 *   a byte is a word byte when fold(x) is in 'a'..'z', '0'..'9' or '\'';
 *   a token is a maximal run of word bytes inside one document; its word is the folded run.
 * Document d is bytes [offsets[d], offsets[d+1]) of the corpus; offsets must be
 * non-decreasing and offsets[n_docs] <= corpus_len; bytes outside [offsets[0],
 * offsets[n_docs]) are ignored; empty documents are allowed; a word never spans two
 * documents and has no length limit. Counts are exact: never approximated or dropped.
 *
 * Memory and streams. Every device buffer is owned by the caller (the Python binding uses
 * PyTorch tensors). The library allocates no device memory in wc_count / wc_merge /
 * wc_topk_ratio and keeps no pointer after they return; their outputs live inside the
 * caller's workspace. Work is enqueued on the caller's stream, passed as void* (a
 * hipStream_t; NULL = the null stream). These calls synchronise that stream once before
 * returning (to read sizes and error flags) and are safe to call from several host threads
 * on different streams and workspaces.
 *
 * Errors: every call returns a wc_status. Device errors return WC_EDEVICE and
 * wc_last_hip_error() gives the hipError_t of the calling thread's last failure.
 */
#ifndef WC_H
#define WC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t wc_status;
#define WC_OK          0
#define WC_EINVAL     -1  /* bad argument: null pointer, non-monotone offsets, bad k, ... */
#define WC_ENOMEM     -2  /* workspace too small, or a request over the memory budget */
#define WC_ETABLEFULL -3  /* hash table full: rerun with more slots (the binding doubles) */
#define WC_EOVERFLOW  -4  /* a count does not fit the requested count width */
#define WC_EDEVICE    -5  /* HIP error; see wc_last_hip_error() */
#define WC_EAGAIN     -6  /* not ready yet (server) */

/* counting modes */
#define WC_GLOBAL  0u  /* one table over all documents */
#define WC_PER_DOC 1u  /* one table per document, returned as CSR over documents */

/* flush policies of the per-workgroup LDS table */
#define WC_FLUSH_ALL    0u  /* when the LDS table passes its load limit, flush all of it */
#define WC_FLUSH_BYPASS 1u  /* never flush early; a word that finds no LDS slot goes global */

/* debug flags (wc_opts.debug_flags) */
#define WC_DEBUG_TIME   1u  /* time the count kernel with HIP events (wc_result.kernel_ms) */
#define WC_DEBUG_NO_LDS 2u  /* skip the LDS table: every token goes to the global table */
#define WC_DEBUG_DIRECT 4u  /* global mode: one-pass kernel (LDS table + global atomics);
                               per-document mode: the same kernel over one (document, word)
                               table, sorted into the CSR afterwards */
#define WC_DEBUG_SPILL  8u  /* global mode: two-pass kernels (LDS table + partitioned spill)
                               even for small inputs; by default they run from 256 MiB up */
#define WC_DEBUG_DOCS   16u /* per-document mode: the document-centric kernel whatever the
                               document sizes; by default it runs when documents average at
                               most 64 KiB (larger ones leave too few documents per CU, since
                               each document is counted by one workgroup), else as DIRECT */

/* tokenisers (wc_opts.tokenizer) */
#define WC_TOKENIZE_ASCII 0u  /* the tokeniser above: bytes >= 0x80 are delimiters */
#define WC_TOKENIZE_UTF8  1u  /* the "other languages" of Section 5.2: a byte is a word byte
                                 when it belongs to a well-formed UTF-8 sequence (Unicode,
                                 Table 3-7) inside its document whose code point is a word
                                 character: ASCII word bytes, or any code point from U+0080
                                 except U+0080..U+00BF, U+00D7, U+00F7, U+2000..U+206F,
                                 U+3000..U+303F and U+FEFF; folding stays ASCII-only. Counted
                                 by the one-pass kernel (global, and per-document through one
                                 (document, word) table); wc_batch_* take ASCII only */

/* Launch tuning; a zero field takes the library default. */
typedef struct wc_tuning {
  uint32_t stage_bytes;   /* bytes one workgroup scans per step: 4096 or 8192 (= 16 B/thread) */
  uint32_t lds_entries;   /* LDS table entries per workgroup, power of two, 256..4096 */
  uint32_t flush_policy;  /* WC_FLUSH_ALL or WC_FLUSH_BYPASS */
  uint32_t grid_blocks;   /* workgroups in the count launch (0 = 2 per CU) */
  uint32_t lds_load_pct;  /* LDS table load at which it is flushed (one-pass kernel) or at
                             which a document counts as overflowed (document-centric kernel:
                             it is then counted again with a private table); 0 = default
                             (50 % for the one-pass kernel, 85 % for the document-centric) */
  uint32_t chunk_bytes;   /* per-document mode: bytes per work item, power of two in
                             16 KiB..1 MiB (0 = 32 KiB) */
  uint32_t direct_kib;    /* per-document mode, document-centric kernel: a document longer
                             than chunk_bytes and than this many KiB skips the first,
                             optimistic count (in which it would likely overflow the LDS
                             table) and is counted once, by the second pass (0 = 9/4 of
                             chunk_bytes; WC_DIRECT_NEVER = no document skips it) */
} wc_tuning;

#define WC_DIRECT_NEVER 0xffffffffu

typedef struct wc_opts {
  uint32_t count_bytes;      /* width of exported counts: 4 (int32) or 8 (int64) */
  uint32_t mode;             /* WC_GLOBAL or WC_PER_DOC */
  uint64_t table_slots;      /* global table slots, power of two; 0 = sized from the input */
  const wc_tuning* tuning;   /* NULL = defaults */
  uint32_t debug_flags;      /* WC_DEBUG_* */
  uint32_t debug_hash_bits;  /* 0 = full 64-bit keys; 1..63 keep only the low bits of every
                                key, forcing key collisions so the byte compare decides */
  uint64_t word_bytes_cap;   /* capacity reserved for exported word bytes; 0 = auto */
  uint64_t debug_count_bias; /* 0 normally; otherwise added to every exported count, so that
                                the count-width check (WC_EOVERFLOW) and wide counts can be
                                exercised without 2^31 tokens (the sums themselves are
                                unchanged; total_tokens is not biased) */
  uint32_t tokenizer;        /* WC_TOKENIZE_ASCII (0) or WC_TOKENIZE_UTF8 */
  uint32_t reserved;         /* 0 */
} wc_opts;

typedef struct wc_plan {
  uint64_t table_slots;      /* slots the call will use */
  uint64_t workspace_bytes;  /* bytes of device workspace to pass */
  uint64_t max_entries;      /* capacity of the exported arrays (= table_slots) */
  uint64_t word_bytes_cap;   /* capacity of the exported word bytes */
} wc_plan;

/* A word table in device memory: entry e is the folded word
 * d_words[d_word_offsets[e] .. d_word_offsets[e+1]) with count d_counts[e]. Entry order is
 * unspecified. Per-document tables are grouped by document: the entries of document d are
 * the d_doc_len[d] entries starting at d_doc_ptr[d]; documents follow each other in an
 * unspecified order; d_docs[e] is the document of entry e. */
typedef struct wc_result {
  uint64_t n_entries;
  uint64_t total_tokens;     /* tokens counted (= sum of counts) */
  uint64_t word_bytes;       /* = d_word_offsets[n_entries] */
  uint64_t n_docs;           /* documents (per-document tables) */
  uint64_t table_slots;      /* slots of the table the result was compacted from */
  uint32_t count_bytes;      /* 4 or 8 */
  uint32_t mode;             /* WC_GLOBAL or WC_PER_DOC */
  uint64_t* d_word_offsets;  /* uint64[n_entries + 1] */
  uint8_t* d_words;          /* uint8[word_bytes] */
  void* d_counts;            /* int32 or int64 [n_entries] */
  uint64_t* d_doc_ptr;       /* WC_PER_DOC: uint64[n_docs] first entry of each document */
  uint64_t* d_doc_len;       /* WC_PER_DOC: uint64[n_docs] entries of each document */
  uint64_t* d_docs;          /* WC_PER_DOC: uint64[n_entries], else NULL */
  float kernel_ms;           /* WC_DEBUG_TIME: duration of the count (or merge) kernel */
  float total_ms;            /* WC_DEBUG_TIME: duration of the whole call on the device */
  /* Per-call statistics (zero where a path has none). Two-pass global count:
   * [0] tokens written as records to the hash partitions (words missing the dictionary),
   * [1] records pass 1 added straight to the global table because the workgroup's share of
   *     their partition's arena blocks was used up,
   * [2] dictionary words,
   * [4] records pass 2 could not sum in its LDS table (added to the global table).
   * Document-centric per-document count (the batch API, and wc_count in per-document mode for
   * small documents):
   * [3] documents counted in the kernel's second pass, with a private table in device
   *     memory: those whose words did not fit the LDS table, and those that skipped the
   *     first pass by size (wc_tuning.direct_kib). */
  uint64_t stats[5];
} wc_result;

/* Text of a status code (static storage). */
const char* wc_strerror(wc_status s);

/* hipError_t of the calling thread's last WC_EDEVICE. */
int32_t wc_last_hip_error(void);

/* Plan a wc_count call: slots, workspace bytes and output capacities for a corpus of
 * corpus_len bytes in n_docs documents. No device work. Returns WC_EINVAL for bad options. */
wc_status wc_count_plan(uint64_t corpus_len, uint64_t n_docs, const wc_opts* opts,
                        wc_plan* out);

/* Count the words of a device-resident corpus (Section 3.1 map + Section 3.2 reduce, fused).
 *   d_corpus     device uint8[corpus_len], any alignment; not modified.
 *   d_offsets    device uint64[n_docs + 1] document offsets (see the top of this file).
 *   d_workspace  device buffer of at least wc_count_plan(...).workspace_bytes bytes; it holds
 *                the hash table and the exported arrays that *out points into, so it must
 *                outlive every use of *out.
 *   out          filled on WC_OK (device pointers into d_workspace + host-side sizes).
 * Errors: WC_EINVAL (null pointer with non-zero size, bad options, invalid offsets),
 * WC_ENOMEM (workspace smaller than planned, or more word bytes than word_bytes_cap; then
 * out->word_bytes holds the bytes needed), WC_ETABLEFULL (more distinct words than the table
 * takes at a load of 7/8; rerun with more slots), WC_EOVERFLOW (count_bytes = 4 and a count
 * above INT32_MAX), WC_EDEVICE. */
wc_status wc_count(const uint8_t* d_corpus, uint64_t corpus_len, const uint64_t* d_offsets,
                   uint64_t n_docs, const wc_opts* opts, void* d_workspace,
                   uint64_t workspace_bytes, wc_result* out, void* stream);

/* Count a corpus that is in host memory, overlapping its transfer with the count (Section
 * 4.1 names the host-to-device copy as the main cost of the GPU reduce): the text is cut into
 * pieces of about piece_bytes (at least 1 MiB), each cut made right after an ASCII delimiter
 * byte or at a document start so that no token spans two pieces; piece p+1 is copied on a
 * second stream of the library while piece p is counted on `stream`, all into one global
 * table exported once at the end. Same result as wc_count of the whole corpus.
 *   h_corpus   host uint8[corpus_len] (pinned memory lets the copies run asynchronously);
 *              read, never written; must stay valid until the call returns.
 *   h_offsets  host uint64[n_docs + 1] document offsets.
 *   d_text     device uint8[corpus_len] that receives the text ([offsets[0], offsets[n_docs])
 *              is written); long words in the result refer to it, so it must outlive *out.
 *   d_workspace of wc_count_host_plan() bytes.
 * opts->mode must be WC_GLOBAL. Synchronous: returns when the table is exported. Errors as
 * wc_count. */
wc_status wc_count_host_plan(uint64_t corpus_len, uint64_t n_docs, const wc_opts* opts,
                             uint64_t piece_bytes, wc_plan* out);
wc_status wc_count_host(const uint8_t* h_corpus, uint64_t corpus_len, const uint64_t* h_offsets,
                        uint64_t n_docs, const wc_opts* opts, uint64_t piece_bytes,
                        uint8_t* d_text, void* d_workspace, uint64_t workspace_bytes,
                        wc_result* out, void* stream);

/* wc_count for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same count into one global
 * table (opts->mode must be WC_GLOBAL; the one-pass kernel always runs), with the hash table,
 * header and other scratch in a static device array of the library (34 MiB per GPU, loaded
 * with the library and held until the process ends) instead of a caller workspace. The
 * caller passes the outputs: d_word_offsets uint64[max_entries + 1], d_counts
 * (count_bytes each) [max_entries] and d_words uint8[word_bytes_cap]; *out points into them.
 * Limits: table_slots at most 2^20 (0 = sized from the input as wc_count_plan, capped at
 * 2^20), max_entries >= the table slots used, and a corpus whose per-stage cursor still fits
 * the array (about 1 GiB); beyond them the call returns WC_ENOMEM before any device work.
 * Makes no hipMalloc/hipFree and calls no allocating library routine. Every call on a GPU
 * uses that GPU's one array, so calls that overlap on one GPU (two host threads, or two
 * streams in flight) race and must be serialised by the caller; each call clears what must
 * start at zero. Errors otherwise as wc_count (WC_ETABLEFULL: rerun with more slots, up to the
 * limit; WC_ENOMEM also when the words exceed word_bytes_cap, out->word_bytes then holding
 * the bytes needed). */
wc_status wc_count_static(const uint8_t* d_corpus, uint64_t corpus_len, const uint64_t* d_offsets,
                          uint64_t n_docs, const wc_opts* opts, uint64_t* d_word_offsets,
                          void* d_counts, uint64_t max_entries, uint8_t* d_words,
                          uint64_t word_bytes_cap, wc_result* out, void* stream);

/* Plan a wc_merge of k tables (Section 3.3: the grouped counts of each word are summed).
 * Uses the inputs' host-side sizes only. */
wc_status wc_merge_plan(const wc_result* const* tables, uint32_t k, const wc_opts* opts,
                        wc_plan* out);

/* Merge k tables into one global table holding the pointwise sum of counts over the union of
 * words (per-document inputs are summed over their documents). Inputs are untouched and must
 * stay valid during the call; the result lives in d_workspace. Associative and commutative;
 * merging per-document tables equals counting the concatenation. Errors as wc_count. */
wc_status wc_merge(const wc_result* const* tables, uint32_t k, const wc_opts* opts,
                   void* d_workspace, uint64_t workspace_bytes, wc_result* out, void* stream);

/* The paper's reduce (Section 3.3; the "reduce on GPU" of the Section 4.1 table): the counts of
 * a per-document table laid out as a zero-padded matrix with one row per distinct word and one
 * column per document (uint32 cells, rows x n_docs x 4 bytes), and one kernel summing each
 * row. Same result as wc_merge of that table (a global table, pointwise sums over the
 * documents); kept as the comparison point the paper measured. per_doc must be a WC_PER_DOC
 * table (its d_docs is read). wc_merge_dense_plan gives the workspace for a matrix of `rows`
 * rows (0 = per_doc->n_entries, an upper bound of the distinct words). When the matrix of
 * the actual distinct words does not fit the workspace, wc_merge_dense returns WC_ENOMEM with
 * out->n_entries = the rows needed (plan again with them). WC_DEBUG_TIME: out->kernel_ms is
 * the row-sum kernel alone, out->total_ms the whole call. Errors as wc_merge. */
wc_status wc_merge_dense_plan(const wc_result* per_doc, const wc_opts* opts, uint64_t rows,
                              uint64_t* workspace_bytes);
wc_status wc_merge_dense(const wc_result* per_doc, const wc_opts* opts, void* d_workspace,
                         uint64_t workspace_bytes, wc_result* out, void* stream);

/* Per-corpus distinctive words (Section 4.3 compares presidents by the words each uses more
 * than the others). Over n corpora with joint vocabulary V (the union of their words): for
 * corpus c and word w with n_c(w) >= max(min_count, 1), n_R(w) = the other corpora's count;
 * words are ranked by (n_c+1)/(n_R+1) descending, compared exactly, then n_c descending, then
 * word bytes ascending (unsigned, a proper prefix first); a total order, so the answer is
 * unique. score = ((n_c+1)/(N_c+V)) / ((n_R+1)/(N_R+V)) in double, N_c = tokens of corpus
 * c, N_R = tokens of the others. Row r of corpus c is at index c*k + r; n_rows[c] <= k rows
 * are valid (fewer when fewer words are eligible). */
typedef struct wc_topk {
  uint32_t n_corpora;
  uint32_t k;
  uint64_t vocab_size;       /* V */
  uint64_t* d_word_offsets;  /* uint64[n_corpora*k + 1]: row words in d_words */
  uint8_t* d_words;          /* folded words of the rows, row-major */
  uint64_t* d_n_c;           /* uint64[n_corpora*k] */
  uint64_t* d_n_rest;        /* uint64[n_corpora*k] */
  double* d_score;           /* double[n_corpora*k] */
  uint64_t n_rows[64];       /* host: valid rows per corpus */
  uint64_t word_bytes;       /* host: bytes used in d_words */
} wc_topk;

/* Plan wc_topk_ratio: workspace bytes for n corpora (at most 64) and k rows per corpus
 * (1 <= k <= 4096). */
wc_status wc_topk_ratio_plan(const wc_result* const* corpora, uint32_t n_corpora, uint32_t k,
                             uint64_t* workspace_bytes);

/* Top-k distinctive words per corpus (see wc_topk). Inputs are global word tables (for
 * example wc_count results of each corpus). Errors: WC_EINVAL (n_corpora 0 or > 64, k 0 or
 * > 4096, null pointers), WC_ENOMEM, WC_EDEVICE. */
wc_status wc_topk_ratio(const wc_result* const* corpora, uint32_t n_corpora, uint32_t k,
                        uint64_t min_count, void* d_workspace, uint64_t workspace_bytes,
                        wc_topk* out, void* stream);

/* Batched per-document counting (Section 3.1 counts every document in its own dictionary):
 * all documents of a corpus are counted into per-document tables by one persistent launch
 * that takes 32 KiB windows of documents from a device-side queue. The first wc_batch_run
 * captures the whole call (task upload, clears, kernels, size readback) into a HIP graph; later
 * runs only update a pinned host task description and replay the graph, so a run makes no
 * allocation and one graph launch. Device memory is the caller's workspace of
 * wc_batch_plan() bytes, sized for at most max_docs documents of max_bytes bytes in total
 * (max_bytes < 2^32). The batch object itself holds only host-side resources (a stream, pinned
 * host memory, the graph). Results point into the workspace and stay valid until the next run.
 * opts->mode must be WC_PER_DOC; opts->tuning selects lds_entries and grid_blocks. */
typedef struct wc_batch wc_batch;

wc_status wc_batch_plan(const wc_opts* opts, uint64_t max_docs, uint64_t max_bytes,
                        uint64_t* workspace_bytes);

wc_status wc_batch_create(const wc_opts* opts, uint64_t max_docs, uint64_t max_bytes,
                          void* d_workspace, uint64_t workspace_bytes, wc_batch** out);

/* Count one corpus (device pointers, as wc_count). The caller's stream is ordered before the
 * graph launch and the call returns after the results are complete. Errors: WC_EINVAL
 * (larger than the plan, invalid offsets), WC_ENOMEM (outputs or private tables short: plan
 * with larger word_bytes_cap / table_slots), WC_ETABLEFULL, WC_EOVERFLOW, WC_EDEVICE. */
wc_status wc_batch_run(wc_batch* b, const uint8_t* d_corpus, uint64_t corpus_len,
                       const uint64_t* d_offsets, uint64_t n_docs, wc_result* out, void* stream);

wc_status wc_batch_destroy(wc_batch* b);

/* Serving. A server counts texts submitted at any time and keeps each result resident on
 * the device until released, answering merge queries over resident tables. It owns one
 * device pool of mem_budget bytes (allocated at creation): count memory (text, offsets,
 * workspace) is taken from its low end and resident tables from its high end. A request
 * waits for admission until the memory its count needs is free, as long as some running
 * request holds count memory (it will return it); requests larger than the budget fail with
 * WC_ENOMEM at submission, and a request fails with WC_ENOMEM when nothing runs and resident
 * tables leave no block large enough (only wc_server_release can free them). A finished count
 * waits for its resident block while another running request can still return memory, and
 * fails with WC_ENOMEM otherwise. max_streams worker threads (1..16)
 * each drive one HIP stream, so admitted requests overlap on the device; small
 * single-document requests queued together are counted in one per-document launch and split
 * into one table per request. Results are global word tables in the server's memory, valid
 * until wc_server_release(id). Thread-safe: submit/poll/wait/merge/release may be called from
 * any host thread. */
typedef struct wc_server wc_server;

wc_status wc_server_create(int device, uint64_t mem_budget, uint32_t max_streams,
                           wc_server** out);

/* Where the text of a submitted request is (wc_server_submit's text_on_device): */
#define WC_TEXT_HOST_COPY     0  /* host memory, copied at submission (free it at once) */
#define WC_TEXT_DEVICE        1  /* device memory, valid until the request completes */
#define WC_TEXT_HOST_IN_PLACE 2  /* host memory read in place, valid until the request
                                    completes; pinned memory is transferred without staging */

/* Submit a count: text (see WC_TEXT_*), host offsets[n_docs + 1]. opts->mode must be
 * WC_GLOBAL. Returns the request id in *req_id. */
wc_status wc_server_submit(wc_server* s, const uint8_t* text, uint64_t len,
                           const uint64_t* offsets, uint64_t n_docs, int text_on_device,
                           const wc_opts* opts, uint64_t* req_id);

/* WC_EAGAIN until request id is complete; then its status, and *out describes its table. */
wc_status wc_server_poll(wc_server* s, uint64_t id, wc_result* out);

/* Block until request id is complete; its status, and *out describes its table. */
wc_status wc_server_wait(wc_server* s, uint64_t id, wc_result* out);

/* Host clock times (seconds, steady clock) of submission, start and completion. */
wc_status wc_server_times(wc_server* s, uint64_t id, double* submit_s, double* start_s,
                          double* done_s);

/* Queue the merge of k resident tables (Section 3.3) into a new resident table. The inputs
 * must be requests of this server that have not been released (WC_EINVAL otherwise); they are
 * pinned at submission, so releasing one before the merge has read it defers freeing its
 * memory until the merge is done. */
wc_status wc_server_merge(wc_server* s, const uint64_t* ids, uint32_t k, const wc_opts* opts,
                          uint64_t* new_id);

/* Wait for request id, then release it: its id is no longer valid and its resident table is
 * freed (once no queued or running merge still reads it). */
wc_status wc_server_release(wc_server* s, uint64_t id);

/* Count launches the server has made (packing makes this smaller than the requests). */
uint64_t wc_server_launches(wc_server* s);

wc_status wc_server_destroy(wc_server* s);

/* Autotuner: time wc_count on a calibration sample (device-resident, as wc_count) for each
 * point of a small grid of launch tunings (per-document mode: one point, 32 KiB work items
 * with 4096 LDS entries at an 85 % load, which a calibration sample of a few thousand
 * documents cannot rank against others; global mode: LDS entries x flush load x flush
 * policy) with HIP events on
 * `stream`, and return the
 * fastest in *best (its time per call in *best_ms). The workspace must hold
 * wc_autotune_plan() bytes. The sample's counts are not returned. Output and private-table
 * sizes come from opts (word_bytes_cap, table_slots) as in wc_count; a grid point that runs
 * out of that room is skipped, and WC_ENOMEM is returned when no point fits. */
wc_status wc_autotune_plan(uint64_t len, uint64_t n_docs, const wc_opts* opts,
                           uint64_t* workspace_bytes);
wc_status wc_autotune(const uint8_t* d_sample, uint64_t len, const uint64_t* d_offsets,
                      uint64_t n_docs, const wc_opts* opts, void* d_workspace,
                      uint64_t workspace_bytes, wc_tuning* best, float* best_ms, void* stream);

/* Copy a table to host buffers (synchronous): word_offsets[n_entries + 1] (as stored),
 * words[word_bytes] (starting at d_words[d_word_offsets[0]]), counts[n_entries] (count_bytes
 * each). Any output pointer may be NULL to skip it. */
wc_status wc_table_to_host(const wc_result* t, uint64_t* word_offsets, uint8_t* words,
                           void* counts);

/* Host helper: canonical order of a table copied to host memory (for example by
 * wc_table_to_host): perm[i] = the entry that comes i-th when the entries are ordered by
 * document (docs may be NULL for a global table), then by word bytes, unsigned and bytewise,
 * a proper prefix first. word_offsets[n + 1] as stored (word e is words[word_offsets[e] -
 * word_offsets[0] .. word_offsets[e+1] - word_offsets[0])), docs[n] or NULL, perm[n] out.
 * The library's entry order is unspecified; this is the order to compare tables in. No
 * device work. Errors: WC_EINVAL (null pointers, decreasing offsets). */
wc_status wc_sort_canonical(uint64_t n, const uint64_t* word_offsets, const uint8_t* words,
                            const uint64_t* docs, uint64_t* perm);

/* FNV-1a 64 (Fowler, Noll, Vo) of n byte strings on the device: d_out[i] = FNV-1a 64 of
 * fold(d_bytes[d_offsets[i] .. d_offsets[i+1])), computed by the same device function the
 * counter uses (offset basis 0xcbf29ce484222325, prime 0x100000001b3; a result of 0 is
 * stored as 1 since 0 marks an empty slot). Exposed so the hash can be checked against
 * published test vectors. */
wc_status wc_hash_words(const uint8_t* d_bytes, const uint64_t* d_offsets, uint64_t n,
                        uint64_t* d_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* WC_H */
