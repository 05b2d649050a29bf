// Host side of the C ABI declared in include/wc.h: argument checks, workspace layout,
// kernel launches on the caller's stream, and the single synchronisation that reads sizes
// and error flags back.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "wc_internal.h"

using namespace wc;

namespace {

thread_local int32_t g_last_hip = 0;

constexpr uint64_t kAlign = 256;
constexpr uint32_t kDefaultLds = 2048;
constexpr uint32_t kDefaultBlock = 512;
constexpr uint32_t kReduceLds = 5632;         // pass-2 LDS entries (110 KiB + 32 KiB of slots)
constexpr uint64_t kDocKernelMaxMean = 64ull << 10;  // per-document mode: see use_doc_kernel
constexpr uint64_t kSpillMinBytes = 256ull << 20;  // two-pass global count from this size
constexpr uint64_t kMaxWgBytes = 1ull << 31;  // text per pass-1 workgroup (32-bit LDS counts)

uint64_t align_up(uint64_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }
bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }
uint64_t next_pow2(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

#define HIPCHK(expr)                                  \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) {                           \
      g_last_hip = (int32_t)e_;                       \
      return WC_EDEVICE;                              \
    }                                                 \
  } while (0)

// Bump allocation inside the caller's workspace (base may be null when only sizing).
struct Bump {
  uint8_t* base;
  uint64_t off = 0;
  explicit Bump(void* b) : base((uint8_t*)b) {}
  template <class T>
  T* take(uint64_t bytes) {
    uint64_t o = off;
    off = align_up(off + bytes);
    return base ? (T*)(base + o) : (T*)nullptr;
  }
};

struct Tune {
  uint32_t block, stage, lds, policy, grid, flush_at, pct, chunk;
  uint32_t direct_kib;  // document-centric kernel: 0 = no document skips the first count
};

int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

bool resolve_tuning(const wc_tuning* t, Tune* out) {
  Tune u;
  u.stage = t && t->stage_bytes ? t->stage_bytes : kDefaultBlock * 16;
  if (u.stage != 4096 && u.stage != 8192) return false;
  u.block = u.stage / 16;
  u.lds = t && t->lds_entries ? t->lds_entries : kDefaultLds;
  if (!is_pow2(u.lds) || u.lds < 256 || u.lds > 4096) return false;
  u.policy = t ? t->flush_policy : WC_FLUSH_ALL;
  if (u.policy > WC_FLUSH_BYPASS) return false;
  u.grid = t ? t->grid_blocks : 0;
  uint32_t pct = t && t->lds_load_pct ? t->lds_load_pct : 50;
  if (pct > 100) return false;
  u.pct = t && t->lds_load_pct ? t->lds_load_pct : 0;
  u.flush_at = (uint32_t)((uint64_t)u.lds * pct / 100);
  u.chunk = t && t->chunk_bytes ? t->chunk_bytes : (uint32_t)kWin;
  if (!is_pow2(u.chunk) || u.chunk < kMinWin || u.chunk > (1u << 20)) return false;
  const uint32_t dk = t ? t->direct_kib : 0u;
  u.direct_kib = dk == WC_DIRECT_NEVER ? 0u : dk ? dk : (u.chunk >> 10) * 9 / 4;
  *out = u;
  return true;
}

bool opts_ok(const wc_opts* o) {
  if (!o) return false;
  if (o->count_bytes != 4 && o->count_bytes != 8) return false;
  if (o->mode != WC_GLOBAL && o->mode != WC_PER_DOC) return false;
  if (o->table_slots && (!is_pow2(o->table_slots) || o->table_slots < 64)) return false;
  if (o->debug_hash_bits > 63) return false;
  if (o->tokenizer != WC_TOKENIZE_ASCII && o->tokenizer != WC_TOKENIZE_UTF8) return false;
  return true;
}

uint64_t key_mask_of(const wc_opts* o) {
  return o->debug_hash_bits ? ((1ull << o->debug_hash_bits) - 1) : ~0ull;
}

struct CountLayout {
  uint64_t S, n_stages, n_blocks, word_cap;
  Header* hdr;
  Slot* table;
  uint64_t* stage_doc;
  uint64_t* bsum;
  uint64_t* woff;
  void* counts;
  uint8_t* words;
  // per-document
  uint64_t *docs, *doc_ptr, *doc_len, *list_docs, *list_slots, *sorted_docs, *sorted_slots, *lens;
  uint64_t* doc_fill;  // per-document scatter cursors
  uint64_t* sums;  // scan block totals
  // two-pass global count
  bool spill = false;
  uint32_t spill_grid = 0, static_blocks = 0, dict_cap = 0;
  uint64_t spill_spw = 0;
  uint4* arena = nullptr;
  uint16_t* fill = nullptr;
  Slot* sample_table = nullptr;
  Header* sample_hdr = nullptr;
  DictImage* dict = nullptr;
  uint32_t* dict_part = nullptr;
  uint64_t total;
};

bool use_spill(uint64_t len, const wc_opts* o) {
  if (o->mode != WC_GLOBAL) return false;
  if (o->tokenizer == WC_TOKENIZE_UTF8) return false;  // the one-pass kernel reads UTF-8
  if (o->debug_flags & WC_DEBUG_SPILL) return true;
  if (o->debug_flags & (WC_DEBUG_DIRECT | WC_DEBUG_NO_LDS)) return false;
  return len >= kSpillMinBytes;
}

// The two-pass kernels scan kGlobalStage-byte stages; the stage size tunes only the one-pass
// kernel.
void global_stage(uint64_t len, const wc_opts* o, Tune* tu) {
  if (use_spill(len, o)) {
    tu->stage = kGlobalStage;
    tu->block = kGlobalStage / 16;
  }
}

int64_t base_offset(const uint8_t* corpus) {
  return -(int64_t)((uintptr_t)corpus & 15);
}

// Per-document count (document-centric kernel): outputs and private tables of large documents.
struct DocLayout {
  uint64_t n_win, cap_e, cap_b, arena_slots;
  Header* hdr;
  DocTask* task;
  uint64_t* win_doc;
  uint64_t* woff;
  uint8_t* words;
  void* counts;
  uint64_t* docs;
  uint64_t* doc_ptr;
  uint64_t* doc_len;
  Slot* arena;
  uint64_t* over_docs;
  uint64_t* over_sorted;
  uint64_t total;
};

// The document-centric kernel counts each document in one workgroup: it wins with many small
// documents and loses badly with a few large ones (a 1 MiB document keeps one workgroup busy
// while the others idle), where the one-pass kernel over a (document, word) table spreads the
// text over every CU.
bool use_doc_kernel(const wc_opts* o, uint64_t len, uint64_t n_docs) {
  if (o->mode != WC_PER_DOC || (o->debug_flags & WC_DEBUG_DIRECT)) return false;
  if (o->tokenizer == WC_TOKENIZE_UTF8) return false;  // the one-pass kernel reads UTF-8
  if (o->debug_flags & WC_DEBUG_DOCS) return true;
  return n_docs == 0 || len / n_docs <= kDocKernelMaxMean;
}

void layout_docs(uint64_t len, uint64_t n_docs, const wc_opts* o, void* ws, DocLayout* L) {
  L->n_win = len / kMinWin + 1;  // room for any work-item size
  L->cap_b = o->word_bytes_cap ? o->word_bytes_cap : std::max<uint64_t>(len / 4, 4096);
  L->cap_e = L->cap_b / 3 + n_docs + 64;
  L->arena_slots = o->table_slots ? o->table_slots
                                  : std::max<uint64_t>(1ull << 16, len / 16 + 64 * 4096);
  Bump B(ws);
  L->hdr = B.take<Header>(sizeof(Header));
  L->task = B.take<DocTask>(sizeof(DocTask));
  L->win_doc = B.take<uint64_t>((L->n_win + 1) * 8);
  L->woff = B.take<uint64_t>((L->cap_e + 1) * 8);
  L->words = B.take<uint8_t>(L->cap_b);
  L->counts = B.take<uint8_t>(L->cap_e * o->count_bytes);
  L->docs = B.take<uint64_t>(L->cap_e * 8);
  L->doc_ptr = B.take<uint64_t>(std::max<uint64_t>(n_docs, 1) * 8);
  L->doc_len = B.take<uint64_t>(std::max<uint64_t>(n_docs, 1) * 8);
  L->arena = B.take<Slot>(L->arena_slots * sizeof(Slot));
  L->over_docs = B.take<uint64_t>(std::max<uint64_t>(n_docs, 1) * 8);
  L->over_sorted = B.take<uint64_t>(std::max<uint64_t>(n_docs, 1) * 8);
  L->total = B.off;
}

DocParams doc_params(const DocLayout& L, const wc_opts* o, uint32_t lds, uint32_t pct,
                     uint32_t chunk, uint32_t direct_kib) {
  DocParams P;
  P.lds_cap = (uint32_t)((uint64_t)lds * (pct ? pct : 85) / 100);
  if (P.lds_cap < 1) P.lds_cap = 1;
  if (P.lds_cap > lds - lds / 8) P.lds_cap = lds - lds / 8;
  P.direct_kib = direct_kib;
  P.win_bytes = chunk;
  P.task = L.task;
  P.hdr = L.hdr;
  P.win_doc = L.win_doc;
  P.max_win = L.n_win;
  P.word_offsets = L.woff;
  P.words = L.words;
  P.counts = L.counts;
  P.count_bytes = o->count_bytes;
  P.lds_entries = lds;
  P.rc_entries = recount_entries();
  P.pad1 = 0;
  P.docs = L.docs;
  P.doc_ptr = L.doc_ptr;
  P.doc_len = L.doc_len;
  P.cap_e = L.cap_e;
  P.cap_b = L.cap_b;
  P.arena = L.arena;
  P.over_docs = L.over_docs;
  P.over_sorted = L.over_sorted;
  P.arena_slots = L.arena_slots;
  P.key_mask = key_mask_of(o);
  P.count_bias = o->debug_count_bias;
  return P;
}

// Caller-owned output arrays (the allocation-free entry point); NULL: they come from the
// workspace.
struct OutBufs {
  uint64_t* woff;
  void* counts;
  uint8_t* words;
  uint64_t word_cap;
};

bool layout_count(uint64_t len, uint64_t n_docs, const wc_opts* o, const Tune& tu,
                  const uint8_t* corpus, void* ws, CountLayout* L,
                  const OutBufs* outs = nullptr) {
  const bool per_doc = o->mode == WC_PER_DOC;
  uint64_t S = o->table_slots;
  if (!S) {
    // one slot per 16 bytes of text: short texts have many distinct words per byte (Zipf 1.05
    // text over 500,000 words has one distinct word per 16 bytes at 32 KiB, per 22 at 256 KiB,
    // per 30 at 1 MiB), and a table that overflows costs a whole second count; long texts hit
    // the cap below
    // per document: a (document, word) pair per 8 bytes, and room for two per document (a
    // corpus of tiny documents has about one pair per document)
    uint64_t want = per_doc ? std::max<uint64_t>(len / 8, 2 * n_docs) : len / 16;
    want = std::max<uint64_t>(want, 4096);
    want = std::min<uint64_t>(want, per_doc ? (1ull << 28) : (1ull << 22));
    S = next_pow2(want);
  }
  L->S = S;
  int64_t b0 = corpus ? base_offset(corpus) : -15;
  L->n_stages = len ? (uint64_t)(((int64_t)len - b0 + tu.stage - 1) / tu.stage) : 0;
  L->n_blocks = (S + kExportSpan - 1) / kExportSpan;
  uint64_t cap = o->word_bytes_cap;
  if (!cap) cap = std::min<uint64_t>(len, std::max<uint64_t>(S * 24, 1ull << 20));
  L->word_cap = std::max<uint64_t>(cap, 16);
  Bump B(ws);
  L->hdr = B.take<Header>(sizeof(Header));
  L->table = B.take<Slot>(S * sizeof(Slot));
  L->stage_doc = B.take<uint64_t>((L->n_stages + 2) * 8);
  L->bsum = B.take<uint64_t>(L->n_blocks * 16);
  if (outs) {
    L->woff = outs->woff;
    L->counts = outs->counts;
    L->words = outs->words;
    L->word_cap = outs->word_cap;
  } else {
    L->woff = B.take<uint64_t>((S + 1) * 8);
    L->counts = B.take<uint8_t>(S * o->count_bytes);
    L->words = B.take<uint8_t>(L->word_cap);
  }
  L->docs = L->doc_ptr = L->doc_len = L->list_docs = L->list_slots = L->sorted_docs =
      L->sorted_slots = L->lens = L->doc_fill = L->sums = nullptr;
  if (per_doc) {
    L->docs = B.take<uint64_t>(S * 8);
    L->doc_ptr = B.take<uint64_t>((n_docs + 1) * 8);
    L->doc_len = B.take<uint64_t>((n_docs + 1) * 8);
    L->list_docs = B.take<uint64_t>(S * 8);
    L->list_slots = B.take<uint64_t>(S * 8);
    L->sorted_docs = B.take<uint64_t>(S * 8);
    L->sorted_slots = B.take<uint64_t>(S * 8);
    L->lens = B.take<uint64_t>((S + 1) * 8);
    L->doc_fill = B.take<uint64_t>((n_docs + 1) * 8);
    L->sums = B.take<uint64_t>(std::max(excl_scan_scratch(S + 1), excl_scan_scratch(n_docs)));
  }
  L->spill = use_spill(len, o) && L->n_stages > 0;
  if (L->spill) {
    // pass 1: one workgroup per CU (or the tuning's grid), contiguous stage ranges of at most
    // kMaxWgBytes of text each
    // sized from the stage count at the worst corpus alignment, so that the plan (which
    // does not know the pointer) and the call lay out the same workspace; a workgroup whose
    // range starts past the last stage only closes its blocks
    const uint64_t ns_max = (len + 15 + tu.stage - 1) / tu.stage;
    uint64_t grid = tu.grid ? tu.grid : (uint64_t)device_cus();
    grid = std::min<uint64_t>(grid, ns_max);
    uint64_t spw = (ns_max + grid - 1) / grid;
    spw = std::min<uint64_t>(spw, kMaxWgBytes / kGlobalStage);
    grid = (ns_max + spw - 1) / spw;
    L->spill_grid = (uint32_t)grid;
    L->spill_spw = spw;
    L->dict_cap = std::min<uint32_t>(o->tuning && o->tuning->lds_entries ? tu.lds : kDictMax,
                                     kDictMax);
    // Each workgroup owns J interleaved blocks of every partition: room for one record per
    // 12.8 bytes of text spread evenly (Zipf text spills about one per 23 bytes); a partition
    // of a workgroup that runs out counts the rest in the global table.
    const uint64_t blk_bytes = (uint64_t)kBlockRec * 16;
    const uint64_t per = grid * kParts * kBlockRec;  // records per static round of blocks
    const uint64_t J = std::max<uint64_t>(1, (len * 5 / 64 + per - 1) / per);
    const uint64_t S = J * grid;
    if ((uint64_t)kParts * S >= (1ull << 32)) return false;  // block indices are 32-bit
    L->static_blocks = (uint32_t)S;
    L->arena = B.take<uint4>((uint64_t)kParts * S * blk_bytes);
    L->fill = B.take<uint16_t>((uint64_t)kParts * S * 2);
    L->sample_table = B.take<Slot>(kSampleSlots * sizeof(Slot));
    L->sample_hdr = B.take<Header>(sizeof(Header));
    L->dict = B.take<DictImage>(sizeof(DictImage));
    L->dict_part = B.take<uint32_t>(grid * L->dict_cap * 4);
  }
  L->total = B.off;
  return true;
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr, c = nullptr, d = nullptr;
  bool on = false;
  hipError_t init(bool enable) {
    on = enable;
    if (!on) return hipSuccess;
    hipError_t e;
    if ((e = hipEventCreate(&a)) != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) return e;
    if ((e = hipEventCreate(&c)) != hipSuccess) return e;
    return hipEventCreate(&d);
  }
  ~Timer() {
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
    if (c) hipEventDestroy(c);
    if (d) hipEventDestroy(d);
  }
};


hipError_t ensure_smem_attr() {
  static hipError_t once = [] {
    hipError_t e = set_count_smem(512, 160 * 1024 - 40 * 1024);
    if (e == hipSuccess) e = set_count_smem(256, 160 * 1024 - 24 * 1024);
    if (e == hipSuccess) e = set_global_smem(kDictMax, kReduceLds);
    if (e == hipSuccess) e = set_doc_smem(doc_dyn(kDocLds));
    return e;
  }();
  return once;
}

// phases of count_table: all three for a plain call; a corpus counted in pieces clears once,
// counts each piece into the same table and exports once
constexpr unsigned kPhaseClear = 1u, kPhaseCount = 2u, kPhaseExport = 4u;
constexpr unsigned kPhaseAll = kPhaseClear | kPhaseCount | kPhaseExport;

wc_status count_table(const uint8_t* d_corpus, uint64_t corpus_len, const uint64_t* d_offsets,
                      uint64_t n_docs, const wc_opts* opts, const Tune& tu, const CountLayout& L,
                      wc_result* out, hipStream_t s, unsigned phases = kPhaseAll);

wc_status finish_flags(const Header& h) {
  if (h.flags & kFlagBadOffsets) return WC_EINVAL;
  if (h.flags & kFlagTableFull) return WC_ETABLEFULL;
  if (h.flags & kFlagWordCap) return WC_ENOMEM;
  if (h.flags & kFlagCountOverflow) return WC_EOVERFLOW;
  if (h.flags & kFlagStall) return WC_EDEVICE;
  return WC_OK;
}

}  // namespace

extern "C" {

const char* wc_strerror(wc_status s) {
  switch (s) {
    case WC_OK: return "ok";
    case WC_EINVAL: return "invalid argument";
    case WC_ENOMEM: return "workspace too small or over the memory budget";
    case WC_ETABLEFULL: return "hash table full; use more slots";
    case WC_EOVERFLOW: return "count does not fit the requested width";
    case WC_EDEVICE: return "HIP error";
    case WC_EAGAIN: return "not ready";
    default: return "unknown status";
  }
}

int32_t wc_last_hip_error(void) { return g_last_hip; }

wc_status wc_count_plan(uint64_t corpus_len, uint64_t n_docs, const wc_opts* opts,
                        wc_plan* out) {
  if (!opts_ok(opts) || !out) return WC_EINVAL;
  Tune tu;
  if (!resolve_tuning(opts->tuning, &tu)) return WC_EINVAL;
  global_stage(corpus_len, opts, &tu);
  if (opts->mode == WC_PER_DOC && n_docs >= 0xffffffffull) return WC_EINVAL;
  if (use_doc_kernel(opts, corpus_len, n_docs)) {
    if (corpus_len >= (1ull << 32)) return WC_EINVAL;  // packed output cursor: 32-bit fields
    DocLayout D;
    layout_docs(corpus_len, n_docs, opts, nullptr, &D);
    out->table_slots = D.arena_slots;
    out->workspace_bytes = D.total;
    out->max_entries = D.cap_e;
    out->word_bytes_cap = D.cap_b;
    return WC_OK;
  }
  CountLayout L;
  if (!layout_count(corpus_len, n_docs, opts, tu, nullptr, nullptr, &L)) return WC_EDEVICE;
  out->table_slots = L.S;
  out->workspace_bytes = L.total + kAlign;  // room for any corpus alignment
  out->max_entries = L.S;
  out->word_bytes_cap = L.word_cap;
  return WC_OK;
}

wc_status wc_count(const uint8_t* d_corpus, uint64_t corpus_len, const uint64_t* d_offsets,
                   uint64_t n_docs, const wc_opts* opts, void* d_workspace,
                   uint64_t workspace_bytes, wc_result* out, void* stream) {
  if (!opts_ok(opts) || !out || !d_workspace) return WC_EINVAL;
  if (corpus_len && !d_corpus) return WC_EINVAL;
  if (!d_offsets) return WC_EINVAL;
  Tune tu;
  if (!resolve_tuning(opts->tuning, &tu)) return WC_EINVAL;
  global_stage(corpus_len, opts, &tu);
  const bool per_doc = opts->mode == WC_PER_DOC;
  if (per_doc && n_docs >= 0xffffffffull) return WC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(ensure_smem_attr());
  if (use_doc_kernel(opts, corpus_len, n_docs)) {
    if (corpus_len >= (1ull << 32)) return WC_EINVAL;
    DocLayout D;
    layout_docs(corpus_len, n_docs, opts, d_workspace, &D);
    if (D.total > workspace_bytes) return WC_ENOMEM;
    uint32_t lds = opts->tuning && opts->tuning->lds_entries ? tu.lds : kDocLds;
    Timer tm;
    HIPCHK(tm.init(opts->debug_flags & WC_DEBUG_TIME));
    if (tm.on) HIPCHK(hipEventRecord(tm.c, s));
    DocTask task{d_corpus, corpus_len, d_offsets, n_docs};
    HIPCHK(hipMemcpyAsync(D.task, &task, sizeof(task), hipMemcpyHostToDevice, s));
    HIPCHK(launch_fill_zero(D.hdr, sizeof(Header), s));
    uint32_t grid = tu.grid ? tu.grid : (uint32_t)device_cus();
    DocParams P = doc_params(D, opts, lds, tu.pct, tu.chunk, tu.direct_kib);
    if (tm.on) HIPCHK(hipEventRecord(tm.a, s));
    HIPCHK(launch_docs(P, grid, doc_dyn(lds), s));
    if (tm.on) HIPCHK(hipEventRecord(tm.b, s));
    Header h;
    HIPCHK(hipMemcpyAsync(&h, D.hdr, sizeof(Header), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    memset(out, 0, sizeof(*out));
    out->n_entries = h.out_cursor >> 32;
    out->word_bytes = h.out_cursor & 0xffffffffull;
    out->total_tokens = h.total_tokens;
    out->n_docs = n_docs;
    out->table_slots = std::max<uint64_t>(h.arena_next, D.arena_slots);
    out->stats[3] = h.over_n;
    out->count_bytes = opts->count_bytes;
    out->mode = WC_PER_DOC;
    out->d_word_offsets = D.woff;
    out->d_words = D.words;
    out->d_counts = D.counts;
    out->d_doc_ptr = D.doc_ptr;
    out->d_doc_len = D.doc_len;
    out->d_docs = D.docs;
    if (tm.on) {
      HIPCHK(hipEventRecord(tm.d, s));
      HIPCHK(hipEventSynchronize(tm.d));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, tm.a, tm.b));
      out->kernel_ms = ms;
      HIPCHK(hipEventElapsedTime(&ms, tm.c, tm.d));
      out->total_ms = ms;
    }
    return finish_flags(h);
  }
  CountLayout L;
  if (!layout_count(corpus_len, n_docs, opts, tu, d_corpus, d_workspace, &L)) return WC_EDEVICE;
  if (L.total > workspace_bytes) return WC_ENOMEM;
  return count_table(d_corpus, corpus_len, d_offsets, n_docs, opts, tu, L, out, s);
}

}  // extern "C"

namespace {

// The table path of wc_count (one global table, or one (document, word) table sorted into a
// CSR) over a laid-out workspace: clear, count (one- or two-pass), export. `phases` selects
// the steps (a global count in pieces: clear with the first piece, export after the last).
wc_status count_table(const uint8_t* d_corpus, uint64_t corpus_len, const uint64_t* d_offsets,
                      uint64_t n_docs, const wc_opts* opts, const Tune& tu, const CountLayout& L,
                      wc_result* out, hipStream_t s, unsigned phases) {
  const bool per_doc = opts->mode == WC_PER_DOC;
  Timer tm;
  HIPCHK(tm.init((opts->debug_flags & WC_DEBUG_TIME) && phases == kPhaseAll));
  if (tm.on) HIPCHK(hipEventRecord(tm.c, s));

  if (phases & kPhaseClear) {
    HIPCHK(launch_fill_zero(L.hdr, sizeof(Header), s));
    HIPCHK(launch_fill_zero(L.table, L.S * sizeof(Slot), s));
  }
  const uint64_t occ_limit = L.S - L.S / 8;
  if ((phases & kPhaseCount) && corpus_len && n_docs) {
    HIPCHK(launch_validate(d_offsets, n_docs, corpus_len, L.hdr, s));
    const int64_t b0 = base_offset(d_corpus);
    HIPCHK(launch_stage_doc(d_offsets, n_docs, b0, tu.stage, L.n_stages, L.stage_doc, s));
    CountParams P;
    P.corpus = d_corpus;
    P.len = corpus_len;
    P.offsets = d_offsets;
    P.n_docs = n_docs;
    P.R0 = 0;
    P.R1 = 0;
    P.table = L.table;
    P.mask = L.S - 1;
    P.occ_limit = occ_limit;
    P.key_mask = key_mask_of(opts);
    P.hdr = L.hdr;
    P.stage_doc = L.stage_doc;
    P.base_off = b0;
    P.n_stages = L.n_stages;
    uint32_t grid = tu.grid ? tu.grid : (uint32_t)device_cus() * 2;
    if (grid > L.n_stages) grid = (uint32_t)L.n_stages;
    P.stages_per_wg = (L.n_stages + grid - 1) / grid;
    grid = (uint32_t)((L.n_stages + P.stages_per_wg - 1) / P.stages_per_wg);
    P.lds_entries = tu.lds;
    P.lds_flush_at = tu.flush_at;
    P.policy = tu.policy;
    P.no_lds = (opts->debug_flags & WC_DEBUG_NO_LDS) ? 1u : 0u;
    P.utf8 = opts->tokenizer == WC_TOKENIZE_UTF8 ? 1u : 0u;
    P.pad0 = 0;
    size_t dyn = (size_t)tu.lds * (per_doc ? 24 : 20);
    if (!L.spill) {
      if (tm.on) HIPCHK(hipEventRecord(tm.a, s));
      HIPCHK(launch_count(P, per_doc, grid, tu.block, dyn, s));
      if (tm.on) HIPCHK(hipEventRecord(tm.b, s));
    } else {
      GlobalParams G;
      memset(&G, 0, sizeof(G));
      G.corpus = d_corpus;
      G.len = corpus_len;
      G.offsets = d_offsets;
      G.n_docs = n_docs;
      G.table = L.table;
      G.mask = L.S - 1;
      G.occ_limit = occ_limit;
      G.key_mask = key_mask_of(opts);
      G.hdr = L.hdr;
      G.stage_doc = L.stage_doc;
      G.base_off = b0;
      G.n_stages = L.n_stages;
      G.stages_per_wg = L.spill_spw;
      G.map_grid = L.spill_grid;
      G.dict_cap = L.dict_cap;
      G.dict = L.dict;
      G.dict_part = L.dict_part;
      G.sample_table = L.sample_table;
      G.sample_hdr = L.sample_hdr;
      G.S = L.static_blocks;
      G.reduce_entries = kReduceLds;
      uint32_t pct = opts->tuning && opts->tuning->lds_load_pct ? opts->tuning->lds_load_pct : 100;
      pct = std::min<uint32_t>(std::max<uint32_t>(pct, 10), 100);
      G.reduce_cap = (uint32_t)((uint64_t)kReduceLds * pct / 100);
      G.arena = L.arena;
      G.fill = L.fill;
      HIPCHK(launch_fill_zero(L.fill, (uint64_t)kParts * L.static_blocks * 2, s));
      HIPCHK(launch_fill_zero(L.sample_table, kSampleSlots * sizeof(Slot), s));
      HIPCHK(launch_fill_zero(L.sample_hdr, sizeof(Header), s));
      HIPCHK(launch_fill_zero(L.dict, sizeof(DictImage), s));
      HIPCHK(launch_global(G, tm.on ? tm.a : nullptr, tm.on ? tm.b : nullptr, s));
    }
  }
  if (!(phases & kPhaseExport)) return WC_OK;

  ExportParams E;
  memset(&E, 0, sizeof(E));
  E.table = L.table;
  E.slots = L.S;
  E.hdr = L.hdr;
  E.block_sums = L.bsum;
  E.n_blocks = L.n_blocks;
  E.count_bytes = opts->count_bytes;
  E.count_bias = opts->debug_count_bias;
  E.per_doc = per_doc ? 1u : 0u;
  if (!per_doc) {
    E.word_offsets = L.woff;
    E.words = L.words;
    E.word_cap = L.word_cap;
    E.counts = L.counts;
    HIPCHK(launch_export(E, s));
  } else {
    E.word_cap = ~0ull;
    E.docs = L.list_docs;
    E.slot_of_entry = L.list_slots;
    HIPCHK(launch_export_list(E, s));
  }
  Header h;
  HIPCHK(hipMemcpyAsync(&h, L.hdr, sizeof(Header), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (h.flags & (kFlagBadOffsets | kFlagTableFull | kFlagStall)) return finish_flags(h);

  memset(out, 0, sizeof(*out));
  out->n_entries = h.n_entries;
  out->total_tokens = h.total_tokens;
  out->n_docs = n_docs;
  out->table_slots = L.S;
  out->count_bytes = opts->count_bytes;
  out->mode = opts->mode;
  out->d_word_offsets = L.woff;
  out->d_words = L.words;
  out->d_counts = L.counts;
  if (L.spill) memcpy(out->stats, h.stat, sizeof(out->stats));

  if (per_doc) {
    const uint64_t n = h.n_entries;
    // group entries by document (counting sort), then word offsets by a prefix sum of lengths
    HIPCHK(group_by_doc(L.list_docs, L.list_slots, n, n_docs, L.doc_ptr, L.doc_len, L.doc_fill,
                        L.sums, L.sorted_docs, L.sorted_slots, s));
    HIPCHK(launch_slot_lens(L.table, L.sorted_slots, n, L.lens, s));
    HIPCHK(excl_scan_u64(L.lens, L.woff, n + 1, L.sums, s));
    uint64_t wb = 0;
    HIPCHK(hipMemcpyAsync(&wb, L.woff + n, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (wb > L.word_cap) {
      out->word_bytes = wb;
      return WC_ENOMEM;
    }
    HIPCHK(launch_slot_write(L.table, L.sorted_slots, n, L.woff, L.words, L.counts,
                             opts->count_bytes, opts->debug_count_bias, L.docs, L.hdr, s));
    HIPCHK(hipMemcpyAsync(&h, L.hdr, sizeof(Header), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    h.word_bytes = wb;
    out->d_doc_ptr = L.doc_ptr;
    out->d_doc_len = L.doc_len;
    out->d_docs = L.docs;
  }
  out->word_bytes = h.word_bytes;
  if (tm.on) {
    HIPCHK(hipEventRecord(tm.d, s));
    HIPCHK(hipEventSynchronize(tm.d));
    float ms = 0;
    if (corpus_len && n_docs) {
      HIPCHK(hipEventElapsedTime(&ms, tm.a, tm.b));
      out->kernel_ms = ms;
    }
    HIPCHK(hipEventElapsedTime(&ms, tm.c, tm.d));
    out->total_ms = ms;
  }
  return finish_flags(h);
}

}  // namespace

extern "C" {

// ------------------------------------------------------------------------------------------
// merge
// ------------------------------------------------------------------------------------------
namespace {

struct MergeLayout {
  uint64_t S, n_blocks, word_cap, total;
  Header* hdr;
  Slot* table;
  uint64_t* bsum;
  uint64_t* woff;
  void* counts;
  uint8_t* words;
};

bool tables_ok(const wc_result* const* t, uint32_t k) {
  if (!t && k) return false;
  for (uint32_t i = 0; i < k; ++i) {
    if (!t[i]) return false;
    if (t[i]->count_bytes != 4 && t[i]->count_bytes != 8) return false;
    if (t[i]->n_entries && (!t[i]->d_word_offsets || !t[i]->d_counts || !t[i]->d_words))
      return false;
  }
  return true;
}

void layout_merge(const wc_result* const* t, uint32_t k, const wc_opts* o, void* ws,
                  MergeLayout* L) {
  uint64_t n = 0, wb = 0;
  for (uint32_t i = 0; i < k; ++i) {
    n += t[i]->n_entries;
    wb += t[i]->word_bytes;
  }
  uint64_t S = o && o->table_slots ? o->table_slots : next_pow2(std::max<uint64_t>(4096, 2 * n));
  L->S = S;
  L->n_blocks = (S + kExportSpan - 1) / kExportSpan;
  L->word_cap = std::max<uint64_t>(o && o->word_bytes_cap ? o->word_bytes_cap : wb, 16);
  uint32_t cb = o ? o->count_bytes : 8;
  Bump B(ws);
  L->hdr = B.take<Header>(sizeof(Header));
  L->table = B.take<Slot>(S * sizeof(Slot));
  L->bsum = B.take<uint64_t>(L->n_blocks * 16);
  L->woff = B.take<uint64_t>((S + 1) * 8);
  L->counts = B.take<uint8_t>(S * cb);
  L->words = B.take<uint8_t>(L->word_cap);
  L->total = B.off;
}

}  // namespace

wc_status wc_merge_plan(const wc_result* const* tables, uint32_t k, const wc_opts* opts,
                        wc_plan* out) {
  if (!out || !tables_ok(tables, k)) return WC_EINVAL;
  if (opts && (opts->count_bytes != 4 && opts->count_bytes != 8)) return WC_EINVAL;
  if (opts && opts->table_slots && !is_pow2(opts->table_slots)) return WC_EINVAL;
  MergeLayout L;
  layout_merge(tables, k, opts, nullptr, &L);
  out->table_slots = L.S;
  out->workspace_bytes = L.total;
  out->max_entries = L.S;
  out->word_bytes_cap = L.word_cap;
  return WC_OK;
}

wc_status wc_merge(const wc_result* const* tables, uint32_t k, const wc_opts* opts,
                   void* d_workspace, uint64_t workspace_bytes, wc_result* out, void* stream) {
  if (!out || !d_workspace || !tables_ok(tables, k)) return WC_EINVAL;
  if (opts && (opts->count_bytes != 4 && opts->count_bytes != 8)) return WC_EINVAL;
  if (opts && opts->table_slots && !is_pow2(opts->table_slots)) return WC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  MergeLayout L;
  layout_merge(tables, k, opts, d_workspace, &L);
  if (L.total > workspace_bytes) return WC_ENOMEM;
  const uint32_t cb = opts ? opts->count_bytes : 8;
  const uint64_t km = opts ? key_mask_of(opts) : ~0ull;
  Timer tm;
  HIPCHK(tm.init(opts && (opts->debug_flags & WC_DEBUG_TIME)));
  if (tm.on) HIPCHK(hipEventRecord(tm.c, s));
  HIPCHK(launch_fill_zero(L.hdr, sizeof(Header), s));
  HIPCHK(launch_fill_zero(L.table, L.S * sizeof(Slot), s));
  const uint64_t occ_limit = L.S - L.S / 8;
  if (tm.on) HIPCHK(hipEventRecord(tm.a, s));
  for (uint32_t i = 0; i < k; ++i) {
    MergeInput in;
    in.word_offsets = tables[i]->d_word_offsets;
    in.words = tables[i]->d_words;
    in.counts = tables[i]->d_counts;
    in.n = tables[i]->n_entries;
    in.count_bytes = tables[i]->count_bytes;
    in.column = 0;
    HIPCHK(launch_merge_insert(in, L.table, L.S - 1, occ_limit, km, L.hdr, nullptr, 1, s));
  }
  if (tm.on) HIPCHK(hipEventRecord(tm.b, s));
  ExportParams E;
  memset(&E, 0, sizeof(E));
  E.table = L.table;
  E.slots = L.S;
  E.hdr = L.hdr;
  E.block_sums = L.bsum;
  E.n_blocks = L.n_blocks;
  E.word_offsets = L.woff;
  E.words = L.words;
  E.word_cap = L.word_cap;
  E.counts = L.counts;
  E.count_bytes = cb;
  E.count_bias = opts ? opts->debug_count_bias : 0;
  HIPCHK(launch_export(E, s));
  Header h;
  HIPCHK(hipMemcpyAsync(&h, L.hdr, sizeof(Header), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  memset(out, 0, sizeof(*out));
  out->n_entries = h.n_entries;
  uint64_t total = 0;
  out->word_bytes = h.word_bytes;
  out->table_slots = L.S;
  out->count_bytes = cb;
  out->mode = WC_GLOBAL;
  out->d_word_offsets = L.woff;
  out->d_words = L.words;
  out->d_counts = L.counts;
  for (uint32_t i = 0; i < k; ++i) total += tables[i]->total_tokens;
  out->total_tokens = total;
  if (tm.on) {
    HIPCHK(hipEventRecord(tm.d, s));
    HIPCHK(hipEventSynchronize(tm.d));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, tm.a, tm.b));
    out->kernel_ms = ms;
    HIPCHK(hipEventElapsedTime(&ms, tm.c, tm.d));
    out->total_ms = ms;
  }
  return finish_flags(h);
}

// ------------------------------------------------------------------------------------------
// top-k distinctive words
// ------------------------------------------------------------------------------------------
namespace {

struct TopkLayout {
  uint64_t S, n_blocks, word_cap, row_word_cap, total;
  uint32_t C, k;
  Header* hdr;
  Slot* table;
  uint64_t* joint_slots;   // [S * C]
  uint64_t* bsum;
  uint64_t* woff;          // joint vocabulary
  uint64_t* entry_total;   // [S] int64 counts of the joint table
  uint8_t* words;
  uint64_t* slot_of_entry;
  uint64_t* joint_dense;   // [S * C]
  uint64_t* totals;        // [64]
  uint32_t* lists;
  uint32_t* list_len;
  uint64_t* out_entry;
  uint64_t* n_rows;        // [64]
  uint64_t* row_woff;
  uint8_t* row_words;
  uint64_t* row_nc;
  uint64_t* row_nr;
  double* row_score;
};

void layout_topk(const wc_result* const* t, uint32_t C, uint32_t k, void* ws, TopkLayout* L) {
  uint64_t n = 0, wb = 0;
  for (uint32_t i = 0; i < C; ++i) {
    n += t[i]->n_entries;
    wb += t[i]->word_bytes;
  }
  L->C = C;
  L->k = k;
  L->S = next_pow2(std::max<uint64_t>(4096, 2 * n));
  L->n_blocks = (L->S + kExportSpan - 1) / kExportSpan;
  L->word_cap = std::max<uint64_t>(wb, 16);
  L->row_word_cap = std::max<uint64_t>(std::min<uint64_t>(wb, (uint64_t)C * wb), 16);
  Bump B(ws);
  L->hdr = B.take<Header>(sizeof(Header));
  L->table = B.take<Slot>(L->S * sizeof(Slot));
  L->joint_slots = B.take<uint64_t>(L->S * C * 8);
  L->bsum = B.take<uint64_t>(L->n_blocks * 16);
  L->woff = B.take<uint64_t>((L->S + 1) * 8);
  L->entry_total = B.take<uint64_t>(L->S * 8);
  L->words = B.take<uint8_t>(L->word_cap);
  L->slot_of_entry = B.take<uint64_t>(L->S * 8);
  L->joint_dense = B.take<uint64_t>(L->S * C * 8);
  L->totals = B.take<uint64_t>(64 * 8);
  L->lists = B.take<uint32_t>((uint64_t)C * 2 * kTopkThreads * k * 4);
  L->list_len = B.take<uint32_t>((uint64_t)C * 2 * kTopkThreads * 4);
  L->out_entry = B.take<uint64_t>((uint64_t)C * k * 8);
  L->n_rows = B.take<uint64_t>(64 * 8);
  L->row_woff = B.take<uint64_t>(((uint64_t)C * k + 1) * 8);
  L->row_words = B.take<uint8_t>(L->row_word_cap * C);
  L->row_nc = B.take<uint64_t>((uint64_t)C * k * 8);
  L->row_nr = B.take<uint64_t>((uint64_t)C * k * 8);
  L->row_score = B.take<double>((uint64_t)C * k * 8);
  L->total = B.off;
}

__global__ void gather_joint_kernel(const uint64_t* joint_slots, const uint64_t* slot_of_entry,
                                    const Header* hdr, uint32_t C, uint64_t* dense) {
  uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (e >= hdr->n_entries) return;
  uint64_t i = slot_of_entry[e];
  for (uint32_t c = 0; c < C; ++c) dense[e * C + c] = joint_slots[i * C + c];
}

}  // namespace

wc_status wc_topk_ratio_plan(const wc_result* const* corpora, uint32_t n_corpora, uint32_t k,
                             uint64_t* workspace_bytes) {
  if (!workspace_bytes || n_corpora == 0 || n_corpora > 64 || k == 0 || k > 4096)
    return WC_EINVAL;
  if (!tables_ok(corpora, n_corpora)) return WC_EINVAL;
  TopkLayout L;
  layout_topk(corpora, n_corpora, k, nullptr, &L);
  *workspace_bytes = L.total;
  return WC_OK;
}

wc_status wc_topk_ratio(const wc_result* const* corpora, uint32_t n_corpora, uint32_t k,
                        uint64_t min_count, void* d_workspace, uint64_t workspace_bytes,
                        wc_topk* out, void* stream) {
  if (!out || !d_workspace || n_corpora == 0 || n_corpora > 64 || k == 0 || k > 4096)
    return WC_EINVAL;
  if (!tables_ok(corpora, n_corpora)) return WC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  TopkLayout L;
  layout_topk(corpora, n_corpora, k, d_workspace, &L);
  if (L.total > workspace_bytes) return WC_ENOMEM;
  const uint32_t C = n_corpora;
  HIPCHK(launch_fill_zero(L.hdr, sizeof(Header), s));
  HIPCHK(launch_fill_zero(L.table, L.S * sizeof(Slot), s));
  HIPCHK(launch_fill_zero(L.joint_slots, L.S * C * 8, s));
  HIPCHK(launch_fill_zero(L.totals, 64 * 8, s));
  const uint64_t occ_limit = L.S - L.S / 8;
  for (uint32_t c = 0; c < C; ++c) {
    MergeInput in;
    in.word_offsets = corpora[c]->d_word_offsets;
    in.words = corpora[c]->d_words;
    in.counts = corpora[c]->d_counts;
    in.n = corpora[c]->n_entries;
    in.count_bytes = corpora[c]->count_bytes;
    in.column = c;
    HIPCHK(launch_merge_insert(in, L.table, L.S - 1, occ_limit, ~0ull, L.hdr, L.joint_slots, C, s));
  }
  ExportParams E;
  memset(&E, 0, sizeof(E));
  E.table = L.table;
  E.slots = L.S;
  E.hdr = L.hdr;
  E.block_sums = L.bsum;
  E.n_blocks = L.n_blocks;
  E.word_offsets = L.woff;
  E.words = L.words;
  E.word_cap = L.word_cap;
  E.counts = L.entry_total;
  E.count_bytes = 8;
  E.slot_of_entry = L.slot_of_entry;
  HIPCHK(launch_export(E, s));
  uint32_t grid = (uint32_t)((L.S + 255) / 256);
  hipLaunchKernelGGL(gather_joint_kernel, dim3(grid), dim3(256), 0, s, L.joint_slots,
                     L.slot_of_entry, L.hdr, C, L.joint_dense);
  HIPCHK(hipGetLastError());
  Header h;
  HIPCHK(hipMemcpyAsync(&h, L.hdr, sizeof(Header), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (h.flags) return finish_flags(h);
  TopkParams P;
  P.word_offsets = L.woff;
  P.words = L.words;
  P.joint = L.joint_dense;
  P.V = h.n_entries;
  P.C = C;
  P.k = k;
  P.min_count = min_count;
  P.totals = L.totals;
  P.lists = L.lists;
  P.list_len = L.list_len;
  P.out_entry = L.out_entry;
  P.n_rows = L.n_rows;
  P.out_word_offsets = L.row_woff;
  P.out_words = L.row_words;
  P.out_nc = L.row_nc;
  P.out_nr = L.row_nr;
  P.out_score = L.row_score;
  P.entry_total = L.entry_total;
  HIPCHK(launch_topk(P, s));
  memset(out, 0, sizeof(*out));
  HIPCHK(hipMemcpyAsync(out->n_rows, L.n_rows, 8 * C, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&out->word_bytes, L.row_woff + (uint64_t)C * k, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  out->n_corpora = C;
  out->k = k;
  out->vocab_size = h.n_entries;
  out->d_word_offsets = L.row_woff;
  out->d_words = L.row_words;
  out->d_n_c = L.row_nc;
  out->d_n_rest = L.row_nr;
  out->d_score = L.row_score;
  return WC_OK;
}

wc_status wc_table_to_host(const wc_result* t, uint64_t* word_offsets, uint8_t* words,
                           void* counts) {
  if (!t) return WC_EINVAL;
  const uint64_t n = t->n_entries;
  if (word_offsets && t->d_word_offsets)
    HIPCHK(hipMemcpy(word_offsets, t->d_word_offsets, (n + 1) * 8, hipMemcpyDeviceToHost));
  if (words && t->word_bytes) {
    uint64_t b0 = 0;
    HIPCHK(hipMemcpy(&b0, t->d_word_offsets, 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(words, t->d_words + b0, t->word_bytes, hipMemcpyDeviceToHost));
  }
  if (counts && n) HIPCHK(hipMemcpy(counts, t->d_counts, n * t->count_bytes, hipMemcpyDeviceToHost));
  return WC_OK;
}

wc_status wc_hash_words(const uint8_t* d_bytes, const uint64_t* d_offsets, uint64_t n,
                        uint64_t* d_out, void* stream) {
  if (n && (!d_bytes || !d_offsets || !d_out)) return WC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(launch_hash_words(d_bytes, d_offsets, n, d_out, s));
  HIPCHK(hipStreamSynchronize(s));
  return WC_OK;
}

// ------------------------------------------------------------------------------------------
// batched per-document counting with a captured HIP graph
// ------------------------------------------------------------------------------------------
}  // extern "C"

struct wc_batch {
  wc_opts opts;
  wc_tuning tuning;
  uint64_t max_docs = 0, max_bytes = 0;
  DocLayout D;
  uint32_t lds = kDocLds, grid = 0;
  DocTask* h_task = nullptr;  // pinned
  Header* h_hdr = nullptr;    // pinned
  hipStream_t bs = nullptr;
  hipEvent_t ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

wc_status wc_batch_plan(const wc_opts* opts, uint64_t max_docs, uint64_t max_bytes,
                        uint64_t* workspace_bytes) {
  if (!opts_ok(opts) || !workspace_bytes || opts->mode != WC_PER_DOC) return WC_EINVAL;
  if (opts->tokenizer != WC_TOKENIZE_ASCII) return WC_EINVAL;  // the batch kernel reads ASCII
  if (max_bytes >= (1ull << 32)) return WC_EINVAL;
  Tune tu;
  if (!resolve_tuning(opts->tuning, &tu)) return WC_EINVAL;
  DocLayout D;
  layout_docs(max_bytes, max_docs, opts, nullptr, &D);
  *workspace_bytes = D.total;
  return WC_OK;
}

wc_status wc_batch_create(const wc_opts* opts, uint64_t max_docs, uint64_t max_bytes,
                          void* d_workspace, uint64_t workspace_bytes, wc_batch** out) {
  if (!out || !d_workspace) return WC_EINVAL;
  uint64_t need = 0;
  wc_status st = wc_batch_plan(opts, max_docs, max_bytes, &need);
  if (st != WC_OK) return st;
  if (workspace_bytes < need) return WC_ENOMEM;
  Tune tu;
  resolve_tuning(opts->tuning, &tu);
  HIPCHK(ensure_smem_attr());
  wc_batch* b = new wc_batch();
  b->opts = *opts;
  if (opts->tuning) {
    b->tuning = *opts->tuning;
    b->opts.tuning = &b->tuning;
  }
  b->max_docs = max_docs;
  b->max_bytes = max_bytes;
  layout_docs(max_bytes, max_docs, &b->opts, d_workspace, &b->D);
  b->lds = opts->tuning && opts->tuning->lds_entries ? tu.lds : kDocLds;
  b->grid = tu.grid ? tu.grid : (uint32_t)device_cus();
  hipError_t e = hipHostMalloc((void**)&b->h_task, sizeof(DocTask), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_hdr, sizeof(Header), hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->bs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    g_last_hip = (int32_t)e;
    wc_batch_destroy(b);
    return WC_EDEVICE;
  }
  *out = b;
  return WC_OK;
}

wc_status wc_batch_run(wc_batch* b, const uint8_t* d_corpus, uint64_t corpus_len,
                       const uint64_t* d_offsets, uint64_t n_docs, wc_result* out, void* stream) {
  if (!b || !out || !d_offsets || (corpus_len && !d_corpus)) return WC_EINVAL;
  if (corpus_len > b->max_bytes || n_docs > b->max_docs) return WC_EINVAL;
  hipStream_t cs = (hipStream_t)stream;
  // the caller's stream (where the corpus was produced) comes first
  HIPCHK(hipEventRecord(b->ev, cs));
  HIPCHK(hipStreamWaitEvent(b->bs, b->ev, 0));
  *b->h_task = DocTask{d_corpus, corpus_len, d_offsets, n_docs};
  if (!b->exec) {
    HIPCHK(hipStreamBeginCapture(b->bs, hipStreamCaptureModeThreadLocal));
    Tune tu;
    resolve_tuning(b->opts.tuning, &tu);
    DocParams P = doc_params(b->D, &b->opts, b->lds, tu.pct, tu.chunk, tu.direct_kib);
    hipError_t e = hipMemcpyAsync(b->D.task, b->h_task, sizeof(DocTask), hipMemcpyHostToDevice,
                                  b->bs);
    if (e == hipSuccess) e = launch_fill_zero(b->D.hdr, sizeof(Header), b->bs);
    if (e == hipSuccess) e = launch_docs(P, b->grid, doc_dyn(b->lds), b->bs);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->h_hdr, b->D.hdr, sizeof(Header), hipMemcpyDeviceToHost, b->bs);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->bs, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      if (g) hipGraphDestroy(g);
      b->exec = nullptr;
      g_last_hip = (int32_t)e;
      return WC_EDEVICE;
    }
    b->graph = g;
  }
  HIPCHK(hipGraphLaunch(b->exec, b->bs));
  HIPCHK(hipStreamSynchronize(b->bs));
  const Header& h = *b->h_hdr;
  memset(out, 0, sizeof(*out));
  out->n_entries = h.out_cursor >> 32;
  out->word_bytes = h.out_cursor & 0xffffffffull;
  out->total_tokens = h.total_tokens;
  out->n_docs = n_docs;
  out->table_slots = std::max<uint64_t>(h.arena_next, b->D.arena_slots);
  out->stats[3] = h.over_n;
  out->count_bytes = b->opts.count_bytes;
  out->mode = WC_PER_DOC;
  out->d_word_offsets = b->D.woff;
  out->d_words = b->D.words;
  out->d_counts = b->D.counts;
  out->d_doc_ptr = b->D.doc_ptr;
  out->d_doc_len = b->D.doc_len;
  out->d_docs = b->D.docs;
  return finish_flags(h);
}

wc_status wc_batch_destroy(wc_batch* b) {
  if (!b) return WC_OK;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->ev) hipEventDestroy(b->ev);
  if (b->bs) hipStreamDestroy(b->bs);
  if (b->h_task) hipHostFree(b->h_task);
  if (b->h_hdr) hipHostFree(b->h_hdr);
  delete b;
  return WC_OK;
}

// ------------------------------------------------------------------------------------------
// autotuner
// ------------------------------------------------------------------------------------------
}  // extern "C"

namespace {

std::vector<wc_tuning> tune_grid(const wc_opts* o) {
  std::vector<wc_tuning> g;
  if (o->mode == WC_PER_DOC) {
    // One point: 32 KiB work items, the full LDS table at the highest load. On a calibration
    // sample of a few thousand documents the second pass lasts as long as its largest
    // document, whatever else it counts, so the sample favours points that send more
    // documents there: it chose a smaller table and load (batched-100k 21.7 ms, nearly every
    // document counted twice instead of 8,400) or 16 KiB items (15.1 ms, 24,600) over this
    // point (13.1 ms); 64 KiB items overflow the default private-table arena.
    g.push_back(wc_tuning{0, 4096, 0, 0, 85, 32u << 10, 0});
  } else {
    // one-pass kernel: LDS entries x flush load x flush policy (the two-pass kernels, from
    // 256 MiB, take lds_entries as the dictionary size and ignore the rest)
    for (uint32_t lds : {2048u, 4096u})
      for (uint32_t pct : {60u, 75u, 90u})
        for (uint32_t pol : {WC_FLUSH_ALL, WC_FLUSH_BYPASS})
          g.push_back(wc_tuning{0, lds, pol, 0, pct, 0, 0});
  }
  return g;
}

}  // namespace

extern "C" {

wc_status wc_autotune_plan(uint64_t len, uint64_t n_docs, const wc_opts* opts,
                           uint64_t* workspace_bytes) {
  if (!opts_ok(opts) || !workspace_bytes) return WC_EINVAL;
  uint64_t need = 0;
  for (const wc_tuning& t : tune_grid(opts)) {
    wc_opts o = *opts;
    o.tuning = &t;
    if (o.mode == WC_PER_DOC) o.debug_flags |= WC_DEBUG_DOCS;  // the kernel the grid tunes
    wc_plan p;
    wc_status st = wc_count_plan(len, n_docs, &o, &p);
    if (st != WC_OK) return st;
    need = std::max<uint64_t>(need, p.workspace_bytes);
  }
  *workspace_bytes = need;
  return WC_OK;
}

wc_status wc_autotune(const uint8_t* d_sample, uint64_t len, const uint64_t* d_offsets,
                      uint64_t n_docs, const wc_opts* opts, void* d_workspace,
                      uint64_t workspace_bytes, wc_tuning* best, float* best_ms, void* stream) {
  if (!best || !opts_ok(opts)) return WC_EINVAL;
  float best_t = 3.4e38f;
  bool found = false;
  // times one point (two calls after a warm-up); false when it needs more room than planned.
  // (direct_kib keeps its default: on a calibration sample of a few thousand documents the
  // second pass's time is that of its largest document, whatever the size limit, and the
  // sample favoured sending every long document straight to it, which was slower on the
  // whole corpus.)
  auto try_point = [&](const wc_tuning& t, wc_status* err) -> bool {
    wc_opts o = *opts;
    o.tuning = &t;
    o.debug_flags |= WC_DEBUG_TIME;
    if (o.mode == WC_PER_DOC) o.debug_flags |= WC_DEBUG_DOCS;  // the kernel the grid tunes
    float ms = 0;
    wc_status st = WC_OK;
    for (int rep = 0; rep < 3 && st == WC_OK; ++rep) {  // first run warms up
      wc_result r;
      st = wc_count(d_sample, len, d_offsets, n_docs, &o, d_workspace, workspace_bytes, &r,
                    stream);
      if (rep) ms += r.total_ms;
    }
    if (st == WC_EDEVICE) *err = st;
    if (st != WC_OK) return false;  // a point that needs more room than planned is skipped
    if (ms < best_t) {
      best_t = ms;
      *best = t;
      found = true;
    }
    return true;
  };
  wc_status err = WC_OK;
  for (const wc_tuning& t : tune_grid(opts)) {
    try_point(t, &err);
    if (err != WC_OK) return err;
  }
  if (!found) return WC_ENOMEM;
  if (best_ms) *best_ms = best_t / 2;
  return WC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------
// dense reduce: the paper's zero-padded keys x documents matrix and a row-sum kernel
// ------------------------------------------------------------------------------------------
namespace {

struct DenseLayout {
  uint64_t S, n_blocks, word_cap, fixed, rows_cap;
  Header* hdr;
  Slot* table;
  uint64_t* bsum;
  uint64_t* slot_of_input;
  uint64_t* entry_of_slot;
  uint64_t* woff;
  void* counts;
  uint8_t* words;
  uint32_t* matrix;
};

bool dense_input_ok(const wc_result* t) {
  return t && t->mode == WC_PER_DOC && (t->count_bytes == 4 || t->count_bytes == 8) &&
         (!t->n_entries || (t->d_word_offsets && t->d_words && t->d_counts && t->d_docs));
}

// rows: matrix rows to lay out; ws_bytes (when ws is set): the matrix takes what is left
void layout_dense(const wc_result* t, const wc_opts* o, uint64_t rows, void* ws,
                  uint64_t ws_bytes, DenseLayout* L) {
  const uint64_t n = t->n_entries;
  uint64_t S = o && o->table_slots ? o->table_slots : next_pow2(std::max<uint64_t>(4096, 2 * n));
  L->S = S;
  L->n_blocks = (S + kExportSpan - 1) / kExportSpan;
  L->word_cap = std::max<uint64_t>(o && o->word_bytes_cap ? o->word_bytes_cap : t->word_bytes, 16);
  const uint32_t cb = o ? o->count_bytes : 8;
  Bump B(ws);
  L->hdr = B.take<Header>(sizeof(Header));
  L->table = B.take<Slot>(S * sizeof(Slot));
  L->bsum = B.take<uint64_t>(L->n_blocks * 16);
  L->slot_of_input = B.take<uint64_t>(std::max<uint64_t>(n, 1) * 8);
  L->entry_of_slot = B.take<uint64_t>(S * 8);
  L->woff = B.take<uint64_t>((S + 1) * 8);
  L->counts = B.take<uint8_t>(S * cb);
  L->words = B.take<uint8_t>(L->word_cap);
  L->fixed = B.off;
  L->matrix = B.take<uint32_t>(0);
  const uint64_t row_bytes = std::max<uint64_t>(t->n_docs, 1) * 4;
  L->rows_cap = ws ? (ws_bytes > L->fixed ? (ws_bytes - L->fixed) / row_bytes : 0) : rows;
  (void)rows;
}

}  // namespace

extern "C" {

wc_status wc_merge_dense_plan(const wc_result* per_doc, const wc_opts* opts, uint64_t rows,
                              uint64_t* workspace_bytes) {
  if (!workspace_bytes || !dense_input_ok(per_doc)) return WC_EINVAL;
  if (opts && (opts->count_bytes != 4 && opts->count_bytes != 8)) return WC_EINVAL;
  if (opts && opts->table_slots && !is_pow2(opts->table_slots)) return WC_EINVAL;
  DenseLayout L;
  if (!rows) rows = per_doc->n_entries;
  layout_dense(per_doc, opts, rows, nullptr, 0, &L);
  *workspace_bytes = L.fixed + rows * std::max<uint64_t>(per_doc->n_docs, 1) * 4;
  return WC_OK;
}

wc_status wc_merge_dense(const wc_result* per_doc, const wc_opts* opts, void* d_workspace,
                         uint64_t workspace_bytes, wc_result* out, void* stream) {
  if (!out || !d_workspace || !dense_input_ok(per_doc)) return WC_EINVAL;
  if (opts && (opts->count_bytes != 4 && opts->count_bytes != 8)) return WC_EINVAL;
  if (opts && opts->table_slots && !is_pow2(opts->table_slots)) return WC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  DenseLayout L;
  layout_dense(per_doc, opts, 0, d_workspace, workspace_bytes, &L);
  if (L.fixed > workspace_bytes) return WC_ENOMEM;
  const uint32_t cb = opts ? opts->count_bytes : 8;
  const uint64_t n_docs = per_doc->n_docs;
  Timer tm;
  HIPCHK(tm.init(opts && (opts->debug_flags & WC_DEBUG_TIME)));
  if (tm.on) HIPCHK(hipEventRecord(tm.c, s));
  HIPCHK(launch_fill_zero(L.hdr, sizeof(Header), s));
  HIPCHK(launch_fill_zero(L.table, L.S * sizeof(Slot), s));
  MergeInput in;
  in.word_offsets = per_doc->d_word_offsets;
  in.words = per_doc->d_words;
  in.counts = per_doc->d_counts;
  in.n = per_doc->n_entries;
  in.count_bytes = per_doc->count_bytes;
  in.column = 0;
  HIPCHK(launch_dense_keys(in, L.table, L.S - 1, L.S - L.S / 8, opts ? key_mask_of(opts) : ~0ull,
                           L.hdr, L.slot_of_input, s));
  ExportParams E;
  memset(&E, 0, sizeof(E));
  E.table = L.table;
  E.slots = L.S;
  E.hdr = L.hdr;
  E.block_sums = L.bsum;
  E.n_blocks = L.n_blocks;
  E.word_offsets = L.woff;
  E.words = L.words;
  E.word_cap = L.word_cap;
  E.counts = L.counts;
  E.count_bytes = cb;
  E.entry_of_slot = L.entry_of_slot;
  HIPCHK(launch_export(E, s));
  Header h;
  HIPCHK(hipMemcpyAsync(&h, L.hdr, sizeof(Header), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  memset(out, 0, sizeof(*out));
  if (h.flags) return finish_flags(h);
  const uint64_t V = h.n_entries;
  if (V > L.rows_cap) {
    out->n_entries = V;  // rows the matrix needs: plan again with them
    return WC_ENOMEM;
  }
  HIPCHK(launch_fill_zero(L.matrix, V * std::max<uint64_t>(n_docs, 1) * 4, s));
  HIPCHK(launch_dense_scatter(in.n, L.slot_of_input, L.entry_of_slot, per_doc->d_docs,
                              per_doc->d_counts, per_doc->count_bytes, n_docs, L.matrix, s));
  if (tm.on) HIPCHK(hipEventRecord(tm.a, s));
  HIPCHK(launch_dense_rowsum(L.matrix, V, n_docs, L.counts, cb,
                             opts ? opts->debug_count_bias : 0, L.hdr, s));
  if (tm.on) HIPCHK(hipEventRecord(tm.b, s));
  HIPCHK(hipMemcpyAsync(&h, L.hdr, sizeof(Header), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  out->n_entries = V;
  out->total_tokens = per_doc->total_tokens;
  out->word_bytes = h.word_bytes;
  out->table_slots = L.S;
  out->count_bytes = cb;
  out->mode = WC_GLOBAL;
  out->d_word_offsets = L.woff;
  out->d_words = L.words;
  out->d_counts = L.counts;
  if (tm.on) {
    HIPCHK(hipEventRecord(tm.d, s));
    HIPCHK(hipEventSynchronize(tm.d));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, tm.a, tm.b));
    out->kernel_ms = ms;
    HIPCHK(hipEventElapsedTime(&ms, tm.c, tm.d));
    out->total_ms = ms;
  }
  return finish_flags(h);
}

}  // extern "C"

// ------------------------------------------------------------------------------------------
// canonical order of a host copy of a table (comparisons; no device work)
// ------------------------------------------------------------------------------------------
extern "C" wc_status wc_sort_canonical(uint64_t n, const uint64_t* word_offsets,
                                       const uint8_t* words, const uint64_t* docs,
                                       uint64_t* perm) {
  if (n && (!word_offsets || !perm)) return WC_EINVAL;
  if (!n) return WC_OK;
  const uint64_t base = word_offsets[0];
  for (uint64_t e = 0; e < n; ++e)
    if (word_offsets[e + 1] < word_offsets[e]) return WC_EINVAL;
  if (word_offsets[n] > base && !words) return WC_EINVAL;
  std::vector<uint64_t> idx(n);
  for (uint64_t e = 0; e < n; ++e) idx[e] = e;
  std::sort(idx.begin(), idx.end(), [&](uint64_t a, uint64_t b) {
    if (docs && docs[a] != docs[b]) return docs[a] < docs[b];
    const uint64_t la = word_offsets[a + 1] - word_offsets[a];
    const uint64_t lb = word_offsets[b + 1] - word_offsets[b];
    const int c = memcmp(words + (word_offsets[a] - base), words + (word_offsets[b] - base),
                         la < lb ? la : lb);
    if (c) return c < 0;
    if (la != lb) return la < lb;  // a proper prefix first
    return a < b;
  });
  memcpy(perm, idx.data(), n * 8);
  return WC_OK;
}

// ------------------------------------------------------------------------------------------
// count from host memory: transfer pieces overlapped with the count of the pieces before
// ------------------------------------------------------------------------------------------
namespace {

constexpr uint64_t kMinPiece = 1ull << 20;

inline bool ascii_delimiter(uint8_t x) {
  if (x >= 0x80) return false;  // may belong to a UTF-8 sequence: not taken as a cut
  const uint8_t f = (x >= 'A' && x <= 'Z') ? (uint8_t)(x + 32) : x;
  return !((f >= 'a' && f <= 'z') || (f >= '0' && f <= '9') || f == '\'');
}

// Cut [R0, R1) into pieces of about `piece` bytes, each cut right after an ASCII delimiter
// byte (or at a document start), so that no token spans two pieces: every piece is then
// counted on its own into the same table. Reads only the bytes just after each target.
std::vector<uint64_t> plan_cuts(const uint8_t* h, const uint64_t* off, uint64_t n_docs,
                                uint64_t piece) {
  std::vector<uint64_t> cuts;
  const uint64_t R0 = off[0], R1 = off[n_docs];
  cuts.push_back(R0);
  uint64_t d = 0;  // next document start to look at
  while (cuts.back() < R1) {
    uint64_t c = cuts.back() + piece;
    if (c >= R1) {
      cuts.push_back(R1);
      break;
    }
    while (d <= n_docs && off[d] < c) ++d;
    const uint64_t next_doc = d <= n_docs ? off[d] : R1;
    while (c < next_doc && !ascii_delimiter(h[c - 1])) ++c;  // a token never spans a delimiter
    cuts.push_back(std::min(c, next_doc));
  }
  return cuts;
}

struct HostPieces {
  std::vector<uint64_t> cuts;     // piece p is [cuts[p], cuts[p+1])
  std::vector<uint64_t> first;    // offsets of piece p start at first[p] in `offs`
  std::vector<uint64_t> count;    // documents of piece p
  std::vector<uint64_t> offs;     // per piece: offsets relative to the piece start
  uint64_t max_len = 0, max_docs = 0;
};

void plan_pieces(const uint8_t* h, const uint64_t* off, uint64_t n_docs, uint64_t piece,
                 HostPieces* P) {
  P->cuts = plan_cuts(h, off, n_docs, piece);
  uint64_t d = 1;  // first document start after the current cut
  for (size_t p = 0; p + 1 < P->cuts.size(); ++p) {
    const uint64_t a = P->cuts[p], b = P->cuts[p + 1];
    P->first.push_back(P->offs.size());
    P->offs.push_back(0);
    while (d < n_docs && off[d] <= a) ++d;
    for (; d < n_docs && off[d] < b; ++d) P->offs.push_back(off[d] - a);
    P->offs.push_back(b - a);
    P->count.push_back(P->offs.size() - P->first.back() - 1);
    P->max_len = std::max(P->max_len, b - a);
    P->max_docs = std::max(P->max_docs, P->count.back());
  }
}

// Options of a count in pieces: the table is sized from the whole corpus (auto sizing would
// size it from one piece), and so are the exported word bytes.
wc_opts piece_opts(const wc_opts* o, uint64_t corpus_len) {
  wc_opts q = *o;
  q.debug_flags &= ~WC_DEBUG_TIME;
  if (!q.table_slots) {
    wc_plan p;
    if (wc_count_plan(corpus_len, 1, o, &p) == WC_OK) q.table_slots = p.table_slots;
  }
  if (!q.word_bytes_cap) {
    wc_plan p;
    if (wc_count_plan(corpus_len, 1, &q, &p) == WC_OK) q.word_bytes_cap = p.word_bytes_cap;
  }
  return q;
}

}  // namespace

extern "C" {

wc_status wc_count_host_plan(uint64_t corpus_len, uint64_t n_docs, const wc_opts* opts,
                             uint64_t piece_bytes, wc_plan* out) {
  if (!opts_ok(opts) || !out || opts->mode != WC_GLOBAL) return WC_EINVAL;
  const wc_opts q = piece_opts(opts, corpus_len);
  // any piece is at most piece_bytes + the longest run without a delimiter; the layout of the
  // whole corpus covers every piece's
  wc_status st = wc_count_plan(corpus_len, n_docs, &q, out);
  if (st != WC_OK) return st;
  const uint64_t n_pieces = corpus_len / std::max<uint64_t>(piece_bytes, kMinPiece) + 2;
  out->workspace_bytes += align_up((n_docs + 1 + 2 * n_pieces) * 8) + kAlign;
  return WC_OK;
}

wc_status wc_count_host(const uint8_t* h_corpus, uint64_t corpus_len, const uint64_t* h_offsets,
                        uint64_t n_docs, const wc_opts* opts, uint64_t piece_bytes,
                        uint8_t* d_text, void* d_workspace, uint64_t workspace_bytes,
                        wc_result* out, void* stream) {
  if (!opts_ok(opts) || !out || !d_workspace || !h_offsets || opts->mode != WC_GLOBAL)
    return WC_EINVAL;
  if (corpus_len && (!h_corpus || !d_text)) return WC_EINVAL;
  for (uint64_t d = 0; d < n_docs; ++d)
    if (h_offsets[d] > h_offsets[d + 1]) return WC_EINVAL;
  if (n_docs && h_offsets[n_docs] > corpus_len) return WC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(ensure_smem_attr());
  const wc_opts q = piece_opts(opts, corpus_len);
  Tune tu;
  if (!resolve_tuning(q.tuning, &tu)) return WC_EINVAL;
  HostPieces H;
  if (n_docs) plan_pieces(h_corpus, h_offsets, n_docs, std::max<uint64_t>(piece_bytes, kMinPiece), &H);
  // piece offset arrays at the end of the workspace, after the largest piece's layout
  CountLayout L0;
  global_stage(corpus_len, &q, &tu);
  if (!layout_count(corpus_len, std::max<uint64_t>(n_docs, 1), &q, tu, nullptr, nullptr, &L0))
    return WC_EDEVICE;
  const uint64_t off_at = align_up(L0.total + kAlign);
  if (off_at + H.offs.size() * 8 > workspace_bytes) return WC_ENOMEM;
  uint64_t* d_offs = (uint64_t*)((uint8_t*)d_workspace + off_at);
  if (!H.offs.empty())
    HIPCHK(hipMemcpyAsync(d_offs, H.offs.data(), H.offs.size() * 8, hipMemcpyHostToDevice, s));
  hipStream_t cs = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  std::vector<hipEvent_t> ev(H.count.size(), nullptr);
  wc_status st = WC_OK;
  hipError_t e = hipSuccess;
  CountLayout L;
  // the table is cleared before the first piece (also for an empty corpus)
  Tune t0 = tu;
  global_stage(H.max_len, &q, &t0);
  if (!layout_count(std::max<uint64_t>(H.max_len, 1), 1, &q, t0, d_text, d_workspace, &L))
    st = WC_EDEVICE;
  if (st == WC_OK) st = count_table(nullptr, 0, nullptr, 0, &q, t0, L, out, s, kPhaseClear);
  for (size_t p = 0; st == WC_OK && e == hipSuccess && p < H.count.size(); ++p) {
    const uint64_t a = H.cuts[p], n = H.cuts[p + 1] - a;
    e = hipEventCreateWithFlags(&ev[p], hipEventDisableTiming);
    if (e == hipSuccess && n) e = hipMemcpyAsync(d_text + a, h_corpus + a, n, hipMemcpyHostToDevice, cs);
    if (e == hipSuccess) e = hipEventRecord(ev[p], cs);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, ev[p], 0);
    if (e != hipSuccess) break;
    Tune tp = tu;
    global_stage(n, &q, &tp);
    CountLayout Lp;
    if (!layout_count(n, H.count[p], &q, tp, d_text + a, d_workspace, &Lp)) {
      st = WC_EDEVICE;
      break;
    }
    if (Lp.total > off_at || Lp.table != L.table || Lp.hdr != L.hdr) {
      st = WC_ENOMEM;
      break;
    }
    st = count_table(d_text + a, n, d_offs + H.first[p], H.count[p], &q, tp, Lp, out, s,
                     kPhaseCount);
  }
  if (e == hipSuccess && st == WC_OK)
    st = count_table(nullptr, 0, nullptr, 0, &q, t0, L, out, s, kPhaseExport);
  hipError_t e2 = hipStreamSynchronize(cs);
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  (void)hipStreamDestroy(cs);
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) {
    g_last_hip = (int32_t)e;
    return WC_EDEVICE;
  }
  if (st == WC_OK) out->n_docs = n_docs;
  return st;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------
// allocation-free count: wc_count's one-pass global table in a static device array
// ------------------------------------------------------------------------------------------
namespace {

constexpr uint64_t kStaticScratchBytes = 34ull << 20;
constexpr uint64_t kStaticMaxSlots = 1ull << 20;  // 32 MiB of table
constexpr int kMaxDevices = 64;

// Header, table, per-stage document cursor and export block sums of wc_count_static. One copy
// per GPU, loaded with the library and held until the process ends; host code reaches it only
// through the address hipGetSymbolAddress gives on each device.
__device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
hipError_t scratch_addr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

wc_status wc_count_static(const uint8_t* d_corpus, uint64_t corpus_len, const uint64_t* d_offsets,
                          uint64_t n_docs, const wc_opts* opts, uint64_t* d_word_offsets,
                          void* d_counts, uint64_t max_entries, uint8_t* d_words,
                          uint64_t word_bytes_cap, wc_result* out, void* stream) {
  if (!opts_ok(opts) || !out || !d_offsets || !d_word_offsets || !d_counts || !d_words)
    return WC_EINVAL;
  if (corpus_len && !d_corpus) return WC_EINVAL;
  if (opts->mode != WC_GLOBAL || (opts->debug_flags & WC_DEBUG_SPILL)) return WC_EINVAL;
  if (opts->table_slots > kStaticMaxSlots) return WC_ENOMEM;
  wc_opts o = *opts;
  o.debug_flags = (o.debug_flags | WC_DEBUG_DIRECT) & ~WC_DEBUG_TIME;  // one-pass, no events
  if (!o.table_slots) {
    wc_plan p;
    wc_status st = wc_count_plan(corpus_len, n_docs, &o, &p);
    if (st != WC_OK) return st;
    o.table_slots = std::min<uint64_t>(p.table_slots, kStaticMaxSlots);
  }
  Tune tu;
  if (!resolve_tuning(o.tuning, &tu)) return WC_EINVAL;
  global_stage(corpus_len, &o, &tu);
  if (max_entries < o.table_slots) return WC_ENOMEM;
  OutBufs ob{d_word_offsets, d_counts, d_words, word_bytes_cap};
  CountLayout L;
  if (!layout_count(corpus_len, n_docs, &o, tu, d_corpus, nullptr, &L, &ob)) return WC_EDEVICE;
  if (L.total > kStaticScratchBytes) return WC_ENOMEM;  // the stage cursor of a huge corpus
  void* base = nullptr;
  HIPCHK(scratch_addr(&base));
  if (!layout_count(corpus_len, n_docs, &o, tu, d_corpus, base, &L, &ob)) return WC_EDEVICE;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(ensure_smem_attr());
  // count_table clears the header and the table (fill kernels) before counting
  return count_table(d_corpus, corpus_len, d_offsets, n_docs, &o, tu, L, out, s);
}

}  // extern "C"

namespace wc {
// the calling thread's last HIP error, for entry points defined in other files
void set_last_hip(int32_t e) { g_last_hip = e; }
}  // namespace wc
