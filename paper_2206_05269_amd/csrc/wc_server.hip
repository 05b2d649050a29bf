// Serving: a request loop that counts texts as they arrive, keeps the resulting tables
// resident on the device and answers merge queries (Section 3.3's summation of grouped counts,
// across requests).
//
// Admission. The server owns one device pool of `mem_budget` bytes; the policy (count memory
// from the low end, resident tables from the high end, when to wait and when to fail) is the
// host-only wc::Admission of wc_admission.h. A request is admitted when the memory its count
// needs (text, offsets, workspace) is free; until then it waits in arrival order. Results are
// compacted into an exact-size resident block, and the count memory is returned at once.
//
// Continuous batching. `max_streams` worker threads each own a HIP stream (default priority),
// so admitted requests run concurrently on the device. A worker that takes a small
// single-document request also takes the small single-document requests queued right behind
// it (up to kPackDocs requests / kPackBytes bytes) and counts them in one per-document launch,
// then splits the per-document tables into one resident table per request.
//
// Uploads. Each worker owns two pinned host buffers: it copies a request's text into one while
// the other is on its way to the device, so host copies of several workers and their DMA
// transfers overlap (a copy straight from pageable memory goes through the runtime's own
// staging, one transfer at a time).
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "wc_admission.h"
#include "wc_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr uint32_t kPackDocs = 64;
constexpr uint64_t kPackBytes = 4ull << 20;
constexpr uint64_t kSmallBytes = 1ull << 20;
constexpr uint64_t kStageBytes = 8ull << 20;  // per pinned upload buffer (two per worker)

struct Request {
  uint64_t id = 0;
  std::vector<uint8_t> text;      // host copy (host input)
  const uint8_t* dev_text = nullptr;
  const uint8_t* host_text = nullptr;  // caller's host memory, read in place (not copied)
  uint64_t len = 0;
  std::vector<uint64_t> offsets;
  wc_opts opts{};
  wc_tuning tuning{};
  bool merge = false;
  std::vector<uint64_t> merge_ids;
  // state
  std::vector<std::shared_ptr<Request>> merge_inputs;  // pinned at submission
  int state = 0;  // 0 queued, 1 running, 2 done
  wc_status status = WC_EAGAIN;
  uint8_t* resident = nullptr;
  wc::ResidentLife life;  // merges reading the resident table; released by the client
  wc_result res{};
  double t_submit = 0, t_start = 0, t_done = 0;
};

double now_s() {
  return std::chrono::duration<double>(Clock::now().time_since_epoch()).count();
}

}  // namespace

struct wc_server {
  int device = 0;
  uint64_t budget = 0;
  uint8_t* pool_mem = nullptr;
  wc::Admission adm;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_mem;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> reqs;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  struct Staging {
    uint8_t* buf[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool used[2] = {false, false};
    uint32_t next = 0;
    uint64_t* small = nullptr;  // pinned: a few values read back from the device
    unsigned long long* d_small = nullptr;  // device: per-request token totals of a group
  };
  std::vector<Staging> staging;  // one per worker
  uint64_t next_id = 1;
  bool stop = false;
  std::atomic<uint64_t> launches{0};
};

namespace {

// compact a table (device arrays) into one resident block: [word_offsets | counts | words]
// d[i] = s[i] - s[0] for i < n1: a table's word offsets rebased to its first word
__global__ void rebase_offsets_kernel(const uint64_t* src, uint64_t n1, uint64_t* dst) {
  const uint64_t b0 = src[0];
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n1;
       i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i] - b0;
}

// *out += sum of n counts (4 or 8 bytes each); integer, so the order of additions is free
__global__ void sum_counts_kernel(const void* counts, uint32_t cb, uint64_t n,
                                  unsigned long long* out) {
  unsigned long long v = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    v += cb == 4 ? (unsigned long long)((const int32_t*)counts)[i]
                 : (unsigned long long)((const int64_t*)counts)[i];
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(out, v);
}

uint32_t small_grid(uint64_t n) {
  const uint64_t g = (n + 255) / 256;
  return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(g, 1), 1024);
}

// Copy entries [e_begin, e_begin + n) of table t into an exact-size resident block. Only the
// byte range of their words crosses to the host (two values); offsets are rebased and counts
// and words copied on the device.
wc_status keep_resident(wc_server* S, wc_server::Staging& W, hipStream_t s, const wc_result& t,
                        uint64_t e_begin, uint64_t n, Request* R) {
  const uint32_t cb = t.count_bytes;
  if (hipMemcpyAsync(&W.small[0], t.d_word_offsets + e_begin, 8, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(&W.small[1], t.d_word_offsets + e_begin + n, 8, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return WC_EDEVICE;
  const uint64_t b0 = W.small[0], nb = W.small[1] - W.small[0];
  const uint64_t bytes = (n + 1) * 8 + n * cb + nb + 64;
  uint8_t* mem = nullptr;
  {
    // This worker holds count memory; the policy (wc::Admission::try_resident) lets it wait
    // only while another holder that is not itself waiting here can still return memory.
    std::unique_lock<std::mutex> lk(S->mu);
    uint64_t off = 0;
    wc::Admit a;
    while ((a = S->adm.try_resident(bytes, &off)) == wc::Admit::kWait && !S->stop) {
      ++S->adm.resident_waiters;
      S->cv_mem.wait(lk);
      --S->adm.resident_waiters;
    }
    if (a != wc::Admit::kGranted) return WC_ENOMEM;
    mem = S->pool_mem + off;
  }
  uint64_t* d_off = (uint64_t*)mem;
  uint8_t* d_cnt = mem + (((n + 1) * 8 + 15) & ~15ull);
  uint8_t* d_words = d_cnt + ((n * cb + 15) & ~15ull);
  hipLaunchKernelGGL(rebase_offsets_kernel, dim3(small_grid(n + 1)), dim3(256), 0, s,
                     (const uint64_t*)(t.d_word_offsets + e_begin), n + 1, d_off);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && n)
    e = hipMemcpyAsync(d_cnt, (const uint8_t*)t.d_counts + e_begin * cb, n * cb,
                       hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && nb)
    e = hipMemcpyAsync(d_words, t.d_words + b0, nb, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->adm.free_resident((uint64_t)(mem - S->pool_mem));
    S->cv_mem.notify_all();
    return WC_EDEVICE;
  }
  R->resident = mem;
  memset(&R->res, 0, sizeof(R->res));
  R->res.n_entries = n;
  R->res.word_bytes = nb;
  R->res.count_bytes = cb;
  R->res.mode = WC_GLOBAL;
  R->res.n_docs = 1;
  R->res.d_word_offsets = d_off;
  R->res.d_words = d_words;
  R->res.d_counts = d_cnt;
  return WC_OK;
}

// Take count memory for a request (wc::Admission::try_count): wait while other requests
// hold count memory (they will return it); when none does, the memory is held by resident
// tables, which only the client can release, so the request fails with WC_ENOMEM.
uint8_t* pool_alloc_wait(wc_server* S, uint64_t bytes) {
  std::unique_lock<std::mutex> lk(S->mu);
  uint64_t off = 0;
  wc::Admit a;
  while ((a = S->adm.try_count(bytes, &off)) == wc::Admit::kWait && !S->stop) S->cv_mem.wait(lk);
  return a == wc::Admit::kGranted ? S->pool_mem + off : nullptr;
}

void pool_free(wc_server* S, uint8_t* p) {
  std::lock_guard<std::mutex> lk(S->mu);
  S->adm.free_count((uint64_t)(p - S->pool_mem));
  S->cv_mem.notify_all();
}

// Free a resident table (under the lock).
void free_resident_locked(wc_server* S, Request* R) {
  if (R->resident) S->adm.free_resident((uint64_t)(R->resident - S->pool_mem));
  R->resident = nullptr;
  S->cv_mem.notify_all();
}

// A merge is done with its inputs: a released input whose last reader this was is freed.
void unpin_inputs(wc_server* S, Request* M) {
  std::lock_guard<std::mutex> lk(S->mu);
  for (auto& in : M->merge_inputs)
    if (in->life.unpin()) free_resident_locked(S, in.get());
  M->merge_inputs.clear();
}

void finish(wc_server* S, Request* R, wc_status st) {
  std::lock_guard<std::mutex> lk(S->mu);
  R->status = st;
  R->state = 2;
  R->t_done = now_s();
  R->text.clear();
  R->text.shrink_to_fit();
  S->cv_done.notify_all();
}

// Count a group of requests. One request: its own wc_count (its opts). Several small
// single-document requests: one per-document count, split per request.
// Host text to device memory through the worker's two pinned buffers, in order on stream s.
hipError_t upload(wc_server::Staging& W, uint8_t* dst, const uint8_t* src, uint64_t n,
                  hipStream_t s) {
  for (uint64_t off = 0; off < n; off += kStageBytes, W.next ^= 1) {
    const uint32_t k = W.next;  // alternates across calls too: small texts overlap as well
    const uint64_t m = std::min<uint64_t>(kStageBytes, n - off);
    if (W.used[k]) {
      hipError_t e = hipEventSynchronize(W.ev[k]);  // its previous transfer has finished
      if (e != hipSuccess) return e;
    }
    memcpy(W.buf[k], src + off, m);
    hipError_t e = hipMemcpyAsync(dst + off, W.buf[k], m, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(W.ev[k], s);
    if (e != hipSuccess) return e;
    W.used[k] = true;
  }
  return hipSuccess;
}

void run_group(wc_server* S, int idx, std::vector<std::shared_ptr<Request>>& G) {
  hipStream_t s = S->streams[idx];
  const double t0 = now_s();
  for (auto& r : G) r->t_start = t0;
  if (G.size() == 1 && G[0]->merge) {
    Request* R = G[0].get();
    // The inputs were pinned when the merge was submitted (a release defers freeing their
    // resident tables until this merge is done); they were submitted before it, so they are
    // running or done: wait for them.
    std::vector<const wc_result*> ins;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (auto& in : R->merge_inputs) {
        S->cv_done.wait(lk, [&] { return in->state == 2; });
        if (in->status != WC_OK) {
          ins.clear();
          break;
        }
        ins.push_back(&in->res);
      }
    }
    wc_status st = ins.empty() ? WC_EINVAL : WC_OK;
    wc_opts o = R->opts;
    wc_plan p;
    if (st == WC_OK) st = wc_merge_plan(ins.data(), (uint32_t)ins.size(), &o, &p);
    uint8_t* ws = nullptr;
    if (st == WC_OK && !(ws = pool_alloc_wait(S, p.workspace_bytes))) st = WC_ENOMEM;
    if (st == WC_OK) {
      wc_result t;
      st = wc_merge(ins.data(), (uint32_t)ins.size(), &o, ws, p.workspace_bytes, &t, s);
      S->launches++;
      if (st == WC_OK) st = keep_resident(S, S->staging[idx], s, t, 0, t.n_entries, R);
      if (st == WC_OK) R->res.total_tokens = t.total_tokens;
    }
    if (ws) pool_free(S, ws);
    unpin_inputs(S, R);  // the merge's stream is synchronised: nothing reads the inputs now
    return finish(S, R, st);
  }
  // stage the texts on the device (one buffer for the group)
  uint64_t total = 0;
  for (auto& r : G) total += r->len;
  const bool packed = G.size() > 1;
  uint64_t n_docs_all = 0;
  for (auto& r : G) n_docs_all += packed ? 1 : r->offsets.size() - 1;
  wc_opts o = G[0]->opts;
  if (packed) {
    o.mode = WC_PER_DOC;
    o.tuning = nullptr;
    o.table_slots = 0;
    o.word_bytes_cap = 0;
  }
  wc_status st = WC_OK;
  for (int attempt = 0; attempt < 8; ++attempt) {
    wc_plan p;
    st = wc_count_plan(total, n_docs_all, &o, &p);
    if (st != WC_OK) break;
    if (packed && !(o.debug_flags & WC_DEBUG_DOCS) && p.workspace_bytes > S->budget / 4) {
      // the one-pass (document, word) table needs about 12 bytes per text byte; under a
      // tight budget the document-centric kernel (a fraction of that) is counted instead
      o.debug_flags |= WC_DEBUG_DOCS;
      st = wc_count_plan(total, n_docs_all, &o, &p);
      if (st != WC_OK) break;
    }
    const uint64_t off_bytes = (n_docs_all + 1) * 8;
    const uint64_t need = p.workspace_bytes + ((total + 255) & ~255ull) + off_bytes + 512;
    if (need > S->budget) {
      st = WC_ENOMEM;
      break;
    }
    uint8_t* mem = pool_alloc_wait(S, need);
    if (!mem) {
      st = WC_ENOMEM;
      break;
    }
    uint8_t* d_text = mem;
    uint64_t* d_off = (uint64_t*)(mem + ((total + 255) & ~255ull));
    uint8_t* ws = (uint8_t*)d_off + ((off_bytes + 255) & ~255ull);
    std::vector<uint64_t> off;
    off.reserve(n_docs_all + 1);
    uint64_t pos = 0;
    hipError_t e = hipSuccess;
    for (auto& r : G) {
      if (r->dev_text) e = hipMemcpyAsync(d_text + pos, r->dev_text, r->len, hipMemcpyDeviceToDevice, s);
      else if (r->host_text && r->len)  // in place: pinned memory goes straight to the DMA engine
        e = hipMemcpyAsync(d_text + pos, r->host_text, r->len, hipMemcpyHostToDevice, s);
      else if (r->len) e = upload(S->staging[idx], d_text + pos, r->text.data(), r->len, s);
      if (e != hipSuccess) break;
      if (packed) {
        off.push_back(pos);
      } else {
        for (size_t i = 0; i + 1 < r->offsets.size(); ++i) off.push_back(pos + r->offsets[i]);
      }
      pos += r->len;
    }
    if (packed) off.push_back(pos);
    else off.push_back(pos - G[0]->len + G[0]->offsets.back());
    if (e == hipSuccess) e = hipMemcpyAsync(d_off, off.data(), off_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
      pool_free(S, mem);
      st = WC_EDEVICE;
      break;
    }
    wc_result t;
    st = wc_count(d_text, total, d_off, n_docs_all, &o, ws, p.workspace_bytes, &t, s);
    S->launches++;
    if (st == WC_ETABLEFULL) {  // a global or (document, word) table: twice the slots
      o.table_slots = 2 * p.table_slots;
      pool_free(S, mem);
      continue;
    }
    if (st == WC_ENOMEM && !(t.word_bytes <= p.word_bytes_cap && t.table_slots <= p.table_slots)) {
      o.word_bytes_cap = std::max<uint64_t>(t.word_bytes, 3 * t.n_entries) * 5 / 4 + 4096;
      if (o.mode == WC_PER_DOC && t.table_slots > p.table_slots) {
        uint64_t want = 1;
        while (want < 2 * t.table_slots) want <<= 1;
        o.table_slots = want;
      }
      pool_free(S, mem);
      continue;
    }
    if (st == WC_OK) {
      if (!packed) {
        st = keep_resident(S, S->staging[idx], s, t, 0, t.n_entries, G[0].get());
        if (st == WC_OK) G[0]->res.total_tokens = t.total_tokens;
      } else {
        std::vector<uint64_t> dptr(n_docs_all), dlen(n_docs_all);
        e = hipMemcpyAsync(dptr.data(), t.d_doc_ptr, n_docs_all * 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
          e = hipMemcpyAsync(dlen.data(), t.d_doc_len, n_docs_all * 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = WC_EDEVICE;
        for (size_t i = 0; st == WC_OK && i < G.size(); ++i) {
          wc_status si = keep_resident(S, S->staging[idx], s, t, dptr[i], dlen[i], G[i].get());
          if (si != WC_OK) st = si;
        }
        // token totals per request: sum of its counts, on the device, read back together
        wc_server::Staging& W = S->staging[idx];
        if (st == WC_OK) {
          e = hipMemsetAsync(W.d_small, 0, G.size() * 8, s);
          for (size_t i = 0; e == hipSuccess && i < G.size(); ++i) {
            const Request* R = G[i].get();
            if (!R->res.n_entries) continue;
            hipLaunchKernelGGL(sum_counts_kernel, dim3(small_grid(R->res.n_entries)), dim3(256), 0,
                               s, R->res.d_counts, R->res.count_bytes, R->res.n_entries,
                               W.d_small + i);
            e = hipGetLastError();
          }
          if (e == hipSuccess)
            e = hipMemcpyAsync(W.small, W.d_small, G.size() * 8, hipMemcpyDeviceToHost, s);
          if (e == hipSuccess) e = hipStreamSynchronize(s);
          if (e != hipSuccess) st = WC_EDEVICE;
          for (size_t i = 0; st == WC_OK && i < G.size(); ++i) G[i]->res.total_tokens = W.small[i];
        }
      }
    }
    pool_free(S, mem);
    break;
  }
  for (auto& r : G) finish(S, r.get(), st);
}

void release_staging(wc_server* S) {
  for (auto& W : S->staging) {
    for (int k = 0; k < 2; ++k) {
      if (W.ev[k]) (void)hipEventSynchronize(W.ev[k]);
      if (W.ev[k]) (void)hipEventDestroy(W.ev[k]);
      if (W.buf[k]) (void)hipHostFree(W.buf[k]);
      W.ev[k] = nullptr;
      W.buf[k] = nullptr;
    }
    if (W.small) (void)hipHostFree(W.small);
    if (W.d_small) (void)hipFree(W.d_small);
    W.small = nullptr;
    W.d_small = nullptr;
  }
}

void worker(wc_server* S, int idx) {
  hipSetDevice(S->device);
  while (true) {
    std::vector<std::shared_ptr<Request>> G;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
      if (S->stop && S->queue.empty()) return;
      auto first = S->queue.front();
      S->queue.pop_front();
      first->state = 1;
      G.push_back(first);
      auto small = [](const Request& r) {
        return !r.merge && r.offsets.size() == 2 && r.offsets[0] == 0 && r.offsets[1] == r.len &&
               r.len <= kSmallBytes;
      };
      if (small(*first)) {
        uint64_t bytes = first->len;
        while (!S->queue.empty() && G.size() < kPackDocs) {
          auto& nx = S->queue.front();
          if (!small(*nx) || bytes + nx->len > kPackBytes ||
              nx->opts.count_bytes != first->opts.count_bytes ||
              nx->opts.debug_hash_bits != first->opts.debug_hash_bits)
            break;
          bytes += nx->len;
          nx->state = 1;
          G.push_back(nx);
          S->queue.pop_front();
        }
      }
    }
    run_group(S, idx, G);
  }
}

}  // namespace

extern "C" {

wc_status wc_server_create(int device, uint64_t mem_budget, uint32_t max_streams,
                           wc_server** out) {
  if (!out || mem_budget < (1ull << 20) || max_streams == 0 || max_streams > 16) return WC_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return WC_EDEVICE;
  wc_server* S = new wc_server();
  S->device = device;
  S->budget = mem_budget;
  if (hipMalloc((void**)&S->pool_mem, mem_budget) != hipSuccess) {
    delete S;
    return WC_ENOMEM;
  }
  S->adm.init(mem_budget);
  for (uint32_t i = 0; i < max_streams; ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : S->streams) hipStreamDestroy(x);
      hipFree(S->pool_mem);
      delete S;
      return WC_EDEVICE;
    }
    S->streams.push_back(s);
  }
  S->staging.resize(max_streams);
  for (auto& W : S->staging) {
    for (int k = 0; k < 2; ++k) {
      if (hipHostMalloc((void**)&W.buf[k], kStageBytes, hipHostMallocDefault) != hipSuccess ||
          hipEventCreateWithFlags(&W.ev[k], hipEventDisableTiming) != hipSuccess ||
          (k == 0 && (hipHostMalloc((void**)&W.small, kPackDocs * 8, hipHostMallocDefault) !=
                          hipSuccess ||
                      hipMalloc((void**)&W.d_small, kPackDocs * 8) != hipSuccess))) {
        release_staging(S);
        for (auto x : S->streams) hipStreamDestroy(x);
        hipFree(S->pool_mem);
        delete S;
        return WC_EDEVICE;
      }
    }
  }
  for (uint32_t i = 0; i < max_streams; ++i) S->workers.emplace_back(worker, S, (int)i);
  *out = S;
  return WC_OK;
}

wc_status wc_server_submit(wc_server* S, const uint8_t* text, uint64_t len,
                           const uint64_t* offsets, uint64_t n_docs, int text_on_device,
                           const wc_opts* opts, uint64_t* req_id) {
  if (!S || !req_id || !opts || (len && !text) || !offsets) return WC_EINVAL;
  if (text_on_device != WC_TEXT_HOST_COPY && text_on_device != WC_TEXT_DEVICE &&
      text_on_device != WC_TEXT_HOST_IN_PLACE)
    return WC_EINVAL;
  if (opts->count_bytes != 4 && opts->count_bytes != 8) return WC_EINVAL;
  if (opts->mode != WC_GLOBAL) return WC_EINVAL;  // per-request tables are global tables
  for (uint64_t i = 0; i < n_docs; ++i)
    if (offsets[i] > offsets[i + 1]) return WC_EINVAL;
  if (offsets[n_docs] > len) return WC_EINVAL;
  // admission test: the request must fit the budget on its own
  wc_plan p;
  wc_opts o = *opts;
  o.tuning = nullptr;
  wc_status st = wc_count_plan(len, n_docs, &o, &p);
  if (st != WC_OK) return st;
  if (p.workspace_bytes + len + (n_docs + 1) * 8 + 1024 > S->budget) return WC_ENOMEM;
  auto R = std::make_shared<Request>();
  R->len = len;
  if (text_on_device == WC_TEXT_DEVICE) R->dev_text = text;
  else if (text_on_device == WC_TEXT_HOST_IN_PLACE) R->host_text = text;
  else R->text.assign(text, text + len);
  R->offsets.assign(offsets, offsets + n_docs + 1);
  R->opts = o;
  R->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    R->id = S->next_id++;
    S->reqs[R->id] = R;
    S->queue.push_back(R);
    *req_id = R->id;
  }
  S->cv_work.notify_one();
  return WC_OK;
}

wc_status wc_server_poll(wc_server* S, uint64_t id, wc_result* out) {
  if (!S || !out) return WC_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return WC_EINVAL;
  if (it->second->state != 2) return WC_EAGAIN;
  *out = it->second->res;
  return it->second->status;
}

wc_status wc_server_wait(wc_server* S, uint64_t id, wc_result* out) {
  if (!S || !out) return WC_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return WC_EINVAL;
  auto R = it->second;
  S->cv_done.wait(lk, [&] { return R->state == 2; });
  *out = R->res;
  return R->status;
}

wc_status wc_server_times(wc_server* S, uint64_t id, double* submit_s, double* start_s,
                          double* done_s) {
  if (!S) return WC_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return WC_EINVAL;
  if (submit_s) *submit_s = it->second->t_submit;
  if (start_s) *start_s = it->second->t_start;
  if (done_s) *done_s = it->second->t_done;
  return it->second->state == 2 ? WC_OK : WC_EAGAIN;
}

wc_status wc_server_merge(wc_server* S, const uint64_t* ids, uint32_t k, const wc_opts* opts,
                          uint64_t* new_id) {
  if (!S || !new_id || !ids || k == 0) return WC_EINVAL;
  if (opts && opts->count_bytes != 4 && opts->count_bytes != 8) return WC_EINVAL;
  auto R = std::make_shared<Request>();
  R->merge = true;
  R->merge_ids.assign(ids, ids + k);
  wc_opts o{};
  o.count_bytes = opts ? opts->count_bytes : 8;
  R->opts = o;
  R->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    // pin the inputs now: releasing one before the merge has read it defers the free
    for (uint32_t i = 0; i < k; ++i) {
      auto it = S->reqs.find(ids[i]);
      if (it == S->reqs.end()) return WC_EINVAL;  // nothing pinned yet
      R->merge_inputs.push_back(it->second);
    }
    for (auto& in : R->merge_inputs) in->life.pin();
    R->id = S->next_id++;
    S->reqs[R->id] = R;
    S->queue.push_back(R);
    *new_id = R->id;
  }
  S->cv_work.notify_one();
  return WC_OK;
}

wc_status wc_server_release(wc_server* S, uint64_t id) {
  if (!S) return WC_EINVAL;
  std::shared_ptr<Request> R;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return WC_EINVAL;
    R = it->second;
    S->cv_done.wait(lk, [&] { return R->state == 2; });
    auto again = S->reqs.find(id);  // the wait may have let another thread in
    if (again == S->reqs.end() || again->second != R) return WC_EINVAL;
    S->reqs.erase(again);
    // a merge that will read the table frees it when done (ResidentLife)
    if (R->life.release()) free_resident_locked(S, R.get());
  }
  return WC_OK;
}

uint64_t wc_server_launches(wc_server* S) { return S ? S->launches.load() : 0; }

wc_status wc_server_destroy(wc_server* S) {
  if (!S) return WC_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  S->cv_mem.notify_all();
  for (auto& t : S->workers) t.join();
  release_staging(S);
  for (auto s : S->streams) hipStreamDestroy(s);
  hipFree(S->pool_mem);
  delete S;
  return WC_OK;
}

}  // extern "C"
