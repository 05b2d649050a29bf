// The paper's CPU design of the count, as a timed baseline beside the GPU counter. TEST AND
// BENCHMARK INFRASTRUCTURE ONLY (the benchmark's CPU legs and the tests call it; the product
// path never does); it shares no code with the GPU library.
//
// Section 3.1 maps on CPU threads, each counting its share of the text in its own dictionary;
// Section 3.2 reduces the dictionaries into one. Here the share of a thread is a byte range
// of the corpus (so one long document is split too), with the ownership rule of the GPU
// counter: a token belongs to the range holding its first byte, and its owner reads past the
// range end to finish it. The reduce is parallel as well: thread t sums the words whose hash
// falls in part t of every thread's dictionary. Tokeniser as in wc_oracle.cpp (ASCII fold,
// word bytes [a-z0-9'], documents end tokens).
#include <algorithm>
#include <chrono>
#include <cstdint>
#include <functional>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

inline uint8_t fold_b(uint8_t x) { return (x >= 'A' && x <= 'Z') ? uint8_t(x + 32) : x; }
inline bool word_b(uint8_t x) {
  const uint8_t f = fold_b(x);
  return (f >= 'a' && f <= 'z') || (f >= '0' && f <= '9') || f == '\'';
}

using Dict = std::unordered_map<std::string, uint64_t>;

struct Counted {
  std::vector<Dict> parts;  // the reduced table, split by hash into parts
  uint64_t total = 0;
  double seconds = 0;
};

// Count the tokens that start in [a, b) of the corpus (documents from offsets) into d.
uint64_t count_range(const uint8_t* t, const uint64_t* off, uint64_t n_docs, uint64_t a,
                     uint64_t b, Dict& d) {
  // first document containing a: the last offset <= a
  uint64_t k = (uint64_t)(std::upper_bound(off, off + n_docs + 1, a) - off);
  k = k ? k - 1 : 0;
  uint64_t tokens = 0;
  std::string w;
  uint64_t i = std::max(a, off[0]);
  while (i < b && k < n_docs) {
    const uint64_t d0 = off[k], d1 = off[k + 1];
    if (i >= d1) {
      ++k;
      continue;
    }
    if (i < d0) i = d0;
    if (i >= b) break;
    // skip to a token start inside this document: a word byte at the document start or
    // after a non-word byte
    if (word_b(t[i]) && (i == d0 || !word_b(t[i - 1]))) {
      uint64_t j = i;
      w.clear();
      while (j < d1 && word_b(t[j])) w.push_back((char)fold_b(t[j++]));
      ++d[w];
      ++tokens;
      i = j;
    } else {
      ++i;
    }
  }
  return tokens;
}

}  // namespace

extern "C" {

// Count with `threads` threads; returns a handle (free with cpu_parallel_free).
void* cpu_parallel_count(const uint8_t* text, uint64_t len, const uint64_t* offsets,
                         uint64_t n_docs, uint32_t threads) {
  (void)len;
  auto* C = new Counted();
  if (threads == 0) threads = 1;
  const auto t0 = std::chrono::steady_clock::now();
  const uint64_t lo = n_docs ? offsets[0] : 0, hi = n_docs ? offsets[n_docs] : 0;
  std::vector<Dict> local(threads);
  std::vector<uint64_t> tok(threads, 0);
  {
    std::vector<std::thread> th;
    for (uint32_t t = 0; t < threads; ++t) {
      const uint64_t a = lo + (hi - lo) * t / threads, b = lo + (hi - lo) * (t + 1) / threads;
      th.emplace_back([&, t, a, b] { tok[t] = count_range(text, offsets, n_docs, a, b, local[t]); });
    }
    for (auto& x : th) x.join();
  }
  C->parts.resize(threads);
  {
    std::vector<std::thread> th;
    for (uint32_t p = 0; p < threads; ++p) {
      th.emplace_back([&, p] {
        std::hash<std::string> hs;
        Dict& out = C->parts[p];
        for (uint32_t t = 0; t < threads; ++t)
          for (auto& kv : local[t])
            if (hs(kv.first) % threads == p) out[kv.first] += kv.second;
      });
    }
    for (auto& x : th) x.join();
  }
  for (uint32_t t = 0; t < threads; ++t) C->total += tok[t];
  C->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return C;
}

uint64_t cpu_parallel_size(void* h) {
  uint64_t n = 0;
  for (auto& p : ((Counted*)h)->parts) n += p.size();
  return n;
}
uint64_t cpu_parallel_total(void* h) { return ((Counted*)h)->total; }
double cpu_parallel_seconds(void* h) { return ((Counted*)h)->seconds; }
uint64_t cpu_parallel_word_bytes(void* h) {
  uint64_t n = 0;
  for (auto& p : ((Counted*)h)->parts)
    for (auto& kv : p) n += kv.first.size();
  return n;
}
// words (concatenated, in no particular order), offsets[n + 1], counts[n]
void cpu_parallel_export(void* h, uint8_t* words, uint64_t* offsets, uint64_t* counts) {
  uint64_t e = 0, pos = 0;
  offsets[0] = 0;
  for (auto& p : ((Counted*)h)->parts)
    for (auto& kv : p) {
      std::copy(kv.first.begin(), kv.first.end(), words + pos);
      pos += kv.first.size();
      counts[e] = kv.second;
      offsets[++e] = pos;
    }
}
void cpu_parallel_free(void* h) { delete (Counted*)h; }

}  // extern "C"
