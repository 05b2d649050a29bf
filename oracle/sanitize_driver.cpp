// Exercises the oracle's entry points under AddressSanitizer / UBSan (built by
// tests/test_oracle_sanitize.py). Test infrastructure only.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

extern "C" {
void* oracle_count(const uint8_t*, uint64_t, const uint64_t*, uint64_t, int);
void* oracle_merge(uint32_t, const uint8_t* const*, const uint64_t* const*,
                   const uint64_t* const*, const uint64_t*);
uint64_t oracle_table_size(void*);
uint64_t oracle_table_total(void*);
uint64_t oracle_table_word_bytes(void*);
void oracle_table_export(void*, uint8_t*, uint64_t*, uint64_t*, uint64_t*);
void oracle_table_free(void*);
uint64_t oracle_topk_ratio(uint32_t, const uint8_t* const*, const uint64_t* const*,
                           const uint64_t* const*, const uint64_t*, uint32_t, uint64_t,
                           uint64_t*, uint64_t*, uint64_t*, double*, uint64_t*, uint64_t*,
                           uint8_t*);
}

struct Exported {
  std::vector<uint8_t> words;
  std::vector<uint64_t> offs, cnts, docs;
};

static Exported take(void* h) {
  Exported e;
  uint64_t n = oracle_table_size(h), wb = oracle_table_word_bytes(h);
  e.words.resize(wb + 1);
  e.offs.resize(n + 1);
  e.cnts.resize(n + 1);
  e.docs.resize(n + 1);
  oracle_table_export(h, e.words.data(), e.offs.data(), e.cnts.data(), e.docs.data());
  e.cnts.resize(n);
  oracle_table_free(h);
  return e;
}

int main() {
  const char* a = "I want to test MapReduce";
  const char* b = "MapReduce is a cool algorithm to test. Dog dog. (Applause) x";
  std::string text = std::string(a) + b;
  std::vector<uint64_t> off = {0, strlen(a), text.size()};
  void* h = oracle_count((const uint8_t*)text.data(), text.size(), off.data(), 2, 0);
  if (!h) return 2;
  Exported g = take(h);
  void* hp = oracle_count((const uint8_t*)text.data(), text.size(), off.data(), 2, 1);
  Exported pd = take(hp);
  const uint8_t* W[2] = {g.words.data(), pd.words.data()};
  const uint64_t* O[2] = {g.offs.data(), pd.offs.data()};
  const uint64_t* C[2] = {g.cnts.data(), pd.cnts.data()};
  uint64_t N[2] = {g.cnts.size(), pd.cnts.size()};
  Exported m = take(oracle_merge(2, W, O, C, N));
  std::vector<uint64_t> ow(2 * 5), onc(2 * 5), onr(2 * 5), rows(2), joff(64);
  std::vector<double> sc(2 * 5);
  std::vector<uint8_t> jw(512);
  uint64_t V = oracle_topk_ratio(2, W, O, C, N, 5, 1, ow.data(), onc.data(), onr.data(), sc.data(),
                                 rows.data(), joff.data(), jw.data());
  // invalid offsets are rejected
  std::vector<uint64_t> bad = {0, 5, 3};
  if (oracle_count((const uint8_t*)text.data(), text.size(), bad.data(), 2, 0)) return 3;
  // empty corpus
  Exported z = take(oracle_count(nullptr, 0, off.data(), 0, 0));
  std::printf("entries %zu merged %zu vocab %llu empty %zu\n", g.cnts.size(), m.cnts.size(),
              (unsigned long long)V, z.cnts.size());
  return (g.cnts.size() == m.cnts.size() && z.cnts.empty()) ? 0 : 4;
}
