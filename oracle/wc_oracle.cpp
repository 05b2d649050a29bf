// Word-frequency oracle: a plain, single-threaded CPU implementation of what the GPU counter
// computes. TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
// baseline call it; the product path never does. It shares no code with the GPU library.
//
// What it computes (the paper, "MapReduce for Counting Word Frequencies with MPI and GPUs"):
//  * Section 2 and Section 3.1: text is lower-cased and punctuation removed so that "Dog" and
//    "dog." are one word, then split into words; Section 3.1 / 3.2: each document's words are
//    counted in a dictionary, adding counts while the dictionary is populated.
//  * Section 3.3: per-document counts of one word are grouped and summed, e.g. a word seen
//    10, 4 and 3 times in three documents totals 17 (merge = pointwise sum over the union).
//  * Section 4.3: words that distinguish one corpus (one president's speeches) from the rest.
// Tokeniser reading used throughout (the paper deletes punctuation before splitting; this
// counter treats every byte outside the word alphabet as a delimiter, which agrees with the
// paper on text whose punctuation only separates words):
//  * fold(x) = x + 32 for 'A'..'Z', else x (ASCII only);
//  * a byte is a word byte when fold(x) is in 'a'..'z', '0'..'9' or '\'';
//  * a token is a maximal run of word bytes inside one document; its word is the folded run.
// Document d is bytes [offsets[d], offsets[d+1]); document boundaries always end a token.
// Canonical order (for comparison only): (document, word bytes) ascending, unsigned bytewise.
//
// Distinctive-word ranking (Section 4.3 compares presidents by eye; the ranking below is the
// reading this counter uses): over C corpora with joint vocabulary V (the union), for corpus
// c and word w with n_c(w) >= min_count, n_R(w) = sum of the other corpora's counts; rank by
// (n_c + 1) / (n_R + 1) descending (exact, by 128-bit cross products), ties by n_c descending,
// then word ascending. score = ((n_c + 1) / (N_c + V)) / ((n_R + 1) / (N_R + V)) as a double,
// N_c = total tokens of corpus c, N_R = total tokens of the other corpora.

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

namespace {

inline uint8_t fold(uint8_t x) { return (x >= 'A' && x <= 'Z') ? uint8_t(x + 32) : x; }

inline bool is_word_byte(uint8_t x) {
  uint8_t f = fold(x);
  return (f >= 'a' && f <= 'z') || (f >= '0' && f <= '9') || f == '\'';
}

struct Entry {
  uint64_t doc;
  std::string word;
  uint64_t count;
};

struct Table {
  std::vector<Entry> entries;  // canonical order
  uint64_t total = 0;          // tokens
  uint64_t word_bytes = 0;     // sum of word lengths over entries
};

bool entry_less(const Entry& a, const Entry& b) {
  if (a.doc != b.doc) return a.doc < b.doc;
  return a.word < b.word;  // std::string compares as unsigned char, a prefix sorts first
}

Table from_maps(std::vector<std::unordered_map<std::string, uint64_t>>& maps, uint64_t total) {
  Table t;
  t.total = total;
  for (size_t d = 0; d < maps.size(); ++d)
    for (auto& kv : maps[d]) {
      t.entries.push_back(Entry{d, kv.first, kv.second});
      t.word_bytes += kv.first.size();
    }
  std::sort(t.entries.begin(), t.entries.end(), entry_less);
  return t;
}

// ---- UTF-8 mode (the "other languages" of Section 5.2) ---------------------------------------
// Reading used: a document is decoded as UTF-8 (the well-formed byte sequences of the Unicode
// Standard, Table 3-7); a byte that does not belong to a well-formed sequence inside the
// document is a delimiter. A code point below U+0080 is classified as in ASCII mode; a
// higher one is a word character unless it is in U+0080..U+00BF (Latin-1 controls,
// punctuation and symbols), U+00D7, U+00F7, U+2000..U+206F (general punctuation),
// U+3000..U+303F (CJK symbols and punctuation) or U+FEFF. Folding stays ASCII-only; the
// word is the folded run of bytes.
bool is_word_cp(uint32_t cp) {
  if (cp < 0x80) return is_word_byte((uint8_t)cp);
  if (cp <= 0xBF || cp == 0xD7 || cp == 0xF7 || cp == 0xFEFF) return false;
  if (cp >= 0x2000 && cp <= 0x206F) return false;
  if (cp >= 0x3000 && cp <= 0x303F) return false;
  return true;
}

// Length (1..4) and code point of the well-formed sequence starting at t[i] within [i, end),
// or 0 when the byte at i does not start one.
int utf8_seq(const uint8_t* t, uint64_t i, uint64_t end, uint32_t* cp) {
  const uint8_t b = t[i];
  if (b < 0x80) {
    *cp = b;
    return 1;
  }
  int n;
  uint8_t lo = 0x80, hi = 0xBF;  // allowed range of the second byte
  uint32_t v;
  if (b >= 0xC2 && b <= 0xDF) {
    n = 2;
    v = b & 0x1F;
  } else if (b >= 0xE0 && b <= 0xEF) {
    n = 3;
    v = b & 0x0F;
    if (b == 0xE0) lo = 0xA0;
    if (b == 0xED) hi = 0x9F;
  } else if (b >= 0xF0 && b <= 0xF4) {
    n = 4;
    v = b & 0x07;
    if (b == 0xF0) lo = 0x90;
    if (b == 0xF4) hi = 0x8F;
  } else {
    return 0;
  }
  if (i + n > end) return 0;
  for (int k = 1; k < n; ++k) {
    const uint8_t c = t[i + k];
    const uint8_t l = k == 1 ? lo : 0x80, h = k == 1 ? hi : 0xBF;
    if (c < l || c > h) return 0;
    v = (v << 6) | (c & 0x3F);
  }
  *cp = v;
  return n;
}

bool offsets_valid(uint64_t len, const uint64_t* off, uint64_t n_docs) {
  if (n_docs > 0 && off == nullptr) return false;
  if (n_docs == 0) return true;
  for (uint64_t d = 0; d < n_docs; ++d)
    if (off[d] > off[d + 1]) return false;
  return off[n_docs] <= len;
}

}  // namespace

extern "C" {

// Count words. per_doc = 0: one table over all documents (doc field 0); 1: one table per
// document. Returns a handle (>0) or 0 when offsets are invalid (non-decreasing offsets,
// offsets[n_docs] <= len are required). text may be null when len == 0.
void* oracle_count(const uint8_t* text, uint64_t len, const uint64_t* offsets, uint64_t n_docs,
                   int per_doc) {
  if (!offsets_valid(len, offsets, n_docs)) return nullptr;
  std::vector<std::unordered_map<std::string, uint64_t>> maps(per_doc ? n_docs : 1);
  uint64_t total = 0;
  for (uint64_t d = 0; d < n_docs; ++d) {
    auto& m = maps[per_doc ? d : 0];
    uint64_t i = offsets[d], end = offsets[d + 1];
    while (i < end) {
      if (!is_word_byte(text[i])) { ++i; continue; }
      std::string w;
      while (i < end && is_word_byte(text[i])) w.push_back(char(fold(text[i++])));
      m[w] += 1;
      ++total;
    }
  }
  return new Table(from_maps(maps, total));
}

// Count words as oracle_count, with the UTF-8 reading above: each document is decoded, the
// bytes of its word code points are word bytes, every other byte a delimiter.
void* oracle_count_utf8(const uint8_t* text, uint64_t len, const uint64_t* offsets,
                        uint64_t n_docs, int per_doc) {
  if (!offsets_valid(len, offsets, n_docs)) return nullptr;
  std::vector<std::unordered_map<std::string, uint64_t>> maps(per_doc ? n_docs : 1);
  uint64_t total = 0;
  std::vector<uint8_t> word;
  for (uint64_t d = 0; d < n_docs; ++d) {
    auto& m = maps[per_doc ? d : 0];
    const uint64_t a = offsets[d], end = offsets[d + 1];
    word.assign(end - a, 0);
    for (uint64_t i = a; i < end;) {
      uint32_t cp = 0;
      const int n = utf8_seq(text, i, end, &cp);
      if (n == 0) {  // not part of a well-formed sequence: a delimiter
        ++i;
        continue;
      }
      const uint8_t wb = is_word_cp(cp) ? 1 : 0;
      for (int k = 0; k < n; ++k) word[i - a + k] = wb;
      i += n;
    }
    for (uint64_t i = a; i < end;) {
      if (!word[i - a]) {
        ++i;
        continue;
      }
      std::string w;
      while (i < end && word[i - a]) w.push_back(char(fold(text[i++])));
      m[w] += 1;
      ++total;
    }
  }
  return new Table(from_maps(maps, total));
}

// Merge k tables given as arrays (words concatenated, word_offsets[n+1], counts[n]): the
// result is one table (doc 0) holding the pointwise sum over the union of words.
void* oracle_merge(uint32_t k, const uint8_t* const* words, const uint64_t* const* word_offsets,
                   const uint64_t* const* counts, const uint64_t* n_entries) {
  std::vector<std::unordered_map<std::string, uint64_t>> maps(1);
  uint64_t total = 0;
  for (uint32_t t = 0; t < k; ++t)
    for (uint64_t e = 0; e < n_entries[t]; ++e) {
      std::string w(reinterpret_cast<const char*>(words[t]) + word_offsets[t][e],
                    word_offsets[t][e + 1] - word_offsets[t][e]);
      maps[0][w] += counts[t][e];
      total += counts[t][e];
    }
  return new Table(from_maps(maps, total));
}

uint64_t oracle_table_size(void* h) { return static_cast<Table*>(h)->entries.size(); }
uint64_t oracle_table_total(void* h) { return static_cast<Table*>(h)->total; }
uint64_t oracle_table_word_bytes(void* h) { return static_cast<Table*>(h)->word_bytes; }

// Export in canonical order into caller buffers: words[word_bytes], word_offsets[n+1],
// counts[n], docs[n] (docs may be null).
void oracle_table_export(void* h, uint8_t* words, uint64_t* word_offsets, uint64_t* counts,
                         uint64_t* docs) {
  const Table* t = static_cast<Table*>(h);
  uint64_t pos = 0;
  for (size_t e = 0; e < t->entries.size(); ++e) {
    const Entry& x = t->entries[e];
    word_offsets[e] = pos;
    if (!x.word.empty()) std::memcpy(words + pos, x.word.data(), x.word.size());
    pos += x.word.size();
    counts[e] = x.count;
    if (docs) docs[e] = x.doc;
  }
  word_offsets[t->entries.size()] = pos;
}

void oracle_table_free(void* h) { delete static_cast<Table*>(h); }

// Per-corpus distinctive words (see the header comment for the ranking). Inputs: c tables as
// arrays. Output rows (corpus-major, at most k per corpus): index into the joint vocabulary
// sorted by word (joint_word_offsets / joint_words give the words), n_c, n_R, score; n_rows[c]
// rows are written for corpus c at out + c*k. Returns the joint vocabulary size V, and fills
// joint_* when those buffers are non-null (sizes: V+1 offsets, sum of lengths bytes).
uint64_t oracle_topk_ratio(uint32_t c, const uint8_t* const* words,
                           const uint64_t* const* word_offsets, const uint64_t* const* counts,
                           const uint64_t* n_entries, uint32_t k, uint64_t min_count,
                           uint64_t* out_word, uint64_t* out_nc, uint64_t* out_nr,
                           double* out_score, uint64_t* n_rows, uint64_t* joint_word_offsets,
                           uint8_t* joint_words) {
  std::unordered_map<std::string, std::vector<uint64_t>> joint;
  std::vector<uint64_t> N(c, 0);
  for (uint32_t t = 0; t < c; ++t)
    for (uint64_t e = 0; e < n_entries[t]; ++e) {
      std::string w(reinterpret_cast<const char*>(words[t]) + word_offsets[t][e],
                    word_offsets[t][e + 1] - word_offsets[t][e]);
      auto it = joint.find(w);
      if (it == joint.end()) it = joint.emplace(w, std::vector<uint64_t>(c, 0)).first;
      it->second[t] += counts[t][e];
      N[t] += counts[t][e];
    }
  std::vector<std::pair<std::string, std::vector<uint64_t>>> vocab(joint.begin(), joint.end());
  std::sort(vocab.begin(), vocab.end(),
            [](const auto& a, const auto& b) { return a.first < b.first; });
  const uint64_t V = vocab.size();
  uint64_t Nall = 0;
  for (uint32_t t = 0; t < c; ++t) Nall += N[t];
  for (uint32_t t = 0; t < c; ++t) {
    std::vector<uint64_t> cand;
    for (uint64_t i = 0; i < V; ++i)
      if (vocab[i].second[t] >= min_count && vocab[i].second[t] > 0) cand.push_back(i);
    auto n_rest = [&](uint64_t i) {
      uint64_t s = 0;
      for (uint32_t u = 0; u < c; ++u)
        if (u != t) s += vocab[i].second[u];
      return s;
    };
    std::sort(cand.begin(), cand.end(), [&](uint64_t a, uint64_t b) {
      unsigned __int128 na = vocab[a].second[t], nb = vocab[b].second[t];
      unsigned __int128 ra = n_rest(a), rb = n_rest(b);
      unsigned __int128 lhs = (na + 1) * (rb + 1), rhs = (nb + 1) * (ra + 1);
      if (lhs != rhs) return lhs > rhs;
      if (na != nb) return na > nb;
      return vocab[a].first < vocab[b].first;
    });
    uint64_t rows = std::min<uint64_t>(k, cand.size());
    n_rows[t] = rows;
    const double Nc = double(N[t]), Nr = double(Nall - N[t]), Vd = double(V);
    for (uint64_t r = 0; r < rows; ++r) {
      uint64_t i = cand[r];
      uint64_t nc = vocab[i].second[t], nr = n_rest(i);
      out_word[uint64_t(t) * k + r] = i;
      out_nc[uint64_t(t) * k + r] = nc;
      out_nr[uint64_t(t) * k + r] = nr;
      out_score[uint64_t(t) * k + r] =
          ((double(nc) + 1.0) / (Nc + Vd)) / ((double(nr) + 1.0) / (Nr + Vd));
    }
  }
  if (joint_word_offsets) {
    uint64_t pos = 0;
    for (uint64_t i = 0; i < V; ++i) {
      joint_word_offsets[i] = pos;
      if (joint_words && !vocab[i].first.empty())
        std::memcpy(joint_words + pos, vocab[i].first.data(), vocab[i].first.size());
      pos += vocab[i].first.size();
    }
    joint_word_offsets[V] = pos;
  }
  return V;
}

// Joint vocabulary byte total, to size joint_words before oracle_topk_ratio fills it.
uint64_t oracle_joint_word_bytes(uint32_t c, const uint8_t* const* words,
                                 const uint64_t* const* word_offsets, const uint64_t* n_entries) {
  std::unordered_map<std::string, int> seen;
  uint64_t bytes = 0;
  for (uint32_t t = 0; t < c; ++t)
    for (uint64_t e = 0; e < n_entries[t]; ++e) {
      std::string w(reinterpret_cast<const char*>(words[t]) + word_offsets[t][e],
                    word_offsets[t][e + 1] - word_offsets[t][e]);
      if (seen.emplace(w, 1).second) bytes += w.size();
    }
  return bytes;
}

}  // extern "C"
