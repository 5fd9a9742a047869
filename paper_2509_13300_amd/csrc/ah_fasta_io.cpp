// FASTA text -> records, on the host (the bytes come from storage through
// host memory in any case).  The tool's input is genomes in FASTA
// (Section 2.1); each record is its own linear sequence, and a genome of
// several contigs is several records (windows never cross records).  The
// text is cut at line starts into parts read by concurrent threads: a count
// pass, an exclusive prefix over the parts, and a copy pass that writes the
// sequence bytes without line breaks, ready for ah_pack_genomes.
#include <algorithm>
#include <cstring>
#include <thread>
#include <vector>

#include "ah.h"
#include "ah_internal.h"

namespace {

struct Part {
  uint64_t beg = 0, end = 0;     // [beg, end) of the text, starting at a line start
  uint64_t records = 0, seq = 0;  // counted in the first pass
  uint64_t rec0 = 0, seq0 = 0;    // prefix over the parts
  bool lead = false;              // sequence bytes before the part's first header line
};

inline bool is_break(char c) { return c == '\n' || c == '\r' || c == ' ' || c == '\t'; }

// Walks [beg, end) line by line.  on_header(name_beg, name_end) for a '>'
// line; on_seq(p, n) for each run of sequence bytes (line breaks and blanks
// removed).
template <class H, class S>
void walk(const char* t, uint64_t beg, uint64_t end, H on_header, S on_seq) {
  uint64_t i = beg;
  while (i < end) {
    const char* nl = (const char*)memchr(t + i, '\n', end - i);
    const uint64_t le = nl ? (uint64_t)(nl - t) : end;  // line end (exclusive)
    if (t[i] == '>') {
      uint64_t ne = le;
      while (ne > i + 1 && is_break(t[ne - 1])) --ne;
      on_header(i + 1, ne);
    } else {
      uint64_t a = i;
      while (a < le) {
        while (a < le && is_break(t[a])) ++a;
        uint64_t b = a;
        while (b < le && !is_break(t[b])) ++b;
        if (b > a) on_seq(a, b - a);
        a = b;
      }
    }
    i = le + 1;
  }
}

std::vector<Part> cut(const char* t, uint64_t bytes, unsigned threads) {
  std::vector<Part> parts;
  const uint64_t step = std::max<uint64_t>(1, bytes / std::max(1u, threads));
  uint64_t at = 0;
  while (at < bytes) {
    uint64_t e = std::min(bytes, at + step);
    if (e < bytes) {  // extend to the next line start
      const char* nl = (const char*)memchr(t + e, '\n', bytes - e);
      e = nl ? (uint64_t)(nl - t) + 1 : bytes;
    }
    Part p;
    p.beg = at;
    p.end = e;
    parts.push_back(p);
    at = e;
  }
  return parts;
}

unsigned reader_threads() {
  const unsigned hw = std::thread::hardware_concurrency();
  return std::max(1u, std::min(hw ? hw : 1u, 16u));
}

void count_parts(const char* t, std::vector<Part>& parts) {
  std::vector<std::thread> th;
  for (Part& p : parts)
    th.emplace_back([t, &p] {
      bool seen_header = false;
      walk(
          t, p.beg, p.end,
          [&](uint64_t, uint64_t) {
            ++p.records;
            seen_header = true;
          },
          [&](uint64_t, uint64_t n) {
            p.seq += n;
            if (!seen_header) p.lead = true;
          });
    });
  for (auto& x : th) x.join();
  uint64_t r = 0, q = 0;
  for (Part& p : parts) {
    p.rec0 = r;
    p.seq0 = q;
    r += p.records;
    q += p.seq;
  }
}

}  // namespace

extern "C" {

ah_status ah_fasta_count(const char* text, uint64_t bytes, uint64_t* n_records, uint64_t* seq_bytes) {
  if ((!text && bytes) || !n_records || !seq_bytes)
    return ah::set_error(AH_ERR_INVALID_ARG, "ah_fasta_count: null argument");
  std::vector<Part> parts = cut(text, bytes, reader_threads());
  count_parts(text, parts);
  if (!parts.empty() && parts.front().lead)
    return ah::set_error(AH_ERR_INVALID_ARG, "FASTA: sequence bytes before the first '>' line");
  uint64_t r = 0, q = 0;
  for (const Part& p : parts) {
    r += p.records;
    q += p.seq;
  }
  *n_records = r;
  *seq_bytes = q;
  return AH_OK;
}

ah_status ah_fasta_read(const char* text, uint64_t bytes, uint8_t* seq, uint64_t seq_capacity,
                        uint64_t* seq_off, uint64_t* name_span, uint64_t max_records) {
  if ((!text && bytes) || !seq_off || (max_records && !name_span))
    return ah::set_error(AH_ERR_INVALID_ARG, "ah_fasta_read: null argument");
  std::vector<Part> parts = cut(text, bytes, reader_threads());
  count_parts(text, parts);
  if (!parts.empty() && parts.front().lead)
    return ah::set_error(AH_ERR_INVALID_ARG, "FASTA: sequence bytes before the first '>' line");
  const uint64_t records = parts.empty() ? 0 : parts.back().rec0 + parts.back().records;
  const uint64_t total = parts.empty() ? 0 : parts.back().seq0 + parts.back().seq;
  if (records > max_records || total > seq_capacity || (total && !seq))
    return ah::set_error(AH_ERR_LIMIT, "ah_fasta_read: %llu records and %llu bytes, room for %llu "
                         "and %llu (ah_fasta_count gives the sizes)",
                         (unsigned long long)records, (unsigned long long)total,
                         (unsigned long long)max_records, (unsigned long long)seq_capacity);
  std::vector<std::thread> th;
  for (const Part& p : parts)
    th.emplace_back([=, &p] {
      uint64_t r = p.rec0, q = p.seq0;
      walk(
          text, p.beg, p.end,
          [&](uint64_t nb, uint64_t ne) {
            seq_off[r] = q;
            name_span[2 * r] = nb;
            name_span[2 * r + 1] = ne;
            ++r;
          },
          [&](uint64_t a, uint64_t n) {
            memcpy(seq + q, text + a, n);
            q += n;
          });
    });
  for (auto& x : th) x.join();
  seq_off[records] = total;
  return AH_OK;
}

}  // extern "C"
