// Host runtime of libah: argument and primer validation, the primer compiler
// (IUPAC sets, reverse complements, clamp positions), generation and
// compilation of the per-primer-set scan program, per-device caches, and the
// C entry points declared in ah.h.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <dlfcn.h>
#include <spawn.h>
#include <sys/wait.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ah.h"
#include "ah_dev.h"
#include "ah_internal.h"

namespace {

const char kScanCore[] =
#include "scan_core_src.inc"
    ;

thread_local std::string g_err;

ah_status fail(ah_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define AH_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(AH_ERR_HIP, "%s: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                          \
  } while (0)

// ------------------------------------------------------- primer compiler --
// IUPAC nucleotide codes as 4-bit sets: A=1 C=2 G=4 T=8.
int iupac_mask(char c) {
  switch (c | 0x20) {
    case 'a': return 1;
    case 'c': return 2;
    case 'g': return 4;
    case 't': return 8;
    case 'r': return 1 | 4;
    case 'y': return 2 | 8;
    case 's': return 2 | 4;
    case 'w': return 1 | 8;
    case 'k': return 4 | 8;
    case 'm': return 1 | 2;
    case 'b': return 2 | 4 | 8;
    case 'd': return 1 | 4 | 8;
    case 'h': return 1 | 2 | 8;
    case 'v': return 1 | 2 | 4;
    case 'n': return 15;
    default: return 0;
  }
}

// Complement of a set: A<->T (bit 0 <-> bit 3), C<->G (bit 1 <-> bit 2).
inline uint8_t comp_mask(uint8_t m) {
  return (uint8_t)(((m & 1) << 3) | ((m & 8) >> 3) | ((m & 2) << 1) | ((m & 4) >> 1));
}

struct Primer {
  int L = 0;
  uint8_t mask[32] = {};
};

ah_status parse_primer(const char* s, const char* what, uint32_t pair, Primer& p) {
  if (!s) return fail(AH_ERR_INVALID_ARG, "pair %u: %s primer is NULL", pair, what);
  const size_t L = strlen(s);
  if (L < AH_MIN_PRIMER_LEN || L > AH_MAX_PRIMER_LEN)
    return fail(AH_ERR_LIMIT, "pair %u: %s primer has %zu nt (allowed %d..%d)", pair, what, L,
                AH_MIN_PRIMER_LEN, AH_MAX_PRIMER_LEN);
  p.L = (int)L;
  for (size_t j = 0; j < L; ++j) {
    const int m = iupac_mask(s[j]);
    if (!m)
      return fail(AH_ERR_INVALID_PRIMER, "pair %u: %s primer: '%c' at %zu is not an IUPAC code",
                  pair, what, s[j], j);
    p.mask[j] = (uint8_t)m;
  }
  return AH_OK;
}

// One pattern: a primer (or its reverse complement) in top-strand window
// orientation, with its clamp positions in window coordinates.
struct Pattern {
  uint32_t pair, primer, strand, k;
  int L;
  uint8_t mask[32];
  uint32_t clamp_bits;  // window positions that must match
};

struct PairSet {
  std::vector<Primer> fwd, rev;
  std::vector<uint32_t> k, clamp, flags;
};

ah_status compile_pairs(const ah_primer_pair* pairs, uint32_t n_pairs, PairSet& ps) {
  if (!pairs || n_pairs == 0) return fail(AH_ERR_INVALID_ARG, "no primer pairs");
  if (n_pairs > 65535) return fail(AH_ERR_LIMIT, "at most 65535 primer pairs per call");
  ps.fwd.resize(n_pairs);
  ps.rev.resize(n_pairs);
  ps.k.resize(n_pairs);
  ps.clamp.resize(n_pairs);
  ps.flags.resize(n_pairs);
  for (uint32_t q = 0; q < n_pairs; ++q) {
    ah_status s = parse_primer(pairs[q].fwd, "fwd", q, ps.fwd[q]);
    if (s) return s;
    s = parse_primer(pairs[q].rev, "rev", q, ps.rev[q]);
    if (s) return s;
    if (pairs[q].k > AH_MAX_K) return fail(AH_ERR_LIMIT, "pair %u: k = %u > %d", q, pairs[q].k, AH_MAX_K);
    const int lmin = ps.fwd[q].L < ps.rev[q].L ? ps.fwd[q].L : ps.rev[q].L;
    if ((int)pairs[q].clamp > lmin)
      return fail(AH_ERR_LIMIT, "pair %u: clamp %u longer than a primer", q, pairs[q].clamp);
    if (pairs[q].flags & ~AH_PAIR_DECOY)
      return fail(AH_ERR_INVALID_ARG, "pair %u: unknown flags 0x%x", q, pairs[q].flags);
    ps.k[q] = pairs[q].k;
    ps.clamp[q] = pairs[q].clamp;
    ps.flags[q] = pairs[q].flags;
  }
  return AH_OK;
}

std::vector<Pattern> patterns_of(const PairSet& ps) {
  std::vector<Pattern> out;
  for (uint32_t q = 0; q < ps.fwd.size(); ++q) {
    for (uint32_t primer = 0; primer < 2; ++primer) {
      // a decoy pair scans the position-wise complement of each primer
      // (reverse(G) read for P is G read for that primer; see ah.h)
      Primer p = primer ? ps.rev[q] : ps.fwd[q];
      if (ps.flags[q] & AH_PAIR_DECOY)
        for (int j = 0; j < p.L; ++j) p.mask[j] = comp_mask(p.mask[j]);
      const int c = (int)ps.clamp[q];
      for (uint32_t strand = 0; strand < 2; ++strand) {
        Pattern t{};
        t.pair = q;
        t.primer = primer;
        t.strand = strand;
        t.k = ps.k[q];
        t.L = p.L;
        for (int j = 0; j < p.L; ++j)
          t.mask[j] = strand ? comp_mask(p.mask[p.L - 1 - j]) : p.mask[j];
        // the primer's 3' end: right end of the window on +, left end on -
        for (int j = 0; j < c; ++j) t.clamp_bits |= 1u << (strand ? j : p.L - 1 - j);
        out.push_back(t);
      }
    }
  }
  return out;
}

// Mismatch indicator of IUPAC set m for the 2-bit code (h, l): A=00 C=01
// G=10 T=11.  Empty string for N (never a mismatch).
std::string mism_expr(uint8_t m, int j) {
  char h[16], l[16];
  snprintf(h, sizeof h, "h[%d]", j);
  snprintf(l, sizeof l, "l[%d]", j);
  std::string H = h, Lw = l;
  switch (m) {
    case 1: return "(" + H + " | " + Lw + ")";          // A
    case 2: return "(" + H + " | ~" + Lw + ")";         // C
    case 4: return "(~" + H + " | " + Lw + ")";         // G
    case 8: return "~(" + H + " & " + Lw + ")";         // T
    case 5: return Lw;                                  // R = A/G: low bit must be 0
    case 10: return "~" + Lw;                           // Y = C/T
    case 6: return "~(" + H + " ^ " + Lw + ")";         // S = C/G
    case 9: return "(" + H + " ^ " + Lw + ")";          // W = A/T
    case 12: return "~" + H;                            // K = G/T
    case 3: return H;                                   // M = A/C
    case 14: return "~(" + H + " | " + Lw + ")";        // B: only A mismatches
    case 13: return "(~" + H + " & " + Lw + ")";        // D: only C
    case 11: return "(" + H + " & ~" + Lw + ")";        // H: only G
    case 7: return "(" + H + " & " + Lw + ")";          // V: only T
    default: return "";                                 // N
  }
}

// Window words per lane of the scan kernel (AH_SCAN_U, odd, 3..31; default
// 19, the fastest measured for the collection workload): each lane converts the U + L - 1 words of its U window words once, so
// larger U amortises the conversion and the halo, but the tile of
// AH_BLOCK * U words plus the halo staged in LDS leaves room for fewer
// workgroups per CU.  Odd U puts the lanes' 8-byte LDS reads in distinct banks.
int scan_u() {
  const char* e = getenv("AH_SCAN_U");
  const int u = e ? atoi(e) : ah::kScanU;
  return (u >= 3 && u <= 31 && (u & 1)) ? u : ah::kScanU;
}

// ---- v_bitop3_b32 truth tables.  The table of f over operands (S0, S1, S2)
// is f evaluated bitwise on the 8-bit vectors S0 = 0xF0, S1 = 0xCC,
// S2 = 0xAA (bit i of the table is f at S0 = i>>2 & 1, S1 = i>>1 & 1,
// S2 = i & 1).
constexpr uint8_t kS0 = 0xF0, kS1 = 0xCC, kS2 = 0xAA;

// Mismatch indicator of IUPAC set m, bitwise over the code planes (h, l):
// A = 00, C = 01, G = 10, T = 11.
uint8_t tt_mism(uint8_t m, uint8_t H, uint8_t L) {
  unsigned r = 0;
  if (!(m & 1)) r |= ~H & ~L;
  if (!(m & 2)) r |= ~H & L;
  if (!(m & 4)) r |= H & ~L;
  if (!(m & 8)) r |= H & L;
  return (uint8_t)r;
}

std::string bitop3(const std::string& a, const std::string& b, const std::string& c, uint8_t tt) {
  char t[16];
  snprintf(t, sizeof t, "0x%02x", tt);
  return "__builtin_amdgcn_bitop3_b32(" + a + ", " + b + ", " + c + ", " + t + ")";
}

std::string hj(int j) { return "h[" + std::to_string(j) + "]"; }
std::string lj(int j) { return "l[" + std::to_string(j) + "]"; }

// x = mismatch of position j (one op)
std::string mism_op(uint8_t m, int j) { return bitop3(hj(j), lj(j), hj(j), tt_mism(m, kS0, kS1)); }
// acc | mismatch of position j (one op)
std::string acc_mism_op(const std::string& acc, uint8_t m, int j) {
  return bitop3(acc, hj(j), lj(j), (uint8_t)(kS0 | tt_mism(m, kS1, kS2)));
}

// ---- filter codegen over bit planes.  In the scan kernel each lane holds,
// for the words of its windows, the one-hot planes pa/pc/pg/pt (bit b set
// iff that base is A/C/G/T) and the planes ph = h, pl = l, px = h ^ l of the
// 2-bit code (A=00, C=01, G=10, T=11).  Every IUPAC code but N is then one
// literal: a single base is a one-hot plane, three bases the complement of
// the missing base's plane, and each of the six two-base codes one bit
// plane or its complement (M = AC: ~h, K = GT: h, R = AG: ~l, Y = CT: l,
// S = CG: h ^ l, W = AT: ~(h ^ l)).  N always matches.
const char* const kPlane[4] = {"pa", "pc", "pg", "pt"};

struct Lit {
  std::string v;
  bool neg;
};
// A factor of an AND: one literal, or the OR of two.
struct Factor {
  Lit a, b;
  int n;
};

int set_size(uint8_t m) { return __builtin_popcount(m); }

// Whether two-base codes read the code planes (one literal, but up to three
// more live registers per ring word) or OR two one-hot planes
// (AH_SCAN_CODE_PLANES, default 0).
bool code_planes() {
  const char* e = getenv("AH_SCAN_CODE_PLANES");
  return e && e[0] == '1';
}

Factor match_factor(uint8_t m, int j) {
  const std::string sj = "[" + std::to_string(j) + "]";
  int bases[4], nb = 0;
  for (int b = 0; b < 4; ++b)
    if (m >> b & 1) bases[nb++] = b;
  Factor f;
  f.n = 1;
  if (nb == 1) {
    f.a = {kPlane[bases[0]] + sj, false};
  } else if (nb == 3) {
    int miss = 0;
    while (m >> miss & 1) ++miss;
    f.a = {kPlane[miss] + sj, true};
  } else if (!code_planes()) {  // nb == 2, as the OR of two one-hot planes
    f.a = {kPlane[bases[0]] + sj, false};
    f.b = {kPlane[bases[1]] + sj, false};
    f.n = 2;
  } else {  // nb == 2: bit masks over A=1, C=2, G=4, T=8
    switch (m) {
      case 0x3: f.a = {"ph" + sj, true}; break;    // M
      case 0xc: f.a = {"ph" + sj, false}; break;   // K
      case 0x5: f.a = {"pl" + sj, true}; break;    // R
      case 0xa: f.a = {"pl" + sj, false}; break;   // Y
      case 0x6: f.a = {"px" + sj, false}; break;   // S
      default: f.a = {"px" + sj, true}; break;     // W (0x9)
    }
  }
  return f;
}

// One v_bitop3_b32 computing acc? & factors (at most 3 literals in total).
std::string and_op(const std::string& acc, const std::vector<Factor>& fs) {
  std::vector<Lit> in;
  if (!acc.empty()) in.push_back({acc, false});
  for (const Factor& f : fs) {
    in.push_back(f.a);
    if (f.n == 2) in.push_back(f.b);
  }
  const uint8_t sv[3] = {kS0, kS1, kS2};
  auto lit = [&](size_t i, bool neg) -> unsigned { return neg ? (uint8_t)~sv[i] : sv[i]; };
  unsigned tt = 0xff;
  size_t i = 0;
  if (!acc.empty()) tt &= lit(i++, false);
  for (const Factor& f : fs) {
    if (f.n == 1) {
      tt &= lit(i++, f.a.neg);
    } else {
      tt &= lit(i, f.a.neg) | lit(i + 1, f.b.neg);
      i += 2;
    }
  }
  std::vector<std::string> v;
  for (const Lit& l : in) v.push_back(l.v);
  while (v.size() < 3) v.push_back(v[0]);  // unused operand slots
  return bitop3(v[0], v[1], v[2], (uint8_t)tt);
}

// AND of a list of factors as a chain of 3-input operations; returns the
// statements and the number of operations (0 for an empty list).
int and_chain(const std::vector<Factor>& fs, const std::string& dst, std::string* out) {
  std::vector<Factor> one, two;
  for (const Factor& f : fs) (f.n == 1 ? one : two).push_back(f);
  size_t i1 = 0, i2 = 0;
  int ops = 0;
  std::string acc;
  while (i1 < one.size() || i2 < two.size()) {
    std::vector<Factor> take;
    int slots = acc.empty() ? 3 : 2;
    if (i2 < two.size()) {
      take.push_back(two[i2++]);
      slots -= 2;
    }
    while (slots > 0 && i1 < one.size()) {
      take.push_back(one[i1++]);
      --slots;
    }
    if (out) *out += "  " + std::string(acc.empty() ? "u32 " : "") + dst + " = " + and_op(acc, take) + ";\n";
    acc = dst;
    ++ops;
  }
  return ops;
}

// "At least `need` of the B clean indicators k0..k{B-1}" into `dst`; returns
// the number of operations.  Small cases use full adders (sum = xor3, carry
// = maj3, one operation each); larger ones a running count of clean blocks.
int threshold(int B, int need, const std::string& dst, std::string* out) {
  auto k = [](int i) { return "k" + std::to_string(i); };
  int ops = 0;
  auto op = [&](const std::string& d, const std::string& a, const std::string& b,
                const std::string& c, uint8_t tt) {
    if (out) *out += "  u32 " + d + " = " + bitop3(a, b, c, tt) + ";\n";
    ++ops;
  };
  const uint8_t kXor3 = kS0 ^ kS1 ^ kS2;
  const uint8_t kMaj = (kS0 & kS1) | (kS0 & kS2) | (kS1 & kS2);
  const uint8_t kOr3 = kS0 | kS1 | kS2, kAnd3 = kS0 & kS1 & kS2;
  if (need == 1 || need == B) {  // OR / AND of all, three at a time
    const uint8_t tt3 = need == 1 ? kOr3 : kAnd3;
    std::string acc = k(0);
    int i = 1;
    if (B == 1) {
      op(dst, acc, acc, acc, kS0);
      return ops;
    }
    int step = 0;
    while (i < B) {
      const std::string a = k(i), b = i + 1 < B ? k(i + 1) : k(i);
      const std::string d = (i + 2 >= B) ? dst : dst + "_" + std::to_string(step++);
      op(d, acc, a, b, tt3);
      acc = d;
      i += 2;
    }
    return ops;
  }
  if (B == 3 && need == 2) {
    op(dst, k(0), k(1), k(2), kMaj);
  } else if (B == 4) {
    op(dst + "_s", k(0), k(1), k(2), kXor3);
    op(dst + "_y", k(0), k(1), k(2), kMaj);
    // need 2: y | (s & k3); need 3: y & (s | k3)
    op(dst, dst + "_y", dst + "_s", k(3),
       need == 2 ? (uint8_t)(kS0 | (kS1 & kS2)) : (uint8_t)(kS0 & (kS1 | kS2)));
  } else if (B == 5 && need == 2) {
    op(dst + "_y", k(0), k(1), k(2), kMaj);
    op(dst + "_o", k(0), k(1), k(2), kOr3);
    op(dst + "_t", dst + "_o", k(3), k(4), kMaj);
    op(dst, dst + "_y", dst + "_t", dst + "_t", kS0 | kS1);
  } else if (B == 5 && need == 3) {
    op(dst + "_s1", k(0), k(1), k(2), kXor3);
    op(dst + "_y1", k(0), k(1), k(2), kMaj);
    op(dst + "_s2", dst + "_s1", k(3), k(4), kXor3);
    op(dst + "_y2", dst + "_s1", k(3), k(4), kMaj);
    op(dst, dst + "_y1", dst + "_y2", dst + "_s2", kMaj);
  } else if (B == 6 && (need == 2 || need == 3)) {
    op(dst + "_s1", k(0), k(1), k(2), kXor3);
    op(dst + "_y1", k(0), k(1), k(2), kMaj);
    op(dst + "_s2", k(3), k(4), k(5), kXor3);
    op(dst + "_y2", k(3), k(4), k(5), kMaj);
    if (need == 2) {  // y1 | y2 | (s1 & s2)
      op(dst + "_t", dst + "_s1", dst + "_s2", dst + "_s2", kS0 & kS1);
      op(dst, dst + "_y1", dst + "_y2", dst + "_t", kOr3);
    } else {  // maj(y1, y2, s1 | s2)
      op(dst + "_t", dst + "_s1", dst + "_s2", dst + "_s2", kS0 | kS1);
      op(dst, dst + "_y1", dst + "_y2", dst + "_t", kMaj);
    }
  } else {
    // y_j: at least j clean among the blocks so far
    std::vector<std::string> y(need + 1);
    for (int j = 1; j <= need; ++j) y[j] = dst + "_y" + std::to_string(j);
    op(y[1], k(0), k(0), k(0), kS0);
    for (int j = 2; j <= need; ++j) {
      if (out) *out += "  u32 " + y[j] + " = 0u;\n";
    }
    for (int b = 1; b < B; ++b) {
      for (int j = need; j >= 2; --j) {
        if (out) *out += "  " + y[j] + " = " + bitop3(y[j], y[j - 1], k(b), kS0 | (kS1 & kS2)) + ";\n";
        ++ops;
      }
      if (out) *out += "  " + y[1] + " |= " + k(b) + ";\n";
      ++ops;
    }
    if (out) *out += "  u32 " + dst + " = " + y[need] + ";\n";
  }
  return ops;
}

// Filter of one pattern.  mode 1 (pigeonhole): the non-clamp, non-N positions
// are split into k + need blocks; a window with at most k mismatches there
// leaves at least `need` of them clean.  mode 0 (exact): the bit-sliced
// mismatch count itself, for patterns whose blocks would pass too many
// windows.  In both modes the clamp positions must match.
struct FilterPlan {
  int mode = 0;
  int need = 0;
  std::vector<std::vector<int>> blocks;
  double rate = 1.0;  // chance a random window passes (uniform bases)
  double cost = 0.0;  // estimated lane operations per window word
};

// P(at least `need` of the independent events with probabilities p occur)
double at_least(const std::vector<double>& p, int need) {
  std::vector<double> d(p.size() + 1, 0.0);  // d[c] = P(exactly c so far)
  d[0] = 1.0;
  for (size_t i = 0; i < p.size(); ++i)
    for (size_t c = i + 1;; --c) {  // c = i + 1 down to 0
      const double stay = d[c] * (1.0 - p[i]);
      const double up = c ? d[c - 1] * p[i] : 0.0;
      d[c] = stay + up;
      if (c == 0) break;
    }
  double r = 0.0;
  for (size_t c = (size_t)need; c < d.size(); ++c) r += d[c];
  return r;
}

// Cost of candidates: the append branch runs when any lane of the wave has
// one (64 lanes x 32 windows), and each candidate costs its exact count in
// the verify kernel (about 8 operations per position, lane-parallel).
// Weight of a candidate's exact count against filter operations
// (AH_SCAN_CAND_WEIGHT, default 20, measured: the exact count, in its own
// kernels and reading the candidate's words from HBM at random, costs about
// twenty times the estimate below in filter-equivalent time): larger values
// choose stronger filters.
double cand_weight() {
  const char* e = getenv("AH_SCAN_CAND_WEIGHT");
  const double w = e ? atof(e) : 20.0;
  return w > 0 ? w : 20.0;
}

double cand_cost(double rate, int L) {
  const double wave = 1.0 - std::pow(1.0 - std::min(rate, 1.0), 32.0 * 64.0);
  const double per_word = 1.0 - std::pow(1.0 - std::min(rate, 1.0), 32.0);
  return 14.0 * wave + cand_weight() * per_word * 8.0 * L;
}

// Development knob (AH_SCAN_FORCE_NEED = 1, 2 or 3): plan only pigeonhole
// filters with that many clean blocks required (tests use it to make weak
// filters on purpose).
int forced_need() {
  const char* e = getenv("AH_SCAN_FORCE_NEED");
  const int n = e ? atoi(e) : 0;
  return n >= 1 && n <= 3 ? n : 0;
}

FilterPlan plan_filter(const Pattern& p, bool allow) {
  std::vector<int> free_pos;
  std::vector<Factor> clampf;
  double clamp_p = 1.0;
  std::vector<double> miss;  // mismatch probabilities of the free positions
  int exact_ops = 0;
  for (int j = 0; j < p.L; ++j) {
    const int sz = set_size(p.mask[j]);
    if (sz == 4) continue;
    if (p.clamp_bits >> j & 1u) {
      clamp_p *= sz / 4.0;
      clampf.push_back(match_factor(p.mask[j], j));
    } else {
      free_pos.push_back(j);
      miss.push_back(1.0 - sz / 4.0);
      exact_ops += (int)p.k + 1 + (sz == 2 ? 1 : 0);
    }
  }
  const int clamp_ops = clampf.empty() ? 0 : and_chain(clampf, "cl", nullptr) + 1;
  // exact: P(at most k of the free positions mismatch)
  std::vector<double> mm(miss);
  const double exact_rate = clamp_p * (1.0 - at_least(mm, (int)p.k + 1));
  FilterPlan best;
  best.mode = 0;
  best.rate = exact_rate;
  best.cost = exact_ops + clamp_ops + 2 + cand_cost(exact_rate, p.L);
  if (!allow) return best;
  const int force = forced_need();
  if (force) best.cost = 1e300;  // any pigeonhole plan with that need wins
  for (int need = 1; need <= 3; ++need) {
    if (force && need != force) continue;
    const int B = (int)p.k + need;
    if ((int)free_pos.size() < B) break;
    // balance information content over the blocks (largest first)
    std::vector<int> order = free_pos;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return set_size(p.mask[a]) < set_size(p.mask[b]);
    });
    std::vector<std::vector<int>> blocks(B);
    std::vector<double> bits(B, 0.0);
    for (int j : order) {
      int at = 0;
      for (int b = 1; b < B; ++b)
        if (blocks[b].size() < blocks[at].size() ? bits[b] <= bits[at] : bits[b] < bits[at]) at = b;
      // every block needs a position: fill empty ones first
      for (int b = 0; b < B; ++b)
        if (blocks[b].empty()) { at = b; break; }
      blocks[at].push_back(j);
      bits[at] += std::log2(4.0 / set_size(p.mask[j]));
    }
    // cost of a partition: chain operations (a 3-input chain over I inputs
    // takes ceil((I - 1) / 2), so odd input counts waste no slot), the
    // threshold, the clamp, and the candidates it lets through
    auto evaluate = [&](const std::vector<std::vector<int>>& bl, double* rate_out) {
      std::vector<double> clean(B);
      int ops = 0;
      for (int b = 0; b < B; ++b) {
        double bb = 0.0;
        std::vector<Factor> fs;
        for (int j : bl[b]) {
          fs.push_back(match_factor(p.mask[j], j));
          bb += std::log2(4.0 / set_size(p.mask[j]));
        }
        clean[b] = std::exp2(-bb);
        ops += and_chain(fs, "k", nullptr);
      }
      ops += threshold(B, need, "r", nullptr);
      const double rate = clamp_p * at_least(clean, need);
      if (rate_out) *rate_out = rate;
      return ops + clamp_ops + 1 + cand_cost(rate, p.L);
    };
    double rate = 1.0;
    double cost = evaluate(blocks, &rate);
    // local search: move one position to another block while that lowers
    // the cost (typically evening out input counts to odd ones)
    for (int iter = 0; iter < 64; ++iter) {
      double best_move = cost;
      int ba = -1, bb = -1, ja = -1;
      for (int a = 0; a < B; ++a) {
        if (blocks[a].size() < 2) continue;
        for (size_t q = 0; q < blocks[a].size(); ++q)
          for (int b = 0; b < B; ++b) {
            if (b == a) continue;
            auto trial = blocks;
            trial[b].push_back(trial[a][q]);
            trial[a].erase(trial[a].begin() + (long)q);
            const double c2 = evaluate(trial, nullptr);
            if (c2 < best_move - 1e-9) {
              best_move = c2;
              ba = a;
              bb = b;
              ja = (int)q;
            }
          }
      }
      if (ba < 0) break;
      blocks[bb].push_back(blocks[ba][ja]);
      blocks[ba].erase(blocks[ba].begin() + ja);
      cost = evaluate(blocks, &rate);
    }
    if (cost < best.cost) {
      best.mode = 1;
      best.need = need;
      best.blocks = blocks;
      best.rate = rate;
      best.cost = cost;
    }
  }
  return best;
}

// Patterns per group (AH_SCAN_GROUP, default 16): each group's code runs
// over the whole staged tile before the next group's.
int scan_group() {
  const char* e = getenv("AH_SCAN_GROUP");
  const int g = e ? atoi(e) : 16;
  return g >= 1 && g <= 1024 ? g : 16;
}

bool valid_u(int u) { return u >= 3 && u <= 31 && (u & 1); }

struct Tuning {
  int u;      // window words per lane (odd) and tile
  int group;  // patterns per group
};

Tuning default_tuning() { return Tuning{scan_u(), scan_group()}; }

bool filter_enabled() {
  const char* e = getenv("AH_SCAN_PREFILTER");
  return !(e && e[0] == '0');
}

// Filter of pattern i over one-hot planes: returns the candidate windows.
std::string gen_filter(size_t i, const Pattern& p, const FilterPlan& fp) {
  char buf[512];
  snprintf(buf, sizeof buf,
           "// pattern %zu: pair %u primer %u strand %u, L %d, k %u, %s (random pass rate %.3g, "
           "~%.1f ops per window word)\n"
           "__device__ __forceinline__ u32 ah_pf_%zu(const u32* pa, const u32* pc, const u32* pg,"
           " const u32* pt, const u32* ph, const u32* pl, const u32* px) {\n",
           i, p.pair, p.primer, p.strand, p.L, p.k,
           fp.mode ? ("prefilter: " + std::to_string(fp.need) + " of " +
                      std::to_string(fp.blocks.size()) + " blocks").c_str()
                   : "exact count",
           fp.rate, fp.cost, i);
  std::string s = buf;
  std::vector<Factor> clampf;
  for (int j = 0; j < p.L; ++j)
    if ((p.clamp_bits >> j & 1u) && set_size(p.mask[j]) < 4) clampf.push_back(match_factor(p.mask[j], j));
  if (!clampf.empty()) and_chain(clampf, "cl", &s);
  std::string r;
  if (fp.mode == 1) {
    const int B = (int)fp.blocks.size();
    for (int b = 0; b < B; ++b) {
      std::vector<Factor> fs;
      for (int j : fp.blocks[b]) fs.push_back(match_factor(p.mask[j], j));
      and_chain(fs, "k" + std::to_string(b), &s);
    }
    threshold(B, fp.need, "r", &s);
    r = "r";
  } else {
    // bit-sliced count: s_m set iff more than m mismatches so far; a
    // position's mismatch is the complement of its match factor
    const int K = (int)p.k;
    for (int m = 0; m <= K; ++m) s += "  u32 s" + std::to_string(m) + " = 0u;\n";
    for (int j = 0; j < p.L; ++j) {
      if ((p.clamp_bits >> j & 1u) || set_size(p.mask[j]) == 4) continue;
      Factor f = match_factor(p.mask[j], j);
      Lit x;  // mismatch literal
      if (f.n == 1) {
        x = {f.a.v, !f.a.neg};
      } else {
        s += "  const u32 x" + std::to_string(j) + " = " +
             bitop3(f.a.v, f.b.v, f.a.v, (uint8_t)~(kS0 | kS1)) + ";\n";
        x = {"x" + std::to_string(j), false};
      }
      const uint8_t xv = x.neg ? (uint8_t)~kS2 : kS2;
      for (int m = K; m >= 1; --m) {
        const std::string sm = "s" + std::to_string(m), sp = "s" + std::to_string(m - 1);
        s += "  " + sm + " = " + bitop3(sm, sp, x.v, (uint8_t)(kS0 | (kS1 & xv))) + ";\n";
      }
      s += "  s0 = " + bitop3("s0", x.v, x.v, (uint8_t)(kS0 | (x.neg ? (uint8_t)~kS1 : kS1))) + ";\n";
    }
    s += "  u32 r = ~s" + std::to_string(K) + ";\n";
    r = "r";
  }
  if (!clampf.empty()) s += "  return " + r + " & cl;\n}\n";
  else s += "  return " + r + ";\n}\n";
  return s;
}

// Exact count of pattern i for the candidate windows `cand` at window word t
// (h, l: the L words from t on), and append of the binding sites.
std::string gen_exact(size_t i, const Pattern& p, bool has_n) {
  const int K = (int)p.k;
  char buf[512];
  snprintf(buf, sizeof buf,
           "__device__ __forceinline__ u32 ah_ex_%zu(const u32* h, const u32* l, const AhCtx& c,"
           " u32 t, u32 cand, AhHitRec* out, u64 cap, u64 slot, bool emit) {\n"
           "  cand &= ah_valid(c, t, %du);\n  if (!cand) return 0u;\n",
           i, p.L);
  std::string s = buf;
  if (has_n) {
    snprintf(buf, sizeof buf,
             "  u32 nm[%d];\n#pragma unroll\n  for (int j = 0; j < %d; ++j) nm[j] = c.gn[t + j];\n",
             p.L, p.L);
    s += buf;
  }
  s += "  u32 x, cf = 0u;\n";
  for (int m = 0; m <= K; ++m) s += "  u32 s" + std::to_string(m) + " = 0u;\n";
  for (int j = 0; j < p.L; ++j) {
    const bool isN = set_size(p.mask[j]) == 4;
    if (isN && !has_n) continue;
    std::string e = isN ? std::string("0u") : mism_op(p.mask[j], j);
    if (has_n) e = isN ? "nm[" + std::to_string(j) + "]" : "(" + e + " | nm[" + std::to_string(j) + "])";
    s += "  x = " + e + ";";
    if (p.clamp_bits >> j & 1u) {
      s += " cf |= x;\n";  // a clamp mismatch rejects the window outright
      continue;
    }
    for (int m = K; m >= 1; --m) {
      const std::string sm = "s" + std::to_string(m), sp = "s" + std::to_string(m - 1);
      s += " " + sm + " = " + bitop3(sm, sp, "x", (uint8_t)(kS0 | (kS1 & kS2))) + ";";
    }
    s += " s0 |= x;\n";
  }
  snprintf(buf, sizeof buf, "  const u32 hb = cand & ~(s%d | cf);\n", K);
  s += buf;
  if (K == 0) {
    snprintf(buf, sizeof buf,
             "  if (hb && emit) { const u32 lv[1] = {0u}; ah_emit<0>(c, out, cap, slot, t, hb, lv, %uu, "
             "%uu); }\n  return (u32)__popc(hb);\n}\n",
             p.pair, (p.strand << 1) | p.primer);
  } else {
    std::string lv = "s0";
    for (int m = 1; m < K; ++m) lv += ", s" + std::to_string(m);
    snprintf(buf, sizeof buf,
             "  if (hb && emit) { const u32 lv[%d] = {%s}; ah_emit<%d>(c, out, cap, slot, t, hb, lv, "
             "%uu, %uu); }\n  return (u32)__popc(hb);\n}\n",
             K, lv.c_str(), K, p.pair, (p.strand << 1) | p.primer);
  }
  s += buf;
  return s;
}

// Candidate appends of a group's patterns a .. b - 1 (their filter outputs
// c0, c1, ... relative to a), one record per quad of patterns: in tile mode
// only from lanes with a candidate in the quad; in wave mode every lane calls
// (the slot comes from a ballot over the wave).
std::string quad_appends(size_t a, size_t b, bool wave) {
  std::string s;
  char buf[512];
  for (size_t q = a; q < b; q += 4) {
    std::string m[4];
    for (int r = 0; r < 4; ++r)
      m[r] = q + r < b ? "c" + std::to_string(q + r - a) : std::string("0u");
    if (wave) {
      snprintf(buf, sizeof buf, "      cnt = ah_wcand(c, k, t, %zuu, %s, %s, %s, %s, cnt, s);\n", q,
               m[0].c_str(), m[1].c_str(), m[2].c_str(), m[3].c_str());
    } else {
      snprintf(buf, sizeof buf,
               "      if (%s | %s | %s | %s) ah_cand(c, k, t, %zuu, %s, %s, %s, %s);\n",
               m[0].c_str(), m[1].c_str(), m[2].c_str(), m[3].c_str(), q, m[0].c_str(),
               m[1].c_str(), m[2].c_str(), m[3].c_str());
    }
    s += buf;
  }
  return s;
}

// Wave mode (see the scan core): per group, lane `lane` of the wave converts
// its AH_U own words of the staged wave tile, the last group then issues the
// copy of the wave's next tile, and every step takes the planes of the one
// word past its own range that it newly needs from the next lane (the next
// lane's own word of the same index: ds_bpermute).  The ring arrays hold the
// own words at [0, AH_U) and those halo words after them, so the filters read
// position j of window word u at index u + j as in tile mode.
std::string gen_wave_groups(const std::vector<Pattern>& pats, size_t G) {
  const size_t ngroups = (pats.size() + G - 1) / G;
  std::string s;
  char buf[2048];
  for (size_t gi = 0; gi < ngroups; ++gi) {
    const size_t a = gi * G, b = std::min(pats.size(), a + G);
    int lg = 0;
    for (size_t i = a; i < b; ++i) lg = std::max(lg, pats[i].L);
    const bool last = gi + 1 == ngroups;
    snprintf(buf, sizeof buf,
             "__device__ %s u32 ah_wgroup_%zu(ah_lds_uint2* tw, u32 t0, const AhCtx& c, "
             "const AhCands& k, u32 lane, uint4* my, const AhNext& nx, u32 cnt, u32 s) {\n"
             "  const u32 base = lane * (u32)AH_U;\n"
             "  u32 pa[AH_U + %d], pc[AH_U + %d], pg[AH_U + %d], pt[AH_U + %d];\n"
             "  u32 ph[AH_U + %d], pl[AH_U + %d], px[AH_U + %d];\n"
             "#pragma unroll\n"
             "  for (int w = 0; w < AH_U; ++w)\n"
             "    ah_planes(tw[base + (u32)w], pa[w], pc[w], pg[w], pt[w], ph[w], pl[w], px[w]);\n"
             "%s"
             "  const int src = (int)(((lane + 1u) & 63u) << 2);\n"
             "  constexpr int kHalo = %d;  // the group's longest primer - 1\n"
             "  // the planes of halo word hw, from the next lane's own word hw\n"
             "  auto halo = [&](int hw) {\n"
             "    pa[AH_U + hw] = __builtin_amdgcn_ds_bpermute(src, (int)pa[hw]);\n"
             "    pc[AH_U + hw] = __builtin_amdgcn_ds_bpermute(src, (int)pc[hw]);\n"
             "    pg[AH_U + hw] = __builtin_amdgcn_ds_bpermute(src, (int)pg[hw]);\n"
             "    pt[AH_U + hw] = __builtin_amdgcn_ds_bpermute(src, (int)pt[hw]);\n"
             "    ph[AH_U + hw] = __builtin_amdgcn_ds_bpermute(src, (int)ph[hw]);\n"
             "    pl[AH_U + hw] = __builtin_amdgcn_ds_bpermute(src, (int)pl[hw]);\n"
             "    px[AH_U + hw] = __builtin_amdgcn_ds_bpermute(src, (int)px[hw]);\n"
             "  };\n"
             "  // halo word u + kHalo - AH_U is first read at step u; it is fetched a\n"
             "  // step earlier, so that the exchange is done when the step starts\n"
             "  if (kHalo - AH_U >= 0) halo(kHalo - AH_U);\n"
             "#pragma unroll\n"
             "  for (int u = 0; u < AH_U; ++u) {\n"
             "    if (u + 1 < AH_U && u + 1 + kHalo - AH_U >= 0) halo(u + 1 + kHalo - AH_U);\n"
             "    const u32 t = lane < 63u ? t0 + base + (u32)u : 0xffffffffu;  // lane 63: no windows\n",
             ngroups > 1 ? "__noinline__" : "__forceinline__", gi, lg - 1, lg - 1, lg - 1, lg - 1,
             lg - 1, lg - 1, lg - 1,
             last ? "  // every lane holds its planes: the slice is free for the next tile\n"
                    "  __builtin_amdgcn_s_waitcnt(AH_WAIT_LGKMCNT0);\n"
                    "  if (nx.valid) ah_wstage(nx.c, nx.t0, my, lane);\n"
                  : "",
             lg - 1);
    s += buf;
    std::string any;
    for (size_t i = a; i < b; ++i) {
      snprintf(buf, sizeof buf,
               "    const u32 c%zu = ah_pf_%zu(pa + u, pc + u, pg + u, pt + u, ph + u, pl + u, px + u);\n",
               i - a, i);
      s += buf;
      any += (i > a ? " | c" : "c") + std::to_string(i - a);
    }
    // a wave-wide vote, so that every lane takes the branch and keeps the same
    // candidate count (the count is uniform over the wave).  With an even
    // number of patterns the last filter's result is compared with the OR of
    // the others as one 64-bit pair (v_cmp_ne_u64 into a lane mask, the
    // branch on that mask is scalar): one OR fewer per window word than a
    // 32-bit compare of the OR of all of them.
    const size_t gn = b - a;
    if (gn >= 2 && gn % 2 == 0) {
      std::string rest;
      for (size_t i = 0; i + 1 < gn; ++i) rest += (i ? " | c" : "c") + std::to_string(i);
      s += "    u64 any_c;\n"
           "    asm volatile(\"v_cmp_ne_u64_e64 %0, 0, %1\" : \"=s\"(any_c) : \"v\"((u64)(" + rest +
           ") | ((u64)c" + std::to_string(gn - 1) + " << 32)));\n";
      s += "    if (any_c != 0ull) {\n";
    } else {
      s += "    if (__any((" + any + ") != 0u)) {\n";
    }
    s += quad_appends(a, b, true);
    s += "    }\n  }\n  return cnt;\n}\n";
  }
  s += "__device__ u32 ah_wgroups(ah_lds_uint2* tw, u32 t0, const AhCtx& c, const AhCands& k, "
       "u32 lane, uint4* my, const AhNext& nx, u32 cnt, u32 s) {\n";
  for (size_t gi = 0; gi < ngroups; ++gi)
    s += "  cnt = ah_wgroup_" + std::to_string(gi) + "(tw, t0, c, k, lane, my, nx, cnt, s);\n";
  s += "  return cnt;\n}\n";
  return s;
}

// Wave mode applies when every halo word lies in the next lane's own words
// (AH_U >= longest primer - 1) and is not switched off (AH_SCAN_WAVE=0).
bool wave_mode(const std::vector<Pattern>& pats, Tuning tn) {
  const char* e = getenv("AH_SCAN_WAVE");
  if (e && e[0] == '0') return false;
  int lmax = 0;
  for (const Pattern& p : pats) lmax = p.L > lmax ? p.L : lmax;
  return tn.u >= lmax - 1;
}

// In tile mode the filter takes the exact count after its last tile for
// programs of up to this many patterns (4 pairs).  With more, every
// workgroup filters to the end, nothing overlaps the count, and a launch of
// its own runs it at a higher occupancy (64-pair batch: 1.6 ms slower in the
// filter, against 1.2 ms saved over 64 single-pair tile-mode queries).
constexpr size_t kTileCountPatterns = 16;

std::string gen_program_uncached(const std::vector<Pattern>& pats, bool has_n, Tuning tn) {
  int lmax = 0;
  for (const Pattern& p : pats) lmax = p.L > lmax ? p.L : lmax;
  const bool allow = filter_enabled();
  const bool wave = wave_mode(pats, tn);
  const bool tile_count = !wave && pats.size() <= kTileCountPatterns;
  std::string s;
  char buf[2048];
  // every quad of patterns (4 from the start of each group) within one pair
  bool uniform = true;
  for (size_t a = 0; a < pats.size(); a += (size_t)tn.group)
    for (size_t q = a; q < std::min(pats.size(), a + (size_t)tn.group); q += 4)
      for (size_t r = q + 1; r < std::min({pats.size(), a + (size_t)tn.group, q + 4}); ++r)
        uniform &= pats[r].pair == pats[q].pair;
  snprintf(buf, sizeof buf,
           "#define AH_U %d\n#define AH_HALO %d\n#define AH_HAS_N %d\n#define AH_WAVE %d\n"
           "#define AH_QUAD_ONE_PAIR %d\n#define AH_TILE_COUNT %d\n",
           tn.u, lmax - 1, has_n ? 1 : 0, wave ? 1 : 0, uniform ? 1 : 0, tile_count ? 1 : 0);
  std::string head = buf;
  for (size_t i = 0; i < pats.size(); ++i) {
    s += gen_filter(i, pats[i], plan_filter(pats[i], allow));
    s += gen_exact(i, pats[i], has_n);
  }
  // groups of consecutive patterns; one function per group walks the tile:
  // each lane converts the words of its AH_U window words once and runs
  // every filter of the group on each window word
  const size_t G = (size_t)tn.group;
  const size_t ngroups = wave ? 0 : (pats.size() + G - 1) / G;
  for (size_t gi = 0; gi < ngroups; ++gi) {
    const size_t a = gi * G, b = std::min(pats.size(), a + G);
    int lg = 0;
    for (size_t i = a; i < b; ++i) lg = std::max(lg, pats[i].L);
    snprintf(buf, sizeof buf,
             "__device__ %s void ah_group_%zu(ah_lds_uint2* tw, u32 t0, const AhCtx& c, "
             "const AhCands& k) {\n"
             "  const u32 base = threadIdx.x * (u32)AH_U;\n"
             "  if (t0 + base >= c.S) return;\n"
             "  u32 pa[AH_U + %d], pc[AH_U + %d], pg[AH_U + %d], pt[AH_U + %d];\n"
             "  u32 ph[AH_U + %d], pl[AH_U + %d], px[AH_U + %d];\n"
             "#pragma unroll\n"
             "  for (int w = 0; w < %d; ++w)\n"
             "    ah_planes(tw[base + (u32)w], pa[w], pc[w], pg[w], pt[w], ph[w], pl[w], px[w]);\n"
             "  uint2 nxt = tw[base + %du];  // read one step ahead\n"
             "#pragma unroll\n"
             "  for (int u = 0; u < AH_U; ++u) {\n"
             "    ah_planes(nxt, pa[u + %d], pc[u + %d], pg[u + %d], pt[u + %d], ph[u + %d], pl[u + %d],"
             " px[u + %d]);\n"
             "    if (u + 1 < AH_U) nxt = tw[base + (u32)u + %du];\n"
             "    const u32 t = t0 + base + (u32)u;\n",
             ngroups > 1 ? "__noinline__" : "__forceinline__", gi, lg - 1, lg - 1, lg - 1, lg - 1,
             lg - 1, lg - 1, lg - 1, lg - 1, lg - 1, lg - 1, lg - 1, lg - 1, lg - 1, lg - 1, lg - 1,
             lg - 1, lg);
    s += buf;
    // one branch per window word for the whole group: candidates are rare
    std::string any;
    for (size_t i = a; i < b; ++i) {
      snprintf(buf, sizeof buf,
               "    const u32 c%zu = ah_pf_%zu(pa + u, pc + u, pg + u, pt + u, ph + u, pl + u, px + u);\n",
               i - a, i);
      s += buf;
      any += (i > a ? " | c" : "c") + std::to_string(i - a);
    }
    s += "    if (" + any + ") {\n";
    s += quad_appends(a, b, false);
    s += "    }\n  }\n}\n";
  }
  if (wave) {
    s += gen_wave_groups(pats, G);
  } else {
    s += "__device__ void ah_groups(ah_lds_uint2* tw, u32 t0, const AhCtx& c, const AhCands& k) {\n";
    for (size_t gi = 0; gi < ngroups; ++gi) s += "  ah_group_" + std::to_string(gi) + "(tw, t0, c, k);\n";
    s += "}\n";
  }
  // verification: the candidate's words from HBM, then the pattern's count
  snprintf(buf, sizeof buf,
           "template <class W>\n"
           "__device__ u32 ah_verify_one(const AhCtx& c, W w, u32 t, u32 p, u32 cand, AhHitRec* out,"
           " u64 cap, u64 slot, bool emit) {\n"
           "  u32 h[%d], l[%d];\n#pragma unroll\n"
           "  for (int j = 0; j < %d; ++j) { const uint2 v = w[j]; h[j] = v.x; l[j] = v.y; }\n"
           "  switch (p) {\n",
           lmax, lmax, lmax);
  s += buf;
  for (size_t i = 0; i < pats.size(); ++i) {
    snprintf(buf, sizeof buf, "    case %zuu: return ah_ex_%zu(h, l, c, t, cand, out, cap, slot, emit);\n",
             i, i);
    s += buf;
  }
  s += "    default: return 0u;\n  }\n}\n";
  s += "__device__ u32 ah_pat_pair(u32 p) {\n  switch (p) {\n";
  for (size_t i = 0; i < pats.size(); ++i) {
    snprintf(buf, sizeof buf, "    case %zuu: return %uu;\n", i, pats[i].pair);
    s += buf;
  }
  s += "    default: return 0u;\n  }\n}\n";
  return head + std::string(kScanCore) + s;
}

// The generated source of a pattern set, memoised: planning the filters
// (a local search per pattern) costs far more than a scan launch.  The key
// holds every input of the generator, the planner's knobs included.
std::string gen_program(const std::vector<Pattern>& pats, bool has_n, Tuning tn) {
  static std::mutex mu;
  static std::map<std::string, std::string> cache;
  std::string key;
  key.reserve(pats.size() * sizeof(Pattern) + 64);
  for (const Pattern& p : pats) {
    Pattern q{};  // a zeroed copy: the key holds no padding bytes
    q.pair = p.pair; q.primer = p.primer; q.strand = p.strand; q.k = p.k; q.L = p.L;
    memcpy(q.mask, p.mask, sizeof q.mask);
    q.clamp_bits = p.clamp_bits;
    key.append((const char*)&q, sizeof q);
  }
  char buf[160];
  snprintf(buf, sizeof buf, "|%d|%d|%d|%d|%.17g|%d|%d|%d", has_n ? 1 : 0, tn.u, tn.group,
           filter_enabled() ? 1 : 0, cand_weight(), forced_need(), code_planes() ? 1 : 0,
           wave_mode(pats, tn) ? 1 : 0);
  key += buf;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  std::string src = gen_program_uncached(pats, has_n, tn);
  std::lock_guard<std::mutex> lk(mu);
  if (cache.size() >= 512) cache.clear();  // bounded: pattern sets are few in practice
  cache.emplace(key, src);
  return src;
}

// --------------------------------------------------------------- caches --
// The kernels of a specialised scan program.
struct ScanFns {
  hipFunction_t scan = nullptr;    // filter: appends candidates (and counts them, below)
  hipFunction_t verify = nullptr;  // exact count of the candidates: sites per candidate
  hipFunction_t emit = nullptr;    // the site records, the result and the statistics
  hipFunction_t emit_seg = nullptr;  // the same, each segment (pair, genome) together
  bool wave = false;               // wave mode: wave tiles of 63 x U words, 4 per workgroup
  bool tile_count = false;         // tile mode, the filter takes the exact count
};

struct JitEntry {
  hipModule_t mod = nullptr;
  ScanFns fn;
};

std::mutex g_mu;
std::map<std::pair<int, std::string>, JitEntry> g_jit;
std::map<std::pair<int, std::string>, void*> g_tables;
uint64_t g_jit_n = 0;
double g_jit_ms = 0.0;
std::map<int, int> g_cus;

std::mutex g_stats_mu;

// The compile helper (ah_jitc) installed beside this library, or "" if
// there is none.  hipRTC compiles one program at a time per process, so
// concurrent compiles (several primer sets prepared at once, the serving
// form's compile threads, the autotuner's shapes) only overlap when each runs
// in a process of its own.
const std::string& jit_helper() {
  static const std::string path = [] {
    Dl_info info;
    if (!dladdr((const void*)&ah_status_str, &info) || !info.dli_fname) return std::string();
    std::string p = info.dli_fname;
    const size_t slash = p.rfind('/');
    p = (slash == std::string::npos ? std::string(".") : p.substr(0, slash)) + "/ah_jitc";
    return access(p.c_str(), X_OK) == 0 ? p : std::string();
  }();
  return path;
}

const char* const kRtcOpts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17"};

// Compile in a child process running the helper: the source and the code
// object travel through two temporary files.
ah_status rtc_compile_child(const std::string& helper, const std::string& src,
                            std::vector<char>& code) {
  const char* tmp = getenv("TMPDIR");
  std::string dir = tmp && tmp[0] ? tmp : "/tmp";
  std::string in = dir + "/ah_jit_XXXXXX", out = dir + "/ah_jit_XXXXXX";
  const int fi = mkstemp(&in[0]);
  if (fi < 0) return fail(AH_ERR_JIT, "cannot create a temporary file in %s", dir.c_str());
  const int fo = mkstemp(&out[0]);
  if (fo < 0) {
    close(fi);
    unlink(in.c_str());
    return fail(AH_ERR_JIT, "cannot create a temporary file in %s", dir.c_str());
  }
  close(fo);
  struct Cleanup {
    std::string a, b;
    ~Cleanup() {
      unlink(a.c_str());
      unlink(b.c_str());
    }
  } cleanup{in, out};
  size_t done = 0;
  while (done < src.size()) {
    const ssize_t w = write(fi, src.data() + done, src.size() - done);
    if (w <= 0) {
      close(fi);
      return fail(AH_ERR_JIT, "cannot write the scan program to %s", in.c_str());
    }
    done += (size_t)w;
  }
  close(fi);
  std::vector<char*> argv = {const_cast<char*>(helper.c_str()), &in[0], &out[0]};
  for (const char* o : kRtcOpts) argv.push_back(const_cast<char*>(o));
  argv.push_back(nullptr);
  pid_t pid = 0;
  const auto t0 = std::chrono::steady_clock::now();
  if (posix_spawn(&pid, helper.c_str(), nullptr, nullptr, argv.data(), environ) != 0)
    return fail(AH_ERR_JIT, "cannot start %s", helper.c_str());
  int wst = 0;
  while (waitpid(pid, &wst, 0) < 0)
    if (errno != EINTR) return fail(AH_ERR_JIT, "waiting for %s failed", helper.c_str());
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  std::vector<char> data;
  if (FILE* f = fopen(out.c_str(), "rb")) {
    char buf[1 << 16];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) data.insert(data.end(), buf, buf + n);
    fclose(f);
  }
  if (!WIFEXITED(wst) || WEXITSTATUS(wst) != 0) {
    data.push_back('\0');
    return fail(AH_ERR_JIT, "%.400s", data.size() > 1 ? data.data() : "the compile helper failed");
  }
  code.swap(data);
  std::lock_guard<std::mutex> lk(g_stats_mu);
  g_jit_n += 1;
  g_jit_ms += ms;
  return AH_OK;
}

ah_status rtc_compile(const std::string& src, std::vector<char>& code) {
  if (!jit_helper().empty()) return rtc_compile_child(jit_helper(), src, code);
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "ah_scan.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    return fail(AH_ERR_JIT, "hiprtcCreateProgram failed");
  const auto t0 = std::chrono::steady_clock::now();
  const hiprtcResult r = hiprtcCompileProgram(prog, 3, const_cast<const char**>(kRtcOpts));
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n + 1, '\0');
    hiprtcGetProgramLog(prog, &log[0]);
    hiprtcDestroyProgram(&prog);
    return fail(AH_ERR_JIT, "scan program failed to compile: %.400s", log.c_str());
  }
  size_t n = 0;
  hiprtcGetCodeSize(prog, &n);
  code.resize(n);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  std::lock_guard<std::mutex> lk(g_stats_mu);
  g_jit_n += 1;
  g_jit_ms += ms;
  return AH_OK;
}

// Loaded scan kernel for an already compiled program (cached per device).
ah_status load_scan_kernel(int dev, const std::string& src, const std::vector<char>& code,
                           ScanFns& fn) {
  std::lock_guard<std::mutex> lk(g_mu);
  const auto key = std::make_pair(dev, src);
  auto it = g_jit.find(key);  // another thread may have loaded it meanwhile
  if (it != g_jit.end()) {
    fn = it->second.fn;
    return AH_OK;
  }
  JitEntry e;
  AH_HIP(hipModuleLoadData(&e.mod, code.data()));
  AH_HIP(hipModuleGetFunction(&e.fn.scan, e.mod, "ah_scan_kernel"));
  AH_HIP(hipModuleGetFunction(&e.fn.verify, e.mod, "ah_verify_kernel"));
  AH_HIP(hipModuleGetFunction(&e.fn.emit, e.mod, "ah_emit_kernel"));
  AH_HIP(hipModuleGetFunction(&e.fn.emit_seg, e.mod, "ah_emit_seg_kernel"));
  e.fn.wave = src.find("#define AH_WAVE 1\n") != std::string::npos;
  e.fn.tile_count = src.find("#define AH_TILE_COUNT 1\n") != std::string::npos;
  g_jit[key] = e;
  fn = e.fn;
  return AH_OK;
}

// Compiled and loaded scan kernel for `src` on the current device (cached;
// compiles outside the cache lock so that several programs can compile at
// once).
// The kernels of a primer set, looked up by the set itself (the pairs'
// strings and parameters, the mask flag, the tuning, the planner's knobs)
// before the generated source is built: the per-call path then does no code
// generation and no comparison of sources.
std::map<std::pair<int, std::string>, ScanFns> g_fns;

std::string fns_key(const std::string& set, bool has_n, Tuning tn) {
  char buf[160];
  snprintf(buf, sizeof buf, "#%d|%d|%d|%d|%.17g|%d|%d", has_n ? 1 : 0, tn.u, tn.group,
           filter_enabled() ? 1 : 0, cand_weight(), forced_need(), code_planes() ? 1 : 0);
  return set + buf;
}

ah_status get_scan_kernel(const std::string& src, ScanFns& fn);
std::string set_key(const ah_primer_pair* pairs, uint32_t n_pairs);

ah_status scan_kernels_for(const ah_primer_pair* pairs, uint32_t n_pairs, const PairSet& ps,
                           bool has_n, Tuning tn, ScanFns& fn) {
  int dev = 0;
  AH_HIP(hipGetDevice(&dev));
  const auto key = std::make_pair(dev, fns_key(set_key(pairs, n_pairs), has_n, tn));
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_fns.find(key);
    if (it != g_fns.end()) {
      fn = it->second;
      return AH_OK;
    }
  }
  ah_status s = get_scan_kernel(gen_program(patterns_of(ps), has_n, tn), fn);
  if (s) return s;
  std::lock_guard<std::mutex> lk(g_mu);
  g_fns[key] = fn;
  return AH_OK;
}

// The kernels of a primer set when they are already loaded on the current
// device (nothing is compiled or loaded).
bool find_scan_kernels(const ah_primer_pair* pairs, uint32_t n_pairs, const PairSet& ps,
                       bool has_n, Tuning tn, ScanFns& fn) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  const auto key = std::make_pair(dev, fns_key(set_key(pairs, n_pairs), has_n, tn));
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_fns.find(key);
    if (it != g_fns.end()) {
      fn = it->second;
      return true;
    }
  }
  const std::string src = gen_program(patterns_of(ps), has_n, tn);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_jit.find(std::make_pair(dev, src));
  if (it == g_jit.end()) return false;
  fn = it->second.fn;
  g_fns[key] = fn;
  return true;
}

ah_status get_scan_kernel(const std::string& src, ScanFns& fn) {
  int dev = 0;
  AH_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_jit.find(std::make_pair(dev, src));
    if (it != g_jit.end()) {
      fn = it->second.fn;
      return AH_OK;
    }
  }
  std::vector<char> code;
  ah_status s = rtc_compile(src, code);
  if (s) return s;
  return load_scan_kernel(dev, src, code, fn);
}

// Tile shape and grouping chosen for a primer set (by the autotuner or the
// caller), per device.
std::map<std::pair<int, std::string>, Tuning> g_tuning;

std::string set_key(const ah_primer_pair* pairs, uint32_t n_pairs) {
  std::string k;
  for (uint32_t q = 0; q < n_pairs; ++q) {
    k += pairs[q].fwd;
    k += '|';
    k += pairs[q].rev;
    k += '|' + std::to_string(pairs[q].k) + '|' + std::to_string(pairs[q].clamp) + '|' +
         std::to_string(pairs[q].flags) + ';';
  }
  return k;
}

Tuning tuning_for(const ah_primer_pair* pairs, uint32_t n_pairs) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_tuning.find(std::make_pair(dev, set_key(pairs, n_pairs)));
  return it != g_tuning.end() ? it->second : default_tuning();
}

// Device copy of a small immutable table, uploaded once per device.
ah_status get_table(const void* host, size_t bytes, void** dptr) {
  int dev = 0;
  AH_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, std::string((const char*)host, bytes));
  auto it = g_tables.find(key);
  if (it != g_tables.end()) {
    *dptr = it->second;
    return AH_OK;
  }
  void* p = nullptr;
  AH_HIP(hipMalloc(&p, bytes));
  AH_HIP(hipMemcpy(p, host, bytes, hipMemcpyHostToDevice));
  g_tables[key] = p;
  *dptr = p;
  return AH_OK;
}

int cu_count() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cus.find(dev);
  if (it != g_cus.end()) return it->second;
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
    n = 256;
  g_cus[dev] = n;
  return n;
}

// ------------------------------------------------------------ profiling --
struct ProfEntry {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  uint64_t launches = 0;
  double ms = 0.0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::map<std::string, ProfEntry> g_prof;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one or more launches on `st` with events when profiling is on.
// Set while a call that must not create HIP objects runs on this thread.
thread_local bool t_prof_off = false;

struct ProfScope {
  const char* name;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(const char* n, hipStream_t s) : name(n), st(s) {
    if (t_prof_off) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    a = take_event();
    b = take_event();
    if (a && b) (void)hipEventRecord(a, st);
  }
  ~ProfScope() {
    if (!a || !b) return;
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof[name].pending.emplace_back(a, b);
  }
};

int bits_for(uint64_t max_value) {  // bits to hold 0..max_value
  int b = 0;
  while (b < 64 && (max_value >> b) != 0) ++b;
  return b;
}

// ------------------------------------------------------------ workspace --
struct Carver {
  uintptr_t base, cur, end;
  explicit Carver(void* p, size_t bytes) : base((uintptr_t)p), cur((uintptr_t)p), end((uintptr_t)p + bytes) {}
  template <class T>
  T* take(uint64_t count) {
    cur = (cur + 255) & ~(uintptr_t)255;
    T* p = (T*)cur;
    cur += (uintptr_t)(count * sizeof(T));
    return p;
  }
  size_t used() const { return (size_t)(cur - base) + 256; }
};

struct ScanWs {
  uint64_t *counts, *tile_prefix, *scan_tmp, *n_sort;
  ah_hit* staging;
  uint4* cands;           // filter output: 2 uint4 per record ({genome, window word, first
                          // pattern of the quad, 0}, the quad's window masks)
  uint32_t* slice_cnt;    // [kMaxScanGrid] candidates kept per workgroup
  uint32_t* slice_tot;    // [kMaxScanGrid] candidates found per workgroup
  uint64_t* slice_win;    // [kMaxScanGrid] windows in them
  uint64_t* slice_sites;  // [kMaxScanGrid] sites in the kept ones
  uint64_t* group_sites;  // [kMaxScanGrid / 64, stride 32] sites of each group of 64 slices
  uint32_t* cand_sites;   // [ccap] sites of each kept candidate
  uint64_t* cstat;        // [0] candidates, [1] windows in them, [2] full slices, [3] most per workgroup
  uint64_t ccap;
  ah::SortBuffers sb;
};

// Workgroups of the scan's filter at most (each owns a slice of the list).
constexpr uint32_t kMaxScanGrid = 4096;
// LDS bytes per compute unit on gfx950 (160 KiB).
constexpr uint64_t kLdsPerCu = 160ull * 1024;

// Candidate records the workspace must hold at least: the hit capacity (a
// candidate holds one or more windows; every window of a site is in one), and
// at least 2^16.  Extra workspace lengthens the list.
uint64_t min_cands(uint64_t cap) { return std::max<uint64_t>(cap, 1ull << 16); }

// Candidate records per window word expected from the filters of a primer set
// (uniform bases).
double cand_per_word(const std::vector<Pattern>& pats) {
  const bool allow = filter_enabled();
  double r = 0.0;
  for (const Pattern& p : pats) {
    const double rate = std::min(plan_filter(p, allow).rate, 1.0);
    r += 1.0 - std::pow(1.0 - rate, 32.0);
  }
  return r;
}

// Recommended list length: twice the expected records over `window_words`
// window words plus 2^16 (at most 2^28 records unless the hit capacity is
// larger).
uint64_t recommended_cands(uint64_t window_words, double per_word, uint64_t cap) {
  const double e = std::min(2.0 * (double)window_words * per_word + 65536.0, (double)(1ull << 28));
  return std::max(min_cands(cap), (uint64_t)e);
}

// Fixed parts first, then the candidate list, which takes `ccap` records or,
// when ccap is 0, everything up to the end of the workspace.
ScanWs carve_scan(Carver& c, uint32_t n, uint64_t cap, uint64_t ccap) {
  ScanWs w;
  w.counts = c.take<uint64_t>(n ? n : 1);
  w.tile_prefix = c.take<uint64_t>((uint64_t)n + 1);
  w.scan_tmp = c.take<uint64_t>(ah::kScanGrid + 1);
  w.n_sort = c.take<uint64_t>(1);
  w.staging = c.take<ah_hit>(cap ? cap : 1);
  w.sb.keys[0] = c.take<uint64_t>(cap ? cap : 1);
  w.sb.keys[1] = c.take<uint64_t>(cap ? cap : 1);
  w.sb.idx[0] = c.take<uint32_t>(cap ? cap : 1);
  w.sb.idx[1] = c.take<uint32_t>(cap ? cap : 1);
  w.sb.hstride = ah::sort_hist_stride(cap);
  for (int b = 0; b < 3; ++b)
    w.sb.hist[b] = c.take<uint32_t>((uint64_t)ah::kSortDigits * w.sb.hstride);
  w.cstat = c.take<uint64_t>(4);
  w.slice_cnt = c.take<uint32_t>(kMaxScanGrid);
  w.slice_tot = c.take<uint32_t>(kMaxScanGrid);
  w.slice_win = c.take<uint64_t>(kMaxScanGrid);
  w.slice_sites = c.take<uint64_t>(kMaxScanGrid);
  w.group_sites = c.take<uint64_t>(kMaxScanGrid / 64 * 32);
  // The candidate records and their site counts: `ccap` of them, or (ccap =
  // 0) as many as the rest holds.  A size computed for some ccap carries 512
  // spare bytes, so that the rest of a workspace of that size holds at least
  // ccap records, whatever the alignment of the workspace (one 256-byte
  // alignment pad between the two arrays, one for the base).
  constexpr uint64_t kPerCand = 2 * sizeof(uint4) + sizeof(uint32_t);
  const bool rest = ccap == 0;
  if (rest) {
    const uintptr_t at = (c.cur + 255) & ~(uintptr_t)255;
    ccap = c.end > at + 256 ? (uint64_t)(c.end - at - 256) / kPerCand : 0;
  }
  w.ccap = ccap;
  w.cands = c.take<uint4>(2 * ccap);
  w.cand_sites = c.take<uint32_t>(ccap);
  if (!rest) c.cur += 512;
  return w;
}

size_t scan_ws_bytes(uint32_t n, uint64_t cap, uint64_t ccap) {
  Carver c(nullptr, 0);
  carve_scan(c, n, cap, ccap);
  return c.used();
}

ah::PairBuffers carve_pair(Carver& c, uint64_t cap) {
  const uint64_t m = cap ? cap : 1;
  ah::PairBuffers b;
  b.cf = c.take<uint64_t>(ah::kPairGrid);
  b.cr = c.take<uint64_t>(ah::kPairGrid);
  b.cc = c.take<uint64_t>(ah::kPairGrid);
  b.mtot = c.take<uint64_t>(2);
  b.mkey_f = c.take<uint64_t>(m);
  b.mpos_f = c.take<uint32_t>(m);
  b.midx_f = c.take<uint32_t>(m);
  b.mkey_r = c.take<uint64_t>(m);
  b.mpos_r = c.take<uint32_t>(m);
  b.midx_r = c.take<uint32_t>(m);
  b.cnt = c.take<uint32_t>(m);
  b.pre_f = c.take<uint32_t>(m);
  b.pre_r = c.take<uint32_t>(m);
  b.rng = c.take<uint32_t>(8 * m);
  return b;
}

ah_status check_genomes(const ah_genomes* g) {
  if (!g) return fail(AH_ERR_INVALID_ARG, "genomes is NULL");
  if (g->n > 0 && (!g->words || !g->word_off || !g->len))
    return fail(AH_ERR_INVALID_ARG, "genomes: words, word_off and len must be device pointers");
  if (g->max_len == 0 && g->n > 0) return fail(AH_ERR_INVALID_ARG, "genomes: max_len must be >= 1");
  return AH_OK;
}

// Segment buffers of ah_query, carved from the workspace's radix-sort
// buffers, which its segmented tail does not use.  False when the segments
// are more than kSegMax or do not fit there.
bool carve_seg(const ScanWs& w, uint32_t n_genomes, uint64_t n_seg, ah::SegBuffers& sg) {
  if (n_seg == 0 || n_seg > ah::kSegMax) return false;
  const uintptr_t beg = (uintptr_t)w.sb.keys[0];
  const uintptr_t end = (uintptr_t)w.sb.hist[2] +
                        (uintptr_t)ah::kSortDigits * w.sb.hstride * sizeof(uint32_t);
  Carver c((void*)beg, (size_t)(end - beg));
  sg.cnt = c.take<uint32_t>(4 * n_seg);  // counts, fill counters, look-back words
  sg.fill = sg.cnt + n_seg;
  sg.lb = (uint64_t*)(sg.cnt + 2 * n_seg);
  sg.off = c.take<uint64_t>(n_seg + 1);
  sg.n_seg = (uint32_t)n_seg;
  sg.n_genomes = n_genomes;
  return c.cur <= c.end;
}

// The segmented tail gives each (pair, genome) segment one wave, which takes
// the segment's sites 64 at a time: past a few hundred sites per segment the
// radix tail, which spreads every site over the whole device, is faster.  The
// expected random sites of a pair's segment on the longest genome (both
// primers, both strands) decide, against kSegExpected; AH_QUERY_SEGMENTED=1
// or 0 forces one tail (the segmented one still only up to kSegMax segments).
constexpr double kSegExpected = 512.0;
bool seg_mode(const ah_primer_pair* pairs, uint32_t n_pairs, uint32_t max_len) {
  const char* e = getenv("AH_QUERY_SEGMENTED");
  if (e && e[0] == '0') return false;
  if (e && e[0] == '1') return true;
  for (uint32_t q = 0; q < n_pairs; ++q) {
    const double rate = 2.0 * (ah::site_probability(pairs[q].fwd, pairs[q].k, pairs[q].clamp) +
                               ah::site_probability(pairs[q].rev, pairs[q].k, pairs[q].clamp));
    if (rate * (double)max_len > kSegExpected) return false;
  }
  return true;
}

// Reset of d_res, tile counts and prefix, then the filter, the exact count
// and the emit pass, which writes the sites to the staging area in slice
// order, the final d_res (required, count, status), n_sort and the
// candidate-list statistics.  With seg set, the segmented emit instead puts
// the sites of each segment (pair, genome) together (n_sort is not written).
ah_status launch_scan_kernel(const ScanFns& fn, Tuning tn, const ah_genomes* g, const ScanWs& w,
                             ah_result* d_res, uint64_t capacity, hipStream_t st,
                             const ah::KeyBits* kb, const ah::SegBuffers* seg = nullptr) {
  if (g->n == 0) {
    AH_HIP(ah::launch_result_init(d_res, st));
    AH_HIP(ah::launch_zero_u64(w.cstat, 4, st));
    AH_HIP(ah::launch_zero_u64(w.n_sort, 1, st));
    return AH_OK;
  }
  // window words per tile: a workgroup's in tile mode, a wave's (63 lanes
  // with windows) in wave mode
  const uint32_t tile = fn.wave ? (uint32_t)(63 * tn.u) : (uint32_t)(ah::kBlock * tn.u);
  // persistent grid, no larger than an upper bound on the tiles (so that small
  // inputs get long slices); each workgroup owns ccap / grid records
  const uint64_t words_ub = ((uint64_t)g->max_len + 31) / 32;
  const uint64_t tiles_ub = (uint64_t)g->n * ((words_ub + tile - 1) / tile);
  // wave mode: as many workgroups as are resident at once (LDS bound: four
  // wave slices of 32 U + 1 16-byte pairs each), so that every wave keeps
  // its slice busy until the tiles run out; at most one tile per wave
  const uint64_t wave_res = fn.wave ? std::max<uint64_t>(1, kLdsPerCu / (4ull * (32 * tn.u + 1) * 16)) : 8;
  const uint64_t want = fn.wave ? (tiles_ub + 3) / 4 : tiles_ub;
  const unsigned grid = (unsigned)std::max<uint64_t>(
      1, std::min<uint64_t>({(uint64_t)cu_count() * wave_res, want,
                             fn.wave ? kMaxScanGrid / 4 : kMaxScanGrid}));
  // the sums of the groups of 64 slices, cleared before the filter (in wave
  // mode its waves add to them as they finish)
  const uint32_t group_words = (grid + 63) / 64 * 32;
  if (g->n <= ah::kSmallPrefix) {  // one launch, result reset and clearing included
    AH_HIP(ah::launch_tile_prefix_small(g->len, g->n, tile, w.tile_prefix, d_res, st,
                                        seg ? seg->cnt : nullptr, seg ? 4 * seg->n_seg : 0,
                                        w.group_sites, group_words));
  } else {
    if (seg) AH_HIP(ah::launch_zero_u64((uint64_t*)seg->cnt, 2 * seg->n_seg, st));
    AH_HIP(ah::launch_zero_u64(w.group_sites, group_words, st));
    AH_HIP(ah::launch_result_init(d_res, st));
    AH_HIP(ah::launch_tile_counts(g->len, g->n, tile, w.counts, st));
    AH_HIP(ah::launch_exclusive_scan(w.counts, w.tile_prefix, g->n, nullptr, w.scan_tmp, st));
  }
  // candidate slices: one per workgroup, one per wave in wave mode
  const unsigned n_slices = fn.wave ? grid * 4u : grid;
  const void* words = g->words;
  const uint32_t* nmask = g->nmask;
  const uint64_t* word_off = g->word_off;
  const uint32_t* len = g->len;
  const uint64_t* tp = w.tile_prefix;
  uint32_t n = g->n;
  uint4* cands = w.cands;
  uint32_t slice = (uint32_t)std::min<uint64_t>(w.ccap / n_slices, 0xffffffffu);
  uint32_t* slice_cnt = w.slice_cnt;
  uint32_t* slice_tot = w.slice_tot;
  uint64_t* slice_win = w.slice_win;
  uint64_t* group_sites = w.group_sites;
  uint32_t* cand_sites = w.cand_sites;
  uint64_t* slice_sites = w.slice_sites;
  // the sort's start (kb set): emit writes the keys and counts the first
  // digit into hist[0]; the exact count (in the filter in wave mode) clears
  // hist[0] and hist[1] before
  const int dbits = kb ? ah::sort_digit_bits(*kb) : 0;
  uint64_t* sort_keys = kb ? (uint64_t*)w.sb.keys[0] : nullptr;
  uint32_t* sort_idx = kb ? w.sb.idx[0] : nullptr;
  uint32_t* hist_a = kb ? w.sb.hist[0] : nullptr;
  uint32_t* hist_b = kb ? w.sb.hist[1] : nullptr;
  uint64_t hist_words = kb ? ((uint64_t)1 << dbits) * w.sb.hstride : 0;
  uint32_t sort_hs = w.sb.hstride;
  uint32_t sort_dmask = kb ? (1u << dbits) - 1u : 0u;
  uint32_t sort_gshift = kb ? (uint32_t)(kb->pb + 2) : 0u;
  uint32_t sort_qshift = kb ? (uint32_t)(kb->gb + kb->pb + 2) : 0u;
  uint32_t sort_grid = (uint32_t)ah::kSortGrid;
  uint32_t sort_chunk_min = ah::kSortChunkMin;
  uint32_t* seg_cnt = seg ? seg->cnt : nullptr;
  uint32_t seg_n = seg ? seg->n_genomes : 0;
  void* args[] = {&words,      &nmask,      &word_off,   &len,         &tp,
                  &n,          &cands,      &slice,      &slice_cnt,   &slice_tot,
                  &slice_win,  &group_sites, &cand_sites, &slice_sites, &hist_a,
                  &hist_b,     &hist_words, &seg_cnt,    &seg_n};
  {
    ProfScope prof_scan("scan", st);
    AH_HIP(hipModuleLaunchKernel(fn.scan, grid, 1, 1, ah::kBlock, 1, 1, 0, st, args, nullptr));
  }
  const uint4* ccands = w.cands;
  const uint32_t* cslice_cnt = w.slice_cnt;
  void* vargs[] = {&words,      &nmask,      &word_off,    &len,         &ccands,    &slice,
                   &cslice_cnt, &cand_sites, &slice_sites, &group_sites, &slice_win, &hist_a,
                   &hist_b,     &hist_words, &seg_cnt,     &seg_n};
  {
    ProfScope prof_verify("verify", st);
    if (!fn.wave && !fn.tile_count)  // otherwise the filter counted its own candidates
      AH_HIP(hipModuleLaunchKernel(fn.verify, grid, 1, 1, ah::kBlock, 1, 1, 0, st, vargs, nullptr));
    if (seg) {
      const uint32_t* cslice_tot = w.slice_tot;
      const uint64_t* cslice_win = w.slice_win;
      const uint32_t* ccand_sites = w.cand_sites;
      const uint32_t* cseg_cnt = seg->cnt;
      uint32_t n_seg = seg->n_seg;
      uint64_t* seg_off = seg->off;
      uint32_t* seg_fill = seg->fill;
      ah_hit* out = w.staging;
      uint64_t cap = capacity;
      uint64_t* cstat = w.cstat;
      void* sargs[] = {&words,      &nmask,       &word_off, &len,      &ccands,
                       &slice,      &cslice_cnt,  &cslice_tot, &cslice_win, &ccand_sites,
                       &cseg_cnt,   &n_seg,       &seg_n,    &seg_off,  &seg_fill,
                       &out,        &cap,         &d_res,    &cstat};
      AH_HIP(hipModuleLaunchKernel(fn.emit_seg, grid, 1, 1, ah::kBlock, 1, 1, 0, st, sargs,
                                   nullptr));
      return AH_OK;
    }
    ah_hit* out = w.staging;
    uint64_t cap = capacity;
    const uint32_t* cslice_tot = w.slice_tot;
    const uint64_t* cslice_win = w.slice_win;
    const uint32_t* ccand_sites = w.cand_sites;
    const uint64_t* cslice_sites = w.slice_sites;
    const uint64_t* cgroup_sites = w.group_sites;
    uint64_t* n_out = w.n_sort;
    uint64_t* cstat = w.cstat;
    void* eargs[] = {&words,       &nmask,       &word_off,    &len,         &ccands,
                     &slice,       &cslice_cnt,  &cslice_tot,  &cslice_win,  &ccand_sites,
                     &cslice_sites, &cgroup_sites, &out,       &cap,         &d_res,
                     &n_out,       &cstat,       &sort_keys,   &sort_idx,    &hist_a,
                     &sort_hs,     &sort_dmask,  &sort_gshift, &sort_qshift, &sort_grid,
                     &sort_chunk_min};
    AH_HIP(hipModuleLaunchKernel(fn.emit, grid, 1, 1, ah::kBlock, 1, 1, 0, st, eargs, nullptr));
  }
  return AH_OK;
}

// Salt correction of the melting temperature, from the ion concentrations.
// Method 5 is an entropy term; 1-4 shift Tm; 6 (Owczarzy 2004) and 7
// (Owczarzy 2008, magnesium) add a + b fGC to 1/T, the terms derived here
// (a = a0 + a_len / (2 (N - 1)) for a primer of N bases).  Methods 1-6 take
// the sodium equivalent Na + K + Tris/2 + 120 sqrt(Mg - dNTPs) mM; method 7
// the monovalent ions Na + K + Tris/2 and the magnesium left free by 1:1
// binding to dNTPs (association constant 3e4 per M).
struct SaltTerms {
  bool ok = true;
  const char* why = "";
  double ln_na = 0.0;  // ln of the sodium equivalent in M (methods 1-6)
  double shift = 0.0;  // methods 1-4, degrees
  bool recip = false;  // methods 6, 7
  double a0 = 0.0, a_len = 0.0, b = 0.0;
};

SaltTerms salt_terms(const ah_tm_params& p) {
  SaltTerms r;
  const int m = p.saltcorr;
  if (m == 0) return r;
  const double mg_excess = p.Mg_mM - p.dNTPs_mM;
  const double na_eq =
      p.Na_mM + p.K_mM + p.Tris_mM / 2.0 + (mg_excess > 0 ? 120.0 * std::sqrt(mg_excess) : 0.0);
  // 1/T terms of Owczarzy et al. (2004) for a monovalent concentration in M
  auto mono = [&r](double molar) {
    const double ln = std::log(molar);
    r.recip = true;
    r.a0 = -3.95e-5 * ln + 9.40e-6 * ln * ln;
    r.b = 4.29e-5 * ln;
  };
  if (m <= 6) {
    if (!(na_eq > 0)) {
      r.ok = false;
      r.why = "needs a positive sodium equivalent";
      return r;
    }
    const double na = na_eq / 1000.0;
    r.ln_na = std::log(na);
    const double l10 = std::log10(na);
    if (m == 1) r.shift = 16.6 * l10;
    if (m == 2) r.shift = 16.6 * std::log10(na / (1.0 + 0.7 * na));
    if (m == 3) r.shift = 12.5 * l10;
    if (m == 4) r.shift = 11.7 * l10;
    if (m == 6) mono(na);
    return r;
  }
  const double mon = (p.Na_mM + p.K_mM + p.Tris_mM / 2.0) / 1000.0;
  double mg = p.Mg_mM > 0 ? p.Mg_mM / 1000.0 : 0.0;
  const double dn = p.dNTPs_mM / 1000.0;
  if (mg > 0 && dn > 0) {  // free Mg: Ka x^2 + (Ka (D - M) + 1) x - M = 0
    const double ka = 3e4, q = ka * (dn - mg) + 1.0;
    mg = (-q + std::sqrt(q * q + 4.0 * ka * mg)) / (2.0 * ka);
  }
  if (!(mon > 0) && !(mg > 0)) {
    r.ok = false;
    r.why = "needs monovalent ions or free magnesium";
    return r;
  }
  if (!(mg > 0) || (mon > 0 && std::sqrt(mg) / mon < 0.22)) {
    mono(mon);
    return r;
  }
  double a = 3.92e-5, b = -9.11e-6, c = 6.26e-5, d = 1.42e-5, e = -4.82e-4, f = 5.25e-4,
         g = 8.31e-5;
  if (mon > 0 && std::sqrt(mg) / mon < 6.0) {
    const double lm = std::log(mon);
    a *= 0.843 - 0.352 * std::sqrt(mon) * lm;
    d *= 1.279 - 4.03e-3 * lm - 8.03e-3 * lm * lm;
    g *= 0.486 - 0.258 * lm + 5.25e-3 * lm * lm * lm;
  }
  const double lg = std::log(mg);
  r.recip = true;
  r.a0 = a + b * lg;
  r.a_len = e + f * lg + g * lg * lg;
  r.b = c + d * lg;
  return r;
}

// Total strand concentration in M entering R ln C: dnac1 for a
// self-complementary duplex, else max - min / 2 of the two strands.
double strand_conc(const ah_tm_params& p) {
  if (p.selfcomp) return p.dnac1_nM * 1e-9;
  const double hi = p.dnac1_nM > p.dnac2_nM ? p.dnac1_nM : p.dnac2_nM;
  const double lo = p.dnac1_nM > p.dnac2_nM ? p.dnac2_nM : p.dnac1_nM;
  return (hi - lo / 2.0) * 1e-9;
}

// SantaLucia (1998) unified nearest-neighbour stacks in double precision for
// the host-side duplex helper, indexed by (5' base * 4 + 3' base) of the
// stack read on the oligo strand (A0 C1 G2 T3): Delta-H in kcal/mol and
// Delta-S in cal/(K mol).  A stack and the one read on the other strand
// (e.g. AC and GT) share their values.
const double kNnH[16] = {-7.9, -8.4, -7.8, -7.2, -8.5, -8.0, -10.6, -7.8,
                         -8.2, -9.8, -8.0, -8.4, -7.2, -8.2, -8.5, -7.9};
const double kNnS[16] = {-22.2, -22.4, -21.0, -20.4, -22.7, -19.9, -27.2, -21.0,
                         -22.2, -24.4, -19.9, -22.4, -21.3, -22.2, -22.7, -22.2};

int base_code(char ch) {
  switch (ch) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
  }
}

// Pairings the Tm kernel evaluates per site at most for a primer: the
// representative oligo and every way of turning at most k of the degenerate
// non-clamp positions into mismatches (every position in its set is the
// worst case), sum over e <= min(k, nd) of C(nd, e).
uint64_t worst_tm_pairings(const Primer& pr, uint32_t k, uint32_t clamp) {
  uint32_t nd = 0;
  for (int j = 0; j < pr.L; ++j)
    if (set_size(pr.mask[j]) > 1 && j < pr.L - (int)clamp) ++nd;
  uint64_t sum = 0, c = 1;  // c = C(nd, e)
  for (uint32_t e = 0; e <= std::min(k, nd); ++e) {
    sum += c;
    c = c * (nd - e) / (e + 1);
  }
  return sum;
}

// Constant part of the Tm denominator for a primer of L bases, cal/(K mol):
// method 5's salt entropy, R ln C and the symmetry term.
double tm_denominator_const(const ah_tm_params& p, const SaltTerms& salt_t, int L) {
  const double salt = p.saltcorr == 5 ? 0.368 * (L - 1) * salt_t.ln_na : 0.0;
  return salt + 1.987 * std::log(strand_conc(p)) + (p.selfcomp ? -1.4 : 0.0);
}

// The largest Delta-S a set of paired positions can have: two A.T
// initiations and no stack (every stack's Delta-S is negative).
constexpr double kMaxPairingDs = 8.2;

// AH_TM_EXACT=1 sends every primer the exact route can take there (salt
// methods 0-5), not only those above the enumeration bound.
bool tm_exact_forced() {
  const char* e = std::getenv("AH_TM_EXACT");
  return e && e[0] == '1';
}

// Whether the route applies: a Tm that depends on the pairing alone and a
// negative denominator for every pairing.
bool tm_exact_applies(const ah_tm_params& p, const SaltTerms& salt_t, int L) {
  return !salt_t.recip && tm_denominator_const(p, salt_t, L) + kMaxPairingDs < 0.0;
}

// Whether the Tm kernels take a primer's best pairing by the exact ratio
// iteration rather than by enumerating its pairings (a request above the
// bound where it does not apply is refused by check_tm_request).
bool tm_exact_route(const Primer& pr, uint32_t k, uint32_t clamp, const ah_tm_params& p,
                    const SaltTerms& salt_t) {
  if (!tm_exact_applies(p, salt_t, pr.L)) return false;
  return worst_tm_pairings(pr, k, clamp) > (uint64_t)AH_TM_MAX_PAIRINGS || tm_exact_forced();
}

// Everything ah_tm checks before any device work: the pairs, the salt
// method and its ion concentrations, a positive strand concentration, and
// for a primer above the enumeration bound what the exact route needs: a
// salt method whose Tm depends on the pairing alone (not 6 or 7) and a
// denominator that stays negative for every pairing.
ah_status check_tm_request(const ah_primer_pair* pairs, uint32_t n_pairs, const ah_tm_params* p,
                           PairSet& ps) {
  ah_status s = compile_pairs(pairs, n_pairs, ps);
  if (s) return s;
  if (!p) return fail(AH_ERR_INVALID_ARG, "Tm parameters are required");
  if (p->saltcorr < 0 || p->saltcorr > 7)
    return fail(AH_ERR_INVALID_ARG, "salt correction method %d (supported: 0-7)", p->saltcorr);
  const SaltTerms salt_t = salt_terms(*p);
  if (!salt_t.ok)
    return fail(AH_ERR_INVALID_ARG, "salt correction %d: %s", p->saltcorr, salt_t.why);
  if (!(strand_conc(*p) > 0)) return fail(AH_ERR_INVALID_ARG, "strand concentration must be positive");
  for (uint32_t q = 0; q < n_pairs; ++q)
    for (int primer = 0; primer < 2; ++primer) {
      const Primer& pr = primer ? ps.rev[q] : ps.fwd[q];
      const uint64_t w = worst_tm_pairings(pr, ps.k[q], ps.clamp[q]);
      if (w <= (uint64_t)AH_TM_MAX_PAIRINGS) continue;
      if (salt_t.recip)
        return fail(AH_ERR_LIMIT,
                    "pair %u: up to %llu pairings per site for Tm (at most %d under salt method %d, "
                    "whose Tm also depends on the oligo's G+C count: lower k, or the degenerate "
                    "positions outside the clamp, or use a method of 0-5)",
                    q, (unsigned long long)w, (int)AH_TM_MAX_PAIRINGS, p->saltcorr);
      if (!(tm_denominator_const(*p, salt_t, pr.L) + kMaxPairingDs < 0.0))
        return fail(AH_ERR_LIMIT,
                    "pair %u: up to %llu pairings per site for Tm, whose exact route needs "
                    "R ln C + salt entropy < -%.1f cal/(K mol) (a lower strand concentration)",
                    q, (unsigned long long)w, kMaxPairingDs);
    }
  return AH_OK;
}

// The Tm kernel's per-primer tables of a validated request (check_tm_request),
// uploaded once per content (get_table); *exact: some primer takes the exact
// route (the kernels' variant that carries it).
ah_status tm_table(const PairSet& ps, uint32_t n_pairs, const ah_tm_params& pp, void** dt,
                   bool* exact) {
  const ah_tm_params* p = &pp;
  const SaltTerms salt_t = salt_terms(*p);
  bool any_exact = false;
  std::vector<ah::PrimerTab> tabs(2 * (size_t)n_pairs);
  for (uint32_t q = 0; q < n_pairs; ++q) {
    for (int primer = 0; primer < 2; ++primer) {
      const Primer& pr = primer ? ps.rev[q] : ps.fwd[q];
      ah::PrimerTab t;
      memset(&t, 0, sizeof t);
      t.L = (uint32_t)pr.L;
      t.k = ps.k[q];
      uint64_t deg = 1;
      for (int j = 0; j < pr.L; ++j) {
        const uint8_t m = pr.mask[j];
        const int cnt = __builtin_popcount(m);
        t.lanes |= 1ull << (2 * j);
        if (j < pr.L - 1) t.stackm |= 1ull << (2 * j);
        if (cnt == 1) {
          t.fixed |= (uint64_t)__builtin_ctz(m) << (2 * j);
        } else {
          uint8_t packed = 0;
          int r = 0;
          for (int b = 0; b < 4; ++b)
            if (m >> b & 1) packed |= (uint8_t)(b << (2 * r++));
          t.dpos[t.nd] = (uint8_t)j;
          t.nmem[t.nd] = (uint8_t)cnt;
          t.mem[t.nd] = packed;
          t.nd++;
          deg = deg > (~0ull >> 2) ? ~0ull : deg * (uint64_t)cnt;  // saturates
        }
      }
      for (uint32_t j = 0; j < ps.clamp[q]; ++j) t.clampm |= 1ull << (2 * (pr.L - 1 - (int)j));
      t.deg = deg;
      t.decoy = (ps.flags[q] & AH_PAIR_DECOY) ? 1u : 0u;
      t.KL = tm_denominator_const(*p, salt_t, pr.L);
      t.dp = tm_exact_route(pr, ps.k[q], ps.clamp[q], *p, salt_t) ? 1u : 0u;
      any_exact |= t.dp != 0u;
      t.tshift = salt_t.shift;
      if (salt_t.recip) {
        t.recip = 1;
        t.rA = salt_t.a0 + salt_t.a_len / (2.0 * (pr.L - 1));
        t.rB = salt_t.b;
      }
      tabs[2 * q + primer] = t;
    }
  }
  *exact = any_exact;
  return get_table(tabs.data(), tabs.size() * sizeof(ah::PrimerTab), dt);
}

// The pairing kernels' per-pair table (primer lengths, window, Tm filter),
// uploaded once per content.
ah_status pair_table(const PairSet& ps, const ah_window* windows, uint32_t n_pairs, void** dt) {
  std::vector<ah::PairTab> tabs(n_pairs);
  for (uint32_t q = 0; q < n_pairs; ++q) {
    if (windows[q].min_len > windows[q].max_len)
      return fail(AH_ERR_INVALID_ARG, "pair %u: min_len > max_len", q);
    tabs[q].lf = (uint32_t)ps.fwd[q].L;
    tabs[q].lr = (uint32_t)ps.rev[q].L;
    tabs[q].min_len = windows[q].min_len;
    tabs[q].max_len = windows[q].max_len;
    tabs[q].filter_tm = windows[q].filter_tm ? 1 : 0;
    tabs[q].min_tm = windows[q].min_tm;
  }
  return get_table(tabs.data(), tabs.size() * sizeof(ah::PairTab), dt);
}

}  // namespace

namespace ah {
// Members of an IUPAC code (0 for anything else; primers are validated first).
static int code_size(char c) {
  switch (c | 0x20) {
    case 'a': case 'c': case 'g': case 't': return 1;
    case 'r': case 'y': case 's': case 'w': case 'k': case 'm': return 2;
    case 'b': case 'd': case 'h': case 'v': return 3;
    case 'n': return 4;
    default: return 0;
  }
}

// A Poisson-binomial over the non-clamp positions (each mismatches with
// chance 1 - |set| / 4), times the clamp's chance to match.
double site_probability(const std::string& primer, uint32_t k, uint32_t clamp) {
  const int L = (int)primer.size();
  const int free_len = L - (int)std::min<uint32_t>(clamp, (uint32_t)L);
  std::vector<double> d(L + 2, 0.0);
  d[0] = 1.0;
  for (int j = 0; j < free_len; ++j) {
    const double p = code_size(primer[j]) / 4.0;
    for (int m = j + 1; m >= 1; --m) d[m] = d[m] * p + d[m - 1] * (1.0 - p);
    d[0] *= p;
  }
  double pk = 0.0;
  for (int m = 0; m <= (int)k && m <= L; ++m) pk += d[m];
  for (int j = free_len; j < L; ++j) pk *= code_size(primer[j]) / 4.0;
  return pk;
}

ah_status check_tm(const ah_primer_pair* pairs, uint32_t n_pairs, const ah_tm_params* p) {
  PairSet ps;
  return check_tm_request(pairs, n_pairs, p, ps);
}

size_t scan_workspace_for(uint32_t n, uint64_t window_words, const ah_primer_pair* pairs,
                          uint32_t n_pairs, uint64_t capacity) {
  uint64_t ccap = min_cands(capacity);
  PairSet ps;
  if (pairs && n_pairs) {
    const std::string saved = g_err;  // a sizing query reports no error
    if (compile_pairs(pairs, n_pairs, ps) == AH_OK)
      ccap = recommended_cands(window_words, cand_per_word(patterns_of(ps)), capacity);
    g_err = saved;
  }
  return scan_ws_bytes(n, capacity, ccap);
}

ah_status set_error(ah_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}
void clear_error() { g_err.clear(); }
int cu_count_current() { return cu_count(); }
}  // namespace ah

// =================================================================== C ABI
extern "C" {

const char* ah_status_str(int s) {
  switch (s) {
    case AH_OK: return "ok";
    case AH_ERR_INVALID_ARG: return "invalid argument";
    case AH_ERR_INVALID_PRIMER: return "invalid primer";
    case AH_ERR_LIMIT: return "limit exceeded";
    case AH_ERR_OVERFLOW: return "output capacity exceeded";
    case AH_ERR_WORKSPACE: return "workspace too small";
    case AH_ERR_HIP: return "HIP error";
    case AH_ERR_JIT: return "scan specialisation failed";
    case AH_ERR_AGAIN: return "not ready";
    default: return "unknown status";
  }
}

const char* ah_last_error(void) { return g_err.c_str(); }

void ah_jit_stats(uint64_t* n, double* ms) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (n) *n = g_jit_n;
  if (ms) *ms = g_jit_ms;
}

void ah_release_caches(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_jit) (void)hipModuleUnload(kv.second.mod);
  g_jit.clear();
  g_fns.clear();
  for (auto& kv : g_tables) (void)hipFree(kv.second);
  g_tables.clear();
}

uint64_t ah_pack_layout(const uint64_t* h_len, uint32_t n, uint64_t* h_word_off) {
  g_err.clear();
  if (h_len)
    for (uint32_t g = 0; g < n; ++g)
      if (h_len[g] > 0xffffffffull) {
        fail(AH_ERR_INVALID_ARG, "genome %u has %llu bases; at most 2^32 - 1 are supported", g,
             (unsigned long long)h_len[g]);
        return UINT64_MAX;
      }
  uint64_t off = 0;
  if (h_word_off) h_word_off[0] = 0;
  for (uint32_t g = 0; g < n; ++g) {
    const uint64_t S = h_len ? (h_len[g] + 31) / 32 : 0;
    off += (S + AH_HALO_WORDS + 1) & ~(uint64_t)1;  // even: every genome 16-byte aligned
    if (h_word_off) h_word_off[g + 1] = off;
  }
  return off;
}

ah_status ah_pack_genomes(const uint8_t* d_ascii, const uint64_t* d_ascii_off, uint32_t n,
                          const uint64_t* d_word_off, uint32_t* d_words, uint32_t* d_len,
                          uint32_t* d_nmask, uint64_t* d_non_acgt, void* stream) {
  g_err.clear();
  if (n == 0) return AH_OK;
  if (!d_ascii || !d_ascii_off || !d_word_off || !d_words || !d_len)
    return fail(AH_ERR_INVALID_ARG, "ah_pack_genomes: null device pointer");
  const int grid = cu_count() * 8;
  ProfScope prof_pack("pack", (hipStream_t)stream);
  AH_HIP(ah::launch_pack(d_ascii, d_ascii_off, n, d_word_off, d_words, d_len, d_nmask, d_non_acgt,
                         grid, (hipStream_t)stream));
  return AH_OK;
}

size_t ah_scan_workspace_bytes(const ah_genomes* g, const ah_primer_pair* pairs, uint32_t n_pairs,
                               uint64_t capacity) {
  const uint32_t n = g ? g->n : 0;
  const uint64_t words = g ? (uint64_t)n * (((uint64_t)g->max_len + 31) / 32) : 0;
  return ah::scan_workspace_for(n, words, pairs, n_pairs, capacity);
}

ah_status ah_scan_primers(const ah_genomes* g, const ah_primer_pair* pairs, uint32_t n_pairs,
                          ah_hit* d_hits, uint64_t capacity, ah_result* d_res, void* d_work,
                          size_t work_bytes, void* stream) {
  g_err.clear();
  ah_status s = check_genomes(g);
  if (s) return s;
  if (!d_res) return fail(AH_ERR_INVALID_ARG, "d_res is NULL");
  if (capacity > 0 && !d_hits) return fail(AH_ERR_INVALID_ARG, "d_hits is NULL");
  if (capacity >= (1ull << 32)) return fail(AH_ERR_LIMIT, "hit capacity must be < 2^32");
  PairSet ps;
  s = compile_pairs(pairs, n_pairs, ps);
  if (s) return s;
  ah::KeyBits kb{bits_for(n_pairs - 1), bits_for(g->n ? g->n - 1 : 0), bits_for(g->max_len)};
  if (kb.total() > 64) return fail(AH_ERR_LIMIT, "sort key needs %d > 64 bits", kb.total());
  const size_t need = scan_ws_bytes(g->n, capacity, min_cands(capacity));
  if (!d_work || work_bytes < need)
    return fail(AH_ERR_WORKSPACE, "scan workspace: %zu bytes given, %zu needed", work_bytes, need);
  const Tuning tn = tuning_for(pairs, n_pairs);
  ScanFns fn;
  s = scan_kernels_for(pairs, n_pairs, ps, g->nmask != nullptr, tn, fn);
  if (s) return s;

  hipStream_t st = (hipStream_t)stream;
  Carver c(d_work, work_bytes);
  ScanWs w = carve_scan(c, g->n, capacity, 0);
  // the result, the records to sort (n_sort) and the candidate statistics
  s = launch_scan_kernel(fn, tn, g, w, d_res, capacity, st, &kb);
  if (s) return s;
  ProfScope prof_sort("sort", st);
  AH_HIP(ah::launch_sort_hits(w.staging, d_hits, w.n_sort, kb, w.sb, st));
  return AH_OK;
}

ah_status ah_scan_primers_noalloc(const ah_genomes* g, const ah_primer_pair* pairs,
                                  uint32_t n_pairs, ah_hit* d_hits, uint64_t capacity,
                                  ah_result* d_res, void* stream) {
  g_err.clear();
  ah_status s = check_genomes(g);
  if (s) return s;
  if (!d_res) return fail(AH_ERR_INVALID_ARG, "d_res is NULL");
  if (capacity > 0 && !d_hits) return fail(AH_ERR_INVALID_ARG, "d_hits is NULL");
  if (capacity >= (1ull << 32)) return fail(AH_ERR_LIMIT, "hit capacity must be < 2^32");
  PairSet ps;
  s = compile_pairs(pairs, n_pairs, ps);
  if (s) return s;
  ah::KeyBits kb{bits_for(n_pairs - 1), bits_for(g->n ? g->n - 1 : 0), bits_for(g->max_len)};
  if (kb.total() > 64) return fail(AH_ERR_LIMIT, "sort key needs %d > 64 bits", kb.total());
  const size_t need = scan_ws_bytes(g->n, capacity, min_cands(capacity));
  if (need > (size_t)AH_SCAN_SCRATCH_BYTES)
    return fail(AH_ERR_WORKSPACE,
                "ah_scan_primers_noalloc: %u genomes and capacity %llu need %zu bytes of "
                "workspace; the scratch array holds %d",
                g->n, (unsigned long long)capacity, need, (int)AH_SCAN_SCRATCH_BYTES);
  const Tuning tn = tuning_for(pairs, n_pairs);
  ScanFns fn;
  if (!find_scan_kernels(pairs, n_pairs, ps, g->nmask != nullptr, tn, fn))
    return fail(AH_ERR_INVALID_ARG,
                "ah_scan_primers_noalloc: this primer set's kernels are not loaded on the current "
                "device (ah_scan_prepare compiles and loads them)");
  void* scratch = nullptr;
  AH_HIP(ah::scan_scratch(&scratch));
  struct NoProf {  // no profiling events: creating them is not allowed here
    bool was;
    NoProf() : was(t_prof_off) { t_prof_off = true; }
    ~NoProf() { t_prof_off = was; }
  } no_prof;
  hipStream_t st = (hipStream_t)stream;
  Carver c(scratch, (size_t)AH_SCAN_SCRATCH_BYTES);
  ScanWs w = carve_scan(c, g->n, capacity, 0);
  s = launch_scan_kernel(fn, tn, g, w, d_res, capacity, st, &kb);
  if (s) return s;
  AH_HIP(ah::launch_sort_hits(w.staging, d_hits, w.n_sort, kb, w.sb, st));
  return AH_OK;
}

ah_status ah_tm(const ah_genomes* g, const ah_primer_pair* pairs, uint32_t n_pairs,
                const ah_tm_params* p, ah_hit* d_hits, const ah_result* d_nhits, uint64_t capacity,
                void* stream) {
  g_err.clear();
  ah_status s = check_genomes(g);
  if (s) return s;
  if (!p || !d_nhits) return fail(AH_ERR_INVALID_ARG, "ah_tm: params and d_nhits are required");
  if (capacity > 0 && !d_hits) return fail(AH_ERR_INVALID_ARG, "d_hits is NULL");
  PairSet ps;
  s = check_tm_request(pairs, n_pairs, p, ps);
  if (s) return s;
  void* dt = nullptr;
  bool exact = false;
  s = tm_table(ps, n_pairs, *p, &dt, &exact);
  if (s) return s;
  ProfScope prof_tm("tm", (hipStream_t)stream);
  AH_HIP(ah::launch_tm(*g, (const ah::PrimerTab*)dt, n_pairs, d_hits, d_nhits, capacity,
                       cu_count() * 4, exact, (hipStream_t)stream));
  return AH_OK;
}

ah_status ah_tm_duplex(const char* oligo, const char* opposite, const ah_tm_params* p,
                       double* tm_c) {
  g_err.clear();
  if (!oligo || !opposite || !p || !tm_c)
    return fail(AH_ERR_INVALID_ARG, "ah_tm_duplex: oligo, opposite, params and tm_c are required");
  const size_t n = strlen(oligo);
  if (strlen(opposite) != n)
    return fail(AH_ERR_INVALID_ARG, "ah_tm_duplex: oligo (%zu) and opposite (%zu) differ in length",
                n, strlen(opposite));
  if (n < 2 || n > AH_TM_DUPLEX_MAX_LEN)
    return fail(AH_ERR_LIMIT, "ah_tm_duplex: length %zu outside 2..%d", n, AH_TM_DUPLEX_MAX_LEN);
  if (p->saltcorr < 0 || p->saltcorr > 7)
    return fail(AH_ERR_INVALID_ARG, "salt correction method %d (supported: 0-7)", p->saltcorr);
  const SaltTerms salt_t = salt_terms(*p);
  if (!salt_t.ok)
    return fail(AH_ERR_INVALID_ARG, "salt correction %d: %s", p->saltcorr, salt_t.why);
  const double C = strand_conc(*p);
  if (!(C > 0)) return fail(AH_ERR_INVALID_ARG, "strand concentration must be positive");
  std::vector<int> o(n);
  std::vector<char> paired(n);
  int gc = 0;
  for (size_t j = 0; j < n; ++j) {
    o[j] = base_code(oligo[j]);
    if (o[j] < 0)
      return fail(AH_ERR_INVALID_PRIMER, "ah_tm_duplex: oligo byte %zu ('%c') is not A/C/G/T", j,
                  oligo[j]);
    const int t = base_code(opposite[j]);
    paired[j] = t >= 0 && t == 3 - o[j];  // opposite base is the complement
    gc += o[j] == 1 || o[j] == 2;
  }
  // Stacks whose two pairs both form, then one initiation term per duplex
  // end at the outermost formed pairs (none if no pair forms).
  double dh = 0.0, ds = 0.0;
  int lo = -1, hi = -1;
  for (size_t j = 0; j < n; ++j) {
    if (!paired[j]) continue;
    if (lo < 0) lo = (int)j;
    hi = (int)j;
    if (j + 1 < n && paired[j + 1]) {
      dh += kNnH[o[j] * 4 + o[j + 1]];
      ds += kNnS[o[j] * 4 + o[j + 1]];
    }
  }
  if (lo >= 0) {
    for (int end : {lo, hi}) {
      const bool g_or_c = o[end] == 1 || o[end] == 2;
      dh += g_or_c ? 0.1 : 2.3;
      ds += g_or_c ? -2.8 : 4.1;
    }
  }
  if (p->saltcorr == 5) ds += 0.368 * (double)(n - 1) * salt_t.ln_na;
  if (p->selfcomp) ds += -1.4;
  double tm = 1000.0 * dh / (ds + 1.987 * std::log(C)) - 273.15;
  if (salt_t.recip) {
    const double rA = salt_t.a0 + salt_t.a_len / (2.0 * (double)(n - 1));
    tm = 1.0 / (1.0 / (tm + 273.15) + rA + salt_t.b * (double)gc / (double)n) - 273.15;
  }
  *tm_c = tm + salt_t.shift;
  return AH_OK;
}

ah_status ah_query(const ah_genomes* g, const ah_primer_pair* pairs, const ah_window* windows,
                   uint32_t n_pairs, const ah_tm_params* tm, ah_hit* d_hits, uint64_t hit_capacity,
                   ah_result* d_hit_res, ah_amplicon* d_amp, uint64_t amp_capacity,
                   ah_result* d_amp_res, void* d_scan_work, size_t scan_work_bytes,
                   void* d_pair_work, size_t pair_work_bytes, void* stream) {
  g_err.clear();
  ah_status s = check_genomes(g);
  if (s) return s;
  if (!d_hit_res || !d_amp_res || !windows || !tm)
    return fail(AH_ERR_INVALID_ARG, "ah_query: results, windows and Tm parameters are required");
  if (hit_capacity > 0 && !d_hits) return fail(AH_ERR_INVALID_ARG, "d_hits is NULL");
  if (amp_capacity > 0 && !d_amp) return fail(AH_ERR_INVALID_ARG, "d_amp is NULL");
  if (hit_capacity >= (1ull << 32)) return fail(AH_ERR_LIMIT, "hit capacity must be < 2^32");
  PairSet ps;
  s = check_tm_request(pairs, n_pairs, tm, ps);
  if (s) return s;
  for (uint32_t q = 0; q < n_pairs; ++q)
    if (windows[q].min_len > windows[q].max_len)
      return fail(AH_ERR_INVALID_ARG, "pair %u: min_len > max_len", q);
  ah::KeyBits kb{bits_for(n_pairs - 1), bits_for(g->n ? g->n - 1 : 0), bits_for(g->max_len)};
  if (kb.total() > 64) return fail(AH_ERR_LIMIT, "sort key needs %d > 64 bits", kb.total());
  const size_t sneed = scan_ws_bytes(g->n, hit_capacity, min_cands(hit_capacity));
  if (!d_scan_work || scan_work_bytes < sneed)
    return fail(AH_ERR_WORKSPACE, "scan workspace: %zu bytes given, %zu needed", scan_work_bytes,
                sneed);
  const size_t pneed = ah_pair_workspace_bytes(hit_capacity, n_pairs);
  if (!d_pair_work || pair_work_bytes < pneed)
    return fail(AH_ERR_WORKSPACE, "pair workspace: %zu bytes given, %zu needed", pair_work_bytes,
                pneed);
  void* tm_tabs = nullptr;
  bool exact = false;
  s = tm_table(ps, n_pairs, *tm, &tm_tabs, &exact);
  if (s) return s;
  void* pair_tabs = nullptr;
  s = pair_table(ps, windows, n_pairs, &pair_tabs);
  if (s) return s;
  const Tuning tn = tuning_for(pairs, n_pairs);
  ScanFns fn;
  s = scan_kernels_for(pairs, n_pairs, ps, g->nmask != nullptr, tn, fn);
  if (s) return s;

  hipStream_t st = (hipStream_t)stream;
  Carver c(d_scan_work, scan_work_bytes);
  ScanWs w = carve_scan(c, g->n, hit_capacity, 0);
  Carver cp(d_pair_work, pair_work_bytes);
  ah::PairBuffers pb = carve_pair(cp, hit_capacity);
  const auto* ttab = (const ah::PrimerTab*)tm_tabs;
  const auto* ptab = (const ah::PairTab*)pair_tabs;
  ah::SegBuffers sg{};
  if (g->n > 0 && seg_mode(pairs, n_pairs, g->max_len) &&
      carve_seg(w, g->n, (uint64_t)n_pairs * g->n, sg)) {
    // each segment (pair, genome) sorted, its Tm and amplicons, by one workgroup
    s = launch_scan_kernel(fn, tn, g, w, d_hit_res, hit_capacity, st, nullptr, &sg);
    if (s) return s;
    ProfScope prof_sort("sort", st);
    AH_HIP(ah::launch_seg_tail(w.staging, d_hits, hit_capacity, sg, d_hit_res, kb.pb + 2, *g, ttab,
                               n_pairs, ptab, pb, d_amp, amp_capacity, d_amp_res, exact, st));
    return AH_OK;
  }
  s = launch_scan_kernel(fn, tn, g, w, d_hit_res, hit_capacity, st, &kb);
  if (s) return s;
  bool marked = false;
  {
    ProfScope prof_sort("sort", st);
    if (ah::sort_fusable(kb)) {  // Tm and the pairing's first step inside the sort
      AH_HIP(ah::launch_sort_tm_mark(w.staging, d_hits, w.n_sort, kb, w.sb, *g, ttab, n_pairs, ptab,
                                     pb, cu_count() * 4, exact, st));
      marked = true;
    } else {
      AH_HIP(ah::launch_sort_hits(w.staging, d_hits, w.n_sort, kb, w.sb, st));
    }
  }
  if (!marked) {
    ProfScope prof_tm("tm", st);
    AH_HIP(ah::launch_tm(*g, ttab, n_pairs, d_hits, d_hit_res, hit_capacity, cu_count() * 4, exact,
                         st));
  }
  ProfScope prof_pair("pair", st);
  AH_HIP(ah::launch_pair(d_hits, d_hit_res, hit_capacity, ptab, d_amp, amp_capacity, d_amp_res, pb,
                         st, marked, true));
  return AH_OK;
}

size_t ah_pair_workspace_bytes(uint64_t hit_capacity, uint32_t n_pairs) {
  (void)n_pairs;
  Carver c(nullptr, 0);
  carve_pair(c, hit_capacity);
  return c.used();
}

ah_status ah_pair_amplicons(const ah_hit* d_hits, const ah_result* d_nhits, uint64_t hit_capacity,
                            const ah_primer_pair* pairs, const ah_window* windows, uint32_t n_pairs,
                            ah_amplicon* d_amp, uint64_t capacity, ah_result* d_res, void* d_work,
                            size_t work_bytes, void* stream) {
  g_err.clear();
  if (!d_nhits || !d_res || !windows) return fail(AH_ERR_INVALID_ARG, "ah_pair_amplicons: null argument");
  if (hit_capacity > 0 && !d_hits) return fail(AH_ERR_INVALID_ARG, "d_hits is NULL");
  if (capacity > 0 && !d_amp) return fail(AH_ERR_INVALID_ARG, "d_amp is NULL");
  if (hit_capacity >= (1ull << 32)) return fail(AH_ERR_LIMIT, "hit capacity must be < 2^32");
  PairSet ps;
  ah_status s = compile_pairs(pairs, n_pairs, ps);
  if (s) return s;
  for (uint32_t q = 0; q < n_pairs; ++q)
    if (windows[q].min_len > windows[q].max_len)
      return fail(AH_ERR_INVALID_ARG, "pair %u: min_len > max_len", q);
  const size_t need = ah_pair_workspace_bytes(hit_capacity, n_pairs);
  if (!d_work || work_bytes < need)
    return fail(AH_ERR_WORKSPACE, "pair workspace: %zu bytes given, %zu needed", work_bytes, need);
  void* dt = nullptr;
  s = pair_table(ps, windows, n_pairs, &dt);
  if (s) return s;
  Carver c(d_work, work_bytes);
  ah::PairBuffers pb = carve_pair(c, hit_capacity);
  ProfScope prof_pair("pair", (hipStream_t)stream);
  AH_HIP(ah::launch_pair(d_hits, d_nhits, hit_capacity, (const ah::PairTab*)dt, d_amp, capacity,
                         d_res, pb, (hipStream_t)stream));
  return AH_OK;
}

size_t ah_fasta_workspace_bytes(uint64_t amp_capacity) {
  Carver c(nullptr, 0);
  c.take<uint32_t>(amp_capacity ? amp_capacity : 1);
  c.take<uint64_t>(amp_capacity ? amp_capacity : 1);
  c.take<uint64_t>(ah::kPairGrid);
  return c.used();
}

ah_status ah_amplicon_fasta(const ah_genomes* g, const ah_hit* d_hits, const ah_amplicon* d_amp,
                            const ah_result* d_namp, uint64_t amp_capacity, uint32_t n_pairs,
                            char* d_text, uint64_t text_capacity, ah_result* d_text_res,
                            uint64_t* d_seq_hash, uint64_t* d_amplitype, uint32_t* d_amplitype_n,
                            void* d_work, size_t work_bytes, void* stream) {
  g_err.clear();
  ah_status s = check_genomes(g);
  if (s) return s;
  if (!d_namp || !d_text_res) return fail(AH_ERR_INVALID_ARG, "ah_amplicon_fasta: null result");
  if (amp_capacity > 0 && (!d_amp || !d_hits))
    return fail(AH_ERR_INVALID_ARG, "ah_amplicon_fasta: amplicons and hits are required");
  if (text_capacity > 0 && !d_text) return fail(AH_ERR_INVALID_ARG, "d_text is NULL");
  if ((d_amplitype || d_amplitype_n) && n_pairs == 0)
    return fail(AH_ERR_INVALID_ARG, "amplitypes need n_pairs >= 1");
  const size_t need = ah_fasta_workspace_bytes(amp_capacity);
  if (!d_work || work_bytes < need)
    return fail(AH_ERR_WORKSPACE, "fasta workspace: %zu bytes given, %zu needed", work_bytes, need);
  Carver c(d_work, work_bytes);
  uint32_t* rec_len = c.take<uint32_t>(amp_capacity ? amp_capacity : 1);
  uint64_t* rec_at = c.take<uint64_t>(amp_capacity ? amp_capacity : 1);
  uint64_t* cc = c.take<uint64_t>(ah::kPairGrid);
  // writers: up to 32 waves per CU, no more than the amplicons can use
  const uint64_t waves = std::min<uint64_t>(std::max<uint64_t>(amp_capacity, 1),
                                            (uint64_t)cu_count() * 32u);
  ProfScope prof("fasta", (hipStream_t)stream);
  AH_HIP(ah::launch_fasta(*g, d_hits, d_amp, d_namp, amp_capacity, n_pairs, d_text, text_capacity,
                          d_text_res, d_seq_hash, d_amplitype, d_amplitype_n, rec_len, rec_at, cc,
                          (int)waves, (hipStream_t)stream));
  return AH_OK;
}

// ------------------------------------------------------------ dev helpers
size_t ah_scan_program_source(const ah_primer_pair* pairs, uint32_t n_pairs, int has_nmask,
                              char* buf, size_t buf_bytes) {
  g_err.clear();
  PairSet ps;
  if (compile_pairs(pairs, n_pairs, ps)) return 0;
  const std::string src = gen_program(patterns_of(ps), has_nmask != 0, tuning_for(pairs, n_pairs));
  if (buf && buf_bytes) {
    const size_t n = src.size() < buf_bytes - 1 ? src.size() : buf_bytes - 1;
    memcpy(buf, src.data(), n);
    buf[n] = '\0';
  }
  return src.size() + 1;
}

ah_status ah_scan_program_compile(const ah_primer_pair* pairs, uint32_t n_pairs, int has_nmask,
                                  size_t* code_bytes) {
  g_err.clear();
  PairSet ps;
  ah_status s = compile_pairs(pairs, n_pairs, ps);
  if (s) return s;
  std::vector<char> code;
  s = rtc_compile(gen_program(patterns_of(ps), has_nmask != 0, tuning_for(pairs, n_pairs)), code);
  if (s) return s;
  if (code_bytes) *code_bytes = code.size();
  return AH_OK;
}

ah_status ah_scan_prepare(const ah_primer_pair* pairs, uint32_t n_pairs, int has_nmask) {
  g_err.clear();
  PairSet ps;
  ah_status s = compile_pairs(pairs, n_pairs, ps);
  if (s) return s;
  ScanFns fn;
  return get_scan_kernel(gen_program(patterns_of(ps), has_nmask != 0, tuning_for(pairs, n_pairs)),
                         fn);
}

ah_status ah_set_scan_tuning(const ah_primer_pair* pairs, uint32_t n_pairs,
                             const ah_scan_tuning* tuning) {
  g_err.clear();
  PairSet ps;
  ah_status s = compile_pairs(pairs, n_pairs, ps);
  if (s) return s;
  int dev = 0;
  AH_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  const auto key = std::make_pair(dev, set_key(pairs, n_pairs));
  if (!tuning) {
    g_tuning.erase(key);
    return AH_OK;
  }
  if (!valid_u((int)tuning->words_per_lane) || tuning->patterns_per_group < 1 ||
      tuning->patterns_per_group > 1024)
    return fail(AH_ERR_INVALID_ARG,
                "tuning: words_per_lane odd in 3..31, patterns_per_group in 1..1024");
  g_tuning[key] = Tuning{(int)tuning->words_per_lane, (int)tuning->patterns_per_group};
  return AH_OK;
}

ah_status ah_get_scan_tuning(const ah_primer_pair* pairs, uint32_t n_pairs, ah_scan_tuning* tuning) {
  g_err.clear();
  if (!tuning) return fail(AH_ERR_INVALID_ARG, "tuning is NULL");
  PairSet ps;
  ah_status s = compile_pairs(pairs, n_pairs, ps);
  if (s) return s;
  const Tuning t = tuning_for(pairs, n_pairs);
  tuning->words_per_lane = (uint32_t)t.u;
  tuning->patterns_per_group = (uint32_t)t.group;
  return AH_OK;
}

ah_status ah_autotune_scan(const ah_genomes* g, const ah_primer_pair* pairs, uint32_t n_pairs,
                           ah_hit* d_hits, uint64_t capacity, ah_result* d_res, void* d_work,
                           size_t work_bytes, void* stream, uint32_t repeats,
                           ah_scan_tuning* chosen, double* best_ms) {
  g_err.clear();
  ah_status s = check_genomes(g);
  if (s) return s;
  if (!d_res || !chosen) return fail(AH_ERR_INVALID_ARG, "ah_autotune_scan: d_res and chosen are required");
  if (capacity > 0 && !d_hits) return fail(AH_ERR_INVALID_ARG, "d_hits is NULL");
  PairSet ps;
  s = compile_pairs(pairs, n_pairs, ps);
  if (s) return s;
  const size_t need = scan_ws_bytes(g->n, capacity, min_cands(capacity));
  if (!d_work || work_bytes < need)
    return fail(AH_ERR_WORKSPACE, "scan workspace: %zu bytes given, %zu needed", work_bytes, need);
  const std::vector<Pattern> pats = patterns_of(ps);
  // candidates: the default shape first (kept unless another one is
  // faster), then tile words per lane x patterns per group (a single group
  // when the set is small)
  std::vector<Tuning> cand;
  auto add = [&](Tuning t) {
    t.group = std::min(t.group, (int)pats.size());
    for (const Tuning& c : cand)
      if (c.u == t.u && c.group == t.group) return;
    cand.push_back(t);
  };
  add(default_tuning());
  for (int u : {9, 15, 19, 21})
    for (int grp : {4, 8, 16}) {
      if (grp > (int)pats.size() && grp != 4) continue;
      add(Tuning{u, grp});
    }
  // compile every candidate concurrently (host threads), then time each
  std::vector<std::string> srcs(cand.size());
  std::vector<std::vector<char>> codes(cand.size());
  std::vector<ah_status> st(cand.size(), AH_OK);
  std::vector<std::string> errs(cand.size());
  for (size_t i = 0; i < cand.size(); ++i) srcs[i] = gen_program(pats, g->nmask != nullptr, cand[i]);
  // AH_VERBOSE=1: a line on stderr as each candidate is compiled and timed
  const char* verbose_env = getenv("AH_VERBOSE");
  const bool verbose = verbose_env && verbose_env[0] == '1';
  const auto t_start = std::chrono::steady_clock::now();
  auto since = [&t_start] {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  };
  {
    std::atomic<int> done{0};
    std::mutex print_mu;
    std::vector<std::thread> th;
    for (size_t i = 0; i < cand.size(); ++i)
      th.emplace_back([&, i] {
        st[i] = rtc_compile(srcs[i], codes[i]);
        if (st[i]) errs[i] = g_err;
        const int k = ++done;
        if (verbose) {
          std::lock_guard<std::mutex> lk(print_mu);
          fprintf(stderr, "ah_autotune_scan: shape %d x %d compiled (%d of %zu) at %.1f s\n",
                  cand[i].u, cand[i].group, k, cand.size(), since());
          fflush(stderr);
        }
      });
    for (auto& t : th) t.join();
  }
  int dev = 0;
  AH_HIP(hipGetDevice(&dev));
  hipStream_t strm = (hipStream_t)stream;
  Carver c(d_work, work_bytes);
  ScanWs w = carve_scan(c, g->n, capacity, 0);
  hipEvent_t e0, e1;
  AH_HIP(hipEventCreate(&e0));
  AH_HIP(hipEventCreate(&e1));
  double best = 1e30;
  size_t besti = 0;
  const uint32_t reps = repeats ? repeats : 3;
  for (size_t i = 0; i < cand.size(); ++i) {
    if (st[i]) return fail(st[i], "%s", errs[i].c_str());
    ScanFns fn;
    s = load_scan_kernel(dev, srcs[i], codes[i], fn);
    if (s) return s;
    double total = 0.0;
    for (uint32_t r = 0; r <= reps; ++r) {  // the first run warms up
      AH_HIP(ah::launch_result_init(d_res, strm));
      AH_HIP(hipEventRecord(e0, strm));
      s = launch_scan_kernel(fn, cand[i], g, w, d_res, capacity, strm, nullptr);
      if (s) return s;
      AH_HIP(hipEventRecord(e1, strm));
      AH_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      AH_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (r) total += ms;
    }
    const double avg = total / reps;
    if (verbose) {
      fprintf(stderr, "ah_autotune_scan: shape %d x %d: %.3f ms at %.1f s\n", cand[i].u,
              cand[i].group, avg, since());
      fflush(stderr);
    }
    if (avg < best) {
      best = avg;
      besti = i;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  AH_HIP(ah::launch_result_init(d_res, strm));
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuning[std::make_pair(dev, set_key(pairs, n_pairs))] = cand[besti];
  }
  chosen->words_per_lane = (uint32_t)cand[besti].u;
  chosen->patterns_per_group = (uint32_t)cand[besti].group;
  if (best_ms) *best_ms = best;
  return AH_OK;
}

void ah_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
}

void ah_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& kv : g_prof) {
    for (auto& ev : kv.second.pending) {
      (void)hipEventSynchronize(ev.second);
      g_event_pool.push_back(ev.first);
      g_event_pool.push_back(ev.second);
    }
  }
  g_prof.clear();
}

ah_status ah_profile_query(const char* name, uint64_t* launches, double* total_ms) {
  g_err.clear();
  if (!name) return fail(AH_ERR_INVALID_ARG, "profile name is NULL");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  ProfEntry& e = g_prof[name];
  for (auto& ev : e.pending) {
    AH_HIP(hipEventSynchronize(ev.second));
    float ms = 0.f;
    AH_HIP(hipEventElapsedTime(&ms, ev.first, ev.second));
    e.ms += ms;
    e.launches += 1;
    g_event_pool.push_back(ev.first);
    g_event_pool.push_back(ev.second);
  }
  e.pending.clear();
  if (launches) *launches = e.launches;
  if (total_ms) *total_ms = e.ms;
  return AH_OK;
}

ah_status ah_scan_candidate_stats(const void* d_work, size_t work_bytes, uint32_t n_genomes,
                                  uint64_t capacity, uint64_t out[4]) {
  g_err.clear();
  if (!d_work || !out) return fail(AH_ERR_INVALID_ARG, "d_work and out are required");
  Carver c((void*)d_work, work_bytes);
  const ScanWs w = carve_scan(c, n_genomes, capacity, 0);
  AH_HIP(hipDeviceSynchronize());
  AH_HIP(hipMemcpy(out, w.cstat, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost));
  return AH_OK;
}

uint64_t ah_scan_candidate_capacity(size_t base_offset, size_t work_bytes, uint32_t n_genomes,
                                    uint64_t capacity) {
  Carver c((void*)(uintptr_t)(base_offset & 255u), work_bytes);
  return carve_scan(c, n_genomes, capacity, 0).ccap;
}

ah_status ah_validate_tm(const ah_primer_pair* pairs, uint32_t n_pairs, const ah_tm_params* p) {
  g_err.clear();
  PairSet ps;
  return check_tm_request(pairs, n_pairs, p, ps);
}

ah_status ah_validate_pairs(const ah_primer_pair* pairs, uint32_t n_pairs) {
  g_err.clear();
  PairSet ps;
  return compile_pairs(pairs, n_pairs, ps);
}

}  // extern "C"
