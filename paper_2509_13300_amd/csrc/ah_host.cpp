// Host runtime of libah: argument and primer validation, the primer compiler
// (IUPAC sets, reverse complements, clamp positions), generation and
// compilation of the per-primer-set scan program, per-device caches, and the
// C entry points declared in ah.h.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
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
  std::vector<uint32_t> k, clamp;
};

ah_status compile_pairs(const ah_primer_pair* pairs, uint32_t n_pairs, PairSet& ps) {
  if (!pairs || n_pairs == 0) return fail(AH_ERR_INVALID_ARG, "no primer pairs");
  if (n_pairs > 65535) return fail(AH_ERR_LIMIT, "at most 65535 primer pairs per call");
  ps.fwd.resize(n_pairs);
  ps.rev.resize(n_pairs);
  ps.k.resize(n_pairs);
  ps.clamp.resize(n_pairs);
  for (uint32_t q = 0; q < n_pairs; ++q) {
    ah_status s = parse_primer(pairs[q].fwd, "fwd", q, ps.fwd[q]);
    if (s) return s;
    s = parse_primer(pairs[q].rev, "rev", q, ps.rev[q]);
    if (s) return s;
    if (pairs[q].k > AH_MAX_K) return fail(AH_ERR_LIMIT, "pair %u: k = %u > %d", q, pairs[q].k, AH_MAX_K);
    const int lmin = ps.fwd[q].L < ps.rev[q].L ? ps.fwd[q].L : ps.rev[q].L;
    if ((int)pairs[q].clamp > lmin)
      return fail(AH_ERR_LIMIT, "pair %u: clamp %u longer than a primer", q, pairs[q].clamp);
    ps.k[q] = pairs[q].k;
    ps.clamp[q] = pairs[q].clamp;
  }
  return AH_OK;
}

std::vector<Pattern> patterns_of(const PairSet& ps) {
  std::vector<Pattern> out;
  for (uint32_t q = 0; q < ps.fwd.size(); ++q) {
    for (uint32_t primer = 0; primer < 2; ++primer) {
      const Primer& p = primer ? ps.rev[q] : ps.fwd[q];
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

// Window words per lane and tile of the scan kernel (AH_SCAN_U = 2, 4, 8 or
// 16; default 4): the tile of AH_BLOCK * U words plus the halo is staged in
// LDS twice (double buffer), so larger tiles amortise the halo and the
// per-tile set-up but leave room for fewer workgroups per CU.
int scan_u() {
  const char* e = getenv("AH_SCAN_U");
  const int u = e ? atoi(e) : ah::kScanU;
  return (u == 2 || u == 4 || u == 8 || u == 16) ? u : ah::kScanU;
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

// Prefilter of one pattern (pigeonhole): the non-clamp positions whose set is
// not N are split into `blocks`; a window with at most k mismatches there
// leaves at least `need` blocks without a mismatch (k + need blocks, each
// holding at least one position).  need == 0: no prefilter.
struct FilterPlan {
  int need = 0;
  std::vector<std::vector<int>> blocks;
  double rate = 1.0;  // chance a random window passes (uniform bases)
};

int set_size(uint8_t m) { return __builtin_popcount(m); }

// P(at least `need` of the independent events with probabilities p occur)
double at_least(const std::vector<double>& p, int need) {
  std::vector<double> d(p.size() + 1, 0.0);  // d[c] = P(exactly c so far)
  d[0] = 1.0;
  for (size_t i = 0; i < p.size(); ++i)
    for (size_t c = i + 1; c-- > 0;) {
      const double stay = d[c] * (1.0 - p[i]);
      const double up = c ? d[c - 1] * p[i] : 0.0;
      d[c] = stay + up;
    }
  double r = 0.0;
  for (size_t c = (size_t)need; c < d.size(); ++c) r += d[c];
  return r;
}

FilterPlan plan_filter(const Pattern& p, bool allow) {
  std::vector<int> free_pos;
  double clamp_p = 1.0;
  int clamp_ops = 0, verify_ops = 0;
  for (int j = 0; j < p.L; ++j) {
    if (set_size(p.mask[j]) == 4) continue;
    verify_ops += (p.clamp_bits >> j & 1u) ? 2 : (int)p.k + 2;
    if (p.clamp_bits >> j & 1u) {
      clamp_p *= set_size(p.mask[j]) / 4.0;
      ++clamp_ops;
    } else {
      free_pos.push_back(j);
    }
  }
  FilterPlan best;
  best.rate = clamp_p;
  // cost per window word of this pattern, in lane operations: prefilter ops
  // plus the exact count whenever any lane of the wave has a candidate
  auto slot = [](double r) { return 1.0 - std::pow(1.0 - std::min(r, 1.0), 32.0 * 64.0); };
  double best_cost = clamp_ops + slot(clamp_p) * verify_ops;
  if (!allow) return best;
  for (int need = 1; need <= 3; ++need) {
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
    std::vector<double> clean(B);
    for (int b = 0; b < B; ++b) clean[b] = std::exp2(-bits[b]);
    const double rate = clamp_p * at_least(clean, need);
    const double cost = clamp_ops + (double)free_pos.size() + 2.0 * need * B + slot(rate) * verify_ops;
    if (cost < best_cost) {
      best_cost = cost;
      best.need = need;
      best.blocks = blocks;
      best.rate = rate;
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

bool valid_u(int u) { return u == 2 || u == 4 || u == 8 || u == 16; }

struct Tuning {
  int u;      // window words per lane and tile
  int group;  // patterns per group
};

Tuning default_tuning() { return Tuning{scan_u(), scan_group()}; }

bool filter_enabled() {
  const char* e = getenv("AH_SCAN_PREFILTER");
  return !(e && e[0] == '0');
}

std::string gen_program(const std::vector<Pattern>& pats, bool has_n, Tuning tn) {
  int lmax = 0;
  for (const Pattern& p : pats) lmax = p.L > lmax ? p.L : lmax;
  const bool allow = filter_enabled();
  std::string s;
  char buf[640];
  snprintf(buf, sizeof buf,
           "#define AH_U %d\n#define AH_HALO %d\n#define AH_HAS_N %d\n", tn.u, lmax - 1,
           has_n ? 1 : 0);
  std::string head = buf;
  for (size_t i = 0; i < pats.size(); ++i) {
    const Pattern& p = pats[i];
    const int K = (int)p.k;
    const FilterPlan fp = plan_filter(p, allow);
    // ---- prefilter (hot): clamp positions must match, `need` blocks be clean
    snprintf(buf, sizeof buf,
             "// pattern %zu: pair %u primer %u strand %u, L %d, k %d, prefilter: %d of %zu blocks "
             "(random pass rate %.3g)\n"
             "__device__ __forceinline__ void ah_pat_%zu(const u32* h, const u32* l, const AhCtx& c,"
             " u32 t) {\n",
             i, p.pair, p.primer, p.strand, p.L, K, fp.need, fp.blocks.size(), fp.rate, i);
    s += buf;
    // clamp mismatches
    std::string cl;
    for (int j = 0; j < p.L; ++j) {
      if (!(p.clamp_bits >> j & 1u) || set_size(p.mask[j]) == 4) continue;
      if (cl.empty()) {
        s += "  u32 cl = " + mism_op(p.mask[j], j) + ";\n";
        cl = "cl";
      } else {
        s += "  cl = " + acc_mism_op("cl", p.mask[j], j) + ";\n";
      }
    }
    std::string cand_expr;
    if (fp.need > 0) {
      // a_b: some position of block b mismatches ("dirty")
      for (size_t b = 0; b < fp.blocks.size(); ++b) {
        const std::string ab = "a" + std::to_string(b);
        for (size_t q = 0; q < fp.blocks[b].size(); ++q) {
          const int j = fp.blocks[b][q];
          if (q == 0) s += "  u32 " + ab + " = " + mism_op(p.mask[j], j) + ";\n";
          else s += "  " + ab + " = " + acc_mism_op(ab, p.mask[j], j) + ";\n";
        }
      }
      // z_m: at most m blocks clean so far; a window is a candidate iff
      // z_{need-1} is clear after the last block (and the clamp matches)
      const int B = (int)fp.blocks.size();
      const int need = fp.need;
      s += "  u32 z0 = a0;\n";
      for (int m = 1; m < need; ++m) s += "  u32 z" + std::to_string(m) + " = 0xffffffffu;\n";
      for (int b = 1; b < B; ++b) {
        const std::string ab = "a" + std::to_string(b);
        for (int m = need - 1; m >= 1; --m) {
          // z_m' = (z_m & a_b) | z_{m-1}
          const std::string zm = "z" + std::to_string(m), zp = "z" + std::to_string(m - 1);
          s += "  " + zm + " = " + bitop3(zm, ab, zp, (uint8_t)((kS0 & kS1) | kS2)) + ";\n";
        }
        if (b < B - 1 || need == 1) s += "  z0 &= " + ab + ";\n";
      }
      const std::string zl = "z" + std::to_string(need - 1);
      cand_expr = cl.empty() ? "~" + zl : bitop3(zl, "cl", zl, (uint8_t)(~(kS0 | kS1)));
    } else {
      cand_expr = cl.empty() ? "0xffffffffu" : "~cl";
    }
    s += "  u32 cand = " + cand_expr + ";\n  if (!cand) return;\n";
    // ---- exact count for candidate windows (rare), from the same registers
    snprintf(buf, sizeof buf, "  cand &= ah_valid(c, t, %du);\n  if (!cand) return;\n", p.L);
    s += buf;
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
               "  if (hb) { const u32 lv[1] = {0u}; ah_emit<0>(c, t, hb, lv, %uu, %uu); }\n}\n",
               p.pair, (p.strand << 1) | p.primer);
    } else {
      std::string lv = "s0";
      for (int m = 1; m < K; ++m) lv += ", s" + std::to_string(m);
      snprintf(buf, sizeof buf,
               "  if (hb) { const u32 lv[%d] = {%s}; ah_emit<%d>(c, t, hb, lv, %uu, %uu); }\n}\n", K,
               lv.c_str(), K, p.pair, (p.strand << 1) | p.primer);
    }
    s += buf;
  }
  // groups of consecutive patterns; one function per group walks the tile
  const size_t G = (size_t)tn.group;
  const size_t ngroups = (pats.size() + G - 1) / G;
  for (size_t gi = 0; gi < ngroups; ++gi) {
    const size_t a = gi * G, b = std::min(pats.size(), a + G);
    int lg = 0;
    for (size_t i = a; i < b; ++i) lg = std::max(lg, pats[i].L);
    snprintf(buf, sizeof buf,
             "__device__ %s void ah_group_%zu(ah_lds_uint2* tw, u32 t0, AhCtx c) {\n"
             "  for (u32 i = threadIdx.x; i < (u32)AH_TILE; i += AH_BLOCK) {\n"
             "    const u32 t = t0 + i;\n    if (t >= c.S) break;\n"
             "    u32 h[%d], l[%d];\n#pragma unroll\n"
             "    for (int j = 0; j < %d; ++j) { const uint2 v = tw[i + (u32)j]; h[j] = v.x; l[j] = v.y; }\n",
             ngroups > 1 ? "__noinline__" : "__forceinline__", gi, lg, lg, lg);
    s += buf;
    for (size_t i = a; i < b; ++i) s += "    ah_pat_" + std::to_string(i) + "(h, l, c, t);\n";
    s += "  }\n}\n";
  }
  s += "__device__ void ah_groups(ah_lds_uint2* tw, u32 t0, const AhCtx& c) {\n";
  for (size_t gi = 0; gi < ngroups; ++gi) s += "  ah_group_" + std::to_string(gi) + "(tw, t0, c);\n";
  s += "}\n";
  return head + std::string(kScanCore) + s;
}

// --------------------------------------------------------------- caches --
struct JitEntry {
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
};

std::mutex g_mu;
std::map<std::pair<int, std::string>, JitEntry> g_jit;
std::map<std::pair<int, std::string>, void*> g_tables;
uint64_t g_jit_n = 0;
double g_jit_ms = 0.0;
std::map<int, int> g_cus;

std::mutex g_stats_mu;

ah_status rtc_compile(const std::string& src, std::vector<char>& code) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "ah_scan.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    return fail(AH_ERR_JIT, "hiprtcCreateProgram failed");
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17"};
  const auto t0 = std::chrono::steady_clock::now();
  const hiprtcResult r = hiprtcCompileProgram(prog, 3, opts);
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
                           hipFunction_t& fn) {
  std::lock_guard<std::mutex> lk(g_mu);
  const auto key = std::make_pair(dev, src);
  auto it = g_jit.find(key);  // another thread may have loaded it meanwhile
  if (it != g_jit.end()) {
    fn = it->second.fn;
    return AH_OK;
  }
  JitEntry e;
  AH_HIP(hipModuleLoadData(&e.mod, code.data()));
  AH_HIP(hipModuleGetFunction(&e.fn, e.mod, "ah_scan_kernel"));
  g_jit[key] = e;
  fn = e.fn;
  return AH_OK;
}

// Compiled and loaded scan kernel for `src` on the current device (cached;
// compiles outside the cache lock so that several programs can compile at
// once).
ah_status get_scan_kernel(const std::string& src, hipFunction_t& fn) {
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
    k += '|' + std::to_string(pairs[q].k) + '|' + std::to_string(pairs[q].clamp) + ';';
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
struct ProfScope {
  const char* name;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(const char* n, hipStream_t s) : name(n), st(s) {
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
  ah::SortBuffers sb;
};

ScanWs carve_scan(Carver& c, uint32_t n, uint64_t cap) {
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
  w.sb.hist = c.take<uint64_t>((uint64_t)256 * ah::kSortGrid);
  w.sb.hist_off = c.take<uint64_t>((uint64_t)256 * ah::kSortGrid + 1);
  w.sb.scan_tmp = w.scan_tmp;
  return w;
}

ah::PairBuffers carve_pair(Carver& c, uint64_t cap) {
  const uint64_t m = cap ? cap : 1;
  ah::PairBuffers b;
  b.n = c.take<uint64_t>(1);
  b.flag_f = c.take<uint32_t>(m);
  b.flag_r = c.take<uint32_t>(m);
  b.off_f = c.take<uint64_t>(m + 1);
  b.off_r = c.take<uint64_t>(m + 1);
  b.mkey_f = c.take<uint64_t>(m);
  b.mpos_f = c.take<uint32_t>(m);
  b.midx_f = c.take<uint32_t>(m);
  b.mkey_r = c.take<uint64_t>(m);
  b.mpos_r = c.take<uint32_t>(m);
  b.midx_r = c.take<uint32_t>(m);
  b.cnt = c.take<uint32_t>(m);
  b.cnt_off = c.take<uint64_t>(m + 1);
  b.scan_tmp = c.take<uint64_t>(ah::kScanGrid + 1);
  return b;
}

ah_status check_genomes(const ah_genomes* g) {
  if (!g) return fail(AH_ERR_INVALID_ARG, "genomes is NULL");
  if (g->n > 0 && (!g->words || !g->word_off || !g->len))
    return fail(AH_ERR_INVALID_ARG, "genomes: words, word_off and len must be device pointers");
  if (g->max_len == 0 && g->n > 0) return fail(AH_ERR_INVALID_ARG, "genomes: max_len must be >= 1");
  return AH_OK;
}

// Tile counts, tile prefix and the scan kernel itself (hits appended to the
// staging area, counted in d_res->required).
ah_status launch_scan_kernel(hipFunction_t fn, Tuning tn, const ah_genomes* g, const ScanWs& w,
                             ah_result* d_res, uint64_t capacity, hipStream_t st) {
  if (g->n == 0) return AH_OK;
  AH_HIP(ah::launch_tile_counts(g->len, g->n, (uint32_t)(ah::kBlock * tn.u), w.counts, st));
  AH_HIP(ah::launch_exclusive_scan(w.counts, w.tile_prefix, g->n, nullptr, w.scan_tmp, st));
  const void* words = g->words;
  const uint32_t* nmask = g->nmask;
  const uint64_t* word_off = g->word_off;
  const uint32_t* len = g->len;
  const uint64_t* tp = w.tile_prefix;
  uint32_t n = g->n;
  ah_hit* out = w.staging;
  uint64_t cap = capacity;
  uint64_t* counter = &d_res->required;
  void* args[] = {&words, &nmask, &word_off, &len, &tp, &n, &out, &cap, &counter};
  const unsigned grid = (unsigned)cu_count() * 8u;
  ProfScope prof_scan("scan", st);
  AH_HIP(hipModuleLaunchKernel(fn, grid, 1, 1, ah::kBlock, 1, 1, 0, st, args, nullptr));
  return AH_OK;
}

}  // namespace

namespace ah {
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
  for (auto& kv : g_tables) (void)hipFree(kv.second);
  g_tables.clear();
}

uint64_t ah_pack_layout(const uint64_t* h_len, uint32_t n, uint64_t* h_word_off) {
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

size_t ah_scan_workspace_bytes(const ah_genomes* g, uint32_t n_pairs, uint64_t capacity) {
  (void)n_pairs;
  Carver c(nullptr, 0);
  carve_scan(c, g ? g->n : 0, capacity);
  return c.used();
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
  const size_t need = ah_scan_workspace_bytes(g, n_pairs, capacity);
  if (!d_work || work_bytes < need)
    return fail(AH_ERR_WORKSPACE, "scan workspace: %zu bytes given, %zu needed", work_bytes, need);
  const Tuning tn = tuning_for(pairs, n_pairs);
  hipFunction_t fn;
  s = get_scan_kernel(gen_program(patterns_of(ps), g->nmask != nullptr, tn), fn);
  if (s) return s;

  hipStream_t st = (hipStream_t)stream;
  Carver c(d_work, work_bytes);
  ScanWs w = carve_scan(c, g->n, capacity);
  AH_HIP(ah::launch_result_init(d_res, st));
  s = launch_scan_kernel(fn, tn, g, w, d_res, capacity, st);
  if (s) return s;
  AH_HIP(ah::launch_result_finalize(d_res, capacity, w.n_sort, st));
  ProfScope prof_sort("sort", st);
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
  s = compile_pairs(pairs, n_pairs, ps);
  if (s) return s;
  if (p->saltcorr != 0 && p->saltcorr != 5)
    return fail(AH_ERR_INVALID_ARG, "salt correction method %d (supported: 0, 5)", p->saltcorr);
  const double mg = p->Mg_mM - p->dNTPs_mM;
  const double na_eq = p->Na_mM + p->K_mM + p->Tris_mM / 2.0 + (mg > 0 ? 120.0 * std::sqrt(mg) : 0.0);
  if (p->saltcorr == 5 && !(na_eq > 0))
    return fail(AH_ERR_INVALID_ARG, "salt correction needs a positive sodium equivalent");
  double C;
  if (p->selfcomp) {
    C = p->dnac1_nM * 1e-9;
  } else {
    const double hi = p->dnac1_nM > p->dnac2_nM ? p->dnac1_nM : p->dnac2_nM;
    const double lo = p->dnac1_nM > p->dnac2_nM ? p->dnac2_nM : p->dnac1_nM;
    C = (hi - lo / 2.0) * 1e-9;
  }
  if (!(C > 0)) return fail(AH_ERR_INVALID_ARG, "strand concentration must be positive");
  const double R = 1.987;
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
          deg *= (uint64_t)cnt;
        }
      }
      for (uint32_t j = 0; j < ps.clamp[q]; ++j) t.clampm |= 1ull << (2 * (pr.L - 1 - (int)j));
      if (deg > (1ull << 20))
        return fail(AH_ERR_LIMIT, "pair %u: primer degeneracy %llu exceeds 2^20 for Tm", q,
                    (unsigned long long)deg);
      t.deg = deg;
      const double salt = p->saltcorr == 5 ? 0.368 * (pr.L - 1) * std::log(na_eq / 1000.0) : 0.0;
      t.KL = salt + R * std::log(C) + (p->selfcomp ? -1.4 : 0.0);
      tabs[2 * q + primer] = t;
    }
  }
  void* dt = nullptr;
  s = get_table(tabs.data(), tabs.size() * sizeof(ah::PrimerTab), &dt);
  if (s) return s;
  ProfScope prof_tm("tm", (hipStream_t)stream);
  AH_HIP(ah::launch_tm(*g, (const ah::PrimerTab*)dt, d_hits, d_nhits, capacity, cu_count() * 4,
                       (hipStream_t)stream));
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
  const size_t need = ah_pair_workspace_bytes(hit_capacity, n_pairs);
  if (!d_work || work_bytes < need)
    return fail(AH_ERR_WORKSPACE, "pair workspace: %zu bytes given, %zu needed", work_bytes, need);
  void* dt = nullptr;
  s = get_table(tabs.data(), tabs.size() * sizeof(ah::PairTab), &dt);
  if (s) return s;
  Carver c(d_work, work_bytes);
  ah::PairBuffers pb = carve_pair(c, hit_capacity);
  ProfScope prof_pair("pair", (hipStream_t)stream);
  AH_HIP(ah::launch_pair(d_hits, d_nhits, hit_capacity, (const ah::PairTab*)dt, d_amp, capacity,
                         d_res, pb, cu_count() * 4, (hipStream_t)stream));
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
  hipFunction_t fn;
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
    return fail(AH_ERR_INVALID_ARG, "tuning: words_per_lane in {2,4,8,16}, patterns_per_group in 1..1024");
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
  const size_t need = ah_scan_workspace_bytes(g, n_pairs, capacity);
  if (!d_work || work_bytes < need)
    return fail(AH_ERR_WORKSPACE, "scan workspace: %zu bytes given, %zu needed", work_bytes, need);
  const std::vector<Pattern> pats = patterns_of(ps);
  // candidates: tile words per lane x patterns per group (a single group when
  // the set is small)
  std::vector<Tuning> cand;
  for (int u : {2, 4, 8})
    for (int grp : {8, 16, 32}) {
      if (grp > (int)pats.size() && grp != 8) continue;
      cand.push_back(Tuning{u, std::min(grp, (int)pats.size())});
    }
  // compile every candidate concurrently (host threads), then time each
  std::vector<std::string> srcs(cand.size());
  std::vector<std::vector<char>> codes(cand.size());
  std::vector<ah_status> st(cand.size(), AH_OK);
  std::vector<std::string> errs(cand.size());
  for (size_t i = 0; i < cand.size(); ++i) srcs[i] = gen_program(pats, g->nmask != nullptr, cand[i]);
  {
    std::vector<std::thread> th;
    for (size_t i = 0; i < cand.size(); ++i)
      th.emplace_back([&, i] {
        st[i] = rtc_compile(srcs[i], codes[i]);
        if (st[i]) errs[i] = g_err;
      });
    for (auto& t : th) t.join();
  }
  int dev = 0;
  AH_HIP(hipGetDevice(&dev));
  hipStream_t strm = (hipStream_t)stream;
  Carver c(d_work, work_bytes);
  ScanWs w = carve_scan(c, g->n, capacity);
  hipEvent_t e0, e1;
  AH_HIP(hipEventCreate(&e0));
  AH_HIP(hipEventCreate(&e1));
  double best = 1e30;
  size_t besti = 0;
  const uint32_t reps = repeats ? repeats : 3;
  for (size_t i = 0; i < cand.size(); ++i) {
    if (st[i]) return fail(st[i], "%s", errs[i].c_str());
    hipFunction_t fn;
    s = load_scan_kernel(dev, srcs[i], codes[i], fn);
    if (s) return s;
    double total = 0.0;
    for (uint32_t r = 0; r <= reps; ++r) {  // the first run warms up
      AH_HIP(ah::launch_result_init(d_res, strm));
      AH_HIP(hipEventRecord(e0, strm));
      s = launch_scan_kernel(fn, cand[i], g, w, d_res, capacity, strm);
      if (s) return s;
      AH_HIP(hipEventRecord(e1, strm));
      AH_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      AH_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (r) total += ms;
    }
    const double avg = total / reps;
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

ah_status ah_validate_pairs(const ah_primer_pair* pairs, uint32_t n_pairs) {
  g_err.clear();
  PairSet ps;
  return compile_pairs(pairs, n_pairs, ps);
}

}  // extern "C"
