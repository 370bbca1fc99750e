// Host planner: pivots, homogeneity, sample set, plan orders, twiddle schedule.
//
// Pivots (Sec. VI, Remark 2): level e is a pivot iff 2^e exactly divides
// j1 - j2 for some pair in J.  Sorting J by the bit-reversed value lists the
// leaves of the congruence tree (an LSB-first binary trie) in depth-first
// order; every branching node is then the lowest common ancestor of two
// neighbours in that list, and the LCA level of two leaves is the lowest bit
// in which they differ (Remark 1).  So the pivot set is the set of lowest
// differing bits of neighbours: O(k log k) instead of the O(k^2) pair scan.
#include "plan_core.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>

namespace hidft {

uint64_t bit_reverse(uint64_t x, unsigned nbits) {
  if (nbits == 0) return 0;
  x = ((x >> 1) & 0x5555555555555555ULL) | ((x & 0x5555555555555555ULL) << 1);
  x = ((x >> 2) & 0x3333333333333333ULL) | ((x & 0x3333333333333333ULL) << 2);
  x = ((x >> 4) & 0x0F0F0F0F0F0F0F0FULL) | ((x & 0x0F0F0F0F0F0F0F0FULL) << 4);
  x = ((x >> 8) & 0x00FF00FF00FF00FFULL) | ((x & 0x00FF00FF00FF00FFULL) << 8);
  x = ((x >> 16) & 0x0000FFFF0000FFFFULL) | ((x & 0x0000FFFF0000FFFFULL) << 16);
  x = (x >> 32) | (x << 32);
  return x >> (64 - nbits);
}

static void set_err(std::string* err, const char* fmt, unsigned long long a = 0,
                    unsigned long long b = 0) {
  if (!err) return;
  char buf[256];
  std::snprintf(buf, sizeof buf, fmt, a, b);
  *err = buf;
}

hidft_status analyze_core(uint32_t M, const uint64_t* J, uint64_t k,
                          uint64_t* pivot_mask, std::string* err) {
  if (M > HIDFT_MAX_LOG2_N) {
    set_err(err, "log2_n = %llu exceeds 63", M);
    return HIDFT_ERR_INVALID_ARGUMENT;
  }
  if (k == 0 || J == nullptr) {
    set_err(err, "J must be a non-null array of k >= 1 indices");
    return HIDFT_ERR_INVALID_ARGUMENT;
  }
  if (M < 64 && k > (1ULL << M)) {
    set_err(err, "k = %llu exceeds N = 2^%llu", k, M);
    return HIDFT_ERR_INVALID_ARGUMENT;
  }
  const uint64_t limit_mask = (M == 64) ? ~0ULL : ((1ULL << M) - 1);
  std::vector<uint64_t> key(k);
  for (uint64_t t = 0; t < k; ++t) {
    if (J[t] & ~limit_mask) {
      set_err(err, "J[%llu] = %llu is outside [0, N)", t, J[t]);
      return HIDFT_ERR_INDEX_OUT_OF_RANGE;
    }
    key[t] = bit_reverse(J[t], 64);
  }
  std::sort(key.begin(), key.end());
  uint64_t mask = 0;
  for (uint64_t t = 1; t < k; ++t) {
    if (key[t] == key[t - 1]) {
      set_err(err, "index %llu appears more than once in J", bit_reverse(key[t], 64));
      return HIDFT_ERR_DUPLICATE_INDEX;
    }
    const uint64_t d = bit_reverse(key[t], 64) ^ bit_reverse(key[t - 1], 64);
    mask |= d & (~d + 1);  // lowest differing bit = 2^{nu2(j_a - j_b)}
  }
  *pivot_mask = mask;
  return HIDFT_OK;
}

hidft_status build_plan_core(uint32_t M, const uint64_t* J, uint64_t k,
                             uint32_t max_log2_k, PlanCore* pc, std::string* err) {
  uint64_t mask = 0;
  hidft_status st = analyze_core(M, J, k, &mask, err);
  if (st != HIDFT_OK) return st;
  if ((k & (k - 1)) != 0) {
    set_err(err, "k = %llu is not a power of two, so J cannot be homogeneous", k);
    return HIDFT_ERR_SIZE_NOT_POW2;
  }
  const uint32_t s = static_cast<uint32_t>(__builtin_ctzll(k));
  const uint32_t npiv = static_cast<uint32_t>(__builtin_popcountll(mask));
  if (npiv != s) {
    set_err(err, "J has %llu pivots but log2 k = %llu: not homogeneous", npiv, s);
    return HIDFT_ERR_NOT_HOMOGENEOUS;
  }
  if (s > max_log2_k) {
    set_err(err, "k = 2^%llu exceeds the supported 2^%llu", s, max_log2_k);
    return HIDFT_ERR_UNSUPPORTED;
  }
  pc->M = M;
  pc->s = s;
  pc->k = k;
  pc->J.assign(J, J + k);
  pc->pivots.clear();
  for (uint32_t e = 0; e < 64; ++e)
    if ((mask >> e) & 1) pc->pivots.push_back(e);
  const std::vector<uint32_t>& r = pc->pivots;

  // Frequency order of Corollary 2: q(j) = sum_u bit_{r_u}(j) 2^{u-1}.
  // Homogeneity makes it a bijection J -> [0, k): every pivot level splits
  // every node, so two elements first differ at some pivot level.
  pc->freq_pos.assign(k, 0);
  std::vector<uint64_t> j_of_q(k, 0);
  std::vector<uint8_t> hit(k, 0);
  for (uint64_t t = 0; t < k; ++t) {
    uint32_t q = 0;
    for (uint32_t u = 0; u < s; ++u) q |= static_cast<uint32_t>((J[t] >> r[u]) & 1) << u;
    if (hit[q]) {
      set_err(err, "internal: frequency order is not a bijection (q = %llu)", q);
      return HIDFT_ERR_NOT_HOMOGENEOUS;
    }
    hit[q] = 1;
    pc->freq_pos[t] = q;
    j_of_q[q] = J[t];
  }

  // Sample set (Sec. VII): position p of the recursion order holds
  // i_p = sum_u bit_{u-1}(p) 2^{M-1-r_u}.  The weights decrease with u, so the
  // ascending order of I_r is the bit-reversed recursion order.
  pc->samples.assign(k, 0);
  for (uint64_t a = 0; a < k; ++a) {
    const uint64_t p = bit_reverse(a, s);
    uint64_t i = 0;
    for (uint32_t u = 0; u < s; ++u)
      if ((p >> u) & 1) i |= 1ULL << (M - 1 - r[u]);
    pc->samples[a] = i;
  }

  // Twiddles of Lemma 3, stage u (pivot r_u) and node q_lo < 2^{u-1}: the
  // factor exp(-2 pi i j / 2^{r_u + 1}) at the left descendant j (bit r_u of
  // j is 0), i.e. exp(-i pi m / 2^{r_u}) with m = j mod 2^{r_u}.
  const uint64_t ntw = k - 1;
  pc->tw_num.assign(ntw, 0);
  pc->tw_log2den.assign(ntw, 0);
  for (uint32_t u = 1; u <= s; ++u) {
    const uint32_t ru = r[u - 1];
    const uint64_t mmask = (1ULL << ru) - 1;
    const uint64_t off = (1ULL << (u - 1)) - 1;
    for (uint64_t q_lo = 0; q_lo < (1ULL << (u - 1)); ++q_lo) {
      pc->tw_num[off + q_lo] = j_of_q[q_lo] & mmask;
      pc->tw_log2den[off + q_lo] = static_cast<uint8_t>(ru);
    }
  }
  return HIDFT_OK;
}

// Nodes of J at `level` (classes modulo 2^level): counts and mu*.
static void node_sizes(const uint64_t* J, uint64_t k, uint32_t level, uint64_t* mu_max,
                       double* sum_sq) {
  const uint64_t mask = level >= 64 ? ~0ULL : ((1ULL << level) - 1);
  std::vector<uint64_t> res(k);
  for (uint64_t t = 0; t < k; ++t) res[t] = J[t] & mask;
  std::sort(res.begin(), res.end());
  *mu_max = 0;
  *sum_sq = 0;
  for (uint64_t a = 0; a < k;) {
    uint64_t b = a;
    while (b < k && res[b] == res[a]) ++b;
    const uint64_t m = b - a;
    *mu_max = std::max(*mu_max, m);
    *sum_sq += (double)m * (double)m;
    a = b;
  }
}

// ---------------------------------------------------------------------------
// Conditioning of the leaf systems (Algorithm 2, Eq. alg1_system).
//
// Node v at level r_max + 1 holds elements l_0..l_{mu-1}; the mu* shifted
// Hi-DFTs give y_j(v) = sum_t c_t z_t^j (j < mu*), z_t = exp(2 pi i l_t / N),
// and the leaf solve inverts the square system of its first mu(v) rows,
// V_v[j][t] = z_t^j.  With D_v the mu* x mu(v) matrix of all the rows, the
// FP32 errors dy of the Hi-DFT outputs reach the coefficients as
//   |dc| <= max_v |V_v^{-1}|_2 |dy|   and   |y| <= max_v |D_v|_2 |c|,
// so their relative error is at most A = max_v |V_v^{-1}|_2 max_v |D_v|_2
// times the Hi-DFTs' own relative error.  The paper treats arithmetic as
// exact; this bound is the library's.
// ---------------------------------------------------------------------------
namespace {

struct cd {
  double re, im;
};
inline cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline cd cconj_mul(cd a, cd b) { return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }
inline double cabs2(cd a) { return a.re * a.re + a.im * a.im; }

// exp(2 pi i m / 2^M) for the integer m mod 2^M, the fraction reduced to
// [-1/2, 1/2) before the angle is formed.
cd unit_root(uint64_t m, uint32_t M) {
  const uint64_t mask = M >= 64 ? ~0ULL : ((1ULL << M) - 1);
  m &= mask;
  double x = std::ldexp((double)m, -(int)M);
  if (x >= 0.5) x -= 1.0;
  const double a = 2.0 * 3.14159265358979323846 * x;
  return {std::cos(a), std::sin(a)};
}

// Largest singular value of the rows x cols matrix A (row-major): power
// iteration on A^H A from a fixed generic start, until the estimate settles.
double spectral_norm(const std::vector<cd>& A, uint32_t rows, uint32_t cols) {
  std::vector<cd> x(cols), y(rows), z(cols);
  for (uint32_t t = 0; t < cols; ++t) x[t] = {std::cos(0.7 + 1.3 * t), std::sin(0.3 + 0.9 * t)};
  double nx = 0;
  for (const cd& v : x) nx += cabs2(v);
  nx = std::sqrt(nx);
  for (cd& v : x) v = {v.re / nx, v.im / nx};
  double lam = 0;
  for (int it = 0; it < 300; ++it) {
    for (uint32_t j = 0; j < rows; ++j) {
      cd acc{0, 0};
      for (uint32_t t = 0; t < cols; ++t) {
        const cd p = cmul(A[(size_t)j * cols + t], x[t]);
        acc.re += p.re;
        acc.im += p.im;
      }
      y[j] = acc;
    }
    for (uint32_t t = 0; t < cols; ++t) {
      cd acc{0, 0};
      for (uint32_t j = 0; j < rows; ++j) {
        const cd p = cconj_mul(A[(size_t)j * cols + t], y[j]);
        acc.re += p.re;
        acc.im += p.im;
      }
      z[t] = acc;
    }
    double nz = 0;
    for (const cd& v : z) nz += cabs2(v);
    nz = std::sqrt(nz);  // = |A^H A x| for |x| = 1, a lower bound of sigma_max^2
    if (!(nz > 0) || !std::isfinite(nz)) return nz > 0 ? nz : 0.0;
    for (uint32_t t = 0; t < cols; ++t) x[t] = {z[t].re / nz, z[t].im / nz};
    const bool settled = std::fabs(nz - lam) <= 1e-10 * nz;
    lam = nz;
    if (settled) break;
  }
  return std::sqrt(lam);
}

// Inverse of the n x n matrix A by Gauss-Jordan elimination with partial
// pivoting; false if a pivot vanishes (the matrix is singular in FP64).
bool invert(std::vector<cd> A, uint32_t n, std::vector<cd>* inv) {
  std::vector<cd>& B = *inv;
  B.assign((size_t)n * n, cd{0, 0});
  for (uint32_t i = 0; i < n; ++i) B[(size_t)i * n + i] = {1, 0};
  for (uint32_t c = 0; c < n; ++c) {
    uint32_t piv = c;
    for (uint32_t r = c + 1; r < n; ++r)
      if (cabs2(A[(size_t)r * n + c]) > cabs2(A[(size_t)piv * n + c])) piv = r;
    const double p2 = cabs2(A[(size_t)piv * n + c]);
    if (!(p2 > 1e-300)) return false;
    if (piv != c)
      for (uint32_t t = 0; t < n; ++t) {
        std::swap(A[(size_t)piv * n + t], A[(size_t)c * n + t]);
        std::swap(B[(size_t)piv * n + t], B[(size_t)c * n + t]);
      }
    const cd pc = A[(size_t)c * n + c];
    const cd ip = {pc.re / p2, -pc.im / p2};
    for (uint32_t t = 0; t < n; ++t) {
      A[(size_t)c * n + t] = cmul(A[(size_t)c * n + t], ip);
      B[(size_t)c * n + t] = cmul(B[(size_t)c * n + t], ip);
    }
    for (uint32_t r = 0; r < n; ++r) {
      if (r == c) continue;
      const cd f = A[(size_t)r * n + c];
      if (f.re == 0 && f.im == 0) continue;
      for (uint32_t t = 0; t < n; ++t) {
        const cd a = cmul(f, A[(size_t)c * n + t]);
        const cd b = cmul(f, B[(size_t)c * n + t]);
        A[(size_t)r * n + t].re -= a.re;
        A[(size_t)r * n + t].im -= a.im;
        B[(size_t)r * n + t].re -= b.re;
        B[(size_t)r * n + t].im -= b.im;
      }
    }
  }
  return true;
}

struct NodeNorms {
  double fwd = 1, inv = 1, shifts = 1;  // |V_v|_2, |V_v^{-1}|_2, |D_v|_2
};

// Norms of one node's systems.  They depend only on the differences
// l_t - l_0 (a common factor z_0^j scales row j by a unit number), which
// is the key the caller memoises on.
NodeNorms node_norms(const std::vector<uint64_t>& diff, uint32_t M, uint32_t mu_star) {
  const uint32_t mu = (uint32_t)diff.size();
  NodeNorms n;
  if (mu == 1) {
    n.shifts = std::sqrt((double)mu_star);
    return n;
  }
  std::vector<cd> D((size_t)mu_star * mu);
  for (uint32_t j = 0; j < mu_star; ++j)
    for (uint32_t t = 0; t < mu; ++t) D[(size_t)j * mu + t] = unit_root((uint64_t)j * diff[t], M);
  const std::vector<cd> V(D.begin(), D.begin() + (size_t)mu * mu);
  n.shifts = spectral_norm(D, mu_star, mu);
  n.fwd = spectral_norm(V, mu, mu);
  std::vector<cd> W;
  n.inv = invert(V, mu, &W) ? spectral_norm(W, mu, mu) : HUGE_VAL;
  return n;
}

// Nodes of J at `level`: the elements of each class modulo 2^level.
std::vector<std::vector<uint64_t>> level_nodes(const uint64_t* J, uint64_t k, uint32_t level) {
  const uint64_t mask = level >= 64 ? ~0ULL : ((1ULL << level) - 1);
  std::vector<std::pair<uint64_t, uint64_t>> v(k);
  for (uint64_t t = 0; t < k; ++t) v[t] = {J[t] & mask, J[t]};
  std::sort(v.begin(), v.end());
  std::vector<std::vector<uint64_t>> out;
  for (uint64_t a = 0; a < k;) {
    uint64_t b = a;
    std::vector<uint64_t> e;
    while (b < k && v[b].first == v[a].first) e.push_back(v[b++].second);
    out.push_back(std::move(e));
    a = b;
  }
  return out;
}

}  // namespace

double sas_hidft_rel_error(uint32_t s) { return 0.5 * (2.0 + s) * std::ldexp(1.0, -24); }

LeafAccuracy leaf_accuracy(uint32_t M, uint32_t s, const uint64_t* J, uint64_t k,
                           uint32_t level) {
  const std::vector<std::vector<uint64_t>> nodes = level_nodes(J, k, level);
  uint32_t mu_star = 1;
  for (const auto& e : nodes) mu_star = std::max<uint32_t>(mu_star, (uint32_t)e.size());
  const uint64_t mask = M >= 64 ? ~0ULL : ((1ULL << M) - 1);
  std::map<std::vector<uint64_t>, NodeNorms> memo;
  LeafAccuracy a;
  a.mu_star = mu_star;
  double inv_max = 0, shift_max = 0;
  for (const auto& e : nodes) {
    std::vector<uint64_t> diff(e.size());
    for (size_t t = 0; t < e.size(); ++t) diff[t] = (e[t] - e[0]) & mask;
    auto it = memo.find(diff);
    if (it == memo.end()) it = memo.emplace(diff, node_norms(diff, M, mu_star)).first;
    const NodeNorms& n = it->second;
    a.cond = std::max(a.cond, n.fwd * n.inv);
    inv_max = std::max(inv_max, n.inv);
    shift_max = std::max(shift_max, n.shifts);
  }
  a.amplification = inv_max * shift_max;
  a.rel_err_bound = a.amplification * sas_hidft_rel_error(s) + std::ldexp(1.0, -24);
  if (!std::isfinite(a.rel_err_bound)) a.rel_err_bound = HUGE_VAL;
  return a;
}

hidft_status build_part_plan(uint32_t M, const uint64_t* J, uint64_t k, const uint32_t* r,
                             uint32_t nr, uint32_t max_s, uint32_t max_s_mu1, uint32_t max_mu,
                             double max_err, PartPlan* pp, std::string* err) {
  uint64_t mask = 0;
  hidft_status st = analyze_core(M, J, k, &mask, err);
  if (st != HIDFT_OK) return st;
  std::vector<uint32_t> piv;
  for (uint32_t e = 0; e < 64; ++e)
    if ((mask >> e) & 1) piv.push_back(e);

  std::vector<uint32_t> rv;
  LeafAccuracy acc;
  bool have_acc = false;
  if (r != nullptr) {
    for (uint32_t u = 0; u < nr; ++u) {
      if (r[u] >= M || (u > 0 && r[u] <= r[u - 1])) {
        set_err(err, "pivot vector must be strictly ascending in [0, M) (entry %llu)", u);
        return HIDFT_ERR_INVALID_ARGUMENT;
      }
      rv.push_back(r[u]);
    }
    if (!rv.empty())
      for (uint32_t p : piv)
        if (p <= rv.back() && !std::binary_search(rv.begin(), rv.end(), p)) {
          set_err(err, "J has pivot %llu below r_max = %llu that is not in r: "
                       "not part-homogeneous at r", p, rv.back());
          return HIDFT_ERR_NOT_HOMOGENEOUS;
        }
    if (rv.size() > max_s_mu1) {
      set_err(err, "2^%llu samples per Hi-DFT exceed the supported 2^%llu", rv.size(),
              max_s_mu1);
      return HIDFT_ERR_UNSUPPORTED;
    }
  } else {
    // Candidates t (the first t pivots): mu* <= max_mu, 2^t <= 2^max_s, in
    // ascending order of Lemma 4's cost; the first whose leaf systems keep
    // the error bound within max_err wins.
    struct Cand {
      double cost;
      uint32_t t;
    };
    std::vector<Cand> cands;
    for (uint32_t t = 0; t <= piv.size() && t <= max_s_mu1; ++t) {
      uint64_t mu = 0;
      double sq = 0;
      node_sizes(J, k, t ? piv[t - 1] + 1 : 0, &mu, &sq);
      if (mu > max_mu || (t > max_s && mu > 1)) continue;
      cands.push_back({1.5 * t * (double)(1ULL << t) * (double)mu + 6.0 * sq, t});
    }
    std::stable_sort(cands.begin(), cands.end(),
                     [](const Cand& a, const Cand& b) { return a.cost < b.cost; });
    bool found = false;
    double best_bound = HUGE_VAL;
    for (const Cand& c : cands) {
      const LeafAccuracy a = leaf_accuracy(M, c.t, J, k, c.t ? piv[c.t - 1] + 1 : 0);
      best_bound = std::min(best_bound, a.rel_err_bound);
      if (a.rel_err_bound <= max_err) {
        rv.assign(piv.begin(), piv.begin() + c.t);
        acc = a;
        have_acc = found = true;
        break;
      }
    }
    if (!found) {
      char buf[320];
      std::snprintf(buf, sizeof buf,
                    "no prefix of the pivots of J keeps mu* <= %u with 2^s <= 2^%u (2^%u "
                    "for mu* = 1) and the leaf systems' error bound within %.1e (best bound "
                    "%.3e)",
                    max_mu, max_s, max_s_mu1, max_err, best_bound);
      if (err) *err = buf;
      return HIDFT_ERR_UNSUPPORTED;
    }
  }

  const uint32_t s = (uint32_t)rv.size();
  const uint32_t level = s ? rv.back() + 1 : 0;
  const uint64_t lmask = level >= 64 ? ~0ULL : ((1ULL << level) - 1);
  pp->M = M;
  pp->s = s;
  pp->level = level;
  pp->k = k;
  pp->J.assign(J, J + k);
  pp->pivots = rv;

  // Nodes: positions sorted by (slot, t).
  auto slot_of = [&](uint64_t x) {
    uint32_t q = 0;
    for (uint32_t u = 0; u < s; ++u) q |= (uint32_t)((x >> rv[u]) & 1) << u;
    return q;
  };
  std::vector<std::pair<uint64_t, uint32_t>> order(k);  // (slot << 32 | 0, t) via residue
  std::vector<uint32_t> slot_t(k);
  for (uint64_t t = 0; t < k; ++t) {
    slot_t[t] = slot_of(J[t] & lmask);
    order[t] = {((uint64_t)slot_t[t] << 32) | 0u, (uint32_t)t};
  }
  std::sort(order.begin(), order.end());
  pp->node_slot.clear();
  pp->node_residue.clear();
  pp->node_first.clear();
  pp->node_count.clear();
  pp->elem_t.resize(k);
  pp->mu_max = 0;
  double sq = 0;
  for (uint64_t a = 0; a < k;) {
    uint64_t b = a;
    while (b < k && (order[b].first >> 32) == (order[a].first >> 32)) ++b;
    const uint64_t res = J[order[a].second] & lmask;
    for (uint64_t i = a; i < b; ++i) {
      if ((J[order[i].second] & lmask) != res) {
        set_err(err, "internal: one slot holds two residues (not part-homogeneous)");
        return HIDFT_ERR_NOT_HOMOGENEOUS;
      }
      pp->elem_t[i] = order[i].second;
    }
    pp->node_slot.push_back((uint32_t)(order[a].first >> 32));
    pp->node_residue.push_back(res);
    pp->node_first.push_back((uint32_t)a);
    pp->node_count.push_back((uint32_t)(b - a));
    pp->mu_max = std::max<uint32_t>(pp->mu_max, (uint32_t)(b - a));
    sq += (double)(b - a) * (double)(b - a);
    a = b;
  }
  pp->cost = 1.5 * s * (double)(1ULL << s) * pp->mu_max + 6.0 * sq;
  if (s > max_s && pp->mu_max > 1) {
    if (err) {
      char buf[200];
      std::snprintf(buf, sizeof buf,
                    "2^%u samples per Hi-DFT exceed the supported 2^%u for mu* = %u (above "
                    "it, only plans with one element per node)",
                    s, max_s, pp->mu_max);
      *err = buf;
    }
    return HIDFT_ERR_UNSUPPORTED;
  }
  if (!have_acc) {
    if (pp->mu_max <= max_mu) {
      acc = leaf_accuracy(M, s, J, k, level);
    } else {  // too large for the leaf solver: not analysed
      acc.mu_star = pp->mu_max;
      acc.cond = acc.amplification = acc.rel_err_bound = HUGE_VAL;
    }
  }
  pp->leaf = acc;

  // Sample set I_r ascending, as in build_plan_core.
  const uint64_t ks = 1ULL << s;
  pp->samples.assign(ks, 0);
  for (uint64_t a = 0; a < ks; ++a) {
    const uint64_t p = bit_reverse(a, s);
    uint64_t i = 0;
    for (uint32_t u = 0; u < s; ++u)
      if ((p >> u) & 1) i |= 1ULL << (M - 1 - rv[u]);
    pp->samples[a] = i;
  }

  // Twiddles of Lemma 3 from node representatives: all elements whose first
  // u-1 pivot bits spell q_lo agree modulo 2^{r_u}; prefixes without any
  // element get 0 (their outputs belong to no node).
  const uint64_t ntw = ks - 1;
  pp->tw_num.assign(ntw, 0);
  pp->tw_log2den.assign(ntw, 0);
  for (uint32_t u = 1; u <= s; ++u) {
    const uint32_t ru = rv[u - 1];
    const uint64_t off = (1ULL << (u - 1)) - 1;
    for (uint64_t q_lo = 0; q_lo < (1ULL << (u - 1)); ++q_lo) pp->tw_log2den[off + q_lo] = (uint8_t)ru;
    for (size_t v = 0; v < pp->node_slot.size(); ++v) {
      const uint64_t q_lo = pp->node_slot[v] & ((1ULL << (u - 1)) - 1);
      pp->tw_num[off + q_lo] = pp->node_residue[v] & ((1ULL << ru) - 1);
    }
  }
  return HIDFT_OK;
}

}  // namespace hidft
