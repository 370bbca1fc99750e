// Host planner of the homogeneous-support DFT: index work only, no HIP.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "hidft.h"

namespace hidft {

// Everything the executor needs, derived from (M, J) by integer arithmetic.
struct PlanCore {
  uint32_t M = 0;                   // N = 2^M
  uint32_t s = 0;                   // k = 2^s
  uint64_t k = 0;
  std::vector<uint64_t> J;          // caller order
  std::vector<uint32_t> pivots;     // r_1 < ... < r_s
  std::vector<uint64_t> samples;    // I_r ascending; samples[a] = i_{bitrev_s(a)}
  std::vector<uint32_t> freq_pos;   // q(J[t])
  std::vector<uint64_t> tw_num;     // schedule order: stage u major, q_lo minor
  std::vector<uint8_t> tw_log2den;  // r_u of each twiddle
};

// Reverses the low nbits bits of x (nbits <= 64); bits above are dropped.
uint64_t bit_reverse(uint64_t x, unsigned nbits);

// Validates (M, J) and returns the pivot levels as a bit mask.
hidft_status analyze_core(uint32_t M, const uint64_t* J, uint64_t k,
                          uint64_t* pivot_mask, std::string* err);

// Full plan derivation; fails unless J is homogeneous and k <= 2^max_log2_k.
hidft_status build_plan_core(uint32_t M, const uint64_t* J, uint64_t k,
                             uint32_t max_log2_k, PlanCore* pc, std::string* err);

// Accuracy of Shift-and-Sample's leaf solves at one level (Algorithm 2,
// Eq. alg1_system): with V_v the mu(v) x mu(v) system of node v and D_v its
// mu* x mu(v) matrix of all shifted rows, the coefficients' relative error is
// at most `amplification` = max_v |V_v^{-1}|_2 max_v |D_v|_2 times that of the
// FP32 Hi-DFT outputs.  rel_err_bound adds the model of the latter
// (sas_hidft_rel_error) and the final rounding to FP32.
struct LeafAccuracy {
  uint32_t mu_star = 1;
  double cond = 1;           // max_v |V_v|_2 |V_v^{-1}|_2
  double amplification = 1;
  double rel_err_bound = 0;
};

// Relative error model of the FP32 Hi-DFT at 2^s points: (2 + s) / 2 units of
// FP32 roundoff (measured: 1.75 units at 2^6 points, 2.5 at 2^14).
double sas_hidft_rel_error(uint32_t s);

// Leaf accuracy of J's nodes at `level` with 2^s-point Hi-DFTs.  O(sum_v
// mu(v)^3) FP64 work; nodes of equal shape are analysed once.
LeafAccuracy leaf_accuracy(uint32_t M, uint32_t s, const uint64_t* J, uint64_t k,
                           uint32_t level);

// Plan of the Hi-DFT at a pivot vector r of an r-part-homogeneous J
// (Sec. VI Def. part-homogeneous, Sec. VII-B, Algorithm 2): nodes of T(J) at
// level r_max + 1 are indexed by the slot q = sum_u bit_{r_u}(residue) 2^{u-1},
// which part-homogeneity makes injective on nodes.
struct PartPlan {
  uint32_t M = 0;
  uint32_t s = 0;                   // |r|; the Hi-DFT has 2^s samples and slots
  uint32_t level = 0;               // r_max + 1 (0 when r is empty)
  uint32_t mu_max = 0;              // mu*: largest node
  uint64_t k = 0;                   // |J|
  std::vector<uint64_t> J;
  std::vector<uint32_t> pivots;     // r, ascending
  std::vector<uint64_t> samples;    // I_r ascending (2^s)
  std::vector<uint64_t> tw_num;     // 2^s - 1 twiddles, schedule order (stage u, q_lo)
  std::vector<uint8_t> tw_log2den;
  std::vector<uint32_t> node_slot;  // per node, nodes in ascending slot order
  std::vector<uint64_t> node_residue;
  std::vector<uint32_t> node_first; // into elem_t
  std::vector<uint32_t> node_count; // mu(v)
  std::vector<uint32_t> elem_t;     // caller positions, grouped by node, ascending within
  double cost = 0;                  // Lemma 4 with c1 = 3/2, c2 = 6
  LeafAccuracy leaf;                // conditioning of the leaf systems (infinite if mu* > max_mu)
};

// Builds the plan.  If r == nullptr the pivot vector is chosen: the first t
// pivots of J (J is part-homogeneous at any such prefix) for the t that
// minimises Lemma 4's cost among those with mu* <= max_mu, t <= max_s (or
// t <= max_s_mu1 when every node holds one element) and a leaf error bound
// <= max_err (UNSUPPORTED if there is none).  A given r is only checked for
// part-homogeneity and the same size limits; its accuracy is recorded (when
// mu* <= max_mu) for the caller to judge.
hidft_status build_part_plan(uint32_t M, const uint64_t* J, uint64_t k, const uint32_t* r,
                             uint32_t nr, uint32_t max_s, uint32_t max_s_mu1, uint32_t max_mu,
                             double max_err, PartPlan* pp, std::string* err);

}  // namespace hidft
