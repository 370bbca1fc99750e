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

}  // namespace hidft
