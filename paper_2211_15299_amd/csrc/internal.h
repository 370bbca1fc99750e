// Library-internal types shared by the C ABI, the group API and the server.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "hidft.h"
#include "launch.h"
#include "plan_core.h"

struct hidft_plan_s {
  hidft::PlanCore core;
  bool host_only = true;
  int device = -1;
  float2* d_tw = nullptr;      // k-1 twiddles in a-order (at least one slot)
  uint16_t* d_src = nullptr;   // k output gather positions (k <= 2^14); 2k for larger plans
  uint32_t* d_pos = nullptr;   // k > 2^14: the placement pass's workspace indices
  // Split operands of the group-1 matrix (k >= 16), built on the first
  // matrix-core execution (hidft::plan_amat) and kept until destroy.
  std::atomic<void*> d_amat{nullptr};
  std::mutex amat_mu;
  std::atomic<size_t> device_bytes{0};
  float scale = 1.0f;          // N / k
};

namespace hidft {

// Device bytes of a plan's tables at creation: k - 1 twiddles (at least one)
// and k gather positions (2 bytes each up to 2^14; larger plans: 8 bytes
// per point of pass tables).  (The
// matrix-core operands come later, on demand.)
size_t plan_table_bytes(uint64_t k);

// Entry of the device twiddle table that holds stage u's twiddle for the
// node named by the top u - 1 bits n of the position (a-order).  Up to
// 2^HIDFT_MAX_LOG2_K_DEVICE points: (2^{u-1} - 1) + n.  Above, the split
// layout of the passes (launch_large): stages 1..s1 as before, then for each
// subtree (the top s1 bits of n) the table of its 2^s2-point transform.
uint64_t device_tw_index(uint32_t s, uint32_t u, uint64_t n);

// Tables of the passes of a transform of 2^s > 2^HIDFT_MAX_LOG2_K_DEVICE
// points (launch_large) that keeps n_out = pos.size() outputs, output t
// being the value at position pos[t] (distinct, < 2^s).  Subtree j holds
// the outputs t with pos[t] >> s2 == j; L_j lists them by increasing t.
//   src16[0, 2^s): per subtree j, entry i < |L_j| = pos[L_j[i]] mod 2^s2 (the
//                subtree's gather, so its kept outputs come first, ordered by
//                t; the other entries are 0);
//   src16[2^s, 2^s + n) and src32[0, n), n = n_out rounded up to whole
//                chunks of large_chunk(s): per output chunk, the chunk's values subtree
//                by subtree: the workspace index j 2^s2 + i of L_j[i] (src32)
//                and its place L_j[i] - chunk start (src16[2^s + ...]).
void large_tables(uint32_t s, const std::vector<uint32_t>& pos, std::vector<uint16_t>* src16,
                  std::vector<uint32_t>* src32);

// HIDFT_ERR_UNSUPPORTED (with a message naming fn) for a plan of more than
// 2^HIDFT_MAX_LOG2_K_DEVICE points, which only hidft_execute and
// hidft_execute_ws run; HIDFT_OK otherwise.
hidft_status require_single_pass(const hidft_plan plan, const char* fn);

// The plan's matrix-core operands, built on first use: allocated, computed
// in FP64 on the device on `stream` and waited for (the first matrix-core
// execution of a plan is synchronous).  Thread-safe.
hidft_status plan_amat(hidft_plan plan, hipStream_t stream, void** amat, const char* fn);

// Records a failure message for hidft_last_error() and returns `st`.
hidft_status set_error(hidft_status st, const std::string& msg);

// HIP error -> status (OUT_OF_MEMORY or DEVICE) with a message.
hidft_status hip_error(hipError_t e, const char* what);

// Public execution variant -> launch variant for this plan (records the
// error message and returns INVALID_ARGUMENT / UNSUPPORTED when it has none).
hidft_status resolve_config(const hidft_plan plan, const hidft_exec_config* cfg,
                            ExecConfig* out, const char* fn);

// The tuned variant recorded by hidft_autotune for this plan's device and
// size, the precision and the class of `batch`; false if there is none.
bool tune_lookup(const hidft_plan plan, uint32_t precision, uint64_t batch,
                 hidft_exec_config* cfg);

// The schedule of one grouped launch.
struct GroupSchedule {
  std::vector<GroupPack> packs;    // n_wide wide packs, then the narrow packs by lane
  std::vector<GroupSlot> slots;    // instance descriptors, in pack order
  std::vector<uint32_t> lane_end;  // GROUP_NARROW_PER_BLOCK * grid entries
  uint32_t n_wide = 0;
  uint32_t grid = 0;               // blocks of the launch
  uint32_t n_narrow() const { return (uint32_t)packs.size() - n_wide; }
};

// Orders instances (size log2, descriptor) by size, largest first, and packs
// instances of equal size into packs of at most grouped_slots_per_pack(s):
// wide packs for s >= GROUP_WIDE_MIN_S, narrow ones below.  max_grid is the
// persistent grid's block count.
//
// Wide packs: block b of the launch takes wide packs b, b + grid, ...  When
// they do not fill whole rounds of max_grid, the packs of the last, partial
// round are split into packs of fewer instances until that round has one
// pack per block (or no pack has two instances left), so the last round
// spreads over every CU instead of a few.  alternate: the wide packs are
// reordered so that the blocks take, in alternate rounds, the largest and
// the smallest remaining packs (a block with a long first pack gets a short
// second one); else largest first.
//
// Narrow packs: split likewise until there are GROUP_NARROW_SPREAD per
// block of max_grid (or single instances), then scheduled by a longest-first
// greedy: each pack, largest first, goes to the block with the least
// estimated time so far (a block starts from its wide packs), and a block's
// narrow packs go, in the same way, to its four lanes (quarter blocks, lane
// = 4 block + quarter).  The estimate of a pack is its points plus
// GROUP_PACK_COST_POINTS: the lanes of a CU share its throughput.
// short_first: the packs of sizes with two schedules run with the short
// group first (GROUP_SHORT_FIRST in GroupPack::log2_k), else last.
void pack_instances(const std::vector<std::pair<uint32_t, GroupSlot>>& inst, uint32_t max_grid,
                    bool short_first, bool alternate, GroupSchedule* out);

}  // namespace hidft
