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
  uint16_t* d_src = nullptr;   // k output gather positions
  // Split operands of the group-1 matrix (k >= 16), built on the first
  // matrix-core execution (hidft::plan_amat) and kept until destroy.
  std::atomic<void*> d_amat{nullptr};
  std::mutex amat_mu;
  std::atomic<size_t> device_bytes{0};
  float scale = 1.0f;          // N / k
};

namespace hidft {

// Device bytes of a plan's tables at creation: k - 1 twiddles (at least one)
// and k gather positions.  (The matrix-core operands come later, on demand.)
size_t plan_table_bytes(uint64_t k);

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

// Orders instances (size log2, descriptor) by size, largest first, and packs
// instances of equal size into packs of at most grouped_slots_per_pack(s).
// short_first: the packs of sizes with two schedules run with the short
// group first (GROUP_SHORT_FIRST in GroupPack::log2_k), else last.
// grid > 0 (the persistent grid's block count): when the packs do not fill
// whole rounds of the grid, the packs of the last, partial round are split
// into packs of fewer instances until that round has one pack per block (or
// no pack has two instances left), so the last round spreads over every
// CU instead of a few; 0 leaves the packs full.
// snake_rounds > 0: the pack list is reordered so that the persistent grid
// of snake_rounds blocks takes, in alternate rounds, the largest and the
// smallest remaining packs (a block with a long first pack gets a short
// second one); 0 keeps largest first.
void pack_instances(const std::vector<std::pair<uint32_t, GroupSlot>>& inst,
                    std::vector<GroupPack>* packs, std::vector<GroupSlot>* slots,
                    uint32_t grid, bool short_first = false, uint32_t snake_rounds = 0);

}  // namespace hidft
