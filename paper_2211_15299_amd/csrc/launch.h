// Internal launchers of the HIP kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdint.h>

#include "hidft.h"

namespace hidft {

// Twiddles exp(-i pi num[i] / 2^den[i]) in FP64, rounded to complex64.
hipError_t launch_twiddle_gen(const uint64_t* d_num, const uint8_t* d_den, float2* d_tw,
                              uint64_t n, hipStream_t stream);

// Where the short radix group goes when 4 does not divide s.
enum Sched : int { SCHED_SHORT_FIRST = 0, SCHED_SHORT_LAST = 1 };
// Arithmetic of group 1 (values equal the public HIDFT_PREC_*).
enum Prec : int { PREC_FP32 = 0, PREC_F16X2 = 1, PREC_BF16X3 = 2 };

// Launch variant of the fused kernel.  blocks_per_cu caps the persistent grid
// (sizes up to 2^12) at that many blocks per CU; 0 = as many as fit.
struct ExecConfig {
  int sched = SCHED_SHORT_LAST;
  int prec = PREC_FP32;
  int rho = 4;  // log2 points per thread and stages per group: 4 (radix 16) or 5 (radix 32)
  int blocks_per_cu = 0;
};

// Bytes of a plan's split operands of the group-1 matrix (s >= 4).
constexpr size_t AMAT_BYTES = 10 * 64 * 16;

// Split operands of the group-1 matrix in FP64 from the exponents of stages
// 1..4 (a-order entries 0..14), into d_amat (AMAT_BYTES); with radix32 also
// those of the radix-32 group 1 (stages 1..5, entries 0..30) as four 16 x 16
// blocks after them (AMAT32_BYTES more).
constexpr size_t AMAT32_BYTES = 4 * AMAT_BYTES;
hipError_t launch_stage_matrix(const uint64_t* d_num, const uint8_t* d_den, void* d_amat,
                               bool radix32, hipStream_t stream);

// Fused batched transform of size 2^s (s <= HIDFT_MAX_LOG2_K_DEVICE).
// amat may be NULL for PREC_FP32.  hipErrorInvalidValue for a variant that
// does not exist (matrix cores with s < 4, or with the short group first).
// n_out: outputs stored per signal, the first n_out of the gather order
// (0 = all 2^s); the gather table still has 2^s entries.
hipError_t launch_fused(uint32_t s, const float2* in, int64_t ld_in, float2* out,
                        int64_t ld_out, uint64_t batch, const float2* tw, const uint16_t* src,
                        const void* amat, float scale, ExecConfig cfg, hipStream_t stream,
                        uint32_t n_out = 0);

// Transform of size 2^s for HIDFT_MAX_LOG2_K_DEVICE < s <= HIDFT_MAX_LOG2_K_LARGE
// in three passes through `work` (batch * 2^s complex64, not overlapping in
// or out): the top s1 = s - large_split(s) stages per column, the remaining
// s2 stages per subtree of 2^s2 points, whose gather (src2: 2^s2 16-bit LDS
// positions per subtree) puts first each subtree's kept outputs ordered by
// their output index t, then the placement of chunks of large_chunk(s)
// outputs (src3: for each chunk, the workspace index of each of its values,
// in runs per subtree; dest3: the value's place t - chunk start) scaled by
// `scale`.
// n_out: outputs per signal (0 = 2^s); output row b holds n_out values.  The
// tables come from large_tables.  tw holds the twiddles in the split layout
// of device_tw_index.  in may equal out.
uint32_t large_split(uint32_t s);
// Outputs per placement chunk: 4096, or 16384 from s1 = 7 on, where a
// chunk of 4096 would take runs of 32 or fewer outputs from each subtree.
uint32_t large_chunk(uint32_t s);
hipError_t launch_large(uint32_t s, const float2* in, int64_t ld_in, float2* out,
                        int64_t ld_out, uint64_t batch, float2* work, const float2* tw,
                        const uint16_t* src2, const uint32_t* src3, const uint16_t* dest3,
                        float scale, hipStream_t stream, uint64_t n_out = 0);

// Inverse map of the same sizes: the adjoint of launch_large's passes in
// reverse (coefficients in J's order -> workspace by the placement tables,
// subtree inverses, the adjoint column stages), samples in ascending order
// of I_r scaled by `scale`.  Plans that keep all 2^s outputs only.
hipError_t launch_large_inverse(uint32_t s, const float2* coefs, int64_t ld_in, float2* out,
                                int64_t ld_out, uint64_t batch, float2* work, const float2* tw,
                                const uint16_t* src2, const uint32_t* src3,
                                const uint16_t* dest3, float scale, hipStream_t stream);

// Whether launch_fused has the variant (s, sched, prec, rho).
bool fused_variant_exists(uint32_t s, int sched, int prec, int rho);

// Inverse (adjoint) transform of size 2^s: coefficients -> samples, scaled.
hipError_t launch_inverse(uint32_t s, const float2* in, int64_t ld_in, float2* out,
                          int64_t ld_out, uint64_t batch, const float2* tw, const uint16_t* src,
                          float scale, hipStream_t stream);

// LDS bytes of one fused block for size 2^s.
size_t fused_lds_bytes(uint32_t s);

// One instance of a grouped launch: a row of samples, its row of coefficients
// and the plan tables of its size.
struct GroupSlot {
  const float2* in;
  float2* out;
  const float2* tw;
  const uint16_t* src;
  float scale;
};

// A pack: n_slots consecutive slots of the same size 2^log2_k.
struct GroupPack {
  uint32_t first_slot;
  uint16_t log2_k;
  uint16_t n_slots;
};

// GroupPack::log2_k flag: run the pack with the short group first (sizes
// with two schedules); without it, the short group is last.
constexpr uint16_t GROUP_SHORT_FIRST = 0x100;
// GroupPack::log2_k flag: wavefronts whose slots are all empty skip the
// arithmetic (set by the server, whose batches are mostly empty packs).
constexpr uint16_t GROUP_SKIP_IDLE = 0x200;

// Sizes 2^s with s >= GROUP_WIDE_MIN_S go in wide packs (the whole block:
// 1024 threads, up to 2^14 points), smaller ones in narrow packs (a 256-thread
// sub-block: up to 2^12 points).
constexpr uint32_t GROUP_WIDE_MIN_S = 13;
// Narrow sub-blocks per block of the grouped kernel.
constexpr uint32_t GROUP_NARROW_PER_BLOCK = 4;
// The host schedule's fixed cost of a pack, in points (its latency).
constexpr uint64_t GROUP_PACK_COST_POINTS = 2048;
// Narrow packs are split until there are this many per block of the grid:
// fewer, fuller packs than lanes, since a pack has a latency floor.
constexpr uint32_t GROUP_NARROW_SPREAD = 2;

// Instances of size 2^s that one pack holds.
int grouped_slots_per_pack(uint32_t s);

// Blocks of the persistent grouped launch on the current device.
hipError_t grouped_grid(uint32_t* blocks);

// Completion signal of a grouped launch: device counter of finished blocks
// (only grows; *count_base is its value before the launch and is advanced by
// the launch's grid), and a host-mapped flag that the last block sets to seq.
struct GroupDone {
  uint32_t* d_count;
  uint32_t* count_base;
  uint32_t* d_flag;
  uint32_t seq;
};

// Grouped persistent launch of `grid` blocks (at most grouped_grid's): the
// first n_wide packs of d_packs are wide (block b takes packs b, b + grid,
// ...), the next n_narrow narrow; lane l (quarter l % 4 of block l / 4) takes
// narrow packs [d_lane_end[l - 1], d_lane_end[l]) (from 0 for l = 0), so
// d_lane_end holds GROUP_NARROW_PER_BLOCK * grid non-decreasing entries, the
// last n_narrow.  `done` (optional) signals the launch's completion through
// memory.
hipError_t launch_grouped(const GroupPack* d_packs, uint32_t n_wide, uint32_t n_narrow,
                          const GroupSlot* d_slots, const uint32_t* d_lane_end, uint32_t grid,
                          hipStream_t stream, const GroupDone* done = nullptr);
// The same kernel for a few instances, one block each: their descriptors
// and pack codes (a GroupPack::log2_k, flags included) passed by value, so
// no table is read before the transforms.
constexpr uint32_t GROUP_FEW_MAX = 4;
struct GroupFew {
  GroupSlot slot[GROUP_FEW_MAX];
  uint32_t code[GROUP_FEW_MAX];
};
hipError_t launch_grouped_few(const GroupFew& few, uint32_t n, hipStream_t stream,
                              const GroupDone* done = nullptr);

// Largest node (number of aliased coefficients) the leaf solves handle.
constexpr int SAS_MAX_MU = 32;

// Shift-and-Sample leaf solves, plan time: each node's inverse dual
// Vandermonde matrix in FP64, row-major at inv + inv_off[v] (complex128).
hipError_t launch_sas_inverse(uint32_t n_nodes, const uint32_t* node_first,
                              const uint32_t* node_count, const uint32_t* inv_off,
                              const uint64_t* elem_val, uint32_t log2_n, void* inv,
                              hipStream_t stream);

// Per signal: the coefficients c = V_v^{-1} y(v) of every node, from the
// shifted Hi-DFT values y ([signal][shift][node], n_nodes per row), written
// to the caller's positions elem_t of each output row.
// elem_rec: per element (node order), {node | caller position << 16, offset
// of its inverse row, mu(v), 0} as uint4; required when the plan's
// mu* n_nodes + k values fit in SAS_LDS_VALUES (one block per signal).
constexpr uint32_t SAS_LDS_VALUES = 8192;  // 64 KB of complex64
// Zero entries after the inverse table: the solve kernels read four entries
// of every row whatever its length.
constexpr uint32_t SAS_INV_PAD = 16;
hipError_t launch_sas_apply(const float2* y, uint32_t n_nodes, uint32_t mu_star, uint64_t batch,
                            uint32_t k, const uint32_t* elem_node, const uint32_t* node_first,
                            const uint32_t* node_count, const uint32_t* inv_off, const void* inv,
                            const uint32_t* elem_t, const void* elem_rec, float2* out,
                            int64_t ld_out, hipStream_t stream);

// Shift-and-Sample in one kernel: the mu* shifted Hi-DFTs of a signal
// (sample rows j * 2^s of its input row, ld_in >= mu* 2^s) gathered into LDS
// and solved there, with no workspace.  sas_fused_fits tells whether a plan
// qualifies (2^s <= 2^13, mu* = 2..4, k and the LDS within the kernel's
// bounds); elem_rec as for launch_sas_apply.
bool sas_fused_fits(uint32_t s, uint32_t mu_star, uint32_t n_nodes, uint32_t k);
hipError_t launch_sas_fused(uint32_t s, const float2* in, int64_t ld_in, float2* out,
                            int64_t ld_out, uint64_t batch, uint32_t mu_star, uint32_t n_nodes,
                            uint32_t k, const float2* tw, const uint16_t* src_node, float scale,
                            const void* elem_rec, const void* inv, hipStream_t stream);

// Scratch of the allocation-free Shift-and-Sample entry point: a file-scope
// device array of SAS_SCRATCH_BYTES, one copy per GPU, held until the process
// ends.  *ptr receives the current device's copy; its address is looked up
// (hipGetSymbolAddress) on the first call on that device and cached.
constexpr size_t SAS_SCRATCH_BYTES = HIDFT_SAS_SCRATCH_BYTES;
hipError_t sas_scratch(void** ptr);

// Plain method: one signal, one block, one radix-2 stage per barrier.
hipError_t launch_plain(uint32_t s, const float2* in, float2* out, const float2* tw,
                        const uint16_t* src, float scale, hipStream_t stream);

}  // namespace hidft
