// C ABI of the homogeneous-support DFT: argument checks, plan lifecycle and
// dispatch to the HIP kernels.  Nothing throws across this boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include <algorithm>
#include <functional>
#include <queue>
#include <vector>

#include "hidft.h"
#include "internal.h"

struct hidft_group_s {
  int device = -1;
  uint64_t n_instances = 0;
  uint32_t n_packs = 0;
  uint32_t n_wide = 0;          // the first n_wide packs are wide
  uint32_t grid = 0;            // blocks of the launch
  hidft::GroupPack* d_packs = nullptr;
  uint32_t* d_lanes = nullptr;  // lane_end of the schedule (4 per block)
  hidft::GroupSlot* d_slots = nullptr;
  size_t device_bytes = 0;
  std::vector<std::pair<uint32_t, hidft::GroupSlot>> inst;  // for re-packing
  hidft_group_config cfg{HIDFT_SCHED_DEFAULT, HIDFT_GROUP_ORDER_LARGEST_FIRST};
};

namespace {

thread_local std::string g_last_error;

hidft_status fail(hidft_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

hidft_status ok() {
  g_last_error.clear();
  return HIDFT_OK;
}

hidft_status hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory)
    return fail(HIDFT_ERR_OUT_OF_MEMORY, "%s: %s", what, hipGetErrorString(e));
  return fail(HIDFT_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void release_device(hidft_plan p) {
  if (p->d_tw) (void)hipFree(p->d_tw);
  if (p->d_src) (void)hipFree(p->d_src);
  if (p->d_pos) (void)hipFree(p->d_pos);
  p->d_pos = nullptr;
  void* am = p->d_amat.exchange(nullptr);
  if (am) (void)hipFree(am);
  p->d_tw = nullptr;
  p->d_src = nullptr;
}

// Twiddle exponents in the device order of the twiddle table: stage u's
// node q_lo (schedule order) is node bitrev_{u-1}(q_lo) in a-order.
void device_exponents(const hidft::PlanCore& c, std::vector<uint64_t>* num,
                      std::vector<uint8_t>* den) {
  const uint64_t ntw = c.k - 1;
  num->assign(ntw ? ntw : 1, 0);
  den->assign(ntw ? ntw : 1, 0);
  for (uint32_t u = 1; u <= c.s; ++u) {
    const uint64_t off = (1ULL << (u - 1)) - 1;
    for (uint64_t q_lo = 0; q_lo < (1ULL << (u - 1)); ++q_lo) {
      const uint64_t at = hidft::device_tw_index(c.s, u, hidft::bit_reverse(q_lo, u - 1));
      (*num)[at] = c.tw_num[off + q_lo];
      (*den)[at] = c.tw_log2den[off + q_lo];
    }
  }
}

// Uploads the device tables and generates the twiddles on `stream`.
hidft_status upload(hidft_plan p, hipStream_t stream) {
  const hidft::PlanCore& c = p->core;
  const uint64_t k = c.k;
  const uint64_t ntw = k - 1;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");

  std::vector<uint64_t> num;
  std::vector<uint8_t> den;
  device_exponents(c, &num, &den);
  // Output positions (a-order) of the caller's coefficients, for the
  // single-pass gather; larger plans get the tables of their passes.
  const bool large = c.s > HIDFT_MAX_LOG2_K_DEVICE;
  std::vector<uint16_t> src;
  std::vector<uint32_t> pos;
  if (!large) {
    src.resize(k);
    for (uint64_t t = 0; t < k; ++t)
      src[t] = static_cast<uint16_t>(hidft::bit_reverse(c.freq_pos[t], c.s));
  } else {
    std::vector<uint32_t> p(k);
    for (uint64_t t = 0; t < k; ++t)
      p[t] = static_cast<uint32_t>(hidft::bit_reverse(c.freq_pos[t], c.s));
    hidft::large_tables(c.s, p, &src, &pos);
  }

  const size_t ntw_alloc = ntw ? ntw : 1;
  uint64_t* d_num = nullptr;
  uint8_t* d_den = nullptr;
  hidft_status st = HIDFT_OK;
  if ((e = hipMalloc(&p->d_tw, ntw_alloc * sizeof(float2))) != hipSuccess ||
      (e = hipMalloc(&p->d_src, src.size() * sizeof(uint16_t))) != hipSuccess ||
      (large && (e = hipMalloc(&p->d_pos, pos.size() * sizeof(uint32_t))) != hipSuccess) ||
      (e = hipMalloc(&d_num, ntw_alloc * sizeof(uint64_t))) != hipSuccess ||
      (e = hipMalloc(&d_den, ntw_alloc)) != hipSuccess) {
    st = hip_fail(e, "hipMalloc of plan tables");
  } else if ((e = hipMemcpyAsync(d_num, num.data(), ntw_alloc * sizeof(uint64_t),
                                 hipMemcpyHostToDevice, stream)) != hipSuccess ||
             (e = hipMemcpyAsync(d_den, den.data(), ntw_alloc, hipMemcpyHostToDevice,
                                 stream)) != hipSuccess ||
             (e = hipMemcpyAsync(p->d_src, src.data(), src.size() * sizeof(uint16_t),
                                 hipMemcpyHostToDevice, stream)) != hipSuccess ||
             (large && (e = hipMemcpyAsync(p->d_pos, pos.data(), pos.size() * sizeof(uint32_t),
                                           hipMemcpyHostToDevice, stream)) != hipSuccess)) {
    st = hip_fail(e, "hipMemcpyAsync of plan tables");
  } else if ((e = hidft::launch_twiddle_gen(d_num, d_den, p->d_tw, ntw, stream)) !=
             hipSuccess) {
    st = hip_fail(e, "twiddle generation launch");
  } else if ((e = hipStreamSynchronize(stream)) != hipSuccess) {
    st = hip_fail(e, "hipStreamSynchronize after plan upload");
  }
  if (d_num) (void)hipFree(d_num);
  if (d_den) (void)hipFree(d_den);
  if (st != HIDFT_OK) {
    release_device(p);
    return st;
  }
  p->device_bytes = hidft::plan_table_bytes(k);
  return HIDFT_OK;
}

// Common argument checks of the execute calls.
hidft_status check_exec(hidft_plan plan, const void* d_in, int64_t ld_in, const void* d_out,
                        int64_t ld_out, uint64_t batch, const char* fn) {
  if (!plan) return fail(HIDFT_ERR_INVALID_ARGUMENT, "%s: plan is NULL", fn);
  if (plan->host_only)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "%s: plan was created HOST_ONLY", fn);
  if (batch == 0) return HIDFT_OK;
  const uint64_t k = plan->core.k;
  if (!d_in || !d_out) return fail(HIDFT_ERR_INVALID_ARGUMENT, "%s: NULL buffer", fn);
  if ((reinterpret_cast<uintptr_t>(d_in) | reinterpret_cast<uintptr_t>(d_out)) & 7u)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "%s: buffers must be 8-byte aligned", fn);
  if (ld_in < 0 || ld_out < 0 || (uint64_t)ld_in < k || (uint64_t)ld_out < k)
    return fail(HIDFT_ERR_INVALID_ARGUMENT,
                "%s: leading dimensions (%lld, %lld) must be >= k = %llu", fn,
                (long long)ld_in, (long long)ld_out, (unsigned long long)k);
  if (batch > (1ULL << 40))
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "%s: batch too large", fn);
  const uint64_t span_in = ((batch - 1) * (uint64_t)ld_in + k) * sizeof(float2);
  const uint64_t span_out = ((batch - 1) * (uint64_t)ld_out + k) * sizeof(float2);
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(d_in), a1 = a0 + span_in;
  const uintptr_t b0 = reinterpret_cast<uintptr_t>(d_out), b1 = b0 + span_out;
  const bool overlap = a0 < b1 && b0 < a1;
  if (overlap && !(a0 == b0 && ld_in == ld_out))
    return fail(HIDFT_ERR_INVALID_ARGUMENT,
                "%s: input and output overlap other than exactly in place", fn);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, fn);
  if (dev != plan->device)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "%s: current device %d, plan lives on device %d",
                fn, dev, plan->device);
  return HIDFT_OK;
}

}  // namespace

namespace hidft {

// Entry of the device twiddle table that holds stage u's twiddle for the
// node named by the top u - 1 bits n of the position (a-order).  Up to
// 2^HIDFT_MAX_LOG2_K_DEVICE points: (2^{u-1} - 1) + n.  Above, the split
// layout of the passes (launch_large): stages 1..s1 as before, then for each
// subtree (the top s1 bits of n) the table of its 2^s2-point transform.
uint64_t device_tw_index(uint32_t s, uint32_t u, uint64_t n) {
  if (s <= HIDFT_MAX_LOG2_K_DEVICE) return ((1ULL << (u - 1)) - 1) + n;
  const uint32_t s2 = hidft::large_split(s), s1 = s - s2;
  if (u <= s1) return ((1ULL << (u - 1)) - 1) + n;
  const uint32_t u2 = u - s1;
  const uint64_t sub = n >> (u2 - 1), n2 = n & ((1ULL << (u2 - 1)) - 1);
  return ((1ULL << s1) - 1) + sub * ((1ULL << s2) - 1) + ((1ULL << (u2 - 1)) - 1) + n2;
}

void large_tables(uint32_t s, const std::vector<uint32_t>& pos, std::vector<uint16_t>* src16,
                  std::vector<uint32_t>* src32) {
  const uint64_t k = 1ULL << s, n_out = pos.size();
  const uint32_t s2 = large_split(s), s1 = s - s2;
  const uint64_t K2 = 1ULL << s2, C = large_chunk(s);
  const uint64_t chunks = (n_out + C - 1) / C;
  std::vector<std::vector<uint32_t>> L(1ULL << s1);
  for (uint64_t t = 0; t < n_out; ++t) L[pos[t] >> s2].push_back(static_cast<uint32_t>(t));
  src16->assign(k + chunks * C, 0);
  src32->assign(chunks * C, 0);
  for (uint64_t j = 0; j < L.size(); ++j)
    for (uint64_t i = 0; i < L[j].size(); ++i)
      (*src16)[j * K2 + i] = static_cast<uint16_t>(pos[L[j][i]] & (K2 - 1));
  std::vector<uint64_t> next(L.size(), 0);
  for (uint64_t ch = 0; ch < chunks; ++ch) {
    uint64_t e = ch * C;
    for (uint64_t j = 0; j < L.size(); ++j) {
      for (uint64_t& i = next[j]; i < L[j].size() && L[j][i] < (ch + 1) * C; ++i, ++e) {
        (*src32)[e] = static_cast<uint32_t>(j * K2 + i);
        (*src16)[k + e] = static_cast<uint16_t>(L[j][i] - ch * C);
      }
    }
  }
}

size_t plan_table_bytes(uint64_t k) {
  // gather positions: 2 bytes per point; the passes of larger plans: 8
  const size_t pos_bytes = k > (1ULL << HIDFT_MAX_LOG2_K_DEVICE) ? 8 : 2;
  return (k > 1 ? k - 1 : 1) * sizeof(float2) + k * pos_bytes;
}

hidft_status require_single_pass(const hidft_plan plan, const char* fn) {
  if (plan && plan->core.s > HIDFT_MAX_LOG2_K_DEVICE)
    return fail(HIDFT_ERR_UNSUPPORTED,
                "%s: k = 2^%u runs only through hidft_execute / hidft_execute_ws (this call "
                "needs k <= 2^%u, one signal staged in LDS)",
                fn, plan->core.s, HIDFT_MAX_LOG2_K_DEVICE);
  return HIDFT_OK;
}

hidft_status plan_amat(hidft_plan p, hipStream_t stream, void** amat, const char* fn) {
  void* am = p->d_amat.load(std::memory_order_acquire);
  if (am) {
    *amat = am;
    return HIDFT_OK;
  }
  std::lock_guard<std::mutex> lk(p->amat_mu);
  am = p->d_amat.load(std::memory_order_acquire);
  if (am) {
    *amat = am;
    return HIDFT_OK;
  }
  const hidft::PlanCore& c = p->core;
  if (c.s < 4) return fail(HIDFT_ERR_UNSUPPORTED, "%s: matrix cores need k >= 16", fn);
  if (hidft_status st = require_single_pass(p, fn)) return st;
  // Radix-16 operands for k >= 16, the radix-32 ones after them for k >= 2^13.
  const bool with_amat32 = c.s >= 13;
  const size_t amat_bytes = AMAT_BYTES + (with_amat32 ? AMAT32_BYTES : 0);
  std::vector<uint64_t> num;
  std::vector<uint8_t> den;
  device_exponents(c, &num, &den);
  uint64_t* d_num = nullptr;
  uint8_t* d_den = nullptr;
  hipError_t e;
  hidft_status st = HIDFT_OK;
  if ((e = hipMalloc(&am, amat_bytes)) != hipSuccess ||
      (e = hipMalloc(&d_num, num.size() * sizeof(uint64_t))) != hipSuccess ||
      (e = hipMalloc(&d_den, den.size())) != hipSuccess ||
      (e = hipMemcpyAsync(d_num, num.data(), num.size() * sizeof(uint64_t),
                          hipMemcpyHostToDevice, stream)) != hipSuccess ||
      (e = hipMemcpyAsync(d_den, den.data(), den.size(), hipMemcpyHostToDevice, stream)) !=
          hipSuccess ||
      (e = launch_stage_matrix(d_num, d_den, am, with_amat32, stream)) != hipSuccess ||
      (e = hipStreamSynchronize(stream)) != hipSuccess)
    st = hip_fail(e, "matrix operands of the first group");
  if (d_num) (void)hipFree(d_num);
  if (d_den) (void)hipFree(d_den);
  if (st != HIDFT_OK) {
    if (am) (void)hipFree(am);
    return st;
  }
  p->device_bytes.fetch_add(amat_bytes, std::memory_order_relaxed);
  p->d_amat.store(am, std::memory_order_release);
  *amat = am;
  return HIDFT_OK;
}

hidft_status set_error(hidft_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

hidft_status hip_error(hipError_t e, const char* what) { return hip_fail(e, what); }

namespace {

// Splits the largest packs of `tail` in two (its first slots stay, the rest
// become a new pack) until it has `want` packs or no pack has two instances.
void spread_packs(std::vector<GroupPack>* tail, size_t want) {
  while (tail->size() < want) {
    size_t big = 0;
    for (size_t i = 1; i < tail->size(); ++i)
      if ((*tail)[i].n_slots > (*tail)[big].n_slots) big = i;
    if (tail->empty() || (*tail)[big].n_slots < 2) break;
    GroupPack rest = (*tail)[big];
    (*tail)[big].n_slots = (uint16_t)((rest.n_slots + 1) / 2);
    rest.first_slot += (*tail)[big].n_slots;
    rest.n_slots = (uint16_t)(rest.n_slots - (*tail)[big].n_slots);
    tail->push_back(rest);
  }
}

}  // namespace

void pack_instances(const std::vector<std::pair<uint32_t, GroupSlot>>& inst, uint32_t max_grid,
                    bool short_first, bool alternate, GroupSchedule* out) {
  std::vector<uint64_t> per_size(HIDFT_MAX_LOG2_K_DEVICE + 1, 0);
  for (const auto& x : inst) per_size[x.first]++;
  std::vector<uint64_t> next(HIDFT_MAX_LOG2_K_DEVICE + 1, 0);
  uint64_t off = 0;
  for (int s = HIDFT_MAX_LOG2_K_DEVICE; s >= 0; --s) {
    next[s] = off;
    off += per_size[s];
  }
  out->slots.resize(inst.size());
  for (const auto& x : inst) out->slots[next[x.first]++] = x.second;
  std::vector<GroupPack> wide, narrow;
  off = 0;
  for (int s = HIDFT_MAX_LOG2_K_DEVICE; s >= 0; --s) {
    const uint64_t per = (uint64_t)grouped_slots_per_pack((uint32_t)s);
    for (uint64_t first = 0; first < per_size[s]; first += per) {
      GroupPack pk;
      pk.first_slot = (uint32_t)(off + first);
      pk.log2_k = (uint16_t)(s | (short_first ? GROUP_SHORT_FIRST : 0));
      pk.n_slots = (uint16_t)std::min<uint64_t>(per, per_size[s] - first);
      ((uint32_t)s >= GROUP_WIDE_MIN_S ? wide : narrow).push_back(pk);
    }
    off += per_size[s];
  }
  if (max_grid == 0) max_grid = 1;
  const size_t full = wide.size() / max_grid * max_grid;
  if (full > 0 && full < wide.size()) {
    // Measured on the uneven configuration with whole-block packs only (348
    // packs on 256 blocks): 46 -> 38.5 us, the same results.
    std::vector<GroupPack> tail(wide.begin() + full, wide.end());
    spread_packs(&tail, max_grid);
    wide.resize(full);
    wide.insert(wide.end(), tail.begin(), tail.end());
  }
  if (alternate && wide.size() > max_grid) {
    // Round r of the grid takes packs [r G, (r + 1) G) of the new list;
    // rounds alternate between the largest and the smallest packs left.
    std::vector<GroupPack> alt;
    alt.reserve(wide.size());
    size_t lo = 0, hi = wide.size();
    for (uint32_t r = 0; lo < hi; ++r) {
      const size_t n = std::min<size_t>(max_grid, hi - lo);
      if (r % 2 == 0) {
        for (size_t i = 0; i < n; ++i) alt.push_back(wide[lo + i]);
        lo += n;
      } else {
        // smallest first, so that block b (whose first pack was among the
        // largest) gets one of the smallest
        for (size_t i = 0; i < n; ++i) alt.push_back(wide[hi - 1 - i]);
        hi -= n;
      }
    }
    wide.swap(alt);
  }
  spread_packs(&narrow, (size_t)max_grid * GROUP_NARROW_SPREAD);
  const size_t blocks = std::max(wide.size(), narrow.size());
  out->grid = (uint32_t)std::max<size_t>(1, std::min<size_t>(max_grid, blocks));
  out->n_wide = (uint32_t)wide.size();
  const uint32_t grid = out->grid, lanes = grid * GROUP_NARROW_PER_BLOCK;
  // A CU's packs share its throughput: the estimated time of a block is the
  // points of its packs, plus a fixed cost per pack for its latency.
  auto cost = [](const GroupPack& pk) {
    return ((uint64_t)pk.n_slots << (pk.log2_k & 0xffu)) + GROUP_PACK_COST_POINTS;
  };
  // Longest-first greedy over the blocks (ties: lower block first), the
  // blocks starting from their wide packs; then, within a block, over its
  // lanes (ties: lower quarter first).
  std::vector<uint64_t> block_time(grid, 0);
  for (size_t i = 0; i < wide.size(); ++i) block_time[i % grid] += cost(wide[i]);
  using Key = std::pair<uint64_t, uint32_t>;
  std::priority_queue<Key, std::vector<Key>, std::greater<Key>> heap;
  for (uint32_t b = 0; b < grid; ++b) heap.emplace(block_time[b], b);
  std::vector<std::vector<uint32_t>> block_packs(grid);
  for (uint32_t i = 0; i < (uint32_t)narrow.size(); ++i) {
    const Key top = heap.top();
    heap.pop();
    block_packs[top.second].push_back(i);
    heap.emplace(top.first + cost(narrow[i]), top.second);
  }
  std::vector<std::vector<uint32_t>> lane_packs(lanes);
  for (uint32_t b = 0; b < grid; ++b) {
    uint64_t lane_time[GROUP_NARROW_PER_BLOCK] = {};
    for (uint32_t i : block_packs[b]) {
      uint32_t q = 0;
      for (uint32_t j = 1; j < GROUP_NARROW_PER_BLOCK; ++j)
        if (lane_time[j] < lane_time[q]) q = j;
      lane_time[q] += cost(narrow[i]);
      lane_packs[b * GROUP_NARROW_PER_BLOCK + q].push_back(i);
    }
  }
  out->packs.swap(wide);
  out->lane_end.assign(lanes, 0);
  for (uint32_t l = 0; l < lanes; ++l) {
    for (uint32_t i : lane_packs[l]) out->packs.push_back(narrow[i]);
    out->lane_end[l] = (uint32_t)out->packs.size() - out->n_wide;
  }
}

}  // namespace hidft

namespace hidft {

hidft_status resolve_config(const hidft_plan plan, const hidft_exec_config* cfg, ExecConfig* out,
                            const char* fn) {
  const uint32_t s = plan->core.s;
  if (hidft_status st = require_single_pass(plan, fn)) return st;
  if (cfg->precision > HIDFT_PREC_BF16X3)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "%s: unknown precision %u", fn, cfg->precision);
  if (cfg->schedule > HIDFT_SCHED_SHORT_LAST)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "%s: unknown schedule %u", fn, cfg->schedule);
  if (cfg->radix != 0 && cfg->radix != 16 && cfg->radix != 32)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "%s: radix %u is not 0, 16 or 32", fn, cfg->radix);
  ExecConfig c;
  c.prec = (int)cfg->precision;  // HIDFT_PREC_* values equal Prec
  c.sched = cfg->schedule == HIDFT_SCHED_SHORT_FIRST ? SCHED_SHORT_FIRST : SCHED_SHORT_LAST;
  c.rho = cfg->radix == 32 ? 5 : 4;
  c.blocks_per_cu = cfg->blocks_per_cu > 1024 ? 1024 : (int)cfg->blocks_per_cu;
  if (c.prec != PREC_FP32 && s < 4)
    return fail(HIDFT_ERR_UNSUPPORTED,
                "%s: the matrix-core precisions need k >= 16 (a radix-16 first group), k = %llu",
                fn, (unsigned long long)plan->core.k);
  if (c.rho == 5 && s < 13)
    return fail(HIDFT_ERR_UNSUPPORTED, "%s: radix 32 needs k >= 2^13 (s = %u)", fn, s);
  if (!fused_variant_exists(s, c.sched, c.prec, c.rho))
    return fail(HIDFT_ERR_UNSUPPORTED,
                "%s: the matrix-core precisions need a full radix-%u group first "
                "(schedule SHORT_LAST or DEFAULT) when %u does not divide s = %u",
                fn, c.rho == 5 ? 32u : 16u, (unsigned)c.rho, s);
  *out = c;
  return HIDFT_OK;
}

}  // namespace hidft

extern "C" {

const char* hidft_status_string(hidft_status st) {
  switch (st) {
    case HIDFT_OK: return "HIDFT_OK";
    case HIDFT_ERR_INVALID_ARGUMENT: return "HIDFT_ERR_INVALID_ARGUMENT";
    case HIDFT_ERR_INDEX_OUT_OF_RANGE: return "HIDFT_ERR_INDEX_OUT_OF_RANGE";
    case HIDFT_ERR_DUPLICATE_INDEX: return "HIDFT_ERR_DUPLICATE_INDEX";
    case HIDFT_ERR_SIZE_NOT_POW2: return "HIDFT_ERR_SIZE_NOT_POW2";
    case HIDFT_ERR_NOT_HOMOGENEOUS: return "HIDFT_ERR_NOT_HOMOGENEOUS";
    case HIDFT_ERR_OUT_OF_MEMORY: return "HIDFT_ERR_OUT_OF_MEMORY";
    case HIDFT_ERR_DEVICE: return "HIDFT_ERR_DEVICE";
    case HIDFT_ERR_UNSUPPORTED: return "HIDFT_ERR_UNSUPPORTED";
  }
  return "HIDFT_ERR_UNKNOWN";
}

const char* hidft_last_error(void) { return g_last_error.c_str(); }

hidft_status hidft_analyze(uint32_t log2_n, const uint64_t* J, uint64_t k, uint32_t* pivots,
                           uint32_t* n_pivots, int32_t* is_homogeneous) {
  try {
    uint64_t mask = 0;
    std::string err;
    hidft_status st = hidft::analyze_core(log2_n, J, k, &mask, &err);
    if (st != HIDFT_OK) return fail(st, "hidft_analyze: %s", err.c_str());
    uint32_t n = 0;
    for (uint32_t e = 0; e < 64; ++e)
      if ((mask >> e) & 1) {
        if (pivots) pivots[n] = e;
        ++n;
      }
    if (n_pivots) *n_pivots = n;
    if (is_homogeneous)
      *is_homogeneous = ((k & (k - 1)) == 0 && (uint32_t)__builtin_ctzll(k) == n) ? 1 : 0;
    return ok();
  } catch (const std::bad_alloc&) {
    return fail(HIDFT_ERR_OUT_OF_MEMORY, "hidft_analyze: host allocation failed");
  } catch (...) {
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_analyze: unexpected exception");
  }
}

hidft_status hidft_plan_create(uint32_t log2_n, const uint64_t* J, uint64_t k, uint32_t flags,
                               void* stream, hidft_plan* out) {
  if (!out) return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_plan_create: out is NULL");
  *out = nullptr;
  if (flags & ~HIDFT_PLAN_HOST_ONLY)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_plan_create: unknown flags 0x%x", flags);
  const bool host_only = (flags & HIDFT_PLAN_HOST_ONLY) != 0;
  hidft_plan p = nullptr;
  try {
    p = new hidft_plan_s;
    std::string err;
    const uint32_t max_s = host_only ? HIDFT_MAX_LOG2_K_HOST : HIDFT_MAX_LOG2_K_LARGE;
    hidft_status st = hidft::build_plan_core(log2_n, J, k, max_s, &p->core, &err);
    if (st != HIDFT_OK) {
      delete p;
      return fail(st, "hidft_plan_create: %s", err.c_str());
    }
    p->host_only = host_only;
    p->scale = std::ldexp(1.0f, (int)(p->core.M - p->core.s));
    if (!host_only) {
      st = upload(p, static_cast<hipStream_t>(stream));
      if (st != HIDFT_OK) {
        std::string msg = g_last_error;
        delete p;
        return fail(st, "hidft_plan_create: %s", msg.c_str());
      }
    }
    *out = p;
    return ok();
  } catch (const std::bad_alloc&) {
    if (p) {
      release_device(p);
      delete p;
    }
    return fail(HIDFT_ERR_OUT_OF_MEMORY, "hidft_plan_create: host allocation failed");
  } catch (...) {
    if (p) {
      release_device(p);
      delete p;
    }
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_plan_create: unexpected exception");
  }
}

hidft_status hidft_plan_destroy(hidft_plan plan) {
  if (!plan) return ok();
  release_device(plan);
  delete plan;
  return ok();
}

hidft_status hidft_plan_get_info(hidft_plan plan, uint32_t* log2_n, uint64_t* k,
                                 uint32_t* n_pivots) {
  if (!plan) return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_plan_get_info: plan is NULL");
  if (log2_n) *log2_n = plan->core.M;
  if (k) *k = plan->core.k;
  if (n_pivots) *n_pivots = plan->core.s;
  return ok();
}

hidft_status hidft_plan_get_pivots(hidft_plan plan, uint32_t* pivots) {
  if (!plan || !pivots)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_plan_get_pivots: NULL argument");
  std::memcpy(pivots, plan->core.pivots.data(), plan->core.s * sizeof(uint32_t));
  return ok();
}

hidft_status hidft_plan_get_samples(hidft_plan plan, uint64_t* sample_idx) {
  if (!plan || !sample_idx)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_plan_get_samples: NULL argument");
  std::memcpy(sample_idx, plan->core.samples.data(), plan->core.k * sizeof(uint64_t));
  return ok();
}

hidft_status hidft_plan_get_schedule(hidft_plan plan, uint32_t* freq_pos, uint64_t* tw_num,
                                     uint8_t* tw_log2den) {
  if (!plan) return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_plan_get_schedule: plan is NULL");
  const hidft::PlanCore& c = plan->core;
  if (freq_pos) std::memcpy(freq_pos, c.freq_pos.data(), c.k * sizeof(uint32_t));
  if (tw_num && c.k > 1) std::memcpy(tw_num, c.tw_num.data(), (c.k - 1) * sizeof(uint64_t));
  if (tw_log2den && c.k > 1) std::memcpy(tw_log2den, c.tw_log2den.data(), c.k - 1);
  return ok();
}

hidft_status hidft_plan_get_twiddles(hidft_plan plan, float* twiddles) {
  if (!plan || !twiddles)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_plan_get_twiddles: NULL argument");
  if (plan->host_only)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_plan_get_twiddles: HOST_ONLY plan");
  const hidft::PlanCore& c = plan->core;
  if (c.k < 2) return ok();
  std::vector<float2> dev(c.k - 1);
  hipError_t e = hipMemcpy(dev.data(), plan->d_tw, (c.k - 1) * sizeof(float2),
                           hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hidft_plan_get_twiddles");
  for (uint32_t u = 1; u <= c.s; ++u) {
    const uint64_t off = (1ULL << (u - 1)) - 1;
    for (uint64_t q_lo = 0; q_lo < (1ULL << (u - 1)); ++q_lo) {
      const float2 w = dev[hidft::device_tw_index(c.s, u, hidft::bit_reverse(q_lo, u - 1))];
      twiddles[2 * (off + q_lo)] = w.x;
      twiddles[2 * (off + q_lo) + 1] = w.y;
    }
  }
  return ok();
}

hidft_status hidft_plan_device_bytes(hidft_plan plan, size_t* bytes) {
  if (!plan || !bytes)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_plan_device_bytes: NULL argument");
  *bytes = plan->device_bytes.load(std::memory_order_relaxed);
  return ok();
}

hidft_status hidft_plan_workspace_bytes(hidft_plan plan, uint64_t batch, size_t* bytes) {
  if (!plan || !bytes)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_plan_workspace_bytes: NULL argument");
  *bytes = 0;
  if (plan->core.s <= HIDFT_MAX_LOG2_K_DEVICE || batch == 0) return ok();
  if (batch > (~0ULL >> (plan->core.s + 4)))
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_plan_workspace_bytes: batch too large");
  *bytes = (size_t)(batch << plan->core.s) * sizeof(float2);
  return ok();
}

}  // extern "C"

namespace {

// The workspace of the passes: present, large enough, aligned, and
// overlapping neither the input rows nor the output rows.
hidft_status check_workspace(hidft_plan plan, const void* d_in, int64_t ld_in, const void* d_out,
                             int64_t ld_out, uint64_t batch, const void* d_work,
                             size_t work_bytes, const char* fn) {
  size_t need = 0;
  hidft_status st = hidft_plan_workspace_bytes(plan, batch, &need);
  if (st != HIDFT_OK) return st;
  if (!d_work || work_bytes < need)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "%s: workspace of %zu bytes needed, %zu given", fn,
                need, d_work ? work_bytes : (size_t)0);
  if (reinterpret_cast<uintptr_t>(d_work) & 7u)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "%s: workspace must be 8-byte aligned", fn);
  const uintptr_t w0 = reinterpret_cast<uintptr_t>(d_work), w1 = w0 + need;
  const uint64_t k = plan->core.k;
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(d_in);
  const uintptr_t a1 = a0 + ((batch - 1) * (uint64_t)ld_in + k) * sizeof(float2);
  const uintptr_t b0 = reinterpret_cast<uintptr_t>(d_out);
  const uintptr_t b1 = b0 + ((batch - 1) * (uint64_t)ld_out + k) * sizeof(float2);
  if ((w0 < a1 && a0 < w1) || (w0 < b1 && b0 < w1))
    return fail(HIDFT_ERR_INVALID_ARGUMENT,
                "%s: the workspace overlaps the input or output rows", fn);
  return HIDFT_OK;
}

}  // namespace

extern "C" {

hidft_status hidft_execute_ws(hidft_plan plan, const void* d_samples, int64_t ld_in,
                              void* d_coefs, int64_t ld_out, uint64_t batch, void* d_work,
                              size_t work_bytes, void* stream) {
  const char* fn = "hidft_execute_ws";
  hidft_status st = check_exec(plan, d_samples, ld_in, d_coefs, ld_out, batch, fn);
  if (st != HIDFT_OK || batch == 0) return st == HIDFT_OK ? ok() : st;
  if (plan->core.s <= HIDFT_MAX_LOG2_K_DEVICE) return hidft_execute(plan, d_samples, ld_in,
                                                                    d_coefs, ld_out, batch,
                                                                    stream);
  if ((st = check_workspace(plan, d_samples, ld_in, d_coefs, ld_out, batch, d_work, work_bytes,
                            fn)) != HIDFT_OK)
    return st;
  hipError_t e = hidft::launch_large(plan->core.s, static_cast<const float2*>(d_samples), ld_in,
                                     static_cast<float2*>(d_coefs), ld_out, batch,
                                     static_cast<float2*>(d_work), plan->d_tw, plan->d_src,
                                     plan->d_pos, plan->d_src + plan->core.k, plan->scale,
                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hidft_execute_ws: kernel launch");
  return ok();
}

hidft_status hidft_execute(hidft_plan plan, const void* d_samples, int64_t ld_in,
                           void* d_coefs, int64_t ld_out, uint64_t batch, void* stream) {
  hidft_status st = check_exec(plan, d_samples, ld_in, d_coefs, ld_out, batch, "hidft_execute");
  if (st != HIDFT_OK || batch == 0) return st == HIDFT_OK ? ok() : st;
  if (plan->core.s > HIDFT_MAX_LOG2_K_DEVICE) {
    // The passes' workspace, from the stream-ordered allocator: taken and
    // returned on `stream`, around the launches.
    size_t need = 0;
    if ((st = hidft_plan_workspace_bytes(plan, batch, &need)) != HIDFT_OK) return st;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    void* work = nullptr;
    hipError_t e = hipMallocAsync(&work, need, hs);
    if (e != hipSuccess) return hip_fail(e, "hidft_execute: workspace allocation");
    e = hidft::launch_large(plan->core.s, static_cast<const float2*>(d_samples), ld_in,
                            static_cast<float2*>(d_coefs), ld_out, batch,
                            static_cast<float2*>(work), plan->d_tw, plan->d_src, plan->d_pos,
                            plan->d_src + plan->core.k, plan->scale, hs);
    const hipError_t ef = hipFreeAsync(work, hs);
    if (e != hipSuccess) return hip_fail(e, "hidft_execute: kernel launch");
    if (ef != hipSuccess) return hip_fail(ef, "hidft_execute: workspace release");
    return ok();
  }
  hipError_t e = hidft::launch_fused(plan->core.s, static_cast<const float2*>(d_samples), ld_in,
                                     static_cast<float2*>(d_coefs), ld_out, batch, plan->d_tw,
                                     plan->d_src, nullptr, plan->scale, hidft::ExecConfig{},
                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hidft_execute: kernel launch");
  return ok();
}


hidft_status hidft_execute_config(hidft_plan plan, const hidft_exec_config* config,
                                  const void* d_samples, int64_t ld_in, void* d_coefs,
                                  int64_t ld_out, uint64_t batch, void* stream) {
  const char* fn = "hidft_execute_config";
  if (!config) return fail(HIDFT_ERR_INVALID_ARGUMENT, "%s: config is NULL", fn);
  hidft_status st = check_exec(plan, d_samples, ld_in, d_coefs, ld_out, batch, fn);
  if (st != HIDFT_OK) return st;
  hidft_exec_config eff = *config;
  if (eff.schedule == HIDFT_SCHED_TUNED) {
    hidft_exec_config tuned;
    if (hidft::tune_lookup(plan, eff.precision, batch, &tuned))
      eff = tuned;
    else
      eff.schedule = HIDFT_SCHED_DEFAULT;
  }
  hidft::ExecConfig c;
  if ((st = hidft::resolve_config(plan, &eff, &c, fn)) != HIDFT_OK) return st;
  if (batch == 0) return ok();
  void* amat = nullptr;
  if (c.prec != hidft::PREC_FP32 &&
      (st = hidft::plan_amat(plan, static_cast<hipStream_t>(stream), &amat, fn)) != HIDFT_OK)
    return st;
  hipError_t e = hidft::launch_fused(plan->core.s, static_cast<const float2*>(d_samples), ld_in,
                                     static_cast<float2*>(d_coefs), ld_out, batch, plan->d_tw,
                                     plan->d_src, amat, plan->scale, c,
                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hidft_execute_config: kernel launch");
  return ok();
}

hidft_status hidft_execute_inverse(hidft_plan plan, const void* d_coefs, int64_t ld_in,
                                   void* d_samples, int64_t ld_out, uint64_t batch,
                                   void* stream) {
  hidft_status st =
      check_exec(plan, d_coefs, ld_in, d_samples, ld_out, batch, "hidft_execute_inverse");
  if (st != HIDFT_OK || batch == 0) return st == HIDFT_OK ? ok() : st;
  const float inv_n = std::ldexp(1.0f, -(int)plan->core.M);
  if (plan->core.s > HIDFT_MAX_LOG2_K_DEVICE) {
    size_t need = 0;
    if ((st = hidft_plan_workspace_bytes(plan, batch, &need)) != HIDFT_OK) return st;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    void* work = nullptr;
    hipError_t e = hipMallocAsync(&work, need, hs);
    if (e != hipSuccess) return hip_fail(e, "hidft_execute_inverse: workspace allocation");
    e = hidft::launch_large_inverse(plan->core.s, static_cast<const float2*>(d_coefs), ld_in,
                                    static_cast<float2*>(d_samples), ld_out, batch,
                                    static_cast<float2*>(work), plan->d_tw, plan->d_src,
                                    plan->d_pos, plan->d_src + plan->core.k, inv_n, hs);
    const hipError_t ef = hipFreeAsync(work, hs);
    if (e != hipSuccess) return hip_fail(e, "hidft_execute_inverse: kernel launch");
    if (ef != hipSuccess) return hip_fail(ef, "hidft_execute_inverse: workspace release");
    return ok();
  }
  hipError_t e = hidft::launch_inverse(plan->core.s, static_cast<const float2*>(d_coefs), ld_in,
                                       static_cast<float2*>(d_samples), ld_out, batch, plan->d_tw,
                                       plan->d_src, inv_n, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hidft_execute_inverse: kernel launch");
  return ok();
}

hidft_status hidft_execute_inverse_ws(hidft_plan plan, const void* d_coefs, int64_t ld_in,
                                      void* d_samples, int64_t ld_out, uint64_t batch,
                                      void* d_work, size_t work_bytes, void* stream) {
  const char* fn = "hidft_execute_inverse_ws";
  hidft_status st = check_exec(plan, d_coefs, ld_in, d_samples, ld_out, batch, fn);
  if (st != HIDFT_OK || batch == 0) return st == HIDFT_OK ? ok() : st;
  if (plan->core.s <= HIDFT_MAX_LOG2_K_DEVICE)
    return hidft_execute_inverse(plan, d_coefs, ld_in, d_samples, ld_out, batch, stream);
  if ((st = check_workspace(plan, d_coefs, ld_in, d_samples, ld_out, batch, d_work, work_bytes,
                            fn)) != HIDFT_OK)
    return st;
  hipError_t e = hidft::launch_large_inverse(
      plan->core.s, static_cast<const float2*>(d_coefs), ld_in, static_cast<float2*>(d_samples),
      ld_out, batch, static_cast<float2*>(d_work), plan->d_tw, plan->d_src, plan->d_pos,
      plan->d_src + plan->core.k, std::ldexp(1.0f, -(int)plan->core.M),
      static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hidft_execute_inverse_ws: kernel launch");
  return ok();
}

hidft_status hidft_execute_plain(hidft_plan plan, const void* d_samples, int64_t ld_in,
                                 void* d_coefs, int64_t ld_out, uint64_t batch, void* stream) {
  hidft_status st =
      check_exec(plan, d_samples, ld_in, d_coefs, ld_out, batch, "hidft_execute_plain");
  if (st == HIDFT_OK) st = hidft::require_single_pass(plan, "hidft_execute_plain");
  if (st != HIDFT_OK || batch == 0) return st == HIDFT_OK ? ok() : st;
  const float2* in = static_cast<const float2*>(d_samples);
  float2* out = static_cast<float2*>(d_coefs);
  for (uint64_t b = 0; b < batch; ++b) {
    hipError_t e = hidft::launch_plain(plan->core.s, in + b * (uint64_t)ld_in,
                                       out + b * (uint64_t)ld_out, plan->d_tw, plan->d_src,
                                       plan->scale, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hidft_execute_plain: kernel launch");
  }
  return ok();
}

hidft_status hidft_group_create(const hidft_work* items, uint64_t n_items, void* stream,
                                hidft_group* out) {
  if (!out) return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_group_create: out is NULL");
  *out = nullptr;
  if (!items || n_items == 0)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_group_create: no work items");
  hidft_group g = nullptr;
  try {
    // Validate every item and count instances.
    uint64_t n_inst = 0;
    int device = -1;
    for (uint64_t i = 0; i < n_items; ++i) {
      const hidft_work& w = items[i];
      char fn[64];
      std::snprintf(fn, sizeof fn, "hidft_group_create: item %llu", (unsigned long long)i);
      hidft_status st = check_exec(w.plan, w.d_samples, w.ld_in, w.d_coefs, w.ld_out, w.batch, fn);
      if (st == HIDFT_OK) st = hidft::require_single_pass(w.plan, fn);
      if (st != HIDFT_OK) return st;
      if (w.batch == 0) continue;
      device = w.plan->device;
      n_inst += w.batch;
    }
    if (n_inst == 0) return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_group_create: no rows");
    if (n_inst > (1ULL << 31))
      return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_group_create: more than 2^31 instances");
    std::vector<std::pair<uint32_t, hidft::GroupSlot>> inst;
    inst.reserve(n_inst);
    for (uint64_t i = 0; i < n_items; ++i) {
      const hidft_work& w = items[i];
      const hidft_plan p = w.plan;
      for (uint64_t b = 0; b < w.batch; ++b) {
        hidft::GroupSlot d;
        d.in = static_cast<const float2*>(w.d_samples) + b * (uint64_t)w.ld_in;
        d.out = static_cast<float2*>(w.d_coefs) + b * (uint64_t)w.ld_out;
        d.tw = p->d_tw;
        d.src = p->d_src;
        d.scale = p->scale;
        inst.emplace_back(p->core.s, d);
      }
    }
    uint32_t max_grid = 0;
    hipError_t ge = hidft::grouped_grid(&max_grid);
    if (ge != hipSuccess) return hip_fail(ge, "hidft_group_create: grid");
    hidft::GroupSchedule sch;
    hidft::pack_instances(inst, max_grid, false, false, &sch);
    g = new hidft_group_s;
    g->device = device;
    g->n_instances = n_inst;
    g->n_packs = (uint32_t)sch.packs.size();
    g->n_wide = sch.n_wide;
    g->grid = sch.grid;
    g->inst = std::move(inst);
    const size_t pack_bytes = sch.packs.size() * sizeof(hidft::GroupPack);
    const size_t slot_bytes = sch.slots.size() * sizeof(hidft::GroupSlot);
    const size_t lane_bytes = sch.lane_end.size() * sizeof(uint32_t);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = hipMalloc(&g->d_packs, pack_bytes)) != hipSuccess ||
        (e = hipMalloc(&g->d_slots, slot_bytes)) != hipSuccess ||
        (e = hipMalloc(&g->d_lanes, lane_bytes)) != hipSuccess ||
        (e = hipMemcpyAsync(g->d_packs, sch.packs.data(), pack_bytes, hipMemcpyHostToDevice,
                            st)) != hipSuccess ||
        (e = hipMemcpyAsync(g->d_slots, sch.slots.data(), slot_bytes, hipMemcpyHostToDevice,
                            st)) != hipSuccess ||
        (e = hipMemcpyAsync(g->d_lanes, sch.lane_end.data(), lane_bytes, hipMemcpyHostToDevice,
                            st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
      hidft_status r = hip_fail(e, "hidft_group_create: descriptor upload");
      hidft_group_destroy(g);
      return r;
    }
    g->device_bytes = pack_bytes + slot_bytes + lane_bytes;
    *out = g;
    return ok();
  } catch (const std::bad_alloc&) {
    if (g) hidft_group_destroy(g);
    return fail(HIDFT_ERR_OUT_OF_MEMORY, "hidft_group_create: host allocation failed");
  } catch (...) {
    if (g) hidft_group_destroy(g);
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_group_create: unexpected exception");
  }
}

hidft_status hidft_group_execute(hidft_group g, void* stream) {
  if (!g) return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_group_execute: group is NULL");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hidft_group_execute");
  if (dev != g->device)
    return fail(HIDFT_ERR_INVALID_ARGUMENT,
                "hidft_group_execute: current device %d, group lives on device %d", dev,
                g->device);
  e = hidft::launch_grouped(g->d_packs, g->n_wide, g->n_packs - g->n_wide, g->d_slots,
                            g->d_lanes, g->grid, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hidft_group_execute: kernel launch");
  return ok();
}

hidft_status hidft_group_set_config(hidft_group g, const hidft_group_config* cfg,
                                    void* stream) {
  if (!g || !cfg) return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_group_set_config: NULL argument");
  if (cfg->schedule > HIDFT_SCHED_SHORT_LAST)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_group_set_config: unknown schedule %u",
                cfg->schedule);
  if (cfg->order > HIDFT_GROUP_ORDER_ALTERNATE)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_group_set_config: unknown order %u", cfg->order);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hidft_group_set_config");
  if (dev != g->device)
    return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_group_set_config: group lives on device %d",
                g->device);
  uint32_t max_grid = 0;
  if ((e = hidft::grouped_grid(&max_grid)) != hipSuccess)
    return hip_fail(e, "hidft_group_set_config: grid");
  try {
    hidft::GroupSchedule sch;
    hidft::pack_instances(g->inst, max_grid, cfg->schedule == HIDFT_SCHED_SHORT_FIRST,
                          cfg->order == HIDFT_GROUP_ORDER_ALTERNATE, &sch);
    // The same packs and slots as at creation, in another order or with the
    // schedule flag: the device arrays keep their sizes.
    if (sch.packs.size() != g->n_packs || sch.n_wide != g->n_wide || sch.grid != g->grid)
      return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_group_set_config: the grid changed");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((e = hipMemcpyAsync(g->d_packs, sch.packs.data(),
                            sch.packs.size() * sizeof(hidft::GroupPack), hipMemcpyHostToDevice,
                            st)) != hipSuccess ||
        (e = hipMemcpyAsync(g->d_slots, sch.slots.data(),
                            sch.slots.size() * sizeof(hidft::GroupSlot), hipMemcpyHostToDevice,
                            st)) != hipSuccess ||
        (e = hipMemcpyAsync(g->d_lanes, sch.lane_end.data(),
                            sch.lane_end.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                            st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return hip_fail(e, "hidft_group_set_config: descriptor upload");
  } catch (const std::bad_alloc&) {
    return fail(HIDFT_ERR_OUT_OF_MEMORY, "hidft_group_set_config: host allocation failed");
  }
  g->cfg = *cfg;
  return ok();
}

hidft_status hidft_group_get_config(hidft_group g, hidft_group_config* cfg) {
  if (!g || !cfg) return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_group_get_config: NULL argument");
  *cfg = g->cfg;
  return ok();
}

hidft_status hidft_group_autotune(hidft_group g, uint32_t reps, void* stream,
                                  hidft_group_config* best, double* best_us) {
  if (!g || !best) return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_group_autotune: NULL argument");
  if (reps == 0) return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_group_autotune: reps must be positive");
  const hidft_group_config cands[] = {
      {HIDFT_SCHED_SHORT_LAST, HIDFT_GROUP_ORDER_LARGEST_FIRST},
      {HIDFT_SCHED_SHORT_FIRST, HIDFT_GROUP_ORDER_LARGEST_FIRST},
      {HIDFT_SCHED_SHORT_LAST, HIDFT_GROUP_ORDER_ALTERNATE},
      {HIDFT_SCHED_SHORT_FIRST, HIDFT_GROUP_ORDER_ALTERNATE}};
  constexpr int NC = (int)(sizeof cands / sizeof cands[0]);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(e, "hidft_group_autotune: hipEventCreate");
  }
  double us[NC];
  for (double& x : us) x = 1e300;
  hidft_status rs = HIDFT_OK;
  // Two interleaved rounds; each candidate keeps its better one.
  for (int round = 0; round < 2 && rs == HIDFT_OK; ++round) {
    for (int i = 0; i < NC && rs == HIDFT_OK; ++i) {
      if ((rs = hidft_group_set_config(g, &cands[i], stream)) != HIDFT_OK) break;
      for (int w = 0; w < 2 && rs == HIDFT_OK; ++w) rs = hidft_group_execute(g, stream);
      if (rs != HIDFT_OK) break;
      float ms = 0.f;
      if ((e = hipEventRecord(e0, st)) != hipSuccess) {
        rs = hip_fail(e, "hidft_group_autotune: hipEventRecord");
        break;
      }
      for (uint32_t r = 0; r < reps && rs == HIDFT_OK; ++r) rs = hidft_group_execute(g, stream);
      if (rs != HIDFT_OK) break;
      if ((e = hipEventRecord(e1, st)) != hipSuccess ||
          (e = hipEventSynchronize(e1)) != hipSuccess ||
          (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
        rs = hip_fail(e, "hidft_group_autotune: timing");
        break;
      }
      us[i] = std::min(us[i], 1e3 * (double)ms / reps);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rs != HIDFT_OK) return rs;
  int ib = 0;
  for (int i = 1; i < NC; ++i)
    if (us[i] < us[ib]) ib = i;
  if ((rs = hidft_group_set_config(g, &cands[ib], stream)) != HIDFT_OK) return rs;
  *best = cands[ib];
  if (best_us) *best_us = us[ib];
  return ok();
}

hidft_status hidft_group_destroy(hidft_group g) {
  if (!g) return ok();
  if (g->d_packs) (void)hipFree(g->d_packs);
  if (g->d_slots) (void)hipFree(g->d_slots);
  if (g->d_lanes) (void)hipFree(g->d_lanes);
  delete g;
  return ok();
}

hidft_status hidft_group_get_info(hidft_group g, uint64_t* n_instances, uint64_t* n_packs,
                                  size_t* device_bytes) {
  if (!g) return fail(HIDFT_ERR_INVALID_ARGUMENT, "hidft_group_get_info: group is NULL");
  if (n_instances) *n_instances = g->n_instances;
  if (n_packs) *n_packs = g->n_packs;
  if (device_bytes) *device_bytes = g->device_bytes;
  return ok();
}

}  // extern "C"
