// Shift-and-Sample plans (Sec. IX, Algorithm 2) and the Hi-DFT of
// part-homogeneous supports (Sec. VII-B): C ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hidft.h"
#include "internal.h"

struct hidft_sas_s {
  hidft::PartPlan core;
  int device = -1;
  float scale = 1.0f;              // N / 2^s
  float2* d_tw = nullptr;          // 2^s - 1 twiddles, a-order
  uint16_t* d_src = nullptr;       // slot order: src[t] = bitrev_s(t) (induced weights)
  uint16_t* d_src_node = nullptr;  // node order: bitrev_s(slot of node v), padded to 2^s
  uint16_t* d_src_elem = nullptr;  // mu* = 1: caller order, bitrev_s(slot of J[t]'s node)
  uint32_t* d_node_first = nullptr;
  uint32_t* d_node_count = nullptr;
  uint32_t* d_elem_t = nullptr;
  uint32_t* d_elem_node = nullptr;  // node of each element, elements in node order
  uint32_t* d_inv_off = nullptr;    // offset of each node's inverse (complex128 units)
  void* d_inv = nullptr;            // inverse dual Vandermonde matrices, FP64
  uint4* d_elem_rec = nullptr;      // per element: {v | t << 16, row offset, mu(v), 0}
  // 2^s > 2^HIDFT_MAX_LOG2_K_DEVICE (mu* = 1): the passes of launch_large.
  // d_src holds their 16-bit tables, d_pos the 32-bit ones, d_tw the split
  // twiddle layout.
  uint32_t* d_pos = nullptr;
  bool large = false;
  bool fused = false;               // one kernel per launch, no workspace
  bool weights_only = false;        // HIDFT_SAS_WEIGHTS_ONLY: no leaf-solve tables
  size_t device_bytes = 0;
};

namespace {

void release(hidft_sas p) {
  void* ptrs[] = {p->d_tw,         p->d_src,      p->d_src_node,  p->d_src_elem, p->d_node_first,
                  p->d_node_count, p->d_elem_t,   p->d_elem_node, p->d_inv_off,  p->d_inv,
                  p->d_elem_rec,   p->d_pos};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  p->d_tw = nullptr;
  p->d_src = p->d_src_node = p->d_src_elem = nullptr;
  p->d_node_first = p->d_node_count = p->d_elem_t = p->d_elem_node = p->d_inv_off = nullptr;
  p->d_inv = nullptr;
  p->d_elem_rec = nullptr;
  p->d_pos = nullptr;
}

template <typename T>
hipError_t upload_vec(T** dst, const std::vector<T>& v, hipStream_t st, size_t* total) {
  const size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
  hipError_t e = hipMalloc(dst, bytes);
  if (e != hipSuccess) return e;
  *total += bytes;
  if (v.empty()) return hipSuccess;
  return hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

hidft_status upload(hidft_sas p, hipStream_t st) {
  const hidft::PartPlan& c = p->core;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) return hidft::hip_error(e, "hidft_sas_create");
  const uint64_t ks = 1ULL << c.s;
  const uint64_t ntw = ks - 1;
  std::vector<uint64_t> num(ntw ? ntw : 1, 0);
  std::vector<uint8_t> den(ntw ? ntw : 1, 0);
  for (uint32_t u = 1; u <= c.s; ++u) {
    const uint64_t off = (1ULL << (u - 1)) - 1;
    for (uint64_t q_lo = 0; q_lo < (1ULL << (u - 1)); ++q_lo) {
      const uint64_t h = hidft::bit_reverse(q_lo, u - 1);
      num[off + h] = c.tw_num[off + q_lo];
      den[off + h] = c.tw_log2den[off + q_lo];
    }
  }
  const uint32_t n_nodes = (uint32_t)c.node_slot.size();
  if (p->large) {
    // One element per node: the Hi-DFT's value at the slot of J[t]'s node is
    // the answer for t, through the passes of launch_large.
    std::vector<uint32_t> pos(c.k);
    for (uint32_t v = 0; v < n_nodes; ++v)
      pos[c.elem_t[c.node_first[v]]] = (uint32_t)hidft::bit_reverse(c.node_slot[v], c.s);
    std::vector<uint16_t> src16;
    std::vector<uint32_t> src32;
    hidft::large_tables(c.s, pos, &src16, &src32);
    for (uint32_t u = 1; u <= c.s; ++u) {
      const uint64_t off = (1ULL << (u - 1)) - 1;
      for (uint64_t q_lo = 0; q_lo < (1ULL << (u - 1)); ++q_lo) {
        const uint64_t at = hidft::device_tw_index(c.s, u, hidft::bit_reverse(q_lo, u - 1));
        num[at] = c.tw_num[off + q_lo];
        den[at] = c.tw_log2den[off + q_lo];
      }
    }
    uint64_t* d_num = nullptr;
    uint8_t* d_den = nullptr;
    size_t total = 0, tmp = 0;
    hidft_status status = HIDFT_OK;
    if ((e = hipMalloc(&p->d_tw, (ntw ? ntw : 1) * sizeof(float2))) != hipSuccess ||
        (e = upload_vec(&d_num, num, st, &tmp)) != hipSuccess ||
        (e = upload_vec(&d_den, den, st, &tmp)) != hipSuccess ||
        (e = upload_vec(&p->d_src, src16, st, &total)) != hipSuccess ||
        (e = upload_vec(&p->d_pos, src32, st, &total)) != hipSuccess ||
        (e = hidft::launch_twiddle_gen(d_num, d_den, p->d_tw, ntw, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      status = hidft::hip_error(e, "hidft_sas_create: table upload");
    if (d_num) (void)hipFree(d_num);
    if (d_den) (void)hipFree(d_den);
    if (status != HIDFT_OK) {
      release(p);
      return status;
    }
    p->device_bytes = total + (ntw ? ntw : 1) * sizeof(float2);
    return HIDFT_OK;
  }
  std::vector<uint16_t> src(ks), src_node(ks, 0), src_elem;
  for (uint64_t t = 0; t < ks; ++t) src[t] = (uint16_t)hidft::bit_reverse(t, c.s);
  if (p->weights_only) {
    // The Hi-DFT alone: twiddles and the slot-order gather table.
    uint64_t* d_num = nullptr;
    uint8_t* d_den = nullptr;
    size_t total = 0, tmp = 0;
    hidft_status status = HIDFT_OK;
    if ((e = hipMalloc(&p->d_tw, (ntw ? ntw : 1) * sizeof(float2))) != hipSuccess ||
        (e = upload_vec(&d_num, num, st, &tmp)) != hipSuccess ||
        (e = upload_vec(&d_den, den, st, &tmp)) != hipSuccess ||
        (e = upload_vec(&p->d_src, src, st, &total)) != hipSuccess ||
        (e = hidft::launch_twiddle_gen(d_num, d_den, p->d_tw, ntw, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      status = hidft::hip_error(e, "hidft_sas_create: table upload");
    if (d_num) (void)hipFree(d_num);
    if (d_den) (void)hipFree(d_den);
    if (status != HIDFT_OK) {
      release(p);
      return status;
    }
    p->device_bytes = total + (ntw ? ntw : 1) * sizeof(float2);
    return HIDFT_OK;
  }
  for (uint32_t v = 0; v < n_nodes; ++v)
    src_node[v] = (uint16_t)hidft::bit_reverse(c.node_slot[v], c.s);
  std::vector<uint64_t> elem_val(c.k);
  std::vector<uint32_t> elem_node(c.k), inv_off(n_nodes);
  uint64_t inv_entries = 0;
  for (uint32_t v = 0; v < n_nodes; ++v) {
    inv_off[v] = (uint32_t)inv_entries;
    inv_entries += (uint64_t)c.node_count[v] * c.node_count[v];
    for (uint32_t i = 0; i < c.node_count[v]; ++i) {
      elem_node[c.node_first[v] + i] = v;
      elem_val[c.node_first[v] + i] = c.J[c.elem_t[c.node_first[v] + i]];
    }
  }
  // Element records of the one-block-per-signal solve (node and caller
  // position fit in 16 bits there: both are below SAS_LDS_VALUES).
  std::vector<uint4> elem_rec;
  if (c.mu_max > 1 && (p->fused || (uint64_t)c.mu_max * n_nodes + c.k <= hidft::SAS_LDS_VALUES)) {
    elem_rec.resize(c.k);
    for (uint32_t v = 0; v < n_nodes; ++v) {
      const uint32_t mu = c.node_count[v];
      for (uint32_t i = 0; i < mu; ++i) {
        const uint32_t e = c.node_first[v] + i;
        elem_rec[e] = make_uint4(v | (c.elem_t[e] << 16), inv_off[v] + i * mu, mu, 0u);
      }
    }
  }
  if (c.mu_max == 1) {  // one element per node: the Hi-DFT output is the answer
    src_elem.assign(ks, 0);
    for (uint32_t v = 0; v < n_nodes; ++v) src_elem[c.elem_t[c.node_first[v]]] = src_node[v];
  }
  uint64_t* d_num = nullptr;
  uint8_t* d_den = nullptr;
  uint64_t* d_elem_val = nullptr;
  size_t total = 0, tmp = 0;
  const size_t inv_bytes = (size_t)(inv_entries + hidft::SAS_INV_PAD) * 16;
  hidft_status status = HIDFT_OK;
  if ((e = hipMalloc(&p->d_tw, (ntw ? ntw : 1) * sizeof(float2))) != hipSuccess ||
      (e = hipMalloc(&p->d_inv, inv_bytes)) != hipSuccess ||
      (e = hipMemsetAsync(static_cast<char*>(p->d_inv) + inv_entries * 16, 0,
                          hidft::SAS_INV_PAD * 16, st)) != hipSuccess ||
      (e = upload_vec(&d_num, num, st, &tmp)) != hipSuccess ||
      (e = upload_vec(&d_den, den, st, &tmp)) != hipSuccess ||
      (e = upload_vec(&d_elem_val, elem_val, st, &tmp)) != hipSuccess ||
      (e = upload_vec(&p->d_src, src, st, &total)) != hipSuccess ||
      (e = upload_vec(&p->d_src_node, src_node, st, &total)) != hipSuccess ||
      (!src_elem.empty() && (e = upload_vec(&p->d_src_elem, src_elem, st, &total)) != hipSuccess) ||
      (e = upload_vec(&p->d_node_first, c.node_first, st, &total)) != hipSuccess ||
      (e = upload_vec(&p->d_node_count, c.node_count, st, &total)) != hipSuccess ||
      (e = upload_vec(&p->d_elem_t, c.elem_t, st, &total)) != hipSuccess ||
      (e = upload_vec(&p->d_elem_node, elem_node, st, &total)) != hipSuccess ||
      (e = upload_vec(&p->d_inv_off, inv_off, st, &total)) != hipSuccess ||
      (!elem_rec.empty() && (e = upload_vec(&p->d_elem_rec, elem_rec, st, &total)) != hipSuccess) ||
      (e = hidft::launch_twiddle_gen(d_num, d_den, p->d_tw, ntw, st)) != hipSuccess ||
      (e = hidft::launch_sas_inverse(n_nodes, p->d_node_first, p->d_node_count, p->d_inv_off,
                                     d_elem_val, c.M, p->d_inv, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    status = hidft::hip_error(e, "hidft_sas_create: table upload");
  }
  total += inv_bytes;
  if (d_num) (void)hipFree(d_num);
  if (d_den) (void)hipFree(d_den);
  if (d_elem_val) (void)hipFree(d_elem_val);
  if (status != HIDFT_OK) {
    release(p);
    return status;
  }
  p->device_bytes = total + (ntw ? ntw : 1) * sizeof(float2);
  return HIDFT_OK;
}

hidft_status check_rows(hidft_sas p, const void* in, int64_t ld_in, uint64_t in_len,
                        const void* out, int64_t ld_out, uint64_t out_len, uint64_t batch,
                        const char* fn) {
  if (!p) return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, std::string(fn) + ": plan is NULL");
  if (batch == 0) return HIDFT_OK;
  if (!in || !out)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, std::string(fn) + ": NULL buffer");
  if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 7u)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT,
                            std::string(fn) + ": buffers must be 8-byte aligned");
  if (ld_in < 0 || ld_out < 0 || (uint64_t)ld_in < in_len || (uint64_t)ld_out < out_len)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT,
                            std::string(fn) + ": leading dimension smaller than a row");
  if (batch > (1ULL << 31))
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, std::string(fn) + ": batch too large");
  const uint64_t a0 = reinterpret_cast<uintptr_t>(in);
  const uint64_t a1 = a0 + ((batch - 1) * (uint64_t)ld_in + in_len) * 8;
  const uint64_t b0 = reinterpret_cast<uintptr_t>(out);
  const uint64_t b1 = b0 + ((batch - 1) * (uint64_t)ld_out + out_len) * 8;
  if (a0 < b1 && b0 < a1)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT,
                            std::string(fn) + ": input and output overlap");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hidft::hip_error(e, fn);
  if (dev != p->device)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT,
                            std::string(fn) + ": current device differs from the plan's");
  return HIDFT_OK;
}

}  // namespace

extern "C" {

hidft_status hidft_sas_create(uint32_t log2_n, const uint64_t* J, uint64_t k,
                              const uint32_t* pivots, uint32_t n_pivots, uint32_t flags,
                              void* stream, hidft_sas* out) {
  if (!out) return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_sas_create: out is NULL");
  *out = nullptr;
  if (flags & ~(HIDFT_PLAN_HOST_ONLY | HIDFT_SAS_TWO_PASS | HIDFT_SAS_WEIGHTS_ONLY))
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_sas_create: unknown flags");
  hidft_sas p = nullptr;
  try {
    p = new hidft_sas_s;
    std::string err;
    hidft_status st = hidft::build_part_plan(log2_n, J, k, pivots, n_pivots,
                                             HIDFT_MAX_LOG2_K_DEVICE, HIDFT_MAX_LOG2_K_LARGE,
                                             HIDFT_SAS_MAX_MU, HIDFT_SAS_MAX_REL_ERR, &p->core,
                                             &err);
    if (st != HIDFT_OK) {
      delete p;
      return hidft::set_error(st, "hidft_sas_create: " + err);
    }
    p->weights_only = (flags & HIDFT_SAS_WEIGHTS_ONLY) != 0;
    p->large = p->core.s > HIDFT_MAX_LOG2_K_DEVICE;  // then mu* = 1 (build_part_plan)
    if (p->large && p->weights_only) {
      delete p;
      return hidft::set_error(HIDFT_ERR_UNSUPPORTED,
                              "hidft_sas_create: the induced weights need 2^s <= 2^" +
                                  std::to_string(HIDFT_MAX_LOG2_K_DEVICE));
    }
    if (!p->weights_only) {
      // A plan that will solve must be solvable within the accuracy target.
      const hidft::LeafAccuracy& a = p->core.leaf;
      char buf[320];
      buf[0] = 0;
      if (p->core.mu_max > HIDFT_SAS_MAX_MU)
        std::snprintf(buf, sizeof buf,
                      "mu* = %u exceeds the leaf solver's %u (HIDFT_SAS_WEIGHTS_ONLY plans "
                      "compute the Hi-DFT alone)", p->core.mu_max, HIDFT_SAS_MAX_MU);
      else if (!(a.rel_err_bound <= HIDFT_SAS_MAX_REL_ERR))
        std::snprintf(buf, sizeof buf,
                      "the leaf systems at r are ill-conditioned: condition number %.3e, "
                      "error amplification %.3e, relative error bound %.3e > %.1e",
                      a.cond, a.amplification, a.rel_err_bound, HIDFT_SAS_MAX_REL_ERR);
      if (buf[0]) {
        delete p;
        return hidft::set_error(HIDFT_ERR_UNSUPPORTED, std::string("hidft_sas_create: ") + buf);
      }
    }
    p->scale = std::ldexp(1.0f, (int)p->core.M - (int)p->core.s);
    p->fused = !p->weights_only && !p->large && !(flags & HIDFT_SAS_TWO_PASS) &&
               hidft::sas_fused_fits(p->core.s, p->core.mu_max,
                                     (uint32_t)p->core.node_slot.size(), (uint32_t)p->core.k);
    if (!(flags & HIDFT_PLAN_HOST_ONLY)) {
      st = upload(p, static_cast<hipStream_t>(stream));
      if (st != HIDFT_OK) {
        delete p;
        return st;
      }
    }
    *out = p;
    return hidft::set_error(HIDFT_OK, "");
  } catch (const std::bad_alloc&) {
    if (p) {
      release(p);
      delete p;
    }
    return hidft::set_error(HIDFT_ERR_OUT_OF_MEMORY, "hidft_sas_create: host allocation failed");
  }
}

hidft_status hidft_sas_destroy(hidft_sas p) {
  if (!p) return hidft::set_error(HIDFT_OK, "");
  release(p);
  delete p;
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_sas_get_info(hidft_sas p, uint32_t* n_pivots, uint32_t* mu_max,
                                uint64_t* n_nodes, uint64_t* samples_per_signal, double* cost) {
  if (!p) return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_sas_get_info: plan is NULL");
  if (n_pivots) *n_pivots = p->core.s;
  if (mu_max) *mu_max = p->core.mu_max;
  if (n_nodes) *n_nodes = p->core.node_slot.size();
  if (samples_per_signal) *samples_per_signal = (uint64_t)p->core.mu_max << p->core.s;
  if (cost) *cost = p->core.cost;
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_sas_get_accuracy(hidft_sas p, double* cond, double* amplification,
                                    double* rel_err_bound) {
  if (!p)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_sas_get_accuracy: plan is NULL");
  if (cond) *cond = p->core.leaf.cond;
  if (amplification) *amplification = p->core.leaf.amplification;
  if (rel_err_bound) *rel_err_bound = p->core.leaf.rel_err_bound;
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_sas_get_pivots(hidft_sas p, uint32_t* pivots) {
  if (!p || !pivots)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_sas_get_pivots: NULL argument");
  std::memcpy(pivots, p->core.pivots.data(), p->core.s * sizeof(uint32_t));
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_sas_get_samples(hidft_sas p, uint64_t* idx) {
  if (!p || !idx)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_sas_get_samples: NULL argument");
  const uint64_t ks = 1ULL << p->core.s;
  const uint64_t mask = p->core.M >= 64 ? ~0ULL : ((1ULL << p->core.M) - 1);
  for (uint32_t j = 0; j < p->core.mu_max; ++j)
    for (uint64_t a = 0; a < ks; ++a) idx[j * ks + a] = (p->core.samples[a] + j) & mask;
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_sas_get_nodes(hidft_sas p, uint32_t* node_of_t, uint32_t* slot_of_node) {
  if (!p) return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_sas_get_nodes: plan is NULL");
  const hidft::PartPlan& c = p->core;
  if (node_of_t)
    for (size_t v = 0; v < c.node_slot.size(); ++v)
      for (uint32_t i = 0; i < c.node_count[v]; ++i) node_of_t[c.elem_t[c.node_first[v] + i]] = (uint32_t)v;
  if (slot_of_node) std::memcpy(slot_of_node, c.node_slot.data(), c.node_slot.size() * 4);
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_sas_workspace_bytes(hidft_sas p, uint64_t batch, size_t* bytes) {
  if (!p || !bytes)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_sas_workspace_bytes: NULL");
  // [signal][shift][node]; none when every node holds one element (mu* = 1)
  // or when the plan runs as one kernel.  Above 2^HIDFT_MAX_LOG2_K_DEVICE
  // samples per Hi-DFT: the passes' intermediate, 2^s values per signal.
  if (p->large)
    *bytes = (size_t)(batch << p->core.s) * sizeof(float2);
  else
    *bytes = p->core.mu_max == 1 || p->fused || p->weights_only
                 ? 0
                 : (size_t)batch * p->core.mu_max * p->core.node_slot.size() * sizeof(float2);
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_sas_weights(hidft_sas p, const void* d_samples, int64_t ld_in, void* d_weights,
                               int64_t ld_out, uint64_t batch, void* stream) {
  const uint64_t ks = p ? (1ULL << p->core.s) : 0;
  hidft_status st = check_rows(p, d_samples, ld_in, ks, d_weights, ld_out, ks, batch,
                               "hidft_sas_weights");
  if (st != HIDFT_OK || batch == 0) return st == HIDFT_OK ? hidft::set_error(HIDFT_OK, "") : st;
  if (!p->d_tw)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_sas_weights: HOST_ONLY plan");
  if (p->large)
    return hidft::set_error(HIDFT_ERR_UNSUPPORTED,
                            "hidft_sas_weights: the induced weights need 2^s <= 2^" +
                                std::to_string(HIDFT_MAX_LOG2_K_DEVICE));
  hipError_t e = hidft::launch_fused(p->core.s, static_cast<const float2*>(d_samples), ld_in,
                                     static_cast<float2*>(d_weights), ld_out, batch, p->d_tw,
                                     p->d_src, nullptr, p->scale, hidft::ExecConfig{},
                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hidft::hip_error(e, "hidft_sas_weights: kernel launch");
  return hidft::set_error(HIDFT_OK, "");
}

}  // extern "C"

namespace {

// Validation shared by the execute entry points (HIDFT_OK with batch == 0
// means there is nothing to do).
hidft_status check_execute(hidft_sas p, const void* d_samples, int64_t ld_in, void* d_coefs,
                           int64_t ld_out, uint64_t batch, const char* fn) {
  const uint64_t ks = p ? (1ULL << p->core.s) : 0;
  const uint64_t mu = p ? p->core.mu_max : 0;
  if (p && mu > HIDFT_SAS_MAX_MU)
    return hidft::set_error(HIDFT_ERR_UNSUPPORTED,
                            std::string(fn) + ": mu* = " + std::to_string(mu) +
                                " exceeds the leaf solver's " + std::to_string(HIDFT_SAS_MAX_MU));
  hidft_status st = check_rows(p, d_samples, ld_in, mu * ks, d_coefs, ld_out, p ? p->core.k : 0,
                               batch, fn);
  if (st != HIDFT_OK || batch == 0) return st;
  if (!p->d_tw)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, std::string(fn) + ": HOST_ONLY plan");
  if (p->weights_only)
    return hidft::set_error(HIDFT_ERR_UNSUPPORTED,
                            std::string(fn) + ": the plan was created for the induced weights only");
  return HIDFT_OK;
}

// The paths that need no workspace: mu* = 1 (the Hi-DFT gathered into the
// caller's order of J is the answer) and the one-kernel form.
hidft_status run_direct(hidft_sas p, const float2* in, int64_t ld_in, float2* coefs,
                        int64_t ld_out, uint64_t batch, hipStream_t s, const char* fn) {
  const uint64_t mu = p->core.mu_max;
  hipError_t e;
  if (mu == 1) {
    e = hidft::launch_fused(p->core.s, in, ld_in, coefs, ld_out, batch, p->d_tw, p->d_src_elem,
                            nullptr, p->scale, hidft::ExecConfig{}, s, (uint32_t)p->core.k);
  } else {
    // Shifted Hi-DFTs and leaf solves in one kernel, node values in LDS.
    e = hidft::launch_sas_fused(p->core.s, in, ld_in, coefs, ld_out, batch, (uint32_t)mu,
                                (uint32_t)p->core.node_slot.size(), (uint32_t)p->core.k, p->d_tw,
                                p->d_src_node, p->scale, p->d_elem_rec, p->d_inv, s);
  }
  if (e != hipSuccess) return hidft::hip_error(e, fn);
  return hidft::set_error(HIDFT_OK, "");
}

// The two-launch form through a workspace of batch mu* n_nodes values.
hipError_t run_two_pass(hidft_sas p, const float2* in, int64_t ld_in, float2* coefs,
                        int64_t ld_out, uint64_t batch, float2* work, hipStream_t s) {
  const uint64_t ks = 1ULL << p->core.s;
  const uint64_t mu = p->core.mu_max;
  const uint64_t nn = p->core.node_slot.size();
  hipError_t e = hipSuccess;
  // Steps 2-4: the mu* shifted Hi-DFTs, each gathered in node order (the
  // first nn outputs), as one batched launch when the rows are packed, else
  // one launch per shift.
  if ((uint64_t)ld_in == mu * ks) {
    e = hidft::launch_fused(p->core.s, in, (int64_t)ks, work, (int64_t)nn, batch * mu, p->d_tw,
                            p->d_src_node, nullptr, p->scale, hidft::ExecConfig{}, s,
                            (uint32_t)nn);
  } else {
    for (uint64_t j = 0; j < mu && e == hipSuccess; ++j)
      e = hidft::launch_fused(p->core.s, in + j * ks, ld_in, work + j * nn, (int64_t)(mu * nn),
                              batch, p->d_tw, p->d_src_node, nullptr, p->scale,
                              hidft::ExecConfig{}, s, (uint32_t)nn);
  }
  // Steps 5-7: every node's solve, one row of its inverse per element.
  if (e == hipSuccess)
    e = hidft::launch_sas_apply(work, (uint32_t)nn, (uint32_t)mu, batch, (uint32_t)p->core.k,
                                p->d_elem_node, p->d_node_first, p->d_node_count, p->d_inv_off,
                                p->d_inv, p->d_elem_t, p->d_elem_rec, coefs, ld_out, s);
  return e;
}

// 2^s > 2^HIDFT_MAX_LOG2_K_DEVICE with mu* = 1: the Hi-DFT in passes through
// a workspace of 2^s values per signal, its k kept outputs in J's order.
hipError_t run_large(hidft_sas p, const float2* in, int64_t ld_in, float2* coefs,
                     int64_t ld_out, uint64_t batch, float2* work, hipStream_t s) {
  const uint64_t ks = 1ULL << p->core.s;
  return hidft::launch_large(p->core.s, in, ld_in, coefs, ld_out, batch, work, p->d_tw, p->d_src,
                             p->d_pos, p->d_src + ks, p->scale, s, p->core.k);
}

}  // namespace

extern "C" {

hidft_status hidft_sas_execute(hidft_sas p, const void* d_samples, int64_t ld_in, void* d_coefs,
                               int64_t ld_out, uint64_t batch, void* d_work, void* stream) {
  const char* fn = "hidft_sas_execute";
  hidft_status st = check_execute(p, d_samples, ld_in, d_coefs, ld_out, batch, fn);
  if (st != HIDFT_OK || batch == 0) return st == HIDFT_OK ? hidft::set_error(HIDFT_OK, "") : st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const float2* in = static_cast<const float2*>(d_samples);
  float2* coefs = static_cast<float2*>(d_coefs);
  if (!p->large && (p->core.mu_max == 1 || p->fused))
    return run_direct(p, in, ld_in, coefs, ld_out, batch, s, fn);
  const uint64_t ks = 1ULL << p->core.s;
  const uint64_t mu = p->core.mu_max;
  if (!d_work || (reinterpret_cast<uintptr_t>(d_work) & 7u))
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT,
                            "hidft_sas_execute: workspace missing or misaligned");
  {
    // The workspace is written while the samples are read and read while the
    // coefficients are written: it must overlap neither.
    size_t wbytes = 0;
    (void)hidft_sas_workspace_bytes(p, batch, &wbytes);
    const uint64_t w0 = reinterpret_cast<uintptr_t>(d_work);
    const uint64_t w1 = w0 + wbytes;
    const uint64_t a0 = reinterpret_cast<uintptr_t>(d_samples);
    const uint64_t a1 = a0 + ((batch - 1) * (uint64_t)ld_in + mu * ks) * sizeof(float2);
    const uint64_t b0 = reinterpret_cast<uintptr_t>(d_coefs);
    const uint64_t b1 = b0 + ((batch - 1) * (uint64_t)ld_out + p->core.k) * sizeof(float2);
    if ((w0 < a1 && a0 < w1) || (w0 < b1 && b0 < w1))
      return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT,
                              "hidft_sas_execute: workspace overlaps the samples or coefficients");
  }
  hipError_t e = p->large ? run_large(p, in, ld_in, coefs, ld_out, batch,
                                      static_cast<float2*>(d_work), s)
                          : run_two_pass(p, in, ld_in, coefs, ld_out, batch,
                                         static_cast<float2*>(d_work), s);
  if (e != hipSuccess) return hidft::hip_error(e, "hidft_sas_execute: kernel launch");
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_sas_execute_noalloc(hidft_sas p, const void* d_samples, int64_t ld_in,
                                       void* d_coefs, int64_t ld_out, uint64_t batch,
                                       void* stream) {
  const char* fn = "hidft_sas_execute_noalloc";
  hidft_status st = check_execute(p, d_samples, ld_in, d_coefs, ld_out, batch, fn);
  if (st != HIDFT_OK || batch == 0) return st == HIDFT_OK ? hidft::set_error(HIDFT_OK, "") : st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const float2* in = static_cast<const float2*>(d_samples);
  float2* coefs = static_cast<float2*>(d_coefs);
  if (!p->large && (p->core.mu_max == 1 || p->fused))
    return run_direct(p, in, ld_in, coefs, ld_out, batch, s, fn);
  // One signal's intermediate values (the shifted Hi-DFT outputs, or the
  // passes' 2^s values) must fit the scratch; the batch runs in chunks of as
  // many signals as fit, in stream order.
  const uint64_t per_signal =
      p->large ? (uint64_t)sizeof(float2) << p->core.s
               : (uint64_t)p->core.mu_max * p->core.node_slot.size() * sizeof(float2);
  if (per_signal > hidft::SAS_SCRATCH_BYTES)
    return hidft::set_error(HIDFT_ERR_UNSUPPORTED,
                            std::string(fn) + ": one signal needs " + std::to_string(per_signal) +
                                " bytes of scratch, more than the " +
                                std::to_string(hidft::SAS_SCRATCH_BYTES) + " available");
  void* scratch = nullptr;
  hipError_t e = hidft::sas_scratch(&scratch);
  if (e != hipSuccess) return hidft::hip_error(e, "hidft_sas_execute_noalloc: scratch lookup");
  const uint64_t chunk = hidft::SAS_SCRATCH_BYTES / per_signal;
  for (uint64_t first = 0; first < batch && e == hipSuccess; first += chunk) {
    const uint64_t n = batch - first < chunk ? batch - first : chunk;
    e = p->large ? run_large(p, in + first * (uint64_t)ld_in, ld_in,
                             coefs + first * (uint64_t)ld_out, ld_out, n,
                             static_cast<float2*>(scratch), s)
                 : run_two_pass(p, in + first * (uint64_t)ld_in, ld_in,
                                coefs + first * (uint64_t)ld_out, ld_out, n,
                                static_cast<float2*>(scratch), s);
  }
  if (e != hipSuccess) return hidft::hip_error(e, "hidft_sas_execute_noalloc: kernel launch");
  return hidft::set_error(HIDFT_OK, "");
}

}  // extern "C"
