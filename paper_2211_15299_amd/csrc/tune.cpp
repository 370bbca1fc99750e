// Autotuner of the fused transform: measures the execution variants of a plan
// on the caller's buffers and keeps the fastest per (device, size, precision,
// batch class) in a process-wide table that can be saved and loaded as text.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "hidft.h"
#include "internal.h"

namespace {

// Table key: device architecture name and CU count, s = log2 k, precision,
// batch class = floor(log2 batch).
using TuneKey = std::tuple<std::string, uint32_t, uint32_t, uint32_t>;

struct TuneEntry {
  hidft_exec_config cfg;
  double us;  // mean launch time when measured
};

std::mutex g_mu;
std::map<TuneKey, TuneEntry> g_table;

uint32_t batch_class(uint64_t batch) {
  uint32_t c = 0;
  while (batch > 1) {
    batch >>= 1;
    ++c;
  }
  return c;
}

// "<gcnArchName>/<CUs>" of a device, e.g. "gfx950:sramecc+:xnack-/256";
// queried once per device.
hidft_status device_tag(int device, std::string* tag) {
  static std::mutex mu;
  static std::map<int, std::string> tags;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = tags.find(device);
    if (it != tags.end()) {
      *tag = it->second;
      return HIDFT_OK;
    }
  }
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hidft::hip_error(e, "hipGetDeviceProperties");
  std::string arch(prop.gcnArchName);
  for (char& ch : arch)
    if (ch == ' ' || ch == '\t') ch = '_';
  *tag = arch + "/" + std::to_string(prop.multiProcessorCount);
  std::lock_guard<std::mutex> lock(mu);
  tags[device] = *tag;
  return HIDFT_OK;
}

// Candidate variants for size s and a precision.
std::vector<hidft_exec_config> candidates(uint32_t s, uint32_t precision) {
  std::vector<hidft_exec_config> out;
  std::vector<uint32_t> scheds;
  if (precision == HIDFT_PREC_FP32) {
    scheds.push_back(HIDFT_SCHED_SHORT_FIRST);
    if (s > 4 && s % 4 != 0) scheds.push_back(HIDFT_SCHED_SHORT_LAST);
  } else {
    scheds.push_back(HIDFT_SCHED_DEFAULT);
  }
  std::vector<uint32_t> radices = {16};
  if (s >= 13) radices.push_back(32);
  // Persistent sizes: the grid is resident blocks per CU times the CUs.
  std::vector<uint32_t> bpcs = {0};
  if (s <= 12) bpcs = {0, 1, 2, 3};
  for (uint32_t sc : scheds)
    for (uint32_t r : radices)
      for (uint32_t b : bpcs) out.push_back(hidft_exec_config{precision, sc, r, b});
  return out;
}

}  // namespace

namespace hidft {

bool tune_lookup(const hidft_plan plan, uint32_t precision, uint64_t batch,
                 hidft_exec_config* cfg) {
  std::string tag;
  if (device_tag(plan->device, &tag) != HIDFT_OK) return false;
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_table.find(TuneKey{tag, plan->core.s, precision, batch_class(batch)});
  if (it == g_table.end()) return false;
  *cfg = it->second.cfg;
  return true;
}

}  // namespace hidft

extern "C" {

hidft_status hidft_autotune(hidft_plan plan, uint32_t precision, const void* d_samples,
                            int64_t ld_in, void* d_coefs, int64_t ld_out, uint64_t batch,
                            uint32_t reps, void* stream, hidft_exec_config* best,
                            double* best_us) {
  const char* fn = "hidft_autotune";
  if (!plan || !best) return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_autotune: NULL");
  if (plan->host_only)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_autotune: HOST_ONLY plan");
  if (batch == 0 || reps == 0)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT,
                            "hidft_autotune: batch and reps must be positive");
  if (d_samples == d_coefs)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT,
                            "hidft_autotune: needs distinct input and output buffers");
  if (precision > HIDFT_PREC_BF16X3)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT,
                            "hidft_autotune: unknown precision " + std::to_string(precision));
  const std::vector<hidft_exec_config> cands = candidates(plan->core.s, precision);
  // Every candidate must be runnable (this also checks the buffers).
  for (const hidft_exec_config& c : cands) {
    hidft::ExecConfig ec;
    hidft_status st = hidft::resolve_config(plan, &c, &ec, fn);
    if (st != HIDFT_OK) return st;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipError_t e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventCreate(&ev1);
  if (e != hipSuccess) {
    if (ev0) (void)hipEventDestroy(ev0);
    return hidft::hip_error(e, "hidft_autotune: hipEventCreate");
  }
  std::vector<double> mean_us(cands.size(), 1e300);
  hidft_status st = HIDFT_OK;
  // Two interleaved rounds over the candidates; a candidate keeps its better
  // round, which damps drift of the device's clocks during the search.
  for (int round = 0; round < 2 && st == HIDFT_OK; ++round) {
    for (size_t i = 0; i < cands.size() && st == HIDFT_OK; ++i) {
      for (int w = 0; w < 2 && st == HIDFT_OK; ++w)
        st = hidft_execute_config(plan, &cands[i], d_samples, ld_in, d_coefs, ld_out, batch,
                                  stream);
      if (st != HIDFT_OK) break;
      if ((e = hipEventRecord(ev0, s)) != hipSuccess) {
        st = hidft::hip_error(e, "hidft_autotune: hipEventRecord");
        break;
      }
      for (uint32_t r = 0; r < reps && st == HIDFT_OK; ++r)
        st = hidft_execute_config(plan, &cands[i], d_samples, ld_in, d_coefs, ld_out, batch,
                                  stream);
      if (st != HIDFT_OK) break;
      float ms = 0.f;
      if ((e = hipEventRecord(ev1, s)) != hipSuccess ||
          (e = hipEventSynchronize(ev1)) != hipSuccess ||
          (e = hipEventElapsedTime(&ms, ev0, ev1)) != hipSuccess) {
        st = hidft::hip_error(e, "hidft_autotune: timing");
        break;
      }
      mean_us[i] = std::min(mean_us[i], 1e3 * (double)ms / reps);
    }
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if (st != HIDFT_OK) return st;
  const size_t ib = (size_t)(std::min_element(mean_us.begin(), mean_us.end()) - mean_us.begin());
  *best = cands[ib];
  if (best_us) *best_us = mean_us[ib];
  std::string tag;
  if ((st = device_tag(plan->device, &tag)) != HIDFT_OK) return st;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    g_table[TuneKey{tag, plan->core.s, precision, batch_class(batch)}] =
        TuneEntry{cands[ib], mean_us[ib]};
  }
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_tune_lookup(hidft_plan plan, uint32_t precision, uint64_t batch,
                               hidft_exec_config* config, int* found) {
  if (!plan || !config || !found)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_tune_lookup: NULL argument");
  if (plan->host_only)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_tune_lookup: HOST_ONLY plan");
  *found = hidft::tune_lookup(plan, precision, batch, config) ? 1 : 0;
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_tune_clear(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_table.clear();
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_tune_save(const char* path) {
  if (!path) return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_tune_save: NULL path");
  std::string text = "hidft-tune 1\n";
  {
    std::lock_guard<std::mutex> lock(g_mu);
    char line[512];
    for (const auto& kv : g_table) {
      const TuneKey& k = kv.first;
      const TuneEntry& v = kv.second;
      std::snprintf(line, sizeof line, "%s %u %u %u %u %u %u %.3f\n", std::get<0>(k).c_str(),
                    std::get<1>(k), std::get<2>(k), std::get<3>(k), v.cfg.schedule, v.cfg.radix,
                    v.cfg.blocks_per_cu, v.us);
      text += line;
    }
  }
  std::FILE* f = std::fopen(path, "w");
  if (!f) return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT,
                                  std::string("hidft_tune_save: cannot open ") + path);
  const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
  if (std::fclose(f) != 0 || !ok)
    return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT,
                            std::string("hidft_tune_save: write failed for ") + path);
  return hidft::set_error(HIDFT_OK, "");
}

hidft_status hidft_tune_load(const char* path) {
  if (!path) return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT, "hidft_tune_load: NULL path");
  std::FILE* f = std::fopen(path, "r");
  if (!f) return hidft::set_error(HIDFT_ERR_INVALID_ARGUMENT,
                                  std::string("hidft_tune_load: cannot open ") + path);
  std::map<TuneKey, TuneEntry> loaded;
  char buf[512];
  int lineno = 0;
  hidft_status st = HIDFT_OK;
  std::string msg;
  while (std::fgets(buf, sizeof buf, f)) {
    ++lineno;
    if (lineno == 1) {
      if (std::strncmp(buf, "hidft-tune 1", 12) != 0) {
        st = HIDFT_ERR_INVALID_ARGUMENT;
        msg = "not a tuning table (missing 'hidft-tune 1' header)";
        break;
      }
      continue;
    }
    char tag[256];
    unsigned s = 0, prec = 0, bc = 0, sched = 0, radix = 0, bpc = 0;
    double us = 0;
    const int n = std::sscanf(buf, "%255s %u %u %u %u %u %u %lf", tag, &s, &prec, &bc, &sched,
                              &radix, &bpc, &us);
    if (n == EOF || (n <= 0 && buf[0] == '\n')) continue;
    if (n != 8 || s > HIDFT_MAX_LOG2_K_DEVICE || prec > HIDFT_PREC_BF16X3 || bc > 63 ||
        sched > HIDFT_SCHED_SHORT_LAST || (radix != 0 && radix != 16 && radix != 32) ||
        bpc > 1024) {
      st = HIDFT_ERR_INVALID_ARGUMENT;
      msg = "malformed entry on line " + std::to_string(lineno);
      break;
    }
    loaded[TuneKey{tag, s, prec, bc}] =
        TuneEntry{hidft_exec_config{prec, sched, radix, bpc}, us};
  }
  std::fclose(f);
  if (st != HIDFT_OK) return hidft::set_error(st, std::string("hidft_tune_load: ") + path + ": " + msg);
  {
    std::lock_guard<std::mutex> lock(g_mu);
    for (const auto& kv : loaded) g_table[kv.first] = kv.second;
  }
  return hidft::set_error(HIDFT_OK, "");
}

}  // extern "C"
