// Per-kernel timing: when enabled, every launcher brackets its kernel with a
// pair of HIP events recorded on the launch stream; tfhe_timing_read resolves
// them.  Off by default (no events are recorded).
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace tfhe {

namespace {
struct Rec {
  int id;
  hipEvent_t a, b;
};
std::mutex g_mu;
std::atomic<bool> g_on{false};  // read without the lock by every launcher
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

const char* kNames[] = {"ntt_mfma_pass1", "ntt_mfma_pass2", "ntt_bf_single", "ntt_bf_cols",
                        "ntt_bf_rows",    "elementwise",    "ckks_tensor",   "ckks_modup",
                        "ckks_inner",     "ckks_moddown_conv", "ckks_moddown_final", "frobenius",
                        "ckks_rescale_bcast", "ckks_rescale_final",
                        "ntt_co_pass1",       "ntt_co_pass2",       "ntt_mfma_onepass",
                        "ntt_mfma_pass2_inner"};
constexpr int kNumNames = sizeof(kNames) / sizeof(kNames[0]);
}  // namespace

bool timing_on() { return g_on; }

void* timing_begin(int id, hipStream_t s) {
  if (!g_on) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  Rec r{id, take(), take()};
  if (!r.a || !r.b) {  // event creation failed: this launch goes untimed
    if (r.a) g_pool.push_back(r.a);
    if (r.b) g_pool.push_back(r.b);
    return nullptr;
  }
  (void)hipEventRecord(r.a, s);
  g_recs.push_back(r);
  return &g_recs.back() - &g_recs[0] + (char*)1;  // index + 1 as an opaque token
}

void timing_end(void* token, hipStream_t s) {
  if (!token) return;
  std::lock_guard<std::mutex> lk(g_mu);
  size_t idx = (size_t)((char*)token - (char*)1);
  if (idx < g_recs.size()) (void)hipEventRecord(g_recs[idx].b, s);
}

static void clear_locked() {
  for (Rec& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
}

}  // namespace tfhe

using namespace tfhe;

extern "C" {

tfhe_status tfhe_timing_enable(int enable) {
  std::lock_guard<std::mutex> lk(g_mu);
  clear_locked();
  g_on = enable != 0;
  return TFHE_OK;
}

tfhe_status tfhe_timing_read(const char* kernel, uint64_t* launches, double* total_ms) {
  if (!kernel || !launches || !total_ms) return fail(TFHE_EINVAL, "timing_read: null argument");
  int id = -1;
  for (int i = 0; i < kNumNames; ++i)
    if (std::string(kernel) == kNames[i]) id = i;
  if (id < 0) return fail(TFHE_EINVAL, std::string("timing_read: unknown kernel ") + kernel);
  std::lock_guard<std::mutex> lk(g_mu);
  uint64_t n = 0;
  double ms = 0;
  for (Rec& r : g_recs) {
    if (r.id != id) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(TFHE_EHIP, "timing_read: event sync");
    float t = 0;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return fail(TFHE_EHIP, "timing_read: elapsed");
    ms += t;
    ++n;
  }
  *launches = n;
  *total_ms = ms;
  return TFHE_OK;
}

}  // extern "C"
