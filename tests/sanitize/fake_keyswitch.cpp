// Stand-in for the CKKS operations the request dispatcher calls, for the
// ThreadSanitizer build of the dispatcher: instead of a key switch each
// writes an easily checked function of its inputs (host memory, the HIP
// stand-in runtime), so a driver can verify that every request got the
// result of its own inputs, key and Galois element.
//   HMULT:   out = a + 2 b + key[0]          (element-wise, mod 2^32)
//   HROTATE: out = 3 a + galois + key[0]
// Test infrastructure only.
#include <atomic>
#include <chrono>
#include <thread>

#include "../../paper_2212_14191_amd/csrc/ckks_internal.hpp"

using namespace tfhe;

// batched calls seen (B > 1), read by the driver; each call also takes a
// little time, as a launch would, so that requests queue up into batches
std::atomic<int> fake_batched_calls{0};
std::atomic<int> fake_mixed_calls{0};     // batches holding more than one level
std::atomic<int> fake_mixed_op_calls{0};  // batches holding HMULTs and rotations
static void pause() { std::this_thread::sleep_for(std::chrono::microseconds(50)); }

extern "C" tfhe_status tfhe_hmult_workspace_size(tfhe_ckks_ctx ctx, uint32_t level, uint32_t batch, size_t* bytes) {
  if (!ctx || !bytes || level < 1 || level > ctx->L) return TFHE_EINVAL;
  *bytes = (size_t)2 * level * batch * ctx->n * 4 + 256;
  return TFHE_OK;
}

extern "C" tfhe_status tfhe_hmult(tfhe_ckks_ctx ctx, const uint32_t* a, const uint32_t* b, uint32_t* out,
                                  const uint32_t* evk, uint32_t level, uint32_t batch, void*, size_t,
                                  tfhe_stream_t) {
  pause();
  const size_t n = (size_t)2 * level * batch * ctx->n;
  for (size_t i = 0; i < n; ++i) out[i] = a[i] + 2 * b[i] + evk[0];
  return TFHE_OK;
}

extern "C" tfhe_status tfhe_rotate(tfhe_ckks_ctx ctx, const uint32_t* in, uint32_t* out, const uint32_t* rk,
                                   uint32_t galois, uint32_t level, uint32_t batch, void*, size_t,
                                   tfhe_stream_t) {
  pause();
  const size_t n = (size_t)2 * level * batch * ctx->n;
  for (size_t i = 0; i < n; ++i) out[i] = 3 * in[i] + galois + rk[0];
  return TFHE_OK;
}

namespace tfhe {

size_t levels_ws_bytes(const tfhe_ckks_ctx_s* c, const LvReq* r, uint32_t count) {
  size_t b = 256;
  for (uint32_t k = 0; k < count; ++k) b += (size_t)2 * r[k].level * c->n * 4;
  return b;
}

// each request's result written straight to its own buffer
hipError_t levels_run(const tfhe_ckks_ctx_s* c, const LvReq* r, uint32_t count, unsigned char*, hipStream_t) {
  pause();
  if (count > 1) ++fake_batched_calls;
  for (uint32_t k = 1; k < count; ++k)
    if (r[k].level != r[0].level) {
      ++fake_mixed_calls;
      break;
    }
  for (uint32_t k = 1; k < count; ++k)
    if (r[k].op != r[0].op) {
      ++fake_mixed_op_calls;
      break;
    }
  for (uint32_t k = 0; k < count; ++k) {
    const size_t n = (size_t)2 * r[k].level * c->n;
    for (size_t i = 0; i < n; ++i)
      r[k].out[i] = r[k].op == 0 ? r[k].a[i] + 2 * r[k].b[i] + r[k].key[0] : 3 * r[k].a[i] + r[k].galois + r[k].key[0];
  }
  return hipSuccess;
}

}  // namespace tfhe
