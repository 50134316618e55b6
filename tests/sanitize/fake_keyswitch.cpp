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

// batch layout [2][level][batch][N]; request b's input [2][level][N]
hipError_t hmult_ptrs(const tfhe_ckks_ctx_s* c, const CtPtrs& a, const CtPtrs& b, uint32_t* out,
                      const uint32_t* evk, uint32_t level, uint32_t batch, unsigned char*, hipStream_t) {
  pause();
  if (batch > 1) ++fake_batched_calls;
  const size_t n = c->n;
  for (uint32_t r = 0; r < 2 * level; ++r)
    for (uint32_t k = 0; k < batch; ++k)
      for (size_t i = 0; i < n; ++i)
        out[((size_t)r * batch + k) * n + i] = a.p[k][r * n + i] + 2 * b.p[k][r * n + i] + evk[0];
  return hipSuccess;
}

hipError_t rotate_ptrs(const tfhe_ckks_ctx_s* c, const CtPtrs& in, uint32_t* out, const KeySet& keys,
                       const GaloisSet& gs, uint32_t level, uint32_t batch, unsigned char*, hipStream_t) {
  pause();
  if (batch > 1) ++fake_batched_calls;
  const size_t n = c->n;
  for (uint32_t r = 0; r < 2 * level; ++r)
    for (uint32_t k = 0; k < batch; ++k) {
      const uint32_t key0 = keys.k[keys.count == 1 ? 0 : k][0];
      for (size_t i = 0; i < n; ++i)
        out[((size_t)r * batch + k) * n + i] = 3 * in.p[k][r * n + i] + gs.g[k % gs.batch] + key0;
    }
  return hipSuccess;
}

}  // namespace tfhe
