// Host-side table construction and argument handling of the C ABI under
// ASan / UBSan (built against the HIP stand-in runtime): NTT plans at every
// supported N, CKKS contexts of several shapes (including fewer special
// primes than a digit has limbs), workspace queries, plan parameters, and
// the refusal paths.  Exit status 0 when every call behaved as expected.
#include <cstdio>
#include <vector>

#include "tfhe.h"

static int failures = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

int main() {
  for (uint32_t log_n = 4; log_n <= 16; ++log_n) {
    std::vector<uint32_t> q(3);
    EXPECT(tfhe_find_primes(31, 2ull << log_n, 3, q.data()) == TFHE_OK);
    tfhe_ntt_plan p = nullptr;
    EXPECT(tfhe_ntt_plan_create(&p, log_n, 3, q.data(), nullptr, TFHE_NTT_AUTO) == TFHE_OK);
    uint32_t ln = 0, nl = 0;
    tfhe_ntt_algo a;
    EXPECT(tfhe_ntt_plan_info(p, &ln, &nl, &a) == TFHE_OK && ln == log_n && nl == 3);
    for (int param = 1; param <= 6; ++param) {
      int64_t v = -1;
      EXPECT(tfhe_ntt_plan_get_param(p, (tfhe_plan_param)param, &v) == TFHE_OK);
    }
    EXPECT(tfhe_ntt_plan_set_param(p, TFHE_PARAM_FS_PASSES, 1) == TFHE_OK);
    EXPECT(tfhe_ntt_plan_set_param(p, TFHE_PARAM_FS_PASSES, 3) == TFHE_EINVAL);
    EXPECT(tfhe_ntt_plan_set_param(p, TFHE_PARAM_FS_RING, 2) == TFHE_OK);
    EXPECT(tfhe_ntt_plan_set_param(p, TFHE_PARAM_FS_RING, 1) == TFHE_EINVAL);
    EXPECT(tfhe_ntt_plan_set_param(p, TFHE_PARAM_FS_RING, 4) == TFHE_EINVAL);
    int64_t ring = 0;
    EXPECT(tfhe_ntt_plan_get_param(p, TFHE_PARAM_FS_RING, &ring) == TFHE_OK && ring == 2);
    size_t ws = 0;
    EXPECT(tfhe_ntt_workspace_size(p, TFHE_NTT_BUTTERFLY, 3, 5, &ws) == TFHE_OK);
    uint32_t qq = 0, psi = 0;
    EXPECT(tfhe_ntt_plan_modulus(p, 2, &qq, &psi) == TFHE_OK && qq == q[2]);
    EXPECT(tfhe_ntt_plan_modulus(p, 3, &qq, &psi) == TFHE_EINVAL);
    EXPECT(tfhe_ntt_plan_destroy(p) == TFHE_OK);
  }
  // refusals
  tfhe_ntt_plan p = nullptr;
  std::vector<uint32_t> q3(3);
  EXPECT(tfhe_find_primes(31, 1ull << 17, 3, q3.data()) == TFHE_OK);
  EXPECT(tfhe_ntt_plan_create(&p, 3, 3, q3.data(), nullptr, TFHE_NTT_AUTO) == TFHE_EINVAL && p == nullptr);
  EXPECT(tfhe_ntt_plan_create(&p, 17, 3, q3.data(), nullptr, TFHE_NTT_AUTO) == TFHE_EINVAL && p == nullptr);
  uint32_t bad[2] = {1000003u, 7u};
  EXPECT(tfhe_ntt_plan_create(&p, 10, 2, bad, nullptr, TFHE_NTT_AUTO) != TFHE_OK && p == nullptr);
  EXPECT(tfhe_ntt_plan_create(nullptr, 10, 2, bad, nullptr, TFHE_NTT_AUTO) == TFHE_EINVAL);

  struct Shape { uint32_t log_n, L, K, dnum; } shapes[] = {
      {10, 6, 2, 3}, {12, 8, 4, 2}, {13, 24, 8, 3}, {16, 24, 8, 3}, {10, 8, 1, 1}, {5, 6, 2, 3}, {10, 12, 2, 12}};
  for (const Shape& s : shapes) {
    tfhe_ckks_ctx c = nullptr;
    EXPECT(tfhe_ckks_ctx_create(&c, s.log_n, s.L, s.K, s.dnum, nullptr, nullptr, TFHE_NTT_AUTO) == TFHE_OK);
    if (!c) continue;
    for (uint32_t level = 1; level <= s.L; ++level)
      for (uint32_t batch : {1u, 3u, 64u}) {
        size_t b = 0;
        EXPECT(tfhe_hmult_workspace_size(c, level, batch, &b) == TFHE_OK && b > 0);
        if (level >= 2) EXPECT(tfhe_rescale_workspace_size(c, level, batch, &b) == TFHE_OK);
      }
    size_t b = 0;
    EXPECT(tfhe_hmult_workspace_size(c, s.L + 1, 1, &b) == TFHE_EINVAL);
    tfhe_ntt_plan cp = nullptr;
    EXPECT(tfhe_ckks_ctx_plan(c, &cp) == TFHE_OK && cp != nullptr);
    EXPECT(tfhe_ckks_ctx_destroy(c) == TFHE_OK);
  }
  tfhe_ckks_ctx c = nullptr;
  EXPECT(tfhe_ckks_ctx_create(&c, 10, 24, 8, 5, nullptr, nullptr, TFHE_NTT_AUTO) == TFHE_EINVAL);
  EXPECT(tfhe_ckks_ctx_create(&c, 10, 24, 8, 2, nullptr, nullptr, TFHE_NTT_AUTO) == TFHE_EUNSUPPORTED);
  std::printf("tables driver: %d failures\n", failures);
  return failures != 0;
}
