// Workspace audit of the CKKS operations, on the host under AddressSanitizer:
// every buffer (workspace, ciphertexts, keys) is allocated at exactly the
// size the C ABI asks for, and the kernel stand-ins (kernel_stubs.cpp) touch
// the first and the last word of every range the real launches read or
// write.  An undersized workspace region, a slice laid out past the end of
// its buffer or a wrong extent of an input or output is therefore reported
// by the sanitizer.  Covers HMULT, HROTATE (one and several Galois
// elements), RESCALE, the allocation-free HMULT and the mixed-level batches
// (one operation, and HMULTs with rotations),
// for four-step and butterfly contexts (fewer special primes than a digit
// has limbs included) and both inner-product paths.  Exit status 0 when
// every call succeeded.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "tfhe.h"
#include "../../paper_2212_14191_amd/csrc/ckks_internal.hpp"

static int failures = 0;
#define EXPECT(cond)                                                                            \
  do {                                                                                          \
    if (!(cond)) {                                                                              \
      std::fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond);        \
      ++failures;                                                                               \
    }                                                                                           \
  } while (0)

// "device" memory of exactly `bytes` (a multiple of 256 here), 256-aligned
struct Buf {
  void* p = nullptr;
  explicit Buf(size_t bytes) { p = std::aligned_alloc(256, bytes ? bytes : 256); }
  ~Buf() { std::free(p); }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  uint32_t* u() const { return (uint32_t*)p; }
};

int main() {
  struct Shape {
    uint32_t log_n, L, K, dnum;
    tfhe_ntt_algo algo;
  } shapes[] = {{12, 8, 4, 2, TFHE_NTT_FOURSTEP_MFMA}, {12, 24, 8, 3, TFHE_NTT_FOURSTEP_MFMA},
                {12, 8, 1, 1, TFHE_NTT_FOURSTEP_MFMA}, {12, 12, 2, 6, TFHE_NTT_FOURSTEP_MFMA},
                {13, 8, 2, 4, TFHE_NTT_BUTTERFLY},     {10, 8, 1, 1, TFHE_NTT_BUTTERFLY},
                {10, 6, 2, 3, TFHE_NTT_AUTO}};
  int calls = 0;
  for (const Shape& s : shapes) {
    tfhe_ckks_ctx c = nullptr;
    EXPECT(tfhe_ckks_ctx_create(&c, s.log_n, s.L, s.K, s.dnum, nullptr, nullptr, s.algo) == TFHE_OK);
    if (!c) continue;
    tfhe_ntt_plan plan = nullptr;
    EXPECT(tfhe_ckks_ctx_plan(c, &plan) == TFHE_OK);
    const size_t n = (size_t)1 << s.log_n, limb = n * 4;
    Buf evk((size_t)s.dnum * 2 * (s.L + s.K) * limb);
    const uint32_t alpha = s.L / s.dnum;
    std::vector<uint32_t> levels;
    for (uint32_t lv : {1u, 2u, alpha, alpha + 1, s.L - 1, s.L})
      if (lv >= 1 && lv <= s.L) levels.push_back(lv);
    for (int ks_inner : {1, 2}) {
      EXPECT(tfhe_ntt_plan_set_param(plan, TFHE_PARAM_KS_INNER, ks_inner) == TFHE_OK);
      for (uint32_t level : levels)
        for (uint32_t batch : {1u, 3u}) {
          const size_t ct = 2 * (size_t)level * batch * limb;
          size_t wsb = 0;
          EXPECT(tfhe_hmult_workspace_size(c, level, batch, &wsb) == TFHE_OK);
          Buf ws(wsb), a(ct), b(ct), out(ct);
          EXPECT(tfhe_hmult(c, a.u(), b.u(), out.u(), evk.u(), level, batch, ws.p, wsb, nullptr) == TFHE_OK);
          EXPECT(tfhe_hmult(c, a.u(), b.u(), out.u(), evk.u(), level, batch, ws.p, wsb - 256, nullptr) ==
                 TFHE_EINVAL);
          EXPECT(tfhe_rotate(c, a.u(), out.u(), evk.u(), 5, level, batch, ws.p, wsb, nullptr) == TFHE_OK);
          std::vector<const uint32_t*> keys(batch, evk.u());
          std::vector<uint32_t> gal(batch);
          for (uint32_t k = 0; k < batch; ++k) gal[k] = 2 * k + 3;
          EXPECT(tfhe_rotate_multi(c, a.u(), out.u(), keys.data(), gal.data(), level, batch, ws.p, wsb, nullptr) ==
                 TFHE_OK);
          if (wsb <= (size_t)TFHE_HMULT_NOALLOC_MAX_BYTES)
            EXPECT(tfhe_hmult_noalloc(c, a.u(), b.u(), out.u(), evk.u(), level, batch, nullptr) == TFHE_OK);
          if (level >= 2) {
            size_t rsb = 0;
            EXPECT(tfhe_rescale_workspace_size(c, level, batch, &rsb) == TFHE_OK);
            Buf rws(rsb), rout(2 * (size_t)(level - 1) * batch * limb);
            EXPECT(tfhe_rescale(c, a.u(), rout.u(), level, batch, rws.p, rsb, nullptr) == TFHE_OK);
          }
          calls += 5;
        }
      // mixed levels: unsorted, repeated, with a single one
      std::vector<uint32_t> mix;
      for (uint32_t lv : {s.L, 1u, (s.L + 1) / 2, (s.L + 1) / 2, alpha + 1, s.L, 2u})
        if (lv >= 1 && lv <= s.L) mix.push_back(lv);
      size_t wsb = 0;
      EXPECT(tfhe_hmult_levels_workspace_size(c, mix.data(), (uint32_t)mix.size(), &wsb) == TFHE_OK);
      Buf ws(wsb);
      std::vector<Buf*> bufs;
      std::vector<const uint32_t*> ins_a, ins_b, keys;
      std::vector<uint32_t*> outs;
      std::vector<uint32_t> gal;
      for (size_t i = 0; i < mix.size(); ++i) {
        const size_t ct = 2 * (size_t)mix[i] * limb;
        for (int k = 0; k < 3; ++k) bufs.push_back(new Buf(ct));
        ins_a.push_back(bufs[bufs.size() - 3]->u());
        ins_b.push_back(bufs[bufs.size() - 2]->u());
        outs.push_back(bufs[bufs.size() - 1]->u());
        keys.push_back(evk.u());
        gal.push_back(i % 2 ? 5u : 25u);
      }
      EXPECT(tfhe_hmult_levels(c, ins_a.data(), ins_b.data(), outs.data(), mix.data(), (uint32_t)mix.size(), evk.u(),
                               ws.p, wsb, nullptr) == TFHE_OK);
      EXPECT(tfhe_hmult_levels(c, ins_a.data(), ins_b.data(), outs.data(), mix.data(), (uint32_t)mix.size(), evk.u(),
                               ws.p, wsb - 256, nullptr) == TFHE_EINVAL);
      EXPECT(tfhe_rotate_levels(c, ins_a.data(), outs.data(), keys.data(), gal.data(), mix.data(),
                                (uint32_t)mix.size(), ws.p, wsb, nullptr) == TFHE_OK);
      // a result written over an input (allowed)
      EXPECT(tfhe_hmult_levels(c, ins_a.data(), ins_b.data(), (uint32_t* const*)ins_a.data(), mix.data(),
                               (uint32_t)mix.size(), evk.u(), ws.p, wsb, nullptr) == TFHE_OK);
      // HMULTs and rotations in one batch (as the request dispatcher runs
      // them), in a workspace of exactly the size it asks for
      std::vector<tfhe::LvReq> both;
      for (size_t i = 0; i < mix.size(); ++i)
        both.push_back(tfhe::LvReq{ins_a[i], i % 2 ? nullptr : ins_b[i], outs[i], keys[i], mix[i],
                                   i % 2 ? gal[i] : 0u, (uint32_t)(i % 2)});
      Buf ws2(tfhe::levels_ws_bytes(c, both.data(), (uint32_t)both.size()));
      EXPECT(tfhe::levels_run(c, both.data(), (uint32_t)both.size(), (unsigned char*)ws2.p, nullptr) == hipSuccess);
      calls += 4;
      for (Buf* p : bufs) delete p;
    }
    EXPECT(tfhe_ckks_ctx_destroy(c) == TFHE_OK);
  }
  std::printf("workspace audit: %d calls, %d failures\n", calls, failures);
  return failures != 0;
}
