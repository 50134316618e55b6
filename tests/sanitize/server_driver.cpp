// The request dispatcher (server.cpp) under ThreadSanitizer, with the HIP
// stand-in runtime and stand-in key switching (fake_keyswitch.cpp): four
// submitter threads queue HMULT / HROTATE requests of two ring sizes and
// random levels in groups, a poller thread collects completions, another
// thread changes a batch limit meanwhile; every result must be the one its
// own inputs, key and Galois element give.  Exit status 0 on success.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "../../paper_2212_14191_amd/csrc/ckks_internal.hpp"

extern std::atomic<int> fake_batched_calls;
extern std::atomic<int> fake_mixed_calls;
extern std::atomic<int> fake_mixed_op_calls;

struct Request {
  uint32_t op, log_n, level, galois;
  std::vector<uint32_t> a, b, out;
};

int main() {
  const uint32_t L = 4, per_thread = 120, threads = 4;
  tfhe_ckks_ctx_s ctx6, ctx7;
  for (auto [c, ln] : {std::pair<tfhe_ckks_ctx_s*, uint32_t>{&ctx6, 6u}, {&ctx7, 7u}}) {
    c->log_n = ln;
    c->n = 1u << ln;
    c->L = L;
    c->K = 2;
    c->dnum = 2;
    c->alpha = 2;
  }
  std::vector<uint32_t> evk6(64, 11), evk7(64, 13), rk6a(64, 101), rk6b(64, 103), rk7a(64, 107);
  void* pool = nullptr;
  const size_t pool_bytes = 4 * (size_t)(4 << 20);
  hipMalloc(&pool, pool_bytes);
  tfhe_server s = nullptr;
  if (tfhe_server_create(&s, 4, 8, pool, pool_bytes) != TFHE_OK) return 2;
  tfhe_server_add_context(s, &ctx6, evk6.data());
  tfhe_server_add_context(s, &ctx7, evk7.data());
  tfhe_server_add_rotation_key(s, 6, 5, rk6a.data());
  tfhe_server_add_rotation_key(s, 6, 25, rk6b.data());
  tfhe_server_add_rotation_key(s, 7, 5, rk7a.data());
  tfhe_server_set_max_batch(s, 6, 3);

  std::vector<Request> reqs(threads * per_thread);
  std::mt19937 rng(7);
  for (Request& r : reqs) {
    r.op = rng() % 2;
    r.log_n = 6 + rng() % 2;
    r.level = 1 + rng() % L;
    r.galois = r.op == 1 ? (r.log_n == 6 ? (rng() % 2 ? 5u : 25u) : 5u) : 0u;
    const size_t n = (size_t)2 * r.level << r.log_n;
    r.a.resize(n);
    r.b.resize(n);
    r.out.assign(n, 0);
    for (size_t i = 0; i < n; ++i) {
      r.a[i] = rng();
      r.b[i] = rng();
    }
  }
  std::atomic<uint32_t> completed{0};
  std::vector<int32_t> status(reqs.size(), 1);
  std::atomic<bool> submit_error{false};
  std::vector<std::thread> ts;
  for (uint32_t t = 0; t < threads; ++t)
    ts.emplace_back([&, t] {
      std::mt19937 r2(100 + t);
      uint32_t i = t * per_thread, end = i + per_thread;
      while (i < end) {
        const uint32_t g = std::min<uint32_t>(1 + r2() % 7, end - i);
        std::vector<tfhe_server_request> group(g);
        for (uint32_t k = 0; k < g; ++k) {
          Request& q = reqs[i + k];
          group[k] = tfhe_server_request{q.op, q.log_n, q.level, q.galois, q.a.data(),
                                         q.op == 0 ? q.b.data() : nullptr, q.out.data(), i + k};
        }
        if (tfhe_server_submit_many(s, group.data(), g, nullptr, nullptr) != TFHE_OK) submit_error = true;
        i += g;
      }
    });
  std::thread limiter([&] {
    for (int k = 0; k < 200 && completed.load() < reqs.size(); ++k) tfhe_server_set_max_batch(s, 7, k % 3);
  });
  std::thread poller([&] {
    std::vector<uint64_t> tags(64);
    std::vector<int32_t> st(64);
    while (completed.load() < reqs.size() && !submit_error) {
      const uint32_t k = tfhe_server_poll(s, tags.data(), st.data(), 64);
      for (uint32_t j = 0; j < k; ++j) status[tags[j]] = st[j];
      completed += k;
    }
  });
  for (auto& t : ts) t.join();
  limiter.join();
  poller.join();
  tfhe_server_destroy(s);
  hipFree(pool);
  if (submit_error) {
    std::fprintf(stderr, "a submission failed: %s\n", tfhe_last_error());
    return 1;
  }
  int bad = 0;
  for (size_t q = 0; q < reqs.size(); ++q) {
    const Request& r = reqs[q];
    if (status[q] != 0) ++bad;
    const uint32_t key0 = r.op == 0 ? (r.log_n == 6 ? 11u : 13u)
                                    : (r.log_n == 6 ? (r.galois == 5 ? 101u : 103u) : 107u);
    for (size_t i = 0; i < r.out.size(); ++i) {
      const uint32_t want = r.op == 0 ? r.a[i] + 2 * r.b[i] + key0 : 3 * r.a[i] + r.galois + key0;
      if (r.out[i] != want) {
        ++bad;
        break;
      }
    }
  }
  std::printf("server driver: %zu requests, %d wrong, %d batched calls, %d of mixed levels, %d of mixed operations\n",
              reqs.size(), bad, fake_batched_calls.load(), fake_mixed_calls.load(), fake_mixed_op_calls.load());
  return bad != 0 || fake_batched_calls.load() == 0 || fake_mixed_calls.load() == 0 ||
         fake_mixed_op_calls.load() == 0;
}
