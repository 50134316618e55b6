// Native request dispatcher for HMULT / HROTATE serving (the API layer of
// Sec. IV-E: requests are collected, grouped into batched kernel workflows
// and dispatched; keys and ciphertexts stay resident in device memory).
//
// Each of `slots` worker threads owns a HIP stream and an equal share of the
// caller's memory pool.  Pending requests are indexed by batching key (N,
// context): a batch may mix levels and operations (operation-level
// batching, Sec. IV-D: HMULT and HROTATE share every kernel of the key
// switch).  Whenever a worker is free, the oldest request and up to
// max_batch - 1 later ones of its key form a batch whose workspace fits the
// worker's share (otherwise the batch is halved until it fits).  A batch of
// one runs in place on the request's own buffers; a larger one runs as one
// launch sequence (levels_run) that reads its inputs where they are and
// copies each result out to its request.  Rotations by different amounts
// share a batch (one key and Galois element per ciphertext).  Every request
// waits for an event recorded on its submitter's stream at submission.
// Completed tags are collected by tfhe_server_poll.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "ckks_internal.hpp"

namespace tfhe {
namespace {

struct Req {
  uint32_t op, log_n, level, galois;
  const uint32_t *a, *b;
  uint32_t* out;
  uint64_t tag, seq;     // caller's tag; arrival number
  hipEvent_t ready;      // recorded on the submitter's stream
  tfhe_ckks_ctx ctx;     // resolved at submission, so that launches read
  const uint32_t* key;   // no shared map: evk (HMULT) or rotation key
};

struct Key {
  uint32_t log_n;
  tfhe_ckks_ctx ctx;  // requests submitted before a context was replaced batch apart
  bool operator<(const Key& o) const { return std::tie(log_n, ctx) < std::tie(o.log_n, o.ctx); }
};

LvReq lv(const Req& r) { return LvReq{r.a, r.b, r.out, r.key, r.level, r.galois, r.op}; }

struct Slot {
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;
  unsigned char* mem = nullptr;  // this slot's share of the pool
  size_t bytes = 0;
};

struct Ctx {
  tfhe_ckks_ctx ctx = nullptr;
  const uint32_t* evk = nullptr;
  std::map<uint32_t, const uint32_t*> rk;  // Galois element -> rotation key
  uint32_t max_batch = 0;                  // this N's batch limit (0: the server's)
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace tfhe

using namespace tfhe;

struct tfhe_server_s {
  int device = 0;
  uint32_t max_batch = 16;
  std::vector<Slot> slots;
  std::map<uint32_t, Ctx> ctxs;  // log_n -> context
  std::mutex mu;
  std::condition_variable cv;
  std::map<Key, std::deque<Req>> pending;  // per batching key, FIFO
  std::deque<std::pair<uint64_t, Key>> order;  // arrival order (seq, key)
  uint64_t next_seq = 0;
  std::vector<std::pair<uint64_t, int32_t>> done;
  std::vector<hipEvent_t> event_pool;
  std::map<hipEvent_t, uint32_t> ev_refs;  // readiness events in use -> requests holding them
  bool stop = false;
  std::vector<std::thread> workers;

  // slot memory the batch of the B requests from `first` needs: a batch of
  // one runs in place with tfhe_hmult's workspace
  template <typename It>
  static size_t need(It first, uint32_t B) {
    const tfhe_ckks_ctx ctx = first->ctx;
    if (B == 1) {
      size_t ws = 0;
      tfhe_hmult_workspace_size(ctx, first->level, 1, &ws);
      return align256(ws);
    }
    std::vector<LvReq> r;
    for (uint32_t k = 0; k < B; ++k, ++first) r.push_back(lv(*first));
    return align256(levels_ws_bytes(ctx, r.data(), B));
  }
  // a request holding e is done with it (caller holds mu)
  void release_event(hipEvent_t e) {
    auto it = ev_refs.find(e);
    if (it != ev_refs.end() && --it->second == 0) {
      ev_refs.erase(it);
      event_pool.push_back(e);
    }
  }
  tfhe_status check(const tfhe_server_request& q, Req& out);
  bool take(const Slot& sl, std::vector<Req>& reqs);
  void worker(Slot& sl);
  int launch(Slot& sl, std::vector<Req>& reqs);
};

int tfhe_server_s::launch(Slot& sl, std::vector<Req>& reqs) {
  const Req& r0 = reqs[0];
  const uint32_t B = (uint32_t)reqs.size();
  hipEvent_t waited = nullptr;  // requests submitted together share one event
  for (const Req& r : reqs) {
    if (r.ready == waited) continue;
    if (hipStreamWaitEvent(sl.s, r.ready, 0) != hipSuccess) return TFHE_EHIP;
    waited = r.ready;
  }
  if (B == 1) {
    // in place on the request's own buffers, through the public entry points
    size_t ws_bytes = 0;
    tfhe_hmult_workspace_size(r0.ctx, r0.level, 1, &ws_bytes);
    void* ws = sl.mem;
    tfhe_status st = r0.op == 0
        ? tfhe_hmult(r0.ctx, r0.a, r0.b, r0.out, r0.key, r0.level, 1, ws, ws_bytes, (tfhe_stream_t)sl.s)
        : tfhe_rotate(r0.ctx, r0.a, r0.out, r0.key, r0.galois, r0.level, 1, ws, ws_bytes, (tfhe_stream_t)sl.s);
    if (st != TFHE_OK) return st;
  } else {
    // one launch sequence for the whole batch, whatever its levels and
    // operations; the inputs are read where they are and each result is
    // copied out
    std::vector<LvReq> r;
    for (const Req& q : reqs) r.push_back(lv(q));
    if (levels_run(r0.ctx, r.data(), B, sl.mem, sl.s) != hipSuccess)
      return fail(TFHE_EHIP, "server: batch launch failed");
  }
  if (hipGetLastError() != hipSuccess) return TFHE_EHIP;
  if (hipEventRecord(sl.done, sl.s) != hipSuccess) return TFHE_EHIP;
  return TFHE_OK;
}

// Takes the next batch for slot sl: the oldest pending request and up to
// max_batch - 1 later ones of its key, halved until it fits the slot's
// memory.  Caller holds mu.
bool tfhe_server_s::take(const Slot& sl, std::vector<Req>& reqs) {
  // entries of requests already batched with an older one are stale
  while (!order.empty()) {
    auto it = pending.find(order.front().second);
    if (it != pending.end() && !it->second.empty() && it->second.front().seq == order.front().first) break;
    order.pop_front();
  }
  if (order.empty()) return false;
  const Key key = order.front().second;
  std::deque<Req>& q = pending[key];
  auto ci = ctxs.find(key.log_n);
  const uint32_t mb = ci != ctxs.end() && ci->second.max_batch ? ci->second.max_batch : max_batch;
  // the oldest request, then the others of its level and operation, then
  // the rest (each group in arrival order): fewer groups per batch
  std::vector<size_t> pick{0};
  const uint32_t lv = q.front().level, op = q.front().op;
  for (int pass = 0; pass < 2; ++pass)
    for (size_t i = 1; i < q.size() && pick.size() < mb; ++i)
      if ((q[i].level == lv && q[i].op == op) == (pass == 0)) pick.push_back(i);
  std::vector<Req> cand;
  for (size_t i : pick) cand.push_back(q[i]);
  uint32_t B = (uint32_t)cand.size();
  while (B > 1 && need(cand.begin(), B) > sl.bytes) B /= 2;
  if (need(cand.begin(), B) > sl.bytes) return false;  // cannot happen: submission checks one request
  reqs.assign(cand.begin(), cand.begin() + B);
  std::vector<size_t> gone(pick.begin(), pick.begin() + B);
  std::sort(gone.rbegin(), gone.rend());
  for (size_t i : gone) q.erase(q.begin() + i);
  if (q.empty()) pending.erase(key);
  order.pop_front();  // the requests taken from further back leave stale entries
  return true;
}

// One worker per slot: take a batch, launch it on the slot's stream, wait
// for it (spinning: a completed batch is reported within microseconds),
// report it, repeat.  Workers launch concurrently.
void tfhe_server_s::worker(Slot& sl) {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    std::vector<Req> reqs;
    while (!stop && !take(sl, reqs)) cv.wait(lk);
    if (reqs.empty()) break;  // stopping
    lk.unlock();
    int st = launch(sl, reqs);
    if (st == TFHE_OK) {
      hipError_t q;
      while ((q = hipEventQuery(sl.done)) == hipErrorNotReady) std::this_thread::yield();
      if (q != hipSuccess) st = TFHE_EHIP;
    } else {
      (void)hipStreamSynchronize(sl.s);  // a failed batch reports at once: let what it queued finish first
    }
    lk.lock();
    for (const Req& r : reqs) {
      done.emplace_back(r.tag, st);
      release_event(r.ready);
    }
  }
}

// Validates one request and resolves its context and key (caller holds mu).
tfhe_status tfhe_server_s::check(const tfhe_server_request& q, Req& out) {
  if (q.op > 1) return fail(TFHE_EINVAL, "server_submit: op is 0 (HMULT) or 1 (HROTATE)");
  auto it = ctxs.find(q.log_n);
  if (it == ctxs.end()) return fail(TFHE_EINVAL, "server_submit: no context for this N");
  const Ctx& c = it->second;
  if (q.level < 1 || q.level > c.ctx->L) return fail(TFHE_EINVAL, "server_submit: level must be in [1, L]");
  const auto al16 = [](const void* p) { return p && (uintptr_t)p % 16 == 0; };
  if (!al16(q.ct_a) || !al16(q.ct_out) || (q.op == 0 && !al16(q.ct_b)))
    return fail(TFHE_EINVAL, "server_submit: null or unaligned ciphertext");
  if (q.op == 1 && q.ct_a == q.ct_out) return fail(TFHE_EINVAL, "server_submit: rotation input and output alias");
  const uint32_t* key = c.evk;
  if (q.op == 1) {
    auto k = c.rk.find(q.galois_elt);
    if (k == c.rk.end()) return fail(TFHE_EINVAL, "server_submit: no rotation key for this element");
    key = k->second;
  }
  out = Req{q.op, q.log_n, q.level, q.galois_elt, q.ct_a, q.ct_b, q.ct_out, q.tag, 0, nullptr, c.ctx, key};
  if (need(&out, 1) > slots[0].bytes)
    return fail(TFHE_ENOMEM, "server_submit: one request exceeds a slot's share of the pool");
  return TFHE_OK;
}

extern "C" {

tfhe_status tfhe_server_create(tfhe_server* out, uint32_t slots, uint32_t max_batch, void* pool,
                               size_t pool_bytes) {
  if (!out) return fail(TFHE_EINVAL, "server_create: null out");
  *out = nullptr;
  if (slots < 1 || slots > 16) return fail(TFHE_EINVAL, "server_create: slots in [1, 16]");
  if (max_batch < 1 || max_batch > kMaxRotBatch)
    return fail(TFHE_EINVAL, "server_create: max_batch in [1, TFHE_ROTATE_MULTI_MAX]");
  if (!pool || (uintptr_t)pool % 256 || pool_bytes < 256 * (size_t)slots)
    return fail(TFHE_EINVAL, "server_create: pool must be 256-byte aligned device memory");
  tfhe_server_s* s = new (std::nothrow) tfhe_server_s();
  if (!s) return fail(TFHE_ENOMEM, "server_create: host allocation");
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(TFHE_EHIP, "server_create: no current device");
  }
  s->max_batch = max_batch;
  s->slots.resize(slots);
  const size_t share = pool_bytes / slots / 256 * 256;
  for (uint32_t i = 0; i < slots; ++i) {
    Slot& sl = s->slots[i];
    if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      tfhe_server_destroy(s);
      return fail(TFHE_EHIP, "server_create: stream or event creation");
    }
    sl.mem = (unsigned char*)pool + i * share;
    sl.bytes = share;
  }
  for (Slot& sl : s->slots) s->workers.emplace_back([s, &sl] { s->worker(sl); });
  *out = s;
  return TFHE_OK;
}

tfhe_status tfhe_server_add_context(tfhe_server s, tfhe_ckks_ctx ctx, const uint32_t* evk) {
  if (!s || !ctx || !evk) return fail(TFHE_EINVAL, "server_add_context: null argument");
  if ((uintptr_t)evk % 16) return fail(TFHE_EINVAL, "server_add_context: evk not 16-byte aligned");
  std::lock_guard<std::mutex> g(s->mu);
  Ctx& c = s->ctxs[ctx->log_n];
  // rotation keys belong to the context they were registered for
  if (c.ctx != ctx) c.rk.clear();
  c.ctx = ctx;
  c.evk = evk;
  return TFHE_OK;
}

tfhe_status tfhe_server_set_max_batch(tfhe_server s, uint32_t log_n, uint32_t max_batch) {
  if (!s) return fail(TFHE_EINVAL, "server_set_max_batch: null server");
  if (max_batch > kMaxRotBatch) return fail(TFHE_EINVAL, "server_set_max_batch: max_batch above TFHE_ROTATE_MULTI_MAX");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->ctxs.find(log_n);
  if (it == s->ctxs.end()) return fail(TFHE_EINVAL, "server_set_max_batch: no context for this N");
  it->second.max_batch = max_batch;
  return TFHE_OK;
}

tfhe_status tfhe_server_add_rotation_key(tfhe_server s, uint32_t log_n, uint32_t galois_elt,
                                         const uint32_t* rotkey) {
  if (!s || !rotkey) return fail(TFHE_EINVAL, "server_add_rotation_key: null argument");
  if ((uintptr_t)rotkey % 16) return fail(TFHE_EINVAL, "server_add_rotation_key: key not 16-byte aligned");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->ctxs.find(log_n);
  if (it == s->ctxs.end()) return fail(TFHE_EINVAL, "server_add_rotation_key: no context for this N");
  if ((galois_elt & 1) == 0 || galois_elt >= 2 * it->second.ctx->n)
    return fail(TFHE_EINVAL, "server_add_rotation_key: galois element must be odd and < 2N");
  it->second.rk[galois_elt] = rotkey;
  return TFHE_OK;
}

tfhe_status tfhe_server_submit_many(tfhe_server s, const tfhe_server_request* reqs, uint32_t count,
                                    tfhe_stream_t stream, uint32_t* bad) {
  if (!s) return fail(TFHE_EINVAL, "server_submit: null server");
  if (count == 0) return TFHE_OK;
  if (!reqs) return fail(TFHE_EINVAL, "server_submit_many: null request array");
  std::vector<Req> batch(count);
  hipEvent_t ev = nullptr;
  {
    std::lock_guard<std::mutex> g(s->mu);
    for (uint32_t i = 0; i < count; ++i) {
      const tfhe_status st = s->check(reqs[i], batch[i]);
      if (st != TFHE_OK) {
        if (bad) *bad = i;
        return st;
      }
    }
    if (!s->event_pool.empty()) {
      ev = s->event_pool.back();
      s->event_pool.pop_back();
    }
  }
  if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
    return fail(TFHE_EHIP, "server_submit: event creation");
  if (hipEventRecord(ev, (hipStream_t)stream) != hipSuccess) {
    (void)hipEventDestroy(ev);
    return fail(TFHE_EHIP, "server_submit: event record");
  }
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->ev_refs[ev] = count;
    for (Req& r : batch) {
      const Key k{r.log_n, r.ctx};
      r.seq = s->next_seq++;
      r.ready = ev;
      s->pending[k].push_back(r);
      s->order.emplace_back(r.seq, k);
    }
  }
  if (count == 1) s->cv.notify_one();
  else s->cv.notify_all();
  return TFHE_OK;
}

tfhe_status tfhe_server_submit(tfhe_server s, uint32_t op, uint32_t log_n, uint32_t level, const uint32_t* ct_a,
                               const uint32_t* ct_b, uint32_t galois_elt, uint32_t* ct_out, uint64_t tag,
                               tfhe_stream_t stream) {
  const tfhe_server_request r{op, log_n, level, galois_elt, ct_a, ct_b, ct_out, tag};
  return tfhe_server_submit_many(s, &r, 1, stream, nullptr);
}

uint32_t tfhe_server_poll(tfhe_server s, uint64_t* tags, int32_t* status, uint32_t max) {
  if (!s || !tags || !status) return 0;
  std::lock_guard<std::mutex> g(s->mu);
  const uint32_t k = (uint32_t)std::min<size_t>(max, s->done.size());
  for (uint32_t i = 0; i < k; ++i) {
    tags[i] = s->done[i].first;
    status[i] = s->done[i].second;
  }
  s->done.erase(s->done.begin(), s->done.begin() + k);
  return k;
}

tfhe_status tfhe_server_destroy(tfhe_server s) {
  if (!s) return TFHE_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (std::thread& t : s->workers) t.join();  // each finishes its batch in flight
  for (Slot& sl : s->slots) {
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.s) (void)hipStreamDestroy(sl.s);
  }
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  for (auto& kv : s->ev_refs) (void)hipEventDestroy(kv.first);  // held by requests never dispatched
  delete s;
  return TFHE_OK;
}

}  // extern "C"
