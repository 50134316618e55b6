// C ABI entry points (include/tfhe.h): argument validation, error reporting
// and dispatch to the kernels.  No exception crosses the ABI.
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

namespace tfhe {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

tfhe_status fail(tfhe_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

tfhe_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return TFHE_OK;
  return fail(TFHE_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

tfhe_status plan_build(tfhe_ntt_plan_s* p);
void plan_free(tfhe_ntt_plan_s* p);

static bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Shared validation of a (plan, limb range, batch) compute call.
static tfhe_status check_range(const tfhe_ntt_plan_s* p, uint32_t limb_begin, uint32_t limb_count,
                               uint32_t batch) {
  if (!p) return fail(TFHE_EINVAL, "null plan");
  if ((uint64_t)limb_begin + limb_count > p->n_limbs)
    return fail(TFHE_EINVAL, "limb range exceeds the plan's limbs");
  if ((uint64_t)limb_count * batch * p->n > (1ull << 40))
    return fail(TFHE_EINVAL, "batch too large");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail(TFHE_EINVAL, "the plan's device is not the current device");
  return TFHE_OK;
}

static tfhe_status check_ptr(const void* ptr, const char* name) {
  if (!ptr) return fail(TFHE_EINVAL, std::string("null pointer: ") + name);
  if (!aligned(ptr, 16)) return fail(TFHE_EINVAL, std::string("pointer not 16-byte aligned: ") + name);
  return TFHE_OK;
}

static tfhe_ntt_algo resolve(const tfhe_ntt_plan_s* p, tfhe_ntt_algo a) {
  return a == TFHE_NTT_AUTO ? p->algo : a;
}

}  // namespace tfhe

using namespace tfhe;

extern "C" {

const char* tfhe_status_string(tfhe_status s) {
  switch (s) {
    case TFHE_OK: return "TFHE_OK";
    case TFHE_EINVAL: return "TFHE_EINVAL";
    case TFHE_ENOTNTT: return "TFHE_ENOTNTT";
    case TFHE_ENOMEM: return "TFHE_ENOMEM";
    case TFHE_EHIP: return "TFHE_EHIP";
    case TFHE_EUNSUPPORTED: return "TFHE_EUNSUPPORTED";
  }
  return "TFHE_UNKNOWN";
}

const char* tfhe_last_error(void) { return g_last_error.c_str(); }

tfhe_status tfhe_find_primes(uint32_t bits, uint64_t two_n, uint32_t count, uint32_t* out) {
  if (!out || bits < 30 || bits > 31 || two_n < 2 || (two_n & (two_n - 1)))
    return fail(TFHE_EINVAL, "find_primes: bits in [30,31], two_n a power of two, out non-null");
  uint64_t q = ((1ull << bits) - 1) / two_n * two_n + 1;
  if (q >= (1ull << bits)) q -= two_n;
  uint32_t found = 0;
  while (found < count && q > (1ull << 29)) {
    if (is_prime_u32((uint32_t)q)) out[found++] = (uint32_t)q;
    q -= two_n;
  }
  if (found < count) return fail(TFHE_EINVAL, "find_primes: not enough primes above 2^29");
  return TFHE_OK;
}

tfhe_status tfhe_default_psi(uint32_t q, uint32_t log_n, uint32_t* psi) {
  if (!psi || log_n < 1 || log_n > 20) return fail(TFHE_EINVAL, "default_psi: bad argument");
  uint32_t r = default_psi(q, log_n);
  if (!r) return fail(TFHE_ENOTNTT, "default_psi: q is not a prime = 1 mod 2N");
  *psi = r;
  return TFHE_OK;
}

tfhe_status tfhe_ntt_plan_create(tfhe_ntt_plan* out, uint32_t log_n, uint32_t n_limbs,
                                 const uint32_t* q, const uint32_t* psi, tfhe_ntt_algo algo) {
  if (!out || !q) return fail(TFHE_EINVAL, "plan_create: null argument");
  *out = nullptr;
  if (log_n < 4 || log_n > 16) return fail(TFHE_EINVAL, "plan_create: log_n must be in [4, 16]");
  if (n_limbs == 0 || n_limbs > 4096) return fail(TFHE_EINVAL, "plan_create: n_limbs in [1, 4096]");
  if (algo != TFHE_NTT_AUTO && algo != TFHE_NTT_BUTTERFLY && algo != TFHE_NTT_FOURSTEP_MFMA)
    return fail(TFHE_EINVAL, "plan_create: unknown algorithm");
  const uint64_t two_n = 2ull << log_n;
  tfhe_ntt_plan_s* p = new (std::nothrow) tfhe_ntt_plan_s();
  if (!p) return fail(TFHE_ENOMEM, "plan_create: host allocation");
  p->log_n = log_n;
  p->n = 1u << log_n;
  p->n_limbs = n_limbs;
  for (uint32_t l = 0; l < n_limbs; ++l) {
    uint32_t ql = q[l];
    char msg[160];
    if (ql <= (1u << 29) || ql >= (1u << 31) || !is_prime_u32(ql) || (ql - 1) % two_n != 0) {
      snprintf(msg, sizeof msg, "limb %u: q=%u must be a prime in (2^29, 2^31) with q = 1 mod 2N", l, ql);
      delete p;
      return fail(TFHE_ENOTNTT, msg);
    }
    uint32_t s = psi ? psi[l] : default_psi(ql, log_n);
    // primitive 2N-th root <=> s^N = -1 (2N is a power of two)
    if (s == 0 || s >= ql || pow_mod(s, p->n, ql) != ql - 1) {
      snprintf(msg, sizeof msg, "limb %u: psi=%u is not a primitive 2N-th root of unity mod %u", l, s, ql);
      delete p;
      return fail(TFHE_ENOTNTT, msg);
    }
    p->q.push_back(ql);
    p->psi.push_back(s);
  }
  tfhe_status st = plan_build(p);
  if (st != TFHE_OK) {
    plan_free(p);
    delete p;
    return st;
  }
  if (algo == TFHE_NTT_FOURSTEP_MFMA && !p->has_mfma) {
    plan_free(p);
    delete p;
    return fail(TFHE_EUNSUPPORTED, "plan_create: the MFMA four-step NTT does not cover this N");
  }
  p->algo = algo == TFHE_NTT_AUTO ? (p->has_mfma ? TFHE_NTT_FOURSTEP_MFMA : TFHE_NTT_BUTTERFLY) : algo;
  *out = p;
  return TFHE_OK;
}

tfhe_status tfhe_ntt_plan_destroy(tfhe_ntt_plan plan) {
  if (!plan) return TFHE_OK;
  plan_free(plan);
  delete plan;
  return TFHE_OK;
}

tfhe_status tfhe_ntt_plan_info(tfhe_ntt_plan plan, uint32_t* log_n, uint32_t* n_limbs,
                               tfhe_ntt_algo* algo) {
  if (!plan) return fail(TFHE_EINVAL, "null plan");
  if (log_n) *log_n = plan->log_n;
  if (n_limbs) *n_limbs = plan->n_limbs;
  if (algo) *algo = plan->algo;
  return TFHE_OK;
}

tfhe_status tfhe_ntt_plan_modulus(tfhe_ntt_plan plan, uint32_t limb, uint32_t* q, uint32_t* psi) {
  if (!plan || limb >= plan->n_limbs) return fail(TFHE_EINVAL, "plan_modulus: bad plan or limb");
  if (q) *q = plan->q[limb];
  if (psi) *psi = plan->psi[limb];
  return TFHE_OK;
}

tfhe_status tfhe_ntt_plan_set_param(tfhe_ntt_plan plan, tfhe_plan_param param, int64_t value) {
  if (!plan) return fail(TFHE_EINVAL, "null plan");
  switch (param) {
    case TFHE_PARAM_FS_WG_PER_CU:
      if (value < 0 || value > 32) return fail(TFHE_EINVAL, "fs_wg_per_cu must be in [0, 32]");
      plan->fs_wg_per_cu = (uint32_t)value;
      return TFHE_OK;
    case TFHE_PARAM_AUTO_ALGO:
      if (value == TFHE_NTT_BUTTERFLY || (value == TFHE_NTT_FOURSTEP_MFMA && plan->has_mfma)) {
        plan->algo = (tfhe_ntt_algo)value;
        return TFHE_OK;
      }
      if (value == TFHE_NTT_AUTO) {
        plan->algo = plan->has_mfma ? TFHE_NTT_FOURSTEP_MFMA : TFHE_NTT_BUTTERFLY;
        return TFHE_OK;
      }
      return fail(TFHE_EINVAL, "auto_algo: not an algorithm this plan supports");
    case TFHE_PARAM_FS_WIDE:
      if (value < 0 || value > 2) return fail(TFHE_EINVAL, "fs_wide must be 0, 1 or 2");
      plan->fs_wide = (uint32_t)value;
      return TFHE_OK;
    case TFHE_PARAM_FS_PASSES:
      if (value < 0 || value > 2) return fail(TFHE_EINVAL, "fs_passes must be 0, 1 or 2");
      plan->fs_passes = (uint32_t)value;
      return TFHE_OK;
    case TFHE_PARAM_KS_INNER:
      if (value < 0 || value > 2) return fail(TFHE_EINVAL, "ks_inner must be 0, 1 or 2");
      plan->ks_inner = (uint32_t)value;
      return TFHE_OK;
    case TFHE_PARAM_FS_RING:
      if (value != 0 && value != 2 && value != 3) return fail(TFHE_EINVAL, "fs_ring must be 0, 2 or 3");
      plan->fs_ring = (uint32_t)value;
      return TFHE_OK;
  }
  return fail(TFHE_EINVAL, "unknown plan parameter");
}

tfhe_status tfhe_ntt_plan_get_param(tfhe_ntt_plan plan, tfhe_plan_param param, int64_t* value) {
  if (!plan || !value) return fail(TFHE_EINVAL, "null argument");
  switch (param) {
    case TFHE_PARAM_FS_WG_PER_CU: *value = plan->fs_wg_per_cu; return TFHE_OK;
    case TFHE_PARAM_AUTO_ALGO: *value = plan->algo; return TFHE_OK;
    case TFHE_PARAM_FS_WIDE: *value = plan->fs_wide; return TFHE_OK;
    case TFHE_PARAM_FS_PASSES: *value = plan->fs_passes; return TFHE_OK;
    case TFHE_PARAM_KS_INNER: *value = plan->ks_inner; return TFHE_OK;
    case TFHE_PARAM_FS_RING: *value = plan->fs_ring; return TFHE_OK;
  }
  return fail(TFHE_EINVAL, "unknown plan parameter");
}

tfhe_status tfhe_ntt_workspace_size(tfhe_ntt_plan plan, tfhe_ntt_algo algo, uint32_t limb_count,
                                    uint32_t batch, size_t* bytes) {
  if (!plan || !bytes) return fail(TFHE_EINVAL, "workspace_size: null argument");
  tfhe_ntt_algo a = resolve(plan, algo);
  if (a == TFHE_NTT_FOURSTEP_MFMA && !plan->has_mfma)
    return fail(TFHE_EUNSUPPORTED, "MFMA four-step not available for this plan");
  if (a == TFHE_NTT_FOURSTEP_VALU && !plan->has_co)
    return fail(TFHE_EUNSUPPORTED, "vector-ALU four-step is available for N = 2^16 only");
  *bytes = a == TFHE_NTT_BUTTERFLY ? bf_workspace_bytes(plan, limb_count, batch)
                                   : fs_workspace_bytes(plan, limb_count, batch);
  return TFHE_OK;
}

static tfhe_status ntt_dispatch(bool inverse, tfhe_ntt_plan plan, tfhe_ntt_algo algo,
                                const uint32_t* in, uint32_t* out, uint32_t limb_begin,
                                uint32_t limb_count, uint32_t batch, void* ws, size_t ws_bytes,
                                tfhe_stream_t stream) {
  tfhe_status st = check_range(plan, limb_begin, limb_count, batch);
  if (st != TFHE_OK) return st;
  if (limb_count == 0 || batch == 0) return TFHE_OK;
  if ((st = check_ptr(in, "in")) != TFHE_OK || (st = check_ptr(out, "out")) != TFHE_OK) return st;
  const tfhe_ntt_algo a = resolve(plan, algo);
  if (a != TFHE_NTT_BUTTERFLY && a != TFHE_NTT_FOURSTEP_MFMA && a != TFHE_NTT_FOURSTEP_VALU)
    return fail(TFHE_EINVAL, "unknown algorithm");
  if (a == TFHE_NTT_FOURSTEP_MFMA && !plan->has_mfma)
    return fail(TFHE_EUNSUPPORTED, "MFMA four-step not available for this plan");
  if (a == TFHE_NTT_FOURSTEP_VALU && !plan->has_co)
    return fail(TFHE_EUNSUPPORTED, "vector-ALU four-step is available for N = 2^16 only");
  const size_t need = a == TFHE_NTT_BUTTERFLY ? bf_workspace_bytes(plan, limb_count, batch)
                                              : fs_workspace_bytes(plan, limb_count, batch);
  if (need) {
    if (!ws || ws_bytes < need) return fail(TFHE_EINVAL, "workspace missing or too small");
    if (!aligned(ws, 256)) return fail(TFHE_EINVAL, "workspace not 256-byte aligned");
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (a == TFHE_NTT_FOURSTEP_VALU)
    e = co_transform(plan, inverse, in, out, ws, limb_begin, limb_count, batch, s);
  else if (a == TFHE_NTT_FOURSTEP_MFMA)
    e = inverse ? fs_inverse(plan, in, out, ws, limb_begin, limb_count, batch, s)
                : fs_forward(plan, in, out, ws, limb_begin, limb_count, batch, s);
  else
    e = inverse ? bf_inverse(plan, in, out, ws, limb_begin, limb_count, batch, s)
                : bf_forward(plan, in, out, ws, limb_begin, limb_count, batch, s);
  return hip_check(e, inverse ? "ntt_inv launch" : "ntt_fwd launch");
}

tfhe_status tfhe_ntt_fwd(tfhe_ntt_plan plan, tfhe_ntt_algo algo, const uint32_t* in, uint32_t* out,
                         uint32_t limb_begin, uint32_t limb_count, uint32_t batch, void* ws,
                         size_t ws_bytes, tfhe_stream_t stream) {
  return ntt_dispatch(false, plan, algo, in, out, limb_begin, limb_count, batch, ws, ws_bytes, stream);
}

tfhe_status tfhe_ntt_inv(tfhe_ntt_plan plan, tfhe_ntt_algo algo, const uint32_t* in, uint32_t* out,
                         uint32_t limb_begin, uint32_t limb_count, uint32_t batch, void* ws,
                         size_t ws_bytes, tfhe_stream_t stream) {
  return ntt_dispatch(true, plan, algo, in, out, limb_begin, limb_count, batch, ws, ws_bytes, stream);
}

// Resolve a batch's algorithm: MFMA only if every plan has it.
static tfhe_status batch_algo(const tfhe_ntt_desc* d, uint32_t count, tfhe_ntt_algo algo, bool* mfma) {
  bool all = true;
  for (uint32_t k = 0; k < count; ++k) {
    if (!d[k].plan) return fail(TFHE_EINVAL, "ntt_batch: null plan in a descriptor");
    all = all && d[k].plan->has_mfma;
  }
  if (algo == TFHE_NTT_FOURSTEP_MFMA && !all)
    return fail(TFHE_EUNSUPPORTED, "ntt_batch: a plan lacks the MFMA four-step transform");
  if (algo != TFHE_NTT_AUTO && algo != TFHE_NTT_BUTTERFLY && algo != TFHE_NTT_FOURSTEP_MFMA)
    return fail(TFHE_EINVAL, "ntt_batch: unknown algorithm");
  *mfma = algo == TFHE_NTT_FOURSTEP_MFMA || (algo == TFHE_NTT_AUTO && all && count > 0 &&
                                             d[0].plan->algo == TFHE_NTT_FOURSTEP_MFMA);
  return TFHE_OK;
}

tfhe_status tfhe_ntt_batch_workspace_size(const tfhe_ntt_desc* descs, uint32_t count,
                                          tfhe_ntt_algo algo, size_t* bytes) {
  if (!bytes || (count && !descs)) return fail(TFHE_EINVAL, "ntt_batch_workspace_size: null argument");
  bool mfma = false;
  tfhe_status st = batch_algo(descs, count, algo, &mfma);
  if (st != TFHE_OK) return st;
  size_t total = 0;
  for (uint32_t k = 0; k < count; ++k) {
    NttUnit u{descs[k].plan, descs[k].inverse != 0, descs[k].in, descs[k].out, descs[k].limb_begin,
              descs[k].limb_count, descs[k].batch};
    total += (unit_ws_bytes(u, mfma) + 255) & ~(size_t)255;
  }
  *bytes = total;
  return TFHE_OK;
}

tfhe_status tfhe_ntt_batch(const tfhe_ntt_desc* descs, uint32_t count, tfhe_ntt_algo algo, void* ws,
                           size_t ws_bytes, tfhe_stream_t stream) {
  if (count == 0) return TFHE_OK;
  if (!descs) return fail(TFHE_EINVAL, "ntt_batch: null descriptors");
  bool mfma = false;
  tfhe_status st = batch_algo(descs, count, algo, &mfma);
  if (st != TFHE_OK) return st;
  std::vector<NttUnit> units;
  size_t need = 0;
  for (uint32_t k = 0; k < count; ++k) {
    const tfhe_ntt_desc& d = descs[k];
    if ((st = check_range(d.plan, d.limb_begin, d.limb_count, d.batch)) != TFHE_OK) return st;
    if (d.limb_count == 0 || d.batch == 0) continue;
    if ((st = check_ptr(d.in, "in")) != TFHE_OK || (st = check_ptr(d.out, "out")) != TFHE_OK) return st;
    units.push_back(NttUnit{d.plan, d.inverse != 0, d.in, d.out, d.limb_begin, d.limb_count, d.batch});
    need += (unit_ws_bytes(units.back(), mfma) + 255) & ~(size_t)255;
  }
  if (need) {
    if (!ws || ws_bytes < need) return fail(TFHE_EINVAL, "ntt_batch: workspace missing or too small");
    if (!aligned(ws, 256)) return fail(TFHE_EINVAL, "ntt_batch: workspace not 256-byte aligned");
  }
  if (units.empty()) return TFHE_OK;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = mfma ? fs_run_units(units.data(), (uint32_t)units.size(), ws, s)
                      : bf_run_units(units.data(), (uint32_t)units.size(), ws, s);
  return hip_check(e, "ntt_batch launch");
}

static tfhe_status ew_dispatch(EwOp op, tfhe_ntt_plan plan, const uint32_t* a, const uint32_t* b,
                               uint32_t* c, uint32_t limb_begin, uint32_t limb_count,
                               uint32_t batch, tfhe_stream_t stream) {
  tfhe_status st = check_range(plan, limb_begin, limb_count, batch);
  if (st != TFHE_OK) return st;
  if (limb_count == 0 || batch == 0) return TFHE_OK;
  if ((st = check_ptr(a, "a")) != TFHE_OK || (st = check_ptr(b, "b")) != TFHE_OK ||
      (st = check_ptr(c, "c")) != TFHE_OK)
    return st;
  return hip_check(ew_launch(op, plan->d_mod + limb_begin, a, b, c, limb_count, batch, plan->n,
                             (hipStream_t)stream),
                   "element-wise launch");
}

tfhe_status tfhe_pointwise_mul(tfhe_ntt_plan plan, const uint32_t* a, const uint32_t* b, uint32_t* c,
                               uint32_t limb_begin, uint32_t limb_count, uint32_t batch,
                               tfhe_stream_t stream) {
  return ew_dispatch(EW_MUL, plan, a, b, c, limb_begin, limb_count, batch, stream);
}

tfhe_status tfhe_pointwise_add(tfhe_ntt_plan plan, const uint32_t* a, const uint32_t* b, uint32_t* c,
                               uint32_t limb_begin, uint32_t limb_count, uint32_t batch,
                               tfhe_stream_t stream) {
  return ew_dispatch(EW_ADD, plan, a, b, c, limb_begin, limb_count, batch, stream);
}

tfhe_status tfhe_pointwise_sub(tfhe_ntt_plan plan, const uint32_t* a, const uint32_t* b, uint32_t* c,
                               uint32_t limb_begin, uint32_t limb_count, uint32_t batch,
                               tfhe_stream_t stream) {
  return ew_dispatch(EW_SUB, plan, a, b, c, limb_begin, limb_count, batch, stream);
}

tfhe_status tfhe_pointwise_mul_bcast(tfhe_ntt_plan plan, const uint32_t* a, const uint32_t* b,
                                     uint32_t* c, uint32_t limb_begin, uint32_t limb_count,
                                     uint32_t batch, tfhe_stream_t stream) {
  return ew_dispatch(EW_MUL_BCAST, plan, a, b, c, limb_begin, limb_count, batch, stream);
}

tfhe_status tfhe_load_small(tfhe_ntt_plan plan, const int32_t* in, uint32_t* out,
                            uint32_t limb_begin, uint32_t limb_count, uint32_t batch,
                            tfhe_stream_t stream) {
  tfhe_status st = check_range(plan, limb_begin, limb_count, batch);
  if (st != TFHE_OK) return st;
  if (limb_count == 0 || batch == 0) return TFHE_OK;
  if ((st = check_ptr(in, "in")) != TFHE_OK || (st = check_ptr(out, "out")) != TFHE_OK) return st;
  return hip_check(load_small_launch(plan->d_mod + limb_begin, in, out, limb_count, batch, plan->n,
                                     (hipStream_t)stream),
                   "load_small launch");
}

tfhe_status tfhe_frobenius_map(tfhe_ntt_plan plan, const uint32_t* in, uint32_t* out,
                               uint32_t galois_elt, uint32_t limb_count, uint32_t batch,
                               tfhe_stream_t stream) {
  if (!plan) return fail(TFHE_EINVAL, "null plan");
  if ((galois_elt & 1) == 0 || galois_elt >= 2 * plan->n)
    return fail(TFHE_EINVAL, "frobenius_map: galois element must be odd and < 2N");
  if (limb_count == 0 || batch == 0) return TFHE_OK;
  tfhe_status st;
  if ((st = check_ptr(in, "in")) != TFHE_OK || (st = check_ptr(out, "out")) != TFHE_OK) return st;
  if (in == out) return fail(TFHE_EINVAL, "frobenius_map: out must not alias in");
  return hip_check(frobenius_launch(in, out, galois_elt, limb_count * batch, plan->log_n,
                                    (hipStream_t)stream),
                   "frobenius launch");
}

}  // extern "C"
