// RNS-CKKS context and the HMULT / HROTATE operations (Sec. II-B, Sec. IV-A,
// Table 2) as stream-ordered kernel sequences on the device.
//
// Key switching follows the hybrid method the paper adopts (Sec. II-B,
// "Generalized Key-Switching"): Dcomp splits the limbs of the input into
// digits of alpha = L/dnum limbs, ModUp extends each digit to Q_l * P by fast
// basis conversion (no overflow correction), the inner product with the key
// accumulates over the digits, and ModDown divides by P (no rounding offset).
#include <string.h>

#include <mutex>
#include <new>
#include <set>
#include <vector>

#include "ckks_internal.hpp"

namespace tfhe {

// Scratch memory of tfhe_hmult_noalloc: a fixed device array in the code
// object, one copy per GPU.  Its name is a host-side stand-in; host code
// uses only the device address resolved per device by scratch_bind.
static __device__ __attribute__((aligned(256))) unsigned char scratch[TFHE_HMULT_NOALLOC_MAX_BYTES];

static std::mutex g_scratch_mu;
static std::vector<unsigned char*> g_scratch_ptr;  // per device ordinal, null until bound

// Resolves this device's copy of `scratch` (the device must be current).
// Called once per device, at context creation.
static tfhe_status scratch_bind(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0) return fail(TFHE_EINVAL, "scratch_bind: bad device");
  if ((size_t)dev < g_scratch_ptr.size() && g_scratch_ptr[dev]) return TFHE_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return hip_check(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
  if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize(dev + 1, nullptr);
  g_scratch_ptr[dev] = (unsigned char*)ptr;
  return TFHE_OK;
}

static unsigned char* scratch_of(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (dev >= 0 && (size_t)dev < g_scratch_ptr.size()) ? g_scratch_ptr[dev] : nullptr;
}

tfhe_status plan_build(tfhe_ntt_plan_s* p);
void plan_free(tfhe_ntt_plan_s* p);

static uint32_t mulm(uint32_t a, uint32_t b, uint32_t q) { return (uint32_t)((uint64_t)a * b % q); }

static uint2 with_companion(uint32_t w, uint32_t q) { return make_uint2(w, shoup_companion(w, q)); }

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Fused NTT launches over several units with the plan's algorithm.
static hipError_t ntt_units(const tfhe_ntt_plan_s* p, const std::vector<NttUnit>& u, void* ws,
                            hipStream_t s) {
  if (u.empty()) return hipSuccess;
  return p->algo == TFHE_NTT_FOURSTEP_MFMA ? fs_run_units(u.data(), (uint32_t)u.size(), ws, s)
                                           : bf_run_units(u.data(), (uint32_t)u.size(), ws, s);
}

// Whether the ModUp transforms' second pass runs fused with the inner
// product (ip_run): four-step plans that ask for it (TFHE_PARAM_KS_INNER =
// 1; the separate kernels are the default, measured as fast or faster at
// N = 2^15, 2^16).
static bool fused_inner(const tfhe_ckks_ctx_s* c) {
  return c->plan->algo == TFHE_NTT_FOURSTEP_MFMA && c->plan->ks_inner == 1;
}

// Workspace regions (byte offsets).
struct KsLayout {
  size_t d2, x, up, acc, tp, conv, ntt, total;
};

static KsLayout ks_layout(const tfhe_ckks_ctx_s* c, uint32_t level, uint32_t batch) {
  const size_t plane = (size_t)batch * c->n * sizeof(uint32_t);
  const uint32_t digits = (level + c->alpha - 1) / c->alpha;
  const uint32_t ext = level + c->K;
  // The transform region holds the largest of key_switch's four fused
  // transforms, each unit's slice rounded to 256 bytes as fs_run_units /
  // bf_run_units lay them out: INTT of the input (level limbs); the NTT of
  // every digit's converted limbs; the INTT of both accumulators' K special
  // limbs; the final NTT of both components (2 x level limbs).
  const tfhe_ntt_plan_s* p = c->plan;
  const bool mfma = p->algo == TFHE_NTT_FOURSTEP_MFMA;
  auto ws = [&](uint32_t limbs) {
    return limbs ? align256(unit_ws_bytes(NttUnit{p, false, nullptr, nullptr, 0, limbs, batch}, mfma)) : 0;
  };
  size_t modup = 0;
  for (uint32_t j = 0; j < digits; ++j) {
    const uint32_t d0 = c->alpha * j, nd = std::min(c->alpha, level - d0);
    modup += ws(d0) + ws(level - d0 - nd) + ws(c->K);
  }
  // with the fused second pass + inner product, the ModUp transforms'
  // intermediates sit in a regular [digits][level + K] array of planes
  if (fused_inner(c)) modup = std::max(modup, align256(plane * (size_t)digits * ext));
  const size_t ntt_bytes = std::max(std::max(ws(level), modup), std::max(2 * ws(c->K), 2 * ws(level)));
  KsLayout l;
  size_t off = 0;
  l.d2 = off; off += align256(plane * level);
  l.x = off; off += align256(plane * level);
  l.up = off; off += align256(plane * (size_t)digits * ext);
  l.acc = off; off += align256(plane * 2 * ext);
  l.tp = off; off += align256(plane * 2 * c->K);
  l.conv = off; off += align256(plane * 2 * level);
  l.ntt = off; off += align256(ntt_bytes);
  l.total = off;
  return l;
}

// ModUp conversion of digit [d0, d0 + nd) on the matrix cores: every
// extended-basis position outside the digit, in launches of <= 32 targets.
static void modup_mfma(const tfhe_ckks_ctx_s* c, const uint32_t* x, uint32_t* up, uint32_t key_idx,
                       uint32_t d0, uint32_t nd, uint32_t level, uint64_t plane, ConvQueue& cq) {
  ConvArgs a;
  a.in = x + (uint64_t)d0 * plane;
  a.out = up;
  a.plane = plane;
  a.nin = nd;
  for (uint32_t r = 0; r < nd; ++r) {
    a.in_q[r] = c->h_mod[d0 + r].q;
    a.in_mult[r] = c->h_up_inv[(size_t)key_idx * kMaxAlpha + r];
  }
  a.nout = 0;
  for (uint32_t pos = 0; pos < level + c->K; ++pos) {
    if (pos >= d0 && pos < d0 + nd) continue;
    const uint32_t t = pos < level ? pos : c->L + (pos - level);
    a.out_plane[a.nout] = pos;
    a.out_q[a.nout] = c->h_mod[t].q;
    a.out_qneg[a.nout] = c->h_mod[t].qneg;
    a.out_k[a.nout] = c->h_up_k[(size_t)key_idx * (c->L + c->K) + t];
    a.a_tab[a.nout] = c->d_up_mfma + ((size_t)key_idx * (c->L + c->K) + t) * 32;
    if (++a.nout == kConvMaxOut) {
      cq.q.push_back(a);
      a.nout = 0;
    }
  }
  if (a.nout) cq.q.push_back(a);
}

// ModDown conversion of the K special limbs to the level q-limbs.
static void moddown_conv_mfma(const tfhe_ckks_ctx_s* c, const uint32_t* tp, uint32_t* conv,
                              uint32_t level, uint64_t plane, ConvQueue& cq) {
  ConvArgs a;
  a.in = tp;
  a.out = conv;
  a.plane = plane;
  a.nin = c->K;
  for (uint32_t k = 0; k < c->K; ++k) {
    a.in_q[k] = c->h_mod[c->L + k].q;
    a.in_mult[k] = c->h_dn_invp[k];
  }
  a.nout = 0;
  for (uint32_t i = 0; i < level; ++i) {
    a.out_plane[a.nout] = i;
    a.out_q[a.nout] = c->h_mod[i].q;
    a.out_qneg[a.nout] = c->h_mod[i].qneg;
    a.out_k[a.nout] = c->h_dn_k[i];
    a.a_tab[a.nout] = c->d_dn_mfma + (size_t)i * 32;
    if (++a.nout == kConvMaxOut) {
      cq.q.push_back(a);
      a.nout = 0;
    }
  }
  if (a.nout) cq.q.push_back(a);
}

// Key switching of d (NTT domain, [level][B][N]) with keys [dnum][2][L+K][N]
// (one for the batch, or one per batch element);
// out0 (+)= ModDown(acc0), out1 (+)= ModDown(acc1).
static hipError_t key_switch(const tfhe_ckks_ctx_s* c, const uint32_t* d, const KeySet& keys,
                             uint32_t* out0, uint32_t* out1, bool acc0_add, bool acc1_add,
                             uint32_t level, uint32_t batch, unsigned char* ws, hipStream_t s) {
  const tfhe_ntt_plan_s* p = c->plan;
  const KsLayout lay = ks_layout(c, level, batch);
  const uint64_t plane = (uint64_t)batch * c->n;
  const uint32_t ext = level + c->K;
  const uint32_t digits = (level + c->alpha - 1) / c->alpha;
  uint32_t* x = (uint32_t*)(ws + lay.x);
  uint32_t* up = (uint32_t*)(ws + lay.up);
  uint32_t* acc = (uint32_t*)(ws + lay.acc);
  uint32_t* tp = (uint32_t*)(ws + lay.tp);
  uint32_t* conv = (uint32_t*)(ws + lay.conv);
  void* nws = ws + lay.ntt;
  // matrix-core conversion needs planes in whole 64-word chunks
  const bool mfma_conv = plane % 64 == 0;
  hipError_t e;
  // INTT of the input (coefficient domain for the basis conversion)
  if ((e = ntt_units(p, {NttUnit{p, true, d, x, 0, level, batch}}, nws, s)) != hipSuccess) return e;
  // Dcomp + ModUp of every digit, then one fused NTT of all converted limbs:
  // the q-limbs before and after the digit, and the p-limbs
  std::vector<NttUnit> fwd;
  ConvQueue cq;  // the matrix-core conversions of all digits, launched together
  // fused: the transforms' first pass writes digit j's intermediate of
  // position pos at inter + (j ext + pos) plane; ip_run finishes them
  const bool fused = fused_inner(c);
  uint32_t* inter = (uint32_t*)nws;
  for (uint32_t j = 0; j < digits; ++j) {
    const uint32_t d0 = c->alpha * j, nd = std::min(c->alpha, level - d0);
    const uint32_t key_idx = d0 + nd - 1;
    uint32_t* upj = up + (uint64_t)j * ext * plane;
    if (mfma_conv)
      modup_mfma(c, x, upj, key_idx, d0, nd, level, plane, cq);
    else if ((e = launch_modup(x, upj, p->d_mod, c->d_up_inv + (size_t)key_idx * kMaxAlpha,
                               c->d_up_conv + (size_t)key_idx * (c->L + c->K) * kMaxAlpha, d0, nd, level,
                               c->L, c->K, batch, c->n, s)) != hipSuccess)
      return e;
    uint32_t* outj = fused ? inter + (uint64_t)j * ext * plane : upj;
    auto unit = [&](uint32_t pos, uint32_t limb_begin, uint32_t count) {
      NttUnit u{p, false, upj + (uint64_t)pos * plane, outj + (uint64_t)pos * plane, limb_begin, count, batch};
      u.pass1_only = fused;
      fwd.push_back(u);
    };
    if (d0) unit(0, 0, d0);
    if (level > d0 + nd) unit(d0 + nd, d0 + nd, level - d0 - nd);
    unit(level, c->L, c->K);
  }
  if ((e = cq.flush(p->num_cus, K_MODUP, s)) != hipSuccess) return e;
  if ((e = ntt_units(p, fwd, nws, s)) != hipSuccess) return e;
  uint32_t* a0 = acc;
  uint32_t* a1 = acc + (uint64_t)ext * plane;
  if (fused) {
    IpArgs ia;
    ia.inter = inter;
    ia.d2 = d;
    ia.acc = acc;
    ia.batch = batch;
    ia.level = level;
    ia.L = c->L;
    ia.K = c->K;
    ia.alpha = c->alpha;
    ia.digits = digits;
    ia.keys = keys;
    if ((e = ip_run(p, ia, s)) != hipSuccess) return e;
  } else if ((e = launch_inner_product(d, up, keys, a0, a1, p->d_mod, c->alpha, digits, level, c->L, c->K,
                                       batch, c->log_n, s)) != hipSuccess) {
    return e;
  }
  // ModDown of both accumulators, their transforms fused
  uint32_t* tp1 = tp + (uint64_t)c->K * plane;
  uint32_t* conv1 = conv + (uint64_t)level * plane;
  if ((e = ntt_units(p, {NttUnit{p, true, a0 + (uint64_t)level * plane, tp, c->L, c->K, batch},
                         NttUnit{p, true, a1 + (uint64_t)level * plane, tp1, c->L, c->K, batch}},
                     nws, s)) != hipSuccess)
    return e;
  for (int comp = 0; comp < 2; ++comp)
    if (mfma_conv)
      moddown_conv_mfma(c, comp ? tp1 : tp, comp ? conv1 : conv, level, plane, cq);
    else if ((e = launch_moddown_conv(comp ? tp1 : tp, comp ? conv1 : conv, p->d_mod, c->d_dn_invp,
                                      c->d_dn_conv, level, c->L, c->K, batch, c->n, s)) != hipSuccess)
      return e;
  if ((e = cq.flush(p->num_cus, K_MD_CONV, s)) != hipSuccess) return e;
  if (p->algo == TFHE_NTT_FOURSTEP_MFMA) {
    // the transform's second pass finishes ModDown in its store epilogue:
    // out (+)= (acc - NTT(conv)) P^{-1}
    NttUnit u0{p, false, conv, out0, 0, level, batch};
    NttUnit u1{p, false, conv1, out1, 0, level, batch};
    u0.acc = a0;
    u1.acc = a1;
    u0.epi_mult = u1.epi_mult = c->d_dn_pinv;
    u0.epi_add = acc0_add;
    u1.epi_add = acc1_add;
    return ntt_units(p, {u0, u1}, nws, s);
  }
  if ((e = ntt_units(p, {NttUnit{p, false, conv, conv, 0, level, batch},
                         NttUnit{p, false, conv1, conv1, 0, level, batch}},
                     nws, s)) != hipSuccess)
    return e;
  for (int comp = 0; comp < 2; ++comp)
    if ((e = launch_moddown_final(comp ? a1 : a0, comp ? conv1 : conv, comp ? out1 : out0, p->d_mod,
                                  c->d_dn_pinv, level, batch, c->n, comp ? acc1_add : acc0_add, s)) !=
        hipSuccess)
      return e;
  return hipSuccess;
}

hipError_t hmult_ptrs(const tfhe_ckks_ctx_s* c, const CtPtrs& a, const CtPtrs& b, uint32_t* out,
                      const uint32_t* evk, uint32_t level, uint32_t batch, unsigned char* ws, hipStream_t s) {
  const uint64_t plane = (uint64_t)level * batch * c->n;
  uint32_t* d2 = (uint32_t*)(ws + ks_layout(c, level, batch).d2);
  hipError_t e = launch_tensor_ptrs(a, b, out, d2, c->plan->d_mod, level, batch, c->log_n, s);
  KeySet keys{};
  keys.count = 1;
  keys.k[0] = evk;
  if (e == hipSuccess) e = key_switch(c, d2, keys, out, out + plane, true, true, level, batch, ws, s);
  return e;
}

hipError_t rotate_ptrs(const tfhe_ckks_ctx_s* c, const CtPtrs& in, uint32_t* out, const KeySet& keys,
                       const GaloisSet& gs, uint32_t level, uint32_t batch, unsigned char* ws, hipStream_t s) {
  const uint64_t plane = (uint64_t)level * batch * c->n;
  uint32_t* r1 = (uint32_t*)(ws + ks_layout(c, level, batch).d2);
  hipError_t e = launch_frobenius_pair_ptrs(in, out, r1, gs, level, batch, c->log_n, s);
  if (e == hipSuccess) e = key_switch(c, r1, keys, out, out + plane, true, false, level, batch, ws, s);
  return e;
}

// RESCALE workspace: the top limbs in the coefficient domain [2][B][N], their
// broadcast to the remaining limbs [2][top][B][N], the transforms' workspace.
struct RsLayout {
  size_t t, u, ntt, total;
};

static RsLayout rs_layout(const tfhe_ckks_ctx_s* c, uint32_t level, uint32_t batch) {
  const size_t plane = (size_t)batch * c->n * sizeof(uint32_t);
  const uint32_t top = level - 1;
  const tfhe_ntt_plan_s* p = c->plan;
  const bool mfma = p->algo == TFHE_NTT_FOURSTEP_MFMA;
  // the larger of the two fused transforms (2 x one limb, 2 x top limbs)
  const size_t a = 2 * align256(unit_ws_bytes(NttUnit{p, true, nullptr, nullptr, top, 1, batch}, mfma));
  const size_t b = 2 * align256(unit_ws_bytes(NttUnit{p, false, nullptr, nullptr, 0, top, batch}, mfma));
  RsLayout l;
  size_t off = 0;
  l.t = off; off += align256(2 * plane);
  l.u = off; off += align256(2 * plane * top);
  l.ntt = off; off += std::max(a, b);
  l.total = off;
  return l;
}

// RESCALE of ct [2][level][B][N] (NTT domain) into out [2][level-1][B][N].
static hipError_t rescale(const tfhe_ckks_ctx_s* c, const uint32_t* ct, uint32_t* out, uint32_t level,
                          uint32_t batch, unsigned char* ws, hipStream_t s) {
  const tfhe_ntt_plan_s* p = c->plan;
  const RsLayout lay = rs_layout(c, level, batch);
  const uint64_t plane = (uint64_t)batch * c->n;
  const uint32_t top = level - 1;
  uint32_t* t = (uint32_t*)(ws + lay.t);
  uint32_t* u = (uint32_t*)(ws + lay.u);
  void* nws = ws + lay.ntt;
  hipError_t e;
  // INTT of both components' top limb
  if ((e = ntt_units(p, {NttUnit{p, true, ct + (uint64_t)top * plane, t, top, 1, batch},
                         NttUnit{p, true, ct + (uint64_t)(level + top) * plane, t + plane, top, 1, batch}},
                     nws, s)) != hipSuccess)
    return e;
  // reduce into every remaining limb, back to the NTT domain
  if ((e = launch_rescale_bcast(t, u, p->d_mod, top, batch, c->n, s)) != hipSuccess) return e;
  if (p->algo == TFHE_NTT_FOURSTEP_MFMA) {
    // NTT of the broadcast, finished in the store epilogue: (c_i - u_i) q_top^{-1}
    NttUnit u0{p, false, u, out, 0, top, batch};
    NttUnit u1{p, false, u + (uint64_t)top * plane, out + (uint64_t)top * plane, 0, top, batch};
    u0.acc = ct;
    u1.acc = ct + (uint64_t)level * plane;
    u0.epi_mult = u1.epi_mult = c->d_rs_qinv + (size_t)top * c->L;
    return ntt_units(p, {u0, u1}, nws, s);
  }
  if ((e = ntt_units(p, {NttUnit{p, false, u, u, 0, top, batch},
                         NttUnit{p, false, u + (uint64_t)top * plane, u + (uint64_t)top * plane, 0, top, batch}},
                     nws, s)) != hipSuccess)
    return e;
  // (c_i - u_i) q_top^{-1}
  for (int comp = 0; comp < 2; ++comp)
    if ((e = launch_moddown_final(ct + (uint64_t)comp * level * plane, u + (uint64_t)comp * top * plane,
                                  out + (uint64_t)comp * top * plane, p->d_mod,
                                  c->d_rs_qinv + (size_t)top * c->L, top, batch, c->n, false, s,
                                  K_RS_FINAL)) != hipSuccess)
      return e;
  return hipSuccess;
}

template <typename T>
static hipError_t upload(T** dst, const std::vector<T>& src, std::vector<void*>& owned) {
  hipError_t e = hipMalloc((void**)dst, sizeof(T) * std::max<size_t>(src.size(), 1));
  if (e != hipSuccess) return e;
  owned.push_back(*dst);
  return hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

static tfhe_status ctx_build(tfhe_ckks_ctx_s* c) {
  const uint32_t L = c->L, K = c->K, A = c->alpha;
  const std::vector<uint32_t>& m = c->plan->q;  // q_0..q_{L-1}, p_0..p_{K-1}
  std::vector<uint2> up_inv((size_t)L * kMaxAlpha, make_uint2(0, 0));
  std::vector<uint2> up_conv((size_t)L * (L + K) * kMaxAlpha, make_uint2(0, 0));
  for (uint32_t e = 1; e <= L; ++e) {
    const uint32_t d0 = A * ((e - 1) / A), nd = e - d0;
    for (uint32_t r = 0; r < nd; ++r) {
      const uint32_t i = d0 + r;
      uint32_t prod = 1;  // Q_D / q_i mod q_i
      for (uint32_t i2 = d0; i2 < e; ++i2)
        if (i2 != i) prod = mulm(prod, m[i2] % m[i], m[i]);
      up_inv[(size_t)(e - 1) * kMaxAlpha + r] = with_companion(inv_mod(prod, m[i]), m[i]);
      for (uint32_t t = 0; t < L + K; ++t) {
        uint32_t pt = 1;  // Q_D / q_i mod m_t
        for (uint32_t i2 = d0; i2 < e; ++i2)
          if (i2 != i) pt = mulm(pt, m[i2] % m[t], m[t]);
        up_conv[((size_t)(e - 1) * (L + K) + t) * kMaxAlpha + r] = with_companion(pt, m[t]);
      }
    }
  }
  std::vector<uint2> invp(kMaxK, make_uint2(0, 0)), dconv((size_t)L * kMaxK, make_uint2(0, 0)), pinv(L);
  for (uint32_t k = 0; k < K; ++k) {
    const uint32_t pk = m[L + k];
    uint32_t prod = 1;
    for (uint32_t k2 = 0; k2 < K; ++k2)
      if (k2 != k) prod = mulm(prod, m[L + k2] % pk, pk);
    invp[k] = with_companion(inv_mod(prod, pk), pk);
  }
  for (uint32_t i = 0; i < L; ++i) {
    const uint32_t qi = m[i];
    uint32_t P = 1;
    for (uint32_t k = 0; k < K; ++k) P = mulm(P, m[L + k] % qi, qi);
    pinv[i] = with_companion(inv_mod(P, qi), qi);
    for (uint32_t k = 0; k < K; ++k) {
      uint32_t prod = 1;
      for (uint32_t k2 = 0; k2 < K; ++k2)
        if (k2 != k) prod = mulm(prod, m[L + k2] % qi, qi);
      dconv[(size_t)i * kMaxK + k] = with_companion(prod, qi);
    }
  }
  // Matrix-core conversion operands: dword (j, r) of target t packs, for
  // d = 0..3, digit j of the balanced expansion of 2^{8d} C[t][r] 2^32 mod m_t.
  auto pack = [&](uint32_t C, uint32_t mt, int j) {
    const uint32_t c32 = mulm(C, (uint32_t)((1ull << 32) % mt), mt);
    uint32_t w = 0;
    for (int d = 0; d < 4; ++d) {
      const uint32_t v = mulm(c32, (uint32_t)((1ull << (8 * d)) % mt), mt);
      w |= ((balanced_digits(to_window(v, mt)) >> (8 * j)) & 0xFFu) << (8 * d);
    }
    return w;
  };
  std::vector<uint32_t> up_mfma((size_t)L * (L + K) * 32, 0), dn_mfma((size_t)L * 32, 0);
  for (uint32_t e = 1; e <= L; ++e) {
    const uint32_t d0 = A * ((e - 1) / A), nd = e - d0;
    for (uint32_t t = 0; t < L + K; ++t)
      for (int j = 0; j < 4; ++j)
        for (uint32_t r = 0; r < nd; ++r)
          up_mfma[((size_t)(e - 1) * (L + K) + t) * 32 + 8 * j + r] =
              pack(up_conv[((size_t)(e - 1) * (L + K) + t) * kMaxAlpha + r].x, m[t], j);
  }
  for (uint32_t i = 0; i < L; ++i)
    for (int j = 0; j < 4; ++j)
      for (uint32_t k = 0; k < K; ++k) dn_mfma[(size_t)i * 32 + 8 * j + k] = pack(dconv[(size_t)i * kMaxK + k].x, m[i], j);
  // offset corrections: 2^30 sum_r C[t][r] mod m_t
  const auto k30 = [&](uint32_t mt) { return (uint32_t)((1ull << 30) % mt); };
  c->h_up_k.assign((size_t)L * (L + K), 0);
  for (uint32_t e = 1; e <= L; ++e) {
    const uint32_t d0 = A * ((e - 1) / A), nd = e - d0;
    for (uint32_t t = 0; t < L + K; ++t) {
      uint32_t sum = 0;
      for (uint32_t r = 0; r < nd; ++r)
        sum = (uint32_t)(((uint64_t)sum + up_conv[((size_t)(e - 1) * (L + K) + t) * kMaxAlpha + r].x) % m[t]);
      c->h_up_k[(size_t)(e - 1) * (L + K) + t] = mulm(sum, k30(m[t]), m[t]);
    }
  }
  c->h_dn_k.assign(L, 0);
  for (uint32_t i = 0; i < L; ++i) {
    uint32_t sum = 0;
    for (uint32_t k = 0; k < K; ++k) sum = (uint32_t)(((uint64_t)sum + dconv[(size_t)i * kMaxK + k].x) % m[i]);
    c->h_dn_k[i] = mulm(sum, k30(m[i]), m[i]);
  }
  c->h_up_inv = up_inv;
  c->h_dn_invp = invp;
  c->h_mod.resize(L + K);
  for (uint32_t t = 0; t < L + K; ++t) c->h_mod[t] = make_modconst(m[t]);
  std::vector<uint2> rsq((size_t)L * L, make_uint2(0, 0));
  for (uint32_t t = 1; t < L; ++t)
    for (uint32_t i = 0; i < t; ++i)
      rsq[(size_t)t * L + i] = with_companion(inv_mod(m[t] % m[i], m[i]), m[i]);
  hipError_t e;
  if ((e = upload(&c->d_rs_qinv, rsq, c->owned)) != hipSuccess ||
      (e = upload(&c->d_up_mfma, up_mfma, c->owned)) != hipSuccess ||
      (e = upload(&c->d_dn_mfma, dn_mfma, c->owned)) != hipSuccess ||
      (e = upload(&c->d_up_inv, up_inv, c->owned)) != hipSuccess ||
      (e = upload(&c->d_up_conv, up_conv, c->owned)) != hipSuccess ||
      (e = upload(&c->d_dn_invp, invp, c->owned)) != hipSuccess ||
      (e = upload(&c->d_dn_conv, dconv, c->owned)) != hipSuccess ||
      (e = upload(&c->d_dn_pinv, pinv, c->owned)) != hipSuccess)
    return e == hipErrorOutOfMemory ? fail(TFHE_ENOMEM, "ckks constants: out of device memory")
                                    : hip_check(e, "ckks constants");
  return TFHE_OK;
}

static void ctx_free(tfhe_ckks_ctx_s* c) {
  for (void* p : c->owned) (void)hipFree(p);
  c->owned.clear();
  if (c->plan) tfhe_ntt_plan_destroy(c->plan);
  c->plan = nullptr;
}

static tfhe_status check_ct_call(const tfhe_ckks_ctx_s* c, uint32_t level, uint32_t batch, void* ws,
                                 size_t ws_bytes, bool ks_ws = true) {
  if (!c) return fail(TFHE_EINVAL, "null context");
  if (level < 1 || level > c->L) return fail(TFHE_EINVAL, "level must be in [1, L]");
  if ((uint64_t)batch * c->n * (c->L + c->K) > (1ull << 38)) return fail(TFHE_EINVAL, "batch too large");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->plan->device)
    return fail(TFHE_EINVAL, "the context's device is not the current device");
  if (batch == 0 || !ks_ws) return TFHE_OK;
  const size_t need = ks_layout(c, level, batch).total;
  if (!ws || ws_bytes < need) return fail(TFHE_EINVAL, "workspace missing or too small");
  if ((uintptr_t)ws % 256) return fail(TFHE_EINVAL, "workspace not 256-byte aligned");
  return TFHE_OK;
}

static bool al16(const void* p) { return p && ((uintptr_t)p % 16) == 0; }

}  // namespace tfhe

using namespace tfhe;

extern "C" {

tfhe_status tfhe_ckks_ctx_create(tfhe_ckks_ctx* out, uint32_t log_n, uint32_t L, uint32_t K,
                                 uint32_t dnum, const uint32_t* moduli, const uint32_t* psi,
                                 tfhe_ntt_algo algo) {
  if (!out) return fail(TFHE_EINVAL, "ckks_ctx_create: null out");
  *out = nullptr;
  if (L == 0 || K == 0 || dnum == 0 || L % dnum != 0)
    return fail(TFHE_EINVAL, "ckks_ctx_create: need L, K, dnum > 0 and dnum | L");
  if (L / dnum > (uint32_t)kMaxAlpha || K > (uint32_t)kMaxK)
    return fail(TFHE_EUNSUPPORTED, "ckks_ctx_create: alpha = L/dnum and K must be <= 8");
  std::vector<uint32_t> mods(L + K);
  if (moduli) {
    memcpy(mods.data(), moduli, sizeof(uint32_t) * (L + K));
  } else {
    std::vector<uint32_t> pr(L + K);
    tfhe_status st = tfhe_find_primes(31, 1ull << 17, L + K, pr.data());
    if (st != TFHE_OK) return st;
    for (uint32_t i = 0; i < L; ++i) mods[i] = pr[K + i];
    for (uint32_t k = 0; k < K; ++k) mods[L + k] = pr[k];
  }
  if (std::set<uint32_t>(mods.begin(), mods.end()).size() != mods.size())
    return fail(TFHE_ENOTNTT, "ckks_ctx_create: moduli must be distinct");
  tfhe_ckks_ctx_s* c = new (std::nothrow) tfhe_ckks_ctx_s();
  if (!c) return fail(TFHE_ENOMEM, "ckks_ctx_create: host allocation");
  c->log_n = log_n;
  c->n = 1u << log_n;
  c->L = L;
  c->K = K;
  c->dnum = dnum;
  c->alpha = L / dnum;
  tfhe_ntt_plan plan = nullptr;
  tfhe_status st = tfhe_ntt_plan_create(&plan, log_n, L + K, mods.data(), psi, algo);
  if (st != TFHE_OK) {
    delete c;
    return st;
  }
  c->plan = plan;
  if ((st = scratch_bind(plan->device)) != TFHE_OK || (st = ctx_build(c)) != TFHE_OK) {
    ctx_free(c);
    delete c;
    return st;
  }
  *out = c;
  return TFHE_OK;
}

tfhe_status tfhe_ckks_ctx_destroy(tfhe_ckks_ctx ctx) {
  if (!ctx) return TFHE_OK;
  ctx_free(ctx);
  delete ctx;
  return TFHE_OK;
}

tfhe_status tfhe_ckks_ctx_plan(tfhe_ckks_ctx ctx, tfhe_ntt_plan* plan) {
  if (!ctx || !plan) return fail(TFHE_EINVAL, "ckks_ctx_plan: null argument");
  *plan = ctx->plan;
  return TFHE_OK;
}

tfhe_status tfhe_hmult_workspace_size(tfhe_ckks_ctx ctx, uint32_t level, uint32_t batch,
                                      size_t* bytes) {
  if (!ctx || !bytes) return fail(TFHE_EINVAL, "hmult_workspace_size: null argument");
  if (level < 1 || level > ctx->L) return fail(TFHE_EINVAL, "level must be in [1, L]");
  *bytes = ks_layout(ctx, level, batch).total;
  return TFHE_OK;
}

}  // extern "C"

// The launch sequence of tfhe_hmult with a validated workspace.
static tfhe_status hmult_run(tfhe_ckks_ctx ctx, const uint32_t* ct_a, const uint32_t* ct_b,
                             uint32_t* ct_out, const uint32_t* evk, uint32_t level, uint32_t batch,
                             void* ws, tfhe_stream_t stream) {
  if (!al16(ct_a) || !al16(ct_b) || !al16(ct_out) || !al16(evk))
    return fail(TFHE_EINVAL, "hmult: null or unaligned pointer");
  hipStream_t s = (hipStream_t)stream;
  const uint64_t plane = (uint64_t)level * batch * ctx->n;
  unsigned char* w = (unsigned char*)ws;
  uint32_t* d2 = (uint32_t*)(w + ks_layout(ctx, level, batch).d2);
  hipError_t e = launch_tensor(ct_a, ct_b, ct_out, d2, ctx->plan->d_mod, level, batch, ctx->n, s);
  KeySet keys{};
  keys.count = 1;
  keys.k[0] = evk;
  if (e == hipSuccess)
    e = key_switch(ctx, d2, keys, ct_out, ct_out + plane, true, true, level, batch, w, s);
  return hip_check(e, "hmult");
}

extern "C" {

tfhe_status tfhe_hmult(tfhe_ckks_ctx ctx, const uint32_t* ct_a, const uint32_t* ct_b,
                       uint32_t* ct_out, const uint32_t* evk, uint32_t level, uint32_t batch,
                       void* ws, size_t ws_bytes, tfhe_stream_t stream) {
  tfhe_status st = check_ct_call(ctx, level, batch, ws, ws_bytes);
  if (st != TFHE_OK || batch == 0) return st;
  return hmult_run(ctx, ct_a, ct_b, ct_out, evk, level, batch, ws, stream);
}

tfhe_status tfhe_hmult_noalloc(tfhe_ckks_ctx ctx, const uint32_t* ct_a, const uint32_t* ct_b,
                               uint32_t* ct_out, const uint32_t* evk, uint32_t level,
                               uint32_t batch, tfhe_stream_t stream) {
  tfhe_status st = check_ct_call(ctx, level, batch, nullptr, 0, false);
  if (st != TFHE_OK || batch == 0) return st;
  const size_t need = ks_layout(ctx, level, batch).total;
  if (need > (size_t)TFHE_HMULT_NOALLOC_MAX_BYTES)
    return fail(TFHE_EINVAL, "hmult_noalloc: this level and batch need " + std::to_string(need) +
                                 " bytes of scratch, above TFHE_HMULT_NOALLOC_MAX_BYTES (" +
                                 std::to_string((size_t)TFHE_HMULT_NOALLOC_MAX_BYTES) +
                                 "); use a smaller batch or tfhe_hmult with a workspace");
  unsigned char* w = scratch_of(ctx->plan->device);
  if (!w) return fail(TFHE_EINVAL, "hmult_noalloc: scratch not bound on this device");
  return hmult_run(ctx, ct_a, ct_b, ct_out, evk, level, batch, w, stream);
}

tfhe_status tfhe_rotate(tfhe_ckks_ctx ctx, const uint32_t* ct_in, uint32_t* ct_out,
                        const uint32_t* rotkey, uint32_t galois_elt, uint32_t level, uint32_t batch,
                        void* ws, size_t ws_bytes, tfhe_stream_t stream) {
  tfhe_status st = check_ct_call(ctx, level, batch, ws, ws_bytes);
  if (st != TFHE_OK || batch == 0) return st;
  if (!al16(ct_in) || !al16(ct_out) || !al16(rotkey))
    return fail(TFHE_EINVAL, "rotate: null or unaligned pointer");
  if ((galois_elt & 1) == 0 || galois_elt >= 2 * ctx->n)
    return fail(TFHE_EINVAL, "rotate: galois element must be odd and < 2N");
  const uint64_t plane = (uint64_t)level * batch * ctx->n;
  if (ct_in < ct_out + 2 * plane && ct_out < ct_in + 2 * plane)
    return fail(TFHE_EINVAL, "rotate: ct_out must not alias ct_in");
  hipStream_t s = (hipStream_t)stream;
  unsigned char* w = (unsigned char*)ws;
  uint32_t* r1 = (uint32_t*)(w + ks_layout(ctx, level, batch).d2);
  GaloisSet gs{};
  gs.batch = 1;
  gs.g[0] = galois_elt;
  hipError_t e = launch_frobenius_pair(ct_in, ct_out, ct_in + plane, r1, gs, level * batch, ctx->log_n, s);
  KeySet keys{};
  keys.count = 1;
  keys.k[0] = rotkey;
  if (e == hipSuccess)
    e = key_switch(ctx, r1, keys, ct_out, ct_out + plane, true, false, level, batch, w, s);
  return hip_check(e, "rotate");
}

tfhe_status tfhe_rotate_multi(tfhe_ckks_ctx ctx, const uint32_t* ct_in, uint32_t* ct_out,
                              const uint32_t* const* rotkeys, const uint32_t* galois_elts,
                              uint32_t level, uint32_t batch, void* ws, size_t ws_bytes,
                              tfhe_stream_t stream) {
  tfhe_status st = check_ct_call(ctx, level, batch, ws, ws_bytes);
  if (st != TFHE_OK || batch == 0) return st;
  if (batch > kMaxRotBatch) return fail(TFHE_EINVAL, "rotate_multi: batch exceeds TFHE_ROTATE_MULTI_MAX");
  if (!rotkeys || !galois_elts) return fail(TFHE_EINVAL, "rotate_multi: null key or Galois array");
  if (!al16(ct_in) || !al16(ct_out)) return fail(TFHE_EINVAL, "rotate_multi: null or unaligned pointer");
  KeySet keys{};
  GaloisSet gs{};
  keys.count = gs.batch = batch;
  for (uint32_t b = 0; b < batch; ++b) {
    if (!al16(rotkeys[b])) return fail(TFHE_EINVAL, "rotate_multi: null or unaligned rotation key");
    if ((galois_elts[b] & 1) == 0 || galois_elts[b] >= 2 * ctx->n)
      return fail(TFHE_EINVAL, "rotate_multi: galois elements must be odd and < 2N");
    keys.k[b] = rotkeys[b];
    gs.g[b] = galois_elts[b];
  }
  const uint64_t plane = (uint64_t)level * batch * ctx->n;
  if (ct_in < ct_out + 2 * plane && ct_out < ct_in + 2 * plane)
    return fail(TFHE_EINVAL, "rotate_multi: ct_out must not alias ct_in");
  hipStream_t s = (hipStream_t)stream;
  unsigned char* w = (unsigned char*)ws;
  uint32_t* r1 = (uint32_t*)(w + ks_layout(ctx, level, batch).d2);
  hipError_t e = launch_frobenius_pair(ct_in, ct_out, ct_in + plane, r1, gs, level * batch, ctx->log_n, s);
  if (e == hipSuccess)
    e = key_switch(ctx, r1, keys, ct_out, ct_out + plane, true, false, level, batch, w, s);
  return hip_check(e, "rotate_multi");
}

tfhe_status tfhe_rescale_workspace_size(tfhe_ckks_ctx ctx, uint32_t level, uint32_t batch,
                                        size_t* bytes) {
  if (!ctx || !bytes) return fail(TFHE_EINVAL, "rescale_workspace_size: null argument");
  if (level < 2 || level > ctx->L) return fail(TFHE_EINVAL, "rescale: level must be in [2, L]");
  *bytes = rs_layout(ctx, level, batch).total;
  return TFHE_OK;
}

tfhe_status tfhe_rescale(tfhe_ckks_ctx ctx, const uint32_t* ct_in, uint32_t* ct_out, uint32_t level,
                         uint32_t batch, void* ws, size_t ws_bytes, tfhe_stream_t stream) {
  tfhe_status st = check_ct_call(ctx, level, batch, nullptr, 0, false);
  if (st != TFHE_OK) return st;
  if (level < 2) return fail(TFHE_EINVAL, "rescale: level must be in [2, L]");
  if (batch == 0) return TFHE_OK;
  if (!al16(ct_in) || !al16(ct_out)) return fail(TFHE_EINVAL, "rescale: null or unaligned pointer");
  const uint64_t plane = (uint64_t)batch * ctx->n;
  if (ct_in < ct_out + 2 * (level - 1) * plane && ct_out < ct_in + 2 * level * plane)
    return fail(TFHE_EINVAL, "rescale: ct_out must not alias ct_in");
  const size_t need = rs_layout(ctx, level, batch).total;
  if (!ws || ws_bytes < need) return fail(TFHE_EINVAL, "rescale: workspace missing or too small");
  if ((uintptr_t)ws % 256) return fail(TFHE_EINVAL, "rescale: workspace not 256-byte aligned");
  return hip_check(rescale(ctx, ct_in, ct_out, level, batch, (unsigned char*)ws, (hipStream_t)stream),
                   "rescale");
}

tfhe_status tfhe_cmult(tfhe_ckks_ctx ctx, const uint32_t* ct, const uint32_t* pt, uint32_t* ct_out,
                       uint32_t level, uint32_t batch, tfhe_stream_t stream) {
  tfhe_status st = check_ct_call(ctx, level, batch, nullptr, 0, false);
  if (st != TFHE_OK || batch == 0) return st;
  if (!al16(ct) || !al16(pt) || !al16(ct_out)) return fail(TFHE_EINVAL, "cmult: null or unaligned pointer");
  const uint64_t plane = (uint64_t)level * batch * ctx->n;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = ew_launch(EW_MUL, ctx->plan->d_mod, ct, pt, ct_out, level, batch, ctx->n, s);
  if (e == hipSuccess) e = ew_launch(EW_MUL, ctx->plan->d_mod, ct + plane, pt, ct_out + plane, level, batch, ctx->n, s);
  return hip_check(e, "cmult");
}

tfhe_status tfhe_hadd(tfhe_ckks_ctx ctx, const uint32_t* ct_a, const uint32_t* ct_b, uint32_t* ct_out,
                      uint32_t level, uint32_t batch, tfhe_stream_t stream) {
  tfhe_status st = check_ct_call(ctx, level, batch, nullptr, 0, false);
  if (st != TFHE_OK || batch == 0) return st;
  if (!al16(ct_a) || !al16(ct_b) || !al16(ct_out)) return fail(TFHE_EINVAL, "hadd: null or unaligned pointer");
  const uint64_t plane = (uint64_t)level * batch * ctx->n;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = ew_launch(EW_ADD, ctx->plan->d_mod, ct_a, ct_b, ct_out, level, batch, ctx->n, s);
  if (e == hipSuccess)
    e = ew_launch(EW_ADD, ctx->plan->d_mod, ct_a + plane, ct_b + plane, ct_out + plane, level, batch, ctx->n, s);
  return hip_check(e, "hadd");
}

}  // extern "C"
