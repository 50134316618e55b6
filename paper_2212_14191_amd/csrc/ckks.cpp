// RNS-CKKS context and the HMULT / HROTATE operations (Sec. II-B, Sec. IV-A,
// Table 2) as stream-ordered kernel sequences on the device.
//
// Key switching follows the hybrid method the paper adopts (Sec. II-B,
// "Generalized Key-Switching"): Dcomp splits the limbs of the input into
// digits of alpha = L/dnum limbs, ModUp extends each digit to Q_l * P by fast
// basis conversion (no overflow correction), the inner product with the key
// accumulates over the digits, and ModDown divides by P (no rounding offset).
#include <string.h>

#include <algorithm>
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
// product (ip_run): four-step plans unless TFHE_PARAM_KS_INNER asks for the
// separate kernels (2).
static bool fused_inner(const tfhe_ckks_ctx_s* c) {
  return c->plan->algo == TFHE_NTT_FOURSTEP_MFMA && c->plan->ks_inner != 2;
}

// Workspace of one key-switching batch: its own regions (byte offsets from
// the batch's base) and the workspace of its four fused transforms.
struct KsLayout {
  size_t d2, x, up, acc, tp, conv;
  size_t own;       // the own regions' total
  size_t stage[4];  // INTT of the input; ModUp NTTs; ModDown INTTs; final NTTs
  size_t inter;     // fused inner product: the ModUp intermediates (inside stage 1)
  size_t ntt, total;  // the batch alone: transform region after the own ones
};

static KsLayout ks_layout(const tfhe_ckks_ctx_s* c, uint32_t level, uint32_t batch) {
  const size_t plane = (size_t)batch * c->n * sizeof(uint32_t);
  const uint32_t digits = (level + c->alpha - 1) / c->alpha;
  const uint32_t ext = level + c->K;
  // Each transform's region holds its units' slices, each rounded to 256
  // bytes as fs_run_units / bf_run_units lay them out: INTT of the input
  // (level limbs); the NTT of every digit's converted limbs; the INTT of
  // both accumulators' K special limbs; the final NTT of both components
  // (2 x level limbs).
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
  KsLayout l;
  // with the fused second pass + inner product, the ModUp transforms'
  // intermediates sit in a regular [digits][level + K] array of planes
  l.inter = fused_inner(c) ? align256(plane * (size_t)digits * ext) : 0;
  l.stage[0] = ws(level);
  l.stage[1] = std::max(modup, l.inter);
  l.stage[2] = 2 * ws(c->K);
  l.stage[3] = 2 * ws(level);
  size_t off = 0;
  l.d2 = off; off += align256(plane * level);
  l.x = off; off += align256(plane * level);
  l.up = off; off += align256(plane * (size_t)digits * ext);
  l.acc = off; off += align256(plane * 2 * ext);
  l.tp = off; off += align256(plane * 2 * c->K);
  l.conv = off; off += align256(plane * 2 * level);
  l.own = off;
  l.ntt = off;
  l.total = off + align256(*std::max_element(l.stage, l.stage + 4));
  return l;
}

// ModUp conversion of digit [d0, d0 + nd) on the matrix cores: every
// extended-basis position outside the digit, in descriptors of <= 32 targets.
static void modup_mfma(const uint32_t* x, uint32_t* up, uint32_t key_idx, uint32_t d0, uint32_t nd,
                       uint32_t level, uint32_t K, uint64_t plane, ConvQueue& cq) {
  const uint32_t targets = level + K - nd;  // every extended-basis position outside the digit
  for (uint32_t first = 0; first < targets; first += kConvMaxOut)
    cq.q.push_back(ConvDesc{x + (uint64_t)d0 * plane, up, plane, nd,
                            std::min<uint32_t>(kConvMaxOut, targets - first), first, key_idx, d0, level});
}

// ModDown conversion of the K special limbs to the level q-limbs.
static void moddown_conv_mfma(const uint32_t* tp, uint32_t* conv, uint32_t level, uint32_t K, uint64_t plane,
                              ConvQueue& cq) {
  for (uint32_t first = 0; first < level; first += kConvMaxOut)
    cq.q.push_back(ConvDesc{tp, conv, plane, K, std::min<uint32_t>(kConvMaxOut, level - first), first, kConvDown,
                            0, level});
}

static ConvTabs conv_tabs(const tfhe_ckks_ctx_s* c) {
  return ConvTabs{c->plan->d_mod, c->d_up_inv, c->d_dn_invp, c->d_up_k, c->d_dn_k, c->d_up_mfma, c->d_dn_mfma,
                  c->L, c->K};
}

// One batch of a key switch: d (NTT domain, [level][batch][N]);
// out0 (+)= ModDown(acc0), out1 (+)= ModDown(acc1).  own: the batch's
// regions (KsLayout offsets); key0: its element 0's index in the key set.
struct KsJob {
  const uint32_t* d;
  uint32_t key0;
  uint32_t *out0, *out1;
  bool add0, add1;
  uint32_t level, batch;
  unsigned char* own;
};

// Key switching of several batches (of different levels) with every
// transform, basis conversion and inner product launched once for all of
// them.  keys [dnum][2][L+K][N]: one for every element (count 1) or one per
// element, batch g's from jobs[g].key0.  nws: the transforms' region, at
// least the largest over the four stages of the batches' stage sums (the
// fused inner product's intermediates of batch g at the sum of stage 1
// before it).
static hipError_t key_switch_multi(const tfhe_ckks_ctx_s* c, const KsJob* jobs, uint32_t nj, const KeySet& keys,
                                   unsigned char* nws, hipStream_t s) {
  if (nj > (uint32_t)kMaxIpGroups) return hipErrorInvalidValue;
  const tfhe_ntt_plan_s* p = c->plan;
  const bool fused = fused_inner(c);
  struct Ptrs {
    uint32_t *x, *up, *acc, *tp, *conv, *inter;
    uint64_t plane;
    uint32_t ext, digits;
  };
  std::vector<Ptrs> w(nj);
  size_t inter_off = 0;
  bool mfma_conv = true;  // matrix-core conversion needs planes in whole 64-word chunks
  for (uint32_t g = 0; g < nj; ++g) {
    const KsJob& j = jobs[g];
    const KsLayout lay = ks_layout(c, j.level, j.batch);
    w[g] = Ptrs{(uint32_t*)(j.own + lay.x),   (uint32_t*)(j.own + lay.up),   (uint32_t*)(j.own + lay.acc),
                (uint32_t*)(j.own + lay.tp),  (uint32_t*)(j.own + lay.conv), (uint32_t*)(nws + inter_off),
                (uint64_t)j.batch * c->n,     j.level + c->K,                (j.level + c->alpha - 1) / c->alpha};
    inter_off += lay.stage[1];
    mfma_conv = mfma_conv && w[g].plane % 64 == 0;
  }
  hipError_t e;
  // INTT of the inputs (coefficient domain for the basis conversion)
  std::vector<NttUnit> units;
  for (uint32_t g = 0; g < nj; ++g)
    units.push_back(NttUnit{p, true, jobs[g].d, w[g].x, 0, jobs[g].level, jobs[g].batch});
  if ((e = ntt_units(p, units, nws, s)) != hipSuccess) return e;
  // Dcomp + ModUp of every digit, then one fused NTT of all converted limbs:
  // the q-limbs before and after the digit, and the p-limbs.  Fused: the
  // transforms' first pass writes digit j's intermediate of position pos at
  // inter + (j ext + pos) plane; ip_run finishes them.
  units.clear();
  ConvQueue cq;  // the matrix-core conversions, launched together
  cq.tabs = conv_tabs(c);
  for (uint32_t g = 0; g < nj; ++g) {
    const uint32_t level = jobs[g].level, batch = jobs[g].batch, ext = w[g].ext;
    const uint64_t plane = w[g].plane;
    for (uint32_t j = 0; j < w[g].digits; ++j) {
      const uint32_t d0 = c->alpha * j, nd = std::min(c->alpha, level - d0);
      const uint32_t key_idx = d0 + nd - 1;
      uint32_t* upj = w[g].up + (uint64_t)j * ext * plane;
      if (mfma_conv)
        modup_mfma(w[g].x, upj, key_idx, d0, nd, level, c->K, plane, cq);
      else if ((e = launch_modup(w[g].x, upj, p->d_mod, c->d_up_inv + (size_t)key_idx * kMaxAlpha,
                                 c->d_up_conv + (size_t)key_idx * (c->L + c->K) * kMaxAlpha, d0, nd, level,
                                 c->L, c->K, batch, c->n, s)) != hipSuccess)
        return e;
      uint32_t* outj = fused ? w[g].inter + (uint64_t)j * ext * plane : upj;
      auto unit = [&](uint32_t pos, uint32_t limb_begin, uint32_t count) {
        NttUnit u{p, false, upj + (uint64_t)pos * plane, outj + (uint64_t)pos * plane, limb_begin, count, batch};
        u.pass1_only = fused;
        units.push_back(u);
      };
      if (d0) unit(0, 0, d0);
      if (level > d0 + nd) unit(d0 + nd, d0 + nd, level - d0 - nd);
      unit(level, c->L, c->K);
    }
  }
  if ((e = cq.flush(p->num_cus, K_MODUP, s)) != hipSuccess) return e;
  if ((e = ntt_units(p, units, nws, s)) != hipSuccess) return e;
  IpSet ip{};
  ip.count = nj;
  ip.L = c->L;
  ip.K = c->K;
  ip.alpha = c->alpha;
  ip.keys = keys;
  for (uint32_t g = 0; g < nj; ++g)
    ip.g[g] = IpGroup{fused ? w[g].inter : w[g].up, jobs[g].d, w[g].acc, jobs[g].level, jobs[g].batch,
                      w[g].digits, jobs[g].key0, 0};
  if ((e = fused ? ip_run(p, ip, s) : launch_inner_product(ip, p->d_mod, c->log_n, s)) != hipSuccess) return e;
  // ModDown of both accumulators, their transforms fused
  units.clear();
  for (uint32_t g = 0; g < nj; ++g) {
    const uint64_t plane = w[g].plane;
    const uint32_t level = jobs[g].level, batch = jobs[g].batch;
    uint32_t* a1 = w[g].acc + (uint64_t)w[g].ext * plane;
    units.push_back(NttUnit{p, true, w[g].acc + (uint64_t)level * plane, w[g].tp, c->L, c->K, batch});
    units.push_back(NttUnit{p, true, a1 + (uint64_t)level * plane, w[g].tp + (uint64_t)c->K * plane, c->L, c->K, batch});
  }
  if ((e = ntt_units(p, units, nws, s)) != hipSuccess) return e;
  for (uint32_t g = 0; g < nj; ++g) {
    const uint64_t plane = w[g].plane;
    const uint32_t level = jobs[g].level;
    for (int comp = 0; comp < 2; ++comp) {
      const uint32_t* tpc = w[g].tp + (comp ? (uint64_t)c->K * plane : 0);
      uint32_t* convc = w[g].conv + (comp ? (uint64_t)level * plane : 0);
      if (mfma_conv)
        moddown_conv_mfma(tpc, convc, level, c->K, plane, cq);
      else if ((e = launch_moddown_conv(tpc, convc, p->d_mod, c->d_dn_invp, c->d_dn_conv, level, c->L, c->K,
                                        jobs[g].batch, c->n, s)) != hipSuccess)
        return e;
    }
  }
  if ((e = cq.flush(p->num_cus, K_MD_CONV, s)) != hipSuccess) return e;
  units.clear();
  for (uint32_t g = 0; g < nj; ++g) {
    const KsJob& j = jobs[g];
    const uint64_t plane = w[g].plane;
    uint32_t* conv1 = w[g].conv + (uint64_t)j.level * plane;
    uint32_t* a1 = w[g].acc + (uint64_t)w[g].ext * plane;
    if (p->algo == TFHE_NTT_FOURSTEP_MFMA) {
      // the transform's second pass finishes ModDown in its store epilogue:
      // out (+)= (acc - NTT(conv)) P^{-1}
      NttUnit u0{p, false, w[g].conv, j.out0, 0, j.level, j.batch};
      NttUnit u1{p, false, conv1, j.out1, 0, j.level, j.batch};
      u0.acc = w[g].acc;
      u1.acc = a1;
      u0.epi_mult = u1.epi_mult = c->d_dn_pinv;
      u0.epi_add = j.add0;
      u1.epi_add = j.add1;
      units.push_back(u0);
      units.push_back(u1);
    } else {
      units.push_back(NttUnit{p, false, w[g].conv, w[g].conv, 0, j.level, j.batch});
      units.push_back(NttUnit{p, false, conv1, conv1, 0, j.level, j.batch});
    }
  }
  if ((e = ntt_units(p, units, nws, s)) != hipSuccess) return e;
  if (p->algo == TFHE_NTT_FOURSTEP_MFMA) return hipSuccess;
  for (uint32_t g = 0; g < nj; ++g) {
    const KsJob& j = jobs[g];
    const uint64_t plane = w[g].plane;
    for (int comp = 0; comp < 2; ++comp)
      if ((e = launch_moddown_final(w[g].acc + (comp ? (uint64_t)w[g].ext * plane : 0),
                                    w[g].conv + (comp ? (uint64_t)j.level * plane : 0), comp ? j.out1 : j.out0,
                                    p->d_mod, c->d_dn_pinv, j.level, j.batch, c->n, comp ? j.add1 : j.add0, s)) !=
          hipSuccess)
        return e;
  }
  return hipSuccess;
}

// Key switching of one batch with workspace ws (ks_layout(level, batch)).
static hipError_t key_switch(const tfhe_ckks_ctx_s* c, const uint32_t* d, const KeySet& keys,
                             uint32_t* out0, uint32_t* out1, bool acc0_add, bool acc1_add,
                             uint32_t level, uint32_t batch, unsigned char* ws, hipStream_t s) {
  const KsJob job{d, 0, out0, out1, acc0_add, acc1_add, level, batch, ws};
  return key_switch_multi(c, &job, 1, keys, ws + ks_layout(c, level, batch).ntt, s);
}

// Groups of a mixed batch: request indices sorted by (level, op) (stable),
// and the workspace layout (per group its result staging [2][level][B][N]
// and its own key-switching regions; then the transforms' region shared by
// all groups).
static_assert(TFHE_HMULT_LEVELS_MAX == kMaxRotBatch, "one bound for mixed-level batches");

struct LvPlan {
  std::vector<uint32_t> order;                 // request indices by level
  std::vector<std::pair<uint32_t, uint32_t>> groups;  // [begin, end) in order
  std::vector<size_t> staging, own;            // byte offsets per group
  size_t ntt = 0, total = 0;
};

static LvPlan lv_plan(const tfhe_ckks_ctx_s* c, const LvReq* r, uint32_t count) {
  LvPlan l;
  l.order.resize(count);
  for (uint32_t i = 0; i < count; ++i) l.order[i] = i;
  std::stable_sort(l.order.begin(), l.order.end(), [&](uint32_t x, uint32_t y) {
    return r[x].level != r[y].level ? r[x].level < r[y].level : r[x].op < r[y].op;
  });
  for (uint32_t i = 0; i < count;) {
    uint32_t j = i;
    while (j < count && r[l.order[j]].level == r[l.order[i]].level && r[l.order[j]].op == r[l.order[i]].op) ++j;
    l.groups.emplace_back(i, j);
    i = j;
  }
  size_t off = 0, stage[4] = {0, 0, 0, 0};
  for (auto& g : l.groups) {
    const uint32_t level = r[l.order[g.first]].level, B = g.second - g.first;
    const KsLayout lay = ks_layout(c, level, B);
    l.staging.push_back(off);
    off += align256((size_t)2 * level * B * c->n * sizeof(uint32_t));
    l.own.push_back(off);
    off += lay.own;
    for (int k = 0; k < 4; ++k) stage[k] += lay.stage[k];
  }
  l.ntt = off;
  l.total = off + align256(*std::max_element(stage, stage + 4));
  return l;
}

size_t levels_ws_bytes(const tfhe_ckks_ctx_s* c, const LvReq* r, uint32_t count) {
  return count ? lv_plan(c, r, count).total : 0;
}

hipError_t levels_run(const tfhe_ckks_ctx_s* c, const LvReq* r, uint32_t count, unsigned char* ws,
                      hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (count > kMaxRotBatch) return hipErrorInvalidValue;
  const LvPlan l = lv_plan(c, r, count);
  std::vector<KsJob> jobs;
  ScatterSet sc{};
  CtDescSet cs[2] = {};  // the HMULTs' tensor products, the rotations' Frobenius maps
  KeySet keys{};
  bool same = true;  // one operation and key (and Galois element) for the whole batch
  for (uint32_t i = 0; i < count; ++i)
    same = same && r[i].op == r[0].op && r[i].key == r[0].key && (r[i].op == 0 || r[i].galois == r[0].galois);
  keys.count = same ? 1 : count;
  for (size_t g = 0; g < l.groups.size(); ++g) {
    const uint32_t b0 = l.groups[g].first, B = l.groups[g].second - b0;
    const uint32_t level = r[l.order[b0]].level, op = r[l.order[b0]].op ? 1 : 0;
    const KsLayout lay = ks_layout(c, level, B);
    uint32_t* stg = (uint32_t*)(ws + l.staging[g]);
    unsigned char* own = ws + l.own[g];
    uint32_t* d = (uint32_t*)(own + lay.d2);
    const uint64_t plane = (uint64_t)level * B * c->n;
    for (uint32_t k = 0; k < B; ++k) {
      const LvReq& q = r[l.order[b0 + k]];
      keys.k[same ? 0 : b0 + k] = q.key;
      cs[op].c[cs[op].count++] = CtDesc{q.a, q.b, stg, d, level, B, k, q.galois};
      sc.src[b0 + k] = stg;
      sc.dst[b0 + k] = q.out;
      sc.rows[b0 + k] = 2 * level;
      sc.batch[b0 + k] = B;
      sc.b[b0 + k] = k;
    }
    jobs.push_back(KsJob{d, b0, stg, stg + plane, true, op == 0, level, B, own});
  }
  // every input is read here, before any result is written (by the final
  // copies): a result may alias any request's input
  hipError_t e = launch_tensor_multi(cs[0], c->plan->d_mod, c->log_n, s);
  if (e == hipSuccess) e = launch_frobenius_multi(cs[1], c->log_n, s);
  if (e != hipSuccess) return e;
  if ((e = key_switch_multi(c, jobs.data(), (uint32_t)jobs.size(), keys, ws + l.ntt, s)) != hipSuccess) return e;
  return launch_scatter(sc, count, c->log_n, s);
}

// RESCALE workspace: the top limbs in the coefficient domain [2][B][N], their
// broadcast to the remaining limbs [2][top][B][N] (butterfly contexts; the
// four-step transform reads the top limbs directly), the transforms'
// workspace.
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
  l.u = off; off += mfma ? 0 : align256(2 * plane * top);  // the broadcast (butterfly path only)
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
  if (p->algo == TFHE_NTT_FOURSTEP_MFMA) {
    // NTT of the top limb's coefficients modulo every remaining limb (each
    // limb's first pass reads the same plane of t, whose values lie below
    // 2^31), finished in the store epilogue: (c_i - NTT(t)_i) q_top^{-1}
    NttUnit u0{p, false, t, out, 0, top, batch};
    NttUnit u1{p, false, t + plane, out + (uint64_t)top * plane, 0, top, batch};
    u0.in_bcast = u1.in_bcast = true;
    u0.acc = ct;
    u1.acc = ct + (uint64_t)level * plane;
    u0.epi_mult = u1.epi_mult = c->d_rs_qinv + (size_t)top * c->L;
    return ntt_units(p, {u0, u1}, nws, s);
  }
  // reduce into every remaining limb, back to the NTT domain
  if ((e = launch_rescale_bcast(t, u, p->d_mod, top, batch, c->n, s)) != hipSuccess) return e;
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
  std::vector<uint32_t> up_k((size_t)L * (L + K), 0), dn_k(L, 0);
  for (uint32_t e = 1; e <= L; ++e) {
    const uint32_t d0 = A * ((e - 1) / A), nd = e - d0;
    for (uint32_t t = 0; t < L + K; ++t) {
      uint32_t sum = 0;
      for (uint32_t r = 0; r < nd; ++r)
        sum = (uint32_t)(((uint64_t)sum + up_conv[((size_t)(e - 1) * (L + K) + t) * kMaxAlpha + r].x) % m[t]);
      up_k[(size_t)(e - 1) * (L + K) + t] = mulm(sum, k30(m[t]), m[t]);
    }
  }
  for (uint32_t i = 0; i < L; ++i) {
    uint32_t sum = 0;
    for (uint32_t k = 0; k < K; ++k) sum = (uint32_t)(((uint64_t)sum + dconv[(size_t)i * kMaxK + k].x) % m[i]);
    dn_k[i] = mulm(sum, k30(m[i]), m[i]);
  }
  std::vector<uint2> rsq((size_t)L * L, make_uint2(0, 0));
  for (uint32_t t = 1; t < L; ++t)
    for (uint32_t i = 0; i < t; ++i)
      rsq[(size_t)t * L + i] = with_companion(inv_mod(m[t] % m[i], m[i]), m[i]);
  hipError_t e;
  if ((e = upload(&c->d_rs_qinv, rsq, c->owned)) != hipSuccess ||
      (e = upload(&c->d_up_mfma, up_mfma, c->owned)) != hipSuccess ||
      (e = upload(&c->d_dn_mfma, dn_mfma, c->owned)) != hipSuccess ||
      (e = upload(&c->d_up_k, up_k, c->owned)) != hipSuccess ||
      (e = upload(&c->d_dn_k, dn_k, c->owned)) != hipSuccess ||
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

tfhe_status tfhe_hmult_levels_workspace_size(tfhe_ckks_ctx ctx, const uint32_t* levels, uint32_t count,
                                             size_t* bytes) {
  if (!ctx || !bytes || (count && !levels)) return fail(TFHE_EINVAL, "hmult_levels_workspace_size: null argument");
  if (count > kMaxRotBatch) return fail(TFHE_EINVAL, "hmult_levels: count exceeds TFHE_HMULT_LEVELS_MAX");
  std::vector<LvReq> r(count);
  for (uint32_t i = 0; i < count; ++i) {
    if (levels[i] < 1 || levels[i] > ctx->L) return fail(TFHE_EINVAL, "level must be in [1, L]");
    r[i].level = levels[i];
  }
  *bytes = levels_ws_bytes(ctx, r.data(), count);
  return TFHE_OK;
}

// Checks of a mixed-level call shared by tfhe_hmult_levels and
// tfhe_rotate_levels (r filled in by the caller).
static tfhe_status check_levels_call(tfhe_ckks_ctx ctx, const std::vector<LvReq>& r, void* ws, size_t ws_bytes,
                                     const char* what) {
  const uint32_t count = (uint32_t)r.size();
  for (uint32_t i = 0; i < count; ++i) {
    if (r[i].level < 1 || r[i].level > ctx->L) return fail(TFHE_EINVAL, "level must be in [1, L]");
    if (!al16(r[i].a) || !al16(r[i].out) || !al16(r[i].key) || (r[i].b && !al16(r[i].b)))
      return fail(TFHE_EINVAL, std::string(what) + ": null or unaligned ciphertext or key");
  }
  // results must not overlap one another (each may alias any input)
  const size_t limb = (size_t)ctx->n * sizeof(uint32_t);
  for (uint32_t i = 0; i < count; ++i)
    for (uint32_t j = i + 1; j < count; ++j) {
      const char *p = (const char*)r[i].out, *q = (const char*)r[j].out;
      if (p < q + 2 * r[j].level * limb && q < p + 2 * r[i].level * limb)
        return fail(TFHE_EINVAL, std::string(what) + ": result buffers overlap");
    }
  const size_t need = levels_ws_bytes(ctx, r.data(), count);
  if (!ws || ws_bytes < need) return fail(TFHE_EINVAL, "workspace missing or too small");
  if ((uintptr_t)ws % 256) return fail(TFHE_EINVAL, "workspace not 256-byte aligned");
  return TFHE_OK;
}

tfhe_status tfhe_hmult_levels(tfhe_ckks_ctx ctx, const uint32_t* const* ct_a, const uint32_t* const* ct_b,
                              uint32_t* const* ct_out, const uint32_t* levels, uint32_t count,
                              const uint32_t* evk, void* ws, size_t ws_bytes, tfhe_stream_t stream) {
  tfhe_status st = check_ct_call(ctx, 1, 1, nullptr, 0, false);
  if (st != TFHE_OK || count == 0) return st;
  if (count > kMaxRotBatch) return fail(TFHE_EINVAL, "hmult_levels: count exceeds TFHE_HMULT_LEVELS_MAX");
  if (!ct_a || !ct_b || !ct_out || !levels) return fail(TFHE_EINVAL, "hmult_levels: null array");
  if (!al16(evk)) return fail(TFHE_EINVAL, "hmult_levels: null or unaligned evk");
  std::vector<LvReq> r(count);
  for (uint32_t i = 0; i < count; ++i) {
    if (!ct_b[i]) return fail(TFHE_EINVAL, "hmult_levels: null ciphertext");
    r[i] = LvReq{ct_a[i], ct_b[i], ct_out[i], evk, levels[i], 0, 0};
  }
  if ((st = check_levels_call(ctx, r, ws, ws_bytes, "hmult_levels")) != TFHE_OK) return st;
  return hip_check(levels_run(ctx, r.data(), count, (unsigned char*)ws, (hipStream_t)stream), "hmult_levels");
}

tfhe_status tfhe_rotate_levels(tfhe_ckks_ctx ctx, const uint32_t* const* ct_in, uint32_t* const* ct_out,
                               const uint32_t* const* rotkeys, const uint32_t* galois_elts, const uint32_t* levels,
                               uint32_t count, void* ws, size_t ws_bytes, tfhe_stream_t stream) {
  tfhe_status st = check_ct_call(ctx, 1, 1, nullptr, 0, false);
  if (st != TFHE_OK || count == 0) return st;
  if (count > kMaxRotBatch) return fail(TFHE_EINVAL, "rotate_levels: count exceeds TFHE_HMULT_LEVELS_MAX");
  if (!ct_in || !ct_out || !rotkeys || !galois_elts || !levels) return fail(TFHE_EINVAL, "rotate_levels: null array");
  std::vector<LvReq> r(count);
  for (uint32_t i = 0; i < count; ++i) {
    if ((galois_elts[i] & 1) == 0 || galois_elts[i] >= 2 * ctx->n)
      return fail(TFHE_EINVAL, "rotate_levels: galois elements must be odd and < 2N");
    r[i] = LvReq{ct_in[i], nullptr, ct_out[i], rotkeys[i], levels[i], galois_elts[i], 1};
  }
  if ((st = check_levels_call(ctx, r, ws, ws_bytes, "rotate_levels")) != TFHE_OK) return st;
  return hip_check(levels_run(ctx, r.data(), count, (unsigned char*)ws, (hipStream_t)stream), "rotate_levels");
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
