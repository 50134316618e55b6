// RNS-CKKS context state and the launchers of ckks_kernels.hip.
#pragma once
#include "internal.hpp"

namespace tfhe {

constexpr int kMaxAlpha = 8;  // limbs per key-switching digit
constexpr int kMaxK = 8;      // special primes

struct CkksCtxImpl {
  uint32_t log_n = 0, n = 0, L = 0, K = 0, dnum = 0, alpha = 0;
  tfhe_ntt_plan_s* plan = nullptr;  // over q_0..q_{L-1}, p_0..p_{K-1}
  // ModUp constants of digit D = [alpha*j, e), indexed by e-1 in [0, L):
  uint2* d_up_inv = nullptr;   // [L][kMaxAlpha]        [(Q_D/q_i)^{-1}]_{q_i}
  uint2* d_up_conv = nullptr;  // [L][L+K][kMaxAlpha]   [Q_D/q_i]_{t}
  // ModDown constants:
  uint2* d_dn_invp = nullptr;  // [kMaxK]               [(P/p_k)^{-1}]_{p_k}
  uint2* d_dn_conv = nullptr;  // [L][kMaxK]            [P/p_k]_{q_i}
  uint2* d_dn_pinv = nullptr;  // [L]                   [P^{-1}]_{q_i}
  // RESCALE constants:
  uint2* d_rs_qinv = nullptr;  // [L][L]                [q_t^{-1}]_{q_i} at row t
  // Matrix-core basis conversion operands (32 dwords per target):
  uint32_t* d_up_mfma = nullptr;  // [L (digit end - 1)][L+K (target)][4][8]
  uint32_t* d_dn_mfma = nullptr;  // [L (target)][4][8]
  // their offset constants 2^30 sum_r C[t][r] mod m_t
  uint32_t* d_up_k = nullptr;     // [L (digit end - 1)][L+K (target)]
  uint32_t* d_dn_k = nullptr;     // [L (target)]
  std::vector<void*> owned;
};

// Basis conversion on the matrix cores: out_t = sum_r y_r C[t][r] mod m_t
// with y_r = in_r * mult_r mod q_r in [0, q_r) (the integer itself matters:
// q_r != m_t), for up to 8 inputs and 32 targets.
constexpr int kConvMaxIn = 8, kConvMaxOut = 32;
constexpr uint32_t kConvDown = 0xFFFFFFFFu;  // ConvDesc::key_idx of a ModDown conversion
// One conversion: inputs at in + r plane (r < nin); targets u = first ..
// first + nout - 1 (nout <= kConvMaxOut) of its list, target u written to
// out + conv_pos(u) plane.  ModUp of the digit [d0, d0 + nin) (key_idx: the
// row of its constants, the digit's last limb): the list is the extended-
// basis positions 0 .. level + K - 1 without the digit.  ModDown (key_idx
// kConvDown): the positions 0 .. level - 1, from the K special limbs.  The
// moduli, multipliers and matrix operands come from the context's tables
// (ConvSet), so a descriptor is small and one launch takes many.
struct ConvDesc {
  const uint32_t* in;
  uint32_t* out;
  uint64_t plane;  // words per plane (batch * N), a multiple of 64
  uint32_t nin, nout, first, key_idx, d0, level;
};
TFHE_HD uint32_t conv_pos(const ConvDesc& a, uint32_t u) {
  return a.key_idx != kConvDown && u >= a.d0 ? u + a.nin : u;
}

hipError_t launch_tensor(const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t* d2,
                         const ModConst* mods, uint32_t level, uint32_t batch, uint32_t n,
                         hipStream_t s);
hipError_t launch_modup(const uint32_t* x, uint32_t* up, const ModConst* mods, const uint2* inv,
                        const uint2* conv, uint32_t d0, uint32_t nd, uint32_t level, uint32_t L,
                        uint32_t K, uint32_t batch, uint32_t n, hipStream_t s);
// Keys of a key switch: one for the whole batch (count = 1) or one per batch
// element (count = batch <= kMaxRotBatch), each [dnum][2][L+K][N].
struct KeySet {
  uint32_t count;
  const uint32_t* k[kMaxRotBatch];
};

// The key-switching inner product of one batch of one level (a level
// group): for every extended-basis position t < level + K and batch element
// b, acc_c[t][b] = sum_j y_j evk_j[c][t], with y_j = d2[t][b] where t is in
// digit j (already in the NTT domain) and otherwise the ModUp result of
// digit j at (j, t, b).  Layouts: src [digits][level + K][batch][N] (slots of
// a digit's own limbs unused), d2 [level][batch][N], acc [2][level + K][batch][N];
// keys as KeySet (limb index t for q-limbs, L + t - level for the special
// ones).
struct IpGroup {
  const uint32_t* src;  // ip_run: the ModUp transforms' pass-1 intermediates
                        // (tiled); launch_inner_product: the ModUp results
  const uint32_t* d2;
  uint32_t* acc;
  uint32_t level, batch, digits;
  uint32_t key0;   // keys.k index of the group's element 0 (keys.count > 1)
  uint32_t item0;  // ip_run: the group's first work item (filled in by ip_run)
};
constexpr int kMaxIpGroups = kMaxRotBatch;
// The inner products of several level groups in one launch.
struct IpSet {
  uint32_t count, L, K, alpha;
  KeySet keys;  // one key for every element, or one per element (group by group)
  IpGroup g[kMaxIpGroups];
};
static_assert(sizeof(IpSet) <= 4096, "an IpSet is passed as a kernel argument");
// The ModUp forward transforms' second pass fused with the inner product
// (ntt_fourstep.hip): y_j of a position outside digit j is the second pass of
// digit j's tiled intermediate.
hipError_t ip_run(const tfhe_ntt_plan_s* p, IpSet& set, hipStream_t s);
// The inner product over finished ModUp results (ckks_kernels.hip).
hipError_t launch_inner_product(const IpSet& set, const ModConst* mods, uint32_t log_n, hipStream_t s);
hipError_t launch_moddown_conv(const uint32_t* a, uint32_t* conv, const ModConst* mods,
                               const uint2* invp, const uint2* cp, uint32_t level, uint32_t L,
                               uint32_t K, uint32_t batch, uint32_t n, hipStream_t s);
hipError_t launch_moddown_final(const uint32_t* acc, const uint32_t* conv, uint32_t* out,
                                const ModConst* mods, const uint2* pinv, uint32_t level,
                                uint32_t batch, uint32_t n, bool accumulate, hipStream_t s,
                                KernelId id = K_MD_FINAL);
// Conversions of any plane sizes in one launch (blockIdx.y selects), with
// the context's constant tables.
constexpr int kConvPerLaunch = 64;
struct ConvTabs {
  const ModConst* mods;                        // [L+K]
  const uint2 *up_inv, *dn_invp;               // as CkksCtxImpl::d_up_inv, d_dn_invp
  const uint32_t *up_k, *dn_k, *up_mfma, *dn_mfma;
  uint32_t L, K;
};
struct ConvSet {
  ConvTabs tabs;
  uint32_t count;
  ConvDesc d[kConvPerLaunch];
};
static_assert(sizeof(ConvSet) <= 4096, "a ConvSet is passed as a kernel argument");
hipError_t launch_conv_mfma(const ConvSet& set, uint32_t num_cus, KernelId id, hipStream_t s);
// Collects conversions and launches them kConvPerLaunch at a time.
struct ConvQueue {
  ConvTabs tabs;
  std::vector<ConvDesc> q;
  hipError_t flush(uint32_t num_cus, KernelId id, hipStream_t s);
};
// FrobeniusMap of both ciphertext components (in0 -> out0, in1 -> out1, each
// [rows][N]) in one launch; row r uses gs.g[r % gs.batch].
hipError_t launch_frobenius_pair(const uint32_t* in0, uint32_t* out0, const uint32_t* in1, uint32_t* out1,
                                 const GaloisSet& gs, uint32_t rows, uint32_t log_n, hipStream_t s);
hipError_t launch_rescale_bcast(const uint32_t* t, uint32_t* u, const ModConst* mods,
                                uint32_t top, uint32_t batch, uint32_t n, hipStream_t s);

// One ciphertext of a mixed-level batch for launch_tensor_multi /
// launch_frobenius_multi: inputs [2][level][N] where they are; outputs at
// element idx of its level group's [level][B][N] planes.
struct CtDesc {
  const uint32_t* a;  // input (HMULT: first operand)
  const uint32_t* b;  // HMULT: second operand
  uint32_t* out;      // group [2][level][B][N]: (d0, d1), or sigma(c0) and unused
  uint32_t* d;        // group [level][B][N]: d2, or sigma(c1)
  uint32_t level, B, idx, galois;
};
struct CtDescSet {
  uint32_t count;
  CtDesc c[kMaxRotBatch];
};
static_assert(sizeof(CtDescSet) <= 4096, "a CtDescSet is passed as a kernel argument");
// Tensor product of every ciphertext pair of the set in one launch:
// d0 = c0c0', d1 = c0c1' + c1c0' into out, d2 = c1c1' into d.
hipError_t launch_tensor_multi(const CtDescSet& set, const ModConst* mods, uint32_t log_n, hipStream_t s);
// FrobeniusMap of both components of every ciphertext of the set (its own
// Galois element) in one launch: sigma(c0) into out, sigma(c1) into d.
hipError_t launch_frobenius_multi(const CtDescSet& set, uint32_t log_n, hipStream_t s);

}  // namespace tfhe

struct tfhe_ckks_ctx_s : tfhe::CkksCtxImpl {};

namespace tfhe {
// HMULT / HROTATE of a batch whose inputs are separate ciphertexts (the
// request dispatcher's batches), with the result in the batch layout
// [2][level][batch][N] at out.  Arguments are not validated (the caller
// has); ws holds at least tfhe_hmult_workspace_size bytes, 256-aligned.
// Per-ciphertext copies out of level-group results (launch_scatter): element
// r reads row k (component, limb; k < rows[r]) of its group's [rows][batch][N]
// result at src[r] + (k batch[r] + b[r]) N and writes dst[r] + k N.
struct ScatterSet {
  const uint32_t* src[kMaxRotBatch];
  uint32_t* dst[kMaxRotBatch];
  uint32_t rows[kMaxRotBatch], batch[kMaxRotBatch], b[kMaxRotBatch];
};
static_assert(sizeof(ScatterSet) <= 4096, "a ScatterSet is passed as a kernel argument");
hipError_t launch_scatter(const ScatterSet& e, uint32_t count, uint32_t log_n, hipStream_t s);

// One request of a batch of mixed levels and operations (levels_run).
struct LvReq {
  const uint32_t* a;    // input [2][level][N] (HMULT: first operand)
  const uint32_t* b;    // HMULT: second operand [2][level][N]
  uint32_t* out;        // result [2][level][N]
  const uint32_t* key;  // evk (HMULT) or the rotation key
  uint32_t level, galois;
  uint32_t op;          // 0: HMULT, 1: HROTATE
};
// Workspace bytes levels_run needs for these requests.
size_t levels_ws_bytes(const tfhe_ckks_ctx_s* c, const LvReq* r, uint32_t count);
// count <= kMaxRotBatch HMULT and HROTATE requests (r[i].op) of any levels
// in one batched launch sequence: the requests are grouped by (level, op);
// one launch forms every HMULT's tensor product and one every rotation's
// Frobenius map, and every transform, basis conversion and inner product of
// the key switch (the part the two operations share) runs once for all
// groups; the results are copied out to each request's buffer.  Each result
// equals the single call's.
hipError_t levels_run(const tfhe_ckks_ctx_s* c, const LvReq* r, uint32_t count, unsigned char* ws,
                      hipStream_t s);
}  // namespace tfhe
