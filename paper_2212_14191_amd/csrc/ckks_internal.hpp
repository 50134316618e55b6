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
  // Matrix-core basis conversion operands (ConvArgs::a_tab layout):
  uint32_t* d_up_mfma = nullptr;  // [L (digit end - 1)][L+K (target)][4][8]
  uint32_t* d_dn_mfma = nullptr;  // [L (target)][4][8]
  // host copies of the per-input multipliers and per-limb Montgomery constants
  std::vector<uint2> h_up_inv, h_dn_invp;  // as d_up_inv, d_dn_invp
  std::vector<uint32_t> h_up_k, h_dn_k;    // [L][L+K], [L]: ConvArgs::out_k
  std::vector<ModConst> h_mod;             // [L+K]
  std::vector<void*> owned;
};

// Basis conversion on the matrix cores: out_t = sum_r y_r C[t][r] mod m_t
// with y_r = in_r * mult_r mod q_r in [0, q_r) (the integer itself matters:
// q_r != m_t), for up to 8 inputs and 32 targets.
constexpr int kConvMaxIn = 8, kConvMaxOut = 32;
struct ConvArgs {
  const uint32_t* in;   // input plane r at in + r * plane
  uint32_t* out;        // target t written to out + out_plane[t] * plane
  uint64_t plane;       // words per plane (batch * N), a multiple of 64
  uint32_t nin, nout;
  uint32_t in_q[kConvMaxIn];
  uint2 in_mult[kConvMaxIn];       // Shoup pair of mult_r
  uint32_t out_plane[kConvMaxOut];
  uint32_t out_q[kConvMaxOut], out_qneg[kConvMaxOut];
  uint32_t out_k[kConvMaxOut];         // 2^30 sum_r C[t][r] mod m_t (offset correction)
  const uint32_t* a_tab[kConvMaxOut];  // 32 dwords per target: [plane j][8]
};

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

// The ModUp forward transforms' second pass fused with the inner product
// (ntt_fourstep.hip): for every extended-basis position t < level + K and
// batch element b, acc_c[t][b] = sum_j y_j evk_j[c][t] with y_j the second
// pass of digit j's tiled intermediate at (j, t, b) (t outside digit j) or
// d2[t][b] (t in digit j, already in the NTT domain).  Layouts:
//   inter [digits][level + K][batch][N] (pass-1 output, tiled per polynomial;
//         slots of a digit's own limbs unused), d2 [level][batch][N],
//   acc [2][level + K][batch][N], keys as KeySet (limb index t for q-limbs,
//         L + t - level for the special ones).
struct IpArgs {
  const uint32_t* inter;
  const uint32_t* d2;
  uint32_t* acc;
  uint32_t batch, level, L, K, alpha, digits;
  KeySet keys;
};
hipError_t ip_run(const tfhe_ntt_plan_s* p, const IpArgs& a, hipStream_t s);
hipError_t launch_inner_product(const uint32_t* d2, const uint32_t* up, const KeySet& keys,
                                uint32_t* acc0, uint32_t* acc1, const ModConst* mods,
                                uint32_t alpha, uint32_t ndigits, uint32_t level, uint32_t L,
                                uint32_t K, uint32_t batch, uint32_t log_n, hipStream_t s);
hipError_t launch_moddown_conv(const uint32_t* a, uint32_t* conv, const ModConst* mods,
                               const uint2* invp, const uint2* cp, uint32_t level, uint32_t L,
                               uint32_t K, uint32_t batch, uint32_t n, hipStream_t s);
hipError_t launch_moddown_final(const uint32_t* acc, const uint32_t* conv, uint32_t* out,
                                const ModConst* mods, const uint2* pinv, uint32_t level,
                                uint32_t batch, uint32_t n, bool accumulate, hipStream_t s,
                                KernelId id = K_MD_FINAL);
// Several conversions of one plane size in one launch (blockIdx.y selects).
constexpr int kConvPerLaunch = 3;
struct ConvSet {
  uint32_t count;
  ConvArgs a[kConvPerLaunch];
};
static_assert(sizeof(ConvSet) <= 4096, "a ConvSet is passed as a kernel argument");
hipError_t launch_conv_mfma(const ConvSet& set, uint32_t num_cus, KernelId id, hipStream_t s);
// Collects conversions and launches them kConvPerLaunch at a time.
struct ConvQueue {
  std::vector<ConvArgs> q;
  hipError_t flush(uint32_t num_cus, KernelId id, hipStream_t s);
};
// FrobeniusMap of both ciphertext components (in0 -> out0, in1 -> out1, each
// [rows][N]) in one launch; row r uses gs.g[r % gs.batch].
hipError_t launch_frobenius_pair(const uint32_t* in0, uint32_t* out0, const uint32_t* in1, uint32_t* out1,
                                 const GaloisSet& gs, uint32_t rows, uint32_t log_n, hipStream_t s);
hipError_t launch_rescale_bcast(const uint32_t* t, uint32_t* u, const ModConst* mods,
                                uint32_t top, uint32_t batch, uint32_t n, hipStream_t s);

// A batch of separately allocated ciphertexts [2][level][N], read as one
// [2][level][batch][N] array: element b lives at p[b].
struct CtPtrs {
  const uint32_t* p[kMaxRotBatch];
};
// launch_tensor / launch_frobenius_pair reading their inputs through CtPtrs
// (outputs in the batch layout).
hipError_t launch_tensor_ptrs(const CtPtrs& a, const CtPtrs& b, uint32_t* out, uint32_t* d2,
                              const ModConst* mods, uint32_t level, uint32_t batch, uint32_t log_n,
                              hipStream_t s);
hipError_t launch_frobenius_pair_ptrs(const CtPtrs& in, uint32_t* out0, uint32_t* out1, const GaloisSet& gs,
                                      uint32_t level, uint32_t batch, uint32_t log_n, hipStream_t s);

}  // namespace tfhe

struct tfhe_ckks_ctx_s : tfhe::CkksCtxImpl {};

namespace tfhe {
// HMULT / HROTATE of a batch whose inputs are separate ciphertexts (the
// request dispatcher's batches), with the result in the batch layout
// [2][level][batch][N] at out.  Arguments are not validated (the caller
// has); ws holds at least tfhe_hmult_workspace_size bytes, 256-aligned.
hipError_t hmult_ptrs(const tfhe_ckks_ctx_s* c, const CtPtrs& a, const CtPtrs& b, uint32_t* out,
                      const uint32_t* evk, uint32_t level, uint32_t batch, unsigned char* ws, hipStream_t s);
hipError_t rotate_ptrs(const tfhe_ckks_ctx_s* c, const CtPtrs& in, uint32_t* out, const KeySet& keys,
                       const GaloisSet& gs, uint32_t level, uint32_t batch, unsigned char* ws, hipStream_t s);
}  // namespace tfhe
