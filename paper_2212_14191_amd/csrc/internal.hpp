// Internal types of the library: plan and context state, error plumbing,
// kernel launchers.  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <string>
#include <vector>

#include "../../include/tfhe.h"
#include "modarith.hpp"

namespace tfhe {

void set_error(const std::string& msg);
tfhe_status fail(tfhe_status s, const std::string& msg);
tfhe_status hip_check(hipError_t e, const char* what);

// Tables of one pass of the four-step algorithm (per limb and direction).
// A pass transforms vectors of P = 16 r points (r in {1, 2, 4, 8, 16}),
// decomposed as 16 x r: a radix-16 level on the matrix cores (level A), a
// twist, and a radix-r level (level B: matrix cores when r = 16, VALU
// butterflies otherwise).  Laid out exactly as the kernels load them.
//   opA[j][lane][4]   level-A twiddle operand, digit plane j (4 dwords/lane)
//   opB[j][lane][4]   level-B twiddle operand (r = 16 only)
//   twist[lane][j]    twist after level A, {T 2^32 mod q, companion}
//   lb[16]            level-B constants (r < 16): lb[0..3] = rho^0..rho^3 of
//                     the radix-r root rho; lb[8 + t] = factor of output t
struct PassTables {
  uint32_t opA[4][64][4];
  uint32_t opB[4][64][4];
  uint2 twist[64][4];
  uint2 lb[16];
};

// Plain matrices of one 256-point pass (16 x 16 split) for the vector-ALU
// GEMM variant, as Shoup pairs {w, companion}: level A WA[u][s], twist
// T[s][v], level B WB[t][v].
// Vector-ALU variant: the two 16-point matrices in Montgomery form with
// R = 2^64 (W 2^64 mod q), stored output-major (WA[s][u], WB[t][v]), and the
// twist as Shoup pairs T[s][v].
struct CoPass {
  uint32_t WA[16][16], WB[16][16];
  uint2 T[16][16];
};

// Tables of the one-pass four-step kernel (N = 2^12..2^15) for one limb and
// direction; its first pass uses the two-pass kernel's pass-1 tables.
//   p2       second pass.  Forward (256-point): level B's twiddles unscaled
//            and the twist carrying 2^64, so opB equals opA (the 16-point DFT
//            matrix is symmetric).  Inverse (N1-point): opA with the level-A
//            index u = g + 4c for lane (i, g), dword c, instead of 4g + c.
//   post_b   [lane][j][set] first-pass post-twist, the factor fixed per lane:
//            P(4m + set, out) (times 2^32 after a matrix-core level B), Shoup
//   post_a   [step][lane][j] the factor of a step whose first column quad is
//            Q0 = step * 16 / r: P(4 Q0 + 4m, out) / P(4m, out), times 2^32
//            (Montgomery form); (m, out) as lane / register j hold them.
struct OnePassTables {
  PassTables p2;
  uint2 post_b[64][4][4];
  uint32_t post_a[32][64][4];
};

// Device-side description of one limb for the four-step kernels.
struct FourStepLimb {
  const PassTables* pass1;  // first pass (its post-twist: post1)
  const PassTables* pass2;  // second pass
  const uint2* post1;       // [256 column bases][64 lanes][4]: post-twist of pass 1
  const CoPass* co1;        // vector-ALU variant (N = 2^16 only): pass matrices
  const CoPass* co2;
  const uint2* co_post;     // [256 columns][256 outputs]: post-twist of pass 1
  const OnePassTables* op;  // one-pass kernel (N = 2^12..2^15), else null
  uint32_t q, qneg;         // modulus and -q^{-1} mod 2^32
};

struct tfhe_plan_impl {
  uint32_t log_n = 0, n = 0, n_limbs = 0;
  tfhe_ntt_algo algo = TFHE_NTT_BUTTERFLY;  // what AUTO resolves to
  bool has_mfma = false;
  bool has_co = false;            // vector-ALU four-step variant (N = 2^16)
  int device = 0;
  uint32_t num_cus = 256;         // compute units of the device
  uint32_t fs_wg_per_cu = 0;      // persistent four-step workgroups per CU (0: occupancy)
  uint32_t fs_wide = 0;           // 256-point stage items: 0 auto, 1 narrow, 2 wide when possible
  uint32_t fs_passes = 0;         // four-step HBM passes: 0 auto (one at 2^12..2^14 for large launches), 1 one, 2 two
  uint32_t fs_ring = 0;           // LDS ring stages of the wide-item passes: 0 auto (2), 2, 3
  uint32_t ks_inner = 0;          // key switching: 0 default (fused), 1 fused second pass + inner product, 2 separate
  std::vector<uint32_t> q, psi;
  // device arrays
  ModConst* d_mod = nullptr;      // [n_limbs]
  uint2* d_bf_fwd = nullptr;      // [n_limbs][N] {psi^{brv(i)}, companion}
  uint2* d_bf_inv = nullptr;      // [n_limbs][N] {psi^{-brv(i)}, companion}
  uint2* d_ninv = nullptr;        // [n_limbs] {N^{-1}, companion}
  FourStepLimb* d_fs_fwd = nullptr;  // [n_limbs]
  FourStepLimb* d_fs_inv = nullptr;  // [n_limbs]
  void* d_fs_blob = nullptr;          // owns all four-step tables
  std::vector<void*> owned;
};

}  // namespace tfhe

struct tfhe_ntt_plan_s : tfhe::tfhe_plan_impl {};

namespace tfhe {

// ---- operation-level batching: one fused launch over many transforms
// A transform unit: `batch` polynomials of limbs [limb_begin, +limb_count) of
// a plan, forward or inverse, in -> out (in == out allowed), with its own
// slice of the workspace.
struct NttUnit {
  const tfhe_ntt_plan_s* plan;
  bool inverse;
  const uint32_t* in;
  uint32_t* out;
  uint32_t limb_begin, limb_count, batch;
  // Forward four-step transforms only: instead of the transform y, write
  // out = (acc - y) mult_l (epi_add: out += ...), mult_l the Shoup pair of
  // limb limb_begin + l; acc has the layout of out.
  const uint32_t* acc = nullptr;
  const uint2* epi_mult = nullptr;
  bool epi_add = false;
  // Forward four-step transforms only: run the first pass alone, writing its
  // tiled intermediate to `out` (the second pass is left to a fused
  // consumer, ip_run)
  bool pass1_only = false;
  // Forward four-step transforms only: every limb of the unit reads the same
  // input plane `in` ([batch][N], values below 2^31, not reduced by the
  // limb's modulus), i.e. the transform of that integer polynomial modulo
  // each of the unit's limbs
  bool in_bcast = false;
};
// Runs every unit with the four-step algorithm (all units need has_mfma) or
// the butterfly; ws must hold the sum of the units' workspaces.
hipError_t fs_run_units(const NttUnit* u, uint32_t count, void* ws, hipStream_t s);
hipError_t bf_run_units(const NttUnit* u, uint32_t count, void* ws, hipStream_t s);
size_t unit_ws_bytes(const NttUnit& u, bool mfma);

// ---- butterfly launchers (ntt_butterfly.hip)
size_t bf_workspace_bytes(const tfhe_ntt_plan_s* p, uint32_t limb_count, uint32_t batch);
hipError_t bf_forward(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws,
                      uint32_t limb_begin, uint32_t limb_count, uint32_t batch, hipStream_t s);
hipError_t bf_inverse(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws,
                      uint32_t limb_begin, uint32_t limb_count, uint32_t batch, hipStream_t s);

// ---- four-step MFMA launchers (ntt_fourstep.hip)
bool fs_supported(uint32_t log_n);
size_t fs_workspace_bytes(const tfhe_ntt_plan_s* p, uint32_t limb_count, uint32_t batch);
hipError_t fs_forward(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws,
                      uint32_t limb_begin, uint32_t limb_count, uint32_t batch, hipStream_t s);
hipError_t fs_inverse(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws,
                      uint32_t limb_begin, uint32_t limb_count, uint32_t batch, hipStream_t s);
// Vector-ALU GEMM variant of the same passes (plan->has_co); same workspace.
hipError_t co_transform(const tfhe_ntt_plan_s* p, bool inverse, const uint32_t* in, uint32_t* out,
                        void* ws, uint32_t limb_begin, uint32_t limb_count, uint32_t batch,
                        hipStream_t s);

// ---- element-wise launchers (elementwise.hip)
enum EwOp { EW_MUL = 0, EW_ADD = 1, EW_SUB = 2, EW_MUL_BCAST = 3 };
hipError_t ew_launch(EwOp op, const ModConst* mods, const uint32_t* a, const uint32_t* b,
                     uint32_t* c, uint32_t limb_count, uint32_t batch, uint32_t n, hipStream_t s);
hipError_t frobenius_launch(const uint32_t* in, uint32_t* out, uint32_t galois, uint32_t rows,
                            uint32_t log_n, hipStream_t s);
// Per-batch-element Galois elements of a multi-rotation: row r of the
// [rows][N] array (rows = limbs x batch, batch fastest) uses g[r % batch].
constexpr uint32_t kMaxRotBatch = TFHE_ROTATE_MULTI_MAX;
struct GaloisSet {
  uint32_t batch;
  uint32_t g[kMaxRotBatch];
};

// ---- per-kernel event timing (timing.cpp)
enum KernelId {
  K_FS_PASS1 = 0, K_FS_PASS2, K_BF_SINGLE, K_BF_COLS, K_BF_ROWS, K_EW, K_TENSOR, K_MODUP,
  K_INNER, K_MD_CONV, K_MD_FINAL, K_FROB, K_RS_BCAST, K_RS_FINAL, K_CO_PASS1, K_CO_PASS2, K_OP, K_IP
};
// Resident workgroups per CU of a kernel, queried once per process: the
// dispatcher's workers may race to fill the cache; they store one value.
template <typename K>
int occupancy_cached(std::atomic<int>& cache, K kernel, int threads) {
  int v = cache.load(std::memory_order_relaxed);
  if (v == 0) {
    int n = 0;
    v = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) == hipSuccess && n > 0 ? n : 1;
    cache.store(v, std::memory_order_relaxed);
  }
  return v;
}

bool timing_on();
void* timing_begin(int id, hipStream_t s);
void timing_end(void* token, hipStream_t s);
// Launch with optional event bracketing.
#define TFHE_TIMED(id, stream, ...)                  \
  do {                                               \
    void* tfhe_tok_ = ::tfhe::timing_begin(id, stream); \
    __VA_ARGS__;                                     \
    ::tfhe::timing_end(tfhe_tok_, stream);           \
  } while (0)

hipError_t load_small_launch(const ModConst* mods, const int32_t* in, uint32_t* out,
                             uint32_t limb_count, uint32_t batch, uint32_t n, hipStream_t s);

// ---- host-side number theory (plan.cpp)
bool is_prime_u32(uint32_t q);
ModConst make_modconst(uint32_t q);
uint32_t pow_mod(uint32_t b, uint64_t e, uint32_t q);
uint32_t inv_mod(uint32_t x, uint32_t q);
uint32_t default_psi(uint32_t q, uint32_t log_n);  // 0 if none

}  // namespace tfhe
