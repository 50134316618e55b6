// Four-step NTT on INT8 matrix cores (Sec. III-B/III-C, Eq. 8 and Eq. 9),
// re-designed for gfx950.
//
// N = 2^16 is viewed as a 256 x 256 matrix (n = 256 n1 + n2, k = k1 + 256 k2):
//   pass 1, per column n2:  Y[k1] = sum_{n1} phi^{(2k1+1) n1} a[n1][n2],
//                           Z[k1][n2] = Y[k1] * psi^{(2k1+1) n2}   (the W2 twist)
//   pass 2, per row k1:     A[k1 + 256 k2] = sum_{n2} w^{k2 n2} Z[k1][n2]
// (phi = psi^256, w = psi^512).  Each 256-point stage runs as two radix-16
// levels (n = 16u + v, k = s + 16t): a dense 16 x 16 contraction on the
// matrix cores, an element-wise twist, a second 16 x 16 contraction.
//
// Exactness (the segment-fusion idea of Sec. III-C, Fig. 4): every operand
// enters the matrix core as four balanced signed byte digits.  A data word x
// (taken in [-0x80808080, 0x7F7F7F7F]) is x = sum_d 2^{8d} x_d; a twiddle w
// is supplied as the digits j of W^(d) = 2^{8d} w mod q for d = 0..3.  With
// the four data digits of a coefficient packed into four consecutive K
// bytes, one v_mfma_i32_16x16x64_i8 per twiddle digit plane j yields
//   C_j = sum_u sum_d x_d[u] * digit_j(W^(d)[u])   (|C_j| <= 2^20, exact)
// and sum_j 2^{8j} C_j = sum_u x[u] w[u] (mod q).  The "fusion" step recombines
// L = C_0 + 2^8 C_1, H = C_2 + 2^8 C_3 (32-bit exact; C_0 and C_2 start at q so
// both are positive) and reduces z = L*t + H*(2^16 t) mod q with two Shoup
// products, t being the twist of that position; z is then re-sliced into
// digits for the next contraction (two VALU operations).
//
// Data movement: a workgroup takes 16 vectors (columns of a 256 x 256 row-
// major matrix) of one polynomial through LDS; each wave transforms four of
// them, one vector per 16 x 16 tile with four coefficients per lane.  Both
// passes load column blocks; pass 1 writes its digit-form result row-wise to
// the workspace (the transpose), pass 2 writes canonical residues back as a
// column block through LDS.  The inverse runs the same two kernels with the
// inverse tables (w^{-1}, phi^{-2}, psi^{-(2k1+1) n2}, N^{-1} folded into the
// last level).
#include "internal.hpp"

namespace tfhe {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kCols = 16;     // vectors per workgroup
constexpr int kStride = 324;  // LDS words per vector: 256 + 64 pad, = 4 (mod 64)

__device__ __forceinline__ int lds_pos(int col, int n) { return col * kStride + n + 16 * (n >> 6); }

__device__ __forceinline__ v4i mfma(v4i a, v4i b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// Fusion + twist + re-slice of one coefficient (see the file comment).
__device__ __forceinline__ uint32_t fuse_twist_digits(int c0, int c1, int c2, int c3, uint4 t,
                                                      uint32_t q) {
  uint32_t lo = (uint32_t)c0 + ((uint32_t)c1 << 8);
  uint32_t hi = (uint32_t)c2 + ((uint32_t)c3 << 8);
  uint32_t r1 = reduce_once(mul_shoup_lazy(lo, t.x, t.y, q), q);
  uint32_t r2 = reduce_once(mul_shoup_lazy(hi, t.z, t.w, q), q);
  int32_t z = (int32_t)(r1 + r2 - q);          // in [-q, q)
  z = z > 0x7F7F7F7F ? z - (int32_t)q : z;     // only when q > 0x7F7F7F7F
  return balanced_digits(z);
}

// Fusion + canonical reduction (no twist): (L + 2^16 H) mod q in [0, q).
__device__ __forceinline__ uint32_t fuse_final(int c0, int c1, int c2, int c3, uint32_t c16,
                                               uint32_t c16p, uint32_t q) {
  uint32_t lo = (uint32_t)c0 + ((uint32_t)c1 << 8);
  uint32_t hi = (uint32_t)c2 + ((uint32_t)c3 << 8);
  return add_mod(reduce_once(lo, q), mul_shoup(hi, c16, c16p, q), q);
}

// One 256-point stage of one vector: level A, twist, level B.  x holds the
// lane's four input words as digits (lane (v, g), word c: element 64g+16c+v);
// on return acc[j][r] is plane j of output s + 16 (4g + r) for lane (s, g).
__device__ __forceinline__ void stage256(v4i x, const v4i* opA, const v4i* opB, const uint4* tw,
                                         uint32_t q, v4i* acc) {
  const v4i bias = {(int)q, (int)q, (int)q, (int)q};
  const v4i zero = {0, 0, 0, 0};
  v4i c0 = mfma(x, opA[0], bias);
  v4i c1 = mfma(x, opA[1], zero);
  v4i c2 = mfma(x, opA[2], bias);
  v4i c3 = mfma(x, opA[3], zero);
  v4i z;
#pragma unroll
  for (int r = 0; r < 4; ++r) z[r] = (int)fuse_twist_digits(c0[r], c1[r], c2[r], c3[r], tw[r], q);
  acc[0] = mfma(opB[0], z, bias);
  acc[1] = mfma(opB[1], z, zero);
  acc[2] = mfma(opB[2], z, bias);
  acc[3] = mfma(opB[3], z, zero);
}

template <bool kFirst>
__global__ void __launch_bounds__(kThreads)
fs_pass(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
        const FourStepLimb* __restrict__ limbs, uint32_t batch) {
  __shared__ uint32_t lds[kCols * kStride];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t blk = blockIdx.x % (256 / kCols), poly = blockIdx.x / (256 / kCols);
  const FourStepLimb L = limbs[poly / batch];
  const uint32_t q = L.q;
  const PassTables* P = kFirst ? L.pass1 : L.pass2;
  const size_t base = (size_t)poly << 16;

  // column block -> LDS (each thread: four 16-byte row segments)
  const uint32_t* src = in + base + blk * kCols;
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    int row = it * 64 + (tid >> 2), c0 = 4 * (tid & 3);
    uint4 v = *(const uint4*)(src + row * 256 + c0);
    lds[lds_pos(c0 + 0, row)] = v.x;
    lds[lds_pos(c0 + 1, row)] = v.y;
    lds[lds_pos(c0 + 2, row)] = v.z;
    lds[lds_pos(c0 + 3, row)] = v.w;
  }

  v4i opA[4], opB[4];
  uint4 tw[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    opA[j] = *(const v4i*)&P->opA[j][lane][0];
    opB[j] = *(const v4i*)&P->opB[j][lane][0];
    tw[j] = P->twist[lane][j];
  }
  __syncthreads();

  const int v = lane & 15, g = lane >> 4;
#pragma unroll 2
  for (int cc = 0; cc < 4; ++cc) {
    const int col = 4 * wave + cc;
    v4i x;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      uint32_t w = lds[lds_pos(col, 64 * g + 16 * c + v)];
      x[c] = kFirst ? (int)balanced_digits(to_window(w, q)) : (int)w;
    }
    v4i acc[4];
    stage256(x, opA, opB, tw, q, acc);
    if (kFirst) {
      // post twist and row store: output k = s + 64g + 16r of vector col
      const uint32_t gcol = blk * kCols + col;
      const uint4* pt = L.post1 + ((size_t)gcol * 64 + lane) * 4;
      uint32_t* dst = out + base + gcol * 256 + v + 64 * g;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        dst[16 * r] = fuse_twist_digits(acc[0][r], acc[1][r], acc[2][r], acc[3][r], pt[r], q);
    } else {
      // the wave owns this vector's LDS column: overwrite it with the output
#pragma unroll
      for (int r = 0; r < 4; ++r)
        lds[lds_pos(col, v + 64 * g + 16 * r)] =
            fuse_final(acc[0][r], acc[1][r], acc[2][r], acc[3][r], L.c16, L.c16p, q);
    }
  }

  if (!kFirst) {
    __syncthreads();
    uint32_t* dst = out + base + blk * kCols;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      int row = it * 64 + (tid >> 2), c0 = 4 * (tid & 3);
      uint4 v4 = make_uint4(lds[lds_pos(c0, row)], lds[lds_pos(c0 + 1, row)],
                            lds[lds_pos(c0 + 2, row)], lds[lds_pos(c0 + 3, row)]);
      *(uint4*)(dst + row * 256 + c0) = v4;
    }
  }
}

}  // namespace

bool fs_supported(uint32_t log_n) { return log_n == 16; }

size_t fs_workspace_bytes(const tfhe_ntt_plan_s* p, uint32_t limb_count, uint32_t batch) {
  return (size_t)limb_count * batch * p->n * sizeof(uint32_t);
}

static hipError_t fs_run(const FourStepLimb* limbs, const uint32_t* in, uint32_t* out, void* ws,
                         uint32_t limb_count, uint32_t batch, hipStream_t s) {
  const uint32_t polys = limb_count * batch;
  dim3 grid(polys * (256 / kCols));
  TFHE_TIMED(K_FS_PASS1, s,
             hipLaunchKernelGGL(fs_pass<true>, grid, dim3(kThreads), 0, s, in, (uint32_t*)ws, limbs,
                                batch));
  TFHE_TIMED(K_FS_PASS2, s,
             hipLaunchKernelGGL(fs_pass<false>, grid, dim3(kThreads), 0, s, (const uint32_t*)ws, out,
                                limbs, batch));
  return hipGetLastError();
}

hipError_t fs_forward(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws,
                      uint32_t limb_begin, uint32_t limb_count, uint32_t batch, hipStream_t s) {
  return fs_run(p->d_fs_fwd + limb_begin, in, out, ws, limb_count, batch, s);
}

hipError_t fs_inverse(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws,
                      uint32_t limb_begin, uint32_t limb_count, uint32_t batch, hipStream_t s) {
  return fs_run(p->d_fs_inv + limb_begin, in, out, ws, limb_count, batch, s);
}

}  // namespace tfhe
