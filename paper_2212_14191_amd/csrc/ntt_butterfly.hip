// Radix-2 butterfly NTT / INTT on the vector ALUs: the plain baseline the
// paper compares against (Sec. II-A, Fig. 2; "TensorFHE-NT" in Sec. V).
//
// Forward: Cooley-Tukey butterflies with the negacyclic twist merged into the
// twiddles (psi^{bitrev(m+i)} for group i of stage m), natural-order input,
// bit-reversed intermediate; the final store gathers through the bit
// reversal so the output is in natural order (index k = evaluation at
// psi^{2k+1}, Eq. 4).  Inverse: Gentleman-Sande butterflies with
// psi^{-bitrev(h+i)}, reading the natural-order input through the bit
// reversal, then N^{-1}.
//
// N <= 2^12: one workgroup owns a polynomial, all stages in LDS.
// N  > 2^12: two passes over an R x 256 view (R = N/256): the stages with
// butterfly stride >= 256 act within columns (pass A), the rest within rows
// of 256 (pass B); the intermediate goes through the caller's workspace.
#include "internal.hpp"

namespace tfhe {
namespace {

constexpr int kThreads = 256;
constexpr int kRow = 256;   // row length of the two-pass view
constexpr int kBlk = 16;    // columns (pass A) or rows (pass B) per workgroup

__device__ __forceinline__ uint32_t brev(uint32_t x, uint32_t bits) {
  return __builtin_bitreverse32(x) >> (32 - bits);
}

__device__ __forceinline__ void ct_bfly(uint32_t* lds, uint32_t j, uint32_t t, uint2 w, uint32_t q) {
  uint32_t u = lds[j];
  uint32_t v = mul_shoup(lds[j + t], w.x, w.y, q);
  lds[j] = add_mod(u, v, q);
  lds[j + t] = sub_mod(u, v, q);
}

__device__ __forceinline__ void gs_bfly(uint32_t* lds, uint32_t j, uint32_t t, uint2 w, uint32_t q) {
  uint32_t u = lds[j];
  uint32_t v = lds[j + t];
  lds[j] = add_mod(u, v, q);
  lds[j + t] = mul_shoup(sub_mod(u, v, q), w.x, w.y, q);
}

// ---------------------------------------------------------- single pass
__global__ void __launch_bounds__(kThreads)
bf_single_fwd(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, const uint2* __restrict__ tw,
              const ModConst* __restrict__ mods, uint32_t log_n, uint32_t batch) {
  extern __shared__ uint32_t lds[];
  const uint32_t n = 1u << log_n;
  const uint32_t poly = blockIdx.x, limb = poly / batch;
  const uint32_t q = mods[limb].q;
  const uint2* w = tw + (size_t)limb * n;
  const uint32_t* src = in + (size_t)poly * n;
  for (uint32_t i = threadIdx.x; i < n; i += kThreads) lds[i] = src[i];
  __syncthreads();
  for (uint32_t m = 1, t = n >> 1; m < n; m <<= 1, t >>= 1) {
    for (uint32_t b = threadIdx.x; b < (n >> 1); b += kThreads) {
      uint32_t i = b / t, j = 2 * i * t + (b % t);
      ct_bfly(lds, j, t, w[m + i], q);
    }
    __syncthreads();
  }
  uint32_t* dst = out + (size_t)poly * n;
  for (uint32_t k = threadIdx.x; k < n; k += kThreads) dst[k] = lds[brev(k, log_n)];
}

__global__ void __launch_bounds__(kThreads)
bf_single_inv(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, const uint2* __restrict__ tw,
              const uint2* __restrict__ ninv, const ModConst* __restrict__ mods, uint32_t log_n,
              uint32_t batch) {
  extern __shared__ uint32_t lds[];
  const uint32_t n = 1u << log_n;
  const uint32_t poly = blockIdx.x, limb = poly / batch;
  const uint32_t q = mods[limb].q;
  const uint2* w = tw + (size_t)limb * n;
  const uint32_t* src = in + (size_t)poly * n;
  for (uint32_t k = threadIdx.x; k < n; k += kThreads) lds[brev(k, log_n)] = src[k];
  __syncthreads();
  for (uint32_t h = n >> 1, t = 1; h >= 1; h >>= 1, t <<= 1) {
    for (uint32_t b = threadIdx.x; b < (n >> 1); b += kThreads) {
      uint32_t i = b / t, j = 2 * i * t + (b % t);
      gs_bfly(lds, j, t, w[h + i], q);
    }
    __syncthreads();
  }
  const uint2 ni = ninv[limb];
  uint32_t* dst = out + (size_t)poly * n;
  for (uint32_t k = threadIdx.x; k < n; k += kThreads) dst[k] = mul_shoup(lds[k], ni.x, ni.y, q);
}

// ------------------------------------------------------------ two passes
// Column pass: a workgroup owns kBlk consecutive columns of one polynomial,
// tile lds[r][c] (R x kBlk).  Forward runs stages m = 1 .. R/2; inverse runs
// h = R/2 .. 1 then scales by N^{-1}.
template <bool kInverse>
__global__ void __launch_bounds__(kThreads)
bf_cols(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, const uint2* __restrict__ tw,
        const uint2* __restrict__ ninv, const ModConst* __restrict__ mods, uint32_t log_n,
        uint32_t batch) {
  __shared__ uint32_t lds[kRow * kBlk];
  const uint32_t n = 1u << log_n, R = n / kRow;
  const uint32_t cb = blockIdx.x % (kRow / kBlk), poly = blockIdx.x / (kRow / kBlk);
  const uint32_t limb = poly / batch;
  const uint32_t q = mods[limb].q;
  const uint2* w = tw + (size_t)limb * n;
  const uint32_t* src = in + (size_t)poly * n + cb * kBlk;
  for (uint32_t e = threadIdx.x; e < R * kBlk; e += kThreads) {
    uint32_t r = e / kBlk, c = e % kBlk;
    lds[e] = src[r * kRow + c];
  }
  __syncthreads();
  const uint32_t nb = (R / 2) * kBlk;  // butterflies per stage
  if (!kInverse) {
    for (uint32_t m = 1, tr = R / 2; m < R; m <<= 1, tr >>= 1) {
      for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
        uint32_t c = b % kBlk, rb = b / kBlk;
        uint32_t i = rb / tr, r = 2 * i * tr + (rb % tr);
        ct_bfly(lds, r * kBlk + c, tr * kBlk, w[m + i], q);
      }
      __syncthreads();
    }
  } else {
    for (uint32_t h = R / 2, tr = 1; h >= 1; h >>= 1, tr <<= 1) {
      for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
        uint32_t c = b % kBlk, rb = b / kBlk;
        uint32_t i = rb / tr, r = 2 * i * tr + (rb % tr);
        gs_bfly(lds, r * kBlk + c, tr * kBlk, w[h + i], q);
      }
      __syncthreads();
    }
  }
  uint32_t* dst = out + (size_t)poly * n + cb * kBlk;
  const uint2 ni = ninv[limb];
  for (uint32_t e = threadIdx.x; e < R * kBlk; e += kThreads) {
    uint32_t r = e / kBlk, c = e % kBlk;
    uint32_t v = lds[e];
    if (kInverse) v = mul_shoup(v, ni.x, ni.y, q);
    dst[r * kRow + c] = v;
  }
}

// Row pass: a workgroup owns the kBlk rows whose bit-reversed indices are
// consecutive, {row = bitrev(kBlk*rb + i)}, tile lds[i][col].  Position
// row*256 + col of the bit-reversed order holds the natural-order index
// bitrev8(col)*R + kBlk*rb + i, so the natural-order side is accessed in
// runs of kBlk consecutive words.
// Forward: input = pass-A result (natural rows), stages m = R .. N/2, store
// gathered to natural order.  Inverse: load gathered from the natural-order
// input, stages h = N/2 .. R, store natural rows.
template <bool kInverse>
__global__ void __launch_bounds__(kThreads)
bf_rows(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, const uint2* __restrict__ tw,
        const ModConst* __restrict__ mods, uint32_t log_n, uint32_t batch) {
  __shared__ uint32_t lds[kBlk * kRow];
  const uint32_t n = 1u << log_n, R = n / kRow, log_r = log_n - 8;
  const uint32_t rb = blockIdx.x % (R / kBlk), poly = blockIdx.x / (R / kBlk);
  const uint32_t limb = poly / batch;
  const uint32_t q = mods[limb].q;
  const uint2* w = tw + (size_t)limb * n;
  const uint32_t* src = in + (size_t)poly * n;
  for (uint32_t e = threadIdx.x; e < kBlk * kRow; e += kThreads) {
    if (!kInverse) {
      uint32_t i = e / kRow, col = e % kRow;
      lds[e] = src[brev(kBlk * rb + i, log_r) * kRow + col];
    } else {
      uint32_t i = e % kBlk, cn = e / kBlk;  // natural index cn*R + kBlk*rb + i
      lds[i * kRow + brev(cn, 8)] = src[cn * R + kBlk * rb + i];
    }
  }
  __syncthreads();
  const uint32_t nb = kBlk * kRow / 2;
  if (!kInverse) {
    for (uint32_t m = R, t = kRow / 2; m < n; m <<= 1, t >>= 1) {
      for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
        uint32_t i = b / (kRow / 2), bb = b % (kRow / 2);
        uint32_t row = brev(kBlk * rb + i, log_r);
        uint32_t g = bb / t, j = 2 * g * t + (bb % t);
        uint32_t grp = (row * kRow + j) / (2 * t);
        ct_bfly(lds, i * kRow + j, t, w[m + grp], q);
      }
      __syncthreads();
    }
  } else {
    for (uint32_t h = n / 2, t = 1; h >= R; h >>= 1, t <<= 1) {
      for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
        uint32_t i = b / (kRow / 2), bb = b % (kRow / 2);
        uint32_t row = brev(kBlk * rb + i, log_r);
        uint32_t g = bb / t, j = 2 * g * t + (bb % t);
        uint32_t grp = (row * kRow + j) / (2 * t);
        gs_bfly(lds, i * kRow + j, t, w[h + grp], q);
      }
      __syncthreads();
    }
  }
  uint32_t* dst = out + (size_t)poly * n;
  for (uint32_t e = threadIdx.x; e < kBlk * kRow; e += kThreads) {
    if (!kInverse) {
      uint32_t i = e % kBlk, cn = e / kBlk;
      dst[cn * R + kBlk * rb + i] = lds[i * kRow + brev(cn, 8)];
    } else {
      uint32_t i = e / kRow, col = e % kRow;
      dst[brev(kBlk * rb + i, log_r) * kRow + col] = lds[e];
    }
  }
}

dim3 poly_grid(uint32_t x, uint32_t polys) { return dim3(x * polys); }

}  // namespace

size_t bf_workspace_bytes(const tfhe_ntt_plan_s* p, uint32_t limb_count, uint32_t batch) {
  if (p->log_n <= 12) return 0;
  return (size_t)limb_count * batch * p->n * sizeof(uint32_t);
}

hipError_t bf_forward(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws,
                      uint32_t limb_begin, uint32_t limb_count, uint32_t batch, hipStream_t s) {
  const uint32_t polys = limb_count * batch;
  const uint2* tw = p->d_bf_fwd + (size_t)limb_begin * p->n;
  const ModConst* mods = p->d_mod + limb_begin;
  if (p->log_n <= 12) {
    TFHE_TIMED(K_BF_SINGLE, s, hipLaunchKernelGGL(bf_single_fwd, dim3(polys), dim3(kThreads), p->n * sizeof(uint32_t), s, in,
                       out, tw, mods, p->log_n, batch));
  } else {
    uint32_t* mid = (uint32_t*)ws;
    const uint32_t R = p->n / kRow;
    TFHE_TIMED(K_BF_COLS, s, hipLaunchKernelGGL(bf_cols<false>, poly_grid(kRow / kBlk, polys), dim3(kThreads), 0, s, in,
                       mid, tw, p->d_ninv + limb_begin, mods, p->log_n, batch));
    TFHE_TIMED(K_BF_ROWS, s, hipLaunchKernelGGL(bf_rows<false>, poly_grid(R / kBlk, polys), dim3(kThreads), 0, s, mid, out,
                       tw, mods, p->log_n, batch));
  }
  return hipGetLastError();
}

hipError_t bf_inverse(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws,
                      uint32_t limb_begin, uint32_t limb_count, uint32_t batch, hipStream_t s) {
  const uint32_t polys = limb_count * batch;
  const uint2* tw = p->d_bf_inv + (size_t)limb_begin * p->n;
  const ModConst* mods = p->d_mod + limb_begin;
  if (p->log_n <= 12) {
    TFHE_TIMED(K_BF_SINGLE, s, hipLaunchKernelGGL(bf_single_inv, dim3(polys), dim3(kThreads), p->n * sizeof(uint32_t), s, in,
                       out, tw, p->d_ninv + limb_begin, mods, p->log_n, batch));
  } else {
    uint32_t* mid = (uint32_t*)ws;
    const uint32_t R = p->n / kRow;
    TFHE_TIMED(K_BF_ROWS, s, hipLaunchKernelGGL(bf_rows<true>, poly_grid(R / kBlk, polys), dim3(kThreads), 0, s, in, mid,
                       tw, mods, p->log_n, batch));
    TFHE_TIMED(K_BF_COLS, s, hipLaunchKernelGGL(bf_cols<true>, poly_grid(kRow / kBlk, polys), dim3(kThreads), 0, s, mid,
                       out, tw, p->d_ninv + limb_begin, mods, p->log_n, batch));
  }
  return hipGetLastError();
}

}  // namespace tfhe
