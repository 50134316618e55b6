// Element-wise kernels of the hierarchical reconstruction (Sec. IV-A,
// Table 2): Hada-Mult, Ele-Add, Ele-Sub and FrobeniusMap, over the
// (limb, batch, N) layout.  All are HBM-bound: 16-byte accesses, one pass.
#include "internal.hpp"

namespace tfhe {
namespace {

constexpr int kThreads = 256;

template <int kOp>
__global__ void __launch_bounds__(kThreads)
ew_kernel(const ModConst* __restrict__ mods, const uint4* __restrict__ a, const uint4* __restrict__ b,
          uint4* __restrict__ c, uint64_t total4, uint64_t per_limb4, uint32_t n4) {
  for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < total4;
       i += (uint64_t)gridDim.x * kThreads) {
    const uint32_t limb = (uint32_t)(i / per_limb4);
    const ModConst m = mods[limb];
    const uint4 x = a[i];
    const uint4 y = kOp == EW_MUL_BCAST ? b[(uint64_t)limb * n4 + (i % n4)] : b[i];
    uint4 z;
    if (kOp == EW_MUL || kOp == EW_MUL_BCAST) {
      z.x = mul_mod(x.x, y.x, m); z.y = mul_mod(x.y, y.y, m);
      z.z = mul_mod(x.z, y.z, m); z.w = mul_mod(x.w, y.w, m);
    } else if (kOp == EW_ADD) {
      z.x = add_mod(x.x, y.x, m.q); z.y = add_mod(x.y, y.y, m.q);
      z.z = add_mod(x.z, y.z, m.q); z.w = add_mod(x.w, y.w, m.q);
    } else {
      z.x = sub_mod(x.x, y.x, m.q); z.y = sub_mod(x.y, y.y, m.q);
      z.z = sub_mod(x.z, y.z, m.q); z.w = sub_mod(x.w, y.w, m.q);
    }
    c[i] = z;
  }
}

// out_j = in_{pi(j)}, pi(j) = ((2j+1) k mod 2N - 1) / 2 (FrobeniusMap).
__global__ void __launch_bounds__(kThreads)
frobenius_kernel(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, uint32_t galois,
                 uint64_t total, uint32_t log_n) {
  const uint32_t n = 1u << log_n, mask2n = 2 * n - 1;
  for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * kThreads) {
    const uint32_t j = (uint32_t)(i & (n - 1));
    const uint32_t src = (((2 * j + 1) * galois) & mask2n) >> 1;
    out[i] = in[(i - j) + src];
  }
}

// out[l][b][i] = in[b][i] mod q_l for small signed integers in (-2^31, 2^31).
__global__ void __launch_bounds__(kThreads)
load_small_kernel(const ModConst* __restrict__ mods, const int32_t* __restrict__ in,
                  uint32_t* __restrict__ out, uint64_t total, uint64_t per_limb) {
  for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * kThreads) {
    const uint32_t l = (uint32_t)(i / per_limb);
    const uint32_t q = mods[l].q;
    const int32_t x = in[i % per_limb];
    uint32_t r = (uint32_t)(x < 0 ? -(int64_t)x : x) % q;
    out[i] = (x < 0 && r) ? q - r : r;
  }
}

uint32_t grid_for(uint64_t items) {
  uint64_t blocks = (items + kThreads - 1) / kThreads;
  return (uint32_t)(blocks < 8192 ? (blocks ? blocks : 1) : 8192);
}

}  // namespace

hipError_t ew_launch(EwOp op, const ModConst* mods, const uint32_t* a, const uint32_t* b,
                     uint32_t* c, uint32_t limb_count, uint32_t batch, uint32_t n, hipStream_t s) {
  const uint64_t total4 = (uint64_t)limb_count * batch * n / 4;
  const uint64_t per_limb4 = (uint64_t)batch * n / 4;
  const uint32_t n4 = n / 4;
  const uint32_t grid = grid_for(total4);
  const uint4 *A = (const uint4*)a, *B = (const uint4*)b;
  uint4* C = (uint4*)c;
  switch (op) {
    case EW_MUL:
      TFHE_TIMED(K_EW, s, hipLaunchKernelGGL(ew_kernel<EW_MUL>, dim3(grid), dim3(kThreads), 0, s, mods, A, B, C, total4, per_limb4, n4));
      break;
    case EW_ADD:
      TFHE_TIMED(K_EW, s, hipLaunchKernelGGL(ew_kernel<EW_ADD>, dim3(grid), dim3(kThreads), 0, s, mods, A, B, C, total4, per_limb4, n4));
      break;
    case EW_SUB:
      TFHE_TIMED(K_EW, s, hipLaunchKernelGGL(ew_kernel<EW_SUB>, dim3(grid), dim3(kThreads), 0, s, mods, A, B, C, total4, per_limb4, n4));
      break;
    case EW_MUL_BCAST:
      TFHE_TIMED(K_EW, s, hipLaunchKernelGGL(ew_kernel<EW_MUL_BCAST>, dim3(grid), dim3(kThreads), 0, s, mods, A, B, C, total4, per_limb4, n4));
      break;
  }
  return hipGetLastError();
}

hipError_t load_small_launch(const ModConst* mods, const int32_t* in, uint32_t* out,
                             uint32_t limb_count, uint32_t batch, uint32_t n, hipStream_t s) {
  const uint64_t per_limb = (uint64_t)batch * n, total = per_limb * limb_count;
  TFHE_TIMED(K_EW, s, hipLaunchKernelGGL(load_small_kernel, dim3(grid_for(total)), dim3(kThreads), 0, s,
                                         mods, in, out, total, per_limb));
  return hipGetLastError();
}

hipError_t frobenius_launch(const uint32_t* in, uint32_t* out, uint32_t galois, uint32_t rows,
                            uint32_t log_n, hipStream_t s) {
  const uint64_t total = (uint64_t)rows << log_n;
  TFHE_TIMED(K_FROB, s, hipLaunchKernelGGL(frobenius_kernel, dim3(grid_for(total)), dim3(kThreads), 0, s, in, out,
                     galois, total, log_n));
  return hipGetLastError();
}

}  // namespace tfhe
