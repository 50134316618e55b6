// Kernels of HMULT / HROTATE other than the NTT (Sec. III-A, Table 2):
// the tensor product (Hada-Mult, Ele-Add), the fast basis conversion (Conv)
// of ModUp and ModDown, the key-switching inner product (Hada-Mult, Ele-Add)
// and the ModDown finalisation (Ele-Sub, Hada-Mult).  All run over the
// (limb, batch, N) layout, one thread per coefficient position, so each
// limb-plane access is a coalesced stream.
#include "ckks_internal.hpp"

namespace tfhe {
namespace {

constexpr int kThreads = 256;

uint32_t grid_for(uint64_t items) {
  uint64_t blocks = (items + kThreads - 1) / kThreads;
  return (uint32_t)(blocks < 16384 ? (blocks ? blocks : 1) : 16384);
}

// d0 = c0 e0, d1 = c0 e1 + c1 e0 (into out), d2 = c1 e1 (into d2).
__global__ void __launch_bounds__(kThreads)
tensor_kernel(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b, uint32_t* out,
              uint32_t* __restrict__ d2, const ModConst* __restrict__ mods, uint64_t plane,
              uint64_t per_limb) {
  for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < plane;
       i += (uint64_t)gridDim.x * kThreads) {
    const ModConst m = mods[i / per_limb];
    const uint32_t c0 = a[i], c1 = a[plane + i], e0 = b[i], e1 = b[plane + i];
    const uint32_t d0 = mul_mod(c0, e0, m);
    const uint32_t d1 = add_mod(mul_mod(c0, e1, m), mul_mod(c1, e0, m), m.q);
    d2[i] = mul_mod(c1, e1, m);
    out[i] = d0;
    out[plane + i] = d1;
  }
}

// ModUp of one digit D = [d0, d0+nd) (coefficient domain x, [level][B][N]):
// y_i = x_i [(Q_D/q_i)^{-1}]_{q_i};  up[p] = sum_i y_i [Q_D/q_i]_{t(p)} for
// every extended-basis position p outside D (p < level: q-limb p; else
// p-limb L + p - level).
__global__ void __launch_bounds__(kThreads)
modup_kernel(const uint32_t* __restrict__ x, uint32_t* __restrict__ up,
             const ModConst* __restrict__ mods, const uint2* __restrict__ inv,
             const uint2* __restrict__ conv, uint32_t d0, uint32_t nd, uint32_t level, uint32_t L,
             uint32_t K, uint64_t bn) {
  for (uint64_t pos = blockIdx.x * (uint64_t)kThreads + threadIdx.x; pos < bn;
       pos += (uint64_t)gridDim.x * kThreads) {
    uint32_t y[kMaxAlpha];
#pragma unroll
    for (int r = 0; r < kMaxAlpha; ++r) {
      if (r < (int)nd) {
        const uint32_t qi = mods[d0 + r].q;
        y[r] = mul_shoup(x[(uint64_t)(d0 + r) * bn + pos], inv[r].x, inv[r].y, qi);
      }
    }
    const uint32_t ext = level + K;
    for (uint32_t p = 0; p < ext; ++p) {
      if (p >= d0 && p < d0 + nd) continue;
      const uint32_t t = p < level ? p : L + (p - level);
      const uint32_t m = mods[t].q;
      const uint2* c = conv + (uint64_t)t * kMaxAlpha;
      uint32_t acc = 0;
#pragma unroll
      for (int r = 0; r < kMaxAlpha; ++r)
        if (r < (int)nd) acc = add_mod(acc, mul_shoup(y[r], c[r].x, c[r].y, m), m);
      up[(uint64_t)p * bn + pos] = acc;
    }
  }
}

// acc_c[p] = sum_j dt_j[p] o key[j][c][t(p)] over the digits, where dt_j is
// d2 (NTT domain) on the digit's own limbs and the ModUp result elsewhere.
__global__ void __launch_bounds__(kThreads)
inner_product_kernel(const uint32_t* __restrict__ d2, const uint32_t* __restrict__ up,
                     const uint32_t* __restrict__ key, uint32_t* __restrict__ acc0,
                     uint32_t* __restrict__ acc1, const ModConst* __restrict__ mods,
                     uint32_t alpha, uint32_t ndigits, uint32_t level, uint32_t L, uint32_t K,
                     uint32_t batch, uint32_t log_n) {
  const uint32_t n = 1u << log_n;
  const uint64_t bn = (uint64_t)batch * n;
  const uint64_t total = (uint64_t)(level + K) * bn;
  const uint64_t key_plane = (uint64_t)(L + K) * n;  // one key component
  for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * kThreads) {
    const uint32_t p = (uint32_t)(i / bn);
    const uint32_t coef = (uint32_t)(i & (n - 1));
    const uint32_t t = p < level ? p : L + (p - level);
    const ModConst m = mods[t];
    uint32_t s0 = 0, s1 = 0;
    for (uint32_t j = 0; j < ndigits; ++j) {
      const bool own = p < level && p / alpha == j;
      const uint32_t v = own ? d2[i] : up[(uint64_t)j * total + i];
      const uint32_t* kj = key + (uint64_t)j * 2 * key_plane + (uint64_t)t * n + coef;
      s0 = add_mod(s0, mul_mod(v, kj[0], m), m.q);
      s1 = add_mod(s1, mul_mod(v, kj[key_plane], m), m.q);
    }
    acc0[i] = s0;
    acc1[i] = s1;
  }
}

// ModDown conversion: y_k = a_k [(P/p_k)^{-1}]_{p_k} (coefficient domain
// p-limbs a, [K][B][N]); conv_i = sum_k y_k [P/p_k]_{q_i} for i < level.
__global__ void __launch_bounds__(kThreads)
moddown_conv_kernel(const uint32_t* __restrict__ a, uint32_t* __restrict__ conv,
                    const ModConst* __restrict__ mods, const uint2* __restrict__ invp,
                    const uint2* __restrict__ cp, uint32_t level, uint32_t L, uint32_t K,
                    uint64_t bn) {
  for (uint64_t pos = blockIdx.x * (uint64_t)kThreads + threadIdx.x; pos < bn;
       pos += (uint64_t)gridDim.x * kThreads) {
    uint32_t y[kMaxK];
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
      if (k < (int)K) y[k] = mul_shoup(a[(uint64_t)k * bn + pos], invp[k].x, invp[k].y, mods[L + k].q);
    for (uint32_t i = 0; i < level; ++i) {
      const uint32_t qi = mods[i].q;
      const uint2* c = cp + (uint64_t)i * kMaxK;
      uint32_t acc = 0;
#pragma unroll
      for (int k = 0; k < kMaxK; ++k)
        if (k < (int)K) acc = add_mod(acc, mul_shoup(y[k], c[k].x, c[k].y, qi), qi);
      conv[(uint64_t)i * bn + pos] = acc;
    }
  }
}

// out_i (+)= (acc_i - conv_i) [P^{-1}]_{q_i}  (NTT domain, q-limbs).
template <bool kAccumulate>
__global__ void __launch_bounds__(kThreads)
moddown_final_kernel(const uint32_t* __restrict__ acc, const uint32_t* __restrict__ conv,
                     uint32_t* __restrict__ out, const ModConst* __restrict__ mods,
                     const uint2* __restrict__ pinv, uint64_t total, uint64_t bn) {
  for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * kThreads) {
    const uint32_t l = (uint32_t)(i / bn);
    const uint32_t q = mods[l].q;
    uint32_t v = mul_shoup(sub_mod(acc[i], conv[i], q), pinv[l].x, pinv[l].y, q);
    out[i] = kAccumulate ? add_mod(out[i], v, q) : v;
  }
}

}  // namespace

hipError_t launch_tensor(const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t* d2,
                         const ModConst* mods, uint32_t level, uint32_t batch, uint32_t n,
                         hipStream_t s) {
  const uint64_t per_limb = (uint64_t)batch * n, plane = per_limb * level;
  TFHE_TIMED(K_TENSOR, s, hipLaunchKernelGGL(tensor_kernel, dim3(grid_for(plane)), dim3(kThreads), 0, s, a, b, out, d2,
                     mods, plane, per_limb));
  return hipGetLastError();
}

hipError_t launch_modup(const uint32_t* x, uint32_t* up, const ModConst* mods, const uint2* inv,
                        const uint2* conv, uint32_t d0, uint32_t nd, uint32_t level, uint32_t L,
                        uint32_t K, uint32_t batch, uint32_t n, hipStream_t s) {
  const uint64_t bn = (uint64_t)batch * n;
  TFHE_TIMED(K_MODUP, s, hipLaunchKernelGGL(modup_kernel, dim3(grid_for(bn)), dim3(kThreads), 0, s, x, up, mods, inv, conv,
                     d0, nd, level, L, K, bn));
  return hipGetLastError();
}

hipError_t launch_inner_product(const uint32_t* d2, const uint32_t* up, const uint32_t* key,
                                uint32_t* acc0, uint32_t* acc1, const ModConst* mods,
                                uint32_t alpha, uint32_t ndigits, uint32_t level, uint32_t L,
                                uint32_t K, uint32_t batch, uint32_t log_n, hipStream_t s) {
  const uint64_t total = (uint64_t)(level + K) * batch << log_n;
  TFHE_TIMED(K_INNER, s, hipLaunchKernelGGL(inner_product_kernel, dim3(grid_for(total)), dim3(kThreads), 0, s, d2, up, key,
                     acc0, acc1, mods, alpha, ndigits, level, L, K, batch, log_n));
  return hipGetLastError();
}

hipError_t launch_moddown_conv(const uint32_t* a, uint32_t* conv, const ModConst* mods,
                               const uint2* invp, const uint2* cp, uint32_t level, uint32_t L,
                               uint32_t K, uint32_t batch, uint32_t n, hipStream_t s) {
  const uint64_t bn = (uint64_t)batch * n;
  TFHE_TIMED(K_MD_CONV, s, hipLaunchKernelGGL(moddown_conv_kernel, dim3(grid_for(bn)), dim3(kThreads), 0, s, a, conv, mods,
                     invp, cp, level, L, K, bn));
  return hipGetLastError();
}

hipError_t launch_moddown_final(const uint32_t* acc, const uint32_t* conv, uint32_t* out,
                                const ModConst* mods, const uint2* pinv, uint32_t level,
                                uint32_t batch, uint32_t n, bool accumulate, hipStream_t s) {
  const uint64_t bn = (uint64_t)batch * n, total = bn * level;
  if (accumulate)
    TFHE_TIMED(K_MD_FINAL, s, hipLaunchKernelGGL(moddown_final_kernel<true>, dim3(grid_for(total)), dim3(kThreads), 0, s, acc,
                       conv, out, mods, pinv, total, bn));
  else
    TFHE_TIMED(K_MD_FINAL, s, hipLaunchKernelGGL(moddown_final_kernel<false>, dim3(grid_for(total)), dim3(kThreads), 0, s,
                       acc, conv, out, mods, pinv, total, bn));
  return hipGetLastError();
}

}  // namespace tfhe
