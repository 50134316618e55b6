// Kernels of HMULT / HROTATE / RESCALE other than the NTT (Sec. III-A, Table 2):
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

// Four consecutive coefficients per thread (16-byte accesses); every plane
// holds a multiple of 4 words.
template <typename F>
__device__ __forceinline__ uint4 map4(uint4 a, F f) {
  return make_uint4(f(a.x, 0), f(a.y, 1), f(a.z, 2), f(a.w, 3));
}
__device__ __forceinline__ uint32_t comp(const uint4& a, int i) {
  return i == 0 ? a.x : i == 1 ? a.y : i == 2 ? a.z : a.w;
}

// d0 = c0 e0, d1 = c0 e1 + c1 e0 (into out), d2 = c1 e1 (into d2).
__global__ void __launch_bounds__(kThreads)
tensor_kernel(const uint4* __restrict__ a, const uint4* __restrict__ b, uint4* out,
              uint4* __restrict__ d2, const ModConst* __restrict__ mods, uint64_t plane4,
              uint64_t per_limb4) {
  for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < plane4;
       i += (uint64_t)gridDim.x * kThreads) {
    const ModConst m = mods[i / per_limb4];
    const uint4 c0 = a[i], c1 = a[plane4 + i], e0 = b[i], e1 = b[plane4 + i];
    d2[i] = map4(c1, [&](uint32_t x, int k) { return mul_mod(x, comp(e1, k), m); });
    out[i] = map4(c0, [&](uint32_t x, int k) { return mul_mod(x, comp(e0, k), m); });
    out[plane4 + i] = map4(c0, [&](uint32_t x, int k) {
      return add_mod(mul_mod(x, comp(e1, k), m), mul_mod(comp(c1, k), comp(e0, k), m), m.q);
    });
  }
}

// ModUp of one digit D = [d0, d0+nd) (coefficient domain x, [level][B][N]):
// y_i = x_i [(Q_D/q_i)^{-1}]_{q_i};  up[p] = sum_i y_i [Q_D/q_i]_{t(p)} for
// every extended-basis position p outside D (p < level: q-limb p; else
// p-limb L + p - level).
__global__ void __launch_bounds__(kThreads)
modup_kernel(const uint4* __restrict__ x, uint4* __restrict__ up,
             const ModConst* __restrict__ mods, const uint2* __restrict__ inv,
             const uint2* __restrict__ conv, uint32_t d0, uint32_t nd, uint32_t level, uint32_t L,
             uint32_t K, uint64_t bn4) {
  for (uint64_t pos = blockIdx.x * (uint64_t)kThreads + threadIdx.x; pos < bn4;
       pos += (uint64_t)gridDim.x * kThreads) {
    uint4 y[kMaxAlpha];
#pragma unroll
    for (int r = 0; r < kMaxAlpha; ++r) {
      if (r < (int)nd) {
        const uint32_t qi = mods[d0 + r].q;
        const uint2 c = inv[r];
        y[r] = map4(x[(uint64_t)(d0 + r) * bn4 + pos],
                    [&](uint32_t v, int) { return mul_shoup(v, c.x, c.y, qi); });
      }
    }
    const uint32_t ext = level + K;
    for (uint32_t p = 0; p < ext; ++p) {
      if (p >= d0 && p < d0 + nd) continue;
      const uint32_t t = p < level ? p : L + (p - level);
      const uint32_t m = mods[t].q;
      const uint2* c = conv + (uint64_t)t * kMaxAlpha;
      uint4 acc = make_uint4(0, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < kMaxAlpha; ++r)
        if (r < (int)nd) {
          const uint2 cr = c[r];
          acc = map4(acc, [&](uint32_t s, int k) {
            return add_mod(s, mul_shoup(comp(y[r], k), cr.x, cr.y, m), m);
          });
        }
      up[(uint64_t)p * bn4 + pos] = acc;
    }
  }
}

// acc_c[p] = sum_j dt_j[p] o key[j][c][t(p)] over the digits, where dt_j is
// d2 (NTT domain) on the digit's own limbs and the ModUp result elsewhere.
__global__ void __launch_bounds__(kThreads)
inner_product_kernel(const uint4* __restrict__ d2, const uint4* __restrict__ up,
                     const uint4* __restrict__ key, uint4* __restrict__ acc0,
                     uint4* __restrict__ acc1, const ModConst* __restrict__ mods,
                     uint32_t alpha, uint32_t ndigits, uint32_t level, uint32_t L, uint32_t K,
                     uint32_t batch, uint32_t log_n) {
  const uint32_t n4 = (1u << log_n) / 4;
  const uint64_t bn4 = (uint64_t)batch * n4;
  const uint64_t total = (uint64_t)(level + K) * bn4;
  const uint64_t key_plane = (uint64_t)(L + K) * n4;  // one key component
  for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * kThreads) {
    const uint32_t p = (uint32_t)(i / bn4);
    const uint32_t coef = (uint32_t)(i % n4);
    const uint32_t t = p < level ? p : L + (p - level);
    const ModConst m = mods[t];
    uint4 s0 = make_uint4(0, 0, 0, 0), s1 = s0;
    for (uint32_t j = 0; j < ndigits; ++j) {
      const bool own = p < level && p / alpha == j;
      const uint4 v = own ? d2[i] : up[(uint64_t)j * total + i];
      const uint4* kj = key + (uint64_t)j * 2 * key_plane + (uint64_t)t * n4 + coef;
      const uint4 k0 = kj[0], k1 = kj[key_plane];
      s0 = map4(s0, [&](uint32_t a, int c) { return add_mod(a, mul_mod(comp(v, c), comp(k0, c), m), m.q); });
      s1 = map4(s1, [&](uint32_t a, int c) { return add_mod(a, mul_mod(comp(v, c), comp(k1, c), m), m.q); });
    }
    acc0[i] = s0;
    acc1[i] = s1;
  }
}

// ModDown conversion: y_k = a_k [(P/p_k)^{-1}]_{p_k} (coefficient domain
// p-limbs a, [K][B][N]); conv_i = sum_k y_k [P/p_k]_{q_i} for i < level.
__global__ void __launch_bounds__(kThreads)
moddown_conv_kernel(const uint4* __restrict__ a, uint4* __restrict__ conv,
                    const ModConst* __restrict__ mods, const uint2* __restrict__ invp,
                    const uint2* __restrict__ cp, uint32_t level, uint32_t L, uint32_t K,
                    uint64_t bn4) {
  for (uint64_t pos = blockIdx.x * (uint64_t)kThreads + threadIdx.x; pos < bn4;
       pos += (uint64_t)gridDim.x * kThreads) {
    uint4 y[kMaxK];
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
      if (k < (int)K) {
        const uint32_t pk = mods[L + k].q;
        const uint2 c = invp[k];
        y[k] = map4(a[(uint64_t)k * bn4 + pos], [&](uint32_t v, int) { return mul_shoup(v, c.x, c.y, pk); });
      }
    for (uint32_t i = 0; i < level; ++i) {
      const uint32_t qi = mods[i].q;
      const uint2* c = cp + (uint64_t)i * kMaxK;
      uint4 acc = make_uint4(0, 0, 0, 0);
#pragma unroll
      for (int k = 0; k < kMaxK; ++k)
        if (k < (int)K) {
          const uint2 ck = c[k];
          acc = map4(acc, [&](uint32_t s, int j) {
            return add_mod(s, mul_shoup(comp(y[k], j), ck.x, ck.y, qi), qi);
          });
        }
      conv[(uint64_t)i * bn4 + pos] = acc;
    }
  }
}

// out_i (+)= (acc_i - conv_i) [P^{-1}]_{q_i}  (NTT domain, q-limbs).
template <bool kAccumulate>
__global__ void __launch_bounds__(kThreads)
moddown_final_kernel(const uint4* __restrict__ acc, const uint4* __restrict__ conv,
                     uint4* __restrict__ out, const ModConst* __restrict__ mods,
                     const uint2* __restrict__ pinv, uint64_t total4, uint64_t bn4) {
  for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < total4;
       i += (uint64_t)gridDim.x * kThreads) {
    const uint32_t l = (uint32_t)(i / bn4);
    const uint32_t q = mods[l].q;
    const uint2 c = pinv[l];
    const uint4 a = acc[i], b = conv[i];
    uint4 v = map4(a, [&](uint32_t x, int k) { return mul_shoup(sub_mod(x, comp(b, k), q), c.x, c.y, q); });
    if (kAccumulate) {
      const uint4 o = out[i];
      v = map4(v, [&](uint32_t x, int k) { return add_mod(x, comp(o, k), q); });
    }
    out[i] = v;
  }
}

// RESCALE broadcast: t holds the two components' top limbs in the
// coefficient domain, [2][B][N] in [0, q_top); u[c][i] = t[c] mod q_i for
// i < top.  Every modulus exceeds 2^29 and t < 2^31 < 4 q_i, so two
// conditional subtractions reduce exactly.
__global__ void __launch_bounds__(kThreads)
rescale_bcast_kernel(const uint4* __restrict__ t, uint4* __restrict__ u,
                     const ModConst* __restrict__ mods, uint32_t top, uint64_t bn4) {
  for (uint64_t pos = blockIdx.x * (uint64_t)kThreads + threadIdx.x; pos < 2 * bn4;
       pos += (uint64_t)gridDim.x * kThreads) {
    const uint64_t c = pos / bn4, r = pos - c * bn4;
    const uint4 x = t[pos];
    uint4* dst = u + c * top * bn4 + r;
    for (uint32_t i = 0; i < top; ++i) {
      const uint32_t q = mods[i].q, q2 = 2 * q;
      dst[(uint64_t)i * bn4] = map4(x, [&](uint32_t v, int) {
        v = v >= q2 ? v - q2 : v;
        return v >= q ? v - q : v;
      });
    }
  }
}

}  // namespace

hipError_t launch_rescale_bcast(const uint32_t* t, uint32_t* u, const ModConst* mods,
                                uint32_t top, uint32_t batch, uint32_t n, hipStream_t s) {
  const uint64_t bn4 = (uint64_t)batch * n / 4;
  TFHE_TIMED(K_RS_BCAST, s, hipLaunchKernelGGL(rescale_bcast_kernel, dim3(grid_for(2 * bn4)), dim3(kThreads),
                                               0, s, (const uint4*)t, (uint4*)u, mods, top, bn4));
  return hipGetLastError();
}

hipError_t launch_tensor(const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t* d2,
                         const ModConst* mods, uint32_t level, uint32_t batch, uint32_t n,
                         hipStream_t s) {
  const uint64_t per_limb4 = (uint64_t)batch * n / 4, plane4 = per_limb4 * level;
  TFHE_TIMED(K_TENSOR, s, hipLaunchKernelGGL(tensor_kernel, dim3(grid_for(plane4)), dim3(kThreads), 0, s,
                                             (const uint4*)a, (const uint4*)b, (uint4*)out, (uint4*)d2,
                                             mods, plane4, per_limb4));
  return hipGetLastError();
}

hipError_t launch_modup(const uint32_t* x, uint32_t* up, const ModConst* mods, const uint2* inv,
                        const uint2* conv, uint32_t d0, uint32_t nd, uint32_t level, uint32_t L,
                        uint32_t K, uint32_t batch, uint32_t n, hipStream_t s) {
  const uint64_t bn4 = (uint64_t)batch * n / 4;
  TFHE_TIMED(K_MODUP, s, hipLaunchKernelGGL(modup_kernel, dim3(grid_for(bn4)), dim3(kThreads), 0, s,
                                            (const uint4*)x, (uint4*)up, mods, inv, conv, d0, nd, level,
                                            L, K, bn4));
  return hipGetLastError();
}

hipError_t launch_inner_product(const uint32_t* d2, const uint32_t* up, const uint32_t* key,
                                uint32_t* acc0, uint32_t* acc1, const ModConst* mods,
                                uint32_t alpha, uint32_t ndigits, uint32_t level, uint32_t L,
                                uint32_t K, uint32_t batch, uint32_t log_n, hipStream_t s) {
  const uint64_t total4 = ((uint64_t)(level + K) * batch << log_n) / 4;
  TFHE_TIMED(K_INNER, s, hipLaunchKernelGGL(inner_product_kernel, dim3(grid_for(total4)), dim3(kThreads), 0, s,
                                            (const uint4*)d2, (const uint4*)up, (const uint4*)key,
                                            (uint4*)acc0, (uint4*)acc1, mods, alpha, ndigits, level, L, K,
                                            batch, log_n));
  return hipGetLastError();
}

hipError_t launch_moddown_conv(const uint32_t* a, uint32_t* conv, const ModConst* mods,
                               const uint2* invp, const uint2* cp, uint32_t level, uint32_t L,
                               uint32_t K, uint32_t batch, uint32_t n, hipStream_t s) {
  const uint64_t bn4 = (uint64_t)batch * n / 4;
  TFHE_TIMED(K_MD_CONV, s, hipLaunchKernelGGL(moddown_conv_kernel, dim3(grid_for(bn4)), dim3(kThreads), 0, s,
                                              (const uint4*)a, (uint4*)conv, mods, invp, cp, level, L, K,
                                              bn4));
  return hipGetLastError();
}

hipError_t launch_moddown_final(const uint32_t* acc, const uint32_t* conv, uint32_t* out,
                                const ModConst* mods, const uint2* pinv, uint32_t level,
                                uint32_t batch, uint32_t n, bool accumulate, hipStream_t s,
                                KernelId id) {
  const uint64_t bn4 = (uint64_t)batch * n / 4, total4 = bn4 * level;
  const uint4 *A = (const uint4*)acc, *C = (const uint4*)conv;
  uint4* O = (uint4*)out;
  if (accumulate)
    TFHE_TIMED(id, s, hipLaunchKernelGGL(moddown_final_kernel<true>, dim3(grid_for(total4)),
                                                 dim3(kThreads), 0, s, A, C, O, mods, pinv, total4, bn4));
  else
    TFHE_TIMED(id, s, hipLaunchKernelGGL(moddown_final_kernel<false>, dim3(grid_for(total4)),
                                                 dim3(kThreads), 0, s, A, C, O, mods, pinv, total4, bn4));
  return hipGetLastError();
}

}  // namespace tfhe
