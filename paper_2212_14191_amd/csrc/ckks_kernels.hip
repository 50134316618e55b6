// Kernels of HMULT / HROTATE / RESCALE other than the NTT (Sec. IV-A, Table 2):
// the tensor product (Hada-Mult, Ele-Add), the fast basis conversion (Conv)
// of ModUp and ModDown, the key-switching inner product (Hada-Mult, Ele-Add)
// and the ModDown finalisation (Ele-Sub, Hada-Mult).  All run over the
// (limb, batch, N) layout, one thread per coefficient position, so each
// limb-plane access is a coalesced stream.
#include <algorithm>

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
// d2 (NTT domain) on the digit's own limbs and the ModUp result elsewhere;
// blockIdx.y selects the level group.  Products are summed as 64-bit values
// below q 2^32 and reduced once per output.
__global__ void __launch_bounds__(kThreads)
inner_product_kernel(const IpSet set, const ModConst* __restrict__ mods, uint32_t log_n) {
  const IpGroup& G = set.g[blockIdx.y];
  const uint32_t n4 = (1u << log_n) / 4;
  const uint64_t bn4 = (uint64_t)G.batch * n4;
  const uint64_t total = (uint64_t)(G.level + set.K) * bn4;
  const uint64_t key_plane = (uint64_t)(set.L + set.K) * n4;  // one key component
  const uint4* d2 = (const uint4*)G.d2;
  const uint4* up = (const uint4*)G.src;
  uint4* acc0 = (uint4*)G.acc;
  uint4* acc1 = acc0 + total;
  for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * kThreads) {
    const uint32_t p = (uint32_t)(i / bn4);
    const uint32_t coef = (uint32_t)(i % n4);
    const uint32_t t = p < G.level ? p : set.L + (p - G.level);
    const ModConst m = mods[t];
    // the key of this element (one key for all when count = 1)
    const uint32_t e = (uint32_t)((i % bn4) / n4);
    const uint4* key = (const uint4*)set.keys.k[set.keys.count == 1 ? 0 : G.key0 + e];
    uint64_t s0[4] = {0, 0, 0, 0}, s1[4] = {0, 0, 0, 0};  // below q 2^32
    for (uint32_t j = 0; j < G.digits; ++j) {
      const bool own = p < G.level && p / set.alpha == j;
      const uint4 v = own ? d2[i] : up[(uint64_t)j * total + i];
      const uint4* kj = key + (uint64_t)j * 2 * key_plane + (uint64_t)t * n4 + coef;
      const uint4 k0 = kj[0], k1 = kj[key_plane];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        s0[c] = mac_lazy(s0[c], comp(v, c), comp(k0, c), m.q);
        s1[c] = mac_lazy(s1[c], comp(v, c), comp(k1, c), m.q);
      }
    }
    acc0[i] = make_uint4(reduce_lazy(s0[0], m), reduce_lazy(s0[1], m), reduce_lazy(s0[2], m), reduce_lazy(s0[3], m));
    acc1[i] = make_uint4(reduce_lazy(s1[0], m), reduce_lazy(s1[1], m), reduce_lazy(s1[2], m), reduce_lazy(s1[3], m));
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

// Basis conversion (the Conv kernel of ModUp / ModDown) as a skinny matrix
// product on the INT8 matrix cores: D[t][pos] = sum_{r,d} A[t][(r,d)] *
// digit_d(y_r[pos]), K = 4 digits x 8 inputs = 32 with
// v_mfma_i32_16x16x32_i8, one product per digit plane j of the constants
// (A_j[t][(r,d)] = digit j of 2^{8d} C[t][r] 2^32 mod m_t), fused as in the
// four-step NTT: V = (C_0 + 2^8 C_1) + 2^16 (C_2 + 2^8 C_3), one Montgomery
// step (the 2^32 in the constants cancels it), one conditional subtraction.
// The inputs enter as y_r - 2^30 in [-2^30, 2^30), inside the digit window
// for every modulus below 2^31; the offset comes back as the per-target
// constant 2^30 sum_r C[t][r] mod m_t.  Lane (n, g) loads four consecutive positions 4n..4n+3 of inputs 2g and
// 2g+1 (16-byte loads) and the product for sub-tile p pairs MFMA column n
// with position 4n + p; after the four sub-tiles it holds targets 4g..4g+3
// at positions 4n..4n+3 and stores them as 16-byte runs.
typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t conv_fuse(int c0, int c1, int c2, int c3, uint32_t q, uint32_t qneg) {
  const uint32_t lo = (uint32_t)c0 + ((uint32_t)c1 << 8);
  const uint32_t hi = (uint32_t)c2 + ((uint32_t)c3 << 8);
  const uint64_t V = ((uint64_t)hi << 16) + lo;
  const uint32_t m = (uint32_t)V * qneg;
  // V + m q is a multiple of 2^32 below 2^64: its high word is exact
  return reduce_once((uint32_t)(((uint64_t)m * q + V) >> 32), q);
}

// The per-target constants (A operands, moduli, Montgomery and offset
// constants) are read from the context's tables into LDS and read there per
// use, which keeps the kernel at four resident waves per SIMD for latency
// hiding; targets beyond nout have zero operands and modulus 1 (their
// results are not stored).  Conversions of one launch may differ in plane
// size: the grid covers the largest, and the workgroups beyond a smaller
// one's chunks leave at once.
__global__ void __launch_bounds__(kThreads, 4)
conv_mfma_kernel(const ConvSet set) {
  const ConvDesc& a = set.d[blockIdx.y];
  const ConvTabs& tb = set.tabs;
  const uint64_t chunks = a.plane / 64;
  if ((uint64_t)blockIdx.x * (kThreads / 64) >= chunks) return;  // the whole workgroup
  const bool up = a.key_idx != kConvDown;
  // plan limb of target t of this descriptor
  auto limb_of = [&](uint32_t t) {
    const uint32_t pos = conv_pos(a, a.first + t);
    return pos < a.level ? pos : tb.L + (pos - a.level);
  };
  __shared__ __attribute__((aligned(16))) uint32_t s_a[kConvMaxOut * 32];
  __shared__ __attribute__((aligned(16))) uint32_t s_q[kConvMaxOut], s_qn[kConvMaxOut], s_k[kConvMaxOut];
  for (int i = threadIdx.x; i < kConvMaxOut * 32; i += kThreads) {
    const uint32_t t = i / 32;
    const uint32_t* row = t < a.nout ? (up ? tb.up_mfma + ((size_t)a.key_idx * (tb.L + tb.K) + limb_of(t)) * 32
                                           : tb.dn_mfma + (size_t)limb_of(t) * 32)
                                     : nullptr;
    s_a[i] = row ? row[i % 32] : 0u;
  }
  if (threadIdx.x < kConvMaxOut) {
    const uint32_t t = threadIdx.x;
    const bool live = t < a.nout;
    const uint32_t l = live ? limb_of(t) : 0;
    s_q[t] = live ? tb.mods[l].q : 1u;
    s_qn[t] = live ? tb.mods[l].qneg : 0u;
    s_k[t] = live ? (up ? tb.up_k[(size_t)a.key_idx * (tb.L + tb.K) + l] : tb.dn_k[l]) : 0u;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
  const uint64_t wave_id = (blockIdx.x * (uint64_t)kThreads + threadIdx.x) / 64;
  const uint64_t waves = (uint64_t)gridDim.x * (kThreads / 64);
  const int r0 = 2 * g, r1 = 2 * g + 1;
  const bool h0 = r0 < (int)a.nin, h1 = r1 < (int)a.nin;
  // input r: ModUp q-limb d0 + r with [(Q_D/q_r)^{-1}]; ModDown p-limb r with [(P/p_r)^{-1}]
  auto in_q = [&](int r) { return tb.mods[up ? a.d0 + r : tb.L + r].q; };
  auto in_mult = [&](int r) { return up ? tb.up_inv[(size_t)a.key_idx * kMaxAlpha + r] : tb.dn_invp[r]; };
  const uint32_t q0 = h0 ? in_q(r0) : 1, q1 = h1 ? in_q(r1) : 1;
  const uint2 m0 = h0 ? in_mult(r0) : make_uint2(0, 0), m1 = h1 ? in_mult(r1) : make_uint2(0, 0);
  const int blocks = a.nout > 16 ? 2 : 1;
  const v4i zero = {0, 0, 0, 0};
  // the next chunk's inputs are loaded while this one is converted
  uint4 nx0 = make_uint4(0, 0, 0, 0), nx1 = nx0;
  if (wave_id < chunks) {
    if (h0) nx0 = *(const uint4*)(a.in + (uint64_t)r0 * a.plane + wave_id * 64 + 4 * n);
    if (h1) nx1 = *(const uint4*)(a.in + (uint64_t)r1 * a.plane + wave_id * 64 + 4 * n);
  }
  for (uint64_t c = wave_id; c < chunks; c += waves) {
    const uint64_t pos = c * 64 + 4 * n;
    const uint4 x0 = nx0, x1 = nx1;
    if (c + waves < chunks) {
      if (h0) nx0 = *(const uint4*)(a.in + (uint64_t)r0 * a.plane + pos + waves * 64);
      if (h1) nx1 = *(const uint4*)(a.in + (uint64_t)r1 * a.plane + pos + waves * 64);
    }
    // y = x * mult mod q in [0, q), then the digits of y - 2^30
    const uint4 d0 = map4(x0, [&](uint32_t v, int) {
      return h0 ? balanced_digits((int32_t)(mul_shoup(v, m0.x, m0.y, q0) - (1u << 30))) : 0u;
    });
    const uint4 d1 = map4(x1, [&](uint32_t v, int) {
      return h1 ? balanced_digits((int32_t)(mul_shoup(v, m1.x, m1.y, q1) - (1u << 30))) : 0u;
    });
    for (int b = 0; b < blocks; ++b) {
      // A rows: target 16 b + n, K slice 8 g .. 8 g + 7 of each digit plane j
      long av[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) av[j] = *(const long*)(s_a + (16 * b + n) * 32 + 8 * j + 2 * g);
      const int t0 = 16 * b + 4 * g;  // this lane's output targets t0 .. t0 + 3
      const uint4 tq = *(const uint4*)(s_q + t0), tn = *(const uint4*)(s_qn + t0);
      const v4i bias = {(int)tq.x, (int)tq.y, (int)tq.z, (int)tq.w};
      uint32_t res[4][4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const long bv = (long)((uint64_t)comp(d0, p) | ((uint64_t)comp(d1, p) << 32));
        const v4i c0 = __builtin_amdgcn_mfma_i32_16x16x32_i8(av[0], bv, bias, 0, 0, 0);
        const v4i c1 = __builtin_amdgcn_mfma_i32_16x16x32_i8(av[1], bv, zero, 0, 0, 0);
        const v4i c2 = __builtin_amdgcn_mfma_i32_16x16x32_i8(av[2], bv, bias, 0, 0, 0);
        const v4i c3 = __builtin_amdgcn_mfma_i32_16x16x32_i8(av[3], bv, zero, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) res[i][p] = conv_fuse(c0[i], c1[i], c2[i], c3[i], comp(tq, i), comp(tn, i));
        // one sub-tile's products in flight at a time (register budget)
        __builtin_amdgcn_sched_barrier(0);
      }
      const uint4 tk = *(const uint4*)(s_k + t0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t t = t0 + i, q = comp(tq, i), k = comp(tk, i);
        if (t < a.nout)
          *(uint4*)(a.out + (uint64_t)conv_pos(a, a.first + t) * a.plane + pos) =
              make_uint4(add_mod(res[i][0], k, q), add_mod(res[i][1], k, q), add_mod(res[i][2], k, q),
                         add_mod(res[i][3], k, q));
      }
    }
  }
}

// FrobeniusMap out_j = in_{pi(j)} of two arrays in one launch (the two
// components of a ciphertext), with the Galois element of each row's batch
// element.
__global__ void __launch_bounds__(kThreads)
frobenius_pair_kernel(const uint32_t* __restrict__ in0, uint32_t* __restrict__ out0,
                      const uint32_t* __restrict__ in1, uint32_t* __restrict__ out1, const GaloisSet gs,
                      uint64_t per, uint32_t log_n) {
  const uint32_t n = 1u << log_n, mask2n = 2 * n - 1;
  for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < 2 * per;
       i += (uint64_t)gridDim.x * kThreads) {
    const bool second = i >= per;
    const uint64_t k = second ? i - per : i;
    const uint32_t j = (uint32_t)(k & (n - 1));
    const uint32_t galois = gs.g[(uint32_t)((k >> log_n) % gs.batch)];
    const uint32_t src = (((2 * j + 1) * galois) & mask2n) >> 1;
    (second ? out1 : out0)[k] = (second ? in1 : in0)[(k - j) + src];
  }
}

// Tensor product of the ciphertext pairs of a mixed-level batch, blockIdx.y
// selecting the pair: element i = limb N/4 + k of its inputs goes to
// (limb B + idx) N/4 + k of its group's planes.
__global__ void __launch_bounds__(kThreads)
tensor_multi_kernel(const CtDescSet set, const ModConst* __restrict__ mods, uint32_t log_n4) {
  const CtDesc& c = set.c[blockIdx.y];
  const uint64_t n4 = 1ull << log_n4, per4 = (uint64_t)c.level << log_n4;
  const uint64_t gplane4 = per4 * c.B;  // one component of the group
  const uint4* A = (const uint4*)c.a;
  const uint4* B = (const uint4*)c.b;
  uint4* out = (uint4*)c.out;
  uint4* d2 = (uint4*)c.d;
  for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < per4;
       i += (uint64_t)gridDim.x * kThreads) {
    const uint32_t limb = (uint32_t)(i >> log_n4);
    const uint64_t o = (((uint64_t)limb * c.B + c.idx) << log_n4) + (i & (n4 - 1));
    const ModConst m = mods[limb];
    const uint4 c0 = A[i], c1 = A[per4 + i], e0 = B[i], e1 = B[per4 + i];
    d2[o] = map4(c1, [&](uint32_t x, int k) { return mul_mod(x, comp(e1, k), m); });
    out[o] = map4(c0, [&](uint32_t x, int k) { return mul_mod(x, comp(e0, k), m); });
    out[gplane4 + o] = map4(c0, [&](uint32_t x, int k) {
      return add_mod(mul_mod(x, comp(e1, k), m), mul_mod(comp(c1, k), comp(e0, k), m), m.q);
    });
  }
}

// FrobeniusMap of both components of each ciphertext of a mixed-level batch
// (blockIdx.y selects it, with its own Galois element): out_j = in_{pi(j)}
// per limb; component 0 to out, component 1 to d, at (limb B + idx) N.
__global__ void __launch_bounds__(kThreads)
frobenius_multi_kernel(const CtDescSet set, uint32_t log_n) {
  const CtDesc& c = set.c[blockIdx.y];
  const uint32_t n = 1u << log_n, mask2n = 2 * n - 1;
  const uint64_t per = (uint64_t)c.level << log_n;
  for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < 2 * per;
       i += (uint64_t)gridDim.x * kThreads) {
    const bool second = i >= per;
    const uint64_t k = second ? i - per : i;
    const uint32_t j = (uint32_t)(k & (n - 1)), limb = (uint32_t)(k >> log_n);
    const uint32_t src = (((2 * j + 1) * c.galois) & mask2n) >> 1;
    const uint64_t o = (((uint64_t)limb * c.B + c.idx) << log_n) + j;
    (second ? c.d : c.out)[o] = c.a[(second ? per : 0) + ((uint64_t)limb << log_n) + src];
  }
}

// Copies each ciphertext of a mixed-level batch out of its level group's
// result [2][level][B][N] (element e.b[r]) to its own [2][level][N]
// (e.dst[r]); blockIdx.y selects the ciphertext, 16 bytes per element.
__global__ void __launch_bounds__(kThreads)
scatter_kernel(const ScatterSet e, uint32_t log_n4) {
  const uint32_t r = blockIdx.y;
  const uint64_t n4 = 1ull << log_n4, total = (uint64_t)e.rows[r] << log_n4;
  const uint4* src = (const uint4*)e.src[r];
  uint4* dst = (uint4*)e.dst[r];
  for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * kThreads) {
    const uint64_t row = i >> log_n4;
    dst[i] = src[((row * e.batch[r] + e.b[r]) << log_n4) + (i & (n4 - 1))];
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

hipError_t launch_conv_mfma(const ConvSet& set, uint32_t num_cus, KernelId id, hipStream_t s) {
  uint64_t chunks = 0;  // the largest conversion's
  for (uint32_t k = 0; k < set.count; ++k) chunks = std::max<uint64_t>(chunks, set.d[k].plane / 64);
  const uint64_t blocks = (chunks + 3) / 4;  // 4 waves per block, one chunk each per round
  // about one resident round (four workgroups per CU): each wave then
  // converts several chunks with its next inputs in flight
  const uint64_t resident = 4ull * (num_cus ? num_cus : 1);
  const uint32_t grid = (uint32_t)(blocks < resident ? (blocks ? blocks : 1) : resident);
  TFHE_TIMED(id, s, hipLaunchKernelGGL(conv_mfma_kernel, dim3(grid, set.count), dim3(kThreads), 0, s, set));
  return hipGetLastError();
}

hipError_t ConvQueue::flush(uint32_t num_cus, KernelId id, hipStream_t s) {
  for (size_t i = 0; i < q.size();) {
    ConvSet set{};
    set.tabs = tabs;
    set.count = 0;
    while (i < q.size() && set.count < (uint32_t)kConvPerLaunch) set.d[set.count++] = q[i++];
    hipError_t e = launch_conv_mfma(set, num_cus, id, s);
    if (e != hipSuccess) {
      q.clear();
      return e;
    }
  }
  q.clear();
  return hipSuccess;
}

hipError_t launch_frobenius_pair(const uint32_t* in0, uint32_t* out0, const uint32_t* in1, uint32_t* out1,
                                 const GaloisSet& gs, uint32_t rows, uint32_t log_n, hipStream_t s) {
  const uint64_t per = (uint64_t)rows << log_n;
  TFHE_TIMED(K_FROB, s, hipLaunchKernelGGL(frobenius_pair_kernel, dim3(grid_for(2 * per)), dim3(kThreads), 0, s,
                                           in0, out0, in1, out1, gs, per, log_n));
  return hipGetLastError();
}

// blocks per ciphertext of a CtDescSet launch: the grid covers the largest
uint32_t multi_grid(const CtDescSet& set, uint32_t per_level) {
  uint32_t lv = 0;
  for (uint32_t r = 0; r < set.count; ++r) lv = std::max(lv, set.c[r].level);
  return std::max<uint32_t>(1, std::min<uint32_t>(grid_for((uint64_t)lv * per_level), 1024));
}

hipError_t launch_tensor_multi(const CtDescSet& set, const ModConst* mods, uint32_t log_n, hipStream_t s) {
  if (set.count == 0) return hipSuccess;
  TFHE_TIMED(K_TENSOR, s, hipLaunchKernelGGL(tensor_multi_kernel, dim3(multi_grid(set, (1u << log_n) / 4), set.count),
                                             dim3(kThreads), 0, s, set, mods, log_n - 2));
  return hipGetLastError();
}

hipError_t launch_frobenius_multi(const CtDescSet& set, uint32_t log_n, hipStream_t s) {
  if (set.count == 0) return hipSuccess;
  TFHE_TIMED(K_FROB, s, hipLaunchKernelGGL(frobenius_multi_kernel, dim3(multi_grid(set, 2u << log_n), set.count),
                                           dim3(kThreads), 0, s, set, log_n));
  return hipGetLastError();
}

hipError_t launch_scatter(const ScatterSet& e, uint32_t count, uint32_t log_n, hipStream_t s) {
  if (count == 0) return hipSuccess;
  uint32_t rows = 0;
  for (uint32_t r = 0; r < count; ++r) rows = std::max(rows, e.rows[r]);
  const uint64_t per = ((uint64_t)rows << log_n) / 4;
  const uint32_t gx = std::max<uint32_t>(1, std::min<uint32_t>(grid_for(per), 1024));
  hipLaunchKernelGGL(scatter_kernel, dim3(gx, count), dim3(kThreads), 0, s, e, log_n - 2);
  return hipGetLastError();
}

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

hipError_t launch_inner_product(const IpSet& set, const ModConst* mods, uint32_t log_n, hipStream_t s) {
  if (set.count == 0) return hipSuccess;
  uint64_t most = 0;  // the largest group's elements (16 bytes each)
  for (uint32_t g = 0; g < set.count; ++g)
    most = std::max<uint64_t>(most, ((uint64_t)(set.g[g].level + set.K) * set.g[g].batch << log_n) / 4);
  // one block column per group; about 16384 blocks over the whole launch
  const uint32_t gx = std::max<uint32_t>(1, std::min<uint32_t>(grid_for(most), std::max<uint32_t>(64, 16384 / set.count)));
  TFHE_TIMED(K_INNER, s, hipLaunchKernelGGL(inner_product_kernel, dim3(gx, set.count), dim3(kThreads), 0, s, set,
                                            mods, log_n));
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
