// One-pass four-step NTT (Sec. IV-B/IV-C, Eq. 9 and Eq. 10) for N = N1 x 256,
// N = 2^12..2^15: the same two matrix-core stages as the two-pass kernels
// (ntt_fourstep.hip: the map n = 256 n1 + n2, k = k1 + N1 k2, byte-digit
// contractions, Montgomery fusion, twists), but a workgroup keeps whole
// polynomials in LDS, so each polynomial crosses HBM once in each direction
// instead of twice (the paper's Stages 1-5 as one pipeline per transform).
//
// Per polynomial: direct-to-LDS loads of the natural-order input; pass 1
// (the first stage over the columns of the P1 x S view) in place; pass 2
// (the second stage over its rows), whose results are held in registers
// until every wave has read its rows, then written into LDS in natural output
// order (position = pass-1 index + P1 x pass-2 index); 16-byte streaming
// stores.  For N <= 2^14 a workgroup has 4 waves and one polynomial buffer,
// so that two or three workgroups share a CU: one's loads and stores overlap
// the others' arithmetic (measured faster than one 8-wave workgroup that
// double-buffers: 1.2-1.25 x at 2^13 and 2^14).  At 2^15 the polynomial
// takes 128 KiB and one workgroup of 8 waves owns the CU.
//
// LDS layout: 1 KiB chunks of the polynomial in order; inside a chunk the
// 16-byte quads are XOR-swizzled (quad Q at Q ^ X, X a function of the chunk
// and of Q's bits 4-5, below 16), which the direct-to-LDS loads realise by
// choosing each lane's global address.  The constants make every access of
// both passes free of bank conflicts (64 banks; 16 lanes per 16-byte access,
// 64 per 4-byte access), verified by enumeration of the access patterns.
// The output order uses its own swizzle.
//
// The first pass's post-twist P(column, output) is split into a factor fixed
// per lane (Shoup form, staged in LDS, or read through the caches at 2^14
// where two workgroups' polynomials fill the LDS) and a factor per step
// (Montgomery form, in registers).
#include "fourstep_dev.hpp"

namespace tfhe {
namespace {

// Per (log N, direction): waves per workgroup, polynomial buffers, and the
// swizzle constants: input X = (a c + b (Q >> 4)) & 15; output
// X = (a c + b (Q >> sh)) & (2^sh - 1), with c the chunk and Q the quad.
template <int kLogN, bool kInv>
struct OpCfg;
#define TFHE_OPCFG(LN, INV, W, B, IA, IB, OA, OB, OS, PB)                   \
  template <>                                                              \
  struct OpCfg<LN, INV> {                                                  \
    static constexpr int waves = W, bufs = B;                              \
    static constexpr uint32_t in_a = IA, in_b = IB, out_a = OA, out_b = OB; \
    static constexpr uint32_t out_sh = OS;                                 \
    static constexpr bool pb_lds = PB;                                     \
  };
TFHE_OPCFG(12, false, 4, 1, 1, 4, 0, 1, 4, true)
TFHE_OPCFG(13, false, 4, 1, 9, 4, 1, 1, 3, true)
TFHE_OPCFG(14, false, 4, 1, 5, 4, 1, 4, 4, false)
TFHE_OPCFG(15, false, 8, 1, 9, 4, 1, 4, 4, true)
TFHE_OPCFG(12, true, 4, 1, 4, 1, 1, 0, 4, true)
TFHE_OPCFG(13, true, 4, 1, 4, 1, 1, 0, 4, true)
TFHE_OPCFG(14, true, 4, 1, 4, 1, 1, 0, 4, false)
TFHE_OPCFG(15, true, 8, 1, 5, 4, 1, 0, 4, true)
#undef TFHE_OPCFG

template <uint32_t kA, uint32_t kB>
__device__ __forceinline__ uint32_t sw_in(uint32_t w) {
  const uint32_t c = w >> 8, Q = (w >> 2) & 63u;
  const uint32_t X = (kA * c + kB * (Q >> 4)) & 15u;
  return (c << 8) | ((Q ^ X) << 2) | (w & 3u);
}

template <uint32_t kA, uint32_t kB, uint32_t kSh>
__device__ __forceinline__ uint32_t sw_out(uint32_t w) {
  const uint32_t c = w >> 8, Q = (w >> 2) & 63u;
  const uint32_t X = (kA * c + kB * (Q >> kSh)) & ((1u << kSh) - 1u);
  return (c << 8) | ((Q ^ X) << 2) | (w & 3u);
}

// The value, opaque to the optimiser: address arithmetic derived from it is
// recomputed where it is used instead of being hoisted out of the
// polynomial loop, where dozens of precomputed LDS addresses would occupy
// registers for the whole kernel.
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <int kLogN, bool kInv>
__global__ void __launch_bounds__((64 * OpCfg<kLogN, kInv>::waves), (OpCfg<kLogN, kInv>::waves <= 4 ? 2 : 1))
op_kernel(const FsTable tab) {
  using C = OpCfg<kLogN, kInv>;
  constexpr int N = 1 << kLogN, N1 = N >> 8;
  constexpr int kR1 = kInv ? 16 : N1 / 16, kR2 = kInv ? N1 / 16 : 16;
  constexpr int P1 = 16 * kR1, S = N / P1;   // pass 1: S columns of P1 points
  constexpr int Mt1 = 16 / kR1, Mt2 = 16 / kR2;
  constexpr int W = C::waves, NB = C::bufs;
  constexpr int St1 = S / (4 * Mt1) / W, St2 = P1 / (4 * Mt2) / W;  // steps per wave
  constexpr int CH = N / 256 / W;  // 1 KiB chunks per wave and polynomial
  constexpr bool kUA = kInv;       // second-pass level-A index u = g + 4c
  static_assert(St1 >= 1 && St2 >= 1 && CH >= 1, "shape");
  static_assert(3 * CH <= 63, "vmcnt range");
  // polynomial buffers, then the limb's matrix-core operands and twists
  // (both passes) and the per-lane post-twist factors, staged once per limb
  // (the post-twist factors stay in global memory, read per polynomial
  // through the caches, where LDS must hold two workgroups' polynomials)
  constexpr bool kPbLds = C::pb_lds;
  constexpr int kTabOpA1 = NB * N, kTabTw1 = kTabOpA1 + 1024, kTabOpA2 = kTabTw1 + 512;
  constexpr int kTabTw2 = kTabOpA2 + 1024, kTabPb = kTabTw2 + 512, kLdsWords = kTabPb + (kPbLds ? 2048 : 0);
  __shared__ __attribute__((aligned(16))) uint32_t lds[kLdsWords];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const uint32_t p_begin = (uint32_t)((uint64_t)blockIdx.x * tab.total / gridDim.x);
  const uint32_t p_end = (uint32_t)((uint64_t)(blockIdx.x + 1) * tab.total / gridDim.x);
  if (p_begin >= p_end) return;

  uint32_t kf = 0, kc = 0;  // running unit indices of the load and compute walks
  // direct-to-LDS loads of polynomial p into buffer b: chunk c = wave + k W;
  // LDS slot L of the chunk receives natural quad L ^ X(c, L >> 4)
  auto issue_load = [&](uint32_t p, int b) {
    const Item it = locate(tab, p, kf);
    const uint32_t* src = tab.u[it.unit].in + it.poly_base;
    const uint32_t al = (uint32_t)opaque(lane);
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const uint32_t c = wave + k * W;
      const uint32_t X = (C::in_a * c + C::in_b * (al >> 4)) & 15u;
      const uint32_t* gp = src + c * 256 + 4 * (al ^ X);
      const uint32_t lds_addr = (uint32_t)(uintptr_t)(lds_void_t*)(lds + b * N + c * 256);
      asm volatile(
          "s_mov_b32 m0, %0\n\t"
          "global_load_lds_dwordx4 %1, off nt"
          :
          : "s"(__builtin_amdgcn_readfirstlane(lds_addr)), "v"(gp)
          : "memory", "m0");
    }
  };
  issue_load(p_begin, 0);
  if (NB == 2 && p_begin + 1 < p_end) issue_load(p_begin + 1, 1);

  // per-limb values in registers (the rest of the limb's tables is in LDS)
  const FourStepLimb* cur_limb = nullptr;
  const uint2* pb_src = nullptr;  // the limb's post-twist factors (global)
  uint32_t q = 0, qneg = 0, nq = 0;
  uint64_t cq = 0;
  uint2 lb1[4], lb2[16];  // level-B constants (uniform: scalar registers)
  // post-twist step factors: the wave's first step's, and the ratio between
  // consecutive steps of a wave (the factor is geometric in the step index)
  uint32_t pa0[4], pad[4];

  uint32_t n = 0;
  for (uint32_t p = p_begin; p < p_end; ++p, ++n) {
    const int b = NB == 2 ? (int)(n & 1) : 0;
    uint32_t* const buf = lds + b * N;
    const Item it = locate(tab, p, kc);
    // this polynomial's loads: issued after them are, in order, the stores
    // of p - 2, the loads of p + 1 and the stores of p - 1 (double buffer),
    // or nothing (single buffer)
    if (NB == 2) {
      const int after = (n >= 2 ? CH : 0) + (p + 1 < p_end ? CH : 0) + (n >= 1 ? CH : 0);
      if (after >= 3 * CH) wait_vmcnt<3 * CH>();
      else if (after >= 2 * CH) wait_vmcnt<2 * CH>();
      else if (after >= CH) wait_vmcnt<CH>();
      else wait_vmcnt<0>();
    } else {
      wait_vmcnt<0>();  // the loads were issued last
    }
    const FourStepLimb* limb = tab.u[it.unit].limbs + it.limb;
    if (limb != cur_limb) {
      // rare (a few times per workgroup), and every wave is past the
      // previous polynomial's last barrier, so the staged tables are free:
      // copy the new limb's into LDS (waiting here keeps the pipeline free
      // of waits on these loads)
      const FourStepLimb L = *limb;
      const PassTables* T1 = L.pass1;
      const OnePassTables* O = L.op;
      q = L.q;
      qneg = L.qneg;
      nq = 0u - q;
      cq = (uint32_t)(0x80808080u - q);
      const uint32_t* srcs[5] = {&T1->opA[0][0][0], (const uint32_t*)&T1->twist[0][0], &O->p2.opA[0][0][0],
                                 (const uint32_t*)&O->p2.twist[0][0], (const uint32_t*)&O->post_b[0][0][0]};
      const int offs[5] = {kTabOpA1, kTabTw1, kTabOpA2, kTabTw2, kTabPb};
      const int lens[5] = {1024, 512, 1024, 512, 2048};
      pb_src = &O->post_b[0][0][0];
#pragma unroll
      for (int k = 0; k < (kPbLds ? 5 : 4); ++k)
        for (int i = 4 * tid; i < lens[k]; i += 4 * 64 * W)
          *(uint4*)(lds + offs[k] + i) = *(const uint4*)(srcs[k] + i);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (kR1 < 16) lb1[j] = T1->lb[j];

        pa0[j] = O->post_a[wave][lane][j];
        pad[j] = St1 > 1 ? O->post_a[W][lane][j] : 0u;
      }
      if (kR2 < 16) {
#pragma unroll
        for (int i = 0; i < 16; ++i) lb2[i] = O->p2.lb[i];
      }
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
      cur_limb = limb;
    }
    lds_barrier();  // the polynomial is in LDS (every wave's loads landed)

    const v4i bias = {(int)q, (int)q, (int)q, (int)q};
    const v4i zero = {0, 0, 0, 0};

    // ---- pass 1: columns, in place.  Lane (i, g) reads row
    // kR1 (4g + c) + i % kR1 of quad Q0 + i / kR1 (the four sets are the
    // quad's four columns) and writes output s + 16 t of column quad Q0 + m.
    auto pass1 = [&](auto big_q) {
      constexpr bool kBigQ = decltype(big_q)::value;
      v4i opA1[4];
      uint2 tw1[4], pb[4][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        opA1[j] = *(const v4i*)(lds + kTabOpA1 + (j * 64 + lane) * 4);
        tw1[j] = *(const uint2*)(lds + kTabTw1 + (lane * 4 + j) * 2);
#pragma unroll
        for (int sg = 0; sg < 4; ++sg)
          pb[j][sg] = kPbLds ? *(const uint2*)(lds + kTabPb + ((lane * 4 + j) * 4 + sg) * 2)
                             : pb_src[(lane * 4 + j) * 4 + sg];
      }
      uint32_t pa[4] = {pa0[0], pa0[1], pa0[2], pa0[3]};
#pragma unroll
      for (int st = 0; st < St1; ++st) {
        const int Q0 = (wave + st * W) * Mt1;
        const int ai = opaque(i16), ag = opaque(g);  // for addresses
        if (st > 0) {
#pragma unroll
          for (int j = 0; j < 4; ++j) pa[j] = mont_mul_lazy(pa[j], pad[j], q, qneg);
        }
        uint4 rows[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int row = kR1 * (4 * ag + c) + ai % kR1, quad = Q0 + ai / kR1;
          rows[c] = *(const uint4*)(buf + sw_in<C::in_a, C::in_b>(row * S + 4 * quad));
        }
        uint32_t o[4][4];  // [register j][set]
        uint2 rj[4];
        if (kR1 == 8) {
#pragma unroll
          for (int j = 0; j < 4; ++j) rj[j] = (g & 1) ? lb1[j] : lb1[0];
        }
#pragma unroll
        for (int sg = 0; sg < 4; ++sg) {
          v4i x;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const uint32_t w = sg == 0 ? rows[c].x : sg == 1 ? rows[c].y : sg == 2 ? rows[c].z : rows[c].w;
            x[c] = (int)balanced_digits(kBigQ ? to_window(w, q) : (int32_t)w);
          }
          const v4i a0 = mfma(x, opA1[0], bias);
          const v4i a1 = mfma(x, opA1[1], zero);
          const v4i a2 = mfma(x, opA1[2], bias);
          const v4i a3 = mfma(x, opA1[3], zero);
          uint32_t y[4];
          if (kR1 == 16) {
            v4i z;
#pragma unroll
            for (int j = 0; j < 4; ++j)
              z[j] = (int)twist_digits<kBigQ>(fuse_redc(a0[j], a1[j], a2[j], a3[j], q, qneg), tw1[j], q, nq, cq);
            // level B (only the inverse's 256-point stage here): the same
            // symmetric matrix, unscaled, so opB equals opA
            const v4i b0 = mfma(opA1[0], z, bias);
            const v4i b1 = mfma(opA1[1], z, zero);
            const v4i b2 = mfma(opA1[2], z, bias);
            const v4i b3 = mfma(opA1[3], z, zero);
#pragma unroll
            for (int j = 0; j < 4; ++j) y[j] = fuse_redc(b0[j], b1[j], b2[j], b3[j], q, qneg);
          } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
              y[j] = reduce_once(mul_shoup_lazy(fuse_redc(a0[j], a1[j], a2[j], a3[j], q, qneg), tw1[j].x,
                                                tw1[j].y, q), q);
            level_b<kR1>(y, lb1, rj, g, q);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j)
            o[j][sg] = twist_digits<kBigQ>(mont_mul_lazy(y[j], pa[j], q, qneg), pb[j][sg], q, nq, cq);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          int m, t;
          lane_out<kR1>(ag, j, m, t);
          const int row = ai + 16 * t;
          *(uint4*)(buf + sw_in<C::in_a, C::in_b>(row * S + 4 * (Q0 + m))) =
              make_uint4(o[j][0], o[j][1], o[j][2], o[j][3]);
        }
      }
    };
    if (q > 0x7F7F7F7Fu) pass1(std::true_type{});
    else pass1(std::false_type{});
    lds_barrier();

    // ---- pass 2: rows.  Step rows R0 .. R0 + 4 Mt2 - 1; set sg and tile
    // vector m take row R0 + 4m + sg; lane (i, g), dword c reads element
    // kR2 u + i % kR2 (u = 4g + c, or g + 4c for the inverse).
    uint4 res[St2][4];
    auto pass2 = [&](auto big_q) {
      constexpr bool kBigQ = decltype(big_q)::value;
      v4i opA2[4];
      uint2 tw2[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        opA2[j] = *(const v4i*)(lds + kTabOpA2 + (j * 64 + lane) * 4);
        tw2[j] = *(const uint2*)(lds + kTabTw2 + (lane * 4 + j) * 2);
      }
      uint2 rj[4], pf[4];  // level-B multipliers; factor of output t (lb2[8 + t])
      if (kR2 < 16) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          int m, t;
          lane_out<kR2>(g, j, m, t);
          pf[j] = lb2[8 + t];
          rj[j] = (g & 1) ? lb2[j] : lb2[0];
        }
      }
#pragma unroll
      for (int st = 0; st < St2; ++st) {
        const int R0 = (wave + st * W) * 4 * Mt2;
#pragma unroll
        for (int sg = 0; sg < 4; ++sg) {
          const int ai = opaque(i16), ag = opaque(g);  // for addresses
          v4i x;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int u = kUA ? ag + 4 * c : 4 * ag + c;
            const int row = R0 + 4 * (ai / kR2) + sg, e = kR2 * u + ai % kR2;
            x[c] = (int)buf[sw_in<C::in_a, C::in_b>(row * S + e)];
          }
          const v4i a0 = mfma(x, opA2[0], bias);
          const v4i a1 = mfma(x, opA2[1], zero);
          const v4i a2 = mfma(x, opA2[2], bias);
          const v4i a3 = mfma(x, opA2[3], zero);
          uint32_t y[4];
          if (kR2 == 16) {
            v4i z;
#pragma unroll
            for (int j = 0; j < 4; ++j)
              z[j] = (int)twist_digits<kBigQ>(fuse_redc(a0[j], a1[j], a2[j], a3[j], q, qneg), tw2[j], q, nq, cq);
            const v4i b0 = mfma(opA2[0], z, bias);  // level B: the same symmetric matrix
            const v4i b1 = mfma(opA2[1], z, zero);
            const v4i b2 = mfma(opA2[2], z, bias);
            const v4i b3 = mfma(opA2[3], z, zero);
#pragma unroll
            for (int j = 0; j < 4; ++j) y[j] = reduce_once(fuse_redc(b0[j], b1[j], b2[j], b3[j], q, qneg), q);
          } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
              y[j] = reduce_once(mul_shoup_lazy(fuse_redc(a0[j], a1[j], a2[j], a3[j], q, qneg), tw2[j].x,
                                                tw2[j].y, q), q);
            level_b<kR2>(y, lb2, rj, g, q);
#pragma unroll
            for (int j = 0; j < 4; ++j) y[j] = mul_shoup(y[j], pf[j].x, pf[j].y, q);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (sg == 0) res[st][j].x = y[j];
            else if (sg == 1) res[st][j].y = y[j];
            else if (sg == 2) res[st][j].z = y[j];
            else res[st][j].w = y[j];
          }
        }
      }
    };
    // (only the 256-point second stage re-slices with the digit window)
    if (kR2 == 16 && q > 0x7F7F7F7Fu) pass2(std::true_type{});
    else pass2(std::false_type{});
    lds_barrier();  // every wave has read its rows
#pragma unroll
    for (int st = 0; st < St2; ++st) {
      const int R0 = (wave + st * W) * 4 * Mt2;
      const int ai = opaque(i16), ag = opaque(g);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int m, t;
        lane_out<kR2>(ag, j, m, t);
        const uint32_t pos = R0 + 4 * m + P1 * (ai + 16 * t);
        *(uint4*)(buf + sw_out<C::out_a, C::out_b, C::out_sh>(pos)) = res[st][j];
      }
    }
    lds_barrier();

    // ---- store: natural order, whole 1 KiB chunks per instruction.  With
    // two buffers the wave reads all its chunks, and once every wave has
    // (barrier) the buffer takes the polynomial after next while the stores
    // drain; with one buffer the chunks are stored as they are read and the
    // next polynomial is loaded after the barrier.
    const int al = opaque(lane);
    uint32_t* const dst = tab.u[it.unit].out + it.poly_base;
    if (NB == 2) {
      uint4 outq[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const uint32_t c = wave + k * W;
        outq[k] = *(const uint4*)(buf + sw_out<C::out_a, C::out_b, C::out_sh>(c * 256 + 4 * al));
      }
      lds_barrier();  // every wave has read the buffer: it may be refilled
      if (p + NB < p_end) issue_load(p + NB, b);
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const uint32_t c = wave + k * W;
        __builtin_nontemporal_store(*(const v4u*)&outq[k], (v4u*)(dst + c * 256 + 4 * al));
      }
    } else {
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const uint32_t c = wave + k * W;
        const uint4 v = *(const uint4*)(buf + sw_out<C::out_a, C::out_b, C::out_sh>(c * 256 + 4 * al));
        __builtin_nontemporal_store(*(const v4u*)&v, (v4u*)(dst + c * 256 + 4 * al));
      }
      lds_barrier();
      if (p + 1 < p_end) issue_load(p + 1, 0);
    }
  }
}

template <int kLogN, bool kInv>
void op_launch(const tfhe_ntt_plan_s* p, const FsTable& t, hipStream_t s) {
  using C = OpCfg<kLogN, kInv>;
  static std::atomic<int> occ{0};
  const uint32_t w =
      p->fs_wg_per_cu ? p->fs_wg_per_cu : (uint32_t)occupancy_cached(occ, op_kernel<kLogN, kInv>, 64 * C::waves);
  const uint32_t grid = std::min(std::max(1u, p->num_cus * w), t.total);
  TFHE_TIMED(K_OP, s, hipLaunchKernelGGL((op_kernel<kLogN, kInv>), dim3(grid), dim3(64 * C::waves), 0, s, t));
}

}  // namespace

bool op_supported(uint32_t log_n) { return log_n >= 12 && log_n <= 15; }

// One launch over every unit of the table (same N and direction).
hipError_t op_run(const tfhe_ntt_plan_s* p, bool inverse, const FsTable& t, hipStream_t s) {
  if (t.total == 0) return hipSuccess;
  switch (p->log_n * 2 + (inverse ? 1 : 0)) {
    case 24: op_launch<12, false>(p, t, s); break;
    case 25: op_launch<12, true>(p, t, s); break;
    case 26: op_launch<13, false>(p, t, s); break;
    case 27: op_launch<13, true>(p, t, s); break;
    case 28: op_launch<14, false>(p, t, s); break;
    case 29: op_launch<14, true>(p, t, s); break;
    case 30: op_launch<15, false>(p, t, s); break;
    case 31: op_launch<15, true>(p, t, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tfhe
