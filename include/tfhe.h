/*
 * tfhe.h - C ABI of the MI355X (gfx950) NTT / HMULT library, an
 * implementation of the hot path of TensorFHE (arXiv 2212.14191).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Moduli are primes q with 2^29 < q < 2^31 and q = 1 (mod 2N).
 * - Residue arrays are uint32, canonical (each value in [0, q)), standard
 *   (non-Montgomery) form, in the (limb, batch, N) layout the paper uses for
 *   operation-level batching (Sec. IV-D): limb-major, then polynomial, then
 *   coefficient.  Element (l, b, i) of an array with `batch` polynomials is
 *   at index (l * batch + b) * N + i.
 * - NTT-domain order is natural: index k holds the evaluation at psi^{2k+1}
 *   (Eq. 4).  Both transform algorithms produce the same bits.
 * - Device pointers are plain HIP device addresses (for example a torch
 *   tensor's data_ptr()).  The caller owns every buffer it passes; the
 *   library owns only what its *_create functions allocate.
 * - Compute calls are asynchronous on `stream` (NULL = the default stream)
 *   and validate their arguments synchronously.  A kernel fault surfaces as
 *   TFHE_EHIP from a later call or from the caller's own synchronisation.
 * - Host arrays passed to *_create are copied; the caller may free them.
 * - Out-of-range inputs (values >= q) give unspecified results.
 * - Every function returns a tfhe_status; on failure tfhe_last_error()
 *   describes the cause (thread-local, valid until the next call on the
 *   same thread).
 */
#ifndef TFHE_H_
#define TFHE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TFHE_OK = 0,
  TFHE_EINVAL = -1,      /* bad argument: null/unaligned pointer, size, level */
  TFHE_ENOTNTT = -2,     /* modulus not prime, q != 1 mod 2N, q out of range,
                            or psi not a primitive 2N-th root of unity */
  TFHE_ENOMEM = -3,      /* device or host allocation failed */
  TFHE_EHIP = -4,        /* a HIP runtime call failed */
  TFHE_EUNSUPPORTED = -5 /* valid request the library does not implement */
} tfhe_status;

typedef enum {
  TFHE_NTT_AUTO = 0,          /* the library's choice (tuned table, else MFMA
                                 when available for N, else butterfly) */
  TFHE_NTT_BUTTERFLY = 1,     /* radix-2 Cooley-Tukey / Gentleman-Sande
                                 butterflies on the vector ALUs, two stages
                                 per LDS round trip (Sec. II-A, Fig. 2) */
  TFHE_NTT_FOURSTEP_MFMA = 2, /* four-step NTT whose DFT stages are exact
                                 INT8 matrix-core contractions over byte
                                 slices (Sec. IV-C, Eq. 9, Eq. 10) */
  TFHE_NTT_FOURSTEP_VALU = 3  /* the same four-step passes with each 16 x 16
                                 matrix product on the vector ALUs, 96-bit
                                 accumulation and one reduction per output
                                 (Sec. IV-B, Eq. 7 to Eq. 9); N = 2^16 only,
                                 tfhe_ntt_fwd / tfhe_ntt_inv only; never
                                 chosen by AUTO */
} tfhe_ntt_algo;

typedef struct tfhe_ntt_plan_s* tfhe_ntt_plan;
typedef struct tfhe_ckks_ctx_s* tfhe_ckks_ctx;
typedef struct ihipStream_t* tfhe_stream_t; /* binary-compatible with hipStream_t */

/* ------------------------------------------------------------- utilities */

/* Human-readable name of a status code (static string). */
const char* tfhe_status_string(tfhe_status s);

/* Detail of the last failure on the calling thread ("" if none). */
const char* tfhe_last_error(void);

/* The `count` largest primes q < 2^bits with q = 1 (mod two_n), written in
 * descending order to the host array out[count].  This is the modulus
 * selection rule the library applies when a caller gives none (the paper
 * leaves the choice open, Table 1).  bits in [30, 31]. */
tfhe_status tfhe_find_primes(uint32_t bits, uint64_t two_n, uint32_t count, uint32_t* out);

/* psi = g^{(q-1)/2N} for the smallest primitive root g of q (Sec. II-A);
 * the root used when a plan is created with psi == NULL. */
tfhe_status tfhe_default_psi(uint32_t q, uint32_t log_n, uint32_t* psi);

/* -------------------------------------------------------------- NTT plan */

/* Create an immutable plan for N = 2^log_n over n_limbs primes.
 *   q[n_limbs], psi[n_limbs]: host arrays; psi may be NULL (default root).
 *   algo: transform used by tfhe_ntt_fwd/inv; AUTO resolves to the
 *     four-step MFMA transform where the plan supports it (log_n in [12, 16])
 *     and to the butterfly elsewhere; tfhe_ntt_plan_info reports the choice.
 * Builds the twiddle tables of both algorithms on the device (Sec. IV-B:
 * "pre-computed in the initialization and reused").  Synchronous.
 * log_n in [4, 16].  The four-step split is fixed at N = N1 x 256 (N1 =
 * 2^(log_n - 8), the 256-point stage a 16 x 16 matrix-core contraction,
 * the N1-point stage 16 x N1/16); there is no split parameter.
 * Errors: TFHE_ENOTNTT for a bad modulus/root, TFHE_EINVAL, TFHE_ENOMEM. */
tfhe_status tfhe_ntt_plan_create(tfhe_ntt_plan* out, uint32_t log_n, uint32_t n_limbs,
                                 const uint32_t* q, const uint32_t* psi, tfhe_ntt_algo algo);
tfhe_status tfhe_ntt_plan_destroy(tfhe_ntt_plan plan);

/* Plan properties: modulus and root of limb `limb`, N, limb count, the
 * algorithm AUTO resolved to. */
tfhe_status tfhe_ntt_plan_info(tfhe_ntt_plan plan, uint32_t* log_n, uint32_t* n_limbs,
                               tfhe_ntt_algo* algo);
tfhe_status tfhe_ntt_plan_modulus(tfhe_ntt_plan plan, uint32_t limb, uint32_t* q, uint32_t* psi);

/* Tuning knobs of a plan (written by an autotuner; the defaults are sound):
 *   TFHE_PARAM_FS_WG_PER_CU  persistent four-step workgroups per compute
 *                            unit (0 = as many as fit, the default)
 *   TFHE_PARAM_AUTO_ALGO     what TFHE_NTT_AUTO resolves to (a tfhe_ntt_algo;
 *                            MFMA only where the plan supports it)
 *   TFHE_PARAM_FS_WIDE       work items of the four-step 256-point stage:
 *                            0 = library default (wide for N >= 2^15),
 *                            1 = always 16 vectors (4 waves), 2 = 32 vectors
 *                            (8 waves) whenever N >= 2^13.  The key switch's
 *                            fused second pass takes wide items whenever
 *                            N >= 2^13 unless this is 1.
 *   TFHE_PARAM_FS_PASSES     HBM round trips of a four-step transform
 *                            (the paper's Stages 1-5 as one pipeline,
 *                            Sec. IV-C): 1 = one (the polynomial stays in
 *                            LDS; N = 2^12..2^15, not for the key switch's
 *                            fused passes or the ModDown / RESCALE
 *                            epilogue, which keep two), 2 = two (a
 *                            transposed intermediate in the workspace
 *                            between two passes), 0 = library default: one
 *                            at N = 2^12..2^14 for launches of at least two
 *                            polynomials per compute unit, else two.  Same
 *                            results.
 *   TFHE_PARAM_KS_INNER      key switching with a four-step plan (the plan
 *                            of a CKKS context): 0 = library default (1),
 *                            1 = the ModUp transforms' second pass fused
 *                            with the key inner product (Sec. IV-A: NTT,
 *                            then Inner-product, in one kernel), 2 = a
 *                            separate inner-product kernel.  Same results;
 *                            tfhe_hmult_workspace_size depends on it.
 *   TFHE_PARAM_FS_RING       LDS ring depth (work items in flight per
 *                            workgroup) of the two-pass four-step kernels
 *                            with 8-wave items (the 256-point stage, see
 *                            TFHE_PARAM_FS_WIDE): 0 = library default (2),
 *                            2 or 3; the 4-wave items always use 3.  Same
 *                            results.
 * Not thread-safe against concurrent compute calls on the same plan. */
typedef enum {
  TFHE_PARAM_FS_WG_PER_CU = 1,
  TFHE_PARAM_AUTO_ALGO = 2,
  TFHE_PARAM_FS_WIDE = 3,
  TFHE_PARAM_FS_PASSES = 4,
  TFHE_PARAM_KS_INNER = 5,
  TFHE_PARAM_FS_RING = 6
} tfhe_plan_param;
tfhe_status tfhe_ntt_plan_set_param(tfhe_ntt_plan plan, tfhe_plan_param param, int64_t value);
tfhe_status tfhe_ntt_plan_get_param(tfhe_ntt_plan plan, tfhe_plan_param param, int64_t* value);

/* Bytes of device workspace tfhe_ntt_fwd/inv need for `batch` polynomials
 * of `limb_count` limbs (the transposed intermediate between the two
 * passes).  0 is possible; the value never exceeds limb_count*batch*N*4. */
tfhe_status tfhe_ntt_workspace_size(tfhe_ntt_plan plan, tfhe_ntt_algo algo, uint32_t limb_count,
                                    uint32_t batch, size_t* bytes);

/* Forward negacyclic NTT, Eq. (4): out_k = sum_n in_n psi^{(2k+1)n} mod q,
 * for limbs [limb_begin, limb_begin+limb_count) of the plan and `batch`
 * polynomials per limb.  in/out: device [limb_count][batch][N] uint32,
 * 16-byte aligned; in == out allowed (no other overlap).  ws: device
 * workspace of at least tfhe_ntt_workspace_size bytes, 256-byte aligned.
 * algo: AUTO uses the plan's algorithm. */
tfhe_status tfhe_ntt_fwd(tfhe_ntt_plan plan, tfhe_ntt_algo algo, const uint32_t* in, uint32_t* out,
                         uint32_t limb_begin, uint32_t limb_count, uint32_t batch, void* ws,
                         size_t ws_bytes, tfhe_stream_t stream);

/* Inverse, Eq. (2) with the negacyclic twist of Eq. (3):
 * out_n = N^{-1} psi^{-n} sum_k in_k psi^{-2nk} mod q.  Same arguments. */
tfhe_status tfhe_ntt_inv(tfhe_ntt_plan plan, tfhe_ntt_algo algo, const uint32_t* in, uint32_t* out,
                         uint32_t limb_begin, uint32_t limb_count, uint32_t batch, void* ws,
                         size_t ws_bytes, tfhe_stream_t stream);

/* Operation-level batching (Sec. IV-D): one fused launch per kernel pass
 * covers every descriptor, whatever its N, modulus set, limb range, batch
 * and direction.  Descriptors are host structs; they are copied into the
 * launch, so the array may be reused after the call returns. */
typedef struct {
  tfhe_ntt_plan plan;
  const uint32_t* in;   /* device [limb_count][batch][N] of the plan's N */
  uint32_t* out;        /* device, same shape; == in allowed */
  uint32_t limb_begin;  /* first plan limb */
  uint32_t limb_count;
  uint32_t batch;
  int32_t inverse;      /* 0 forward (Eq. 4), 1 inverse */
} tfhe_ntt_desc;

/* Workspace bytes tfhe_ntt_batch needs for these descriptors and algorithm
 * (AUTO: the four-step MFMA transform where every plan supports it, else
 * the butterfly). */
tfhe_status tfhe_ntt_batch_workspace_size(const tfhe_ntt_desc* descs, uint32_t count,
                                          tfhe_ntt_algo algo, size_t* bytes);

/* Run every descriptor's transform.  Descriptors must not overlap each other
 * except in == out within one descriptor.  ws: >= the size above, 256-byte
 * aligned.  Errors as for tfhe_ntt_fwd; TFHE_EUNSUPPORTED if algo is MFMA
 * and some plan lacks it. */
tfhe_status tfhe_ntt_batch(const tfhe_ntt_desc* descs, uint32_t count, tfhe_ntt_algo algo,
                           void* ws, size_t ws_bytes, tfhe_stream_t stream);

/* Element-wise kernels of Sec. IV-A over the same layout (a, b, c device,
 * [limb_count][batch][N]; c may alias a or b):
 *   Hada-Mult c = a o b mod q;  Ele-Add c = a + b mod q;  Ele-Sub c = a - b mod q. */
tfhe_status tfhe_pointwise_mul(tfhe_ntt_plan plan, const uint32_t* a, const uint32_t* b,
                               uint32_t* c, uint32_t limb_begin, uint32_t limb_count,
                               uint32_t batch, tfhe_stream_t stream);
tfhe_status tfhe_pointwise_add(tfhe_ntt_plan plan, const uint32_t* a, const uint32_t* b,
                               uint32_t* c, uint32_t limb_begin, uint32_t limb_count,
                               uint32_t batch, tfhe_stream_t stream);
tfhe_status tfhe_pointwise_sub(tfhe_ntt_plan plan, const uint32_t* a, const uint32_t* b,
                               uint32_t* c, uint32_t limb_begin, uint32_t limb_count,
                               uint32_t batch, tfhe_stream_t stream);
/* c = a o b for a b broadcast over the batch: b is [limb_count][N]. */
tfhe_status tfhe_pointwise_mul_bcast(tfhe_ntt_plan plan, const uint32_t* a, const uint32_t* b,
                                     uint32_t* c, uint32_t limb_begin, uint32_t limb_count,
                                     uint32_t batch, tfhe_stream_t stream);

/* Residues of small signed integers: out[l][b][i] = in[b][i] mod q_{limb_begin+l}
 * for every plan limb in the range (how secrets, errors and scaled messages
 * enter the RNS representation, Sec. II-B).  in: device int32 [batch][N];
 * out: device [limb_count][batch][N]. */
tfhe_status tfhe_load_small(tfhe_ntt_plan plan, const int32_t* in, uint32_t* out,
                            uint32_t limb_begin, uint32_t limb_count, uint32_t batch,
                            tfhe_stream_t stream);

/* ------------------------------------------------------------ CKKS context */

/* RNS-CKKS context (Sec. II-B) with hybrid key switching: L q-limbs, K
 * special p-limbs, dnum digits of alpha = L/dnum limbs (P must exceed every
 * digit's modulus).  moduli[L+K]: q_0..q_{L-1} then p_0..p_{K-1} (host;
 * NULL = tfhe_find_primes(31, 2^17, L+K) with the K largest as the p-limbs
 * and the rest, descending, as q_0..q_{L-1}).  psi[L+K] may be NULL.
 * Builds an NTT plan over all L+K moduli plus the basis-conversion
 * constants of ModUp/ModDown for every level.  Synchronous. */
tfhe_status tfhe_ckks_ctx_create(tfhe_ckks_ctx* out, uint32_t log_n, uint32_t L, uint32_t K,
                                 uint32_t dnum, const uint32_t* moduli, const uint32_t* psi,
                                 tfhe_ntt_algo algo);
tfhe_status tfhe_ckks_ctx_destroy(tfhe_ckks_ctx ctx);

/* The context's NTT plan (over the L+K moduli, q-limbs first); owned by the
 * context, valid until tfhe_ckks_ctx_destroy. */
tfhe_status tfhe_ckks_ctx_plan(tfhe_ckks_ctx ctx, tfhe_ntt_plan* plan);

/* Device workspace (bytes) tfhe_hmult / tfhe_rotate need at this level and
 * batch. */
tfhe_status tfhe_hmult_workspace_size(tfhe_ckks_ctx ctx, uint32_t level, uint32_t batch,
                                      size_t* bytes);

/* HMULT (Sec. II-B; kernels of Table 2): for each of `batch` ciphertext
 * pairs, ct_out = (d0, d1) + KeySwitch(d2) with d0 = c0c0', d1 = c0c1' +
 * c1c0', d2 = c1c1'.  KeySwitch = INTT, Dcomp into digits, ModUp by fast
 * basis conversion (no overflow correction), NTT, inner product with evk,
 * ModDown (no rounding offset) (Sec. IV-A).  No rescale.
 *   ct_a, ct_b, ct_out: device [2][level][batch][N], NTT domain; ct_out may
 *     alias ct_a or ct_b.
 *   evk: device [dnum][2][L+K][N], NTT domain, evk[j] = (b_j, a_j) with
 *     b_j = -a_j s + e_j + g_j s^2, g_j = [P]_{q_i} on the limbs of digit j.
 *   level in [1, L]; ws: >= tfhe_hmult_workspace_size bytes, 256-aligned. */
tfhe_status tfhe_hmult(tfhe_ckks_ctx ctx, const uint32_t* ct_a, const uint32_t* ct_b,
                       uint32_t* ct_out, const uint32_t* evk, uint32_t level, uint32_t batch,
                       void* ws, size_t ws_bytes, tfhe_stream_t stream);

/* tfhe_hmult without a caller workspace and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops that forbid allocation on their hot path).  It runs the
 * same kernels as tfhe_hmult (same results, bit for bit) with the
 * workspace placed in a fixed device array of TFHE_HMULT_NOALLOC_MAX_BYTES
 * that the library holds on every GPU it has created a context on, until
 * the process ends; the array's address is resolved once per device by
 * tfhe_ckks_ctx_create.  The caller still passes inputs and outputs (same
 * layout and rules as tfhe_hmult).
 *   Returns TFHE_EINVAL when tfhe_hmult_workspace_size(level, batch)
 *   exceeds TFHE_HMULT_NOALLOC_MAX_BYTES (at N = 2^16, L = 24, K = 8,
 *   dnum = 3: batch 1 at every level).
 *   Every call on one GPU uses that GPU's one array, whatever the context
 *   or stream: calls that may overlap on one GPU (different streams, or
 *   threads without ordering) race and give undefined results; order them
 *   on one stream.  Nothing in the array needs clearing between calls. */
#define TFHE_HMULT_NOALLOC_MAX_BYTES (128u << 20)
tfhe_status tfhe_hmult_noalloc(tfhe_ckks_ctx ctx, const uint32_t* ct_a, const uint32_t* ct_b,
                               uint32_t* ct_out, const uint32_t* evk, uint32_t level,
                               uint32_t batch, tfhe_stream_t stream);

/* HMULT of ciphertext pairs of different levels in one batched launch
 * sequence (operation-level batching across levels, Sec. IV-D): pair i is
 * multiplied at levels[i] exactly as tfhe_hmult would do for it alone (same
 * result, bit for bit).  The pairs are grouped by level; one launch forms
 * every pair's tensor product, and every NTT/INTT, basis conversion and key
 * inner product of all groups shares one launch per key-switching step (the
 * transforms run over a descriptor table of the groups' limbs).
 *   ct_a, ct_b, ct_out: host arrays [count] of device pointers, each a
 *     single ciphertext [2][levels[i]][N], NTT domain, 16-byte aligned.  An
 *     output may alias any input (results are written after every input has
 *     been read); outputs must not overlap one another.
 *   levels: host [count], each in [1, L]; count <= TFHE_HMULT_LEVELS_MAX.
 *   evk: as for tfhe_hmult; ws: >= tfhe_hmult_levels_workspace_size bytes
 *     for the same levels, 256-aligned.
 * The host arrays are read during the call only. */
#define TFHE_HMULT_LEVELS_MAX 64
tfhe_status tfhe_hmult_levels_workspace_size(tfhe_ckks_ctx ctx, const uint32_t* levels, uint32_t count,
                                             size_t* bytes);
tfhe_status tfhe_hmult_levels(tfhe_ckks_ctx ctx, const uint32_t* const* ct_a, const uint32_t* const* ct_b,
                              uint32_t* const* ct_out, const uint32_t* levels, uint32_t count,
                              const uint32_t* evk, void* ws, size_t ws_bytes, tfhe_stream_t stream);

/* HROTATE of ciphertexts of different levels and rotation amounts in one
 * batched launch sequence (as tfhe_hmult_levels): ciphertext i, ct_in[i]
 * [2][levels[i]][N], is rotated by galois_elts[i] (odd, < 2N) with
 * rotkeys[i] (layout as for tfhe_rotate; entries may repeat) into
 * ct_out[i], exactly as tfhe_rotate would do for it alone.  Pointer rules,
 * count and workspace (tfhe_hmult_levels_workspace_size of the same levels)
 * as for tfhe_hmult_levels. */
tfhe_status tfhe_rotate_levels(tfhe_ckks_ctx ctx, const uint32_t* const* ct_in, uint32_t* const* ct_out,
                               const uint32_t* const* rotkeys, const uint32_t* galois_elts, const uint32_t* levels,
                               uint32_t count, void* ws, size_t ws_bytes, tfhe_stream_t stream);

/* HROTATE (Sec. II-B): ct_out = (sigma(c0), 0) + KeySwitch_rk(sigma(c1)),
 * sigma the automorphism X -> X^galois_elt applied in the NTT domain as the
 * FrobeniusMap permutation of Sec. IV-A: out_j = in_{pi(j)},
 * pi(j) = ((2j+1) galois_elt mod 2N - 1)/2.  galois_elt odd, < 2N (5^r mod
 * 2N rotates the slots by r).  rotkey: device [dnum][2][L+K][N] for
 * s' = sigma(s).  ct_in, ct_out: device [2][level][batch][N], must not alias. */
tfhe_status tfhe_rotate(tfhe_ckks_ctx ctx, const uint32_t* ct_in, uint32_t* ct_out,
                        const uint32_t* rotkey, uint32_t galois_elt, uint32_t level,
                        uint32_t batch, void* ws, size_t ws_bytes, tfhe_stream_t stream);

/* HROTATE of a batch whose ciphertexts rotate by different amounts, in one
 * batched launch sequence (operation-level batching, Sec. IV-D): ciphertext
 * b of ct_in is rotated by galois_elts[b] with the rotation key rotkeys[b],
 * exactly as tfhe_rotate would do for it alone.
 *   rotkeys: host array [batch] of device pointers, each [dnum][2][L+K][N]
 *     (entries may repeat); galois_elts: host array [batch], each odd, < 2N.
 *   ct_in, ct_out: device [2][level][batch][N], must not alias.
 *   batch <= TFHE_ROTATE_MULTI_MAX; ws: >= tfhe_hmult_workspace_size bytes.
 * The host arrays are read during the call only. */
#define TFHE_ROTATE_MULTI_MAX 64
tfhe_status tfhe_rotate_multi(tfhe_ckks_ctx ctx, const uint32_t* ct_in, uint32_t* ct_out,
                              const uint32_t* const* rotkeys, const uint32_t* galois_elts,
                              uint32_t level, uint32_t batch, void* ws, size_t ws_bytes,
                              tfhe_stream_t stream);

/* Device workspace (bytes) tfhe_rescale needs at this level (>= 2) and
 * batch. */
tfhe_status tfhe_rescale_workspace_size(tfhe_ckks_ctx ctx, uint32_t level, uint32_t batch,
                                        size_t* bytes);

/* RESCALE (Sec. II-B; kernels of Table 2: NTT and Ele-Sub): divides every
 * ciphertext by the top modulus q_t = q_{level-1} and drops that limb.  Per
 * component: t = INTT(c_t) in [0, q_t); c'_i = (c_i - NTT(t mod q_i)) *
 * q_t^{-1} mod q_i for i < level-1, i.e. floor(C / q_t) of the CRT value C
 * in [0, Q_level) (no rounding offset).
 *   ct_in: device [2][level][batch][N], NTT domain, level in [2, L].
 *   ct_out: device [2][level-1][batch][N]; must not overlap ct_in.
 *   ws: >= tfhe_rescale_workspace_size bytes, 256-byte aligned. */
tfhe_status tfhe_rescale(tfhe_ckks_ctx ctx, const uint32_t* ct_in, uint32_t* ct_out, uint32_t level,
                         uint32_t batch, void* ws, size_t ws_bytes, tfhe_stream_t stream);

/* CMULT (Sec. II-B; Hada-Mult): ct_out = (c0 o p, c1 o p) for each of
 * `batch` ciphertexts with its own plaintext.
 *   ct, ct_out: device [2][level][batch][N]; pt: device [level][batch][N];
 *   all NTT domain; ct_out may alias ct (element-wise). */
tfhe_status tfhe_cmult(tfhe_ckks_ctx ctx, const uint32_t* ct, const uint32_t* pt, uint32_t* ct_out,
                       uint32_t level, uint32_t batch, tfhe_stream_t stream);

/* HADD (Sec. II-B; Ele-Add): ct_out = ct_a + ct_b component-wise.
 *   device [2][level][batch][N] each; ct_out may alias either input. */
tfhe_status tfhe_hadd(tfhe_ckks_ctx ctx, const uint32_t* ct_a, const uint32_t* ct_b, uint32_t* ct_out,
                      uint32_t level, uint32_t batch, tfhe_stream_t stream);

/* FrobeniusMap alone (Sec. IV-A): out_j = in_{pi(j)} on every polynomial of
 * a [limb_count][batch][N] array (NTT domain).  out must not alias in. */
tfhe_status tfhe_frobenius_map(tfhe_ntt_plan plan, const uint32_t* in, uint32_t* out,
                               uint32_t galois_elt, uint32_t limb_count, uint32_t batch,
                               tfhe_stream_t stream);

/* ---------------------------------------------------------------- serving */

/* Request dispatcher (the API layer of Sec. IV-E with operation-level
 * batching, Sec. IV-D): callers submit single-ciphertext HMULT and HROTATE
 * requests; `slots` worker threads, each with its own stream, group
 * requests of equal N into batches of up to max_batch, whatever their levels
 * and operations, run each batch as one launch sequence (as
 * tfhe_hmult_levels does, with the tensor products of its HMULTs and the
 * Frobenius maps of its rotations each in one launch and every kernel of the
 * key switch, which the two operations share, once for the whole batch; a
 * batch of one with tfhe_hmult / tfhe_rotate on the request's own buffers),
 * and report each request's completion through tfhe_server_poll.
 * The result of a request is exactly what tfhe_hmult / tfhe_rotate computes
 * for it alone.
 *
 * tfhe_server_create: pool is caller-owned device memory, 256-byte aligned,
 * pool_bytes >= 256*slots, split evenly among the slots; it holds each
 * batch's workspace (with its staged results) and must outlive the
 * server.  The server belongs to the device current at creation.
 *   slots in [1, 16]; max_batch in [1, TFHE_ROTATE_MULTI_MAX].
 * Errors: TFHE_EINVAL, TFHE_ENOMEM (host), TFHE_EHIP. */
typedef struct tfhe_server_s* tfhe_server;
tfhe_status tfhe_server_create(tfhe_server* out, uint32_t slots, uint32_t max_batch, void* pool,
                               size_t pool_bytes);

/* Registers the context of ring dimension 2^ctx.log_n (replacing an
 * earlier one of that N for later submissions; requests already queued
 * keep theirs) and its relinearisation key evk (device, layout as for
 * tfhe_hmult, 16-byte aligned).  Registering a different context for an N
 * drops the rotation keys registered for the previous one (re-registering
 * the same context keeps them).  Contexts and keys must outlive the server:
 * queued requests hold raw pointers to them. */
tfhe_status tfhe_server_add_context(tfhe_server s, tfhe_ckks_ctx ctx, const uint32_t* evk);

/* Batch limit for requests of N = 2^log_n (a context must be registered):
 * the best batch size differs per kernel shape (Sec. IV-E, Sec. VI-E),
 * which the autotuner measures; 0 restores the server's max_batch.
 *   max_batch in [0, TFHE_ROTATE_MULTI_MAX]. */
tfhe_status tfhe_server_set_max_batch(tfhe_server s, uint32_t log_n, uint32_t max_batch);

/* Registers the rotation key (device, layout as for tfhe_rotate, 16-byte
 * aligned; it must outlive the server) of Galois element galois_elt (odd,
 * < 2N) for the context of N = 2^log_n. */
tfhe_status tfhe_server_add_rotation_key(tfhe_server s, uint32_t log_n, uint32_t galois_elt,
                                         const uint32_t* rotkey);

/* Queues one request and returns at once.
 *   op 0: HMULT of ct_a and ct_b (galois_elt ignored); op 1: HROTATE of
 *     ct_a by galois_elt (ct_b ignored; ct_out must not alias ct_a).
 *   ct_a, ct_b, ct_out: device [2][level][N], NTT domain, 16-byte aligned;
 *     the inputs must stay unchanged and all three allocated until the
 *     request completes.
 *   The request waits for the work queued on `stream` before this call
 *   (the inputs may still be in production there).
 *   tag: the caller's identifier, returned by tfhe_server_poll.
 * Errors (nothing queued): TFHE_EINVAL (no context for N, level out of
 * [1, L], no rotation key for galois_elt, null or unaligned pointer),
 * TFHE_ENOMEM (one request alone exceeds a slot's share of the pool),
 * TFHE_EHIP. */
tfhe_status tfhe_server_submit(tfhe_server s, uint32_t op, uint32_t log_n, uint32_t level,
                               const uint32_t* ct_a, const uint32_t* ct_b, uint32_t galois_elt,
                               uint32_t* ct_out, uint64_t tag, tfhe_stream_t stream);

/* One request of tfhe_server_submit_many (fields as the arguments of
 * tfhe_server_submit). */
typedef struct {
  uint32_t op, log_n, level, galois_elt;
  const uint32_t* ct_a;
  const uint32_t* ct_b;
  uint32_t* ct_out;
  uint64_t tag;
} tfhe_server_request;

/* Queues reqs[0..count) (host array, read during the call) with the checks
 * of tfhe_server_submit; all of them wait for the work queued on `stream`
 * before this call.  If one fails its checks nothing is queued, the error
 * is returned and *bad (if not NULL) is set to its index. */
tfhe_status tfhe_server_submit_many(tfhe_server s, const tfhe_server_request* reqs, uint32_t count,
                                    tfhe_stream_t stream, uint32_t* bad);

/* Moves up to `max` completed requests into tags[] / status[] (host
 * arrays) and returns how many.  status is TFHE_OK once the result is in
 * ct_out (the device work has finished), else the error of its batch. */
uint32_t tfhe_server_poll(tfhe_server s, uint64_t* tags, int32_t* status, uint32_t max);

/* Waits for the batches in flight, then frees the server; requests not yet
 * dispatched are dropped without completion.  The other tfhe_server_* calls
 * may come from any thread, but none may overlap this one. */
tfhe_status tfhe_server_destroy(tfhe_server s);

/* ------------------------------------------------------------ measurement */

/* Per-kernel timing.  While enabled, the library brackets every kernel of
 * the transform, element-wise and CKKS entry points (also when the request
 * dispatcher runs them; its result scatter is not timed) with a pair of
 * HIP events recorded on that kernel's stream.  tfhe_timing_enable(0 or 1)
 * also discards earlier records. */
tfhe_status tfhe_timing_enable(int enable);

/* Launch count and summed event-measured duration (ms) of the kernel named
 * `kernel` since timing was enabled; waits for the recorded events.  Names:
 * ntt_mfma_pass1, ntt_mfma_pass2, ntt_mfma_onepass, ntt_mfma_pass2_inner, ntt_co_pass1,
 * ntt_co_pass2, ntt_bf_single,
 * ntt_bf_cols, ntt_bf_rows,
 * elementwise, ckks_tensor, ckks_modup, ckks_inner, ckks_moddown_conv,
 * ckks_moddown_final, frobenius, ckks_rescale_bcast, ckks_rescale_final.
 * Unknown name: TFHE_EINVAL. */
tfhe_status tfhe_timing_read(const char* kernel, uint64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* TFHE_H_ */
