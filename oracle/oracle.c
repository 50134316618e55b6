/*
 * Plain CPU oracle for the negacyclic NTT / INTT and negacyclic polynomial
 * product of TensorFHE (arXiv 2212.14191).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the GPU
 * path.
 *
 * Every reduction is a plain `%` on unsigned __int128: slow and obviously
 * correct.  Moduli are primes below 2^32.
 *
 *   or_ntt_direct    Eq. (4): A_k = sum_n a_n psi^{(2k+1) n} mod q, natural
 *                    order, evaluated as the O(N^2) double sum.
 *   or_ntt_radix2    the same transform computed as the textbook route of
 *                    Sec. II-A: pre-twist by psi^n (Eq. (3)), cyclic radix-2
 *                    Cooley-Tukey NTT with omega = psi^2 (Fig. 2), and the
 *                    mirror image for the inverse (Eq. (2)): cyclic INTT with
 *                    omega^{-1}, then N^{-1} and the psi^{-n} post-twist.
 *   or_negacyclic_schoolbook   the product in Z_q[X]/(X^N+1) (Sec. II-A),
 *                    c_m = sum_{i+j=m} a_i b_j - sum_{i+j=m+N} a_i b_j.
 *   or_primitive_root / or_psi  the root construction of Sec. II-A:
 *                    g = smallest primitive root of q, psi = g^{(q-1)/2N}.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) {
  return (uint64_t)(((u128)a * (u128)b) % (u128)q);
}

static uint64_t powmod(uint64_t b, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  b %= q;
  while (e) {
    if (e & 1) r = mulmod(r, b, q);
    b = mulmod(b, b, q);
    e >>= 1;
  }
  return r;
}

/* Inverse by Fermat's little theorem (Sec. II-A): x^{-1} = x^{q-2}. */
static uint64_t invmod(uint64_t x, uint64_t q) { return powmod(x, q - 2, q); }

/* Trial division: plain and obviously correct for q < 2^32. */
int or_is_prime(uint64_t q) {
  if (q < 2) return 0;
  if (q < 4) return 1;
  if (q % 2 == 0) return 0;
  for (uint64_t d = 3; d * d <= q; d += 2)
    if (q % d == 0) return 0;
  return 1;
}

/* Smallest primitive root g of the prime q: g^{(q-1)/f} != 1 for every prime
 * factor f of q-1.  Returns 0 on success, -1 if q is not a prime < 2^32. */
int or_primitive_root(uint64_t q, uint64_t* g_out) {
  if (q >= (1ull << 32) || !or_is_prime(q)) return -1;
  if (q == 2) { *g_out = 1; return 0; }
  uint64_t fac[64];
  int nf = 0;
  uint64_t m = q - 1;
  for (uint64_t d = 2; d * d <= m; ++d) {
    if (m % d == 0) {
      fac[nf++] = d;
      while (m % d == 0) m /= d;
    }
  }
  if (m > 1) fac[nf++] = m;
  for (uint64_t g = 2; g < q; ++g) {
    int ok = 1;
    for (int i = 0; i < nf && ok; ++i)
      if (powmod(g, (q - 1) / fac[i], q) == 1) ok = 0;
    if (ok) { *g_out = g; return 0; }
  }
  return -1;
}

/* psi = g^{(q-1)/(2N)}, a primitive 2N-th root of unity mod q.  Returns 0 on
 * success, -1 if q is not prime or 2N does not divide q-1. */
int or_psi(uint64_t q, uint32_t n, uint64_t* psi_out) {
  uint64_t g;
  if (n == 0 || (n & (n - 1))) return -1;
  if (or_primitive_root(q, &g) != 0) return -1;
  if ((q - 1) % (2ull * n) != 0) return -1;
  *psi_out = powmod(g, (q - 1) / (2ull * n), q);
  return 0;
}

/* Eq. (4) as written (forward), and its inverse
 *   a_n = N^{-1} sum_k A_k psi^{-(2k+1) n}
 * as an O(N^2) double sum over a table of psi^e, e in [0, 2N). */
void or_ntt_direct(uint32_t n, uint64_t q, uint64_t psi, const uint32_t* in,
                   uint32_t* out, int inverse) {
  uint64_t two_n = 2ull * n;
  uint64_t root = inverse ? invmod(psi, q) : psi;
  uint64_t* pw = (uint64_t*)malloc(sizeof(uint64_t) * two_n);
  pw[0] = 1;
  for (uint64_t e = 1; e < two_n; ++e) pw[e] = mulmod(pw[e - 1], root, q);
  uint64_t ninv = invmod(n % q, q);
  for (uint64_t k = 0; k < n; ++k) {
    u128 acc = 0;
    for (uint64_t j = 0; j < n; ++j) {
      /* forward: output k, input j, exponent (2k+1) j;
       * inverse: output k (= coefficient index), input j (= evaluation
       * index), exponent -(2j+1) k. */
      uint64_t e = inverse ? ((2 * j + 1) * k) % two_n : ((2 * k + 1) * j) % two_n;
      acc += (u128)in[j] * pw[e];
    }
    uint64_t v = (uint64_t)(acc % q);
    if (inverse) v = mulmod(v, ninv, q);
    out[k] = (uint32_t)v;
  }
  free(pw);
}

static uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

/* In-place cyclic radix-2 Cooley-Tukey NTT of length n with root w, where
 * pw[e] = w^e for e in [0, n).  Bit-reversed load, natural-order result. */
static void cyclic_ntt(uint32_t n, uint64_t q, const uint64_t* pw, uint64_t* x) {
  int bits = 0;
  while ((1u << bits) < n) ++bits;
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t j = bitrev(i, bits);
    if (j > i) { uint64_t t = x[i]; x[i] = x[j]; x[j] = t; }
  }
  for (uint32_t len = 2; len <= n; len <<= 1) {
    uint32_t half = len / 2, step = n / len;
    for (uint32_t i = 0; i < n; i += len) {
      for (uint32_t j = 0; j < half; ++j) {
        uint64_t u = x[i + j];
        uint64_t v = mulmod(x[i + j + half], pw[(uint64_t)j * step], q);
        x[i + j] = (u + v) % q;
        x[i + j + half] = (u + q - v) % q;
      }
    }
  }
}

/* psi powers: tw[e] = psi^e, e in [0, 2N), for forward; psi^{-e} for inverse */
static void psi_table(uint32_t n, uint64_t q, uint64_t psi, int inverse, uint64_t* tw) {
  uint64_t root = inverse ? invmod(psi, q) : psi;
  tw[0] = 1;
  for (uint64_t e = 1; e < 2ull * n; ++e) tw[e] = mulmod(tw[e - 1], root, q);
}

static void ntt_radix2_tab(uint32_t n, uint64_t q, const uint64_t* tw, const uint64_t* pw,
                           uint64_t ninv, const uint32_t* in, uint32_t* out, int inverse,
                           uint64_t* x) {
  if (!inverse) {
    for (uint32_t i = 0; i < n; ++i) x[i] = mulmod(in[i], tw[i], q); /* a_n psi^n */
    cyclic_ntt(n, q, pw, x);                                          /* omega = psi^2 */
    for (uint32_t i = 0; i < n; ++i) out[i] = (uint32_t)x[i];
  } else {
    for (uint32_t i = 0; i < n; ++i) x[i] = in[i];
    cyclic_ntt(n, q, pw, x);                                          /* omega^{-1} */
    for (uint32_t i = 0; i < n; ++i)
      out[i] = (uint32_t)mulmod(mulmod(x[i], ninv, q), tw[i], q);     /* N^{-1} psi^{-n} */
  }
}

static void make_tables(uint32_t n, uint64_t q, uint64_t psi, int inverse, uint64_t* tw,
                        uint64_t* pw, uint64_t* ninv) {
  psi_table(n, q, psi, inverse, tw);
  for (uint32_t e = 0; e < n; ++e) pw[e] = tw[2 * e]; /* (psi^{+-1})^{2e} = omega^{+-e} */
  *ninv = invmod(n % q, q);
}

void or_ntt_radix2(uint32_t n, uint64_t q, uint64_t psi, const uint32_t* in, uint32_t* out,
                   int inverse) {
  uint64_t* tw = (uint64_t*)malloc(sizeof(uint64_t) * 2 * n);
  uint64_t* pw = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t* x = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t ninv;
  make_tables(n, q, psi, inverse, tw, pw, &ninv);
  ntt_radix2_tab(n, q, tw, pw, ninv, in, out, inverse, x);
  free(tw); free(pw); free(x);
}

/* Batched radix-2 NTT/INTT over the (limb, batch, N) layout: limb l uses
 * (q[l], psi[l]).  Parallel over (limb, poly) units with `threads` OpenMP
 * threads (<= 0: runtime default).  Returns the thread count used. */
int or_ntt_batch(uint32_t n, uint32_t nlimbs, uint32_t batch, const uint64_t* q,
                 const uint64_t* psi, const uint32_t* in, uint32_t* out, int inverse,
                 int threads) {
  uint64_t* tw = (uint64_t*)malloc(sizeof(uint64_t) * 2ull * n * nlimbs);
  uint64_t* pw = (uint64_t*)malloc(sizeof(uint64_t) * (uint64_t)n * nlimbs);
  uint64_t* ninv = (uint64_t*)malloc(sizeof(uint64_t) * nlimbs);
  for (uint32_t l = 0; l < nlimbs; ++l)
    make_tables(n, q[l], psi[l], inverse, tw + 2ull * n * l, pw + (uint64_t)n * l, &ninv[l]);
  int used = 1;
#ifdef _OPENMP
  if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel num_threads(threads)
#endif
  {
#ifdef _OPENMP
#pragma omp single
    used = omp_get_num_threads();
#endif
    uint64_t* x = (uint64_t*)malloc(sizeof(uint64_t) * n);
    int64_t units = (int64_t)nlimbs * batch;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
    for (int64_t u = 0; u < units; ++u) {
      uint32_t l = (uint32_t)(u / batch);
      const uint32_t* src = in + (uint64_t)u * n;
      uint32_t* dst = out + (uint64_t)u * n;
      ntt_radix2_tab(n, q[l], tw + 2ull * n * l, pw + (uint64_t)n * l, ninv[l], src, dst,
                     inverse, x);
    }
    free(x);
  }
  free(tw); free(pw); free(ninv);
  return used;
}

/* Schoolbook product in Z_q[X]/(X^N + 1). */
void or_negacyclic_schoolbook(uint32_t n, uint64_t q, const uint32_t* a, const uint32_t* b,
                              uint32_t* c) {
  for (uint32_t m = 0; m < n; ++m) {
    u128 pos = 0, neg = 0;
    for (uint32_t i = 0; i <= m; ++i) pos += (u128)a[i] * b[m - i];
    for (uint32_t i = m + 1; i < n; ++i) neg += (u128)a[i] * b[n + m - i];
    uint64_t p = (uint64_t)(pos % q), ng = (uint64_t)(neg % q);
    c[m] = (uint32_t)((p + q - ng) % q);
  }
}

/* Batched schoolbook over (limb, batch, N); returns the thread count used. */
int or_negacyclic_batch(uint32_t n, uint32_t nlimbs, uint32_t batch, const uint64_t* q,
                        const uint32_t* a, const uint32_t* b, uint32_t* c, int threads) {
  int used = 1;
  int64_t units = (int64_t)nlimbs * batch;
#ifdef _OPENMP
  if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel num_threads(threads)
#endif
  {
#ifdef _OPENMP
#pragma omp single
    used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 1)
#endif
    for (int64_t u = 0; u < units; ++u) {
      uint32_t l = (uint32_t)(u / batch);
      or_negacyclic_schoolbook(n, q[l], a + (uint64_t)u * n, b + (uint64_t)u * n,
                               c + (uint64_t)u * n);
    }
  }
  return used;
}
