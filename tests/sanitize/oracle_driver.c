/* The C oracle under ASan / UBSan: prime and root construction, the O(N^2)
 * and radix-2 transforms against each other and their round trips, the
 * batched transform, and the schoolbook product.  Exit status 0 when every
 * check holds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int or_is_prime(uint64_t q);
int or_primitive_root(uint64_t q, uint64_t* g_out);
int or_psi(uint64_t q, uint32_t n, uint64_t* psi_out);
void or_ntt_direct(uint32_t n, uint64_t q, uint64_t psi, const uint32_t* in, uint32_t* out, int inverse);
void or_ntt_radix2(uint32_t n, uint64_t q, uint64_t psi, const uint32_t* in, uint32_t* out, int inverse);
int or_ntt_batch(uint32_t n, uint32_t nlimbs, uint32_t batch, const uint64_t* q, const uint64_t* psi,
                 const uint32_t* in, uint32_t* out, int inverse, int threads);
void or_negacyclic_schoolbook(uint32_t n, uint64_t q, const uint32_t* a, const uint32_t* b, uint32_t* c);

static int failures = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #c); ++failures; } } while (0)

static uint64_t rnd(uint64_t* s) {
  *s ^= *s << 13; *s ^= *s >> 7; *s ^= *s << 17;
  return *s;
}

int main(void) {
  const uint64_t q = 2147352577ull; /* 2^31 - 2^17 + 1 */
  uint64_t s = 88172645463325252ull, g = 0, psi = 0;
  CHECK(or_is_prime(q) && !or_is_prime(q + 2) && or_is_prime(17) && !or_is_prime(1));
  CHECK(or_primitive_root(q, &g) == 0 && g > 1);
  for (uint32_t n = 2; n <= 1024; n *= 2) {
    CHECK(or_psi(q, n, &psi) == 0);
    uint32_t* a = malloc(4 * n); uint32_t* x = malloc(4 * n); uint32_t* y = malloc(4 * n); uint32_t* z = malloc(4 * n);
    for (uint32_t i = 0; i < n; ++i) a[i] = (uint32_t)(rnd(&s) % q);
    or_ntt_direct(n, q, psi, a, x, 0);
    or_ntt_radix2(n, q, psi, a, y, 0);
    CHECK(memcmp(x, y, 4 * n) == 0);
    or_ntt_direct(n, q, psi, x, z, 1);
    CHECK(memcmp(z, a, 4 * n) == 0);
    or_ntt_radix2(n, q, psi, y, z, 1);
    CHECK(memcmp(z, a, 4 * n) == 0);
    if (n <= 256) {
      uint32_t* b = malloc(4 * n); uint32_t* c = malloc(4 * n);
      for (uint32_t i = 0; i < n; ++i) b[i] = (uint32_t)(rnd(&s) % q);
      or_negacyclic_schoolbook(n, q, a, b, c);
      /* X^0 * b = b */
      memset(x, 0, 4 * n); x[0] = 1;
      or_negacyclic_schoolbook(n, q, x, b, z);
      CHECK(memcmp(z, b, 4 * n) == 0);
      free(b); free(c);
    }
    free(a); free(x); free(y); free(z);
  }
  for (uint32_t log_n = 12; log_n <= 16; log_n += 4) {
    const uint32_t n = 1u << log_n, limbs = 2, batch = 2;
    uint64_t qs[2] = {q, 2146959361ull}, ps[2];
    CHECK(or_psi(qs[0], n, &ps[0]) == 0 && or_psi(qs[1], n, &ps[1]) == 0);
    size_t total = (size_t)limbs * batch * n;
    uint32_t* a = malloc(4 * total); uint32_t* x = malloc(4 * total); uint32_t* z = malloc(4 * total);
    for (size_t i = 0; i < total; ++i) a[i] = (uint32_t)(rnd(&s) % qs[i / ((size_t)batch * n)]);
    CHECK(or_ntt_batch(n, limbs, batch, qs, ps, a, x, 0, 2) >= 1);
    CHECK(or_ntt_batch(n, limbs, batch, qs, ps, x, z, 1, 2) >= 1);
    CHECK(memcmp(z, a, 4 * total) == 0);
    free(a); free(x); free(z);
  }
  printf("oracle driver: %d failures\n", failures);
  return failures != 0;
}
