/* The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer: the
 * field, matrices, and encode/decode round trips on small blocks over every
 * erasure set of up to p blocks, for several codecs and block sizes. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_gf_exp(int i);
int oracle_gf_log(int a);
uint8_t oracle_gf_mul(uint8_t a, uint8_t b);
uint8_t oracle_gf_inv(uint8_t a);
int oracle_cauchy(int n, int p, uint8_t *gen);
int oracle_vandermonde_rows(int n, int p, uint8_t *gen);
int oracle_invert(int n, const uint8_t *m, uint8_t *inv);
void oracle_bitmatrix(int rows, int cols, const uint8_t *mat, uint8_t *bits);
int oracle_encode(int n, int p, const uint8_t *gen, const uint8_t *const *data, uint8_t *const *parity, size_t S);
int oracle_decode(int n, int p, const uint8_t *gen, const int *erased, int ne, const uint8_t *const *blocks,
                  uint8_t *const *out, size_t S);

static int failures = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c); ++failures; } } while (0)

static unsigned rng = 2021;
static uint8_t next_byte(void) { rng = rng * 1103515245u + 12345u; return (uint8_t)(rng >> 16); }

/* every erasure set of 1..p blocks, as bitmasks over n+p blocks */
static void round_trips(int n, int p, size_t S, int vandermonde) {
  const int nb = n + p;
  uint8_t *gen = malloc((size_t)nb * n);
  CHECK((vandermonde ? oracle_vandermonde_rows(n, p, gen) : oracle_cauchy(n, p, gen)) == 0);
  uint8_t **blk = malloc(sizeof(uint8_t *) * nb);
  uint8_t **rec = malloc(sizeof(uint8_t *) * (p > 0 ? p : 1));
  for (int b = 0; b < nb; ++b) blk[b] = malloc(S);
  for (int j = 0; j < p; ++j) rec[j] = malloc(S);
  for (int i = 0; i < n; ++i)
    for (size_t k = 0; k < S; ++k) blk[i][k] = next_byte();
  CHECK(oracle_encode(n, p, gen, (const uint8_t *const *)blk, blk + n, S) == 0);
  int sets = 0;
  for (unsigned m = 1; m < (1u << nb); ++m) {
    int er[32], ne = 0;
    for (int b = 0; b < nb; ++b)
      if (m >> b & 1u) er[ne++] = b;
    if (ne > p) continue;
    const uint8_t *in[32];
    for (int b = 0; b < nb; ++b) in[b] = (m >> b & 1u) ? NULL : blk[b];
    for (int j = 0; j < ne; ++j) memset(rec[j], 0xA5, S);
    const int rc = oracle_decode(n, p, gen, er, ne, in, rec, S);
    if (vandermonde && rc == -1) continue; /* not every Vandermonde-row submatrix is invertible */
    CHECK(rc == 0);
    for (int j = 0; j < ne; ++j) CHECK(memcmp(rec[j], blk[er[j]], S) == 0);
    ++sets;
  }
  CHECK(sets > 0 || p == 0);
  for (int b = 0; b < nb; ++b) free(blk[b]);
  for (int j = 0; j < p; ++j) free(rec[j]);
  free(blk); free(rec); free(gen);
}

int main(void) {
  /* field: inverses, log/exp, bitmatrix of the identity */
  for (int a = 1; a < 256; ++a) {
    CHECK(oracle_gf_mul((uint8_t)a, oracle_gf_inv((uint8_t)a)) == 1);
    CHECK(oracle_gf_exp(oracle_gf_log(a)) == a);
  }
  uint8_t one = 1, bits[64];
  oracle_bitmatrix(1, 1, &one, bits);
  for (int r = 0; r < 8; ++r)
    for (int c = 0; c < 8; ++c) CHECK(bits[r * 8 + c] == (r == c));
  uint8_t m[4] = {1, 1, 1, 1}, inv[4];
  CHECK(oracle_invert(2, m, inv) != 0); /* singular */
  const size_t sizes[] = {8, 128, 8 * 37};
  for (int s = 0; s < 3; ++s) {
    round_trips(6, 3, sizes[s], 0);
    round_trips(4, 2, sizes[s], 0);
    round_trips(2, 1, sizes[s], 0);
    round_trips(1, 0, sizes[s], 0);
  }
  round_trips(10, 4, 64, 0);
  round_trips(10, 4, 64, 1);
  uint8_t small[16];
  CHECK(oracle_cauchy(200, 100, small) != 0); /* n + p > 256: refused before any write */
  CHECK(oracle_cauchy(0, 1, small) != 0);
  printf("oracle_driver: %d check failures\n", failures);
  return failures == 0 ? 0 : 1;
}
