/*
 * rs_oracle.c -- CPU oracle for RS(n,p) erasure coding over GF(2^8).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only tests/, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, table or header with the HIP path.
 *
 * It is the plain definition of what the XOR-program path must reproduce:
 * every output byte is computed symbol by symbol with log/antilog tables,
 * never through a bitmatrix or a straight-line program.
 *
 *  - Field: GF(2^8) with the primitive polynomial x^8+x^4+x^3+x^2+1 (0x11D),
 *    the field of the paper's evaluation setup (Sec. 7.1, "Dataset").
 *  - Coding: systematic generator G = [I_n ; P]; a data vector D of n
 *    symbols is coded as G.D, and decoding inverts the n x n submatrix of G
 *    formed by n surviving rows (Sec. 1, the RS encode/decode equations).
 *  - Layout: each S-byte block is cut into 8 contiguous strips of L = S/8
 *    bytes.  For a byte offset k and a bit position b, block i carries the
 *    field symbol X_i = sum_c bit_b(strip_c[k]) * x^c.  This is the
 *    byte <-> 8-bit-vector isomorphism of Sec. 1 applied "vertically": strip
 *    c holds the coefficient of x^c.  Parity symbol bit r goes to bit b of
 *    parity strip r at offset k.
 *
 * Single-threaded on purpose: it is the slow, obviously-correct checker.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_POLY 0x11D

static uint8_t g_exp[512];
static int g_log[256];
static int g_ready = 0;

/* exp[i] = alpha^i with alpha = x (0x02); log is its inverse on nonzero
 * bytes.  The table is doubled so exp[a+b] needs no reduction mod 255. */
static void tables(void) {
  if (g_ready) return;
  unsigned v = 1;
  for (int i = 0; i < 255; ++i) {
    g_exp[i] = (uint8_t)v;
    g_log[v] = i;
    v <<= 1;
    if (v & 0x100) v ^= ORACLE_POLY;
  }
  for (int i = 255; i < 512; ++i) g_exp[i] = g_exp[i - 255];
  g_log[0] = -1;
  g_ready = 1;
}

int oracle_gf_exp(int i) {
  tables();
  i %= 255;
  if (i < 0) i += 255;
  return g_exp[i];
}

int oracle_gf_log(int a) {
  tables();
  return g_log[a & 0xFF];
}

uint8_t oracle_gf_mul(uint8_t a, uint8_t b) {
  tables();
  if (a == 0 || b == 0) return 0;
  return g_exp[g_log[a] + g_log[b]];
}

/* Multiplicative inverse; 0 has none and maps to 0. */
uint8_t oracle_gf_inv(uint8_t a) {
  tables();
  if (a == 0) return 0;
  return g_exp[255 - g_log[a]];
}

/* Cauchy generator: G = [I_n ; P] with P[i][j] = 1/(x_i + y_j),
 * x_i = i (i < p), y_j = p + j (j < n).  All x_i, y_j are distinct, so every
 * square submatrix of P is nonsingular and G is MDS.
 * gen is (n+p) x n, row-major.  Returns 0, or -1 if n+p > 256. */
int oracle_cauchy(int n, int p, uint8_t *gen) {
  if (n <= 0 || p < 0 || n + p > 256) return -1;
  memset(gen, 0, (size_t)(n + p) * n);
  for (int i = 0; i < n; ++i) gen[i * n + i] = 1;
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < n; ++j)
      gen[(n + i) * n + j] = oracle_gf_inv((uint8_t)(i ^ (p + j)));
  return 0;
}

/* Vandermonde-row generator used for comparison with the paper's printed
 * operation counts: P[r][j] = alpha^(r*j), r < p, j < n (Sec. 7.1; the
 * reading under which the printed XOR counts of the encode and decode
 * programs are reproduced exactly).  gen is (n+p) x n. */
int oracle_vandermonde_rows(int n, int p, uint8_t *gen) {
  if (n <= 0 || p < 0 || n + p > 256) return -1;
  memset(gen, 0, (size_t)(n + p) * n);
  for (int i = 0; i < n; ++i) gen[i * n + i] = 1;
  for (int r = 0; r < p; ++r)
    for (int j = 0; j < n; ++j) gen[(n + r) * n + j] = (uint8_t)oracle_gf_exp(r * j);
  return 0;
}

/* Gauss-Jordan inverse of an n x n matrix over GF(2^8).
 * Returns 0 on success, -1 if the matrix is singular. */
int oracle_invert(int n, const uint8_t *m, uint8_t *inv) {
  uint8_t *a = (uint8_t *)malloc((size_t)n * n);
  if (!a) return -2;
  memcpy(a, m, (size_t)n * n);
  memset(inv, 0, (size_t)n * n);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1;
  for (int col = 0; col < n; ++col) {
    int piv = -1;
    for (int r = col; r < n; ++r)
      if (a[r * n + col]) { piv = r; break; }
    if (piv < 0) { free(a); return -1; }
    if (piv != col) {
      for (int c = 0; c < n; ++c) {
        uint8_t t = a[col * n + c]; a[col * n + c] = a[piv * n + c]; a[piv * n + c] = t;
        t = inv[col * n + c]; inv[col * n + c] = inv[piv * n + c]; inv[piv * n + c] = t;
      }
    }
    uint8_t s = oracle_gf_inv(a[col * n + col]);
    for (int c = 0; c < n; ++c) {
      a[col * n + c] = oracle_gf_mul(a[col * n + c], s);
      inv[col * n + c] = oracle_gf_mul(inv[col * n + c], s);
    }
    for (int r = 0; r < n; ++r) {
      if (r == col || a[r * n + col] == 0) continue;
      uint8_t f = a[r * n + col];
      for (int c = 0; c < n; ++c) {
        a[r * n + c] ^= oracle_gf_mul(f, a[col * n + c]);
        inv[r * n + c] ^= oracle_gf_mul(f, inv[col * n + c]);
      }
    }
  }
  free(a);
  return 0;
}

/* Bitmatrix of an rows x cols GF(2^8) matrix: element e becomes the 8x8 GF(2)
 * block whose column c holds the bits of e * x^c, so that
 * mat-times-symbol in GF(2^8) equals bitmatrix-times-bitvector in GF(2)
 * (Sec. 1, properties (i) and (ii)).  bits is (8 rows) x (8 cols), one byte
 * per entry (0/1), row-major. */
void oracle_bitmatrix(int rows, int cols, const uint8_t *mat, uint8_t *bits) {
  const int W = 8 * cols;
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) {
      uint8_t e = mat[i * cols + j];
      for (int c = 0; c < 8; ++c) {
        uint8_t col = oracle_gf_mul(e, (uint8_t)(1u << c));
        for (int r = 0; r < 8; ++r)
          bits[(size_t)(8 * i + r) * W + 8 * j + c] = (uint8_t)((col >> r) & 1u);
      }
    }
}

/* Core of both encode and decode: out_j = sum_i mat[j][i] * in_i, symbol by
 * symbol, for the byte offsets k0 <= k < k1 of the strips and every bit
 * position b.  in: cols pointers to S-byte blocks; out: rows pointers to
 * S-byte blocks, of which only offsets [k0, k1) of each strip are written.
 * Byte offsets are independent of each other (the symbols at offset k are
 * made of the strips' bytes at k alone), so disjoint ranges may run on
 * separate threads. */
int oracle_apply_range(int rows, int cols, const uint8_t *mat, const uint8_t *const *in,
                       uint8_t *const *out, size_t S, size_t k0, size_t k1) {
  if (S % 8) return -1;
  const size_t L = S / 8;
  if (k0 > k1 || k1 > L) return -1;
  uint8_t *x = (uint8_t *)malloc((size_t)cols);
  uint8_t *acc = (uint8_t *)malloc((size_t)rows * 8);
  if (!x || !acc) { free(x); free(acc); return -2; }
  for (size_t k = k0; k < k1; ++k) {
    memset(acc, 0, (size_t)rows * 8);
    for (int b = 0; b < 8; ++b) {
      /* gather: symbol of block i at (k, b) */
      for (int i = 0; i < cols; ++i) {
        unsigned s = 0;
        for (int c = 0; c < 8; ++c) s |= (unsigned)((in[i][c * L + k] >> b) & 1u) << c;
        x[i] = (uint8_t)s;
      }
      /* multiply and scatter bit r of each output symbol into strip r */
      for (int j = 0; j < rows; ++j) {
        uint8_t y = 0;
        for (int i = 0; i < cols; ++i) y ^= oracle_gf_mul(mat[j * cols + i], x[i]);
        for (int r = 0; r < 8; ++r) acc[j * 8 + r] |= (uint8_t)(((y >> r) & 1u) << b);
      }
    }
    for (int j = 0; j < rows; ++j)
      for (int r = 0; r < 8; ++r) out[j][r * L + k] = acc[j * 8 + r];
  }
  free(x);
  free(acc);
  return 0;
}

/* The whole strips: offsets [0, S/8). */
int oracle_apply(int rows, int cols, const uint8_t *mat, const uint8_t *const *in,
                 uint8_t *const *out, size_t S) {
  if (S % 8) return -1;
  return oracle_apply_range(rows, cols, mat, in, out, S, 0, S / 8);
}

/* Encode: parity_j = sum_i P[j][i] * data_i, with P the last p rows of gen. */
int oracle_encode(int n, int p, const uint8_t *gen, const uint8_t *const *data,
                  uint8_t *const *parity, size_t S) {
  return oracle_apply(p, n, gen + (size_t)n * n, data, parity, S);
}

/* Survivors: the n lowest-indexed blocks not in the erased set.
 * Returns the number found. */
static int survivors(int n, int p, const int *erased, int ne, int *R) {
  int cnt = 0;
  for (int b = 0; b < n + p && cnt < n; ++b) {
    int gone = 0;
    for (int e = 0; e < ne; ++e) gone |= (erased[e] == b);
    if (!gone) R[cnt++] = b;
  }
  return cnt;
}

/* Decode matrix: rows G[e,:] . M^{-1} for each erased block e, where M is the
 * n x n submatrix of gen on the survivor rows (Sec. 1).  out is ne x n.
 * in_rows (n ints) receives the survivor block indices.
 * Returns 0, -1 singular, -3 too many erasures / bad index. */
int oracle_decode_matrix(int n, int p, const uint8_t *gen, const int *erased, int ne,
                         uint8_t *out, int *in_rows) {
  if (ne < 0 || ne > p) return -3;
  for (int e = 0; e < ne; ++e)
    if (erased[e] < 0 || erased[e] >= n + p) return -3;
  int *R = (int *)malloc(sizeof(int) * (size_t)n);
  uint8_t *M = (uint8_t *)malloc((size_t)n * n);
  uint8_t *Mi = (uint8_t *)malloc((size_t)n * n);
  int rc = 0;
  if (!R || !M || !Mi) { rc = -2; goto done; }
  if (survivors(n, p, erased, ne, R) != n) { rc = -3; goto done; }
  for (int i = 0; i < n; ++i) memcpy(M + (size_t)i * n, gen + (size_t)R[i] * n, (size_t)n);
  if (oracle_invert(n, M, Mi) != 0) { rc = -1; goto done; }
  for (int e = 0; e < ne; ++e)
    for (int c = 0; c < n; ++c) {
      uint8_t s = 0;
      for (int t = 0; t < n; ++t) s ^= oracle_gf_mul(gen[(size_t)erased[e] * n + t], Mi[t * n + c]);
      out[e * n + c] = s;
    }
  if (in_rows) memcpy(in_rows, R, sizeof(int) * (size_t)n);
done:
  free(R); free(M); free(Mi);
  return rc;
}

/* Decode: blocks holds n+p pointers (erased entries are ignored and may be
 * NULL); out receives one block per erased index, in the order given. */
int oracle_decode(int n, int p, const uint8_t *gen, const int *erased, int ne,
                  const uint8_t *const *blocks, uint8_t *const *out, size_t S) {
  uint8_t *D = (uint8_t *)malloc((size_t)(ne > 0 ? ne : 1) * n);
  int *R = (int *)malloc(sizeof(int) * (size_t)n);
  const uint8_t **in = (const uint8_t **)malloc(sizeof(void *) * (size_t)n);
  int rc = -2;
  if (!D || !R || !in) goto done;
  rc = oracle_decode_matrix(n, p, gen, erased, ne, D, R);
  if (rc != 0) goto done;
  for (int i = 0; i < n; ++i) in[i] = blocks[R[i]];
  rc = ne > 0 ? oracle_apply(ne, n, D, in, out, S) : 0;
done:
  free(D); free(R); free((void *)in);
  return rc;
}
