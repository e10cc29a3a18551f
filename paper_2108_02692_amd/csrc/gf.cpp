// gf.cpp -- GF(2^8)/0x11D field and coding matrices (Secs. 1 and 7.1).
#include "gf.hpp"

#include <algorithm>

namespace ec {
namespace gf {
namespace {

struct Tables {
  uint8_t prod[256][256];
  uint8_t inverse[256];
  Tables() {
    // Shift-and-add: for every bit of b, add a*x^k reduced mod 0x11D.
    for (int a = 0; a < 256; ++a) {
      for (int b = 0; b < 256; ++b) {
        unsigned acc = 0, aa = (unsigned)a, bb = (unsigned)b;
        while (bb) {
          if (bb & 1u) acc ^= aa;
          bb >>= 1;
          aa <<= 1;
          if (aa & 0x100u) aa ^= 0x11Du;
        }
        prod[a][b] = (uint8_t)acc;
      }
    }
    inverse[0] = 0;
    for (int a = 1; a < 256; ++a)
      for (int b = 1; b < 256; ++b)
        if (prod[a][b] == 1) { inverse[a] = (uint8_t)b; break; }
  }
};

const Tables &T() {
  static const Tables t;  // thread-safe initialisation
  return t;
}

}  // namespace

uint8_t mul(uint8_t a, uint8_t b) { return T().prod[a][b]; }
uint8_t inv(uint8_t a) { return T().inverse[a]; }
uint8_t pow_x(int e) {
  uint8_t r = 1;
  e %= 255;
  for (int i = 0; i < e; ++i) r = mul(r, 2);
  return r;
}

}  // namespace gf

Mat cauchy_generator(int n, int p) {
  Mat g((size_t)(n + p) * n, 0);
  for (int i = 0; i < n; ++i) g[(size_t)i * n + i] = 1;
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < n; ++j) g[(size_t)(n + i) * n + j] = gf::inv((uint8_t)(i ^ (p + j)));
  return g;
}

Mat vandermonde_rows_generator(int n, int p) {
  Mat g((size_t)(n + p) * n, 0);
  for (int i = 0; i < n; ++i) g[(size_t)i * n + i] = 1;
  for (int r = 0; r < p; ++r)
    for (int j = 0; j < n; ++j) g[(size_t)(n + r) * n + j] = gf::pow_x(r * j);
  return g;
}

bool invert(int n, const Mat &m, Mat &out) {
  // Augmented [m | I] reduced to [I | m^-1].
  const int w = 2 * n;
  std::vector<uint8_t> a((size_t)n * w, 0);
  for (int r = 0; r < n; ++r) {
    for (int c = 0; c < n; ++c) a[(size_t)r * w + c] = m[(size_t)r * n + c];
    a[(size_t)r * w + n + r] = 1;
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    while (piv < n && a[(size_t)piv * w + c] == 0) ++piv;
    if (piv == n) return false;
    if (piv != c)
      for (int k = 0; k < w; ++k) std::swap(a[(size_t)piv * w + k], a[(size_t)c * w + k]);
    const uint8_t s = gf::inv(a[(size_t)c * w + c]);
    for (int k = 0; k < w; ++k) a[(size_t)c * w + k] = gf::mul(a[(size_t)c * w + k], s);
    for (int r = 0; r < n; ++r) {
      const uint8_t f = a[(size_t)r * w + c];
      if (r == c || f == 0) continue;
      for (int k = 0; k < w; ++k) a[(size_t)r * w + k] ^= gf::mul(f, a[(size_t)c * w + k]);
    }
  }
  out.assign((size_t)n * n, 0);
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) out[(size_t)r * n + c] = a[(size_t)r * w + n + c];
  return true;
}

int decode_rows(int n, int p, const Mat &gen, const std::vector<int> &erased, Mat &rows,
                std::vector<int> &survivors) {
  survivors.clear();
  for (int b = 0; b < n + p && (int)survivors.size() < n; ++b)
    if (std::find(erased.begin(), erased.end(), b) == erased.end()) survivors.push_back(b);
  Mat M((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < n; ++c) M[(size_t)i * n + c] = gen[(size_t)survivors[i] * n + c];
  Mat Mi;
  if (!invert(n, M, Mi)) return -1;
  rows.assign(erased.size() * (size_t)n, 0);
  for (size_t e = 0; e < erased.size(); ++e)
    for (int c = 0; c < n; ++c) {
      uint8_t s = 0;
      for (int t = 0; t < n; ++t) s ^= gf::mul(gen[(size_t)erased[e] * n + t], Mi[(size_t)t * n + c]);
      rows[e * n + c] = s;
    }
  return 0;
}

}  // namespace ec
