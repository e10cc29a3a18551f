// gf.hpp -- GF(2^8) arithmetic and coding matrices for the SLP compiler.
//
// The field is GF(2)[x]/(x^8+x^4+x^3+x^2+1) (0x11D, Sec. 7.1).  Products come
// from a 256x256 table filled by shift-and-add multiplication; inverses from
// a search of that table.  Matrices are row-major byte vectors.
#pragma once

#include <cstdint>
#include <vector>

namespace ec {

namespace gf {
uint8_t mul(uint8_t a, uint8_t b);
uint8_t inv(uint8_t a);  // 0 -> 0
uint8_t pow_x(int e);    // x^e, e >= 0
}  // namespace gf

using Mat = std::vector<uint8_t>;  // row-major

// [I_n ; P], P[i][j] = 1/(i + (p + j)).
Mat cauchy_generator(int n, int p);
// [I_n ; P], P[r][j] = x^(r*j).
Mat vandermonde_rows_generator(int n, int p);

// Gauss-Jordan inverse of an n x n matrix; false if singular.
bool invert(int n, const Mat &m, Mat &inv);

// Decode rows for an erasure pattern (Sec. 1): the survivors are the n
// lowest-indexed blocks not erased; M = gen[survivors]; for each erased block
// e (in the given order) the row gen[e] . M^-1.  Returns 0, or -1 singular.
int decode_rows(int n, int p, const Mat &gen, const std::vector<int> &erased, Mat &rows,
                std::vector<int> &survivors);

}  // namespace ec
