// Exact integer lattice algebra for the planner (host only).
//
// All arithmetic is on int64 with every product and sum checked through
// __int128; anything that would not fit throws IntOverflow, which the C ABI
// reports as LFFT_E_OVERFLOW.  d <= 4.
//
// Paper references: Section 2.2 (congruence mod M, pattern P(M), generating
// group G(M), Smith normal form eq. (SNF), group isomorphisms), Section 3
// (pattern basis eq. (basisPM), generating-group basis eq. (basisGM),
// Lemma 1) and Section 4.1, Remark 1 (any biorthogonal pair of bases gives
// the Kronecker form of the Fourier matrix).
#pragma once
#include <cstdint>
#include <vector>

namespace lfft {

using i64 = int64_t;
using i128 = __int128;

struct IntOverflow {};
struct SingularMatrix {};
struct NotIntegral {};

constexpr int kMaxD = 4;

i64 narrow(i128 v);
inline i64 cadd(i64 a, i64 b) { return narrow((i128)a + (i128)b); }
inline i64 csub(i64 a, i64 b) { return narrow((i128)a - (i128)b); }
inline i64 cmul(i64 a, i64 b) { return narrow((i128)a * (i128)b); }
i64 floordiv(i64 a, i64 b);
i64 posmod(i64 a, i64 b);            // b > 0, result in [0, b)
i64 gcd64(i64 a, i64 b);             // >= 0
i64 egcd(i64 a, i64 b, i64& x, i64& y);
i64 modinv(i64 a, i64 n);            // a invertible mod n > 0; result in [0, n)
i64 mulmod(i64 a, i64 b, i64 n);     // (a*b) mod n in [0, n), any signs

struct Mat {
  int d = 0;
  i64 a[kMaxD][kMaxD] = {};
  static Mat identity(int d);
  static Mat from(int d, const i64* rowmajor);
  i64& operator()(int i, int j) { return a[i][j]; }
  i64 operator()(int i, int j) const { return a[i][j]; }
};

Mat matmul(const Mat& A, const Mat& B);
Mat transpose(const Mat& A);
bool equal(const Mat& A, const Mat& B);
i64 det(const Mat& A);
Mat adjugate(const Mat& A);          // adj(A) = det(A) A^{-1}
// exact B = A^{-1} for unimodular A
Mat unimodular_inverse(const Mat& A);
// N = J^{-1} M; throws NotIntegral
Mat left_quotient(const Mat& J, const Mat& M);
void matvec(const Mat& A, const i64* v, i64* out);

// Column Hermite normal form H = M U (U unimodular): upper triangular,
// H_ii > 0, 0 <= H_ij < H_ii for j > i.  H Z^d = M Z^d.
void hnf(const Mat& M, Mat& H, Mat& U);
// representative of v + H Z^d in prod_i [0, H_ii) (H from hnf)
void reduce_box(const Mat& H, i64* v);
i64 box_index(const Mat& H, const i64* v);

// Smith normal form M = Q E R with Q, R unimodular, E = diag(eps),
// eps_1 | eps_2 | ... | eps_d (eq. (SNF)).  Qinv, Rinv are exact inverses.
struct Smith {
  int d = 0;
  Mat Q, Qinv, R, Rinv;
  i64 eps[kMaxD] = {};
};
Smith smith(const Mat& M);

// Basis choice (Remark 1): replace (Q, R) by another Smith factorisation of M
// whose largest cycle is spanned by the unit vector e_c of the sample keys,
// i.e. Q^{-1} e_c = e_{d-1} (mod eps).  The new pair is obtained by an
// automorphism of Z_eps1 x ... x Z_epsd lifted to unimodular matrices, so
// M = Q E R still holds.  Returns false (and leaves S unchanged) if e_c does
// not have maximal order or an intermediate would overflow.
bool align_last_cycle(Smith& S, const Mat& M, int c);

}  // namespace lfft
