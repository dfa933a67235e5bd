// Exact integer lattice algebra for the planner.  See intmat.hpp.
#include "intmat.hpp"

#include <algorithm>
#include <cstdlib>
#include <utility>

namespace lfft {

i64 narrow(i128 v) {
  if (v > (i128)INT64_MAX || v < (i128)INT64_MIN) throw IntOverflow{};
  return (i64)v;
}

i64 floordiv(i64 a, i64 b) {
  i64 q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

i64 posmod(i64 a, i64 b) {
  i64 r = a % b;
  return r < 0 ? r + b : r;
}

i64 gcd64(i64 a, i64 b) {
  a = a < 0 ? -a : a;
  b = b < 0 ? -b : b;
  while (b) {
    i64 t = a % b;
    a = b;
    b = t;
  }
  return a;
}

i64 egcd(i64 a, i64 b, i64& x, i64& y) {
  // iterative extended Euclid on int128 to stay exact
  i128 r0 = a, r1 = b, s0 = 1, s1 = 0, t0 = 0, t1 = 1;
  while (r1 != 0) {
    i128 q = r0 / r1;
    i128 r2 = r0 - q * r1; r0 = r1; r1 = r2;
    i128 s2 = s0 - q * s1; s0 = s1; s1 = s2;
    i128 t2 = t0 - q * t1; t0 = t1; t1 = t2;
  }
  if (r0 < 0) { r0 = -r0; s0 = -s0; t0 = -t0; }
  x = narrow(s0);
  y = narrow(t0);
  return narrow(r0);
}

i64 modinv(i64 a, i64 n) {
  if (n == 1) return 0;
  i64 x, y;
  i64 g = egcd(posmod(a, n), n, x, y);
  if (g != 1) throw NotIntegral{};
  return posmod(x, n);
}

i64 mulmod(i64 a, i64 b, i64 n) {
  i128 p = ((i128)a * (i128)b) % (i128)n;
  if (p < 0) p += n;
  return (i64)p;
}

Mat Mat::identity(int d) {
  Mat I;
  I.d = d;
  for (int i = 0; i < d; ++i) I.a[i][i] = 1;
  return I;
}

Mat Mat::from(int d, const i64* rm) {
  Mat A;
  A.d = d;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) A.a[i][j] = rm[i * d + j];
  return A;
}

Mat matmul(const Mat& A, const Mat& B) {
  Mat C;
  C.d = A.d;
  for (int i = 0; i < A.d; ++i)
    for (int j = 0; j < A.d; ++j) {
      i128 s = 0;
      for (int k = 0; k < A.d; ++k) {
        s += (i128)A.a[i][k] * (i128)B.a[k][j];
        narrow(s);
      }
      C.a[i][j] = narrow(s);
    }
  return C;
}

Mat transpose(const Mat& A) {
  Mat T;
  T.d = A.d;
  for (int i = 0; i < A.d; ++i)
    for (int j = 0; j < A.d; ++j) T.a[i][j] = A.a[j][i];
  return T;
}

bool equal(const Mat& A, const Mat& B) {
  if (A.d != B.d) return false;
  for (int i = 0; i < A.d; ++i)
    for (int j = 0; j < A.d; ++j)
      if (A.a[i][j] != B.a[i][j]) return false;
  return true;
}

// Laplace expansion over int128 (d <= 4, so at most 24 terms).
static i128 det128(const i64 a[kMaxD][kMaxD], int d, const int* rows, const int* cols) {
  if (d == 1) return a[rows[0]][cols[0]];
  i128 s = 0;
  int sub[kMaxD];
  for (int c = 0; c < d; ++c) {
    int k = 0;
    for (int cc = 0; cc < d; ++cc)
      if (cc != c) sub[k++] = cols[cc];
    i128 m = det128(a, d - 1, rows + 1, sub);
    i128 t = (i128)a[rows[0]][cols[c]] * m;
    s += (c % 2 == 0) ? t : -t;
  }
  return s;
}

i64 det(const Mat& A) {
  int r[kMaxD], c[kMaxD];
  for (int i = 0; i < A.d; ++i) r[i] = c[i] = i;
  return narrow(det128(A.a, A.d, r, c));
}

Mat adjugate(const Mat& A) {
  Mat adj;
  adj.d = A.d;
  if (A.d == 1) {
    adj.a[0][0] = 1;
    return adj;
  }
  int rows[kMaxD], cols[kMaxD];
  for (int i = 0; i < A.d; ++i)
    for (int j = 0; j < A.d; ++j) {
      // adj_ij = (-1)^{i+j} minor with row j and column i removed
      int k = 0;
      for (int r = 0; r < A.d; ++r)
        if (r != j) rows[k++] = r;
      k = 0;
      for (int c = 0; c < A.d; ++c)
        if (c != i) cols[k++] = c;
      i128 m = det128(A.a, A.d - 1, rows, cols);
      adj.a[i][j] = narrow(((i + j) % 2 == 0) ? m : -m);
    }
  return adj;
}

Mat unimodular_inverse(const Mat& A) {
  i64 D = det(A);
  if (D != 1 && D != -1) throw NotIntegral{};
  Mat adj = adjugate(A);
  if (D == -1)
    for (int i = 0; i < A.d; ++i)
      for (int j = 0; j < A.d; ++j) adj.a[i][j] = -adj.a[i][j];
  return adj;
}

Mat left_quotient(const Mat& J, const Mat& M) {
  i64 D = det(J);
  if (D == 0) throw SingularMatrix{};
  Mat adj = adjugate(J);
  Mat P = matmul(adj, M);  // = D * J^{-1} M
  Mat N;
  N.d = M.d;
  for (int i = 0; i < M.d; ++i)
    for (int j = 0; j < M.d; ++j) {
      if (P.a[i][j] % D != 0) throw NotIntegral{};
      N.a[i][j] = P.a[i][j] / D;
    }
  return N;
}

void matvec(const Mat& A, const i64* v, i64* out) {
  for (int i = 0; i < A.d; ++i) {
    i128 s = 0;
    for (int j = 0; j < A.d; ++j) {
      s += (i128)A.a[i][j] * (i128)v[j];
      narrow(s);
    }
    out[i] = narrow(s);
  }
}

void hnf(const Mat& M, Mat& H, Mat& U) {
  const int d = M.d;
  if (det(M) == 0) throw SingularMatrix{};
  H = M;
  U = Mat::identity(d);
  auto colop = [&](int dst, int src, i64 f) {  // col_dst -= f * col_src
    if (!f) return;
    for (int r = 0; r < d; ++r) {
      H.a[r][dst] = csub(H.a[r][dst], cmul(f, H.a[r][src]));
      U.a[r][dst] = csub(U.a[r][dst], cmul(f, U.a[r][src]));
    }
  };
  auto colswap = [&](int x, int y) {
    for (int r = 0; r < d; ++r) {
      std::swap(H.a[r][x], H.a[r][y]);
      std::swap(U.a[r][x], U.a[r][y]);
    }
  };
  for (int i = d - 1; i >= 0; --i) {
    // Euclid on row i over columns 0..i; the gcd ends in column i
    for (;;) {
      int p = -1, nnz = 0;
      for (int c = 0; c <= i; ++c)
        if (H.a[i][c] != 0) {
          ++nnz;
          if (p < 0 || std::llabs(H.a[i][c]) < std::llabs(H.a[i][p])) p = c;
        }
      if (nnz <= 1) {
        if (p != i) colswap(p, i);
        break;
      }
      for (int c = 0; c <= i; ++c)
        if (c != p && H.a[i][c] != 0) colop(c, p, floordiv(H.a[i][c], H.a[i][p]));
    }
    if (H.a[i][i] < 0)
      for (int r = 0; r < d; ++r) {
        H.a[r][i] = -H.a[r][i];
        U.a[r][i] = -U.a[r][i];
      }
  }
  for (int i = d - 1; i >= 0; --i)
    for (int j = i + 1; j < d; ++j) colop(j, i, floordiv(H.a[i][j], H.a[i][i]));
}

void reduce_box(const Mat& H, i64* v) {
  for (int i = H.d - 1; i >= 0; --i) {
    i64 q = floordiv(v[i], H.a[i][i]);
    if (q)
      for (int r = 0; r <= i; ++r) v[r] = csub(v[r], cmul(q, H.a[r][i]));
  }
}

i64 box_index(const Mat& H, const i64* v) {
  i64 idx = 0;
  for (int i = 0; i < H.d; ++i) idx = cadd(cmul(idx, H.a[i][i]), v[i]);
  return idx;
}

// ---------------------------------------------------------------------------
// Smith normal form with tracked transforms.  Invariant: Q * A * R = M, with
// Qinv = Q^{-1} and Rinv = R^{-1}; A is driven to diag(eps).
namespace {
struct SnfState {
  int d;
  Mat A, Q, Qinv, R, Rinv;
  // row_i -= f * row_t
  void rowop(int i, int t, i64 f) {
    if (!f) return;
    for (int c = 0; c < d; ++c) A.a[i][c] = csub(A.a[i][c], cmul(f, A.a[t][c]));
    for (int r = 0; r < d; ++r) Q.a[r][t] = cadd(Q.a[r][t], cmul(f, Q.a[r][i]));
    for (int c = 0; c < d; ++c) Qinv.a[i][c] = csub(Qinv.a[i][c], cmul(f, Qinv.a[t][c]));
  }
  // col_j -= f * col_t
  void colop(int j, int t, i64 f) {
    if (!f) return;
    for (int r = 0; r < d; ++r) A.a[r][j] = csub(A.a[r][j], cmul(f, A.a[r][t]));
    for (int c = 0; c < d; ++c) R.a[t][c] = cadd(R.a[t][c], cmul(f, R.a[j][c]));
    for (int r = 0; r < d; ++r) Rinv.a[r][j] = csub(Rinv.a[r][j], cmul(f, Rinv.a[r][t]));
  }
  void rowswap(int i, int t) {
    if (i == t) return;
    for (int c = 0; c < d; ++c) std::swap(A.a[i][c], A.a[t][c]);
    for (int r = 0; r < d; ++r) std::swap(Q.a[r][i], Q.a[r][t]);
    for (int c = 0; c < d; ++c) std::swap(Qinv.a[i][c], Qinv.a[t][c]);
  }
  void colswap(int j, int t) {
    if (j == t) return;
    for (int r = 0; r < d; ++r) std::swap(A.a[r][j], A.a[r][t]);
    for (int c = 0; c < d; ++c) std::swap(R.a[j][c], R.a[t][c]);
    for (int r = 0; r < d; ++r) std::swap(Rinv.a[r][j], Rinv.a[r][t]);
  }
  void rowneg(int t) {
    for (int c = 0; c < d; ++c) A.a[t][c] = -A.a[t][c];
    for (int r = 0; r < d; ++r) Q.a[r][t] = -Q.a[r][t];
    for (int c = 0; c < d; ++c) Qinv.a[t][c] = -Qinv.a[t][c];
  }
};
}  // namespace

Smith smith(const Mat& M) {
  const int d = M.d;
  if (det(M) == 0) throw SingularMatrix{};
  SnfState s;
  s.d = d;
  s.A = M;
  s.Q = s.Qinv = s.R = s.Rinv = Mat::identity(d);
  for (int t = 0; t < d; ++t) {
    for (;;) {
      // pivot: smallest non-zero |entry| of the trailing block
      int pi = -1, pj = -1;
      for (int i = t; i < d; ++i)
        for (int j = t; j < d; ++j)
          if (s.A.a[i][j] != 0 && (pi < 0 || std::llabs(s.A.a[i][j]) < std::llabs(s.A.a[pi][pj]))) {
            pi = i;
            pj = j;
          }
      s.rowswap(pi, t);
      s.colswap(pj, t);
      bool clean = true;
      for (int i = t + 1; i < d; ++i) {
        s.rowop(i, t, floordiv(s.A.a[i][t], s.A.a[t][t]));
        if (s.A.a[i][t] != 0) clean = false;
      }
      for (int j = t + 1; j < d; ++j) {
        s.colop(j, t, floordiv(s.A.a[t][j], s.A.a[t][t]));
        if (s.A.a[t][j] != 0) clean = false;
      }
      if (!clean) continue;
      // divisibility of the trailing block by the pivot
      int bad = -1;
      for (int i = t + 1; i < d && bad < 0; ++i)
        for (int j = t + 1; j < d; ++j)
          if (s.A.a[i][j] % s.A.a[t][t] != 0) {
            bad = i;
            break;
          }
      if (bad < 0) break;
      s.rowop(t, bad, -1);  // row_t += row_bad
    }
    if (s.A.a[t][t] < 0) s.rowneg(t);
  }
  Smith S;
  S.d = d;
  S.Q = s.Q;
  S.Qinv = s.Qinv;
  S.R = s.R;
  S.Rinv = s.Rinv;
  for (int i = 0; i < d; ++i) S.eps[i] = s.A.a[i][i];
  return S;
}

// ---------------------------------------------------------------------------
// Basis alignment through automorphisms of the eps-grid.
//
// An integer matrix A acts on grid coordinates lambda -> A lambda.  It is a
// well defined automorphism of Z_eps1 x ... x Z_epsd lifting to a new Smith
// factorisation when A is unimodular and B = E^{-1} A E is integral
// (A_ji divisible by eps_j/eps_i for i < j).  Then M = (Q A^{-1}) E (B R).
namespace {
struct Gamma {
  Smith& S;
  explicit Gamma(Smith& s) : S(s) {}
  void apply(const Mat& A, const Mat& Ainv) {
    const int d = S.d;
    Mat B, Binv;
    B.d = Binv.d = d;
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        i128 nb = (i128)A.a[i][j] * S.eps[j];
        i128 ni = (i128)Ainv.a[i][j] * S.eps[j];
        if (nb % S.eps[i] != 0 || ni % S.eps[i] != 0) throw NotIntegral{};
        B.a[i][j] = narrow(nb / S.eps[i]);
        Binv.a[i][j] = narrow(ni / S.eps[i]);
      }
    S.Qinv = matmul(A, S.Qinv);
    S.Q = matmul(S.Q, Ainv);
    S.R = matmul(B, S.R);
    S.Rinv = matmul(S.Rinv, Binv);
  }
  // lambda_j += f * lambda_i
  void add(int j, int i, i64 f) {
    if (!f) return;
    Mat A = Mat::identity(S.d), Ai = Mat::identity(S.d);
    A.a[j][i] = f;
    Ai.a[j][i] = -f;
    apply(A, Ai);
  }
  void neg(int j) {
    Mat A = Mat::identity(S.d);
    A.a[j][j] = -1;
    apply(A, A);
  }
};

std::vector<i64> prime_factors(i64 n) {
  std::vector<i64> p;
  for (i64 q = 2; q * q <= n; ++q)
    if (n % q == 0) {
      p.push_back(q);
      while (n % q == 0) n /= q;
    }
  if (n > 1) p.push_back(n);
  return p;
}
}  // namespace

bool align_last_cycle(Smith& S0, const Mat& M, int c) {
  const int d = S0.d;
  const int L = d - 1;
  const i64 n = S0.eps[L];
  if (n <= 1) return false;
  Smith S = S0;
  try {
    Gamma G(S);
    auto coords = [&](i64* x) {
      for (int j = 0; j < d; ++j) x[j] = posmod(S.Qinv.a[j][c], S.eps[j]);
    };
    i64 x[kMaxD];
    coords(x);
    // 1. make x_L a unit mod n by adding multiples of (n/eps_i) x_i, i < L
    std::vector<i64> primes = prime_factors(n);
    i64 rad = 1;
    for (i64 p : primes) rad *= p;
    i64 cf[kMaxD] = {0, 0, 0, 0};
    for (i64 p : primes) {
      if (x[L] % p != 0) continue;
      int use = -1;
      for (int i = 0; i < L; ++i) {
        i64 b = mulmod(n / S.eps[i], x[i], p);
        if (b != 0) {
          use = i;
          break;
        }
      }
      if (use < 0) return false;  // e_c does not have maximal order
      // CRT: c_use = 1 (mod p), other coefficients 0 (mod p)
      i64 Rp = rad / p;
      i64 e = mulmod(Rp, modinv(Rp % p, p), rad);
      cf[use] = (cf[use] + e) % rad;
    }
    for (int i = 0; i < L; ++i) G.add(L, i, cmul(cf[i], n / S.eps[i]));
    coords(x);
    if (gcd64(x[L], n) != 1) return false;
    // 2. clear the other coordinates: lambda_j += f lambda_L
    for (int j = 0; j < L; ++j) {
      if (S.eps[j] == 1) continue;
      i64 u = x[L] % S.eps[j];
      i64 f = posmod(-mulmod(x[j], modinv(u, S.eps[j]), S.eps[j]), S.eps[j]);
      G.add(j, L, f);
    }
    coords(x);
    // 3. scale the last coordinate to 1
    i64 u = x[L];
    if (u == n - 1) {
      G.neg(L);
    } else if (u != 1) {
      if (d < 2) return false;
      const int k = L - 1;
      i64 v = modinv(u, n);
      i128 uv1 = (i128)u * v - 1;
      i64 beta = narrow(uv1 / n);
      Mat A = Mat::identity(d), Ai = Mat::identity(d);
      A.a[k][k] = u;
      A.a[k][L] = cmul(S.eps[k], beta);
      A.a[L][k] = n / S.eps[k];
      A.a[L][L] = v;
      Ai.a[k][k] = v;
      Ai.a[k][L] = -A.a[k][L];
      Ai.a[L][k] = -A.a[L][k];
      Ai.a[L][L] = u;
      G.apply(A, Ai);
    }
    coords(x);
    for (int j = 0; j < L; ++j)
      if (x[j] != 0) return false;
    if (x[L] != 1) return false;
    // verify the factorisation exactly
    Mat E = Mat::identity(d);
    for (int i = 0; i < d; ++i) E.a[i][i] = S.eps[i];
    if (!equal(matmul(matmul(S.Q, E), S.R), M)) return false;
    if (!equal(matmul(S.Q, S.Qinv), Mat::identity(d))) return false;
    if (!equal(matmul(S.R, S.Rinv), Mat::identity(d))) return false;
  } catch (const IntOverflow&) {
    return false;
  } catch (const NotIntegral&) {
    return false;
  }
  S0 = S;
  return true;
}

}  // namespace lfft
