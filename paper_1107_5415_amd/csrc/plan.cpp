// Host planner: Smith bases, pass schedules, index tables and twiddles.
//
// The lattice DFT (Section 2.2, eq. Fouriermatrix) becomes a dense
// multi-dimensional DFT over the grid Z_eps1 x ... x Z_epsd once samples and
// frequencies are addressed through a pair of biorthogonal bases (Section 3,
// eqs. basisPM/basisGM, Lemma 1; Theorem 1 and Remark 1 of Section 4.1).
// All integer work happens here, exactly; the kernels only add reduced
// coordinate vectors and look up FP32 twiddles built in FP64.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>

#include "batch.hpp"
#include "fiber.hpp"
#include "kernels.hpp"
#include "ktrace.hpp"

namespace lfft {

namespace {
constexpr i64 kMaxPencil = 8192;   // longest digit handled on chip
constexpr i64 kMaxTile = 8192;     // elements of one single-pass tile
constexpr i64 kMaxBlueAxis = i64(1) << 23;   // longest chirp-z axis (convolution <= 2^24)
constexpr i64 kTileTarget = 4096;  // elements per tile for short pencils
// pyramid levels whose channel (all signals) has at most this many points
// run their channel FFTs in one batched launch
constexpr i64 kChannelBatchElems = i64(1) << 22;

Vec4 zero4() { return Vec4{0, 0, 0, 0}; }

Vec4 reduce4(const Mat& H, Vec4 v) {
  reduce_box(H, v.data());
  return v;
}

Vec4 add4(const Mat& H, const Vec4& a, const Vec4& b) {
  Vec4 c;
  for (int i = 0; i < 4; ++i) c[i] = cadd(a[i], b[i]);
  return reduce4(H, c);
}

Vec4 scale4(const Mat& H, const Vec4& u, i64 k) {
  Vec4 c;
  for (int i = 0; i < 4; ++i) c[i] = cmul(u[i], k);
  return reduce4(H, c);
}

std::vector<int> nontrivial_axes(const Smith& S) {
  std::vector<int> t;
  for (int i = 0; i < S.d; ++i)
    if (S.eps[i] > 1) t.push_back(i);
  return t;
}

// Sample side of basis S on lattice A: natural box of A, unit steps Q e_t.
Side sample_side(const Smith& S, const Mat& A) {
  Side s;
  Mat U;
  hnf(A, s.H, U);
  for (int t : nontrivial_axes(S)) {
    Vec4 u = zero4();
    for (int i = 0; i < S.d; ++i) u[i] = S.Q.a[i][t];
    s.unit.push_back(reduce4(s.H, u));
  }
  return s;
}

// Frequency side of basis S on lattice A: natural box of A^T, unit steps R^T e_t.
Side freq_side(const Smith& S, const Mat& A) {
  Side s;
  Mat U;
  hnf(transpose(A), s.H, U);
  for (int t : nontrivial_axes(S)) {
    Vec4 u = zero4();
    for (int i = 0; i < S.d; ++i) u[i] = S.R.a[t][i];
    s.unit.push_back(reduce4(s.H, u));
  }
  return s;
}

std::vector<int> radices_of(i64 n) {
  std::vector<int> r;
  while (n % 16 == 0 && n > 16 * 1) {
    r.push_back(16);
    n /= 16;
  }
  // remaining power of two as one radix from {2,4,8,16}
  if (n % 16 == 0) {
    r.push_back(16);
    n /= 16;
  } else if (n % 8 == 0) {
    r.push_back(8);
    n /= 8;
  } else if (n % 4 == 0) {
    r.push_back(4);
    n /= 4;
  } else if (n % 2 == 0) {
    r.push_back(2);
    n /= 2;
  }
  for (i64 p = 3; n > 1; p += 2) {
    while (n % p == 0) {
      r.push_back((int)p);
      n /= p;
    }
    if (p * p > n && n > 1) {
      r.push_back((int)n);
      n = 1;
    }
  }
  return r;
}

bool is_pow2(i64 n) { return n > 0 && (n & (n - 1)) == 0; }

// Two on-chip digits n = hi * lo (lo the longest divisor of at most
// kMaxPencil points with hi = n / lo on chip too); 0 if there is none.
i64 two_digit_lo(i64 n) {
  for (i64 c = kMaxPencil; c >= 2; --c)
    if (n % c == 0 && n / c <= kMaxPencil) return c;
  return 0;
}

// Three on-chip digits n = n1 * n2 * n3 for cycles beyond two pencils.  The
// natural-order tables of the first pass span n2 n3 points and those of the
// last pass n1 n2, so the choice keeps both within 2^20 entries where it can
// and then takes the longest shortest digit (pencils of the register-resident
// kernels), then the longest last digit.
bool three_digits(i64 n, i64& n1, i64& n2, i64& n3) {
  std::vector<i64> dv;
  for (i64 c = 2; c <= kMaxPencil; ++c)
    if (n % c == 0) dv.push_back(c);
  bool found = false;
  int best_bucket = 0;
  i64 best_min = 0, best_last = 0;
  for (i64 c : dv) {
    for (i64 a : dv) {
      if ((n / c) % a != 0) continue;
      const i64 b = n / c / a;
      if (b < 2 || b > kMaxPencil) continue;
      const i64 table = std::max(a * b, b * c);
      int bucket = 0;
      while ((i64(1) << (20 + bucket)) < table) ++bucket;
      const i64 mn = std::min(a, std::min(b, c));
      if (!found || bucket < best_bucket ||
          (bucket == best_bucket && (mn > best_min || (mn == best_min && c > best_last)))) {
        found = true;
        best_bucket = bucket;
        best_min = mn;
        best_last = c;
        n1 = a;
        n2 = b;
        n3 = c;
      }
    }
  }
  return found;
}

int ilog2(i64 n) {
  int l = 0;
  while ((i64(1) << l) < n) ++l;
  return l;
}

// power-of-two digit as radices of at most 16, largest first
std::vector<int> pow2_radices(i64 n) {
  std::vector<int> r;
  while (n >= 16) {
    r.push_back(16);
    n /= 16;
  }
  if (n > 1) r.push_back((int)n);
  return r;
}

// Chirp-z tables of one axis of length n: chirp[j] = exp(-pi i (j^2 mod 2n) / n)
// for j < n, and the plain DFT of the convolution kernel b (b_t = conj(chirp)
// at t and at N - t for 0 <= t < n, zero elsewhere) over N points, both built
// in FP64 and rounded once.
struct BlueTables {
  i64 N;
  const float2* chirp;
  const float2* bhat;
};

void fft_host(std::vector<std::complex<double>>& a) {
  // iterative radix-2 decimation in time, exp(-2 pi i jk / N), N a power of two
  const size_t N = a.size();
  for (size_t i = 1, j = 0; i < N; ++i) {
    size_t bit = N >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= N; len <<= 1) {
    for (size_t i = 0; i < N; i += len)
      for (size_t k = 0; k < len / 2; ++k) {
        const double ang = -2.0 * M_PI * (double)k / (double)len;
        const std::complex<double> w(std::cos(ang), std::sin(ang));
        const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
  }
}

struct TwCache {
  Blob* blob;
  std::map<i64, BlueTables> blue;
  BlueTables bluestein(i64 n) {
    auto it = blue.find(n);
    if (it != blue.end()) return it->second;
    i64 N = 1;
    while (N < 2 * n - 1) N *= 2;
    std::vector<std::complex<double>> c(n), b(N, 0.0);
    for (i64 j = 0; j < n; ++j) {
      const i64 r = (i64)(((i128)j * j) % (2 * n));
      const double a = -M_PI * (double)r / (double)n;
      c[j] = std::complex<double>(std::cos(a), std::sin(a));
    }
    for (i64 t = 0; t < n; ++t) {
      b[t] = std::conj(c[t]);
      if (t) b[N - t] = std::conj(c[t]);
    }
    fft_host(b);
    std::vector<float2> cf(n), bf(N);
    for (i64 j = 0; j < n; ++j) cf[j] = make_float2((float)c[j].real(), (float)c[j].imag());
    for (i64 k = 0; k < N; ++k) bf[k] = make_float2((float)b[k].real(), (float)b[k].imag());
    BlueTables t{N, blob->ref(cf), blob->ref(bf)};
    blue[n] = t;
    return t;
  }
  std::map<i64, const float2*> full;
  std::map<i64, std::pair<const float2*, const float2*>> two;
  const float2* table(i64 n) {
    auto it = full.find(n);
    if (it != full.end()) return it->second;
    std::vector<float2> t(n);
    for (i64 k = 0; k < n; ++k) {
      // exact residue k/n; angle reduced by symmetry in double precision
      double a = -2.0 * M_PI * (double)k / (double)n;
      t[k] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    const float2* p = blob->ref(t);
    full[n] = p;
    return p;
  }
  std::pair<const float2*, const float2*> twolevel(i64 N) {
    auto it = two.find(N);
    if (it != two.end()) return it->second;
    std::vector<float2> lo(4096), hi((N + 4095) / 4096);
    for (i64 k = 0; k < 4096; ++k) {
      double a = -2.0 * M_PI * (double)(k % N) / (double)N;
      lo[k] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    for (i64 k = 0; k < (i64)hi.size(); ++k) {
      double a = -2.0 * M_PI * (double)((k * 4096) % N) / (double)N;
      hi[k] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    auto pr = std::make_pair(blob->ref(hi), blob->ref(lo));
    two[N] = pr;
    return pr;
  }
};

struct TableSpec {
  const std::vector<Digit>* digits;
  int a, b;  // digit range enumerated in C order
};

i64 range_count(const std::vector<Digit>& dg, int a, int b) {
  i64 c = 1;
  for (int g = a; g < b; ++g) c *= dg[g].n;
  return c;
}

// natural coordinates of every index of the digit range [a, b)
std::vector<int4> natural_table(const Side& side, const std::vector<Digit>& dg, int a, int b,
                                bool out_weights) {
  i64 cnt = range_count(dg, a, b);
  std::vector<int4> t(cnt);
  std::vector<i64> val(dg.size(), 0);
  for (i64 idx = 0; idx < cnt; ++idx) {
    i64 r = idx;
    for (int g = b - 1; g >= a; --g) {
      val[g] = r % dg[g].n;
      r /= dg[g].n;
    }
    Vec4 c = zero4();
    for (int g = a; g < b; ++g) {
      i64 w = out_weights ? dg[g].w_out : dg[g].w_in;
      c = add4(side.H, c, scale4(side.H, side.unit[dg[g].axis], cmul(val[g], w)));
    }
    t[idx] = make_int4((int)c[0], (int)c[1], (int)c[2], (int)c[3]);
  }
  return t;
}

// linear grid offsets (output weights) of every index of the digit range
std::vector<int4> linear_table(const std::vector<i64>& eps, const std::vector<Digit>& dg, int a,
                               int b) {
  std::vector<i64> gstride(eps.size(), 1);
  for (int j = (int)eps.size() - 2; j >= 0; --j) gstride[j] = gstride[j + 1] * eps[j + 1];
  i64 cnt = range_count(dg, a, b);
  std::vector<int4> t(cnt);
  for (i64 idx = 0; idx < cnt; ++idx) {
    i64 r = idx, off = 0;
    for (int g = b - 1; g >= a; --g) {
      i64 v = r % dg[g].n;
      r /= dg[g].n;
      off += v * dg[g].w_out * gstride[dg[g].axis];
    }
    t[idx] = make_int4((int)off, 0, 0, 0);
  }
  return t;
}

MapDesc natural_map(Blob& blob, const Side& side, int d, const std::vector<Digit>& dg, int a,
                    int b, bool out_weights) {
  MapDesc m{};
  m.mode = MAP_NATURAL;
  m.d = d;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) m.H[i][j] = (i < d && j < d) ? (int)side.H.a[i][j] : 0;
  i64 st = 1;
  for (int i = d - 1; i >= 0; --i) {
    m.box_stride[i] = st;
    st *= side.H.a[i][i];
  }
  for (int i = d; i < 4; ++i) m.box_stride[i] = 0;
  m.To = blob.ref(natural_table(side, dg, 0, a, out_weights));
  m.Tl = blob.ref(natural_table(side, dg, a, b, out_weights));
  m.Ts = blob.ref(natural_table(side, dg, b, (int)dg.size(), out_weights));
  return m;
}

MapDesc identity_map() {
  MapDesc m{};
  m.mode = MAP_IDENTITY;
  return m;
}

// Schedule for fixed tiles of T = 2^tile_lg elements (the batched persistent
// launch): every pass is one power-of-two pencil of 32..T points, so every
// pass runs the register-resident kernel with W = T / L pencils per tile.
// A lattice of m <= T points is one pass.  Otherwise the digits split into a
// leading and a trailing chunk of at most T points each; the boundary lies on
// an axis boundary when one is in range (order bit 2 clear), else in the
// middle of an axis, which is then done four-step: its high digit closes the
// leading chunk and its low digit opens the trailing one.
void tiled_schedule(LatticePlan* p) {
  const int T = p->tile_lg;
  std::vector<int> lg;
  int s = 0;
  for (i64 e : p->eps) {
    if (!is_pow2(e)) throw StatusError{E_UNSUPPORTED};
    lg.push_back(ilog2(e));
    s += lg.back();
  }
  if (s < 5 || s > 2 * T) throw StatusError{E_UNSUPPORTED};
  const int n = (int)lg.size();
  if (s <= T) {
    for (int j = 0; j < n; ++j) p->digits.push_back(Digit{j, p->eps[j], 0, 1, 1});
    p->ranges.push_back(PassRange{0, (int)p->digits.size(), false, 0});
    return;
  }
  // c = log2 of the trailing chunk
  const int lo_c = std::max(5, s - T), hi_c = std::min(T, s - 5);
  int c = -1;
  if (!(p->order & 4)) {
    int suf = 0;
    for (int k = n - 1; k >= 1; --k) {
      suf += lg[k];
      if (suf >= lo_c && suf <= hi_c && (c < 0 || std::abs(2 * suf - s) < std::abs(2 * c - s))) c = suf;
    }
  }
  if (c < 0) c = std::min(hi_c, std::max(lo_c, (s + 1) / 2));
  std::vector<Digit> rev;
  int acc = 0, first_trailing = -1;
  bool split = false;
  for (int j = n - 1; j >= 0; --j) {
    if (acc < c && acc + lg[j] > c) {
      const int lob = c - acc, hib = lg[j] - lob;
      rev.push_back(Digit{j, i64(1) << lob, 2, 1, i64(1) << hib});
      rev.push_back(Digit{j, i64(1) << hib, 1, i64(1) << lob, 1});
      split = true;
    } else {
      rev.push_back(Digit{j, p->eps[j], 0, 1, 1});
    }
    acc += lg[j];
  }
  p->digits.assign(rev.rbegin(), rev.rend());
  const int D = (int)p->digits.size();
  // first digit of the trailing chunk
  int bits = 0;
  for (int g = D - 1; g >= 0; --g) {
    bits += ilog2(p->digits[g].n);
    if (bits == c) {
      first_trailing = g;
      break;
    }
  }
  if (first_trailing <= 0) throw StatusError{E_STATE};
  const PassRange lead{0, first_trailing, split, 0};
  const PassRange trail{first_trailing, D, false, 0};
  if (split || (p->order & 1)) {
    p->ranges.push_back(lead);
    p->ranges.push_back(trail);
  } else {
    p->ranges.push_back(trail);
    p->ranges.push_back(lead);
  }
}

i64 batch_pencils(const LatticePlan* p, const PassDesc& pd) {
  return p->batch * (i64)pd.O * pd.S;
}

void build_engine(LatticePlan* p, Engine& E, const Side& in_side, const Side& out_side, int sign,
                  TwCache& tw) {
  E.sign = sign;
  const auto& dg = p->digits;
  const int D = (int)dg.size();
  const int np = (int)p->ranges.size();
  bool any_split = false;
  for (auto& g : dg) any_split |= (g.part != 0);
  for (int pi = 0; pi < np; ++pi) {
    const PassRange& R = p->ranges[pi];
    PassDesc pd{};
    pd.batch = p->batch;
    pd.O = (int)range_count(dg, 0, R.a);
    pd.L = (int)range_count(dg, R.a, R.b);
    pd.S = (int)range_count(dg, R.b, D);
    i64 tp = std::max<i64>(1, kTileTarget / pd.L);
    if (pd.S > 1) {
      tp = std::min<i64>(tp, pd.S);
      while (pd.S % tp) --tp;
    }
    pd.TP = (int)tp;
    // register-resident kernel for power-of-two pencils of at least 32 points
    bool pow2 = pd.L >= 32 && pd.L <= kMaxPencil && (p->m < (i64(1) << 30));
    for (int g = R.a; g < R.b; ++g) pow2 = pow2 && is_pow2(dg[g].n);
    if (p->tile_lg > 0) {
      // fixed tiles of 2^tile_lg elements (the schedule guarantees the shapes)
      pd.kind = (p->flags & kPlanSplitBf16) ? 3 : 1;
      pd.P = 16;
      pd.W = (int)((i64(1) << p->tile_lg) / pd.L);
      pd.split = 0;
    } else if (pow2) {
      pd.kind = 1;
      if (pd.S == 1) {
        pd.P = 16;
        pd.W = (int)std::max<i64>(1, 4096 / pd.L);
        pd.split = 0;
      } else {
        // widest column tile that divides S and fits 16384 elements; passes
        // with fewer than 512 such tiles get narrower tiles (down to 8
        // columns, whole 64-byte segments) so that every CU has work
        const i64 npen = batch_pencils(p, pd);
        int Wc = 64;
        while (Wc > 1 && (pd.S % Wc != 0 || (i64)Wc * pd.L > 16384)) Wc /= 2;
        while (Wc > 8 && npen / Wc < 512) Wc /= 2;
        pd.W = Wc;
        pd.P = 16;
        pd.split = ((i64)Wc * pd.L * 17 / 16 * 8 > 72 * 1024) ? 1 : 0;
      }
      if ((i64)pd.W * pd.L / pd.P > 1024) pd.kind = 0;
      // the streaming kernel assumes full tiles inside one signal and
      // 32-bit element offsets
      if (pd.kind == 1 && R.b - R.a == 1 && stream_supported(pd.L, pd.W, pd.S > 1) &&
          ((i64)pd.O * pd.S) % pd.W == 0 && p->m < (i64(1) << 28))
        pd.kind = 2;
    }
    pd.nst = 0;
    if (R.b - R.a == 1 && dg[R.a].part == 3) {
      // one whole axis by chirp-z: tables shared by every engine of the plan
      pd.kind = 4;
      int bi = 0;
      for (int g = 0; g < R.a; ++g) bi += dg[g].part == 3 ? 1 : 0;
      pd.blue = bi;
      const BlueTables bt = tw.bluestein(dg[R.a].n);
      pd.bN = (int)bt.N;
      pd.chirp = bt.chirp;
      pd.bhat = bt.bhat;
    }
    for (int g = R.a; g < R.b && pd.kind != 4; ++g) {
      int stride = (int)range_count(dg, g + 1, R.b);
      i64 Ns = 1;
      std::vector<int> rads = pd.kind == 1 ? pow2_radices(dg[g].n) : radices_of(dg[g].n);
      if (pd.kind == 1 && (p->order & 2)) std::reverse(rads.begin(), rads.end());
      for (int r : rads) {
        if (pd.nst >= kMaxStages) throw StatusError{E_UNSUPPORTED};
        StageDesc& s = pd.st[pd.nst++];
        s.radix = r;
        s.n = (int)dg[g].n;
        s.stride = stride;
        s.Ns = (int)Ns;
        s.tw = tw.table(dg[g].n);
        s.lg_r = ilog2(r);
        s.lg_n = ilog2(dg[g].n);
        s.lg_stride = ilog2(stride);
        s.lg_Ns = ilog2(Ns);
        Ns *= r;
      }
    }
    pd.sign = sign;
    pd.scale = (pi == np - 1) ? (float)(1.0 / std::sqrt((double)p->m)) : 1.0f;
    pd.post = R.post ? 1 : 0;
    if (R.post) {
      // the high digit closes this pass (digit b - 1); the still untransformed
      // lower digits of its axis follow it (digits b .. e, the last one the
      // low digit): twiddle exponent k_hi * (their combined input index)
      // modulo the product of the axis's digits from the high one on
      const int hi = R.b - 1;
      if (dg[hi].part != 1 && dg[hi].part != 4) throw StatusError{E_STATE};
      int e = R.b;
      while (e < D && dg[e].part == 4 && dg[e].axis == dg[hi].axis) ++e;
      if (e >= D || dg[e].part != 2 || dg[e].axis != dg[hi].axis) throw StatusError{E_STATE};
      const i64 lo_n = range_count(dg, R.b, e + 1);
      const i64 N = dg[hi].n * lo_n;
      if (N >= (i64(1) << 31)) throw StatusError{E_UNSUPPORTED};
      pd.postN = (int)N;
      pd.post_lmod = (int)dg[hi].n;
      pd.lo_n = (int)lo_n;
      pd.lo_div = (int)range_count(dg, e + 1, D);
      auto pr = tw.twolevel(N);
      pd.tw_hi = pr.first;
      pd.tw_lo = pr.second;
    }
    pd.in = identity_map();
    pd.out = identity_map();
    E.passes.push_back(pd);
  }
  // map variants of the first and the last pass
  const PassRange& R0 = p->ranges.front();
  const PassRange& R1 = p->ranges.back();
  E.in_grid = identity_map();
  E.in_nat = natural_map(p->blob, in_side, p->d, dg, R0.a, R0.b, false);
  E.has_nat_in = true;
  if (any_split) {
    MapDesc m{};
    m.mode = MAP_LINEAR;
    m.To = p->blob.ref(linear_table(p->eps, dg, 0, R1.a));
    m.Tl = p->blob.ref(linear_table(p->eps, dg, R1.a, R1.b));
    m.Ts = p->blob.ref(linear_table(p->eps, dg, R1.b, D));
    E.out_grid = m;
  } else {
    E.out_grid = identity_map();
  }
  E.out_nat = natural_map(p->blob, out_side, p->d, dg, R1.a, R1.b, true);
  E.has_nat_out = true;
}

template <class T>
void patch(T*& ptr, uintptr_t base) {
  if (ptr) ptr = reinterpret_cast<T*>(base + reinterpret_cast<uintptr_t>(ptr) - 1);
}

void patch_map(MapDesc& m, uintptr_t base) {
  patch(m.To, base);
  patch(m.Tl, base);
  patch(m.Ts, base);
}

void patch_engine(Engine& E, uintptr_t base) {
  for (auto& pd : E.passes) {
    for (int i = 0; i < pd.nst; ++i) patch(pd.st[i].tw, base);
    patch(pd.tw_hi, base);
    patch(pd.tw_lo, base);
    patch(pd.chirp, base);
    patch(pd.bhat, base);
    patch_map(pd.in, base);
    patch_map(pd.out, base);
  }
  patch_map(E.in_nat, base);
  patch_map(E.in_grid, base);
  patch_map(E.out_nat, base);
  patch_map(E.out_grid, base);
}

void* upload_blob(const Blob& b) {
  if (b.bytes.empty()) return nullptr;
  void* d = nullptr;
  if (hipMalloc(&d, b.bytes.size()) != hipSuccess) throw StatusError{E_NOMEM};
  if (hipMemcpy(d, b.bytes.data(), b.bytes.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    throw StatusError{E_HIP};
  }
  return d;
}
}  // namespace

size_t Blob::add(const void* p, size_t n) {
  size_t off = (bytes.size() + 255) & ~size_t(255);
  bytes.resize(off + std::max<size_t>(n, 1));
  if (n) std::memcpy(bytes.data() + off, p, n);
  return off;
}

LatticePlan* build_lattice_plan(int d, const i64* Mrm, i64 batch, uint32_t flags, int tile_lg,
                                int order) {
  if (d < 1 || d > kMaxD || !Mrm || batch < 1) throw StatusError{E_ARG};
  auto* p = new LatticePlan();
  try {
    p->d = d;
    p->M = Mat::from(d, Mrm);
    p->batch = batch;
    p->flags = flags;
    // the split-BF16 MFMA kernel works on fixed tiles of 4096 elements
    if ((flags & kPlanSplitBf16) && tile_lg == 0) tile_lg = 12;
    if ((flags & kPlanSplitBf16) && tile_lg != 12) throw StatusError{E_ARG};
    p->tile_lg = tile_lg;
    p->order = order;
    if (tile_lg != 0 && (tile_lg < 8 || tile_lg > 13)) throw StatusError{E_ARG};
    i64 D = det(p->M);
    if (D == 0) throw StatusError{E_SINGULAR};
    p->m = D < 0 ? -D : D;
    if (p->m >= (i64(1) << 31)) throw StatusError{E_UNSUPPORTED};
    if (cmul(p->m, batch) >= (i64(1) << 40)) throw StatusError{E_UNSUPPORTED};
    hnf(p->M, p->HM, p->UM);
    hnf(transpose(p->M), p->HMT, p->UMT);
    p->Sf = smith(p->M);
    p->Sf_aligned = align_last_cycle(p->Sf, p->M, d - 1);
    p->Si = smith(transpose(p->M));
    p->Si_aligned = align_last_cycle(p->Si, transpose(p->M), d - 1);
    for (int i = 0; i < d; ++i)
      if (p->Sf.eps[i] > 1) p->eps.push_back(p->Sf.eps[i]);
    // digits
    if (tile_lg > 0) {
      tiled_schedule(p);
    } else if (p->eps.empty()) {
      p->digits.push_back(Digit{0, 1, 0, 1, 1});
    } else {
      for (int j = 0; j < (int)p->eps.size(); ++j) {
        i64 n = p->eps[j];
        if (n <= kMaxPencil || p->m <= kMaxTile) {
          if (n > kMaxTile) throw StatusError{E_UNSUPPORTED};
          p->digits.push_back(Digit{j, n, 0, 1, 1});
        } else {
          i64 lo = two_digit_lo(n);
          if (!lo) {
            // beyond two pencils: three on-chip digits with two four-step
            // twiddles (input index n1-digit * n2 n3 + n2-digit * n3 +
            // n3-digit, output index k1 + n1 k2 + n1 n2 k3)
            i64 n1 = 0, n2 = 0, n3 = 0;
            if (three_digits(n, n1, n2, n3)) {
              p->digits.push_back(Digit{j, n1, 1, n2 * n3, 1});
              p->digits.push_back(Digit{j, n2, 4, n3, n1});
              p->digits.push_back(Digit{j, n3, 2, 1, n1 * n2});
              continue;
            }
            // no split into on-chip digits: the whole axis by chirp-z
            if (n > kMaxBlueAxis) throw StatusError{E_UNSUPPORTED};
            p->digits.push_back(Digit{j, n, 3, 1, 1});
            continue;
          }
          // power-of-two axes: a high digit of at least 32 points, so that
          // both passes run the register-resident kernels (2^15 = 32 x 1024
          // rather than 4 x 8192; 1.7-2.3 times faster on 2^14 .. 2^17
          // cycles).  Not beyond the streaming kernels' 2^28 bound, where the
          // wider low digit measured faster overall.
          if (is_pow2(n) && n / lo < 32 && n >= 32 * 32 && p->m < (i64(1) << 28)) lo = n / 32;
          i64 hi = n / lo;
          p->digits.push_back(Digit{j, hi, 1, lo, 1});
          p->digits.push_back(Digit{j, lo, 2, 1, hi});
        }
      }
    }
    if (tile_lg == 0 && p->m > kMaxTile) {
      // Leading axes shorter than 32 points in all that cannot share a pass
      // with the next axis: split that axis four-step so that its high digit
      // joins them (a pass of at least 32 points on the register-resident
      // kernels instead of a pass over the short axes alone).
      size_t k = 0;
      i64 P = 1;
      while (k < p->digits.size() && p->digits[k].part == 0 && P * p->digits[k].n < 32) {
        P *= p->digits[k].n;
        ++k;
      }
      // (not beyond the streaming kernels' 2^28 bound, like the long-cycle
      // split above: unmeasured there)
      if (k >= 1 && k < p->digits.size() && p->digits[k].part == 0 && is_pow2(P) &&
          p->m < (i64(1) << 28)) {
        const Digit g = p->digits[k];
        if (is_pow2(g.n) && P * g.n > kMaxPencil) {
          const i64 hi = 32 / P, lo = g.n / hi;
          if (hi >= 2 && lo >= 32) {
            p->digits[k] = Digit{g.axis, hi, 1, lo, 1};
            p->digits.insert(p->digits.begin() + (long)k + 1, Digit{g.axis, lo, 2, 1, hi});
          }
        }
      }
    }
    const int Dg = (int)p->digits.size();
    if (tile_lg > 0) {
      // ranges set by the tiled schedule
    } else if (p->m <= kMaxTile) {
      p->ranges.push_back(PassRange{0, Dg, false, 0});
    } else {
      int i = Dg - 1;
      while (i >= 0) {
        if (p->digits[i].part == 2 && i >= 2 && p->digits[i - 1].part == 4) {
          // an axis split in three: high digit (with the whole axes before
          // it that fit one pencil), then the middle, then the low digit,
          // each of the first two followed by its four-step twiddle
          int a = i - 2;
          i64 prod = p->digits[a].n;
          while (a - 1 >= 0 && p->digits[a - 1].part == 0 && prod * p->digits[a - 1].n <= kMaxPencil) {
            --a;
            prod *= p->digits[a].n;
          }
          p->ranges.push_back(PassRange{a, i - 1, true, p->digits[i].axis});
          p->ranges.push_back(PassRange{i - 1, i, true, p->digits[i].axis});
          p->ranges.push_back(PassRange{i, i + 1, false, 0});
          i = a - 1;
        } else if (p->digits[i].part == 2) {
          // the high digit closes a pass that also takes the whole axes
          // before it while they fit one pencil (no pass over a short axis
          // alone); its four-step twiddle follows the pass
          int a = i - 1;
          i64 prod = p->digits[a].n;
          while (a - 1 >= 0 && p->digits[a - 1].part == 0 && prod * p->digits[a - 1].n <= kMaxPencil) {
            --a;
            prod *= p->digits[a].n;
          }
          p->ranges.push_back(PassRange{a, i, true, p->digits[i].axis});
          p->ranges.push_back(PassRange{i, i + 1, false, 0});
          i = a - 1;
        } else {
          int a = i;
          i64 prod = p->digits[i].n;
          while (a - 1 >= 0 && p->digits[a - 1].part == 0 && prod * p->digits[a - 1].n <= kMaxPencil) {
            --a;
            prod *= p->digits[a].n;
          }
          p->ranges.push_back(PassRange{a, i + 1, false, 0});
          i = a - 1;
        }
      }
    }
    p->ws_elems = p->ranges.size() > 1 ? (size_t)(p->m * batch) : 0;
    // chirp-z axes: inner FFT plans and their share of the workspace
    for (const auto& g : p->digits) {
      if (g.part != 3) continue;
      i64 N = 1;
      while (N < 2 * g.n - 1) N *= 2;
      const i64 pencils = batch * (p->m / g.n);
      LatticePlan* in = build_lattice_plan(1, &N, pencils, flags & kPlanHostOnly);
      p->blue.push_back(in);
      p->blue_ws = std::max(p->blue_ws, (size_t)(2 * pencils * N) + in->ws_elems);
    }
    p->ws_elems += p->blue_ws;
    TwCache tw{&p->blob, {}, {}, {}};
    Side fs = sample_side(p->Sf, p->M);
    Side ff = freq_side(p->Sf, p->M);
    Mat MT = transpose(p->M);
    Side is = sample_side(p->Si, MT);
    Side iff = freq_side(p->Si, MT);
    if (p->eps.empty()) {
      fs.unit.assign(1, zero4());
      ff.unit.assign(1, zero4());
      is.unit.assign(1, zero4());
      iff.unit.assign(1, zero4());
    }
    // the inverse basis must have the same grid (same elementary divisors)
    for (int i = 0; i < d; ++i)
      if (p->Si.eps[i] != p->Sf.eps[i]) throw StatusError{E_STATE};
    build_engine(p, p->fwd, fs, ff, -1, tw);
    build_engine(p, p->inv_grid, ff, fs, +1, tw);
    build_engine(p, p->inv_nat, is, iff, +1, tw);
    bool posts = false;
    for (const auto& R : p->ranges) posts |= R.post;
    if (p->Sf_aligned && !p->Si_aligned && !posts && p->ranges.size() >= 2) {
      // the axes are independent DFTs, so their order is free
      const auto ranges = p->ranges;
      std::reverse(p->ranges.begin(), p->ranges.end());
      build_engine(p, p->inv_rev, ff, fs, +1, tw);
      p->ranges = ranges;
      p->has_inv_rev = true;
    }
    if (p->Si_aligned && !p->Sf_aligned && !posts && p->ranges.size() >= 2 && tile_lg == 0) {
      // the mirror case: a first pass over rows of unaligned samples would
      // gather scattered elements, so the forward runs on the inverse basis
      // with the rows pass last, writing the aligned frequency rows (the
      // fixed-tile schedules keep their forward order)
      const auto ranges = p->ranges;
      std::reverse(p->ranges.begin(), p->ranges.end());
      build_engine(p, p->fwd_rev, iff, is, -1, tw);
      p->ranges = ranges;
      p->has_fwd_rev = true;
    }
    // the reversed engines end with a rows pass onto the aligned side: whole
    // rows of the output, written once and not read again by the call
    for (Engine* E : {p->has_inv_rev ? &p->inv_rev : nullptr, p->has_fwd_rev ? &p->fwd_rev : nullptr}) {
      if (!E || E->passes.empty()) continue;
      PassDesc& last = E->passes.back();
      if (last.kind == 2 && last.S == 1) last.stream_out = 1;
    }
    // the engines in natural order start with a rows pass over the input
    // side that their basis aligns: whole rows of the input, read once
    for (Engine* E : {p->Sf_aligned ? &p->fwd : nullptr, p->Si_aligned ? &p->inv_nat : nullptr}) {
      if (!E || E->passes.empty()) continue;
      PassDesc& first = E->passes.front();
      if (first.kind == 2 && first.S == 1) first.stream_in = 1;
    }
  } catch (const StatusError&) {
    delete p;
    throw;
  } catch (const IntOverflow&) {
    delete p;
    throw StatusError{E_OVERFLOW};
  } catch (const SingularMatrix&) {
    delete p;
    throw StatusError{E_SINGULAR};
  } catch (const NotIntegral&) {
    delete p;
    throw StatusError{E_STATE};
  }
  return p;
}

void upload_plan(LatticePlan* p) {
  for (LatticePlan* in : p->blue) upload_plan(in);
  if (p->dtab) return;
  p->dtab = upload_blob(p->blob);
  uintptr_t base = reinterpret_cast<uintptr_t>(p->dtab);
  patch_engine(p->fwd, base);
  patch_engine(p->inv_grid, base);
  patch_engine(p->inv_nat, base);
  if (p->has_inv_rev) patch_engine(p->inv_rev, base);
  if (p->has_fwd_rev) patch_engine(p->fwd_rev, base);
}

void free_plan(LatticePlan* p) {
  if (!p) return;
  if (p->dtab) (void)hipFree(p->dtab);
  if (p->dbnd) (void)hipFree(p->dbnd);
  for (LatticePlan* in : p->blue) free_plan(in);
  delete p;
}

void build_boundary(LatticePlan* p) {
  static std::mutex mu;
  std::lock_guard<std::mutex> g(mu);
  if (p->bnd_built) return;
  // r(h) = #{j : (sgn adj(M)^T h)_j = m/2 mod m}: only for even m
  const int d = p->d;
  const i64 m = p->m;
  std::vector<i64> idx;
  std::vector<int> rr;
  if (m % 2 == 0) {
    const Mat A = adjugate(p->M);
    const i64 sg = det(p->M) < 0 ? -1 : 1;
    const Mat& H = p->HMT;
    std::vector<i64> v(d, 0);
    for (i64 k = 0; k < m; ++k) {
      i64 r = k;
      for (int i = d - 1; i >= 0; --i) {
        v[i] = r % H.a[i][i];
        r /= H.a[i][i];
      }
      int cnt = 0;
      for (int j = 0; j < d; ++j) {
        i128 acc = 0;
        for (int i = 0; i < d; ++i) acc += (i128)A.a[i][j] * v[i];
        acc = (acc * sg) % m;
        if (acc < 0) acc += m;
        if (acc == m / 2) ++cnt;
      }
      if (cnt) {
        idx.push_back(k);
        rr.push_back(cnt);
      }
    }
  }
  void* dev = nullptr;
  if (p->dtab && !idx.empty()) {
    const size_t n = idx.size();
    if (hipMalloc(&dev, n * (sizeof(i64) + sizeof(int))) != hipSuccess) throw StatusError{E_NOMEM};
    if (hipMemcpy(dev, idx.data(), n * sizeof(i64), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(static_cast<char*>(dev) + n * sizeof(i64), rr.data(), n * sizeof(int),
                  hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(dev);
      throw StatusError{E_HIP};
    }
  }
  p->bnd_idx.swap(idx);
  p->bnd_r.swap(rr);
  p->dbnd = dev;
  p->bnd_built = true;
}

void scale_boundary(const LatticePlan* p, int dir, void* data, long long batch, long long bstride,
                    hipStream_t s) {
  if (!p->bnd_built) throw StatusError{E_STATE};
  const long long n = (long long)p->bnd_idx.size();
  if (n == 0) return;
  float fac[5];
  for (int r = 0; r < 5; ++r) fac[r] = (float)std::pow(2.0, dir * 0.5 * r);
  const i64* idx = static_cast<const i64*>(p->dbnd);
  const int* rr = reinterpret_cast<const int*>(idx + n);
  TraceScope ts(trace_on() ? "boundary_scale_kernel" : nullptr, 16.0 * (double)batch * (double)n,
                s);
  hipError_t e = launch_boundary_scale(reinterpret_cast<const long long*>(idx), rr, n, fac,
                                       static_cast<float2*>(data), batch, bstride, s);
  if (e != hipSuccess) throw StatusError{E_HIP};
}

void natural_to_grid(const LatticePlan* p, int which, i64* out) {
  // which: 0 samples (forward basis), 1 freqs (forward basis),
  //        2 samples of M^T (inverse basis), 3 freqs of M^T (inverse basis)
  const Smith& S = (which < 2) ? p->Sf : p->Si;
  bool freq = (which % 2) == 1;
  const Mat& H = ((which == 0) || (which == 3)) ? p->HM : p->HMT;
  const int d = p->d;
  std::vector<int> t = nontrivial_axes(S);
  i64 cnt = p->m;
  std::vector<i64> v(d, 0);
  for (i64 idx = 0; idx < cnt; ++idx) {
    i64 r = idx;
    for (int i = d - 1; i >= 0; --i) {
      v[i] = r % H.a[i][i];
      r /= H.a[i][i];
    }
    i64 lin = 0;
    for (int tj : t) {
      i128 acc = 0;
      for (int i = 0; i < d; ++i) {
        // lambda = Q^{-1} g ; mu = R^{-T} h  (row t of R^{-T} = column t of R^{-1})
        i64 c = freq ? S.Rinv.a[i][tj] : S.Qinv.a[tj][i];
        acc += (i128)c * v[i];
      }
      i64 e = S.eps[tj];
      i64 x = (i64)(acc % e);
      if (x < 0) x += e;
      lin = lin * e + x;
    }
    out[idx] = lin;
  }
}

void points(const LatticePlan* p, int which, i64* keys, i64* sym) {
  // which 0: keys g of G(M) (Hermite box of M), m M^{-1} g = sgn adj(M) g;
  // which 1: keys h of G(M^T) (Hermite box of M^T), m M^{-T} h = sgn adj(M)^T h.
  // Every coordinate of the second is reduced into [-m/2, m/2) (the symmetric
  // pattern Lambda(M) cap [-1/2, 1/2)^d of Section 6.2, scaled by m).
  const int d = p->d;
  const bool freq = which == 1;
  const Mat& H = freq ? p->HMT : p->HM;
  const Mat A = adjugate(p->M);
  const i64 D = det(p->M);
  const i64 sg = D < 0 ? -1 : 1;
  const i64 m = p->m, half = m / 2;
  std::vector<i64> v(d, 0);
  for (i64 idx = 0; idx < m; ++idx) {
    i64 r = idx;
    for (int i = d - 1; i >= 0; --i) {
      v[i] = r % H.a[i][i];
      r /= H.a[i][i];
    }
    for (int j = 0; j < d; ++j) {
      if (keys) keys[idx * d + j] = v[j];
      if (!sym) continue;
      i128 acc = 0;
      for (int k = 0; k < d; ++k) acc += (i128)(freq ? A.a[k][j] : A.a[j][k]) * v[k];
      acc *= sg;
      i128 t = (acc + half) % m;
      if (t < 0) t += m;
      sym[idx * d + j] = (i64)t - half;
    }
  }
}

namespace {
// One chirp-z pass: gather with the chirp into A (pencils x N), A -> B by the
// inner forward FFT, B times the kernel's DFT, B -> A by the inner inverse
// FFT, scatter with the chirp and the pass's scale.  The inner FFTs are
// unitary, so bhat carries the plain DFT of the kernel: F^{-1}(F a . bhat)
// is the cyclic convolution.  wb: 2 pencils N + the inner plan's workspace.
void exec_chirp_z(const LatticePlan* p, const PassDesc& pd, const float2* src, float2* dst,
                  float2* wb, hipStream_t s) {
  const LatticePlan* in = p->blue[pd.blue];
  const long long tot = in->batch * (long long)pd.bN;
  float2* A = wb;
  float2* B = wb + tot;
  float2* iw = wb + 2 * tot;
  const double by = 8.0 * (double)tot;
  {
    TraceScope ts(trace_on() ? "blue_pre_kernel" : nullptr, by + 8.0 * p->batch * p->m, s);
    if (launch_blue_pre(pd, src, A, s) != hipSuccess) throw StatusError{E_HIP};
  }
  exec_lattice(in, false, false, false, A, B, iw, pd.bN, pd.bN, s);
  {
    TraceScope ts(trace_on() ? "blue_mul_kernel" : nullptr, 2.0 * by, s);
    if (launch_blue_mul(pd, B, s) != hipSuccess) throw StatusError{E_HIP};
  }
  exec_lattice(in, true, false, false, B, A, iw, pd.bN, pd.bN, s);
  {
    TraceScope ts(trace_on() ? "blue_post_kernel" : nullptr, by + 8.0 * p->batch * p->m, s);
    if (launch_blue_post(pd, A, dst, s) != hipSuccess) throw StatusError{E_HIP};
  }
}
}  // namespace

void exec_lattice(const LatticePlan* p, bool inverse, bool in_grid, bool out_grid, const void* in,
                  void* out, void* ws, long long bin, long long bout, hipStream_t s,
                  float scale_mul) {
  const bool nat = !in_grid && !out_grid;
  const Engine& E = !inverse ? ((nat && p->has_fwd_rev) ? p->fwd_rev : p->fwd)
                             : (!nat ? p->inv_grid : (p->has_inv_rev ? p->inv_rev : p->inv_nat));
  const int np = (int)E.passes.size();
  for (int i = 0; i < np; ++i) {
    PassDesc pd = E.passes[i];
    const float2* src = (i == 0) ? static_cast<const float2*>(in) : static_cast<const float2*>(ws);
    float2* dst = (i == np - 1) ? static_cast<float2*>(out) : static_cast<float2*>(ws);
    pd.in.bstride = p->m;
    pd.out.bstride = p->m;
    if (i == 0) {
      pd.in = in_grid ? E.in_grid : E.in_nat;
      pd.in.bstride = bin;
      if (in_grid) pd.stream_in = 0;
    }
    if (i == np - 1) {
      pd.out = out_grid ? E.out_grid : E.out_nat;
      pd.out.bstride = bout;
      pd.scale *= scale_mul;
      if (out_grid) pd.stream_out = 0;
    }
    const double fft_bytes = 16.0 * (double)p->batch * (double)p->m;
    if (pd.kind == 4) {
      exec_chirp_z(p, pd, src, dst, static_cast<float2*>(ws) + (np > 1 ? p->batch * p->m : 0), s);
      continue;
    }
    TraceScope ts(trace_on() ? pass_kernel_name(pd) : nullptr, fft_bytes / np, fft_bytes, s);
    hipError_t e = launch_pass(pd, src, dst, s);
    if (e != hipSuccess) throw StatusError{E_HIP};
  }
}

// ---------------------------------------------------------------------------
// Wavelet plans (Section 5.3)

namespace {
// Multiply-shift division by d (1 <= d < 2^31); checked on boundary values.
FastDiv make_fast_div(i64 d) {
  if (d < 1 || d >= (i64(1) << 31)) throw StatusError{E_STATE};
  int sh = 0;
  while ((i64(1) << sh) < d) ++sh;
  const unsigned long long mag = ((1ull << (31 + sh)) / (unsigned long long)d) + 1;
  if (mag >> 32) throw StatusError{E_STATE};
  FastDiv f{(unsigned)mag, sh};
  const i64 top = (i64(1) << 31) - 1;
  const i64 probes[] = {0, 1, d - 1, d, d + 1, top, top - 1, (top / d) * d, (top / d) * d - 1};
  for (i64 n : probes)
    if (n >= 0 && n <= top && (i64)fast_div((unsigned)n, f) != n / d) throw StatusError{E_STATE};
  return f;
}

// (g0, y0 numerators, v) for |det J| = 2: g0 a unit vector outside J^T Z^d,
// y0 = num/2 the non-zero point of P(J) in [-1/2, 1/2)^d, v = J y0.
void dilation_data(const Mat& J, Vec4& g0, Vec4& v) {
  const int d = J.d;
  i64 DJ = det(J);
  Mat adj = adjugate(J);
  Mat adjT = adjugate(transpose(J));
  g0 = zero4();
  bool found = false;
  for (int i = 0; i < d && !found; ++i) {
    // J^{-T} e_i = adj(J^T) e_i / det J
    for (int r = 0; r < d; ++r)
      if (adjT.a[r][i] % DJ != 0) {
        g0[i] = 1;
        found = true;
        break;
      }
  }
  if (!found) throw StatusError{E_STATE};
  Vec4 num = zero4();
  found = false;
  for (int i = 0; i < d && !found; ++i) {
    bool nonint = false;
    for (int r = 0; r < d; ++r)
      if (adj.a[r][i] % DJ != 0) nonint = true;
    if (!nonint) continue;
    // y = adj(J) e_i / det J = (sgn * adj(J) e_i) / 2; reduce numerator into [-1, 1)
    i64 sg = DJ < 0 ? -1 : 1;
    for (int r = 0; r < d; ++r) {
      i64 n = sg * adj.a[r][i];
      n = posmod(n, 2);          // 0 or 1  ->  y in {0, 1/2}
      num[r] = n == 1 ? -1 : 0;  // 1/2 == -1/2 (mod 1), and [-1/2, 1/2) holds -1/2
    }
    found = true;
  }
  if (!found) throw StatusError{E_STATE};
  v = zero4();
  for (int r = 0; r < d; ++r) {
    i64 acc = 0;
    for (int c = 0; c < d; ++c) acc = cadd(acc, cmul(J.a[r][c], num[c]));
    if (acc % 2 != 0) throw StatusError{E_STATE};
    v[r] = acc / 2;
  }
}
}  // namespace

namespace {
// 32-bit fiber maps: every intermediate of the reductions below 2^30 in
// magnitude.  The reduction starts from k (< KN) or h0 + s (< 2 HM_ii per
// coordinate); reducing coordinate i subtracts q_i * column i with
// |q_i| <= bound_i / HM_ii + 1 from the coordinates above it.
bool fiber_maps_fit_32(const Mat& HN, const Mat& HMt, i64 ml) {
  const int d = HN.d;
  const i64 lim = i64(1) << 30;
  std::vector<i64> bnd(d);
  for (int i = 0; i < d; ++i) bnd[i] = std::max<i64>(HN.a[i][i], 2 * HMt.a[i][i]);
  bool ok = ml < (i64(1) << 28);
  for (int i = d - 1; i >= 0 && ok; --i) {
    const i64 t = bnd[i] / HMt.a[i][i] + 1;
    for (int r = 0; r < i; ++r) {
      bnd[r] += t * HMt.a[r][i];
      if (bnd[r] >= lim) ok = false;
    }
    bnd[i] = HMt.a[i][i];
  }
  return ok;
}

// q-channel split descriptor of one level (q > 2): the natural boxes of
// N_l^T and M_l^T and the fiber offsets s_l = N_l^T g_l.
void fill_split_q(WaveLevel& L, const std::vector<Vec4>& gcls, int q) {
  SplitQDesc& sq = L.sq;
  const int d = L.Ml.d;
  sq.mM = L.ml;
  sq.mN = L.ml / q;
  sq.d = d;
  sq.q = q;
  Mat HN, UN, HMt, UMt;
  hnf(transpose(L.Nl), HN, UN);
  hnf(transpose(L.Ml), HMt, UMt);
  i64 st = 1;
  for (int i = d - 1; i >= 0; --i) {
    sq.hstride[i] = st;
    st *= HMt.a[i][i];
  }
  for (int i = 0; i < 4; ++i) {
    sq.KN[i] = i < d ? (int)HN.a[i][i] : 1;
    if (i >= d) sq.hstride[i] = 0;
    for (int j = 0; j < 4; ++j) sq.HM[i][j] = (i < d && j < d) ? (int)HMt.a[i][j] : 0;
  }
  for (int l = 0; l < kMaxQ; ++l)
    for (int i = 0; i < 4; ++i) sq.s[l][i] = 0;
  for (int l = 0; l < q; ++l) {
    Vec4 s = zero4();
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) s[i] = cadd(s[i], cmul(L.Nl.a[j][i], gcls[l][j]));
    s = reduce4(HMt, s);
    for (int i = 0; i < 4; ++i) sq.s[l][i] = (int)s[i];
  }
  sq.rsq = (float)(1.0 / std::sqrt((double)q));
  sq.narrow = fiber_maps_fit_32(HN, HMt, L.ml) ? 1 : 0;
  for (int i = 0; i < 4; ++i) {
    sq.fKN[i] = make_fast_div(i < d ? HN.a[i][i] : 1);
    sq.fHM[i] = make_fast_div(i < d ? HMt.a[i][i] : 1);
  }
}
}  // namespace

WavePlan* build_wave_plan(int d, const i64* Mrm, const i64* Jrm, int levels, i64 batch,
                          uint32_t flags) {
  if (d < 1 || d > kMaxD || !Mrm || !Jrm || levels < 1 || batch < 1) throw StatusError{E_ARG};
  auto* w = new WavePlan();
  try {
    w->d = d;
    w->M = Mat::from(d, Mrm);
    w->J = Mat::from(d, Jrm);
    w->levels = levels;
    w->batch = batch;
    w->single_stream = (flags & kPlanSingleStream) != 0;
    w->samples = (flags & kPlanSamples) != 0;
    flags &= kPlanHostOnly;
    i64 DJ = det(w->J);
    if (DJ == 0) throw StatusError{E_SINGULAR};
    const i64 q = DJ < 0 ? -DJ : DJ;
    if (q < 2 || q > kMaxQ) throw StatusError{E_UNSUPPORTED};
    w->q = (int)q;
    i64 DM = det(w->M);
    if (DM == 0) throw StatusError{E_SINGULAR};
    w->m = DM < 0 ? -DM : DM;
    w->fftM = build_lattice_plan(d, Mrm, batch, flags);
    Vec4 g0 = zero4(), v = zero4();
    if (q == 2) dilation_data(w->J, g0, v);
    // q > 2: the classes of G(J^T), natural order of the Hermite box of J^T
    std::vector<Vec4> gcls;
    if (q > 2) {
      Mat HJ, UJ;
      hnf(transpose(w->J), HJ, UJ);
      for (i64 idx = 0; idx < q; ++idx) {
        Vec4 g = zero4();
        i64 r = idx;
        for (int i = d - 1; i >= 0; --i) {
          g[i] = r % HJ.a[i][i];
          r /= HJ.a[i][i];
        }
        gcls.push_back(g);
      }
    }
    TwCache tw{&w->blob, {}, {}, {}};
    Mat Ml = w->M;
    for (int l = 0; l < levels; ++l) {
      WaveLevel L;
      L.Ml = Ml;
      try {
        L.Nl = left_quotient(w->J, Ml);
      } catch (const NotIntegral&) {
        throw StatusError{E_NOT_INTEGRAL};
      }
      i64 dm = det(Ml);
      L.ml = dm < 0 ? -dm : dm;
      if (L.ml % q != 0) throw StatusError{E_NOT_INTEGRAL};
      i64 nrm[16];
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) nrm[i * d + j] = L.Nl.a[i][j];
      L.fftN = build_lattice_plan(d, nrm, batch, flags);
      if (q > 2) {
        L.fftW = build_lattice_plan(d, nrm, q - 1, flags);
        fill_split_q(L, gcls, (int)q);
        w->lv.push_back(L);
        Ml = L.Nl;
        continue;
      }
      // split descriptor
      SplitDesc& sd = L.sd;
      sd.mM = L.ml;
      sd.mN = L.ml / 2;
      sd.d = d;
      Mat HN, UN, HMt, UMt;
      hnf(transpose(L.Nl), HN, UN);
      hnf(transpose(Ml), HMt, UMt);
      i64 st = 1;
      for (int i = d - 1; i >= 0; --i) {
        sd.KN[i] = (int)HN.a[i][i];
        sd.kstride[i] = st;
        st *= HN.a[i][i];
      }
      st = 1;
      for (int i = d - 1; i >= 0; --i) {
        sd.hstride[i] = st;
        st *= HMt.a[i][i];
      }
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) sd.HM[i][j] = (i < d && j < d) ? (int)HMt.a[i][j] : 0;
      for (int i = d; i < 4; ++i) sd.KN[i] = 1, sd.kstride[i] = 0, sd.hstride[i] = 0;
      // s = N^T g0
      Vec4 s = zero4();
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) s[i] = cadd(s[i], cmul(L.Nl.a[j][i], g0[j]));
      s = reduce4(HMt, s);
      for (int i = 0; i < 4; ++i) sd.s[i] = (int)s[i];
      // phase: h^T M^{-1} v = (sgn adj(M) v . h) / m ; E = largest eps of M
      Smith Sm = smith(Ml);
      i64 E = 1;
      for (int i = 0; i < d; ++i) E = std::max<i64>(E, Sm.eps[i]);
      Mat adj = adjugate(Ml);
      i64 sg = dm < 0 ? -1 : 1;
      for (int i = 0; i < 4; ++i) sd.w[i] = 0;
      for (int i = 0; i < d; ++i) {
        i128 c = 0;
        for (int j = 0; j < d; ++j) c += (i128)adj.a[i][j] * v[j];
        c *= sg;
        // coefficient of h_i is c / m; times E must be integral
        i128 num = c * E;
        if (num % L.ml != 0) throw StatusError{E_STATE};
        i64 wi = narrow(num / L.ml);
        sd.w[i] = (int)posmod(wi, E);
      }
      sd.E = (int)E;
      sd.tw = tw.table(E);
      // 32-bit index path: bound every intermediate of the fiber maps.  The
      // reduction starts from k (< KN) or h0 + s (< 2 HM_ii per coordinate);
      // reducing coordinate i subtracts q_i * column i with
      // |q_i| <= bound_i / HM_ii + 1 from the coordinates above it.
      {
        bool ok = fiber_maps_fit_32(HN, HMt, L.ml);
        i64 hsum = 0;
        for (int i = 0; i < d; ++i) hsum += HMt.a[i][i];
        if (hsum * E >= (i64(1) << 31)) ok = false;
        sd.narrow = ok ? 1 : 0;
        for (int i = 0; i < 4; ++i) {
          sd.fKN[i] = make_fast_div(i < d ? sd.KN[i] : 1);
          sd.fHM[i] = make_fast_div(i < d ? HMt.a[i][i] : 1);
        }
        sd.fE = make_fast_div(E);
      }
      w->lv.push_back(L);
      Ml = L.Nl;
    }
    size_t fws = w->fftM->ws_elems;
    for (auto& L : w->lv) {
      fws = std::max(fws, L.fftN->ws_elems);
      if (L.fftW) fws = std::max(fws, L.fftW->ws_elems);
    }
    // small levels: their q - 1 wavelet channels (all signals) hold at most
    // kChannelBatchElems points
    w->small_from = levels;
    while (w->small_from > 0 &&
           batch * (q - 1) * (w->lv[w->small_from - 1].ml / q) <= kChannelBatchElems)
      --w->small_from;
    size_t chan_ws = 0;
    w->stage_lvl.assign(levels, 0);
    if (w->small_from < levels) {
      // staging of level l: [B][q-1][m_l/q]; then the final low-pass [B][m_L/q]
      i64 o = 0;
      for (int l = w->small_from; l < levels; ++l) {
        w->stage_lvl[l] = o;
        o += batch * (q - 1) * (w->lv[l].ml / q);
      }
      w->stage_d1 = o;
      o += batch * (w->lv[levels - 1].ml / q);
      w->stage_elems = (size_t)o;
      chan_ws = (size_t)o;   // one workspace slot per channel signal
    }
    w->fw_elems = std::max(fws, chan_ws);
    w->big_d2.assign(levels, 0);
    w->bd_elems = 0;
    size_t fws2 = 0;
    for (int l = 0; l < (q == 2 ? w->small_from : 0); ++l) {
      w->big_d2[l] = (i64)w->bd_elems;
      w->bd_elems += (size_t)(batch * (w->lv[l].ml / 2));
      fws2 = std::max(fws2, w->lv[l].fftN->ws_elems);
    }
    w->fw2_elems = fws2;
    // F0 (m), F1 (m/2), D2 (m/2), FW, staging, BD, FW2
    w->ws_elems = (size_t)(batch * w->m) * 2 + w->fw_elems + w->stage_elems + w->bd_elems +
                  w->fw2_elems;
  } catch (const StatusError&) {
    free_wave_plan(w);
    throw;
  } catch (const IntOverflow&) {
    free_wave_plan(w);
    throw StatusError{E_OVERFLOW};
  } catch (const SingularMatrix&) {
    free_wave_plan(w);
    throw StatusError{E_SINGULAR};
  } catch (const NotIntegral&) {
    free_wave_plan(w);
    throw StatusError{E_NOT_INTEGRAL};
  }
  return w;
}

namespace {
// Batched channel plans: one lattice per (small level, signal, wavelet
// channel) and one per signal for the final low-pass channel.  dec: staging
// -> coefficients (inverse FFTs), rec: coefficients -> staging (forward
// FFTs).
void build_channel_batches(WavePlan* w) {
  if (w->small_from >= w->levels) return;
  const int d = w->d;
  const i64 B = w->batch, q = w->q;
  std::vector<i64> Ms, st, co, wo;
  i64 coff = 0;
  std::vector<i64> coeff_off(w->levels + 1, 0);
  for (int l = 0; l < w->levels; ++l) {
    coeff_off[l] = coff;
    coff += (q - 1) * (w->lv[l].ml / q);
  }
  coeff_off[w->levels] = coff;
  i64 wsx = 0;
  // ch channels of n points per signal, [B][ch][n] in the staging area and
  // ch consecutive blocks of the signal's coefficients
  auto add = [&](const Mat& N, i64 n, i64 ch, i64 stage, i64 cblock) {
    for (i64 b = 0; b < B; ++b) {
      for (i64 j = 0; j < ch; ++j) {
        for (int r = 0; r < d; ++r)
          for (int c = 0; c < d; ++c) Ms.push_back(N.a[r][c]);
        st.push_back(stage + (b * ch + j) * n);
        co.push_back(b * w->m + cblock + j * n);
        wo.push_back(wsx);
        wsx += n;
      }
    }
  };
  for (int l = w->small_from; l < w->levels; ++l)
    add(w->lv[l].Nl, w->lv[l].ml / q, q - 1, w->stage_lvl[l], coeff_off[l]);
  add(w->lv[w->levels - 1].Nl, w->lv[w->levels - 1].ml / q, 1, w->stage_d1, coeff_off[w->levels]);
  const int count = (int)st.size();
  // tiles of 2^13 elements; the forward channels (reconstruction) take
  // their smallest radix first (the fastest of the measured schedules on
  // 2^16 .. 2^22 point channels)
  w->chan_dec = build_batch_plan_at(count, d, Ms.data(), st.data(), co.data(), wo.data(),
                                    (size_t)wsx, 0, 13, 0);
  w->chan_rec = build_batch_plan_at(count, d, Ms.data(), co.data(), st.data(), wo.data(),
                                    (size_t)wsx, 0, 13, 2);
}
}  // namespace

void upload_wave_plan(WavePlan* w) {
  upload_plan(w->fftM);
  if (w->samples) build_boundary(w->fftM);
  for (auto& L : w->lv) {
    upload_plan(L.fftN);
    if (L.fftW) upload_plan(L.fftW);
  }
  if (!w->chan_dec) build_channel_batches(w);
  if (!w->s2) {
    if (hipStreamCreateWithFlags(&w->s2, hipStreamNonBlocking) != hipSuccess) {
      w->s2 = nullptr;
      throw StatusError{E_HIP};
    }
    w->ev.assign(w->levels, nullptr);
    for (auto& e : w->ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) throw StatusError{E_HIP};
    if (hipEventCreateWithFlags(&w->ev_join, hipEventDisableTiming) != hipSuccess)
      throw StatusError{E_HIP};
  }
  if (!w->dtab && !w->blob.bytes.empty()) {
    w->dtab = upload_blob(w->blob);
    uintptr_t base = reinterpret_cast<uintptr_t>(w->dtab);
    for (auto& L : w->lv) patch(L.sd.tw, base);
  }
  w->uploaded = true;
}

void free_wave_plan(WavePlan* w) {
  if (!w) return;
  for (auto e : w->ev)
    if (e) (void)hipEventDestroy(e);
  if (w->ev_join) (void)hipEventDestroy(w->ev_join);
  if (w->s2) (void)hipStreamDestroy(w->s2);
  free_batch_plan(w->chan_dec);
  free_batch_plan(w->chan_rec);
  free_plan(w->fftM);
  for (auto& L : w->lv) {
    free_plan(L.fftN);
    free_plan(L.fftW);
  }
  if (w->dtab) (void)hipFree(w->dtab);
  delete w;
}

void dirichlet_mask(const WavePlan* w, int level, float* out) {
  const WaveLevel& L = w->lv[level];
  const Mat& M = L.Ml;
  const Mat& N = L.Nl;
  const int d = M.d;
  i64 DM = det(M), DN = det(N);
  i64 m = DM < 0 ? -DM : DM, n = DN < 0 ? -DN : DN;
  i64 sM = DM < 0 ? -1 : 1, sN = DN < 0 ? -1 : 1;
  Mat adjM = adjugate(M), adjN = adjugate(N);
  Mat HMt, U;
  hnf(transpose(M), HMt, U);
  std::vector<i64> h(d);
  for (i64 idx = 0; idx < m; ++idx) {
    i64 r = idx;
    for (int i = d - 1; i >= 0; --i) {
      h[i] = r % HMt.a[i][i];
      r /= HMt.a[i][i];
    }
    // t = M^{-T} h * m  reduced into [-m/2, m/2)
    i64 t[kMaxD], hs[kMaxD], wv[kMaxD];
    int rM = 0;
    for (int j = 0; j < d; ++j) {
      i128 acc = 0;
      for (int k = 0; k < d; ++k) acc += (i128)adjM.a[k][j] * h[k];
      acc *= sM;
      i128 x = acc % m;
      if (x < 0) x += m;
      i64 tv = (i64)x;
      if (tv >= m - m / 2) tv -= m;  // [-floor(m/2), m - floor(m/2))
      t[j] = tv;
      if (2 * (i128)tv == -(i128)m) ++rM;
    }
    // h* = M^T t / m
    for (int i = 0; i < d; ++i) {
      i128 acc = 0;
      for (int j = 0; j < d; ++j) acc += (i128)M.a[j][i] * t[j];
      hs[i] = narrow(acc / m);
    }
    // w = N^{-T} h* * n = sgn(det N) adj(N)^T h*
    bool inside = true;
    int rN = 0;
    for (int j = 0; j < d; ++j) {
      i128 acc = 0;
      for (int k = 0; k < d; ++k) acc += (i128)adjN.a[k][j] * hs[k];
      acc *= sN;
      wv[j] = narrow(acc);
      i128 tw2 = 2 * (i128)(wv[j] < 0 ? -wv[j] : wv[j]);
      if (tw2 > n) inside = false;
      if (tw2 == n) ++rN;
    }
    // sqrt(q) 2^{(rM - rN)/2}, q = m / n (the quotient of the Dirichlet
    // kernels' coefficients); 2^{(1 + rM - rN)/2} for q = 2
    double val = 0.0;
    if (inside) {
      const i64 q = m / n;
      const int e = rM - rN;
      const double p2 = (e % 2 == 0) ? std::ldexp(1.0, e / 2) : std::ldexp(std::sqrt(2.0), (e - 1) / 2);
      val = q == 2 ? ((e + 1) % 2 == 0 ? std::ldexp(1.0, (e + 1) / 2)
                                       : std::ldexp(std::sqrt(2.0), e / 2))
                   : std::sqrt((double)q) * p2;
    }
    out[idx] = (float)val;
  }
}

void fiber_map(const WavePlan* w, int level, int path, i64 k0, i64 count, i64* lifts,
               i64* phase) {
  if (level < 0 || level >= w->levels || path < 0 || path > 2 || k0 < 0 || count < 0)
    throw StatusError{E_ARG};
  const WaveLevel& L = w->lv[level];
  const i64 q = w->q;
  if (k0 + count > L.ml / q) throw StatusError{E_ARG};
  if (q > 2) {
    if (phase) throw StatusError{E_UNSUPPORTED};
    const bool narrow = path == 0 ? L.sq.narrow != 0 : path == 1;
    if (narrow && !L.sq.narrow) throw StatusError{E_UNSUPPORTED};
    long long idx[kMaxQ];
    for (i64 c = 0; c < count; ++c) {
      fib::fiber_q_index<0>(L.sq, k0 + c, idx, narrow);
      if (lifts)
        for (i64 l = 0; l < q; ++l) lifts[c * q + l] = idx[l];
    }
    return;
  }
  const SplitDesc& sd = L.sd;
  const bool narrow = path == 0 ? sd.narrow != 0 : path == 1;
  if (narrow && !sd.narrow) throw StatusError{E_UNSUPPORTED};
  // phi(h0) = exp(-2 pi i rho / E) = exp(-2 pi i (rho m_l / E) / m_l)
  const i64 scale = L.ml / sd.E;
  for (i64 c = 0; c < count; ++c) {
    const fib::FiberIdx f = narrow ? fib::fiber_index32(sd, k0 + c) : fib::fiber_index64(sd, k0 + c);
    if (lifts) {
      lifts[2 * c] = f.i0;
      lifts[2 * c + 1] = f.i1;
    }
    if (phase) phase[c] = f.rho * scale;
  }
}

void level_scaling(const WavePlan* w, int level, int& d_M, int& d_N, i64* key, i64* grid) {
  const WaveLevel& L = w->lv[level];
  const LatticePlan* pM = level == 0 ? w->fftM : w->lv[level - 1].fftN;
  const Smith& S = pM->Sf;
  const int d = w->d;
  d_M = 0;
  d_N = 0;
  for (int i = 0; i < d; ++i) {
    d_M += S.eps[i] > 1;
    d_N += L.fftN->Sf.eps[i] > 1;
  }
  // first key g of G(J) (natural order of the Hermite box of J) whose class
  // has order q: J^{-1} g = adj(J) g / det J, so the order is the least
  // common multiple of q / gcd(q, (adj(J) g)_i)
  const i64 DJ = det(w->J);
  const i64 q = DJ < 0 ? -DJ : DJ;
  const Mat adj = adjugate(w->J);
  Mat HJ, UJ;
  hnf(w->J, HJ, UJ);
  auto gcd = [](i64 a, i64 b) {
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) {
      const i64 t = a % b;
      a = b;
      b = t;
    }
    return a;
  };
  Vec4 g = zero4();
  bool found = false;
  for (i64 idx = 0; idx < q && !found; ++idx) {
    i64 r = idx;
    for (int i = d - 1; i >= 0; --i) {
      g[i] = r % HJ.a[i][i];
      r /= HJ.a[i][i];
    }
    i64 order = 1;
    for (int i = 0; i < d; ++i) {
      i64 c = 0;
      for (int j = 0; j < d; ++j) c = cadd(c, cmul(adj.a[i][j], g[j]));
      const i64 oi = q / gcd(q, c);
      order = order / gcd(order, oi) * oi;
    }
    found = order == q;
  }
  if (!found) throw StatusError{E_UNSUPPORTED};
  const Vec4 k = reduce4(pM->HM, g);
  for (int i = 0; i < d; ++i) {
    key[i] = k[i];
    i128 acc = 0;
    for (int j = 0; j < d; ++j) acc += (i128)S.Qinv.a[i][j] * k[j];
    const i64 e = S.eps[i];
    i64 x = (i64)(acc % e);
    if (x < 0) x += e;
    grid[i] = x;
  }
}

}  // namespace lfft
