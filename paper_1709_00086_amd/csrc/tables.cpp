// Monomial-sum -> a_lm conversion coefficients (host code).
//
// On the unit sphere every Y_lm is a polynomial in the direction cosines, so
// a_lm = sum_j w_j conj(Y_lm(u_j)) is a fixed linear combination of monomial
// sums (paper, Sec. 3.1: the coefficients are weighted sums of the power
// combinations of eq. 1).  With the Condon-Shortley phase,
//
//   conj(Y_lm(u)) = N_lm (-1)^m (u_x - i u_y)^m  d^m P_l / dz^m (u_z),
//   N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!),
//   d^m P_l/dz^m (z) = 2^-l sum_k (-1)^k C(l,k) C(2l-2k,l) (l-2k)!/(l-2k-m)! z^{l-2k-m}
//
// (explicit form of P_l from Rodrigues' formula, differentiated m times).
//
// Spin basis: the sums S_{m,n} = sum w (u_x - i u_y)^m u_z^n give
//   a_lm = N_lm (-1)^m sum_k c_lmk S_{m, l-m-2k}   (real c_lmk).
// Cartesian basis (the paper's monomials): every term above is made
// homogeneous of degree l with (u_x^2 + u_y^2 + u_z^2)^k = 1 and expanded with
// the binomial and trinomial theorems, so only degree-l monomials
// u_x^K u_y^P u_z^Q (K + P + Q = l) appear.
//
// Integer parts are accumulated exactly in int64, then scaled in double.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "internal.h"

namespace g3 {

namespace {

int64_t binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

int64_t falling(int n, int k) {  // n! / (n-k)!
  int64_t r = 1;
  for (int i = 0; i < k; ++i) r *= (n - i);
  return r;
}

int64_t fact(int n) { return falling(n, n); }

double norm_lm(int l, int m) {
  double ratio = 1.0;  // (l-m)!/(l+m)!
  for (int i = l - m + 1; i <= l + m; ++i) ratio /= double(i);
  return std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * ratio);
}

// 2^l * c_lmk (an integer), c_lmk as defined above.
int64_t c_int(int l, int m, int k) {
  int64_t v = binom(l, k) * binom(2 * l - 2 * k, l) * falling(l - 2 * k, m);
  return (k & 1) ? -v : v;
}

}  // namespace

// Canonical term index of the cartesian monomial u_x^k u_y^p u_z^q
// (q outermost, then p, then k), matching the pair kernels.
int cart_index(int k, int p, int q) {
  int t = 0;
  for (int qq = 0; qq < q; ++qq) {
    const int n = kDeg - qq;
    t += (n + 1) * (n + 2) / 2;
  }
  for (int pp = 0; pp < p; ++pp) t += kDeg - q - pp + 1;
  return t + k;
}

// Canonical term index of Re/Im S_{m,n} in the spin basis.
int spin_index(int m, int n, int part) {
  if (m == 0) return n;
  int base = kDeg + 1;
  for (int mm = 1; mm < m; ++mm) base += 2 * (kDeg + 1 - mm);
  return base + 2 * n + part;
}

void build_conv_table(int basis, ConvTable* t) {
  std::memset(t, 0, sizeof(*t));
  int o = 0, nnz = 0;
  for (int m = 0; m <= kDeg; ++m) {
    for (int part = 0; part < (m == 0 ? 1 : 2); ++part) {
      for (int l = m; l <= kDeg; ++l) {
        t->out_m[o] = short(m);
        t->out_l[o] = short(l);
        t->out_part[o] = short(part);
        t->rowptr[o] = nnz;
        const double scale = norm_lm(l, m) * ((m & 1) ? -1.0 : 1.0) / std::ldexp(1.0, l);
        if (basis == G3PCF_BASIS_SPIN) {
          for (int k = 0; 2 * k <= l - m; ++k) {
            t->term[nnz] = short(spin_index(m, l - m - 2 * k, part));
            t->coef[nnz] = scale * double(c_int(l, m, k));
            ++nnz;
          }
        } else if (basis == G3PCF_BASIS_SPIN_T) {
          // u_z^n = 2^(1-n) sum_j binom(n, j) T_{n-2j}(u_z), the T_0 term halved
          std::map<int, double> acc;
          for (int k = 0; 2 * k <= l - m; ++k) {
            const int n = l - m - 2 * k;
            const double c = scale * double(c_int(l, m, k));
            for (int j = 0; 2 * j <= n; ++j) {
              const double a = std::ldexp(double(binom(n, j)), (2 * j == n) ? -n : 1 - n);
              acc[n - 2 * j] += c * a;
            }
          }
          for (auto& kv : acc) {
            t->term[nnz] = short(spin_index(m, kv.first, part));
            t->coef[nnz] = kv.second;
            ++nnz;
          }
        } else {
          // exact integer coefficients of u_x^K u_y^P u_z^Q for this (l, m, part)
          std::map<std::tuple<int, int, int>, int64_t> acc;
          for (int k = 0; 2 * k <= l - m; ++k) {
            const int64_t ck = c_int(l, m, k);
            for (int a = 0; a <= m; ++a) {
              // (-i)^a: a%4 = 0 -> +1 (real), 1 -> -i, 2 -> -1 (real), 3 -> +i
              const int am = a & 3;
              const bool is_real = (am == 0 || am == 2);
              if ((part == 0) != is_real) continue;
              const int sgn = (am == 0 || am == 3) ? 1 : -1;
              const int64_t cma = binom(m, a);
              for (int k1 = 0; k1 <= k; ++k1)
                for (int k2 = 0; k1 + k2 <= k; ++k2) {
                  const int k3 = k - k1 - k2;
                  const int64_t multi = fact(k) / (fact(k1) * fact(k2) * fact(k3));
                  const int K = m - a + 2 * k1, P = a + 2 * k2, Q = l - m - 2 * k + 2 * k3;
                  acc[std::make_tuple(K, P, Q)] += sgn * ck * cma * multi;
                }
            }
          }
          for (auto& kv : acc) {
            if (kv.second == 0) continue;
            int K, P, Q;
            std::tie(K, P, Q) = kv.first;
            t->term[nnz] = short(cart_index(K, P, Q));
            t->coef[nnz] = scale * double(kv.second);
            ++nnz;
          }
        }
        ++o;
      }
    }
  }
  t->rowptr[o] = nnz;
  t->nout = o;
  t->nnz = nnz;
  // transpose: entries grouped by term
  const int nterm = (basis == G3PCF_BASIS_CARTESIAN) ? kTermsCart : kTermsSpin;
  std::vector<int> cnt(nterm + 1, 0);
  for (int e = 0; e < nnz; ++e) cnt[t->term[e] + 1]++;
  for (int k = 0; k < nterm; ++k) cnt[k + 1] += cnt[k];
  for (int k = 0; k <= nterm; ++k) t->trowptr[k] = cnt[k];
  for (int k = nterm + 1; k <= kTermsCart; ++k) t->trowptr[k] = cnt[nterm];
  std::vector<int> fillp(cnt.begin(), cnt.end() - 1);
  for (int oo = 0; oo < o; ++oo)
    for (int e = t->rowptr[oo]; e < t->rowptr[oo + 1]; ++e) {
      const int at = fillp[t->term[e]]++;
      t->tout[at] = short(oo);
      t->tcoef[at] = t->coef[e];
    }
}

// Degenerate-triangle table.  For one secondary at unit separation u the j = k
// term of zeta^m_{ll'} is w_i w_j^2 conj(Y_lm(u)) Y_l'm(u) = w_i w_j^2
// Pbar_lm(u_z) Pbar_l'm(u_z) (the azimuthal factors cancel, Pbar_lm = N_lm P_l^m,
// the Condon-Shortley signs square to one): a polynomial of degree l + l' in
// u_z alone, expanded here in Legendre polynomials,
//   Pbar_lm(z) Pbar_l'm(z) = sum_n G[m][l][l'][n] P_n(z),
//   G = (2n + 1) / 2 int_{-1}^{1} Pbar_lm Pbar_l'm P_n dz,
// by Gauss-Legendre quadrature with 32 nodes (exact to degree 63 >= 40).
namespace {

// P_l^m(z) (Condon-Shortley phase) for m <= l <= kDeg: p[l] for fixed m.
void assoc_legendre(int m, double z, double* p) {
  const double s = std::sqrt(std::fmax(0.0, 1.0 - z * z));
  double pmm = 1.0;
  for (int k = 1; k <= m; ++k) pmm *= -(2.0 * k - 1.0) * s;
  for (int l = 0; l <= kDeg; ++l) p[l] = 0.0;
  p[m] = pmm;
  if (m + 1 <= kDeg) p[m + 1] = z * (2.0 * m + 1.0) * pmm;
  for (int l = m + 2; l <= kDeg; ++l)
    p[l] = ((2.0 * l - 1.0) * z * p[l - 1] - (l + m - 1.0) * p[l - 2]) / double(l - m);
}

void legendre_all(double z, int nmax, double* p) {  // P_n(z), n <= nmax
  p[0] = 1.0;
  if (nmax >= 1) p[1] = z;
  for (int n = 1; n < nmax; ++n) p[n + 1] = ((2.0 * n + 1.0) * z * p[n] - n * p[n - 1]) / (n + 1.0);
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton iteration on P_K from
// the Chebyshev-like first guesses cos(pi (i + 3/4) / (K + 1/2)).
void gauss_legendre(int K, double* x, double* w) {
  std::vector<double> p(K + 1);
  for (int i = 0; i < K; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (K + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      legendre_all(z, K, p.data());
      dp = K * (z * p[K] - p[K - 1]) / (z * z - 1.0);  // P_K'(z)
      const double dz = p[K] / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    legendre_all(z, K, p.data());
    dp = K * (z * p[K] - p[K - 1]) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

}  // namespace

void build_deg_table(double* G) {
  constexpr int K = 32;
  double x[K], wq[K];
  gauss_legendre(K, x, wq);
  std::memset(G, 0, sizeof(double) * kDegTable);
  double pl[kDeg + 1], pn[kTermsDeg];
  for (int m = 0; m <= kDeg; ++m) {
    for (int q = 0; q < K; ++q) {
      assoc_legendre(m, x[q], pl);
      legendre_all(x[q], kTermsDeg - 1, pn);
      for (int l = m; l <= kDeg; ++l) {
        const double nl =
            std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * double(fact(l - m)) / double(fact(l + m)));
        for (int lp = m; lp <= kDeg; ++lp) {
          const double nlp = std::sqrt((2.0 * lp + 1.0) / (4.0 * M_PI) * double(fact(lp - m)) /
                                       double(fact(lp + m)));
          const double f = wq[q] * nl * pl[l] * nlp * pl[lp];
          for (int n = 0; n <= l + lp; ++n)
            G[deg_index(m, l, lp, n)] += 0.5 * (2.0 * n + 1.0) * f * pn[n];
        }
      }
    }
  }
}

}  // namespace g3

// Host-side evaluation of the library's conversion for one unit vector and
// unit weight: out[(l*(l+1)/2 + m)*2 + {0,1}] = conj(Y_lm(u)) via the monomial
// sums of `basis`.  Declared in g3pcf.h as a diagnostic.
extern "C" int g3pcf_conj_ylm_via_monomials(int basis, int lmax, double ux, double uy,
                                            double uz, double* out) {
  using namespace g3;
  if ((basis != G3PCF_BASIS_CARTESIAN && basis != G3PCF_BASIS_SPIN &&
       basis != G3PCF_BASIS_SPIN_T) ||
      lmax < 0 || lmax > kDeg || out == nullptr)
    return G3PCF_EINVAL;
  static thread_local ConvTable tab[kConvTables];
  static thread_local bool built[kConvTables] = {};
  if (!built[basis]) {
    build_conv_table(basis, &tab[basis]);
    built[basis] = true;
  }
  const ConvTable& t = tab[basis];
  std::vector<double> M(basis == G3PCF_BASIS_CARTESIAN ? kTermsCart : kTermsSpin, 0.0);
  if (basis != G3PCF_BASIS_CARTESIAN) {
    // u_z^n, or T_n(u_z) from T_{n+1} = 2 u_z T_n - T_{n-1}
    double zn[kDeg + 1];
    zn[0] = 1.0;
    zn[1] = uz;
    for (int n = 1; n < kDeg; ++n)
      zn[n + 1] = (basis == G3PCF_BASIS_SPIN_T) ? 2.0 * uz * zn[n] - zn[n - 1] : zn[n] * uz;
    double cr = 1.0, ci = 0.0;  // (ux - i uy)^m
    for (int m = 0; m <= kDeg; ++m) {
      for (int n = 0; m + n <= kDeg; ++n) {
        if (m == 0) {
          M[spin_index(0, n, 0)] = zn[n];
        } else {
          M[spin_index(m, n, 0)] = cr * zn[n];
          M[spin_index(m, n, 1)] = ci * zn[n];
        }
      }
      const double nr = cr * ux + ci * uy, ni = ci * ux - cr * uy;
      cr = nr;
      ci = ni;
    }
  } else {
    for (int q = 0; q <= kDeg; ++q)
      for (int p = 0; p + q <= kDeg; ++p)
        for (int k = 0; k + p + q <= kDeg; ++k)
          M[cart_index(k, p, q)] = std::pow(ux, k) * std::pow(uy, p) * std::pow(uz, q);
  }
  for (int l = 0; l <= lmax; ++l)
    for (int m = 0; m <= l; ++m) {
      out[2 * (l * (l + 1) / 2 + m)] = 0.0;
      out[2 * (l * (l + 1) / 2 + m) + 1] = 0.0;
    }
  for (int o = 0; o < t.nout; ++o) {
    const int l = t.out_l[o], m = t.out_m[o], part = t.out_part[o];
    if (l > lmax) continue;
    double s = 0.0;
    for (int e = t.rowptr[o]; e < t.rowptr[o + 1]; ++e) s += t.coef[e] * M[t.term[e]];
    out[2 * (l * (l + 1) / 2 + m) + part] = s;
  }
  return G3PCF_OK;
}
