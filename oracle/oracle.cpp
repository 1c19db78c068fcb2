// FP64 CPU oracle for the anisotropic 3PCF multipoles.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file; only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark do.  It shares no code, table or constant with the HIP
// library: no cell list, no monomials, no conversion table.
//
// What it computes (paper, Sec. 3.1 "O(N^2) algorithm for the anisotropic
// 3PCF", the expansion zeta(r1,r2) = sum_{l l' m} zeta^m_{l l'} Y_lm Y*_l'm and
// Algorithm 1):
//
//   a^{(i)}_{lm}(b) = sum_{j != i, 0 < r_ij < R_max, bin(r_ij) = b} w_j conj(Y_lm(u_ij))
//   zeta^m_{l l'}(b1, b2) = sum_{i primary} w_i a^{(i)}_{lm}(b1) conj(a^{(i)}_{l'm}(b2))
//
// with u_ij the unit separation vector rotated into the line-of-sight frame of
// the primary.  Readings of points the paper leaves open (all listed in the
// design notes):
//   * a_lm projects onto conj(Y_lm), which is what the expansion above needs
//     (the text's plain sum of Y_lm would give conj(zeta));
//   * orthonormal Y_lm with the Condon-Shortley phase;
//   * weights: w_j inside a_lm, w_i on the primary (unit weights = the paper);
//   * self pairs (r = 0) excluded; degenerate triangles j = k included;
//   * equal-width shells [b dr, (b+1) dr), dr = R_max / nbins, r < R_max;
//   * periodic boxes use the minimum image and need R_max <= L/2;
//   * raw weighted sums, no normalisation or edge correction.
//
// Build: g++ -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <complex>
#include <omp.h>

namespace {

using cd = std::complex<double>;

constexpr double kPi = 3.14159265358979323846;

// Index of (l, m), 0 <= m <= l, in a triangular array.
inline int lm_index(int l, int m) { return l * (l + 1) / 2 + m; }

// Orthonormal spherical harmonics Y_lm(theta, phi) for 0 <= m <= l <= lmax,
// Condon-Shortley phase, from the stable recurrence for the normalised
// associated Legendre functions of Press, Teukolsky, Vetterling & Flannery,
// Numerical Recipes 3rd ed., Sec. 6.7 (eqs. 6.7.9-6.7.10):
//   Pt_mm     = (-1)^m sqrt((2m+1)/(4 pi) * prod_{i=1..m} (2i-1)/(2i)) (1-x^2)^{m/2}
//   Pt_{m+1,m} = x sqrt(2m+3) Pt_mm
//   Pt_lm     = sqrt((4l^2-1)/(l^2-m^2)) [x Pt_{l-1,m}
//                 - sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)) Pt_{l-2,m}]
// and Y_lm = Pt_lm(cos theta) e^{i m phi}.  The direction is given as a unit
// vector u: cos theta = u_z, sin theta = sqrt(u_x^2 + u_y^2) (so that
// (1-x^2)^{1/2} keeps full relative accuracy near the poles), and
// phi = atan2(u_y, u_x) (phi = 0 on the z axis, where every m != 0 term
// vanishes anyway).
void ylm(double ux, double uy, double uz, int lmax, cd* out) {
  const double x = uz;
  const double s = std::sqrt(ux * ux + uy * uy);
  const double phi = (s > 0.0) ? std::atan2(uy, ux) : 0.0;
  for (int m = 0; m <= lmax; ++m) {
    double prod = 1.0;
    for (int i = 1; i <= m; ++i) prod *= (2.0 * i - 1.0) / (2.0 * i);
    double pmm = std::sqrt((2.0 * m + 1.0) / (4.0 * kPi) * prod);
    if (m & 1) pmm = -pmm;
    pmm *= std::pow(s, m);
    const cd e = std::polar(1.0, m * phi);
    out[lm_index(m, m)] = pmm * e;
    if (m == lmax) continue;
    double pm1 = x * std::sqrt(2.0 * m + 3.0) * pmm;
    out[lm_index(m + 1, m)] = pm1 * e;
    double p2 = pmm, p1 = pm1;
    for (int l = m + 2; l <= lmax; ++l) {
      const double l2 = double(l) * l, m2 = double(m) * m;
      const double a = std::sqrt((4.0 * l2 - 1.0) / (l2 - m2));
      const double lp = l - 1.0;
      const double b = std::sqrt((lp * lp - m2) / (4.0 * lp * lp - 1.0));
      const double pl = a * (x * p1 - b * p2);
      out[lm_index(l, m)] = pl * e;
      p2 = p1;
      p1 = pl;
    }
  }
}

struct Problem {
  int64_t n;
  const double* pos;     // [n][3]
  const double* w;       // [n]
  double L[3];
  double lo[3];
  int periodic;
  double obs[3];
  double rmax;
  int nbins, lmax, los;  // los: 0 = box z axis, 1 = towards the observer
  const uint8_t* mask;   // [n] or null
};

// Positions are wrapped into [lo, lo + L) when the box is periodic.
double wrap(double x, double lo, double L) {
  double t = std::fmod(x - lo, L);
  if (t < 0.0) t += L;
  if (t >= L) t = 0.0;
  return lo + t;
}

// Rotation taking the unit line of sight n to the z axis: R = R_y(-theta) R_z(-phi)
// where (theta, phi) are the polar and azimuthal angles of n (Fig. 2: the
// primary is rotated onto the z axis of its line of sight).
void los_rotation(const double n[3], double R[3][3]) {
  const double theta = std::acos(std::fmax(-1.0, std::fmin(1.0, n[2])));
  const double phi = std::atan2(n[1], n[0]);
  const double ct = std::cos(theta), st = std::sin(theta);
  const double cp = std::cos(phi), sp = std::sin(phi);
  // R_z(-phi)
  const double Rz[3][3] = {{cp, sp, 0.0}, {-sp, cp, 0.0}, {0.0, 0.0, 1.0}};
  // R_y(-theta)
  const double Ry[3][3] = {{ct, 0.0, -st}, {0.0, 1.0, 0.0}, {st, 0.0, ct}};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += Ry[r][k] * Rz[k][c];
      R[r][c] = acc;
    }
}

struct Ctx {
  const Problem& p;
  std::vector<double> X;  // wrapped positions [n][3]
  int nlm;
  explicit Ctx(const Problem& pp) : p(pp) {
    X.resize(size_t(p.n) * 3);
    for (int64_t i = 0; i < p.n; ++i)
      for (int c = 0; c < 3; ++c) {
        const double v = p.pos[3 * i + c];
        X[3 * i + c] = p.periodic ? wrap(v, p.lo[c], p.L[c]) : v;
      }
    nlm = (p.lmax + 1) * (p.lmax + 2) / 2;
  }

  // Frame rotation of primary i: identity in z mode, and also where the line
  // of sight is undefined: a primary exactly on the observer, or one with a
  // non-finite coordinate (which has no neighbours anyway).  The paper is
  // silent on both; the box frame is the reading taken.
  void frame(int64_t i, double R[3][3]) const {
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) R[r][c] = (r == c) ? 1.0 : 0.0;
    if (p.los == 0) return;
    double d[3], nn = 0.0;
    for (int c = 0; c < 3; ++c) {
      d[c] = X[3 * i + c] - p.obs[c];
      nn += d[c] * d[c];
    }
    nn = std::sqrt(nn);
    if (!(nn > 0.0) || !std::isfinite(nn)) return;
    for (int c = 0; c < 3; ++c) d[c] /= nn;
    los_rotation(d, R);
  }

  // Visit every accepted secondary j of primary i: f(j, bin, u[3]).
  template <class F>
  void neighbours(int64_t i, const double R[3][3], F&& f) const {
    const double r2max = p.rmax * p.rmax;
    for (int64_t j = 0; j < p.n; ++j) {
      if (j == i) continue;
      double d[3];
      for (int c = 0; c < 3; ++c) {
        double v = X[3 * j + c] - X[3 * i + c];
        if (p.periodic) v -= p.L[c] * std::nearbyint(v / p.L[c]);
        d[c] = v;
      }
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (!(r2 > 0.0) || !(r2 < r2max)) continue;
      const double r = std::sqrt(r2);
      int b = int(std::floor(r * double(p.nbins) / p.rmax));
      if (b > p.nbins - 1) b = p.nbins - 1;
      double u[3];
      for (int c = 0; c < 3; ++c)
        u[c] = (R[c][0] * d[0] + R[c][1] * d[1] + R[c][2] * d[2]) / r;
      f(j, b, u);
    }
  }

  // a[b][lm] for primary i; returns the number of accepted pairs.
  int64_t alm(int64_t i, const double R[3][3], std::vector<cd>& a, std::vector<cd>& y) const {
    std::fill(a.begin(), a.end(), cd(0.0, 0.0));
    int64_t np = 0;
    neighbours(i, R, [&](int64_t j, int b, const double* u) {
      ylm(u[0], u[1], u[2], p.lmax, y.data());
      cd* ab = a.data() + size_t(b) * nlm;
      for (int k = 0; k < nlm; ++k) ab[k] += p.w[j] * std::conj(y[k]);
      ++np;
    });
    return np;
  }

  bool is_primary(int64_t i) const { return p.mask == nullptr || p.mask[i] != 0; }
};

inline size_t zidx(int lmax, int nb, int m, int l, int lp, int b1, int b2) {
  const size_t L1 = size_t(lmax) + 1;
  return ((((size_t(m) * L1 + l) * L1 + lp) * nb + b1) * nb + b2) * 2;
}

int check(const Problem& p) {
  if (p.n < 0 || p.nbins < 1 || p.lmax < 0 || p.lmax > 20 || !(p.rmax > 0.0)) return -1;
  if (p.periodic)
    for (int c = 0; c < 3; ++c)
      if (!(p.L[c] > 0.0) || p.rmax > 0.5 * p.L[c]) return -1;
  return 0;
}

}  // namespace

extern "C" {

// Y_lm(u) for 0 <= m <= l <= lmax as (re, im) pairs in triangular (l, m) order.
void oracle_ylm(double ux, double uy, double uz, int lmax, double* out) {
  std::vector<cd> y((lmax + 1) * (lmax + 2) / 2);
  ylm(ux, uy, uz, lmax, y.data());
  for (size_t k = 0; k < y.size(); ++k) {
    out[2 * k] = y[k].real();
    out[2 * k + 1] = y[k].imag();
  }
}

// zeta: dense [m][l][l'][b1][b2][re,im], zero where l < m or l' < m.
// distinct = 1 leaves out the degenerate triangles j = k (the same secondary on
// both sides, so b1 = b2): their terms w_i w_j^2 conj(Y_lm(u_ij)) Y_l'm(u_ij)
// are subtracted from the product of the a_lm (Sec. 3.1 writes zeta as that
// product, which contains them).
// Returns 0, or -1 on invalid arguments.
int oracle_zeta(int64_t n, const double* pos, const double* w, const double* L,
                const double* lo, int periodic, const double* obs, double rmax, int nbins,
                int lmax, int los, const uint8_t* mask, double* zeta, int64_t* pairs_out,
                int nthreads, int distinct) {
  Problem p{n, pos, w, {L[0], L[1], L[2]}, {lo[0], lo[1], lo[2]}, periodic,
            {obs[0], obs[1], obs[2]}, rmax, nbins, lmax, los, mask};
  if (check(p)) return -1;
  Ctx ctx(p);
  const size_t zlen = size_t(lmax + 1) * (lmax + 1) * (lmax + 1) * nbins * nbins * 2;
  if (nthreads < 1) nthreads = 1;
  std::vector<std::vector<double>> part(nthreads, std::vector<double>(zlen, 0.0));
  std::vector<int64_t> npart(nthreads, 0);
  // Static contiguous split: deterministic for a given thread count.
#pragma omp parallel num_threads(nthreads)
  {
    const int t = omp_get_thread_num();
    const int T = omp_get_num_threads();
    std::vector<cd> a(size_t(nbins) * ctx.nlm), y(ctx.nlm);
    double* z = part[t].data();
    const int64_t i0 = n * t / T, i1 = n * (t + 1) / T;
    for (int64_t i = i0; i < i1; ++i) {
      if (!ctx.is_primary(i)) continue;
      double R[3][3];
      ctx.frame(i, R);
      npart[t] += ctx.alm(i, R, a, y);
      const double wi = w[i];
      for (int m = 0; m <= lmax; ++m)
        for (int l = m; l <= lmax; ++l)
          for (int lp = m; lp <= lmax; ++lp)
            for (int b1 = 0; b1 < nbins; ++b1)
              for (int b2 = 0; b2 < nbins; ++b2) {
                const cd v = wi * a[size_t(b1) * ctx.nlm + lm_index(l, m)] *
                             std::conj(a[size_t(b2) * ctx.nlm + lm_index(lp, m)]);
                double* o = z + zidx(lmax, nbins, m, l, lp, b1, b2);
                o[0] += v.real();
                o[1] += v.imag();
              }
      if (distinct) {
        // the j = k terms, one secondary at a time
        ctx.neighbours(i, R, [&](int64_t j, int b, const double* u) {
          ylm(u[0], u[1], u[2], lmax, y.data());
          const double f = wi * w[j] * w[j];
          for (int m = 0; m <= lmax; ++m)
            for (int l = m; l <= lmax; ++l)
              for (int lp = m; lp <= lmax; ++lp) {
                const cd v = f * std::conj(y[lm_index(l, m)]) * y[lm_index(lp, m)];
                double* o = z + zidx(lmax, nbins, m, l, lp, b, b);
                o[0] -= v.real();
                o[1] -= v.imag();
              }
        });
      }
    }
  }
  std::memset(zeta, 0, zlen * sizeof(double));
  int64_t np = 0;
  for (int t = 0; t < nthreads; ++t) {
    for (size_t k = 0; k < zlen; ++k) zeta[k] += part[t][k];
    np += npart[t];
  }
  if (pairs_out) *pairs_out = np;
  return 0;
}

// Gradient of L = sum over the real view of c * zeta with respect to every
// weight w_k (c laid out like zeta).  With G = c_re + i c_im, L = Re sum conj(G) zeta:
//   primary term   dL/dw_i += Re sum conj(G^m_{ll'}(b1,b2)) a_lm(b1) conj(a_l'm(b2))
//   secondary term for each accepted pair (i, k), bin beta, Y = Y(u_ik):
//     dL/dw_k += w_i Re[ sum_lm conj(Y_lm) U_lm(beta) + sum_l'm Y_l'm V_l'm(beta) ]
//   U_lm(beta)  = sum_{l', b2} conj(G^m_{ll'}(beta, b2)) conj(a_l'm(b2))
//   V_l'm(beta) = sum_{l, b1}  conj(G^m_{ll'}(b1, beta)) a_lm(b1)
// (zeta is linear in w_i as a primary and quadratic in w_k as a secondary.)
int oracle_grad(int64_t n, const double* pos, const double* w, const double* L,
                const double* lo, int periodic, const double* obs, double rmax, int nbins,
                int lmax, int los, const uint8_t* mask, const double* c, double* grad,
                int nthreads) {
  Problem p{n, pos, w, {L[0], L[1], L[2]}, {lo[0], lo[1], lo[2]}, periodic,
            {obs[0], obs[1], obs[2]}, rmax, nbins, lmax, los, mask};
  if (check(p)) return -1;
  Ctx ctx(p);
  if (nthreads < 1) nthreads = 1;
  const int nlm = ctx.nlm;
  std::vector<std::vector<double>> part(nthreads, std::vector<double>(size_t(n), 0.0));
  auto G = [&](int m, int l, int lp, int b1, int b2) {
    const double* q = c + zidx(lmax, nbins, m, l, lp, b1, b2);
    return cd(q[0], q[1]);
  };
#pragma omp parallel num_threads(nthreads)
  {
    const int t = omp_get_thread_num();
    const int T = omp_get_num_threads();
    std::vector<cd> a(size_t(nbins) * nlm), y(nlm), U(size_t(nbins) * nlm),
        V(size_t(nbins) * nlm);
    double* g = part[t].data();
    const int64_t i0 = n * t / T, i1 = n * (t + 1) / T;
    for (int64_t i = i0; i < i1; ++i) {
      if (!ctx.is_primary(i)) continue;
      double R[3][3];
      ctx.frame(i, R);
      ctx.alm(i, R, a, y);
      auto A = [&](int b, int l, int m) { return a[size_t(b) * nlm + lm_index(l, m)]; };
      // primary term
      double prim = 0.0;
      for (int m = 0; m <= lmax; ++m)
        for (int l = m; l <= lmax; ++l)
          for (int lp = m; lp <= lmax; ++lp)
            for (int b1 = 0; b1 < nbins; ++b1)
              for (int b2 = 0; b2 < nbins; ++b2)
                prim += (std::conj(G(m, l, lp, b1, b2)) * A(b1, l, m) *
                         std::conj(A(b2, lp, m))).real();
      g[i] += prim;
      // U and V
      for (int beta = 0; beta < nbins; ++beta)
        for (int m = 0; m <= lmax; ++m)
          for (int l = m; l <= lmax; ++l) {
            cd u(0.0, 0.0), v(0.0, 0.0);
            for (int lp = m; lp <= lmax; ++lp)
              for (int bb = 0; bb < nbins; ++bb) {
                u += std::conj(G(m, l, lp, beta, bb)) * std::conj(A(bb, lp, m));
                v += std::conj(G(m, lp, l, bb, beta)) * A(bb, lp, m);
              }
            U[size_t(beta) * nlm + lm_index(l, m)] = u;
            V[size_t(beta) * nlm + lm_index(l, m)] = v;
          }
      // secondary terms
      const double wi = w[i];
      ctx.neighbours(i, R, [&](int64_t k, int beta, const double* u) {
        ylm(u[0], u[1], u[2], lmax, y.data());
        double s = 0.0;
        for (int m = 0; m <= lmax; ++m)
          for (int l = m; l <= lmax; ++l) {
            const int q = lm_index(l, m);
            s += (std::conj(y[q]) * U[size_t(beta) * nlm + q]).real();
            s += (y[q] * V[size_t(beta) * nlm + q]).real();
          }
        g[k] += wi * s;
      });
    }
  }
  std::memset(grad, 0, size_t(n) * sizeof(double));
  for (int t = 0; t < nthreads; ++t)
    for (int64_t k = 0; k < n; ++k) grad[k] += part[t][k];
  return 0;
}

}  // extern "C"
