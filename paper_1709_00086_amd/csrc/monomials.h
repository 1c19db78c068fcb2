// Device helpers of the pair kernels: wave-uniform broadcasts, DPP wave sums
// and the two monomial bases with their register-resident accumulators.
//
// Included by pairs.hip only (it opens an anonymous namespace).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "internal.h"

namespace g3 {
namespace {

// ---------------------------------------------------------------- utilities
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <typename Real>
struct V4;
template <>
struct V4<float> {
  using T = float4;
};
template <>
struct V4<double> {
  using T = double4;
};

// Copies of a wave-uniform value in scalar registers.  The value passes
// through an empty asm statement first: the compiler drops readfirstlane of a
// value it already knows to be uniform, and such values then stay in (and
// spill from) vector registers.
__device__ __forceinline__ int uniform_int(int v) {
  asm("" : "+v"(v));
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ float uniform_real(float v) {
  return __int_as_float(uniform_int(__float_as_int(v)));
}

__device__ __forceinline__ double uniform_double(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = uniform_int(int(b & 0xffffffffll));
  const int hi = uniform_int(int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              (static_cast<unsigned int>(lo)));
}
__device__ __forceinline__ double uniform_real(double v) { return uniform_double(v); }

// DPP move with compile-time controls (old value 0 where the row is masked).
// With bound_ctrl set and full masks the compiler folds the move into the add.
template <int CTRL, int ROW, int BANK>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW, BANK, true);
}

// Sum over the 64 lanes; the total is valid in lanes 48..63.
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_ror 4, row_ror 8 give every
// lane its row sum; row_bcast 15 and row_bcast 31 then fold rows 0-2 into 3.
__device__ __forceinline__ float wave_sum(float v) {
  v += __int_as_float(dpp_i<0xB1, 0xF, 0xF>(__float_as_int(v)));
  v += __int_as_float(dpp_i<0x4E, 0xF, 0xF>(__float_as_int(v)));
  v += __int_as_float(dpp_i<0x124, 0xF, 0xF>(__float_as_int(v)));
  v += __int_as_float(dpp_i<0x128, 0xF, 0xF>(__float_as_int(v)));
  v += __int_as_float(dpp_i<0x142, 0xA, 0xF>(__float_as_int(v)));
  v += __int_as_float(dpp_i<0x143, 0xC, 0xF>(__float_as_int(v)));
  return v;
}

template <int CTRL, int ROW, int BANK>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<CTRL, ROW, BANK>(int(b & 0xffffffffll));
  const int hi = dpp_i<CTRL, ROW, BANK>(int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              (static_cast<unsigned int>(lo)));
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xB1, 0xF, 0xF>(v);
  v += dpp_d<0x4E, 0xF, 0xF>(v);
  v += dpp_d<0x124, 0xF, 0xF>(v);
  v += dpp_d<0x128, 0xF, 0xF>(v);
  v += dpp_d<0x142, 0xA, 0xF>(v);
  v += dpp_d<0x143, 0xC, 0xF>(v);
  return v;
}

// Sum over the 16 lanes of each row (every lane gets its row's sum).
__device__ __forceinline__ float row_sum(float v) {
  v += __int_as_float(dpp_i<0xB1, 0xF, 0xF>(__float_as_int(v)));
  v += __int_as_float(dpp_i<0x4E, 0xF, 0xF>(__float_as_int(v)));
  v += __int_as_float(dpp_i<0x124, 0xF, 0xF>(__float_as_int(v)));
  v += __int_as_float(dpp_i<0x128, 0xF, 0xF>(__float_as_int(v)));
  return v;
}
__device__ __forceinline__ double row_sum(double v) {
  v += dpp_d<0xB1, 0xF, 0xF>(v);
  v += dpp_d<0x4E, 0xF, 0xF>(v);
  v += dpp_d<0x124, 0xF, 0xF>(v);
  v += dpp_d<0x128, 0xF, 0xF>(v);
  return v;
}

// Fold four values a, e, b, f across rows: lane i of row 0 of the result
// holds a summed over lanes i, i + 16, i + 32 and i + 48, row 1 the same for
// e, row 2 for b, row 3 for f, so a row sum of the result gives the four
// totals (and given row sums as inputs, the result holds the totals):
// permlane32_swap exchanges the upper half of its first operand with the
// lower half of its second, permlane16_swap the odd rows of its first with the
// even rows of its second.
__device__ __forceinline__ unsigned pl32(unsigned& x, unsigned y) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
  x = r[0];
  return r[1];
}
__device__ __forceinline__ unsigned pl16(unsigned& x, unsigned y) {
  const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
  x = r[0];
  return r[1];
}
__device__ __forceinline__ float fold4(float a, float e, float b, float f) {
  unsigned ua = __float_as_uint(a), ue = __float_as_uint(e);
  const unsigned ub = pl32(ua, __float_as_uint(b));
  const unsigned uf = pl32(ue, __float_as_uint(f));
  const float c = __uint_as_float(ua) + __uint_as_float(ub);
  const float d = __uint_as_float(ue) + __uint_as_float(uf);
  unsigned uc = __float_as_uint(c);
  const unsigned ud = pl16(uc, __float_as_uint(d));
  return __uint_as_float(uc) + __uint_as_float(ud);
}
__device__ __forceinline__ double swap32_d(double& x, double y) {
  const long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
  unsigned xl = unsigned(bx), xh = unsigned(bx >> 32);
  const unsigned yl = pl32(xl, unsigned(by)), yh = pl32(xh, unsigned(by >> 32));
  x = __longlong_as_double((static_cast<long long>(xh) << 32) | xl);
  return __longlong_as_double((static_cast<long long>(yh) << 32) | yl);
}
__device__ __forceinline__ double swap16_d(double& x, double y) {
  const long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
  unsigned xl = unsigned(bx), xh = unsigned(bx >> 32);
  const unsigned yl = pl16(xl, unsigned(by)), yh = pl16(xh, unsigned(by >> 32));
  x = __longlong_as_double((static_cast<long long>(xh) << 32) | xl);
  return __longlong_as_double((static_cast<long long>(yh) << 32) | yl);
}
__device__ __forceinline__ double fold4(double a, double e, double b, double f) {
  const double b2 = swap32_d(a, b);
  const double f2 = swap32_d(e, f);
  double c = a + b2;
  const double d = e + f2;
  const double d2 = swap16_d(c, d);
  return c + d2;
}

__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------- monomial bases
// Canonical cartesian index (q outermost, then p, then k); must match tables.cpp.
__host__ __device__ constexpr int cart_index_c(int k, int p, int q) {
  int t = 0;
  for (int qq = 0; qq < q; ++qq) t += (kDeg - qq + 1) * (kDeg - qq + 2) / 2;
  for (int pp = 0; pp < p; ++pp) t += kDeg - q - pp + 1;
  return t + k;
}
__host__ __device__ constexpr int spin_index_c(int m, int n, int part) {
  int base = (m == 0) ? 0 : kDeg + 1;
  for (int mm = 1; mm < m; ++mm) base += 2 * (kDeg + 1 - mm);
  return (m == 0) ? n : base + 2 * n + part;
}

__host__ __device__ constexpr int cart_count(unsigned qmask) {
  int c = 0;
  for (int q = 0; q <= kDeg; ++q)
    if ((qmask >> q) & 1u) c += (kDeg - q + 1) * (kDeg - q + 2) / 2;
  return c;
}
// local index of (k, p, q) inside a chunk holding the q's of qmask
__host__ __device__ constexpr int cart_local(unsigned qmask, int k, int p, int q) {
  int t = 0;
  for (int qq = 0; qq < q; ++qq)
    if ((qmask >> qq) & 1u) t += (kDeg - qq + 1) * (kDeg - qq + 2) / 2;
  for (int pp = 0; pp < p; ++pp) t += kDeg - q - pp + 1;
  return t + k;
}

// Global term index of the i-th accumulator of a cartesian chunk.
__host__ __device__ constexpr int cart_term_of(unsigned qmask, int i) {
  int t = 0;
  for (int q = 0; q <= kDeg; ++q) {
    if (!((qmask >> q) & 1u)) continue;
    for (int p = 0; p + q <= kDeg; ++p)
      for (int k = 0; k + p + q <= kDeg; ++k) {
        if (t == i) return cart_index_c(k, p, q);
        ++t;
      }
  }
  return -1;
}

// Cartesian chunk: the monomials u_x^k u_y^p u_z^q whose z power q is in QMASK.
// Per pair: P = w u_y^p u_z^q by running products, then acc += u_x^k * P
// (one FMA per monomial).
template <typename Real, unsigned QMASK>
struct CartChunk {
  static constexpr int NT = cart_count(QMASK);
  Real acc[NT];
  static __host__ __device__ constexpr int term_of(int i) { return cart_term_of(QMASK, i); }

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = Real(0);
  }

  __device__ __forceinline__ void add(Real x, Real y, Real z, Real w) {
    Real xp[kDeg + 1];
    xp[0] = Real(1);
#pragma unroll
    for (int k = 1; k <= kDeg; ++k) xp[k] = xp[k - 1] * x;
    Real wz = w;
    static_for<kDeg + 1>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      if constexpr (q > 0) wz = wz * z;
      if constexpr (((QMASK >> q) & 1u) != 0) {
        Real P = wz;
        static_for<kDeg + 1 - q>([&](auto pc) {
          constexpr int p = decltype(pc)::value;
          if constexpr (p > 0) P = P * y;
          static_for<kDeg + 1 - q - p>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            constexpr int t = cart_local(QMASK, k, p, q);
            if constexpr (k == 0)
              acc[t] += P;
            else
              acc[t] = fma_r(xp[k], P, acc[t]);
          });
        });
      }
    });
  }

  // adjoint: sum over this chunk's monomials of g_t * monomial.  Powers of x
  // and y are formed first so that every coefficient enters as a multiplicand
  // (a scalar-register operand when the coefficients are uniform).
  template <typename GetG>
  static __device__ __forceinline__ Real poly(Real x, Real y, Real z, GetG&& g) {
    Real xp[kDeg + 1], yp[kDeg + 1];
    xp[0] = Real(1);
    yp[0] = Real(1);
#pragma unroll
    for (int k = 1; k <= kDeg; ++k) {
      xp[k] = xp[k - 1] * x;
      yp[k] = yp[k - 1] * y;
    }
    Real total = Real(0);
    Real zq = Real(1);
    static_for<kDeg + 1>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      if constexpr (q > 0) zq = zq * z;
      if constexpr (((QMASK >> q) & 1u) != 0) {
        Real ysum = Real(0);
        static_for<kDeg + 1 - q>([&](auto pc) {
          constexpr int p = decltype(pc)::value;
          constexpr int KM = kDeg - q - p;  // highest power of x
          if constexpr (KM == 0) {
            ysum = fma_r(g(cart_index_c(0, p, q)), yp[p], ysum);
          } else {
            // start from a product and add the constant term last, so that no
            // coefficient has to be copied into a vector register first
            Real hx = g(cart_index_c(1, p, q)) * xp[1];
            static_for<KM - 1>([&](auto kc) {
              constexpr int k = decltype(kc)::value + 2;
              hx = fma_r(g(cart_index_c(k, p, q)), xp[k], hx);
            });
            hx = hx + g(cart_index_c(0, p, q));
            ysum = fma_r(hx, yp[p], ysum);
          }
        });
        total = fma_r(ysum, zq, total);
      }
    });
    return total;
  }

  template <typename Store>
  __device__ __forceinline__ void for_each_term(Store&& st) {
    static_for<kDeg + 1>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      if constexpr (((QMASK >> q) & 1u) != 0) {
        static_for<kDeg + 1 - q>([&](auto pc) {
          constexpr int p = decltype(pc)::value;
          static_for<kDeg + 1 - q - p>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            st(acc[cart_local(QMASK, k, p, q)], cart_index_c(k, p, q));
          });
        });
      }
    });
  }
};

__host__ __device__ constexpr int spin_count(int m0, int m1) {
  int c = 0;
  for (int m = m0; m <= m1; ++m) c += (m == 0) ? (kDeg + 1) : 2 * (kDeg + 1 - m);
  return c;
}
__host__ __device__ constexpr int spin_local(int m0, int m, int n, int part) {
  int t = 0;
  for (int mm = m0; mm < m; ++mm) t += (mm == 0) ? (kDeg + 1) : 2 * (kDeg + 1 - mm);
  return (m == 0) ? t + n : t + 2 * n + part;
}

// Global term index of the i-th accumulator of a spin chunk (m0..m1).
__host__ __device__ constexpr int spin_term_of(int m0, int m1, int i) {
  int t = 0;
  for (int m = m0; m <= m1; ++m)
    for (int n = 0; m + n <= kDeg; ++n)
      for (int part = 0; part < (m == 0 ? 1 : 2); ++part) {
        if (t == i) return spin_index_c(m, n, part);
        ++t;
      }
  return -1;
}

// Chebyshev polynomials T_0..T_NMAX of z by their three-term recurrence
// T_{n+1} = 2 z T_n - T_{n-1} (one FMA each).  In this basis the
// coefficients of the spherical harmonics do not cancel: those of the powers
// z^n do, by up to three orders of magnitude at l = 10 (for m = 0 they are
// the power-basis coefficients of the Legendre polynomials), which costs
// FP32 sums as many digits.
template <int NMAX, typename Real>
__device__ __forceinline__ void chebyshev(Real z, Real (&tn)[kDeg + 1]) {
  tn[0] = Real(1);
  tn[1] = z;
  const Real z2 = z + z;
  static_for<(NMAX > 1 ? NMAX - 1 : 0)>([&](auto nc) {
    constexpr int n = decltype(nc)::value + 1;
    tn[n + 1] = fma_r(z2, tn[n], -tn[n - 1]);
  });
}

// Spin chunk: S_{m,n} = sum w (u_x - i u_y)^m T_n(u_z) for M0 <= m <= M1,
// with T_n the Chebyshev polynomials (the conversion to a_lm uses the
// spin-Chebyshev table).
template <typename Real, int M0, int M1>
struct SpinChunk {
  static constexpr int NT = spin_count(M0, M1);
  Real acc[NT];
  static __host__ __device__ constexpr int term_of(int i) { return spin_term_of(M0, M1, i); }

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = Real(0);
  }

  __device__ __forceinline__ void add(Real x, Real y, Real z, Real w) {
    constexpr int NMAX = kDeg - (M0 > 0 ? M0 : 0);
    Real zn[kDeg + 1];
    chebyshev<NMAX>(z, zn);
    if constexpr (M0 == 0) {
      acc[spin_local(M0, 0, 0, 0)] += w;
      static_for<kDeg>([&](auto nc) {
        constexpr int n = decltype(nc)::value + 1;
        acc[spin_local(M0, 0, n, 0)] = fma_r(w, zn[n], acc[spin_local(M0, 0, n, 0)]);
      });
    }
    if constexpr (M1 >= 1) {
      Real cr = w * x, ci = -(w * y);  // w (x - i y)
      static_for<M1>([&](auto mc) {
        constexpr int m = decltype(mc)::value + 1;
        if constexpr (m > 1) {
          const Real nr = fma_r(cr, x, ci * y);
          const Real ni = fma_r(ci, x, -(cr * y));
          cr = nr;
          ci = ni;
        }
        if constexpr (m >= M0) {
          acc[spin_local(M0, m, 0, 0)] += cr;
          acc[spin_local(M0, m, 0, 1)] += ci;
          static_for<kDeg - m>([&](auto nc) {
            constexpr int n = decltype(nc)::value + 1;
            acc[spin_local(M0, m, n, 0)] = fma_r(cr, zn[n], acc[spin_local(M0, m, n, 0)]);
            acc[spin_local(M0, m, n, 1)] = fma_r(ci, zn[n], acc[spin_local(M0, m, n, 1)]);
          });
        }
      });
    }
  }

  // adjoint: sum over this chunk of g_t * Re/Im parts of (x - i y)^m T_n(z),
  // with the T_n formed first so that every coefficient enters as a
  // multiplicand (a scalar-register operand when the coefficients are uniform).
  template <typename GetG>
  static __device__ __forceinline__ Real poly(Real x, Real y, Real z, GetG&& g) {
    Real zn[kDeg + 1];
    chebyshev<kDeg>(z, zn);
    Real total = Real(0);
    Real cr = Real(1), ci = Real(0);
    static_for<M1 + 1>([&](auto mc) {
      constexpr int m = decltype(mc)::value;
      if constexpr (m > 0) {
        const Real nr = fma_r(cr, x, ci * y);
        const Real ni = fma_r(ci, x, -(cr * y));
        cr = nr;
        ci = ni;
      }
      if constexpr (m >= M0) {
        constexpr int NM = kDeg - m;  // highest power of z
        if constexpr (NM == 0) {
          // m = kDeg: only the constant coefficients
          if constexpr (m == 0)
            total += g(spin_index_c(m, 0, 0));
          else
            total = fma_r(cr, g(spin_index_c(m, 0, 0)), fma_r(ci, g(spin_index_c(m, 0, 1)), total));
        } else {
          // start from a product and add the constant term last, so that no
          // coefficient has to be copied into a vector register first
          Real hr = g(spin_index_c(m, 1, 0)) * zn[1];
          Real hi = Real(0);
          if constexpr (m > 0) hi = g(spin_index_c(m, 1, 1)) * zn[1];
          static_for<NM - 1>([&](auto nc) {
            constexpr int n = decltype(nc)::value + 2;
            hr = fma_r(g(spin_index_c(m, n, 0)), zn[n], hr);
            if constexpr (m > 0) hi = fma_r(g(spin_index_c(m, n, 1)), zn[n], hi);
          });
          hr = hr + g(spin_index_c(m, 0, 0));
          if constexpr (m > 0) hi = hi + g(spin_index_c(m, 0, 1));
          if constexpr (m == 0)
            total += hr;
          else
            total = fma_r(cr, hr, fma_r(ci, hi, total));
        }
      }
    });
    return total;
  }

  template <typename Store>
  __device__ __forceinline__ void for_each_term(Store&& st) {
    static_for<M1 - M0 + 1>([&](auto mc) {
      constexpr int m = decltype(mc)::value + M0;
      static_for<kDeg - m + 1>([&](auto nc) {
        constexpr int n = decltype(nc)::value;
        st(acc[spin_local(M0, m, n, 0)], spin_index_c(m, n, 0));
        if constexpr (m > 0) st(acc[spin_local(M0, m, n, 1)], spin_index_c(m, n, 1));
      });
    });
  }
};

// Adjoint polynomial of the FP32 path (either basis): the sum over (m, n) of the
// coefficients times the Re / Im parts of (x - i y)^m T_n(z), with Chebyshev
// polynomials T_n in place of z^n.  In this basis the coefficients of the
// spherical harmonics do not cancel (those of z^n do, by two to three orders
// of magnitude at l = 10), so FP32 evaluation keeps close to FP32 accuracy.
// The coefficients are the same for every lane (one set per primary and
// shell) and are held in vector registers: an FMA with a scalar-register
// operand issues more slowly than one with three vector registers.
struct SpinTPoly {
  float g[kTermsSpin];

  template <typename Ptr>
  __device__ __forceinline__ void load(Ptr gc) {
#pragma unroll
    for (int t = 0; t < kTermsSpin; ++t) g[t] = float(gc[t]);
  }

  __device__ __forceinline__ float eval(float x, float y, float z) const {
    float tn[kDeg + 1];
    chebyshev<kDeg>(z, tn);
    float total = g[spin_index_c(0, 0, 0)];
    static_for<kDeg>([&](auto nc) {
      constexpr int n = decltype(nc)::value + 1;
      total = fma_r(g[spin_index_c(0, n, 0)], tn[n], total);
    });
    float cr = x, ci = -y;  // (x - i y)^m, m = 1
    static_for<kDeg>([&](auto mc) {
      constexpr int m = decltype(mc)::value + 1;
      if constexpr (m > 1) {
        const float nr = fma_r(cr, x, ci * y);
        const float ni = fma_r(ci, x, -(cr * y));
        cr = nr;
        ci = ni;
      }
      float hr = g[spin_index_c(m, 0, 0)], hi = g[spin_index_c(m, 0, 1)];
      static_for<kDeg - m>([&](auto nc) {
        constexpr int n = decltype(nc)::value + 1;
        hr = fma_r(g[spin_index_c(m, n, 0)], tn[n], hr);
        hi = fma_r(g[spin_index_c(m, n, 1)], tn[n], hi);
      });
      total = fma_r(cr, hr, fma_r(ci, hi, total));
    });
    return total;
  }
};

template <class... C>
struct ChunkList {};

// Chunking keeps each chunk's accumulators within the 256 architected VGPRs.
template <typename Real, int BASIS>
struct Chunks;
template <>
struct Chunks<float, G3PCF_BASIS_CARTESIAN> {
  // z powers {0, 5, 9, 10}, {1, 4, 7, 8}, {2, 3, 6}: 91, 99 and 96 sums, so
  // that each chunk fits three waves per SIMD (two chunks at two waves
  // measured 7% slower)
  using type = ChunkList<CartChunk<float, 0x621u>, CartChunk<float, 0x192u>,
                         CartChunk<float, 0x04Cu>>;
};
template <>
struct Chunks<double, G3PCF_BASIS_CARTESIAN> {
  using type = ChunkList<CartChunk<double, 0x601u>, CartChunk<double, 0x182u>,
                         CartChunk<double, 0x00Cu>, CartChunk<double, 0x070u>>;
};
template <>
struct Chunks<float, G3PCF_BASIS_SPIN> {
  using type = ChunkList<SpinChunk<float, 0, kDeg>>;
};
template <>
struct Chunks<double, G3PCF_BASIS_SPIN> {
  using type = ChunkList<SpinChunk<double, 0, 3>, SpinChunk<double, 4, kDeg>>;
};

// Degenerate-triangle sums: D_n = sum w^2 P_n(z), n <= 2 kDeg, with the
// Legendre polynomials from their three-term recurrence (bounded by 1 on
// [-1, 1], so FP32 is accurate).  conj(Y_lm) Y_l'm depends on z alone and is
// a polynomial of degree l + l', i.e. a combination of these P_n.
template <typename Real>
struct DegChunk {
  static constexpr int NT = kTermsDeg;
  Real acc[NT];
  static __host__ __device__ constexpr int term_of(int i) { return i; }

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = Real(0);
  }

  __device__ __forceinline__ void add(Real, Real, Real z, Real w) {
    const Real w2 = w * w;
    Real p0 = Real(1), p1 = z;
    acc[0] += w2;
    acc[1] = fma_r(w2, p1, acc[1]);
    static_for<NT - 2>([&](auto nc) {
      constexpr int n = decltype(nc)::value + 1;  // P_{n+1} from P_n and P_{n-1}
      constexpr Real a = Real(2 * n + 1) / Real(n + 1), c = Real(n) / Real(n + 1);
      const Real p2 = fma_r(a * z, p1, -(c * p0));
      acc[n + 1] = fma_r(w2, p2, acc[n + 1]);
      p0 = p1;
      p1 = p2;
    });
  }
};
template <typename Real>
struct Chunks<Real, kBasisDeg> {
  using type = ChunkList<DegChunk<Real>>;
};

template <class... C, typename F>
__device__ __forceinline__ void for_each_chunk(ChunkList<C...>, F&& f) {
  (f(static_cast<C*>(nullptr)), ...);
}

}  // namespace
}  // namespace g3
