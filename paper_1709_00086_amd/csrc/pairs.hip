// The pair stage: neighbour gather, line-of-sight rotation, radial binning and
// monomial accumulation (paper, Algorithm 1 and eq. 1), followed by the FP64
// conversion of the monomial sums to a_lm (Sec. 3.1).
//
// One wavefront owns one primary at a time and pulls primaries from a shared
// counter (dynamic scheduling over primaries, as the paper's OpenMP dynamic
// schedule).  For its primary the wave
//   1. counts the accepted secondaries per radial shell (search pass 1);
//   2. writes their indices into per-shell lists in its own scratch (search
//      pass 2) -- the GPU form of the paper's per-shell pair buckets;
//   3. for each shell streams its list with one pair per lane, accumulating
//      every monomial sum in registers (vectorised over pairs, not over
//      monomials, as in the paper's vectorisation section), then reduces the
//      per-lane partials once per (primary, shell) with DPP;
//   4. converts the shell's monomial sums to a_lm in FP64 and writes them to
//      the primary's row of A.
// The candidate search walks (cy, cz) rows of the cell grid; each row's cells
// within reach form one contiguous run of galaxies, read with coalesced loads.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <type_traits>
#include <utility>

#include "internal.h"

namespace g3 {

__device__ ConvTable g_conv[2];

hipError_t upload_tables(int basis) {
  static ConvTable host[2];
  static bool built[2] = {false, false};
  if (!built[basis]) {
    build_conv_table(basis, &host[basis]);
    built[basis] = true;
  }
  return hipMemcpyToSymbol(HIP_SYMBOL(g_conv), &host[basis], sizeof(ConvTable),
                           sizeof(ConvTable) * basis, hipMemcpyHostToDevice);
}

hipError_t conv_table_device(int basis, const ConvTable** out) {
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_conv));
  if (e != hipSuccess) return e;
  *out = static_cast<const ConvTable*>(p) + basis;
  return hipSuccess;
}

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

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ double uniform_double(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane(int(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane(int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              (static_cast<unsigned int>(lo)));
}

// DPP move with compile-time controls (old value 0 where the row is masked).
template <int CTRL, int ROW, int BANK>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW, BANK, false);
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

// Cartesian chunk: the monomials u_x^k u_y^p u_z^q whose z power q is in QMASK.
// Per pair: P = w u_y^p u_z^q by running products, then acc += u_x^k * P
// (one FMA per monomial).
template <typename Real, unsigned QMASK>
struct CartChunk {
  static constexpr int NT = cart_count(QMASK);
  Real acc[NT];

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

  // adjoint: sum over this chunk's monomials of g_t * monomial (Horner in x)
  template <typename GetG>
  static __device__ __forceinline__ Real poly(Real x, Real y, Real z, GetG&& g) {
    Real total = Real(0);
    Real zq = Real(1);
    static_for<kDeg + 1>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      if constexpr (q > 0) zq = zq * z;
      if constexpr (((QMASK >> q) & 1u) != 0) {
        Real ysum = Real(0);  // sum_p y^p * (sum_k g x^k), Horner in y
        static_for<kDeg + 1 - q>([&](auto pr) {
          constexpr int p = kDeg - q - decltype(pr)::value;
          Real hx = Real(0);
          static_for<kDeg + 1 - q - p>([&](auto kr) {
            constexpr int k = kDeg - q - p - decltype(kr)::value;
            hx = fma_r(hx, x, g(cart_index_c(k, p, q)));
          });
          ysum = fma_r(ysum, y, hx);
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

// Spin chunk: S_{m,n} = sum w (u_x - i u_y)^m u_z^n for M0 <= m <= M1.
template <typename Real, int M0, int M1>
struct SpinChunk {
  static constexpr int NT = spin_count(M0, M1);
  Real acc[NT];

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = Real(0);
  }

  __device__ __forceinline__ void add(Real x, Real y, Real z, Real w) {
    constexpr int NMAX = kDeg - (M0 > 0 ? M0 : 0);
    Real zn[kDeg + 1];
    zn[0] = Real(1);
#pragma unroll
    for (int n = 1; n <= NMAX; ++n) zn[n] = zn[n - 1] * z;
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

  // adjoint: sum over this chunk of g_t * Re/Im parts of (x - i y)^m z^n
  template <typename GetG>
  static __device__ __forceinline__ Real poly(Real x, Real y, Real z, GetG&& g) {
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
        // Horner in z over n for the Re and Im coefficient sets
        Real hr = Real(0), hi = Real(0);
        static_for<kDeg - m + 1>([&](auto nr_) {
          constexpr int n = kDeg - m - decltype(nr_)::value;
          hr = fma_r(hr, z, g(spin_index_c(m, n, 0)));
          if constexpr (m > 0) hi = fma_r(hi, z, g(spin_index_c(m, n, 1)));
        });
        if constexpr (m == 0)
          total += hr;
        else
          total = fma_r(cr, hr, fma_r(ci, hi, total));
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

template <class... C>
struct ChunkList {};

// Chunking keeps each chunk's accumulators within the 256 architected VGPRs.
template <typename Real, int BASIS>
struct Chunks;
template <>
struct Chunks<float, G3PCF_BASIS_CARTESIAN> {
  using type = ChunkList<CartChunk<float, 0x023u>, CartChunk<float, 0x7DCu>>;
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

template <class... C, typename F>
__device__ __forceinline__ void for_each_chunk(ChunkList<C...>, F&& f) {
  (f(static_cast<C*>(nullptr)), ...);
}

// ---------------------------------------------------------------- per-wave LDS
template <typename Real>
struct WaveLds {
  int cnt[kMaxBins];
  int cur[kMaxBins];
  int off[kMaxBins];
  Real M[kTermsCart];
};

constexpr int kWavesPerBlock = 4;

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------- candidate search
__device__ __forceinline__ double axis_box_dist(double p, int c_u, int nc, double lo, double s,
                                                int periodic, int tight, double L) {
  if (tight) {  // min over the images of wrapped cell c_u
    double best = 1e300;
    for (int k = -1; k <= 1; ++k) {
      const double a = lo + c_u * s + k * L, b = a + s;
      const double d = fmax(0.0, fmax(a - p, p - b));
      best = fmin(best, d);
    }
    return best;
  }
  double a = lo + c_u * s, b = a + s;
  if (!periodic) {
    if (c_u == 0) a = -1e300;
    if (c_u == nc - 1) b = 1e300;
  }
  return fmax(0.0, fmax(a - p, p - b));
}

__device__ __forceinline__ int floor_div(int a, int b) {
  int q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

__device__ __forceinline__ int cell_floor(double x, double lo, double inv_s) {
  return int(floor((x - lo) * inv_s));
}

// Visit every run of candidate galaxies for a primary at p (search radius R):
// seg(g0, g1, sx, sy, sz) with the image shift of the run.
template <typename SegF>
__device__ __forceinline__ void for_each_segment(const PairArgs& a, const int* __restrict__ cs,
                                                 const double p[3], SegF&& seg) {
  const double R = a.rmax_search;
  int c0[3], c1[3];
  for (int ax = 0; ax < 3; ++ax) {
    if (a.tight[ax]) {
      c0[ax] = 0;
      c1[ax] = a.nc[ax] - 1;
    } else {
      c0[ax] = cell_floor(p[ax] - R, a.lo[ax], a.inv_s[ax]);
      c1[ax] = cell_floor(p[ax] + R, a.lo[ax], a.inv_s[ax]);
      if (!a.periodic) {
        c0[ax] = min(max(c0[ax], 0), a.nc[ax] - 1);
        c1[ax] = min(max(c1[ax], 0), a.nc[ax] - 1);
      }
    }
  }
  const int nx = a.nc[0], ny = a.nc[1], nz = a.nc[2];
  for (int czu = c0[2]; czu <= c1[2]; ++czu) {
    const double dz = axis_box_dist(p[2], czu, nz, a.lo[2], a.s[2], a.periodic, a.tight[2], a.L[2]);
    if (dz >= R) continue;
    int cz = czu;
    double sz = 0.0;
    if (a.periodic && !a.tight[2]) {
      const int k = floor_div(czu, nz);
      cz = czu - k * nz;
      sz = k * a.L[2];
    }
    for (int cyu = c0[1]; cyu <= c1[1]; ++cyu) {
      const double dy =
          axis_box_dist(p[1], cyu, ny, a.lo[1], a.s[1], a.periodic, a.tight[1], a.L[1]);
      const double d2 = dy * dy + dz * dz;
      if (d2 >= R * R) continue;
      int cy = cyu;
      double sy = 0.0;
      if (a.periodic && !a.tight[1]) {
        const int k = floor_div(cyu, ny);
        cy = cyu - k * ny;
        sy = k * a.L[1];
      }
      const int row = (cz * ny + cy) * nx;
      if (a.tight[0]) {
        const int g0 = cs[row], g1 = cs[row + nx];
        if (g1 > g0) seg(g0, g1, 0.0, sy, sz);
        continue;
      }
      const double hx = sqrt(R * R - d2);
      int x0 = cell_floor(p[0] - hx, a.lo[0], a.inv_s[0]);
      int x1 = cell_floor(p[0] + hx, a.lo[0], a.inv_s[0]);
      if (!a.periodic) {
        x0 = min(max(x0, 0), nx - 1);
        x1 = min(max(x1, 0), nx - 1);
        const int g0 = cs[row + x0], g1 = cs[row + x1 + 1];
        if (g1 > g0) seg(g0, g1, 0.0, sy, sz);
        continue;
      }
      const int k0 = floor_div(x0, nx);
      const int a0 = x0 - k0 * nx;
      const int b0 = x1 - k0 * nx;
      if (b0 < nx) {
        const int g0 = cs[row + a0], g1 = cs[row + b0 + 1];
        if (g1 > g0) seg(g0, g1, k0 * a.L[0], sy, sz);
      } else {
        int g0 = cs[row + a0], g1 = cs[row + nx];
        if (g1 > g0) seg(g0, g1, k0 * a.L[0], sy, sz);
        g0 = cs[row];
        g1 = cs[row + (b0 - nx) + 1];
        if (g1 > g0) seg(g0, g1, (k0 + 1) * a.L[0], sy, sz);
      }
    }
  }
}

// Separation, acceptance and shell of one candidate (identical in both passes).
template <typename Real>
struct PairTest {
  Real ref[3];   // primary position minus the run's image shift
  Real L[3], invL[3];
  bool minimg;   // recompute the minimum image per candidate
  Real r2max;
  Real nb_over_r;
  int nbins;
  double rmax_d;

  __device__ __forceinline__ int bin_of(const typename V4<Real>::T& q) const;
};

template <>
__device__ __forceinline__ int PairTest<float>::bin_of(const float4& q) const {
  // explicit rounding everywhere: both search passes must bin identically
  float dx = __fsub_rn(q.x, ref[0]), dy = __fsub_rn(q.y, ref[1]), dz = __fsub_rn(q.z, ref[2]);
  if (minimg) {
    dx = fma_r(-L[0], __builtin_rintf(__fmul_rn(dx, invL[0])), dx);
    dy = fma_r(-L[1], __builtin_rintf(__fmul_rn(dy, invL[1])), dy);
    dz = fma_r(-L[2], __builtin_rintf(__fmul_rn(dz, invL[2])), dz);
  }
  const float r2 = fma_r(dz, dz, fma_r(dy, dy, __fmul_rn(dx, dx)));
  if (!(r2 > 0.0f) || !(r2 < r2max)) return -1;
  const int b = int(__fmul_rn(__builtin_amdgcn_sqrtf(r2), nb_over_r));
  return b < nbins ? b : nbins - 1;
}

// FP64: the same operations, in the same order and without contraction, as
// the plain definition (minimum image by nearbyint(d / L), r = sqrt(r^2),
// shell = floor(r * nbins / R_max)).
template <>
__device__ __forceinline__ int PairTest<double>::bin_of(const double4& q) const {
  double d[3] = {__dsub_rn(q.x, ref[0]), __dsub_rn(q.y, ref[1]), __dsub_rn(q.z, ref[2])};
  if (minimg) {
    // L * k is exact for k in {-1, 0, 1}, so one rounding as in the definition
    for (int c = 0; c < 3; ++c) d[c] = __dsub_rn(d[c], __dmul_rn(L[c], rint(__ddiv_rn(d[c], L[c]))));
  }
  const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(d[0], d[0]), __dmul_rn(d[1], d[1])),
                              __dmul_rn(d[2], d[2]));
  if (!(r2 > 0.0) || !(r2 < r2max)) return -1;
  const double r = sqrt(r2);
  const int b = int(floor(__ddiv_rn(__dmul_rn(r, double(nbins)), rmax_d)));
  return b < nbins ? b : nbins - 1;
}

// ---------------------------------------------------------------- the kernel
template <typename Real, int BASIS, bool ADJOINT>
struct PairKernel {
  using V = typename V4<Real>::T;

  static __device__ __forceinline__ void run(const PairArgs& a) {
    extern __shared__ char smem_raw[];
    WaveLds<Real>* lds = reinterpret_cast<WaveLds<Real>*>(smem_raw);
    const int wid = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    WaveLds<Real>& W = lds[wid];
    const int gwave = blockIdx.x * kWavesPerBlock + wid;
    int* scratch = a.scratch + size_t(gwave) * a.scratch_per_wave;
    const V* __restrict__ pos4 = static_cast<const V*>(a.pos4);
    const int* __restrict__ cs = a.cell_start;
    const long long P = min(a.p_count, (long long)(*a.nprim) - a.p_begin);
    const int nb = a.nbins;
    const int S = a.scratch_per_wave;
    unsigned long long my_pairs = 0;

    while (true) {
      int q = 0;
      if (lane == 0) q = atomicAdd(a.queue, 1);
      q = uniform_int(__shfl(q, 0));
      if (q >= P) break;
      const int slot = uniform_int(a.plist[a.p_begin + q]);
      const V pv = pos4[slot];
      double p[3] = {uniform_double(double(pv.x)), uniform_double(double(pv.y)),
                     uniform_double(double(pv.z))};

      // line-of-sight frame (Rodrigues rotation taking the LOS to +z)
      Real Rm[9] = {Real(1), Real(0), Real(0), Real(0), Real(1), Real(0), Real(0), Real(0), Real(1)};
      if (a.los == G3PCF_LOS_OBSERVER) {
        double n[3] = {p[0] - a.obs[0], p[1] - a.obs[1], p[2] - a.obs[2]};
        const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (nn > 0.0) {
          for (int c = 0; c < 3; ++c) n[c] /= nn;
          const double c = n[2];
          if (c < -1.0 + 1e-12) {
            Rm[4] = Real(-1);
            Rm[8] = Real(-1);
          } else {
            const double vx = n[1], vy = -n[0];  // v = n x z
            const double f = 1.0 / (1.0 + c);
            const double vv = vx * vx + vy * vy;
            // R = I + [v]x + (v v^T - |v|^2 I) / (1 + c), v_z = 0
            Rm[0] = Real(1.0 + (vx * vx - vv) * f);
            Rm[1] = Real(vx * vy * f);
            Rm[2] = Real(vy);
            Rm[3] = Real(vx * vy * f);
            Rm[4] = Real(1.0 + (vy * vy - vv) * f);
            Rm[5] = Real(-vx);
            Rm[6] = Real(-vy);
            Rm[7] = Real(vx);
            Rm[8] = Real(1.0 - vv * f);
          }
        }
      }

      PairTest<Real> T;
      for (int c = 0; c < 3; ++c) {
        T.L[c] = Real(a.L[c]);
        T.invL[c] = Real(1.0 / a.L[c]);
      }
      T.minimg = a.periodic && (std::is_same<Real, double>::value || a.tight[0] || a.tight[1] ||
                                a.tight[2]);
      T.r2max = Real(a.rmax * a.rmax);
      T.nb_over_r = Real(double(nb) / a.rmax);
      T.nbins = nb;
      T.rmax_d = a.rmax;
      auto set_ref = [&](double sx, double sy, double sz) {
        if (T.minimg) {
          T.ref[0] = Real(p[0]);
          T.ref[1] = Real(p[1]);
          T.ref[2] = Real(p[2]);
        } else {
          T.ref[0] = Real(p[0] - sx);
          T.ref[1] = Real(p[1] - sy);
          T.ref[2] = Real(p[2] - sz);
        }
      };

      // ---- pass 1: count accepted secondaries per shell
      if (lane < nb) W.cnt[lane] = 0;
      wave_lds_fence();
      for_each_segment(a, cs, p, [&](int g0, int g1, double sx, double sy, double sz) {
        set_ref(sx, sy, sz);
        for (int base = g0; base < g1; base += kWave) {
          const int j = base + lane;
          if (j < g1) {
            const int b = T.bin_of(pos4[j]);
            if (b >= 0) atomicAdd(&W.cnt[b], 1);
          }
        }
      });
      wave_lds_fence();

      int total = 0;
      for (int b = 0; b < nb; ++b) total += W.cnt[b];
      my_pairs += (unsigned long long)total;

      const long long row = q;  // row of A within this pair-block

      // adjoint: primary weight
      double w_prim = 0.0;
      if constexpr (ADJOINT) w_prim = a.wsort[slot];

      // ---- passes 2 and 3 over groups of shells that fit in the scratch
      int b = 0;
      while (b < nb) {
        const int cb = uniform_int(W.cnt[b]);
        if (cb > S) {
          process_sliced(a, W, scratch, pos4, cs, p, T, set_ref, Rm, b, cb, row, slot, w_prim);
          ++b;
          continue;
        }
        int e = b, tot = 0;
        while (e < nb) {
          const int ce = uniform_int(W.cnt[e]);
          if (tot + ce > S) break;
          if (lane == 0) {
            W.off[e] = tot;
            W.cur[e] = 0;
          }
          tot += ce;
          ++e;
        }
        wave_lds_fence();
        if (tot > 0) {
          const int gb0 = b, gb1 = e;
          for_each_segment(a, cs, p, [&](int g0, int g1, double sx, double sy, double sz) {
            set_ref(sx, sy, sz);
            for (int base = g0; base < g1; base += kWave) {
              const int j = base + lane;
              if (j < g1) {
                const int bb = T.bin_of(pos4[j]);
                if (bb >= gb0 && bb < gb1) {
                  const int at = atomicAdd(&W.cur[bb], 1);
                  if (at < W.cnt[bb]) scratch[W.off[bb] + at] = j;
                }
              }
            }
          });
          wave_lds_fence();
        }
        for (int bb = b; bb < e; ++bb) {
          const int cbb = uniform_int(W.cnt[bb]);
          const int* list = scratch + uniform_int(W.off[bb]);
          shell(a, W, pos4, p, Rm, bb, list, cbb, row, slot, w_prim);
        }
        b = e;
      }
    }

    // pairs counted once per primary by lane 0
    if (lane == 0 && my_pairs) atomicAdd(a.pairs, my_pairs);
  }

  // Unit separation (rotated) and weight of list entry i (w = 0 past the end).
  static __device__ __forceinline__ void load_pair(const PairArgs& a, const V* __restrict__ pos4,
                                                   const double p[3], const Real* Rm,
                                                   const int* __restrict__ list, int count,
                                                   int i, Real& ux, Real& uy, Real& uz,
                                                   Real& w, int& j) {
    const bool valid = i < count;
    j = valid ? list[i] : -1;
    Real dx = Real(0), dy = Real(0), dz = Real(1);
    w = Real(0);
    if (valid) {
      const V qv = pos4[j];
      dx = qv.x - Real(p[0]);
      dy = qv.y - Real(p[1]);
      dz = qv.z - Real(p[2]);
      if (a.periodic) {
        dx -= Real(a.L[0]) * rint(dx * Real(1.0 / a.L[0]));
        dy -= Real(a.L[1]) * rint(dy * Real(1.0 / a.L[1]));
        dz -= Real(a.L[2]) * rint(dz * Real(1.0 / a.L[2]));
      }
      w = qv.w;
    }
    Real inv;
    if constexpr (std::is_same<Real, float>::value) {
      inv = __builtin_amdgcn_rsqf(fma_r(dz, dz, fma_r(dy, dy, dx * dx)));
    } else {
      inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    }
    dx *= inv;
    dy *= inv;
    dz *= inv;
    if (a.los == G3PCF_LOS_OBSERVER) {
      ux = Rm[0] * dx + Rm[1] * dy + Rm[2] * dz;
      uy = Rm[3] * dx + Rm[4] * dy + Rm[5] * dz;
      uz = Rm[6] * dx + Rm[7] * dy + Rm[8] * dz;
    } else {
      ux = dx;
      uy = dy;
      uz = dz;
    }
  }

  // Forward: accumulate one chunk over a list of pairs.
  template <class Chunk>
  static __device__ __forceinline__ void accumulate(const PairArgs& a, const V* __restrict__ pos4,
                                                    const double p[3], const Real* Rm,
                                                    const int* __restrict__ list, int count,
                                                    Chunk& ch) {
    const int lane = threadIdx.x % kWave;
    for (int base = 0; base < count; base += kWave) {
      Real ux, uy, uz, w;
      int j;
      load_pair(a, pos4, p, Rm, list, count, base + lane, ux, uy, uz, w, j);
      ch.add(ux, uy, uz, w);
    }
  }

  template <class Chunk>
  static __device__ __forceinline__ void reduce_store(WaveLds<Real>& W, Chunk& ch) {
    const int lane = threadIdx.x % kWave;
    ch.for_each_term([&](Real& v, int) { v = wave_sum(v); });
    if (lane == kWave - 1) ch.for_each_term([&](Real& v, int t) { W.M[t] = v; });
  }

  // Adjoint: sum_t g_t mono_t(u) over a chunk for a list, scattered into grad.
  template <class Chunk>
  static __device__ __forceinline__ void scatter(const PairArgs& a, const V* __restrict__ pos4,
                                                 const double p[3], const Real* Rm,
                                                 const int* __restrict__ list, int count,
                                                 const WaveLds<Real>& W, double w_prim) {
    const int lane = threadIdx.x % kWave;
    for (int base = 0; base < count; base += kWave) {
      Real ux, uy, uz, w;
      int j;
      load_pair(a, pos4, p, Rm, list, count, base + lane, ux, uy, uz, w, j);
      const Real v = Chunk::poly(ux, uy, uz, [&](int t) { return W.M[t]; });
      if (j >= 0) unsafeAtomicAdd(&a.grad_w[j], w_prim * double(v));
    }
  }

  // Convert the shell's monomial sums in W.M to a_lm (FP64) and write them.
  static __device__ __forceinline__ void convert(const PairArgs& a, const WaveLds<Real>& W,
                                                 int b, long long row) {
    const int lane = threadIdx.x % kWave;
    const ConvTable& t = g_conv[BASIS];
    const RowLayout& L = a.lay;
    double* out = a.A + row * L.W;
    for (int o = lane; o < kOutPerBin; o += kWave) {
      const int l = t.out_l[o];
      if (l > L.lmax) continue;
      const int m = t.out_m[o], part = t.out_part[o];
      double s = 0.0;
      for (int e = t.rowptr[o]; e < t.rowptr[o + 1]; ++e)
        s = __builtin_fma(t.coef[e], double(W.M[t.term[e]]), s);
      out[L.off[m] + part * L.d[m] + (l - m) * L.nb + b] = s;
    }
  }

  template <typename SetRef>
  static __device__ void process_sliced(const PairArgs& a, WaveLds<Real>& W, int* scratch,
                                        const V* __restrict__ pos4, const int* __restrict__ cs,
                                        const double p[3], PairTest<Real>& T, SetRef& set_ref,
                                        const Real* Rm, int b, int cb, long long row, int slot,
                                        double w_prim) {
    const int lane = threadIdx.x % kWave;
    const int S = a.scratch_per_wave;
    // fill one slice [s0, s0 + S) of shell b with deterministic ranks
    auto fill_slice = [&](int s0) {
      int rank_base = 0;
      for_each_segment(a, cs, p, [&](int g0, int g1, double sx, double sy, double sz) {
        set_ref(sx, sy, sz);
        for (int base = g0; base < g1; base += kWave) {
          const int j = base + lane;
          const bool hit = (j < g1) && (T.bin_of(pos4[j]) == b);
          const unsigned long long m = __ballot(hit);
          const int r = rank_base + __builtin_amdgcn_mbcnt_hi(
                                        unsigned(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo(unsigned(m), 0));
          if (hit && r >= s0 && r < s0 + S) scratch[r - s0] = j;
          rank_base += __popcll(m);
        }
      });
      wave_lds_fence();
    };
    using CL = typename Chunks<Real, BASIS>::type;
    if constexpr (!ADJOINT) {
      for_each_chunk(CL{}, [&](auto* tag) {
        using Chunk = std::remove_pointer_t<decltype(tag)>;
        Chunk ch;
        ch.zero();
        for (int s0 = 0; s0 < cb; s0 += S) {
          fill_slice(s0);
          accumulate(a, pos4, p, Rm, scratch, min(S, cb - s0), ch);
        }
        reduce_store(W, ch);
      });
      wave_lds_fence();
      convert(a, W, b, row);
    } else {
      load_gcoef(a, W, b, row);
      for (int s0 = 0; s0 < cb; s0 += S) {
        fill_slice(s0);
        for_each_chunk(CL{}, [&](auto* tag) {
          using Chunk = std::remove_pointer_t<decltype(tag)>;
          scatter<Chunk>(a, pos4, p, Rm, scratch, min(S, cb - s0), W, w_prim);
        });
      }
    }
    (void)slot;
  }

  static __device__ __forceinline__ void load_gcoef(const PairArgs& a, WaveLds<Real>& W, int b,
                                                    long long row) {
    const int lane = threadIdx.x % kWave;
    constexpr int T = (BASIS == G3PCF_BASIS_SPIN) ? kTermsSpin : kTermsCart;
    const double* g = a.gcoef + (row * a.nbins + b) * T;
    for (int t = lane; t < T; t += kWave) W.M[t] = Real(g[t]);
    wave_lds_fence();
  }

  static __device__ __forceinline__ void shell(const PairArgs& a, WaveLds<Real>& W,
                                               const V* __restrict__ pos4, const double p[3],
                                               const Real* Rm, int b, const int* list,
                                               int count, long long row, int slot,
                                               double w_prim) {
    using CL = typename Chunks<Real, BASIS>::type;
    if constexpr (!ADJOINT) {
      for_each_chunk(CL{}, [&](auto* tag) {
        using Chunk = std::remove_pointer_t<decltype(tag)>;
        Chunk ch;
        ch.zero();
        accumulate(a, pos4, p, Rm, list, count, ch);
        reduce_store(W, ch);
      });
      wave_lds_fence();
      convert(a, W, b, row);
      wave_lds_fence();
    } else {
      if (count == 0) return;
      load_gcoef(a, W, b, row);
      for_each_chunk(CL{}, [&](auto* tag) {
        using Chunk = std::remove_pointer_t<decltype(tag)>;
        scatter<Chunk>(a, pos4, p, Rm, list, count, W, w_prim);
      });
      wave_lds_fence();
    }
    (void)slot;
  }
};

template <typename Real, int BASIS, bool ADJOINT>
__global__ __launch_bounds__(kWave* kWavesPerBlock) void k_pairs(PairArgs a) {
  PairKernel<Real, BASIS, ADJOINT>::run(a);
}

__global__ void k_zero_queue(int* q) { *q = 0; }

template <typename Real, int BASIS, bool ADJOINT>
hipError_t launch_one(const PairArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(1), 0, st, a.queue);
  const long long want = (a.p_count + kWavesPerBlock - 1) / kWavesPerBlock;
  const unsigned blocks = unsigned(std::min<long long>(want, kPairWaves / kWavesPerBlock));
  const size_t lds = sizeof(WaveLds<Real>) * kWavesPerBlock;
  hipLaunchKernelGGL((k_pairs<Real, BASIS, ADJOINT>), dim3(blocks > 0 ? blocks : 1),
                     dim3(kWave * kWavesPerBlock), lds, st, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pair_forward(const PairArgs& a, int fp64, int basis, hipStream_t st) {
  if (fp64)
    return basis == G3PCF_BASIS_SPIN ? launch_one<double, G3PCF_BASIS_SPIN, false>(a, st)
                                     : launch_one<double, G3PCF_BASIS_CARTESIAN, false>(a, st);
  return basis == G3PCF_BASIS_SPIN ? launch_one<float, G3PCF_BASIS_SPIN, false>(a, st)
                                   : launch_one<float, G3PCF_BASIS_CARTESIAN, false>(a, st);
}

hipError_t launch_pair_adjoint(const PairArgs& a, int fp64, int basis, hipStream_t st) {
  if (fp64)
    return basis == G3PCF_BASIS_SPIN ? launch_one<double, G3PCF_BASIS_SPIN, true>(a, st)
                                     : launch_one<double, G3PCF_BASIS_CARTESIAN, true>(a, st);
  return basis == G3PCF_BASIS_SPIN ? launch_one<float, G3PCF_BASIS_SPIN, true>(a, st)
                                   : launch_one<float, G3PCF_BASIS_CARTESIAN, true>(a, st);
}

}  // namespace g3
