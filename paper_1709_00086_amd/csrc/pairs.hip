// The pair stage: neighbour gather, line-of-sight rotation, radial binning and
// monomial accumulation (paper, Algorithm 1 and eq. 1), followed by the FP64
// conversion of the monomial sums to a_lm (Sec. 3.1).
//
// One wavefront owns one primary at a time and pulls primaries from a shared
// counter (dynamic scheduling over primaries, as the paper's OpenMP dynamic
// schedule).  For its primary the wave
//   0. builds a table of candidate runs in LDS: one lane per (cy, cz) row of
//      cells, all cell-start lookups in flight at once;
//   1. searches the runs once, counting the accepted secondaries per radial
//      shell and appending (index, shell) to an unsorted list in its own
//      scratch;
//   2. sorts that list by shell (counting sort through LDS counters) into
//      per-shell lists -- the GPU form of the paper's per-shell pair buckets.
//      A primary with more pairs than the scratch holds instead fills groups
//      of shells by repeated searches;
//   3. for each shell streams its list with one pair per lane, accumulating
//      every monomial sum in registers (vectorised over pairs, not over
//      monomials, as in the paper's vectorisation section) with the gathers of
//      the next pairs in flight, then reduces the per-lane partials once per
//      (primary, shell) with DPP;
//   4. converts the shell's monomial sums to a_lm in FP64 and writes them to
//      the primary's row of A.
// The search loads four candidates per lane before testing any, so a wave
// keeps four loads in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <utility>

#include "internal.h"
#include "monomials.h"

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

// ---------------------------------------------------------------- per-wave LDS
// M holds the shell's reduced monomial sums (forward) or, in the adjoint, the
// FP64 polynomial coefficients g_t of the shell.
template <typename Real, bool ADJ>
struct WaveLds {
  using MT = std::conditional_t<ADJ, double, Real>;
  int cnt[kMaxBins];
  int cur[kMaxBins];
  int off[kMaxBins];
  int nseg;
  int seg_g0[kMaxSegments];
  int seg_g1[kMaxSegments];
  int seg_code[kMaxSegments];  // image shift (kx+1) + 3 (ky+1) + 9 (kz+1)
  MT M[kTermsCart + 1];        // (+1 padding slot)
};

constexpr int kWavesPerBlock = 4;
constexpr int kUnroll = 4;  // candidate loads in flight per lane
constexpr unsigned kShellShift = 27;  // list entry = galaxy index | shell << 27 (unsigned)

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi(unsigned(m >> 32), __builtin_amdgcn_mbcnt_lo(unsigned(m), 0));
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
  if (!periodic) {  // the outer cells also hold any point beyond the box
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

// Table of candidate runs of a primary at p: one lane per (cy, cz) row of
// cells within reach; each row contributes one or two contiguous runs of
// galaxies (two where the x window wraps around a periodic box).
template <typename Lds>
__device__ __forceinline__ void build_segments(const PairArgs& a, const int* __restrict__ cs,
                                               const double p[3], Lds& W) {
  const int lane = threadIdx.x % kWave;
  const double R = a.rmax_search;
  int c0[3], c1[3];
  for (int ax = 1; ax < 3; ++ax) {
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
  const int nyr = c1[1] - c0[1] + 1, nzr = c1[2] - c0[2] + 1;
  const int nrows = nyr * nzr;
  int nseg = 0;
  for (int rb = 0; rb < nrows; rb += kWave) {
    const int r = rb + lane;
    int n_here = 0;
    int g0a = 0, g1a = 0, ca = 0, g0b = 0, g1b = 0, cb = 0;
    if (r < nrows) {
      const int czu = c0[2] + r / nyr, cyu = c0[1] + r % nyr;
      const double dz =
          axis_box_dist(p[2], czu, nz, a.lo[2], a.s[2], a.periodic, a.tight[2], a.L[2]);
      const double dy =
          axis_box_dist(p[1], cyu, ny, a.lo[1], a.s[1], a.periodic, a.tight[1], a.L[1]);
      const double d2 = dy * dy + dz * dz;
      if (d2 < R * R) {
        int cz = czu, cy = cyu, kz = 0, ky = 0;
        if (a.periodic && !a.tight[2]) {
          kz = floor_div(czu, nz);
          cz = czu - kz * nz;
        }
        if (a.periodic && !a.tight[1]) {
          ky = floor_div(cyu, ny);
          cy = cyu - ky * ny;
        }
        const int row = (cz * ny + cy) * nx;
        const int cyz = 3 * (ky + 1) + 9 * (kz + 1);
        if (a.tight[0]) {
          g0a = cs[row];
          g1a = cs[row + nx];
          ca = 1 + cyz;
          n_here = 1;
        } else {
          const double hx = sqrt(R * R - d2);
          int x0 = cell_floor(p[0] - hx, a.lo[0], a.inv_s[0]);
          int x1 = cell_floor(p[0] + hx, a.lo[0], a.inv_s[0]);
          if (!a.periodic) {
            x0 = min(max(x0, 0), nx - 1);
            x1 = min(max(x1, 0), nx - 1);
            g0a = cs[row + x0];
            g1a = cs[row + x1 + 1];
            ca = 1 + cyz;
            n_here = 1;
          } else {
            const int k0 = floor_div(x0, nx);
            const int a0 = x0 - k0 * nx, b0 = x1 - k0 * nx;
            if (b0 < nx) {
              g0a = cs[row + a0];
              g1a = cs[row + b0 + 1];
              ca = (k0 + 1) + cyz;
              n_here = 1;
            } else {
              g0a = cs[row + a0];
              g1a = cs[row + nx];
              ca = (k0 + 1) + cyz;
              g0b = cs[row];
              g1b = cs[row + (b0 - nx) + 1];
              cb = (k0 + 2) + cyz;
              n_here = 2;
            }
          }
        }
      }
    }
    const unsigned long long m1 = __ballot(n_here >= 1), m2 = __ballot(n_here >= 2);
    const int at = nseg + lanes_below(m1) + lanes_below(m2);
    if (n_here >= 1 && at < kMaxSegments) {
      W.seg_g0[at] = g0a;
      W.seg_g1[at] = g1a;
      W.seg_code[at] = ca;
    }
    if (n_here >= 2 && at + 1 < kMaxSegments) {
      W.seg_g0[at + 1] = g0b;
      W.seg_g1[at + 1] = g1b;
      W.seg_code[at + 1] = cb;
    }
    nseg += __popcll(m1) + __popcll(m2);
  }
  if (lane == 0) W.nseg = min(nseg, kMaxSegments);
  wave_lds_fence();
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
    for (int c = 0; c < 3; ++c)
      d[c] = __dsub_rn(d[c], __dmul_rn(L[c], rint(__ddiv_rn(d[c], L[c]))));
  }
  const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(d[0], d[0]), __dmul_rn(d[1], d[1])),
                              __dmul_rn(d[2], d[2]));
  if (!(r2 > 0.0) || !(r2 < r2max)) return -1;
  const double r = sqrt(r2);
  const int b = int(floor(__ddiv_rn(__dmul_rn(r, double(nbins)), rmax_d)));
  return b < nbins ? b : nbins - 1;
}

// Occupancy target per kernel (waves per SIMD); the register budget is
// 512 / target per lane, so every accumulator chunk must fit.
template <typename Real, int BASIS, bool ADJOINT>
struct Occ {
  static constexpr int value =
      ADJOINT ? 3 : ((std::is_same<Real, float>::value && BASIS == G3PCF_BASIS_SPIN) ? 3 : 2);
};

// ---------------------------------------------------------------- the kernel
template <typename Real, int BASIS, bool ADJOINT>
struct PairKernel {
  using V = typename V4<Real>::T;
  using Lds = WaveLds<Real, ADJOINT>;

  // All lanes visit every candidate of the segment table; f(j, bin) is called
  // by every lane (bin = -1 for a rejected or absent candidate).
  template <typename F>
  static __device__ __forceinline__ void scan(const PairArgs& a, const Lds& W,
                                              const V* __restrict__ pos4, const double p[3],
                                              PairTest<Real>& T, F&& f) {
    const int lane = threadIdx.x % kWave;
    const int nseg = uniform_int(W.nseg);
    for (int s = 0; s < nseg; ++s) {
      const int g0 = uniform_int(W.seg_g0[s]), g1 = uniform_int(W.seg_g1[s]);
      if (g1 <= g0) continue;
      if (!T.minimg) {
        const int code = uniform_int(W.seg_code[s]);
        const int kx = code % 3 - 1, ky = (code / 3) % 3 - 1, kz = code / 9 - 1;
        T.ref[0] = Real(p[0] - kx * a.L[0]);
        T.ref[1] = Real(p[1] - ky * a.L[1]);
        T.ref[2] = Real(p[2] - kz * a.L[2]);
      }
      for (int base = g0; base < g1; base += kUnroll * kWave) {
        V q[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) q[u] = pos4[min(base + u * kWave + lane, g1 - 1)];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int j = base + u * kWave + lane;
          const int b = (j < g1) ? T.bin_of(q[u]) : -1;
          f(j, b);
        }
      }
    }
  }

  static __device__ __forceinline__ void run(const PairArgs& a) {
    extern __shared__ char smem_raw[];
    Lds* lds = reinterpret_cast<Lds*>(smem_raw);
    // wave index made uniform so that per-wave pointers live in scalar registers
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    Lds& W = lds[wid];
    const int gwave = blockIdx.x * kWavesPerBlock + wid;
    int* scratch = a.scratch + size_t(gwave) * 2 * a.scratch_per_wave;
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
        T.ref[c] = Real(p[c]);
      }
      T.minimg = a.periodic && (std::is_same<Real, double>::value || a.tight[0] || a.tight[1] ||
                                a.tight[2]);
      T.r2max = Real(a.rmax * a.rmax);
      T.nb_over_r = Real(double(nb) / a.rmax);
      T.nbins = nb;
      T.rmax_d = a.rmax;

      // ---- pass 0: candidate runs.  Pass 1: one search that counts the
      // accepted secondaries per shell and appends (index | shell << 27) to an
      // unsorted list in the second half of the scratch.
      build_segments(a, cs, p, W);
      if (lane < nb) W.cnt[lane] = 0;
      wave_lds_fence();
      unsigned* unsorted = reinterpret_cast<unsigned*>(scratch + S);
      int appended = 0;
      scan(a, W, pos4, p, T, [&](int j, int b) {
        const bool hit = b >= 0;
        if (hit) atomicAdd(&W.cnt[b], 1);
        const unsigned long long m = __ballot(hit);
        const int at = appended + lanes_below(m);
        if (hit && at < S && a.packed_lists) unsorted[at] = unsigned(j) | (unsigned(b) << kShellShift);
        appended += __popcll(m);
      });
      wave_lds_fence();

      int total = 0;
      for (int b = 0; b < nb; ++b) total += W.cnt[b];
      my_pairs += (unsigned long long)total;

      const long long row = q;  // row of A within this pair-block
      double w_prim = 0.0;
      if constexpr (ADJOINT) w_prim = a.wsort[slot];

      if (total <= S && a.packed_lists) {
        // ---- pass 2: counting sort of the unsorted list by shell
        if (lane == 0) {
          int off = 0;
          for (int b = 0; b < nb; ++b) {
            W.off[b] = off;
            W.cur[b] = 0;
            off += W.cnt[b];
          }
        }
        wave_lds_fence();
        // eight entries per lane in flight: loads, then the LDS slot atomics,
        // then the stores
        constexpr int kSortUnroll = 8;
        for (int base = 0; base < total; base += kSortUnroll * kWave) {
          unsigned e[kSortUnroll];
          int at[kSortUnroll];
#pragma unroll
          for (int u = 0; u < kSortUnroll; ++u)
            e[u] = unsorted[min(base + u * kWave + lane, total - 1)];
#pragma unroll
          for (int u = 0; u < kSortUnroll; ++u) {
            const bool ok = base + u * kWave + lane < total;
            at[u] = ok ? atomicAdd(&W.cur[e[u] >> kShellShift], 1) : 0;
          }
#pragma unroll
          for (int u = 0; u < kSortUnroll; ++u) {
            if (base + u * kWave + lane < total)
              scratch[W.off[e[u] >> kShellShift] + at[u]] = int(e[u] & ((1u << kShellShift) - 1u));
          }
        }
        wave_lds_fence();
        // ---- pass 3: every shell from its list
        for (int b = 0; b < nb; ++b) {
          const int cb = uniform_int(W.cnt[b]);
          const int* list = scratch + uniform_int(W.off[b]);
          shell(a, W, pos4, p, Rm, b, list, cb, row, w_prim);
        }
        continue;
      }

      // ---- more pairs than the scratch holds: groups of shells that fit,
      // each filled by a repeated search
      int b = 0;
      while (b < nb) {
        const int cb = uniform_int(W.cnt[b]);
        if (cb > S) {
          process_sliced(a, W, scratch, pos4, p, T, Rm, b, cb, row, w_prim);
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
          scan(a, W, pos4, p, T, [&](int j, int bb) {
            if (bb >= gb0 && bb < gb1) {
              const int at = atomicAdd(&W.cur[bb], 1);
              if (at < W.cnt[bb]) scratch[W.off[bb] + at] = j;
            }
          });
          wave_lds_fence();
        }
        for (int bb = b; bb < e; ++bb) {
          const int cbb = uniform_int(W.cnt[bb]);
          const int* list = scratch + uniform_int(W.off[bb]);
          shell(a, W, pos4, p, Rm, bb, list, cbb, row, w_prim);
        }
        b = e;
      }
    }

    if (lane == 0 && my_pairs) atomicAdd(a.pairs, my_pairs);
  }

  // Unit separation (rotated) and weight from a loaded secondary.
  static __device__ __forceinline__ void unit_pair(const PairArgs& a, const V& qv, bool valid,
                                                   const double p[3], const Real* Rm, Real& ux,
                                                   Real& uy, Real& uz, Real& w) {
    Real dx = qv.x - Real(p[0]);
    Real dy = qv.y - Real(p[1]);
    Real dz = qv.z - Real(p[2]);
    if (a.periodic) {
      dx -= Real(a.L[0]) * rint(dx * Real(1.0 / a.L[0]));
      dy -= Real(a.L[1]) * rint(dy * Real(1.0 / a.L[1]));
      dz -= Real(a.L[2]) * rint(dz * Real(1.0 / a.L[2]));
    }
    w = valid ? qv.w : Real(0);
    if (!valid) {
      dx = Real(0);
      dy = Real(0);
      dz = Real(1);
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

  // Stream a list with the gather of the next pair and the index two pairs
  // ahead already in flight; body(ux, uy, uz, w, j, valid) per lane.
  template <typename Body>
  static __device__ __forceinline__ void stream(const PairArgs& a, const V* __restrict__ pos4,
                                                const double p[3], const Real* Rm,
                                                const int* __restrict__ list, int count,
                                                Body&& body) {
    if (count <= 0) return;
    const int lane = threadIdx.x % kWave;
    const int last = count - 1;
    int j0 = list[min(lane, last)];
    int j1 = list[min(kWave + lane, last)];
    V q0 = pos4[j0];
    for (int base = 0; base < count; base += kWave) {
      const V qc = q0;
      const int jc = j0;
      const bool valid = base + lane < count;
      q0 = pos4[j1];
      j0 = j1;
      j1 = list[min(base + 2 * kWave + lane, last)];
      Real ux, uy, uz, w;
      unit_pair(a, qc, valid, p, Rm, ux, uy, uz, w);
      body(ux, uy, uz, w, jc, valid);
    }
  }

  // Wave sums of a chunk's accumulators into W.M, four at a time: row sums by
  // DPP, then one fold across rows leaves the four totals in rows 0..3, and
  // every lane stores its row's total (16 lanes write the same value).
  template <class Chunk>
  static __device__ __forceinline__ void reduce_store(Lds& W, Chunk& ch) {
    constexpr int NT = Chunk::NT;
    constexpr int kJunk = kTermsCart;  // slot that absorbs padding in the last group
    const int row = (threadIdx.x % kWave) >> 4;
    static_for<(NT + 3) / 4>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      constexpr int i0 = 4 * g, i1 = 4 * g + 1, i2 = 4 * g + 2, i3 = 4 * g + 3;
      const Real a = row_sum(ch.acc[i0]);
      Real e = Real(0), b = Real(0), f = Real(0);
      if constexpr (i1 < NT) e = row_sum(ch.acc[i1]);
      if constexpr (i2 < NT) b = row_sum(ch.acc[i2]);
      if constexpr (i3 < NT) f = row_sum(ch.acc[i3]);
      const Real tot = fold4(a, e, b, f);
      constexpr int ta = Chunk::term_of(i0);
      constexpr int te = (i1 < NT) ? Chunk::term_of(i1) : kJunk;
      constexpr int tb = (i2 < NT) ? Chunk::term_of(i2) : kJunk;
      constexpr int tf = (i3 < NT) ? Chunk::term_of(i3) : kJunk;
      const int t = row == 0 ? ta : (row == 1 ? te : (row == 2 ? tb : tf));
      W.M[t] = tot;
    });
  }

  // Convert the shell's monomial sums in W.M to a_lm (FP64) and write them.
  static __device__ __forceinline__ void convert(const PairArgs& a, const Lds& W,
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

  static __device__ __forceinline__ void load_gcoef(const PairArgs& a, Lds& W, int b,
                                                    long long row) {
    const int lane = threadIdx.x % kWave;
    constexpr int T = (BASIS == G3PCF_BASIS_SPIN) ? kTermsSpin : kTermsCart;
    const double* g = a.gcoef + (row * a.nbins + b) * T;
    for (int t = lane; t < T; t += kWave) W.M[t] = g[t];
    wave_lds_fence();
  }

  // Adjoint scatter over a list: per pair the full polynomial
  // sum_t g_t mono_t(u) in FP64 (its coefficients cancel strongly at l = 10),
  // with the coefficients read from LDS through an offset the compiler cannot
  // hoist out of the loop, so they do not occupy registers.
  static __device__ __forceinline__ void scatter(const PairArgs& a, const Lds& W,
                                                 const V* __restrict__ pos4, const double p[3],
                                                 const Real* Rm, const int* list, int count,
                                                 double w_prim) {
    using Poly = std::conditional_t<BASIS == G3PCF_BASIS_SPIN, SpinChunk<double, 0, kDeg>,
                                    CartChunk<double, (1u << (kDeg + 1)) - 1>>;
    stream(a, pos4, p, Rm, list, count, [&](Real ux, Real uy, Real uz, Real, int j, bool valid) {
      int off = 0;
      asm volatile("" : "+v"(off));
      const double v = Poly::poly(double(ux), double(uy), double(uz),
                                  [&](int t) { return W.M[t + off]; });
      if (valid) unsafeAtomicAdd(&a.grad_w[j], w_prim * v);
    });
  }

  // Forward: all chunks of one shell from a list, then conversion.
  static __device__ __forceinline__ void shell(const PairArgs& a, Lds& W,
                                               const V* __restrict__ pos4, const double p[3],
                                               const Real* Rm, int b, const int* list,
                                               int count, long long row, double w_prim) {
    using CL = typename Chunks<Real, BASIS>::type;
    if constexpr (!ADJOINT) {
      for_each_chunk(CL{}, [&](auto* tag) {
        using Chunk = std::remove_pointer_t<decltype(tag)>;
        Chunk ch;
        ch.zero();
        stream(a, pos4, p, Rm, list, count,
               [&](Real ux, Real uy, Real uz, Real w, int, bool) { ch.add(ux, uy, uz, w); });
        reduce_store(W, ch);
      });
      wave_lds_fence();
      convert(a, W, b, row);
      wave_lds_fence();
    } else {
      if (count == 0) return;
      load_gcoef(a, W, b, row);
      scatter(a, W, pos4, p, Rm, list, count, w_prim);
      wave_lds_fence();
    }
  }

  // A shell with more pairs than the scratch holds: slices of S pairs in a
  // deterministic order (ballot ranks), the search repeated per slice.
  static __device__ void process_sliced(const PairArgs& a, Lds& W, int* scratch,
                                        const V* __restrict__ pos4, const double p[3],
                                        PairTest<Real>& T, const Real* Rm, int b, int cb,
                                        long long row, double w_prim) {
    const int S = a.scratch_per_wave;
    auto fill_slice = [&](int s0) {
      int rank_base = 0;
      scan(a, W, pos4, p, T, [&](int j, int bb) {
        const bool hit = (bb == b);
        const unsigned long long m = __ballot(hit);
        const int r = rank_base + lanes_below(m);
        if (hit && r >= s0 && r < s0 + S) scratch[r - s0] = j;
        rank_base += __popcll(m);
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
          stream(a, pos4, p, Rm, scratch, min(S, cb - s0),
                 [&](Real ux, Real uy, Real uz, Real w, int, bool) { ch.add(ux, uy, uz, w); });
        }
        reduce_store(W, ch);
      });
      wave_lds_fence();
      convert(a, W, b, row);
      wave_lds_fence();
    } else {
      load_gcoef(a, W, b, row);
      for (int s0 = 0; s0 < cb; s0 += S) {
        fill_slice(s0);
        scatter(a, W, pos4, p, Rm, scratch, min(S, cb - s0), w_prim);
      }
      wave_lds_fence();
    }
  }
};

template <typename Real, int BASIS, bool ADJOINT>
__global__ __launch_bounds__(kWave* kWavesPerBlock)
    __attribute__((amdgpu_waves_per_eu(Occ<Real, BASIS, ADJOINT>::value))) void k_pairs(
        PairArgs a) {
  PairKernel<Real, BASIS, ADJOINT>::run(a);
}

__global__ void k_zero_queue(int* q) { *q = 0; }

template <typename Real, int BASIS, bool ADJOINT>
hipError_t launch_one(const PairArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(1), 0, st, a.queue);
  const long long want = (a.p_count + kWavesPerBlock - 1) / kWavesPerBlock;
  const unsigned blocks = unsigned(std::min<long long>(want, kPairWaves / kWavesPerBlock));
  const size_t lds = sizeof(typename PairKernel<Real, BASIS, ADJOINT>::Lds) * kWavesPerBlock;
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
