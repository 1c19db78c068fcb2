// The pair stage: neighbour gather, line-of-sight rotation, radial binning and
// monomial accumulation (paper, Algorithm 1 and eq. 1), followed by the FP64
// conversion of the monomial sums to a_lm (Sec. 3.1).
//
// One wavefront owns one primary at a time and pulls primaries from a shared
// counter (dynamic scheduling over primaries, as the paper's OpenMP dynamic
// schedule; one counter per XCD over a contiguous share of the primaries, so
// that the primaries an XCD works on at once share candidates in its L2).
// For its primary the wave takes the radial shells one after the other; for
// shell b it
//   1. builds, 64 rows of cells at a time (one lane per (cy, cz) row), the
//      runs of galaxies that can lie in the annulus: per row the x-interval
//      of the outer sphere minus the x-interval of the inner sphere, i.e. at
//      most two contiguous ranges of cells (four where they wrap around a
//      periodic box).  All cell-start lookups of the 64 rows are in flight at
//      once, and the runs go into a table in LDS with their prefix sums;
//   2. streams the runs' galaxies with one candidate per lane (a lane finds
//      its run among the run starts, which the wave keeps in a register; the
//      next window's loads are in flight while one is binned), bins each
//      candidate with the shell's squared edges, and appends the accepted
//      separations to a ring of pairs in LDS -- the GPU form of the paper's
//      per-bin pair buckets;
//   3. whenever the ring holds a full wave of pairs, normalises and rotates
//      them and accumulates them, one pair per lane, into every monomial sum
//      of the shell held in registers (vectorised over pairs, not over
//      monomials, as in the paper's vectorisation section);
//   4. reduces the per-lane partials once per (primary, shell) with DPP and
//      converts the shell's monomial sums to a_lm in FP64.
// No neighbour list ever leaves the compute unit.  A basis whose sums do not
// fit in registers at once is accumulated in chunks: the first chunk's
// search also writes the shell's secondary indices to the wave's spill list,
// which the later chunks replay (a repeated search if the list overflowed).
//
// The adjoint kernel runs the same search and, per accepted pair, evaluates
// the shell's adjoint polynomial in FP64 and adds it to the secondary's
// gradient with one atomic (FP32 on the FP32 path, FP64 on the FP64 path).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <type_traits>
#include <utility>

#include "internal.h"
#include "monomials.h"

namespace g3 {

__device__ ConvTable g_conv[kConvTables];

hipError_t upload_tables(int basis) {
  static ConvTable host[kConvTables];
  static bool built[kConvTables] = {};
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

constexpr int kWavesPerBlock = 4;
constexpr int kMaxRuns = 4 * kWave;  // runs of one chunk of 64 rows (<= 4 per row)
constexpr int kRing = 2 * kWave;     // accepted pairs waiting for a full wave
constexpr int kAdjStripes = 16;      // interleaved stripes of an XCD's share (adjoint)
// Run-start marks: one bit per virtual candidate index, for a span of
// kMarkSpan candidates of the run table at a time (64 windows).
constexpr int kMarkSpan = 64 * kWave;
constexpr int kMarkWords = kMarkSpan / 32;

// A run of the table: g0 is the cell-order slot of its first galaxy minus the
// run's first virtual candidate index (so candidate c of the run is slot
// g0 + c).  FP32 keeps the primary's position minus the run's periodic image
// shift (the reference the candidates are measured from).
template <typename Real>
struct RunEntry;
template <>
struct RunEntry<float> {
  float rx, ry, rz;
  int g0;
};
template <>
struct RunEntry<double> {
  int g0;
};

// ---------------------------------------------------------------- per-wave LDS
// M holds the shell's reduced monomial sums (forward only).
// FP32 adjoint: (secondary, term) pairs waiting for their atomic add.
constexpr int kOutBuf = 8 * kWave;

template <typename Real, bool ADJ, bool SPINT = false>
struct WaveLds {
  using V = typename V4<Real>::T;
  int pre[kMaxRuns + 1];       // first virtual candidate index of each run
  alignas(16) RunEntry<Real> run[kMaxRuns + 1];  // (+1: the FP32 search's sentinel run)
  V ring[kRing];               // (d_x, d_y, d_z, w) forward; (d_x, d_y, d_z, index) adjoint
  int ring_j[kRing];           // secondary index of a ring entry (when spilled)
  // bit c of the span: a run starts at virtual candidate index mbase + c
  __attribute__((aligned(16))) unsigned marks[kMarkWords];
  // forward: the reduced sums (+1 padding slot); FP32 adjoint: the
  // shell's polynomial coefficients on their way into vector registers
  Real M[ADJ ? (SPINT ? kTermsSpin + 3 : 1) : kTermsCart + 1];
  int2 out[SPINT ? kOutBuf : 1];
};

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// Lane index computed in place (the compiler cannot hoist an asm statement),
// so that no lane-dependent address has to stay live, or be spilled, across
// the accumulation loops.
__device__ __forceinline__ int lane_here() {
  int v;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(v));
  return v;
}

// Mask of the lanes where c holds (the compare result itself, without
// materialising the predicate in a vector register first).
__device__ __forceinline__ unsigned long long ballot(bool c) {
  return __builtin_amdgcn_ballot_w64(c);
}

__device__ __forceinline__ int lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi(unsigned(m >> 32), __builtin_amdgcn_mbcnt_lo(unsigned(m), 0));
}

// Inclusive prefix sum over the 64 lanes with DPP moves only (no lane
// addresses to keep live): row_shr 1, 2, 4 and 8 give every lane the sum of
// its row up to itself (lanes shifted in from outside the row read 0), then
// row_bcast 15 adds the last lane of rows 0 and 2 to rows 1 and 3, and
// row_bcast 31 the last lane of row 1 (rows 0-1 by then) to rows 2 and 3.
__device__ __forceinline__ int wave_incl_scan(int x) {
  x += dpp_i<0x111, 0xF, 0xF>(x);
  x += dpp_i<0x112, 0xF, 0xF>(x);
  x += dpp_i<0x114, 0xF, 0xF>(x);
  x += dpp_i<0x118, 0xF, 0xF>(x);
  x += dpp_i<0x142, 0xA, 0xF>(x);
  x += dpp_i<0x143, 0xC, 0xF>(x);
  return x;
}

// index <-> last component of a ring entry
__device__ __forceinline__ float pack_index(int j, float) { return __int_as_float(j); }
__device__ __forceinline__ double pack_index(int j, double) { return double(j); }
__device__ __forceinline__ int unpack_index(float v) { return __float_as_int(v); }
__device__ __forceinline__ int unpack_index(double v) { return int(v); }

// ---------------------------------------------------------------- geometry
// Distance range along one axis from the primary to cell c_u (unwrapped
// index): the nearest and farthest points of the cell.  The outer cells of an
// open box also hold any point beyond it, and on a tight periodic axis the
// nearest distance is taken over the images (the farthest is then not used).
// Computed in cell units measured from the primary: prel is the primary's
// coordinate in cells ((p - lo) / s, FP64), the result in length units (FP32).  The rounding (about 1e-6 cells) is far inside the search
// margin, which enters the squared distances as 2 R_max * margin.
__device__ __forceinline__ void axis_range_f(double prel, int c_u, int nc, float s,
                                             int periodic, int tight, float& dmin,
                                             float& dmax) {
  const float t0 = float(double(c_u) - prel);
  if (tight) {  // min over the images of wrapped cell c_u
    float best = __builtin_huge_valf();
    for (int k = -1; k <= 1; ++k) {
      const float lo = t0 + float(k * nc), hi = lo + 1.0f;
      best = fminf(best, fmaxf(0.0f, fmaxf(lo, -hi)));
    }
    dmin = best * s;
    dmax = __builtin_huge_valf();
    return;
  }
  float lo = t0, hi = t0 + 1.0f;
  if (!periodic) {  // the outer cells also hold any point beyond the box
    if (c_u == 0) lo = -__builtin_huge_valf();
    if (c_u == nc - 1) hi = __builtin_huge_valf();
  }
  dmin = fmaxf(0.0f, fmaxf(lo, -hi)) * s;
  dmax = fmaxf(fabsf(lo), fabsf(hi)) * s;
}

__device__ __forceinline__ int cell_of(double c) { return int(fmin(fmax(floor(c), -1e9), 1e9)); }

// Periodic wrap of an unwrapped cell index c in [-n, 2n) (a search window on a
// non-tight axis spans less than one box): c -> c - k n with k in {-1, 0, 1}.
__device__ __forceinline__ int wrap_cell(int c, int n, int& k) {
  k = (c < 0) ? -1 : (c >= n ? 1 : 0);
  return c - k * n;
}

// q = r / d and r - q d for 0 <= r < 2^24 and a uniform d > 0, from a float
// reciprocal corrected by one step.
__device__ __forceinline__ int div_small(int r, int d, float inv_d, int& rem) {
  int q = int(float(r) * inv_d);
  rem = r - q * d;
  if (rem < 0) {
    --q;
    rem += d;
  } else if (rem >= d) {
    ++q;
    rem -= d;
  }
  return q;
}

__device__ __forceinline__ int cell_floor(double x, double lo, double inv_s) {
  // clamp before the conversion so that far-away coordinates cannot overflow
  const double c = floor((x - lo) * inv_s);
  return int(fmin(fmax(c, -1e9), 1e9));
}

// ---------------------------------------------------------------- binning
// FP64 shell of a candidate: the same operations, in the same order and
// without contraction, as the plain definition (minimum image by
// nearbyint(d / L), r = sqrt(r^2), shell = floor(r * nbins / R_max)).
// Returns -1 for a rejected candidate.
struct Bin64 {
  double L[3];
  bool minimg;
  double r2max;
  int nbins;
  double rmax;

  __device__ __forceinline__ int classify(const double4& q, const double ref[3], double d[3],
                                          double& r2) const {
    d[0] = __dsub_rn(q.x, ref[0]);
    d[1] = __dsub_rn(q.y, ref[1]);
    d[2] = __dsub_rn(q.z, ref[2]);
    if (minimg) {
      // L * k is exact for k in {-1, 0, 1}, so one rounding as in the definition
      for (int c = 0; c < 3; ++c)
        d[c] = __dsub_rn(d[c], __dmul_rn(L[c], rint(__ddiv_rn(d[c], L[c]))));
    }
    r2 = __dadd_rn(__dadd_rn(__dmul_rn(d[0], d[0]), __dmul_rn(d[1], d[1])),
                   __dmul_rn(d[2], d[2]));
    if (!(r2 > 0.0) || !(r2 < r2max)) return -1;
    const double r = sqrt(r2);
    const int b = int(floor(__ddiv_rn(__dmul_rn(r, double(nbins)), rmax)));
    return b < nbins ? b : nbins - 1;
  }
};

// Occupancy target per kernel (waves per SIMD); the register budget is
// 512 / target per lane, so every accumulator chunk must fit.  The FP64 and
// cartesian adjoints hold no accumulators: at four waves they spill a few
// values outside their loops and hide more of their atomics' latency (5-11%
// faster than three).  The FP32 adjoint (the spin-basis instantiation, used
// after a forward pass in either basis) holds its 121 coefficients in
// vector registers, like the forward's 121 sums: three waves.
template <typename Real, int BASIS, bool ADJOINT>
struct Occ {
  static constexpr bool kSpinT =
      ADJOINT && std::is_same<Real, float>::value && BASIS == G3PCF_BASIS_SPIN;
  static constexpr int value = kSpinT ? 3
                               : (ADJOINT || BASIS == kBasisDeg)
                                   ? 4
                                   : (std::is_same<Real, float>::value ? 3 : 2);
};

template <class... C>
constexpr int n_chunks(ChunkList<C...>) {
  return int(sizeof...(C));
}

// ---------------------------------------------------------------- the kernel
// kRot: line of sight towards the observer (every separation is rotated);
// kMin: FP32 minimum image per candidate (a periodic axis where the search
// window can wrap onto itself).  Both are fixed per launch, so each kernel
// holds the code and the live values of one mode only.
template <typename Real, int BASIS, bool ADJOINT, bool kRot, bool kMin>
struct PairKernel {
  using V = typename V4<Real>::T;
  // FP32 adjoint: Chebyshev-basis polynomial in FP32 (SpinTPoly)
  static constexpr bool kSpinT = Occ<Real, BASIS, ADJOINT>::kSpinT;
  using Lds = WaveLds<Real, ADJOINT, kSpinT>;
  static constexpr bool kF32 = std::is_same<Real, float>::value;
  static constexpr int kTerms = (BASIS == G3PCF_BASIS_SPIN) ? kTermsSpin
                                : (BASIS == kBasisDeg)      ? kTermsDeg
                                                            : kTermsCart;
  // read-only device memory in the constant address space (scalar loads)
  using CoefPtr = const double __attribute__((address_space(4)))*;

  // Per-primary state shared by the shell searches.
  struct Primary {
    double p[3];
    Real pref[3];  // primary position in the working precision
    double invLd[3];
    double prel[3];  // primary position in cell units, (p - lo) / s
    float sf[3];     // cell sides
    Real L[3], invL[3];
    Real Rm[9];    // line-of-sight rotation (kRot)
    bool minimg;   // minimum image per candidate (else the run's image shift)
    Bin64 bin64;
  };

  // Runs of the rows [rb, rb + 64) of the window for the annulus
  // r0 <= r < r1 (given as r0^2, r1^2) into the LDS table; returns the number
  // of runs and sets `total` to their summed length.
  static __device__ __forceinline__ int build_runs(const PairArgs& a, const int* __restrict__ cs,
                                                   const Primary& P, double r0sq, double r1sq,
                                                   const int c0[3], int nyr, float inv_nyr,
                                                   int rb, int nrows, Lds& W, int& total) {
    const int lane = threadIdx.x % kWave;
    const double* p = P.p;
    const int nx = a.nc[0], ny = a.nc[1], nz = a.nc[2];
    int n_here = 0;
    int g0v[4] = {0, 0, 0, 0}, lenv[4] = {0, 0, 0, 0}, kxv[4] = {0, 0, 0, 0};
    int ky = 0, kz = 0;
    const int r = rb + lane;
    if (r < nrows) {
      int ry;
      const int czu = c0[2] + div_small(r, nyr, inv_nyr, ry), cyu = c0[1] + ry;
      float dzmin, dzmax, dymin, dymax;
      axis_range_f(P.prel[2], czu, nz, P.sf[2], a.periodic, a.tight[2], dzmin, dzmax);
      axis_range_f(P.prel[1], cyu, ny, P.sf[1], a.periodic, a.tight[1], dymin, dymax);
      const float d2min = dymin * dymin + dzmin * dzmin;
      if (double(d2min) < r1sq) {
        int cz = czu, cy = cyu;
        if (a.periodic && !a.tight[2]) cz = wrap_cell(czu, nz, kz);
        if (a.periodic && !a.tight[1]) cy = wrap_cell(cyu, ny, ky);
        const int row = (cz * ny + cy) * nx;
        // up to two x-intervals of cells (unwrapped indices)
        int ia[2] = {0, 0}, ib[2] = {0, 0}, ni = 0;
        if (a.tight[0]) {
          ia[0] = 0;
          ib[0] = nx - 1;
          ni = 1;
        } else {
          // half-chords in FP32, widened by a relative 2e-6 (inside the margin)
          const float hx1 =
              __builtin_sqrtf(float(r1sq - double(d2min))) * (1.0f + 2e-6f) + 1e-6f;
          const float d2max = dymax * dymax + dzmax * dzmax;
          const bool cut = r0sq > 0.0 && !a.tight[1] && !a.tight[2] && r0sq > double(d2max);
          const float hx0 =
              cut ? fmaxf(0.0f, __builtin_sqrtf(float(r0sq - double(d2max))) * (1.0f - 2e-6f) -
                                    1e-6f)
                  : 0.0f;
          const double px = P.prel[0], ix = a.inv_s[0];
          int a1 = cell_of(px - double(hx1) * ix);
          int b1 = cell_of(px - double(hx0) * ix);
          int a2 = cell_of(px + double(hx0) * ix);
          int b2 = cell_of(px + double(hx1) * ix);
          if (!a.periodic) {
            a1 = min(max(a1, 0), nx - 1);
            b1 = min(max(b1, 0), nx - 1);
            a2 = min(max(a2, 0), nx - 1);
            b2 = min(max(b2, 0), nx - 1);
          }
          if (a2 <= b1 + 1) {
            ia[0] = a1;
            ib[0] = b2;
            ni = 1;
          } else {
            ia[0] = a1;
            ib[0] = b1;
            ia[1] = a2;
            ib[1] = b2;
            ni = 2;
          }
        }
        // cell ranges -> galaxy runs (a periodic interval may wrap once)
        int ca[4] = {0, 0, 0, 0}, cb[4] = {0, 0, 0, 0}, kk[4] = {0, 0, 0, 0}, nr = 0;
        for (int i = 0; i < ni; ++i) {
          if (a.periodic && !a.tight[0]) {
            int k0;
            const int lo_c = wrap_cell(ia[i], nx, k0), hi_c = ib[i] - k0 * nx;
            if (hi_c < nx) {
              ca[nr] = lo_c;
              cb[nr] = hi_c;
              kk[nr++] = k0;
            } else {
              ca[nr] = lo_c;
              cb[nr] = nx - 1;
              kk[nr++] = k0;
              ca[nr] = 0;
              cb[nr] = hi_c - nx;
              kk[nr++] = k0 + 1;
            }
          } else {
            ca[nr] = ia[i];
            cb[nr] = ib[i];
            kk[nr++] = 0;
          }
        }
        int g0s[4], g1s[4];
        for (int i = 0; i < nr; ++i) {
          g0s[i] = cs[row + ca[i]];
          g1s[i] = cs[row + cb[i] + 1];
        }
        for (int i = 0; i < nr; ++i) {
          if (g1s[i] > g0s[i]) {
            g0v[n_here] = g0s[i];
            lenv[n_here] = g1s[i] - g0s[i];
            kxv[n_here] = kk[i];
            ++n_here;
          }
        }
      }
    }
    // table slots: a lane's runs follow those of the lower lanes
    const unsigned long long m1 = ballot(n_here >= 1), m2 = ballot(n_here >= 2),
                             m3 = ballot(n_here >= 3), m4 = ballot(n_here >= 4);
    const int at = lanes_below(m1) + lanes_below(m2) + lanes_below(m3) + lanes_below(m4);
    const int tot = lenv[0] + lenv[1] + lenv[2] + lenv[3];
    const int incl = wave_incl_scan(tot);
    int v = incl - tot;
    for (int i = 0; i < 4; ++i) {
      if (i < n_here) {
        W.pre[at + i] = v;
        RunEntry<Real> e;
        e.g0 = g0v[i] - v;  // galaxy slot of virtual candidate index c: e.g0 + c
        if constexpr (kF32) {
          e.rx = float(p[0] - kxv[i] * a.L[0]);
          e.ry = float(p[1] - ky * a.L[1]);
          e.rz = float(p[2] - kz * a.L[2]);
        }
        W.run[at + i] = e;
        v += lenv[i];
      }
    }
    total = uniform_int(__builtin_amdgcn_readlane(incl, kWave - 1));
    const int nrun = __popcll(m1) + __popcll(m2) + __popcll(m3) + __popcll(m4);
    if constexpr (kF32) {
      // the sentinel run after the last one: the lanes of a window past the
      // last candidate map onto the NaN entries after the catalogue
      if (lane == 0) {
        W.pre[nrun] = total;
        RunEntry<Real> e;
        e.g0 = a.sentinel - total;
        e.rx = e.ry = e.rz = 0.0f;
        W.run[nrun] = e;
      }
    }
    // marks of the first span [0, kMarkSpan)
    clear_marks(W);
    v = incl - tot;
    for (int i = 0; i < 4; ++i) {
      if (i < n_here && v < kMarkSpan) set_mark(W, v);
      v += lenv[i];
    }
    if (kF32 && lane == 0 && total < kMarkSpan) set_mark(W, total);
    wave_lds_fence();
    return nrun;
  }

  static __device__ __forceinline__ void clear_marks(Lds& W) {
    const int lane = threadIdx.x % kWave;
    static_assert(kMarkWords == 2 * kWave, "two mark words per lane");
    reinterpret_cast<unsigned long long*>(W.marks)[lane] = 0ull;
    // LDS operations of one wave complete in order; the empty statement keeps
    // the compiler from moving the marks' updates above the clear
    asm volatile("" ::: "memory");
  }
  static __device__ __forceinline__ void set_mark(Lds& W, int c) {
    __hip_atomic_fetch_or(&W.marks[c >> 5], 1u << (c & 31), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_WAVEFRONT);
  }
  // The 64 marks from offset c (a multiple of 64) of the span, wave-uniform.
  static __device__ __forceinline__ unsigned long long window_marks(const Lds& W, int c) {
    const unsigned long long w = reinterpret_cast<const unsigned long long*>(W.marks)[c >> 6];
    return (static_cast<unsigned long long>(uniform_int(int(w >> 32))) << 32) |
           static_cast<unsigned>(uniform_int(int(unsigned(w))));
  }
  // The marks of two adjacent windows from offset c (a multiple of 128) of
  // the span, wave-uniform, in one LDS read.
  static __device__ __forceinline__ void window_marks2(const Lds& W, int c,
                                                       unsigned long long& m0,
                                                       unsigned long long& m1) {
    const uint4 q = reinterpret_cast<const uint4*>(W.marks)[c >> 7];
    m0 = (static_cast<unsigned long long>(uniform_int(int(q.y))) << 32) |
         static_cast<unsigned>(uniform_int(int(q.x)));
    m1 = (static_cast<unsigned long long>(uniform_int(int(q.w))) << 32) |
         static_cast<unsigned>(uniform_int(int(q.z)));
  }
  // Marks of the span starting at mbase, from the run starts in LDS (and the
  // FP32 search's sentinel run).
  static __device__ __forceinline__ void span_marks(Lds& W, int nrun, int mbase) {
    const int lane = threadIdx.x % kWave;
    wave_lds_fence();
    clear_marks(W);
    const int nr = kF32 ? nrun + 1 : nrun;
    for (int r = lane; r < nr; r += kWave) {
      const int c = W.pre[r] - mbase;
      if (c >= 0 && c < kMarkSpan) set_mark(W, c);
    }
    wave_lds_fence();
  }

  // Candidate of each lane in the window [v0, v0 + 64) of the chunk's runs.
  // Lanes past the end: FP32, one of the NaN entries after the catalogue
  // (through the sentinel run, whose start at `total` is marked like the
  // others); FP64, the last candidate again.  Windows come in order:
  // kb is the run holding v0 - 1 on entry (-1 before the first window) and the
  // run holding the window's last candidate on return.  The run starts inside
  // the window are the window's 64 bits of the marks (runs are never empty, so
  // starts are distinct positions), and a lane's run is kb plus the marks at or
  // below its position.  mbase is the first index of the span the marks hold.
  // Windows come in pairs, an even one (v0 a multiple of 128) and the odd one
  // after it, in the same span: the even one reads both windows' marks and
  // leaves the odd one's in nextm.
  template <bool ODD>
  static __device__ __forceinline__ int map_window(Lds& W, int nrun, int total, int v0, int& kb,
                                                   int& mbase, Real ref[3],
                                                   unsigned long long& nextm) {
    const int lane = threadIdx.x % kWave;
    int vc = kF32 ? v0 + lane : min(v0 + lane, total - 1);
    // the window's 64 marks; one test on the common path, where v0 is below
    // both the end and the end of the marked span
    unsigned long long pm = 0;
    if (__builtin_expect(v0 < min(total, mbase + kMarkSpan), 1)) {
      if constexpr (ODD) {
        pm = nextm;
      } else {
        window_marks2(W, v0 - mbase, pm, nextm);
      }
    } else if (v0 < total) {
      // a new span starts at an even window (spans hold 64 windows), so an
      // odd window below the end is always in its even window's span
      mbase = v0 & ~(kMarkSpan - 1);
      span_marks(W, nrun, mbase);
      if constexpr (ODD) {
        pm = window_marks(W, v0 - mbase);
      } else {
        window_marks2(W, v0 - mbase, pm, nextm);
      }
    } else if constexpr (kF32) {
      // a window past the end: every lane on the sentinel run's entries
      kb = nrun;
      vc = total + lane;
    }
    // the lane's own mark as the count's starting value (the mask itself
    // selects it, one instruction)
    int f;
    asm("v_cndmask_b32_e64 %0, 0, 1, %1" : "=v"(f) : "s"(pm));
    const int k = kb + __builtin_amdgcn_mbcnt_hi(unsigned(pm >> 32),
                                                 __builtin_amdgcn_mbcnt_lo(unsigned(pm), f));
    kb += __popcll(pm);
    const RunEntry<Real> e = W.run[k];
    if constexpr (kF32) {
      ref[0] = e.rx;
      ref[1] = e.ry;
      ref[2] = e.rz;
    }
    return e.g0 + vc;
  }

  // Galaxy j of the cell-ordered catalogue through a 32-bit byte offset from
  // the scalar base address (the catalogue is below 4 GiB: n < 2^27).
  static __device__ __forceinline__ V load_galaxy(const V* __restrict__ pos4, int j) {
    return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(pos4) +
                                       (unsigned(j) * unsigned(sizeof(V))));
  }

  // Unit separation (rotated into the line-of-sight frame) of a ring entry.
  template <bool ROT>
  static __device__ __forceinline__ void unit(const Primary& P, const V& e, Real& ux, Real& uy,
                                              Real& uz) {
    Real inv;
    if constexpr (kF32) {
      inv = __builtin_amdgcn_rsqf(fma_r(e.z, e.z, fma_r(e.y, e.y, e.x * e.x)));
    } else {
      inv = 1.0 / sqrt(e.x * e.x + e.y * e.y + e.z * e.z);
    }
    const Real dx = e.x * inv, dy = e.y * inv, dz = e.z * inv;
    if constexpr (ROT) {
      const Real* R = P.Rm;
      ux = R[0] * dx + R[1] * dy + R[2] * dz;
      uy = R[3] * dx + R[4] * dy + R[5] * dz;
      uz = R[6] * dx + R[7] * dy + R[8] * dz;
    } else {
      ux = dx;
      uy = dy;
      uz = dz;
    }
  }

  // One search of shell b over the annulus [r0, r1): every accepted pair is
  // appended to the LDS ring as (separation, weight or index), and every full
  // wave of pairs is handed to consume(entry, index, valid) (one pair per
  // lane; the index only with SPILL); the
  // remainder at the end.  The position loads of the next window are issued
  // before the current window is binned.
  template <bool MINIMG, bool SPILL, typename Consume>
  static __device__ __forceinline__ unsigned search_shell(const PairArgs& a, Lds& W,
                                                          const V* __restrict__ pos4,
                                                          const Primary& P, int b, double r0,
                                                          double r1, Consume&& consume) {
    const int lane = threadIdx.x % kWave;
    const int* __restrict__ cs = a.cell_start;
    const double* p = P.p;
    int c0[3] = {0, 0, 0}, c1[3] = {0, 0, 0};
    for (int ax = 1; ax < 3; ++ax) {
      if (a.tight[ax]) {
        c0[ax] = 0;
        c1[ax] = a.nc[ax] - 1;
      } else {
        c0[ax] = cell_floor(p[ax] - r1, a.lo[ax], a.inv_s[ax]);
        c1[ax] = cell_floor(p[ax] + r1, a.lo[ax], a.inv_s[ax]);
        if (!a.periodic) {
          c0[ax] = min(max(c0[ax], 0), a.nc[ax] - 1);
          c1[ax] = min(max(c1[ax], 0), a.nc[ax] - 1);
        }
      }
    }
    // uniform per shell: kept in scalar registers across the window loops
    for (int ax = 1; ax < 3; ++ax) c0[ax] = uniform_int(c0[ax]);
    const int nyr = uniform_int(c1[1] - c0[1] + 1), nzr = uniform_int(c1[2] - c0[2] + 1);
    const int nrows = nyr * nzr;
    const float inv_nyr = uniform_real(1.0f / float(nyr));
    const double r0sq = uniform_double(r0 * r0), r1sq = uniform_double(r1 * r1);
    float lo2 = 0.0f, hi2 = 0.0f;
    if constexpr (kF32) {
      lo2 = a.r2_lo[b];
      hi2 = a.r2_hi[b];
    }
    int cnt = 0;
    unsigned accepted = 0;
    // Wave priority: the search (run tables, window mapping, binning) is a
    // chain of dependent LDS reads, position loads and compares, the
    // accumulation independent arithmetic; a search at priority 1 over
    // accumulations at 0 issues first when both are ready on a SIMD, and
    // its next loads start sooner (the adjoint also raises the mapping and
    // load issue to 2 over its binning).
    __builtin_amdgcn_s_setprio(1);
    for (int rb = 0; rb < nrows; rb += kWave) {
      int total = 0;
      const int nrun = build_runs(a, cs, P, r0sq, r1sq, c0, nyr, inv_nyr, rb, nrows, W, total);
      if (total == 0) continue;
      int kb = -1, mbase = 0;
      // bin one window and append its accepted pairs to the ring; consume a
      // full wave of pairs when there is one
      auto step = [&](const V& q, const Real* rref, int j, int v0) {
        Real d[3];
        bool acc;
        unsigned long long m;
        if constexpr (kF32) {
          const float* ref = MINIMG ? P.pref : rref;
          float dx = __fsub_rn(q.x, ref[0]), dy = __fsub_rn(q.y, ref[1]),
                dz = __fsub_rn(q.z, ref[2]);
          if constexpr (MINIMG) {
            dx = fma_r(-P.L[0], __builtin_rintf(__fmul_rn(dx, P.invL[0])), dx);
            dy = fma_r(-P.L[1], __builtin_rintf(__fmul_rn(dy, P.invL[1])), dy);
            dz = fma_r(-P.L[2], __builtin_rintf(__fmul_rn(dz, P.invL[2])), dz);
          }
          const float r2 = fma_r(dz, dz, fma_r(dy, dy, __fmul_rn(dx, dx)));
          d[0] = dx;
          d[1] = dy;
          d[2] = dz;
          // no short circuit: no branches; lanes past the end hold NaN and
          // fail both tests.  The mask from the two compares' own lane masks
          // (a ballot of their conjunction would first materialise it)
          acc = (r2 > lo2) & (r2 < hi2);
          m = ballot(r2 > lo2) & ballot(r2 < hi2);
        } else {
          double r2;
          const int bin = P.bin64.classify(q, P.p, d, r2);
          acc = (v0 + lane < total) && bin == b;
          m = ballot(acc);
        }
        if (acc) {
          V ent;
          ent.x = d[0];
          ent.y = d[1];
          ent.z = d[2];
          if constexpr (ADJOINT) {
            ent.w = pack_index(j, Real(0));
          } else {
            ent.w = q.w;
          }
          const int slot = cnt + lanes_below(m);  // below kRing: cnt < kWave here
          W.ring[slot] = ent;
          if constexpr (SPILL) W.ring_j[slot] = j;
        }
        const int got = __popcll(m);
        cnt += got;
        accepted += unsigned(got);
        if (cnt >= kWave) {
          // the first wave of pairs out, the rest (fewer than kWave) moved to
          // the front, so that slots need no wrap-around
          wave_lds_fence();
          const V ent = W.ring[lane];
          const V rest = W.ring[kWave + lane];
          int jj = 0;
          if constexpr (SPILL) {
            jj = W.ring_j[lane];
            W.ring_j[lane] = W.ring_j[kWave + lane];
          }
          W.ring[lane] = rest;
          __builtin_amdgcn_s_setprio(0);
          consume(ent, jj, true);
          __builtin_amdgcn_s_setprio(1);
          cnt -= kWave;
        }
      };
      // two windows in flight: while one is binned the other's loads are
      // outstanding (the buffers alternate, so no copy waits on a load).
      // Windows past the end accept nothing (FP32: every lane on a NaN
      // entry; FP64: on the last candidate, rejected by the index test).
      Real refa[3] = {P.pref[0], P.pref[1], P.pref[2]};
      Real refb[3] = {P.pref[0], P.pref[1], P.pref[2]};
      unsigned long long nextm = 0;
      int ja = map_window<false>(W, nrun, total, 0, kb, mbase, refa, nextm);
      V qa = load_galaxy(pos4, ja);
      for (int v0 = 0; v0 < total; v0 += 2 * kWave) {
        if constexpr (ADJOINT) __builtin_amdgcn_s_setprio(2);
        const int jb = map_window<true>(W, nrun, total, v0 + kWave, kb, mbase, refb, nextm);
        const V qb = load_galaxy(pos4, jb);
        if constexpr (ADJOINT) __builtin_amdgcn_s_setprio(1);
        step(qa, refa, ja, v0);
        if constexpr (ADJOINT) __builtin_amdgcn_s_setprio(2);
        ja = map_window<false>(W, nrun, total, v0 + 2 * kWave, kb, mbase, refa, nextm);
        qa = load_galaxy(pos4, ja);
        if constexpr (ADJOINT) __builtin_amdgcn_s_setprio(1);
        step(qb, refb, jb, v0 + kWave);
      }
      wave_lds_fence();
    }
    __builtin_amdgcn_s_setprio(0);
    if (cnt > 0) {
      wave_lds_fence();
      V ent;
      int jj = 0;
      if (lane < cnt) {
        ent = W.ring[lane];
        if constexpr (SPILL) jj = W.ring_j[lane];
      } else {
        ent.x = Real(0);
        ent.y = Real(0);
        ent.z = Real(1);
        ent.w = ADJOINT ? pack_index(0, Real(0)) : Real(0);
      }
      consume(ent, jj, lane < cnt);
      wave_lds_fence();
    }
    return accepted;
  }

  // Separation of secondary j from the primary exactly as the search forms
  // it (same reference point or minimum image, same rounding).
  template <bool MINIMG>
  static __device__ __forceinline__ void separation(const PairArgs& a, const Primary& P,
                                                    const V& q, Real d[3]) {
    if constexpr (kF32) {
      float ref[3] = {P.pref[0], P.pref[1], P.pref[2]};
      if (!MINIMG && a.periodic) {
        // the run's image shift: the unique k with |q - p + k L| < L / 2
        const double qq[3] = {double(q.x), double(q.y), double(q.z)};
        // |q - p + k L| stays far from L / 2 on a non-tight axis, so the
        // product with 1/L rounds to the same k as the quotient would
        for (int c = 0; c < 3; ++c) {
          const double k = -rint((qq[c] - P.p[c]) * P.invLd[c]);
          ref[c] = float(P.p[c] - k * a.L[c]);
        }
      }
      float dx = __fsub_rn(q.x, ref[0]), dy = __fsub_rn(q.y, ref[1]), dz = __fsub_rn(q.z, ref[2]);
      if constexpr (MINIMG) {
        dx = fma_r(-P.L[0], __builtin_rintf(__fmul_rn(dx, P.invL[0])), dx);
        dy = fma_r(-P.L[1], __builtin_rintf(__fmul_rn(dy, P.invL[1])), dy);
        dz = fma_r(-P.L[2], __builtin_rintf(__fmul_rn(dz, P.invL[2])), dz);
      }
      d[0] = dx;
      d[1] = dy;
      d[2] = dz;
    } else {
      double r2;
      P.bin64.classify(q, P.p, d, r2);
    }
  }

  // Stream `count` spilled secondaries of a shell, one per lane, into
  // body(unit vector, weight, index, valid).  Two batches alternate so that
  // the next batch's gathers and the batch after that's indices are in flight
  // while one batch is used.
  template <bool ROT, bool MINIMG, typename Body>
  static __device__ __forceinline__ void replay_all(const PairArgs& a,
                                                    const V* __restrict__ pos4,
                                                    const Primary& P, const int* __restrict__ sp,
                                                    int count, Body&& body) {
    if (count <= 0) return;
    const int lane = threadIdx.x % kWave;
    const int last = count - 1;
    auto use = [&](const V& q, int j, int base) {
      const bool valid = base + lane < count;
      Real d[3];
      separation<MINIMG>(a, P, q, d);
      V e;
      e.x = valid ? d[0] : Real(0);
      e.y = valid ? d[1] : Real(0);
      e.z = valid ? d[2] : Real(1);
      Real ux, uy, uz;
      unit<ROT>(P, e, ux, uy, uz);
      body(ux, uy, uz, valid ? q.w : Real(0), j, valid);
    };
    int ja = sp[min(lane, last)];
    int jb = sp[min(kWave + lane, last)];
    V qa = load_galaxy(pos4, ja);
    for (int base = 0; base < count; base += 2 * kWave) {
      const V qb = load_galaxy(pos4, jb);
      const int jn = sp[min(base + 2 * kWave + lane, last)];
      use(qa, ja, base);
      ja = jn;
      qa = load_galaxy(pos4, ja);
      const int jbb = jb;
      jb = sp[min(base + 3 * kWave + lane, last)];
      use(qb, jbb, base + kWave);
    }
  }

  template <bool ROT, bool MINIMG, typename Body>
  static __device__ __forceinline__ void replay(const PairArgs& a, const V* __restrict__ pos4,
                                                const Primary& P, const int* __restrict__ sp,
                                                int count, Body&& body) {
    replay_all<ROT, MINIMG>(a, pos4, P, sp, count,
                            [&](Real ux, Real uy, Real uz, Real w, int, bool) {
                              body(ux, uy, uz, w);
                            });
  }

  // All chunks (forward) or the adjoint of shell b, with the line-of-sight
  // rotation and the minimum-image mode fixed at compile time.  With several
  // chunks, the first search also writes the shell's secondaries to the
  // wave's spill list, and the later chunks replay it instead of searching
  // again (unless it overflowed).
  template <bool ROT, bool MINIMG>
  static __device__ __forceinline__ unsigned shell(const PairArgs& a, Lds& W,
                                                   const V* __restrict__ pos4, const Primary& P,
                                                   int b, double r0, double r1, long long row,
                                                   double w_prim, int* __restrict__ sp) {
    const int lane = threadIdx.x % kWave;
    unsigned got = 0;
    if constexpr (!ADJOINT) {
      using CL = typename Chunks<Real, BASIS>::type;
      constexpr bool kMulti = n_chunks(CL{}) > 1;
      const int cap = a.spill_cap;
      bool first = true;
      bool replayable = false;
      for_each_chunk(CL{}, [&](auto* tag) {
        using Chunk = std::remove_pointer_t<decltype(tag)>;
        Chunk ch;
        ch.zero();
        auto add = [&](const V& e) {
          Real ux, uy, uz;
          unit<ROT>(P, e, ux, uy, uz);
          ch.add(ux, uy, uz, e.w);
        };
        if (first && kMulti && cap > 0) {
          int nsp = 0;
          got = search_shell<MINIMG, true>(a, W, pos4, P, b, r0, r1,
                                           [&](const V& e, int j, bool valid) {
                                             if (valid && nsp + lane < cap) sp[nsp + lane] = j;
                                             nsp += __popcll(ballot(valid));
                                             add(e);
                                           });
          replayable = got <= unsigned(cap);
        } else if (!first && replayable) {
          replay<ROT, MINIMG>(a, pos4, P, sp, int(got), [&](Real ux, Real uy, Real uz, Real w) {
            ch.add(ux, uy, uz, w);
          });
        } else {
          const unsigned g = search_shell<MINIMG, false>(a, W, pos4, P, b, r0, r1,
                                                         [&](const V& e, int, bool) { add(e); });
          if (first) got = g;
        }
        first = false;
        reduce_store(W, ch);
      });
      wave_lds_fence();
      if constexpr (BASIS == kBasisDeg) {
        store_deg(a, W, b, row);
      } else {
        convert(a, W, b, row);
      }
      wave_lds_fence();
    } else {
      if constexpr (kSpinT) {
        // FP32: Chebyshev-basis coefficients, formed from the H row once per
        // shell and staged through LDS (broadcast reads) into vector
        // registers; FP32 polynomial and FP32 atomics
        shell_coefficients(a, W, row, b);
        wave_lds_fence();
        SpinTPoly poly;
        poly.load(W.M);
        wave_lds_fence();
        const float wp = float(w_prim);
        // Each wave of terms goes to the LDS buffer and the buffer to the
        // atomics every kOutBuf / kWave waves: a wait for the candidate loads
        // then finds atomics outstanding (and has to wait for them, vmcnt
        // counting both) once per flush instead of after every wave of pairs.
        // A full buffer is flushed before the next wave's polynomial, which
        // then runs while the atomics complete.
        int nout = 0;
        got = search_shell<MINIMG, false>(
            a, W, pos4, P, b, r0, r1, [&](const V& e, int, bool valid) {
              if (nout == kOutBuf) {
                flush_terms(a, W, nout);
                nout = 0;
              }
              Real ux, uy, uz;
              unit<ROT>(P, e, ux, uy, uz);
              const float v = poly.eval(ux, uy, uz);
              W.out[nout + lane_here()] =
                  make_int2(valid ? unpack_index(e.w) : -1, __float_as_int(wp * v));
              nout += kWave;
            });
        if (nout > 0) flush_terms(a, W, nout);
      } else {
        // the shell's coefficients, read through the scalar cache (uniform)
        const CoefPtr gc = (CoefPtr)(a.gcoef + (row * a.nbins + b) * kTerms);
        got = search_shell<MINIMG, false>(a, W, pos4, P, b, r0, r1,
                                          [&](const V& e, int, bool valid) {
                                            Real ux, uy, uz;
                                            unit<ROT>(P, e, ux, uy, uz);
                                            scatter_one(a, gc, ux, uy, uz, unpack_index(e.w),
                                                        valid, w_prim);
                                          });
      }
      wave_lds_fence();
    }
    return got;
  }

  static __device__ __forceinline__ void run(const PairArgs& a) {
    extern __shared__ char smem_raw[];
    Lds* lds = reinterpret_cast<Lds*>(smem_raw);
    // wave index made uniform so that per-wave pointers live in scalar registers
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    Lds& W = lds[wid];
    const V* __restrict__ pos4 = static_cast<const V*>(a.pos4);
    const long long NP = min(a.p_count, (long long)(*a.nprim) - a.p_begin);
    const int nb = a.nbins;
    const double margin = a.rmax_search - a.rmax;
    // this wave's spill list (multi-chunk bases)
    int* sp = a.spill + size_t(blockIdx.x * kWavesPerBlock + wid) * size_t(a.spill_cap);
    unsigned long long my_pairs = 0;

    // The pair-block's primaries (in cell order) are split into kQueues
    // contiguous shares, one per XCD: a wave takes primaries from its own XCD's
    // share first, so the candidates of the primaries an XCD works on at once
    // are neighbours in its L2, then helps the other shares.
    const int xcc = int(blockIdx.x % kQueues);
    const long long share = (NP + kQueues - 1) / kQueues;
    int qx = 0;  // shares visited
    while (true) {
      long long qi = 0;
      bool found = false;
      while (qx < kQueues) {
        const int x = (xcc + qx) % kQueues;
        const long long lo = x * share, hi = min(NP, lo + share);
        int t = 0;
        if (lane == 0) t = atomicAdd(a.queue + x * kQueueStride, 1);
        t = uniform_int(__shfl(t, 0));
        if (lo + t < hi) {
          long long tt = t;
          if constexpr (ADJOINT) {
            // the adjoint hands out its share in kAdjStripes interleaved
            // stripes: the waves of an XCD then work on primaries in
            // kAdjStripes places at once, and their atomic adds into the
            // secondaries' gradient meet on the same cache lines far less
            // often than when all of them work on neighbouring primaries
            const long long q = (hi - lo) / kAdjStripes;
            if (tt < kAdjStripes * q) tt = (tt % kAdjStripes) * q + tt / kAdjStripes;
          }
          qi = lo + tt;
          found = true;
          break;
        }
        ++qx;
      }
      if (!found) break;
      const int slot = uniform_int(a.plist[a.p_begin + qi]);
      const V pv = pos4[slot];
      Primary P;
      P.p[0] = uniform_double(double(pv.x));
      P.p[1] = uniform_double(double(pv.y));
      P.p[2] = uniform_double(double(pv.z));
      const long long row = qi;  // row of A within this pair-block
      if (!(isfinite(P.p[0]) && isfinite(P.p[1]) && isfinite(P.p[2]))) {
        // no separation from a non-finite position is accepted: no neighbours,
        // a zero row of sums (forward), no secondary terms (adjoint)
        if constexpr (!ADJOINT) {
          double* out = a.A + row * a.lay.W;
          for (int k = lane; k < a.lay.W; k += kWave) out[k] = 0.0;
        }
        continue;
      }
      if constexpr (kRot) {
        frame(a, P);
        // uniform per primary: held in scalar registers
        for (int i = 0; i < 9; ++i) P.Rm[i] = uniform_real(P.Rm[i]);
      }
      for (int c = 0; c < 3; ++c) {
        P.L[c] = uniform_real(Real(a.L[c]));
        P.invL[c] = uniform_real(Real(1.0 / a.L[c]));
        P.pref[c] = uniform_real(Real(P.p[c]));
        P.invLd[c] = 1.0 / a.L[c];
        P.prel[c] = uniform_double((P.p[c] - a.lo[c]) * a.inv_s[c]);
        P.sf[c] = uniform_real(float(a.s[c]));
        P.bin64.L[c] = a.L[c];
      }
      // FP64 always measures from the primary with the minimum image (the
      // plain definition); FP32 only where a search window can wrap onto
      // itself (kMin)
      P.minimg = kF32 ? kMin : (a.periodic != 0);
      P.bin64.minimg = P.minimg;
      P.bin64.r2max = a.rmax * a.rmax;
      P.bin64.nbins = nb;
      P.bin64.rmax = a.rmax;

      double w_prim = 0.0;
      if constexpr (ADJOINT) w_prim = a.wsort[slot];
      if constexpr (kSpinT) primary_term(a, row, slot);

      for (int bb = 0; bb < nb; ++bb) {
        const int b = uniform_int(bb);  // in a scalar register throughout the shell
        // annulus of shell b, widened by the search margin on both sides
        const double r0 = uniform_double(fmax(0.0, b * a.rmax / nb - margin));
        const double r1 =
            uniform_double((b + 1 == nb) ? a.rmax_search : (b + 1) * a.rmax / nb + margin);
        my_pairs += shell<kRot, kF32 && kMin>(a, W, pos4, P, b, r0, r1, row, w_prim, sp);
      }
    }

    if (lane == 0 && my_pairs) atomicAdd(a.pairs, my_pairs);
  }

  // Line-of-sight frame of the primary: the Rodrigues rotation taking the
  // direction from the observer to +z (the identity for a primary on the
  // observer, which has no line of sight).
  static __device__ __forceinline__ void frame(const PairArgs& a, Primary& P) {
    for (int i = 0; i < 9; ++i) P.Rm[i] = Real((i % 4 == 0) ? 1 : 0);
    const double* p = P.p;
    double n[3] = {p[0] - a.obs[0], p[1] - a.obs[1], p[2] - a.obs[2]};
    const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (!(nn > 0.0)) return;
    for (int c = 0; c < 3; ++c) n[c] /= nn;
    const double c = n[2];
    if (c < -1.0 + 1e-12) {
      P.Rm[4] = Real(-1);
      P.Rm[8] = Real(-1);
      return;
    }
    const double vx = n[1], vy = -n[0];  // v = n x z
    const double f = 1.0 / (1.0 + c);
    const double vv = vx * vx + vy * vy;
    // R = I + [v]x + (v v^T - |v|^2 I) / (1 + c), v_z = 0
    P.Rm[0] = Real(1.0 + (vx * vx - vv) * f);
    P.Rm[1] = Real(vx * vy * f);
    P.Rm[2] = Real(vy);
    P.Rm[3] = Real(vx * vy * f);
    P.Rm[4] = Real(1.0 + (vy * vy - vv) * f);
    P.Rm[5] = Real(-vx);
    P.Rm[6] = Real(-vy);
    P.Rm[7] = Real(vx);
    P.Rm[8] = Real(1.0 - vv * f);
  }

  // Wave sums of a chunk's accumulators into W.M, four at a time: one fold
  // across rows first (each lane of row r then holds four lanes' worth of
  // value r), then row sums by DPP leave the four totals in rows 0..3, and
  // every lane stores its row's total (16 lanes write the same value): ten
  // instructions per four values instead of 22 with the row sums first.
  template <class Chunk>
  static __device__ __forceinline__ void reduce_store(Lds& W, Chunk& ch) {
    constexpr int NT = Chunk::NT;
    constexpr int kJunk = kTermsCart;  // slot that absorbs padding in the last group
    const int lane = lane_here();
    const int row = lane >> 4;
    const bool ge1 = row >= 1, ge2 = row >= 2, ge3 = row >= 3;
    const bool leader = (lane & 15) == 0;  // one store per row
    static_for<(NT + 3) / 4>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      constexpr int i0 = 4 * g, i1 = 4 * g + 1, i2 = 4 * g + 2, i3 = 4 * g + 3;
      Real e = Real(0), b = Real(0), f = Real(0);
      if constexpr (i1 < NT) e = ch.acc[i1];
      if constexpr (i2 < NT) b = ch.acc[i2];
      if constexpr (i3 < NT) f = ch.acc[i3];
      const Real tot = row_sum(fold4(ch.acc[i0], e, b, f));
      constexpr int ta = Chunk::term_of(i0);
      constexpr int te = (i1 < NT) ? Chunk::term_of(i1) : kJunk;
      constexpr int tb = (i2 < NT) ? Chunk::term_of(i2) : kJunk;
      constexpr int tf = (i3 < NT) ? Chunk::term_of(i3) : kJunk;
      int t;
      if constexpr (te == ta + 1 && tb == ta + 2 && tf == ta + 3) {
        t = ta + row;
      } else {
        t = ta;
        t = ge1 ? te : t;
        t = ge2 ? tb : t;
        t = ge3 ? tf : t;
      }
      if (leader) W.M[t] = tot;
    });
  }

  // Convert the shell's monomial sums in W.M to a_lm (FP64) and write them.
  static __device__ __forceinline__ void convert(const PairArgs& a, const Lds& W, int b,
                                                 long long row) {
    const int lane = threadIdx.x % kWave;
    const ConvTable& t = g_conv[conv_table_of(BASIS)];
    const RowLayout& L = a.lay;
    double* out = a.A + row * L.W;
    for (int o = lane; o < kOutPerBin; o += kWave) {
      const int l = t.out_l[o];
      if (l > L.lmax) continue;
      const int m = t.out_m[o], part = t.out_part[o];
      double s = 0.0;
      for (int e = t.rowptr[o]; e < t.rowptr[o + 1]; ++e)
        s = __builtin_fma(t.coef[e], double(W.M[t.term[e]]), s);
      out[L.off[m] + part * L.d[m] + L.pos(m, l, b)] = s;
    }
  }

  // The shell's degenerate-triangle sums D_n, n <= 2 lmax, into the row of the
  // pair-block (FP64, [shell][n]).
  static __device__ __forceinline__ void store_deg(const PairArgs& a, const Lds& W, int b,
                                                   long long row) {
    const int lane = threadIdx.x % kWave;
    const int nd = 2 * a.lmax + 1;
    if (lane < nd) a.A[row * a.lay.W + b * nd + lane] = double(W.M[lane]);
  }

  // FP32 adjoint, per primary: its term as a primary, Re(a^T H) / 2 in FP64
  // over its A and H rows (the imaginary half of each m >= 1 block with a
  // minus sign), added to its FP64 gradient entry (one wave per primary).
  static __device__ __forceinline__ void primary_term(const PairArgs& a, long long row, int slot) {
    const int lane = threadIdx.x % kWave;
    const double* x = a.A + row * a.lay.W;
    const double* h = a.H + row * a.lay.W;
    double s = 0.0;
    for (int m = 0; m <= a.lay.lmax; ++m) {
      const int off = a.lay.off[m], wm = a.lay.wm[m], dm = a.lay.d[m];
      for (int j = lane; j < wm; j += kWave) {
        const double v = x[off + j] * h[off + j];
        s += (m > 0 && j >= dm) ? -v : v;
      }
    }
    s = wave_sum(s);
    if (lane == kWave - 1) a.grad_w[slot] += 0.5 * s;
  }

  // FP32 adjoint, per primary and shell b: the 121 coefficients of the
  // polynomial in (x - i y)^m T_n(z), g_t = sum over the spin-Chebyshev
  // table's entries (t, lm) of Re c Re H_lm(b) - Im c Im H_lm(b), formed in
  // FP64 and stored to LDS as FP32 (one or two terms a lane).  The shell's
  // 121 H values are first staged in the table's output order, the
  // imaginary parts negated and l > l_max as zero (one load a lane, all in
  // flight together), in the ring's LDS, which is empty between shells.
  static __device__ __forceinline__ void shell_coefficients(const PairArgs& a, Lds& W,
                                                            long long row, int b) {
    const int lane = threadIdx.x % kWave;
    const double* h = a.H + row * a.lay.W;
    const ConvTable& t = g_conv[G3PCF_BASIS_SPIN_T];
    double* hs = reinterpret_cast<double*>(W.ring);
    static_assert(sizeof(W.ring) >= kTermsSpin * sizeof(double), "staging fits the ring");
    for (int o = lane; o < kTermsSpin; o += kWave) {
      const int l = t.out_l[o], m = t.out_m[o];
      const bool im = t.out_part[o] != 0;
      double v = 0.0;
      if (l <= a.lay.lmax) {
        v = h[a.lay.off[m] + a.lay.pos(m, l, b) + (im ? a.lay.d[m] : 0)];
        if (im) v = -v;
      }
      hs[o] = v;
    }
    wave_lds_fence();
    for (int term = lane; term < kTermsSpin; term += kWave) {
      double s = 0.0;
      const int e1 = t.trowptr[term + 1];
#pragma unroll 4
      for (int e = t.trowptr[term]; e < e1; ++e) s = __builtin_fma(t.tcoef[e], hs[t.tout[e]], s);
      W.M[term] = float(s);
    }
  }

  // The buffered secondary terms of the FP32 adjoint into the FP32
  // gradient (n: a multiple of the wave size; index -1 marks an empty lane).
  static __device__ __forceinline__ void flush_terms(const PairArgs& a, Lds& W, int n) {
    wave_lds_fence();
    for (int k = 0; k < n; k += kWave) {
      const int2 o = W.out[k + lane_here()];
      if (o.x >= 0) unsafeAtomicAdd(&a.grad_w32[o.x], __int_as_float(o.y));
    }
    wave_lds_fence();
  }

  // FP64 adjoint for one pair per lane: the full polynomial sum_t g_t
  // mono_t(u) in the forward's monomial basis, in FP64 (its coefficients
  // cancel strongly at l = 10).  The coefficients are the same for every
  // lane, so they are read into scalar registers.
  static __device__ __forceinline__ void scatter_one(const PairArgs& a, CoefPtr gc, Real ux,
                                                     Real uy, Real uz, int j, bool valid,
                                                     double w_prim) {
    static_assert(!kF32, "the FP32 adjoint evaluates SpinTPoly");
    using Poly = std::conditional_t<BASIS == G3PCF_BASIS_SPIN, SpinChunk<double, 0, kDeg>,
                                    CartChunk<double, (1u << (kDeg + 1)) - 1>>;
    const double v = Poly::poly(double(ux), double(uy), double(uz), [&](int t) { return gc[t]; });
    if (valid) unsafeAtomicAdd(&a.grad_w[j], w_prim * v);
  }
};

template <typename Real, int BASIS, bool ADJOINT, bool ROT, bool MIN>
__global__ __launch_bounds__(kWave* kWavesPerBlock)
    __attribute__((amdgpu_waves_per_eu(Occ<Real, BASIS, ADJOINT>::value))) void k_pairs(
        PairArgs a) {
  PairKernel<Real, BASIS, ADJOINT, ROT, MIN>::run(a);
}

__global__ void k_zero_queue(int* q) {
  if (threadIdx.x < kQueues) q[threadIdx.x * kQueueStride] = 0;
}

template <typename Real, int BASIS, bool ADJOINT, bool ROT, bool MIN>
hipError_t launch_mode(const PairArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(kWave), 0, st, a.queue);
  const long long want = (a.p_count + kWavesPerBlock - 1) / kWavesPerBlock;
  const unsigned blocks = unsigned(std::min<long long>(want, kPairWaves / kWavesPerBlock));
  const size_t lds =
      sizeof(typename PairKernel<Real, BASIS, ADJOINT, ROT, MIN>::Lds) * kWavesPerBlock;
  hipLaunchKernelGGL((k_pairs<Real, BASIS, ADJOINT, ROT, MIN>), dim3(blocks > 0 ? blocks : 1),
                     dim3(kWave * kWavesPerBlock), lds, st, a);
  return hipGetLastError();
}

// The kernel of the problem's mode: rotation (observer line of sight) and,
// for FP32, the minimum image (FP64 always applies it on a periodic box).
template <typename Real, int BASIS, bool ADJOINT>
hipError_t launch_one(const PairArgs& a, hipStream_t st) {
  const bool rot = a.los == G3PCF_LOS_OBSERVER;
  if constexpr (std::is_same<Real, float>::value) {
    const bool mi = a.periodic && (a.tight[0] || a.tight[1] || a.tight[2]);
    if (rot)
      return mi ? launch_mode<Real, BASIS, ADJOINT, true, true>(a, st)
                : launch_mode<Real, BASIS, ADJOINT, true, false>(a, st);
    return mi ? launch_mode<Real, BASIS, ADJOINT, false, true>(a, st)
              : launch_mode<Real, BASIS, ADJOINT, false, false>(a, st);
  } else {
    return rot ? launch_mode<Real, BASIS, ADJOINT, true, false>(a, st)
               : launch_mode<Real, BASIS, ADJOINT, false, false>(a, st);
  }
}

}  // namespace

hipError_t launch_pair_forward(const PairArgs& a, int fp64, int basis, hipStream_t st) {
  if (fp64)
    return basis == G3PCF_BASIS_SPIN ? launch_one<double, G3PCF_BASIS_SPIN, false>(a, st)
                                     : launch_one<double, G3PCF_BASIS_CARTESIAN, false>(a, st);
  return basis == G3PCF_BASIS_SPIN ? launch_one<float, G3PCF_BASIS_SPIN, false>(a, st)
                                   : launch_one<float, G3PCF_BASIS_CARTESIAN, false>(a, st);
}

hipError_t launch_pair_distinct(const PairArgs& a, int fp64, hipStream_t st) {
  return fp64 ? launch_one<double, kBasisDeg, false>(a, st)
              : launch_one<float, kBasisDeg, false>(a, st);
}

hipError_t launch_pair_adjoint(const PairArgs& a, int fp64, int basis, hipStream_t st) {
  if (fp64)
    return basis == G3PCF_BASIS_SPIN ? launch_one<double, G3PCF_BASIS_SPIN, true>(a, st)
                                     : launch_one<double, G3PCF_BASIS_CARTESIAN, true>(a, st);
  // The per-pair polynomial represents sum_lm H_lm conj(Y_lm(u)) whatever
  // monomial basis the forward pass accumulated in: the FP32 adjoint always
  // evaluates it in the spin-Chebyshev basis (coefficients from that table).
  return launch_one<float, G3PCF_BASIS_SPIN, true>(a, st);
}

}  // namespace g3
