// The zeta stage: sum over primaries of w_i a_lm(b1) conj(a_l'm(b2)).
//
// The paper adds the per-primary products a_lm(r1) a*_l'm(r2) (Sec. 3.1) and
// combines per-thread partial multipoles at the end of the loop over primaries
// (single-node optimisations section).  Here the per-primary coefficients of a
// block of K primaries are the rows of A, and for every m the block's
// contribution is a Gram product on the matrix cores:
//   B_m = [Re A^m | Im A^m]  (K x W_m),   C_m = (diag(w) B_m)^T B_m,
//   Re zeta^m = C_pp + C_qq,   Im zeta^m = C_qp - C_pq.
// For m = 0 every a_l0 is real and B_0 = Re A^0.  The blocks' C_m (FP32 or
// FP64 accumulation on the matrix cores) are added into zeta in FP64, in
// block order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace g3 {

namespace {

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ long long valid_rows(const ZetaArgs& z) {
  // primaries in the pair-block, then rows of this sub-block
  const long long in_block = (long long)(*z.nprim) - z.row_begin;
  long long kv = in_block - z.sub_begin;
  if (kv > z.K) kv = z.K;
  return kv < 0 ? 0 : kv;
}

// ---- FP32 / FP64: one workgroup per (m, 64 x 64 macro tile of C_m on or
// above the diagonal, block of 4096 primaries).  Each step stages 32 rows of
// the two column ranges in LDS (weights applied to the left operand, FP64 rows
// converted to the working precision on the way), and each wave accumulates a
// 32 x 32 quadrant as 2 x 2 MFMA tiles over the block's rows.  The next step's
// rows are loaded into registers while the current step is multiplied.  In
// FP32 the MFMA accumulators are added into FP64 ones every 512 rows, so the
// block's partial is FP64 like the sum across blocks.
constexpr int kMT = 64;     // macro tile
constexpr int kKS = 32;     // rows per step
constexpr int kFlush = 512; // rows per FP32 accumulation before the FP64 sum

struct MDims {
  int nm;
  int W[kDeg + 1];
  int off[kDeg + 1];
  int cw[kDeg + 2];       // offsets of each C_m in a partial
  int mt[kDeg + 2];       // cumulative macro tiles on or above the diagonal
  int csize;
};

MDims make_mdims(const RowLayout& L) {
  MDims d{};
  d.nm = L.lmax + 1;
  int cw = 0, mt = 0;
  for (int m = 0; m < d.nm; ++m) {
    d.W[m] = L.wm[m];
    d.off[m] = L.off[m];
    d.cw[m] = cw;
    d.mt[m] = mt;
    cw += L.wm[m] * L.wm[m];
    const int t = (L.wm[m] + kMT - 1) / kMT;
    mt += t * (t + 1) / 2;
  }
  d.cw[d.nm] = cw;
  d.mt[d.nm] = mt;
  d.csize = cw;
  return d;
}

__device__ __forceinline__ void macro_tile_of(const MDims& d, int t, int& m, int& ti, int& tj) {
  m = 0;
  while (m + 1 < d.nm && t >= d.mt[m + 1]) ++m;
  int r = t - d.mt[m];
  const int nt = (d.W[m] + kMT - 1) / kMT;
  ti = 0;
  while (r >= nt - ti) {
    r -= nt - ti;
    ++ti;
  }
  tj = ti + r;
}

template <typename Real>
struct MfmaAcc;
template <>
struct MfmaAcc<float> {
  using T = float4_t;
  static __device__ __forceinline__ T mma(float a, float b, T c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of register r of lane group g in the 16 x 16 result
  static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
};
template <>
struct MfmaAcc<double> {
  using T = double4_t;
  static __device__ __forceinline__ T mma(double a, double b, T c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // the FP64 16x16x4 result interleaves rows (measured on gfx950)
  static __device__ __forceinline__ int row(int g, int r) { return g + 4 * r; }
};

template <typename Real>
__global__ __launch_bounds__(256) void k_gram_mt(ZetaArgs z, MDims d, double* __restrict__ Cpart) {
  constexpr int kPad = (sizeof(Real) == 4) ? 16 : 8;  // row stride off the bank period
  __shared__ Real Xs[2][kKS][kMT + kPad];
  __shared__ Real Ys[2][kKS][kMT + kPad];
  using Acc = MfmaAcc<Real>;
  using AT = typename Acc::T;

  const int tid = threadIdx.x;
  const int lane = tid % kWave, wv = tid / kWave;
  const int s = blockIdx.y;
  int m, ti, tj;
  macro_tile_of(d, blockIdx.x, m, ti, tj);
  const int W = d.W[m];
  const bool diag = (ti == tj);
  const long long Kv = valid_rows(z);
  const long long r0 = (long long)s * kZetaBlock;
  const long long r1 = min(Kv, r0 + kZetaBlock);
  const double* A = z.A + d.off[m];
  const int* plist = z.plist + z.row_begin;

  // staging: thread -> (row srow, 8 columns from scol) of both column ranges
  const int srow = tid / 8, scol = (tid % 8) * 8;
  const int ci0 = ti * kMT + scol, cj0 = tj * kMT + scol;
  double xr[8], yr[8], wr = 0.0;
  auto load = [&](long long kb) {
    const long long r = kb + srow;
    const bool ok = r < r1;
    wr = ok ? z.wsort[plist[r]] : 0.0;
    const double* row = A + (ok ? r : r0) * (long long)z.lay.W;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      xr[c] = (ok && ci0 + c < W) ? row[ci0 + c] : 0.0;
      if (!diag) yr[c] = (ok && cj0 + c < W) ? row[cj0 + c] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      Xs[buf][srow][scol + c] = Real(wr * xr[c]);
      Ys[buf][srow][scol + c] = Real(diag ? xr[c] : yr[c]);
    }
  };

  AT acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = AT{0, 0, 0, 0};
  const int qi = (wv >> 1) * 32, qj = (wv & 1) * 32;
  const int li = lane % 16, g = lane / 16;

  // FP32 accumulation runs over kFlush rows at a time and is then added into
  // FP64 accumulators (the FP64 form accumulates in FP64 throughout)
  double4_t tot[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) tot[a][b] = double4_t{0.0, 0.0, 0.0, 0.0};
  auto flush = [&]() {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          tot[a][b][r] += double(acc[a][b][r]);
          acc[a][b][r] = Real(0);
        }
  };

  int buf = 0;
  if (r0 < r1) {
    load(r0);
    store(0);
  }
  __syncthreads();
  for (long long kb = r0; kb < r1; kb += kKS) {
    const bool more = kb + kKS < r1;
    if constexpr (sizeof(Real) == 4) {
      if (kb > r0 && (kb - r0) % kFlush == 0) flush();
    }
    if (more) load(kb + kKS);
#pragma unroll
    for (int k = 0; k < kKS; k += 4) {
      const int kk = k + g;
      Real xa[2], yb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) xa[a] = Xs[buf][kk][qi + a * 16 + li];
#pragma unroll
      for (int b = 0; b < 2; ++b) yb[b] = Ys[buf][kk][qj + b * 16 + li];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = Acc::mma(xa[a], yb[b], acc[a][b]);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  flush();
  double* C = Cpart + (long long)s * d.csize + d.cw[m];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ti * kMT + qi + a * 16 + Acc::row(g, r);
        const int j = tj * kMT + qj + b * 16 + li;
        if (i < W && j < W) C[i * W + j] = tot[a][b][r];
      }
}

// ---- BF16x3: the same macro tiles and blocks as k_gram_mt, with every FP32
// operand x split as x0 + x1 + x2, each xk the round-to-nearest-even bfloat16
// of what is left, and the six products with i + j <= 2 on the bfloat16
// matrix cores (FP32 accumulation over kFlush rows, then FP64).  Wave w stages
// rows 8w..8w+7 of each 32-row step, one column per lane: the eight values of
// a column are split and written to LDS as one 16-byte vector per part, laid
// out [column][row] so that an MFMA lane reads its eight rows of a column with
// one load.  The rows' weights come from lanes 0..31 of each wave by readlane.
constexpr int kBPad = 8;  // bf16 padding of a column's 32 rows (bank spread)

__global__ __launch_bounds__(256) void k_gram_bf16x3_mt(ZetaArgs z, MDims d,
                                                        double* __restrict__ Cpart) {
  __shared__ bf16x8_t Xs[2][3][kMT][(kKS + kBPad) / 8];
  __shared__ bf16x8_t Ys[2][3][kMT][(kKS + kBPad) / 8];
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int s = blockIdx.y;
  int m, ti, tj;
  macro_tile_of(d, blockIdx.x, m, ti, tj);
  const int W = d.W[m];
  const bool diag = (ti == tj);
  const long long Kv = valid_rows(z);
  const long long r0 = (long long)s * kZetaBlock;
  const long long r1 = min(Kv, r0 + kZetaBlock);
  const double* A = z.A + d.off[m];
  const int* plist = z.plist + z.row_begin;
  const int ci = ti * kMT + lane, cj = tj * kMT + lane;

  double xr[8], yr[8], wgt[8];
  auto load = [&](long long kb) {
    // lanes 0..31 fetch the step's weights; every lane takes its wave's 8
    const long long rw = kb + lane;
    const double wl = (lane < kKS && rw < r1) ? z.wsort[plist[rw]] : 0.0;
    const long long wb = __double_as_longlong(wl);
    const int wlo = int(wb & 0xffffffffll), whi = int(wb >> 32);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int lo = __builtin_amdgcn_readlane(wlo, 8 * wv + q);
      const int hi = __builtin_amdgcn_readlane(whi, 8 * wv + q);
      wgt[q] = __longlong_as_double((static_cast<long long>(hi) << 32) |
                                    static_cast<unsigned int>(lo));
      const long long r = kb + 8 * wv + q;
      const bool ok = r < r1;
      const double* row = A + (ok ? r : r0) * (long long)z.lay.W;
      xr[q] = (ok && ci < W) ? row[ci] : 0.0;
      if (!diag) yr[q] = (ok && cj < W) ? row[cj] : 0.0;
    }
  };
  auto split8 = [](const float v[8], bf16x8_t parts[3]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      float rem = v[q];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const __bf16 h = static_cast<__bf16>(rem);
        parts[k][q] = h;
        rem -= float(h);
      }
    }
  };
  auto store = [&](int buf) {
    float xv[8], yv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      xv[q] = float(wgt[q] * xr[q]);
      yv[q] = float(diag ? xr[q] : yr[q]);
    }
    bf16x8_t xp[3], yp[3];
    split8(xv, xp);
    split8(yv, yp);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Xs[buf][k][lane][wv] = xp[k];
      Ys[buf][k][lane][wv] = yp[k];
    }
  };

  float4_t acc[2][2];
  double4_t tot[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};
      tot[a][b] = double4_t{0.0, 0.0, 0.0, 0.0};
    }
  auto flush = [&]() {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          tot[a][b][r] += double(acc[a][b][r]);
          acc[a][b][r] = 0.f;
        }
  };
  const int qi = (wv >> 1) * 32, qj = (wv & 1) * 32;
  const int li = lane % 16, g = lane / 16;

  int buf = 0;
  if (r0 < r1) {
    load(r0);
    store(0);
  }
  __syncthreads();
  for (long long kb = r0; kb < r1; kb += kKS) {
    const bool more = kb + kKS < r1;
    if (kb > r0 && (kb - r0) % kFlush == 0) flush();
    if (more) load(kb + kKS);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const bf16x8_t x0 = Xs[buf][0][qi + a * 16 + li][g], x1 = Xs[buf][1][qi + a * 16 + li][g],
                       x2 = Xs[buf][2][qi + a * 16 + li][g];
        const bf16x8_t y0 = Ys[buf][0][qj + b * 16 + li][g], y1 = Ys[buf][1][qj + b * 16 + li][g],
                       y2 = Ys[buf][2][qj + b * 16 + li][g];
        float4_t c = acc[a][b];
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x2, y0, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, y1, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, y2, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, y0, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, y1, c, 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, y0, c, 0, 0, 0);
      }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  flush();
  double* C = Cpart + (long long)s * d.csize + d.cw[m];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ti * kMT + qi + a * 16 + 4 * g + r;
        const int j = tj * kMT + qj + b * 16 + li;
        if (i < W && j < W) C[i * W + j] = tot[a][b][r];
      }
}

// zeta[m][l][l'][b1][b2] += sum over the pair-block's 4096-primary blocks (in
// order, FP64) of the block Gram products.  Only macro tiles on or above the
// diagonal are stored; C_m is symmetric.
template <typename CT>
__global__ void k_zeta_accum_mt(const CT* __restrict__ C, int nsub, MDims d, RowLayout L,
                                double* __restrict__ zeta) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int nb = L.nb, nm = L.lmax + 1;
  const long long per_m = (long long)nm * nm * nb * nb;
  if (idx >= per_m * nm) return;
  long long t = idx;
  const int b2 = int(t % nb); t /= nb;
  const int b1 = int(t % nb); t /= nb;
  const int lp = int(t % nm); t /= nm;
  const int l = int(t % nm); t /= nm;
  const int m = int(t);
  if (l < m || lp < m) return;
  const int W = d.W[m];
  auto at = [&](int i, int j) {
    if (i / kMT > j / kMT) {
      const int x = i;
      i = j;
      j = x;
    }
    return d.cw[m] + i * W + j;
  };
  const int P = L.pos(m, l, b1), Pp = L.pos(m, lp, b2);
  const int dm = L.d[m];
  const int Q = dm + P, Qp = dm + Pp;
  const int iPP = at(P, Pp);
  const int iQQ = (m > 0) ? at(Q, Qp) : 0, iQP = (m > 0) ? at(Q, Pp) : 0,
            iPQ = (m > 0) ? at(P, Qp) : 0;
  double re = 0.0, im = 0.0;
  for (int s = 0; s < nsub; ++s) {
    const CT* c = C + (long long)s * d.csize;
    if (m == 0) {
      re += double(c[iPP]);
    } else {
      re += double(c[iPP]) + double(c[iQQ]);
      im += double(c[iQP]) - double(c[iPQ]);
    }
  }
  double* o = zeta + idx * 2;
  o[0] += re;
  o[1] += im;
}

}  // namespace

int sum_wm2(const RowLayout& L) {
  int s = 0;
  for (int m = 0; m <= L.lmax; ++m) s += L.wm[m] * L.wm[m];
  return s;
}

RowLayout make_layout(int lmax, int nb) {
  RowLayout L{};
  L.lmax = lmax;
  L.nb = nb;
  int off = 0;
  for (int m = 0; m <= lmax; ++m) {
    L.off[m] = off;
    L.d[m] = (lmax + 1 - m) * nb;
    L.wm[m] = (m == 0) ? L.d[m] : 2 * L.d[m];
    off += L.wm[m];
  }
  L.off[lmax + 1] = off;
  L.W = off;
  return L;
}

size_t zeta_partial_doubles(const RowLayout& L, long long PB) {
  const long long nsub_max = (PB + kZetaBlock - 1) / kZetaBlock;
  return size_t(std::max<long long>(nsub_max, kZetaSplitK)) * size_t(sum_wm2(L));
}

// All blocks of 4096 primaries of a pair-block (z.sub_begin = 0, z.K = rows).
hipError_t launch_zeta_pairblock(const ZetaArgs& z, hipStream_t st) {
  const MDims d = make_mdims(z.lay);
  const int nsub = int((z.K + kZetaBlock - 1) / kZetaBlock);
  if (nsub <= 0) return hipSuccess;
  const dim3 grid(unsigned(d.mt[d.nm]), unsigned(nsub));
  if (z.prec == G3PCF_PREC_FP32)
    hipLaunchKernelGGL((k_gram_mt<float>), grid, dim3(256), 0, st, z, d, z.C64);
  else if (z.prec == G3PCF_PREC_BF16X3)
    hipLaunchKernelGGL(k_gram_bf16x3_mt, grid, dim3(256), 0, st, z, d, z.C64);
  else
    hipLaunchKernelGGL((k_gram_mt<double>), grid, dim3(256), 0, st, z, d, z.C64);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long entries = (long long)(z.lay.lmax + 1) * (z.lay.lmax + 1) * (z.lay.lmax + 1) *
                            z.lay.nb * z.lay.nb;
  const unsigned ab = unsigned((entries + 255) / 256);
  hipLaunchKernelGGL((k_zeta_accum_mt<double>), dim3(ab), dim3(256), 0, st, z.C64, nsub, d,
                     z.lay, z.zeta);
  return hipGetLastError();
}

// ---------------------------------------------------------------- degenerate triangles
// The triangles j = k (the same secondary on both sides, so b1 = b2) are part
// of the product a_lm conj(a_l'm) (Sec. 3.1).  Without them, zeta^m_{ll'}(b, b)
// loses sum_i w_i sum_{j in b} w_j^2 conj(Y_lm(u_ij)) Y_l'm(u_ij), which is
// sum_n G[m][l][l'][n] D(b, n) with D(b, n) = sum_i w_i sum_{j in b} w_j^2 P_n(u_z).

__device__ double g_deg[kDegTable];

namespace {

constexpr int kDegRows = 512;  // rows of a pair-block summed per workgroup

// partial[blk][c] = sum over the workgroup's rows r, in order, of w_r X[r][c]
// (c < ncols; rows of the pair-block that are not primaries are skipped).
__global__ __launch_bounds__(256) void k_deg_partial(const double* __restrict__ X, int rowW,
                                                     int ncols, const double* __restrict__ wsort,
                                                     const int* __restrict__ plist,
                                                     const long long* __restrict__ nprim,
                                                     long long p_begin, long long p_count,
                                                     double* __restrict__ partial) {
  const long long valid = min(p_count, (long long)(*nprim) - p_begin);
  const long long r0 = (long long)blockIdx.x * kDegRows;
  const long long r1 = min(r0 + kDegRows, valid);
  for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
    double s = 0.0;
    for (long long r = r0; r < r1; ++r) s += wsort[plist[p_begin + r]] * X[r * rowW + c];
    partial[(long long)blockIdx.x * ncols + c] = s;
  }
}

// D[c] += sum over the workgroups, in order, of partial[blk][c]
__global__ void k_deg_accum(const double* __restrict__ partial, int nblk, int ncols,
                            double* __restrict__ D) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[(long long)b * ncols + c];
  D[c] += s;
}

__device__ __forceinline__ long long zpos(int lmax, int nb, int m, int l, int lp, int b1,
                                          int b2) {
  const int L1 = lmax + 1;
  return ((((long long)m * L1 + l) * L1 + lp) * nb + b1) * nb + b2;
}

// Re zeta^m_{ll'}(b, b) -= sum_n G[m][l][l'][n] D[b][n]  (the removed terms are real)
__global__ void k_deg_apply(const double* __restrict__ D, int lmax, int nb,
                            double* __restrict__ zeta) {
  const int L1 = lmax + 1;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)L1 * L1 * L1 * nb) return;
  const int b = int(idx % nb);
  long long t = idx / nb;
  const int lp = int(t % L1);
  t /= L1;
  const int l = int(t % L1);
  const int m = int(t / L1);
  if (l < m || lp < m) return;
  const int nd = 2 * lmax + 1;
  double s = 0.0;
  for (int n = 0; n <= l + lp; ++n) s += g_deg[deg_index(m, l, lp, n)] * D[b * nd + n];
  zeta[zpos(lmax, nb, m, l, lp, b, b) * 2] -= s;
}

// iso[l][b1][b2] = 4 pi / (2l + 1) (zeta^0_ll + 2 sum_{m >= 1} Re zeta^m_ll)(b1, b2)
__global__ void k_isotropic(const double* __restrict__ zeta, int lmax, int nb,
                            double* __restrict__ iso) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)(lmax + 1) * nb * nb) return;
  const int b2 = int(idx % nb);
  const int b1 = int((idx / nb) % nb);
  const int l = int(idx / ((long long)nb * nb));
  double s = 0.0;
  for (int m = 1; m <= l; ++m) s += zeta[zpos(lmax, nb, m, l, l, b1, b2) * 2];
  s = zeta[zpos(lmax, nb, 0, l, l, b1, b2) * 2] + 2.0 * s;
  iso[idx] = 4.0 * M_PI / (2.0 * l + 1.0) * s;
}

}  // namespace

hipError_t upload_deg_table() {
  static double host[kDegTable];
  static bool built = false;
  if (!built) {
    build_deg_table(host);
    built = true;
  }
  return hipMemcpyToSymbol(HIP_SYMBOL(g_deg), host, sizeof(host), 0, hipMemcpyHostToDevice);
}

size_t deg_partial_doubles(long long PB, int nb, int lmax) {
  return size_t((PB + kDegRows - 1) / kDegRows) * size_t(nb) * size_t(2 * lmax + 1);
}

hipError_t launch_deg_reduce(const double* X, int rowW, int nb, int lmax, const double* wsort,
                             const int* plist, const long long* nprim, long long p_begin,
                             long long p_count, double* partial, double* D, hipStream_t st) {
  if (p_count <= 0) return hipSuccess;
  const int ncols = nb * (2 * lmax + 1);
  const unsigned nblk = unsigned((p_count + kDegRows - 1) / kDegRows);
  hipLaunchKernelGGL(k_deg_partial, dim3(nblk), dim3(256), 0, st, X, rowW, ncols, wsort, plist,
                     nprim, p_begin, p_count, partial);
  hipLaunchKernelGGL(k_deg_accum, dim3((ncols + 255) / 256), dim3(256), 0, st, partial,
                     int(nblk), ncols, D);
  return hipGetLastError();
}

hipError_t launch_deg_apply(const double* D, int lmax, int nb, double* zeta, hipStream_t st) {
  const long long n = (long long)(lmax + 1) * (lmax + 1) * (lmax + 1) * nb;
  hipLaunchKernelGGL(k_deg_apply, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, D, lmax,
                     nb, zeta);
  return hipGetLastError();
}

hipError_t launch_isotropic(const double* zeta, int lmax, int nb, double* iso, hipStream_t st) {
  const long long n = (long long)(lmax + 1) * nb * nb;
  hipLaunchKernelGGL(k_isotropic, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, zeta, lmax,
                     nb, iso);
  return hipGetLastError();
}

}  // namespace g3
