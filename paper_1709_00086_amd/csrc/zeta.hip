// The zeta stage: sum over primaries of w_i a_lm(b1) conj(a_l'm(b2)).
//
// The paper adds the per-primary products a_lm(r1) a*_l'm(r2) (Sec. 3.1) and
// combines per-thread partial multipoles at the end of the loop over primaries
// (single-node optimisations section).  Here the per-primary coefficients of a
// block of K primaries are the rows of A, and for every m the block's
// contribution is a Gram product on the matrix cores:
//   B_m = [Re A^m | Im A^m]  (K x W_m),   C_m = (diag(w) B_m)^T B_m,
//   Re zeta^m = C_pp + C_qq,   Im zeta^m = C_qp - C_pq.
// For m = 0 every a_l0 is real and B_0 = Re A^0.  Each block's C_m is added
// into zeta in FP64.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace g3 {

namespace {

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

constexpr int kTile = 16;

struct Dims {
  int nm;                 // lmax + 1
  int W[kDeg + 1];        // block widths
  int off[kDeg + 1];      // column offsets in an A row
  int cw[kDeg + 2];       // offsets of each C_m in the partial buffer
  int tiles[kDeg + 2];    // cumulative tile counts
  int rowW;               // A row width
  int csize;              // sum W_m^2
};

Dims make_dims(const RowLayout& L) {
  Dims d{};
  d.nm = L.lmax + 1;
  d.rowW = L.W;
  int cw = 0, tiles = 0;
  for (int m = 0; m < d.nm; ++m) {
    d.W[m] = L.wm[m];
    d.off[m] = L.off[m];
    d.cw[m] = cw;
    d.tiles[m] = tiles;
    cw += L.wm[m] * L.wm[m];
    const int t = (L.wm[m] + kTile - 1) / kTile;
    tiles += t * t;
  }
  d.cw[d.nm] = cw;
  d.tiles[d.nm] = tiles;
  d.csize = cw;
  return d;
}

__device__ __forceinline__ void tile_of(const Dims& d, int t, int& m, int& ti, int& tj) {
  m = 0;
  while (m + 1 < d.nm && t >= d.tiles[m + 1]) ++m;
  const int r = t - d.tiles[m];
  const int nt = (d.W[m] + kTile - 1) / kTile;
  ti = r / nt;
  tj = r % nt;
}

__device__ __forceinline__ long long valid_rows(const ZetaArgs& z) {
  // primaries in the pair-block, then rows of this sub-block
  const long long in_block = (long long)(*z.nprim) - z.row_begin;
  long long kv = in_block - z.sub_begin;
  if (kv > z.K) kv = z.K;
  return kv < 0 ? 0 : kv;
}

// One wave per (m, 16x16 tile, K slice).  A operand = (w B_m)^T, B operand = B_m.
// Lane l holds A[i = l % 16][k = l / 16] and B[k = l / 16][j = l % 16]; the
// FP32 16x16 result sits in lanes as C[4 (l / 16) + r][l % 16], r = 0..3.
template <typename Real>
__global__ __launch_bounds__(256) void k_gram_direct(ZetaArgs z, Dims d) {
  const int wave = blockIdx.x * 4 + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int ntile = d.tiles[d.nm];
  if (wave >= ntile * kZetaSplitK) return;
  const int s = wave / ntile;
  int m, ti, tj;
  tile_of(d, wave % ntile, m, ti, tj);
  const long long Kv = valid_rows(z);
  const int W = d.W[m];
  const int i = ti * kTile + lane % 16, j = tj * kTile + lane % 16;
  const int g = lane / 16;
  const long long per = ((Kv + 4 * kZetaSplitK - 1) / (4 * kZetaSplitK)) * 4;
  const long long k0 = s * per, k1 = min(Kv, k0 + per);
  const double* A = z.A + (z.sub_begin) * (long long)d.rowW + d.off[m];
  const int* plist = z.plist + z.row_begin + z.sub_begin;
  if constexpr (sizeof(Real) == 4) {
    float4_t acc = {0.f, 0.f, 0.f, 0.f};
    for (long long k = k0; k < k1; k += 4) {
      const long long r = k + g;
      float av = 0.f, bv = 0.f;
      if (r < k1) {
        const double wr = z.wsort[plist[r]];
        const double* row = A + r * d.rowW;
        if (i < W) av = float(wr * row[i]);
        if (j < W) bv = float(row[j]);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
    }
    float* C = z.C32 + (long long)s * d.csize + d.cw[m];
    for (int r = 0; r < 4; ++r) {
      const int ii = ti * kTile + 4 * g + r;
      if (ii < W && j < W) C[ii * W + j] = acc[r];
    }
  } else {
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    for (long long k = k0; k < k1; k += 4) {
      const long long r = k + g;
      double av = 0.0, bv = 0.0;
      if (r < k1) {
        const double wr = z.wsort[plist[r]];
        const double* row = A + r * d.rowW;
        if (i < W) av = wr * row[i];
        if (j < W) bv = row[j];
      }
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    // The FP64 16x16x4 result interleaves rows: lane group g, register r
    // holds row g + 4 r (measured on gfx950; the FP32 form holds 4 g + r).
    double* C = z.C64 + (long long)s * d.csize + d.cw[m];
    for (int r = 0; r < 4; ++r) {
      const int ii = ti * kTile + g + 4 * r;
      if (ii < W && j < W) C[ii * W + j] = acc[r];
    }
  }
}

// ---- BF16x3: x = x0 + x1 + x2 with each xk the round-to-nearest-even bfloat16
// of what is left, stored transposed ([column][row], rows padded to 32).
__device__ __forceinline__ __bf16 to_bf16(float x) { return static_cast<__bf16>(x); }

__global__ void k_split_bf16(ZetaArgs z, Dims d, int Kp) {
  // one thread per (column c, row r), rows fastest
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)d.rowW * Kp;
  if (idx >= total) return;
  const int c = int(idx / Kp);
  const int r = int(idx % Kp);
  const long long Kv = valid_rows(z);
  float x = 0.f, y = 0.f;
  if (r < Kv) {
    const double a = z.A[(z.sub_begin + r) * (long long)d.rowW + c];
    const double wr = z.wsort[z.plist[z.row_begin + z.sub_begin + r]];
    x = float(wr * a);
    y = float(a);
  }
  __bf16* ops = static_cast<__bf16*>(z.ops);
  const long long plane = (long long)d.rowW * Kp;
  const long long at = (long long)c * Kp + r;
  float rx = x, ry = y;
  for (int k = 0; k < 3; ++k) {
    const __bf16 hx = to_bf16(rx), hy = to_bf16(ry);
    ops[k * plane + at] = hx;
    ops[(3 + k) * plane + at] = hy;
    rx -= float(hx);
    ry -= float(hy);
  }
}

__device__ __forceinline__ bf16x8_t load8(const __bf16* p) {
  return *reinterpret_cast<const bf16x8_t*>(p);
}

// Products kept: (x0 y0), (x0 y1), (x1 y0), (x0 y2), (x1 y1), (x2 y0).
__global__ __launch_bounds__(256) void k_gram_bf16x3(ZetaArgs z, Dims d, int Kp) {
  const int wave = blockIdx.x * 4 + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int ntile = d.tiles[d.nm];
  if (wave >= ntile * kZetaSplitK) return;
  const int s = wave / ntile;
  int m, ti, tj;
  tile_of(d, wave % ntile, m, ti, tj);
  const int W = d.W[m];
  const int i = ti * kTile + lane % 16, j = tj * kTile + lane % 16;
  const int g = lane / 16;
  const int per = ((Kp + 32 * kZetaSplitK - 1) / (32 * kZetaSplitK)) * 32;
  const int k0 = s * per, k1 = min(Kp, k0 + per);
  const __bf16* ops = static_cast<const __bf16*>(z.ops);
  const long long plane = (long long)d.rowW * Kp;
  const int ci = d.off[m] + min(i, W - 1), cj = d.off[m] + min(j, W - 1);
  const __bf16* X0 = ops + (long long)ci * Kp;
  const __bf16* Y0 = ops + 3 * plane + (long long)cj * Kp;
  float4_t acc = {0.f, 0.f, 0.f, 0.f};
  const bf16x8_t zero8 = {};
  for (int k = k0; k < k1; k += 32) {
    const int kk = k + 8 * g;
    bf16x8_t x0 = load8(X0 + kk), x1 = load8(X0 + plane + kk), x2 = load8(X0 + 2 * plane + kk);
    bf16x8_t y0 = load8(Y0 + kk), y1 = load8(Y0 + plane + kk), y2 = load8(Y0 + 2 * plane + kk);
    if (i >= W) x0 = x1 = x2 = zero8;
    if (j >= W) y0 = y1 = y2 = zero8;
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x2, y0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, y1, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, y2, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, y0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, y1, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, y0, acc, 0, 0, 0);
  }
  float* C = z.C32 + (long long)s * d.csize + d.cw[m];
  for (int r = 0; r < 4; ++r) {
    const int ii = ti * kTile + 4 * g + r;
    if (ii < W && j < W) C[ii * W + j] = acc[r];
  }
}

// zeta[m][l][l'][b1][b2] += block contribution, summed over K slices in order.
template <typename CT>
__global__ void k_zeta_accum(const CT* __restrict__ C, Dims d, RowLayout L,
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
  const int P = (l - m) * nb + b1, Pp = (lp - m) * nb + b2;
  double re = 0.0, im = 0.0;
  for (int s = 0; s < kZetaSplitK; ++s) {
    const CT* c = C + (long long)s * d.csize + d.cw[m];
    if (m == 0) {
      re += double(c[P * W + Pp]);
    } else {
      const int dm = L.d[m];
      const int Q = dm + P, Qp = dm + Pp;
      re += double(c[P * W + Pp]) + double(c[Q * W + Qp]);
      im += double(c[Q * W + Pp]) - double(c[P * W + Qp]);
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

hipError_t launch_zeta_block(const ZetaArgs& z, hipStream_t st) {
  const Dims d = make_dims(z.lay);
  const int waves = d.tiles[d.nm] * kZetaSplitK;
  const unsigned blocks = unsigned((waves + 3) / 4);
  if (z.prec == G3PCF_PREC_BF16X3) {
    const int Kp = ((z.K + 31) / 32) * 32;
    const long long total = (long long)d.rowW * Kp;
    hipLaunchKernelGGL(k_split_bf16, dim3(unsigned((total + 255) / 256)), dim3(256), 0, st, z, d,
                       Kp);
    hipLaunchKernelGGL(k_gram_bf16x3, dim3(blocks), dim3(256), 0, st, z, d, Kp);
  } else if (z.prec == G3PCF_PREC_FP32) {
    hipLaunchKernelGGL((k_gram_direct<float>), dim3(blocks), dim3(256), 0, st, z, d);
  } else {
    hipLaunchKernelGGL((k_gram_direct<double>), dim3(blocks), dim3(256), 0, st, z, d);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long entries = (long long)(z.lay.lmax + 1) * (z.lay.lmax + 1) * (z.lay.lmax + 1) *
                            z.lay.nb * z.lay.nb;
  const unsigned ab = unsigned((entries + 255) / 256);
  if (z.prec == G3PCF_PREC_FP64)
    hipLaunchKernelGGL((k_zeta_accum<double>), dim3(ab), dim3(256), 0, st, z.C64, d, z.lay,
                       z.zeta);
  else
    hipLaunchKernelGGL((k_zeta_accum<float>), dim3(ab), dim3(256), 0, st, z.C32, d, z.lay,
                       z.zeta);
  return hipGetLastError();
}

}  // namespace g3
