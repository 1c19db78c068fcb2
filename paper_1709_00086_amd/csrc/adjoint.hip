// Adjoint of zeta with respect to the weights.
//
// With G = grad_re + i grad_im and L = Re sum conj(G) zeta, for a primary i
// with coefficients a_lm(b):
//   U_lm(b)  = sum_{l', b2} conj(G^m_{l l'}(b, b2)) conj(a_l'm(b2)),
//   V_lm(b)  = sum_{l', b1} conj(G^m_{l' l}(b1, b)) a_l'm(b1),
//   H_lm(b)  = U_lm(b) + conj(V_lm(b)),
//   dL/dw_i (as a primary)            = Re sum_{lm, b} a_lm(b) U_lm(b),
//   dL/dw_k (k a secondary in shell b) += w_i Re sum_lm conj(Y_lm(u_ik)) H_lm(b).
//
// For one m write x = [Re a | Im a] (the primary's block of its A row) and
// G^m = Gr + i Gi over the (l, b) indices.  Then
//   H = M_H x,  M_H = [[S, A], [A, -S]],  S = Gr + Gr^T,  A = Gi^T - Gi,
// (for m = 0, x = Re a and only S is needed), and since
// Re(a^T U) = Re(a^T conj(V)), the primary term is Re(a^T H) / 2.
// So for a block of primaries H = X M_H^T per m: a GEMM of the same shapes as
// the forward Gram products, run on FP64 MFMA.
//
// Because conj(Y_lm(u)) = sum_t c_{lm,t} mono_t(u) with the same monomials the
// forward pass accumulates, the secondary term is a polynomial in u with
// coefficients g_t(b) = sum_lm (Re c_{lm,t} Re H_lm(b) - Im c_{lm,t} Im H_lm(b)),
// evaluated per pair by the pair kernel's adjoint mode.  With FP64 pairs
// k_adj_finish forms the primary terms and these coefficients here; with FP32
// pairs the adjoint pair kernel forms both from the H rows itself.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace g3 {

namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ size_t zidx(int lmax, int nb, int m, int l, int lp, int b1, int b2) {
  const size_t L1 = size_t(lmax) + 1;
  return ((((size_t(m) * L1 + l) * L1 + lp) * nb + b1) * nb + b2) * 2;
}

struct AdjDims {
  int nm;
  int W[kDeg + 1], off[kDeg + 1], d[kDeg + 1];
  int cw[kDeg + 2];     // offset of M_H^m in the matrix buffer
  int rowW, nb, lmax;
};

AdjDims make_adj_dims(const RowLayout& L) {
  AdjDims d{};
  d.nm = L.lmax + 1;
  d.rowW = L.W;
  d.nb = L.nb;
  d.lmax = L.lmax;
  int cw = 0;
  for (int m = 0; m < d.nm; ++m) {
    d.W[m] = L.wm[m];
    d.off[m] = L.off[m];
    d.d[m] = L.d[m];
    d.cw[m] = cw;
    cw += L.wm[m] * L.wm[m];
  }
  d.cw[d.nm] = cw;
  return d;
}

// M_H^m stored transposed: MHt[cw_m + k * W_m + j] = M_H^m[j][k].
__global__ void k_build_mh(const double* __restrict__ gz, AdjDims d, double* __restrict__ MHt) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.cw[d.nm]) return;
  int m = 0;
  while (m + 1 < d.nm && idx >= d.cw[m + 1]) ++m;
  const int W = d.W[m], dm = d.d[m], nb = d.nb;
  const int r = idx - d.cw[m];
  const int k = r / W, j = r % W;  // entry M_H[j][k]
  const int nl = d.lmax + 1 - m;  // l values per shell in block m
  auto G = [&](int a, int b, int part) {  // G^m[a][b] over (l, b) indices
    const int l = m + a % nl, b1 = a / nl, lp = m + b % nl, b2 = b / nl;
    return gz[zidx(d.lmax, nb, m, l, lp, b1, b2) + part];
  };
  double v;
  if (m == 0) {
    v = G(j, k, 0) + G(k, j, 0);
  } else {
    const bool jr = j < dm, kr = k < dm;
    const int jj = jr ? j : j - dm, kk = kr ? k : k - dm;
    if (jr && kr) v = G(jj, kk, 0) + G(kk, jj, 0);            // S
    else if (!jr && !kr) v = -(G(jj, kk, 0) + G(kk, jj, 0));  // -S
    else v = G(kk, jj, 1) - G(jj, kk, 1);                     // A = Gi^T - Gi
  }
  MHt[idx] = v;
}

// H rows = X rows times M_H^T, per m, on FP64 MFMA.  One workgroup per
// (64 primaries, 64 output columns of one m): each step stages a 64 x 16 slice
// of X and a 16 x 64 slice of M_H^T in LDS (two stages, the next slice loaded
// during the current one's MFMAs), and each wave accumulates a 32 x 32
// quadrant as 2 x 2 MFMA tiles.  Lane l supplies A[i = l % 16][k = l / 16] and
// B[k = l / 16][j = l % 16]; the FP64 result holds row g + 4 r (g = l / 16) in
// register r.
constexpr int kHT = 64;   // rows and columns of a macro tile
constexpr int kHK = 16;   // k per step

struct HDims {
  int nm;
  int W[kDeg + 1], off[kDeg + 1];
  int cw[kDeg + 1];
  int ct[kDeg + 2];       // cumulative 64-column tiles
  int rowW;
};

HDims make_hdims(const RowLayout& L) {
  HDims d{};
  d.nm = L.lmax + 1;
  d.rowW = L.W;
  int cw = 0, ct = 0;
  for (int m = 0; m < d.nm; ++m) {
    d.W[m] = L.wm[m];
    d.off[m] = L.off[m];
    d.cw[m] = cw;
    d.ct[m] = ct;
    cw += L.wm[m] * L.wm[m];
    ct += (L.wm[m] + kHT - 1) / kHT;
  }
  d.ct[d.nm] = ct;
  return d;
}

__global__ __launch_bounds__(256) void k_h_gemm(const double* __restrict__ A,
                                                const double* __restrict__ MHt, HDims d,
                                                const long long* __restrict__ nprim,
                                                long long p_begin, long long p_count,
                                                double* __restrict__ H) {
  // two stages: the next k slice's global loads are in flight (in
  // registers) while the MFMAs work on the current one, one barrier a step
  __shared__ double Xs[2][kHT][kHK + 1];   // odd row stride: rows spread over banks
  __shared__ double Ms[2][kHK][kHT + 8];
  const int tid = threadIdx.x;
  const int lane = tid % kWave, wv = tid / kWave;
  const long long rows = min(p_count, (long long)(*nprim) - p_begin);
  const long long R0 = (long long)blockIdx.y * kHT;
  if (R0 >= rows) return;
  int m = 0;
  while (m + 1 < d.nm && int(blockIdx.x) >= d.ct[m + 1]) ++m;
  const int W = d.W[m];
  const int J0 = (int(blockIdx.x) - d.ct[m]) * kHT;
  const double* B = MHt + d.cw[m];
  // staging coordinates: X (row, 4 k's), M (k, 4 columns)
  const int xr = tid / 4, xk = (tid % 4) * 4;
  const int mk = tid / 16, mc = (tid % 16) * 4;
  const long long xrow = R0 + xr;
  const double* xp = A + (xrow < rows ? xrow : R0) * (long long)d.rowW + d.off[m];
  const int qi = (wv >> 1) * 32, qj = (wv & 1) * 32;
  const int li = lane % 16, g = lane / 16;
  double xv[4], mv[4];
  auto fetch = [&](int k0) {
    for (int c = 0; c < 4; ++c) {
      const int k = k0 + xk + c;
      xv[c] = (xrow < rows && k < W) ? xp[k] : 0.0;
      const int kk = k0 + mk, j = J0 + mc + c;
      mv[c] = (kk < W && j < W) ? B[(long long)kk * W + j] : 0.0;
    }
  };
  auto stage = [&](int s) {
    for (int c = 0; c < 4; ++c) {
      Xs[s][xr][xk + c] = xv[c];
      Ms[s][mk][mc + c] = mv[c];
    }
  };
  double4_t acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = double4_t{0.0, 0.0, 0.0, 0.0};
  fetch(0);
  stage(0);
  __syncthreads();
  int cur = 0;
  for (int k0 = 0; k0 < W; k0 += kHK) {
    const bool more = k0 + kHK < W;
    if (more) fetch(k0 + kHK);
#pragma unroll
    for (int k = 0; k < kHK; k += 4) {
      double xa[2], yb[2];
      for (int a = 0; a < 2; ++a) xa[a] = Xs[cur][qi + a * 16 + li][k + g];
      for (int b = 0; b < 2; ++b) yb[b] = Ms[cur][k + g][qj + b * 16 + li];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a], yb[b], acc[a][b], 0, 0, 0);
    }
    // the other stage was last read before the previous barrier
    if (more) stage(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int q = 0; q < 4; ++q) {
        const long long rr = R0 + qi + a * 16 + g + 4 * q;
        const int j = J0 + qj + b * 16 + li;
        if (rr < rows && j < W) H[rr * d.rowW + d.off[m] + j] = acc[a][b][q];
      }
}

// Per primary: the primary term Re(a^T H) / 2 and the coefficients g_t(b).
// One thread per monomial term: its conversion entries are read once and
// applied to every shell.
constexpr int kFinThreads = 128;
constexpr int kFinShells = 8;   // shells per pass over a term's entries

__global__ __launch_bounds__(kFinThreads) void k_adj_finish(AdjArgs a, AdjDims d) {
  const long long row = blockIdx.x;
  const long long valid = min(a.p_count, (long long)(*a.nprim) - a.p_begin);
  if (row >= valid) return;
  const int slot = a.plist[a.p_begin + row];
  const double* x = a.A + row * (long long)d.rowW;
  const double* h = a.H + row * (long long)d.rowW;
  extern __shared__ double fin_smem[];
  double* red = fin_smem;                // [kFinThreads]
  double* hs = fin_smem + kFinThreads;   // [rowW]
  double prim = 0.0;
  for (int c = threadIdx.x; c < d.rowW; c += blockDim.x) {
    const double hv = h[c];
    hs[c] = hv;
    // column c belongs to block m; the imaginary half enters with a minus sign
    int m = 0;
    while (m + 1 < d.nm && c >= d.off[m + 1]) ++m;
    const bool imag = (m > 0) && (c - d.off[m] >= d.d[m]);
    prim += imag ? -x[c] * hv : x[c] * hv;
  }
  red[threadIdx.x] = prim;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.grad_w[slot] += 0.5 * red[0];

  const ConvTable& t = *a.table;
  const int nb = d.nb;
  const int T = (a.basis == G3PCF_BASIS_SPIN) ? kTermsSpin : kTermsCart;
  double* gout = a.gcoef + row * (long long)nb * T;
  for (int term = threadIdx.x; term < T; term += blockDim.x) {
    const int e0 = t.trowptr[term], e1 = t.trowptr[term + 1];
    for (int b0 = 0; b0 < nb; b0 += kFinShells) {
      double sacc[kFinShells];
      for (int q = 0; q < kFinShells; ++q) sacc[q] = 0.0;
      for (int e = e0; e < e1; ++e) {
        const int out = t.tout[e];
        const int l = t.out_l[out];
        if (l > d.lmax) continue;
        const int m = t.out_m[out], part = t.out_part[out];
        const int nl = d.lmax + 1 - m;  // column stride between shells
        const int col = d.off[m] + (l - m) + (part ? d.d[m] : 0);
        const double c = part ? -t.tcoef[e] : t.tcoef[e];
        for (int q = 0; q < kFinShells; ++q)
          if (b0 + q < nb) sacc[q] += c * hs[col + (b0 + q) * nl];
      }
      for (int q = 0; q < kFinShells; ++q)
        if (b0 + q < nb) gout[(b0 + q) * T + term] = sacc[q];
    }
  }
}

__global__ void k_unpermute(const double* __restrict__ gs, const float* __restrict__ gs32,
                            const int* __restrict__ perm, int64_t n, int accumulate,
                            const unsigned long long* __restrict__ fp_saved,
                            const unsigned long long* __restrict__ fp_now,
                            double* __restrict__ grad) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int i = perm[s];
  double g = gs32 ? gs[s] + double(gs32[s]) : gs[s];
  // a_lm kept from a forward pass over other inputs: no valid gradient
  if (fp_saved && *fp_saved != *fp_now) g = __builtin_nan("");
  grad[i] = accumulate ? grad[i] + g : g;
}

}  // namespace

size_t adj_matrix_doubles(const RowLayout& L) { return size_t(sum_wm2(L)); }

hipError_t launch_adj_matrix(const double* gz, const RowLayout& L, double* MHt,
                             hipStream_t st) {
  const AdjDims d = make_adj_dims(L);
  const int n = d.cw[d.nm];
  hipLaunchKernelGGL(k_build_mh, dim3((n + 255) / 256), dim3(256), 0, st, gz, d, MHt);
  return hipGetLastError();
}

hipError_t launch_h_gemm(const AdjArgs& a, hipStream_t st) {
  const HDims hd = make_hdims(a.lay);
  const long long row_tiles = (a.p_count + kHT - 1) / kHT;
  hipLaunchKernelGGL(k_h_gemm, dim3(unsigned(hd.ct[hd.nm]), unsigned(row_tiles)), dim3(256), 0,
                     st, a.A, a.MHt, hd, a.nprim, a.p_begin, a.p_count, a.H);
  return hipGetLastError();
}

hipError_t launch_adj_finish(const AdjArgs& a, hipStream_t st) {
  const AdjDims d = make_adj_dims(a.lay);
  const size_t shm = size_t(kFinThreads + d.rowW) * sizeof(double);
  hipLaunchKernelGGL(k_adj_finish, dim3(unsigned(a.p_count)), dim3(kFinThreads), shm, st, a, d);
  return hipGetLastError();
}

hipError_t launch_unpermute(const double* gs, const float* gs32, const int* perm, int64_t n,
                            int accumulate, const unsigned long long* fp_saved,
                            const unsigned long long* fp_now, double* grad, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpermute, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, gs, gs32,
                     perm, n, accumulate, fp_saved, fp_now, grad);
  return hipGetLastError();
}

}  // namespace g3
