// Adjoint of zeta with respect to the weights.
//
// With G = grad_re + i grad_im and L = Re sum conj(G) zeta, for a primary i
// with coefficients a_lm(b):
//   U_lm(b)  = sum_{l', b2} conj(G^m_{l l'}(b, b2)) conj(a_l'm(b2)),
//   V_lm(b)  = sum_{l', b1} conj(G^m_{l' l}(b1, b)) a_l'm(b1),
//   H_lm(b)  = U_lm(b) + conj(V_lm(b)),
//   dL/dw_i (as a primary)            = Re sum_{lm, b} a_lm(b) U_lm(b),
//   dL/dw_k (k a secondary in shell b) += w_i Re sum_lm conj(Y_lm(u_ik)) H_lm(b).
// Because conj(Y_lm(u)) = sum_t c_{lm,t} mono_t(u) with the same monomials the
// forward pass accumulates, the secondary term is a polynomial in u with
// coefficients g_t(b) = sum_lm (Re c_{lm,t} Re H_lm(b) - Im c_{lm,t} Im H_lm(b)),
// evaluated per pair by the pair kernel's adjoint mode.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace g3 {

namespace {

constexpr int kAdjThreads = 256;

__device__ __forceinline__ size_t zidx(int lmax, int nb, int m, int l, int lp, int b1, int b2) {
  const size_t L1 = size_t(lmax) + 1;
  return ((((size_t(m) * L1 + l) * L1 + lp) * nb + b1) * nb + b2) * 2;
}

// one block per primary row of the pair-block
__global__ __launch_bounds__(kAdjThreads) void k_adj_coef(AdjArgs a) {
  extern __shared__ double sh[];
  const RowLayout& L = a.lay;
  const int nb = L.nb, lmax = L.lmax;
  const long long row = blockIdx.x;
  const long long valid = min(a.p_count, (long long)(*a.nprim) - a.p_begin);
  if (row >= valid) return;
  const int slot = a.plist[a.p_begin + row];
  double* arow = sh;                 // [W]
  double* H = sh + L.W;              // [nb][nlm][2]
  __shared__ double red[kAdjThreads];
  const int nlm = (lmax + 1) * (lmax + 2) / 2;
  const double* A = a.A + row * (long long)L.W;
  for (int c = threadIdx.x; c < L.W; c += blockDim.x) arow[c] = A[c];
  __syncthreads();

  auto a_re = [&](int l, int m, int b) { return arow[L.off[m] + (l - m) * nb + b]; };
  auto a_im = [&](int l, int m, int b) {
    return m == 0 ? 0.0 : arow[L.off[m] + L.d[m] + (l - m) * nb + b];
  };

  double prim = 0.0;
  for (int o = threadIdx.x; o < nb * nlm; o += blockDim.x) {
    const int b = o / nlm;
    int lm = o % nlm;
    int l = 0;
    while ((l + 1) * (l + 2) / 2 <= lm) ++l;
    const int m = lm - l * (l + 1) / 2;
    double ur = 0.0, ui = 0.0, vr = 0.0, vi = 0.0;
    for (int lp = m; lp <= lmax; ++lp)
      for (int bb = 0; bb < nb; ++bb) {
        // U += conj(G(m,l,lp,b,bb)) conj(a_lp,m(bb))
        const double* g = a.gz + zidx(lmax, nb, m, l, lp, b, bb);
        const double xr = a_re(lp, m, bb), xi = a_im(lp, m, bb);
        // (gr - i gi)(xr - i xi) = gr xr - gi xi - i (gr xi + gi xr)
        ur += g[0] * xr - g[1] * xi;
        ui -= g[0] * xi + g[1] * xr;
        // V += conj(G(m,lp,l,bb,b)) a_lp,m(bb)
        const double* h = a.gz + zidx(lmax, nb, m, lp, l, bb, b);
        // (hr - i hi)(xr + i xi) = hr xr + hi xi + i (hr xi - hi xr)
        vr += h[0] * xr + h[1] * xi;
        vi += h[0] * xi - h[1] * xr;
      }
    // primary term: Re(a U)
    prim += a_re(l, m, b) * ur - a_im(l, m, b) * ui;
    H[(b * nlm + lm) * 2] = ur + vr;
    H[(b * nlm + lm) * 2 + 1] = ui - vi;
  }
  red[threadIdx.x] = prim;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.grad_w[slot] += red[0];

  // g_t(b) from the by-term table
  const ConvTable& t = *a.table;
  const int T = (a.basis == G3PCF_BASIS_SPIN) ? kTermsSpin : kTermsCart;
  double* gout = a.gcoef + row * (long long)nb * T;
  for (int o = threadIdx.x; o < nb * T; o += blockDim.x) {
    const int b = o / T, term = o % T;
    double s = 0.0;
    for (int e = t.trowptr[term]; e < t.trowptr[term + 1]; ++e) {
      const int out = t.tout[e];
      const int l = t.out_l[out];
      if (l > lmax) continue;
      const int m = t.out_m[out], part = t.out_part[out];
      const int lm = l * (l + 1) / 2 + m;
      const double* h = H + (b * nlm + lm) * 2;
      s += (part == 0) ? t.tcoef[e] * h[0] : -t.tcoef[e] * h[1];
    }
    gout[o] = s;
  }
}

__global__ void k_unpermute(const double* __restrict__ gs, const int* __restrict__ perm,
                            int64_t n, int accumulate, double* __restrict__ grad) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int i = perm[s];
  grad[i] = accumulate ? grad[i] + gs[s] : gs[s];
}

}  // namespace

hipError_t launch_adj_coef(const AdjArgs& a, hipStream_t st) {
  const int nlm = (a.lay.lmax + 1) * (a.lay.lmax + 2) / 2;
  const size_t lds = sizeof(double) * (size_t(a.lay.W) + 2 * size_t(a.lay.nb) * nlm);
  hipLaunchKernelGGL(k_adj_coef, dim3(unsigned(a.p_count)), dim3(kAdjThreads), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_unpermute(const double* gs, const int* perm, int64_t n, int accumulate,
                            double* grad, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpermute, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, gs, perm,
                     n, accumulate, grad);
  return hipGetLastError();
}

}  // namespace g3
