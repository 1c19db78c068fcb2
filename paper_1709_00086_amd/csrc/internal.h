// Internal declarations shared by the g3pcf HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/g3pcf.h"

namespace g3 {

// The pair kernels always accumulate monomials up to this total degree; a
// smaller lmax only drops coefficients at conversion time.
constexpr int kDeg = 10;
constexpr int kTermsCart = (kDeg + 1) * (kDeg + 2) * (kDeg + 3) / 6;  // 286
constexpr int kTermsSpin = (kDeg + 1) * (kDeg + 1);                   // 121 real sums
// Conversion tables: G3PCF_BASIS_CARTESIAN, G3PCF_BASIS_SPIN and
// G3PCF_BASIS_SPIN_T (the spin terms with T_n(u_z) in place of u_z^n; only the
// FP32 adjoint uses it, after a forward pass in either basis).
constexpr int kConvTables = 3;
// Internal "basis" of the pass that collects the degenerate (j = k) triangles:
// per shell the sums w_j^2 P_n(u_z) of Legendre polynomials, n <= 2 kDeg.
constexpr int kBasisDeg = 3;
constexpr int kTermsDeg = 2 * kDeg + 1;                               // 21
constexpr int kMaxBins = 32;
constexpr int kWave = 64;
// Entries after the catalogue in the cell-ordered position array, every
// coordinate NaN: the FP32 pair search maps the lanes of a window past the
// end of its candidates onto them, and no shell test accepts a NaN distance.
constexpr int kSentinel = kWave;
constexpr int kOutPerBin = (kDeg + 1) * (kDeg + 1);  // real a_lm outputs per shell (121)

// Rows of A (primaries) reduced per Gram product on MFMA.
constexpr int kZetaBlock = 4096;
// Split-K slices of the Gram product (partials summed in order in FP64).
constexpr int kZetaSplitK = 4;
// Primary queues of the pair kernel: one per XCD (workgroups are dispatched to
// the 8 XCDs round-robin), each counter on its own 64-byte line.
constexpr int kQueues = 8;
constexpr int kQueueStride = 16;
// Persistent waves of the pair kernel.
constexpr int kPairWaves = 4096;
// Spill-list entries per wave: a shell's secondaries kept for the later
// accumulator chunks of a multi-chunk basis.
constexpr int kSpillCap = 1 << 14;
// Maximum pair-block (primaries whose a_lm rows are held at once).
constexpr int kPairBlockMax = 524288;

// Sparse monomial -> a_lm conversion table, one row per real output of a
// shell.  Output o = (m, part, l) with part 0 = Re, 1 = Im (m >= 1 only).
struct ConvTable {
  int nout;            // 121
  int nnz;
  short out_m[kOutPerBin], out_l[kOutPerBin], out_part[kOutPerBin];
  int rowptr[kOutPerBin + 1];
  short term[4096];
  double coef[4096];
  // the same entries grouped by monomial term (for the adjoint)
  int trowptr[kTermsCart + 1];
  short tout[4096];
  double tcoef[4096];
};

// Host: build the conversion table for a basis (0 cartesian, 1 spin with
// powers u_z^n, 2 spin with Chebyshev polynomials T_n(u_z)).
void build_conv_table(int basis, ConvTable* t);
// The table a problem basis accumulates and converts with: the spin basis
// sums (u_x - i u_y)^m T_n(u_z), so it converts with the spin-Chebyshev table.
__host__ __device__ constexpr int conv_table_of(int basis) {
  return basis == G3PCF_BASIS_SPIN ? int(G3PCF_BASIS_SPIN_T) : basis;
}

// Degenerate-triangle table G[m][l][l'][n]: Pbar_lm Pbar_l'm = sum_n G P_n.
constexpr int kDegTable = (kDeg + 1) * (kDeg + 1) * (kDeg + 1) * kTermsDeg;
__host__ __device__ inline int deg_index(int m, int l, int lp, int n) {
  return ((m * (kDeg + 1) + l) * (kDeg + 1) + lp) * kTermsDeg + n;
}
void build_deg_table(double* G);  // host

// Cell grid of the sorted catalogue.
struct Grid {
  double rsearch;      // search radius: R_max plus a margin for FP32 rounding
  int nc[3];
  double s[3], inv_s[3];
  double lo[3], L[3];
  int periodic;
  int tight[3];        // periodic axis where the search window can exceed the box
  int64_t ncell;
};

Grid make_grid(const g3pcf_problem& p);

// Layout of the real outputs of a primary inside an A row: block m holds the
// real parts, then (m >= 1) the imaginary parts, of a_lm(b) for l >= m; within
// a half, shell-major (one shell's l values are adjacent, so the pair kernel
// writes each shell's outputs as short contiguous runs).
struct RowLayout {
  int lmax, nb;
  int W;               // total row width
  int off[kDeg + 2];   // column offset of each m block
  int d[kDeg + 1];     // (lmax + 1 - m) * nb
  int wm[kDeg + 1];    // block width: d for m = 0, 2d for m >= 1
  // column of (l, shell b) within a half of block m
  __host__ __device__ int pos(int m, int l, int b) const { return b * (lmax + 1 - m) + (l - m); }
};

RowLayout make_layout(int lmax, int nb);

// Arguments of the pair kernels (forward accumulation and adjoint scatter).
struct PairArgs {
  const void* pos4;          // [n + kSentinel] (x, y, z, w) in cell order, float4 or double4
  int sentinel;              // slot of the first NaN entry (n)
  const int* cell_start;     // [ncell + 1]
  const int* plist;          // [*nprim] primary slots in cell order
  const long long* nprim;    // device scalar: number of primaries
  int* spill;                // per-wave lists of a shell's secondaries
  int spill_cap;             // entries per wave (0: no spill lists: one search per shell and chunk)
  int* queue;                // kQueues counters (stride kQueueStride): next primary of each XCD's share
  unsigned long long* pairs; // device scalar: accepted pairs
  long long p_begin;         // first primary of this pair-block
  long long p_count;         // primaries in this pair-block (upper bound)
  // geometry (double, used for the candidate search)
  int nc[3];
  double s[3], inv_s[3], lo[3], L[3];
  int periodic;
  int tight[3];
  double rmax, rmax_search;
  // FP32 shell test: shell b holds r^2 with r2_lo[b] < r^2 < r2_hi[b] (floats
  // next to the squared shell edges, so the shells partition the floats)
  float r2_lo[kMaxBins], r2_hi[kMaxBins];
  int nbins;
  int lmax;
  int los;                   // 0 z, 1 observer
  double obs[3];
  // outputs
  double* A;                 // [p_count][W] a_lm rows (forward)
  RowLayout lay;
  // adjoint
  const double* gcoef;       // [p_count][nbins][T] monomial-space adjoint coefficients (FP64 pairs)
  const double* H;           // [p_count][W] H rows (FP32 pairs: converted per shell in the kernel)
  const int* perm;           // [n] slot -> original index
  double* grad_w;            // [n] cell order: FP64 pair path (secondary terms added atomically)
  float* grad_w32;           // [n] cell order: FP32 pair path (secondary terms added atomically)
  const double* wsort;       // [n] weights in cell order (FP64)
};

// ---- launchers (each returns hipGetLastError after the launch) ----
// Buffers of the cell-list stage (all device, n = galaxies).
struct CellBufs {
  void* pos4;          // [n + kSentinel] out: cell-order (x, y, z, w), float4 or double4, then NaN
  void* stage4;        // [n] scratch: the same values in input order
  int* cell_start;     // [ncell + 1] out
  int* cell_count;     // [ncell + 1] scratch
  int* key_a;          // [n] scratch: cell ids (radix keys)
  int* key_b;          // [n] scratch
  int* val_a;          // [n] scratch: radix values
  int* perm;           // [n] out: cell-order slot -> input index
  int* hist;           // [2 radix_hist_ints(n)] scratch: digit counts and offsets
  double* wsort;       // [n] out: FP64 weights in cell order
  void* scan_tmp;      // scan scratch for max(ncell + 1, n + 1, radix_hist_ints(n)) entries
  size_t scan_bytes;
};
size_t radix_hist_ints(int64_t n);
hipError_t launch_cells(const g3pcf_problem& p, const Grid& g, const CellBufs& b, int fp64,
                        hipStream_t st);
// Primary list (cell order): galaxies in the mask (NULL: all) and, if region
// is not NULL, with region[i] == r.
hipError_t launch_primaries(const uint8_t* mask, const int32_t* region, int r, const int* perm,
                            int64_t n, int* flags, int* plist, long long* nprim,
                            void* scan_tmp, size_t scan_tmp_bytes, hipStream_t st);
// *out += order-independent hash of the cell-order catalogue (slot -> index,
// stored position words, weight) and the primary list, keyed by `seed` (a hash
// of the settings); *out must be cleared first.
hipError_t launch_fingerprint(const void* pos4, int fp64, const double* wsort, const int* perm,
                              const int* plist, const long long* nprim, int64_t n,
                              unsigned long long seed, unsigned long long* out, hipStream_t st);
hipError_t launch_fill_int(int* p, int64_t count, int value, hipStream_t st);
hipError_t launch_fill_double(double* p, int64_t count, double value, hipStream_t st);
hipError_t launch_pair_forward(const PairArgs& a, int fp64, int basis, hipStream_t st);
hipError_t launch_pair_adjoint(const PairArgs& a, int fp64, int basis, hipStream_t st);
// Degenerate-triangle pass: per primary and shell the sums w_j^2 P_n(u_z),
// n <= 2 lmax, into A[row][shell * (2 lmax + 1) + n] (FP64).
hipError_t launch_pair_distinct(const PairArgs& a, int fp64, hipStream_t st);
hipError_t upload_tables(int basis);

struct ZetaArgs {
  const double* A;           // [rows][W]
  const double* wsort;       // weights in cell order
  const int* plist;
  const long long* nprim;
  long long row_begin;       // global primary index of A row 0
  long long sub_begin;       // first row of this sub-block (relative to A)
  long long K;               // rows in this sub-block (upper bound)
  RowLayout lay;
  double* C64;               // per-block partial Gram products (FP64)
  double* zeta;
  int prec;
};
// Every block of kZetaBlock primaries of a pair-block: z.sub_begin = 0 and
// z.K = rows of the pair-block.
hipError_t launch_zeta_pairblock(const ZetaArgs& z, hipStream_t st);
// Doubles of the partial-Gram buffer (per-block partials of a pair-block of
// at most PB primaries).
size_t zeta_partial_doubles(const RowLayout& L, long long PB);

// Adjoint helpers
struct AdjArgs {
  const double* A;           // [rows][W]
  const double* gz;          // grad_zeta
  const double* wsort;
  const int* plist;
  const int* perm;
  const long long* nprim;
  long long p_begin;
  long long p_count;
  RowLayout lay;
  int basis;
  const ConvTable* table;    // device copy of the conversion table
  const double* MHt;         // adjoint matrices M_H^m, transposed
  double* H;                 // [p_count][W] H rows
  double* gcoef;             // [p_count][nbins][T]
  double* grad_w;            // [n] cell order
};
size_t adj_matrix_doubles(const RowLayout& L);
hipError_t launch_adj_matrix(const double* gz, const RowLayout& L, double* MHt, hipStream_t st);
// H = X M_H^T (k_h_gemm) and, for the FP64 pair path, the primary terms and
// the per-shell monomial coefficients (k_adj_finish); the FP32 adjoint pair
// kernel forms both from H itself.
hipError_t launch_h_gemm(const AdjArgs& a, hipStream_t st);
hipError_t launch_adj_finish(const AdjArgs& a, hipStream_t st);
// grad[perm[s]] (=|+=) gs[s] (+ gs32[s] when gs32 is not null); NaN instead
// when fp_saved is not null and *fp_saved != *fp_now
hipError_t launch_unpermute(const double* gs, const float* gs32, const int* perm, int64_t n,
                            int accumulate, const unsigned long long* fp_saved,
                            const unsigned long long* fp_now, double* grad, hipStream_t st);
// Device address of the uploaded conversion table of a basis.
hipError_t conv_table_device(int basis, const ConvTable** out);

size_t scan_tmp_bytes(int64_t count);
hipError_t launch_scan(const int* in, int* out, int64_t count, void* tmp, size_t tmp_bytes,
                       hipStream_t st);

int sum_wm2(const RowLayout& lay);

// Degenerate triangles (distinct secondaries): table upload, the weighted sum
// over a pair-block's rows X[r][b (2 lmax + 1) + n] into D (FP64, in order),
// and the correction of zeta^m_{ll'}(b, b).
hipError_t upload_deg_table();
size_t deg_partial_doubles(long long PB, int nb, int lmax);
hipError_t launch_deg_reduce(const double* X, int rowW, int nb, int lmax, const double* wsort,
                             const int* plist, const long long* nprim, long long p_begin,
                             long long p_count, double* partial, double* D, hipStream_t st);
hipError_t launch_deg_apply(const double* D, int lmax, int nb, double* zeta, hipStream_t st);
// Isotropic multipoles from zeta (addition theorem).
hipError_t launch_isotropic(const double* zeta, int lmax, int nb, double* iso, hipStream_t st);

}  // namespace g3
