// Catalogue staging: wrap, cell assignment, a stable sort into cell order
// (members of a cell in input order), and the compacted primary list.
//
// The paper keeps its galaxies in a node-local k-d tree for the range search
// (Algorithm 1, "search node-local k-d tree").  On the GPU a uniform cell grid
// sorted by a counting sort serves the same purpose: every (cy, cz) row of
// cells is one contiguous run of galaxies in memory, so the pair kernels read
// candidates with coalesced loads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace g3 {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;  // per thread
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ inline double wrap_coord(double x, double lo, double L) {
  double t = fmod(x - lo, L);
  if (t < 0.0) t += L;
  if (t >= L) t = 0.0;
  return lo + t;
}

template <typename Real>
struct Vec4;
template <>
struct Vec4<float> {
  using T = float4;
};
template <>
struct Vec4<double> {
  using T = double4;
};

struct GridDev {
  int nc[3];
  double inv_s[3], lo[3], L[3];
  int periodic;
};

// Cell along one axis; coordinates outside the box (open boxes) go to the
// edge cells, and a non-finite coordinate to cell 0 (such a galaxy is never
// accepted as a secondary and has no neighbours as a primary).
__device__ inline int cell_axis(double x, double lo, double inv_s, int nc) {
  const double f = floor((x - lo) * inv_s);
  if (!(f >= 0.0)) return 0;
  return f >= double(nc) ? nc - 1 : int(f);
}

// Wrap (periodic), convert to the compute precision and assign a cell.
template <typename Real, typename In>
__global__ void k_assign(const In* __restrict__ pos, const double* __restrict__ w, int64_t n,
                         GridDev g, typename Vec4<Real>::T* __restrict__ out4,
                         int* __restrict__ cid, int* __restrict__ count) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x[3];
  for (int a = 0; a < 3; ++a) {
    double v = double(pos[3 * i + a]);
    if (g.periodic) {
      v = wrap_coord(v, g.lo[a], g.L[a]);
      Real r = Real(v);
      // a float that rounds up onto the upper box edge wraps to the lower edge
      if (double(r) >= g.lo[a] + g.L[a]) r = Real(g.lo[a]);
      v = double(r);
    } else {
      v = double(Real(v));
    }
    x[a] = v;
  }
  const int cx = cell_axis(x[0], g.lo[0], g.inv_s[0], g.nc[0]);
  const int cy = cell_axis(x[1], g.lo[1], g.inv_s[1], g.nc[1]);
  const int cz = cell_axis(x[2], g.lo[2], g.inv_s[2], g.nc[2]);
  const int c = (cz * g.nc[1] + cy) * g.nc[0] + cx;
  typename Vec4<Real>::T v4;
  v4.x = Real(x[0]);
  v4.y = Real(x[1]);
  v4.z = Real(x[2]);
  v4.w = Real(w[i]);
  out4[i] = v4;
  cid[i] = c;
  atomicAdd(&count[c], 1);
}

// ---- stable LSD radix sort of the cell ids (values: original indices) ----
// The galaxies come in input order, so a stable sort by cell id leaves every
// cell's members in increasing input order: the cell list is deterministic
// whatever the data (no atomics decide an order, and a crowded cell costs no
// more than a sparse one).  Digits of kRadixBits bits; each pass counts the
// digits of every tile of kRadixTile keys, scans the counts digit-major across
// tiles, and scatters each tile in order.
constexpr int kRadixBits = 8;
constexpr int kRadixDigits = 1 << kRadixBits;
constexpr int kRadixThreads = 256;
constexpr int kRadixRounds = 8;
constexpr int kRadixTile = kRadixThreads * kRadixRounds;
constexpr int kRadixWaves = kRadixThreads / kWave;

__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const int* __restrict__ keys,
                                                              int64_t n, int shift, int ntiles,
                                                              int* __restrict__ hist) {
  __shared__ int cnt[kRadixDigits];
  for (int d = threadIdx.x; d < kRadixDigits; d += kRadixThreads) cnt[d] = 0;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * kRadixTile;
  for (int k = 0; k < kRadixRounds; ++k) {
    const int64_t e = base + k * kRadixThreads + threadIdx.x;
    if (e < n) atomicAdd(&cnt[(keys[e] >> shift) & (kRadixDigits - 1)], 1);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kRadixDigits; d += kRadixThreads)
    hist[int64_t(d) * ntiles + blockIdx.x] = cnt[d];
}

// keys_in / vals_in (vals_in NULL: the value is the key's own index) into
// keys_out (NULL: not written) / vals_out at the scanned offsets.  Within a
// round of kRadixThreads keys, a key's rank among the keys of its wave with
// the same digit comes from eight ballots; the waves' counts per digit give
// the offsets across waves, and `base` carries each digit's running offset
// from round to round.
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(
    const int* __restrict__ keys_in, const int* __restrict__ vals_in, int64_t n, int shift,
    int ntiles, const int* __restrict__ offs, int* __restrict__ keys_out,
    int* __restrict__ vals_out) {
  __shared__ int base[kRadixDigits];
  __shared__ int wcnt[kRadixWaves][kRadixDigits];
  for (int d = threadIdx.x; d < kRadixDigits; d += kRadixThreads) {
    base[d] = offs[int64_t(d) * ntiles + blockIdx.x];
    for (int w = 0; w < kRadixWaves; ++w) wcnt[w][d] = 0;
  }
  __syncthreads();
  const int wave = threadIdx.x / kWave;
  const int64_t tile0 = int64_t(blockIdx.x) * kRadixTile;
  for (int k = 0; k < kRadixRounds; ++k) {
    const int64_t e = tile0 + k * kRadixThreads + threadIdx.x;
    const bool valid = e < n;
    const int key = valid ? keys_in[e] : 0;
    const int val = valid ? (vals_in ? vals_in[e] : int(e)) : 0;
    const int d = (key >> shift) & (kRadixDigits - 1);
    unsigned long long peers = __builtin_amdgcn_ballot_w64(valid);
    for (int bit = 0; bit < kRadixBits; ++bit) {
      const bool on = (d >> bit) & 1;
      const unsigned long long b = __builtin_amdgcn_ballot_w64(on);
      peers &= on ? b : ~b;
    }
    const int rank = __builtin_amdgcn_mbcnt_hi(unsigned(peers >> 32),
                                               __builtin_amdgcn_mbcnt_lo(unsigned(peers), 0));
    if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int off = base[d] + rank;
      for (int w = 0; w < wave; ++w) off += wcnt[w][d];
      if (keys_out) keys_out[off] = key;
      vals_out[off] = val;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kRadixDigits; t += kRadixThreads) {
      int add = 0;
      for (int w = 0; w < kRadixWaves; ++w) {
        add += wcnt[w][t];
        wcnt[w][t] = 0;
      }
      base[t] += add;
    }
    __syncthreads();
  }
}

// Cell-order arrays from the sorted original indices, and the kSentinel NaN
// entries after them.
template <typename V4>
__global__ void k_gather_sorted(const V4* __restrict__ in4, const int* __restrict__ perm,
                                int64_t n, const double* __restrict__ w,
                                V4* __restrict__ out4, double* __restrict__ wsort) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n) {
    if (s < n + kSentinel) {
      using T = decltype(out4[0].x);
      const T nan = T(__builtin_nan(""));
      out4[s] = V4{nan, nan, nan, nan};
    }
    return;
  }
  const int i = perm[s];
  out4[s] = in4[i];
  wsort[s] = w[i];
}

// primary flag of the galaxy in cell-order slot s: in the mask (if any) and,
// when region ids are given, in region r
__global__ void k_primary_flags(const uint8_t* __restrict__ mask,
                                const int32_t* __restrict__ region, int r,
                                const int* __restrict__ perm, int64_t n,
                                int* __restrict__ flags) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s > n) return;
  if (s == n) {
    flags[s] = 0;
    return;
  }
  const int i = perm[s];
  flags[s] = ((mask == nullptr || mask[i] != 0) && (region == nullptr || region[i] == r)) ? 1 : 0;
}

__global__ void k_primary_list(const int* __restrict__ flags, const int* __restrict__ pos,
                               int64_t n, int* __restrict__ plist,
                               long long* __restrict__ nprim) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s > n) return;
  if (s == n) {
    *nprim = pos[n];
    return;
  }
  if (flags[s]) plist[pos[s]] = int(s);
}

__global__ void k_fill_int(int* p, int64_t count, int value) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

__global__ void k_fill_double(double* p, int64_t count, double value) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

// ---- exclusive scan of int32 (three phases, recursive over tile sums) ----
__global__ void k_scan_tiles(const int* __restrict__ in, int* __restrict__ out, int64_t count,
                             int* __restrict__ tile_sums) {
  __shared__ int sh[kScanBlock];
  const int64_t base = int64_t(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    v[k] = (i < count) ? in[i] : 0;
    s += v[k];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int t = (threadIdx.x >= off) ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - s;  // exclusive prefix of this thread
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < count) out[i] = run;
    run += v[k];
  }
  if (threadIdx.x == kScanBlock - 1) tile_sums[blockIdx.x] = sh[threadIdx.x];
}

__global__ void k_scan_add(int* __restrict__ out, int64_t count,
                           const int* __restrict__ tile_offsets) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) out[i] += tile_offsets[i / kScanTile];
}

inline unsigned blocks_for(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

// splitmix64 output function (Steele, Lea and Flood, OOPSLA 2014)
__device__ __forceinline__ unsigned long long mix64(unsigned long long x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

constexpr int kPrintBlocks = 1024;

// Fingerprint of everything the a_lm rows depend on besides the settings:
// per cell-order slot its original index, stored position words and weight,
// and the primary list.  A wrapping sum of per-slot hashes (one atomic per
// workgroup), so the value does not depend on the order of the atomics.
__global__ __launch_bounds__(256) void k_fingerprint(const unsigned* __restrict__ pos_words,
                                                     int words, const double* __restrict__ wsort,
                                                     const int* __restrict__ perm,
                                                     const int* __restrict__ plist,
                                                     const long long* __restrict__ nprim,
                                                     int64_t n, unsigned long long seed,
                                                     unsigned long long* __restrict__ out) {
  __shared__ unsigned long long part[256 / kWave];
  const long long np = *nprim;
  unsigned long long h = 0;
  for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < n;
       s += int64_t(gridDim.x) * blockDim.x) {
    unsigned long long x = mix64(seed + (unsigned long long)s);
    x = mix64(x ^ (unsigned)perm[s]);
    for (int k = 0; k < words; ++k) x = mix64(x ^ pos_words[s * words + k]);
    x = mix64(x ^ (unsigned long long)__double_as_longlong(wsort[s]));
    h += x;
    if (s < np) h += mix64(~seed ^ ((unsigned long long)s << 32) ^ (unsigned)plist[s]);
  }
  for (int off = kWave / 2; off > 0; off >>= 1) h += __shfl_xor(h, off);
  const int wave = threadIdx.x / kWave;
  if (threadIdx.x % kWave == 0) part[wave] = h;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int k = 0; k < int(blockDim.x) / kWave; ++k) t += part[k];
    atomicAdd(out, t);
  }
}

}  // namespace

hipError_t launch_fingerprint(const void* pos4, int fp64, const double* wsort, const int* perm,
                              const int* plist, const long long* nprim, int64_t n,
                              unsigned long long seed, unsigned long long* out, hipStream_t st) {
  const unsigned nb = std::min<unsigned>(kPrintBlocks, std::max(1u, blocks_for(n, 256)));
  hipLaunchKernelGGL(k_fingerprint, dim3(nb), dim3(256), 0, st,
                     static_cast<const unsigned*>(pos4), fp64 ? 8 : 4, wsort, perm, plist, nprim,
                     n, seed, out);
  return hipGetLastError();
}

size_t scan_tmp_bytes(int64_t count) {
  size_t total = 0;
  int64_t c = count;
  while (c > 1) {
    const int64_t tiles = (c + kScanTile - 1) / kScanTile;
    total += size_t(2 * tiles + 64) * sizeof(int);
    c = tiles;
  }
  return total + 256;
}

hipError_t launch_scan(const int* in, int* out, int64_t count, void* tmp, size_t tmp_bytes,
                       hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int64_t tiles = (count + kScanTile - 1) / kScanTile;
  int* sums = static_cast<int*>(tmp);
  int* offs = sums + tiles + 32;
  hipLaunchKernelGGL(k_scan_tiles, dim3(unsigned(tiles)), dim3(kScanBlock), 0, st, in, out,
                     count, sums);
  if (tiles > 1) {
    const size_t used = size_t(2 * tiles + 64) * sizeof(int);
    hipError_t e = launch_scan(sums, offs, tiles, static_cast<char*>(tmp) + used,
                               tmp_bytes - used, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3(blocks_for(count, 256)), dim3(256), 0, st, out, count,
                       offs);
  }
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int64_t count, int value, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(count, 256)), dim3(256), 0, st, p, count,
                     value);
  return hipGetLastError();
}

hipError_t launch_fill_double(double* p, int64_t count, double value, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_double, dim3(blocks_for(count, 256)), dim3(256), 0, st, p, count,
                     value);
  return hipGetLastError();
}

Grid make_grid(const g3pcf_problem& p) {
  Grid g{};
  g.periodic = p.periodic ? 1 : 0;
  // Margin so that every candidate the FP32 acceptance test can accept is
  // visited: positions carry about 1e-7 relative rounding.
  double ext = 0.0;
  for (int a = 0; a < 3; ++a)
    ext = std::max(ext, std::fabs(p.box_lo[a]) + std::fabs(p.box[a]));
  g.rsearch = p.rmax * (1.0 + 1e-5) + 1e-6 * ext + 1e-9;
  // Cells of about R_max / 8 across the rows and R_max / 64 along x: a row
  // (cy, cz) of cells is a contiguous run of galaxies, and the x-interval of
  // an annulus in a row is cut to within one thin cell at each end.
  const double target[3] = {p.rmax / 64.0, p.rmax / 8.0, p.rmax / 8.0};
  int64_t cap = std::max<int64_t>(64, 4 * p.n);
  cap = std::min<int64_t>(cap, int64_t(1) << 24);
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = p.box_lo[a];
    g.L[a] = p.box[a];
    double nc = std::floor(p.box[a] / target[a]);
    nc = std::max(1.0, std::min(nc, 4096.0));
    g.nc[a] = int(nc);
  }
  while (int64_t(g.nc[0]) * g.nc[1] * g.nc[2] > cap) {
    for (int a = 0; a < 3; ++a) g.nc[a] = std::max(1, (g.nc[a] * 4) / 5);
  }
  for (int a = 0; a < 3; ++a) {
    g.s[a] = g.L[a] / g.nc[a];
    g.inv_s[a] = double(g.nc[a]) / g.L[a];
    // periodic axis where [x - R, x + R] can touch more than nc cells
    g.tight[a] = (g.periodic && (2.0 * g.rsearch + 2.0 * g.s[a] >= g.L[a])) ? 1 : 0;
  }
  g.ncell = int64_t(g.nc[0]) * g.nc[1] * g.nc[2];
  return g;
}

size_t radix_hist_ints(int64_t n) {
  const int64_t ntiles = std::max<int64_t>(1, (n + kRadixTile - 1) / kRadixTile);
  return size_t(ntiles) * kRadixDigits;
}

hipError_t launch_cells(const g3pcf_problem& p, const Grid& g, const CellBufs& b, int fp64,
                        hipStream_t st) {
  const int64_t n = p.n;
  GridDev gd;
  for (int a = 0; a < 3; ++a) {
    gd.nc[a] = g.nc[a];
    gd.inv_s[a] = g.inv_s[a];
    gd.lo[a] = g.lo[a];
    gd.L[a] = g.L[a];
  }
  gd.periodic = g.periodic;
  hipError_t e = launch_fill_int(b.cell_count, g.ncell + 1, 0, st);
  if (e != hipSuccess) return e;
  if (n == 0) return launch_fill_int(b.cell_start, g.ncell + 1, 0, st);
  const unsigned nb = blocks_for(n, 256);
  // staged values (input order) into stage4, the cell id of every galaxy
  // into key_a, and the cell counts
  if (fp64) {
    if (p.pos_dtype == G3PCF_F64)
      hipLaunchKernelGGL((k_assign<double, double>), dim3(nb), dim3(256), 0, st,
                         static_cast<const double*>(p.pos), p.w, n, gd,
                         static_cast<double4*>(b.stage4), b.key_a, b.cell_count);
    else
      hipLaunchKernelGGL((k_assign<double, float>), dim3(nb), dim3(256), 0, st,
                         static_cast<const float*>(p.pos), p.w, n, gd,
                         static_cast<double4*>(b.stage4), b.key_a, b.cell_count);
  } else {
    if (p.pos_dtype == G3PCF_F64)
      hipLaunchKernelGGL((k_assign<float, double>), dim3(nb), dim3(256), 0, st,
                         static_cast<const double*>(p.pos), p.w, n, gd,
                         static_cast<float4*>(b.stage4), b.key_a, b.cell_count);
    else
      hipLaunchKernelGGL((k_assign<float, float>), dim3(nb), dim3(256), 0, st,
                         static_cast<const float*>(p.pos), p.w, n, gd,
                         static_cast<float4*>(b.stage4), b.key_a, b.cell_count);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // cell_start = exclusive scan of the counts (ncell + 1 entries, last = n)
  if ((e = launch_scan(b.cell_count, b.cell_start, g.ncell + 1, b.scan_tmp, b.scan_bytes, st)) !=
      hipSuccess)
    return e;
  // perm = input indices sorted stably by cell id
  int bits = 0;
  while ((int64_t(1) << bits) < g.ncell) ++bits;
  const int passes = std::max(1, (bits + kRadixBits - 1) / kRadixBits);
  const int ntiles = int((n + kRadixTile - 1) / kRadixTile);
  const int64_t nh = int64_t(ntiles) * kRadixDigits;
  int* hist = b.hist;
  int* offs = b.hist + nh;
  const int* kin = b.key_a;
  const int* vin = nullptr;
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = pass * kRadixBits;
    const bool last = pass + 1 == passes;
    int* kout = last ? nullptr : (kin == b.key_a ? b.key_b : b.key_a);
    // the last pass writes perm; the ones before alternate so that it does
    int* vout = ((passes - 1 - pass) % 2 == 0) ? b.perm : b.val_a;
    hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(kRadixThreads), 0, st, kin, n, shift,
                       ntiles, hist);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_scan(hist, offs, nh, b.scan_tmp, b.scan_bytes, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(kRadixThreads), 0, st, kin, vin, n,
                       shift, ntiles, offs, kout, vout);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    kin = kout;
    vin = vout;
  }
  // the gather also writes the kSentinel NaN entries after the catalogue
  const unsigned ng = blocks_for(n + kSentinel, 256);
  if (fp64)
    hipLaunchKernelGGL((k_gather_sorted<double4>), dim3(ng), dim3(256), 0, st,
                       static_cast<const double4*>(b.stage4), b.perm, n, p.w,
                       static_cast<double4*>(b.pos4), b.wsort);
  else
    hipLaunchKernelGGL((k_gather_sorted<float4>), dim3(ng), dim3(256), 0, st,
                       static_cast<const float4*>(b.stage4), b.perm, n, p.w,
                       static_cast<float4*>(b.pos4), b.wsort);
  return hipGetLastError();
}

hipError_t launch_primaries(const uint8_t* mask, const int32_t* region, int r, const int* perm,
                            int64_t n, int* flags, int* plist, long long* nprim,
                            void* scan_tmp, size_t scan_tmp_bytes_, hipStream_t st) {
  const unsigned nb = blocks_for(n + 1, 256);
  hipLaunchKernelGGL(k_primary_flags, dim3(nb), dim3(256), 0, st, mask, region, r, perm, n,
                     flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // positions: exclusive scan into flags + (n + 1)
  int* pos = flags + (n + 1);
  if ((e = launch_scan(flags, pos, n + 1, scan_tmp, scan_tmp_bytes_, st)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_primary_list, dim3(nb), dim3(256), 0, st, flags, pos, n, plist, nprim);
  return hipGetLastError();
}

}  // namespace g3
