// C ABI of libg3pcf: argument validation, workspace layout and the order of
// the stages on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <utility>

#include <vector>

#include "internal.h"

struct g3pcf_trace {
  int capacity = 0;
  int count = 0;
  int dropped = 0;
  std::vector<hipEvent_t> ev;  // start, stop per record
  std::vector<int> stage;
};

namespace g3 {
namespace {

// Records a start event now and a stop event when the scope ends.
struct StageScope {
  g3pcf_trace* t;
  hipStream_t st;
  int slot = -1;
  StageScope(g3pcf_trace* tr, int stg, hipStream_t s) : t(tr), st(s) {
    if (!t) return;
    if (t->count < t->capacity) {
      slot = t->count++;
      t->stage[slot] = stg;
      (void)hipEventRecord(t->ev[2 * slot], st);
    } else {
      ++t->dropped;
    }
  }
  ~StageScope() {
    if (slot >= 0) (void)hipEventRecord(t->ev[2 * slot + 1], st);
  }
};

thread_local std::string t_err;

int fail(int code, const std::string& msg) {
  t_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(G3PCF_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
constexpr size_t kCountersBytes = 1024;
size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Ws {
  size_t pos4, tmp4, cid, perm, tmp_perm, rkey, rhist, wsort, cell_start, cell_count, flags,
      plist, scan, counters, spill, A, C, gcoef, gsort, gsort32, mht, hrows, degD, degP;
  size_t scan_bytes;
  size_t total;
  int64_t PB;   // primaries per pair-block
  int spill_cap;  // spill-list entries per wave (0: none)
  Grid grid;
  RowLayout lay;
};

// Workspace layout.  pb_max caps the primaries of a pair-block (the a_lm rows
// held at once); spill = false leaves out the spill lists (a multi-chunk basis
// then repeats its search per chunk).
Ws plan(const g3pcf_problem& p, int backward, int64_t pb_max = kPairBlockMax,
        bool spill = true) {
  Ws w{};
  const int64_t n = p.n;
  const int fp64 = (p.pair_prec == G3PCF_PREC_FP64);
  const size_t rb = fp64 ? 32 : 16;
  w.grid = make_grid(p);
  w.lay = make_layout(p.lmax, p.nbins);
  const int64_t ncell = w.grid.ncell;
  w.PB = std::max<int64_t>(1, std::min<int64_t>(n, pb_max));
  const int64_t nhist = int64_t(radix_hist_ints(n));
  w.scan_bytes = scan_tmp_bytes(std::max<int64_t>(std::max<int64_t>(ncell + 1, n + 1), nhist));
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t o = at;
    at += up(std::max<size_t>(bytes, 1));
    return o;
  };
  w.pos4 = take(size_t(n + kSentinel) * rb);
  w.tmp4 = take(size_t(n) * rb);
  w.cid = take(size_t(n) * 4);
  w.perm = take(size_t(n) * 4);
  w.tmp_perm = take(size_t(n) * 4);
  w.rkey = take(size_t(n) * 4);
  w.rhist = take(size_t(2 * nhist) * 4);
  w.wsort = take(size_t(n) * 8);
  w.cell_start = take(size_t(ncell + 1) * 4);
  w.cell_count = take(size_t(ncell + 1) * 4);
  w.flags = take(size_t(2 * (n + 1)) * 4);
  w.plist = take(size_t(n) * 4);
  w.scan = take(w.scan_bytes);
  w.counters = take(kCountersBytes);
  // per-wave spill lists for bases accumulated in several register chunks
  const bool multi = spill && (fp64 || p.basis == G3PCF_BASIS_CARTESIAN);
  w.spill = take(multi ? size_t(kPairWaves) * kSpillCap * 4 : 0);
  w.spill_cap = multi ? kSpillCap : 0;
  w.A = take(size_t(w.PB) * w.lay.W * 8);
  w.C = take(zeta_partial_doubles(w.lay, w.PB) * 8);
  // degenerate triangles: per-shell Legendre sums and their per-workgroup partials
  const bool deg = !backward && p.distinct;
  w.degD = take(deg ? size_t(p.nbins) * (2 * p.lmax + 1) * 8 : 0);
  w.degP = take(deg ? deg_partial_doubles(w.PB, p.nbins, p.lmax) * 8 : 0);
  if (backward) {
    // adjoint coefficients per primary and shell in the forward's basis (FP64
    // pair path only: the FP32 adjoint pair kernel forms its spin-Chebyshev
    // coefficients from the H rows)
    const int T = (p.basis == G3PCF_BASIS_SPIN) ? kTermsSpin : kTermsCart;
    w.gcoef = take(fp64 ? size_t(w.PB) * p.nbins * T * 8 : 0);
    w.gsort = take(size_t(n) * 8);
    w.gsort32 = take(fp64 ? 0 : size_t(n) * 4);  // FP32 secondary terms (FP32 pair path)
    w.mht = take(adj_matrix_doubles(w.lay) * 8);
    w.hrows = take(size_t(w.PB) * w.lay.W * 8);
  }
  w.total = at;
  return w;
}

bool finite3(const double* v) {
  return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

int validate(const g3pcf_problem* p) {
  if (!p) return fail(G3PCF_EINVAL, "problem is NULL");
  // the pair kernels address the cell-ordered catalogue (16 or 32 bytes per
  // galaxy) with 32-bit byte offsets
  if (p->n < 0 || p->n >= (int64_t(1) << 27))
    return fail(G3PCF_EINVAL, "n must satisfy 0 <= n < 2^27");
  if (p->n > 0 && (!p->pos || !p->w)) return fail(G3PCF_EINVAL, "pos and w must be non-NULL");
  if (p->pos_dtype != G3PCF_F32 && p->pos_dtype != G3PCF_F64)
    return fail(G3PCF_EINVAL, "pos_dtype must be G3PCF_F32 or G3PCF_F64");
  if (!finite3(p->box) || !finite3(p->box_lo) || p->box[0] <= 0 || p->box[1] <= 0 ||
      p->box[2] <= 0)
    return fail(G3PCF_EINVAL, "box must be finite and positive, box_lo finite");
  if (!(p->rmax > 0) || !std::isfinite(p->rmax)) return fail(G3PCF_EINVAL, "rmax must be > 0");
  if (p->periodic) {
    const double mn = std::min(p->box[0], std::min(p->box[1], p->box[2]));
    if (p->rmax > 0.5 * mn)
      return fail(G3PCF_EINVAL, "periodic box needs rmax <= min(box) / 2");
  }
  if (p->nbins < 1 || p->nbins > kMaxBins) return fail(G3PCF_EINVAL, "nbins must be 1..32");
  if (p->lmax < 0 || p->lmax > kDeg) return fail(G3PCF_EINVAL, "lmax must be 0..10");
  if (p->los != G3PCF_LOS_Z && p->los != G3PCF_LOS_OBSERVER)
    return fail(G3PCF_EINVAL, "los must be G3PCF_LOS_Z or G3PCF_LOS_OBSERVER");
  if (p->los == G3PCF_LOS_OBSERVER && !finite3(p->observer))
    return fail(G3PCF_EINVAL, "observer must be finite");
  if (p->pair_prec != G3PCF_PREC_FP64 && p->pair_prec != G3PCF_PREC_FP32)
    return fail(G3PCF_EINVAL, "pair_prec must be G3PCF_PREC_FP64 or G3PCF_PREC_FP32");
  if (p->zeta_prec != G3PCF_PREC_FP64 && p->zeta_prec != G3PCF_PREC_FP32 &&
      p->zeta_prec != G3PCF_PREC_BF16X3)
    return fail(G3PCF_EINVAL, "zeta_prec must be FP64, FP32 or BF16X3");
  if (p->basis != G3PCF_BASIS_CARTESIAN && p->basis != G3PCF_BASIS_SPIN)
    return fail(G3PCF_EINVAL, "basis must be G3PCF_BASIS_CARTESIAN or G3PCF_BASIS_SPIN");
  if (p->distinct != 0 && p->distinct != 1)
    return fail(G3PCF_EINVAL, "distinct must be 0 or 1");
  if (p->accumulate != 0 && p->accumulate != 1)
    return fail(G3PCF_EINVAL, "accumulate must be 0 or 1");
  return G3PCF_OK;
}

std::mutex g_tab_mu;
std::set<std::pair<int, int>> g_tab_done;

int ensure_tables(int basis) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_tab_mu);
  if (g_tab_done.count({dev, basis})) return G3PCF_OK;
  e = (basis == kBasisDeg) ? upload_deg_table() : upload_tables(basis);
  if (e != hipSuccess) return hip_fail(e, "table upload");
  g_tab_done.insert({dev, basis});
  return G3PCF_OK;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

struct Counters {
  long long nprim;
  unsigned long long pairs;
  unsigned long long pairs_adj;
  unsigned long long pairs_deg;  // counted again by the degenerate-triangle pass
  unsigned long long inputs_hash;  // backward: fingerprint of its inputs (a_lm store check)
  int pad[6];
  int queue[kQueues * kQueueStride];  // one primary counter per XCD, 64 B apart
};
static_assert(sizeof(Counters) <= kCountersBytes, "counters block");

// Stages shared by forward and backward: cell list and primary list.
int stage_catalogue(const g3pcf_problem& p, const Ws& w, void* ws, hipStream_t st) {
  const int fp64 = (p.pair_prec == G3PCF_PREC_FP64);
  CellBufs b{};
  b.pos4 = at<void>(ws, w.pos4);
  b.stage4 = at<void>(ws, w.tmp4);
  b.cell_start = at<int>(ws, w.cell_start);
  b.cell_count = at<int>(ws, w.cell_count);
  b.key_a = at<int>(ws, w.cid);
  b.key_b = at<int>(ws, w.rkey);
  b.val_a = at<int>(ws, w.tmp_perm);
  b.perm = at<int>(ws, w.perm);
  b.hist = at<int>(ws, w.rhist);
  b.wsort = at<double>(ws, w.wsort);
  b.scan_tmp = at<void>(ws, w.scan);
  b.scan_bytes = w.scan_bytes;
  hipError_t e = launch_cells(p, w.grid, b, fp64, st);
  if (e != hipSuccess) return hip_fail(e, "cell list");
  Counters* c = at<Counters>(ws, w.counters);
  e = launch_fill_int(reinterpret_cast<int*>(c), sizeof(Counters) / 4, 0, st);
  if (e != hipSuccess) return hip_fail(e, "counters");
  e = launch_primaries(p.primary_mask, nullptr, 0, at<int>(ws, w.perm), p.n,
                       at<int>(ws, w.flags), at<int>(ws, w.plist), &c->nprim, at<void>(ws, w.scan),
                       w.scan_bytes, st);
  if (e != hipSuccess) return hip_fail(e, "primary list");
  return G3PCF_OK;
}

PairArgs pair_args(const g3pcf_problem& p, const Ws& w, void* ws) {
  PairArgs a{};
  Counters* c = at<Counters>(ws, w.counters);
  a.pos4 = at<void>(ws, w.pos4);
  a.sentinel = int(p.n);
  a.cell_start = at<int>(ws, w.cell_start);
  a.plist = at<int>(ws, w.plist);
  a.nprim = &c->nprim;
  a.spill = at<int>(ws, w.spill);
  a.spill_cap = w.spill_cap;
  a.queue = c->queue;
  a.pairs = &c->pairs;
  for (int k = 0; k < 3; ++k) {
    a.nc[k] = w.grid.nc[k];
    a.s[k] = w.grid.s[k];
    a.inv_s[k] = w.grid.inv_s[k];
    a.lo[k] = w.grid.lo[k];
    a.L[k] = w.grid.L[k];
    a.tight[k] = w.grid.tight[k];
    a.obs[k] = p.observer[k];
  }
  a.periodic = w.grid.periodic;
  a.rmax = p.rmax;
  a.rmax_search = w.grid.rsearch;
  // squared shell edges rounded to float; the lower bound is exclusive, so it
  // is the float just below the edge (0 for the innermost shell, r > 0)
  for (int b = 0; b < p.nbins; ++b) {
    const double e0 = b * p.rmax / p.nbins, e1 = (b + 1) * p.rmax / p.nbins;
    const float t0 = float(e0 * e0);
    a.r2_lo[b] = (b == 0) ? 0.0f : std::nextafter(t0, 0.0f);
    a.r2_hi[b] = (b + 1 == p.nbins) ? float(p.rmax * p.rmax) : float(e1 * e1);
  }
  a.nbins = p.nbins;
  a.lmax = p.lmax;
  a.los = p.los;
  a.A = at<double>(ws, w.A);
  a.lay = w.lay;
  a.perm = at<int>(ws, w.perm);
  a.wsort = at<double>(ws, w.wsort);
  return a;
}

int check_workspace(const Ws& w, void* ws, size_t ws_bytes) {
  if (!ws || ws_bytes < w.total)
    return fail(G3PCF_EWORKSPACE, "workspace needs " + std::to_string(w.total) + " bytes");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign)
    return fail(G3PCF_EWORKSPACE, "workspace must be 256-byte aligned");
  return G3PCF_OK;
}

// The a_lm store: a 256-byte header (the fingerprint of the forward pass's
// inputs) and then one row of W doubles per primary in primary-list order.
constexpr size_t kAlmHeader = 256;

size_t alm_total(const g3pcf_problem& p, const RowLayout& lay) {
  return kAlmHeader + size_t(p.n) * size_t(lay.W) * 8;
}

int check_alm(const g3pcf_problem& p, const Ws& w) {
  if (!p.alm) return G3PCF_OK;
  const size_t need = alm_total(p, w.lay);
  if (p.alm_bytes < need)
    return fail(G3PCF_EWORKSPACE, "alm store needs " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(p.alm) % kAlign)
    return fail(G3PCF_EWORKSPACE, "alm store must be 256-byte aligned");
  return G3PCF_OK;
}

double* alm_rows(const g3pcf_problem& p) {
  return reinterpret_cast<double*>(static_cast<char*>(p.alm) + kAlmHeader);
}

// splitmix64 output function (Steele, Lea and Flood, OOPSLA 2014), host side
uint64_t hmix(uint64_t x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

// Hash of the settings that change the a_lm rows (zeta_prec, accumulate and
// the output pointers do not).
uint64_t settings_seed(const g3pcf_problem& p) {
  uint64_t h = hmix(0x6733706366ull + uint64_t(p.n));
  auto put_d = [&](double v) {
    uint64_t b;
    std::memcpy(&b, &v, 8);
    h = hmix(h ^ b);
  };
  auto put_i = [&](int64_t v) { h = hmix(h ^ uint64_t(v)); };
  for (int k = 0; k < 3; ++k) {
    put_d(p.box[k]);
    put_d(p.box_lo[k]);
    put_d(p.los == G3PCF_LOS_OBSERVER ? p.observer[k] : 0.0);
  }
  put_d(p.rmax);
  put_i(p.periodic);
  put_i(p.nbins);
  put_i(p.lmax);
  put_i(p.los);
  put_i(p.pair_prec);
  put_i(p.basis);
  put_i(p.pos_dtype);
  return h;
}

hipError_t fingerprint(const g3pcf_problem& p, const Ws& w, void* ws, unsigned long long* out,
                       hipStream_t st) {
  hipError_t e = launch_fill_int(reinterpret_cast<int*>(out), 2, 0, st);
  if (e != hipSuccess) return e;
  Counters* c = at<Counters>(ws, w.counters);
  return launch_fingerprint(at<void>(ws, w.pos4), p.pair_prec == G3PCF_PREC_FP64,
                            at<double>(ws, w.wsort), at<int>(ws, w.perm), at<int>(ws, w.plist),
                            &c->nprim, p.n, settings_seed(p), out, st);
}

int forward_tables(const g3pcf_problem& p) {
  int rc = ensure_tables(conv_table_of(p.basis));
  if (!rc && p.distinct) rc = ensure_tables(kBasisDeg);
  return rc;
}

// The pair-blocks of the current primary list (at most `cover` primaries):
// pair kernel, Gram products into zeta, and (distinct) the degenerate-triangle
// pass and its correction.  rows: where the a_lm rows go (NULL: the
// workspace's pair-block rows; else rows of every primary, kept).
int forward_pairs(const g3pcf_problem& p, const Ws& w, void* ws, double* zeta, int64_t cover,
                  double* rows, hipStream_t st) {
  hipError_t e;
  PairArgs a = pair_args(p, w, ws);
  const int fp64 = (p.pair_prec == G3PCF_PREC_FP64);
  Counters* c = at<Counters>(ws, w.counters);
  double* degD = at<double>(ws, w.degD);
  if (p.distinct &&
      (e = launch_fill_double(degD, int64_t(p.nbins) * (2 * p.lmax + 1), 0.0, st)) != hipSuccess)
    return hip_fail(e, "degenerate sums clear");
  for (int64_t b0 = 0; b0 < cover; b0 += w.PB) {
    a.p_begin = b0;
    a.p_count = std::min<int64_t>(w.PB, cover - b0);
    a.pairs = &c->pairs;
    if (rows) a.A = rows + size_t(b0) * w.lay.W;
    {
      StageScope sc(p.trace, G3PCF_STAGE_PAIRS, st);
      if ((e = launch_pair_forward(a, fp64, p.basis, st)) != hipSuccess)
        return hip_fail(e, "pair kernel");
    }
    {
      StageScope scz(p.trace, G3PCF_STAGE_ZETA, st);
      ZetaArgs z{};
      z.A = a.A;
      z.wsort = a.wsort;
      z.plist = a.plist;
      z.nprim = &c->nprim;
      z.row_begin = b0;
      z.sub_begin = 0;
      z.K = a.p_count;
      z.lay = w.lay;
      z.C64 = at<double>(ws, w.C);
      z.zeta = zeta;
      z.prec = p.zeta_prec;
      if ((e = launch_zeta_pairblock(z, st)) != hipSuccess) return hip_fail(e, "zeta");
    }
    if (p.distinct) {
      // the same pairs again for their sums w_j^2 P_n(u_z), written over the
      // pair-block's A rows (already reduced into zeta), then summed with w_i
      StageScope scd(p.trace, G3PCF_STAGE_DISTINCT, st);
      a.pairs = &c->pairs_deg;
      if ((e = launch_pair_distinct(a, fp64, st)) != hipSuccess)
        return hip_fail(e, "degenerate-triangle pass");
      if ((e = launch_deg_reduce(a.A, w.lay.W, p.nbins, p.lmax, a.wsort, a.plist, &c->nprim, b0,
                                 a.p_count, at<double>(ws, w.degP), degD, st)) != hipSuccess)
        return hip_fail(e, "degenerate-triangle sums");
    }
  }
  if (p.distinct) {
    StageScope scd(p.trace, G3PCF_STAGE_DISTINCT, st);
    if ((e = launch_deg_apply(degD, p.lmax, p.nbins, zeta, st)) != hipSuccess)
      return hip_fail(e, "degenerate-triangle correction");
  }
  return G3PCF_OK;
}

// pairs_out from the forward count (or, adj = true, the adjoint pass's count)
int finish_pairs(const g3pcf_problem& p, const Ws& w, void* ws, hipStream_t st,
                 bool adj = false) {
  if (!p.pairs_out) return G3PCF_OK;
  unsigned long long host = 0;
  Counters* c = at<Counters>(ws, w.counters);
  hipError_t e = hipMemcpyAsync(&host, adj ? &c->pairs_adj : &c->pairs, sizeof(host),
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "pair count read-back");
  *p.pairs_out = (int64_t)host;
  return G3PCF_OK;
}

// The forward pass in a workspace laid out by `w` (already checked).
int forward_run(const g3pcf_problem& p, const Ws& w, double* zeta, void* ws, hipStream_t st) {
  int rc;
  if (p.alm && p.distinct)
    return fail(G3PCF_EINVAL, "alm store with distinct = 1 (the adjoint does not cover it)");
  if ((rc = check_alm(p, w))) return rc;
  if ((rc = forward_tables(p))) return rc;
  const size_t zlen = g3pcf_zeta_len(p.lmax, p.nbins);
  hipError_t e;
  if (!p.accumulate && (e = launch_fill_double(zeta, int64_t(zlen), 0.0, st)) != hipSuccess)
    return hip_fail(e, "zeta clear");
  if (p.n == 0) {
    if (p.alm && (e = launch_fill_int(static_cast<int*>(p.alm), 2, 0, st)) != hipSuccess)
      return hip_fail(e, "alm store header");
    if (p.pairs_out) *p.pairs_out = 0;
    return G3PCF_OK;
  }
  {
    StageScope sc(p.trace, G3PCF_STAGE_CELLS, st);
    if ((rc = stage_catalogue(p, w, ws, st))) return rc;
    if (p.alm && (e = fingerprint(p, w, ws, static_cast<unsigned long long*>(p.alm), st)) !=
                     hipSuccess)
      return hip_fail(e, "alm store fingerprint");
  }
  if ((rc = forward_pairs(p, w, ws, zeta, p.n, p.alm ? alm_rows(p) : nullptr, st))) return rc;
  return finish_pairs(p, w, ws, st);
}


// Scratch of the allocation-free entry point g3pcf_forward_noalloc: one
// array per device, held until the process ends.  In host code the array's
// name is a stand-in only; its device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kScratchBytes = size_t(128) << 20;
// Primaries per pair-block in the scratch (one zeta block of 4096 rows).
constexpr int64_t kScratchPairBlock = kZetaBlock;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;

int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr || reinterpret_cast<uintptr_t>(ptr) % kAlign)
      return fail(G3PCF_EHIP, "scratch array has no usable device address");
    it = g_scratch_ptr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return G3PCF_OK;
}

}  // namespace
}  // namespace g3

using namespace g3;

extern "C" {

size_t g3pcf_zeta_len(int lmax, int nbins) {
  if (lmax < 0 || nbins < 1) return 0;
  const size_t L1 = size_t(lmax) + 1;
  return L1 * L1 * L1 * size_t(nbins) * size_t(nbins) * 2;
}

int g3pcf_num_terms(int basis) {
  if (basis == G3PCF_BASIS_CARTESIAN) return kTermsCart;
  if (basis == G3PCF_BASIS_SPIN) return kTermsSpin;
  return -1;
}

const char* g3pcf_last_error(void) { return t_err.c_str(); }

g3pcf_trace* g3pcf_trace_create(int capacity) {
  if (capacity < 1) {
    fail(G3PCF_EINVAL, "trace capacity must be >= 1");
    return nullptr;
  }
  g3pcf_trace* t = new g3pcf_trace;
  t->capacity = capacity;
  t->ev.assign(2 * size_t(capacity), nullptr);
  t->stage.assign(size_t(capacity), -1);
  for (auto& e : t->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      g3pcf_trace_destroy(t);
      fail(G3PCF_EHIP, "hipEventCreate failed");
      return nullptr;
    }
  }
  return t;
}

void g3pcf_trace_reset(g3pcf_trace* t) {
  if (!t) return;
  t->count = 0;
  t->dropped = 0;
}

int g3pcf_trace_read(g3pcf_trace* t, int* stage, float* ms, int max, int* dropped) {
  if (!t || !stage || !ms || max < 0) return fail(G3PCF_EINVAL, "NULL trace or output");
  const int n = std::min(max, t->count);
  for (int k = 0; k < n; ++k) {
    float v = 0.f;
    hipError_t e = hipEventElapsedTime(&v, t->ev[2 * k], t->ev[2 * k + 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    stage[k] = t->stage[k];
    ms[k] = v;
  }
  if (dropped) *dropped = t->dropped;
  return n;
}

void g3pcf_trace_destroy(g3pcf_trace* t) {
  if (!t) return;
  for (auto& e : t->ev)
    if (e) (void)hipEventDestroy(e);
  delete t;
}

int g3pcf_workspace_bytes(const g3pcf_problem* prob, int backward, size_t* bytes) {
  int rc = validate(prob);
  if (rc) return rc;
  if (!bytes) return fail(G3PCF_EINVAL, "bytes is NULL");
  if (backward != 0 && backward != 1) return fail(G3PCF_EINVAL, "backward must be 0 or 1");
  *bytes = plan(*prob, backward).total;
  return G3PCF_OK;
}

int g3pcf_alm_bytes(const g3pcf_problem* prob, size_t* bytes) {
  int rc = validate(prob);
  if (rc) return rc;
  if (!bytes) return fail(G3PCF_EINVAL, "bytes is NULL");
  *bytes = alm_total(*prob, make_layout(prob->lmax, prob->nbins));
  return G3PCF_OK;
}

int g3pcf_forward(const g3pcf_problem* prob, double* zeta, void* ws, size_t ws_bytes,
                  void* stream) {
  int rc = validate(prob);
  if (rc) return rc;
  if (!zeta) return fail(G3PCF_EINVAL, "zeta is NULL");
  const Ws w = plan(*prob, 0);
  if ((rc = check_workspace(w, ws, ws_bytes))) return rc;
  return forward_run(*prob, w, zeta, ws, static_cast<hipStream_t>(stream));
}

int g3pcf_forward_noalloc(const g3pcf_problem* prob, double* zeta, void* stream) {
  int rc = validate(prob);
  if (rc) return rc;
  if (!zeta) return fail(G3PCF_EINVAL, "zeta is NULL");
  const Ws w = plan(*prob, 0, kScratchPairBlock, false);
  if (w.total > kScratchBytes)
    return fail(G3PCF_EINVAL, "g3pcf_forward_noalloc: this problem needs " +
                                  std::to_string(w.total) + " bytes of scratch, the library "
                                  "holds " + std::to_string(kScratchBytes) +
                                  " (use g3pcf_forward with a workspace)");
  void* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  return forward_run(*prob, w, zeta, ws, static_cast<hipStream_t>(stream));
}


int g3pcf_forward_regions(const g3pcf_problem* prob, const int32_t* region, int nregions,
                          double* zeta, void* ws, size_t ws_bytes, void* stream) {
  int rc = validate(prob);
  if (rc) return rc;
  if (nregions < 1 || nregions > (1 << 20)) return fail(G3PCF_EINVAL, "nregions must be 1..2^20");
  if (!zeta) return fail(G3PCF_EINVAL, "zeta is NULL");
  if (!region && prob->n > 0) return fail(G3PCF_EINVAL, "region is NULL");
  if (prob->alm) return fail(G3PCF_EINVAL, "alm store is not kept per region (set it to NULL)");
  const g3pcf_problem& p = *prob;
  const Ws w = plan(p, 0);
  if ((rc = check_workspace(w, ws, ws_bytes))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = forward_tables(p))) return rc;
  const size_t zlen = g3pcf_zeta_len(p.lmax, p.nbins);
  hipError_t e;
  if (!p.accumulate &&
      (e = launch_fill_double(zeta, int64_t(zlen) * nregions, 0.0, st)) != hipSuccess)
    return hip_fail(e, "zeta clear");
  if (p.n == 0) {
    if (p.pairs_out) *p.pairs_out = 0;
    return G3PCF_OK;
  }
  {
    StageScope sc(p.trace, G3PCF_STAGE_CELLS, st);
    if ((rc = stage_catalogue(p, w, ws, st))) return rc;
  }
  // one cell list; per region its own primary list and pair-blocks, sized by
  // the region's primary count (read back: one wait per region)
  Counters* c = at<Counters>(ws, w.counters);
  for (int r = 0; r < nregions; ++r) {
    long long count = 0;
    {
      StageScope sc(p.trace, G3PCF_STAGE_CELLS, st);
      if ((e = launch_primaries(p.primary_mask, region, r, at<int>(ws, w.perm), p.n,
                                at<int>(ws, w.flags), at<int>(ws, w.plist), &c->nprim,
                                at<void>(ws, w.scan), w.scan_bytes, st)) != hipSuccess)
        return hip_fail(e, "region primary list");
    }
    if ((e = hipMemcpyAsync(&count, &c->nprim, sizeof(count), hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return hip_fail(e, "region primary count");
    if (count > 0 && (rc = forward_pairs(p, w, ws, zeta + zlen * size_t(r), count, nullptr, st)))
      return rc;
  }
  return finish_pairs(p, w, ws, st);
}

int g3pcf_forward_batch(const g3pcf_problem* prob, int ncat, const int64_t* offsets,
                        double* zeta, void* ws, size_t ws_bytes, void* stream) {
  int rc = validate(prob);
  if (rc) return rc;
  if (ncat < 1 || ncat > (1 << 20)) return fail(G3PCF_EINVAL, "ncat must be 1..2^20");
  if (!offsets || !zeta) return fail(G3PCF_EINVAL, "offsets and zeta must be non-NULL");
  if (offsets[0] != 0 || offsets[ncat] != prob->n)
    return fail(G3PCF_EINVAL, "offsets must start at 0 and end at n");
  for (int c = 0; c < ncat; ++c)
    if (offsets[c + 1] < offsets[c]) return fail(G3PCF_EINVAL, "offsets must not decrease");
  if (prob->alm) return fail(G3PCF_EINVAL, "alm store is not kept per catalogue (set it to NULL)");
  const g3pcf_problem& p = *prob;
  if ((rc = check_workspace(plan(p, 0), ws, ws_bytes))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = forward_tables(p))) return rc;
  const size_t zlen = g3pcf_zeta_len(p.lmax, p.nbins);
  hipError_t e;
  if (!p.accumulate &&
      (e = launch_fill_double(zeta, int64_t(zlen) * ncat, 0.0, st)) != hipSuccess)
    return hip_fail(e, "zeta clear");
  const size_t pos_row = (p.pos_dtype == G3PCF_F32 ? 4 : 8) * 3;
  int64_t total = 0;
  // one catalogue after another in the same workspace, in stream order (no
  // host synchronisation unless pairs_out asks for the counts)
  for (int c = 0; c < ncat; ++c) {
    g3pcf_problem q = p;
    q.n = offsets[c + 1] - offsets[c];
    if (q.n == 0) continue;
    q.pos = static_cast<const char*>(p.pos) + size_t(offsets[c]) * pos_row;
    q.w = p.w + offsets[c];
    q.primary_mask = p.primary_mask ? p.primary_mask + offsets[c] : nullptr;
    int64_t pairs_c = 0;
    q.pairs_out = p.pairs_out ? &pairs_c : nullptr;
    const Ws w = plan(q, 0);
    if ((rc = check_workspace(w, ws, ws_bytes))) return rc;
    {
      StageScope sc(p.trace, G3PCF_STAGE_CELLS, st);
      if ((rc = stage_catalogue(q, w, ws, st))) return rc;
    }
    if ((rc = forward_pairs(q, w, ws, zeta + zlen * size_t(c), q.n, nullptr, st))) return rc;
    if ((rc = finish_pairs(q, w, ws, st))) return rc;
    total += pairs_c;
  }
  if (p.pairs_out) *p.pairs_out = total;
  return G3PCF_OK;
}

int g3pcf_backward(const g3pcf_problem* prob, const double* grad_zeta, double* grad_w, void* ws,
                   size_t ws_bytes, void* stream) {
  int rc = validate(prob);
  if (rc) return rc;
  if (!grad_zeta || (!grad_w && prob->n > 0))
    return fail(G3PCF_EINVAL, "grad_zeta and grad_w must be non-NULL");
  if (prob->distinct)
    return fail(G3PCF_EUNSUPPORTED, "the adjoint does not cover distinct = 1");
  const g3pcf_problem& p = *prob;
  const Ws w = plan(p, 1);
  if ((rc = check_workspace(w, ws, ws_bytes))) return rc;
  if ((rc = check_alm(p, w))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the FP32 adjoint (either basis) evaluates its per-pair polynomial in
  // (x - i y)^m T_n(z) (coefficients from the spin-Chebyshev table); the
  // FP64 adjoint in the forward's own basis
  const bool fp32 = (p.pair_prec == G3PCF_PREC_FP32);
  const int adj_table = fp32 ? int(G3PCF_BASIS_SPIN_T) : conv_table_of(p.basis);
  const int adj_basis = fp32 ? int(G3PCF_BASIS_SPIN) : int(p.basis);
  if ((rc = ensure_tables(conv_table_of(p.basis))) || (rc = ensure_tables(adj_table)))
    return rc;
  if (p.n == 0) {
    if (p.pairs_out) *p.pairs_out = 0;
    return G3PCF_OK;
  }
  hipError_t e;
  Counters* c = at<Counters>(ws, w.counters);
  {
    StageScope sc(p.trace, G3PCF_STAGE_CELLS, st);
    if ((rc = stage_catalogue(p, w, ws, st))) return rc;
    if (p.alm && (e = fingerprint(p, w, ws, &c->inputs_hash, st)) != hipSuccess)
      return hip_fail(e, "input fingerprint");
  }
  double* gsort = at<double>(ws, w.gsort);
  if ((e = launch_fill_double(gsort, p.n, 0.0, st)) != hipSuccess)
    return hip_fail(e, "gradient clear");
  // FP32 pair path: the secondary terms are summed in FP32 on their own array
  float* gsort32 = (p.pair_prec == G3PCF_PREC_FP64) ? nullptr : at<float>(ws, w.gsort32);
  if (gsort32 && (e = launch_fill_int(reinterpret_cast<int*>(gsort32), p.n, 0, st)) != hipSuccess)
    return hip_fail(e, "gradient clear");
  {
    StageScope sc(p.trace, G3PCF_STAGE_ADJ_COEF, st);
    if ((e = launch_adj_matrix(grad_zeta, w.lay, at<double>(ws, w.mht), st)) != hipSuccess)
      return hip_fail(e, "adjoint matrices");
  }
  PairArgs a = pair_args(p, w, ws);
  const int fp64 = (p.pair_prec == G3PCF_PREC_FP64);
  const ConvTable* tab = nullptr;
  if ((e = conv_table_device(adj_table, &tab)) != hipSuccess) return hip_fail(e, "table address");
  a.gcoef = at<double>(ws, w.gcoef);
  a.H = at<double>(ws, w.hrows);
  a.grad_w = gsort;
  a.grad_w32 = gsort32;
  for (int64_t b0 = 0; b0 < p.n; b0 += w.PB) {
    a.p_begin = b0;
    a.p_count = std::min<int64_t>(w.PB, p.n - b0);
    a.pairs = &c->pairs;
    if (p.alm) {
      // the a_lm rows the forward pass kept
      a.A = alm_rows(p) + size_t(b0) * w.lay.W;
    } else {
      StageScope sc(p.trace, G3PCF_STAGE_PAIRS, st);
      if ((e = launch_pair_forward(a, fp64, p.basis, st)) != hipSuccess)
        return hip_fail(e, "pair kernel (recompute)");
    }
    AdjArgs j{};
    j.A = a.A;
    j.gz = grad_zeta;
    j.wsort = a.wsort;
    j.plist = a.plist;
    j.perm = a.perm;
    j.nprim = &c->nprim;
    j.p_begin = b0;
    j.p_count = a.p_count;
    j.lay = w.lay;
    j.basis = adj_basis;
    j.table = tab;
    j.gcoef = at<double>(ws, w.gcoef);
    j.grad_w = gsort;
    j.MHt = at<double>(ws, w.mht);
    j.H = at<double>(ws, w.hrows);
    {
      StageScope sc(p.trace, G3PCF_STAGE_ADJ_COEF, st);
      if ((e = launch_h_gemm(j, st)) != hipSuccess) return hip_fail(e, "adjoint GEMM");
      if (fp64 && (e = launch_adj_finish(j, st)) != hipSuccess)
        return hip_fail(e, "adjoint coefficients");
    }
    a.pairs = &c->pairs_adj;
    {
      StageScope sc(p.trace, G3PCF_STAGE_PAIR_ADJOINT, st);
      if ((e = launch_pair_adjoint(a, fp64, p.basis, st)) != hipSuccess)
        return hip_fail(e, "pair adjoint kernel");
    }
  }
  const unsigned long long* saved = p.alm ? static_cast<const unsigned long long*>(p.alm) : nullptr;
  if ((e = launch_unpermute(gsort, gsort32, a.perm, p.n, p.accumulate, saved, &c->inputs_hash, grad_w,
                            st)) != hipSuccess)
    return hip_fail(e, "gradient permute");
  return finish_pairs(p, w, ws, st, true);
}

int g3pcf_isotropic(int lmax, int nbins, const double* zeta, double* iso, void* stream) {
  if (lmax < 0 || lmax > kDeg) return fail(G3PCF_EINVAL, "lmax must be 0..10");
  if (nbins < 1 || nbins > kMaxBins) return fail(G3PCF_EINVAL, "nbins must be 1..32");
  if (!zeta || !iso) return fail(G3PCF_EINVAL, "zeta and iso must be non-NULL");
  const hipError_t e = launch_isotropic(zeta, lmax, nbins, iso, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? G3PCF_OK : hip_fail(e, "isotropic");
}

int g3pcf_degenerate_term(int lmax, double uz, double* out) {
  if (lmax < 0 || lmax > kDeg || !out) return fail(G3PCF_EINVAL, "lmax 0..10 and out required");
  static std::vector<double> G;
  static std::mutex mu;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (G.empty()) {
      G.resize(kDegTable);
      build_deg_table(G.data());
    }
  }
  double pn[kTermsDeg];
  pn[0] = 1.0;
  pn[1] = uz;
  for (int n = 1; n + 1 < kTermsDeg; ++n)
    pn[n + 1] = ((2.0 * n + 1.0) * uz * pn[n] - n * pn[n - 1]) / (n + 1.0);
  const int L1 = lmax + 1;
  for (int m = 0; m <= lmax; ++m)
    for (int l = 0; l <= lmax; ++l)
      for (int lp = 0; lp <= lmax; ++lp) {
        double s = 0.0;
        if (l >= m && lp >= m)
          for (int n = 0; n <= l + lp; ++n) s += G[deg_index(m, l, lp, n)] * pn[n];
        out[(m * L1 + l) * L1 + lp] = s;
      }
  return G3PCF_OK;
}

}  // extern "C"
