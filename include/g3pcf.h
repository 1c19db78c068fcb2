/*
 * g3pcf: anisotropic three-point correlation function multipoles on one
 * AMD Instinct MI355X (gfx950).
 *
 * For every primary galaxy i the library gathers its secondaries j within
 * R_max, rotates each separation into the line-of-sight frame of i, bins it
 * into one of nbins equal-width radial shells and accumulates
 *
 *     a^{(i)}_{lm}(b) = sum_{j in shell b} w_j conj(Y_lm(u_ij))
 *
 * through sums of monomials of the unit separation (paper: Sec. 3.1 and its
 * eq. 1; Algorithm 1), converts the monomial sums to spherical-harmonic
 * coefficients in FP64, and reduces
 *
 *     zeta^m_{l l'}(b1, b2) = sum_i w_i a^{(i)}_{lm}(b1) conj(a^{(i)}_{l'm}(b2))
 *
 * over all primaries (the per-primary product a_lm(r1) a*_l'm(r2) of Sec. 3.1,
 * summed over primaries as the expansion zeta = sum zeta^m_{ll'} Y_lm Y*_l'm
 * requires).  The projection uses conj(Y_lm) so that zeta is the coefficient
 * of Y_lm(r1) Y*_l'm(r2) in that expansion.  Y_lm is orthonormal with the
 * Condon-Shortley phase (zeta does not depend on the phase convention).
 *
 * Conventions shared by every entry point
 *   - Every pointer is a DEVICE pointer unless its comment says HOST.
 *   - The caller owns all memory.  The library keeps no allocation between
 *     calls; scratch lives in the caller's workspace `ws` (except for
 *     g3pcf_forward_noalloc, whose scratch is a static device array).
 *   - Arguments are validated synchronously, before anything is enqueued; an
 *     invalid call returns a negative g3pcf_status and enqueues nothing.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *     default stream).  The call returns without synchronising unless
 *     `pairs_out` is set.
 *   - Calls are reentrant given distinct workspaces.  Two calls that share a
 *     workspace must be ordered on one stream.
 *   - g3pcf_last_error() returns a thread-local message for the last non-OK
 *     return on the calling thread.
 */
#ifndef G3PCF_H
#define G3PCF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  G3PCF_OK = 0,
  G3PCF_EINVAL = -1,       /* an argument is out of range or inconsistent     */
  G3PCF_EWORKSPACE = -2,   /* ws is NULL or smaller than g3pcf_workspace_bytes */
  G3PCF_EHIP = -3,         /* a HIP runtime call or kernel launch failed       */
  G3PCF_EUNSUPPORTED = -4  /* valid request this build does not implement      */
} g3pcf_status;

typedef enum {
  G3PCF_LOS_Z = 0,        /* line of sight = box z axis for every primary      */
  G3PCF_LOS_OBSERVER = 1  /* line of sight from `observer` through the primary;
                             each separation is rotated so that this line maps
                             to +z (Sec. 3.1, Fig. 2)                           */
} g3pcf_los;

typedef enum {
  G3PCF_PREC_FP64 = 0,    /* plain FP64 throughout                             */
  G3PCF_PREC_FP32 = 1,    /* pair stage: FP32 accumulation (the adjoint also sums
                             each galaxy's secondary terms in FP32); zeta stage:
                             FP32 MFMA                                            */
  G3PCF_PREC_BF16X3 = 2   /* zeta stage only: each FP32 operand split into three
                             bfloat16 terms, the six products with i+j <= 2 on
                             BF16 MFMA with FP32 accumulation                   */
} g3pcf_prec;

typedef enum { G3PCF_F32 = 0, G3PCF_F64 = 1 } g3pcf_dtype;

typedef enum {
  G3PCF_BASIS_CARTESIAN = 0, /* the paper's monomials (dx/r)^k (dy/r)^p (dz/r)^q,
                                k+p+q <= 10: 286 sums per shell (eq. 1)          */
  G3PCF_BASIS_SPIN = 1,      /* (dx/r - i dy/r)^m T_n(dz/r), m+n <= 10, with the
                                Chebyshev polynomials T_n: 121 real sums per
                                shell; the same zeta with fewer FMAs.  T_n in
                                place of the powers (dz/r)^n (the same span)
                                keeps the conversion to Y_lm free of the
                                cancellation that costs FP32 sums up to three
                                digits at l = 10                                 */
  G3PCF_BASIS_SPIN_T = 2     /* diagnostic only (g3pcf_conj_ylm_via_monomials),
                                not a problem setting: the table of the spin
                                basis above, (dx/r - i dy/r)^m T_n(dz/r); with
                                G3PCF_BASIS_SPIN the diagnostic evaluates the
                                plain powers (dx/r - i dy/r)^m (dz/r)^n instead  */
} g3pcf_basis;

/* Stages reported by a trace (see g3pcf_trace_create). */
typedef enum {
  G3PCF_STAGE_CELLS = 0,        /* wrap, cell assignment, counting sort, primaries */
  G3PCF_STAGE_PAIRS = 1,        /* pair kernel: search, rotate, bin, accumulate, convert */
  G3PCF_STAGE_ZETA = 2,         /* Gram products on MFMA + FP64 accumulation       */
  G3PCF_STAGE_ADJ_COEF = 3,     /* adjoint: U, V, H and monomial coefficients      */
  G3PCF_STAGE_PAIR_ADJOINT = 4, /* adjoint pair kernel: polynomial + scatter        */
  G3PCF_STAGE_DISTINCT = 5      /* degenerate-triangle pass, sums and correction   */
} g3pcf_stage;

/* Opaque record of per-stage GPU time.  Created on the current device. */
typedef struct g3pcf_trace g3pcf_trace;

typedef struct {
  int64_t n;               /* number of galaxies, 0 <= n < 2^27                  */
  const void* pos;         /* [n][3] row-major positions, dtype pos_dtype         */
  g3pcf_dtype pos_dtype;
  const double* w;         /* [n] weights                                         */
  double box[3];           /* box side lengths; > 0                              */
  double box_lo[3];        /* low corner of the box                              */
  int periodic;            /* 1: minimum-image separations, positions are wrapped
                              into [box_lo, box_lo + box); needs rmax <= box/2.
                              0: positions should lie in the box (points outside
                              are still handled exactly, only more slowly)       */
  double observer[3];      /* read only when los == G3PCF_LOS_OBSERVER           */
  double rmax;             /* outer radius R_max > 0; pairs with 0 < r < R_max   */
  int nbins;               /* 1..32 equal-width shells [b dr, (b+1) dr), dr = R_max/nbins */
  int lmax;                /* 0..10                                              */
  g3pcf_los los;
  g3pcf_prec pair_prec;    /* G3PCF_PREC_FP64 or G3PCF_PREC_FP32                 */
  g3pcf_prec zeta_prec;    /* G3PCF_PREC_FP64, _FP32 or _BF16X3; the sum over
                              blocks of primaries is always FP64                 */
  g3pcf_basis basis;
  const uint8_t* primary_mask; /* [n] nonzero = primary, or NULL (all galaxies are
                              primaries); secondaries are always all n galaxies  */
  int accumulate;          /* 0: overwrite the outputs; 1: add into them         */
  int64_t* pairs_out;      /* HOST pointer or NULL.  If set, the call waits for
                              the stream and stores the number of accepted
                              ordered (primary, secondary) pairs                 */
  g3pcf_trace* trace;      /* HOST handle or NULL.  If set, a pair of HIP events is
                              recorded on `stream` around every stage launch
                              (no synchronisation); read with g3pcf_trace_read */
  int distinct;            /* 0: zeta as the product of the a_lm (Sec. 3.1), which
                              contains the degenerate triangles j = k (the same
                              secondary on both sides, b1 = b2).  1: leave them
                              out, i.e. subtract sum_i w_i sum_j w_j^2
                              conj(Y_lm(u_ij)) Y_l'm(u_ij) at b1 = b2 = b_ij
                              (a second pass over the pairs; forward only:
                              g3pcf_backward returns G3PCF_EUNSUPPORTED)     */
  void* alm;               /* DEVICE buffer or NULL: the a_lm store, i.e. the
                              forward pass's a_lm kept for the backward pass (the
                              adjoint's secondary and primary terms are built from
                              them, Sec. 3.1).  At least g3pcf_alm_bytes bytes,
                              256-byte aligned, owned by the caller.
                              g3pcf_forward: fills it (a fingerprint of the inputs
                              and one FP64 row of every primary's a_lm(b), in the
                              library's own order); distinct = 1 is rejected.
                              g3pcf_backward: reads the a_lm from it instead of
                              recomputing them on the pair kernel.  If the store
                              was written for other positions, weights, primary
                              mask or settings (anything but zeta_prec,
                              accumulate and the output pointers), the backward
                              pass fills grad_w with NaN (checked on the device).
                              g3pcf_forward_regions: must be NULL.               */
  size_t alm_bytes;        /* size of the alm buffer in bytes                    */
} g3pcf_problem;

/* Trace with room for `capacity` stage records (2 * capacity HIP events on the
 * current device).  Returns NULL if capacity < 1 or event creation fails. */
g3pcf_trace* g3pcf_trace_create(int capacity);

/* Forget all records (events are reused).  The caller must make sure no
 * recorded event is still pending on a stream. */
void g3pcf_trace_reset(g3pcf_trace* trace);

/* After the traced streams are synchronised: copy up to `max` records as
 * (stage, milliseconds) into HOST arrays and return the number copied, or a
 * negative status (G3PCF_EINVAL for NULL arguments, G3PCF_EHIP if an event is
 * not complete).  Records beyond the capacity were dropped; *dropped (HOST,
 * may be NULL) receives their number. */
int g3pcf_trace_read(g3pcf_trace* trace, int* stage, float* ms, int max, int* dropped);

/* Destroy the trace and its events. */
void g3pcf_trace_destroy(g3pcf_trace* trace);

/* Number of doubles in zeta for (lmax, nbins): (lmax+1)^3 * nbins^2 * 2.
 * Layout [m][l][l'][b1][b2][re, im]; entries with l < m or l' < m are zero.
 * zeta^{-m} = conj(zeta^m) is not stored. */
size_t g3pcf_zeta_len(int lmax, int nbins);

/* Monomial sums accumulated per (primary, shell) by the pair stage:
 * 286 for the cartesian basis (the paper's count (l+1)(l+2)(l+3)/6 at
 * l = 10, vectorisation section), 121 for the spin basis.  The kernels always
 * accumulate to degree 10; lmax only selects which coefficients are kept.
 * Returns -1 for an unknown basis. */
int g3pcf_num_terms(int basis);

/* Bytes of device workspace needed by g3pcf_forward (backward = 0) or
 * g3pcf_backward (backward = 1) for this problem.  Depends only on the
 * problem's sizes and settings, never on the data.  Returns G3PCF_OK and stores
 * the size in *bytes, or a negative status. */
int g3pcf_workspace_bytes(const g3pcf_problem* prob, int backward, size_t* bytes);

/* Bytes of the a_lm store (problem field alm): 256 + n * W * 8 with
 * W = nbins (lmax+1)^2 doubles per primary (Re a_lm(b) for 0 <= m <= l <= lmax
 * and Im a_lm(b) for m >= 1), e.g. 10.2 GB for n = 2^20, lmax = 10, 10 shells.  Returns G3PCF_OK and stores the size in
 * *bytes, or a negative status. */
int g3pcf_alm_bytes(const g3pcf_problem* prob, size_t* bytes);

/* Forward pass.  zeta: [g3pcf_zeta_len] doubles (device).  ws: device
 * workspace of at least g3pcf_workspace_bytes(prob, 0) bytes, 256-byte aligned.
 * Steps: wrap positions and build a cell list (counting sort); for every
 * primary gather its secondaries, rotate, bin and accumulate monomial sums on
 * the pair kernel; convert them to a_lm in FP64; reduce zeta per block of
 * primaries as a Gram product A^H W A on MFMA; add the block into zeta in FP64.
 * Errors: G3PCF_EINVAL, G3PCF_EWORKSPACE, G3PCF_EHIP (message in
 * g3pcf_last_error).  On error the contents of zeta are unspecified. */
int g3pcf_forward(const g3pcf_problem* prob, double* zeta, void* ws, size_t ws_bytes,
                  void* stream);

/* Forward pass that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Computes what g3pcf_forward computes for the same
 * problem, with the scratch held in a static device array of the library
 * (128 MiB per GPU, kept until the process ends) instead of a caller
 * workspace: pair-blocks of 4096 primaries and no spill lists (a multi-chunk
 * basis repeats its search per chunk).  The caller passes only the inputs and
 * zeta (and, if set, the alm store).  Results equal g3pcf_forward's up to the
 * order of the FP64 sums across blocks of primaries.
 * Errors: as g3pcf_forward, and G3PCF_EINVAL when the problem needs more
 * scratch than the array holds (at l_max = 10 and 10 shells, roughly above
 * 1.2 million galaxies with FP32 pairs, with either FP32 zeta stage, and 0.8
 * million with FP64 pairs; the message states the size); nothing
 * is enqueued then.  Every call on one GPU uses that
 * GPU's one array: calls that overlap on one GPU (other streams, other host
 * threads) race and must be ordered by the caller. */
int g3pcf_forward_noalloc(const g3pcf_problem* prob, double* zeta, void* stream);

/* Forward pass per region of primaries (the partial zeta of each region, e.g.
 * for jack-knife resampling: zeta without region r is the full zeta minus
 * region r's).  region: device [n] int32; galaxy i is a primary of region
 * region[i] when 0 <= region[i] < nregions (and, if primary_mask is set,
 * primary_mask[i] != 0); every galaxy is a secondary of every region.
 * zeta: device [nregions][g3pcf_zeta_len] doubles, region-major, overwritten
 * (or added into with accumulate = 1).  The cell list is built once; each
 * region runs its own primary list through the pair stage, so the pair work
 * is that of one forward pass over all assigned primaries; the call waits for
 * the stream once per region to read the region's primary count.  ws: at least
 * g3pcf_workspace_bytes(prob, 0) bytes.  pairs_out (if set): accepted pairs
 * summed over the regions.  Errors as g3pcf_forward, and G3PCF_EINVAL for
 * nregions outside 1..2^20 or a NULL region with n > 0. */
int g3pcf_forward_regions(const g3pcf_problem* prob, const int32_t* region, int nregions,
                          double* zeta, void* ws, size_t ws_bytes, void* stream);

/* Forward pass over a batch of ncat catalogues of one geometry (randoms or
 * mocks sharing the box, shells, lmax, line of sight and precision), the
 * paper's downstream use (Sec. 6.1): catalogue c is the galaxies
 * [offsets[c], offsets[c+1]) of prob's arrays (positions, weights and, if set,
 * primary_mask), and its zeta goes to zeta + c * g3pcf_zeta_len, computed as
 * g3pcf_forward would for that catalogue alone (pairs never cross
 * catalogues).  offsets: HOST [ncat+1], offsets[0] = 0, non-decreasing,
 * offsets[ncat] = n.  zeta: device [ncat][g3pcf_zeta_len] doubles.  ws: at
 * least g3pcf_workspace_bytes(prob, 0) bytes for the whole batch; the
 * catalogues run one after another in it on `stream`.  pairs_out (if set): the
 * pairs of all catalogues (one wait per catalogue).  alm must be NULL.
 * Errors as g3pcf_forward, and G3PCF_EINVAL for ncat outside 1..2^20 or
 * inconsistent offsets. */
int g3pcf_forward_batch(const g3pcf_problem* prob, int ncat, const int64_t* offsets,
                        double* zeta, void* ws, size_t ws_bytes, void* stream);

/* Adjoint pass.  With L = sum over the real view of grad_zeta * zeta
 * (grad_zeta laid out like zeta), stores dL/dw_k for every galaxy k in
 * grad_w [n] (added to it when accumulate = 1).  zeta is linear in the weight
 * of a primary and quadratic in the weight of a secondary:
 *   primary term   dL/dw_i = Re sum conj(G) a_lm(b1) conj(a_l'm(b2)),
 *   secondary term dL/dw_k += w_i Re sum_lm conj(Y_lm(u_ik)) H_lm(b_ik)
 * with G = grad_re + i grad_im and H_lm(b) = U_lm(b) + conj(V_lm(b)),
 *   U_lm(b)  = sum_{l',b2} conj(G^m_{ll'}(b, b2)) conj(a_l'm(b2)),
 *   V_l'm(b) = sum_{l,b1}  conj(G^m_{ll'}(b1, b)) a_lm(b1).
 * The a_lm are recomputed from the pairs on the pair kernel, or, when
 * prob->alm is set, read from the store g3pcf_forward filled (see the alm
 * field).  Position gradients are not provided.  ws: at least
 * g3pcf_workspace_bytes(prob, 1) bytes.  pairs_out (if set): the pairs the
 * adjoint pass visited.  Same errors as g3pcf_forward. */
int g3pcf_backward(const g3pcf_problem* prob, const double* grad_zeta, double* grad_w,
                   void* ws, size_t ws_bytes, void* stream);

/* Isotropic multipoles from zeta by the addition theorem (the Legendre
 * polynomial of the angle between two directions is 4 pi / (2l + 1) times the
 * sum over m of Y_lm Y*_lm, Sec. 2):
 *   iso[l][b1][b2] = 4 pi / (2l + 1) (zeta^0_ll + 2 sum_{m >= 1} Re zeta^m_ll)(b1, b2)
 *                  = sum_i w_i sum_{j in b1, k in b2} w_j w_k P_l(u_ij . u_ik).
 * zeta: device, laid out as g3pcf_forward writes it for (lmax, nbins);
 * iso: device, [lmax+1][nbins][nbins] doubles, overwritten.  Asynchronous on
 * `stream`.  Returns G3PCF_OK, G3PCF_EINVAL (lmax outside 0..10, nbins outside
 * 1..32, NULL pointers) or G3PCF_EHIP. */
int g3pcf_isotropic(int lmax, int nbins, const double* zeta, double* iso, void* stream);

/* Diagnostic, host only, no device use: the degenerate-triangle term
 * conj(Y_lm(u)) Y_l'm(u) (real; it depends on u_z alone) as the library's
 * distinct = 1 correction represents it, a Legendre series in u_z.
 * out: HOST array [lmax+1][lmax+1][lmax+1] as [m][l][l'], zero where l < m or
 * l' < m.  Returns G3PCF_OK or G3PCF_EINVAL (lmax outside 0..10, NULL). */
int g3pcf_degenerate_term(int lmax, double uz, double* out);

/* Message for the last non-OK return on this thread ("" if none). */
const char* g3pcf_last_error(void);

/* Diagnostic, host only, no device use: evaluates the library's own
 * monomial-sum -> a_lm conversion (a coefficient table the pair kernels use:
 * G3PCF_BASIS_CARTESIAN, or G3PCF_BASIS_SPIN_T for the spin basis; or the
 * spin basis in plain powers, G3PCF_BASIS_SPIN) for a single unit vector u
 * with unit weight, i.e. conj(Y_lm(u)) as the pair stage represents it.  out: HOST array of (lmax+1)(lmax+2) doubles,
 * (re, im) pairs in triangular order (l(l+1)/2 + m), 0 <= m <= l <= lmax.
 * Returns G3PCF_OK or G3PCF_EINVAL (unknown basis, lmax outside 0..10, NULL). */
int g3pcf_conj_ylm_via_monomials(int basis, int lmax, double ux, double uy, double uz,
                                 double* out);

#ifdef __cplusplus
}
#endif

#endif /* G3PCF_H */
