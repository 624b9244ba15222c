/*
 * chi0.h -- C ABI of libchi0: the imaginary-axis polarization chi0(q, i omega)
 * of the quasiparticle self-consistent GW method and its dielectric step, on
 * one AMD Instinct MI355X (gfx950).
 *
 * The operation (Eq.(polfx) on the imaginary axis, Eq.(dielectricfunction),
 * Eq.(wc) of the paper; Algorithm "hrcxq" accumulates Pi and then inverts eps):
 *
 *   chi0[w][I][J] = sum_blocks w_k sum_{n occ} sum_{n' unocc, included}
 *                   f(D, omega_w) * conj(Z_{nn'}(I)) * Z_{nn'}(J)
 *   f(D, omega)   = -2 D / (D^2 + omega^2),   D = eps_unocc[n'] - eps_occ[n]
 *   a pair is included iff D > 0 and D >= delta_min
 *   eps[w]        = 1 - diag(s) chi0[w] diag(s),   s = vsqrt (square roots of
 *                   the Coulomb eigenvalues v_mu)
 *   W^c[w]        = diag(s) (eps[w]^{-1} - 1) diag(s)
 *
 * chi0 is Hermitian and negative semidefinite; eps is Hermitian with every
 * eigenvalue >= 1.
 *
 * Conventions shared by every entry point
 *   - Complex numbers are interleaved (re, im) pairs of float (complex64) or
 *     double (complex128).  Matrices are row-major, [nomega][npb][npb].
 *   - "DEVICE" pointers are device memory of the handle's GPU; "HOST"
 *     pointers are ordinary host memory read during the call only.  The
 *     library never frees, retains or writes caller memory other than the
 *     documented outputs.
 *   - Calls are asynchronous on the given HIP stream (hipStream_t passed as
 *     void*; NULL is the default stream).  Argument errors are returned
 *     synchronously and nothing is enqueued.  Device-side failures (launch
 *     errors, a zero pivot during inversion, pairs with D <= 0) are reported
 *     by chi0_sync().
 *   - A handle may be used from one host thread at a time.  Its calls share
 *     the handle's device workspace, so they are ordered: a call made on a
 *     different stream from the previous call first makes its stream wait
 *     for the previous call's work (an event recorded at the end of every
 *     call).  A stream being captured into a graph is not made to wait; the
 *     caller orders captured work.
 *   - Return values are chi0_status codes; chi0_last_error() gives a message
 *     for the calling thread's most recent failure.
 *   - Debugging: with the environment variable CHI0_LOG set (to anything but
 *     "0") when the library is first used, every rank-K launch (tile,
 *     units, workgroups, workspace bytes) and every inversion (method,
 *     workspace) is described on stderr, one line each.
 */
#ifndef CHI0_H
#define CHI0_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CHI0_OK = 0,
  CHI0_EINVAL = -1,        /* invalid argument                                */
  CHI0_ENOMEM = -2,        /* device workspace allocation failed              */
  CHI0_EDEVICE = -3,       /* HIP runtime / kernel launch failure             */
  CHI0_ENOTHPD = -4,       /* eps is not Hermitian positive definite (a
                              non-positive pivot in CHI0_INV_HPD)             */
  CHI0_ESINGULAR = -5,     /* exact zero pivot met while inverting eps        */
  CHI0_EUNSUPPORTED = -6   /* valid but unsupported combination               */
} chi0_status;

/* Arithmetic of the rank-K contraction.  Cross-block accumulation of chi0 is
 * FP64 on every path; the inversion of eps is always FP64. */
typedef enum {
  CHI0_PREC_FP64 = 0,      /* complex128 Z, FP64 matrix cores                 */
  CHI0_PREC_FP32 = 1,      /* complex64 Z, FP32 matrix cores, FP32 runs of at
                              most the flush length, then FP64 accumulation   */
  CHI0_PREC_BF16X3 = 2,    /* complex64 Z; each operand split into bf16
                              hi + lo, products hi*hi + hi*lo + lo*hi on BF16
                              matrix cores with FP32 accumulation, FP64 flush */
  /* not precisions: these two make every int a value of the type, so an
     unknown value passed from C is rejected (CHI0_EINVAL) rather than
     undefined in the C++ library */
  CHI0_PREC_RANGE_MIN_ = -2147483647 - 1,
  CHI0_PREC_RANGE_MAX_ = 2147483647
} chi0_precision;

typedef enum {
  CHI0_Z_C128 = 0,         /* Z is complex128 (required by CHI0_PREC_FP64)    */
  CHI0_Z_C64 = 1,          /* Z is complex64 (required by FP32 and BF16X3)    */
  CHI0_Z_RANGE_MIN_ = -2147483647 - 1,   /* not types: as for chi0_precision */
  CHI0_Z_RANGE_MAX_ = 2147483647
} chi0_ztype;

/* chi0_accumulate flags (bitwise or) */
enum {
  CHI0_OVERWRITE = 0,      /* chi0 output is overwritten                      */
  CHI0_ACCUMULATE = 1,     /* chi0 output += this call's sum (the lower
                              triangle of the existing contents is taken as the
                              Hermitian matrix to add to)                      */
  CHI0_BF16_LOLO = 2,      /* BF16X3 path also adds the lo*lo product         */
  CHI0_USE_GRAPH = 4       /* replay the call's kernels from a cached hipGraph
                              keyed by the problem shapes                     */
};

/* dielectric_invert flags: one inversion method (the low two bits) or'd
 * with the output options */
enum {
  CHI0_INV_GJ = 0,         /* blocked Gauss-Jordan with partial pivoting      */
  CHI0_INV_HPD = 1,        /* eps Hermitian positive definite (it is, since
                              chi0 is negative semidefinite): blocked
                              symmetric Gauss-Jordan sweeps without pivoting on
                              the lower triangle, half the work of
                              CHI0_INV_GJ; eps_inv is mirrored from the lower
                              triangle (exactly Hermitian, real diagonal); a
                              non-positive pivot makes chi0_sync() return
                              CHI0_ENOTHPD                                    */
  CHI0_INV_HPD_FALLBACK_GJ = 2, /* CHI0_INV_HPD, then (synchronising the
                              stream) CHI0_INV_GJ if a pivot was not positive */
  CHI0_INV_METHOD_MASK = 3,
  CHI0_OUT_WC = 8          /* also write W^c                                  */
};

typedef struct chi0_ctx* chi0_handle;

/* One k-point (x spin) block of one q-point: nocc x nunocc pairs. */
typedef struct {
  int32_t nocc;            /* >= 0                                            */
  int32_t nunocc;          /* >= 0                                            */
  const void* z;           /* DEVICE [nocc][nunocc][npb] complex, row-major
                              (npb contiguous; the Fortran Z(npb, n', n) of
                              Algorithm "hrcxq"), 16-byte aligned; may be
                              NULL when nocc * nunocc == 0                    */
  const double* eps_occ;   /* DEVICE [nocc]   eps_{k, n}                      */
  const double* eps_unocc; /* DEVICE [nunocc] eps_{k+q, n'} (caller maps k+q) */
  double wk;               /* k-point weight, finite, >= 0 (carries the
                              Brillouin-zone and any spin normalisation)      */
} chi0_block;

/* One q-point. */
typedef struct {
  int32_t npb;             /* product-basis size, >= 1                        */
  int32_t nblocks;         /* >= 0                                            */
  const chi0_block* blocks;/* HOST [nblocks]                                  */
  int32_t nomega;          /* >= 1                                            */
  const double* omega;     /* DEVICE [nomega] imaginary frequencies (same
                              energy unit as eps); only omega^2 enters        */
  void* chi0;              /* DEVICE out [nomega][npb][npb] complex128,
                              written as an exactly Hermitian matrix (imaginary
                              part of the diagonal is 0), 16-byte aligned     */
} chi0_problem;

/* Create a handle on HIP device `device`.  The handle owns device workspace,
 * cached plans and graphs, and the tile table.  Returns CHI0_EDEVICE when the
 * device is absent or not gfx950. */
int chi0_create(chi0_handle* h, int device);

/* Destroy a handle (synchronises its device first).  NULL is accepted. */
int chi0_destroy(chi0_handle h);

/* chi0 for `nprob` q-points (Eq.(polfx) at i*omega; Algorithm "hrcxq",
 * accumulation of Pi over k, pairs and frequencies), all in one persistent
 * launch plus one reduction launch.  Each (frequency, lower-triangle tile) of
 * each problem is a weighted Hermitian rank-K update; blocks with uneven
 * nocc / nunocc are balanced across the GPU by the planner.
 *
 * zt must match prec (C128 for FP64, C64 otherwise), else CHI0_EUNSUPPORTED.
 * delta_min >= 0 is the intraband cut; pairs with 0 < D < delta_min
 * contribute nothing.  A pair with D <= 0 is not a transition of
 * Eq.(polfx): it contributes nothing either, and since the energies live on
 * the device such pairs are counted there and chi0_sync() returns
 * CHI0_EINVAL with their number.  Problems may have different npb and
 * nomega.  Output buffers of different problems must not overlap.  The
 * FP64 partial tiles of one launch are bounded by the handle's cap
 * (chi0_set_partial_cap); a call whose (problem, frequency, tile) jobs
 * exceed it runs as several launches over consecutive problems and
 * frequency ranges, and a single frequency of a problem that alone exceeds
 * it returns CHI0_ENOMEM. */
int chi0_accumulate(chi0_handle h, const chi0_problem* probs, int32_t nprob,
                    chi0_ztype zt, chi0_precision prec, double delta_min,
                    uint32_t flags, void* hip_stream);

/* Exchange self-energy (Eq.(sigx)) of one q-point, one k-point block:
 *   Sigma^x[n][m] = - sum_blocks w_k sum_{n' occ} sum_mu
 *                   conj(Z[n'][mu][n]) v[mu] Z[n'][mu][m]
 * with Z[n'][mu][n] the matrix element of Eq.(defz) between product-basis
 * function mu of k and the states (q-k, n') and (q, n). */
typedef struct {
  int32_t nocc;            /* occupied intermediate states n', >= 0          */
  int32_t nmu;             /* product-basis functions mu, >= 0               */
  const void* z;           /* DEVICE [nocc][nmu][nqp] complex, row-major (n
                              contiguous), 16-byte aligned; may be NULL when
                              nocc * nmu == 0                                 */
  const double* v;         /* DEVICE [nmu] Coulomb eigenvalues v_mu(k) >= 0   */
  double wk;               /* k-point weight, finite, >= 0 (1 for the bare
                              Brillouin-zone sum)                             */
} sigx_block;

typedef struct {
  int32_t nqp;             /* quasiparticle states n, m, >= 1                 */
  int32_t nblocks;         /* >= 0                                            */
  const sigx_block* blocks;/* HOST [nblocks]                                  */
  void* sigx;              /* DEVICE out [nqp][nqp] complex128, written as an
                              exactly Hermitian matrix, 16-byte aligned       */
} sigx_problem;

/* Sigma^x for `nprob` q-points in one persistent launch: the same weighted
 * Hermitian rank-K update as chi0_accumulate (rows (n', mu) with weight
 * w_k v_mu, one output matrix per problem), on the same FP64 / FP32 / BF16x3
 * matrix-core paths, FP64 cross-block reduction, planner and tile table.
 * zt / prec / flags as for chi0_accumulate (CHI0_ACCUMULATE,
 * CHI0_BF16_LOLO, CHI0_USE_GRAPH). */
int sigx_accumulate(chi0_handle h, const sigx_problem* probs, int32_t nprob,
                    chi0_ztype zt, chi0_precision prec, uint32_t flags,
                    void* hip_stream);

/* The paper's real-axis route for chi0 (Eq.(impolf), Eq.(tetw),
 * Eq.(hilbert); the histogram steps of the polarization algorithm): the
 * anti-Hermitian part is accumulated into histogram bins of the transition
 * energy and chi0 at any frequency follows by a Hilbert transform, so the
 * rank-K work does not grow with the number of frequencies.
 *   Bins j = [edges[j], edges[j+1]).  A pair of a block enters as for
 *   chi0_accumulate (D = eps_unocc[n'] - eps_occ[n] > 0, D >= delta_min; pairs
 *   with D <= 0 are counted for chi0_sync() as there); its
 *   weight w_k is spread uniformly over [D (1 - sigma), D (1 + sigma)]
 *   (sigma = 0: all at D) -- a stand-in for the tetrahedron weights of
 *   Eq.(tetw), which need a k mesh -- and the fraction inside bin j is its
 *   bin weight; weight outside [edges[0], edges[nbins]) is dropped.
 *   hist_j = -sum_pairs weight_j conj(Z_pair) Z_pair^T.
 *   Imaginary axis: chi0(i w) = sum_j hist_j
 *     [ln(e_{j+1}^2 + w^2) - ln(e_j^2 + w^2)] / (e_{j+1} - e_j).
 *   Real axis (w not on an edge): chi0(w) = sum_j hist_j
 *     ([ln|e_{j+1} - w| - ln|e_j - w| + ln(e_{j+1} + w) - ln(e_j + w)]
 *      + i pi [w in bin j]) / (e_{j+1} - e_j)
 *   (uniform spectral density within each bin; principal value).
 * Each problem's chi0 output receives chi0(i omega) at its nomega imaginary
 * frequencies (omega on the device, as for chi0_accumulate). */
typedef struct {
  int32_t nbins;           /* >= 1; all problems together at most 16384      */
  int32_t nreal;           /* real frequencies, >= 0                          */
  const double* edges;     /* HOST [nbins + 1]: 0 < e_0 < e_1 < ..., finite   */
  double sigma;            /* relative half-width of a pair's spread, [0, 1)  */
  const double* omega_re;  /* HOST [nreal]: finite, >= 0, none on an edge     */
  void* chi0_re;           /* DEVICE out [nreal][npb][npb] complex128, used iff
                              nreal > 0, 16-byte aligned                      */
  void* hist;              /* DEVICE out [nbins][npb][npb] complex128 (hist_j),
                              or NULL; 16-byte aligned                         */
} chi0_hist;

/* Histogram route for `nprob` problems (hists[p] belongs to probs[p]).
 * prec: CHI0_PREC_FP64 (zt CHI0_Z_C128) or CHI0_PREC_BF16X3 (zt
 * CHI0_Z_C64); FP32 returns CHI0_EUNSUPPORTED.  flags: 0 or CHI0_BF16_LOLO
 * (outputs are overwritten).  Binning and a stable counting sort run on the
 * device; the call then waits for the bin counts (one device-to-host copy)
 * to plan the per-bin rank-K updates, so it synchronises hip_stream and
 * cannot be captured in a graph. */
int chi0_hist_accumulate(chi0_handle h, const chi0_problem* probs, const chi0_hist* hists,
                         int32_t nprob, chi0_ztype zt, chi0_precision prec,
                         double delta_min, uint32_t flags, void* hip_stream);

/* Records (pair, bin) kept and bins used (all problems together) by the
 * handle's last chi0_hist_accumulate call; 0 before the first. */
int chi0_hist_stats(chi0_handle h, int64_t* records, int32_t* bins_used);

/* Imaginary-axis part I^c of the correlation self-energy (Eq.(sigci),
 * Section "Self-energy"; the QK-Omega^I block of the self-energy algorithm)
 * of one q-point, one k-point block:
 *   I^c[n][m] += -w_k sum_{n'} sum_i w_i(eps_qp[n] - eps_mid[n'])
 *                sum_{mu,nu} conj(Z[n'][mu][n]) W^c_i[mu][nu] Z[n'][nu][m].
 * n' runs over all intermediate states (occupied and unoccupied); the row n
 * alone sets the energy difference, so I^c is not Hermitian in general.
 * The integration weights w_i(dE) (the Aryasetiawan-Gunnarsson weights the
 * paper cites but does not print) are the exact integrals of
 * dE / (pi (dE^2 + w^2)) over [0, inf) against the interpolant of W^c on the
 * mesh: constant below omega[0], linear between nodes, W^c(omega_last)
 * (omega_last / w)^2 beyond the last node; at dE = 0 they are 0. */
typedef struct {
  int32_t nall;            /* intermediate states n', >= 0                    */
  int32_t nmu;             /* product-basis functions mu, >= 1                */
  const void* z;           /* DEVICE [nall][nmu][nqp] complex128, Z_k[n'][mu][n],
                              16-byte aligned                                 */
  const void* wc;          /* DEVICE [nomega][nmu][nmu] complex128,
                              W^c_k(i omega_i)[mu][nu] (e.g. the CHI0_OUT_WC
                              output of dielectric_invert), 16-byte aligned   */
  const double* eps_mid;   /* HOST [nall]: eps_{q-k, n'}, finite              */
  double wk;               /* >= 0, finite; Brillouin-zone / spin weight      */
} sigc_block;

typedef struct {
  int32_t nqp;             /* quasiparticle states n, m, >= 1                 */
  int32_t nblocks;         /* >= 0                                            */
  const sigc_block* blocks;/* HOST [nblocks]                                  */
  const double* eps_qp;    /* HOST [nqp]: eps_{q n}, finite                   */
  int32_t nomega;          /* imaginary-axis mesh size, >= 1                  */
  int32_t pad;
  const double* omega;     /* HOST [nomega]: 0 <= omega[0] < omega[1] < ...   */
  void* sigc;              /* DEVICE out [nqp][nqp] complex128, 16-byte aligned */
} sigc_problem;

/* I^c for `nprob` q-points.  zt = CHI0_Z_C128; prec = CHI0_PREC_FP64 or
 * CHI0_PREC_BF16X3 (anything else returns CHI0_EUNSUPPORTED).  flags:
 * CHI0_ACCUMULATE adds to sigc instead of overwriting it.  Work: a first
 * matrix-core contraction ZW[n'][n][nu] = sum_{i,mu} t conj(Z) W^c_i
 * (t = -w_k w_i) into a workspace the size of Z, blocks grouped so that it
 * stays under the workspace cap, then sum_{n', nu} ZW Z in segments whose
 * FP64 partial tiles are summed in a fixed order (deterministic).  FP64: both
 * contractions in FP64.  BF16X3: both contractions as three bf16 split
 * products per real product with FP32 runs of at most 4096 rows added in
 * FP64 (relative Frobenius error a few 1e-6: the entries are sums of terms
 * of both signs); it needs, per block, the split operands besides ZW (W^c,
 * and Z weighted for every mesh point: about nomega times the size of Z at
 * half its precision), groups being capped at four times the workspace cap.
 * Asynchronous on hip_stream like chi0_accumulate; inputs must stay valid
 * until the stream reaches the call's end. */
int sigc_accumulate(chi0_handle h, const sigc_problem* probs, int32_t nprob,
                    chi0_ztype zt, chi0_precision prec, uint32_t flags,
                    void* hip_stream);

/* Kernel variant of the FP64 first contraction (0: 4 waves of 64 x 64 per
 * 128 x 128 tile, 1: 8 waves of 64 x 32, the default); CHI0_EINVAL when out
 * of range. */
int sigc_set_variant(chi0_handle h, int32_t variant);

/* Cap in bytes of the ZW workspace of one group of blocks (0: the default,
 * 4 GiB; a block larger than the cap forms a group of its own). */
int sigc_set_workspace_cap(chi0_handle h, int64_t bytes);

/* Cap in bytes of the FP64 partial tiles of one rank-K launch of
 * chi0_accumulate, sigx_accumulate and chi0_hist_accumulate (0: the
 * default, 12e9).  Work above the cap is split into sequential launches on
 * the call's stream; a cap below one frequency's tiles of a problem makes
 * the call return CHI0_ENOMEM.  CHI0_EINVAL for a negative value. */
int chi0_set_partial_cap(chi0_handle h, int64_t bytes);

/* Dielectric step for one q-point (Eq.(dielectricfunction), Eq.(wc);
 * Algorithm "hrcxq" builds eps, inverts it, forms W^c):
 *   eps[w] = 1 - diag(vsqrt) chi0[w] diag(vsqrt), eps_inv[w] = eps[w]^{-1}
 * in FP64 by the method in the low two flag bits (CHI0_INV_GJ: blocked
 * Gauss-Jordan elimination with partial pivoting, which reads all of eps;
 * CHI0_INV_HPD: symmetric sweeps, which read its lower triangle only), and
 * W^c[w] = diag(vsqrt) (eps_inv[w] - 1) diag(vsqrt) when CHI0_OUT_WC is set.
 *   vsqrt   DEVICE [npb] double, > 0
 *   chi0    DEVICE [nomega][npb][npb] complex128 (input, not modified)
 *   eps     DEVICE out, same shape, or NULL
 *   eps_inv DEVICE out, same shape (must not alias chi0 or eps)
 *   wc      DEVICE out, same shape, used iff CHI0_OUT_WC (else may be NULL)
 * A zero pivot makes chi0_sync() return CHI0_ESINGULAR, a non-positive
 * pivot of CHI0_INV_HPD CHI0_ENOTHPD (eps_inv is then undefined for that
 * frequency).  CHI0_INV_HPD_FALLBACK_GJ waits for the stream before it
 * returns and reports neither for a matrix the fallback inverted. */
int dielectric_invert(chi0_handle h, int32_t npb, int32_t nomega,
                      const double* vsqrt, const void* chi0, void* eps,
                      void* eps_inv, void* wc, uint32_t flags,
                      void* hip_stream);

/* Bytes of the fixed device array behind dielectric_invert_noalloc (one per
 * GPU, held until the process ends). */
#define CHI0_NOALLOC_SCRATCH_BYTES (256u << 20)

/* dielectric_invert without allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid it).  Same arguments, methods, results and error
 * reports as dielectric_invert; its workspace (the eps matrices being
 * inverted, the panel buffers and the pivots: about
 * nomega * npb * (16 npb + 1544) bytes) is carved from a fixed device array
 * of CHI0_NOALLOC_SCRATCH_BYTES instead of the handle's buffers.  A call that
 * needs more returns CHI0_EINVAL and enqueues nothing (npb = 2048: at most 3
 * frequencies per call; npb = 1024: 14; npb = 512: 53).  It calls no
 * allocation routine.
 * Every call on one GPU, from any handle, uses that GPU's one array, which
 * keeps the last call's contents: calls that overlap on one GPU race, so the
 * caller orders them (one stream, or events).  CHI0_INV_HPD_FALLBACK_GJ waits
 * for the stream before it returns, as for dielectric_invert, so it cannot
 * be captured into a graph. */
int dielectric_invert_noalloc(chi0_handle h, int32_t npb, int32_t nomega,
                              const double* vsqrt, const void* chi0, void* eps,
                              void* eps_inv, void* wc, uint32_t flags,
                              void* hip_stream);

/* Wait for all work the handle enqueued, then report deferred failures since
 * the previous chi0_sync(), in this order: CHI0_EDEVICE for a runtime error,
 * CHI0_EINVAL for pairs with D <= 0 met by chi0_accumulate or
 * chi0_hist_accumulate (the message gives their number), CHI0_ESINGULAR for
 * a zero pivot, CHI0_ENOTHPD for a non-positive CHI0_INV_HPD pivot.  The
 * deferred flags are cleared when reported. */
int chi0_sync(chi0_handle h);

/* Static description of a status code. */
const char* chi0_status_string(int status);

/* Message describing the calling thread's most recent failing call. */
const char* chi0_last_error(void);

/* Tile configurations of the rank-K kernels.  chi0_tile_count() gives the
 * number of configurations for a precision, chi0_tile_info() describes one
 * (tile rows x tile cols in complex elements, pairs per LDS stage, FP32 run
 * length before an FP64 flush; 0 for FP64).  chi0_set_tile() fixes the
 * configuration used for a precision (-1 = the autotuned or built-in
 * default).  chi0_get_tile() reports the fixed, else the autotuned, else the
 * built-in default configuration.  With none fixed or tuned, calls that do
 * not gather rows choose per call by a cost model of the padded tile area
 * (rows x padded lower-triangle area x frequencies x a per-configuration
 * cost; BF16X3 and FP32 take their frequency-group default for several
 * frequencies and small square tiles for one frequency at small npb, FP64
 * its large default tiles for large npb and smaller square ones when npb is
 * a few hundred); chi0_tile_choice() returns that model's choice for
 * a set of problems (host data only: nocc, nunocc, npb, nomega; no handle,
 * no device), and chi0_last_tile() reports the configuration of the handle's
 * last rank-K launch for a precision (-1 before the first). */
int chi0_tile_count(chi0_precision prec);
int chi0_tile_info(chi0_precision prec, int32_t tile, int32_t* tile_p,
                   int32_t* tile_q, int32_t* kchunk, int32_t* flush_len);
int chi0_set_tile(chi0_handle h, chi0_precision prec, int32_t tile);
int chi0_get_tile(chi0_handle h, chi0_precision prec, int32_t* tile);
int chi0_last_tile(chi0_handle h, chi0_precision prec, int32_t* tile);
int chi0_tile_choice(chi0_precision prec, const chi0_problem* probs, int32_t nprob, int32_t* tile);
/* Work lists per workgroup of a configuration: 1 when a workgroup takes
 * each unit as a whole (tile_p x tile_q units), 4 when each of its four
 * waves takes units of its own; CHI0_EINVAL for an unknown configuration. */
int chi0_tile_lists(chi0_precision prec, int32_t tile);
/* 1 when the configuration's tiles that cross the diagonal (tile_p =
 * 2 tile_q) leave out their 32 x 32 MFMA blocks lying entirely above it
 * (3 of 8 blocks computed right of the diagonal, 7 of 8 left of it), 0
 * when every tile is computed whole; CHI0_EINVAL for an unknown
 * configuration.  The chi0 produced is the same either way. */
int chi0_tile_diag_skip(chi0_precision prec, int32_t tile);

/* FP32 run length of the reduced-precision paths: the number of pairs summed
 * in FP32 before the partial sum is added into FP64.  By default it is
 * 4 sqrt(K) pairs for a problem with K pairs (at least 64, at most the tile
 * configuration's run length), which keeps the FP32 rounding of the chi0 sum
 * near 1.4 units of FP32 roundoff, relative, for any K.  A value set here (a
 * multiple of 16 in [16, 65536]) replaces that choice for every problem; 0
 * restores it. */
int chi0_set_flush(chi0_handle h, int32_t pairs);

/* XCD lockstep of the BF16X3 and FP32 frequency-group configurations that
 * use it (their defaults among them): with units dealt round-robin, the workgroups on
 * one XCD, which stream the same pair ranges, wait before each FP32 run
 * while they are more than `stages` 32-pair stages ahead of the slowest of
 * them, so their shared rows stay in the XCD's L2.  The wait is bounded
 * (and a workgroup whose wait reaches the bound stops waiting for the rest
 * of the launch); results do not depend on it.  stages: -1 the
 * configuration's value (16), 0 off, > 0 the slack (at most 2^20); -2 makes
 * every wait unmeetable, so each workgroup waits the full bound once and
 * then runs without the lockstep (for tests of the bound). */
int chi0_set_xcd_slack(chi0_handle h, int32_t stages);

/* Autotuner: time every tile configuration of `prec` on the given problems
 * (their chi0 outputs are overwritten), keep the fastest as the handle's
 * default for `prec`, and return its index in *best (may be NULL).  Timings
 * (milliseconds per configuration) are written to ms_out[0 .. count-1] when
 * ms_out is not NULL. */
int chi0_autotune(chi0_handle h, const chi0_problem* probs, int32_t nprob,
                  chi0_ztype zt, chi0_precision prec, double delta_min,
                  int32_t reps, int32_t* best, double* ms_out,
                  void* hip_stream);

/* Kernel timing.  When enabled, every launch of the rank-K kernel is
 * bracketed by HIP events on the stream it runs on; chi0_profile_read()
 * waits for them and returns the summed duration (ms) and the number of
 * launches since the last read. */
int chi0_profile_enable(chi0_handle h, int on);
int chi0_profile_read(chi0_handle h, double* kernel_ms, int64_t* launches);

/* Host-only inspection of the work decomposition chi0_accumulate would use
 * for these problem shapes with `nwg` persistent workgroups and tile
 * configuration `tile` (no device call; only npb, nomega, nblocks and the
 * blocks' nocc / nunocc are read).  Returns the number of units and of tile
 * jobs; when units_out is not NULL (capacity units_cap units), writes 10
 * int32 per unit: problem, frequency, tile row, tile column, first block,
 * first pair, last block, end pair (exclusive), partial slot, work list
 * (the workgroup; for configurations with a list per wave,
 * workgroup * chi0_tile_lists() + wave).  load_max / load_mean give the
 * planned cost per work list (pairs). */
int chi0_plan_inspect(const chi0_problem* probs, int32_t nprob, chi0_precision prec,
                      int32_t tile, int32_t nwg, int32_t* nunits, int32_t* njobs,
                      int32_t* units_out, int32_t units_cap, double* load_max,
                      double* load_mean);

/* ABI version (major * 10000 + minor * 100 + patch). */
int chi0_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CHI0_H */
