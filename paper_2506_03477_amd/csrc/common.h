// Shared host/device definitions of libchi0 (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chi0 {

// One k-point (x spin) block as the kernels see it (device table entry).
struct BlockDesc {
  const void* z;            // [nocc][nunocc][npb] complex, row-major
  const double* eps_occ;    // [nocc]
  const double* eps_unocc;  // [nunocc]
  double wk;
  int32_t nocc;
  int32_t nunocc;
  int64_t pair_base;        // first pair of this block in its problem's pair list
  int32_t prob;             // problem index
  int32_t pad;
  // BF16 hi / lo planes of Z split once per call (only for kernels that read
  // the P side pre-split): plane[g][col][4] words, g = group of 4 pairs,
  // padded with zero pairs to whole 16-pair stages; lo = hi + zs_plane bytes.
  void* zs;
  int64_t zs_plane;
  // Gathered blocks (histogram bins): byte address of the Z row of each of
  // the block's rows, which then need not be contiguous; NULL: row p is at
  // z + p * npb elements.
  const uint64_t* rows = nullptr;
};

// One q-point (device table entry).
struct ProbDesc {
  double2* chi0;            // [nomega][npb][npb] complex128 output
  const double* omega;      // [nomega]
  void* wts;                // [nomega][ktot] pair weights (float, or double for FP64)
  int64_t ktot;             // pairs of the problem (all blocks)
  int32_t npb;
  int32_t nomega;
  int32_t flush;            // FP32 run length in pairs (reduced-precision paths)
  int32_t pad;
};

// A unit of rank-K work: a contiguous range of pairs (from pair p0 of block
// b0 to pair p1 (exclusive) of block b1, blocks in between complete; block
// indices refer to the flat block table) contracted into one lower-triangle
// tile (tp >= tq) of one frequency of one problem and written to FP64
// partial slot `slot`.
struct Unit {
  int32_t prob;
  int32_t iw;
  int32_t tp;
  int32_t tq;
  int32_t b0;     // first block (flat block table index)
  int32_t p0;     // first pair of block b0
  int32_t b1;     // last block (inclusive)
  int32_t p1;     // end pair (exclusive) of block b1
  int32_t slot;
  // Frequency-group units (tile configurations with omega_group > 1): the
  // unit covers frequencies iw .. iw + nw - 1, frequency iw + w writing
  // partial slot slot + w * wstride.  Otherwise nw = 1.
  int32_t nw;
  int32_t wstride;
  int32_t pad;
};

// Reduction job: the partial slots [slot0, slot0 + nslot) of one tile are
// summed in order, negated, written to the lower triangle and mirrored.
struct TileJob {
  int32_t prob;
  int32_t iw;
  int32_t tp;
  int32_t tq;
  int32_t slot0;
  int32_t nslot;
};

// Arguments of the persistent rank-K kernels.
struct HerkArgs {
  const Unit* units;
  const int32_t* wg_offsets;  // [nwg + 1]: units of workgroup w are
  const int32_t* wg_units;    // wg_units[wg_offsets[w] .. wg_offsets[w+1])
  const BlockDesc* blocks;
  const ProbDesc* probs;
  double2* partials;          // [nslots][T][T] complex128
  int32_t* sync_prog;         // [nwg] stages done per workgroup (null: no lockstep)
  double delta_min;
  int32_t flags;
  int32_t sync_slack;         // with sync_prog: a workgroup more than this many
                              // stages ahead of the slowest one on its XCD waits
                              // (bounded)
  int32_t z16;                // 1: every npb even, so Z rows (16-byte aligned
                              // blocks) may be read in 16-byte chunks
  int32_t pad;
};

struct ReduceArgs {
  const TileJob* jobs;
  const ProbDesc* probs;
  const double2* partials;
  int32_t tile_p;             // tile rows
  int32_t tile_q;             // tile columns
  int32_t accumulate;
  int32_t planar;             // 1: each partial tile is a plane of real parts,
                              // then one of imaginary parts (FP64 each)
};

// Imaginary-axis correlation self-energy (Eq.(sigci)): one k-point block of
// one q-point as the kernels see it.
struct SigcDesc {
  const double2* z;       // [nall][nmu][nqp] Z_k[n'][mu][n]
  const double2* wc;      // [nomega][nmu][nmu] W^c_k(i w_i)[mu][nu]
  double2* zw;            // [nall][nmu][nqp] workspace: conj(sum_i Z_w^H W^c_i), per n'
  double* wt;             // [nomega][nall * nqp] integration weights times -w_k
  const double* eps_mid;  // [nall]
  const double* eps_qp;   // [nqp] (the problem's)
  const double* omega;    // [nomega] (the problem's mesh)
  double wk;
  int32_t nall, nmu, nqp, nomega;
  int32_t prob, groups;   // groups: 4-row groups of mu, padded to 16-row stages
  // BF16x3 first contraction: hi planes of W^c (per mesh point i: group g of
  // 4 rows mu, column nu at ((i * groups + g) * nmu + nu) * 16 bytes) and of
  // the weighted Z, t_i(r) Z[mu][r] (per mesh point i: group g, column
  // r = n' * nqp + n at ((i * groups + g) * nall * nqp + r) * 16 bytes); each
  // lo plane follows its hi plane at + *_plane bytes.
  void* wsp;
  int64_t wsp_plane;
  void* zsp;
  int64_t zsp_plane;
  // BF16x3 second contraction: hi planes of zw and of Z as [kappa][n]
  // matrices (kappa = n' * nmu + nu; group g of 4 rows kappa, column n at
  // (g * nqp + n) * 16 bytes), each lo plane at + k_plane bytes; kgroups
  // groups (whole 16-row stages, rows beyond nall * nmu are zero).
  void* zwsp;
  void* zksp;
  int64_t k_plane;
  int32_t kgroups, pad2;
};

// Work unit of the two contractions: block, tile row (P side), tile column
// (Q side) and contraction segment (second contraction only).
struct SigcUnit {
  int32_t blk, tp, tc, seg;
};

// Reduction job: the partial slots slot_list[slot0 .. slot0 + nslot) of one
// output tile of one problem are summed in order into its FP64 accumulator.
struct SigcJob {
  int32_t prob, tp, tc, slot0, nslot, pad;
};

struct SigcProb {
  double2* acc;           // [nqp][nqp] FP64 accumulator (workspace)
  double2* out;           // [nqp][nqp] caller's output
  int32_t nqp, pad;
};

struct SigcArgs {
  const SigcUnit* units;
  const SigcDesc* descs;
  double2* partials;      // second contraction: [unit][T][T] (BF16x3: [unit][2][T][T])
  int32_t nunits;
  int32_t seg_len;        // second contraction: rows (n', nu) per segment
};

hipError_t sigc_weights_launch(const SigcDesc* descs, int nblocks, int64_t max_elems, hipStream_t s);
hipError_t sigc_zw_launch(int variant, const SigcArgs& a, hipStream_t s);
hipError_t sigc_zwz_launch(const SigcArgs& a, hipStream_t s);
hipError_t sigc_reduce_launch(const SigcJob* jobs, const int32_t* slot_list, const double2* partials,
                              const SigcProb* probs, int njobs, hipStream_t s);
hipError_t sigc_clear_launch(const SigcProb* probs, int nprob, int max_nqp, hipStream_t s);
hipError_t sigc_store_launch(const SigcProb* probs, int nprob, int max_nqp, bool accumulate,
                             hipStream_t s);
int sigc_zw_variants();
int sigc_tile();
hipError_t sigc_presplit_launch(const SigcDesc* descs, int nblocks, int max_nmu, int64_t max_m,
                                int max_groups_w, int max_groups_z, hipStream_t s);
hipError_t sigc_bf16x3_launch(const SigcArgs& a, hipStream_t s);
// BF16x3 second contraction: units (block, 256-row P tile, 128-column Q
// tile, segment of seg_len rows kappa, a multiple of 16, at most 4096), each
// storing its 256 x 128 FP64 partial as partial tiles 2 unit and 2 unit + 1.
hipError_t sigc_bf16x3_zwz_launch(const SigcArgs& a, hipStream_t s);
// Split the [nall * nmu][nqp] complex128 matrix zw (which = 0) or Z
// (which = 1) of each block into the second contraction's planes.
hipError_t sigc_split_rows_launch(const SigcDesc* descs, int nblocks, int which, int max_nqp,
                                  int max_kgroups, hipStream_t s);

// Histogram route (Eq.(impolf), Eq.(hilbert)): one k-point block as the
// binning kernel sees it.
struct HistBlock {
  const void* z;            // [nocc][nunocc][npb] complex
  const double* eps_occ;    // [nocc]
  const double* eps_unocc;  // [nunocc]
  double wk;
  int32_t nocc, nunocc;
  int64_t rec0;             // first record slot (R slots per pair)
  int32_t prob;
  int32_t row_bytes;        // bytes of one Z row (npb complex values)
};

struct HistProb {
  const double* edges;      // [nbins + 1]
  double sigma;             // relative half-width of a transition's spread
  int32_t nbins;
  int32_t bin0;             // first bin of this problem in the global bin list
};

// Hilbert transform of one problem: outputs sum_k coeff[o][k] hist[slots[k]]
// over the problem's non-empty bins.
struct HilbertProb {
  const double2* hist;      // base of the problem's bin matrices [.][npb][npb]
  const int32_t* slots;     // [nbins_used] matrix index of each non-empty bin
  const int32_t* bins;      // [nbins_used] its bin index j
  const double* edges;      // [nbins + 1]
  const double* omega;      // [nimag] imaginary frequencies
  const double* omega_re;   // [nreal] real frequencies
  double2* coeff;           // [nimag + nreal][nbins_used] (written by the kernels)
  double2* out;             // [nimag][npb][npb]
  double2* out_re;          // [nreal][npb][npb]
  int32_t npb, nimag, nreal, nbins_used;
};

int hist_chunk();
hipError_t hist_records_launch(const HistBlock* blocks, const HistProb* probs, int nblocks, int64_t max_pairs,
                               int R, double delta_min, int32_t* rbin, double* rw, uint64_t* rrow,
                               int32_t* nonpositive, hipStream_t s);
hipError_t hist_sort_launch(const int32_t* rbin, const double* rw, const uint64_t* rrow, int64_t nrec, int nbt,
                            int32_t* cnt, int64_t* off, uint64_t* srow, void* sw, bool f64, hipStream_t s);
hipError_t hilbert_launch(const HilbertProb* hp, int nprob, int max_out, int max_bins, int64_t max_n2,
                          hipStream_t s);
hipError_t hist_zero_launch(double2* const* mats, int nmats, int64_t n2, hipStream_t s);

// Kernel variants of the rank-K contraction.
enum HerkKind { HERK_FP64 = 0, HERK_FP32 = 1, HERK_BF16X3 = 2 };

struct TileConfig {
  int32_t tile;      // tile rows (P side), complex elements
  int32_t kchunk;    // pairs staged in LDS per step
  int32_t flush;     // FP32 run length in pairs (0: FP64 accumulation)
  int32_t threads;   // workgroup size
  int32_t tile_q;    // tile columns (Q side); tile = tile_q or tile = 2 tile_q
  int32_t presplit;  // 1: the kernel reads the P side from BlockDesc::zs
  int32_t wave_lists;  // work lists per workgroup: 0 or 1 (the workgroup takes
                       // a unit as a whole), or one per wave (each wave takes
                       // its own units, of tile x tile_q)
  int32_t omega_group; // 0 or 1: a unit is one frequency; G > 1: a unit holds
                       // up to G frequencies of one tile and pair range
  int32_t diag_skip;   // 1, 2: tiles crossing the diagonal (tile = 2 tile_q)
                       // leave out their 32 x 32 blocks entirely above it; the
                       // light units right of it are dealt after the others
                       // (1) or in locality order like the rest (2)
  int32_t xcd_sync;    // > 0: with round-robin dealing, the workgroups of an
                       // XCD keep within this many stages of one another
  int32_t planar;      // 1: the kernel writes partial tiles as separate real
                       // and imaginary FP64 planes
};

// Groups of 4 pairs in a block's pre-split planes (whole 16-pair stages).
__host__ __device__ inline int64_t presplit_groups(int64_t pairs) { return (pairs + 15) / 16 * 4; }

// Host launchers (defined next to their kernels).
hipError_t coulomb_weights_launch(const BlockDesc* blocks, const ProbDesc* probs, int nblocks,
                                  int kmax, bool f64, hipStream_t s);
hipError_t presplit_launch(const BlockDesc* blocks, const ProbDesc* probs, int nblocks,
                           int64_t max_groups, int max_npb, hipStream_t s);
hipError_t pair_weights_launch(const BlockDesc* blocks, const ProbDesc* probs, int nblocks,
                               int kmax, double delta_min, bool f64, int32_t* nonpositive,
                               hipStream_t s);
int herk_tile_count(int kind);
int herk_default_tile(int kind);
int herk_gather_tile(int kind);
TileConfig herk_tile_config(int kind, int idx);
int herk_max_wg_per_cu(int kind, int idx);
hipError_t herk_launch(int kind, int idx, const HerkArgs& a, int nwg,
                       hipStream_t s, bool gather = false);
// Tile configurations whose kernels read gathered rows (BlockDesc::rows).
bool herk_tile_gathers(int kind, int idx);
hipError_t reduce_launch(const ReduceArgs& a, int njobs, hipStream_t s);

hipError_t dielectric_build_launch(const double2* chi0, const double* vsqrt,
                                   double2* work, double2* eps_out, int n,
                                   int nomega, hipStream_t s);
hipError_t gj_panel_launch(double2* work, int n, int nomega, int k0, int nb,
                           int32_t* piv, int32_t* status, hipStream_t s);
// Both restricted to the columns [jlo, jhi) outside the panel [k0, k0 + nb).
hipError_t gj_swap_extract_launch(double2* work, double2* wrow, int n,
                                  int nomega, int k0, int nb,
                                  const int32_t* piv, int jlo, int jhi,
                                  hipStream_t s);
hipError_t gj_update_launch(double2* work, const double2* wrow, int n,
                            int nomega, int k0, int nb, int jlo, int jhi,
                            hipStream_t s);
hipError_t gj_finish_launch(const double2* work, double2* eps_inv,
                            double2* wc, const double* vsqrt,
                            const int32_t* piv, int32_t* perm, int n,
                            int nomega, hipStream_t s);
int gj_panel_width();
int gj_subpanel_width();

// Hermitian positive definite inverse (symmetric Gauss-Jordan sweeps).
int hpd_block_width();
hipError_t hpd_status_clear_launch(int32_t* status, hipStream_t s);
hipError_t hpd_step_launch(double2* work, double2* dinv, double2* pbuf, double2* cbuf, int n,
                           int nomega, int k0, int nb, int32_t* status, bool report,
                           hipStream_t s);
hipError_t hpd_finish_launch(const double2* work, double2* eps_inv, double2* wc,
                             const double* vsqrt, int n, int nomega, hipStream_t s);

}  // namespace chi0
