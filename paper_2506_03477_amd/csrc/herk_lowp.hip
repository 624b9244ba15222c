// Reduced-precision weighted Hermitian rank-K update on gfx950 matrix cores:
// BF16x3 split products and FP32, both with FP32 runs flushed into FP64.
//
// Per unit (problem, frequency, lower tile (tp, tq), pair range) the kernels
// accumulate S[P][Q] = sum_pairs conj(Z[pair][P]) * (c * Z[pair][Q]),
// c = w_k 2 D / (D^2 + omega^2) (chi0 = -S, Eq.(polfx) at i*omega).
// The pair weight (precomputed per pair and frequency) scales the Q-side
// operand only, in FP32.
//
// BF16x3: every FP32 operand x is split into bf16 hi = rn(x) and
// lo = rn(x - hi) (x - hi is exact in FP32); the product a * b is taken as
// hi_a hi_b + hi_a lo_b + lo_a hi_b (optionally + lo_a lo_b) on
// v_mfma_f32_32x32x16_bf16.  The complex product is stacked along the
// contraction index: 8 pairs x (re, im) per MFMA,
//   Re S += [ar, ai] . [br, bi],   Im S += [ar, ai] . [bi, -br],
// where (bi, -br) is obtained from the packed (br, bi) by a 16-bit rotate and
// a sign flip.
//
// FP32: v_mfma_f32_32x32x2f32 with the (re, im) of one pair as the two
// contraction slots.
//
// Kernels: T x T complex tiles (T = 128 or 64, 4 waves of T/2 x T/2) and
// tall 256 x 128 tiles (4 waves of 128 x 64, or 8 waves), operands staged once
// per workgroup into double-buffered, XOR-swizzled LDS (the split / the
// scaling happens while staging; the tall kernels read the P side
// pre-split), one barrier per 16-pair stage, later stages' global loads (Z
// and the precomputed pair weights) issued before the current stage's MFMAs.
// Each workgroup adds its FP32 accumulators into its FP64 partial tile in
// global memory every `flush` pairs (per problem) and at the end of the unit,
// so no FP32 sum runs over more than `flush` pairs.
//
// The default BF16x3 and FP32 configurations are the frequency-group
// kernels of herk_wgroup.hip (128 x 64 tiles, four frequencies per
// workgroup); the register-direct BF16x3 kernels are in herk_direct.hip.
// This file holds the tile tables of both paths and dispatches every
// configuration.
#include "bf16_tall.h"
#include "common.h"
#include "herk_common.h"

namespace chi0 {
namespace {

// Z is read through a global-address-space pointer (global_load rather than
// flat_load); one complex64 = one 64-bit word.
typedef const uint64_t __attribute__((address_space(1)))* gf2ptr;

typedef const float __attribute__((address_space(1)))* gfptr;

__device__ __forceinline__ float2 ld_c64(gf2ptr p) {
  const uint64_t v = *p;
  return float2{__uint_as_float(static_cast<uint32_t>(v)), __uint_as_float(static_cast<uint32_t>(v >> 32))};
}

// Byte offset of a tile column within a Z row; a column beyond npb reads
// column 0 instead (its products are never used).
__device__ __forceinline__ uint32_t col_offset(int col, int npb) {
  return static_cast<uint32_t>(col < npb ? col : 0) * 8u;
}

// Operand and weight loads of one stage for one thread: NP pairs
// p0 + poff[k] of the current block, tile column byte offsets offP / offQ.
// Every kernel gives all lanes of a wave the same pair offsets, so the pair
// rows, their validity and their weights are wave-uniform: the row address
// and the weight live in scalar registers (the weight comes through the
// scalar cache) and a lane only adds its fixed column offset.  Loads are
// issued unconditionally with the row clamped into the block; bit k of the
// returned (uniform) mask says whether pair k exists, and the consumer gives
// a missing pair weight 0.  The loads of a stage thus form one straight-line
// group that is only waited for when the stage is staged.
template <int NP>
__device__ __forceinline__ uint32_t load_pairs(const HerkArgs& a, const ProbDesc& pd, int iw,
                                               const Cursor& c, const int (&poff)[NP], int npb,
                                               uint32_t offP, uint32_t offQ, float2 (&ra)[NP],
                                               float2 (&rb)[NP], float (&rw)[NP]) {
  typedef const char __attribute__((address_space(1)))* gcptr;
  const int b = __builtin_amdgcn_readfirstlane(c.b);
  const int p0 = __builtin_amdgcn_readfirstlane(c.p0);
  const int last = __builtin_amdgcn_readfirstlane(c.pend) - 1 - p0;  // last valid offset
  const BlockDesc* bp = a.blocks + b;
  const uint32_t row_bytes = static_cast<uint32_t>(npb) * 8u;
  // stage base: row p0 of the block, and its weights
  const gcptr z = (gcptr)(ld_const(&bp->z, 0)) + static_cast<size_t>(p0) * row_bytes;
  const int64_t pbase = ld_const(&bp->pair_base, 0);
  const float* w = static_cast<const float*>(pd.wts) + static_cast<size_t>(iw) * pd.ktot + pbase + p0;
  uint32_t mask = 0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int o = __builtin_amdgcn_readfirstlane(poff[k]);
    const bool valid = o <= last;
    const int oc = valid ? o : last;
    mask |= valid ? (1u << k) : 0u;
    const gcptr row = z + static_cast<uint32_t>(oc) * row_bytes;
    ra[k] = ld_c64((gf2ptr)(row + offP));
    rb[k] = ld_c64((gf2ptr)(row + offQ));
    rw[k] = ld_const(w, oc);
  }
  return mask;
}

// Add (or store, when first) the (T/2) x (T/2) wave tile of FP32 accumulators
// into the FP64 partial tile.  32x32 MFMA result layout: lane holds column
// (lane % 32) of rows 8 (r / 4) + 4 (lane / 32) + (r % 4).
template <int T, int NB>
__device__ __forceinline__ void flush_tile(double2* __restrict__ part, const f32x16 (&cr)[NB][NB],
                                           const f32x16 (&ci)[NB][NB], int wr, int wc, int lane,
                                           bool first) {
  const int g = lane >> 5;
  const int cl = lane & 31;
  // Per-lane base offset, made opaque so that the 16 NB^2 element addresses
  // are formed here instead of being hoisted (and kept live) across the
  // stage loop.
  int base = (wr * (T / 2) + 4 * g) * T + wc * (T / 2) + cl;
  asm volatile("" : "+v"(base));
  // One 32x32 block at a time: its 16 old values are loaded as one group
  // before any of them is added and stored, so a flush waits for memory
  // NB^2 times rather than once per element.
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      double2* blk = part + base + i * 32 * T + j * 32;
      double2 o[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) o[r] = double2{0.0, 0.0};
      if (!first) {
#pragma unroll
        for (int r = 0; r < 16; ++r) o[r] = blk[(8 * (r >> 2) + (r & 3)) * T];
      }
#pragma unroll
      for (int r = 0; r < 16; ++r)
        blk[(8 * (r >> 2) + (r & 3)) * T] =
            double2{static_cast<double>(cr[i][j][r]) + o[r].x,
                    static_cast<double>(ci[i][j][r]) + o[r].y};
    }
}

template <int NB>
__device__ __forceinline__ void zero_acc(f32x16 (&cr)[NB][NB], f32x16 (&ci)[NB][NB]) {
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      cr[i][j] = f32x16{0};
      ci[i][j] = f32x16{0};
    }
}

// ---------------------------------------------------------------------------
// BF16x3
// ---------------------------------------------------------------------------

// LDS of the BF16x3 kernels: bf16 hi / lo planes of both operands, two
// buffers; with ROT also the Q side rotated to (im, -re) for the imaginary
// part (staged once instead of rotated by every wave at every k-step, at
// the price of 50% more LDS).
template <int T, bool ROT>
struct Bf16Lds {
  static constexpr int kRot = ROT ? 2 : 0;
  uint32_t ah[2][T * 16];
  uint32_t al[2][T * 16];
  uint32_t bh[2][T * 16];
  uint32_t bl[2][T * 16];
  uint32_t bih[kRot][T * 16];
  uint32_t bil[kRot][T * 16];
};

// Stage one thread's 4 GPT pairs into LDS buffer `buf`: split the P side,
// scale (by the pair weight, 0 for a missing pair) and split the Q side, and
// store the Q side also rotated.  Thread owns tile column lc and pair groups
// q = lg + LG gi (4 pairs each).  Columns beyond npb hold real (clamped)
// data whose products land in tile rows / columns the reduction ignores.
template <int T, bool ROT, int GPT, int LG>
__device__ __forceinline__ void bf16_stage(Bf16Lds<T, ROT>& L, int buf, int lc, int lg,
                                           const float2 (&ra)[4 * GPT], const float2 (&rb)[4 * GPT],
                                           const float (&rw)[4 * GPT], uint32_t mask) {
#pragma unroll
  for (int gi = 0; gi < GPT; ++gi) {
    const int q = lg + LG * gi;
    uint32_t ah[4], al[4], bh[4], bl[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = 4 * gi + e;
      const float wq = ((mask >> k) & 1u) ? rw[k] : 0.f;
      split2(ra[k].x, ra[k].y, ah[e], al[e]);
      split2(rb[k].x * wq, rb[k].y * wq, bh[e], bl[e]);
    }
    const int o = swz(lc, q);
    *reinterpret_cast<uint4*>(&L.ah[buf][o]) = uint4{ah[0], ah[1], ah[2], ah[3]};
    *reinterpret_cast<uint4*>(&L.al[buf][o]) = uint4{al[0], al[1], al[2], al[3]};
    *reinterpret_cast<uint4*>(&L.bh[buf][o]) = uint4{bh[0], bh[1], bh[2], bh[3]};
    *reinterpret_cast<uint4*>(&L.bl[buf][o]) = uint4{bl[0], bl[1], bl[2], bl[3]};
    if constexpr (ROT) {
      *reinterpret_cast<uint4*>(&L.bih[buf][o]) = rot_neg4(uint4{bh[0], bh[1], bh[2], bh[3]});
      *reinterpret_cast<uint4*>(&L.bil[buf][o]) = rot_neg4(uint4{bl[0], bl[1], bl[2], bl[3]});
    }
  }
}

// The 2 k-steps (8 pairs each) of one stage from LDS buffer `buf`.  One
// product kind at a time over the accumulators, so dependent MFMAs on the
// same accumulator are 2 NB^2 instructions apart.
template <int T, bool ROT, int NB, bool LOLO>
__device__ __forceinline__ void bf16_mfma(const Bf16Lds<T, ROT>& L, int buf, int wr, int wc, int g8,
                                          int l32, f32x16 (&cr)[NB][NB], f32x16 (&ci)[NB][NB]) {
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    const int q = 2 * ks + g8;
    bf16x8 fah[NB], fal[NB], fbh[NB], fbl[NB], fih[NB], fil[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int row = wr * (T / 2) + i * 32 + l32;
      fah[i] = as_bf16x8(*reinterpret_cast<const uint4*>(&L.ah[buf][swz(row, q)]));
      fal[i] = as_bf16x8(*reinterpret_cast<const uint4*>(&L.al[buf][swz(row, q)]));
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int row = wc * (T / 2) + j * 32 + l32;
      const uint4 bh = *reinterpret_cast<const uint4*>(&L.bh[buf][swz(row, q)]);
      const uint4 bl = *reinterpret_cast<const uint4*>(&L.bl[buf][swz(row, q)]);
      fbh[j] = as_bf16x8(bh);
      fbl[j] = as_bf16x8(bl);
      if constexpr (ROT) {  // (bi, -br) for the imaginary part
        fih[j] = as_bf16x8(*reinterpret_cast<const uint4*>(&L.bih[buf][swz(row, q)]));
        fil[j] = as_bf16x8(*reinterpret_cast<const uint4*>(&L.bil[buf][swz(row, q)]));
      } else {
        fih[j] = as_bf16x8(rot_neg4(bh));
        fil[j] = as_bf16x8(rot_neg4(bl));
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[i], fbh[j], cr[i][j], 0, 0, 0);
        ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[i], fih[j], ci[i][j], 0, 0, 0);
      }
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[i], fbl[j], cr[i][j], 0, 0, 0);
        ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[i], fil[j], ci[i][j], 0, 0, 0);
      }
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fal[i], fbh[j], cr[i][j], 0, 0, 0);
        ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fal[i], fih[j], ci[i][j], 0, 0, 0);
      }
    if (LOLO) {
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fal[i], fbl[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fal[i], fil[j], ci[i][j], 0, 0, 0);
        }
    }
  }
}

// BF16x3 kernel, staging and MFMAs in sequence.  T = 128: waves of 64 x 64
// (2 x 2 MFMA blocks); T = 64: waves of 32 x 32.  OCC = workgroups per CU
// the register allocation must allow (2: at most 256 registers per lane, so
// two workgroups' barriers and memory waits can hide each other).
template <int T, bool LOLO, int OCC>
__global__ __launch_bounds__(kNT, OCC) void herk_bf16x3_kernel(HerkArgs a) {
  constexpr int NB = T / 64;          // 32x32 blocks per wave side
  constexpr int LG = kNT / T;         // loader groups
  constexpr int GPT = 4 / LG;         // pair groups (of 4) per thread
  constexpr int NP = 4 * GPT;         // pairs per thread per stage
  constexpr bool ROT = OCC == 1;      // two workgroups per CU: no rotated planes
  __shared__ __attribute__((aligned(16))) Bf16Lds<T, ROT> L;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int g8 = lane >> 5;
  const int l32 = lane & 31;
  const int lc = tid & (T - 1);
  const int lg = tid / T;
  int poff[NP];
#pragma unroll
  for (int gi = 0; gi < GPT; ++gi)
#pragma unroll
    for (int e = 0; e < 4; ++e) poff[4 * gi + e] = 4 * (lg + LG * gi) + e;

  const int beg = a.wg_offsets[blockIdx.x];
  const int end = a.wg_offsets[blockIdx.x + 1];
  for (int ui = beg; ui < end; ++ui) {
    const Unit u = a.units[a.wg_units[ui]];
    const ProbDesc pd = a.probs[u.prob];
    const int npb = pd.npb;
    const int flush_stages = pd.flush > kKC ? pd.flush / kKC : 1;
    double2* part = a.partials + static_cast<size_t>(u.slot) * T * T;

    f32x16 cr[NB][NB], ci[NB][NB];
    zero_acc<NB>(cr, ci);
    float2 ra[NP], rb[NP];
    float rw[NP];
    uint32_t mk = 0;
    const uint32_t cP = col_offset(u.tp * T + lc, npb), cQ = col_offset(u.tq * T + lc, npb);
    Cursor cur;
    bool have = cursor_first(u, a.blocks, cur);
    __syncthreads();  // previous unit's last MFMAs are done with the LDS
    if (have) mk = load_pairs<NP>(a, pd, u.iw, cur, poff, npb, cP, cQ, ra, rb, rw);
    int buf = 0;
    bool first_flush = true;
    while (have) {
      for (int ns = 0; ns < flush_stages && have; ++ns) {
        bf16_stage<T, ROT, GPT, LG>(L, buf, lc, lg, ra, rb, rw, mk);
        // next stage's loads in flight during this stage's MFMAs (the cursor
        // stays on a valid stage when there is no next one)
        Cursor nxt = cur;
        const bool more = cursor_next<kKC>(u, a.blocks, nxt);
        mk = load_pairs<NP>(a, pd, u.iw, nxt, poff, npb, cP, cQ, ra, rb, rw);
        __syncthreads();
        bf16_mfma<T, ROT, NB, LOLO>(L, buf, wr, wc, g8, l32, cr, ci);
        cur = nxt;
        have = more;
        buf ^= 1;
      }
      flush_tile<T, NB>(part, cr, ci, wr, wc, lane, first_flush);
      first_flush = false;
      zero_acc<NB>(cr, ci);
    }
    if (first_flush) flush_tile<T, NB>(part, cr, ci, wr, wc, lane, true);  // empty unit: zeros
  }
}

// Software-pipelined BF16x3 kernel (T = 128).  Stage s (16 pairs):
//   1. issue the global loads of stage s + 2 into register set s % 2 (freed
//      when stage s was staged into LDS one stage earlier);
//   2. the MFMAs of stage s (LDS buffer s % 2) and the staging of stage s + 1
//      (register set (s + 1) % 2 -> LDS buffer (s + 1) % 2) in one basic
//      block, with scheduling hints interleaving one MFMA with five VALU
//      instructions, so the split / scale work overlaps the matrix cores;
//   3. one barrier.
// The stage loop is unrolled by two so every buffer index is a constant.
template <bool LOLO, bool HINT>
__global__ __launch_bounds__(kNT, 1) void herk_bf16x3_pipe_kernel(HerkArgs a) {
  constexpr int T = 128, NB = 2, LG = 2, GPT = 2, NP = 8;
  constexpr bool ROT = true;
  __shared__ __attribute__((aligned(16))) Bf16Lds<T, ROT> L;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int g8 = lane >> 5;
  const int l32 = lane & 31;
  const int lc = tid & (T - 1);
  const int lg = tid / T;
  int poff[NP];
#pragma unroll
  for (int gi = 0; gi < GPT; ++gi)
#pragma unroll
    for (int e = 0; e < 4; ++e) poff[4 * gi + e] = 4 * (lg + LG * gi) + e;

  const int beg = a.wg_offsets[blockIdx.x];
  const int end = a.wg_offsets[blockIdx.x + 1];
  for (int ui = beg; ui < end; ++ui) {
    const Unit u = a.units[a.wg_units[ui]];
    const ProbDesc pd = a.probs[u.prob];
    const int npb = pd.npb;
    const int flush_pairs = pd.flush > 2 * kKC ? pd.flush / (2 * kKC) : 1;  // stage pairs per run
    const uint32_t cP = col_offset(u.tp * T + lc, npb), cQ = col_offset(u.tq * T + lc, npb);
    double2* part = a.partials + static_cast<size_t>(u.slot) * T * T;

    f32x16 cr[NB][NB], ci[NB][NB];
    zero_acc<NB>(cr, ci);
    float2 ra0[NP], rb0[NP], ra1[NP], rb1[NP];
    float rw0[NP], rw1[NP];
    uint32_t mk0 = 0, mk1 = 0;

    auto interleave = [&]() {
      if constexpr (HINT) {
#pragma unroll
        for (int k = 0; k < (LOLO ? 64 : 48); ++k) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // 1 MFMA
          __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);   // 5 VALU
        }
      }
    };

    // pipeline state: stage s (staged in LDS), s + 1 (in registers),
    // s + 2 (being loaded).  Cursors stay on a valid stage when the unit has
    // no further stage, so every load reads valid memory.
    Cursor c_s, c_1, c_2;
    bool h_s = cursor_first(u, a.blocks, c_s);
    c_1 = c_s;
    bool h_1 = h_s && cursor_next<kKC>(u, a.blocks, c_1);
    __syncthreads();  // previous unit's last MFMAs are done with the LDS
    if (h_s) {
      mk0 = load_pairs<NP>(a, pd, u.iw, c_s, poff, npb, cP, cQ, ra0, rb0, rw0);
      mk1 = load_pairs<NP>(a, pd, u.iw, c_1, poff, npb, cP, cQ, ra1, rb1, rw1);
      bf16_stage<T, ROT, GPT, LG>(L, 0, lc, lg, ra0, rb0, rw0, mk0);
    }
    __syncthreads();
    bool first_flush = true;
    while (h_s) {
      for (int np = 0; np < flush_pairs && h_s; ++np) {
        // ---- even stage: LDS 0, register set 1 -> LDS 1, loads -> set 0
        c_2 = c_1;
        bool h_2 = h_1 && cursor_next<kKC>(u, a.blocks, c_2);
        mk0 = load_pairs<NP>(a, pd, u.iw, c_2, poff, npb, cP, cQ, ra0, rb0, rw0);
        bf16_mfma<T, ROT, NB, LOLO>(L, 0, wr, wc, g8, l32, cr, ci);
        bf16_stage<T, ROT, GPT, LG>(L, 1, lc, lg, ra1, rb1, rw1, mk1);   // unused when !h_1
        interleave();
        __syncthreads();
        c_s = c_1; h_s = h_1; c_1 = c_2; h_1 = h_2;
        if (!h_s) break;
        // ---- odd stage: LDS 1, register set 0 -> LDS 0, loads -> set 1
        c_2 = c_1;
        h_2 = h_1 && cursor_next<kKC>(u, a.blocks, c_2);
        mk1 = load_pairs<NP>(a, pd, u.iw, c_2, poff, npb, cP, cQ, ra1, rb1, rw1);
        bf16_mfma<T, ROT, NB, LOLO>(L, 1, wr, wc, g8, l32, cr, ci);
        bf16_stage<T, ROT, GPT, LG>(L, 0, lc, lg, ra0, rb0, rw0, mk0);
        interleave();
        __syncthreads();
        c_s = c_1; h_s = h_1; c_1 = c_2; h_1 = h_2;
      }
      flush_tile<T, NB>(part, cr, ci, wr, wc, lane, first_flush);
      first_flush = false;
      zero_acc<NB>(cr, ci);
    }
    if (first_flush) flush_tile<T, NB>(part, cr, ci, wr, wc, lane, true);  // empty unit: zeros
  }
}

// ---------------------------------------------------------------------------
// Tall tiles: 256 (P) x 128 (Q), P side pre-split.  The Q side (scaled and
// split per frequency) is shared by twice as many P rows as in a square
// tile, and the P side arrives already split (presplit.hip): its 16-byte
// chunks are copied to LDS through registers without arithmetic, so the only
// staging arithmetic left is the Q side's.  Each wave's
// 128 x 64 sub-tile (4 x 2 blocks, 256 FP32 accumulators per lane) does 48
// MFMAs per 16 fragment reads.
// ---------------------------------------------------------------------------
// Q-side loads of one stage: column offQ of the 8 pairs 4 (lg + 2 gi) + e,
// and their weights (wave-uniform rows, see load_pairs).
template <bool GATHER>
__device__ __forceinline__ uint32_t tall_load_q(const HerkArgs& a, const ProbDesc& pd, int iw,
                                                const Cursor& c, int lg, int npb, uint32_t offQ,
                                                float2 (&rb)[8], float (&rw)[8]) {
  typedef const char __attribute__((address_space(1)))* gcptr;
  const int b = __builtin_amdgcn_readfirstlane(c.b);
  const int p0 = __builtin_amdgcn_readfirstlane(c.p0);
  const int last = __builtin_amdgcn_readfirstlane(c.pend) - 1 - p0;
  const int g = __builtin_amdgcn_readfirstlane(lg);
  const BlockDesc* bp = a.blocks + b;
  const uint32_t row_bytes = static_cast<uint32_t>(npb) * 8u;
  const gcptr z = (gcptr)(ld_const(&bp->z, 0)) + static_cast<size_t>(p0) * row_bytes;
  const uint64_t* rows = GATHER ? ld_const(&bp->rows, 0) + p0 : nullptr;
  const int64_t pbase = ld_const(&bp->pair_base, 0);
  const float* w = static_cast<const float*>(pd.wts) + static_cast<size_t>(iw) * pd.ktot + pbase + p0;
  uint32_t mask = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int o = 4 * (g + 2 * (k >> 2)) + (k & 3);
    const bool valid = o <= last;
    const int oc = valid ? o : last;
    mask |= valid ? (1u << k) : 0u;
    const gcptr row = GATHER ? (gcptr)ld_const(rows, oc) : z + static_cast<uint32_t>(oc) * row_bytes;
    rb[k] = ld_c64((gf2ptr)(row + offQ));
    rw[k] = ld_const(w, oc);
  }
  return mask;
}

// P side of one stage (16 pairs, starting at a multiple of 16 within the
// block) from the pre-split planes: thread t loads tile row t's four 16-byte
// chunks (4 pairs each) of the hi and of the lo plane, column offset offP.
// No arithmetic: the words go to LDS as they are (tall_stage_p).
__device__ __forceinline__ void tall_load_p(const HerkArgs& a, const Cursor& c, int npb,
                                            uint32_t offP, uint4 (&ph)[4], uint4 (&pl)[4]) {
  typedef const char __attribute__((address_space(1)))* gcptr;
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  typedef const u32x4 __attribute__((address_space(1)))* gu4ptr;
  const int b = __builtin_amdgcn_readfirstlane(c.b);
  const int p0 = __builtin_amdgcn_readfirstlane(c.p0);
  const BlockDesc* bp = a.blocks + b;
  const size_t chunk_bytes = static_cast<size_t>(npb) * 16;
  const gcptr hi = (gcptr)(ld_const(&bp->zs, 0)) + static_cast<size_t>(p0 >> 2) * chunk_bytes;
  const gcptr lo = hi + ld_const(&bp->zs_plane, 0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t o = static_cast<uint32_t>(q) * static_cast<uint32_t>(chunk_bytes) + offP;
    const u32x4 h = *(gu4ptr)(hi + o);
    const u32x4 l = *(gu4ptr)(lo + o);
    ph[q] = uint4{h.x, h.y, h.z, h.w};
    pl[q] = uint4{l.x, l.y, l.z, l.w};
  }
}

// Q side of one stage into LDS buffer `buf`: column lq, pair chunks lg and
// lg + 2, scaled (0 for a missing pair), split and rotated.
__device__ __forceinline__ void tall_stage_q(Bf16TallLds& L, int buf, int lq, int lg,
                                             const float2 (&rb)[8], const float (&rw)[8],
                                             uint32_t mask) {
#pragma unroll
  for (int gi = 0; gi < 2; ++gi) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = 4 * gi + e;
      const float wq = ((mask >> k) & 1u) ? rw[k] : 0.f;
      split2(rb[k].x * wq, rb[k].y * wq, h[e], l[e]);
    }
    const int o = swz(lq, lg + 2 * gi);
    const uint4 vh = uint4{h[0], h[1], h[2], h[3]};
    const uint4 vl = uint4{l[0], l[1], l[2], l[3]};
    *reinterpret_cast<uint4*>(&L.bh[buf][o]) = vh;
    *reinterpret_cast<uint4*>(&L.bl[buf][o]) = vl;
    *reinterpret_cast<uint4*>(&L.bih[buf][o]) = rot_neg4(vh);
    *reinterpret_cast<uint4*>(&L.bil[buf][o]) = rot_neg4(vl);
  }
}

// Software-pipelined tall-tile kernel.  Stage s (buffer s % 2):
//   1. the P loads of stage s + 1 (one register set) and the Q loads of stage
//      s + 2 (register set s % 2);
//   2. the MFMAs of stage s and the Q staging of stage s + 1 (register set
//      (s + 1) % 2) in one block with interleaving hints;
//   3. the P staging of stage s + 1 (its loads have had the MFMA phase to
//      land), then one barrier.
template <bool LOLO, bool HINT, bool GATHER = false>
__global__ __launch_bounds__(kNT, 1) void herk_bf16x3_tall_kernel(HerkArgs a) {
  constexpr int TP = 256, TQ = 128;
  __shared__ __attribute__((aligned(16))) Bf16TallLds L;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int g8 = lane >> 5;
  const int l32 = lane & 31;
  const int lp = tid;              // P row of the tile
  const int lq = tid & (TQ - 1);   // Q column
  const int lg = tid >> 7;         // Q pair group (wave-uniform)

  const int beg = a.wg_offsets[blockIdx.x];
  const int end = a.wg_offsets[blockIdx.x + 1];
  for (int ui = beg; ui < end; ++ui) {
    const Unit u = a.units[a.wg_units[ui]];
    const ProbDesc pd = a.probs[u.prob];
    const int npb = pd.npb;
    const int flush_pairs = pd.flush > 2 * kKC ? pd.flush / (2 * kKC) : 1;
    const uint32_t cQ = col_offset(u.tq * TQ + lq, npb);
    const uint32_t cP = (u.tp * TP + lp < npb ? static_cast<uint32_t>(u.tp * TP + lp) : 0u) * 16u;
    double2* part = a.partials + static_cast<size_t>(u.slot) * TP * TQ;

    f32x16 cr[4][2], ci[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        cr[i][j] = f32x16{0};
        ci[i][j] = f32x16{0};
      }
    float2 rb0[8], rb1[8];
    float rw0[8], rw1[8];
    uint4 ph[4], pl[4];
    uint32_t mk0 = 0, mk1 = 0;

    auto interleave = [&]() {
      if constexpr (HINT) {
#pragma unroll
        for (int k = 0; k < (LOLO ? 128 : 96); ++k) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // 1 MFMA
          __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);   // 2 VALU
        }
      }
    };

    Cursor c_s, c_1, c_2;
    bool h_s = cursor_first(u, a.blocks, c_s);
    c_1 = c_s;
    bool h_1 = h_s && cursor_next<kKC>(u, a.blocks, c_1);
    __syncthreads();  // previous unit's last MFMAs are done with the LDS
    if (h_s) {
      tall_load_p(a, c_s, npb, cP, ph, pl);
      mk0 = tall_load_q<GATHER>(a, pd, u.iw, c_s, lg, npb, cQ, rb0, rw0);
      mk1 = tall_load_q<GATHER>(a, pd, u.iw, c_1, lg, npb, cQ, rb1, rw1);
      tall_stage_p(L, 0, lp, ph, pl);
      tall_stage_q(L, 0, lq, lg, rb0, rw0, mk0);
    }
    __syncthreads();
    bool first_flush = true;
    while (h_s) {
      for (int np = 0; np < flush_pairs && h_s; ++np) {
        // ---- even stage: LDS 0; stage s + 1 -> LDS 1
        c_2 = c_1;
        bool h_2 = h_1 && cursor_next<kKC>(u, a.blocks, c_2);
        tall_load_p(a, c_1, npb, cP, ph, pl);                     // unused when !h_1
        mk0 = tall_load_q<GATHER>(a, pd, u.iw, c_2, lg, npb, cQ, rb0, rw0);
        tall_mfma<LOLO>(L, 0, wr, wc, g8, l32, cr, ci);
        tall_stage_q(L, 1, lq, lg, rb1, rw1, mk1);
        interleave();
        tall_stage_p(L, 1, lp, ph, pl);
        __syncthreads();
        c_s = c_1; h_s = h_1; c_1 = c_2; h_1 = h_2;
        if (!h_s) break;
        // ---- odd stage: LDS 1; stage s + 1 -> LDS 0
        c_2 = c_1;
        h_2 = h_1 && cursor_next<kKC>(u, a.blocks, c_2);
        tall_load_p(a, c_1, npb, cP, ph, pl);
        mk1 = tall_load_q<GATHER>(a, pd, u.iw, c_2, lg, npb, cQ, rb1, rw1);
        tall_mfma<LOLO>(L, 1, wr, wc, g8, l32, cr, ci);
        tall_stage_q(L, 0, lq, lg, rb0, rw0, mk0);
        interleave();
        tall_stage_p(L, 0, lp, ph, pl);
        __syncthreads();
        c_s = c_1; h_s = h_1; c_1 = c_2; h_1 = h_2;
      }
      tall_flush(part, cr, ci, wr, wc, lane, first_flush);
      first_flush = false;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cr[i][j] = f32x16{0};
          ci[i][j] = f32x16{0};
        }
    }
    if (first_flush) tall_flush(part, cr, ci, wr, wc, lane, true);  // empty unit: zeros
  }
}

// Tall tiles with 8 waves (two per SIMD, so one wave's matrix-core work can
// issue while the other waits on LDS or a barrier): waves of 64 x 64 (2 x 2
// blocks, 128 accumulators, at most 256 registers per lane).  Thread t stages
// P row t % 256 (chunks 2 (t / 256), + 1 of both planes) and Q column t % 128,
// chunk t / 128 (wave-uniform); one register set, staged after the MFMAs.
template <bool LOLO>
__global__ __launch_bounds__(512, 1) void herk_bf16x3_tall8_kernel(HerkArgs a) {
  constexpr int TP = 256, TQ = 128;
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  typedef const u32x4 __attribute__((address_space(1)))* gu4ptr;
  typedef const char __attribute__((address_space(1)))* gcptr;
  __shared__ __attribute__((aligned(16))) Bf16TallLds L;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int g8 = lane >> 5;
  const int l32 = lane & 31;
  const int lp = tid & (TP - 1);
  const int pq0 = 2 * (tid >> 8);     // first P chunk (wave-uniform)
  const int lq = tid & (TQ - 1);
  const int lg = tid >> 7;            // Q chunk (wave-uniform)

  // P: chunks pq0, pq0 + 1 of tile row lp from the pre-split planes
  auto load_p = [&](const Cursor& c, int npb, uint32_t offP, uint4 (&ph)[2], uint4 (&pl)[2]) {
    const int b = __builtin_amdgcn_readfirstlane(c.b);
    const int p0 = __builtin_amdgcn_readfirstlane(c.p0);
    const int q0 = __builtin_amdgcn_readfirstlane(pq0);
    const BlockDesc* bp = a.blocks + b;
    const size_t chunk_bytes = static_cast<size_t>(npb) * 16;
    const gcptr hi = (gcptr)(ld_const(&bp->zs, 0)) +
                     static_cast<size_t>((p0 >> 2) + q0) * chunk_bytes;
    const gcptr lo = hi + ld_const(&bp->zs_plane, 0);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const uint32_t o = static_cast<uint32_t>(j) * static_cast<uint32_t>(chunk_bytes) + offP;
      const u32x4 h = *(gu4ptr)(hi + o);
      const u32x4 l = *(gu4ptr)(lo + o);
      ph[j] = uint4{h.x, h.y, h.z, h.w};
      pl[j] = uint4{l.x, l.y, l.z, l.w};
    }
  };
  auto stage_p = [&](int buf, const uint4 (&ph)[2], const uint4 (&pl)[2]) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int o = swz(lp, pq0 + j);
      *reinterpret_cast<uint4*>(&L.ah[buf][o]) = ph[j];
      *reinterpret_cast<uint4*>(&L.al[buf][o]) = pl[j];
    }
  };
  // Q: the 4 pairs of chunk lg, column offQ, with weights (wave-uniform rows)
  auto load_q = [&](const ProbDesc& pd, int iw, const Cursor& c, int npb, uint32_t offQ,
                    float2 (&rb)[4], float (&rw)[4]) -> uint32_t {
    const int b = __builtin_amdgcn_readfirstlane(c.b);
    const int p0 = __builtin_amdgcn_readfirstlane(c.p0);
    const int last = __builtin_amdgcn_readfirstlane(c.pend) - 1 - p0;
    const int g = __builtin_amdgcn_readfirstlane(lg);
    const BlockDesc* bp = a.blocks + b;
    const uint32_t row_bytes = static_cast<uint32_t>(npb) * 8u;
    const gcptr z = (gcptr)(ld_const(&bp->z, 0)) + static_cast<size_t>(p0) * row_bytes;
    const int64_t pbase = ld_const(&bp->pair_base, 0);
    const float* w = static_cast<const float*>(pd.wts) + static_cast<size_t>(iw) * pd.ktot + pbase + p0;
    uint32_t mask = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int o = 4 * g + e;
      const bool valid = o <= last;
      const int oc = valid ? o : last;
      mask |= valid ? (1u << e) : 0u;
      rb[e] = ld_c64((gf2ptr)(z + static_cast<uint32_t>(oc) * row_bytes + offQ));
      rw[e] = ld_const(w, oc);
    }
    return mask;
  };
  auto stage_q = [&](int buf, const float2 (&rb)[4], const float (&rw)[4], uint32_t mask) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float wq = ((mask >> e) & 1u) ? rw[e] : 0.f;
      split2(rb[e].x * wq, rb[e].y * wq, h[e], l[e]);
    }
    const int o = swz(lq, lg);
    const uint4 vh = uint4{h[0], h[1], h[2], h[3]};
    const uint4 vl = uint4{l[0], l[1], l[2], l[3]};
    *reinterpret_cast<uint4*>(&L.bh[buf][o]) = vh;
    *reinterpret_cast<uint4*>(&L.bl[buf][o]) = vl;
    *reinterpret_cast<uint4*>(&L.bih[buf][o]) = rot_neg4(vh);
    *reinterpret_cast<uint4*>(&L.bil[buf][o]) = rot_neg4(vl);
  };

  const int beg = a.wg_offsets[blockIdx.x];
  const int end = a.wg_offsets[blockIdx.x + 1];
  for (int ui = beg; ui < end; ++ui) {
    const Unit u = a.units[a.wg_units[ui]];
    const ProbDesc pd = a.probs[u.prob];
    const int npb = pd.npb;
    const int flush_pairs = pd.flush > 2 * kKC ? pd.flush / (2 * kKC) : 1;
    const uint32_t cQ = col_offset(u.tq * TQ + lq, npb);
    const uint32_t cP = (u.tp * TP + lp < npb ? static_cast<uint32_t>(u.tp * TP + lp) : 0u) * 16u;
    double2* part = a.partials + static_cast<size_t>(u.slot) * TP * TQ;
    // a wave whose 64 x 64 sub-tile lies entirely above the diagonal has no
    // entry the reduction reads: it stages and synchronises but skips its
    // MFMAs, leaving its SIMD to the other wave (tiles on the diagonal band)
    const bool active =
        __builtin_amdgcn_readfirstlane(u.tp * TP + wr * 64 + 63 >= u.tq * TQ + wc * 64) != 0;

    f32x16 cr[2][2], ci[2][2];
    zero_acc<2>(cr, ci);
    float2 rb[4];
    float rw[4];
    uint4 ph[2], pl[2];
    uint32_t mk = 0;

    // stage s: loads of stage s + 1 in flight during the MFMAs of stage s,
    // then staged into the other buffer; the second wave of each SIMD covers
    // the waits of the first.
    Cursor cur;
    bool have = cursor_first(u, a.blocks, cur);
    __syncthreads();  // previous unit's last MFMAs are done with the LDS
    if (have) {
      load_p(cur, npb, cP, ph, pl);
      mk = load_q(pd, u.iw, cur, npb, cQ, rb, rw);
      stage_p(0, ph, pl);
      stage_q(0, rb, rw, mk);
    }
    __syncthreads();
    int buf = 0;
    bool first_flush = true;
    while (have) {
      for (int ns = 0; ns < flush_pairs * 2 && have; ++ns) {
        Cursor nxt = cur;
        const bool more = cursor_next<kKC>(u, a.blocks, nxt);
        load_p(nxt, npb, cP, ph, pl);                       // unused when !more
        mk = load_q(pd, u.iw, nxt, npb, cQ, rb, rw);
        if (active) tall_mfma<LOLO, 2>(L, buf, wr, wc, g8, l32, cr, ci);
        stage_p(buf ^ 1, ph, pl);
        stage_q(buf ^ 1, rb, rw, mk);
        __syncthreads();
        cur = nxt;
        have = more;
        buf ^= 1;
      }
      tall_flush<2>(part, cr, ci, wr, wc, lane, first_flush);
      first_flush = false;
      zero_acc<2>(cr, ci);
    }
    if (first_flush) tall_flush<2>(part, cr, ci, wr, wc, lane, true);  // empty unit: zeros
  }
}

// ---------------------------------------------------------------------------
// FP32: v_mfma_f32_32x32x2f32, contraction slots (re, im) of one pair.  LDS
// holds the operands as complex64, rows = tile columns, 16 pairs per row
// (8 chunks of 2 pairs, XOR-swizzled).
// ---------------------------------------------------------------------------
// q: chunk of 2 pairs (16 B); slot q ^ ((r & 7) ^ r3): 8 consecutive rows and
// the 8 even (or odd) rows of 16 consecutive ones use distinct slots.
__device__ __forceinline__ int swz32(int row, int q) {
  return row * 32 + 4 * (q ^ ((row & 7) ^ ((row >> 3) & 1)));
}

template <int T>
__global__ __launch_bounds__(kNT, 1) void herk_fp32_kernel(HerkArgs a) {
  constexpr int NB = T / 64;
  constexpr int LG = kNT / T;         // loader groups
  constexpr int PPT = kKC / LG;       // pairs per thread
  __shared__ __attribute__((aligned(16))) float sA[2][T * 32];
  __shared__ __attribute__((aligned(16))) float sB[2][T * 32];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int g = lane >> 5;  // contraction slot: 0 = re, 1 = im
  const int l32 = lane & 31;
  const int lc = tid & (T - 1);
  const int lg = tid / T;
  int poff[PPT];
#pragma unroll
  for (int e = 0; e < PPT; ++e) poff[e] = PPT * lg + e;

  const int beg = a.wg_offsets[blockIdx.x];
  const int end = a.wg_offsets[blockIdx.x + 1];
  for (int ui = beg; ui < end; ++ui) {
    const Unit u = a.units[a.wg_units[ui]];
    const ProbDesc pd = a.probs[u.prob];
    const int npb = pd.npb;
    const int flush_stages = pd.flush > kKC ? pd.flush / kKC : 1;
    double2* part = a.partials + static_cast<size_t>(u.slot) * T * T;

    f32x16 cr[NB][NB], ci[NB][NB];
    zero_acc<NB>(cr, ci);
    float2 ra[PPT], rb[PPT];
    float rw[PPT];
    uint32_t mk = 0;
    const uint32_t cP = col_offset(u.tp * T + lc, npb), cQ = col_offset(u.tq * T + lc, npb);
    Cursor cur;
    bool have = cursor_first(u, a.blocks, cur);
    __syncthreads();
    if (have) mk = load_pairs<PPT>(a, pd, u.iw, cur, poff, npb, cP, cQ, ra, rb, rw);
    int buf = 0;
    bool first_flush = true;
    while (have) {
      for (int ns = 0; ns < flush_stages && have; ++ns) {
#pragma unroll
        for (int h = 0; h < PPT / 2; ++h) {
          const int q = (PPT / 2) * lg + h;  // chunk of pairs 2q, 2q + 1
          const float w0 = ((mk >> (2 * h)) & 1u) ? rw[2 * h] : 0.f;
          const float w1 = ((mk >> (2 * h + 1)) & 1u) ? rw[2 * h + 1] : 0.f;
          const float2 x0 = ra[2 * h];
          const float2 x1 = ra[2 * h + 1];
          const int o = swz32(lc, q);
          *reinterpret_cast<float4*>(&sA[buf][o]) = float4{x0.x, x0.y, x1.x, x1.y};
          *reinterpret_cast<float4*>(&sB[buf][o]) =
              float4{rb[2 * h].x * w0, rb[2 * h].y * w0, rb[2 * h + 1].x * w1, rb[2 * h + 1].y * w1};
        }
        Cursor nxt = cur;
        const bool more = cursor_next<kKC>(u, a.blocks, nxt);
        mk = load_pairs<PPT>(a, pd, u.iw, nxt, poff, npb, cP, cQ, ra, rb, rw);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q) {  // two pairs per chunk
          float4 av[NB], bv[NB];
#pragma unroll
          for (int i = 0; i < NB; ++i)
            av[i] = *reinterpret_cast<const float4*>(&sA[buf][swz32(wr * (T / 2) + i * 32 + l32, q)]);
#pragma unroll
          for (int j = 0; j < NB; ++j)
            bv[j] = *reinterpret_cast<const float4*>(&sB[buf][swz32(wc * (T / 2) + j * 32 + l32, q)]);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            float a0[NB], b0r[NB], b0i[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
              const float re = h ? av[i].z : av[i].x;
              const float im = h ? av[i].w : av[i].y;
              a0[i] = g ? im : re;
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
              const float re = h ? bv[j].z : bv[j].x;
              const float im = h ? bv[j].w : bv[j].y;
              b0r[j] = g ? im : re;
              b0i[j] = g ? -re : im;
            }
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
              for (int j = 0; j < NB; ++j) {
                cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[i], b0r[j], cr[i][j], 0, 0, 0);
                ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[i], b0i[j], ci[i][j], 0, 0, 0);
              }
          }
        }
        cur = nxt;
        have = more;
        buf ^= 1;
      }
      flush_tile<T, NB>(part, cr, ci, wr, wc, lane, first_flush);
      first_flush = false;
      zero_acc<NB>(cr, ci);
    }
    if (first_flush) flush_tile<T, NB>(part, cr, ci, wr, wc, lane, true);  // empty unit: zeros
  }
}

}  // namespace

// Tile tables: {tile, pairs per stage, cap of the FP32 run length (pairs),
// threads}.  BF16X3 with CHI0_BF16_LOLO selects the variant adding lo*lo.
static const TileConfig kBf16Tiles[] = {
    {128, kKC, 4096, kNT, 128},   // 0: software-pipelined kernel
    {128, kKC, 4096, kNT, 128},   // 1: staging and MFMAs in sequence
    {64, kKC, 4096, kNT, 64},     // 2
    {128, kKC, 1024, kNT, 128},   // 3: pipelined, shorter FP32 runs
    {128, kKC, 4096, kNT, 128},   // 4: in sequence, two workgroups per CU
    {256, kKC, 4096, kNT, 128, 1},   // 5: pipelined, tall 256 x 128 tiles, P pre-split
    {128, kKC, 4096, kNT, 128},      // 6: as 0, compiler scheduling (no interleave hints)
    {256, kKC, 4096, kNT, 128, 1},   // 7: as 5, compiler scheduling
    {256, kKC, 4096, 512, 128, 1},   // 8: tall tiles, 8 waves (two per SIMD)
    {256, kKC, 4096, kNT, 128, 1},   // 9: tall tiles, operands straight to registers
    {256, kKC, 4096, kNT, 128, 1},   // 10: as 9, with issue-order hints
    {128, kKC, 4096, kNT, 64, 1, 4},  // 11: as 9, one 128 x 64 work list per wave
    {128, kKC, 4096, kNT, 64, 1, 4},  // 12: as 11, with issue-order hints
    {128, kKC, 4096, kNT, 64, 1, 1, 4},  // 13: 128 x 64 tiles, four frequencies per
                                         //     workgroup sharing LDS-staged operands
    {128, kKC, 4096, kNT, 64, 1, 1, 4},  // 14: as 13, with issue-order hints
    {128, kKC, 4096, kNT, 64, 1, 1, 4},  // 15: as 14, flushes by FP64 atomic adds
    {128, kKC, 4096, kNT, 64, 1, 1, 4, 1},  // 16: as 15, diagonal tiles leave out their
                                            //     blocks above the diagonal
    {128, kKC, 4096, kNT, 64, 1, 1, 4, 2},  // 17: as 16, light units dealt in locality order
    {128, kKC, 4096, kNT, 64, 1, 1, 4, 1, 16},  // 18: as 16, workgroups of an XCD in lockstep
    {128, kKC, 4096, kNT, 64, 1, 1, 4, 1, 16, 1},  // 19: as 18, planar partial tiles
    {128, kKC, 4096, kNT, 64, 1, 1, 4, 1, 16, 1},  // 20: as 19, Z loaded in 16-byte chunks
};
static const TileConfig kFp32Tiles[] = {
    {128, kKC, 4096, kNT, 128},
    {64, kKC, 4096, kNT, 64},
    {128, kKC, 4096, kNT, 64, 0, 1, 4, 1, 16, 1},   // 2: frequency groups on 128 x 64 tiles
};

int herk_bf16x3_tile_count() { return sizeof(kBf16Tiles) / sizeof(kBf16Tiles[0]); }
TileConfig herk_bf16x3_tile(int idx) { return kBf16Tiles[idx]; }
template <int T, int OCC>
static void launch_bf16_seq(bool lolo, const HerkArgs& a, int nwg, hipStream_t s) {
  if (lolo)
    hipLaunchKernelGGL((herk_bf16x3_kernel<T, true, OCC>), dim3(nwg), dim3(kNT), 0, s, a);
  else
    hipLaunchKernelGGL((herk_bf16x3_kernel<T, false, OCC>), dim3(nwg), dim3(kNT), 0, s, a);
}

#define CHI0_BF16_KERNEL_LAUNCH(kern, lolo, hint, nwg, s, a)                                   \
  do {                                                                                         \
    if (lolo) {                                                                                \
      if (hint) hipLaunchKernelGGL((kern<true, true>), dim3(nwg), dim3(kNT), 0, s, a);         \
      else hipLaunchKernelGGL((kern<true, false>), dim3(nwg), dim3(kNT), 0, s, a);             \
    } else {                                                                                   \
      if (hint) hipLaunchKernelGGL((kern<false, true>), dim3(nwg), dim3(kNT), 0, s, a);        \
      else hipLaunchKernelGGL((kern<false, false>), dim3(nwg), dim3(kNT), 0, s, a);            \
    }                                                                                          \
  } while (0)

#define CHI0_BF16_TALL_GATHER_LAUNCH(lolo, hint, nwg, s, a)                                      \
  do {                                                                                           \
    if (lolo) {                                                                                  \
      if (hint) hipLaunchKernelGGL((herk_bf16x3_tall_kernel<true, true, true>), dim3(nwg),       \
                                   dim3(kNT), 0, s, a);                                          \
      else hipLaunchKernelGGL((herk_bf16x3_tall_kernel<true, false, true>), dim3(nwg),           \
                              dim3(kNT), 0, s, a);                                               \
    } else {                                                                                     \
      if (hint) hipLaunchKernelGGL((herk_bf16x3_tall_kernel<false, true, true>), dim3(nwg),      \
                                   dim3(kNT), 0, s, a);                                          \
      else hipLaunchKernelGGL((herk_bf16x3_tall_kernel<false, false, true>), dim3(nwg),          \
                              dim3(kNT), 0, s, a);                                               \
    }                                                                                            \
  } while (0)

hipError_t herk_bf16x3_launch(int idx, const HerkArgs& a, int nwg, hipStream_t s, bool gather) {
  if (idx < 0 || idx >= herk_bf16x3_tile_count()) return hipErrorInvalidValue;
  const bool lolo = (a.flags & 2) != 0;
  switch (idx) {
    case 0:
    case 3: CHI0_BF16_KERNEL_LAUNCH(herk_bf16x3_pipe_kernel, lolo, true, nwg, s, a); break;
    case 6: CHI0_BF16_KERNEL_LAUNCH(herk_bf16x3_pipe_kernel, lolo, false, nwg, s, a); break;
    case 1: launch_bf16_seq<128, 1>(lolo, a, nwg, s); break;
    case 2: launch_bf16_seq<64, 1>(lolo, a, nwg, s); break;
    case 4: launch_bf16_seq<128, 2>(lolo, a, nwg, s); break;
    case 5:
      if (gather) CHI0_BF16_TALL_GATHER_LAUNCH(lolo, true, nwg, s, a);
      else CHI0_BF16_KERNEL_LAUNCH(herk_bf16x3_tall_kernel, lolo, true, nwg, s, a);
      break;
    case 7:
      if (gather) CHI0_BF16_TALL_GATHER_LAUNCH(lolo, false, nwg, s, a);
      else CHI0_BF16_KERNEL_LAUNCH(herk_bf16x3_tall_kernel, lolo, false, nwg, s, a);
      break;
    case 9:
    case 10:
    case 11:
    case 12:
      return herk_bf16x3_direct_launch(lolo, idx == 10 || idx == 12, idx >= 11, a, nwg, s);
    case 13:
    case 14:
    case 15:
    case 16:
    case 17:
    case 18:
    case 19:
    case 20:
      return herk_bf16x3_wgroup_launch(lolo, idx >= 19 ? idx - 15 : idx >= 16 ? 3 : idx - 13, a, nwg, s);
    default:
      if (lolo)
        hipLaunchKernelGGL(herk_bf16x3_tall8_kernel<true>, dim3(nwg), dim3(512), 0, s, a);
      else
        hipLaunchKernelGGL(herk_bf16x3_tall8_kernel<false>, dim3(nwg), dim3(512), 0, s, a);
      break;
  }
  return hipGetLastError();
}
int herk_bf16x3_max_wg_per_cu(int idx) {
  int n = 0;
  hipError_t e;
  switch (idx) {
    case 0:
    case 3:
    case 6:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, herk_bf16x3_pipe_kernel<false, true>, kNT, 0);
      break;
    case 1:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, herk_bf16x3_kernel<128, false, 1>, kNT, 0);
      break;
    case 2:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, herk_bf16x3_kernel<64, false, 1>, kNT, 0);
      break;
    case 4:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, herk_bf16x3_kernel<128, false, 2>, kNT, 0);
      break;
    case 5:
    case 7:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, herk_bf16x3_tall_kernel<false, true>, kNT, 0);
      break;
    case 9:
    case 10:
    case 11:
    case 12:
      return herk_bf16x3_direct_max_wg_per_cu();
    case 13:
    case 14:
    case 15:
    case 16:
    case 17:
    case 18:
    case 19:
    case 20:
      return herk_bf16x3_wgroup_max_wg_per_cu();
    default:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, herk_bf16x3_tall8_kernel<false>, 512, 0);
      break;
  }
  return e == hipSuccess && n > 0 ? n : 1;
}

int herk_fp32_tile_count() { return sizeof(kFp32Tiles) / sizeof(kFp32Tiles[0]); }
TileConfig herk_fp32_tile(int idx) { return kFp32Tiles[idx]; }
hipError_t herk_fp32_launch(int idx, const HerkArgs& a, int nwg, hipStream_t s) {
  if (idx < 0 || idx >= herk_fp32_tile_count()) return hipErrorInvalidValue;
  if (idx == 2) return herk_fp32_wgroup_launch(a, nwg, s);
  if (kFp32Tiles[idx].tile == 128)
    hipLaunchKernelGGL(herk_fp32_kernel<128>, dim3(nwg), dim3(kNT), 0, s, a);
  else
    hipLaunchKernelGGL(herk_fp32_kernel<64>, dim3(nwg), dim3(kNT), 0, s, a);
  return hipGetLastError();
}
int herk_fp32_max_wg_per_cu(int idx) {
  if (idx == 2) return herk_fp32_wgroup_max_wg_per_cu();
  int n = 0;
  hipError_t e = kFp32Tiles[idx].tile == 128
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, herk_fp32_kernel<128>, kNT, 0)
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, herk_fp32_kernel<64>, kNT, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}

}  // namespace chi0
