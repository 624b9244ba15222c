// BF16x3 (and FP32) weighted Hermitian rank-K update on frequency-group
// units.  The FP32 form, further down, shares the units, runs, lockstep and
// flushes and replaces the split stage (see "FP32 path").
//
// Same contraction as the other rank-K kernels (S[P][Q] = sum_pairs
// conj(Z[pair][P]) * (c * Z[pair][Q]) on one 128 x 64 lower tile, chi0 = -S,
// Eq.(polfx) at i*omega), but a unit holds up to four frequencies of one tile
// and pair range, and wave w of the workgroup accumulates frequency iw + w.
// The frequencies share their operands -- Z and its pre-split planes are the
// same, only the pair weight c differs -- so the workgroup stages each
// 32-pair stage of the tile's operands once into LDS:
//   P: the pre-split bf16 hi / lo words of the 128 tile rows (32 KB),
//   Q: the raw complex64 Z of the 64 tile columns (16 KB),
//   the pair weights of the four frequencies (512 B),
// and every wave reads its MFMA fragments from there, scales its Q side by its
// own frequency's weights, splits it into bf16 hi / lo words (plain and
// rotated to (im, -re)) and issues the BF16x3 MFMAs.  Global traffic is a
// quarter of what four waves loading their own operands would need, and the
// barrier of every stage keeps the four waves, which do the same work, on
// the same pairs.
//
// Pipeline of a stage (three LDS buffers, one barrier per stage): the next
// stage is loaded straight from global memory into another LDS buffer
// (buffer loads with an LDS destination: no staging registers) while the
// current one is computed; the barrier before the stage's last k-step waits
// for those loads, and the third buffer lets the loads of the stage after
// next start right after that barrier.  Within a stage, the fragments of a
// k-step (8 pairs) are read from LDS while the previous k-step's MFMAs issue,
// and each column block's conversion runs while the other column block's
// MFMAs issue.  Loads past the run's pairs or the block's planes read zeros
// (raw buffer bounds), so the tails need no masks.  The FP32 accumulators
// are flushed to FP64 between runs of at most the problem's flush length.
#include "bf16_tall.h"
#include "common.h"
#include "herk_common.h"

namespace chi0 {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef const char __attribute__((address_space(1)))* gcptr;

constexpr int kWgPairs = 32;                          // pairs per stage
constexpr int kWgPBytes = 2 * (kWgPairs / 4) * 128 * 16;   // hi + lo planes, 128 rows
constexpr int kWgQBytes = kWgPairs * 64 * 8;          // raw Z, 64 columns
constexpr int kWgWBytes = 4 * 64 * 4;                 // weights, 64 pairs per frequency
constexpr int kWgBuf = kWgPBytes + kWgQBytes + kWgWBytes;

// Raw buffer resource over [base, base + bytes): loads past the end read 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t wg_rsrc(gcptr base, int32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, 0, bytes > 0 ? bytes : 0, 0x00020000);
}

// Byte counts of a run capped at 2^31 - 1 (far beyond what a run reads).
__device__ __forceinline__ int32_t wg_cap(int64_t bytes) {
  return bytes >= INT32_MAX ? INT32_MAX : static_cast<int32_t>(bytes);
}

typedef __attribute__((address_space(3))) void* lds_ptr;

// Bases of one run (pairs [q0, q0 + nv) of a block).
struct WgRun {
  gcptr hi, lo;       // pre-split planes at the run's first 4-pair group
  gcptr z;            // Z row of the run's first pair
  gcptr w;            // this wave's frequency's weight of the run's first pair
  int32_t pbytes;     // plane bytes from there to the block's padded end (capped)
  int32_t zbytes;     // Z bytes of the run's pairs
  int32_t wbytes;     // weight bytes from there to the end of the problem's table (capped)
  int32_t chunk;      // bytes per 4-pair group of a plane (npb * 16)
  int32_t row;        // bytes per Z row (npb * 8)
};

// Per-lane byte offsets of the stage loads.  P: chunk m (16 bytes) of thread
// t is group (t / 128) + 2 (m % 4) of plane m / 4, tile row t % 128.  Z:
// dword m of thread t is pair (t + 256 m) / 128, tile column
// ((t + 256 m) % 128) / 2, part (re / im) t % 2; or, with 16-byte loads
// (launched only when npb is even: Z rows then stay 16-byte aligned), chunk m of
// lane l of wave w is pair 2 w + l / 32 + 8 m, tile columns 2 (l % 32) and
// 2 (l % 32) + 1 (an even column: below npb, or clamped to 0, together with
// the next one).
struct WgLane {
  uint32_t p[4];
  uint32_t q[2];      // m even / odd (4 (m / 2) rows are added per load)
  uint32_t q16;       // 16-byte Z loads: chunk 0 (8 m rows are added per load)
  uint32_t pf;        // FP32 path: dword t of a pair's 128 raw P values (row t / 2, part t % 2)
};

// Part PART (0..3) of the loads of stage st of the run into LDS buffer buf
// (0: P hi words, 1: P lo words, 2: Z dwords 0..7 (Q16: chunks 0, 1) and
// the weights, 3: Z dwords 8..15 (Q16: chunks 2, 3)): every wave writes
// 1 KB (16-byte loads) or 256 bytes (dword loads) per instruction, lane i
// at offset 16 i or 4 i of the wave's destination.  Both Z forms give the
// same LDS layout ([pair][column], complex64).
template <int PART, bool Q16>
__device__ __forceinline__ void wg_dma(const WgRun& r, int st, const WgLane& o, int wave, int lane,
                                       char* buf) {
  if constexpr (PART < 2) {
    const int32_t po = st * (kWgPairs / 4) * r.chunk;
    const __amdgpu_buffer_rsrc_t h = wg_rsrc((PART == 0 ? r.hi : r.lo) + po, r.pbytes - po);
#pragma unroll
    for (int m = 0; m < 4; ++m)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          h, (lds_ptr)(buf + (64 * wave + 256 * (m + 4 * PART)) * 16), 16, o.p[m], 0, 0, 0);
  } else {
    const int32_t zo = st * kWgPairs * r.row;
    const __amdgpu_buffer_rsrc_t z = wg_rsrc(r.z + zo, r.zbytes - zo);
    if constexpr (Q16) {
#pragma unroll
      for (int mm = 0; mm < 2; ++mm) {
        const int m = mm + 2 * (PART - 2);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            z, (lds_ptr)(buf + kWgPBytes + (64 * wave + 256 * m) * 16), 16,
            o.q16 + static_cast<uint32_t>(8 * m) * static_cast<uint32_t>(r.row), 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int mm = 0; mm < 8; ++mm) {
        const int m = mm + 8 * (PART - 2);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            z, (lds_ptr)(buf + kWgPBytes + (64 * wave + 256 * m) * 4), 4,
            o.q[m & 1] + static_cast<uint32_t>(4 * (m >> 1)) * static_cast<uint32_t>(r.row), 0, 0, 0);
      }
    }
    if constexpr (PART == 2) {
      const int32_t wo = st * kWgPairs * 4;
      const __amdgpu_buffer_rsrc_t w = wg_rsrc(r.w + wo, r.wbytes - wo);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(w, (lds_ptr)(buf + kWgPBytes + kWgQBytes + wave * 256),
                                               4, static_cast<uint32_t>(lane) * 4u, 0, 0, 0);
    }
  }
}

template <bool Q16>
__device__ __forceinline__ void wg_dma_all(const WgRun& r, int st, const WgLane& o, int wave,
                                           int lane, char* buf) {
  wg_dma<0, Q16>(r, st, o, wave, lane, buf);
  wg_dma<1, Q16>(r, st, o, wave, lane, buf);
  wg_dma<2, Q16>(r, st, o, wave, lane, buf);
  wg_dma<3, Q16>(r, st, o, wave, lane, buf);
}

// One k-step's fragments of one wave, read from a stage in LDS.
struct WgFrag {
  u32x4 ph[4], pl[4];  // P hi / lo words of row blocks 0..3
  u32x2 q[2][4];       // Z of column blocks 0..1, pairs 4 g + e
  u32x4 w;             // the wave's weights of pairs 4 g .. 4 g + 3
};

template <int DIAG>
__device__ __forceinline__ void wg_read(const char* buf, int ks, int g8, int l32, int wave,
                                        WgFrag& f) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (!diag_block_needed<DIAG>(i, 0) && !diag_block_needed<DIAG>(i, 1)) continue;
    const int off = ((2 * ks + g8) * 128 + 32 * i + l32) * 16;
    f.ph[i] = *reinterpret_cast<const u32x4*>(buf + off);
    f.pl[i] = *reinterpret_cast<const u32x4*>(buf + off + kWgPBytes / 2);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      f.q[j][e] = *reinterpret_cast<const u32x2*>(
          buf + kWgPBytes + ((8 * ks + 4 * g8 + e) * 64 + 32 * j + l32) * 8);
  f.w = *reinterpret_cast<const u32x4*>(buf + kWgPBytes + kWgQBytes + wave * 256 +
                                          (8 * ks + 4 * g8) * 4);
}

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt not waited for).
constexpr int kVmcnt0 = 0x3F70;

__device__ __forceinline__ uint32_t wg_pack_rot(float re, float im) {
  uint32_t r;
  asm("v_cvt_pk_bf16_f32 %0, %1, -%2" : "=v"(r) : "v"(im), "v"(re));
  return r;
}

struct WgWords {
  u32x4 h[2], l[2], rh[2], rl[2];
};

// Column block j of a k-step into the wave's Q words (c Z split into bf16 hi
// / lo, plain (re, im) and rotated (im, -re)).
__device__ __forceinline__ void wg_convert(const WgFrag& f, int j, WgWords& o) {
#pragma clang fp contract(off)
  uint32_t h[4], l[4], rh[4], rl[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const float c = __uint_as_float(f.w[e]);
    const float x = __uint_as_float(f.q[j][e].x) * c;
    const float y = __uint_as_float(f.q[j][e].y) * c;
    h[e] = pack_bf16x2(x, y);
    // the packed word itself is unpacked: left visible, the compiler
    // re-packs x alone for its low half (one more conversion per value)
    asm("" : "+v"(h[e]));
    const float x1 = x - bf16_lo_to_f32(h[e]);
    const float y1 = y - bf16_hi_to_f32(h[e]);
    l[e] = pack_bf16x2(x1, y1);
    rh[e] = wg_pack_rot(x, y);
    rl[e] = wg_pack_rot(x1, y1);
  }
  o.h[j] = u32x4{h[0], h[1], h[2], h[3]};
  o.l[j] = u32x4{l[0], l[1], l[2], l[3]};
  o.rh[j] = u32x4{rh[0], rh[1], rh[2], rh[3]};
  o.rl[j] = u32x4{rl[0], rl[1], rl[2], rl[3]};
}

__device__ __forceinline__ bf16x8 wfrag(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

template <bool LOLO, int DIAG>
__device__ __forceinline__ void wg_mfma(const WgFrag& p, const WgWords& q, int j, f32x16 (&cr)[4][2],
                                        f32x16 (&ci)[4][2]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (!diag_block_needed<DIAG>(i, j)) continue;
    cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wfrag(p.ph[i]), wfrag(q.h[j]), cr[i][j], 0, 0, 0);
    ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wfrag(p.ph[i]), wfrag(q.rh[j]), ci[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (!diag_block_needed<DIAG>(i, j)) continue;
    cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wfrag(p.ph[i]), wfrag(q.l[j]), cr[i][j], 0, 0, 0);
    ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wfrag(p.ph[i]), wfrag(q.rl[j]), ci[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (!diag_block_needed<DIAG>(i, j)) continue;
    cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wfrag(p.pl[i]), wfrag(q.h[j]), cr[i][j], 0, 0, 0);
    ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wfrag(p.pl[i]), wfrag(q.rh[j]), ci[i][j], 0, 0, 0);
  }
  if (LOLO) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (!diag_block_needed<DIAG>(i, j)) continue;
      cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wfrag(p.pl[i]), wfrag(q.l[j]), cr[i][j], 0, 0, 0);
      ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wfrag(p.pl[i]), wfrag(q.rl[j]), ci[i][j], 0, 0, 0);
    }
  }
}

__device__ __forceinline__ void wg_zero(f32x16 (&cr)[4][2], f32x16 (&ci)[4][2]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cr[i][j] = f32x16{0};
      ci[i][j] = f32x16{0};
    }
}

// Issue order of a k-step with NDMA stage loads: the column-block-0 MFMAs
// with the column-block-1 conversion (two VALU per MFMA), the next
// k-step's fragment reads and the loads between them, then the
// column-block-1 MFMAs with the next k-step's column-block-0 conversion.
template <int NDMA>
__device__ __forceinline__ void wg_order() {
#pragma unroll
  for (int m = 0; m < 24; ++m) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
    __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);   // VALU
    if (m < 17) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);    // LDS read
    if (m < NDMA) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // buffer load
  }
#pragma unroll
  for (int m = 0; m < 24; ++m) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
  }
}

// K-step ks of the stage in `cur` (fragments in fc, its column-block-0 words
// already in W), reading the next k-step's fragments (k-step ks + 1 of `cur`,
// or k-step 0 of the next stage from `nxt`) into fn and converting their
// column block 0.
template <bool LOLO, int DIAG>
__device__ __forceinline__ void wg_kstep(const char* src, int ksn, int g8, int l32, int wave,
                                         const WgFrag& fc, WgFrag& fn, WgWords& W,
                                         f32x16 (&cr)[4][2], f32x16 (&ci)[4][2]) {
  wg_read<DIAG>(src, ksn, g8, l32, wave, fn);
  wg_convert(fc, 1, W);
  wg_mfma<LOLO, DIAG>(fc, W, 0, cr, ci);
  wg_convert(fn, 0, W);
  wg_mfma<LOLO, DIAG>(fc, W, 1, cr, ci);
}

// The stages of one run (nst stages of 32 pairs) into the accumulators.
// Three LDS buffers, stage s in buffer s % 3.  The barrier of stage s (after
// its k-step 2) follows the loads of stage s + 1, issued since the previous
// barrier, and every read of stage s - 1; the loads of stage s + 2 start
// after it, and so do the reads of stage s + 1 (k-step 3 prefetches its
// first fragments).  DIAG (tiles crossing the diagonal) leaves out the
// MFMAs and P reads of blocks entirely above it.
template <bool LOLO, bool HINT, int DIAG, bool Q16>
__device__ __forceinline__ void wg_stages(const WgRun& r, const WgLane& o, int nst, int wave,
                                          int lane, int g8, int l32, char (*lds)[kWgBuf],
                                          f32x16 (&cr)[4][2], f32x16 (&ci)[4][2]) {
  wg_dma_all<Q16>(r, 0, o, wave, lane, lds[0]);
  __builtin_amdgcn_s_waitcnt(kVmcnt0);
  __syncthreads();
  WgFrag F0, F1;
  WgWords W;
  wg_read<DIAG>(lds[0], 0, g8, l32, wave, F0);
  wg_convert(F0, 0, W);
  wg_dma<0, Q16>(r, 1, o, wave, lane, lds[1]);
  int bc = 0;   // buffer of stage st
  for (int st = 0; st < nst; ++st) {
    const int bn = bc == 2 ? 0 : bc + 1, bnn = bn == 2 ? 0 : bn + 1;
    const char* cur = lds[bc];
    wg_kstep<LOLO, DIAG>(cur, 1, g8, l32, wave, F0, F1, W, cr, ci);
    wg_dma<1, Q16>(r, st + 1, o, wave, lane, lds[bn]);
    if (HINT) wg_order<4>();
    __builtin_amdgcn_sched_barrier(0);
    wg_kstep<LOLO, DIAG>(cur, 2, g8, l32, wave, F1, F0, W, cr, ci);
    wg_dma<2, Q16>(r, st + 1, o, wave, lane, lds[bn]);
    if (HINT) wg_order<Q16 ? 3 : 9>();
    __builtin_amdgcn_sched_barrier(0);
    wg_kstep<LOLO, DIAG>(cur, 3, g8, l32, wave, F0, F1, W, cr, ci);
    wg_dma<3, Q16>(r, st + 1, o, wave, lane, lds[bn]);
    if (HINT) wg_order<Q16 ? 2 : 8>();
    __builtin_amdgcn_s_waitcnt(kVmcnt0);   // this wave's loads of stage st + 1
    __syncthreads();
    wg_kstep<LOLO, DIAG>(lds[bn], 0, g8, l32, wave, F1, F0, W, cr, ci);
    wg_dma<0, Q16>(r, st + 2, o, wave, lane, lds[bnn]);
    if (HINT) wg_order<4>();
    __builtin_amdgcn_sched_barrier(0);
    bc = bn;
  }
  __builtin_amdgcn_s_waitcnt(kVmcnt0);     // loads past the run's stages
  __syncthreads();
}

// FP32 path.  A 32-pair stage in LDS holds the raw complex64 Z of the tile's
// 128 P rows as [pair][row] (32 KB, where the BF16x3 stage holds the
// pre-split words), the 64 Q columns as [pair][column] and the weights, as
// the BF16x3 stage does; stage s + 1 is loaded while stage s is computed
// (two buffers: a buffer is refilled only after the barrier that ends the
// stage that read it).  Per pair and wave: the A operand of row block i is
// lane l -> (row 32 i + l % 32, re if l < 32 else im), the B operand of
// column block j is c (re, im) of column 32 j + l % 32 and the rotated one
// c (im, -re), so one v_mfma_f32_32x32x2f32 gives Re and one Im of
// conj(Z_P) c Z_Q (the contraction index runs over re and im).
__device__ __forceinline__ void f32_dma(const WgRun& r, int st, const WgLane& o, int wave, int lane,
                                        char* buf) {
  const int32_t zo = st * kWgPairs * r.row;
  const __amdgpu_buffer_rsrc_t z = wg_rsrc(r.z + zo, r.zbytes - zo);
  // Running offsets, opaque to the compiler, so that the 48 offsets are not
  // all kept in registers across the stage (their reloads would wait for
  // the loads in flight).  P: pair m, dword t of its 128 rows.  Q: dword
  // t + 256 m is pair t / 128 + 2 m, column (t % 128) / 2, part t % 2.
  uint32_t off = o.pf;
#pragma unroll
  for (int m = 0; m < kWgPairs; ++m) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(z, (lds_ptr)(buf + (256 * m + 64 * wave) * 4), 4, off,
                                             0, 0, 0);
    off += static_cast<uint32_t>(r.row);
    asm volatile("" : "+v"(off));
  }
  off = o.q[0];
#pragma unroll
  for (int m = 0; m < kWgPairs / 2; ++m) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(
        z, (lds_ptr)(buf + kWgPBytes + (64 * wave + 256 * m) * 4), 4, off, 0, 0, 0);
    off += 2u * static_cast<uint32_t>(r.row);
    asm volatile("" : "+v"(off));
  }
  const int32_t wo = st * kWgPairs * 4;
  const __amdgpu_buffer_rsrc_t w = wg_rsrc(r.w + wo, r.wbytes - wo);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(w, (lds_ptr)(buf + kWgPBytes + kWgQBytes + wave * 256),
                                           4, static_cast<uint32_t>(lane) * 4u, 0, 0, 0);
}

// One pair's operands as read from LDS (weight applied later).
struct F32Frag {
  float a[4];    // A operands of the row blocks
  float q[2];    // (re or im) of column block j, the B operand before scaling
  float qr[2];   // the other part, for the rotated B operand
};

template <int DIAG>
__device__ __forceinline__ void f32_read(const float* P, const float* Q, int p, int l32, int h,
                                         F32Frag& f) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
    f.a[i] = (diag_block_needed<DIAG>(i, 0) || diag_block_needed<DIAG>(i, 1))
                 ? P[(p * 128 + 32 * i + l32) * 2 + h] : 0.0f;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    f.q[j] = Q[(p * 64 + 32 * j + l32) * 2 + h];
    f.qr[j] = Q[(p * 64 + 32 * j + l32) * 2 + (1 - h)];
  }
}

template <int DIAG>
__device__ __forceinline__ void f32_mfma(const F32Frag& f, float c, float cs, f32x16 (&cr)[4][2],
                                         f32x16 (&ci)[4][2]) {
  float b[2], bp[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    b[j] = f.q[j] * c;
    bp[j] = f.qr[j] * cs;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (!diag_block_needed<DIAG>(i, j)) continue;
      cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(f.a[i], b[j], cr[i][j], 0, 0, 0);
      ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(f.a[i], bp[j], ci[i][j], 0, 0, 0);
    }
}

// The 32 pairs of a stage, software-pipelined: the operands of pair p + 1
// are read from LDS while the MFMAs of pair p issue.
template <int DIAG>
__device__ __forceinline__ void f32_pairs(const char* buf, int wave, int lane, f32x16 (&cr)[4][2],
                                          f32x16 (&ci)[4][2]) {
  const int l32 = lane & 31, h = lane >> 5;
  const float sgn = h ? -1.0f : 1.0f;
  const float* P = reinterpret_cast<const float*>(buf);
  const float* Q = reinterpret_cast<const float*>(buf + kWgPBytes);
  const float* W = reinterpret_cast<const float*>(buf + kWgPBytes + kWgQBytes + wave * 256);
  F32Frag f0, f1;
  f32_read<DIAG>(P, Q, 0, l32, h, f0);
#pragma unroll 2
  for (int p = 0; p < kWgPairs; p += 2) {
    const float c0 = W[p], c1 = W[p + 1];
    f32_read<DIAG>(P, Q, p + 1, l32, h, f1);
    f32_mfma<DIAG>(f0, c0, c0 * sgn, cr, ci);
    if (p + 2 < kWgPairs) f32_read<DIAG>(P, Q, p + 2, l32, h, f0);
    f32_mfma<DIAG>(f1, c1, c1 * sgn, cr, ci);
  }
}

template <int DIAG>
__device__ __forceinline__ void f32_stages(const WgRun& r, const WgLane& o, int nst, int wave,
                                           int lane, char (*lds)[kWgBuf], f32x16 (&cr)[4][2],
                                           f32x16 (&ci)[4][2]) {
  f32_dma(r, 0, o, wave, lane, lds[0]);
  __builtin_amdgcn_s_waitcnt(kVmcnt0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int b = st & 1;
    if (st + 1 < nst) f32_dma(r, st + 1, o, wave, lane, lds[b ^ 1]);
    f32_pairs<DIAG>(lds[b], wave, lane, cr, ci);
    __builtin_amdgcn_s_waitcnt(kVmcnt0);   // this wave's loads of stage st + 1
    __syncthreads();
  }
}

// Lockstep of the workgroups of one XCD (workgroup b runs on XCD b % 8):
// before a run, wave 0 publishes the stages its workgroup has done and, while
// that is more than sync_slack stages ahead of the slowest peer on the XCD,
// sleeps and polls again, at most kSyncPolls times (the wait always ends;
// it only keeps the peers, which stream the same pair ranges in the same
// rounds, close enough to share the XCD's L2).  A wait that reaches the
// limit turns the lockstep off for the rest of the launch in this workgroup
// (returns false), so a peer that never catches up costs one bounded wait.
// A finished workgroup publishes INT_MAX, so it never holds the others, in
// this launch or the next.  The other waves meet wave 0 at the run's first
// barrier.
constexpr int kSyncPolls = 2048;

__device__ __forceinline__ bool wg_sync(const HerkArgs& a, int done, int wave, int lane) {
  if (wave != 0) return true;
  int32_t* prog = a.sync_prog;
  if (lane == 0) __hip_atomic_store(prog + blockIdx.x, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int peer = static_cast<int>(blockIdx.x & 7u) + 8 * lane;
  const bool mine = peer < static_cast<int>(gridDim.x);
  for (int it = 0; it < kSyncPolls; ++it) {
    int v = mine ? __hip_atomic_load(prog + peer, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                 : INT32_MAX;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    v = __builtin_amdgcn_readfirstlane(v);
    if (done - v <= a.sync_slack) return true;
    __builtin_amdgcn_s_sleep(8);
  }
  return false;
}

// The wave's 128 x 64 accumulators into its partial tile stored as two
// planes (128 x 64 real parts, then 128 x 64 imaginary parts): the real and
// the imaginary atomic adds of a flush then each cover whole cache lines
// (32 lanes, 256 contiguous bytes) instead of every other 8 bytes of the
// same lines.  Blocks above the diagonal of a diagonal tile are skipped as
// in tall_flush.
template <bool ATOM, int DIAG>
__device__ __forceinline__ void wg_flush_planar(double2* slot, const f32x16 (&cr)[4][2],
                                                const f32x16 (&ci)[4][2], int lane, bool first) {
  constexpr int TQ = 64, NE = 128 * 64;
  typedef double __attribute__((address_space(1)))* gdp;
  double* pre = reinterpret_cast<double*>(slot);
  double* pim = pre + NE;
  int base = 4 * (lane >> 5) * TQ + (lane & 31);
  asm volatile("" : "+v"(base));
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (!diag_block_needed<DIAG>(i, j)) continue;
      const int b0 = base + i * 32 * TQ + j * 32;
      if (ATOM && !first) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int e = b0 + (8 * (r >> 2) + (r & 3)) * TQ;
          __builtin_amdgcn_global_atomic_fadd_f64((gdp)(pre + e), static_cast<double>(cr[i][j][r]));
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int e = b0 + (8 * (r >> 2) + (r & 3)) * TQ;
          __builtin_amdgcn_global_atomic_fadd_f64((gdp)(pim + e), static_cast<double>(ci[i][j][r]));
        }
        continue;
      }
      double o[16], q[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) o[r] = q[r] = 0.0;
      if (!first) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int e = b0 + (8 * (r >> 2) + (r & 3)) * TQ;
          o[r] = pre[e];
          q[r] = pim[e];
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int e = b0 + (8 * (r >> 2) + (r & 3)) * TQ;
        pre[e] = static_cast<double>(cr[i][j][r]) + o[r];
        pim[e] = static_cast<double>(ci[i][j][r]) + q[r];
      }
    }
}

// One unit (a tile, a pair range, up to four frequencies: wave w takes
// frequency u.iw + w) from its ranges' stages into the wave's partial tile.
// DIAG (0, or 1 / 2 for the tiles left / right of the diagonal) is fixed per
// unit, so each kind has its own copy of the run loop and registers.
template <bool LOLO, bool HINT, bool ATOM, bool PLANAR, int DIAG, bool F32, bool Q16>
__device__ __forceinline__ void wg_unit(const HerkArgs& a, const Unit& u, const ProbDesc& pd,
                                        int tid, int wave, int lane, int g8, int l32,
                                        char (*lds)[kWgBuf], int& done, bool& sync_on) {
  constexpr int TP = 128, TQ = 64;
  const int npb = pd.npb;
  const bool active = wave < u.nw;
  const int r0 = u.tp * TP, c0 = u.tq * TQ;
  const int32_t chunk = npb * 16, row = npb * 8;
  WgLane o;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int col = r0 + (tid & 127);
    o.p[m] = static_cast<uint32_t>((tid >> 7) + 2 * m) * static_cast<uint32_t>(chunk) +
             static_cast<uint32_t>(col < npb ? col : 0) * 16u;
  }
#pragma unroll
  for (int h2 = 0; h2 < 2; ++h2) {
    // dword t + 256 m, m = 2 m2 + h2: pair 2 m2 + (t + 256 h2) / 128, column
    // ((t + 256 h2) % 128) / 2, part t % 2
    const int d = tid + 256 * h2;
    const int col = c0 + ((d & 127) >> 1);
    o.q[h2] = static_cast<uint32_t>(d >> 7) * static_cast<uint32_t>(row) +
              static_cast<uint32_t>(col < npb ? col : 0) * 8u + static_cast<uint32_t>(d & 1) * 4u;
  }
  {
    const int col = c0 + 2 * (lane & 31);
    o.q16 = static_cast<uint32_t>(2 * wave + (lane >> 5)) * static_cast<uint32_t>(row) +
            static_cast<uint32_t>(col < npb ? col : 0) * 8u;
  }
  {
    const int prow = r0 + (tid >> 1);
    o.pf = static_cast<uint32_t>(prow < npb ? prow : 0) * 8u + static_cast<uint32_t>(tid & 1) * 4u;
  }
  // FP32 runs of at most the problem's flush length (a multiple of 16
  // pairs), made of granules of R pairs: whole 32-pair stages when the
  // length allows, else 16 pairs (the stage's second half then reads zeros)
  const int R = pd.flush >= kWgPairs ? kWgPairs : 16;
  const int fr = max(1, pd.flush / R);
  double2* part = a.partials + static_cast<size_t>(u.slot + wave * u.wstride) * TP * TQ;
  // this wave's frequency (a wave past the group's frequencies computes
  // with the last one's weights and writes nothing)
  const int wv = min(wave, u.nw - 1);
  const float* wbase = static_cast<const float*>(pd.wts) + static_cast<size_t>(u.iw + wv) * pd.ktot;
  const int64_t wend = (static_cast<int64_t>(pd.nomega) - u.iw - wv) * pd.ktot;  // floats from wbase

  f32x16 cr[4][2], ci[4][2];
  wg_zero(cr, ci);
  bool first = true;
  int acc = 0;   // granules in the FP32 accumulators
  for (int b = u.b0; b <= u.b1; ++b) {
    const BlockDesc* bp = a.blocks + b;
    const int kb = block_pairs(a.blocks, b);
    const int p0 = (b == u.b0) ? u.p0 : 0;
    const int p1 = (b == u.b1) ? u.p1 : kb;
    if (p0 >= p1) continue;
    const gcptr zs = (gcptr)ld_const(&bp->zs, 0);
    const int64_t plane = ld_const(&bp->zs_plane, 0);
    const gcptr z = (gcptr)ld_const(&bp->z, 0);
    const int64_t pbase = ld_const(&bp->pair_base, 0);
    const int64_t groups = presplit_groups(kb);
    const int ng = (p1 - p0 + R - 1) / R;   // granules of the segment (p0: a multiple of 16)
    for (int g0 = 0; g0 < ng;) {
      const int len = min(fr - acc, ng - g0);
      const int q0 = p0 + R * g0;
      const int nv = min(p1, q0 + R * len) - q0;
      WgRun r;
      r.chunk = chunk;
      r.row = row;
      r.hi = zs + static_cast<int64_t>(q0 >> 2) * chunk;
      r.lo = r.hi + plane;
      r.pbytes = wg_cap((groups - (q0 >> 2)) * static_cast<int64_t>(chunk));
      r.z = z + static_cast<int64_t>(q0) * row;
      r.zbytes = wg_cap(static_cast<int64_t>(nv) * row);
      r.w = (gcptr)(wbase + pbase + q0);
      r.wbytes = wg_cap((wend - pbase - q0) * 4);
      const int nst = (nv + kWgPairs - 1) / kWgPairs;
      if (a.sync_prog != nullptr && sync_on) sync_on = wg_sync(a, done, wave, lane);
      if constexpr (F32) f32_stages<DIAG>(r, o, nst, wave, lane, lds, cr, ci);
      else wg_stages<LOLO, HINT, DIAG, Q16>(r, o, nst, wave, lane, g8, l32, lds, cr, ci);
      done += nst;
      g0 += len;
      acc += len;
      if (acc >= fr) {
        if (active) {
          if (PLANAR) wg_flush_planar<ATOM, DIAG>(part, cr, ci, lane, first);
          else tall_flush<4, TQ, ATOM, DIAG>(part, cr, ci, 0, 0, lane, first);
        }
        first = false;
        acc = 0;
        wg_zero(cr, ci);
      }
    }
  }
  if (active && (first || acc > 0)) {
    if (PLANAR) wg_flush_planar<ATOM, DIAG>(part, cr, ci, lane, first);
    else tall_flush<4, TQ, ATOM, DIAG>(part, cr, ci, 0, 0, lane, first);
  }
}

template <bool LOLO, bool HINT, bool ATOM, bool SKIP, bool PLANAR, bool F32, bool Q16>
__device__ __forceinline__ void wg_body(const HerkArgs& a, char (*lds)[kWgBuf]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g8 = lane >> 5;
  const int l32 = lane & 31;

  // work list, units and problem descriptors through the scalar cache (they
  // are uniform: every branch on them stays a scalar branch)
  const int beg = ld_const(a.wg_offsets, static_cast<int>(blockIdx.x));
  const int end = ld_const(a.wg_offsets, static_cast<int>(blockIdx.x) + 1);
  int done = 0;          // stages of this workgroup's runs so far (XCD lockstep)
  bool sync_on = true;    // lockstep still on for this workgroup
  for (int ui = beg; ui < end; ++ui) {
    const Unit u = ld_unit(a.units, ld_const(a.wg_units, ui));
    const ProbDesc pd = ld_prob(a.probs, u.prob);
    // tiles crossing the diagonal (TP = 2 TQ): their blocks above it are
    // left out with SKIP (the reduction never reads those entries)
    const int diag = !SKIP ? 0 : u.tq == 2 * u.tp ? 1 : u.tq == 2 * u.tp + 1 ? 2 : 0;
    if (diag == 0) wg_unit<LOLO, HINT, ATOM, PLANAR, 0, F32, Q16>(a, u, pd, tid, wave, lane, g8, l32, lds, done, sync_on);
    else if (diag == 1) wg_unit<LOLO, HINT, ATOM, PLANAR, 1, F32, Q16>(a, u, pd, tid, wave, lane, g8, l32, lds, done, sync_on);
    else wg_unit<LOLO, HINT, ATOM, PLANAR, 2, F32, Q16>(a, u, pd, tid, wave, lane, g8, l32, lds, done, sync_on);
  }
  if (a.sync_prog != nullptr && tid == 0)
    __hip_atomic_store(a.sync_prog + blockIdx.x, INT32_MAX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool LOLO, bool HINT, bool ATOM, bool SKIP, bool PLANAR, bool Q16>
__global__ __launch_bounds__(kNT, 1) void herk_bf16x3_wgroup_kernel(HerkArgs a) {
  __shared__ __attribute__((aligned(16))) char lds[3][kWgBuf];
  wg_body<LOLO, HINT, ATOM, SKIP, PLANAR, false, Q16>(a, lds);
}

// FP32 contraction on the same units (frequency groups, diagonal blocks
// left out, XCD lockstep, planar partial tiles, atomic flushes).
__global__ __launch_bounds__(kNT, 1) void herk_fp32_wgroup_kernel(HerkArgs a) {
  __shared__ __attribute__((aligned(16))) char lds[2][kWgBuf];
  wg_body<false, false, true, true, true, true, false>(a, lds);
}

}  // namespace

hipError_t herk_bf16x3_wgroup_launch(bool lolo, int variant, const HerkArgs& a, int nwg,
                                     hipStream_t s) {
  // variant 0: compiler scheduling; 1: issue-order hints; 2: hints and
  // atomic flushes; 3: as 2, leaving out the blocks above the diagonal; 4:
  // as 3, partial tiles as real and imaginary planes; 5: as 4, Z loaded in
  // 16-byte chunks (only when every npb is even, so that Z rows are 16-byte
  // aligned; else 4)
  if (variant == 5 && !a.z16) variant = 4;
#define CHI0_WG_LAUNCH(L, H, A, K, P, Q) \
  hipLaunchKernelGGL((herk_bf16x3_wgroup_kernel<L, H, A, K, P, Q>), dim3(nwg), dim3(kNT), 0, s, a)
  if (lolo) {
    if (variant == 0) CHI0_WG_LAUNCH(true, false, false, false, false, false);
    else if (variant == 1) CHI0_WG_LAUNCH(true, true, false, false, false, false);
    else if (variant == 2) CHI0_WG_LAUNCH(true, true, true, false, false, false);
    else if (variant == 3) CHI0_WG_LAUNCH(true, true, true, true, false, false);
    else if (variant == 4) CHI0_WG_LAUNCH(true, true, true, true, true, false);
    else CHI0_WG_LAUNCH(true, true, true, true, true, true);
  } else {
    if (variant == 0) CHI0_WG_LAUNCH(false, false, false, false, false, false);
    else if (variant == 1) CHI0_WG_LAUNCH(false, true, false, false, false, false);
    else if (variant == 2) CHI0_WG_LAUNCH(false, true, true, false, false, false);
    else if (variant == 3) CHI0_WG_LAUNCH(false, true, true, true, false, false);
    else if (variant == 4) CHI0_WG_LAUNCH(false, true, true, true, true, false);
    else CHI0_WG_LAUNCH(false, true, true, true, true, true);
  }
#undef CHI0_WG_LAUNCH
  return hipGetLastError();
}

hipError_t herk_fp32_wgroup_launch(const HerkArgs& a, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(herk_fp32_wgroup_kernel, dim3(nwg), dim3(kNT), 0, s, a);
  return hipGetLastError();
}

int herk_fp32_wgroup_max_wg_per_cu() {
  int n = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, herk_fp32_wgroup_kernel, kNT, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}

int herk_bf16x3_wgroup_max_wg_per_cu() {
  int n = 0;
  const hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, herk_bf16x3_wgroup_kernel<false, true, true, false, false, false>, kNT, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}

}  // namespace chi0
