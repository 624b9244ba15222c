// BF16x3 building blocks shared by the tall-tile kernels (the chi0 rank-K
// update and the first contraction of the correlation self-energy): bf16
// packing and the hi / lo split, the 16-bit rotation that turns a packed
// (re, im) into (im, -re), the swizzled LDS layout of 256 x 128 complex tiles
// with 16 contraction rows per stage, and the MFMA core of one stage.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chi0 {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int kKC = 16;   // pairs per stage

constexpr int kNT = 256;  // threads

// LDS row = tile column (0..T-1), 16 dwords = 4 chunks of 4 pairs; chunk q of
// row r lives at slot q ^ g(r), g(r) = (r1 ^ r3) + 2 r2 (r_i = bit i of r).
// A 16-byte access of consecutive rows (same q) then hits distinct banks
// within every 8 lanes for 32 banks (8 rows span 128 bytes) and within every
// 16 lanes for 64 banks, so the fragment reads and the staging writes are
// conflict-free with either bank count.
__device__ __forceinline__ int swz(int row, int q) {
  const int g = (((row >> 1) ^ (row >> 3)) & 1) | (((row >> 2) & 1) << 1);
  return row * 16 + 4 * (q ^ g);
}

__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  bf16x2 v;
  v[0] = static_cast<__bf16>(lo);
  v[1] = static_cast<__bf16>(hi);
  return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ float bf16_lo_to_f32(uint32_t p) { return __uint_as_float(p << 16); }
__device__ __forceinline__ float bf16_hi_to_f32(uint32_t p) { return __uint_as_float(p & 0xFFFF0000u); }

// (x_re, x_im) -> packed hi and lo bf16x2 words (re in the low half).
__device__ __forceinline__ void split2(float re, float im, uint32_t& hi, uint32_t& lo) {
  // no contraction: re, im are the FP32-rounded operands (for the scaled
  // side, the rounded product), and x - hi is exact in FP32
#pragma clang fp contract(off)
  hi = pack_bf16x2(re, im);
  // the packed word itself is unpacked: left visible, the compiler re-packs
  // re alone for its low half (one more conversion per value)
  asm("" : "+v"(hi));
  lo = pack_bf16x2(re - bf16_lo_to_f32(hi), im - bf16_hi_to_f32(hi));
}

// (br, bi) packed -> (bi, -br) packed.
__device__ __forceinline__ uint32_t rot_neg(uint32_t x) {
  return __builtin_amdgcn_alignbit(x, x, 16) ^ 0x80000000u;
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ uint4 rot_neg4(uint4 v) {
  return uint4{rot_neg(v.x), rot_neg(v.y), rot_neg(v.z), rot_neg(v.w)};
}

// LDS of the tall-tile kernels: double-buffered bf16 hi / lo planes of a
// 256-row P side and a 128-row Q side, the Q side also rotated to (im, -re).
struct Bf16TallLds {
  uint32_t ah[2][256 * 16];
  uint32_t al[2][256 * 16];
  uint32_t bh[2][128 * 16];
  uint32_t bl[2][128 * 16];
  uint32_t bih[2][128 * 16];
  uint32_t bil[2][128 * 16];
};

__device__ __forceinline__ void tall_stage_p(Bf16TallLds& L, int buf, int lp, const uint4 (&ph)[4],
                                             const uint4 (&pl)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int o = swz(lp, q);
    *reinterpret_cast<uint4*>(&L.ah[buf][o]) = ph[q];
    *reinterpret_cast<uint4*>(&L.al[buf][o]) = pl[q];
  }
}

// The 2 k-steps of one stage for a wave's (32 NBI) x 64 sub-tile at P rows
// 32 NBI wr and Q columns 64 wc.
template <bool LOLO, int NBI = 4>
__device__ __forceinline__ void tall_mfma(const Bf16TallLds& L, int buf, int wr, int wc, int g8,
                                          int l32, f32x16 (&cr)[NBI][2], f32x16 (&ci)[NBI][2]) {
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    const int q = 2 * ks + g8;
    bf16x8 fah[NBI], fal[NBI], fbh[2], fbl[2], fih[2], fil[2];
#pragma unroll
    for (int i = 0; i < NBI; ++i) {
      const int row = wr * (32 * NBI) + i * 32 + l32;
      fah[i] = as_bf16x8(*reinterpret_cast<const uint4*>(&L.ah[buf][swz(row, q)]));
      fal[i] = as_bf16x8(*reinterpret_cast<const uint4*>(&L.al[buf][swz(row, q)]));
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int row = wc * 64 + j * 32 + l32;
      fbh[j] = as_bf16x8(*reinterpret_cast<const uint4*>(&L.bh[buf][swz(row, q)]));
      fbl[j] = as_bf16x8(*reinterpret_cast<const uint4*>(&L.bl[buf][swz(row, q)]));
      fih[j] = as_bf16x8(*reinterpret_cast<const uint4*>(&L.bih[buf][swz(row, q)]));
      fil[j] = as_bf16x8(*reinterpret_cast<const uint4*>(&L.bil[buf][swz(row, q)]));
    }
#pragma unroll
    for (int i = 0; i < NBI; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[i], fbh[j], cr[i][j], 0, 0, 0);
        ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[i], fih[j], ci[i][j], 0, 0, 0);
      }
#pragma unroll
    for (int i = 0; i < NBI; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[i], fbl[j], cr[i][j], 0, 0, 0);
        ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[i], fil[j], ci[i][j], 0, 0, 0);
      }
#pragma unroll
    for (int i = 0; i < NBI; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fal[i], fbh[j], cr[i][j], 0, 0, 0);
        ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fal[i], fih[j], ci[i][j], 0, 0, 0);
      }
    if (LOLO) {
#pragma unroll
      for (int i = 0; i < NBI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fal[i], fbl[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fal[i], fil[j], ci[i][j], 0, 0, 0);
        }
    }
  }
}

// Add (or store, when first) a wave's (32 NBI) x 64 accumulators into the
// FP64 partial tile (TQ columns, row-major: 256 x 128 for a workgroup's tile,
// 128 x 64 for a wave's own); 16 old values are loaded as a group.  With
// ATOM the additions are FP64 atomic adds without return, done in L2: the
// wave issues them all and waits for none (a slot belongs to one wave, whose
// accesses to one address stay in order, so the sums are those of the
// load-add-store form, in the same order).
// 32 x 32 block (i, j) of a 128 x 64 tile that crosses the diagonal:
// DIAG 1 for tile column 2 tp (left half of the diagonal 128 x 128 square),
// DIAG 2 for tile column 2 tp + 1 (its right half), 0 for any other tile.
// A block is needed iff it holds an entry on or below the diagonal (rows
// 32 i .. 32 i + 31, columns 32 j .. 32 j + 31, plus 64 for DIAG 2).
template <int DIAG>
__host__ __device__ constexpr bool diag_block_needed(int i, int j) {
  return DIAG == 0 ? true : DIAG == 1 ? (i >= j) : (i >= j + 2);
}

template <int NBI = 4, int TQ = 128, bool ATOM = false, int DIAG = 0>
__device__ __forceinline__ void tall_flush(double2* __restrict__ part, const f32x16 (&cr)[NBI][2],
                                           const f32x16 (&ci)[NBI][2], int wr, int wc, int lane,
                                           bool first) {
  const int g = lane >> 5;
  const int cl = lane & 31;
  int base = (wr * (32 * NBI) + 4 * g) * TQ + wc * 64 + cl;
  asm volatile("" : "+v"(base));
#pragma unroll
  for (int i = 0; i < NBI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (!diag_block_needed<DIAG>(i, j)) continue;   // never read by the reduction
      double2* blk = part + base + i * 32 * TQ + j * 32;
      if (ATOM && !first) {
        typedef double __attribute__((address_space(1)))* gdp;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          double* d = reinterpret_cast<double*>(blk + (8 * (r >> 2) + (r & 3)) * TQ);
          __builtin_amdgcn_global_atomic_fadd_f64((gdp)d, static_cast<double>(cr[i][j][r]));
          __builtin_amdgcn_global_atomic_fadd_f64((gdp)(d + 1), static_cast<double>(ci[i][j][r]));
        }
        continue;
      }
      double2 o[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) o[r] = double2{0.0, 0.0};
      if (!first) {
#pragma unroll
        for (int r = 0; r < 16; ++r) o[r] = blk[(8 * (r >> 2) + (r & 3)) * TQ];
      }
#pragma unroll
      for (int r = 0; r < 16; ++r)
        blk[(8 * (r >> 2) + (r & 3)) * TQ] =
            double2{static_cast<double>(cr[i][j][r]) + o[r].x,
                    static_cast<double>(ci[i][j][r]) + o[r].y};
    }
}

}  // namespace
}  // namespace chi0
