// Correlation self-energy on the BF16x3 path: both contractions of
// Eq.(sigci) on the tall-tile MFMA core (bf16_tall.h).
#include "bf16_tall.h"
#include "common.h"

namespace chi0 {
namespace {

// ---------------------------------------------------------------------------
// Correlation self-energy (Eq.(sigci)), first contraction on the BF16x3 path:
//   D[nu][r] = sum_i t_i(r) sum_mu conj(W_i[mu][nu]) Z[n'][mu][n],
// r = (n', n), t = -w_k w_i(eps_qn - eps_n').  Both operands arrive pre-split
// (sigc_split_w_kernel, sigc_split_z_kernel), the Z side already multiplied by
// t_i(r) for every mesh point, so staging is a copy (plus the 16-bit rotation
// of the Z side for the imaginary part) and the rows (i, mu) form one
// contraction; tiles are 256 nu x 128 r with the tall kernels' LDS layout and
// MFMA core.  The FP32 accumulators are flushed into the FP64 output
// zw[n'][nu][n] every 4096 rows at most.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kNT, 1) void sigc_bf16x3_kernel(SigcArgs args) {
  typedef const char __attribute__((address_space(1)))* gcptr;
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  typedef const u32x4 __attribute__((address_space(1)))* gu4ptr;
  constexpr int TP = 256, TQ = 128, FL = 256;   // FL: stages between flushes at most
  __shared__ __attribute__((aligned(16))) Bf16TallLds L;

  const int per = (args.nunits + 7) / 8;
  const int lu = static_cast<int>(blockIdx.x % 8) * per + static_cast<int>(blockIdx.x / 8);
  if (lu >= args.nunits) return;
  const SigcUnit u = args.units[lu];
  const SigcDesc bd = args.descs[u.blk];
  const int nmu = bd.nmu, nqp = bd.nqp;
  const int64_t M = static_cast<int64_t>(bd.nall) * nqp;
  const int ns = bd.groups / 4;                  // 16-row stages per mesh point
  const int total = bd.nomega * ns;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int g8 = lane >> 5;
  const int l32 = lane & 31;
  const int lp = tid;
  const int lq = tid & (TQ - 1);
  const int lg = tid >> 7;

  const int pcol = u.tp * TP + lp;
  const int64_t qcol = static_cast<int64_t>(u.tc) * TQ + lq;
  const uint64_t offP = static_cast<uint64_t>(pcol < nmu ? pcol : 0) * 16u;
  const uint64_t offQ = static_cast<uint64_t>(qcol < M ? qcol : 0) * 16u;
  const uint64_t chunkP = static_cast<uint64_t>(nmu) * 16u;   // one group of W rows
  const uint64_t chunkQ = static_cast<uint64_t>(M) * 16u;     // one group of Z rows
  const gcptr wh = (gcptr)bd.wsp;
  const gcptr zh = (gcptr)bd.zsp;

  f32x16 cr[4][2], ci[4][2];
  auto zero = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        cr[i][j] = f32x16{0};
        ci[i][j] = f32x16{0};
      }
  };
  zero();
  uint4 ph[4], pl[4], qh[2], ql[2];

  auto load = [&](int st) __attribute__((always_inline)) {
    const int i = st / ns;
    const int g0 = 4 * (st - i * ns);
    const uint64_t gi = static_cast<uint64_t>(i) * bd.groups + g0;
    const gcptr wb = wh + gi * chunkP + offP;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const u32x4 h = *(gu4ptr)(wb + q * chunkP);
      const u32x4 l = *(gu4ptr)(wb + bd.wsp_plane + q * chunkP);
      ph[q] = uint4{h.x, h.y, h.z, h.w};
      pl[q] = uint4{l.x, l.y, l.z, l.w};
    }
    const gcptr zb = zh + gi * chunkQ + offQ;
#pragma unroll
    for (int gi2 = 0; gi2 < 2; ++gi2) {
      const uint64_t o = static_cast<uint64_t>(lg + 2 * gi2) * chunkQ;
      const u32x4 h = *(gu4ptr)(zb + o);
      const u32x4 l = *(gu4ptr)(zb + bd.zsp_plane + o);
      qh[gi2] = uint4{h.x, h.y, h.z, h.w};
      ql[gi2] = uint4{l.x, l.y, l.z, l.w};
    }
  };
  auto stage = [&](int buf) __attribute__((always_inline)) {
    tall_stage_p(L, buf, lp, ph, pl);
#pragma unroll
    for (int gi = 0; gi < 2; ++gi) {
      const int o = swz(lq, lg + 2 * gi);
      *reinterpret_cast<uint4*>(&L.bh[buf][o]) = qh[gi];
      *reinterpret_cast<uint4*>(&L.bl[buf][o]) = ql[gi];
      *reinterpret_cast<uint4*>(&L.bih[buf][o]) = rot_neg4(qh[gi]);
      *reinterpret_cast<uint4*>(&L.bil[buf][o]) = rot_neg4(ql[gi]);
    }
  };
  // Add the accumulators (columns r of this lane, all its rows nu) into zw in
  // FP64; plain stores for the unit's first flush.  A block of 32 rows that
  // lies inside nmu (the rule) takes no per-row test, so its 16 reads are in
  // flight together.
  auto flush = [&](bool first) {
    const int g = lane >> 5;
    const int64_t rstride = nqp;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t col = static_cast<int64_t>(u.tc) * TQ + wc * 64 + j * 32 + (lane & 31);
      if (col >= M) continue;
      const int64_t a2 = col / nqp;
      double2* dst = bd.zw + a2 * nmu * nqp + (col - a2 * nqp);
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) {
        const int rb = u.tp * TP + wr * 128 + bi * 32;   // wave-uniform
        double2* p0 = dst + static_cast<int64_t>(rb + 4 * g) * rstride;
        if (rb + 32 <= nmu) {
          double2 o[16];
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            o[r] = double2{0.0, 0.0};
            if (!first) o[r] = p0[(8 * (r >> 2) + (r & 3)) * rstride];
          }
#pragma unroll
          for (int r = 0; r < 16; ++r)
            p0[(8 * (r >> 2) + (r & 3)) * rstride] = double2{o[r].x + static_cast<double>(cr[bi][j][r]),
                                                             o[r].y + static_cast<double>(ci[bi][j][r])};
        } else {
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            if (rb + 4 * g + 8 * (r >> 2) + (r & 3) >= nmu) continue;
            double2* p = p0 + (8 * (r >> 2) + (r & 3)) * rstride;
            const double vr = static_cast<double>(cr[bi][j][r]);
            const double vi = static_cast<double>(ci[bi][j][r]);
            if (first) {
              *p = double2{vr, vi};
            } else {
              const double2 o = *p;
              *p = double2{o.x + vr, o.y + vi};
            }
          }
        }
        // one 32 x 32 block at a time: keeps the in-flight FP64 values few
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    zero();
  };

  load(0);
  stage(0);
  __syncthreads();
  int buf = 0, st = 0;
  bool first = true;
  // The weights are folded into Z, so the stages of all mesh points form one
  // sum, taken in FP32 runs of at most FL stages (4096 rows mu) that are added
  // into zw in FP64.
  while (st < total) {
    st = __builtin_amdgcn_readfirstlane(st);
    const int run_end = __builtin_amdgcn_readfirstlane(st + FL < total ? st + FL : total);
    for (; st < run_end; ++st) {
      const bool more = st + 1 < total;
      if (more) load(st + 1);
      tall_mfma<false, 4>(L, buf, wr, wc, g8, l32, cr, ci);
      if (more) stage(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
    flush(first);
    first = false;
  }
}

// ---------------------------------------------------------------------------
// Second contraction on the BF16x3 path:
//   I[n][m] = sum_kappa conj(zw[kappa][n]) Z[kappa][m],  kappa = (n', nu),
// both operands pre-split as [kappa][n] matrices (sigc_split_rows_kernel).
// A unit is one 256 (n) x 128 (m) tile over one segment of at most 4096 rows
// kappa: a single FP32 run, stored as an FP64 partial (rows 0-127 and
// 128-255 as two 128 x 128 partial tiles) and summed in a fixed order by the
// FP64 reduction.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kNT, 1) void sigc_bf16x3_zwz_kernel(SigcArgs args) {
  typedef const char __attribute__((address_space(1)))* gcptr;
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  typedef const u32x4 __attribute__((address_space(1)))* gu4ptr;
  constexpr int TP = 256, TQ = 128, T = 128;
  __shared__ __attribute__((aligned(16))) Bf16TallLds L;

  const int per = (args.nunits + 7) / 8;
  const int lu = static_cast<int>(blockIdx.x % 8) * per + static_cast<int>(blockIdx.x / 8);
  if (lu >= args.nunits) return;
  const SigcUnit u = args.units[lu];
  const SigcDesc bd = args.descs[u.blk];
  const int nqp = bd.nqp;
  const int total = bd.kgroups / 4;                 // 16-row stages
  const int sps = args.seg_len / 16;                // stages per segment
  const int s0 = u.seg * sps;
  const int s1 = s0 + sps < total ? s0 + sps : total;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int g8 = lane >> 5;
  const int l32 = lane & 31;
  const int lp = tid;
  const int lq = tid & (TQ - 1);
  const int lg = tid >> 7;

  const int pcol = u.tp * TP + lp;
  const int qcol = u.tc * TQ + lq;
  const uint64_t offP = static_cast<uint64_t>(pcol < nqp ? pcol : 0) * 16u;
  const uint64_t offQ = static_cast<uint64_t>(qcol < nqp ? qcol : 0) * 16u;
  const uint64_t chunk = static_cast<uint64_t>(nqp) * 16u;   // one group of 4 rows
  const gcptr ah = (gcptr)bd.zwsp;
  const gcptr bh = (gcptr)bd.zksp;
  const int64_t plane = bd.k_plane;

  f32x16 cr[4][2], ci[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cr[i][j] = f32x16{0};
      ci[i][j] = f32x16{0};
    }
  uint4 ph[4], pl[4], qh[2], ql[2];

  auto load = [&](int st) __attribute__((always_inline)) {
    const uint64_t g0 = 4 * static_cast<uint64_t>(st);
    const gcptr wb = ah + g0 * chunk + offP;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const u32x4 h = *(gu4ptr)(wb + q * chunk);
      const u32x4 l = *(gu4ptr)(wb + plane + q * chunk);
      ph[q] = uint4{h.x, h.y, h.z, h.w};
      pl[q] = uint4{l.x, l.y, l.z, l.w};
    }
    const gcptr zb = bh + g0 * chunk + offQ;
#pragma unroll
    for (int gi = 0; gi < 2; ++gi) {
      const uint64_t o = static_cast<uint64_t>(lg + 2 * gi) * chunk;
      const u32x4 h = *(gu4ptr)(zb + o);
      const u32x4 l = *(gu4ptr)(zb + plane + o);
      qh[gi] = uint4{h.x, h.y, h.z, h.w};
      ql[gi] = uint4{l.x, l.y, l.z, l.w};
    }
  };
  auto stage = [&](int buf) __attribute__((always_inline)) {
    tall_stage_p(L, buf, lp, ph, pl);
#pragma unroll
    for (int gi = 0; gi < 2; ++gi) {
      const int o = swz(lq, lg + 2 * gi);
      *reinterpret_cast<uint4*>(&L.bh[buf][o]) = qh[gi];
      *reinterpret_cast<uint4*>(&L.bl[buf][o]) = ql[gi];
      *reinterpret_cast<uint4*>(&L.bih[buf][o]) = rot_neg4(qh[gi]);
      *reinterpret_cast<uint4*>(&L.bil[buf][o]) = rot_neg4(ql[gi]);
    }
  };

  if (s0 < s1) {
    load(s0);
    stage(0);
  }
  __syncthreads();
  int buf = 0;
  for (int st = s0; st < s1; ++st) {
    const bool more = st + 1 < s1;
    if (more) load(st + 1);
    tall_mfma<false, 4>(L, buf, wr, wc, g8, l32, cr, ci);
    if (more) stage(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // 256 x 128 partial, row-major: rows 0-127 are partial tile 2 lu, rows
  // 128-255 partial tile 2 lu + 1 (tile rows beyond nqp are never read)
  double2* out = args.partials + static_cast<size_t>(lu) * 2 * T * T;
  const int g = lane >> 5;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int col = wc * 64 + j * 32 + (lane & 31);
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr * 128 + bi * 32 + 4 * g + 8 * (r >> 2) + (r & 3);
        out[row * T + col] = double2{static_cast<double>(cr[bi][j][r]), static_cast<double>(ci[bi][j][r])};
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

}  // namespace

hipError_t sigc_bf16x3_zwz_launch(const SigcArgs& a, hipStream_t s) {
  if (a.nunits <= 0) return hipSuccess;
  const unsigned grid = static_cast<unsigned>((a.nunits + 7) / 8 * 8);
  hipLaunchKernelGGL(sigc_bf16x3_zwz_kernel, dim3(grid), dim3(kNT), 0, s, a);
  return hipGetLastError();
}

hipError_t sigc_bf16x3_launch(const SigcArgs& a, hipStream_t s) {
  if (a.nunits <= 0) return hipSuccess;
  const unsigned grid = static_cast<unsigned>((a.nunits + 7) / 8 * 8);
  hipLaunchKernelGGL(sigc_bf16x3_kernel, dim3(grid), dim3(kNT), 0, s, a);
  return hipGetLastError();
}

}  // namespace chi0
