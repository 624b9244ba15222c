// BF16x3 weighted Hermitian rank-K update with register-direct operands.
//
// Same contraction as the tall-tile kernels (S[P][Q] = sum_pairs
// conj(Z[pair][P]) * (c * Z[pair][Q]) over one 256 x 128 lower tile per unit,
// chi0 = -S, Eq.(polfx) at i*omega), but every wave loads its own operands
// from global memory straight into registers: no LDS, no barriers.  The four
// waves of a workgroup take the 128 x 64 sub-tiles of the unit's tile; the two
// waves that share P rows (or Q columns) read the same lines, which the
// compute unit's L1 serves once.
//
// Per k-step (8 pairs, one 32x32x16 MFMA contraction depth) a lane loads
//   P: the pre-split hi / lo words of 4 pairs of one tile row per 32-row
//      block (16 bytes each, the MFMA A-operand layout as stored, so 32 lanes
//      read 512 contiguous bytes);
//   Q: the complex64 Z values of 4 pairs of one tile column per 32-column
//      block, and the 4 pair weights (same address in 32 lanes);
// and turns the Q side into bf16 hi / lo words of c Z, plain and rotated to
// (im, -re) (the rotation comes from converting (im, -re) directly).
// The P words are loaded two k-steps ahead of their MFMAs and the raw Q
// operands about one and a half (each column block's conversion runs while
// the MFMAs of the other column block issue), so the loads have 48 to 96
// MFMAs to land.  Pair rows are clamped into the segment and
// pairs past its end get weight 0, so the last k-steps of a segment need no
// separate code.
//
// Units and partial slots are those of the tall-tile kernels (the same
// planner tile configuration): a wave whose sub-tile lies entirely above the
// diagonal or outside the matrix skips the unit, since the reduction never
// reads those entries.
#include "bf16_tall.h"
#include "common.h"
#include "herk_common.h"

namespace chi0 {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef const char __attribute__((address_space(1)))* gcptr;

// Raw buffer resource over [base, base + bytes): loads at offsets past the
// end return 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(gcptr base, int32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, 0, bytes > 0 ? bytes : 0, 0x00020000);
}

// Byte counts of a run, capped at 2^31 - 1 (far beyond the offsets a run
// reads).
__device__ __forceinline__ int32_t cap32(int64_t bytes) {
  return bytes >= INT32_MAX ? INT32_MAX : static_cast<int32_t>(bytes);
}

// Registers of one k-step: the P words and the raw Q operands.
struct PStep {
  u32x4 ph[4], pl[4];  // hi / lo words of row blocks 0..3
};
struct QRaw {
  u32x2 q[2][4];       // complex64 of column blocks 0..1, pairs 4 g + e
  float w[4];          // pair weights of pairs 4 g + e
};
// c Z split into bf16 hi / lo words, plain (re, im) and rotated (im, -re),
// per column block.
struct QWords {
  u32x4 h[2], l[2], rh[2], rl[2];
};

// One run of k-steps within a block: base addresses at the run's first
// pair and the bytes from there to the end of what may be read.  Past the
// end of the run's pairs, Z and the weights read as 0, so those pairs add
// nothing; past the block's pre-split planes, P reads as 0.
struct DirectRun {
  gcptr hi, lo;        // P hi / lo planes at the run's first 4-pair group
  int32_t pbytes;      // plane bytes from there to the block's padded end
  int32_t chunk;       // bytes per 4-pair group of a plane (npb * 16)
  gcptr z;             // Z row of the run's first pair
  int32_t zbytes;      // Z bytes of the run's pairs
  int32_t row;         // bytes per Z row (npb * 8)
  gcptr w;             // weight of the run's first pair at this frequency
  int32_t wbytes;      // weight bytes of the run's pairs
};

// Lane offsets (bytes): P tile rows of the 4 row blocks (with the lane's
// 4-pair group), Q tile columns of the 2 column blocks with the lane's first
// pair row.
struct DirectLane {
  uint32_t p[4];
  uint32_t q[2];
  uint32_t w;
};

__device__ __forceinline__ void load_p(const DirectRun& r, int k, const DirectLane& o, PStep& d) {
  const int32_t off = 2 * k * r.chunk;
  const __amdgpu_buffer_rsrc_t h = rsrc(r.hi + off, r.pbytes - off);
  const __amdgpu_buffer_rsrc_t l = rsrc(r.lo + off, r.pbytes - off);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    d.ph[i] = __builtin_amdgcn_raw_buffer_load_b128(h, o.p[i], 0, 0);
    d.pl[i] = __builtin_amdgcn_raw_buffer_load_b128(l, o.p[i], 0, 0);
  }
}

__device__ __forceinline__ void load_q(const DirectRun& r, int k, const DirectLane& o, QRaw& d) {
  const int32_t zo = 8 * k * r.row;
  const int32_t wo = 32 * k;
  const __amdgpu_buffer_rsrc_t z = rsrc(r.z + zo, r.zbytes - zo);
  const __amdgpu_buffer_rsrc_t w = rsrc(r.w + wo, r.wbytes - wo);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
#pragma unroll
    for (int j = 0; j < 2; ++j)
      d.q[j][e] = __builtin_amdgcn_raw_buffer_load_b64(z, o.q[j] + e * r.row, 0, 0);
    d.w[e] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(w, o.w + 4 * e, 0, 0));
  }
}

// bf16 (im, -re), round to nearest even (the negation is a source modifier).
__device__ __forceinline__ uint32_t pack_rot(float re, float im) {
  uint32_t r;
  asm("v_cvt_pk_bf16_f32 %0, %1, -%2" : "=v"(r) : "v"(im), "v"(re));
  return r;
}

// Column block j of a k-step's raw Q into the Q words.
__device__ __forceinline__ void convert_q(const QRaw& d, int j, QWords& o) {
#pragma clang fp contract(off)
  uint32_t h[4], l[4], rh[4], rl[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const float x = __uint_as_float(d.q[j][e].x) * d.w[e];
    const float y = __uint_as_float(d.q[j][e].y) * d.w[e];
    h[e] = pack_bf16x2(x, y);
    const float x1 = x - __uint_as_float(__builtin_amdgcn_alignbit(h[e], 0u, 16));
    const float y1 = y - bf16_hi_to_f32(h[e]);
    l[e] = pack_bf16x2(x1, y1);
    rh[e] = pack_rot(x, y);
    rl[e] = pack_rot(x1, y1);
  }
  o.h[j] = u32x4{h[0], h[1], h[2], h[3]};
  o.l[j] = u32x4{l[0], l[1], l[2], l[3]};
  o.rh[j] = u32x4{rh[0], rh[1], rh[2], rh[3]};
  o.rl[j] = u32x4{rl[0], rl[1], rl[2], rl[3]};
}

__device__ __forceinline__ bf16x8 frag(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// The MFMAs of one k-step for column block j (4 row blocks x (re, im) x the
// split terms); an accumulator's updates are 8 MFMAs apart.
template <bool LOLO>
__device__ __forceinline__ void direct_mfma(const PStep& p, const QWords& q, int j,
                                            f32x16 (&cr)[4][2], f32x16 (&ci)[4][2]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag(p.ph[i]), frag(q.h[j]), cr[i][j], 0, 0, 0);
    ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag(p.ph[i]), frag(q.rh[j]), ci[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag(p.ph[i]), frag(q.l[j]), cr[i][j], 0, 0, 0);
    ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag(p.ph[i]), frag(q.rl[j]), ci[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag(p.pl[i]), frag(q.h[j]), cr[i][j], 0, 0, 0);
    ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag(p.pl[i]), frag(q.rh[j]), ci[i][j], 0, 0, 0);
  }
  if (LOLO) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag(p.pl[i]), frag(q.l[j]), cr[i][j], 0, 0, 0);
      ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag(p.pl[i]), frag(q.rl[j]), ci[i][j], 0, 0, 0);
    }
  }
}

// Issue order of one k-step: the column-block-0 MFMAs with the P loads and
// the column-block-1 conversion between them (two VALU per MFMA), then the
// column-block-1 MFMAs with the Q loads and the next k-step's column-block-0
// conversion.
__device__ __forceinline__ void step_order() {
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
    __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // VMEM read
    __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);   // VALU
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
  }
#pragma unroll
  for (int m = 0; m < 12; ++m) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
  }
}

__device__ __forceinline__ void zero8(f32x16 (&cr)[4][2], f32x16 (&ci)[4][2]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cr[i][j] = f32x16{0};
      ci[i][j] = f32x16{0};
    }
}

// WAVE_UNITS = false: the workgroup takes 256 x 128 units, wave (wr, wc)
// their 128 x 64 sub-tile.  WAVE_UNITS = true: every wave has its own work
// list of 128 x 64 units (the planner deals a tile's frequencies to the
// waves of one workgroup, so the four waves read the same rows of Z and the
// L1 serves them once), and diagonal tiles cost no idle waves.
template <bool LOLO, bool HINT, bool WAVE_UNITS>
__global__ __launch_bounds__(kNT, 1) void herk_bf16x3_direct_kernel(HerkArgs a) {
  constexpr int TP = WAVE_UNITS ? 128 : 256, TQ = WAVE_UNITS ? 64 : 128;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = WAVE_UNITS ? 0 : wave >> 1, wc = WAVE_UNITS ? 0 : wave & 1;
  const int g8 = lane >> 5;
  const int l32 = lane & 31;

  // work list, units and problem descriptors through the scalar cache (they
  // are uniform: every branch on them stays a scalar branch)
  const int list = WAVE_UNITS ? static_cast<int>(blockIdx.x) * (kNT / 64) + wave
                              : static_cast<int>(blockIdx.x);
  const int beg = ld_const(a.wg_offsets, list);
  const int end = ld_const(a.wg_offsets, list + 1);
  for (int ui = beg; ui < end; ++ui) {
    // The four waves of a workgroup-wide unit start it together: a wave
    // that skips its sub-tile must not run ahead into later units, or the
    // workgroups of an XCD stop streaming the same rows of Z at the same
    // time and its L2 no longer serves them (measured: L2 hit rate 36%
    // without this, HBM traffic ten times that of the LDS-staged kernel).
    if (!WAVE_UNITS) __syncthreads();
    const Unit u = ld_unit(a.units, ld_const(a.wg_units, ui));
    const ProbDesc pd = ld_prob(a.probs, u.prob);
    const int npb = pd.npb;
    const int r0 = u.tp * TP + wr * 128;
    const int c0 = u.tq * TQ + wc * 64;
    if (!WAVE_UNITS && (r0 >= npb || c0 >= npb || r0 + 127 < c0)) continue;   // nothing read
    const uint32_t chunk = static_cast<uint32_t>(npb) * 16u;
    const uint32_t row = static_cast<uint32_t>(npb) * 8u;
    DirectLane lo;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int col = r0 + 32 * i + l32;
      lo.p[i] = static_cast<uint32_t>(g8) * chunk + static_cast<uint32_t>(col < npb ? col : 0) * 16u;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = c0 + 32 * j + l32;
      lo.q[j] = static_cast<uint32_t>(4 * g8) * row + static_cast<uint32_t>(col < npb ? col : 0) * 8u;
    }
    lo.w = static_cast<uint32_t>(16 * g8);
    // FP32 runs of at most the problem's flush length (a multiple of 16
    // pairs), in k-steps; a multiple of the 6-step loop body when possible
    const int fsteps = pd.flush >= 16 ? pd.flush / 8 : 2;
    const int frun = fsteps >= 6 ? fsteps / 6 * 6 : fsteps;
    double2* part = a.partials + static_cast<size_t>(u.slot) * TP * TQ;
    const float* wts = static_cast<const float*>(pd.wts) + static_cast<size_t>(u.iw) * pd.ktot;

    f32x16 cr[4][2], ci[4][2];
    zero8(cr, ci);
    bool first = true;
    int steps = 0;   // k-steps in the FP32 accumulators
    for (int b = u.b0; b <= u.b1; ++b) {
      const BlockDesc* bp = a.blocks + b;
      const int kb = block_pairs(a.blocks, b);
      const int p0 = (b == u.b0) ? u.p0 : 0;
      const int p1 = (b == u.b1) ? u.p1 : kb;
      if (p0 >= p1) continue;
      const int n = p1 - p0;
      const int nk = (n + 7) >> 3;
      const gcptr zs = (gcptr)ld_const(&bp->zs, 0);
      const int64_t plane = ld_const(&bp->zs_plane, 0);
      const gcptr z = (gcptr)ld_const(&bp->z, 0);
      const float* wb = wts + ld_const(&bp->pair_base, 0);
      const int64_t groups = presplit_groups(kb);

      // Runs of k-steps, each a software pipeline of its own (the loads in
      // flight at its end are dropped), so that the FP64 flush between runs
      // holds no pipeline registers.  Register sets: P[k % 3] holds the P
      // words of k-step k, R[k % 2] the raw Q of k-step k; W holds converted
      // Q words, column block 0 one k-step ahead of column block 1.  K-step
      // k: the P loads of k-step k + 2; column block 1 of k-step k converted
      // while the column-block-0 MFMAs issue; the raw Q of k-step k + 2
      // loaded into the freed set; column block 0 of k-step k + 1 converted
      // while the column-block-1 MFMAs issue.  K-steps past the run's end
      // (at most 5) read zeros.
      for (int t0 = 0; t0 < nk;) {
        const int len = min(frun - steps, nk - t0);
        const int q0 = p0 + 8 * t0;                 // the run's first pair
        const int nv = min(p1, q0 + 8 * len) - q0;  // its pairs
        DirectRun r;
        r.chunk = static_cast<int32_t>(chunk);
        r.row = static_cast<int32_t>(row);
        r.hi = zs + static_cast<int64_t>(q0 >> 2) * chunk;
        r.lo = r.hi + plane;
        r.pbytes = cap32((groups - (q0 >> 2)) * static_cast<int64_t>(chunk));
        r.z = z + static_cast<int64_t>(q0) * row;
        r.zbytes = cap32(static_cast<int64_t>(nv) * row);
        r.w = (gcptr)(wb + q0);
        r.wbytes = nv * 4;
        PStep P[3];
        QRaw R[2];
        QWords W;
        // the prologue issues its loads in pipeline order, so that the
        // loop's waits on them are the steady-state ones
        load_p(r, 0, lo, P[0]);
        __builtin_amdgcn_sched_barrier(0);
        load_q(r, 0, lo, R[0]);
        __builtin_amdgcn_sched_barrier(0);
        load_p(r, 1, lo, P[1]);
        __builtin_amdgcn_sched_barrier(0);
        load_q(r, 1, lo, R[1]);
        __builtin_amdgcn_sched_barrier(0);
        convert_q(R[0], 0, W);
        for (int t = 0; t < len; t += 6) {
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            load_p(r, t + k + 2, lo, P[(k + 2) % 3]);
            convert_q(R[k % 2], 1, W);
            direct_mfma<LOLO>(P[k % 3], W, 0, cr, ci);
            load_q(r, t + k + 2, lo, R[k % 2]);
            convert_q(R[(k + 1) % 2], 0, W);
            direct_mfma<LOLO>(P[k % 3], W, 1, cr, ci);
            if (HINT) step_order();
          }
        }
        t0 += len;
        steps += len;
        if (steps >= frun) {
          tall_flush<4, TQ>(part, cr, ci, wr, wc, lane, first);
          first = false;
          steps = 0;
          zero8(cr, ci);
        }
      }
    }
    if (first || steps > 0) tall_flush<4, TQ>(part, cr, ci, wr, wc, lane, first);
  }
}

}  // namespace

template <bool WU>
static void direct_launch(bool lolo, bool hint, const HerkArgs& a, int nwg, hipStream_t s) {
  if (lolo) {
    if (hint) hipLaunchKernelGGL((herk_bf16x3_direct_kernel<true, true, WU>), dim3(nwg), dim3(kNT), 0, s, a);
    else hipLaunchKernelGGL((herk_bf16x3_direct_kernel<true, false, WU>), dim3(nwg), dim3(kNT), 0, s, a);
  } else {
    if (hint) hipLaunchKernelGGL((herk_bf16x3_direct_kernel<false, true, WU>), dim3(nwg), dim3(kNT), 0, s, a);
    else hipLaunchKernelGGL((herk_bf16x3_direct_kernel<false, false, WU>), dim3(nwg), dim3(kNT), 0, s, a);
  }
}

hipError_t herk_bf16x3_direct_launch(bool lolo, bool hint, bool wave_units, const HerkArgs& a,
                                     int nwg, hipStream_t s) {
  if (wave_units) direct_launch<true>(lolo, hint, a, nwg, s);
  else direct_launch<false>(lolo, hint, a, nwg, s);
  return hipGetLastError();
}

int herk_bf16x3_direct_max_wg_per_cu() {
  int n = 0;
  const hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, herk_bf16x3_direct_kernel<false, false, true>, kNT, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}

}  // namespace chi0
