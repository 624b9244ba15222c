// FP64 weighted Hermitian rank-K update on gfx950 matrix cores.
//
// For one unit (problem, frequency, lower-triangle tile (tp, tq), block range)
// the kernel accumulates, in FP64,
//   S[P][Q] = sum_pairs c * conj(Z[pair][P]) * Z[pair][Q],
//   c = w_k * 2 D / (D^2 + omega^2) >= 0,
// over the tile's T x T complex entries; chi0 = -S (Eq.(polfx) at i*omega).
// The complex product is four real products stacked along the contraction
// index of v_mfma_f64_16x16x4f64: k-slots (re, im) of two pairs per MFMA,
//   Re S += [ar, ai] . [br, bi],   Im S += [ar, ai] . [bi, -br].
// The pair weight (precomputed per call, pair_weights_kernel) scales the
// Q-side operand as it is staged into LDS.
#include "common.h"
#include "herk_common.h"

namespace chi0 {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int T, int KC>
__global__ __launch_bounds__(256) void herk_fp64_kernel(HerkArgs a) {
  static_assert(T % 32 == 0 && KC % 2 == 0, "tile shape");
  constexpr int NT = 256;
  constexpr int WT = T / 2;        // wave sub-tile (2 x 2 waves)
  constexpr int NB = WT / 16;      // 16x16 MFMA blocks per wave side
  __shared__ double2 sA[KC][T];
  __shared__ double2 sB[KC][T];
  __shared__ double sW[KC];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int m = lane & 15;
  const int kk = lane >> 4;
  const int prr = kk >> 1;          // pair of the k-step held by this lane
  const bool isim = (kk & 1) != 0;  // real or imaginary k-slot

  const int beg = a.wg_offsets[blockIdx.x];
  const int end = a.wg_offsets[blockIdx.x + 1];
  for (int ui = beg; ui < end; ++ui) {
    const Unit u = a.units[a.wg_units[ui]];
    const ProbDesc pd = a.probs[u.prob];
    const int npb = pd.npb;
    const double* wts = static_cast<const double*>(pd.wts) + static_cast<size_t>(u.iw) * pd.ktot;
    const int colP0 = u.tp * T;
    const int colQ0 = u.tq * T;

    f64x4 accR[NB][NB], accI[NB][NB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        accR[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
        accI[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
      }

    for (int b = u.b0; b <= u.b1; ++b) {
      const BlockDesc bd = a.blocks[b];
      const int pbeg = (b == u.b0) ? u.p0 : 0;
      const int K = (b == u.b1) ? u.p1 : bd.nocc * bd.nunocc;  // end pair
      const double2* z = static_cast<const double2*>(bd.z);
      for (int p0 = pbeg; p0 < K; p0 += KC) {
        if (tid < KC) sW[tid] = p0 + tid < K ? wts[bd.pair_base + p0 + tid] : 0.0;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < KC * T / NT; ++i) {
          const int e = tid + i * NT;
          const int r = e / T;
          const int c = e % T;
          const int p = p0 + r;
          double2 va = {0.0, 0.0}, vb = {0.0, 0.0};
          if (p < K) {
            const size_t row = static_cast<size_t>(p) * npb;
            if (colP0 + c < npb) va = z[row + colP0 + c];
            if (colQ0 + c < npb) vb = z[row + colQ0 + c];
          }
          const double s = sW[r];
          vb.x *= s;
          vb.y *= s;
          sA[r][c] = va;
          sB[r][c] = vb;
        }
        __syncthreads();
#pragma unroll
        for (int st = 0; st < KC / 2; ++st) {
          const int pair = 2 * st + prr;
          double av[NB], br[NB], bi[NB];
#pragma unroll
          for (int i = 0; i < NB; ++i) {
            const double2 x = sA[pair][wr * WT + i * 16 + m];
            av[i] = isim ? x.y : x.x;
          }
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            const double2 y = sB[pair][wc * WT + j * 16 + m];
            br[j] = isim ? y.y : y.x;
            bi[j] = isim ? -y.x : y.y;
          }
#pragma unroll
          for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
              accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], br[j], accR[i][j], 0, 0, 0);
              accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bi[j], accI[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
      }
    }

    // Result layout of 16x16x4 f64: lane holds column (lane % 16) of rows
    // (lane / 16) + 4 r, r = 0..3.
    double2* out = a.partials + static_cast<size_t>(u.slot) * T * T;
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wr * WT + i * 16 + kk + 4 * r;
          const int col = wc * WT + j * 16 + m;
          out[row * T + col] = double2{accR[i][j][r], accI[i][j][r]};
        }
  }
}


// Pipelined variant: 128 x 128 complex tiles, 4 waves of 64 x 64 (one
// workgroup per CU, up to 512 registers per lane), 8 pairs per stage in
// double-buffered LDS, next stage's Z and (precomputed) weight loads issued
// unconditionally before the current stage's MFMAs, one barrier per stage.
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef const dvec2 __attribute__((address_space(1)))* gd2ptr;
typedef const double __attribute__((address_space(1)))* gdptr;

// Operand and weight loads of one stage for one thread: pairs p0 + poff[k]
// (the same for every lane of a wave, so rows, validity and weights are
// wave-uniform and live in scalar registers), tile column byte offsets offP /
// offQ (a column beyond npb reads column 0; its products are never used).
// Loads are issued unconditionally with the row clamped into the block; bit
// k of the returned mask says whether pair k exists (a missing pair gets
// weight 0).
template <int NP, bool GATHER>
__device__ __forceinline__ uint32_t load_pairs64(const HerkArgs& a, const ProbDesc& pd, int iw,
                                                 const Cursor& c, const int (&poff)[NP], int npb,
                                                 uint32_t offP, uint32_t offQ, double2 (&ra)[NP],
                                                 double2 (&rb)[NP], double (&rw)[NP]) {
  typedef const char __attribute__((address_space(1)))* gcptr;
  const int b = __builtin_amdgcn_readfirstlane(c.b);
  const int p0 = __builtin_amdgcn_readfirstlane(c.p0);
  const int last = __builtin_amdgcn_readfirstlane(c.pend) - 1 - p0;
  const BlockDesc* bp = a.blocks + b;
  const uint32_t row_bytes = static_cast<uint32_t>(npb) * 16u;
  const gcptr z = (gcptr)(ld_const(&bp->z, 0)) + static_cast<size_t>(p0) * row_bytes;
  const uint64_t* rows = GATHER ? ld_const(&bp->rows, 0) + p0 : nullptr;
  const int64_t pbase = ld_const(&bp->pair_base, 0);
  const double* w = static_cast<const double*>(pd.wts) + static_cast<size_t>(iw) * pd.ktot + pbase + p0;
  uint32_t mask = 0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int o = __builtin_amdgcn_readfirstlane(poff[k]);
    const bool valid = o <= last;
    const int oc = valid ? o : last;
    mask |= valid ? (1u << k) : 0u;
    const gcptr row = GATHER ? (gcptr)ld_const(rows, oc) : z + static_cast<uint32_t>(oc) * row_bytes;
    const dvec2 va = *(gd2ptr)(row + offP);
    const dvec2 vb = *(gd2ptr)(row + offQ);
    ra[k] = double2{va.x, va.y};
    rb[k] = double2{vb.x, vb.y};
    rw[k] = ld_const(w, oc);
  }
  return mask;
}

// NW = 4: 2 x 2 waves of 64 x 64 (one wave per SIMD, 256 accumulator
// registers); NW = 8: 2 x 4 waves of 64 x 32 (two waves per SIMD, so one
// wave's MFMAs can issue while the other waits).
template <int NW, bool GATHER>
__global__ __launch_bounds__(64 * NW, 1) void herk_fp64_pipe_kernel(HerkArgs a) {
  constexpr int T = 128, KC = 8, NT = 64 * NW;
  constexpr int WC = NW / 2;          // wave columns
  constexpr int NBI = 4;              // 16x16 blocks per wave: 64 rows
  constexpr int NBJ = T / WC / 16;    // and T / WC columns
  constexpr int LG = NT / T;          // loader pair groups
  constexpr int NP = KC / LG;         // pairs per thread per stage
  __shared__ double2 sA[2][KC][T];
  __shared__ double2 sB[2][KC][T];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int m = lane & 15;
  const int kk = lane >> 4;
  const int prr = kk >> 1;
  const bool isim = (kk & 1) != 0;
  const int lc = tid & (T - 1);   // loader: tile column
  const int lg = tid / T;         // loader: pairs lg, lg + LG, ... (wave-uniform)
  int poff[NP];
#pragma unroll
  for (int e = 0; e < NP; ++e) poff[e] = lg + LG * e;

  const int beg = a.wg_offsets[blockIdx.x];
  const int end = a.wg_offsets[blockIdx.x + 1];
  for (int ui = beg; ui < end; ++ui) {
    const Unit u = a.units[a.wg_units[ui]];
    const ProbDesc pd = a.probs[u.prob];
    const int npb = pd.npb;
    const uint32_t cP = static_cast<uint32_t>(u.tp * T + lc < npb ? u.tp * T + lc : 0) * 16u;
    const uint32_t cQ = static_cast<uint32_t>(u.tq * T + lc < npb ? u.tq * T + lc : 0) * 16u;

    f64x4 accR[NBI][NBJ], accI[NBI][NBJ];
#pragma unroll
    for (int i = 0; i < NBI; ++i)
#pragma unroll
      for (int j = 0; j < NBJ; ++j) {
        accR[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
        accI[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
      }
    double2 ra[NP], rb[NP];
    double rw[NP];
    uint32_t mk = 0;
    Cursor cur;
    bool have = cursor_first(u, a.blocks, cur);
    __syncthreads();
    if (have) mk = load_pairs64<NP, GATHER>(a, pd, u.iw, cur, poff, npb, cP, cQ, ra, rb, rw);
    int buf = 0;
    while (have) {
#pragma unroll
      for (int e = 0; e < NP; ++e) {
        const int r = lg + LG * e;
        const double w = ((mk >> e) & 1u) ? rw[e] : 0.0;
        sA[buf][r][lc] = ra[e];
        sB[buf][r][lc] = double2{rb[e].x * w, rb[e].y * w};
      }
      Cursor nxt = cur;
      const bool more = cursor_next<KC>(u, a.blocks, nxt);
      mk = load_pairs64<NP, GATHER>(a, pd, u.iw, nxt, poff, npb, cP, cQ, ra, rb, rw);
      __syncthreads();
#pragma unroll
      for (int st = 0; st < KC / 2; ++st) {
        const int pair = 2 * st + prr;
        double av[NBI], br[NBJ], bi[NBJ];
#pragma unroll
        for (int i = 0; i < NBI; ++i) {
          const double2 x = sA[buf][pair][wr * 64 + i * 16 + m];
          av[i] = isim ? x.y : x.x;
        }
#pragma unroll
        for (int j = 0; j < NBJ; ++j) {
          const double2 y = sB[buf][pair][wc * (T / WC) + j * 16 + m];
          br[j] = isim ? y.y : y.x;
          bi[j] = isim ? -y.x : y.y;
        }
#pragma unroll
        for (int i = 0; i < NBI; ++i)
#pragma unroll
          for (int j = 0; j < NBJ; ++j) {
            accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], br[j], accR[i][j], 0, 0, 0);
            accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bi[j], accI[i][j], 0, 0, 0);
          }
      }
      cur = nxt;
      have = more;
      buf ^= 1;
    }
    double2* out = a.partials + static_cast<size_t>(u.slot) * T * T;
#pragma unroll
    for (int i = 0; i < NBI; ++i)
#pragma unroll
      for (int j = 0; j < NBJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wr * 64 + i * 16 + kk + 4 * r;
          const int col = wc * (T / WC) + j * 16 + m;
          out[row * T + col] = double2{accR[i][j][r], accI[i][j][r]};
        }
  }
}

}  // namespace

// Tile table of the FP64 path.
static const TileConfig kFp64Tiles[] = {
    {128, 8, 0, 256, 128},   // 0: pipelined, 4 waves of 64 x 64
    {64, 16, 0, 256, 64},    // 1
    {32, 16, 0, 256, 32},    // 2
    {128, 8, 0, 512, 128},   // 3: pipelined, 8 waves of 64 x 32 (two per SIMD)
};

int herk_fp64_tile_count() { return sizeof(kFp64Tiles) / sizeof(kFp64Tiles[0]); }
TileConfig herk_fp64_tile(int idx) { return kFp64Tiles[idx]; }

hipError_t herk_fp64_launch(int idx, const HerkArgs& a, int nwg, hipStream_t s, bool gather) {
  switch (idx) {
    case 0:
      if (gather)
        hipLaunchKernelGGL((herk_fp64_pipe_kernel<4, true>), dim3(nwg), dim3(256), 0, s, a);
      else
        hipLaunchKernelGGL((herk_fp64_pipe_kernel<4, false>), dim3(nwg), dim3(256), 0, s, a);
      break;
    case 3:
      if (gather)
        hipLaunchKernelGGL((herk_fp64_pipe_kernel<8, true>), dim3(nwg), dim3(512), 0, s, a);
      else
        hipLaunchKernelGGL((herk_fp64_pipe_kernel<8, false>), dim3(nwg), dim3(512), 0, s, a);
      break;
    case 1:
      hipLaunchKernelGGL((herk_fp64_kernel<64, 16>), dim3(nwg), dim3(256), 0, s, a);
      break;
    case 2:
      hipLaunchKernelGGL((herk_fp64_kernel<32, 16>), dim3(nwg), dim3(256), 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int herk_fp64_max_wg_per_cu(int idx) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  if (idx == 0)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, herk_fp64_pipe_kernel<4, false>, 256, 0);
  else if (idx == 3)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, herk_fp64_pipe_kernel<8, false>, 512, 0);
  else if (idx == 1)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, herk_fp64_kernel<64, 16>, 256, 0);
  else if (idx == 2)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, herk_fp64_kernel<32, 16>, 256, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}

}  // namespace chi0
