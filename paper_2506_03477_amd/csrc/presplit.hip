// BF16 hi / lo split of the unscaled P-side operand, once per call.
//
// The P side of the rank-K update (conj(Z_P) without the pair weight) does
// not depend on the frequency, so kernels that read it pre-split save the
// split in every (tile, frequency) unit.  For every block, group g of four
// pairs and product-basis column c, the four pairs' (re, im) values are
// rounded to bf16 hi = RNE(x) and lo = RNE(x - hi) (x - hi is exact in FP32)
// and stored as 16-byte chunks
//   hi plane: zs + (g * npb + c) * 16,  lo plane: the same + zs_plane,
// each 32-bit word holding (re, im) of one pair, re in the low half; pairs
// beyond the block's end (padding to whole 16-pair stages) are zero.  A
// gathered block (BlockDesc::rows) reads row p at the address rows[p].
#include "common.h"
#include "herk_common.h"

namespace chi0 {
namespace {

__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  bf16x2 v;
  v[0] = static_cast<__bf16>(lo);
  v[1] = static_cast<__bf16>(hi);
  return __builtin_bit_cast(uint32_t, v);
}

__global__ __launch_bounds__(256) void presplit_kernel(const BlockDesc* __restrict__ blocks,
                                                       const ProbDesc* __restrict__ probs,
                                                       int block0) {
#pragma clang fp contract(off)
  const BlockDesc bd = blocks[block0 + blockIdx.z];
  const int npb = probs[bd.prob].npb;
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= npb) return;
  const int64_t K = static_cast<int64_t>(bd.nocc) * bd.nunocc;
  const int64_t G = presplit_groups(K);
  const float2* z = static_cast<const float2*>(bd.z);
  char* hi_plane = static_cast<char*>(bd.zs);
  char* lo_plane = hi_plane + bd.zs_plane;
  for (int64_t g = blockIdx.y; g < G; g += gridDim.y) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t p = 4 * g + e;
      const float2 x = p >= K   ? float2{0.f, 0.f}
                       : bd.rows ? reinterpret_cast<const float2*>(bd.rows[p])[c]
                                 : z[p * npb + c];
      h[e] = pack2(x.x, x.y);
      const float hr = __uint_as_float(h[e] << 16);
      const float hm = __uint_as_float(h[e] & 0xFFFF0000u);
      l[e] = pack2(x.x - hr, x.y - hm);
    }
    const size_t off = (static_cast<size_t>(g) * npb + c) * 16;
    *reinterpret_cast<uint4*>(hi_plane + off) = uint4{h[0], h[1], h[2], h[3]};
    *reinterpret_cast<uint4*>(lo_plane + off) = uint4{l[0], l[1], l[2], l[3]};
  }
}

__device__ __forceinline__ void split_chunk(const float2 (&x)[4], uint4& hi, uint4& lo) {
  uint32_t h[4], l[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    h[e] = pack2(x[e].x, x[e].y);
    const float hr = __uint_as_float(h[e] << 16);
    const float hm = __uint_as_float(h[e] & 0xFFFF0000u);
    l[e] = pack2(x[e].x - hr, x[e].y - hm);
  }
  hi = uint4{h[0], h[1], h[2], h[3]};
  lo = uint4{l[0], l[1], l[2], l[3]};
}

// Correlation self-energy, BF16x3 first contraction: W^c of every mesh point
// (rows mu, columns nu) and the weighted Z of every mesh point (rows mu,
// columns r = (n', n)) of one block (blockIdx.z) rounded to FP32 and split
// into the planes SigcDesc describes; rows beyond nmu are zero.
__global__ __launch_bounds__(256) void sigc_split_w_kernel(const SigcDesc* __restrict__ descs, int blk0) {
#pragma clang fp contract(off)
  const SigcDesc bd = descs[blk0 + blockIdx.z];
  const int nu = blockIdx.x * 256 + threadIdx.x;
  if (nu >= bd.nmu) return;
  const int64_t total = static_cast<int64_t>(bd.nomega) * bd.groups;
  for (int64_t gi = blockIdx.y; gi < total; gi += gridDim.y) {
    const int i = static_cast<int>(gi / bd.groups);
    const int g = static_cast<int>(gi - static_cast<int64_t>(i) * bd.groups);
    float2 x[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int mu = 4 * g + e;
      double2 v = {0.0, 0.0};
      if (mu < bd.nmu) v = bd.wc[(static_cast<int64_t>(i) * bd.nmu + mu) * bd.nmu + nu];
      x[e] = float2{static_cast<float>(v.x), static_cast<float>(v.y)};
    }
    uint4 hi, lo;
    split_chunk(x, hi, lo);
    const size_t off = (static_cast<size_t>(gi) * bd.nmu + nu) * 16;
    *reinterpret_cast<uint4*>(static_cast<char*>(bd.wsp) + off) = hi;
    *reinterpret_cast<uint4*>(static_cast<char*>(bd.wsp) + bd.wsp_plane + off) = lo;
  }
}

// Z scaled by the weight of each mesh point: the plane of mesh point i holds
// t_i(r) Z[mu][r] (product in FP64, rounded to FP32, split), so the first
// contraction sums every mesh point into one FP32 accumulator.
__global__ __launch_bounds__(256) void sigc_split_z_kernel(const SigcDesc* __restrict__ descs, int blk0) {
#pragma clang fp contract(off)
  const SigcDesc bd = descs[blk0 + blockIdx.z];
  const int64_t M = static_cast<int64_t>(bd.nall) * bd.nqp;
  const int64_t r = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (r >= M) return;
  const int64_t a = r / bd.nqp;
  const int64_t n = r - a * bd.nqp;
  const double2* zr = bd.z + a * bd.nmu * bd.nqp + n;
  for (int g = blockIdx.y; g < bd.groups; g += gridDim.y) {
    double2 v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int mu = 4 * g + e;
      v[e] = mu < bd.nmu ? zr[static_cast<int64_t>(mu) * bd.nqp] : double2{0.0, 0.0};
    }
    for (int i = 0; i < bd.nomega; ++i) {
      const double t = bd.wt[static_cast<int64_t>(i) * M + r];
      float2 x[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) x[e] = float2{static_cast<float>(t * v[e].x), static_cast<float>(t * v[e].y)};
      uint4 hi, lo;
      split_chunk(x, hi, lo);
      const size_t off = ((static_cast<size_t>(i) * bd.groups + g) * M + r) * 16;
      *reinterpret_cast<uint4*>(static_cast<char*>(bd.zsp) + off) = hi;
      *reinterpret_cast<uint4*>(static_cast<char*>(bd.zsp) + bd.zsp_plane + off) = lo;
    }
  }
}

// Second contraction of the correlation self-energy on the BF16x3 path: the
// [nall * nmu][nqp] matrix zw (which = 0) or Z (which = 1) of one block
// (blockIdx.z) rounded to FP32 and split: group g of 4 rows kappa, column n
// at (g * nqp + n) * 16 bytes; rows beyond nall * nmu are zero.
__global__ __launch_bounds__(256) void sigc_split_rows_kernel(const SigcDesc* __restrict__ descs, int blk0,
                                                              int which) {
  const SigcDesc bd = descs[blk0 + blockIdx.z];
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= bd.nqp) return;
  const int64_t K = static_cast<int64_t>(bd.nall) * bd.nmu;
  const double2* src = which ? bd.z : bd.zw;
  char* dst = static_cast<char*>(which ? bd.zksp : bd.zwsp);
  for (int64_t g = blockIdx.y; g < bd.kgroups; g += gridDim.y) {
    float2 x[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t kap = 4 * g + e;
      const double2 v = kap < K ? src[kap * bd.nqp + n] : double2{0.0, 0.0};
      x[e] = float2{static_cast<float>(v.x), static_cast<float>(v.y)};
    }
    uint4 hi, lo;
    split_chunk(x, hi, lo);
    const size_t off = (static_cast<size_t>(g) * bd.nqp + n) * 16;
    *reinterpret_cast<uint4*>(dst + off) = hi;
    *reinterpret_cast<uint4*>(dst + bd.k_plane + off) = lo;
  }
}

}  // namespace

hipError_t sigc_split_rows_launch(const SigcDesc* descs, int nblocks, int which, int max_nqp,
                                  int max_kgroups, hipStream_t s) {
  if (nblocks <= 0 || max_nqp <= 0) return hipSuccess;
  const unsigned gy = static_cast<unsigned>(max_kgroups < 8192 ? (max_kgroups > 0 ? max_kgroups : 1) : 8192);
  for (int b0 = 0; b0 < nblocks; b0 += 65535) {
    const int nb = nblocks - b0 < 65535 ? nblocks - b0 : 65535;
    hipLaunchKernelGGL(sigc_split_rows_kernel, dim3((max_nqp + 255) / 256, gy, nb), dim3(256), 0, s, descs,
                       b0, which);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t sigc_presplit_launch(const SigcDesc* descs, int nblocks, int max_nmu, int64_t max_m,
                                int max_groups_w, int max_groups_z, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  for (int b0 = 0; b0 < nblocks; b0 += 65535) {
    const int nb = nblocks - b0 < 65535 ? nblocks - b0 : 65535;
    const unsigned gyw = static_cast<unsigned>(max_groups_w < 4096 ? max_groups_w : 4096);
    hipLaunchKernelGGL(sigc_split_w_kernel, dim3((max_nmu + 255) / 256, gyw, nb), dim3(256), 0, s, descs, b0);
    const unsigned gyz = static_cast<unsigned>(max_groups_z < 64 ? max_groups_z : 64);
    hipLaunchKernelGGL(sigc_split_z_kernel, dim3(static_cast<unsigned>((max_m + 255) / 256), gyz, nb),
                       dim3(256), 0, s, descs, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t presplit_launch(const BlockDesc* blocks, const ProbDesc* probs, int nblocks,
                           int64_t max_groups, int max_npb, hipStream_t s) {
  if (nblocks <= 0 || max_groups <= 0 || max_npb <= 0) return hipSuccess;
  const unsigned gy = static_cast<unsigned>(max_groups < 4096 ? max_groups : 4096);
  for (int b0 = 0; b0 < nblocks; b0 += 65535) {
    const int nb = nblocks - b0 < 65535 ? nblocks - b0 : 65535;
    hipLaunchKernelGGL(presplit_kernel, dim3((max_npb + 255) / 256, gy, nb), dim3(256), 0, s,
                       blocks, probs, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace chi0
