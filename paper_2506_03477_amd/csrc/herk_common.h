// Device helpers shared by the rank-K kernels.
#pragma once

#include "common.h"

namespace chi0 {

// Transition weight of pair p (= n * nunocc + n') of a block on the imaginary
// axis, without the overall minus sign of Eq.(polfx) at i*omega:
//   c = w_k * 2 D / (D^2 + omega^2),  D = eps_unocc[n'] - eps_occ[n],
// and 0 for pairs outside the block or excluded (D <= 0 or D < delta_min).
// D is formed by one FP64 subtraction, so the inclusion decision matches any
// other FP64 evaluation of the same inputs exactly.
__device__ __forceinline__ double pair_weight(const BlockDesc& bd, int p, int K,
                                              double w2, double delta_min) {
  if (p >= K) return 0.0;
  const int n = p / bd.nunocc;
  const int m = p - n * bd.nunocc;
  const double d = bd.eps_unocc[m] - bd.eps_occ[n];
  if (!(d > 0.0 && d >= delta_min)) return 0.0;
  return bd.wk * 2.0 * d / (d * d + w2);
}

// Host-side dispatch tables of the three precision paths.
int herk_fp64_tile_count();
TileConfig herk_fp64_tile(int idx);
hipError_t herk_fp64_launch(int idx, const HerkArgs& a, int nwg, hipStream_t s);
int herk_fp64_max_wg_per_cu(int idx);

int herk_fp32_tile_count();
TileConfig herk_fp32_tile(int idx);
hipError_t herk_fp32_launch(int idx, const HerkArgs& a, int nwg, hipStream_t s);
int herk_fp32_max_wg_per_cu(int idx);

int herk_bf16x3_tile_count();
TileConfig herk_bf16x3_tile(int idx);
hipError_t herk_bf16x3_launch(int idx, const HerkArgs& a, int nwg, hipStream_t s);
int herk_bf16x3_max_wg_per_cu(int idx);

}  // namespace chi0
