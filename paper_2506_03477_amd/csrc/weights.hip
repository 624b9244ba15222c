// Pair weights (Eq.(polfx) on the imaginary axis) for every pair of every
// block and every frequency, written once per call into the problems'
// weight arrays [nomega][ktot]:
//   w = w_k * 2 D / (D^2 + omega^2),  D = eps_unocc[n'] - eps_occ[n],
// and 0 for excluded pairs (D <= 0 or D < delta_min).  The rank-K kernels
// read these as plain loads next to Z.  Pairs with D <= 0 are also counted
// into a status word that chi0_sync reports as an argument error.
#include "common.h"
#include "herk_common.h"

namespace chi0 {
namespace {

template <class W>
__global__ __launch_bounds__(256) void pair_weights_kernel(const BlockDesc* __restrict__ blocks,
                                                           const ProbDesc* __restrict__ probs,
                                                           double delta_min, int32_t* nonpositive) {
  const BlockDesc bd = blocks[blockIdx.y];
  const int K = bd.nocc * bd.nunocc;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= K) return;
  {
    const int n = p / bd.nunocc;
    const double d = bd.eps_unocc[p - n * bd.nunocc] - bd.eps_occ[n];
    count_lanes(nonpositive, !(d > 0.0));
  }
  const ProbDesc pd = probs[bd.prob];
  W* out = static_cast<W*>(pd.wts) + bd.pair_base + p;
  for (int iw = 0; iw < pd.nomega; ++iw) {
    const double om = pd.omega[iw];
    out[static_cast<size_t>(iw) * pd.ktot] = static_cast<W>(pair_weight(bd, p, K, om * om, delta_min));
  }
}

// Exchange self-energy rows (Eq.(sigx)): row p = n' nmu + mu of a block has
// weight w_k v[mu]; the block's nunocc is nmu and eps_unocc holds v.
template <class W>
__global__ __launch_bounds__(256) void coulomb_weights_kernel(const BlockDesc* __restrict__ blocks,
                                                              const ProbDesc* __restrict__ probs) {
  const BlockDesc bd = blocks[blockIdx.y];
  const int K = bd.nocc * bd.nunocc;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= K) return;
  const ProbDesc pd = probs[bd.prob];
  W* out = static_cast<W*>(pd.wts) + bd.pair_base + p;
  const double w = bd.wk * bd.eps_unocc[p % bd.nunocc];
  for (int iw = 0; iw < pd.nomega; ++iw) out[static_cast<size_t>(iw) * pd.ktot] = static_cast<W>(w);
}

}  // namespace

hipError_t coulomb_weights_launch(const BlockDesc* blocks, const ProbDesc* probs, int nblocks,
                                  int kmax, bool f64, hipStream_t s) {
  if (nblocks <= 0 || kmax <= 0) return hipSuccess;
  const dim3 grid((kmax + 255) / 256, nblocks);
  if (f64)
    hipLaunchKernelGGL(coulomb_weights_kernel<double>, grid, dim3(256), 0, s, blocks, probs);
  else
    hipLaunchKernelGGL(coulomb_weights_kernel<float>, grid, dim3(256), 0, s, blocks, probs);
  return hipGetLastError();
}

hipError_t pair_weights_launch(const BlockDesc* blocks, const ProbDesc* probs, int nblocks, int kmax,
                               double delta_min, bool f64, int32_t* nonpositive, hipStream_t s) {
  if (nblocks <= 0 || kmax <= 0) return hipSuccess;
  const dim3 grid((kmax + 255) / 256, nblocks);
  if (f64)
    hipLaunchKernelGGL(pair_weights_kernel<double>, grid, dim3(256), 0, s, blocks, probs, delta_min,
                       nonpositive);
  else
    hipLaunchKernelGGL(pair_weights_kernel<float>, grid, dim3(256), 0, s, blocks, probs, delta_min,
                       nonpositive);
  return hipGetLastError();
}

}  // namespace chi0
