// Cross-block FP64 reduction of the partial tiles and Hermitian write of chi0.
//
// Every lower-triangle tile (tp >= tq) of every frequency owns a contiguous
// run of FP64 partial slots (one per block range), complex interleaved or,
// for kernels that write them so, as a real plane and an imaginary plane.
// They are summed in slot order, so the result does not depend on which
// workgroup produced which slot.  chi0 = -S (Eq.(polfx) at i*omega carries
// the minus sign); the lower triangle is written and mirrored with
// conjugation, and the imaginary part of the diagonal is set to zero, so
// chi0 is exactly Hermitian.
#include "common.h"
#include "herk_common.h"

namespace chi0 {
namespace {

__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a) {
  const TileJob j = a.jobs[blockIdx.y];
  const int TP = a.tile_p, TQ = a.tile_q;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= TP * TQ) return;
  const int row = e / TQ;
  const int col = e - row * TQ;
  const ProbDesc pd = a.probs[j.prob];
  const int npb = pd.npb;
  const int I = j.tp * TP + row;
  const int J = j.tq * TQ + col;
  if (I >= npb || J >= npb) return;
  if (J > I) return;  // upper triangle: mirrored from the lower half
  double re = 0.0, im = 0.0;
  const size_t slot = static_cast<size_t>(TP) * TQ;
  if (a.planar) {
    // slot s: TP x TQ real parts, then TP x TQ imaginary parts
    const double* src = reinterpret_cast<const double*>(a.partials + static_cast<size_t>(j.slot0) * slot) + e;
    for (int s = 0; s < j.nslot; ++s) {
      re += src[2 * static_cast<size_t>(s) * slot];
      im += src[2 * static_cast<size_t>(s) * slot + slot];
    }
  } else {
    const double2* src = a.partials + static_cast<size_t>(j.slot0) * slot + e;
    for (int s = 0; s < j.nslot; ++s) {
      const double2 v = src[static_cast<size_t>(s) * slot];
      re += v.x;
      im += v.y;
    }
  }
  re = -re;
  im = -im;
  double2* out = pd.chi0 + static_cast<size_t>(j.iw) * npb * npb;
  const size_t lo = static_cast<size_t>(I) * npb + J;
  if (a.accumulate) {
    const double2 o = out[lo];
    re += o.x;
    im += o.y;
  }
  if (I == J) im = 0.0;
  out[lo] = double2{re, im};
  if (I != J) out[static_cast<size_t>(J) * npb + I] = double2{re, -im};
}

}  // namespace

hipError_t reduce_launch(const ReduceArgs& a, int njobs, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  const int nthr = 256;
  const int nx = (a.tile_p * a.tile_q + nthr - 1) / nthr;
  hipLaunchKernelGGL(reduce_kernel, dim3(nx, njobs), dim3(nthr), 0, s, a);
  return hipGetLastError();
}

// Built-in default configuration per path (fastest measured on the
// npb = 2048 and spin-polarised workloads: the BF16x3 and FP32
// frequency-group kernels on 128 x 64 tiles; the 8-wave FP64 kernel); the
// autotuner or chi0_set_tile overrides it.
int herk_default_tile(int kind) {
  switch (kind) {
    case HERK_FP64: return 3;
    case HERK_FP32: return 2;
    case HERK_BF16X3: return 20;
  }
  return 0;
}

// Default configuration of calls that read gathered rows (the histogram
// route): the fastest of the configurations that can.
int herk_gather_tile(int kind) {
  switch (kind) {
    case HERK_FP64: return 3;
    case HERK_BF16X3: return 7;
  }
  return herk_default_tile(kind);
}

int herk_tile_count(int kind) {
  switch (kind) {
    case HERK_FP64: return herk_fp64_tile_count();
    case HERK_FP32: return herk_fp32_tile_count();
    case HERK_BF16X3: return herk_bf16x3_tile_count();
  }
  return 0;
}

TileConfig herk_tile_config(int kind, int idx) {
  switch (kind) {
    case HERK_FP64: return herk_fp64_tile(idx);
    case HERK_FP32: return herk_fp32_tile(idx);
    case HERK_BF16X3: return herk_bf16x3_tile(idx);
  }
  return TileConfig{0, 0, 0, 0};
}

int herk_max_wg_per_cu(int kind, int idx) {
  switch (kind) {
    case HERK_FP64: return herk_fp64_max_wg_per_cu(idx);
    case HERK_FP32: return herk_fp32_max_wg_per_cu(idx);
    case HERK_BF16X3: return herk_bf16x3_max_wg_per_cu(idx);
  }
  return 1;
}

hipError_t herk_launch(int kind, int idx, const HerkArgs& a, int nwg, hipStream_t s, bool gather) {
  if (gather && !herk_tile_gathers(kind, idx)) return hipErrorInvalidValue;
  switch (kind) {
    case HERK_FP64: return herk_fp64_launch(idx, a, nwg, s, gather);
    case HERK_FP32: return herk_fp32_launch(idx, a, nwg, s);
    case HERK_BF16X3: return herk_bf16x3_launch(idx, a, nwg, s, gather);
  }
  return hipErrorInvalidValue;
}

bool herk_tile_gathers(int kind, int idx) {
  if (kind == HERK_FP64) return idx == 0 || idx == 3;
  if (kind == HERK_BF16X3) return idx == 5 || idx == 7;
  return false;
}

}  // namespace chi0
