// GPU side of the seeded input generator: fills a block of Z from Philox4x32-10
// counters exactly as synth/workloads.py does on the CPU (same counters, same
// integer arithmetic, one rounding of an exact integer times F[I], then an
// optional round-to-nearest to complex64), so both sides hold bit-identical
// inputs.  Input generation only; no polarization arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
constexpr uint32_t kKey0 = 2506u, kKey1 = 3477u;

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint32_t hi0 = __umulhi(kM0, c[0]), lo0 = kM0 * c[0];
    const uint32_t hi1 = __umulhi(kM1, c[2]), lo1 = kM1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ int halves(uint32_t a, uint32_t b) {
  return static_cast<int>((a & 0xFFFFu) + (a >> 16) + (b & 0xFFFFu) + (b >> 16));
}

template <bool C64>
__global__ __launch_bounds__(256) void z_fill_kernel(void* out, int npb, uint64_t total, uint32_t bid,
                                                     uint32_t c3, const double* __restrict__ F) {
  for (uint64_t e = blockIdx.x * 256ull + threadIdx.x; e < total; e += static_cast<uint64_t>(gridDim.x) * 256ull) {
    uint32_t c[4] = {static_cast<uint32_t>(e), static_cast<uint32_t>(e >> 32), bid, c3};
    philox4x32_10(c, kKey0, kKey1);
    const int col = static_cast<int>(e % static_cast<uint64_t>(npb));
    const double f = F[col];
    const double re = static_cast<double>(halves(c[0], c[1]) - 131070) * f;
    const double im = static_cast<double>(halves(c[2], c[3]) - 131070) * f;
    if (C64)
      static_cast<float2*>(out)[e] = float2{static_cast<float>(re), static_cast<float>(im)};
    else
      static_cast<double2*>(out)[e] = double2{re, im};
  }
}

// Synthetic W^c for the correlation workloads: element (i, mu, nu) of
// [nomega][nmu][nmu] is -(C[i][mu] C[i][nu]) h[mu][nu] with h = 1 on the
// diagonal and h = x F2[|mu - nu|] below it (x the centred Irwin-Hall draw of
// element e = mu * nmu + nu), conjugated above it.  Products only, each
// correctly rounded, in the order the CPU generator uses.
__global__ __launch_bounds__(256) void wc_fill_kernel(double2* __restrict__ out, int nmu, int nomega,
                                                      uint32_t bid, uint32_t c3,
                                                      const double* __restrict__ F2,
                                                      const double* __restrict__ C) {
  const uint64_t plane = static_cast<uint64_t>(nmu) * nmu;
  const uint64_t total = plane * nomega;
  for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < total; t += static_cast<uint64_t>(gridDim.x) * 256ull) {
    const int i = static_cast<int>(t / plane);
    const uint64_t rem = t - static_cast<uint64_t>(i) * plane;
    const int mu = static_cast<int>(rem / nmu);
    const int nu = static_cast<int>(rem - static_cast<uint64_t>(mu) * nmu);
    double hr = 1.0, hi = 0.0;
    if (mu != nu) {
      const int a = mu > nu ? mu : nu, b = mu > nu ? nu : mu;
      const uint64_t e = static_cast<uint64_t>(a) * nmu + b;
      uint32_t c[4] = {static_cast<uint32_t>(e), static_cast<uint32_t>(e >> 32), bid, c3};
      philox4x32_10(c, kKey0, kKey1);
      const double f = F2[a - b];
      hr = static_cast<double>(halves(c[0], c[1]) - 131070) * f;
      hi = static_cast<double>(halves(c[2], c[3]) - 131070) * f;
      if (mu < nu) hi = -hi;
    }
    const double cc = C[static_cast<size_t>(i) * nmu + mu] * C[static_cast<size_t>(i) * nmu + nu];
    out[t] = double2{-(cc * hr), -(cc * hi)};
  }
}

}  // namespace

extern "C" int synth_wc_fill(void* out, int nmu, int nomega, uint32_t bid, uint32_t c3,
                             const double* F2, const double* C, void* stream) {
  if (!out || !F2 || !C || nmu < 1 || nomega < 1) return -1;
  const uint64_t total = static_cast<uint64_t>(nmu) * nmu * nomega;
  uint64_t nblk = (total + 255) / 256;
  if (nblk > 1u << 20) nblk = 1u << 20;
  hipLaunchKernelGGL(wc_fill_kernel, dim3(static_cast<unsigned>(nblk)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), static_cast<double2*>(out), nmu, nomega, bid, c3,
                     F2, C);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

extern "C" int synth_z_fill(void* out, int is_c64, int npb, int nocc, int nunocc, uint32_t bid,
                            uint32_t c3, const double* F, void* stream) {
  if (!out || !F || npb < 1 || nocc < 0 || nunocc < 0) return -1;
  const uint64_t total = static_cast<uint64_t>(nocc) * nunocc * npb;
  if (total == 0) return 0;
  uint64_t nblk = (total + 255) / 256;
  if (nblk > 1u << 20) nblk = 1u << 20;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (is_c64)
    hipLaunchKernelGGL(z_fill_kernel<true>, dim3(static_cast<unsigned>(nblk)), dim3(256), 0, s, out, npb,
                       total, bid, c3, F);
  else
    hipLaunchKernelGGL(z_fill_kernel<false>, dim3(static_cast<unsigned>(nblk)), dim3(256), 0, s, out, npb,
                       total, bid, c3, F);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}
