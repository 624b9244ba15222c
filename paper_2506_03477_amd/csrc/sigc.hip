// Imaginary-axis part I^c of the correlation self-energy (Eq.(sigci)) on
// gfx950 matrix cores, FP64.
//
// For one q-point and one k-point block (intermediate states n', product-
// basis functions mu, nu, quasiparticle states n, m, mesh w_i):
//   I^c[n][m] -= w_k sum_{n'} sum_i w_i(eps_qn - eps_n') sum_{mu,nu}
//                conj(Z[n'][mu][n]) W_i[mu][nu] Z[n'][nu][m].
// It runs as two complex contractions, in the order of the paper's
// self-energy algorithm (weighted Z, then Z_w^H W^c summed over the mesh,
// then the product with Z):
//  1. ZW[n'][n][nu] = sum_{i, mu} t_i(n', n) conj(Z[n'][mu][n]) W_i[mu][nu],
//     with t = -w_k w_i(eps_qn - eps_n').  Contraction index (i, mu) of
//     length nomega * nmu, output rows r = (n', n), columns nu.  The kernel
//     forms D[nu][r] = sum conj(W_i[mu][nu]) t Z[n'][mu][n] = conj(ZW) and
//     stores it as zw[n'][nu][n], the layout of Z itself.
//  2. I^c[n][m] = sum_{(n', nu)} ZW[n'][n][nu] Z[n'][nu][m]
//              = sum_kappa conj(zw[kappa][n]) Z[kappa][m],  kappa = (n', nu),
//     split along kappa into segments whose FP64 partial tiles are summed in
//     a fixed order.
// Both are "conj(P) . Q" contractions over a k-major operand pair, run by one
// kernel template with FP64 MFMAs (v_mfma_f64_16x16x4f64, (re, im) of two
// contraction rows as its four k-slots), 128 x 128 complex tiles, register
// prefetch and double-buffered LDS.
//
// Integration weights w_i(dE): X(iw) interpolated on the mesh (constant below
// the first node, linear between nodes, X(w_last) (w_last / w)^2 beyond),
// times the Lorentzian dE / (pi (dE^2 + w^2)), integrated exactly over
// [0, inf); 0 at dE = 0.
#include "common.h"

namespace chi0 {
namespace {

constexpr int kT = 128;
constexpr double kPi = 3.141592653589793238462643383279502884;

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef const char __attribute__((address_space(1)))* gcptr;
typedef const dvec2 __attribute__((address_space(1)))* gd2ptr;

// (t - atan t) / t^2, t >= 0, without cancellation at small t.
__device__ double tail_factor(double t) {
  if (t < 0.3) {
    const double u = t * t;
    double s = 0.0;
#pragma unroll
    for (int k = 15; k >= 0; --k) s = s * u + ((k & 1) ? -1.0 : 1.0) / (2 * k + 3);
    return t * s;
  }
  return (1.0 - atan(t) / t) / t;
}

// d times the integral of w / (d^2 + w^2) over [a, b] (0 <= a < b), i.e.
// (d/2) ln((d^2 + b^2) / (d^2 + a^2)), without cancellation for |d| >> b or
// overflow for tiny |d|.
__device__ double lorentz_first_moment(double d, double a, double b) {
  if (a > 0.0) return 0.5 * d * log1p((b - a) * (b + a) / (d * d + a * a));
  const double ad = fabs(d);
  if (b < 1e100 * ad) {
    const double r = b / ad;
    return 0.5 * d * log1p(r * r);
  }
  const double r = ad / b;
  return d * (log(b) - log(ad)) + 0.5 * d * log1p(r * r);
}

// Weight of mesh node i for the energy difference d (times pi).
__device__ double ag_weight_pi(double d, const double* om, int n, int i) {
  if (d == 0.0) return 0.0;
  double s = 0.0;
  if (i == 0 && om[0] > 0.0) s += atan(om[0] / d);
  // rising half of node i's basis function on [w_{i-1}, w_i]
  if (i > 0) {
    const double a = om[i - 1], b = om[i], h = b - a;
    const double i0 = atan(d * h / (d * d + a * b));
    const double i1 = lorentz_first_moment(d, a, b);
    s += (i1 - a * i0) / h;
  }
  // falling half on [w_i, w_{i+1}]
  if (i < n - 1) {
    const double a = om[i], b = om[i + 1], h = b - a;
    const double i0 = atan(d * h / (d * d + a * b));
    const double i1 = lorentz_first_moment(d, a, b);
    s += (b * i0 - i1) / h;
  }
  if (i == n - 1) {
    const double c = om[n - 1];
    if (c > 0.0)
      s += copysign(tail_factor(fabs(d) / c), d);
    else
      s += copysign(0.5 * kPi, d);
  }
  return s;
}

__global__ __launch_bounds__(256) void sigc_weights_kernel(const SigcDesc* __restrict__ descs) {
  const SigcDesc bd = descs[blockIdx.y];
  const int64_t M = static_cast<int64_t>(bd.nall) * bd.nqp;
  const int64_t total = M * bd.nomega;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < total; e += static_cast<int64_t>(gridDim.x) * 256) {
    const int i = static_cast<int>(e / M);
    const int64_t r = e - i * M;
    const int a = static_cast<int>(r / bd.nqp);
    const int n = static_cast<int>(r - static_cast<int64_t>(a) * bd.nqp);
    const double d = bd.eps_qp[n] - bd.eps_mid[a];
    bd.wt[e] = -bd.wk * (ag_weight_pi(d, bd.omega, bd.nomega, i) / kPi);
  }
}

// The two contractions.  STAGE1: P = W^c (rows (i, mu), columns nu), Q =
// weighted Z (columns r = (n', n)), output zw.  Otherwise: P = zw, Q = Z
// (rows kappa = (n', nu), columns n resp. m), output a partial tile.
//
// NW = 4: 2 x 2 waves of 64 x 64; NW = 8: 2 x 4 waves of 64 x 32.
template <bool STAGE1, int NW>
__global__ __launch_bounds__(64 * NW, 1) void sigc_gemm_kernel(SigcArgs args) {
  constexpr int T = kT, KC = 8, NT = 64 * NW;
  constexpr int WC = NW / 2;
  constexpr int NBI = 4;
  constexpr int NBJ = T / WC / 16;
  constexpr int LG = NT / T;
  constexpr int NP = KC / LG;
  __shared__ double2 sA[2][KC][T];
  __shared__ double2 sB[2][KC][T];

  // XCD-major placement: consecutive logical units share an XCD (and its L2)
  const int per = (args.nunits + 7) / 8;
  const int lu = static_cast<int>(blockIdx.x % 8) * per + static_cast<int>(blockIdx.x / 8);
  if (lu >= args.nunits) return;
  const SigcUnit u = args.units[lu];
  const SigcDesc bd = args.descs[u.blk];
  const int nqp = bd.nqp, nmu = bd.nmu;
  const int64_t M = static_cast<int64_t>(bd.nall) * nqp;

  // contraction rows [k0, k1) of every mesh point i in [0, ni)
  int ni, k0, k1, ldP, pcols;
  int64_t qcols;
  const char* pbase;
  const char* qbase = reinterpret_cast<const char*>(bd.z);
  if (STAGE1) {
    ni = bd.nomega;
    k0 = 0;
    k1 = nmu;
    ldP = nmu;
    pcols = nmu;
    qcols = M;
    pbase = reinterpret_cast<const char*>(bd.wc);
  } else {
    const int64_t K = static_cast<int64_t>(bd.nall) * nmu;
    ni = 1;
    k0 = u.seg * args.seg_len;
    k1 = static_cast<int>(K - k0 < args.seg_len ? K : k0 + args.seg_len);
    ldP = nqp;
    pcols = nqp;
    qcols = nqp;
    pbase = reinterpret_cast<const char*>(bd.zw);
  }

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int m = lane & 15;
  const int kk = lane >> 4;
  const int prr = kk >> 1;
  const bool isim = (kk & 1) != 0;
  const int lc = tid & (T - 1);
  const int lg = tid / T;

  // this thread's loader columns: P column p, Q column c (clamped into range)
  const int p = u.tp * T + lc;
  const int64_t c = static_cast<int64_t>(u.tc) * T + lc;
  const uint64_t offP = static_cast<uint64_t>(p < pcols ? p : 0) * 16u;
  const int64_t cc = c < qcols ? c : 0;
  const int64_t an = cc / nqp;
  const uint64_t offQ = static_cast<uint64_t>(an * nmu * nqp + (cc - an * nqp)) * 16u;
  const uint64_t rowP = static_cast<uint64_t>(ldP) * 16u;
  const uint64_t rowQ = static_cast<uint64_t>(nqp) * 16u;

  f64x4 accR[NBI][NBJ], accI[NBI][NBJ];
#pragma unroll
  for (int i = 0; i < NBI; ++i)
#pragma unroll
    for (int j = 0; j < NBJ; ++j) {
      accR[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
      accI[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    }

  // stage loads: rows kr = kc + lg + LG * e of mesh point iw; a row beyond k1
  // reads row k1 - 1 with weight 0
  auto load = [&](int iw, int kc, double2 (&ra)[NP], double2 (&rb)[NP], double (&rw)[NP]) {
    const int last = k1 - 1;
    double t = 1.0;
    if (STAGE1) t = bd.wt[static_cast<int64_t>(iw) * M + cc];
#pragma unroll
    for (int e = 0; e < NP; ++e) {
      const int kr = kc + lg + LG * e;
      const bool valid = kr <= last;
      const int ks = valid ? kr : last;
      const gcptr prow = (gcptr)pbase + (static_cast<uint64_t>(iw) * (STAGE1 ? nmu : 0) + ks) * rowP;
      const gcptr qrow = (gcptr)qbase + static_cast<uint64_t>(ks) * rowQ;
      const dvec2 va = *(gd2ptr)(prow + offP);
      const dvec2 vb = *(gd2ptr)(qrow + offQ);
      ra[e] = double2{va.x, va.y};
      rb[e] = double2{vb.x, vb.y};
      rw[e] = valid ? t : 0.0;
    }
  };

  double2 ra[NP], rb[NP];
  double rw[NP];
  int iw = 0, kc = k0;
  bool have = ni > 0 && k0 < k1;
  __syncthreads();
  if (have) load(iw, kc, ra, rb, rw);
  int buf = 0;
  while (have) {
#pragma unroll
    for (int e = 0; e < NP; ++e) {
      const int r = lg + LG * e;
      sA[buf][r][lc] = ra[e];
      sB[buf][r][lc] = double2{rb[e].x * rw[e], rb[e].y * rw[e]};
    }
    int niw = iw, nkc = kc + KC;
    if (nkc >= k1) {
      nkc = k0;
      ++niw;
    }
    const bool more = niw < ni;
    if (more) load(niw, nkc, ra, rb, rw);
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
    iw = niw;
    kc = nkc;
    have = more;
    buf ^= 1;
  }

  if (STAGE1) {
    // D[nu][r] -> zw[n'][nu][n]: column r of this lane, rows nu
#pragma unroll
    for (int j = 0; j < NBJ; ++j) {
      const int64_t col = static_cast<int64_t>(u.tc) * T + wc * (T / WC) + j * 16 + m;
      if (col >= M) continue;
      const int64_t a2 = col / nqp;
      double2* dst = bd.zw + a2 * nmu * nqp + (col - a2 * nqp);
#pragma unroll
      for (int i = 0; i < NBI; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = u.tp * T + wr * 64 + i * 16 + kk + 4 * r;
          if (row < nmu) dst[static_cast<int64_t>(row) * nqp] = double2{accR[i][j][r], accI[i][j][r]};
        }
    }
  } else {
    double2* out = args.partials + static_cast<size_t>(lu) * T * T;
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

__global__ __launch_bounds__(256) void sigc_reduce_kernel(const SigcJob* __restrict__ jobs,
                                                          const int32_t* __restrict__ slots,
                                                          const double2* __restrict__ partials,
                                                          const SigcProb* __restrict__ probs) {
  const SigcJob jb = jobs[blockIdx.y];
  const SigcProb pr = probs[jb.prob];
  const int e = blockIdx.x * 256 + threadIdx.x;   // element of the T x T tile
  const int row = jb.tp * kT + e / kT, col = jb.tc * kT + e % kT;
  if (row >= pr.nqp || col >= pr.nqp) return;
  double re = 0.0, im = 0.0;
  for (int s = 0; s < jb.nslot; ++s) {
    const double2 v = partials[static_cast<size_t>(slots[jb.slot0 + s]) * kT * kT + e];
    re += v.x;
    im += v.y;
  }
  double2* acc = pr.acc + static_cast<size_t>(row) * pr.nqp + col;
  *acc = double2{acc->x + re, acc->y + im};
}

__global__ __launch_bounds__(256) void sigc_clear_kernel(const SigcProb* __restrict__ probs) {
  const SigcProb pr = probs[blockIdx.y];
  const int64_t n = static_cast<int64_t>(pr.nqp) * pr.nqp;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < n; e += static_cast<int64_t>(gridDim.x) * 256)
    pr.acc[e] = double2{0.0, 0.0};
}

__global__ __launch_bounds__(256) void sigc_store_kernel(const SigcProb* __restrict__ probs, int accumulate) {
  const SigcProb pr = probs[blockIdx.y];
  const int64_t n = static_cast<int64_t>(pr.nqp) * pr.nqp;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < n; e += static_cast<int64_t>(gridDim.x) * 256) {
    const double2 a = pr.acc[e];
    if (accumulate) {
      const double2 o = pr.out[e];
      pr.out[e] = double2{o.x + a.x, o.y + a.y};
    } else {
      pr.out[e] = a;
    }
  }
}

}  // namespace

int sigc_tile() { return kT; }
int sigc_zw_variants() { return 2; }

hipError_t sigc_weights_launch(const SigcDesc* descs, int nblocks, int64_t max_elems, hipStream_t s) {
  if (nblocks <= 0 || max_elems <= 0) return hipSuccess;
  int64_t gx = (max_elems + 255) / 256;
  if (gx > 4096) gx = 4096;
  for (int b0 = 0; b0 < nblocks; b0 += 65535) {
    const int nb = nblocks - b0 < 65535 ? nblocks - b0 : 65535;
    hipLaunchKernelGGL(sigc_weights_kernel, dim3(static_cast<unsigned>(gx), nb), dim3(256), 0, s, descs + b0);
  }
  return hipGetLastError();
}

hipError_t sigc_zw_launch(int variant, const SigcArgs& a, hipStream_t s) {
  if (a.nunits <= 0) return hipSuccess;
  const unsigned grid = static_cast<unsigned>((a.nunits + 7) / 8 * 8);
  if (variant == 1)
    hipLaunchKernelGGL((sigc_gemm_kernel<true, 8>), dim3(grid), dim3(512), 0, s, a);
  else
    hipLaunchKernelGGL((sigc_gemm_kernel<true, 4>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t sigc_zwz_launch(const SigcArgs& a, hipStream_t s) {
  if (a.nunits <= 0) return hipSuccess;
  const unsigned grid = static_cast<unsigned>((a.nunits + 7) / 8 * 8);
  hipLaunchKernelGGL((sigc_gemm_kernel<false, 8>), dim3(grid), dim3(512), 0, s, a);
  return hipGetLastError();
}

hipError_t sigc_reduce_launch(const SigcJob* jobs, const int32_t* slot_list, const double2* partials,
                              const SigcProb* probs, int njobs, hipStream_t s) {
  for (int j0 = 0; j0 < njobs; j0 += 65535) {
    const int nj = njobs - j0 < 65535 ? njobs - j0 : 65535;
    hipLaunchKernelGGL(sigc_reduce_kernel, dim3(kT * kT / 256, nj), dim3(256), 0, s, jobs + j0, slot_list,
                       partials, probs);
  }
  return hipGetLastError();
}

hipError_t sigc_clear_launch(const SigcProb* probs, int nprob, int max_nqp, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  int64_t gx = (static_cast<int64_t>(max_nqp) * max_nqp + 255) / 256;
  if (gx > 1024) gx = 1024;
  hipLaunchKernelGGL(sigc_clear_kernel, dim3(static_cast<unsigned>(gx), nprob), dim3(256), 0, s, probs);
  return hipGetLastError();
}

hipError_t sigc_store_launch(const SigcProb* probs, int nprob, int max_nqp, bool accumulate, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  int64_t gx = (static_cast<int64_t>(max_nqp) * max_nqp + 255) / 256;
  if (gx > 1024) gx = 1024;
  hipLaunchKernelGGL(sigc_store_kernel, dim3(static_cast<unsigned>(gx), nprob), dim3(256), 0, s, probs,
                     accumulate ? 1 : 0);
  return hipGetLastError();
}

}  // namespace chi0
