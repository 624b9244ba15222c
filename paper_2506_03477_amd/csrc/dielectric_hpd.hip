// Inverse of a Hermitian positive definite eps (eps >= 1 because chi0 is
// negative semidefinite) by blocked symmetric Gauss-Jordan sweeps without
// pivoting, on the lower triangle only: half the work and memory traffic of
// the pivoted Gauss-Jordan inverse.
//
// Sweeping index block K (nb columns) of the Hermitian matrix X maps
//   X_KK -> -D^{-1},  X_RK -> X_RK D^{-1},  X_KR -> D^{-1} X_KR,
//   X_RR -> X_RR - X_RK D^{-1} X_KR         (D = X_KK, R = every other index),
// which keeps X Hermitian; after every block has been swept X = -eps^{-1}.
// Every D met is a Schur complement of eps, hence Hermitian positive definite
// when eps is; a pivot that is not positive marks eps as not HPD (the
// result is then undefined and the caller may fall back to the pivoted
// inverse).  Per block:
//   1. hpd_diag:   D^{-1} by nb scalar sweeps of D in LDS; X_KK <- -D^{-1};
//   2. hpd_panel:  C = P D^{-1} for the panel column P = X_RK, which is kept
//                  (P) and written back as the new panel (C);
//   3. hpd_update: X_RR -= C P^H on the lower-triangle tiles (FP64 MFMA).
// Finally eps^{-1} = -X, mirrored from the lower triangle (and W^c).
#include "common.h"

namespace chi0 {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kNb = 32;   // block width
constexpr int kRowsPerPanelWg = 64;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ double2 conjd(double2 a) { return double2{a.x, -a.y}; }

__global__ __launch_bounds__(kNb * kNb) void hpd_diag_kernel(double2* __restrict__ work,
                                                             double2* __restrict__ dinv, int n,
                                                             int k0, int nb,
                                                             int32_t* __restrict__ status,
                                                             int report) {
  __shared__ double2 M[kNb][kNb + 1];
  const int mat = blockIdx.x;
  double2* X = work + static_cast<size_t>(mat) * n * n;
  const int r = threadIdx.x / kNb, c = threadIdx.x % kNb;
  const bool in = r < nb && c < nb;
  double2 v = double2{0.0, 0.0};
  if (in)
    v = c <= r ? X[static_cast<size_t>(k0 + r) * n + k0 + c]
               : conjd(X[static_cast<size_t>(k0 + c) * n + k0 + r]);
  if (r == c) v.y = 0.0;  // the diagonal of a Hermitian matrix is real
  M[r][c] = v;
  __syncthreads();
  bool ok = true;
  for (int t = 0; t < nb; ++t) {
    const double d = M[t][t].x;
    ok = ok && d > 0.0;
    const double2 mrt = M[r][t], mtc = M[t][c], mrc = M[r][c];
    __syncthreads();
    if (in) {
      double2 nv;
      if (r == t && c == t) {
        nv = double2{-1.0 / d, 0.0};
      } else if (c == t) {
        nv = double2{mrt.x / d, mrt.y / d};
      } else if (r == t) {
        nv = double2{mtc.x / d, mtc.y / d};
      } else {
        const double2 p = cmul(mrt, mtc);
        nv = double2{mrc.x - p.x / d, mrc.y - p.y / d};
      }
      M[r][c] = nv;
    }
    __syncthreads();
  }
  if (in) {
    if (c <= r) X[static_cast<size_t>(k0 + r) * n + k0 + c] = M[r][c];
  }
  const double2 m = M[r][c];
  dinv[static_cast<size_t>(mat) * kNb * kNb + r * kNb + c] =
      in ? double2{-m.x, -m.y} : double2{0.0, 0.0};
  if (!ok && threadIdx.x == 0) {
    status[1] = 1;                 // this call: not HPD
    if (report) status[2] = 1;     // reported by chi0_sync
  }
}

// 64 rows per workgroup: P_i = X[i][K] for the rows i outside the block
// (gathered from the lower triangle into LDS), C_i = P_i D^{-1}; P and C are
// kept row-major [n][kNb] for the update, and C is written back as the new
// X[i][K].  Thread (t, g) computes C[i][t] for the rows i = g + 8 k.
__global__ __launch_bounds__(256) void hpd_panel_kernel(
    double2* __restrict__ work, const double2* __restrict__ dinv, double2* __restrict__ pbuf,
    double2* __restrict__ cbuf, int n, int k0, int nb) {
  constexpr int RW = kRowsPerPanelWg;
  __shared__ double2 Di[kNb][kNb];
  __shared__ double2 sP[RW][kNb + 1];
  const int mat = blockIdx.y;
  const int r0 = blockIdx.x * RW;
  const int tid = threadIdx.x;
  double2* X = work + static_cast<size_t>(mat) * n * n;
  const double2* dm = dinv + static_cast<size_t>(mat) * kNb * kNb;
  for (int e = tid; e < kNb * kNb; e += 256) Di[e / kNb][e % kNb] = dm[e];
  // rows above the block read a row segment of the block rows (row index
  // fastest for coalescing), rows below read their own row
  const bool above_wg = r0 < k0;
  for (int e = tid; e < RW * kNb; e += 256) {
    const int rr = above_wg ? e % RW : e / kNb;
    const int u = above_wg ? e / RW : e % kNb;
    const int i = r0 + rr;
    double2 x = double2{0.0, 0.0};
    if (i < n && u < nb && !(i >= k0 && i < k0 + nb))
      x = i >= k0 + nb ? X[static_cast<size_t>(i) * n + k0 + u]
                       : conjd(X[static_cast<size_t>(k0 + u) * n + i]);
    sP[rr][u] = x;
  }
  __syncthreads();
  const int t = tid % kNb;
  const int g = tid / kNb;
  double2 acc[RW / 8];
#pragma unroll
  for (int k = 0; k < RW / 8; ++k) acc[k] = double2{0.0, 0.0};
#pragma unroll 4
  for (int u = 0; u < kNb; ++u) {
    const double2 d = Di[u][t];
#pragma unroll
    for (int k = 0; k < RW / 8; ++k) {
      const double2 pr = cmul(sP[g + 8 * k][u], d);
      acc[k].x += pr.x;
      acc[k].y += pr.y;
    }
  }
#pragma unroll
  for (int k = 0; k < RW / 8; ++k) {
    const int rr = g + 8 * k;
    const int i = r0 + rr;
    if (i >= n || (i >= k0 && i < k0 + nb)) continue;
    const size_t row = (static_cast<size_t>(mat) * n + i) * kNb;
    pbuf[row + t] = sP[rr][t];
    cbuf[row + t] = acc[k];
    if (t < nb) {
      if (i >= k0 + nb)
        X[static_cast<size_t>(i) * n + k0 + t] = acc[k];
      else
        X[static_cast<size_t>(k0 + t) * n + i] = conjd(acc[k]);
    }
  }
}

// X[i][j] -= sum_t C[i][t] conj(P[j][t]) for i, j outside the block, j <= i.
// One 64 x 64 lower-triangle tile per workgroup (blockIdx.x enumerates the
// tiles (I, J), J <= I), 4 waves of 32 x 32, FP64 16x16x4 MFMA with (re, im)
// stacked along the contraction index:
//   Re += [Cr, Ci] . [Pr, Pi],   Im += [Cr, Ci] . [-Pi, Pr].
__global__ __launch_bounds__(256) void hpd_update_kernel(double2* __restrict__ work,
                                                         const double2* __restrict__ pbuf,
                                                         const double2* __restrict__ cbuf,
                                                         int n, int k0, int nb) {
  constexpr int T = 64;
  __shared__ double2 sC[kNb][T];
  __shared__ double2 sP[kNb][T];
  const int mat = blockIdx.y;
  // triangular decode of the tile index
  const int L = blockIdx.x;
  int I = static_cast<int>((sqrt(8.0 * L + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= L) ++I;
  while (I * (I + 1) / 2 > L) --I;
  const int J = L - I * (I + 1) / 2;
  const int i0 = I * T, j0 = J * T;
  const int tid = threadIdx.x;
  const double2* Cm = cbuf + static_cast<size_t>(mat) * n * kNb;
  const double2* Pm = pbuf + static_cast<size_t>(mat) * n * kNb;
  double2* X = work + static_cast<size_t>(mat) * n * n;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int m = lane & 15;
  const int kk = lane >> 4;
  // the 16 old values of this thread's outputs, read before the tile is
  // staged so that their latency overlaps the staging and the MFMAs
  double2 xo[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr * 32 + a * 16 + kk + 4 * r;
        const int j = j0 + wc * 32 + c * 16 + m;
        const bool keep = i < n && j <= i && !(i >= k0 && i < k0 + nb) && !(j >= k0 && j < k0 + nb);
        xo[a][c][r] = keep ? X[static_cast<size_t>(i) * n + j] : double2{0.0, 0.0};
      }
  for (int e = tid; e < kNb * T; e += 256) {
    const int b = e % kNb;
    const int rr = e / kNb;
    const int ri = i0 + rr, rj = j0 + rr;
    const bool oki = ri < n && !(ri >= k0 && ri < k0 + nb) && b < nb;
    const bool okj = rj < n && !(rj >= k0 && rj < k0 + nb) && b < nb;
    // rows XOR-swizzled by b: the 32 b of one row spread over the LDS banks
    sC[b][rr ^ (b & 15)] = oki ? Cm[static_cast<size_t>(ri) * kNb + b] : double2{0.0, 0.0};
    sP[b][rr ^ (b & 15)] = okj ? Pm[static_cast<size_t>(rj) * kNb + b] : double2{0.0, 0.0};
  }
  __syncthreads();
  const int prr = kk >> 1;
  const bool isim = (kk & 1) != 0;
  f64x4 accR[2][2], accI[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      accR[a][c] = f64x4{0.0, 0.0, 0.0, 0.0};
      accI[a][c] = f64x4{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll 4
  for (int st = 0; st < kNb / 2; ++st) {
    const int b = 2 * st + prr;
    double av[2], br[2], bi[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const double2 x = sC[b][wr * 32 + a * 16 + (m ^ (b & 15))];
      av[a] = isim ? x.y : x.x;
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double2 y = sP[b][wc * 32 + c * 16 + (m ^ (b & 15))];
      br[c] = isim ? y.y : y.x;
      bi[c] = isim ? y.x : -y.y;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        accR[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], br[c], accR[a][c], 0, 0, 0);
        accI[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bi[c], accI[a][c], 0, 0, 0);
      }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr * 32 + a * 16 + kk + 4 * r;  // f64 16x16x4 result rows
        const int j = j0 + wc * 32 + c * 16 + m;
        if (i >= n || j > i || (i >= k0 && i < k0 + nb) || (j >= k0 && j < k0 + nb)) continue;
        const size_t ad = static_cast<size_t>(i) * n + j;
        X[ad] = double2{xo[a][c][r].x - accR[a][c][r], xo[a][c][r].y - accI[a][c][r]};
      }
}

// eps^{-1} = -X mirrored from the lower triangle (real diagonal), and
// W^c = diag(s) (eps^{-1} - 1) diag(s).  32 x 32 output tiles; the source
// tile (max(I, J), min(I, J)) is staged through LDS so both the direct and
// the mirrored reads are coalesced.
__global__ __launch_bounds__(256) void hpd_finish_kernel(const double2* __restrict__ work,
                                                         double2* __restrict__ eps_inv,
                                                         double2* __restrict__ wc,
                                                         const double* __restrict__ s, int n) {
#pragma clang fp contract(off)
  __shared__ double2 t[32][33];
  const int mat = blockIdx.z;
  const int I = blockIdx.y, J = blockIdx.x;
  const int SI = I >= J ? I : J, SJ = I >= J ? J : I;
  const double2* X = work + static_cast<size_t>(mat) * n * n;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int i = SI * 32 + r, j = SJ * 32 + tx;
    t[r][tx] = (i < n && j < n) ? X[static_cast<size_t>(i) * n + j] : double2{0.0, 0.0};
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = I * 32 + r, j = J * 32 + tx;
    if (i >= n || j >= n) continue;
    double2 x;
    if (I > J || (I == J && tx <= r))
      x = t[r][tx];
    else
      x = conjd(t[tx][r]);
    if (i == j) x.y = 0.0;
    const double2 v = double2{-x.x, -x.y};
    const size_t ad = static_cast<size_t>(mat) * n * n + static_cast<size_t>(i) * n + j;
    eps_inv[ad] = v;
    if (wc) {
      const double si = s[i], sj = s[j];
      double2 w;
      w.x = (si * (v.x - (i == j ? 1.0 : 0.0))) * sj;
      w.y = (si * v.y) * sj;
      wc[ad] = w;
    }
  }
}

__global__ void hpd_status_clear_kernel(int32_t* __restrict__ status) {
  if (threadIdx.x == 0) status[1] = 0;
}

}  // namespace

int hpd_block_width() { return kNb; }

hipError_t hpd_status_clear_launch(int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(hpd_status_clear_kernel, dim3(1), dim3(64), 0, s, status);
  return hipGetLastError();
}

hipError_t hpd_step_launch(double2* work, double2* dinv, double2* pbuf, double2* cbuf, int n,
                           int nomega, int k0, int nb, int32_t* status, bool report,
                           hipStream_t s) {
  hipLaunchKernelGGL(hpd_diag_kernel, dim3(nomega), dim3(kNb * kNb), 0, s, work, dinv, n, k0, nb,
                     status, report ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (n == nb) return hipSuccess;  // a single block: nothing else to sweep
  hipLaunchKernelGGL(hpd_panel_kernel, dim3((n + kRowsPerPanelWg - 1) / kRowsPerPanelWg, nomega),
                     dim3(256), 0, s, work, dinv, pbuf, cbuf, n, k0, nb);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nt = (n + 63) / 64;
  hipLaunchKernelGGL(hpd_update_kernel, dim3(nt * (nt + 1) / 2, nomega), dim3(256), 0, s, work,
                     pbuf, cbuf, n, k0, nb);
  return hipGetLastError();
}

hipError_t hpd_finish_launch(const double2* work, double2* eps_inv, double2* wc,
                             const double* vsqrt, int n, int nomega, hipStream_t s) {
  const int nt = (n + 31) / 32;
  hipLaunchKernelGGL(hpd_finish_kernel, dim3(nt, nt, nomega), dim3(256), 0, s, work, eps_inv, wc,
                     vsqrt, n);
  return hipGetLastError();
}

}  // namespace chi0
