// Dielectric step on gfx950: eps = 1 - diag(s) chi0 diag(s)
// (Eq.(dielectricfunction)), its FP64 inverse by blocked Gauss-Jordan
// elimination with partial pivoting (Algorithm "hrcxq" inverts eps for every
// frequency), and W^c = diag(s) (eps^{-1} - 1) diag(s) (Eq.(wc)).
//
// The matrices of all frequencies are processed together (the batch index is
// the last grid dimension).  Gauss-Jordan works in place on a workspace copy:
// for each panel of nb columns
//   1. gj_panel: the nb elimination steps restricted to the n x nb panel,
//      pivot = entry of largest modulus at or below the diagonal; the panel
//      ends up holding the combined elimination columns C;
//   2. gj_swap_extract: the panel's row interchanges applied, in order, to
//      every other column; the nb pivot rows copied out (W);
//   3. gj_update: every other column j gets X[:, j] = X[:, j] (rows outside
//      the panel) + C W[:, j]  -- a complex FP64 GEMM on the matrix cores.
// Finally the columns are unscrambled (the interchanges applied in reverse
// order to the column index).
#include "common.h"

namespace chi0 {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kPanel = 32;     // nb
constexpr int kPanelThreads = 1024;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

__global__ __launch_bounds__(256) void dielectric_build_kernel(
    const double2* __restrict__ chi0, const double* __restrict__ s,
    double2* __restrict__ work, double2* __restrict__ eps_out, int n, size_t total) {
#pragma clang fp contract(off)
  const size_t nn = static_cast<size_t>(n) * n;
  for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const size_t r = e % nn;
    const int i = static_cast<int>(r / n);
    const int j = static_cast<int>(r - static_cast<size_t>(i) * n);
    const double2 c = chi0[e];
    const double si = s[i], sj = s[j];
    double2 v;
    v.x = (i == j ? 1.0 : 0.0) - (si * c.x) * sj;
    v.y = -((si * c.y) * sj);
    work[e] = v;
    if (eps_out) eps_out[e] = v;
  }
}

__global__ __launch_bounds__(kPanelThreads) void gj_panel_kernel(
    double2* __restrict__ work, int n, int k0, int nb, int32_t* __restrict__ piv,
    int32_t* __restrict__ status) {
  constexpr int NW = kPanelThreads / 64;
  __shared__ double red_v[NW];
  __shared__ int red_i[NW];
  __shared__ double2 rowk[kPanel];
  __shared__ double2 s_d;
  __shared__ int s_p;
  const int mat = blockIdx.x;
  double2* S = work + static_cast<size_t>(mat) * n * n;
  int32_t* pv = piv + static_cast<size_t>(mat) * n;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;

  for (int kk = 0; kk < nb; ++kk) {
    const int k = k0 + kk;
    // 1. pivot: largest |S[i][k]|^2 over i >= k (smallest index on ties)
    double best = -1.0;
    int bi = n;
    for (int i = k + tid; i < n; i += kPanelThreads) {
      const double2 v = S[static_cast<size_t>(i) * n + k];
      const double m2 = v.x * v.x + v.y * v.y;
      if (m2 > best) {
        best = m2;
        bi = i;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      red_v[wave] = best;
      red_i[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double bv = red_v[0];
      int bix = red_i[0];
      for (int w = 1; w < NW; ++w)
        if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < bix)) {
          bv = red_v[w];
          bix = red_i[w];
        }
      if (bix >= n) bix = k;
      if (!(bv > 0.0)) status[0] = 1;
      s_p = bix;
      pv[k] = bix;
    }
    __syncthreads();
    const int p = s_p;
    // 2. interchange rows k and p inside the panel
    if (p != k && tid < nb) {
      const size_t a0 = static_cast<size_t>(k) * n + k0 + tid;
      const size_t a1 = static_cast<size_t>(p) * n + k0 + tid;
      const double2 t0 = S[a0];
      S[a0] = S[a1];
      S[a1] = t0;
    }
    __syncthreads();
    if (tid == 0) {
      const double2 pvt = S[static_cast<size_t>(k) * n + k];
      const double den = pvt.x * pvt.x + pvt.y * pvt.y;
      s_d = double2{pvt.x / den, -pvt.y / den};
    }
    __syncthreads();
    // 3. scale the pivot row (S[k][k] <- 1 first, so it ends up as 1/pivot)
    if (tid < nb) {
      const size_t a0 = static_cast<size_t>(k) * n + k0 + tid;
      const double2 v = (k0 + tid == k) ? double2{1.0, 0.0} : S[a0];
      const double2 r = cmul(v, s_d);
      rowk[tid] = r;
      S[a0] = r;
    }
    __syncthreads();
    // 4. eliminate column k from every other row (S[i][k] <- 0 first)
    for (int i = tid; i < n; i += kPanelThreads) {
      if (i == k) continue;
      double2* Si = S + static_cast<size_t>(i) * n + k0;
      const double2 f = Si[kk];
      for (int t = 0; t < nb; ++t) {
        double2 x = (t == kk) ? double2{0.0, 0.0} : Si[t];
        const double2 fr = cmul(f, rowk[t]);
        x.x -= fr.x;
        x.y -= fr.y;
        Si[t] = x;
      }
    }
    __syncthreads();
  }
}

// Register-resident panel for n <= 2048 (R = rows per thread, 1024 threads).
// The panel's nb columns are processed as sub-panels of 8: a sub-panel lives
// in registers (thread t owns rows t + 1024 r) through its 8 elimination
// steps (pivot search by wave shuffles, row interchange and pivot-row
// broadcast through LDS); it is then stored and, for nb > 8, its combined
// transformation is applied to the other columns of the panel as a rank-8
// update:
//   y = (interchanges) x;   x <- y (rows outside the sub-panel) + C y[sub-panel rows].
// The inverse launches it one sub-panel at a time (nb <= 8) and applies each
// sub-panel with the interchange and update kernels restricted to the panel,
// which use every CU.
template <int R>
__global__ __launch_bounds__(kPanelThreads) void gj_panel_reg_kernel(
    double2* __restrict__ work, int n, int k0, int nb, int32_t* __restrict__ piv,
    int32_t* __restrict__ status) {
  constexpr int NT = kPanelThreads;
  constexpr int NW = NT / 64;
  constexpr int SB = 8;  // sub-panel width
  __shared__ double red_v[NW];
  __shared__ int red_i[NW];
  __shared__ double2 swapP[SB], swapC[SB], rowk[SB];
  __shared__ double2 wsub[SB][kPanel];
  const int mat = blockIdx.x;
  double2* S = work + static_cast<size_t>(mat) * n * n;
  int32_t* pv = piv + static_cast<size_t>(mat) * n;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;

  for (int j0 = 0; j0 < nb; j0 += SB) {
    const int sw = min(SB, nb - j0);     // width of this sub-panel
    const int c0 = k0 + j0;
    double2 v[R][SB];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + NT * r;
#pragma unroll
      for (int t = 0; t < SB; ++t)
        v[r][t] = (i < n && t < sw) ? S[static_cast<size_t>(i) * n + c0 + t] : double2{0.0, 0.0};
    }
    for (int s = 0; s < sw; ++s) {
      const int c = c0 + s;
      // 1. pivot: largest |x|^2 in column c over rows >= c (smallest index on ties)
      double best = -1.0;
      int bi = n;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = tid + NT * r;
        double2 x = double2{0.0, 0.0};
#pragma unroll
        for (int t = 0; t < SB; ++t)
          if (t == s) x = v[r][t];
        const double m2 = x.x * x.x + x.y * x.y;
        if (i >= c && i < n && m2 > best) {
          best = m2;
          bi = i;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > best || (ov == best && oi < bi)) {
          best = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        red_v[wave] = best;
        red_i[wave] = bi;
      }
      __syncthreads();
      double bv = red_v[0];
      int p = red_i[0];
      for (int w = 1; w < NW; ++w)
        if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < p)) {
          bv = red_v[w];
          p = red_i[w];
        }
      if (p >= n) p = c;
      if (tid == 0) {
        pv[c] = p;
        if (!(bv > 0.0)) status[0] = 1;
      }
      // 2. interchange rows c and p (sub-panel registers)
      const int oc = c % NT, rc = c / NT;
      const int op = p % NT, rp = p / NT;
      if (p != c) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (tid == op && r == rp)
#pragma unroll
            for (int t = 0; t < SB; ++t) swapP[t] = v[r][t];
          if (tid == oc && r == rc)
#pragma unroll
            for (int t = 0; t < SB; ++t) swapC[t] = v[r][t];
        }
      }
      __syncthreads();
      if (p != c) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (tid == oc && r == rc)
#pragma unroll
            for (int t = 0; t < SB; ++t) v[r][t] = swapP[t];
          if (tid == op && r == rp)
#pragma unroll
            for (int t = 0; t < SB; ++t) v[r][t] = swapC[t];
        }
      }
      // 3. scale the pivot row (entry s <- 1 first, so it ends up 1/pivot)
      if (tid == oc) {
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (r == rc) {
            double2 pvt = double2{0.0, 0.0};
#pragma unroll
            for (int t = 0; t < SB; ++t)
              if (t == s) pvt = v[r][t];
            const double den = pvt.x * pvt.x + pvt.y * pvt.y;
            const double2 d = double2{pvt.x / den, -pvt.y / den};
#pragma unroll
            for (int t = 0; t < SB; ++t) {
              const double2 x = (t == s) ? double2{1.0, 0.0} : v[r][t];
              v[r][t] = cmul(x, d);
              rowk[t] = v[r][t];
            }
          }
      }
      __syncthreads();
      // 4. eliminate column c from every other row (entry s <- 0 first)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = tid + NT * r;
        if (i == c || i >= n) continue;
        double2 f = double2{0.0, 0.0};
#pragma unroll
        for (int t = 0; t < SB; ++t)
          if (t == s) f = v[r][t];
#pragma unroll
        for (int t = 0; t < SB; ++t) {
          double2 x = (t == s) ? double2{0.0, 0.0} : v[r][t];
          const double2 fr = cmul(f, rowk[t]);
          x.x -= fr.x;
          x.y -= fr.y;
          v[r][t] = x;
        }
      }
    }
    // store the sub-panel
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + NT * r;
      if (i < n)
#pragma unroll
        for (int t = 0; t < SB; ++t)
          if (t < sw) S[static_cast<size_t>(i) * n + c0 + t] = v[r][t];
    }
    // apply the sub-panel to the other panel columns
    const int nother = nb - sw;
    if (nother > 0) {
      if (tid < nother) {  // interchanges, in order, one column per thread
        const int col = k0 + (tid < j0 ? tid : tid + sw);
        for (int s = 0; s < sw; ++s) {
          const int c = c0 + s;
          const int p = pv[c];
          if (p != c) {
            const size_t a0 = static_cast<size_t>(c) * n + col;
            const size_t a1 = static_cast<size_t>(p) * n + col;
            const double2 t0 = S[a0];
            S[a0] = S[a1];
            S[a1] = t0;
          }
        }
      }
      __syncthreads();
      if (tid < SB * nother) {
        const int b = tid / nother;
        const int o = tid % nother;
        const int col = k0 + (o < j0 ? o : o + sw);
        wsub[b][o] = (b < sw) ? S[static_cast<size_t>(c0 + b) * n + col] : double2{0.0, 0.0};
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = tid + NT * r;
        if (i >= n) continue;
        const bool inb = i >= c0 && i < c0 + sw;
        for (int o = 0; o < nother; ++o) {
          const int col = k0 + (o < j0 ? o : o + sw);
          const size_t ad = static_cast<size_t>(i) * n + col;
          double2 x = inb ? double2{0.0, 0.0} : S[ad];
#pragma unroll
          for (int b = 0; b < SB; ++b) {
            const double2 fr = cmul(v[r][b], wsub[b][o]);
            x.x += fr.x;
            x.y += fr.y;
          }
          S[ad] = x;
        }
      }
      __syncthreads();
    }
  }
}

// Columns j in [jlo, jhi) outside the panel [k0, k0 + nb): the panel's row
// interchanges, in order, then its pivot rows copied to wrow.
__global__ __launch_bounds__(256) void gj_swap_extract_kernel(
    double2* __restrict__ work, double2* __restrict__ wrow, int n, int k0, int nb,
    const int32_t* __restrict__ piv, int jlo, int jhi) {
  const int mat = blockIdx.y;
  const int j = jlo + blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= jhi || (j >= k0 && j < k0 + nb)) return;
  double2* S = work + static_cast<size_t>(mat) * n * n;
  const int32_t* pv = piv + static_cast<size_t>(mat) * n;
  double2* W = wrow + static_cast<size_t>(mat) * kPanel * n;
  for (int b = 0; b < nb; ++b) {
    const int r = k0 + b;
    const int p = pv[r];
    if (p != r) {
      const size_t a0 = static_cast<size_t>(r) * n + j;
      const size_t a1 = static_cast<size_t>(p) * n + j;
      const double2 t0 = S[a0];
      S[a0] = S[a1];
      S[a1] = t0;
    }
  }
  for (int b = 0; b < nb; ++b) W[static_cast<size_t>(b) * n + j] = S[static_cast<size_t>(k0 + b) * n + j];
}

// X[i][j] = (i in panel rows ? 0 : X[i][j]) + sum_b C[i][b] W[b][j], j in
// [jlo, jhi) outside the panel.  64 x 64 complex output tile per workgroup
// (tile columns from the one holding jlo), 4 waves of 32 x 32, FP64 16x16x4
// MFMA with (re, im) stacked along the contraction index:
//   Re += [Cr, Ci] . [Wr, -Wi],  Im += [Cr, Ci] . [Wi, Wr].
__global__ __launch_bounds__(256) void gj_update_kernel(
    double2* __restrict__ work, const double2* __restrict__ wrow, int n, int k0, int nb, int jlo,
    int jhi) {
  constexpr int T = 64;
  __shared__ double2 sC[kPanel][T];
  __shared__ double2 sW[kPanel][T];
  const int mat = blockIdx.z;
  const int i0 = blockIdx.y * T;
  const int j0 = (jlo / T) * T + blockIdx.x * T;
  if (j0 + T > k0 && j0 < k0 + nb && j0 >= k0 && j0 + T <= k0 + nb) return;  // inside panel
  double2* S = work + static_cast<size_t>(mat) * n * n;
  const double2* W = wrow + static_cast<size_t>(mat) * kPanel * n;
  const int tid = threadIdx.x;
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
        const bool keep = i < n && j >= jlo && j < jhi && !(j >= k0 && j < k0 + nb) &&
                          !(i >= k0 && i < k0 + nb);
        xo[a][c][r] = keep ? S[static_cast<size_t>(i) * n + j] : double2{0.0, 0.0};
      }
  for (int e = tid; e < kPanel * T; e += 256) {
    const int b = e % kPanel;
    const int i = e / kPanel;
    double2 v = {0.0, 0.0};
    if (b < nb && i0 + i < n) v = S[static_cast<size_t>(i0 + i) * n + k0 + b];
    sC[b][i ^ (b & 15)] = v;   // rows XOR-swizzled by b: the 32 b of one row spread over the banks
    const int bj = e / T;
    const int jj = e % T;
    double2 w = {0.0, 0.0};
    if (bj < nb && j0 + jj < n) w = W[static_cast<size_t>(bj) * n + j0 + jj];
    sW[bj][jj] = w;
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
  for (int st = 0; st < kPanel / 2; ++st) {
    const int b = 2 * st + prr;
    double av[2], wr_[2], wi_[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const double2 x = sC[b][wr * 32 + a * 16 + (m ^ (b & 15))];
      av[a] = isim ? x.y : x.x;
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double2 y = sW[b][wc * 32 + c * 16 + m];
      wr_[c] = isim ? -y.y : y.x;
      wi_[c] = isim ? y.x : y.y;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        accR[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], wr_[c], accR[a][c], 0, 0, 0);
        accI[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], wi_[c], accI[a][c], 0, 0, 0);
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
        if (i >= n || j < jlo || j >= jhi || (j >= k0 && j < k0 + nb)) continue;
        const size_t ad = static_cast<size_t>(i) * n + j;
        S[ad] = double2{xo[a][c][r].x + accR[a][c][r], xo[a][c][r].y + accI[a][c][r]};
      }
}

__global__ void gj_perm_kernel(const int32_t* __restrict__ piv, int32_t* __restrict__ perm, int n) {
  const int mat = blockIdx.x;
  if (threadIdx.x != 0) return;
  const int32_t* pv = piv + static_cast<size_t>(mat) * n;
  int32_t* ix = perm + static_cast<size_t>(mat) * n;
  for (int j = 0; j < n; ++j) ix[j] = j;
  for (int k = n - 1; k >= 0; --k) {
    const int p = pv[k];
    const int32_t t = ix[k];
    ix[k] = ix[p];
    ix[p] = t;
  }
}

__global__ __launch_bounds__(256) void gj_finish_kernel(
    const double2* __restrict__ work, double2* __restrict__ eps_inv, double2* __restrict__ wc,
    const double* __restrict__ s, const int32_t* __restrict__ perm, int n) {
#pragma clang fp contract(off)
  const int mat = blockIdx.z;
  const int i = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const size_t base = static_cast<size_t>(mat) * n * n + static_cast<size_t>(i) * n;
  const int src = perm[static_cast<size_t>(mat) * n + j];
  const double2 x = work[base + src];
  eps_inv[base + j] = x;
  if (wc) {
    const double si = s[i], sj = s[j];
    double2 w;
    w.x = (si * (x.x - (i == j ? 1.0 : 0.0))) * sj;
    w.y = (si * x.y) * sj;
    wc[base + j] = w;
  }
}

}  // namespace

int gj_panel_width() { return kPanel; }

hipError_t dielectric_build_launch(const double2* chi0, const double* vsqrt, double2* work,
                                   double2* eps_out, int n, int nomega, hipStream_t s) {
  const size_t total = static_cast<size_t>(n) * n * nomega;
  size_t nblk = (total + 255) / 256;
  if (nblk > 65536) nblk = 65536;
  hipLaunchKernelGGL(dielectric_build_kernel, dim3(static_cast<unsigned>(nblk)), dim3(256), 0, s,
                     chi0, vsqrt, work, eps_out, n, total);
  return hipGetLastError();
}

hipError_t gj_panel_launch(double2* work, int n, int nomega, int k0, int nb, int32_t* piv,
                           int32_t* status, hipStream_t s) {
  if (n <= kPanelThreads)
    hipLaunchKernelGGL(gj_panel_reg_kernel<1>, dim3(nomega), dim3(kPanelThreads), 0, s, work, n,
                       k0, nb, piv, status);
  else if (n <= 2 * kPanelThreads)
    hipLaunchKernelGGL(gj_panel_reg_kernel<2>, dim3(nomega), dim3(kPanelThreads), 0, s, work, n,
                       k0, nb, piv, status);
  else
    hipLaunchKernelGGL(gj_panel_kernel, dim3(nomega), dim3(kPanelThreads), 0, s, work, n, k0, nb,
                       piv, status);
  return hipGetLastError();
}

int gj_subpanel_width() { return 8; }

hipError_t gj_swap_extract_launch(double2* work, double2* wrow, int n, int nomega, int k0, int nb,
                                  const int32_t* piv, int jlo, int jhi, hipStream_t s) {
  if (jhi <= jlo) return hipSuccess;
  hipLaunchKernelGGL(gj_swap_extract_kernel, dim3((jhi - jlo + 255) / 256, nomega), dim3(256), 0, s,
                     work, wrow, n, k0, nb, piv, jlo, jhi);
  return hipGetLastError();
}

hipError_t gj_update_launch(double2* work, const double2* wrow, int n, int nomega, int k0, int nb,
                            int jlo, int jhi, hipStream_t s) {
  if (jhi <= jlo) return hipSuccess;
  const int nt = (n + 63) / 64;
  const int ntj = (jhi - 1) / 64 - jlo / 64 + 1;
  hipLaunchKernelGGL(gj_update_kernel, dim3(ntj, nt, nomega), dim3(256), 0, s, work, wrow, n, k0,
                     nb, jlo, jhi);
  return hipGetLastError();
}

hipError_t gj_finish_launch(const double2* work, double2* eps_inv, double2* wc,
                            const double* vsqrt, const int32_t* piv, int32_t* perm, int n,
                            int nomega, hipStream_t s) {
  hipLaunchKernelGGL(gj_perm_kernel, dim3(nomega), dim3(64), 0, s, piv, perm, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gj_finish_kernel, dim3((n + 255) / 256, n, nomega), dim3(256), 0, s, work,
                     eps_inv, wc, vsqrt, perm, n);
  return hipGetLastError();
}

}  // namespace chi0
