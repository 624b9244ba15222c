// The paper's real-axis route for the polarization: transition energies
// binned into a histogram (Eq.(impolf), Eq.(tetw), with a uniform spread of
// each transition standing in for the tetrahedron weights), the
// per-bin weighted Hermitian rank-K updates (the rank-K kernels with gathered
// rows), and the Hilbert transform (Eq.(hilbert)) to imaginary and real
// frequencies.
//
// Binning is deterministic: every pair owns R record slots (R bounds the
// bins one spread can touch), filled in pair order; a counting sort by bin
// (per-chunk counts, a scan, and a one-wave-per-chunk stable scatter) makes
// each bin's records contiguous in pair order, so the rank-K sums run in a
// fixed order.
#include "common.h"
#include "herk_common.h"

namespace chi0 {
namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

// Records of every pair of one block (blockIdx.y): bin (or -1), weight
// w_k * fraction, byte address of the pair's Z row.
__global__ __launch_bounds__(256) void hist_records_kernel(const HistBlock* __restrict__ blocks,
                                                           const HistProb* __restrict__ probs, int R,
                                                           double delta_min, int32_t* __restrict__ rbin,
                                                           double* __restrict__ rw,
                                                           uint64_t* __restrict__ rrow,
                                                           int32_t* nonpositive) {
#pragma clang fp contract(off)
  const HistBlock bd = blocks[blockIdx.y];
  const HistProb pr = probs[bd.prob];
  const int64_t K = static_cast<int64_t>(bd.nocc) * bd.nunocc;
  const double* e = pr.edges;
  const int nb = pr.nbins;
  for (int64_t p = blockIdx.x * 256ll + threadIdx.x; p < K; p += static_cast<int64_t>(gridDim.x) * 256) {
    const int n = static_cast<int>(p / bd.nunocc);
    const int m = static_cast<int>(p - static_cast<int64_t>(n) * bd.nunocc);
    const int64_t slot0 = bd.rec0 + p * R;
    const uint64_t row = reinterpret_cast<uint64_t>(bd.z) + static_cast<uint64_t>(p) * bd.row_bytes;
    int t = 0;
    const double d = bd.eps_unocc[m] - bd.eps_occ[n];
    count_lanes(nonpositive, !(d > 0.0));
    if (d > 0.0 && d >= delta_min) {
      if (pr.sigma == 0.0) {
        if (d >= e[0] && d < e[nb]) {
          int lo = 0, hi = nb;           // largest j with e[j] <= d
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (e[mid] <= d) lo = mid; else hi = mid;
          }
          rbin[slot0] = pr.bin0 + lo;
          rw[slot0] = bd.wk * 1.0;
          rrow[slot0] = row;
          t = 1;
        }
      } else {
        const double wlo = d * (1.0 - pr.sigma), whi = d * (1.0 + pr.sigma);
        const double width = whi - wlo;
        int lo = 0, hi = nb + 1;         // first edge index with e[k] > wlo
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (e[mid] > wlo) hi = mid; else lo = mid + 1;
        }
        for (int j = lo > 0 ? lo - 1 : 0; j < nb && e[j] < whi && t < R; ++j) {
          const double a = wlo > e[j] ? wlo : e[j];
          const double b = whi < e[j + 1] ? whi : e[j + 1];
          if (b > a) {
            rbin[slot0 + t] = pr.bin0 + j;
            rw[slot0 + t] = bd.wk * ((b - a) / width);
            rrow[slot0 + t] = row;
            ++t;
          }
        }
      }
    }
    for (; t < R; ++t) rbin[slot0 + t] = -1;
  }
}

// Records per bin in each chunk of kChunk records: cnt[bin][chunk].
constexpr int kChunk = 16384;

__global__ __launch_bounds__(256) void hist_chunk_count_kernel(const int32_t* __restrict__ rbin, int64_t nrec,
                                                               int nbt, int nchunks, int32_t* __restrict__ cnt) {
  extern __shared__ int32_t lh[];
  for (int b = threadIdx.x; b < nbt; b += 256) lh[b] = 0;
  __syncthreads();
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kChunk;
  for (int i = threadIdx.x; i < kChunk; i += 256) {
    const int64_t r = r0 + i;
    if (r < nrec) {
      const int b = rbin[r];
      if (b >= 0) atomicAdd(&lh[b], 1);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbt; b += 256) cnt[static_cast<int64_t>(b) * nchunks + blockIdx.x] = lh[b];
}

// One workgroup: cnt[bin][chunk] becomes the first sorted position of the
// bin's records of that chunk; off[bin] the bin's first position, off[nbt]
// the number of records kept.
__global__ __launch_bounds__(1024) void hist_scan_kernel(int32_t* __restrict__ cnt, int nbt, int nchunks,
                                                         int64_t* __restrict__ off) {
  __shared__ int64_t part[1024];
  const int per = (nbt + 1023) / 1024;
  const int b0 = threadIdx.x * per;
  int64_t local = 0;
  for (int b = b0; b < b0 + per && b < nbt; ++b) {
    int64_t s = 0;
    for (int c = 0; c < nchunks; ++c) {
      const int64_t i = static_cast<int64_t>(b) * nchunks + c;
      const int v = cnt[i];
      cnt[i] = static_cast<int32_t>(s);
      s += v;
    }
    off[b] = s;                          // bin total for now
    local += s;
  }
  part[threadIdx.x] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int i = 0; i < 1024; ++i) {
      const int64_t v = part[i];
      part[i] = run;
      run += v;
    }
    off[nbt] = run;
  }
  __syncthreads();
  int64_t run = part[threadIdx.x];
  for (int b = b0; b < b0 + per && b < nbt; ++b) {
    const int64_t tot = off[b];
    off[b] = run;
    for (int c = 0; c < nchunks; ++c) cnt[static_cast<int64_t>(b) * nchunks + c] += static_cast<int32_t>(run);
    run += tot;
  }
}

// Stable scatter, one wave per chunk: within each group of 64 records a
// record's rank among the group's records of the same bin comes from the
// other lanes' bins (read lane by lane); a per-bin cursor in LDS advances
// after each group.
template <class W>
__global__ __launch_bounds__(64) void hist_scatter_kernel(const int32_t* __restrict__ rbin,
                                                          const double* __restrict__ rw,
                                                          const uint64_t* __restrict__ rrow, int64_t nrec,
                                                          int nbt, int nchunks, const int32_t* __restrict__ cnt,
                                                          uint64_t* __restrict__ srow, W* __restrict__ sw) {
  extern __shared__ int32_t cur[];
  const int lane = threadIdx.x;
  for (int b = lane; b < nbt; b += 64) cur[b] = cnt[static_cast<int64_t>(b) * nchunks + blockIdx.x];
  __syncthreads();
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kChunk;
  for (int g = 0; g < kChunk; g += 64) {
    const int64_t r = r0 + g + lane;
    const int b = r < nrec ? rbin[r] : -1;
    int rank = 0, later = 0;
#pragma unroll
    for (int k = 0; k < 64; ++k) {
      const int bk = __builtin_amdgcn_readlane(b, k);
      const bool same = bk == b;
      rank += (same && k < lane) ? 1 : 0;
      later += (same && k > lane) ? 1 : 0;
    }
    int pos = 0;
    if (b >= 0) pos = cur[b] + rank;   // every lane reads before any lane writes
    __builtin_amdgcn_wave_barrier();
    if (b >= 0) {
      srow[pos] = rrow[r];
      sw[pos] = static_cast<W>(rw[r]);
      if (later == 0) cur[b] = pos + 1;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Hilbert coefficients of one problem's non-empty bins: rows 0 .. nimag-1
// for the imaginary frequencies (real), then the real frequencies.
__global__ __launch_bounds__(256) void hist_coeff_kernel(const HilbertProb* __restrict__ hp, int nprob) {
  const HilbertProb pr = hp[blockIdx.y];
  const int nout = pr.nimag + pr.nreal;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < nout * pr.nbins_used; e += gridDim.x * 256) {
    const int o = e / pr.nbins_used;
    const int k = e - o * pr.nbins_used;
    const int j = pr.bins[k];
    const double lo = pr.edges[j], hi = pr.edges[j + 1], h = hi - lo;
    double cr, ci = 0.0;
    if (o < pr.nimag) {
      const double w = pr.omega[o];
      cr = log1p(h * (hi + lo) / (lo * lo + w * w)) / h;
    } else {
      const double w = pr.omega_re[o - pr.nimag];
      const bool inside = w > lo && w < hi;
      const double near = inside ? log(fabs(hi - w)) - log(fabs(lo - w)) : log1p(h / (lo - w));
      const double far = log1p(h / (lo + w));
      cr = (near + far) / h;
      ci = inside ? kPi / h : 0.0;
    }
    pr.coeff[e] = double2{cr, ci};
  }
}

// out_o[I][J] = sum_k coeff[o][k] hist_k[I][J] over the problem's non-empty
// bins, up to kOut outputs per pass; HBM-bound (every bin is read once per
// pass, coalesced).
constexpr int kOut = 16;

__global__ __launch_bounds__(256) void hilbert_kernel(const HilbertProb* __restrict__ hp, int o0) {
  const HilbertProb pr = hp[blockIdx.y];
  const int nout = pr.nimag + pr.nreal;
  const int64_t n2 = static_cast<int64_t>(pr.npb) * pr.npb;
  const int no = nout - o0 < kOut ? nout - o0 : kOut;
  if (no <= 0) return;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < n2; e += static_cast<int64_t>(gridDim.x) * 256) {
    double ar[kOut], ai[kOut];
#pragma unroll
    for (int o = 0; o < kOut; ++o) ar[o] = ai[o] = 0.0;
    for (int k = 0; k < pr.nbins_used; ++k) {
      const double2 v = pr.hist[static_cast<int64_t>(pr.slots[k]) * n2 + e];
#pragma unroll
      for (int o = 0; o < kOut; ++o) {
        if (o < no) {
          const double2 c = pr.coeff[static_cast<int64_t>(o0 + o) * pr.nbins_used + k];
          ar[o] += c.x * v.x - c.y * v.y;
          ai[o] += c.x * v.y + c.y * v.x;
        }
      }
    }
#pragma unroll
    for (int o = 0; o < kOut; ++o) {
      if (o < no) {
        const int oo = o0 + o;
        double2* dst = oo < pr.nimag ? pr.out + static_cast<int64_t>(oo) * n2
                                     : pr.out_re + static_cast<int64_t>(oo - pr.nimag) * n2;
        dst[e] = double2{ar[o], ai[o]};
      }
    }
  }
}

__global__ __launch_bounds__(256) void hist_zero_kernel(double2* const* __restrict__ mats, int64_t n2) {
  double2* m = mats[blockIdx.y];
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < n2; e += static_cast<int64_t>(gridDim.x) * 256)
    m[e] = double2{0.0, 0.0};
}

}  // namespace

int hist_chunk() { return kChunk; }

hipError_t hist_records_launch(const HistBlock* blocks, const HistProb* probs, int nblocks, int64_t max_pairs,
                               int R, double delta_min, int32_t* rbin, double* rw, uint64_t* rrow,
                               int32_t* nonpositive, hipStream_t s) {
  if (nblocks <= 0 || max_pairs <= 0) return hipSuccess;
  int64_t gx = (max_pairs + 255) / 256;
  if (gx > 4096) gx = 4096;
  for (int b0 = 0; b0 < nblocks; b0 += 65535) {
    const int nb = nblocks - b0 < 65535 ? nblocks - b0 : 65535;
    hipLaunchKernelGGL(hist_records_kernel, dim3(static_cast<unsigned>(gx), nb), dim3(256), 0, s, blocks + b0,
                       probs, R, delta_min, rbin, rw, rrow, nonpositive);
  }
  return hipGetLastError();
}

hipError_t hist_sort_launch(const int32_t* rbin, const double* rw, const uint64_t* rrow, int64_t nrec, int nbt,
                            int32_t* cnt, int64_t* off, uint64_t* srow, void* sw, bool f64, hipStream_t s) {
  const int nchunks = static_cast<int>((nrec + kChunk - 1) / kChunk);
  if (nchunks <= 0) {
    hipLaunchKernelGGL(hist_scan_kernel, dim3(1), dim3(1024), 0, s, cnt, nbt, 0, off);
    return hipGetLastError();
  }
  const size_t lds = static_cast<size_t>(nbt) * sizeof(int32_t);
  hipLaunchKernelGGL(hist_chunk_count_kernel, dim3(nchunks), dim3(256), lds, s, rbin, nrec, nbt, nchunks, cnt);
  hipLaunchKernelGGL(hist_scan_kernel, dim3(1), dim3(1024), 0, s, cnt, nbt, nchunks, off);
  if (f64)
    hipLaunchKernelGGL(hist_scatter_kernel<double>, dim3(nchunks), dim3(64), lds, s, rbin, rw, rrow, nrec, nbt,
                       nchunks, cnt, srow, static_cast<double*>(sw));
  else
    hipLaunchKernelGGL(hist_scatter_kernel<float>, dim3(nchunks), dim3(64), lds, s, rbin, rw, rrow, nrec, nbt,
                       nchunks, cnt, srow, static_cast<float*>(sw));
  return hipGetLastError();
}

hipError_t hilbert_launch(const HilbertProb* hp, int nprob, int max_out, int max_bins, int64_t max_n2,
                          hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  int64_t gc = (static_cast<int64_t>(max_out) * max_bins + 255) / 256;
  if (gc < 1) gc = 1;
  if (gc > 1024) gc = 1024;
  hipLaunchKernelGGL(hist_coeff_kernel, dim3(static_cast<unsigned>(gc), nprob), dim3(256), 0, s, hp, nprob);
  int64_t gx = (max_n2 + 255) / 256;
  if (gx > 8192) gx = 8192;
  for (int o0 = 0; o0 < max_out; o0 += kOut)
    hipLaunchKernelGGL(hilbert_kernel, dim3(static_cast<unsigned>(gx), nprob), dim3(256), 0, s, hp, o0);
  return hipGetLastError();
}

hipError_t hist_zero_launch(double2* const* mats, int nmats, int64_t n2, hipStream_t s) {
  if (nmats <= 0) return hipSuccess;
  int64_t gx = (n2 + 255) / 256;
  if (gx > 1024) gx = 1024;
  for (int m0 = 0; m0 < nmats; m0 += 65535) {
    const int nm = nmats - m0 < 65535 ? nmats - m0 : 65535;
    hipLaunchKernelGGL(hist_zero_kernel, dim3(static_cast<unsigned>(gx), nm), dim3(256), 0, s, mats + m0, n2);
  }
  return hipGetLastError();
}

}  // namespace chi0
