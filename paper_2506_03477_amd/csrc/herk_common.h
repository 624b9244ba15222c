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

// Adds the number of lanes with `bad` set to *count: one vector-memory
// atomic per wave, from the lowest such lane.  Used to report pairs with
// D <= 0, which the polarization sum does not define.
__device__ __forceinline__ void count_lanes(int32_t* count, bool bad) {
  const unsigned long long m = __ballot(bad);
  if (m == 0ull) return;
  if (static_cast<int>(__lane_id()) == __ffsll(static_cast<long long>(m)) - 1)
    atomicAdd(count, static_cast<int32_t>(__popcll(m)));
}

// Read-only tables are read through the constant address space: they do not
// change during a launch, so uniform reads become scalar loads that do not
// wait behind the vector memory traffic.
template <class X>
__device__ __forceinline__ X ld_const(const X* p, int i) {
  return ((const X __attribute__((address_space(4)))*)(p))[i];
}

// A unit and a problem descriptor read field by field through the scalar
// cache (uniform values in scalar registers).
__device__ __forceinline__ Unit ld_unit(const Unit* units, int idx) {
  const Unit* p = units + idx;
  Unit u;
  u.prob = ld_const(&p->prob, 0);
  u.iw = ld_const(&p->iw, 0);
  u.tp = ld_const(&p->tp, 0);
  u.tq = ld_const(&p->tq, 0);
  u.b0 = ld_const(&p->b0, 0);
  u.p0 = ld_const(&p->p0, 0);
  u.b1 = ld_const(&p->b1, 0);
  u.p1 = ld_const(&p->p1, 0);
  u.slot = ld_const(&p->slot, 0);
  u.nw = ld_const(&p->nw, 0);
  u.wstride = ld_const(&p->wstride, 0);
  u.pad = 0;
  return u;
}

__device__ __forceinline__ ProbDesc ld_prob(const ProbDesc* probs, int idx) {
  const ProbDesc* p = probs + idx;
  ProbDesc d;
  d.chi0 = ld_const(&p->chi0, 0);
  d.omega = ld_const(&p->omega, 0);
  d.wts = ld_const(&p->wts, 0);
  d.ktot = ld_const(&p->ktot, 0);
  d.npb = ld_const(&p->npb, 0);
  d.nomega = ld_const(&p->nomega, 0);
  d.flush = ld_const(&p->flush, 0);
  d.pad = 0;
  return d;
}

__device__ __forceinline__ int block_pairs(const BlockDesc* blocks, int b) {
  const BlockDesc* bp = blocks + b;
  const int* f = reinterpret_cast<const int*>(&bp->nocc);
  return ld_const(f, 0) * ld_const(f, 1);
}

// Pair cursor over a unit's range: block b, stage start p0, end of the
// block's part of the range pend.  Uniform across the workgroup.
struct Cursor {
  int b;
  int p0;
  int pend;
};

__device__ __forceinline__ bool cursor_first(const Unit& u, const BlockDesc* blocks, Cursor& c) {
  for (int b = u.b0; b <= u.b1; ++b) {
    const int beg = (b == u.b0) ? u.p0 : 0;
    const int end = (b == u.b1) ? u.p1 : block_pairs(blocks, b);
    if (beg < end) {
      c.b = b;
      c.p0 = beg;
      c.pend = end;
      return true;
    }
  }
  return false;
}

// Advances c by one stage of KC pairs; returns false (leaving c on the last
// stage) when the unit has no further stage.
template <int KC>
__device__ __forceinline__ bool cursor_next(const Unit& u, const BlockDesc* blocks, Cursor& c) {
  if (c.p0 + KC < c.pend) {
    c.p0 += KC;
    return true;
  }
  for (int b = c.b + 1; b <= u.b1; ++b) {
    const int end = (b == u.b1) ? u.p1 : block_pairs(blocks, b);
    if (0 < end) {
      c.b = b;
      c.p0 = 0;
      c.pend = end;
      return true;
    }
  }
  return false;
}

// Host-side dispatch tables of the three precision paths.
int herk_fp64_tile_count();
TileConfig herk_fp64_tile(int idx);
hipError_t herk_fp64_launch(int idx, const HerkArgs& a, int nwg, hipStream_t s, bool gather);
int herk_fp64_max_wg_per_cu(int idx);

int herk_fp32_tile_count();
TileConfig herk_fp32_tile(int idx);
hipError_t herk_fp32_launch(int idx, const HerkArgs& a, int nwg, hipStream_t s);
int herk_fp32_max_wg_per_cu(int idx);

int herk_bf16x3_tile_count();
TileConfig herk_bf16x3_tile(int idx);
hipError_t herk_bf16x3_launch(int idx, const HerkArgs& a, int nwg, hipStream_t s, bool gather);
int herk_bf16x3_max_wg_per_cu(int idx);
// Register-direct BF16x3 kernel (P side pre-split): 256 x 128 workgroup
// units, or 128 x 64 units on one work list per wave.
hipError_t herk_bf16x3_direct_launch(bool lolo, bool hint, bool wave_units, const HerkArgs& a,
                                     int nwg, hipStream_t s);
int herk_bf16x3_direct_max_wg_per_cu();
// BF16x3 kernel on frequency-group units (128 x 64 tiles, up to four
// frequencies per workgroup, operands staged once in LDS).
hipError_t herk_bf16x3_wgroup_launch(bool lolo, int variant, const HerkArgs& a, int nwg,
                                     hipStream_t s);
int herk_bf16x3_wgroup_max_wg_per_cu();
// FP32 contraction on the same frequency-group units.
hipError_t herk_fp32_wgroup_launch(const HerkArgs& a, int nwg, hipStream_t s);
int herk_fp32_wgroup_max_wg_per_cu();

}  // namespace chi0
