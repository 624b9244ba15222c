// libchi0 host library: C ABI, argument validation, work planning, workspace,
// hipGraph cache, kernel timing and the tile autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <queue>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/chi0.h"
#include "common.h"

using namespace chi0;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(CHI0_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

// Device buffer that only grows.
struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  int reserve(size_t bytes, uint64_t* gen) {
    if (bytes <= n) return CHI0_OK;
    if (p) {
      hipDeviceSynchronize();
      hipFree(p);
      p = nullptr;
      n = 0;
    }
    size_t want = std::max(bytes, static_cast<size_t>(256));
    if (hipMalloc(&p, want) != hipSuccess) {
      hipGetLastError();
      p = nullptr;
      return fail(CHI0_ENOMEM, "device allocation of %zu bytes failed", want);
    }
    n = want;
    if (gen) ++*gen;
    return CHI0_OK;
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    n = 0;
  }
};

struct Plan {
  int kind = 0;
  int tile_idx = 0;
  TileConfig tc{};
  int nwg = 0;
  int nunits = 0;
  int64_t nslots = 0;
  int njobs = 0;
  bool round_robin = false;    // units dealt round-robin (equal costs)
  int nblocks_total = 0;
  int nprob = 0;
  DevBuf d_units, d_wg_off, d_wg_units, d_jobs, d_blocks, d_probs;
  // graph per accumulate flag, valid for workspace generation graph_gen
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  uint64_t graph_gen[2] = {0, 0};
  ~Plan() {
    for (auto& g : graph)
      if (g) hipGraphExecDestroy(g);
    d_units.release();
    d_wg_off.release();
    d_wg_units.release();
    d_jobs.release();
    d_blocks.release();
    d_probs.release();
  }
};

}  // namespace

struct chi0_ctx {
  int device = 0;
  int ncu = 0;
  DevBuf partials;
  DevBuf wts;           // pair weights of the current call
  DevBuf zsplit;        // pre-split P-side planes of the current call
  DevBuf sync_prog;     // per-workgroup progress words of the XCD lockstep
  DevBuf gj_work, gj_wrow, gj_piv, gj_perm;
  DevBuf hpd_p, hpd_c, hpd_dinv;  // HPD inverse: kept panel, new panel, D^{-1}
  DevBuf sigc_tab, sigc_wt, sigc_zw, sigc_part, sigc_acc, sigc_split;  // correlation self-energy
  DevBuf hist_tab, hist_rec, hist_sorted, hist_cnt, hist_mats, hist_coeff;  // histogram route
  int64_t* hist_off_host = nullptr;  // pinned copy of the bin offsets
  size_t hist_off_host_n = 0;
  std::unique_ptr<Plan> gather_plan;  // plan of the last gathered (histogram) call
  std::string gather_key;
  int64_t hist_records = 0;           // records kept by the last histogram call
  int32_t hist_bins_used = 0;         // non-empty bins of the last histogram call
  int sigc_variant = 1;
  int64_t sigc_zw_cap = int64_t(4) << 30;
  double partial_cap = 12.0e9;  // FP64 partial tiles per rank-K launch (bytes)
  uint64_t ws_gen = 1;
  int32_t* d_status = nullptr;
  void* staging = nullptr;  // pinned host staging for table uploads
  size_t staging_n = 0;
  hipEvent_t staging_done = nullptr;
  bool staging_pending = false;
  std::unordered_map<std::string, std::unique_ptr<Plan>> plans;
  int tile_sel[3] = {-1, -1, -1};
  int tile_tuned[3] = {-1, -1, -1};
  int tile_last[3] = {-1, -1, -1};   // configuration of the last rank-K launch
  int flush_override = 0;
  int xcd_slack = -1;   // -1: the configuration's; 0: off; > 0: stages; -2: unmeetable (tests)
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pending;
  std::vector<hipEvent_t> event_pool;
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
  bool sticky_error = false;
  // end of the previous call's work, on the stream it was enqueued on
  hipEvent_t last_done = nullptr;
  hipStream_t last_stream = nullptr;
  bool last_valid = false;
};

namespace {

int kind_of(chi0_precision p) {
  switch (p) {
    case CHI0_PREC_FP64: return HERK_FP64;
    case CHI0_PREC_FP32: return HERK_FP32;
    case CHI0_PREC_BF16X3: return HERK_BF16X3;
    default: return -1;
  }
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Debug log: with the environment variable CHI0_LOG set to a non-empty value
// other than "0", every launch decision (plan, tile, workspace) is printed
// to stderr, one line each.
bool log_on() {
  static const bool on = [] {
    const char* v = std::getenv("CHI0_LOG");
    return v && *v && std::strcmp(v, "0") != 0;
  }();
  return on;
}

void debug_log(const char* fmt, ...) {
  if (!log_on()) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[libchi0] %s\n", buf);
}

// Calls share the handle's workspace (partial tiles, weights, split planes,
// plan tables, inverse buffers), so they are ordered across streams: a call
// on another stream than the previous call's first waits for the event that
// call recorded at its end.  A stream under capture is left alone (the
// caller orders what it captures).
bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
    hipGetLastError();
    return false;
  }
  return cs != hipStreamCaptureStatusNone;
}

int call_begin(chi0_ctx* h, hipStream_t s) {
  if (h->last_valid && s != h->last_stream && !capturing(s))
    HIP_TRY(hipStreamWaitEvent(s, h->last_done, 0));
  return CHI0_OK;
}

int call_end(chi0_ctx* h, hipStream_t s, int rc) {
  if (capturing(s)) return rc;
  if (hipEventRecord(h->last_done, s) != hipSuccess) {
    hipGetLastError();
    return rc ? rc : fail(CHI0_EDEVICE, "event record on the call's stream failed");
  }
  h->last_stream = s;
  h->last_valid = true;
  return rc;
}

hipEvent_t get_event(chi0_ctx* h) {
  if (!h->event_pool.empty()) {
    hipEvent_t e = h->event_pool.back();
    h->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int validate_sigx(const sigx_problem* probs, int32_t nprob, chi0_ztype zt, chi0_precision prec,
                  uint32_t flags) {
  if (nprob < 0) return fail(CHI0_EINVAL, "nprob = %d < 0", nprob);
  if (nprob > 0 && !probs) return fail(CHI0_EINVAL, "probs is NULL");
  if (prec != CHI0_PREC_FP64 && prec != CHI0_PREC_FP32 && prec != CHI0_PREC_BF16X3)
    return fail(CHI0_EINVAL, "unknown precision %d", static_cast<int>(prec));
  if (zt != CHI0_Z_C128 && zt != CHI0_Z_C64)
    return fail(CHI0_EINVAL, "unknown Z type %d", static_cast<int>(zt));
  if (flags & ~static_cast<uint32_t>(CHI0_ACCUMULATE | CHI0_BF16_LOLO | CHI0_USE_GRAPH))
    return fail(CHI0_EINVAL, "unknown flag bits 0x%x", flags);
  for (int p = 0; p < nprob; ++p) {
    const sigx_problem& pr = probs[p];
    if (pr.nqp < 1) return fail(CHI0_EINVAL, "problem %d: nqp = %d < 1", p, pr.nqp);
    if (pr.nblocks < 0) return fail(CHI0_EINVAL, "problem %d: nblocks = %d < 0", p, pr.nblocks);
    if (pr.nblocks > 0 && !pr.blocks) return fail(CHI0_EINVAL, "problem %d: blocks is NULL", p);
    if (!pr.sigx) return fail(CHI0_EINVAL, "problem %d: sigx is NULL", p);
    if (!aligned(pr.sigx, 16)) return fail(CHI0_EINVAL, "problem %d: sigx not 16-byte aligned", p);
    for (int b = 0; b < pr.nblocks; ++b) {
      const sigx_block& bl = pr.blocks[b];
      if (bl.nocc < 0 || bl.nmu < 0)
        return fail(CHI0_EINVAL, "problem %d block %d: negative nocc/nmu", p, b);
      const int64_t K = static_cast<int64_t>(bl.nocc) * bl.nmu;
      if (K > 0x7fffffffLL)
        return fail(CHI0_EINVAL, "problem %d block %d: more than 2^31-1 rows", p, b);
      if (!std::isfinite(bl.wk) || bl.wk < 0.0)
        return fail(CHI0_EINVAL, "problem %d block %d: wk must be finite and >= 0", p, b);
      if (K > 0) {
        if (!bl.z) return fail(CHI0_EINVAL, "problem %d block %d: z is NULL", p, b);
        if (!aligned(bl.z, 16))
          return fail(CHI0_EINVAL, "problem %d block %d: z not 16-byte aligned", p, b);
        if (!bl.v) return fail(CHI0_EINVAL, "problem %d block %d: v is NULL", p, b);
      }
    }
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(pr.sigx);
    const uintptr_t a1 = a0 + static_cast<uintptr_t>(pr.nqp) * pr.nqp * 16;
    for (int q = 0; q < p; ++q) {
      const uintptr_t b0 = reinterpret_cast<uintptr_t>(probs[q].sigx);
      const uintptr_t b1 = b0 + static_cast<uintptr_t>(probs[q].nqp) * probs[q].nqp * 16;
      if (a0 < b1 && b0 < a1) return fail(CHI0_EINVAL, "problems %d and %d: outputs overlap", q, p);
    }
  }
  const bool need128 = prec == CHI0_PREC_FP64;
  if (need128 != (zt == CHI0_Z_C128))
    return fail(CHI0_EUNSUPPORTED, "precision %d needs Z type %s", static_cast<int>(prec),
                need128 ? "CHI0_Z_C128" : "CHI0_Z_C64");
  return CHI0_OK;
}

int validate_problems(const chi0_problem* probs, int32_t nprob, chi0_ztype zt,
                      chi0_precision prec, double delta_min, uint32_t flags) {
  if (nprob < 0) return fail(CHI0_EINVAL, "nprob = %d < 0", nprob);
  if (nprob > 0 && !probs) return fail(CHI0_EINVAL, "probs is NULL");
  if (prec != CHI0_PREC_FP64 && prec != CHI0_PREC_FP32 && prec != CHI0_PREC_BF16X3)
    return fail(CHI0_EINVAL, "unknown precision %d", static_cast<int>(prec));
  if (zt != CHI0_Z_C128 && zt != CHI0_Z_C64)
    return fail(CHI0_EINVAL, "unknown Z type %d", static_cast<int>(zt));
  if (!(delta_min >= 0.0) || !std::isfinite(delta_min))
    return fail(CHI0_EINVAL, "delta_min must be finite and >= 0 (got %g)", delta_min);
  if (flags & ~static_cast<uint32_t>(CHI0_ACCUMULATE | CHI0_BF16_LOLO | CHI0_USE_GRAPH))
    return fail(CHI0_EINVAL, "unknown flag bits 0x%x", flags);
  for (int p = 0; p < nprob; ++p) {
    const chi0_problem& pr = probs[p];
    if (pr.npb < 1) return fail(CHI0_EINVAL, "problem %d: npb = %d < 1", p, pr.npb);
    if (pr.nomega < 1) return fail(CHI0_EINVAL, "problem %d: nomega = %d < 1", p, pr.nomega);
    if (pr.nblocks < 0) return fail(CHI0_EINVAL, "problem %d: nblocks = %d < 0", p, pr.nblocks);
    if (pr.nblocks > 0 && !pr.blocks) return fail(CHI0_EINVAL, "problem %d: blocks is NULL", p);
    if (!pr.omega) return fail(CHI0_EINVAL, "problem %d: omega is NULL", p);
    if (!pr.chi0) return fail(CHI0_EINVAL, "problem %d: chi0 is NULL", p);
    if (!aligned(pr.chi0, 16)) return fail(CHI0_EINVAL, "problem %d: chi0 not 16-byte aligned", p);
    if (!aligned(pr.omega, 8)) return fail(CHI0_EINVAL, "problem %d: omega not 8-byte aligned", p);
    for (int b = 0; b < pr.nblocks; ++b) {
      const chi0_block& bl = pr.blocks[b];
      if (bl.nocc < 0 || bl.nunocc < 0)
        return fail(CHI0_EINVAL, "problem %d block %d: negative nocc/nunocc", p, b);
      const int64_t K = static_cast<int64_t>(bl.nocc) * bl.nunocc;
      if (K > 0x7fffffffLL)
        return fail(CHI0_EINVAL, "problem %d block %d: more than 2^31-1 pairs", p, b);
      if (!std::isfinite(bl.wk) || bl.wk < 0.0)
        return fail(CHI0_EINVAL, "problem %d block %d: wk must be finite and >= 0", p, b);
      if (K > 0) {
        if (!bl.z) return fail(CHI0_EINVAL, "problem %d block %d: z is NULL", p, b);
        if (!aligned(bl.z, 16))
          return fail(CHI0_EINVAL, "problem %d block %d: z not 16-byte aligned", p, b);
        if (!bl.eps_occ || !bl.eps_unocc)
          return fail(CHI0_EINVAL, "problem %d block %d: energies are NULL", p, b);
      }
    }
    // output buffers of different problems must not overlap
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(pr.chi0);
    const uintptr_t a1 = a0 + static_cast<uintptr_t>(pr.nomega) * pr.npb * pr.npb * 16;
    for (int q = 0; q < p; ++q) {
      const uintptr_t b0 = reinterpret_cast<uintptr_t>(probs[q].chi0);
      const uintptr_t b1 = b0 + static_cast<uintptr_t>(probs[q].nomega) * probs[q].npb * probs[q].npb * 16;
      if (a0 < b1 && b0 < a1) return fail(CHI0_EINVAL, "problems %d and %d: chi0 outputs overlap", q, p);
    }
  }
  const bool need128 = prec == CHI0_PREC_FP64;
  if (need128 != (zt == CHI0_Z_C128))
    return fail(CHI0_EUNSUPPORTED, "precision %d needs Z type %s", static_cast<int>(prec),
                need128 ? "CHI0_Z_C128" : "CHI0_Z_C64");
  return CHI0_OK;
}

std::string plan_key(int kind, int tile_idx, int nwg, const chi0_problem* probs, int nprob) {
  std::string k;
  k.reserve(64 + nprob * 16);
  char buf[64];
  snprintf(buf, sizeof(buf), "%d/%d/%d/%d|", kind, tile_idx, nwg, nprob);
  k += buf;
  for (int p = 0; p < nprob; ++p) {
    snprintf(buf, sizeof(buf), "%d,%d,%d:", probs[p].npb, probs[p].nomega, probs[p].nblocks);
    k += buf;
    for (int b = 0; b < probs[p].nblocks; ++b) {
      snprintf(buf, sizeof(buf), "%d.%d;", probs[p].blocks[b].nocc, probs[p].blocks[b].nunocc);
      k += buf;
    }
  }
  return k;
}

template <class T>
int upload_sync(DevBuf& d, const std::vector<T>& v) {
  const size_t bytes = std::max<size_t>(sizeof(T), v.size() * sizeof(T));
  int rc = d.reserve(bytes, nullptr);
  if (rc) return rc;
  if (!v.empty()) HIP_TRY(hipMemcpy(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return CHI0_OK;
}

// Work decomposition (host only).
//  * Every (problem, frequency, lower tile) is split into s_p contiguous
//    ranges of the problem's pairs (blocks concatenated); s_p is chosen so
//    that there are several units per workgroup.
//  * Units are ordered range-major (then tile, then frequency) so that the
//    workgroups running at the same time stream the same rows of Z, and are
//    dealt to workgroups by greedy list scheduling in that order (each unit
//    goes to the workgroup that becomes free first, by the pair-count cost
//    model).
//  * Logical workgroups are placed XCD-major: consecutive logical
//    workgroups share an XCD (workgroups are dispatched round-robin over the
//    8 XCDs), so units that read the same Z columns share an L2.
struct HostPlan {
  std::vector<Unit> units;      // work items (a unit may hold several frequencies)
  int64_t nslots = 0;           // FP64 partial slots (one per frequency, tile and range)
  std::vector<TileJob> jobs;
  std::vector<int32_t> wg_off, wg_units;
  std::vector<double> cost;
  std::vector<double> wg_load;
  int nblocks_total = 0;
  bool round_robin = false;
};

// Default upper bound on the FP64 partial tiles of one rank-K launch (bytes).
constexpr double kMaxPartialBytes = 12.0e9;

// Tiles right of the diagonal in a configuration that leaves out the blocks
// above it (TP = 2 TQ, tile column 2 tp + 1): 3 of their 8 blocks are
// computed, so their units are light.
constexpr double kLightCost = 0.5;
bool light_tile(const TileConfig& tc, int tp, int tq) {
  return tc.diag_skip && tc.tile == 2 * tc.tile_q && tq == 2 * tp + 1;
}
// diag_skip 1: light units are costed as such and dealt after the others;
// 2: they keep their place in the locality order and a full unit's cost
bool deal_light_apart(const TileConfig& tc, int tp, int tq) {
  return tc.diag_skip == 1 && light_tile(tc, tp, tq);
}

// Lower-triangle tiles of a TP x TQ tiling of an npb x npb matrix: tile
// (tp, tq) is needed iff it holds an entry on or below the diagonal.
void lower_tiles(int npb, int TP, int TQ, std::vector<std::pair<int, int>>& out) {
  out.clear();
  const int ntp = (npb + TP - 1) / TP;
  for (int tp = 0; tp < ntp; ++tp) {
    const int last_row = std::min((tp + 1) * TP, npb) - 1;
    for (int tq = 0; tq * TQ <= last_row; ++tq) out.emplace_back(tp, tq);
  }
}

void plan_host(const TileConfig& tc, int nwg_launch, const chi0_problem* probs, int nprob,
               HostPlan& hp, double max_partial_bytes = kMaxPartialBytes) {
  const int TP = tc.tile, TQ = tc.tile_q;
  // work lists: one per workgroup, or one per wave (W per workgroup); the
  // dealing below is over lists, the placement keeps the W lists of a
  // workgroup together
  const int W = std::max(1, static_cast<int>(tc.wave_lists));
  const int nwg = nwg_launch * W;
  // frequencies per unit (frequency-group configurations); ngrp: units per
  // (tile, range) of a problem with nomega frequencies
  const int G = std::max(1, static_cast<int>(tc.omega_group));
  auto ngrp = [G](int nomega) { return (nomega + G - 1) / G; };
  struct P {
    int npb, nomega, ntl, b0, nb;
    int64_t K;
    std::vector<int64_t> cum;  // cumulative pairs at block starts
    std::vector<std::pair<int, int>> tiles;
  };
  std::vector<P> ps(nprob);
  int bflat = 0;
  double work = 0.0;
  for (int p = 0; p < nprob; ++p) {
    P& q = ps[p];
    q.npb = probs[p].npb;
    q.nomega = probs[p].nomega;
    lower_tiles(q.npb, TP, TQ, q.tiles);
    q.ntl = static_cast<int>(q.tiles.size());
    q.b0 = bflat;
    q.nb = probs[p].nblocks;
    q.cum.resize(q.nb + 1);
    q.cum[0] = 0;
    for (int b = 0; b < q.nb; ++b)
      q.cum[b + 1] = q.cum[b] + static_cast<int64_t>(probs[p].blocks[b].nocc) * probs[p].blocks[b].nunocc;
    q.K = q.cum[q.nb];
    bflat += q.nb;
    work += static_cast<double>(ngrp(q.nomega)) * q.ntl * static_cast<double>(q.K);
  }
  hp.nblocks_total = bflat;

  // target pairs per unit: ~8 units per workgroup, at least 1024 pairs, and
  // partial storage bounded
  const double min_pairs = 1024.0;
  double per_unit = std::max(min_pairs, work / (8.0 * nwg));
  const double slot_bytes = static_cast<double>(TP) * TQ * 16.0;
  auto count_units = [&](double pu) {
    double n = 0;
    for (auto& q : ps)
      n += static_cast<double>(q.nomega) * q.ntl * std::max<int64_t>(1, std::llround(std::ceil(q.K / pu)));
    return n;
  };
  // Once a unit may hold a whole problem every job has one unit and larger
  // units change nothing; callers split work whose jobs alone exceed the cap
  // (run_accumulate), so the loop ends with the storage bounded.
  double kmax_all = 0.0;
  for (auto& q : ps) kmax_all = std::max(kmax_all, static_cast<double>(q.K));
  while (count_units(per_unit) * slot_bytes > max_partial_bytes && per_unit < kmax_all) per_unit *= 1.5;
  // one problem shape: pick the range count so that the units fill whole
  // rounds of the persistent grid (round-robin dealing is then exact; with
  // diag_skip the light units of the tiles right of the diagonal, dealt
  // after the others, fill whole rounds too)
  if (nprob == 1 && ps[0].K > 0) {
    const double jobs = static_cast<double>(ps[0].nomega) * ps[0].ntl;
    int nlight = 0;
    for (const auto& t : ps[0].tiles) nlight += deal_light_apart(tc, t.first, t.second) ? 1 : 0;
    const double light_per_range = static_cast<double>(ngrp(ps[0].nomega)) * nlight;
    const double units_per_range = static_cast<double>(ngrp(ps[0].nomega)) * ps[0].ntl - light_per_range;
    const int64_t s0 = std::max<int64_t>(1, std::llround(std::ceil(ps[0].K / per_unit)));
    for (int64_t sr = s0; sr <= s0 + 16 && sr <= ps[0].K; ++sr) {
      const double nu = units_per_range * sr;
      if (std::fmod(nu, static_cast<double>(nwg)) == 0.0 &&
          std::fmod(light_per_range * sr, static_cast<double>(nwg)) == 0.0 &&
          jobs * sr * slot_bytes <= max_partial_bytes) {
        per_unit = static_cast<double>(ps[0].K) / sr * (1.0 + 1e-9);
        break;
      }
    }
  }

  struct Range { int b0, p0, b1, p1; int64_t n; };
  std::vector<std::vector<Range>> ranges(nprob);
  for (int p = 0; p < nprob; ++p) {
    P& q = ps[p];
    int64_t s = std::max<int64_t>(1, std::llround(std::ceil(static_cast<double>(q.K) / per_unit)));
    if (q.K == 0) s = 1;
    // range boundaries fall on multiples of the staging chunk within their
    // block, so every stage of a unit is a whole, aligned chunk of a block
    // (or that block's tail)
    auto align = [&](int64_t g) {
      if (q.nb == 0 || g <= 0 || g >= q.K) return std::max<int64_t>(0, std::min(g, q.K));
      int bb = static_cast<int>(std::upper_bound(q.cum.begin(), q.cum.end(), g) - q.cum.begin()) - 1;
      bb = std::min(bb, q.nb - 1);
      const int64_t kb = q.cum[bb + 1] - q.cum[bb];
      const int64_t loc = std::min(kb, (g - q.cum[bb] + tc.kchunk / 2) / tc.kchunk * tc.kchunk);
      return q.cum[bb] + loc;
    };
    for (int64_t r = 0; r < s; ++r) {
      const int64_t g0 = align(q.K * r / s), g1 = align(q.K * (r + 1) / s);
      Range rg{};
      rg.n = g1 - g0;
      if (q.nb == 0) {
        rg.b0 = q.b0; rg.p0 = 0; rg.b1 = q.b0 - 1; rg.p1 = 0;  // empty: no block visited
      } else {
        int bb = static_cast<int>(std::upper_bound(q.cum.begin(), q.cum.end(), g0) - q.cum.begin()) - 1;
        bb = std::min(bb, q.nb - 1);
        rg.b0 = q.b0 + bb;
        rg.p0 = static_cast<int>(g0 - q.cum[bb]);
        int be = static_cast<int>(std::lower_bound(q.cum.begin(), q.cum.end(), g1) - q.cum.begin()) - 1;
        be = std::max(be, 0);
        be = std::min(be, q.nb - 1);
        rg.b1 = q.b0 + be;
        rg.p1 = static_cast<int>(g1 - q.cum[be]);
        if (g1 == g0) { rg.b1 = rg.b0; rg.p1 = rg.p0; }
      }
      ranges[p].push_back(rg);
    }
  }
  // units in tile-job order (slots of a job contiguous)
  std::vector<int> unit_range_idx;
  for (int p = 0; p < nprob; ++p) {
    P& q = ps[p];
    for (int iw = 0; iw < q.nomega; ++iw)
      for (const auto& t : q.tiles) {
        const int tp = t.first, tq = t.second;
        TileJob j{p, iw, tp, tq, static_cast<int32_t>(hp.units.size()),
                  static_cast<int32_t>(ranges[p].size())};
        hp.jobs.push_back(j);
        for (size_t r = 0; r < ranges[p].size(); ++r) {
          const Range& rg = ranges[p][r];
          Unit u{};
          u.prob = p; u.iw = iw; u.tp = tp; u.tq = tq;
          u.b0 = rg.b0; u.p0 = rg.p0; u.b1 = rg.b1; u.p1 = rg.p1;
          u.slot = static_cast<int32_t>(hp.units.size());
          u.nw = 1;
          u.wstride = 0;
          hp.units.push_back(u);
          unit_range_idx.push_back(static_cast<int>(r));
          // cost: pairs rounded up to staging chunks per block touched, plus a
          // fixed per-unit cost (zeroing and writing the tile); a light unit
          // (3 of its 8 blocks) costs about half
          const double nblk = std::max(0, rg.b1 - rg.b0 + 1);
          hp.cost.push_back((static_cast<double>(rg.n) + nblk * tc.kchunk + 64.0) *
                            (deal_light_apart(tc, tp, tq) ? kLightCost : 1.0));
        }
      }
  }
  hp.nslots = static_cast<int64_t>(hp.units.size());
  // frequency groups: the units of up to G consecutive frequencies of one
  // (problem, tile, range) become one unit (their slots are a fixed stride
  // apart: the units above are in (problem, frequency, tile, range) order)
  if (G > 1) {
    std::vector<Unit> gu;
    std::vector<double> gc;
    std::vector<int> gr;
    size_t base = 0;
    for (int p = 0; p < nprob; ++p) {
      const P& q = ps[p];
      const size_t s_p = ranges[p].size(), ntl = q.tiles.size();
      for (size_t t = 0; t < ntl; ++t)
        for (size_t r = 0; r < s_p; ++r)
          for (int iw0 = 0; iw0 < q.nomega; iw0 += G) {
            const size_t idx = base + (static_cast<size_t>(iw0) * ntl + t) * s_p + r;
            Unit u = hp.units[idx];
            u.nw = std::min(G, q.nomega - iw0);
            u.wstride = static_cast<int32_t>(ntl * s_p);
            gu.push_back(u);
            gc.push_back(hp.cost[idx]);
            gr.push_back(static_cast<int>(r));
          }
      base += static_cast<size_t>(q.nomega) * ntl * s_p;
    }
    hp.units.swap(gu);
    hp.cost.swap(gc);
    unit_range_idx.swap(gr);
  }
  // locality order: (problem, range, tile, frequency)
  std::vector<int> order(hp.units.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int>(i);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const Unit& ua = hp.units[a];
    const Unit& ub = hp.units[b];
    if (ua.prob != ub.prob) return ua.prob < ub.prob;
    if (unit_range_idx[a] != unit_range_idx[b]) return unit_range_idx[a] < unit_range_idx[b];
    if (ua.tp != ub.tp) return ua.tp < ub.tp;
    if (ua.tq != ub.tq) return ua.tq < ub.tq;
    return ua.iw < ub.iw;
  });
  // Dealing.  When the units cost about the same (one problem shape: every
  // tile has the same pairs), they are dealt round-robin in locality order,
  // so that in every round the frequencies of a tile start together on
  // neighbouring logical workgroups (one XCD) and stream the same rows of Z
  // at the same time, sharing that XCD's L2.  Otherwise greedy list
  // scheduling (each unit to the workgroup that becomes free first) keeps
  // uneven problems balanced.
  // With diag_skip the light units are dealt round-robin after the others
  // (each list ends with its share of them).
  std::vector<std::vector<int>> lists(nwg);
  std::vector<double> load(nwg, 0.0);
  std::vector<int> heavy, light;
  for (int id : order) {
    const Unit& u = hp.units[id];
    (deal_light_apart(tc, u.tp, u.tq) ? light : heavy).push_back(id);
  }
  double cmin = 0.0, cmax = 0.0;
  for (size_t i = 0; i < heavy.size(); ++i) {
    const double c = hp.cost[heavy[i]];
    cmin = i ? std::min(cmin, c) : c;
    cmax = i ? std::max(cmax, c) : c;
  }
  const size_t nu = heavy.size();
  const bool uniform = nu > 0 && cmax <= 1.05 * cmin &&
                       (nu % nwg == 0 || nu / nwg >= 16 || nu < static_cast<size_t>(nwg));
  hp.round_robin = uniform;
  if (uniform) {
    for (size_t i = 0; i < nu + light.size(); ++i) {
      const int w = static_cast<int>(i % nwg);
      const int id = i < nu ? heavy[i] : light[i - nu];
      lists[w].push_back(id);
      load[w] += hp.cost[id];
    }
  } else {
    typedef std::pair<double, int> Slot;
    std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
    for (int w = 0; w < nwg; ++w) heap.push(Slot(0.0, w));
    for (int id : order) {
      Slot sl = heap.top();
      heap.pop();
      lists[sl.second].push_back(id);
      sl.first += hp.cost[id];
      load[sl.second] = sl.first;
      heap.push(sl);
    }
  }
  // logical -> physical placement (XCD-major over workgroups; a
  // workgroup's W lists stay together)
  const int nxcd = 8;
  std::vector<int> phys_of(nwg);
  if (nwg_launch % nxcd == 0) {
    const int per = nwg_launch / nxcd;
    for (int L = 0; L < nwg; ++L) {
      const int lw = L / W;
      phys_of[L] = ((lw % per) * nxcd + lw / per) * W + L % W;
    }
  } else {
    for (int L = 0; L < nwg; ++L) phys_of[L] = L;
  }
  std::vector<std::vector<int>> plists(nwg);
  hp.wg_load.assign(nwg, 0.0);
  for (int L = 0; L < nwg; ++L) {
    plists[phys_of[L]] = std::move(lists[L]);
    hp.wg_load[phys_of[L]] = load[L];
  }
  hp.wg_off.assign(nwg + 1, 0);
  hp.wg_units.clear();
  hp.wg_units.reserve(hp.units.size());
  for (int w = 0; w < nwg; ++w) {
    hp.wg_off[w] = static_cast<int32_t>(hp.wg_units.size());
    for (int id : plists[w]) hp.wg_units.push_back(id);
  }
  hp.wg_off[nwg] = static_cast<int32_t>(hp.wg_units.size());
}

int build_plan(chi0_ctx* h, Plan& pl, int kind, int tile_idx, const chi0_problem* probs,
               int nprob) {
  const TileConfig tc = herk_tile_config(kind, tile_idx);
  const int wg_per_cu = std::max(1, herk_max_wg_per_cu(kind, tile_idx));
  const int nwg = h->ncu * wg_per_cu;
  pl.kind = kind;
  pl.tile_idx = tile_idx;
  pl.tc = tc;
  pl.nwg = nwg;
  pl.nprob = nprob;
  HostPlan hp;
  plan_host(tc, nwg, probs, nprob, hp, h->partial_cap);
  pl.nblocks_total = hp.nblocks_total;
  pl.nunits = static_cast<int>(hp.units.size());
  pl.nslots = hp.nslots;
  pl.njobs = static_cast<int>(hp.jobs.size());
  pl.round_robin = hp.round_robin;
  int rc;
  if ((rc = upload_sync(pl.d_units, hp.units))) return rc;
  if ((rc = upload_sync(pl.d_wg_off, hp.wg_off))) return rc;
  if ((rc = upload_sync(pl.d_wg_units, hp.wg_units))) return rc;
  if ((rc = upload_sync(pl.d_jobs, hp.jobs))) return rc;
  if ((rc = pl.d_blocks.reserve(std::max(1, hp.nblocks_total) * sizeof(BlockDesc), nullptr))) return rc;
  if ((rc = pl.d_probs.reserve(std::max(1, nprob) * sizeof(ProbDesc), nullptr))) return rc;
  return CHI0_OK;
}

// FP32 run length for a problem.  A run of L pairs sums about 3 L / 8 MFMA
// results per output in FP32; with R = K / L runs combined in FP64 the
// relative rounding error of a positive sum is about u L / sqrt(8 K), so
// L = 4 sqrt(K) keeps it near 1.4 u for every problem size (capped by the
// tile configuration's run length, floored at 64 pairs).
int32_t flush_length(const chi0_ctx* h, const TileConfig& tc, const chi0_problem& pr) {
  if (h->flush_override > 0) return h->flush_override;
  if (tc.flush <= 0) return 0;
  double K = 0.0;
  for (int b = 0; b < pr.nblocks; ++b) K += static_cast<double>(pr.blocks[b].nocc) * pr.blocks[b].nunocc;
  int32_t L = static_cast<int32_t>(4.0 * std::sqrt(K)) / 16 * 16;
  return std::max<int32_t>(64, std::min<int32_t>(tc.flush, L));
}

int staging_reserve(chi0_ctx* h, size_t bytes) {
  if (h->staging_pending) {
    HIP_TRY(hipEventSynchronize(h->staging_done));
    h->staging_pending = false;
  }
  if (bytes <= h->staging_n) return CHI0_OK;
  if (h->staging) hipHostFree(h->staging);
  h->staging = nullptr;
  h->staging_n = 0;
  HIP_TRY(hipHostMalloc(&h->staging, bytes, hipHostMallocDefault));
  h->staging_n = bytes;
  return CHI0_OK;
}

// Row weights of a call: the chi0 transition weights (Eq.(polfx) at i omega)
// or, for the exchange self-energy, w_k v_mu (Eq.(sigx)).
enum WeightMode { kWeightsChi0 = 0, kWeightsCoulomb = 1 };

// Status words of a handle (int32, device): zero pivot of the pivoted
// inverse, non-positive HPD pivot of the current call and since the last
// sync, pairs with D <= 0 since the last sync.
enum { kStZeroPivot = 0, kStHpdCall = 1, kStHpdSeen = 2, kStNonpositive = 3, kStWords = 4 };

hipError_t weights_launch(int mode, const BlockDesc* blocks, const ProbDesc* probs, int nblocks,
                          int kmax, double delta_min, bool f64, int32_t* status, hipStream_t s) {
  return mode == kWeightsCoulomb
             ? coulomb_weights_launch(blocks, probs, nblocks, kmax, f64, s)
             : pair_weights_launch(blocks, probs, nblocks, kmax, delta_min, f64, status + kStNonpositive, s);
}

// Gathered rows and given weights (the histogram path): problem p's single
// block reads its rows at rows[off[p] ..] and its weights at wts[off[p] ..]
// (double for FP64, float otherwise).
struct GatherHook {
  const uint64_t* rows;
  const void* wts;
  const int64_t* off;
};

// Configuration for a call with no tile fixed or tuned.  Modeled time of a
// candidate: rows x padded lower-triangle tile area x frequencies (for a
// frequency-group kernel, the frequencies rounded up to whole groups) x a
// per-kernel cost, plus the pre-split pass (rows x npb) of kernels that read
// it.  Costs relative to the built-in default, fitted to MI355X timings at
// npb 287, 384 and 2048: BF16x3 frequency groups on 128 x 64 tiles (20) 1.0,
// tall 256 x 128 (7) 1.20, 128^2 with two workgroups per CU (4) 1.34, 64^2
// (2) 2.04, the pre-split pass 173 per row and column; FP64 128^2 with 8
// waves (3) 1.0, 64^2 (1) 1.36, 32^2 (2) 1.42; FP32 frequency groups on
// 128 x 64 tiles (2) 1.0, 64^2 (1) 1.27, 128^2 (0) 1.16.  Another tile
// replaces the default only when modeled at least 5% faster.
int tile_for(int kind, const chi0_problem* probs, int nprob) {
  struct Cand {
    int idx;
    double cost;
  };
  static const Cand bf16[] = {{20, 1.0}, {7, 1.20}, {4, 1.34}, {2, 2.04}};
  static const Cand fp64[] = {{3, 1.0}, {1, 1.36}, {2, 1.42}};
  static const Cand fp32[] = {{2, 1.0}, {1, 1.27}, {0, 1.16}};
  const int ndef = herk_default_tile(kind);
  const Cand* cands = kind == HERK_BF16X3 ? bf16 : kind == HERK_FP64 ? fp64 : fp32;
  const int ncand = kind == HERK_BF16X3 ? 4 : 3;
  double def_time = -1.0, best_time = -1.0;
  int best = ndef;
  for (int ci = 0; ci < ncand; ++ci) {
    const Cand& c = cands[ci];
    if (c.idx >= herk_tile_count(kind)) continue;
    const TileConfig tc = herk_tile_config(kind, c.idx);
    const int TP = tc.tile, TQ = tc.tile_q;
    double t = 0.0;
    for (int p = 0; p < nprob; ++p) {
      double rows = 0.0;
      for (int b = 0; b < probs[p].nblocks; ++b)
        rows += static_cast<double>(probs[p].blocks[b].nocc) * probs[p].blocks[b].nunocc;
      const int npb = probs[p].npb;
      const int ntp = (npb + TP - 1) / TP, ntq = (npb + TQ - 1) / TQ;
      double area = 0.0;
      for (int tp = 0; tp < ntp; ++tp) {
        const int nt = std::min(ntq, (tp * TP + TP - 1) / TQ + 1);
        area += static_cast<double>(nt) * TP * TQ;
        if (2 * tp + 1 < nt && light_tile(tc, tp, 2 * tp + 1)) area -= (1.0 - kLightCost) * TP * TQ;
      }
      const int G = std::max(1, static_cast<int>(tc.omega_group));
      const int nw = (std::max(1, probs[p].nomega) + G - 1) / G * G;
      t += rows * area * nw * c.cost;
      if (tc.presplit) t += rows * npb * 173.0;
    }
    if (c.idx == ndef) def_time = t;
    if (best_time < 0.0 || t < best_time) {
      best_time = t;
      best = c.idx;
    }
  }
  return def_time >= 0.0 && best != ndef && best_time >= 0.95 * def_time ? ndef : best;
}

// One rank-K launch (weights, pre-split, rank-K kernel, reduction) over a set
// of problems whose minimal partial storage fits the handle's cap.
int run_accumulate_group(chi0_ctx* h, const chi0_problem* probs, int32_t nprob, chi0_precision prec,
                         double delta_min, uint32_t flags, hipStream_t stream, int tile_idx,
                         int mode, const GatherHook* hk) {
  const int kind = kind_of(prec);
  int wg_per_cu = std::max(1, herk_max_wg_per_cu(kind, tile_idx));
  const int nwg = h->ncu * wg_per_cu;
  std::string key = plan_key(kind, tile_idx, nwg, probs, nprob);
  if (h->partial_cap != kMaxPartialBytes) {
    char cb[40];
    snprintf(cb, sizeof(cb), "#cap%a", h->partial_cap);
    key += cb;
  }
  Plan* pl;
  if (hk) {
    // histogram bins change with the data: one reusable slot, not the cache
    if (!h->gather_plan || h->gather_key != key) {
      std::unique_ptr<Plan> np(new Plan());
      int rc = build_plan(h, *np, kind, tile_idx, probs, nprob);
      if (rc) return rc;
      h->gather_plan = std::move(np);
      h->gather_key = key;
    }
    pl = h->gather_plan.get();
  } else {
    auto it = h->plans.find(key);
    if (it == h->plans.end()) {
      std::unique_ptr<Plan> np(new Plan());
      int rc = build_plan(h, *np, kind, tile_idx, probs, nprob);
      if (rc) return rc;
      pl = np.get();
      h->plans.emplace(key, std::move(np));
    } else {
      pl = it->second.get();
    }
  }
  if (pl->nunits == 0) return CHI0_OK;
  const int TP = pl->tc.tile, TQ = pl->tc.tile_q;
  int rc = h->partials.reserve(static_cast<size_t>(pl->nslots) * TP * TQ * sizeof(double2), &h->ws_gen);
  if (rc) return rc;
  const int nblocks_total = pl->nblocks_total;

  // pair weights: [nomega][ktot] per problem, float (FP64 path: double)
  const size_t wsize = kind == HERK_FP64 ? sizeof(double) : sizeof(float);
  size_t wbytes = 0;
  int kmax = 0;
  for (int p = 0; p < nprob; ++p) {
    int64_t kt = 0;
    for (int b = 0; b < probs[p].nblocks; ++b) {
      const int64_t k = static_cast<int64_t>(probs[p].blocks[b].nocc) * probs[p].blocks[b].nunocc;
      kt += k;
      kmax = std::max<int>(kmax, static_cast<int>(k));
    }
    wbytes += ((static_cast<size_t>(kt) * probs[p].nomega * wsize + 255) / 256) * 256;
  }
  if (!hk && (rc = h->wts.reserve(std::max<size_t>(wbytes, 256), &h->ws_gen))) return rc;

  // pre-split P-side planes (kernels that read them only)
  const bool presplit = pl->tc.presplit != 0;
  size_t zbytes = 0;
  int64_t max_groups = 0;
  int max_npb = 0;
  if (presplit) {
    for (int p = 0; p < nprob; ++p)
      for (int b = 0; b < probs[p].nblocks; ++b) {
        const int64_t G = presplit_groups(static_cast<int64_t>(probs[p].blocks[b].nocc) *
                                          probs[p].blocks[b].nunocc);
        const size_t plane = ((static_cast<size_t>(G) * probs[p].npb * 16 + 255) / 256) * 256;
        zbytes += 2 * plane;
        max_groups = std::max(max_groups, G);
        max_npb = std::max(max_npb, probs[p].npb);
      }
    if ((rc = h->zsplit.reserve(std::max<size_t>(zbytes, 256), &h->ws_gen))) return rc;
  }

  // per-call tables (pointers change between calls) via pinned staging
  std::vector<BlockDesc> bt;
  bt.reserve(pl->nblocks_total);
  std::vector<ProbDesc> ptab(nprob);
  size_t woff = 0, zoff = 0;
  bool z16 = true;
  for (int p = 0; p < nprob; ++p) {
    ptab[p].chi0 = static_cast<double2*>(probs[p].chi0);
    ptab[p].omega = probs[p].omega;
    ptab[p].wts = hk ? const_cast<char*>(static_cast<const char*>(hk->wts)) + hk->off[p] * wsize
                     : static_cast<char*>(h->wts.p) + woff;
    ptab[p].npb = probs[p].npb;
    ptab[p].nomega = probs[p].nomega;
    ptab[p].flush = flush_length(h, pl->tc, probs[p]);
    ptab[p].pad = 0;
    int64_t base = 0;
    for (int b = 0; b < probs[p].nblocks; ++b) {
      const chi0_block& bl = probs[p].blocks[b];
      BlockDesc d;
      d.z = bl.z;
      if (probs[p].npb & 1) z16 = false;   // (every Z is 16-byte aligned: validated)
      d.eps_occ = bl.eps_occ;
      d.eps_unocc = bl.eps_unocc;
      d.wk = bl.wk;
      d.nocc = bl.nocc;
      d.nunocc = bl.nunocc;
      d.pair_base = base;
      d.prob = p;
      d.pad = 0;
      d.zs = nullptr;
      d.zs_plane = 0;
      d.rows = hk ? hk->rows + hk->off[p] : nullptr;
      if (presplit) {
        const int64_t G = presplit_groups(static_cast<int64_t>(bl.nocc) * bl.nunocc);
        const size_t plane = ((static_cast<size_t>(G) * probs[p].npb * 16 + 255) / 256) * 256;
        d.zs = static_cast<char*>(h->zsplit.p) + zoff;
        d.zs_plane = static_cast<int64_t>(plane);
        zoff += 2 * plane;
      }
      base += static_cast<int64_t>(bl.nocc) * bl.nunocc;
      bt.push_back(d);
    }
    ptab[p].ktot = base;
    woff += ((static_cast<size_t>(base) * probs[p].nomega * wsize + 255) / 256) * 256;
  }
  const size_t bt_bytes = bt.size() * sizeof(BlockDesc);
  const size_t pt_bytes = ptab.size() * sizeof(ProbDesc);
  if ((rc = staging_reserve(h, bt_bytes + pt_bytes + 64))) return rc;
  char* st = static_cast<char*>(h->staging);
  if (bt_bytes) memcpy(st, bt.data(), bt_bytes);
  memcpy(st + bt_bytes, ptab.data(), pt_bytes);
  if (bt_bytes) HIP_TRY(hipMemcpyAsync(pl->d_blocks.p, st, bt_bytes, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(pl->d_probs.p, st + bt_bytes, pt_bytes, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipEventRecord(h->staging_done, stream));
  h->staging_pending = true;

  HerkArgs ha;
  ha.units = static_cast<const Unit*>(pl->d_units.p);
  ha.wg_offsets = static_cast<const int32_t*>(pl->d_wg_off.p);
  ha.wg_units = static_cast<const int32_t*>(pl->d_wg_units.p);
  ha.blocks = static_cast<const BlockDesc*>(pl->d_blocks.p);
  ha.probs = static_cast<const ProbDesc*>(pl->d_probs.p);
  ha.partials = static_cast<double2*>(h->partials.p);
  ha.delta_min = delta_min;
  ha.flags = static_cast<int32_t>(flags);
  ha.sync_prog = nullptr;
  ha.sync_slack = 0;
  ha.z16 = z16 ? 1 : 0;
  ha.pad = 0;
  const int slack = h->xcd_slack == -1 ? pl->tc.xcd_sync : h->xcd_slack;
  if (pl->tc.xcd_sync > 0 && slack != 0 && pl->round_robin) {
    // one progress word per workgroup; a fresh buffer starts at 0 (the
    // kernel leaves INT_MAX in each word when its workgroup finishes)
    const size_t bytes = static_cast<size_t>(pl->nwg) * sizeof(int32_t);
    if (h->sync_prog.n < bytes) {
      if ((rc = h->sync_prog.reserve(bytes, &h->ws_gen))) return rc;
      HIP_TRY(hipMemset(h->sync_prog.p, 0, h->sync_prog.n));
    }
    ha.sync_prog = static_cast<int32_t*>(h->sync_prog.p);
    ha.sync_slack = slack == -2 ? INT32_MIN / 2 : slack;
  }
  ReduceArgs ra;
  ra.jobs = static_cast<const TileJob*>(pl->d_jobs.p);
  ra.probs = ha.probs;
  ra.partials = ha.partials;
  ra.tile_p = TP;
  ra.tile_q = TQ;
  ra.planar = pl->tc.planar ? 1 : 0;
  ra.accumulate = (flags & CHI0_ACCUMULATE) ? 1 : 0;

  const bool use_graph = (flags & CHI0_USE_GRAPH) && !h->profiling && !hk;
  debug_log("rank-K launch: kind %d tile %d (%d x %d, %d threads), %d problem(s), %d units on %d "
       "workgroups, %d tile jobs, partials %zu B, weights %zu B, pre-split %zu B%s%s%s",
       kind, pl->tile_idx, TP, TQ, pl->tc.threads, nprob, pl->nunits, pl->nwg, pl->njobs,
       static_cast<size_t>(pl->nslots) * TP * TQ * sizeof(double2), hk ? static_cast<size_t>(0) : wbytes,
       zbytes, use_graph ? ", graph" : "", hk ? ", gathered rows" : "",
       ha.sync_prog ? ", XCD lockstep" : "");
  if (use_graph) {
    // delta_min and the LO*LO flag are kernel arguments: the cached graph is
    // only reused with the same values, so they join the key
    const int gi = ra.accumulate;
    char kb[96];
    snprintf(kb, sizeof(kb), "#g%d/%a/%u/m%d/z%d", gi, delta_min, flags, mode, ha.z16);
    const std::string gkey = key + kb;
    auto git = h->plans.find(gkey);
    Plan* gp = nullptr;
    if (git == h->plans.end()) {
      std::unique_ptr<Plan> holder(new Plan());
      gp = holder.get();
      h->plans.emplace(gkey, std::move(holder));
    } else {
      gp = git->second.get();
    }
    if (!gp->graph[0] || gp->graph_gen[0] != h->ws_gen) {
      if (gp->graph[0]) hipGraphExecDestroy(gp->graph[0]);
      gp->graph[0] = nullptr;
      hipStream_t cs;
      HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess)
        e = weights_launch(mode, ha.blocks, ha.probs, nblocks_total, kmax, delta_min,
                           kind == HERK_FP64, h->d_status, cs);
      if (e == hipSuccess && presplit)
        e = presplit_launch(ha.blocks, ha.probs, nblocks_total, max_groups, max_npb, cs);
      if (e == hipSuccess) e = herk_launch(kind, pl->tile_idx, ha, pl->nwg, cs);
      if (e == hipSuccess) e = reduce_launch(ra, pl->njobs, cs);
      hipError_t e2 = hipStreamEndCapture(cs, &g);
      hipStreamDestroy(cs);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return fail(CHI0_EDEVICE, "graph capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
      }
      hipGraphExec_t ex = nullptr;
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (e != hipSuccess) return fail(CHI0_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
      gp->graph[0] = ex;
      gp->graph_gen[0] = h->ws_gen;
    }
    HIP_TRY(hipGraphLaunch(gp->graph[0], stream));
    return CHI0_OK;
  }

  hipError_t ew = hk ? hipSuccess
                     : weights_launch(mode, ha.blocks, ha.probs, nblocks_total, kmax, delta_min,
                                      kind == HERK_FP64, h->d_status, stream);
  if (ew != hipSuccess) return fail(CHI0_EDEVICE, "pair-weight launch: %s", hipGetErrorString(ew));
  if (presplit) {
    ew = presplit_launch(ha.blocks, ha.probs, nblocks_total, max_groups, max_npb, stream);
    if (ew != hipSuccess) return fail(CHI0_EDEVICE, "pre-split launch: %s", hipGetErrorString(ew));
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->profiling) {
    e0 = get_event(h);
    e1 = get_event(h);
    if (e0) HIP_TRY(hipEventRecord(e0, stream));
  }
  hipError_t e = herk_launch(kind, pl->tile_idx, ha, pl->nwg, stream, hk != nullptr);
  if (e != hipSuccess) return fail(CHI0_EDEVICE, "rank-K kernel launch: %s", hipGetErrorString(e));
  if (h->profiling && e0 && e1) {
    HIP_TRY(hipEventRecord(e1, stream));
    h->prof_pending.emplace_back(e0, e1);
  }
  e = reduce_launch(ra, pl->njobs, stream);
  if (e != hipSuccess) return fail(CHI0_EDEVICE, "reduction launch: %s", hipGetErrorString(e));
  return CHI0_OK;
}

// Partial-tile bytes of one frequency of a problem (one unit per tile).
double job_bytes(const TileConfig& tc, int npb) {
  std::vector<std::pair<int, int>> t;
  lower_tiles(npb, tc.tile, tc.tile_q, t);
  return static_cast<double>(t.size()) * tc.tile * tc.tile_q * 16.0;
}

// A call's rank-K work: the tile configuration is resolved once, then the
// problems run as one launch, or, when their (problem, frequency, tile) jobs
// alone would need more than the handle's cap of partial tiles, as a
// sequence of launches on the same stream over consecutive problems, a
// problem split into frequency ranges if one does not fit (frequencies are
// independent outputs).
int run_accumulate(chi0_ctx* h, const chi0_problem* probs, int32_t nprob, chi0_precision prec,
                   double delta_min, uint32_t flags, hipStream_t stream, int tile_override,
                   int mode = kWeightsChi0, const GatherHook* hk = nullptr) {
  const int kind = kind_of(prec);
  const int ntile = herk_tile_count(kind);
  if (ntile <= 0) return fail(CHI0_EUNSUPPORTED, "precision %d has no kernel in this library", prec);
  int tile_idx = tile_override >= 0 ? tile_override
                 : h->tile_sel[kind] >= 0 ? h->tile_sel[kind]
                 : h->tile_tuned[kind] >= 0 ? h->tile_tuned[kind]
                 : !hk ? tile_for(kind, probs, nprob) : herk_gather_tile(kind);
  if (tile_idx >= ntile) tile_idx = 0;
  if (hk && !herk_tile_gathers(kind, tile_idx)) tile_idx = herk_gather_tile(kind);
  if (hk && !herk_tile_gathers(kind, tile_idx))
    return fail(CHI0_EUNSUPPORTED, "precision %d has no gathering kernel", prec);
  h->tile_last[kind] = tile_idx;
  const TileConfig tc = herk_tile_config(kind, tile_idx);
  const double cap = h->partial_cap;
  double total = 0.0;
  for (int p = 0; p < nprob; ++p) total += job_bytes(tc, probs[p].npb) * probs[p].nomega;
  if (total <= cap)
    return run_accumulate_group(h, probs, nprob, prec, delta_min, flags, stream, tile_idx, mode, hk);
  // sub-problems: frequency ranges of each problem that fit the cap
  std::vector<chi0_problem> sub;
  std::vector<int> orig;
  std::vector<double> bytes;
  for (int p = 0; p < nprob; ++p) {
    const double per_w = job_bytes(tc, probs[p].npb);
    if (per_w > cap)
      return fail(CHI0_ENOMEM, "problem %d: one frequency needs %.3g bytes of partial tiles (limit %.3g)",
                  p, per_w, cap);
    const int wmax = static_cast<int>(std::min<double>(probs[p].nomega, std::floor(cap / per_w)));
    if (hk && wmax < probs[p].nomega)
      return fail(CHI0_ENOMEM, "gathered problem %d needs %.3g bytes of partial tiles (limit %.3g)", p,
                  per_w * probs[p].nomega, cap);
    const size_t n2 = static_cast<size_t>(probs[p].npb) * probs[p].npb;
    for (int w0 = 0; w0 < probs[p].nomega; w0 += wmax) {
      chi0_problem q = probs[p];
      q.nomega = std::min(wmax, probs[p].nomega - w0);
      q.omega = probs[p].omega ? probs[p].omega + w0 : nullptr;
      q.chi0 = static_cast<double2*>(probs[p].chi0) + static_cast<size_t>(w0) * n2;
      sub.push_back(q);
      orig.push_back(p);
      bytes.push_back(per_w * q.nomega);
    }
  }
  // consecutive sub-problems per launch while they fit
  for (size_t g0 = 0; g0 < sub.size();) {
    size_t g1 = g0;
    double acc = 0.0;
    while (g1 < sub.size() && (g1 == g0 || acc + bytes[g1] <= cap)) acc += bytes[g1++];
    GatherHook sh{};
    if (hk) sh = GatherHook{hk->rows, hk->wts, hk->off + orig[g0]};
    const int rc = run_accumulate_group(h, sub.data() + g0, static_cast<int32_t>(g1 - g0), prec,
                                        delta_min, flags, stream, tile_idx, mode, hk ? &sh : nullptr);
    if (rc) return rc;
    g0 = g1;
  }
  return CHI0_OK;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int validate_hist(const chi0_problem* probs, const chi0_hist* hists, int32_t nprob, chi0_ztype zt,
                  chi0_precision prec, double delta_min, uint32_t flags) {
  if (flags & ~static_cast<uint32_t>(CHI0_BF16_LOLO))
    return fail(CHI0_EINVAL, "unknown flag bits 0x%x", flags);
  int rc = validate_problems(probs, nprob, zt, prec, delta_min, 0);
  if (rc) return rc;
  if (nprob > 0 && !hists) return fail(CHI0_EINVAL, "hists is NULL");
  int64_t nbt = 0;
  for (int p = 0; p < nprob; ++p) {
    const chi0_hist& hs = hists[p];
    if (hs.nbins < 1) return fail(CHI0_EINVAL, "problem %d: nbins = %d < 1", p, hs.nbins);
    if (hs.nreal < 0) return fail(CHI0_EINVAL, "problem %d: nreal = %d < 0", p, hs.nreal);
    if (!hs.edges) return fail(CHI0_EINVAL, "problem %d: edges is NULL", p);
    nbt += hs.nbins;
    for (int j = 0; j <= hs.nbins; ++j) {
      if (!std::isfinite(hs.edges[j]) || !(hs.edges[j] > 0.0))
        return fail(CHI0_EINVAL, "problem %d: edges[%d] must be finite and > 0", p, j);
      if (j > 0 && !(hs.edges[j] > hs.edges[j - 1]))
        return fail(CHI0_EINVAL, "problem %d: edges must be strictly increasing", p);
    }
    if (!std::isfinite(hs.sigma) || hs.sigma < 0.0 || hs.sigma >= 1.0)
      return fail(CHI0_EINVAL, "problem %d: sigma must be in [0, 1)", p);
    if (hs.nreal > 0) {
      if (!hs.omega_re || !hs.chi0_re)
        return fail(CHI0_EINVAL, "problem %d: omega_re or chi0_re is NULL", p);
      if (!aligned(hs.chi0_re, 16)) return fail(CHI0_EINVAL, "problem %d: chi0_re not 16-byte aligned", p);
      for (int i = 0; i < hs.nreal; ++i) {
        const double w = hs.omega_re[i];
        if (!std::isfinite(w) || w < 0.0)
          return fail(CHI0_EINVAL, "problem %d: omega_re[%d] must be finite and >= 0", p, i);
        if (std::binary_search(hs.edges, hs.edges + hs.nbins + 1, w))
          return fail(CHI0_EINVAL, "problem %d: omega_re[%d] lies on a bin edge", p, i);
      }
    }
    if (hs.hist && !aligned(hs.hist, 16)) return fail(CHI0_EINVAL, "problem %d: hist not 16-byte aligned", p);
  }
  if (nbt > 16384) return fail(CHI0_EINVAL, "%lld bins in all, more than 16384", static_cast<long long>(nbt));
  if (prec == CHI0_PREC_FP32)
    return fail(CHI0_EUNSUPPORTED, "the histogram route runs on the FP64 and BF16x3 paths");
  return CHI0_OK;
}

// Records one pair can produce: 1 + the most edges inside one spread
// [x (1 - s), x (1 + s)]; every edge inside such a spread lies in
// [e_k, rho e_k) for the first edge e_k above its lower end, rho = (1+s)/(1-s).
int hist_records_per_pair(const chi0_hist& hs) {
  if (hs.sigma == 0.0) return 1;
  const double rho = (1.0 + hs.sigma) / (1.0 - hs.sigma) * (1.0 + 1e-12);
  int best = 0;
  int m = 0;
  for (int k = 0; k <= hs.nbins; ++k) {
    if (m < k) m = k;
    while (m <= hs.nbins && hs.edges[m] < rho * hs.edges[k]) ++m;
    best = std::max(best, m - k);
  }
  return 1 + best;
}

int run_hist(chi0_ctx* h, const chi0_problem* probs, const chi0_hist* hists, int32_t nprob,
             chi0_precision prec, double delta_min, uint32_t flags, hipStream_t stream) {
  const bool f64 = prec == CHI0_PREC_FP64;
  int R = 1;
  for (int p = 0; p < nprob; ++p) R = std::max(R, hist_records_per_pair(hists[p]));
  if (R > 64) return fail(CHI0_EINVAL, "a spread covers up to %d bins (more than 63)", R - 1);

  // blocks, record slots and bins
  std::vector<HistBlock> hb;
  std::vector<HistProb> hp(nprob);
  std::vector<double> dbl;          // edges of every problem
  std::vector<size_t> edge_off(nprob);
  int64_t nrs = 0, max_pairs = 0;
  int nbt = 0;
  for (int p = 0; p < nprob; ++p) {
    edge_off[p] = dbl.size();
    dbl.insert(dbl.end(), hists[p].edges, hists[p].edges + hists[p].nbins + 1);
    hp[p].sigma = hists[p].sigma;
    hp[p].nbins = hists[p].nbins;
    hp[p].bin0 = nbt;
    nbt += hists[p].nbins;
    for (int b = 0; b < probs[p].nblocks; ++b) {
      const chi0_block& bl = probs[p].blocks[b];
      const int64_t K = static_cast<int64_t>(bl.nocc) * bl.nunocc;
      if (K == 0) continue;
      HistBlock d;
      d.z = bl.z;
      d.eps_occ = bl.eps_occ;
      d.eps_unocc = bl.eps_unocc;
      d.wk = bl.wk;
      d.nocc = bl.nocc;
      d.nunocc = bl.nunocc;
      d.rec0 = nrs;
      d.prob = p;
      d.row_bytes = probs[p].npb * (f64 ? 16 : 8);
      hb.push_back(d);
      nrs += K * R;
      max_pairs = std::max(max_pairs, K);
    }
  }
  if (nrs > 0x7fffffffLL)
    return fail(CHI0_EINVAL, "%lld record slots (pairs x %d), more than 2^31-1", static_cast<long long>(nrs), R);
  const int nchunks = static_cast<int>((nrs + hist_chunk() - 1) / hist_chunk());
  const size_t wsz = f64 ? 8 : 4;
  int rc;
  const size_t rec_bytes = align256(nrs * 4) + align256(nrs * 8) + align256(nrs * 8);
  if ((rc = h->hist_rec.reserve(std::max<size_t>(rec_bytes, 256), &h->ws_gen))) return rc;
  const size_t sorted_bytes = align256(nrs * 8) + align256(nrs * wsz);
  if ((rc = h->hist_sorted.reserve(std::max<size_t>(sorted_bytes, 256), &h->ws_gen))) return rc;
  const size_t cnt_bytes = align256(static_cast<size_t>(nbt) * std::max(nchunks, 1) * 4) +
                           align256(static_cast<size_t>(nbt + 1) * 8);
  if ((rc = h->hist_cnt.reserve(cnt_bytes, &h->ws_gen))) return rc;
  char* rec = static_cast<char*>(h->hist_rec.p);
  int32_t* rbin = reinterpret_cast<int32_t*>(rec);
  double* rwt = reinterpret_cast<double*>(rec + align256(nrs * 4));
  uint64_t* rrow = reinterpret_cast<uint64_t*>(rec + align256(nrs * 4) + align256(nrs * 8));
  uint64_t* srow = static_cast<uint64_t*>(h->hist_sorted.p);
  void* swt = static_cast<char*>(h->hist_sorted.p) + align256(nrs * 8);
  int32_t* cnt = static_cast<int32_t*>(h->hist_cnt.p);
  int64_t* doff = reinterpret_cast<int64_t*>(static_cast<char*>(h->hist_cnt.p) +
                                             align256(static_cast<size_t>(nbt) * std::max(nchunks, 1) * 4));

  // tables A (edges | HistProb | HistBlock) and, after the bin counts are
  // known, tables B (Hilbert descriptors | slot and bin lists | real
  // frequencies | zero list) in one buffer sized for the most bins up front
  const size_t a_prob = align256(dbl.size() * 8);
  const size_t a_blk = a_prob + align256(hp.size() * sizeof(HistProb));
  const size_t a_bytes = a_blk + align256(std::max<size_t>(hb.size(), 1) * sizeof(HistBlock));
  int64_t nreal_all = 0;
  for (int p = 0; p < nprob; ++p) nreal_all += hists[p].nreal;
  const size_t b_hp = 0;
  const size_t b_int = align256(nprob * sizeof(HilbertProb));
  const size_t b_ore = b_int + align256(static_cast<size_t>(2 * nbt) * 4);
  const size_t b_zero = b_ore + align256(static_cast<size_t>(std::max<int64_t>(nreal_all, 1)) * 8);
  const size_t b_bytes = b_zero + align256(static_cast<size_t>(nbt) * sizeof(void*));
  if ((rc = h->hist_tab.reserve(a_bytes + b_bytes, &h->ws_gen))) return rc;
  char* dtab = static_cast<char*>(h->hist_tab.p);
  for (int p = 0; p < nprob; ++p) hp[p].edges = reinterpret_cast<const double*>(dtab) + edge_off[p];
  if ((rc = staging_reserve(h, a_bytes))) return rc;
  char* st = static_cast<char*>(h->staging);
  memcpy(st, dbl.data(), dbl.size() * 8);
  memcpy(st + a_prob, hp.data(), hp.size() * sizeof(HistProb));
  if (!hb.empty()) memcpy(st + a_blk, hb.data(), hb.size() * sizeof(HistBlock));
  HIP_TRY(hipMemcpyAsync(dtab, st, a_bytes, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipEventRecord(h->staging_done, stream));
  h->staging_pending = true;

  hipError_t e = hist_records_launch(reinterpret_cast<const HistBlock*>(dtab + a_blk),
                                     reinterpret_cast<const HistProb*>(dtab + a_prob),
                                     static_cast<int>(hb.size()), max_pairs, R, delta_min, rbin, rwt, rrow,
                                     h->d_status + kStNonpositive, stream);
  if (e != hipSuccess) return fail(CHI0_EDEVICE, "binning launch: %s", hipGetErrorString(e));
  e = hist_sort_launch(rbin, rwt, rrow, nrs, nbt, cnt, doff, srow, swt, f64, stream);
  if (e != hipSuccess) return fail(CHI0_EDEVICE, "bin sort launch: %s", hipGetErrorString(e));
  if (h->hist_off_host_n < static_cast<size_t>(nbt + 1)) {
    if (h->hist_off_host) hipHostFree(h->hist_off_host);
    h->hist_off_host = nullptr;
    h->hist_off_host_n = 0;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h->hist_off_host), (nbt + 1) * 8, hipHostMallocDefault));
    h->hist_off_host_n = nbt + 1;
  }
  HIP_TRY(hipMemcpyAsync(h->hist_off_host, doff, (nbt + 1) * 8, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  const int64_t* off = h->hist_off_host;

  h->hist_records = off[nbt];
  h->hist_bins_used = 0;
  for (int b = 0; b < nbt; ++b) h->hist_bins_used += off[b + 1] > off[b] ? 1 : 0;

  // one rank-K problem per non-empty bin
  std::vector<chi0_problem> iprob;
  std::vector<chi0_block> iblk;
  std::vector<int64_t> ioff;
  std::vector<std::vector<int32_t>> slots(nprob), bins(nprob);
  std::vector<int> empty_prob, empty_bin;
  size_t ws_mats = 0;
  std::vector<size_t> mat_off(nprob, 0);
  for (int p = 0; p < nprob; ++p) {
    mat_off[p] = ws_mats;
    const size_t n2 = static_cast<size_t>(probs[p].npb) * probs[p].npb;
    int used = 0;
    for (int j = 0; j < hists[p].nbins; ++j) {
      const int64_t c = off[hp[p].bin0 + j + 1] - off[hp[p].bin0 + j];
      if (c > 0x7fffffffLL) return fail(CHI0_EINVAL, "bin %d of problem %d holds more than 2^31-1 records", j, p);
      if (c > 0) {
        bins[p].push_back(j);
        slots[p].push_back(hists[p].hist ? j : used);
        ++used;
      } else if (hists[p].hist) {
        empty_prob.push_back(p);
        empty_bin.push_back(j);
      }
    }
    if (!hists[p].hist) ws_mats += static_cast<size_t>(used) * n2 * 16;
  }
  if ((rc = h->hist_mats.reserve(std::max<size_t>(ws_mats, 256), &h->ws_gen))) return rc;
  for (int p = 0; p < nprob; ++p) {
    const size_t n2 = static_cast<size_t>(probs[p].npb) * probs[p].npb;
    double2* base = hists[p].hist ? static_cast<double2*>(hists[p].hist)
                                  : reinterpret_cast<double2*>(static_cast<char*>(h->hist_mats.p) + mat_off[p]);
    for (size_t k = 0; k < bins[p].size(); ++k) {
      const int j = bins[p][k];
      chi0_block b{};
      b.nocc = static_cast<int32_t>(off[hp[p].bin0 + j + 1] - off[hp[p].bin0 + j]);
      b.nunocc = 1;
      iblk.push_back(b);
      chi0_problem q{};
      q.npb = probs[p].npb;
      q.nblocks = 1;
      q.nomega = 1;
      q.omega = probs[p].omega;
      q.chi0 = base + static_cast<size_t>(slots[p][k]) * n2;
      iprob.push_back(q);
      ioff.push_back(off[hp[p].bin0 + j]);
    }
  }
  for (size_t q = 0; q < iprob.size(); ++q) iprob[q].blocks = &iblk[q];

  // tables B: Hilbert descriptors, slot / bin lists, zero list; coefficients
  size_t coeff_bytes = 0;
  std::vector<size_t> coeff_off(nprob);
  int max_out = 0, max_bins = 0;
  int64_t max_n2 = 0;
  for (int p = 0; p < nprob; ++p) {
    coeff_off[p] = coeff_bytes;
    const int nout = probs[p].nomega + hists[p].nreal;
    coeff_bytes += align256(static_cast<size_t>(nout) * std::max<size_t>(bins[p].size(), 1) * 16);
    max_out = std::max(max_out, nout);
    max_bins = std::max(max_bins, static_cast<int>(bins[p].size()));
    max_n2 = std::max<int64_t>(max_n2, static_cast<int64_t>(probs[p].npb) * probs[p].npb);
  }
  if ((rc = h->hist_coeff.reserve(std::max<size_t>(coeff_bytes, 256), &h->ws_gen))) return rc;
  std::vector<int32_t> ints;
  std::vector<size_t> slot_off(nprob), bin_off(nprob);
  for (int p = 0; p < nprob; ++p) {
    slot_off[p] = ints.size();
    ints.insert(ints.end(), slots[p].begin(), slots[p].end());
    bin_off[p] = ints.size();
    ints.insert(ints.end(), bins[p].begin(), bins[p].end());
  }
  std::vector<double> oreal;
  std::vector<size_t> ore_off(nprob);
  for (int p = 0; p < nprob; ++p) {
    ore_off[p] = oreal.size();
    if (hists[p].nreal > 0) oreal.insert(oreal.end(), hists[p].omega_re, hists[p].omega_re + hists[p].nreal);
  }
  char* btab = dtab + a_bytes;
  std::vector<HilbertProb> hb2(nprob);
  for (int p = 0; p < nprob; ++p) {
    HilbertProb& x = hb2[p];
    x.hist = hists[p].hist ? static_cast<const double2*>(hists[p].hist)
                           : reinterpret_cast<const double2*>(static_cast<char*>(h->hist_mats.p) + mat_off[p]);
    x.slots = reinterpret_cast<const int32_t*>(btab + b_int) + slot_off[p];
    x.bins = reinterpret_cast<const int32_t*>(btab + b_int) + bin_off[p];
    x.edges = reinterpret_cast<const double*>(dtab) + edge_off[p];
    x.omega = probs[p].omega;
    x.omega_re = reinterpret_cast<const double*>(btab + b_ore) + ore_off[p];
    x.coeff = reinterpret_cast<double2*>(static_cast<char*>(h->hist_coeff.p) + coeff_off[p]);
    x.out = static_cast<double2*>(probs[p].chi0);
    x.out_re = static_cast<double2*>(hists[p].chi0_re);
    x.npb = probs[p].npb;
    x.nimag = probs[p].nomega;
    x.nreal = hists[p].nreal;
    x.nbins_used = static_cast<int32_t>(bins[p].size());
  }
  std::vector<double2*> zero_ptrs(empty_prob.size());
  for (size_t i = 0; i < empty_prob.size(); ++i)
    zero_ptrs[i] = static_cast<double2*>(hists[empty_prob[i]].hist) +
                   static_cast<size_t>(empty_bin[i]) * probs[empty_prob[i]].npb * probs[empty_prob[i]].npb;
  if ((rc = staging_reserve(h, b_bytes))) return rc;
  st = static_cast<char*>(h->staging);
  memcpy(st + b_hp, hb2.data(), nprob * sizeof(HilbertProb));
  if (!ints.empty()) memcpy(st + b_int, ints.data(), ints.size() * 4);
  if (!oreal.empty()) memcpy(st + b_ore, oreal.data(), oreal.size() * 8);
  if (!zero_ptrs.empty()) memcpy(st + b_zero, zero_ptrs.data(), zero_ptrs.size() * sizeof(void*));
  HIP_TRY(hipMemcpyAsync(btab, st, b_bytes, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipEventRecord(h->staging_done, stream));
  h->staging_pending = true;

  if (!iprob.empty()) {
    GatherHook hk{srow, swt, ioff.data()};
    rc = run_accumulate(h, iprob.data(), static_cast<int32_t>(iprob.size()), prec, 0.0,
                        flags & CHI0_BF16_LOLO, stream, -1, kWeightsChi0, &hk);
    if (rc) return rc;
  }
  // zero lists are grouped by problem size: one launch per distinct npb
  for (size_t i = 0; i < empty_prob.size();) {
    size_t k = i;
    const int npb = probs[empty_prob[i]].npb;
    while (k < empty_prob.size() && probs[empty_prob[k]].npb == npb) ++k;
    e = hist_zero_launch(reinterpret_cast<double2* const*>(btab + b_zero) + i, static_cast<int>(k - i),
                         static_cast<int64_t>(npb) * npb, stream);
    if (e != hipSuccess) return fail(CHI0_EDEVICE, "zero launch: %s", hipGetErrorString(e));
    i = k;
  }
  e = hilbert_launch(reinterpret_cast<const HilbertProb*>(btab + b_hp), nprob, max_out, max_bins, max_n2, stream);
  if (e != hipSuccess) return fail(CHI0_EDEVICE, "Hilbert launch: %s", hipGetErrorString(e));
  return CHI0_OK;
}

int validate_sigc(const sigc_problem* probs, int32_t nprob, chi0_ztype zt, chi0_precision prec,
                  uint32_t flags) {
  if (nprob < 0) return fail(CHI0_EINVAL, "nprob = %d < 0", nprob);
  if (nprob > 0 && !probs) return fail(CHI0_EINVAL, "probs is NULL");
  if (prec != CHI0_PREC_FP64 && prec != CHI0_PREC_FP32 && prec != CHI0_PREC_BF16X3)
    return fail(CHI0_EINVAL, "unknown precision %d", static_cast<int>(prec));
  if (zt != CHI0_Z_C128 && zt != CHI0_Z_C64)
    return fail(CHI0_EINVAL, "unknown Z type %d", static_cast<int>(zt));
  if (flags & ~static_cast<uint32_t>(CHI0_ACCUMULATE))
    return fail(CHI0_EINVAL, "unknown flag bits 0x%x", flags);
  for (int p = 0; p < nprob; ++p) {
    const sigc_problem& pr = probs[p];
    if (pr.nqp < 1) return fail(CHI0_EINVAL, "problem %d: nqp = %d < 1", p, pr.nqp);
    if (pr.nblocks < 0) return fail(CHI0_EINVAL, "problem %d: nblocks = %d < 0", p, pr.nblocks);
    if (pr.nblocks > 0 && !pr.blocks) return fail(CHI0_EINVAL, "problem %d: blocks is NULL", p);
    if (pr.nomega < 1) return fail(CHI0_EINVAL, "problem %d: nomega = %d < 1", p, pr.nomega);
    if (!pr.omega || !pr.eps_qp) return fail(CHI0_EINVAL, "problem %d: omega or eps_qp is NULL", p);
    for (int i = 0; i < pr.nomega; ++i) {
      if (!std::isfinite(pr.omega[i]) || pr.omega[i] < 0.0)
        return fail(CHI0_EINVAL, "problem %d: omega[%d] must be finite and >= 0", p, i);
      if (i > 0 && !(pr.omega[i] > pr.omega[i - 1]))
        return fail(CHI0_EINVAL, "problem %d: omega must be strictly increasing", p);
    }
    for (int n = 0; n < pr.nqp; ++n)
      if (!std::isfinite(pr.eps_qp[n])) return fail(CHI0_EINVAL, "problem %d: eps_qp[%d] not finite", p, n);
    if (!pr.sigc) return fail(CHI0_EINVAL, "problem %d: sigc is NULL", p);
    if (!aligned(pr.sigc, 16)) return fail(CHI0_EINVAL, "problem %d: sigc not 16-byte aligned", p);
    for (int b = 0; b < pr.nblocks; ++b) {
      const sigc_block& bl = pr.blocks[b];
      if (bl.nall < 0) return fail(CHI0_EINVAL, "problem %d block %d: nall = %d < 0", p, b, bl.nall);
      if (bl.nmu < 1) return fail(CHI0_EINVAL, "problem %d block %d: nmu = %d < 1", p, b, bl.nmu);
      if (static_cast<int64_t>(bl.nall) * bl.nmu > 0x7fffffffLL ||
          static_cast<int64_t>(bl.nall) * pr.nqp > 0x7fffffffLL)
        return fail(CHI0_EINVAL, "problem %d block %d: nall * nmu or nall * nqp above 2^31-1", p, b);
      if (!std::isfinite(bl.wk) || bl.wk < 0.0)
        return fail(CHI0_EINVAL, "problem %d block %d: wk must be finite and >= 0", p, b);
      if (bl.nall > 0) {
        if (!bl.z || !bl.wc || !bl.eps_mid)
          return fail(CHI0_EINVAL, "problem %d block %d: z, wc or eps_mid is NULL", p, b);
        if (!aligned(bl.z, 16) || !aligned(bl.wc, 16))
          return fail(CHI0_EINVAL, "problem %d block %d: z or wc not 16-byte aligned", p, b);
        for (int a = 0; a < bl.nall; ++a)
          if (!std::isfinite(bl.eps_mid[a]))
            return fail(CHI0_EINVAL, "problem %d block %d: eps_mid[%d] not finite", p, b, a);
      }
    }
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(pr.sigc);
    const uintptr_t a1 = a0 + static_cast<uintptr_t>(pr.nqp) * pr.nqp * 16;
    for (int q = 0; q < p; ++q) {
      const uintptr_t b0 = reinterpret_cast<uintptr_t>(probs[q].sigc);
      const uintptr_t b1 = b0 + static_cast<uintptr_t>(probs[q].nqp) * probs[q].nqp * 16;
      if (a0 < b1 && b0 < a1) return fail(CHI0_EINVAL, "problems %d and %d: outputs overlap", q, p);
    }
  }
  if (prec == CHI0_PREC_FP32)
    return fail(CHI0_EUNSUPPORTED, "the correlation self-energy runs on the FP64 and BF16x3 paths");
  if (zt != CHI0_Z_C128)
    return fail(CHI0_EUNSUPPORTED, "the correlation self-energy reads Z and W^c as CHI0_Z_C128");
  return CHI0_OK;
}

int run_sigc(chi0_ctx* h, const sigc_problem* probs, int32_t nprob, chi0_precision prec, uint32_t flags,
             hipStream_t stream) {
  const int T = sigc_tile();
  const bool bf16 = prec == CHI0_PREC_BF16X3;
  // first-contraction tiles: nu x r = 128 x 128 (FP64) or 256 x 128 (BF16x3)
  const int T1P = bf16 ? 256 : T, T1Q = T;
  // flat block list (blocks with nall = 0 contribute nothing and are dropped)
  struct Ref {
    int prob, blk;
  };
  std::vector<Ref> refs;
  int max_nqp = 0;
  for (int p = 0; p < nprob; ++p) {
    max_nqp = std::max(max_nqp, probs[p].nqp);
    for (int b = 0; b < probs[p].nblocks; ++b)
      if (probs[p].blocks[b].nall > 0) refs.push_back({p, b});
  }
  const int nb = static_cast<int>(refs.size());

  // chunks of consecutive blocks whose zw workspace stays under the cap
  std::vector<int> chunk0{0};
  int64_t zw_max = 0, cur = 0;
  std::vector<int64_t> zw_off(nb, 0), sp_off(nb, 0);
  int64_t sp_cur = 0, sp_max = 0;
  for (int i = 0; i < nb; ++i) {
    const sigc_problem& pr = probs[refs[i].prob];
    const sigc_block& bl = pr.blocks[refs[i].blk];
    const int64_t bytes = static_cast<int64_t>(align256(static_cast<size_t>(bl.nall) * bl.nmu * pr.nqp * 16));
    const int64_t groups = presplit_groups(bl.nmu);
    const int64_t sbytes =
        bf16 ? 2 * static_cast<int64_t>(align256(static_cast<size_t>(pr.nomega) * groups * bl.nmu * 16)) +
                   2 * static_cast<int64_t>(
                           align256(static_cast<size_t>(pr.nomega) * groups * bl.nall * pr.nqp * 16)) +
                   4 * static_cast<int64_t>(align256(
                           static_cast<size_t>(presplit_groups(static_cast<int64_t>(bl.nall) * bl.nmu)) *
                           pr.nqp * 16))
             : 0;
    // the split planes (weighted Z per mesh point) are held to four times the cap
    if (cur > 0 && (cur + bytes > h->sigc_zw_cap || sp_cur + sbytes > 4 * h->sigc_zw_cap)) {
      chunk0.push_back(i);
      cur = 0;
      sp_cur = 0;
    }
    zw_off[i] = cur;
    sp_off[i] = sp_cur;
    cur += bytes;
    sp_cur += sbytes;
    zw_max = std::max(zw_max, cur);
    sp_max = std::max(sp_max, sp_cur);
  }
  chunk0.push_back(nb);
  const int nchunks = static_cast<int>(chunk0.size()) - 1;

  // host-side tables: energies and meshes, block descriptors, problems, and
  // per chunk the units of both contractions and the reduction jobs
  std::vector<double> dbl;
  std::vector<size_t> qp_off(nprob), om_off(nprob), mid_off(nb);
  for (int p = 0; p < nprob; ++p) {
    qp_off[p] = dbl.size();
    dbl.insert(dbl.end(), probs[p].eps_qp, probs[p].eps_qp + probs[p].nqp);
    om_off[p] = dbl.size();
    dbl.insert(dbl.end(), probs[p].omega, probs[p].omega + probs[p].nomega);
  }
  size_t wt_bytes = 0;
  std::vector<size_t> wt_off(nb);
  int64_t max_wt_elems = 0;
  for (int i = 0; i < nb; ++i) {
    const sigc_problem& pr = probs[refs[i].prob];
    const sigc_block& bl = pr.blocks[refs[i].blk];
    mid_off[i] = dbl.size();
    dbl.insert(dbl.end(), bl.eps_mid, bl.eps_mid + bl.nall);
    wt_off[i] = wt_bytes;
    const int64_t elems = static_cast<int64_t>(bl.nall) * pr.nqp * pr.nomega;
    max_wt_elems = std::max(max_wt_elems, elems);
    wt_bytes += align256(static_cast<size_t>(elems) * 8);
  }

  struct ChunkTabs {
    std::vector<SigcUnit> u1, u2;
    std::vector<SigcJob> jobs;
    std::vector<int32_t> slots;
    int seg_len = 0;
  };
  std::vector<ChunkTabs> ct(nchunks);
  size_t max_part_units = 0;
  for (int c = 0; c < nchunks; ++c) {
    ChunkTabs& t = ct[c];
    int64_t rows_tiles = 0;
    for (int i = chunk0[c]; i < chunk0[c + 1]; ++i) {
      const sigc_problem& pr = probs[refs[i].prob];
      const sigc_block& bl = pr.blocks[refs[i].blk];
      const int64_t M = static_cast<int64_t>(bl.nall) * pr.nqp;
      const int tps = (bl.nmu + T1P - 1) / T1P;
      const int64_t tcs = (M + T1Q - 1) / T1Q;
      for (int64_t tc = 0; tc < tcs; ++tc)
        for (int tp = 0; tp < tps; ++tp) t.u1.push_back({i, tp, static_cast<int32_t>(tc), 0});
      const int tq = (pr.nqp + T - 1) / T;
      rows_tiles += static_cast<int64_t>(bl.nall) * bl.nmu * tq * tq;
    }
    // segment length: about four second-contraction units per CU; BF16x3
    // units are 256 x 128 tiles and one FP32 run each (a multiple of 16 rows,
    // at most 4096)
    const int64_t target = std::max<int64_t>(1, 4LL * h->ncu);
    int64_t seg;
    if (bf16) {
      int64_t rt = 0;
      for (int i = chunk0[c]; i < chunk0[c + 1]; ++i) {
        const sigc_problem& pr = probs[refs[i].prob];
        const sigc_block& bl = pr.blocks[refs[i].blk];
        rt += static_cast<int64_t>(bl.nall) * bl.nmu * ((pr.nqp + 255) / 256) * ((pr.nqp + T - 1) / T);
      }
      seg = (rt + target - 1) / target;
      seg = std::min<int64_t>(4096, std::max<int64_t>(256, (seg + 15) / 16 * 16));
    } else {
      seg = (rows_tiles + target - 1) / target;
      seg = std::max<int64_t>(64, (seg + 7) / 8 * 8);
      seg = std::min<int64_t>(seg, 0x40000000LL);
    }
    t.seg_len = static_cast<int>(seg);
    // units ordered (block, segment, tile) so the tiles of one segment are
    // adjacent; jobs per (problem, tile) list their slots in unit order
    std::vector<std::vector<int32_t>> tile_slots;
    std::vector<std::array<int, 3>> tile_key;
    std::unordered_map<int64_t, int> key_index;
    for (int i = chunk0[c]; i < chunk0[c + 1]; ++i) {
      const int p = refs[i].prob;
      const sigc_problem& pr = probs[p];
      const sigc_block& bl = pr.blocks[refs[i].blk];
      const int64_t K = static_cast<int64_t>(bl.nall) * bl.nmu;
      const int nseg = static_cast<int>((K + seg - 1) / seg);
      const int tq = (pr.nqp + T - 1) / T;
      auto add_slot = [&](int tp, int tc, int32_t slot) {
        const int64_t key = (static_cast<int64_t>(p) * tq + tp) * tq + tc;
        auto it = key_index.find(key);
        int k;
        if (it == key_index.end()) {
          k = static_cast<int>(tile_slots.size());
          key_index.emplace(key, k);
          tile_slots.emplace_back();
          tile_key.push_back({p, tp, tc});
        } else {
          k = it->second;
        }
        tile_slots[k].push_back(slot);
      };
      if (bf16) {
        // unit (block, 256-row tile tp2, column tile tc, segment): partial
        // tiles 2 unit (rows 256 tp2 ..) and 2 unit + 1 (rows 256 tp2 + 128 ..)
        const int tp2n = (pr.nqp + 255) / 256;
        for (int sg = 0; sg < nseg; ++sg)
          for (int tp2 = 0; tp2 < tp2n; ++tp2)
            for (int tc = 0; tc < tq; ++tc) {
              const int32_t un = static_cast<int32_t>(t.u2.size());
              for (int h2 = 0; h2 < 2; ++h2)
                if (2 * tp2 + h2 < tq) add_slot(2 * tp2 + h2, tc, 2 * un + h2);
              t.u2.push_back({i, tp2, tc, sg});
            }
      } else {
        for (int sg = 0; sg < nseg; ++sg)
          for (int tp = 0; tp < tq; ++tp)
            for (int tc = 0; tc < tq; ++tc) {
              add_slot(tp, tc, static_cast<int32_t>(t.u2.size()));
              t.u2.push_back({i, tp, tc, sg});
            }
      }
    }
    for (size_t k = 0; k < tile_slots.size(); ++k) {
      SigcJob j;
      j.prob = tile_key[k][0];
      j.tp = tile_key[k][1];
      j.tc = tile_key[k][2];
      j.slot0 = static_cast<int32_t>(t.slots.size());
      j.nslot = static_cast<int32_t>(tile_slots[k].size());
      j.pad = 0;
      t.slots.insert(t.slots.end(), tile_slots[k].begin(), tile_slots[k].end());
      t.jobs.push_back(j);
    }
    max_part_units = std::max(max_part_units, (bf16 ? 2 : 1) * t.u2.size());
  }

  // workspace
  int rc;
  size_t acc_bytes = 0;
  std::vector<size_t> acc_off(nprob);
  for (int p = 0; p < nprob; ++p) {
    acc_off[p] = acc_bytes;
    acc_bytes += align256(static_cast<size_t>(probs[p].nqp) * probs[p].nqp * 16);
  }
  if ((rc = h->sigc_acc.reserve(std::max<size_t>(acc_bytes, 256), &h->ws_gen))) return rc;
  if ((rc = h->sigc_wt.reserve(std::max<size_t>(wt_bytes, 256), &h->ws_gen))) return rc;
  if ((rc = h->sigc_zw.reserve(std::max<size_t>(static_cast<size_t>(zw_max), 256), &h->ws_gen))) return rc;
  if (bf16 && (rc = h->sigc_split.reserve(std::max<size_t>(static_cast<size_t>(sp_max), 256), &h->ws_gen)))
    return rc;
  if ((rc = h->sigc_part.reserve(std::max<size_t>(max_part_units * T * T * 16, 256), &h->ws_gen)))
    return rc;

  // one device table: doubles | descs | probs | per chunk (u1 | u2 | jobs | slots)
  size_t off = align256(dbl.size() * 8);
  const size_t desc_off = off;
  off += align256(static_cast<size_t>(nb) * sizeof(SigcDesc));
  const size_t prob_off = off;
  off += align256(static_cast<size_t>(nprob) * sizeof(SigcProb));
  std::vector<std::array<size_t, 4>> coff(nchunks);
  for (int c = 0; c < nchunks; ++c) {
    coff[c][0] = off;
    off += align256(ct[c].u1.size() * sizeof(SigcUnit));
    coff[c][1] = off;
    off += align256(ct[c].u2.size() * sizeof(SigcUnit));
    coff[c][2] = off;
    off += align256(ct[c].jobs.size() * sizeof(SigcJob));
    coff[c][3] = off;
    off += align256(ct[c].slots.size() * sizeof(int32_t));
  }
  const size_t tab_bytes = off;
  if ((rc = h->sigc_tab.reserve(tab_bytes, &h->ws_gen))) return rc;
  char* dtab = static_cast<char*>(h->sigc_tab.p);
  const double* ddbl = reinterpret_cast<const double*>(dtab);

  std::vector<SigcDesc> descs(nb);
  for (int i = 0; i < nb; ++i) {
    const int p = refs[i].prob;
    const sigc_problem& pr = probs[p];
    const sigc_block& bl = pr.blocks[refs[i].blk];
    SigcDesc& d = descs[i];
    d.z = static_cast<const double2*>(bl.z);
    d.wc = static_cast<const double2*>(bl.wc);
    d.zw = reinterpret_cast<double2*>(static_cast<char*>(h->sigc_zw.p) + zw_off[i]);
    d.wt = reinterpret_cast<double*>(static_cast<char*>(h->sigc_wt.p) + wt_off[i]);
    d.eps_mid = ddbl + mid_off[i];
    d.eps_qp = ddbl + qp_off[p];
    d.omega = ddbl + om_off[p];
    d.wk = bl.wk;
    d.nall = bl.nall;
    d.nmu = bl.nmu;
    d.nqp = pr.nqp;
    d.nomega = pr.nomega;
    d.prob = p;
    d.groups = static_cast<int32_t>(presplit_groups(bl.nmu));
    d.wsp = nullptr;
    d.wsp_plane = 0;
    d.zsp = nullptr;
    d.zsp_plane = 0;
    d.zwsp = nullptr;
    d.zksp = nullptr;
    d.k_plane = 0;
    d.kgroups = static_cast<int32_t>(presplit_groups(static_cast<int64_t>(bl.nall) * bl.nmu));
    d.pad2 = 0;
    if (bf16) {
      char* base = static_cast<char*>(h->sigc_split.p) + sp_off[i];
      d.wsp_plane = static_cast<int64_t>(align256(static_cast<size_t>(pr.nomega) * d.groups * bl.nmu * 16));
      d.zsp_plane = static_cast<int64_t>(
          align256(static_cast<size_t>(pr.nomega) * d.groups * bl.nall * pr.nqp * 16));
      d.wsp = base;
      d.zsp = base + 2 * d.wsp_plane;
      d.k_plane = static_cast<int64_t>(align256(static_cast<size_t>(d.kgroups) * pr.nqp * 16));
      d.zwsp = static_cast<char*>(d.zsp) + 2 * d.zsp_plane;
      d.zksp = static_cast<char*>(d.zwsp) + 2 * d.k_plane;
    }
  }
  std::vector<SigcProb> ptab(nprob);
  for (int p = 0; p < nprob; ++p) {
    ptab[p].acc = reinterpret_cast<double2*>(static_cast<char*>(h->sigc_acc.p) + acc_off[p]);
    ptab[p].out = static_cast<double2*>(probs[p].sigc);
    ptab[p].nqp = probs[p].nqp;
    ptab[p].pad = 0;
  }
  if ((rc = staging_reserve(h, tab_bytes))) return rc;
  char* st = static_cast<char*>(h->staging);
  memcpy(st, dbl.data(), dbl.size() * 8);
  if (nb) memcpy(st + desc_off, descs.data(), nb * sizeof(SigcDesc));
  memcpy(st + prob_off, ptab.data(), nprob * sizeof(SigcProb));
  for (int c = 0; c < nchunks; ++c) {
    if (!ct[c].u1.empty()) memcpy(st + coff[c][0], ct[c].u1.data(), ct[c].u1.size() * sizeof(SigcUnit));
    if (!ct[c].u2.empty()) memcpy(st + coff[c][1], ct[c].u2.data(), ct[c].u2.size() * sizeof(SigcUnit));
    if (!ct[c].jobs.empty()) memcpy(st + coff[c][2], ct[c].jobs.data(), ct[c].jobs.size() * sizeof(SigcJob));
    if (!ct[c].slots.empty())
      memcpy(st + coff[c][3], ct[c].slots.data(), ct[c].slots.size() * sizeof(int32_t));
  }
  HIP_TRY(hipMemcpyAsync(dtab, st, tab_bytes, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipEventRecord(h->staging_done, stream));
  h->staging_pending = true;

  const SigcDesc* d_desc = reinterpret_cast<const SigcDesc*>(dtab + desc_off);
  const SigcProb* d_prob = reinterpret_cast<const SigcProb*>(dtab + prob_off);
  hipError_t e = sigc_clear_launch(d_prob, nprob, max_nqp, stream);
  if (e != hipSuccess) return fail(CHI0_EDEVICE, "clear launch: %s", hipGetErrorString(e));
  e = sigc_weights_launch(d_desc, nb, max_wt_elems, stream);
  if (e != hipSuccess) return fail(CHI0_EDEVICE, "weight launch: %s", hipGetErrorString(e));
  for (int c = 0; c < nchunks; ++c) {
    SigcArgs a1;
    a1.units = reinterpret_cast<const SigcUnit*>(dtab + coff[c][0]);
    a1.descs = d_desc;
    a1.partials = nullptr;
    a1.nunits = static_cast<int32_t>(ct[c].u1.size());
    a1.seg_len = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->profiling) {
      e0 = get_event(h);
      e1 = get_event(h);
    }
    int max_kg = 0;
    if (bf16) {
      int max_nmu = 0, max_gw = 0, max_gz = 0;
      int64_t max_m = 0;
      max_kg = 0;
      for (int i = chunk0[c]; i < chunk0[c + 1]; ++i) {
        max_nmu = std::max(max_nmu, descs[i].nmu);
        max_gw = std::max(max_gw, descs[i].nomega * descs[i].groups);
        max_gz = std::max(max_gz, descs[i].groups);
        max_kg = std::max(max_kg, descs[i].kgroups);
        max_m = std::max<int64_t>(max_m, static_cast<int64_t>(descs[i].nall) * descs[i].nqp);
      }
      e = sigc_presplit_launch(d_desc + chunk0[c], chunk0[c + 1] - chunk0[c], max_nmu, max_m, max_gw, max_gz,
                               stream);
      if (e == hipSuccess) e = sigc_split_rows_launch(d_desc + chunk0[c], chunk0[c + 1] - chunk0[c], 1, max_nqp,
                                                      max_kg, stream);
      if (e != hipSuccess) return fail(CHI0_EDEVICE, "pre-split launch: %s", hipGetErrorString(e));
    }
    if (h->profiling && e0) HIP_TRY(hipEventRecord(e0, stream));
    e = bf16 ? sigc_bf16x3_launch(a1, stream) : sigc_zw_launch(h->sigc_variant, a1, stream);
    if (e != hipSuccess) return fail(CHI0_EDEVICE, "first contraction launch: %s", hipGetErrorString(e));
    if (h->profiling && e0 && e1) {
      HIP_TRY(hipEventRecord(e1, stream));
      h->prof_pending.emplace_back(e0, e1);
    }
    SigcArgs a2;
    a2.units = reinterpret_cast<const SigcUnit*>(dtab + coff[c][1]);
    a2.descs = d_desc;
    a2.partials = static_cast<double2*>(h->sigc_part.p);
    a2.nunits = static_cast<int32_t>(ct[c].u2.size());
    a2.seg_len = ct[c].seg_len;
    if (bf16) {
      e = sigc_split_rows_launch(d_desc + chunk0[c], chunk0[c + 1] - chunk0[c], 0, max_nqp, max_kg, stream);
      if (e == hipSuccess) e = sigc_bf16x3_zwz_launch(a2, stream);
    } else {
      e = sigc_zwz_launch(a2, stream);
    }
    if (e != hipSuccess) return fail(CHI0_EDEVICE, "second contraction launch: %s", hipGetErrorString(e));
    e = sigc_reduce_launch(reinterpret_cast<const SigcJob*>(dtab + coff[c][2]),
                           reinterpret_cast<const int32_t*>(dtab + coff[c][3]), a2.partials, d_prob,
                           static_cast<int>(ct[c].jobs.size()), stream);
    if (e != hipSuccess) return fail(CHI0_EDEVICE, "reduction launch: %s", hipGetErrorString(e));
  }
  e = sigc_store_launch(d_prob, nprob, max_nqp, (flags & CHI0_ACCUMULATE) != 0, stream);
  if (e != hipSuccess) return fail(CHI0_EDEVICE, "store launch: %s", hipGetErrorString(e));
  return CHI0_OK;
}

// Fixed workspace of the no-allocation inverse (dielectric_invert_noalloc):
// a device array of CHI0_NOALLOC_SCRATCH_BYTES that every GPU the library
// runs on holds until the process ends.  On the host its name is only a
// stand-in; the device address, different on every GPU, is looked up once
// per device (chi0_create) and used instead.
static __device__ __align__(256) char scratch[CHI0_NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
std::vector<char*> g_scratch_ptr;  // per device; NULL until looked up

// Looks up this device's copy of `scratch` (the device must be current).
int scratch_lookup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device >= static_cast<int>(g_scratch_ptr.size())) g_scratch_ptr.resize(device + 1, nullptr);
  if (g_scratch_ptr[device]) return CHI0_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    hipGetLastError();
    return fail(CHI0_EDEVICE, "device address of the no-allocation scratch on device %d: %s", device,
                hipGetErrorString(e));
  }
  g_scratch_ptr[device] = static_cast<char*>(p);
  return CHI0_OK;
}

char* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return device < static_cast<int>(g_scratch_ptr.size()) ? g_scratch_ptr[device] : nullptr;
}

// Argument checks shared by the two inverse entry points.
int validate_invert(chi0_handle h, int32_t npb, int32_t nomega, const double* vsqrt,
                    const void* chi0, const void* eps, const void* eps_inv, const void* wc,
                    uint32_t flags) {
  if (npb < 1) return fail(CHI0_EINVAL, "npb = %d < 1", npb);
  if (nomega < 1) return fail(CHI0_EINVAL, "nomega = %d < 1", nomega);
  if (flags & ~static_cast<uint32_t>(CHI0_OUT_WC | CHI0_INV_METHOD_MASK))
    return fail(CHI0_EINVAL, "unknown flag bits 0x%x", flags);
  const uint32_t method = flags & CHI0_INV_METHOD_MASK;
  if (method != CHI0_INV_GJ && method != CHI0_INV_HPD && method != CHI0_INV_HPD_FALLBACK_GJ)
    return fail(CHI0_EINVAL, "unknown inversion method %u", method);
  if (!vsqrt || !chi0 || !eps_inv) return fail(CHI0_EINVAL, "vsqrt, chi0 and eps_inv must be non-NULL");
  if ((flags & CHI0_OUT_WC) && !wc) return fail(CHI0_EINVAL, "CHI0_OUT_WC set but wc is NULL");
  if (!aligned(chi0, 16) || !aligned(eps_inv, 16) || (eps && !aligned(eps, 16)) ||
      ((flags & CHI0_OUT_WC) && !aligned(wc, 16)) || !aligned(vsqrt, 8))
    return fail(CHI0_EINVAL, "buffers must be 16-byte aligned (vsqrt 8-byte)");
  const size_t bytes = static_cast<size_t>(nomega) * npb * npb * 16;
  auto overlap = [bytes](const void* a, const void* b) {
    if (!a || !b) return false;
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bytes && y < x + bytes;
  };
  if (overlap(eps_inv, chi0) || overlap(eps_inv, eps) || ((flags & CHI0_OUT_WC) && (overlap(wc, eps_inv) || overlap(wc, chi0))))
    return fail(CHI0_EINVAL, "eps_inv / wc must not overlap chi0, eps or each other");
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  return CHI0_OK;
}

// Workspace of one inversion call: either the handle's growing buffers or
// pieces of the fixed no-allocation array.
struct InvWs {
  double2* work = nullptr;               // [nomega][npb][npb] eps being inverted
  double2 *hpd_p = nullptr, *hpd_c = nullptr, *hpd_dinv = nullptr;
  double2* wrow = nullptr;               // Gauss-Jordan pivot rows
  int32_t *piv = nullptr, *perm = nullptr;
};

// Layout of an inversion's workspace from byte 0 of one region (every piece
// 256-byte aligned); returns the bytes used.
size_t inv_layout(int32_t npb, int32_t nomega, char* base, InvWs* ws) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  const size_t n = static_cast<size_t>(npb), w = static_cast<size_t>(nomega);
  const size_t hb = static_cast<size_t>(hpd_block_width()), gb = static_cast<size_t>(gj_panel_width());
  InvWs t;
  t.work = reinterpret_cast<double2*>(take(w * n * n * 16));
  t.hpd_p = reinterpret_cast<double2*>(take(w * n * hb * 16));
  t.hpd_c = reinterpret_cast<double2*>(take(w * n * hb * 16));
  t.hpd_dinv = reinterpret_cast<double2*>(take(w * hb * hb * 16));
  t.wrow = reinterpret_cast<double2*>(take(w * gb * n * 16));
  t.piv = reinterpret_cast<int32_t*>(take(w * n * 4));
  t.perm = reinterpret_cast<int32_t*>(take(w * n * 4));
  if (ws) *ws = t;
  return off;
}

// eps = 1 - v^1/2 chi0 v^1/2 and its inverse.  fixed: the workspace to use
// (the no-allocation entry point); NULL: the handle's buffers, grown as
// needed.
int run_invert(chi0_ctx* h, int32_t npb, int32_t nomega, const double* vsqrt, const void* chi0,
               void* eps, void* eps_inv, void* wc, uint32_t flags, hipStream_t s,
               const InvWs* fixed = nullptr) {
  const size_t bytes = static_cast<size_t>(nomega) * npb * npb * 16;
  const uint32_t method = flags & CHI0_INV_METHOD_MASK;
  double2* wc_out = (flags & CHI0_OUT_WC) ? static_cast<double2*>(wc) : nullptr;
  int rc;
  debug_log("inverse: npb %d, %d frequencies, method %u%s, workspace %s", npb, nomega, method,
       wc_out ? ", W^c" : "", fixed ? "fixed array" : "handle buffers");
  if (!fixed && (rc = h->gj_work.reserve(bytes, &h->ws_gen))) return rc;
  double2* work = fixed ? fixed->work : static_cast<double2*>(h->gj_work.p);
  hipError_t e = dielectric_build_launch(static_cast<const double2*>(chi0), vsqrt, work,
                                         static_cast<double2*>(eps), npb, nomega, s);
  if (e != hipSuccess) return fail(CHI0_EDEVICE, "eps build launch: %s", hipGetErrorString(e));

  if (method != CHI0_INV_GJ) {
    const int nb = hpd_block_width();
    if (!fixed) {
      if ((rc = h->hpd_p.reserve(static_cast<size_t>(nomega) * npb * nb * 16, &h->ws_gen))) return rc;
      if ((rc = h->hpd_c.reserve(static_cast<size_t>(nomega) * npb * nb * 16, &h->ws_gen))) return rc;
      if ((rc = h->hpd_dinv.reserve(static_cast<size_t>(nomega) * nb * nb * 16, &h->ws_gen))) return rc;
    }
    double2* pb = fixed ? fixed->hpd_p : static_cast<double2*>(h->hpd_p.p);
    double2* cb = fixed ? fixed->hpd_c : static_cast<double2*>(h->hpd_c.p);
    double2* di = fixed ? fixed->hpd_dinv : static_cast<double2*>(h->hpd_dinv.p);
    const bool fallback = method == CHI0_INV_HPD_FALLBACK_GJ;
    e = hpd_status_clear_launch(h->d_status, s);
    for (int k0 = 0; k0 < npb && e == hipSuccess; k0 += nb)
      e = hpd_step_launch(work, di, pb, cb, npb, nomega, k0, std::min(nb, npb - k0), h->d_status,
                          !fallback, s);
    if (e == hipSuccess)
      e = hpd_finish_launch(work, static_cast<double2*>(eps_inv), wc_out, vsqrt, npb, nomega, s);
    if (e != hipSuccess) return fail(CHI0_EDEVICE, "HPD inverse launch: %s", hipGetErrorString(e));
    if (!fallback) return CHI0_OK;
    // fallback: wait for this call's sweeps and redo the pivoted inverse if
    // a pivot was not positive
    int32_t st[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(st, h->d_status, sizeof(st), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (!st[1]) return CHI0_OK;
    e = dielectric_build_launch(static_cast<const double2*>(chi0), vsqrt, work, nullptr, npb,
                                nomega, s);
    if (e != hipSuccess) return fail(CHI0_EDEVICE, "eps build launch: %s", hipGetErrorString(e));
  }

  const int nb = gj_panel_width();
  if (!fixed) {
    if ((rc = h->gj_wrow.reserve(static_cast<size_t>(nomega) * nb * npb * 16, &h->ws_gen))) return rc;
    if ((rc = h->gj_piv.reserve(static_cast<size_t>(nomega) * npb * 4, &h->ws_gen))) return rc;
    if ((rc = h->gj_perm.reserve(static_cast<size_t>(nomega) * npb * 4, &h->ws_gen))) return rc;
  }
  double2* wrow = fixed ? fixed->wrow : static_cast<double2*>(h->gj_wrow.p);
  int32_t* piv = fixed ? fixed->piv : static_cast<int32_t*>(h->gj_piv.p);
  int32_t* perm = fixed ? fixed->perm : static_cast<int32_t*>(h->gj_perm.p);
  // Each panel of nb columns is eliminated as sub-panels: a sub-panel is
  // factored by one workgroup per frequency, then applied to the panel's
  // other columns by the interchange / pivot-row and update kernels
  // restricted to the panel (all CUs); the whole panel is then applied to
  // every other column.
  const int sb = gj_subpanel_width();
  for (int k0 = 0; k0 < npb; k0 += nb) {
    const int nbk = std::min(nb, npb - k0);
    for (int j0 = 0; j0 < nbk && e == hipSuccess; j0 += sb) {
      const int sw = std::min(sb, nbk - j0);
      e = gj_panel_launch(work, npb, nomega, k0 + j0, sw, piv, h->d_status, s);
      if (e == hipSuccess && sw < nbk)
        e = gj_swap_extract_launch(work, wrow, npb, nomega, k0 + j0, sw, piv, k0, k0 + nbk, s);
      if (e == hipSuccess && sw < nbk)
        e = gj_update_launch(work, wrow, npb, nomega, k0 + j0, sw, k0, k0 + nbk, s);
    }
    if (e == hipSuccess) e = gj_swap_extract_launch(work, wrow, npb, nomega, k0, nbk, piv, 0, npb, s);
    if (e == hipSuccess) e = gj_update_launch(work, wrow, npb, nomega, k0, nbk, 0, npb, s);
    if (e != hipSuccess) return fail(CHI0_EDEVICE, "Gauss-Jordan launch: %s", hipGetErrorString(e));
  }
  e = gj_finish_launch(work, static_cast<double2*>(eps_inv), wc_out, vsqrt, piv, perm, npb, nomega,
                       s);
  if (e != hipSuccess) return fail(CHI0_EDEVICE, "Gauss-Jordan finish launch: %s", hipGetErrorString(e));
  return CHI0_OK;
}

}  // namespace

extern "C" {

int chi0_version(void) { return 10000; }

const char* chi0_status_string(int s) {
  switch (s) {
    case CHI0_OK: return "ok";
    case CHI0_EINVAL: return "invalid argument";
    case CHI0_ENOMEM: return "device allocation failed";
    case CHI0_EDEVICE: return "HIP device or launch failure";
    case CHI0_ENOTHPD: return "eps is not Hermitian positive definite";
    case CHI0_ESINGULAR: return "zero pivot while inverting eps";
    case CHI0_EUNSUPPORTED: return "unsupported combination";
  }
  return "unknown status";
}

const char* chi0_last_error(void) { return g_err.c_str(); }

int chi0_create(chi0_handle* out, int device) {
  if (!out) return fail(CHI0_EINVAL, "handle pointer is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    hipGetLastError();
    return fail(CHI0_EDEVICE, "no HIP device visible");
  }
  if (device < 0 || device >= ndev) return fail(CHI0_EINVAL, "device %d out of range [0, %d)", device, ndev);
  HIP_TRY(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(CHI0_EDEVICE, "device %d is %s; libchi0 is built for gfx950 only", device, prop.gcnArchName);
  std::unique_ptr<chi0_ctx> h(new chi0_ctx());
  h->device = device;
  h->ncu = prop.multiProcessorCount;
  int rc = scratch_lookup(device);
  if (rc) return rc;
  HIP_TRY(hipMalloc(&h->d_status, 64));
  HIP_TRY(hipMemset(h->d_status, 0, 64));
  HIP_TRY(hipEventCreateWithFlags(&h->staging_done, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&h->last_done, hipEventDisableTiming));
  *out = h.release();
  return CHI0_OK;
}

int chi0_destroy(chi0_handle h) {
  if (!h) return CHI0_OK;
  hipSetDevice(h->device);
  hipDeviceSynchronize();
  h->plans.clear();
  h->partials.release();
  h->wts.release();
  h->zsplit.release();
  h->sync_prog.release();
  h->gj_work.release();
  h->gj_wrow.release();
  h->gj_piv.release();
  h->gj_perm.release();
  h->hpd_p.release();
  h->hpd_c.release();
  h->hpd_dinv.release();
  h->sigc_tab.release();
  h->sigc_wt.release();
  h->sigc_zw.release();
  h->sigc_part.release();
  h->sigc_acc.release();
  h->sigc_split.release();
  h->gather_plan.reset();
  h->hist_tab.release();
  h->hist_rec.release();
  h->hist_sorted.release();
  h->hist_cnt.release();
  h->hist_mats.release();
  h->hist_coeff.release();
  if (h->hist_off_host) hipHostFree(h->hist_off_host);
  if (h->d_status) hipFree(h->d_status);
  if (h->staging) hipHostFree(h->staging);
  if (h->staging_done) hipEventDestroy(h->staging_done);
  if (h->last_done) hipEventDestroy(h->last_done);
  for (auto& pr : h->prof_pending) {
    hipEventDestroy(pr.first);
    hipEventDestroy(pr.second);
  }
  for (auto e : h->event_pool) hipEventDestroy(e);
  delete h;
  return CHI0_OK;
}

int sigx_accumulate(chi0_handle h, const sigx_problem* probs, int32_t nprob, chi0_ztype zt,
                    chi0_precision prec, uint32_t flags, void* hip_stream) {
  int rc = validate_sigx(probs, nprob, zt, prec, flags);
  if (rc) return rc;
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  if (nprob == 0) return CHI0_OK;
  HIP_TRY(hipSetDevice(h->device));
  // the exchange sum is the same weighted Hermitian rank-K update: rows
  // (n', mu) of nqp values, weight w_k v_mu, one "frequency", output -S
  std::vector<chi0_problem> cp(nprob);
  std::vector<std::vector<chi0_block>> cb(nprob);
  for (int p = 0; p < nprob; ++p) {
    cb[p].resize(std::max(1, probs[p].nblocks));
    for (int b = 0; b < probs[p].nblocks; ++b) {
      const sigx_block& s = probs[p].blocks[b];
      chi0_block& d = cb[p][b];
      d.nocc = s.nocc;
      d.nunocc = s.nmu;
      d.z = s.z;
      d.eps_occ = nullptr;
      d.eps_unocc = s.v;
      d.wk = s.wk;
    }
    cp[p].npb = probs[p].nqp;
    cp[p].nblocks = probs[p].nblocks;
    cp[p].blocks = cb[p].data();
    cp[p].nomega = 1;
    cp[p].omega = nullptr;
    cp[p].chi0 = probs[p].sigx;
  }
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((rc = call_begin(h, s))) return rc;
  return call_end(h, s, run_accumulate(h, cp.data(), nprob, prec, 0.0, flags, s, -1, kWeightsCoulomb));
}

int sigc_accumulate(chi0_handle h, const sigc_problem* probs, int32_t nprob, chi0_ztype zt,
                    chi0_precision prec, uint32_t flags, void* hip_stream) {
  int rc = validate_sigc(probs, nprob, zt, prec, flags);
  if (rc) return rc;
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  if (nprob == 0) return CHI0_OK;
  HIP_TRY(hipSetDevice(h->device));
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((rc = call_begin(h, s))) return rc;
  return call_end(h, s, run_sigc(h, probs, nprob, prec, flags, s));
}

int chi0_hist_accumulate(chi0_handle h, const chi0_problem* probs, const chi0_hist* hists, int32_t nprob,
                         chi0_ztype zt, chi0_precision prec, double delta_min, uint32_t flags,
                         void* hip_stream) {
  int rc = validate_hist(probs, hists, nprob, zt, prec, delta_min, flags);
  if (rc) return rc;
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  if (nprob == 0) return CHI0_OK;
  HIP_TRY(hipSetDevice(h->device));
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((rc = call_begin(h, s))) return rc;
  return call_end(h, s, run_hist(h, probs, hists, nprob, prec, delta_min, flags, s));
}

int chi0_hist_stats(chi0_handle h, int64_t* records, int32_t* bins_used) {
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  if (records) *records = h->hist_records;
  if (bins_used) *bins_used = h->hist_bins_used;
  return CHI0_OK;
}

int sigc_set_variant(chi0_handle h, int32_t variant) {
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  if (variant < 0 || variant >= sigc_zw_variants())
    return fail(CHI0_EINVAL, "variant %d out of range [0, %d)", variant, sigc_zw_variants());
  h->sigc_variant = variant;
  return CHI0_OK;
}

int chi0_set_partial_cap(chi0_handle h, int64_t bytes) {
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  if (bytes < 0) return fail(CHI0_EINVAL, "cap %lld < 0", static_cast<long long>(bytes));
  h->partial_cap = bytes == 0 ? kMaxPartialBytes : static_cast<double>(bytes);
  return CHI0_OK;
}

int sigc_set_workspace_cap(chi0_handle h, int64_t bytes) {
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  if (bytes < 0) return fail(CHI0_EINVAL, "cap %lld < 0", static_cast<long long>(bytes));
  h->sigc_zw_cap = bytes == 0 ? (int64_t(4) << 30) : bytes;
  return CHI0_OK;
}

int chi0_accumulate(chi0_handle h, const chi0_problem* probs, int32_t nprob, chi0_ztype zt,
                    chi0_precision prec, double delta_min, uint32_t flags, void* hip_stream) {
  int rc = validate_problems(probs, nprob, zt, prec, delta_min, flags);
  if (rc) return rc;
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  if (nprob == 0) return CHI0_OK;
  HIP_TRY(hipSetDevice(h->device));
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((rc = call_begin(h, s))) return rc;
  return call_end(h, s, run_accumulate(h, probs, nprob, prec, delta_min, flags, s, -1));
}

int dielectric_invert(chi0_handle h, int32_t npb, int32_t nomega, const double* vsqrt,
                      const void* chi0, void* eps, void* eps_inv, void* wc, uint32_t flags,
                      void* hip_stream) {
  int rc = validate_invert(h, npb, nomega, vsqrt, chi0, eps, eps_inv, wc, flags);
  if (rc) return rc;
  HIP_TRY(hipSetDevice(h->device));
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((rc = call_begin(h, s))) return rc;
  return call_end(h, s, run_invert(h, npb, nomega, vsqrt, chi0, eps, eps_inv, wc, flags, s));
}

int dielectric_invert_noalloc(chi0_handle h, int32_t npb, int32_t nomega, const double* vsqrt,
                              const void* chi0, void* eps, void* eps_inv, void* wc, uint32_t flags,
                              void* hip_stream) {
  int rc = validate_invert(h, npb, nomega, vsqrt, chi0, eps, eps_inv, wc, flags);
  if (rc) return rc;
  const size_t need = inv_layout(npb, nomega, nullptr, nullptr);
  if (need > static_cast<size_t>(CHI0_NOALLOC_SCRATCH_BYTES))
    return fail(CHI0_EINVAL, "npb = %d, nomega = %d needs %zu bytes of workspace; the no-allocation "
                "inverse has %zu", npb, nomega, need, static_cast<size_t>(CHI0_NOALLOC_SCRATCH_BYTES));
  char* base = scratch_of(h->device);
  if (!base) return fail(CHI0_EDEVICE, "no-allocation scratch of device %d not looked up", h->device);
  InvWs ws;
  inv_layout(npb, nomega, base, &ws);
  HIP_TRY(hipSetDevice(h->device));
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((rc = call_begin(h, s))) return rc;
  return call_end(h, s, run_invert(h, npb, nomega, vsqrt, chi0, eps, eps_inv, wc, flags, s, &ws));
}

int chi0_sync(chi0_handle h) {
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  HIP_TRY(hipSetDevice(h->device));
  HIP_TRY(hipDeviceSynchronize());
  int32_t st[kStWords] = {0, 0, 0, 0};
  HIP_TRY(hipMemcpy(st, h->d_status, sizeof(st), hipMemcpyDeviceToHost));
  if (st[kStZeroPivot] || st[kStHpdSeen] || st[kStNonpositive]) {
    HIP_TRY(hipMemset(h->d_status, 0, sizeof(st)));
    if (st[kStNonpositive])
      return fail(CHI0_EINVAL, "%d pair(s) with D = eps_unocc - eps_occ <= 0 since the last sync "
                  "(they contributed nothing)%s", st[kStNonpositive],
                  st[kStZeroPivot] || st[kStHpdSeen] ? "; an inversion also failed" : "");
    if (st[kStZeroPivot]) return fail(CHI0_ESINGULAR, "a zero pivot was met while inverting eps");
    return fail(CHI0_ENOTHPD, "a non-positive pivot was met: eps is not Hermitian positive definite");
  }
  return CHI0_OK;
}

int chi0_tile_count(chi0_precision prec) {
  const int k = kind_of(prec);
  return k < 0 ? fail(CHI0_EINVAL, "unknown precision") : herk_tile_count(k);
}

int chi0_tile_info(chi0_precision prec, int32_t tile, int32_t* tile_p, int32_t* tile_q,
                   int32_t* kchunk, int32_t* flush_len) {
  const int k = kind_of(prec);
  if (k < 0) return fail(CHI0_EINVAL, "unknown precision");
  if (tile < 0 || tile >= herk_tile_count(k)) return fail(CHI0_EINVAL, "tile %d out of range", tile);
  const TileConfig tc = herk_tile_config(k, tile);
  if (tile_p) *tile_p = tc.tile;
  if (tile_q) *tile_q = tc.tile_q;
  if (kchunk) *kchunk = tc.kchunk;
  if (flush_len) *flush_len = tc.flush;
  return CHI0_OK;
}

int chi0_tile_diag_skip(chi0_precision prec, int32_t tile) {
  const int k = kind_of(prec);
  if (k < 0) return fail(CHI0_EINVAL, "unknown precision");
  if (tile < 0 || tile >= herk_tile_count(k)) return fail(CHI0_EINVAL, "tile %d out of range", tile);
  const TileConfig tc = herk_tile_config(k, tile);
  return tc.diag_skip && tc.tile == 2 * tc.tile_q ? 1 : 0;
}

int chi0_tile_lists(chi0_precision prec, int32_t tile) {
  const int k = kind_of(prec);
  if (k < 0) return fail(CHI0_EINVAL, "unknown precision");
  if (tile < 0 || tile >= herk_tile_count(k)) return fail(CHI0_EINVAL, "tile %d out of range", tile);
  return std::max(1, static_cast<int>(herk_tile_config(k, tile).wave_lists));
}

int chi0_set_tile(chi0_handle h, chi0_precision prec, int32_t tile) {
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  const int k = kind_of(prec);
  if (k < 0) return fail(CHI0_EINVAL, "unknown precision");
  if (tile < -1 || tile >= herk_tile_count(k)) return fail(CHI0_EINVAL, "tile %d out of range", tile);
  h->tile_sel[k] = tile;
  return CHI0_OK;
}

int chi0_get_tile(chi0_handle h, chi0_precision prec, int32_t* tile) {
  if (!h || !tile) return fail(CHI0_EINVAL, "NULL argument");
  const int k = kind_of(prec);
  if (k < 0) return fail(CHI0_EINVAL, "unknown precision");
  *tile = h->tile_sel[k] >= 0 ? h->tile_sel[k] : h->tile_tuned[k] >= 0 ? h->tile_tuned[k]
                                                                         : herk_default_tile(k);
  return CHI0_OK;
}

int chi0_tile_choice(chi0_precision prec, const chi0_problem* probs, int32_t nprob, int32_t* tile) {
  if (!tile) return fail(CHI0_EINVAL, "tile is NULL");
  const int k = kind_of(prec);
  if (k < 0) return fail(CHI0_EINVAL, "unknown precision");
  if (nprob < 0 || (nprob > 0 && !probs)) return fail(CHI0_EINVAL, "bad problem list");
  for (int p = 0; p < nprob; ++p) {
    if (probs[p].npb < 1) return fail(CHI0_EINVAL, "problem %d: npb = %d < 1", p, probs[p].npb);
    if (probs[p].nblocks < 0 || (probs[p].nblocks > 0 && !probs[p].blocks))
      return fail(CHI0_EINVAL, "problem %d: bad block list", p);
    for (int b = 0; b < probs[p].nblocks; ++b)
      if (probs[p].blocks[b].nocc < 0 || probs[p].blocks[b].nunocc < 0)
        return fail(CHI0_EINVAL, "problem %d block %d: negative count", p, b);
  }
  *tile = tile_for(k, probs, nprob);
  return CHI0_OK;
}

int chi0_last_tile(chi0_handle h, chi0_precision prec, int32_t* tile) {
  if (!h || !tile) return fail(CHI0_EINVAL, "NULL argument");
  const int k = kind_of(prec);
  if (k < 0) return fail(CHI0_EINVAL, "unknown precision");
  *tile = h->tile_last[k];
  return CHI0_OK;
}

int chi0_set_flush(chi0_handle h, int32_t pairs) {
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  if (pairs != 0 && (pairs < 16 || pairs > 65536 || pairs % 16 != 0))
    return fail(CHI0_EINVAL, "flush length %d must be 0 or a multiple of 16 in [16, 65536]", pairs);
  h->flush_override = pairs;
  return CHI0_OK;
}

int chi0_set_xcd_slack(chi0_handle h, int32_t stages) {
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  if (stages < -2 || stages > 1 << 20)
    return fail(CHI0_EINVAL, "XCD lockstep slack %d must be -2, -1 or in [0, 2^20]", stages);
  h->xcd_slack = stages;
  return CHI0_OK;
}

int chi0_autotune(chi0_handle h, const chi0_problem* probs, int32_t nprob, chi0_ztype zt,
                  chi0_precision prec, double delta_min, int32_t reps, int32_t* best,
                  double* ms_out, void* hip_stream) {
  int rc = validate_problems(probs, nprob, zt, prec, delta_min, 0);
  if (rc) return rc;
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  if (reps < 1) return fail(CHI0_EINVAL, "reps must be >= 1");
  HIP_TRY(hipSetDevice(h->device));
  const int k = kind_of(prec);
  const int n = herk_tile_count(k);
  if (n <= 0) return fail(CHI0_EUNSUPPORTED, "precision has no kernel in this library");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((rc = call_begin(h, s))) return rc;
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    hipEventDestroy(a);
    return fail(CHI0_EDEVICE, "event creation failed");
  }
  int bi = 0;
  double bms = 1e300;
  const bool prof = h->profiling;
  h->profiling = false;
  for (int t = 0; t < n; ++t) {
    rc = run_accumulate(h, probs, nprob, prec, delta_min, 0, s, t);  // warm-up + plan
    if (rc) break;
    hipEventRecord(a, s);
    for (int r = 0; r < reps && !rc; ++r) rc = run_accumulate(h, probs, nprob, prec, delta_min, 0, s, t);
    hipEventRecord(b, s);
    if (rc) break;
    if (hipEventSynchronize(b) != hipSuccess) { rc = fail(CHI0_EDEVICE, "autotune sync failed"); break; }
    float ms = 0.f;
    hipEventElapsedTime(&ms, a, b);
    const double per = ms / reps;
    if (ms_out) ms_out[t] = per;
    if (per < bms) {
      bms = per;
      bi = t;
    }
  }
  h->profiling = prof;
  hipEventDestroy(a);
  hipEventDestroy(b);
  rc = call_end(h, s, rc);
  if (rc) return rc;
  h->tile_tuned[k] = bi;
  if (best) *best = bi;
  return CHI0_OK;
}

int chi0_plan_inspect(const chi0_problem* probs, int32_t nprob, chi0_precision prec,
                      int32_t tile, int32_t nwg, int32_t* nunits, int32_t* njobs,
                      int32_t* units_out, int32_t units_cap, double* load_max,
                      double* load_mean) {
  if (nprob < 0 || (nprob > 0 && !probs)) return fail(CHI0_EINVAL, "bad problem list");
  if (nwg < 1) return fail(CHI0_EINVAL, "nwg must be >= 1");
  const int k = kind_of(prec);
  if (k < 0) return fail(CHI0_EINVAL, "unknown precision");
  if (tile < 0 || tile >= herk_tile_count(k)) return fail(CHI0_EINVAL, "tile %d out of range", tile);
  for (int p = 0; p < nprob; ++p) {
    if (probs[p].npb < 1 || probs[p].nomega < 1 || probs[p].nblocks < 0 ||
        (probs[p].nblocks > 0 && !probs[p].blocks))
      return fail(CHI0_EINVAL, "problem %d: bad shape", p);
    for (int b = 0; b < probs[p].nblocks; ++b)
      if (probs[p].blocks[b].nocc < 0 || probs[p].blocks[b].nunocc < 0)
        return fail(CHI0_EINVAL, "problem %d block %d: negative size", p, b);
  }
  HostPlan hp;
  plan_host(herk_tile_config(k, tile), nwg, probs, nprob, hp);
  // one row per frequency of every unit (a frequency-group unit gives one
  // row for each of its frequencies, all owned by the unit's list)
  if (nunits) *nunits = static_cast<int32_t>(hp.nslots);
  if (njobs) *njobs = static_cast<int32_t>(hp.jobs.size());
  if (units_out) {
    if (units_cap < hp.nslots)
      return fail(CHI0_EINVAL, "units_out holds %d units, %lld needed", units_cap,
                  static_cast<long long>(hp.nslots));
    // per row: prob, iw, tp, tq, b0, p0, b1, p1, slot, work list
    std::vector<int32_t> owner(hp.units.size(), -1);
    const int nlists = static_cast<int>(hp.wg_off.size()) - 1;
    for (int w = 0; w < nlists; ++w)
      for (int i = hp.wg_off[w]; i < hp.wg_off[w + 1]; ++i) owner[hp.wg_units[i]] = w;
    size_t row = 0;
    for (size_t u = 0; u < hp.units.size(); ++u) {
      const Unit& x = hp.units[u];
      for (int w = 0; w < std::max(1, static_cast<int>(x.nw)); ++w, ++row) {
        int32_t* o = units_out + 10 * row;
        o[0] = x.prob; o[1] = x.iw + w; o[2] = x.tp; o[3] = x.tq; o[4] = x.b0;
        o[5] = x.p0; o[6] = x.b1; o[7] = x.p1; o[8] = x.slot + w * x.wstride; o[9] = owner[u];
      }
    }
  }
  double mx = 0.0, sum = 0.0;
  for (double v : hp.wg_load) {
    mx = std::max(mx, v);
    sum += v;
  }
  if (load_max) *load_max = mx;
  if (load_mean) *load_mean = hp.wg_load.empty() ? 0.0 : sum / hp.wg_load.size();
  return CHI0_OK;
}

int chi0_profile_enable(chi0_handle h, int on) {
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  h->profiling = on != 0;
  return CHI0_OK;
}

int chi0_profile_read(chi0_handle h, double* kernel_ms, int64_t* launches) {
  if (!h) return fail(CHI0_EINVAL, "handle is NULL");
  for (auto& pr : h->prof_pending) {
    HIP_TRY(hipEventSynchronize(pr.second));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
    h->prof_ms += ms;
    h->prof_launches += 1;
    h->event_pool.push_back(pr.first);
    h->event_pool.push_back(pr.second);
  }
  h->prof_pending.clear();
  if (kernel_ms) *kernel_ms = h->prof_ms;
  if (launches) *launches = h->prof_launches;
  h->prof_ms = 0.0;
  h->prof_launches = 0;
  return CHI0_OK;
}

}  // extern "C"
