// pf_runtime.hip - the C-ABI of include/pf.h: handle, stage planner, device
// buffers, kernel launches, state access and error handling.
#include <hip/hip_runtime.h>

#include <cstddef>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/pf.h"
#include "pf_host.h"

using namespace pfk;
using namespace pfh;

namespace {

thread_local std::string g_create_error;

// The allocator of handles and batches created from now on (pf_set_allocator).
std::mutex g_alloc_mu;
DevAllocator g_alloc;

}  // namespace

namespace pfh {
DevAllocator current_allocator() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc;
}
// The message pf_last_error(NULL) returns (failed creates and calls without
// a handle).
void set_create_error(const char* msg) { g_create_error = msg; }
}  // namespace pfh

struct pf_handle {
  int kind = 0, d = 0, D = 1, mk = 0;
  int dtype = PF_DTYPE_F32;
  int resampler = PF_RESAMPLE_MULTINOMIAL;
  uint64_t N = 0, radix = 0;
  uint64_t seed = 0;
  uint32_t sid = 0;
  bool global = false;
  std::vector<StagePlan> stages;
  hipStream_t stream = nullptr;
  size_t tsz = 4, ssz = 4;  // compute / storage element sizes
  void* x[2] = {nullptr, nullptr};
  void* lw[2] = {nullptr, nullptr};
  int cur = 0;
  void* mp = nullptr;        // ModelParams<T>
  // tile partials: a ring of `ring` steps, part_stride elements each
  void* partials = nullptr;
  uint32_t ring = 1;
  uint64_t part_stride = 0;
  // steps whose partials have not been reduced yet (oldest first)
  std::vector<FinStep> pending;
  Ctl* ctl = nullptr;
  pf_estimate_t* hist = nullptr;
  uint32_t hist_cap = 1;
  uint32_t* anc = nullptr;
  void* gcdf = nullptr;
  void* gcoarse = nullptr;
  void* gx = nullptr;
  uint32_t* gfirst = nullptr;  // systematic global draw: first output per tile, then the work items
  uint32_t* gwork = nullptr;
  double* gpre = nullptr;
  double* gscale = nullptr;
  uint32_t g_tile = 0, g_ntiles = 0, g_nt = 256, g_ppt = 1;
  uint64_t t = 0;
  uint64_t u = 0;            // offset-slot index: one per kernel launch of the tile path
  bool full_cycle = false;   // every step runs all S stages
  uint64_t model_hash = 0;   // FNV-1a of the model parameters (checkpoint check)
  bool lw_zero = true;       // every log-weight is 0 (global path and island filter)
  // island filter (AIRPF): islands of M = 2^log2M particles, m = 2^log2m
  uint32_t island = 0, log2M = 0, log2m = 0;
  bool island_no_swap = true;
  uint32_t* ianc = nullptr;  // within-island ancestors (N)
  void* isl_lw = nullptr;    // carried log-weight per island (m, compute type)
  uint32_t* isl_src = nullptr;  // source island of each destination island (m)
  void* isl_lv = nullptr;    // island log-weights when they do not fit in LDS (m, compute type)
  // ESS-gated stages (threshold > 0): stage table, per-tile ESS records of a
  // stage, the stage slots' grid and LDS, tiles of the weighting launch
  double ess_theta = 0.0;
  AdStage* stab = nullptr;
  void* ess_part = nullptr;
  uint32_t ad_grid = 0, w_ntiles = 0;
  size_t ad_lds = 0;
  uint64_t bytes = 0;
  pf_status sticky = PF_OK;
  bool numeric = false;  // the device flagged unusable weights (sticky until re-initialised)
  std::string err;
  DevAllocator dalloc_fn;    // the allocator current at create time
  std::vector<void*> allocs;
};

namespace {

// Most stages of a plan (radix 2 at N = 2^30 has 30).
constexpr uint32_t kMaxStages = 32;

pf_status fail(pf_handle* h, pf_status s, const std::string& msg) {
  if (h) {
    h->err = msg;
    if (s == PF_E_HIP) h->sticky = PF_E_STATE;
  } else {
    g_create_error = msg;
  }
  return s;
}

pf_status hip_fail(pf_handle* h, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(h, PF_E_HIP, m);
}

pf_status dalloc(pf_handle* h, void** p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  hipError_t e = dev_alloc(h->dalloc_fn, p, bytes);
  if (e == hipErrorInvalidValue)
    return fail(h, PF_E_INVALID, "the installed allocator returned a pointer not aligned to 256 bytes");
  if (e != hipSuccess)
    return fail(h, PF_E_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  h->allocs.push_back(*p);
  h->bytes += bytes;
  return PF_OK;
}

// Checkpoint blob: this header, then the d state planes (storage type), the
// raw log-weights (compute type) and the estimate record of the last step.
struct BlobHeader {
  char magic[8];
  uint32_t version, header_bytes;
  uint64_t n_particles, radix, model_hash, seed;
  int32_t kind, d, resampler, dtype;
  uint32_t stream_id, lw_zero;
  uint32_t next_stage, reserved;  // ESS-gated stages: where the next resampling starts
  uint64_t t;
  double log_norm, offset;
  uint64_t x_bytes, lw_bytes, rec_bytes;
};
constexpr char kBlobMagic[8] = {'P', 'F', 'B', 'F', 'L', 'Y', 'C', 'K'};
constexpr uint32_t kBlobVersion = 2;

hipError_t launch(pf_handle* h, const LaunchReq& rq, const void* args) {
  switch (h->dtype) {
    case PF_DTYPE_F32: return launch_f32(rq, args, h->stream);
    case PF_DTYPE_BF16: return launch_bf16(rq, args, h->stream);
    default: return launch_f64(rq, args, h->stream);
  }
}

template <typename T, typename S> void fill_common(pf_handle* h, StepArgs<T, S>& a) {
  std::memset(&a, 0, sizeof(a));
  a.x_in = reinterpret_cast<const S*>(h->x[h->cur]);
  a.x_out = reinterpret_cast<S*>(h->x[h->cur ^ 1]);
  a.lw_in = reinterpret_cast<const T*>(h->lw[h->cur]);
  a.lw_out = reinterpret_cast<T*>(h->lw[h->cur ^ 1]);
  a.anc = h->anc;
  a.mp = reinterpret_cast<const ModelParams<T>*>(h->mp);
  a.part_out = reinterpret_cast<T*>(h->partials) + (size_t)(h->t % h->ring) * h->part_stride;
  a.ctl = h->ctl;
  a.hist = h->hist;
  a.hist_cap = h->hist_cap;
  a.d = (uint32_t)h->d;
  a.N = h->N;
  a.k0 = (uint32_t)(h->seed & 0xFFFFFFFFu);
  a.k1 = (uint32_t)(h->seed >> 32);
  a.sid = h->sid;
  a.systematic = h->resampler == PF_RESAMPLE_SYSTEMATIC ? 1 : 0;
  a.gcdf = reinterpret_cast<T*>(h->gcdf);
  a.gcoarse = reinterpret_cast<T*>(h->gcoarse);
  a.gx = reinterpret_cast<S*>(h->gx);
  a.gpre = h->gpre;
  a.gscale = h->gscale;
  a.gfirst = h->gfirst;
  a.gwork = h->gwork;
}

template <typename T, typename S>
pf_status run_init(pf_handle* h) {
  StepArgs<T, S> a;
  fill_common<T, S>(h, a);
  // the initial cloud goes to the current buffer
  a.x_out = reinterpret_cast<S*>(h->x[h->cur]);
  a.lw_out = reinterpret_cast<T*>(h->lw[h->cur]);
  LaunchReq rq{};
  rq.what = LW_INIT;
  rq.D = h->D;
  rq.mk = h->mk;
  rq.nt = 256;
  const uint64_t npair = h->N / 2;
  uint64_t g = (npair + 255) / 256;
  rq.grid = (uint32_t)(g > 65536 ? 65536 : g);
  hipError_t e = launch(h, rq, &a);
  if (e != hipSuccess) return hip_fail(h, e, "init kernel launch");
  h->t = 0;
  h->u = 0;
  h->lw_zero = true;
  h->pending.clear();
  return PF_OK;
}

pf_status flush(pf_handle* h);

// One launch of the fused tile kernel for stage k with the given flags.
template <typename T, typename S>
pf_status launch_stage(pf_handle* h, const double* y_host, const void* y_dev, uint32_t k, uint32_t flags,
                       uint32_t utau) {
  const StagePlan& sp = h->stages[k];
  StepArgs<T, S> a;
  fill_common<T, S>(h, a);
  if (y_dev) {
    a.y_dev = reinterpret_cast<const T*>(y_dev);
  } else {
    for (int j = 0; j < h->d; ++j) a.y_val[j] = (T)y_host[j];
  }
  a.t = (uint32_t)h->t;
  a.k = k;
  a.u = (uint32_t)h->u;
  a.flags = flags;
  a.utau = utau;
  a.radix = sp.r;
  a.log2r = sp.log2r;
  a.log2R = sp.log2R;
  a.lnr = (T)std::log((double)sp.r);
  a.log2C = sp.log2C;
  a.pad = sp.pad;
  a.xrow = sp.xrow;
  a.ntiles = sp.ntiles;
  LaunchReq rq{};
  rq.what = LW_STEP_TILE;
  rq.D = h->D;
  rq.mk = h->mk;
  rq.nt = sp.nt;
  rq.ppt = sp.ppt;
  rq.blockpath = sp.blockpath;
  rq.full = h->d == h->D ? 1 : 0;
  rq.grid = sp.ntiles;
  rq.lds = sp.lds;
  hipError_t e = launch(h, rq, &a);
  if (e != hipSuccess) return hip_fail(h, e, "step kernel launch");
  h->cur ^= 1;
  h->u += 1;
  return PF_OK;
}

// One step of the island filter (Algorithm 4): the within-island launch of
// the tile kernel (weights, estimate partials, Algorithm 5), the island
// stages (Algorithm 6 or 7, one block) and the island gather with the
// mutation. The output is unweighted.
template <typename T, typename S>
pf_status run_island_step(pf_handle* h, const double* y_host, const void* y_dev) {
  const StagePlan& sp = h->stages[0];
  StepArgs<T, S> a;
  fill_common<T, S>(h, a);
  if (y_dev) {
    a.y_dev = reinterpret_cast<const T*>(y_dev);
  } else {
    for (int j = 0; j < h->d; ++j) a.y_val[j] = (T)y_host[j];
  }
  a.t = (uint32_t)h->t;
  a.k = 0;
  a.u = (uint32_t)h->u;
  a.flags = kStepWeight | kStepIsland | (h->lw_zero ? kStepLwZero : 0u);
  a.utau = (uint32_t)h->t + 1u;
  a.radix = sp.r;
  a.log2r = sp.log2r;
  a.log2R = sp.log2R;
  a.lnr = (T)std::log((double)sp.r);
  a.log2C = sp.log2C;
  a.pad = sp.pad;
  a.xrow = sp.xrow;
  a.ntiles = sp.ntiles;
  a.anc = h->ianc;
  a.isl_lw = reinterpret_cast<T*>(h->isl_lw);
  LaunchReq rq{};
  rq.what = LW_STEP_TILE;
  rq.D = h->D;
  rq.mk = h->mk;
  rq.nt = sp.nt;
  rq.ppt = sp.ppt;
  rq.blockpath = sp.blockpath;
  rq.full = h->d == h->D ? 1 : 0;
  rq.island = 1;
  rq.grid = sp.ntiles;
  rq.lds = sp.lds;
  hipError_t e = launch(h, rq, &a);
  if (e != hipSuccess) return hip_fail(h, e, "within-island launch");
  h->u += 1;

  const uint32_t m = 1u << h->log2m;
  IslandArgs ia{};
  ia.isl_lw = h->isl_lw;
  ia.lv = h->isl_lv;
  ia.src = h->isl_src;
  ia.m = m;
  ia.log2m = h->log2m;
  ia.tau = (uint32_t)h->t + 1u;
  ia.sid = h->sid;
  ia.k0 = a.k0;
  ia.k1 = a.k1;
  ia.no_swap = h->island_no_swap ? 1u : 0u;
  ia.use_lds = (size_t)m * (h->tsz + 8) <= kIslandLdsBytes ? 1u : 0u;
  // LDS of a launch over blocks of mb islands running nst stages
  auto draw_lds = [&](IslandArgs& x, uint32_t mb, uint32_t nst) {
    x.uni_all = (size_t)mb * (h->tsz + 4 + 4 * (size_t)nst) <= kIslandLdsBytes ? 1u : 0u;
    return !x.use_lds ? (size_t)0 : (size_t)mb * (h->tsz + 4 + (x.uni_all ? 4 * (size_t)nst : 4));
  };
  LaunchReq rd{};
  rd.what = LW_ISLAND_DRAW;
  rd.D = h->D;
  rd.mk = h->mk;
  constexpr uint32_t kLgBlockIslands = 10;
  if (ia.use_lds && h->log2m > kLgBlockIslands) {
    // the first stages inside blocks of 1024 islands, one block each (one
    // pair per thread), then the rest on one block
    IslandArgs p1 = ia;
    p1.mb = 1u << kLgBlockIslands;
    p1.s_begin = 0;
    p1.s_end = kLgBlockIslands;
    p1.lv_out = 1;
    rd.grid = m >> kLgBlockIslands;
    rd.nt = 512;
    rd.lds = draw_lds(p1, p1.mb, kLgBlockIslands);
    rd.ia = &p1;
    e = launch(h, rd, &a);
    if (e != hipSuccess) return hip_fail(h, e, "island stage launch");
    IslandArgs p2 = ia;
    p2.mb = m;
    p2.s_begin = kLgBlockIslands;
    p2.s_end = h->log2m;
    p2.from_prev = 1;
    rd.grid = 1;
    rd.nt = 1024;
    rd.lds = draw_lds(p2, m, h->log2m - kLgBlockIslands);
    rd.ia = &p2;
    e = launch(h, rd, &a);
    if (e != hipSuccess) return hip_fail(h, e, "island stage launch");
  } else {
    ia.mb = m;
    ia.s_begin = 0;
    ia.s_end = h->log2m;
    rd.grid = 1;
    rd.nt = 1024;
    rd.lds = draw_lds(ia, m, h->log2m);
    rd.ia = &ia;
    e = launch(h, rd, &a);
    if (e != hipSuccess) return hip_fail(h, e, "island stage launch");
  }

  StepArgs<T, S> g = a;
  g.anc = h->anc;
  g.isl_src = h->isl_src;
  g.isl_anc = h->ianc;
  g.log2M = h->log2M;
  LaunchReq rg{};
  rg.what = LW_ISLAND_GATHER;
  rg.D = h->D;
  rg.mk = h->mk;
  // one block per destination island when the island has 1024, 2048 or
  // 4096 particles, its states fit in LDS and a plane of it spans at least
  // 8 KB: below that the scattered loads of the plain gather stay within few
  // cache lines per wave and it is the faster one (LG-8 with islands of
  // 1024: 18.7 against 19.9 us; SV with islands of 4096: 63.8 against 24.2)
  const size_t island_vals = (size_t)h->d << h->log2M;
  if (h->log2M >= 10 && h->log2M <= 12 && ((size_t)h->tsz << h->log2M) >= 8192u &&
      island_vals * h->tsz <= kIslandGatherLds) {
    rg.grid = m;
    rg.ppt = 1 << (h->log2M - 10);
    rg.lds = island_vals * h->tsz;
  } else {
    const uint64_t blocks = (h->N / 2 + 255) / 256;
    rg.grid = (uint32_t)std::min<uint64_t>(blocks, 65536);
  }
  e = launch(h, rg, &g);
  if (e != hipSuccess) return hip_fail(h, e, "island gather launch");
  h->cur ^= 1;
  h->lw_zero = true;
  return PF_OK;
}

// One step with ESS-gated stages (FP32 states): weighting, a decision, S
// stage slots each followed by a decision (a slot the decisions have closed
// does nothing), the mutation. The stages run in place on the current
// buffers; the mutation writes the other pair.
template <typename T, typename S>
pf_status run_adaptive_step(pf_handle* h, const double* y_host, const void* y_dev) {
  if constexpr (!(std::is_same<T, float>::value && std::is_same<S, float>::value)) {
    return fail(h, PF_E_UNSUPPORTED, "ESS-gated stages need FP32 states");
  } else {
    StepArgs<T, S> a;
    fill_common<T, S>(h, a);
    if (y_dev) {
      a.y_dev = reinterpret_cast<const T*>(y_dev);
    } else {
      for (int j = 0; j < h->d; ++j) a.y_val[j] = (T)y_host[j];
    }
    a.t = (uint32_t)h->t;
    a.u = (uint32_t)h->u;
    a.utau = (uint32_t)h->t + 1u;
    a.lw_out = reinterpret_cast<T*>(h->lw[h->cur]);  // weights stored in place
    LaunchReq rq{};
    rq.D = h->D;
    rq.mk = h->mk;
    rq.what = LW_AD_WEIGHT;
    rq.grid = h->w_ntiles;
    hipError_t e = launch(h, rq, &a);
    if (e != hipSuccess) return hip_fail(h, e, "weighting launch");

    AdDecide ad{};
    ad.ctl = h->ctl;
    ad.stab = h->stab;
    ad.rec = a.part_out;
    ad.stride = (uint32_t)partial_stride(h->D);
    ad.ntiles_first = h->w_ntiles;
    ad.first = 1u;
    ad.S = (uint32_t)h->stages.size();
    ad.t = (uint32_t)h->t;
    ad.N = h->N;
    ad.theta = h->ess_theta;
    ad.hist = h->hist;
    ad.hist_cap = h->hist_cap;
    LaunchReq rd{};
    rd.D = h->D;
    rd.mk = h->mk;
    rd.what = LW_AD_DECIDE;
    rd.ad = &ad;
    e = launch(h, rd, &a);
    if (e != hipSuccess) return hip_fail(h, e, "decision launch");

    StepArgs<T, S> b = a;
    b.x_out = reinterpret_cast<S*>(h->x[h->cur]);  // in place
    b.lw_in = reinterpret_cast<const T*>(h->lw[h->cur]);
    b.lw_out = reinterpret_cast<T*>(h->lw[h->cur]);
    b.flags = kStepLwRaw | kStepNoFold;
    b.ess_out = reinterpret_cast<T*>(h->ess_part);
    b.stab = h->stab;
    b.anc = nullptr;
    LaunchReq rs{};
    rs.D = h->D;
    rs.mk = h->mk;
    rs.what = LW_AD_STAGE;
    rs.nt = h->stages[0].nt;
    rs.grid = h->ad_grid;
    rs.lds = h->ad_lds;
    ad.first = 0u;
    ad.rec = h->ess_part;
    ad.stride = 3u;
    for (uint32_t j = 0; j < ad.S; ++j) {
      e = launch(h, rs, &b);
      if (e != hipSuccess) return hip_fail(h, e, "stage slot launch");
      e = launch(h, rd, &a);
      if (e != hipSuccess) return hip_fail(h, e, "decision launch");
    }

    StepArgs<T, S> c = a;
    c.x_in = reinterpret_cast<const S*>(h->x[h->cur]);
    c.x_out = reinterpret_cast<S*>(h->x[h->cur ^ 1]);
    c.lw_in = reinterpret_cast<const T*>(h->lw[h->cur]);
    c.lw_out = reinterpret_cast<T*>(h->lw[h->cur ^ 1]);
    LaunchReq rp{};
    rp.D = h->D;
    rp.mk = h->mk;
    rp.what = LW_AD_PROPAGATE;
    rp.grid = (uint32_t)std::min<uint64_t>((h->N / 2 + 255) / 256, 65536);
    e = launch(h, rp, &c);
    if (e != hipSuccess) return hip_fail(h, e, "mutation launch");
    h->cur ^= 1;
    h->u += 1;
    h->lw_zero = false;
    return PF_OK;
  }
}

// One time step; y either by value (y_host) or in device memory (y_dev).
// Rotating mode: stage k = t mod S. Full-cycle mode: stages 0..S-1 in one
// step (only the first weights, only the last propagates).
template <typename T, typename S>
pf_status run_step(pf_handle* h, const double* y_host, const void* y_dev) {
  const uint32_t S_ = (uint32_t)h->stages.size();
  FinStep fs;
  fs.t = (uint32_t)h->t;
  if (h->global) {
    const uint32_t k = 0;
    const StagePlan& sp = h->stages[k];
    StepArgs<T, S> a;
    fill_common<T, S>(h, a);
    if (y_dev) {
      a.y_dev = reinterpret_cast<const T*>(y_dev);
    } else {
      for (int j = 0; j < h->d; ++j) a.y_val[j] = (T)y_host[j];
    }
    a.t = (uint32_t)h->t;
    a.k = k;
    a.u = (uint32_t)h->u;
    a.flags = kStepWeight | kStepPropagate;
    a.utau = (uint32_t)h->t + 1u;
    a.radix = sp.r;
    a.log2r = sp.log2r;
    a.lnr = (T)std::log((double)sp.r);
    a.ntiles = h->g_ntiles;
    a.lw_nonzero = h->lw_zero ? 0 : 1;
    LaunchReq rq{};
    rq.D = h->D;
    rq.mk = h->mk;
    rq.what = LW_GLOBAL_WEIGHT;
    rq.nt = (int)h->g_nt;
    rq.ppt = (int)h->g_ppt;
    rq.grid = h->g_ntiles;
    hipError_t e = launch(h, rq, &a);
    if (e != hipSuccess) return hip_fail(h, e, "global weight launch");
    rq.what = LW_GLOBAL_PREFIX;
    rq.nt = 256;
    rq.grid = 1;
    rq.lds = 0;
    e = launch(h, rq, &a);
    if (e != hipSuccess) return hip_fail(h, e, "global prefix launch");
    rq.nt = 256;
    rq.tile_elems = h->g_tile;
    if (h->gwork != nullptr) {
      // systematic: the merge over the items kernel 2 planned
      rq.what = LW_GLOBAL_SYS_DRAW;
      rq.grid = (uint32_t)std::min<uint64_t>(sys_max_items(h->N, h->g_ntiles), kDrawBlocks);
      rq.lds = sys_draw_lds(h->D, h->tsz, h->ssz, h->g_tile);
    } else {
      rq.what = LW_GLOBAL_DRAW;
      rq.ppt = kDrawPPT;
      const uint64_t pairs_per_block = 256ull * kDrawPPT;
      rq.nchunks = (uint32_t)((h->N / 2 + pairs_per_block - 1) / pairs_per_block);
      rq.grid = std::min<uint32_t>(rq.nchunks, kDrawBlocks);
      rq.lds = h->g_ntiles <= 4096 ? (size_t)(h->g_ntiles + 1) * 8 : 16;
    }
    e = launch(h, rq, &a);
    if (e != hipSuccess) return hip_fail(h, e, "global draw launch");
    // the global path does not store log-weights: after it every one is 0
    h->cur ^= 1;
    h->u += 1;
    h->lw_zero = true;
    fs.k = k;
    fs.radix = (uint32_t)std::min<uint64_t>(h->N, 0xFFFFFFFFu);
    fs.ntiles = h->g_ntiles;
  } else if (h->ess_theta > 0.0) {
    pf_status st = run_adaptive_step<T, S>(h, y_host, y_dev);
    if (st != PF_OK) return st;
    fs.k = kStageFromDevice;
    fs.radix = (uint32_t)std::min<uint64_t>(h->radix, 0xFFFFFFFFu);
    fs.ntiles = h->w_ntiles;
  } else if (h->island) {
    pf_status st = run_island_step<T, S>(h, y_host, y_dev);
    if (st != PF_OK) return st;
    fs.k = h->log2m;
    fs.radix = h->island;
    fs.ntiles = h->stages[0].ntiles;
  } else if (!h->full_cycle) {
    const uint32_t k = (uint32_t)(h->t % S_);
    pf_status st = launch_stage<T, S>(h, y_host, y_dev, k, kStepWeight | kStepPropagate, (uint32_t)h->t + 1u);
    if (st != PF_OK) return st;
    h->lw_zero = false;
    fs.k = k;
    fs.radix = h->stages[k].r;
    fs.ntiles = h->stages[k].ntiles;
  } else {
    if (h->t + 1 >= kStageTau || S_ > 255)
      return fail(h, PF_E_UNSUPPORTED, "full-cycle steps need t + 1 < 2^24 and S < 256");
    for (uint32_t k = 0; k < S_; ++k) {
      const uint32_t flags = (k == 0 ? kStepWeight : 0u) | (k + 1 == S_ ? kStepPropagate : 0u);
      const uint32_t tau = (uint32_t)h->t + 1u;
      pf_status st = launch_stage<T, S>(h, y_host, y_dev, k, flags, tau + k * kStageTau);
      if (st != PF_OK) return st;
    }
    h->lw_zero = false;
    fs.k = S_;
    fs.radix = (uint32_t)std::min<uint64_t>(h->radix, 0xFFFFFFFFu);
    fs.ntiles = h->stages[0].ntiles;
  }
  fs.unext = (uint32_t)h->u;
  h->pending.push_back(fs);
  h->t += 1;
  // the ring of partials is full: reduce the pending steps now
  if (h->pending.size() >= h->ring) return flush(h);
  return PF_OK;
}

// Reduce the pending steps' partials (estimate records, log-normaliser):
// one step with the complete single-block reduction, several with one
// block per step and a pass adding the log-normaliser in step order.
pf_status flush(pf_handle* h) {
  const size_t n = h->pending.size();
  if (n == 0) return PF_OK;
  char dummy[sizeof(StepArgs<double, double>)] = {0};  // dispatch only reads the request
  LaunchReq rq{};
  rq.D = h->D;
  rq.mk = h->mk;
  rq.grid = 1;
  if (n == 1) {
    const FinStep& fs = h->pending[0];
    rq.what = LW_FINALIZE;
    rq.fin.ctl = h->ctl;
    rq.fin.hist = h->hist;
    rq.fin.hist_cap = h->hist_cap;
    rq.fin.t = fs.t;
    rq.fin.k = fs.k;
    rq.fin.radix = fs.radix;
    rq.fin.d = (uint32_t)h->d;
    rq.fin.N = h->N;
    rq.fin.multi = 0u;
    rq.fin.slot = 0u;
    rq.fin.write_rec = 1u;
    rq.fin.use_step_off = 0u;
    rq.fin.unext = fs.unext;
    rq.fin_part = reinterpret_cast<const char*>(h->partials) + (size_t)(fs.t % h->ring) * h->part_stride * h->tsz;
    rq.fin_ntiles = fs.ntiles;
    hipError_t e = launch(h, rq, dummy);
    if (e != hipSuccess) return hip_fail(h, e, "finalize launch");
  } else {
    FinMulti fm;
    std::memset(&fm, 0, sizeof(fm));
    fm.ctl = h->ctl;
    fm.hist = h->hist;
    fm.part_base = h->partials;
    fm.part_stride = h->part_stride;
    fm.N = h->N;
    fm.hist_cap = h->hist_cap;
    fm.d = (uint32_t)h->d;
    fm.n = (uint32_t)n;
    fm.ring = h->ring;
    for (size_t i = 0; i < n; ++i) fm.steps[i] = h->pending[i];
    rq.fm = &fm;
    rq.what = LW_FINALIZE_MULTI;
    hipError_t e = launch(h, rq, dummy);
    if (e != hipSuccess) return hip_fail(h, e, "finalize launch");
    rq.what = LW_FINALIZE_PREFIX;
    e = launch(h, rq, dummy);
    if (e != hipSuccess) return hip_fail(h, e, "finalize launch");
  }
  h->pending.clear();
  return PF_OK;
}

pf_status do_init(pf_handle* h) {
  switch (h->dtype) {
    case PF_DTYPE_F32: return run_init<float, float>(h);
    case PF_DTYPE_BF16: return run_init<float, bf16>(h);
    default: return run_init<double, double>(h);
  }
}

pf_status do_step(pf_handle* h, const double* y_host, const void* y_dev) {
  switch (h->dtype) {
    case PF_DTYPE_F32: return run_step<float, float>(h, y_host, y_dev);
    case PF_DTYPE_BF16: return run_step<float, bf16>(h, y_host, y_dev);
    default: return run_step<double, double>(h, y_host, y_dev);
  }
}

}  // namespace

namespace pfh {
// Stage plan of the butterfly path (radix < N) into out[0 .. *n_out): mixed
// radix, tile shape, LDS. The island filter's within-island launch is one
// stage of radix M and stride 1 (island = true, radix = M). No heap memory,
// so a caller that must not allocate can plan with it. On failure `err` (errlen
// bytes) receives the reason.
pf_status plan_butterfly(uint64_t N, uint64_t radix, int D, int d, size_t tsz, bool island, StagePlan* out,
                         uint32_t max_out, uint32_t* n_out, char* err, size_t errlen) {
  const uint32_t n = ilog2(N);
  const uint32_t b = ilog2(radix);
  const uint32_t S = (n + b - 1) / b;
  const uint32_t last = n - (S - 1) * b;
  const uint32_t nst = island ? 1u : S;
  if (nst > max_out) {
    std::snprintf(err, errlen, "%u stages exceed the limit of %u", nst, max_out);
    return PF_E_UNSUPPORTED;
  }
  uint64_t R = 1;
  for (uint32_t k = 0; k < nst; ++k) {
    StagePlan sp{};
    sp.log2r = (k + 1 < S) ? b : last;
    sp.r = 1u << sp.log2r;
    sp.R = R;
    sp.log2R = ilog2(R);
    R *= sp.r;
    uint32_t E;
    if (sp.r <= 64) {
      sp.blockpath = 0;
      sp.nt = 256;
      sp.ppt = ppt_wave(D);
      E = 2u * sp.nt * sp.ppt;
      if (E > N) {
        sp.nt = 64;
        sp.ppt = 1;
        E = 128;
      }
    } else {
      sp.blockpath = 1;
      // 256-thread tiles of at least two groups; larger tiles give longer
      // contiguous rows at wide strides
      const uint32_t pb = (uint32_t)ppt_block(D);
      // d <= 2: tiles whose registers leave several blocks per compute unit
      // (two pairs per thread: 74 VGPRs; four: 139; eight would hold 256); a
      // stride-1 stage may hold a single group per tile
      if (D <= 2 && ((sp.r <= 256 && N >= 1024u) || (sp.r <= 1024 && sp.log2R == 0 && N >= 1024u))) {
        sp.nt = 256;
        sp.ppt = 2;
      } else if (D <= 2 && sp.r <= 1024 && N >= 2048u) {
        sp.nt = 256;
        sp.ppt = 4;
      } else if (512u * pb >= 2u * sp.r && 512u * pb <= N) {
        sp.nt = 256;
        sp.ppt = (int)pb;
      } else if (island && sp.log2R == 0 && sp.r <= 1024 && 512u * pb >= sp.r && 512u * pb <= N) {
        // the within-island launch: one island per 256-thread tile
        sp.nt = 256;
        sp.ppt = (int)pb;
      } else if (sp.r <= 1024 && N >= 2048) {
        sp.nt = 1024;
        sp.ppt = 1;
      } else if (sp.r <= 256) {
        sp.nt = 256;
        sp.ppt = 1;
      } else if (sp.r == 2048 && D <= 4) {
        sp.nt = 1024;
        sp.ppt = 2;
      } else if (sp.r == 4096 && D <= 4) {
        sp.nt = 1024;
        sp.ppt = 4;
      } else if (sp.log2R == 0 && sp.r == 2048 && sp.r <= N) {
        // stride 1: a group is a contiguous run, so a tile of one group still
        // loads coalesced rows
        sp.nt = 1024;
        sp.ppt = 1;
      } else {
        std::snprintf(err, errlen, "stage radix %u is not supported for d = %d (use r <= 1024, or r >= N)",
                      sp.r, d);
        return PF_E_UNSUPPORTED;
      }
      E = 2u * sp.nt * sp.ppt;
    }
    if (E > N || E < (sp.log2R == 0 ? sp.r : 2u * sp.r)) {
      std::snprintf(err, errlen, "N = %llu is too small for a tile of radix %u", (unsigned long long)N, sp.r);
      return PF_E_UNSUPPORTED;
    }
    sp.C = E / sp.r;
    sp.log2C = ilog2(sp.C);
    sp.ntiles = (uint32_t)(N / E);
    sp.pad = choose_pad_eval(sp.r, sp.C, sp.log2R, sp.nt);
    sp.xrow = state_row_pitch(sp.C, sp.log2R, sp.log2C);
    // the within-island launch of the island filter stages no states
    sp.lds = tile_lds_bytes(island ? 0 : d, D, tsz, sp.r, sp.C, sp.pad, sp.nt, sp.blockpath != 0, sp.xrow);
    if (sp.lds > 160 * 1024) {
      std::snprintf(err, errlen, "tile of radix %u needs %zu bytes of LDS (> 160 KiB)", sp.r, sp.lds);
      return PF_E_UNSUPPORTED;
    }
    out[k] = sp;
  }
  *n_out = nst;
  return PF_OK;
}
}  // namespace pfh

namespace {

pf_status plan_stages(pf_handle* h) {
  const uint64_t N = h->N;
  const uint32_t n = ilog2(N);
  if (h->radix >= N) {
    h->global = true;
    StagePlan sp{};
    sp.r = (uint32_t)std::min<uint64_t>(N, 0xFFFFFFFFu);
    sp.log2r = n;
    sp.R = 1;
    sp.log2R = 0;
    h->stages.push_back(sp);
    // weight tiles
    uint32_t nt = 256, ppt = (uint32_t)ppt_gweight(h->D);
    uint64_t E = 2ull * nt * ppt;
    if (E > N) {
      nt = 64;
      ppt = 1;
      E = 128;
    }
    if (E > N) return fail(h, PF_E_UNSUPPORTED, "N must be at least 128 on the device");
    h->g_nt = nt;
    h->g_ppt = ppt;
    h->g_tile = (uint32_t)E;
    h->g_ntiles = (uint32_t)(N / E);
    return PF_OK;
  }
  StagePlan plan[kMaxStages];
  uint32_t S = 0;
  char why[160];
  const pf_status st = plan_butterfly(N, h->radix, h->D, h->d, h->tsz, h->island != 0, plan, kMaxStages, &S, why,
                                      sizeof(why));
  if (st != PF_OK) return fail(h, st, why);
  h->stages.assign(plan, plan + S);
  return PF_OK;
}

void release(pf_handle* h) {
  for (void* p : h->allocs) dev_free(h->dalloc_fn, p);
  h->allocs.clear();
}

bool poisoned(pf_handle* h) { return h->sticky != PF_OK; }

pf_status numeric_fail(pf_handle* h) {
  return fail(h, PF_E_NUMERIC,
              "a step's weights were not usable (non-finite, or none positive); pf_reset, pf_set_state "
              "or pf_load start the filter again");
}

// After a synchronisation: the device's sticky flag of unusable weights.
pf_status check_numeric(pf_handle* h) {
  if (!h->numeric) {
    uint32_t fl = 0;
    hipError_t e = hipMemcpy(&fl, reinterpret_cast<const char*>(h->ctl) + offsetof(Ctl, fail_t), sizeof(fl),
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "control copy");
    h->numeric = fl != kNoFail;
  }
  return h->numeric ? numeric_fail(h) : PF_OK;
}

}  // namespace

extern "C" {

const char* pf_status_string(pf_status s) {
  switch (s) {
    case PF_OK: return "ok";
    case PF_E_INVALID: return "invalid argument";
    case PF_E_UNSUPPORTED: return "unsupported";
    case PF_E_OOM: return "out of device memory";
    case PF_E_HIP: return "HIP runtime error";
    case PF_E_NUMERIC: return "non-finite value";
    case PF_E_STATE: return "handle in error state";
  }
  return "unknown status";
}

pf_status pf_set_allocator(void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* ctx) {
  if ((alloc == nullptr) != (free_ == nullptr)) return PF_E_INVALID;
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc.alloc = alloc;
  g_alloc.free_ = free_;
  g_alloc.ctx = alloc ? ctx : nullptr;
  return PF_OK;
}

const char* pf_last_error(const pf_handle* h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

pf_status pf_create(const pf_model* model, const pf_config* cfg, void* hip_stream, pf_handle** out) {
  g_create_error.clear();
  if (!out) return fail(nullptr, PF_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!model || !cfg) return fail(nullptr, PF_E_INVALID, "model or config is NULL");
  const int d = model->d;
  {
    std::string msg;
    if (validate_model(model, msg) != PF_OK) return fail(nullptr, PF_E_INVALID, msg);
  }
  const uint64_t N = cfg->n_particles;
  if (!is_pow2(N) || N < 2 || N > (1ull << 30))
    return fail(nullptr, PF_E_INVALID, "n_particles must be a power of two in [2, 2^30]");
  if (!is_pow2(cfg->radix) || cfg->radix < 2)
    return fail(nullptr, PF_E_INVALID, "radix must be a power of two >= 2");
  if (cfg->resampler != PF_RESAMPLE_MULTINOMIAL && cfg->resampler != PF_RESAMPLE_SYSTEMATIC)
    return fail(nullptr, PF_E_INVALID, "unknown resampler");
  if (cfg->state_dtype != PF_DTYPE_F32 && cfg->state_dtype != PF_DTYPE_BF16 &&
      cfg->state_dtype != PF_DTYPE_F64)
    return fail(nullptr, PF_E_INVALID, "unknown state dtype");

  pf_handle* h = new (std::nothrow) pf_handle();
  if (!h) return fail(nullptr, PF_E_OOM, "host allocation failed");
  h->kind = model->kind;
  h->d = d;
  h->D = compiled_dim(d);
  h->dtype = cfg->state_dtype;
  h->resampler = cfg->resampler;
  h->N = N;
  h->radix = cfg->radix;
  h->seed = cfg->seed;
  h->sid = cfg->stream_id;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  h->tsz = h->dtype == PF_DTYPE_F64 ? 8 : 4;
  h->ssz = h->dtype == PF_DTYPE_F64 ? 8 : (h->dtype == PF_DTYPE_BF16 ? 2 : 4);
  h->hist_cap = cfg->history ? cfg->history : 1;
  h->full_cycle = cfg->full_cycle != 0;
  h->model_hash = model_hash(model);
  h->dalloc_fn = current_allocator();
  if (cfg->ess_threshold != 0.0) {
    const double th = cfg->ess_threshold;
    std::string why;
    if (!(th > 0.0 && th <= 1.0)) why = "ess_threshold must be 0 (off) or in (0, 1]";
    else if (cfg->state_dtype != PF_DTYPE_F32) why = "ESS-gated stages need FP32 states";
    else if (cfg->radix > 64 || cfg->radix >= N) why = "ESS-gated stages need a radix of at most 64 (and below N)";
    else if (N < 512) why = "ESS-gated stages need N >= 512";
    else if (cfg->full_cycle || cfg->island) why = "ESS-gated stages exclude full_cycle and the island filter";
    else if (cfg->keep_ancestors) why = "ESS-gated stages do not record ancestors";
    if (!why.empty()) {
      delete h;
      return fail(nullptr, PF_E_INVALID, why);
    }
    h->ess_theta = th;
  }
  if (cfg->island) {
    const uint64_t M = cfg->island;
    if (!is_pow2(M) || M < 2 || M > N / 2 || M > 4096) {
      delete h;
      return fail(nullptr, PF_E_INVALID, "island size must be a power of two in [2, min(N / 2, 4096)]");
    }
    if (h->full_cycle) {
      delete h;
      return fail(nullptr, PF_E_INVALID, "the island filter runs all island stages; full_cycle must be 0");
    }
    h->island = (uint32_t)M;
    h->log2M = ilog2(M);
    h->log2m = ilog2(N / M);
    h->island_no_swap = cfg->island_swap == 0;
    h->radix = M;  // the within-island stage: radix M, stride 1
  }

  auto bail = [&](pf_status s) {
    g_create_error = h->err;
    release(h);
    delete h;
    return s;
  };
  pf_status s = plan_stages(h);
  if (s != PF_OK) return bail(s);

  // model parameters
  int mk = 0;
  if (h->dtype == PF_DTYPE_F64) {
    ModelParams<double> P;
    fill_params<double>(model, d, &P, &mk);
    if ((s = dalloc(h, &h->mp, sizeof(P))) != PF_OK) return bail(s);
    hipError_t e = hipMemcpy(h->mp, &P, sizeof(P), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(hip_fail(h, e, "model upload"));
  } else {
    ModelParams<float> P;
    fill_params<float>(model, d, &P, &mk);
    if ((s = dalloc(h, &h->mp, sizeof(P))) != PF_OK) return bail(s);
    hipError_t e = hipMemcpy(h->mp, &P, sizeof(P), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(hip_fail(h, e, "model upload"));
  }
  h->mk = mk;

  // buffers
  for (int i = 0; i < 2; ++i) {
    if ((s = dalloc(h, &h->x[i], (size_t)d * N * h->ssz)) != PF_OK) return bail(s);
    if ((s = dalloc(h, &h->lw[i], (size_t)N * h->tsz)) != PF_OK) return bail(s);
  }
  uint32_t max_tiles = h->global ? h->g_ntiles : 0;
  for (auto& sp : h->stages) max_tiles = std::max(max_tiles, sp.ntiles);
  if (h->ess_theta > 0.0) {
    h->w_ntiles = (uint32_t)(N / 512);
    max_tiles = std::max(max_tiles, h->w_ntiles);
  }
  // ring of deferred partials: up to kMaxPending steps within 64 MiB
  h->part_stride = (uint64_t)max_tiles * partial_stride(h->D);
  {
    const uint64_t per = h->part_stride * h->tsz;
    const uint64_t fit = (64ull << 20) / (per ? per : 1);
    // full-cycle steps use S offset indices each: the deferred reductions
    // read the recorded offsets of up to kMaxPending indices
    const uint64_t per_step = (h->full_cycle && !h->global) ? h->stages.size() : 1;
    h->ring = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(kMaxPending / per_step, fit));
  }
  if ((s = dalloc(h, &h->partials, (size_t)h->ring * h->part_stride * h->tsz)) != PF_OK) return bail(s);
  void* p = nullptr;
  if ((s = dalloc(h, &p, sizeof(Ctl))) != PF_OK) return bail(s);
  h->ctl = reinterpret_cast<Ctl*>(p);
  if ((s = dalloc(h, &p, sizeof(pf_estimate_t) * h->hist_cap)) != PF_OK) return bail(s);
  h->hist = reinterpret_cast<pf_estimate_t*>(p);
  {
    hipError_t e = hipMemset(h->hist, 0, sizeof(pf_estimate_t) * h->hist_cap);
    if (e != hipSuccess) return bail(hip_fail(h, e, "history clear"));
  }
  if (cfg->keep_ancestors) {
    if ((s = dalloc(h, &p, (size_t)N * 4)) != PF_OK) return bail(s);
    h->anc = reinterpret_cast<uint32_t*>(p);
  }
  if (h->ess_theta > 0.0) {
    std::vector<AdStage> tab(h->stages.size());
    uint32_t stage_tiles = 0;
    for (size_t k = 0; k < h->stages.size(); ++k) {
      const StagePlan& sp = h->stages[k];
      if (sp.blockpath || sp.nt != h->stages[0].nt)
        return bail(fail(h, PF_E_UNSUPPORTED, "ESS-gated stages need wave-path tiles of one shape"));
      tab[k] = AdStage{sp.log2r, sp.log2R, sp.log2C, sp.pad, sp.xrow, sp.ntiles, (float)std::log((double)sp.r), 0u};
      stage_tiles = std::max(stage_tiles, sp.ntiles);
      h->ad_lds = std::max(h->ad_lds, sp.lds);
    }
    h->ad_grid = stage_tiles;
    if ((s = dalloc(h, &p, tab.size() * sizeof(AdStage))) != PF_OK) return bail(s);
    h->stab = reinterpret_cast<AdStage*>(p);
    hipError_t e = hipMemcpy(h->stab, tab.data(), tab.size() * sizeof(AdStage), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(hip_fail(h, e, "stage table upload"));
    if ((s = dalloc(h, &h->ess_part, (size_t)stage_tiles * 3 * h->tsz)) != PF_OK) return bail(s);
  }
  if (h->island) {
    const size_t m = (size_t)1 << h->log2m;
    if ((s = dalloc(h, &p, (size_t)N * 4)) != PF_OK) return bail(s);
    h->ianc = reinterpret_cast<uint32_t*>(p);
    if ((s = dalloc(h, &h->isl_lw, m * h->tsz)) != PF_OK) return bail(s);
    if ((s = dalloc(h, &p, m * 4)) != PF_OK) return bail(s);
    h->isl_src = reinterpret_cast<uint32_t*>(p);
    if ((s = dalloc(h, &p, m * h->tsz)) != PF_OK) return bail(s);
    h->isl_lv = p;
  }
  if (h->global) {
    // d = 1: the CDF in runs of 16 paired with the states (2 N values);
    // d > 1: the CDF (N) and the states particle-major (N D storage values)
    // (systematic: the CDF alone; its draw reads the states where they are)
    const bool sys = h->resampler == PF_RESAMPLE_SYSTEMATIC;
    if ((s = dalloc(h, &h->gcdf, (size_t)N * h->tsz * (h->D == 1 && !sys ? 2 : 1))) != PF_OK) return bail(s);
    if (h->D > 1 && !sys && (s = dalloc(h, &h->gx, (size_t)N * h->D * h->ssz)) != PF_OK) return bail(s);
    if ((s = dalloc(h, &h->gcoarse, (size_t)global_coarse_elems(N, h->g_ntiles) * h->tsz)) != PF_OK)
      return bail(s);
    if ((s = dalloc(h, &p, (size_t)(h->g_ntiles + 1) * 8)) != PF_OK) return bail(s);
    h->gpre = reinterpret_cast<double*>(p);
    if ((s = dalloc(h, &p, (size_t)h->g_ntiles * 8)) != PF_OK) return bail(s);
    h->gscale = reinterpret_cast<double*>(p);
    if (h->resampler == PF_RESAMPLE_SYSTEMATIC) {
      if ((s = dalloc(h, &p, (size_t)(h->g_ntiles + 1) * 4)) != PF_OK) return bail(s);
      h->gfirst = reinterpret_cast<uint32_t*>(p);
      if ((s = dalloc(h, &p, (size_t)(2 + 2 * sys_max_items(N, h->g_ntiles)) * 4)) != PF_OK) return bail(s);
      h->gwork = reinterpret_cast<uint32_t*>(p);
    }
  }
  s = do_init(h);
  if (s != PF_OK) return bail(s);
  *out = h;
  return PF_OK;
}

pf_status pf_destroy(pf_handle* h) {
  if (!h) return PF_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  release(h);
  delete h;
  return PF_OK;
}

pf_status pf_reset(pf_handle* h) {
  if (!h) return PF_E_INVALID;
  if (poisoned(h)) return PF_E_STATE;
  h->cur = 0;
  h->numeric = false;  // the initialisation clears the device flag
  return do_init(h);
}

pf_status pf_step(pf_handle* h, const double* y_host) {
  if (!h) return PF_E_INVALID;
  if (poisoned(h)) return PF_E_STATE;
  if (!y_host) return fail(h, PF_E_INVALID, "y is NULL");
  if (!finite_all(y_host, h->d)) return fail(h, PF_E_NUMERIC, "non-finite observation");
  if (h->numeric) return numeric_fail(h);
  return do_step(h, y_host, nullptr);
}

pf_status pf_run(pf_handle* h, const void* y_dev, uint32_t n_steps, uint64_t y_stride, int32_t use_graph) {
  if (!h) return PF_E_INVALID;
  if (poisoned(h)) return PF_E_STATE;
  if (!y_dev) return fail(h, PF_E_INVALID, "y_dev is NULL");
  if (y_stride < (uint64_t)h->d) return fail(h, PF_E_INVALID, "y_stride < d");
  if (h->numeric) return numeric_fail(h);
  if (n_steps == 0) return PF_OK;
  const char* yb = reinterpret_cast<const char*>(y_dev);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (use_graph) {
    if (!h->stream) return fail(h, PF_E_INVALID, "graph capture needs a non-default stream");
    hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamBeginCapture");
  }
  const uint64_t t0 = h->t;
  const int cur0 = h->cur;
  void* lw0[2] = {h->lw[0], h->lw[1]};
  pf_status st = PF_OK;
  for (uint32_t j = 0; j < n_steps && st == PF_OK; ++j)
    st = do_step(h, nullptr, yb + (size_t)j * y_stride * h->tsz);
  if (st == PF_OK) st = flush(h);
  if (use_graph) {
    hipError_t e = hipStreamEndCapture(h->stream, &graph);
    if (st != PF_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(h, e, "hipGraphInstantiate");
    }
    e = hipGraphLaunch(exec, h->stream);
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(h, e, "hipGraphLaunch");
    (void)t0;
    (void)cur0;
    (void)lw0;
  }
  return st;
}

pf_status pf_sync(pf_handle* h) {
  if (!h) return PF_E_INVALID;
  if (!poisoned(h)) {
    pf_status fs = flush(h);
    if (fs != PF_OK) return fs;
  }
  hipError_t e = h->stream ? hipStreamSynchronize(h->stream) : hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(h, e, "synchronize");
  return PF_OK;
}

pf_status pf_estimate(pf_handle* h, pf_estimate_t* out) {
  if (!h || !out) return PF_E_INVALID;
  if (poisoned(h)) return PF_E_STATE;
  if (h->t == 0) return fail(h, PF_E_STATE, "no step has run");
  pf_status s = pf_sync(h);
  if (s != PF_OK) return s;
  const uint64_t slot = (h->t - 1) % h->hist_cap;
  hipError_t e = hipMemcpy(out, h->hist + slot, sizeof(*out), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(h, e, "estimate copy");
  return check_numeric(h);
}

pf_status pf_history(pf_handle* h, pf_estimate_t* out, uint32_t n_max, uint32_t* n_out) {
  if (!h || !out || !n_out) return PF_E_INVALID;
  if (poisoned(h)) return PF_E_STATE;
  pf_status s = pf_sync(h);
  if (s != PF_OK) return s;
  uint64_t n = std::min<uint64_t>(h->t, h->hist_cap);
  n = std::min<uint64_t>(n, n_max);
  std::vector<pf_estimate_t> all(h->hist_cap);
  hipError_t e = hipMemcpy(all.data(), h->hist, sizeof(pf_estimate_t) * h->hist_cap, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(h, e, "history copy");
  for (uint64_t i = 0; i < n; ++i) {
    const uint64_t t = h->t - n + i;
    out[i] = all[t % h->hist_cap];
  }
  *n_out = (uint32_t)n;
  return check_numeric(h);
}

pf_status pf_get_state(pf_handle* h, void* x_host, void* logw_host, uint32_t* t_out, double* log_norm) {
  if (!h) return PF_E_INVALID;
  if (poisoned(h)) return PF_E_STATE;
  pf_status s = pf_sync(h);
  if (s != PF_OK) return s;
  hipError_t e;
  if (x_host) {
    e = hipMemcpy(x_host, h->x[h->cur], (size_t)h->d * h->N * h->ssz, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "state copy");
  }
  Ctl c;
  e = hipMemcpy(&c, h->ctl, sizeof(c), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(h, e, "control copy");
  if (logw_host && h->lw_zero) {
    std::memset(logw_host, 0, (size_t)h->N * h->tsz);
  } else if (logw_host) {
    e = hipMemcpy(logw_host, h->lw[h->cur], (size_t)h->N * h->tsz, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "log-weight copy");
    // stored log-weights are normalised by the offset the next step would subtract
    double off = -INFINITY;
    for (int sl = 0; sl < kOffSlots; ++sl)
      off = std::max(off, ord_decode(c.offs[(h->u % kOffRing) * kOffSlots * kOffStride + sl * kOffStride]));
    if (h->tsz == 8) {
      double* w = reinterpret_cast<double*>(logw_host);
      for (uint64_t i = 0; i < h->N; ++i) w[i] -= off;
    } else {
      float* w = reinterpret_cast<float*>(logw_host);
      const float o = (float)off;
      for (uint64_t i = 0; i < h->N; ++i) w[i] -= o;
    }
  }
  if (t_out) *t_out = (uint32_t)h->t;
  if (log_norm) *log_norm = c.log_norm;
  return PF_OK;
}

pf_status pf_set_state(pf_handle* h, const void* x_host, const void* logw_host, uint32_t t, double log_norm) {
  if (!h || !x_host) return PF_E_INVALID;
  if (poisoned(h)) return PF_E_STATE;
  pf_status s = pf_sync(h);
  if (s != PF_OK) return s;
  hipError_t e = hipMemcpy(h->x[h->cur], x_host, (size_t)h->d * h->N * h->ssz, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(h, e, "state upload");
  if (logw_host) {
    e = hipMemcpy(h->lw[h->cur], logw_host, (size_t)h->N * h->tsz, hipMemcpyHostToDevice);
    h->lw_zero = false;
  } else {
    e = hipMemset(h->lw[h->cur], 0, (size_t)h->N * h->tsz);
    h->lw_zero = true;
  }
  if (e != hipSuccess) return hip_fail(h, e, "log-weight upload");
  Ctl c;
  e = hipMemcpy(&c, h->ctl, sizeof(c), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(h, e, "control copy");
  c.log_norm = log_norm;
  c.ad_active = c.ad_stage = c.ad_run = c.ad_next = 0u;  // ESS-gated stages start at stage 0
  c.fail_t = kNoFail;
  h->numeric = false;
  for (int i = 0; i < kOffEntries; ++i) c.offs[i] = ord_encode(-INFINITY);
  c.offs[(t % kOffRing) * kOffSlots * kOffStride] = ord_encode(0.0);
  c.t = t;
  h->pending.clear();
  e = hipMemcpy(h->ctl, &c, sizeof(c), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(h, e, "control upload");
  h->t = t;
  h->u = t;
  return PF_OK;
}

pf_status pf_save(pf_handle* h, void* buf, uint64_t cap, uint64_t* len_out) {
  if (!h || !len_out) return PF_E_INVALID;
  if (poisoned(h)) return PF_E_STATE;
  const uint64_t xb = (uint64_t)h->d * h->N * h->ssz, lb = h->N * h->tsz, rb = sizeof(pf_estimate_t);
  const uint64_t need = sizeof(BlobHeader) + xb + lb + rb;
  *len_out = need;
  if (!buf) return PF_OK;
  if (cap < need) return fail(h, PF_E_INVALID, "checkpoint buffer too small");
  pf_status s = pf_sync(h);
  if (s != PF_OK) return s;
  Ctl c;
  hipError_t e = hipMemcpy(&c, h->ctl, sizeof(c), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(h, e, "control copy");
  BlobHeader hd;
  std::memset(&hd, 0, sizeof(hd));
  std::memcpy(hd.magic, kBlobMagic, 8);
  hd.version = kBlobVersion;
  hd.header_bytes = sizeof(BlobHeader);
  hd.n_particles = h->N;
  hd.radix = h->radix;
  hd.model_hash = h->model_hash;
  hd.seed = h->seed;
  hd.kind = h->kind;
  hd.d = h->d;
  hd.resampler = h->resampler;
  hd.dtype = h->dtype;
  hd.stream_id = h->sid;
  hd.lw_zero = h->lw_zero ? 1u : 0u;
  hd.next_stage = c.ad_next;
  hd.t = h->t;
  hd.log_norm = c.log_norm;
  double off = -INFINITY;
  for (int sl = 0; sl < kOffSlots; ++sl)
    off = std::max(off, ord_decode(c.offs[(h->u % kOffRing) * kOffSlots * kOffStride + sl * kOffStride]));
  hd.offset = off;
  hd.x_bytes = xb;
  hd.lw_bytes = lb;
  hd.rec_bytes = rb;
  char* out = reinterpret_cast<char*>(buf);
  std::memcpy(out, &hd, sizeof(hd));
  out += sizeof(hd);
  e = hipMemcpy(out, h->x[h->cur], xb, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(h, e, "state copy");
  out += xb;
  if (h->lw_zero) {
    std::memset(out, 0, lb);
  } else {
    e = hipMemcpy(out, h->lw[h->cur], lb, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "log-weight copy");
  }
  out += lb;
  if (h->t > 0) {
    e = hipMemcpy(out, h->hist + (h->t - 1) % h->hist_cap, rb, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "record copy");
  } else {
    std::memset(out, 0, rb);
  }
  return PF_OK;
}

pf_status pf_load(pf_handle* h, const void* buf, uint64_t len) {
  if (!h || !buf) return PF_E_INVALID;
  if (poisoned(h)) return PF_E_STATE;
  BlobHeader hd;
  if (len < sizeof(hd)) return fail(h, PF_E_INVALID, "checkpoint shorter than its header");
  std::memcpy(&hd, buf, sizeof(hd));
  if (std::memcmp(hd.magic, kBlobMagic, 8) != 0 || hd.version != kBlobVersion ||
      hd.header_bytes != sizeof(BlobHeader))
    return fail(h, PF_E_INVALID, "not a checkpoint of this library version");
  const uint64_t xb = (uint64_t)h->d * h->N * h->ssz, lb = h->N * h->tsz, rb = sizeof(pf_estimate_t);
  if (hd.n_particles != h->N || hd.radix != h->radix || hd.model_hash != h->model_hash ||
      hd.kind != h->kind || hd.d != h->d || hd.resampler != h->resampler || hd.dtype != h->dtype ||
      hd.x_bytes != xb || hd.lw_bytes != lb || hd.rec_bytes != rb)
    return fail(h, PF_E_INVALID, "checkpoint of a different model or configuration");
  if (len < sizeof(hd) + xb + lb + rb) return fail(h, PF_E_INVALID, "checkpoint truncated");
  if (hd.t > 0xFFFFFFFFull || !std::isfinite(hd.log_norm) || !std::isfinite(hd.offset))
    return fail(h, PF_E_INVALID, "checkpoint header corrupt");
  pf_status s = pf_sync(h);
  if (s != PF_OK) return s;
  const char* in = reinterpret_cast<const char*>(buf) + sizeof(hd);
  hipError_t e = hipMemcpy(h->x[h->cur], in, xb, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(h, e, "state upload");
  in += xb;
  e = hipMemcpy(h->lw[h->cur], in, lb, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(h, e, "log-weight upload");
  in += lb;
  h->lw_zero = hd.lw_zero != 0;
  h->t = hd.t;
  h->u = hd.t;
  h->pending.clear();
  Ctl c;
  e = hipMemcpy(&c, h->ctl, sizeof(c), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(h, e, "control copy");
  c.log_norm = hd.log_norm;
  c.fail_t = kNoFail;
  h->numeric = false;
  c.t = (uint32_t)hd.t;
  c.ad_active = c.ad_stage = c.ad_run = 0u;
  c.ad_next = hd.next_stage < h->stages.size() ? hd.next_stage : 0u;
  for (int i = 0; i < kOffEntries; ++i) c.offs[i] = ord_encode(-INFINITY);
  // the raw log-weights come back with the offset the next step subtracts
  c.offs[(hd.t % kOffRing) * kOffSlots * kOffStride] = ord_encode(hd.offset);
  e = hipMemcpy(h->ctl, &c, sizeof(c), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(h, e, "control upload");
  if (hd.t > 0) {
    e = hipMemcpy(h->hist + (hd.t - 1) % h->hist_cap, in, rb, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(h, e, "record upload");
  }
  return PF_OK;
}

pf_status pf_get_ancestors(pf_handle* h, uint32_t* anc_host) {
  if (!h || !anc_host) return PF_E_INVALID;
  if (poisoned(h)) return PF_E_STATE;
  if (!h->anc) return fail(h, PF_E_STATE, "created without keep_ancestors");
  pf_status s = pf_sync(h);
  if (s != PF_OK) return s;
  hipError_t e = hipMemcpy(anc_host, h->anc, (size_t)h->N * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(h, e, "ancestor copy");
  return PF_OK;
}

pf_status pf_info(pf_handle* h, pf_info_t* out) {
  if (!h || !out) return PF_E_INVALID;
  std::memset(out, 0, sizeof(*out));
  out->n_particles = h->N;
  out->d = (uint32_t)h->d;
  out->n_stages = (uint32_t)h->stages.size();
  for (size_t k = 0; k < h->stages.size() && k < 32; ++k) {
    out->radices[k] = h->stages[k].r;
    out->tile_elems[k] = h->global ? h->g_tile : h->stages[k].r * h->stages[k].C;
  }
  out->global_path = h->global ? 1u : 0u;
  out->state_dtype = (uint32_t)h->dtype;
  out->device_bytes = h->bytes;
  out->t = (uint32_t)h->t;
  return PF_OK;
}


}  // extern "C"
