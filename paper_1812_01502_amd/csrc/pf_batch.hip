// pf_batch.hip - C-ABI of the batched filters (pf_batch_* in include/pf.h):
// many independent butterfly filters of different N, state dimension and
// model, advanced together by one launch per (dimension, model kind) class.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/pf.h"
#include "pf_host.h"

using namespace pfk;
using namespace pfh;

namespace {

thread_local std::string g_batch_create_error;

constexpr uint32_t kAutoRadices[] = {2, 4, 8, 16, 32, 64};
constexpr double kAutoSlack = 1.10;  // radix choice: largest within 10 % of the fastest

struct FilterHost {
  int kind, d, D, mk;
  uint64_t N;
  uint64_t radix;      // 0 while the autotuner has not chosen
  bool autotune;
  uint64_t seed;
  uint32_t sid, systematic, yoff;
  std::vector<uint32_t> radices;
  uint32_t ntiles, first_block, stage0;
  size_t x_off, lw_off, part_off;  // element offsets into the pools
};

struct ClassHost {
  int D, mk, ppt;
  int full = 1;  // every filter has d = D
  std::vector<uint32_t> filters;
  uint32_t nblocks = 0;
  size_t lds = 0;
  uint32_t* d_block_filter = nullptr;
  uint32_t* d_class_filters = nullptr;
};

}  // namespace

struct pf_batch {
  hipStream_t stream = nullptr;
  uint32_t n = 0;
  uint32_t y_len = 0;
  std::vector<FilterHost> fh;
  std::vector<ClassHost> classes;
  // device
  BatchFilter* d_filt = nullptr;
  BatchStage* d_stages = nullptr;
  uint32_t* d_tcur = nullptr;
  ModelParams<float>* d_mp = nullptr;
  float* d_x = nullptr;
  float* d_lw = nullptr;
  float* d_part = nullptr;
  Ctl* d_ctl = nullptr;
  pf_estimate_t* d_rec = nullptr;
  std::vector<BatchFilter> filt;  // host copy of the table
  std::vector<BatchStage> stages;
  std::vector<pf_batch_tune_t> tune;
  uint64_t bytes = 0;
  pf_status sticky = PF_OK;
  std::string err;
  DevAllocator dalloc_fn;  // the allocator current at create time
  std::vector<void*> allocs;
};

namespace {

pf_status bfail(pf_batch* b, pf_status s, const std::string& msg) {
  if (b) {
    b->err = msg;
    if (s == PF_E_HIP) b->sticky = PF_E_STATE;
  } else {
    g_batch_create_error = msg;
  }
  return s;
}

pf_status bhip(pf_batch* b, hipError_t e, const char* what) {
  return bfail(b, PF_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

pf_status balloc(pf_batch* b, void** p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  hipError_t e = dev_alloc(b->dalloc_fn, p, bytes);
  if (e == hipErrorInvalidValue)
    return bfail(b, PF_E_INVALID, "the installed allocator returned a pointer not aligned to 256 bytes");
  if (e != hipSuccess)
    return bfail(b, PF_E_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  b->allocs.push_back(*p);
  b->bytes += bytes;
  return PF_OK;
}

void brelease(pf_batch* b) {
  for (void* p : b->allocs) dev_free(b->dalloc_fn, p);
  b->allocs.clear();
}

// Stage tables of every filter for the current radices and class tiles;
// block maps of every class. Host tables only.
pf_status plan_batch(pf_batch* b) {
  b->stages.clear();
  for (auto& c : b->classes) {
    const uint32_t E = 2u * kBatchNT * (uint32_t)c.ppt;
    c.nblocks = 0;
    c.lds = 0;
    for (uint32_t f : c.filters) {
      FilterHost& F = b->fh[f];
      if (F.N < E) return bfail(b, PF_E_UNSUPPORTED, "filter " + std::to_string(f) + ": N below the tile size");
      F.radices = mixed_radices(F.N, F.radix);
      F.stage0 = (uint32_t)b->stages.size();
      F.ntiles = (uint32_t)(F.N / E);
      F.first_block = c.nblocks;
      c.nblocks += F.ntiles;
      uint64_t R = 1;
      for (uint32_t r : F.radices) {
        if (r > 64 || 2u * r > E)
          return bfail(b, PF_E_UNSUPPORTED, "filter " + std::to_string(f) + ": batched stages need r <= 64");
        BatchStage s{};
        s.log2r = ilog2(r);
        s.log2R = ilog2(R);
        const uint32_t C = E / r;
        s.log2C = ilog2(C);
        s.pad = choose_pad(r, C, s.log2R, kBatchNT);
        s.lnr = (float)std::log((double)r);
        s.xrow = state_row_pitch(C, s.log2R, s.log2C);
        b->stages.push_back(s);
        c.lds = std::max(c.lds, tile_lds_bytes(F.d, F.D, 4, r, C, s.pad, kBatchNT, false, s.xrow));
        R *= r;
      }
    }
    if (c.lds > 160 * 1024) return bfail(b, PF_E_UNSUPPORTED, "batched tile needs more than 160 KiB of LDS");
  }
  return PF_OK;
}

// Device tables from the host plan (filter table, stages, block maps).
pf_status upload_tables(pf_batch* b) {
  b->filt.assign(b->n, BatchFilter{});
  for (uint32_t f = 0; f < b->n; ++f) {
    const FilterHost& F = b->fh[f];
    BatchFilter& T = b->filt[f];
    T.x[0] = b->d_x + F.x_off;
    T.x[1] = b->d_x + F.x_off + (size_t)F.d * F.N;
    T.lw[0] = b->d_lw + F.lw_off;
    T.lw[1] = b->d_lw + F.lw_off + F.N;
    T.mp = b->d_mp + f;
    T.part = b->d_part + F.part_off;
    T.ctl = b->d_ctl + f;
    T.rec = b->d_rec + f;
    T.N = F.N;
    T.d = (uint32_t)F.d;
    T.S = (uint32_t)F.radices.size();
    T.stage0 = F.stage0;
    T.ntiles = F.ntiles;
    T.first_block = F.first_block;
    T.yoff = F.yoff;
    T.sid = F.sid;
    T.k0 = (uint32_t)(F.seed & 0xFFFFFFFFu);
    T.k1 = (uint32_t)(F.seed >> 32);
    T.systematic = F.systematic;
  }
  hipError_t e = hipMemcpy(b->d_filt, b->filt.data(), sizeof(BatchFilter) * b->n, hipMemcpyHostToDevice);
  if (e != hipSuccess) return bhip(b, e, "filter table upload");
  e = hipMemcpy(b->d_stages, b->stages.data(), sizeof(BatchStage) * b->stages.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bhip(b, e, "stage table upload");
  for (auto& c : b->classes) {
    std::vector<uint32_t> map(c.nblocks);
    for (uint32_t f : c.filters)
      for (uint32_t i = 0; i < b->fh[f].ntiles; ++i) map[b->fh[f].first_block + i] = f;
    e = hipMemcpy(c.d_block_filter, map.data(), sizeof(uint32_t) * map.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bhip(b, e, "block map upload");
    e = hipMemcpy(c.d_class_filters, c.filters.data(), sizeof(uint32_t) * c.filters.size(),
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) return bhip(b, e, "class map upload");
  }
  return PF_OK;
}

// Initialisation (Algorithm 1) of filter f with its current seed.
pf_status init_filter(pf_batch* b, uint32_t f) {
  const FilterHost& F = b->fh[f];
  StepArgs<float, float> a;
  std::memset(&a, 0, sizeof(a));
  a.x_out = b->d_x + F.x_off;
  a.lw_out = b->d_lw + F.lw_off;
  a.mp = b->d_mp + f;
  a.ctl = b->d_ctl + f;
  a.d = (uint32_t)F.d;
  a.N = F.N;
  a.k0 = (uint32_t)(F.seed & 0xFFFFFFFFu);
  a.k1 = (uint32_t)(F.seed >> 32);
  a.sid = F.sid;
  LaunchReq rq{};
  rq.what = LW_INIT;
  rq.D = F.D;
  rq.mk = F.mk;
  rq.nt = 256;
  const uint64_t g = (F.N / 2 + 255) / 256;
  rq.grid = (uint32_t)std::min<uint64_t>(g, 65536);
  hipError_t e = launch_f32(rq, &a, b->stream);
  if (e != hipSuccess) return bhip(b, e, "init kernel launch");
  return PF_OK;
}

pf_status init_all(pf_batch* b) {
  for (uint32_t f = 0; f < b->n; ++f) {
    pf_status s = init_filter(b, f);
    if (s != PF_OK) return s;
  }
  hipError_t e = hipMemsetAsync(b->d_tcur, 0, sizeof(uint32_t) * b->n, b->stream);
  if (e != hipSuccess) return bhip(b, e, "step counter clear");
  e = hipMemsetAsync(b->d_rec, 0, sizeof(pf_estimate_t) * b->n, b->stream);
  if (e != hipSuccess) return bhip(b, e, "record clear");
  return PF_OK;
}

// One batched step: every class's step kernel, then every class's
// reductions. No host data besides the two device pointers.
pf_status batch_step(pf_batch* b, const float* y_dev, const uint8_t* active) {
  BatchArgs a{};
  a.filt = b->d_filt;
  a.stages = b->d_stages;
  a.active = active;
  a.y = y_dev;
  a.tcur = b->d_tcur;
  for (auto& c : b->classes) {
    a.block_filter = c.d_block_filter;
    BatchReq rq{0, c.D, c.mk, c.ppt, c.full, c.nblocks, c.lds};
    hipError_t e = launch_batch(rq, a, b->stream);
    if (e != hipSuccess) return bhip(b, e, "batched step launch");
  }
  for (auto& c : b->classes) {
    a.class_filters = c.d_class_filters;
    BatchReq rq{1, c.D, c.mk, c.ppt, c.full, (uint32_t)c.filters.size(), 0};
    hipError_t e = launch_batch(rq, a, b->stream);
    if (e != hipSuccess) return bhip(b, e, "batched finalize launch");
  }
  return PF_OK;
}

// Time `steps` batched steps (after `warm`) on the current plan, in ms.
pf_status time_steps(pf_batch* b, const float* y0, int warm, int steps, float* ms) {
  for (int i = 0; i < warm; ++i) {
    pf_status s = batch_step(b, y0, nullptr);
    if (s != PF_OK) return s;
  }
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return bhip(b, e, "event create");
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return bhip(b, e, "event create");
  }
  (void)hipEventRecord(e0, b->stream);
  pf_status s = PF_OK;
  for (int i = 0; i < steps && s == PF_OK; ++i) s = batch_step(b, y0, nullptr);
  (void)hipEventRecord(e1, b->stream);
  e = hipEventSynchronize(e1);
  if (s == PF_OK && e != hipSuccess) s = bhip(b, e, "event sync");
  if (s == PF_OK) (void)hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return s;
}

// Autotuner: for every class holding filters with radix 0, time the
// candidate tile sizes and radices on the batch itself (observations 0)
// and keep, at the fastest tile size, the largest radix whose step time is
// within kAutoSlack of the fastest (more interaction at almost no cost).
pf_status autotune(pf_batch* b) {
  float* y0 = nullptr;
  pf_status s = balloc(b, reinterpret_cast<void**>(&y0), sizeof(float) * std::max<uint32_t>(b->y_len, 1));
  if (s != PF_OK) return s;
  hipError_t e = hipMemset(y0, 0, sizeof(float) * std::max<uint32_t>(b->y_len, 1));
  if (e != hipSuccess) return bhip(b, e, "tuning observations");
  for (size_t ci = 0; ci < b->classes.size(); ++ci) {
    ClassHost& c = b->classes[ci];
    bool any = false;
    uint64_t nmin = ~0ull;
    for (uint32_t f : c.filters) {
      any |= b->fh[f].autotune;
      nmin = std::min(nmin, b->fh[f].N);
    }
    if (!any) continue;
    std::vector<int> ppts;
    for (int p : {1, 2})
      if (batch_ppt_ok(c.D, p) && 512ull * p <= nmin) ppts.push_back(p);
    struct Trial {
      int ppt;
      uint32_t r;
      float ms;
    };
    std::vector<Trial> trials;
    for (int p : ppts) {
      for (uint32_t r : kAutoRadices) {
        c.ppt = p;
        bool ok = true;
        for (uint32_t f : c.filters)
          if (b->fh[f].autotune) {
            if (r >= b->fh[f].N) ok = false;
            b->fh[f].radix = r;
          }
        if (!ok) continue;
        s = plan_batch(b);
        if (s == PF_OK) s = upload_tables(b);
        if (s != PF_OK) return s;
        float ms = 0.f;
        s = time_steps(b, y0, 2, 4, &ms);
        if (s != PF_OK) return s;
        trials.push_back({p, r, ms});
        pf_batch_tune_t rec{};
        rec.class_index = (uint32_t)ci;
        rec.dim = (uint32_t)c.D;
        rec.model_kind = (uint32_t)c.mk;
        rec.pairs_per_thread = (uint32_t)p;
        rec.radix = r;
        rec.ms_per_step = ms / 4.0f;
        b->tune.push_back(rec);
      }
    }
    if (trials.empty()) return bfail(b, PF_E_UNSUPPORTED, "no batched tile fits the class");
    const Trial* best = &trials[0];
    for (const Trial& t : trials)
      if (t.ms < best->ms) best = &t;
    const Trial* pick = best;
    for (const Trial& t : trials)
      if (t.ppt == best->ppt && t.ms <= kAutoSlack * best->ms && t.r > pick->r) pick = &t;
    c.ppt = pick->ppt;
    for (uint32_t f : c.filters)
      if (b->fh[f].autotune) b->fh[f].radix = pick->r;
    for (auto& rec : b->tune)
      if (rec.class_index == ci && rec.pairs_per_thread == (uint32_t)pick->ppt && rec.radix == pick->r)
        rec.chosen = 1u;
  }
  return PF_OK;
}

bool bpoisoned(pf_batch* b) { return b->sticky != PF_OK; }

pf_status bsync(pf_batch* b) {
  hipError_t e = b->stream ? hipStreamSynchronize(b->stream) : hipDeviceSynchronize();
  if (e != hipSuccess) return bhip(b, e, "synchronize");
  return PF_OK;
}

}  // namespace

extern "C" {

pf_status pf_batch_create(const pf_model* models, const pf_config* cfgs, uint32_t n, void* hip_stream,
                          pf_batch** out) {
  g_batch_create_error.clear();
  if (!out) return bfail(nullptr, PF_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!models || !cfgs || n == 0) return bfail(nullptr, PF_E_INVALID, "models, configs or n missing");
  pf_batch* b = new (std::nothrow) pf_batch();
  if (!b) return bfail(nullptr, PF_E_OOM, "host allocation failed");
  b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  b->dalloc_fn = current_allocator();
  b->n = n;
  b->fh.resize(n);
  auto bail = [&](pf_status s) {
    g_batch_create_error = b->err;
    brelease(b);
    delete b;
    return s;
  };
  std::vector<ModelParams<float>> mps(n);
  std::map<std::pair<int, int>, size_t> cls_of;
  size_t x_elems = 0, lw_elems = 0;
  for (uint32_t f = 0; f < n; ++f) {
    const pf_model* m = models + f;
    const pf_config* c = cfgs + f;
    const std::string who = "filter " + std::to_string(f) + ": ";
    std::string msg;
    if (validate_model(m, msg) != PF_OK) return bail(bfail(b, PF_E_INVALID, who + msg));
    if (!is_pow2(c->n_particles) || c->n_particles < 512 || c->n_particles > (1ull << 30))
      return bail(bfail(b, PF_E_INVALID, who + "n_particles must be a power of two in [512, 2^30]"));
    if (c->radix != 0 && (!is_pow2(c->radix) || c->radix < 2 || c->radix > 64))
      return bail(bfail(b, PF_E_INVALID, who + "radix must be 0 (autotune) or a power of two in [2, 64]"));
    if (c->radix >= c->n_particles)
      return bail(bfail(b, PF_E_UNSUPPORTED, who + "the global path (r >= N) is not batched"));
    if (c->resampler != PF_RESAMPLE_MULTINOMIAL && c->resampler != PF_RESAMPLE_SYSTEMATIC)
      return bail(bfail(b, PF_E_INVALID, who + "unknown resampler"));
    if (c->state_dtype != PF_DTYPE_F32)
      return bail(bfail(b, PF_E_UNSUPPORTED, who + "batched filters use FP32 states"));
    if (c->keep_ancestors) return bail(bfail(b, PF_E_UNSUPPORTED, who + "keep_ancestors is not batched"));
    if (c->full_cycle) return bail(bfail(b, PF_E_UNSUPPORTED, who + "full-cycle steps are not batched"));
    if (c->island) return bail(bfail(b, PF_E_UNSUPPORTED, who + "the island filter is not batched"));
    if (c->ess_threshold != 0.0) return bail(bfail(b, PF_E_UNSUPPORTED, who + "ESS-gated stages are not batched"));
    FilterHost& F = b->fh[f];
    F.kind = m->kind;
    F.d = m->d;
    F.D = compiled_dim(m->d);
    fill_params<float>(m, m->d, &mps[f], &F.mk);
    F.N = c->n_particles;
    F.autotune = c->radix == 0;
    F.radix = c->radix;
    F.seed = c->seed;
    F.sid = c->stream_id;
    F.systematic = c->resampler == PF_RESAMPLE_SYSTEMATIC ? 1u : 0u;
    F.yoff = b->y_len;
    b->y_len += (uint32_t)m->d;
    F.x_off = x_elems;
    x_elems += 2ull * F.d * F.N;
    F.lw_off = lw_elems;
    lw_elems += 2ull * F.N;
    auto key = std::make_pair(F.D, F.mk);
    if (!cls_of.count(key)) {
      cls_of[key] = b->classes.size();
      ClassHost ch;
      ch.D = F.D;
      ch.mk = F.mk;
      ch.ppt = 1;
      b->classes.push_back(ch);
    }
    b->classes[cls_of[key]].filters.push_back(f);
    if (F.d != F.D) b->classes[cls_of[key]].full = 0;
  }
  // default tile: two pairs per thread where every filter of the class has
  // at least 1024 particles
  for (auto& c : b->classes) {
    uint64_t nmin = ~0ull;
    for (uint32_t f : c.filters) nmin = std::min(nmin, b->fh[f].N);
    c.ppt = (batch_ppt_ok(c.D, 2) && nmin >= 1024) ? 2 : 1;
  }
  // partial records: at most N / 512 tiles per filter
  size_t part_elems = 0;
  for (auto& F : b->fh) {
    F.part_off = part_elems;
    part_elems += (F.N / 512) * (size_t)partial_stride(F.D);
    if (F.autotune) F.radix = std::min<uint64_t>(64, F.N / 2);
  }
  pf_status s;
  void* p = nullptr;
  if ((s = balloc(b, &p, sizeof(float) * x_elems)) != PF_OK) return bail(s);
  b->d_x = reinterpret_cast<float*>(p);
  if ((s = balloc(b, &p, sizeof(float) * lw_elems)) != PF_OK) return bail(s);
  b->d_lw = reinterpret_cast<float*>(p);
  if ((s = balloc(b, &p, sizeof(float) * part_elems)) != PF_OK) return bail(s);
  b->d_part = reinterpret_cast<float*>(p);
  if ((s = balloc(b, &p, sizeof(Ctl) * n)) != PF_OK) return bail(s);
  b->d_ctl = reinterpret_cast<Ctl*>(p);
  if ((s = balloc(b, &p, sizeof(pf_estimate_t) * n)) != PF_OK) return bail(s);
  b->d_rec = reinterpret_cast<pf_estimate_t*>(p);
  if ((s = balloc(b, &p, sizeof(ModelParams<float>) * n)) != PF_OK) return bail(s);
  b->d_mp = reinterpret_cast<ModelParams<float>*>(p);
  if ((s = balloc(b, &p, sizeof(uint32_t) * n)) != PF_OK) return bail(s);
  b->d_tcur = reinterpret_cast<uint32_t*>(p);
  if ((s = balloc(b, &p, sizeof(BatchFilter) * n)) != PF_OK) return bail(s);
  b->d_filt = reinterpret_cast<BatchFilter*>(p);
  size_t max_stages = 0;
  for (auto& F : b->fh) max_stages += ilog2(F.N);  // radix 2 is the longest plan
  if ((s = balloc(b, &p, sizeof(BatchStage) * max_stages)) != PF_OK) return bail(s);
  b->d_stages = reinterpret_cast<BatchStage*>(p);
  for (auto& c : b->classes) {
    size_t maxblocks = 0;
    for (uint32_t f : c.filters) maxblocks += b->fh[f].N / 512;
    if ((s = balloc(b, &p, sizeof(uint32_t) * maxblocks)) != PF_OK) return bail(s);
    c.d_block_filter = reinterpret_cast<uint32_t*>(p);
    if ((s = balloc(b, &p, sizeof(uint32_t) * c.filters.size())) != PF_OK) return bail(s);
    c.d_class_filters = reinterpret_cast<uint32_t*>(p);
  }
  hipError_t e = hipMemcpy(b->d_mp, mps.data(), sizeof(ModelParams<float>) * n, hipMemcpyHostToDevice);
  if (e != hipSuccess) return bail(bhip(b, e, "model upload"));
  if ((s = plan_batch(b)) != PF_OK) return bail(s);
  if ((s = upload_tables(b)) != PF_OK) return bail(s);
  if ((s = init_all(b)) != PF_OK) return bail(s);
  bool any_auto = false;
  for (auto& F : b->fh) any_auto |= F.autotune;
  if (any_auto) {
    if ((s = autotune(b)) != PF_OK) return bail(s);
    if ((s = plan_batch(b)) != PF_OK) return bail(s);
    if ((s = upload_tables(b)) != PF_OK) return bail(s);
    if ((s = init_all(b)) != PF_OK) return bail(s);
  }
  if ((s = bsync(b)) != PF_OK) return bail(s);
  *out = b;
  return PF_OK;
}

pf_status pf_batch_destroy(pf_batch* b) {
  if (!b) return PF_OK;
  (void)(b->stream ? hipStreamSynchronize(b->stream) : hipDeviceSynchronize());
  brelease(b);
  delete b;
  return PF_OK;
}

pf_status pf_batch_step(pf_batch* b, const float* y_dev, const uint8_t* active_dev) {
  if (!b) return PF_E_INVALID;
  if (bpoisoned(b)) return PF_E_STATE;
  if (!y_dev) return bfail(b, PF_E_INVALID, "y_dev is NULL");
  return batch_step(b, y_dev, active_dev);
}

pf_status pf_batch_run(pf_batch* b, const float* y_dev, uint32_t n_steps, uint64_t y_stride,
                       const uint8_t* active_dev, int32_t use_graph) {
  if (!b) return PF_E_INVALID;
  if (bpoisoned(b)) return PF_E_STATE;
  if (!y_dev) return bfail(b, PF_E_INVALID, "y_dev is NULL");
  if (y_stride < b->y_len) return bfail(b, PF_E_INVALID, "y_stride below the packed observation length");
  if (n_steps == 0) return PF_OK;
  if (use_graph && !b->stream) return bfail(b, PF_E_INVALID, "graph capture needs a non-default stream");
  if (use_graph) {
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bhip(b, e, "hipStreamBeginCapture");
  }
  pf_status st = PF_OK;
  for (uint32_t j = 0; j < n_steps && st == PF_OK; ++j) st = batch_step(b, y_dev + (size_t)j * y_stride, active_dev);
  if (use_graph) {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (st != PF_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return bhip(b, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return bhip(b, e, "hipGraphInstantiate");
    }
    e = hipGraphLaunch(exec, b->stream);
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return bhip(b, e, "hipGraphLaunch");
  }
  return st;
}

pf_status pf_batch_sync(pf_batch* b) {
  if (!b) return PF_E_INVALID;
  return bsync(b);
}

pf_status pf_batch_estimates(pf_batch* b, pf_estimate_t* out) {
  if (!b || !out) return PF_E_INVALID;
  if (bpoisoned(b)) return PF_E_STATE;
  pf_status s = bsync(b);
  if (s != PF_OK) return s;
  hipError_t e = hipMemcpy(out, b->d_rec, sizeof(pf_estimate_t) * b->n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bhip(b, e, "record copy");
  return PF_OK;
}

pf_status pf_batch_filter_info(pf_batch* b, uint32_t f, pf_info_t* out) {
  if (!b || !out || f >= b->n) return PF_E_INVALID;
  std::memset(out, 0, sizeof(*out));
  const FilterHost& F = b->fh[f];
  out->n_particles = F.N;
  out->d = (uint32_t)F.d;
  out->n_stages = (uint32_t)F.radices.size();
  const uint32_t E = F.ntiles ? (uint32_t)(F.N / F.ntiles) : 0u;
  for (size_t k = 0; k < F.radices.size() && k < 32; ++k) {
    out->radices[k] = F.radices[k];
    out->tile_elems[k] = E;
  }
  out->state_dtype = PF_DTYPE_F32;
  out->device_bytes = b->bytes;
  uint32_t t = 0;
  if (!bpoisoned(b) && bsync(b) == PF_OK)
    (void)hipMemcpy(&t, b->d_tcur + f, sizeof(t), hipMemcpyDeviceToHost);
  out->t = t;
  return PF_OK;
}

pf_status pf_batch_tuning(pf_batch* b, pf_batch_tune_t* out, uint32_t n_max, uint32_t* n_out) {
  if (!b || !n_out) return PF_E_INVALID;
  const uint32_t n = (uint32_t)std::min<size_t>(b->tune.size(), n_max);
  if (out)
    for (uint32_t i = 0; i < n; ++i) out[i] = b->tune[i];
  *n_out = out ? n : (uint32_t)b->tune.size();
  return PF_OK;
}

pf_status pf_batch_get_state(pf_batch* b, uint32_t f, float* x_host, float* logw_host, uint32_t* t_out,
                             double* log_norm) {
  if (!b || f >= b->n) return PF_E_INVALID;
  if (bpoisoned(b)) return PF_E_STATE;
  pf_status s = bsync(b);
  if (s != PF_OK) return s;
  const FilterHost& F = b->fh[f];
  uint32_t t = 0;
  hipError_t e = hipMemcpy(&t, b->d_tcur + f, sizeof(t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bhip(b, e, "step counter copy");
  const float* xs = b->d_x + F.x_off + (t & 1u) * (size_t)F.d * F.N;
  const float* ws = b->d_lw + F.lw_off + (t & 1u) * (size_t)F.N;
  if (x_host) {
    e = hipMemcpy(x_host, xs, sizeof(float) * F.d * F.N, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return bhip(b, e, "state copy");
  }
  Ctl c;
  e = hipMemcpy(&c, b->d_ctl + f, sizeof(c), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bhip(b, e, "control copy");
  if (logw_host) {
    e = hipMemcpy(logw_host, ws, sizeof(float) * F.N, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return bhip(b, e, "log-weight copy");
    double off = -INFINITY;
    for (int sl = 0; sl < kOffSlots; ++sl)
      off = std::max(off, ord_decode(c.offs[(t % kOffRing) * kOffSlots * kOffStride + sl * kOffStride]));
    const float o = (float)off;
    for (uint64_t i = 0; i < F.N; ++i) logw_host[i] -= o;
  }
  if (t_out) *t_out = t;
  if (log_norm) *log_norm = c.log_norm;
  return PF_OK;
}

pf_status pf_batch_set_state(pf_batch* b, uint32_t f, const float* x_host, const float* logw_host, uint32_t t,
                             double log_norm) {
  if (!b || f >= b->n || !x_host) return PF_E_INVALID;
  if (bpoisoned(b)) return PF_E_STATE;
  pf_status s = bsync(b);
  if (s != PF_OK) return s;
  const FilterHost& F = b->fh[f];
  float* xs = b->d_x + F.x_off + (t & 1u) * (size_t)F.d * F.N;
  float* ws = b->d_lw + F.lw_off + (t & 1u) * (size_t)F.N;
  hipError_t e = hipMemcpy(xs, x_host, sizeof(float) * F.d * F.N, hipMemcpyHostToDevice);
  if (e != hipSuccess) return bhip(b, e, "state upload");
  if (logw_host) e = hipMemcpy(ws, logw_host, sizeof(float) * F.N, hipMemcpyHostToDevice);
  else e = hipMemset(ws, 0, sizeof(float) * F.N);
  if (e != hipSuccess) return bhip(b, e, "log-weight upload");
  Ctl c;
  e = hipMemcpy(&c, b->d_ctl + f, sizeof(c), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bhip(b, e, "control copy");
  c.log_norm = log_norm;
  c.t = t;
  for (int i = 0; i < kOffEntries; ++i) c.offs[i] = ord_encode(-INFINITY);
  c.offs[(t % kOffRing) * kOffSlots * kOffStride] = ord_encode(0.0);
  e = hipMemcpy(b->d_ctl + f, &c, sizeof(c), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bhip(b, e, "control upload");
  e = hipMemcpy(b->d_tcur + f, &t, sizeof(t), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bhip(b, e, "step counter upload");
  return PF_OK;
}

pf_status pf_batch_reset(pf_batch* b, uint32_t f, uint64_t seed, uint32_t stream_id) {
  if (!b || f >= b->n) return PF_E_INVALID;
  if (bpoisoned(b)) return PF_E_STATE;
  FilterHost& F = b->fh[f];
  F.seed = seed;
  F.sid = stream_id;
  BatchFilter& T = b->filt[f];
  T.sid = stream_id;
  T.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
  T.k1 = (uint32_t)(seed >> 32);
  hipError_t e = hipMemcpyAsync(b->d_filt + f, &T, sizeof(T), hipMemcpyHostToDevice, b->stream);
  if (e != hipSuccess) return bhip(b, e, "filter entry upload");
  pf_status s = init_filter(b, f);
  if (s != PF_OK) return s;
  e = hipMemsetAsync(b->d_tcur + f, 0, sizeof(uint32_t), b->stream);
  if (e != hipSuccess) return bhip(b, e, "step counter clear");
  e = hipMemsetAsync(b->d_rec + f, 0, sizeof(pf_estimate_t), b->stream);
  if (e != hipSuccess) return bhip(b, e, "record clear");
  return bsync(b);
}

const char* pf_batch_last_error(const pf_batch* b) {
  if (!b) return g_batch_create_error.c_str();
  return b->err.c_str();
}

}  // extern "C"
