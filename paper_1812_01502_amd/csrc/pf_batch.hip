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
  bool vacant;                     // no filter: no particle memory, never steps
  float *x, *lw, *part;            // device buffers (in the create-time pools, or own)
  void* own;                       // the slot's own allocation after a rebind (else null)
};

struct ClassHost {
  int D, mk, ppt;
  int full = 1;  // every filter has d = D
  std::vector<uint32_t> filters;
  uint32_t nblocks = 0;
  size_t lds = 0;
  uint32_t* d_block_filter = nullptr;
  uint32_t* d_class_filters = nullptr;
  size_t cap_blocks = 0, cap_filters = 0;  // capacities of the two maps
};

}  // namespace

// Streams besides the caller's over which the dimension classes of a step
// are spread (the classes share no data, so their launches may overlap).
constexpr int kAuxStreams = 3;

struct pf_batch {
  hipStream_t stream = nullptr;
  hipStream_t aux[kAuxStreams] = {};  // created with the batch when `stream` is not the null stream
  hipEvent_t ev_fork = nullptr, ev_join[kAuxStreams] = {};
  int naux = 0;
  uint32_t n = 0;
  uint32_t y_len = 0;
  std::vector<FilterHost> fh;
  std::vector<ClassHost> classes;
  // device
  BatchFilter* d_filt = nullptr;
  BatchStage* d_stages = nullptr;
  size_t cap_stages = 0;
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

// Give back one allocation made by balloc.
void bfree(pf_batch* b, void* p) {
  if (!p) return;
  auto it = std::find(b->allocs.begin(), b->allocs.end(), p);
  if (it != b->allocs.end()) b->allocs.erase(it);
  dev_free(b->dalloc_fn, p);
}

void brelease(pf_batch* b) {
  for (void* p : b->allocs) dev_free(b->dalloc_fn, p);
  b->allocs.clear();
  for (int k = 0; k < b->naux; ++k) {
    if (b->ev_join[k]) (void)hipEventDestroy(b->ev_join[k]);
    if (b->aux[k]) (void)hipStreamDestroy(b->aux[k]);
    b->ev_join[k] = nullptr;
    b->aux[k] = nullptr;
  }
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  b->ev_fork = nullptr;
  b->naux = 0;
}

// The streams the classes run on (default priority, not synchronising with
// the null stream) and the events that fork them from and join them to the
// caller's stream. Only with a caller's stream: work on the null stream is
// not forked.
pf_status create_aux_streams(pf_batch* b) {
  if (!b->stream) return PF_OK;
  hipError_t e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
  if (e != hipSuccess) return bhip(b, e, "event create");
  for (int k = 0; k < kAuxStreams; ++k) {
    e = hipStreamCreateWithFlags(&b->aux[k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join[k], hipEventDisableTiming);
    if (e != hipSuccess) {
      b->naux = k + 1;
      return bhip(b, e, "class stream create");
    }
  }
  b->naux = kAuxStreams;
  return PF_OK;
}

// Stage tables of every filter for the current radices and class tiles;
// block maps of every class. Host tables only.
pf_status plan_batch(pf_batch* b) {
  b->stages.clear();
  b->y_len = 0;
  for (auto& F : b->fh) {
    F.yoff = b->y_len;
    if (!F.vacant) b->y_len += (uint32_t)F.d;
  }
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
    if (F.vacant) continue;  // never addressed: no block and no class lists it
    T.x[0] = F.x;
    T.x[1] = F.x + (size_t)F.d * F.N;
    T.lw[0] = F.lw;
    T.lw[1] = F.lw + F.N;
    T.mp = b->d_mp + f;
    T.part = F.part;
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
  if (!b->stages.empty()) {
    e = hipMemcpy(b->d_stages, b->stages.data(), sizeof(BatchStage) * b->stages.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bhip(b, e, "stage table upload");
  }
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
  a.x_out = F.x;
  a.lw_out = F.lw;
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
    if (b->fh[f].vacant) continue;
    pf_status s = init_filter(b, f);
    if (s != PF_OK) return s;
  }
  hipError_t e = hipMemsetAsync(b->d_tcur, 0, sizeof(uint32_t) * b->n, b->stream);
  if (e != hipSuccess) return bhip(b, e, "step counter clear");
  e = hipMemsetAsync(b->d_rec, 0, sizeof(pf_estimate_t) * b->n, b->stream);
  if (e != hipSuccess) return bhip(b, e, "record clear");
  return PF_OK;
}

// Steps j = 0 .. n_steps - 1 (observations at y_dev + j y_stride): per
// step, each class's step kernel, then its reductions. With `fork`, class i
// runs on stream i mod (1 + naux) (0 = the caller's): the class streams wait
// for the caller's stream first, and it waits for them at the end, so the
// classes' launches may overlap (also inside a captured graph, as parallel
// branches). No host data besides the device pointers.
pf_status batch_steps(pf_batch* b, const float* y_dev, uint32_t n_steps, uint64_t y_stride,
                      const uint8_t* active, bool fork) {
  uint32_t nc = 0;
  for (auto& c : b->classes) nc += c.filters.empty() ? 0u : 1u;
  fork = fork && b->naux > 0 && nc > 1;
  const int nstreams = fork ? std::min<int>(1 + b->naux, (int)nc) : 1;
  hipError_t e;
  if (fork) {
    if ((e = hipEventRecord(b->ev_fork, b->stream)) != hipSuccess) return bhip(b, e, "fork event");
    for (int k = 0; k + 1 < nstreams; ++k)
      if ((e = hipStreamWaitEvent(b->aux[k], b->ev_fork, 0)) != hipSuccess) return bhip(b, e, "fork wait");
  }
  BatchArgs a{};
  a.filt = b->d_filt;
  a.stages = b->d_stages;
  a.active = active;
  a.tcur = b->d_tcur;
  for (uint32_t j = 0; j < n_steps; ++j) {
    a.y = y_dev + (size_t)j * y_stride;
    uint32_t ci = 0;
    for (auto& c : b->classes) {
      if (c.filters.empty()) continue;
      const int k = (int)(ci++ % (uint32_t)nstreams);
      hipStream_t st = k == 0 ? b->stream : b->aux[k - 1];
      a.block_filter = c.d_block_filter;
      BatchReq rq{0, c.D, c.mk, c.ppt, c.full, c.nblocks, c.lds};
      if ((e = launch_batch(rq, a, st)) != hipSuccess) return bhip(b, e, "batched step launch");
      a.class_filters = c.d_class_filters;
      BatchReq rf{1, c.D, c.mk, c.ppt, c.full, (uint32_t)c.filters.size(), 0};
      if ((e = launch_batch(rf, a, st)) != hipSuccess) return bhip(b, e, "batched finalize launch");
    }
  }
  if (fork) {
    for (int k = 0; k + 1 < nstreams; ++k) {
      if ((e = hipEventRecord(b->ev_join[k], b->aux[k])) != hipSuccess) return bhip(b, e, "join event");
      if ((e = hipStreamWaitEvent(b->stream, b->ev_join[k], 0)) != hipSuccess) return bhip(b, e, "join wait");
    }
  }
  return PF_OK;
}
pf_status batch_step(pf_batch* b, const float* y_dev, const uint8_t* active) {
  return batch_steps(b, y_dev, 1, 0, active, false);
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

// Validation of one slot's model and configuration (create and rebind).
// n_particles = 0 asks for a vacant slot: the model is then not used.
pf_status check_slot_config(const pf_model* m, const pf_config* c, std::string& msg) {
  if (!m || !c) {
    msg = "model or configuration is NULL";
    return PF_E_INVALID;
  }
  if (c->n_particles == 0) return PF_OK;
  if (validate_model(m, msg) != PF_OK) return PF_E_INVALID;
  auto bad = [&](pf_status st, const char* why) {
    msg = why;
    return st;
  };
  if (!is_pow2(c->n_particles) || c->n_particles < 512 || c->n_particles > (1ull << 30))
    return bad(PF_E_INVALID, "n_particles must be 0 (vacant) or a power of two in [512, 2^30]");
  if (c->radix != 0 && (!is_pow2(c->radix) || c->radix < 2 || c->radix > 64))
    return bad(PF_E_INVALID, "radix must be 0 (autotune) or a power of two in [2, 64]");
  if (c->radix >= c->n_particles) return bad(PF_E_UNSUPPORTED, "the global path (r >= N) is not batched");
  if (c->resampler != PF_RESAMPLE_MULTINOMIAL && c->resampler != PF_RESAMPLE_SYSTEMATIC)
    return bad(PF_E_INVALID, "unknown resampler");
  if (c->state_dtype != PF_DTYPE_F32) return bad(PF_E_UNSUPPORTED, "batched filters use FP32 states");
  if (c->keep_ancestors) return bad(PF_E_UNSUPPORTED, "keep_ancestors is not batched");
  if (c->full_cycle) return bad(PF_E_UNSUPPORTED, "full-cycle steps are not batched");
  if (c->island) return bad(PF_E_UNSUPPORTED, "the island filter is not batched");
  if (c->ess_threshold != 0.0) return bad(PF_E_UNSUPPORTED, "ESS-gated stages are not batched");
  return PF_OK;
}

// Host description of a slot from a checked model and configuration (the
// device buffers are set by the caller).
void bind_host(FilterHost& F, const pf_model* m, const pf_config* c, ModelParams<float>* mp) {
  F = FilterHost{};
  F.vacant = c->n_particles == 0;
  if (F.vacant) {
    F.d = 0;
    F.D = 1;
    F.N = 0;
    return;
  }
  F.kind = m->kind;
  F.d = m->d;
  F.D = compiled_dim(m->d);
  fill_params<float>(m, m->d, mp, &F.mk);
  F.N = c->n_particles;
  F.autotune = c->radix == 0;
  F.radix = c->radix == 0 ? std::min<uint64_t>(64, F.N / 2) : c->radix;
  F.seed = c->seed;
  F.sid = c->stream_id;
  F.systematic = c->resampler == PF_RESAMPLE_SYSTEMATIC ? 1u : 0u;
}

// Classes (one per state dimension and model kind) of the occupied slots. A
// class that exists keeps its tile (and device maps) while every member
// still fits it; a new class takes two pairs per thread where every member
// has at least 1024 particles.
void rebuild_classes(pf_batch* b) {
  std::vector<ClassHost> old;
  old.swap(b->classes);
  std::map<std::pair<int, int>, size_t> cls_of;
  for (uint32_t f = 0; f < b->n; ++f) {
    const FilterHost& F = b->fh[f];
    if (F.vacant) continue;
    const auto key = std::make_pair(F.D, F.mk);
    if (!cls_of.count(key)) {
      cls_of[key] = b->classes.size();
      ClassHost ch;
      ch.D = F.D;
      ch.mk = F.mk;
      ch.ppt = 0;
      for (auto& o : old)
        if (o.D == F.D && o.mk == F.mk) {
          ch = o;
          ch.filters.clear();
          ch.full = 1;
          o.d_block_filter = nullptr;
          o.d_class_filters = nullptr;
        }
      b->classes.push_back(ch);
    }
    ClassHost& c = b->classes[cls_of[key]];
    c.filters.push_back(f);
    if (F.d != F.D) c.full = 0;
  }
  for (auto& o : old) {  // classes that lost every member
    bfree(b, o.d_block_filter);
    bfree(b, o.d_class_filters);
  }
  for (auto& c : b->classes) {
    uint64_t nmin = ~0ull;
    for (uint32_t f : c.filters) nmin = std::min(nmin, b->fh[f].N);
    if (c.ppt == 0) c.ppt = (batch_ppt_ok(c.D, 2) && nmin >= 1024) ? 2 : 1;
    if (512ull * (uint64_t)c.ppt > nmin) c.ppt = 1;
  }
}

// Device tables large enough for the current slots: the stage table and
// every class's block and member maps (grown, never shrunk).
pf_status ensure_tables(pf_batch* b) {
  size_t need = 1;
  for (auto& F : b->fh)
    if (!F.vacant) need += ilog2(F.N);  // radix 2 is the longest plan
  pf_status s;
  void* p = nullptr;
  if (need > b->cap_stages) {
    if ((s = balloc(b, &p, sizeof(BatchStage) * need)) != PF_OK) return s;
    bfree(b, b->d_stages);
    b->d_stages = reinterpret_cast<BatchStage*>(p);
    b->cap_stages = need;
  }
  for (auto& c : b->classes) {
    size_t blocks = 0;
    for (uint32_t f : c.filters) blocks += b->fh[f].N / 512;
    if (blocks > c.cap_blocks) {
      if ((s = balloc(b, &p, sizeof(uint32_t) * blocks)) != PF_OK) return s;
      bfree(b, c.d_block_filter);
      c.d_block_filter = reinterpret_cast<uint32_t*>(p);
      c.cap_blocks = blocks;
    }
    if (c.filters.size() > c.cap_filters) {
      if ((s = balloc(b, &p, sizeof(uint32_t) * c.filters.size())) != PF_OK) return s;
      bfree(b, c.d_class_filters);
      c.d_class_filters = reinterpret_cast<uint32_t*>(p);
      c.cap_filters = c.filters.size();
    }
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
  size_t x_elems = 0, lw_elems = 0, part_elems = 0;
  for (uint32_t f = 0; f < n; ++f) {
    std::string msg;
    const pf_status cs = check_slot_config(models + f, cfgs + f, msg);
    if (cs != PF_OK) return bail(bfail(b, cs, "filter " + std::to_string(f) + ": " + msg));
    FilterHost& F = b->fh[f];
    bind_host(F, models + f, cfgs + f, &mps[f]);
    if (F.vacant) continue;
    x_elems += 2ull * F.d * F.N;
    lw_elems += 2ull * F.N;
    part_elems += (F.N / 512) * (size_t)partial_stride(F.D);
  }
  pf_status s;
  void* p = nullptr;
  if ((s = balloc(b, &p, sizeof(float) * x_elems)) != PF_OK) return bail(s);
  b->d_x = reinterpret_cast<float*>(p);
  if ((s = balloc(b, &p, sizeof(float) * lw_elems)) != PF_OK) return bail(s);
  b->d_lw = reinterpret_cast<float*>(p);
  if ((s = balloc(b, &p, sizeof(float) * part_elems)) != PF_OK) return bail(s);
  b->d_part = reinterpret_cast<float*>(p);
  x_elems = lw_elems = part_elems = 0;
  for (auto& F : b->fh) {
    if (F.vacant) continue;
    F.x = b->d_x + x_elems;
    F.lw = b->d_lw + lw_elems;
    F.part = b->d_part + part_elems;
    x_elems += 2ull * F.d * F.N;
    lw_elems += 2ull * F.N;
    part_elems += (F.N / 512) * (size_t)partial_stride(F.D);
  }
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
  rebuild_classes(b);
  if ((s = ensure_tables(b)) != PF_OK) return bail(s);
  hipError_t e0 = hipMemset(b->d_rec, 0, sizeof(pf_estimate_t) * n);
  if (e0 != hipSuccess) return bail(bhip(b, e0, "record clear"));
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
  if ((s = create_aux_streams(b)) != PF_OK) return bail(s);
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
  return batch_steps(b, y_dev, 1, 0, active_dev, true);
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
  pf_status st = batch_steps(b, y_dev, n_steps, y_stride, active_dev, true);
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
  if (F.vacant) return bfail(b, PF_E_STATE, "filter " + std::to_string(f) + " is vacant");
  uint32_t t = 0;
  hipError_t e = hipMemcpy(&t, b->d_tcur + f, sizeof(t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bhip(b, e, "step counter copy");
  const float* xs = F.x + (t & 1u) * (size_t)F.d * F.N;
  const float* ws = F.lw + (t & 1u) * (size_t)F.N;
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
  if (F.vacant) return bfail(b, PF_E_STATE, "filter " + std::to_string(f) + " is vacant");
  float* xs = F.x + (t & 1u) * (size_t)F.d * F.N;
  float* ws = F.lw + (t & 1u) * (size_t)F.N;
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
  c.fail_t = kNoFail;
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
  if (F.vacant) return bfail(b, PF_E_STATE, "filter " + std::to_string(f) + " is vacant");
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

pf_status pf_batch_estimates_async(pf_batch* b, pf_estimate_t* out) {
  if (!b || !out) return PF_E_INVALID;
  if (bpoisoned(b)) return PF_E_STATE;
  hipError_t e = hipMemcpyAsync(out, b->d_rec, sizeof(pf_estimate_t) * b->n, hipMemcpyDeviceToHost, b->stream);
  if (e != hipSuccess) return bhip(b, e, "record copy");
  return PF_OK;
}

pf_status pf_batch_rebind(pf_batch* b, uint32_t count, const uint32_t* slots, const pf_model* models,
                          const pf_config* cfgs) {
  if (!b || (count && (!slots || !models || !cfgs))) return PF_E_INVALID;
  if (bpoisoned(b)) return PF_E_STATE;
  std::vector<char> seen(b->n, 0);
  for (uint32_t i = 0; i < count; ++i) {
    const uint32_t f = slots[i];
    if (f >= b->n) return bfail(b, PF_E_INVALID, "slot " + std::to_string(f) + " is out of range");
    if (seen[f]) return bfail(b, PF_E_INVALID, "slot " + std::to_string(f) + " is listed twice");
    seen[f] = 1;
    std::string msg;
    const pf_status cs = check_slot_config(models + i, cfgs + i, msg);
    if (cs != PF_OK) return bfail(b, cs, "filter " + std::to_string(f) + ": " + msg);
  }
  if (count == 0) return PF_OK;
  pf_status s = bsync(b);
  if (s != PF_OK) return s;
  // release first, so that the new filters can reuse the memory
  for (uint32_t i = 0; i < count; ++i) {
    FilterHost& F = b->fh[slots[i]];
    bfree(b, F.own);
    F = FilterHost{};
    F.vacant = true;
  }
  pf_status first_err = PF_OK;
  std::vector<uint32_t> bound;
  for (uint32_t i = 0; i < count; ++i) {
    const uint32_t f = slots[i];
    FilterHost& F = b->fh[f];
    ModelParams<float> mp{};
    bind_host(F, models + i, cfgs + i, &mp);
    F.autotune = false;
    if (F.vacant) continue;
    // one allocation: states (2 d N), log-weights (2 N), tile records
    // ((N / 512) (4 + 3 D)), each part 256-byte aligned
    auto up = [](size_t v) { return (v + 63u) & ~(size_t)63u; };
    const size_t nx = up(2ull * F.d * F.N), nl = up(2ull * F.N), np = up((F.N / 512) * (size_t)partial_stride(F.D));
    void* p = nullptr;
    if ((s = balloc(b, &p, sizeof(float) * (nx + nl + np))) != PF_OK) {
      F = FilterHost{};
      F.vacant = true;  // this slot stays vacant; the others are bound
      if (first_err == PF_OK) first_err = s;
      continue;
    }
    F.own = p;
    F.x = reinterpret_cast<float*>(p);
    F.lw = F.x + nx;
    F.part = F.lw + nl;
    hipError_t e = hipMemcpy(b->d_mp + f, &mp, sizeof(mp), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bhip(b, e, "model upload");
    bound.push_back(f);
  }
  rebuild_classes(b);
  if ((s = ensure_tables(b)) != PF_OK) return s;
  if ((s = plan_batch(b)) != PF_OK) return s;
  if ((s = upload_tables(b)) != PF_OK) return s;
  for (uint32_t f : bound)
    if ((s = init_filter(b, f)) != PF_OK) return s;
  for (uint32_t i = 0; i < count; ++i) {
    const uint32_t f = slots[i];
    hipError_t e = hipMemsetAsync(b->d_tcur + f, 0, sizeof(uint32_t), b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_rec + f, 0, sizeof(pf_estimate_t), b->stream);
    if (e != hipSuccess) return bhip(b, e, "slot clear");
  }
  if ((s = bsync(b)) != PF_OK) return s;
  return first_err;
}

const char* pf_batch_last_error(const pf_batch* b) {
  if (!b) return g_batch_create_error.c_str();
  return b->err.c_str();
}

}  // extern "C"
