// pf_noalloc.hip - pf_run_noalloc: pf_run's butterfly steps on caller-owned
// state buffers, with every other device buffer (control block, model
// parameters, per-tile reduction records) in one fixed-size file-scope
// device array. For callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "../../include/pf.h"
#include "pf_host.h"

using namespace pfk;
using namespace pfh;

namespace pfh {
// defined in pf_runtime.hip
pf_status plan_butterfly(uint64_t N, uint64_t radix, int D, int d, size_t tsz, bool island, StagePlan* out,
                         uint32_t max_out, uint32_t* n_out, char* err, size_t errlen);
void set_create_error(const char* msg);
}  // namespace pfh

namespace {

// Scratch of pf_run_noalloc: [control block | model parameters | tile
// records of one step], each part 256-byte aligned. One copy per device,
// shared by every call on that device.
constexpr size_t kScratchBytes = 1u << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

constexpr size_t up256(size_t v) { return (v + 255u) & ~(size_t)255u; }

// The device address of this device's scratch (looked up once per device).
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Bytes copied into device memory through a kernel's own arguments, so the
// copy needs no host buffer that outlives the call (and can be captured).
constexpr size_t kChunk = 3072;
struct Chunk {
  unsigned char b[kChunk];
};
__global__ void __launch_bounds__(256) pf_noalloc_bytes(unsigned char* dst, Chunk c, uint32_t n) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = c.b[i];
}

// Control block of a fresh run: offset 0 for the first step, no earlier
// failure, log-normaliser 0 (as the initialisation kernel leaves it).
__global__ void __launch_bounds__(64) pf_noalloc_ctl(Ctl* c) {
  clear_offset(c, 0u, 0.0);
  clear_offset(c, 1u, -INFINITY);
  clear_offset(c, 2u, -INFINITY);
  if (threadIdx.x == 0) {
    c->log_norm = 0.0;
    c->t = 0u;
    c->ad_active = c->ad_stage = c->ad_run = c->ad_next = 0u;
    c->fail_t = kNoFail;
  }
}

thread_local char g_err[256];

pf_status nfail(pf_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
pf_status nfail(pf_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  set_create_error(g_err);
  return s;
}

hipError_t launch_dtype(int dtype, const LaunchReq& rq, const void* args, hipStream_t st) {
  switch (dtype) {
    case PF_DTYPE_F32: return launch_f32(rq, args, st);
    case PF_DTYPE_BF16: return launch_bf16(rq, args, st);
    default: return launch_f64(rq, args, st);
  }
}

template <typename T, typename S>
pf_status run_noalloc(const pf_model* model, const pf_config* cfg, void* x_dev, void* logw_dev,
                      const void* y_dev, uint32_t n_steps, uint64_t y_stride, uint32_t t0, pf_estimate_t* est_dev,
                      hipStream_t st) {
  const int d = model->d;
  const int D = compiled_dim(d);
  const uint64_t N = cfg->n_particles;
  StagePlan plan[32];
  uint32_t S_ = 0;
  char why[160];
  pf_status ps = plan_butterfly(N, cfg->radix, D, d, sizeof(T), false, plan, 32, &S_, why, sizeof(why));
  if (ps != PF_OK) return nfail(ps, "pf_run_noalloc: %s", why);
  size_t part = 0;
  for (uint32_t k = 0; k < S_; ++k) part = std::max(part, (size_t)plan[k].ntiles * partial_stride(D) * sizeof(T));
  const size_t off_mp = up256(sizeof(Ctl));
  const size_t off_part = off_mp + up256(sizeof(ModelParams<T>));
  if (off_part + part > kScratchBytes)
    return nfail(PF_E_UNSUPPORTED,
                 "pf_run_noalloc: N = %llu with d = %d needs %zu bytes of scratch, more than its %zu (use pf_create "
                 "and pf_run)",
                 (unsigned long long)N, d, off_part + part, kScratchBytes);
  void* sp = nullptr;
  hipError_t e = scratch_address(&sp);
  if (e != hipSuccess) return nfail(PF_E_HIP, "pf_run_noalloc: scratch address: %s", hipGetErrorString(e));
  unsigned char* base = reinterpret_cast<unsigned char*>(sp);
  Ctl* ctl = reinterpret_cast<Ctl*>(base);
  ModelParams<T>* mp_dev = reinterpret_cast<ModelParams<T>*>(base + off_mp);
  T* part_dev = reinterpret_cast<T*>(base + off_part);
  // model parameters and control block
  ModelParams<T> mp;
  std::memset(&mp, 0, sizeof(mp));
  int mk = 0;
  fill_params<T>(model, d, &mp, &mk);
  const unsigned char* src = reinterpret_cast<const unsigned char*>(&mp);
  for (size_t o = 0; o < sizeof(mp); o += kChunk) {
    Chunk c;
    const size_t n = std::min(kChunk, sizeof(mp) - o);
    std::memcpy(c.b, src + o, n);
    hipLaunchKernelGGL(pf_noalloc_bytes, dim3(1), dim3(256), 0, st, reinterpret_cast<unsigned char*>(mp_dev) + o, c,
                       (uint32_t)n);
  }
  hipLaunchKernelGGL(pf_noalloc_ctl, dim3(1), dim3(64), 0, st, ctl);
  if ((e = hipGetLastError()) != hipSuccess)
    return nfail(PF_E_HIP, "pf_run_noalloc: set-up launch: %s", hipGetErrorString(e));
  // the steps: in place (a tile reads all its particles before it writes
  // any, and no other tile touches them), each reduced by the one-block
  // reduction into record j
  char dummy[sizeof(StepArgs<double, double>)] = {0};
  for (uint32_t j = 0; j < n_steps; ++j) {
    const uint32_t t = t0 + j;
    const uint32_t k = t % S_;
    const StagePlan& sg = plan[k];
    StepArgs<T, S> a;
    std::memset(&a, 0, sizeof(a));
    a.x_in = reinterpret_cast<const S*>(x_dev);
    a.x_out = reinterpret_cast<S*>(x_dev);
    a.lw_in = reinterpret_cast<const T*>(logw_dev);
    a.lw_out = reinterpret_cast<T*>(logw_dev);
    a.y_dev = reinterpret_cast<const T*>(y_dev) + (size_t)j * y_stride;
    a.mp = mp_dev;
    a.part_out = part_dev;
    a.ctl = ctl;
    a.hist = est_dev + j;
    a.hist_cap = 1;
    a.d = (uint32_t)d;
    a.N = N;
    a.k0 = (uint32_t)(cfg->seed & 0xFFFFFFFFu);
    a.k1 = (uint32_t)(cfg->seed >> 32);
    a.sid = cfg->stream_id;
    a.systematic = cfg->resampler == PF_RESAMPLE_SYSTEMATIC ? 1 : 0;
    a.t = t;
    a.k = k;
    a.u = j;
    a.flags = kStepWeight | kStepPropagate;
    a.utau = t + 1u;
    a.radix = sg.r;
    a.log2r = sg.log2r;
    a.log2R = sg.log2R;
    a.lnr = (T)std::log((double)sg.r);
    a.log2C = sg.log2C;
    a.pad = sg.pad;
    a.xrow = sg.xrow;
    a.ntiles = sg.ntiles;
    LaunchReq rq{};
    rq.what = LW_STEP_TILE;
    rq.D = D;
    rq.mk = mk;
    rq.nt = sg.nt;
    rq.ppt = sg.ppt;
    rq.blockpath = sg.blockpath;
    rq.full = d == D ? 1 : 0;
    rq.grid = sg.ntiles;
    rq.lds = sg.lds;
    e = launch_dtype(cfg->state_dtype, rq, &a, st);
    if (e != hipSuccess) return nfail(PF_E_HIP, "pf_run_noalloc: step launch: %s", hipGetErrorString(e));
    LaunchReq rf{};
    rf.what = LW_FINALIZE;
    rf.D = D;
    rf.mk = mk;
    rf.grid = 1;
    rf.fin.ctl = ctl;
    rf.fin.hist = est_dev + j;
    rf.fin.hist_cap = 1;
    rf.fin.t = t;
    rf.fin.k = k;
    rf.fin.radix = sg.r;
    rf.fin.d = (uint32_t)d;
    rf.fin.N = N;
    rf.fin.multi = 0u;
    rf.fin.slot = 0u;
    rf.fin.write_rec = 1u;
    rf.fin.use_step_off = 0u;
    rf.fin.unext = j + 1u;
    rf.fin_part = part_dev;
    rf.fin_ntiles = sg.ntiles;
    e = launch_dtype(cfg->state_dtype, rf, dummy, st);
    if (e != hipSuccess) return nfail(PF_E_HIP, "pf_run_noalloc: reduction launch: %s", hipGetErrorString(e));
  }
  return PF_OK;
}

}  // namespace

extern "C" pf_status pf_run_noalloc(const pf_model* model, const pf_config* cfg, void* x_dev, void* logw_dev,
                                    const void* y_dev, uint32_t n_steps, uint64_t y_stride, uint32_t t0,
                                    pf_estimate_t* est_dev, void* hip_stream) {
  if (!model || !cfg || !x_dev || !logw_dev || (n_steps && (!y_dev || !est_dev)))
    return nfail(PF_E_INVALID, "pf_run_noalloc: NULL argument");
  // the model check writes a message only when it fails
  std::string msg;
  if (validate_model(model, msg) != PF_OK) return nfail(PF_E_INVALID, "pf_run_noalloc: %s", msg.c_str());
  const uint64_t N = cfg->n_particles;
  if (!is_pow2(N) || N < 2 || N > (1ull << 30))
    return nfail(PF_E_INVALID, "pf_run_noalloc: n_particles must be a power of two in [2, 2^30]");
  if (!is_pow2(cfg->radix) || cfg->radix < 2)
    return nfail(PF_E_INVALID, "pf_run_noalloc: radix must be a power of two >= 2");
  if (cfg->radix >= N)
    return nfail(PF_E_UNSUPPORTED, "pf_run_noalloc: the global path (r >= N) needs scratch of N values");
  if (cfg->resampler != PF_RESAMPLE_MULTINOMIAL && cfg->resampler != PF_RESAMPLE_SYSTEMATIC)
    return nfail(PF_E_INVALID, "pf_run_noalloc: unknown resampler");
  if (cfg->state_dtype != PF_DTYPE_F32 && cfg->state_dtype != PF_DTYPE_BF16 && cfg->state_dtype != PF_DTYPE_F64)
    return nfail(PF_E_INVALID, "pf_run_noalloc: unknown state dtype");
  if (cfg->full_cycle || cfg->island || cfg->ess_threshold != 0.0 || cfg->keep_ancestors)
    return nfail(PF_E_UNSUPPORTED, "pf_run_noalloc: plain rotating stages only (no full cycle, island, "
                                   "ESS gating or ancestors)");
  if (y_stride < (uint64_t)model->d) return nfail(PF_E_INVALID, "pf_run_noalloc: y_stride < d");
  if (n_steps == 0) return PF_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  switch (cfg->state_dtype) {
    case PF_DTYPE_F32:
      return run_noalloc<float, float>(model, cfg, x_dev, logw_dev, y_dev, n_steps, y_stride, t0, est_dev, st);
    case PF_DTYPE_BF16:
      return run_noalloc<float, bf16>(model, cfg, x_dev, logw_dev, y_dev, n_steps, y_stride, t0, est_dev, st);
    default:
      return run_noalloc<double, double>(model, cfg, x_dev, logw_dev, y_dev, n_steps, y_stride, t0, est_dev, st);
  }
}
