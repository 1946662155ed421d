// pf_kernels.h - HIP kernels of one particle-filter time step on gfx950.
//
// Butterfly path (radix r < N), one fused kernel per step:
//   phase A  coalesced load of a tile of r x C particles (C contiguous
//            columns per group row, rows at the stage stride R), log-weight
//            l = logW - offset + log g(x, y_t), the pair's block-0 randoms,
//            per-tile estimate partials; states and scalars staged in LDS
//   phase B  per group (a column of the tile): max, exp, inclusive scan,
//            carried weight m_G + ln c_{r-1} - ln r, inverse-CDF draw.
//            r <= 64: one wave segment per group (DPP row operations and
//            cross-lane permutes; up to four 64-lane tasks interleaved);
//            r > 64: runs of consecutive members per thread, scanned in
//            registers, then over lanes, then over waves through LDS; a
//            radix-specialised binary search on a bank-padded column.
//   phase C  gather of the ancestor from LDS, the normals (drawn in phase A
//            already for one pair per thread and 4 to 8 dimensions),
//            propagation, coalesced store of x and the new log-weight.
// The tile partials (estimate record, log-normaliser) are reduced later, a
// few steps at a time (pf_finalize_multi). Block 0 of a step records the
// offset that the step subtracts and clears the slots of a later one. The
// offset subtracted from the stored log-weights at the next load (their
// maximum) is gathered with an order-preserving integer atomicMax.
// Global path (r >= N): weight + tile scan, grid prefix, draw + gather +
// propagate.
#pragma once

#include "pf_device.h"

namespace pfk {

// What a launch of the step kernel does besides resampling: weight with the
// observation (and write the estimate partials), and propagate. A full-cycle
// time step runs every stage: only the first weights, only the last
// propagates.
constexpr uint32_t kStepWeight = 1u;
constexpr uint32_t kStepPropagate = 2u;
// Within-island resampling of the island filter (one stage of radix M and
// stride 1): the launch writes only the ancestor of every particle (into
// `anc`) and each island's carried log-weight (into `isl_lw`); no states, no
// per-particle log-weights.
constexpr uint32_t kStepIsland = 4u;
// Every incoming log-weight is 0: nothing is read (the offset still applies).
constexpr uint32_t kStepLwZero = 8u;
// The incoming log-weights are used as stored: no offset is subtracted (an
// ESS-gated stage after the step's weighting).
constexpr uint32_t kStepLwRaw = 16u;
// The launch does not fold its new log-weights into the next step's offset
// (a later launch of the step writes the final ones).
constexpr uint32_t kStepNoFold = 32u;
// Estimate records whose stage field the step's ESS decisions write.
constexpr uint32_t kStageFromDevice = 0xFFFFFFFFu;

// Geometry of one butterfly stage, for launches that pick their stage on
// the device (ESS-gated stages).
struct AdStage {
  uint32_t log2r, log2R, log2C, pad, xrow, ntiles;
  float lnr;
  uint32_t unused;
};
// Counter word 2 of the island-stage uniforms: island stage s draws word 0
// of the block (island, tau, kIslandBlock + s, stream); particle blocks use
// counter words below 2^16.
constexpr uint32_t kIslandBlock = 1u << 16;
// Uniforms of stage s >= 1 of a full-cycle step come from block 0 of
// counter word tau + s kStageTau (tau = t + 1 < kStageTau).
constexpr uint32_t kStageTau = 1u << 24;

template <typename T, typename S> struct StepArgs {
  const S* x_in;
  S* x_out;
  const T* lw_in;
  T* lw_out;
  uint32_t* anc;            // nullable: global ancestor index per particle
  const T* y_dev;           // nullable: observation (d values) in device memory
  T y_val[kMaxDim];         // observation passed by value when y_dev == nullptr
  const ModelParams<T>* mp;
  T* part_out;              // tile partials of this step
  Ctl* ctl;
  pf_estimate_t* hist;
  uint32_t hist_cap;
  uint32_t d;
  uint64_t N;
  uint32_t log2r, log2R, log2C, pad;  // stage radix, stride, tile columns, LDS row pad
  uint32_t xrow;             // LDS row pitch of the staged states (C, or C + 1)
  uint32_t t, k;
  uint32_t u;                // offset-slot index: steps, or stages of full-cycle steps
  uint32_t flags;            // kStepWeight | kStepPropagate | kStepIsland | kStepLwZero
  uint32_t utau;             // counter word of the resampling uniforms (t + 1, or a stage's)
  uint32_t ntiles;
  uint32_t radix;            // r_k (N on the global path)
  uint32_t k0, k1, sid;
  int32_t systematic;
  int32_t lw_nonzero;        // global path: read logW (else all log-weights are 0)
  T lnr;                     // ln r
  // island filter: carried log-weight per island (within-island launch),
  // source island per destination island and within-island ancestors
  // (island gather launch), log2 of the island size
  T* isl_lw;
  const uint32_t* isl_src;
  const uint32_t* isl_anc;
  uint32_t log2M;
  // ESS-gated stages: per-tile [max, sum w, sum w^2] of the carried weights
  // (nullable) and the stage table
  T* ess_out;
  const AdStage* stab;
  // global path scratch
  T* gcdf;                   // within-tile inclusive CDF (N), for d = 1 paired with the states
  T* gcoarse;                // coarse CDF levels (global_cc_offset)
  S* gx;                     // d > 1: the states particle-major ([N][D]) for the draw's gather
  double* gpre;              // tile prefix, ntiles + 1 entries
  double* gscale;            // e^{m_b - M}, ntiles entries (the draw reads 1 / e^{m_b - M})
  // systematic global draw (nullable otherwise): the first output drawn from
  // each weight tile (ntiles + 1 entries, the last N) and the work items
  // ([0] = count, then (tile, first output) pairs from word 2)
  uint32_t* gfirst;
  uint32_t* gwork;
};

// ---------------------------------------------------------------------------
// Order-preserving encoding of a double as a signed 64-bit integer (for a
// deterministic atomicMax of the new log-weights).
// ---------------------------------------------------------------------------
__host__ __device__ inline long long ord_encode(double v) {
  long long b;
  __builtin_memcpy(&b, &v, 8);
  return b >= 0 ? b : (b ^ 0x7FFFFFFFFFFFFFFFLL);
}
__host__ __device__ inline double ord_decode(long long e) {
  const long long b = e >= 0 ? e : (e ^ 0x7FFFFFFFFFFFFFFFLL);
  double v;
  __builtin_memcpy(&v, &b, 8);
  return v;
}

__device__ __forceinline__ long long* off_slot(Ctl* c, uint32_t step, uint32_t slot) {
  return c->offs + (size_t)(step % kOffRing) * kOffSlots * kOffStride + (size_t)slot * kOffStride;
}
// Max over the slots of `step` (every lane of the calling wave gets it).
__device__ __forceinline__ double read_offset(const Ctl* c, uint32_t step) {
  const uint32_t lane = threadIdx.x & 63u;
  const long long* base = c->offs + (size_t)(step % kOffRing) * kOffSlots * kOffStride;
  long long v = lane < (uint32_t)kOffSlots ? base[(size_t)lane * kOffStride] : LLONG_MIN;
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    const long long o = __shfl_xor(v, s, 64);
    v = o > v ? o : v;
  }
  return ord_decode(v);
}
// Reset the slots of `step` (by threads 0..kOffSlots-1 of a block).
__device__ __forceinline__ void clear_offset(Ctl* c, uint32_t step, double first) {
  if (threadIdx.x < (uint32_t)kOffSlots)
    *off_slot(c, step, threadIdx.x) = ord_encode(threadIdx.x == 0 ? first : -INFINITY);
}

// ---------------------------------------------------------------------------
// Initialisation (Algorithm 1): x_0 = prior(z(tau = 0)), logW = 0, control
// block reset.
// ---------------------------------------------------------------------------
template <int D, int MK, typename T, typename S>
__global__ void __launch_bounds__(256) pf_init_kernel(StepArgs<T, S> a) {
  const uint64_t npair = a.N >> 1;
  const int d = (int)a.d;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npair;
       p += (uint64_t)gridDim.x * blockDim.x) {
    T z0[D], z1[D], x0[D], x1[D];
#pragma unroll
    for (int j = 0; j < D; ++j) z0[j] = z1[j] = 0;
    pair_normals<D, T>((uint32_t)p, 0u, a.sid, a.k0, a.k1, d, z0, z1);
    Model<D, MK, T>::prior(a.mp, z0, x0);
    Model<D, MK, T>::prior(a.mp, z1, x1);
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (j < d) Pair<S, T>::store(a.x_out + (size_t)j * a.N + 2 * p, x0[j], x1[j]);
    a.lw_out[2 * p] = 0;
    a.lw_out[2 * p + 1] = 0;
  }
  if (blockIdx.x == 0) {
    clear_offset(a.ctl, 0u, 0.0);
    clear_offset(a.ctl, 1u, -INFINITY);
    clear_offset(a.ctl, 2u, -INFINITY);
    if (threadIdx.x == 0) {
      a.ctl->log_norm = 0.0;
      a.ctl->t = 0u;
      a.ctl->ad_active = 0u;
      a.ctl->ad_stage = 0u;
      a.ctl->ad_run = 0u;
      a.ctl->ad_next = 0u;
      a.ctl->fail_t = kNoFail;
    }
  }
}

// ---------------------------------------------------------------------------
// Block-wide helpers.
// ---------------------------------------------------------------------------
template <typename T, int NT>
__device__ __forceinline__ T block_max(T v, T* red /* NT/64 */) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  T m = red[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) m = fmaxT(m, red[i]);
  __syncthreads();
  return m;
}

// What the reduction of one step's partials needs.
struct FinArgs {
  Ctl* ctl;
  pf_estimate_t* hist;
  uint32_t hist_cap, t, k, radix, d;
  uint64_t N;
  // deferred reductions: the increment goes to ctl->dlog[slot] and the
  // running log-normaliser is added by a later pass; write_rec = 0 skips the
  // record (a later step owns its history slot); the next offset comes from
  // the following step's bookkeeping (use_step_off) or from the slots
  uint32_t multi, slot, write_rec, use_step_off;
  uint32_t unext;  // offset-slot index of the next step (its offset is this step's next offset)
};

// FP64 reduction of one step's tile partials by one block, in a fixed order.
// Partial record of tile b: [m, S, sw2, swin, A1[D], A2[D], sh[D]] with m the
// tile max of l, w = e^{l - m}, S = sum w, sw2 = sum w^2, swin = sum e^{logW},
// A1 = sum w (x - sh), A2 = sum w (x - sh)^2, sh a tile reference point.
// Thread i takes tiles i, i + NT, ... in rounds of FB tiles whose loads are
// all issued before any is used (one memory round trip per round: the
// stand-alone kernel uses large rounds, the head block of a step kernel
// single tiles so that it needs no more registers than the tiles); sums are
// kept relative to the thread's running max and rescaled when it grows.
// Waves reduce with DPP in a fixed pattern; wave 0 combines the waves in wave
// order, one value per lane. Writes the estimate record of step f.t and adds
// its log-normaliser increment. `red` needs (NT/64) * (4 + 2D) doubles.
template <int D, typename T> constexpr int fin_batch() {
  constexpr int dw = (int)(partial_stride(D) * sizeof(T) / 4);  // registers per record
  constexpr int b = 64 / dw;
  return b < 1 ? 1 : (b > 8 ? 8 : b);
}

// 1 if v is NaN or infinite (minus infinity allowed with neg_inf_ok). The
// kernels are built assuming no NaN operands, so the test looks at the bits
// through an opaque register move that the optimiser cannot see through.
__device__ __forceinline__ uint32_t nonfinite_bits(float v, bool neg_inf_ok) {
  uint32_t w = __float_as_uint(v);
  asm volatile("" : "+v"(w));
  return ((w & 0x7F800000u) == 0x7F800000u && !(neg_inf_ok && w == 0xFF800000u)) ? 1u : 0u;
}
__device__ __forceinline__ uint32_t nonfinite_bits(double v, bool neg_inf_ok) {
  uint64_t w = (uint64_t)__double_as_longlong(v);
  asm volatile("" : "+v"(w));
  return ((w & 0x7FF0000000000000ull) == 0x7FF0000000000000ull && !(neg_inf_ok && w == 0xFFF0000000000000ull))
             ? 1u
             : 0u;
}

template <int D, typename T, int NT, int FB>
__device__ void finalize_partials(const FinArgs& f, const T* __restrict__ part, uint32_t ntiles,
                                  double* red) {
  __shared__ uint32_t s_bad[NT / 64];
  constexpr int PS = partial_stride(D);
  constexpr int NR = 4 + 2 * D;  // per wave: [M_w, swin, S, sw2, Mx[D], Mxx[D]]
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int d = (int)f.d;
  // wave 0 fetches the next step's offset slots and the running normaliser
  // up front: they are only needed at the end
  double offv = -INFINITY, ln0 = 0.0;
  if (wv == 0) {
    if (f.use_step_off) {
      if (lane == 0) offv = f.ctl->step_off[f.unext % kMaxPending];
    } else if (lane < kOffSlots) {
      offv = ord_decode(*off_slot(f.ctl, f.unext, lane));
    }
    if (lane == 0 && !f.multi) ln0 = f.ctl->log_norm;
  }
  double mt = -INFINITY, swin = 0.0, s = 0.0, sw2 = 0.0, a1[D], a2[D];
  uint32_t bad = 0u;
#pragma unroll
  for (int j = 0; j < D; ++j) a1[j] = a2[j] = 0.0;
  for (uint32_t b0 = tid; b0 < ntiles; b0 += NT * FB) {
    T rec[FB][PS];
#pragma unroll
    for (int q = 0; q < FB; ++q) {
      const uint32_t b = b0 + (uint32_t)q * NT;
      const T* pr = part + (size_t)(b < ntiles ? b : 0) * PS;
#pragma unroll
      for (int v = 0; v < PS; ++v) rec[q][v] = pr[v];
    }
    // a tile max may be -inf (no positive weight in the tile); every other
    // value must be finite
#pragma unroll
    for (int q = 0; q < FB; ++q)
      if (b0 + (uint32_t)q * NT < ntiles) {
        bad |= nonfinite_bits(rec[q][0], true);
#pragma unroll
        for (int v = 1; v < 4 + 2 * D; ++v)
          if (v < 4 || (v - 4) % D < d) bad |= nonfinite_bits(rec[q][v], false);
      }
    double mr = mt;
#pragma unroll
    for (int q = 0; q < FB; ++q)
      if (b0 + (uint32_t)q * NT < ntiles) mr = fmax(mr, (double)rec[q][0]);
    if (mr > mt) {
      const double sc = mt == -INFINITY ? 0.0 : exp(mt - mr);
      s *= sc;
      sw2 *= sc * sc;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        a1[j] *= sc;
        a2[j] *= sc;
      }
      mt = mr;
    }
#pragma unroll
    for (int q = 0; q < FB; ++q) {
      if (b0 + (uint32_t)q * NT >= ntiles) continue;
      const double mb = (double)rec[q][0];
      const double e = mb == -INFINITY ? 0.0 : exp(mb - mt);
      const double Sb = (double)rec[q][1];
      s += e * Sb;
      sw2 += e * e * (double)rec[q][2];
      swin += (double)rec[q][3];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        if (j < d) {
          const double c1 = (double)rec[q][4 + j], c2 = (double)rec[q][4 + D + j];
          const double sh = (double)rec[q][4 + 2 * D + j];
          a1[j] += e * (c1 + Sb * sh);
          a2[j] += e * (c2 + 2.0 * sh * c1 + Sb * sh * sh);
        }
      }
    }
  }
  {
    const uint32_t wave_bad = __ballot(bad != 0u) != 0ull ? 1u : 0u;
    if (lane == 0) s_bad[wv] = wave_bad;  // (published by the barrier below)
  }
  // wave level: common max, then fixed-pattern sums
  const double Mw = wave_max(mt);
  {
    const double sc = (mt == -INFINITY) ? 0.0 : exp(mt - Mw);
    s = wave_sum(s * sc);
    sw2 = wave_sum(sw2 * (sc * sc));
    swin = wave_sum(swin);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if (j < d) {
        a1[j] = wave_sum(a1[j] * sc);
        a2[j] = wave_sum(a2[j] * sc);
      }
    }
  }
  if (lane == 0) {
    double* rw = red + wv * NR;
    rw[0] = Mw;
    rw[1] = swin;
    rw[2] = s;
    rw[3] = sw2;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      rw[4 + j] = a1[j];
      rw[4 + D + j] = a2[j];
    }
  }
  __syncthreads();
  if (wv != 0) return;
  // wave 0: lane v combines value v over the waves, in wave order
  double M = red[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) M = fmax(M, red[w * NR]);
  double tv = 0.0;
  if (lane >= 1 && lane < NR) {
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const double mw = red[w * NR];
      const double fw = (lane == 1) ? 1.0 : (mw == -INFINITY ? 0.0 : exp(mw - M));
      tv += (lane == 3 ? fw * fw : fw) * red[w * NR + lane];
    }
  }
  const double swin_t = readlane_d(tv, 1), S = readlane_d(tv, 2), sw2_t = readlane_d(tv, 3);
  const int jl = lane < D ? lane : D - 1;
  const double mx = __shfl(tv, 4 + jl, 64), mxx = __shfl(tv, 4 + D + jl, 64);
  const double nx = wave_max(offv);
  pf_estimate_t* rec = f.hist + (f.t % f.hist_cap);
  if (f.write_rec && lane < kMaxDim) {
    double mean = 0.0, var = 0.0;
    if (lane < D && lane < d) {
      mean = mx / S;
      var = fmax(mxx / S - mean * mean, 0.0);
    }
    rec->mean[lane] = mean;
    rec->var[lane] = var;
  }
  if (lane == 0) {
    // a usable step: finite partial sums, some positive weight now and
    // before, no earlier failure (sticky until re-initialised)
    uint32_t any_bad = 0u;
#pragma unroll
    for (int w = 0; w < NW; ++w) any_bad |= s_bad[w];
    const bool own = any_bad == 0u && S > 0.0 && swin_t > 0.0;
    if (!own) atomicMin(&f.ctl->fail_t, f.t);
    // steps reduced one at a time see an earlier failure here; deferred
    // steps reduced together are fixed up in step order by the prefix pass
    const bool ok = own && f.t < f.ctl->fail_t;
    const double dlog = ok ? (M + log(S)) - log(swin_t) : 0.0;
    const double ln = ln0 + dlog;
    if (f.write_rec) {
      rec->t = f.t;
      if (f.k != kStageFromDevice) rec->stage = f.k;
      rec->radix = f.radix;
      rec->valid = ok ? 1u : 0u;
      rec->log_normaliser = f.multi ? 0.0 : ln;
      rec->ess = S * S / ((double)f.N * sw2_t);
      rec->max_log_weight = M;
      rec->next_offset = nx;
    }
    if (f.multi) {
      f.ctl->dlog[f.slot] = dlog;
    } else {
      f.ctl->log_norm = ln;
      f.ctl->t = f.t + 1;
    }
  }
}

// Stand-alone reduction of the last step's partials (one block).
template <int D, typename T, int NT>
__global__ void __launch_bounds__(NT) pf_finalize_kernel(FinArgs f, const T* part, uint32_t ntiles) {
  __shared__ double red[(NT / 64) * (4 + 2 * D)];
  finalize_partials<D, T, NT, fin_batch<D, T>()>(f, part, ntiles, red);
}

// Several deferred steps at once: block i reduces step fm.steps[i] (its
// partials in ring slot t mod fm.ring); a second launch adds the running
// log-normaliser in step order.
struct FinStep {
  uint32_t t, k, radix, ntiles, unext;
};
struct FinMulti {
  Ctl* ctl;
  pf_estimate_t* hist;
  const void* part_base;
  uint64_t part_stride;  // elements per ring slot
  uint64_t N;
  uint32_t hist_cap, d, n, ring;
  FinStep steps[kMaxPending];
};

template <int D, typename T, int NT>
__global__ void __launch_bounds__(NT) pf_finalize_multi(FinMulti fm) {
  __shared__ double red[(NT / 64) * (4 + 2 * D)];
  const uint32_t i = blockIdx.x;
  const FinStep st = fm.steps[i];
  FinArgs f;
  f.ctl = fm.ctl;
  f.hist = fm.hist;
  f.hist_cap = fm.hist_cap;
  f.t = st.t;
  f.k = st.k;
  f.radix = st.radix;
  f.d = fm.d;
  f.N = fm.N;
  f.multi = 1u;
  f.slot = i;
  f.write_rec = (fm.n - 1u - i) < fm.hist_cap ? 1u : 0u;
  f.use_step_off = (i + 1u < fm.n) ? 1u : 0u;
  f.unext = st.unext;
  const T* part = reinterpret_cast<const T*>(fm.part_base) + (size_t)(st.t % fm.ring) * fm.part_stride;
  finalize_partials<D, T, NT, fin_batch<D, T>()>(f, part, st.ntiles, red);
}

template <typename T>
__global__ void __launch_bounds__(64) pf_finalize_prefix(FinMulti fm) {
  if (threadIdx.x != 0) return;
  double ln = fm.ctl->log_norm;
  const uint32_t fail_t = fm.ctl->fail_t;
  for (uint32_t i = 0; i < fm.n; ++i) {
    const bool ok = fm.steps[i].t < fail_t;
    if (ok) ln += fm.ctl->dlog[i];
    if (fm.n - 1u - i < fm.hist_cap) {
      pf_estimate_t* r = fm.hist + fm.steps[i].t % fm.hist_cap;
      r->log_normaliser = ln;
      if (!ok) r->valid = 0u;
    }
  }
  fm.ctl->log_norm = ln;
  fm.ctl->t = fm.steps[fm.n - 1u].t + 1u;
}

// Per-step bookkeeping by block 0 of a step: record the offset this step
// subtracts (the previous step's next offset, for deferred reductions) and
// clear the offset slots that the next step will gather into.
template <typename T, typename S>
__device__ __forceinline__ void step_bookkeeping(const StepArgs<T, S>& a) {
  if (threadIdx.x < 64u) {
    const double o = read_offset(a.ctl, a.u);
    if (threadIdx.x == 0) a.ctl->step_off[a.u % kMaxPending] = o;
  }
  clear_offset(a.ctl, a.u + 2, -INFINITY);
}

// Partial sums of one tile from per-thread register values (relative to the
// tile max `mtile` and the tile reference point `sh`). Thread v < PS of the
// block writes slot v. `red` needs (NT/64) * PS values of T.
// Wave sums of NV per-lane FP32 values by recursive halving: at each lane
// distance (32, 16, then DPP mirror pairs 8, 4 and quad swaps 2, 1) every
// lane keeps one half of its list (the upper half where the distance bit is
// set) and adds its partner's copy of that half; once one value is left the
// remaining distances are plain pair sums. Lane l ends with the wave total
// of value idx(l) (the sum of the kept upper-half offsets); lanes that differ
// only in the bits of `group` hold the same total. Fixed order.
template <int N, int DIST, int NV>
__device__ __forceinline__ void rh_step_shfl(float (&v)[NV], uint32_t lane, uint32_t& idx, uint32_t& group) {
  const bool hi = (lane & DIST) != 0u;
  if constexpr (N == 1) {
    v[0] += __shfl_xor(v[0], DIST, 64);
    group |= DIST;
  } else {
    constexpr int H = (N + 1) / 2;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const float a = v[i];
      const float b = (i + H < N) ? v[i + H] : 0.f;
      const float recv = __shfl_xor(hi ? a : b, DIST, 64);
      v[i] = (hi ? b : a) + recv;
    }
    if (hi) idx += H;
  }
}
template <int N, int DIST, int CTRL, int NV>
__device__ __forceinline__ void rh_step_dpp(float (&v)[NV], uint32_t lane, uint32_t& idx, uint32_t& group) {
  const bool hi = (lane & DIST) != 0u;
  if constexpr (N == 1) {
    v[0] += dppm<CTRL>(v[0]);
    group |= DIST;
  } else {
    constexpr int H = (N + 1) / 2;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const float a = v[i];
      const float sa = a + dppm<CTRL>(a);
      float sb = 0.f;
      if (i + H < N) sb = v[i + H] + dppm<CTRL>(v[i + H]);
      v[i] = hi ? sb : sa;
    }
    if (hi) idx += H;
  }
}
template <int NV>
__device__ __forceinline__ float wave_sums_rh(float (&v)[NV], uint32_t lane, uint32_t& idx, uint32_t& group) {
  constexpr int n1 = (NV + 1) / 2, n2 = (n1 + 1) / 2, n3 = (n2 + 1) / 2, n4 = (n3 + 1) / 2, n5 = (n4 + 1) / 2;
  static_assert(n5 <= 2, "at most 64 values");
  idx = 0u;
  group = 0u;
  rh_step_shfl<NV, 32>(v, lane, idx, group);
  rh_step_shfl<n1, 16>(v, lane, idx, group);
  rh_step_dpp<n2, 8, kDppRowMirror>(v, lane, idx, group);
  rh_step_dpp<n3, 4, kDppRowHalfMirror>(v, lane, idx, group);
  rh_step_dpp<n4, 2, kDppQuadXor2>(v, lane, idx, group);
  rh_step_dpp<n5, 1, kDppQuadXor1>(v, lane, idx, group);
  return v[0];
}

template <int D, typename T, int NT, int NLOC>
__device__ __forceinline__ void tile_partials(const T (&l)[NLOC], const T (&x)[NLOC][D],
                                              const T (&lwn)[NLOC], const T (&sh)[D], int d,
                                              T mtile, T* red, T* out /* PS values */) {
  constexpr int PS = partial_stride(D);
  T s = 0, sw2 = 0, swin = 0, a1[D], a2[D];
#pragma unroll
  for (int j = 0; j < D; ++j) a1[j] = a2[j] = 0;
#pragma unroll
  for (int e = 0; e < NLOC; ++e) {
    const T w = fexp(l[e] - mtile);
    s += w;
    sw2 += w * w;
    swin += fexp(lwn[e]);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const T dx = x[e][j] - sh[j];
      const T wd = w * dx;
      a1[j] += wd;
      a2[j] += wd * dx;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if constexpr (sizeof(T) == 4) {
    // record values 1 .. 3 + 2D in one recursive-halving reduction
    constexpr int NV = 3 + 2 * D;
    float v[NV];
    v[0] = s;
    v[1] = sw2;
    v[2] = swin;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      v[3 + j] = a1[j];
      v[3 + D + j] = a2[j];
    }
    uint32_t idx, group;
    const float tot = wave_sums_rh<NV>(v, (uint32_t)lane, idx, group);
    if (((uint32_t)lane & group) == 0u && idx < (uint32_t)NV) red[wv * PS + 1 + idx] = tot;
  } else {
    s = wave_sum(s);
    sw2 = wave_sum(sw2);
    swin = wave_sum(swin);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if (j < d) {
        a1[j] = wave_sum(a1[j]);
        a2[j] = wave_sum(a2[j]);
      }
    }
    if (lane == 0) {
      T* rw = red + wv * PS;
      rw[1] = s;
      rw[2] = sw2;
      rw[3] = swin;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        rw[4 + j] = a1[j];
        rw[4 + D + j] = a2[j];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < PS) {
    const int v = threadIdx.x;
    T acc = 0;
    if (v == 0) {
      acc = mtile;
    } else if (v < 4 + 2 * D) {
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) acc += red[w * PS + v];
    } else {
      acc = sh[v - 4 - 2 * D < D ? v - 4 - 2 * D : 0];
    }
    out[v] = acc;
  }
}

// ---------------------------------------------------------------------------
// Tile coordinates. A tile holds E = r C particles: column c of row q.
// wide (R >= C): rows are C contiguous particles at stride R.
// narrow (R < C): the tile is one contiguous run of E particles.
// ---------------------------------------------------------------------------
struct TileGeo {
  uint32_t log2r, log2R, log2C;
  bool wide;
  uint64_t base;
  // launch-uniform helpers of pair_coords
  uint32_t sq, sh2, mlo, rmask;
  bool r1;  // rows of one particle (narrow with R = 1, or wide with C = 1):
            // a pair's second particle is in the next row
};

__device__ __forceinline__ TileGeo tile_geo(uint32_t tile, uint32_t log2r, uint32_t log2R,
                                            uint32_t log2C) {
  TileGeo g;
  g.log2r = log2r;
  g.log2R = log2R;
  g.log2C = log2C;
  g.wide = log2R >= log2C;
  if (g.wide) {
    const uint32_t sh = log2R - log2C;
    const uint64_t hi = tile >> sh;
    const uint64_t lo0 = (uint64_t)(tile & ((1u << sh) - 1u)) << log2C;
    g.base = (hi << (log2r + log2R)) + lo0;
  } else {
    g.base = (uint64_t)tile << (log2r + log2C);
  }
  g.sq = g.wide ? log2C : log2R;
  g.sh2 = g.sq + log2r;
  g.mlo = (1u << (g.wide ? log2C : log2R)) - 1u;
  g.rmask = (1u << log2r) - 1u;
  g.r1 = g.wide ? log2C == 0u : log2R == 0u;
  return g;
}

// Row q, column c and global index of the particles at even tile position f
// and f + 1 (one branch-free formula for wide and narrow tiles: for a wide
// tile f >> sh2 is 0; the pair's global indices are gi and gi + 1).
__device__ __forceinline__ void pair_coords(const TileGeo& g, uint32_t f, uint32_t& q0, uint32_t& c0,
                                            uint32_t& q1, uint32_t& c1, uint64_t& gi) {
  q0 = (f >> g.sq) & g.rmask;
  c0 = ((f >> g.sh2) << g.log2R) | (f & g.mlo);
  gi = g.base + (g.wide ? ((uint64_t)q0 << g.log2R) + c0 : (uint64_t)f);
  q1 = g.r1 ? q0 + 1u : q0;
  c1 = g.r1 ? c0 : c0 + 1u;
}

// Tile index of block b. Blocks are dealt
// round-robin to the 8 XCDs; each XCD gets a contiguous range of tiles, so
// neighbouring column chunks share the XCD's L2.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t ntiles) {
  // the first 8 floor(ntiles / 8) blocks are remapped; a tail of fewer than
  // 8 keeps its order
  const uint32_t q = ntiles >> 3;
  if (b >= 8u * q) return b;
  return (b & 7u) * q + (b >> 3);
}

// Bump allocator over the dynamic LDS block: offsets are plain integers so
// every carved pointer stays an LDS (address space 3) pointer.
struct LdsCarve {
  size_t off = 0;
  __device__ __forceinline__ size_t take(size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 15) & ~(size_t)15;
    return o;
  }
};

// LDS bytes of a tile kernel (must match the carve in pf_step_tile).
__host__ __device__ inline size_t tile_lds_bytes(int d, int D, size_t tsz, uint32_t r, uint32_t C,
                                                 uint32_t pad, int NT, bool blockpath, uint32_t xrow) {
  const size_t P = r + pad;
  const size_t PS = 4 + 3 * (size_t)D;
  size_t b = 0;
  auto add = [&](size_t n) { b = (b + n + 15) & ~(size_t)15; };
  add((size_t)d * r * xrow * tsz);                // xs (d = 0: none, the within-island launch)
  add(C * P * tsz);                               // l / cdf
  add(C * P * tsz);                               // uniforms, then ancestor positions
  const size_t red = (size_t)(NT / 64) * PS * tsz;
  add(red > C * tsz ? red : C * tsz);             // reduction scratch / carried weight
  add((size_t)(D > NT / 64 ? D : NT / 64) * tsz);  // tile reference point / wave maxima
  if (blockpath) {
    add((size_t)(NT / 64) * tsz);  // wave maxima
    add((size_t)(NT / 64) * tsz);  // wave sums
  }
  return b;
}

// ---------------------------------------------------------------------------
// Segmented wave operations for groups of r = 2^lr <= 64 lanes (FP32: DPP
// row operations; FP64: cross-lane shuffles).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float seg_max(float v, uint32_t lr, uint32_t lane) {
  v = fmaxf(v, dpp_f<kDppQuadXor1>(v));
  if (lr >= 2) v = fmaxf(v, dpp_f<kDppQuadXor2>(v));
  if (lr >= 3) v = fmaxf(v, dpp_f<kDppRowHalfMirror>(v));
  if (lr >= 4) v = fmaxf(v, dpp_f<kDppRowMirror>(v));
  if (lr >= 5) {
    float b = dpp_f<kDppRowBcast15, 0xA>(v);
    if (((lane >> 4) & 1u) == 0u) b = v;
    v = fmaxf(v, b);
    if (lr >= 6) {
      float c = dpp_f<kDppRowBcast31, 0xC>(v);
      if ((lane >> 5) == 0u) c = v;
      v = fmaxf(v, c);
    }
    v = __shfl(v, (int)(lane | ((1u << lr) - 1u)), 64);  // the segment's last lane
  }
  return v;
}
__device__ __forceinline__ float seg_scan(float v, uint32_t lr, uint32_t q) {
  float o = dpp_f<0x111>(v);  // row_shr:1
  if (q >= 1u) v += o;
  if (lr >= 2) {
    o = dpp_f<0x112>(v);      // row_shr:2
    if (q >= 2u) v += o;
  }
  if (lr >= 3) {
    o = dpp_f<0x114>(v);      // row_shr:4
    if (q >= 4u) v += o;
  }
  if (lr >= 4) {
    o = dpp_f<0x118>(v);      // row_shr:8
    if (q >= 8u) v += o;
  }
  if (lr >= 5) {
    o = dpp_f<kDppRowBcast15, 0xA>(v);
    if ((q >> 4) & 1u) v += o;
  }
  if (lr >= 6) {
    o = dpp_f<kDppRowBcast31, 0xC>(v);
    if (q >= 32u) v += o;
  }
  return v;
}
__device__ __forceinline__ double seg_max(double v, uint32_t lr, uint32_t lane) {
  for (uint32_t s = 1; s < (1u << lr); s <<= 1) v = fmax(v, __shfl_xor(v, (int)s, 64));
  return v;
}
__device__ __forceinline__ double seg_scan(double v, uint32_t lr, uint32_t q) {
  for (uint32_t s = 1; s < (1u << lr); s <<= 1) {
    const double o = __shfl_up(v, s, 64);
    if (q >= s) v += o;
  }
  return v;
}

// ---------------------------------------------------------------------------
// Groups of r = 2^LR lanes with LR known at compile time (the wave path).
// FP32: DPP lane moves that the compiler fuses into the max / add; the
// value of a group's first or last lane is read with readlane when a group
// is half of the wave or all of it, else with a bpermute.
// ---------------------------------------------------------------------------
template <int CTRL, int RM, bool BC>
__device__ __forceinline__ float dppx(float old, float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                __builtin_bit_cast(int, v), CTRL, RM, 0xF, BC));
}
__device__ __forceinline__ float rdlane(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
// Value of lane l (wave-uniform l).
__device__ __forceinline__ float lane_at(float v, uint32_t l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), (int)l));
}
__device__ __forceinline__ double lane_at(double v, uint32_t l) { return readlane_d(v, (int)l); }
__device__ __forceinline__ float bperm(uint32_t byte_addr, float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute((int)byte_addr, __builtin_bit_cast(int, v)));
}

template <int LR, typename T> struct Grp;

template <int LR> struct Grp<LR, float> {
  static constexpr uint32_t r = 1u << LR;
  // max over the group, in every lane of the group
  static __device__ __forceinline__ float max(float v, uint32_t lane) {
    if constexpr (LR >= 1) v = fmaxf(v, dppm<kDppQuadXor1>(v));
    if constexpr (LR >= 2) v = fmaxf(v, dppm<kDppQuadXor2>(v));
    if constexpr (LR >= 3) v = fmaxf(v, dppm<kDppRowHalfMirror>(v));
    if constexpr (LR >= 4) v = fmaxf(v, dppm<kDppRowMirror>(v));
    // rows not written by a broadcast keep their own value (max(v, v) = v)
    if constexpr (LR >= 5) v = fmaxf(v, dppx<kDppRowBcast15, 0xA, false>(v, v));
    if constexpr (LR >= 6) v = fmaxf(v, dppx<kDppRowBcast31, 0xC, false>(v, v));
    if constexpr (LR == 5) {
      const float a = rdlane(v, 31), b = rdlane(v, 63);
      v = lane < 32u ? a : b;
    }
    if constexpr (LR == 6) v = rdlane(v, 63);
    return v;
  }
  // inclusive prefix sum over the group (q = position in the group)
  static __device__ __forceinline__ float scan(float v, uint32_t q) {
    if constexpr (LR <= 3) {
      // groups inside a row: row shifts and a position test
      float o = dppx<0x111, 0xF, false>(0.f, v);
      if (q >= 1u) v += o;
      if constexpr (LR >= 2) {
        o = dppx<0x112, 0xF, false>(0.f, v);
        if (q >= 2u) v += o;
      }
      if constexpr (LR >= 3) {
        o = dppx<0x114, 0xF, false>(0.f, v);
        if (q >= 4u) v += o;
      }
    } else {
      // groups of whole rows: lanes shifted in from outside the row read 0
      v += dppx<0x111, 0xF, true>(0.f, v);
      v += dppx<0x112, 0xF, true>(0.f, v);
      v += dppx<0x114, 0xF, true>(0.f, v);
      v += dppx<0x118, 0xF, true>(0.f, v);
      if constexpr (LR >= 5) v += dppx<kDppRowBcast15, 0xA, false>(0.f, v);
      if constexpr (LR >= 6) v += dppx<kDppRowBcast31, 0xC, false>(0.f, v);
    }
    return v;
  }
  static __device__ __forceinline__ float last(float v, uint32_t lane, uint32_t seg) {
    if constexpr (LR == 6) return rdlane(v, 63);
    if constexpr (LR == 5) {
      const float a = rdlane(v, 31), b = rdlane(v, 63);
      return lane < 32u ? a : b;
    }
    return bperm((seg + r - 1u) << 2, v);
  }
  static __device__ __forceinline__ float first(float v, uint32_t lane, uint32_t seg) {
    if constexpr (LR == 6) return rdlane(v, 0);
    if constexpr (LR == 5) {
      const float a = rdlane(v, 0), b = rdlane(v, 32);
      return lane < 32u ? a : b;
    }
    return bperm(seg << 2, v);
  }
  // first position p of the group with cdf_p > target, clamped to r - 1
  static __device__ __forceinline__ uint32_t search(float cdf, float target, uint32_t seg) {
    uint32_t pb = seg << 2;  // byte address of the candidate's lane
#pragma unroll
    for (uint32_t s = r >> 1; s >= 1u; s >>= 1) {
      const float v = bperm(pb + ((s - 1u) << 2), cdf);
      if (v <= target) pb += s << 2;
    }
    return (pb >> 2) - seg;
  }
};

template <int LR> struct Grp<LR, double> {
  static constexpr uint32_t r = 1u << LR;
  static __device__ __forceinline__ double max(double v, uint32_t lane) { return seg_max(v, LR, lane); }
  static __device__ __forceinline__ double scan(double v, uint32_t q) { return seg_scan(v, LR, q); }
  static __device__ __forceinline__ double last(double v, uint32_t, uint32_t seg) {
    return __shfl(v, (int)(seg + r - 1u), 64);
  }
  static __device__ __forceinline__ double first(double v, uint32_t, uint32_t seg) {
    return __shfl(v, (int)seg, 64);
  }
  static __device__ __forceinline__ uint32_t search(double cdf, double target, uint32_t seg) {
    uint32_t pos = 0;
#pragma unroll
    for (uint32_t s = r >> 1; s >= 1u; s >>= 1) {
      const double v = __shfl(cdf, (int)(seg + pos + s - 1u), 64);
      if (v <= target) pos += s;
    }
    return pos;
  }
};

// Phase B of the wave path for r = 2^LR <= 64: a group is a segment of r
// lanes; each wave handles 2 PPT tasks of 64 lanes, U of them interleaved.
// Per group: max, scan of e^{l - max}, carried weight, the draw by binary
// search of the scanned weights; positions overwrite the uniforms in LDS.
template <int LR, typename T, int NT, int PPT>
__device__ __forceinline__ void wave_groups(const T* scl, const T* scu, int* sca, T* colw, uint32_t P, T lnr,
                                            bool sys, int wv, uint32_t lane, T& tile_lwmax) {
  using G = Grp<LR, T>;
  constexpr uint32_t r = 1u << LR;
  constexpr int U = (2 * PPT) < 4 ? (2 * PPT) : 4;
  const uint32_t seg = lane & ~(r - 1u);
  const uint32_t q = lane & (r - 1u);
#pragma unroll
  for (int it = 0; it < (2 * PPT) / U; ++it) {
    uint32_t c[U];
    T l[U], m[U], cdf[U], tot[U], target[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t task = wv + (U * it + u) * (NT / 64);
      c[u] = (task << (6 - LR)) + (lane >> LR);
      l[u] = scl[c[u] * P + q];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) m[u] = G::max(l[u], lane);
#pragma unroll
    for (int u = 0; u < U; ++u) cdf[u] = G::scan(fexp(l[u] - m[u]), q);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      tot[u] = G::last(cdf[u], lane, seg);
      const T uu = scu[c[u] * P + q];
      target[u] = sys ? ((T)q + G::first(uu, lane, seg)) * tot[u] / (T)r : uu * tot[u];
    }
    uint32_t pos[U];
#pragma unroll
    for (int u = 0; u < U; ++u) pos[u] = G::search(cdf[u], target[u], seg);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      sca[c[u] * P + q] = (int)pos[u];
      const T lw = m[u] + flog_ge1(tot[u]) - lnr;
      tile_lwmax = fmaxT(tile_lwmax, lw);
      if (q == 0) colw[c[u]] = lw;
    }
  }
}

// ---------------------------------------------------------------------------
// Fused butterfly step (radix r < N) on one tile of r x C particles: the
// body shared by the single-filter kernel and the batched kernel.
// ---------------------------------------------------------------------------
// FULL: the model dimension equals the compiled one (d = D), so every test
// of a component index against d folds away.
// Draw of the r > 64 path: the number of members of a group of r = 2^LR
// whose cumulative weight is <= target, at most r - 1 (binary search).
// `col` holds member q at word q + q / 64. The search keeps the padded word
// pp of its lower bound pos: pos is a multiple of 2s at the step of width s,
// so the probed member pos + s - 1 sits at pp + s - 1 + (s - 1) / 64 and
// pos + s at pp + s + s / 64 (constants once the loop is unrolled); at the
// end pos = pp - pp / 65.
template <int LR, typename T>
__device__ __forceinline__ uint32_t padded_search(const T* col, T target) {
  uint32_t pp = 0;
#pragma unroll
  for (int k = LR - 1; k >= 0; --k) {
    const uint32_t s = 1u << k;
    if (col[pp + (s - 1u) + ((s - 1u) >> 6)] <= target) pp += s + (s >> 6);
  }
  return pp - pp / 65u;
}

// The draws of K consecutive members q0 .. q0 + K - 1 of a group of
// r = 2^LR (cumulative weights in `col`, total `tot`): multinomial targets
// u_q tot, systematic (q + U_0) tot / r; positions overwrite the uniforms
// `us` word for word.
template <int LR, int K, typename T>
__device__ __forceinline__ void draw_run(const T* col, const T* us, int* pos, uint32_t q0, T tot, T u0,
                                         bool sys) {
  const T inv_r = (T)1 / (T)(1u << LR);  // exact: r is a power of two
  T uu[K];
#pragma unroll
  for (int k = 0; k < K; ++k) uu[k] = us[k];
  uint32_t pk[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const T target = sys ? ((T)(q0 + (uint32_t)k) + u0) * tot * inv_r : uu[k] * tot;
    pk[k] = padded_search<LR>(col, target);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) pos[k] = (int)pk[k];
}

// ISL: compiled for the within-island launch only (kStepIsland set, no
// propagation), which keeps the registers of phase C out of the large tiles.
template <int D, int MK, typename T, typename S, int NT, int PPT, bool BLOCKPATH, bool FULL, bool ISL = false>
__device__ __forceinline__ void step_tile_body(const StepArgs<T, S>& a, const uint32_t tile,
                                               unsigned char* smem) {
  constexpr int NLOC = 2 * PPT;
  constexpr int PS = partial_stride(D);
  const int d = FULL ? D : (int)a.d;
  const uint32_t log2r = a.log2r, log2C = a.log2C;
  const uint32_t r = 1u << log2r, C = 1u << log2C;
  const uint32_t P = r + a.pad;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // word of group member q in its column of scl/scu/sca: for r > 64 one word
  // is skipped after every 64 members (the pad holds them), so the lanes of
  // one binary-search step, a multiple of 64 members apart, hit distinct banks
  auto lix = [](uint32_t q) { return BLOCKPATH ? q + (q >> 6) : q; };

  // LDS carve (tile_lds_bytes)
  LdsCarve lc;
  const uint32_t xrow = a.xrow;
  const size_t xplane = (size_t)r * xrow;
  const bool island = ISL || (a.flags & kStepIsland) != 0u;
  T* xs = reinterpret_cast<T*>(smem + lc.take(island ? 0 : (size_t)d * xplane * sizeof(T)));
  T* scl = reinterpret_cast<T*>(smem + lc.take((size_t)C * P * sizeof(T)));
  T* scu = reinterpret_cast<T*>(smem + lc.take((size_t)C * P * sizeof(T)));
  int* sca = reinterpret_cast<int*>(scu);  // positions overwrite the uniforms
  const size_t red_bytes = (size_t)(NT / 64) * PS * sizeof(T);
  T* red = reinterpret_cast<T*>(smem + lc.take(red_bytes > C * sizeof(T) ? red_bytes : C * sizeof(T)));
  T* colw = red;  // carried weights live where the reduction scratch was
  T* shx = reinterpret_cast<T*>(smem + lc.take((size_t)(D > NT / 64 ? D : NT / 64) * sizeof(T)));
  T* chm = reinterpret_cast<T*>(smem + lc.take((size_t)(NT / 64) * sizeof(T)));  // wave maxima
  T* chs = reinterpret_cast<T*>(smem + lc.take((size_t)(NT / 64) * sizeof(T)));  // wave sums

  const TileGeo geo = tile_geo(tile, log2r, a.log2R, log2C);
  const uint64_t N = a.N;
  const T off = (a.flags & kStepLwRaw) != 0u ? (T)0 : (T)read_offset(a.ctl, a.u);
  const bool weight = (a.flags & kStepWeight) != 0u;
  const bool prop = !ISL && (a.flags & kStepPropagate) != 0u;
  const bool lwz = (a.flags & kStepLwZero) != 0u;
  T y[D];
#pragma unroll
  for (int j = 0; j < D; ++j) y[j] = (j < d) ? (a.y_dev ? a.y_dev[j] : a.y_val[j]) : (T)0;
  const uint32_t tau = a.t + 1u;

  // ---- phase A: load, log-weight, block-0 randoms -------------------------
  // all loads are issued first; the block-0 randoms (independent of them)
  // are drawn while they are in flight
  T lr[NLOC], xr[NLOC][D], z0r[NLOC], lwn[NLOC], ur[NLOC];
  uint32_t qa[NLOC], ca[NLOC];
  uint64_t ga[PPT];
#pragma unroll
  for (int it = 0; it < PPT; ++it) {
    pair_coords(geo, 2u * (tid + it * NT), qa[2 * it], ca[2 * it], qa[2 * it + 1], ca[2 * it + 1], ga[it]);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      xr[2 * it][j] = xr[2 * it + 1][j] = 0;
      if (j < d) Pair<S, T>::load(a.x_in + (size_t)j * N + ga[it], xr[2 * it][j], xr[2 * it + 1][j]);
    }
    if (lwz) {
      lwn[2 * it] = lwn[2 * it + 1] = 0;
    } else {
      Pair<T, T>::load(a.lw_in + ga[it], lwn[2 * it], lwn[2 * it + 1]);
    }
  }
  // block 0 of counter word utau: the step's own (utau = tau) or, for a
  // later stage of a full-cycle step, the stage's (utau = tau + s 2^24),
  // whose dimension-0 normals are not used (phase C draws the step's)
#pragma unroll
  for (int it = 0; it < PPT; ++it) {
    if constexpr (BLOCKPATH) {
      // the dimension-0 normals only where this launch propagates (not in
      // the within-island launch or an inner full-cycle stage)
      const Words b0 = philox((uint32_t)(ga[it] >> 1), a.utau, 0u, a.sid, a.k0, a.k1);
      ur[2 * it] = word_uniform<T>(b0.w0);
      ur[2 * it + 1] = word_uniform<T>(b0.w1);
      z0r[2 * it] = z0r[2 * it + 1] = 0;
      if (prop) box_muller(b0.w2, b0.w3, z0r[2 * it], z0r[2 * it + 1]);
    } else {
      pair_block0<T>((uint32_t)(ga[it] >> 1), a.utau, a.sid, a.k0, a.k1, ur[2 * it], ur[2 * it + 1],
                     z0r[2 * it], z0r[2 * it + 1]);
    }
  }
  // one pair per thread and 4 to 8 dimensions: every normal of the step is
  // drawn here too, while the loads are in flight (none of them depends on
  // the loaded values); phase C then only gathers, propagates and stores
  constexpr bool kEarlyZ = PPT == 1 && D >= 4 && D <= 8;
  T zr[2][kEarlyZ ? D : 1];
  if constexpr (kEarlyZ) {
#pragma unroll
    for (int j = 0; j < D; ++j) zr[0][j] = zr[1][j] = 0;
    if (prop) {
      const uint32_t pr = (uint32_t)(ga[0] >> 1);
      zr[0][0] = z0r[0];
      zr[1][0] = z0r[1];
      if (a.utau != tau) {
        const Words w0 = philox(pr, tau, 0u, a.sid, a.k0, a.k1);
        box_muller(w0.w2, w0.w3, zr[0][0], zr[1][0]);
      }
      pair_normals_rest<D, T>(pr, tau, a.sid, a.k0, a.k1, d, zr[0], zr[1]);
    }
  }
  T tmax = -INFINITY;
#pragma unroll
  for (int e = 0; e < NLOC; ++e) {
    lwn[e] -= off;
    lr[e] = weight ? lwn[e] + Model<D, MK, T>::log_g(a.mp, xr[e], y) : lwn[e];
    tmax = fmaxT(tmax, lr[e]);
    if (!island) {
#pragma unroll
      for (int j = 0; j < D; ++j)
        if (j < d) xs[(size_t)j * xplane + qa[e] * xrow + ca[e]] = xr[e][j];
    }
    scl[ca[e] * P + lix(qa[e])] = lr[e];
    scu[ca[e] * P + lix(qa[e])] = ur[e];
  }
  if (weight) {
    // tile reference point for the variance sums: the tile's first particle
    if (tid == 0) {
#pragma unroll
      for (int j = 0; j < D; ++j) shx[j] = xr[0][j];
    }
    const T mtile = block_max<T, NT>(tmax, red);  // (its barriers publish shx)
    T sh[D];
#pragma unroll
    for (int j = 0; j < D; ++j) sh[j] = shx[j];
    T* prt = a.part_out + (size_t)tile * PS;
    tile_partials<D, T, NT, NLOC>(lr, xr, lwn, sh, d, mtile, red, prt);
  }
  __syncthreads();

  // ---- phase B: group max / scan / carried weight / draw -------------------
  const bool sys = a.systematic != 0;
  T tile_lwmax = -INFINITY;
  if (!BLOCKPATH) {
    switch (log2r) {
      case 1: wave_groups<1, T, NT, PPT>(scl, scu, sca, colw, P, a.lnr, sys, wv, lane, tile_lwmax); break;
      case 2: wave_groups<2, T, NT, PPT>(scl, scu, sca, colw, P, a.lnr, sys, wv, lane, tile_lwmax); break;
      case 3: wave_groups<3, T, NT, PPT>(scl, scu, sca, colw, P, a.lnr, sys, wv, lane, tile_lwmax); break;
      case 4: wave_groups<4, T, NT, PPT>(scl, scu, sca, colw, P, a.lnr, sys, wv, lane, tile_lwmax); break;
      case 5: wave_groups<5, T, NT, PPT>(scl, scu, sca, colw, P, a.lnr, sys, wv, lane, tile_lwmax); break;
      default: wave_groups<6, T, NT, PPT>(scl, scu, sca, colw, P, a.lnr, sys, wv, lane, tile_lwmax); break;
    }
  } else {
    // r > 64: thread t takes the K = 2 PPT consecutive members
    // [K j, K j + K) of group c (G = r / K threads per group, t = c G + j).
    // K divides 64, so those members are K consecutive words. A group's
    // maximum and scan run within the thread, then over its lanes, then
    // (G > 64) over its waves through LDS.
    constexpr int K = 2 * PPT;
    constexpr uint32_t LK = K == 2 ? 1u : (K == 4 ? 2u : (K == 8 ? 3u : 4u));
    static_assert((1 << LK) == K && K <= 16, "members per thread");
    const uint32_t lg_g = log2r - LK;
    const uint32_t G = 1u << lg_g;
    const uint32_t lgw = lg_g < 6u ? lg_g : 6u;      // the group's lanes within one wave
    const uint32_t c = (uint32_t)tid >> lg_g, j = (uint32_t)tid & (G - 1u);
    const uint32_t q0 = j << LK;
    T* colp = scl + c * P;
    const uint32_t w0 = lix(q0);
    T v[K];
    T mx = -INFINITY;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      v[k] = colp[w0 + k];
      mx = fmaxT(mx, v[k]);
    }
    mx = lgw == 6u ? wave_max(mx) : seg_max(mx, lgw, (uint32_t)lane);
    const uint32_t nw = G >> 6;                       // waves per group (G > 64)
    const uint32_t gw0 = nw ? ((uint32_t)wv / nw) * nw : 0u;
    if (lg_g > 6u) {
      if (lane == 0) chm[wv] = mx;
      __syncthreads();
      mx = wave_max((uint32_t)lane < nw ? chm[gw0 + lane] : (T)-INFINITY);
    }
    T run = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      run += fexp(v[k] - mx);
      v[k] = run;
    }
    const uint32_t lq = (uint32_t)lane & ((1u << lgw) - 1u);
    const T incl = seg_scan(run, lgw, lq);
    T off = __shfl_up(incl, 1u, 64);
    if (lq == 0u) off = 0;
    T tot;
    if (lg_g > 6u) {
      if (lane == 63) chs[wv] = incl;
      __syncthreads();
      const T ws = seg_scan((uint32_t)lane < nw ? chs[gw0 + lane] : (T)0, 6u, (uint32_t)lane);
      const uint32_t wi = (uint32_t)wv - gw0;
      if (wi != 0u) off += lane_at(ws, wi - 1u);
      tot = lane_at(ws, nw - 1u);
    } else {
      tot = lgw == 6u ? lane_at(incl, 63u) : __shfl(incl, (int)((uint32_t)lane | (G - 1u)), 64);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) colp[w0 + k] = v[k] + off;
    if (j == 0u) {
      const T lw = mx + flog_ge1(tot) - a.lnr;
      tile_lwmax = lw;
      colw[c] = lw;
    }
    // the systematic draw's U_0: the first member's uniform, read before
    // any position overwrites it
    const T u0 = sys ? scu[c * P] : (T)0;
    __syncthreads();
    int* pos_out = sca + c * P + w0;
    const T* us = scu + c * P + w0;
    switch (log2r) {
      case 7: draw_run<7, K>(colp, us, pos_out, q0, tot, u0, sys); break;
      case 8: draw_run<8, K>(colp, us, pos_out, q0, tot, u0, sys); break;
      case 9: draw_run<9, K>(colp, us, pos_out, q0, tot, u0, sys); break;
      case 10: draw_run<10, K>(colp, us, pos_out, q0, tot, u0, sys); break;
      case 11: draw_run<11, K>(colp, us, pos_out, q0, tot, u0, sys); break;
      default: draw_run<12, K>(colp, us, pos_out, q0, tot, u0, sys); break;
    }
  }
  // the next step's offset: max of the new log-weights (deterministic), one
  // atomic per tile into one of the spread slots
  tile_lwmax = wave_max(tile_lwmax);
  if (lane == 0) shx[wv] = tile_lwmax;
  __syncthreads();
  if (tid == 0 && (a.flags & kStepNoFold) == 0u) {
    T mx = shx[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) mx = fmaxT(mx, shx[w]);
    __hip_atomic_fetch_max(off_slot(a.ctl, a.u + 1, tile % kOffSlots), ord_encode((double)mx),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }

  if (a.ess_out != nullptr) {
    // an ESS-gated stage: [max, sum w, sum w^2] of the tile's carried
    // weights (each group's weight counts for its r members)
    T mt = shx[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) mt = fmaxT(mt, shx[w]);
    T s1 = 0, s2 = 0;
    for (uint32_t c = (uint32_t)tid; c < C; c += NT) {
      const T e = fexp(colw[c] - mt);
      s1 += e;
      s2 += e * e;
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    T* scr = scl;  // free after phase B
    if (lane == 0) {
      scr[2 * wv] = s1;
      scr[2 * wv + 1] = s2;
    }
    __syncthreads();
    if (tid == 0) {
      T t1 = 0, t2 = 0;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) {
        t1 += scr[2 * w];
        t2 += scr[2 * w + 1];
      }
      T* o = a.ess_out + (size_t)tile * 3;
      o[0] = mt;
      o[1] = t1 * (T)r;
      o[2] = t2 * (T)r;
    }
  }

  if (island) {
    // the within-island launch of the island filter: each particle's
    // ancestor and, from each island's first member, the island's carried
    // log-weight (islands are the groups of this stride-1 stage); no states
#pragma unroll
    for (int it = 0; it < PPT; ++it) {
      uint32_t q0, c0, q1, c1;
      uint64_t g0;
      pair_coords(geo, 2u * (tid + it * NT), q0, c0, q1, c1, g0);
      const uint32_t a0 = (uint32_t)((int64_t)g0 + (int64_t)sca[c0 * P + lix(q0)] - (int64_t)q0);
      const uint32_t a1 = (uint32_t)((int64_t)g0 + 1 + (int64_t)sca[c1 * P + lix(q1)] - (int64_t)q1);
      *reinterpret_cast<uint2*>(a.anc + g0) = make_uint2(a0, a1);
      if (q0 == 0u) a.isl_lw[g0 >> log2r] = colw[c0];
    }
    return;
  }

  // ---- phase C: gather, then per Philox block: normals, propagate, store ---
  // each component is stored as soon as its normals exist, so only the
  // gathered states (and, for a dense noise factor, the normals so far)
  // stay live
#pragma unroll
  for (int it = 0; it < PPT; ++it) {
    const uint32_t f0 = 2u * (tid + it * NT);
    T xh[2][D], z[2][D], lwo[2];
    uint32_t ai[2];
    uint64_t g0;
    uint32_t qp[2], cp[2];
    pair_coords(geo, f0, qp[0], cp[0], qp[1], cp[1], g0);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const uint32_t q = qp[e], c = cp[e];
      const uint64_t gi = g0 + (uint64_t)e;
      const uint32_t pos = (uint32_t)sca[c * P + lix(q)];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        xh[e][j] = (j < d) ? xs[(size_t)j * xplane + pos * xrow + c] : (T)0;
        z[e][j] = 0;
      }
      lwo[e] = colw[c];
      ai[e] = (uint32_t)((int64_t)gi + ((int64_t)pos - (int64_t)q) * ((int64_t)1 << a.log2R));
    }
    Pair<T, T>::store(a.lw_out + g0, lwo[0], lwo[1]);
    if (a.anc) {
      a.anc[g0] = ai[0];
      a.anc[g0 + 1] = ai[1];
    }
    if (!prop) {
      // an inner stage of a full-cycle step: the gathered states as they are
#pragma unroll
      for (int j = 0; j < D; ++j)
        if (j < d) Pair<S, T>::store(a.x_out + (size_t)j * N + g0, xh[0][j], xh[1][j]);
      continue;
    }
    if constexpr (kEarlyZ) {
#pragma unroll
      for (int j = 0; j < D; ++j)
        if (j < d)
          Pair<S, T>::store(a.x_out + (size_t)j * N + g0, Model<D, MK, T>::row(a.mp, xh[0], zr[0], j),
                            Model<D, MK, T>::row(a.mp, xh[1], zr[1], j));
      continue;
    }
    z[0][0] = z0r[2 * it];
    z[1][0] = z0r[2 * it + 1];
    if (a.utau != tau) {
      const Words w0 = philox((uint32_t)(g0 >> 1), tau, 0u, a.sid, a.k0, a.k1);
      box_muller(w0.w2, w0.w3, z[0][0], z[1][0]);
    }
    Pair<S, T>::store(a.x_out + g0, Model<D, MK, T>::row(a.mp, xh[0], z[0], 0),
                      Model<D, MK, T>::row(a.mp, xh[1], z[1], 0));
    const uint32_t pr = (uint32_t)(g0 >> 1);
#pragma unroll
    for (int b = 1; 2 * b - 1 < D; ++b) {
      if (2 * b - 1 < d) {
        const Words w = philox(pr, tau, (uint32_t)b, a.sid, a.k0, a.k1);
        box_muller(w.w0, w.w1, z[0][2 * b - 1], z[1][2 * b - 1]);
        Pair<S, T>::store(a.x_out + (size_t)(2 * b - 1) * N + g0,
                          Model<D, MK, T>::row(a.mp, xh[0], z[0], 2 * b - 1),
                          Model<D, MK, T>::row(a.mp, xh[1], z[1], 2 * b - 1));
        if (2 * b < D && 2 * b < d) {
          box_muller(w.w2, w.w3, z[0][2 * b], z[1][2 * b]);
          Pair<S, T>::store(a.x_out + (size_t)(2 * b) * N + g0,
                            Model<D, MK, T>::row(a.mp, xh[0], z[0], 2 * b),
                            Model<D, MK, T>::row(a.mp, xh[1], z[1], 2 * b));
        }
      }
    }
  }
}

// Single filter: block b processes tile xcd_tile(b); block 0 also does the
// step's bookkeeping.
template <int D, int MK, typename T, typename S, int NT, int PPT, bool BLOCKPATH, bool FULL, bool ISL = false>
__global__ void __launch_bounds__(NT) pf_step_tile(StepArgs<T, S> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (blockIdx.x == 0) step_bookkeeping(a);
  step_tile_body<D, MK, T, S, NT, PPT, BLOCKPATH, FULL, ISL>(a, xcd_tile(blockIdx.x, a.ntiles), smem);
}

// ---------------------------------------------------------------------------
// Batched filters: many independent filters (each with its own model, N,
// radix, seed and step counter) advanced by one launch per (dimension,
// model kind) class. Each block takes one tile of one filter; a filter's
// stage comes from its own step counter, so the launches need no per-step
// host data beyond the observation pointer and can be replayed from a graph.
// ---------------------------------------------------------------------------
struct BatchStage {   // stage k of one filter
  uint32_t log2r, log2R, log2C, pad;
  float lnr;
  uint32_t xrow;
  uint32_t reserved[2];
};

struct BatchFilter {  // one filter of the batch (device table entry)
  float* x[2];        // state planes [d][N], by step parity
  float* lw[2];       // log-weights [N], by step parity
  const ModelParams<float>* mp;
  float* part;        // tile partial records of the current step
  Ctl* ctl;
  pf_estimate_t* rec; // estimate record of the last step
  uint64_t N;
  uint32_t d, S, stage0, ntiles;
  uint32_t first_block, yoff, sid, k0;
  uint32_t k1, systematic, reserved[2];
};

struct BatchArgs {
  const BatchFilter* filt;
  const BatchStage* stages;
  const uint32_t* block_filter;   // step kernel: block -> filter
  const uint32_t* class_filters;  // finalize kernel: block -> filter
  const uint8_t* active;          // NULL: every filter steps
  const float* y;                 // packed observations of this step
  uint32_t* tcur;                 // completed steps per filter
};

template <int D, int MK, int NT, int PPT, bool FULL>
__global__ void __launch_bounds__(NT) pf_batch_tile(BatchArgs ba) {
  extern __shared__ __align__(16) unsigned char smem[];
  // without an active mask the class's blocks run in XCD order, so that
  // neighbouring tiles of a filter, which share the L2 lines of their rows,
  // run on one XCD; with a mask (some filters idle) launch order spreads the
  // active filters' blocks evenly over the XCDs, which matters more
  const uint32_t bi = ba.active ? blockIdx.x : xcd_tile(blockIdx.x, gridDim.x);
  const uint32_t f = ba.block_filter[bi];
  if (ba.active && !ba.active[f]) return;
  const BatchFilter& F = ba.filt[f];
  const uint32_t t = ba.tcur[f];
  const uint32_t k = t % F.S;
  const BatchStage& sg = ba.stages[F.stage0 + k];
  StepArgs<float, float> a{};  // every field defined: the tile body tests the optional pointers
  a.x_in = F.x[t & 1u];
  a.x_out = F.x[(t + 1u) & 1u];
  a.lw_in = F.lw[t & 1u];
  a.lw_out = F.lw[(t + 1u) & 1u];
  a.anc = nullptr;
  a.y_dev = ba.y + F.yoff;
  a.mp = F.mp;
  a.part_out = F.part;
  a.ctl = F.ctl;
  a.hist = F.rec;
  a.hist_cap = 1u;
  a.d = F.d;
  a.N = F.N;
  a.log2r = sg.log2r;
  a.log2R = sg.log2R;
  a.log2C = sg.log2C;
  a.pad = sg.pad;
  a.xrow = sg.xrow;
  a.t = t;
  a.k = k;
  a.u = t;
  a.flags = kStepWeight | kStepPropagate;
  a.utau = t + 1u;
  a.ntiles = F.ntiles;
  a.radix = 1u << sg.log2r;
  a.sid = F.sid;
  a.k0 = F.k0;
  a.k1 = F.k1;
  a.systematic = F.systematic;
  a.lnr = sg.lnr;
  step_tile_body<D, MK, float, float, NT, PPT, false, FULL>(a, bi - F.first_block, smem);
}

// Reduction of one filter's tile partials per block (after the class's
// step kernel): estimate record, log-normaliser, offset ring, step counter.
template <int D, int NT>
__global__ void __launch_bounds__(NT) pf_batch_finalize(BatchArgs ba) {
  __shared__ double red[(NT / 64) * (4 + 2 * D)];
  const uint32_t f = ba.class_filters[blockIdx.x];
  if (ba.active && !ba.active[f]) return;
  const BatchFilter& F = ba.filt[f];
  const uint32_t t = ba.tcur[f];
  const uint32_t k = t % F.S;
  FinArgs fa;
  fa.ctl = F.ctl;
  fa.hist = F.rec;
  fa.hist_cap = 1u;
  fa.t = t;
  fa.k = k;
  fa.radix = 1u << ba.stages[F.stage0 + k].log2r;
  fa.d = F.d;
  fa.N = F.N;
  fa.multi = 0u;
  fa.slot = 0u;
  fa.write_rec = 1u;
  fa.use_step_off = 0u;
  fa.unext = t + 1u;
  finalize_partials<D, float, NT, fin_batch<D, float>()>(fa, F.part, F.ntiles, red);
  if (threadIdx.x < 64u) {
    clear_offset(F.ctl, t + 2u, -INFINITY);
    if (threadIdx.x == 0) ba.tcur[f] = t + 1u;
  }
}

// ---------------------------------------------------------------------------
// Global path, kernel 1: log-weights, tile max, tile inclusive CDF and
// estimate partials. Every thread owns NLOC contiguous particles.
// ---------------------------------------------------------------------------
// Layout of the global path's coarse CDF levels (elements of the compute
// type from the start of gcoarse): every 16th entry of the CDF (N / 16 of
// them, then room for one run of 16 past the end), then, from a 16-element
// boundary, 16 slots per weight tile for every 256th entry.
__host__ __device__ constexpr uint64_t global_cc_offset(uint64_t N) { return ((N >> 4) + 31u) & ~(uint64_t)15u; }
__host__ __device__ constexpr uint64_t global_coarse_elems(uint64_t N, uint64_t ntiles) {
  return global_cc_offset(N) + 16u * ntiles;
}

// Sixteen bytes as native vectors (kept in registers when held in arrays).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store16(float* p, const float* v) {
  *reinterpret_cast<f32x4*>(p) = f32x4{v[0], v[1], v[2], v[3]};
}
__device__ __forceinline__ void store16(double* p, const double* v) {
  *reinterpret_cast<f64x2*>(p) = f64x2{v[0], v[1]};
}

// Systematic global resampling: output i (0 <= i < N) draws the target
// (i + U) total / N, with U the step's single uniform. N is a power of two,
// so the scale total / N is exact and the target equals ((i + U) total) / N.
// The targets do not decrease with i, so the outputs of each weight tile form
// one contiguous range; the draw works through them in items of at most
// kSysItem outputs.
constexpr uint32_t kSysItem = 8192;
__host__ __device__ constexpr uint64_t sys_max_items(uint64_t N, uint64_t ntiles) {
  return ntiles + N / kSysItem + 1u;
}
__device__ __forceinline__ double sys_target(uint32_t i, double u0, double scale) {
  return ((double)i + u0) * scale;
}
// Smallest i in [0, N] whose target reaches p (N when none below N does):
// a guess from the inverse of the target (inv_scale = 1 / scale), checked,
// then halving.
__device__ inline uint64_t sys_first_output(double p, double u0, double scale, double inv_scale, uint64_t N) {
  auto reaches = [&](uint64_t i) { return i >= N || sys_target((uint32_t)i, u0, scale) >= p; };
  uint64_t lo = 0, hi = N;  // the answer lies in [lo, hi]
  const double x = scale > 0.0 ? p * inv_scale - u0 : 0.0;
  if (x > 2.0 && x < (double)N - 3.0) {  // false for a NaN
    const uint64_t g = (uint64_t)x;
    if (!reaches(g - 2u)) lo = g - 1u;
    if (reaches(g + 2u)) hi = g + 2u;
  }
  while (lo < hi) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (reaches(mid)) {
      hi = mid;
    } else {
      lo = mid + 1u;
    }
  }
  return lo;
}

// In-tile value of output start + j of weight tile b: the target less the
// tile's prefix, in the tile's CDF units (the largest value at or past the
// total, the targets that fall beyond the last tile).
template <typename T>
__device__ __forceinline__ T sys_value(uint32_t i, double u0, double scale, double total, double preb,
                                       double scb) {
  const double tg = sys_target(i, u0, scale);
  return tg >= total ? (T)INFINITY : (T)((tg - preb) * scb);
}
// Number of an item's outputs start + j (0 <= j < n) whose in-tile value is
// below v: the values do not decrease with j, so this is the first j whose
// value reaches v (n when none does). The guess is the ceiling of the inverse
// of the target (ev = 1 / scb, inv_scale = 1 / scale, base = U + start);
// two checks confirm it in the common case, else a bracket and halving.
template <typename T>
__device__ inline uint32_t sys_outputs_below(T v, uint32_t n, uint32_t start, double u0, double base,
                                             double scale, double inv_scale, double total, double preb,
                                             double scb, double ev) {
  auto reaches = [&](uint32_t j) { return j >= n || sys_value<T>(start + j, u0, scale, total, preb, scb) >= v; };
  const double x = ((double)v * ev + preb) * inv_scale - base;
  uint32_t g;
  if (!(x > 0.0)) {
    g = 0u;  // also a NaN
  } else if (x >= (double)n) {
    g = n;
  } else {
    g = (uint32_t)ceil(x);
  }
  if (reaches(g) && (g == 0u || !reaches(g - 1u))) return g;
  // the answer lies in [lo, hi]
  uint32_t lo = g > 1u ? g - 1u : 0u, hi = g + 1u < n ? g + 1u : n;
  if (lo > 0u && reaches(lo - 1u)) {
    hi = lo - 1u;
    lo = 0u;
  } else if (!reaches(hi)) {
    lo = hi + 1u;
    hi = n;
  }
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (reaches(mid)) {
      hi = mid;
    } else {
      lo = mid + 1u;
    }
  }
  return lo;
}

template <int D, int MK, typename T, typename S, int NT, int PPT>
__global__ void __launch_bounds__(NT) pf_global_weight(StepArgs<T, S> a) {
  constexpr int NLOC = 2 * PPT;
  constexpr int PS = partial_stride(D);
  constexpr uint32_t E = 2u * NT * PPT;
  __shared__ T red[(NT / 64) * PS];
  __shared__ T wtot[NT / 64];
  __shared__ T wmx[NT / 64];
  __shared__ T shx[D];
  const int d = (int)a.d;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint32_t tile = blockIdx.x;
  const uint64_t base = (uint64_t)tile * E + (uint64_t)tid * NLOC;
  const uint64_t N = a.N;
  T y[D];
#pragma unroll
  for (int j = 0; j < D; ++j) y[j] = (j < d) ? (a.y_dev ? a.y_dev[j] : a.y_val[j]) : (T)0;
  T lr[NLOC], xr[NLOC][D], lwn[NLOC];
  T tmax = -INFINITY;
#pragma unroll
  for (int e = 0; e < NLOC; e += 2) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      xr[e][j] = xr[e + 1][j] = 0;
      if (j < d) Pair<S, T>::load(a.x_in + (size_t)j * N + base + e, xr[e][j], xr[e + 1][j]);
    }
    lwn[e] = lwn[e + 1] = 0;  // after a global resample every log-weight is 0
    if (a.lw_nonzero) {
      T w0, w1;
      Pair<T, T>::load(a.lw_in + base + e, w0, w1);
      const T off = (T)read_offset(a.ctl, a.u);
      lwn[e] = w0 - off;
      lwn[e + 1] = w1 - off;
    }
    lr[e] = lwn[e] + Model<D, MK, T>::log_g(a.mp, xr[e], y);
    lr[e + 1] = lwn[e + 1] + Model<D, MK, T>::log_g(a.mp, xr[e + 1], y);
    tmax = fmaxT(tmax, fmaxT(lr[e], lr[e + 1]));
  }
  if (tid == 0) {
#pragma unroll
    for (int j = 0; j < D; ++j) shx[j] = xr[0][j];
  }
  const T mtile = block_max<T, NT>(tmax, red);
  T sh[D];
#pragma unroll
  for (int j = 0; j < D; ++j) sh[j] = shx[j];
  // inclusive CDF of e^{l - mtile} over the tile, in particle order
  T w[NLOC];
  T run = 0;
#pragma unroll
  for (int e = 0; e < NLOC; ++e) {
    w[e] = fexp(lr[e] - mtile);
    run += w[e];
  }
  const T incl = wave_incl_scan(run, lane);
  if (lane == 63) wtot[wv] = incl;
  __syncthreads();
  T woff = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    if (i == wv) woff = tot;
    tot += wtot[i];
  }
  // the thread's CDF values; each is then raised to the largest value of
  // the threads before it, so that the tile's CDF never decreases (the
  // per-thread offsets and the running sums round differently)
  T cv[NLOC];
  {
    T c = woff + incl - run;
#pragma unroll
    for (int e = 0; e < NLOC; ++e) {
      c += w[e];
      cv[e] = c;
    }
    T lm = c;  // inclusive max over the wave's lanes
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
      const T o = __shfl_up(lm, (unsigned)s, 64);
      if (lane >= s) lm = fmaxT(lm, o);
    }
    if (lane == 63) wmx[wv] = lm;
    T before = __shfl_up(lm, 1u, 64);
    if (lane == 0) before = 0;  // the CDF is not negative
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NT / 64; ++i)
      if (i < wv) before = fmaxT(before, wmx[i]);
#pragma unroll
    for (int e = 0; e < NLOC; ++e) cv[e] = fmaxT(cv[e], before);
  }
  T* gcc = a.gcoarse + global_cc_offset(N);  // every 256th entry, 16 slots per tile
#pragma unroll
  for (int e = 0; e < NLOC; ++e) {
    const T c = cv[e];
    const uint64_t i = base + e;
    if (a.systematic) continue;  // below: the plain CDF
    if constexpr (D == 1) {
      // runs of 16: the CDF values, then the 16 states, so that the draw's
      // gather reads the cache line its search has just read
      const uint64_t r0 = 2u * (i & ~(uint64_t)15u) + (i & 15u);
      a.gcdf[r0] = c;
      a.gcdf[r0 + 16u] = xr[e][0];
    } else {
      a.gcdf[i] = c;
    }
    // the coarse levels serve the multinomial draw's search
    const uint32_t q = (uint32_t)(tid * NLOC + e);  // position in the tile
    if ((q & 15u) == 15u) a.gcoarse[i >> 4] = c;
    if ((q & 255u) == 255u) gcc[(size_t)tile * 16u + (q >> 8)] = c;
  }
  if (a.systematic) {
    // the systematic draw reads the plain CDF, and the states where they are
    constexpr int VE = (int)(16u / sizeof(T));
    if constexpr (NLOC % VE == 0) {
#pragma unroll
      for (int e = 0; e < NLOC; e += VE) store16(a.gcdf + base + e, cv + e);
    } else {
#pragma unroll
      for (int e = 0; e < NLOC; ++e) a.gcdf[base + e] = cv[e];
    }
  }
  if (D > 1 && !a.systematic) {
    // the states particle-major: one contiguous row per particle to gather
#pragma unroll
    for (int e = 0; e < NLOC; ++e) {
#pragma unroll
      for (int j = 0; j < D; ++j) a.gx[(base + e) * D + j] = Single<S, T>::cvt(j < d ? xr[e][j] : (T)0);
    }
  }
  T* prt = a.part_out + (size_t)tile * PS;
  tile_partials<D, T, NT, NLOC>(lr, xr, lwn, sh, d, mtile, red, prt);
  __syncthreads();
  if (tid == 0) prt[1] = tot;  // the tile's weight sum is the CDF total (same rounding as the CDF)
}

// Block-wide exclusive scan of NT threads under `op` (identity `ident`): a
// wave pass by shuffles, then one exchange of the wave totals through LDS
// (sw: NT / 64 entries, free again on return). `total` gets the block's.
template <int NT, typename V, typename Op>
__device__ __forceinline__ V block_excl_scan(V v, Op op, V ident, V* sw, V& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  V x = v;
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) {
    const V o = __shfl_up(x, (unsigned)s, 64);
    if (lane >= s) x = op(x, o);
  }
  if (lane == 63) sw[wv] = x;
  V ex = __shfl_up(x, 1u, 64);
  if (lane == 0) ex = ident;
  __syncthreads();
  V before = ident, tot = ident;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    if (w < wv) before = op(before, sw[w]);
    tot = op(tot, sw[w]);
  }
  __syncthreads();
  total = tot;
  return op(before, ex);
}

// Global path, kernel 2 (one block): tile prefix in FP64; every new
// log-weight is equal, so the next offset is 0. Each thread owns a
// contiguous run of tiles and issues the loads of a chunk of them before it
// uses any; the block's reductions and scans run by wave shuffles.
template <int D, typename T, typename S, int NT>
__global__ void __launch_bounds__(NT) pf_global_prefix(StepArgs<T, S> a) {
  __shared__ double swd[NT / 64];
  __shared__ uint32_t swu[NT / 64];
  __shared__ uint32_t sfirst[NT + 1];
  constexpr int PS = partial_stride(D);
  constexpr uint32_t CH = NT >= 1024 ? 4 : 16;
  auto dmax = [](double x, double y) { return fmax(x, y); };
  auto dadd = [](double x, double y) { return x + y; };
  auto umax = [](uint32_t x, uint32_t y) { return x > y ? x : y; };
  auto uadd = [](uint32_t x, uint32_t y) { return x + y; };
  const T* part = a.part_out;
  const uint32_t nt = a.ntiles;
  const int tid = threadIdx.x;
  const uint32_t per = (nt + NT - 1) / NT;
  const uint32_t b0 = tid * per, b1 = min(nt, b0 + per);
  // When one chunk covers the thread's tiles (per <= CH, every tile count
  // up to CH NT), their (m, S) and scales stay in registers from the first
  // read on; otherwise each pass reads them again. The records are a
  // stride apart, so every read is a separate line request, and the single
  // block's request rate is what this kernel's time is made of.
  const bool one = per <= CH;
  T mk[CH], sk[CH];
  double ek[CH];
#pragma unroll
  for (uint32_t k = 0; k < CH; ++k) mk[k] = sk[k] = (T)0, ek[k] = 0.0;
  double m = -INFINITY;
  for (uint32_t c = b0; c < b1; c += CH) {
#pragma unroll
    for (uint32_t k = 0; k < CH; ++k) {
      const size_t b = (size_t)(c + k < b1 ? c + k : b0) * PS;
      mk[k] = part[b];
      sk[k] = part[b + 1];
    }
#pragma unroll
    for (uint32_t k = 0; k < CH; ++k)
      if (c + k < b1) m = fmax(m, (double)mk[k]);
  }
  double M;
  (void)block_excl_scan<NT>(m, dmax, (double)-INFINITY, swd, M);
  // exclusive prefix of T_b = S_b e^{m_b - M}: contiguous runs per thread
  double loc = 0.0;
  for (uint32_t c = b0; c < b1; c += CH) {
    T mv[CH], sv[CH];
#pragma unroll
    for (uint32_t k = 0; k < CH; ++k) {
      const size_t b = (size_t)(c + k < b1 ? c + k : b0) * PS;
      mv[k] = one ? mk[k] : part[b];
      sv[k] = one ? sk[k] : part[b + 1];
    }
#pragma unroll
    for (uint32_t k = 0; k < CH; ++k) {
      if (c + k < b1) {
        const double e = exp((double)mv[k] - M);
        ek[k] = e;
        if (!one) a.gscale[c + k] = e;
        loc += e * (double)sv[k];
      }
    }
  }
  double total;
  double run = block_excl_scan<NT>(loc, dadd, 0.0, swd, total);
  // systematic: the first output of each tile, from its prefix
  const bool plan = a.systematic && a.gwork != nullptr;
  const uint64_t N = a.N;
  const double scale = total / (double)N, inv_scale = (double)N / total;
  const double u0 = plan ? word_uniform<double>(philox(0u, a.t + 1u, 0u, a.sid, a.k0, a.k1).w0) : 0.0;
  uint32_t ofirst = 0, omax = 0, cnt = 0;
  uint32_t fk[CH];  // the tiles' first outputs (registers when one chunk)
#pragma unroll
  for (uint32_t k = 0; k < CH; ++k) fk[k] = 0;
  for (uint32_t c = b0; c < b1; c += CH) {
    T sv[CH];
    double ev[CH];
#pragma unroll
    for (uint32_t k = 0; k < CH; ++k) {
      const uint32_t b = c + k < b1 ? c + k : b0;
      sv[k] = one ? sk[k] : part[(size_t)b * PS + 1];
      ev[k] = one ? ek[k] : a.gscale[b];
    }
#pragma unroll
    for (uint32_t k = 0; k < CH; ++k) {
      if (c + k < b1) {
        a.gpre[c + k] = run;
        if (plan) {
          // non-decreasing within the thread; the items of the tile before
          const uint32_t o = (uint32_t)sys_first_output(run, u0, scale, inv_scale, N);
          const uint32_t om = o > omax ? o : omax;
          if (c + k == b0) {
            ofirst = om;
          } else {
            cnt += (om - omax + kSysItem - 1u) / kSysItem;
          }
          omax = om;
          fk[k] = om;
          a.gfirst[c + k] = om;
        }
        run += ev[k] * (double)sv[k];
        // the draw scales by the reciprocal (a tile whose scale underflows
        // to 0 has no weight and is never drawn)
        a.gscale[c + k] = 1.0 / ev[k];
      }
    }
  }
  if (tid == NT - 1) a.gpre[nt] = total;
  if (plan) {
    // the tiles' ranges split [0, N) exactly: the first outputs are made
    // non-decreasing over the block (the last tile also takes any target at
    // the total); then each tile's items of at most kSysItem outputs
    const bool has = b0 < b1;
    uint32_t omax_all;
    const uint32_t before = block_excl_scan<NT>(omax, umax, 0u, swu, omax_all);
    sfirst[tid] = has ? (ofirst > before ? ofirst : before) : (uint32_t)N;
    if (tid == 0) sfirst[NT] = (uint32_t)N;
    if (tid == 0) a.gfirst[nt] = (uint32_t)N;
    __syncthreads();  // sfirst, and every entry of gfirst (this block's global writes)
    const uint32_t next = sfirst[tid + 1];
    if (has) {
      if (ofirst < before) {
        // rare (prefixes that differ in the last place across threads):
        // raise the thread's leading entries and count again
        cnt = 0;
        uint32_t prev = 0;
        if (one) {
#pragma unroll
          for (uint32_t k = 0; k < CH; ++k) {
            if (b0 + k < b1) {
              const uint32_t o = fk[k] > before ? fk[k] : before;
              fk[k] = o;
              a.gfirst[b0 + k] = o;
              if (k > 0) cnt += (o - prev + kSysItem - 1u) / kSysItem;
              prev = o;
            }
          }
        } else {
          for (uint32_t b = b0; b < b1; ++b) {
            const uint32_t o = a.gfirst[b] > before ? a.gfirst[b] : before;
            a.gfirst[b] = o;
            if (b > b0) cnt += (o - prev + kSysItem - 1u) / kSysItem;
            prev = o;
          }
        }
      }
      const uint32_t last = omax > before ? omax : before;
      cnt += (next - last + kSysItem - 1u) / kSysItem;
    }
    uint32_t nwork;
    uint32_t wi = block_excl_scan<NT>(cnt, uadd, 0u, swu, nwork);
    for (uint32_t c = b0; c < b1; c += CH) {
      uint32_t of[CH + 1];
#pragma unroll
      for (uint32_t k = 0; k < CH; ++k) of[k] = c + k < b1 ? (one ? fk[k] : a.gfirst[c + k]) : next;
      of[CH] = !one && c + CH < b1 ? a.gfirst[c + CH] : next;
#pragma unroll
      for (uint32_t k = 0; k < CH; ++k) {
        if (c + k < b1) {
          const uint32_t e = c + k + 1u < b1 ? of[k + 1] : next;
          for (uint32_t o = of[k]; o < e; o += kSysItem) {
            a.gwork[2u + 2u * wi] = c + k;
            a.gwork[3u + 2u * wi] = o;
            ++wi;
          }
        }
      }
    }
    if (tid == 0) a.gwork[0] = nwork;
  }
  if (tid == 0) *off_slot(a.ctl, a.u + 1, 0) = ord_encode(0.0);
  step_bookkeeping(a);
}

// Global path, kernel 3: inverse-CDF draw over the whole population, then
// the gather from HBM, propagation and store. The draw finds the weight tile
// by binary search of the FP64 tile prefix (in LDS), then the position in the
// tile's FP32 CDF through two coarser levels written by kernel 1 (every 256th
// and every 16th entry): each level reads one aligned run of 16 values and
// counts those <= the target, which is the index of the first larger one
// because the CDF does not decrease. A draw is three dependent 64-byte reads;
// the 2 PPT draws of a thread go through the levels together, so their reads
// are in flight at once. Consecutive threads take consecutive pairs, so the
// monotone targets of systematic resampling read neighbouring runs and gather
// neighbouring states.
template <typename T, int ALIGN>
__device__ __forceinline__ uint32_t count_le16(const T* run, T v, uint32_t n) {
  const T* q = reinterpret_cast<const T*>(__builtin_assume_aligned(run, ALIGN));
  T x[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = q[k];
  // entries past n never count
#pragma unroll
  for (int k = 1; k < 16; ++k) x[k] = (uint32_t)k < n ? x[k] : (T)INFINITY;
  // the run does not decrease, so the count is a binary search on the
  // registers: each level keeps the half that holds the boundary
  uint32_t c = 0;
  bool h = x[7] <= v;
  c += h ? 8u : 0u;
  T y[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) y[k] = h ? x[k + 8] : x[k];
  h = y[3] <= v;
  c += h ? 4u : 0u;
  T z[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) z[k] = h ? y[k + 4] : y[k];
  h = z[1] <= v;
  c += h ? 2u : 0u;
  const T w0 = h ? z[2] : z[0], w1 = h ? z[3] : z[1];
  c += (w0 <= v ? 1u : 0u) + (w0 <= v && w1 <= v ? 1u : 0u);
  return c;
}

// Number of tile prefixes pre[1..nt] that are <= target[e], for NP draws
// together (binary search).
template <int NP>
__device__ __forceinline__ void tile_search(const double* pre, uint32_t nt, const double (&target)[NP],
                                            uint32_t (&b)[NP]) {
#pragma unroll
  for (int e = 0; e < NP; ++e) b[e] = 0;
  for (uint32_t s = 1u << (31u - __clz(nt)); s >= 1u; s >>= 1) {
#pragma unroll
    for (int e = 0; e < NP; ++e)
      if (b[e] + s <= nt && pre[b[e] + s] <= target[e]) b[e] += s;
  }
}

// Particle index of the first CDF entry above lt[e] in weight tile b[e] (at
// most the tile's last), for NP draws level by level: the every-256th level
// (16 slots per tile, ncc = E / 256 of them used), the every-16th level, the
// CDF itself. E = 2^lg_e >= 128 particles per tile.
// PAIRED: the CDF is stored in runs of 16 followed by 16 other values (the
// states, for d = 1), so run j of a tile starts at twice its particle index.
template <typename T, int NP, bool PAIRED>
__device__ __forceinline__ void tile_positions(const T* gcc, const T* gcoarse, const T* gcdf, const uint32_t (&b)[NP],
                                               const T (&lt)[NP], uint32_t lg_e, uint64_t (&aidx)[NP]) {
  const uint32_t nb = 1u << (lg_e - 4u);        // 16-entry runs per tile
  const uint32_t ncc = nb >> 4;                 // 256-entry runs per tile (0 below 256)
  const uint32_t nb_run = nb < 16u ? nb : 16u;  // coarse entries in one level-B run
  uint32_t j[NP];
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    uint32_t c = 0;
    if (ncc) {
      c = count_le16<T, 16 * sizeof(T)>(gcc + (size_t)b[e] * 16u, lt[e], ncc);
      c = c < ncc ? c : ncc - 1u;
    }
    j[e] = c;
  }
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    const uint32_t c = count_le16<T, 16>(gcoarse + (size_t)b[e] * nb + 16u * j[e], lt[e], nb_run);
    j[e] = 16u * j[e] + (c < nb_run ? c : nb_run - 1u);
  }
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    const uint64_t run0 = ((uint64_t)b[e] << lg_e) + 16u * j[e];
    const uint32_t c = count_le16<T, 16 * sizeof(T)>(gcdf + (PAIRED ? 2u * run0 : run0), lt[e], 16u);
    aidx[e] = run0 + (c < 16u ? c : 15u);
  }
}

template <int D, int MK, typename T, typename S, int NT, int PPT>
__global__ void __launch_bounds__(NT) pf_global_draw(StepArgs<T, S> a, uint32_t tile_elems, uint32_t nchunks) {
  constexpr int NP = 2 * PPT;
  extern __shared__ __align__(16) unsigned char smem[];
  double* spre = reinterpret_cast<double*>(smem);
  const uint32_t nt = a.ntiles;
  const bool pre_in_lds = nt <= 4096u;
  if (pre_in_lds) {
    for (uint32_t b = threadIdx.x; b <= nt; b += NT) spre[b] = a.gpre[b];
  }
  __syncthreads();
  const double* pre = pre_in_lds ? spre : a.gpre;
  const int d = (int)a.d;
  const uint64_t N = a.N;
  const uint64_t npairs = N >> 1;
  const double total = a.gpre[nt];
  const uint32_t tau = a.t + 1u;
  const uint32_t lg_e = 31u - __clz(tile_elems);
  const T* gcc = a.gcoarse + global_cc_offset(N);
  double u0sys = 0.0;
  if (a.systematic) u0sys = word_uniform<double>(philox(0u, tau, 0u, a.sid, a.k0, a.k1).w0);
  // a persistent grid: block b takes chunks b, b + gridDim.x, ... of NT PPT
  // pairs, so the tile prefix is staged in LDS once per block
  for (uint32_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    // the thread's pairs (clamped for the arithmetic; only valid ones store)
    uint32_t pr[PPT];
    T u[NP], z0[NP];
#pragma unroll
    for (int it = 0; it < PPT; ++it) {
      const uint64_t p = ((uint64_t)chunk * PPT + it) * NT + threadIdx.x;
      pr[it] = (uint32_t)(p < npairs ? p : npairs - 1u);
      pair_block0<T>(pr[it], tau, a.sid, a.k0, a.k1, u[2 * it], u[2 * it + 1], z0[2 * it], z0[2 * it + 1]);
    }
    double target[NP];
#pragma unroll
    for (int e = 0; e < NP; ++e) {
      const uint64_t i = 2ull * pr[e >> 1] + (uint64_t)(e & 1);
      target[e] = a.systematic ? ((double)i + u0sys) * total / (double)N : (double)u[e] * total;
    }
    // tile: number of tile prefixes P_1..P_nt that are <= target (the LDS
    // copy through a pointer the compiler knows is LDS)
    uint32_t b[NP];
    if (pre_in_lds) tile_search<NP>(spre, nt, target, b);
    else tile_search<NP>(a.gpre, nt, target, b);
    // beyond the last tile (target at the total): the last tile's last entry
    T lt[NP];
#pragma unroll
    for (int e = 0; e < NP; ++e) {
      const bool past = b[e] >= nt;
      b[e] = past ? nt - 1u : b[e];
      lt[e] = past ? (T)INFINITY : (T)((target[e] - pre[b[e]]) * a.gscale[b[e]]);
    }
    uint64_t aidx[NP];
    tile_positions<T, NP, D == 1>(gcc, a.gcoarse, a.gcdf, b, lt, lg_e, aidx);
    // gather, propagate, store (one pair at a time)
#pragma unroll
    for (int it = 0; it < PPT; ++it) {
      const uint64_t p = ((uint64_t)chunk * PPT + it) * NT + threadIdx.x;
      if (p >= npairs) continue;
      T z[2][D], xo[2][D];
#pragma unroll
      for (int jj = 0; jj < D; ++jj) z[0][jj] = z[1][jj] = 0;
      z[0][0] = z0[2 * it];
      z[1][0] = z0[2 * it + 1];
      pair_normals_rest<D, T>((uint32_t)p, tau, a.sid, a.k0, a.k1, d, z[0], z[1]);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const uint64_t ai = aidx[2 * it + e];
        T xh[D];
        if constexpr (D == 1) {
          xh[0] = a.gcdf[2u * (ai & ~(uint64_t)15u) + 16u + (ai & 15u)];
        } else {
#pragma unroll
          for (int jj = 0; jj < D; ++jj) xh[jj] = Single<S, T>::load(a.gx + ai * D + jj);
        }
        Model<D, MK, T>::propagate(a.mp, xh, z[e], xo[e]);
      }
#pragma unroll
      for (int jj = 0; jj < D; ++jj)
        if (jj < d) Pair<S, T>::store(a.x_out + (size_t)jj * N + 2 * p, xo[0][jj], xo[1][jj]);
      if (a.anc) {
        a.anc[2 * p] = (uint32_t)aidx[2 * it];
        a.anc[2 * p + 1] = (uint32_t)aidx[2 * it + 1];
      }
    }
  }
}

// Global path, kernel 3 for systematic resampling, by offspring ranges
// instead of a search per draw. A persistent grid works through the items of
// kernel 2's plan (one weight tile, at most kSysItem consecutive outputs).
// Per item: each particle q of the tile takes the outputs j with
// cdf_{q-1} <= value_j < cdf_q (the last particle also every value at or
// above its CDF), found by inverting the monotone values at cdf_q; the CDF
// is read once, coalesced, and never decreases (kernel 1), so the ranges
// split the item's outputs exactly. The particles write their index over
// their range in LDS; then the pairs of outputs draw their normals, gather
// (d = 1: the tile's states staged in LDS), propagate and store, coalesced.
// Item w of the systematic draw: its tile, first output, end of the tile's
// outputs, the tile's prefix and reciprocal scale, and this thread's 16-byte
// loads of the tile's CDF (pc) and, d = 1, of its states (px). Every slot
// loads (a slot past the tile reads the tile's first values, which are not
// used), so that the slots stay in registers.
template <int D, typename T, typename S, int NT, int PF, int PFX>
__device__ __forceinline__ void sys_fetch(const StepArgs<T, S>& a, uint32_t w, uint32_t lg_e, uint32_t& b,
                                          uint32_t& start, uint32_t& lim, double& preb, double& scb,
                                          u32x4 (&pc)[PF], u32x4 (&px)[PFX]) {
  constexpr uint32_t VE = 16u / sizeof(T), VS = 16u / sizeof(S);
  b = a.gwork[2u + 2u * w];
  start = a.gwork[3u + 2u * w];
  lim = a.gfirst[b + 1u];
  preb = a.gpre[b];
  scb = a.gscale[b];
  const uint64_t tb = (uint64_t)b << lg_e;
  const uint32_t E = 1u << lg_e;
  const u32x4* srcc = reinterpret_cast<const u32x4*>(a.gcdf + tb);
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const uint32_t v = threadIdx.x + (uint32_t)k * NT;
    pc[k] = srcc[v < E / VE ? v : 0u];
  }
  if constexpr (D == 1) {
    const u32x4* srcx = reinterpret_cast<const u32x4*>(a.x_in + tb);
#pragma unroll
    for (int k = 0; k < PFX; ++k) {
      const uint32_t v = threadIdx.x + (uint32_t)k * NT;
      px[k] = srcx[v < E / VS ? v : 0u];
    }
  }
}

// Global path, kernel 3 for systematic resampling, by offspring ranges
// instead of a search per draw. A persistent grid works through the items of
// kernel 2's plan (one weight tile, at most kSysItem consecutive outputs).
// Per item: each particle q of the tile takes the outputs j with
// cdf_{q-1} <= value_j < cdf_q (the last particle also every value at or
// above its CDF), found by inverting the monotone values at cdf_q; the CDF
// is read once, coalesced, and never decreases (kernel 1), so the ranges
// split the item's outputs exactly. The particles write their index over
// their range in LDS; then the pairs of outputs draw their normals, gather
// (d = 1: the tile's states staged in LDS; else from the state planes, whose
// reads follow the non-decreasing ancestors), propagate and store, coalesced.
// The next item's loads are issued before the current item's outputs.
template <int D, int MK, typename T, typename S, int NT>
__global__ void __launch_bounds__(NT) pf_global_sys_draw(StepArgs<T, S> a, uint32_t tile_elems) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t E = tile_elems;  // at most 4096
  // LDS: d = 1, the tile's states; the output count below each CDF value;
  // the tile's CDF, whose space then holds each output's ancestor (its
  // position in the tile)
  S* sxs = reinterpret_cast<S*>(smem);
  uint16_t* sf = reinterpret_cast<uint16_t*>(smem + (D == 1 ? (size_t)E * sizeof(S) : 0u));
  T* scdf = reinterpret_cast<T*>(sf + E);
  uint16_t* spos = reinterpret_cast<uint16_t*>(scdf);
  const uint32_t nwork = a.gwork[0];
  const uint32_t nt = a.ntiles;
  const uint64_t N = a.N;
  const double total = a.gpre[nt];
  const double scale = total / (double)N, inv_scale = (double)N / total;
  const uint32_t tau = a.t + 1u;
  const double u0 = word_uniform<double>(philox(0u, tau, 0u, a.sid, a.k0, a.k1).w0);
  const int d = (int)a.d;
  const uint32_t lg_e = 31u - __clz(E);
  constexpr uint32_t VE = 16u / sizeof(T), VS = 16u / sizeof(S);
  constexpr int PF = (int)((4096u / VE + NT - 1u) / NT);
  constexpr int PFX = D == 1 ? (int)((4096u / VS + NT - 1u) / NT) : 1;
  uint32_t b = 0, start = 0, lim = 0;
  double preb = 0.0, scb = 0.0;
  u32x4 pc[PF], px[PFX];
  if (blockIdx.x < nwork) sys_fetch<D, T, S, NT, PF, PFX>(a, blockIdx.x, lg_e, b, start, lim, preb, scb, pc, px);
  for (uint32_t w = blockIdx.x; w < nwork; w += gridDim.x) {
    const uint32_t end = lim - start > kSysItem ? start + kSysItem : lim;
    const uint32_t n = end - start, s0 = start;
    const uint64_t tbase = (uint64_t)b << lg_e;
    const double ev = 1.0 / scb, base = u0 + (double)s0, pb = preb, sb = scb;
    __syncthreads();  // the previous item's reads of LDS are done
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const uint32_t v = threadIdx.x + (uint32_t)k * NT;
      if (v < E / VE) *reinterpret_cast<u32x4*>(scdf + v * VE) = pc[k];
    }
    if constexpr (D == 1) {
#pragma unroll
      for (int k = 0; k < PFX; ++k) {
        const uint32_t v = threadIdx.x + (uint32_t)k * NT;
        if (v < E / VS) *reinterpret_cast<u32x4*>(sxs + v * VS) = px[k];
      }
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < E; q += NT)
      sf[q] = (uint16_t)sys_outputs_below<T>(scdf[q], n, s0, u0, base, scale, inv_scale, total, pb, sb, ev);
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < E; q += NT) {
      const uint32_t lo = q == 0u ? 0u : (uint32_t)sf[q - 1u];
      const uint32_t hi = q == E - 1u ? n : (uint32_t)sf[q];
      for (uint32_t j = lo; j < hi; ++j) spos[j] = (uint16_t)q;
    }
    __syncthreads();
    if (w + gridDim.x < nwork)
      sys_fetch<D, T, S, NT, PF, PFX>(a, w + gridDim.x, lg_e, b, start, lim, preb, scb, pc, px);
    const uint32_t p_lo = s0 >> 1, p_end = (end + 1u) >> 1;
    for (uint32_t p = p_lo + threadIdx.x; p < p_end; p += NT) {
      T z[2][D], xo[2][D];
#pragma unroll
      for (int jj = 0; jj < D; ++jj) z[0][jj] = z[1][jj] = 0;
      T uu0, uu1;
      pair_block0<T>(p, tau, a.sid, a.k0, a.k1, uu0, uu1, z[0][0], z[1][0]);
      pair_normals_rest<D, T>(p, tau, a.sid, a.k0, a.k1, d, z[0], z[1]);
      bool in[2];
      uint32_t q[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const uint32_t i = 2u * p + (uint32_t)e;
        in[e] = i >= s0 && i < end;
        const uint32_t qq = in[e] ? (uint32_t)spos[i - s0] : 0u;
        q[e] = qq < E ? qq : E - 1u;
        T xh[D];
        if constexpr (D == 1) {
          xh[0] = Single<S, T>::load(sxs + q[e]);
        } else {
#pragma unroll
          for (int jj = 0; jj < D; ++jj)
            xh[jj] = jj < d ? Single<S, T>::load(a.x_in + (size_t)jj * N + tbase + q[e]) : (T)0;
        }
        Model<D, MK, T>::propagate(a.mp, xh, z[e], xo[e]);
      }
      if (in[0] && in[1]) {
#pragma unroll
        for (int jj = 0; jj < D; ++jj)
          if (jj < d) Pair<S, T>::store(a.x_out + (size_t)jj * N + 2u * p, xo[0][jj], xo[1][jj]);
        if (a.anc) {
          a.anc[2u * p] = (uint32_t)(tbase + q[0]);
          a.anc[2u * p + 1u] = (uint32_t)(tbase + q[1]);
        }
      } else {
        // a pair split between two items: each writes its own output
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          if (!in[e]) continue;
#pragma unroll
          for (int jj = 0; jj < D; ++jj)
            if (jj < d) a.x_out[(size_t)jj * N + 2u * p + e] = Single<S, T>::cvt(xo[e][jj]);
          if (a.anc) a.anc[2u * p + e] = (uint32_t)(tbase + q[e]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Island filter (AIRPF, Algorithms 4-7). A step is three launches: the step
// tile kernel with kStepIsland (weights, estimate partials, within-island
// resampling of Algorithm 5, one group of M consecutive particles per
// island), pf_island_draw (the log2 m stages of Algorithm 6 over islands, with
// the no-swap rule of Algorithm 7) and pf_island_gather (whole-island copies
// through the within-island ancestors, then the mutation).
// ---------------------------------------------------------------------------
// Island arrays (log-weight, source index, the stage's uniforms) of up to
// this many bytes are kept in LDS by pf_island_draw.
constexpr size_t kIslandLdsBytes = 96u * 1024u;
// Largest source island (d M states) the LDS-staged island gather holds:
// two blocks still fit a CU.
constexpr size_t kIslandGatherLds = 64u * 1024u;

struct IslandArgs {
  const void* isl_lw;  // carried log-weight per island, compute type
  void* lv;            // m values of the compute type: scratch when not in LDS
  uint32_t* src;       // m: the source island of each destination island (output)
  uint32_t m, log2m;
  uint32_t tau, sid, k0, k1;
  uint32_t no_swap;    // Algorithm 7 (else Algorithm 6)
  uint32_t use_lds;    // the island arrays live in LDS ((sizeof(T) + 8) mb bytes)
  uint32_t uni_all;    // with use_lds: every stage's uniforms are drawn first (4 mb stages bytes more)
  // the stages [s_begin, s_end) of islands [b mb, b mb + mb) in block b; the
  // stages below log2 mb pair islands of one block only. from_prev: start
  // from lv and src of the launch before (else from the island weights and
  // the identity); the launch writes src, and lv when lv_out is set. One
  // launch with mb = m runs everything.
  uint32_t mb, s_begin, s_end, from_prev, lv_out;
};

// Uniform of island i at island stage s: word i mod 4 of the Philox block
// (i / 4, tau, kIslandBlock + s, stream).
__device__ __forceinline__ float island_uniform(const IslandArgs& ia, uint32_t i, uint32_t s) {
  const Words w = philox(i >> 2, ia.tau, kIslandBlock + s, ia.sid, ia.k0, ia.k1);
  const uint32_t k = i & 3u;
  return word_uniform<float>(k == 0u ? w.w0 : k == 1u ? w.w1 : k == 2u ? w.w2 : w.w3);
}
// All four uniforms of Philox block q of stage s (islands 4q .. 4q + 3, those
// below m) into us[4q - base ..].
__device__ __forceinline__ void island_uniforms4(const IslandArgs& ia, uint32_t q, uint32_t s, float* us,
                                                 uint32_t base) {
  const Words w = philox(q, ia.tau, kIslandBlock + s, ia.sid, ia.k0, ia.k1);
  const uint32_t i = q << 2, l = i - base;
  us[l] = word_uniform<float>(w.w0);
  if (i + 1u < ia.m) us[l + 1u] = word_uniform<float>(w.w1);
  if (i + 2u < ia.m) us[l + 2u] = word_uniform<float>(w.w2);
  if (i + 3u < ia.m) us[l + 3u] = word_uniform<float>(w.w3);
}

// A block of up to 1024 threads. Stage s pairs island lo (bit s clear) with
// hi = lo + 2^s; each draws, with its own uniform, the island it holds next
// with probability proportional to the pair's weights (members in index
// order, first member whose cumulative weight exceeds the target), both then
// carry the pair mean. With no_swap, a pair whose draws exchange the two
// samples keeps both in place. One thread owns a pair for the whole stage,
// so a stage needs no synchronisation inside it; with the arrays in LDS the
// uniforms are drawn first by all threads (four islands per Philox block),
// for every stage of the launch at once when they fit. Many islands run in
// two launches: the stages inside blocks of mb islands on m / mb blocks,
// then the remaining stages on one block.
template <typename T>
__global__ void __launch_bounds__(1024) pf_island_draw(IslandArgs ia) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t mb = ia.mb, tid = threadIdx.x, nth = blockDim.x;
  const uint32_t base = blockIdx.x * mb;
  const bool in_lds = ia.use_lds != 0u;
  T* lv = in_lds ? reinterpret_cast<T*>(smem) : reinterpret_cast<T*>(ia.lv);
  uint32_t* src = in_lds ? reinterpret_cast<uint32_t*>(smem + (size_t)mb * sizeof(T)) : ia.src;
  float* us = reinterpret_cast<float*>(smem + (size_t)mb * (sizeof(T) + 4));
  const T* w = reinterpret_cast<const T*>(ia.from_prev ? ia.lv : ia.isl_lw);
  for (uint32_t i = tid; i < mb; i += nth) {
    lv[i] = w[base + i];
    src[i] = ia.from_prev ? ia.src[base + i] : base + i;
  }
  __syncthreads();
  const T ln2 = (T)0.6931471805599453;
  // Philox blocks of this block's islands: q0 .. q0 + nq - 1 (four islands each)
  const uint32_t q0 = base >> 2, nq = (mb + 3u) >> 2;
  const uint32_t nst = ia.s_end - ia.s_begin;
  const bool all = in_lds && ia.uni_all != 0u;
  if (all) {
    // every stage's uniforms at once: independent Philox blocks for all threads
    for (uint32_t wq = tid; wq < nq * nst; wq += nth)
      island_uniforms4(ia, q0 + wq % nq, ia.s_begin + wq / nq, us + (size_t)(wq / nq) * mb, base);
    __syncthreads();
  }
  for (uint32_t s = ia.s_begin; s < ia.s_end; ++s) {
    const uint32_t bit = 1u << s;
    if (in_lds && !all) {
      for (uint32_t q = tid; q < nq; q += nth) island_uniforms4(ia, q0 + q, s, us, base);
      __syncthreads();
    }
    const float* ust = all ? us + (size_t)(s - ia.s_begin) * mb : us;
    for (uint32_t p = tid; p < (mb >> 1); p += nth) {
      const uint32_t lo = ((p >> s) << (s + 1)) | (p & (bit - 1u)), hi = lo | bit;
      const float ulo = in_lds ? ust[lo] : island_uniform(ia, base + lo, s);
      const float uhi = in_lds ? ust[hi] : island_uniform(ia, base + hi, s);
      const T vlo = lv[lo], vhi = lv[hi];
      const T mx = fmaxT(vlo, vhi);
      const T clo = fexp(vlo - mx), tot = clo + fexp(vhi - mx);
      uint32_t plo = clo > (T)ulo * tot ? lo : hi;
      uint32_t phi = clo > (T)uhi * tot ? lo : hi;
      if (ia.no_swap && plo == hi && phi == lo) {
        plo = lo;
        phi = hi;
      }
      const uint32_t slo = src[plo], shi = src[phi];
      const T nv = mx + flog_ge1(tot) - ln2;
      src[lo] = slo;
      src[hi] = shi;
      lv[lo] = nv;
      lv[hi] = nv;
    }
    __syncthreads();
  }
  if (in_lds) {
    T* lvo = reinterpret_cast<T*>(ia.lv);
    for (uint32_t i = tid; i < mb; i += nth) {
      ia.src[base + i] = src[i];
      if (ia.lv_out) lvo[base + i] = lv[i];
    }
  }
}

// Destination particle kM + j copies particle isl_anc[src[k] M + j] (the
// within-island draw of its source island), then mutates with the step's
// normals. One particle pair per thread (a pair never straddles an island).
template <int D, int MK, typename T, typename S>
__global__ void __launch_bounds__(256) pf_island_gather(StepArgs<T, S> a) {
  const int d = (int)a.d;
  const uint64_t N = a.N, npair = N >> 1;
  const uint32_t tau = a.t + 1u;
  const uint64_t mmask = ((uint64_t)1 << a.log2M) - 1u;
  for (uint64_t p = (uint64_t)blockIdx.x * 256u + threadIdx.x; p < npair; p += (uint64_t)gridDim.x * 256u) {
    const uint64_t i0 = 2u * p;
    const uint64_t base = (uint64_t)a.isl_src[i0 >> a.log2M] << a.log2M;
    const uint2 aa = *reinterpret_cast<const uint2*>(a.isl_anc + base + (i0 & mmask));
    if (a.anc) *reinterpret_cast<uint2*>(a.anc + i0) = aa;
    T xh[2][D], z[2][D], xo[2][D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      xh[0][j] = (j < d) ? Single<S, T>::load(a.x_in + (size_t)j * N + aa.x) : (T)0;
      xh[1][j] = (j < d) ? Single<S, T>::load(a.x_in + (size_t)j * N + aa.y) : (T)0;
      z[0][j] = z[1][j] = 0;
    }
    T u0, u1;
    pair_randoms<D, T>((uint32_t)p, tau, a.sid, a.k0, a.k1, d, u0, u1, z[0], z[1]);
    Model<D, MK, T>::propagate(a.mp, xh[0], z[0], xo[0]);
    Model<D, MK, T>::propagate(a.mp, xh[1], z[1], xo[1]);
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (j < d) Pair<S, T>::store(a.x_out + (size_t)j * N + i0, xo[0][j], xo[1][j]);
  }
}

// The same mutation with one block per destination island k, for islands
// of M = 1024 PG particles whose states fit in LDS (d M values): the source
// island src[k] is staged with coalesced loads; while they are in flight
// each thread reads the ancestors of its PG pairs and draws their normals
// (none of which depends on the states); then every ancestor is read from
// LDS instead of by a scattered global load. Results are those of
// pf_island_gather.
constexpr int kIslandGatherNT = 512;
template <int D, int MK, typename T, typename S, int PG>
__global__ void __launch_bounds__(kIslandGatherNT) pf_island_gather_lds(StepArgs<T, S> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* xs = reinterpret_cast<T*>(smem);  // [j][member]
  constexpr uint32_t M = 2u * kIslandGatherNT * PG;
  const int d = (int)a.d;
  const uint64_t N = a.N;
  const uint32_t tau = a.t + 1u;
  const uint64_t sbase = (uint64_t)a.isl_src[blockIdx.x] * M;
  const uint64_t dbase = (uint64_t)blockIdx.x * M;
#pragma unroll
  for (int g = 0; g < PG; ++g) {
    const uint32_t q = threadIdx.x + (uint32_t)g * kIslandGatherNT;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if (j < d) {
        T v0, v1;
        Pair<S, T>::load(a.x_in + (size_t)j * N + sbase + 2u * q, v0, v1);
        xs[(size_t)j * M + 2u * q] = v0;
        xs[(size_t)j * M + 2u * q + 1u] = v1;
      }
    }
  }
  uint2 aa[PG];
  T z[PG][2][D];
#pragma unroll
  for (int g = 0; g < PG; ++g) {
    const uint32_t q = threadIdx.x + (uint32_t)g * kIslandGatherNT;
    aa[g] = *reinterpret_cast<const uint2*>(a.isl_anc + sbase + 2u * q);
#pragma unroll
    for (int j = 0; j < D; ++j) z[g][0][j] = z[g][1][j] = 0;
    T u0, u1;
    pair_randoms<D, T>((uint32_t)((dbase >> 1) + q), tau, a.sid, a.k0, a.k1, d, u0, u1, z[g][0], z[g][1]);
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < PG; ++g) {
    const uint32_t q = threadIdx.x + (uint32_t)g * kIslandGatherNT;
    const uint64_t i0 = dbase + 2u * q;
    if (a.anc) *reinterpret_cast<uint2*>(a.anc + i0) = aa[g];
    // ancestors of a within-island draw lie in the source island
    const uint32_t l0 = (uint32_t)(aa[g].x - sbase), l1 = (uint32_t)(aa[g].y - sbase);
    T xh[2][D], xo[2][D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      xh[0][j] = (j < d) ? xs[(size_t)j * M + l0] : (T)0;
      xh[1][j] = (j < d) ? xs[(size_t)j * M + l1] : (T)0;
    }
    Model<D, MK, T>::propagate(a.mp, xh[0], z[g][0], xo[0]);
    Model<D, MK, T>::propagate(a.mp, xh[1], z[g][1], xo[1]);
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (j < d) Pair<S, T>::store(a.x_out + (size_t)j * N + i0, xo[0][j], xo[1][j]);
  }
}

// ---------------------------------------------------------------------------
// ESS-gated stages with a rotating start (Section 1.2, Section 6.4), FP32
// states. A step is a fixed sequence of launches whose work the device
// decides: pf_adapt_weight (weights, estimate partials; the weighted
// log-weights stored in place), pf_adapt_decide, then S stage slots, each a
// pf_adapt_stage (one butterfly stage in place, or nothing) followed by a
// pf_adapt_decide, then pf_adapt_propagate. The control words live in Ctl.
// ---------------------------------------------------------------------------
template <int D, int MK, bool FULL>
__global__ void __launch_bounds__(256) pf_adapt_weight(StepArgs<float, float> a) {
  using T = float;
  constexpr int NT = 256;
  constexpr int PS = partial_stride(D);
  __shared__ T red[(NT / 64) * PS];
  __shared__ T shx[D];
  if (blockIdx.x == 0) step_bookkeeping(a);
  const int d = FULL ? D : (int)a.d;
  const uint64_t N = a.N;
  const uint64_t i0 = 2u * ((uint64_t)blockIdx.x * NT + threadIdx.x);  // grid: N / 512 blocks
  T xr[2][D], lwn[2], lr[2], y[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    xr[0][j] = xr[1][j] = 0;
    if (j < d) Pair<float, T>::load(a.x_in + (size_t)j * N + i0, xr[0][j], xr[1][j]);
    y[j] = (j < d) ? (a.y_dev ? a.y_dev[j] : a.y_val[j]) : (T)0;
  }
  Pair<T, T>::load(a.lw_in + i0, lwn[0], lwn[1]);
  const T off = (T)read_offset(a.ctl, a.u);
  T tmax = -INFINITY;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    lwn[e] -= off;
    lr[e] = lwn[e] + Model<D, MK, T>::log_g(a.mp, xr[e], y);
    tmax = fmaxT(tmax, lr[e]);
  }
  Pair<T, T>::store(a.lw_out + i0, lr[0], lr[1]);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < D; ++j) shx[j] = xr[0][j];
  }
  const T mtile = block_max<T, NT>(tmax, red);
  T sh[D];
#pragma unroll
  for (int j = 0; j < D; ++j) sh[j] = shx[j];
  tile_partials<D, T, NT, 2>(lr, xr, lwn, sh, d, mtile, red, a.part_out + (size_t)blockIdx.x * PS);
}

// One stage slot: the stage the control block names, in place (the tiles
// of a stage are disjoint, and each is read whole before it is written), or
// nothing when the decisions so far stopped the step's resampling.
template <int D, int MK, int NT, int PPT, bool FULL>
__global__ void __launch_bounds__(NT) pf_adapt_stage(StepArgs<float, float> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Ctl* c = a.ctl;
  if (c->ad_active == 0u) return;
  const uint32_t k = c->ad_stage;
  const AdStage g = a.stab[k];
  if (blockIdx.x >= g.ntiles) return;
  StepArgs<float, float> b = a;
  b.k = k;
  b.log2r = g.log2r;
  b.log2R = g.log2R;
  b.log2C = g.log2C;
  b.pad = g.pad;
  b.xrow = g.xrow;
  b.ntiles = g.ntiles;
  b.radix = 1u << g.log2r;
  b.lnr = g.lnr;
  b.utau = a.utau + c->ad_run * kStageTau;
  step_tile_body<D, MK, float, float, NT, PPT, false, FULL>(b, xcd_tile(blockIdx.x, g.ntiles), smem);
}

struct AdDecide {
  Ctl* ctl;
  const AdStage* stab;
  const void* rec;        // per-tile records: [m, S, sw2, ...] with `stride` values
  uint32_t stride;
  uint32_t ntiles_first;  // tiles of the weighting launch
  uint32_t first;         // the decision after the weighting (else after a stage slot)
  uint32_t S, t;
  uint64_t N;
  double theta;
  pf_estimate_t* hist;
  uint32_t hist_cap;
};

// ESS of the records (FP64, fixed order) and the next decision: before the
// first stage, resample only if the ESS is below theta; after a stage, go on
// with the next stage (cyclically) only while it is below theta and fewer
// than S stages ran. The step's record gets the number of stages run.
template <typename T>
__global__ void __launch_bounds__(1024) pf_adapt_decide(AdDecide ad) {
  __shared__ double wm[16], w1[16], w2[16];
  Ctl* c = ad.ctl;
  if (!ad.first && c->ad_active == 0u) return;
  const uint32_t ntiles = ad.first ? ad.ntiles_first : ad.stab[c->ad_stage].ntiles;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double m = -INFINITY, s1 = 0.0, s2 = 0.0;
  for (uint32_t b = tid; b < ntiles; b += 1024u) {
    const T* r = reinterpret_cast<const T*>(ad.rec) + (size_t)b * ad.stride;
    const double mb = (double)r[0];
    if (mb > m) {
      const double sc = m == -INFINITY ? 0.0 : exp(m - mb);
      s1 *= sc;
      s2 *= sc * sc;
      m = mb;
    }
    const double e = mb == -INFINITY ? 0.0 : exp(mb - m);
    s1 += e * (double)r[1];
    s2 += e * e * (double)r[2];
  }
  // waves: common max, fixed-pattern sums; then wave order
  const double Mw = wave_max(m);
  const double sc = m == -INFINITY ? 0.0 : exp(m - Mw);
  s1 = wave_sum(s1 * sc);
  s2 = wave_sum(s2 * (sc * sc));
  if (lane == 0) {
    wm[wv] = Mw;
    w1[wv] = s1;
    w2[wv] = s2;
  }
  __syncthreads();
  if (wv != 0) return;
  // the 16 wave results, one per lane of wave 0 (the rescaling exponentials
  // run in parallel, not one after another)
  const double mw = lane < 16 ? wm[lane] : -INFINITY;
  const double M = wave_max(mw);
  const double e = mw == -INFINITY ? 0.0 : exp(mw - M);
  const double S1 = wave_sum(lane < 16 ? e * w1[lane] : 0.0);
  const double S2 = wave_sum(lane < 16 ? e * e * w2[lane] : 0.0);
  if (lane != 0) return;
  const double E = S1 * S1 / ((double)ad.N * S2);
  uint32_t run, stage, active;
  if (ad.first) {
    run = 0u;
    stage = c->ad_next;
    active = (E < ad.theta) ? 1u : 0u;
  } else {
    run = c->ad_run + 1u;
    stage = (c->ad_stage + 1u) % ad.S;
    active = (E < ad.theta && run < ad.S) ? 1u : 0u;
    if (!active) c->ad_next = stage;
  }
  c->ad_run = run;
  c->ad_stage = stage;
  c->ad_active = active;
  ad.hist[ad.t % ad.hist_cap].stage = run;
}

// The mutation after the step's last stage: the gathered states (in place
// in x_in) propagate with the step's normals into x_out; the carried
// log-weights are copied along, and their maximum becomes the next step's
// offset.
template <int D, int MK>
__global__ void __launch_bounds__(256) pf_adapt_propagate(StepArgs<float, float> a) {
  using T = float;
  __shared__ T red[4];
  T wmax = -INFINITY;
  const int d = (int)a.d;
  const uint64_t N = a.N, npair = N >> 1;
  const uint32_t tau = a.t + 1u;
  for (uint64_t p = (uint64_t)blockIdx.x * 256u + threadIdx.x; p < npair; p += (uint64_t)gridDim.x * 256u) {
    const uint64_t i0 = 2u * p;
    T xh[2][D], z[2][D], xo[2][D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      xh[0][j] = xh[1][j] = 0;
      if (j < d) Pair<float, T>::load(a.x_in + (size_t)j * N + i0, xh[0][j], xh[1][j]);
      z[0][j] = z[1][j] = 0;
    }
    T u0, u1;
    pair_randoms<D, T>((uint32_t)p, tau, a.sid, a.k0, a.k1, d, u0, u1, z[0], z[1]);
    Model<D, MK, T>::propagate(a.mp, xh[0], z[0], xo[0]);
    Model<D, MK, T>::propagate(a.mp, xh[1], z[1], xo[1]);
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (j < d) Pair<float, T>::store(a.x_out + (size_t)j * N + i0, xo[0][j], xo[1][j]);
    T w0, w1;
    Pair<T, T>::load(a.lw_in + i0, w0, w1);
    Pair<T, T>::store(a.lw_out + i0, w0, w1);
    wmax = fmaxT(wmax, fmaxT(w0, w1));
  }
  wmax = block_max<T, 256>(wmax, red);
  if (threadIdx.x == 0)
    __hip_atomic_fetch_max(off_slot(a.ctl, a.u + 1, blockIdx.x % kOffSlots), ord_encode((double)wmax),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace pfk
