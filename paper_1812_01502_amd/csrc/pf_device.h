// pf_device.h - device-side building blocks of the butterfly particle filter
// (gfx950, wave64): counter-based random numbers, model functions, storage
// conversions, wave-level primitives and the per-step control block.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pf.h"

namespace pfk {

constexpr int kMaxDim = PF_MAX_DIM;

// Model variants compiled into the kernels.
enum ModelKind : int {
  MK_LG_DENSE = 0,  // general linear-Gaussian model
  MK_LG_DIAG = 1,   // LG with H = I and diagonal noise factors
  MK_SV = 2         // stochastic volatility
};

// ---------------------------------------------------------------------------
// Storage of particle states.
// ---------------------------------------------------------------------------
struct bf16 {
  uint16_t bits;
};

template <typename S> struct StoragePair;
template <> struct StoragePair<float> { using type = float2; };
template <> struct StoragePair<double> { using type = double2; };
template <> struct StoragePair<bf16> { using type = uint32_t; };

template <typename T> __device__ __forceinline__ T to_compute(float v) { return (T)v; }

// Round-to-nearest-even FP32 -> BF16 (finite inputs).
__device__ __forceinline__ uint32_t f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf16_bits_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

template <typename S, typename T> struct Pair;
template <typename T> struct Pair<float, T> {
  static __device__ __forceinline__ void load(const float* p, T& a, T& b) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    a = (T)v.x;
    b = (T)v.y;
  }
  static __device__ __forceinline__ void store(float* p, T a, T b) {
    *reinterpret_cast<float2*>(p) = make_float2((float)a, (float)b);
  }
};
template <typename T> struct Pair<double, T> {
  static __device__ __forceinline__ void load(const double* p, T& a, T& b) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    a = (T)v.x;
    b = (T)v.y;
  }
  static __device__ __forceinline__ void store(double* p, T a, T b) {
    *reinterpret_cast<double2*>(p) = make_double2((double)a, (double)b);
  }
};
template <typename T> struct Pair<bf16, T> {
  static __device__ __forceinline__ void load(const bf16* p, T& a, T& b) {
    const uint32_t v = *reinterpret_cast<const uint32_t*>(p);
    a = (T)bf16_bits_to_f32(v & 0xFFFFu);
    b = (T)bf16_bits_to_f32(v >> 16);
  }
  static __device__ __forceinline__ void store(bf16* p, T a, T b) {
    *reinterpret_cast<uint32_t*>(p) = f32_to_bf16_bits((float)a) | (f32_to_bf16_bits((float)b) << 16);
  }
};
template <typename S, typename T> struct Single;
template <typename T> struct Single<float, T> {
  static __device__ __forceinline__ T load(const float* p) { return (T)*p; }
  static __device__ __forceinline__ float cvt(T v) { return (float)v; }
};
template <typename T> struct Single<double, T> {
  static __device__ __forceinline__ T load(const double* p) { return (T)*p; }
  static __device__ __forceinline__ double cvt(T v) { return (double)v; }
};
template <typename T> struct Single<bf16, T> {
  static __device__ __forceinline__ T load(const bf16* p) {
    return (T)bf16_bits_to_f32(*reinterpret_cast<const uint16_t*>(p));
  }
  static __device__ __forceinline__ bf16 cvt(T v) {
    const uint16_t b = (uint16_t)f32_to_bf16_bits((float)v);
    bf16 r;
    __builtin_memcpy(&r, &b, 2);
    return r;
  }
};

// ---------------------------------------------------------------------------
// Fast transcendental functions. FP32 uses the hardware exp2/log2/sqrt and the
// revolution-scaled sin/cos; FP64 uses the device math library.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fexp(float x) { return __expf(x); }
__device__ __forceinline__ double fexp(double x) { return exp(x); }
__device__ __forceinline__ float flog(float x) { return __logf(x); }
__device__ __forceinline__ double flog(double x) { return log(x); }
// ln x for x >= 1 (a group's weight total relative to its largest member):
// the hardware log2 needs no denormal scaling there.
__device__ __forceinline__ float flog_ge1(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945f; }
__device__ __forceinline__ double flog_ge1(double x) { return log(x); }
__device__ __forceinline__ float fmaxT(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double fmaxT(double a, double b) { return fmax(a, b); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from the
// published round function: per round the products M0*c0 and M1*c2 (32x32 ->
// 64 bit) give (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key advances by
// the Weyl increments between rounds.
// ---------------------------------------------------------------------------
struct Words {
  uint32_t w0, w1, w2, w3;
};

// a ^ b ^ c as one instruction: the three-input bitwise operation of gfx950
// with truth table 0x96. `c` is wave-uniform (a key word).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}

// Every caller passes wave-uniform counter words c1, c2, c3 (step, block,
// stream) and a per-lane c0 (the pair). The first rounds then mix uniform
// words, which the compiler folds into scalar operations; from the third
// round on (the second output word: the fourth) both XOR inputs vary per lane,
// and the two XORs of each output word are one instruction.
__device__ __forceinline__ Words philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t h0 = (uint32_t)(p0 >> 32), h1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = i >= 2 ? xor3(h1, c1, k0) : h1 ^ c1 ^ k0;
    const uint32_t n2 = i >= 3 ? xor3(h0, c3, k1) : h0 ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Words{c0, c1, c2, c3};
}

// 24-bit uniform in [0, 1): exact in FP32 and FP64.
template <typename T> __device__ __forceinline__ T word_uniform(uint32_t w);
template <> __device__ __forceinline__ float word_uniform<float>(uint32_t w) {
  return (float)(w >> 8) * 0x1p-24f;
}
template <> __device__ __forceinline__ double word_uniform<double>(uint32_t w) {
  return (double)(w >> 8) * 0x1p-24;
}

// Box-Muller: u1 = ((wa >> 8) + 1) 2^-24 in (0, 1], u2 = (wb >> 8) 2^-24;
// cosine branch -> first particle of the pair, sine branch -> second.
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& zc, float& zs) {
  const float u1 = (float)((wa >> 8) + 1u) * 0x1p-24f;
  const float u2 = (float)(wb >> 8) * 0x1p-24f;
  // -2 ln u1 = -2 ln(2) log2(u1), at least about 1.2e-7 (never denormal), so
  // the hardware square root (1 ulp) needs none of the scaling and
  // correction steps of the correctly rounded one
  const float rho = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
  // the hardware sin/cos take their argument in revolutions: sin(2 pi u2)
  zc = rho * __builtin_amdgcn_cosf(u2);
  zs = rho * __builtin_amdgcn_sinf(u2);
}
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double& zc, double& zs) {
  const double u1 = (double)((wa >> 8) + 1u) * 0x1p-24;
  const double u2 = (double)(wb >> 8) * 0x1p-24;
  const double rho = sqrt(-2.0 * log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  zc = rho * c;
  zs = rho * s;
}

// Block 0 of pair p: the resampling uniforms (u0, u1) of the pair's two
// particles and their dimension-0 normals (z0, z1).
template <typename T>
__device__ __forceinline__ void pair_block0(uint32_t p, uint32_t tau, uint32_t sid, uint32_t k0,
                                            uint32_t k1, T& u0, T& u1, T& z0, T& z1) {
  const Words b0 = philox(p, tau, 0u, sid, k0, k1);
  u0 = word_uniform<T>(b0.w0);
  u1 = word_uniform<T>(b0.w1);
  box_muller(b0.w2, b0.w3, z0, z1);
}

// Blocks b >= 1 of pair p: normals of dimensions 2b-1 and 2b (< d) of both
// particles; entries j >= d and j = 0 are left untouched.
template <int D, typename T>
__device__ __forceinline__ void pair_normals_rest(uint32_t p, uint32_t tau, uint32_t sid, uint32_t k0,
                                                  uint32_t k1, int d, T (&z0)[D], T (&z1)[D]) {
#pragma unroll
  for (int b = 1; 2 * b - 1 < D; ++b) {
    if (2 * b - 1 < d) {
      const Words w = philox(p, tau, (uint32_t)b, sid, k0, k1);
      box_muller(w.w0, w.w1, z0[2 * b - 1], z1[2 * b - 1]);
      if (2 * b < D && 2 * b < d) box_muller(w.w2, w.w3, z0[2 * b], z1[2 * b]);
    }
  }
}

// Uniforms and all normals of pair p (counter (p, tau, block, stream)).
template <int D, typename T>
__device__ __forceinline__ void pair_randoms(uint32_t p, uint32_t tau, uint32_t sid, uint32_t k0,
                                             uint32_t k1, int d, T& u0, T& u1, T (&z0)[D],
                                             T (&z1)[D]) {
  pair_block0<T>(p, tau, sid, k0, k1, u0, u1, z0[0], z1[0]);
  pair_normals_rest<D, T>(p, tau, sid, k0, k1, d, z0, z1);
}

// Normals only (prior draws at tau = 0).
template <int D, typename T>
__device__ __forceinline__ void pair_normals(uint32_t p, uint32_t tau, uint32_t sid, uint32_t k0,
                                             uint32_t k1, int d, T (&z0)[D], T (&z1)[D]) {
  T u0, u1;
  pair_randoms<D, T>(p, tau, sid, k0, k1, d, u0, u1, z0, z1);
}

// ---------------------------------------------------------------------------
// Model parameters (device memory, zero-padded to kMaxDim so that padded
// components stay exactly zero through every formula).
// ---------------------------------------------------------------------------
template <typename T> struct ModelParams {
  T A[kMaxDim * kMaxDim];    // transition matrix
  T Lq[kMaxDim * kMaxDim];   // lower Cholesky factor of Q
  T H[kMaxDim * kMaxDim];    // observation matrix
  T Li[kMaxDim * kMaxDim];   // inverse of the lower Cholesky factor of R
  T L0[kMaxDim * kMaxDim];   // lower Cholesky factor of P0
  T m0[kMaxDim];
  T qd[kMaxDim];             // diag(Lq)   (diagonal variant)
  T lid[kMaxDim];            // diag(Li)   (diagonal variant)
  T lconst;                  // normalising constant of log g
  T phi, sigma, inv2b2, sd0; // SV
};

template <int D, int MK, typename T> struct Model;

template <int D, typename T> struct Model<D, MK_LG_DENSE, T> {
  static __device__ __forceinline__ T log_g(const ModelParams<T>* __restrict__ P, const T (&x)[D],
                                            const T (&y)[D]) {
    T e[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T hx = 0;
#pragma unroll
      for (int k = 0; k < D; ++k) hx += P->H[j * kMaxDim + k] * x[k];
      e[j] = y[j] - hx;
    }
    T qf = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T u = 0;
#pragma unroll
      for (int k = 0; k <= j; ++k) u += P->Li[j * kMaxDim + k] * e[k];
      qf += u * u;
    }
    return P->lconst - (T)0.5 * qf;
  }
  // component j of f(xh, z): needs z[0..j] (Lq is lower-triangular)
  static __device__ __forceinline__ T row(const ModelParams<T>* __restrict__ P, const T (&xh)[D],
                                          const T (&z)[D], const int j) {
    T v = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) v += P->A[j * kMaxDim + k] * xh[k];
#pragma unroll
    for (int k = 0; k < D; ++k)
      if (k <= j) v += P->Lq[j * kMaxDim + k] * z[k];
    return v;
  }
  static __device__ __forceinline__ void propagate(const ModelParams<T>* __restrict__ P,
                                                   const T (&xh)[D], const T (&z)[D], T (&xo)[D]) {
#pragma unroll
    for (int j = 0; j < D; ++j) xo[j] = row(P, xh, z, j);
  }
  static __device__ __forceinline__ void prior(const ModelParams<T>* __restrict__ P, const T (&z)[D],
                                               T (&xo)[D]) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T v = P->m0[j];
#pragma unroll
      for (int k = 0; k <= j; ++k) v += P->L0[j * kMaxDim + k] * z[k];
      xo[j] = v;
    }
  }
};

template <int D, typename T> struct Model<D, MK_LG_DIAG, T> {
  static __device__ __forceinline__ T log_g(const ModelParams<T>* __restrict__ P, const T (&x)[D],
                                            const T (&y)[D]) {
    T qf = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const T u = (y[j] - x[j]) * P->lid[j];
      qf += u * u;
    }
    return P->lconst - (T)0.5 * qf;
  }
  // component j of f(xh, z): needs z[j] only. Explicit FMAs: a sum of two
  // products could otherwise be fused on either one, and two kernels holding
  // this code could round differently.
  static __device__ __forceinline__ T row(const ModelParams<T>* __restrict__ P, const T (&xh)[D],
                                          const T (&z)[D], const int j) {
    T v = P->qd[j] * z[j];
#pragma unroll
    for (int k = 0; k < D; ++k) v = fmaT(P->A[j * kMaxDim + k], xh[k], v);
    return v;
  }
  static __device__ __forceinline__ void propagate(const ModelParams<T>* __restrict__ P,
                                                   const T (&xh)[D], const T (&z)[D], T (&xo)[D]) {
#pragma unroll
    for (int j = 0; j < D; ++j) xo[j] = row(P, xh, z, j);
  }
  static __device__ __forceinline__ void prior(const ModelParams<T>* __restrict__ P, const T (&z)[D],
                                               T (&xo)[D]) {
    Model<D, MK_LG_DENSE, T>::prior(P, z, xo);
  }
};

template <int D, typename T> struct Model<D, MK_SV, T> {
  static_assert(D == 1, "the SV model is one-dimensional");
  static __device__ __forceinline__ T log_g(const ModelParams<T>* __restrict__ P, const T (&x)[D],
                                            const T (&y)[D]) {
    return P->lconst - (T)0.5 * x[0] - y[0] * y[0] * fexp(-x[0]) * P->inv2b2;
  }
  static __device__ __forceinline__ T row(const ModelParams<T>* __restrict__ P, const T (&xh)[D],
                                          const T (&z)[D], const int) {
    return fmaT(P->phi, xh[0], P->sigma * z[0]);
  }
  static __device__ __forceinline__ void propagate(const ModelParams<T>* __restrict__ P,
                                                   const T (&xh)[D], const T (&z)[D], T (&xo)[D]) {
    xo[0] = row(P, xh, z, 0);
  }
  static __device__ __forceinline__ void prior(const ModelParams<T>* __restrict__ P, const T (&z)[D],
                                               T (&xo)[D]) {
    xo[0] = P->sd0 * z[0];
  }
};

// ---------------------------------------------------------------------------
// Per-handle control block in device memory.
// ---------------------------------------------------------------------------
// The maximum of the new log-weights of a step (the offset subtracted at the
// next load) is gathered in kOffSlots slots, one cache line apart, so that
// the tiles' atomicMax operations spread over memory channels; a ring of 3
// steps lets the offset of step t be read while step t+1's is gathered and
// step t+2's slots are cleared.
constexpr int kOffSlots = 32;
constexpr int kOffStride = 16;   // 16 x 8 B = one 128-B line per slot
constexpr int kOffRing = 3;
constexpr int kOffEntries = kOffRing * kOffSlots * kOffStride;
// Steps whose reductions may be deferred and done together.
constexpr int kMaxPending = 64;

constexpr uint32_t kNoFail = 0xFFFFFFFFu;
struct Ctl {
  double log_norm;           // running log-normaliser (FP64)
  uint32_t t;                // steps reduced so far (diagnostic)
  // ESS-gated stages: the next stage slot runs (ad_active), the stage it
  // runs, stages run so far in the step, the stage the next step starts at
  uint32_t ad_active, ad_stage, ad_run, ad_next;
  // the first step whose weights were unusable (a non-finite partial sum,
  // or no positive weight), kNoFail if none: that step and every later one
  // are invalid; reset by the initialisation and by state uploads
  uint32_t fail_t;
  uint32_t pad[8];
  long long offs[kOffEntries];  // encoded maxima, [ring][slot * stride]
  double step_off[kMaxPending]; // offset step t subtracted, at t mod kMaxPending
  double dlog[kMaxPending];     // log-normaliser increments of deferred reductions
};

// Per-tile partial record: [m, S, sw2, swin, A1[D], A2[D], sh[D]].
__host__ __device__ constexpr int partial_stride(int D) { return 4 + 3 * D; }

// ---------------------------------------------------------------------------
// Wave-level helpers (wave64). FP32 reductions use DPP lane moves (VALU)
// instead of LDS-routed shuffles: xor-1, xor-2 quad permutes, half-row and
// row mirrors (16-lane rows), then row broadcasts 15 and 31; the total ends
// in lane 63 and is broadcast with readlane.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                                ROW_MASK, 0xF, false));
}
constexpr int kDppQuadXor1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

// Lane move with every lane's source valid (quad permutes, mirrors): no old
// value, so the compiler can fuse it into the consuming add or max.
template <int CTRL> __device__ __forceinline__ float dppm(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<kDppQuadXor1>(v);
  v += dpp_f<kDppQuadXor2>(v);
  v += dpp_f<kDppRowHalfMirror>(v);
  v += dpp_f<kDppRowMirror>(v);
  v += dpp_f<kDppRowBcast15, 0xA>(v);
  v += dpp_f<kDppRowBcast31, 0xC>(v);
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ float wave_max(float v) {
  // disabled rows of the broadcasts receive 0 from update_dpp: use the
  // identity -inf explicitly there
  v = fmaxf(v, dpp_f<kDppQuadXor1>(v));
  v = fmaxf(v, dpp_f<kDppQuadXor2>(v));
  v = fmaxf(v, dpp_f<kDppRowHalfMirror>(v));
  v = fmaxf(v, dpp_f<kDppRowMirror>(v));
  const int lane = __lane_id();
  float b15 = dpp_f<kDppRowBcast15, 0xA>(v);
  if (((lane >> 4) & 1) == 0) b15 = v;
  v = fmaxf(v, b15);
  float b31 = dpp_f<kDppRowBcast31, 0xC>(v);
  if ((lane >> 5) == 0) b31 = v;
  v = fmaxf(v, b31);
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
// FP64 lane moves: the two 32-bit halves move with the same DPP control.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW_MASK, 0xF, false);
  const unsigned hi =
      (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW_MASK, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<kDppQuadXor1>(v);
  v += dpp_d<kDppQuadXor2>(v);
  v += dpp_d<kDppRowHalfMirror>(v);
  v += dpp_d<kDppRowMirror>(v);
  v += dpp_d<kDppRowBcast15, 0xA>(v);
  v += dpp_d<kDppRowBcast31, 0xC>(v);
  return readlane_d(v, 63);
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_d<kDppQuadXor1>(v));
  v = fmax(v, dpp_d<kDppQuadXor2>(v));
  v = fmax(v, dpp_d<kDppRowHalfMirror>(v));
  v = fmax(v, dpp_d<kDppRowMirror>(v));
  const int lane = __lane_id();
  double b15 = dpp_d<kDppRowBcast15, 0xA>(v);
  if (((lane >> 4) & 1) == 0) b15 = v;
  v = fmax(v, b15);
  double b31 = dpp_d<kDppRowBcast31, 0xC>(v);
  if ((lane >> 5) == 0) b31 = v;
  v = fmax(v, b31);
  return readlane_d(v, 63);
}
// Inclusive prefix sum over the 64 lanes.
template <typename T> __device__ __forceinline__ T wave_incl_scan(T v, int lane) {
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) {
    const T o = __shfl_up(v, (unsigned)s, 64);
    if (lane >= s) v += o;
  }
  return v;
}

}  // namespace pfk
