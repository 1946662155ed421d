// pf_launch.h - host-side dispatch from a launch request to a compiled
// kernel instantiation. Each dtype translation unit (pf_kernels_*.hip)
// instantiates PFK_DEFINE_LAUNCHER once.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "pf_kernels.h"

namespace pfk {

enum LaunchWhat : int {
  LW_INIT = 0,
  LW_STEP_TILE = 1,
  LW_GLOBAL_WEIGHT = 2,
  LW_GLOBAL_PREFIX = 3,
  LW_GLOBAL_DRAW = 4,
  LW_FINALIZE = 5,
  LW_FINALIZE_MULTI = 6,
  LW_FINALIZE_PREFIX = 7,
  LW_ISLAND_DRAW = 8,
  LW_ISLAND_GATHER = 9,
  LW_AD_WEIGHT = 10,
  LW_AD_STAGE = 11,
  LW_AD_DECIDE = 12,
  LW_AD_PROPAGATE = 13,
  LW_GLOBAL_SYS_DRAW = 14
};

// What the runtime asks for.
struct LaunchReq {
  int what;
  int D;         // compiled dimension (1, 2, 4, 8, 16)
  int mk;        // ModelKind
  int nt;        // threads per block
  int ppt;       // particle pairs per thread
  int blockpath; // tile kernels: 1 = r > 64
  int full;      // tile kernels: d equals the compiled dimension
  int island;    // tile kernels: the within-island launch of the island filter
  uint32_t grid;
  size_t lds;    // dynamic LDS bytes
  uint32_t tile_elems;  // global draw: particles per weight tile
  uint32_t nchunks;     // global draw: chunks of pairs the (persistent) grid works through
  // finalize (LW_FINALIZE): the step whose partials are reduced
  FinArgs fin;
  const void* fin_part;
  uint32_t fin_ntiles;
  // deferred reductions (LW_FINALIZE_MULTI / LW_FINALIZE_PREFIX)
  const FinMulti* fm;
  // island stages (LW_ISLAND_DRAW)
  const IslandArgs* ia;
  // ESS decisions (LW_AD_DECIDE)
  const AdDecide* ad;
};

// Pairs per thread of the butterfly wave path (256 threads) by dimension:
// keeps the registers held across the step (states, normals) bounded.
constexpr int ppt_wave(int D) { return D <= 2 ? 4 : 1; }
// Pairs per thread of the butterfly block path (256 threads): tiles of
// 512 PPT particles hold at least two groups of r <= 256 PPT.
constexpr int ppt_block(int D) { return D <= 2 ? 8 : (D <= 4 ? 4 : (D <= 8 ? 2 : 1)); }
// Pairs per thread of the global weight kernel (256 threads).
constexpr int ppt_gweight(int D) { return D <= 2 ? 8 : (D == 4 ? 4 : (D == 8 ? 2 : 1)); }
constexpr int kDrawPPT = 2;
// Threads per block of the systematic global draw: 512 where the registers
// allow two blocks per compute unit.
constexpr int sys_draw_nt(int D) { return D <= 2 ? 512 : 256; }
// Threads of the one-block global prefix kernel.
constexpr int kPrefixNT = 1024;
// LDS of the systematic global draw: d = 1, the tile's states; the output
// count below each CDF value; the tile's CDF, then the item's ancestor
// positions in the same space.
constexpr size_t sys_draw_lds(int D, size_t tsz, size_t ssz, uint32_t tile_elems) {
  const size_t cdf = (size_t)tile_elems * tsz, pos = (size_t)kSysItem * 2u;
  return (D == 1 ? (size_t)tile_elems * ssz : 0u) + (size_t)tile_elems * 2u + (cdf > pos ? cdf : pos);
}
// Blocks of the persistent global draw: four per compute unit of MI355X.
constexpr uint32_t kDrawBlocks = 1024;

template <typename K> static hipError_t ensure_lds(K* kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// The fused step kernel for the request's tile shape.
template <int D, int MK, typename T, typename S, bool FULL>
static hipError_t launch_step_tile(const LaunchReq& rq, const StepArgs<T, S>& a, hipStream_t st) {
  if (!rq.blockpath) {
    if (rq.nt == 256 && rq.ppt == ppt_wave(D)) {
      auto k = pf_step_tile<D, MK, T, S, 256, ppt_wave(D), false, FULL>;
      hipError_t e = ensure_lds(k, rq.lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, dim3(rq.grid), dim3(256), rq.lds, st, a);
      return hipGetLastError();
    }
    if (rq.nt == 64 && rq.ppt == 1) {
      auto k = pf_step_tile<D, MK, T, S, 64, 1, false, FULL>;
      hipError_t e = ensure_lds(k, rq.lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, dim3(rq.grid), dim3(64), rq.lds, st, a);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  if (rq.nt == 256 && rq.ppt == ppt_block(D)) {
    auto k = pf_step_tile<D, MK, T, S, 256, ppt_block(D), true, FULL>;
    hipError_t e = ensure_lds(k, rq.lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(rq.grid), dim3(256), rq.lds, st, a);
    return hipGetLastError();
  }
  if constexpr (D <= 2) {
    if (rq.nt == 256 && rq.ppt == 4) {
      auto k = pf_step_tile<D, MK, T, S, 256, 4, true, FULL>;
      hipError_t e = ensure_lds(k, rq.lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, dim3(rq.grid), dim3(256), rq.lds, st, a);
      return hipGetLastError();
    }
    if (rq.nt == 256 && rq.ppt == 2) {
      auto k = pf_step_tile<D, MK, T, S, 256, 2, true, FULL>;
      hipError_t e = ensure_lds(k, rq.lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, dim3(rq.grid), dim3(256), rq.lds, st, a);
      return hipGetLastError();
    }
  }
  if (rq.nt == 256 && rq.ppt == 1) {
    auto k = pf_step_tile<D, MK, T, S, 256, 1, true, FULL>;
    hipError_t e = ensure_lds(k, rq.lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(rq.grid), dim3(256), rq.lds, st, a);
    return hipGetLastError();
  }
  if (rq.nt == 1024 && rq.ppt == 1) {
    auto k = rq.island ? pf_step_tile<D, MK, T, S, 1024, 1, true, FULL, true>
                       : pf_step_tile<D, MK, T, S, 1024, 1, true, FULL>;
    hipError_t e = ensure_lds(k, rq.lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(rq.grid), dim3(1024), rq.lds, st, a);
    return hipGetLastError();
  }
  if constexpr (D <= 4) {
    if (rq.nt == 1024 && rq.ppt == 2) {
      auto k = rq.island ? pf_step_tile<D, MK, T, S, 1024, 2, true, FULL, true>
                       : pf_step_tile<D, MK, T, S, 1024, 2, true, FULL>;
      hipError_t e = ensure_lds(k, rq.lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, dim3(rq.grid), dim3(1024), rq.lds, st, a);
      return hipGetLastError();
    }
    if (rq.nt == 1024 && rq.ppt == 4) {
      auto k = rq.island ? pf_step_tile<D, MK, T, S, 1024, 4, true, FULL, true>
                       : pf_step_tile<D, MK, T, S, 1024, 4, true, FULL>;
      hipError_t e = ensure_lds(k, rq.lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, dim3(rq.grid), dim3(1024), rq.lds, st, a);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

template <int D, int MK, typename T, typename S>
static hipError_t launch_model(const LaunchReq& rq, const StepArgs<T, S>& a, hipStream_t st) {
  switch (rq.what) {
    case LW_INIT: {
      hipLaunchKernelGGL((pf_init_kernel<D, MK, T, S>), dim3(rq.grid), dim3(256), 0, st, a);
      return hipGetLastError();
    }
    case LW_STEP_TILE:
      return launch_step_tile<D, MK, T, S, false>(rq, a, st);
    case LW_GLOBAL_WEIGHT: {
      if (rq.nt == 256 && rq.ppt == ppt_gweight(D)) {
        hipLaunchKernelGGL((pf_global_weight<D, MK, T, S, 256, ppt_gweight(D)>), dim3(rq.grid),
                           dim3(256), 0, st, a);
        return hipGetLastError();
      }
      if (rq.nt == 64 && rq.ppt == 1) {
        hipLaunchKernelGGL((pf_global_weight<D, MK, T, S, 64, 1>), dim3(rq.grid), dim3(64), 0, st, a);
        return hipGetLastError();
      }
      return hipErrorInvalidValue;
    }
    case LW_GLOBAL_PREFIX: {
      auto k = pf_global_prefix<D, T, S, kPrefixNT>;
      hipError_t e = ensure_lds(k, rq.lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, dim3(1), dim3(kPrefixNT), rq.lds, st, a);
      return hipGetLastError();
    }
    case LW_FINALIZE_MULTI: {
      hipLaunchKernelGGL((pf_finalize_multi<D, T, 512>), dim3(rq.fm->n), dim3(512), 0, st, *rq.fm);
      return hipGetLastError();
    }
    case LW_FINALIZE_PREFIX: {
      hipLaunchKernelGGL((pf_finalize_prefix<T>), dim3(1), dim3(64), 0, st, *rq.fm);
      return hipGetLastError();
    }
    case LW_FINALIZE: {
      hipLaunchKernelGGL((pf_finalize_kernel<D, T, 512>), dim3(1), dim3(512), 0, st, rq.fin,
                         reinterpret_cast<const T*>(rq.fin_part), rq.fin_ntiles);
      return hipGetLastError();
    }
    case LW_AD_WEIGHT:
    case LW_AD_STAGE:
    case LW_AD_DECIDE:
    case LW_AD_PROPAGATE:
      if constexpr (std::is_same<T, float>::value && std::is_same<S, float>::value) {
        if (rq.what == LW_AD_WEIGHT) {
          hipLaunchKernelGGL((pf_adapt_weight<D, MK, false>), dim3(rq.grid), dim3(256), 0, st, a);
        } else if (rq.what == LW_AD_STAGE && rq.nt == 64) {
          // small N: the 64-thread tiles of the wave path
          hipLaunchKernelGGL((pf_adapt_stage<D, MK, 64, 1, false>), dim3(rq.grid), dim3(64), rq.lds, st, a);
        } else if (rq.what == LW_AD_STAGE) {
          auto k = pf_adapt_stage<D, MK, 256, ppt_wave(D), false>;
          hipError_t e = ensure_lds(k, rq.lds);
          if (e != hipSuccess) return e;
          hipLaunchKernelGGL(k, dim3(rq.grid), dim3(256), rq.lds, st, a);
        } else if (rq.what == LW_AD_DECIDE) {
          hipLaunchKernelGGL(pf_adapt_decide<float>, dim3(1), dim3(1024), 0, st, *rq.ad);
        } else {
          hipLaunchKernelGGL((pf_adapt_propagate<D, MK>), dim3(rq.grid), dim3(256), 0, st, a);
        }
        return hipGetLastError();
      }
      return hipErrorInvalidValue;
    case LW_ISLAND_DRAW: {
      auto k = pf_island_draw<T>;
      hipError_t e = ensure_lds(k, rq.lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, dim3(rq.grid), dim3(rq.nt), rq.lds, st, *rq.ia);
      return hipGetLastError();
    }
    case LW_ISLAND_GATHER: {
      if (rq.lds > 0) {
        // one block per destination island, its source island staged in LDS
        // (islands of 1024 ppt particles)
        auto k = rq.ppt == 1 ? pf_island_gather_lds<D, MK, T, S, 1>
                             : (rq.ppt == 2 ? pf_island_gather_lds<D, MK, T, S, 2> : pf_island_gather_lds<D, MK, T, S, 4>);
        if (rq.ppt != 1 && rq.ppt != 2 && rq.ppt != 4) return hipErrorInvalidValue;
        hipError_t e = ensure_lds(k, rq.lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3(rq.grid), dim3(kIslandGatherNT), rq.lds, st, a);
      } else {
        hipLaunchKernelGGL((pf_island_gather<D, MK, T, S>), dim3(rq.grid), dim3(256), 0, st, a);
      }
      return hipGetLastError();
    }
    case LW_GLOBAL_SYS_DRAW: {
      auto k = pf_global_sys_draw<D, MK, T, S, sys_draw_nt(D)>;
      hipError_t e = ensure_lds(k, rq.lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, dim3(rq.grid), dim3(sys_draw_nt(D)), rq.lds, st, a, rq.tile_elems);
      return hipGetLastError();
    }
    case LW_GLOBAL_DRAW: {
      auto k = pf_global_draw<D, MK, T, S, 256, kDrawPPT>;
      hipError_t e = ensure_lds(k, rq.lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, dim3(rq.grid), dim3(256), rq.lds, st, a, rq.tile_elems, rq.nchunks);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

template <typename T, typename S>
static hipError_t launch_any(const LaunchReq& rq, const void* args, hipStream_t st) {
  const StepArgs<T, S>& a = *reinterpret_cast<const StepArgs<T, S>*>(args);
  if (rq.mk == MK_SV) {
    if (rq.D != 1) return hipErrorInvalidValue;
    return launch_model<1, MK_SV, T, S>(rq, a, st);
  }
#define PFK_DIMS(MKV)                                                \
  switch (rq.D) {                                                    \
    case 1: return launch_model<1, MKV, T, S>(rq, a, st);            \
    case 2: return launch_model<2, MKV, T, S>(rq, a, st);            \
    case 4: return launch_model<4, MKV, T, S>(rq, a, st);            \
    case 8: return launch_model<8, MKV, T, S>(rq, a, st);            \
    case 16: return launch_model<16, MKV, T, S>(rq, a, st);          \
    default: return hipErrorInvalidValue;                            \
  }
  if (rq.mk == MK_LG_DENSE) { PFK_DIMS(MK_LG_DENSE) }
  if (rq.mk == MK_LG_DIAG) { PFK_DIMS(MK_LG_DIAG) }
#undef PFK_DIMS
  return hipErrorInvalidValue;
}

// Batched filters (FP32): the step kernel of one (D, model kind, PPT) class
// or its finalize kernel.
struct BatchReq {
  int finalize;  // 0: step tiles, 1: reductions
  int D, mk, ppt;
  int full;      // every filter of the class has d = D
  uint32_t grid;
  size_t lds;
};
constexpr int kBatchNT = 256;
// Pairs per thread of the batched tiles (E = 512 PPT particles per tile).
constexpr bool batch_ppt_ok(int D, int ppt) { return ppt == 1 || (ppt == 2 && D <= 8); }

template <int D, int MK, bool FULL>
static hipError_t launch_batch_tiles(const BatchReq& rq, const BatchArgs& a, hipStream_t st) {
  if (rq.ppt == 1) {
    auto k = pf_batch_tile<D, MK, kBatchNT, 1, FULL>;
    hipError_t e = ensure_lds(k, rq.lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(rq.grid), dim3(kBatchNT), rq.lds, st, a);
    return hipGetLastError();
  }
  if constexpr (D <= 8) {
    if (rq.ppt == 2) {
      auto k = pf_batch_tile<D, MK, kBatchNT, 2, FULL>;
      hipError_t e = ensure_lds(k, rq.lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, dim3(rq.grid), dim3(kBatchNT), rq.lds, st, a);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

template <int D, int MK>
static hipError_t launch_batch_model(const BatchReq& rq, const BatchArgs& a, hipStream_t st) {
  if (rq.finalize) {
    hipLaunchKernelGGL((pf_batch_finalize<D, kBatchNT>), dim3(rq.grid), dim3(kBatchNT), 0, st, a);
    return hipGetLastError();
  }
  return rq.full ? launch_batch_tiles<D, MK, true>(rq, a, st) : launch_batch_tiles<D, MK, false>(rq, a, st);
}

hipError_t launch_batch(const BatchReq& rq, const BatchArgs& a, hipStream_t st);

// Step-tile launches with d = D (instantiated in their own translation unit).
template <typename T, typename S>
static hipError_t launch_full_any(const LaunchReq& rq, const void* args, hipStream_t st) {
  const StepArgs<T, S>& a = *reinterpret_cast<const StepArgs<T, S>*>(args);
  if (rq.mk == MK_SV) return rq.D == 1 ? launch_step_tile<1, MK_SV, T, S, true>(rq, a, st) : hipErrorInvalidValue;
#define PFK_FULL_DIMS(MKV)                                                   \
  switch (rq.D) {                                                            \
    case 1: return launch_step_tile<1, MKV, T, S, true>(rq, a, st);          \
    case 2: return launch_step_tile<2, MKV, T, S, true>(rq, a, st);          \
    case 4: return launch_step_tile<4, MKV, T, S, true>(rq, a, st);          \
    case 8: return launch_step_tile<8, MKV, T, S, true>(rq, a, st);          \
    case 16: return launch_step_tile<16, MKV, T, S, true>(rq, a, st);        \
    default: return hipErrorInvalidValue;                                    \
  }
  if (rq.mk == MK_LG_DENSE) { PFK_FULL_DIMS(MK_LG_DENSE) }
  if (rq.mk == MK_LG_DIAG) { PFK_FULL_DIMS(MK_LG_DIAG) }
#undef PFK_FULL_DIMS
  return hipErrorInvalidValue;
}
hipError_t launch_f32_full(const LaunchReq& rq, const void* args, hipStream_t st);

// Entry points of the three dtype translation units.
hipError_t launch_f32(const LaunchReq& rq, const void* args, hipStream_t st);
hipError_t launch_bf16(const LaunchReq& rq, const void* args, hipStream_t st);
hipError_t launch_f64(const LaunchReq& rq, const void* args, hipStream_t st);

}  // namespace pfk
