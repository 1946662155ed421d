// pf_host.h - host-side helpers shared by the single-filter and the batched
// runtimes: stage plans, model validation and upload, the LDS pad choice.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pf.h"
#include "pf_launch.h"

namespace pfh {

using namespace pfk;

// Device memory of handles and batches: hipMalloc/hipFree, or the callbacks
// installed by pf_set_allocator. A handle or batch keeps the allocator that
// was current when it was created and frees every buffer with it.
struct DevAllocator {
  void* (*alloc)(size_t, void*) = nullptr;  // nullptr: hipMalloc
  void (*free_)(void*, void*) = nullptr;
  void* ctx = nullptr;
};
// The allocator pf_set_allocator installed (defined in pf_runtime.hip).
DevAllocator current_allocator();
// Pointers handed out by an allocator callback must be aligned to this many
// bytes (vector loads of the state planes, 64-bit atomics of the control
// block).
constexpr uintptr_t kAllocAlign = 256;

// Allocate `bytes` (at least 16) of device memory with `a`. Returns
// hipSuccess, or hipErrorOutOfMemory when the allocator gave nothing,
// hipErrorInvalidValue when it gave a misaligned pointer (which is then
// returned to it).
inline hipError_t dev_alloc(const DevAllocator& a, void** p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (!a.alloc) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      *p = nullptr;
      (void)hipGetLastError();
    }
    return e;
  }
  *p = a.alloc(bytes, a.ctx);
  if (!*p) return hipErrorOutOfMemory;
  if ((reinterpret_cast<uintptr_t>(*p) & (kAllocAlign - 1)) != 0) {
    a.free_(*p, a.ctx);
    *p = nullptr;
    return hipErrorInvalidValue;
  }
  return hipSuccess;
}
inline void dev_free(const DevAllocator& a, void* p) {
  if (!p) return;
  if (a.free_) a.free_(p, a.ctx);
  else (void)hipFree(p);
}

// Row pitch of a tile's staged states in LDS: at strides below the tile
// width consecutive particles fall in consecutive rows, so an odd pitch keeps
// their writes in different banks; wider strides write along rows.
inline uint32_t state_row_pitch(uint32_t C, uint32_t log2R, uint32_t log2C) {
  return log2R < log2C ? C + 1u : C;
}

struct StagePlan {
  uint32_t r, log2r;
  uint64_t R;
  uint32_t log2R;
  // tile kernel geometry
  int blockpath, nt, ppt;
  uint32_t C, log2C, pad, ntiles, xrow;
  size_t lds;
};

inline bool is_pow2(uint64_t v) { return v && !(v & (v - 1)); }
inline uint32_t ilog2(uint64_t v) {
  uint32_t l = 0;
  while ((1ull << l) < v) ++l;
  return l;
}

inline bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// FNV-1a over the bytes of the model's parameters: a checkpoint may only be
// loaded into a handle of the same model.
inline uint64_t model_hash(const pf_model* m) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* b = reinterpret_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
      h ^= b[i];
      h *= 1099511628211ull;
    }
  };
  mix(&m->kind, sizeof(m->kind));
  mix(&m->d, sizeof(m->d));
  const size_t dd = (size_t)m->d * m->d;
  if (m->kind == PF_MODEL_LG) {
    for (const double* a : {m->A, m->Q_chol, m->H, m->R_chol, m->P0_chol}) mix(a, dd * sizeof(double));
    mix(m->m0, (size_t)m->d * sizeof(double));
  } else {
    mix(&m->phi, sizeof(double));
    mix(&m->sigma, sizeof(double));
    mix(&m->beta, sizeof(double));
  }
  return h;
}

// Inverse of a lower-triangular matrix (row-major d x d), FP64.
inline void lower_inverse(const double* L, int d, double* out) {
  for (int i = 0; i < d * d; ++i) out[i] = 0.0;
  for (int j = 0; j < d; ++j) {
    out[j * d + j] = 1.0 / L[j * d + j];
    for (int i = j + 1; i < d; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[i * d + k] * out[k * d + j];
      out[i * d + j] = -s / L[i * d + i];
    }
  }
}

template <typename T>
inline void fill_params(const pf_model* m, int d, ModelParams<T>* P, int* mk_out) {
  std::memset(P, 0, sizeof(*P));
  if (m->kind == PF_MODEL_SV) {
    P->phi = (T)m->phi;
    P->sigma = (T)m->sigma;
    P->inv2b2 = (T)(1.0 / (2.0 * m->beta * m->beta));
    P->sd0 = (T)(m->sigma / std::sqrt(1.0 - m->phi * m->phi));
    P->lconst = (T)(-0.5 * std::log(2.0 * M_PI * m->beta * m->beta));
    *mk_out = MK_SV;
    return;
  }
  std::vector<double> Li(d * d);
  lower_inverse(m->R_chol, d, Li.data());
  double logdet = 0.0;
  for (int j = 0; j < d; ++j) logdet += std::log(m->R_chol[j * d + j]);
  P->lconst = (T)(-logdet - 0.5 * d * std::log(2.0 * M_PI));
  bool diag = true;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      const double hij = m->H[i * d + j];
      if (hij != (i == j ? 1.0 : 0.0)) diag = false;
      if (i != j && (m->R_chol[i * d + j] != 0.0 || m->Q_chol[i * d + j] != 0.0)) diag = false;
    }
  for (int i = 0; i < d; ++i) {
    P->m0[i] = (T)m->m0[i];
    P->qd[i] = (T)m->Q_chol[i * d + i];
    P->lid[i] = (T)Li[i * d + i];
    for (int j = 0; j < d; ++j) {
      P->A[i * kMaxDim + j] = (T)m->A[i * d + j];
      P->H[i * kMaxDim + j] = (T)m->H[i * d + j];
      if (j <= i) {
        P->Lq[i * kMaxDim + j] = (T)m->Q_chol[i * d + j];
        P->Li[i * kMaxDim + j] = (T)Li[i * d + j];
        P->L0[i * kMaxDim + j] = (T)m->P0_chol[i * d + j];
      }
    }
  }
  *mk_out = diag ? MK_LG_DIAG : MK_LG_DENSE;
}

// Bank-conflict cost of the LDS pad for the per-group scalar arrays
// (layout [column][r + pad]): phase-A/C accesses by consecutive pairs and
// phase-B accesses by group lanes, evaluated for 32 and 64 banks. For
// r > 64 member q of a column sits at word q + q / 64 (one skipped word per
// 64 members, so the lanes of one step of the draw's binary search, which
// lie a multiple of 64 members apart, fall in distinct banks); the returned
// pad then includes those r / 64 words.
inline uint32_t choose_pad_eval(uint32_t r, uint32_t C, uint32_t log2R, int nt);

// Memoised: the batched planner asks for the same geometries many times.
inline uint32_t choose_pad(uint32_t r, uint32_t C, uint32_t log2R, int nt) {
  thread_local std::map<std::tuple<uint32_t, uint32_t, uint32_t, int>, uint32_t> cache;
  const auto key = std::make_tuple(r, C, log2R, nt);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  const uint32_t p = choose_pad_eval(r, C, log2R, nt);
  cache.emplace(key, p);
  return p;
}

inline uint32_t choose_pad_eval(uint32_t r, uint32_t C, uint32_t log2R, int nt) {
  const uint32_t log2r = ilog2(r), log2C = ilog2(C);
  const bool wide = log2R >= log2C;
  auto coords = [&](uint32_t f, uint32_t& q, uint32_t& c) {
    if (wide) {
      q = f >> log2C;
      c = f & (C - 1);
    } else {
      const uint32_t sh = log2r + log2R;
      const uint32_t hb = f >> sh, rem = f & ((1u << sh) - 1);
      q = rem >> log2R;
      c = (hb << log2R) | (rem & ((1u << log2R) - 1));
    }
  };
  const uint32_t skip = r > 64 ? r >> 6 : 0u;
  auto lix = [&](uint32_t q) { return r > 64 ? q + (q >> 6) : q; };
  // LDS cycles of one access of n <= 64 lanes: per group of lanes served
  // together, the largest number of distinct addresses that share a bank
  // (fixed-size arrays: the planner allocates no memory)
  auto degree = [](const uint32_t* addr, int n, int banks, int lanes_per_cycle) {
    double tot = 0;
    for (int g = 0; g < n; g += lanes_per_cycle) {
      int cnt[64] = {0};
      int mx = 0;
      const int e = g + lanes_per_cycle < n ? g + lanes_per_cycle : n;
      for (int i = g; i < e; ++i) {
        bool seen = false;
        for (int j = g; j < i; ++j) seen |= (addr[j] == addr[i]);
        if (seen) continue;
        const int bk = (int)(addr[i] % (uint32_t)banks);
        mx = std::max(mx, ++cnt[bk]);
      }
      tot += mx;
    }
    return tot;
  };
  uint32_t best = 0;
  double best_cost = 1e30;
  const uint32_t cands[] = {0, 1, 2, 3, 4, 5, 8};
  for (uint32_t pad : cands) {
    const uint32_t P = r + skip + pad;
    double cost = 0;
    for (int banks : {32, 64}) {
      const int lpc = banks == 32 ? 32 : 64;
      uint32_t addr[64];
      for (int e = 0; e < 2; ++e) {
        int n = 0;
        for (int l = 0; l < 64 && l < nt; ++l) {
          uint32_t q, c;
          coords(2u * l + e, q, c);
          addr[n++] = c * P + lix(q);
        }
        cost += degree(addr, n, banks, lpc);
      }
      for (uint32_t l = 0; l < 64; ++l) addr[l] = r <= 64 ? (l >> log2r) * P + (l & (r - 1)) : l;
      cost += 2 * degree(addr, 64, banks, lpc);
    }
    cost += 0.01 * pad;  // prefer the smaller pad on ties
    if (cost < best_cost) {
      best_cost = cost;
      best = pad;
    }
  }
  return skip + best;
}

// Argument checks of a model (eq. HMM of Section 1.1 as the header states
// it). Returns PF_OK or PF_E_INVALID with a message.
inline pf_status validate_model(const pf_model* model, std::string& msg) {
  if (!model) {
    msg = "model is NULL";
    return PF_E_INVALID;
  }
  const int d = model->d;
  if (model->kind != PF_MODEL_LG && model->kind != PF_MODEL_SV) {
    msg = "unknown model kind";
    return PF_E_INVALID;
  }
  if (d < 1 || d > PF_MAX_DIM) {
    msg = "d must be in [1, 16]";
    return PF_E_INVALID;
  }
  if (model->kind == PF_MODEL_SV) {
    if (d != 1) {
      msg = "the SV model has d = 1";
      return PF_E_INVALID;
    }
    if (!(std::fabs(model->phi) < 1.0) || !(model->sigma > 0.0) || !(model->beta > 0.0) ||
        !std::isfinite(model->sigma) || !std::isfinite(model->beta)) {
      msg = "SV parameters need |phi| < 1, sigma > 0, beta > 0";
      return PF_E_INVALID;
    }
    return PF_OK;
  }
  const double* ms[] = {model->A, model->Q_chol, model->H, model->R_chol, model->P0_chol};
  for (const double* m : ms)
    if (!m || !finite_all(m, (size_t)d * d)) {
      msg = "LG matrix NULL or non-finite";
      return PF_E_INVALID;
    }
  if (!model->m0 || !finite_all(model->m0, d)) {
    msg = "m0 NULL or non-finite";
    return PF_E_INVALID;
  }
  const double* tri[] = {model->Q_chol, model->R_chol, model->P0_chol};
  for (const double* L : tri)
    for (int i = 0; i < d; ++i) {
      if (!(L[i * d + i] > 0.0)) {
        msg = "Cholesky factor needs a positive diagonal";
        return PF_E_INVALID;
      }
      for (int j = i + 1; j < d; ++j)
        if (L[i * d + j] != 0.0) {
          msg = "Cholesky factor must be lower-triangular";
          return PF_E_INVALID;
        }
    }
  return PF_OK;
}

// Compiled dimension for a model dimension d.
inline int compiled_dim(int d) { return d <= 1 ? 1 : d <= 2 ? 2 : d <= 4 ? 4 : d <= 8 ? 8 : 16; }

// Mixed-radix stage radices of N = 2^n for radix r = 2^b < N: S - 1 digits
// of radix r from the least significant end, the top digit takes the rest.
inline std::vector<uint32_t> mixed_radices(uint64_t N, uint64_t radix) {
  const uint32_t n = ilog2(N), b = ilog2(radix);
  const uint32_t S = (n + b - 1) / b;
  const uint32_t last = n - (S - 1) * b;
  std::vector<uint32_t> out;
  for (uint32_t k = 0; k < S; ++k) out.push_back(1u << ((k + 1 < S) ? b : last));
  return out;
}

}  // namespace pfh
