// internal.hpp -- shared declarations of the ccfmm HIP library (gfx950).
//
// Indexing of Cartesian multi-indices n = (nx, ny, nz) (Sec. 3 notation):
// degree-major, then nx descending, then ny descending.  The flat index of n
// with degree d = |n| is N(d-1) + u(u+1)/2 + nz with u = d - nx, where
// N(d) = (d+1)(d+2)(d+3)/6 counts the multi-indices of degree <= d.
// Expansions keep only the "active" coefficients 1 <= |n| <= p: a dipole
// distribution has no monopole (Q_0 = 0) and the field needs no V_0.
// Active coefficient a <-> flat index a + 1.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ccfmm.h"

namespace ccfmm {

constexpr int kPMax = CCFMM_PMAX;
constexpr int kLMax = CCFMM_LMAX;
constexpr int kKMax = 2 * kPMax;  // derivative tensors up to order 2p
// M2L kernel variants and their tile widths in (target cell, configuration)
// columns: a block of 4 wavefronts sharing one operator per step (64), or
// independent wavefronts gathering operator entries themselves (16)
constexpr int kM2LAuto = -1;  // the default: chosen from order, precision and form at plan creation
constexpr int kM2LBlock = 0;
constexpr int kM2LWave = 1;
constexpr int kM2LWide4 = 2;  // FP32, 256-column tiles
constexpr int kM2LWide2 = 3;  // FP32, 128-column tiles
constexpr int kM2LWide1 = 4;  // FP32, 64-column tiles
inline int m2l_tile_cols(int variant) {
  return variant == kM2LWave ? 16 : variant == kM2LWide4 ? 256 : variant == kM2LWide2 ? 128 : 64;
}
// the wide (FP32) M2L kernels serve orders up to 6 in the full form and up
// to 8 in the traceless form (its operator is p(p+2) square: 80 rows at p = 8)
inline int wide_max_order(bool traceless) { return traceless ? 8 : 6; }
// whether an M2L kernel variant exists for this order, precision and form
inline bool m2l_variant_ok(int variant, int order, bool fp64, bool traceless) {
  if (variant == kM2LBlock) return true;
  if (variant == kM2LWave) return order <= 6;
  if (variant == kM2LWide4 || variant == kM2LWide2 || variant == kM2LWide1)
    return order <= wide_max_order(traceless) && (traceless || !fp64);  // FP64: traceless form only
  return false;
}
// the variant a plan gets when the caller names none: the 64-column wide
// kernel wherever it exists (the fastest one measured, single configurations
// and batches of 64 alike), else the block kernel
inline int m2l_default_variant(int order, bool fp64, bool traceless) {
  return m2l_variant_ok(kM2LWide1, order, fp64, traceless) ? kM2LWide1 : kM2LBlock;
}

// configurations per M2L tile for a batch of nb: the next power of two, at
// most one tile width
inline int tile_batch(int nb, int cols) {
  int t = 1;
  while (t < nb && t < cols) t <<= 1;
  return t;
}

__host__ __device__ constexpr int ncoef(int d) { return d < 0 ? 0 : (d + 1) * (d + 2) * (d + 3) / 6; }
__host__ __device__ constexpr int midx(int a, int b, int c) {
  return ncoef(a + b + c - 1) + (b + c) * (b + c + 1) / 2 + c;
}
// active coefficients of order p, and the padded stride of one expansion
__host__ __device__ constexpr int nact(int p) { return ncoef(p) - 1; }
__host__ __device__ constexpr int nstride(int p) { return (nact(p) + 3) & ~3; }
// traceless (folded) rows: the n_z <= 1 components, 2l + 1 of degree l, and
// their padded stride
__host__ __device__ constexpr int nred(int p) { return p * (p + 2); }
__host__ __device__ constexpr int nred_stride(int p) { return (nred(p) + 3) & ~3; }
// A row of the derivative table: the ncoef(2p) entries D_k of one offset, then
// one zero (read by the padding entries of the M2L operator)
__host__ __device__ constexpr int drow_stride(int p) { return ncoef(2 * p) + 1; }

template <int K>
struct MultiIndexTable {
  int8_t x[ncoef(K)], y[ncoef(K)], z[ncoef(K)];
  constexpr MultiIndexTable() : x{}, y{}, z{} {
    int t = 0;
    for (int d = 0; d <= K; d++)
      for (int a = d; a >= 0; a--)
        for (int b = d - a; b >= 0; b--) {
          x[t] = (int8_t)a;
          y[t] = (int8_t)b;
          z[t] = (int8_t)(d - a - b);
          t++;
        }
  }
};
__device__ constexpr MultiIndexTable<kKMax> kMI{};

// 1/k! for k <= 16
struct InvFact {
  double v[kKMax + 1];
  constexpr InvFact() : v{} {
    double f = 1.0;
    v[0] = 1.0;
    for (int k = 1; k <= kKMax; k++) {
      f *= k;
      v[k] = 1.0 / f;
    }
  }
};
__device__ constexpr InvFact kInvFact{};

// ---------------------------------------------------------------------------
// Geometry of one tree level (uniform-depth bisection tree).
//   h[a]  cell side, s = smallest side (the level's length unit),
//   g[a]  = h[a] / s, k[a] = halvings of axis a so far, axis = axis halved to
//   reach this level (-1 at the root).
// Scaled expansions at level l: Qt_n = Q_n s^(1-|n|), Vt_n = V_n s^(|n|+2);
// then M2L reads Vt_n = (-1)^|n| sum_q D_{n+q}(delta*g) Qt_q with integer
// cell offsets delta, independent of the level's absolute size.
// ---------------------------------------------------------------------------
struct LevelGeom {
  double h[3];
  double g[3];
  double s;
  int k[3];
  int axis;
};

struct Workspace;

// Flat description of one M2L work tile for one wavefront: up to 16 columns
// (target cell, configuration); the Q columns of step t come from
// step_src[(step0 + t) * 16 + col].
struct M2LTile {
  int32_t level;
  int32_t step0;
  int32_t nsteps;
  int32_t tgt0;     // first entry in tile_tgt (16 entries, -1 = unused column group)
  int32_t b0;       // first configuration of the tile
  int32_t rows;     // local rows its targets need (smallest cells of a lower order: fewer)
  int32_t pad[2];
};

// P2P / L2P work chunk: up to 64 consecutive sorted dipoles of one leaf.
struct P2PChunk {
  int32_t leaf;     // compact leaf index at level L
  int32_t first;    // first sorted dipole
  int32_t count;    // <= 64
  int32_t pad;
};

// ---------------------------------------------------------------------------
// Device memory budget of one plan: the bytes its buffers hold and an optional
// cap.  Buffers allocated while a plan's call runs are charged to its budget
// (current_budget) and uncharged when they release their memory.
// ---------------------------------------------------------------------------
struct MemBudget {
  int64_t cap = 0;   // 0: no cap
  int64_t used = 0;
};
MemBudget*& current_budget();  // per thread; null outside plan calls
struct BudgetScope {
  MemBudget* prev;
  explicit BudgetScope(MemBudget* b) : prev(current_budget()) { current_budget() = b; }
  ~BudgetScope() { current_budget() = prev; }
  BudgetScope(const BudgetScope&) = delete;
  BudgetScope& operator=(const BudgetScope&) = delete;
};

// ---------------------------------------------------------------------------
// Device buffer with grow-only capacity.  Growing past the current budget's
// cap throws CCFMM_ENOMEM before the old memory is released (the buffer keeps
// its contents).
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  MemBudget* budget = nullptr;  // the budget this buffer's memory counts against
  void* ensure(size_t bytes);
  void release();
  template <typename T>
  T* as() const { return reinterpret_cast<T*>(p); }
  ~DevBuf() { release(); }
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

struct HipError {
  hipError_t code;
  std::string what;
};
struct StatusError {
  int status;
  std::string what;
};

void check_hip(hipError_t e, const char* what);
uint64_t devbuf_allocs();  // device allocations made so far (DevBuf::ensure)
#define CCFMM_HIP(x) ::ccfmm::check_hip((x), #x)
[[noreturn]] void fail(int status, const std::string& msg);

// ---------------------------------------------------------------------------
// Primitives (tree.hip)
// ---------------------------------------------------------------------------
// exclusive scan of n int32 values into out (out may alias in); returns nothing,
// total is written to out[n] (out must hold n+1 ints).
void scan_exclusive(const int32_t* in, int32_t* out, int64_t n, DevBuf& tmp, hipStream_t st);
// two independent scans of n values each (one launch when n is small)
void scan_exclusive2(const int32_t* in0, int32_t* out0, const int32_t* in1, int32_t* out1, int64_t n, DevBuf& tmp,
                     hipStream_t st);
// stable LSD radix sort of (key, val) pairs by the low `bits` bits of key
void radix_sort_pairs(uint32_t* key, int32_t* val, uint32_t* key_tmp, int32_t* val_tmp, int64_t n,
                      int bits, DevBuf& tmp, hipStream_t st);

}  // namespace ccfmm
