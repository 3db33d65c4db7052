// api.hip -- the C ABI: plan life cycle, evaluation, info, errors.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>

#include "plan.hpp"

namespace ccfmm {

static thread_local std::string g_last_error;

// device allocations made so far (a captured evaluation stays valid only while
// none of the buffers it reads is reallocated)
static std::atomic<uint64_t> g_devbuf_allocs{0};
uint64_t devbuf_allocs() { return g_devbuf_allocs.load(); }

MemBudget*& current_budget() {
  static thread_local MemBudget* b = nullptr;
  return b;
}

void* DevBuf::ensure(size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (bytes <= cap) return p;
  MemBudget* b = current_budget();
  if (b && b->cap > 0) {
    const int64_t after = b->used - (budget == b ? (int64_t)cap : 0) + (int64_t)bytes;
    if (after > b->cap)
      throw StatusError{CCFMM_ENOMEM, "plan device-memory cap of " + std::to_string(b->cap) + " bytes: holding " +
                                          std::to_string(b->used) + ", a buffer of " + std::to_string(bytes) +
                                          " bytes does not fit"};
  }
  release();
  g_devbuf_allocs.fetch_add(1);
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess || q == nullptr) {
    (void)hipGetLastError();
    throw StatusError{CCFMM_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
  }
  p = q;
  cap = bytes;
  budget = b;
  if (b) b->used += (int64_t)bytes;
  return p;
}

void DevBuf::release() {
  // buffers are only released while rebuilding or destroying; work queued on
  // any stream may still read them, so drain the device first
  if (p) {
    (void)hipDeviceSynchronize();
    (void)hipFree(p);
  }
  if (budget) budget->used -= (int64_t)cap;
  budget = nullptr;
  p = nullptr;
  cap = 0;
}

void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError{e, std::string(what) + ": " + hipGetErrorString(e)};
}

void fail(int status, const std::string& msg) { throw StatusError{status, msg}; }

int selftest_mfma_impl(int device);

// ---------------------------------------------------------------- geometry
__global__ void k_bbox_partial(const double* __restrict__ pos, int64_t n, double* part, int32_t* bad) {
  __shared__ double smin[3][256], smax[3][256];
  const int t = threadIdx.x;
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * 256 + t; i < n; i += (int64_t)gridDim.x * 256) {
    for (int a = 0; a < 3; a++) {
      const double v = pos[3 * i + a];
      if (!isfinite(v)) bad[0] = 1;
      mn[a] = fmin(mn[a], v);
      mx[a] = fmax(mx[a], v);
    }
  }
  for (int a = 0; a < 3; a++) {
    smin[a][t] = mn[a];
    smax[a][t] = mx[a];
  }
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off)
      for (int a = 0; a < 3; a++) {
        smin[a][t] = fmin(smin[a][t], smin[a][t + off]);
        smax[a][t] = fmax(smax[a][t], smax[a][t + off]);
      }
    __syncthreads();
  }
  if (t == 0)
    for (int a = 0; a < 3; a++) {
      part[6 * blockIdx.x + a] = smin[a][0];
      part[6 * blockIdx.x + 3 + a] = smax[a][0];
    }
}

static void device_bbox(const double* d_pos, int64_t n, DevBuf& tmp, hipStream_t st, double mn[3], double mx[3],
                        bool& bad) {
  const int nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256));
  char* buf = reinterpret_cast<char*>(tmp.ensure(sizeof(double) * 6 * nblk + 64));
  double* part = reinterpret_cast<double*>(buf + 64);
  int32_t* dbad = reinterpret_cast<int32_t*>(buf);
  CCFMM_HIP(hipMemsetAsync(dbad, 0, sizeof(int32_t), st));
  k_bbox_partial<<<nblk, 256, 0, st>>>(d_pos, n, part, dbad);
  CCFMM_HIP(hipGetLastError());
  std::vector<double> h(6 * nblk);
  int32_t hb = 0;
  CCFMM_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * 6 * nblk, hipMemcpyDeviceToHost, st));
  CCFMM_HIP(hipMemcpyAsync(&hb, dbad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CCFMM_HIP(hipStreamSynchronize(st));
  for (int a = 0; a < 3; a++) {
    mn[a] = INFINITY;
    mx[a] = -INFINITY;
  }
  for (int b = 0; b < nblk; b++)
    for (int a = 0; a < 3; a++) {
      mn[a] = std::min(mn[a], h[6 * b + a]);
      mx[a] = std::max(mx[a], h[6 * b + 3 + a]);
    }
  bad = hb != 0;
}

// Positions against the caller's box, on the device: [0] = 1 if a coordinate
// is not finite, [1] = 1 if one lies outside [lo, hi] (every writer stores the
// same value)
struct BoxBounds {
  double lo[3], hi[3];
};
__global__ void k_check_in_box(const double* __restrict__ pos, int64_t n, BoxBounds b, int32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * n) return;
  const int a = (int)(i % 3);
  const double v = pos[i];
  if (!isfinite(v)) bad[0] = 1;
  else if (v < b.lo[a] || v > b.hi[a]) bad[1] = 1;
}

static double s_opt(int p) { return p > 3 ? 0.74 * (double)p * (double)p : 8.0; }

// Root box, level count and split sequence.  Root: the caller's box, else the
// tight bounding box (an axis without extent takes the smallest nonzero side,
// or 1).  Levels: the depth whose mean dipoles per smallest cell, N / 2^L, is
// closest to s (ties to the shallower tree).  Split: halve the longest side,
// ties x < y < z.
// the halving sequence to depth L: each level halves the longest side of the
// previous cell shape, ties x < y < z (Sec. 2 and 4)
static void make_geometry(const double lo[3], const double W[3], int L, TreeGeom& G) {
  std::memset(&G, 0, sizeof(G));
  G.L = L;
  double h[3] = {W[0], W[1], W[2]};
  int k[3] = {0, 0, 0};
  for (int l = 0; l <= L; l++) {
    if (l > 0) {
      int a = 0;
      if (h[1] > h[a]) a = 1;
      if (h[2] > h[a]) a = 2;
      h[a] = h[a] / 2.0;
      k[a]++;
      G.lev[l].axis = a;
    } else {
      G.lev[l].axis = -1;
    }
    const double s = std::min(h[0], std::min(h[1], h[2]));
    G.lev[l].s = s;
    for (int a = 0; a < 3; a++) {
      G.lev[l].h[a] = h[a];
      G.lev[l].g[a] = h[a] / s;
      G.lev[l].k[a] = k[a];
    }
  }
  for (int a = 0; a < 3; a++) {
    G.lo[a] = lo[a];
    G.W[a] = W[a];
  }
}

static void setup_geometry(Plan& P, const double mn[3], const double mx[3], const double* d_pos, hipStream_t st) {
  double lo[3], W[3];
  if (P.prm.has_box) {
    for (int a = 0; a < 3; a++) {
      lo[a] = P.prm.box_lo[a];
      W[a] = P.prm.box_hi[a] - P.prm.box_lo[a];
      if (!(W[a] > 0.0) || !std::isfinite(W[a])) fail(CCFMM_EINVAL, "empty or non-finite box");
      if (mn[a] < P.prm.box_lo[a] || mx[a] > P.prm.box_hi[a]) fail(CCFMM_EINVAL, "a dipole lies outside the box");
    }
  } else {
    double smallest = 0.0;
    for (int a = 0; a < 3; a++) {
      const double w = mx[a] - mn[a];
      if (w > 0.0 && (smallest == 0.0 || w < smallest)) smallest = w;
    }
    if (smallest == 0.0) smallest = 1.0;
    for (int a = 0; a < 3; a++) {
      lo[a] = mn[a];
      W[a] = (mx[a] - mn[a] > 0.0) ? (mx[a] - mn[a]) : smallest;
    }
  }
  P.s_used = P.prm.leaf_target > 0.0 ? P.prm.leaf_target : s_opt(P.p);
  // Level count: the depth whose mean dipoles per smallest cell is closest to
  // s, ties to the shallower tree (Sec. 4).  Rule 0 averages over all 2^L
  // cells (the paper's N/2^L); rule 1 over the occupied ones.
  int64_t occupied[kLMax + 1];
  if (P.prm.leaf_rule == 1) {
    TreeGeom G24;
    make_geometry(lo, W, kLMax, G24);
    count_occupied_by_depth(P, d_pos, G24, st, occupied);
  }
  int best = 0;
  double bestd = INFINITY;
  for (int L = 0; L <= kLMax; L++) {
    const double avg = P.prm.leaf_rule == 1 ? (double)P.n / (double)occupied[L] : (double)P.n / std::ldexp(1.0, L);
    const double d = std::fabs(avg - P.s_used);
    if (d < bestd) {
      bestd = d;
      best = L;
    }
  }
  P.L = best;
  make_geometry(lo, W, P.L, P.geo);
}

// Expansion and moment buffers for nb configurations; the level offsets are
// committed only once every buffer has its size (a failed allocation leaves
// the previous layout in place).
static void size_expansions(Plan& P, int nb) {
  const int NS = nstride(P.p);
  int64_t off = 0;
  std::vector<int64_t> qoff(P.L + 1);
  for (int l = 0; l <= P.L; l++) {
    qoff[l] = off;
    off += (int64_t)P.lev[l]->ncells * nb * NS;
  }
  const size_t es = P.precision == CCFMM_PREC_FP64 ? sizeof(double) : sizeof(float);
  P.Q.ensure(es * std::max<int64_t>(1, off));
  P.V.ensure(es * std::max<int64_t>(1, off));
  if (P.prm.m2l_traceless && P.p <= wide_max_order(true))
    P.Qr.ensure(es * std::max<int64_t>(1, off / NS * ((P.p * (P.p + 2) + 3) & ~3)));
  P.m_sorted.ensure(es * 3 * (size_t)P.n * nb);
  if (nb >= P.batched_min) P.m_sorted_t.ensure(es * 3 * (size_t)P.n * nb);
  for (int l = 0; l <= P.L; l++) P.lev[l]->qoff = qoff[l];
  P.qv_elems = off;
  P.qv_batch = nb;
}

// sum over smallest cells of (its dipoles) x (the dipoles of its near cells):
// wavefronts stride over the cells, each block adds its total once (an
// integer sum: exact in any order, and a few thousand atomics instead of one
// per cell)
constexpr int kPairCountBlocks = 2048;
__global__ void __launch_bounds__(256) k_count_p2p_pairs(int32_t nl, const int32_t* near_ptr,
                                                         const int32_t* near_idx, const int32_t* lcount,
                                                         unsigned long long* out) {
  __shared__ long long part[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  long long s = 0;
  for (int i = blockIdx.x * 4 + w; i < nl; i += gridDim.x * 4) {
    long long c = 0;
    for (int e = near_ptr[i] + lane; e < near_ptr[i + 1]; e += 64) c += lcount[near_idx[e]];
    s += c * lcount[i];
  }
  for (int off = 1; off < 64; off <<= 1) s += __shfl_xor(s, off);
  if (lane == 0) part[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, (unsigned long long)(part[0] + part[1] + part[2] + part[3]));
}

// scattered device counters gathered into one small array (one copy back);
// the last two words are cleared for the direct-pair count
struct InfoSources {
  const int32_t* at[2 * (kLMax + 1) + 3];
  int32_t n;
};
__global__ void k_info_gather(InfoSources src, int cidx, int32_t* out) {
  const int i = threadIdx.x;
  if (i < src.n) out[i] = *src.at[i];
  if (i == 0) out[cidx] = out[cidx + 1] = 0;
}

// direct-pair count of the current cells and lists into *dcnt (cleared by the caller)
static void launch_pair_count(Plan& P, unsigned long long* dcnt, hipStream_t st) {
  LevelData& D = *P.lev[P.L];
  const int nblk = (int)std::min<int64_t>(kPairCountBlocks, std::max<int64_t>(1, ceil_div(D.ncells, 4)));
  k_count_p2p_pairs<<<nblk, 256, 0, st>>>(D.ncells, D.near_ptr.as<int32_t>(), D.near_idx.as<int32_t>(),
                                          P.lcount.as<int32_t>(), dcnt);
  CCFMM_HIP(hipGetLastError());
}

// count_pairs = false (an update that kept the lists) leaves the direct-pair
// count, a statistic only, to the next ccfmm_plan_info
static void fill_info(Plan& P, hipStream_t st, bool count_pairs = true) {
  // list totals, chunk counts, error flags and the direct-pair count come
  // back in one copy and one synchronisation
  const int L = P.L;
  const int nl = P.lev[L]->ncells;
  InfoSources src{};
  for (int l = 0; l <= L; l++) {
    LevelData& D = *P.lev[l];
    src.at[2 * l] = D.near_ptr.as<int32_t>() + D.ncells;
    src.at[2 * l + 1] = D.far_ptr.as<int32_t>() + D.ncells;
  }
  src.at[2 * (L + 1)] = P.chunk_cnt.as<int32_t>() + (nl + 1) + nl;
  src.at[2 * (L + 1) + 1] = P.flags.as<int32_t>();
  src.at[2 * (L + 1) + 2] = P.chunk_cnt.as<int32_t>() + 3 * (nl + 1) + nl;
  src.n = 2 * (L + 1) + 3;
  const int cidx = (src.n + 1) & ~1;  // the 64-bit pair count, 8-byte aligned
  const int nw = cidx + 2;
  int32_t* dbuf = reinterpret_cast<int32_t*>(P.scratch2.ensure(sizeof(int32_t) * (nw + 2)));
  k_info_gather<<<1, 64, 0, st>>>(src, cidx, dbuf);
  CCFMM_HIP(hipGetLastError());
  if (count_pairs) launch_pair_count(P, reinterpret_cast<unsigned long long*>(dbuf + cidx), st);
  P.pairs_stale = !count_pairs;
  std::vector<int32_t> tot(nw, 0);
  CCFMM_HIP(hipMemcpyAsync(tot.data(), dbuf, sizeof(int32_t) * nw, hipMemcpyDeviceToHost, st));
  CCFMM_HIP(hipStreamSynchronize(st));
  unsigned long long npairs = 0;
  std::memcpy(&npairs, &tot[cidx], sizeof(npairs));
  P.nchunks32 = tot[2 * (L + 1) + 2];
  if (tot[2 * (L + 1) + 1]) fail(CCFMM_EHIP, "internal: a cell list exceeded its bound");
  for (int l = 0; l <= L; l++) {
    P.lev[l]->nnear = tot[2 * l];
    P.lev[l]->nfar = tot[2 * l + 1];
  }
  P.nchunks = tot[2 * (L + 1)];
  ccfmm_info& I = P.info;
  std::memset(&I, 0, sizeof(I));
  I.n = P.n;
  I.order = P.p;
  I.levels = P.L;
  I.precision = P.precision;
  I.max_batch = P.nbmax;
  for (int l = 0; l <= kLMax; l++) I.split_axis[l] = (l >= 1 && l <= P.L) ? P.geo.lev[l].axis : -1;
  for (int a = 0; a < 3; a++) {
    I.box_lo[a] = P.geo.lo[a];
    I.box_hi[a] = P.geo.lo[a] + P.geo.W[a];
    I.leaf_side[a] = P.geo.lev[P.L].h[a];
  }
  I.s_used = P.s_used;
  I.n_leaves = P.lev[P.L]->ncells;
  int64_t cells = 0, m2l = 0;
  for (int l = 0; l <= P.L; l++) {
    cells += P.lev[l]->ncells;
    I.m2l_pairs_per_level[l] = P.lev[l]->nfar;
    m2l += P.lev[l]->nfar;
  }
  I.n_cells = cells;
  I.n_delta = P.nrows;
  I.n_m2l_pairs = m2l;
  I.n_p2p_leaf_pairs = P.lev[P.L]->nnear;
  I.n_m2l_tiles = P.ntiles;
  I.n_m2l_steps = P.nsteps;
  I.m2l_class_bits = P.class_bits;
  I.m2l_variant = P.m2l_variant;
  I.n_rebuilds_kept = P.n_rebuilds_kept;
  const double np = (double)nact(P.p);
  I.m2l_flops_per_config = 2.0 * np * np * (double)m2l;
  // direct pairs (self pairs included in the count)
  I.n_p2p_pairs = (int64_t)npairs;
  I.p2p_pairs_per_config = (double)npairs;
}

static void validate_params(const ccfmm_params* prm, int64_t n) {
  if (!prm) fail(CCFMM_EINVAL, "params is NULL");
  if (n < 1) fail(CCFMM_EINVAL, "n must be >= 1");
  if (n > (int64_t)INT32_MAX / 3) fail(CCFMM_EINVAL, "n too large");
  if (prm->order < 1 || prm->order > kPMax) fail(CCFMM_EINVAL, "order must be in 1..8");
  if (!(prm->theta > 0.0 && prm->theta < 1.0)) fail(CCFMM_EINVAL, "theta must be in (0, 1)");
  if (!std::isfinite(prm->leaf_target)) fail(CCFMM_EINVAL, "leaf_target not finite");
  if (prm->leaf_rule != 0 && prm->leaf_rule != 1) fail(CCFMM_EINVAL, "leaf_rule must be 0 or 1");
  if (prm->precision != CCFMM_PREC_FP64 && prm->precision != CCFMM_PREC_MIXED)
    fail(CCFMM_EINVAL, "precision must be FP64 or MIXED");
  if (prm->selector != 0 && prm->selector != 1) fail(CCFMM_EINVAL, "selector must be 0 or 1");
  if (prm->selector == 1) {
    if (prm->order < 2) fail(CCFMM_EINVAL, "the learned selector needs order >= 2 (candidate orders 2..6)");
    if (!(prm->err_bound > 0.0) || !std::isfinite(prm->err_bound))
      fail(CCFMM_EINVAL, "err_bound must be finite and > 0 with the selector");
    if (!(prm->sel_margin >= 0.0) || !std::isfinite(prm->sel_margin))
      fail(CCFMM_EINVAL, "sel_margin must be finite and >= 0");
    if (!std::isfinite(prm->sel_cost_far)) fail(CCFMM_EINVAL, "sel_cost_far not finite");
  }
  if (prm->max_batch < 1 || prm->max_batch > 4096) fail(CCFMM_EINVAL, "max_batch must be in 1..4096");
  if (prm->truncation != 0 && prm->truncation != 1) fail(CCFMM_EINVAL, "truncation must be 0 or 1");
  if (prm->m2l_traceless != 0 && prm->m2l_traceless != 1) fail(CCFMM_EINVAL, "m2l_traceless must be 0 or 1");
  if (prm->device_mem_cap < 0) fail(CCFMM_EINVAL, "device_mem_cap must be >= 0");
  if (prm->has_box)
    for (int a = 0; a < 3; a++)
      if (!std::isfinite(prm->box_lo[a]) || !std::isfinite(prm->box_hi[a])) fail(CCFMM_EINVAL, "box not finite");
}

// Build (or rebuild) everything that depends on the positions.
// With the same geometry and the same occupied cells at every level, the cell
// lists, the M2L tiles and the derivative tables depend on nothing that
// moved: a rebuild then redoes the tree (keys, sort, dipole ranges) and the
// near-field chunks only, and keeps the captured evaluation if no buffer it
// reads was reallocated and its launch sizes stand.  This is the usual case
// of a time step in a dense system (dipoles move, cells stay occupied).
static void build_all(Plan& P, const double* d_pos, hipStream_t st, bool was_built = false) {
  // the current lists (fixed, or with per-cell parameters) can be kept if the
  // cells stay: per-cell parameters are in compact leaf order, which the same
  // occupied cells leave unchanged
  const bool prev_kept_ok = was_built && P.prm.keep_lists != 0;
  const TreeGeom geo0 = P.geo;
  const int L0 = P.L;
  const uint64_t allocs0 = devbuf_allocs();
  double mn[3], mx[3];
  // With the caller's box and the paper's level rule the bounds are only a
  // check: it runs on the device and comes back with the level sizes (the
  // tree kernels clamp any coordinate into the box, so nothing they index
  // depends on it), saving a wait.  Otherwise the bounds set the root cell.
  const bool check_later = P.prm.has_box && P.prm.leaf_rule == 0;
  int32_t check[2] = {0, 0};
  if (check_later) {
    int32_t* dchk = reinterpret_cast<int32_t*>(P.pos_check.ensure(sizeof(int32_t) * 2));
    CCFMM_HIP(hipMemsetAsync(dchk, 0, sizeof(int32_t) * 2, st));  // not captured: an update runs eagerly
    BoxBounds bb;
    for (int a = 0; a < 3; a++) {
      bb.lo[a] = mn[a] = P.prm.box_lo[a];
      bb.hi[a] = mx[a] = P.prm.box_hi[a];
    }
    k_check_in_box<<<ceil_div(3 * P.n, 256), 256, 0, st>>>(d_pos, P.n, bb, dchk);
    CCFMM_HIP(hipGetLastError());
  } else {
    bool bad = false;
    device_bbox(d_pos, P.n, P.scratch, st, mn, mx, bad);
    if (bad) fail(CCFMM_EINVAL, "non-finite position");
  }
  setup_geometry(P, mn, mx, d_pos, st);
  const bool same_geo = prev_kept_ok && P.L == L0 && std::memcmp(&geo0, &P.geo, sizeof(TreeGeom)) == 0;
  const int64_t n = P.n;
  P.key.ensure(sizeof(uint32_t) * n);
  P.val.ensure(sizeof(int32_t) * n);
  P.key_tmp.ensure(sizeof(uint32_t) * n);
  P.val_tmp.ensure(sizeof(int32_t) * n);
  P.perm.ensure(sizeof(int32_t) * n);
  P.yd.ensure(sizeof(double) * 3 * n);
  P.yf.ensure(sizeof(float) * 6 * n);
  P.leaf_start.ensure(sizeof(int32_t) * ((1ll << P.L) + 1));
  const int64_t nheap = (2ll << P.L) - 1;
  P.heap_flag.ensure(sizeof(int32_t) * (nheap + 1));
  P.heap_scan.ensure(sizeof(int32_t) * (nheap + 1));
  P.cmap.ensure(sizeof(int32_t) * nheap);
  while ((int)P.lev.size() < P.L + 1) P.lev.emplace_back(new LevelData());
  bool same_cells = false;
  build_tree(P, d_pos, st, same_geo ? &same_cells : nullptr, check_later ? P.pos_check.as<int32_t>() : nullptr,
             check);
  if (check[0]) fail(CCFMM_EINVAL, "non-finite position");
  if (check[1]) fail(CCFMM_EINVAL, "a dipole lies outside the box");
  if (same_geo && same_cells) {
    // nothing to wait for: the near-field launches cover the chunk lists'
    // capacity (unchanged with the cells) and read their lengths on the GPU;
    // the plan statistics are those of the same lists, the direct-pair count
    // is taken at the next ccfmm_plan_info
    build_p2p_chunks(P, st);
    P.n_rebuilds_kept++;
    P.info.n_rebuilds_kept = P.n_rebuilds_kept;
    P.pairs_stale = true;
    if (devbuf_allocs() != allocs0) P.drop_graph();
    P.built = P.ever_built = true;
    return;
  }
  // new cells: per-cell parameters belong to the previous ones; a learned
  // plan chooses again at its next evaluation
  P.has_leaf = false;
  P.h_leaf_p.clear();
  P.h_leaf_theta.clear();
  P.sel_stale = true;
  P.drop_graph();
  build_lists(P, st);
  build_dtensors(P, st);
  build_p2p_chunks(P, st);
  build_m2l_tiles(P, P.nbmax, st);
  P.qv_batch = 0;
  fill_info(P, st);
  P.info.learned = 0;
  P.built = P.ever_built = true;
}

static void prepare_batch_impl(Plan& P, int nb, hipStream_t st);

// On failure (an allocation past the plan's cap, say) the batch layout and
// the tiles are marked stale, so the next call lays them out anew.
static void prepare_batch(Plan& P, int nb, hipStream_t st) {
  try {
    prepare_batch_impl(P, nb, st);
  } catch (...) {
    P.qv_batch = 0;
    P.tiles_variant = -1;
    P.drop_graph();
    throw;
  }
}

static void prepare_batch_impl(Plan& P, int nb, hipStream_t st) {
  if (nb < 1 || nb > P.nbmax) fail(CCFMM_EINVAL, "nbatch must be in 1..max_batch");
  const int tb = tile_batch(nb, m2l_tile_cols(P.m2l_variant));
  if (tb != P.TB || ceil_div(nb, tb) != P.ncg || P.tiles_variant != P.m2l_variant ||
      P.tiles_class_bits != P.class_bits) {
    P.drop_graph();
    build_m2l_tiles(P, nb, st);
    P.info.n_m2l_tiles = P.ntiles;
    P.info.n_m2l_steps = P.nsteps;
  }
  if (P.qv_batch != nb) {
    P.drop_graph();
    size_expansions(P, nb);
  }
}

static void eval_passes(Plan& P, int nb, const double* d_m, double* d_H, hipStream_t st, hipEvent_t* ev,
                        bool fuse_near = true);

// Timing events between passes: released at device scope, so recording one
// does not write back and invalidate the caches before the next pass (that
// made the pass after it start cold and time up to 12% slower than in a
// plain evaluation).  The last event of a call keeps the default release.
static void create_pass_events(hipEvent_t* ev, int count, int last) {
  for (int i = 0; i < count; i++)
    CCFMM_HIP(hipEventCreateWithFlags(&ev[i], i == last ? hipEventDefault : hipEventReleaseToDevice));
}

// One evaluation.  With graphs on (and a capturable stream), the pass sequence
// is captured once per (nbatch, moments, fields) and replayed; the capture
// holds kernel launches only.
int auto_select(Plan& P, int nb, const double* d_m, hipStream_t st);

// Returns CCFMM_OK, or CCFMM_W_FALLBACK when this call made the learned choice
// and the judge rejected it.
static int eval_run(Plan& P, int nb, const double* d_m, double* d_H, hipStream_t st) {
  if (nb < 1 || nb > P.nbmax) fail(CCFMM_EINVAL, "nbatch must be in 1..max_batch");
  const int rc = auto_select(P, nb, d_m, st);
  prepare_batch(P, nb, st);
  if (!P.use_graph || st == nullptr) {
    eval_passes(P, nb, d_m, d_H, st, nullptr);
    return rc;
  }
  if (!P.gexec || P.g_nb != nb || P.g_m != d_m || P.g_H != d_H) {
    P.drop_graph();
    CCFMM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      eval_passes(P, nb, d_m, d_H, st, nullptr);
    } catch (...) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(st, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      throw;
    }
    hipGraph_t g = nullptr;
    CCFMM_HIP(hipStreamEndCapture(st, &g));
    hipError_t e = hipGraphInstantiate(&P.gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) P.gexec = nullptr;
    CCFMM_HIP(e);
    P.g_nb = nb;
    P.g_m = d_m;
    P.g_H = d_H;
  }
  CCFMM_HIP(hipGraphLaunch(P.gexec, st));
  return rc;
}

static void ensure_side_stream(Plan& P) {
  if (P.side) return;
  CCFMM_HIP(hipStreamCreateWithFlags(&P.side, hipStreamNonBlocking));
  CCFMM_HIP(hipEventCreateWithFlags(&P.ev_fork, hipEventDisableTiming));
  CCFMM_HIP(hipEventCreateWithFlags(&P.ev_join, hipEventDisableTiming));
}

// The passes of one evaluation.  With overlap, the near field (VALU-bound)
// runs on the plan's side stream while P2M, M2M, M2L (MFMA-bound) and L2L run
// on the caller's stream; the smooth field is added after the join.  The side
// stream forks as soon as the moments are in tree order: the near field needs
// nothing else, and it is the longest pass.  Timing
// events (ev, 9 of them): [0] start, [1] after P2M, [2] after M2M, [3] after
// M2L, [4] after L2L, [8] L2P start, [5] end, all on the caller's stream;
// [6], [7] around the near field.
static void eval_passes(Plan& P, int nb, const double* d_m, double* d_H, hipStream_t st, hipEvent_t* ev,
                        bool fuse_near) {
  if (ev) CCFMM_HIP(hipEventRecord(ev[0], st));
  run_permute(P, nb, d_m, st);
  if (P.overlap) {
    ensure_side_stream(P);
    CCFMM_HIP(hipEventRecord(P.ev_fork, st));
    CCFMM_HIP(hipStreamWaitEvent(P.side, P.ev_fork, 0));
    if (ev) CCFMM_HIP(hipEventRecord(ev[6], P.side));
    run_near(P, nb, d_H, P.side);
    if (ev) CCFMM_HIP(hipEventRecord(ev[7], P.side));
    CCFMM_HIP(hipEventRecord(P.ev_join, P.side));
  }
  run_p2m(P, nb, d_m, st);
  if (ev) CCFMM_HIP(hipEventRecord(ev[1], st));
  run_m2m(P, nb, st);
  if (ev) CCFMM_HIP(hipEventRecord(ev[2], st));
  run_m2l(P, nb, st);
  if (ev) CCFMM_HIP(hipEventRecord(ev[3], st));
  run_l2l(P, nb, st);
  if (ev) CCFMM_HIP(hipEventRecord(ev[4], st));
  if (P.overlap) {
    CCFMM_HIP(hipStreamWaitEvent(st, P.ev_join, 0));
    if (ev) CCFMM_HIP(hipEventRecord(ev[8], st));
    run_l2p(P, nb, d_H, st);
  } else if (nb >= P.batched_min || (nb >= 2 && !fuse_near)) {  // two kernels, timed apart
    if (ev) CCFMM_HIP(hipEventRecord(ev[6], st));
    run_near(P, nb, d_H, st);
    if (ev) {
      CCFMM_HIP(hipEventRecord(ev[7], st));
      CCFMM_HIP(hipEventRecord(ev[8], st));
    }
    run_l2p(P, nb, d_H, st);
  } else {
    if (ev) CCFMM_HIP(hipEventRecord(ev[6], st));
    run_p2p_l2p(P, nb, d_H, st);
    if (ev) {
      CCFMM_HIP(hipEventRecord(ev[7], st));
      CCFMM_HIP(hipEventRecord(ev[8], st));
    }
  }
  if (ev) CCFMM_HIP(hipEventRecord(ev[5], st));
}

// one evaluation, plain stream launches (no capture, no learned choice)
void eval_once(Plan& P, int nb, const double* d_m, double* d_H, hipStream_t st) {
  prepare_batch(P, nb, st);
  eval_passes(P, nb, d_m, d_H, st, nullptr);
}

template <typename F>
static int guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const StatusError& e) {
    g_last_error = e.what;
    return e.status;
  } catch (const HipError& e) {
    g_last_error = e.what;
    return CCFMM_EHIP;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return CCFMM_ENOMEM;
  } catch (...) {
    g_last_error = "unexpected internal error";
    return CCFMM_EHIP;
  }
}

}  // namespace ccfmm

using namespace ccfmm;

extern "C" {

const char* ccfmm_status_string(int status) {
  switch (status) {
    case CCFMM_OK: return "ok";
    case CCFMM_EINVAL: return "invalid argument";
    case CCFMM_ENOMEM: return "out of memory";
    case CCFMM_EHIP: return "HIP runtime error";
    case CCFMM_ESTATE: return "invalid plan state";
    case CCFMM_W_FALLBACK: return "learned selector fell back to fixed parameters";
    case CCFMM_W_NOWEIGHTS: return "selector weights file missing, fixed parameters kept";
    default: return "unknown status";
  }
}

const char* ccfmm_last_error(void) { return g_last_error.c_str(); }

int ccfmm_params_default(ccfmm_params* prm) {
  if (!prm) return CCFMM_EINVAL;
  std::memset(prm, 0, sizeof(*prm));
  prm->order = 4;
  prm->theta = 0.5;
  prm->leaf_target = 0.0;
  prm->leaf_rule = 0;
  prm->precision = CCFMM_PREC_FP64;
  prm->selector = 0;
  prm->err_bound = 1e-5;
  prm->sel_margin = 0.3;
  prm->sel_cost_far = 0.0;
  prm->overlap_near = 1;
  prm->keep_lists = 1;
  prm->truncation = 0;
  prm->m2l_traceless = 1;
  prm->has_box = 0;
  prm->max_batch = 1;
  prm->m2l_class_bits = 3;
  prm->m2l_variant = kM2LAuto;
  prm->use_graph = 1;
  return CCFMM_OK;
}

static int create_common(ccfmm_plan* out, int64_t n, const double* d_pos, const ccfmm_params* prm, hipStream_t st,
                         bool own) {
  return guarded([&] {
    if (!out) fail(CCFMM_EINVAL, "out is NULL");
    *out = nullptr;
    validate_params(prm, n);
    if (!d_pos) fail(CCFMM_EINVAL, "positions are NULL");
    ccfmm_plan pl = new ccfmm_plan_s();
    Plan& P = pl->P;
    P.mem.cap = prm->device_mem_cap;
    try {
      BudgetScope bs(&P.mem);
      CCFMM_HIP(hipGetDevice(&P.device));
      P.n = n;
      P.prm = *prm;
      P.p = prm->order;
      P.precision = prm->precision;
      P.nbmax = prm->max_batch;
      P.class_bits = prm->m2l_class_bits < 0 ? 3 : std::min(prm->m2l_class_bits, 12);
      const bool fp64 = prm->precision == CCFMM_PREC_FP64, traceless = prm->m2l_traceless != 0;
      if (prm->m2l_variant == kM2LAuto)
        P.m2l_variant = m2l_default_variant(prm->order, fp64, traceless);
      else
        P.m2l_variant = m2l_variant_ok(prm->m2l_variant, prm->order, fp64, traceless) ? prm->m2l_variant
                                                                                       : kM2LBlock;
      P.use_graph = prm->use_graph != 0;
      P.overlap = prm->overlap_near != 0;
      if (own) {
        CCFMM_HIP(hipStreamCreateWithFlags(&P.own_stream, hipStreamNonBlocking));
        st = P.own_stream;
      }
      build_all(P, d_pos, st);
    } catch (...) {
      if (P.own_stream) (void)hipStreamDestroy(P.own_stream);
      delete pl;
      throw;
    }
    *out = pl;
    return CCFMM_OK;
  });
}

int ccfmm_plan_create(ccfmm_plan* out, int32_t device, int64_t n, const double* pos, const ccfmm_params* prm) {
  return guarded([&] {
    if (!out) fail(CCFMM_EINVAL, "out is NULL");
    *out = nullptr;
    validate_params(prm, n);
    if (!pos) fail(CCFMM_EINVAL, "positions are NULL");
    for (int64_t i = 0; i < 3 * n; i++)
      if (!std::isfinite(pos[i])) fail(CCFMM_EINVAL, "non-finite position");
    CCFMM_HIP(hipSetDevice(device));
    DevBuf dpos;
    dpos.ensure(sizeof(double) * 3 * n);
    CCFMM_HIP(hipMemcpy(dpos.p, pos, sizeof(double) * 3 * n, hipMemcpyHostToDevice));
    int rc = create_common(out, n, dpos.as<double>(), prm, nullptr, true);
    if (rc == CCFMM_OK) {
      // keep the device copy: the host-pointer plan owns its positions (and
      // they count against its budget)
      Plan& P = (*out)->P;
      std::swap(P.pos.p, dpos.p);
      std::swap(P.pos.cap, dpos.cap);
      P.pos.budget = &P.mem;
      P.mem.used += (int64_t)P.pos.cap;
      if (P.mem.cap > 0 && P.mem.used > P.mem.cap) {
        ccfmm_plan_destroy(*out);
        *out = nullptr;
        fail(CCFMM_ENOMEM, "plan device-memory cap of " + std::to_string(prm->device_mem_cap) +
                               " bytes: the positions do not fit beside the plan");
      }
      CCFMM_HIP(hipStreamSynchronize((*out)->P.own_stream));
    }
    return rc;  // on failure the message set by create_common stands
  });
}

int ccfmm_plan_create_device(ccfmm_plan* out, int64_t n, const double* d_pos, const ccfmm_params* prm,
                             void* stream) {
  return create_common(out, n, d_pos, prm, reinterpret_cast<hipStream_t>(stream), false);
}

int ccfmm_plan_update_positions_device(ccfmm_plan plan, const double* d_pos, void* stream) {
  return guarded([&] {
    if (!plan || !plan->P.ever_built) fail(CCFMM_ESTATE, "plan not built");
    if (!d_pos) fail(CCFMM_EINVAL, "positions are NULL");
    Plan& P = plan->P;
    BudgetScope bs(&P.mem);
    CCFMM_HIP(hipSetDevice(P.device));
    // after a failed update only a full rebuild is trusted
    const bool was_built = P.built;
    P.built = false;  // stays false if the rebuild fails
    build_all(P, d_pos, reinterpret_cast<hipStream_t>(stream), was_built);
    return CCFMM_OK;
  });
}

int ccfmm_eval_device(ccfmm_plan plan, int32_t nbatch, const double* d_m, double* d_H, void* stream) {
  return guarded([&] {
    if (!plan || !plan->P.built) fail(CCFMM_ESTATE, "plan not built");
    if (!d_m || !d_H) fail(CCFMM_EINVAL, "moment or field pointer is NULL");
    Plan& P = plan->P;
    BudgetScope bs(&P.mem);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    CCFMM_HIP(hipSetDevice(P.device));
    return eval_run(P, nbatch, d_m, d_H, st);
  });
}

int ccfmm_eval_device_timed(ccfmm_plan plan, int32_t nbatch, const double* d_m, double* d_H, void* stream,
                            ccfmm_pass_times* times) {
  return guarded([&] {
    if (!plan || !plan->P.built) fail(CCFMM_ESTATE, "plan not built");
    if (!d_m || !d_H || !times) fail(CCFMM_EINVAL, "NULL argument");
    Plan& P = plan->P;
    BudgetScope bs(&P.mem);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    CCFMM_HIP(hipSetDevice(P.device));
    if (nbatch < 1 || nbatch > P.nbmax) fail(CCFMM_EINVAL, "nbatch must be in 1..max_batch");
    const int rc = auto_select(P, nbatch, d_m, st);
    prepare_batch(P, nbatch, st);
    hipEvent_t ev[9];
    create_pass_events(ev, 9, 5);
    // every pass alone on the caller's stream (the near field fused with L2P
    // below the batched size), so each time is that pass's own cost
    const bool overlap = P.overlap;
    P.overlap = false;
    try {
      eval_passes(P, nbatch, d_m, d_H, st, ev);
    } catch (...) {
      P.overlap = overlap;
      throw;
    }
    P.overlap = overlap;
    CCFMM_HIP(hipEventSynchronize(ev[5]));
    CCFMM_HIP(hipEventSynchronize(ev[7]));
    float ms[4], near, l2p, tot;
    for (int i = 0; i < 4; i++) CCFMM_HIP(hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]));
    CCFMM_HIP(hipEventElapsedTime(&near, ev[6], ev[7]));
    CCFMM_HIP(hipEventElapsedTime(&l2p, ev[8], ev[5]));
    CCFMM_HIP(hipEventElapsedTime(&tot, ev[0], ev[5]));
    for (int i = 0; i < 9; i++) (void)hipEventDestroy(ev[i]);
    times->p2m = ms[0];
    times->m2m = ms[1];
    times->m2l = ms[2];
    times->l2l = ms[3];
    times->p2p = near;
    times->l2p = l2p;
    times->total = tot;
    return rc;
  });
}

int ccfmm_eval(ccfmm_plan plan, int32_t nbatch, const double* m, double* H) {
  return guarded([&] {
    if (!plan || !plan->P.built) fail(CCFMM_ESTATE, "plan not built");
    if (!m || !H) fail(CCFMM_EINVAL, "moment or field pointer is NULL");
    Plan& P = plan->P;
    BudgetScope bs(&P.mem);
    if (nbatch < 1 || nbatch > P.nbmax) fail(CCFMM_EINVAL, "nbatch must be in 1..max_batch");
    for (int64_t i = 0; i < (int64_t)3 * P.n * nbatch; i++)
      if (!std::isfinite(m[i])) fail(CCFMM_EINVAL, "non-finite moment");
    CCFMM_HIP(hipSetDevice(P.device));
    hipStream_t st = P.own_stream;
    const size_t bytes = sizeof(double) * 3 * (size_t)P.n * nbatch;
    // plan-owned staging keeps the device addresses stable across calls, so the
    // captured graph is reused
    const size_t cap = sizeof(double) * 3 * (size_t)P.n * P.nbmax;
    if (P.host_m.cap < cap) P.drop_graph();
    P.host_m.ensure(cap);
    P.host_H.ensure(cap);
    CCFMM_HIP(hipMemcpyAsync(P.host_m.p, m, bytes, hipMemcpyHostToDevice, st));
    const int rc = eval_run(P, nbatch, P.host_m.as<double>(), P.host_H.as<double>(), st);
    CCFMM_HIP(hipMemcpyAsync(H, P.host_H.p, bytes, hipMemcpyDeviceToHost, st));
    CCFMM_HIP(hipStreamSynchronize(st));
    return rc;
  });
}

// Time per evaluation in the plan's current form: after a warm-up, the
// better of two runs of four evaluations queued back to back (as a caller's
// loop runs them: per-evaluation start-up overlaps the previous one), replayed
// from a graph captured here when the plan's evaluations use one, else plain
// launches.
static double time_eval_form(Plan& P, int nb, const double* d_m, double* d_H, hipStream_t st, hipEvent_t e0,
                             hipEvent_t e1) {
  const bool graph = P.use_graph && st != nullptr;
  hipGraphExec_t gx = nullptr;
  if (graph) {
    CCFMM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      eval_passes(P, nb, d_m, d_H, st, nullptr);
    } catch (...) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(st, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      throw;
    }
    hipGraph_t g = nullptr;
    CCFMM_HIP(hipStreamEndCapture(st, &g));
    const hipError_t e = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) gx = nullptr;
    CCFMM_HIP(e);
  }
  constexpr int kRun = 4;
  auto launch = [&]() {
    if (graph)
      CCFMM_HIP(hipGraphLaunch(gx, st));
    else
      eval_passes(P, nb, d_m, d_H, st, nullptr);
  };
  double best = INFINITY;
  try {
    launch();  // warm-up
    for (int r = 0; r < 2; r++) {
      CCFMM_HIP(hipEventRecord(e0, st));
      for (int i = 0; i < kRun; i++) launch();
      CCFMM_HIP(hipEventRecord(e1, st));
      CCFMM_HIP(hipEventSynchronize(e1));
      float t;
      CCFMM_HIP(hipEventElapsedTime(&t, e0, e1));
      best = std::min(best, (double)t / kRun);
    }
  } catch (...) {
    if (gx) (void)hipGraphExecDestroy(gx);
    throw;
  }
  if (gx) (void)hipGraphExecDestroy(gx);
  return best;
}

int ccfmm_plan_autotune(ccfmm_plan plan, int32_t nbatch, const double* d_m, double* d_H, void* stream,
                        ccfmm_tune_entry* out, int32_t max_out, int32_t* n_out) {
  return guarded([&] {
    if (!plan || !plan->P.built) fail(CCFMM_ESTATE, "plan not built");
    if (!d_m || !d_H) fail(CCFMM_EINVAL, "moment or field pointer is NULL");
    Plan& P = plan->P;
    BudgetScope bs(&P.mem);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    CCFMM_HIP(hipSetDevice(P.device));
    prepare_batch(P, nbatch, st);
    // the multipoles the timed launches read
    run_permute(P, nbatch, d_m, st);
    run_p2m(P, nbatch, d_m, st);
    run_m2m(P, nbatch, st);
    hipEvent_t e0, e1;
    CCFMM_HIP(hipEventCreate(&e0));
    CCFMM_HIP(hipEventCreate(&e1));
    std::vector<ccfmm_tune_entry> res;
    // the wide kernels first (usually the fastest); a combination whose first
    // timed launch takes more than twice the best median so far keeps that
    // one timing and is not repeated (on large batches the others cost
    // several times the best per launch)
    const int variants[5] = {kM2LWide1, kM2LWide2, kM2LWide4, kM2LBlock, kM2LWave};
    const int bits[3] = {0, 3, 6};
    double best_ms = INFINITY;
    auto time_m2l = [&]() {
      CCFMM_HIP(hipEventRecord(e0, st));
      run_m2l(P, nbatch, st);
      CCFMM_HIP(hipEventRecord(e1, st));
      CCFMM_HIP(hipEventSynchronize(e1));
      float t;
      CCFMM_HIP(hipEventElapsedTime(&t, e0, e1));
      return t;
    };
    for (int v : variants) {
      if (!m2l_variant_ok(v, P.p, P.precision == CCFMM_PREC_FP64, P.prm.m2l_traceless != 0)) continue;
      for (int cb : bits) {
        P.m2l_variant = v;
        P.class_bits = cb;
        prepare_batch(P, nbatch, st);
        const float first = time_m2l();  // also the warm-up
        if ((double)first > 2.0 * best_ms) {
          res.push_back(ccfmm_tune_entry{v, cb, (double)first, P.nsteps});
          continue;
        }
        std::vector<float> ms;
        for (int r = 0; r < 3; r++) ms.push_back(time_m2l());
        std::sort(ms.begin(), ms.end());
        res.push_back(ccfmm_tune_entry{v, cb, (double)ms[1], P.nsteps});
        best_ms = std::min(best_ms, (double)ms[1]);
      }
    }
    size_t best = 0;
    for (size_t i = 1; i < res.size(); i++)
      if (res[i].m2l_ms < res[best].m2l_ms) best = i;
    P.m2l_variant = res[best].variant;
    P.class_bits = res[best].class_bits;
    prepare_batch(P, nbatch, st);
    P.info.m2l_class_bits = P.class_bits;
    P.info.m2l_variant = P.m2l_variant;
    // the evaluation form: the near field beside the expansion passes (the
    // plan's second stream) or everything on the caller's stream.  Which is
    // faster depends on the workload: where the near field's blocks fill
    // every compute unit, the passes beside it only slow it down.
    P.drop_graph();
    for (int f = 0; f < 2; f++) {
      P.overlap = f == 0;
      P.tune_eval_ms[f] = time_eval_form(P, nbatch, d_m, d_H, st, e0, e1);
    }
    P.overlap = P.tune_eval_ms[0] <= P.tune_eval_ms[1];
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (n_out) *n_out = 0;
    if (out && max_out > 0) {
      const int k = std::min<int>(max_out, (int)res.size());
      for (int i = 0; i < k; i++) out[i] = res[i];
      if (n_out) *n_out = k;
    }
    return CCFMM_OK;
  });
}

int ccfmm_plan_info(ccfmm_plan plan, ccfmm_info* out) {
  return guarded([&] {
    if (!plan || !plan->P.built) fail(CCFMM_ESTATE, "plan not built");
    if (!out) fail(CCFMM_EINVAL, "out is NULL");
    Plan& P = plan->P;
    BudgetScope bs(&P.mem);
    if (P.pairs_stale) {
      // the direct-pair count after an update that kept the lists: taken now,
      // once every stream's work on the plan has finished
      CCFMM_HIP(hipSetDevice(P.device));
      CCFMM_HIP(hipDeviceSynchronize());
      unsigned long long* dcnt = reinterpret_cast<unsigned long long*>(P.scratch2.ensure(64));
      CCFMM_HIP(hipMemsetAsync(dcnt, 0, sizeof(unsigned long long), nullptr));
      launch_pair_count(P, dcnt, nullptr);
      unsigned long long npairs = 0;
      CCFMM_HIP(hipMemcpy(&npairs, dcnt, sizeof(npairs), hipMemcpyDeviceToHost));
      P.info.n_p2p_pairs = (int64_t)npairs;
      P.info.p2p_pairs_per_config = (double)npairs;
      P.pairs_stale = false;
    }
    *out = P.info;
    out->device_bytes = P.mem.used;
    out->overlap_near = P.overlap ? 1 : 0;
    out->tune_eval_ms[0] = P.tune_eval_ms[0];
    out->tune_eval_ms[1] = P.tune_eval_ms[1];
    return CCFMM_OK;
  });
}

int ccfmm_energy(int64_t n, int32_t nbatch, const double* m, const double* H, double* E) {
  return guarded([&] {
    if (n < 1 || nbatch < 1 || !m || !H || !E) fail(CCFMM_EINVAL, "invalid argument");
    for (int b = 0; b < nbatch; b++) {
      double s = 0.0;
      const double* mb = m + (int64_t)b * n * 3;
      const double* hb = H + (int64_t)b * n * 3;
      for (int64_t i = 0; i < 3 * n; i++) s += mb[i] * hb[i];
      E[b] = -0.5 * s;
    }
    return CCFMM_OK;
  });
}

void ccfmm_plan_destroy(ccfmm_plan plan) {
  if (!plan) return;
  try {
    (void)hipSetDevice(plan->P.device);
    (void)hipDeviceSynchronize();
    if (plan->P.own_stream) (void)hipStreamDestroy(plan->P.own_stream);
    delete plan;
  } catch (...) {
  }
}

}  // extern "C"

namespace ccfmm {
// Install (or clear) per-cell parameters given on the host and rebuild every
// list, tile and count that depends on them (the tree is unchanged).
void apply_leaf_params(Plan& P, const int32_t* hp, const double* hth, hipStream_t st) {
  const int nl = P.lev[P.L]->ncells;
  if (hp && hth) {
    std::vector<double> th2(nl);
    double tmin = 1.0;
    for (int i = 0; i < nl; i++) {
      if (hp[i] < 1 || hp[i] > P.p) fail(CCFMM_EINVAL, "per-cell order outside 1..order");
      if (!(hth[i] > 0.0 && hth[i] < 1.0)) fail(CCFMM_EINVAL, "per-cell theta outside (0,1)");
      th2[i] = hth[i] * hth[i];
      tmin = std::min(tmin, hth[i]);
    }
    P.h_leaf_p.assign(hp, hp + nl);
    P.h_leaf_theta.assign(hth, hth + nl);
    P.leaf_p.ensure(sizeof(int32_t) * nl);
    P.leaf_th2.ensure(sizeof(double) * nl);
    CCFMM_HIP(hipMemcpyAsync(P.leaf_p.p, hp, sizeof(int32_t) * nl, hipMemcpyHostToDevice, st));
    CCFMM_HIP(hipMemcpyAsync(P.leaf_th2.p, th2.data(), sizeof(double) * nl, hipMemcpyHostToDevice, st));
    CCFMM_HIP(hipStreamSynchronize(st));
    P.has_leaf = true;
    P.leaf_theta_min = tmin;
  } else {
    P.has_leaf = false;
    P.h_leaf_p.clear();
    P.h_leaf_theta.clear();
  }
  P.drop_graph();
  build_lists(P, st);
  build_dtensors(P, st);
  build_m2l_tiles(P, P.tiles_nb, st);
  fill_info(P, st);
}

// The learned choice on these moments: the fixed-parameter field gives each
// cell's squared field F_c; features -> network -> per-cell (p, theta) with
// the least cost whose predicted global relative RMS error is within
// err_bound x 10^-margin.  With judge, the learned field is compared with the
// fixed one; above the bound the plan returns to the fixed parameters
// (CCFMM_W_FALLBACK).
int select_impl(Plan& P, const float* d_params, double err_bound, double margin, double cost_far, int nbatch,
                const double* d_m, bool judge, hipStream_t st, ccfmm_select_info* out) {
  if (P.has_leaf) apply_leaf_params(P, nullptr, nullptr, st);
  const int nl = P.lev[P.L]->ncells;
  const size_t bytes = sizeof(double) * 3 * (size_t)P.n * nbatch;
  double* Hf = reinterpret_cast<double*>(P.judge_a.ensure(bytes));
  prepare_batch(P, nbatch, st);
  eval_passes(P, nbatch, d_m, Hf, st, nullptr);
  DevBuf dp, dt, dnum, dF;
  dp.ensure(sizeof(int32_t) * nl);
  dt.ensure(sizeof(double) * nl);
  dnum.ensure(sizeof(double) * nl);
  dF.ensure(sizeof(double) * nl);
  run_leaf_errors(P, nbatch, Hf, Hf, dnum.as<double>(), dF.as<double>(), st);
  std::vector<int32_t> hist;
  double pred_err = 0.0;
  run_select(P, d_params, std::log10(err_bound) - margin, cost_far, nbatch, d_m, dF.as<double>(), dp.as<int32_t>(),
             dt.as<double>(), hist, &pred_err, st);
  std::vector<int32_t> hp(nl);
  std::vector<double> ht(nl);
  CCFMM_HIP(hipMemcpyAsync(hp.data(), dp.p, sizeof(int32_t) * nl, hipMemcpyDeviceToHost, st));
  CCFMM_HIP(hipMemcpyAsync(ht.data(), dt.p, sizeof(double) * nl, hipMemcpyDeviceToHost, st));
  CCFMM_HIP(hipStreamSynchronize(st));
  apply_leaf_params(P, hp.data(), ht.data(), st);
  int rc = CCFMM_OK;
  double jerr = 0.0;
  int fb = 0;
  if (judge) {
    double* Hl = reinterpret_cast<double*>(P.judge_b.ensure(bytes));
    prepare_batch(P, nbatch, st);
    eval_passes(P, nbatch, d_m, Hl, st, nullptr);
    jerr = run_rel_rms(Hl, Hf, (int64_t)3 * P.n * nbatch, P.scratch, st);
    if (!(jerr <= err_bound)) {
      apply_leaf_params(P, nullptr, nullptr, st);
      fb = 1;
      rc = CCFMM_W_FALLBACK;
    }
  }
  P.info.fallback = fb;
  P.info.learned = fb ? 0 : 1;
  P.info.judge_err = jerr;
  P.info.sel_cost_far = cost_far;
  if (out) {
    std::memset(out, 0, sizeof(*out));
    out->n_leaves = nl;
    for (int i = 0; i < CCFMM_MLP_OUT && i < (int)hist.size(); i++) out->hist[i] = hist[i];
    out->judge_err = jerr;
    out->fallback = fb;
    out->pred_err = pred_err;
  }
  return rc;
}

// direct pairs of the current lists, if the last update left them uncounted
static void refresh_pair_count(Plan& P) {
  if (!P.pairs_stale) return;
  CCFMM_HIP(hipDeviceSynchronize());
  unsigned long long* dcnt = reinterpret_cast<unsigned long long*>(P.scratch2.ensure(64));
  CCFMM_HIP(hipMemsetAsync(dcnt, 0, sizeof(unsigned long long), nullptr));
  launch_pair_count(P, dcnt, nullptr);
  unsigned long long npairs = 0;
  CCFMM_HIP(hipMemcpy(&npairs, dcnt, sizeof(npairs), hipMemcpyDeviceToHost));
  P.info.n_p2p_pairs = (int64_t)npairs;
  P.info.p2p_pairs_per_config = (double)npairs;
  P.pairs_stale = false;
}

// Cost of one far cell (M2L pair) relative to one direct dipole pair, from
// one evaluation of these moments on the fixed-parameter lists with every
// pass alone on the stream (the second of two, the first warming up).
static double measure_cost_far(Plan& P, int nb, const double* d_m, hipStream_t st) {
  if (P.has_leaf) apply_leaf_params(P, nullptr, nullptr, st);
  refresh_pair_count(P);
  prepare_batch(P, nb, st);
  double* Hs = reinterpret_cast<double*>(P.judge_a.ensure(sizeof(double) * 3 * (size_t)P.n * nb));
  hipEvent_t ev[9];
  create_pass_events(ev, 9, 5);
  const bool overlap = P.overlap;
  P.overlap = false;
  float m2l = 0.f, near = 0.f;
  try {
    // the near field alone (not fused with the smooth field): the per-pair cost
    for (int rep = 0; rep < 2; rep++) eval_passes(P, nb, d_m, Hs, st, ev, false);
    CCFMM_HIP(hipEventSynchronize(ev[5]));
    CCFMM_HIP(hipEventElapsedTime(&m2l, ev[2], ev[3]));
    CCFMM_HIP(hipEventElapsedTime(&near, ev[6], ev[7]));
  } catch (...) {
    P.overlap = overlap;
    for (int i = 0; i < 9; i++) (void)hipEventDestroy(ev[i]);
    throw;
  }
  P.overlap = overlap;
  for (int i = 0; i < 9; i++) (void)hipEventDestroy(ev[i]);
  const double per_m2l = (double)m2l / (double)std::max<int64_t>(1, P.info.n_m2l_pairs);
  const double per_near = (double)near / std::max(1.0, P.info.p2p_pairs_per_config);
  return per_near > 0.0 ? per_m2l / per_near : 1.0;
}

// Learned mode: choose per-cell parameters when the plan has weights and the
// current choice is stale (first evaluation of the cells, new weights).
int auto_select(Plan& P, int nb, const double* d_m, hipStream_t st) {
  if (P.prm.selector != 1 || !P.has_sel_w || !P.sel_stale) return CCFMM_OK;
  const double cf = P.prm.sel_cost_far > 0.0 ? P.prm.sel_cost_far : measure_cost_far(P, nb, d_m, st);
  const int rc = select_impl(P, P.sel_w.as<float>(), P.prm.err_bound, P.prm.sel_margin, cf, nb, d_m, true, st,
                             nullptr);
  P.sel_stale = false;
  return rc;
}
}  // namespace ccfmm

extern "C" {

int ccfmm_plan_set_leaf_params(ccfmm_plan plan, const int32_t* d_p, const double* d_theta, void* stream) {
  return guarded([&] {
    if (!plan || !plan->P.built) fail(CCFMM_ESTATE, "plan not built");
    if ((d_p == nullptr) != (d_theta == nullptr)) fail(CCFMM_EINVAL, "give both per-cell arrays or neither");
    Plan& P = plan->P;
    BudgetScope bs(&P.mem);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    CCFMM_HIP(hipSetDevice(P.device));
    if (!d_p) {
      apply_leaf_params(P, nullptr, nullptr, st);
      return CCFMM_OK;
    }
    const int nl = P.lev[P.L]->ncells;
    std::vector<int32_t> hp(nl);
    std::vector<double> ht(nl);
    CCFMM_HIP(hipMemcpyAsync(hp.data(), d_p, sizeof(int32_t) * nl, hipMemcpyDeviceToHost, st));
    CCFMM_HIP(hipMemcpyAsync(ht.data(), d_theta, sizeof(double) * nl, hipMemcpyDeviceToHost, st));
    CCFMM_HIP(hipStreamSynchronize(st));
    apply_leaf_params(P, hp.data(), ht.data(), st);
    return CCFMM_OK;
  });
}

int ccfmm_plan_get_leaf_params(ccfmm_plan plan, int32_t* h_p, double* h_theta, int32_t* n_leaves) {
  return guarded([&] {
    if (!plan || !plan->P.built) fail(CCFMM_ESTATE, "plan not built");
    Plan& P = plan->P;
    BudgetScope bs(&P.mem);
    const int nl = P.lev[P.L]->ncells;
    if (n_leaves) *n_leaves = nl;
    for (int i = 0; i < nl; i++) {
      if (h_p) h_p[i] = P.has_leaf ? P.h_leaf_p[i] : P.p;
      if (h_theta) h_theta[i] = P.has_leaf ? P.h_leaf_theta[i] : P.prm.theta;
    }
    return CCFMM_OK;
  });
}

int ccfmm_plan_leaf_ids(ccfmm_plan plan, int32_t* d_out, void* stream) {
  return guarded([&] {
    if (!plan || !plan->P.built) fail(CCFMM_ESTATE, "plan not built");
    if (!d_out) fail(CCFMM_EINVAL, "output is NULL");
    BudgetScope bs(&plan->P.mem);
    CCFMM_HIP(hipSetDevice(plan->P.device));
    run_leaf_ids(plan->P, d_out, reinterpret_cast<hipStream_t>(stream));
    return CCFMM_OK;
  });
}

int ccfmm_plan_leaf_features(ccfmm_plan plan, int32_t nbatch, const double* d_m, float* d_feat, void* stream) {
  return guarded([&] {
    if (!plan || !plan->P.built) fail(CCFMM_ESTATE, "plan not built");
    if (!d_m || !d_feat || nbatch < 1) fail(CCFMM_EINVAL, "invalid argument");
    Plan& P = plan->P;
    BudgetScope bs(&P.mem);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    CCFMM_HIP(hipSetDevice(P.device));
    if (P.has_leaf) apply_leaf_params(P, nullptr, nullptr, st);  // features use the fixed lists
    run_leaf_features(P, nbatch, d_m, d_feat, st);
    return CCFMM_OK;
  });
}

int ccfmm_plan_leaf_errors(ccfmm_plan plan, int32_t nbatch, const double* d_H, const double* d_Href, double* d_num,
                           double* d_den, void* stream) {
  return guarded([&] {
    if (!plan || !plan->P.built) fail(CCFMM_ESTATE, "plan not built");
    if (!d_H || !d_Href || !d_num || !d_den || nbatch < 1) fail(CCFMM_EINVAL, "invalid argument");
    BudgetScope bs(&plan->P.mem);
    CCFMM_HIP(hipSetDevice(plan->P.device));
    run_leaf_errors(plan->P, nbatch, d_H, d_Href, d_num, d_den, reinterpret_cast<hipStream_t>(stream));
    return CCFMM_OK;
  });
}

int ccfmm_mlp_forward(const float* d_params, int64_t rows, const float* d_x, float* d_y, void* stream) {
  return guarded([&] {
    if (!d_params || rows < 0 || (rows > 0 && (!d_x || !d_y))) fail(CCFMM_EINVAL, "invalid argument");
    run_mlp_forward(d_params, rows, d_x, d_y, reinterpret_cast<hipStream_t>(stream));
    return CCFMM_OK;
  });
}

// gradient partials (one training loop at a time per process); never freed, so
// nothing touches the runtime during process teardown
static DevBuf& mlp_tmp() {
  static DevBuf* b = new DevBuf();
  return *b;
}

int ccfmm_mlp_loss_grad(const float* d_params, int64_t rows, const float* d_x, const float* d_t, const float* d_mask,
                        float* d_grad, float* d_loss, void* stream) {
  return guarded([&] {
    if (!d_params || !d_grad || rows < 1 || !d_x || !d_t || !d_mask) fail(CCFMM_EINVAL, "invalid argument");
    run_mlp_loss_grad(d_params, rows, d_x, d_t, d_mask, d_grad, d_loss, mlp_tmp(),
                      reinterpret_cast<hipStream_t>(stream));
    return CCFMM_OK;
  });
}

int ccfmm_mlp_adam(float* d_params, const float* d_grad, float* d_m1, float* d_m2, int32_t step, float lr,
                   void* stream) {
  return guarded([&] {
    if (!d_params || !d_grad || !d_m1 || !d_m2 || step < 1 || !(lr > 0.f)) fail(CCFMM_EINVAL, "invalid argument");
    run_mlp_adam(d_params, d_grad, d_m1, d_m2, step, lr, reinterpret_cast<hipStream_t>(stream));
    return CCFMM_OK;
  });
}

int ccfmm_plan_select(ccfmm_plan plan, const float* d_params, double err_bound, double margin, double cost_far,
                      int32_t nbatch, const double* d_m, int32_t judge, void* stream, ccfmm_select_info* out) {
  return guarded([&] {
    if (!plan || !plan->P.built) fail(CCFMM_ESTATE, "plan not built");
    if (!d_params || !d_m || !(err_bound > 0.0) || !(cost_far >= 0.0)) fail(CCFMM_EINVAL, "invalid argument");
    Plan& P = plan->P;
    BudgetScope bs(&P.mem);
    if (nbatch < 1 || nbatch > P.nbmax) fail(CCFMM_EINVAL, "nbatch must be in 1..max_batch");
    // the candidate orders are 2..6: a plan of order 1 has none
    if (P.p < 2) fail(CCFMM_EINVAL, "learned selection needs a plan of order >= 2");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    CCFMM_HIP(hipSetDevice(P.device));
    return select_impl(P, d_params, err_bound, margin, cost_far, nbatch, d_m, judge != 0, st, out);
  });
}

int ccfmm_selector_write(const char* path, const float* h_params) {
  return guarded([&] {
    selector_file_write(path, h_params);
    return CCFMM_OK;
  });
}

int ccfmm_selector_read(const char* path, float* h_params) {
  return guarded([&] {
    std::vector<float> h(CCFMM_MLP_PARAMS);
    if (!selector_file_read(path, h.data())) {
      g_last_error = std::string("selector weights file not found: ") + (path ? path : "");
      return CCFMM_W_NOWEIGHTS;
    }
    std::copy(h.begin(), h.end(), h_params);
    return CCFMM_OK;
  });
}

// new weights in the plan: a learned plan chooses again at its next evaluation
static void install_weights(Plan& P, const void* src, hipMemcpyKind kind, hipStream_t st) {
  P.sel_w.ensure(sizeof(float) * CCFMM_MLP_PARAMS);
  CCFMM_HIP(hipMemcpyAsync(P.sel_w.p, src, sizeof(float) * CCFMM_MLP_PARAMS, kind, st));
  CCFMM_HIP(hipStreamSynchronize(st));
  P.has_sel_w = true;
  P.sel_stale = true;
}

int ccfmm_selector_load(ccfmm_plan plan, const char* path) {
  return guarded([&] {
    if (!plan || !plan->P.ever_built) fail(CCFMM_ESTATE, "plan not built");
    Plan& P = plan->P;
    BudgetScope bs(&P.mem);
    std::vector<float> h(CCFMM_MLP_PARAMS);
    if (!selector_file_read(path, h.data())) {
      g_last_error = std::string("selector weights file not found, fixed parameters kept: ") + (path ? path : "");
      return CCFMM_W_NOWEIGHTS;
    }
    CCFMM_HIP(hipSetDevice(P.device));
    install_weights(P, h.data(), hipMemcpyHostToDevice, nullptr);
    return CCFMM_OK;
  });
}

int ccfmm_selector_set(ccfmm_plan plan, const float* d_params, void* stream) {
  return guarded([&] {
    if (!plan || !plan->P.ever_built) fail(CCFMM_ESTATE, "plan not built");
    if (!d_params) fail(CCFMM_EINVAL, "parameters are NULL");
    BudgetScope bs(&plan->P.mem);
    CCFMM_HIP(hipSetDevice(plan->P.device));
    install_weights(plan->P, d_params, hipMemcpyDeviceToDevice, reinterpret_cast<hipStream_t>(stream));
    return CCFMM_OK;
  });
}

int ccfmm_selector_save(ccfmm_plan plan, const char* path) {
  return guarded([&] {
    if (!plan || !plan->P.ever_built) fail(CCFMM_ESTATE, "plan not built");
    Plan& P = plan->P;
    BudgetScope bs(&P.mem);
    if (!P.has_sel_w) fail(CCFMM_ESTATE, "the plan holds no selector weights");
    CCFMM_HIP(hipSetDevice(P.device));
    std::vector<float> h(CCFMM_MLP_PARAMS);
    CCFMM_HIP(hipMemcpy(h.data(), P.sel_w.p, sizeof(float) * CCFMM_MLP_PARAMS, hipMemcpyDeviceToHost));
    selector_file_write(path, h.data());
    return CCFMM_OK;
  });
}

int ccfmm_selector_train(const ccfmm_train_spec* spec, const char* out_path, float* h_params_out,
                         ccfmm_train_info* info) {
  return guarded([&] {
    train_selector(spec, out_path, h_params_out, info);
    return CCFMM_OK;
  });
}

int ccfmm_plan_energy_device(ccfmm_plan plan, int32_t nbatch, const double* d_m, const double* d_H, double* d_E,
                             void* stream) {
  return guarded([&] {
    if (!plan || !plan->P.built) fail(CCFMM_ESTATE, "plan not built");
    if (nbatch < 1 || !d_m || !d_H || !d_E) fail(CCFMM_EINVAL, "invalid argument");
    Plan& P = plan->P;
    BudgetScope bs(&P.mem);
    CCFMM_HIP(hipSetDevice(P.device));
    run_energy(P, nbatch, d_m, d_H, d_E, reinterpret_cast<hipStream_t>(stream));
    return CCFMM_OK;
  });
}

int ccfmm_energy_device_noalloc(int64_t n, int32_t nbatch, const double* d_m, const double* d_H, double* d_E,
                                void* stream) {
  return guarded([&] {
    if (n < 1 || !d_m || !d_H || !d_E) fail(CCFMM_EINVAL, "invalid argument");
    run_energy_noalloc(n, nbatch, d_m, d_H, d_E, reinterpret_cast<hipStream_t>(stream));
    return CCFMM_OK;
  });
}

int ccfmm_direct_targets_device(int64_t n, const double* d_pos, const double* d_m, int64_t nt, const int64_t* d_idx,
                                double* d_H, void* stream) {
  return guarded([&] {
    if (n < 1 || nt < 0 || !d_pos || !d_m || (nt > 0 && (!d_idx || !d_H))) fail(CCFMM_EINVAL, "invalid argument");
    run_direct_targets(n, d_pos, d_m, nt, d_idx, d_H, reinterpret_cast<hipStream_t>(stream));
    return CCFMM_OK;
  });
}

int ccfmm_selftest_mfma(int32_t device) {
  return guarded([&] { return selftest_mfma_impl(device); });
}

}  // extern "C"
