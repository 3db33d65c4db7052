// tree.hip -- bisection tree on the GPU: leaf keys, stable radix sort,
// smallest-cell ranges, sorted SoA offsets and the occupied cells per level.
//
// The system box is halved recursively (Sec. 2); level l halves the longest
// side of the level-(l-1) cell, ties x < y < z, so the smallest cells are as
// cubic as the halving allows (Sec. 4).  The key of a cell at level l is the
// sequence of its l half-choices (1 = upper half), so the children of key k
// are 2k and 2k+1 and a dipole's smallest-cell key orders dipoles cell by
// cell (a Morton order in the split sequence).
#include "plan.hpp"

namespace ccfmm {

// ---------------------------------------------------------------- scan
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t* sh, int32_t& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    int32_t add = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int32_t incl = sh[t];
  total = sh[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const int32_t* in, int32_t* out,
                                                             int32_t* sums, int64_t n) {
  __shared__ int32_t sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int32_t s = 0;
  for (int i = 0; i < kScanItems; i++) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    s += v[i];
  }
  int32_t total;
  int32_t ex = block_exclusive_scan(s, sh, total);
  for (int i = 0; i < kScanItems; i++) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void k_scan_add(int32_t* out, const int32_t* sums, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
  const int32_t add = sums[blockIdx.x];
  for (int r = 0; r < kScanItems; r++) {
    int64_t j = i + (int64_t)r * kScanThreads;
    if (j < n) out[j] += add;
  }
}

static void scan_rec(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, hipStream_t st) {
  const int nb = ceil_div(n, kScanTile);
  int32_t* sums = tmp;
  k_scan_tiles<<<nb, kScanThreads, 0, st>>>(in, out, sums, n);
  CCFMM_HIP(hipGetLastError());
  if (nb > 1) {
    scan_rec(sums, sums, nb, tmp + nb, st);
    k_scan_add<<<nb, kScanThreads, 0, st>>>(out, sums, n);
    CCFMM_HIP(hipGetLastError());
  }
}

__global__ void k_copy_last(const int32_t* in, int64_t n, int32_t* last) {
  if (threadIdx.x == 0 && blockIdx.x == 0) last[0] = (n > 0) ? in[n - 1] : 0;
}
__global__ void k_finish_total(int32_t* out, int64_t n, const int32_t* last) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[n] = (n > 0) ? out[n - 1] + last[0] : 0;
}

// One block scans up to kScanSingleMax values in a single launch, in chunks of
// 16384 values: wavefront w owns the 16 rows of 64 consecutive values from
// 1024 w, and lane l holds column l of each row, so every load and store
// covers 64 consecutive words.  Each row is scanned by shuffles and offset by
// the rows before it; the 16 wavefront totals are scanned by the first
// wavefront, and a carry links the chunks.  All loads of a chunk are issued
// before any is used.  The total lands in out[n] (out may alias in: each
// value is read before it is written, by the same lane).
constexpr int kScanSingleThreads = 1024;
constexpr int kScanSingleRows = 16;
constexpr int64_t kScanSingleMax = 64 * kScanSingleThreads;

__device__ __forceinline__ int32_t wave_incl_scan(int32_t x, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  return x;
}

__device__ __forceinline__ void scan_single_block(const int32_t* in, int32_t* out, int64_t n) {
  constexpr int NW = kScanSingleThreads / 64;
  constexpr int R = kScanSingleRows;
  constexpr int CH = R * kScanSingleThreads;
  __shared__ int32_t wsum[NW];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int32_t carry = 0;
  for (int64_t c0 = 0; c0 < n; c0 += CH) {
    const int64_t m = min((int64_t)CH, n - c0);
    const int32_t base = w * (R * 64) + lane;  // row i of this wavefront: base + 64 i
    // rows of this wavefront that hold values (the rest are zero and skipped)
    const int rows = (int)max((int64_t)0, min((int64_t)R, (m - (int64_t)w * R * 64 + 63) / 64));
    const int32_t* src = in + c0;
    int32_t v[R];
#pragma unroll
    for (int i = 0; i < R; i++) v[i] = (base + 64 * i < m) ? src[base + 64 * i] : 0;
    int32_t rowoff = 0;  // sum of this wavefront's rows before row i
#pragma unroll
    for (int i = 0; i < R; i++) {
      if (i >= rows) break;
      const int32_t x = wave_incl_scan(v[i], lane);
      const int32_t ex = rowoff + x - v[i];
      rowoff += __builtin_amdgcn_readlane(x, 63);
      v[i] = ex;  // exclusive prefix inside the wavefront's segment
    }
    if (lane == 0) wsum[w] = rowoff;
    __syncthreads();
    if (w == 0) {
      int32_t x = lane < NW ? wsum[lane] : 0;
      x = wave_incl_scan(x, lane);
      if (lane < NW) wsum[lane] = x;
    }
    __syncthreads();
    const int32_t add = carry + (w > 0 ? wsum[w - 1] : 0);
    int32_t* dst = out + c0;
#pragma unroll
    for (int i = 0; i < R; i++)
      if (base + 64 * i < m) dst[base + 64 * i] = add + v[i];
    carry += wsum[NW - 1];
    __syncthreads();  // wsum is rewritten by the next chunk
  }
  if (t == 0) out[n] = carry;
}

__global__ void __launch_bounds__(kScanSingleThreads) k_scan_single(const int32_t* in, int32_t* out, int64_t n) {
  scan_single_block(in, out, n);
}

// two arrays of the same length scanned in one launch (one block each)
__global__ void __launch_bounds__(kScanSingleThreads) k_scan_single2(const int32_t* in0, int32_t* out0,
                                                                     const int32_t* in1, int32_t* out1, int64_t n) {
  if (blockIdx.x == 0)
    scan_single_block(in0, out0, n);
  else
    scan_single_block(in1, out1, n);
}

void scan_exclusive2(const int32_t* in0, int32_t* out0, const int32_t* in1, int32_t* out1, int64_t n, DevBuf& tmp,
                     hipStream_t st) {
  if (n <= kScanSingleMax) {
    k_scan_single2<<<2, kScanSingleThreads, 0, st>>>(in0, out0, in1, out1, n < 0 ? 0 : n);
    CCFMM_HIP(hipGetLastError());
    return;
  }
  scan_exclusive(in0, out0, n, tmp, st);
  scan_exclusive(in1, out1, n, tmp, st);
}

void scan_exclusive(const int32_t* in, int32_t* out, int64_t n, DevBuf& tmp, hipStream_t st) {
  if (n <= kScanSingleMax) {
    k_scan_single<<<1, kScanSingleThreads, 0, st>>>(in, out, n < 0 ? 0 : n);
    CCFMM_HIP(hipGetLastError());
    return;
  }
  // temporaries: block sums of every recursion level + the saved last input
  int64_t need = 4;
  for (int64_t m = n; m > 1; m = ceil_div(m, kScanTile)) need += ceil_div(m, kScanTile) + 1;
  int32_t* t = reinterpret_cast<int32_t*>(tmp.ensure(sizeof(int32_t) * (need + 8)));
  if (n <= 0) {
    k_finish_total<<<1, 1, 0, st>>>(out, 0, t);
    return;
  }
  k_copy_last<<<1, 1, 0, st>>>(in, n, t);
  scan_rec(in, out, n, t + 4, st);
  k_finish_total<<<1, 1, 0, st>>>(out, n, t);
  CCFMM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- radix sort
// Stable LSD radix sort, 8-bit digits.  Each block owns a tile of
// kSortThreads * kSortRounds keys processed in rounds of kSortThreads; inside
// a round the rank of a key among equal digits of lower thread index comes
// from wavefront ballots, then a prefix over the block's wavefronts.
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;
constexpr int kWaves = kSortThreads / 64;

__global__ void __launch_bounds__(kSortThreads) k_digit_hist(const uint32_t* key, int64_t n, int shift,
                                                             int32_t* hist, int nblocks) {
  __shared__ int32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; r++) {
    int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(key[i] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(kSortThreads) k_digit_scatter(const uint32_t* key, const int32_t* val,
                                                                uint32_t* key_out, int32_t* val_out,
                                                                int64_t n, int shift,
                                                                const int32_t* offs, int nblocks) {
  __shared__ int32_t base[256];
  __shared__ int32_t wcnt[kWaves][256];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  base[t] = offs[(int64_t)t * nblocks + blockIdx.x];
  const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kSortRounds; r++) {
    for (int q = 0; q < kWaves; q++) wcnt[q][t] = 0;
    __syncthreads();
    const int64_t i = tile0 + (int64_t)r * kSortThreads + t;
    const bool valid = i < n;
    uint32_t k = valid ? key[i] : 0u;
    int32_t v = valid ? val[i] : 0;
    const uint32_t d = (k >> shift) & 255u;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < 8; b++) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & lt);
    if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    // prefix over wavefronts for digit t, and this round's total
    int32_t run = 0;
    int32_t pre[kWaves];
    for (int q = 0; q < kWaves; q++) {
      pre[q] = run;
      run += wcnt[q][t];
    }
    __syncthreads();
    for (int q = 0; q < kWaves; q++) wcnt[q][t] = pre[q];
    __syncthreads();
    if (valid) {
      const int32_t pos = base[d] + wcnt[w][d] + rank;
      key_out[pos] = k;
      val_out[pos] = v;
    }
    __syncthreads();
    base[t] += run;
    __syncthreads();
  }
}

void radix_sort_pairs(uint32_t* key, int32_t* val, uint32_t* key_tmp, int32_t* val_tmp, int64_t n,
                      int bits, DevBuf& tmp, hipStream_t st) {
  if (n <= 1 || bits <= 0) return;
  const int nblocks = ceil_div(n, kSortTile);
  const int64_t nh = (int64_t)256 * nblocks;
  // histogram + its scan live behind the scan temporaries in a second region
  DevBuf& hb = tmp;
  int64_t scan_need = 4;
  for (int64_t m = nh; m > 1; m = ceil_div(m, kScanTile)) scan_need += ceil_div(m, kScanTile) + 1;
  size_t bytes = sizeof(int32_t) * (2 * (nh + 1) + scan_need + 16);
  int32_t* h = reinterpret_cast<int32_t*>(hb.ensure(bytes));
  int32_t* hist = h;
  int32_t* offs = h + nh + 1;
  int32_t* stmp = offs + nh + 1;
  uint32_t* kin = key;
  int32_t* vin = val;
  uint32_t* kout = key_tmp;
  int32_t* vout = val_tmp;
  int passes = (bits + 7) / 8;
  for (int ps = 0; ps < passes; ps++) {
    const int shift = 8 * ps;
    k_digit_hist<<<nblocks, kSortThreads, 0, st>>>(kin, n, shift, hist, nblocks);
    CCFMM_HIP(hipGetLastError());
    // exclusive scan of the digit-major histogram
    scan_rec(hist, offs, nh, stmp + 4, st);
    k_digit_scatter<<<nblocks, kSortThreads, 0, st>>>(kin, vin, kout, vout, n, shift, offs, nblocks);
    CCFMM_HIP(hipGetLastError());
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  if (kin != key) {
    CCFMM_HIP(hipMemcpyAsync(key, kin, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));
    CCFMM_HIP(hipMemcpyAsync(val, vin, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  }
}

// ---------------------------------------------------------------- tree
// Smallest-cell coordinate along one axis: floor((x - lo) 2^k / W) clamped to
// [0, 2^k - 1] (a point on a face goes to the upper cell, the top face to the
// last cell), with exactly this IEEE sequence and no contraction.
__device__ __forceinline__ int32_t leaf_coord(double x, double lo, double W, int k) {
#pragma clang fp contract(off)
  double t = x - lo;
  t = t * ldexp(1.0, k);
  double u = t / W;
  double f = floor(u);
  int32_t top = (1 << k) - 1;
  if (!(f >= 0.0)) return 0;  // below the box, or not a number
  if (f > (double)top) return top;
  return (int32_t)f;
}

__global__ void k_leaf_keys(const double* __restrict__ pos, int64_t n, TreeGeom G, uint32_t* key,
                            int32_t* val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int L = G.L;
  int32_t c[3];
  for (int a = 0; a < 3; a++) c[a] = leaf_coord(pos[3 * i + a], G.lo[a], G.W[a], G.lev[L].k[a]);
  uint32_t k = 0;
  for (int l = 1; l <= L; l++) {
    const int a = G.lev[l].axis;
    const uint32_t bit = (uint32_t)(c[a] >> (G.lev[L].k[a] - G.lev[l].k[a])) & 1u;
    k = (k << 1) | bit;
  }
  key[i] = k;
  val[i] = (int32_t)i;
}

// Occupied cells at every depth 0..24 from one sort of the depth-24 keys: the
// depth-l key of a dipole is the top l bits of its depth-24 key (the leaf
// index at depth l is the depth-24 index shifted right, since scaling by a
// power of two commutes with the rounding), so neighbours in sorted order
// that first differ at depth l add one occupied cell at every depth >= l.
__global__ void __launch_bounds__(256) k_first_diff_hist(const uint32_t* __restrict__ key, int64_t n, int32_t* hist) {
  __shared__ int32_t h[32];
  if (threadIdx.x < 32) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 1 && i < n) {
    const uint32_t x = key[i] ^ key[i - 1];
    if (x) atomicAdd(&h[24 - (31 - __clz(x))], 1);
  }
  __syncthreads();
  if (threadIdx.x < 25 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void k_zero_i32(int32_t* p, int n) {
  const int i = threadIdx.x;
  if (i < n) p[i] = 0;
}

void count_occupied_by_depth(Plan& P, const double* d_pos, const TreeGeom& G24, hipStream_t st, int64_t* occupied) {
  const int64_t n = P.n;
  const int T = 256;
  uint32_t* key = reinterpret_cast<uint32_t*>(P.key.ensure(sizeof(uint32_t) * n));
  int32_t* val = reinterpret_cast<int32_t*>(P.val.ensure(sizeof(int32_t) * n));
  uint32_t* key2 = reinterpret_cast<uint32_t*>(P.key_tmp.ensure(sizeof(uint32_t) * n));
  int32_t* val2 = reinterpret_cast<int32_t*>(P.val_tmp.ensure(sizeof(int32_t) * n));
  k_leaf_keys<<<ceil_div(n, T), T, 0, st>>>(d_pos, n, G24, key, val);
  CCFMM_HIP(hipGetLastError());
  radix_sort_pairs(key, val, key2, val2, n, 24, P.scratch, st);
  int32_t* hist = reinterpret_cast<int32_t*>(P.scratch2.ensure(sizeof(int32_t) * 32));
  k_zero_i32<<<1, 32, 0, st>>>(hist, 32);
  CCFMM_HIP(hipGetLastError());
  k_first_diff_hist<<<ceil_div(n, T), T, 0, st>>>(key, n, hist);
  CCFMM_HIP(hipGetLastError());
  int32_t h[32];
  CCFMM_HIP(hipMemcpyAsync(h, hist, sizeof(h), hipMemcpyDeviceToHost, st));
  CCFMM_HIP(hipStreamSynchronize(st));
  int64_t c = 1;
  occupied[0] = 1;
  for (int l = 1; l <= 24; l++) {
    c += h[l];
    occupied[l] = c;
  }
}

// integer coordinates of the cell with key `key` at level l
__device__ __forceinline__ void cell_coords(const TreeGeom& G, int l, uint32_t key, int32_t c[3]) {
  c[0] = c[1] = c[2] = 0;
  for (int j = 1; j <= l; j++) {
    const int a = G.lev[j].axis;
    const int32_t bit = (int32_t)((key >> (l - j)) & 1u);
    c[a] |= bit << (G.lev[l].k[a] - G.lev[j].k[a]);
  }
}

__global__ void k_leaf_start(const uint32_t* key, int64_t n, int64_t nleaf, int32_t* start) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k > nleaf) return;
  // lower bound of k in the sorted keys
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if ((int64_t)key[mid] < k)
      lo = mid + 1;
    else
      hi = mid;
  }
  start[k] = (int32_t)lo;
}

// yd (FP64 coordinates) only for FP64 plans: null skips it
__global__ void k_gather_sorted(const double* __restrict__ pos, const uint32_t* __restrict__ key,
                                const int32_t* __restrict__ perm, int64_t n, TreeGeom G, double inv_s, double* yd,
                                float* yf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int L = G.L;
  int32_t c[3];
  cell_coords(G, L, key[i], c);
  const int64_t src = perm[i];
  for (int a = 0; a < 3; a++) {
    const double center = G.lo[a] + ((double)c[a] + 0.5) * G.lev[L].h[a];
    const double y = (pos[3 * src + a] - center) * inv_s;
    if (yd) yd[a * n + i] = y;
    const float hi = (float)y;
    yf[a * n + i] = hi;
    yf[(3 + a) * n + i] = (float)(y - (double)hi);  // residual: y = hi + lo to ~1e-16
  }
}

// occupancy of every heap cell (level l, key k) <-> heap id 2^l - 1 + k
__global__ void k_heap_flags(const int32_t* __restrict__ leaf_start, int L, int64_t nheap,
                             int32_t* flag) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nheap) return;
  int l = 63 - __clzll((unsigned long long)(h + 1));
  int64_t k = h - ((1ll << l) - 1);
  int sh = L - l;
  int64_t a = k << sh, b = (k + 1) << sh;
  flag[h] = (leaf_start[b] > leaf_start[a]) ? 1 : 0;
}

struct LevelPtrs {
  int32_t* key[kLMax + 1];
  int32_t* parent[kLMax + 1];
  int32_t* child[kLMax + 1];
  int64_t start[kLMax + 2];  // compact start of each level in the heap scan
};

__global__ void k_compact_cells(const int32_t* __restrict__ flag, const int32_t* __restrict__ scan,
                                int L, int64_t nheap, LevelPtrs lp, int32_t* cmap) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nheap) return;
  int l = 63 - __clzll((unsigned long long)(h + 1));
  if (!flag[h]) {
    cmap[h] = -1;
    return;
  }
  const int32_t c = (int32_t)(scan[h] - lp.start[l]);
  cmap[h] = c;
  const int64_t k = h - ((1ll << l) - 1);
  lp.key[l][c] = (int32_t)k;
}

__global__ void k_link_cells(const int32_t* __restrict__ flag, const int32_t* __restrict__ cmap, int L,
                             int64_t nheap, LevelPtrs lp) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nheap || !flag[h]) return;
  int l = 63 - __clzll((unsigned long long)(h + 1));
  const int32_t c = cmap[h];
  if (l > 0) lp.parent[l][c] = cmap[(h - 1) >> 1];
  if (l < L) {
    lp.child[l][2 * c] = cmap[2 * h + 1];
    lp.child[l][2 * c + 1] = cmap[2 * h + 2];
  }
}

// integer coordinates of every cell of every level (global index = compact
// start of the level + compact index)
struct LevelCoords {
  int32_t* coord[kLMax + 1];
};
__global__ void k_cell_coords(LevelPtrs lp, LevelCoords lc, int L, TreeGeom G) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= lp.start[L + 1]) return;
  int l = 0;
  while (l < L && i >= lp.start[l + 1]) l++;
  const int64_t c = i - lp.start[l];
  int32_t x[3];
  cell_coords(G, l, (uint32_t)lp.key[l][c], x);
  lc.coord[l][3 * c] = x[0];
  lc.coord[l][3 * c + 1] = x[1];
  lc.coord[l][3 * c + 2] = x[2];
}

__global__ void k_leaf_ranges(const int32_t* __restrict__ lkey, const int32_t* __restrict__ leaf_start,
                              int32_t nl, int32_t* lstart, int32_t* lcount) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nl) return;
  const int32_t k = lkey[i];
  lstart[i] = leaf_start[k];
  lcount[i] = leaf_start[k + 1] - leaf_start[k];
}

// level starts in the heap scan: scan[2^l - 1], l = 0..L+1
__global__ void k_level_starts(const int32_t* scan, int L, int32_t* out) {
  const int l = threadIdx.x;
  if (l <= L + 1) out[l] = scan[(1ll << l) - 1];
}

// 1 into *diff if the occupancy of any heap cell differs from the previous build's
__global__ void k_flags_differ(const int32_t* __restrict__ a, const int32_t* __restrict__ b, int64_t n,
                               int32_t* diff) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && a[i] != b[i]) *diff = 1;  // every writer stores the same value
}

// same_cells (optional): set to whether every heap cell's occupancy equals the
// previous build's (read back with the level sizes, no extra wait).
// d_check (optional): two device words copied to h_check in the same wait.
void build_tree(Plan& P, const double* d_pos, hipStream_t st, bool* same_cells, const int32_t* d_check,
                int32_t* h_check) {
  const int64_t n = P.n;
  const int L = P.L;
  TreeGeom& G = P.geo;
  const int T = 256;
  uint32_t* key = P.key.as<uint32_t>();
  int32_t* val = P.val.as<int32_t>();
  k_leaf_keys<<<ceil_div(n, T), T, 0, st>>>(d_pos, n, G, key, val);
  CCFMM_HIP(hipGetLastError());
  radix_sort_pairs(key, val, P.key_tmp.as<uint32_t>(), P.val_tmp.as<int32_t>(), n, L, P.scratch, st);
  const int64_t nleaf = 1ll << L;
  int32_t* ls = P.leaf_start.as<int32_t>();
  k_leaf_start<<<ceil_div(nleaf + 1, T), T, 0, st>>>(key, n, nleaf, ls);
  CCFMM_HIP(hipGetLastError());
  // sorted -> input order is the sorted val array
  CCFMM_HIP(hipMemcpyAsync(P.perm.p, val, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  k_gather_sorted<<<ceil_div(n, T), T, 0, st>>>(d_pos, key, P.perm.as<int32_t>(), n, G, 1.0 / G.lev[L].s,
                                                P.precision == CCFMM_PREC_FP64 ? P.yd.as<double>() : nullptr,
                                                P.yf.as<float>());
  CCFMM_HIP(hipGetLastError());

  const int64_t nheap = (2ll << L) - 1;
  int32_t* flag = P.heap_flag.as<int32_t>();
  int32_t* scan = P.heap_scan.as<int32_t>();
  k_heap_flags<<<ceil_div(nheap, T), T, 0, st>>>(ls, L, nheap, flag);
  CCFMM_HIP(hipGetLastError());
  int32_t* g = reinterpret_cast<int32_t*>(P.scratch2.ensure(sizeof(int32_t) * (L + 3)));
  const bool compare = same_cells && P.heap_flag_prev.cap >= sizeof(int32_t) * (size_t)nheap;
  if (compare) {
    k_zero_i32<<<1, 64, 0, st>>>(g + L + 2, 1);
    k_flags_differ<<<ceil_div(nheap, T), T, 0, st>>>(flag, P.heap_flag_prev.as<int32_t>(), nheap, g + L + 2);
    CCFMM_HIP(hipGetLastError());
    // the verdict first: with every cell's occupancy as before, the compact
    // cells, their links, coordinates and level sizes are those of the
    // previous build, and only the dipole ranges of the smallest cells change
    int32_t differ = 1;
    CCFMM_HIP(hipMemcpyAsync(&differ, g + L + 2, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (d_check) CCFMM_HIP(hipMemcpyAsync(h_check, d_check, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, st));
    CCFMM_HIP(hipStreamSynchronize(st));
    d_check = nullptr;  // read
    if (differ == 0) {
      *same_cells = true;
      const int32_t nl = P.lev[L]->ncells;
      k_leaf_ranges<<<ceil_div(nl, T), T, 0, st>>>(P.lev[L]->key.as<int32_t>(), ls, nl, P.lstart.as<int32_t>(),
                                                    P.lcount.as<int32_t>());
      CCFMM_HIP(hipGetLastError());
      return;
    }
  }
  int32_t* prev = reinterpret_cast<int32_t*>(P.heap_flag_prev.ensure(sizeof(int32_t) * nheap));
  CCFMM_HIP(hipMemcpyAsync(prev, flag, sizeof(int32_t) * nheap, hipMemcpyDeviceToDevice, st));
  scan_exclusive(flag, scan, nheap, P.scratch, st);
  // level starts: scan[2^l - 1] for l = 0..L+1 (the last is the total), then
  // the occupancy-changed word
  std::vector<int32_t> starts(L + 3, 1);
  {
    k_level_starts<<<1, 64, 0, st>>>(scan, L, g);
    CCFMM_HIP(hipGetLastError());
    CCFMM_HIP(hipMemcpyAsync(starts.data(), g, sizeof(int32_t) * (compare ? L + 3 : L + 2), hipMemcpyDeviceToHost,
                             st));
    if (d_check) CCFMM_HIP(hipMemcpyAsync(h_check, d_check, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, st));
    CCFMM_HIP(hipStreamSynchronize(st));
  }
  if (same_cells) *same_cells = false;  // a kept tree returned above
  LevelPtrs lp{};
  for (int l = 0; l <= L; l++) {
    LevelData& D = *P.lev[l];
    D.ncells = starts[l + 1] - starts[l];
    D.heap0 = (1ll << l) - 1;
    const int nc = D.ncells > 0 ? D.ncells : 1;
    lp.key[l] = reinterpret_cast<int32_t*>(D.key.ensure(sizeof(int32_t) * nc));
    lp.parent[l] = reinterpret_cast<int32_t*>(D.parent.ensure(sizeof(int32_t) * nc));
    lp.child[l] = reinterpret_cast<int32_t*>(D.child.ensure(sizeof(int32_t) * 2 * nc));
    lp.start[l] = starts[l];
  }
  lp.start[L + 1] = starts[L + 1];
  int32_t* cmap = P.cmap.as<int32_t>();
  k_compact_cells<<<ceil_div(nheap, T), T, 0, st>>>(flag, scan, L, nheap, lp, cmap);
  CCFMM_HIP(hipGetLastError());
  k_link_cells<<<ceil_div(nheap, T), T, 0, st>>>(flag, cmap, L, nheap, lp);
  CCFMM_HIP(hipGetLastError());
  LevelCoords lc{};
  for (int l = 0; l <= L; l++) {
    LevelData& D = *P.lev[l];
    lc.coord[l] = reinterpret_cast<int32_t*>(D.coord.ensure(sizeof(int32_t) * 3 * (D.ncells > 0 ? D.ncells : 1)));
  }
  k_cell_coords<<<ceil_div(lp.start[L + 1], T), T, 0, st>>>(lp, lc, L, G);
  CCFMM_HIP(hipGetLastError());
  const int32_t nl = P.lev[L]->ncells;
  P.lstart.ensure(sizeof(int32_t) * nl);
  P.lcount.ensure(sizeof(int32_t) * nl);
  k_leaf_ranges<<<ceil_div(nl, T), T, 0, st>>>(lp.key[L], ls, nl, P.lstart.as<int32_t>(),
                                                P.lcount.as<int32_t>());
  CCFMM_HIP(hipGetLastError());
}

}  // namespace ccfmm
