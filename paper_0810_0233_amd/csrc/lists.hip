// lists.hip -- near/far cell lists (Sec. 2 and Appendix, createPartners),
// the M2L work tiles and the P2P work chunks, all built on the GPU.
//
// Level by level, the candidates of a cell are the children of the cells near
// its parent (the parent itself included, which supplies the sibling).  A
// candidate at opening angle 2r/d > theta is near (passed down, or kept for
// the near-field sum at the smallest cells); otherwise it is far and enters
// the cell's M2L list.  Empty cells are never created, which leaves every
// field unchanged (their moments vanish and they hold no field points).
//
// One wavefront per cell walks its candidates 256 at a time (four ballot
// rounds whose loads are in flight together); ballots give each
// near/far candidate its slot, so the lists come out in candidate order, the
// same order a serial walk produces.  Buffers are sized from exact per-cell
// bounds computed on the host, so no level waits on the host.
#include <algorithm>
#include <cmath>

#include "plan.hpp"

namespace ccfmm {

// Exact opening-angle test.  With delta the integer offset of the two cells
// and g the cell sides over the smallest side, alpha = |g| / |delta*g|; the
// pair is far iff theta^2 |delta*g|^2 >= |g|^2 (alpha == theta is far).  The
// sums run x, y, z with no contraction.
__host__ __device__ __forceinline__ bool is_near(const LevelGeom& lg, double theta2, int dx, int dy, int dz) {
#pragma clang fp contract(off)
  const double ax = (double)dx * lg.g[0];
  const double ay = (double)dy * lg.g[1];
  const double az = (double)dz * lg.g[2];
  double D = ax * ax;
  D = D + ay * ay;
  D = D + az * az;
  double R = lg.g[0] * lg.g[0];
  R = R + lg.g[1] * lg.g[1];
  R = R + lg.g[2] * lg.g[2];
  const bool far = (theta2 * D >= R);
  return !far;
}

struct ListArgs {
  const int32_t* parent;      // level l
  const int32_t* coord;       // level l
  const int32_t* pnear_ptr;   // level l-1
  const int32_t* pnear_idx;
  const int32_t* pchild;      // level l-1
  const double* cell_th2;     // per-cell squared opening angle (smallest cells), or null
  int32_t ncells;
  int level;
  double theta2;
  int wfar[3];
  int64_t near_cap, far_cap;
};

__device__ __forceinline__ uint64_t lanemask_lt(int lane) { return lane ? (~0ull >> (64 - lane)) : 0ull; }

// Candidate i of cell c: child (i & 1) of the (i >> 1)-th near cell of the parent.
// A lane takes candidates i, i + 64, i + 128, i + 192 (kCandRounds rounds of
// a wavefront) and issues their dependent loads together; X = -1: none.
constexpr int kCandRounds = 4;
struct Cands {
  int X[kCandRounds];
  int d[kCandRounds][3];  // candidate minus cell, integer offset
};
__device__ __forceinline__ Cands load_cands(const ListArgs& a, int e0, int ncand, int i0, int cx, int cy, int cz) {
  Cands q;
  int pn[kCandRounds];
#pragma unroll
  for (int u = 0; u < kCandRounds; u++) {
    const int i = i0 + 64 * u;
    pn[u] = i < ncand ? a.pnear_idx[e0 + (i >> 1)] : -1;
  }
#pragma unroll
  for (int u = 0; u < kCandRounds; u++) q.X[u] = pn[u] >= 0 ? a.pchild[2 * pn[u] + ((i0 + 64 * u) & 1)] : -1;
#pragma unroll
  for (int u = 0; u < kCandRounds; u++) {
    const int X = q.X[u] >= 0 ? q.X[u] : 0;
    q.d[u][0] = a.coord[3 * X] - cx;
    q.d[u][1] = a.coord[3 * X + 1] - cy;
    q.d[u][2] = a.coord[3 * X + 2] - cz;
  }
  return q;
}

__global__ void __launch_bounds__(256) k_list_count(ListArgs a, TreeGeom G, int32_t* near_cnt, int32_t* far_cnt) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= a.ncells) return;
  const LevelGeom& lg = G.lev[a.level];
  const int pc = a.parent[c];
  const int e0 = a.pnear_ptr[pc], ncand = 2 * (a.pnear_ptr[pc + 1] - e0);
  const int cx = a.coord[3 * c], cy = a.coord[3 * c + 1], cz = a.coord[3 * c + 2];
  const double th2 = a.cell_th2 ? a.cell_th2[c] : a.theta2;  // a smallest cell may use its own angle
  int nn = 0, nf = 0;
  for (int base = 0; base < ncand; base += 64 * kCandRounds) {
    const Cands q = load_cands(a, e0, ncand, base + lane, cx, cy, cz);
#pragma unroll
    for (int u = 0; u < kCandRounds; u++) {
      bool isn = false, isf = false;
      if (q.X[u] >= 0) {
        const bool nr = is_near(lg, th2, q.d[u][0], q.d[u][1], q.d[u][2]);
        isn = nr;
        isf = !nr;
      }
      nn += __popcll(__ballot(isn));
      nf += __popcll(__ballot(isf));
    }
  }
  if (lane == 0) {
    near_cnt[c] = nn;
    far_cnt[c] = nf;
  }
}

__global__ void __launch_bounds__(256) k_list_fill(ListArgs a, TreeGeom G, const int32_t* near_ptr, int32_t* near_idx,
                                                   const int32_t* far_ptr, int32_t* far_idx, int32_t* far_did,
                                                   int32_t* flags) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= a.ncells) return;
  const LevelGeom& lg = G.lev[a.level];
  const int pc = a.parent[c];
  const int e0 = a.pnear_ptr[pc], ncand = 2 * (a.pnear_ptr[pc + 1] - e0);
  const int cx = a.coord[3 * c], cy = a.coord[3 * c + 1], cz = a.coord[3 * c + 2];
  const double th2 = a.cell_th2 ? a.cell_th2[c] : a.theta2;  // a smallest cell may use its own angle
  int64_t jn = near_ptr[c], jf = far_ptr[c];
  const uint64_t lt = lanemask_lt(lane);
  for (int base = 0; base < ncand; base += 64 * kCandRounds) {
    const Cands q = load_cands(a, e0, ncand, base + lane, cx, cy, cz);
#pragma unroll
    for (int u = 0; u < kCandRounds; u++) {
      bool isn = false, isf = false;
      const int X = q.X[u], dx = q.d[u][0], dy = q.d[u][1], dz = q.d[u][2];
      if (X >= 0) {
        const bool nr = is_near(lg, th2, dx, dy, dz);
        isn = nr;
        isf = !nr;
      }
      const uint64_t mn = __ballot(isn), mf = __ballot(isf);
      if (isn) {
        const int64_t at = jn + __popcll(mn & lt);
        if (at < a.near_cap)
          near_idx[at] = X;
        else
          flags[0] = 1;
      }
      if (isf) {
        const int64_t at = jf + __popcll(mf & lt);
        const bool inbox = abs(dx) <= a.wfar[0] && abs(dy) <= a.wfar[1] && abs(dz) <= a.wfar[2];
        if (at < a.far_cap && inbox) {
          far_idx[at] = X;
          far_did[at] = (int32_t)box_index(a.wfar, dx, dy, dz);
        } else {
          flags[0] = 1;
        }
      }
      jn += __popcll(mn);
      jf += __popcll(mf);
    }
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static void fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n <= 0) return;
  k_fill_i32<<<ceil_div(n, 256), 256, 0, st>>>(p, n, v);
  CCFMM_HIP(hipGetLastError());
}

// Smallest level: each cell's near list reordered so that the cell itself and
// its face/edge/corner neighbours come first (stable within both parts).  Only
// those cells can hold dipoles arbitrarily close to the cell's own, so the
// near-field sum gives them its exact-separation path and packs them into its
// first batches.  One wavefront per cell; ballots give the slots.
__global__ void __launch_bounds__(256) k_near_adjacent_first(int32_t nc, const int32_t* near_ptr,
                                                             const int32_t* near_idx, const int32_t* coord,
                                                             int32_t* out) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= nc) return;
  const int cx = coord[3 * c], cy = coord[3 * c + 1], cz = coord[3 * c + 2];
  const int base = near_ptr[c], cnt = near_ptr[c + 1] - base;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  int w = 0;
  if (cnt <= 256) {  // the usual case: every entry loaded once, four per lane in flight
    int S[4];
    bool adj[4];
#pragma unroll
    for (int u = 0; u < 4; u++) S[u] = lane + 64 * u < cnt ? near_idx[base + lane + 64 * u] : -1;
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int X = S[u] >= 0 ? S[u] : 0;
      adj[u] = S[u] >= 0 && abs(coord[3 * X] - cx) <= 1 && abs(coord[3 * X + 1] - cy) <= 1 &&
               abs(coord[3 * X + 2] - cz) <= 1;
    }
    for (int pass = 0; pass < 2; pass++) {
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const bool take = S[u] >= 0 && (pass == 0 ? adj[u] : !adj[u]);
        const uint64_t m = __ballot(take);
        if (take) out[base + w + __popcll(m & lt)] = S[u];
        w += __popcll(m);
      }
    }
    return;
  }
  for (int pass = 0; pass < 2; pass++) {
    for (int k0 = 0; k0 < cnt; k0 += 64) {
      const int k = k0 + lane;
      const bool valid = k < cnt;
      const int S = valid ? near_idx[base + k] : 0;
      const bool adj = valid && abs(coord[3 * S] - cx) <= 1 && abs(coord[3 * S + 1] - cy) <= 1 &&
                       abs(coord[3 * S + 2] - cz) <= 1;
      const bool take = valid && (pass == 0 ? adj : !adj);
      const uint64_t m = __ballot(take);
      if (take) out[base + w + __popcll(m & lt)] = S;
      w += __popcll(m);
    }
  }
}

// Offset bounds of every level: near offsets satisfy |delta_a g_a| < |g|/theta;
// candidates are children of near cells of the parent, so their offsets are
// those of the parent level, doubled (+1) along the axis halved at this level.
static void level_bounds(Plan& P) {
  for (int l = 0; l <= P.L; l++) {
    // smallest cells with their own angles are bounded by the smallest of them
    const double th = (l == P.L && P.has_leaf) ? std::min(P.prm.theta, P.leaf_theta_min) : P.prm.theta;
    LevelData& D = *P.lev[l];
    const LevelGeom& lg = P.geo.lev[l];
    const double R = lg.g[0] * lg.g[0] + lg.g[1] * lg.g[1] + lg.g[2] * lg.g[2];
    for (int a = 0; a < 3; a++) {
      const double grid = std::ldexp(1.0, lg.k[a]) - 1.0;
      const double w = std::floor(std::sqrt(R) / (th * lg.g[a])) + 1.0;
      D.wnear[a] = (int)std::min(w, grid);
      if (l == 0) {
        D.wfar[a] = 0;
      } else {
        const LevelData& U = *P.lev[l - 1];
        const double wf = (a == lg.axis) ? 2.0 * U.wnear[a] + 1.0 : (double)U.wnear[a];
        D.wfar[a] = (int)std::min(wf, grid);
      }
    }
    // most near cells of one cell: near offsets counted in the near box, with a
    // small relative margin so that no tie is under-counted
    int64_t cn = 0;
    const double th2 = th * th;
    for (int dx = -D.wnear[0]; dx <= D.wnear[0]; dx++)
      for (int dy = -D.wnear[1]; dy <= D.wnear[1]; dy++)
        for (int dz = -D.wnear[2]; dz <= D.wnear[2]; dz++) {
          const double ax = dx * lg.g[0], ay = dy * lg.g[1], az = dz * lg.g[2];
          if (th2 * (ax * ax + ay * ay + az * az) < R * (1.0 + 1e-9)) cn++;
        }
    D.cnear = std::max<int64_t>(1, cn);
    D.nbox = (int64_t)(2 * D.wfar[0] + 1) * (2 * D.wfar[1] + 1) * (2 * D.wfar[2] + 1);
  }
}

void build_lists(Plan& P, hipStream_t st) {
  const int L = P.L;
  const int T = 256;
  const double theta2 = P.prm.theta * P.prm.theta;
  level_bounds(P);
  int32_t* flags = reinterpret_cast<int32_t*>(P.flags.ensure(64));
  fill_i32(flags, 16, 0, st);
  // level 0: the root is near itself, no far cells
  {
    LevelData& D = *P.lev[0];
    int32_t* np = reinterpret_cast<int32_t*>(D.near_ptr.ensure(sizeof(int32_t) * 2));
    int32_t* ni = reinterpret_cast<int32_t*>(D.near_idx.ensure(sizeof(int32_t) * 1));
    int32_t* fp = reinterpret_cast<int32_t*>(D.far_ptr.ensure(sizeof(int32_t) * 2));
    fill_i32(np, 1, 0, st);
    fill_i32(np + 1, 1, 1, st);
    fill_i32(ni, 1, 0, st);
    fill_i32(fp, 2, 0, st);
  }
  for (int l = 1; l <= L; l++) {
    LevelData& D = *P.lev[l];
    LevelData& U = *P.lev[l - 1];
    const int nc = D.ncells;
    const int64_t near_cap = (int64_t)nc * D.cnear;
    const int64_t far_cap = (int64_t)nc * std::min<int64_t>(2 * U.cnear, D.nbox);
    if (near_cap > (1ll << 31) - 1 || far_cap > (1ll << 31) - 1)
      fail(CCFMM_EINVAL, "opening angle too small for this tree (lists would exceed 2^31 entries)");
    int32_t* c = reinterpret_cast<int32_t*>(P.scratch2.ensure(sizeof(int32_t) * 2 * (size_t)(nc + 1)));
    int32_t* near_cnt = c;
    int32_t* far_cnt = c + (nc + 1);
    ListArgs a;
    a.parent = D.parent.as<int32_t>();
    a.coord = D.coord.as<int32_t>();
    a.pnear_ptr = U.near_ptr.as<int32_t>();
    a.pnear_idx = U.near_idx.as<int32_t>();
    a.pchild = U.child.as<int32_t>();
    a.ncells = nc;
    a.level = l;
    a.theta2 = theta2;
    a.cell_th2 = (l == L && P.has_leaf) ? P.leaf_th2.as<double>() : nullptr;
    for (int q = 0; q < 3; q++) a.wfar[q] = D.wfar[q];
    a.near_cap = near_cap;
    a.far_cap = far_cap;
    const int nblk = ceil_div(nc, 4);
    k_list_count<<<nblk, T, 0, st>>>(a, P.geo, near_cnt, far_cnt);
    CCFMM_HIP(hipGetLastError());
    int32_t* nptr = reinterpret_cast<int32_t*>(D.near_ptr.ensure(sizeof(int32_t) * (nc + 1)));
    int32_t* fptr = reinterpret_cast<int32_t*>(D.far_ptr.ensure(sizeof(int32_t) * (nc + 1)));
    scan_exclusive2(near_cnt, nptr, far_cnt, fptr, nc, P.scratch, st);
    int32_t* nidx = reinterpret_cast<int32_t*>(D.near_idx.ensure(sizeof(int32_t) * std::max<int64_t>(1, near_cap)));
    int32_t* fidx = reinterpret_cast<int32_t*>(D.far_idx.ensure(sizeof(int32_t) * std::max<int64_t>(1, far_cap)));
    int32_t* fdid = reinterpret_cast<int32_t*>(D.far_did.ensure(sizeof(int32_t) * std::max<int64_t>(1, far_cap)));
    k_list_fill<<<nblk, T, 0, st>>>(a, P.geo, nptr, nidx, fptr, fidx, fdid, flags);
    CCFMM_HIP(hipGetLastError());
    if (l == L) {
      int32_t* reord = reinterpret_cast<int32_t*>(P.near_tmp.ensure(sizeof(int32_t) * std::max<int64_t>(1, near_cap)));
      k_near_adjacent_first<<<nblk, T, 0, st>>>(nc, nptr, nidx, D.coord.as<int32_t>(), reord);
      CCFMM_HIP(hipGetLastError());
      std::swap(D.near_idx.p, P.near_tmp.p);
      std::swap(D.near_idx.cap, P.near_tmp.cap);
    }
  }
}

// ---------------------------------------------------------------- M2L tiles
// Targets of a level are ordered by (low class bits of the key, key): cells in
// the same position inside their ancestors have the same set of far offsets,
// so a tile of TC such cells shares one list of offsets.  The tile's steps are
// the union of its cells' offsets; a cell without a source at that offset
// gets a null column.  All levels are tiled together: cells and target groups
// are numbered globally (level by level), each kernel below runs once for
// the whole tree and finds a cell's or a group's level in a small table.
struct TileLevel {
  const int32_t* key;       // compact -> key
  const int32_t* far_ptr;   // far lists (null at the root level)
  const int32_t* far_idx;
  const int32_t* far_did;
  int64_t cell0;            // first global cell of the level
  int64_t g0;               // first global target group
  int64_t bm0;              // first bitmap word
  int64_t drow0;            // derivative-tensor row of dense offset id 0
  int32_t nc;
  int32_t words;            // bitmap words per group
};
struct TileLevels {
  TileLevel lv[kLMax + 1];
  int32_t nlev;
  int32_t TC;
  // per-cell orders of the smallest cells (compact order; null: none): their
  // tiles are grouped by order and compute the local rows of that order only
  const int32_t* leaf_p;
  int32_t L;
  int32_t red;    // traceless rows (q (q + 2) for order q) or full rows (N(q) - 1)
  int32_t pbits;  // order bits in the sort key
};

// local-expansion rows of order q, a prefix of the row order in either form
__device__ __forceinline__ int local_rows(int q, int red) { return red ? q * (q + 2) : ncoef(q) - 1; }

__device__ __forceinline__ int level_of_cell(const TileLevels& T, int64_t i) {
  int l = 0;
  while (l + 1 < T.nlev && i >= T.lv[l + 1].cell0) l++;
  return l;
}
__device__ __forceinline__ int level_of_group(const TileLevels& T, int64_t b) {
  int l = 0;
  while (l + 1 < T.nlev && b >= T.lv[l + 1].g0) l++;
  return l;
}

// sort key (level, low class bits of the cell key, 16-bit signature of the
// cell's set of far offsets); the value is the global cell.  The signature is
// an order-free hash (a sum of mixed offset ids), so cells with the same set
// of offsets -- interior cells of one class, and boundary cells cut the same
// way -- sort next to each other and share tiles without empty columns.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
// one wavefront per cell: the far list is read coalesced and the hash summed
// across the lanes
__global__ void __launch_bounds__(256) k_tile_class_keys(TileLevels T, int64_t ncell, int cb, int sigbits,
                                                         uint32_t* key, int32_t* val) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= ncell) return;
  const int l = level_of_cell(T, i);
  const TileLevel& lv = T.lv[l];
  const int c = (int)(i - lv.cell0);
  uint32_t h = 0;
  if (sigbits && lv.far_ptr) {
    const int e1 = lv.far_ptr[c + 1];
    for (int e = lv.far_ptr[c] + lane; e < e1; e += 256) {  // four loads in flight per lane
      int d[4];
#pragma unroll
      for (int u = 0; u < 4; u++) d[u] = e + 64 * u < e1 ? lv.far_did[e + 64 * u] : -1;
#pragma unroll
      for (int u = 0; u < 4; u++)
        if (d[u] >= 0) h += mix32((uint32_t)d[u] + 1u);
    }
  }
  for (int off = 1; off < 64; off <<= 1) h += (uint32_t)__shfl_xor((int)h, off);
  if (lane == 0) {
    const int cbl = min(cb, l);
    const uint32_t cls = (uint32_t)lv.key[c] & ((1u << cbl) - 1u);
    const uint32_t sig = sigbits ? h >> (32 - sigbits) : 0u;
    // smallest cells with their own order: grouped by it (orders 1..8 -> 0..7)
    const uint32_t pg = (T.pbits && l == T.L && T.leaf_p) ? (uint32_t)(T.leaf_p[c] - 1) : 0u;
    key[i] = ((((((uint32_t)l << T.pbits) | pg) << cb) | cls) << sigbits) | sig;
    val[i] = (int32_t)i;
  }
}


// One block per target group: the union of its cells' far offsets as a bitmap
// over the level's offset box (built in LDS by 16 wavefronts, each lane with
// four far entries in flight), the exclusive popcount prefix over its words
// (a step's rank, by the first 256 threads) and its step count.
constexpr int kGroupBitsThreads = 1024;
__global__ void __launch_bounds__(kGroupBitsThreads) k_group_bits(TileLevels T, const int32_t* sorted,
                                                                  uint32_t* bitmap, int32_t* wpre, int32_t* cnt) {
  extern __shared__ uint32_t sb[];
  __shared__ int32_t ssum[256];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  constexpr int NW = kGroupBitsThreads / 64;
  const int64_t b = blockIdx.x;
  const int l = level_of_group(T, b);
  const TileLevel& lv = T.lv[l];
  const int words = lv.words;
  const int64_t gi = b - lv.g0;
  for (int w = t; w < words; w += kGroupBitsThreads) sb[w] = 0u;
  __syncthreads();
  if (lv.far_ptr) {
    const int64_t p0 = gi * T.TC, p1 = min((int64_t)lv.nc, p0 + T.TC);
    for (int64_t p = p0 + wv; p < p1; p += NW) {
      const int c = sorted[lv.cell0 + p] - (int32_t)lv.cell0;
      const int e1 = lv.far_ptr[c + 1];
      for (int e = lv.far_ptr[c] + lane; e < e1; e += 256) {
        int d[4];
#pragma unroll
        for (int u = 0; u < 4; u++) d[u] = e + 64 * u < e1 ? lv.far_did[e + 64 * u] : -1;
#pragma unroll
        for (int u = 0; u < 4; u++)
          if (d[u] >= 0) atomicOr(&sb[d[u] >> 5], 1u << (d[u] & 31));
      }
    }
  }
  __syncthreads();
  // thread t < 256 owns words [t per, (t + 1) per)
  const bool own = t < 256;
  const int per = (words + 255) / 256;
  int s = 0;
  if (own)
    for (int i = 0; i < per; i++) {
      const int w = t * per + i;
      if (w < words) s += __popc(sb[w]);
    }
  if (own) ssum[t] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int32_t add = (own && t >= off) ? ssum[t - off] : 0;
    __syncthreads();
    if (own) ssum[t] += add;
    __syncthreads();
  }
  if (!own) return;
  int ex = ssum[t] - s;
  const int64_t base = lv.bm0 + gi * words;
  for (int i = 0; i < per; i++) {
    const int w = t * per + i;
    if (w < words) {
      const uint32_t m = sb[w];
      bitmap[base + w] = m;
      wpre[base + w] = ex;
      ex += __popc(m);
    }
  }
  if (t == 255) cnt[b] = ssum[255];
}

// one wavefront per group: the derivative-tensor row of every step, in
// offset-id order (word w, bit k has rank wpre[w] + popcount of lower bits)
__global__ void __launch_bounds__(256) k_group_steps(TileLevels T, int64_t ngroups, const uint32_t* bitmap,
                                                     const int32_t* wpre, const int32_t* goff,
                                                     int32_t* step_delta) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= ngroups) return;
  const TileLevel& lv = T.lv[level_of_group(T, b)];
  const int64_t base = lv.bm0 + (b - lv.g0) * lv.words;
  for (int w = lane; w < lv.words; w += 64) {
    uint32_t m = bitmap[base + w];
    int64_t s = (int64_t)goff[b] + wpre[base + w];
    while (m) {
      const int k = __ffs(m) - 1;
      m &= m - 1;
      step_delta[s++] = (int32_t)(lv.drow0 + 32 * w + k);
    }
  }
}

// One block of 16 wavefronts per group: the group's rows of the column-source
// table are filled in LDS, a band of rows at a time (-1 where a column has no
// source at that step), and stored contiguously, so the table is written once
// with whole-line stores (a far entry's row is the rank of its offset among
// the group's steps; its column is its cell's place in the group).  A
// wavefront takes every 16th column, each lane four far entries per round so
// their loads are in flight together.
constexpr int kStepSrcThreads = 1024;
constexpr int kStepSrcLdsBytes = 64 * 1024;

__global__ void __launch_bounds__(kStepSrcThreads) k_step_src(TileLevels T, const int32_t* sorted,
                                                              const uint32_t* bitmap, const int32_t* wpre,
                                                              const int32_t* goff, int32_t* step_src) {
  extern __shared__ int32_t sband[];
  const int TC = T.TC;
  const int band_rows = kStepSrcLdsBytes / (int)sizeof(int32_t) / TC;
  const int64_t b = blockIdx.x;
  const TileLevel& lv = T.lv[level_of_group(T, b)];
  const int64_t gi = b - lv.g0;
  const int64_t base = lv.bm0 + gi * lv.words;
  const int64_t s0 = goff[b], ns = goff[b + 1] - s0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int NW = kStepSrcThreads / 64;
  for (int64_t r0 = 0; r0 < ns; r0 += band_rows) {
    const int rows = (int)min((int64_t)band_rows, ns - r0);
    for (int k = threadIdx.x; k < rows * TC; k += kStepSrcThreads) sband[k] = -1;
    __syncthreads();
    if (lv.far_ptr) {
      for (int tc = wv; tc < TC; tc += NW) {
        const int64_t pos = gi * TC + tc;
        if (pos >= lv.nc) break;
        const int c = sorted[lv.cell0 + pos] - (int32_t)lv.cell0;
        const int e0 = lv.far_ptr[c], e1 = lv.far_ptr[c + 1];
        for (int e = e0 + lane; e < e1; e += 256) {
          int d[4], src[4];
#pragma unroll
          for (int u = 0; u < 4; u++) {
            const int eu = e + 64 * u;
            d[u] = eu < e1 ? lv.far_did[eu] : -1;
            src[u] = eu < e1 ? lv.far_idx[eu] : -1;
          }
#pragma unroll
          for (int u = 0; u < 4; u++) {
            if (d[u] < 0) continue;
            const int rank = wpre[base + (d[u] >> 5)] +
                             __popc(bitmap[base + (d[u] >> 5)] & ((1u << (d[u] & 31)) - 1u));
            const int64_t r = rank - r0;
            if (r >= 0 && r < rows) sband[r * TC + tc] = src[u];
          }
        }
      }
    }
    __syncthreads();
    int32_t* out = step_src + (s0 + r0) * TC;
    for (int k = threadIdx.x; k < rows * TC; k += kStepSrcThreads) out[k] = sband[k];
    __syncthreads();
  }
}

// column targets (compact cell of the level, -1 past the level's cells) and
// the tiles: one per group and configuration group
__global__ void k_tile_tgt(TileLevels T, int64_t ncol, const int32_t* sorted, int32_t* tgt) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncol) return;
  const int64_t b = j / T.TC;
  const TileLevel& lv = T.lv[level_of_group(T, b)];
  const int64_t pos = (b - lv.g0) * T.TC + j % T.TC;
  tgt[j] = pos < lv.nc ? sorted[lv.cell0 + pos] - (int32_t)lv.cell0 : -1;
}

// full_rows: the local rows of the plan's order.  A tile of smallest cells
// with their own orders needs the rows of the largest of them.
__global__ void k_tiles(TileLevels T, int64_t ngroups, int TB, int ncg, const int32_t* goff,
                        const int32_t* tile_tgt, int full_rows, M2LTile* tiles) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= ngroups) return;
  const int l = level_of_group(T, b);
  int rows = full_rows;
  if (l == T.L && T.leaf_p) {
    int q = 0;
    for (int j = 0; j < T.TC; j++) {
      const int c = tile_tgt[b * T.TC + j];
      if (c >= 0) q = max(q, T.leaf_p[c]);
    }
    rows = q > 0 ? min(full_rows, local_rows(q, T.red)) : full_rows;
  }
  for (int cg = 0; cg < ncg; cg++) {
    M2LTile t;
    t.level = l;
    t.step0 = goff[b];
    t.nsteps = goff[b + 1] - goff[b];
    t.tgt0 = (int32_t)(b * T.TC);
    t.b0 = cg * TB;
    t.rows = rows;
    t.pad[0] = t.pad[1] = 0;
    tiles[b * ncg + cg] = t;
  }
}

__global__ void k_tile_keys(int64_t ntiles, const M2LTile* tiles, uint32_t* key, int32_t* ord) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntiles) return;
  key[i] = 0xffffu - (uint32_t)min(tiles[i].nsteps, 0xffff);
  ord[i] = (int32_t)i;
}

void build_m2l_tiles(Plan& P, int nbatch, hipStream_t st) {
  const int L = P.L;
  const int T = 256;
  const int cols = m2l_tile_cols(P.m2l_variant);
  const int tb = tile_batch(nbatch, cols);
  P.TB = tb;
  P.TC = cols / tb;
  P.tiles_variant = P.m2l_variant;
  P.tiles_class_bits = P.class_bits;
  P.tiles_nb = nbatch;
  P.ncg = ceil_div(nbatch, tb);
  const int TC = P.TC;
  TileLevels TL{};
  TL.nlev = L + 1;
  TL.TC = TC;
  TL.L = L;
  const bool red = P.prm.m2l_traceless != 0 && P.p <= wide_max_order(true) &&
                   (P.m2l_variant == kM2LWide4 || P.m2l_variant == kM2LWide2 || P.m2l_variant == kM2LWide1);
  TL.red = red ? 1 : 0;
  TL.leaf_p = P.has_leaf ? P.leaf_p.as<int32_t>() : nullptr;
  TL.pbits = P.has_leaf ? 3 : 0;
  int64_t ncell = 0, ngroups = 0, nbm = 0;
  int maxwords = 1;
  for (int l = 0; l <= L; l++) {
    LevelData& D = *P.lev[l];
    TileLevel& v = TL.lv[l];
    v.key = D.key.as<int32_t>();
    v.far_ptr = l > 0 ? D.far_ptr.as<int32_t>() : nullptr;
    v.far_idx = l > 0 ? D.far_idx.as<int32_t>() : nullptr;
    v.far_did = l > 0 ? D.far_did.as<int32_t>() : nullptr;
    v.cell0 = ncell;
    v.g0 = ngroups;
    v.bm0 = nbm;
    v.drow0 = D.drow0;
    v.nc = D.ncells;
    v.words = (int)std::max<int64_t>(1, ceil_div(D.nbox, 32));
    maxwords = std::max(maxwords, v.words);
    const int64_t ng = ceil_div(D.ncells, TC);
    ncell += D.ncells;
    ngroups += ng;
    nbm += ng * v.words;
  }
  if (sizeof(uint32_t) * (size_t)maxwords > 60 * 1024)
    fail(CCFMM_EINVAL, "opening angle too small for the M2L tiling (offset box too large)");
  // target order: (level, class, key) by one stable sort of all cells
  const int cb = std::min(P.class_bits, 11);
  int lbits = 1;
  while ((1 << lbits) <= L) lbits++;
  int32_t* sbuf = reinterpret_cast<int32_t*>(P.tile_sort.ensure(sizeof(int32_t) * 4 * ncell));
  uint32_t* skey = reinterpret_cast<uint32_t*>(sbuf);
  int32_t* sorted = sbuf + ncell;
  uint32_t* skey2 = reinterpret_cast<uint32_t*>(sbuf + 2 * ncell);
  int32_t* sval2 = sbuf + 3 * ncell;
  // the sort key is (level, order group, class bits, signature) in 32 bits:
  // the signature gives way when the other fields need its bits
  const int sigbits = P.tile_signature ? std::min(16, 32 - (cb + lbits + TL.pbits)) : 0;
  k_tile_class_keys<<<ceil_div(ncell, 4), T, 0, st>>>(TL, ncell, cb, sigbits, skey, sorted);
  CCFMM_HIP(hipGetLastError());
  radix_sort_pairs(skey, sorted, skey2, sval2, ncell, cb + lbits + TL.pbits + sigbits, P.scratch, st);
  // bitmaps, ranks and step counts of every group; global step offsets
  uint32_t* bitmap = reinterpret_cast<uint32_t*>(P.bitmap.ensure(sizeof(uint32_t) * 2 * std::max<int64_t>(1, nbm)));
  int32_t* wpre = reinterpret_cast<int32_t*>(bitmap + std::max<int64_t>(1, nbm));
  int32_t* gbuf = reinterpret_cast<int32_t*>(P.gcount.ensure(sizeof(int32_t) * 2 * (ngroups + 1)));
  int32_t* gcnt = gbuf;
  int32_t* goff = gbuf + ngroups + 1;
  k_group_bits<<<(unsigned)ngroups, kGroupBitsThreads, sizeof(uint32_t) * maxwords, st>>>(TL, sorted, bitmap, wpre,
                                                                                         gcnt);
  CCFMM_HIP(hipGetLastError());
  scan_exclusive(gcnt, goff, ngroups, P.scratch, st);
  int32_t total = 0;
  CCFMM_HIP(hipMemcpyAsync(&total, goff + ngroups, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CCFMM_HIP(hipStreamSynchronize(st));
  const int64_t nsteps = total;
  const int64_t ntiles = ngroups * P.ncg;
  P.nsteps = nsteps;
  P.ntiles = ntiles;
  int32_t* step_delta = reinterpret_cast<int32_t*>(P.step_delta.ensure(sizeof(int32_t) * std::max<int64_t>(1, nsteps)));
  int32_t* step_src = reinterpret_cast<int32_t*>(P.step_src.ensure(sizeof(int32_t) * std::max<int64_t>(1, nsteps * TC)));
  int32_t* tile_tgt = reinterpret_cast<int32_t*>(P.tile_tgt.ensure(sizeof(int32_t) * std::max<int64_t>(1, ngroups * TC)));
  M2LTile* tiles = reinterpret_cast<M2LTile*>(P.tiles.ensure(sizeof(M2LTile) * std::max<int64_t>(1, ntiles)));
  k_group_steps<<<ceil_div(ngroups, 4), T, 0, st>>>(TL, ngroups, bitmap, wpre, goff, step_delta);
  CCFMM_HIP(hipGetLastError());
  if (ngroups > 0) {
    if (kStepSrcLdsBytes / (int)sizeof(int32_t) / TC < 1) fail(CCFMM_EINVAL, "M2L tile too wide");
    k_step_src<<<(unsigned)ngroups, kStepSrcThreads, kStepSrcLdsBytes, st>>>(TL, sorted, bitmap, wpre, goff,
                                                                           step_src);
    CCFMM_HIP(hipGetLastError());
  }
  k_tile_tgt<<<ceil_div(ngroups * TC, T), T, 0, st>>>(TL, ngroups * TC, sorted, tile_tgt);
  CCFMM_HIP(hipGetLastError());
  k_tiles<<<ceil_div(ngroups, T), T, 0, st>>>(TL, ngroups, P.TB, P.ncg, goff, tile_tgt,
                                              red ? P.p * (P.p + 2) : nact(P.p), tiles);
  CCFMM_HIP(hipGetLastError());
  // launch order: longest step lists first, so the dispatcher's greedy,
  // round-robin placement balances the XCDs and their compute units
  if (ntiles > 0) {
    int32_t* ord = reinterpret_cast<int32_t*>(P.tile_order.ensure(sizeof(int32_t) * 4 * ntiles));
    uint32_t* key = reinterpret_cast<uint32_t*>(ord + ntiles);
    int32_t* ord2 = ord + 2 * ntiles;
    uint32_t* key2 = reinterpret_cast<uint32_t*>(ord + 3 * ntiles);
    k_tile_keys<<<ceil_div(ntiles, T), T, 0, st>>>(ntiles, tiles, key, ord);
    CCFMM_HIP(hipGetLastError());
    radix_sort_pairs(key, ord, key2, ord2, ntiles, 16, P.scratch, st);
  }
}

// ---------------------------------------------------------------- P2P chunks
// Every occupied smallest cell is cut into chunks of at most 64 dipoles; the
// chunk count stays in device memory (the P2P launch is sized by its bound).
__global__ void k_chunk_count(int32_t nl, const int32_t* lcount, int32_t* cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nl) cnt[i] = (lcount[i] + 63) >> 6;
}

__global__ void k_chunk_fill(int32_t nl, const int32_t* lstart, const int32_t* lcount, const int32_t* off,
                             P2PChunk* ch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nl) return;
  for (int k = 0, o = off[i]; k < lcount[i]; k += 64, o++) {
    P2PChunk c;
    c.leaf = i;
    c.first = lstart[i] + k;
    c.count = min(64, lcount[i] - k);
    c.pad = 0;
    ch[o] = c;
  }
}

// chunks of at most 32 dipoles (batched near field on the matrix cores)
__global__ void k_chunk_count32(int32_t nl, const int32_t* lcount, int32_t* cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nl) cnt[i] = (lcount[i] + 31) >> 5;
}

__global__ void k_chunk_fill32(int32_t nl, const int32_t* lstart, const int32_t* lcount, const int32_t* off,
                               P2PChunk* ch, int32_t* dleaf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nl) return;
  for (int k = 0, o = off[i]; k < lcount[i]; k += 32, o++) {
    P2PChunk c;
    c.leaf = i;
    c.first = lstart[i] + k;
    c.count = min(32, lcount[i] - k);
    c.pad = 0;
    ch[o] = c;
  }
  for (int k = 0; k < lcount[i]; k++) dleaf[lstart[i] + k] = i;
}

// dipole -> smallest cell (tree order) alone, for plans that never run the
// batched near field; the 32-chunk total is then zero
__global__ void k_dleaf(int32_t nl, const int32_t* lstart, const int32_t* lcount, int32_t* dleaf, int32_t* total32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *total32 = 0;
  if (i >= nl) return;
  for (int k = 0; k < lcount[i]; k++) dleaf[lstart[i] + k] = i;
}

void build_p2p_chunks(Plan& P, hipStream_t st) {
  const int nl = P.lev[P.L]->ncells;
  P.nchunks_cap = (int64_t)nl + P.n / 64 + 1;
  // counts | offsets (64-chunks) | counts | offsets (32-chunks)
  int32_t* cnt = reinterpret_cast<int32_t*>(P.chunk_cnt.ensure(sizeof(int32_t) * 4 * (nl + 1)));
  int32_t* off = cnt + nl + 1;
  int32_t* cnt32 = off + nl + 1;
  int32_t* off32 = cnt32 + nl + 1;
  k_chunk_count<<<ceil_div(nl, 256), 256, 0, st>>>(nl, P.lcount.as<int32_t>(), cnt);
  CCFMM_HIP(hipGetLastError());
  scan_exclusive(cnt, off, nl, P.scratch, st);  // off[nl] = number of chunks
  P2PChunk* ch = reinterpret_cast<P2PChunk*>(P.chunks.ensure(sizeof(P2PChunk) * P.nchunks_cap));
  k_chunk_fill<<<ceil_div(nl, 256), 256, 0, st>>>(nl, P.lstart.as<int32_t>(), P.lcount.as<int32_t>(), off, ch);
  CCFMM_HIP(hipGetLastError());
  int32_t* dleaf = reinterpret_cast<int32_t*>(P.dleaf.ensure(sizeof(int32_t) * P.n));
  if (P.nbmax < P.batched_min) {  // no batch of this plan reaches the matrix-core near field
    k_dleaf<<<ceil_div(std::max(nl, 1), 256), 256, 0, st>>>(nl, P.lstart.as<int32_t>(), P.lcount.as<int32_t>(), dleaf,
                                                            off32 + nl);
    CCFMM_HIP(hipGetLastError());
    return;
  }
  k_chunk_count32<<<ceil_div(nl, 256), 256, 0, st>>>(nl, P.lcount.as<int32_t>(), cnt32);
  CCFMM_HIP(hipGetLastError());
  scan_exclusive(cnt32, off32, nl, P.scratch, st);
  P.nchunks32_cap = (int64_t)nl + P.n / 32 + 1;
  P2PChunk* ch32 = reinterpret_cast<P2PChunk*>(P.chunks32.ensure(sizeof(P2PChunk) * P.nchunks32_cap));
  k_chunk_fill32<<<ceil_div(nl, 256), 256, 0, st>>>(nl, P.lstart.as<int32_t>(), P.lcount.as<int32_t>(), off32, ch32,
                                                    dleaf);
  CCFMM_HIP(hipGetLastError());
}

}  // namespace ccfmm
