// lists.hip -- near/far cell lists (Sec. 2 and Appendix, createPartners),
// the distinct cell offsets of the far pairs, the M2L work tiles and the
// P2P work chunks.
//
// Level by level, the candidates of a cell are the children of the cells near
// its parent (the parent itself included, which supplies the sibling).  A
// candidate at opening angle 2r/d > theta is near (passed down, or kept for
// the near-field sum at the smallest cells); otherwise it is far and enters
// the cell's M2L list.  Empty cells are never created, which leaves every
// field unchanged (their moments vanish and they hold no field points).
#include <algorithm>

#include "plan.hpp"

namespace ccfmm {

// Exact opening-angle test.  With delta the integer offset of the two cells
// and g the cell sides over the smallest side, alpha = |g| / |delta*g|; the
// pair is far iff theta^2 |delta*g|^2 >= |g|^2 (alpha == theta is far).  The
// sums run x, y, z with no contraction.
__device__ __forceinline__ bool is_near(const LevelGeom& lg, double theta2, int dx, int dy, int dz) {
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
  int32_t ncells;
  int level;
  double theta2;
  int wbox[3];
};

__global__ void k_list_count(ListArgs a, TreeGeom G, int32_t* near_cnt, int32_t* far_cnt) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncells) return;
  const LevelGeom lg = G.lev[a.level];
  const int pc = a.parent[c];
  const int cx = a.coord[3 * c], cy = a.coord[3 * c + 1], cz = a.coord[3 * c + 2];
  int nn = 0, nf = 0;
  for (int e = a.pnear_ptr[pc]; e < a.pnear_ptr[pc + 1]; e++) {
    const int A = a.pnear_idx[e];
    for (int s = 0; s < 2; s++) {
      const int X = a.pchild[2 * A + s];
      if (X < 0) continue;
      const int dx = a.coord[3 * X] - cx, dy = a.coord[3 * X + 1] - cy, dz = a.coord[3 * X + 2] - cz;
      if (is_near(lg, a.theta2, dx, dy, dz))
        nn++;
      else
        nf++;
    }
  }
  near_cnt[c] = nn;
  far_cnt[c] = nf;
}

__device__ __forceinline__ int64_t box_index(const int w[3], int dx, int dy, int dz) {
  return ((int64_t)(dx + w[0]) * (2 * w[1] + 1) + (dy + w[1])) * (2 * w[2] + 1) + (dz + w[2]);
}

__global__ void k_list_fill(ListArgs a, TreeGeom G, const int32_t* near_ptr, int32_t* near_idx,
                            const int32_t* far_ptr, int32_t* far_idx, int32_t* far_box, int32_t* box_flag,
                            int32_t* overflow) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncells) return;
  const LevelGeom lg = G.lev[a.level];
  const int pc = a.parent[c];
  const int cx = a.coord[3 * c], cy = a.coord[3 * c + 1], cz = a.coord[3 * c + 2];
  int jn = near_ptr[c], jf = far_ptr[c];
  for (int e = a.pnear_ptr[pc]; e < a.pnear_ptr[pc + 1]; e++) {
    const int A = a.pnear_idx[e];
    for (int s = 0; s < 2; s++) {
      const int X = a.pchild[2 * A + s];
      if (X < 0) continue;
      const int dx = a.coord[3 * X] - cx, dy = a.coord[3 * X + 1] - cy, dz = a.coord[3 * X + 2] - cz;
      if (is_near(lg, a.theta2, dx, dy, dz)) {
        near_idx[jn++] = X;
      } else {
        far_idx[jf] = X;
        if (abs(dx) > a.wbox[0] || abs(dy) > a.wbox[1] || abs(dz) > a.wbox[2]) {
          overflow[0] = 1;
          far_box[jf] = 0;
        } else {
          const int64_t b = box_index(a.wbox, dx, dy, dz);
          far_box[jf] = (int32_t)b;
          box_flag[b] = 1;
        }
        jf++;
      }
    }
  }
}

__global__ void k_far_did(int64_t nfar, const int32_t* far_box, const int32_t* box_scan, int32_t* far_did) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nfar) return;
  far_did[e] = box_scan[far_box[e]];
}

__global__ void k_delta_vecs(int64_t nbox, const int32_t* box_flag, const int32_t* box_scan, int w0, int w1,
                             int w2, int32_t* dvec) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbox || !box_flag[b]) return;
  const int nz = 2 * w2 + 1, ny = 2 * w1 + 1;
  const int dz = (int)(b % nz) - w2;
  const int dy = (int)((b / nz) % ny) - w1;
  const int dx = (int)(b / ((int64_t)nz * ny)) - w0;
  const int id = box_scan[b];
  dvec[3 * id] = dx;
  dvec[3 * id + 1] = dy;
  dvec[3 * id + 2] = dz;
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

static int32_t read_i32(const int32_t* d, hipStream_t st) {
  int32_t v = 0;
  CCFMM_HIP(hipMemcpyAsync(&v, d, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CCFMM_HIP(hipStreamSynchronize(st));
  return v;
}

void build_lists(Plan& P, hipStream_t st) {
  const int L = P.L;
  const int T = 256;
  const double theta2 = P.prm.theta * P.prm.theta;
  // level 0: the root is near itself
  {
    LevelData& D = *P.lev[0];
    int32_t* np = reinterpret_cast<int32_t*>(D.near_ptr.ensure(sizeof(int32_t) * 2));
    int32_t* ni = reinterpret_cast<int32_t*>(D.near_idx.ensure(sizeof(int32_t) * 1));
    const int32_t h_np[2] = {0, 1}, h_ni[1] = {0};
    CCFMM_HIP(hipMemcpyAsync(np, h_np, sizeof(h_np), hipMemcpyHostToDevice, st));
    CCFMM_HIP(hipMemcpyAsync(ni, h_ni, sizeof(h_ni), hipMemcpyHostToDevice, st));
    D.nnear = 1;
    int32_t* fp = reinterpret_cast<int32_t*>(D.far_ptr.ensure(sizeof(int32_t) * 2));
    fill_i32(fp, 2, 0, st);
    D.nfar = 0;
    D.ndelta = 0;
    CCFMM_HIP(hipStreamSynchronize(st));  // host arrays above go out of scope
  }
  DevBuf& cnt = P.scratch2;
  for (int l = 1; l <= L; l++) {
    LevelData& D = *P.lev[l];
    LevelData& U = *P.lev[l - 1];
    const int nc = D.ncells;
    // offset box for the far pairs of this level: a far pair's parents are near
    // at level l-1, which bounds their offset; the halved axis doubles it
    const LevelGeom& pg = P.geo.lev[l - 1];
    const double Rp = pg.g[0] * pg.g[0] + pg.g[1] * pg.g[1] + pg.g[2] * pg.g[2];
    for (int a = 0; a < 3; a++) {
      double wp = std::floor(std::sqrt(Rp) / (P.prm.theta * pg.g[a])) + 1.0;
      double w = (a == P.geo.lev[l].axis) ? 2.0 * wp + 1.0 : wp;
      double gridmax = (double)((1ll << P.geo.lev[l].k[a]) - 1);
      D.wbox[a] = (int)std::min(w, gridmax);
    }
    const int64_t nbox = (int64_t)(2 * D.wbox[0] + 1) * (2 * D.wbox[1] + 1) * (2 * D.wbox[2] + 1);
    if (nbox > (1ll << 26)) fail(CCFMM_EINVAL, "opening angle too small for this tree (offset box too large)");

    int32_t* c = reinterpret_cast<int32_t*>(cnt.ensure(sizeof(int32_t) * (2 * (size_t)(nc + 1) + nbox + 1 + 8)));
    int32_t* near_cnt = c;
    int32_t* far_cnt = c + (nc + 1);
    int32_t* ovf = far_cnt + (nc + 1);
    int32_t* box_flag = ovf + 8;
    ListArgs a;
    a.parent = D.parent.as<int32_t>();
    a.coord = D.coord.as<int32_t>();
    a.pnear_ptr = U.near_ptr.as<int32_t>();
    a.pnear_idx = U.near_idx.as<int32_t>();
    a.pchild = U.child.as<int32_t>();
    a.ncells = nc;
    a.level = l;
    a.theta2 = theta2;
    for (int q = 0; q < 3; q++) a.wbox[q] = D.wbox[q];
    k_list_count<<<ceil_div(nc, T), T, 0, st>>>(a, P.geo, near_cnt, far_cnt);
    CCFMM_HIP(hipGetLastError());
    int32_t* nptr = reinterpret_cast<int32_t*>(D.near_ptr.ensure(sizeof(int32_t) * (nc + 1)));
    int32_t* fptr = reinterpret_cast<int32_t*>(D.far_ptr.ensure(sizeof(int32_t) * (nc + 1)));
    scan_exclusive(near_cnt, nptr, nc, P.scratch, st);
    scan_exclusive(far_cnt, fptr, nc, P.scratch, st);
    int32_t tot[2];
    CCFMM_HIP(hipMemcpyAsync(&tot[0], nptr + nc, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CCFMM_HIP(hipMemcpyAsync(&tot[1], fptr + nc, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CCFMM_HIP(hipStreamSynchronize(st));
    D.nnear = tot[0];
    D.nfar = tot[1];
    int32_t* nidx = reinterpret_cast<int32_t*>(D.near_idx.ensure(sizeof(int32_t) * std::max<int64_t>(1, D.nnear)));
    int32_t* fidx = reinterpret_cast<int32_t*>(D.far_idx.ensure(sizeof(int32_t) * std::max<int64_t>(1, D.nfar)));
    int32_t* fdid = reinterpret_cast<int32_t*>(D.far_did.ensure(sizeof(int32_t) * std::max<int64_t>(1, D.nfar)));
    fill_i32(ovf, 1, 0, st);
    fill_i32(box_flag, nbox, 0, st);
    // far_did first holds the box index of each far entry
    k_list_fill<<<ceil_div(nc, T), T, 0, st>>>(a, P.geo, nptr, nidx, fptr, fidx, fdid, box_flag, ovf);
    CCFMM_HIP(hipGetLastError());
    if (read_i32(ovf, st)) fail(CCFMM_EINVAL, "internal: far offset outside its bound");
    // compact the offsets that occur
    DevBuf& bs = P.scratch;  // scan output must not alias scratch used by scan itself
    int32_t* box_scan = reinterpret_cast<int32_t*>(P.bitmap.ensure(sizeof(int32_t) * (nbox + 1)));
    (void)bs;
    scan_exclusive(box_flag, box_scan, nbox, P.scratch, st);
    D.ndelta = read_i32(box_scan + nbox, st);
    int32_t* dvec = reinterpret_cast<int32_t*>(D.delta_vec.ensure(sizeof(int32_t) * 3 * std::max(1, D.ndelta)));
    k_delta_vecs<<<ceil_div(nbox, T), T, 0, st>>>(nbox, box_flag, box_scan, D.wbox[0], D.wbox[1], D.wbox[2], dvec);
    CCFMM_HIP(hipGetLastError());
    if (D.nfar > 0) {
      k_far_did<<<ceil_div(D.nfar, T), T, 0, st>>>(D.nfar, fdid, box_scan, fdid);
      CCFMM_HIP(hipGetLastError());
    }
  }
  // derivative-tensor rows: levels in order
  int64_t r = 0;
  for (int l = 0; l <= L; l++) {
    P.lev[l]->drow0 = r;
    r += P.lev[l]->ndelta;
  }
  P.nrows = r;
}

// ---------------------------------------------------------------- M2L tiles
// Targets of a level are ordered by (low class bits of the key, remaining key
// bits): cells in the same position inside their ancestors have the same set
// of far offsets, so a tile of TC such cells shares one list of offsets.  The
// tile's steps are the union of its cells' offsets; a cell without a source
// at that offset gets a null column.
__global__ void k_rot_keys(const int32_t* key, int32_t nc, int l, int cb, uint32_t* rot, int32_t* idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const uint32_t k = (uint32_t)key[i];
  const uint32_t mask = (1u << cb) - 1u;
  rot[i] = ((k & mask) << (l - cb)) | (k >> cb);
  idx[i] = i;
}

__global__ void k_inverse(const int32_t* order, int32_t nc, int32_t* inv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nc) inv[order[i]] = i;
}

__global__ void k_group_bitmap(int32_t nc, const int32_t* far_ptr, const int32_t* far_did, const int32_t* inv,
                               int TC, int words, uint32_t* bitmap) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int gidx = inv[c] / TC;
  uint32_t* bm = bitmap + (int64_t)gidx * words;
  for (int e = far_ptr[c]; e < far_ptr[c + 1]; e++) {
    const int d = far_did[e];
    atomicOr(&bm[d >> 5], 1u << (d & 31));
  }
}

__global__ void k_group_count(int32_t ng, int words, const uint32_t* bitmap, int32_t* cnt) {
  const int gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= ng) return;
  int s = 0;
  for (int w = 0; w < words; w++) s += __popc(bitmap[(int64_t)gi * words + w]);
  cnt[gi] = s;
}

__global__ void k_group_steps(int32_t ng, int words, const uint32_t* bitmap, const int32_t* goff,
                              int64_t step_base, int64_t drow0, int32_t* step_delta) {
  const int gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= ng) return;
  int64_t s = step_base + goff[gi];
  for (int w = 0; w < words; w++) {
    uint32_t m = bitmap[(int64_t)gi * words + w];
    while (m) {
      const int b = __ffs(m) - 1;
      m &= m - 1;
      step_delta[s++] = (int32_t)(drow0 + 32 * w + b);
    }
  }
}

__global__ void k_step_src(int32_t nc, const int32_t* far_ptr, const int32_t* far_idx, const int32_t* far_did,
                           const int32_t* inv, int TC, int words, const uint32_t* bitmap, const int32_t* goff,
                           int64_t step_base, int32_t* step_src) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int pos = inv[c];
  const int gi = pos / TC, tc = pos % TC;
  const uint32_t* bm = bitmap + (int64_t)gi * words;
  for (int e = far_ptr[c]; e < far_ptr[c + 1]; e++) {
    const int d = far_did[e];
    int rank = 0;
    for (int w = 0; w < (d >> 5); w++) rank += __popc(bm[w]);
    rank += __popc(bm[d >> 5] & ((1u << (d & 31)) - 1u));
    const int64_t s = step_base + goff[gi] + rank;
    step_src[s * TC + tc] = far_idx[e];
  }
}

__global__ void k_tiles(int32_t ng, int level, int TC, int TB, int ncg, int64_t step_base, int64_t tgt_base,
                        const int32_t* goff, M2LTile* tiles, int64_t tile_base) {
  const int gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= ng) return;
  for (int cg = 0; cg < ncg; cg++) {
    M2LTile t;
    t.level = level;
    t.step0 = (int32_t)(step_base + goff[gi]);
    t.nsteps = goff[gi + 1] - goff[gi];
    t.tgt0 = (int32_t)(tgt_base + (int64_t)gi * TC);
    t.b0 = cg * TB;
    t.pad[0] = t.pad[1] = t.pad[2] = 0;
    tiles[tile_base + (int64_t)gi * ncg + cg] = t;
  }
}

__global__ void k_tile_tgt(int32_t nc, int32_t ng, int TC, const int32_t* order, int32_t* tgt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ng * TC) return;
  tgt[i] = (i < nc) ? order[i] : -1;
}

void build_m2l_tiles(Plan& P, int nbatch, hipStream_t st) {
  const int L = P.L;
  const int T = 256;
  // columns of a wavefront tile: TC targets x TB configurations (TC*TB = 16)
  int tb = 1;
  while (tb < nbatch && tb < 16) tb <<= 1;
  P.TB = tb;
  P.TC = 16 / tb;
  P.ncg = ceil_div(nbatch, tb);
  const int TC = P.TC;
  // pass 1: ordering, bitmaps, step counts per target group
  std::vector<int64_t> bm_off(L + 2, 0), g_off(L + 2, 0);
  std::vector<int> words(L + 1, 0);
  for (int l = 0; l <= L; l++) {
    LevelData& D = *P.lev[l];
    D.ngroups = ceil_div(D.ncells, TC);
    words[l] = std::max(1, ceil_div(D.ndelta, 32));
    bm_off[l + 1] = bm_off[l] + (int64_t)D.ngroups * words[l];
    g_off[l + 1] = g_off[l] + D.ngroups + 1;
  }
  uint32_t* bitmap = reinterpret_cast<uint32_t*>(P.bitmap.ensure(sizeof(uint32_t) * std::max<int64_t>(1, bm_off[L + 1])));
  int32_t* gbuf = reinterpret_cast<int32_t*>(P.scratch2.ensure(sizeof(int32_t) * 2 * (g_off[L + 1] + 1)));
  int32_t* gcnt = gbuf;
  int32_t* goff = gbuf + g_off[L + 1] + 1;
  fill_i32(reinterpret_cast<int32_t*>(bitmap), bm_off[L + 1], 0, st);
  std::vector<int32_t> lsteps(L + 1, 0);
  for (int l = 0; l <= L; l++) {
    LevelData& D = *P.lev[l];
    const int nc = D.ncells;
    int32_t* order = reinterpret_cast<int32_t*>(D.order.ensure(sizeof(int32_t) * 2 * std::max(1, nc)));
    int32_t* inv = order + std::max(1, nc);
    const int cb = std::min(P.class_bits, l);
    k_rot_keys<<<ceil_div(nc, T), T, 0, st>>>(D.key.as<int32_t>(), nc, l, cb, P.key_tmp.as<uint32_t>(), order);
    CCFMM_HIP(hipGetLastError());
    // sort by rotated key (stable; compact order is key order)
    radix_sort_pairs(P.key_tmp.as<uint32_t>(), order, P.key.as<uint32_t>(), inv, nc, l, P.scratch, st);
    k_inverse<<<ceil_div(nc, T), T, 0, st>>>(order, nc, inv);
    CCFMM_HIP(hipGetLastError());
    if (D.nfar > 0) {
      k_group_bitmap<<<ceil_div(nc, T), T, 0, st>>>(nc, D.far_ptr.as<int32_t>(), D.far_did.as<int32_t>(), inv, TC,
                                                     words[l], bitmap + bm_off[l]);
      CCFMM_HIP(hipGetLastError());
    }
    k_group_count<<<ceil_div(D.ngroups, T), T, 0, st>>>(D.ngroups, words[l], bitmap + bm_off[l], gcnt + g_off[l]);
    CCFMM_HIP(hipGetLastError());
    scan_exclusive(gcnt + g_off[l], goff + g_off[l], D.ngroups, P.scratch, st);
    CCFMM_HIP(hipMemcpyAsync(&lsteps[l], goff + g_off[l] + D.ngroups, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  }
  CCFMM_HIP(hipStreamSynchronize(st));
  int64_t nsteps = 0, ntiles = 0, ntgt = 0;
  for (int l = 0; l <= L; l++) {
    LevelData& D = *P.lev[l];
    D.step0 = nsteps;
    D.nsteps = lsteps[l];
    D.tile0 = ntiles;
    D.ntiles = (int64_t)D.ngroups * P.ncg;
    nsteps += D.nsteps;
    ntiles += D.ntiles;
    ntgt += (int64_t)D.ngroups * TC;
  }
  // level 0 (the root) never has far cells; it still gets a tile so that its
  // (zero) local expansion is written like every other cell's
  P.nsteps = nsteps;
  P.ntiles = ntiles;
  int32_t* step_delta = reinterpret_cast<int32_t*>(P.step_delta.ensure(sizeof(int32_t) * std::max<int64_t>(1, nsteps)));
  int32_t* step_src = reinterpret_cast<int32_t*>(P.step_src.ensure(sizeof(int32_t) * std::max<int64_t>(1, nsteps * TC)));
  int32_t* tile_tgt = reinterpret_cast<int32_t*>(P.tile_tgt.ensure(sizeof(int32_t) * std::max<int64_t>(1, ntgt)));
  M2LTile* tiles = reinterpret_cast<M2LTile*>(P.tiles.ensure(sizeof(M2LTile) * std::max<int64_t>(1, ntiles)));
  fill_i32(step_src, nsteps * TC, -1, st);
  int64_t tgt_base = 0;
  for (int l = 0; l <= L; l++) {
    LevelData& D = *P.lev[l];
    const int nc = D.ncells;
    int32_t* order = D.order.as<int32_t>();
    int32_t* inv = order + std::max(1, nc);
    k_group_steps<<<ceil_div(D.ngroups, T), T, 0, st>>>(D.ngroups, words[l], bitmap + bm_off[l], goff + g_off[l],
                                                          D.step0, D.drow0, step_delta);
    CCFMM_HIP(hipGetLastError());
    if (D.nfar > 0) {
      k_step_src<<<ceil_div(nc, T), T, 0, st>>>(nc, D.far_ptr.as<int32_t>(), D.far_idx.as<int32_t>(),
                                                 D.far_did.as<int32_t>(), inv, TC, words[l], bitmap + bm_off[l],
                                                 goff + g_off[l], D.step0, step_src);
      CCFMM_HIP(hipGetLastError());
    }
    k_tile_tgt<<<ceil_div((int64_t)D.ngroups * TC, T), T, 0, st>>>(nc, D.ngroups, TC, order, tile_tgt + tgt_base);
    CCFMM_HIP(hipGetLastError());
    k_tiles<<<ceil_div(D.ngroups, T), T, 0, st>>>(D.ngroups, l, TC, P.TB, P.ncg, D.step0, tgt_base,
                                                  goff + g_off[l], tiles, D.tile0);
    CCFMM_HIP(hipGetLastError());
    tgt_base += (int64_t)D.ngroups * TC;
  }
  CCFMM_HIP(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------- P2P chunks
void build_p2p_chunks(Plan& P, hipStream_t st) {
  LevelData& D = *P.lev[P.L];
  const int nl = D.ncells;
  std::vector<int32_t> start(nl), count(nl);
  CCFMM_HIP(hipMemcpyAsync(start.data(), P.lstart.p, sizeof(int32_t) * nl, hipMemcpyDeviceToHost, st));
  CCFMM_HIP(hipMemcpyAsync(count.data(), P.lcount.p, sizeof(int32_t) * nl, hipMemcpyDeviceToHost, st));
  CCFMM_HIP(hipStreamSynchronize(st));
  std::vector<P2PChunk> ch;
  ch.reserve(nl);
  for (int i = 0; i < nl; i++) {
    for (int off = 0; off < count[i]; off += 64) {
      P2PChunk c;
      c.leaf = i;
      c.first = start[i] + off;
      c.count = std::min(64, count[i] - off);
      c.pad = 0;
      ch.push_back(c);
    }
  }
  P.nchunks = (int64_t)ch.size();
  void* d = P.chunks.ensure(sizeof(P2PChunk) * std::max<size_t>(1, ch.size()));
  CCFMM_HIP(hipMemcpyAsync(d, ch.data(), sizeof(P2PChunk) * ch.size(), hipMemcpyHostToDevice, st));
  CCFMM_HIP(hipStreamSynchronize(st));
}

}  // namespace ccfmm
