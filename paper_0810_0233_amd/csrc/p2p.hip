// p2p.hip -- the field at the dipoles: smooth part from the local expansion
// (Eq. H, with H = -grad V) plus the direct sum over the near smallest cells
// (Eq. H2, read as the field of source dipole j: (3 (m_j.u) u - m_j)/r^3, pairs
// at zero separation skipped), accumulated in FP64 and written in the
// caller's dipole order.
//
// One wavefront per chunk of <= 64 dipoles of one smallest cell.  The c
// dipoles of a chunk are split as c = a + b (a the largest power of two <= c):
// the first a get G1 = 64/a lanes each, the other b get G2 = floor(64/b)
// lanes each, so nearly every lane works in both roles whatever c is.  The
// lanes of a dipole split the sources, and their partial fields are combined
// at the end (butterflies in the first role, a segmented tree in the second).  Sources are staged 64 at a time in LDS,
// packed from consecutive near cells (each shifted by the integer offset of its
// cell so all coordinates stay cell-relative) and padded with null sources
// (zero moment, far away) that add exactly zero, so every lane runs the same
// trip count; the next batch is loaded while the current one is summed.
#include <mutex>
#include <type_traits>

#include "mfma.hpp"
#include "plan.hpp"

namespace ccfmm {

template <typename T>
__device__ __forceinline__ T rsqrt_t(T x);
template <>
__device__ __forceinline__ float rsqrt_t<float>(float x) {
  return __builtin_amdgcn_rsqf(x);
}
template <>
__device__ __forceinline__ double rsqrt_t<double>(double x) {
  // hardware estimate refined by two Newton steps y <- y (3 - x y^2) / 2
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kP2PWaves = 4;

struct P2PArgs {
  const P2PChunk* chunks;
  const int32_t* nchunks;    // device: the number of chunks (the launch covers the capacity)
  const int32_t* near_ptr;   // level L, compact leaves
  const int32_t* near_idx;
  const int32_t* coord;      // level L, compact leaves
  const int32_t* lstart;
  const int32_t* lcount;
  const int32_t* perm;
  int64_t n;
  int nb;
  double g[3];               // leaf sides / smallest leaf side
  double inv_s3;             // 1 / s_L^3
  int64_t voff;              // offset of level L in V
  const int32_t* leaf_p;     // per-cell local order (compact leaves), or null
  const float* ylo;          // FP32 residuals of the positions (SoA [3][n]); null in FP64
};

// readlane of a float or double held as bits
__device__ __forceinline__ uint32_t readlane_t(float v, int k) {
  return (uint32_t)__builtin_amdgcn_readlane((int)__builtin_bit_cast(uint32_t, v), k);
}
__device__ __forceinline__ uint64_t readlane_t(double v, int k) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, k);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), k);
  return ((uint64_t)hi << 32) | lo;
}

// One staged source: position (cell-relative, shifted to the target cell) and
// moment, padded to 8 elements so a lane reads it with two 16-byte loads.
template <typename T>
struct alignas(8 * sizeof(T)) P2PSrc {
  T x, y, z, mx, my, mz, p0, p1;
};
// FP32 residuals of a staged position (exact position = x + lx, ...)
template <typename T>
struct alignas(4 * sizeof(T)) P2PLo {
  T x, y, z, p;
};
// A target dipole: position and its residual (zero in FP64)
template <typename T>
struct P2PTgt {
  T x, y, z, lx, ly, lz;
};

// Blocks of a launch go to the 8 XCDs in turn, each XCD with its own L2.
// Chunks in key order that are close in the list are close in space and share
// source cells, so each XCD is given runs of kXcdRun consecutive block slots:
// XCD x runs block slots x, x + 8, ... of the remapped order, i.e. runs x,
// x + 8, x + 16, ... of kXcdRun chunks-blocks each.  Within a run the sources
// stay in one L2; every XCD still draws runs from the whole domain, which
// keeps uneven work (clustered dipoles) balanced across the XCDs.  Blocks
// past the last whole group of 8 runs keep their order.
constexpr int kXcdRun = 32;
__device__ __forceinline__ int64_t xcd_run_block(int nblk, int bid) {
  const int full = nblk / (8 * kXcdRun) * (8 * kXcdRun);
  if (bid >= full) return bid;
  const int x = bid & 7, s = bid >> 3;
  return ((int64_t)(s / kXcdRun) * 8 + x) * kXcdRun + s % kXcdRun;
}

// One source on one target: f += (3 (m.r) r / r^2 - m) / r^3, written as
// inv3 * (k r - m) with k = 3 (m.r) / r^2.  Only the target's own cell can
// hold a source at zero separation (a position determines its cell), so only
// that cell pays for the test.  With kAcc the separation is formed as
// (hi_t - hi_s) + (lo_t - lo_s): the first difference is exact for close
// points, so r keeps its digits however close the pair (own and adjacent
// cells only; elsewhere r is at least a cell side).
template <typename T, bool kSelf, bool kAcc>
__device__ __forceinline__ void p2p_pair(const P2PSrc<T>& s, const P2PLo<T>* l, const P2PTgt<T>& t, T& fx, T& fy,
                                         T& fz) {
  T rx = t.x - s.x, ry = t.y - s.y, rz = t.z - s.z;
  if (kAcc) {
    const P2PLo<T> q = *l;
    rx += t.lx - q.x;
    ry += t.ly - q.y;
    rz += t.lz - q.z;
  }
  const T r2 = rx * rx + ry * ry + rz * rz;
  T inv = rsqrt_t<T>(r2);
  if (kSelf) inv = (r2 > (T)0) ? inv : (T)0;
  const T inv2 = inv * inv;
  const T inv3 = inv2 * inv;
  const T mr = s.mx * rx + s.my * ry + s.mz * rz;
  const T k = ((T)3 * inv2) * mr;
  fx += inv3 * (k * rx - s.mx);
  fy += inv3 * (k * ry - s.my);
  fz += inv3 * (k * rz - s.mz);
}

// K sources q = sub, sub + G, ... of the staged batch for one target.
template <typename T, int G, bool kSelf, bool kAcc>
__device__ __forceinline__ void p2p_run(const P2PSrc<T>* __restrict__ src, const P2PLo<T>* __restrict__ lo, int sub,
                                        int K, const P2PTgt<T>& t, T& fx, T& fy, T& fz) {
  const P2PSrc<T>* q = src + sub;
  const P2PLo<T>* ql = lo + sub;
  int k = 0;
  for (; k + 4 <= K; k += 4, q += 4 * G, ql += 4 * G) {
#pragma unroll
    for (int u = 0; u < 4; u++) p2p_pair<T, kSelf, kAcc>(q[u * G], ql + u * G, t, fx, fy, fz);
  }
  for (; k < K; k++, q += G, ql += G) p2p_pair<T, kSelf, kAcc>(q[0], ql, t, fx, fy, fz);
}

// G lanes per target: a power of two (first role) or floor(64 / b) for the b
// targets of the second role.  A lane reads slots sub + k G < K G, which can
// pass the 64 staged sources by up to 20 (G = 21): those slots hold null
// sources.
constexpr int kP2PPad = 24;

template <typename T, bool kSelf, bool kAcc>
__device__ __forceinline__ void p2p_role(const P2PSrc<T>* __restrict__ src, const P2PLo<T>* __restrict__ lo, int G,
                                         int sub, int nsrc, const P2PTgt<T>& t, T& fx, T& fy, T& fz) {
  const int K = (nsrc + G - 1) / G;
  switch (G) {
    case 1: p2p_run<T, 1, kSelf, kAcc>(src, lo, sub, K, t, fx, fy, fz); break;
    case 2: p2p_run<T, 2, kSelf, kAcc>(src, lo, sub, K, t, fx, fy, fz); break;
    case 3: p2p_run<T, 3, kSelf, kAcc>(src, lo, sub, K, t, fx, fy, fz); break;
    case 4: p2p_run<T, 4, kSelf, kAcc>(src, lo, sub, K, t, fx, fy, fz); break;
    case 5: p2p_run<T, 5, kSelf, kAcc>(src, lo, sub, K, t, fx, fy, fz); break;
    case 6: p2p_run<T, 6, kSelf, kAcc>(src, lo, sub, K, t, fx, fy, fz); break;
    case 7: p2p_run<T, 7, kSelf, kAcc>(src, lo, sub, K, t, fx, fy, fz); break;
    case 8: p2p_run<T, 8, kSelf, kAcc>(src, lo, sub, K, t, fx, fy, fz); break;
    case 9: p2p_run<T, 9, kSelf, kAcc>(src, lo, sub, K, t, fx, fy, fz); break;
    case 10: p2p_run<T, 10, kSelf, kAcc>(src, lo, sub, K, t, fx, fy, fz); break;
    case 12: p2p_run<T, 12, kSelf, kAcc>(src, lo, sub, K, t, fx, fy, fz); break;
    case 16: p2p_run<T, 16, kSelf, kAcc>(src, lo, sub, K, t, fx, fy, fz); break;
    case 21: p2p_run<T, 21, kSelf, kAcc>(src, lo, sub, K, t, fx, fy, fz); break;
    case 32: p2p_run<T, 32, kSelf, kAcc>(src, lo, sub, K, t, fx, fy, fz); break;
    default: p2p_run<T, 64, kSelf, kAcc>(src, lo, sub, K, t, fx, fy, fz); break;
  }
}

// Smooth field of one dipole from its cell's local expansion,
// H_a = -sum_{|k| <= pl-1} Vt_{k+e_a} yt^k / k!, plus the near field.
template <typename T, int P>
__device__ __forceinline__ void l2p_write(const T* __restrict__ v, int pl, T yx, T yy, T yz, double hx, double hy,
                                          double hz, double s3, double* __restrict__ Ho) {
  constexpr int NM = ncoef(P - 1);
  T px[P], py[P], pz[P];
  px[0] = py[0] = pz[0] = (T)1;
#pragma unroll
  for (int j = 1; j < P; j++) {
    const T inv = (T)(1.0 / j);
    px[j] = px[j - 1] * yx * inv;
    py[j] = py[j - 1] * yy * inv;
    pz[j] = pz[j - 1] * yz * inv;
  }
  (void)NM;
  T ex = (T)0, ey = (T)0, ez = (T)0;
  // degree by degree (the monomials are ordered by degree): a smallest cell
  // with its own order pl keeps |n| <= pl, i.e. |k| <= pl - 1, and stops there
#pragma unroll
  for (int d = 0; d < P; d++) {
    if (d >= pl) break;
#pragma unroll
    for (int k = ncoef(d - 1); k < ncoef(d); k++) {
      const int kx = kMI.x[k], ky = kMI.y[k], kz = kMI.z[k];
      const T mono = px[kx] * py[ky] * pz[kz];
      ex += v[midx(kx + 1, ky, kz) - 1] * mono;
      ey += v[midx(kx, ky + 1, kz) - 1] * mono;
      ez += v[midx(kx, ky, kz + 1) - 1] * mono;
    }
  }
  Ho[0] = s3 * (hx - (double)ex);
  Ho[1] = s3 * (hy - (double)ey);
  Ho[2] = s3 * (hz - (double)ez);
}

// kL2P: also add the smooth field of the cell's local expansion (one pass);
// without it the kernel writes the near field alone and the smooth part is
// added later by k_l2p_batched (so the near field can run beside M2L).
// FP32 asks for 6 waves per SIMD, which spills a few registers (44 bytes a
// lane, held in the caches); at 5 waves nothing spills but the 2^20-dipole
// ferrofluid's near field took 3.15 ms instead of 3.03.
template <typename T, int P, bool kL2P>
__global__ void __launch_bounds__(64 * kP2PWaves, sizeof(T) == 4 ? 6 : 2) k_p2p_l2p(P2PArgs a, const T* __restrict__ y,
                                                           const T* __restrict__ msort, const T* __restrict__ V,
                                                           double* __restrict__ H) {
  constexpr int NS = nstride(P);
  __shared__ P2PSrc<T> sS[kP2PWaves][64 + kP2PPad];
  __shared__ P2PLo<T> sL[kP2PWaves][64 + kP2PPad];
  // the wave index is uniform: say so, so chunk data, counts and loop bounds
  // live in scalar registers and branch on scalar conditions
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t blk = xcd_run_block(gridDim.x, blockIdx.x);
  const int64_t item = blk * kP2PWaves + w;
  const int b = blockIdx.y;
  if (item >= *a.nchunks) return;
  const P2PChunk ch = a.chunks[item];
  const int n = (int)a.n;
  const int c = ch.count;
  int A = 1;
  while (2 * A <= c) A <<= 1;
  const int B = c - A;
  const int G1 = 64 / A, G2 = B > 0 ? 64 / B : 64;  // G2 in {1..10, 12, 16, 21, 32, 64}
  const int t1 = lane / G1, sub1 = lane % G1;
  const int t2 = A + lane / G2, sub2 = lane % G2;
  const bool act2 = B > 0 && t2 < c;
  const int64_t i1 = ch.first + t1, i2 = ch.first + (act2 ? t2 : 0);
  const T x1 = y[i1], y1 = y[n + i1], z1 = y[2 * n + i1];
  const T x2 = y[i2], y2 = y[n + i2], z2 = y[2 * n + i2];
  constexpr bool kLo = std::is_same<T, float>::value;  // FP32 keeps residuals for close pairs
  P2PTgt<T> tg1{x1, y1, z1, (T)0, (T)0, (T)0}, tg2{x2, y2, z2, (T)0, (T)0, (T)0};
  if constexpr (kLo) {
    tg1.lx = (T)a.ylo[i1];
    tg1.ly = (T)a.ylo[n + i1];
    tg1.lz = (T)a.ylo[2 * n + i1];
    tg2.lx = (T)a.ylo[i2];
    tg2.ly = (T)a.ylo[n + i2];
    tg2.lz = (T)a.ylo[2 * n + i2];
  }
  const T* mb = msort + (int64_t)b * 3 * n;
  const int cx = a.coord[3 * ch.leaf], cy = a.coord[3 * ch.leaf + 1], cz = a.coord[3 * ch.leaf + 2];
  P2PSrc<T>* src = sS[w];
  P2PLo<T>* srclo = sL[w];
  if (lane < kP2PPad) {  // null sources past the batch (read by strides that do not divide 64)
    P2PSrc<T> z;
    z.x = z.y = z.z = (T)1e4;
    z.mx = z.my = z.mz = z.p0 = z.p1 = (T)0;
    src[64 + lane] = z;
    P2PLo<T> zl;
    zl.x = zl.y = zl.z = zl.p = (T)0;
    srclo[64 + lane] = zl;
  }
  const int e0 = a.near_ptr[ch.leaf], e1 = a.near_ptr[ch.leaf + 1];
  // Near-list metadata, 64 entries at a time, one entry per lane: first sorted
  // dipole, count, and the cell offset in cell-relative units.  The batch
  // builder below reads it back with readlane (no dependent loads per cell).
  int wb = e0;
  int mstart = 0, mcnt = 0, mself = 0, madj = 0;
  T mox = (T)0, moy = (T)0, moz = (T)0;
  auto load_meta = [&](int base) {
    const int e = base + lane;
    mcnt = 0;
    mself = 0;
    madj = 0;
    if (e < e1) {
      const int S = a.near_idx[e];
      mstart = a.lstart[S];
      mcnt = a.lcount[S];
      mself = S == ch.leaf;
      madj = abs(a.coord[3 * S] - cx) <= 1 && abs(a.coord[3 * S + 1] - cy) <= 1 && abs(a.coord[3 * S + 2] - cz) <= 1;
      mox = (T)((a.coord[3 * S] - cx) * a.g[0]);
      moy = (T)((a.coord[3 * S + 1] - cy) * a.g[1]);
      moz = (T)((a.coord[3 * S + 2] - cz) * a.g[2]);
    }
  };
  load_meta(wb);
  // Batches of up to 64 sources drawn from consecutive near cells (a cell
  // may be split between batches); (e, off) is the cursor.
  int e = e0, off = 0;
  struct Batch {
    int filled;
    bool self;
    bool adj;    // holds the target cell or a neighbour of it (close pairs possible)
    bool valid;  // this lane's slot holds a source
    int64_t j;   // its sorted index
    T ox, oy, oz;
  };
  auto next_batch = [&]() -> Batch {
    Batch bt;
    bt.filled = 0;
    bt.self = false;
    bt.adj = false;
    bt.valid = false;
    bt.j = 0;
    bt.ox = bt.oy = bt.oz = (T)0;
    while (bt.filled < 64 && e < e1) {
      if (e - wb >= 64) {
        wb = e;
        load_meta(wb);
      }
      const int k = e - wb;
      const int cnt = __builtin_amdgcn_readlane(mcnt, k);
      const int st = __builtin_amdgcn_readlane(mstart, k);
      const int take = min(64 - bt.filled, cnt - off);
      if (lane >= bt.filled && lane < bt.filled + take) {
        bt.valid = true;
        bt.j = st + off + (lane - bt.filled);
        bt.ox = __builtin_bit_cast(T, readlane_t(mox, k));
        bt.oy = __builtin_bit_cast(T, readlane_t(moy, k));
        bt.oz = __builtin_bit_cast(T, readlane_t(moz, k));
      }
      bt.self = bt.self || __builtin_amdgcn_readlane(mself, k);
      bt.adj = bt.adj || __builtin_amdgcn_readlane(madj, k);
      bt.filled += take;
      off += take;
      if (off == cnt) {
        e++;
        off = 0;
      }
    }
    return bt;
  };
  // A source shifted into the target cell's frame: hi + o is rounded; with
  // |o| >= |hi| (o a nonzero multiple of the cell side, |hi| at most half of
  // it) the rounding error is exactly hi - ((hi + o) - o), which joins the
  // stored residual.  Returned by value (no address-taken temporaries).
  auto load_src = [&](const Batch& bt) -> P2PSrc<T> {
    P2PSrc<T> q;
    if (bt.valid) {
      const int64_t j = bt.j;
      q.x = y[j] + bt.ox;
      q.y = y[n + j] + bt.oy;
      q.z = y[2 * n + j] + bt.oz;
      q.mx = mb[j];
      q.my = mb[n + j];
      q.mz = mb[2 * n + j];
    } else {  // null source: zero moment, far from every target
      q.x = q.y = q.z = (T)1e4;
      q.mx = q.my = q.mz = (T)0;
    }
    q.p0 = q.p1 = (T)0;
    return q;
  };
  auto load_lo = [&](const Batch& bt, const P2PSrc<T>& q) -> P2PLo<T> {
    P2PLo<T> l;
    l.x = l.y = l.z = l.p = (T)0;
    if (kLo && bt.adj && bt.valid) {
      const int64_t j = bt.j;
      l.x = (y[j] - (q.x - bt.ox)) + (T)a.ylo[j];
      l.y = (y[n + j] - (q.y - bt.oy)) + (T)a.ylo[n + j];
      l.z = (y[2 * n + j] - (q.z - bt.oz)) + (T)a.ylo[2 * n + j];
    }
    return l;
  };
  double hx1 = 0.0, hy1 = 0.0, hz1 = 0.0, hx2 = 0.0, hy2 = 0.0, hz2 = 0.0;  // near field, cell-relative units
  Batch cur = next_batch();
  P2PSrc<T> qc = load_src(cur);
  P2PLo<T> lc = load_lo(cur, qc);
  while (cur.filled > 0) {
    src[lane] = qc;
    if (kLo && cur.adj) srclo[lane] = lc;
    wave_lds_sync();
    // the next batch's loads fly while this one is summed
    const Batch nxt = next_batch();
    const P2PSrc<T> qn = load_src(nxt);
    const P2PLo<T> ln = load_lo(nxt, qn);
    const int nsrc = cur.filled;
    T fx1 = (T)0, fy1 = (T)0, fz1 = (T)0, fx2 = (T)0, fy2 = (T)0, fz2 = (T)0;
    if (cur.self) {
      p2p_role<T, true, kLo>(src, srclo, G1, sub1, nsrc, tg1, fx1, fy1, fz1);
      if (B > 0) p2p_role<T, true, kLo>(src, srclo, G2, sub2, nsrc, tg2, fx2, fy2, fz2);
    } else if (kLo && cur.adj) {
      p2p_role<T, false, kLo>(src, srclo, G1, sub1, nsrc, tg1, fx1, fy1, fz1);
      if (B > 0) p2p_role<T, false, kLo>(src, srclo, G2, sub2, nsrc, tg2, fx2, fy2, fz2);
    } else {
      p2p_role<T, false, false>(src, srclo, G1, sub1, nsrc, tg1, fx1, fy1, fz1);
      if (B > 0) p2p_role<T, false, false>(src, srclo, G2, sub2, nsrc, tg2, fx2, fy2, fz2);
    }
    wave_lds_sync();
    hx1 += (double)fx1;
    hy1 += (double)fy1;
    hz1 += (double)fz1;
    hx2 += (double)fx2;
    hy2 += (double)fy2;
    hz2 += (double)fz2;
    cur = nxt;
    qc = qn;
    lc = ln;
  }
  // combine the lanes of each dipole (they are contiguous: lane = t G + sub)
  for (int off = 1; off < G1; off <<= 1) {
    hx1 += __shfl_xor(hx1, off);
    hy1 += __shfl_xor(hy1, off);
    hz1 += __shfl_xor(hz1, off);
  }
  // second role: G2 need not be a power of two; a segmented tree leaves each
  // dipole's sum in its first lane (sub2 = 0, the one that writes)
  for (int off = 1; off < G2; off <<= 1) {
    const double ox = __shfl_down(hx2, off), oy = __shfl_down(hy2, off), oz = __shfl_down(hz2, off);
    if (sub2 + off < G2) {
      hx2 += ox;
      hy2 += oy;
      hz2 += oz;
    }
  }
  const double s3 = a.inv_s3;
  if constexpr (kL2P) {
    const T* v = V + a.voff + ((int64_t)ch.leaf * a.nb + b) * NS;
    const int pl = a.leaf_p ? a.leaf_p[ch.leaf] : P;
    if (sub1 == 0) l2p_write<T, P>(v, pl, x1, y1, z1, hx1, hy1, hz1, s3, H + ((int64_t)b * n + a.perm[i1]) * 3);
    if (act2 && sub2 == 0)
      l2p_write<T, P>(v, pl, x2, y2, z2, hx2, hy2, hz2, s3, H + ((int64_t)b * n + a.perm[i2]) * 3);
  } else {
    (void)V;
    (void)NS;
    if (sub1 == 0) {
      double* o = H + ((int64_t)b * n + a.perm[i1]) * 3;
      o[0] = s3 * hx1;
      o[1] = s3 * hy1;
      o[2] = s3 * hz1;
    }
    if (act2 && sub2 == 0) {
      double* o = H + ((int64_t)b * n + a.perm[i2]) * 3;
      o[0] = s3 * hx2;
      o[1] = s3 * hy2;
      o[2] = s3 * hz2;
    }
  }
}

// ------------------------------------------------------------ a few configurations
// Near field for 2..31 configurations on the vector units.  The geometry of a
// pair -- separation, reciprocal distance, r^-2 and r^-3 -- is the same for
// every configuration, so it is formed once and applied to KB configurations
// held by the same lane: about 13 + 10 KB operations per pair instead of
// 23 KB.  One wavefront per chunk of <= 64 target dipoles of one smallest
// cell; the c targets get G = floor(64/c) lanes each (the lanes of a target
// split the sources; a chunk of a full 32-dipole cell uses every lane), and
// blockIdx.y runs over groups of KB configurations.  Sources are staged 64 at
// a time in LDS with their moments for the group (zero for configurations
// past the batch), packed from consecutive near cells and padded with null
// sources as in k_p2p_l2p; the next batch is loaded while the current one is
// summed.  FP32 partial fields of a batch are added into FP64 accumulators.

// words of one staged source: position (x, y, z, unused), then m[KB][3],
// rounded up to whole 16-byte LDS reads
template <typename T, int KB>
constexpr int p2pk_words() {
  return ((4 + 3 * KB) * (int)sizeof(T) + 15) / 16 * 16 / (int)sizeof(T);
}

// a staged source in registers: whole 16-byte LDS reads (4 floats or 2
// doubles each); element i of the record is v[i / W][i % W]
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int W = 4;
};
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int W = 2;
};
template <typename T, int KB>
struct SrcRegs {
  static constexpr int W = Vec16<T>::W;
  static constexpr int NV = p2pk_words<T, KB>() / W;
  typename Vec16<T>::type v[NV];
  __device__ __forceinline__ T at(int i) const { return v[i / W][i % W]; }
};
template <typename T, int KB>
__device__ __forceinline__ SrcRegs<T, KB> load_regs(const typename Vec16<T>::type* __restrict__ p) {
  SrcRegs<T, KB> r;
#pragma unroll
  for (int i = 0; i < SrcRegs<T, KB>::NV; i++) r.v[i] = p[i];
  return r;
}

// one source on one target for KB configurations; kSelf: the pair may be at
// zero separation (target's own cell); kAcc: separations formed from the
// FP32 residuals too (own and adjacent cells, where pairs can be close)
template <typename T, int KB, bool kSelf, bool kAcc>
__device__ __forceinline__ void p2pk_pair(const SrcRegs<T, KB>& q, const P2PLo<T>& lo, const P2PTgt<T>& t,
                                          T (&f)[KB][3]) {
  T rx = t.x - q.at(0), ry = t.y - q.at(1), rz = t.z - q.at(2);
  if (kAcc) {
    rx += t.lx - lo.x;
    ry += t.ly - lo.y;
    rz += t.lz - lo.z;
  }
  const T r2 = rx * rx + ry * ry + rz * rz;
  T inv = rsqrt_t<T>(r2);
  if (kSelf) inv = (r2 > (T)0) ? inv : (T)0;
  const T inv2 = inv * inv;
  const T inv3 = inv2 * inv;
  const T c3 = (T)3 * inv2;
#pragma unroll
  for (int b = 0; b < KB; b++) {
    const T mx = q.at(4 + 3 * b), my = q.at(5 + 3 * b), mz = q.at(6 + 3 * b);
    const T k = c3 * (mx * rx + my * ry + mz * rz);
    f[b][0] += inv3 * (k * rx - mx);
    f[b][1] += inv3 * (k * ry - my);
    f[b][2] += inv3 * (k * rz - mz);
  }
}

// the slots sub, sub + G, ... (K >= 1 of them) of the staged batch; the
// next slot's record is read while the current one is summed (the last
// iteration re-reads its own slot rather than pass the batch)
template <typename T, int KB, bool kSelf, bool kAcc>
__device__ __forceinline__ void p2pk_run(const T* __restrict__ src, const P2PLo<T>* __restrict__ lo, int G,
                                         int sub, int K, const P2PTgt<T>& t, T (&f)[KB][3]) {
  using V = typename Vec16<T>::type;
  constexpr int NV = SrcRegs<T, KB>::NV;
  const V* q = reinterpret_cast<const V*>(src) + sub * NV;
  const P2PLo<T>* ql = lo + sub;
  const int step = G * NV;
  SrcRegs<T, KB> cur = load_regs<T, KB>(q);
  P2PLo<T> lcur{(T)0, (T)0, (T)0, (T)0};
  if (kAcc) lcur = ql[0];
  for (int k = 0; k < K; k++) {
    const int kn = min(k + 1, K - 1);
    const SrcRegs<T, KB> nxt = load_regs<T, KB>(q + kn * step);
    P2PLo<T> lnxt{(T)0, (T)0, (T)0, (T)0};
    if (kAcc) lnxt = ql[kn * G];
    p2pk_pair<T, KB, kSelf, kAcc>(cur, lcur, t, f);
    cur = nxt;
    lcur = lnxt;
  }
}

// PL > 0: also add the smooth field of the cell's local expansion (order PL),
// the single-stream form; PL = 0: the near field alone (written, not added),
// the form that runs beside the expansion passes
// Waves per SIMD asked of the compiler: 3, except in FP64 with four
// configurations a block (the LDS records allow 2 blocks per CU, 1 with the
// smooth field) and with the smooth field at the highest orders, whose
// registers would spill at 3.
template <typename T, int KB, int PL>
constexpr int multi_waves() {
  if (sizeof(T) == 8 && KB >= 4) return PL > 0 ? 1 : 2;
  if (sizeof(T) == 8 && PL >= 8) return 1;  // the smooth field's registers at high orders
  if (sizeof(T) == 8 && PL >= 7) return 2;
  if (KB >= 8 && PL >= 8) return 2;
  return 3;
}

template <typename T, int KB, int PL>
__global__ void __launch_bounds__(64 * kP2PWaves, (multi_waves<T, KB, PL>())) k_p2p_multi(P2PArgs a, const T* __restrict__ y,
                                                                 const T* __restrict__ msort, const T* __restrict__ V,
                                                                 double* __restrict__ H) {
  constexpr int NW = p2pk_words<T, KB>();
  constexpr int kSlots = 64 + kP2PPad;
  __shared__ __attribute__((aligned(16))) T sS[kP2PWaves][kSlots * NW];
  __shared__ P2PLo<T> sL[kP2PWaves][kSlots];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t blk = xcd_run_block(gridDim.x, blockIdx.x);
  const int64_t item = blk * kP2PWaves + w;
  if (item >= *a.nchunks) return;
  const int cfg0 = blockIdx.y * KB;
  const int ncfg = min(KB, a.nb - cfg0);  // configurations of this group inside the batch
  const P2PChunk ch = a.chunks[item];
  const int n = (int)a.n;
  const int c = ch.count;
  const int G = 64 / c;  // lanes per target
  const int tt = lane / G, sub = lane % G;
  const bool act = tt < c;
  const int64_t it = ch.first + (act ? tt : 0);
  constexpr bool kLo = std::is_same<T, float>::value;  // FP32 keeps residuals for close pairs
  P2PTgt<T> tg{y[it], y[n + it], y[2 * n + it], (T)0, (T)0, (T)0};
  if constexpr (kLo) {
    tg.lx = (T)a.ylo[it];
    tg.ly = (T)a.ylo[n + it];
    tg.lz = (T)a.ylo[2 * n + it];
  }
  const int cx = a.coord[3 * ch.leaf], cy = a.coord[3 * ch.leaf + 1], cz = a.coord[3 * ch.leaf + 2];
  T* src = sS[w];
  P2PLo<T>* srclo = sL[w];
  if (lane < kP2PPad) {  // null sources past the batch (read by strides that do not divide 64)
    T* z = src + (64 + lane) * NW;
    z[0] = z[1] = z[2] = (T)1e4;
    for (int q = 3; q < NW; q++) z[q] = (T)0;
    P2PLo<T> zl;
    zl.x = zl.y = zl.z = zl.p = (T)0;
    srclo[64 + lane] = zl;
  }
  const int e0 = a.near_ptr[ch.leaf], e1 = a.near_ptr[ch.leaf + 1];
  // near-list metadata, 64 entries at a time (first dipole, count, own cell,
  // adjacent cell, offset in cell-relative units), read back with readlane
  int wb = e0;
  int mstart = 0, mcnt = 0, mself = 0, madj = 0;
  T mox = (T)0, moy = (T)0, moz = (T)0;
  auto load_meta = [&](int base) {
    const int e = base + lane;
    mcnt = 0;
    mself = 0;
    madj = 0;
    if (e < e1) {
      const int S = a.near_idx[e];
      mstart = a.lstart[S];
      mcnt = a.lcount[S];
      mself = S == ch.leaf;
      madj = abs(a.coord[3 * S] - cx) <= 1 && abs(a.coord[3 * S + 1] - cy) <= 1 && abs(a.coord[3 * S + 2] - cz) <= 1;
      mox = (T)((a.coord[3 * S] - cx) * a.g[0]);
      moy = (T)((a.coord[3 * S + 1] - cy) * a.g[1]);
      moz = (T)((a.coord[3 * S + 2] - cz) * a.g[2]);
    }
  };
  load_meta(wb);
  int e = e0, off = 0;
  struct Batch {
    int filled;
    bool self, adj, valid;
    int64_t j;
    T ox, oy, oz;
  };
  auto next_batch = [&]() -> Batch {
    Batch bt;
    bt.filled = 0;
    bt.self = bt.adj = bt.valid = false;
    bt.j = 0;
    bt.ox = bt.oy = bt.oz = (T)0;
    while (bt.filled < 64 && e < e1) {
      if (e - wb >= 64) {
        wb = e;
        load_meta(wb);
      }
      const int k = e - wb;
      const int cnt = __builtin_amdgcn_readlane(mcnt, k);
      const int st = __builtin_amdgcn_readlane(mstart, k);
      const int take = min(64 - bt.filled, cnt - off);
      if (lane >= bt.filled && lane < bt.filled + take) {
        bt.valid = true;
        bt.j = st + off + (lane - bt.filled);
        bt.ox = __builtin_bit_cast(T, readlane_t(mox, k));
        bt.oy = __builtin_bit_cast(T, readlane_t(moy, k));
        bt.oz = __builtin_bit_cast(T, readlane_t(moz, k));
      }
      bt.self = bt.self || __builtin_amdgcn_readlane(mself, k);
      bt.adj = bt.adj || __builtin_amdgcn_readlane(madj, k);
      bt.filled += take;
      off += take;
      if (off == cnt) {
        e++;
        off = 0;
      }
    }
    return bt;
  };
  // this lane's source of a batch: shifted position, its exact rounding
  // error joined to the stored residual (adjacent batches only), moments
  struct Src {
    T v[4 + 3 * KB];
    P2PLo<T> l;
  };
  auto load_src = [&](const Batch& bt) -> Src {
    Src q;
    q.l.x = q.l.y = q.l.z = q.l.p = (T)0;
    q.v[3] = (T)0;
    if (bt.valid) {
      const int64_t j = bt.j;
      const T hx = y[j], hy = y[n + j], hz = y[2 * n + j];
      q.v[0] = hx + bt.ox;
      q.v[1] = hy + bt.oy;
      q.v[2] = hz + bt.oz;
      if (kLo && bt.adj) {
        q.l.x = (hx - (q.v[0] - bt.ox)) + (T)a.ylo[j];
        q.l.y = (hy - (q.v[1] - bt.oy)) + (T)a.ylo[n + j];
        q.l.z = (hz - (q.v[2] - bt.oz)) + (T)a.ylo[2 * n + j];
      }
#pragma unroll
      for (int b = 0; b < KB; b++) {
        const bool in = b < ncfg;
        const T* mb = msort + (int64_t)(in ? cfg0 + b : 0) * 3 * n;
        q.v[4 + 3 * b] = in ? mb[j] : (T)0;
        q.v[5 + 3 * b] = in ? mb[n + j] : (T)0;
        q.v[6 + 3 * b] = in ? mb[2 * n + j] : (T)0;
      }
    } else {  // null source: zero moments, far from every target
      q.v[0] = q.v[1] = q.v[2] = (T)1e4;
#pragma unroll
      for (int b = 0; b < 3 * KB; b++) q.v[4 + b] = (T)0;
    }
    return q;
  };
  double h[KB][3];
#pragma unroll
  for (int b = 0; b < KB; b++) h[b][0] = h[b][1] = h[b][2] = 0.0;
  Batch cur = next_batch();
  Src qc = load_src(cur);
  while (cur.filled > 0) {
    T* slot = src + lane * NW;
#pragma unroll
    for (int q = 0; q < 4 + 3 * KB; q++) slot[q] = qc.v[q];
    if (kLo && cur.adj) srclo[lane] = qc.l;
    wave_lds_sync();
    const Batch nxt = next_batch();
    const Src qn = load_src(nxt);
    const int K = (cur.filled + G - 1) / G;
    T f[KB][3];
#pragma unroll
    for (int b = 0; b < KB; b++) f[b][0] = f[b][1] = f[b][2] = (T)0;
    if (cur.self)
      p2pk_run<T, KB, true, kLo>(src, srclo, G, sub, K, tg, f);
    else if (kLo && cur.adj)
      p2pk_run<T, KB, false, kLo>(src, srclo, G, sub, K, tg, f);
    else
      p2pk_run<T, KB, false, false>(src, srclo, G, sub, K, tg, f);
    wave_lds_sync();
#pragma unroll
    for (int b = 0; b < KB; b++) {
      h[b][0] += (double)f[b][0];
      h[b][1] += (double)f[b][1];
      h[b][2] += (double)f[b][2];
    }
    cur = nxt;
    qc = qn;
  }
  // the G lanes of a target are contiguous (lane = t G + sub), G need not be
  // a power of two: a segmented tree leaves each sum in the lane with sub = 0
  for (int o = 1; o < G; o <<= 1) {
#pragma unroll
    for (int b = 0; b < KB; b++) {
      const double ox = __shfl_down(h[b][0], o), oy = __shfl_down(h[b][1], o), oz = __shfl_down(h[b][2], o);
      if (sub + o < G) {
        h[b][0] += ox;
        h[b][1] += oy;
        h[b][2] += oz;
      }
    }
  }
  if (act && sub == 0) {
    const double s3 = a.inv_s3;
    const int64_t pi = a.perm[it];
    if constexpr (PL > 0) {
      constexpr int NS = nstride(PL);
      const int pl = a.leaf_p ? a.leaf_p[ch.leaf] : PL;
#pragma unroll
      for (int b = 0; b < KB; b++)
        if (b < ncfg)
          l2p_write<T, PL>(V + a.voff + ((int64_t)ch.leaf * a.nb + cfg0 + b) * NS, pl, tg.x, tg.y, tg.z, h[b][0],
                           h[b][1], h[b][2], s3, H + ((int64_t)(cfg0 + b) * n + pi) * 3);
    } else {
      (void)V;
#pragma unroll
      for (int b = 0; b < KB; b++) {
        if (b < ncfg) {
          double* o = H + ((int64_t)(cfg0 + b) * n + pi) * 3;
          o[0] = s3 * h[b][0];
          o[1] = s3 * h[b][1];
          o[2] = s3 * h[b][2];
        }
      }
    }
  }
}

// ------------------------------------------------------------ batched form
// Smooth field for many configurations: one thread per (dipole, configuration),
// written (FP64, caller order) before the batched near field adds to it.
template <typename T, int P, bool kAdd>
__global__ void k_l2p_batched(int64_t n, int nb, const int32_t* __restrict__ dleaf, const int32_t* __restrict__ perm,
                              const T* __restrict__ y, const T* __restrict__ V, int64_t voff, double inv_s3,
                              const int32_t* __restrict__ leaf_p, double* __restrict__ H) {
  constexpr int NS = nstride(P);
  constexpr int NM = ncoef(P - 1);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nb) return;
  const int64_t i = t / nb;
  const int b = (int)(t % nb);
  const T yx = y[i], yy = y[n + i], yz = y[2 * n + i];
  const T* v = V + voff + ((int64_t)dleaf[i] * nb + b) * NS;
  T px[P], py[P], pz[P];
  px[0] = py[0] = pz[0] = (T)1;
#pragma unroll
  for (int j = 1; j < P; j++) {
    const T inv = (T)(1.0 / j);
    px[j] = px[j - 1] * yx * inv;
    py[j] = py[j - 1] * yy * inv;
    pz[j] = pz[j - 1] * yz * inv;
  }
  const int pl = leaf_p ? leaf_p[dleaf[i]] : P;
  (void)NM;
  T ex = (T)0, ey = (T)0, ez = (T)0;
#pragma unroll
  for (int d = 0; d < P; d++) {  // degree by degree, stopping at the cell's order
    if (d >= pl) break;
#pragma unroll
    for (int k = ncoef(d - 1); k < ncoef(d); k++) {
      const int kx = kMI.x[k], ky = kMI.y[k], kz = kMI.z[k];
      const T mono = px[kx] * py[ky] * pz[kz];
      ex += v[midx(kx + 1, ky, kz) - 1] * mono;
      ey += v[midx(kx, ky + 1, kz) - 1] * mono;
      ez += v[midx(kx, ky, kz + 1) - 1] * mono;
    }
  }
  const int64_t o = ((int64_t)b * n + perm[i]) * 3;
  if (kAdd) {  // the near field is already there
    H[o] -= inv_s3 * (double)ex;
    H[o + 1] -= inv_s3 * (double)ey;
    H[o + 2] -= inv_s3 * (double)ez;
  } else {
    H[o] = -inv_s3 * (double)ex;
    H[o + 1] = -inv_s3 * (double)ey;
    H[o + 2] = -inv_s3 * (double)ez;
  }
}

// Near field for many configurations on the matrix cores.  For a chunk of
// <= 32 target dipoles and a batch of source dipoles the field is a product
//   H[(t, a)][b] += sum_{(s, c)} K_ts[a][c] m_s[c][b],
//   K_ts = (3 r r^T / r^2 - I) / r^3,  r = y_t - y_s  (zero for r = 0),
// with 96 rows (32 targets x 3), 48 inner entries (16 sources x 3) and 64
// configuration columns per block (16 per wavefront).  The pair geometry is
// computed once per block and shared by every configuration.  FP32 partial
// products of one source cell are added into FP64 accumulators.
constexpr int kBT = 32;  // targets per chunk
constexpr int kBS = 16;  // sources per step

template <typename T>
__global__ void __launch_bounds__(256) k_p2p_batched(P2PArgs a, const P2PChunk* __restrict__ chunks,
                                                      const int32_t* __restrict__ nchunks,
                                                     const T* __restrict__ y, const T* __restrict__ mt,
                                                     double* __restrict__ H) {
  constexpr int MB = 3 * kBT / 16;  // 6 row blocks
  constexpr int KS = 3 * kBS / 4;   // 12 k steps
  __shared__ T sA[MB * KS * 64];
  __shared__ T sB[4 * KS * 64];
  __shared__ T st[kBT][6];  // position, then its FP32 residual (zero in FP64)
  __shared__ T ss[kBS][6];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int64_t item = blockIdx.x;
  if (item >= *nchunks) return;
  const P2PChunk ch = chunks[item];
  const int nb = a.nb;
  const int cfg0 = blockIdx.y * 64;
  const int64_t n = a.n;
  if (tid < kBT) {
    const bool ok = tid < ch.count;
    const int64_t i = ch.first + (ok ? tid : 0);
    st[tid][0] = y[i];
    st[tid][1] = y[n + i];
    st[tid][2] = y[2 * n + i];
    for (int c = 0; c < 3; c++) st[tid][3 + c] = a.ylo ? (T)a.ylo[c * n + i] : (T)0;
  }
  using AccT = typename Acc<T>::type;
  AccT acc[MB];
  double acc64[MB][4];
#pragma unroll
  for (int mb = 0; mb < MB; mb++) {
    acc[mb] = AccT{0, 0, 0, 0};
    for (int r = 0; r < 4; r++) acc64[mb][r] = 0.0;
  }
  const int cx = a.coord[3 * ch.leaf], cy = a.coord[3 * ch.leaf + 1], cz = a.coord[3 * ch.leaf + 2];
  for (int e = a.near_ptr[ch.leaf]; e < a.near_ptr[ch.leaf + 1]; e++) {
    const int S = a.near_idx[e];
    const T ox = (T)((a.coord[3 * S] - cx) * a.g[0]);
    const T oy = (T)((a.coord[3 * S + 1] - cy) * a.g[1]);
    const T oz = (T)((a.coord[3 * S + 2] - cz) * a.g[2]);
    const int s0 = a.lstart[S], sn = a.lcount[S];
    for (int base = 0; base < sn; base += kBS) {
      const int ns = min(kBS, sn - base);
      __syncthreads();  // previous step's operands fully consumed
      if (tid < kBS) {
        // shifted positions and their exact rounding errors (|offset| >= |y|
        // when the offset is nonzero), joined to the stored residuals: the
        // pair separations below stay exact to rounding for close pairs
        const int64_t j = s0 + base + (tid < ns ? tid : 0);
        const T o[3] = {ox, oy, oz};
        for (int c = 0; c < 3; c++) {
          const T hi = y[c * n + j];
          const T sh = hi + o[c];
          ss[tid][c] = sh;
          ss[tid][3 + c] = (hi - (sh - o[c])) + (a.ylo ? (T)a.ylo[c * n + j] : (T)0);
        }
      }
      // B: rows (source s, component c), columns configurations
#pragma unroll
      for (int r = 0; r < (3 * kBS * 64) / 256; r++) {
        const int q = tid + 256 * r;
        const int row = q >> 6, col = q & 63;
        const int s = row / 3, c = row % 3, b = cfg0 + col;
        T v = (T)0;
        if (s < ns && b < nb) v = mt[((int64_t)(s0 + base + s) * 3 + c) * nb + b];
        sB[((col >> 4) * KS + (row >> 2)) * 64 + (col & 15) + 16 * (row & 3)] = v;
      }
      __syncthreads();
      // A: the 3x3 pair kernels of kBT x kBS pairs, two pairs per thread
#pragma unroll
      for (int r = 0; r < (kBT * kBS) / 256; r++) {
        const int q = tid + 256 * r;
        const int t = q / kBS, s = q % kBS;
        const T rx = (st[t][0] - ss[s][0]) + (st[t][3] - ss[s][3]);
        const T ry = (st[t][1] - ss[s][1]) + (st[t][4] - ss[s][4]);
        const T rz = (st[t][2] - ss[s][2]) + (st[t][5] - ss[s][5]);
        const T r2 = rx * rx + ry * ry + rz * rz;
        const bool ok = t < ch.count && s < ns && r2 > (T)0;
        const T inv = ok ? rsqrt_t<T>(r2) : (T)0;
        const T inv3 = inv * inv * inv;
        const T c5 = (T)3 * inv3 * inv * inv;
        const T rv[3] = {rx, ry, rz};
#pragma unroll
        for (int aa = 0; aa < 3; aa++)
#pragma unroll
          for (int cc = 0; cc < 3; cc++) {
            const T kv = c5 * rv[aa] * rv[cc] - (aa == cc ? inv3 : (T)0);
            const int m = 3 * t + aa, k = 3 * s + cc;
            sA[((m >> 4) * KS + (k >> 2)) * 64 + (m & 15) + 16 * (k & 3)] = kv;
          }
      }
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < KS; ks++) {
        const T bq = sB[(w * KS + ks) * 64 + lane];
#pragma unroll
        for (int mb = 0; mb < MB; mb++) acc[mb] = mfma16x16x4(sA[(mb * KS + ks) * 64 + lane], bq, acc[mb]);
      }
    }
    // fold this source cell's partial products into FP64
#pragma unroll
    for (int mb = 0; mb < MB; mb++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        acc64[mb][r] += (double)acc[mb][r];
        acc[mb][r] = (T)0;
      }
  }
  const int col = lane & 15, kq = lane >> 4;
  const int b = cfg0 + 16 * w + col;
  if (b >= nb) return;
#pragma unroll
  for (int mb = 0; mb < MB; mb++)
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int m = 16 * mb + acc_row<T>(kq, r);
      const int t = m / 3, aa = m % 3;
      if (t < ch.count) {
        const int64_t o = ((int64_t)b * n + a.perm[ch.first + t]) * 3 + aa;
        H[o] = a.inv_s3 * acc64[mb][r];  // first writer: the smooth part is added afterwards
      }
    }
}

// FP32 form of the same product with the pair geometry off the critical path.
// A chunk of <= 32 targets (96 rows) meets blocks of 32 source dipoles (96
// contraction entries) packed from consecutive near cells and padded with null
// sources (zero kernel), so a cell of 28 dipoles does not leave a ragged block.
// Each wavefront owns 16 of the block's 64 configuration columns.  The pair
// kernels of block i+1 are written by all four wavefronts into the other half
// of a double-buffered LDS operator while the matrix cores multiply block i,
// and the moments of block i+1 are loaded into registers meanwhile, so a block
// costs a single barrier.  Separations always take the exact form
// (hi_t - hi_s) + (lo_t - lo_s), whatever the cells.  Block products are added
// into FP64 accumulators.
//
// Contraction order: in matrix step ks (0..23) lane group kq = lane / 16 holds
// source s = 8 kq + ks / 3, component ks % 3.  Operator layout per buffer: the
// fragment of row block mb, steps 4 k4 .. 4 k4 + 3 is one float4 per lane at
// ((mb * 6 + k4) * 64 + lane) * 4.  The pair (t, s) is built by the lane with
// t % 16 = lane % 16 of wavefront s / 8, whose 64 lanes then write 64 distinct
// banks per store.
constexpr int kMT = 32;  // target dipoles per chunk
constexpr int kMS = 32;  // source dipoles per block

// a slot of a source block (lane % 32 holds slot lane % 32): sorted index
// (-1: null source) and the offset of its cell from the target cell
struct MSlot {
  int j;
  float ox, oy, oz;
};
struct MBlock {
  int filled;
  MSlot s;
};
// one source of a thread's pairs as loaded: position, residual, cell offset
struct MSrc {
  float x, y, z, lx, ly, lz, ox, oy, oz;
  int ok;
};

constexpr int kMK4 = 3 * kMS / 16;              // float4 groups of matrix steps (6)
constexpr int kMNA = (3 * kMT / 16) * kMK4 * 256;  // operator words per buffer

// One chunk with MBU of its six 16-row blocks in use (rows 3 count .. 95 hold
// no target and are skipped).
template <int MBU>
__device__ __forceinline__ void p2p_mfma_chunk(const P2PArgs& a, const P2PChunk& ch, const float* __restrict__ y,
                                               const float* __restrict__ mt, double* __restrict__ H,
                                               float (*__restrict__ sA)[kMNA]) {
  constexpr int KS = 3 * kMS / 4;  // 24 matrix steps per block
  constexpr int K4 = kMK4;
  constexpr int MB = MBU;
  constexpr bool kHi = MBU > 3;    // second target (t0 + 16, rows >= 48) in use
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t n = a.n;
  const int nb = a.nb;
  const float* __restrict__ ylo = a.ylo;

  // targets of this thread's pairs (t0 and t0 + 16) and their store offsets
  const int t0 = lane & 15, sq = lane >> 4;
  float tx[2], ty[2], tz[2], tlx[2], tly[2], tlz[2];
  int rowoff[2][3], coloff[2][3];
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const int t = t0 + 16 * h;
    const int64_t i = ch.first + (t < ch.count ? t : 0);
    tx[h] = y[i];
    ty[h] = y[n + i];
    tz[h] = y[2 * n + i];
    tlx[h] = ylo[i];
    tly[h] = ylo[n + i];
    tlz[h] = ylo[2 * n + i];
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const int m = 3 * t + c;
      rowoff[h][c] = ((m >> 4) * K4 * 64 + (m & 15)) * 4;
      const int ks = 3 * (sq + 4 * h) + c;  // this thread's sources: 8 w + sq + 4 h
      coloff[h][c] = ((ks >> 2) * 64 + 16 * w) * 4 + (ks & 3);
    }
  }
  // this lane's configuration column and fragment rows
  const int kq = lane >> 4;
  const int b = blockIdx.y * 64 + 16 * w + (lane & 15);
  const int bcl = b < nb ? b : nb - 1;

  // near-list metadata, 64 entries at a time, one per lane (read by readlane)
  const int cx = a.coord[3 * ch.leaf], cy = a.coord[3 * ch.leaf + 1], cz = a.coord[3 * ch.leaf + 2];
  const int e1 = a.near_ptr[ch.leaf + 1];
  int e = a.near_ptr[ch.leaf], off = 0, wb = e;
  int mstart = 0, mcnt = 0;
  float mox = 0.f, moy = 0.f, moz = 0.f;
  auto load_meta = [&](int base) {
    const int q = base + lane;
    mcnt = 0;
    if (q < e1) {
      const int S = a.near_idx[q];
      mstart = a.lstart[S];
      mcnt = a.lcount[S];
      mox = (float)((a.coord[3 * S] - cx) * a.g[0]);
      moy = (float)((a.coord[3 * S + 1] - cy) * a.g[1]);
      moz = (float)((a.coord[3 * S + 2] - cz) * a.g[2]);
    }
  };
  load_meta(wb);
  const int slot = lane & 31;
  // next block of up to 32 sources from consecutive near cells; (e, off) is
  // the cursor, identical in all wavefronts (same data, same steps)
  auto next_block = [&]() -> MBlock {
    MBlock bk;
    bk.filled = 0;
    bk.s.j = -1;
    bk.s.ox = bk.s.oy = bk.s.oz = 0.f;
    while (bk.filled < kMS && e < e1) {
      if (e - wb >= 64) {
        wb = e;
        load_meta(wb);
      }
      const int k = e - wb;
      const int cnt = __builtin_amdgcn_readlane(mcnt, k);
      const int st = __builtin_amdgcn_readlane(mstart, k);
      const int take = min(kMS - bk.filled, cnt - off);
      if (slot >= bk.filled && slot < bk.filled + take) {
        bk.s.j = st + off + slot - bk.filled;
        bk.s.ox = __builtin_bit_cast(float, readlane_t(mox, k));
        bk.s.oy = __builtin_bit_cast(float, readlane_t(moy, k));
        bk.s.oz = __builtin_bit_cast(float, readlane_t(moz, k));
      }
      bk.filled += take;
      off += take;
      if (off == cnt) {
        e++;
        off = 0;
      }
    }
    return bk;
  };
  // source 8 w + sq + 4 h of a block, as this thread's pairs need it
  auto fetch = [&](const MSlot& S, int h) -> MSrc {
    const int s = 8 * w + sq + 4 * h;
    MSrc q;
    const int j = __shfl(S.j, s);
    q.ok = j >= 0;
    const int64_t jj = j >= 0 ? j : 0;
    q.ox = __shfl(S.ox, s);
    q.oy = __shfl(S.oy, s);
    q.oz = __shfl(S.oz, s);
    q.x = y[jj];
    q.y = y[n + jj];
    q.z = y[2 * n + jj];
    q.lx = ylo[jj];
    q.ly = ylo[n + jj];
    q.lz = ylo[2 * n + jj];
    return q;
  };
  // moments of a block, fragment rows of this lane (null sources read dipole 0:
  // their operator entries are zero)
  auto load_b = [&](const MSlot& S, float (&B)[KS]) {
#pragma unroll
    for (int q = 0; q < 8; q++) {
      const int j = __shfl(S.j, 8 * kq + q);
      const float* p = mt + (int64_t)(j >= 0 ? j : 0) * 3 * nb + bcl;
#pragma unroll
      for (int c = 0; c < 3; c++) B[3 * q + c] = p[c * nb];
    }
  };
  // pair kernels of one source with this thread's two targets, into buffer dst.
  // The shifted source is rounded; with |offset| >= |position| (a nonzero
  // offset is a multiple of the cell side) the rounding error is exactly
  // x - ((x + o) - o), which joins the stored residual.
  auto gen = [&](float* __restrict__ dst, const MSrc& q, int h) {
    const float sx = q.x + q.ox, sy = q.y + q.oy, sz = q.z + q.oz;
    const float slx = (q.x - (sx - q.ox)) + q.lx;
    const float sly = (q.y - (sy - q.oy)) + q.ly;
    const float slz = (q.z - (sz - q.oz)) + q.lz;
#pragma unroll
    for (int tt = 0; tt < (kHi ? 2 : 1); tt++) {
      const float rx = (tx[tt] - sx) + (tlx[tt] - slx);
      const float ry = (ty[tt] - sy) + (tly[tt] - sly);
      const float rz = (tz[tt] - sz) + (tlz[tt] - slz);
      const float r2 = rx * rx + ry * ry + rz * rz;
      const bool ok = q.ok != 0 && r2 > 0.f;
      const float inv = ok ? rsqrt_t<float>(r2) : 0.f;
      const float inv2 = inv * inv;
      const float inv3 = inv2 * inv;
      const float c5 = 3.f * inv3 * inv2;
      const float ux = c5 * rx, uy = c5 * ry, uz = c5 * rz;
      const float kxy = ux * ry, kxz = ux * rz, kyz = uy * rz;
      const int* ro = rowoff[tt];
      const int* co = coloff[h];
      dst[ro[0] + co[0]] = ux * rx - inv3;
      dst[ro[0] + co[1]] = kxy;
      dst[ro[0] + co[2]] = kxz;
      dst[ro[1] + co[0]] = kxy;
      dst[ro[1] + co[1]] = uy * ry - inv3;
      dst[ro[1] + co[2]] = kyz;
      dst[ro[2] + co[0]] = kxz;
      dst[ro[2] + co[1]] = kyz;
      dst[ro[2] + co[2]] = uz * rz - inv3;
    }
  };
  f32x4 acc[MB];
  double acc64[MB][4];
#pragma unroll
  for (int mb = 0; mb < MB; mb++)
#pragma unroll
    for (int r = 0; r < 4; r++) acc64[mb][r] = 0.0;
  auto products = [&](const float* __restrict__ A, const float (&B)[KS]) {
#pragma unroll
    for (int mb = 0; mb < MB; mb++) acc[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k4 = 0; k4 < K4; k4++) {
      f32x4 av[MB];
#pragma unroll
      for (int mb = 0; mb < MB; mb++) av[mb] = *reinterpret_cast<const f32x4*>(A + ((mb * K4 + k4) * 64 + lane) * 4);
#pragma unroll
      for (int ku = 0; ku < 4; ku++)
#pragma unroll
        for (int mb = 0; mb < MB; mb++) acc[mb] = mfma16x16x4(av[mb][ku], B[4 * k4 + ku], acc[mb]);
    }
#pragma unroll
    for (int mb = 0; mb < MB; mb++)
#pragma unroll
      for (int r = 0; r < 4; r++) acc64[mb][r] += (double)acc[mb][r];
  };

  // all of this wavefront's memory loads have landed (vmcnt = 0)
  auto wait_loads = [] { __builtin_amdgcn_s_waitcnt(0x0F70); };
  // Loads from read-only memory may otherwise be sunk below the barrier to
  // their first use in the next step, where they would stall the products:
  // an empty consumer holds each value here, where the wait is anyway.
  auto hold = [](float v) { asm volatile("" ::"v"(v)); };
  auto hold_b = [&](const float (&B)[KS]) {
#pragma unroll
    for (int k = 0; k < KS; k++) hold(B[k]);
  };
  auto hold_r = [&](const MSrc (&R)[2]) {
#pragma unroll
    for (int h = 0; h < 2; h++) {
      hold(R[h].x);
      hold(R[h].y);
      hold(R[h].z);
      hold(R[h].lx);
      hold(R[h].ly);
      hold(R[h].lz);
    }
  };
  // prologue: block 0 built into buffer 0 with its moments loaded, block 1 fetched
  const MBlock b0 = next_block();
  MBlock bn = next_block();
  float B0[KS], B1[KS];
  MSrc RA[2], RB[2];
  int fc = b0.filled;
  RB[0] = fetch(b0.s, 0);
  RB[1] = fetch(b0.s, 1);
  load_b(b0.s, B0);
  RA[0] = fetch(bn.s, 0);
  RA[1] = fetch(bn.s, 1);
  gen(sA[0], RB[0], 0);
  gen(sA[0], RB[1], 1);
  wait_loads();
  hold_b(B0);
  hold_r(RA);
  __syncthreads();
  // one block: the builder runs while no load is in flight; then the moments
  // of block i+1 and the sources of block i+2 are requested, and the products
  // of buffer cur run beside the construction of block i+1 in the other one.
  // Loads are unconditional (an empty block reads dipole 0 and builds zeros).
  auto step = [&](int cur, float (&Bc)[KS], float (&Bn)[KS], MSrc (&Rc)[2], MSrc (&Rn)[2]) {
    const MBlock b2 = next_block();
    load_b(bn.s, Bn);
    Rn[0] = fetch(b2.s, 0);
    Rn[1] = fetch(b2.s, 1);
    __builtin_amdgcn_sched_barrier(0);  // issue the loads before the products
    products(sA[cur], Bc);
    gen(sA[cur ^ 1], Rc[0], 0);
    gen(sA[cur ^ 1], Rc[1], 1);
    __builtin_amdgcn_sched_barrier(0);
    wait_loads();
    hold_b(Bn);
    hold_r(Rn);
    __syncthreads();
    fc = bn.filled;
    bn = b2;
  };
  while (fc > 0) {
    step(0, B0, B1, RA, RB);
    if (fc == 0) break;
    step(1, B1, B0, RB, RA);
  }

  // write: lane holds rows 16 mb + 4 kq + r of column b
  if (b >= nb) return;
#pragma unroll
  for (int mb = 0; mb < MB; mb++)
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int m = 16 * mb + acc_row<float>(kq, r);
      const int t = m / 3, aa = m % 3;
      if (t < ch.count) {
        const int64_t o = ((int64_t)b * n + a.perm[ch.first + t]) * 3 + aa;
        H[o] = a.inv_s3 * acc64[mb][r];  // first writer: the smooth part is added afterwards
      }
    }
}

__global__ void __launch_bounds__(256, 2) k_p2p_mfma(P2PArgs a, const P2PChunk* __restrict__ chunks,
                                                     const int32_t* __restrict__ nchunks, const float* __restrict__ y,
                                                     const float* __restrict__ mt, double* __restrict__ H) {
  __shared__ __attribute__((aligned(16))) float sA[2][kMNA];
  const int64_t item = xcd_run_block(gridDim.x, blockIdx.x);
  if (item >= *nchunks) return;
  const P2PChunk ch = chunks[item];
  switch ((3 * ch.count + 15) / 16) {  // row blocks in use (uniform over the block)
    case 1: p2p_mfma_chunk<1>(a, ch, y, mt, H, sA); break;
    case 2: p2p_mfma_chunk<2>(a, ch, y, mt, H, sA); break;
    case 3: p2p_mfma_chunk<3>(a, ch, y, mt, H, sA); break;
    case 4: p2p_mfma_chunk<4>(a, ch, y, mt, H, sA); break;
    case 5: p2p_mfma_chunk<5>(a, ch, y, mt, H, sA); break;
    default: p2p_mfma_chunk<6>(a, ch, y, mt, H, sA); break;
  }
}

static P2PArgs p2p_args(Plan& P, int nb, bool fp64) {
  LevelData& D = *P.lev[P.L];
  P2PArgs a;
  a.chunks = P.chunks.as<P2PChunk>();
  a.nchunks = P.chunk_cnt.as<int32_t>() + (P.lev[P.L]->ncells + 1) + P.lev[P.L]->ncells;  // off[nl]
  a.near_ptr = D.near_ptr.as<int32_t>();
  a.near_idx = D.near_idx.as<int32_t>();
  a.coord = D.coord.as<int32_t>();
  a.lstart = P.lstart.as<int32_t>();
  a.lcount = P.lcount.as<int32_t>();
  a.perm = P.perm.as<int32_t>();
  a.n = P.n;
  a.nb = nb;
  for (int q = 0; q < 3; q++) a.g[q] = P.geo.lev[P.L].g[q];
  const double s = P.geo.lev[P.L].s;
  a.inv_s3 = 1.0 / (s * s * s);
  a.voff = D.qoff;
  a.leaf_p = P.has_leaf ? P.leaf_p.as<int32_t>() : nullptr;
  a.ylo = fp64 ? nullptr : P.yf.as<float>() + 3 * P.n;
  return a;
}

// configurations per lane of the few-configuration near field: the group
// size with the fewest vector operations, ceil(nb / KB) (13 + 10 KB) per
// pair (FP64 stops at 4, its registers being twice as wide)
static int multi_group(int nb, bool fp64) {
  int best = 2;
  double best_ops = 1e300;
  for (int kb : {2, 4, 8}) {
    if (fp64 && kb > 4) continue;
    const double ops = (double)ceil_div(nb, kb) * (13.0 + 10.0 * kb);
    if (ops < best_ops) {
      best_ops = ops;
      best = kb;
    }
  }
  return best;
}

template <typename T, int KB, int PL>
static void multi_launch(Plan& P, const P2PArgs& a, const T* y, int nb, double* d_H, hipStream_t st) {
  dim3 grid(ceil_div(P.nchunks_cap, kP2PWaves), ceil_div(nb, KB));
  k_p2p_multi<T, KB, PL><<<grid, 64 * kP2PWaves, 0, st>>>(a, y, P.m_sorted.as<T>(), P.V.as<T>(), d_H);
}

// the few-configuration near field in groups of multi_group(nb); PL > 0 adds
// the smooth field of order PL
template <typename T, int PL>
static void multi_dispatch(Plan& P, const P2PArgs& a, const T* y, int nb, double* d_H, hipStream_t st) {
  const int kb = multi_group(nb, std::is_same<T, double>::value);
  if (kb == 2)
    multi_launch<T, 2, PL>(P, a, y, nb, d_H, st);
  else if (kb == 4)
    multi_launch<T, 4, PL>(P, a, y, nb, d_H, st);
  else if constexpr (!std::is_same<T, double>::value)
    multi_launch<T, 8, PL>(P, a, y, nb, d_H, st);
}

// near field alone: written (not added) to H in the caller's order
template <typename T, int PP>
static void near_impl(Plan& P, int nb, double* d_H, hipStream_t st) {
  const bool fp64 = std::is_same<T, double>::value;
  const T* y = fp64 ? (const T*)P.yd.p : (const T*)P.yf.p;
  P2PArgs a = p2p_args(P, nb, fp64);
  if (nb >= 2 && nb < P.batched_min) {
    multi_dispatch<T, 0>(P, a, y, nb, d_H, st);
  } else if (nb >= P.batched_min) {
    const int nl = P.lev[P.L]->ncells;
    const int32_t* n32 = P.chunk_cnt.as<int32_t>() + 3 * (nl + 1) + nl;  // off32[nl]
    dim3 grid((unsigned)P.nchunks32_cap, ceil_div(nb, 64));
    if constexpr (std::is_same<T, float>::value)
      k_p2p_mfma<<<grid, 256, 0, st>>>(a, P.chunks32.as<P2PChunk>(), n32, y, P.m_sorted_t.as<float>(), d_H);
    else
      k_p2p_batched<T><<<grid, 256, 0, st>>>(a, P.chunks32.as<P2PChunk>(), n32, y, P.m_sorted_t.as<T>(),
                                             d_H);
  } else {
    dim3 grid(ceil_div(P.nchunks_cap, kP2PWaves), nb);
    k_p2p_l2p<T, PP, false><<<grid, 64 * kP2PWaves, 0, st>>>(a, y, P.m_sorted.as<T>(), P.V.as<T>(), d_H);
  }
  CCFMM_HIP(hipGetLastError());
}

// smooth field of the local expansions, added to the near field in H
template <typename T, int PP>
static void l2p_impl(Plan& P, int nb, double* d_H, hipStream_t st) {
  const T* y = std::is_same<T, double>::value ? (const T*)P.yd.p : (const T*)P.yf.p;
  const double s = P.geo.lev[P.L].s;
  k_l2p_batched<T, PP, true><<<ceil_div(P.n * nb, 256), 256, 0, st>>>(
      P.n, nb, P.dleaf.as<int32_t>(), P.perm.as<int32_t>(), y, P.V.as<T>(), P.lev[P.L]->qoff, 1.0 / (s * s * s),
      P.has_leaf ? P.leaf_p.as<int32_t>() : nullptr, d_H);
  CCFMM_HIP(hipGetLastError());
}

// both in one pass (single stream): one configuration, or 2..31 configurations
// sharing each pair's geometry; from the matrix-core size, two kernels
template <typename T, int PP>
static void fused_impl(Plan& P, int nb, double* d_H, hipStream_t st) {
  if (nb >= P.batched_min) {  // matrix-core near field, then the smooth field added
    near_impl<T, PP>(P, nb, d_H, st);
    l2p_impl<T, PP>(P, nb, d_H, st);
    return;
  }
  const bool fp64 = std::is_same<T, double>::value;
  const T* y = fp64 ? (const T*)P.yd.p : (const T*)P.yf.p;
  P2PArgs a = p2p_args(P, nb, fp64);
  if (nb >= 2) {
    multi_dispatch<T, PP>(P, a, y, nb, d_H, st);
    CCFMM_HIP(hipGetLastError());
    return;
  }
  dim3 grid(ceil_div(P.nchunks_cap, kP2PWaves), nb);
  k_p2p_l2p<T, PP, true><<<grid, 64 * kP2PWaves, 0, st>>>(a, y, P.m_sorted.as<T>(), P.V.as<T>(), d_H);
  CCFMM_HIP(hipGetLastError());
}

template <int PP>
static void near_d(Plan& P, int nb, double* d_H, hipStream_t st) {
  if (P.precision == CCFMM_PREC_FP64)
    near_impl<double, PP>(P, nb, d_H, st);
  else
    near_impl<float, PP>(P, nb, d_H, st);
}
template <int PP>
static void l2p_d(Plan& P, int nb, double* d_H, hipStream_t st) {
  if (P.precision == CCFMM_PREC_FP64)
    l2p_impl<double, PP>(P, nb, d_H, st);
  else
    l2p_impl<float, PP>(P, nb, d_H, st);
}
template <int PP>
static void fused_d(Plan& P, int nb, double* d_H, hipStream_t st) {
  if (P.precision == CCFMM_PREC_FP64)
    fused_impl<double, PP>(P, nb, d_H, st);
  else
    fused_impl<float, PP>(P, nb, d_H, st);
}

#define CCFMM_P2P_DISPATCH(FN)                                \
  switch (P.p) {                                              \
    case 1: FN<1>(P, nb, d_H, st); break;                     \
    case 2: FN<2>(P, nb, d_H, st); break;                     \
    case 3: FN<3>(P, nb, d_H, st); break;                     \
    case 4: FN<4>(P, nb, d_H, st); break;                     \
    case 5: FN<5>(P, nb, d_H, st); break;                     \
    case 6: FN<6>(P, nb, d_H, st); break;                     \
    case 7: FN<7>(P, nb, d_H, st); break;                     \
    case 8: FN<8>(P, nb, d_H, st); break;                     \
    default: fail(CCFMM_EINVAL, "order out of range");        \
  }

void run_near(Plan& P, int nb, double* d_H, hipStream_t st) { CCFMM_P2P_DISPATCH(near_d) }
void run_l2p(Plan& P, int nb, double* d_H, hipStream_t st) { CCFMM_P2P_DISPATCH(l2p_d) }
void run_p2p_l2p(Plan& P, int nb, double* d_H, hipStream_t st) { CCFMM_P2P_DISPATCH(fused_d) }
#undef CCFMM_P2P_DISPATCH

// ------------------------------------------------------------ direct sum
// FP64 O(N) per target: the plain definition of the field at sampled targets,
// one wavefront per target, sources split over lanes and reduced by butterfly.
__global__ void __launch_bounds__(256) k_direct_targets(int64_t n, const double* __restrict__ pos,
                                                        const double* __restrict__ m, int64_t nt,
                                                        const int64_t* __restrict__ idx, double* __restrict__ H) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + w;
  if (t >= nt) return;
  const int64_t i = idx[t];
  if (i < 0 || i >= n) {  // out-of-range target: report NaN, touch nothing
    if (lane == 0) H[3 * t] = H[3 * t + 1] = H[3 * t + 2] = __builtin_nan("");
    return;
  }
  const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
  double hx = 0.0, hy = 0.0, hz = 0.0;
  for (int64_t j = lane; j < n; j += 64) {
    const double rx = xi - pos[3 * j], ry = yi - pos[3 * j + 1], rz = zi - pos[3 * j + 2];
    const double r2 = rx * rx + ry * ry + rz * rz;
    if (r2 == 0.0) continue;
    const double inv = 1.0 / sqrt(r2);
    const double inv3 = inv * inv * inv;
    const double mr = m[3 * j] * rx + m[3 * j + 1] * ry + m[3 * j + 2] * rz;
    const double c = 3.0 * mr * inv * inv * inv3;
    hx += c * rx - inv3 * m[3 * j];
    hy += c * ry - inv3 * m[3 * j + 1];
    hz += c * rz - inv3 * m[3 * j + 2];
  }
  for (int off = 1; off < 64; off <<= 1) {
    hx += __shfl_xor(hx, off);
    hy += __shfl_xor(hy, off);
    hz += __shfl_xor(hz, off);
  }
  if (lane == 0) {
    H[3 * t] = hx;
    H[3 * t + 1] = hy;
    H[3 * t + 2] = hz;
  }
}

// ------------------------------------------------------------ energy
// E_b = -1/2 sum_i m_i . H_i (Sec. 3 with the Appendix's factor 1/2) per
// configuration, FP64.  A fixed grid of kEnergyBlocks blocks per
// configuration each sums a contiguous range of the 3n products (threads
// strided, then a tree in LDS); one block per configuration adds the partial
// sums in block order.  The order of every addition depends on n only, so
// the result is the same on every call.
constexpr int kEnergyBlocks = 256;

__global__ void __launch_bounds__(256) k_energy_part(int64_t n3, const double* __restrict__ m,
                                                     const double* __restrict__ H, double* __restrict__ part) {
  __shared__ double sh[256];
  const int b = blockIdx.y, g = blockIdx.x, t = threadIdx.x;
  const int64_t chunk = (n3 + kEnergyBlocks - 1) / kEnergyBlocks;
  const int64_t lo = (int64_t)g * chunk, hi = min(n3, lo + chunk);
  const double* mb = m + (int64_t)b * n3;
  const double* hb = H + (int64_t)b * n3;
  double s = 0.0;
  for (int64_t i = lo + t; i < hi; i += 256) s += mb[i] * hb[i];
  sh[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  if (t == 0) part[(int64_t)b * kEnergyBlocks + g] = sh[0];
}

__global__ void __launch_bounds__(256) k_energy_final(const double* __restrict__ part, double* __restrict__ E) {
  __shared__ double sh[256];
  const int b = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int g = t; g < kEnergyBlocks; g += 256) s += part[(int64_t)b * kEnergyBlocks + g];
  sh[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  if (t == 0) E[b] = -0.5 * sh[0];
}

void run_energy(Plan& P, int nb, const double* d_m, const double* d_H, double* d_E, hipStream_t st) {
  double* part = reinterpret_cast<double*>(P.energy_part.ensure(sizeof(double) * (size_t)kEnergyBlocks * nb));
  k_energy_part<<<dim3(kEnergyBlocks, nb), 256, 0, st>>>(3 * P.n, d_m, d_H, part);
  CCFMM_HIP(hipGetLastError());
  k_energy_final<<<nb, 256, 0, st>>>(part, d_E);
  CCFMM_HIP(hipGetLastError());
}

// ------------------------------------------------------------ energy, no allocation
// The same energy with its partial sums in a fixed device array instead of a
// plan buffer, for callers that cannot allocate device memory (graph capture,
// serving loops).  Every GPU the library runs on holds its own copy of the
// array until the process ends.  Host code never passes the array's name to
// a kernel (that is a host-side stand-in); it looks up the device address
// once per device and passes that.  k_energy_part writes every slot that
// k_energy_final reads, so nothing needs clearing; overlapping calls on one
// GPU share the array and race.
static __device__ __align__(256) double scratch[kEnergyBlocks * CCFMM_NOALLOC_MAX_BATCH];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's scratch array (looked up on first use)
static double* scratch_for_current_device() {
  int dev = -1;
  CCFMM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(CCFMM_EINVAL, "device ordinal beyond the supported 64");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    CCFMM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(CCFMM_EHIP, "no device address for the energy scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  return static_cast<double*>(g_scratch_ptr[dev]);
}

void run_energy_noalloc(int64_t n, int nb, const double* d_m, const double* d_H, double* d_E, hipStream_t st) {
  if (nb < 1 || nb > CCFMM_NOALLOC_MAX_BATCH)
    fail(CCFMM_EINVAL, "nbatch must be in 1.." + std::to_string(CCFMM_NOALLOC_MAX_BATCH) +
                           " (the fixed partial-sum array holds that many configurations)");
  double* part = scratch_for_current_device();
  k_energy_part<<<dim3(kEnergyBlocks, nb), 256, 0, st>>>(3 * n, d_m, d_H, part);
  CCFMM_HIP(hipGetLastError());
  k_energy_final<<<nb, 256, 0, st>>>(part, d_E);
  CCFMM_HIP(hipGetLastError());
}

void run_direct_targets(int64_t n, const double* d_pos, const double* d_m, int64_t nt, const int64_t* d_idx,
                        double* d_H, hipStream_t st) {
  if (nt <= 0) return;
  k_direct_targets<<<ceil_div(nt, 4), 256, 0, st>>>(n, d_pos, d_m, nt, d_idx, d_H);
  CCFMM_HIP(hipGetLastError());
}

}  // namespace ccfmm
