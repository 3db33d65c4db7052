// m2l.hip -- the M2L pass, Eq.(taylorcalc), on the matrix cores.
//
// For target cell C and source cell A at integer offset delta (same level),
//   Vt_n(C) += (-1)^|n| sum_q D_{n+q}(c) Qt_q(A),   1 <= |n|, |q| <= p,
// in the level's scaled units (c = target minus source centre).  The operator
// depends only on the offset, so the pairs are grouped by offset: a block of
// four wavefronts owns a tile of 64 columns (target cell, configuration) whose
// cells share one list of offsets, and walks that list.  Each step is a dense
// [NP x NP] x [NP x 64] product on the MFMA units: the step's operator is
// materialised once in LDS, in MFMA operand order, from the ncoef(2p)
// derivative-tensor entries (it is Hankel-like: entry (n, q) is D_{n+q}), and
// all four wavefronts read it conflict-free for their 16 columns each.  The
// accumulators stay in registers for the whole walk, so each target column is
// written once and no atomics are needed.
#include <type_traits>

#include "mfma.hpp"
#include "plan.hpp"

namespace ccfmm {

struct LevelOffsets {
  int64_t qoff[kLMax + 1];
};

// Compile-time shape of the M2L kernel for order P and element type T.
template <typename T, int P>
struct M2LShape {
  static constexpr int NP = nact(P);
  static constexpr int NS = nstride(P);      // K extent (multiple of 4)
  static constexpr int MB = (NP + 15) / 16;  // 16-row blocks
  static constexpr int KS = NS / 4;          // k steps of 4
  static constexpr int ND = ncoef(2 * P);    // derivative-tensor entries
  static constexpr int QST = 65;             // padded stride of one Q fragment
  static constexpr int LDS_Q = 4 * KS * QST * (int)sizeof(T);
  static constexpr int LDS_D = (ND + 1) * (int)sizeof(T);
  static constexpr int LDS_MB = KS * 64 * (int)sizeof(T);  // one M-block of operator
  // two blocks per CU when the operator fits in ~76 KB, else one
  static constexpr int BUDGET = (LDS_Q + LDS_D + LDS_MB <= 76 * 1024) ? 76 * 1024 : 156 * 1024;
  static constexpr int MBC_FIT = (BUDGET - LDS_Q - LDS_D) / LDS_MB;
  static constexpr int MBC = MBC_FIT < MB ? MBC_FIT : MB;   // M-blocks per operator chunk
  static constexpr int NCH = (MB + MBC - 1) / MBC;
  static constexpr int NT = MBC * KS * 64;                  // operator entries per chunk
  static constexpr int TR = (NT + 255) / 256;               // per thread per chunk
  static constexpr int TRA = TR * NCH;                      // per thread, all chunks
  static constexpr int NQ = 64 * NS;
  static constexpr int QR = (NQ + 255) / 256;
  static constexpr int DR = (ND + 255) / 256;
};

// Flat index of n + q for operator entry (m, k) (active coefficients m, k);
// ND (a zero entry) for padding rows/columns.
template <int P>
__device__ __forceinline__ int op_index(int m, int k) {
  constexpr int NP = nact(P);
  if (m >= NP || k >= NP) return ncoef(2 * P);
  const int a = m + 1, b = k + 1;
  return midx(kMI.x[a] + kMI.x[b], kMI.y[a] + kMI.y[b], kMI.z[a] + kMI.z[b]);
}

template <typename T, int P>
__global__ void __launch_bounds__(256, (sizeof(T) == 4 && P <= 6) ? 2 : 1) k_m2l(const M2LTile* __restrict__ tiles, const int32_t* __restrict__ tile_order, int64_t ntiles,
                                             const int32_t* __restrict__ tile_tgt,
                                             const int32_t* __restrict__ step_delta,
                                             const int32_t* __restrict__ step_src, const T* __restrict__ Dtab,
                                             const T* __restrict__ Q, T* __restrict__ V, LevelOffsets lo, int nb,
                                             int TB, int TC) {
  using S = M2LShape<T, P>;
  constexpr int MB = S::MB, KS = S::KS, NS = S::NS, ND = S::ND, QST = S::QST;
  constexpr int MBC = S::MBC, NCH = S::NCH, NT = S::NT, TR = S::TR;
  __shared__ T sD[ND + 1];
  __shared__ T sT[NT];
  __shared__ T sQ[4 * KS * QST];

  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  // tiles are launched longest first (greedy balance over the compute units)
  if ((int64_t)blockIdx.x >= ntiles) return;
  const M2LTile tl = tiles[tile_order[blockIdx.x]];
  const T* Ql = Q + lo.qoff[tl.level];

  // this thread's operator entries (step independent): (chunk, r) -> index
  uint32_t myidx[(NCH * TR + 1) / 2];
#pragma unroll
  for (int i = 0; i < (NCH * TR + 1) / 2; i++) myidx[i] = 0;
#pragma unroll
  for (int ch = 0; ch < NCH; ch++) {
#pragma unroll
    for (int r = 0; r < TR; r++) {
      const int e = t + 256 * r;
      int v = ND;
      if (e < NT) {
        const int mbl = e / (KS * 64), rem = e % (KS * 64);
        const int ks = rem >> 6, l = rem & 63;
        const int mb = ch * MBC + mbl;
        if (mb < MB) v = op_index<P>(16 * mb + (l & 15), 4 * ks + (l >> 4));
      }
      const int q = ch * TR + r;
      myidx[q >> 1] |= (uint32_t)v << (16 * (q & 1));
    }
  }

  using AccT = typename Acc<T>::type;
  AccT acc[MB];
#pragma unroll
  for (int mb = 0; mb < MB; mb++) acc[mb] = AccT{0, 0, 0, 0};

  T rD[S::DR], rQ[S::QR];
  auto fetch = [&](int s) {
    const int64_t st = (int64_t)tl.step0 + s;
    const T* drow = Dtab + (int64_t)step_delta[st] * drow_stride(P);
#pragma unroll
    for (int r = 0; r < S::DR; r++) {
      const int e = t + 256 * r;
      rD[r] = (e < ND) ? drow[e] : (T)0;
    }
#pragma unroll
    for (int r = 0; r < S::QR; r++) {
      const int e = t + 256 * r;
      T v = (T)0;
      if (e < S::NQ) {
        const int j = e / NS, k = e % NS;
        const int tc = j / TB, b = tl.b0 + (j % TB);
        if (tc < TC && b < nb) {
          const int src = step_src[st * TC + tc];
          if (src >= 0) v = Ql[((int64_t)src * nb + b) * NS + k];
        }
      }
      rQ[r] = v;
    }
  };
  if (tl.nsteps > 0) fetch(0);
  for (int s = 0; s < tl.nsteps; s++) {
    // stage the step's derivative tensor and its Q columns (fragment order)
#pragma unroll
    for (int r = 0; r < S::DR; r++) {
      const int e = t + 256 * r;
      if (e < ND) sD[e] = rD[r];
    }
    if (t == 0) sD[ND] = (T)0;
#pragma unroll
    for (int r = 0; r < S::QR; r++) {
      const int e = t + 256 * r;
      if (e < S::NQ) {
        const int j = e / NS, k = e % NS;
        sQ[((j >> 4) * KS + (k >> 2)) * QST + (j & 15) + 16 * (k & 3)] = rQ[r];
      }
    }
    if (s + 1 < tl.nsteps) fetch(s + 1);  // next step's loads overlap this step's products
#pragma unroll
    for (int ch = 0; ch < NCH; ch++) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < TR; r++) {
        const int e = t + 256 * r;
        const int q = ch * TR + r;
        if (e < NT) sT[e] = sD[(myidx[q >> 1] >> (16 * (q & 1))) & 0xffffu];
      }
      __syncthreads();
#pragma unroll 7
      for (int ks = 0; ks < KS; ks++) {
        const T bq = sQ[(w * KS + ks) * QST + lane];
#pragma unroll
        for (int mbl = 0; mbl < MBC; mbl++) {
          const int mb = ch * MBC + mbl;
          if (mb < MB) acc[mb] = mfma16x16x4(sT[(mbl * KS + ks) * 64 + lane], bq, acc[mb]);
        }
      }
    }
    __syncthreads();
  }
  // write: lane holds rows 16 mb + acc_row(l/16, r) of column 16 w + l % 16
  const int col = 16 * w + (lane & 15), kq = lane >> 4;
  const int tc = col / TB, b = tl.b0 + (col % TB);
  if (tc < TC && b < nb) {
    const int tgt = tile_tgt[tl.tgt0 + tc];
    if (tgt >= 0) {
      T* out = V + lo.qoff[tl.level] + ((int64_t)tgt * nb + b) * NS;
#pragma unroll
      for (int mb = 0; mb < MB; mb++) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int m = 16 * mb + acc_row<T>(kq, r);
          if (m < NS) {
            T v = (T)0;
            if (m < S::NP) {
              const int f = m + 1;
              const int deg = kMI.x[f] + kMI.y[f] + kMI.z[f];
              v = (deg & 1) ? -acc[mb][r] : acc[mb][r];
            }
            out[m] = v;
          }
        }
      }
    }
  }
}

// Variant with independent wavefronts: one tile of 16 columns per wavefront,
// no block synchronisation.  Each lane keeps the derivative-tensor index of
// its operator entries (row 16 mb + l%16, column 4 ks + l/16) in registers, so
// every MFMA A operand is a single LDS gather from the step's 455-entry tensor.
// Used for orders up to 6 (the index registers grow as p^6).
template <typename T, int P>
__global__ void __launch_bounds__(256, 2) k_m2l_wave(const M2LTile* __restrict__ tiles,
                                                  const int32_t* __restrict__ tile_order, int64_t ntiles,
                                                  const int32_t* __restrict__ tile_tgt,
                                                  const int32_t* __restrict__ step_delta,
                                                  const int32_t* __restrict__ step_src, const T* __restrict__ Dtab,
                                                  const T* __restrict__ Q, T* __restrict__ V, LevelOffsets lo,
                                                  int nb, int TB, int TC) {
  constexpr int NP = nact(P), NS = nstride(P), MB = (NP + 15) / 16, KS = NS / 4, ND = ncoef(2 * P);
  constexpr int QST = 65;
  constexpr int NQ = 16 * NS;
  constexpr int DR = (ND + 63) / 64, QR = (NQ + 63) / 64;
  constexpr int NI = MB * KS;
  __shared__ T sD[4][ND + 1];
  __shared__ T sQ[4][KS * QST];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t slot = (int64_t)blockIdx.x * 4 + w;
  // operator index of (ks, mb, lane), read back as 64 consecutive u16 per wave
  __shared__ uint16_t sIdx[NI * 64];
  for (int e = threadIdx.x; e < NI * 64; e += 256) {
    const int l = e & 63, i = e >> 6;
    const int ks = i / MB, mb = i % MB;
    sIdx[e] = (uint16_t)op_index<P>(16 * mb + (l & 15), 4 * ks + (l >> 4));
  }
  __syncthreads();
  if (slot >= ntiles) return;
  const M2LTile tl = tiles[tile_order[slot]];
  const T* Ql = Q + lo.qoff[tl.level];
  using AccT = typename Acc<T>::type;
  AccT acc[MB];
#pragma unroll
  for (int mb = 0; mb < MB; mb++) acc[mb] = AccT{0, 0, 0, 0};
  T rD[DR], rQ[QR];
  auto fetch = [&](int s) {
    const int64_t st = (int64_t)tl.step0 + s;
    const T* drow = Dtab + (int64_t)step_delta[st] * drow_stride(P);
#pragma unroll
    for (int r = 0; r < DR; r++) {
      const int e = lane + 64 * r;
      rD[r] = (e < ND) ? drow[e] : (T)0;
    }
#pragma unroll
    for (int r = 0; r < QR; r++) {
      const int e = lane + 64 * r;
      T v = (T)0;
      if (e < NQ) {
        const int j = e / NS, k = e % NS;
        const int tc = j / TB, b = tl.b0 + (j % TB);
        if (tc < TC && b < nb) {
          const int src = step_src[st * TC + tc];
          if (src >= 0) v = Ql[((int64_t)src * nb + b) * NS + k];
        }
      }
      rQ[r] = v;
    }
  };
  if (tl.nsteps > 0) fetch(0);
  for (int s = 0; s < tl.nsteps; s++) {
#pragma unroll
    for (int r = 0; r < DR; r++) {
      const int e = lane + 64 * r;
      if (e < ND) sD[w][e] = rD[r];
    }
    if (lane == 0) sD[w][ND] = (T)0;
#pragma unroll
    for (int r = 0; r < QR; r++) {
      const int e = lane + 64 * r;
      if (e < NQ) {
        const int j = e / NS, k = e % NS;
        sQ[w][(k >> 2) * QST + j + 16 * (k & 3)] = rQ[r];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (s + 1 < tl.nsteps) fetch(s + 1);
#pragma unroll 3
    for (int ks = 0; ks < KS; ks++) {
      const T bq = sQ[w][ks * QST + lane];
#pragma unroll
      for (int mb = 0; mb < MB; mb++) {
        const int ix = sIdx[(ks * MB + mb) * 64 + lane];
        acc[mb] = mfma16x16x4(sD[w][ix], bq, acc[mb]);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  const int col = lane & 15, kq = lane >> 4;
  const int tc = col / TB, b = tl.b0 + (col % TB);
  if (tc < TC && b < nb) {
    const int tgt = tile_tgt[tl.tgt0 + tc];
    if (tgt >= 0) {
      T* out = V + lo.qoff[tl.level] + ((int64_t)tgt * nb + b) * NS;
#pragma unroll
      for (int mb = 0; mb < MB; mb++) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int m = 16 * mb + acc_row<T>(kq, r);
          if (m < NS) {
            T v = (T)0;
            if (m < NP) {
              const int f = m + 1;
              const int deg = kMI.x[f] + kMI.y[f] + kMI.z[f];
              v = (deg & 1) ? -acc[mb][r] : acc[mb][r];
            }
            out[m] = v;
          }
        }
      }
    }
  }
}

// Wide variant (FP32; orders <= 6, <= 8 in the traceless form): a block of four wavefronts owns a tile of
// 4 x 16 CB columns (16 CB per wavefront); each wavefront keeps MB x CB accumulator blocks, so every
// operator fragment it reads from LDS feeds CB matrix products.  The contraction
// index is permuted so lane group kq = lane / 16 holds k = kq KS + ks: a lane's
// B fragments for one column are then KS consecutive words of Q, loaded
// straight from memory into registers one step ahead.  The operator of the next
// step is gathered from the derivative tensor in memory straight into the other
// half of a double-buffered LDS array (global-to-LDS loads, no registers) while
// the current step's products run, so each step needs a single block barrier
// and two blocks fit on a compute unit.
// Zeros read by empty columns: selecting an address instead of a loaded value
// keeps the loads free of consumers until the products that need them.
// (128 doubles: zero words for either element type)
__device__ const double g_zero_row[128] = {};

// four consecutive expansion or operator entries: one 16-byte (FP32) or two
// 16-byte (FP64) accesses
template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  typedef f32x4 type;
};
template <>
struct Vec4<double> {
  typedef f64x4 type;
};


// Operator layout of the wide kernels: slot e of row block mb holds, for
// steps 4 k4 .. 4 k4 + 3 of lane l, the float4 at k4 * 256 + 4 l (so a lane
// reads four steps' fragments at once); the KT steps past the last full
// group follow as one word per lane each.
// Rows past the last full block of 16 (RV of them, when there are at most 8
// and at least one full block) are not padded to a matrix-core block: they
// are summed on the vector units, and follow the matrix fragments as four
// runs of KSTR words, one per lane group kq, each holding T[16 MB + j][kq KS +
// ks] at ks RV + j (read as broadcast float4s; KSTR is an odd number of
// float4s so the four groups sit in different banks).
// Row length padded to a multiple of 256 words (whole 16-byte loads of one
// wavefront).
// Traceless form.  D is harmonic (sum_a D_{k+2e_a} = 0), so in the M2L sum
// every moment with q_z >= 2 can be moved onto q - 2e_z + 2e_x and
// q - 2e_z + 2e_y with a minus sign (highest q_z first) without changing any
// V_n, and the sum then runs over the q_z <= 1 components only, 2l + 1 per
// degree.  V is harmonic too, so only its n_z <= 1 components need the
// product; the others follow from V_{m+2e_z} = -V_{m+2e_x} - V_{m+2e_y}
// (lowest n_z first).  At p = 6 the operator shrinks from 83 x 84 to 48 x 48.

// Reduced index r -> full index f (expansion position f - 1): the f with
// f_z <= 1 in increasing order.  The multi-indices are graded by degree, so
// the list for order p is a prefix of this one for every p <= 8.
struct RedFull {
  uint8_t full[nred(8)];
  constexpr RedFull() : full{} {
    MultiIndexTable<8> mi;
    int r = 0;
    for (int f = 1; f < ncoef(8); f++)
      if (mi.z[f] <= 1) full[r++] = (uint8_t)f;
  }
};
__device__ constexpr RedFull kRedFull{};

// Moves of the fold, highest z first: the moment at src goes, negated, onto
// d1 (two more in x, two less in z) and d2 (two more in y).
template <int P>
struct FoldTable {
  static constexpr int NF = nact(P) - nred(P) > 0 ? nact(P) - nred(P) : 1;
  int src[NF], d1[NF], d2[NF];
  constexpr FoldTable() : src{}, d1{}, d2{} {
    MultiIndexTable<P> mi;
    int t = 0;
    for (int z = P; z >= 2; z--)
      for (int f = 1; f < ncoef(P); f++)
        if (mi.z[f] == z) {
          src[t] = f;
          d1[t] = midx(mi.x[f] + 2, mi.y[f], z - 2);
          d2[t] = midx(mi.x[f], mi.y[f] + 2, z - 2);
          t++;
        }
  }
};

// Folded moments Qr[row][nred_stride(P)] from the full moments (one thread per
// expansion row): the rows of levels 0 and 1 after M2M wrote the deeper levels'
// folded rows, or every row.
template <typename T, int P>
__global__ void k_fold_moments(int64_t rows, const T* __restrict__ Q, T* __restrict__ Qr) {
  using V4 = typename Vec4<T>::type;
  constexpr int NSF = nstride(P), NR = nred(P), NRS = nred_stride(P), NF = nact(P) - nred(P);
  constexpr FoldTable<P> F{};
  constexpr RedFull R{};
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  T q[NSF];
  const V4* in = reinterpret_cast<const V4*>(Q + r * NSF);
#pragma unroll
  for (int i = 0; i < NSF / 4; i++) {
    const V4 v = in[i];
    q[4 * i] = v[0];
    q[4 * i + 1] = v[1];
    q[4 * i + 2] = v[2];
    q[4 * i + 3] = v[3];
  }
#pragma unroll
  for (int i = 0; i < NF; i++) {
    const T v = q[F.src[i] - 1];
    q[F.d1[i] - 1] -= v;
    q[F.d2[i] - 1] -= v;
  }
  V4* out = reinterpret_cast<V4*>(Qr + r * NRS);
#pragma unroll
  for (int i = 0; i < NRS / 4; i++) {
    V4 v;
#pragma unroll
    for (int u = 0; u < 4; u++) v[u] = 4 * i + u < NR ? q[R.full[4 * i + u] - 1] : (T)0;
    out[i] = v;
  }
}

// The n_z >= 2 components of local expansions whose n_z <= 1 components the
// traceless M2L wrote (lowest z first); padding positions set to zero.  Runs
// on the rows of levels 0 and 1 (the first parents of L2L); L2L forms the same
// components of every deeper level.
template <typename T, int P>
__global__ void k_fill_locals(int64_t rows, T* __restrict__ V) {
  using V4 = typename Vec4<T>::type;
  constexpr int NSF = nstride(P), NA = nact(P), NF = nact(P) - nred(P);
  constexpr FoldTable<P> F{};
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  T v[NSF];
  V4* row = reinterpret_cast<V4*>(V + r * NSF);
#pragma unroll
  for (int i = 0; i < NSF / 4; i++) {
    const V4 a = row[i];
    v[4 * i] = a[0];
    v[4 * i + 1] = a[1];
    v[4 * i + 2] = a[2];
    v[4 * i + 3] = a[3];
  }
#pragma unroll
  for (int i = NF - 1; i >= 0; i--) v[F.src[i] - 1] = -v[F.d1[i] - 1] - v[F.d2[i] - 1];
#pragma unroll
  for (int i = NA; i < NSF; i++) v[i] = (T)0;
#pragma unroll
  for (int i = 0; i < NSF / 4; i++) row[i] = V4{v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]};
}

template <int P, bool RED = false>
struct WideOp {
  static constexpr int NP = RED ? nred(P) : nact(P), NS = RED ? nred_stride(P) : nstride(P), KS = NS / 4,
                       ND = ncoef(2 * P);
  static constexpr int MF = NP / 16, RF = NP % 16;
  static constexpr bool VROWS = MF >= 1 && RF > 0 && RF <= 8;
  static constexpr int MB = VROWS ? MF : (NP + 15) / 16;  // matrix-core row blocks
  static constexpr int RV = VROWS ? RF : 0;               // rows on the vector units
  static constexpr int K4 = KS / 4, KT = KS % 4;
  static constexpr int KSTR0 = (RV * KS + 3) / 4 * 4;
  static constexpr int KSTR = (KSTR0 / 4) % 2 == 0 && RV > 0 ? KSTR0 + 4 : KSTR0;
  static constexpr int NEM = MB * KS * 64;               // matrix-core operator entries
  static constexpr int NE = NEM + 4 * KSTR;              // all operator entries
  static constexpr int NEP = (NE + 255) / 256 * 256;     // padded row length
};

// operator entry (row m, column k) of the wide layout: the full form's
// op_index, or in the traceless form D_{n+q} over the reduced rows and columns
template <int P, bool RED>
__device__ __forceinline__ int wide_op_index(int m, int k) {
  if constexpr (RED) {
    if (m >= nred(P) || k >= nred(P)) return ncoef(2 * P);
    const int a = kRedFull.full[m], b = kRedFull.full[k];
    return midx(kMI.x[a] + kMI.x[b], kMI.y[a] + kMI.y[b], kMI.z[a] + kMI.z[b]);
  } else {
    return op_index<P>(m, k);
  }
}

// derivative-tensor index of slot e (ND, the row's trailing zero, for padding)
template <int P, bool RED = false>
__device__ __forceinline__ int wide_slot_dindex(int e) {
  using W = WideOp<P, RED>;
  if (e >= W::NE) return W::ND;
  if constexpr (W::RV > 0) {  // the vector-unit rows (none when every row is in a matrix-core block)
    if (e >= W::NEM) {
      const int kq = (e - W::NEM) / W::KSTR, r = (e - W::NEM) % W::KSTR;
      if (r >= W::RV * W::KS) return W::ND;
      return wide_op_index<P, RED>(16 * W::MB + r % W::RV, kq * W::KS + r / W::RV);
    }
  }
  const int mb = e / (W::KS * 64), r0 = e % (W::KS * 64);
  int ks, l;
  if (r0 < W::K4 * 256) {
    ks = 4 * (r0 / 256) + (r0 & 3);
    l = (r0 % 256) >> 2;
  } else {
    ks = 4 * W::K4 + (r0 - W::K4 * 256) / 64;
    l = r0 & 63;
  }
  return wide_op_index<P, RED>(16 * mb + (l & 15), (l >> 4) * W::KS + ks);
}

// Every derivative-table row expanded into that layout (in the plan's
// precision), once per table: a step's operator is then one contiguous block
// of memory.
template <typename T, int P, bool RED>
__global__ void k_expand_ops(int64_t nrows, const T* __restrict__ Df, T* __restrict__ Dx) {
  using W = WideOp<P, RED>;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * W::NEP) return;
  const int64_t r = t / W::NEP;
  const int e = (int)(t % W::NEP);
  Dx[t] = Df[r * drow_stride(P) + wide_slot_dindex<P, RED>(e)];
}

template <typename T, int P, bool RED>
static void expand_ops_red(Plan& P_, const T* D, hipStream_t st) {
  using W = WideOp<P, RED>;
  T* Dx = reinterpret_cast<T*>(P_.Dx.ensure(sizeof(T) * (size_t)P_.nrows * W::NEP));
  const int64_t nt = P_.nrows * W::NEP;
  k_expand_ops<T, P, RED><<<ceil_div(nt, 256), 256, 0, st>>>(P_.nrows, D, Dx);
  CCFMM_HIP(hipGetLastError());
}

// FP64 plans use the wide kernels in the traceless form only
template <int P>
static void expand_ops_impl(Plan& P_, hipStream_t st) {
  if (P_.precision == CCFMM_PREC_FP64) {
    if (P_.prm.m2l_traceless) expand_ops_red<double, P, true>(P_, P_.Dd.as<double>(), st);
  } else if (P_.prm.m2l_traceless) {
    expand_ops_red<float, P, true>(P_, P_.Df.as<float>(), st);
  } else {
    if constexpr (P <= 6) expand_ops_red<float, P, false>(P_, P_.Df.as<float>(), st);
  }
}

void build_wide_ops(Plan& P, hipStream_t st) {
  switch (P.p) {
    case 1: expand_ops_impl<1>(P, st); break;
    case 2: expand_ops_impl<2>(P, st); break;
    case 3: expand_ops_impl<3>(P, st); break;
    case 4: expand_ops_impl<4>(P, st); break;
    case 5: expand_ops_impl<5>(P, st); break;
    case 6: expand_ops_impl<6>(P, st); break;
    case 7: expand_ops_impl<7>(P, st); break;
    case 8: expand_ops_impl<8>(P, st); break;
    default: break;
  }
}

// RED: the traceless form (Q holds the folded moments, nred_stride(P) per
// row; only the n_z <= 1 rows of V are written: k_fill_locals completes levels
// 0 and 1, L2L the deeper levels).
// Share of a full-order M2L tile's work that a tile of smallest cells of
// order q takes in the wide traceless kernels: the matrix-core row blocks its
// rows need (a tile needing the vector-unit rows takes the full form).
double m2l_row_share(const Plan& P, int q) {
  const bool wide = P.m2l_variant == kM2LWide4 || P.m2l_variant == kM2LWide2 || P.m2l_variant == kM2LWide1;
  if (!wide || P.prm.m2l_traceless == 0 || q >= P.p) return 1.0;
  const int np = nred(P.p), mf = np / 16, rf = np % 16;
  const int mb = (mf >= 1 && rf > 0 && rf <= 8) ? mf : (np + 15) / 16;
  const int rows = nred(q);
  if (rows > 16 * mb) return 1.0;
  return (double)((rows + 15) / 16) / (double)mb;
}

// f(std::integral_constant<int, k>) for the k = mbu in 1..MB (uniform per block)
template <int MB, int K = 1, typename F>
__device__ __forceinline__ void with_row_blocks(int mbu, F& f) {
  if constexpr (K >= MB) {
    f(std::integral_constant<int, MB>{});
  } else {
    if (mbu <= K)
      f(std::integral_constant<int, K>{});
    else
      with_row_blocks<MB, K + 1>(mbu, f);
  }
}

// two blocks per CU where the double-buffered operator leaves room for them
// (FP64 at order 8 holds 100 KB of LDS: one)
template <typename T, int P, int CB, bool RED>
__global__ void __launch_bounds__(256, (CB <= 2 && !(sizeof(T) == 8 && P >= 8)) ? 2 : 1) k_m2l_wide(const M2LTile* __restrict__ tiles,
                                                   const int32_t* __restrict__ tile_order, int64_t ntiles,
                                                   const int32_t* __restrict__ tile_tgt,
                                                   const int32_t* __restrict__ step_delta,
                                                   const int32_t* __restrict__ step_src,
                                                   const T* __restrict__ Dop, const T* __restrict__ Q,
                                                   T* __restrict__ V, LevelOffsets lo, int nb, int TB, int TC) {
  using W = WideOp<P, RED>;
  using V4 = typename Vec4<T>::type;
  using AccT = typename Acc<T>::type;
  constexpr int NS = W::NS, KS = W::KS, MB = W::MB, NP = W::NP, RV = W::RV;
  constexpr int NSV = nstride(P);  // row stride of V (and of Q in the full form)
  constexpr int K4 = W::K4, KT = W::KT;  // full groups of 4 steps, steps left over
  constexpr int NEP = W::NEP;             // operator words per step (padded)
  __shared__ __attribute__((aligned(32))) T sT[2][NEP];
  constexpr int kOpBytes = NEP * (int)sizeof(T);  // a multiple of 1024 (rows padded to 256 entries)
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  // tiles are launched longest first (greedy balance over the compute units)
  if ((int64_t)blockIdx.x >= ntiles) return;
  const M2LTile tl = tiles[tile_order[blockIdx.x]];
  const T* Ql = Q + (RED ? lo.qoff[tl.level] / NSV * NS : lo.qoff[tl.level]);
  const int nsteps = tl.nsteps;

  // this lane's columns: 16 CB w + 16 cb + lane % 16, fragment rows kq KS .. kq KS + KS - 1
  const int kq = lane >> 4;
  int ctc[CB], cb_b[CB];
#pragma unroll
  for (int cb = 0; cb < CB; cb++) {
    const int col = 16 * CB * w + 16 * cb + (lane & 15);
    ctc[cb] = col / TB;
    cb_b[cb] = tl.b0 + col % TB;
    if (!(ctc[cb] < TC && cb_b[cb] < nb)) ctc[cb] = -1;
  }
  // Loads are unconditional: an empty column reads g_zero_row through a
  // selected address, so no loaded value has a consumer before the products
  // that need it and the loads stay in flight meanwhile.
  auto load_src = [&](int s, int (&src)[CB]) {
    const int64_t st = (int64_t)tl.step0 + s;
#pragma unroll
    for (int cb = 0; cb < CB; cb++) src[cb] = step_src[st * TC + (ctc[cb] >= 0 ? ctc[cb] : 0)];
  };
  auto load_b = [&](const int (&src)[CB], T (&B)[CB][KS]) {
#pragma unroll
    for (int cb = 0; cb < CB; cb++) {
      const bool ok = ctc[cb] >= 0 && src[cb] >= 0;
      // both candidates in the global address space: a generic pointer would
      // make these flat loads, which the LDS wait counter also tracks, so
      // every wait for an operator fragment would wait for them too
      typedef const __attribute__((address_space(1))) T* gptr;
      const gptr q = ok ? (gptr)(Ql + ((int64_t)src[cb] * nb + cb_b[cb]) * NS + kq * KS) : (gptr)g_zero_row;
#pragma unroll
      for (int ks = 0; ks < KS; ks++) B[cb][ks] = q[ks];
    }
  };
  // the operator of step s (its expanded row, already in LDS order) goes from
  // memory straight into sT[buf] (no registers): 16-byte loads, lane l of
  // wavefront w covering bytes 4096 r + 1024 w + 16 l .. + 15
  // (the first nbytes of the row: the row blocks in use)
  auto load_op = [&](int s, int buf, int nbytes) {
    const char* orow = reinterpret_cast<const char*>(Dop + (int64_t)step_delta[tl.step0 + s] * NEP);
    char* dst = reinterpret_cast<char*>(&sT[buf][0]);
#pragma unroll
    for (int r = 0; r < (kOpBytes + 4095) / 4096; r++) {
      const int o = 4096 * r + 1024 * w;
      if (o < nbytes)  // uniform over the wavefront
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(orow + o + 16 * lane),
                                         (__attribute__((address_space(3))) void*)(dst + o), 16, 0, 0);
    }
  };
  // all of this wavefront's memory loads have landed (vmcnt = 0)
  auto wait_loads = [] { __builtin_amdgcn_s_waitcnt(0x0F70); };

  // The products for the first MBU row blocks (MBU = MB: all rows, the vector
  // rows included); tiles of smallest cells with a lower order of their own
  // need fewer rows, and write zeros past them (their L2P reads none of those).
  auto body = [&](auto mbu_c) {
  constexpr int MBU = decltype(mbu_c)::value;
  constexpr bool kAllRows = MBU == MB;
  constexpr int kOpUsed = kAllRows ? kOpBytes : (MBU * KS * 64 * (int)sizeof(T) + 1023) / 1024 * 1024;
  AccT acc[MB][CB];
#pragma unroll
  for (int mb = 0; mb < MB; mb++)
#pragma unroll
    for (int cb = 0; cb < CB; cb++) acc[mb][cb] = AccT{0, 0, 0, 0};
  // vector-unit rows: this lane's partial sums over its lane group's k range
  T pv[CB][RV > 0 ? RV : 1];
#pragma unroll
  for (int cb = 0; cb < CB; cb++)
#pragma unroll
    for (int j = 0; j < (RV > 0 ? RV : 1); j++) pv[cb][j] = (T)0;

  T B0[CB][KS], B1[CB][KS];
  int srcA[CB], srcB[CB];
  if (nsteps > 0) {
    load_op(0, 0, kOpUsed);
    load_src(0, srcA);
    load_b(srcA, B0);
    if (nsteps > 1) load_src(1, srcB);
  }
  wait_loads();
  __syncthreads();
  // one step: products on sT[cur] x Bc while the next operator and B arrive
  auto step = [&](int s, int cur, T (&Bc)[CB][KS], T (&Bn)[CB][KS], int (&srcN)[CB], int (&srcN2)[CB]) {
    const bool more = s + 1 < nsteps;
    if (more) {
      load_op(s + 1, cur ^ 1, kOpUsed);
      load_b(srcN, Bn);
      if (s + 2 < nsteps) load_src(s + 2, srcN2);
    }
    __builtin_amdgcn_sched_barrier(0);  // issue the loads before the products
    const T* T0 = sT[cur];
#pragma unroll
    for (int k4 = 0; k4 < K4; k4++) {
      V4 av[MBU];
#pragma unroll
      for (int mb = 0; mb < MBU; mb++)
        av[mb] = *reinterpret_cast<const V4*>(T0 + mb * KS * 64 + k4 * 256 + 4 * lane);
#pragma unroll
      for (int ku = 0; ku < 4; ku++)
#pragma unroll
        for (int mb = 0; mb < MBU; mb++)
#pragma unroll
          for (int cb = 0; cb < CB; cb++) acc[mb][cb] = mfma16x16x4(av[mb][ku], Bc[cb][4 * k4 + ku], acc[mb][cb]);
    }
#pragma unroll
    for (int t = 0; t < KT; t++) {
#pragma unroll
      for (int mb = 0; mb < MBU; mb++) {
        const T a = T0[mb * KS * 64 + K4 * 256 + t * 64 + lane];
#pragma unroll
        for (int cb = 0; cb < CB; cb++) acc[mb][cb] = mfma16x16x4(a, Bc[cb][4 * K4 + t], acc[mb][cb]);
      }
    }
    if constexpr (RV > 0 && kAllRows) {
      const T* Tv = T0 + W::NEM + kq * W::KSTR;
#pragma unroll
      for (int i = 0; i < W::KSTR / 4; i++) {
        const V4 tv = *reinterpret_cast<const V4*>(Tv + 4 * i);
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const int r = 4 * i + u;
          if (r < RV * KS) {
#pragma unroll
            for (int cb = 0; cb < CB; cb++) pv[cb][r % RV] = fma(tv[u], Bc[cb][r / RV], pv[cb][r % RV]);
          }
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    wait_loads();  // next operator in LDS, next B in registers
    __syncthreads();
  };
  for (int s = 0; s < nsteps; s += 2) {
    step(s, 0, B0, B1, srcB, srcA);
    if (s + 1 < nsteps) step(s + 1, 1, B1, B0, srcA, srcB);
  }
  // write: lane holds rows 16 mb + 4 kq + r of column 16 CB w + 16 cb + lane % 16
#pragma unroll
  for (int cb = 0; cb < CB; cb++) {
    if (ctc[cb] < 0) continue;
    const int tgt = tile_tgt[tl.tgt0 + ctc[cb]];
    if (tgt < 0) continue;
    T* out = V + lo.qoff[tl.level] + ((int64_t)tgt * nb + cb_b[cb]) * NSV;
#pragma unroll
    for (int mb = 0; mb < MB; mb++) {
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int m = 16 * mb + acc_row<T>(kq, r);
        if (m < NP) {
          const int f = RED ? (int)kRedFull.full[m] : m + 1;
          const int deg = kMI.x[f] + kMI.y[f] + kMI.z[f];
          const T v = mb < MBU ? acc[mb][cb][r] : (T)0;
          out[f - 1] = (deg & 1) ? -v : v;
        } else if (!RED && m < NS) {
          out[m] = (T)0;
        }
      }
    }
  }
  if constexpr (RV > 0) {
    // vector-unit rows: sum the four lane groups' partial sums; lane group kq
    // writes rows 16 MB + kq, + 4, ... (the stride's padding rows as zeros)
#pragma unroll
    for (int cb = 0; cb < CB; cb++) {
#pragma unroll
      for (int j = 0; j < RV; j++) {
        pv[cb][j] += __shfl_xor(pv[cb][j], 16);
        pv[cb][j] += __shfl_xor(pv[cb][j], 32);
      }
    }
#pragma unroll
    for (int cb = 0; cb < CB; cb++) {
      if (ctc[cb] < 0) continue;
      const int tgt = tile_tgt[tl.tgt0 + ctc[cb]];
      if (tgt < 0) continue;
      T* out = V + lo.qoff[tl.level] + ((int64_t)tgt * nb + cb_b[cb]) * NSV;
      // the traceless form writes the RV rows only (the fill writes the rest)
      constexpr int NW = RED ? RV : NS - 16 * MB;
#pragma unroll
      for (int j0 = 0; j0 < NW; j0 += 4) {
        const int j = j0 + kq;
        if (j < NW) {
          T v = (T)0;
          int f = 16 * MB + j + 1;
#pragma unroll
          for (int jj = 0; jj < RV; jj++)
            if (jj == j) {
              f = RED ? (int)kRedFull.full[16 * MB + jj] : 16 * MB + jj + 1;
              const int deg = kMI.x[f] + kMI.y[f] + kMI.z[f];
              const T pj = kAllRows ? pv[cb][jj] : (T)0;
              v = (deg & 1) ? -pj : pj;
            }
          out[f - 1] = v;
        }
      }
    }
  }
  };
  // row blocks in use: a tile needing rows past the matrix-core blocks (the
  // vector rows) or all of them takes the full form
  const int rows = tl.rows > 0 ? tl.rows : NP;
  const int mbu = rows > 16 * MB ? MB : (rows + 15) / 16;
  with_row_blocks<MB>(mbu, body);
}

template <typename T, int PP>
static void m2l_impl(Plan& P, int nb, hipStream_t st) {
  LevelOffsets lo{};
  for (int l = 0; l <= P.L; l++) lo.qoff[l] = P.lev[l]->qoff;
  const T* D = std::is_same<T, double>::value ? (const T*)P.Dd.p : (const T*)P.Df.p;
  P.v_folded = false;
  if (P.ntiles == 0) return;
  constexpr bool kFP64 = std::is_same<T, double>::value;
  if constexpr (PP <= 8) {
    const bool red = P.prm.m2l_traceless != 0;
    if ((P.tiles_variant == kM2LWide4 || P.tiles_variant == kM2LWide2 || P.tiles_variant == kM2LWide1) &&
        PP <= wide_max_order(red) && (red || !kFP64)) {
      const unsigned nblk = (unsigned)P.ntiles;
      const int64_t rows = P.qv_elems / nstride(PP);
      if (red) {
        // levels 0 and 1 folded here when M2M folded the deeper ones
        const int64_t ftop = P.q_folded ? P.lev[2]->qoff / nstride(PP) : rows;
        k_fold_moments<T, PP><<<ceil_div(ftop, 256), 256, 0, st>>>(ftop, P.Q.as<T>(), P.Qr.as<T>());
        CCFMM_HIP(hipGetLastError());
      }
#define CCFMM_WIDE(CB, RED)                                                                                          \
  k_m2l_wide<T, PP, CB, RED><<<nblk, 256, 0, st>>>(                                                                  \
      P.tiles.as<M2LTile>(), P.tile_order.as<int32_t>(), P.ntiles, P.tile_tgt.as<int32_t>(),                        \
      P.step_delta.as<int32_t>(), P.step_src.as<int32_t>(), P.Dx.as<T>(), RED ? P.Qr.as<T>() : P.Q.as<T>(),         \
      P.V.as<T>(), lo, nb, P.TB, P.TC)
      if (red) {
        if (P.tiles_variant == kM2LWide4)
          CCFMM_WIDE(4, true);
        else if (P.tiles_variant == kM2LWide2)
          CCFMM_WIDE(2, true);
        else
          CCFMM_WIDE(1, true);
      } else {
        if constexpr (PP <= 6 && !kFP64) {  // the full form's operator fits up to order 6
          if (P.tiles_variant == kM2LWide4)
            CCFMM_WIDE(4, false);
          else if (P.tiles_variant == kM2LWide2)
            CCFMM_WIDE(2, false);
          else
            CCFMM_WIDE(1, false);
        }
      }
#undef CCFMM_WIDE
      CCFMM_HIP(hipGetLastError());
      if (red) {
        // levels 0 and 1 completed here; L2L completes each deeper level as it
        // adds the parent's shifted expansion (one pass over those rows)
        // (the staged L2L only: the form beside the near field takes complete rows)
        const bool deep = shifts_staged(P) && P.L >= 2;
        const int64_t top = deep ? P.lev[2]->qoff / nstride(PP) : rows;
        k_fill_locals<T, PP><<<ceil_div(top, 256), 256, 0, st>>>(top, P.V.as<T>());
        CCFMM_HIP(hipGetLastError());
        P.v_folded = deep;
      }
      return;
    }
  }
  if (P.tiles_variant == kM2LWide4 || P.tiles_variant == kM2LWide2 || P.tiles_variant == kM2LWide1)
    fail(CCFMM_EINVAL, "wide M2L variants need order <= 8 in the traceless form (mixed precision: <= 6 in the "
                       "full form)");
  if (P.tiles_variant == kM2LWave) {
    if constexpr (PP <= 6) {
      k_m2l_wave<T, PP><<<ceil_div(P.ntiles, 4), 256, 0, st>>>(
          P.tiles.as<M2LTile>(), P.tile_order.as<int32_t>(), P.ntiles, P.tile_tgt.as<int32_t>(), P.step_delta.as<int32_t>(),
          P.step_src.as<int32_t>(), D, P.Q.as<T>(), P.V.as<T>(), lo, nb, P.TB, P.TC);
      CCFMM_HIP(hipGetLastError());
      return;
    }
    fail(CCFMM_EINVAL, "wavefront M2L variant supports orders up to 6");
  }
  k_m2l<T, PP><<<(unsigned)P.ntiles, 256, 0, st>>>(P.tiles.as<M2LTile>(), P.tile_order.as<int32_t>(), P.ntiles, P.tile_tgt.as<int32_t>(),
                                                   P.step_delta.as<int32_t>(), P.step_src.as<int32_t>(), D,
                                                   P.Q.as<T>(), P.V.as<T>(), lo, nb, P.TB, P.TC);
  CCFMM_HIP(hipGetLastError());
}

template <int PP>
static void m2l_d(Plan& P, int nb, hipStream_t st) {
  if (P.precision == CCFMM_PREC_FP64)
    m2l_impl<double, PP>(P, nb, st);
  else
    m2l_impl<float, PP>(P, nb, st);
}

void run_m2l(Plan& P, int nb, hipStream_t st) {
  switch (P.p) {
    case 1: m2l_d<1>(P, nb, st); break;
    case 2: m2l_d<2>(P, nb, st); break;
    case 3: m2l_d<3>(P, nb, st); break;
    case 4: m2l_d<4>(P, nb, st); break;
    case 5: m2l_d<5>(P, nb, st); break;
    case 6: m2l_d<6>(P, nb, st); break;
    case 7: m2l_d<7>(P, nb, st); break;
    case 8: m2l_d<8>(P, nb, st); break;
    default: fail(CCFMM_EINVAL, "order out of range");
  }
}

// ------------------------------------------------------------ MFMA self-test
__global__ void k_mfma_probe(const float* A, const float* B, float* Cf, const double* Ad, const double* Bd,
                             double* Cd) {
  const int lane = threadIdx.x;
  const int i = lane & 15, k = lane >> 4;
  f32x4 c = {0, 0, 0, 0};
  c = mfma16x16x4(A[i * 4 + k], B[k * 16 + i], c);
  f64x4 cd = {0, 0, 0, 0};
  cd = mfma16x16x4(Ad[i * 4 + k], Bd[k * 16 + i], cd);
  for (int r = 0; r < 4; r++) {
    Cf[acc_row<float>(k, r) * 16 + i] = c[r];
    Cd[acc_row<double>(k, r) * 16 + i] = cd[r];
  }
}

int selftest_mfma_impl(int device) {
  CCFMM_HIP(hipSetDevice(device));
  std::vector<float> A(64), B(64), C(256);
  std::vector<double> Ad(64), Bd(64), Cd(256);
  for (int t = 0; t < 64; t++) {
    A[t] = (float)((t * 7) % 11 - 5);
    B[t] = (float)((t * 5) % 13 - 6);
    Ad[t] = A[t] * 0.5;
    Bd[t] = B[t] * 0.25;
  }
  DevBuf dA, dB, dC, dAd, dBd, dCd;
  dA.ensure(256);
  dB.ensure(256);
  dC.ensure(1024);
  dAd.ensure(512);
  dBd.ensure(512);
  dCd.ensure(2048);
  CCFMM_HIP(hipMemcpy(dA.p, A.data(), 256, hipMemcpyHostToDevice));
  CCFMM_HIP(hipMemcpy(dB.p, B.data(), 256, hipMemcpyHostToDevice));
  CCFMM_HIP(hipMemcpy(dAd.p, Ad.data(), 512, hipMemcpyHostToDevice));
  CCFMM_HIP(hipMemcpy(dBd.p, Bd.data(), 512, hipMemcpyHostToDevice));
  k_mfma_probe<<<1, 64>>>(dA.as<float>(), dB.as<float>(), dC.as<float>(), dAd.as<double>(), dBd.as<double>(),
                          dCd.as<double>());
  CCFMM_HIP(hipGetLastError());
  CCFMM_HIP(hipDeviceSynchronize());
  CCFMM_HIP(hipMemcpy(C.data(), dC.p, 1024, hipMemcpyDeviceToHost));
  CCFMM_HIP(hipMemcpy(Cd.data(), dCd.p, 2048, hipMemcpyDeviceToHost));
  for (int i = 0; i < 16; i++)
    for (int j = 0; j < 16; j++) {
      double s = 0.0, sd = 0.0;
      for (int k = 0; k < 4; k++) {
        s += (double)A[i * 4 + k] * B[k * 16 + j];
        sd += Ad[i * 4 + k] * Bd[k * 16 + j];
      }
      if (s != (double)C[i * 16 + j] || sd != Cd[i * 16 + j])
        fail(CCFMM_EHIP, "MFMA layout mismatch at (" + std::to_string(i) + "," + std::to_string(j) +
                             "): f32 got " + std::to_string(C[i * 16 + j]) + " want " + std::to_string(s) +
                             ", f64 got " + std::to_string(Cd[i * 16 + j]) + " want " + std::to_string(sd));
    }
  return CCFMM_OK;
}

}  // namespace ccfmm
