// m2l.hip -- the M2L pass, Eq.(taylorcalc), on the matrix cores.
//
// For target cell C and source cell A at integer offset delta (same level),
//   Vt_n(C) += (-1)^|n| sum_q D_{n+q}(delta*g) Qt_q(A),   1 <= |n|, |q| <= p,
// in the level's scaled units.  The operator depends only on delta, so pairs
// are grouped by offset: a wavefront owns a tile of 16 columns (target cell,
// configuration) and walks the tile's offsets; every step is a dense
// [NP x NP] x [NP x 16] product on the MFMA units with the accumulators kept
// in registers for the whole walk, so each target column is written once.
// The [NP x NP] operator of a step is never stored: its entries are gathered
// from the step's derivative tensor (ncoef(2p) values in LDS) through a
// per-block index table idx(n+q) (the operator is Hankel-like in n+q).
#include "plan.hpp"

namespace ccfmm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16x16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16x16x4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename T>
struct Acc;
template <>
struct Acc<float> {
  using type = f32x4;
};
template <>
struct Acc<double> {
  using type = f64x4;
};
// Accumulator layout of the 16x16x4 MFMA (A row i / B column j at lane
// i|j + 16 k): lane l holds column l % 16; its item r is row 4 (l/16) + r for
// FP32 and row l/16 + 4 r for FP64 (checked by ccfmm_selftest_mfma).
template <typename T>
__device__ __forceinline__ int acc_row(int kq, int r);
template <>
__device__ __forceinline__ int acc_row<float>(int kq, int r) {
  return 4 * kq + r;
}
template <>
__device__ __forceinline__ int acc_row<double>(int kq, int r) {
  return kq + 4 * r;
}

__device__ __forceinline__ void lds_wave_sync() {
  // DS instructions of one wavefront execute in issue order; this keeps the
  // compiler from moving LDS accesses across the point and waits for them.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct LevelOffsets {
  int64_t qoff[kLMax + 1];
};

// Launch geometry: WPB wavefronts per block, one tile per wavefront.
template <typename T, int P, int WPB>
__global__ void __launch_bounds__(64 * WPB) k_m2l(const M2LTile* __restrict__ tiles, int64_t ntiles,
                                                 const int32_t* __restrict__ tile_tgt,
                                                 const int32_t* __restrict__ step_delta,
                                                 const int32_t* __restrict__ step_src, const T* __restrict__ Dtab,
                                                 const T* __restrict__ Q, T* __restrict__ V, LevelOffsets lo, int nb,
                                                 int TB, int TC) {
  constexpr int NP = nact(P);
  constexpr int NS = nstride(P);       // K extent, multiple of 4
  constexpr int MB = (NP + 15) / 16;   // 16-row blocks
  constexpr int KS = NS / 4;           // k steps
  constexpr int ND = ncoef(2 * P);     // derivative tensor entries
  constexpr int NQ = 16 * NS;          // Q tile entries
  constexpr int LD_ROUNDS = (ND + 63) / 64;
  constexpr int LQ_ROUNDS = (NQ + 63) / 64;

  __shared__ uint16_t sidx[MB * 16][NS];   // idx(n+q) (ND = zero entry for padding)
  __shared__ T sD[WPB][ND + 1];
  __shared__ T sQ[WPB][16][NS + 1];

  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // index table: row m <-> active coefficient m (flat m+1), column k likewise
  for (int e = threadIdx.x; e < MB * 16 * NS; e += 64 * WPB) {
    const int m = e / NS, k = e % NS;
    uint16_t v = (uint16_t)ND;
    if (m < NP && k < NP) {
      const int a = m + 1, b = k + 1;
      v = (uint16_t)midx(kMI.x[a] + kMI.x[b], kMI.y[a] + kMI.y[b], kMI.z[a] + kMI.z[b]);
    }
    sidx[m][k] = v;
  }
  __syncthreads();

  // blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous
  // range of tiles so neighbouring tiles (shared sources) share an L2
  const int nblk = gridDim.x;
  const int bid = blockIdx.x;
  const int lb = (nblk % 8 == 0) ? (bid & 7) * (nblk >> 3) + (bid >> 3) : bid;
  const int64_t tile = (int64_t)lb * WPB + w;
  if (tile >= ntiles) return;

  const M2LTile tl = tiles[tile];
  const T* Ql = Q + lo.qoff[tl.level];
  T* Vl = V + lo.qoff[tl.level];
  using AccT = typename Acc<T>::type;
  AccT acc[MB];
#pragma unroll
  for (int mb = 0; mb < MB; mb++) acc[mb] = AccT{0, 0, 0, 0};

  const int col = lane & 15, kq = lane >> 4;
  // columns handled by this lane when loading Q: entry e = lane + 64 r
  T rD[LD_ROUNDS], rQ[LQ_ROUNDS];
  auto fetch = [&](int s) {
    const int64_t st = (int64_t)tl.step0 + s;
    const T* drow = Dtab + (int64_t)step_delta[st] * ND;
#pragma unroll
    for (int r = 0; r < LD_ROUNDS; r++) {
      const int e = lane + 64 * r;
      rD[r] = (e < ND) ? drow[e] : (T)0;
    }
#pragma unroll
    for (int r = 0; r < LQ_ROUNDS; r++) {
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
    // stage this step's operator entries and Q columns
#pragma unroll
    for (int r = 0; r < LD_ROUNDS; r++) {
      const int e = lane + 64 * r;
      if (e < ND) sD[w][e] = rD[r];
    }
    if (lane == 0) sD[w][ND] = (T)0;
#pragma unroll
    for (int r = 0; r < LQ_ROUNDS; r++) {
      const int e = lane + 64 * r;
      if (e < NQ) sQ[w][e / NS][e % NS] = rQ[r];
    }
    lds_wave_sync();
    if (s + 1 < tl.nsteps) fetch(s + 1);  // overlap the next step's loads with this step's products
#pragma unroll
    for (int ks = 0; ks < KS; ks++) {
      const T bq = sQ[w][col][4 * ks + kq];
#pragma unroll
      for (int mb = 0; mb < MB; mb++) {
        const T a = sD[w][sidx[16 * mb + col][4 * ks + kq]];
        acc[mb] = mfma16x16x4(a, bq, acc[mb]);
      }
    }
    lds_wave_sync();
  }
  // write: lane holds rows 16 mb + acc_row(kq, r) of column col
  const int tc = col / TB, b = tl.b0 + (col % TB);
  if (tc < TC && b < nb) {
    const int tgt = tile_tgt[tl.tgt0 + tc];
    if (tgt >= 0) {
      T* out = Vl + ((int64_t)tgt * nb + b) * NS;
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

template <typename T, int PP>
static void m2l_impl(Plan& P, int nb, hipStream_t st) {
  constexpr int WPB = (PP >= 7 && sizeof(T) == 8) ? 2 : 4;
  LevelOffsets lo{};
  for (int l = 0; l <= P.L; l++) lo.qoff[l] = P.lev[l]->qoff;
  const T* D = std::is_same<T, double>::value ? (const T*)P.Dd.p : (const T*)P.Df.p;
  const int nblk = ceil_div(P.ntiles, WPB);
  if (nblk == 0) return;
  k_m2l<T, PP, WPB><<<nblk, 64 * WPB, 0, st>>>(P.tiles.as<M2LTile>(), P.ntiles, P.tile_tgt.as<int32_t>(),
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
    Cf[(4 * k + r) * 16 + i] = c[r];
    Cd[(k + 4 * r) * 16 + i] = cd[r];
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
