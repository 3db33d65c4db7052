// expansions.hip -- derivative tensors (Eqs. Dn, Dnr), multipole moments of
// dipoles (Eq. multipolemoments), moment shifts up the tree (Eq. momentshift)
// and Taylor shifts down the tree (Eq. taylorshift).
//
// All expansions are stored per level in scaled form (s = smallest side of the
// level's cells):  Qt_n = Q_n s^(1-|n|),  Vt_n = V_n s^(|n|+2),  and the dipole
// offsets inside a smallest cell are yt = (x - centre) / s.  In these units the
// numbers stay O(1) at every level, which the FP32 form relies on.
#include <algorithm>
#include <map>
#include <type_traits>

#include "plan.hpp"

namespace ccfmm {

// ------------------------------------------------------------ F table (host)
// D_k(r) = r^-(2|k|+1) sum_{|q|=|k|} F_k(q) r^q.  Going from k to k + e_v
// applies -d/dr_v, which maps the term r^q / r^(2|k|+1) onto
//   (2|k|+1-q_v) r^(q+e_v) - q_v r^(q-e_v+2e_u) - q_v r^(q-e_v+2e_w)
// over r^(2|k|+3).  Here every k is reached from k - e_v with v the last axis
// on which k is nonzero; the table is unique, so the choice is free.
struct FTableHost {
  std::vector<int32_t> ptr;   // ncoef(K) + 1
  std::vector<int32_t> q;     // flat index of q (same degree as k)
  std::vector<double> val;
};

static FTableHost make_ftable(int K) {
  const int NK = ncoef(K);
  std::vector<std::map<int, long double>> F(NK);
  F[0][0] = 1.0L;
  std::vector<int> mx(NK), my(NK), mz(NK);
  {
    int t = 0;
    for (int d = 0; d <= K; d++)
      for (int a = d; a >= 0; a--)
        for (int b = d - a; b >= 0; b--) {
          mx[t] = a;
          my[t] = b;
          mz[t] = d - a - b;
          t++;
        }
  }
  for (int t = 1; t < NK; t++) {
    int k[3] = {mx[t], my[t], mz[t]};
    int v = k[2] > 0 ? 2 : (k[1] > 0 ? 1 : 0);
    int n[3] = {k[0], k[1], k[2]};
    n[v]--;
    const int deg = n[0] + n[1] + n[2];
    const int src = midx(n[0], n[1], n[2]);
    for (const auto& kv : F[src]) {
      const int qi = kv.first;
      const long double f = kv.second;
      int q[3] = {mx[qi], my[qi], mz[qi]};
      {
        int r[3] = {q[0], q[1], q[2]};
        r[v]++;
        F[t][midx(r[0], r[1], r[2])] += (long double)(2 * deg + 1 - q[v]) * f;
      }
      if (q[v] > 0) {
        for (int u = 0; u < 3; u++) {
          if (u == v) continue;
          int r[3] = {q[0], q[1], q[2]};
          r[v]--;
          r[u] += 2;
          F[t][midx(r[0], r[1], r[2])] -= (long double)q[v] * f;
        }
      }
    }
  }
  FTableHost out;
  out.ptr.push_back(0);
  for (int t = 0; t < NK; t++) {
    for (const auto& kv : F[t]) {
      if (kv.second == 0.0L) continue;
      out.q.push_back(kv.first);
      out.val.push_back((double)kv.second);
    }
    out.ptr.push_back((int32_t)out.q.size());
  }
  return out;
}

// One thread per (dense offset id, k): D_k(c) in FP64, then an FP32 copy.
// Dense id d enumerates the offsets delta of the box [-w, w]^3 (source minus
// target cell); Eq.(taylorcalc) takes c = target minus source centre, i.e.
// c = -delta * g in the level's units.  The zero offset (never a far pair) is
// stored as zeros.
__global__ void k_dtensor(int64_t nbox, int w0, int w1, int w2, double g0, double g1, double g2, int K, int kmax,
                          const int32_t* __restrict__ fptr, const int32_t* __restrict__ fq,
                          const double* __restrict__ fval, int64_t row0, double* Dd, float* Df) {
  const int NK = ncoef(K), NR = NK + 1;  // row: NK entries, then a zero
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbox * NR) return;
  const int64_t d = t / NR;
  const int k = (int)(t % NR);
  const int nz = 2 * w2 + 1, ny = 2 * w1 + 1;
  const int dz = (int)(d % nz) - w2;
  const int dy = (int)((d / nz) % ny) - w1;
  const int dx = (int)(d / ((int64_t)nz * ny)) - w0;
  const double c[3] = {-dx * g0, -dy * g1, -dz * g2};
  const double r2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
  const int64_t o = (row0 + d) * NR + k;
  // |k| > kmax: total-degree truncation keeps only |n| + |q| = |n + q| <= p
  if (r2 == 0.0 || k == NK || kMI.x[k] + kMI.y[k] + kMI.z[k] > kmax) {
    Dd[o] = 0.0;
    Df[o] = 0.0f;
    return;
  }
  const int qx0 = kMI.x[k], qy0 = kMI.y[k], qz0 = kMI.z[k];
  const int deg = qx0 + qy0 + qz0;
  double s = 0.0;
  for (int e = fptr[k]; e < fptr[k + 1]; e++) {
    const int q = fq[e];
    double m = fval[e];
    for (int j = 0; j < kMI.x[q]; j++) m *= c[0];
    for (int j = 0; j < kMI.y[q]; j++) m *= c[1];
    for (int j = 0; j < kMI.z[q]; j++) m *= c[2];
    s += m;
  }
  // r^-(2 deg + 1)
  const double rinv = 1.0 / sqrt(r2);
  double rp = rinv;
  const double rinv2 = rinv * rinv;
  for (int j = 0; j < deg; j++) rp *= rinv2;
  const double v = s * rp;
  Dd[o] = v;
  Df[o] = (float)v;
}

// Derivative tensors for every offset of each level's box.  Levels with the
// same cell shape (g) and box share one table; the tables are kept across
// rebuilds as long as order, shapes and boxes do not change.
void build_dtensors(Plan& P, hipStream_t st) {
  const int K = 2 * P.p;
  std::vector<std::array<double, 6>> keys;
  std::vector<int64_t> key_row, key_nbox;
  std::vector<int> lev_key(P.L + 1, -1);
  int64_t rows = 0;
  for (int l = 1; l <= P.L; l++) {
    LevelData& D = *P.lev[l];
    const LevelGeom& lg = P.geo.lev[l];
    std::array<double, 6> k = {lg.g[0], lg.g[1], lg.g[2], (double)D.wfar[0], (double)D.wfar[1], (double)D.wfar[2]};
    int found = -1;
    for (size_t i = 0; i < keys.size(); i++)
      if (keys[i] == k) found = (int)i;
    if (found < 0) {
      found = (int)keys.size();
      keys.push_back(k);
      key_row.push_back(rows);
      key_nbox.push_back(D.nbox);
      rows += D.nbox;
    }
    lev_key[l] = found;
    D.drow0 = key_row[found];
  }
  P.lev[0]->drow0 = 0;
  if (P.dtab_p == P.p && P.dtab_keys == keys && P.Dd.p) return;  // unchanged: reuse
  static FTableHost ft[kPMax + 1];
  static bool have[kPMax + 1] = {false};
  if (!have[P.p]) {
    ft[P.p] = make_ftable(K);
    have[P.p] = true;
  }
  const FTableHost& F = ft[P.p];
  const size_t nb_ptr = sizeof(int32_t) * F.ptr.size(), nb_q = sizeof(int32_t) * F.q.size();
  const size_t nb_val = sizeof(double) * F.val.size();
  const size_t off_val = (nb_ptr + nb_q + 15) & ~size_t(15);
  char* buf = reinterpret_cast<char*>(P.scratch2.ensure(off_val + nb_val + 64));
  int32_t* dptr = reinterpret_cast<int32_t*>(buf);
  int32_t* dq = reinterpret_cast<int32_t*>(buf + nb_ptr);
  double* dval = reinterpret_cast<double*>(buf + off_val);
  CCFMM_HIP(hipMemcpyAsync(dptr, F.ptr.data(), nb_ptr, hipMemcpyHostToDevice, st));
  CCFMM_HIP(hipMemcpyAsync(dq, F.q.data(), nb_q, hipMemcpyHostToDevice, st));
  CCFMM_HIP(hipMemcpyAsync(dval, F.val.data(), nb_val, hipMemcpyHostToDevice, st));
  P.nrows = std::max<int64_t>(1, rows);
  const int NR = drow_stride(P.p);
  double* Dd = reinterpret_cast<double*>(P.Dd.ensure(sizeof(double) * P.nrows * NR));
  float* Df = reinterpret_cast<float*>(P.Df.ensure(sizeof(float) * P.nrows * NR));
  for (size_t i = 0; i < keys.size(); i++) {
    const auto& k = keys[i];
    const int64_t nt = key_nbox[i] * NR;
    k_dtensor<<<ceil_div(nt, 256), 256, 0, st>>>(key_nbox[i], (int)k[3], (int)k[4], (int)k[5], k[0], k[1], k[2], K,
                                                 P.prm.truncation == 1 ? P.p : K, dptr, dq, dval, key_row[i], Dd,
                                                 Df);
    CCFMM_HIP(hipGetLastError());
  }
  if (P.p <= wide_max_order(P.prm.m2l_traceless != 0) && (P.precision != CCFMM_PREC_FP64 || P.prm.m2l_traceless))
    build_wide_ops(P, st);
  CCFMM_HIP(hipStreamSynchronize(st));  // the host table copies above must finish before scratch2 is reused
  P.dtab_p = P.p;
  P.dtab_keys = keys;
}

// ------------------------------------------------------------ moments in tree order
template <typename T>
__global__ void k_permute_moments(const double* __restrict__ m, const int32_t* __restrict__ perm, int64_t n,
                                  int nb, T* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= n) return;
  const int64_t src = perm[i];
  const double* mi = m + ((int64_t)b * n + src) * 3;
  T* o = out + (int64_t)b * 3 * n;
  o[i] = (T)mi[0];
  o[n + i] = (T)mi[1];
  o[2 * n + i] = (T)mi[2];
}

// configuration-major copy [i][a][b] for the batched near field
template <typename T>
__global__ void k_permute_moments_t(const double* __restrict__ m, const int32_t* __restrict__ perm, int64_t n,
                                    int nb, T* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nb) return;
  const int64_t i = t / nb;
  const int b = (int)(t % nb);
  const double* mi = m + ((int64_t)b * n + perm[i]) * 3;
  T* o = out + i * 3 * nb + b;
  o[0] = (T)mi[0];
  o[nb] = (T)mi[1];
  o[2 * nb] = (T)mi[2];
}

// ------------------------------------------------------------ P2M
// One wavefront per (occupied smallest cell, group of up to CG
// configurations; CG = 1 for a single configuration, else kP2MConfigs).  Eq. (multipolemoments) in scaled units:
// Qt_n = sum_i sum_{a: n_a>0} m_ia yt^(n-e_a)/(n-e_a)!.  Lanes first tabulate
// yt^k/k! (|k| <= p-1) of kP2MChunk dipoles in LDS (once for the whole group:
// the monomials do not depend on the moments), then each lane sums whole
// coefficients over those dipoles for every configuration of the group.
constexpr int kP2MWaves = 4;
constexpr int kP2MChunk = 16;
constexpr int kP2MConfigs = 8;

template <typename T, int P, int CG>
__global__ void __launch_bounds__(64 * kP2MWaves) k_p2m(const int32_t* __restrict__ lstart,
                                                       const int32_t* __restrict__ lcount, int32_t nleaf,
                                                       const T* __restrict__ y, const T* __restrict__ msort,
                                                       int64_t n, int nb, T* __restrict__ Q) {
  constexpr int NM = ncoef(P - 1);  // monomials of degree <= p-1
  constexpr int NP = nact(P);
  constexpr int NS = nstride(P);
  constexpr int NR = (NP + 63) / 64;
  __shared__ T mono[kP2MWaves][kP2MChunk][NM + 1];
  __shared__ T mm[kP2MWaves][kP2MChunk][CG][3];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ngrp = (nb + CG - 1) / CG;
  const int64_t item = (int64_t)blockIdx.x * kP2MWaves + w;
  if (item >= (int64_t)nleaf * ngrp) return;
  const int leaf = (int)(item / ngrp), b0 = (int)(item % ngrp) * CG;
  const int nbg = min(CG, nb - b0);
  const int first = lstart[leaf], cnt = lcount[leaf];
  // source indices of coefficient n - e_a for this lane's coefficients (NM,
  // a slot kept zero, where the term is absent)
  int srcx[NR], srcy[NR], srcz[NR];
  T acc[CG][NR];
#pragma unroll
  for (int r = 0; r < NR; r++) {
    const int t = lane + 64 * r + 1;  // flat index, |n| >= 1
#pragma unroll
    for (int c = 0; c < CG; c++) acc[c][r] = (T)0;
    srcx[r] = srcy[r] = srcz[r] = NM;
    if (t <= NP) {
      const int x = kMI.x[t], yy = kMI.y[t], z = kMI.z[t];
      if (x > 0) srcx[r] = midx(x - 1, yy, z);
      if (yy > 0) srcy[r] = midx(x, yy - 1, z);
      if (z > 0) srcz[r] = midx(x, yy, z - 1);
    }
  }
  if (lane < kP2MChunk) mono[w][lane][NM] = (T)0;
  for (int base = 0; base < cnt; base += kP2MChunk) {
    const int nchunk = min(kP2MChunk, cnt - base);
    if (lane < nchunk) {
      const int64_t i = first + base + lane;
      const T yx = y[i], yy = y[n + i], yz = y[2 * n + i];
      T px[P], py[P], pz[P];
      px[0] = py[0] = pz[0] = (T)1;
#pragma unroll
      for (int j = 1; j < P; j++) {
        const T inv = (T)(1.0 / j);
        px[j] = px[j - 1] * yx * inv;
        py[j] = py[j - 1] * yy * inv;
        pz[j] = pz[j - 1] * yz * inv;
      }
#pragma unroll
      for (int t = 0; t < NM; t++) mono[w][lane][t] = px[kMI.x[t]] * py[kMI.y[t]] * pz[kMI.z[t]];
    }
    // the group's moments of these dipoles, one (dipole, configuration) per
    // lane; zeros past the group's last configuration, so the sums below run
    // over all CG without a test per configuration (those sums are not stored)
    for (int q = lane; q < nchunk * CG; q += 64) {
      const int j = q / CG, c = q % CG;
      const int64_t i = first + base + j;
      const bool ok = c < nbg;
      const T* mb = msort + (int64_t)(b0 + (ok ? c : 0)) * 3 * n;
      mm[w][j][c][0] = ok ? mb[i] : (T)0;
      mm[w][j][c][1] = ok ? mb[n + i] : (T)0;
      mm[w][j][c][2] = ok ? mb[2 * n + i] : (T)0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int j = 0; j < nchunk; j++) {
      // this lane's monomials of dipole j (zero where the term is absent)
      T vx[NR], vy[NR], vz[NR];
#pragma unroll
      for (int r = 0; r < NR; r++) {
        vx[r] = mono[w][j][srcx[r]];
        vy[r] = mono[w][j][srcy[r]];
        vz[r] = mono[w][j][srcz[r]];
      }
#pragma unroll
      for (int c = 0; c < CG; c++) {
        const T m0 = mm[w][j][c][0], m1 = mm[w][j][c][1], m2 = mm[w][j][c][2];
#pragma unroll
        for (int r = 0; r < NR; r++) {
          T s = acc[c][r];
          s += m0 * vx[r];
          s += m1 * vy[r];
          s += m2 * vz[r];
          acc[c][r] = s;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
#pragma unroll
  for (int c = 0; c < CG; c++) {
    if (c < nbg) {
      T* q = Q + ((int64_t)leaf * nb + b0 + c) * NS;
#pragma unroll
      for (int r = 0; r < NR; r++) {
        const int a = lane + 64 * r;
        if (a < NS) q[a] = (a < NP) ? acc[c][r] : (T)0;
      }
    }
  }
}

// ------------------------------------------------------------ M2M
// Eq.(momentshift) from level l+1 to l.  The two children sit at -/+ h_a/2 of
// the parent centre along the halved axis a only, so Q_n(P) sums Q_{n-k e_a}(C)
// over k; in scaled units the weight is gamma^k/k! rho^(|n|-k-1) with
// gamma = (child centre - parent centre)_a / s_l and rho = s_{l+1}/s_l.
// The weights of a level are tabulated on the host (ShiftW): w[k][d] =
// gamma^k/k! rho^(d-1) for the child at +gamma; the child at -gamma takes
// (-1)^k of it.
struct ShiftW {
  double w[kPMax + 1][kPMax + 1];
};

static ShiftW m2m_weights(double gam, double rho, int p) {
  ShiftW W{};
  double gk = 1.0;  // gamma^k / k!
  for (int k = 0; k <= p; k++) {
    for (int d = 1; d <= p; d++) {
      double w = gk;
      for (int j = 0; j < d - 1; j++) w *= rho;
      W.w[k][d] = w;
    }
    gk = gk * gam / (double)(k + 1);
  }
  return W;
}

// Multi-index (x, y, z) of coefficient f in the graded order of midx, at
// compile time: degree d, then s = y + z and z from f - ncoef(d - 1) =
// s (s + 1) / 2 + z.
constexpr int mi_deg(int f) {
  int d = 0;
  while (ncoef(d) <= f) d++;
  return d;
}
constexpr int mi_s(int f) {
  const int r = f - ncoef(mi_deg(f) - 1);
  int s = 0;
  while ((s + 1) * (s + 2) / 2 <= r) s++;
  return s;
}
constexpr int mi_z(int f) { return f - ncoef(mi_deg(f) - 1) - mi_s(f) * (mi_s(f) + 1) / 2; }
constexpr int mi_x(int f) { return mi_deg(f) - mi_s(f); }
constexpr int mi_y(int f) { return mi_s(f) - mi_z(f); }
// i-th f with f_z <= 1 (the traceless rows' order)
constexpr int red_full(int i) {
  int f = 1;
  for (;; f++)
    if (mi_z(f) <= 1 && i-- == 0) return f;
}
constexpr int binom(int n, int k) {
  int r = 1;
  for (int i = 0; i < k; i++) r = r * (n - i) / (i + 1);
  return r;
}

template <int A, int B, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (A < B) {
    f(std::integral_constant<int, A>{});
    static_for<A + 1, B>(f);
  }
}

typedef float shift_f4 __attribute__((ext_vector_type(4)));
typedef double shift_d4 __attribute__((ext_vector_type(4)));
template <typename T>
using RowVec4 = typename std::conditional<std::is_same<T, float>::value, shift_f4, shift_d4>::type;

// Expansion rows per M2M and L2L block: two rows of LDS per row (the two
// children, or parent and child), 43.5 KB at order 6 in either precision
constexpr int kShiftThreads = 256;
template <typename T>
constexpr int shift_rows() {
  return sizeof(T) == 4 ? 64 : 32;
}

// The two child rows of every parent row are read with coalesced vector loads
// into LDS (rows padded to an odd stride); each thread forms one share of one
// parent row's coefficients with compile-time indices, and the rows go back
// through LDS with coalesced stores.
// FOLD: the children's folded (traceless-form) rows, which the wide M2L
// kernels read, are written from the same LDS rows.  Moving each moment with
// q_z >= 2 onto q - 2e_z + 2e_x and q - 2e_z + 2e_y with a minus sign, highest
// q_z first, adds (-1)^k C(k, j) Q(x - 2j, y - 2(k - j), e + 2k) onto the
// position (x, y, e), e <= 1 (the transpose of the local rows' completion).
template <typename T, int P, int AX, int C0, int C1>
__device__ __forceinline__ void m2m_coefs(const T* __restrict__ c0r, const T* __restrict__ c1r, const ShiftW& W,
                                          T* res) {
  static_for<C0, C1>([&](auto ac) {
    constexpr int a = decltype(ac)::value;
    constexpr int f = a + 1, x = mi_x(f), y = mi_y(f), z = mi_z(f), deg = x + y + z;
    constexpr int na = AX == 0 ? x : AX == 1 ? y : z;
    double s = 0.0;
    static_for<0, na + 1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      if constexpr (deg - k >= 1) {  // (Q_0 = 0: no monopole term)
        constexpr int src = midx(x - (AX == 0 ? k : 0), y - (AX == 1 ? k : 0), z - (AX == 2 ? k : 0)) - 1;
        const double c1 = (double)c1r[src], c0 = (double)c0r[src];  // the child at +gamma, at -gamma
        s = fma(W.w[k][deg - k], (k & 1) ? c1 - c0 : c1 + c0, s);
      }
    });
    res[a - C0] = (T)s;
  });
}

template <typename T, int P, int R0, int R1>
__device__ __forceinline__ void fold_coefs(const T* __restrict__ q, T* res) {
  static_for<R0, R1>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int f = red_full(i), x = mi_x(f), y = mi_y(f), e = mi_z(f);
    double s = (double)q[f - 1];
    static_for<1, (x + y) / 2 + 1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      static_for<0, k + 1>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if constexpr (x - 2 * j >= 0 && y - 2 * (k - j) >= 0) {
          constexpr int src = midx(x - 2 * j, y - 2 * (k - j), e + 2 * k) - 1;
          constexpr double cf = (k & 1) ? -(double)binom(k, j) : (double)binom(k, j);
          s = fma(cf, (double)q[src], s);
        }
      });
    });
    res[i - R0] = (T)s;
  });
}

template <typename T, int P, int AX, bool FOLD>
__global__ void __launch_bounds__(kShiftThreads) k_m2m(int64_t nitems, const int32_t* __restrict__ child, ShiftW W,
                                                      int nb, const T* __restrict__ Qc, T* __restrict__ Qp,
                                                      T* __restrict__ Qrc) {
  using V4 = RowVec4<T>;
  constexpr int NP = nact(P), NS = nstride(P), NQ = NS / 4, LS = NS + 1;
  constexpr int NR = nred(P), NRS = nred_stride(P), NRQ = NRS / 4, LR = NRS + 1;
  constexpr int R = shift_rows<T>();
  constexpr int CH = kShiftThreads / R;     // shares of a row
  constexpr int CW = (NP + CH - 1) / CH;    // parent coefficients per share
  constexpr int CWR = (NR + CH - 1) / CH;   // folded child coefficients per share
  constexpr int QU = (2 * R * NQ + kShiftThreads - 1) / kShiftThreads;
  __shared__ T sc[2 * R * LS];  // child rows 2 r + e of parent row r
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * R;
  const int nr = (int)(nitems - i0 < R ? nitems - i0 : R);
  // parent row i0 + r is (cell c0 + (b0 + r) / nb, configuration (b0 + r) % nb)
  const int64_t c0 = i0 / nb;
  const int b0 = (int)(i0 - c0 * nb);
  V4 cv[QU];
#pragma unroll
  for (int u = 0; u < QU; u++) {
    const int q = tid + u * kShiftThreads;
    if (q < 2 * nr * NQ) {
      const int row2 = q / NQ, t = b0 + (row2 >> 1), dc = t / nb;
      const int32_t ch = child[2 * (c0 + dc) + (row2 & 1)];
      cv[u] = ch >= 0 ? reinterpret_cast<const V4*>(Qc + ((int64_t)ch * nb + (t - dc * nb)) * NS)[q % NQ]
                      : V4{(T)0, (T)0, (T)0, (T)0};  // an absent child reads as a zero row
    }
  }
#pragma unroll
  for (int u = 0; u < QU; u++) {
    const int q = tid + u * kShiftThreads;
    if (q < 2 * nr * NQ) {
      T* d = sc + (q / NQ) * LS + 4 * (q % NQ);
#pragma unroll
      for (int e = 0; e < 4; e++) d[e] = cv[u][e];
    }
  }
  __syncthreads();
  const int r = tid % R, share = tid / R;
  T res[CW];
  T fr[2][CWR];
  if (r < nr) {
    const T* c0r = sc + (2 * r) * LS;
    const T* c1r = sc + (2 * r + 1) * LS;
    static_for<0, CH>([&](auto hc) {
      constexpr int h = decltype(hc)::value;
      if (share == h) {
        m2m_coefs<T, P, AX, h * CW, (h + 1) * CW < NP ? (h + 1) * CW : NP>(c0r, c1r, W, res);
        if constexpr (FOLD) {
          constexpr int F0 = h * CWR, F1 = (h + 1) * CWR < NR ? (h + 1) * CWR : NR;
          fold_coefs<T, P, F0, F1>(c0r, fr[0]);
          fold_coefs<T, P, F0, F1>(c1r, fr[1]);
        }
      }
    });
  }
  __syncthreads();
  if constexpr (FOLD) {
    // the children's folded rows, stride LR in LDS
    if (r < nr) {
#pragma unroll
      for (int e = 0; e < 2; e++) {
#pragma unroll
        for (int i = 0; i < CWR; i++) {
          const int a = share * CWR + i;
          if (a < NR) sc[(2 * r + e) * LR + a] = fr[e][i];
        }
        if (share == 0)
          for (int a = NR; a < NRS; a++) sc[(2 * r + e) * LR + a] = (T)0;
      }
    }
    __syncthreads();
    for (int q = tid; q < 2 * nr * NRQ; q += kShiftThreads) {
      const int row2 = q / NRQ, t = b0 + (row2 >> 1), dc = t / nb;
      const int32_t ch = child[2 * (c0 + dc) + (row2 & 1)];
      if (ch >= 0) {
        const T* d = sc + row2 * LR + 4 * (q % NRQ);
        reinterpret_cast<V4*>(Qrc + ((int64_t)ch * nb + (t - dc * nb)) * NRS)[q % NRQ] = V4{d[0], d[1], d[2], d[3]};
      }
    }
    __syncthreads();
  }
  if (r < nr) {
#pragma unroll
    for (int i = 0; i < CW; i++) {
      const int a = share * CW + i;
      if (a < NP) sc[r * LS + a] = res[i];
    }
    if (share == 0)
      for (int a = NP; a < NS; a++) sc[r * LS + a] = (T)0;
  }
  __syncthreads();
  V4* out = reinterpret_cast<V4*>(Qp + i0 * NS);
  for (int q = tid; q < nr * NQ; q += kShiftThreads) {
    const T* d = sc + (q / NQ) * LS + 4 * (q % NQ);
    out[q] = V4{d[0], d[1], d[2], d[3]};
  }
}

// The form beside the near field (few registers, one wavefront per parent and
// group of configurations; it fits beside the near field's waves where the
// LDS-staged form above waits for room).  Along the halved axis the shift acts
// on lines of coefficients: the two other components (u, v) of n fixed, n_a = t running over 0..p-u-v.  One
// lane per (line, configuration): Q_n(P) at n_a = t sums the children's
// Q at n_a = t - k, k = 0..t, so a lane needs no per-term index search and
// every lane of a line runs the same loop.  A wavefront takes LPW = 64 / lines
// configurations of one parent cell; rows move through LDS whole (coalesced).
constexpr int kShiftWaves = 4;

// line l (0 .. (p+1)(p+2)/2 - 1) -> the two other components (u, v), by u + v
__device__ __forceinline__ void line_uv(int l, int& u, int& v) {
  int q = 0;
  while (l > q) {
    l -= q + 1;
    q++;
  }
  u = q - l;
  v = l;
}
// active index of the multi-index with component t on axis ax and (u, v) on
// the other two (in x, y, z order)
__device__ __forceinline__ int line_index(int ax, int u, int v, int t) {
  return ax == 0 ? midx(t, u, v) - 1 : ax == 1 ? midx(u, t, v) - 1 : midx(u, v, t) - 1;
}
template <int P>
constexpr int shift_lines() {
  return (P + 1) * (P + 2) / 2;
}
template <int P>
constexpr int shift_cpw() {
  return 64 / shift_lines<P>() >= 1 ? 64 / shift_lines<P>() : 1;
}

template <typename T, int P>
__global__ void __launch_bounds__(64 * kShiftWaves) k_m2m_lines(int32_t ncells, const int32_t* __restrict__ child, int axis,
                                                          ShiftW W, int nb, const T* __restrict__ Qc,
                                                          T* __restrict__ Qp) {
  constexpr int NP = nact(P);
  constexpr int NS = nstride(P);
  constexpr int NL = shift_lines<P>();
  constexpr int CPW = shift_cpw<P>();
  __shared__ double sw[(P + 1) * (P + 1)];  // the weights, read at per-lane indices
  __shared__ T sq[kShiftWaves][CPW][2][NS];
  __shared__ T so[kShiftWaves][CPW][NS];
  for (int i = threadIdx.x; i < (P + 1) * (P + 1); i += blockDim.x) sw[i] = W.w[i / (P + 1)][i % (P + 1)];
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ngrp = (nb + CPW - 1) / CPW;
  const int64_t item = (int64_t)blockIdx.x * kShiftWaves + w;
  if (item >= (int64_t)ncells * ngrp) return;
  const int c = (int)(item / ngrp), b0 = (int)(item % ngrp) * CPW;
  const int nbg = min(CPW, nb - b0);
  const int ch[2] = {child[2 * c], child[2 * c + 1]};
  for (int i = lane; i < nbg * 2 * NS; i += 64) {  // an absent child reads as a zero row
    const int cf = i / (2 * NS), e = (i / NS) & 1, a = i % NS;
    sq[w][cf][e][a] = ch[e] >= 0 ? Qc[((int64_t)ch[e] * nb + b0 + cf) * NS + a] : (T)0;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int cf = lane / NL;
  if (cf < nbg) {
    int u, v;
    line_uv(lane % NL, u, v);
    const int q = u + v;
    // the line of both children in registers (zero past its end and at the
    // monopole), read together; then every loop below is unrolled with the
    // line's bounds as predicates
    double x0[P + 1], x1[P + 1];
#pragma unroll
    for (int j = 0; j <= P; j++) {
      const bool ok = j <= P - q && j + q >= 1;
      const int idx = ok ? line_index(axis, u, v, j) : 0;
      x0[j] = ok ? (double)sq[w][cf][0][idx] : 0.0;
      x1[j] = ok ? (double)sq[w][cf][1][idx] : 0.0;
    }
#pragma unroll
    for (int t = 0; t <= P; t++) {
      if (t <= P - q && t + q >= 1) {
        double s = 0.0;
#pragma unroll
        for (int e = 0; e < 2; e++) {
#pragma unroll
          for (int k = 0; k <= t; k++) {
            const int j = t - k;  // the child's component on the axis; its degree is j + q
            if (j + q >= 1) {     // (Q_0 = 0: no monopole term)
              const double wv = sw[k * (P + 1) + j + q];
              const double wk = (e == 0 && (k & 1)) ? -wv : wv;
              s += wk * (e == 0 ? x0[j] : x1[j]);
            }
          }
        }
        so[w][cf][line_index(axis, u, v, t)] = (T)s;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int i = lane; i < nbg * NS; i += 64) {
    const int f = i / NS, a = i % NS;
    Qp[((int64_t)c * nb + b0 + f) * NS + a] = a < NP ? so[w][f][a] : (T)0;
  }
}

// ------------------------------------------------------------ L2L
// Eq.(taylorshift) from level l to l+1 along the halved axis:
// Vt_n(C) += sum_k gamma^k/k! rho^(|n|+2) Vt_{n+k e_a}(P).  Tabulated on the
// host per level: g[k] = gamma^k/k! (the child at -gamma takes (-1)^k of it)
// and r[d] = rho^(d+2).
struct TaylorW {
  double g[kPMax + 1];
  double r[kPMax + 1];
};

static TaylorW l2l_weights(double gam, double rho, int p) {
  TaylorW W{};
  double gk = 1.0;
  for (int k = 0; k <= p; k++) {
    W.g[k] = gk;
    gk = gk * gam / (double)(k + 1);
  }
  for (int d = 0; d <= p; d++) {
    double rp = 1.0;
    for (int j = 0; j < d + 2; j++) rp *= rho;
    W.r[d] = rp;
  }
  return W;
}

// Coefficients C0 <= a < C1 of one child row: pr and cr are the parent's and
// the child's rows in LDS, gs the signed weights gamma^k/k! of this child.
// FOLDED: the child's row holds only its n_z <= 1 components (the traceless
// M2L's output).  A local expansion satisfies the Laplace equation, so its
// other components follow from those: unrolling
// V(x, y, z) = -V(x + 2, y, z - 2) - V(x, y + 2, z - 2) gives, for z = 2k + e,
// V(x, y, z) = (-1)^k sum_j C(k, j) V(x + 2j, y + 2(k - j), e).  They are formed
// here before the shifted parent is added, so the row is read and written once.
template <typename T, int P, bool FOLDED, int AX, int C0, int C1>
__device__ __forceinline__ void l2l_coefs(const T* __restrict__ pr, const T* __restrict__ cr, const double* gs,
                                          const TaylorW& W, T* res) {
  static_for<C0, C1>([&](auto ac) {
    constexpr int a = decltype(ac)::value;
    constexpr int f = a + 1, x = mi_x(f), y = mi_y(f), z = mi_z(f), deg = x + y + z;
    double base;
    if constexpr (FOLDED && z >= 2) {
      constexpr int kz = z / 2, e = z % 2;
      double t = 0.0;
      static_for<0, kz + 1>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int src = midx(x + 2 * j, y + 2 * (kz - j), e) - 1;
        t += (double)binom(kz, j) * (double)cr[src];
      });
      base = (kz & 1) ? -t : t;
    } else {
      base = (double)cr[a];
    }
    double sh = 0.0;
    static_for<0, P - deg + 1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr int src = midx(x + (AX == 0 ? k : 0), y + (AX == 1 ? k : 0), z + (AX == 2 ? k : 0)) - 1;
      sh = fma(gs[k], (double)pr[src], sh);
    });
    res[a - C0] = (T)(base + W.r[deg] * sh);
  });
}

// Eq.(taylorshift) from level l to l+1 along the halved axis AX, one block per
// l2l_rows() consecutive (child cell, configuration) rows.  The child rows
// (contiguous) and each one's parent row are read with coalesced vector loads
// into LDS (rows padded to an odd stride), each thread forms one share of one
// row's coefficients with compile-time indices, and the finished rows go back
// through LDS with coalesced stores.
template <typename T, int P, bool FOLDED, int AX>
__global__ void __launch_bounds__(kShiftThreads) k_l2l(int64_t nitems, const int32_t* __restrict__ parent,
                                                     const int32_t* __restrict__ key, TaylorW W, int nb,
                                                     const T* __restrict__ Vp, T* __restrict__ Vc) {
  using V4 = RowVec4<T>;
  constexpr int NP = nact(P), NS = nstride(P), NQ = NS / 4, LS = NS + 1;
  constexpr int R = shift_rows<T>();
  constexpr int CH = kShiftThreads / R;     // shares of a row
  constexpr int CW = (NP + CH - 1) / CH;  // coefficients per share
  constexpr int QU = (R * NQ + kShiftThreads - 1) / kShiftThreads;  // vector loads per thread and row kind
  __shared__ T sp[R * LS], sc[R * LS];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * R;
  const int nr = (int)(nitems - i0 < R ? nitems - i0 : R);
  // row i0 + r is (cell c0 + (b0 + r) / nb, configuration (b0 + r) % nb)
  const int64_t c0 = i0 / nb;
  const int b0 = (int)(i0 - c0 * nb);
  const V4* cin = reinterpret_cast<const V4*>(Vc + i0 * NS);
  V4 cv[QU], pv[QU];
#pragma unroll
  for (int u = 0; u < QU; u++) {
    const int q = tid + u * kShiftThreads;
    if (q < nr * NQ) {
      const int t = b0 + q / NQ, dc = t / nb;
      const int64_t prow = (int64_t)parent[c0 + dc] * nb + (t - dc * nb);
      cv[u] = cin[q];
      pv[u] = reinterpret_cast<const V4*>(Vp + prow * NS)[q % NQ];
    }
  }
#pragma unroll
  for (int u = 0; u < QU; u++) {
    const int q = tid + u * kShiftThreads;
    if (q < nr * NQ) {
      const int o = (q / NQ) * LS + 4 * (q % NQ);
#pragma unroll
      for (int e = 0; e < 4; e++) {
        sc[o + e] = cv[u][e];
        sp[o + e] = pv[u][e];
      }
    }
  }
  __syncthreads();
  const int r = tid % R, share = tid / R;
  T res[CW];
  if (r < nr) {
    const int64_t c = c0 + (b0 + r) / nb;
    const bool neg = (key[c] & 1) == 0;  // the child at -gamma
    double gs[P + 1];
#pragma unroll
    for (int k = 0; k <= P; k++) gs[k] = (neg && (k & 1)) ? -W.g[k] : W.g[k];
    const T* pr = sp + r * LS;
    const T* cr = sc + r * LS;
    static_for<0, CH>([&](auto hc) {
      constexpr int h = decltype(hc)::value;
      if (share == h) l2l_coefs<T, P, FOLDED, AX, h * CW, (h + 1) * CW < NP ? (h + 1) * CW : NP>(pr, cr, gs, W, res);
    });
  }
  __syncthreads();
  if (r < nr) {
#pragma unroll
    for (int i = 0; i < CW; i++) {
      const int a = share * CW + i;
      if (a < NP) sp[r * LS + a] = res[i];
    }
    if (share == 0)
      for (int a = NP; a < NS; a++) sp[r * LS + a] = (T)0;
  }
  __syncthreads();
  V4* cout = reinterpret_cast<V4*>(Vc + i0 * NS);
  for (int q = tid; q < nr * NQ; q += kShiftThreads) {
    const T* d = sp + (q / NQ) * LS + 4 * (q % NQ);
    cout[q] = V4{d[0], d[1], d[2], d[3]};
  }
}

// The form beside the near field (few registers; the local rows arrive
// complete): one wavefront per (child cell, configuration), the parent's row
// read whole (coalesced) into LDS, then each lane adds its coefficients.  (The
// line form of M2M measured slower here: a child's row is read and written
// besides the parent's, and each line has half the terms.)
template <typename T, int P>
__global__ void __launch_bounds__(64 * kShiftWaves) k_l2l_lanes(int32_t ncells, const int32_t* __restrict__ parent,
                                                          const int32_t* __restrict__ key, int axis, TaylorW W,
                                                          int nb, const T* __restrict__ Vp, T* __restrict__ Vc) {
  constexpr int NP = nact(P);
  constexpr int NS = nstride(P);
  constexpr int NR = (NS + 63) / 64;
  __shared__ T sv[kShiftWaves][NS];
  __shared__ double sg[2 * (P + 1)];  // the weights, read at per-lane indices
  for (int i = threadIdx.x; i < 2 * (P + 1); i += blockDim.x) sg[i] = i <= P ? W.g[i] : W.r[i - (P + 1)];
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t item = (int64_t)blockIdx.x * kShiftWaves + w;
  if (item >= (int64_t)ncells * nb) return;
  const int c = (int)(item / nb), b = (int)(item % nb);
  const T* vp = Vp + ((int64_t)parent[c] * nb + b) * NS;
#pragma unroll
  for (int r = 0; r < NR; r++) {
    const int a = lane + 64 * r;
    if (a < NS) sv[w][a] = vp[a];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const bool neg = (key[c] & 1) == 0;  // the child at -gamma
  T* out = Vc + item * NS;
#pragma unroll
  for (int r = 0; r < NR; r++) {
    const int a = lane + 64 * r;
    if (a >= NP) continue;
    const int f = a + 1;
    const int n[3] = {kMI.x[f], kMI.y[f], kMI.z[f]};
    const int deg = n[0] + n[1] + n[2];
    double s = 0.0;
    for (int k = 0; deg + k <= P; k++) {
      int m[3] = {n[0], n[1], n[2]};
      m[axis] += k;
      const double gk = (neg && (k & 1)) ? -sg[k] : sg[k];
      s += gk * (double)sv[w][midx(m[0], m[1], m[2]) - 1];
    }
    out[a] = (T)((double)out[a] + sg[P + 1 + deg] * s);
  }
}

// ------------------------------------------------------------ launchers
template <typename T>
static T* qptr(Plan& P, DevBuf& buf, int l) {
  return buf.as<T>() + P.lev[l]->qoff;
}

template <typename T, int PP>
static void p2m_impl(Plan& P, int nb, const double* d_m, hipStream_t st) {
  (void)d_m;
  T* ms = P.m_sorted.as<T>();
  const int nl = P.lev[P.L]->ncells;
  const T* y = std::is_same<T, double>::value ? (const T*)P.yd.p : (const T*)P.yf.p;
  if (nb == 1) {
    k_p2m<T, PP, 1><<<ceil_div(nl, kP2MWaves), 64 * kP2MWaves, 0, st>>>(P.lstart.as<int32_t>(), P.lcount.as<int32_t>(),
                                                                       nl, y, ms, P.n, nb, qptr<T>(P, P.Q, P.L));
  } else {
    const int64_t items = (int64_t)nl * ceil_div(nb, kP2MConfigs);
    k_p2m<T, PP, kP2MConfigs><<<ceil_div(items, kP2MWaves), 64 * kP2MWaves, 0, st>>>(
        P.lstart.as<int32_t>(), P.lcount.as<int32_t>(), nl, y, ms, P.n, nb, qptr<T>(P, P.Q, P.L));
  }
  CCFMM_HIP(hipGetLastError());
}

template <typename T, int PP, bool FOLD>
static void m2m_level(int axis, int64_t nitems, const int32_t* child, const ShiftW& W, int nb, const T* Qc, T* Qp,
                      T* Qrc, hipStream_t st) {
  const unsigned grid = (unsigned)ceil_div(nitems, shift_rows<T>());
  if (axis == 0)
    k_m2m<T, PP, 0, FOLD><<<grid, kShiftThreads, 0, st>>>(nitems, child, W, nb, Qc, Qp, Qrc);
  else if (axis == 1)
    k_m2m<T, PP, 1, FOLD><<<grid, kShiftThreads, 0, st>>>(nitems, child, W, nb, Qc, Qp, Qrc);
  else
    k_m2m<T, PP, 2, FOLD><<<grid, kShiftThreads, 0, st>>>(nitems, child, W, nb, Qc, Qp, Qrc);
}

template <typename T, int PP>
static void m2m_impl(Plan& P, int nb, hipStream_t st) {
  const bool staged = shifts_staged(P);
  // the wide traceless M2L kernels read folded moments: the staged M2M writes
  // those of levels >= 2 (every child it reads), the M2L pass folds the rest
  // (all of them if M2M did not)
  const bool wide = P.tiles_variant == kM2LWide4 || P.tiles_variant == kM2LWide2 || P.tiles_variant == kM2LWide1;
  const bool fold = staged && wide && P.prm.m2l_traceless && PP <= wide_max_order(true) && P.L >= 2;
  for (int l = P.L - 1; l >= 1; l--) {
    const LevelData& D = *P.lev[l];
    const int a = P.geo.lev[l + 1].axis;
    const double gam = 0.5 * P.geo.lev[l + 1].h[a] / P.geo.lev[l].s;
    const double rho = P.geo.lev[l + 1].s / P.geo.lev[l].s;
    const ShiftW W = m2m_weights(gam, rho, PP);
    if (!staged) {
      const int64_t nt = (int64_t)D.ncells * ceil_div(nb, shift_cpw<PP>());
      k_m2m_lines<T, PP><<<ceil_div(nt, kShiftWaves), 64 * kShiftWaves, 0, st>>>(
          D.ncells, D.child.as<int32_t>(), a, W, nb, qptr<T>(P, P.Q, l + 1), qptr<T>(P, P.Q, l));
      CCFMM_HIP(hipGetLastError());
      continue;
    }
    const int64_t nt = (int64_t)D.ncells * nb;
    if (nt == 0) continue;
    if (fold)
      m2m_level<T, PP, true>(a, nt, D.child.as<int32_t>(), W, nb, qptr<T>(P, P.Q, l + 1), qptr<T>(P, P.Q, l),
                             P.Qr.as<T>() + P.lev[l + 1]->qoff / nstride(PP) * nred_stride(PP), st);
    else
      m2m_level<T, PP, false>(a, nt, D.child.as<int32_t>(), W, nb, qptr<T>(P, P.Q, l + 1), qptr<T>(P, P.Q, l),
                              nullptr, st);
    CCFMM_HIP(hipGetLastError());
  }
  P.q_folded = fold;
}

template <typename T, int PP, bool FOLDED>
static void l2l_level(int axis, int64_t nitems, const int32_t* parent, const int32_t* key, const TaylorW& W, int nb,
                      const T* Vp, T* Vc, hipStream_t st) {
  const unsigned grid = (unsigned)ceil_div(nitems, shift_rows<T>());
  if (axis == 0)
    k_l2l<T, PP, FOLDED, 0><<<grid, kShiftThreads, 0, st>>>(nitems, parent, key, W, nb, Vp, Vc);
  else if (axis == 1)
    k_l2l<T, PP, FOLDED, 1><<<grid, kShiftThreads, 0, st>>>(nitems, parent, key, W, nb, Vp, Vc);
  else
    k_l2l<T, PP, FOLDED, 2><<<grid, kShiftThreads, 0, st>>>(nitems, parent, key, W, nb, Vp, Vc);
}

template <typename T, int PP>
static void l2l_impl(Plan& P, int nb, hipStream_t st) {
  const bool staged = shifts_staged(P);
  for (int l = 1; l < P.L; l++) {
    const LevelData& C = *P.lev[l + 1];
    const int a = P.geo.lev[l + 1].axis;
    const double gam = 0.5 * P.geo.lev[l + 1].h[a] / P.geo.lev[l].s;
    const double rho = P.geo.lev[l + 1].s / P.geo.lev[l].s;
    const int64_t nt = (int64_t)C.ncells * nb;
    if (nt == 0) continue;
    const TaylorW W = l2l_weights(gam, rho, PP);
    if (!staged)
      k_l2l_lanes<T, PP><<<ceil_div(nt, kShiftWaves), 64 * kShiftWaves, 0, st>>>(
          C.ncells, C.parent.as<int32_t>(), C.key.as<int32_t>(), a, W, nb, qptr<T>(P, P.V, l),
          qptr<T>(P, P.V, l + 1));
    else if (P.v_folded)
      l2l_level<T, PP, true>(a, nt, C.parent.as<int32_t>(), C.key.as<int32_t>(), W, nb, qptr<T>(P, P.V, l),
                             qptr<T>(P, P.V, l + 1), st);
    else
      l2l_level<T, PP, false>(a, nt, C.parent.as<int32_t>(), C.key.as<int32_t>(), W, nb, qptr<T>(P, P.V, l),
                              qptr<T>(P, P.V, l + 1), st);
    CCFMM_HIP(hipGetLastError());
  }
}

#define CCFMM_DISPATCH_P(P_, FN, ...)                        \
  switch (P_) {                                              \
    case 1: FN<1>(__VA_ARGS__); break;                       \
    case 2: FN<2>(__VA_ARGS__); break;                       \
    case 3: FN<3>(__VA_ARGS__); break;                       \
    case 4: FN<4>(__VA_ARGS__); break;                       \
    case 5: FN<5>(__VA_ARGS__); break;                       \
    case 6: FN<6>(__VA_ARGS__); break;                       \
    case 7: FN<7>(__VA_ARGS__); break;                       \
    case 8: FN<8>(__VA_ARGS__); break;                       \
    default: fail(CCFMM_EINVAL, "order out of range");       \
  }

template <int PP>
static void p2m_d(Plan& P, int nb, const double* d_m, hipStream_t st) {
  if (P.precision == CCFMM_PREC_FP64)
    p2m_impl<double, PP>(P, nb, d_m, st);
  else
    p2m_impl<float, PP>(P, nb, d_m, st);
}
template <int PP>
static void m2m_d(Plan& P, int nb, hipStream_t st) {
  if (P.precision == CCFMM_PREC_FP64)
    m2m_impl<double, PP>(P, nb, st);
  else
    m2m_impl<float, PP>(P, nb, st);
}
template <int PP>
static void l2l_d(Plan& P, int nb, hipStream_t st) {
  if (P.precision == CCFMM_PREC_FP64)
    l2l_impl<double, PP>(P, nb, st);
  else
    l2l_impl<float, PP>(P, nb, st);
}

// moments in sorted order (FP64 or FP32 per the plan): [config][3][n], plus
// [n][3][config] for the batched near field
template <typename T>
static void permute_impl(Plan& P, int nb, const double* d_m, hipStream_t st) {
  dim3 g1(ceil_div(P.n, 256), nb);
  k_permute_moments<T><<<g1, 256, 0, st>>>(d_m, P.perm.as<int32_t>(), P.n, nb, P.m_sorted.as<T>());
  CCFMM_HIP(hipGetLastError());
  if (nb >= P.batched_min) {
    k_permute_moments_t<T><<<ceil_div(P.n * nb, 256), 256, 0, st>>>(d_m, P.perm.as<int32_t>(), P.n, nb,
                                                                     P.m_sorted_t.as<T>());
    CCFMM_HIP(hipGetLastError());
  }
}

void run_permute(Plan& P, int nb, const double* d_m, hipStream_t st) {
  if (P.precision == CCFMM_PREC_FP64)
    permute_impl<double>(P, nb, d_m, st);
  else
    permute_impl<float>(P, nb, d_m, st);
}

void run_p2m(Plan& P, int nb, const double* d_m, hipStream_t st) { CCFMM_DISPATCH_P(P.p, p2m_d, P, nb, d_m, st); }
void run_m2m(Plan& P, int nb, hipStream_t st) { CCFMM_DISPATCH_P(P.p, m2m_d, P, nb, st); }
void run_l2l(Plan& P, int nb, hipStream_t st) { CCFMM_DISPATCH_P(P.p, l2l_d, P, nb, st); }

}  // namespace ccfmm
