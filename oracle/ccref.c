/*
 * ccref.c -- CPU oracle: FP64 brute-force dipole sum and the paper's recursive
 * Cartesian FMM (Zhang & Haas).  TEST INFRASTRUCTURE ONLY: nothing on the GPU
 * product path may link, load or call this file.  Plain, slow and literal on
 * purpose; every routine names the passage of the paper it follows.
 *
 * Readings of passages where the paper is silent or garbled (all documented in
 * the design notes of the repository):
 *  - truncation: multipoles |q| <= p, locals |n| <= p, D up to order 2p
 *    (params.truncation = 1 selects the other reading, |n| + |q| <= p);
 *  - near/far tie alpha == alpha_m counts as far, evaluated exactly with
 *    squared, per-level normalised distances (see near_pair);
 *  - a point on a cell face belongs to the upper cell; the top face is clamped
 *    into the last cell (see leaf_coord);
 *  - Eq.(H) carries the minus sign of H = -grad V, Eq.(H2) is used as the
 *    field of source dipole j, (3 (m_j.u) u - m_j)/r^3, and the energy carries
 *    the 1/2 of the Appendix;
 *  - pairs at zero separation do not interact (this covers the self term);
 *  - empty cells are not created (their moments are zero and they hold no
 *    field points, so the result is unchanged).
 *
 * Compile with -ffp-contract=off: the discrete decisions (leaf index, near
 * test) must be the plain IEEE sequence written here.
 */
#include "ccref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KMAX (2 * CCREF_PMAX)
#define CUBE(K) (((K) + 1) * ((K) + 1) * ((K) + 1))

static inline int cidx(int nx, int ny, int nz, int K) { return (nx * (K + 1) + ny) * (K + 1) + nz; }

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

/* n! for n <= KMAX, as doubles (exact up to 18!). */
static double fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; i++) f *= i;
  return f;
}

static double ipow(double x, int e) {
  double r = 1.0;
  for (int i = 0; i < e; i++) r *= x;
  return r;
}

/* ------------------------------------------------------------------------- */
/* F-table, Eqs.(Dn) and (Dnr).                                               */
/* D_k(r) = r^-(2|k|+1) sum_{|q|=|k|} F_k(q) r^q.  F_0(0) = 1 and F_{n+e_v} is */
/* obtained from F_n by applying -d/dr_v to each term r^q / r^(2|n|+1):        */
/*   (2|n|+1 - q_v) r^(q+e_v) - q_v r^(q-e_v+2e_u) - q_v r^(q-e_v+2e_w).       */
/* The table is stored, as the paper suggests, as a list of the q with a     */
/* nonzero F_k(q) and their values, for every k.                             */
/* ------------------------------------------------------------------------- */
typedef struct {
  int cnt;
  int* q;      /* 3*cnt exponents */
  double* f;   /* cnt values */
} fentry;

static fentry ftab[CUBE(KMAX)];
static int ftab_ready = 0;

static void fentry_add(fentry* e, int qx, int qy, int qz, double v, int* cap) {
  for (int i = 0; i < e->cnt; i++) {
    if (e->q[3 * i] == qx && e->q[3 * i + 1] == qy && e->q[3 * i + 2] == qz) {
      e->f[i] += v;
      return;
    }
  }
  if (e->cnt == *cap) {
    *cap = *cap ? 2 * *cap : 8;
    e->q = (int*)realloc(e->q, sizeof(int) * 3 * (*cap));
    e->f = (double*)realloc(e->f, sizeof(double) * (*cap));
  }
  e->q[3 * e->cnt] = qx;
  e->q[3 * e->cnt + 1] = qy;
  e->q[3 * e->cnt + 2] = qz;
  e->f[e->cnt] = v;
  e->cnt++;
}

static void build_ftable(void) {
  if (ftab_ready) return;
  memset(ftab, 0, sizeof(ftab));
  int cap0 = 0;
  fentry_add(&ftab[cidx(0, 0, 0, KMAX)], 0, 0, 0, 1.0, &cap0);
  for (int deg = 1; deg <= KMAX; deg++) {
    for (int kx = deg; kx >= 0; kx--) {
      for (int ky = deg - kx; ky >= 0; ky--) {
        int kz = deg - kx - ky;
        int k[3] = {kx, ky, kz};
        /* pick nu with k_nu > 0: x first, then y, then z */
        int nu = (kx > 0) ? 0 : (ky > 0 ? 1 : 2);
        int n[3] = {kx, ky, kz};
        n[nu] -= 1;
        int nn = n[0] + n[1] + n[2];
        const fentry* src = &ftab[cidx(n[0], n[1], n[2], KMAX)];
        fentry* dst = &ftab[cidx(k[0], k[1], k[2], KMAX)];
        int cap = 0;
        for (int t = 0; t < src->cnt; t++) {
          int q[3] = {src->q[3 * t], src->q[3 * t + 1], src->q[3 * t + 2]};
          double F = src->f[t];
          /* (2n+1 - q_nu) r^(q + e_nu) */
          {
            int a[3] = {q[0], q[1], q[2]};
            a[nu] += 1;
            double c = (double)(2 * nn + 1 - q[nu]);
            if (c != 0.0) fentry_add(dst, a[0], a[1], a[2], c * F, &cap);
          }
          if (q[nu] > 0) {
            for (int mu = 0; mu < 3; mu++) {
              if (mu == nu) continue;
              int a[3] = {q[0], q[1], q[2]};
              a[nu] -= 1;
              a[mu] += 2;
              fentry_add(dst, a[0], a[1], a[2], -(double)q[nu] * F, &cap);
            }
          }
        }
        /* drop exact zeros produced by cancellation */
        int w = 0;
        for (int t = 0; t < dst->cnt; t++) {
          if (dst->f[t] != 0.0) {
            dst->q[3 * w] = dst->q[3 * t];
            dst->q[3 * w + 1] = dst->q[3 * t + 1];
            dst->q[3 * w + 2] = dst->q[3 * t + 2];
            dst->f[w] = dst->f[t];
            w++;
          }
        }
        dst->cnt = w;
      }
    }
  }
  ftab_ready = 1;
}

double ccref_ftable(int32_t kx, int32_t ky, int32_t kz, int32_t qx, int32_t qy, int32_t qz) {
  if (kx < 0 || ky < 0 || kz < 0 || kx + ky + kz > KMAX) return 0.0;
  build_ftable();
  const fentry* e = &ftab[cidx(kx, ky, kz, KMAX)];
  for (int t = 0; t < e->cnt; t++)
    if (e->q[3 * t] == qx && e->q[3 * t + 1] == qy && e->q[3 * t + 2] == qz) return e->f[t];
  return 0.0;
}

/* Eq.(Dn): D_k(c) for all |k| <= K into the dense cube of side K+1. */
static void dtensor(int K, const double c[3], double* D) {
  double px[KMAX + 1], py[KMAX + 1], pz[KMAX + 1];
  px[0] = py[0] = pz[0] = 1.0;
  for (int i = 1; i <= K; i++) {
    px[i] = px[i - 1] * c[0];
    py[i] = py[i - 1] * c[1];
    pz[i] = pz[i - 1] * c[2];
  }
  double r2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
  double r = sqrt(r2);
  memset(D, 0, sizeof(double) * CUBE(K));
  for (int kx = 0; kx <= K; kx++)
    for (int ky = 0; kx + ky <= K; ky++)
      for (int kz = 0; kx + ky + kz <= K; kz++) {
        int deg = kx + ky + kz;
        const fentry* e = &ftab[cidx(kx, ky, kz, KMAX)];
        double s = 0.0;
        for (int t = 0; t < e->cnt; t++)
          s += e->f[t] * px[e->q[3 * t]] * py[e->q[3 * t + 1]] * pz[e->q[3 * t + 2]];
        D[cidx(kx, ky, kz, K)] = s / ipow(r, 2 * deg + 1);
      }
}

int ccref_dtensor(int32_t K, const double c[3], double* D) {
  if (K < 0 || K > KMAX) return -1;
  build_ftable();
  dtensor(K, c, D);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Expansion operators, Sec. 3.                                              */
/* ------------------------------------------------------------------------- */

/* Eq.(multipolemoments): Q_n += (1/n!) m . grad(y^n), y = x - center.
 * grad_a y^n = n_a y^(n - e_a). */
static void p2m_one(int p, const double y[3], const double mm[3], double* Q) {
  for (int nx = 0; nx <= p; nx++)
    for (int ny = 0; nx + ny <= p; ny++)
      for (int nz = 0; nx + ny + nz <= p; nz++) {
        double inv_nf = 1.0 / (fact(nx) * fact(ny) * fact(nz));
        double g = 0.0;
        if (nx > 0) g += mm[0] * nx * ipow(y[0], nx - 1) * ipow(y[1], ny) * ipow(y[2], nz);
        if (ny > 0) g += mm[1] * ny * ipow(y[0], nx) * ipow(y[1], ny - 1) * ipow(y[2], nz);
        if (nz > 0) g += mm[2] * nz * ipow(y[0], nx) * ipow(y[1], ny) * ipow(y[2], nz - 1);
        Q[cidx(nx, ny, nz, p)] += g * inv_nf;
      }
}

int ccref_p2m(int32_t p, const double center[3], int64_t n, const double* pos, const double* m,
              double* Q) {
  if (p < 0 || p > CCREF_PMAX || n < 0) return -1;
  memset(Q, 0, sizeof(double) * CUBE(p));
  for (int64_t i = 0; i < n; i++) {
    double y[3] = {pos[3 * i] - center[0], pos[3 * i + 1] - center[1], pos[3 * i + 2] - center[2]};
    p2m_one(p, y, &m[3 * i], Q);
  }
  return 0;
}

/* Charge moments of Sec. 3: Q_n = (1/n!) sum_i q_i y_i^n. */
int ccref_charge_moments(int32_t p, const double center[3], int64_t n, const double* pos,
                         const double* q, double* Q) {
  if (p < 0 || p > KMAX || n < 0) return -1;
  memset(Q, 0, sizeof(double) * CUBE(p));
  for (int64_t i = 0; i < n; i++) {
    double y[3] = {pos[3 * i] - center[0], pos[3 * i + 1] - center[1], pos[3 * i + 2] - center[2]};
    for (int nx = 0; nx <= p; nx++)
      for (int ny = 0; nx + ny <= p; ny++)
        for (int nz = 0; nx + ny + nz <= p; nz++)
          Q[cidx(nx, ny, nz, p)] += q[i] * ipow(y[0], nx) * ipow(y[1], ny) * ipow(y[2], nz) /
                                    (fact(nx) * fact(ny) * fact(nz));
  }
  return 0;
}

/* Eq.(momentshift): Q_n = sum_q c^q/q! Q'_{n-q}, Q' about the child center,
 * c = child center - parent center. Accumulates into Qp. */
static void m2m(int p, const double c[3], const double* Qc, double* Qp) {
  for (int nx = 0; nx <= p; nx++)
    for (int ny = 0; nx + ny <= p; ny++)
      for (int nz = 0; nx + ny + nz <= p; nz++) {
        double s = 0.0;
        for (int qx = 0; qx <= nx; qx++)
          for (int qy = 0; qy <= ny; qy++)
            for (int qz = 0; qz <= nz; qz++)
              s += ipow(c[0], qx) * ipow(c[1], qy) * ipow(c[2], qz) /
                   (fact(qx) * fact(qy) * fact(qz)) * Qc[cidx(nx - qx, ny - qy, nz - qz, p)];
        Qp[cidx(nx, ny, nz, p)] += s;
      }
}

int ccref_m2m(int32_t p, const double c[3], const double* Qchild, double* Qparent) {
  if (p < 0 || p > CCREF_PMAX) return -1;
  m2m(p, c, Qchild, Qparent);
  return 0;
}

/* Eq.(taylorshift): V'_n = sum_q c^q/q! V_{n+q}, c = child center - parent center. */
static void l2l(int p, const double c[3], const double* Vp, double* Vc) {
  for (int nx = 0; nx <= p; nx++)
    for (int ny = 0; nx + ny <= p; ny++)
      for (int nz = 0; nx + ny + nz <= p; nz++) {
        double s = 0.0;
        for (int qx = 0; nx + qx <= p; qx++)
          for (int qy = 0; nx + qx + ny + qy <= p; qy++)
            for (int qz = 0; nx + qx + ny + qy + nz + qz <= p; qz++)
              s += ipow(c[0], qx) * ipow(c[1], qy) * ipow(c[2], qz) /
                   (fact(qx) * fact(qy) * fact(qz)) * Vp[cidx(nx + qx, ny + qy, nz + qz, p)];
        Vc[cidx(nx, ny, nz, p)] = s;
      }
}

int ccref_l2l(int32_t p, const double c[3], const double* Vparent, double* Vchild) {
  if (p < 0 || p > CCREF_PMAX) return -1;
  l2l(p, c, Vparent, Vchild);
  return 0;
}

/* Eq.(taylorcalc): V_n += (-1)^|n| sum_q D_{n+q}(c) Q_q, c = target center -
 * source center; |n| <= p, |q| <= p, so D is needed up to order 2p.  With
 * total != 0 only the terms with |n| + |q| <= p are kept (the other reading
 * of "truncate after the p-th order").  D is the caller's scratch of side
 * 2p+1. */
static void m2l(int p, const double c[3], const double* Q, double* V, double* D, int total) {
  int K = 2 * p;
  dtensor(K, c, D);
  for (int nx = 0; nx <= p; nx++)
    for (int ny = 0; nx + ny <= p; ny++)
      for (int nz = 0; nx + ny + nz <= p; nz++) {
        const int qmax = total ? p - (nx + ny + nz) : p;
        double s = 0.0;
        for (int qx = 0; qx <= qmax; qx++)
          for (int qy = 0; qx + qy <= qmax; qy++)
            for (int qz = 0; qx + qy + qz <= qmax; qz++)
              s += D[cidx(nx + qx, ny + qy, nz + qz, K)] * Q[cidx(qx, qy, qz, p)];
        double sign = ((nx + ny + nz) & 1) ? -1.0 : 1.0;
        V[cidx(nx, ny, nz, p)] += sign * s;
      }
}

static int m2l_call(int32_t p, const double c[3], const double* Q, double* V, int total) {
  if (p < 0 || p > CCREF_PMAX) return -1;
  build_ftable();
  double* D = (double*)malloc(sizeof(double) * CUBE(2 * p));
  m2l(p, c, Q, V, D, total);
  free(D);
  return 0;
}

int ccref_m2l(int32_t p, const double c[3], const double* Q, double* V) { return m2l_call(p, c, Q, V, 0); }

int ccref_m2l_total(int32_t p, const double c[3], const double* Q, double* V) { return m2l_call(p, c, Q, V, 1); }

/* Eq.(H) with the sign of H = -grad V: H_a = -sum_n V_n n_a y^(n-e_a) / n!. */
static void l2p(int p, const double* V, const double y[3], double H[3]) {
  double h[3] = {0.0, 0.0, 0.0};
  for (int nx = 0; nx <= p; nx++)
    for (int ny = 0; nx + ny <= p; ny++)
      for (int nz = 0; nx + ny + nz <= p; nz++) {
        double v = V[cidx(nx, ny, nz, p)] / (fact(nx) * fact(ny) * fact(nz));
        if (nx > 0) h[0] += v * nx * ipow(y[0], nx - 1) * ipow(y[1], ny) * ipow(y[2], nz);
        if (ny > 0) h[1] += v * ny * ipow(y[0], nx) * ipow(y[1], ny - 1) * ipow(y[2], nz);
        if (nz > 0) h[2] += v * nz * ipow(y[0], nx) * ipow(y[1], ny) * ipow(y[2], nz - 1);
      }
  H[0] = -h[0];
  H[1] = -h[1];
  H[2] = -h[2];
}

int ccref_l2p(int32_t p, const double* V, const double y[3], double H[3]) {
  if (p < 0 || p > CCREF_PMAX) return -1;
  l2p(p, V, y, H);
  return 0;
}

/* Eq.(Vm): V(x) = sum_n D_n(x) Q_n. */
double ccref_multipole_potential(int32_t p, const double* Q, const double x[3]) {
  if (p < 0 || p > KMAX) return NAN;
  build_ftable();
  double* D = (double*)malloc(sizeof(double) * CUBE(p));
  dtensor(p, x, D);
  double s = 0.0;
  for (int nx = 0; nx <= p; nx++)
    for (int ny = 0; nx + ny <= p; ny++)
      for (int nz = 0; nx + ny + nz <= p; nz++) s += D[cidx(nx, ny, nz, p)] * Q[cidx(nx, ny, nz, p)];
  free(D);
  return s;
}

/* Eq.(taylorexpansion): V(y) = sum_n V_n y^n / n!. */
double ccref_local_potential(int32_t p, const double* V, const double y[3]) {
  double s = 0.0;
  for (int nx = 0; nx <= p; nx++)
    for (int ny = 0; nx + ny <= p; ny++)
      for (int nz = 0; nx + ny + nz <= p; nz++)
        s += V[cidx(nx, ny, nz, p)] * ipow(y[0], nx) * ipow(y[1], ny) * ipow(y[2], nz) /
             (fact(nx) * fact(ny) * fact(nz));
  return s;
}

/* ------------------------------------------------------------------------- */
/* Pair field, Eq.(H2) read as the field of dipole j at i (units mu0/4pi=1):  */
/*   H = (3 (m_j . u) u - m_j) / r^3,  r = x_i - x_j,  u = r/|r|.            */
/* ------------------------------------------------------------------------- */
static inline void pair_field(const double* xi, const double* xj, const double* mj, double* H) {
  double rx = xi[0] - xj[0], ry = xi[1] - xj[1], rz = xi[2] - xj[2];
  double r2 = rx * rx + ry * ry + rz * rz;
  if (r2 == 0.0) return; /* the dipole at the field point itself, or a coincident one */
  double r = sqrt(r2);
  double ux = rx / r, uy = ry / r, uz = rz / r;
  double mu = mj[0] * ux + mj[1] * uy + mj[2] * uz;
  double r3 = r2 * r;
  H[0] += (3.0 * mu * ux - mj[0]) / r3;
  H[1] += (3.0 * mu * uy - mj[1]) / r3;
  H[2] += (3.0 * mu * uz - mj[2]) / r3;
}

static void set_threads(int32_t nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int ccref_bruteforce(int64_t n, const double* pos, const double* m, double* H, int32_t nthreads) {
  if (n < 0) return -1;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; i++) {
    double h[3] = {0.0, 0.0, 0.0};
    for (int64_t j = 0; j < n; j++) pair_field(&pos[3 * i], &pos[3 * j], &m[3 * j], h);
    H[3 * i] = h[0];
    H[3 * i + 1] = h[1];
    H[3 * i + 2] = h[2];
  }
  return 0;
}

int ccref_bruteforce_targets(int64_t n, const double* pos, const double* m, int64_t nt,
                             const int64_t* idx, double* H, int32_t nthreads) {
  if (n < 0 || nt < 0) return -1;
  for (int64_t t = 0; t < nt; t++)
    if (idx[t] < 0 || idx[t] >= n) return -1;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < nt; t++) {
    int64_t i = idx[t];
    double h[3] = {0.0, 0.0, 0.0};
    for (int64_t j = 0; j < n; j++) pair_field(&pos[3 * i], &pos[3 * j], &m[3 * j], h);
    H[3 * t] = h[0];
    H[3 * t + 1] = h[1];
    H[3 * t + 2] = h[2];
  }
  return 0;
}

double ccref_energy(int64_t n, const double* m, const double* H) {
  double e = 0.0;
  for (int64_t i = 0; i < n; i++)
    e += m[3 * i] * H[3 * i] + m[3 * i + 1] * H[3 * i + 1] + m[3 * i + 2] * H[3 * i + 2];
  return -0.5 * e;
}

/* ------------------------------------------------------------------------- */
/* Tree: recursive halving (Sec. 2) with the level rule of Sec. 4.            */
/* ------------------------------------------------------------------------- */

typedef struct cell cell;
typedef struct {
  cell** v;
  int64_t n, cap;
} cellvec;

struct cell {
  int level;
  int64_t i[3];      /* integer coordinates at this level */
  double center[3];
  cell* parent;
  cell* child[2];    /* NULL if empty (pruned) or leaf */
  int is_leaf;       /* smallest cell */
  int64_t* idx;      /* dipole indices (smallest cells only) */
  int64_t count;
  double* Q;         /* multipole moments, dense cube side p+1 */
  double* V;         /* local (Taylor) coefficients, dense cube side p+1 */
  cellvec partners;
  cellvec near;
};

static void cv_push(cellvec* v, cell* c) {
  if (v->n == v->cap) {
    v->cap = v->cap ? 2 * v->cap : 8;
    v->v = (cell**)realloc(v->v, sizeof(cell*) * v->cap);
  }
  v->v[v->n++] = c;
}

typedef struct {
  int p, L;
  double theta, theta2;
  double lo[3], W[3];
  int axis[CCREF_LMAX + 1];   /* axis[l]: split from level l-1 to l */
  int k[CCREF_LMAX + 1][3];   /* split counts per axis at level l */
  double h[CCREF_LMAX + 1][3];
  double g[CCREF_LMAX + 1][3]; /* h / min side at that level */
  const double* pos;
  const double* m;
  double* H;
  int64_t ncells;
  int64_t m2l_pairs[CCREF_LMAX + 1];
  int64_t p2p_leaf_pairs;
  int64_t nleaves;
  /* optional per-smallest-cell parameters, given per dipole (all dipoles of a
   * smallest cell carry the same values): local order and opening angle */
  const int32_t* leaf_p;
  const double* leaf_theta;
  int total; /* M2L keeps only |n| + |q| <= p */
} tree;

/* Eq.(so): optimal dipoles per smallest cell. */
static double s_opt(int p) { return p > 3 ? 0.74 * (double)p * (double)p : 8.0; }

/* Root cell (reading: caller box, else tight bounding box; a degenerate axis
 * takes the smallest nonzero side, all-coincident points a side of 1). */
static int root_box(int64_t n, const double* pos, const ccref_params* prm, double lo[3], double W[3]) {
  if (prm->has_box) {
    for (int a = 0; a < 3; a++) {
      lo[a] = prm->box_lo[a];
      W[a] = prm->box_hi[a] - prm->box_lo[a];
      if (!(W[a] > 0.0) || !isfinite(W[a])) return -1;
    }
    for (int64_t i = 0; i < n; i++)
      for (int a = 0; a < 3; a++)
        if (pos[3 * i + a] < prm->box_lo[a] || pos[3 * i + a] > prm->box_hi[a]) return -1;
    return 0;
  }
  double mn[3], mx[3];
  for (int a = 0; a < 3; a++) {
    mn[a] = pos[a];
    mx[a] = pos[a];
  }
  for (int64_t i = 1; i < n; i++)
    for (int a = 0; a < 3; a++) {
      if (pos[3 * i + a] < mn[a]) mn[a] = pos[3 * i + a];
      if (pos[3 * i + a] > mx[a]) mx[a] = pos[3 * i + a];
    }
  double smallest = 0.0;
  for (int a = 0; a < 3; a++) {
    double w = mx[a] - mn[a];
    if (w > 0.0 && (smallest == 0.0 || w < smallest)) smallest = w;
  }
  if (smallest == 0.0) smallest = 1.0;
  for (int a = 0; a < 3; a++) {
    lo[a] = mn[a];
    W[a] = (mx[a] - mn[a] > 0.0) ? (mx[a] - mn[a]) : smallest;
  }
  return 0;
}

/* Split sequence: each level halves the currently longest side, ties broken
 * x before y before z, so the smallest cells end up as close to cubic as the
 * halving allows (rule of thumb of Sec. 4). */
static void split_sequence(tree* T, int L) {
  double w[3] = {T->W[0], T->W[1], T->W[2]};
  int k[3] = {0, 0, 0};
  T->axis[0] = -1;
  for (int a = 0; a < 3; a++) {
    T->k[0][a] = 0;
    T->h[0][a] = w[a];
  }
  for (int l = 1; l <= L; l++) {
    int a = 0;
    if (w[1] > w[a]) a = 1;
    if (w[2] > w[a]) a = 2;
    w[a] = w[a] / 2.0;
    k[a]++;
    T->axis[l] = a;
    for (int b = 0; b < 3; b++) {
      T->k[l][b] = k[b];
      T->h[l][b] = w[b];
    }
  }
  for (int l = 0; l <= L; l++) {
    double mn = T->h[l][0];
    if (T->h[l][1] < mn) mn = T->h[l][1];
    if (T->h[l][2] < mn) mn = T->h[l][2];
    for (int b = 0; b < 3; b++) T->g[l][b] = T->h[l][b] / mn;
  }
}

/* Leaf coordinate along axis a (reading: floor rule, top face clamped). */
static int64_t leaf_coord(double x, double lo, double W, int k) {
  double t = x - lo;
  t = t * ldexp(1.0, k);
  double u = t / W;
  double f = floor(u);
  int64_t i = (int64_t)f;
  int64_t top = ((int64_t)1 << k) - 1;
  if (f < 0.0) i = 0;
  if (i > top) i = top;
  return i;
}

/* Number of distinct smallest cells for a trial level count (leaf rule 1). */
static int64_t count_nonempty(const tree* T, int64_t n, int L) {
  tree tmp = *T;
  split_sequence(&tmp, L);
  int64_t* keys = (int64_t*)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
  for (int64_t i = 0; i < n; i++) {
    int64_t c[3];
    for (int a = 0; a < 3; a++) c[a] = leaf_coord(T->pos[3 * i + a], T->lo[a], T->W[a], tmp.k[L][a]);
    keys[i] = (c[0] << (tmp.k[L][1] + tmp.k[L][2])) | (c[1] << tmp.k[L][2]) | c[2];
  }
  /* count distinct by sorting (insertion into a simple open hash) */
  int64_t cap = 1;
  while (cap < 2 * n + 2) cap <<= 1;
  int64_t* tab = (int64_t*)malloc(sizeof(int64_t) * cap);
  for (int64_t i = 0; i < cap; i++) tab[i] = -1;
  int64_t distinct = 0;
  for (int64_t i = 0; i < n; i++) {
    uint64_t h = (uint64_t)keys[i] * 0x9E3779B97F4A7C15ull;
    int64_t s = (int64_t)(h >> 20) & (cap - 1);
    while (tab[s] != -1 && tab[s] != keys[i]) s = (s + 1) & (cap - 1);
    if (tab[s] == -1) {
      tab[s] = keys[i];
      distinct++;
    }
  }
  free(tab);
  free(keys);
  return distinct;
}

/* Level count: the tree depth that makes the average dipoles per smallest
 * cell closest to s (Sec. 4); ties go to the shallower tree. */
static int choose_levels(tree* T, int64_t n, double s, int rule) {
  int best = 0;
  double bestd = INFINITY;
  for (int L = 0; L <= CCREF_LMAX; L++) {
    double avg;
    if (rule == 0) {
      avg = (double)n / ldexp(1.0, L);
    } else {
      avg = (double)n / (double)count_nonempty(T, n, L);
    }
    double d = fabs(avg - s);
    if (d < bestd) {
      bestd = d;
      best = L;
    }
  }
  return best;
}

static cell* new_cell(tree* T, cell* parent, int level, const int64_t i[3]) {
  cell* c = (cell*)calloc(1, sizeof(cell));
  c->level = level;
  c->parent = parent;
  for (int a = 0; a < 3; a++) {
    c->i[a] = i[a];
    c->center[a] = T->lo[a] + ((double)i[a] + 0.5) * T->h[level][a];
  }
  int side = T->p + 1;
  c->Q = (double*)calloc((size_t)side * side * side, sizeof(double));
  c->V = (double*)calloc((size_t)side * side * side, sizeof(double));
  T->ncells++;
  return c;
}

/* Recursive halving: a cell at level l splits along axis[l+1]; each dipole
 * goes to the half that holds its smallest cell. */
static void build(tree* T, cell* c, int64_t* idx, int64_t count, const int64_t* leafc) {
  if (c->level == T->L) {
    c->is_leaf = 1;
    c->idx = idx;
    c->count = count;
    T->nleaves++;
    return;
  }
  int l1 = c->level + 1;
  int a = T->axis[l1];
  int shift = T->k[T->L][a] - T->k[l1][a];
  int64_t* part[2];
  int64_t cnt[2] = {0, 0};
  part[0] = (int64_t*)malloc(sizeof(int64_t) * (count ? count : 1));
  part[1] = (int64_t*)malloc(sizeof(int64_t) * (count ? count : 1));
  for (int64_t t = 0; t < count; t++) {
    int64_t d = idx[t];
    int bit = (int)((leafc[3 * d + a] >> shift) & 1);
    part[bit][cnt[bit]++] = d;
  }
  free(idx);
  for (int b = 0; b < 2; b++) {
    if (cnt[b] == 0) {
      free(part[b]);
      c->child[b] = NULL;
      continue;
    }
    int64_t ci[3] = {c->i[0], c->i[1], c->i[2]};
    ci[a] = 2 * ci[a] + b;
    c->child[b] = new_cell(T, c, l1, ci);
    build(T, c->child[b], part[b], cnt[b], leafc);
  }
}

/* Opening-angle test of Sec. 2: alpha = 2r/d with r the cell radius and d
 * the center distance; near iff alpha > alpha_m.  Evaluated exactly as
 * far <=> theta^2 * |delta*g|^2 >= |g|^2 with delta the integer offset at the
 * level and g the sides divided by the smallest side (so alpha == alpha_m is
 * far).  Sums run x, y, z in this order. */
static int near_pair(const tree* T, const cell* A, const cell* C) {
  int l = C->level;
  const double* g = T->g[l];
  double dx = (double)(A->i[0] - C->i[0]) * g[0];
  double dy = (double)(A->i[1] - C->i[1]) * g[1];
  double dz = (double)(A->i[2] - C->i[2]) * g[2];
  double D = dx * dx;
  D = D + dy * dy;
  D = D + dz * dz;
  double R = g[0] * g[0];
  R = R + g[1] * g[1];
  R = R + g[2] * g[2];
  double th2 = T->theta2;
  if (T->leaf_theta && C->is_leaf && C->count > 0) {
    /* a smallest cell re-splits its candidates with its own opening angle */
    double th = T->leaf_theta[C->idx[0]];
    th2 = th * th;
  }
  int far = (th2 * D >= R);
  return !far;
}

/* Appendix, cell::createPartners. */
static void create_partners(tree* T, cell* c) {
  cellvec keep = {0};
  for (int64_t t = 0; t < c->partners.n; t++) {
    cell* A = c->partners.v[t];
    if (near_pair(T, A, c)) {
      if (!c->is_leaf) {
        for (int b = 0; b < 2; b++) {
          if (!c->child[b]) continue;
          for (int e = 0; e < 2; e++)
            if (A->child[e]) cv_push(&c->child[b]->partners, A->child[e]);
        }
      } else {
        cv_push(&c->near, A);
      }
      /* erased from Partners */
    } else {
      cv_push(&keep, A);
    }
  }
  free(c->partners.v);
  c->partners = keep;
  if (!c->is_leaf) {
    if (c->child[0] && c->child[1]) {
      cv_push(&c->child[0]->partners, c->child[1]);
      cv_push(&c->child[1]->partners, c->child[0]);
    }
    for (int b = 0; b < 2; b++)
      if (c->child[b]) create_partners(T, c->child[b]);
  } else {
    cv_push(&c->near, c);
  }
}

/* Appendix, cell::updateMoment. */
static void update_moment(tree* T, cell* c) {
  int side = T->p + 1;
  memset(c->Q, 0, sizeof(double) * side * side * side);
  if (!c->is_leaf) {
    for (int b = 0; b < 2; b++) {
      if (!c->child[b]) continue;
#pragma omp task if (c->level < 12) firstprivate(b)
      update_moment(T, c->child[b]);
    }
#pragma omp taskwait
    for (int b = 0; b < 2; b++) {
      cell* ch = c->child[b];
      if (!ch) continue;
      double cc[3] = {ch->center[0] - c->center[0], ch->center[1] - c->center[1],
                      ch->center[2] - c->center[2]};
      m2m(T->p, cc, ch->Q, c->Q);
    }
  } else if (c->count > 0) {
    for (int64_t t = 0; t < c->count; t++) {
      int64_t d = c->idx[t];
      double y[3] = {T->pos[3 * d] - c->center[0], T->pos[3 * d + 1] - c->center[1],
                     T->pos[3 * d + 2] - c->center[2]};
      p2m_one(T->p, y, &T->m[3 * d], c->Q);
    }
  }
}

/* Appendix, cell::updateField (returns the energy of the cell). */
static double update_field(tree* T, cell* c) {
  int side = T->p + 1;
  if (c->parent) {
    double cc[3] = {c->center[0] - c->parent->center[0], c->center[1] - c->parent->center[1],
                    c->center[2] - c->parent->center[2]};
    l2l(T->p, cc, c->parent->V, c->V);
  } else {
    memset(c->V, 0, sizeof(double) * side * side * side);
  }
  if (c->partners.n > 0) {
    double* D = (double*)malloc(sizeof(double) * CUBE(2 * T->p));
    for (int64_t t = 0; t < c->partners.n; t++) {
      cell* A = c->partners.v[t];
      double cc[3] = {c->center[0] - A->center[0], c->center[1] - A->center[1],
                      c->center[2] - A->center[2]};
      m2l(T->p, cc, A->Q, c->V, D, T->total);
    }
    free(D);
  }
  double energy = 0.0;
  if (!c->is_leaf) {
    double e[2] = {0.0, 0.0};
    for (int b = 0; b < 2; b++) {
      if (!c->child[b]) continue;
#pragma omp task if (c->level < 12) firstprivate(b) shared(e)
      e[b] = update_field(T, c->child[b]);
    }
#pragma omp taskwait
    energy = e[0] + e[1];
  } else {
    for (int64_t t = 0; t < c->count; t++) {
      int64_t d = c->idx[t];
      const double* x = &T->pos[3 * d];
      double y[3] = {x[0] - c->center[0], x[1] - c->center[1], x[2] - c->center[2]};
      double h[3];
      if (T->leaf_p) {
        /* the smallest cell's local expansion truncated at its own order */
        int pl = T->leaf_p[c->idx[0]];
        if (pl > T->p) pl = T->p;
        int side = T->p + 1;
        double* Vt = (double*)calloc((size_t)side * side * side, sizeof(double));
        for (int nx = 0; nx <= pl; nx++)
          for (int ny = 0; nx + ny <= pl; ny++)
            for (int nz = 0; nx + ny + nz <= pl; nz++) Vt[cidx(nx, ny, nz, T->p)] = c->V[cidx(nx, ny, nz, T->p)];
        l2p(T->p, Vt, y, h);
        free(Vt);
      } else {
        l2p(T->p, c->V, y, h);
      }
      for (int64_t u = 0; u < c->near.n; u++) {
        cell* A = c->near.v[u];
        for (int64_t s = 0; s < A->count; s++) {
          int64_t j = A->idx[s];
          pair_field(x, &T->pos[3 * j], &T->m[3 * j], h);
        }
      }
      T->H[3 * d] = h[0];
      T->H[3 * d + 1] = h[1];
      T->H[3 * d + 2] = h[2];
      energy += T->m[3 * d] * h[0] + T->m[3 * d + 1] * h[1] + T->m[3 * d + 2] * h[2];
    }
    energy = -0.5 * energy;
  }
  return energy;
}

static void count_lists(tree* T, cell* c) {
  T->m2l_pairs[c->level] += c->partners.n;
  if (c->is_leaf) T->p2p_leaf_pairs += c->near.n;
  for (int b = 0; b < 2; b++)
    if (c->child[b]) count_lists(T, c->child[b]);
}

static void free_tree(cell* c) {
  if (!c) return;
  free_tree(c->child[0]);
  free_tree(c->child[1]);
  free(c->idx);
  free(c->Q);
  free(c->V);
  free(c->partners.v);
  free(c->near.v);
  free(c);
}

static int check_params(int64_t n, const double* pos, const ccref_params* prm) {
  if (!prm || n < 1) return -1;
  if (prm->order < 1 || prm->order > CCREF_PMAX) return -1;
  if (!(prm->theta > 0.0 && prm->theta < 1.0)) return -1;
  if (prm->truncation != 0 && prm->truncation != 1) return -1;
  for (int64_t i = 0; i < 3 * n; i++)
    if (!isfinite(pos[i])) return -1;
  return 0;
}

static int setup_tree(tree* T, int64_t n, const double* pos, const ccref_params* prm, double* s_out) {
  memset(T, 0, sizeof(*T));
  T->p = prm->order;
  T->theta = prm->theta;
  T->theta2 = prm->theta * prm->theta;
  T->pos = pos;
  if (root_box(n, pos, prm, T->lo, T->W)) return -1;
  double s = prm->leaf_target > 0.0 ? prm->leaf_target : s_opt(prm->order);
  *s_out = s;
  T->L = choose_levels(T, n, s, prm->leaf_rule);
  split_sequence(T, T->L);
  return 0;
}

static void fill_shape(const tree* T, double s, ccref_stats* st) {
  st->levels = T->L;
  for (int l = 0; l <= CCREF_LMAX; l++) st->split_axis[l] = (l <= T->L) ? T->axis[l] : -1;
  for (int a = 0; a < 3; a++) {
    st->box_lo[a] = T->lo[a];
    st->box_hi[a] = T->lo[a] + T->W[a];
    st->leaf_side[a] = T->h[T->L][a];
  }
  st->s_used = s;
}

int ccref_tree_shape(int64_t n, const double* pos, const ccref_params* prm, ccref_stats* stats) {
  if (check_params(n, pos, prm) || !stats) return -1;
  tree T;
  double s;
  memset(stats, 0, sizeof(*stats));
  if (setup_tree(&T, n, pos, prm, &s)) return -1;
  fill_shape(&T, s, stats);
  return 0;
}

int ccref_fmm(int64_t n, const double* pos, const double* m, const ccref_params* prm, double* H,
              ccref_stats* stats) {
  return ccref_fmm_leaf(n, pos, m, prm, NULL, NULL, H, stats);
}

int ccref_fmm_leaf(int64_t n, const double* pos, const double* m, const ccref_params* prm, const int32_t* leaf_p,
                   const double* leaf_theta, double* H, ccref_stats* stats) {
  if (check_params(n, pos, prm)) return -1;
  for (int64_t i = 0; i < 3 * n; i++)
    if (!isfinite(m[i])) return -1;
  if (leaf_p)
    for (int64_t i = 0; i < n; i++)
      if (leaf_p[i] < 1 || leaf_p[i] > prm->order) return -1;
  if (leaf_theta)
    for (int64_t i = 0; i < n; i++)
      if (!(leaf_theta[i] > 0.0 && leaf_theta[i] < 1.0)) return -1;
  build_ftable();
  set_threads(prm->nthreads);
  tree T;
  double s;
  if (setup_tree(&T, n, pos, prm, &s)) return -1;
  T.m = m;
  T.H = H;
  T.leaf_p = leaf_p;
  T.leaf_theta = leaf_theta;
  T.total = prm->truncation == 1;

  double t0 = now_s();
  int64_t* leafc = (int64_t*)malloc(sizeof(int64_t) * 3 * n);
  for (int64_t i = 0; i < n; i++)
    for (int a = 0; a < 3; a++) leafc[3 * i + a] = leaf_coord(pos[3 * i + a], T.lo[a], T.W[a], T.k[T.L][a]);
  int64_t* all = (int64_t*)malloc(sizeof(int64_t) * n);
  for (int64_t i = 0; i < n; i++) all[i] = i;
  int64_t zero[3] = {0, 0, 0};
  cell* root = new_cell(&T, NULL, 0, zero);
  build(&T, root, all, n, leafc);
  free(leafc);
  double t1 = now_s();
  create_partners(&T, root);
  double t2 = now_s();
#pragma omp parallel
#pragma omp single
  update_moment(&T, root);
  double t3 = now_s();
#pragma omp parallel
#pragma omp single
  (void)update_field(&T, root);
  double t4 = now_s();

  if (stats) {
    memset(stats, 0, sizeof(*stats));
    fill_shape(&T, s, stats);
    count_lists(&T, root);
    stats->n_cells = T.ncells;
    stats->n_leaves = T.nleaves;
    int64_t tot = 0;
    for (int l = 0; l <= CCREF_LMAX; l++) {
      stats->m2l_pairs_per_level[l] = T.m2l_pairs[l];
      tot += T.m2l_pairs[l];
    }
    stats->n_m2l_pairs = tot;
    stats->n_p2p_leaf_pairs = T.p2p_leaf_pairs;
    stats->t_build = t1 - t0;
    stats->t_partners = t2 - t1;
    stats->t_upward = t3 - t2;
    stats->t_downward = t4 - t3;
  }
  free_tree(root);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Selector MLP reference (FP64): 8 -> h1 -> h2 -> out with ReLU hidden      */
/* layers, masked squared-error loss.  Not from the paper (the learned       */
/* selector extends its parameter study of Sec. 4).                          */
/* ------------------------------------------------------------------------- */
static void mlp_offsets(int in, int h1, int h2, int out, int64_t off[6]) {
  off[0] = 0;                       /* W1 [h1][in] */
  off[1] = off[0] + (int64_t)h1 * in; /* b1 */
  off[2] = off[1] + h1;               /* W2 [h2][h1] */
  off[3] = off[2] + (int64_t)h2 * h1; /* b2 */
  off[4] = off[3] + h2;               /* W3 [out][h2] */
  off[5] = off[4] + (int64_t)out * h2; /* b3 */
}

static void mlp_row(int in, int h1, int h2, int out, const double* P, const int64_t* off,
                    const double* x, double* a1, double* a2, double* y) {
  for (int j = 0; j < h1; j++) {
    double s = P[off[1] + j];
    for (int i = 0; i < in; i++) s += P[off[0] + (int64_t)j * in + i] * x[i];
    a1[j] = s > 0.0 ? s : 0.0;
  }
  for (int j = 0; j < h2; j++) {
    double s = P[off[3] + j];
    for (int i = 0; i < h1; i++) s += P[off[2] + (int64_t)j * h1 + i] * a1[i];
    a2[j] = s > 0.0 ? s : 0.0;
  }
  for (int o = 0; o < out; o++) {
    double s = P[off[5] + o];
    for (int i = 0; i < h2; i++) s += P[off[4] + (int64_t)o * h2 + i] * a2[i];
    y[o] = s;
  }
}

int ccref_mlp_forward(int32_t in, int32_t h1, int32_t h2, int32_t out, const double* params,
                      int64_t rows, const double* x, double* y) {
  if (in < 1 || h1 < 1 || h2 < 1 || out < 1 || rows < 0) return -1;
  int64_t off[6];
  mlp_offsets(in, h1, h2, out, off);
  double* a1 = (double*)malloc(sizeof(double) * h1);
  double* a2 = (double*)malloc(sizeof(double) * h2);
  for (int64_t r = 0; r < rows; r++) mlp_row(in, h1, h2, out, params, off, &x[r * in], a1, a2, &y[r * out]);
  free(a1);
  free(a2);
  return 0;
}

double ccref_mlp_loss_grad(int32_t in, int32_t h1, int32_t h2, int32_t out, const double* params,
                           int64_t rows, const double* x, const double* t, const double* mask,
                           double* grads) {
  int64_t off[6];
  mlp_offsets(in, h1, h2, out, off);
  int64_t np = off[5] + out;
  if (grads) memset(grads, 0, sizeof(double) * np);
  double msum = 0.0;
  for (int64_t i = 0; i < rows * out; i++) msum += mask[i];
  double norm = msum > 1.0 ? msum : 1.0;
  double* a1 = (double*)malloc(sizeof(double) * h1);
  double* a2 = (double*)malloc(sizeof(double) * h2);
  double* y = (double*)malloc(sizeof(double) * out);
  double* dy = (double*)malloc(sizeof(double) * out);
  double* d2 = (double*)malloc(sizeof(double) * h2);
  double* d1 = (double*)malloc(sizeof(double) * h1);
  double loss = 0.0;
  for (int64_t r = 0; r < rows; r++) {
    const double* xr = &x[r * in];
    mlp_row(in, h1, h2, out, params, off, xr, a1, a2, y);
    for (int o = 0; o < out; o++) {
      double e = y[o] - t[r * out + o];
      double w = mask[r * out + o];
      loss += 0.5 * w * e * e;
      dy[o] = w * e / norm;
    }
    if (!grads) continue;
    for (int o = 0; o < out; o++) {
      grads[off[5] + o] += dy[o];
      for (int i = 0; i < h2; i++) grads[off[4] + (int64_t)o * h2 + i] += dy[o] * a2[i];
    }
    for (int i = 0; i < h2; i++) {
      double s = 0.0;
      for (int o = 0; o < out; o++) s += params[off[4] + (int64_t)o * h2 + i] * dy[o];
      d2[i] = a2[i] > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < h2; j++) {
      grads[off[3] + j] += d2[j];
      for (int i = 0; i < h1; i++) grads[off[2] + (int64_t)j * h1 + i] += d2[j] * a1[i];
    }
    for (int i = 0; i < h1; i++) {
      double s = 0.0;
      for (int j = 0; j < h2; j++) s += params[off[2] + (int64_t)j * h1 + i] * d2[j];
      d1[i] = a1[i] > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < h1; j++) {
      grads[off[1] + j] += d1[j];
      for (int i = 0; i < in; i++) grads[off[0] + (int64_t)j * in + i] += d1[j] * xr[i];
    }
  }
  free(a1);
  free(a2);
  free(y);
  free(dy);
  free(d2);
  free(d1);
  return loss / norm;
}
