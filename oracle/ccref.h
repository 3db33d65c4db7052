/*
 * ccref.h -- CPU oracle for the Cartesian fast multipole method for point
 * dipoles (Zhang & Haas, "Adaptation and Performance of the Cartesian
 * Coordinates Fast Multipole Method for Nanomagnetic Simulations").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, FP64 reference
 * that the GPU path is checked against.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Units: mu0/4pi = 1.  Layouts: positions, moments and fields are [n][3]
 * (x, y, z per dipole, row-major), FP64, caller-owned host memory.
 * Every call returns 0 on success and a negative value on invalid input.
 *
 * Expansion storage used by the introspection calls: a dense cube indexed
 * [nx][ny][nz] with nx, ny, nz in 0..K (K = order for Q and V, 2*order for D),
 * i.e. element (nx, ny, nz) sits at ((nx*(K+1)) + ny)*(K+1) + nz; entries with
 * nx+ny+nz > K are zero.
 */
#ifndef CCREF_H
#define CCREF_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define CCREF_PMAX 8
#define CCREF_LMAX 24

typedef struct {
  int32_t order;        /* p_m >= 1, multipole and local truncation order (Sec. 3) */
  double theta;         /* alpha_m in (0,1): a cell pair is near iff 2r/d > theta (Sec. 2) */
  double leaf_target;   /* s > 0; <= 0 selects s_o(p) of Eq.(so) */
  int32_t leaf_rule;    /* 0: L = argmin |N/2^L - s|; 1: mean over non-empty leaves */
  int32_t has_box;      /* 1: root cell is [box_lo, box_hi]; 0: bounding box */
  double box_lo[3], box_hi[3];
  int32_t nthreads;     /* OpenMP threads (<= 0: library default) */
  int32_t truncation;   /* 0: multipoles and locals each to order p (the reading of Sec. 3);
                           1: total degree, only terms with |n| + |q| <= p in M2L */
} ccref_params;

typedef struct {
  int32_t levels;                 /* L: number of bisection levels */
  int32_t split_axis[CCREF_LMAX + 1];  /* axis split when going from level l-1 to l (index l) */
  double box_lo[3], box_hi[3];    /* root cell used */
  double leaf_side[3];            /* smallest-cell sides */
  double s_used;                  /* target s after defaulting */
  int64_t n_cells;                /* cells created (empty cells pruned) */
  int64_t n_leaves;               /* non-empty smallest cells */
  int64_t n_m2l_pairs;            /* sum over cells of |Partners| after createPartners */
  int64_t n_p2p_leaf_pairs;       /* sum over leaves of |NearPartners| (self included) */
  int64_t m2l_pairs_per_level[CCREF_LMAX + 1];
  double t_build, t_partners, t_upward, t_downward;   /* seconds */
} ccref_stats;

/* O(N^2) dipole field, FP64, j-ascending summation; pairs with r = 0 skipped. */
int ccref_bruteforce(int64_t n, const double* pos, const double* m, double* H, int32_t nthreads);
/* Same, at the nt targets idx[0..nt) only; H is [nt][3]. */
int ccref_bruteforce_targets(int64_t n, const double* pos, const double* m, int64_t nt,
                             const int64_t* idx, double* H, int32_t nthreads);
/* The paper's recursive FMM (three passes); H is [n][3] in input order. stats may be NULL. */
int ccref_fmm(int64_t n, const double* pos, const double* m, const ccref_params* prm, double* H,
              ccref_stats* stats);
/* Same with per-smallest-cell parameters, given per dipole (every dipole of a
 * smallest cell carries its cell's values; NULL = the fixed parameters):
 * leaf_p in 1..order truncates the cell's local expansion before L2P, and
 * leaf_theta in (0,1) is the opening angle with which the cell re-splits its
 * own candidates into near and far cells (the levels above keep theta). */
int ccref_fmm_leaf(int64_t n, const double* pos, const double* m, const ccref_params* prm,
                   const int32_t* leaf_p, const double* leaf_theta, double* H, ccref_stats* stats);
/* Level count and split sequence only (the rule of Sec. 4); fills stats->levels, split_axis,
 * box, leaf_side, s_used.  No lists are built. */
int ccref_tree_shape(int64_t n, const double* pos, const ccref_params* prm, ccref_stats* stats);
/* E = -1/2 sum_i m_i . H_i (Appendix, energy with the double-counting factor). */
double ccref_energy(int64_t n, const double* m, const double* H);

/* ---- introspection of single operators, expansions in the dense cube layout ---- */
/* F-table entry F_k(q) (Eqs. Dn, Dnr); returns 0 if |q| != |k| or q outside the table. */
double ccref_ftable(int32_t kx, int32_t ky, int32_t kz, int32_t qx, int32_t qy, int32_t qz);
/* D_k(c) for |k| <= K, dense cube of side K+1. */
int ccref_dtensor(int32_t K, const double c[3], double* D);
/* Multipole moments of dipoles about center, Eq.(multipolemoments), |n| <= p. */
int ccref_p2m(int32_t p, const double center[3], int64_t n, const double* pos, const double* m,
              double* Q);
/* Charge moments Q_n = (1/n!) sum q_i r_i^n about center (Sec. 3), |n| <= p. */
int ccref_charge_moments(int32_t p, const double center[3], int64_t n, const double* pos,
                         const double* q, double* Q);
/* Eq.(momentshift): Qparent += shift of Qchild, c = child center - parent center. */
int ccref_m2m(int32_t p, const double c[3], const double* Qchild, double* Qparent);
/* Eq.(taylorshift): Vchild = shift of Vparent, c = child center - parent center. */
int ccref_l2l(int32_t p, const double c[3], const double* Vparent, double* Vchild);
/* Eq.(taylorcalc): V += M2L(Q), c = target center - source center. */
int ccref_m2l(int32_t p, const double c[3], const double* Q, double* V);
/* The same keeping only the terms of total degree |n| + |q| <= p. */
int ccref_m2l_total(int32_t p, const double c[3], const double* Q, double* V);
/* Eq.(H) with H = -grad V: field at offset y from the expansion center. */
int ccref_l2p(int32_t p, const double* V, const double y[3], double H[3]);
/* Potential of a multipole expansion at x (relative to its center), Eq.(Vm): sum_n D_n(x) Q_n. */
double ccref_multipole_potential(int32_t p, const double* Q, const double x[3]);
/* Local expansion value sum_n V_n y^n / n! (Eq. taylorexpansion). */
double ccref_local_potential(int32_t p, const double* V, const double y[3]);

/* ---- selector MLP reference (FP64): 8 -> H1 -> H2 -> O, ReLU hidden ----
 * Weights are row-major W1[H1][IN], b1[H1], W2[H2][H1], b2[H2], W3[O][H2], b3[O].
 * Loss = mean over rows of 0.5*sum_o mask[o]*(y[o]-t[o])^2 / max(1, sum mask).
 * grads has the same layout as the packed parameter vector. */
int ccref_mlp_forward(int32_t in, int32_t h1, int32_t h2, int32_t out, const double* params,
                      int64_t rows, const double* x, double* y);
double ccref_mlp_loss_grad(int32_t in, int32_t h1, int32_t h2, int32_t out, const double* params,
                           int64_t rows, const double* x, const double* t, const double* mask,
                           double* grads);

#ifdef __cplusplus
}
#endif
#endif
