/* Exercises the oracle's entry points on small inputs so that the address and
 * undefined-behaviour sanitizers see every code path the CPU tests use:
 * direct sums, the recursive FMM (both leaf rules, both truncations, orders
 * 1..8, a caller box, per-cell parameters), the expansion helpers, the
 * network reference and the refusals of invalid input.  Exit status 0 when
 * every call returned what it should. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/ccref.h"

static unsigned long long g_state = 88172645463325252ull;
static double uni(void) { /* xorshift64 */
  g_state ^= g_state << 13;
  g_state ^= g_state >> 7;
  g_state ^= g_state << 17;
  return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}

static int g_bad = 0;
#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      g_bad++;                                                \
    }                                                         \
  } while (0)

static void defaults(ccref_params* p, int order, double theta) {
  memset(p, 0, sizeof(*p));
  p->order = order;
  p->theta = theta;
  p->leaf_target = 0.0;
  p->nthreads = 2;
}

int main(void) {
  enum { N = 700 };
  double* pos = malloc(sizeof(double) * 3 * N);
  double* m = malloc(sizeof(double) * 3 * N);
  double* H = malloc(sizeof(double) * 3 * N);
  double* H2 = malloc(sizeof(double) * 3 * N);
  for (int i = 0; i < N; i++) {
    for (int a = 0; a < 3; a++) {
      pos[3 * i + a] = (a == 2 ? 4.0 : 10.0) * uni();
      m[3 * i + a] = uni() - 0.5;
    }
  }
  memcpy(pos + 3 * 5, pos, 3 * sizeof(double)); /* a coincident pair */
  CHECK(ccref_bruteforce(N, pos, m, H, 2) == 0);
  int64_t idx[7] = {0, 5, 17, 100, 333, 512, N - 1};
  double Ht[21];
  CHECK(ccref_bruteforce_targets(N, pos, m, 7, idx, Ht, 2) == 0);
  CHECK(fabs(Ht[3] - H[15]) <= 1e-12 * (1.0 + fabs(H[15])));
  ccref_params prm;
  ccref_stats st;
  for (int order = 1; order <= CCREF_PMAX; order++) {
    for (int rule = 0; rule < 2; rule++) {
      for (int trunc = 0; trunc < 2; trunc++) {
        defaults(&prm, order, 0.5);
        prm.leaf_rule = rule;
        prm.truncation = trunc;
        prm.leaf_target = 6.0;
        CHECK(ccref_fmm(N, pos, m, &prm, H2, &st) == 0);
        CHECK(st.levels >= 1 && st.n_leaves >= 1);
      }
    }
  }
  defaults(&prm, 6, 0.4);
  prm.has_box = 1;
  for (int a = 0; a < 3; a++) {
    prm.box_lo[a] = -0.5;
    prm.box_hi[a] = a == 2 ? 4.5 : 10.5;
  }
  CHECK(ccref_fmm(N, pos, m, &prm, H2, &st) == 0);
  CHECK(ccref_tree_shape(N, pos, &prm, &st) == 0);
  int32_t* lp = malloc(sizeof(int32_t) * N);
  double* lt = malloc(sizeof(double) * N);
  for (int i = 0; i < N; i++) {
    lp[i] = 2 + (i % 5);
    lt[i] = 0.3 + 0.1 * (i % 5);
  }
  CHECK(ccref_fmm_leaf(N, pos, m, &prm, lp, lt, H2, &st) == 0);
  (void)ccref_energy(N, m, H2);
  /* expansion helpers at the highest order */
  const int P = CCREF_PMAX;
  const int NC = (P + 1) * (P + 1) * (P + 1);
  double* Q = calloc(NC, sizeof(double));
  double* Q2 = calloc(NC, sizeof(double));
  double* V = calloc(NC, sizeof(double));
  double* V2 = calloc(NC, sizeof(double));
  double* D = calloc((2 * P + 1) * (2 * P + 1) * (2 * P + 1), sizeof(double));
  const double c0[3] = {0.1, -0.2, 0.3}, far[3] = {7.0, 5.0, -6.0}, y[3] = {0.05, 0.1, -0.07};
  double h3[3];
  CHECK(ccref_p2m(P, c0, 20, pos, m, Q) == 0);
  CHECK(ccref_charge_moments(P, c0, 20, pos, m, Q2) == 0);
  CHECK(ccref_m2m(P, c0, Q, Q2) == 0);
  CHECK(ccref_m2l(P, far, Q, V) == 0);
  CHECK(ccref_m2l_total(P, far, Q, V2) == 0);
  CHECK(ccref_l2l(P, c0, V, V2) == 0);
  CHECK(ccref_l2p(P, V, y, h3) == 0);
  CHECK(ccref_dtensor(2 * P, far, D) == 0);
  (void)ccref_ftable(2, 1, 0, 2, 1, 0);
  (void)ccref_multipole_potential(P, Q, far);
  (void)ccref_local_potential(P, V, y);
  /* the network reference */
  const int in = 8, h1 = 16, h2 = 16, out = 5, rows = 9;
  const int np = h1 * in + h1 + h2 * h1 + h2 + out * h2 + out;
  double* w = malloc(sizeof(double) * np);
  double* g = malloc(sizeof(double) * np);
  double* x = malloc(sizeof(double) * rows * in);
  double* t = malloc(sizeof(double) * rows * out);
  double* mk = malloc(sizeof(double) * rows * out);
  double* yo = malloc(sizeof(double) * rows * out);
  for (int i = 0; i < np; i++) w[i] = uni() - 0.5;
  for (int i = 0; i < rows * in; i++) x[i] = uni();
  for (int i = 0; i < rows * out; i++) {
    t[i] = uni();
    mk[i] = uni() < 0.7 ? 1.0 : 0.0;
  }
  CHECK(ccref_mlp_forward(in, h1, h2, out, w, rows, x, yo) == 0);
  (void)ccref_mlp_loss_grad(in, h1, h2, out, w, rows, x, t, mk, g);
  /* refusals */
  defaults(&prm, 4, 1.0);
  CHECK(ccref_fmm(N, pos, m, &prm, H2, &st) != 0);
  defaults(&prm, 0, 0.5);
  CHECK(ccref_fmm(N, pos, m, &prm, H2, &st) != 0);
  defaults(&prm, 4, 0.5);
  CHECK(ccref_fmm(0, pos, m, &prm, H2, &st) != 0);
  pos[7] = NAN;
  CHECK(ccref_fmm(N, pos, m, &prm, H2, &st) != 0);
  free(pos), free(m), free(H), free(H2), free(lp), free(lt), free(Q), free(Q2), free(V), free(V2), free(D);
  free(w), free(g), free(x), free(t), free(mk), free(yo);
  if (g_bad) return 1;
  printf("oracle driver OK\n");
  return 0;
}
