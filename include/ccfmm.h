/*
 * ccfmm.h -- C ABI of the MI355X (gfx950) Cartesian fast multipole method for
 * point-dipole fields (Zhang & Haas, "Adaptation and Performance of the
 * Cartesian Coordinates Fast Multipole Method for Nanomagnetic Simulations").
 *
 * Problem (Sec. 1-3 of the paper): given point dipoles m_i at positions r_i
 * under open boundaries, return the dipolar field at every dipole,
 *     H_i = sum_{j : r_j != r_i} (3 (m_j . u) u - m_j) / |r_i - r_j|^3,
 *     u = (r_i - r_j) / |r_i - r_j|,   in units mu0/4pi = 1,
 * approximated by the Cartesian FMM with expansion order p (p_m), opening
 * angle theta (alpha_m) and target dipoles per smallest cell s.
 *
 * Conventions shared by every entry point:
 *  - Every function returns int: CCFMM_OK (0), a negative error, or a positive
 *    warning.  No C++ exception, longjmp or abort crosses the ABI.  Details of
 *    the last error of the calling thread are in ccfmm_last_error().
 *  - Positions are [n][3] FP64 (x, y, z per dipole).  Moments and fields are
 *    [nbatch][n][3] FP64: nbatch magnetisation configurations on one geometry.
 *    Fields come back in the caller's dipole order.
 *  - The caller owns every buffer it passes, host or device; the library never
 *    keeps a caller pointer after the call returns.  The library owns the
 *    plan's device memory; ccfmm_plan_destroy frees it.
 *  - Host-pointer calls are synchronous.  Device-pointer calls are ordered on
 *    the given HIP stream (hipStream_t passed as void*, NULL = default stream)
 *    and return before the GPU work ends.
 *  - A plan is not thread-safe: one call at a time per plan.
 */
#ifndef CCFMM_H
#define CCFMM_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define CCFMM_PMAX 8   /* highest expansion order supported */
#define CCFMM_LMAX 24  /* deepest bisection tree supported */

/* status codes */
#define CCFMM_OK 0
#define CCFMM_EINVAL (-1)     /* invalid argument (sizes, NaN/inf, theta, order, box) */
#define CCFMM_ENOMEM (-2)     /* device or host allocation failed; the plan stays destroyable */
#define CCFMM_EHIP (-3)       /* HIP runtime error (message in ccfmm_last_error) */
#define CCFMM_ESTATE (-4)     /* call not valid in the plan's state */
#define CCFMM_W_FALLBACK 1    /* learned selector rejected, fixed-parameter result returned */
#define CCFMM_W_NOWEIGHTS 2   /* selector weights file missing: nothing loaded, fixed parameters kept */

#define CCFMM_PREC_FP64 0     /* every pass in FP64 */
#define CCFMM_PREC_MIXED 1    /* FP32 bulk arithmetic; FP64 derivative tensors and final sums */

typedef struct ccfmm_plan_s* ccfmm_plan;

/* Parameters (Sec. 2-4).  Fill with ccfmm_params_default, then override. */
typedef struct {
  int32_t order;        /* p_m: multipole and local truncation order, 1..CCFMM_PMAX (Sec. 3) */
  double theta;         /* alpha_m in (0,1): a cell pair is near iff 2r/d > theta (Sec. 2);
                           a pair with 2r/d == theta is far */
  double leaf_target;   /* s, dipoles per smallest cell; <= 0 selects Eq.(so):
                           s_o = 0.74 p^2 for p > 3, else 8 */
  int32_t leaf_rule;    /* 0: levels L = argmin_L |N/2^L - s| (Sec. 4);
                           1: same with N/2^L replaced by the mean over occupied cells */
  int32_t precision;    /* CCFMM_PREC_FP64 or CCFMM_PREC_MIXED */
  int32_t selector;     /* 0: fixed (order, theta) everywhere.  1: learned per smallest cell:
                           once the plan holds selector weights (ccfmm_selector_load / _set),
                           the first evaluation after the plan is built, or after a position
                           update that changed the occupied cells, chooses (p, theta) per cell
                           from that call's moments, has the fixed-parameter FMM judge the
                           choice against err_bound and keeps it, or falls back to the fixed
                           parameters (that call returns CCFMM_W_FALLBACK).  Needs order >= 2.
                           Without weights the plan evaluates with the fixed parameters. */
  double err_bound;     /* selector = 1: bound on the relative RMS difference between the
                           learned and the fixed-parameter field (e.g. 1e-5), > 0 */
  int32_t has_box;      /* 1: root cell is [box_lo, box_hi]; 0: tight bounding box */
  double box_lo[3], box_hi[3];
  int32_t max_batch;    /* largest nbatch the plan will evaluate (device buffers sized) */
  int32_t m2l_class_bits; /* M2L target ordering: cells grouped by their low key bits
                             (position inside their ancestors) before tiling; 0..12 */
  int32_t m2l_variant;    /* M2L kernel: -1 (default) = chosen at plan creation: 4 where the
                             order, precision and form allow it, else 0; 0 = block of 4
                             wavefronts sharing one operator per
                             step (64-column tiles), 1 = independent wavefronts (16 columns,
                             orders <= 6), 2 / 3 / 4 = wide blocks with a double-buffered
                             operator (256 / 128 / 64 columns; orders <= 8 with m2l_traceless,
                             FP64 included; mixed precision only and orders <= 6 without).
                             A variant the order or precision cannot use falls back to 0;
                             ccfmm_plan_autotune can choose.  With per-cell orders, the
                             wide traceless kernels compute for a tile of smallest cells
                             only the local rows of the largest order among its targets */
  int32_t use_graph;      /* 1: evaluations are captured once into a HIP graph (per batch size
                             and buffer pair) and replayed; 0: plain stream launches */
  int32_t overlap_near;   /* 1 (default): the near field runs on a plan-owned second stream
                             (default priority) beside P2M..L2L, joined before L2P;
                             0: everything on the caller's stream, near field and L2P fused.
                             ccfmm_plan_autotune times both and keeps the faster */
  int32_t keep_lists;     /* 1 (default): a position update with the same geometry and the same
                             occupied cells keeps the cell lists, M2L tiles and captured
                             evaluation (exactly what a full rebuild would produce);
                             0: every update rebuilds everything */
  int32_t truncation;     /* 0 (default): multipoles and locals each to order p, M2L with D up to
                             order 2p (the reading of Sec. 3); 1: total degree, M2L keeps only the
                             terms with |n| + |q| <= p (D_k = 0 for |k| > p) */
  int32_t m2l_traceless;  /* 1 (default): the wide M2L kernels (mixed and FP64) contract folded
                             moments over their 2l+1 components per degree and fill the rest of
                             V from the Laplace equation (D and V are harmonic; the same sums,
                             rounded differently; on one stream M2M folds the moments and L2L
                             completes the local rows as they shift); 0: the full 83 x 84
                             operator at p = 6 */
  double sel_margin;      /* selector = 1: the choice keeps the predicted global relative RMS
                             error within err_bound x 10^-sel_margin (default 0.3, >= 0);
                             see ccfmm_plan_select */
  double sel_cost_far;    /* selector = 1: cost of one far cell relative to one direct dipole
                             pair in the selection; <= 0 (default): measured on the plan (M2L and
                             near-field times of one evaluation, each pass alone) */
  int64_t device_mem_cap; /* bytes of device memory the plan may hold (its buffers and the
                             temporaries of its calls); 0 (default): no cap.  A call that would
                             pass it fails with CCFMM_ENOMEM; the plan stays destroyable, and
                             after a failed evaluation it evaluates again at sizes that fit */
} ccfmm_params;

/* One timed M2L configuration of ccfmm_plan_autotune. */
typedef struct {
  int32_t variant, class_bits;
  double m2l_ms;   /* median of the timed launches */
  int64_t steps;   /* MFMA operator steps of the tiling */
} ccfmm_tune_entry;

/* Plan summary (counts are exact properties of the tree and lists). */
typedef struct {
  int64_t n;
  int32_t order, levels, precision, max_batch;
  int32_t split_axis[CCFMM_LMAX + 1];   /* axis halved going to level l (index l >= 1) */
  double box_lo[3], box_hi[3], leaf_side[3];
  double s_used;
  int64_t n_leaves;                     /* occupied smallest cells */
  int64_t n_cells;                      /* occupied cells, all levels */
  int64_t n_m2l_pairs;                  /* far (M2L) cell pairs, all levels */
  int64_t m2l_pairs_per_level[CCFMM_LMAX + 1];
  int64_t n_p2p_leaf_pairs;             /* near (P2P) leaf pairs, self included */
  int64_t n_p2p_pairs;                  /* dipole pairs evaluated directly */
  int64_t n_m2l_tiles, n_m2l_steps;     /* MFMA work units of the M2L pass */
  int64_t n_delta;                      /* distinct cell offsets with an M2L operator */
  int32_t m2l_class_bits;
  int32_t fallback;                     /* learned mode fell back to fixed parameters */
  double m2l_flops_per_config;          /* algorithmic: 2 * (N(p)-1)^2 * M2L pairs */
  double p2p_pairs_per_config;
  int32_t m2l_variant;                  /* kernel in use (see ccfmm_params) */
  int64_t n_rebuilds_kept;              /* position updates that kept the cell lists, M2L tiles and the
                                           captured evaluation's structure: same geometry and the same
                                           occupied cells at every level (only the dipoles moved) */
  int32_t learned;                      /* per-cell parameters of the learned selector in use */
  double judge_err;                     /* the judge's relative RMS difference at the last selection */
  double sel_cost_far;                  /* far-cell cost used at the last selection */
  int64_t device_bytes;                 /* device memory the plan holds now */
  int32_t overlap_near;                 /* evaluation form in use (see ccfmm_params; the autotuner chooses) */
  double tune_eval_ms[2];               /* the last autotune's evaluation times: [0] near field beside the
                                           expansion passes, [1] one stream; 0 before any autotune */
} ccfmm_info;

/* Per-pass device times (milliseconds) of one evaluation, from HIP events.
 * p2m includes the moment permutation; p2p is the near field (on the plan's
 * side stream when overlap_near is on, so it overlaps m2m..l2l); l2p adds the
 * smooth field (0 when fused into p2p); total spans the whole evaluation. */
typedef struct {
  double p2m, m2m, m2l, l2l, p2p, l2p, total;
} ccfmm_pass_times;

const char* ccfmm_status_string(int status);
/* Message of the last failing call on this thread ("" if none). */
const char* ccfmm_last_error(void);
int ccfmm_params_default(ccfmm_params* prm);

/* Build the plan: tree by recursive halving (Sec. 2, level rule of Sec. 4),
 * near/far lists by the opening angle (Sec. 2, Appendix createPartners),
 * derivative tensors (Eqs. Dn, Dnr) and the M2L work tiles.
 *  pos: host [n][3] FP64, copied.  device: HIP device ordinal.
 * Errors: EINVAL (n < 1, non-finite positions, order/theta/box invalid, a point
 * outside a caller box), ENOMEM, EHIP.  On error *out is NULL. */
int ccfmm_plan_create(ccfmm_plan* out, int32_t device, int64_t n, const double* pos,
                      const ccfmm_params* prm);
/* Same from device positions d_pos [n][3] FP64 on the current device, ordered
 * on stream (the call synchronises the stream once to size the lists). */
int ccfmm_plan_create_device(ccfmm_plan* out, int64_t n, const double* d_pos,
                             const ccfmm_params* prm, void* stream);
/* Rebuild tree, lists and tensors in place for new device positions of the
 * same count (moving dipoles); buffers are reused when large enough.  With
 * keep_lists, an update that leaves the geometry and the occupied cells as
 * they were keeps the lists, tiles and captured evaluation.  With a caller
 * box, the positions are checked against it on the device (CCFMM_EINVAL for a
 * non-finite coordinate or a dipole outside).  After a failed update the plan
 * evaluates nothing (CCFMM_ESTATE) until an update succeeds, which then
 * rebuilds everything. */
int ccfmm_plan_update_positions_device(ccfmm_plan plan, const double* d_pos, void* stream);

/* Evaluate H for nbatch configurations (1 <= nbatch <= max_batch).
 * Host version: m and H are host [nbatch][n][3]; synchronous.
 * Device version: d_m and d_H are device [nbatch][n][3], stream-ordered.
 * Passes: P2M Eq.(multipolemoments), M2M Eq.(momentshift), M2L Eq.(taylorcalc),
 * L2L Eq.(taylorshift), L2P Eq.(H) and the near-field sum Eq.(H2). */
int ccfmm_eval(ccfmm_plan plan, int32_t nbatch, const double* m, double* H);
int ccfmm_eval_device(ccfmm_plan plan, int32_t nbatch, const double* d_m, double* d_H, void* stream);
/* As ccfmm_eval_device, with HIP events between the passes (synchronises).
 * The passes run one after another on the caller's stream whatever the
 * plan's overlap_near, so each time is that pass alone (M2M and L2L in their
 * single-stream form, with the moment fold and the completion of the local
 * rows of the traceless M2L inside them); below the batched size the near
 * field and L2P are one fused kernel (timed as p2p, l2p 0). */
int ccfmm_eval_device_timed(ccfmm_plan plan, int32_t nbatch, const double* d_m, double* d_H,
                            void* stream, ccfmm_pass_times* times);

/* M2L autotuner: times every (kernel variant, class bits) combination on this
 * plan's tiles for nbatch configurations of the device moments d_m (d_H is a
 * scratch field buffer of the same shape), keeps the fastest in the plan and
 * writes up to max_out timings to out (*n_out = number written): the median of
 * three launches, or a single launch for a combination whose first launch took
 * more than twice the best median so far.  Then it times whole evaluations in
 * both forms (near field beside the expansion passes, and everything on one
 * stream; per evaluation, the better of two runs of four queued back to back,
 * replayed from a graph when the plan uses graphs) and keeps the faster as the
 * plan's overlap_near (reported with both times in ccfmm_plan_info).
 * Synchronises the stream.  The field values do not depend on the choices
 * (beyond rounding). */
int ccfmm_plan_autotune(ccfmm_plan plan, int32_t nbatch, const double* d_m, double* d_H, void* stream,
                        ccfmm_tune_entry* out, int32_t max_out, int32_t* n_out);

int ccfmm_plan_info(ccfmm_plan plan, ccfmm_info* out);
/* Energy E_b = -1/2 sum_i m_i . H_i per configuration (Sec. 3 and Appendix),
 * host arrays; E is [nbatch]. */
int ccfmm_energy(int64_t n, int32_t nbatch, const double* m, const double* H, double* E);
/* The same energy on the GPU for device arrays d_m and d_H of the plan's n
 * dipoles, [nbatch][n][3] each (any order of the dipoles, the same in both);
 * d_E is [nbatch] FP64, caller-owned.  FP64 sums in an order that depends on n
 * only (the same result on every call).  Stream-ordered; the partial sums live
 * in a plan-owned buffer (allocated on the first call for a larger nbatch), so
 * calls on one plan must not overlap. */
int ccfmm_plan_energy_device(ccfmm_plan plan, int32_t nbatch, const double* d_m, const double* d_H, double* d_E,
                             void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the energy
 * of ccfmm_plan_energy_device with no plan and no allocation.  d_m, d_H:
 * device [nbatch][n][3] FP64 (caller-owned, any dipole order, the same in
 * both); d_E: device [nbatch] FP64.  Runs on the calling thread's current
 * device, ordered on stream; same kernels and summation order as
 * ccfmm_plan_energy_device (bitwise the same result).  The partial sums live
 * in a fixed library array of CCFMM_NOALLOC_MAX_BATCH x 256 doubles (8 MiB)
 * that every GPU the library runs on holds until the process ends.  Errors:
 * EINVAL for n < 1, NULL pointers or nbatch outside 1..CCFMM_NOALLOC_MAX_BATCH
 * (checked before any device call).  Calls that overlap on one GPU share the
 * array and race: order them on one stream. */
#define CCFMM_NOALLOC_MAX_BATCH 4096
int ccfmm_energy_device_noalloc(int64_t n, int32_t nbatch, const double* d_m, const double* d_H, double* d_E,
                                void* stream);
/* NULL-safe. */
void ccfmm_plan_destroy(ccfmm_plan plan);

/* ---------------------------------------------------------------------------
 * Per-smallest-cell parameters and the learned selector.
 *
 * Extends the paper's parameter choice (Sec. 4: one (p_m, alpha_m) for the
 * whole system, chosen from timings and the estimate [alpha/(2-alpha)]^p) to a
 * choice per smallest cell.  The levels above the smallest cells keep the
 * plan's (order, theta).  A smallest cell with its own theta_l re-splits its
 * own candidates (children of the cells near its parent) into near and far
 * cells by 2r/d > theta_l; its own p_l <= order truncates its local expansion
 * before L2P.  Cells are in "compact leaf order": occupied smallest cells by
 * increasing bisection key (ccfmm_plan_leaf_ids gives each dipole's cell).
 * ------------------------------------------------------------------------- */
#define CCFMM_MLP_IN 8       /* features per cell */
#define CCFMM_MLP_HIDDEN 64  /* two hidden layers of this width, ReLU */
#define CCFMM_MLP_OUT 25     /* predicted log10 error for p in {2..6} x theta in {.3,.4,.5,.6,.7},
                                output index (p-2)*5 + theta index */
/* number of packed FP32 parameters: W1[64][8] b1[64] W2[64][64] b2[64] W3[25][64] b3[25] */
#define CCFMM_MLP_PARAMS (64 * 8 + 64 + 64 * 64 + 64 + 25 * 64 + 25)

typedef struct {
  int32_t n_leaves;
  int32_t hist[CCFMM_MLP_OUT];  /* cells per chosen (p, theta), index as the network output */
  double judge_err;             /* relative RMS of the learned vs the fixed-parameter field */
  int32_t fallback;             /* 1: learned choice rejected, plan back on fixed parameters */
  double pred_err;              /* the network's prediction of the chosen field's relative RMS error */
} ccfmm_select_info;

/* Set (d_p, d_theta: device arrays of n_leaves int32 / FP64, compact leaf
 * order) or clear (both NULL) the per-cell parameters; rebuilds the lists.
 * A cell's order truncates its local expansion for the smooth field (and the
 * M2L rows computed for it); its theta sets the opening test of its
 * neighbour candidates at the smallest level.
 * EINVAL if a p is outside 1..order or a theta outside (0,1). */
int ccfmm_plan_set_leaf_params(ccfmm_plan plan, const int32_t* d_p, const double* d_theta, void* stream);
/* Current per-cell parameters into host arrays of n_leaves (p, theta); with no
 * per-cell parameters set, every cell reports (order, theta).  *n_leaves may be
 * queried with NULL arrays. */
int ccfmm_plan_get_leaf_params(ccfmm_plan plan, int32_t* h_p, double* h_theta, int32_t* n_leaves);
/* Compact leaf index of every dipole, input order: d_out [n] int32. */
int ccfmm_plan_leaf_ids(ccfmm_plan plan, int32_t* d_out, void* stream);
/* The selector's 8 features of every cell from device moments [nbatch][n][3]
 * (on the plan's fixed-parameter lists): d_feat [n_leaves][8] FP32. */
int ccfmm_plan_leaf_features(ccfmm_plan plan, int32_t nbatch, const double* d_m, float* d_feat, void* stream);
/* Per cell: sum over its dipoles and configurations of |H - Href|^2 (d_num)
 * and |Href|^2 (d_den), FP64 [n_leaves]; H, Href are [nbatch][n][3]. */
int ccfmm_plan_leaf_errors(ccfmm_plan plan, int32_t nbatch, const double* d_H, const double* d_Href,
                           double* d_num, double* d_den, void* stream);
/* Selector network (FP32, device arrays): forward pass of rows x [8] -> [25]. */
int ccfmm_mlp_forward(const float* d_params, int64_t rows, const float* d_x, float* d_y, void* stream);
/* Loss 0.5 sum mask (y - t)^2 / max(1, sum mask) and its gradient (d_grad
 * [CCFMM_MLP_PARAMS]); d_loss (1 float) may be NULL.  Deterministic. */
int ccfmm_mlp_loss_grad(const float* d_params, int64_t rows, const float* d_x, const float* d_t,
                        const float* d_mask, float* d_grad, float* d_loss, void* stream);
/* One Adam step (beta 0.9 / 0.999, bias-corrected; step counts from 1). */
int ccfmm_mlp_adam(float* d_params, const float* d_grad, float* d_m1, float* d_m2, int32_t step, float lr,
                   void* stream);
/* Learned selection on the current moments: the fixed-parameter field gives
 * each cell's squared field F_c; features -> network -> predicted log10
 * relative error y_c(p, theta) per cell and candidate; the choice minimises
 * the total cost (own dipoles x near source dipoles + cost_far x far cells x
 * the share of the M2L rows order p needs + the smooth field's work at order
 * p, per cell) subject to the predicted
 * global relative RMS error sqrt(sum F_c 10^(2 y_c) / sum F_c) being at most
 * err_bound x 10^-margin (Lagrange multiplier found by bisection), and is set
 * as the plan's per-cell parameters.  With judge != 0 the learned field of
 * these moments is compared with the fixed-parameter field; above err_bound
 * the plan returns to fixed parameters and the call returns
 * CCFMM_W_FALLBACK.  Synchronises the stream. */
int ccfmm_plan_select(ccfmm_plan plan, const float* d_params, double err_bound, double margin, double cost_far,
                      int32_t nbatch, const double* d_m, int32_t judge, void* stream, ccfmm_select_info* out);

/* Selector weights files.  Format (little-endian): "CCFMMSEL", uint32
 * version (1), uint32 inputs, hidden width, outputs, parameter count
 * (8, 64, 25, CCFMM_MLP_PARAMS), uint32 lowest and highest candidate order
 * (2, 6), FP64 candidate angles [5] (0.3 .. 0.7), FP32 parameters (packed as
 * for ccfmm_mlp_forward), uint64 FNV-1a hash of all preceding bytes.
 * Reading checks every field: a mismatch (other network shape, candidate
 * set or version, truncated or altered file) is CCFMM_EINVAL; a file that
 * does not exist gives the warning CCFMM_W_NOWEIGHTS and leaves h_params or
 * the plan unchanged (the plan keeps its fixed parameters). */
int ccfmm_selector_write(const char* path, const float* h_params);  /* h_params: host [CCFMM_MLP_PARAMS] */
int ccfmm_selector_read(const char* path, float* h_params);
/* The plan's selector weights (device copy owned by the plan): from a file,
 * from device memory d_params [CCFMM_MLP_PARAMS] (stream-ordered), or to a
 * file (ESTATE if the plan holds none).  Loading or setting weights makes the
 * next evaluation of a selector = 1 plan choose the per-cell parameters anew. */
int ccfmm_selector_load(ccfmm_plan plan, const char* path);
int ccfmm_selector_set(ccfmm_plan plan, const float* d_params, void* stream);
int ccfmm_selector_save(ccfmm_plan plan, const char* path);

/* Training of the selector network on the GPU (the precursor is the
 * parameter study of Sec. 4: error estimate and timings per (p, alpha)).
 * Labels: for each geometry, every candidate (p, theta) in {2..6} x
 * {0.3..0.7} is applied to all smallest cells, the FMM (fixed order and angle
 * above the smallest cells) is evaluated, and each labelled cell gets log10 of
 * its relative RMS field error against the FP64 direct sum at its dipoles
 * (computed on the GPU).  Features: those of ccfmm_plan_leaf_features.  Then
 * `steps` full-batch Adam steps on the masked squared error from seeded
 * He-normal weights.  All arithmetic runs in the library's kernels; the host
 * only sequences them.  The weights go to out_path (a weights file, if not
 * NULL) and to h_params_out (host [CCFMM_MLP_PARAMS], if not NULL). */
typedef struct {
  int64_t n;             /* dipoles */
  const double* pos;     /* host [n][3] positions */
  const double* m;       /* host [n][3] moments (one configuration) */
  int32_t has_box;       /* 1: root cell [box_lo, box_hi]; 0: the tight bounding box */
  double box_lo[3], box_hi[3];
} ccfmm_train_geometry;
typedef struct {
  int32_t device;
  int32_t n_geom;
  const ccfmm_train_geometry* geom;
  int32_t order;         /* fixed order above the smallest cells, 2..CCFMM_PMAX */
  double theta;          /* fixed opening angle above the smallest cells */
  double leaf_target;    /* s (<= 0: Eq. so) */
  int32_t precision;     /* precision of the labelling evaluations */
  int32_t sample_cells;  /* smallest cells labelled per geometry (<= 0: all of them) */
  int32_t steps;         /* Adam steps, >= 1 */
  float lr;              /* Adam step size, > 0 */
  uint64_t seed;         /* initial weights and cell sample */
} ccfmm_train_spec;
typedef struct {
  int64_t rows;          /* labelled cells over all geometries */
  float loss_first, loss_last;  /* masked loss at the first and the last step */
  double label_seconds, train_seconds;
} ccfmm_train_info;
int ccfmm_selector_train(const ccfmm_train_spec* spec, const char* out_path, float* h_params_out,
                         ccfmm_train_info* info);

/* Direct O(N^2) FP64 field on the GPU at nt sampled targets (error reference at
 * scale): d_pos [n][3], d_m [n][3], d_idx [nt] int64, d_H [nt][3]; stream-ordered. */
int ccfmm_direct_targets_device(int64_t n, const double* d_pos, const double* d_m, int64_t nt,
                                const int64_t* d_idx, double* d_H, void* stream);

/* Self-test of the matrix-core operand layout used by the M2L kernels: runs one
 * 16x16x4 FP32 and one FP64 MFMA tile on known data and compares with a plain
 * product on the host.  Returns CCFMM_OK if both match. */
int ccfmm_selftest_mfma(int32_t device);

#ifdef __cplusplus
}
#endif
#endif
