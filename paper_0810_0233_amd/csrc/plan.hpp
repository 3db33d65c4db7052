// plan.hpp -- the plan object: tree, lists, derivative tensors and M2L tiles
// of one geometry, plus the expansion buffers of its evaluations.
#pragma once
#include <array>
#include <memory>

#include "internal.hpp"

namespace ccfmm {

// Geometry passed by value to kernels that need the level table.
struct TreeGeom {
  LevelGeom lev[kLMax + 1];
  double lo[3];
  double W[3];
  int L;
  int pad;
};

struct LevelData {
  int32_t ncells = 0;   // occupied cells
  int64_t heap0 = 0;    // first heap id of the level (2^l - 1)
  DevBuf key;           // compact -> key (int32)
  DevBuf coord;         // compact -> integer cell coordinates (3 int32)
  DevBuf parent;        // compact -> parent compact (int32), level >= 1
  DevBuf child;         // compact -> 2 child compact (int32, -1 empty), level < L
  DevBuf near_ptr;      // CSR (ncells+1) of near cells (compact), self included
  DevBuf near_idx;
  int64_t nnear = 0;
  DevBuf far_ptr;       // CSR (ncells+1) of far cells (M2L sources)
  DevBuf far_idx;
  DevBuf far_did;       // dense offset id of each far entry (box wfar)
  int64_t nfar = 0;
  // offset bounds (host): near offsets lie in [-wnear, wnear], every candidate
  // (near or far) in [-wfar, wfar]; cnear = most near cells any cell can have
  int wnear[3] = {0, 0, 0};
  int wfar[3] = {0, 0, 0};
  int64_t cnear = 1;
  int64_t nbox = 1;     // dense offset ids of the level: prod(2 wfar + 1)
  int64_t drow0 = 0;    // derivative-tensor row of dense id 0
  int64_t qoff = 0;     // element offset of the level in Q/V
};

struct Plan {
  MemBudget mem;  // first member: destroyed after every buffer charged to it
  int device = 0;
  int64_t n = 0;
  ccfmm_params prm{};
  int p = 0, L = 0;
  int precision = 0;
  int nbmax = 1;
  int class_bits = 3;
  double s_used = 0.0;
  TreeGeom geo{};
  hipStream_t own_stream = nullptr;
  // the near field runs on a second stream beside the expansion passes
  // (forked after the moment permutation, joined before L2P)
  bool overlap = true;
  double tune_eval_ms[2] = {0.0, 0.0};  // the last autotune's evaluation times: [0] overlapped, [1] one stream
  DevBuf heap_flag_prev;       // occupancy of every heap cell at the previous build
  DevBuf pos_check;            // [0] a position is not finite, [1] one lies outside the caller's box
  bool pairs_stale = false;    // info's direct-pair count not yet taken for the current cells
  bool ever_built = false;     // a build succeeded once (buffers and parameters in place)
  int64_t n_rebuilds_kept = 0;  // rebuilds that kept lists and tiles (same geometry and occupied cells)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  // sorted dipoles
  DevBuf pos;        // [n][3] FP64 input order (device copy)
  DevBuf key, val, key_tmp, val_tmp;
  DevBuf perm;       // sorted -> input index (int32)
  DevBuf yd;         // SoA [3][n] FP64 leaf-relative scaled offsets
  DevBuf yf;         // SoA [3][n] FP32, then [3][n] FP32 residuals (yd - yf)
  DevBuf leaf_start; // 2^L + 1 (int32), by leaf key
  DevBuf lstart, lcount;  // per occupied leaf (compact)
  DevBuf heap_flag, heap_scan;  // occupancy and compact ids over all heap cells
  DevBuf cmap;       // heap id -> compact id within its level, -1 if empty
  std::vector<std::unique_ptr<LevelData>> lev;

  // derivative tensors: one dense table per distinct (g, wfar) of the levels,
  // kept across rebuilds while the keys do not change
  int64_t nrows = 0;
  DevBuf Dd, Df;
  DevBuf Dx;  // FP32 rows expanded into the wide M2L kernels' LDS order (mixed precision)
  DevBuf Qr;  // folded (traceless-form) moments, nred_stride(p) per row, for the wide M2L kernels
  int dtab_p = 0;
  std::vector<std::array<double, 6>> dtab_keys;
  // M2L tiles
  int TB = 64, TC = 1, ncg = 1;  // configs per tile, targets per tile, config groups
  int m2l_variant = kM2LBlock;    // kernel used by run_m2l
  // the last M2L left the local rows of levels >= 2 folded (their n_z <= 1
  // components only); L2L completes them
  bool v_folded = false;
  // the last M2M wrote the folded moments of levels >= 2 (the M2L pass folds
  // levels 0 and 1)
  bool q_folded = false;
  int tiles_variant = -1, tiles_class_bits = -1;  // what the current tiles were built for
  DevBuf tiles, tile_tgt, step_delta, step_src, bitmap, gcount;
  DevBuf tile_order;  // launch order of the M2L tiles: longest step list first (+ sort temporaries)
  DevBuf tile_sort;   // target ordering of all levels (keys, order, temporaries, inverse)
  DevBuf near_tmp;    // reordering buffer of the smallest level's near lists
  bool tile_signature = true;  // M2L targets also grouped by their set of far offsets
  int64_t ntiles = 0, nsteps = 0;
  // P2P chunks (built on the device; their count stays in device memory)
  DevBuf chunks, chunk_cnt;
  int64_t nchunks_cap = 0;
  int64_t nchunks = 0;  // filled at info time
  // expansions (compact cells of all levels)
  DevBuf Q, V;
  int64_t qv_elems = 0;
  int qv_batch = 0;  // nbatch the Q/V buffers are laid out for
  DevBuf m_sorted;   // moments in sorted order [b][3][n] (FP64 or FP32)
  // batched near field (many configurations): moments [n][3][b] (configuration
  // fastest), target chunks of <= 32 dipoles, smallest cell of each dipole
  DevBuf m_sorted_t;
  DevBuf chunks32, dleaf;
  int64_t nchunks32 = 0;
  int64_t nchunks32_cap = 0;  // capacity of the 32-chunk list (launch size of the batched near field)
  int batched_min = 32;  // nbatch from which the near field runs on the matrix cores
  DevBuf scratch;    // scan/sort temporaries
  DevBuf scratch2;
  DevBuf flags;      // device error flags
  // per-smallest-cell order and opening angle (compact leaf order); the levels
  // above keep (p, theta).  theta is stored squared, as the list test uses it.
  bool has_leaf = false;
  DevBuf leaf_p, leaf_th2;
  std::vector<int32_t> h_leaf_p;    // host copies of the per-cell parameters
  std::vector<double> h_leaf_theta;
  double leaf_theta_min = 1.0;
  int tiles_nb = 1;                 // nbatch the M2L tiles were built for
  DevBuf judge_a, judge_b;          // field buffers of the selector's judge
  // learned mode (selector = 1): network weights, and whether the per-cell
  // choice must be made at the next evaluation (new plan, new weights, or an
  // update that changed the occupied cells)
  DevBuf sel_w;
  bool has_sel_w = false;
  bool sel_stale = true;
  // captured evaluation graph, valid for (g_nb, g_m, g_H) until the next rebuild
  bool use_graph = true;
  hipGraphExec_t gexec = nullptr;
  int g_nb = 0;
  const void* g_m = nullptr;
  void* g_H = nullptr;
  DevBuf host_m, host_H;  // staging of the host-pointer evaluation (stable addresses)
  DevBuf energy_part;     // per-block partial sums of the energy (nbatch x kEnergyBlocks)
  ccfmm_info info{};
  bool built = false;
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
  }
  ~Plan() {
    drop_graph();
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
  }
};

// build steps (tree.hip, lists.hip, expansions.hip)
// occupied smallest cells for every depth 0..24 (G24: the geometry at depth 24)
void count_occupied_by_depth(Plan& P, const double* d_pos, const TreeGeom& G24, hipStream_t st, int64_t* occupied);
void build_tree(Plan& P, const double* d_pos, hipStream_t st, bool* same_cells = nullptr,
                const int32_t* d_check = nullptr, int32_t* h_check = nullptr);
void build_lists(Plan& P, hipStream_t st);
void build_dtensors(Plan& P, hipStream_t st);
void build_m2l_tiles(Plan& P, int nbatch, hipStream_t st);
void build_p2p_chunks(Plan& P, hipStream_t st);

// evaluation passes
void run_p2m(Plan& P, int nb, const double* d_m, hipStream_t st);
void run_m2m(Plan& P, int nb, hipStream_t st);
// M2M and L2L in their LDS-staged form (the fastest alone, with the fold and
// the local rows' completion fused in), or, while the near field runs beside
// them, the form with few registers that fits beside the near field's waves
inline bool shifts_staged(const Plan& P) { return !P.overlap; }
void run_m2l(Plan& P, int nb, hipStream_t st);
void run_l2l(Plan& P, int nb, hipStream_t st);
void run_p2p_l2p(Plan& P, int nb, double* d_H, hipStream_t st);  // near + smooth field, one stream
void run_near(Plan& P, int nb, double* d_H, hipStream_t st);     // near field written to H
void run_l2p(Plan& P, int nb, double* d_H, hipStream_t st);      // smooth field added to H
void run_permute(Plan& P, int nb, const double* d_m, hipStream_t st);
void build_wide_ops(Plan& P, hipStream_t st);  // expanded operator rows (Dx) from Df
double m2l_row_share(const Plan& P, int q);  // smallest-level M2L tile work at order q (0..1]
void run_energy(Plan& P, int nb, const double* d_m, const double* d_H, double* d_E, hipStream_t st);
void run_energy_noalloc(int64_t n, int nb, const double* d_m, const double* d_H, double* d_E, hipStream_t st);
void run_direct_targets(int64_t n, const double* d_pos, const double* d_m, int64_t nt,
                        const int64_t* d_idx, double* d_H, hipStream_t st);

// learned selector and per-cell data (selector.hip)
void run_leaf_ids(Plan& P, int32_t* d_out, hipStream_t st);
void run_leaf_errors(Plan& P, int nb, const double* d_H, const double* d_Href, double* d_num, double* d_den,
                     hipStream_t st);
void run_leaf_features(Plan& P, int nb, const double* d_m, float* d_feat, hipStream_t st);
void run_mlp_forward(const float* d_params, int64_t rows, const float* d_x, float* d_y, hipStream_t st);
void run_mlp_loss_grad(const float* d_params, int64_t rows, const float* d_x, const float* d_t, const float* d_mask,
                       float* d_grad, float* d_loss, DevBuf& tmp, hipStream_t st);
void run_mlp_adam(float* d_params, const float* d_grad, float* d_m1, float* d_m2, int step, float lr,
                  hipStream_t st);
void run_select(Plan& P, const float* d_params, double log_bound, double cost_far, int nb, const double* d_m,
                const double* d_F, int32_t* d_p, double* d_theta, std::vector<int32_t>& hist, double* pred_err,
                hipStream_t st);
double run_rel_rms(const double* d_A, const double* d_B, int64_t count, DevBuf& tmp, hipStream_t st);
void run_scatter_rows(int64_t nt, const int64_t* d_idx, const double* d_src, double* d_dst, hipStream_t st);

// plan-level steps shared by the C ABI and the selector trainer (api.hip)
void apply_leaf_params(Plan& P, const int32_t* hp, const double* hth, hipStream_t st);
void eval_once(Plan& P, int nb, const double* d_m, double* d_H, hipStream_t st);
int select_impl(Plan& P, const float* d_params, double err_bound, double margin, double cost_far, int nbatch,
                const double* d_m, bool judge, hipStream_t st, ccfmm_select_info* out);
// selector weights files (train.hip): write, and read (false if the file
// does not exist; any other problem throws CCFMM_EINVAL)
void selector_file_write(const char* path, const float* h_params);
bool selector_file_read(const char* path, float* h_params);
void train_selector(const ccfmm_train_spec* spec, const char* out_path, float* h_out, ccfmm_train_info* info);

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// dense offset id of (dx, dy, dz) in the box [-w, w]^3
__host__ __device__ inline int64_t box_index(const int w[3], int dx, int dy, int dz) {
  return ((int64_t)(dx + w[0]) * (2 * w[1] + 1) + (dy + w[1])) * (2 * w[2] + 1) + (dz + w[2]);
}

}  // namespace ccfmm

// the opaque plan handle of the C ABI
struct ccfmm_plan_s {
  ccfmm::Plan P;
};
