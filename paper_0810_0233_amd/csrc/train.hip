// train.hip -- the learned selector's weights files and its training driver.
//
// The paper picks one (p_m, alpha_m) per system from the error estimate and
// timings (Sec. 4, Table II).  The selector makes that choice per smallest
// cell from a network trained here: labels are the per-cell field errors of
// the library's own FMM for every candidate (p, theta) against the FP64
// direct sum, and the network is fitted with the library's forward/backward
// and Adam kernels.  The host only sequences kernels and holds the seeded
// choices (initial weights, sampled cells).
#include <algorithm>
#include <cerrno>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>

#include "plan.hpp"
#include "selfile.hpp"

namespace ccfmm {

// ---------------------------------------------------------------- weights files
// (parsing lives in selfile.cpp, host code only)
void selector_file_write(const char* path, const float* h_params) {
  std::string err;
  if (selfile_write(path, h_params, &err) != CCFMM_OK) fail(CCFMM_EINVAL, err);
}

bool selector_file_read(const char* path, float* h_params) {
  std::string err;
  const int rc = selfile_read(path, h_params, &err);
  if (rc == CCFMM_W_NOWEIGHTS) return false;
  if (rc != CCFMM_OK) fail(CCFMM_EINVAL, err);
  return true;
}

// ---------------------------------------------------------------- training
// splitmix64 (Steele, Lea and Flood, 2014): seeded uniforms for the host-side
// choices; normals by the Box-Muller transform.
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }  // [0, 1)
  double normal() {
    const double u1 = 1.0 - uniform(), u2 = uniform();  // u1 in (0, 1]
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

// He-normal initial weights packed as the forward kernel reads them; the
// output bias starts at -5 (log10 errors of interest lie around there)
static std::vector<float> initial_params(uint64_t seed) {
  constexpr int i = CCFMM_MLP_IN, h = CCFMM_MLP_HIDDEN, o = CCFMM_MLP_OUT;
  SplitMix64 rng{seed * 0x2545f4914f6cdd1dull + 1};
  std::vector<float> P;
  P.reserve(CCFMM_MLP_PARAMS);
  for (int k = 0; k < h * i; k++) P.push_back((float)(rng.normal() * std::sqrt(2.0 / i)));
  for (int k = 0; k < h; k++) P.push_back(0.f);
  for (int k = 0; k < h * h; k++) P.push_back((float)(rng.normal() * std::sqrt(2.0 / h)));
  for (int k = 0; k < h; k++) P.push_back(0.f);
  for (int k = 0; k < o * h; k++) P.push_back((float)(rng.normal() * std::sqrt(1.0 / h)));
  for (int k = 0; k < o; k++) P.push_back(-5.f);
  return P;
}

struct PlanGuard {
  ccfmm_plan p = nullptr;
  ~PlanGuard() { ccfmm_plan_destroy(p); }
};
struct StreamGuard {
  hipStream_t s = nullptr;
  ~StreamGuard() {
    if (s) (void)hipStreamDestroy(s);
  }
};

static double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Rows of one geometry: features [cells][8] and labels / mask [cells][25].
static void label_geometry(const ccfmm_train_spec& sp, int gi, std::vector<float>& X, std::vector<float>& Y,
                           std::vector<float>& M, hipStream_t st) {
  const ccfmm_train_geometry& g = sp.geom[gi];
  ccfmm_params prm;
  ccfmm_params_default(&prm);
  prm.order = sp.order;
  prm.theta = sp.theta;
  prm.leaf_target = sp.leaf_target;
  prm.precision = sp.precision;
  prm.max_batch = 1;
  prm.has_box = g.has_box;
  for (int a = 0; a < 3; a++) {
    prm.box_lo[a] = g.box_lo[a];
    prm.box_hi[a] = g.box_hi[a];
  }
  PlanGuard pg;
  const int rc = ccfmm_plan_create(&pg.p, sp.device, g.n, g.pos, &prm);
  if (rc < 0) fail(rc, "training geometry " + std::to_string(gi) + ": " + ccfmm_last_error());
  Plan& P = pg.p->P;
  const int64_t n = P.n;
  const int nl = P.lev[P.L]->ncells;
  DevBuf dm, feat, ids, didx, dHd, dH, dref, num, den;
  dm.ensure(sizeof(double) * 3 * n);
  CCFMM_HIP(hipMemcpyAsync(dm.p, g.m, sizeof(double) * 3 * n, hipMemcpyHostToDevice, st));
  feat.ensure(sizeof(float) * CCFMM_MLP_IN * (size_t)nl);
  run_leaf_features(P, 1, dm.as<double>(), feat.as<float>(), st);
  // the labelled cells: a seeded sample, or all of them
  std::vector<int> cells(nl);
  for (int c = 0; c < nl; c++) cells[c] = c;
  if (sp.sample_cells > 0 && sp.sample_cells < nl) {
    SplitMix64 rng{sp.seed * 0x9e3779b97f4a7c15ull + (uint64_t)gi + 7};
    for (int k = 0; k < sp.sample_cells; k++) {  // partial Fisher-Yates
      const int j = k + (int)(rng.uniform() * (double)(nl - k));
      std::swap(cells[k], cells[std::min(j, nl - 1)]);
    }
    cells.resize(sp.sample_cells);
    std::sort(cells.begin(), cells.end());
  }
  std::vector<char> chosen(nl, 0);
  for (int c : cells) chosen[c] = 1;
  // their dipoles, and the FP64 direct sum there
  ids.ensure(sizeof(int32_t) * n);
  run_leaf_ids(P, ids.as<int32_t>(), st);
  std::vector<int32_t> hid(n);
  CCFMM_HIP(hipMemcpyAsync(hid.data(), ids.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
  CCFMM_HIP(hipStreamSynchronize(st));
  std::vector<int64_t> idx;
  for (int64_t i = 0; i < n; i++)
    if (chosen[hid[i]]) idx.push_back(i);
  const int64_t nt = (int64_t)idx.size();
  didx.ensure(sizeof(int64_t) * std::max<int64_t>(1, nt));
  dHd.ensure(sizeof(double) * 3 * std::max<int64_t>(1, nt));
  CCFMM_HIP(hipMemcpyAsync(didx.p, idx.data(), sizeof(int64_t) * nt, hipMemcpyHostToDevice, st));
  run_direct_targets(n, P.pos.as<double>(), dm.as<double>(), nt, didx.as<int64_t>(), dHd.as<double>(), st);
  dH.ensure(sizeof(double) * 3 * n);
  dref.ensure(sizeof(double) * 3 * n);
  num.ensure(sizeof(double) * nl);
  den.ensure(sizeof(double) * nl);
  const size_t row0 = Y.size() / CCFMM_MLP_OUT;
  const size_t rows = cells.size();
  Y.resize((row0 + rows) * CCFMM_MLP_OUT, 0.f);
  M.resize((row0 + rows) * CCFMM_MLP_OUT, 0.f);
  std::vector<int32_t> hp(nl);
  std::vector<double> ht(nl), hn(nl), hd(nl);
  for (int pi = 0; pi < 5; pi++) {
    for (int ti = 0; ti < 5; ti++) {
      std::fill(hp.begin(), hp.end(), std::min<int>((int)kSelPLo + pi, P.p));
      std::fill(ht.begin(), ht.end(), kSelTheta[ti]);
      apply_leaf_params(P, hp.data(), ht.data(), st);
      eval_once(P, 1, dm.as<double>(), dH.as<double>(), st);
      // reference: the FMM's own field, with the direct sum at the labelled
      // cells' dipoles (the other rows are not used)
      CCFMM_HIP(hipMemcpyAsync(dref.p, dH.p, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st));
      run_scatter_rows(nt, didx.as<int64_t>(), dHd.as<double>(), dref.as<double>(), st);
      run_leaf_errors(P, 1, dH.as<double>(), dref.as<double>(), num.as<double>(), den.as<double>(), st);
      CCFMM_HIP(hipMemcpyAsync(hn.data(), num.p, sizeof(double) * nl, hipMemcpyDeviceToHost, st));
      CCFMM_HIP(hipMemcpyAsync(hd.data(), den.p, sizeof(double) * nl, hipMemcpyDeviceToHost, st));
      CCFMM_HIP(hipStreamSynchronize(st));
      const int col = pi * 5 + ti;
      for (size_t r = 0; r < rows; r++) {
        const int c = cells[r];
        if (hd[c] > 0.0 && hn[c] > 0.0) {
          Y[(row0 + r) * CCFMM_MLP_OUT + col] = (float)std::log10(std::sqrt(hn[c] / hd[c]));
          M[(row0 + r) * CCFMM_MLP_OUT + col] = 1.f;
        }
      }
    }
  }
  std::vector<float> hf((size_t)nl * CCFMM_MLP_IN);
  CCFMM_HIP(hipMemcpyAsync(hf.data(), feat.p, sizeof(float) * hf.size(), hipMemcpyDeviceToHost, st));
  CCFMM_HIP(hipStreamSynchronize(st));
  for (int c : cells) X.insert(X.end(), hf.begin() + (size_t)c * CCFMM_MLP_IN, hf.begin() + (size_t)(c + 1) * CCFMM_MLP_IN);
}

void train_selector(const ccfmm_train_spec* sp, const char* out_path, float* h_out, ccfmm_train_info* info) {
  if (!sp) fail(CCFMM_EINVAL, "spec is NULL");
  if (sp->n_geom < 1 || !sp->geom) fail(CCFMM_EINVAL, "no training geometry");
  if (sp->order < 2 || sp->order > kPMax) fail(CCFMM_EINVAL, "training order must be in 2..8");
  if (!(sp->theta > 0.0 && sp->theta < 1.0)) fail(CCFMM_EINVAL, "training theta must be in (0, 1)");
  if (sp->steps < 1 || !(sp->lr > 0.f)) fail(CCFMM_EINVAL, "training needs steps >= 1 and lr > 0");
  if (sp->precision != CCFMM_PREC_FP64 && sp->precision != CCFMM_PREC_MIXED)
    fail(CCFMM_EINVAL, "precision must be FP64 or MIXED");
  for (int g = 0; g < sp->n_geom; g++)
    if (sp->geom[g].n < 1 || !sp->geom[g].pos || !sp->geom[g].m)
      fail(CCFMM_EINVAL, "training geometry " + std::to_string(g) + " is empty or NULL");
  if (!out_path && !h_out) fail(CCFMM_EINVAL, "neither an output file nor an output array");
  CCFMM_HIP(hipSetDevice(sp->device));
  StreamGuard sg;
  CCFMM_HIP(hipStreamCreateWithFlags(&sg.s, hipStreamNonBlocking));
  const hipStream_t st = sg.s;
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<float> X, Y, M;
  for (int g = 0; g < sp->n_geom; g++) label_geometry(*sp, g, X, Y, M, st);
  const int64_t rows = (int64_t)(Y.size() / CCFMM_MLP_OUT);
  if (rows < 1) fail(CCFMM_EINVAL, "no labelled cell");
  const double t_label = seconds_since(t0);
  const auto t1 = std::chrono::steady_clock::now();
  DevBuf dx, dy, dk, dP, dg, dm1, dm2, dl, tmp;
  dx.ensure(sizeof(float) * X.size());
  dy.ensure(sizeof(float) * Y.size());
  dk.ensure(sizeof(float) * M.size());
  dP.ensure(sizeof(float) * CCFMM_MLP_PARAMS);
  dg.ensure(sizeof(float) * CCFMM_MLP_PARAMS);
  dm1.ensure(sizeof(float) * CCFMM_MLP_PARAMS);
  dm2.ensure(sizeof(float) * CCFMM_MLP_PARAMS);
  dl.ensure(sizeof(float));
  const std::vector<float> P0 = initial_params(sp->seed);
  CCFMM_HIP(hipMemcpyAsync(dx.p, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice, st));
  CCFMM_HIP(hipMemcpyAsync(dy.p, Y.data(), sizeof(float) * Y.size(), hipMemcpyHostToDevice, st));
  CCFMM_HIP(hipMemcpyAsync(dk.p, M.data(), sizeof(float) * M.size(), hipMemcpyHostToDevice, st));
  CCFMM_HIP(hipMemcpyAsync(dP.p, P0.data(), sizeof(float) * P0.size(), hipMemcpyHostToDevice, st));
  CCFMM_HIP(hipMemsetAsync(dm1.p, 0, sizeof(float) * CCFMM_MLP_PARAMS, st));
  CCFMM_HIP(hipMemsetAsync(dm2.p, 0, sizeof(float) * CCFMM_MLP_PARAMS, st));
  float loss_first = 0.f, loss_last = 0.f;
  for (int k = 1; k <= sp->steps; k++) {
    const bool want = k == 1 || k == sp->steps;
    run_mlp_loss_grad(dP.as<float>(), rows, dx.as<float>(), dy.as<float>(), dk.as<float>(), dg.as<float>(),
                      want ? dl.as<float>() : nullptr, tmp, st);
    if (want) {
      float l = 0.f;
      CCFMM_HIP(hipMemcpyAsync(&l, dl.p, sizeof(float), hipMemcpyDeviceToHost, st));
      CCFMM_HIP(hipStreamSynchronize(st));
      (k == 1 ? loss_first : loss_last) = l;
      if (k == 1 && sp->steps == 1) loss_last = l;
    }
    run_mlp_adam(dP.as<float>(), dg.as<float>(), dm1.as<float>(), dm2.as<float>(), k, sp->lr, st);
  }
  std::vector<float> P1(CCFMM_MLP_PARAMS);
  CCFMM_HIP(hipMemcpyAsync(P1.data(), dP.p, sizeof(float) * P1.size(), hipMemcpyDeviceToHost, st));
  CCFMM_HIP(hipStreamSynchronize(st));
  if (out_path) selector_file_write(out_path, P1.data());
  if (h_out) std::copy(P1.begin(), P1.end(), h_out);
  if (info) {
    info->rows = rows;
    info->loss_first = loss_first;
    info->loss_last = loss_last;
    info->label_seconds = t_label;
    info->train_seconds = seconds_since(t1);
  }
}

}  // namespace ccfmm
