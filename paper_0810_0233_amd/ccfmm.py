"""Thin ctypes binding of the C ABI in include/ccfmm.h (libccfmm.so).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  The library must have been built (``paper_0810_0233_amd.build``);
loading fails loudly otherwise -- there is no CPU fallback.

Device arrays are passed as raw pointers (e.g. ``tensor.data_ptr()`` of a
torch CUDA tensor) and streams as raw ``hipStream_t`` handles
(``torch.cuda.current_stream().cuda_stream``).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccfmm.so")

PMAX = 8
LMAX = 24
OK, EINVAL, ENOMEM, EHIP, ESTATE, W_FALLBACK, W_NOWEIGHTS = 0, -1, -2, -3, -4, 1, 2
PREC_FP64, PREC_MIXED = 0, 1
# M2L kernel variants (ccfmm_params.m2l_variant)
M2L_AUTO, M2L_BLOCK, M2L_WAVE, M2L_WIDE4, M2L_WIDE2, M2L_WIDE1 = -1, 0, 1, 2, 3, 4


class ccfmm_params(C.Structure):
    _fields_ = [("order", C.c_int32), ("theta", C.c_double), ("leaf_target", C.c_double),
                ("leaf_rule", C.c_int32), ("precision", C.c_int32), ("selector", C.c_int32),
                ("err_bound", C.c_double), ("has_box", C.c_int32),
                ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
                ("max_batch", C.c_int32), ("m2l_class_bits", C.c_int32), ("m2l_variant", C.c_int32),
                ("use_graph", C.c_int32), ("overlap_near", C.c_int32), ("keep_lists", C.c_int32),
                ("truncation", C.c_int32), ("m2l_traceless", C.c_int32),
                ("sel_margin", C.c_double), ("sel_cost_far", C.c_double), ("device_mem_cap", C.c_int64)]


class ccfmm_tune_entry(C.Structure):
    _fields_ = [("variant", C.c_int32), ("class_bits", C.c_int32), ("m2l_ms", C.c_double), ("steps", C.c_int64)]


class ccfmm_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("order", C.c_int32), ("levels", C.c_int32),
                ("precision", C.c_int32), ("max_batch", C.c_int32),
                ("split_axis", C.c_int32 * (LMAX + 1)),
                ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3), ("leaf_side", C.c_double * 3),
                ("s_used", C.c_double), ("n_leaves", C.c_int64), ("n_cells", C.c_int64),
                ("n_m2l_pairs", C.c_int64), ("m2l_pairs_per_level", C.c_int64 * (LMAX + 1)),
                ("n_p2p_leaf_pairs", C.c_int64), ("n_p2p_pairs", C.c_int64),
                ("n_m2l_tiles", C.c_int64), ("n_m2l_steps", C.c_int64), ("n_delta", C.c_int64),
                ("m2l_class_bits", C.c_int32), ("fallback", C.c_int32),
                ("m2l_flops_per_config", C.c_double), ("p2p_pairs_per_config", C.c_double),
                ("m2l_variant", C.c_int32), ("n_rebuilds_kept", C.c_int64),
                ("learned", C.c_int32), ("judge_err", C.c_double), ("sel_cost_far", C.c_double),
                ("device_bytes", C.c_int64), ("overlap_near", C.c_int32), ("tune_eval_ms", C.c_double * 2)]


class ccfmm_train_geometry(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", C.c_void_p), ("m", C.c_void_p), ("has_box", C.c_int32),
                ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3)]


class ccfmm_train_spec(C.Structure):
    _fields_ = [("device", C.c_int32), ("n_geom", C.c_int32), ("geom", C.POINTER(ccfmm_train_geometry)),
                ("order", C.c_int32), ("theta", C.c_double), ("leaf_target", C.c_double),
                ("precision", C.c_int32), ("sample_cells", C.c_int32), ("steps", C.c_int32),
                ("lr", C.c_float), ("seed", C.c_uint64)]


class ccfmm_train_info(C.Structure):
    _fields_ = [("rows", C.c_int64), ("loss_first", C.c_float), ("loss_last", C.c_float),
                ("label_seconds", C.c_double), ("train_seconds", C.c_double)]


class ccfmm_pass_times(C.Structure):
    _fields_ = [("p2m", C.c_double), ("m2m", C.c_double), ("m2l", C.c_double), ("l2l", C.c_double),
                ("p2p", C.c_double), ("l2p", C.c_double), ("total", C.c_double)]


# every symbol the header declares (checked by the CPU tests)
EXPORTS = [
    "ccfmm_status_string", "ccfmm_last_error", "ccfmm_params_default", "ccfmm_plan_create",
    "ccfmm_plan_create_device", "ccfmm_plan_update_positions_device", "ccfmm_eval", "ccfmm_eval_device",
    "ccfmm_eval_device_timed", "ccfmm_plan_autotune", "ccfmm_plan_info", "ccfmm_energy", "ccfmm_plan_energy_device", "ccfmm_plan_destroy",
    "ccfmm_direct_targets_device", "ccfmm_selftest_mfma",
    "ccfmm_plan_set_leaf_params", "ccfmm_plan_get_leaf_params", "ccfmm_plan_leaf_ids", "ccfmm_plan_leaf_features",
    "ccfmm_plan_leaf_errors", "ccfmm_mlp_forward", "ccfmm_mlp_loss_grad", "ccfmm_mlp_adam", "ccfmm_plan_select",
    "ccfmm_energy_device_noalloc", "ccfmm_selector_write", "ccfmm_selector_read", "ccfmm_selector_load",
    "ccfmm_selector_set", "ccfmm_selector_save", "ccfmm_selector_train",
]

NOALLOC_MAX_BATCH = 4096
MLP_IN, MLP_HIDDEN, MLP_OUT = 8, 64, 25
MLP_PARAMS = 64 * 8 + 64 + 64 * 64 + 64 + 25 * 64 + 25
SEL_P = (2, 3, 4, 5, 6)
SEL_THETA = (0.3, 0.4, 0.5, 0.6, 0.7)


class ccfmm_select_info(C.Structure):
    _fields_ = [("n_leaves", C.c_int32), ("hist", C.c_int32 * MLP_OUT), ("judge_err", C.c_double),
                ("fallback", C.c_int32), ("pred_err", C.c_double)]

_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


class CCFMMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (status_string(status), status, msg))
        self.status = status


def lib():
    """Load libccfmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libccfmm.so is not built (run paper_0810_0233_amd.build.build())")
        # One HIP runtime per process: PyTorch ships its own libamdhip64 under
        # the same SONAME; loading torch first makes libccfmm bind to that copy
        # instead of pulling in a second runtime that torch could not share.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        L.ccfmm_status_string.argtypes = [C.c_int]
        L.ccfmm_status_string.restype = C.c_char_p
        L.ccfmm_last_error.restype = C.c_char_p
        L.ccfmm_params_default.argtypes = [C.POINTER(ccfmm_params)]
        L.ccfmm_plan_create.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.c_int64, _dp, C.POINTER(ccfmm_params)]
        L.ccfmm_plan_create_device.argtypes = [C.POINTER(C.c_void_p), C.c_int64, C.c_void_p,
                                               C.POINTER(ccfmm_params), C.c_void_p]
        L.ccfmm_plan_update_positions_device.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.ccfmm_eval.argtypes = [C.c_void_p, C.c_int32, _dp, _dp]
        L.ccfmm_eval_device.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ccfmm_eval_device_timed.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.POINTER(ccfmm_pass_times)]
        L.ccfmm_plan_autotune.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.POINTER(ccfmm_tune_entry), C.c_int32, C.POINTER(C.c_int32)]
        L.ccfmm_plan_info.argtypes = [C.c_void_p, C.POINTER(ccfmm_info)]
        L.ccfmm_energy.argtypes = [C.c_int64, C.c_int32, _dp, _dp, _dp]
        L.ccfmm_plan_energy_device.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                               C.c_void_p]
        L.ccfmm_plan_destroy.argtypes = [C.c_void_p]
        L.ccfmm_plan_destroy.restype = None
        L.ccfmm_direct_targets_device.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                                  C.c_void_p, C.c_void_p]
        L.ccfmm_selftest_mfma.argtypes = [C.c_int32]
        L.ccfmm_energy_device_noalloc.argtypes = [C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                                  C.c_void_p]
        vp = C.c_void_p
        L.ccfmm_selector_write.argtypes = [C.c_char_p, vp]
        L.ccfmm_selector_read.argtypes = [C.c_char_p, vp]
        L.ccfmm_selector_load.argtypes = [vp, C.c_char_p]
        L.ccfmm_selector_set.argtypes = [vp, vp, vp]
        L.ccfmm_selector_save.argtypes = [vp, C.c_char_p]
        L.ccfmm_selector_train.argtypes = [C.POINTER(ccfmm_train_spec), C.c_char_p, vp,
                                           C.POINTER(ccfmm_train_info)]
        L.ccfmm_plan_set_leaf_params.argtypes = [vp, vp, vp, vp]
        L.ccfmm_plan_get_leaf_params.argtypes = [vp, vp, vp, C.POINTER(C.c_int32)]
        L.ccfmm_plan_leaf_ids.argtypes = [vp, vp, vp]
        L.ccfmm_plan_leaf_features.argtypes = [vp, C.c_int32, vp, vp, vp]
        L.ccfmm_plan_leaf_errors.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp]
        L.ccfmm_mlp_forward.argtypes = [vp, C.c_int64, vp, vp, vp]
        L.ccfmm_mlp_loss_grad.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp, vp]
        L.ccfmm_mlp_adam.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_float, vp]
        L.ccfmm_plan_select.argtypes = [vp, vp, C.c_double, C.c_double, C.c_double, C.c_int32, vp, C.c_int32, vp,
                                        C.POINTER(ccfmm_select_info)]
        _lib = L
    return _lib


def status_string(status):
    return lib().ccfmm_status_string(status).decode()


def last_error():
    return lib().ccfmm_last_error().decode()


def _check(rc):
    if rc < 0:
        raise CCFMMError(rc, last_error())
    return rc


def params(order=4, theta=0.5, leaf_target=0.0, leaf_rule=0, precision=PREC_FP64, selector=0,
           err_bound=1e-5, box=None, max_batch=1, m2l_class_bits=3, m2l_variant=-1, use_graph=1, overlap_near=1,
           keep_lists=1, truncation=0, m2l_traceless=1, sel_margin=0.3, sel_cost_far=0.0, device_mem_cap=0):
    p = ccfmm_params()
    _check(lib().ccfmm_params_default(C.byref(p)))
    p.order = int(order)
    p.theta = float(theta)
    p.leaf_target = float(leaf_target)
    p.leaf_rule = int(leaf_rule)
    p.precision = int(precision)
    p.selector = int(selector)
    p.err_bound = float(err_bound)
    if box is not None:
        p.has_box = 1
        for a in range(3):
            p.box_lo[a] = float(box[0][a])
            p.box_hi[a] = float(box[1][a])
    p.max_batch = int(max_batch)
    p.m2l_class_bits = int(m2l_class_bits)
    p.m2l_variant = int(m2l_variant)
    p.use_graph = int(use_graph)
    p.overlap_near = int(overlap_near)
    p.keep_lists = int(keep_lists)
    p.truncation = int(truncation)
    p.m2l_traceless = int(m2l_traceless)
    p.sel_margin = float(sel_margin)
    p.sel_cost_far = float(sel_cost_far)
    p.device_mem_cap = int(device_mem_cap)
    return p


def info_dict(inf):
    L = inf.levels
    d = {f: getattr(inf, f) for f, _ in ccfmm_info._fields_
         if f not in ("split_axis", "box_lo", "box_hi", "leaf_side", "m2l_pairs_per_level", "tune_eval_ms")}
    d["tune_eval_ms"] = list(inf.tune_eval_ms)
    d["split_axis"] = [inf.split_axis[l] for l in range(1, L + 1)]
    d["box_lo"] = list(inf.box_lo)
    d["box_hi"] = list(inf.box_hi)
    d["leaf_side"] = list(inf.leaf_side)
    d["m2l_pairs_per_level"] = [inf.m2l_pairs_per_level[l] for l in range(L + 1)]
    return d


class Plan:
    """A ccfmm plan (tree, lists, derivative tensors) of one geometry."""

    def __init__(self, handle):
        self.h = handle

    @classmethod
    def create(cls, pos, prm, device=0):
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        h = C.c_void_p()
        _check(lib().ccfmm_plan_create(C.byref(h), device, pos.shape[0], pos, C.byref(prm)))
        return cls(h)

    @classmethod
    def create_device(cls, n, d_pos, prm, stream=0):
        h = C.c_void_p()
        _check(lib().ccfmm_plan_create_device(C.byref(h), int(n), C.c_void_p(d_pos), C.byref(prm),
                                              C.c_void_p(stream)))
        return cls(h)

    def update_positions_device(self, d_pos, stream=0):
        _check(lib().ccfmm_plan_update_positions_device(self.h, C.c_void_p(d_pos), C.c_void_p(stream)))

    def eval(self, m):
        """Host moments [nbatch][n][3] (or [n][3]) -> host fields, same shape."""
        m = np.ascontiguousarray(m, dtype=np.float64)
        shape = m.shape
        m3 = m.reshape(-1, self.info()["n"], 3)
        H = np.empty_like(m3)
        self.last_status = _check(lib().ccfmm_eval(self.h, m3.shape[0], m3, H))
        return H.reshape(shape)

    def eval_device(self, nbatch, d_m, d_H, stream=0):
        """Returns the status (OK, or W_FALLBACK when a learned plan's choice was rejected)."""
        self.last_status = _check(lib().ccfmm_eval_device(self.h, int(nbatch), C.c_void_p(d_m), C.c_void_p(d_H),
                                                          C.c_void_p(stream)))
        return self.last_status

    def selector_load(self, path):
        """Weights from a file; returns OK or W_NOWEIGHTS (file missing: fixed parameters kept)."""
        return _check(lib().ccfmm_selector_load(self.h, os.fsencode(path)))

    def selector_set(self, d_params, stream=0):
        _check(lib().ccfmm_selector_set(self.h, C.c_void_p(d_params), C.c_void_p(stream)))

    def selector_save(self, path):
        _check(lib().ccfmm_selector_save(self.h, os.fsencode(path)))

    def energy_device(self, nbatch, d_m, d_H, d_E, stream=0):
        """E_b = -1/2 sum_i m_i . H_i on the GPU into d_E [nbatch] (FP64)."""
        _check(lib().ccfmm_plan_energy_device(self.h, int(nbatch), C.c_void_p(d_m), C.c_void_p(d_H), C.c_void_p(d_E),
                                              C.c_void_p(stream)))

    def eval_device_timed(self, nbatch, d_m, d_H, stream=0):
        t = ccfmm_pass_times()
        _check(lib().ccfmm_eval_device_timed(self.h, int(nbatch), C.c_void_p(d_m), C.c_void_p(d_H),
                                             C.c_void_p(stream), C.byref(t)))
        return {f: getattr(t, f) for f, _ in ccfmm_pass_times._fields_}

    def autotune(self, nbatch, d_m, d_H, stream=0):
        """Time the M2L variants on this plan and keep the fastest, then the two
        evaluation forms (near field beside the expansion passes, or one stream)
        and keep the faster; returns the M2L timings (the forms' times are in
        info()["tune_eval_ms"])."""
        out = (ccfmm_tune_entry * 32)()
        n = C.c_int32(0)
        _check(lib().ccfmm_plan_autotune(self.h, int(nbatch), C.c_void_p(d_m), C.c_void_p(d_H),
                                         C.c_void_p(stream), out, 32, C.byref(n)))
        return [{"variant": out[i].variant, "class_bits": out[i].class_bits, "m2l_ms": out[i].m2l_ms,
                 "steps": out[i].steps} for i in range(n.value)]

    def set_leaf_params(self, d_p, d_theta, stream=0):
        """Per-cell (order, theta) from device arrays (compact leaf order); 0/None clears."""
        _check(lib().ccfmm_plan_set_leaf_params(self.h, C.c_void_p(d_p or None), C.c_void_p(d_theta or None),
                                                C.c_void_p(stream)))

    def get_leaf_params(self):
        nl = C.c_int32(0)
        _check(lib().ccfmm_plan_get_leaf_params(self.h, None, None, C.byref(nl)))
        p = np.zeros(nl.value, dtype=np.int32)
        th = np.zeros(nl.value)
        _check(lib().ccfmm_plan_get_leaf_params(self.h, p.ctypes.data_as(C.c_void_p), th.ctypes.data_as(C.c_void_p),
                                                C.byref(nl)))
        return p, th

    def leaf_ids(self, d_out, stream=0):
        _check(lib().ccfmm_plan_leaf_ids(self.h, C.c_void_p(d_out), C.c_void_p(stream)))

    def leaf_features(self, nbatch, d_m, d_feat, stream=0):
        _check(lib().ccfmm_plan_leaf_features(self.h, int(nbatch), C.c_void_p(d_m), C.c_void_p(d_feat),
                                              C.c_void_p(stream)))

    def leaf_errors(self, nbatch, d_H, d_Href, d_num, d_den, stream=0):
        _check(lib().ccfmm_plan_leaf_errors(self.h, int(nbatch), C.c_void_p(d_H), C.c_void_p(d_Href),
                                            C.c_void_p(d_num), C.c_void_p(d_den), C.c_void_p(stream)))

    def select(self, d_params, err_bound, margin, cost_far, nbatch, d_m, judge=True, stream=0):
        """Learned per-cell (p, theta); returns (status, info dict).  status 1 = fell back."""
        out = ccfmm_select_info()
        rc = _check(lib().ccfmm_plan_select(self.h, C.c_void_p(d_params), float(err_bound), float(margin),
                                            float(cost_far), int(nbatch), C.c_void_p(d_m), int(bool(judge)),
                                            C.c_void_p(stream), C.byref(out)))
        return rc, {"n_leaves": out.n_leaves, "hist": list(out.hist), "judge_err": out.judge_err,
                    "fallback": out.fallback, "pred_err": out.pred_err}

    def info(self):
        inf = ccfmm_info()
        _check(lib().ccfmm_plan_info(self.h, C.byref(inf)))
        return info_dict(inf)

    def destroy(self):
        if self.h:
            lib().ccfmm_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def energy(m, H):
    m = np.ascontiguousarray(m, dtype=np.float64)
    H = np.ascontiguousarray(H, dtype=np.float64)
    n = m.shape[-2]
    nb = m.size // (3 * n)
    E = np.zeros(nb)
    _check(lib().ccfmm_energy(n, nb, m.reshape(-1), H.reshape(-1), E))
    return E


def selector_write(path, params):
    P = np.ascontiguousarray(params, dtype=np.float32)
    if P.size != MLP_PARAMS:
        raise ValueError("expected %d parameters" % MLP_PARAMS)
    _check(lib().ccfmm_selector_write(os.fsencode(path), P.ctypes.data_as(C.c_void_p)))


def selector_read(path):
    """Weights from a file, or None if the file does not exist."""
    P = np.zeros(MLP_PARAMS, dtype=np.float32)
    rc = _check(lib().ccfmm_selector_read(os.fsencode(path), P.ctypes.data_as(C.c_void_p)))
    return None if rc == W_NOWEIGHTS else P


def selector_train(geoms, order=6, theta=0.4, leaf_target=0.0, precision=PREC_MIXED, sample_cells=0, steps=600,
                   lr=3e-3, seed=1, out_path=None, device=0):
    """GPU training of the selector network (labels, features and Adam in the
    library).  geoms: list of dicts with pos [n][3], m [n][3] and box (or
    None).  Returns (params, info dict)."""
    keep = []
    G = (ccfmm_train_geometry * len(geoms))()
    for i, g in enumerate(geoms):
        pos = np.ascontiguousarray(g["pos"], dtype=np.float64).reshape(-1, 3)
        m = np.ascontiguousarray(g["m"], dtype=np.float64).reshape(-1, 3)
        keep += [pos, m]
        G[i].n = pos.shape[0]
        G[i].pos = pos.ctypes.data
        G[i].m = m.ctypes.data
        box = g.get("box")
        if box is not None:
            G[i].has_box = 1
            for a in range(3):
                G[i].box_lo[a] = float(box[0][a])
                G[i].box_hi[a] = float(box[1][a])
    sp = ccfmm_train_spec(device=device, n_geom=len(geoms), geom=G, order=order, theta=theta,
                          leaf_target=leaf_target, precision=precision, sample_cells=sample_cells, steps=steps,
                          lr=lr, seed=seed)
    P = np.zeros(MLP_PARAMS, dtype=np.float32)
    inf = ccfmm_train_info()
    _check(lib().ccfmm_selector_train(C.byref(sp), None if out_path is None else os.fsencode(out_path),
                                      P.ctypes.data_as(C.c_void_p), C.byref(inf)))
    return P, {f: getattr(inf, f) for f, _ in ccfmm_train_info._fields_}


def energy_device_noalloc(n, nbatch, d_m, d_H, d_E, stream=0):
    """Energy per configuration from device arrays with no allocation (fixed
    library scratch); nbatch <= NOALLOC_MAX_BATCH."""
    _check(lib().ccfmm_energy_device_noalloc(int(n), int(nbatch), C.c_void_p(d_m), C.c_void_p(d_H),
                                             C.c_void_p(d_E), C.c_void_p(stream)))


def direct_targets_device(n, d_pos, d_m, nt, d_idx, d_H, stream=0):
    _check(lib().ccfmm_direct_targets_device(int(n), C.c_void_p(d_pos), C.c_void_p(d_m), int(nt),
                                             C.c_void_p(d_idx), C.c_void_p(d_H), C.c_void_p(stream)))


def mlp_forward(d_params, rows, d_x, d_y, stream=0):
    _check(lib().ccfmm_mlp_forward(C.c_void_p(d_params), int(rows), C.c_void_p(d_x), C.c_void_p(d_y),
                                   C.c_void_p(stream)))


def mlp_loss_grad(d_params, rows, d_x, d_t, d_mask, d_grad, d_loss=None, stream=0):
    _check(lib().ccfmm_mlp_loss_grad(C.c_void_p(d_params), int(rows), C.c_void_p(d_x), C.c_void_p(d_t),
                                     C.c_void_p(d_mask), C.c_void_p(d_grad), C.c_void_p(d_loss),
                                     C.c_void_p(stream)))


def mlp_adam(d_params, d_grad, d_m1, d_m2, step, lr, stream=0):
    _check(lib().ccfmm_mlp_adam(C.c_void_p(d_params), C.c_void_p(d_grad), C.c_void_p(d_m1), C.c_void_p(d_m2),
                                int(step), float(lr), C.c_void_p(stream)))


def selftest_mfma(device=0):
    return lib().ccfmm_selftest_mfma(device)
