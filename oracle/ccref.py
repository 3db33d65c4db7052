"""ctypes binding of the C oracle (``ccref.c``).  Test infrastructure only.

Arrays are numpy float64, [n][3] row-major.  Dense expansion cubes are
returned as arrays of shape (K+1, K+1, K+1) indexed [nx, ny, nz].
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ccref.c")
_LIB = os.path.join(_HERE, "libccref.so")

PMAX = 8
LMAX = 24


def build(force=True):
    """Compile the oracle with gcc (OpenMP, no FP contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99",
           "-D_POSIX_C_SOURCE=200809L", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("order", C.c_int32), ("theta", C.c_double), ("leaf_target", C.c_double),
                ("leaf_rule", C.c_int32), ("has_box", C.c_int32),
                ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3), ("nthreads", C.c_int32),
                ("truncation", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("levels", C.c_int32), ("split_axis", C.c_int32 * (LMAX + 1)),
                ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
                ("leaf_side", C.c_double * 3), ("s_used", C.c_double),
                ("n_cells", C.c_int64), ("n_leaves", C.c_int64), ("n_m2l_pairs", C.c_int64),
                ("n_p2p_leaf_pairs", C.c_int64), ("m2l_pairs_per_level", C.c_int64 * (LMAX + 1)),
                ("t_build", C.c_double), ("t_partners", C.c_double), ("t_upward", C.c_double),
                ("t_downward", C.c_double)]


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        L.ccref_bruteforce.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_int32]
        L.ccref_bruteforce_targets.argtypes = [C.c_int64, _dp, _dp, C.c_int64, _ip, _dp, C.c_int32]
        L.ccref_fmm.argtypes = [C.c_int64, _dp, _dp, C.POINTER(Params), _dp, C.POINTER(Stats)]
        L.ccref_fmm_leaf.argtypes = [C.c_int64, _dp, _dp, C.POINTER(Params), C.c_void_p, C.c_void_p, _dp,
                                     C.POINTER(Stats)]
        L.ccref_tree_shape.argtypes = [C.c_int64, _dp, C.POINTER(Params), C.POINTER(Stats)]
        L.ccref_energy.argtypes = [C.c_int64, _dp, _dp]
        L.ccref_energy.restype = C.c_double
        L.ccref_ftable.argtypes = [C.c_int32] * 6
        L.ccref_ftable.restype = C.c_double
        L.ccref_dtensor.argtypes = [C.c_int32, _dp, _dp]
        L.ccref_p2m.argtypes = [C.c_int32, _dp, C.c_int64, _dp, _dp, _dp]
        L.ccref_charge_moments.argtypes = [C.c_int32, _dp, C.c_int64, _dp, _dp, _dp]
        L.ccref_m2m.argtypes = [C.c_int32, _dp, _dp, _dp]
        L.ccref_l2l.argtypes = [C.c_int32, _dp, _dp, _dp]
        L.ccref_m2l.argtypes = [C.c_int32, _dp, _dp, _dp]
        L.ccref_m2l_total.argtypes = [C.c_int32, _dp, _dp, _dp]
        L.ccref_l2p.argtypes = [C.c_int32, _dp, _dp, _dp]
        L.ccref_multipole_potential.argtypes = [C.c_int32, _dp, _dp]
        L.ccref_multipole_potential.restype = C.c_double
        L.ccref_local_potential.argtypes = [C.c_int32, _dp, _dp]
        L.ccref_local_potential.restype = C.c_double
        L.ccref_mlp_forward.argtypes = [C.c_int32] * 4 + [_dp, C.c_int64, _dp, _dp]
        L.ccref_mlp_loss_grad.argtypes = [C.c_int32] * 4 + [_dp, C.c_int64, _dp, _dp, _dp, C.c_void_p]
        L.ccref_mlp_loss_grad.restype = C.c_double
        _lib = L
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def make_params(order, theta, leaf_target=0.0, leaf_rule=0, box=None, nthreads=0, truncation=0):
    """truncation 0: multipoles and locals each to order p; 1: M2L terms of
    total degree |n| + |q| <= p only."""
    p = Params()
    p.order = int(order)
    p.theta = float(theta)
    p.leaf_target = float(leaf_target)
    p.leaf_rule = int(leaf_rule)
    if box is not None:
        p.has_box = 1
        for a in range(3):
            p.box_lo[a] = float(box[0][a])
            p.box_hi[a] = float(box[1][a])
    else:
        p.has_box = 0
    p.nthreads = int(nthreads)
    p.truncation = int(truncation)
    return p


def bruteforce(pos, m, nthreads=0):
    pos = _f64(pos, (-1, 3))
    m = _f64(m, (-1, 3))
    H = np.zeros_like(pos)
    rc = lib().ccref_bruteforce(pos.shape[0], pos, m, H, nthreads)
    if rc:
        raise ValueError("ccref_bruteforce: invalid input")
    return H


def bruteforce_targets(pos, m, idx, nthreads=0):
    pos = _f64(pos, (-1, 3))
    m = _f64(m, (-1, 3))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    H = np.zeros((idx.shape[0], 3))
    rc = lib().ccref_bruteforce_targets(pos.shape[0], pos, m, idx.shape[0], idx, H, nthreads)
    if rc:
        raise ValueError("ccref_bruteforce_targets: invalid input")
    return H


def _stats_dict(st):
    L = st.levels
    return {
        "levels": L,
        "split_axis": [st.split_axis[l] for l in range(1, L + 1)],
        "box_lo": list(st.box_lo), "box_hi": list(st.box_hi),
        "leaf_side": list(st.leaf_side), "s_used": st.s_used,
        "n_cells": st.n_cells, "n_leaves": st.n_leaves, "n_m2l_pairs": st.n_m2l_pairs,
        "n_p2p_leaf_pairs": st.n_p2p_leaf_pairs,
        "m2l_pairs_per_level": [st.m2l_pairs_per_level[l] for l in range(L + 1)],
        "t_build": st.t_build, "t_partners": st.t_partners, "t_upward": st.t_upward,
        "t_downward": st.t_downward,
    }


def fmm(pos, m, order, theta, leaf_target=0.0, leaf_rule=0, box=None, nthreads=0, return_stats=False,
        truncation=0):
    pos = _f64(pos, (-1, 3))
    m = _f64(m, (-1, 3))
    H = np.zeros_like(pos)
    st = Stats()
    prm = make_params(order, theta, leaf_target, leaf_rule, box, nthreads, truncation)
    rc = lib().ccref_fmm(pos.shape[0], pos, m, C.byref(prm), H, C.byref(st))
    if rc:
        raise ValueError("ccref_fmm: invalid input")
    if return_stats:
        return H, _stats_dict(st)
    return H


def fmm_leaf(pos, m, order, theta, leaf_p=None, leaf_theta=None, leaf_target=0.0, leaf_rule=0, box=None,
             nthreads=0, return_stats=False):
    """The FMM with per-smallest-cell order / opening angle, given per dipole."""
    pos = _f64(pos, (-1, 3))
    m = _f64(m, (-1, 3))
    H = np.zeros_like(pos)
    st = Stats()
    prm = make_params(order, theta, leaf_target, leaf_rule, box, nthreads)
    lp = None if leaf_p is None else np.ascontiguousarray(leaf_p, dtype=np.int32)
    lt = None if leaf_theta is None else np.ascontiguousarray(leaf_theta, dtype=np.float64)
    rc = lib().ccref_fmm_leaf(pos.shape[0], pos, m, C.byref(prm),
                              None if lp is None else lp.ctypes.data_as(C.c_void_p),
                              None if lt is None else lt.ctypes.data_as(C.c_void_p), H, C.byref(st))
    if rc:
        raise ValueError("ccref_fmm_leaf: invalid input")
    if return_stats:
        return H, _stats_dict(st)
    return H


def tree_shape(pos, order, theta=0.5, leaf_target=0.0, leaf_rule=0, box=None):
    pos = _f64(pos, (-1, 3))
    st = Stats()
    prm = make_params(order, theta, leaf_target, leaf_rule, box, 0)
    rc = lib().ccref_tree_shape(pos.shape[0], pos, C.byref(prm), C.byref(st))
    if rc:
        raise ValueError("ccref_tree_shape: invalid input")
    return _stats_dict(st)


def energy(m, H):
    m = _f64(m, (-1, 3))
    H = _f64(H, (-1, 3))
    return lib().ccref_energy(m.shape[0], m, H)


def ftable(k, q):
    return lib().ccref_ftable(int(k[0]), int(k[1]), int(k[2]), int(q[0]), int(q[1]), int(q[2]))


def dtensor(K, c):
    D = np.zeros((K + 1,) * 3)
    rc = lib().ccref_dtensor(K, _f64(c), D)
    if rc:
        raise ValueError("ccref_dtensor: bad order")
    return D


def p2m(p, center, pos, m):
    pos = _f64(pos, (-1, 3))
    Q = np.zeros((p + 1,) * 3)
    lib().ccref_p2m(p, _f64(center), pos.shape[0], pos, _f64(m, (-1, 3)), Q)
    return Q


def charge_moments(p, center, pos, q):
    pos = _f64(pos, (-1, 3))
    Q = np.zeros((p + 1,) * 3)
    lib().ccref_charge_moments(p, _f64(center), pos.shape[0], pos, _f64(q), Q)
    return Q


def m2m(p, c, Qchild, Qparent=None):
    Qp = np.zeros((p + 1,) * 3) if Qparent is None else _f64(Qparent).copy()
    lib().ccref_m2m(p, _f64(c), _f64(Qchild), Qp)
    return Qp


def l2l(p, c, Vparent):
    Vc = np.zeros((p + 1,) * 3)
    lib().ccref_l2l(p, _f64(c), _f64(Vparent), Vc)
    return Vc


def m2l(p, c, Q, V=None, total=False):
    Vo = np.zeros((p + 1,) * 3) if V is None else _f64(V).copy()
    (lib().ccref_m2l_total if total else lib().ccref_m2l)(p, _f64(c), _f64(Q), Vo)
    return Vo


def l2p(p, V, y):
    H = np.zeros(3)
    lib().ccref_l2p(p, _f64(V), _f64(y), H)
    return H


def multipole_potential(p, Q, x):
    return lib().ccref_multipole_potential(p, _f64(Q), _f64(x))


def local_potential(p, V, y):
    return lib().ccref_local_potential(p, _f64(V), _f64(y))


def mlp_param_count(nin, h1, h2, nout):
    return h1 * nin + h1 + h2 * h1 + h2 + nout * h2 + nout


def mlp_forward(params, x, nin, h1, h2, nout):
    x = _f64(x, (-1, nin))
    y = np.zeros((x.shape[0], nout))
    lib().ccref_mlp_forward(nin, h1, h2, nout, _f64(params), x.shape[0], x, y)
    return y


def mlp_loss_grad(params, x, t, mask, nin, h1, h2, nout):
    x = _f64(x, (-1, nin))
    t = _f64(t, (-1, nout))
    mask = _f64(mask, (-1, nout))
    g = np.zeros(mlp_param_count(nin, h1, h2, nout))
    loss = lib().ccref_mlp_loss_grad(nin, h1, h2, nout, _f64(params), x.shape[0], x, t, mask,
                                     g.ctypes.data_as(C.c_void_p))
    return loss, g


def rel_rms(H, Href):
    """Relative RMS error sqrt(sum |H - Href|^2 / sum |Href|^2) over all entries."""
    H = np.asarray(H, dtype=np.float64)
    Href = np.asarray(Href, dtype=np.float64)
    return float(np.sqrt(np.sum((H - Href) ** 2) / np.sum(Href ** 2)))
