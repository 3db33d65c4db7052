"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (autotuned M2L, device buffers, graph replay).

* Ferrofluid, 2^20 dipoles, p = 6, theta = 0.5: structure bit-exact and the
  whole FP64 field within 1e-10 of the oracle FMM; mixed within 1e-5 of FP64.
* Sphere cut, 2^18 sites x 64 configurations, p = 5: configurations 0 and 63
  of the FP64 batch within 1e-10 of the oracle; mixed within 1e-5 of FP64.
* Thin film with holes (1024 x 1024 x 16 lattice, 16 holes, 8 configurations,
  p = 6, theta = 0.4): tree shape equal to the oracle's, mixed within 1e-5 of
  FP64, both within 2e-5 of the oracle's direct sum at sampled dipoles; the
  learned per-cell parameters of the film weights within 1e-5 of fixed FP64
  and of the direct sum.
* Reduced film (256 x 128 x 16, 4 holes): FP64 within 1e-10 of the oracle
  FMM, structure bit-exact; mixed x 8 per dipole against the oracle; the
  learned per-cell parameters in FP64 within 1e-10 of the oracle's per-cell
  FMM.
* Mixed precision against the oracle per dipole (ferrofluid, sphere, films):
  99th percentile of |dH|/|H| <= 1e-5, largest |dH| <= 1e-4 of the RMS field.

The direct-sum bar: the method's own error at these (p, theta) is a few
1e-6 on these inputs (the oracle FMM shows the same); 2e-5 is the stated
bound of the truncation error here, the 1e-5 bar is for precision only.
"""
import numpy as np
import pytest

from paper_0810_0233_amd import ccfmm, inputs, selector
from parity_bars import check_per_dipole

pytestmark = pytest.mark.gpu

FP64_BAR = 1e-10
MIXED_BAR = 1e-5
TRUNC_BAR = 2e-5


def rel_rms(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def run_device(c, precision, nb=None):
    """Plan on device positions, autotune, two graph-replayed evaluations."""
    import torch

    pos, box, m = c["pos"], c["box"], c["m"]
    nb = nb or m.shape[0]
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    d_pos = torch.from_numpy(pos).to(dev)
    d_m = torch.from_numpy(np.ascontiguousarray(m[:nb])).to(dev)
    d_H = torch.empty_like(d_m)
    prm = ccfmm.params(order=c["order"], theta=c["theta"], leaf_target=0.0, box=box, precision=precision,
                       max_batch=nb)
    pl = ccfmm.Plan.create_device(pos.shape[0], d_pos.data_ptr(), prm, st)
    pl.autotune(nb, d_m.data_ptr(), d_H.data_ptr(), st)
    pl.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), st)
    pl.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), st)
    torch.cuda.synchronize()
    H = d_H.cpu().numpy()
    info = pl.info()
    pl.destroy()
    return H, info


def test_ferrofluid_full_size(ref):
    c = inputs.config_ferrofluid()
    pos, box, m = c["pos"], c["box"], c["m"][0]
    print("case ferrofluid n=%d p=6 theta=0.5" % pos.shape[0], flush=True)
    H64, inf = run_device(c, ccfmm.PREC_FP64)
    Hmx, _ = run_device(c, ccfmm.PREC_MIXED)
    H_ref, st = ref.fmm(pos, m, 6, 0.5, box=box, return_stats=True)
    assert inf["levels"] == st["levels"] == 15
    assert inf["split_axis"] == st["split_axis"]
    assert inf["n_leaves"] == st["n_leaves"]
    assert inf["m2l_pairs_per_level"] == st["m2l_pairs_per_level"]
    assert inf["n_p2p_leaf_pairs"] == st["n_p2p_leaf_pairs"]
    e64 = rel_rms(H64[0], H_ref)
    emx = rel_rms(Hmx[0], H64[0])
    idx = np.sort(np.random.default_rng(5).choice(pos.shape[0], 512, replace=False)).astype(np.int64)
    Hd = ref.bruteforce_targets(pos, m, idx)
    et = rel_rms(Hmx[0][idx], Hd)
    print("fp64 vs oracle %.3e, mixed vs fp64 %.3e, mixed vs direct %.3e" % (e64, emx, et), flush=True)
    assert e64 <= FP64_BAR
    assert emx <= MIXED_BAR
    assert et <= TRUNC_BAR
    check_per_dipole(Hmx[0], H_ref, "ferrofluid mixed")


def test_sphere_batched_full_size(ref):
    c = inputs.config_sphere()
    pos, box, m = c["pos"], c["box"], c["m"]
    print("case sphere n=%d x %d p=5 theta=0.5" % (pos.shape[0], m.shape[0]), flush=True)
    H64, inf = run_device(c, ccfmm.PREC_FP64)
    Hmx, _ = run_device(c, ccfmm.PREC_MIXED)
    for b in (0, m.shape[0] - 1):
        H_ref = ref.fmm(pos, m[b], 5, 0.5, box=box)
        e = rel_rms(H64[b], H_ref)
        print("configuration %d: fp64 vs oracle %.3e" % (b, e), flush=True)
        assert e <= FP64_BAR
        check_per_dipole(Hmx[b], H_ref, "sphere configuration %d mixed" % b)
    emx = rel_rms(Hmx, H64)
    print("mixed vs fp64 over %d configurations %.3e" % (m.shape[0], emx), flush=True)
    assert emx <= MIXED_BAR


def test_film_full_size(ref):
    c = inputs.config_film()
    pos, box, m = c["pos"], c["box"], c["m"]
    n = pos.shape[0]
    print("case film n=%d x %d p=6 theta=0.4" % (n, m.shape[0]), flush=True)
    shape = ref.tree_shape(pos, 6, 0.4, box=box)
    Hmx, inf = run_device(c, ccfmm.PREC_MIXED)
    assert inf["levels"] == shape["levels"]
    assert inf["split_axis"] == shape["split_axis"]
    H64, _ = run_device(c, ccfmm.PREC_FP64)
    emx = rel_rms(Hmx, H64)
    idx = np.sort(np.random.default_rng(6).choice(n, 256, replace=False)).astype(np.int64)
    Hd = ref.bruteforce_targets(pos, m[0], idx)
    e64 = rel_rms(H64[0][idx], Hd)
    et = rel_rms(Hmx[0][idx], Hd)
    print("mixed vs fp64 %.3e, fp64 vs direct %.3e, mixed vs direct %.3e" % (emx, e64, et), flush=True)
    assert emx <= MIXED_BAR
    assert e64 <= TRUNC_BAR and et <= TRUNC_BAR
    # learned per-cell parameters (the package's film weights), judged against
    # fixed (6, 0.4): within the 1e-5 bound of the fixed field and of the
    # oracle's direct sum at the sampled dipoles
    import torch

    st = torch.cuda.current_stream().cuda_stream
    d_pos = torch.from_numpy(pos).cuda()
    d_m = torch.from_numpy(np.ascontiguousarray(m)).cuda()
    d_H = torch.empty_like(d_m)
    prm = ccfmm.params(order=6, theta=0.4, box=box, precision=ccfmm.PREC_MIXED, max_batch=m.shape[0], selector=1,
                       err_bound=MIXED_BAR)
    pl = ccfmm.Plan.create_device(n, d_pos.data_ptr(), prm, st)
    import os

    assert pl.selector_load(os.path.join(selector.WEIGHTS_DIR, selector.FILM_WEIGHTS)) == ccfmm.OK
    rc = pl.eval_device(m.shape[0], d_m.data_ptr(), d_H.data_ptr(), st)
    torch.cuda.synchronize()
    inf = pl.info()
    Hl = d_H.cpu().numpy()
    el = rel_rms(Hl[0][idx], Hd)
    print("learned: status %d judge %.3e vs fixed fp64 %.3e vs direct %.3e" % (
        rc, inf["judge_err"], rel_rms(Hl, H64), el), flush=True)
    assert rc == ccfmm.OK and inf["learned"] == 1
    assert inf["judge_err"] <= MIXED_BAR and rel_rms(Hl, H64) <= MIXED_BAR and el <= MIXED_BAR
    pl.destroy()


def test_film_reduced_matches_oracle(ref):
    """A film of the same recipe at 256 x 128 x 16 sites with four holes (the
    smallest cells 2 x 4 x 4 sites, top cells 16:8:1 flat): FP64 against the
    oracle FMM at (6, 0.4) with the structure bit-exact; 8 configurations in
    mixed precision (the few-configuration near field) against the oracle
    per dipole; the per-cell parameters the film weights choose, in FP64,
    against the oracle's per-cell FMM."""
    import os

    pos, box = inputs.film_with_holes(256, 128, 16, 4, 5201, rmin=10.0, rmax=30.0)
    n = pos.shape[0]
    m = np.stack([inputs.random_moments(n, 5202 + b) for b in range(8)])
    c = dict(pos=pos, box=box, m=m, order=6, theta=0.4)
    print("case film 256x128x16 n=%d x 8" % n, flush=True)
    H64, inf = run_device(c, ccfmm.PREC_FP64, nb=1)
    H_ref, st = ref.fmm(pos, m[0], 6, 0.4, box=box, return_stats=True)
    assert inf["levels"] == st["levels"] and inf["split_axis"] == st["split_axis"]
    assert inf["n_leaves"] == st["n_leaves"]
    assert inf["m2l_pairs_per_level"] == st["m2l_pairs_per_level"]
    assert inf["n_p2p_leaf_pairs"] == st["n_p2p_leaf_pairs"]
    assert np.allclose(inf["leaf_side"], [2.0, 4.0, 4.0])
    e64 = rel_rms(H64[0], H_ref)
    print("fp64 vs oracle %.3e" % e64, flush=True)
    assert e64 <= FP64_BAR
    Hmx, _ = run_device(c, ccfmm.PREC_MIXED)
    assert rel_rms(Hmx[0], H_ref) <= MIXED_BAR
    check_per_dipole(Hmx[0], H_ref, "reduced film configuration 0 mixed")
    H_ref7 = ref.fmm(pos, m[7], 6, 0.4, box=box)
    check_per_dipole(Hmx[7], H_ref7, "reduced film configuration 7 mixed")
    # per-cell parameters chosen by the film weights on this geometry, in FP64
    import torch

    prm = ccfmm.params(order=6, theta=0.4, box=box, precision=ccfmm.PREC_FP64, max_batch=1, selector=1,
                       err_bound=MIXED_BAR)
    pl = ccfmm.Plan.create(pos, prm)
    assert pl.selector_load(os.path.join(selector.WEIGHTS_DIR, selector.FILM_WEIGHTS)) == ccfmm.OK
    Hl = pl.eval(m[0])
    li = pl.info()
    p, th = pl.get_leaf_params()
    ids = torch.empty(n, dtype=torch.int32, device="cuda:0")
    pl.leaf_ids(ids.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ids = ids.cpu().numpy()
    print("reduced film learned: status %d learned %d judge %.3e choices %s" % (
        pl.last_status, li["learned"], li["judge_err"],
        sorted(set(zip(p.tolist(), np.round(th, 1).tolist())))), flush=True)
    H_leaf, sl = ref.fmm_leaf(pos, m[0], 6, 0.4, leaf_p=p[ids], leaf_theta=th[ids], box=box, return_stats=True)
    if li["learned"]:
        assert li["m2l_pairs_per_level"] == sl["m2l_pairs_per_level"]
        assert li["n_p2p_leaf_pairs"] == sl["n_p2p_leaf_pairs"]
    assert rel_rms(Hl, H_leaf) <= FP64_BAR
    pl.destroy()
