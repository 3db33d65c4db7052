"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bars (written here, derived in the design notes):
* FP64 plan: whole-FMM relative RMS vs the oracle FMM at the same (p, theta, s)
  <= 1e-10 (the two differ only by summation order and the scaled-unit
  roundings, ~1e-15 per operation); discrete structure (levels, split axes,
  occupied cells, list sizes per level) bit-exact.
* theta -> 0 (everything near): vs brute force <= 1e-12.
* MIXED plan: vs the FP64 GPU plan <= 1e-5 relative RMS.
"""
import numpy as np
import pytest

from paper_0810_0233_amd import ccfmm, inputs
from parity_bars import check_per_dipole

pytestmark = pytest.mark.gpu

FP64_BAR = 1e-10
MIXED_BAR = 1e-5
def rel_rms(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


@pytest.fixture(scope="module")
def ref():
    import oracle

    return oracle


def plan_for(pos, order, theta, leaf_target=0.0, box=None, precision=ccfmm.PREC_FP64, max_batch=1, **kw):
    prm = ccfmm.params(order=order, theta=theta, leaf_target=leaf_target, box=box, precision=precision,
                       max_batch=max_batch, **kw)
    return ccfmm.Plan.create(pos, prm)


def test_mfma_operand_layout():
    assert ccfmm.selftest_mfma(0) == ccfmm.OK


def test_lattice_1000_fp64_matches_oracle(ref):
    c = inputs.config_lattice_1000()
    pos, m = c["pos"], c["m"][0]
    print("case lattice_1000 p=4 theta=0.5 s=8", flush=True)
    H_ref, st = ref.fmm(pos, m, 4, 0.5, leaf_target=8, box=c["box"], return_stats=True)
    pl = plan_for(pos, 4, 0.5, 8, c["box"])
    inf = pl.info()
    assert inf["levels"] == st["levels"] == 7
    assert inf["split_axis"] == st["split_axis"]
    assert inf["leaf_side"] == st["leaf_side"]
    assert inf["n_leaves"] == st["n_leaves"]
    assert inf["m2l_pairs_per_level"] == st["m2l_pairs_per_level"]
    assert inf["n_p2p_leaf_pairs"] == st["n_p2p_leaf_pairs"]
    H = pl.eval(m)
    assert rel_rms(H, H_ref) <= FP64_BAR
    Hb = ref.bruteforce(pos, m)
    assert rel_rms(H, Hb) < 2e-4  # the truncation error of (4, 0.5), as the oracle has it


def test_theta_to_zero_is_bruteforce(ref):
    c = inputs.config_lattice_1000()
    pos, m = c["pos"], c["m"][0]
    pl = plan_for(pos, 4, 1e-3, 8, c["box"])
    assert pl.info()["n_m2l_pairs"] == 0
    H = pl.eval(m)
    assert rel_rms(H, ref.bruteforce(pos, m)) <= 1e-12


@pytest.mark.parametrize("order", [1, 2, 3, 5, 6, 7, 8])
def test_orders_fp64_match_oracle(ref, order):
    pos, box = inputs.lattice(12, 12, 12)
    m = inputs.random_moments(pos.shape[0], 77 + order)
    print("case lattice12 order=%d" % order, flush=True)
    H_ref, st = ref.fmm(pos, m, order, 0.5, leaf_target=8, box=box, return_stats=True)
    pl = plan_for(pos, order, 0.5, 8, box)
    assert pl.info()["m2l_pairs_per_level"] == st["m2l_pairs_per_level"]
    assert rel_rms(pl.eval(m), H_ref) <= FP64_BAR


@pytest.mark.parametrize("theta", [0.3, 0.45, 0.7])
def test_ferrofluid_fp64_matches_oracle(ref, theta):
    pos, box = inputs.ferrofluid(6000, 2001)
    m = inputs.random_moments(6000, 2002)
    print("case ferrofluid6000 theta=%g" % theta, flush=True)
    H_ref, st = ref.fmm(pos, m, 6, theta, box=box, return_stats=True)
    pl = plan_for(pos, 6, theta, 0.0, box)
    inf = pl.info()
    assert inf["levels"] == st["levels"]
    assert inf["m2l_pairs_per_level"] == st["m2l_pairs_per_level"]
    assert inf["n_p2p_leaf_pairs"] == st["n_p2p_leaf_pairs"]
    assert rel_rms(pl.eval(m), H_ref) <= FP64_BAR


def test_bounding_box_and_clusters(ref):
    pos, _ = inputs.clusters(6, 700, 4001, box_side=128.0)
    m = inputs.random_moments(pos.shape[0], 4002)
    H_ref, st = ref.fmm(pos, m, 5, 0.4, return_stats=True)  # tight bounding box
    pl = plan_for(pos, 5, 0.4)
    assert pl.info()["box_lo"] == st["box_lo"]
    assert pl.info()["n_leaves"] == st["n_leaves"]
    assert rel_rms(pl.eval(m), H_ref) <= FP64_BAR


def test_mixed_precision_vs_fp64(ref):
    pos, box = inputs.ferrofluid(20000, 2001)
    m = inputs.random_moments(20000, 2002)
    H64 = plan_for(pos, 6, 0.5, 0.0, box).eval(m)
    H32 = plan_for(pos, 6, 0.5, 0.0, box, precision=ccfmm.PREC_MIXED).eval(m)
    e = rel_rms(H32, H64)
    print("mixed vs fp64 rel rms = %.3e" % e, flush=True)
    assert e <= MIXED_BAR
    H_ref = ref.fmm(pos, m, 6, 0.5, box=box)
    assert rel_rms(H64, H_ref) <= FP64_BAR
    check_per_dipole(H32, H_ref, "ferrofluid 20000 mixed")


def test_batched_equals_single(ref):
    pos, box = inputs.sphere_cut(3000, 20)
    mb = inputs.aligned_moments(3000, 5, 3000)
    pl = plan_for(pos, 5, 0.5, 0.0, box, max_batch=8)
    Hb = pl.eval(mb)
    for b in range(5):
        Hs = pl.eval(mb[b:b + 1])[0]
        assert rel_rms(Hb[b], Hs) <= 1e-14
        if b in (0, 4):
            assert rel_rms(Hb[b], ref.fmm(pos, mb[b], 5, 0.5, box=box)) <= FP64_BAR


def test_maximum_batch(ref):
    """The largest batch a plan accepts, 4096 configurations in one launch:
    FP64 configurations equal the same configuration evaluated alone (to
    summation order) and the oracle at the first and last; the mixed plan
    (matrix-core near field over 64 column blocks) stays within the mixed bar
    of FP64 on every configuration."""
    n, nb = 1500, 4096
    pos, box = inputs.sphere_cut(n, 16)
    mb = inputs.aligned_moments(n, nb, 4100)
    print("case maximum batch fp64 n=%d nb=%d" % (n, nb), flush=True)
    pl = plan_for(pos, 4, 0.5, 0.0, box, max_batch=nb)
    Hb = pl.eval(mb)
    for b in (0, 1, 2047, nb - 1):
        Hs = pl.eval(mb[b:b + 1])[0]
        assert rel_rms(Hb[b], Hs) <= 1e-14
    for b in (0, nb - 1):
        assert rel_rms(Hb[b], ref.fmm(pos, mb[b], 4, 0.5, box=box)) <= FP64_BAR
    pl.destroy()
    print("case maximum batch mixed n=%d nb=%d" % (n, nb), flush=True)
    pm = plan_for(pos, 4, 0.5, 0.0, box, precision=ccfmm.PREC_MIXED, max_batch=nb)
    Hm = pm.eval(mb)
    pm.destroy()
    err = np.sqrt(np.sum((Hm - Hb) ** 2, axis=(1, 2)) / np.sum(Hb ** 2, axis=(1, 2)))
    print("maximum batch: worst mixed vs fp64 %.3e" % err.max(), flush=True)
    assert err.max() <= MIXED_BAR


def test_default_m2l_variant_is_chosen_per_plan(ref):
    """With no variant named, a plan gets the 64-column wide kernel where the
    order, precision and form allow it (p <= 8 in the traceless form, FP64
    included; mixed p <= 6 in the full form) and the block kernel elsewhere
    (FP64 full form, mixed p > 6 full form), and the field is that of the
    named variant."""
    pos, box = inputs.ferrofluid(3000, 77)
    m = inputs.random_moments(3000, 78)
    cases = ((ccfmm.PREC_MIXED, 6, 1, 4), (ccfmm.PREC_MIXED, 8, 1, 4), (ccfmm.PREC_MIXED, 8, 0, 0),
             (ccfmm.PREC_FP64, 6, 1, 4), (ccfmm.PREC_FP64, 8, 1, 4), (ccfmm.PREC_FP64, 6, 0, 0))
    for prec, order, red, want in cases:
        print("case default variant precision=%d order=%d traceless=%d" % (prec, order, red), flush=True)
        pd = plan_for(pos, order, 0.5, 0.0, box, precision=prec, m2l_traceless=red)
        assert pd.info()["m2l_variant"] == want
        Hd = pd.eval(m)
        pd.destroy()
        pn = plan_for(pos, order, 0.5, 0.0, box, precision=prec, m2l_traceless=red, m2l_variant=want)
        Hn = pn.eval(m)
        pn.destroy()
        assert rel_rms(Hd, Hn) <= 1e-14


def test_edge_cases(ref):
    # one dipole: no field
    pl = plan_for(np.array([[0.3, 0.2, 0.1]]), 3, 0.5)
    np.testing.assert_array_equal(pl.eval(np.array([[1.0, 0, 0]])), 0.0)
    # two coincident dipoles and one apart
    pos = np.array([[0.0, 0, 0], [0.0, 0, 0], [1.0, 0, 0]])
    m = np.array([[0, 0, 1.0], [0, 1.0, 0], [1.0, 0, 0]])
    H = plan_for(pos, 3, 0.5).eval(m)
    np.testing.assert_allclose(H, ref.bruteforce(pos, m), rtol=1e-14, atol=1e-15)
    # ragged occupancy: a dense blob plus a few far points (leaf chunks > 64)
    rng = np.random.default_rng(3)
    pos = np.concatenate([rng.normal(size=(900, 3)) * 0.5, rng.uniform(-40, 40, size=(60, 3))])
    m = inputs.unit_moments(960, rng)
    H_ref = ref.fmm(pos, m, 4, 0.5, leaf_target=20)
    assert rel_rms(plan_for(pos, 4, 0.5, 20).eval(m), H_ref) <= FP64_BAR


def test_device_path_and_determinism():
    import torch

    pos, box = inputs.ferrofluid(5000, 11)
    m = inputs.random_moments(5000, 12)
    dev = torch.device("cuda:0")
    d_pos = torch.from_numpy(pos).to(dev)
    d_m = torch.from_numpy(m).to(dev)
    d_H = torch.empty_like(d_m)
    st = torch.cuda.current_stream().cuda_stream
    prm = ccfmm.params(order=5, theta=0.5, box=box)
    pl = ccfmm.Plan.create_device(5000, d_pos.data_ptr(), prm, st)
    pl.eval_device(1, d_m.data_ptr(), d_H.data_ptr(), st)
    torch.cuda.synchronize()
    H1 = d_H.cpu().numpy().copy()
    pl.eval_device(1, d_m.data_ptr(), d_H.data_ptr(), st)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(d_H.cpu().numpy(), H1)  # FP64 path is bitwise repeatable
    H_host = ccfmm.Plan.create(pos, prm).eval(m)
    np.testing.assert_array_equal(H_host, H1)
    # moving the dipoles and rebuilding in place gives the fresh-plan answer
    pos2 = pos + 0.01
    d_pos.copy_(torch.from_numpy(pos2))
    prm2 = ccfmm.params(order=5, theta=0.5)
    pl2 = ccfmm.Plan.create_device(5000, d_pos.data_ptr(), prm2, st)
    pl2.eval_device(1, d_m.data_ptr(), d_H.data_ptr(), st)
    torch.cuda.synchronize()
    Ha = d_H.cpu().numpy().copy()
    pl3 = ccfmm.Plan.create_device(5000, torch.from_numpy(pos).to(dev).data_ptr(), prm2, st)
    pl3.update_positions_device(d_pos.data_ptr(), st)
    pl3.eval_device(1, d_m.data_ptr(), d_H.data_ptr(), st)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(d_H.cpu().numpy(), Ha)


def test_direct_targets_matches_oracle(ref):
    import torch

    pos, _ = inputs.ferrofluid(4000, 5)
    m = inputs.random_moments(4000, 6)
    idx = np.array([0, 17, 3999, 2000], dtype=np.int64)
    dev = torch.device("cuda:0")
    d_pos = torch.from_numpy(pos).to(dev)
    d_m = torch.from_numpy(m).to(dev)
    d_idx = torch.from_numpy(idx).to(dev)
    d_H = torch.zeros((4, 3), dtype=torch.float64, device=dev)
    ccfmm.direct_targets_device(4000, d_pos.data_ptr(), d_m.data_ptr(), 4, d_idx.data_ptr(), d_H.data_ptr(),
                                torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    np.testing.assert_allclose(d_H.cpu().numpy(), ref.bruteforce_targets(pos, m, idx), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("precision", [ccfmm.PREC_FP64, ccfmm.PREC_MIXED])
def test_m2l_variants_and_autotune_agree(ref, precision):
    """Every M2L kernel (the block and wavefront kernels on the full operator,
    the wide kernels on the traceless one, in FP64 too), every target
    grouping and the autotuner's pick (kernel, grouping and evaluation form)
    give the same fields; FP64 matches the oracle.  FP64 bar between variants 1e-13: the traceless form adds folded
    moments and sums 48 instead of 83 terms per row, a different rounding of
    the same sums (1e-16 per operation)."""
    import torch

    pos, box = inputs.ferrofluid(12000, 21)
    m = inputs.random_moments(12000, 22)
    base = None
    variants = (0, 1, 2, 3, 4)
    for variant in variants:
        for cb in (0, 3, 6):
            H = plan_for(pos, 6, 0.5, 0.0, box, precision=precision, m2l_variant=variant,
                         m2l_class_bits=cb).eval(m)
            if base is None:
                base = H
            else:
                assert rel_rms(H, base) <= (1e-13 if precision == ccfmm.PREC_FP64 else 1e-6)
            if precision == ccfmm.PREC_FP64 and cb == 3:
                assert rel_rms(H, ref.fmm(pos, m, 6, 0.5, box=box)) <= FP64_BAR
    if precision == ccfmm.PREC_FP64:
        assert rel_rms(base, ref.fmm(pos, m, 6, 0.5, box=box)) <= FP64_BAR
    dev = torch.device("cuda:0")
    d_m = torch.from_numpy(m).to(dev)
    d_H = torch.empty_like(d_m)
    st = torch.cuda.current_stream().cuda_stream
    pl = plan_for(pos, 6, 0.5, 0.0, box, precision=precision)
    res = pl.autotune(1, d_m.data_ptr(), d_H.data_ptr(), st)
    assert len(res) == 3 * len(variants) and all(r["m2l_ms"] > 0 for r in res)
    inf = pl.info()
    best = min(res, key=lambda r: r["m2l_ms"])
    assert (inf["m2l_variant"], inf["m2l_class_bits"]) == (best["variant"], best["class_bits"])
    # the evaluation form: both timed, the faster kept
    t_beside, t_one = inf["tune_eval_ms"]
    assert t_beside > 0 and t_one > 0
    assert inf["overlap_near"] == (1 if t_beside <= t_one else 0)
    pl.eval_device(1, d_m.data_ptr(), d_H.data_ptr(), st)
    torch.cuda.synchronize()
    assert rel_rms(d_H.cpu().numpy(), base) <= (1e-13 if precision == ccfmm.PREC_FP64 else 1e-6)


@pytest.mark.parametrize("order", [2, 3, 4, 5, 6, 7, 8])
def test_wide_m2l_variants(order):
    """The wide FP32 M2L kernels (128- and 256-column tiles, permuted
    contraction order) equal the block kernel for several orders and a batch
    that splits tiles into (cell, configuration) columns; the FP64 wide
    kernel (traceless form) equals the FP64 block kernel (full form)."""
    pos, box = inputs.ferrofluid(9000, 31 + order)
    nb = 3
    m = np.stack([inputs.random_moments(9000, 40 + order + b) for b in range(nb)])
    H = {}
    for variant in (0, 2, 3, 4):
        pl = plan_for(pos, order, 0.5, 0.0, box, precision=ccfmm.PREC_MIXED, max_batch=nb, m2l_variant=variant,
                      m2l_class_bits=3)
        assert pl.info()["m2l_variant"] == variant
        H[variant] = pl.eval(m)
        pl.destroy()
    errs = {v: rel_rms(H[v], H[0]) for v in (2, 3, 4)}
    print("order %d wide-vs-block %s" % (order, errs), flush=True)
    for variant in (2, 3, 4):
        assert errs[variant] <= 1e-6
    # the full (83 x 84 at p = 6) operator in the wide kernels: the same sums,
    # rounded differently from the traceless (folded) form used by default
    for variant in ((2, 4) if order <= 6 else ()):  # the full form's wide kernels stop at order 6
        pl = plan_for(pos, order, 0.5, 0.0, box, precision=ccfmm.PREC_MIXED, max_batch=nb, m2l_variant=variant,
                      m2l_class_bits=3, m2l_traceless=0)
        e = rel_rms(pl.eval(m), H[variant])
        print("order %d variant %d traceless-vs-full %.3e" % (order, variant, e), flush=True)
        assert e <= 1e-6
        pl.destroy()
    # FP64: the wide kernels in the traceless form; in the full form a plan
    # asking for them gets the block kernel; the two agree to FP64 rounding
    p64 = plan_for(pos, order, 0.5, 0.0, box, precision=ccfmm.PREC_FP64, max_batch=nb, m2l_variant=2)
    assert p64.info()["m2l_variant"] == 2
    p64f = plan_for(pos, order, 0.5, 0.0, box, precision=ccfmm.PREC_FP64, max_batch=nb, m2l_variant=2,
                    m2l_traceless=0)
    assert p64f.info()["m2l_variant"] == 0
    H64 = p64.eval(m)
    e64 = rel_rms(H64, p64f.eval(m))
    print("order %d fp64 wide traceless vs block full %.3e" % (order, e64), flush=True)
    assert e64 <= 1e-13
    p64f.destroy()
    if order > 6:  # the full form's wide kernels stop at order 6: such a plan gets the block kernel
        pf = plan_for(pos, order, 0.5, 0.0, box, precision=ccfmm.PREC_MIXED, max_batch=nb, m2l_variant=2,
                      m2l_traceless=0)
        assert pf.info()["m2l_variant"] == 0
        pf.destroy()
    assert rel_rms(H[2], H64) <= MIXED_BAR
    p64.destroy()


@pytest.mark.parametrize("precision", [ccfmm.PREC_FP64, ccfmm.PREC_MIXED])
def test_batched_matrix_core_near_field(ref, precision):
    """40 configurations (the matrix-core near field) equal one-at-a-time
    evaluations, and the FP64 form matches the oracle per configuration."""
    pos, box = inputs.sphere_cut(4000, 20)
    nb = 40
    mb = inputs.aligned_moments(4000, nb, 3000)
    pl = plan_for(pos, 5, 0.5, 0.0, box, precision=precision, max_batch=nb)
    Hb = pl.eval(mb)
    single = plan_for(pos, 5, 0.5, 0.0, box, precision=precision, max_batch=1)
    for b in (0, 7, 39):
        Hs = single.eval(mb[b:b + 1])[0]
        e = rel_rms(Hb[b], Hs)
        print("batched vs single b=%d: %.3e" % (b, e), flush=True)
        assert e <= (1e-13 if precision == ccfmm.PREC_FP64 else 2e-6)
        if b != 7:
            H_ref = ref.fmm(pos, mb[b], 5, 0.5, box=box)
            if precision == ccfmm.PREC_FP64:
                assert rel_rms(Hb[b], H_ref) <= FP64_BAR
            else:
                check_per_dipole(Hb[b], H_ref, "matrix-core near field b=%d" % b)


@pytest.mark.parametrize("leaf_target", [0.0, 90.0])
def test_matrix_core_near_field_ragged(ref, leaf_target):
    """The FP32 matrix-core near field with 70 configurations (a full and a
    partial 64-column block) and, with about 90 dipoles per smallest cell,
    cells split into several 32-target chunks and source blocks that straddle
    cells: every configuration equals its one-at-a-time evaluation, and the
    batch is within the mixed bar of the FP64 batch, which matches the oracle."""
    pos, box = inputs.sphere_cut(6000, 24)
    nb = 70
    mb = inputs.aligned_moments(6000, nb, 3100)
    print("case sphere_cut 6000 nb=70 leaf_target=%g" % leaf_target, flush=True)
    pm = plan_for(pos, 4, 0.5, leaf_target, box, precision=ccfmm.PREC_MIXED, max_batch=nb)
    Hm = pm.eval(mb)
    info = pm.info()
    pm.destroy()
    p64 = plan_for(pos, 4, 0.5, leaf_target, box, precision=ccfmm.PREC_FP64, max_batch=nb)
    H64 = p64.eval(mb)
    p64.destroy()
    single = plan_for(pos, 4, 0.5, leaf_target, box, precision=ccfmm.PREC_MIXED, max_batch=1)
    for b in (0, 33, 63, 64, 69):
        e = rel_rms(Hm[b], single.eval(mb[b:b + 1])[0])
        print("leaves %d, b=%d batched vs single %.3e" % (info["n_leaves"], b, e), flush=True)
        assert e <= 2e-6
    single.destroy()
    assert rel_rms(Hm, H64) <= MIXED_BAR
    for b in (0, 69):
        assert rel_rms(H64[b], ref.fmm(pos, mb[b], 4, 0.5, box=box, leaf_target=leaf_target)) <= FP64_BAR


def test_graph_replays_match_eager():
    """The captured evaluation, replayed with new moments in the same buffers and
    eager work in between, equals the uncaptured evaluation every time."""
    import torch

    pos, box = inputs.ferrofluid(8000, 31)
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    d_pos = torch.from_numpy(pos).to(dev)
    nb = 3
    d_m = torch.empty((nb, 8000, 3), dtype=torch.float64, device=dev)
    d_H = torch.empty_like(d_m)
    d_Hr = torch.empty_like(d_m)
    graphed = ccfmm.Plan.create_device(8000, d_pos.data_ptr(), ccfmm.params(order=5, theta=0.5, box=box,
                                                                              max_batch=nb, use_graph=1), st)
    eager = ccfmm.Plan.create_device(8000, d_pos.data_ptr(), ccfmm.params(order=5, theta=0.5, box=box,
                                                                            max_batch=nb, use_graph=0), st)
    for rep in range(4):
        m = np.stack([inputs.random_moments(8000, 100 * rep + b) for b in range(nb)])
        d_m.copy_(torch.from_numpy(m))
        junk = torch.randn(1 << 20, device=dev).sum()  # unrelated eager work between replays
        graphed.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), st)
        eager.eval_device(nb, d_m.data_ptr(), d_Hr.data_ptr(), st)
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        np.testing.assert_array_equal(d_H.cpu().numpy(), d_Hr.cpu().numpy())


def close_pair_geometry(seed=3):
    """A 16^3 lattice plus partners at 1e-5..1e-3 (lattice units) from random
    sites, and pairs straddling the plane x = 1.5 (a cell face for cell sides
    that divide 2): the close pairs that FP32 positions alone cannot resolve."""
    rng = np.random.default_rng(seed)
    base, box = inputs.lattice(16, 16, 16)
    k = 512
    pick = rng.choice(base.shape[0], k, replace=False)
    d = 10.0 ** rng.uniform(-5, -3, k)
    u = rng.normal(size=(k, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    partners = base[pick] + d[:, None] * u
    f = 64
    yz = rng.uniform(0.0, 15.0, (f, 2))
    h = 0.5 * 10.0 ** rng.uniform(-5, -3, f)
    face = np.concatenate([np.stack([1.5 - h, yz[:, 0], yz[:, 1]], 1), np.stack([1.5 + h, yz[:, 0], yz[:, 1]], 1)])
    pos = np.concatenate([base, partners, face])
    return pos, box


@pytest.mark.parametrize("nb", [1, 8, 40])
def test_mixed_close_pairs(ref, nb):
    """Mixed precision keeps the 1e-5 bound when dipoles nearly touch (inside
    a cell and across a face): the near field forms close separations
    exactly.  The batched matrix-core form (40 configurations) too.  FP64
    still matches the oracle."""
    pos, box = close_pair_geometry()
    n = pos.shape[0]
    m = np.stack([inputs.random_moments(n, 60 + b) for b in range(nb)])
    out = {}
    for prec in (ccfmm.PREC_FP64, ccfmm.PREC_MIXED):
        pl = plan_for(pos, 6, 0.5, 0.0, box, precision=prec, max_batch=nb)
        out[prec] = pl.eval(m)
        pl.destroy()
    err = rel_rms(out[ccfmm.PREC_MIXED], out[ccfmm.PREC_FP64])
    print("close pairs nb=%d: mixed vs fp64 %.3e" % (nb, err), flush=True)
    assert err <= MIXED_BAR
    H_ref = ref.fmm(pos, m[0], 6, 0.5, box=box)
    assert rel_rms(out[ccfmm.PREC_FP64][0], H_ref) <= FP64_BAR
    check_per_dipole(out[ccfmm.PREC_MIXED][0], H_ref, "close pairs nb=%d mixed" % nb)


@pytest.mark.parametrize("geom", ["sphere", "clusters"])
def test_leaf_rule_occupied_mean(ref, geom):
    """Leaf rule 1 (mean dipoles over the occupied smallest cells) on the GPU:
    the same depth, cells and pair counts as the oracle, and the same field."""
    if geom == "sphere":
        pos, box = inputs.sphere_cut(6000, 30)
    else:
        pos, box = inputs.clusters(6, 1000, 77, sigma=4.0, box_side=128.0, margin=12.0)
    m = inputs.random_moments(pos.shape[0], 91)
    H_ref, st = ref.fmm(pos, m, 5, 0.5, leaf_target=0.0, leaf_rule=1, box=box, return_stats=True)
    st0 = ref.tree_shape(pos, 5, leaf_target=0.0, leaf_rule=0, box=box)
    pl = plan_for(pos, 5, 0.5, 0.0, box, leaf_rule=1)
    inf = pl.info()
    print("%s: rule-1 depth %d (rule 0: %d), %d cells" % (geom, inf["levels"], st0["levels"], inf["n_leaves"]),
          flush=True)
    assert inf["levels"] == st["levels"] and inf["levels"] > st0["levels"]
    assert inf["split_axis"] == st["split_axis"]
    assert inf["n_leaves"] == st["n_leaves"]
    assert inf["m2l_pairs_per_level"] == st["m2l_pairs_per_level"]
    assert inf["n_p2p_leaf_pairs"] == st["n_p2p_leaf_pairs"]
    assert rel_rms(pl.eval(m), H_ref) <= FP64_BAR
    pl.destroy()


@pytest.mark.parametrize("order,traceless,variant", [(1, 1, ccfmm.M2L_AUTO), (2, 1, ccfmm.M2L_AUTO),
                                                     (3, 1, ccfmm.M2L_AUTO), (4, 1, ccfmm.M2L_AUTO),
                                                     (6, 1, ccfmm.M2L_AUTO), (7, 1, ccfmm.M2L_AUTO),
                                                     (8, 1, ccfmm.M2L_AUTO), (6, 0, ccfmm.M2L_AUTO),
                                                     (5, 1, ccfmm.M2L_BLOCK)])
def test_shift_forms_agree(ref, order, traceless, variant):
    """M2M and L2L in their two forms: staged through LDS (single-stream
    evaluations; with the wide traceless M2L the moment fold and the
    completion of the local rows are fused in, with the full operator or the
    block kernel they are not needed), and the form with few registers beside
    the near field (overlapped evaluations).  FP64: the two agree to rounding
    and the staged form equals the oracle FMM; mixed: within the FP32 variant
    bar; one configuration, three (rows of a block that straddle cells) and,
    at order 5, seventy (a cell's rows spread over two blocks)."""
    n = 6000
    pos, box = inputs.ferrofluid(n, 43)
    # 70 configurations: a cell's rows span two blocks of either precision
    for nb in ((1, 3, 70) if order == 5 else (1, 3)):
        m = np.stack([inputs.random_moments(n, 500 + b) for b in range(nb)])
        for prec, bar in ((ccfmm.PREC_FP64, 1e-13), (ccfmm.PREC_MIXED, 2e-6)):
            H = {}
            for ov in (0, 1):
                print("case order=%d traceless=%d variant=%d nb=%d precision=%d overlap_near=%d" % (
                    order, traceless, variant, nb, prec, ov), flush=True)
                pl = plan_for(pos, order, 0.5, 0.0, box, precision=prec, max_batch=nb, overlap_near=ov,
                              m2l_traceless=traceless, m2l_variant=variant)
                H[ov] = pl.eval(m)
                pl.destroy()
            e = rel_rms(H[0], H[1])
            print("order=%d nb=%d precision=%d staged vs beside %.3e" % (order, nb, prec, e), flush=True)
            assert e <= bar
            if prec == ccfmm.PREC_FP64 and nb == 1:
                assert rel_rms(H[0][0], ref.fmm(pos, m[0], order, 0.5, box=box)) <= FP64_BAR


@pytest.mark.parametrize("nb", [1, 8, 40])
def test_overlapped_near_field_equals_single_stream(nb):
    """The near field on the side stream beside the expansion passes (joined
    before the smooth part is added) gives the field of the single-stream
    evaluation, through graph replays too, for one and for many configurations."""
    import torch

    pos, box = inputs.ferrofluid(8000, 41)
    m = np.stack([inputs.random_moments(8000, 300 + b) for b in range(nb)])
    out = {}
    for ov in (0, 1):
        pl = plan_for(pos, 5, 0.5, 0.0, box, precision=ccfmm.PREC_MIXED, max_batch=nb, overlap_near=ov)
        dev = torch.device("cuda:0")
        st = torch.cuda.current_stream().cuda_stream
        d_m = torch.from_numpy(m).to(dev)
        d_H = torch.empty_like(d_m)
        res = []
        for _ in range(3):
            pl.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), st)
            torch.cuda.synchronize()
            res.append(d_H.cpu().numpy().copy())
        # the timed evaluation runs every pass alone on one stream, with the same
        # field (the single-stream form's M2M and L2L: FP32 rounding apart from
        # the overlapped form's)
        t = pl.eval_device_timed(nb, d_m.data_ptr(), d_H.data_ptr(), st)
        torch.cuda.synchronize()
        assert t["p2p"] > 0 and t["total"] > 0
        assert rel_rms(d_H.cpu().numpy(), res[0]) <= (1e-12 if ov == 0 else 2e-6)
        # and leaves the plan's own (overlapped, graph-replayed) evaluation as it was
        pl.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), st)
        torch.cuda.synchronize()
        res.append(d_H.cpu().numpy().copy())
        assert all(np.array_equal(r, res[0]) for r in res[1:])
        out[ov] = res[0]
        pl.destroy()
    # the two forms run different M2M and L2L kernels: FP32 rounding apart
    assert rel_rms(out[1], out[0]) <= 2e-6


def test_energy_device_matches_oracle(ref):
    """The GPU energy E_b = -1/2 sum m.H (FP64, fixed summation order) equals the
    oracle's energy of the same arrays per configuration, and is the same on
    repeated calls."""
    import torch

    pos, box = inputs.ferrofluid(3001, 5)
    nb = 3
    m = np.stack([inputs.random_moments(3001, 90 + b) for b in range(nb)])
    H = np.random.default_rng(9).normal(size=m.shape)
    pl = plan_for(pos, 4, 0.5, 0.0, box, max_batch=nb)
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    d_m, d_H = torch.from_numpy(m).to(dev), torch.from_numpy(H).to(dev)
    d_E = torch.empty(nb, dtype=torch.float64, device=dev)
    pl.energy_device(nb, d_m.data_ptr(), d_H.data_ptr(), d_E.data_ptr(), st)
    E1 = d_E.cpu().numpy().copy()
    pl.energy_device(nb, d_m.data_ptr(), d_H.data_ptr(), d_E.data_ptr(), st)
    E2 = d_E.cpu().numpy()
    pl.destroy()
    assert np.array_equal(E1, E2)
    for b in range(nb):
        Eo = ref.energy(m[b], H[b])
        assert abs(E1[b] - Eo) <= 1e-13 * np.sum(np.abs(m[b] * H[b]))


def test_time_stepping_with_plan_reuse(ref):
    """Repeated evaluation as the moments evolve: one FP64 plan whose captured
    evaluation is replayed into the same buffers after each in-place precession
    step, with the energy taken on the GPU every step, follows the same loop run
    on the CPU with the oracle FMM, the oracle energy and a numpy step."""
    import torch

    from paper_0810_0233_amd import dynamics

    pos, box = inputs.lattice(12, 12, 12)
    n = pos.shape[0]
    m0 = inputs.random_moments(n, 77)
    dt, steps = 0.05, 4
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    pl = plan_for(pos, 5, 0.5, 0.0, box, max_batch=1, use_graph=1)
    d_m = torch.from_numpy(m0[None].copy()).to(dev)
    d_H = torch.empty_like(d_m)
    d_E = torch.empty(1, dtype=torch.float64, device=dev)
    gpu = []
    for k in range(steps):
        print("time step %d" % k, flush=True)
        pl.eval_device(1, d_m.data_ptr(), d_H.data_ptr(), st)
        pl.energy_device(1, d_m.data_ptr(), d_H.data_ptr(), d_E.data_ptr(), st)
        torch.cuda.synchronize()
        gpu.append((d_m[0].cpu().numpy().copy(), d_H[0].cpu().numpy().copy(), float(d_E.item())))
        dynamics.precession_step_(d_m, d_H, dt)
    pl.destroy()
    mc = m0.copy()
    for k in range(steps):
        H = ref.fmm(pos, mc, 5, 0.5, box=box)
        E = ref.energy(mc, H)
        mg, Hg, Eg = gpu[k]
        # the fields agree to the FP64 bar; the moments and the energy inherit it
        assert rel_rms(mg, mc) <= FP64_BAR
        assert rel_rms(Hg, H) <= FP64_BAR
        assert abs(Eg - E) <= FP64_BAR * np.sum(np.abs(mc * H))
        c = mc + dt * np.cross(mc, H)
        mc = c / np.linalg.norm(c, axis=1, keepdims=True)


@pytest.mark.parametrize("order,theta", [(3, 0.54), (6, 0.76)])
@pytest.mark.parametrize("dl", [-2, 2])
def test_leaf_sweep_points_match_oracle(ref, order, theta, dl):
    """The leaf-size study runs the path unchanged at trees two levels above and
    below the paper's choice (Table II's (p, alpha) pairs): there too the FP64
    GPU field equals the oracle FMM and the tree structure is the same."""
    from paper_0810_0233_amd import study

    pos, box = inputs.lattice(16, 16, 16)
    n = pos.shape[0]
    m = inputs.random_moments(n, 120 + order)
    L = study.paper_levels(n, study.paper_s(order)) + dl
    s = n / 2.0 ** L
    H_ref, st = ref.fmm(pos, m, order, theta, leaf_target=s, box=box, return_stats=True)
    pl = plan_for(pos, order, theta, s, box)
    inf = pl.info()
    assert inf["levels"] == st["levels"] == L
    assert inf["m2l_pairs_per_level"] == st["m2l_pairs_per_level"]
    assert inf["n_p2p_leaf_pairs"] == st["n_p2p_leaf_pairs"]
    assert rel_rms(pl.eval(m), H_ref) <= FP64_BAR
    pl.destroy()


@pytest.mark.parametrize("precision,nb", [(ccfmm.PREC_FP64, 1), (ccfmm.PREC_MIXED, 1), (ccfmm.PREC_MIXED, 40)])
def test_rebuild_keeps_lists_when_cells_stay_occupied(precision, nb):
    """A position update that moves dipoles without emptying or filling any
    cell (same geometry, same occupied cells at every level) keeps the cell
    lists, the M2L tiles and the captured evaluation; the replayed evaluation
    then equals that of a new plan on the new positions.  An update that
    changes the occupied cells rebuilds everything, with the same result."""
    import torch

    n = 20000
    pos0, box = inputs.ferrofluid(n, 51)
    lo, hi = np.asarray(box[0], float), np.asarray(box[1], float)
    rng = np.random.default_rng(52)
    pos1 = np.clip(pos0 + 0.05 * rng.normal(size=pos0.shape), lo + 1e-9, hi - 1e-9)
    pos2 = pos1.copy()
    W = hi - lo
    slab = pos2[:, 0] < lo[0] + 0.25 * W[0]
    pos2[slab, 0] += 0.5 * W[0]  # the slab x < 1/4 emptied: its cells are no longer occupied
    m = np.stack([inputs.random_moments(n, 53 + b) for b in range(nb)])  # 40: the matrix-core near field
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    d_m = torch.from_numpy(m).to(dev)

    def fresh(pos, with_info=False):
        d_pos = torch.from_numpy(pos).to(dev)
        prm = ccfmm.params(order=5, theta=0.5, box=box, precision=precision, max_batch=nb)
        pl = ccfmm.Plan.create_device(n, d_pos.data_ptr(), prm, st)
        d_H = torch.empty_like(d_m)
        pl.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), st)
        torch.cuda.synchronize()
        inf = pl.info()
        pl.destroy()
        return (d_H.cpu().numpy(), inf) if with_info else d_H.cpu().numpy()

    d_pos = torch.from_numpy(pos0.copy()).to(dev)
    prm = ccfmm.params(order=5, theta=0.5, box=box, precision=precision, max_batch=nb)
    pl = ccfmm.Plan.create_device(n, d_pos.data_ptr(), prm, st)
    d_H = torch.empty_like(d_m)
    pl.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), st)  # captured
    tol = 1e-13 if precision == ccfmm.PREC_FP64 else 1e-6
    for k, (pos, kept) in enumerate([(pos1, 1), (pos1, 2), (pos2, 2), (pos0, 2)]):
        print("case rebuild %d, kept so far %d" % (k, kept), flush=True)
        d_pos.copy_(torch.from_numpy(pos))
        pl.update_positions_device(d_pos.data_ptr(), st)
        pl.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), st)
        torch.cuda.synchronize()
        H_new, inf_new = fresh(pos, with_info=True)
        inf = pl.info()  # the direct-pair count of a kept update is taken here
        assert inf["n_rebuilds_kept"] == kept
        for key in ("n_leaves", "n_cells", "n_m2l_pairs", "n_p2p_leaf_pairs", "n_p2p_pairs"):
            assert inf[key] == inf_new[key], key
        assert rel_rms(d_H.cpu().numpy(), H_new) <= tol
    pl.destroy()
    # keep_lists = 0: every update rebuilds everything, with the same field
    d_pos.copy_(torch.from_numpy(pos0))
    prm0 = ccfmm.params(order=5, theta=0.5, box=box, precision=precision, max_batch=nb, keep_lists=0)
    p0 = ccfmm.Plan.create_device(n, d_pos.data_ptr(), prm0, st)
    d_pos.copy_(torch.from_numpy(pos1))
    p0.update_positions_device(d_pos.data_ptr(), st)
    assert p0.info()["n_rebuilds_kept"] == 0
    p0.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), st)
    torch.cuda.synchronize()
    assert rel_rms(d_H.cpu().numpy(), fresh(pos1)) <= tol
    p0.destroy()



def test_positions_checked_against_the_box_on_the_device():
    """With the caller's box the bounds check runs on the device and reports
    with the level sizes: a non-finite coordinate or a dipole outside the box
    is rejected at creation and at update, and a rejected update leaves the
    plan usable after a valid one (same field as a new plan)."""
    import torch

    n = 5000
    pos0, box = inputs.ferrofluid(n, 61)
    m = inputs.random_moments(n, 62)[None]
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    prm = ccfmm.params(order=4, theta=0.5, box=box, precision=ccfmm.PREC_FP64, max_batch=1)
    d_m = torch.from_numpy(m).to(dev)
    d_H = torch.empty_like(d_m)
    hi = np.asarray(box[1], float)
    bad_nan = pos0.copy()
    bad_nan[17, 2] = np.nan
    bad_out = pos0.copy()
    bad_out[4321, 0] = hi[0] + 1e-6
    for bad, msg in ((bad_nan, "non-finite"), (bad_out, "outside the box")):
        d_bad = torch.from_numpy(bad).to(dev)
        with pytest.raises(ccfmm.CCFMMError) as e:
            ccfmm.Plan.create_device(n, d_bad.data_ptr(), prm, st)
        assert e.value.status == ccfmm.EINVAL and msg in ccfmm.last_error()
    d_pos = torch.from_numpy(pos0.copy()).to(dev)
    pl = ccfmm.Plan.create_device(n, d_pos.data_ptr(), prm, st)
    pl.eval_device(1, d_m.data_ptr(), d_H.data_ptr(), st)
    for bad, msg in ((bad_out, "outside the box"), (bad_nan, "non-finite")):
        d_pos.copy_(torch.from_numpy(bad))
        with pytest.raises(ccfmm.CCFMMError) as e:
            pl.update_positions_device(d_pos.data_ptr(), st)
        assert e.value.status == ccfmm.EINVAL and msg in ccfmm.last_error()
    pos1 = pos0.copy()
    pos1[:, 1] = np.minimum(pos1[:, 1] + 0.01, hi[1])
    d_pos.copy_(torch.from_numpy(pos1))
    pl.update_positions_device(d_pos.data_ptr(), st)
    pl.eval_device(1, d_m.data_ptr(), d_H.data_ptr(), st)
    torch.cuda.synchronize()
    H = d_H.cpu().numpy().copy()
    pl.destroy()
    p2 = ccfmm.Plan.create_device(n, d_pos.data_ptr(), prm, st)
    p2.eval_device(1, d_m.data_ptr(), d_H.data_ptr(), st)
    torch.cuda.synchronize()
    assert rel_rms(H, d_H.cpu().numpy()) <= 1e-13
    p2.destroy()


@pytest.mark.parametrize("order", [3, 6, 8])
def test_total_degree_truncation_matches_oracle(ref, order):
    """truncation = 1 (M2L keeps |n| + |q| <= p): the FP64 GPU FMM equals the
    oracle FMM of the same reading to the 1e-10 bar on the 10^3 lattice and a
    ragged ferrofluid, and differs from the separate truncation; mixed
    precision stays within 1e-5 of FP64 through every M2L kernel the order
    allows."""
    c = inputs.config_lattice_1000()
    pos, box, m = c["pos"], c["box"], c["m"][0]
    print("case lattice p=%d total degree" % order, flush=True)
    H_ref = ref.fmm(pos, m, order, 0.5, leaf_target=8, box=box, truncation=1)
    H = plan_for(pos, order, 0.5, 8, box, truncation=1).eval(m)
    assert rel_rms(H, H_ref) <= FP64_BAR
    H_sep = plan_for(pos, order, 0.5, 8, box).eval(m)
    assert rel_rms(H_sep, H) > 1e3 * FP64_BAR
    pos2, box2 = inputs.ferrofluid(6000, 77)
    m2 = inputs.random_moments(6000, 78)
    print("case ferrofluid n=6000 p=%d total degree" % order, flush=True)
    H_ref2 = ref.fmm(pos2, m2, order, 0.5, box=box2, truncation=1)
    H64 = plan_for(pos2, order, 0.5, 0.0, box2, truncation=1).eval(m2)
    assert rel_rms(H64, H_ref2) <= FP64_BAR
    variants = [0, 1, 2, 3, 4] if order <= 6 else [0]
    for v in variants:
        Hm = plan_for(pos2, order, 0.5, 0.0, box2, precision=ccfmm.PREC_MIXED, truncation=1,
                      m2l_variant=v).eval(m2)
        assert rel_rms(Hm, H64) <= 1e-5, v


@pytest.mark.parametrize("precision", [ccfmm.PREC_FP64, ccfmm.PREC_MIXED])
@pytest.mark.parametrize("nb", [2, 3, 8, 12, 31])
def test_few_configuration_near_field(ref, precision, nb):
    """2..31 configurations: the near field forms each pair's geometry once for
    a group of 2, 4 or 8 configurations (the last group partly past the batch
    for 3, 12 and 31).  On clusters (uneven cells: 1 to ~150 dipoles, several
    64-dipole chunks, so every lanes-per-target split occurs) every
    configuration equals its one-at-a-time evaluation; the FP64 plan matches
    the oracle per configuration; the mixed plan meets the per-dipole bars
    against the oracle."""
    pos, box = inputs.clusters(10, 500, 811, sigma=5.0, box_side=192.0, margin=12.0)
    n = pos.shape[0]
    mb = np.stack([inputs.random_moments(n, 900 + b) for b in range(nb)])
    print("case clusters n=%d nb=%d precision=%d" % (n, nb, precision), flush=True)
    pl = plan_for(pos, 5, 0.5, 12.0, box, precision=precision, max_batch=nb)
    Hb = pl.eval(mb)
    pl.destroy()
    # one stream: the near field and the smooth field in one kernel
    one = plan_for(pos, 5, 0.5, 12.0, box, precision=precision, max_batch=nb, overlap_near=0)
    e = rel_rms(one.eval(mb), Hb)
    print("nb=%d single-stream (fused) vs overlapped %.3e" % (nb, e), flush=True)
    assert e <= (1e-13 if precision == ccfmm.PREC_FP64 else 2e-6)
    one.destroy()
    single = plan_for(pos, 5, 0.5, 12.0, box, precision=precision, max_batch=1)
    for b in sorted({0, nb // 2, nb - 1}):
        e = rel_rms(Hb[b], single.eval(mb[b:b + 1])[0])
        print("nb=%d b=%d batch vs single %.3e" % (nb, b, e), flush=True)
        assert e <= (1e-13 if precision == ccfmm.PREC_FP64 else 2e-6)
    single.destroy()
    for b in sorted({0, nb - 1}):
        H_ref = ref.fmm(pos, mb[b], 5, 0.5, box=box, leaf_target=12.0)
        if precision == ccfmm.PREC_FP64:
            assert rel_rms(Hb[b], H_ref) <= FP64_BAR
        else:
            assert rel_rms(Hb[b], H_ref) <= MIXED_BAR
            check_per_dipole(Hb[b], H_ref, "nb=%d b=%d mixed" % (nb, b))


def test_device_memory_cap_gives_enomem(ref):
    """A plan-level device-memory cap: creation that cannot fit fails with
    CCFMM_ENOMEM (nothing left behind); a plan created within its cap reports
    what it holds; an evaluation whose larger batch would pass the cap fails
    with CCFMM_ENOMEM, and the plan then still evaluates the batch sizes that
    fit (same field as before) and is destroyed normally."""
    pos, box = inputs.ferrofluid(20000, 2001)
    m = np.stack([inputs.random_moments(20000, 2101 + b) for b in range(8)])
    with pytest.raises(ccfmm.CCFMMError) as e:
        plan_for(pos, 6, 0.5, 0.0, box, precision=ccfmm.PREC_MIXED, max_batch=8, device_mem_cap=1 << 20)
    assert e.value.status == ccfmm.ENOMEM and "cap" in str(e.value)
    free = plan_for(pos, 6, 0.5, 0.0, box, precision=ccfmm.PREC_MIXED, max_batch=8)
    H1 = free.eval(m[:1])
    need1 = free.info()["device_bytes"]
    H8 = free.eval(m)
    need8 = free.info()["device_bytes"]
    free.destroy()
    print("device bytes: one configuration %d, eight %d" % (need1, need8), flush=True)
    assert 0 < need1 < need8
    capped = plan_for(pos, 6, 0.5, 0.0, box, precision=ccfmm.PREC_MIXED, max_batch=8,
                      device_mem_cap=(need1 + need8) // 2)
    assert np.array_equal(capped.eval(m[:1]), H1)
    assert capped.info()["device_bytes"] <= (need1 + need8) // 2
    with pytest.raises(ccfmm.CCFMMError) as e:
        capped.eval(m)
    assert e.value.status == ccfmm.ENOMEM
    assert np.array_equal(capped.eval(m[:1]), H1)  # the sizes that fit still evaluate
    assert rel_rms(H8[0], H1[0]) <= 1e-6
    capped.destroy()
