"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
independently of the oracle's own code (closed forms, symbolic derivatives,
finite differences, identities, brute force on small inputs, the paper's
worked examples).  CPU only."""
import math

import numpy as np
import pytest
import sympy as sp

from paper_0810_0233_amd import inputs


def dense_multi_indices(p):
    return [(a, b, c) for a in range(p + 1) for b in range(p + 1 - a) for c in range(p + 1 - a - b)]


def potential_fd_field(pos, m, x, h=1e-4):
    """-grad of the dipole potential phi(x) = sum_j m_j.(x-x_j)/|x-x_j|^3 by
    4th-order central differences (an independent route to the field)."""
    def phi(y):
        r = y[None, :] - pos
        d = np.sqrt(np.sum(r * r, axis=1))
        ok = d > 0
        return np.sum(np.sum(m[ok] * r[ok], axis=1) / d[ok] ** 3)

    g = np.zeros(3)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        g[a] = (-phi(x + 2 * e) + 8 * phi(x + e) - 8 * phi(x - e) + phi(x - 2 * e)) / (12 * h)
    return -g


# ---------------------------------------------------------------- brute force
def test_single_dipole_closed_form(ref):
    """Field of one dipole: on its axis 2m/r^3, perpendicular -m/r^3
    (the pair field of Eq.(H2) with the sign of H = -grad V)."""
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 2.0], [3.0, 0.0, 0.0]])
    m = np.array([[0.0, 0.0, 1.5], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    H = ref.bruteforce(pos, m)
    np.testing.assert_allclose(H[1], [0, 0, 2 * 1.5 / 8.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(H[2], [0, 0, -1.5 / 27.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(H[0], [0, 0, 0], atol=0)  # the other two carry no moment


def test_bruteforce_is_minus_grad_potential(ref):
    rng = np.random.default_rng(7)
    pos = rng.random((40, 3)) * 5
    m = inputs.unit_moments(40, rng)
    H = ref.bruteforce(pos, m)
    for i in [0, 7, 23]:
        others = np.ones(40, dtype=bool)
        others[i] = False
        fd = potential_fd_field(pos[others], m[others], pos[i])
        np.testing.assert_allclose(H[i], fd, rtol=1e-7, atol=1e-9)


def test_energy_closed_form_pairs(ref):
    """Energy of two dipoles (Sec. 3 with the Appendix's factor 1/2): the
    interaction energy of a pair is counted once.  Coaxial parallel unit
    dipoles at distance r: E = -2/r^3; coaxial antiparallel: +2/r^3; parallel
    side by side (moments perpendicular to the separation): +1/r^3.  Dropping
    the 1/2 doubles these and flipping the sign negates them."""
    r = 1.7
    z = np.array([0.0, 0.0, 1.0])
    cases = [
        (np.array([[0.0, 0, 0], [0, 0, r]]), np.array([z, z]), -2.0 / r**3),
        (np.array([[0.0, 0, 0], [0, 0, r]]), np.array([z, -z]), 2.0 / r**3),
        (np.array([[0.0, 0, 0], [r, 0, 0]]), np.array([z, z]), 1.0 / r**3),
        (np.array([[0.0, 0, 0], [0, r, 0]]), np.array([z, z]), 1.0 / r**3),
    ]
    for pos, m, e in cases:
        assert abs(ref.energy(m, ref.bruteforce(pos, m)) - e) <= 1e-14 * abs(e)
    # the same from fields written by hand: on the axis each dipole sees
    # 2m/r^3, beside each other -m/r^3
    H_axis = np.array([2 * z / r**3, 2 * z / r**3])
    assert abs(ref.energy(np.array([z, z]), H_axis) + 2.0 / r**3) <= 1e-15
    H_side = np.array([-z / r**3, -z / r**3])
    assert abs(ref.energy(np.array([z, z]), H_side) - 1.0 / r**3) <= 1e-15


def test_energy_is_sum_of_pair_interactions(ref):
    """Three (and more) dipoles: the energy equals the sum over unordered pairs
    of the pair interaction energy (m_i.m_j - 3 (m_i.u)(m_j.u)) / r^3, a sum
    that never forms a field."""
    rng = np.random.default_rng(11)
    for n in (3, 7):
        pos = rng.random((n, 3)) * 4
        m = rng.standard_normal((n, 3))
        e_pairs = 0.0
        for i in range(n):
            for j in range(i + 1, n):
                d = pos[i] - pos[j]
                rr = float(np.sqrt(d @ d))
                u = d / rr
                e_pairs += (m[i] @ m[j] - 3.0 * (m[i] @ u) * (m[j] @ u)) / rr**3
        e = ref.energy(m, ref.bruteforce(pos, m))
        assert abs(e - e_pairs) <= 1e-12 * max(1.0, abs(e_pairs))


def test_bruteforce_coincident_points_do_not_interact(ref):
    pos = np.array([[0.0, 0, 0], [0.0, 0, 0], [1.0, 0, 0]])
    m = np.array([[0, 0, 1.0], [0, 1.0, 0], [1.0, 0, 0]])
    H = ref.bruteforce(pos, m)
    # dipoles 0 and 1 only see dipole 2 at distance 1 along x: 2 m_x along x
    np.testing.assert_allclose(H[0], [2.0, 0, 0], atol=1e-15)
    np.testing.assert_allclose(H[1], [2.0, 0, 0], atol=1e-15)
    np.testing.assert_allclose(H[2], [0, -1.0, -1.0], atol=1e-15)  # -(m0+m1)/1, both perpendicular
    Ht = ref.bruteforce_targets(pos, m, np.array([2, 0]))
    np.testing.assert_array_equal(Ht, H[[2, 0]])


# ------------------------------------------------------------ D tensor, F table
def _sym_D(K):
    x, y, z = sp.symbols("x y z", real=True)
    f = 1 / sp.sqrt(x ** 2 + y ** 2 + z ** 2)
    out = {}
    for k in dense_multi_indices(K):
        d = f
        for var, cnt in zip((x, y, z), k):
            if cnt:
                d = sp.diff(d, var, cnt)
        out[k] = (-1) ** sum(k) * d  # D_k = d^k / d(-r)^k (1/r), Eq.(Vm)
    return (x, y, z), out


def test_dtensor_low_orders_closed_form(ref):
    c = np.array([0.7, -1.3, 2.1])
    r = np.linalg.norm(c)
    D = ref.dtensor(2, c)
    assert D[0, 0, 0] == pytest.approx(1 / r, rel=1e-15)
    assert D[1, 0, 0] == pytest.approx(c[0] / r ** 3, rel=1e-14)
    assert D[0, 0, 1] == pytest.approx(c[2] / r ** 3, rel=1e-14)
    assert D[2, 0, 0] == pytest.approx((2 * c[0] ** 2 - c[1] ** 2 - c[2] ** 2) / r ** 5, rel=1e-13)
    assert D[1, 1, 0] == pytest.approx(3 * c[0] * c[1] / r ** 5, rel=1e-13)


def test_dtensor_matches_symbolic_derivatives(ref):
    K = 8
    (x, y, z), sym = _sym_D(K)
    c = (sp.Rational(7, 10), sp.Rational(-13, 10), sp.Rational(21, 10))
    D = ref.dtensor(K, np.array([float(v) for v in c]))
    for k, expr in sym.items():
        exact = float(expr.subs({x: c[0], y: c[1], z: c[2]}))
        assert D[k] == pytest.approx(exact, rel=1e-12, abs=1e-15), k


def test_dtensor_identities(ref):
    K = 12
    rng = np.random.default_rng(3)
    c = rng.normal(size=3) * 2
    D = ref.dtensor(K, c)
    # harmonic: sum_a D_{k + 2 e_a} = 0
    for k in dense_multi_indices(K - 2):
        tr = D[k[0] + 2, k[1], k[2]] + D[k[0], k[1] + 2, k[2]] + D[k[0], k[1], k[2] + 2]
        scale = max(abs(D[k[0] + 2, k[1], k[2]]), abs(D[k[0], k[1] + 2, k[2]]), abs(D[k[0], k[1], k[2] + 2]))
        assert abs(tr) <= 1e-12 * scale + 1e-300
    # homogeneity of degree -(|k|+1) and parity
    D2 = ref.dtensor(K, 2.5 * c)
    Dm = ref.dtensor(K, -c)
    # (F-table sums cancel at high order: compare against the size of the order)
    scale = {n: max(abs(D[k]) for k in dense_multi_indices(K) if sum(k) == n) for n in range(K + 1)}
    for k in dense_multi_indices(K):
        n = sum(k)
        assert abs(D2[k] - D[k] * 2.5 ** (-(n + 1))) <= 1e-12 * scale[n] * 2.5 ** (-(n + 1))
        assert abs(Dm[k] - D[k] * (-1) ** n) <= 1e-13 * scale[n]


def test_ftable_structure(ref):
    """F_k(q) is an integer, zero unless |q| = |k| and q = k (mod 2) componentwise."""
    assert ref.ftable((0, 0, 0), (0, 0, 0)) == 1.0
    assert ref.ftable((1, 0, 0), (1, 0, 0)) == 1.0
    assert ref.ftable((2, 0, 0), (2, 0, 0)) == 2.0
    assert ref.ftable((2, 0, 0), (0, 2, 0)) == -1.0
    for k in dense_multi_indices(8):
        n = sum(k)
        for q in dense_multi_indices(n):
            f = ref.ftable(k, q)
            if f != 0.0:
                assert sum(q) == n
                assert all((kk - qq) % 2 == 0 for kk, qq in zip(k, q))
                assert f == round(f)


# --------------------------------------------------------- multipole moments
def test_p2m_single_dipole_at_center(ref):
    """A dipole at the expansion centre has Q_{e_a} = m_a and nothing else (Sec. 3)."""
    m = np.array([[0.3, -0.4, 0.5]])
    Q = ref.p2m(6, [1.0, 2.0, 3.0], np.array([[1.0, 2.0, 3.0]]), m)
    expect = np.zeros_like(Q)
    expect[1, 0, 0], expect[0, 1, 0], expect[0, 0, 1] = m[0]
    np.testing.assert_array_equal(Q, expect)


def test_p2m_is_limit_of_charge_pairs(ref):
    """Eq.(multipolemoments) is the d -> 0 limit of +-q at y +- d with 2qd = m.
    The charge-pair moments differ from the limit by O(d^2); Richardson
    extrapolation removes that term."""
    p = 6
    rng = np.random.default_rng(11)
    y = rng.normal(size=(5, 3)) * 0.6
    m = inputs.unit_moments(5, rng)
    center = np.zeros(3)
    Qd = ref.p2m(p, center, y, m)

    def pair_moments(d):
        u = m / np.linalg.norm(m, axis=1, keepdims=True)
        q = np.linalg.norm(m, axis=1) / (2 * d)
        pos = np.concatenate([y + d * u, y - d * u])
        qq = np.concatenate([q, -q])
        return ref.charge_moments(p, center, pos, qq)

    d = 1e-2
    rich = (4 * pair_moments(d / 2) - pair_moments(d)) / 3
    scale = np.max(np.abs(Qd))
    assert np.max(np.abs(rich - Qd)) < 1e-8 * scale
    assert np.max(np.abs(pair_moments(d) - Qd)) > 1e-7 * scale  # the O(d^2) term is really there


def test_m2m_equals_direct_moments(ref):
    """Eq.(momentshift): moments taken about the parent centre equal the shifted
    child moments (exact polynomial identity)."""
    p = 6
    rng = np.random.default_rng(5)
    child = np.array([0.4, -0.2, 0.9])
    parent = np.array([0.0, 0.3, 0.1])
    pos = child + rng.uniform(-0.5, 0.5, size=(12, 3))
    m = inputs.unit_moments(12, rng)
    Qc = ref.p2m(p, child, pos, m)
    Qp_direct = ref.p2m(p, parent, pos, m)
    Qp = ref.m2m(p, child - parent, Qc)
    np.testing.assert_allclose(Qp, Qp_direct, rtol=1e-13, atol=1e-14 * np.max(np.abs(Qp_direct)))


def test_l2l_is_exact_reexpansion(ref):
    """Eq.(taylorshift): the child expansion is the parent polynomial re-centred."""
    p = 6
    rng = np.random.default_rng(9)
    V = np.zeros((p + 1,) * 3)
    for k in dense_multi_indices(p):
        V[k] = rng.normal()
    c = np.array([0.25, -0.5, 0.125])
    Vc = ref.l2l(p, c, V)
    for _ in range(5):
        y = rng.uniform(-0.3, 0.3, size=3)
        a = ref.local_potential(p, V, c + y)
        b = ref.local_potential(p, Vc, y)
        assert a == pytest.approx(b, rel=1e-13, abs=1e-13)


def test_multipole_potential_converges(ref):
    """Eq.(Vm): sum_{|n|<=p} D_n(x) Q_n tends to the exact dipole potential."""
    rng = np.random.default_rng(2)
    src = rng.uniform(-0.5, 0.5, size=(8, 3))
    m = inputs.unit_moments(8, rng)
    x = np.array([2.0, 1.5, -1.0])
    r = x[None] - src
    exact = np.sum(np.sum(m * r, axis=1) / np.linalg.norm(r, axis=1) ** 3)
    errs = []
    for p in range(1, 9):
        Q = ref.p2m(p, np.zeros(3), src, m)
        errs.append(abs(ref.multipole_potential(p, Q, x) - exact))
    assert errs[-1] < 1e-4 * abs(exact)
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))
    # geometric decay: rho = max|src| / |x|
    rho = np.max(np.linalg.norm(src, axis=1)) / np.linalg.norm(x)
    for p in (2, 4, 8):
        assert errs[p - 1] < 50 * rho ** (p + 1) * np.sum(np.abs(m)) / np.linalg.norm(x) ** 2


def test_m2l_coefficients_are_taylor_derivatives(ref):
    """Eq.(taylorcalc): V_n is the n-th derivative, at the target centre, of the
    truncated multipole potential of the source (symbolic check, p = 3)."""
    p = 3
    X, Y, Z = sp.symbols("X Y Z", real=True)
    rng = np.random.default_rng(4)
    Q = np.zeros((p + 1,) * 3)
    for k in dense_multi_indices(p):
        if sum(k) >= 1:
            Q[k] = float(sp.Rational(int(rng.integers(-9, 10)), 8))
    cvec = (sp.Rational(5, 2), sp.Rational(-3, 2), sp.Rational(1, 1))
    r = sp.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    phi = 0
    for k in dense_multi_indices(p):
        if Q[k] == 0.0:
            continue
        d = 1 / r
        for var, cnt in zip((X, Y, Z), k):
            if cnt:
                d = sp.diff(d, var, cnt)
        phi += sp.nsimplify(Q[k]) * (-1) ** sum(k) * d
    V = ref.m2l(p, np.array([float(v) for v in cvec]), Q)
    for n in dense_multi_indices(p):
        e = phi
        for var, cnt in zip((X, Y, Z), n):
            if cnt:
                e = sp.diff(e, var, cnt)
        exact = float(e.subs({X: cvec[0], Y: cvec[1], Z: cvec[2]}))
        assert V[n] == pytest.approx(exact, rel=1e-12, abs=1e-14), n


def test_l2p_is_minus_gradient_of_local_expansion(ref):
    p = 5
    rng = np.random.default_rng(8)
    V = np.zeros((p + 1,) * 3)
    for k in dense_multi_indices(p):
        V[k] = rng.normal()
    y = np.array([0.11, -0.07, 0.05])
    H = ref.l2p(p, V, y)
    h = 1e-5
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        g = (ref.local_potential(p, V, y + e) - ref.local_potential(p, V, y - e)) / (2 * h)
        assert H[a] == pytest.approx(-g, rel=1e-8, abs=1e-9)


# ------------------------------------------------------------------ whole FMM
def test_fmm_reduces_to_bruteforce(ref):
    """theta -> 0: every pair is near, the FMM is the direct sum; a single leaf
    (s >= N) gives the same."""
    c = inputs.config_lattice_1000()
    pos, m = c["pos"], c["m"][0]
    Hb = ref.bruteforce(pos, m)
    H = ref.fmm(pos, m, 4, 1e-3, leaf_target=8, box=c["box"])
    assert ref.rel_rms(H, Hb) < 1e-13
    H1, st = ref.fmm(pos, m, 4, 0.5, leaf_target=5000, box=c["box"], return_stats=True)
    assert st["levels"] == 0
    assert ref.rel_rms(H1, Hb) < 1e-13


def test_fmm_far_field_sign_and_scale(ref):
    """Two clusters far apart: the FMM far field equals brute force to the
    truncation error (a wrong sign or factor in any operator fails this)."""
    rng = np.random.default_rng(12)
    a = rng.uniform(0, 1, size=(200, 3))
    b = rng.uniform(0, 1, size=(200, 3)) + np.array([6.0, 0, 0])
    pos = np.concatenate([a, b])
    m = inputs.unit_moments(400, rng)
    Hb = ref.bruteforce(pos, m)
    H, st = ref.fmm(pos, m, 8, 0.5, leaf_target=8, return_stats=True)
    assert st["n_m2l_pairs"] > 0
    assert ref.rel_rms(H, Hb) < 1e-6


@pytest.mark.parametrize("geom", ["lattice", "ferro"])
def test_fmm_error_decreases_with_order_and_angle(ref, geom):
    if geom == "lattice":
        pos, box = inputs.lattice(16, 16, 16)
    else:
        pos, box = inputs.ferrofluid(4096, 77)
    m = inputs.random_moments(pos.shape[0], 1234)
    Hb = ref.bruteforce(pos, m)
    errs_p = [ref.rel_rms(ref.fmm(pos, m, p, 0.5, leaf_target=8, box=box), Hb) for p in range(1, 8)]
    assert all(errs_p[i + 1] < errs_p[i] for i in range(len(errs_p) - 1)), errs_p
    errs_t = [ref.rel_rms(ref.fmm(pos, m, 4, t, leaf_target=8, box=box), Hb) for t in (0.8, 0.6, 0.4, 0.25)]
    assert all(errs_t[i + 1] < errs_t[i] for i in range(len(errs_t) - 1)), errs_t
    # the error tracks the paper's estimate e = [a/(2-a)]^p (Sec. 3) within a modest factor
    for p, e in zip(range(1, 8), errs_p):
        est = (0.5 / 1.5) ** p
        assert e < 3 * est


def _golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        return json.load(f)


def test_tree_rule_worked_examples(ref):
    """The three smallest-cell choices worked out in Sec. 4."""
    g = _golden("tree_rule_examples.json")
    for ex in g["examples"]:
        pos, box = inputs.lattice(*ex["lattice"])
        st = ref.tree_shape(pos, ex["order"], box=box)
        assert st["levels"] == ex["levels"]
        assert sorted(st["leaf_side"]) == sorted(ex["leaf_side"])
        # printed to 3 significant digits
        assert pos.shape[0] / 2 ** ex["levels"] == pytest.approx(ex["per_leaf_printed"], abs=0.03)
    assert ref.tree_shape(np.zeros((1, 3)) + 1, 4)["s_used"] == pytest.approx(0.74 * 16)
    assert ref.tree_shape(np.zeros((1, 3)) + 1, 3)["s_used"] == 8.0


def test_tree_lattice_1000_shape(ref):
    c = inputs.config_lattice_1000()
    H, st = ref.fmm(c["pos"], c["m"][0], 4, 0.5, leaf_target=8, box=c["box"], return_stats=True)
    assert st["levels"] == 7
    assert st["split_axis"] == [0, 1, 2, 0, 1, 2, 0]
    assert st["leaf_side"] == [1.25, 2.5, 2.5]
    assert st["n_leaves"] == 128  # sites on the cell faces still fill every smallest cell


def test_opening_angle_tie_is_far(ref):
    """alpha == alpha_m (theta = 0.5, offset (2,2,2) on cubic cells) is far:
    the lists at theta = 0.5 equal those just above 0.5, not just below."""
    pos, box = inputs.lattice(16, 16, 16)
    kw = dict(leaf_target=8, box=box, return_stats=True)
    m = np.zeros_like(pos)
    _, s0 = ref.fmm(pos, m, 1, 0.5, **kw)
    _, sp_ = ref.fmm(pos, m, 1, 0.5 + 1e-9, **kw)
    _, sm = ref.fmm(pos, m, 1, 0.5 - 1e-9, **kw)
    assert s0["n_m2l_pairs"] == sp_["n_m2l_pairs"]
    assert s0["n_p2p_leaf_pairs"] == sp_["n_p2p_leaf_pairs"]
    assert s0["n_p2p_leaf_pairs"] != sm["n_p2p_leaf_pairs"]


def test_table2_parameter_sets_have_equal_error_estimate():
    """Table II lists (p, alpha) pairs for e = [alpha/(2-alpha)]^p = 0.05 (Sec. 4)."""
    g = _golden("table2_error_estimate.json")
    for p, a in g["pairs"]:
        assert abs((a / (2 - a)) ** p - g["target_e"]) < 0.005


@pytest.mark.slow
def test_energy_accuracy_32cube(ref):
    """Sec. 4: at e = 0.05, (p, alpha) = (5, 0.71), the magnetostatic energy error
    is below 1%; at (6, 0.48) the error is far smaller."""
    pos, box = inputs.lattice(32, 32, 32)
    m = inputs.random_moments(pos.shape[0], 42)
    Hb = ref.bruteforce(pos, m)
    Eb = ref.energy(m, Hb)
    E5 = ref.energy(m, ref.fmm(pos, m, 5, 0.71, box=box))
    E6 = ref.energy(m, ref.fmm(pos, m, 6, 0.48, box=box))
    assert abs(E5 - Eb) < 0.01 * abs(Eb)
    assert abs(E6 - Eb) < 0.001 * abs(Eb)


def test_leaf_rule_mean_over_nonempty(ref):
    """Leaf rule 1 counts only occupied smallest cells: for a sphere cut it picks a
    deeper tree than the N/2^L rule."""
    pos, box = inputs.sphere_cut(4000, 24)
    s0 = ref.tree_shape(pos, 4, leaf_target=8, box=box, leaf_rule=0)
    s1 = ref.tree_shape(pos, 4, leaf_target=8, box=box, leaf_rule=1)
    assert s0["levels"] == int(np.argmin([abs(4000 / 2 ** L - 8) for L in range(25)]))
    assert s1["levels"] >= s0["levels"]
    # occupied smallest cells counted directly (numpy unique over the cell
    # indices of the halving sequence), then the argmin of the rule
    lo, hi = np.asarray(box[0], float), np.asarray(box[1], float)
    W = hi - lo

    def occupied(L):
        h, k = W.copy(), np.zeros(3, dtype=np.int64)
        for _ in range(L):
            a = 0
            if h[1] > h[a]:
                a = 1
            if h[2] > h[a]:
                a = 2
            h[a] /= 2.0
            k[a] += 1
        c = np.floor((pos - lo) * (2.0 ** k) / W).astype(np.int64)
        c = np.minimum(np.maximum(c, 0), (1 << k) - 1)
        return len(np.unique(c, axis=0))

    d = [abs(4000 / occupied(L) - 8) for L in range(25)]
    assert s1["levels"] == int(np.argmin(d))


def test_invalid_inputs(ref):
    pos = np.zeros((3, 3))
    m = np.zeros((3, 3))
    for bad in [dict(order=0, theta=0.5), dict(order=9, theta=0.5), dict(order=3, theta=1.0),
                dict(order=3, theta=0.0)]:
        with pytest.raises(ValueError):
            ref.fmm(pos, m, **bad)
    with pytest.raises(ValueError):
        ref.fmm(np.array([[np.nan, 0, 0]]), np.zeros((1, 3)), 3, 0.5)
    with pytest.raises(ValueError):
        ref.fmm(np.array([[2.0, 0, 0]]), np.zeros((1, 3)), 3, 0.5, box=([0, 0, 0], [1, 1, 1]))


def _bar_case(seed=21, n=64):
    """Dipoles in the box [0,4]x[0,1]x[0,1] with s = 16: two levels, both
    splits along x, so the smallest cells are the unit cubes [k, k+1) x ..."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 1, size=(n, 3)) * np.array([4.0, 1.0, 1.0])
    m = inputs.unit_moments(n, rng)
    return pos, m, ([0.0, 0.0, 0.0], [4.0, 1.0, 1.0]), np.floor(pos[:, 0]).astype(int)


def test_fmm_leaf_uniform_equals_fixed(ref):
    pos, m, box, cell = _bar_case()
    H, st = ref.fmm(pos, m, 5, 0.6, leaf_target=16, box=box, return_stats=True)
    assert st["levels"] == 2 and st["split_axis"] == [0, 0]
    n = pos.shape[0]
    H2 = ref.fmm_leaf(pos, m, 5, 0.6, leaf_p=np.full(n, 5), leaf_theta=np.full(n, 0.6), leaf_target=16, box=box)
    assert np.array_equal(H, H2)


def test_fmm_leaf_angle_and_order_act_on_own_cell(ref):
    """A smallest cell's angle decides which of the candidate cells are far for
    its own dipoles only: cell 0 sees cell 3 at offset 3 (far iff
    9 theta^2 >= 3, unit cubes), cell 2 at offset 2 (never far for theta < 1).
    With theta = 0.3 everything is near -> cell 0 gets the direct sum; with 0.7
    cell 3 is far -> truncation error that falls with the cell's own order."""
    pos, m, box, cell = _bar_case()
    n = pos.shape[0]
    Hb = ref.bruteforce(pos, m)
    in0 = cell == 0
    base_p, base_t = np.full(n, 4), np.full(n, 0.7)

    t = base_t.copy()
    t[in0] = 0.3
    H = ref.fmm_leaf(pos, m, 4, 0.7, leaf_p=base_p, leaf_theta=t, leaf_target=16, box=box)
    assert ref.rel_rms(H[in0], Hb[in0]) < 1e-13
    H_fixed = ref.fmm(pos, m, 4, 0.7, leaf_target=16, box=box)
    assert np.array_equal(H[~in0], H_fixed[~in0])  # the other cells are untouched
    assert ref.rel_rms(H_fixed[in0], Hb[in0]) > 1e-8  # at 0.7 cell 3 is far for cell 0

    errs = []
    for p in (1, 2, 4):
        pp = base_p.copy()
        pp[in0] = p
        Hp = ref.fmm_leaf(pos, m, 4, 0.7, leaf_p=pp, leaf_theta=base_t, leaf_target=16, box=box)
        assert np.array_equal(Hp[~in0], H_fixed[~in0])
        errs.append(ref.rel_rms(Hp[in0], Hb[in0]))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] == ref.rel_rms(H_fixed[in0], Hb[in0])


def test_fmm_leaf_rejects_bad_parameters(ref):
    pos, m, box, _ = _bar_case()
    n = pos.shape[0]
    for lp, lt in [(np.full(n, 5), None), (np.full(n, 0), None), (None, np.full(n, 1.0)), (None, np.zeros(n))]:
        with pytest.raises(ValueError):
            ref.fmm_leaf(pos, m, 4, 0.5, leaf_p=lp, leaf_theta=lt, leaf_target=16, box=box)


MLP_DIMS = (8, 64, 64, 25)


def _mlp_unpack(P):
    i, h1, h2, o = MLP_DIMS
    k = 0
    out = []
    for shape in [(h1, i), (h1,), (h2, h1), (h2,), (o, h2), (o,)]:
        size = int(np.prod(shape))
        out.append(P[k:k + size].reshape(shape))
        k += size
    return out


def test_mlp_reference_special_cases(ref):
    """The selector network (not in the paper): with positive weights and
    inputs no ReLU clips, so the network is the plain product chain; with
    negative pre-activations in both hidden layers only the last bias
    survives; the masked loss is the squared error over the masked entries."""
    rng = np.random.default_rng(5)
    n = ref.mlp_param_count(*MLP_DIMS)
    P = rng.uniform(0.0, 0.1, n)
    W1, b1, W2, b2, W3, b3 = _mlp_unpack(P)
    x = rng.uniform(0.0, 1.0, (7, MLP_DIMS[0]))
    y = ref.mlp_forward(P, x, *MLP_DIMS)
    y_lin = ((x @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    assert np.allclose(y, y_lin, rtol=1e-13, atol=0)
    Pn = P.copy()
    W1n, b1n, _, b2n = _mlp_unpack(Pn)[:4]
    W1n[...] = -np.abs(W1n)
    b1n[...] = -1.0  # every first hidden unit clipped ...
    b2n[...] = -1.0  # ... so the second layer sees only its (negative) bias
    yn = ref.mlp_forward(Pn, x, *MLP_DIMS)
    assert np.array_equal(yn, np.broadcast_to(_mlp_unpack(Pn)[5], yn.shape))
    # loss: zero at the targets, zero with an empty mask, one entry -> (y - t)^2 / 2
    t = y.copy()
    mask = np.ones_like(y)
    loss, g = ref.mlp_loss_grad(P, x, t, mask, *MLP_DIMS)
    assert loss == 0.0 and not np.any(g)
    t2 = y + 1.0
    loss0, g0 = ref.mlp_loss_grad(P, x, t2, np.zeros_like(y), *MLP_DIMS)
    assert loss0 == 0.0 and not np.any(g0)
    m1 = np.zeros_like(y)
    m1[3, 7] = 1.0
    t3 = y.copy()
    t3[3, 7] -= 0.25
    loss1, _ = ref.mlp_loss_grad(P, x, t3, m1, *MLP_DIMS)
    assert abs(loss1 - 0.25 ** 2 / 2) < 1e-15


def test_mlp_reference_gradient_finite_differences(ref):
    rng = np.random.default_rng(9)
    n = ref.mlp_param_count(*MLP_DIMS)
    P = rng.normal(0.0, 0.3, n)
    x = rng.normal(size=(11, MLP_DIMS[0]))
    t = rng.normal(size=(11, MLP_DIMS[3]))
    mask = (rng.random((11, MLP_DIMS[3])) < 0.6).astype(float)
    _, g = ref.mlp_loss_grad(P, x, t, mask, *MLP_DIMS)
    h = 1e-6
    idx = rng.choice(n, 60, replace=False)
    for k in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        lp, _ = ref.mlp_loss_grad(Pp, x, t, mask, *MLP_DIMS)
        lm, _ = ref.mlp_loss_grad(Pm, x, t, mask, *MLP_DIMS)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


# ------------------------------------------------------- total-degree truncation
def test_total_degree_m2l_is_the_legendre_series(ref):
    """M2L keeping only |n| + |q| <= p, then the local expansion, gives the
    potential of a unit charge at x (source cell) at y (target cell) as the
    Taylor polynomial of 1/|c + w| in w = y - x of degree p, i.e. the Legendre
    series sum_{j<=p} |w|^j P_j(-c.w/(|c||w|)) / |c|^(j+1) (generating
    function of the Legendre polynomials).  The separate truncation (each
    index to p) is not this polynomial."""
    from numpy.polynomial import legendre

    rng = np.random.default_rng(31)
    for p in (2, 4, 6, 8):
        for _ in range(3):
            src, tgt = np.zeros(3), np.array([3.0, -2.0, 1.5])
            x = rng.uniform(-0.5, 0.5, 3)
            y = rng.uniform(-0.5, 0.5, 3)
            c = tgt - src
            Q = ref.charge_moments(p, src, x[None], np.array([1.0]))
            V = ref.m2l(p, c, Q, total=True)
            got = ref.local_potential(p, V, y)
            w = y - x
            cw = -np.dot(c, w) / (np.linalg.norm(c) * np.linalg.norm(w))
            want = sum(np.linalg.norm(w) ** j / np.linalg.norm(c) ** (j + 1) * legendre.legval(cw, [0] * j + [1])
                       for j in range(p + 1))
            assert got == pytest.approx(want, rel=1e-13), p
            # the separate form keeps some terms of degree p+1..2p: it differs
            # from the polynomial by a fair share of the truncation error
            exact = 1.0 / np.linalg.norm(c + w)
            sep = ref.local_potential(p, ref.m2l(p, c, Q), y)
            assert abs(sep - want) > 1e-2 * abs(exact - want)
            assert abs(got - exact) < 2 * (np.linalg.norm(w) / np.linalg.norm(c)) ** (p + 1) / np.linalg.norm(c)


def test_total_degree_fmm_converges_to_bruteforce(ref):
    """Whole FMM with total-degree truncation: theta -> 0 is the direct sum,
    and the error against the direct sum falls as p rises."""
    c = inputs.config_lattice_1000()
    pos, box, m = c["pos"], c["box"], c["m"][0]
    Hd = ref.bruteforce(pos, m)
    H0 = ref.fmm(pos, m, 4, 1e-3, leaf_target=8, box=box, truncation=1)
    assert ref.rel_rms(H0, Hd) <= 1e-13
    errs = [ref.rel_rms(ref.fmm(pos, m, p, 0.5, leaf_target=8, box=box, truncation=1), Hd) for p in (2, 4, 6, 8)]
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    # at the same order the total-degree form keeps fewer terms: never more accurate here
    e_sep = ref.rel_rms(ref.fmm(pos, m, 4, 0.5, leaf_target=8, box=box), Hd)
    assert errs[1] > e_sep


def test_traceless_fold_and_fill_reproduce_m2l(ref):
    """D is harmonic (sum_a D_{k+2e_a} = 0).  Hence moving every moment with
    q_z >= 2 onto q - 2e_z + 2e_x and q - 2e_z + 2e_y with a minus sign
    (highest q_z first) leaves every V_n of M2L unchanged while the sum runs
    over the 2l+1 components with q_z <= 1 only, and V's n_z >= 2 components
    follow from V_{m+2e_z} = -V_{m+2e_x} - V_{m+2e_y}.  Checked here against
    the oracle's M2L and derivative tensor for random moments."""
    for p in (2, 3, 4, 5, 6):
        rng = np.random.default_rng(60 + p)
        full = [(x, y, d - x - y) for d in range(1, p + 1) for x in range(d, -1, -1) for y in range(d - x, -1, -1)]
        Q = np.zeros((p + 1,) * 3)
        for c in full:
            Q[c] = rng.normal()
        cvec = np.array([2.0, -3.0, 1.0]) + rng.uniform(-0.2, 0.2, 3)
        V = ref.m2l(p, cvec, Q)
        D = ref.dtensor(2 * p, cvec)
        Qf = Q.copy()
        for z in range(p, 1, -1):
            for x, y, zz in full:
                if zz == z:
                    Qf[x + 2, y, z - 2] -= Qf[x, y, z]
                    Qf[x, y + 2, z - 2] -= Qf[x, y, z]
        red = [c for c in full if c[2] <= 1]
        assert len(red) == p * (p + 2)
        Vr = np.zeros_like(V)
        for n in [(0, 0, 0)] + red:
            Vr[n] = (-1) ** sum(n) * sum(D[n[0] + q[0], n[1] + q[1], n[2] + q[2]] * Qf[q] for q in red)
        for z in range(2, p + 1):
            for x, y, zz in full:
                if zz == z:
                    Vr[x, y, z] = -Vr[x + 2, y, z - 2] - Vr[x, y + 2, z - 2]
        assert np.max(np.abs(Vr - V)) <= 1e-12 * np.max(np.abs(V)), p
