"""GPU re-study of the paper's leaf-size choice (Sec. 4, Table I and Eq. (so)).

The paper times its CPU code against the mean number s of dipoles per smallest
cell and fits the optimal s_o(p) = 0.74 p^2 (p > 3; 8 below).  Here the same
sweep runs on the GPU path unchanged: for each (p, theta) the number of levels
L is stepped around the paper's choice (s = N / 2^L selects exactly L), and
each tree is timed (one full step: rebuild for the positions plus the
evaluation; and the captured evaluation alone) and its error measured against
the FP64 direct sum at sampled dipoles.  The GPU-optimal s per order comes
from a parabola through the three fastest levels in log2 s, and c in
s_o = c p^2 from a least-squares fit over the orders above 3.
"""
import time

import numpy as np


def paper_s(p):
    """Eq. (so): s_o = 0.74 p^2 for p > 3, else 8."""
    return 0.74 * p * p if p > 3 else 8.0


def paper_levels(n, s):
    """The paper's level rule: L = argmin |N / 2^L - s| (ties: the smaller L)."""
    return int(np.argmin([abs(n / 2.0 ** L - s) for L in range(40)]))


def _timed(fn, reps, torch):
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def leaf_sweep(pos, box, m, pairs, dL=(-2, -1, 0, 1, 2), precision=None, reps=7, samples=1024, seed=11,
               progress=None):
    """Sweep the number of levels for each (p, theta) in pairs.

    pos [n][3], m [n][3] FP64 host arrays; box (lo, hi) or None.  Returns a list
    of records, one per (p, theta), with the swept points and the fitted
    optimum.  progress(str), if given, is called after every point."""
    import torch

    from paper_0810_0233_amd import ccfmm

    if precision is None:
        precision = ccfmm.PREC_MIXED
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    n = pos.shape[0]
    d_pos = torch.from_numpy(np.ascontiguousarray(pos)).to(dev)
    d_m = torch.from_numpy(np.ascontiguousarray(m[None])).to(dev)
    d_H = torch.empty_like(d_m)
    idx = np.sort(np.random.default_rng(seed).choice(n, size=min(samples, n), replace=False)).astype(np.int64)
    d_idx = torch.from_numpy(idx).to(dev)
    d_Hd = torch.empty((idx.size, 3), dtype=torch.float64, device=dev)
    ccfmm.direct_targets_device(n, d_pos.data_ptr(), d_m[0].data_ptr(), idx.size, d_idx.data_ptr(), d_Hd.data_ptr(),
                                st)
    torch.cuda.synchronize()
    Hd = d_Hd.cpu().numpy()
    out = []
    for p, th in pairs:
        L0 = paper_levels(n, paper_s(p))
        pts = []
        for d in dL:
            L = L0 + d
            if L < 1:
                continue
            prm = ccfmm.params(order=p, theta=th, leaf_target=n / 2.0 ** L, box=box, precision=precision,
                               max_batch=1)
            pl = ccfmm.Plan.create_device(n, d_pos.data_ptr(), prm, st)
            if precision == ccfmm.PREC_MIXED:
                pl.autotune(1, d_m.data_ptr(), d_H.data_ptr(), st)
            t_eval = _timed(lambda: pl.eval_device(1, d_m.data_ptr(), d_H.data_ptr(), st), reps, torch)

            def step():
                pl.update_positions_device(d_pos.data_ptr(), st)
                pl.eval_device(1, d_m.data_ptr(), d_H.data_ptr(), st)

            t_step = _timed(step, reps, torch)
            H = d_H[0].cpu().numpy()
            err = float(np.sqrt(np.sum((H[idx] - Hd) ** 2) / np.sum(Hd ** 2)))
            inf = pl.info()
            pl.destroy()
            pts.append({"levels": L, "s": n / 2.0 ** L, "eval_ms": 1e3 * t_eval, "step_ms": 1e3 * t_step,
                        "eps_abs": err, "m2l_pairs": inf["n_m2l_pairs"], "p2p_pairs": inf["n_p2p_pairs"]})
            if progress:
                progress("p=%d theta=%.2f L=%d s=%.2f: step %.3f ms, eval %.3f ms, eps_abs %.2e" % (
                    p, th, L, n / 2.0 ** L, 1e3 * t_step, 1e3 * t_eval, err))
        best = min(pts, key=lambda r: r["step_ms"])
        out.append({"order": p, "theta": th, "paper_s": paper_s(p), "paper_levels": L0, "points": pts,
                    "best_levels": best["levels"], "s_opt": optimum_s(pts, "step_ms"),
                    "s_opt_eval": optimum_s(pts, "eval_ms"),
                    "speedup_best_vs_paper": next(r["step_ms"] for r in pts if r["levels"] == L0) / best["step_ms"]})
    return out


def lattice_size_fit(sides, pairs, seed=6100, progress=None):
    """The paper's fit of s_o(p) over many system sizes (its Fig. 2) redone on
    the GPU: for every cubic lattice side in sides and every (p, theta) in
    pairs, a sweep of one level either side of the paper's tree gives the
    GPU-optimal s (parabola in log2 s through the three points).  Returns the
    records per side and the least-squares c in s_o = c p^2 over all of them
    (orders above 3)."""
    from . import inputs

    per_side = []
    for side in sides:
        pos, box = inputs.lattice(side, side, side)
        m = inputs.random_moments(pos.shape[0], seed + side)
        recs = leaf_sweep(pos, box, m, pairs, dL=(-1, 0, 1), reps=5, samples=256)
        per_side.append({"side": side, "n": int(pos.shape[0]), "records": recs})
        if progress:
            progress("lattice %d^3: %s" % (side, ", ".join("p=%d s_opt %.1f" % (r["order"], r["s_opt"]) for r in recs)))
    allrec = [r for ps in per_side for r in ps["records"]]
    by_p = {}
    for r in allrec:
        by_p.setdefault(r["order"], []).append(r["s_opt"])
    return {"sides": per_side, "c_fit": fit_c(allrec),
            "s_opt_mean": {p: float(np.mean(v)) for p, v in by_p.items()},
            "s_opt_median": {p: float(np.median(v)) for p, v in by_p.items()}}


def alpha_for_error(p, e):
    """The opening angle at which Sec. 3's estimate [alpha/(2-alpha)]^p equals e."""
    r = e ** (1.0 / p)
    return 2.0 * r / (1.0 + r)


def param_sweep(pos, box, m, errors, orders, reps=5, samples=0, seed=17, min_alpha=0.25, progress=None):
    """The paper's choice of (p, alpha) per error level (Table II, Fig. 3) on
    the GPU: for every estimate e in errors and order p in orders, alpha is set
    so that [alpha/(2-alpha)]^p = e, the tree follows the paper's s_o(p), and
    one full step (update for the positions + evaluation, mixed precision,
    M2L autotuned) is timed; the field error against the FP64 direct sum is
    measured.  Angles below min_alpha are skipped, and a plan the library
    refuses (lists beyond its limits) is recorded as such.  Returns the
    points and, per e, the fastest (p, alpha)."""
    import torch

    from . import ccfmm

    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    n = pos.shape[0]
    d_pos = torch.from_numpy(np.ascontiguousarray(pos)).to(dev)
    d_m = torch.from_numpy(np.ascontiguousarray(m[None])).to(dev)
    d_H = torch.empty_like(d_m)
    idx = np.arange(n) if not samples or samples >= n else np.sort(
        np.random.default_rng(seed).choice(n, samples, replace=False))
    d_idx = torch.from_numpy(idx.astype(np.int64)).to(dev)
    d_Hd = torch.empty((idx.size, 3), dtype=torch.float64, device=dev)
    ccfmm.direct_targets_device(n, d_pos.data_ptr(), d_m[0].data_ptr(), idx.size, d_idx.data_ptr(), d_Hd.data_ptr(),
                                st)
    pts = []
    for e in errors:
        for p in orders:
            a = alpha_for_error(p, e)
            if not min_alpha <= a < 1.0:  # tiny angles: near lists of whole regions, never the fastest
                continue
            prm = ccfmm.params(order=p, theta=a, box=box, precision=ccfmm.PREC_MIXED, max_batch=1)
            try:
                pl = ccfmm.Plan.create_device(n, d_pos.data_ptr(), prm, st)
            except ccfmm.CCFMMError as err:  # lists beyond the plan's limits at this size
                pts.append({"e": e, "order": p, "alpha": a, "refused": str(err)})
                continue
            pl.autotune(1, d_m.data_ptr(), d_H.data_ptr(), st)

            def step():
                pl.update_positions_device(d_pos.data_ptr(), st)
                pl.eval_device(1, d_m.data_ptr(), d_H.data_ptr(), st)

            t = _timed(step, reps, torch)
            H = d_H[0][d_idx]
            err = float(torch.sqrt(torch.sum((H - d_Hd) ** 2) / torch.sum(d_Hd ** 2)))
            pl.destroy()
            pts.append({"e": e, "order": p, "alpha": a, "step_ms": 1e3 * t, "eps_abs": err})
            if progress:
                progress("e=%.3g p=%d alpha=%.3f: step %.3f ms, eps_abs %.2e" % (e, p, a, 1e3 * t, err))
    best = {}
    for e in errors:
        cand = [q for q in pts if q["e"] == e and "step_ms" in q]
        if cand:
            b = min(cand, key=lambda q: q["step_ms"])
            best[str(e)] = {"order": b["order"], "alpha": b["alpha"], "step_ms": b["step_ms"], "eps_abs": b["eps_abs"]}
    return {"points": pts, "best": best}


def optimum_s(pts, key):
    """s at the minimum of a parabola through the fastest point and its two
    neighbours in log2 s (the fastest point itself at an end of the sweep)."""
    pts = sorted(pts, key=lambda r: r["s"])
    k = min(range(len(pts)), key=lambda i: pts[i][key])
    if k == 0 or k == len(pts) - 1:
        return pts[k]["s"]
    x = np.log2([pts[k - 1]["s"], pts[k]["s"], pts[k + 1]["s"]])
    y = np.array([pts[k - 1][key], pts[k][key], pts[k + 1][key]])
    a, b, _ = np.polyfit(x, y, 2)
    if a <= 0:
        return pts[k]["s"]
    return float(2.0 ** np.clip(-b / (2 * a), x[0], x[2]))


def fit_c(records):
    """Least-squares c in s_opt = c p^2 over the orders above 3 (Eq. (so)'s form)."""
    rs = [r for r in records if r["order"] > 3]
    if not rs:
        return None
    p2 = np.array([r["order"] ** 2 for r in rs], dtype=float)
    s = np.array([r["s_opt"] for r in rs], dtype=float)
    return float(np.dot(p2, s) / np.dot(p2, p2))


def paper_error_estimate(p, theta):
    """Sec. 3: the truncation error of a multipole expansion of order p at
    opening angle theta is of order e = [theta / (2 - theta)]^p."""
    return (theta / (2.0 - theta)) ** p


def truncation_study(pos, box, m, settings, precision=None, reps=5, samples=0, seed=13, progress=None):
    """Both readings of Sec. 3's truncation on the GPU path: for every (p,
    theta) in settings and truncation 0 (multipoles and locals each to order
    p) and 1 (total degree |n| + |q| <= p), the field error against the FP64
    direct sum (at every dipole, or at `samples` seeded dipoles), the relative
    energy error (every dipole only), the evaluation time (median of reps) and
    the M2L pass time (M2L kernel autotuned per plan).  One configuration m
    [n][3]."""
    import torch

    from . import ccfmm

    precision = ccfmm.PREC_FP64 if precision is None else precision
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    n = pos.shape[0]
    d_pos = torch.from_numpy(np.ascontiguousarray(pos)).to(dev)
    d_m = torch.from_numpy(np.ascontiguousarray(m)).to(dev)
    d_H = torch.empty_like(d_m)
    idx = np.arange(n) if not samples or samples >= n else np.sort(
        np.random.default_rng(seed).choice(n, samples, replace=False))
    d_idx = torch.from_numpy(idx.astype(np.int64)).to(dev)
    d_Hd = torch.empty((idx.size, 3), dtype=torch.float64, device=dev)
    ccfmm.direct_targets_device(n, d_pos.data_ptr(), d_m.data_ptr(), idx.size, d_idx.data_ptr(), d_Hd.data_ptr(), st)
    torch.cuda.synchronize()
    E_d = float(-0.5 * torch.sum(d_m * d_Hd)) if idx.size == n else None
    out = []
    for p, theta in settings:
        for trunc in (0, 1):
            prm = ccfmm.params(order=p, theta=theta, box=box, precision=precision, max_batch=1, truncation=trunc)
            pl = ccfmm.Plan.create_device(n, d_pos.data_ptr(), prm, st)
            pl.autotune(1, d_m.data_ptr(), d_H.data_ptr(), st)
            t = _timed(lambda: pl.eval_device(1, d_m.data_ptr(), d_H.data_ptr(), st), reps, torch)
            H = d_H[d_idx]
            err = float(torch.sqrt(torch.sum((H - d_Hd) ** 2) / torch.sum(d_Hd ** 2)))
            rec = {"order": p, "theta": theta, "truncation": trunc, "eps_abs": err,
                   "e_paper": paper_error_estimate(p, theta), "eval_ms": 1e3 * t,
                   "m2l_ms": pl.eval_device_timed(1, d_m.data_ptr(), d_H.data_ptr(), st)["m2l"],
                   "levels": pl.info()["levels"]}
            if E_d is not None:
                E = float(-0.5 * torch.sum(d_m * d_H))
                rec["energy_rel_err"] = abs(E - E_d) / abs(E_d)
            pl.destroy()
            out.append(rec)
            if progress:
                progress("  p=%d theta=%.2f truncation=%d: eps_abs %.3e (paper e %.3e) eval %.3f ms m2l %.3f ms" % (
                    p, theta, trunc, rec["eps_abs"], rec["e_paper"], rec["eval_ms"], rec["m2l_ms"]))
    return out
