"""Benchmark: dipole-field evaluations per second of the Cartesian FMM on one GPU.

Default workload (`--workload film`): the 1024 x 1024 x 16 thin-film lattice
with 16 circular holes (radii 20-80; 14,482,960 sites), 8 magnetisation
configurations evaluated together, learned per-cell (p, theta) for a 1e-5
bound against fixed p = 6, theta = 0.4, mixed precision (FP32 bulk arithmetic
on MFMA/VALU, FP64 derivative tensors and final per-dipole sums); the plain
FP64 GPU FMM, the best uniform (p, theta) and the CPU oracle on a window of the
film are reported beside it.  The shipped weights were trained on two films of
the same recipe with other seeds; the selection is made once per geometry, at
the plan's first evaluation, with its judge (timed as selection_ms).

`--workload ferrofluid`: 1,048,576 hard-core dipoles (random sequential
addition, volume fraction 0.1, seed 2001), unit moments in random directions
(seed 2002), order p = 6, opening angle 0.5, s = s_o(6) = 26.64 dipoles per
smallest cell, mixed precision.

`--workload sphere`: 262,144 lattice sites cut as a sphere from an 80^3 cubic
lattice, 64 magnetisation configurations (random directions plus 0-50% of
seeded sites aligned along +z), p = 5, theta = 0.5, evaluated together.

For the ferrofluid and the sphere, a step is one pass of the whole method over
one batch with the positions and moments already in HBM: tree rebuilt in place for moved dipoles (the steps
alternate between the configuration's positions and a copy displaced by
N(0, 0.01^2) per coordinate), cell lists and M2L tiles rebuilt unless the
same cells stay occupied (then they are provably unchanged and kept),
derivative tensors, P2M, M2M, M2L, L2L, L2P and the near-field sum.  The step
with every list and tile rebuilt is reported beside it.  `value` = dipoles x configurations / step time.  The same run reports
the evaluation alone (tree reused, captured graph replayed), the plain FP64
GPU FMM, the error of the mixed result against the FP64 GPU FMM (eps_prec) and
against the direct sum at sampled dipoles (eps_abs), the roofline of the
dominant kernel, and the CPU oracle timed on the same workload (configuration 0).

`--workload clusters`: 2^21 dipoles in 256 Gaussian clusters with learned per-cell
(p, theta) for a 1e-5 bound against fixed p = 6, theta = 0.4 (the network is
trained on the GPU first, from two training geometries of the same recipe).

`--workload dynamics`: the ferrofluid geometry in a time-stepping loop: one plan,
its captured evaluation replayed after every in-place precession step of the
moments, the energy taken on the GPU every step (and the same loop in FP64).

`--workload leaffit`: the paper's fit of s_o(p) over many system sizes (Fig. 2)
on the GPU: 30 cubic lattices of side 16 to 132, p = 4, 5, 6.

`--workload params`: the paper's choice of (p, alpha) per error level (Table II,
Fig. 3) on the GPU, on 32^3 and 128^3 lattices.

`--workload truncation`: both readings of the paper's truncation (each index to
order p, or total degree |n| + |q| <= p): errors against the direct sum, energy
errors and times on the 32^3 lattice and the ferrofluid.

`--workload leafsweep`: the paper's leaf-size study (Table I, Eq. (so)) redone on
the GPU path: trees two levels either side of s_o(p) for Table II's (p, alpha)
pairs, on 32^3 and 128^3 lattices and the ferrofluid.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload film|ferrofluid|sphere|clusters|dynamics|leafsweep|leaffit|params|truncation]
                       [--skip-cpu] [--skip-fp64] [--skip-sweep] [--roofline-only] [--calib-copy]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dipole-field evals/s at ≤1e-5 rel RMS err: mixed/learned FMM vs plain FP64"
PEAK_FP32_MFMA = 157.3e12   # MI355X dense FP32 matrix, FLOP/s
PEAK_FP64_MFMA = 78.6e12
PEAK_FP32_VALU = 157.3e12   # published vector FP32 (packed); see the design notes
PEAK_HBM = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_rms(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def workload(args, inputs):
    if args.workload == "ferrofluid":
        n = args.n or (1 << 20)
        pos, box = inputs.ferrofluid(n, 2001)
        m = inputs.random_moments(n, 2002)[None]
        return dict(name="ferrofluid_rsa_%d" % n, pos=pos, box=box, m=m, order=args.order or 6,
                    theta=args.theta)
    if args.workload == "sphere":
        n = args.n or (1 << 18)
        nb = args.batch or 64
        pos, box = inputs.sphere_cut(n, 80)
        m = inputs.aligned_moments(n, nb, 3000)
        return dict(name="sphere_%d_of_80cube_x%d" % (n, nb), pos=pos, box=box, m=m, order=args.order or 5,
                    theta=args.theta)
    raise SystemExit("unknown workload " + args.workload)


# Algorithmic work per pass (what the method must read, write and compute,
# not what the kernels happen to move):
#  p2m      m (FP64, 24 B) + position (FP32 leaf-relative, 12 B) per dipole
#           and configuration; write Q (4 B x NS) per leaf and configuration;
#           2 * 3 * NP flop per dipole and configuration
#  m2m/l2l  read and write one expansion (4 B x NS) per cell and configuration
#  m2l      read Q and write V once per cell and configuration, one FP32
#           derivative tensor per distinct offset is ignored (< 1 %);
#           2 NP^2 flop per (pair, configuration)
#  p2p      near field: position 12 B + moment 12 B per dipole (sources
#           counted once), FP64 field 24 B written per dipole and configuration;
#           flops per near_flops (one configuration: 26 per pair; 2..31
#           configurations: 10 per pair + 16 per (pair, configuration); the
#           batched matrix-core form: 18 per (pair, configuration))
#  l2p      smooth field added: V per cell, position 12 B per dipole, the FP64
#           field read and written (48 B per dipole and configuration);
#           2 * 3 * N(p-1) flop per dipole and configuration
def pass_work(info, n, nb, order):
    NP = (order + 1) * (order + 2) * (order + 3) // 6 - 1
    NS = (NP + 3) // 4 * 4
    leaves, cells = info["n_leaves"], info["n_cells"]
    pairs = info["n_p2p_pairs"]
    batched = nb >= 32
    exp_b = 4.0 * NS * nb
    l2p_flops = 6.0 * (order * (order + 1) * (order + 2) // 6) * n * nb
    out = {
        "p2m": {"kernel": "k_permute_moments+k_p2m<float,%d>" % order, "bound": "hbm",
                "bytes": n * nb * 24.0 + n * 12.0 + leaves * exp_b, "flops": 6.0 * NP * n * nb},
        # (the passes are timed on one stream: M2M and L2L in their staged form, one launch per level and halved
        # axis; M2M also writes the folded moments, L2L completes the local rows)
        "m2m": {"kernel": "k_m2m<float,%d,axis,true>" % order, "bound": "hbm", "bytes": 2.0 * cells * exp_b,
                "flops": 0.0},
        # the method's own M2L products: 2 NP^2 per pair and configuration, NP = (p+1)(p+2)(p+3)/6 - 1 in the
        # full form, p (p + 2) in the traceless form (the fold and fill are per-cell work)
        "m2l": {"kernel": m2l_kernel_name(info["m2l_variant"], order),
                "bound": "mfma", "bytes": 2.0 * cells * exp_b,
                "flops": (2.0 * (order * (order + 2)) ** 2 * info["n_m2l_pairs"] * nb
                          if m2l_traceless_active(info["m2l_variant"], order) else info["m2l_flops_per_config"] * nb)},
        "l2l": {"kernel": "k_l2l<float,%d,true,axis>" % order, "bound": "hbm", "bytes": 2.0 * cells * exp_b,
                "flops": 0.0},
        # each input read once: FP32 position and residual (24 B), moment (12 B per configuration), caller
        # index (4 B), the smallest cells' local expansions when L2P is fused; FP64 field written (24 B)
        "p2p": {"kernel": near_kernel_name(nb, order),
                "bound": "mfma" if batched else "alu",
                "bytes": n * 28.0 + n * nb * 36.0 + (0.0 if batched else leaves * exp_b),
                "flops": near_flops(pairs, nb) + (0.0 if batched else l2p_flops)},
        "l2p": {"kernel": ("k_l2p_batched<float,%d,true>" % order if batched
                           else "fused into " + near_kernel_name(nb, order)), "bound": "hbm",
                "bytes": leaves * exp_b + n * 12.0 + n * nb * 48.0,
                "flops": l2p_flops},
    }
    for v in out.values():
        v["peak"] = PEAK_FP32_MFMA if v["bound"] == "mfma" else PEAK_FP32_VALU
    return out


def multi_group(nb):
    """Configurations per lane of the library's few-configuration near field
    (2..31 configurations): the group of 2, 4 or 8 with the fewest vector
    operations, ceil(nb / KB) (13 + 10 KB) per pair."""
    return min((2, 4, 8), key=lambda kb: (-(-nb // kb) * (13.0 + 10.0 * kb), kb))


def near_kernel_name(nb, order):
    """The near-field kernel of a pass timed alone (single stream): the smooth
    field is fused into it below the matrix-core size."""
    if nb >= 32:
        return "k_p2p_mfma"
    if nb >= 2:
        return "k_p2p_multi<float,%d,%d>" % (multi_group(nb), order)
    return "k_p2p_l2p<float,%d,true>" % order


def near_flops(pairs, nb):
    """Algorithmic flops of the near field: one configuration 26 per pair (3
    differences, r^2, the reciprocal square root, r^-2 and r^-3, m.r, the
    three components); several configurations share the pair geometry:
    10 per pair + 16 per (pair, configuration); the matrix-core form counts
    its 3x3 tensor product, 18 per (pair, configuration)."""
    if nb >= 32:
        return 18.0 * pairs * nb
    if nb >= 2:
        return pairs * (10.0 + 16.0 * nb)
    return 26.0 * pairs


def m2l_traceless_active(variant, order):
    """Whether the M2L pass runs in the traceless form (the default for the
    mixed-precision wide kernels, orders <= 6)."""
    return variant in (2, 3, 4) and order <= 8


def m2l_kernel_name(variant, order, t="float"):
    """The M2L kernel a plan's variant launches (element type t; the wide
    kernels in the traceless form)."""
    return {0: "k_m2l<%s,%d>" % (t, order), 1: "k_m2l_wave<%s,%d>" % (t, order),
            2: "k_m2l_wide<%s,%d,4,true>" % (t, order), 3: "k_m2l_wide<%s,%d,2,true>" % (t, order),
            4: "k_m2l_wide<%s,%d,1,true>" % (t, order)}[variant]


# the source file that defines each kernel family
KERNEL_SRC = (("k_p2p", "p2p.hip"), ("k_l2p", "p2p.hip"), ("k_m2l", "m2l.hip"), ("k_fold", "m2l.hip"),
              ("k_fill", "m2l.hip"), ("k_p2m", "expansions.hip"),
              ("k_m2m", "expansions.hip"), ("k_l2l", "expansions.hip"), ("k_permute", "expansions.hip"))


def kernel_digest(kernel):
    """SHA-256 over the source file that defines the kernel and the shared
    headers (names and bytes, sorted): what the kernel's machine code is built
    from."""
    import hashlib

    d = os.path.join(ROOT, "paper_0810_0233_amd", "csrc")
    own = sorted({f for prefix, f in KERNEL_SRC if kernel.startswith(prefix)})
    h = hashlib.sha256()
    for f in own + sorted(x for x in os.listdir(d) if x.endswith(".hpp")):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


TRAFFIC_PATH = os.path.join(ROOT, "profiles", "traffic.json")


def counted_traffic(kernel, workload_name):
    """HBM bytes per launch from the committed counter record of this
    workload, or None when there is none or the kernel sources changed since
    the counters were taken."""
    try:
        with open(TRAFFIC_PATH) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    k = rec.get("workloads", {}).get(workload_name, {}).get("kernels", {}).get(kernel)
    if not k or k.get("src_sha256") != kernel_digest(kernel):
        return None
    return k.get("hbm_bytes_per_launch")


def read_counter_csv(d):
    """rocprofv3 --pmc counter CSV (one file under d): per kernel name the
    list of per-dispatch counter values."""
    import csv
    import glob

    files = sorted(glob.glob(os.path.join(d, "**", "*counter_collection*.csv"), recursive=True))
    if not files:
        raise SystemExit("no counter CSV under " + d)
    out = {}
    with open(files[0]) as fh:
        for row in csv.DictReader(fh):
            key = (row["Kernel_Name"], int(row["Dispatch_Id"]))
            out[key] = out.get(key, 0.0) + float(row["Counter_Value"])
    per = {}
    for (name, did), v in sorted(out.items(), key=lambda kv: kv[0][1]):
        per.setdefault(name, []).append(v)
    # the run's closing calibration copy: its last copy dispatch
    copies = [(did, v) for (name, did), v in out.items() if "copy" in name.lower()]
    calib = max(copies)[1] if copies else None
    return per, calib


def short_kernel_name(name):
    """'void ccfmm::k_p2p_multi<float, 8>(...)' -> 'k_p2p_multi<float,8>'"""
    base = name.split("(")[0].replace("void ", "").replace("ccfmm::", "").strip()
    return base.replace(", ", ",")


def write_traffic_record(workload_name, fetch_dir, write_dir, summary_path):
    """Fold two counter runs (FETCH_SIZE, then WRITE_SIZE, in KiB per
    dispatch) into the traffic record of one workload: bytes per launch,
    each counter scaled by what it reads for the run's closing 256 MiB device
    copy (the calibration: a copy fetches and writes 256 MiB)."""
    (fetch, cf), (write, cw) = read_counter_csv(fetch_dir), read_counter_csv(write_dir)
    if not cf or not cw:
        raise SystemExit("no calibration copy in the counter runs")
    fs, ws = (256 << 10) / cf, (256 << 10) / cw
    try:
        with open(TRAFFIC_PATH) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        rec = {}
    rec.setdefault("workloads", {})
    kern = {}
    rows = []
    for name in sorted(set(fetch) & set(write)):
        short = short_kernel_name(name)
        if not short.startswith("k_"):
            continue
        f = float(np.mean(fetch[name]))
        w = float(np.mean(write[name]))
        b = 1024.0 * (f * fs + w * ws)
        kern[short] = {"fetch_kib": f, "write_kib": w, "hbm_bytes_per_launch": b, "src_sha256": kernel_digest(short)}
        rows.append("| `%s` | %d | %.1f | %.1f | %.4g |" % (short, len(fetch[name]), f, w, b))
    rec["workloads"][workload_name] = {"fetch_scale": fs, "write_scale": ws, "source": summary_path,
                                       "kernels": kern}
    with open(TRAFFIC_PATH, "w") as fh:
        json.dump(rec, fh, indent=1)
    return fs, ws, rows


def bench_learned(args, torch, ccfmm, inputs):
    """Learned per-cell parameters for a 1e-5 bound against fixed p = 6,
    theta = 0.4 on clusters: 2^21 dipoles in 256 Gaussian clusters (sigma 8,
    box 512^3).

    The network is trained first (two 1/8-size training geometries of the
    same recipe; GPU labels and GPU training, timed apart).  The learned plan
    makes its choice at its first evaluation, with its judge (timed apart as
    selection_ms); a timed step then updates the plan for the positions (the
    occupied cells stay, so lists and choice are kept) and evaluates."""
    from paper_0810_0233_amd import selector

    dev = torch.device("cuda:0")
    sh = torch.cuda.current_stream().cuda_stream
    t0 = time.time()
    train_cfgs = [inputs.config_clusters_training(4101), inputs.config_clusters_training(4102)]
    params, losses, ncells = selector.train_on(train_cfgs, steps=600)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    log("selector trained on %d cells in %.1f s, loss %s" % (ncells, t_train, losses))
    del train_cfgs
    c = inputs.config_clusters()
    pos, box, m = c["pos"], c["box"], c["m"]
    nb, n = m.shape[0], pos.shape[0]
    bound = 1e-5
    log("inputs: %s n=%d batch=%d" % (c["name"], n, nb))
    d_pos = torch.from_numpy(pos).to(dev)
    d_m = torch.from_numpy(np.ascontiguousarray(m)).to(dev)
    del m
    d_H = torch.empty_like(d_m)
    d_P = torch.from_numpy(params).to(dev)

    def make(prec, **kw):
        prm = ccfmm.params(order=6, theta=0.4, leaf_target=0.0, box=box, precision=prec, max_batch=nb, **kw)
        return ccfmm.Plan.create_device(n, d_pos.data_ptr(), prm, sh)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    def dev_rel_rms(a, b):
        return float(torch.sqrt(torch.sum((a - b) ** 2) / torch.sum(b ** 2)))

    # ---- fixed (6, 0.4)
    plan = make(ccfmm.PREC_MIXED)
    plan.autotune(nb, d_m.data_ptr(), d_H.data_ptr(), sh)
    fixed_info = plan.info()

    def step(pl):
        def f():
            pl.update_positions_device(d_pos.data_ptr(), sh)
            pl.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), sh)
        return f

    t_fixed = timed(step(plan), args.steps, args.warmup)
    H_fixed = d_H.clone()
    passes_fixed = plan.eval_device_timed(nb, d_m.data_ptr(), d_H.data_ptr(), sh)
    plan.destroy()

    # ---- learned: the plan's choice at its first evaluation (with its judge,
    # timed apart), kept by the steps (same cells)
    plan = make(ccfmm.PREC_MIXED, selector=1, err_bound=bound)
    plan.selector_set(d_P.data_ptr(), sh)
    plan.autotune(nb, d_m.data_ptr(), d_H.data_ptr(), sh)
    torch.cuda.synchronize()
    t = time.perf_counter()
    status = plan.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), sh)
    torch.cuda.synchronize()
    t_select = time.perf_counter() - t
    t_learned = timed(step(plan), args.steps, args.warmup)
    H_learned = d_H.clone()
    t_learned_eval = timed(lambda: plan.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), sh), args.steps, 1)
    learned_info = plan.info()
    lp, lth = plan.get_leaf_params()
    hist = {"%d,%.1f" % (p_, t_): int(np.sum((lp == p_) & (np.abs(lth - t_) < 1e-9)))
            for p_ in ccfmm.SEL_P for t_ in ccfmm.SEL_THETA}
    hist = {k: v for k, v in hist.items() if v}
    # pass times, each kernel alone on one stream
    passes = plan.eval_device_timed(nb, d_m.data_ptr(), d_H.data_ptr(), sh)
    log("fixed passes, one stream (ms): %s" % json.dumps({k: round(v, 3) for k, v in passes_fixed.items()}))
    log("learned passes, one stream (ms): %s" % json.dumps({k: round(v, 3) for k, v in passes.items()}))
    log("fixed step %.3f ms, learned step %.3f ms (eval %.3f ms), choice %.1f ms status %d judge %.3e" % (
        1e3 * t_fixed, 1e3 * t_learned, 1e3 * t_learned_eval, 1e3 * t_select, status, learned_info["judge_err"]))
    plan.destroy()
    out = {}
    if not args.skip_fp64:
        p64 = make(ccfmm.PREC_FP64)  # the same forms as the mixed plans (autotuned)
        p64.autotune(nb, d_m.data_ptr(), d_H.data_ptr(), sh)

        t64 = timed(step(p64), max(2, args.steps // 5), 1)
        out["fp64_full_step_ms"] = 1e3 * t64
        out["speedup_vs_fp64_step"] = t64 / t_learned
        out["eps_prec_fixed_mixed"] = dev_rel_rms(H_fixed, d_H)
        out["eps_learned_vs_fp64_fixed"] = dev_rel_rms(H_learned, d_H)
        log("fp64 step %.3f ms; mixed fixed vs fp64 %.3e, learned vs fp64 %.3e" % (
            1e3 * t64, out["eps_prec_fixed_mixed"], out["eps_learned_vs_fp64_fixed"]))
        p64.destroy()
    # error against the FP64 direct sum at sampled dipoles, configuration 0 (GPU)
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(n, size=min(args.samples, n), replace=False)).astype(np.int64)
    d_idx = torch.from_numpy(idx).to(dev)
    d_Hd = torch.empty((idx.size, 3), dtype=torch.float64, device=dev)
    ccfmm.direct_targets_device(n, d_pos.data_ptr(), d_m[0].data_ptr(), idx.size, d_idx.data_ptr(),
                                d_Hd.data_ptr(), sh)
    torch.cuda.synchronize()
    out["eps_abs_fixed"] = dev_rel_rms(H_fixed[0][d_idx], d_Hd)
    out["eps_abs_learned"] = dev_rel_rms(H_learned[0][d_idx], d_Hd)
    kern = pass_work(learned_info, n, nb, 6)
    dom = "m2l" if passes["m2l"] >= passes["p2p"] else "p2p"
    ach = kern[dom]["flops"] / (passes[dom] * 1e-3)
    roof = {"kernel": kern[dom]["kernel"], "bound": kern[dom]["bound"], "achieved": ach / 1e12,
            "peak": kern[dom]["peak"] / 1e12, "unit": "TFLOP/s", "frac": ach / kern[dom]["peak"],
            "traffic": counted_traffic(kern[dom]["kernel"], c["name"])}
    res = {
        "metric": METRIC,
        "value": n * nb / t_learned,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_learned,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": c["name"], "n": n, "batch": nb, "order": 6, "theta": 0.4, "precision": "mixed",
                   "selector": "learned", "err_bound": bound,
                   "step": "position update (lists and choice kept) + evaluation",
                   "selection": "once per geometry at the first evaluation, with its judge (selection_ms)"},
        "selection_ms": 1e3 * t_select,
        "selection_status": status,
        "fixed_full_step_ms": 1e3 * t_fixed,
        "speedup_learned_vs_fixed_step": t_fixed / t_learned,
        "learned_eval_ms": 1e3 * t_learned_eval,
        "passes_ms": passes,
        "passes_fixed_ms": passes_fixed,
        "cost_far": learned_info["sel_cost_far"],
        "choice_hist": hist,
        "judge_err": learned_info["judge_err"],
        "learned": learned_info["learned"],
        "fallback": learned_info["fallback"],
        "p2p_pairs": {"fixed": fixed_info["p2p_pairs_per_config"], "learned": learned_info["p2p_pairs_per_config"]},
        "m2l_pairs": {"fixed": fixed_info["n_m2l_pairs"], "learned": learned_info["n_m2l_pairs"]},
        "selector_training_s": t_train,
        "roofline": roof,
        "cpu_baseline": None,
    }
    res.update(out)
    print(json.dumps(res), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Threads the oracle runs on: the OpenMP setting if given, else every core."""
    try:
        return max(1, int(os.environ.get("OMP_NUM_THREADS", "")))
    except ValueError:
        return os.cpu_count() or 1


def film_window(pos, m, box, w):
    """A w x w window of the film (all layers, holes included): of the film's
    w x w tiles, the one whose site count is closest to the film's mean per
    tile (ties to the first in x, then y), with its root box."""
    lo = np.asarray(box[0], float)
    nx = int(round(box[1][0] - box[0][0]))
    ny = int(round(box[1][1] - box[0][1]))
    tx = ((pos[:, 0] - lo[0]) // w).astype(np.int64)
    ty = ((pos[:, 1] - lo[1]) // w).astype(np.int64)
    ntx, nty = nx // w, ny // w
    cnt = np.bincount(tx * nty + ty, minlength=ntx * nty)
    k = int(np.argmin(np.abs(cnt - pos.shape[0] / (ntx * nty))))
    x0, y0 = lo[0] + (k // nty) * w, lo[1] + (k % nty) * w
    sel = (tx == k // nty) & (ty == k % nty)
    wlo = np.array([x0, y0, lo[2]])
    whi = np.array([x0 + w, y0 + w, box[1][2]])
    return pos[sel], m[sel], (wlo, whi)


def per_dipole_stats(H, Href):
    d = np.linalg.norm(H - Href, axis=-1)
    r = np.linalg.norm(Href, axis=-1)
    e = d[r > 0] / r[r > 0]
    return {"median": float(np.median(e)), "p99": float(np.percentile(e, 99)), "max": float(e.max()),
            "max_over_rms_field": float(d.max() / np.sqrt(np.mean(r * r)))}


def calibration_copy(torch, dev):
    """One plain 256 MiB device-to-device copy: the counter runs' scale (its
    FETCH_SIZE and WRITE_SIZE readings against the bytes it moves)."""
    a = torch.empty(64 << 20, dtype=torch.float32, device=dev)
    b = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    a.copy_(b)
    torch.cuda.synchronize()
    return 256 << 20


def film_roofline(li, pt, n, nb, name):
    """Per-pass work of the film's learned plan and the roofline of its
    dominant pass (times: HIP events the library records on the launch
    stream, every pass alone)."""
    kern = pass_work(li, n, nb, 6)
    if nb < 32:
        pt["l2p"] = 0.0  # fused into the near-field kernel (the timer brackets nothing)
    for k, v in kern.items():
        v["ms"] = pt[k]
        if pt[k] <= 0.0:
            continue
        sec = pt[k] * 1e-3
        v["gb_s"] = v["bytes"] / sec / 1e9
        v["hbm_frac"] = v["bytes"] / sec / PEAK_HBM
        if v["flops"]:
            v["tflop_s"] = v["flops"] / sec / 1e12
            v["flop_frac"] = v["flops"] / sec / v["peak"]
    dom = max(("m2l", "p2p"), key=lambda k: pt[k])
    d = kern[dom]
    ach = d["flops"] / (pt[dom] * 1e-3)
    roof = {"kernel": d["kernel"], "bound": d["bound"], "achieved": ach / 1e12, "peak": d["peak"] / 1e12,
            "unit": "TFLOP/s", "frac": ach / d["peak"], "traffic": counted_traffic(d["kernel"], name),
            "algorithmic_bytes": d["bytes"]}
    return {k: {q: v[q] for q in v if q != "peak"} for k, v in kern.items()}, roof


def bench_film(args, torch, ccfmm, inputs):
    """The thin-film workload: 1024 x 1024 x 16 lattice with 16 circular holes
    (14,482,960 sites), 8 magnetisation configurations evaluated together,
    FP32 bulk arithmetic, learned per-cell (p, theta) for a 1e-5 relative RMS
    bound with fixed (6, 0.4) as judge and fallback.

    The selector weights come from the package's weights file (trained by
    `python -m paper_0810_0233_amd.selector --workload film`); if it is
    missing they are trained here first.  The learned choice (with its judge)
    is made once per geometry, at the first evaluation of the cells, and timed
    apart; a timed step then updates the plan for the film's positions (the
    occupied cells stay, so lists and choice are kept) and evaluates all 8
    configurations."""
    from paper_0810_0233_amd import selector

    dev = torch.device("cuda:0")
    sh = torch.cuda.current_stream().cuda_stream
    t0 = time.time()
    c = inputs.config_film()
    pos, box, m = c["pos"], c["box"], c["m"]
    nb, n = m.shape[0], pos.shape[0]
    bound = 1e-5
    log("inputs: %s n=%d batch=%d (%.1f s)" % (c["name"], n, nb, time.time() - t0))
    d_pos = torch.from_numpy(pos).to(dev)
    d_m = torch.from_numpy(np.ascontiguousarray(m)).to(dev)
    d_H = torch.empty_like(d_m)

    def make(prec, **kw):
        prm = ccfmm.params(order=6, theta=0.4, leaf_target=0.0, box=box, precision=prec, max_batch=nb, **kw)
        return ccfmm.Plan.create_device(n, d_pos.data_ptr(), prm, sh)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    def dev_rel_rms(a, b):
        return float(torch.sqrt(torch.sum((a - b) ** 2) / torch.sum(b ** 2)))

    # ---- the learned plan: weights, then the choice at its first evaluation
    out = {}
    plan = make(ccfmm.PREC_MIXED, selector=1, err_bound=bound, sel_margin=selector.FILM_MARGIN)
    wpath = os.path.join(selector.WEIGHTS_DIR, selector.FILM_WEIGHTS)
    rc = plan.selector_load(wpath)
    if rc == ccfmm.W_NOWEIGHTS:
        log("no weights file %s: training the selector first" % wpath)
        t = time.time()
        params, losses, rows = selector.train_film(None)
        out["selector_training_s"] = time.time() - t
        d_P = torch.from_numpy(params).to(dev)
        plan.selector_set(d_P.data_ptr(), sh)
        out["selector_weights"] = "trained in this run on %d cells, loss %s" % (rows, losses)
    else:
        out["selector_weights"] = os.path.relpath(wpath, ROOT)
    if not args.roofline_only:
        plan.autotune(nb, d_m.data_ptr(), d_H.data_ptr(), sh)
    torch.cuda.synchronize()
    t = time.perf_counter()
    status = plan.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), sh)
    torch.cuda.synchronize()
    t_select = time.perf_counter() - t
    li = plan.info()
    log("learned choice: status %d learned %d judge %.3e cost_far %.1f (%.1f ms with its judge)" % (
        status, li["learned"], li["judge_err"], li["sel_cost_far"], 1e3 * t_select))
    log("evaluation form: %s (tuned: near field beside %.3f ms, one stream %.3f ms)" % (
        "near field beside the expansion passes" if li["overlap_near"] else "one stream", *li["tune_eval_ms"]))

    def step(pl):
        def f():
            pl.update_positions_device(d_pos.data_ptr(), sh)
            pl.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), sh)
        return f

    t_learned = timed(step(plan), args.steps, args.warmup)
    H_learned = d_H.clone()
    t_learned_eval = timed(lambda: plan.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), sh), args.steps, 1)
    passes = [plan.eval_device_timed(nb, d_m.data_ptr(), d_H.data_ptr(), sh) for _ in range(3)]
    pt = {k: float(np.median([p_[k] for p_ in passes])) for k in passes[0]}
    li = plan.info()
    lp, lth = plan.get_leaf_params()
    hist = {"%d,%.1f" % (p_, t_): int(np.sum((lp == p_) & (np.abs(lth - t_) < 1e-9)))
            for p_ in ccfmm.SEL_P for t_ in ccfmm.SEL_THETA}
    hist = {k: v for k, v in hist.items() if v}
    log("learned step %.2f ms, eval %.2f ms; passes (one stream) %s; choice %s" % (
        1e3 * t_learned, 1e3 * t_learned_eval, json.dumps({k: round(v, 2) for k, v in pt.items()}), hist))
    plan.destroy()
    if args.roofline_only:
        # counter runs: the learned plan alone, untuned (the near field beside
        # the expansion passes), so the fused near-field kernel of the roofline
        # runs only in the three timed evaluations
        kern, roof = film_roofline(li, pt, n, nb, c["name"])
        res = {"metric": METRIC, "workload": c["name"], "roofline_only": True, "passes_ms": pt, "roofline": roof,
               "kernels": kern}
        if args.calib_copy:
            res["calib_copy_bytes"] = calibration_copy(torch, dev)
        print(json.dumps(res), flush=True)
        return

    # ---- fixed (6, 0.4), the same step
    fixed = make(ccfmm.PREC_MIXED)
    fixed.autotune(nb, d_m.data_ptr(), d_H.data_ptr(), sh)
    t_fixed = timed(step(fixed), args.steps, args.warmup)
    H_fixed = d_H.clone()
    fi = fixed.info()
    log("fixed (6, 0.4) step %.2f ms" % (1e3 * t_fixed))

    # ---- error references at sampled dipoles, configuration 0: the oracle's
    # FP64 direct sum (and the library's, on the GPU, beside it)
    import oracle

    rng = np.random.default_rng(7)
    S = min(args.samples, n)
    idx = np.sort(rng.choice(n, size=S, replace=False)).astype(np.int64)
    threads = host_threads()
    t = time.perf_counter()
    H_o1 = oracle.bruteforce_targets(pos, m[0], idx, nthreads=threads)
    t_o1 = time.perf_counter() - t
    d_idx = torch.from_numpy(idx).to(dev)
    d_Hd = torch.empty((S, 3), dtype=torch.float64, device=dev)
    ccfmm.direct_targets_device(n, d_pos.data_ptr(), d_m[0].data_ptr(), S, d_idx.data_ptr(), d_Hd.data_ptr(), sh)
    torch.cuda.synchronize()
    out["gpu_direct_vs_oracle_direct"] = rel_rms(d_Hd.cpu().numpy(), H_o1)
    Hl0 = H_learned[0][d_idx].cpu().numpy()
    Hf0 = H_fixed[0][d_idx].cpu().numpy()
    out["eps_abs_learned_vs_oracle"] = rel_rms(Hl0, H_o1)
    out["eps_abs_fixed_vs_oracle"] = rel_rms(Hf0, H_o1)
    out["per_dipole_learned_vs_oracle"] = per_dipole_stats(Hl0, H_o1)
    out["per_dipole_fixed_vs_oracle"] = per_dipole_stats(Hf0, H_o1)
    log("vs the oracle's direct sum at %d dipoles: learned %.3e, fixed %.3e; per dipole learned %s" % (
        S, out["eps_abs_learned_vs_oracle"], out["eps_abs_fixed_vs_oracle"], out["per_dipole_learned_vs_oracle"]))

    # ---- the best uniform (p, theta) of the candidate grid on the same film
    if not args.skip_sweep:
        nl = fi["n_leaves"]
        sweep = []
        for p_ in ccfmm.SEL_P:
            for t_ in ccfmm.SEL_THETA:
                dp = torch.full((nl,), p_, dtype=torch.int32, device=dev)
                dt = torch.full((nl,), t_, dtype=torch.float64, device=dev)
                fixed.set_leaf_params(dp.data_ptr(), dt.data_ptr(), sh)
                ms = 1e3 * timed(lambda: fixed.eval_device(nb, d_m.data_ptr(), d_H.data_ptr(), sh), 2, 1)
                err = rel_rms(d_H[0][d_idx].cpu().numpy(), H_o1)
                sweep.append({"p": p_, "theta": t_, "eval_ms": ms, "eps_abs": err})
                log("uniform (%d, %.1f): eval %.2f ms, error %.3e" % (p_, t_, ms, err))
        fixed.set_leaf_params(0, 0, sh)
        ok = [r for r in sweep if r["eps_abs"] <= bound]
        out["uniform_grid"] = sweep
        if ok:
            best = min(ok, key=lambda r: r["eval_ms"])
            out["best_uniform"] = best
            out["speedup_learned_eval_vs_best_uniform"] = best["eval_ms"] / (1e3 * t_learned_eval)
    fixed.destroy()

    # ---- the plain FP64 GPU FMM, fixed (6, 0.4): the same step, with the
    # same forms as the mixed plans (traceless M2L on the FP64 matrix cores,
    # near field beside the expansion passes)
    if not args.skip_fp64:
        p64 = make(ccfmm.PREC_FP64)
        p64.autotune(nb, d_m.data_ptr(), d_H.data_ptr(), sh)
        t64 = timed(step(p64), max(2, args.steps // 5), 1)
        out["fp64_full_step_ms"] = 1e3 * t64
        out["fp64_m2l_variant"] = p64.info()["m2l_variant"]
        out["fp64_passes_ms"] = p64.eval_device_timed(nb, d_m.data_ptr(), d_H.data_ptr(), sh)
        out["speedup_vs_fp64_step"] = t64 / t_learned
        out["eps_prec_fixed_mixed"] = dev_rel_rms(H_fixed, d_H)
        out["eps_learned_vs_fp64_fixed"] = dev_rel_rms(H_learned, d_H)
        out["eps_abs_fp64_vs_oracle"] = rel_rms(d_H[0][d_idx].cpu().numpy(), H_o1)
        log("fp64 step %.2f ms; mixed fixed vs fp64 %.3e, learned vs fp64 %.3e" % (
            1e3 * t64, out["eps_prec_fixed_mixed"], out["eps_learned_vs_fp64_fixed"]))
        p64.destroy()

    # ---- roofline of the dominant pass (the near field)
    out["kernels"], roof = film_roofline(li, pt, n, nb, c["name"])

    # ---- CPU oracle on a bounded sample of the same workload
    cpu = None
    if not args.skip_cpu:
        wpos, wm, wbox = film_window(pos, m[0], box, 128)
        runs = []
        for _ in range(3):
            t = time.perf_counter()
            oracle.fmm(wpos, wm, 6, 0.4, box=wbox, nthreads=threads)
            runs.append(time.perf_counter() - t)
        t_med = float(np.median(runs))
        spos, sm, sbox = film_window(pos, m[0], box, 64)
        t = time.perf_counter()
        oracle.fmm(spos, sm, 6, 0.4, box=sbox, nthreads=1)
        t_one = time.perf_counter() - t
        cpu = {"value": wpos.shape[0] / t_med, "unit": "evals/s", "cores": threads, "kind": "oracle",
               "sample": "FP64 recursive CPU FMM at (6, 0.4), same leaf rule, on a 128 x 128 x 16 window of the "
                         "film (the tile nearest the mean site density, n=%d, holes included), configuration 0, "
                         "median of 3 runs (%s s); the oracle "
                         "evaluates one configuration at a time, so the 8 configurations take 8x as long "
                         "(x8 extrapolated, evals/s unchanged)" % (wpos.shape[0], ", ".join("%.1f" % r for r in runs)),
               "cpu_model": cpu_model(),
               "one_thread": {"value": spos.shape[0] / t_one, "n": int(spos.shape[0]), "seconds": t_one,
                              "sample": "64 x 64 x 16 window (the tile nearest the mean density), "
                                        "configuration 0, 1 thread"},
               "direct_sum_sampled": {"targets": S, "seconds": t_o1, "threads": threads,
                                      "extrapolated_full_n2_s": t_o1 * n / S,
                                      "sample": "FP64 direct sum at %d sampled dipoles over all %d sources, "
                                                "configuration 0; full N^2 extrapolated" % (S, n)}}
        log("cpu oracle: %.3e evals/s on %d threads (%s), 1 thread %.3e evals/s" % (
            cpu["value"], threads, cpu_model(), cpu["one_thread"]["value"]))

    res = {
        "metric": METRIC,
        "value": n * nb / t_learned,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_learned,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": c["name"], "n": n, "batch": nb, "order": 6, "theta": 0.4, "precision": "mixed",
                   "selector": "learned", "err_bound": bound, "levels": li["levels"],
                   "step": "position update (lists and choice kept) + evaluation of the 8 configurations",
                   "selection": "once per geometry at the first evaluation, with its judge (selection_ms)",
                   "sel_margin": selector.FILM_MARGIN, "overlap_near": li["overlap_near"]},
        "tune_eval_ms": {"near_field_beside": li["tune_eval_ms"][0], "one_stream": li["tune_eval_ms"][1]},
        "selection_ms": 1e3 * t_select,
        "selection_status": status,
        "learned": li["learned"],
        "judge_err": li["judge_err"],
        "cost_far": li["sel_cost_far"],
        "choice_hist": hist,
        "learned_eval_ms": 1e3 * t_learned_eval,
        "fixed_full_step_ms": 1e3 * t_fixed,
        "speedup_learned_vs_fixed_step": t_fixed / t_learned,
        "passes_ms": pt,
        "p2p_pairs": {"fixed": fi["p2p_pairs_per_config"], "learned": li["p2p_pairs_per_config"]},
        "m2l_pairs": {"fixed": fi["n_m2l_pairs"], "learned": li["n_m2l_pairs"]},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    res.update(out)
    if args.calib_copy:
        res["calib_copy_bytes"] = calibration_copy(torch, dev)
    print(json.dumps(res), flush=True)


def bench_dynamics(args, torch, ccfmm, inputs):
    """Repeated evaluation as the moments evolve, on the ferrofluid geometry
    (2^20 dipoles, p = 6, theta = 0.5, mixed precision): one plan, its captured
    evaluation replayed after every in-place precession step of the moments,
    and the energy on the GPU every step.  A step = evaluation + energy +
    moment update; value = dipoles / step time.  The same loop on an FP64 plan
    gives the energy the mixed loop is compared with."""
    from paper_0810_0233_amd import dynamics

    dev = torch.device("cuda:0")
    c = inputs.config_ferrofluid()
    pos, box = c["pos"], c["box"]
    n = pos.shape[0]
    st = torch.cuda.current_stream().cuda_stream
    d_pos = torch.from_numpy(pos).to(dev)
    dt = 0.02

    def run(prec, steps):
        prm = ccfmm.params(order=c["order"], theta=c["theta"], leaf_target=0.0, box=box, precision=prec,
                           max_batch=1, m2l_variant=4 if prec == ccfmm.PREC_MIXED else 0)
        pl = ccfmm.Plan.create_device(n, d_pos.data_ptr(), prm, st)
        d_m = torch.from_numpy(np.ascontiguousarray(c["m"][:1])).to(dev)
        d_H = torch.empty_like(d_m)
        d_E = torch.empty(steps, dtype=torch.float64, device=dev)
        if prec == ccfmm.PREC_MIXED:
            pl.autotune(1, d_m.data_ptr(), d_H.data_ptr(), st)
            d_m.copy_(torch.from_numpy(np.ascontiguousarray(c["m"][:1])))
        pl.eval_device(1, d_m.data_ptr(), d_H.data_ptr(), st)  # capture
        d_m.copy_(torch.from_numpy(np.ascontiguousarray(c["m"][:1])))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            pl.eval_device(1, d_m.data_ptr(), d_H.data_ptr(), st)
            pl.energy_device(1, d_m.data_ptr(), d_H.data_ptr(), d_E[k:k + 1].data_ptr(), st)
            dynamics.precession_step_(d_m, d_H, dt)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        pl.destroy()
        return t, d_E.cpu().numpy()

    steps = max(args.steps, 5)
    run(ccfmm.PREC_MIXED, 2)  # warm-up (first-use allocations)
    t_mx, E_mx = run(ccfmm.PREC_MIXED, steps)
    out = {}
    if not args.skip_fp64:
        t_64, E_64 = run(ccfmm.PREC_FP64, steps)
        out = {"fp64_step_ms": 1e3 * t_64, "speedup_vs_fp64_step": t_64 / t_mx,
               "energy_fp64": [float(x) for x in E_64],
               "energy_rel_diff_max": float(np.max(np.abs(E_mx - E_64) / np.abs(E_64)))}
    res = {
        "metric": METRIC, "value": n / t_mx, "unit": "evals/s", "n_gpus": 1, "steps": steps, "warmup": 2,
        "ms_per_step": 1e3 * t_mx, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ferrofluid_rsa_1048576_precession", "n": n, "batch": 1, "order": c["order"],
                   "theta": c["theta"], "precision": "mixed", "dt": dt,
                   "step": "captured evaluation + energy + moment update (plan reused)"},
        "energy_mixed": [float(x) for x in E_mx],
        "roofline": None, "cpu_baseline": None,
    }
    res.update(out)
    print(json.dumps(res), flush=True)


def bench_leafsweep(args, torch, ccfmm, inputs):
    """GPU re-study of the paper's leaf-size choice (Table I, Eq. (so)): trees two
    levels either side of the paper's s_o(p) for Table II's (p, alpha) pairs on
    the paper's 32^3 lattice and on a 128^3 lattice, and for the ferrofluid at
    (6, 0.5); mixed precision.  One JSON line with every swept point; value =
    ferrofluid evals/s (full step) at the fastest tree of the sweep."""
    from paper_0810_0233_amd import study

    pairs = [(2, 0.36), (3, 0.54), (4, 0.64), (5, 0.71), (6, 0.76)]
    res = {"metric": METRIC, "unit": "evals/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic", "steps": 7, "warmup": 1}
    studies = {}
    for side in (32, 128):
        pos, box = inputs.lattice(side, side, side)
        m = inputs.random_moments(pos.shape[0], 6000 + side)
        log("leaf sweep: %d^3 lattice" % side)
        recs = study.leaf_sweep(pos, box, m, pairs, progress=log)
        for r in recs:
            log("  p=%d theta=%.2f paper s=%.2f (L=%d): best L=%d, s_opt %.1f, %.2fx vs paper" % (
                r["order"], r["theta"], r["paper_s"], r["paper_levels"], r["best_levels"], r["s_opt"],
                r["speedup_best_vs_paper"]))
        studies["lattice_%d" % side] = {"records": recs, "c_fit": study.fit_c(recs)}
    c = inputs.config_ferrofluid()
    log("leaf sweep: ferrofluid")
    recs = study.leaf_sweep(c["pos"], c["box"], c["m"][0], [(6, 0.5)], progress=log)
    studies["ferrofluid_rsa_1048576"] = {"records": recs}
    best = min(recs[0]["points"], key=lambda r: r["step_ms"])
    n = c["pos"].shape[0]
    res.update({"value": n / (best["step_ms"] * 1e-3), "ms_per_step": best["step_ms"],
                "config": {"workload": "leafsweep", "ferrofluid_best_levels": best["levels"],
                           "ferrofluid_paper_levels": recs[0]["paper_levels"]},
                "study": studies, "roofline": None, "cpu_baseline": None})
    print(json.dumps(res), flush=True)


def bench_leaffit(args, torch, ccfmm, inputs):
    """The paper's fit of s_o = c p^2 over many system sizes (Fig. 2), on the
    GPU: 30 cubic lattices of side 16 ... 132, Table II's (p, alpha) pairs for
    p = 4, 5, 6, one level either side of the paper's tree; mixed precision.
    One JSON line; value = evals/s of the 132^3 lattice at p = 6 on its
    fastest tree (full step)."""
    from paper_0810_0233_amd import study

    pairs = [(4, 0.64), (5, 0.71), (6, 0.76)]
    sides = list(range(16, 133, 4))
    fit = study.lattice_size_fit(sides, pairs, progress=log)
    log("c in s_o = c p^2 over %d sizes: %.3f (paper 0.74); mean s_opt %s" % (
        len(sides), fit["c_fit"], {p: round(v, 1) for p, v in fit["s_opt_mean"].items()}))
    last = fit["sides"][-1]
    r6 = next(r for r in last["records"] if r["order"] == 6)
    best = min(r6["points"], key=lambda q: q["step_ms"])
    res = {"metric": METRIC, "unit": "evals/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic", "steps": 5, "warmup": 1,
           "value": last["n"] / (best["step_ms"] * 1e-3), "ms_per_step": best["step_ms"],
           "config": {"workload": "leaffit", "sides": [sides[0], sides[-1], len(sides)]},
           "study": fit, "roofline": None, "cpu_baseline": None}
    print(json.dumps(res), flush=True)


def bench_params(args, torch, ccfmm, inputs):
    """The paper's choice of (p, alpha) per error level (Table II and Fig. 3) on
    the GPU: for e = 0.1 ... 0.001 and p = 2 ... 8, alpha from
    [alpha/(2-alpha)]^p = e, the paper's tree, one timed full step and the
    measured error, on the 32^3 lattice (the paper's size) and a 128^3
    lattice.  One JSON line; value = evals/s of the 128^3 lattice at e = 0.05
    with its fastest (p, alpha)."""
    from paper_0810_0233_amd import study

    errors = [0.1, 0.05, 0.02, 0.01, 0.005, 0.002, 0.001]
    out = {}
    for side in (32, 128):
        pos, box = inputs.lattice(side, side, side)
        m = inputs.random_moments(pos.shape[0], 7000 + side)
        log("parameter sweep: %d^3 lattice" % side)
        out["lattice_%d" % side] = study.param_sweep(pos, box, m, errors, list(range(2, 9)),
                                                     samples=0 if side <= 32 else 4096, progress=log)
        for e, b in out["lattice_%d" % side]["best"].items():
            log("  e=%s: fastest p=%d alpha=%.3f, %.3f ms, eps_abs %.2e" % (e, b["order"], b["alpha"], b["step_ms"],
                                                                              b["eps_abs"]))
    b = out["lattice_128"]["best"]["0.05"]
    n = 128 ** 3
    res = {"metric": METRIC, "unit": "evals/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic", "steps": 5, "warmup": 1,
           "value": n / (b["step_ms"] * 1e-3), "ms_per_step": b["step_ms"],
           "config": {"workload": "params", "order": b["order"], "alpha": b["alpha"], "e": 0.05},
           "study": out, "roofline": None, "cpu_baseline": None}
    print(json.dumps(res), flush=True)


def bench_truncation(args, torch, ccfmm, inputs):
    """Both readings of the paper's truncation (Sec. 3) on the GPU path: each
    index to order p (the default) against total degree |n| + |q| <= p.  On the
    paper's 32^3 lattice (FP64) at Table II's (p, alpha) pairs, at (6, 0.48)
    and at theta = 0.5: field error against the direct sum at every dipole,
    energy error, evaluation time, next to the paper's estimate
    [theta/(2-theta)]^p; and the ferrofluid at (6, 0.5) in mixed precision.
    One JSON line; value = ferrofluid evals/s of the evaluation with the
    default truncation."""
    from paper_0810_0233_amd import study

    res = {"metric": METRIC, "unit": "evals/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic", "steps": 5, "warmup": 1}
    pos, box = inputs.lattice(32, 32, 32)
    m = inputs.random_moments(pos.shape[0], 6032)
    settings = [(2, 0.36), (3, 0.54), (4, 0.64), (5, 0.71), (6, 0.76), (7, 0.79), (8, 0.81), (6, 0.48)]
    settings += [(p, 0.5) for p in range(2, 9)]
    log("truncation study: 32^3 lattice, FP64")
    lat = study.truncation_study(pos, box, m, settings, progress=log)
    c = inputs.config_ferrofluid()
    log("truncation study: ferrofluid, mixed")
    ff = study.truncation_study(c["pos"], c["box"], c["m"][0], [(6, 0.5)], precision=ccfmm.PREC_MIXED,
                                samples=args.samples, progress=log)
    n = c["pos"].shape[0]
    t0 = next(r for r in ff if r["truncation"] == 0)
    res.update({"value": n / (t0["eval_ms"] * 1e-3), "ms_per_step": t0["eval_ms"],
                "config": {"workload": "truncation", "step": "eval"},
                "study": {"lattice_32": lat, "ferrofluid_rsa_1048576": ff}, "roofline": None, "cpu_baseline": None})
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="film")
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--order", type=int, default=0)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--samples", type=int, default=0, help="sampled dipoles for the error against the direct sum "
                    "(default 4096; 1024 on the film)")
    ap.add_argument("--skip-sweep", action="store_true", help="film: skip the uniform (p, theta) grid")
    ap.add_argument("--roofline-only", action="store_true",
                    help="film: the learned plan alone, untuned, then the roofline (for counter runs)")
    ap.add_argument("--traffic-record", nargs=3, metavar=("WORKLOAD", "FETCH_DIR", "WRITE_DIR"),
                    help="write the counter record of WORKLOAD from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--traffic-summary", default="", help="with --traffic-record: the summary file it cites")
    ap.add_argument("--calib-copy", action="store_true",
                    help="end with one plain 256 MiB device copy (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.traffic_record:
        fs, ws, rows = write_traffic_record(args.traffic_record[0], args.traffic_record[1], args.traffic_record[2],
                                            args.traffic_summary)
        print("calibration scales: FETCH_SIZE x%.4f, WRITE_SIZE x%.4f" % (fs, ws))
        print("| kernel | dispatches | FETCH KiB | WRITE KiB | scaled bytes/dispatch |")
        print("|---|---:|---:|---:|---:|")
        print("\n".join(rows))
        return
    if not args.samples:
        args.samples = 1024 if args.workload == "film" else 4096
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (no multi-GPU path); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_0810_0233_amd import ccfmm, inputs

    if args.workload == "film":
        bench_film(args, torch, ccfmm, inputs)
        return
    if args.workload == "clusters":
        bench_learned(args, torch, ccfmm, inputs)
        return
    if args.workload == "dynamics":
        bench_dynamics(args, torch, ccfmm, inputs)
        return
    if args.workload == "leafsweep":
        bench_leafsweep(args, torch, ccfmm, inputs)
        return
    if args.workload == "truncation":
        bench_truncation(args, torch, ccfmm, inputs)
        return
    if args.workload == "leaffit":
        bench_leaffit(args, torch, ccfmm, inputs)
        return
    if args.workload == "params":
        bench_params(args, torch, ccfmm, inputs)
        return
    dev = torch.device("cuda:0")
    t0 = time.time()
    W = workload(args, inputs)
    pos, box, m = W["pos"], W["box"], W["m"]
    nb, n = m.shape[0], m.shape[1]
    order, theta = W["order"], W["theta"]
    log("inputs: %s n=%d batch=%d (%.1f s)" % (W["name"], n, nb, time.time() - t0))
    d_pos = torch.from_numpy(pos).to(dev)
    # the moved copy for time steps: displaced by N(0, 0.01^2) per coordinate, kept inside the root box
    lo_b, hi_b = np.asarray(box[0], float), np.asarray(box[1], float)
    pos_b = np.clip(pos + 0.01 * np.random.default_rng(17).normal(size=pos.shape), lo_b + 1e-9, hi_b - 1e-9)
    d_pos_b = torch.from_numpy(pos_b).to(dev)
    d_m = torch.from_numpy(np.ascontiguousarray(m)).to(dev)
    d_H = torch.empty_like(d_m)
    d_H64 = torch.empty_like(d_m)
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream

    def make(prec, **kw):
        prm = ccfmm.params(order=order, theta=theta, leaf_target=0.0, box=box, precision=prec, max_batch=nb, **kw)
        return ccfmm.Plan.create_device(n, d_pos.data_ptr(), prm, sh)

    def time_steps(plan, out, rebuild, steps, warmup):
        """Mean step time; with rebuild, every step first moves the dipoles
        (alternating the two position sets); the plan ends on the original."""
        sets = (d_pos_b, d_pos)
        for k in range(warmup):
            if rebuild:
                plan.update_positions_device(sets[k % 2].data_ptr(), sh)
            plan.eval_device(nb, d_m.data_ptr(), out.data_ptr(), sh)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k in range(steps):
            if rebuild:
                plan.update_positions_device(sets[k % 2].data_ptr(), sh)
            plan.eval_device(nb, d_m.data_ptr(), out.data_ptr(), sh)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t) / steps
        if rebuild:
            plan.update_positions_device(d_pos.data_ptr(), sh)
            torch.cuda.synchronize()
        return t

    # ---- mixed precision: the headline path
    plan = make(ccfmm.PREC_MIXED)
    tune = plan.autotune(nb, d_m.data_ptr(), d_H.data_ptr(), sh)
    info = plan.info()
    log("evaluation form: %s (tuned: near field beside %.3f ms, one stream %.3f ms)" % (
        "near field beside the expansion passes" if info["overlap_near"] else "one stream", *info["tune_eval_ms"]))
    log("m2l autotune: %s -> variant %d class_bits %d" % (
        json.dumps([(t["variant"], t["class_bits"], round(t["m2l_ms"], 3)) for t in tune]),
        info["m2l_variant"], info["m2l_class_bits"]))
    log("plan: L=%d leaves=%d m2l_pairs=%d p2p_pairs=%d tiles=%d steps=%d" % (
        info["levels"], info["n_leaves"], info["n_m2l_pairs"], info["n_p2p_pairs"], info["n_m2l_tiles"],
        info["n_m2l_steps"]))
    kept0 = plan.info()["n_rebuilds_kept"]
    t_step = time_steps(plan, d_H, True, args.steps, args.warmup)
    kept = plan.info()["n_rebuilds_kept"] - kept0
    log("mixed full step: %.3f ms (%d of %d rebuilds kept the lists)" % (1e3 * t_step, kept,
                                                                          args.steps + args.warmup + 1))
    planr = make(ccfmm.PREC_MIXED, keep_lists=0, m2l_variant=info["m2l_variant"],
                 m2l_class_bits=info["m2l_class_bits"])
    t_step_full = time_steps(planr, d_H, True, args.steps, args.warmup)
    planr.destroy()
    log("mixed step, lists and tiles always rebuilt: %.3f ms" % (1e3 * t_step_full))
    t_eval = time_steps(plan, d_H, False, args.steps, args.warmup)
    log("mixed eval only: %.3f ms" % (1e3 * t_eval))
    torch.cuda.synchronize()
    H_mixed = d_H.cpu().numpy().copy()
    # per-pass times: the timed evaluation runs every kernel alone on one
    # stream (same tiles and kernel variant), the near field and the smooth part fused
    passes = [plan.eval_device_timed(nb, d_m.data_ptr(), d_H.data_ptr(), sh) for _ in range(3)]
    pt = {k: float(np.median([p[k] for p in passes])) for k in passes[0]}
    log("mixed passes, one stream (ms): %s" % json.dumps({k: round(v, 4) for k, v in pt.items()}))

    out = {}
    # ---- plain FP64 GPU FMM
    if not args.skip_fp64:
        # the FP64 plan with the same forms as the mixed one (traceless M2L on
        # the FP64 matrix cores, near field beside the expansion passes)
        plan64 = make(ccfmm.PREC_FP64)
        plan64.autotune(nb, d_m.data_ptr(), d_H64.data_ptr(), sh)
        t_step64 = time_steps(plan64, d_H64, True, max(2, args.steps // 2), 1)
        t_eval64 = time_steps(plan64, d_H64, False, max(2, args.steps // 2), 1)
        passes64 = plan64.eval_device_timed(nb, d_m.data_ptr(), d_H64.data_ptr(), sh)
        torch.cuda.synchronize()
        H64 = d_H64.cpu().numpy().copy()
        out["fp64_full_step_ms"] = 1e3 * t_step64
        out["fp64_eval_ms"] = 1e3 * t_eval64
        out["fp64_passes_ms"] = passes64
        out["fp64_m2l_variant"] = plan64.info()["m2l_variant"]
        out["speedup_vs_fp64_step"] = t_step64 / t_step
        out["speedup_vs_fp64_eval"] = t_eval64 / t_eval
        out["eps_prec"] = rel_rms(H_mixed, H64)
        log("fp64 step %.3f ms eval %.3f ms; eps_prec %.3e" % (1e3 * t_step64, 1e3 * t_eval64, out["eps_prec"]))
        plan64.destroy()
        # beside it, the plain form: one stream, full (dense) M2L operator
        plan64b = make(ccfmm.PREC_FP64, overlap_near=0, m2l_traceless=0)
        t_step64b = time_steps(plan64b, d_H64, True, max(2, args.steps // 2), 1)
        out["fp64_one_stream_full_operator_step_ms"] = 1e3 * t_step64b
        out["speedup_vs_fp64_one_stream_full_operator_step"] = t_step64b / t_step
        log("fp64 one stream, full operator: step %.3f ms" % (1e3 * t_step64b))
        plan64b.destroy()
    # ---- error against the direct sum at sampled dipoles (FP64 on the GPU), configuration 0
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(n, size=min(args.samples, n), replace=False)).astype(np.int64)
    d_idx = torch.from_numpy(idx).to(dev)
    d_Hd = torch.empty((idx.size, 3), dtype=torch.float64, device=dev)
    ccfmm.direct_targets_device(n, d_pos.data_ptr(), d_m[0].data_ptr(), idx.size, d_idx.data_ptr(),
                                d_Hd.data_ptr(), sh)
    torch.cuda.synchronize()
    H_direct = d_Hd.cpu().numpy()
    out["eps_abs_mixed"] = rel_rms(H_mixed[0][idx], H_direct)
    if not args.skip_fp64:
        out["eps_abs_fp64"] = rel_rms(H64[0][idx], H_direct)
    log("eps_abs mixed %.3e" % out["eps_abs_mixed"])

    # ---- per-pass algorithmic work and the roofline of the dominant kernel
    # (times: HIP events recorded by the library on the launch stream)
    kern = pass_work(info, n, nb, order)
    if nb < 32:
        pt["l2p"] = 0.0  # fused into the near-field kernel (the timer brackets nothing)
    for k, v in kern.items():
        v["ms"] = pt[k]
        if pt[k] <= 0.0:  # a pass fused into another
            continue
        sec = pt[k] * 1e-3
        v["gb_s"] = v["bytes"] / sec / 1e9
        v["hbm_frac"] = v["bytes"] / sec / PEAK_HBM
        if v["flops"]:
            v["tflop_s"] = v["flops"] / sec / 1e12
            v["flop_frac"] = v["flops"] / sec / v["peak"]
    dom = "m2l" if pt["m2l"] >= pt["p2p"] else "p2p"
    d = kern[dom]
    ach = d["flops"] / (pt[dom] * 1e-3)
    roof = {"kernel": d["kernel"], "bound": d["bound"], "achieved": ach / 1e12, "peak": d["peak"] / 1e12,
            "unit": "TFLOP/s", "frac": ach / d["peak"],
            "traffic": counted_traffic(d["kernel"], W["name"])}
    out["kernels"] = {k: {q: v[q] for q in v if q != "peak"} for k, v in kern.items()}

    # ---- CPU oracle on the same workload (one configuration)
    cpu = None
    if not args.skip_cpu:
        import oracle

        # the whole workload, configuration 0 (about 10-15 s of CPU work at p = 6)
        ns = n
        threads = min(os.cpu_count() or 1, 16)
        t = time.perf_counter()
        H_ref = oracle.fmm(pos, m[0], order, theta, box=box, nthreads=threads)
        dt = time.perf_counter() - t
        cpu = {"value": ns / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
               "sample": "FP64 recursive CPU FMM (same p, theta, s rule and root box) on the whole workload, "
                         "configuration 0 only (n=%d), %.1f s" % (ns, dt), "cpu_model": cpu_model()}
        log("cpu oracle: %.3e evals/s on %d threads" % (ns / dt, threads))
        # the timed oracle field is also the reference of the mixed field at the
        # same (p, theta, s): every dipole, configuration 0
        out["eps_vs_oracle_fmm"] = rel_rms(H_mixed[0], H_ref)
        out["per_dipole_vs_oracle_fmm"] = per_dipole_stats(H_mixed[0], H_ref)
        log("mixed vs oracle FMM %.3e, per dipole %s" % (out["eps_vs_oracle_fmm"], out["per_dipole_vs_oracle_fmm"]))

    res = {
        "metric": METRIC,
        "value": n * nb / t_step,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": W["name"], "n": n, "batch": nb, "order": order, "theta": theta,
                   "leaf_target": info["s_used"], "levels": info["levels"], "precision": "mixed",
                   "step": "rebuild for moved dipoles (tree; lists and tiles unless the occupied cells are the "
                           "same) + eval",
                   "m2l_variant": info["m2l_variant"], "m2l_class_bits": info["m2l_class_bits"],
                   "overlap_near": info["overlap_near"]},
        "tune_eval_ms": {"near_field_beside": info["tune_eval_ms"][0], "one_stream": info["tune_eval_ms"][1]},
        "rebuilds_keeping_lists": kept,
        "step_lists_always_rebuilt_ms": 1e3 * t_step_full,
        "eval_only_evals_per_s": n * nb / t_eval,
        "eval_ms": 1e3 * t_eval,
        "passes_ms": pt,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    res.update(out)
    if args.calib_copy:
        res["calib_copy_bytes"] = calibration_copy(torch, dev)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
