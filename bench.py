"""Benchmark: band-limited FMM matrix-vector product throughput (points/s) on one MI355X,
and GMRES time to a true residual of 1e-8 with and without the learned preconditioner.

Workload (default): 3-D, N = 2^20 points, half uniform in [0,1]^3 and half from 32
Gaussian blobs (standard deviation 0.01), stored as float32; lambda ~ N(0,1).
* Headline: the Gaussian kernel exp(-r^2/(2 * 0.03^2)) in FP64 with tolerance 1e-6 (relative
  2-norm error against the exact sum); the FP32 path (tol 1e-4) beside it.  A step is one full
  product (permute, near field, aggregation, upward sum, coarse and leaf translation,
  disaggregation) with inputs resident in HBM.
* The same points with the multiquadric sqrt(r^2 + 0.02^2) (banded far field), FP64 at 1e-6
  and FP32 at 1e-4, each checked on 2048 sampled targets against the oracle's direct sum.
* GMRES(50) on the learned-preconditioner workload's recipe (3-D mixed points, multiquadric
  c = 0.02, f = 16 Gaussian bumps of width 0.1) at 2^18 points, FP64 product at tol 1e-8, to a
  true residual of 1e-8 or 200 iterations: plain, block-Jacobi and learned (network trained
  here on pairs from solves of four 10^4-point problems of the family).  The full 2^21-point
  solve is ``--workload solve``.

Prints one JSON line.  ``--gpus`` above 1 is refused: the bench measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VEC_TFLOPS = 78.6
FP64_MFMA_TFLOPS = 78.6   # dense FP64 matrix-core peak (equal to the vector rate on this chip)
FP32_VEC_TFLOPS = 157.3


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def phase_model(info, dtype_bytes, n):
    """Algorithmic work of one launch of each phase: flops for the arithmetic phases, compulsory HBM
    bytes for the memory-bound ones."""
    P = info["half_nodes"]
    d = info["d"]
    nl = info["nleaves"]
    nc = info["ncells"]
    cb = 2 * dtype_bytes
    pairs = info["near_pairs"]
    return {
        # (kind, amount): flops for phases bound by the vector ALUs ("alu") or the matrix cores
        # ("mfma"), bytes for memory-bound ones ("hbm"); the FP64 aggregation runs on the vector
        # ALUs and the disaggregation on the matrix cores
        "p2p": ("alu", pairs * gauss_pair_flops(d, dtype_bytes)),
        "p2m": ("alu", 8.0 * n * P),
        "l2p": ("mfma", 8.0 * n * P),
        "m2m": ("hbm", (nl + nc) * P * cb),
        "m2l_coarse": ("hbm", 2.0 * d * nc * P * cb),
        # compulsory bytes: every leaf expansion read once, every coarse local expansion
        # read once, every leaf local expansion written once (the near-list re-reads are
        # meant to hit in L2 and are not counted)
        "m2l_leaf": ("hbm", (2.0 * nl + nc) * P * cb),
        "permute": ("hbm", n * (2 * dtype_bytes + 4)),
    }


def gauss_pair_flops(d, dtype_bytes):
    """Floating-point operations the near-field kernel executes per Gaussian pair (a fused
    multiply-add counts 2): d differences and d multiply-adds for r^2, the scaling of r^2 and
    the multiply-add into the sum (3 d + 3), plus the exponential as built.  FP64: the table
    method of the kernel (round to nearest, the reduced argument, a degree-4 polynomial in 4
    multiply-adds, the product with the table entry and the exponent scaling: 12).  FP32: the
    hardware exp2 instruction, counted as 1."""
    return 3 * d + 3 + (12 if dtype_bytes == 8 else 1)


def residual_pair_flops(d, dtype_bytes=8, in_q=True):
    """Per near pair of a banded plan (multiquadric kernels), as the kernel executes it (a fused
    multiply-add counts 2): the distance and the accumulation (3 d + 3); the table index and
    local variable (3); the degree-5 polynomial (10).  A table in b = sqrt(r^2 + c^2) (plans
    whose fit in q = r^2 + c^2 misses its bound) adds q, its reciprocal square root and
    b = q / sqrt q (3, and in FP64 one Newton step on the root: 5 more); the inverse
    multiquadric's product with 1 / b there is not counted."""
    return 3 * d + 3 + (0 if in_q else (8 if dtype_bytes == 8 else 3)) + 3 + 10


def measured_traffic(phase):
    """HBM bytes of a phase per product (its launches summed: one for every phase but the three
    axis passes of the coarse translation) from the committed counter table, if that table was
    taken on the current kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_3d_mixed_gauss_n1m.json")
    src = os.path.join(ROOT, "paper_1606_07652_amd", "csrc", "fmm.hip")
    if not os.path.exists(path):
        return None
    tab = json.load(open(path))
    if tab.get("fmm_hip_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return tab.get("bytes_per_product", {}).get(phase)


# kernel name prefix (as the profiler prints it, template arguments stripped) -> phase
TRAFFIC_PHASES = {"k_gather": "permute", "k_phase_dl": "p2m_phase", "k_p2m": "p2m", "k_p2p": "p2p", "k_p2p_queue": "p2p",
                  "k_m2m": "m2m", "k_m2l_axis": "m2l_coarse", "k_m2l_leaf": "m2l_leaf", "k_l2p": "l2p"}


def write_traffic_table(fetch_dir, write_dir, out_path, workload):
    """Turn two rocprofv3 counter runs of the FP64 default workload (``--pmc FETCH_SIZE`` and
    ``--pmc WRITE_SIZE``, each with ``--copy-check``) into the HBM byte table that the bench
    reads: per phase, bytes per product.  Counter values are KiB per dispatch; each counter is
    scaled by what it reads for the 1 GiB copy of ``--copy-check`` (the largest
    ``__amd_rocclr_copyBuffer`` dispatch), and the number of products is the number of
    ``k_l2p<double`` dispatches (one per product)."""
    import csv
    import glob
    import hashlib
    import re

    def load(d, counter):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise SystemExit(f"no counter_collection.csv under {d}")
        per = {}
        for fn in files:
            for row in csv.DictReader(open(fn)):
                if row["Counter_Name"] != counter:
                    continue
                key = (fn, row["Dispatch_Id"])
                name = row["Kernel_Name"]
                per.setdefault(key, [name, 0.0])[1] += float(row["Counter_Value"])
        return list(per.values())

    def phase_of(name):
        m = re.search(r"\b(k_[A-Za-z0-9_]+)", name)
        return TRAFFIC_PHASES.get(m.group(1)) if m else None

    tab = {}
    for key, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = load(d, counter)
        copies = [v for n, v in rows if n.startswith("__amd_rocclr_copyBuffer")]
        if not copies:
            raise SystemExit(f"{counter}: no copy dispatch (run with --copy-check)")
        factor = (1 << 20) / max(copies)            # 1 GiB in KiB over what the counter read
        products = sum(1 for n, _ in rows if "k_l2p<double" in n)
        sums = {}
        for n, v in rows:
            if "<float" in n:
                continue
            ph = phase_of(n)
            if ph is not None:
                sums[ph] = sums.get(ph, 0.0) + v
        tab[key] = {"factor": factor, "products": products,
                    "bytes": {ph: v * 1024.0 * factor / max(products, 1) for ph, v in sums.items()}}
    src = os.path.join(ROOT, "paper_1606_07652_amd", "csrc", "fmm.hip")
    phases = sorted(set(tab["fetch"]["bytes"]) | set(tab["write"]["bytes"]))
    out = {"workload": workload,
           "fmm_hip_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest(),
           "fetch_factor": tab["fetch"]["factor"], "write_factor": tab["write"]["factor"],
           "products": tab["fetch"]["products"],
           "fetch_bytes_per_product": {p: tab["fetch"]["bytes"].get(p, 0.0) for p in phases},
           "write_bytes_per_product": {p: tab["write"]["bytes"].get(p, 0.0) for p in phases},
           "bytes_per_product": {p: tab["fetch"]["bytes"].get(p, 0.0) + tab["write"]["bytes"].get(p, 0.0)
                                for p in phases}}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out, indent=1))


def roofline_of(kind, amount, ms, fp_peak, mfma_peak=FP64_MFMA_TFLOPS):
    secs = ms * 1e-3
    if kind == "hbm":
        r = {"bound": "hbm", "achieved": amount / secs / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    elif kind == "mfma":
        r = {"bound": "mfma", "achieved": amount / secs / 1e12, "peak": mfma_peak, "unit": "TFLOP/s"}
    else:
        r = {"bound": "alu", "achieved": amount / secs / 1e12, "peak": fp_peak, "unit": "TFLOP/s"}
    r["frac"] = r["achieved"] / r["peak"]
    return r


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Measured device-to-device copy rate (GB/s counting the bytes read and written), the
    memory bound of the whole-product roofline."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def product_roofline(model, t_meas_ms, fp_peak, mfma_peak, bw_gbs):
    """Whole-product roofline: t_roof = sum over the phases of their algorithmic work at the
    bound that limits them (flops at the vector or matrix peak, compulsory bytes at the measured
    copy rate), against the measured time per product."""
    per = {}
    for k, (kind, amount) in model.items():
        if kind == "hbm":
            per[k] = amount / (bw_gbs * 1e9) * 1e3
        elif kind == "mfma":
            per[k] = amount / (mfma_peak * 1e12) * 1e3
        else:
            per[k] = amount / (fp_peak * 1e12) * 1e3
    t_roof = sum(per.values())
    return {"t_roof_ms": t_roof, "t_meas_ms": t_meas_ms, "frac": t_roof / t_meas_ms, "copy_GBps": bw_gbs,
            "phase_t_roof_ms": {k: round(v, 4) for k, v in per.items()}}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_path(torch, FmmPlan, w, dtype, tol, steps, warmup, n_max, m2l_schedule=0):
    dev = torch.device("cuda:0")
    x = torch.as_tensor(w.points, dtype=dtype, device=dev)
    lam = torch.as_tensor(w.lam, dtype=dtype, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = FmmPlan(x, kernel=w.kernel, shape=w.shape, tol=tol, n_max=n_max, m2l_schedule=m2l_schedule)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info()
    log(f"[bench] plan {dtype} tol={tol}: {plan_ms:.1f} ms, nodes={info['nodes']} leaves={info['nleaves']} "
        f"lc={info['coarse_level']} r={info['coarse_radius']} near_pairs={info['near_pairs']}")
    u = torch.empty_like(lam)
    for _ in range(warmup):
        plan.matvec(lam, u)
    torch.cuda.synchronize()
    # the timed steps record HIP events around every phase on the plan's stream (one wait
    # per step for the events, inside the timed region)
    plan.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.matvec(lam, u)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ph = plan.phase_times()
    plan.set_profiling(False)
    log(f"[bench] timed {steps} steps: {total * 1e3 / steps:.3f} ms/step")
    calls = max(ph.pop("calls"), 1)
    phase_ms = {k: v / calls for k, v in ph.items()}
    out = u.double().cpu().numpy()
    plan.close()
    del x, lam, u
    torch.cuda.empty_cache()
    return {"ms_per_step": total * 1e3 / steps, "plan_ms": plan_ms, "info": info, "phase_ms": phase_ms,
            "u": out}


def run_batched(args):
    """512 independent 3-D problems (N log-uniform in [2e3, 2e5], Gaussian s log-uniform in
    [0.01, 0.1], float32, tol 1e-4); all products of one step in one graph launch."""
    import torch

    from paper_1606_07652_amd import BatchPlan
    from workloads import c3

    probs = c3(args.nprob)
    off = np.concatenate([[0], np.cumsum([p.points.shape[0] for p in probs])]).astype(np.int64)
    X = torch.as_tensor(np.concatenate([p.points for p in probs]), device="cuda:0")
    lam = torch.as_tensor(np.concatenate([p.lam for p in probs]), device="cuda:0")
    shapes = np.array([p.shape for p in probs])
    n = int(off[-1])
    log(f"[bench] batched workload: {len(probs)} problems, total n={n}")
    t0 = time.perf_counter()
    b = BatchPlan(X, off, shapes, kernel="gaussian", tol=1e-4, autotune=not args.no_autotune)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    inf = b.info()
    log(f"[bench] batch plan {plan_s:.1f} s: groups={inf['ngroups']} far={inf['nfar']} leaves={inf['total_leaves']}")
    u = torch.empty_like(lam)
    for _ in range(args.warmup):
        b.matvec(lam, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.matvec(lam, u)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ms = total * 1e3 / args.steps
    b.set_graph(False)
    for _ in range(args.warmup):
        b.matvec(lam, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.matvec(lam, u)
    torch.cuda.synchronize()
    ms_nograph = (time.perf_counter() - t0) * 1e3 / args.steps
    b.set_graph(True)
    solve = None
    if args.batched_solve:
        # GMRES(50) on every problem at once, f = 8 Fourier modes per problem, capped
        F = torch.as_tensor(np.concatenate([p.f for p in probs]).astype(np.float32), device="cuda:0")
        solve = {}
        for pk in ("none", "block_jacobi"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, infos = b.solve(F, rtol=1e-6, restart=50, max_iters=args.solve_iters, precond=pk)
            secs = time.perf_counter() - t0
            res = np.array([i["true_res"] for i in infos])
            solve[pk] = {"rtol": 1e-6, "max_iters": args.solve_iters, "seconds": secs,
                         "converged": int(sum(i["converged"] for i in infos)), "nprob": len(infos),
                         "median_true_res": float(np.median(res)), "max_true_res": float(res.max()),
                         "max_iters_used": int(max(i["iters"] for i in infos))}
            log(f"[bench] batched solve ({pk}): {solve[pk]['converged']}/{len(infos)} converged, median "
                f"residual {solve[pk]['median_true_res']:.2e}, {secs:.1f} s")
    result = {"metric": "batched RBF-FMM matvec points/s @ rel-L2<=1e-4", "value": n / (ms * 1e-3),
              "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
              "config": {"workload": "batched_512x3d_uniform_gaussian_logN_logs", "nprob": len(probs), "n": n,
                         "tol": 1e-4, "autotune": not args.no_autotune, "groups": inf["ngroups"],
                         "far_problems": inf["nfar"]},
              "plan_seconds": plan_s, "ms_per_step_without_graph": ms_nograph}
    if solve is not None:
        result["batched_solve"] = solve
    if not args.no_cpu:
        from oracle import direct
        u_h = u.double().cpu().numpy()
        rng = np.random.default_rng(7)
        errs = []
        t_full = 0.0   # estimated oracle time for the sampled problems in full
        sample = rng.choice(len(probs), 16, replace=False)
        for q in sample:
            p = probs[q]
            idx = np.sort(rng.choice(p.points.shape[0], min(256, p.points.shape[0]), replace=False))
            xs = p.points.astype(np.float64)
            t0 = time.perf_counter()
            ref = direct.direct_sum(xs, p.lam.astype(np.float64), "gaussian", p.shape, targets=xs[idx])
            t_full += (time.perf_counter() - t0) * p.points.shape[0] / idx.size
            errs.append(direct.rel_l2(u_h[off[q]:off[q + 1]][idx], ref))
        n_sample = sum(probs[q].points.shape[0] for q in sample)
        result["rel_l2_sampled_max"] = max(errs)
        result["cpu_baseline"] = {"value": n_sample / t_full if t_full > 0 else None, "unit": "points/s",
                                  "cores": direct.threads(), "kind": "oracle",
                                  "sample": "16 problems x 256 targets each against all of that problem's sources"}
    print(json.dumps(result), flush=True)


def solve_family(torch, FmmPlan, pc, kernel, shape, n, rtol, cap, n_train=10000, harvest_iters=500):
    """GMRES(50) on the learned-preconditioner recipe (3-D mixed points, f = 16 Gaussian bumps of
    width 0.1) at n points: plain, block-Jacobi and learned, each to the true residual rtol or
    `cap` iterations.  The network is trained here on pairs harvested from solves of four
    n_train-point problems of the same family (seeds 100-103)."""
    from workloads import bumps_rhs, c5, mixed_points

    def dev(a):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")

    t0 = time.perf_counter()
    rows = [[], [], []]
    for sd in (100, 101, 102, 103):
        x = mixed_points(n_train, 3, sd)
        plan = FmmPlan(dev(x), kernel=kernel, shape=shape, tol=1e-8)
        for k, a in enumerate(pc.harvest(plan, dev(bumps_rhs(x, sd)), rtol=1e-10, max_iters=harvest_iters)):
            rows[k].append(a)
        plan.close()
    X, T, W = (torch.cat(r) for r in rows)
    harvest_s = time.perf_counter() - t0
    m = pc.Mlp(seed=0)
    tinfo = m.train(X, T, W, epochs=150, batch=256, lr=1e-3, val_frac=0.25, patience=30, seed=1)
    log(f"[bench] {kernel}: harvest {harvest_s:.1f} s ({X.shape[0]} rows), training {tinfo['seconds']:.1f} s, "
        f"held-out loss {tinfo['init_val_loss']:.3f} -> {tinfo['best_val_loss']:.3f}")
    w = c5(n=n, kernel=kernel)
    plan = FmmPlan(dev(w.points), kernel=kernel, shape=shape, tol=1e-8)
    pc.set_learned(plan, m)
    f = dev(w.f)
    out = {}
    for kind in ("none", "block_jacobi", "learned"):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lam, inf = plan.solve(f, rtol=rtol, restart=50, max_iters=cap, precond=kind)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t1
        out[kind] = {"seconds": secs, "time_to_rtol": secs if inf["converged"] else None,
                     "iters": inf["iters"], "true_res": inf["true_res"], "converged": bool(inf["converged"]),
                     "fallback_used": inf["fallback_used"], "history": inf["history"][:16],
                     # true relative residual against wall time, at every restart
                     "curve_s_res": [[round(t_, 4), r_] for t_, r_ in zip(inf["history_s"][:64], inf["history"][:64])]}
        log(f"[bench] {kernel} {kind}: {inf['iters']} iterations, true residual {inf['true_res']:.3e}, "
            f"{secs:.2f} s")
    plan.close()
    torch.cuda.empty_cache()
    return {"workload": f"3d_mixed_{kernel}_c{shape}_bumps_rhs", "n": int(w.points.shape[0]), "restart": 50,
            "rtol": rtol, "cap_iters": cap, "product_tol": 1e-8, "solves": out,
            "training": {"rows": int(X.shape[0]), "problems": f"4 x {n_train} points (seeds 100-103)",
                         "harvest_seconds": harvest_s, "train_seconds": tinfo["seconds"],
                         "init_val_loss": tinfo["init_val_loss"], "best_val_loss": tinfo["best_val_loss"]}}


def run_solve(args):
    """GMRES(50) on the learned-preconditioner workload as specified: 3-D mixed points (2^21),
    multiquadric c = 0.02, f = 16 bumps of width 0.1, FP64 banded product at tol 1e-8, to a true
    residual of 1e-8 or the iteration cap: plain, block-Jacobi and learned."""
    import torch

    from paper_1606_07652_amd import FmmPlan
    from paper_1606_07652_amd import pc

    res = solve_family(torch, FmmPlan, pc, "multiquadric", 0.02, args.n_solve, 1e-8, args.solve_iters)
    lr = res["solves"]["learned"]
    result = {"metric": "GMRES(50) time to true residual 1e-8 (or the residual at the cap)",
              "value": lr["seconds"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
              "ms_per_step": lr["seconds"] * 1e3, "higher_is_better": False, "scaling": "weak",
              "vs_baseline": None, "dtype": "f64", "data": "synthetic",
              "config": {k: v for k, v in res.items() if k not in ("solves", "training")},
              "solves": res["solves"], "training": res["training"]}
    print(json.dumps(result), flush=True)


def banded_leg(torch, FmmPlan, w, kernel, steps, warmup, idx=None, ref=None, level=-1):
    """The banded product of a multiquadric kernel on the workload's points, FP64 (tol 1e-6)
    and FP32 (tol 1e-4): time per product, phase times and roofline fractions, and the
    sampled error against the oracle's direct sum when given."""
    n = w.points.shape[0]
    out = {}
    for name, dt, tol, bytes_ in (("f64", torch.float64, 1e-6, 8), ("f32", torch.float32, 1e-4, 4)):
        X = torch.as_tensor(w.points, dtype=dt, device="cuda:0")
        lam = torch.as_tensor(w.lam, dtype=dt, device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = FmmPlan(X, kernel=kernel, shape=w.shape, tol=tol, coarse_level=level)
        torch.cuda.synchronize()
        plan_ms = (time.perf_counter() - t0) * 1e3
        info = plan.info()
        bands = plan.bands()
        # aggregation and disaggregation run on the bands that are not transferred
        sum_p = sum(b["half_nodes"] for b in bands if not b["transfer"])
        moved = sum(1 for b in bands if b["transfer"])
        u = torch.empty_like(lam)
        for _ in range(warmup):
            plan.matvec(lam, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.matvec(lam, u)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        plan.set_profiling(True)
        for _ in range(3):
            plan.matvec(lam, u)
        torch.cuda.synchronize()
        ph = plan.phase_times()
        plan.set_profiling(False)
        calls = max(ph.pop("calls"), 1)
        phase_ms = {k: v / calls for k, v in ph.items()}
        fp_peak = FP64_VEC_TFLOPS if bytes_ == 8 else FP32_VEC_TFLOPS
        mfma_peak = FP64_MFMA_TFLOPS if bytes_ == 8 else FP32_VEC_TFLOPS
        model = {"p2p": ("alu", info["near_pairs"] * residual_pair_flops(info["d"], bytes_, info["residual_in_q"] == 1)),
                 "p2m": ("alu" if bytes_ == 8 else "mfma", 8.0 * n * sum_p),
                 "l2p": ("mfma", 8.0 * n * sum_p)}
        roofs = {k: roofline_of(*model[k], phase_ms[k], fp_peak, mfma_peak) for k in model if phase_ms.get(k, 0) > 0}
        dom = max(roofs, key=lambda k: phase_ms[k])
        roof = dict(roofs[dom], kernel=dom, traffic=None)
        out[name] = {"ms_per_step": ms, "points_per_s": n / (ms * 1e-3), "tol": tol, "plan_ms": plan_ms,
                     "bands": len(bands), "transferred_bands": moved, "sum_half_nodes": sum_p, "near_level": info["coarse_level"],
                     "near_pairs": info["near_pairs"], "residual_width": info["residual_width"],
                     "residual_in_q": info["residual_in_q"],
                     "phase_ms": phase_ms, "roofline": roof,
                     "phase_roofline": {k: {"bound": v["bound"], "frac": round(v["frac"], 4),
                                            "achieved": round(v["achieved"], 3), "unit": v["unit"]}
                                        for k, v in roofs.items()}}
        if ref is not None:
            from oracle import direct
            out[name]["rel_l2_sampled"] = direct.rel_l2(u.double().cpu().numpy()[idx], ref)
        log(f"[bench] {kernel} {name}: {ms:.2f} ms per product, {len(bands)} bands, "
            f"err {out[name].get('rel_l2_sampled', float('nan')):.2e}")
        plan.close()
        del X, lam, u
        torch.cuda.empty_cache()
    return out


def run_c4(args):
    """5-D: N = 2^18 uniform in [0,1]^5, Gaussian s = 0.2, float32 at tol 1e-5 (tensor-product
    quadrature over all five dimensions).  The fast product (leaf capacity 512) is timed with
    the device direct sum beside it; the oracle checks 2048 sampled targets."""
    import torch

    from paper_1606_07652_amd import FmmPlan
    from workloads import c4

    w = c4(n=args.n_c4)
    n = w.points.shape[0]
    X = torch.as_tensor(w.points, device="cuda:0")
    lam = torch.as_tensor(w.lam, device="cuda:0")
    t0 = time.perf_counter()
    plan = FmmPlan(X, kernel="gaussian", shape=w.shape, tol=w.tol, n_max=512)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info()
    log(f"[bench] 5-D plan {plan_ms:.0f} ms: nodes={info['nodes']} leaves={info['nleaves']} "
        f"far={info['far_field']} near_pairs={info['near_pairs']}")
    u = torch.empty_like(lam)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn(lam, u)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            fn(lam, u)
        torch.cuda.synchronize()
        return (time.perf_counter() - t1) * 1e3 / steps

    for _ in range(args.warmup):
        plan.matvec(lam, u)
    torch.cuda.synchronize()
    plan.set_profiling(True)
    ms = timed(plan.matvec, args.steps, 0)
    ph = plan.phase_times()
    plan.set_profiling(False)
    u_fmm = u.double().cpu().numpy()
    calls = max(ph.pop("calls"), 1)
    ms_direct = timed(plan.direct, max(2, args.steps // 5), 1)
    u_dir = u.double().cpu().numpy()
    plan.close()
    from paper_1606_07652_amd import autotune
    opts, _ = autotune(X, kernel="gaussian", shape=w.shape, tol=w.tol, reps=2)
    tplan = FmmPlan(X, kernel="gaussian", shape=w.shape, tol=w.tol, **opts)
    ms_tuned = timed(tplan.matvec, args.steps, args.warmup)
    u_tuned = u.double().cpu().numpy()
    tinfo = tplan.info()
    tplan.close()
    log(f"[bench] 5-D autotuned: n_max={opts['n_max']} leaves={tinfo['nleaves']} far={tinfo['far_field']} "
        f"{ms_tuned:.1f} ms")
    result = {"metric": "RBF-FMM matvec points/s @ rel-L2<=1e-5 (5-D)", "value": n / (ms * 1e-3),
              "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
              "data": "synthetic",
              "config": {"workload": "5d_uniform_gaussian_s0.2", "n": n, "tol": w.tol, "n_max": 512,
                         "nodes": info["nodes"], "leaves": info["nleaves"], "half_nodes": info["half_nodes"]},
              "plan_ms": plan_ms, "phase_ms": {k: v / calls for k, v in ph.items()},
              "direct_ms_per_step": ms_direct, "direct_points_per_s": n / (ms_direct * 1e-3),
              "autotuned": {"ms_per_step": ms_tuned, "points_per_s": n / (ms_tuned * 1e-3), "n_max": opts["n_max"],
                            "leaves": tinfo["nleaves"], "far_field": tinfo["far_field"]}}
    if not args.no_cpu:
        from oracle import direct
        rng = np.random.default_rng(4)
        idx = np.sort(rng.choice(n, 2048, replace=False))
        xs = w.points.astype(np.float64)
        t1 = time.perf_counter()
        ref = direct.direct_sum(xs, w.lam.astype(np.float64), "gaussian", w.shape, targets=xs[idx])
        tcpu = time.perf_counter() - t1
        result["rel_l2_sampled"] = direct.rel_l2(u_fmm[idx], ref)
        result["direct_rel_l2_sampled"] = direct.rel_l2(u_dir[idx], ref)
        result["autotuned"]["rel_l2_sampled"] = direct.rel_l2(u_tuned[idx], ref)
        result["cpu_baseline"] = {"value": 2048 / tcpu, "unit": "points/s", "cores": direct.threads(),
                                  "kind": "oracle", "sample": f"2048 seeded targets x all {n} sources ({tcpu:.1f} s)"}
    print(json.dumps(result), flush=True)


def run_c2mq(args):
    """3-D mixed points (as the default workload), multiquadric (or, with --mq-kernel, inverse
    multiquadric) c = 0.02: the banded far field, FP64 at tol 1e-6 and FP32 at 1e-4 (with
    --mq-kernel thin_plate or r5: the exact sum, the only product those kernels have).  The
    oracle checks 2048 targets."""
    import torch

    from paper_1606_07652_amd import FmmPlan
    from workloads import c2

    kern = args.mq_kernel
    w = c2("multiquadric", n=args.n)
    n = w.points.shape[0]
    rng = np.random.default_rng(123)
    idx = np.sort(rng.choice(n, 2048, replace=False))
    ref = None
    if not args.no_cpu:
        from oracle import direct
        xs = w.points.astype(np.float64)
        t1 = time.perf_counter()
        ref = direct.direct_sum(xs, w.lam.astype(np.float64), kern, w.shape, targets=xs[idx])
        tcpu = time.perf_counter() - t1
    if kern in ("multiquadric", "inverse_multiquadric"):
        out = banded_leg(torch, FmmPlan, w, kern, max(2, args.steps // 2), 2, idx, ref, args.mq_level)
        metric = f"RBF-FMM matvec points/s @ rel-L2<=1e-6, {kern.replace('_', ' ')} (banded far field)"
    else:
        out = {}
        for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
            X = torch.as_tensor(w.points, dtype=dt, device="cuda:0")
            lam = torch.as_tensor(w.lam, dtype=dt, device="cuda:0")
            plan = FmmPlan(X, kernel=kern, shape=w.shape, tol=1e-6)
            u = torch.empty_like(lam)
            plan.matvec(lam, u)
            torch.cuda.synchronize()
            steps = max(2, args.steps // 4)
            t0 = time.perf_counter()
            for _ in range(steps):
                plan.matvec(lam, u)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            out[name] = {"ms_per_step": ms, "points_per_s": n / (ms * 1e-3),
                         "pairs_per_s": float(n) * n / (ms * 1e-3)}
            if ref is not None:
                out[name]["rel_l2_sampled"] = direct.rel_l2(u.double().cpu().numpy()[idx], ref)
            log(f"[bench] {kern} {name}: {ms:.1f} ms per product")
            plan.close()
        metric = f"RBF matvec points/s, {kern.replace('_', ' ')} (exact sum)"
    result = {"metric": metric, "value": out["f64"]["points_per_s"],
              "unit": "points/s", "n_gpus": 1, "steps": max(2, args.steps // 2), "warmup": 2,
              "ms_per_step": out["f64"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "f64", "data": "synthetic",
              "config": {"workload": f"3d_mixed_uniform_blobs_{kern}_c0.02", "n": n, "kernel": kern,
                         "shape": w.shape}, "paths": out}
    if "roofline" in out["f64"]:
        result["roofline"] = out["f64"]["roofline"]
    if ref is not None:
        result["cpu_baseline"] = {"value": 2048 / tcpu, "unit": "points/s", "cores": direct.threads(),
                                  "kind": "oracle", "sample": f"2048 seeded targets x all {n} sources ({tcpu:.1f} s)"}
    print(json.dumps(result), flush=True)


# Wendland's function: every candidate (near) pair costs its squared distance (3d flops); a pair
# inside the support also costs the accumulation (3) and the function: e r (the square root
# counted as one flop, one multiply), 1 - e r and the clamp, the cube (two multiplies), 3 e r + 1
# (an fma, 2) and the product of the two factors, 9 flops.  Pairs outside the support add zero
# and the kernel skips the steps where all of them are; they count only their distance.
WENDLAND_PAIR_FLOPS = 9


def run_wendland(args):
    """Wendland's compactly supported function (1 - e r)_+^3 (3 e r + 1) on the default
    workload's 2^20 mixed points, e = 25 (support radius 0.04): a uniform tree at the deepest
    level whose cells hold the support radius, the adjacent cells as near field, no far field,
    so the product is exact.  FP64 and FP32; value = points / time of one FP64 product; the
    roofline is the near-field kernel's flops over its measured time; the oracle checks 2048
    targets."""
    import torch

    from paper_1606_07652_amd import FmmPlan
    from workloads import c2

    w = c2("gaussian", n=args.n)
    e = 25.0
    n, d = w.points.shape
    rng = np.random.default_rng(123)
    idx = np.sort(rng.choice(n, 2048, replace=False))
    # ordered pairs (self pairs included) closer than the support radius: a property of the
    # point set, counted on the host with a k-d tree
    from scipy.spatial import cKDTree
    tree = cKDTree(w.points.astype(np.float64))
    support_pairs = int(tree.count_neighbors(tree, 1.0 / e))
    del tree
    log(f"[bench] wendland: {support_pairs:.3e} pairs inside the support")
    ref = None
    if not args.no_cpu:
        from oracle import direct
        xs = w.points.astype(np.float64)
        t1 = time.perf_counter()
        ref = direct.direct_sum(xs, w.lam.astype(np.float64), "wendland", e, targets=xs[idx])
        tcpu = time.perf_counter() - t1
    out = {}
    for name, dt, peak in (("f64", torch.float64, FP64_VEC_TFLOPS), ("f32", torch.float32, FP32_VEC_TFLOPS)):
        X = torch.as_tensor(w.points, dtype=dt, device="cuda:0")
        lam = torch.as_tensor(w.lam, dtype=dt, device="cuda:0")
        t0 = time.perf_counter()
        plan = FmmPlan(X, kernel="wendland", shape=e, tol=1e-6)
        torch.cuda.synchronize()
        plan_ms = (time.perf_counter() - t0) * 1e3
        inf = plan.info()
        u = torch.empty_like(lam)
        for _ in range(args.warmup):
            plan.matvec(lam, u)
        torch.cuda.synchronize()
        plan.set_profiling(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.matvec(lam, u)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        ph = plan.phase_times()
        plan.set_profiling(False)
        calls = max(ph.pop("calls"), 1)
        phase_ms = {k: v / calls for k, v in ph.items()}
        flops = float(inf["near_pairs"]) * 3 * d + float(support_pairs) * (3 + WENDLAND_PAIR_FLOPS)
        out[name] = {"ms_per_step": ms, "points_per_s": n / (ms * 1e-3), "plan_ms": plan_ms,
                     "phase_ms": phase_ms, "level": inf["coarse_level"], "leaves": inf["nleaves"],
                     "near_pairs": inf["near_pairs"], "support_pairs": support_pairs, "far_field": inf["far_field"],
                     "roofline": roofline_of("alu", flops, phase_ms["p2p"], peak)}
        if ref is not None:
            out[name]["rel_l2_sampled"] = direct.rel_l2(u.double().cpu().numpy()[idx], ref)
        log(f"[bench] wendland {name}: {ms:.2f} ms per product, level {inf['coarse_level']}, "
            f"{inf['near_pairs']:.3e} near pairs")
        plan.close()
        del X, lam, u
        torch.cuda.empty_cache()
    f = out["f64"]
    roof = dict(f["roofline"])
    roof["traffic"] = None
    result = {"metric": "RBF matvec points/s, Wendland (exact, near field only)", "value": f["points_per_s"],
              "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "ms_per_step": f["ms_per_step"], "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "f64", "data": "synthetic",
              "config": {"workload": "3d_mixed_uniform_blobs_wendland_e25", "n": n, "kernel": "wendland",
                         "shape": e},
              "roofline": roof, "paths": out}
    if ref is not None:
        result["cpu_baseline"] = {"value": len(idx) / tcpu, "unit": "points/s", "cores": direct.threads(),
                                  "kind": "oracle",
                                  "sample": f"{len(idx)} seeded targets x all {n} sources ({tcpu:.1f} s)"}
    print(json.dumps(result), flush=True)


def bandlimited_pair_flops(d, deg):
    """Floating-point operations the band-limited kernel executes per pair: per axis the
    difference, its scaling to a piece position, the local variable u = 2 (s - i) - 1 and a
    Horner step of the table's degree (7 in FP64, 3 in FP32: that many FMAs); the product over
    the axes and the weighted accumulation.  3-D: 58 (FP64), 34 (FP32)."""
    return d * (1 + 1 + 2 + 2 * deg) + (d - 1) + 2


def run_bandlimited(args):
    """The band-limited Gaussian as the basis (section 3, eq. 16 with the box of eq. 28):
    Phi_sigma(x) = prod_k phi_sigma(x_k), s = 0.03, s sigma = 3, on 2^16 points of the default
    workload's mixed uniform/blob distribution, as the exact sum over all pairs (tiled direct
    kernel; per-axis tables of degree 7 in FP64, 3 in FP32), FP64 at tol 1e-10 and FP32 at 1e-5.
    value = points / time of one FP64 product;
    the roofline is the direct kernel's executed flops per pair over its time; the oracle
    (closed form through scipy's Faddeeva function) checks 256 seeded targets."""
    import torch

    from paper_1606_07652_amd import FmmPlan
    from workloads import c2

    w = c2("gaussian", n=args.n_bl)
    n, d = w.points.shape
    s, sigma = 0.03, 3.0 / 0.03
    rng = np.random.default_rng(321)
    idx = np.sort(rng.choice(n, min(n, 256), replace=False))
    ref = None
    if not args.no_cpu:
        from oracle import bandlimit
        xs = w.points.astype(np.float64)
        t1 = time.perf_counter()
        ref = bandlimit.direct_sum_phi_sigma(xs, w.lam.astype(np.float64), s, sigma, targets=xs[idx])
        tcpu = time.perf_counter() - t1
    out = {}
    for name, dt, tol, peak in (("f64", torch.float64, 1e-10, FP64_VEC_TFLOPS),
                                ("f32", torch.float32, 1e-5, FP32_VEC_TFLOPS)):
        X = torch.as_tensor(w.points, dtype=dt, device="cuda:0")
        lam = torch.as_tensor(w.lam, dtype=dt, device="cuda:0")
        t0 = time.perf_counter()
        plan = FmmPlan(X, kernel="gaussian_bandlimited", shape=s, tol=tol, band=sigma)
        torch.cuda.synchronize()
        plan_ms = (time.perf_counter() - t0) * 1e3
        u = torch.empty_like(lam)
        for _ in range(args.warmup):
            plan.matvec(lam, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.matvec(lam, u)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        flops = float(n) * n * bandlimited_pair_flops(d, 7 if dt == torch.float64 else 3)
        out[name] = {"ms_per_step": ms, "points_per_s": n / (ms * 1e-3), "pairs_per_s": float(n) * n / (ms * 1e-3),
                     "plan_ms": plan_ms, "tol": tol, "roofline": roofline_of("alu", flops, ms, peak)}
        if ref is not None:
            out[name]["rel_l2_sampled"] = float(np.linalg.norm(u.double().cpu().numpy()[idx] - ref) /
                                                np.linalg.norm(ref))
        log(f"[bench] bandlimited {name}: {ms:.2f} ms per product ({n * n / (ms * 1e-3):.3e} pairs/s), "
            f"plan {plan_ms:.0f} ms")
        plan.close()
        # evaluation at n separate targets uniform over the unit cube (the near-field kernel over
        # the joint set, the table read from global memory)
        from paper_1606_07652_amd import EvalPlan
        from workloads import uniform_points
        Y = torch.as_tensor(uniform_points(n, d, 17), dtype=dt, device="cuda:0")
        ep = EvalPlan(X, Y, kernel="gaussian_bandlimited", shape=s, tol=tol, band=sigma)
        ue = ep.eval(lam)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ep.eval(lam, ue)
        torch.cuda.synchronize()
        ems = (time.perf_counter() - t0) * 1e3 / args.steps
        out[name]["eval_ms"] = ems
        out[name]["eval_pairs_per_s"] = float(n) * n / (ems * 1e-3)
        log(f"[bench] bandlimited {name} evaluation at {n} targets: {ems:.2f} ms")
        ep.close()
        del X, lam, u, Y, ue
        torch.cuda.empty_cache()
    f = out["f64"]
    roof = dict(f["roofline"])
    roof["traffic"] = None
    result = {"metric": "RBF matvec points/s, band-limited Gaussian basis (exact sum)", "value": f["points_per_s"],
              "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "ms_per_step": f["ms_per_step"], "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "f64", "data": "synthetic",
              "config": {"workload": "3d_mixed_uniform_blobs_gaussian_bandlimited_s0.03_ssigma3", "n": n,
                         "kernel": "gaussian_bandlimited", "shape": s, "band": sigma},
              "roofline": roof, "paths": out}
    if ref is not None:
        result["cpu_baseline"] = {"value": len(idx) / tcpu, "unit": "points/s", "cores": 1, "kind": "oracle",
                                  "sample": f"{len(idx)} seeded targets x all {n} sources ({tcpu:.1f} s)"}
    print(json.dumps(result), flush=True)


def run_eval(args):
    """Evaluation at separate targets: the default workload's 2^20 mixed sources and weights,
    2^20 targets uniform over the unit cube (seed 7), FP64 at tol 1e-6 and FP32 at 1e-4.
    value = targets / time of one evaluation; the oracle checks 2048 seeded targets."""
    import torch

    from paper_1606_07652_amd import EvalPlan
    from workloads import c2, uniform_points

    w = c2("gaussian", n=args.n)
    n = w.points.shape[0]
    y = uniform_points(args.n_targets, 3, 7)
    m = y.shape[0]
    rng = np.random.default_rng(124)
    idx = np.sort(rng.choice(m, min(2048, m), replace=False))
    ref = None
    if not args.no_cpu:
        from oracle import direct
        t1 = time.perf_counter()
        ref = direct.direct_sum(w.points.astype(np.float64), w.lam.astype(np.float64), "gaussian", w.shape,
                                targets=y[idx])
        tcpu = time.perf_counter() - t1
    out = {}
    for name, dt, tol in (("f64", torch.float64, 1e-6), ("f32", torch.float32, 1e-4)):
        X = torch.as_tensor(w.points, dtype=dt, device="cuda:0")
        Y = torch.as_tensor(y, dtype=dt, device="cuda:0")
        lam = torch.as_tensor(w.lam, dtype=dt, device="cuda:0")
        t0 = time.perf_counter()
        plan = EvalPlan(X, Y, kernel="gaussian", shape=w.shape, tol=tol, n_max=args.n_max)
        plan_ms = (time.perf_counter() - t0) * 1e3
        u = torch.empty(m, dtype=dt, device="cuda:0")
        for _ in range(args.warmup):
            plan.eval(lam, u)
        torch.cuda.synchronize()
        plan.set_profiling(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.eval(lam, u)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        ph = plan.phase_times()
        plan.set_profiling(False)
        calls = max(ph.pop("calls"), 1)
        inf = plan.info()
        out[name] = {"ms_per_step": ms, "targets_per_s": m / (ms * 1e-3), "plan_ms": plan_ms,
                     "phase_ms": {k: v / calls for k, v in ph.items()}, "nodes": inf["nodes"],
                     "leaves": inf["nleaves"]}
        if ref is not None:
            out[name]["rel_l2_sampled"] = direct.rel_l2(u.double().cpu().numpy()[idx], ref)
        log(f"[bench] eval {name}: {ms:.2f} ms for {m} targets ({n} sources)")
        plan.close()
        del X, Y, lam, u
        torch.cuda.empty_cache()
    f = out["f64"]
    dom = max(f["phase_ms"], key=lambda k: f["phase_ms"][k])
    result = {"metric": "RBF-FMM evaluation targets/s @ rel-L2<=1e-6", "value": f["targets_per_s"],
              "unit": "targets/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "ms_per_step": f["ms_per_step"], "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "f64", "data": "synthetic",
              "config": {"workload": "3d_mixed_sources_uniform_targets_gaussian_s0.03", "n_sources": n,
                         "n_targets": m, "kernel": "gaussian", "shape": w.shape, "tol": 1e-6,
                         "n_max": args.n_max},
              "dominant_phase": dom, "paths": out}
    if ref is not None:
        result["cpu_baseline"] = {"value": len(idx) / tcpu, "unit": "targets/s", "cores": direct.threads(),
                                  "kind": "oracle",
                                  "sample": f"{len(idx)} seeded targets x all {n} sources ({tcpu:.1f} s)"}
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--n-max", type=int, default=256)
    ap.add_argument("--cpu-targets", type=int, default=32768)
    ap.add_argument("--copy-check", action="store_true",
                    help="copy a 1 GiB buffer once (a plain copy kernel of known size, used to scale "
                         "hardware byte counters)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="single", choices=["single", "batched", "solve", "c4", "c2mq", "eval", "wendland",
                                                          "bandlimited"])
    ap.add_argument("--n-bl", type=int, default=1 << 16, help="points of --workload bandlimited")
    ap.add_argument("--n-targets", type=int, default=1 << 20)
    ap.add_argument("--n-c4", type=int, default=1 << 18)
    ap.add_argument("--n-solve", type=int, default=1 << 21)
    ap.add_argument("--solve-iters", type=int, default=300)
    ap.add_argument("--no-mq", action="store_true", help="skip the multiquadric leg of the default run")
    ap.add_argument("--no-solve", action="store_true", help="skip the GMRES leg of the default run")
    ap.add_argument("--n-solve-default", type=int, default=1 << 18,
                    help="points of the GMRES leg of the default run")
    ap.add_argument("--solve-cap-default", type=int, default=200,
                    help="iteration cap of the GMRES leg of the default run")
    ap.add_argument("--nprob", type=int, default=512)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--batched-solve", action="store_true",
                    help="with --workload batched: also run GMRES on all problems at once")
    ap.add_argument("--m2l-schedule", type=int, default=0)
    ap.add_argument("--mq-level", type=int, default=-1,
                    help="with --workload c2mq: level of the near field's uniform tree (-1: the plan's default)")
    ap.add_argument("--mq-kernel", default="multiquadric",
                    choices=["multiquadric", "inverse_multiquadric", "thin_plate", "r5"],
                    help="with --workload c2mq: the kernel of the exact sum")
    ap.add_argument("--traffic-table", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT_JSON"),
                    help="write the HBM byte table from two rocprofv3 counter runs (no GPU work)")
    args = ap.parse_args()
    if args.traffic_table:
        return write_traffic_table(*args.traffic_table,
                                   workload="3-D mixed uniform/blob points, N=2^20, Gaussian s=0.03, "
                                            "FP64 tol 1e-6 (leaf capacity 256)")
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); sharding over several GPUs "
              "is not built", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "solve":
        return run_solve(args)
    if args.workload == "c4":
        return run_c4(args)
    if args.workload == "c2mq":
        return run_c2mq(args)
    if args.workload == "eval":
        return run_eval(args)
    if args.workload == "wendland":
        return run_wendland(args)
    if args.workload == "bandlimited":
        return run_bandlimited(args)

    import torch

    from paper_1606_07652_amd import FmmPlan
    from workloads import c2

    if args.copy_check:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy check: 1 GiB read + 1 GiB written")
        del src, dst
        torch.cuda.empty_cache()

    w = c2("gaussian", n=args.n)
    n = w.points.shape[0]
    log(f"[bench] workload {w.name}: n={n}")
    main_run = run_path(torch, FmmPlan, w, torch.float64, 1e-6, args.steps, args.warmup, args.n_max,
                        args.m2l_schedule)
    f32_run = None if args.no_fp32 else run_path(torch, FmmPlan, w, torch.float32, 1e-4, args.steps,
                                                  args.warmup, args.n_max, args.m2l_schedule)

    # dominant kernel of the headline path and its roofline
    info = main_run["info"]
    model = phase_model(info, 8, n)
    ph = main_run["phase_ms"]
    dom = max((k for k in ph if k in model), key=lambda k: ph[k])
    roof = roofline_of(*model[dom], ph[dom], FP64_VEC_TFLOPS)
    roof["traffic"] = measured_traffic(dom)
    roof["kernel"] = dom
    if dom == "p2p":
        roof["pairs_per_s"] = info["near_pairs"] / (ph[dom] * 1e-3)
        roof["flops_per_pair"] = gauss_pair_flops(info["d"], 8)
    phase_roof = {k: roofline_of(*model[k], ph[k], FP64_VEC_TFLOPS) for k in model if ph.get(k, 0) > 0}
    bw = copy_bandwidth(torch)
    prod_roof = product_roofline(model, main_run["ms_per_step"], FP64_VEC_TFLOPS, FP64_MFMA_TFLOPS, bw)

    result = {
        "metric": "RBF-FMM matvec points/s @ rel-L2<=1e-6; GMRES time-to-1e-8 learned-PC vs plain",
        "value": n / (main_run["ms_per_step"] * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3d_mixed_uniform_blobs_gaussian_s0.03", "n": n, "kernel": "gaussian",
                   "shape": w.shape, "tol": 1e-6, "n_max": args.n_max, "nodes": info["nodes"],
                   "leaves": info["nleaves"], "coarse_level": info["coarse_level"],
                   "coarse_radius": info["coarse_radius"]},
        "plan_ms": main_run["plan_ms"],
        "phase_ms": main_run["phase_ms"],
        "roofline": roof,
        "phase_roofline": {k: {"bound": v["bound"], "frac": round(v["frac"], 4), "achieved": round(v["achieved"], 3),
                               "unit": v["unit"]} for k, v in phase_roof.items()},
        "product_roofline": prod_roof,
    }
    if f32_run is not None:
        result["fp32_path"] = {"value": n / (f32_run["ms_per_step"] * 1e-3), "unit": "points/s", "tol": 1e-4,
                               "ms_per_step": f32_run["ms_per_step"], "nodes": f32_run["info"]["nodes"],
                               "phase_ms": f32_run["phase_ms"],
                               "product_roofline": product_roofline(phase_model(f32_run["info"], 4, n),
                                                                    f32_run["ms_per_step"], FP32_VEC_TFLOPS,
                                                                    FP32_VEC_TFLOPS, bw)}

    if not args.no_mq:
        # the multiquadric half of the workload: same points and weights, c = 0.02
        wm = c2("multiquadric", n=args.n)
        idx_m, ref_m = None, None
        if not args.no_cpu:
            from oracle import direct
            rng = np.random.default_rng(124)
            idx_m = np.sort(rng.choice(n, 2048, replace=False))
            xs = wm.points.astype(np.float64)
            ref_m = direct.direct_sum(xs, wm.lam.astype(np.float64), "multiquadric", wm.shape, targets=xs[idx_m])
        legs = banded_leg(torch, FmmPlan, wm, "multiquadric", max(2, args.steps // 2), 2, idx_m, ref_m)
        result["multiquadric"] = {"value": legs["f64"]["points_per_s"], "unit": "points/s", "shape": wm.shape,
                                  "tol": 1e-6, "ms_per_step": legs["f64"]["ms_per_step"], "paths": legs}
    if not args.no_solve:
        from paper_1606_07652_amd import pc
        result["solve"] = solve_family(torch, FmmPlan, pc, "multiquadric", 0.02, args.n_solve_default, 1e-8,
                                       args.solve_cap_default)

    if not args.no_cpu:
        # cpu_baseline leg: the oracle's direct sum on a bounded sample of targets; the same
        # sample gives the sampled rel-L2 of both GPU paths.
        from oracle import direct
        rng = np.random.default_rng(123)
        idx = np.sort(rng.choice(n, args.cpu_targets, replace=False))
        xs = w.points.astype(np.float64)
        ls = w.lam.astype(np.float64)
        log(f"[bench] cpu oracle on {args.cpu_targets} targets x {n} sources ...")
        t0 = time.perf_counter()
        ref = direct.direct_sum(xs, ls, "gaussian", w.shape, targets=xs[idx])
        tcpu = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": args.cpu_targets / tcpu, "unit": "points/s", "cores": direct.threads(),
                                  "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
                                  "sample": f"{args.cpu_targets} seeded targets x all {n} sources, FP64 direct sum "
                                            f"({tcpu:.1f} s; points/s = targets / time)"}
        result["rel_l2_sampled"] = direct.rel_l2(main_run["u"][idx], ref)
        if f32_run is not None:
            result["fp32_path"]["rel_l2_sampled"] = direct.rel_l2(f32_run["u"][idx], ref)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
