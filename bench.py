#!/usr/bin/env python3
"""Benchmark of the preconditioned Lippmann-Schwinger solver on one MI355X.

One step is one pass of the whole path over one batch: set the medium
(contrast, FP64 kernel table, circulant spectrum), form the incident fields of
all sources, build the preconditioner, and run the preconditioned scattering
series (eq. 11) for every source to the relative residual target.  Inputs
(velocity grid, source positions) are resident before the timed region.  The
default workload is the 1024 x 1024 grid at h = 5 m and 25 Hz with 128
sources on the top row, computed in complex FP32 (QR / LU / leaf inverses in
FP64), with the HODLR preconditioner of Section 2.4 (rank 256, 10 levels, one
power iteration per block); `--pc lowrank` selects the rank-r preconditioner
of Section 2.3 instead.

Printed: one JSON line with the solves/s of sources that reached the target,
the dominant kernel's roofline position (event-timed inside the timed region,
per kernel function), the FFT-convolution throughput of the LS operator, and
the FP64 oracle timed on a bounded sample of the same workload on the host
cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LS solves/s to rel. residual 1e-6 at 1024^2 x128 src; FFT-conv HBM GB/s"
HBM_PEAK_GBPS = 8000.0
MFMA_PEAK_TFLOPS = {"float": 157.3, "double": 78.6, "bf16": 2500.0}   # dense matrix-core peaks
VALU_PEAK_TFLOPS = {"float": 157.3, "double": 78.6}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("ls1024", "uneven", "unet"), default="ls1024",
                    help="ls1024: the 1024^2 x 128-source headline; uneven: 64 instances of uneven size in one batch; "
                         "unet: training steps of the warm-start network on solver-generated 128^2 solutions, then "
                         "the warm-started series at 256^2 and 512^2")
    ap.add_argument("--unet-models", type=int, default=32,
                    help="layered + salt models (32 sources each) solved for the network's training data")
    ap.add_argument("--unet-batch", type=int, default=64, help="training batch (the workload leaves it free)")
    ap.add_argument("--unet-epochs", type=int, default=0,
                    help="unet: untimed training epochs over all generated samples after the timed steps, then the "
                         "error of the warm start on held-out 128^2 models (and the evaluation at 256^2 and 512^2 "
                         "uses the trained network)")
    ap.add_argument("--unet-no-eval", action="store_true",
                    help="skip the warm-started series after the timed training steps (counter runs: the timed "
                         "launches are then each kernel's last dispatches)")
    ap.add_argument("--count", type=int, default=64, help="instances of the uneven batch")
    ap.add_argument("--leaf-cols", type=int, default=1,
                    help="uneven batch: HODLR trees as deep as leaves of at least this many grid columns allow "
                         "(measured: 1 column 114.8 solves/s, 2 columns 112.8, 3 columns 85.5; the FP64 leaf "
                         "inverses grow with the cube of the leaf size)")
    ap.add_argument("--build-streams", type=int, default=8,
                    help="uneven batch: preconditioner builds run concurrently on this many device streams")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1024, help="grid side (default: the 1024^2 workload)")
    ap.add_argument("--nsrc", type=int, default=128)
    ap.add_argument("--pc", choices=("hodlr", "lowrank"), default="hodlr")
    ap.add_argument("--dtype", choices=("c64", "c128", "mixed"), default="c64",
                    help="ls1024: complex FP32 series (c64), plain complex FP64 series (c128), or complex FP32 inner "
                         "series with FP64 residuals and refinement (mixed)")
    ap.add_argument("--no-fp64-compare", action="store_true",
                    help="ls1024: skip the untimed plain FP64 solve after the timed steps (to a relative residual "
                         "of 1e-10: the relative error of every timed solution against it)")
    ap.add_argument("--init", choices=("h_rhs", "learned"), default="h_rhs",
                    help="ls1024: series start H psi0 (the paper's), or the warm-start network's field, kept per "
                         "source only where its true residual is smaller (the network is first trained, untimed, "
                         "on --unet-models solver-generated layered + salt models at 128^2)")
    ap.add_argument("--unet-train-steps", type=int, default=300, help="ls1024 --init learned: training steps")
    ap.add_argument("--solver", choices=("series", "gmres"), default="series",
                    help="ls1024: the preconditioned scattering series (eq. 11), or restarted GMRES right-"
                         "preconditioned by the same H (the paper's comparison method, Section 3.2.3)")
    ap.add_argument("--restart", type=int, default=20, help="ls1024 --solver gmres: Krylov vectors per cycle")
    ap.add_argument("--rank", type=int, default=None, help="probes per block (default 256 hodlr, 64 lowrank)")
    ap.add_argument("--levels", type=int, default=10)
    ap.add_argument("--power-iters", type=int, default=None, help="default 1 hodlr, 0 lowrank")
    ap.add_argument("--q-from-level", type=int, default=None,
                    help="hodlr: power iterations on tree levels >= this one only (ls1024 default 5; measured: "
                         "0 -> 63.9, 2 -> 67.0, 4 -> 68.9, 5 -> 70.1, 6 -> 69.7 (4-5 iterations), 7 -> 65.5 "
                         "(7 iterations) solves/s, 8 does not converge)")
    ap.add_argument("--q-from-frac", type=float, default=0.5,
                    help="uneven: each instance's power iterations on its tree levels >= this fraction of its "
                         "depth only (measured: 0 -> 151.0, 0.3 -> 171.2, 0.5 -> 174.7, 0.7 -> 157.5 solves/s)"),
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sources", type=int, default=2, help="sources in the oracle's timed sample")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 1 GiB device-to-device (a plain copy of known size for rocprofv3 --pmc scaling)")
    ap.add_argument("--dump-profile", default=None,
                    help="write the per-kernel-function event profile of the timed region to this JSON file")
    a = ap.parse_args()
    if a.rank is None:
        a.rank = 256 if a.pc == "hodlr" else 64
    if a.power_iters is None:
        a.power_iters = 1 if a.pc == "hodlr" else 0
    if a.q_from_level is None:
        a.q_from_level = 5 if (a.pc == "hodlr" and a.workload == "ls1024") else 0
    return a


def measure_copy_gbps(nbytes=4 << 30, reps=5):
    """Achievable HBM bandwidth on this GPU: a plain device-to-device copy of nbytes (read + write counted),
    best of `reps`, timed with events on the current stream."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.complex64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / best / 1e9


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def load_traffic(kernel, summary="pmc_traffic.json"):
    """Counter-measured HBM bytes over algorithmic bytes for one kernel function, from the committed
    summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    from paper_2005_01372_amd.profiling import kernel_source_sha
    k = d.get("kernels", {}).get(kernel)
    if not k or d.get("source_sha") != kernel_source_sha():
        return None
    return k.get("hbm_over_algorithmic")


def roofline_for(name, st):
    """Roofline position of one kernel function from its event-timed totals."""
    avg_s = st["ms"] / st["launches"] / 1e3
    bpl, fpl = st["bytes"] / st["launches"], st["flops"] / st["launches"]
    t = "double" if "<double" in name else "float"
    if name.startswith(("k_conv_fwd", "k_conv_wgrad")):
        t = "bf16"   # bf16 operands on the matrix cores, FP32 accumulation
    mfma = name.startswith(("k_bgemm_mfma", "k_gemm_ah_b_mfma", "k_gemm_ah_b_narrow", "k_gemm_update_mfma",
                            "k_gemm_update_tile", "k_conv_fwd", "k_conv_wgrad"))
    small = name.startswith(("k_lu_inverse", "k_gram_orth"))
    out = {"kernel": name, "avg_launch_ms": round(avg_s * 1e3, 4), "launches": st["launches"],
           "algorithmic_bytes_per_launch": bpl, "algorithmic_flops_per_launch": fpl}
    if mfma or small:
        peak_f = (MFMA_PEAK_TFLOPS if mfma else VALU_PEAK_TFLOPS)["double" if small else t]
        ridge = peak_f * 1e12 / (HBM_PEAK_GBPS * 1e9)
        ai = fpl / bpl if bpl > 0 else float("inf")
        out["arithmetic_intensity"] = round(ai, 2)
        if ai >= ridge:
            ach = fpl / avg_s / 1e12
            out.update(bound="mfma" if mfma else "alu", achieved=round(ach, 2), peak=peak_f, unit="TFLOP/s",
                       frac=round(ach / peak_f, 4))
            return out
    ach = bpl / avg_s / 1e9
    out.update(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBPS, unit="GB/s", frac=round(ach / HBM_PEAK_GBPS, 4))
    return out


def cpu_baseline(w, args, iterations, converged, nsrc_sample=2):
    """The FP64 oracle (numpy / scipy, as written) timed on a bounded sample of the same step.

    The oracle's HODLR builds a dense matrix and cannot hold the 1024^2 grid,
    so the step is assembled from the oracle's own primitives, each timed on
    a sample and scaled by how often the GPU step performs it: problem set-up;
    the FFT operator application (every sub-domain convolution of a level
    costs one full-grid application per vector); one dense leaf block and its
    inverse (numpy.linalg.inv), times the number of leaves; Householder QR
    (numpy.linalg.qr) of one half-node block per level, times the number of
    half-nodes; the leaf and low-rank products of one preconditioner
    application per vector; and the series iterations the GPU run needed.
    """
    import numpy as np

    from oracle import lsop_oracle as O

    cores = len(os.sched_getaffinity(0))
    r, L, q = args.rank, args.levels, args.power_iters
    t0 = time.perf_counter()
    prob = O.Problem(w.vel, w.h, w.freq, w.c0)
    prob.workers = cores
    t_setup = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    x = rng.standard_normal((nsrc_sample, prob.nx, prob.nz)) + 0j
    t1 = time.perf_counter()
    prob.apply(x, "G0V")
    t_conv = (time.perf_counter() - t1) / nsrc_sample            # one full-grid convolution, per vector
    n = prob.n
    if args.pc == "hodlr":
        wl = prob.nx >> L
        nl, nleaf = wl * prob.nz, 1 << L
        t2 = time.perf_counter()
        G = O.greens_matrix(prob.K[:wl, :])
        D = np.eye(nl) - G * prob.chi[:wl].reshape(-1)[None, :]
        Dinv = np.linalg.inv(D)
        t_leaf = time.perf_counter() - t2
        t3 = time.perf_counter()
        Dinv @ x[0].reshape(-1)[:nl]
        t_leafmv = (time.perf_counter() - t3) * nleaf                # one vector through all leaves
        # Householder QR of one half-node block at the middle level, scaled to all half-nodes of every level
        lv = L // 2
        seg = (prob.nx >> (lv + 1)) * prob.nz
        Yb = rng.standard_normal((seg, r)) + 1j * rng.standard_normal((seg, r))
        t4 = time.perf_counter()
        np.linalg.qr(Yb)
        t_qr_level = (time.perf_counter() - t4) * (2 << lv)
        Vr = rng.standard_normal((r, seg)) + 0j
        t5 = time.perf_counter()
        Vr.conj() @ Yb[:, 0]
        Vr.T @ (Vr.conj() @ Yb[:, 0])
        t_lr_level = (time.perf_counter() - t5) * (2 << lv)          # V^H y and W s over one level, one vector
        t_h = t_leafmv + L * t_lr_level                              # one preconditioner application, one vector
        # per level: half-masked sub-domain passes, each a full-grid convolution per vector, and the QR passes;
        # the power iterations only on the levels >= q_from_level
        qs = [q if l >= args.q_from_level else 0 for l in range(L)]
        t_build = nleaf * t_leaf + sum((4 + 4 * ql) * r * t_conv + (1 + 2 * ql) * t_qr_level for ql in qs)
        t_build += sum(r * (t_leafmv + (L - 1 - l) * t_lr_level) for l in range(L))   # W = A_{l+1}^{-1} U per level
        desc = (f"set-up; one FFT application ({nsrc_sample} vectors); one {nl}x{nl} leaf formed and inverted (x{nleaf});"
                f" one {seg}x{r} QR (x{2 << lv} half-nodes per level, 1 + 2 q per level); leaf and low-rank "
                f"products of one H application; scaled by the GPU step's counts")
    else:
        Yb = rng.standard_normal((n, r)) + 0j
        t4 = time.perf_counter()
        np.linalg.qr(Yb)
        t_qr = time.perf_counter() - t4
        t5 = time.perf_counter()
        Yb @ (Yb.conj().T @ x[0].reshape(-1))
        t_h = time.perf_counter() - t5
        t_build = 2 * (1 + q) * r * t_conv + (1 + 2 * q) * t_qr
        desc = (f"set-up; one FFT application ({nsrc_sample} vectors); one {n}x{r} QR; one rank-{r} H application; "
                f"scaled by the GPU step's counts")
    it_total = sum(i + 1 for i in iterations)            # residual evaluations, all sources
    h_total = sum(i + 1 for i in iterations)             # H applications (psi_0 = H psi0 plus one per update)
    step_s = t_setup + t_build + it_total * t_conv + h_total * t_h
    return {"value": converged / step_s, "unit": "solves/s", "cores": cores, "cpu_model": cpu_model(),
            "kind": "oracle", "sample": desc + f"; scipy.fft workers={cores}",
            "step_seconds_extrapolated": round(step_s, 2), "setup_s": round(t_setup, 2),
            "build_s_extrapolated": round(t_build, 2), "series_s_extrapolated": round(it_total * t_conv + h_total * t_h, 2)}


def hodlr_policy(n, h, freq, cmin, leaf_cols=1):
    """HODLR parameters for one instance: rank ~3 per wavelength across the grid (16-aligned, 32..256), one
    power iteration, and the deepest tree whose leaves keep at least `leaf_cols` grid columns."""
    import math
    nlam = n * h * freq / cmin
    r = int(min(256, max(32, 16 * math.ceil(3.0 * nlam / 16))))
    levels = 1
    while n % (1 << (levels + 1)) == 0 and (n >> (levels + 1)) >= leaf_cols:
        levels += 1
    return r, levels


def main_uneven(args):
    """64 instances of uneven size (128..512)^2, 5-30 Hz, 1-16 sources each, solved in one lockstep batch."""
    import numpy as np
    import torch

    from paper_2005_01372_amd import lsop, synth

    torch.cuda.init()
    ws = synth.model_uneven_batch(count=args.count)
    vels = [torch.as_tensor(w.vel, device="cuda") for w in ws]
    ops = [lsop.Operator(w.nx, w.nz, lsop.C64, max_vec=max(int(w.nsrc), 1)) for w in ws]
    pcs = []
    for w, op, v in zip(ws, ops, vels):
        op.set_problem(v, w.h, w.freq, w.c0)
        r, lv = hodlr_policy(w.nx, w.h, w.freq, float(w.vel.min()), args.leaf_cols)
        pcs.append(lsop.Preconditioner(op, lsop.PC_HODLR, rank=r, levels=lv, power_iters=1, seed=3,
                                       q_from_level=int(round(args.q_from_frac * lv))))
    batch = lsop.Batch(ops)
    batch.autotune()
    psis = [torch.empty((w.nsrc, w.nx, w.nz), dtype=torch.complex64, device="cuda") for w in ws]
    phase = {"build": 0.0, "series": 0.0}

    def step(streams=args.build_streams):
        rhss = []
        for w, op, v in zip(ws, ops, vels):
            op.set_problem(v, w.h, w.freq, w.c0)
            rhss.append(op.incident(w.src_i, w.src_j))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lsop.build_batch(pcs, streams=streams)
        t1 = time.perf_counter()
        _, res = batch.solve(pcs, rhss, psis=psis, tol=args.tol, max_iter=args.max_iter, use_graph=True)
        phase["build"] += t1 - t0
        phase["series"] += time.perf_counter() - t1
        return res

    for _ in range(args.warmup):
        step()
        print("[bench] warmup step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    phase.update(build=0.0, series=0.0)
    lsop.profile_reset()
    lsop.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
        print("[bench] timed step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lsop.profile_enable(False)
    by_fn = lsop.profile_read(by_kernel=True)
    lsop.profile_reset()
    step_s = (t1 - t0) / args.steps
    flat = [x for r in res for x in r]
    converged = sum(x.status == lsop.OK for x in flat)
    statuses = {}
    for x in flat:
        statuses[x.status_name] = statuses.get(x.status_name, 0) + 1
    build_s, series_s = phase["build"] / args.steps, phase["series"] / args.steps
    roof_src = "timed region"
    if args.build_streams > 1:
        # overlapping builds inflate every launch's event-timed duration by the other streams' time slices, so
        # the roofline comes from one more (untimed) step whose builds run one at a time
        lsop.profile_reset()
        lsop.profile_enable(True)
        step(streams=1)
        torch.cuda.synchronize()
        lsop.profile_enable(False)
        by_fn = lsop.profile_read(by_kernel=True)
        lsop.profile_reset()
        roof_src = "one extra untimed step with the builds on one stream"
    dom = max(by_fn, key=lambda k: by_fn[k]["ms"])
    roof = roofline_for(dom, by_fn[dom])
    ratio = load_traffic(dom)
    roof["traffic"] = None if ratio is None else round(ratio * roof["algorithmic_bytes_per_launch"])
    roof["measured_on"] = roof_src
    sizes = {}
    for w in ws:
        sizes[w.nx] = sizes.get(w.nx, 0) + 1
    line = {
        "metric": "LS solves/s, uneven batch to rel. residual 1e-6", "value": converged / step_s, "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"{len(ws)} instances, sides {sorted(sizes.items())}, h=5 m, 5-30 Hz, smoothed "
                               f"random 1500-4500 m/s, 1-16 top-row sources each, one HODLR H per instance "
                               f"(rank ~3 per wavelength, q=1) built {args.build_streams} at a time on separate streams, "
                               f"lockstep series in one batch with a captured "
                               f"graph per iteration, autotuned column tiles per shape group",
                   "instances": len(ws), "sources": len(flat), "shape_groups": batch.info()[0],
                   "leaf_cols": args.leaf_cols, "build_streams": args.build_streams, "q_from_frac": args.q_from_frac},
        "converged": converged, "statuses": statuses,
        "iterations": [min(x.iters for x in flat), max(x.iters for x in flat)],
        "build_s": round(build_s, 3), "series_s": round(series_s, 3),
        "preconditioner_bytes": sum(pc.info()[2] for pc in pcs), "roofline": roof,
        "kernels": {k: {"launches": v["launches"], "avg_ms": round(v["ms"] / v["launches"], 4)}
                    for k, v in sorted(by_fn.items(), key=lambda kv: -kv[1]["ms"])[:12]},
    }
    line["command"] = " ".join(["python", "bench.py"] + sys.argv[1:])
    print(json.dumps(line), flush=True)


def unet_cpu_baseline(samples=1):
    """The FP64 oracle network (numpy, as written) timed on forward + backward + loss of `samples` 128^2 samples
    (bf16 operand rounding on, as on the device)."""
    import numpy as np

    from oracle import unet as U
    net = U.UNet(U.he_init(4, 32, 4, 2, seed=0), 4, 32, 4, 2, bf16=True)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((samples, 128, 128, 4))
    t = rng.standard_normal((samples, 128, 128, 2))
    t0 = time.perf_counter()
    y = net.forward(x)
    _, dy = U.mse(y, t)
    net.backward(dy)
    dt = time.perf_counter() - t0
    return {"value": round(samples / dt, 4), "unit": "samples/s", "cores": _threads(), "cpu_model": cpu_model(),
            "kind": "oracle",
            "sample": f"{samples} training sample(s) at 128^2 (forward, loss, backward; the Adam update is "
                      f"negligible), oracle network in FP64 numpy with bf16 operand rounding"}


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count()


def train_warm_start(args, batch=16):
    """Warm-start network for ls1024 --init learned (untimed): 4 levels, 32 base channels, trained for
    --unet-train-steps Adam steps on solutions of --unet-models layered + salt models at 128^2 (10-20 Hz,
    32 top-row sources each) that the library's own HODLR series computed; sized for inference on the
    benchmark grid in chunks of `batch` sources."""
    import numpy as np
    import torch

    from paper_2005_01372_amd import lsop, synth

    n, nsrc = 128, 32
    net = lsop.UNet(4, 32, 4, 2, max_batch=batch, max_h=max(args.n, n), max_w=max(args.n, n))
    net.init_params(seed=0)
    rng = np.random.default_rng(1000)
    X, T = [], []
    for m in range(args.unet_models):
        w = synth.model_layered_salt(n=n, h=10.0, freq=float(rng.uniform(10.0, 20.0)), seed=1000 + m, nsrc=nsrc)
        op = lsop.Operator(n, n, lsop.C64, max_vec=nsrc)
        op.set_problem(torch.as_tensor(w.vel, device="cuda"), w.h, w.freq, w.c0)
        pc = lsop.Preconditioner(op, lsop.PC_HODLR, rank=64, levels=4, power_iters=1, seed=m)
        pc.build()
        rhs = op.incident(w.src_i, w.src_j)
        psi, _ = lsop.series_solve(op, pc, rhs, tol=1e-6, max_iter=30)
        for c in range(0, nsrc, batch):
            x, sc = net.pack_inputs(op, rhs[c:c + batch])
            X.append(x)
            T.append(net.pack_target(op, psi[c:c + batch], rhs[c:c + batch], sc))
        del pc, op
    X, T = torch.cat(X), torch.cat(T)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    for _ in range(args.unet_train_steps):
        i = torch.randint(0, X.shape[0], (batch,), device="cuda", generator=gen)
        loss = net.train_step(X[i].contiguous(), T[i].contiguous(), 1e-3)
    print(f"[bench] warm-start network trained on {X.shape[0]} samples, last loss {loss:.4f}", file=sys.stderr,
          flush=True)
    del X, T
    torch.cuda.empty_cache()
    return net


def main_unet(args):
    """Warm-start network (4 levels, 32 base channels, bf16 MFMA, FP32 accumulation and master weights):
    solver-generated training data at 128^2, timed training steps, then the warm start inside the series at
    256^2 and 512^2 (init "best": the candidate or H psi0, whichever has the smaller true residual)."""
    import numpy as np
    import torch

    from paper_2005_01372_amd import lsop, synth

    torch.cuda.init()
    if args.copy_probe:
        a = torch.ones(1 << 27, dtype=torch.complex64, device="cuda")   # 1 GiB
        torch.empty_like(a).copy_(a)
        torch.cuda.synchronize()
        del a
    n, nsrc, bs = 128, 32, args.unet_batch
    net = lsop.UNet(4, 32, 4, 2, max_batch=max(bs, nsrc, 16), max_h=512, max_w=512)
    net.init_params(seed=0)
    # training data: config-2-style layered + salt models at 128^2, 10-20 Hz, solved by the series
    rng = np.random.default_rng(1000)
    X, T, gen_solves = [], [], 0
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for m in range(args.unet_models):
        w = synth.model_layered_salt(n=n, h=10.0, freq=float(rng.uniform(10.0, 20.0)), seed=1000 + m, nsrc=nsrc)
        op = lsop.Operator(n, n, lsop.C64, max_vec=nsrc)
        op.set_problem(torch.as_tensor(w.vel, device="cuda"), w.h, w.freq, w.c0)
        pc = lsop.Preconditioner(op, lsop.PC_HODLR, rank=64, levels=4, power_iters=1, seed=m)
        pc.build()
        rhs = op.incident(w.src_i, w.src_j)
        psi, res = lsop.series_solve(op, pc, rhs, tol=1e-6, max_iter=30)
        gen_solves += sum(r.status == lsop.OK for r in res)
        x, sc = net.pack_inputs(op, rhs)
        X.append(x)
        T.append(net.pack_target(op, psi, rhs, sc))
        del pc, op
    X, T = torch.cat(X), torch.cat(T)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - g0
    print(f"[bench] {X.shape[0]} training samples generated in {gen_s:.1f} s", file=sys.stderr, flush=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    batches = [torch.randint(0, X.shape[0], (bs,), device="cuda", generator=gen)
               for _ in range(args.warmup + args.steps)]
    xb = [X[i].contiguous() for i in batches]
    tb = [T[i].contiguous() for i in batches]
    losses = []
    for s in range(args.warmup):
        losses.append(net.train_step(xb[s], tb[s], 1e-3))
    torch.cuda.synchronize()
    lsop.profile_reset()
    lsop.profile_enable(True)
    t0 = time.perf_counter()
    for s in range(args.warmup, args.warmup + args.steps):
        losses.append(net.train_step(xb[s], tb[s], 1e-3))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lsop.profile_enable(False)
    by_fn = lsop.profile_read(by_kernel=True)
    lsop.profile_reset()
    step_s = (t1 - t0) / args.steps
    print(f"[bench] {args.steps} timed training steps done", file=sys.stderr, flush=True)
    if args.dump_profile:
        with open(args.dump_profile, "w") as f:
            json.dump({"steps": args.steps, "warmup": args.warmup, "kernels": by_fn}, f, indent=1)
    dom = max(by_fn, key=lambda k: by_fn[k]["ms"])
    roof = roofline_for(dom, by_fn[dom])
    ratio = load_traffic(dom, "pmc_traffic_unet.json")
    roof["traffic"] = None if ratio is None else round(ratio * roof["algorithmic_bytes_per_launch"])
    conv_flops = sum(v["flops"] for k, v in by_fn.items() if k.startswith("k_conv"))
    training = None
    if args.unet_epochs > 0:
        nsamp, last = X.shape[0], float("nan")
        g2 = torch.Generator(device="cuda")
        g2.manual_seed(1)
        torch.cuda.synchronize()
        e0 = time.perf_counter()
        for _ in range(args.unet_epochs):
            perm = torch.randperm(nsamp, device="cuda", generator=g2)
            for s in range(nsamp // bs):
                i = perm[s * bs:(s + 1) * bs]
                last = net.train_step(X[i].contiguous(), T[i].contiguous(), 1e-3)
        torch.cuda.synchronize()
        e1 = time.perf_counter()
        # held-out models (seeds never trained on): relative error of the warm start, of psi0 and of zero
        errs, errs0 = [], []
        for m in range(2):
            w = synth.model_layered_salt(n=n, h=10.0, freq=15.0, seed=5001 + m, nsrc=nsrc)
            op = lsop.Operator(n, n, lsop.C64, max_vec=nsrc)
            op.set_problem(torch.as_tensor(w.vel, device="cuda"), w.h, w.freq, w.c0)
            pc = lsop.Preconditioner(op, lsop.PC_HODLR, rank=64, levels=4, power_iters=1, seed=m)
            pc.build()
            rhs = op.incident(w.src_i, w.src_j)
            psi, _ = lsop.series_solve(op, pc, rhs, tol=1e-6, max_iter=30)
            phi0 = net.warm_start(op, rhs)
            nrm = torch.linalg.vector_norm(psi.reshape(nsrc, -1), dim=1)
            errs += (torch.linalg.vector_norm((phi0 - psi).reshape(nsrc, -1), dim=1) / nrm).tolist()
            errs0 += (torch.linalg.vector_norm((rhs - psi).reshape(nsrc, -1), dim=1) / nrm).tolist()
            del pc, op
        training = {"epochs": args.unet_epochs, "samples": nsamp, "steps": args.unet_epochs * (nsamp // bs),
                    "seconds": round(e1 - e0, 2), "last_loss": round(last, 4),
                    "heldout_rel_err_warm_start": [round(min(errs), 3), round(float(np.median(errs)), 3),
                                                   round(max(errs), 3)],
                    "heldout_rel_err_psi0": [round(min(errs0), 3), round(float(np.median(errs0)), 3),
                                             round(max(errs0), 3)],
                    "heldout_rel_err_zero": 1.0,
                    "note": "min / median / max over 64 held-out sources (2 models x 32) at 128^2, 15 Hz"}
        print(f"[bench] {args.unet_epochs} epochs in {e1 - e0:.1f} s, held-out error {np.median(errs):.3f}",
              file=sys.stderr, flush=True)
    # warm start inside the series at 256^2 and 512^2 (16 sources each)
    evals = []
    for m, (side, rank, lv) in enumerate(() if args.unet_no_eval else ((256, 96, 6), (512, 160, 7))):
        w = synth.model_layered_salt(n=side, h=10.0, freq=15.0, seed=77 + m, nsrc=16)
        op = lsop.Operator(side, side, lsop.C64, max_vec=16)
        op.set_problem(torch.as_tensor(w.vel, device="cuda"), w.h, w.freq, w.c0)
        rhs = op.incident(w.src_i, w.src_j)
        pc = lsop.Preconditioner(op, lsop.PC_HODLR, rank=rank, levels=lv, power_iters=1, seed=5)
        pc.build()
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        _, rb = lsop.series_solve(op, pc, rhs, tol=1e-6, max_iter=40)
        torch.cuda.synchronize()
        a1 = time.perf_counter()
        phi0 = net.warm_start(op, rhs)
        torch.cuda.synchronize()
        a2 = time.perf_counter()
        _, rw = lsop.series_solve(op, pc, rhs, psi=phi0, tol=1e-6, max_iter=40, init="best")
        torch.cuda.synchronize()
        a3 = time.perf_counter()
        evals.append({"side": side, "rank": rank, "levels": lv,
                      "series_ms": round((a1 - a0) * 1e3, 2), "warm_start_ms": round((a2 - a1) * 1e3, 2),
                      "warm_series_ms": round((a3 - a2) * 1e3, 2),
                      "iterations": sum(r.iters for r in rb), "warm_iterations": sum(r.iters for r in rw),
                      "converged": sum(r.status == lsop.OK for r in rb),
                      "warm_converged": sum(r.status == lsop.OK for r in rw)})
        del pc, op
    line = {
        "metric": "warm-start network training samples/s (128^2, batch %d)" % bs, "value": bs / step_s,
        "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"4-level U-Net, 32 base channels, bf16 matrix-core operands with FP32 accumulation "
                               f"and FP32 master weights (Adam); inputs (c/c0 - 1, psi0 / rms, k0 h) at 128^2; "
                               f"training data solved by the library's own series on {args.unet_models} "
                               f"layered + salt models x {nsrc} sources; warm start applied inside the series at "
                               f"256^2 and 512^2", "batch": bs, "side": n},
        "conv_tflops": round(conv_flops / (step_s * args.steps) / 1e12, 2),
        "data_generation": {"solves": gen_solves, "seconds": round(gen_s, 2),
                            "solves_per_s": round(gen_solves / gen_s, 1)},
        "loss_first_last": [round(losses[0], 4), round(losses[-1], 4)], "training": training,
        "warm_start_eval": evals,
        "roofline": roof,
        "kernels": {k: {"launches": v["launches"], "avg_ms": round(v["ms"] / v["launches"], 4)}
                    for k, v in sorted(by_fn.items(), key=lambda kv: -kv[1]["ms"])[:12]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = unet_cpu_baseline()
    line["command"] = " ".join(["python", "bench.py"] + sys.argv[1:])
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "lsop runs on one GPU: sharding the sources or the grid over several GPUs is "
                                   "designed but not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "uneven":
        return main_uneven(args)
    if args.workload == "unet":
        return main_unet(args)
    import numpy as np
    import torch

    from paper_2005_01372_amd import lsop, synth

    torch.cuda.init()
    if args.copy_probe:
        a = torch.ones(1 << 27, dtype=torch.complex64, device="cuda")   # 1 GiB
        torch.empty_like(a).copy_(a)
        torch.cuda.synchronize()
        del a

    copy_gbps = measure_copy_gbps()
    w = synth.model_random_ellipses(n=args.n, nsrc=args.nsrc)
    vel = torch.as_tensor(w.vel, device="cuda")
    dt = {"c64": lsop.C64, "c128": lsop.C128, "mixed": lsop.MIXED}[args.dtype]
    net = train_warm_start(args) if args.init == "learned" else None

    def make(dtype):
        o = lsop.Operator(w.nx, w.nz, dtype, max_vec=max(args.nsrc, 64))
        if args.pc == "hodlr":
            p = lsop.Preconditioner(o, lsop.PC_HODLR, rank=args.rank, levels=args.levels,
                                    power_iters=args.power_iters, seed=3, q_from_level=args.q_from_level)
        else:
            p = lsop.Preconditioner(o, lsop.PC_LOWRANK, rank=args.rank, power_iters=args.power_iters, seed=3)
        o.set_problem(vel, w.h, w.freq, w.c0)
        o.autotune(w.nsrc)
        return o, p

    op, pc = make(dt)
    psi = torch.empty((w.nsrc, w.nx, w.nz), dtype=op.vec_dtype, device="cuda")
    phase = {"build": 0.0, "series": 0.0}

    def step(o=op, p=pc, out=psi, learned=net):
        o.set_problem(vel, w.h, w.freq, w.c0)
        rhs = o.incident(w.src_i, w.src_j)
        t0 = time.perf_counter()
        p.build(None)                       # synchronises its stream
        t1 = time.perf_counter()
        init = "h_rhs"
        if learned is not None:             # the network's field as candidate start, chunk by chunk
            for c in range(0, w.nsrc, 16):
                learned.warm_start(o, rhs[c:c + 16], out=out[c:c + 16])
            init = "best"
        if args.solver == "gmres":
            _, info = lsop.gmres_solve(o, p, rhs, psi=out, tol=args.tol, restart=args.restart,
                                       max_iter=args.max_iter, init="user" if learned is not None else "h_rhs")
        else:
            _, info = lsop.series_solve(o, p, rhs, psi=out, tol=args.tol, max_iter=args.max_iter, init=init)
        phase["build"] += t1 - t0
        phase["series"] += time.perf_counter() - t1
        return info

    for _ in range(args.warmup):
        step()
        print(f"[bench] warmup step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    phase.update(build=0.0, series=0.0)
    lsop.profile_reset()
    lsop.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = step()
        print(f"[bench] timed step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lsop.profile_enable(False)
    by_use = lsop.profile_read()
    by_fn = lsop.profile_read(by_kernel=True)
    lsop.profile_reset()
    if args.dump_profile:
        with open(args.dump_profile, "w") as f:
            json.dump({"steps": args.steps, "warmup": args.warmup, "kernels": by_fn}, f, indent=1)
    step_s = (t1 - t0) / args.steps
    converged = sum(i.status == lsop.OK for i in info)
    statuses = {}
    for i in info:
        statuses[i.status_name] = statuses.get(i.status_name, 0) + 1
    iters = [i.iters for i in info]
    col_tile, pc_bytes = op.info().col_tile, pc.info()[2]
    op_lx, op_lz = op.info().lx, op.info().lz

    # the plain FP64 series on the same GPU (untimed): its own solves/s, and every timed solution's relative
    # error against it
    fp64 = None
    if args.dtype != "c128" and not args.no_fp64_compare:
        del pc
        torch.cuda.empty_cache()
        op64, pc64 = make(lsop.C128)
        psi64 = torch.empty((w.nsrc, w.nx, w.nz), dtype=torch.complex128, device="cuda")
        phase64 = dict(phase)
        phase.update(build=0.0, series=0.0)
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        tol_run = args.tol
        args.tol = min(args.tol, 1e-10)          # the reference is solved well below the timed target
        info64 = step(op64, pc64, psi64, None)
        args.tol = tol_run
        torch.cuda.synchronize()
        f1 = time.perf_counter()
        ok64 = sum(i.status == lsop.OK for i in info64)
        err = (torch.linalg.vector_norm((psi.to(torch.complex128) - psi64).reshape(w.nsrc, -1), dim=1)
               / torch.linalg.vector_norm(psi64.reshape(w.nsrc, -1), dim=1)).cpu().numpy()
        fp64 = {"solves_per_s": round(ok64 / (f1 - f0), 2), "converged": ok64,
                "iterations": [min(i.iters for i in info64), max(i.iters for i in info64)],
                "build_s": round(phase["build"], 3), "series_s": round(phase["series"], 3),
                "rel_err_vs_fp64": {"max": float(err.max()), "median": float(np.median(err)),
                                    "min": float(err.min())},
                "tol": min(args.tol, 1e-10),
                "timing": "one untimed complex-FP64 step after the timed region (same workload and preconditioner "
                          "parameters; series solved to the tighter of the timed target and 1e-10, so that the "
                          "errors above are those of the timed solutions)"}
        phase.update(phase64)
        del pc64, op64, psi64
        torch.cuda.empty_cache()
        print("[bench] fp64 comparison done", file=sys.stderr, flush=True)

    # dominant kernel function: largest share of event-timed GPU time in the timed region
    dom = max(by_fn, key=lambda k: by_fn[k]["ms"])
    roof = roofline_for(dom, by_fn[dom])
    ratio = load_traffic(dom)
    roof["traffic"] = None if ratio is None else round(ratio * roof["algorithmic_bytes_per_launch"])
    total_ms = sum(v["ms"] for v in by_fn.values())
    kernels = {k: {"launches": v["launches"], "avg_ms": round(v["ms"] / v["launches"], 4),
                   "share": round(v["ms"] / total_ms, 4)} for k, v in sorted(by_fn.items(), key=lambda kv: -kv[1]["ms"])}
    uses = {k: round(v["ms"] / args.steps, 2) for k, v in sorted(by_use.items(), key=lambda kv: -kv[1]["ms"])}

    # FFT-convolution throughput of the LS operator inside the timed region: its three passes together
    passes = [k for k in ("lsop_rows_fwd", "lsop_cols", "lsop_rows_inv") if k in by_use]
    fft_bytes = sum(by_use[k]["bytes"] for k in passes)
    fft_ms = sum(by_use[k]["ms"] for k in passes)
    fft_gbps = fft_bytes / (fft_ms / 1e3) / 1e9 if fft_ms > 0 else None
    vec_applies = by_use["lsop_cols"]["items"] if "lsop_cols" in by_use else 0
    # the same passes against the compulsory bytes (each vector read and written once: 2 N^2 e) and the
    # counter-measured bytes (each pass's algorithmic bytes times its kernel's measured ratio, when the committed
    # counters were taken on the current sources)
    fft_conv = None
    if fft_ms > 0:
        e = {"c64": 8, "c128": 16}.get(args.dtype)
        t = "float" if args.dtype == "c64" else "double"
        names = {"lsop_rows_fwd": f"k_rows_fwd<{t}, {op_lz}>", "lsop_cols": f"k_cols<{t}, {op_lx}, {col_tile}>",
                 "lsop_rows_inv": f"k_rows_inv<{t}, {op_lz}>"}
        ratios = {k: load_traffic(names[k]) for k in passes} if e else {}
        traffic = sum(ratios[k] * by_use[k]["bytes"] for k in passes) if e and all(
            ratios[k] is not None for k in passes) else None
        compulsory = 2.0 * w.nx * w.nz * e * vec_applies if e else None
        fft_conv = {"kernels": [names[k] for k in passes], "vector_applications": vec_applies,
                    "ms": round(fft_ms, 3), "algorithmic_GB": round(fft_bytes / 1e9, 3),
                    "traffic_GB": None if traffic is None else round(traffic / 1e9, 3),
                    "compulsory_GB": None if compulsory is None else round(compulsory / 1e9, 3),
                    "compulsory_GBps": None if compulsory is None else round(compulsory / (fft_ms / 1e3) / 1e9, 1)}
    growth = [(i.rel_residual / i.rel_residual0) ** (1.0 / i.iters) for i in info if i.iters > 0
              and i.rel_residual0 > 0 and np.isfinite(i.rel_residual)]
    if args.pc == "hodlr":
        pcdesc = f"HODLR H, {args.levels} levels, rank {args.rank}, q={args.power_iters}" + \
                 (f" on levels >= {args.q_from_level}" if args.q_from_level else "")
    else:
        pcdesc = f"low-rank H rank {args.rank} (q={args.power_iters})"
    build_s, series_s = phase["build"] / args.steps, phase["series"] / args.steps
    line = {
        "metric": METRIC, "value": converged / step_s, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(step_s * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"smooth random 1500-5000 m/s + 6 ellipses, {w.nx}x{w.nz}, h={w.h} m, {w.freq} Hz, "
                               f"c0={w.c0} m/s, {w.nsrc} top-row sources, {pcdesc}, "
                               f"{'series' if args.solver == 'series' else f'GMRES({args.restart})'} to rel. residual {args.tol}, "
                               f"cap {args.max_iter}",
                   "grid": [w.nx, w.nz], "sources": w.nsrc, "preconditioner": args.pc, "rank": args.rank,
                   "levels": args.levels if args.pc == "hodlr" else None, "power_iters": args.power_iters,
                   "q_from_level": args.q_from_level if args.pc == "hodlr" else None,
                   "tol": args.tol, "init": args.init, "solver": args.solver,
                   "restart": args.restart if args.solver == "gmres" else None},
        "converged": converged, "statuses": statuses, "iterations": [min(iters), max(iters)],
        "build_s": round(build_s, 3), "series_s": round(series_s, 3),
        "solves_per_s_series_only": round(converged / series_s, 1) if series_s > 0 else None,
        "residual_growth_per_iter": round(float(np.median(growth)), 3) if growth else None,
        "fft_conv_GBps": None if fft_gbps is None else round(fft_gbps, 1),
        "fft_conv_frac_of_peak": None if fft_gbps is None else round(fft_gbps / HBM_PEAK_GBPS, 4),
        "operator_applications_per_s": round(vec_applies / (fft_ms / 1e3), 1) if fft_ms > 0 else None,
        "col_tile": col_tile, "preconditioner_bytes": pc_bytes,
        "hbm_copy_GBps_measured": round(copy_gbps, 1),
        "fft_conv_frac_of_measured_copy": None if fft_gbps is None else round(fft_gbps / copy_gbps, 4),
        "fft_conv": fft_conv,
        "fp64_series": fp64,
        "roofline": roof, "kernels": kernels, "ms_per_step_by_use": uses,
    }
    roof["peak_measured_copy"] = round(copy_gbps, 1) if roof.get("unit") == "GB/s" else None
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args, iters, converged, args.cpu_sources)
    line["command"] = " ".join(["python", "bench.py"] + sys.argv[1:])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
