"""Benchmark of the GPAIR hot path on one MI355X.

A step is one iteration of differentiable iterative reconstruction at the
paper-scale workload (256 x 256 x 128 = 8,388,608 Gaussian kernels at 0.1 mm,
1024 sensors on a 40 mm hemisphere, 4096 samples at 40 MHz, per-kernel sigma
and amplitude both learned):
    forward y = A(x; sigma)  ->  residual delta = (y - b)/||b||^2 and norms
    ->  adjoint (dL/dA, dL/dsigma)  ->  Adam on A (A >= 0) and on sigma (clamped).
Inputs are synthetic (a seeded vessel-tree phantom; b = A(x_true) computed by the
same forward operator) and resident in HBM before the timed region starts.

Metric: fwd+adjoint G-evals/s = 2 * M * N_d * steps / elapsed / 1e9 (kernel-sensor
pair evaluations, each operator once per step).  After the timed steps, the
second half of the metric: wall-clock to relative data residual 1e-2 on a
held-out phantom with 1 % noise, plain zero-start IR against the learned warm
start.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak (published)
PEAK_FP64_TFLOPS = 78.6    # MI355X FP64 vector peak (published)
CUS, CLOCK_HZ = 256, 2.4e9  # MI355X compute units and peak engine clock
# Algorithmic FLOPs (direct definition, exp counted as one): per in-window tap
# and per kernel-sensor pair.
FLOP_TAP_FWD = 7      # d, d^2, scale, exp, * d, * A/(2r), accumulate
FLOP_TAP_ADJ = 10     # d, d^2, scale, exp, * d, * delta, acc A, * d^2, acc sigma, (d^3 reuse)
FLOP_PAIR = 25        # distance (3 sub, 3 fma, sqrt), window bounds, 1/(2r), tap setup
FLOP_TAP_CENTRES = 5  # the centre gradient's extra sums per tap (delta e, delta u^2 e)
FLOP_PAIR_CENTRES = 16  # its per-pair combination along (c - s)/r

# HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE (dense amplitudes,
# scaled by the counts a 256 MiB device copy gives: fetch x2.0, write x1.0), keyed
# by the sha256 prefix of the kernel source they were measured on; when the source
# differs, the figure no longer applies and `traffic` is null.
# wave64 VALU instructions issued per CU per clock (2.4 GHz) by each operator
# kernel: rocprofv3 SQ_INSTS_VALU / (duration x 256 CUs x 2.4 GHz), keyed like
# MEASURED_TRAFFIC.
MEASURED_VALU = {
    "017f0377afb88363": {"forward_kernel": 1.350, "adjoint_kernel": 1.431},
}

MEASURED_TRAFFIC = {
    "017f0377afb88363": {"forward_kernel": 2.330e9, "adjoint_kernel": 0.7538e9},
}


# The same for the anisotropic kernels (aniso.hip).
MEASURED_TRAFFIC_ANISO = {
    "cd32d60d0335da76": {"aniso_forward_kernel": 2.263e+09, "aniso_adjoint_kernel": 8.776e+08},
}

# The same for the ASSA kernels (assa.hip).
MEASURED_TRAFFIC_ASSA = {
    "7c3906cc142edcf9": {"assa_forward_kernel": 2.843e9, "assa_adjoint_kernel": 0.8427e9},
}


# Sources each kernel file's code is built from (the float32 filter's block
# constants live in filter.h, shared by the direct and anisotropic kernels).
KERNEL_SOURCES = {"operators.hip": ("operators.hip", "filter.h"),
                  "aniso.hip": ("aniso.hip", "filter.h")}


def kernel_source_hash(name="operators.hip"):
    import hashlib
    h = hashlib.sha256()
    for part in KERNEL_SOURCES.get(name, (name,)):
        with open(os.path.join(ROOT, "paper_2602_03893_amd", "csrc", part), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def measure_peaks():
    """Measured issue rates of the vector instructions the operators use
    (gpair_peak_probe): wave64 instructions per CU per clock at the 2.4 GHz
    peak clock, and the FLOP rate they give (FMA = 2 FLOP per lane)."""
    from paper_2602_03893_amd import api
    out = {}
    for kind, name in api.PEAK_PROBES.items():
        rate, ms = api.peak_probe(kind, blocks=8192, iters=1024)
        per_clk = rate / (CUS * CLOCK_HZ)
        e = {"wave_instr_per_s": rate, "per_cu_per_clk": per_clk, "kernel_ms": ms}
        if "fma" in name:
            e["tflops"] = rate * 64 * 2 / 1e12
        else:
            e["lane_ops_per_s"] = rate * 64
        out[name] = e
    return out


def cpu_baseline(w, centres, sensors, A, sigma_val, rows=192, stride=6):
    """The float64 oracle on a bounded sample of the same workload: the forward
    for `rows` sensors (all kernels) and the adjoint for every `stride`-th
    kernel (all sensors).  Returns the rate in G pair-evaluations/s."""
    import numpy as np
    from oracle import ops as O
    from paper_2602_03893_amd import inputs as I
    g = O.Geometry(centres, sensors, w.n_samples, w.dt, w.t0, w.c_sound, w.n_sigma)
    M, Nd = w.n_kernels, w.n_sensors
    sig = np.full(M, sigma_val)
    pick = np.linspace(0, Nd - 1, rows).astype(int)
    t = time.perf_counter()
    O.forward(g.subset_sensors(pick), A, sig)
    t_fwd = time.perf_counter() - t
    ks = np.arange(0, M, stride)
    delta = I.standard_normal((Nd, w.n_samples), seed=99, dtype=np.float64)
    t = time.perf_counter()
    O.adjoint(g.subset_kernels(ks), A[ks], sig[ks], delta)
    t_adj = time.perf_counter() - t
    pairs_fwd = M * rows
    pairs_adj = len(ks) * Nd
    rate = (pairs_fwd + pairs_adj) / (t_fwd + t_adj) / 1e9
    return {"value": rate, "unit": "G-evals/s", "cores": O.num_threads(), "kind": "oracle",
            "cpu_model": host_cpu_model(),
            "sample": (f"float64 oracle: forward on {rows} of {Nd} sensors x {M} kernels "
                       f"({t_fwd:.2f} s) + adjoint (A and sigma) on {len(ks)} kernels x {Nd} "
                       f"sensors ({t_adj:.2f} s); rate = pairs / time")}


# Time to the relative data residual 1e-2 at the paper-scale shape (the
# second half of the headline metric): one held-out vessel phantom (seed
# 100000, outside the training and test seeds) with 1 % noise, Adam on A and
# sigma as in the step above, from the zero start and from the learned warm
# start; a start that does not reach the tolerance within the cap is
# reported as not reached with its final residual.
TTR_SEED, TTR_TOL, TTR_CAP = 100000, 1e-2, 4000
# The paper's full reconstructions in vivo (8.4 M kernels, 1024 elements,
# RTX 5090, ASSA operators, iteration count not stated): context only.
PAPER_IR_S = (0.79, 0.82)


def _ttr_leg(r):
    return {"reached": r["reached_tol"], "iters": r["iters"],
            "seconds": r["time_to_tol_s"], "final_rho": r["final_rho"],
            "seconds_to_1.05_rho_true": r["time_to_1.05_rho_true_s"],
            "start_rho": r["start_rho"], "start_seconds": r["start_s"],
            "fell_back": r["fell_back"], "image_rel_l2": r["x_rel_l2"]}


def _ttr_problem(dev):
    import numpy as np
    from paper_2602_03893_amd import warmstart as WS
    problem = WS.Problem(device=dev)
    problem.kappa = WS.TRAINED_KAPPA
    params = np.load(os.path.join(ROOT, "paper_2602_03893_amd", "weights", "unet4_c4.npy"),
                     allow_pickle=False)
    return problem, params


def time_to_rho(dev, cap=TTR_CAP):
    from paper_2602_03893_amd import warmstart as WS
    t = time.perf_counter()
    problem, params = _ttr_problem(dev)
    t_plan = time.perf_counter() - t
    row = WS.evaluate(problem, params, [TTR_SEED], max_iters=cap, tol=TTR_TOL, log=log,
                      starts=("zero", "learned"))[0]
    leg = _ttr_leg
    return {"tol": TTR_TOL, "cap_iters": cap,
            "adam": {"lr_A": WS.EVAL_LR_A, "lr_sigma_rel": WS.EVAL_LR_SIGMA_REL, "beta1": 0.9,
                     "beta2": WS.EVAL_BETA2},
            "phantom": f"vessel tree seed {TTR_SEED} (held out), 1 % noise",
            "rho_x_true": row["rho_x_true"], "zero_start": leg(row["zero"]),
            "learned_start": leg(row["learned"]), "plans_s": t_plan,
            "paper_context": {"gpu": "RTX 5090", "full_ir_in_vivo_s": list(PAPER_IR_S),
                              "operators": "ASSA", "iterations": "not stated"}}


def bench_c5(args):
    """Time to rho <= 1e-2 on held-out phantoms (seeds c5_first, c5_first + 1,
    ...) from each start, with per-phantom rows and medians.  A run that does
    not reach the tolerance within the cap is censored: it counts as not
    reached, with its final rho, and a median is given only when more than
    half of the runs reached the tolerance."""
    import numpy as np
    import torch
    from paper_2602_03893_amd import warmstart as WS
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    problem, params = _ttr_problem(dev)
    starts = tuple(args.ttr_starts.split(","))
    seeds = list(range(args.c5_first, args.c5_first + args.c5))
    rows = WS.evaluate(problem, params, seeds, max_iters=args.ttr_cap, tol=TTR_TOL, log=log,
                       starts=starts)
    summary = {}
    for st in starts:
        legs = [r[st] for r in rows]
        t = sorted(x["time_to_tol_s"] for x in legs if x["reached_tol"])
        t105 = sorted(x["time_to_1.05_rho_true_s"] for x in legs
                      if x["time_to_1.05_rho_true_s"] is not None)
        n = len(legs)
        summary[st] = {
            "runs": n, "reached": len(t),
            "median_seconds": float(np.median(t + [np.inf] * (n - len(t)))) if 2 * len(t) > n else None,
            "median_seconds_to_1.05_rho_true": (float(np.median(t105 + [np.inf] * (n - len(t105))))
                                                if 2 * len(t105) > n else None),
            "final_rho_not_reached": [x["final_rho"] for x in legs if not x["reached_tol"]],
            "median_image_rel_l2": float(np.median([x["x_rel_l2"] for x in legs]))}
    print(json.dumps({"metric": "seconds to relative data residual <= 1e-2", "tol": TTR_TOL,
                      "cap_iters": args.ttr_cap,
                      "adam": {"lr_A": WS.EVAL_LR_A, "lr_sigma_rel": WS.EVAL_LR_SIGMA_REL, "beta1": 0.9,
                     "beta2": WS.EVAL_BETA2},
                      "phantoms": f"vessel trees, seeds {seeds[0]}.."
                      f"{seeds[-1]} (held out), 1 % noise", "summary": summary,
                      "rows": [{"seed": r["seed"], "rho_x_true": r["rho_x_true"],
                                **{st: _ttr_leg(r[st]) for st in starts}} for r in rows]}),
          flush=True)


PEAK_BF16_TFLOPS = 2500.0  # MI355X dense bf16 matrix peak (published)

# ASSA operators: algorithmic FLOPs per kernel-sensor pair (distance 7 with the
# square root as one, snapped index 3, x / r 1, add or multiply-accumulate 2)
# and per decimated output sample (the 2K + 1 taps of h, multiply-add each).
FLOP_PAIR_ASSA = 13
# The paper's ASSA operator times at this workload (RTX 5090): context only.
PAPER_ASSA_MS = {"forward": 37.41, "adjoint": 4.99}


def cpu_baseline_assa(w, centres, sensors, x, sigma, rows=768, stride=2):
    """The float64 ASSA oracle on a bounded sample of the workload: the
    forward for `rows` sensors (all kernels), the back-projection for every
    `stride`-th kernel (all sensors)."""
    import numpy as np
    from oracle import assa as S
    from oracle import ops as O
    from paper_2602_03893_amd import inputs as I
    g = O.Geometry(centres, sensors, w.n_samples, w.dt, w.t0, w.c_sound, w.n_sigma)
    M, Nd = w.n_kernels, w.n_sensors
    pick = np.linspace(0, Nd - 1, rows).astype(int)
    t = time.perf_counter()
    S.forward(g.subset_sensors(pick), x.astype(np.float64), sigma)
    t_fwd = time.perf_counter() - t
    ks = np.arange(0, M, stride)
    delta = I.standard_normal((Nd, w.n_samples), seed=99, dtype=np.float64)
    t = time.perf_counter()
    S.adjoint(g.subset_kernels(ks), sigma, delta)
    t_adj = time.perf_counter() - t
    rate = (M * rows + len(ks) * Nd) / (t_fwd + t_adj) / 1e9
    return {"value": rate, "unit": "G-evals/s", "cores": O.num_threads(), "kind": "oracle",
            "cpu_model": host_cpu_model(),
            "sample": (f"float64 ASSA oracle: forward on {rows} of {Nd} sensors x {M} kernels "
                       f"({t_fwd:.2f} s) + back-projection on {len(ks)} kernels x {Nd} sensors "
                       f"({t_adj:.2f} s); rate = pairs / time")}


# Full objective (--objective): the regulariser's weight and balance, the
# warm-restart schedule.  The paper gives no values; these make the VCR term a
# few percent of the normalised data term at the start and restart every 16
# steps.
OBJ_LAMBDA, OBJ_BETA, OBJ_EPS = 1e-7, 0.5, 1e-8
OBJ_T0, OBJ_TMULT, OBJ_LR_MIN = 16, 2, 1e-4
# VCR traffic per voxel (algorithmic): terms pass reads x (4 B) and writes nine
# float32 terms (36 B); gradient pass reads the nine terms (36 B) and reads and
# writes the gradient (8 B).
VCR_BYTES_PER_VOXEL = 4 + 36 + 36 + 8
PEAK_HBM_GBS = 8000.0


class Objective:
    """NPC + VCR + CAWR around a step's operators (Algorithm 2), timing the
    regulariser with events on the library's stream."""

    def __init__(self, w, dev):
        import torch
        from paper_2602_03893_amd import vcr
        self.w = w
        self.shape = (w.grid[2], w.grid[1], w.grid[0])
        self.z = torch.zeros(w.n_kernels, dtype=torch.float32, device=dev)
        nbytes = ctypes_vcr_bytes(*w.grid)
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.vcr = vcr
        self.ev = []

    def x_from_z(self, x):
        from paper_2602_03893_amd import npc_map
        npc_map(self.z, out=x)

    def add_reg_and_chain(self, x, gx):
        import torch
        from paper_2602_03893_amd import npc_grad
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        self.vcr(x.view(self.shape), OBJ_BETA, OBJ_EPS, OBJ_LAMBDA, grad=gx.view(self.shape),
                 want_value=False, work=self.work)
        e1.record()
        self.ev.append((e0, e1))
        npc_grad(self.z, gx, out=gx)

    def lr(self, t, lr_max):
        from paper_2602_03893_amd import cawr_rate
        return cawr_rate(t - 1, OBJ_LR_MIN, lr_max, OBJ_T0, OBJ_TMULT)

    def vcr_ms(self):
        import numpy as np
        import torch
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in self.ev])) if self.ev else None


def ctypes_vcr_bytes(nx, ny, nz):
    import ctypes
    from paper_2602_03893_amd import _lib
    n = ctypes.c_size_t()
    _lib.check(_lib.gpair_vcr_workspace_size(nx, ny, nz, ctypes.byref(n)),
               "gpair_vcr_workspace_size")
    return int(n.value)


def objective_fields(obj, w):
    t = obj.vcr_ms()
    gbs = VCR_BYTES_PER_VOXEL * w.n_kernels / (t * 1e-3) / 1e9
    return {"objective": {"npc_eps": 1e-8, "vcr_lambda": OBJ_LAMBDA, "vcr_beta": OBJ_BETA,
                          "vcr_eps": OBJ_EPS, "cawr": {"T0": OBJ_T0, "Tmult": OBJ_TMULT,
                                                       "lr_min": OBJ_LR_MIN},
                          "vcr_ms": t, "vcr_GBs": gbs, "vcr_hbm_frac": gbs / PEAK_HBM_GBS}}


def bench_assa(args):
    """Paper-scale IR step with the ASSA operators (one shared sigma, the
    paper's own discretisation): forward -> residual -> back-projection ->
    Adam on A (A >= 0)."""
    import numpy as np
    import torch
    from paper_2602_03893_amd import Plan, adam_update, inputs as I

    w = I.WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    centres, sensors = I.geometry_arrays(w)
    t = time.perf_counter()
    plan = Plan(centres, sensors, w.n_samples, w.dt, w.c_sound, n_sigma=w.n_sigma,
                sigma_max=w.smax, device=dev)
    t_plan = time.perf_counter() - t
    sig = w.sigma
    grid = plan.assa_grid(sig)
    log(f"bench --assa: workload {w.name}, sigma {sig} m, grid {grid}, plan {t_plan:.2f} s")
    M, Nd, Nt = w.n_kernels, w.n_sensors, w.n_samples
    A_true_h = I.phantom(w)
    b = plan.assa_forward(torch.tensor(A_true_h, device=dev), sig).clone()
    A = torch.zeros(M, dtype=torch.float32, device=dev)
    mA, vA = torch.zeros_like(A), torch.zeros_like(A)
    y = torch.empty((Nd, Nt), dtype=torch.float32, device=dev)
    gA = torch.empty(M, dtype=torch.float32, device=dev)
    work = torch.empty(plan.assa_workspace_bytes(sig), dtype=torch.uint8, device=dev)
    scale = 1.0 / float(torch.sum(b.double() ** 2))
    state = {"t": 0}
    obj = Objective(w, dev) if args.objective else None

    def step():
        state["t"] += 1
        if obj:
            obj.x_from_z(A)
        plan.assa_forward(A, sig, out=y)
        plan.residual(y, b, scale=scale, delta=y)
        plan.assa_adjoint(sig, y, out=gA, work=work)
        if obj:
            obj.add_reg_and_chain(A, gA)
            adam_update(obj.z, gA, mA, vA, state["t"], obj.lr(state["t"], 1e-2))
        else:
            adam_update(A, gA, mA, vA, state["t"], 1e-2, lo=0.0)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    f_ms = float(np.mean(plan.kernel_times("assa_forward")))
    a_ms = float(np.mean(plan.kernel_times("assa_adjoint")))
    plan.set_timing(False)
    pairs = float(M) * Nd
    ms_step = 1e3 * elapsed / args.steps
    value = 2.0 * pairs * args.steps / elapsed / 1e9
    flop_fwd = FLOP_PAIR_ASSA * pairs + 2.0 * (2 * grid["K"] + 1) * Nd * Nt
    achieved = flop_fwd / (f_ms * 1e-3) / 1e12
    log(f"bench --assa: {ms_step:.2f} ms/step, forward kernel {f_ms:.2f} ms, back-projection "
        f"kernel {a_ms:.2f} ms, {value:.1f} G-evals/s")
    out = {
        "metric": ("fwd+adjoint G-evals/s (paper-scale IR step, ASSA operators"
                   + (", NPC + VCR + CAWR)" if obj else ")")),
        "value": value,
        "unit": "G-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 snapped index / int32 fixed-point impulses / f32 convolution and sums",
        "data": "synthetic (seeded vessel-tree phantom; b = ASSA forward of x_true)",
        "config": {"workload": "256x256x128 Gaussian kernels (0.1 mm), 1024 sensors on a "
                               "40 mm hemisphere, 4096 samples at 40 MHz, shared sigma "
                               f"{sig} m (alpha {grid['alpha']}, K {grid['K']}), Adam on A",
                   "kernels": M, "sensors": Nd, "samples": Nt, "parallelism": "single GPU"},
        "fwd_kernel_ms": f_ms,
        "adj_kernel_ms": a_ms,
        "paper_context": {"gpu": "RTX 5090", "fwd_ms": PAPER_ASSA_MS["forward"],
                          "adj_ms": PAPER_ASSA_MS["adjoint"]},
        "plan_s": t_plan,
        "roofline": {"bound": "alu", "kernel": "assa_forward_kernel", "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": MEASURED_TRAFFIC_ASSA.get(kernel_source_hash("assa.hip"), {})
                                                     .get("assa_forward_kernel"),
                     "kernel_source_sha256_16": kernel_source_hash("assa.hip")},
    }
    if obj:
        out.update(objective_fields(obj, w))
    if not args.no_cpu_baseline:
        log("bench --assa: timing the float64 ASSA oracle on a sample (cpu_baseline)")
        out["cpu_baseline"] = cpu_baseline_assa(w, centres, sensors, A_true_h, sig)
    print(json.dumps(out), flush=True)



# Anisotropic kernels: algorithmic FLOPs per kernel-sensor pair (float64
# distance 7 with the square root as one, quadratic form 12, sigma_n and the
# window 8, the pair's tap constants 8) and per in-window tap (forward 7,
# adjoint with the covariance gradient 10, as the isotropic operators).
FLOP_PAIR_ANISO = 35


def bench_aniso(args):
    """Paper-scale IR step with anisotropic kernels (learnable anisotropic
    Gaussians): forward -> residual -> adjoint (A and the six covariance
    gradients) -> Adam on A (A >= 0), the covariances held fixed (the
    operators are what is timed; a covariance update needs a positive-definite
    parameterisation that is the caller's)."""
    import numpy as np
    import torch
    from paper_2602_03893_amd import Plan, adam_update, inputs as I

    w = I.WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    centres, sensors = I.geometry_arrays(w)
    t = time.perf_counter()
    plan = Plan(centres, sensors, w.n_samples, w.dt, w.c_sound, n_sigma=w.n_sigma,
                sigma_max=w.smax, device=dev)
    t_plan = time.perf_counter() - t
    M, Nd, Nt = w.n_kernels, w.n_sensors, w.n_samples
    lo, hi = 0.7 * w.sigma, 1.0 * w.sigma
    S6 = torch.tensor(I.covariances(M, seed=300, lo=lo, hi=hi), device=dev)
    log(f"bench --aniso: workload {w.name}, axes U[{lo}, {hi}] m, plan {t_plan:.2f} s")
    A_true_h = I.phantom(w)
    b = plan.forward_aniso(torch.tensor(A_true_h, device=dev), S6).clone()
    A = torch.zeros(M, dtype=torch.float32, device=dev)
    mA, vA = torch.zeros_like(A), torch.zeros_like(A)
    y = torch.empty((Nd, Nt), dtype=torch.float32, device=dev)
    scale = 1.0 / float(torch.sum(b.double() ** 2))
    state = {"t": 0}

    def step():
        state["t"] += 1
        plan.forward_aniso(A, S6, out=y)
        plan.residual(y, b, scale=scale, delta=y)
        gA, _ = plan.adjoint_aniso(A, S6, y, want_sigma=True)
        adam_update(A, gA, mA, vA, state["t"], 1e-2, lo=0.0)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    f_ms = float(np.mean(plan.kernel_times("forward")))
    a_ms = float(np.mean(plan.kernel_times("adjoint")))
    plan.set_timing(False)
    pairs = float(M) * Nd
    ms_step = 1e3 * elapsed / args.steps
    value = 2.0 * pairs * args.steps / elapsed / 1e9
    # in-window taps per pair: 2 n_sigma sigma_n / (v dt) on average over the draw
    taps = pairs * 2.0 * w.n_sigma * (0.5 * (lo + hi)) / (w.c_sound * w.dt)
    flop_adj = FLOP_PAIR_ANISO * pairs + 10.0 * taps
    flop_fwd = FLOP_PAIR_ANISO * pairs + 7.0 * taps
    dom, dms, dfl = ("adjoint_kernel", a_ms, flop_adj) if a_ms >= f_ms else ("forward_kernel", f_ms, flop_fwd)
    achieved = dfl / (dms * 1e-3) / 1e12
    log(f"bench --aniso: {ms_step:.2f} ms/step, forward kernel {f_ms:.2f} ms, adjoint kernel "
        f"{a_ms:.2f} ms, {value:.1f} G-evals/s")
    out = {
        "metric": "fwd+adjoint G-evals/s (paper-scale IR step, anisotropic kernels)",
        "value": value,
        "unit": "G-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 distances, sigma_n and windows / f32 taps and per-stage sums / f64 cross-sensor sums",
        "data": "synthetic (seeded vessel-tree phantom; b = anisotropic forward of x_true)",
        "config": {"workload": "256x256x128 anisotropic Gaussian kernels (0.1 mm), 1024 sensors "
                               "on a 40 mm hemisphere, 4096 samples at 40 MHz, covariances "
                               f"R diag(s^2) R^T with axes U[{lo}, {hi}] m, Adam on A",
                   "kernels": M, "sensors": Nd, "samples": Nt, "parallelism": "single GPU"},
        "fwd_kernel_ms": f_ms,
        "adj_kernel_ms": a_ms,
        "plan_s": t_plan,
        "roofline": {"bound": "alu", "kernel": "aniso_" + dom, "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": MEASURED_TRAFFIC_ANISO.get(kernel_source_hash("aniso.hip"), {})
                                                      .get("aniso_" + dom),
                     "kernel_source_sha256_16": kernel_source_hash("aniso.hip")},
    }
    if not args.no_cpu_baseline:
        log("bench --aniso: timing the float64 oracle on a sample (cpu_baseline)")
        out["cpu_baseline"] = cpu_baseline_aniso(w, centres, sensors, A_true_h,
                                                 S6.cpu().numpy())
    print(json.dumps(out), flush=True)


def bench_centres(args):
    """Paper-scale IR step whose adjoint also returns the gradient with
    respect to every kernel centre (gpair_adjoint_centres, learnable
    centres): forward -> residual -> adjoint (A, sigma, centres) -> Adam on A
    and sigma; the centres stay where the plan put them (moving them means
    re-planning)."""
    import numpy as np
    import torch
    from paper_2602_03893_amd import Plan, adam_update, inputs as I

    w = I.WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    centres, sensors = I.geometry_arrays(w)
    plan = Plan(centres, sensors, w.n_samples, w.dt, w.c_sound, n_sigma=w.n_sigma,
                sigma_max=w.smax, device=dev)
    M, Nd, Nt = w.n_kernels, w.n_sensors, w.n_samples
    A_true = torch.tensor(I.phantom(w), device=dev)
    sig0 = w.sigma
    b = plan.forward(A_true, torch.full((M,), sig0, dtype=torch.float32, device=dev)).clone()
    A = torch.zeros(M, dtype=torch.float32, device=dev)
    sigma = torch.full((M,), sig0, dtype=torch.float32, device=dev)
    mA, vA, mS, vS = (torch.zeros_like(A) for _ in range(4))
    y = torch.empty((Nd, Nt), dtype=torch.float32, device=dev)
    scale = 1.0 / float(torch.sum(b.double() ** 2))
    state = {"t": 0}

    def step():
        state["t"] += 1
        plan.forward(A, sigma, out=y)
        plan.residual(y, b, scale=scale, delta=y)
        gA, gS, _ = plan.adjoint_centres(A, sigma, y, want_sigma=True)
        adam_update(A, gA, mA, vA, state["t"], 1e-2, lo=0.0)
        adam_update(sigma, gS, mS, vS, state["t"], 1e-3 * sig0, lo=0.5 * sig0, hi=w.smax)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    f_ms = float(np.mean(plan.kernel_times("forward")))
    a_ms = float(np.mean(plan.kernel_times("adjoint")))
    plan.set_timing(False)
    ms_step = 1e3 * elapsed / args.steps
    value = 2.0 * float(M) * Nd * args.steps / elapsed / 1e9
    log(f"bench --centres: {ms_step:.2f} ms/step, forward kernel {f_ms:.2f} ms, adjoint kernel "
        f"(A, sigma, centres) {a_ms:.2f} ms, {value:.1f} G-evals/s")
    # in-window taps per operator at the step's sigma; the centre mode adds
    # three sums per tap and the direction terms per pair
    taps = float(torch.sum(sigma.double())) * 2 * w.n_sigma / (w.c_sound * w.dt) * Nd
    pairs = float(M) * Nd
    flop = (FLOP_TAP_ADJ + FLOP_TAP_CENTRES) * taps + (FLOP_PAIR + FLOP_PAIR_CENTRES) * pairs
    achieved = flop / (a_ms * 1e-3) / 1e12
    out = {
        "metric": "fwd+adjoint G-evals/s (paper-scale IR step, adjoint with the centre gradient)",
        "value": value, "unit": "G-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 taps / f64 distances and sums",
        "data": "synthetic (seeded vessel-tree phantom; b = A(x_true))",
        "config": {"workload": "256x256x128 Gaussian kernels (0.1 mm), 1024 sensors on a 40 mm "
                               "hemisphere, 4096 samples at 40 MHz, gradients for A, sigma and "
                               "the centres, Adam on A and sigma",
                   "kernels": M, "sensors": Nd, "samples": Nt, "parallelism": "single GPU"},
        "fwd_kernel_ms": f_ms, "adj_kernel_ms": a_ms,
        "roofline": {"bound": "alu", "kernel": "adjoint_centres_kernel", "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel_source_sha256_16": kernel_source_hash()}}
    if not args.no_cpu_baseline:
        log("bench --centres: timing the float64 oracle's centre gradient on a sample")
        out["cpu_baseline"] = cpu_baseline_centres(w, centres, sensors, I.phantom(w), sig0)
    print(json.dumps(out), flush=True)


def cpu_baseline_centres(w, centres, sensors, A, sigma_val, stride=4):
    """The float64 oracle's centre gradient for every `stride`-th kernel (all
    sensors): a bounded sample of the centre-gradient adjoint."""
    import numpy as np
    from oracle import ops as O
    from paper_2602_03893_amd import inputs as I
    g = O.Geometry(centres, sensors, w.n_samples, w.dt, w.t0, w.c_sound, w.n_sigma)
    ks = np.arange(0, w.n_kernels, stride)
    delta = I.standard_normal((w.n_sensors, w.n_samples), seed=99, dtype=np.float64)
    t = time.perf_counter()
    O.adjoint_centres(g.subset_kernels(ks), A[ks].astype(np.float64),
                      np.full(len(ks), sigma_val), delta)
    el = time.perf_counter() - t
    return {"value": len(ks) * w.n_sensors / el / 1e9, "unit": "G-evals/s",
            "cores": O.num_threads(), "kind": "oracle", "cpu_model": host_cpu_model(),
            "sample": (f"float64 oracle centre gradient on {len(ks)} kernels x {w.n_sensors} "
                       f"sensors ({el:.2f} s); rate = pairs / time")}


def cpu_baseline_aniso(w, centres, sensors, A, S6, rows=160, stride=8):
    """The float64 anisotropic oracle on a bounded sample of the workload: the
    forward for `rows` sensors (all kernels), the adjoint with the covariance
    gradient for every `stride`-th kernel (all sensors)."""
    import numpy as np
    from oracle import ops as O
    from paper_2602_03893_amd import inputs as I
    g = O.Geometry(centres, sensors, w.n_samples, w.dt, w.t0, w.c_sound, w.n_sigma)
    M, Nd = w.n_kernels, w.n_sensors
    s6 = S6.astype(np.float64).T
    pick = np.linspace(0, Nd - 1, rows).astype(int)
    t = time.perf_counter()
    O.forward_aniso(g.subset_sensors(pick), A.astype(np.float64), s6)
    t_fwd = time.perf_counter() - t
    ks = np.arange(0, M, stride)
    delta = I.standard_normal((Nd, w.n_samples), seed=99, dtype=np.float64)
    t = time.perf_counter()
    O.adjoint_aniso(g.subset_kernels(ks), A[ks].astype(np.float64), s6[ks], delta)
    t_adj = time.perf_counter() - t
    rate = (M * rows + len(ks) * Nd) / (t_fwd + t_adj) / 1e9
    return {"value": rate, "unit": "G-evals/s", "cores": O.num_threads(), "kind": "oracle",
            "cpu_model": host_cpu_model(),
            "sample": (f"float64 anisotropic oracle: forward on {rows} of {Nd} sensors x {M} "
                       f"kernels ({t_fwd:.2f} s) + adjoint with the covariance gradient on "
                       f"{len(ks)} kernels x {Nd} sensors ({t_adj:.2f} s); rate = pairs / time")}


def net_flops(levels, n, d, h, w):
    """Algorithmic FLOPs of one training step of the warm-start U-Net (forward,
    data gradients, weight gradients; 2 per multiply-add) and of its forward."""
    fwd = bwd = 0.0
    vox = lambda l: n * (d >> l) * (h >> l) * (w >> l)
    ch = lambda l: 16 << l
    convs = []  # (level, cin, cout, taps, first)
    cin = 1
    for l in range(levels - 1):
        convs += [(l, cin, ch(l), 27, cin == 1), (l, ch(l), ch(l), 27, False)]
        cin = ch(l)
    convs += [(levels - 1, cin, ch(levels - 1), 27, cin == 1),
              (levels - 1, ch(levels - 1), ch(levels - 1), 27, False)]
    for l in range(levels - 2, -1, -1):
        convs += [(l + 1, ch(l + 1), ch(l), 8, False),   # transposed conv, per coarse voxel
                  (l, 2 * ch(l), ch(l), 27, False), (l, ch(l), ch(l), 27, False)]
    for lvl, ci, co, taps, first in convs:
        f = 2.0 * vox(lvl) * taps * ci * co
        fwd += f
        bwd += f * (1 if first else 2)
    return fwd + bwd, fwd


def bench_net(args):
    """The warm-start U-Net: one training step (forward, MSE, backward, Adam)
    on a batch of 4 volumes of 64 x 128 x 128, and the dominant convolution
    (the 32 -> 16 decoder conv at full resolution) timed alone."""
    import numpy as np
    import torch
    from paper_2602_03893_amd import inputs as I
    from paper_2602_03893_amd import nn as m
    levels, shape = 4, (4, 64, 128, 128)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    x = torch.as_tensor(np.abs(I.standard_normal(shape, seed=5))).to(dev)
    t = torch.as_tensor(np.abs(I.standard_normal(shape, seed=6))).to(dev)
    net = m.UNet(levels, shape, seed=1, device=dev)
    for _ in range(args.warmup):
        net.train_step(x, t, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.train_step(x, t, 1e-4)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = 1e3 * elapsed / args.steps
    flop, flop_fwd = net_flops(levels, *shape)
    # dominant layer alone: events on the stream the kernel is launched on
    n, d, h, w = shape
    cin, cout = 32, 16
    xin = torch.randn((n, d, h, w, cin), device=dev).relu_().to(torch.bfloat16)
    wm = torch.randn((27, cin, cout), device=dev) * (2.0 / (27 * cin)) ** 0.5
    wf = torch.empty((27, cout, cin), dtype=torch.bfloat16, device=dev)
    m.pack_weights(wm, 27, cin, cout, wf)
    bias = torch.zeros(cout, device=dev)
    out = torch.empty((n, d, h, w, cout), dtype=torch.bfloat16, device=dev)
    for _ in range(3):
        m.conv3(xin, wf, bias, out)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record(s)
    for _ in range(reps):
        m.conv3(xin, wf, bias, out)
    e1.record(s)
    torch.cuda.synchronize()
    conv_ms = e0.elapsed_time(e1) / reps
    conv_flop = 2.0 * n * d * h * w * 27 * cin * cout
    achieved = conv_flop / (conv_ms * 1e-3) / 1e12
    vox = n * d * h * w
    log(f"bench: U-Net train step {ms:.2f} ms ({flop / (ms * 1e-3) / 1e12:.1f} TFLOP/s), "
        f"conv 32->16 at 4x64x128x128 {conv_ms:.3f} ms ({achieved:.1f} TFLOP/s)")
    # the learned warm start at the paper-scale acquisition (half-resolution
    # adjoint, network, upsampling, rescale forward and dot products)
    from paper_2602_03893_amd import warmstart as W
    prob = W.Problem(device=dev)
    wpath = os.path.join(ROOT, "paper_2602_03893_amd", "weights", "unet4_c4.npy")
    params = np.load(wpath, allow_pickle=False) if os.path.exists(wpath) else \
        m.unet_init_params(levels, 1).numpy()
    kappa = W.TRAINED_KAPPA
    ws = m.WarmStart(prob.full, prob.half, levels, params, prob.vol_half, 1.0 / kappa)
    _, xs, _ = W.phantom_sample(100010)
    bw = prob.traces(xs, 100010)
    for _ in range(2):
        ws(bw, prob.sig_full, prob.sig_half)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(5):
        _, rep = ws(bw, prob.sig_full, prob.sig_half)
    torch.cuda.synchronize()
    warm_ms = 1e3 * (time.perf_counter() - t1) / 5
    log(f"bench: warm start {warm_ms:.2f} ms (rho {rep['rho']:.4f})")
    out = {
        "metric": "warm-start U-Net training voxels/s",
        "value": vox * args.steps / elapsed,
        "unit": "voxels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 (f32 accumulate, f32 master weights)",
        "data": "synthetic (seeded |N(0,1)| volumes)",
        "config": {"workload": "4-level 3D U-Net (16-128 channels), batch 4 x 64x128x128, "
                               "forward + MSE + backward + Adam",
                   "parameters": m.unet_param_count(levels), "parallelism": "single GPU"},
        "train_tflops": flop / (ms * 1e-3) / 1e12,
        "warm_start_ms": warm_ms,
        "warm_start_rho": rep["rho"],
        "roofline": {"bound": "mfma", "kernel": "conv_mfma_kernel<32,16> (32->16, 4x64x128x128)",
                     "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16_TFLOPS, "traffic": None},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-rho", action="store_true",
                    help="skip the time-to-residual leg after the timed steps")
    ap.add_argument("--net", action="store_true",
                    help="benchmark the warm-start U-Net training step instead")
    ap.add_argument("--assa", action="store_true",
                    help="benchmark the IR step with the ASSA operators (shared sigma)")
    ap.add_argument("--aniso", action="store_true",
                    help="the step with anisotropic kernels (covariances held fixed)")
    ap.add_argument("--centres", action="store_true",
                    help="the step whose adjoint also returns the centre gradient")
    ap.add_argument("--objective", action="store_true",
                    help="the step of Algorithm 2 in full: NPC latent, VCR regulariser, "
                         "warm-restart learning rate")
    ap.add_argument("--peaks", action="store_true",
                    help="only measure the issue rates of the vector instructions "
                         "(float32/float64 FMA, exp2, rsq) on this GPU")
    ap.add_argument("--c5", type=int, default=0, metavar="N",
                    help="only the time to rho <= 1e-2 on N held-out phantoms (per-phantom "
                         "rows and medians; zero, learned and scaled-adjoint starts)")
    ap.add_argument("--c5-first", type=int, default=TTR_SEED,
                    help="seed of the first held-out phantom of --c5")
    ap.add_argument("--ttr-cap", type=int, default=TTR_CAP,
                    help="iteration cap of the time-to-rho runs")
    ap.add_argument("--ttr-starts", default="zero,learned,scaled_adjoint",
                    help="starts of --c5, comma separated")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 256 MiB device buffer 3 times (scale reference "
                         "for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = 64 * 1024 * 1024  # float32 elements = 256 MiB
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {4 * n} bytes")
        return
    if args.c5 > 0:
        bench_c5(args)
        return
    if args.peaks:
        import torch
        torch.cuda.set_device(0)
        pk = measure_peaks()
        for k, v in pk.items():
            log(f"peaks: {k}: {v['per_cu_per_clk']:.3f} wave64 instructions per CU per clock")
        print(json.dumps({"peaks": pk, "clock_hz": CLOCK_HZ, "cus": CUS}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "kernel-sharded path is a design, not part of this build", file=sys.stderr)
        sys.exit(2)
    if args.net:
        bench_net(args)
        return
    if args.assa:
        bench_assa(args)
        return
    if args.aniso:
        bench_aniso(args)
        return
    if args.centres:
        bench_centres(args)
        return

    import numpy as np
    import torch
    from paper_2602_03893_amd import Plan, adam_update, inputs as I

    w = I.WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    centres, sensors = I.geometry_arrays(w)
    log(f"bench: workload {w.name}: {w.n_kernels} kernels, {w.n_sensors} sensors, "
        f"{w.n_samples} samples")
    t = time.perf_counter()
    plan = Plan(centres, sensors, w.n_samples, w.dt, w.c_sound, n_sigma=w.n_sigma,
                sigma_max=w.smax, device=dev)
    t_plan = time.perf_counter() - t
    info = plan.info()
    log(f"bench: plan {t_plan:.2f} s, {info['fwd_tiles']} forward tiles of <= {info['fwd_tile']}, "
        f"{info['adj_tiles']} adjoint tiles of <= {info['adj_tile']}")

    M, Nd, Nt = w.n_kernels, w.n_sensors, w.n_samples
    A_true_h = I.phantom(w)
    A_true = torch.tensor(A_true_h, device=dev)
    sig0 = w.sigma
    sig_true = torch.full((M,), sig0, dtype=torch.float32, device=dev)
    b = plan.forward(A_true, sig_true).clone()
    A = torch.zeros(M, dtype=torch.float32, device=dev)
    sigma = torch.full((M,), sig0, dtype=torch.float32, device=dev)
    mA, vA = torch.zeros_like(A), torch.zeros_like(A)
    mS, vS = torch.zeros_like(A), torch.zeros_like(A)
    y = torch.empty((Nd, Nt), dtype=torch.float32, device=dev)
    gA = torch.empty(M, dtype=torch.float32, device=dev)
    gS = torch.empty(M, dtype=torch.float32, device=dev)
    nb2 = float(torch.sum(b.double() ** 2))
    scale = 1.0 / nb2
    # the reconstructions' Adam learning rates (the time-to-rho leg uses the
    # same; the full objective keeps its stated schedule's peak of 1e-2)
    from paper_2602_03893_amd.warmstart import EVAL_BETA2, EVAL_LR_A, EVAL_LR_SIGMA_REL
    lr_A = 1e-2 if args.objective else EVAL_LR_A
    lr_S = EVAL_LR_SIGMA_REL * sig0
    beta2 = 0.999 if args.objective else EVAL_BETA2
    s_lo, s_hi = 0.5 * sig0, w.smax
    state = {"t": 0}
    obj = Objective(w, dev) if args.objective else None

    def step():
        state["t"] += 1
        if obj:
            obj.x_from_z(A)
        plan.prepare(A, sigma)           # records once for both operators
        plan.forward_prepared(out=y)
        plan.residual(y, b, scale=scale, delta=y)
        plan.adjoint_prepared(y, want_sigma=True, out_A=gA, out_sigma=gS)
        if obj:
            obj.add_reg_and_chain(A, gA)
            adam_update(obj.z, gA, mA, vA, state["t"], obj.lr(state["t"], lr_A))
        else:
            adam_update(A, gA, mA, vA, state["t"], lr_A, beta2=beta2, lo=0.0)
        adam_update(sigma, gS, mS, vS, state["t"], lr_S, beta2=beta2, lo=s_lo, hi=s_hi)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    taps_before = float(torch.sum(sigma.double())) * 2 * w.n_sigma / (w.c_sound * w.dt) * Nd
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fwd_ms = plan.kernel_times("forward")
    adj_ms = plan.kernel_times("adjoint")
    plan.set_timing(False)
    taps_after = float(torch.sum(sigma.double())) * 2 * w.n_sigma / (w.c_sound * w.dt) * Nd
    taps = 0.5 * (taps_before + taps_after)   # expected in-window taps per operator
    pairs = float(M) * Nd
    ms_step = 1e3 * elapsed / args.steps
    value = 2.0 * pairs * args.steps / elapsed / 1e9
    t_fwd = float(np.mean(fwd_ms))
    t_adj = float(np.mean(adj_ms))
    flop_fwd = FLOP_TAP_FWD * taps + FLOP_PAIR * pairs
    flop_adj = FLOP_TAP_ADJ * taps + FLOP_PAIR * pairs
    if t_adj >= t_fwd:
        dom, flop, t_dom = "adjoint_kernel", flop_adj, t_adj
    else:
        dom, flop, t_dom = "forward_kernel", flop_fwd, t_fwd
    achieved = flop / (t_dom * 1e-3) / 1e12
    flop64 = FLOP_PAIR * pairs
    frac64 = ((flop - flop64) / (PEAK_FP32_TFLOPS * 1e12) + flop64 / (PEAK_FP64_TFLOPS * 1e12)) \
        / (t_dom * 1e-3)
    exp_rate = 2.0 * pairs / (t_dom * 1e-3)   # two exp2 per pair (first tap, ratio)
    peaks = measure_peaks()
    log(f"bench: measured v_exp_f32 {peaks['v_exp_f32']['per_cu_per_clk']:.3f}, v_fma_f32 "
        f"{peaks['v_fma_f32']['per_cu_per_clk']:.3f}, v_fma_f64 "
        f"{peaks['v_fma_f64']['per_cu_per_clk']:.3f} wave64 instructions per CU per clock")
    log(f"bench: {ms_step:.2f} ms/step, forward kernel {t_fwd:.2f} ms, adjoint kernel "
        f"{t_adj:.2f} ms, {value:.1f} G-evals/s")

    out = {
        "metric": ("fwd+adjoint G-evals/s (paper-scale differentiable IR step"
                   + (", NPC + VCR + CAWR)" if obj else ")")),
        "value": value,
        "unit": "G-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 taps / f64 distances and sums",
        "data": "synthetic (seeded vessel-tree phantom; b = A(x_true))",
        "config": {"workload": "256x256x128 Gaussian kernels (0.1 mm), 1024 sensors on a "
                               "40 mm hemisphere, 4096 samples at 40 MHz, learnable A and "
                               "sigma (init 0.05 mm), Adam",
                   "kernels": M, "sensors": Nd, "samples": Nt, "parallelism": "single GPU"},
        "fwd_kernel_ms": t_fwd,
        "adj_kernel_ms": t_adj,
        "paper_context": {"gpu": "RTX 5090", "operators": "ASSA (shared sigma, no sigma "
                          "gradient)", "fwd_ms": PAPER_ASSA_MS["forward"],
                          "adj_ms": PAPER_ASSA_MS["adjoint"]},
        "taps_per_operator": taps,
        "taps_per_s": 2 * taps * args.steps / elapsed,
        "plan_s": t_plan,
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": MEASURED_TRAFFIC.get(kernel_source_hash(), {}).get(dom),
                     "frac_fp64_at_fp64_peak": frac64,
                     "frac_by_kernel": {
                         "forward_kernel": flop_fwd / (t_fwd * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
                         "adjoint_kernel": flop_adj / (t_adj * 1e-3) / 1e12 / PEAK_FP32_TFLOPS},
                     "exp_per_s": exp_rate,
                     "exp_frac_of_measured": exp_rate / (peaks["v_exp_f32"]["wave_instr_per_s"] * 64),
                     "valu_per_cu_per_clk": MEASURED_VALU.get(kernel_source_hash(), {}).get(dom),
                     "measured_peaks": peaks,
                     "kernel_source_sha256_16": kernel_source_hash()},
    }
    if obj:
        out.update(objective_fields(obj, w))
    if not args.no_cpu_baseline:
        log("bench: timing the float64 oracle on a sample (cpu_baseline)")
        out["cpu_baseline"] = cpu_baseline(w, centres, sensors, A_true_h, sig0)
    if not args.no_time_to_rho and w.name == "paper" and not obj:
        log("bench: time to rho <= 1e-2 on a held-out phantom (zero and learned starts)")
        out["time_to_rho"] = time_to_rho(dev, args.ttr_cap)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
