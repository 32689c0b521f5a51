"""Training data, training loop and evaluation of the learned warm start.

Every operator, network layer and update runs in libgpair's HIP kernels (the
C ABI of include/gpair.h and include/gpair_nn.h); this module only draws the
seeded phantoms (on host worker processes), moves volumes between host and
device, and orders the calls.

Data (one sample per seeded vessel phantom, the paper-scale acquisition):
 - x_true: 256 x 256 x 128 kernels at 0.1 mm (grid order, x fastest);
 - b = A(x_true) with sigma = 0.05 mm, plus white noise of 1 % of the trace
   RMS (the noise drawn on the device from a generator seeded per phantom);
 - network input: A_half^T b on the 128 x 128 x 64 grid at 0.2 mm with
   sigma = 0.1 mm, scaled by 1 / kappa, kappa the largest eigenvalue of
   A_half^T A_half (power iteration);
 - target: the 2 x 2 x 2 block mean of x_true.

CLI (writes a JSON report and the trained parameters):
  python -m paper_2602_03893_amd.warmstart --train 1800 --test 200 --epochs 30 \
      --eval 5 --out DIR
"""
import argparse
import json
import multiprocessing as mp
import os
import time

import numpy as np

from . import inputs as I

FULL = I.WORKLOADS["paper"]
HALF = I.WORKLOADS["half"]
SIGMA_FULL = FULL.sigma          # 0.05 mm: the traces' kernel width
SIGMA_HALF = HALF.sigma          # 0.1 mm on the half-resolution grid
NOISE = 0.01
LEVELS = 4
# kappa of the half-resolution plan as measured when weights/unet4_c4.npy was
# trained (power_kappa(), 30 iterations, seed 0)
TRAINED_KAPPA = 0.0928654670715332


# Training and test phantoms: a vessel tree plus Poisson(1) spheres (radius
# U[0.3, 1.5] mm, value U[0.5, 1]); evaluation phantoms: vessel trees.
TRAIN_SPHERES_MEAN = 1.0
EVAL_SPHERES_MEAN = 0.0


def phantom_sample(seed, n_spheres_mean=TRAIN_SPHERES_MEAN):
    """Host worker: the phantom and its 2 x 2 x 2 block-mean target."""
    x = I.vessel_phantom(FULL.grid, FULL.spacing, seed, n_spheres_mean=n_spheres_mean)
    nx, ny, nz = FULL.grid
    t = x.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(1, 3, 5), dtype=np.float64)
    return seed, x, t.astype(np.float32).reshape(-1)


class Problem:
    """Full- and half-resolution plans of the paper-scale acquisition."""

    def __init__(self, device=None):
        import torch
        from .api import Plan
        self.torch = torch
        cen, sen = I.geometry_arrays(FULL)
        cen2, _ = I.geometry_arrays(HALF)
        self.full = Plan(cen, sen, FULL.n_samples, FULL.dt, FULL.c_sound, n_sigma=FULL.n_sigma,
                         sigma_max=FULL.smax, device=device)
        self.half = Plan(cen2, sen, HALF.n_samples, HALF.dt, HALF.c_sound, n_sigma=HALF.n_sigma,
                         sigma_max=HALF.smax, device=device)
        dev = self.full.device
        self.device = dev
        self.sig_full = torch.full((self.full.n_kernels,), SIGMA_FULL, dtype=torch.float32, device=dev)
        self.sig_half = torch.full((self.half.n_kernels,), SIGMA_HALF, dtype=torch.float32, device=dev)
        nx, ny, nz = HALF.grid
        self.vol_half = (nz, ny, nx)
        self.kappa = None

    def power_kappa(self, iters=30, seed=0):
        """Largest eigenvalue of A_half^T A_half by power iteration (setup)."""
        torch = self.torch
        g = torch.Generator(device=self.device)
        g.manual_seed(seed)
        x = torch.rand(self.half.n_kernels, generator=g, device=self.device)
        lam = 0.0
        for _ in range(iters):
            x = x / torch.linalg.vector_norm(x)
            y = self.half.forward(x, self.sig_half)
            gx = self.half.adjoint(x, self.sig_half, y, want_sigma=False)[0]
            lam = float(torch.dot(gx, x))
            x = gx
        self.kappa = lam
        return lam

    def traces(self, x_true, seed, out=None):
        """b = A(x_true) + 1 % white noise (device float32 [N_d * N_t])."""
        torch = self.torch
        xt = torch.as_tensor(x_true).to(self.device)
        b = self.full.forward(xt, self.sig_full, out=out)
        g = torch.Generator(device=self.device)
        g.manual_seed(int(seed))
        rms = torch.sqrt(torch.mean(b.double() ** 2)).float()
        b.add_(NOISE * rms * torch.randn(b.shape, generator=g, device=self.device))
        return b

    def net_input(self, b, out=None):
        """A_half^T b (unscaled; the network applies 1 / kappa)."""
        return self.half.adjoint(None, self.sig_half, b, want_sigma=False, out_A=out)[0]


def generate(problem, seeds, pool, log=print):
    """Inputs and targets (device float32 [n, 64, 128, 128]) for the seeds;
    the phantoms are drawn by `pool` (host processes forked before the GPU
    was first used)."""
    torch = problem.torch
    d, h, w = problem.vol_half
    n = len(seeds)
    X = torch.empty((n, d, h, w), dtype=torch.float32, device=problem.device)
    T = torch.empty((n, d, h, w), dtype=torch.float32, device=problem.device)
    pos = {s: i for i, s in enumerate(seeds)}
    t0 = time.time()
    for k, (seed, x, t) in enumerate(pool.imap_unordered(phantom_sample, seeds, chunksize=2)):
        i = pos[seed]
        b = problem.traces(x, seed)
        problem.net_input(b, out=X[i].view(-1))
        T[i].view(-1).copy_(torch.as_tensor(t))
        if (k + 1) % 200 == 0 or k + 1 == n:
            torch.cuda.synchronize()
            log(f"data: {k + 1}/{n} samples, {time.time() - t0:.1f} s")
    return X, T


def rel_error(net, X, T, scale, batch):
    """Mean over samples of ||net(x) - t|| / ||t||."""
    import torch
    errs = []
    for i in range(0, X.shape[0] - batch + 1, batch):
        y = net.forward(X[i:i + batch].contiguous(), scale=scale)
        t = T[i:i + batch]
        num = (y - t).flatten(1).norm(dim=1)
        den = t.flatten(1).norm(dim=1).clamp_min(1e-30)
        errs.append((num / den).cpu())
    return float(torch.cat(errs).mean())


def train(problem, X, T, Xte, Tte, epochs, batch=4, lr=1e-3, seed=0, log=print,
          time_budget=None):
    import torch
    from .nn import UNet
    d, h, w = problem.vol_half
    net = UNet(LEVELS, (batch, d, h, w), seed=seed, device=problem.device)
    scale = 1.0 / problem.kappa
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    steps = n // batch
    hist = []
    t0 = time.time()
    step_times = []
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(n), device=problem.device)
        tot = torch.zeros((), dtype=torch.float64, device=problem.device)
        torch.cuda.synchronize()
        te = time.time()
        for s in range(steps):
            idx = perm[s * batch:(s + 1) * batch]
            loss = net.train_step(X[idx], T[idx], lr, scale=scale)
            tot += loss[0]
        torch.cuda.synchronize()
        step_times.append((time.time() - te) / steps)
        test = rel_error(net, Xte, Tte, scale, batch)
        hist.append({"epoch": ep + 1, "train_mse": float(tot) / steps, "test_rel_l2": test})
        log(f"train: epoch {ep + 1}/{epochs} mse {float(tot) / steps:.4e} test rel {test:.4f} "
            f"({step_times[-1] * 1e3:.2f} ms/step, {time.time() - t0:.0f} s)")
        if time_budget is not None and time.time() - t0 > time_budget:
            log("train: time budget reached")
            break
    return net, hist, float(np.median(step_times))


# Adam settings of the reconstructions (learning rate of A, of sigma relative
# to its initial value, second-moment decay), chosen by the time to
# rho <= 1e-2 on training phantoms (seeds 1000-1003, never the held-out ones).
# At beta2 = 0.999: lr_A 1e-2 / 2e-2 / 4e-2 / 8e-2 / 0.16 / 0.32 took 4000+ /
# 1859 / 716 / 436 / 401 / 412 iterations from the zero start (the learned
# start 380-430 at every rate); sigma rates from 0 to 1e-3 changed either by
# under 5 %.  At lr_A 0.16: beta2 0.99 / 0.98 / 0.95 / 0.9 took 289 / 222 /
# 175 / 120 iterations, 0.8 and 0.5 did not converge in 1000; beta1 0.8 or
# 0.95 and warm-restart schedules were slower.  At beta2 0.9, lr_A 0.08 took
# 110-112 iterations on all four seeds from either start (0.32 failed; 0.05
# and 0.12 took 109-117; beta1 0.85 and 0.8 slowed the zero start to
# 104-149 and 189-242).
EVAL_LR_A, EVAL_LR_SIGMA_REL, EVAL_BETA2 = 0.08, 1e-3, 0.9


def evaluate(problem, net_params, seeds, max_iters=500, tol=1e-2, log=print,
             starts=("zero", "learned", "scaled_adjoint"), lr_A=EVAL_LR_A,
             lr_sigma_rel=EVAL_LR_SIGMA_REL, solve_opts=None):
    """Time to rho <= tol from the zero, learned and scaled-adjoint starts
    (Adam on A and sigma with learning rates lr_A and lr_sigma_rel *
    sigma_0), on vessel phantoms with 1 % noise, and the image error
    ||A - x_true|| / ||x_true|| where each run stops.  A start that does not
    reach tol within max_iters is reported as not reached, with its final
    rho.  solve_opts: further options of Plan.solve (beta2 defaults to
    EVAL_BETA2)."""
    import torch
    from .nn import WarmStart
    full = problem.full
    d, h, w = problem.vol_half
    ws = WarmStart(full, problem.half, LEVELS, net_params, (d, h, w), 1.0 / problem.kappa)
    sig0 = SIGMA_FULL
    out = []
    for seed in seeds:
        _, x, _ = phantom_sample(seed, EVAL_SPHERES_MEAN)
        b = problem.traces(x, seed)
        xt = torch.as_tensor(x).to(problem.device)
        norms = full.residual(full.forward(xt, problem.sig_full), b)
        rho_true = float(torch.sqrt(norms[0] / norms[1]))
        row = {"seed": int(seed), "rho_x_true": rho_true}
        for start in starts:
            sigma = torch.full((full.n_kernels,), sig0, dtype=torch.float32, device=problem.device)
            torch.cuda.synchronize()
            t0 = time.time()
            if start == "zero":
                A = torch.zeros(full.n_kernels, dtype=torch.float32, device=problem.device)
                rep0 = {"c_star": 0.0, "rho": 1.0, "fell_back": True}
            elif start == "learned":
                A, rep0 = ws(b, problem.sig_full, problem.sig_half)
            else:
                A = full.adjoint(None, problem.sig_full, b, want_sigma=False)[0]
                from .api import pgd_update
                pgd_update(A, A, 0.0, lo=0.0)  # clamp at zero
                rep0 = full.warm_rescale(A, problem.sig_full, b)
            torch.cuda.synchronize()
            t_start = time.time() - t0
            rep = full.solve(b, A, sigma, method="adam", max_iters=max_iters, tol=tol, lr_A=lr_A,
                             lr_sigma=lr_sigma_rel * sig0, learn_sigma=True, sigma_lo=0.5 * sig0,
                             sigma_hi=FULL.smax, **{"beta2": EVAL_BETA2, **(solve_opts or {})})
            torch.cuda.synchronize()
            t_total = time.time() - t0
            x_err = float(torch.linalg.vector_norm((A - xt).double())
                          / torch.linalg.vector_norm(xt.double()))
            hist = np.array(rep["history"][:rep["iters"] + 1])
            per_it = (t_total - t_start) / max(rep["iters"], 1)
            hit = np.nonzero(hist <= 1.05 * rho_true)[0]
            row[start] = {
                "start_rho": rep0["rho"], "c_star": rep0["c_star"], "fell_back": rep0["fell_back"],
                "iters": rep["iters"], "final_rho": float(hist[-1]), "reached_tol": bool(rep["converged"]),
                "time_s": t_total, "start_s": t_start,
                "time_to_tol_s": t_total if rep["converged"] else None,
                "time_to_1.05_rho_true_s": (t_start + per_it * int(hit[0])) if hit.size else None,
                "x_rel_l2": x_err,
            }
            log(f"eval seed {seed} {start}: start rho {rep0['rho']:.4f}, {rep['iters']} iters, "
                f"final rho {hist[-1]:.5f}, {t_total:.2f} s, image error {x_err:.4f}")
        out.append(row)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train", type=int, default=1800)
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval", type=int, default=5, help="held-out phantoms for time-to-rho")
    ap.add_argument("--eval-first", type=int, default=100000,
                    help="seed of the first held-out phantom")
    ap.add_argument("--kappa", type=float, default=None,
                    help="input normalisation of trained parameters (skips the power iteration)")
    ap.add_argument("--eval-iters", type=int, default=500)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--train-budget", type=float, default=None, help="seconds")
    ap.add_argument("--params", default=None, help="skip training: load parameters (.npy)")
    ap.add_argument("--out", default="warmstart_out")
    a = ap.parse_args(argv)
    os.makedirs(a.out, exist_ok=True)
    t_all = time.time()

    def log(msg):
        print(msg, flush=True)

    # host workers fork before the GPU is first used
    pool = mp.get_context("fork").Pool(a.workers)
    import torch
    problem = Problem()
    if a.kappa is not None:
        problem.kappa = kappa = a.kappa
    else:
        kappa = problem.power_kappa()
    log(f"setup: kappa (largest eigenvalue of A_half^T A_half) = {kappa:.6e}")
    report = {"kappa": kappa, "levels": LEVELS}
    if a.params is None:
        seeds_tr = list(range(1000, 1000 + a.train))
        seeds_te = list(range(50000, 50000 + a.test))
        X, T = generate(problem, seeds_tr, pool, log)
        Xte, Tte = generate(problem, seeds_te, pool, log)
        batch = 4
        scale = 1.0 / kappa
        # the control: scaled adjoint on the half grid (least-squares scalar fit)
        num = float((Xte * Tte).sum() / (Xte * Xte).sum())
        ctrl = float(((num * Xte - Tte).flatten(1).norm(dim=1) / Tte.flatten(1).norm(dim=1)).mean())
        net, hist, ms = train(problem, X, T, Xte, Tte, a.epochs, batch=batch, lr=a.lr, log=log,
                              time_budget=a.train_budget)
        params = net.params.cpu().numpy()
        np.save(os.path.join(a.out, "unet_params.npy"), params)
        report.update({"train_samples": a.train, "test_samples": a.test, "history": hist,
                       "train_step_ms": ms * 1e3, "test_rel_l2": hist[-1]["test_rel_l2"],
                       "control_scaled_adjoint_rel_l2": ctrl})
        del X, T, Xte, Tte
        torch.cuda.empty_cache()
    else:
        params = np.load(a.params, allow_pickle=False)
    if a.eval > 0:
        report["eval"] = evaluate(problem, params,
                                  list(range(a.eval_first, a.eval_first + a.eval)),
                                  max_iters=a.eval_iters, log=log)
    pool.close()
    pool.join()
    report["wall_s"] = time.time() - t_all
    with open(os.path.join(a.out, "report.json"), "w") as f:
        json.dump(report, f, indent=1)
    log(f"done in {report['wall_s']:.0f} s")


if __name__ == "__main__":
    main()
