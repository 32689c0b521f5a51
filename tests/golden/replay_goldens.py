"""Stored expected values of the solver replays, written by the float64 oracle.

Running this file (``python tests/golden/replay_goldens.py [mid] [paper]``)
rewrites ``tests/golden/adam_replay_<name>.npz``.  It calls only ``oracle/``
and the seeded input generators (``paper_2602_03893_amd.inputs``, which hold
none of the method's arithmetic); the GPU tests import ``problem()`` from here
to rebuild the very same float32 inputs.

What is replayed (arXiv 2602.03893, Methods, "Optimization formulation and
algorithm" and Algorithm 2, data term only, A >= 0 by projection; Adam with
bias correction, beta = 0.9 / 0.999, eps = 1e-8, on the loss
0.5 ||A(x; sigma) - b||^2 / ||b||^2):

* ``mid``: 64^3 kernels at 0.1 mm, sigma = 0.05 mm fixed, 512 sensors on a
  20 mm hemisphere, 2048 samples at 40 MHz; b = A(x_true) plus white noise of
  1 % of the clean trace RMS (seed 1002); 100 Adam iterations on A from zero,
  learning rate 1e-2.
* ``paper``: 256 x 256 x 128 kernels at 0.1 mm, 1024 sensors on a 40 mm
  hemisphere, 4096 samples; b = A(x_true; sigma = 0.05 mm), clean; Adam on A
  (lr 1e-2, from zero) and on sigma (lr 1e-3 * 0.05 mm, from 0.05 mm, clamped
  to [0.025, 0.1] mm), 3 iterations.

Stored: the relative residual before every update and after the last one,
and A (and sigma) after the last update on every ``stride``-th kernel.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import ops as O  # noqa: E402
from oracle import solvers as S  # noqa: E402
from paper_2602_03893_amd import inputs as I  # noqa: E402

# name -> replay settings
REPLAYS = {
    "mid": {"iters": 100, "lr_a": 1e-2, "learn_sigma": False, "stride": 16},
    "paper": {"iters": 3, "lr_a": 1e-2, "learn_sigma": True, "stride": 64},
}


def golden_path(name):
    return os.path.join(HERE, f"adam_replay_{name}.npz")


def problem(name):
    """The replay's float32 inputs: (workload, oracle geometry, centres,
    sensors, x_true, sigma0, b).  b is the oracle's forward of x_true (only
    its non-zero kernels are visited: the skipped terms are exact zeros), plus
    the workload's seeded noise, rounded to float32."""
    w = I.WORKLOADS[name]
    cen, sen = I.geometry_arrays(w)
    g = O.Geometry(cen, sen, w.n_samples, w.dt, w.t0, w.c_sound, w.n_sigma)
    x_true = I.phantom(w)
    sigma0 = np.full(w.n_kernels, w.sigma, np.float32)
    nz = np.flatnonzero(x_true)
    b = O.forward(g.subset_kernels(nz), x_true[nz], sigma0[nz].astype(np.float64))
    if w.noise > 0:
        rms = float(np.sqrt(np.mean(b * b)))
        b = b + w.noise * rms * I.standard_normal(b.shape, seed=w.noise_seed, dtype=np.float64)
    return w, g, cen, sen, x_true, sigma0, b.astype(np.float32)


def settings(name):
    w = I.WORKLOADS[name]
    r = dict(REPLAYS[name])
    r["lr_s"] = 1e-3 * w.sigma if r["learn_sigma"] else 0.0
    r["s_lo"], r["s_hi"] = 0.5 * w.sigma, w.smax
    return r


def write(name):
    t = time.perf_counter()
    w, g, _, _, _, sigma0, b = problem(name)
    r = settings(name)
    print(f"{name}: {w.n_kernels} kernels, {w.n_sensors} sensors; Adam x {r['iters']} "
          f"on {O.num_threads()} threads", flush=True)
    a, s, hist = S.adam(g, np.zeros(w.n_kernels), sigma0.astype(np.float64),
                        b.astype(np.float64), r["iters"], lr_a=r["lr_a"], lr_s=r["lr_s"],
                        learn_sigma=r["learn_sigma"], s_lo=r["s_lo"], s_hi=r["s_hi"])
    ks = np.arange(0, w.n_kernels, r["stride"])
    np.savez_compressed(golden_path(name), rho=np.asarray(hist), kernels=ks, A=a[ks],
                        sigma=s[ks], A_norm=np.linalg.norm(a), A_nonzero=np.count_nonzero(a))
    print(f"{name}: rho {hist[0]:.6f} -> {hist[-1]:.6f}, {time.perf_counter() - t:.0f} s -> "
          f"{golden_path(name)}", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(REPLAYS)):
        write(n)
