"""Solver replays at the mid-size and paper-scale workloads: gpair_solve (Adam,
through the C ABI) against stored runs of the float64 oracle's Adam loop
(``tests/golden/replay_goldens.py`` wrote them, calling only the oracle).

* mid: 100 Adam iterations on A, 1 % noise: the relative residual before
  every update within 1e-3 (relative), A after the last update within 1e-3
  relative L2 on every 16th kernel.
* paper scale: 3 Adam iterations on A and per-kernel sigma: residuals within
  1e-3, A within 1e-3 and sigma within 1e-6 relative L2 on every 64th kernel
  (131,072 kernels).

The looser bar of the Adam replays (the operators match to 1e-5) is Adam's
normalisation: a kernel whose gradient is near zero moves by up to the full
learning rate in a direction a float32 rounding can decide.
"""
import numpy as np
import pytest
import torch

from tests.conftest import rel_l2
from tests.golden.replay_goldens import golden_path, problem, settings

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("name", ["mid", "paper"])
def test_adam_replay_against_stored_oracle_run(name):
    from paper_2602_03893_amd import Plan
    gold = np.load(golden_path(name))
    w, _, cen, sen, _, sigma0, b = problem(name)
    r = settings(name)
    _say(f"case: Adam replay, {name} workload ({w.n_kernels} kernels, {w.n_sensors} sensors), "
         f"{r['iters']} iterations, learn_sigma={r['learn_sigma']}")
    plan = Plan(cen, sen, w.n_samples, w.dt, w.c_sound, n_sigma=w.n_sigma, sigma_max=w.smax)
    A = torch.zeros(w.n_kernels, dtype=torch.float32, device="cuda")
    sg = dev(sigma0)
    rep = plan.solve(dev(b), A, sg, method="adam", max_iters=r["iters"], lr_A=r["lr_a"],
                     lr_sigma=r["lr_s"], learn_sigma=r["learn_sigma"], sigma_lo=r["s_lo"],
                     sigma_hi=r["s_hi"])
    hist = np.array(rep["history"])
    ref = gold["rho"]
    assert rep["iters"] == r["iters"] and hist.shape == ref.shape
    erho = np.abs(hist - ref) / ref
    _say(f"  rho gpu {hist[0]:.6f} -> {hist[-1]:.6f}, oracle {ref[0]:.6f} -> {ref[-1]:.6f}; "
         f"max rel diff {erho.max():.2e}")
    assert erho.max() <= 1e-3
    ks = gold["kernels"]
    a = host(A)
    eA = rel_l2(a[ks], gold["A"])
    _say(f"  A on {ks.size} kernels: rel L2 {eA:.2e}; nonzero gpu {np.count_nonzero(a)} "
         f"oracle {int(gold['A_nonzero'])}")
    assert eA <= 1e-3
    if r["learn_sigma"]:
        eS = rel_l2(host(sg)[ks], gold["sigma"])
        _say(f"  sigma on {ks.size} kernels: rel L2 {eS:.2e}")
        assert eS <= 1e-6
