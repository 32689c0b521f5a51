"""GPU parity: the HIP operators (through the C ABI) against the float64 oracle.

Bar (traces and gradients): relative L2 error <= 1e-5.  Window membership is
decided in float64 on both sides; taps are float32 on the GPU.
"""
import numpy as np
import pytest
import torch

from oracle import ops as O
from paper_2602_03893_amd import inputs as I
from tests.conftest import rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _say(msg):
    print(msg, flush=True)


def make_case(centres, sensors, n_samples, sigma_max, dt=I.DT, t0=0.0, c=I.C_SOUND,
              nsig=3.0, fwd_tile=0, adj_tile=0, fwd_waves=0):
    from paper_2602_03893_amd import Plan
    plan = Plan(centres, sensors, n_samples, dt, c, n_sigma=nsig, sigma_max=sigma_max,
                t0=t0, fwd_tile=fwd_tile, adj_tile=adj_tile, fwd_waves=fwd_waves)
    g = O.Geometry(centres, sensors, n_samples, dt, t0, c, nsig)
    return plan, g


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def workload_case(name, **kw):
    w = I.WORKLOADS[name]
    cen, sen = I.geometry_arrays(w)
    plan, g = make_case(cen, sen, w.n_samples, w.smax, **kw)
    return w, plan, g


@pytest.fixture(scope="module")
def toy():
    _say("case: toy workload (16^3 kernels, 64 sensors, 512 samples)")
    return workload_case("toy")


def check_forward(plan, g, A, sigma, label):
    _say(f"forward parity: {label}")
    y = host(plan.forward(dev(A), dev(sigma)))
    ref = O.forward(g, A.astype(np.float64), sigma.astype(np.float32).astype(np.float64))
    err = rel_l2(y, ref)
    _say(f"  rel L2 {err:.3e}")
    assert err <= TOL, err
    return y, ref


def check_adjoint(plan, g, A, sigma, delta, label, want_sigma=True):
    _say(f"adjoint parity: {label}")
    gA, gS = plan.adjoint(dev(A), dev(sigma), dev(delta), want_sigma=want_sigma)
    s64 = sigma.astype(np.float32).astype(np.float64)
    rA, rS = O.adjoint(g, A.astype(np.float64), s64, delta.astype(np.float32).astype(np.float64),
                       want_sigma=want_sigma)
    eA = rel_l2(host(gA), rA)
    _say(f"  gA rel L2 {eA:.3e}")
    assert eA <= TOL, eA
    if want_sigma:
        eS = rel_l2(host(gS), rS)
        _say(f"  gsigma rel L2 {eS:.3e}")
        assert eS <= TOL, eS
    return gA, gS


def test_toy_forward_and_adjoint(toy):
    w, plan, g = toy
    A = I.phantom(w)
    sigma = np.full(w.n_kernels, w.sigma, np.float32)
    check_forward(plan, g, A, sigma, "toy")
    delta = I.standard_normal((w.n_sensors, w.n_samples), seed=21)
    check_adjoint(plan, g, A, sigma, delta, "toy")
    check_adjoint(plan, g, A, sigma, delta, "toy, no sigma", want_sigma=False)


def test_toy_per_kernel_sigma_and_signed_amplitudes(toy):
    w, plan, g = toy
    A = I.uniform(w.n_kernels, seed=3, lo=-1.0, hi=1.0)
    sigma = I.uniform(w.n_kernels, seed=4, lo=0.2 * w.sigma, hi=w.sigma)
    check_forward(plan, g, A, sigma, "toy, sigma_k ~ U[0.2, 1] sigma_max")
    delta = I.standard_normal((w.n_sensors, w.n_samples), seed=22)
    check_adjoint(plan, g, A, sigma, delta, "toy, per-kernel sigma")


def dot_test_bound(Ax, y):
    """Bar of the GPU dot-product test: each float32 output element carries
    its own rounding, so |<Ax, y> - <x, A^T y>| scales with the magnitudes of
    the summed terms, sum |(Ax)_i y_i|, not with |<Ax, y>| (with random-sign y
    the sum cancels: at the toy shape by a factor of about 180).  The bar is
    1e-7 of that scale, under two float32 units."""
    return 1e-7 * float(np.sum(np.abs(Ax * y.astype(np.float64))))


def test_adjointness_on_gpu(toy):
    """<A x, y> = <x, A^T y> from GPU outputs (float64 inner products)."""
    w, plan, g = toy
    x = I.uniform(w.n_kernels, seed=5)
    sigma = np.full(w.n_kernels, w.sigma, np.float32)
    yv = I.standard_normal((w.n_sensors, w.n_samples), seed=6)
    Ax = host(plan.forward(dev(x), dev(sigma)))
    ATy, _ = plan.adjoint(dev(x), dev(sigma), dev(yv), want_sigma=False)
    lhs = float(np.sum(Ax * yv.astype(np.float64)))
    rhs = float(np.dot(x.astype(np.float64), host(ATy)))
    bar = dot_test_bound(Ax, yv)
    _say(f"  <Ax, y> {lhs:.9e}  <x, A^T y> {rhs:.9e}  |diff| {abs(lhs - rhs):.2e}  bar {bar:.2e}")
    assert abs(lhs - rhs) <= bar


@pytest.mark.parametrize("fwd_tile,adj_tile,fwd_waves",
                         [(64, 64, 1), (256, 128, 2), (1024, 256, 4), (64, 256, 8)])
def test_ragged_point_cloud_clipped_windows(fwd_tile, adj_tile, fwd_waves):
    """A random point cloud (not a lattice), N_d not a multiple of 64, tiles of
    several sizes (the last one partly filled), 1, 2 or 4 waves splitting each
    forward tile, and a time origin that cuts the earliest pulses at sample 0
    and the latest at sample N_t - 1."""
    _say(f"case: point cloud M=1000, N_d=70, tiles {fwd_tile}/{adj_tile}, {fwd_waves} waves")
    rng = np.random.default_rng(8)
    cen = rng.uniform(-1.5e-3, 1.5e-3, (1000, 3)).astype(np.float32)
    sen = I.fibonacci_hemisphere(70, 12e-3)
    # pulses arrive between ~9.4 mm and ~14.6 mm: start the trace at 11 mm and
    # stop it at 13 mm so both ends clip
    t0 = 11e-3 / I.C_SOUND
    nt = int((2e-3 / I.C_SOUND) / I.DT)
    smax = 0.08e-3
    plan, g = make_case(cen, sen, nt, smax, t0=t0, fwd_tile=fwd_tile, adj_tile=adj_tile,
                        fwd_waves=fwd_waves)
    assert plan.info()["fwd_waves"] == fwd_waves
    A = I.uniform(1000, seed=9, lo=-0.5, hi=1.0)
    sigma = I.uniform(1000, seed=10, lo=0.3 * smax, hi=smax)
    y, ref = check_forward(plan, g, A, sigma, "point cloud")
    assert np.abs(ref[:, 0]).max() > 0 and np.abs(ref[:, -1]).max() > 0
    delta = I.standard_normal((70, nt), seed=11)
    check_adjoint(plan, g, A, sigma, delta, "point cloud")


def test_forward_amplitudes_over_six_decades(toy):
    """Partial sums are carried in fixed point scaled to each tile's sum of
    |A_k|: amplitudes of both signs spread log-uniformly over six decades (a
    few kernels dominate each tile) still meet the bar, and zero amplitudes
    give an exactly zero trace."""
    w, plan, g = toy
    mag = 10.0 ** I.uniform(w.n_kernels, seed=31, lo=-6.0, hi=0.0)
    sgn = np.where(I.uniform(w.n_kernels, seed=32) < 0.5, -1.0, 1.0)
    A = (sgn * mag).astype(np.float32)
    sigma = I.uniform(w.n_kernels, seed=33, lo=0.5 * w.sigma, hi=w.sigma)
    check_forward(plan, g, A, sigma, "toy, |A| log-uniform over 1e-6..1, random signs")
    y0 = host(plan.forward(dev(np.zeros(w.n_kernels, np.float32)), dev(sigma)))
    assert np.all(y0 == 0.0)


def test_forward_propagates_non_finite_amplitudes(toy):
    w, plan, g = toy
    A = I.phantom(w).copy()
    A[w.n_kernels // 2] = np.nan
    y = host(plan.forward(dev(A), dev(np.full(w.n_kernels, w.sigma, np.float32))))
    assert not np.all(np.isfinite(y))


@pytest.mark.parametrize("spread", [False, True])
def test_wide_kernels_beyond_the_unrolled_tap_counts(spread):
    """sigma up to 0.3 mm at 25 ns sampling: up to 47 taps per pair, beyond the
    unrolled forms (18 taps), so the forward and the adjoint take their
    general tap loops; with a uniform sigma every tile has one tap count, with
    spread sigma the counts run from 13 to 47 within a tile."""
    _say(f"case: wide kernels, sigma {'spread' if spread else 'uniform'}")
    rng = np.random.default_rng(12)
    cen = rng.uniform(-2e-3, 2e-3, (700, 3)).astype(np.float32)
    sen = I.fibonacci_hemisphere(90, 15e-3)
    smax = 0.3e-3
    plan, g = make_case(cen, sen, 700, smax)
    assert plan.info()["max_taps"] > 40
    A = I.uniform(700, seed=13, lo=-0.5, hi=1.0)
    sigma = (I.uniform(700, seed=14, lo=0.25 * smax, hi=smax) if spread
             else np.full(700, smax, np.float32))
    check_forward(plan, g, A, sigma, "wide kernels")
    check_adjoint(plan, g, A, sigma, I.standard_normal((90, 700), seed=15), "wide kernels")


def test_single_kernel_single_sensor():
    _say("case: one kernel, one sensor")
    cen = np.array([[0.3e-3, -0.2e-3, 0.1e-3]], np.float32)
    sen = np.array([[0.0, 0.0, -10e-3]], np.float32)
    plan, g = make_case(cen, sen, 400, 0.1e-3)
    A = np.array([0.8], np.float32)
    sigma = np.array([0.07e-3], np.float32)
    check_forward(plan, g, A, sigma, "1x1")
    check_adjoint(plan, g, A, sigma, I.standard_normal((1, 400), seed=1), "1x1")


def test_sigma_violations_are_counted(toy):
    w, plan, g = toy
    before = plan.sigma_violations()
    sigma = np.full(w.n_kernels, w.sigma, np.float32)
    sigma[[3, 70, 900]] = [2 * w.sigma, -1.0, 0.0]
    plan.forward(dev(np.ones(w.n_kernels, np.float32)), dev(sigma))
    assert plan.sigma_violations() - before == 3


def test_mid_workload_full(request):
    _say("case: mid workload (64^3 kernels, 512 sensors, 2048 samples)")
    w, plan, g = workload_case("mid")
    A = I.phantom(w)
    sigma = np.full(w.n_kernels, w.sigma, np.float32)
    check_forward(plan, g, A, sigma, "mid")
    delta = I.standard_normal((w.n_sensors, w.n_samples), seed=31)
    check_adjoint(plan, g, A, sigma, delta, "mid")


def test_paper_scale_sampled():
    """8,388,608 kernels x 1024 sensors x 4096 samples: the forward on 16
    sensors and the adjoint on 131,072 kernels (every 64th) against the
    oracle, and the sigma-gradient against central differences of the oracle
    loss <y, delta> at 64 random kernels."""
    _say("case: paper workload (256x256x128 kernels, 1024 sensors, 4096 samples)")
    w, plan, g = workload_case("paper")
    A = I.phantom(w)
    sigma = I.uniform(w.n_kernels, seed=12, lo=0.5 * w.smax, hi=w.smax)
    y = host(plan.forward(dev(A), dev(sigma)))
    rows = np.random.default_rng(13).choice(w.n_sensors, 16, replace=False)
    ref = O.forward(g.subset_sensors(rows), A, sigma.astype(np.float64))
    err = rel_l2(y[rows], ref)
    _say(f"  forward (16 sensors) rel L2 {err:.3e}")
    assert err <= TOL
    delta = I.standard_normal((w.n_sensors, w.n_samples), seed=14)
    gA, gS = plan.adjoint(dev(A), dev(sigma), dev(delta))
    gA, gS = host(gA), host(gS)
    ks = np.arange(0, w.n_kernels, 64)
    rA, rS = O.adjoint(g.subset_kernels(ks), A[ks], sigma[ks].astype(np.float64),
                       delta.astype(np.float64))
    eA, eS = rel_l2(gA[ks], rA), rel_l2(gS[ks], rS)
    _say(f"  adjoint (131072 kernels) gA {eA:.3e} gsigma {eS:.3e}")
    assert eA <= TOL and eS <= TOL
    # central differences of L(sigma_k) = <y(sigma), delta> at 64 kernels
    pick = np.random.default_rng(15).choice(w.n_kernels, 64, replace=False)
    d64 = delta.astype(np.float64)
    fd = []
    for k in pick:
        gk = g.subset_kernels([k])
        h = 1e-6 * float(sigma[k])
        lp = np.sum(O.forward(gk, [A[k]], [float(sigma[k]) + h]) * d64)
        lm = np.sum(O.forward(gk, [A[k]], [float(sigma[k]) - h]) * d64)
        fd.append((lp - lm) / (2 * h))
    fd = np.array(fd)
    efd = np.abs(gS[pick] - fd) / np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())
    _say(f"  gsigma vs central differences: max rel {efd.max():.3e}")
    assert efd.max() <= 1e-3


@pytest.mark.parametrize("spread", [0.0, 0.05])
def test_paper_scale_at_the_benchmark_sigma(spread):
    """The configuration the benchmark times: 1024-kernel forward tiles with
    four waves, sigma = 0.05 mm (9-tap windows, the unrolled forward and
    gather) uniform or spread by +-5 % (8 or 9 taps: the ninth tap masked per
    pair, and the adjoint's ranking by tap count).  Forward on 16 sensors,
    adjoint (A and sigma) on 131,072 kernels."""
    _say(f"case: paper workload at sigma = 0.05 mm, spread {spread}")
    w, plan, g = workload_case("paper")
    info = plan.info()
    assert info["fwd_tile"] == 1024 and info["fwd_waves"] == 4 and info["adj_tile"] == 256
    A = I.phantom(w)
    sigma = np.full(w.n_kernels, w.sigma, np.float32)
    if spread:
        sigma = (sigma * I.uniform(w.n_kernels, seed=16, lo=1 - spread, hi=1 + spread))
        sigma = sigma.astype(np.float32)
    taps = np.floor(2 * 3.0 * sigma.astype(np.float64) / (w.c_sound * w.dt)) + 1
    _say(f"  taps per pair: {sorted(set(taps.astype(int).tolist()))}")
    y = host(plan.forward(dev(A), dev(sigma)))
    rows = np.random.default_rng(17).choice(w.n_sensors, 16, replace=False)
    ref = O.forward(g.subset_sensors(rows), A, sigma.astype(np.float64))
    err = rel_l2(y[rows], ref)
    _say(f"  forward (16 sensors) rel L2 {err:.3e}")
    assert np.abs(ref).max() > 0 and err <= TOL
    delta = I.standard_normal((w.n_sensors, w.n_samples), seed=18)
    gA, gS = plan.adjoint(dev(0.5 * A + 0.1), dev(sigma), dev(delta))
    gA, gS = host(gA), host(gS)
    ks = np.arange(5, w.n_kernels, 64)
    A2 = (0.5 * A + 0.1).astype(np.float32)
    rA, rS = O.adjoint(g.subset_kernels(ks), A2[ks], sigma[ks].astype(np.float64),
                       delta.astype(np.float64))
    eA, eS = rel_l2(gA[ks], rA), rel_l2(gS[ks], rS)
    _say(f"  adjoint ({ks.size} kernels) gA {eA:.3e} gsigma {eS:.3e}")
    assert eA <= TOL and eS <= TOL


def test_filter_and_float64_blocks_in_one_plan():
    """Two clusters: a dense one whose blocks take the float32 window filter
    and a sparse one a few block radii from the sensors, whose blocks are
    decided in float64 throughout; both operators against the oracle, and
    adjointness of the GPU pair (the forward and the adjoint run the same
    window arithmetic for every pair)."""
    _say("case: dense + sparse clusters (filter and float64 blocks)")
    rng = np.random.default_rng(21)
    dense = rng.uniform(-0.75e-3, 0.75e-3, (1000, 3))
    sparse = rng.uniform(-2e-3, 2e-3, (150, 3)) + np.array([6e-3, 0.0, 0.0])
    cen = np.concatenate([dense, sparse]).astype(np.float32)
    sen = I.fibonacci_hemisphere(90, 14e-3)
    smax = 0.08e-3
    plan, g = make_case(cen, sen, 1024, smax, fwd_tile=64, adj_tile=64)
    nf64, steps = plan.filter_stats()
    _say(f"  blocks in float64: {nf64} of {plan.info()['adj_tiles']}, filter steps <= {steps}")
    assert 0 < nf64 < plan.info()["adj_tiles"] and steps > 0
    A = I.uniform(len(cen), seed=22, lo=-0.5, hi=1.0)
    sigma = I.uniform(len(cen), seed=23, lo=0.4 * smax, hi=smax)
    check_forward(plan, g, A, sigma, "two clusters")
    delta = I.standard_normal((len(sen), 1024), seed=24)
    check_adjoint(plan, g, A, sigma, delta, "two clusters")
    x = I.uniform(len(cen), seed=25)
    Ax = host(plan.forward(dev(x), dev(sigma)))
    ATy, _ = plan.adjoint(dev(x), dev(sigma), dev(delta), want_sigma=False)
    lhs = float(np.sum(Ax * delta.astype(np.float64)))
    rhs = float(np.dot(x.astype(np.float64), host(ATy)))
    bar = dot_test_bound(Ax, delta)
    _say(f"  <Ax, y> {lhs:.9e}  <x, A^T y> {rhs:.9e}  |diff| {abs(lhs - rhs):.2e}  bar {bar:.2e}")
    assert abs(lhs - rhs) <= bar


@pytest.mark.parametrize("name", ["toy", "paper"])
def test_deterministic_forward_is_bitwise_reproducible(name):
    """With the plan's deterministic flush, two forwards of the same input are
    equal bit for bit (the float-atomic flush is not), and parity with the
    oracle still holds."""
    _say(f"case: deterministic forward, {name} workload")
    w = I.WORKLOADS[name]
    cen, sen = I.geometry_arrays(w)
    from paper_2602_03893_amd import Plan
    plan = Plan(cen, sen, w.n_samples, w.dt, w.c_sound, n_sigma=w.n_sigma, sigma_max=w.smax,
                deterministic=True)
    g = O.Geometry(cen, sen, w.n_samples, w.dt, w.t0, w.c_sound, w.n_sigma)
    A = I.phantom(w)
    if name == "toy":
        A = (A * I.uniform(w.n_kernels, seed=26, lo=-1.0, hi=1.0)).astype(np.float32)
    sigma = (w.sigma * I.uniform(w.n_kernels, seed=27, lo=0.9, hi=1.0)).astype(np.float32)
    y1 = host(plan.forward(dev(A), dev(sigma)))
    y2 = host(plan.forward(dev(A), dev(sigma)))
    assert np.array_equal(y1, y2)
    rows = np.arange(w.n_sensors) if name == "toy" else \
        np.random.default_rng(28).choice(w.n_sensors, 16, replace=False)
    ref = O.forward(g.subset_sensors(rows), A, sigma.astype(np.float64))
    err = rel_l2(y1[rows], ref)
    _say(f"  bitwise equal over two runs; forward rel L2 {err:.3e}")
    assert err <= TOL


def test_prepared_calls_match_and_are_refused_after_assa(toy):
    """gpair_prepare + the _prepared operators give the one-call results (the
    adjoint bit for bit; the forward to its float-atomic flush order), and a
    _prepared call after an ASSA call on the plan is refused."""
    from paper_2602_03893_amd import GpairError
    w, plan, g = toy
    A = I.uniform(w.n_kernels, seed=41, lo=-1.0, hi=1.0)
    sigma = I.uniform(w.n_kernels, seed=42, lo=0.5 * w.sigma, hi=w.sigma)
    delta = I.standard_normal((w.n_sensors, w.n_samples), seed=43)
    y1 = host(plan.forward(dev(A), dev(sigma)))
    a1, s1 = plan.adjoint(dev(A), dev(sigma), dev(delta))
    a1, s1 = host(a1), host(s1)
    plan.prepare(dev(A), dev(sigma))
    y2 = host(plan.forward_prepared())
    a2, s2 = plan.adjoint_prepared(dev(delta))
    assert rel_l2(y2, y1) <= 1e-6
    assert np.array_equal(host(a2), a1) and np.array_equal(host(s2), s1)
    plan.assa_forward(dev(np.abs(A)), w.sigma)
    with pytest.raises(GpairError, match="INVALID_ARG"):
        plan.forward_prepared()
    plan.prepare(dev(A), dev(sigma))
    assert rel_l2(host(plan.forward_prepared()), y1) <= 1e-6
