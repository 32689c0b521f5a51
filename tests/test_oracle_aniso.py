"""Pins of the oracle's anisotropic kernels (learnable anisotropic Gaussians,
the paper's stated future work): the isotropic special case is
Eq. (single_forward) and its gradients; exact axis permutations and
reflections of the geometry with the covariance transformed alike leave the
traces unchanged; the far-field closed form converges to the numerical
Poisson integral of the anisotropic p0 (Eq. (pa_wave), no closed form used)
as sigma/r -> 0; the adjoint is the transpose; the covariance gradient
matches central differences of the forward."""
import numpy as np
import pytest

from oracle import ops as O
from oracle import physics as P
from paper_2602_03893_amd import inputs as I

pytestmark = pytest.mark.filterwarnings("ignore")


def random_cov(m, lo, hi, seed):
    """Covariances R diag(s^2) R^T, s ~ U[lo, hi], R uniform rotations."""
    rng = np.random.default_rng(seed)
    out = np.empty((m, 6))
    for k in range(m):
        q, rr = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(rr))
        c = q @ np.diag(rng.uniform(lo, hi, 3) ** 2) @ q.T
        out[k] = [c[0, 0], c[1, 1], c[2, 2], c[0, 1], c[0, 2], c[1, 2]]
    return out


def full(s6):
    xx, yy, zz, xy, xz, yz = s6
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def cloud(m, nd, nt=512, seed=0):
    rng = np.random.default_rng(seed)
    cen = rng.uniform(-1e-3, 1e-3, (m, 3)).astype(np.float32)
    sen = I.fibonacci_hemisphere(nd, 10e-3)
    g = O.Geometry(cen, sen, nt, I.DT, 0.0, I.C_SOUND, 3.0)
    A = rng.uniform(-1.0, 1.0, m)
    return cen, sen, g, A


def test_isotropic_covariance_is_eq_single_forward():
    cen, sen, g, A = cloud(150, 12, seed=1)
    rng = np.random.default_rng(2)
    sig = rng.uniform(0.04e-3, 0.1e-3, 150)
    s6 = np.zeros((150, 6))
    s6[:, 0] = s6[:, 1] = s6[:, 2] = sig * sig
    y_iso = O.forward(g, A, sig)
    y_an = O.forward_aniso(g, A, s6)
    assert np.abs(y_iso).max() > 0
    assert np.max(np.abs(y_an - y_iso)) <= 1e-12 * np.abs(y_iso).max()
    delta = rng.standard_normal((12, 512))
    ga_iso, gs_iso = O.adjoint(g, A, sig, delta)
    ga_an, gS = O.adjoint_aniso(g, A, s6, delta)
    assert np.max(np.abs(ga_an - ga_iso)) <= 1e-12 * np.abs(ga_iso).max()
    # Sigma = sigma^2 I: d/dsigma = 2 sigma (g_xx + g_yy + g_zz)
    gs_from = 2.0 * sig * (gS[:, 0] + gS[:, 1] + gS[:, 2])
    assert np.max(np.abs(gs_from - gs_iso)) <= 1e-10 * np.abs(gs_iso).max()


def test_axis_permutation_and_reflection():
    """(x, y, z) -> (y, z, -x) is exact in float32; the covariance maps to
    M Sigma M^T.  A swapped or mis-signed covariance entry changes sigma_n for
    most pairs, so this pins the entry order."""
    cen, sen, g, A = cloud(120, 10, seed=3)
    s6 = random_cov(120, 0.03e-3, 0.1e-3, seed=4)
    M = np.array([[0, 1, 0], [0, 0, 1], [-1, 0, 0]], dtype=np.float64)
    cen2 = (cen.astype(np.float64) @ M.T).astype(np.float32)
    sen2 = (np.asarray(sen, np.float64) @ M.T).astype(np.float32)
    s62 = np.empty_like(s6)
    for k in range(120):
        c = M @ full(s6[k]) @ M.T
        s62[k] = [c[0, 0], c[1, 1], c[2, 2], c[0, 1], c[0, 2], c[1, 2]]
    g2 = O.Geometry(cen2, sen2, 512, I.DT, 0.0, I.C_SOUND, 3.0)
    y1 = O.forward_aniso(g, A, s6)
    y2 = O.forward_aniso(g2, A, s62)
    assert np.abs(y1).max() > 0
    assert np.max(np.abs(y1 - y2)) <= 1e-12 * np.abs(y1).max()
    # the unpermuted covariance with the moved geometry gives other traces
    y3 = O.forward_aniso(g2, A, s6)
    assert np.max(np.abs(y1 - y3)) > 1e-3 * np.abs(y1).max()
    delta = np.random.default_rng(5).standard_normal((10, 512))
    ga1, gS1 = O.adjoint_aniso(g, A, s6, delta)
    ga2, gS2 = O.adjoint_aniso(g2, A, s62, delta)
    assert np.max(np.abs(ga1 - ga2)) <= 1e-12 * np.abs(ga1).max()
    # the matrix gradient transforms like Sigma: G2 = M G1 M^T (in matrix form,
    # off-diagonal parameters carry twice the entry)
    def mat(gs):
        xx, yy, zz, xy, xz, yz = gs
        return np.array([[xx, xy / 2, xz / 2], [xy / 2, yy, yz / 2], [xz / 2, yz / 2, zz]])
    worst = max(np.max(np.abs(M @ mat(gS1[k]) @ M.T - mat(gS2[k]))) for k in range(120))
    assert worst <= 1e-10 * np.abs(gS1).max()


def test_far_field_converges_to_the_poisson_integral():
    """The far-field closed form against the numerical Poisson integral of the
    anisotropic p0 (quadrature over the sphere, no closed form): the error
    falls like sigma/r (halves as r doubles) and is below 2.5e-3 of the peak at
    40 mm for axes up to 0.1 mm; with an isotropic covariance the two agree to
    quadrature accuracy."""
    rng = np.random.default_rng(0)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    cov = q @ np.diag([0.04e-3, 0.07e-3, 0.1e-3]) ** 2 @ q.T
    v = I.C_SOUND
    direction = np.array([0.3, 0.5, 0.81]) / np.linalg.norm([0.3, 0.5, 0.81])
    errs = []
    for r in (10e-3, 20e-3, 40e-3):
        c = r * direction
        sn = np.sqrt(direction @ cov @ direction)
        ts = (r + np.array([-2.0, -1.0, -0.5, 0.5, 1.0, 2.0]) * sn) / v
        num = np.array([P.pressure_poisson_aniso(1.0, c, cov, t, v) for t in ts])
        far = np.array([P.pressure_far_aniso(1.0, c, cov, t, v) for t in ts])
        errs.append(np.max(np.abs(num - far)) / np.max(np.abs(far)))
    assert errs[2] < 2.5e-3
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3
    iso = np.eye(3) * (0.07e-3) ** 2
    c = 20e-3 * direction
    ts = (20e-3 + np.array([-1.0, 0.5]) * 0.07e-3) / v
    num = np.array([P.pressure_poisson_aniso(1.0, c, iso, t, v) for t in ts])
    far = np.array([P.pressure_far_aniso(1.0, c, iso, t, v) for t in ts])
    assert np.max(np.abs(num - far)) <= 1e-9 * np.max(np.abs(far))


def test_oracle_forward_is_the_far_field_form():
    """One kernel, one sensor: the oracle's trace equals the closed form at
    every in-window sample and is zero outside |d| <= 3 sigma_n."""
    cen = np.array([[0.2e-3, -0.1e-3, 0.3e-3]], np.float32)
    sen = np.array([[3e-3, 4e-3, 9e-3]], np.float32)
    g = O.Geometry(cen, sen, 512, I.DT, 0.0, I.C_SOUND, 3.0)
    s6 = random_cov(1, 0.04e-3, 0.1e-3, seed=9)
    y = O.forward_aniso(g, [0.7], s6)[0]
    u = sen[0].astype(np.float64) - cen[0].astype(np.float64)
    c = -u  # detector at the origin
    t = np.arange(512) * I.DT
    ref = np.array([P.pressure_far_aniso(0.7, c, full(s6[0]), tt, I.C_SOUND) for tt in t])
    n = u / np.linalg.norm(u)
    sn = np.sqrt(n @ full(s6[0]) @ n)
    inside = np.abs(np.linalg.norm(u) - I.C_SOUND * t) <= 3.0 * sn
    assert inside.sum() >= 5
    assert np.all(y[~inside] == 0.0)
    assert np.max(np.abs(y[inside] - ref[inside])) <= 1e-12 * np.abs(ref).max()


def test_adjoint_is_the_transpose():
    cen, sen, g, A = cloud(200, 16, seed=6)
    s6 = random_cov(200, 0.03e-3, 0.1e-3, seed=7)
    rng = np.random.default_rng(8)
    x = rng.uniform(-1, 1, 200)
    yv = rng.standard_normal((16, 512))
    lhs = np.sum(O.forward_aniso(g, x, s6) * yv)
    ga, _ = O.adjoint_aniso(g, A, s6, yv, want_sigma=False)
    rhs = np.sum(x * ga)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(O.forward_aniso(g, np.abs(x), s6)) * np.abs(yv))


def test_covariance_gradient_against_central_differences():
    """dL/dtheta of L = <A(x; Sigma), delta> for each of the six parameters,
    one kernel at a time; a step that moves a window edge across a sample is
    detected from the supports and skipped."""
    cen, sen, g, A = cloud(60, 12, seed=10)
    s6 = random_cov(60, 0.03e-3, 0.1e-3, seed=11)
    delta = np.random.default_rng(12).standard_normal((12, 512))
    _, gS = O.adjoint_aniso(g, A, s6, delta)
    checked = 0
    for k in range(0, 60, 5):
        gk = g.subset_kernels([k])
        for a in range(6):
            h = 1e-6 * (s6[k, 0] + s6[k, 1] + s6[k, 2])
            sp, sm = s6[k].copy(), s6[k].copy()
            sp[a] += h
            sm[a] -= h
            yp = O.forward_aniso(gk, [A[k]], sp[None])
            ym = O.forward_aniso(gk, [A[k]], sm[None])
            if not np.array_equal(yp != 0, ym != 0):
                continue
            fd = (np.sum(yp * delta) - np.sum(ym * delta)) / (2 * h)
            assert abs(gS[k, a] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(gS[k]).max()), (k, a)
            checked += 1
    assert checked >= 50


def test_centre_gradient_isotropic_case_and_central_differences():
    """The anisotropic centre gradient: with Sigma = sigma^2 I it equals the
    isotropic oracle's centre gradient; with random covariances it matches
    central differences of the forward in float32 centres (steps of ~4 nm; a
    step that moves a window edge across a sample is skipped)."""
    cen, sen, g, A = cloud(80, 12, seed=13)
    rng = np.random.default_rng(14)
    sig = rng.uniform(0.04e-3, 0.1e-3, 80)
    s6 = np.zeros((80, 6))
    s6[:, 0] = s6[:, 1] = s6[:, 2] = sig * sig
    delta = rng.standard_normal((12, 512))
    gc_iso = O.adjoint_centres(g, A, sig, delta)
    gc_an = O.adjoint_aniso_centres(g, A, s6, delta)
    assert np.max(np.abs(gc_an - gc_iso)) <= 1e-10 * np.abs(gc_iso).max()
    s6 = random_cov(80, 0.03e-3, 0.1e-3, seed=15)
    gc = O.adjoint_aniso_centres(g, A, s6, delta)
    checked = 0
    for k in range(0, 80, 4):
        for ax in range(3):
            cp, cm = cen[k].copy(), cen[k].copy()
            cp[ax] = np.float32(cen[k, ax] + np.float32(4e-9))
            cm[ax] = np.float32(cen[k, ax] - np.float32(4e-9))
            gp = O.Geometry(cp[None], sen, g.n_samples, g.dt, g.t0, g.c_sound, g.n_sigma)
            gm = O.Geometry(cm[None], sen, g.n_samples, g.dt, g.t0, g.c_sound, g.n_sigma)
            yp = O.forward_aniso(gp, [A[k]], s6[k][None])
            ym = O.forward_aniso(gm, [A[k]], s6[k][None])
            if not np.array_equal(yp != 0, ym != 0):
                continue
            fd = (np.sum(yp * delta) - np.sum(ym * delta)) / (float(cp[ax]) - float(cm[ax]))
            assert abs(gc[k, ax] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gc).max()), (k, ax)
            checked += 1
    assert checked >= 45


def test_centre_gradient_axis_permutation():
    """(x, y, z) -> (y, z, -x) applied to the geometry and the covariances maps
    the centre gradient by the same matrix."""
    cen, sen, g, A = cloud(60, 10, seed=16)
    s6 = random_cov(60, 0.03e-3, 0.1e-3, seed=17)
    M = np.array([[0, 1, 0], [0, 0, 1], [-1, 0, 0]], dtype=np.float64)
    cen2 = (cen.astype(np.float64) @ M.T).astype(np.float32)
    sen2 = (np.asarray(sen, np.float64) @ M.T).astype(np.float32)
    s62 = np.empty_like(s6)
    for k in range(60):
        c = M @ full(s6[k]) @ M.T
        s62[k] = [c[0, 0], c[1, 1], c[2, 2], c[0, 1], c[0, 2], c[1, 2]]
    g2 = O.Geometry(cen2, sen2, 512, I.DT, 0.0, I.C_SOUND, 3.0)
    delta = np.random.default_rng(18).standard_normal((10, 512))
    gc1 = O.adjoint_aniso_centres(g, A, s6, delta)
    gc2 = O.adjoint_aniso_centres(g2, A, s62, delta)
    assert np.max(np.abs(gc1 @ M.T - gc2)) <= 1e-10 * np.abs(gc1).max()
