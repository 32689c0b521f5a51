"""Float64 oracle of the paper's full objective (NPC, VCR, CAWR) and of
Algorithm 2 with all of them.

TEST INFRASTRUCTURE ONLY (see the package docstring).

arXiv 2602.03893, Methods:
 - "Nonnegative parameterization constraint": x = phi(z) = (z + eps)^2 with
   eps = 1e-8, dL/dz = dL/dx * 2 (z + eps);
 - "Vessel continuity regularization": R_VCR = R_H + beta R_TV with
   R_H  = sum_i sqrt( sum_{p,q in {x,y,z}} (D_pq x_i)^2 + eps ),
   R_TV = sum_i sqrt( sum_{d in {x,y,z}} (D_d x_i)^2 + eps );
 - "Optimization formulation and algorithm": the objective, Adam, the cosine
   annealing warm restart schedule, and the GPAIR algorithm.

Readings (the paper is silent on the discretisation and the boundary):
 - volumes are stored [iz][iy][ix] (x fastest); differences use unit spacing;
 - D_d x_i = x[i + e_d] - x[i]; D_pp x_i = x[i + e_p] - 2 x[i] + x[i - e_p];
   D_pq x_i = x[i + e_p + e_q] - x[i + e_p] - x[i + e_q] + x[i] (p != q, so
   D_pq = D_qp and each mixed term enters the Frobenius sum twice);
 - a difference whose stencil leaves the volume is 0 (so the first differences
   are zero on the far faces, the Neumann condition), and every voxel still
   contributes sqrt(eps);
 - the eps inside the square roots is the same 1e-8 as the NPC's;
 - the schedule follows the cited SGDR: period i has length T_0 T_mult^i and
   T_cur counts iterations since the last restart.  For T_mult = 1 this is the
   printed formula (T_cur = t mod T_0, T_i = T_0); for T_mult > 1 the printed
   formula, read literally, never completes a period after the first, which
   contradicts its own description of a warm restart.

``vcr_value`` and ``vcr_grad`` evaluate the definitions with numpy shifts; the
gradient is the transpose of each difference operator applied to the
normalised differences, derived by hand.  tests/test_oracle_objective.py pins
them against brute-force loops, torch autograd, central differences and closed
forms; ``cawr`` against torch's CosineAnnealingWarmRestarts.
"""
import math

import numpy as np

from . import ops, solvers

NPC_EPS = 1e-8


def npc_map(z, eps=NPC_EPS):
    z = np.asarray(z, dtype=np.float64)
    return (z + eps) ** 2


def npc_grad(z, gx, eps=NPC_EPS):
    return np.asarray(gx, dtype=np.float64) * 2.0 * (np.asarray(z, dtype=np.float64) + eps)


# --- difference operators on a [nz][ny][nx] volume --------------------------
# axis index of the volume for the coordinate letters
_AX = {"x": 2, "y": 1, "z": 0}


def _shift(a, axis, k):
    """b[i] = a[i + k e_axis], 0 where i + k e_axis leaves the volume."""
    b = np.zeros_like(a)
    n = a.shape[axis]
    if abs(k) >= n:
        return b
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if k >= 0:
        src[axis] = slice(k, n)
        dst[axis] = slice(0, n - k)
    else:
        src[axis] = slice(0, n + k)
        dst[axis] = slice(-k, n)
    b[tuple(dst)] = a[tuple(src)]
    return b


def _inside(shape, axis, k):
    """Mask of the voxels i with i + k e_axis inside the volume."""
    return _shift(np.ones(shape), axis, k) > 0


def differences(x):
    """The three first, three pure second and three mixed second differences
    (dicts keyed 'x', 'xx', 'xy', ...), zero where the stencil leaves the volume."""
    x = np.asarray(x, dtype=np.float64)
    sh = x.shape
    first, pure, mixed = {}, {}, {}
    for d, a in _AX.items():
        first[d] = (_shift(x, a, 1) - x) * _inside(sh, a, 1)
        m = _inside(sh, a, 1) & _inside(sh, a, -1)
        pure[d + d] = (_shift(x, a, 1) - 2.0 * x + _shift(x, a, -1)) * m
    for p, q in (("x", "y"), ("x", "z"), ("y", "z")):
        ap, aq = _AX[p], _AX[q]
        xpq = _shift(_shift(x, ap, 1), aq, 1)
        m = _shift(_inside(sh, aq, 1).astype(float), ap, 1) > 0  # i + e_p + e_q inside
        m &= _inside(sh, ap, 1)
        mixed[p + q] = (xpq - _shift(x, ap, 1) - _shift(x, aq, 1) + x) * m
    return first, pure, mixed


def vcr_norms(x, eps=NPC_EPS):
    first, pure, mixed = differences(x)
    s_t = sum(v * v for v in first.values())
    s_h = sum(v * v for v in pure.values()) + 2.0 * sum(v * v for v in mixed.values())
    return np.sqrt(s_h + eps), np.sqrt(s_t + eps)


def vcr_value(x, beta, eps=NPC_EPS):
    """R_H(x) + beta R_TV(x)."""
    n_h, n_t = vcr_norms(x, eps)
    return float(n_h.sum() + beta * n_t.sum())


def vcr_grad(x, beta, eps=NPC_EPS):
    """dR_VCR/dx: the transposes of the difference operators applied to the
    normalised differences."""
    x = np.asarray(x, dtype=np.float64)
    first, pure, mixed = differences(x)
    n_h, n_t = vcr_norms(x, eps)
    g = np.zeros_like(x)
    for d, a in _AX.items():
        u = first[d] / n_t  # dn_t / dD_d
        g += beta * (_shift(u, a, -1) - u)  # transpose of x[i + e_d] - x[i]
        w = pure[d + d] / n_h  # dn_h / dD_dd
        g += _shift(w, a, -1) - 2.0 * w + _shift(w, a, 1)
    for p, q in (("x", "y"), ("x", "z"), ("y", "z")):
        ap, aq = _AX[p], _AX[q]
        w = 2.0 * mixed[p + q] / n_h  # dn_h / dD_pq (the term counts twice)
        g += (_shift(_shift(w, ap, -1), aq, -1) - _shift(w, ap, -1) - _shift(w, aq, -1) + w)
    return g


def cawr(t, eta_min, eta_max, T0, Tmult):
    """Learning rate at iteration t (0-based) of the warm-restart schedule."""
    start, period = 0, int(T0)
    while t >= start + period:
        start += period
        period *= int(Tmult)
    t_cur = t - start
    return eta_min + 0.5 * (eta_max - eta_min) * (1.0 + math.cos(math.pi * t_cur / period))


def gpair(g, sigma, b, grid, iters, lam, beta, eta_min, eta_max, T0, Tmult,
          z0=None, npc_eps=NPC_EPS, reg_eps=NPC_EPS, beta1=0.9, beta2=0.999, adam_eps=1e-8):
    """Algorithm 2 with NPC, VCR and CAWR on the data term 0.5 ||A x - b||^2 /
    ||b||^2 (the normalisation of the library's solver; lambda is relative to
    it).  grid = (nx, ny, nz) of the kernel lattice in caller order.
    Returns (x, z, rho history of length iters + 1)."""
    nx, ny, nz = grid
    M = nx * ny * nz
    z = np.zeros(M) if z0 is None else np.array(z0, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb2 = float(np.dot(b.ravel(), b.ravel()))
    m = np.zeros(M)
    v = np.zeros(M)
    hist = []
    for t in range(iters):
        x = npc_map(z, npc_eps)
        r = ops.forward(g, x, s) - b
        hist.append(float(np.sqrt(np.dot(r.ravel(), r.ravel()) / nb2)))
        gx, _ = ops.adjoint(g, x, s, r / nb2, want_sigma=False)
        if lam != 0.0:
            gx = gx + lam * vcr_grad(x.reshape(nz, ny, nx), beta, reg_eps).ravel()
        gz = npc_grad(z, gx, npc_eps)
        lr = cawr(t, eta_min, eta_max, T0, Tmult)
        z = solvers.adam_step(z, gz, m, v, t + 1, lr, beta1, beta2, adam_eps, -np.inf, np.inf)
    x = npc_map(z, npc_eps)
    hist.append(solvers.rel_residual(g, x, s, b))
    return x, z, hist
