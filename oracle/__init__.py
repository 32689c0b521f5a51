"""Float64 CPU oracle of the GPAIR hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code with
the HIP path (``paper_2602_03893_amd``) and neither imports the other; the only
common module is the seeded input generator ``paper_2602_03893_amd.inputs``,
which holds none of the method's arithmetic and is imported by the tests, not by
this package.

Contents
 - ``ops``      forward / adjoint / sigma-gradient / centre gradient of the
                direct operator (C, float64, OpenMP), Eq. (single_forward) with
                the n_sigma window.
 - ``physics``  closed forms of the Methods derivation (sphere integral,
                two-term pressure) and their numerical Poisson-integral checks.
 - ``solvers``  relative residual, power iteration, projected gradient and Adam
                loops in float64 on top of ``ops``.
 - ``assa``     the ASSA operators (three stages as defined, and per pair).
 - ``objective`` the non-negativity parameterisation, the vessel continuity
                regulariser (value and gradient), the warm-restart schedule and
                the full reconstruction loop with all three.
 - ``nn``       the warm-start network's layers and whole forward/backward.

Pins (what each function is checked against, in ``tests/``):
 - ``ops.forward``   numerical Poisson integral, Eq. (pa_wave), by quadrature
                     (independent of the closed form); special values; linearity;
                     translation / rotation invariance; window edges.
 - ``ops.adjoint``   the dot-product test <A x, y> = <x, A^T y> against the pinned
                     forward; gA and gsigma against central finite differences of
                     the pinned forward.
 - ``ops.adjoint_centres``  central differences of the pinned forward in float32
                     centres; torch autograd of an independent torch
                     formulation over the same windows.
 - ``ops.forward_aniso`` / ``ops.adjoint_aniso``  (anisotropic kernels) the
                     isotropic case against ``ops.forward`` / ``ops.adjoint``;
                     exact axis permutations and reflections; the closed form
                     of ``physics`` at every sample; convergence to the
                     numerical Poisson integral of the anisotropic p0 as
                     sigma/r -> 0; the dot-product test; central differences
                     in the six covariance parameters
                     (tests/test_oracle_aniso.py).
 - ``ops.adjoint_aniso_centres``  the isotropic case against
                     ``ops.adjoint_centres``; central differences of the pinned
                     anisotropic forward in float32 centres; exact axis
                     permutations.
 - ``physics``       Gauss-Legendre quadrature of the surface integral and a
                     numerical derivative of Eq. (pa_wave) (isotropic and
                     anisotropic p0).
 - ``solvers.pgd``   converges to scipy's NNLS solution (a different algorithm).
 - ``solvers.adam``  matches torch.optim.Adam (a library implementation) step by
                     step on the same gradients.
 - ``assa``          tests/test_oracle_assa.py; ``objective``
                     tests/test_oracle_objective.py; ``nn`` tests/test_oracle_nn.py.
"""
from . import ops, physics, solvers  # noqa: F401
