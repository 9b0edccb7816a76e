"""Reference of the RK(5,3) pseudo-time driver around the linear solve.

Paper:
  * section "Generalized RK Scheme for The Mean Flow" (eqn:rk): per pseudo-time step n,
    Q^(0) = Q^n and, for stages k = 1..5, Q^(k) = Q^(0) - Gamma alpha_k K^-1 R^(k)
    (the multigrid term R* is zero for the implicit scheme), Q^(n+1) = Q^(5); Gamma =
    1/eps (implicit) or sigma_CFL (explicit); the stage coefficients are the table of
    the hybrid RK(5,3) scheme, alpha = (1/4, 1/6, 3/8, 1/2, 1) and beta = (1, 0, 14/25,
    0, 11/25) for the viscous part;
  * section "Generalized RK Scheme for Time-Linearized Harmonic Flows" (eqn:rk_lin): the
    same stages with the harmonic perturbation, its residual and K_l = K + i omega_l V I;
  * section "Solution Update": each stage solves A x = B with A = K/(Gamma alpha_k) and
    B = -R^(k), i.e. K x = -Gamma alpha_k R^(k), inexactly by ILU-preconditioned
    relaxation (paper mode: 1e-2 relative, at most 10 sweeps);
  * K is assembled once per pseudo-time step (at Q^n) and kept through the stages.

Residual stand-ins (no Hydra code here): the mean flow's R is the first-order Rusanov
residual of assemble.residual with dissipation coefficients and far-field state taken
from the state it is evaluated at; it has no viscous part, so the beta blending of the
viscous residual leaves it unchanged.  The harmonic residual is the linearisation
R_l(Q^) = (J + i omega_l V) Q^ - f^ about the assembly state, with f^ a given forcing.
"""
import numpy as np

from . import assemble, solve

ALPHA = (0.25, 1.0 / 6.0, 0.375, 0.5, 1.0)
BETA = (1.0, 0.0, 14.0 / 25.0, 0.0, 11.0 / 25.0)


def gamma(scheme, eps, sigma):
    return 1.0 / eps if scheme == "implicit" else sigma


def nonlinear_residual(mesh, Q, Qff=None):
    """R(Q): Rusanov residual with the dissipation and far field of the state itself."""
    lam_e, lam_f, Qf = assemble.frozen_lambdas(Q, mesh.edges, mesh.area, mesh.bface_cell, mesh.bface_area, Qff)
    return assemble.residual(Q, mesh.edges, mesh.area, mesh.bface_cell, mesh.bface_area, lam_e, lam_f, Qf)


def mean_step(mesh, Q, colour, eps=0.6, sigma=50.0, scheme="implicit", rtol=1e-2, max_sweeps=10, kind="DILU",
              Qff=None, part=None):
    """One pseudo-time step of the mean flow; returns (Q^(n+1), ||R(Q^n)||).  part: the
    stage solves use K with the couplings between partitions dropped."""
    K = assemble.assemble(mesh, Q, eps, sigma, scheme, Qff)
    if part is not None:
        K = solve.partition_dropped(K, part)
    G = gamma(scheme, eps, sigma)
    zero = np.zeros(mesh.n_zones)
    Q0 = np.asarray(Q, np.float64)
    Qk = Q0.copy()
    r0 = None
    for k in range(5):
        R = nonlinear_residual(mesh, Qk, Qff)
        if k == 0:
            r0 = float(np.linalg.norm(R))
        b = (-G * ALPHA[k] * R).astype(np.complex128)
        x, _ = solve.richardson(K, mesh.volume, mesh.zone, zero, b, colour, kind, rtol=rtol, max_sweeps=max_sweeps)
        Qk = Q0 + x.real
    return Qk, r0


def harmonic_residual(J, mesh, omega_row, Qh, fh):
    """R_l(Q^) = (J + i omega V) Q^ - f^."""
    Ds = solve.system_diag(J, mesh.volume, mesh.zone, omega_row)
    return solve.apply(J, Ds, Qh) - fh


def harmonic_step(mesh, Q, Qh, fh, omega_row, colour, eps=0.6, sigma=50.0, scheme="implicit", rtol=1e-2,
                  max_sweeps=10, kind="DILU", Qff=None, frozen=False, part=None):
    """One pseudo-time step of a harmonic about the state Q; returns (Q^(n+1), ||R_l||).
    frozen: frozen turbulence, the 5x5 sub-system of J and K with the turbulence
    perturbation held at 0.  part: the stage solves use K with the couplings between
    partitions dropped (the residual keeps the whole J)."""
    J = assemble.residual_jacobian(Q, mesh.edges, mesh.area, mesh.bface_cell, mesh.bface_area, Qff)
    K = assemble.preconditioner_matrix(J, eps, sigma, scheme)
    if part is not None:
        K = solve.partition_dropped(K, part)
    G = gamma(scheme, eps, sigma)
    Q0 = np.asarray(Qh, np.complex128).copy()
    if frozen:
        Q0[:, 5] = 0.0
    Qk = Q0.copy()
    lin = solve.richardson_frozen if frozen else solve.richardson
    r0 = None
    for k in range(5):
        if frozen:
            R = np.zeros_like(Q0)
            R[:, :5] = harmonic_residual(solve.frozen_turbulence(J), mesh, omega_row, Qk[:, :5], fh[:, :5])
        else:
            R = harmonic_residual(J, mesh, omega_row, Qk, fh)
        if k == 0:
            r0 = float(np.linalg.norm(R))
        x, _ = lin(K, mesh.volume, mesh.zone, omega_row, -G * ALPHA[k] * R, colour, kind, rtol=rtol,
                   max_sweeps=max_sweeps)
        Qk = Q0 + x
    return Qk, r0
