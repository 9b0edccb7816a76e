"""Convective flux of the Euler equations plus one convected turbulence variable, its
analytic Jacobian, and the Rusanov (local Lax-Friedrichs) spectral radius.

Paper: section "Brief Description of Hydra" (edge-based finite volume, SA turbulence
model, frozen turbulence for the linearised solver) and section "Generalized RK Scheme
for The Mean Flow" (J is a first-order approximation of dR/dQ built from immediate
neighbours).  Hydra's first-order JST matrix dissipation is replaced by the Rusanov flux
(reading recorded with the design notes); the spectral radius is frozen, i.e. not
differentiated.

State Q = (rho, rho u, rho v, rho w, rho E, rho nu~); ideal gas with gamma = 1.4.
All functions are vectorised over a leading axis and work for complex dtypes too (so the
complex-step derivative pin can call them).
"""
import numpy as np

GAMMA = 1.4


def primitives(Q):
    """rho, velocity [.,3], pressure, total enthalpy H, nu~ from the conservative state."""
    rho = Q[..., 0]
    u = Q[..., 1:4] / rho[..., None]
    E = Q[..., 4]
    q2 = np.sum(u * u, axis=-1)
    p = (GAMMA - 1.0) * (E - 0.5 * rho * q2)
    H = (E + p) / rho
    nut = Q[..., 5] / rho
    return rho, u, p, H, nut


def flux(Q, S):
    """F(Q; S) = [rho U, rho u U + p S_x, rho v U + p S_y, rho w U + p S_z, (rho E + p) U,
    rho nu~ U] with U = u . S (S an area vector, not normalised)."""
    rho, u, p, H, nut = primitives(Q)
    U = np.sum(u * S, axis=-1)
    F = np.empty(np.broadcast_shapes(Q.shape, S.shape[:-1] + (6,)), dtype=np.result_type(Q, S))
    F[..., 0] = rho * U
    F[..., 1:4] = Q[..., 1:4] * U[..., None] + p[..., None] * S
    F[..., 4] = (Q[..., 4] + p) * U
    F[..., 5] = Q[..., 5] * U
    return F


def flux_jacobian(Q, S):
    """A(Q; S) = dF/dQ, shape [..., 6, 6], derived by hand from ``flux``:
    with phi = (gamma-1)|u|^2/2 and U = u.S,
      row 0      : [0, S^T, 0, 0]
      row 1+a    : [-u_a U + phi S_a, U e_a^T + u_a S^T - (gamma-1) S_a u^T, (gamma-1) S_a, 0]
      row 4      : [U (phi - H), H S^T - (gamma-1) U u^T, gamma U, 0]
      row 5      : [-nu~ U, nu~ S^T, 0, U]
    """
    rho, u, p, H, nut = primitives(Q)
    U = np.sum(u * S, axis=-1)
    g1 = GAMMA - 1.0
    phi = 0.5 * g1 * np.sum(u * u, axis=-1)
    shp = np.broadcast_shapes(U.shape, S.shape[:-1])
    A = np.zeros(shp + (6, 6), dtype=np.result_type(Q, S))
    A[..., 0, 1:4] = S
    for a in range(3):
        A[..., 1 + a, 0] = -u[..., a] * U + phi * S[..., a]
        for b in range(3):
            A[..., 1 + a, 1 + b] = u[..., a] * S[..., b] - g1 * S[..., a] * u[..., b]
        A[..., 1 + a, 1 + a] += U
        A[..., 1 + a, 4] = g1 * S[..., a]
    A[..., 4, 0] = U * (phi - H)
    for b in range(3):
        A[..., 4, 1 + b] = H * S[..., b] - g1 * U * u[..., b]
    A[..., 4, 4] = GAMMA * U
    A[..., 5, 0] = -nut * U
    A[..., 5, 1:4] = nut[..., None] * S
    A[..., 5, 5] = U
    return A


def spectral_radius(Q, S):
    """|u . S| + a |S|: largest eigenvalue magnitude of A(Q; S)."""
    rho, u, p, H, nut = primitives(Q)
    a = np.sqrt(GAMMA * p / rho)
    return np.abs(np.sum(u * S, axis=-1)) + a * np.linalg.norm(S, axis=-1)


def rusanov_lambda(Qa, Qb, S):
    """Frozen Rusanov dissipation coefficient of a face: the larger end spectral radius."""
    return np.maximum(spectral_radius(Qa, S), spectral_radius(Qb, S))
