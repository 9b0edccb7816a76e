"""First-order residual Jacobian J, its block diagonal P and the preconditioner matrix K.

Paper, section "Generalized RK Scheme for The Mean Flow":
  * K = P for the explicit scheme, K = P / (eps * sigma_CFL) + J for the implicit one
    (the preconditioner-matrix equation), P = diagonal block of J;
  * J = dR/dQ assembled from immediate neighbours with first-order accuracy;
  * eps = 0.6 is the suggested relaxation factor, sigma_CFL = 2 the explicit default.
The implicit CFL default here is 50 (the paper recommends 40-50 after testing 10-100,
section "Compressor Rotor-Rotor Interaction").

Residual stand-in: for interior face e = (a, b) with area vector S (a -> b)
    F_ab = 1/2 (F(Q_a; S) + F(Q_b; S)) - 1/2 lambda_e (Q_b - Q_a),  R_a += F_ab, R_b -= F_ab
and for a boundary face f of cell c with outward S_f and frozen far-field state Q_f
    R_c += 1/2 (F(Q_c; S_f) + F(Q_f; S_f)) - 1/2 lambda_f (Q_f - Q_c).
lambda is frozen (not differentiated), so
    J_aa += 1/2 A(Q_a;S) + 1/2 lambda I     J_ab = 1/2 A(Q_b;S) - 1/2 lambda I
    J_bb += -1/2 A(Q_b;S) + 1/2 lambda I    J_ba = -1/2 A(Q_a;S) - 1/2 lambda I
    J_cc += 1/2 A(Q_c;S_f) + 1/2 lambda_f I.

Matrix representation (used across the oracle):
    diag  [N, 6, 6]      K_ii
    rows, cols [2E]      directed couplings; entry 2e = (a_e, b_e), 2e+1 = (b_e, a_e)
    offd  [2E, 6, 6]     K_{rows, cols}
"""
from dataclasses import dataclass
import numpy as np

from .flux import flux, flux_jacobian, rusanov_lambda

EPS_DEFAULT = 0.6
SIGMA_DEFAULT = 50.0


@dataclass
class BlockMatrix:
    n: int
    diag: np.ndarray
    rows: np.ndarray
    cols: np.ndarray
    offd: np.ndarray

    def copy(self):
        return BlockMatrix(self.n, self.diag.copy(), self.rows.copy(), self.cols.copy(),
                           self.offd.copy())


def directed(edges):
    """rows/cols of the 2E directed couplings in the fixed convention above."""
    e = np.asarray(edges, dtype=np.int64)
    rows = np.empty(2 * e.shape[0], np.int64)
    cols = np.empty(2 * e.shape[0], np.int64)
    rows[0::2], cols[0::2] = e[:, 0], e[:, 1]
    rows[1::2], cols[1::2] = e[:, 1], e[:, 0]
    return rows, cols


def _far_field(Q, bface_cell, Qff):
    if Qff is None:
        return Q[bface_cell]
    return np.asarray(Qff)


def residual(Q, edges, area, bface_cell, bface_area, lam_e, lam_f, Qff_frozen):
    """Rusanov residual R(Q) with frozen dissipation coefficients lam_e, lam_f and a
    frozen far-field state.  Complex Q is allowed (complex-step pin)."""
    a, b = edges[:, 0], edges[:, 1]
    Fab = 0.5 * (flux(Q[a], area) + flux(Q[b], area)) - 0.5 * lam_e[:, None] * (Q[b] - Q[a])
    R = np.zeros(Q.shape, dtype=np.result_type(Q, area))
    np.add.at(R, a, Fab)
    np.add.at(R, b, -Fab)
    c = bface_cell
    if c.size:
        Ff = 0.5 * (flux(Q[c], bface_area) + flux(Qff_frozen, bface_area)) \
            - 0.5 * lam_f[:, None] * (Qff_frozen - Q[c])
        np.add.at(R, c, Ff)
    return R


def frozen_lambdas(Q, edges, area, bface_cell, bface_area, Qff=None):
    lam_e = rusanov_lambda(Q[edges[:, 0]], Q[edges[:, 1]], area)
    Qf = _far_field(Q, bface_cell, Qff)
    lam_f = rusanov_lambda(Q[bface_cell], Qf, bface_area) if bface_cell.size else np.zeros(0)
    return lam_e, lam_f, Qf


def residual_jacobian(Q, edges, area, bface_cell, bface_area, Qff=None):
    """J = dR/dQ (first order, frozen lambda) as a BlockMatrix."""
    Q = np.asarray(Q, dtype=np.float64)
    n = Q.shape[0]
    edges = np.asarray(edges, dtype=np.int64)
    a, b = edges[:, 0], edges[:, 1]
    lam_e, lam_f, Qf = frozen_lambdas(Q, edges, area, bface_cell, bface_area, Qff)
    I6 = np.eye(6)
    Aa = flux_jacobian(Q[a], area)
    Ab = flux_jacobian(Q[b], area)
    L = 0.5 * lam_e[:, None, None] * I6
    diag = np.zeros((n, 6, 6))
    np.add.at(diag, a, 0.5 * Aa + L)
    np.add.at(diag, b, -0.5 * Ab + L)
    if bface_cell.size:
        Af = flux_jacobian(Q[bface_cell], bface_area)
        np.add.at(diag, bface_cell, 0.5 * Af + 0.5 * lam_f[:, None, None] * I6)
    rows, cols = directed(edges)
    offd = np.empty((2 * edges.shape[0], 6, 6))
    offd[0::2] = 0.5 * Ab - L
    offd[1::2] = -0.5 * Aa - L
    return BlockMatrix(n, diag, rows, cols, offd)


def preconditioner_matrix(J: BlockMatrix, eps=EPS_DEFAULT, sigma=SIGMA_DEFAULT,
                          scheme="implicit"):
    """K = P/(eps sigma) + J (implicit) or K = P (explicit), P = blockdiag(J)."""
    if scheme == "implicit":
        return BlockMatrix(J.n, J.diag * (1.0 + 1.0 / (eps * sigma)), J.rows.copy(),
                           J.cols.copy(), J.offd.copy())
    if scheme == "explicit":
        return BlockMatrix(J.n, J.diag.copy(), J.rows.copy(), J.cols.copy(),
                           np.zeros_like(J.offd))
    raise ValueError(scheme)


def assemble(mesh_like, Q, eps=EPS_DEFAULT, sigma=SIGMA_DEFAULT, scheme="implicit", Qff=None):
    """Convenience: K from an object with edges/area/bface_cell/bface_area attributes."""
    J = residual_jacobian(Q, mesh_like.edges, mesh_like.area, mesh_like.bface_cell,
                          mesh_like.bface_area, Qff)
    return preconditioner_matrix(J, eps, sigma, scheme)
