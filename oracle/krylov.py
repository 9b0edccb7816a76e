"""Reference of the Krylov solve around the ILU(0)/DILU preconditioner (test
infrastructure only; nothing in the product path imports this module).

Paper: section "Generalized RK Scheme for The Mean Flow" notes that the ILU(0)
approximation of K^-1 serves either as a smoother (the Richardson iteration of
oracle.solve, the paper's choice) or as the preconditioner of a Newton-Krylov method.
The paper gives no Krylov algorithm; this is the textbook restarted flexible GMRES
(FGMRES(m): Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Alg. 9.6) on the
system of oracle.solve, (K + i omega V I) x = b, with right preconditioning:

  r0 = b - A x0, beta = ||r0||, v1 = r0 / beta;
  for j = 1..m:  z_j = M_j^-1 v_j;  w = A z_j;
                 h_ij = (v_i, w), w -= h_ij v_i for i = 1..j   (modified Gram-Schmidt);
                 h_{j+1,j} = ||w||;  v_{j+1} = w / h_{j+1,j};
                 y_j = argmin || beta e1 - Hbar_j y ||  (least squares, j+1 by j);
                 the residual norm of x0 + Z_j y_j is that minimum;
  x = x0 + Z_k y_k at the end of the cycle (k the last j); restart from the true residual.

M_j^-1 v: `inner_sweeps` steps of the preconditioned Richardson of oracle.solve from
x = 0 (one step is exactly M^-1 v for the DILU, SGS or Jacobi M).  kind "LEARNED" (a
project addition: the flexible method admits a nonlinear M_j): z0 = alpha d with d =
net(v) the learned correction for the residual v and alpha from learned.line_step (0 when
the step is rejected), then `inner_sweeps` DILU steps of the Richardson iteration on
A z = v starting from z0.  After OFF_AFTER applications in a row whose step was rejected
the network is not evaluated again in this solve (alpha = 0 from then on; a kept step
ends a run of rejections): the controller of the learned part, also a project
addition.  The inner products
are (u, v) = sum conj(u) v over all 6N complex entries; the stop test is
||r|| <= rtol ||r0|| on the least-squares residual norm, or iters = max_iters.
"""
from dataclasses import dataclass, field

import numpy as np

from . import learned, solve


@dataclass
class KrylovInfo:
    status: int
    iters: int
    rel_res: float
    history: list = field(default_factory=list)   # residual norm after each iteration (index 0: ||r0||)
    true_res: float = 0.0                          # ||b - A x|| of the returned x, relative
    learned: int = 0                               # LEARNED: applications that kept the step
    switched_off: bool = False                     # LEARNED: the controller stopped the network


OFF_AFTER = 3   # rejected learned steps in a row after which the network is not evaluated


def _lstsq_min(Hbar, beta):
    """y = argmin ||beta e1 - Hbar y||_2 and that minimum (LAPACK least squares)."""
    rhs = np.zeros(Hbar.shape[0], np.complex128)
    rhs[0] = beta
    y = np.linalg.lstsq(Hbar, rhs, rcond=None)[0]
    return y, float(np.linalg.norm(rhs - Hbar @ y))


def fgmres(K, volume, zone, omega_row, b, colour, kind="DILU", x0=None, restart=20, rtol=1e-8, max_iters=1000,
           inner_sweeps=1, net=None):
    """Restarted flexible GMRES with the inner Richardson preconditioner (kind LEARNED:
    net(r) -> d gives the learned correction).  Returns (x, KrylovInfo)."""
    b = np.asarray(b, np.complex128)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, np.complex128).copy()
    Ds = solve.system_diag(K, volume, zone, omega_row)
    if kind == "LEARNED" and net is None:
        raise ValueError("kind LEARNED needs net")
    kept = [0]
    run = [0, False]    # rejections in a row, switched off

    def A(v):
        return solve.apply(K, Ds, v)

    def M_inv(v):
        z0, sweep_kind = None, kind
        if kind == "LEARNED":
            sweep_kind = "DILU"
            if not run[1]:
                d = net(v)
                alpha, _ = learned.line_step(A, v, d)
                if alpha != 0.0:
                    kept[0] += 1
                    run[0] = 0
                    z0 = alpha * d
                else:
                    run[0] += 1
                    run[1] = run[0] >= OFF_AFTER
        z, _ = solve.richardson(K, volume, zone, omega_row, v, colour, sweep_kind, x0=z0, rtol=0.0,
                                max_sweeps=inner_sweeps, div_factor=np.inf)
        return z

    r = b - A(x)
    beta = float(np.linalg.norm(r))
    n0 = beta
    hist = [beta]
    iters = 0
    res = beta
    status = solve.OK
    while True:
        if res <= rtol * n0:
            status = solve.OK
            break
        if iters >= max_iters:
            status = solve.NOT_CONVERGED
            break
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart), np.complex128)
        y = None
        for j in range(restart):
            Z.append(M_inv(V[j]))
            w = A(Z[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            y, res = _lstsq_min(H[:j + 2, :j + 1], beta)
            iters += 1
            hist.append(res)
            breakdown = H[j + 1, j] == 0.0
            if not breakdown:
                V.append(w / H[j + 1, j])
            if res <= rtol * n0 or iters >= max_iters or breakdown:
                break
        x = x + sum(y[i] * Z[i] for i in range(len(y)))
        r = b - A(x)                 # restart from the true residual
        beta = float(np.linalg.norm(r))
        if not np.isfinite(beta):
            status = solve.DIVERGED
            break
        res = beta
        if beta == 0.0:
            break
    true_rel = float(np.linalg.norm(b - A(x)) / n0) if n0 > 0 else 0.0
    return x, KrylovInfo(status, iters, res / n0 if n0 > 0 else 0.0, hist, true_rel, kept[0], run[1])
