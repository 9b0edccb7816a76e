"""Frequency-shifted block systems and their inexact iterative solution.

Paper:
  * section "Generalized RK Scheme for Time-Linearized Harmonic Flows": the harmonic
    preconditioner matrix is K_l = K + i omega_l I V (I the unit matrix, V the cell
    volume), with the same sparsity pattern as the mean-flow K;
  * section "Solution Update": each RK stage solves A x = B with A = K/(Gamma alpha_k);
    for harmonic l the LHS is A + i omega_l I V/(Gamma alpha_k).  Multiplying by
    Gamma alpha_k gives (K + i omega_l V I) x = Gamma alpha_k B, the canonical form used
    here (the scale goes into the right-hand side).  The explicit scheme inverts the
    block diagonal point by point (block Jacobi); the implicit scheme approximates the
    inverse by ILU(0) with the pattern of A and solves the system iteratively and
    inexactly (ILU used as a smoother);
  * section "Results", table of key parameters: ILU fill 0, linear tolerance 1e-2 on
    ||B - A x||_2 relative to its initial value, at most 10 linear iterations.

The shift multiplies all six unknowns (the unit matrix is 6x6 here: five flow variables
plus the turbulence variable, so omega = 0 reproduces the mean system exactly).  omega
is given per zone and system, omega[s, zone[i]].

Preconditioners M on an ordering given as colour classes (ascending colour):
  JACOBI  M = blockdiag(K_s)
  SGS     M = (D + L) D^-1 (D + U)
  DILU    M = (Dt + L) Dt^-1 (Dt + U),  Dt_i = D_i - sum_{k in N(i), col k < col i} K_ik Dt_k^-1 K_ki
  ILU0    block ILU(0) (IKJ form) on the pattern of K_s in colour-major order
The iteration is preconditioned Richardson (defect correction), x^{m+1} = x^m + M^-1 (b - K_s x^m),
with M^-1 applied as a forward pass over colours ascending and a backward pass
descending; it stops when ||r^m||_2 <= rtol ||r^0||_2 or after max_sweeps steps.
"""
from dataclasses import dataclass, field
import numpy as np

from .assemble import BlockMatrix

I6 = np.eye(6)

OK, NOT_CONVERGED, DIVERGED = 0, 1, 2
KINDS = ("JACOBI", "SGS", "DILU", "ILU0")


def shift(volume, zone, omega_row):
    """omega_{zone(i)} V_i: the imaginary diagonal shift per cell (times I6)."""
    return np.asarray(omega_row, dtype=np.float64)[np.asarray(zone)] * np.asarray(volume)


def system_diag(K: BlockMatrix, volume, zone, omega_row):
    """Diagonal blocks of K_s = K + i omega V I (I of the block size: 6, or 5 for a
    frozen-turbulence system)."""
    I = np.eye(K.diag.shape[-1])
    return K.diag.astype(np.complex128) + 1j * shift(volume, zone, omega_row)[:, None, None] * I


def apply(K: BlockMatrix, Ds, x):
    """K_s x for x [N, 6] (complex): diagonal blocks Ds plus all off-diagonal couplings."""
    y = np.einsum("nij,nj->ni", Ds, x)
    np.add.at(y, K.rows, np.einsum("eij,ej->ei", K.offd, x[K.cols]))
    return y


def phase_lagged(K: BlockMatrix, edge_phase, sigma):
    """K with phase-lagged periodic couplings (section "Solution Update": on periodic
    boundaries each harmonic carries its own inter-blade phase angle sigma, which changes
    its left-hand side but not the sparsity pattern).  A periodic edge e = (a, b) with
    sign s_e = +1 couples a to the image of b one pitch over, whose value is x_b e^{i sigma}:
    the coupling of row a (entry 2e) is multiplied by e^{i s_e sigma} and that of row b
    (entry 2e+1) by e^{-i s_e sigma}.  Non-periodic edges (s_e = 0) are unchanged."""
    s = np.asarray(edge_phase, np.float64)
    ph = np.empty(2 * s.shape[0], np.complex128)
    ph[0::2] = np.exp(1j * s * sigma)
    ph[1::2] = np.exp(-1j * s * sigma)
    return BlockMatrix(K.n, K.diag.copy(), K.rows.copy(), K.cols.copy(), K.offd * ph[:, None, None])


def partition_dropped(K: BlockMatrix, part):
    """K with the couplings between cells of different partitions dropped (section
    "Parallel Implementation": the LHS is split over processors and the entries that
    couple two nodes of different partitions are ignored, leaving one independent
    sub-system per partition).  part[i] is the partition of cell i; the diagonal blocks
    are kept whole.  The dropped blocks are set to zero, so the pattern (and the pairing
    of entries 2e, 2e+1) is unchanged."""
    part = np.asarray(part)
    cross = part[K.rows] != part[K.cols]
    offd = K.offd.copy()
    offd[cross] = 0.0
    return BlockMatrix(K.n, K.diag.copy(), K.rows.copy(), K.cols.copy(), offd)


def dense(K: BlockMatrix, volume, zone, omega_row):
    """K_s as a dense [bN, bN] complex matrix, b the block size (for pins on small meshes)."""
    n, m = K.n, K.diag.shape[-1]
    Ds = system_diag(K, volume, zone, omega_row)
    A = np.zeros((m * n, m * n), dtype=np.complex128)
    for i in range(n):
        A[m * i:m * i + m, m * i:m * i + m] = Ds[i]
    for e in range(K.rows.shape[0]):
        i, k = int(K.rows[e]), int(K.cols[e])
        A[m * i:m * i + m, m * k:m * k + m] += K.offd[e]
    return A


def dense_solve(K, volume, zone, omega_row, b):
    """x = K_s^-1 b by LAPACK gesv: the plain definition of the converged result."""
    A = dense(K, volume, zone, omega_row)
    return np.linalg.solve(A, np.asarray(b, np.complex128).reshape(-1)).reshape(-1, K.diag.shape[-1])


def frozen_turbulence(K: BlockMatrix):
    """The system a frozen-turbulence harmonic solves (section "Brief Description of
    Hydra": the linearisation freezes the turbulence model, and the shift's unit matrix
    is 5x5 in section "Generalized RK Scheme for Time-Linearized Harmonic Flows"): the
    leading 5x5 sub-block of every block, the turbulence unknown left out (held at 0)."""
    return BlockMatrix(K.n, K.diag[:, :5, :5].copy(), K.rows.copy(), K.cols.copy(), K.offd[:, :5, :5].copy())


def richardson_frozen(K: BlockMatrix, volume, zone, omega_row, b, colour, kind="DILU", x0=None, **kw):
    """richardson on the frozen-turbulence system: the first five unknowns from the 5x5
    sub-system with b's first five components, the sixth 0."""
    b = np.asarray(b, np.complex128)
    x5, info = richardson(frozen_turbulence(K), volume, zone, omega_row, b[:, :5], colour, kind,
                          None if x0 is None else np.asarray(x0, np.complex128)[:, :5], **kw)
    x = np.zeros((K.n, 6), np.complex128)
    x[:, :5] = x5
    return x, info


def reverse_index(K: BlockMatrix):
    """Index of the transposed coupling: entry 2e <-> 2e+1 in the directed convention."""
    return np.arange(K.rows.shape[0]) ^ 1


def dilu_diagonal(K: BlockMatrix, Ds, colour):
    """Dt by colour classes ascending (DILU), returned with its block inverses.
    LAPACK inverse (LU with partial pivoting); a singular block raises LinAlgError."""
    colour = np.asarray(colour)
    m = int(colour.max()) + 1 if colour.size else 0
    Dt = Ds.copy()
    Dinv = np.zeros_like(Dt)
    rev = reverse_index(K)
    crow = colour[K.rows]
    ccol = colour[K.cols]
    for c in range(m):
        sel = np.nonzero((crow == c) & (ccol < c))[0]
        if sel.size:
            contrib = K.offd[sel] @ Dinv[K.cols[sel]] @ K.offd[rev[sel]]
            np.add.at(Dt, K.rows[sel], -contrib)
        rc = np.nonzero(colour == c)[0]
        Dinv[rc] = np.linalg.inv(Dt[rc])
    return Dt, Dinv


@dataclass
class Factor:
    kind: str
    colour: np.ndarray
    Dinv: np.ndarray = None          # JACOBI / SGS / DILU
    Dt: np.ndarray = None
    ilu: dict = None                 # ILU0: {(i, k): block}, plus positions
    pos: np.ndarray = None
    nbrs: list = None


def factor(K: BlockMatrix, volume, zone, omega_row, colour, kind="DILU"):
    Ds = system_diag(K, volume, zone, omega_row)
    colour = np.asarray(colour)
    if kind in ("JACOBI", "SGS"):
        return Factor(kind, colour, Dinv=np.linalg.inv(Ds), Dt=Ds)
    if kind == "DILU":
        Dt, Dinv = dilu_diagonal(K, Ds, colour)
        return Factor(kind, colour, Dinv=Dinv, Dt=Dt)
    if kind == "ILU0":
        return _ilu0(K, Ds, colour)
    raise ValueError(kind)


def _ilu0(K, Ds, colour):
    """Textbook block ILU(0), IKJ variant, in the order sorted by (colour, id)."""
    n = K.n
    order = np.lexsort((np.arange(n), colour))
    pos = np.empty(n, np.int64)
    pos[order] = np.arange(n)
    A = {}
    nbrs = [[] for _ in range(n)]
    for i in range(n):
        A[(i, i)] = Ds[i].copy()
    for e in range(K.rows.shape[0]):
        i, k = int(K.rows[e]), int(K.cols[e])
        A[(i, k)] = K.offd[e].astype(np.complex128)
        nbrs[i].append(k)
    for i in order:
        i = int(i)
        row = set(nbrs[i]) | {i}
        for k in sorted((k for k in nbrs[i] if pos[k] < pos[i]), key=lambda q: pos[q]):
            A[(i, k)] = A[(i, k)] @ np.linalg.inv(A[(k, k)])
            for j in nbrs[k]:
                if pos[j] > pos[k] and j in row:
                    A[(i, j)] = A[(i, j)] - A[(i, k)] @ A[(k, j)]
    return Factor("ILU0", colour, ilu=A, pos=pos, nbrs=nbrs)


def precondition(K: BlockMatrix, f: Factor, r):
    """z = M^-1 r: forward pass over colours ascending, backward pass descending."""
    if f.kind == "JACOBI":
        return np.einsum("nij,nj->ni", f.Dinv, r)
    if f.kind == "ILU0":
        return _ilu0_apply(f, r)
    colour = f.colour
    m = int(colour.max()) + 1
    crow = colour[K.rows]
    ccol = colour[K.cols]
    y = np.zeros_like(r)
    for c in range(m):                          # (Dt + L) y = r
        rc = np.nonzero(colour == c)[0]
        t = r[rc].copy()
        sel = np.nonzero((crow == c) & (ccol < c))[0]
        acc = np.zeros_like(r)
        if sel.size:
            np.add.at(acc, K.rows[sel], np.einsum("eij,ej->ei", K.offd[sel], y[K.cols[sel]]))
        t -= acc[rc]
        y[rc] = np.einsum("nij,nj->ni", f.Dinv[rc], t)
    z = np.zeros_like(r)
    for c in range(m - 1, -1, -1):              # (Dt + U) z = Dt y
        rc = np.nonzero(colour == c)[0]
        sel = np.nonzero((crow == c) & (ccol > c))[0]
        acc = np.zeros_like(r)
        if sel.size:
            np.add.at(acc, K.rows[sel], np.einsum("eij,ej->ei", K.offd[sel], z[K.cols[sel]]))
        z[rc] = y[rc] - np.einsum("nij,nj->ni", f.Dinv[rc], acc[rc])
    return z


def _ilu0_apply(f: Factor, r):
    n = r.shape[0]
    order = np.argsort(f.pos)
    y = np.zeros_like(r)
    for i in order:                              # unit lower
        i = int(i)
        t = r[i].copy()
        for k in f.nbrs[i]:
            if f.pos[k] < f.pos[i]:
                t -= f.ilu[(i, k)] @ y[k]
        y[i] = t
    z = np.zeros_like(r)
    for i in order[::-1]:                        # upper
        i = int(i)
        t = y[i].copy()
        for j in f.nbrs[i]:
            if f.pos[j] > f.pos[i]:
                t -= f.ilu[(i, j)] @ z[j]
        z[i] = np.linalg.solve(f.ilu[(i, i)], t)
    return z


@dataclass
class Info:
    status: int
    sweeps: int
    rel_res: float
    history: list = field(default_factory=list)


def richardson(K: BlockMatrix, volume, zone, omega_row, b, colour, kind="DILU", x0=None,
               rtol=1e-8, max_sweeps=5000, div_factor=1e3, iterates=None):
    """Preconditioned Richardson to ||r^m|| <= rtol ||r^0|| (2-norm over all 6N complex
    entries) or m = max_sweeps.  NaN/Inf or ||r^m|| > div_factor ||r^0|| -> DIVERGED.
    Returns (x, Info).  If ``iterates`` is a list, every x^m is appended to it."""
    b = np.asarray(b, np.complex128)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, np.complex128).copy()
    Ds = system_diag(K, volume, zone, omega_row)
    f = factor(K, volume, zone, omega_row, colour, kind)
    hist = []
    r = b - apply(K, Ds, x)
    n0 = float(np.linalg.norm(r))
    m = 0
    while True:
        nr = float(np.linalg.norm(r))
        hist.append(nr)
        if iterates is not None:
            iterates.append(x.copy())
        if nr <= rtol * n0:
            status = OK
            break
        if not np.isfinite(nr) or nr > div_factor * n0:
            status = DIVERGED
            break
        if m == max_sweeps:
            status = NOT_CONVERGED
            break
        x = x + precondition(K, f, r)
        m += 1
        r = b - apply(K, Ds, x)
    rel = nr / n0 if n0 > 0 else 0.0
    return x, Info(status, m, rel, hist)


def paper_mode(K, volume, zone, omega_row, b, colour, kind="DILU", x0=None):
    """The paper's linear-solve setting: relative tolerance 1e-2, at most 10 iterations."""
    return richardson(K, volume, zone, omega_row, b, colour, kind, x0, rtol=1e-2, max_sweeps=10)


def contraction(history):
    """Estimated contraction rho ~ (||r^m|| / ||r^0||)^(1/m)."""
    m = len(history) - 1
    if m <= 0 or history[0] == 0:
        return 0.0
    return float((history[-1] / history[0]) ** (1.0 / m))
