"""Reference of the learned preconditioner (a project addition; the paper has no learned
component).  FP64 NumPy, manual backward, Adam.

A two-layer per-edge message-passing network maps the residual r of one system to a
correction dx (used as x' = x + dx, accepted only if it lowers the FP64 residual):

  scale      sigma = sqrt(sum |r|^2 / (12 N))           (RMS over the 12N real entries)
  node input u_i   = [r_i / sigma, z_i / sigma]          (24 reals; complex entries as
                     (re, im) pairs), z_i = (K_ii + i w_i V_i I)^-1 r_i
  edge input g_ij  = K_ij z_j / sigma                     (12 reals), coupling i <- j
  layer 1    m_ij  = relu(W1^T [u_i; u_j; g_ij])          (60 -> 64)
             a_i   = sum_j m_ij
             h_i   = relu(W2^T [u_i; a_i])                (88 -> 64)
  layer 2    p_ij  = relu(W3^T [h_i; h_j])                (128 -> 64)
             c_i   = sum_j p_ij
             q_i   = relu(W4^T [h_i; c_i])                (128 -> 64)
  decoder    d_i   = W5^T q_i                             (64 -> 12)
  output     dx_i  = sigma * d_i                          (back to complex 6-vectors)

No biases: the map r -> dx is positively homogeneous of degree one (dx(a r) = a dx(r),
a > 0), so the scale normalisation is exact.  Training loss for a pair (r, e) with e the
error x* - x: L = ||d - e/sigma||^2 / ||e/sigma||^2 (scale-free), averaged over a batch.

Weights are one flat FP32-master vector in the order W1 (60x64), W2 (88x64), W3 (128x64),
W4 (128x64), W5 (64x12), each row-major [in][out].
"""
import numpy as np

F_NODE = 24
F_EDGE = 12
HIDDEN = 64
SHAPES = [(2 * F_NODE + F_EDGE, HIDDEN), (F_NODE + HIDDEN, HIDDEN), (2 * HIDDEN, HIDDEN),
          (2 * HIDDEN, HIDDEN), (HIDDEN, 12)]


def n_params():
    return sum(a * b for a, b in SHAPES)


def unpack(w):
    out, o = [], 0
    for a, b in SHAPES:
        out.append(np.asarray(w[o:o + a * b], np.float64).reshape(a, b))
        o += a * b
    return out


def pack(mats):
    return np.concatenate([np.asarray(m, np.float64).reshape(-1) for m in mats])


def init_weights(seed=0):
    """He-normal initialisation (std sqrt(2/fan_in)); the decoder is scaled by 0.1."""
    rng = np.random.default_rng(seed)
    mats = [rng.standard_normal((a, b)) * np.sqrt(2.0 / a) for a, b in SHAPES]
    mats[-1] *= 0.1
    return pack(mats)


def block_jacobi_weights():
    """Weights for which the network's output is exactly the block-Jacobi correction
    dx = (K_ii + i w V_i I)^-1 r_i: layer 1 and the layer-2 messages are switched off
    (W1 = W3 = 0), W2 copies the z/sigma half of u into 12 hidden units and its negative
    into 12 more, W4 passes those 24 on, and W5 takes the difference of each pair,
    relu(t) - relu(-t) = t.  Every weight is 0 or +-1 (exact in any precision)."""
    W = [np.zeros(s) for s in SHAPES]
    for j in range(12):
        W[1][12 + j, j] = 1.0
        W[1][12 + j, 12 + j] = -1.0
        W[4][j, j] = 1.0
        W[4][12 + j, j] = -1.0
    for j in range(24):
        W[3][j, j] = 1.0
    return pack(W)


def c2r(v):
    """complex [N, 6] -> real [N, 12] as (re, im) pairs."""
    out = np.empty(v.shape[:-1] + (12,))
    out[..., 0::2] = v.real
    out[..., 1::2] = v.imag
    return out


def r2c(v):
    return v[..., 0::2] + 1j * v[..., 1::2]


def features(K, Ds, r):
    """u [N, 24], g [2E, 12] and sigma for residual r [N, 6] (complex)."""
    n = r.shape[0]
    sigma = float(np.sqrt(np.sum(np.abs(r) ** 2) / (12.0 * n)))
    if sigma == 0.0:
        sigma = 1.0
    z = np.linalg.solve(Ds, r[..., None])[..., 0]
    u = np.concatenate([c2r(r / sigma), c2r(z / sigma)], axis=1)
    g = c2r(np.einsum("eij,ej->ei", K.offd, z[K.cols] / sigma))
    return u, g, sigma


def relu(x):
    return np.maximum(x, 0.0)


def forward(w, u, g, rows, cols, n):
    """Returns the decoder output d [N, 12] and a cache for backward."""
    W1, W2, W3, W4, W5 = unpack(w)
    X1 = np.concatenate([u[rows], u[cols], g], axis=1)
    pm = X1 @ W1
    m = relu(pm)
    a = np.zeros((n, HIDDEN))
    np.add.at(a, rows, m)
    Y1 = np.concatenate([u, a], axis=1)
    p1 = Y1 @ W2
    h = relu(p1)
    X2 = np.concatenate([h[rows], h[cols]], axis=1)
    pp = X2 @ W3
    p = relu(pp)
    c = np.zeros((n, HIDDEN))
    np.add.at(c, rows, p)
    Y2 = np.concatenate([h, c], axis=1)
    p2 = Y2 @ W4
    q = relu(p2)
    d = q @ W5
    cache = (X1, pm, Y1, p1, h, X2, pp, Y2, p2, q)
    return d, cache


def loss_and_grad(w, u, g, rows, cols, n, ehat):
    """L = ||d - ehat||^2 / ||ehat||^2 and dL/dw (flat), by hand through the graph."""
    W1, W2, W3, W4, W5 = unpack(w)
    d, (X1, pm, Y1, p1, h, X2, pp, Y2, p2, q) = forward(w, u, g, rows, cols, n)
    den = float(np.sum(ehat * ehat))
    diff = d - ehat
    L = float(np.sum(diff * diff)) / den
    dd = 2.0 * diff / den
    gW5 = q.T @ dd
    dq = dd @ W5.T
    dp2 = dq * (p2 > 0)
    gW4 = Y2.T @ dp2
    dY2 = dp2 @ W4.T
    dh = dY2[:, :HIDDEN].copy()
    dc = dY2[:, HIDDEN:]
    dpp = dc[rows] * (pp > 0)               # every edge message of cell i gets dc_i
    gW3 = X2.T @ dpp
    dX2 = dpp @ W3.T
    np.add.at(dh, rows, dX2[:, :HIDDEN])    # receiver part
    np.add.at(dh, cols, dX2[:, HIDDEN:])    # sender part
    dp1 = dh * (p1 > 0)
    gW2 = Y1.T @ dp1
    dY1 = dp1 @ W2.T
    da = dY1[:, F_NODE:]
    dpm = da[rows] * (pm > 0)
    gW1 = X1.T @ dpm
    return L, pack([gW1, gW2, gW3, gW4, gW5])


def apply(w, K, Ds, r):
    """dx = sigma * d(r), complex [N, 6]."""
    u, g, sigma = features(K, Ds, r)
    d, _ = forward(w, u, g, K.rows, K.cols, r.shape[0])
    return sigma * r2c(d)


ACCEPT = 1e-3   # least fractional drop of ||r||^2 for which a learned step is kept


def line_step(A, r, d, accept=ACCEPT):
    """The learned correction d taken as a search direction for the residual r:
    alpha = (y, r) / (y, y) with y = A d minimises ||r - alpha y|| over complex alpha,
    and the squared residual falls by the fraction |(y, r)|^2 / (||y||^2 ||r||^2).  The
    step is kept only if everything is finite and that fraction is >= accept; otherwise
    alpha = 0.  (u, v) = sum conj(u) v.  Returns (alpha, fraction)."""
    y = A(d)
    yr = np.vdot(y, r)
    yy = float(np.vdot(y, y).real)
    rr = float(np.vdot(r, r).real)
    gain = abs(yr) ** 2 / (yy * rr) if (yy > 0.0 and rr > 0.0) else 0.0
    if not (np.isfinite(yr) and np.isfinite(yy)) or not gain >= accept:
        return 0.0 + 0.0j, gain
    return yr / yy, gain


class Adam:
    """Adam (Kingma & Ba) on the flat weight vector; bias-corrected moments."""

    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, w, grad):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * grad
        self.v = self.b2 * self.v + (1 - self.b2) * grad * grad
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return w - self.lr * mh / (np.sqrt(vh) + self.eps)
