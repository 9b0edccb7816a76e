"""Seeded synthetic workloads: turbomachinery-shaped hex meshes stored as edge lists,
smooth mean-flow states, right-hand sides and harmonic frequencies.

This module builds *inputs only*.  It holds none of the solver's arithmetic (no flux,
Jacobian, factorisation or sweep); both the GPU library and the CPU oracle consume what
it returns as plain arrays.

Shapes follow the paper's workloads (blade-row passages meshed with hexahedra, blade
counts in the ratio 3:5:4 for a rotor-stator-rotor stack, 8-16 harmonics per row; see
the "Results" section).  The industrial meshes themselves are not available, so every
geometry here is a seeded stand-in:

* ``passage_block``: one annular passage sector, axial x in [x0, x0+0.3], radius in
  [0.9, 1.1], pitch 2*pi/N_b with a stagger theta += 0.3 x so faces are non-orthogonal;
  optional seeded vertex jitter; random cell-id permutation, shuffled edge order and
  random edge orientation (the area vector is negated with the swap).
* ``multi_row``: several passages stacked axially, joined at each row interface by
  pitch-overlap edges (each upstream exit-face cell couples to two downstream cells),
  which puts triangles into the cell graph.
* ``flow_state``: conservative state (rho, rho u, rho v, rho w, rho E, rho nu~) with
  low-mode Fourier variations, Mach 0.3-0.6, density 1 +/- 5 %, nu~ in [1e-5, 1e-3].
* ``rhs``: i.i.d. N(0,1) real and imaginary parts; the mean (omega = 0) RHS is real.
* ``cascade_block``: a linear-cascade passage (pitchwise direction y) whose two pitchwise
  sides are joined by translationally periodic edges, flagged in ``edge_phase`` for the
  phase-lagged boundary of the harmonic systems; ``n_passages`` > 1 stacks identical
  passages pitchwise (a full wheel when the closing edges carry no phase).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

GAMMA = 1.4


@dataclass
class Mesh:
    """Edge-based finite-volume mesh (the paper's node-centred control volumes).

    edges[e] = (a, b) with area vector area[e] oriented from a to b; boundary face f
    belongs to cell bface_cell[f] with outward area bface_area[f].  ``ijk`` and
    ``row`` are generator metadata (structured position of each cell) used only to
    build smooth states; solvers never look at them.
    """
    n_cells: int
    edges: np.ndarray        # [E, 2] int32
    area: np.ndarray         # [E, 3] float64, a -> b
    volume: np.ndarray       # [N] float64
    zone: np.ndarray         # [N] int32
    bface_cell: np.ndarray   # [B] int32
    bface_area: np.ndarray   # [B, 3] float64, outward
    centroid: np.ndarray     # [N, 3] float64
    n_zones: int = 1
    n_blades: tuple = (36,)
    meta: dict = field(default_factory=dict)
    # per edge: 0, or +1 / -1 for a periodic coupling whose b side is the image of b one
    # pitch above (+1) or below (-1) the a side; None when the mesh has no periodic edges
    edge_phase: np.ndarray = None

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])

    @property
    def n_bfaces(self) -> int:
        return int(self.bface_cell.shape[0])


def _quad_area(p0, p1, p2, p3):
    """Vector area of a (possibly non-planar) quad p0-p1-p2-p3: half the cross product
    of its diagonals; exact for the surface bounded by the four straight edges."""
    return 0.5 * np.cross(p2 - p0, p3 - p1)


def _passage_vertices(nx, nt, nr, n_blades, x0, rng, jitter, theta_shift=0.0):
    i = np.arange(nx + 1)[:, None, None]
    j = np.arange(nt + 1)[None, :, None]
    k = np.arange(nr + 1)[None, None, :]
    x = x0 + 0.3 * i / nx + 0.0 * j + 0.0 * k
    pitch = 2.0 * np.pi / n_blades
    th = pitch * (j / nt + theta_shift) + 0.3 * x
    r = 0.9 + 0.2 * k / nr + 0.0 * x
    th = th + 0.0 * r
    if jitter > 0.0:
        # interior vertices only, so the outer envelope stays a clean sector
        d = rng.uniform(-1.0, 1.0, size=(3,) + x.shape) * jitter
        interior = np.zeros(x.shape, bool)
        interior[1:-1, 1:-1, 1:-1] = True
        x = x + np.where(interior, d[0] * 0.3 / nx, 0.0)
        th = th + np.where(interior, d[1] * pitch / nt, 0.0)
        r = r + np.where(interior, d[2] * 0.2 / nr, 0.0)
    return np.stack([x, r * np.cos(th), r * np.sin(th)], axis=-1), th


def _structured_faces(P, nx, nt, nr):
    """Faces of a structured hex block.  Returns, per direction, vector areas oriented
    towards increasing index and the face centroids."""
    out = {}
    # x-faces at vertex plane i: quad (j,k),(j+1,k),(j+1,k+1),(j,k+1)
    q = [P[:, :-1, :-1], P[:, 1:, :-1], P[:, 1:, 1:], P[:, :-1, 1:]]
    out[0] = (_quad_area(*q), 0.25 * sum(q))          # [nx+1, nt, nr, 3]
    q = [P[:-1, :, :-1], P[:-1, :, 1:], P[1:, :, 1:], P[1:, :, :-1]]
    out[1] = (_quad_area(*q), 0.25 * sum(q))          # [nx, nt+1, nr, 3]
    q = [P[:-1, :-1, :], P[1:, :-1, :], P[1:, 1:, :], P[:-1, 1:, :]]
    out[2] = (_quad_area(*q), 0.25 * sum(q))          # [nx, nt, nr+1, 3]
    return out


@dataclass
class _Block:
    nx: int
    nt: int
    nr: int
    P: np.ndarray
    theta: np.ndarray
    faces: dict
    centroid: np.ndarray
    volume: np.ndarray


def _build_block(nx, nt, nr, n_blades, x0, rng, jitter, theta_shift=0.0):
    P, th = _passage_vertices(nx, nt, nr, n_blades, x0, rng, jitter, theta_shift)
    return _block_from_vertices(P, th, nx, nt, nr)


def _block_from_vertices(P, th, nx, nt, nr):
    faces = _structured_faces(P, nx, nt, nr)
    cen = 0.125 * (P[:-1, :-1, :-1] + P[1:, :-1, :-1] + P[:-1, 1:, :-1] + P[:-1, :-1, 1:]
                   + P[1:, 1:, :-1] + P[1:, :-1, 1:] + P[:-1, 1:, 1:] + P[1:, 1:, 1:])
    # orient each direction's faces towards increasing index (check one face robustly)
    for d in range(3):
        S, c = faces[d]
        ref = np.zeros(3)
        ref[d] = 1.0
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[d] = slice(0, -1)
        sl_hi[d] = slice(1, None)
        dc = cen[tuple(sl_hi)] - cen[tuple(sl_lo)] if cen.shape[d] > 1 else None
        if dc is not None:
            inner = [slice(None)] * 3
            inner[d] = slice(1, -1)
            s = np.sum(S[tuple(inner)] * dc, axis=-1)
            sign = 1.0 if np.sum(s) > 0 else -1.0
        else:
            # single layer: orient by the outward direction of the upper boundary
            up = [slice(None)] * 3
            up[d] = slice(-1, None)
            s = np.sum(S[tuple(up)] * (c[tuple(up)] - cen), axis=-1)
            sign = 1.0 if np.sum(s) > 0 else -1.0
        faces[d] = (sign * S, c)
    # volume by the divergence theorem, V = 1/3 sum_f c_f . S_f (outward)
    vol = np.zeros((nx, nt, nr))
    for d in range(3):
        S, c = faces[d]
        flux = np.sum(c * S, axis=-1) / 3.0
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[d] = slice(0, -1)
        hi[d] = slice(1, None)
        vol += flux[tuple(hi)] - flux[tuple(lo)]
    return _Block(nx, nt, nr, P, th, faces, cen, vol)


def _block_edges(blk: _Block, base: int):
    """Interior edges and boundary faces of one block in structured cell numbering
    cell(i,j,k) = base + (i*nt + j)*nr + k.  Boundary faces are returned per side so a
    caller can replace a side by interface edges."""
    nx, nt, nr = blk.nx, blk.nt, blk.nr
    cid = base + np.arange(nx * nt * nr).reshape(nx, nt, nr)
    E_a, E_b, E_S = [], [], []
    sides = {}
    for d in range(3):
        S, _ = blk.faces[d]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[d] = slice(0, -1)
        hi[d] = slice(1, None)
        inner = [slice(None)] * 3
        inner[d] = slice(1, -1)
        E_a.append(cid[tuple(lo)].ravel())
        E_b.append(cid[tuple(hi)].ravel())
        E_S.append(S[tuple(inner)].reshape(-1, 3))
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[d] = 0
        last[d] = -1
        fs = [slice(None)] * 3
        ls = [slice(None)] * 3
        fs[d] = 0
        ls[d] = S.shape[d] - 1
        sides[(d, 0)] = (cid[tuple(first)], -S[tuple(fs)])   # outward = -increasing
        sides[(d, 1)] = (cid[tuple(last)], S[tuple(ls)])
    return (np.concatenate(E_a), np.concatenate(E_b), np.concatenate(E_S)), sides


def _finish(n_cells, ea, eb, eS, bc, bS, vol, cen, zone, rng, permute, n_zones, n_blades, meta, eph=None):
    ea = ea.astype(np.int64)
    eb = eb.astype(np.int64)
    if permute:
        perm = rng.permutation(n_cells)        # structured id -> user id
        ea, eb, bc = perm[ea], perm[eb], perm[bc]
        inv = np.empty_like(perm)
        inv[perm] = np.arange(n_cells)
        vol, cen, zone = vol[inv], cen[inv], zone[inv]
        meta["struct_to_user"] = perm
        order = rng.permutation(ea.shape[0])
        ea, eb, eS = ea[order], eb[order], eS[order]
        flip = rng.random(ea.shape[0]) < 0.5
        ea, eb = np.where(flip, eb, ea), np.where(flip, ea, eb)
        eS = np.where(flip[:, None], -eS, eS)
        if eph is not None:
            eph = np.where(flip, -eph[order], eph[order])
    else:
        meta["struct_to_user"] = np.arange(n_cells)
    edges = np.stack([ea, eb], axis=1).astype(np.int32)
    return Mesh(n_cells=n_cells, edges=np.ascontiguousarray(edges),
                area=np.ascontiguousarray(eS, dtype=np.float64),
                volume=np.ascontiguousarray(vol, dtype=np.float64),
                zone=np.ascontiguousarray(zone, dtype=np.int32),
                bface_cell=np.ascontiguousarray(bc, dtype=np.int32),
                bface_area=np.ascontiguousarray(bS, dtype=np.float64),
                centroid=np.ascontiguousarray(cen, dtype=np.float64),
                n_zones=n_zones, n_blades=tuple(n_blades), meta=meta,
                edge_phase=None if eph is None else np.ascontiguousarray(eph, dtype=np.int8))


def passage_block(nx: int, nt: int, nr: int, n_blades: int = 36, seed: int = 1,
                  jitter: float = 0.1, permute: bool = True) -> Mesh:
    """One passage sector of nx*nt*nr hex cells as an unstructured edge list."""
    rng = np.random.default_rng(seed)
    blk = _build_block(nx, nt, nr, n_blades, 0.0, rng, jitter)
    (ea, eb, eS), sides = _block_edges(blk, 0)
    bc = np.concatenate([sides[k][0].ravel() for k in sorted(sides)])
    bS = np.concatenate([sides[k][1].reshape(-1, 3) for k in sorted(sides)])
    n = nx * nt * nr
    meta = {"kind": "passage", "shape": (nx, nt, nr), "n_blades": n_blades, "seed": seed,
            "theta": _cell_theta(blk), "radius": _cell_radius(blk),
            "xi": _cell_frac(blk), "row": np.zeros(n, np.int32)}
    return _finish(n, ea, eb, eS, bc, bS, blk.volume.ravel(), blk.centroid.reshape(-1, 3),
                   np.zeros(n, np.int32), rng, permute, 1, (n_blades,), meta)


def cascade_block(nx: int, ny: int, nz: int, n_blades: int = 36, seed: int = 1, jitter: float = 0.1,
                  permute: bool = True, n_passages: int = 1, stagger: float = 0.3) -> Mesh:
    """Linear-cascade passage(s) of nx*ny*nz hex cells: axial x in [0, 0.3], pitchwise y
    over n_passages pitches of 2 pi / n_blades, spanwise z in [0, 0.2], stagger y += 0.3 x.
    The top and bottom pitchwise sides are joined by translationally periodic edges
    (top cell a, bottom cell b, area of a's top face; edge_phase +1).  Vertex jitter and
    the cells' fractional positions repeat with the pitch, so stacked passages are
    identical copies."""
    rng = np.random.default_rng(seed)
    pitch = 2.0 * np.pi / n_blades
    nyt = ny * n_passages
    i = np.arange(nx + 1)[:, None, None] + np.zeros((1, nyt + 1, nz + 1))
    j = np.arange(nyt + 1)[None, :, None] + np.zeros((nx + 1, 1, nz + 1))
    k = np.arange(nz + 1)[None, None, :] + np.zeros((nx + 1, nyt + 1, 1))
    x = 0.3 * i / nx
    y = pitch * j / ny + stagger * x
    z = 0.2 * k / nz
    if jitter > 0.0:
        d = rng.uniform(-1.0, 1.0, size=(3, nx + 1, ny, nz + 1)) * jitter
        jm = (j % ny).astype(np.int64)
        ii = i.astype(np.int64)
        kk = k.astype(np.int64)
        dd = d[:, ii, jm, kk]
        interior = (ii > 0) & (ii < nx) & (kk > 0) & (kk < nz)
        x = x + np.where(interior, dd[0] * 0.3 / nx, 0.0)
        y = y + np.where(interior, dd[1] * pitch / ny, 0.0)
        z = z + np.where(interior, dd[2] * 0.2 / nz, 0.0)
    P = np.stack([x, y, z], axis=-1)
    blk = _block_from_vertices(P, np.zeros_like(x), nx, nyt, nz)
    (ea, eb, eS), sides = _block_edges(blk, 0)
    bc = np.concatenate([sides[kk_][0].ravel() for kk_ in sorted(sides) if kk_[0] != 1])
    bS = np.concatenate([sides[kk_][1].reshape(-1, 3) for kk_ in sorted(sides) if kk_[0] != 1])
    top, S_top = sides[(1, 1)]
    bot, _ = sides[(1, 0)]
    n_int = ea.shape[0]
    ea = np.concatenate([ea, top.ravel()])
    eb = np.concatenate([eb, bot.ravel()])
    eS = np.concatenate([eS, S_top.reshape(-1, 3)])
    eph = np.zeros(ea.shape[0], np.int8)
    eph[n_int:] = 1
    n = nx * nyt * nz
    fx, fy, fz = np.meshgrid((np.arange(nx) + 0.5) / nx, ((np.arange(nyt) % ny) + 0.5) / ny,
                             (np.arange(nz) + 0.5) / nz, indexing="ij")
    passage = np.broadcast_to((np.arange(nyt) // ny)[None, :, None], (nx, nyt, nz)).ravel()
    meta = {"kind": "cascade", "shape": (nx, nyt, nz), "n_blades": n_blades, "seed": seed,
            "theta": np.full(n, -0.5 * np.pi), "radius": np.ones(n),
            "xi": np.stack([fx.ravel(), fy.ravel(), fz.ravel()], axis=1), "row": np.zeros(n, np.int32),
            "passage": passage.copy(), "n_passages": n_passages}
    return _finish(n, ea, eb, eS, bc, bS, blk.volume.ravel(), blk.centroid.reshape(-1, 3),
                   np.zeros(n, np.int32), rng, permute, 1, (n_blades,), meta, eph)


def _cell_theta(blk):
    return (0.125 * (blk.theta[:-1, :-1, :-1] + blk.theta[1:, :-1, :-1] + blk.theta[:-1, 1:, :-1]
                     + blk.theta[:-1, :-1, 1:] + blk.theta[1:, 1:, :-1] + blk.theta[1:, :-1, 1:]
                     + blk.theta[:-1, 1:, 1:] + blk.theta[1:, 1:, 1:])).ravel()


def _cell_radius(blk):
    c = blk.centroid.reshape(-1, 3)
    return np.hypot(c[:, 1], c[:, 2])


def _cell_frac(blk):
    nx, nt, nr = blk.nx, blk.nt, blk.nr
    i, j, k = np.meshgrid((np.arange(nx) + 0.5) / nx, (np.arange(nt) + 0.5) / nt,
                          (np.arange(nr) + 0.5) / nr, indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)


def multi_row(nx: int, nt: int, nr: int, n_blades=(36, 60, 48), seed: int = 5,
              jitter: float = 0.1, permute: bool = True) -> Mesh:
    """Rows stacked axially (x0 = 0, 0.3, 0.6, ...), one zone per row.  At each interface
    the upstream row's exit faces become edges to the two downstream inlet cells they
    overlap in pitch fraction (the downstream grid is offset by half a cell), weighted
    by the overlap; the downstream inlet boundary faces are dropped.  Each upstream cell
    then couples to two mutually adjacent downstream cells: the graph has triangles."""
    rng = np.random.default_rng(seed)
    blocks, EA, EB, ES, BC, BS = [], [], [], [], [], []
    vols, cens, zones, thetas, radii, fracs, rows = [], [], [], [], [], [], []
    base = 0
    for z, nb in enumerate(n_blades):
        shift = 0.5 / nt if z % 2 == 1 else 0.0
        blk = _build_block(nx, nt, nr, nb, 0.3 * z, rng, jitter, theta_shift=shift)
        (ea, eb, eS), sides = _block_edges(blk, base)
        blocks.append((blk, sides, base))
        EA.append(ea)
        EB.append(eb)
        ES.append(eS)
        n = nx * nt * nr
        vols.append(blk.volume.ravel())
        cens.append(blk.centroid.reshape(-1, 3))
        zones.append(np.full(n, z, np.int32))
        thetas.append(_cell_theta(blk))
        radii.append(_cell_radius(blk))
        fracs.append(_cell_frac(blk))
        rows.append(np.full(n, z, np.int32))
        base += n
    nrow = len(n_blades)
    for z in range(nrow):
        blk, sides, b0 = blocks[z]
        for key in sorted(sides):
            cells, S = sides[key]
            if key == (0, 1) and z < nrow - 1:
                continue            # exit side replaced by interface edges
            if key == (0, 0) and z > 0:
                continue            # inlet side replaced by interface edges
            BC.append(cells.ravel())
            BS.append(S.reshape(-1, 3))
    for z in range(nrow - 1):
        _, sA, _ = blocks[z]
        _, sB, _ = blocks[z + 1]
        cA, SA = sA[(0, 1)]        # [nt, nr], outward (+x)
        cB, _ = sB[(0, 0)]
        # odd rows are shifted by half a cell in pitch fraction.  For z even, upstream
        # cell j covers [j, j+1) and downstream cell j' covers [j'+1/2, j'+3/2), so j
        # overlaps j' in {j-1, j}; for z odd the shift is reversed and j' in {j, j+1}.
        # Each overlap is half the upstream face (periodic in j).
        partners = (-1, 0) if z % 2 == 0 else (0, 1)
        for j in range(nt):
            for dj in partners:
                EA.append(cA[j, :].ravel())
                EB.append(cB[(j + dj) % nt, :].ravel())
                ES.append(0.5 * SA[j, :].reshape(-1, 3))
    ea = np.concatenate(EA)
    eb = np.concatenate(EB)
    eS = np.concatenate(ES)
    bc = np.concatenate(BC)
    bS = np.concatenate(BS)
    meta = {"kind": "multi_row", "shape": (nx, nt, nr), "n_blades": tuple(n_blades),
            "seed": seed, "theta": np.concatenate(thetas), "radius": np.concatenate(radii),
            "xi": np.concatenate(fracs), "row": np.concatenate(rows)}
    return _finish(base, ea, eb, eS, bc, bS, np.concatenate(vols), np.concatenate(cens),
                   np.concatenate(zones), rng, permute, nrow, n_blades, meta)


def chain(n: int, seed: int = 3, permute: bool = False) -> Mesh:
    """1-D chain of n cells along x (one cell in the other two directions)."""
    return passage_block(n, 1, 1, 36, seed=seed, jitter=0.0, permute=permute)


def _waves(xi):
    """e[d][k] = exp(i pi k xi_d) for k = 0, 1, 2 in each direction d."""
    out = []
    for d in range(3):
        e1 = np.exp(1j * np.pi * xi[:, d])
        out.append([None, e1, e1 * e1])
    return out


def _lowmode_field(rng, e):
    """Seeded sum of cosines with wave numbers 0..2 in each direction, scaled to [-1, 1]:
    f = sum over (kx, ky, kz) != 0 of c cos(pi (kx x + ky y + kz z) + ph), evaluated as the
    real part of sum_kx e^{i pi kx x} sum_ky e^{i pi ky y} sum_kz c e^{i ph} e^{i pi kz z}
    (e from _waves)."""
    a = np.zeros((3, 3, 3), np.complex128)
    for kx in range(3):
        for ky in range(3):
            for kz in range(3):
                if kx == ky == kz == 0:
                    continue
                c = rng.normal() / (1.0 + kx + ky + kz)
                ph = rng.uniform(0, 2 * np.pi)
                a[kx, ky, kz] = c * np.exp(1j * ph)
    n = e[0][1].shape[0]
    f = np.zeros(n, np.complex128)
    for kx in range(3):
        g = np.zeros(n, np.complex128)
        for ky in range(3):
            h = a[kx, ky, 0] + a[kx, ky, 1] * e[2][1] + a[kx, ky, 2] * e[2][2]
            g += h if ky == 0 else e[1][ky] * h
        f += g if kx == 0 else e[0][kx] * g
    f = f.real
    m = np.max(np.abs(f))
    return f / m if m > 0 else f


def rcb_partition(mesh: Mesh, cells_per_part: int) -> np.ndarray:
    """Partition of the cells into parts of at most cells_per_part cells by recursive
    coordinate bisection of the centroids (each split halves a part across its longest
    extent), the kind of domain decomposition a parallel solver distributes over
    processors.  Returns part[N] int32, parts numbered 0.. in bisection order."""
    part = np.zeros(mesh.n_cells, np.int32)
    if cells_per_part >= mesh.n_cells:
        return part
    c = mesh.centroid
    stack = [np.arange(mesh.n_cells)]
    out = []
    while stack:
        ids = stack.pop()
        if ids.size <= cells_per_part:
            out.append(ids)
            continue
        ext = c[ids].max(axis=0) - c[ids].min(axis=0)
        ax = int(np.argmax(ext))
        order = ids[np.argsort(c[ids, ax], kind="stable")]
        half = order.size // 2
        stack.append(order[half:])
        stack.append(order[:half])
    for k, ids in enumerate(out):
        part[ids] = k
    return part


def flow_state(mesh: Mesh, seed: int = 1) -> np.ndarray:
    """Smooth mean-flow conservative state per cell (user order), shape [N, 6]:
    (rho, rho u, rho v, rho w, rho E, rho nu~).  Ideal gas, gamma = 1.4."""
    rng = np.random.default_rng(10_000 + seed)
    meta = mesh.meta
    # structured fractional position, reordered to user ids
    s2u = meta["struct_to_user"]
    inv = np.empty_like(s2u)
    inv[s2u] = np.arange(mesh.n_cells)
    xi = meta["xi"][inv]
    th = meta["theta"][inv]
    waves = _waves(xi)
    f = [_lowmode_field(rng, waves) for _ in range(6)]
    rho = 1.0 + 0.05 * f[0]
    mach = 0.45 + 0.15 * f[1]
    a = 1.0 + 0.02 * f[2]
    p = rho * a * a / GAMMA
    swirl = 0.5 + 0.1 * f[3]
    speed = mach * a
    ux = speed * np.cos(swirl)
    ut = speed * np.sin(swirl)
    ur = 0.05 * f[4] * speed
    uy = -ut * np.sin(th) + ur * np.cos(th)
    uz = ut * np.cos(th) + ur * np.sin(th)
    nut = 10.0 ** (-4.0 + f[5])
    E = p / (GAMMA - 1.0) + 0.5 * rho * (ux * ux + uy * uy + uz * uz)
    return np.ascontiguousarray(np.stack([rho, rho * ux, rho * uy, rho * uz, E, rho * nut], axis=1))


def rhs(n_cells: int, s: int, real: bool = False, seed_base: int = 1000) -> np.ndarray:
    """Right-hand side of system s: i.i.d. N(0,1) real and imaginary parts (seed 1000+s),
    shape [N, 6] complex128; real when ``real`` (the mean system)."""
    rng = np.random.default_rng(seed_base + s)
    re = rng.standard_normal((n_cells, 6))
    im = np.zeros_like(re) if real else rng.standard_normal((n_cells, 6))
    return re + 1j * im


def blade_passing(n_blades: int, shaft_speed: float = 0.5) -> float:
    """Blade-passing angular frequency N_b * Omega (non-dimensional, a_ref = r_mid = 1)."""
    return n_blades * shaft_speed


def omegas_single_zone(n_harmonics: int, n_blades: int = 36, shaft_speed: float = 0.5) -> np.ndarray:
    """[1 + N_h, 1] table: the mean (0) followed by l * BPF, l = 1..N_h."""
    bpf = blade_passing(n_blades, shaft_speed)
    return np.array([[l * bpf] for l in range(n_harmonics + 1)], dtype=np.float64)


def omegas_multi_row(n_harmonics: int, n_blades=(36, 60, 48), shaft_speed: float = 0.5) -> np.ndarray:
    """[1 + N_h, n_rows] table of mixed per-row frequencies: row z sees multiples of the
    blade-passing frequency of its neighbouring rows (alternating upstream/downstream),
    with the sign flipped for every third harmonic (potential-field modes)."""
    nrow = len(n_blades)
    om = np.zeros((n_harmonics + 1, nrow))
    for l in range(1, n_harmonics + 1):
        for z in range(nrow):
            nb = n_blades[z - 1] if (l % 2 == 1 and z > 0) else n_blades[(z + 1) % nrow]
            sign = -1.0 if l % 3 == 0 else 1.0
            om[l, z] = sign * ((l + 1) // 2) * nb * shaft_speed
    return om


def batch_instances(n_inst: int = 64, total_cells: float = 8.0e6, seed: int = 3,
                    lo: float = 2.0e4, hi: float = 3.0e5):
    """Blade-row instance set: seeded log-uniform sizes in [lo, hi] rescaled towards the
    requested total, each a passage (2n', n', n') with n' = (N/2)^(1/3), blade count
    U{20..80}, harmonic count U{1..8}.  Returns a list of dicts (shape, n_blades,
    n_harmonics, seed)."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(lo), np.log(hi), n_inst))
    sizes = np.clip(sizes * total_cells / sizes.sum(), lo, hi)
    out = []
    for q, n in enumerate(sizes):
        m = max(2, int(round((n / 2.0) ** (1.0 / 3.0))))
        out.append({"shape": (2 * m, m, m), "n_blades": int(rng.integers(20, 81)),
                    "n_harmonics": int(rng.integers(1, 9)), "seed": 100 + q})
    return out


# layer shapes (in, out) of the learned preconditioner's five weight matrices
NN_SHAPES = ((60, 64), (88, 64), (128, 64), (128, 64), (64, 12))


def he_init(seed: int = 0) -> np.ndarray:
    """Initial network weights (float32, W1..W5 row-major [in][out] concatenated):
    normal with standard deviation sqrt(2 / fan_in); the output layer scaled by 0.1 so
    the first corrections are small."""
    rng = np.random.default_rng(seed)
    mats = [rng.standard_normal((a, b)) * np.sqrt(2.0 / a) for a, b in NN_SHAPES]
    mats[-1] = mats[-1] * 0.1
    return np.concatenate([m.reshape(-1) for m in mats]).astype(np.float32)
