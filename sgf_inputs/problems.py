"""Synthetic SPD test matrices on Cartesian grids, in CSR form.

Numbering (shared by every consumer): grid node ``(ix, iy[, iz])`` has id
``ix + gx * (iy + gy * iz)`` (x fastest) and its ``dpn`` unknowns are
``node * dpn + comp``.  ``coords`` holds the physical node positions,
``coords[node, axis]``.

Scalar problems (Poisson-type): cell-centred finite differences for
``-div(a grad u) = f`` on the unit square / cube with Dirichlet data.  The
unknowns sit at ``x_i = (i + 1) h`` with ``h = 1 / (N + 1)``; the face
coefficient is the harmonic mean of ``a`` at the two face end points (the
two-point flux approximation), boundary end points included.  The matrix is
multiplied by ``h**2`` so that its entries are O(1): the row of node ``p``
is ``sum_f a_f`` on the diagonal and ``-a_f`` towards each neighbour.

Vector problem (linear elasticity): trilinear (Q1) hexahedral finite
elements on a uniform node grid over [0,1]^3, 2x2x2 Gauss quadrature,
isotropic material per element, the x = 0 face clamped.  The element matrix
is divided by the element size so that entries are O(1).
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .rng import uniform, normal


@dataclass
class Problem:
    name: str
    grid: tuple          # free grid nodes per axis (gx, gy[, gz])
    dpn: int             # unknowns per grid node
    coords: np.ndarray   # (n_nodes, dim) physical positions
    indptr: np.ndarray   # int64, n + 1
    indices: np.ndarray  # int32, nnz (sorted within each row)
    data: np.ndarray     # float64, nnz
    meta: dict = field(default_factory=dict)

    @property
    def dim(self):
        return len(self.grid)

    @property
    def n(self):
        return int(self.indptr.shape[0] - 1)

    @property
    def nnz(self):
        return int(self.indices.shape[0])

    def csr(self):
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))


def _to_csr(rows, cols, vals, n):
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return (A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64))


def _node_points(grid, h):
    """(n_nodes, dim) positions (i + 1) h, x fastest."""
    axes = [(np.arange(N) + 1.0) * h[a] for a, N in enumerate(grid)]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")  # shape (gz, gy, gx)
    return np.stack([m.ravel() for m in mesh[::-1]], axis=1)


def poisson_fd(grid, coef=None, name="poisson"):
    """Finite-difference ``-div(a grad u)`` with harmonic face means.

    ``coef`` maps an (m, dim) array of positions to m positive values; None
    means a = 1, giving the integer stencil (2 dim, -1).
    """
    grid = tuple(int(g) for g in grid)
    dim = len(grid)
    h = [1.0 / (N + 1) for N in grid]
    pts = _node_points(grid, h)
    n = pts.shape[0]
    shape = tuple(reversed(grid))
    f = (lambda x: np.ones(x.shape[0])) if coef is None else coef
    a_node = f(pts).reshape(shape)
    ids = np.arange(n).reshape(shape)
    diag = np.zeros(shape)
    rows, cols, vals = [], [], []

    def harm(p, q):
        return 2.0 * p * q / (p + q)

    for a in range(dim):
        ax = dim - 1 - a
        sl_lo = [slice(None)] * dim
        sl_hi = [slice(None)] * dim
        sl_lo[ax] = slice(0, -1)
        sl_hi[ax] = slice(1, None)
        ap, aq = a_node[tuple(sl_lo)], a_node[tuple(sl_hi)]
        af = harm(ap, aq)
        diag[tuple(sl_lo)] += af
        diag[tuple(sl_hi)] += af
        ip, iq = ids[tuple(sl_lo)].ravel(), ids[tuple(sl_hi)].ravel()
        rows += [ip, iq]
        cols += [iq, ip]
        vals += [-af.ravel(), -af.ravel()]
        for side, xb in ((0, 0.0), (-1, 1.0)):
            sl = [slice(None)] * dim
            sl[ax] = side
            layer = ids[tuple(sl)].ravel()
            bp = pts[layer].copy()
            bp[:, a] = xb
            ab = f(bp).reshape(a_node[tuple(sl)].shape)
            diag[tuple(sl)] += harm(a_node[tuple(sl)], ab)
    rows.append(ids.ravel())
    cols.append(ids.ravel())
    vals.append(diag.ravel())
    indptr, indices, data = _to_csr(np.concatenate(rows), np.concatenate(cols),
                                    np.concatenate(vals), n)
    return Problem(name=name, grid=grid, dpn=1, coords=pts, indptr=indptr,
                   indices=indices, data=data, meta={"h": h})


def gaussian_field_fourier(seed, dim, modes=64, corr_len=0.05, sigma=1.0):
    """a(x) = exp(g(x)), g a random-Fourier-feature Gaussian field:
    g(x) = sigma sqrt(2/M) sum_m cos(w_m . x + phi_m), w_m ~ N(0, corr_len^-2 I)
    (stream 1), phi_m ~ U[0, 2 pi) (stream 3)."""
    w = normal(seed, 1, modes * dim).reshape(modes, dim) / corr_len
    phi = uniform(seed, 3, modes, 0.0, 2.0 * np.pi)
    scale = sigma * np.sqrt(2.0 / modes)

    def coef(x):
        g = np.zeros(x.shape[0])
        for m in range(modes):
            g += np.cos(x @ w[m] + phi[m])
        return np.exp(scale * g)

    return coef


def blocky_log_field(seed, dim, nblk=8, lo=-2.0, hi=2.0):
    """a(x) = 10**u(x), u constant on each of nblk**dim equal boxes of the unit
    cube, u ~ U(lo, hi) per box (stream 2, box index x fastest)."""
    u = uniform(seed, 2, nblk ** dim, lo, hi)

    def coef(x):
        b = np.minimum(np.floor(x * nblk).astype(np.int64), nblk - 1)
        b = np.maximum(b, 0)
        idx = np.zeros(x.shape[0], dtype=np.int64)
        for a in reversed(range(dim)):
            idx = idx * nblk + b[:, a]
        return 10.0 ** u[idx]

    return coef


def _q1_unit_matrices():
    """Stiffness of the unit-cube Q1 element for (lambda, mu) = (1, 0) and
    (0, 1); node k = bx + 2 by + 4 bz, dof = 3 k + comp."""
    g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    bits = np.array([[k & 1, (k >> 1) & 1, (k >> 2) & 1] for k in range(8)])
    m = np.array([1, 1, 1, 0, 0, 0], dtype=float)
    Dl = np.outer(m, m)
    Dm = np.diag([2.0, 2.0, 2.0, 1.0, 1.0, 1.0])
    Kl = np.zeros((24, 24))
    Km = np.zeros((24, 24))
    for xi in g:
        for eta in g:
            for zeta in g:
                p = np.array([xi, eta, zeta])
                dN = np.zeros((8, 3))
                for k in range(8):
                    fac = np.where(bits[k] == 1, p, 1.0 - p)
                    sgn = np.where(bits[k] == 1, 1.0, -1.0)
                    for a in range(3):
                        o = [fac[c] for c in range(3) if c != a]
                        dN[k, a] = sgn[a] * o[0] * o[1]
                B = np.zeros((6, 24))
                for k in range(8):
                    dx, dy, dz = dN[k]
                    B[0, 3 * k + 0] = dx
                    B[1, 3 * k + 1] = dy
                    B[2, 3 * k + 2] = dz
                    B[3, 3 * k + 0], B[3, 3 * k + 1] = dy, dx
                    B[4, 3 * k + 1], B[4, 3 * k + 2] = dz, dy
                    B[5, 3 * k + 0], B[5, 3 * k + 2] = dz, dx
                Kl += 0.125 * B.T @ Dl @ B
                Km += 0.125 * B.T @ Dm @ B
    return Kl, Km


def elasticity_q1(nodes, seed=0, n_incl=20, r_lo=0.05, r_hi=0.15, E0=1.0,
                  E1=100.0, nu=0.3, name="elasticity"):
    """Q1 hexahedral linear elasticity on ``nodes`` x ``nodes`` x ``nodes``
    nodes over [0,1]^3, x = 0 face clamped.  Elements whose centroid lies in
    one of ``n_incl`` random balls (centres U[0,1]^3 from stream 2, radii
    U[r_lo, r_hi] from stream 4) get Young's modulus E1, the others E0."""
    N = int(nodes)
    ne = N - 1
    h = 1.0 / ne
    Kl, Km = _q1_unit_matrices()
    e = np.arange(ne)
    ez, ey, ex = np.meshgrid(e, e, e, indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    cen = np.stack([(ex + 0.5) * h, (ey + 0.5) * h, (ez + 0.5) * h], axis=1)
    E = np.full(cen.shape[0], E0)
    if n_incl > 0:
        c = uniform(seed, 2, 3 * n_incl).reshape(n_incl, 3)
        r = uniform(seed, 4, n_incl, r_lo, r_hi)
        inside = np.zeros(cen.shape[0], dtype=bool)
        for s in range(n_incl):
            inside |= np.sum((cen - c[s]) ** 2, axis=1) <= r[s] ** 2
        E[inside] = E1
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    # Node-block assembly: G[p, o] is the 3x3 coupling of full-grid node p
    # with its neighbour at offset o (27 offsets, (dz, dy, dx) lexicographic,
    # so neighbours come in ascending node id).  For a fixed corner pair (a, b)
    # every element hits a different node, so each scatter-add is collision-free.
    NN = N ** 3
    G = np.zeros((N, N, N, 27, 3, 3))     # (z, y, x) node, offset, comps
    bit = np.array([[k & 1, (k >> 1) & 1, (k >> 2) & 1] for k in range(8)])
    lam3 = lam.reshape(ne, ne, ne)[..., None, None]
    mu3 = mu.reshape(ne, ne, ne)[..., None, None]
    for a in range(8):
        bx, by, bz = bit[a]
        for b in range(8):
            d = bit[b] - bit[a]
            o = (d[0] + 1) + 3 * (d[1] + 1) + 9 * (d[2] + 1)
            G[bz:bz + ne, by:by + ne, bx:bx + ne, o] += (lam3 * Kl[3 * a:3 * a + 3, 3 * b:3 * b + 3]
                                                       + mu3 * Km[3 * a:3 * a + 3, 3 * b:3 * b + 3])
    G = G.reshape(NN, 27, 3, 3)
    # free numbering: drop ix = 0, free id = (ix - 1) + (N - 1) * (iy + N * iz)
    full = np.arange(NN)
    ix, iy, iz = full % N, (full // N) % N, full // (N * N)
    free_id = np.where(ix > 0, (ix - 1) + (N - 1) * (iy + N * iz), -1)
    off = np.array([(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])
    qx = ix[:, None] + off[None, :, 0]
    qy = iy[:, None] + off[None, :, 1]
    qz = iz[:, None] + off[None, :, 2]
    ok = (qx >= 1) & (qx < N) & (qy >= 0) & (qy < N) & (qz >= 0) & (qz < N) & (ix[:, None] > 0)
    q = np.where(ok, qx + N * (qy + N * qz), 0)
    fn = np.nonzero(ix > 0)[0]            # full ids of the free nodes, in free order
    okf = ok[fn]
    cnt = okf.sum(axis=1)
    n = 3 * (N - 1) * N * N
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.repeat(3 * cnt, 3), out=indptr[1:])
    # valid (node, offset) pairs, offsets ascending per node; j = rank of the pair in its row
    pp, oo = np.nonzero(okf)
    first = np.zeros(okf.shape[0] + 1, dtype=np.int64)
    np.cumsum(cnt, out=first[1:])
    j = np.arange(pp.shape[0]) - first[pp]
    col0 = 3 * free_id[q[fn[pp], oo]]
    blk = G[fn[pp], oo]                   # (M, 3, 3): [row comp, col comp]
    start = indptr[3 * pp]
    c = np.arange(3)
    dest = (start[:, None, None] + c[None, :, None] * (3 * cnt[pp])[:, None, None]
            + 3 * j[:, None, None] + c[None, None, :])
    indices = np.empty(indptr[-1], dtype=np.int32)
    data = np.empty(indptr[-1], dtype=np.float64)
    indices[dest] = (col0[:, None, None] + c[None, None, :]).astype(np.int32)
    data[dest] = blk
    gx = np.arange(1, N) * h
    gy = np.arange(N) * h
    Z, Y, X = np.meshgrid(gy, gy, gx, indexing="ij")
    coords = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return Problem(name=name, grid=(N - 1, N, N), dpn=3, coords=coords,
                   indptr=indptr, indices=indices, data=data,
                   meta={"h": h, "n_incl": n_incl, "E": (E0, E1), "nu": nu})


def random_rhs(seed, n, j=0):
    """Right-hand side j: i.i.d. U[-1, 1] from stream 1000 + j."""
    return uniform(seed, 1000 + j, n, -1.0, 1.0)


def rigid_body_modes(prob):
    """The six rigid-body displacement fields of a 3-D vector problem,
    restricted to its free unknowns: three translations and the rotations
    (-y, x, 0), (-z, 0, x), (0, -z, y)."""
    x, y, z = prob.coords[:, 0], prob.coords[:, 1], prob.coords[:, 2]
    nn = x.shape[0]
    out = np.zeros((3 * nn, 6))
    for c in range(3):
        out[c::3, c] = 1.0
    out[0::3, 3], out[1::3, 3] = -y, x
    out[0::3, 4], out[2::3, 4] = -z, x
    out[1::3, 5], out[2::3, 5] = -z, y
    return out


# Solver settings that go with each synthetic workload.
CONFIGS = {
    "poisson2d_64": dict(kind="poisson", grid=(64, 64), field=None, q=1, leaf=8, tol=1e-10),
    "varcoef2d_1024": dict(kind="poisson", grid=(1024, 1024), field="fourier", q=2, leaf=16, tol=1e-8),
    "varcoef3d_128": dict(kind="poisson", grid=(128, 128, 128), field="blocky", q=1, leaf=8, tol=1e-8),
    "elasticity3d_48": dict(kind="elasticity", nodes=48, q=1, leaf=6, tol=1e-8, nrhs=8),
}


def config_problem(key, seed=0, grid=None):
    """Build the problem of a named workload; ``grid`` overrides its size."""
    cfg = dict(CONFIGS[key])
    if cfg["kind"] == "elasticity":
        nodes = cfg["nodes"] if grid is None else int(grid)
        return elasticity_q1(nodes, seed=seed, name=key), cfg
    g = cfg["grid"] if grid is None else tuple(grid)
    dim = len(g)
    if cfg["field"] == "fourier":
        coef = gaussian_field_fourier(seed, dim)
    elif cfg["field"] == "blocky":
        coef = blocky_log_field(seed, dim)
    else:
        coef = None
    return poisson_fd(g, coef, name=key), cfg
