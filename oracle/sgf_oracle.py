"""Plain FP64 CPU oracle of the Sparse Geometric Factorization (SGF) and of
CG preconditioned by it (Klockiewicz & Darve, arXiv 1907.03406).

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously correct
reference that the GPU library is checked against.  Only the test-suite,
the smoke check and the CPU-baseline leg of the benchmark may import it; the
GPU library never does, and this module never imports the GPU library.

Everything here is a direct transcription of the method's definitions into
NumPy, cluster by cluster, in the order the paper states:

* partition hierarchy of nested-dissection cells on a Cartesian grid
  (Sec. 5.1, Defs. 2.1-2.4),
* polynomial bases Pi^0, Pi^1, Pi^2 and their per-node blocks Phi_B
  (Sec. 3.1; block-diagonal per displacement component for vector
  problems, Eq. 7.4),
* per level: block-Cholesky elimination of interiors (Sec. 4.1, Eq. 4.2),
  polynomial compression of separators (Sec. 3.2, Eqs. 3.1-3.5 and 4.5-4.6),
  coarsening and stacking of Phi (Secs. 4.3-4.4, Eq. 4.7),
* exact Cholesky of the last node (Sec. 4.5), as in Algorithm 4.1,
* the preconditioner apply A_l^{-1} (Sec. 4.7), the product A_l (Sec. 2.1),
* CG with A_l^{-1} as preconditioner (Sec. 7).

Schemes (Sec. 5): Nest-All-All (every interaction of every separator cell but
the single-vertex cells is compressed), Nest-2-All (only the cells of
codimension one: faces in 3D, edges in 2D), Nest-2-2 (those cells, with the
couplings to the lower-dimensional cells on their boundary kept exactly by
putting their span into Q_1), and Gen-All-All (boxes of d^dim vertices, no
interiors, every cell compressed; Sec. 5.2).  Besides the polynomial
compression, the "standard low-rank equivalent" of Sec. 7.4 (Eq. 7.5): the
same factorization with Q taken from the pivoted QR of the scaled
off-diagonal block itself, truncated to the ranks a polynomial run recorded.
A user may also supply the near-kernel basis Pi directly (Secs. 1 and 3.1
allow any near-kernel space) instead of monomials of the coordinates.

Readings taken where the paper is silent (each listed in the design notes):
vertices at (i + 1/2) h with cutting slabs only on internal planes; global
coordinate normalisation for the monomials; ascending cluster ids for every
order; Householder QR with column pivoting whose pivot is the largest
recomputed trailing norm, near-ties (relative 1e-10) going to the lowest
index; numerical rank r = #{k : |R_kk| > rank_tol * |R_00|}; a separator is
compressed only when r < its size.
"""
import numpy as np
import scipy.linalg as sla

NEST_ALL_ALL = 0
NEST_2_ALL = 1
NEST_2_2 = 2
GEN_ALL_ALL = 3

POLYNOMIAL = 0
LOW_RANK = 1

STOP_ROOT = 0
STOP_PAPER = 1

TIE_RTOL = 1e-10


# ---------------------------------------------------------------------------
# Partition hierarchy (Sec. 5.1)
# ---------------------------------------------------------------------------

def axis_classes(N, d):
    """Per-axis cell classes at period d (Sec. 5.1 cutting planes).

    Index i lies on a cutting slab iff (i + 1) is a multiple of d and the slab
    is an internal plane (i <= N - 2).  The class of i is
    2 * (#slabs below i) + [i on a slab]: even classes are the open blocks
    between slabs, odd classes are the slabs.  Returns (classes, #classes).
    """
    i = np.arange(N)
    slab = ((i + 1) % d == 0) & (i <= N - 2)
    below = np.cumsum(slab) - slab
    return (2 * below + slab).astype(np.int64), int(2 * slab.sum() + 1)


def axis_boxes(N, d):
    """Per-axis classes of the general partition at period d (Sec. 5.2): the
    boxes (r d h, (r + 1) d h) hold the vertices r d .. r d + d - 1 (vertex i
    at (i + 1/2) h), so the class of i is i // d; the last box of an axis
    whose length is not a multiple of d is shorter.  Returns (classes,
    #classes)."""
    i = np.arange(N)
    return (i // d).astype(np.int64), int((N + d - 1) // d)


class Level:
    """Cells of one partition P_t: cell id of every grid node, number of
    cells, and each cell's type (number of odd per-axis classes: 0 = interior
    block; 1 = face in 3D / edge in 2D; ...; dim = corner vertex).  In a
    general partition (Sec. 5.2) every box has type 1: none is an interior,
    all are compressed."""

    def __init__(self, grid, d, general=False):
        self.d = d
        self.general = general
        cls, K = zip(*((axis_boxes if general else axis_classes)(N, d) for N in grid))
        self.K = K
        # cell id = cx + Kx * (cy + Ky * cz): lexicographic, x fastest
        mesh = np.meshgrid(*[c for c in cls[::-1]], indexing="ij")
        per_axis = [m.ravel() for m in mesh[::-1]]
        cid = np.zeros_like(per_axis[0])
        odd = np.zeros_like(per_axis[0])
        for a in reversed(range(len(grid))):
            cid = cid * K[a] + per_axis[a]
            odd += per_axis[a] & 1
        self.cell_of_node = cid
        self.ncells = int(np.prod(K))
        self.type = np.zeros(self.ncells, dtype=np.int64)
        self.type[cid] = 1 if general else odd
        self.is_root = all(k == 1 for k in K)

    def classes(self, cid):
        """Per-axis classes of cell cid (x first)."""
        out = []
        for k in self.K:
            out.append(cid % k)
            cid //= k
        return tuple(out)

    def on_boundary(self, B, Y):
        """Whether cell Y lies on the boundary of cell B (Sec. 5.1): Y != B,
        Y has B's class on every axis where B is a slab (odd class), and a
        class within one of B's on the other axes.  For a face these are the
        edges and corners around it; for an edge in 2D its two end corners."""
        if B == Y:
            return False
        for cb, cy in zip(self.classes(B), self.classes(Y)):
            if cb % 2 == 1 and cy != cb:
                return False
            if abs(cy - cb) > 1:
                return False
        return True


def partition_hierarchy(grid, leaf, general=False):
    """Levels t = 1, 2, ... with d_t = leaf * 2^(t-1), up to the first level
    whose partition is the single set V (nested dissection: no axis has an
    internal slab; general boxes: one box per axis)."""
    levels = []
    t = 1
    while True:
        lev = Level(grid, leaf * 2 ** (t - 1), general)
        levels.append(lev)
        if lev.is_root:
            return levels
        t += 1


def father_map(lv, lv_next):
    """Father of every cell of lv in the coarser partition lv_next
    (Sec. 4.3); well defined because the coarser slabs are a subset."""
    f = np.full(lv.ncells, -1, dtype=np.int64)
    f[lv.cell_of_node] = lv_next.cell_of_node
    return f


# ---------------------------------------------------------------------------
# Polynomial basis (Sec. 3.1, Eq. 7.4)
# ---------------------------------------------------------------------------

def monomials(coords, q):
    """Columns 1; x, y[, z]; x^2, y^2[, z^2], xy[, yz, zx] of the globally
    normalised coordinates xh = 2 (x - min) / (max - min) - 1 (0 on a
    degenerate axis)."""
    c = np.asarray(coords, dtype=np.float64)
    lo, hi = c.min(axis=0), c.max(axis=0)
    span = np.where(hi > lo, hi - lo, 1.0)
    xh = np.where(hi > lo, 2.0 * (c - lo) / span - 1.0, 0.0)
    dim = c.shape[1]
    cols = [np.ones(c.shape[0])]
    if q >= 1:
        cols += [xh[:, a] for a in range(dim)]
    if q >= 2:
        cols += [xh[:, a] ** 2 for a in range(dim)]
        if dim == 2:
            cols += [xh[:, 0] * xh[:, 1]]
        else:
            cols += [xh[:, 0] * xh[:, 1], xh[:, 1] * xh[:, 2], xh[:, 2] * xh[:, 0]]
    if q > 2:
        raise ValueError("polynomial degree q must be 0, 1 or 2")
    return np.stack(cols, axis=1)


def poly_basis(coords, q, dpn):
    """Global Pi (n x pi): monomials per node; for dpn > 1, block diagonal
    per displacement component (Eq. 7.4) with node-major unknowns."""
    mono = monomials(coords, q)
    if dpn == 1:
        return mono
    nn, p0 = mono.shape
    Pi = np.zeros((nn * dpn, p0 * dpn))
    for c in range(dpn):
        Pi[c::dpn, c * p0:(c + 1) * p0] = mono
    return Pi


# ---------------------------------------------------------------------------
# Householder QR with column pivoting (the QR of Eq. 3.3)
# ---------------------------------------------------------------------------

def householder(x):
    """Reflector H = I - tau v v^T with v[0] = 1 mapping x to beta e_1.
    beta = -sign(x0) ||x|| (sign(0) = +1); when x[1:] = 0 no reflection is
    taken (tau = 0, beta = x0)."""
    alpha = x[0]
    tail = np.dot(x[1:], x[1:])
    v = np.zeros_like(x)
    v[0] = 1.0
    if tail == 0.0:
        return v, 0.0, alpha
    norm = np.sqrt(alpha * alpha + tail)
    beta = -norm if alpha >= 0.0 else norm
    v[1:] = x[1:] / (alpha - beta)
    return v, (beta - alpha) / beta, beta


def qrcp(N, rank_tol):
    """Column-pivoted Householder QR of N, stopped at the numerical rank.

    Step k picks, among the remaining columns, the one with the largest
    2-norm of its trailing part (recomputed, not downdated); norms within a
    relative TIE_RTOL of the largest count as equal and the lowest column
    index wins.  The factorization stops at the first k with
    max trailing norm <= rank_tol * |R_00|, which defines the rank r.
    Returns (V, tau, r, diagR): V is m x r (unit lower trapezoidal), tau the
    r reflector coefficients, so that Q = H_0 H_1 ... H_{r-1} and its first r
    columns Q_1 span range(N) up to the dropped tail.
    """
    A = np.array(N, dtype=np.float64, copy=True)
    m, c = A.shape
    diag_next = 0.0
    V = np.zeros((m, 0))
    taus = []
    diag = []
    r00 = None
    cols = list(range(c))
    for k in range(min(m, c)):
        norms = np.sqrt(np.sum(A[k:, k:] ** 2, axis=0))
        nmax = norms.max() if norms.size else 0.0
        if r00 is None:
            r00 = nmax
        if nmax == 0.0 or nmax <= rank_tol * r00:
            diag_next = nmax
            break
        j = int(np.nonzero(norms >= nmax * (1.0 - TIE_RTOL))[0][0]) + k
        if j != k:
            A[:, [k, j]] = A[:, [j, k]]
            cols[k], cols[j] = cols[j], cols[k]
        v, tau, beta = householder(A[k:, k].copy())
        if tau != 0.0:
            A[k:, k:] -= tau * np.outer(v, v @ A[k:, k:])
        A[k, k] = beta
        A[k + 1:, k] = 0.0
        col = np.zeros(m)
        col[k:] = v
        V = np.hstack([V, col[:, None]])
        taus.append(tau)
        diag.append(beta)
    qrcp.last_dropped = diag_next / r00 if r00 else 0.0
    return V, np.array(taus), V.shape[1], np.array(diag)


def qrcp_fixed_rank(N, r):
    """The pivoted Householder QR of qrcp (same pivot, tie and reflector
    rules) run for exactly min(r, #rows, #cols) steps instead of stopping at
    a threshold: the truncation of the rank-revealing QR of Eq. 7.5 to a
    given number r of columns of Q_1.  A step whose trailing part is zero
    takes no reflection (tau = 0).  Returns (V, tau, r, diagR) as qrcp,
    with r the requested size of Q_1 (the first r columns of
    Q = H_0 ... H_{k-1})."""
    A = np.array(N, dtype=np.float64, copy=True)
    m, c = A.shape
    V = np.zeros((m, 0))
    taus, diag = [], []
    for k in range(min(r, m, c)):
        norms = np.sqrt(np.sum(A[k:, k:] ** 2, axis=0))
        nmax = norms.max()
        j = k if nmax == 0.0 else int(np.nonzero(norms >= nmax * (1.0 - TIE_RTOL))[0][0]) + k
        if j != k:
            A[:, [k, j]] = A[:, [j, k]]
        v, tau, beta = householder(A[k:, k].copy())
        if tau != 0.0:
            A[k:, k:] -= tau * np.outer(v, v @ A[k:, k:])
        A[k, k] = beta
        A[k + 1:, k] = 0.0
        col = np.zeros(m)
        col[k:] = v
        V = np.hstack([V, col[:, None]])
        taus.append(tau)
        diag.append(beta)
    return V, np.array(taus), r, np.array(diag)


def apply_qt(V, tau, X):
    """Q^T X = H_{r-1} ... H_0 X."""
    Y = np.array(X, dtype=np.float64, copy=True)
    Y2 = Y.reshape(Y.shape[0], -1)
    for k in range(V.shape[1]):
        v = V[:, k]
        Y2 -= tau[k] * np.outer(v, v @ Y2)
    return Y


def apply_q(V, tau, X):
    """Q X = H_0 ... H_{r-1} X."""
    Y = np.array(X, dtype=np.float64, copy=True)
    Y2 = Y.reshape(Y.shape[0], -1)
    for k in reversed(range(V.shape[1])):
        v = V[:, k]
        Y2 -= tau[k] * np.outer(v, v @ Y2)
    return Y


# ---------------------------------------------------------------------------
# The factorization (Algorithm 4.1)
# ---------------------------------------------------------------------------

class Options:
    """compression = POLYNOMIAL (Eq. 3.2) or LOW_RANK (Eq. 7.5, with the
    ranks recorded by a polynomial run in ``ranks``: F.info["ranks"]);
    basis = a user near-kernel basis Pi (n x pi) replacing the monomials of
    degree q (then q and the coordinates are not used).

    low_rank_blocks (LOW_RANK only): "current" forms each separator's
    off-diagonal block from the matrix as it stands when that separator is
    compressed, after the compressions before it in the level (the
    sequential recursion of Sec. 3.2 run with Q from Eq. 7.5); "level" forms
    every separator's block from the matrix as it stands after the level's
    eliminations, before any of its compressions.  For the polynomial
    compression the two are the same operator (the filtered columns of a
    compressed neighbour do not change, Sec. 3.2); for the low-rank
    equivalent they differ, and "level" makes the compressions of a level
    independent of their order."""

    def __init__(self, q=1, leaf=8, compress=True, compress_from_level=1,
                 scheme=NEST_ALL_ALL, rank_tol=1e-12, stop_rule=STOP_ROOT,
                 order="ascending", seed=0, compression=POLYNOMIAL, ranks=None, basis=None,
                 low_rank_blocks="current"):
        self.q = q
        self.leaf = leaf
        self.compress = compress
        self.compress_from_level = compress_from_level
        self.scheme = scheme
        self.rank_tol = rank_tol
        self.stop_rule = stop_rule
        self.order = order      # compression order inside a level
        self.seed = seed        # for order == "shuffled"
        self.compression = compression
        self.ranks = ranks
        self.basis = basis
        if low_rank_blocks not in ("current", "level"):
            raise ValueError("low_rank_blocks must be 'current' or 'level'")
        self.low_rank_blocks = low_rank_blocks


class Factor:
    """A_l as the list of its elementary steps.

    ops[t] for level t holds ('elim', vars_I, L_I, [(vars_S, W_S), ...]) for
    every interior, then ('comp', vars_B, L_B, V_B, tau_B, r_B) for every
    compressed separator.  vars are slots of the global unknown vector: a
    compression rewrites the slots of B in place, its first r slots being
    the coarse unknowns that stay active.  top = (vars, L).
    """

    def __init__(self):
        self.levels = []
        self.top = None
        self.info = {"ranks": [], "sizes": [], "gap": []}


def _compressible(typ, dim, scheme):
    if scheme == GEN_ALL_ALL:       # every box of a general partition
        return True
    if typ == 0 or typ == dim:      # interiors; 0-cells: nothing to compress
        return False
    if scheme == NEST_ALL_ALL:
        return True
    if scheme in (NEST_2_ALL, NEST_2_2):
        return typ == 1             # cells of codimension one
    raise ValueError("unknown scheme")


def factorize(A, coords, grid, dpn, opt):
    """SGF of the sparse SPD matrix A (scipy sparse, n x n) on the Cartesian
    grid ``grid`` with ``dpn`` unknowns per node (Algorithm 4.1)."""
    A = A.tocsr()
    n = A.shape[0]
    dim = len(grid)
    Pi = poly_basis(coords, opt.q, dpn) if opt.basis is None else np.asarray(opt.basis, dtype=np.float64)
    if Pi.shape[0] != n:
        raise ValueError("the basis must have one row per unknown")
    levels = partition_hierarchy(grid, opt.leaf, general=opt.scheme == GEN_ALL_ALL)
    F = Factor()

    # ---- level-1 nodes: active sets, Phi_B = Pi(B, :), blocks of A -------
    lv = levels[0]
    cell_dof = np.repeat(lv.cell_of_node, dpn)
    order = np.argsort(cell_dof, kind="stable")   # ascending dof inside a cell
    bounds = np.searchsorted(cell_dof[order], np.arange(lv.ncells + 1))
    vars_of = {}
    for c in range(lv.ncells):
        if bounds[c + 1] > bounds[c]:
            vars_of[c] = order[bounds[c]:bounds[c + 1]]
    Phi = {c: Pi[v] for c, v in vars_of.items()}
    blocks = {}
    nbr = {c: set() for c in vars_of}
    coo = A.tocoo()
    pair = set(zip(cell_dof[coo.row].tolist(), cell_dof[coo.col].tolist()))
    for (a, b) in pair:
        if a != b:
            nbr[a].add(b)
    for a in vars_of:
        rows = A[vars_of[a]]
        for b in [a] + sorted(nbr[a]):
            blocks[(a, b)] = rows[:, vars_of[b]].toarray()

    max_node = max(len(v) for v in vars_of.values())
    t = 0
    while True:
        lv = levels[t]
        n_active = sum(len(v) for v in vars_of.values())
        stop_now = lv.is_root or (opt.stop_rule == STOP_PAPER and t > 0 and n_active < max_node)
        if stop_now:
            # ---- top: exact Cholesky of what is left (Sec. 4.5) -----------
            ids = sorted(vars_of)
            allv = np.concatenate([vars_of[c] for c in ids]) if ids else np.zeros(0, dtype=np.int64)
            off = np.cumsum([0] + [len(vars_of[c]) for c in ids])
            M = np.zeros((len(allv), len(allv)))
            for i, a in enumerate(ids):
                for j, b in enumerate(ids):
                    if (a, b) in blocks:
                        M[off[i]:off[i + 1], off[j]:off[j + 1]] = blocks[(a, b)]
            L = np.linalg.cholesky(M) if len(allv) else np.zeros((0, 0))
            F.top = (allv, L)
            F.info["top_size"] = len(allv)
            F.info["nlevels"] = t + 1
            return F
        ops = []
        # ---- eliminate interiors (Sec. 4.1, Eq. 4.2) -----------------------
        interiors = sorted(c for c in vars_of if lv.type[c] == 0)
        for I in interiors:
            S = sorted(nbr[I])
            L = np.linalg.cholesky(blocks[(I, I)])
            W = [sla.solve_triangular(L, blocks[(I, s)], lower=True) for s in S]
            for ia, a in enumerate(S):
                for ib, b in enumerate(S):
                    upd = W[ia].T @ W[ib]
                    if (a, b) in blocks:
                        blocks[(a, b)] = blocks[(a, b)] - upd
                    else:
                        blocks[(a, b)] = -upd
                        nbr[a].add(b)
            ops.append(("elim", vars_of[I], L, [(vars_of[s], w) for s, w in zip(S, W)]))
            for s in S:
                nbr[s].discard(I)
                del blocks[(s, I)]
                del blocks[(I, s)]
            del blocks[(I, I)]
            del nbr[I], vars_of[I], Phi[I]
        # ---- compress separators (Sec. 3.2 / 4.2) ---------------------------
        ranks = {}
        do_comp = opt.compress and (t + 1) >= opt.compress_from_level
        seps = sorted(c for c in vars_of if _compressible(lv.type[c], dim, opt.scheme))
        if opt.order == "descending":
            seps = seps[::-1]
        elif opt.order == "shuffled":
            seps = list(np.random.default_rng(opt.seed).permutation(seps))
        # the level's blocks before any of its compressions (low-rank
        # equivalent with blocks taken per level, see Options)
        level_blocks = dict(blocks) if opt.compression == LOW_RANK and opt.low_rank_blocks == "level" else None
        for B in (seps if do_comp else []):
            X = sorted(nbr[B])
            s = len(vars_of[B])
            L = np.linalg.cholesky(blocks[(B, B)])                        # Eq. 3.1
            Mh = [sla.solve_triangular(L, blocks[(B, x)], lower=True) for x in X]
            if opt.compression == LOW_RANK:
                # Eq. 7.5: Q from the pivoted QR of the scaled off-diagonal
                # block [M^_BX1 | M^_BX2 | ...], cut at the recorded size
                r_rec = opt.ranks[t][B]
                if r_rec >= s:
                    ranks[B] = r_rec
                    continue
                src = Mh if level_blocks is None else \
                    [sla.solve_triangular(L, level_blocks[(B, x)], lower=True) for x in X]
                N = np.hstack(src) if src else np.zeros((s, 0))
                V, tau, r, dR = qrcp_fixed_rank(N, r_rec)
                gap_in, dropped = 0.0, 0.0
            else:
                # Eq. 4.5; in Nest-2-2 the couplings to the cells on B's
                # boundary enter N whole, so their span is kept in Q_1 (Sec. 5.1)
                cols = [L.T @ Phi[B]]
                for m, x in zip(Mh, X):
                    full = opt.scheme == NEST_2_2 and lv.on_boundary(B, x)
                    cols.append(m if full else m @ Phi[x])
                N = np.hstack(cols)
                V, tau, r, dR = qrcp(N, opt.rank_tol)                      # Eq. 3.3
                gap_in = abs(dR[-1] / dR[0]) if r else 0.0
                dropped = qrcp.last_dropped
            ranks[B] = r
            F.info["gap"].append((t + 1, B, s, r, gap_in, dropped))
            if r >= s:
                continue
            vB = vars_of[B]
            ops.append(("comp", vB, L, V, tau, r))
            blocks[(B, B)] = np.eye(r)
            for m, x in zip(Mh, X):
                C = apply_qt(V, tau, m)[:r]
                blocks[(B, x)] = C
                blocks[(x, B)] = C.T.copy()
            Phi[B] = apply_qt(V, tau, L.T @ Phi[B])[:r]                    # Eq. 4.6
            vars_of[B] = vB[:r]
        F.levels.append(ops)
        F.info["ranks"].append(ranks)
        F.info["sizes"].append({c: len(v) for c, v in vars_of.items()})
        # ---- coarsen (Secs. 4.3-4.4, Eq. 4.7) -------------------------------
        nxt = levels[t + 1]
        fa = father_map(lv, nxt)
        kids = {}
        for c in sorted(vars_of):
            kids.setdefault(int(fa[c]), []).append(c)
        new_vars, new_phi, new_blocks, new_nbr, loc = {}, {}, {}, {}, {}
        for D, ch in kids.items():
            new_vars[D] = np.concatenate([vars_of[c] for c in ch])
            new_phi[D] = np.vstack([Phi[c] for c in ch])
            o = 0
            for c in ch:
                loc[c] = (D, o)
                o += len(vars_of[c])
            new_nbr[D] = set()
        for (a, b), M in blocks.items():
            Da, oa = loc[a]
            Db, ob = loc[b]
            if (Da, Db) not in new_blocks:
                new_blocks[(Da, Db)] = np.zeros((len(new_vars[Da]), len(new_vars[Db])))
            new_blocks[(Da, Db)][oa:oa + M.shape[0], ob:ob + M.shape[1]] = M
            if Da != Db:
                new_nbr[Da].add(Db)
        vars_of, Phi, blocks, nbr = new_vars, new_phi, new_blocks, new_nbr
        max_node = max([max_node] + [len(v) for v in vars_of.values()])
        t += 1


# ---------------------------------------------------------------------------
# Using the factor (Secs. 2.1 and 4.7)
# ---------------------------------------------------------------------------

def apply_inverse(F, r):
    """z = A_l^{-1} r: G_1^{-1}, B_1^{-1}, ..., top solve, then the
    transposed sweep back (Sec. 4.7).  r may be a vector or n x k."""
    y = np.array(r, dtype=np.float64, copy=True)
    for ops in F.levels:
        for op in ops:
            if op[0] == "elim":
                _, vI, L, Ws = op
                yI = sla.solve_triangular(L, y[vI], lower=True)
                y[vI] = yI
                for vS, W in Ws:
                    y[vS] -= W.T @ yI
        for op in ops:
            if op[0] == "comp":
                _, vB, L, V, tau, rk = op
                y[vB] = apply_qt(V, tau, sla.solve_triangular(L, y[vB], lower=True))
    vT, LT = F.top
    if len(vT):
        y[vT] = sla.cho_solve((LT, True), y[vT])
    for ops in reversed(F.levels):
        for op in ops:
            if op[0] == "comp":
                _, vB, L, V, tau, rk = op
                y[vB] = sla.solve_triangular(L.T, apply_q(V, tau, y[vB]), lower=False)
        for op in ops:
            if op[0] == "elim":
                _, vI, L, Ws = op
                acc = y[vI].copy()
                for vS, W in Ws:
                    acc -= W @ y[vS]
                y[vI] = sla.solve_triangular(L.T, acc, lower=False)
    return y


def multiply(F, v):
    """y = A_l v with A_l = G_1 B_1 ... G_l G_l^T ... B_1^T G_1^T (Sec. 2.1),
    applying the transposed factors first.  Uses only products with L, so it
    stays accurate on ill-conditioned problems."""
    y = np.array(v, dtype=np.float64, copy=True)
    for ops in F.levels:
        for op in ops:
            if op[0] == "elim":                  # G_I^T: y_I <- L^T y_I + W y_S
                _, vI, L, Ws = op
                acc = L.T @ y[vI]
                for vS, W in Ws:
                    acc += W @ y[vS]
                y[vI] = acc
        for op in ops:
            if op[0] == "comp":                  # B^T: y_B <- Q^T L^T y_B
                _, vB, L, V, tau, rk = op
                y[vB] = apply_qt(V, tau, L.T @ y[vB])
    vT, LT = F.top
    if len(vT):
        y[vT] = LT @ (LT.T @ y[vT])
    for ops in reversed(F.levels):
        for op in ops:
            if op[0] == "comp":                  # B: y_B <- L Q y_B
                _, vB, L, V, tau, rk = op
                y[vB] = L @ apply_q(V, tau, y[vB])
        for op in ops:
            if op[0] == "elim":                  # G_I: y_S += W^T y_I, y_I <- L y_I
                _, vI, L, Ws = op
                yI = y[vI].copy()
                for vS, W in Ws:
                    y[vS] += W.T @ yI
                y[vI] = L @ yI
    return y


def pcg(A, b, precond, tol=1e-10, maxit=500):
    """Preconditioned CG (Hestenes-Stiefel), x0 = 0.  Stops when the
    recursively updated residual satisfies ||r|| / ||b|| < tol.  Returns
    (x, iterations, recursive relative residual)."""
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    z = precond(r)
    p = z.copy()
    rz = r @ z
    for k in range(1, maxit + 1):
        Ap = A @ p
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        rel = np.linalg.norm(r) / nb
        if rel < tol:
            return x, k, rel
        z = precond(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit, rel


def factor_entries(F):
    """Number of stored factor entries (L_I, W, L_B, reflectors, top)."""
    tot = 0
    for ops in F.levels:
        for op in ops:
            if op[0] == "elim":
                m = len(op[1])
                tot += m * (m + 1) // 2 + sum(W.size for _, W in op[3])
            else:
                s = len(op[1])
                tot += s * (s + 1) // 2 + op[3].size
    m = len(F.top[0])
    return tot + m * (m + 1) // 2
