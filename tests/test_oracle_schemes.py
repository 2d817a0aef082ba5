"""Pins of the oracle's schemes and compression variants (Secs. 5.1-5.2,
7.4) and of its polynomial spaces, against what the paper and plain dense
linear algebra fix -- never against the oracle's own formulas:

* polynomials of the PHYSICAL coordinates, built here, are preserved
  (Prop. 6.1) for q = 1 and q = 2: a basis with a missing or wrong monomial
  fails, whatever Pi the oracle builds for itself;
* the cells each scheme compresses (closed-form counts per level);
* Nest-2-2 keeps the couplings of a compressed face with the cells on its
  boundary exactly: dense Schur complements of A and of A_l on the
  separators differ only between compressed faces (Sec. 5.1);
* Gen-All-All: closed-form box counts, exact mode = dense Cholesky,
  preservation, SPD (Lemma 3.1);
* the low-rank equivalent (Eq. 7.5): fixed-rank pivoted QR against LAPACK
  geqp3, same sizes as the polynomial run, and the E_1 / E_n contrast of
  Table 7.1 on the analytic eigenvectors of the Laplacian;
* a user-supplied near-kernel basis (rigid-body modes) is preserved, and
  q = 0 needs no coordinates.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import sgf_oracle as O
from sgf_inputs import problems as P


def _fourier(grid, seed=0):
    return P.poisson_fd(grid, P.gaussian_field_fourier(seed, len(grid)))


def _fact(p, **kw):
    A = p.csr()
    return A, O.factorize(A, p.coords, p.grid, p.dpn, O.Options(**kw))


def _physical_polys(coords, q):
    """Monomials of degree <= q in the raw physical coordinates (no
    normalisation, different column order from the oracle's)."""
    c = np.asarray(coords)
    dim = c.shape[1]
    cols = []
    if q >= 2:
        for a in range(dim):
            for b in range(a, dim):
                cols.append(c[:, a] * c[:, b])
    if q >= 1:
        cols += [3.0 * c[:, a] - 0.25 for a in range(dim)]
    cols.append(np.full(c.shape[0], 2.0))
    return np.stack(cols, axis=1)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ---------------------------------------------------------------------------
# Polynomial spaces (Sec. 3.1, Prop. 6.1), independent of the oracle's basis
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("grid,leaf,q,scheme", [((32, 32), 4, 2, O.NEST_ALL_ALL), ((32, 32), 4, 1, O.NEST_ALL_ALL),
                                                ((15, 15, 15), 4, 2, O.NEST_ALL_ALL),
                                                ((13, 12, 11), 3, 1, O.NEST_2_ALL),
                                                ((30, 28), 4, 2, O.GEN_ALL_ALL),
                                                ((12, 12, 12), 3, 1, O.GEN_ALL_ALL)])
def test_physical_polynomials_are_preserved_piecewise(grid, leaf, q, scheme):
    """A_l f = A f for every polynomial f of degree <= q in the physical
    coordinates, also restricted to each cell D of the last compressed
    partition (Prop. 6.1: E_i Pi_B = 0 and the top is exact)."""
    p = _fourier(grid)
    A, F = _fact(p, q=q, leaf=leaf, scheme=scheme)
    assert sum(1 for g in F.info["gap"] if g[3] < g[2]) > 0
    Pf = _physical_polys(p.coords, q)
    assert _rel(O.multiply(F, Pf), A @ Pf) <= 1e-10
    levels = O.partition_hierarchy(p.grid, leaf, general=scheme == O.GEN_ALL_ALL)
    last = levels[F.info["nlevels"] - 2]
    for D in np.unique(last.cell_of_node):
        PD = Pf * (last.cell_of_node == D)[:, None]
        assert _rel(O.multiply(F, PD), A @ PD) <= 1e-10


def test_degree_two_needs_every_quadratic():
    """With q = 1 the squares are NOT preserved (so the q = 2 pins above
    really test the quadratic columns).  x y is: on a 2D separator (a line,
    or a cross {y = y0} u {x = x0}) it equals -x0 y0 + y0 x + x0 y, a linear
    function, so only x^2 and y^2 tell q = 2 from q = 1 in 2D; in 3D y z is
    not linear on a face and needs its own column."""
    p = _fourier((32, 32))
    A, F = _fact(p, q=1, leaf=4)
    c = p.coords
    for f in (c[:, 0] ** 2, c[:, 1] ** 2):
        assert _rel(O.multiply(F, f), A @ f) > 1e-8
    assert _rel(O.multiply(F, c[:, 0] * c[:, 1]), A @ (c[:, 0] * c[:, 1])) <= 1e-12
    p3 = _fourier((15, 15, 15))
    A3, F3 = _fact(p3, q=1, leaf=4)
    c = p3.coords
    for f in (c[:, 0] * c[:, 1], c[:, 1] * c[:, 2], c[:, 2] * c[:, 0], c[:, 2] ** 2):
        assert _rel(O.multiply(F3, f), A3 @ f) > 1e-8


def test_monomial_span_has_full_dimension():
    """pi = 1, dim + 1 and (dim + 1)(dim + 2) / 2 independent columns
    (Sec. 3.1), spanning the physical monomials."""
    rng = np.random.default_rng(0)
    for dim in (2, 3):
        c = rng.uniform(0.1, 0.9, (200, dim))
        for q, pi in ((0, 1), (1, dim + 1), (2, (dim + 1) * (dim + 2) // 2)):
            M = O.monomials(c, q)
            assert M.shape[1] == pi and np.linalg.matrix_rank(M) == pi
            Pf = _physical_polys(c, q)
            coef, *_ = np.linalg.lstsq(M, Pf, rcond=None)
            assert np.abs(M @ coef - Pf).max() <= 1e-10 * np.abs(Pf).max()


# ---------------------------------------------------------------------------
# Which cells each scheme compresses (Sec. 5.1)
# ---------------------------------------------------------------------------

def _closed_form_cells(grid, d):
    """Number of blocks / slabs per axis at period d (internal slabs only)."""
    slabs = [len([i for i in range(N) if (i + 1) % d == 0 and i <= N - 2]) for N in grid]
    return slabs


@pytest.mark.parametrize("scheme,types", [(O.NEST_ALL_ALL, (1, 2)), (O.NEST_2_ALL, (1,)), (O.NEST_2_2, (1,))])
def test_compressed_cell_types_and_counts_3d(scheme, types):
    """3D grid 15^3, b = 4, q = 0: per level, the compression attempts are
    exactly the cells of the scheme's types (faces = type 1, edges = type 2;
    never interiors or single vertices), and their number is the closed
    form #faces = 3 k (k+1)^2, #edges = 3 k^2 (k+1) for k slabs per axis."""
    p = _fourier((15, 15, 15))
    A, F = _fact(p, q=0, leaf=4, scheme=scheme)
    levels = O.partition_hierarchy(p.grid, 4)
    for t in range(F.info["nlevels"] - 1):
        lv = levels[t]
        att = [g[1] for g in F.info["gap"] if g[0] == t + 1]
        assert all(int(lv.type[B]) in types for B in att)
        k = _closed_form_cells(p.grid, lv.d)[0]
        want = (3 * k * (k + 1) ** 2 if 1 in types else 0) + (3 * k * k * (k + 1) if 2 in types else 0)
        assert len(att) == want, (t, len(att), want)


def test_boundary_cells_closed_form():
    """on_boundary: an inner face has 4 edges and 4 corners around it, an
    inner edge of a 2D partition its 2 end corners."""
    lv = O.partition_hierarchy((23, 23, 23), 4)[0]
    faces = [c for c in range(lv.ncells) if lv.type[c] == 1 and all(0 < x < k - 1 for x, k in zip(lv.classes(c), lv.K))]
    for B in faces[:20]:
        nb = [Y for Y in range(lv.ncells) if lv.on_boundary(B, Y)]
        assert sorted(int(lv.type[Y]) for Y in nb) == [2, 2, 2, 2, 3, 3, 3, 3]
    lv2 = O.partition_hierarchy((23, 23), 4)[0]
    for B in range(lv2.ncells):
        if lv2.type[B] == 1 and all(0 < x < k - 1 for x, k in zip(lv2.classes(B), lv2.K)):
            nb = [Y for Y in range(lv2.ncells) if lv2.on_boundary(B, Y)]
            assert len(nb) == 2 and all(lv2.type[Y] == 2 for Y in nb)


def _sep_schur(M, sep):
    """Dense Schur complement of M on the index set sep."""
    itr = np.setdiff1d(np.arange(M.shape[0]), sep)
    return M[np.ix_(sep, sep)] - M[np.ix_(sep, itr)] @ np.linalg.solve(M[np.ix_(itr, itr)], M[np.ix_(itr, sep)])


@pytest.mark.parametrize("grid,leaf,q", [((31, 31), 16, 1), ((11, 11, 11), 6, 0)])
def test_nest22_keeps_boundary_couplings_exact(grid, leaf, q):
    """One compressed level followed by the exact top: the separators' Schur
    complement of A_l equals that of A everywhere except between two
    compressed faces (Sec. 5.1: only 2-cell interactions with non-adjacent
    cells are compressed).  Nest-2-All on the same 3D problem does change
    the face-edge couplings; in 2D it cannot: the cells on an edge's
    boundary are single vertices, whose Phi row holds the constant, so
    M^_BY Phi_Y already spans M^_BY and the two schemes coincide."""
    p = _fourier(grid, seed=3)
    lv = O.partition_hierarchy(p.grid, leaf)[0]
    assert len(O.partition_hierarchy(p.grid, leaf)) == 2
    typ = lv.type[lv.cell_of_node]
    sep = np.nonzero(typ > 0)[0]
    face = typ[sep] == 1
    Ad = p.csr().toarray()
    S = _sep_schur(Ad, sep)
    for scheme in (O.NEST_2_2, O.NEST_2_ALL):
        A, F = _fact(p, q=q, leaf=leaf, scheme=scheme)
        assert sum(1 for g in F.info["gap"] if g[3] < g[2]) > 0
        St = _sep_schur(O.multiply(F, np.eye(p.n)), sep)
        D = np.abs(S - St)
        ff = np.outer(face, face)
        # in compressed-to-compressed blocks only (diagonal blocks stay: L Q Q^T L^T = M_BB)
        cell = lv.cell_of_node[sep]
        same = cell[:, None] == cell[None, :]
        outside = D[~ff | same].max() / np.abs(S).max()
        inside = D[ff & ~same].max() / np.abs(S).max()
        if scheme == O.NEST_2_2 or len(grid) == 2:
            assert outside <= 1e-12, outside
            assert inside > 1e-6
        else:
            assert outside > 1e-6


# ---------------------------------------------------------------------------
# Gen-All-All (Sec. 5.2)
# ---------------------------------------------------------------------------

def test_general_partition_counts():
    """Boxes of d^dim vertices: ceil(N/d) per axis, sizes d (last one
    N - d floor((N-1)/d)), levels until one box remains; every box is
    compressible (no interiors)."""
    levels = O.partition_hierarchy((30, 17), 4, general=True)
    assert [lv.d for lv in levels] == [4, 8, 16, 32]
    for lv in levels:
        assert lv.K == (-(-30 // lv.d), -(-17 // lv.d))
        counts = np.bincount(lv.cell_of_node, minlength=lv.ncells)
        assert counts.max() == min(lv.d, 30) * min(lv.d, 17)
        assert set(np.unique(lv.type)) == {1}
    assert levels[-1].is_root


def test_general_exact_mode_and_spd():
    p = _fourier((20, 18), seed=2)
    A, F = _fact(p, q=1, leaf=4, scheme=O.GEN_ALL_ALL, compress=False)
    b = P.random_rhs(0, p.n)
    assert _rel(O.apply_inverse(F, b), np.linalg.solve(A.toarray(), b)) <= 1e-12
    A, F = _fact(p, q=1, leaf=4, scheme=O.GEN_ALL_ALL)
    Al = O.multiply(F, np.eye(p.n))
    assert np.abs(Al - Al.T).max() <= 1e-12 * np.abs(Al).max()
    assert np.linalg.eigvalsh(Al).min() > 0
    assert np.linalg.norm(Al - A.toarray()) > 1e-4 * np.linalg.norm(A.toarray())


def test_scheme_accuracy_order():
    """Sec. 5.3: Gen-All-All < Nest-All-All <= Nest-2-All <= Nest-2-2 in
    accuracy, seen in the CG iteration counts on a 3D problem."""
    p = P.poisson_fd((15, 15, 15), P.blocky_log_field(1, 3))
    A = p.csr()
    b = P.random_rhs(0, p.n)
    its = {}
    for scheme, leaf in ((O.GEN_ALL_ALL, 4), (O.NEST_ALL_ALL, 4), (O.NEST_2_ALL, 4), (O.NEST_2_2, 4)):
        F = O.factorize(A, p.coords, p.grid, 1, O.Options(q=1, leaf=leaf, scheme=scheme))
        its[scheme] = O.pcg(A, b, lambda r: O.apply_inverse(F, r), tol=1e-10)[1]
    assert its[O.GEN_ALL_ALL] >= its[O.NEST_ALL_ALL] >= its[O.NEST_2_ALL] >= its[O.NEST_2_2], its


# ---------------------------------------------------------------------------
# Standard low-rank equivalent (Sec. 7.4, Eq. 7.5; Table 7.1)
# ---------------------------------------------------------------------------

def test_fixed_rank_qr_matches_lapack_geqp3():
    rng = np.random.default_rng(4)
    N = rng.standard_normal((40, 25)) @ np.diag(np.logspace(0, -6, 25)) @ rng.standard_normal((25, 30))
    Q, R, piv = sla.qr(N, pivoting=True, mode="economic")
    for r in (1, 5, 12):
        V, tau, rr, dR = O.qrcp_fixed_rank(N, r)
        assert rr == r and V.shape[1] == r
        assert np.allclose(np.abs(dR), np.abs(np.diag(R))[:r], rtol=1e-10)
        Q1 = O.apply_q(V, tau, np.eye(40))[:, :r]
        assert np.allclose(Q1 @ Q1.T, Q[:, :r] @ Q[:, :r].T, atol=1e-10)
    # fewer columns than r: Q_1 still has r orthonormal columns
    V, tau, rr, dR = O.qrcp_fixed_rank(N[:, :3], 6)
    Q1 = O.apply_q(V, tau, np.eye(40))[:, :6]
    assert np.allclose(Q1.T @ Q1, np.eye(6), atol=1e-14)
    assert np.linalg.norm(N[:, :3] - Q1 @ (Q1.T @ N[:, :3])) <= 1e-12 * np.linalg.norm(N[:, :3])


def test_low_rank_equivalent_has_the_same_sizes_and_stays_spd():
    p = _fourier((40, 36), seed=5)
    A, F = _fact(p, q=2, leaf=8)
    A, Fl = _fact(p, q=2, leaf=8, compression=O.LOW_RANK, ranks=F.info["ranks"])
    assert Fl.info["sizes"] == F.info["sizes"] and Fl.info["top_size"] == F.info["top_size"]
    assert O.factor_entries(Fl) == O.factor_entries(F)
    Pf = _physical_polys(p.coords, 2)
    assert _rel(O.multiply(Fl, Pf), A @ Pf) > 1e-9       # no longer exact on polynomials (1e-15 above)
    v = P.random_rhs(3, p.n)
    assert _rel(O.multiply(Fl, O.apply_inverse(Fl, v)), v) <= 1e-10
    Al = O.multiply(Fl, np.eye(p.n))
    assert np.linalg.eigvalsh(0.5 * (Al + Al.T)).min() > 0


def _laplace_eigvec(grid, ks):
    """Unit eigenvector prod_a sin(k_a pi x) of the h^2-scaled Dirichlet
    5/7-point Laplacian at x_i = (i + 1) h, and its eigenvalue
    sum_a 4 sin^2(k_a pi h / 2)."""
    h = [1.0 / (N + 1) for N in grid]
    axes = [np.sin(k * np.pi * (np.arange(N) + 1) * hh) for k, N, hh in zip(ks, grid, h)]
    lam = sum(4 * np.sin(k * np.pi * hh / 2) ** 2 for k, hh in zip(ks, h))
    v = axes[0]
    for a in axes[1:]:
        v = np.multiply.outer(a, v)
    v = v.ravel()
    return v / np.linalg.norm(v), lam


def test_table71_extreme_eigenvector_errors():
    """Table 7.1 (Nest-All-All, q = 2, constant-coefficient 3D Poisson):
    E_1 = |(A - A_l) v_1| / lambda_1 is small and about the same for the
    polynomial compression and its low-rank equivalent, while E_n on the
    smoothest eigenvector is orders of magnitude larger for the low-rank
    equivalent and grows with n (grids 13^3 and 15^3, leaf 3)."""
    En_lr = []
    for N in (13, 15):
        p = P.poisson_fd((N, N, N))
        A = p.csr()
        F = O.factorize(A, p.coords, p.grid, 1, O.Options(q=2, leaf=3))
        Fl = O.factorize(A, p.coords, p.grid, 1, O.Options(q=2, leaf=3, compression=O.LOW_RANK,
                                                             ranks=F.info["ranks"]))
        v1, l1 = _laplace_eigvec(p.grid, (N, N, N))
        vn, ln = _laplace_eigvec(p.grid, (1, 1, 1))
        assert np.linalg.norm(A @ vn - ln * vn) <= 1e-12 and np.linalg.norm(A @ v1 - l1 * v1) <= 1e-12 * l1
        E = lambda FF, v, lam: np.linalg.norm(A @ v - O.multiply(FF, v)) / lam
        e1, e1l, en, enl = E(F, v1, l1), E(Fl, v1, l1), E(F, vn, ln), E(Fl, vn, ln)
        print(f"N={N}: E1 {e1:.2e} / {e1l:.2e}, En {en:.2e} / {enl:.2e}")
        assert 0.5 < e1 / e1l < 2.0
        assert enl > 30 * en
        En_lr.append(enl)
    assert En_lr[1] > En_lr[0]


# ---------------------------------------------------------------------------
# User-supplied near-kernel basis (Secs. 1, 3.1)
# ---------------------------------------------------------------------------

def test_user_basis_rigid_body_modes():
    """Pi = the six rigid-body modes of the elasticity problem: A_l keeps
    A's action on them (Prop. 6.1 for this Pi) with smaller ranks than the
    piecewise-linear basis."""
    e = P.elasticity_q1(10, seed=3, n_incl=4)
    A = e.csr()
    R = P.rigid_body_modes(e)
    Fu = O.factorize(A, None, e.grid, 3, O.Options(leaf=3, basis=R))
    Fq = O.factorize(A, e.coords, e.grid, 3, O.Options(q=1, leaf=3))
    assert sum(1 for g in Fu.info["gap"] if g[3] < g[2]) > 0
    AR = A @ R
    assert _rel(O.multiply(Fu, R), AR) <= 1e-10
    assert sum(g[3] for g in Fu.info["gap"]) < sum(g[3] for g in Fq.info["gap"])


def test_constant_basis_needs_no_coordinates():
    p = _fourier((24, 20))
    A = p.csr()
    Fa = O.factorize(A, p.coords, p.grid, 1, O.Options(q=0, leaf=4))
    Fb = O.factorize(A, None, p.grid, 1, O.Options(leaf=4, basis=np.ones((p.n, 1))))
    v = P.random_rhs(1, p.n)
    assert np.array_equal(O.apply_inverse(Fa, v), O.apply_inverse(Fb, v))


def test_factor_size_per_unknown_stays_flat():
    """Prop. 5.1 (Sec. 5.4): with compression every node's active size is
    bounded independently of n, so the top node keeps one size and the
    stored factor entries per unknown level off as the grid grows (2D,
    q = 1, leaf 8: 32^2, 64^2, 128^2): each doubling of the side adds less
    than the one before, while without compression the additions grow (the
    n log n of nested dissection) and the top grows like the grid side."""
    per_n, per_n_exact, tops, tops_exact = [], [], [], []
    for N in (32, 64, 128):
        p = _fourier((N, N))
        _, F = _fact(p, q=1, leaf=8)
        _, Fe = _fact(p, q=1, leaf=8, compress=False)
        per_n.append(O.factor_entries(F) / p.n)
        per_n_exact.append(O.factor_entries(Fe) / p.n)
        tops.append(F.info["top_size"])
        tops_exact.append(Fe.info["top_size"])
    assert tops[0] == tops[1] == tops[2]
    assert tops_exact[2] > 1.9 * tops_exact[1] > 3.6 * tops_exact[0]
    d, de = np.diff(per_n), np.diff(per_n_exact)
    assert d[1] < 0.8 * d[0]
    assert de[1] >= de[0]
    assert per_n[2] < per_n_exact[2]


def test_low_rank_with_level_blocks_is_order_independent_and_matches_dense_schur():
    """The low-rank equivalent whose compressions take their off-diagonal
    blocks from the level's matrix before any of its compressions: (1) the
    compressions of a level no longer depend on their order (ascending,
    descending, shuffled give one operator), unlike the sequential variant,
    whose result changes with the order; (2) on level 1, each compressed
    separator's kept subspace is that of a pivoted QR (LAPACK) of
    chol(S_BB)^{-1} [S_BX1 | S_BX2 | ...], with S the dense Schur complement
    of the level-1 interiors computed here from A."""
    p = _fourier((50, 46), seed=2)
    A = p.csr()
    _, F = _fact(p, q=0, leaf=16)
    kw = dict(q=0, leaf=16, compression=O.LOW_RANK, ranks=F.info["ranks"])
    v = np.stack([P.random_rhs(6, p.n, j) for j in range(2)], axis=1)
    outs = {o: O.apply_inverse(_fact(p, order=o, low_rank_blocks="level", **kw)[1], v)
            for o in ("ascending", "descending", "shuffled")}
    assert _rel(outs["descending"], outs["ascending"]) <= 1e-12
    assert _rel(outs["shuffled"], outs["ascending"]) <= 1e-12
    seq = {o: O.apply_inverse(_fact(p, order=o, **kw)[1], v) for o in ("ascending", "descending")}
    assert _rel(seq["descending"], seq["ascending"]) > 1e-9
    # (2) level 1 against a dense Schur complement
    _, Fl = _fact(p, low_rank_blocks="level", **kw)
    lv = O.partition_hierarchy(p.grid, 16)[0]
    cell = lv.cell_of_node
    interior = lv.type[cell] == 0
    Ad = A.toarray()
    I, S = np.nonzero(interior)[0], np.nonzero(~interior)[0]
    Sch = Ad[np.ix_(S, S)] - Ad[np.ix_(S, I)] @ np.linalg.solve(Ad[np.ix_(I, I)], Ad[np.ix_(I, S)])
    pos = {d: k for k, d in enumerate(S)}
    checked = 0
    for op in Fl.levels[0]:
        if op[0] != "comp":
            continue
        _, vB, Lo, V, tau, r = op
        B = cell[vB[0]]
        rows = [pos[d] for d in vB]
        nbrs = sorted({cell[S[j]] for j in range(len(S)) if cell[S[j]] != B
                       and np.abs(Sch[np.ix_(rows, [j])]).max() > 0})
        cols = [pos[d] for X in nbrs for d in np.nonzero(cell == X)[0]]
        Lb = np.linalg.cholesky(Sch[np.ix_(rows, rows)])
        N = sla.solve_triangular(Lb, Sch[np.ix_(rows, cols)], lower=True)
        Q, R, piv = sla.qr(N, pivoting=True)
        Pd = Q[:, :r] @ Q[:, :r].T
        Qo = O.apply_q(V, tau, np.eye(len(vB)))[:, :r]
        assert np.abs(Qo @ Qo.T - Pd).max() <= 1e-10
        checked += 1
    assert checked >= 8
