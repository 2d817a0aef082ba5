"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the statement it checks.  None of them re-derives the
oracle's own formulas: they use closed forms (partition counts), the exact
special case (no compression = block Cholesky = A), library routines
(LAPACK's pivoted QR, dense solves), and the invariants the paper proves
(Lemma 3.1: SPD; Prop. 6.1: A_l Pi_D = A Pi_D; rigid-body modes, Sec. 7.2).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import sgf_oracle as O
from sgf_inputs import problems as P


def _prob(kind, grid, seed=0):
    if kind == "const":
        return P.poisson_fd(grid)
    if kind == "fourier":
        return P.poisson_fd(grid, P.gaussian_field_fourier(seed, len(grid)))
    if kind == "blocky":
        return P.poisson_fd(grid, P.blocky_log_field(seed, len(grid)))
    raise ValueError(kind)


def _dense_Al(F, n):
    return O.multiply(F, np.eye(n))


# ---------------------------------------------------------------------------
# Partition hierarchy (Sec. 5.1)
# ---------------------------------------------------------------------------

def test_partition_counts_64x64_leaf8():
    """64^2 grid, b = 8: 8 blocks per axis at level 1 (seven of 7 points, the
    last of 8), 7 internal slabs; levels at d = 8, 16, 32, then V."""
    levels = O.partition_hierarchy((64, 64), 8)
    assert [lv.d for lv in levels] == [8, 16, 32, 64]
    assert levels[-1].is_root and levels[-1].ncells == 1
    lv = levels[0]
    counts = np.bincount(lv.cell_of_node, minlength=lv.ncells)
    types = lv.type
    assert (types == 0).sum() == 64 and (types == 1).sum() == 112 and (types == 2).sum() == 49
    sizes = sorted(counts[types == 0])
    assert sizes.count(49) == 49 and sizes.count(56) == 14 and sizes.count(64) == 1
    assert set(counts[types == 1]) == {7, 8}
    assert set(counts[types == 2]) == {1}


def test_partition_counts_3d_and_interior_size_formula():
    """Sec. 7: with b = 3 the level-k interior holds (3 2^(k-1) - 1)^3 points
    (away from the high boundary)."""
    levels = O.partition_hierarchy((47, 47, 47), 3)
    for k, lv in enumerate(levels[:-1], start=1):
        counts = np.bincount(lv.cell_of_node, minlength=lv.ncells)
        side = 3 * 2 ** (k - 1) - 1
        assert side ** 3 in set(counts[lv.type == 0])
        # 2-cells hold (d-1)^2 points, 1-cells d-1, 0-cells one
        assert (side ** 2) in set(counts[lv.type == 1])
        assert side in set(counts[lv.type == 2])
        assert set(counts[lv.type == 3]) == {1}


@pytest.mark.parametrize("grid,leaf", [((64, 64), 8), ((20, 17), 4), ((13, 9, 11), 3), ((47, 48, 48), 6)])
def test_coarsening_unique_father_and_nonadjacent_interiors(grid, leaf):
    """Def. 2.2: every set of P_t lies in exactly one set of P_{t+1};
    interiors do not touch each other under the 3^dim vertex stencil."""
    levels = O.partition_hierarchy(grid, leaf)
    dim = len(grid)
    for a, b in zip(levels[:-1], levels[1:]):
        fa = O.father_map(a, b)
        # all nodes of a cell have the same father
        assert np.array_equal(fa[a.cell_of_node], b.cell_of_node)
    shape = tuple(reversed(grid))
    for lv in levels[:-1]:
        cid = lv.cell_of_node.reshape(shape)
        interior = (lv.type[cid] == 0)
        for off in np.ndindex(*(3,) * dim):
            d = [o - 1 for o in off]
            if not any(d):
                continue
            src = tuple(slice(max(0, -x), s - max(0, x)) for x, s in zip(d, shape))
            dst = tuple(slice(max(0, x), s - max(0, -x)) for x, s in zip(d, shape))
            both = interior[src] & interior[dst]
            assert np.all(cid[src][both] == cid[dst][both])


# ---------------------------------------------------------------------------
# Pivoted QR (Eq. 3.3, LAPACK geqp3 in the paper)
# ---------------------------------------------------------------------------

def test_qrcp_matches_lapack_geqp3_on_generic_matrix():
    rng = np.random.default_rng(0)
    N = rng.standard_normal((30, 12)) @ np.diag(np.logspace(0, -3, 12))
    V, tau, r, dR = O.qrcp(N, 1e-14)
    Q, R, piv = sla.qr(N, pivoting=True, mode="economic")
    assert r == 12
    assert np.allclose(np.abs(dR), np.abs(np.diag(R)), rtol=1e-12)
    Qf = O.apply_q(V, tau, np.eye(30))
    assert np.allclose(Qf.T @ Qf, np.eye(30), atol=1e-14)
    # same pivots => same Q_1 columns up to sign
    assert np.allclose(np.abs(Qf[:, :12]), np.abs(Q), atol=1e-12)


def test_qrcp_rank_and_orthogonal_complement():
    rng = np.random.default_rng(1)
    for rank in (1, 3, 7):
        N = rng.standard_normal((25, rank)) @ rng.standard_normal((rank, 15))
        V, tau, r, dR = O.qrcp(N, 1e-12)
        assert r == rank
        QtN = O.apply_qt(V, tau, N)
        assert np.linalg.norm(QtN[r:]) <= 1e-13 * np.linalg.norm(N)
    # points on a line: [1, x, y] has rank 2
    x = np.linspace(-1, 1, 9)
    N = np.stack([np.ones(9), x, np.full(9, 0.3)], axis=1)
    assert O.qrcp(N, 1e-12)[2] == 2


def test_qrcp_zero_and_tie_rule():
    V, tau, r, dR = O.qrcp(np.zeros((4, 3)), 1e-12)
    assert r == 0
    # equal-norm columns: lowest index wins
    N = np.array([[1.0, 0.0], [0.0, 1.0]])
    V, tau, r, dR = O.qrcp(N, 1e-12)
    assert r == 2 and np.isclose(abs(dR[0]), 1.0)
    assert np.allclose(O.apply_qt(V, tau, N[:, :1])[1:], 0.0)


# ---------------------------------------------------------------------------
# Exact special case: no compression = nested-dissection block Cholesky
# ---------------------------------------------------------------------------

CASES = [("const", (16, 16), 4, 1), ("fourier", (20, 17), 4, 2), ("blocky", (9, 8, 7), 2, 1),
         ("const", (12, 12, 12), 3, 0)]


@pytest.mark.parametrize("kind,grid,leaf,q", CASES)
def test_exact_mode_equals_dense_cholesky(kind, grid, leaf, q):
    p = _prob(kind, grid)
    A = p.csr()
    F = O.factorize(A, p.coords, p.grid, 1, O.Options(q=q, leaf=leaf, compress=False))
    Ad = A.toarray()
    b = P.random_rhs(0, p.n)
    x = O.apply_inverse(F, b)
    assert np.linalg.norm(x - np.linalg.solve(Ad, b)) <= 1e-12 * np.linalg.norm(x)
    Al = _dense_Al(F, p.n)
    assert np.abs(Al - Ad).max() <= 1e-13 * np.abs(Ad).max()
    xs, it, rel = O.pcg(A, b, lambda r: O.apply_inverse(F, r), tol=1e-10)
    assert it == 1


def test_exact_mode_elasticity():
    e = P.elasticity_q1(6, seed=2, n_incl=2)
    A = e.csr()
    F = O.factorize(A, e.coords, e.grid, 3, O.Options(q=1, leaf=2, compress=False))
    b = P.random_rhs(0, e.n)
    x = O.apply_inverse(F, b)
    assert np.linalg.norm(x - np.linalg.solve(A.toarray(), b)) <= 1e-11 * np.linalg.norm(x)


# ---------------------------------------------------------------------------
# Compression: Lemma 3.1 (SPD) and Prop. 6.1 (polynomial preservation)
# ---------------------------------------------------------------------------

PRES = [("const", (32, 32), 4, 1), ("fourier", (32, 32), 4, 2), ("fourier", (24, 20), 4, 0),
        ("blocky", (12, 12, 12), 3, 1), ("const", (14, 14, 14), 3, 2)]


@pytest.mark.parametrize("kind,grid,leaf,q", PRES)
def test_compression_preserves_piecewise_polynomials(kind, grid, leaf, q):
    """Prop. 6.1: E_i Pi_B = 0 for B in P_k, i <= k; with the exact top this
    gives A_l Pi_D = A Pi_D for every D in P_{l-1}, and A_l Pi = A Pi."""
    p = _prob(kind, grid)
    A = p.csr()
    F = O.factorize(A, p.coords, p.grid, 1, O.Options(q=q, leaf=leaf))
    ncomp = sum(1 for g in F.info["gap"] if g[3] < g[2])
    assert ncomp > 0, "test case must actually compress"
    Pi = O.poly_basis(p.coords, q, 1)
    AP = A @ Pi
    assert np.linalg.norm(O.multiply(F, Pi) - AP) <= 1e-10 * np.linalg.norm(AP)
    levels = O.partition_hierarchy(p.grid, leaf)
    last = levels[F.info["nlevels"] - 2]
    for D in np.unique(last.cell_of_node):
        PiD = Pi * (last.cell_of_node == D)[:, None]
        APD = A @ PiD
        assert np.linalg.norm(O.multiply(F, PiD) - APD) <= 1e-10 * np.linalg.norm(APD)


def test_compression_changes_operator_but_stays_spd():
    """Lemma 3.1: the compressed operator is SPD; and compression is not a
    no-op (A_l differs from A away from the polynomial space)."""
    p = _prob("fourier", (24, 24))
    A = p.csr()
    F = O.factorize(A, p.coords, p.grid, 1, O.Options(q=1, leaf=4))
    Al = _dense_Al(F, p.n)
    Ad = A.toarray()
    assert np.abs(Al - Al.T).max() <= 1e-12 * np.abs(Al).max()
    assert np.linalg.eigvalsh(Al).min() > 0
    assert np.linalg.norm(Al - Ad) > 1e-6 * np.linalg.norm(Ad)
    # A_l^{-1} from the apply is the inverse of A_l from the product
    v = P.random_rhs(5, p.n)
    assert np.linalg.norm(Al @ O.apply_inverse(F, v) - v) <= 1e-11 * np.linalg.norm(v)


def test_single_node_compression_lemma():
    """Lemma 3.1 on a dense SPD matrix: compressing one node B keeps
    M Pi_C = M~ Pi_C for every node C and M~ SPD.  M~ is assembled from the
    factor of a one-level run (elimination off: no interiors)."""
    p = _prob("fourier", (15, 15))
    A = p.csr()
    F = O.factorize(A, p.coords, p.grid, 1, O.Options(q=1, leaf=4))
    lv = O.partition_hierarchy(p.grid, 4)[0]
    Pi = O.poly_basis(p.coords, 1, 1)
    Al = _dense_Al(F, p.n)
    for C in range(lv.ncells):
        PiC = Pi * (lv.cell_of_node == C)[:, None]
        assert np.linalg.norm(Al @ PiC - A @ PiC) <= 1e-10 * np.linalg.norm(A @ PiC)


def test_rigid_body_modes_exact_for_elasticity():
    """Sec. 7.2: with the block-diagonal Pi (Eq. 7.4) and q >= 1 the factor
    reproduces A on the six rigid-body modes."""
    e = P.elasticity_q1(10, seed=3, n_incl=4)
    A = e.csr()
    F = O.factorize(A, e.coords, e.grid, 3, O.Options(q=1, leaf=3))
    assert sum(1 for g in F.info["gap"] if g[3] < g[2]) > 0
    R = P.rigid_body_modes(e)
    AR = A @ R
    assert np.linalg.norm(O.multiply(F, R) - AR) <= 1e-10 * np.linalg.norm(AR)
    Z = O.apply_inverse(F, AR)
    assert np.linalg.norm(Z - R) <= 1e-8 * np.linalg.norm(R)


def test_compression_order_within_level_is_irrelevant():
    """The compressions of one level commute (each acts on its own rows and,
    for span Q1 containing range N, sees the same filtered columns)."""
    p = _prob("blocky", (10, 10, 10))
    A = p.csr()
    v = P.random_rhs(1, p.n)
    outs = []
    for order in ("ascending", "descending", "shuffled"):
        F = O.factorize(A, p.coords, p.grid, 1, O.Options(q=1, leaf=3, order=order, seed=4))
        outs.append((O.multiply(F, v), O.apply_inverse(F, v),
                     sorted(F.info["sizes"][0].items())))
    for o in outs[1:]:
        assert o[2] == outs[0][2]
        assert np.linalg.norm(o[0] - outs[0][0]) <= 1e-12 * np.linalg.norm(outs[0][0])
        assert np.linalg.norm(o[1] - outs[0][1]) <= 1e-10 * np.linalg.norm(outs[0][1])


@pytest.mark.parametrize("kind,grid,leaf,q", [("const", (32, 32), 4, 1), ("blocky", (10, 10, 10), 3, 1)])
def test_pcg_solution_agrees_with_dense_solve(kind, grid, leaf, q):
    p = _prob(kind, grid)
    A = p.csr()
    F = O.factorize(A, p.coords, p.grid, 1, O.Options(q=q, leaf=leaf))
    b = P.random_rhs(0, p.n)
    x, it, rel = O.pcg(A, b, lambda r: O.apply_inverse(F, r), tol=1e-12)
    xd = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    assert 1 < it < 60


def test_paper_stop_rule_keeps_preservation():
    p = _prob("fourier", (40, 40))
    A = p.csr()
    F = O.factorize(A, p.coords, p.grid, 1, O.Options(q=1, leaf=4, stop_rule=O.STOP_PAPER))
    Fr = O.factorize(A, p.coords, p.grid, 1, O.Options(q=1, leaf=4))
    assert F.info["nlevels"] <= Fr.info["nlevels"]
    Pi = O.poly_basis(p.coords, 1, 1)
    assert np.linalg.norm(O.multiply(F, Pi) - A @ Pi) <= 1e-10 * np.linalg.norm(A @ Pi)


def test_pcg_zero_rhs_and_iteration_growth_is_slow():
    p = _prob("const", (32, 32))
    A = p.csr()
    F = O.factorize(A, p.coords, p.grid, 1, O.Options(q=1, leaf=4))
    x, it, rel = O.pcg(A, np.zeros(p.n), lambda r: O.apply_inverse(F, r))
    assert it == 0 and not x.any()
    its = []
    for N in (16, 32, 64):
        p = _prob("const", (N, N))
        A = p.csr()
        F = O.factorize(A, p.coords, p.grid, 1, O.Options(q=1, leaf=4))
        its.append(O.pcg(A, P.random_rhs(0, p.n), lambda r: O.apply_inverse(F, r), tol=1e-10)[1])
    # Sec. 7: iteration counts nearly constant in n
    assert its[-1] <= its[0] + 6
