"""GPU parity of the HIP SGF library against the CPU oracle (FP64).

Through the C ABI (ctypes binding), on seeded synthetic problems that span
several clusters per level, ragged last blocks, 2D / 3D, q = 0, 1, 2, and
elasticity.  Bars: structure (cells, sizes, ranks per level) bit-exact;
A_l^{-1} v and A_l v within max(1e-10, 100 x the oracle's own rounding
sensitivity) relative of the oracle (the sensitivity is measured by running
the oracle with the compressions of each level in reverse order and on A
perturbed by one ulp), or, where the rank cut has no spectral gap, within
10 eps / |R_rr| (kept QR directions are determined only to eps / sigma);
exact mode within 1e-12 of a dense solve; A_l Pi = A Pi within 1e-10; CG
solutions within 1e-8 relative and iteration counts within +-1.
"""
import numpy as np
import pytest

from oracle import sgf_oracle as O
from sgf_inputs import problems as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

sgf = pytest.importorskip("paper_1907_03406_amd.sgf")


def _prob(kind, grid, seed=0):
    if kind == "const":
        return P.poisson_fd(grid)
    if kind == "fourier":
        return P.poisson_fd(grid, P.gaussian_field_fourier(seed, len(grid)))
    if kind == "blocky":
        return P.poisson_fd(grid, P.blocky_log_field(seed, len(grid)))
    if kind == "elast":
        return P.elasticity_q1(grid, seed=seed, n_incl=3)
    raise ValueError(kind)


def _gpu(p, **kw):
    s = sgf.Solver.from_problem(p, **kw)
    s.factorize(torch.from_numpy(p.data).cuda())
    torch.cuda.synchronize()
    return s


def _apply(s, v, product=False):
    vin = torch.from_numpy(np.ascontiguousarray(v.T if v.ndim == 2 else v)).cuda()
    out = torch.empty_like(vin)
    (s.multiply if product else s.apply)(vin.T if v.ndim == 2 else vin, out.T if v.ndim == 2 else out)
    torch.cuda.synchronize()
    r = out.cpu().numpy()
    return r.T if v.ndim == 2 else r


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _maxrel(a, b):
    """Largest entry-wise difference of each column relative to the
    column's largest entry, maximised over the columns."""
    a2, b2 = np.atleast_2d(a.T).T, np.atleast_2d(b.T).T
    return float(np.max(np.abs(a2 - b2).max(axis=0) / np.maximum(np.abs(b2).max(axis=0), 1e-300)))


EXACT = [("const", (16, 16), 4, 1), ("fourier", (37, 29), 4, 2), ("blocky", (9, 8, 7), 2, 1),
         ("const", (2, 2), 8, 1), ("blocky", (17, 16, 15), 8, 1)]

# tiled_min_rows: -1 = built-in choice per level; 0 = every level (and the
# top) through the tiled multi-workgroup elimination and its apply kernels
TILED = (-1, 0)


@pytest.mark.parametrize("kind,grid,leaf,q", EXACT)
@pytest.mark.parametrize("tiled", TILED)
def test_exact_mode_is_the_inverse(kind, grid, leaf, q, tiled):
    p = _prob(kind, grid)
    s = _gpu(p, q=q, leaf=leaf, compress=False, tiled_min_rows=tiled)
    A = p.csr()
    b = P.random_rhs(0, p.n)
    x = _apply(s, b)
    xd = np.linalg.solve(A.toarray(), b)
    assert _rel(x, xd) <= 1e-12
    y = _apply(s, b, product=True)
    assert _rel(y, A @ b) <= 1e-13
    xg = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    it, rel = s.pcg(torch.from_numpy(b).cuda(), xg, rtol=1e-10)
    assert it[0] == 1


PAR = [("const", (64, 64), 8, 1), ("fourier", (50, 41), 4, 2), ("fourier", (40, 40), 4, 0),
       ("blocky", (14, 13, 12), 3, 1), ("const", (16, 16, 16), 4, 2), ("elast", 8, 3, 1)]


def _oracle(p, q, leaf):
    return O.factorize(p.csr(), p.coords, p.grid, p.dpn, O.Options(q=q, leaf=leaf))


@pytest.mark.parametrize("kind,grid,leaf,q", PAR)
def test_factor_structure_and_operators_match_oracle(kind, grid, leaf, q):
    p = _prob(kind, grid)
    F = _oracle(p, q, leaf)
    solvers = {t: _gpu(p, q=q, leaf=leaf, tiled_min_rows=t) for t in TILED}
    for s in solvers.values():
        info = s.info()
        assert info["levels"] == F.info["nlevels"]
        assert info["top_size"] == F.info["top_size"]
        for t in range(1, F.info["nlevels"]):
            g = s.level(t)
            post = F.info["sizes"][t - 1]
            seps = g["type"] > 0
            assert sorted(post) == g["cell"][seps].tolist()
            assert [post[c] for c in g["cell"][seps]] == g["rank"][seps].tolist(), f"ranks differ at level {t}"
        assert sum(1 for x in F.info["gap"] if x[3] < x[2]) == info["compressed"]
    V = np.stack([P.random_rhs(7, p.n, j) for j in range(3)], axis=1)
    za, zm = O.apply_inverse(F, V), O.multiply(F, V)
    # Element by element, within 1e-10 of each column's largest entry.  The
    # operator is defined only as well as the rank-truncated QRs define their
    # kept subspaces.  (1) Where the cut at the rank threshold has no spectral
    # gap (smallest kept pivot ratio < 10 x the largest dropped one), a kept
    # direction with |R_rr| ~ rho |R_00| is determined only to about
    # eps / rho by any implementation: parity-unpinned at 1e-10, held to that
    # bound instead.  (2) Otherwise the bar is 1e-10, unless the oracle itself
    # does not reproduce its operator to 1e-11 when A is perturbed by one ulp
    # (near-tied pivots of symmetric constant-coefficient problems): then 10 x
    # that measured sensitivity, printed.
    kept = min(x[4] for x in F.info["gap"] if x[3] > 0)
    dropped = max(x[5] for x in F.info["gap"])
    gapless = kept < 10 * dropped
    sens = 0.0
    for seed in range(2):
        Ap = p.csr().copy()
        Ap.data = Ap.data * (1 + 2e-16 * np.random.default_rng(seed).standard_normal(Ap.nnz))
        Ap = ((Ap + Ap.T) * 0.5).tocsr()
        Fp = O.factorize(Ap, p.coords, p.grid, p.dpn, O.Options(q=q, leaf=leaf))
        sens = max(sens, _maxrel(O.apply_inverse(Fp, V), za), _maxrel(O.multiply(Fp, V), zm))
    if gapless:
        bar, why = max(1e-10, 10 * np.finfo(float).eps / kept), "GAPLESS: parity unpinned at 1e-10"
    elif sens > 1e-11:
        bar, why = 10 * sens, "the oracle's own one-ulp sensitivity exceeds 1e-11"
    else:
        bar, why = 1e-10, ""
    for tiled, s in solvers.items():
        ea, em = _maxrel(_apply(s, V), za), _maxrel(_apply(s, V, product=True), zm)
        print(f"{kind} {grid} tiled_min_rows {tiled}: apply {ea:.1e}, product {em:.1e}, kept>={kept:.1e} "
              f"dropped<={dropped:.1e}, oracle one-ulp sensitivity {sens:.1e}, bar {bar:.1e} {why}")
        assert ea <= bar and em <= bar


@pytest.mark.parametrize("kind,grid,leaf,q", PAR[:5])
def test_preservation_on_gpu(kind, grid, leaf, q):
    """Prop. 6.1 through the device product form: A_l Pi = A Pi."""
    p = _prob(kind, grid)
    s = _gpu(p, q=q, leaf=leaf)
    Pi = O.poly_basis(p.coords, q, p.dpn)
    AP = p.csr() @ Pi
    assert _rel(_apply(s, Pi, product=True), AP) <= 1e-10


@pytest.mark.parametrize("tiled", TILED)
def test_rigid_body_modes_on_gpu(tiled):
    e = _prob("elast", 10, seed=3)
    s = _gpu(e, q=1, leaf=3, tiled_min_rows=tiled)
    assert s.info()["compressed"] > 0
    R = P.rigid_body_modes(e)
    AR = e.csr() @ R
    assert _rel(_apply(s, AR), R) <= 1e-8
    assert _rel(_apply(s, R, product=True), AR) <= 1e-10


@pytest.mark.parametrize("kind,grid,leaf,q,tol,tiled", [("const", (64, 64), 8, 1, 1e-10, -1),
                                                        ("fourier", (96, 80), 8, 2, 1e-8, -1),
                                                        ("blocky", (20, 20, 20), 4, 1, 1e-8, -1),
                                                        ("blocky", (20, 20, 20), 4, 1, 1e-8, 0),
                                                        ("elast", 10, 3, 1, 1e-8, 0)])
def test_pcg_matches_oracle(kind, grid, leaf, q, tol, tiled):
    p = _prob(kind, grid)
    A = p.csr()
    F = _oracle(p, q, leaf)
    b = P.random_rhs(0, p.n)
    xo, ito, _ = O.pcg(A, b, lambda r: O.apply_inverse(F, r), tol=tol)
    s = _gpu(p, q=q, leaf=leaf, tiled_min_rows=tiled)
    xg = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    it, rel = s.pcg(torch.from_numpy(b).cuda(), xg, rtol=tol)
    x = xg.cpu().numpy()
    assert abs(int(it[0]) - ito) <= 1
    assert rel[0] < tol
    assert _rel(x, xo) <= 1e-8 or _rel(x, np.linalg.solve(A.toarray(), b)) <= 1e-8
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) < 10 * tol


@pytest.mark.parametrize("tiled", TILED)
def test_multi_rhs_pcg_columns_are_independent(tiled):
    p = _prob("fourier", (48, 48))
    s = _gpu(p, q=1, leaf=4, tiled_min_rows=tiled)
    B = np.stack([P.random_rhs(3, p.n, j) for j in range(4)], axis=1)
    B[:, 2] = 0.0
    Bt = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    Xt = torch.zeros_like(Bt)
    it, rel = s.pcg(Bt.T, Xt.T, rtol=1e-9)
    assert it[2] == 0
    for j in (0, 1, 3):
        xj = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        itj, _ = s.pcg(Bt[j].contiguous(), xj, rtol=1e-9)
        assert it[j] == itj[0]
        assert _rel(Xt[j].cpu().numpy(), xj.cpu().numpy()) <= 1e-12


def test_refactorize_with_new_values_and_spmv():
    p = _prob("fourier", (33, 31), seed=1)
    p2 = _prob("fourier", (33, 31), seed=2)
    s = sgf.Solver.from_problem(p, q=1, leaf=4)
    s.factorize(torch.from_numpy(p.data).cuda())
    s.factorize(torch.from_numpy(p2.data).cuda())
    F2 = _oracle(p2, 1, 4)
    v = P.random_rhs(9, p.n)
    assert _rel(_apply(s, v), O.apply_inverse(F2, v)) <= 1e-10
    vt = torch.from_numpy(v).cuda()
    y = torch.empty_like(vt)
    s.spmv(vt, y)
    assert _rel(y.cpu().numpy(), p2.csr() @ v) <= 1e-15


@pytest.mark.parametrize("tiled", TILED)
def test_not_spd_reports_cluster(tiled):
    p = _prob("const", (16, 16))
    bad = p.data.copy()
    A = p.csr()
    # make one interior diagonal entry negative
    i = 0
    bad[A.indptr[i]:A.indptr[i + 1]][A.indices[A.indptr[i]:A.indptr[i + 1]] == i] = -4.0
    s = sgf.Solver.from_problem(p, q=1, leaf=4, tiled_min_rows=tiled)
    with pytest.raises(sgf.SgfError) as ei:
        s.factorize(torch.from_numpy(bad).cuda())
    assert ei.value.code == sgf.SGF_ENOTSPD
    assert s.info()["failed_level"] == 1


@pytest.mark.parametrize("kind,grid,leaf,q,tiled", [("fourier", (128, 128), 16, 2, -1), ("blocky", (24, 24, 24), 8, 1, -1),
                                                    ("elast", 12, 3, 1, -1), ("blocky", (24, 24, 24), 8, 1, 0)])
def test_fp32_form_reaches_fp64_accuracy(kind, grid, leaf, q, tiled):
    """Precision form: FP32 factor and apply inside FP64 CG.  CG must still
    reach a true FP64 relative residual below 2e-8, with a bounded increase
    of the iteration count; the distance to the FP64 solution is reported."""
    p = _prob(kind, grid)
    A = p.csr()
    b = P.random_rhs(1, p.n)
    bt = torch.from_numpy(b).cuda()
    out = {}
    for prec in (sgf.FP64, sgf.FP32):
        s = _gpu(p, q=q, leaf=leaf, precision=prec, tiled_min_rows=tiled)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        it, rel = s.pcg(bt, x, rtol=1e-8)
        out[prec] = (int(it[0]), x.cpu().numpy())
    it64, x64 = out[sgf.FP64]
    it32, x32 = out[sgf.FP32]
    true32 = np.linalg.norm(b - A @ x32) / np.linalg.norm(b)
    print(f"fp32 form: it {it32} (fp64 {it64}), true residual {true32:.2e}, |x32-x64|/|x64| {_rel(x32, x64):.2e}")
    assert true32 < 2e-8
    assert it32 <= 2 * it64 + 5


def test_autotuned_levels_match_oracle():
    """After the autotuner picks each level's path, the factor is the same
    operator; the chosen modes are among the candidates."""
    p = _prob("blocky", (20, 19, 18))
    F = _oracle(p, 1, 4)
    s = sgf.Solver.from_problem(p, q=1, leaf=4)
    vals = torch.from_numpy(p.data).cuda()
    modes = s.autotune(vals, napply=10)
    assert len(modes) == F.info["nlevels"]
    assert set(modes.tolist()) <= {-1, 0, 1, 8, 16, 32}
    assert modes[-1] == -1
    with pytest.raises(sgf.SgfError):
        s.apply(vals[:p.n].clone(), torch.empty(p.n, dtype=torch.float64, device="cuda"))
    s.factorize(vals)
    V = np.stack([P.random_rhs(4, p.n, j) for j in range(2)], axis=1)
    assert _rel(_apply(s, V), O.apply_inverse(F, V)) <= 1e-10


@pytest.mark.parametrize("tiled", TILED)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_rhs_apply_equals_columnwise(tiled, prec):
    """Seven right-hand sides in one apply (workgroups take up to four
    columns, so the batch is split 4 + 3) give the same columns as seven
    single applies."""
    p = _prob("elast", 9, seed=5)
    s = _gpu(p, q=1, leaf=3, tiled_min_rows=tiled, precision=sgf.FP64 if prec == "fp64" else sgf.FP32)
    V = np.stack([P.random_rhs(11, p.n, j) for j in range(7)], axis=1)
    Z = _apply(s, V)
    Zc = np.stack([_apply(s, V[:, j]) for j in range(7)], axis=1)
    print(f"batched vs columnwise ({prec}, tiled {tiled}): {np.abs(Z - Zc).max():.1e}")
    assert _rel(Z, Zc) <= (1e-14 if prec == "fp64" else 1e-6)
    if prec == "fp64":
        F = _oracle(p, 1, 3)
        assert _rel(Z, O.apply_inverse(F, V)) <= 1e-10


@pytest.mark.parametrize("tiled", TILED)
def test_graph_replays_match_direct_launches(tiled):
    """One captured apply graph, replayed several times with direct-launch
    applies, a refactorization (which retires the graph) and host
    synchronisations in between, gives exactly the direct-launch result."""
    p = _prob("fourier", (70, 61), seed=3)
    s = _gpu(p, q=2, leaf=4, tiled_min_rows=tiled, precision=sgf.FP32)
    r = torch.from_numpy(np.stack([P.random_rhs(2, p.n, j) for j in range(3)], axis=0)).cuda()
    zg, zd = torch.empty_like(r), torch.empty_like(r)
    for rep in range(5):
        s.set_apply_graph(False)
        s.apply(r.T, zd.T)
        torch.cuda.synchronize()
        s.set_apply_graph(True)
        zg.fill_(float("nan"))
        s.apply(r.T, zg.T)
        torch.cuda.synchronize()
        assert torch.equal(zg, zd), f"replay {rep}"
        if rep == 2:
            s.factorize(torch.from_numpy(p.data).cuda())
    x = torch.zeros_like(r)
    it, rel = s.pcg(r.T, x.T, rtol=1e-9)
    s.set_apply_graph(False)
    x2 = torch.zeros_like(r)
    it2, rel2 = s.pcg(r.T, x2.T, rtol=1e-9)
    assert it.tolist() == it2.tolist() and torch.equal(x, x2)


@pytest.mark.parametrize("kind,grid,leaf,q", [("blocky", (24, 24, 24), 8, 1), ("fourier", (128, 128), 16, 2)])
def test_bf16_n_form_converges(kind, grid, leaf, q):
    """Precision form with N formed from bfloat16 operands: the kept
    subspaces are only accurate to about 2^-8, so polynomial preservation
    degrades to that level; FP64 CG must still reach the 1e-8 true residual,
    with the iteration increase bounded and reported."""
    p = _prob(kind, grid)
    A = p.csr()
    b = P.random_rhs(2, p.n)
    bt = torch.from_numpy(b).cuda()
    its = {}
    for prec in (sgf.FP32, sgf.FP32_BF16N):
        s = _gpu(p, q=q, leaf=leaf, precision=prec)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        it, rel = s.pcg(bt, x, rtol=1e-8)
        its[prec] = int(it[0])
        true = np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b)
        Pi = O.poly_basis(p.coords, q, p.dpn)
        pres = _rel(_apply(s, Pi, product=True), A @ Pi)
        print(f"{kind} {grid} precision {prec}: it {it[0]}, true residual {true:.1e}, preservation {pres:.1e}, "
              f"compressed {s.info()['compressed']}")
        assert true < 2e-8
    assert its[sgf.FP32_BF16N] <= 2 * its[sgf.FP32] + 5


@pytest.mark.parametrize("cap", [1, 3])
def test_persistent_work_lists_match_oracle(cap):
    """Persistent launches of the elimination and compression work lists (a
    few workgroups taking clusters from a counter, costliest first) give the
    same operator as one workgroup per cluster."""
    p = _prob("fourier", (61, 58), seed=4)
    F = _oracle(p, 2, 8)
    s = sgf.Solver.from_problem(p, q=2, leaf=8)
    s.set_persistent(cap)
    s.factorize(torch.from_numpy(p.data).cuda())
    V = np.stack([P.random_rhs(8, p.n, j) for j in range(2)], axis=1)
    assert _rel(_apply(s, V), O.apply_inverse(F, V)) <= 1e-10
    # same kernels apart from the launch shape (persistent launches use the
    # workgroup compression), so the same bits
    ref = sgf.Solver.from_problem(p, q=2, leaf=8)
    ref.set_small_compress(False)
    ref.factorize(torch.from_numpy(p.data).cuda())
    assert np.array_equal(_apply(s, V), _apply(ref, V))


@pytest.mark.parametrize("kind,grid,leaf,q", [("fourier", (100, 90), 16, 2), ("fourier", (61, 58), 8, 2),
                                              ("blocky", (17, 16, 15), 4, 1), ("elast", 9, 3, 1)])
def test_band_sweeps_match_blocked_sweeps_and_oracle(kind, grid, leaf, q):
    """Interior sweeps of the banded kernels (band of L_I staged in LDS, one
    wavefront per column; 2D leaf 16 gives 225-row interiors, four chunks of
    64 with a ragged last one) against the blocked sweeps and the oracle,
    for 1, 5 (4 + 1 per workgroup) and 7 columns."""
    p = _prob(kind, grid)
    F = _oracle(p, q, leaf)
    s = _gpu(p, q=q, leaf=leaf)
    s.set_apply_graph(False)
    for nc in (1, 5, 7):
        V = np.stack([P.random_rhs(9, p.n, j) for j in range(nc)], axis=1)
        s.set_band_apply(True)
        s.profile(True)
        zb = _apply(s, V)
        used = s.profile_read()
        s.profile(False)
        assert used.get("apply_band_fwd", {}).get("launches", 0) >= 1
        assert used.get("apply_band_bwd", {}).get("launches", 0) >= 1
        s.set_band_apply(False)
        s.profile(True)
        zd = _apply(s, V)
        assert "apply_band_fwd" not in s.profile_read()
        s.profile(False)
        print(f"{kind} {grid} leaf {leaf}, {nc} columns: banded vs blocked {_rel(zb, zd):.1e}")
        assert _rel(zb, zd) <= 1e-13
        assert _rel(zb, O.apply_inverse(F, V)) <= 1e-10
        if nc == 1:
            # one wavefront per front (default for one column on levels of the
            # banded elimination) against one workgroup per front: the same bits
            s.set_band_apply(2)
            zw = _apply(s, V)
            assert np.array_equal(zb, zw)
        if nc == 7:
            s.set_band_apply(True)
            zc = np.stack([_apply(s, V[:, j]) for j in range(nc)], axis=1)
            assert np.array_equal(zb, zc)


@pytest.mark.parametrize("kind,grid,leaf,q", [("const", (70, 66), 4, 1), ("blocky", (96, 80), 8, 1),
                                              ("fourier", (61, 58), 8, 2), ("fourier", (200, 190), 16, 2)])
def test_small_front_sweeps_match_blocked_sweeps_and_oracle(kind, grid, leaf, q):
    """One right-hand side on levels whose interiors have at most 64 rows
    (FP32 factor and sweeps, the form whose L_SI fits the kernel's LDS):
    one workgroup per front with every load issued before waiting and the
    solve on one wavefront (k_apply1, both directions) against the sweeps
    several columns take (the same steps and summation orders, so the same
    values) and the FP64 oracle."""
    p = _prob(kind, grid)
    F = _oracle(p, q, leaf)
    s = _gpu(p, q=q, leaf=leaf, precision=sgf.FP32)
    s.set_apply_graph(False)
    v = P.random_rhs(13, p.n)
    s.set_small_apply(True)
    s.profile(True)
    za = _apply(s, v)
    used = s.profile_read()
    s.profile(False)
    assert used.get("apply_small_fwd", {}).get("launches", 0) >= 1
    assert used.get("apply_small_bwd", {}).get("launches", 0) >= 1
    s.set_small_apply(False)
    s.profile(True)
    zb = _apply(s, v)
    assert "apply_small_fwd" not in s.profile_read()
    s.profile(False)
    ref = O.apply_inverse(F, v)
    print(f"{kind} {grid} leaf {leaf}: small vs blocked {_maxrel(za, zb):.1e}, vs oracle {_rel(za, ref):.1e} "
          f"(blocked vs oracle {_rel(zb, ref):.1e})")
    assert np.array_equal(za, zb)
    assert _rel(za, ref) <= 1e-4
    # the graph replays the same kernels
    s.set_small_apply(True)
    s.set_apply_graph(True)
    assert np.array_equal(_apply(s, v), za)


def test_pcg_iteration_graphs_for_several_rhs_counts():
    """The captured PCG iteration is kept per right-hand-side count and is
    independent of the caller's solution buffer: solves with 1, 2, 1 and 3
    columns into fresh tensors, with a refactorization in between, equal
    direct-launch solves bit for bit."""
    p = _prob("fourier", (70, 61), seed=6)
    s = _gpu(p, q=2, leaf=4, precision=sgf.FP32)
    for step, k in enumerate((1, 2, 1, 3)):
        if step == 2:
            s.factorize(torch.from_numpy(p.data).cuda())
        b = torch.from_numpy(np.stack([P.random_rhs(30 + step, p.n, j) for j in range(k)], axis=0)).cuda()
        s.set_apply_graph(True)
        xg = torch.full_like(b, float("nan"))
        itg, relg = s.pcg(b.T, xg.T, rtol=1e-9)
        s.set_apply_graph(False)
        xd = torch.zeros_like(b)
        itd, reld = s.pcg(b.T, xd.T, rtol=1e-9)
        assert itg.tolist() == itd.tolist() and torch.equal(xg, xd), f"step {step}, {k} columns"
        assert float(relg.max()) < 1e-9


@pytest.mark.parametrize("kind,grid,leaf,q", [("fourier", (100, 90), 16, 2), ("fourier", (61, 58), 8, 2),
                                              ("fourier", (35, 130), 16, 1), ("blocky", (45, 45), 4, 1)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_banded_elimination_matches_panel_elimination_and_oracle(kind, grid, leaf, q, prec):
    """Level-1 interiors eliminated one wavefront per front (band Cholesky
    in an LDS ring, L_SI in registers, L_SI L_SI^T on the matrix cores):
    2D leaf 16 (225-row interiors, 14 blocks of 16 columns, ragged last
    block), leaf 8 (49 rows, ring of 8) and leaf 4; against the panel
    kernel and the oracle; same ranks at every level."""
    p = _prob(kind, grid)
    F = _oracle(p, q, leaf)
    pr = sgf.FP64 if prec == "fp64" else sgf.FP32
    out, ranks = {}, {}
    for banded in (True, False):
        s = sgf.Solver.from_problem(p, q=q, leaf=leaf, precision=pr)
        s.set_band_elim(banded)
        s.profile(True)
        s.factorize(torch.from_numpy(p.data).cuda())
        torch.cuda.synchronize()
        st = s.profile_read()
        s.profile(False)
        assert ("elim_banded" in st) == banded
        V = np.stack([P.random_rhs(12, p.n, j) for j in range(2)], axis=1)
        out[banded] = _apply(s, V)
        ranks[banded] = [s.level(t)["rank"].tolist() for t in range(1, s.info()["levels"])]
    assert ranks[True] == ranks[False]
    za = O.apply_inverse(F, V)
    d = _rel(out[True], out[False])
    print(f"{kind} {grid} leaf {leaf} {prec}: banded vs panel {d:.1e}, vs oracle {_rel(out[True], za):.1e} "
          f"(panel vs oracle {_rel(out[False], za):.1e})")
    if prec == "fp64":
        assert d <= 1e-12
        assert _rel(out[True], za) <= 1e-10
    else:
        assert d <= 1e-4
        assert _rel(out[True], za) <= 1e-3


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_refactorization_clears_only_the_band_and_matches_a_fresh_handle(prec):
    """Refactorizing one handle with other coefficients: while the level-1
    fronts are known clean outside the band, the banded path clears only
    the lower band and M_SI of each front (and the pair blocks); the result
    is bitwise that of a fresh handle, also after a factorization through
    the panel path has written the fronts (the next banded one clears them
    all again)."""
    pa, pb = _prob("fourier", (100, 90), seed=0), _prob("fourier", (100, 90), seed=1)
    pr = sgf.FP64 if prec == "fp64" else sgf.FP32
    V = np.stack([P.random_rhs(5, pa.n, j) for j in range(2)], axis=1)
    vals = {"a": torch.from_numpy(pa.data).cuda(), "b": torch.from_numpy(pb.data).cuda()}
    ref = {}
    for key in "ab":
        s = sgf.Solver.from_problem(pa, q=2, leaf=16, precision=pr)
        s.factorize(vals[key])
        ref[key] = _apply(s, V)
        s.close()
    s = sgf.Solver.from_problem(pa, q=2, leaf=16, precision=pr)
    zb = []
    for key, banded in (("a", True), ("b", True), ("a", True), ("b", False), ("a", True), ("b", True)):
        s.set_band_elim(banded)
        s.profile(True)
        s.factorize(vals[key])
        out = _apply(s, V)
        st = s.profile_read()
        s.profile(False)
        assert ("elim_banded" in st) == banded
        zb.append(st["zero@L1"]["bytes"])
        if banded:
            assert np.array_equal(out, ref[key]), (key, _rel(out, ref[key]))
        else:
            assert _rel(out, ref[key]) <= (1e-12 if prec == "fp64" else 1e-4)
    # full clears: the first factorization, the panel one and the banded one
    # after it; band-only clears in between
    print("cleared bytes per factorization:", zb)
    assert zb[0] == zb[3] == zb[4]
    assert zb[1] == zb[2] == zb[5] < zb[0] / 2


def test_refactorization_on_changing_streams_matches_fresh_handles():
    """Descriptor tables go to the device through one pinned staging buffer
    per handle, reused after the stream that read it is synchronized:
    refactorizations of one handle on two side streams and the default
    stream in turn (other coefficients each time, so the upper levels are
    re-planned and re-uploaded) give bitwise the applies of fresh handles."""
    pa, pb = _prob("fourier", (61, 58), seed=2), _prob("fourier", (61, 58), seed=3)
    V = np.stack([P.random_rhs(6, pa.n, j) for j in range(3)], axis=1)
    vals = {"a": torch.from_numpy(pa.data).cuda(), "b": torch.from_numpy(pb.data).cuda()}
    ref = {}
    for key in "ab":
        s = sgf.Solver.from_problem(pa, q=2, leaf=8, precision=sgf.FP32)
        s.factorize(vals[key])
        ref[key] = _apply(s, V)
        s.close()
    s = sgf.Solver.from_problem(pa, q=2, leaf=8, precision=sgf.FP32)
    side = [torch.cuda.Stream(), torch.cuda.Stream()]   # default priority
    streams = [side[0].cuda_stream, side[1].cuda_stream, None]
    for step, key in enumerate("abbaab"):
        st = streams[step % 3]
        torch.cuda.synchronize()
        s.factorize(vals[key], stream=st)
        torch.cuda.synchronize()
        out = _apply(s, V)
        assert np.array_equal(out, ref[key]), (step, key, _rel(out, ref[key]))


def test_profile_select_times_one_kernel_class():
    """With a class selected, only its launches are timed (with their level
    tags); the selection cleared, every launch is timed again."""
    p = _prob("fourier", (100, 90))
    s = sgf.Solver.from_problem(p, q=2, leaf=16, precision=sgf.FP32)
    v = torch.from_numpy(p.data).cuda()
    s.factorize(v)
    s.profile_select("elim_banded")
    s.profile(True)
    s.factorize(v)
    st = s.profile_read()
    s.profile(False)
    assert st and all(k.split("@")[0] == "elim_banded" for k in st), sorted(st)
    assert st["elim_banded"]["launches"] >= 1 and st["elim_banded"]["ms"] > 0 and "elim_banded@L1" in st
    s.profile_select(None)
    s.profile(True)
    s.factorize(v)
    st = s.profile_read()
    s.profile(False)
    assert "elim_banded" in st and "compress" in st and "fill_csr" in st


def test_banded_elimination_reports_non_spd_cluster():
    """A non-positive pivot inside a banded front is reported with its cluster."""
    p = _prob("const", (64, 64))
    vals = p.data.copy()
    A = p.csr()
    s = sgf.Solver.from_problem(p, q=1, leaf=16)
    node = 0   # a corner node: inside the first interior
    row = slice(A.indptr[node], A.indptr[node + 1])
    diag = np.where(A.indices[row] == node)[0][0] + A.indptr[node]
    vals[diag] = -1.0
    s.profile(True)
    with pytest.raises(sgf.SgfError) as ei:
        s.factorize(torch.from_numpy(vals).cuda())
    st = s.profile_read()
    assert "elim_banded@L1" in st, sorted(st)
    assert ei.value.code == sgf.SGF_ENOTSPD
    assert s.info()["failed_level"] == 1 and s.info()["failed_cluster"] >= 0


@pytest.mark.parametrize("kind,grid,leaf,q", [("fourier", (100, 90), 16, 2), ("blocky", (17, 16, 15), 4, 1),
                                              ("elast", 9, 3, 1), ("fourier", (61, 58), 8, 2)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_small_compression_matches_workgroup_compression_and_oracle(kind, grid, leaf, q, prec):
    """Separators compressed one wavefront each (front, Phi and N in LDS)
    against the one-workgroup compression and the oracle: same ranks at
    every level, the same operator up to rounding."""
    p = _prob(kind, grid)
    F = _oracle(p, q, leaf)
    pr = sgf.FP64 if prec == "fp64" else sgf.FP32
    out, ranks = {}, {}
    V = np.stack([P.random_rhs(13, p.n, j) for j in range(2)], axis=1)
    for small in (True, False):
        s = sgf.Solver.from_problem(p, q=q, leaf=leaf, precision=pr)
        s.set_small_compress(small)
        s.factorize(torch.from_numpy(p.data).cuda())
        out[small] = _apply(s, V)
        ranks[small] = [s.level(t)["rank"].tolist() for t in range(1, s.info()["levels"])]
    assert ranks[True] == ranks[False]
    za = O.apply_inverse(F, V)
    d = _rel(out[True], out[False])
    print(f"{kind} {grid} leaf {leaf} {prec}: small vs workgroup {d:.1e}, vs oracle {_rel(out[True], za):.1e} "
          f"(workgroup vs oracle {_rel(out[False], za):.1e})")
    if prec == "fp64":
        assert d <= 1e-12
        assert _rel(out[True], za) <= 1e-10
    else:
        assert d <= 1e-4
        assert _rel(out[True], za) <= 1e-3


@pytest.mark.parametrize("kind,grid,leaf,q", [("fourier", (100, 90), 16, 2), ("blocky", (17, 16, 15), 4, 1),
                                              ("fourier", (61, 58), 8, 2)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_small_compression_on_four_wavefronts_equals_one(kind, grid, leaf, q, prec):
    """Levels with few small separators compress each on four wavefronts
    (staging, neighbour rows, N and the reflector pass spread over them,
    the Cholesky and the pivoted QR on the first); every value comes from
    the same code as on one wavefront, so the ranks and the preconditioner
    are the same bit for bit."""
    p = _prob(kind, grid)
    pr = sgf.FP64 if prec == "fp64" else sgf.FP32
    V = np.stack([P.random_rhs(17, p.n, j) for j in range(2)], axis=1)
    out, ranks = {}, {}
    for mode in (True, "one"):
        s = sgf.Solver.from_problem(p, q=q, leaf=leaf, precision=pr)
        s.set_small_compress(mode)
        s.profile(True)
        s.factorize(torch.from_numpy(p.data).cuda())
        st = s.profile_read()
        s.profile(False)
        assert st.get("compress", {}).get("launches", 0) >= 1
        out[mode] = _apply(s, V)
        ranks[mode] = [s.level(t)["rank"].tolist() for t in range(1, s.info()["levels"])]
        s.close()
    assert ranks[True] == ranks["one"]
    assert np.array_equal(out[True], out["one"])


@pytest.mark.parametrize("order", ["pcg1-apply8-pcg1", "apply1-pcg4-apply1"])
def test_graphs_recaptured_after_work_buffers_grow(order):
    """The captured apply and PCG graphs hold the addresses of the apply's
    work vectors; a call with more columns reallocates them, and a later
    call with fewer columns must not replay a graph recorded on the freed
    buffers.  Each call equals the same call on a fresh handle bit for bit."""
    p = _prob("fourier", (70, 61), seed=7)
    B = torch.from_numpy(np.stack([P.random_rhs(40, p.n, j) for j in range(8)], axis=0)).cuda()

    def run(s, step):
        kind, k = step
        if kind == "pcg":
            x = torch.full((k, p.n), float("nan"), dtype=torch.float64, device="cuda")
            it, _ = s.pcg(B[:k].T, x.T, rtol=1e-9)
            torch.cuda.synchronize()
            return it.tolist(), x.cpu().numpy()
        z = torch.full((k, p.n), float("nan"), dtype=torch.float64, device="cuda")
        s.apply(B[:k].T, z.T)
        torch.cuda.synchronize()
        return None, z.cpu().numpy()

    steps = {"pcg1-apply8-pcg1": [("pcg", 1), ("apply", 8), ("pcg", 1)],
             "apply1-pcg4-apply1": [("apply", 1), ("pcg", 4), ("apply", 1)]}[order]
    s = _gpu(p, q=2, leaf=4, precision=sgf.FP32)
    for i, step in enumerate(steps):
        got = run(s, step)
        fresh = _gpu(p, q=2, leaf=4, precision=sgf.FP32)
        want = run(fresh, step)
        fresh.close()
        assert got[0] == want[0] and np.array_equal(got[1], want[1]), f"step {i} {step}"


def _blockrel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)) if b.size else 0.0


@pytest.mark.parametrize("kind,grid,leaf,q,tiled", [("fourier", (100, 90), 16, 2, -1), ("fourier", (50, 41), 4, 2, -1),
                                                    ("blocky", (14, 13, 12), 3, 1, -1), ("blocky", (14, 13, 12), 3, 1, 0),
                                                    ("elast", 8, 3, 1, -1)])
def test_factor_entries_match_oracle(kind, grid, leaf, q, tiled):
    """FP64 factor entries, block by block, against the oracle's (shared QR
    pivot, tie and sign conventions): L_I and W = L_I^{-1} M_IS of every
    interior (Eq. 4.2), L_B, the Householder vectors and tau of every
    compressed separator (Eqs. 3.1, 3.3), and the top factor (Sec. 4.5),
    each within 1e-10 of its largest entry.  Reflector k is formed from a
    trailing part of size |R_kk|, so rounding of order eps |R_00| moves it
    by about eps |R_00| / |R_kk|: column k of V and tau_k are compared
    within max(1e-10, 100 eps / min_{j<=k} |R_jj / R_00|) (the bar only
    widens for columns whose pivots fall below 2e-4 |R_00|), and the
    number of such columns is printed."""
    p = _prob(kind, grid)
    F = _oracle(p, q, leaf)
    s = _gpu(p, q=q, leaf=leaf, tiled_min_rows=tiled)
    worst = {"L_I": 0.0, "W": 0.0, "L_B": 0.0, "V": 0.0, "tau": 0.0, "top": 0.0}
    widened = ncols = 0
    nlev = s.info()["levels"]
    assert nlev == F.info["nlevels"]
    for t in range(1, nlev):
        blocks = s.blocks(t)
        ops = F.levels[t - 1]
        elims = [o for o in ops if o[0] == "elim"]
        comps = [o for o in ops if o[0] == "comp"]
        gb_e = [b for b in blocks if b["kind"] == sgf.BLOCK_ELIM]
        gb_c = [b for b in blocks if b["kind"] == sgf.BLOCK_COMP]
        assert len(gb_e) == len(elims) and len(gb_c) == len(comps), f"level {t}"
        for g, o in zip(gb_e, elims):
            _, vI, L, Ws = o
            W = np.hstack([w for _, w in Ws]) if Ws else np.zeros((len(vI), 0))
            assert g["L"].shape == L.shape and g["W"].shape == W.shape
            worst["L_I"] = max(worst["L_I"], _blockrel(g["L"], L))
            worst["W"] = max(worst["W"], _blockrel(g["W"], W))
        for g, o in zip(gb_c, comps):
            _, vB, L, V, tau, r = o
            assert g["r"] == r and g["V"].shape == V.shape
            worst["L_B"] = max(worst["L_B"], _blockrel(g["L"], L))
            ratio = np.minimum.accumulate(np.abs(g["rdiag"]) / abs(g["rdiag"][0]))
            bar = np.maximum(1e-10, 100 * np.finfo(float).eps / ratio)
            widened += int(np.sum(bar > 1e-10))
            ncols += r
            vmax = max(np.abs(V).max(), 1.0)
            ev = np.abs(g["V"] - V).max(axis=0) / vmax / bar
            et = np.abs(g["tau"] - tau) / max(np.abs(tau).max(), 1e-300) / bar
            worst["V"] = max(worst["V"], float(ev.max()) * 1e-10)
            worst["tau"] = max(worst["tau"], float(et.max()) * 1e-10)
    top = s.blocks(nlev)
    assert len(top) == 1 and top[0]["kind"] == sgf.BLOCK_TOP
    worst["top"] = _blockrel(top[0]["L"], F.top[1])
    print(f"{kind} {grid} leaf {leaf} q {q} tiled {tiled}: " + ", ".join(f"{k} {v:.1e}" for k, v in worst.items())
          + f" (V, tau: error / bar x 1e-10; {widened} of {ncols} reflector columns with a widened bar)")
    assert max(worst.values()) <= 1e-10, worst


@pytest.mark.parametrize("kind,grid,leaf,q", [("fourier", (100, 90), 16, 2), ("fourier", (61, 58), 8, 2),
                                              ("blocky", (17, 16, 15), 4, 1), ("elast", 9, 3, 1)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pair_kernels_give_the_same_bits(kind, grid, leaf, q, prec):
    """Coarse couplings by one wavefront per pair (intermediate in LDS) and
    by one workgroup per pair (intermediate in device scratch): the same
    products in the same order, so the same factor bit for bit."""
    p = _prob(kind, grid)
    pr = sgf.FP64 if prec == "fp64" else sgf.FP32
    V = np.stack([P.random_rhs(14, p.n, j) for j in range(2)], axis=1)
    out = {}
    for mode in (0, 1):
        s = sgf.Solver.from_problem(p, q=q, leaf=leaf, precision=pr)
        s.set_pair_kernel(mode)
        s.factorize(torch.from_numpy(p.data).cuda())
        out[mode] = (_apply(s, V), _apply(s, V, product=True))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("q", [0, 2])
def test_headline_paths_at_512_match_oracle(q):
    """The kernels the 1024^2 workload runs, on a 512^2 grid with its leaf
    (16): banded level-1 elimination with the 16-wide boundary blocks on
    ring width 24, more than 4096 active pairs (so the one-wavefront
    coupling kernel), one-wavefront compressions, banded sweeps.
    q = 0 has a clear gap at the rank cut (kept pivot ratios >= 6e-8,
    dropped <= 4e-15): FP64 element by element against the oracle within
    1e-10 of each column's largest entry, CG iterations +-1, solution 1e-8;
    the FP32 form within the FP32 bars.
    q = 2 (the headline's degree): the level-1 edges' pivot ratios spread
    continuously over 1e-13 .. 1e-11 around the threshold 1e-12, so no
    implementation determines the FP64 operator beyond about eps / 1e-12:
    parity unpinned at 1e-10; checked instead: the same ranks at every level,
    the operator within 10 eps / (smallest kept ratio), preservation of the
    quadratics (Prop. 6.1) within 1e-9, CG iterations +-1."""
    p = _prob("fourier", (512, 512))
    A = p.csr()
    F = _oracle(p, q, 16)
    kept = min(x[4] for x in F.info["gap"] if x[3] > 0)
    dropped = max(x[5] for x in F.info["gap"])
    gapless = kept < 10 * dropped
    assert gapless == (q == 2)
    bar = max(1e-10, 10 * np.finfo(float).eps / kept) if gapless else 1e-10
    V = np.stack([P.random_rhs(15, p.n, j) for j in range(2)], axis=1)
    za, zm = O.apply_inverse(F, V), O.multiply(F, V)
    b = P.random_rhs(0, p.n)
    xo, ito, _ = O.pcg(A, b, lambda r: O.apply_inverse(F, r), tol=1e-8)
    for prec in (sgf.FP64, sgf.FP32):
        s = sgf.Solver.from_problem(p, q=q, leaf=16, precision=prec)
        s.set_apply_graph(False)
        s.profile(True)
        s.factorize(torch.from_numpy(p.data).cuda())
        ea, em = _maxrel(_apply(s, V), za), _maxrel(_apply(s, V, product=True), zm)
        st = s.profile_read()
        s.profile(False)
        assert "elim_banded@L1" in st and "apply_band_fwd@L1" in st and "apply_band_bwd@L1" in st
        L1 = s.level(1)
        assert np.sum(L1["type"] == 0) == 1024
        xg = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        it, rel = s.pcg(torch.from_numpy(b).cuda(), xg, rtol=1e-8)
        ex = _maxrel(xg.cpu().numpy(), xo)
        print(f"512^2 q {q} precision {prec}: apply {ea:.1e}, product {em:.1e}, CG it {int(it[0])} (oracle {ito}), "
              f"x {ex:.1e}, kept >= {kept:.1e}, dropped <= {dropped:.1e}, bar {bar:.1e}")
        if prec == sgf.FP64:
            for t in range(1, F.info["nlevels"]):
                g = s.level(t)
                post = F.info["sizes"][t - 1]
                seps = g["type"] > 0
                assert [post[c] for c in g["cell"][seps]] == g["rank"][seps].tolist(), f"ranks at level {t}"
            assert ea <= bar and em <= bar
            assert abs(int(it[0]) - ito) <= 1
            if not gapless:
                assert ex <= 1e-8
            else:
                Pi = O.poly_basis(p.coords, q, 1)
                pres = _maxrel(_apply(s, Pi, product=True), A @ Pi)
                print(f"512^2 q {q}: preservation {pres:.1e}")
                assert pres <= 1e-9
        else:
            assert ea <= 1e-3 and em <= 1e-3
            assert np.linalg.norm(b - A @ xg.cpu().numpy()) / np.linalg.norm(b) < 2e-8


@pytest.mark.skip(reason="the device coarsening is switched off: its kernel faulted the GPU (tables uploaded from "
                         "host vectors freed before the upload batch was flushed); fixed, not re-tested on the GPU")
@pytest.mark.parametrize("kind,grid,leaf,q", [("fourier", (100, 90), 16, 2), ("blocky", (17, 16, 15), 4, 1),
                                              ("elast", 9, 3, 1)])
@pytest.mark.parametrize("stop", [sgf.STOP_ROOT, sgf.STOP_PAPER])
def test_device_coarsening_equals_host_copy_lists(kind, grid, leaf, q, stop):
    """Coarsening destinations computed on the device from the two levels'
    structure and the sizes after compression, against the copy list of
    every block built on the host: the same factor bit for bit, also over
    refactorizations with other values (levels re-planned in place)."""
    p = _prob(kind, grid)
    p2 = _prob(kind, grid, seed=1)
    V = np.stack([P.random_rhs(16, p.n, j) for j in range(2)], axis=1)
    out = {}
    for dev in (True, False):
        s = sgf.Solver.from_problem(p, q=q, leaf=leaf, stop_rule=stop, precision=sgf.FP32)
        s.set_device_coarsen(dev)
        res = []
        for vals in (p.data, p2.data, p.data):
            s.factorize(torch.from_numpy(vals).cuda())
            res.append(_apply(s, V))
        out[dev] = res
        s.close()
    for a, b in zip(out[True], out[False]):
        assert np.array_equal(a, b)


def test_full_size_headline_fp64_against_oracle():
    """The 1024^2 workload of the benchmark (q = 2, leaf 16) in the FP64 form
    against the oracle at full size: the same rank at every separator of
    every level, CG iterations +-1 at 1e-8, the solution within 1e-8, and
    the quadratics preserved (Prop. 6.1) through the device product.  (The
    rank cut of this shape has no spectral gap, so the operator itself is
    compared only through these; see the 512^2 tests.)"""
    import time
    from sgf_inputs.problems import config_problem
    p, cfg = config_problem("varcoef2d_1024", seed=0)
    A = p.csr()
    t0 = time.perf_counter()
    F = _oracle(p, cfg["q"], cfg["leaf"])
    b = P.random_rhs(0, p.n)
    xo, ito, _ = O.pcg(A, b, lambda r: O.apply_inverse(F, r), tol=1e-8)
    t1 = time.perf_counter()
    s = _gpu(p, q=cfg["q"], leaf=cfg["leaf"])
    assert s.info()["levels"] == F.info["nlevels"]
    for t in range(1, F.info["nlevels"]):
        g = s.level(t)
        post = F.info["sizes"][t - 1]
        seps = g["type"] > 0
        assert [post[c] for c in g["cell"][seps]] == g["rank"][seps].tolist(), f"ranks at level {t}"
    xg = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    it, rel = s.pcg(torch.from_numpy(b).cuda(), xg, rtol=1e-8)
    ex = _maxrel(xg.cpu().numpy(), xo)
    Pi = O.poly_basis(p.coords, cfg["q"], 1)[:, [0, 3, 5]]   # 1, x^2, xy
    pres = _maxrel(_apply(s, Pi, product=True), A @ Pi)
    print(f"1024^2 FP64: CG it {int(it[0])} (oracle {ito}), x {ex:.1e}, preservation {pres:.1e}, "
          f"oracle {t1 - t0:.0f} s")
    assert abs(int(it[0]) - ito) <= 1 and ex <= 1e-8 and pres <= 1e-9
