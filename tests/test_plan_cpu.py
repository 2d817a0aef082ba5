"""Host-side checks of the HIP library that need no GPU: it loads, exports
every symbol of include/sgf.h, and its symbolic planner reproduces the
oracle's partition hierarchy bit for bit (cells, types, active-set sizes and
the level-1 permutation), given the oracle's compression ranks."""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from oracle import sgf_oracle as O
from sgf_inputs import problems as P

sgf = pytest.importorskip("paper_1907_03406_amd.sgf")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    decl = open(os.path.join(ROOT, "include", "sgf.h")).read()
    names = set(re.findall(r"\b(sgf_[a-z_]+)\s*\(", decl)) - {"sgf_rank_fn"}
    assert names == set(sgf.EXPORTED), names ^ set(sgf.EXPORTED)
    for name in names:
        assert hasattr(sgf._lib, name)


def test_status_strings_and_defaults():
    assert sgf._lib.sgf_status_str(0) == b"ok"
    o = sgf.make_options(2, (4, 4))
    assert o.q == 1 and o.leaf == 8 and o.compress == 1 and o.precision == sgf.FP64


def test_analyze_rejects_bad_input():
    p = P.poisson_fd((6, 5))
    with pytest.raises(sgf.SgfError):
        sgf.Solver(p.n, p.indptr, p.indices, p.coords, sgf.make_options(2, (6, 6)))
    with pytest.raises(sgf.SgfError):
        sgf.Solver(p.n, p.indptr, p.indices, p.coords, sgf.make_options(2, (6, 5), q=3))
    # a pattern that couples nodes two grid steps apart breaks the Sec. 5 assumption
    A = p.csr().tolil()
    A[0, 2] = A[2, 0] = -0.1
    A = A.tocsr()
    with pytest.raises(sgf.SgfError):
        sgf.Solver(p.n, A.indptr, A.indices, p.coords, sgf.make_options(2, (6, 5)))


def _oracle_levels(F, levels):
    return F.info["ranks"], F.info["sizes"]


CASES = [("poisson", (64, 64), 8, 1, 1), ("poisson", (20, 17), 4, 2, 1), ("poisson", (13, 9, 11), 3, 1, 1),
         ("fourier", (40, 33), 4, 0, 1), ("elast", 7, 3, 1, 3), ("poisson", (16, 16, 16), 4, 2, 1)]


def _make(kind, grid):
    if kind == "poisson":
        return P.poisson_fd(grid)
    if kind == "fourier":
        return P.poisson_fd(grid, P.gaussian_field_fourier(2, len(grid)))
    return P.elasticity_q1(grid, seed=1, n_incl=2)


SCHEME_CASES = [(sch, case) for sch in (sgf.NEST_2_ALL, sgf.NEST_2_2)
                for case in (CASES[1], CASES[2], CASES[4], CASES[5])] + \
               [(sgf.GEN_ALL_ALL, c) for c in (("poisson", (20, 17), 4, 1, 1), ("poisson", (13, 9, 11), 3, 0, 1),
                                              ("fourier", (40, 33), 5, 2, 1), ("elast", 7, 3, 1, 3),
                                              ("poisson", (16, 16, 16), 4, 1, 1))]


@pytest.mark.parametrize("kind,grid,leaf,q,dpn", CASES)
@pytest.mark.parametrize("stop", [sgf.STOP_ROOT, sgf.STOP_PAPER])
def test_planner_matches_oracle_hierarchy(kind, grid, leaf, q, dpn, stop):
    _check_hierarchy(kind, grid, leaf, q, stop, sgf.NEST_ALL_ALL)


@pytest.mark.parametrize("scheme,case", SCHEME_CASES)
def test_planner_matches_oracle_hierarchy_of_each_scheme(scheme, case):
    """Nest-2-All and Nest-2-2 compress only the cells of codimension one;
    Gen-All-All has boxes of leaf^dim vertices with no interiors, every one
    compressed at every level (Secs. 5.1-5.2)."""
    kind, grid, leaf, q, dpn = case
    _check_hierarchy(kind, grid, leaf, q, sgf.STOP_ROOT, scheme)


def _check_hierarchy(kind, grid, leaf, q, stop, scheme):
    p = _make(kind, grid)
    general = scheme == sgf.GEN_ALL_ALL
    F = O.factorize(p.csr(), p.coords, p.grid, p.dpn,
                    O.Options(q=q, leaf=leaf, stop_rule=O.STOP_PAPER if stop else O.STOP_ROOT, scheme=scheme))
    s = sgf.Solver.from_problem(p, q=q, leaf=leaf, stop_rule=stop, scheme=scheme)
    # level-1 permutation: cells ascending, unknowns ascending inside a cell
    lv1 = O.partition_hierarchy(p.grid, leaf, general=general)[0]
    cell_dof = np.repeat(lv1.cell_of_node, p.dpn)
    assert np.array_equal(s.perm(), np.argsort(cell_dof, kind="stable"))
    ranks = F.info["ranks"]
    s.plan_dry_run(lambda t, cell, size: ranks[t - 1].get(cell, size))
    nlev = F.info["nlevels"]
    assert s.info()["levels"] == nlev
    levels = O.partition_hierarchy(p.grid, leaf, general=general)
    for t in range(1, nlev):
        g = s.level(t)
        # separators after the level's compressions: cell ids and sizes
        post = F.info["sizes"][t - 1]
        seps = g["type"] > 0
        assert sorted(post) == g["cell"][seps].tolist()
        assert [post[c] for c in g["cell"][seps]] == g["rank"][seps].tolist()
        assert np.array_equal(g["type"], levels[t - 1].type[g["cell"]])
    top = s.level(nlev)
    assert top["size"].sum() == F.info["top_size"]


def test_memory_estimate_is_host_only():
    """sgf_estimate_bytes plans every level with the largest possible ranks
    (host only): it grows with the right-hand sides and leaves the handle
    able to plan again."""
    p = P.poisson_fd((40, 36), P.gaussian_field_fourier(0, 2))
    s = sgf.Solver.from_problem(p, q=1, leaf=4, precision=sgf.FP32)
    e1, e4 = s.estimate_bytes(1), s.estimate_bytes(4)
    assert 0 < e1 < e4
    assert s.estimate_bytes(1) == e1
    # an unfactored handle may be released (nothing to free) and still dry-run
    s.release()
    s.plan_dry_run(lambda t, cell, size: min(size, 3))
    assert s.info()["levels"] >= 2 and s.info()["device_bytes"] == 0


def test_in_place_replanning_matches_planning_afresh(tmp_path):
    """The next level re-planned in place for new ranks (only sizes, slots
    and offsets redone) equals the level planned afresh with those ranks,
    copy maps included, on 2D and 3D grids: a C++ check of the planner
    header built with the host compiler."""
    cxx = shutil.which("g++") or shutil.which("c++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "plan_update_check")
    subprocess.run([cxx, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1907_03406_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "plan_update_check.cpp"), "-o", exe], check=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
