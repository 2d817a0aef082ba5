"""Pins of the seeded input generators (CPU only)."""
import os

import numpy as np

from sgf_inputs import problems as P
from sgf_inputs.rng import splitmix64_bits, splitmix64_uniform, normal

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_matches_published_outputs():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64.txt"))
            if l.strip() and not l.startswith("#")]
    for seed, k, hexval in rows:
        got = int(splitmix64_bits(int(seed), 0, 1, start=int(k))[0])
        assert got == int(hexval, 16), (seed, k)


def test_streams_are_counter_based_and_distinct():
    a = splitmix64_uniform(7, 5, 100)
    b = splitmix64_uniform(7, 5, 40, start=60)
    assert np.array_equal(a[60:], b)
    c = splitmix64_uniform(7, 6, 100)
    assert not np.allclose(a, c)
    assert a.min() >= 0.0 and a.max() < 1.0


def test_normal_moments():
    z = normal(3, 1, 200000)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.02


def test_poisson_constant_is_integer_stencil():
    p2 = P.poisson_fd((5, 4))
    A = p2.csr().toarray()
    assert np.array_equal(np.diag(A), np.full(20, 4.0))
    off = A - np.diag(np.diag(A))
    assert set(np.unique(off)) <= {0.0, -1.0}
    # 5-point: each row couples to its grid neighbours only
    assert np.array_equal((off != 0).sum(axis=1),
                          [sum(0 <= x + dx < 5 and 0 <= y + dy < 4 for dx, dy in
                               ((1, 0), (-1, 0), (0, 1), (0, -1))) for y in range(4) for x in range(5)])
    p3 = P.poisson_fd((3, 3, 3))
    A3 = p3.csr().toarray()
    assert np.array_equal(np.diag(A3), np.full(27, 6.0))


def test_variable_coefficient_is_spd_and_symmetric():
    for coef, g in ((P.gaussian_field_fourier(1, 2), (12, 9)), (P.blocky_log_field(2, 3), (6, 5, 7))):
        p = P.poisson_fd(g, coef)
        A = p.csr().toarray()
        assert np.array_equal(A, A.T)
        assert np.linalg.eigvalsh(A).min() > 0


def test_harmonic_face_mean():
    # two nodes in 1 x 2 grid: coupling is minus the harmonic mean of a
    vals = {0: 1.0, 1: 4.0}
    coef = lambda x: np.where(x[:, 1] < 0.5, vals[0], vals[1])
    p = P.poisson_fd((1, 2), coef)
    A = p.csr().toarray()
    assert np.isclose(A[0, 1], -2 * 1 * 4 / (1 + 4))


def test_elasticity_rigid_modes_in_kernel_away_from_clamp():
    e = P.elasticity_q1(6, seed=1, n_incl=3)
    A = e.csr().toarray()
    assert np.allclose(A, A.T, atol=1e-14)
    assert np.linalg.eigvalsh(A).min() > 0
    R = P.rigid_body_modes(e)
    gx = e.grid[0]
    away = np.repeat((np.arange(e.n // 3) % gx) >= 1, 3)
    assert np.abs((A @ R)[away]).max() < 1e-12 * np.abs(A).max()
    assert np.abs((A @ R)[~away]).max() > 1e-3
