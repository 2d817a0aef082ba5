"""The allocation-free apply (sgf_apply_noalloc): its work vectors live in
the library's static device scratch instead of the handle's buffers.  Its
result must equal sgf_apply's bit for bit (same kernels, same order), on two
calls in a row, the second with a smaller input, through the C ABI; a call
whose work vectors do not fit the scratch is refused with an error."""
import numpy as np
import pytest

from sgf_inputs import problems as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

sgf = pytest.importorskip("paper_1907_03406_amd.sgf")


def _columns(p, k, seed):
    return torch.from_numpy(np.stack([P.random_rhs(seed, p.n, j) for j in range(k)], axis=0)).cuda()


def _solver(p, **kw):
    s = sgf.Solver.from_problem(p, **kw)
    s.factorize(torch.from_numpy(p.data).cuda())
    torch.cuda.synchronize()
    return s


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_apply_equals_apply_on_two_calls(prec):
    pr = sgf.FP32 if prec == "fp32" else sgf.FP64
    big = P.poisson_fd((160, 150), P.gaussian_field_fourier(0, 2))
    small = P.poisson_fd((61, 58), P.gaussian_field_fourier(1, 2))
    calls = [(big, 16, 2, 4), (small, 8, 2, 1)]     # second call: smaller problem, fewer columns
    for step, (p, leaf, q, k) in enumerate(calls):
        s = _solver(p, q=q, leaf=leaf, precision=pr)
        r = _columns(p, k, 50 + step)
        z_ref = torch.full_like(r, float("nan"))
        s.apply(r.T, z_ref.T)
        torch.cuda.synchronize()
        z = torch.full_like(r, float("nan"))
        s.apply_noalloc(r.T, z.T)
        torch.cuda.synchronize()
        assert torch.equal(z, z_ref), f"call {step}: differs from sgf_apply"
        s.close()


def test_noalloc_apply_on_tiled_levels_and_repeat():
    """Tiled levels (their front work vectors) and a compressed-separator
    vector per level come out of the scratch too; a repeated call gives the
    same bits."""
    p = P.poisson_fd((17, 16, 15), P.blocky_log_field(0, 3))
    s = _solver(p, q=1, leaf=4, tiled_min_rows=0)
    r = _columns(p, 3, 60)
    z_ref = torch.empty_like(r)
    s.apply(r.T, z_ref.T)
    for _ in range(2):
        z = torch.full_like(r, float("nan"))
        s.apply_noalloc(r.T, z.T)
        torch.cuda.synchronize()
        assert torch.equal(z, z_ref)


def test_noalloc_apply_refuses_what_does_not_fit():
    p = P.poisson_fd((400, 400), P.gaussian_field_fourier(2, 2))
    s = _solver(p, q=1, leaf=16, precision=sgf.FP64)
    cols = sgf.NOALLOC_SCRATCH_BYTES // (8 * p.n) + 1   # the permuted vector alone overflows
    r = _columns(p, cols, 70)
    z = torch.zeros_like(r)
    with pytest.raises(sgf.SgfError) as ei:
        s.apply_noalloc(r.T, z.T)
    assert ei.value.code == sgf.SGF_EINVAL and "scratch" in str(ei.value)
    # a call that fits still works after the refusal
    z1 = torch.empty_like(r[:1])
    s.apply_noalloc(r[:1].T, z1.T)
    z2 = torch.empty_like(r[:1])
    s.apply(r[:1].T, z2.T)
    torch.cuda.synchronize()
    assert torch.equal(z1, z2)
