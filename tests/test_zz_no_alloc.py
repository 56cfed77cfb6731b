"""GPU: the allocation-free solve (helm_solve_noalloc) against helm_solve.

Both run the same kernels in the same order; only the scratch memory
differs (the library's fixed per-device region instead of its block cache),
so the solutions must be bitwise equal.  Two calls in a row, the second on a
smaller input (fewer columns, a smaller grid), show that what the first call
left in the region does not leak into the second.  A solve whose scratch
would exceed the region is rejected before any launch, and the caller's
output is left untouched.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def helm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_10762_amd import helm as h
    h.lib()
    return h


def _system(helm, nx, nz, S, seed, precision):
    rng = np.random.default_rng(seed)
    h = 0.025
    m = torch.as_tensor(1.0 / (1.5 + 3.0 * rng.random(nx * nz)) ** 2, device="cuda")
    omega = 2 * np.pi * 1.5 / (8.0 * h)
    F = helm.factor(helm.Grid(nx, nz, h, h), m, omega, precision)
    B = torch.as_tensor(rng.standard_normal((S, nx * nz)) + 1j * rng.standard_normal((S, nx * nz)), device="cuda")
    return F, B


@pytest.mark.parametrize("precision", ["fp32_ir", "fp64"])
def test_noalloc_equals_solve_twice_shrinking(helm, precision):
    # (nx, nz, S): several tiles with tails, then a smaller grid and fewer columns
    for k, (nx, nz, S) in enumerate([(130, 47, 37), (40, 23, 5)]):
        print(f"noalloc {precision} call {k}: {nx}x{nz}, {S} columns", flush=True)
        F, B = _system(helm, nx, nz, S, 10 * k + 1, precision)
        X_ref, info_ref = F.solve(B, tol=1e-10)
        X = torch.full_like(B, complex(np.nan, np.nan))
        info = helm.solve_noalloc(F, B, X, tol=1e-10)
        torch.cuda.synchronize()
        F.close()
        assert torch.equal(X, X_ref), (precision, k)
        assert info.max_relres == info_ref.max_relres and info.ir_iters == info_ref.ir_iters
        assert info.max_relres <= 1e-10


def test_noalloc_rejects_scratch_beyond_region(helm):
    """201^2 with complex128 factors and 256 columns: without a tolerance the
    solve needs only the sweep buffers and runs (equal to helm_solve); with a
    tolerance its worst case (a complex128 residual and correction, 2 x 165 MB)
    exceeds the 256 MiB region and is rejected, X untouched."""
    F, B = _system(helm, 201, 201, 256, 7, "fp64")
    X_ref, _ = F.solve(B)
    X = torch.zeros_like(B)
    helm.solve_noalloc(F, B, X)
    torch.cuda.synchronize()
    assert torch.equal(X, X_ref)
    X.zero_()
    with pytest.raises(helm.HelmError) as e:
        helm.solve_noalloc(F, B, X, tol=1e-10)
    assert e.value.code == helm.EINVAL and "allocation-free limit" in str(e.value)
    torch.cuda.synchronize()
    assert not bool(X.abs().max())
    F.close()
