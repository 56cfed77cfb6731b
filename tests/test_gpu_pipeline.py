"""GPU: batches in flight give bitwise the serial results.

The pipeline factors later batches (one or several side by side, each on
its own stream) while batch k is solved on another; the arithmetic of each
batch is unchanged, so every solution must equal the one from factor_batch +
solve_batch, and match the oracle."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def helm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_10762_amd import helm as h
    h.lib()
    return h


@pytest.mark.parametrize("precision,factor_streams", [("fp32_ir", 1), ("fp64", 1), ("fp32_ir", 2), ("fp64", 3)])
def test_pipeline_equals_serial(helm, precision, factor_streams):
    from paper_2301_10762_amd.pipeline import Batch, Pipeline
    rng = np.random.default_rng(5)
    nx, nz, hx, hz = 70, 37, 0.03, 0.03
    g = helm.Grid(nx, nz, hx, hz)
    batches, refs = [], []
    for k in range(4):
        ms = [torch.as_tensor(0.2 + 0.05 * rng.random(nx * nz), device="cuda") for _ in range(3)]
        ws = [2 * np.pi * (2.0 + 0.5 * q + 0.1 * k) for q in range(3)]
        Bs = [torch.as_tensor(rng.standard_normal((5, nx * nz)) + 1j * rng.standard_normal((5, nx * nz)),
                              device="cuda") for _ in range(3)]
        batches.append(Batch([g] * 3, ms, ws, Bs, precision, 1e-10))
        Fs = helm.factor_batch([g] * 3, ms, ws, precision)
        Xs, infos = helm.solve_batch(Fs, Bs, tol=1e-10)
        for F in Fs:
            F.close()
        refs.append([X.cpu().numpy() for X in Xs])
    print(f"pipeline {precision}, {factor_streams} factor streams: 4 batches of 3 systems {nx}x{nz}", flush=True)
    out = Pipeline(factor_streams).run(batches)
    og = oracle.Grid(nx, nz, hx, hz)
    for k, (Xs, infos) in enumerate(out):
        for q, (X, info) in enumerate(zip(Xs, infos)):
            assert info.max_relres <= 1e-10
            Xh = X.cpu().numpy()
            assert np.array_equal(Xh, refs[k][q])
        if k == 0:
            b = batches[0]
            Fo = oracle.Factor(og, b.ms[0].cpu().numpy(), b.omegas[0])
            Xo = Fo.solve(b.Bs[0].cpu().numpy())
            Fo.close()
            assert np.linalg.norm(Xs[0].cpu().numpy() - Xo) / np.linalg.norm(Xo) < 1e-9
