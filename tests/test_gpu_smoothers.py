"""Per-kernel parity of the multigrid smoothers (the relaxations every
V-cycle of the solves runs): henry_level_smooth against the oracle's
red-black Gauss-Seidel on the pressure operator and its zebra x- and
y-line relaxation on the upwind transport operator, with random
coefficients, after 1 and 3 sweeps, on grids from 2x1 to 256x128.  The
FP64 path agrees to 1e-14 of max |x| (4.5e-16 measured), the FP32 path (the kernels inside the
mixed-precision solves) to 1e-6 (2.3e-7 measured)."""
import numpy as np
import pytest

import oracle
import paper_2302_07804_amd as hm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible for a gpu-marked test")
    hm.lib()
    return torch


@pytest.fixture(scope="module")
def ctx(torch_cuda):
    import henry_inputs as hi
    c = hm.Context(hi.PHYS, 0)
    yield c
    c.close()


def dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64).ravel(), device="cuda")


@pytest.mark.parametrize("nx,ny", [(2, 1), (16, 8), (64, 32), (256, 128)])
@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("prec,bar", [(hm.PREC_FP64, 1e-14), (hm.PREC_MIXED, 1e-6)])
def test_level_smoother_matches_oracle(torch_cuda, ctx, nx, ny, kind, prec, bar):
    torch = torch_cuda
    rng = np.random.default_rng(100 * nx + 10 * kind + prec)
    n = nx * ny
    b = rng.normal(size=(ny, nx))
    x0 = rng.normal(size=(ny, nx))
    if kind == 0:
        te, tn = rng.uniform(0.5, 1.5, (ny, nx)), rng.uniform(0.5, 1.5, (ny, nx))
        coef = np.concatenate([te.ravel(), tn.ravel()])
        A = oracle.pressure_operator(te, tn)
    else:
        parts = (rng.uniform(0.1, 1.0, (ny, nx)), rng.uniform(-1, 1, (ny, nx)), rng.uniform(-1, 1, (ny, nx)),
                 rng.uniform(0.05, 0.5, (ny, nx)), rng.uniform(0.05, 0.5, (ny, nx)), rng.uniform(-1, 1, ny),
                 rng.uniform(0.05, 0.5, ny), rng.uniform(0.05, 0.5, ny), rng.uniform(0.0, 1.0, ny))
        coef = np.concatenate([p.ravel() for p in parts])
        A = oracle.transport_operator(*parts)
    sweeps = (1, 3) if n <= 2048 else (1,)
    for sw in sweeps:
        x = dev(torch, x0)
        hm.henry_level_smooth(ctx, nx, ny, kind, prec, sw, dev(torch, coef), dev(torch, b), x)
        torch.cuda.synchronize()
        got = x.cpu().numpy().reshape(ny, nx)
        if kind == 0:
            want = oracle.gauss_seidel_rb(A, b, x0, nx, ny, sw)
        else:
            want = oracle.zebra_lines(A, b, x0, nx, ny, sw, ylines=(kind == 2 and ny > 1))
        err = np.abs(got - want).max() / np.abs(want).max()
        print(f"{nx}x{ny} kind {kind} prec {prec} sweeps {sw}: {err:.2e}")
        assert err <= bar, (sw, err)


def test_level_smoother_rejects_bad_arguments(torch_cuda, ctx):
    torch = torch_cuda
    z = dev(torch, np.zeros(16 * 8 * 5 + 4 * 8))
    for args in ((16, 8, 3, hm.PREC_MIXED, 1), (16, 9, 0, hm.PREC_MIXED, 1), (16, 8, 0, 7, 1),
                 (16, 8, 0, hm.PREC_MIXED, -1)):
        with pytest.raises(hm.HenryError):
            hm.henry_level_smooth(ctx, *args, z, z, z)
