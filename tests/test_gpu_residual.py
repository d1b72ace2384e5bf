"""Per-kernel parity of the FP64 nonlinear residual (the quantity whose
scaled max norm ends every implicit step): henry_residual_batch against the
oracle's residual of the same discrete equations, element by element, at
perturbed states away from any solution (so R is of the size of the face
fluxes and the comparison is not swamped by cancellation).  Both sides are
FP64 and add the same face terms, possibly in another order: the bar is
1e-13 of the largest |R| of each solve and equation."""
import numpy as np
import pytest

import henry_inputs as hi
import oracle
import paper_2302_07804_amd as hm

pytestmark = pytest.mark.gpu

BAR = 1e-13


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible for a gpu-marked test")
    hm.lib()
    return torch


@pytest.fixture(scope="module")
def ctx(torch_cuda):
    c = hm.Context(hi.PHYS, 0)
    yield c
    c.close()


def states(solves, seed):
    """Smooth salt wedge plus noise, a nearby previous level, hydrostatic
    pressure plus noise: [ny][nx] arrays per solve."""
    rng = np.random.default_rng(seed)
    out = []
    for nx, ny, _ in solves:
        x = (np.arange(nx) + 0.5) / ny
        y = -1.0 + (np.arange(ny) + 0.5) / ny
        X, Y = np.meshgrid(x, y)
        c = np.clip(0.5 * (1 + np.tanh(4 * (X - 1.4) - 3 * Y - 1)) + 0.05 * rng.standard_normal((ny, nx)), 0, 1)
        cn = np.clip(c - 0.02 * rng.random((ny, nx)), 0, 1)
        rho = hi.PHYS["rho0"] + (hi.PHYS["rho1"] - hi.PHYS["rho0"]) * c
        p = -rho * hi.PHYS["g"] * Y + 50.0 * rng.standard_normal((ny, nx))
        out.append((p, c, cn))
    return out


def packed(torch, arrs):
    return torch.tensor(np.concatenate([a.ravel() for a in arrs]), dtype=torch.float64, device="cuda")


def check(rp, rc, solves, refs):
    off = 0
    worst = 0.0
    for (nx, ny, _), (Rp, Rc) in zip(solves, refs):
        n = nx * ny
        gp = rp[off:off + n].reshape(ny, nx)
        gc = rc[off:off + n].reshape(ny, nx)
        off += n
        for g, r in ((gp, Rp), (gc, Rc)):
            err = np.abs(g - r).max() / np.abs(r).max()
            worst = max(worst, err)
            assert err <= BAR, f"{nx}x{ny}: rel err {err:.3e}"
    return worst


def test_residual_closed_form_fields(torch_cuda, ctx):
    torch = torch_cuda
    solves = [(2, 1, 3), (16, 8, 50), (64, 32, 200), (128, 64, 37), (256, 128, 800)]
    xi = hm.henry_sample_xi(0, 13, 0, len(solves), 3)
    st = states(solves, 1)
    rp, rc = hm.residual(ctx, solves, packed(torch, [s[0] for s in st]), packed(torch, [s[1] for s in st]),
                         packed(torch, [s[2] for s in st]),
                         xi=torch.tensor(xi, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    refs = []
    for (nx, ny, r), x, (p, c, cn) in zip(solves, xi, st):
        phi, K, q = oracle.fields_closed(hi.PHYS, nx, ny, x)
        refs.append(oracle.residual(hi.PHYS, r, phi, K, q, p, c, cn))
    worst = check(rp.cpu().numpy(), rc.cpu().numpy(), solves, refs)
    print(f"residual, closed-form fields: worst rel err {worst:.3e}")


def test_residual_explicit_fields(torch_cuda, ctx):
    torch = torch_cuda
    solves = [(32, 16, 100), (64, 32, 10)]
    rng = np.random.default_rng(2)
    phis, logks, qs = [], [], []
    for nx, ny, _ in solves:
        phis.append(0.35 * (1 + 0.2 * rng.uniform(-1, 1, (ny, nx))))
        logks.append(np.log(hi.PHYS["k0"]) + 0.6 * rng.uniform(-1, 1, (ny, nx)))
        qs.append(hi.PHYS["q_in"] * (1 + 0.2 * rng.uniform(-1, 1)))
    st = states(solves, 3)
    rp, rc = hm.residual(ctx, solves, packed(torch, [s[0] for s in st]), packed(torch, [s[1] for s in st]),
                         packed(torch, [s[2] for s in st]), phi=packed(torch, phis), logk=packed(torch, logks),
                         qin=torch.tensor(qs, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    refs = [oracle.residual(hi.PHYS, r, phi, np.exp(lk), q, p, c, cn)
            for (nx, ny, r), phi, lk, q, (p, c, cn) in zip(solves, phis, logks, qs, st)]
    worst = check(rp.cpu().numpy(), rc.cpu().numpy(), solves, refs)
    print(f"residual, explicit fields: worst rel err {worst:.3e}")


def test_residual_vanishes_after_a_converged_step(torch_cuda):
    """One FP64 step from a given salt field c0 (tau = T/200 of the
    workload's horizon), converged to tol: the entry point's residual at the
    returned state, with c^n = c0, is within tol in the solver's scaled max
    norm (both evaluate the same equations)."""
    torch = torch_cuda
    nx, ny = 64, 32
    ph = dict(hi.PHYS, T=hi.PHYS["T"] / 200)
    c = hm.Context(ph, 0)
    x = hm.henry_sample_xi(0, 14, 0, 1, 3)
    xi = torch.tensor(x, dtype=torch.float64, device="cuda")
    c0 = states([(nx, ny, 1)], 4)[0][1]
    c0_d = torch.tensor(c0.ravel(), dtype=torch.float64, device="cuda")
    tol = 1e-10
    out = hm.solve(c, [(nx, ny, 1)], xi=xi, c0=c0_d, opts=hm.make_opts(prec=hm.PREC_FP64, tol=tol, max_outer=80),
                   want_p=True)
    torch.cuda.synchronize()
    assert out["status"].item() == hm.STATUS_OK
    rp, rc = hm.residual(c, [(nx, ny, 1)], out["p"], out["c"], c0_d, xi=xi)
    torch.cuda.synchronize()
    phi, K, q = oracle.fields_closed(ph, nx, ny, x[0])
    sc = ph["T"] / ((1.0 / ny) ** 2 * phi * ph["rho0"])
    rp = rp.cpu().numpy().reshape(ny, nx)
    rc = rc.cpu().numpy().reshape(ny, nx)
    assert np.abs(rp * sc).max() <= tol and np.abs(rc * sc).max() <= tol
    # and the oracle agrees at that state
    Rp, Rc = oracle.residual(ph, 1, phi, K, q, out["p"].cpu().numpy().reshape(ny, nx),
                             out["c"].cpu().numpy().reshape(ny, nx), c0)
    assert np.abs(Rp * sc).max() <= 2 * tol and np.abs(Rc * sc).max() <= 2 * tol
    c.close()
