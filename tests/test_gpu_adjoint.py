"""GPU discrete adjoint: against the oracle's adjoint (16x8, 32x16) and
against central finite differences of the GPU forward map (128x64, 400
steps, h = 1e-6), through the C ABI and through torch.autograd."""
import numpy as np
import pytest

import henry_inputs as hi
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
    c = hm.Context(hi.PHYS, 0)
    yield c
    c.close()


def dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("grid,prec", [((16, 8, 50), hm.PREC_FP64), ((32, 16, 100), hm.PREC_FP64),
                                       ((16, 8, 50), hm.PREC_MIXED)])
def test_adjoint_matches_oracle_adjoint(torch_cuda, ctx, grid, prec):
    torch = torch_cuda
    nx, ny, r = grid
    xi = hm.henry_sample_xi(0, 3, 0, 2, 3)
    opts = hm.make_opts(prec=prec, tol=1e-11, max_outer=80)
    out = hm.adjoint(ctx, [grid] * 2, xi=dev(torch, xi), opts=opts, ckpt_every=7, adj_tol=1e-12, adj_max_it=80)
    torch.cuda.synchronize()
    assert list(out["status"].cpu().numpy()) == [0, 0]
    gx = out["dq_dxi"].cpu().numpy()
    glk = out["dq_dlogk"].cpu().numpy().reshape(2, ny, nx)
    gph = out["dq_dphi"].cpu().numpy().reshape(2, ny, nx)
    for s in range(2):
        Q, g, glogk = oracle.adjoint_xi(hi.PHYS, nx, ny, r, xi[s])
        phi, K, q = oracle.fields_closed(hi.PHYS, nx, ny, xi[s])
        _, gphi, gK, gq = oracle.adjoint(hi.PHYS, r, phi, K, q)
        assert abs(out["qoi"][s].item() - Q) <= 1e-9 * Q
        np.testing.assert_allclose(gx[s], g, rtol=1e-6, atol=1e-9 * np.abs(g).max())
        assert np.abs(glk[s] - glogk).max() <= 1e-6 * np.abs(glogk).max()
        assert np.abs(gph[s] - gphi).max() <= 1e-6 * np.abs(gphi).max()
        assert abs(out["dq_dq"][s].item() - gq) <= 1e-6 * abs(gq)


def test_checkpoint_interval_does_not_change_gradients(torch_cuda, ctx):
    torch = torch_cuda
    grid = (16, 8, 50)
    xi = dev(torch, hm.henry_sample_xi(0, 3, 5, 1, 3))
    opts = hm.make_opts(prec=hm.PREC_MIXED, tol=1e-10, max_outer=60)
    a = hm.adjoint(ctx, [grid], xi=xi, opts=opts, ckpt_every=1)
    b = hm.adjoint(ctx, [grid], xi=xi, opts=opts, ckpt_every=13)
    c = hm.adjoint(ctx, [grid], xi=xi, opts=opts, ckpt_every=50)
    torch.cuda.synchronize()
    for k in ("dq_dxi", "dq_dlogk", "dq_dphi", "dq_dq", "qoi"):
        assert torch.equal(a[k], b[k]) and torch.equal(a[k], c[k]), k


@pytest.mark.parametrize("prec", [hm.PREC_MIXED, hm.PREC_FP64])
def test_adjoint_cluster_sizes_are_bitwise_equal(torch_cuda, ctx, prec):
    """The adjoint of a solve shared by 2, 4 or 8 workgroups: every cell and
    line computed with the same arithmetic, norms as maxima, the gradient
    sums taken by the leader in one-workgroup order, so Q, dQ/dxi, dQ/dlog K,
    dQ/dphi, dQ/dq, status and iteration counts equal those of one
    workgroup bitwise (checkpoint segments included)."""
    torch = torch_cuda
    solves = [(256, 128, 160), (128, 64, 40)]
    xi = dev(torch, hm.henry_sample_xi(0, 12, 0, len(solves), 3))
    kw = dict(ckpt_every=30, adj_tol=1e-9, adj_max_it=60)
    ref = hm.adjoint(ctx, solves, xi=xi, opts=hm.make_opts(prec=prec, tol=1e-9, max_outer=60, cluster=1), **kw)
    torch.cuda.synchronize()
    assert list(ref["status"].cpu().numpy()) == [0, 0]
    for K in (2, 4, 8):
        out = hm.adjoint(ctx, solves, xi=xi, opts=hm.make_opts(prec=prec, tol=1e-9, max_outer=60, cluster=K), **kw)
        torch.cuda.synchronize()
        for key in ("qoi", "dq_dxi", "dq_dlogk", "dq_dphi", "dq_dq", "status", "iters"):
            assert torch.equal(out[key], ref[key]), (K, key)


@pytest.mark.parametrize("prec", [hm.PREC_FP64, hm.PREC_MIXED])
def test_adjoint_vs_central_differences_128x64(torch_cuda, ctx, prec):
    """128x64 grid, 400 steps, checkpoints every 20, two samples: dQ/dxi and
    a random direction in per-cell log K against central differences of the
    forward map (h = 1e-6), relative 1e-4."""
    torch = torch_cuda
    nx, ny, r = 128, 64, 400
    ns = 2
    xi = hm.henry_sample_xi(0, 3, 0, ns, 3)
    fwd_opts = hm.make_opts(prec=hm.PREC_FP64, tol=1e-11, max_outer=100)
    adj = hm.adjoint(ctx, [(nx, ny, r)] * ns, xi=dev(torch, xi),
                     opts=hm.make_opts(prec=prec, tol=1e-11, max_outer=100), ckpt_every=20, adj_tol=1e-11,
                     adj_max_it=100)
    torch.cuda.synchronize()
    gx = adj["dq_dxi"].cpu().numpy()
    hfd = 1e-6
    pts = []
    for s in range(ns):
        for d in range(3):
            e = np.zeros(3); e[d] = hfd
            pts += [xi[s] + e, xi[s] - e]
    out = hm.solve(ctx, [(nx, ny, r)] * len(pts), xi=dev(torch, np.array(pts)), opts=fwd_opts)
    torch.cuda.synchronize()
    q = out["qoi"].cpu().numpy().reshape(ns, 3, 2)
    fd = (q[..., 0] - q[..., 1]) / (2 * hfd)
    for s in range(ns):
        assert np.abs(fd[s] - gx[s]).max() <= 1e-4 * np.abs(gx[s]).max(), (fd[s], gx[s])
    # one random direction in per-cell log K (explicit fields)
    phi, K, qv = oracle.fields_closed(hi.PHYS, nx, ny, xi[0])
    v = np.random.default_rng(2).normal(size=(ny, nx))
    logk = np.log(K)
    gl = adj["dq_dlogk"].cpu().numpy()[: nx * ny].reshape(ny, nx)
    pair = hm.solve(ctx, [(nx, ny, r)] * 2, phi=dev(torch, np.concatenate([phi.ravel()] * 2)),
                    logk=dev(torch, np.concatenate([(logk + hfd * v).ravel(), (logk - hfd * v).ravel()])),
                    qin=dev(torch, [qv, qv]), opts=fwd_opts)
    torch.cuda.synchronize()
    qq = pair["qoi"].cpu().numpy()
    fdv = (qq[0] - qq[1]) / (2 * hfd)
    assert abs(fdv - (gl * v).sum()) <= 1e-4 * np.abs(gl * v).sum()


def test_autograd_function_gives_the_adjoint_gradient(torch_cuda, ctx):
    torch = torch_cuda
    grid = (16, 8, 50)
    xi = dev(torch, hm.henry_sample_xi(0, 3, 0, 3, 3)).requires_grad_(True)
    opts = hm.make_opts(prec=hm.PREC_MIXED, tol=1e-10, max_outer=60)
    Q = hm.HenryQoI.apply(xi, ctx, [grid] * 3, opts, 10, 1e-10)
    w = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device="cuda")
    (Q * w).sum().backward()
    ref = hm.adjoint(ctx, [grid] * 3, xi=xi.detach(), opts=opts, ckpt_every=10)
    torch.cuda.synchronize()
    assert torch.allclose(xi.grad, w[:, None] * ref["dq_dxi"], rtol=1e-12, atol=0)
