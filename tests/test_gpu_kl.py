"""GPU parity of the Karhunen-Loeve random fields: solves with
HENRY_FIELD_KL41 against the oracle run on the oracle's own KL fields (its
own basis and field map), and the 41-coefficient adjoint gradient against
the oracle's adjoint composed with its field map.  Bars as for the
closed-form fields: 1e-8 (FP64 inner path), 1e-5 (mixed)."""
import numpy as np
import pytest

import henry_inputs as hi
import oracle
import paper_2302_07804_amd as hm
from oracle import kl

pytestmark = pytest.mark.gpu

GRIDS = [(16, 8), (32, 16), (64, 32)]


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
    for nx, ny in GRIDS:
        c.set_kl(nx, ny, kl.CORR_LEN, kl.SIGMA_PHI, kl.SIGMA_LOGK)
    yield c
    c.close()


@pytest.fixture(scope="module")
def bases():
    return {nx: kl.basis(nx, ny) for nx, ny in GRIDS}


def dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("prec,bar", [(hm.PREC_FP64, 1e-8), (hm.PREC_MIXED, 1e-5)])
def test_kl_solves_match_oracle(torch_cuda, ctx, bases, prec, bar):
    torch = torch_cuda
    solves = [(16, 8, 40), (32, 16, 80), (32, 16, 80), (64, 32, 60), (16, 8, 40)]
    xi = hm.henry_sample_xi_kl(hi.SEED, 1, 0, len(solves))
    opts = hm.make_opts(prec=prec, tol=1e-10, max_outer=60)
    print(f"KL solve parity prec={prec} solves={solves}", flush=True)
    out = hm.solve(ctx, solves, xi=dev(torch, xi), opts=opts)
    torch.cuda.synchronize()
    cs = hm.unpack(out["c"], solves)
    st = out["status"].cpu().numpy()
    q = out["qoi"].cpu().numpy()
    for k, s in enumerate(solves):
        assert st[k] == hm.STATUS_OK
        lam, modes = bases[s[0]]
        Q, c = kl.solve_kl(hi.PHYS, s[0], s[1], s[2], xi[k], lam, modes)
        c_gpu = cs[k].cpu().numpy()
        assert np.abs(c_gpu - c).max() <= bar * np.abs(c).max(), k
        assert abs(q[k] - Q) <= bar * abs(Q), k


def test_kl_solve_requires_a_basis(torch_cuda, ctx):
    torch = torch_cuda
    xi = dev(torch, hm.henry_sample_xi_kl(0, 0, 0, 1))
    with pytest.raises(hm.HenryError) as e:
        hm.solve(ctx, [(128, 64, 10)], xi=xi)
    assert e.value.code == hm.HENRY_EINVAL


@pytest.mark.parametrize("prec", [hm.PREC_FP64, hm.PREC_MIXED])
def test_kl_adjoint_matches_oracle(torch_cuda, ctx, bases, prec):
    torch = torch_cuda
    solves = [(16, 8, 30), (32, 16, 40)]
    xi = hm.henry_sample_xi_kl(hi.SEED, 2, 3, len(solves))
    opts = hm.make_opts(prec=prec, tol=1e-11, max_outer=80)
    print(f"KL adjoint parity prec={prec} solves={solves}", flush=True)
    out = hm.adjoint(ctx, solves, xi=dev(torch, xi), opts=opts, ckpt_every=7, adj_tol=1e-12, adj_max_it=80)
    torch.cuda.synchronize()
    assert list(out["status"].cpu().numpy()) == [0, 0]
    g_gpu = out["dq_dxi"].cpu().numpy()
    for k, s in enumerate(solves):
        lam, modes = bases[s[0]]
        Q, g = kl.adjoint_kl(hi.PHYS, s[2], xi[k], lam, modes)
        assert abs(out["qoi"][k].item() - Q) <= 1e-9 * Q
        assert np.abs(g_gpu[k] - g).max() <= 1e-6 * np.abs(g).max(), (k, g_gpu[k], g)
