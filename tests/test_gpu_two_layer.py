"""The paper's own random input model on the GPU (HENRY_FIELD_TWOLAYER3:
two porosity layers, Kozeny-Carman permeability, recharge +-50 %; Sec. 4
eq:poro_2levels, eq:poro_2levels_C, Sec. 2.2 e_perm_Kozeny_Carman) with
Table 1's constants and T = 6016 s, against the oracle's
fields_two_layer: the residual element by element (1e-13 of max |R|), whole
solves on 16x8/50 and on the paper's coarsest grid 32x16/188 (FP64 path
1e-8, mixed 1e-5 in c and Q), and the adjoint's dQ/dxi through the model's
derivatives (1e-6)."""
import numpy as np
import pytest

import henry_inputs as hi
import oracle
import paper_2302_07804_amd as hm
from test_gpu_residual import check, packed, states

pytestmark = pytest.mark.gpu

PH = hi.PHYS_TABLE1
XI = [[-0.5898, -0.7257, -0.9616], [0.9, 0.8, -0.3], [-1.0, 1.0, 1.0], [0.0, 0.0, 0.0]]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible for a gpu-marked test")
    hm.lib()
    return torch


@pytest.fixture(scope="module")
def ctx(torch_cuda):
    c = hm.Context(PH, 0)
    yield c
    c.close()


def test_two_layer_residual(torch_cuda, ctx):
    torch = torch_cuda
    solves = [(8, 4, 3), (32, 16, 188), (128, 64, 752)]
    xi = np.array([XI[0], XI[1], XI[2]])
    st = states(solves, 5)
    rp, rc = hm.residual(ctx, solves, packed(torch, [s[0] for s in st]), packed(torch, [s[1] for s in st]),
                         packed(torch, [s[2] for s in st]), xi=torch.tensor(xi, dtype=torch.float64, device="cuda"),
                         model="two_layer")
    torch.cuda.synchronize()
    refs = []
    for (nx, ny, r), x, (p, c, cn) in zip(solves, xi, st):
        phi, K, q = oracle.fields_two_layer(PH, nx, ny, x)
        refs.append(oracle.residual(PH, r, phi, K, q, p, c, cn))
    worst = check(rp.cpu().numpy(), rc.cpu().numpy(), solves, refs)
    print(f"residual, two-layer fields: worst rel err {worst:.3e}")


@pytest.mark.parametrize("prec,bar", [(hm.PREC_FP64, 1e-8), (hm.PREC_MIXED, 1e-5)])
def test_two_layer_solves_match_oracle(torch_cuda, ctx, prec, bar):
    torch = torch_cuda
    grids = [(16, 8, 50), (32, 16, 188)]
    jobs = [(g, x) for g in grids for x in XI]
    xi = torch.tensor([x for _, x in jobs], dtype=torch.float64, device="cuda")
    out = hm.solve(ctx, [g for g, _ in jobs], xi=xi, opts=hm.make_opts(prec=prec, tol=1e-10, max_outer=60),
                   model="two_layer")
    torch.cuda.synchronize()
    assert (out["status"].cpu().numpy() == 0).all()
    refs = oracle.solve_many(PH, [(*g, np.array(x), "two_layer") for g, x in jobs])
    c = out["c"].cpu().numpy()
    q = out["qoi"].cpu().numpy()
    off, worst = 0, 0.0
    for k, ((nx, ny, _), _) in enumerate(jobs):
        cr = refs[k]["c"].ravel()
        err = np.abs(c[off:off + nx * ny] - cr).max() / np.abs(cr).max()
        off += nx * ny
        worst = max(worst, err)
        assert err <= bar, (k, err)
        assert abs(q[k] - refs[k]["qoi"]) <= bar * abs(refs[k]["qoi"]), k
    print(f"two-layer solves, prec {prec}: worst rel c err {worst:.3e}")


def test_two_layer_at_zero_is_the_homogeneous_medium(torch_cuda, ctx):
    """At xi = 0 the two-layer model and the closed-form fields both give
    phi0, k0 and q_in (K up to one rounding of the Kozeny-Carman scale)."""
    torch = torch_cuda
    xi = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    opts = hm.make_opts(prec=hm.PREC_FP64, tol=1e-11, max_outer=60)
    a = hm.solve(ctx, [(32, 16, 188)], xi=xi, opts=opts, model="two_layer")
    b = hm.solve(ctx, [(32, 16, 188)], xi=xi, opts=opts)
    torch.cuda.synchronize()
    assert torch.allclose(a["c"], b["c"], rtol=0, atol=1e-10)
    assert abs(a["qoi"].item() - b["qoi"].item()) <= 1e-10 * abs(b["qoi"].item())


def test_two_layer_adjoint_matches_oracle(torch_cuda, ctx):
    torch = torch_cuda
    nx, ny, r = 16, 8, 30
    xi = np.array(XI[:3])
    out = hm.adjoint(ctx, [(nx, ny, r)] * 3, xi=torch.tensor(xi, dtype=torch.float64, device="cuda"),
                     opts=hm.make_opts(prec=hm.PREC_FP64, tol=1e-11, max_outer=80), ckpt_every=7, adj_tol=1e-12,
                     adj_max_it=80, model="two_layer")
    torch.cuda.synchronize()
    assert list(out["status"].cpu().numpy()) == [0, 0, 0]
    gx = out["dq_dxi"].cpu().numpy()
    glk = out["dq_dlogk"].cpu().numpy().reshape(3, ny, nx)
    for s in range(3):
        Q, g, glogk = oracle.adjoint_xi(PH, nx, ny, r, xi[s], model="two_layer")
        assert abs(out["qoi"][s].item() - Q) <= 1e-9 * Q
        np.testing.assert_allclose(gx[s], g, rtol=1e-6, atol=1e-9 * np.abs(g).max())
        assert np.abs(glk[s] - glogk).max() <= 1e-6 * np.abs(glogk).max()
