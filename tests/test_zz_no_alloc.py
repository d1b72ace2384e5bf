"""The allocation-free entry point henry_solve_batch_static, for callers that
cannot allocate device memory: the same solves as henry_solve_batch with the
solves' state in the library's static device buffer instead of a caller
workspace.  Two calls in a row, the second smaller than the first (the
buffer keeps the first call's contents), each compared with
henry_solve_batch on the same inputs: the kernels and their arithmetic are
the same, so c, p, Q, the status and the iteration counts are bitwise
equal.  Batches beyond the buffer and options that would allocate (graph
chunks, profiling events) are rejected before anything is launched."""
import numpy as np
import pytest

import henry_inputs as hi
import paper_2302_07804_amd as hm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible for a gpu-marked test")
    hm.lib()
    return torch


def xi_for(solves, level):
    return hm.henry_sample_xi(hi.SEED, level, 0, len(solves), 3)


def static_solve(torch, ctx, solves, xi, opts):
    dev = torch.device("cuda", ctx.device)
    n = len(solves)
    cells = sum(s[0] * s[1] for s in solves)
    out = dict(c=torch.full((cells,), -1.0, dtype=torch.float64, device=dev),
               p=torch.full((cells,), -1.0, dtype=torch.float64, device=dev),
               qoi=torch.full((n,), -1.0, dtype=torch.float64, device=dev),
               status=torch.full((n,), -7, dtype=torch.int32, device=dev),
               iters=torch.full((n,), -7, dtype=torch.int32, device=dev))
    hm.henry_solve_batch_static(ctx, solves, hm.FIELD_CLOSED3, xi=xi, opts=opts, c_out=out["c"], p_out=out["p"],
                                qoi_out=out["qoi"], status=out["status"], iters=out["iters"])
    return out


def check_same(torch, ctx, solves, level, prec, tol):
    xi = torch.tensor(xi_for(solves, level), dtype=torch.float64, device="cuda")
    opts = hm.make_opts(prec=prec, tol=tol, max_outer=60)
    need = hm.henry_workspace_bytes(solves, opts)
    assert need <= hm.STATIC_SCRATCH_BYTES
    print(f"static vs workspace: {len(solves)} solves, {need / 2**20:.1f} MiB of state", flush=True)
    st = static_solve(torch, ctx, solves, xi, opts)
    ref = hm.solve(ctx, solves, xi=xi, opts=opts, want_p=True)
    torch.cuda.synchronize()
    assert (ref["status"].cpu().numpy() == hm.STATUS_OK).all()
    for k in ("c", "p", "qoi", "status", "iters"):
        a, b = st[k].cpu().numpy(), ref[k].cpu().numpy()
        assert np.array_equal(a, b), (k, np.abs(a.astype(np.float64) - b).max())


def test_static_entry_point_matches_the_workspace_entry_point_twice(torch_cuda):
    torch = torch_cuda
    ctx = hm.Context(hi.PHYS, 0)
    # first call: a cluster group (256x128: four workgroups per solve) and
    # two single-workgroup groups, mixed precision
    big = [(256, 128, 20)] * 2 + [(64, 32, 40)] * 6 + [(16, 8, 50)] * 24
    check_same(torch, ctx, big, 4, hm.PREC_MIXED, 1e-9)
    # second call, smaller, FP64 inner solves: the buffer still holds the
    # first call's state
    small = [(32, 16, 30)] * 3 + [(16, 8, 20)] * 2
    check_same(torch, ctx, small, 1, hm.PREC_FP64, 1e-10)
    ctx.close()


def test_static_entry_point_rejects_what_it_cannot_do(torch_cuda):
    torch = torch_cuda
    ctx = hm.Context(hi.PHYS, 0)
    # beyond the buffer: 6 x 512x256 need about 142 MiB of state
    huge = [(512, 256, 2)] * 6
    assert hm.henry_workspace_bytes(huge, hm.make_opts(prec=hm.PREC_MIXED)) > hm.STATIC_SCRATCH_BYTES
    xi = torch.tensor(xi_for(huge, 0), dtype=torch.float64, device="cuda")
    with pytest.raises(hm.HenryError) as e:
        static_solve(torch, ctx, huge, xi, hm.make_opts(prec=hm.PREC_MIXED))
    assert e.value.code == hm.HENRY_ENOMEM
    small = [(16, 8, 4)] * 2
    xi = torch.tensor(xi_for(small, 0), dtype=torch.float64, device="cuda")
    for bad in (dict(steps_per_launch=2), dict(profile=1)):
        with pytest.raises(hm.HenryError) as e:
            static_solve(torch, ctx, small, xi, hm.make_opts(prec=hm.PREC_MIXED, **bad))
        assert e.value.code == hm.HENRY_EINVAL
    torch.cuda.synchronize()
    ctx.close()
