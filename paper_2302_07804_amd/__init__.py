"""Python binding of the MI355X Henry-solve library (`libhenry.so`).

Argument marshalling only: every step of the solve runs in the HIP kernels
behind the C ABI declared in `include/henry.h`.  PyTorch provides device
memory and streams.  If the shared library is missing, importing works but
every call raises `HenryLibraryMissing`: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
LIB_PATH = os.path.join(_HERE, "libhenry.so")
_SOURCES = [os.path.join(_HERE, "csrc", f) for f in ("henry_api.hip", "henry_solve512.hip", "henry_mlmc_plan.cpp")]
_DEPS = [os.path.join(_HERE, "csrc", f) for f in ("henry_device.hpp", "henry_mlmc.hpp", "henry_adjoint.hpp")] + \
    [os.path.join(_ROOT, "include", "henry.h")]

HENRY_OK, HENRY_EINVAL, HENRY_ENOMEM, HENRY_EHIP, HENRY_ENOCONV, HENRY_ENONFINITE = 0, -1, -2, -3, -4, -5
STATUS_OK, STATUS_NOCONV, STATUS_NONFINITE, STATUS_SYNC = 0, 1, 2, 3
FIELD_CLOSED3, FIELD_KL41, FIELD_EXPLICIT, FIELD_TWOLAYER3 = 0, 1, 2, 3
PREC_FP64, PREC_MIXED = 0, 1

# every symbol the header declares
EXPORTS = ("henry_strerror", "henry_ctx_create", "henry_ctx_destroy", "henry_opts_default", "henry_sample_xi",
           "henry_workspace_bytes", "henry_solve_batch", "henry_profile_last", "henry_tune_set", "henry_tune_get",
           "henry_adjoint_workspace_bytes", "henry_adjoint_batch", "mlmc_level_estimate", "henry_kl_basis",
           "henry_ctx_set_kl", "henry_sample_xi_kl", "henry_residual_batch", "henry_mlmc_allocate",
           "henry_mlmc_rates", "henry_qmc_points", "henry_solve_batch_trace", "henry_sample_stats",
           "henry_first_passage", "henry_level_smooth", "henry_mlmc_telescope", "henry_solve_batch_static")

# bytes of the static device buffer of henry_solve_batch_static (HENRY_STATIC_SCRATCH_BYTES)
STATIC_SCRATCH_BYTES = 128 << 20


class HenryLibraryMissing(RuntimeError):
    pass


class HenryError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {code} ({strerror(code) if _lib else 'library not loaded'})")
        self.code = code


# A build of the library whose solve kernel also accumulates wall-clock time
# per phase of the outer iteration (HENRY_PHASE_TIMERS) into each solve's
# scratch region; for measurement only, never the product path.
PHASE_TIMER_LIB_PATH = os.path.join(_ROOT, "_build", "libhenry_phase_timers.so")


def hipcc_command(out=LIB_PATH, defines=()):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    return [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument",
            "-I", os.path.join(_ROOT, "include"), "-I", os.path.join(_HERE, "csrc")] + \
        [f"-D{d}" for d in defines] + ["-o", out] + _SOURCES


def build(out: str = LIB_PATH, defines=()) -> str:
    """Compile libhenry.so for gfx950 (always recompiles); `defines` are
    preprocessor symbols (HENRY_PHASE_TIMERS for the instrumented build)."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    subprocess.check_call(hipcc_command(tmp, defines), cwd=_HERE)
    os.replace(tmp, out)
    return out


class Phys(ct.Structure):
    _fields_ = [(k, ct.c_double) for k in ("rho0", "rho1", "mu", "g", "D", "phi0", "k0", "q_in", "T")]


class Grid(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("nsteps", ct.c_int32), ("reserved", ct.c_int32)]


class Opts(ct.Structure):
    _fields_ = [("prec", ct.c_int32), ("max_outer", ct.c_int32), ("tol", ct.c_double), ("threads", ct.c_int32),
                ("steps_per_launch", ct.c_int32), ("profile", ct.c_int32), ("serial_groups", ct.c_int32),
                ("cluster", ct.c_int32), ("cluster_wait_us", ct.c_int32), ("predictor", ct.c_int32)]


class GroupTime(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("nsolves", ct.c_int32), ("launches", ct.c_int32),
                ("cell_steps", ct.c_int64), ("ms", ct.c_double), ("threads", ct.c_int32), ("cluster", ct.c_int32)]


_lib = None


def lib():
    """Load libhenry.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise HenryLibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    try:
        import torch  # noqa: F401  (loads the HIP runtime torch uses)
    except ImportError:
        pass
    L = ct.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_double
    L.henry_strerror.argtypes = [ct.c_int]
    L.henry_strerror.restype = ct.c_char_p
    L.henry_ctx_create.argtypes = [ct.POINTER(vp), ct.POINTER(Phys), ct.c_int]
    L.henry_ctx_destroy.argtypes = [vp]
    L.henry_ctx_destroy.restype = None
    L.henry_opts_default.argtypes = [ct.POINTER(Opts)]
    L.henry_opts_default.restype = None
    L.henry_sample_xi.argtypes = [ct.c_uint64, i32, i64, i64, i32, ct.POINTER(ct.c_double)]
    L.henry_workspace_bytes.argtypes = [vp, ct.POINTER(Grid), i32, ct.POINTER(Opts), ct.POINTER(ct.c_size_t)]
    L.henry_solve_batch.argtypes = [vp, ct.POINTER(Grid), i32, i32, vp, vp, vp, vp, vp, ct.POINTER(Opts), vp, vp,
                                    vp, vp, vp, vp, ct.c_size_t, vp]
    L.henry_solve_batch_static.argtypes = [vp, ct.POINTER(Grid), i32, i32, vp, vp, vp, vp, vp, ct.POINTER(Opts),
                                           vp, vp, vp, vp, vp, vp]
    L.henry_solve_batch_trace.argtypes = [vp, ct.POINTER(Grid), i32, i32, vp, vp, vp, vp, vp, ct.POINTER(Opts), i32,
                                          i32, ct.POINTER(ct.c_double), dbl, vp, vp, vp, vp, vp, vp, vp, ct.c_size_t,
                                          vp]
    L.henry_sample_stats.argtypes = [vp, i32, i32, vp, vp, i32, ct.POINTER(ct.c_double), vp, vp, vp, vp]
    L.henry_first_passage.argtypes = [vp, i32, i32, i32, i32, vp, dbl, i32, vp, vp, vp]
    L.henry_level_smooth.argtypes = [vp, i32, i32, i32, i32, i32, vp, vp, vp, vp, ct.c_size_t, vp]
    L.henry_profile_last.argtypes = [vp, ct.POINTER(GroupTime), i32, ct.POINTER(i32)]
    L.henry_mlmc_allocate.argtypes = [i32, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double), dbl,
                                      ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double)]
    L.henry_mlmc_rates.argtypes = [i32, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double), i32,
                                   ct.POINTER(ct.c_double), ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]
    L.henry_residual_batch.argtypes = [vp, ct.POINTER(Grid), i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                       ct.c_size_t, vp]
    L.henry_qmc_points.argtypes = [i64, i64, i32, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]
    L.henry_tune_set.argtypes = [vp, i32, i32, i32, i32, i32]
    L.henry_tune_get.argtypes = [vp, i32, i32, ct.POINTER(i32), ct.POINTER(i32), ct.POINTER(i32)]
    L.henry_adjoint_workspace_bytes.argtypes = [vp, ct.POINTER(Grid), i32, ct.POINTER(Opts), i32,
                                                ct.POINTER(ct.c_size_t)]
    L.henry_adjoint_batch.argtypes = [vp, ct.POINTER(Grid), i32, i32, vp, vp, vp, vp, ct.POINTER(Opts), i32, dbl, i32,
                                      vp, vp, vp, vp, vp, vp, vp, vp, ct.c_size_t, vp]
    L.henry_kl_basis.argtypes = [i32, i32, i32, dbl, i32, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]
    L.henry_ctx_set_kl.argtypes = [vp, i32, i32, dbl, dbl, dbl]
    L.henry_sample_xi_kl.argtypes = [ct.c_uint64, i32, i64, i64, ct.POINTER(ct.c_double)]
    L.mlmc_level_estimate.argtypes = [vp, i32, ct.POINTER(Grid), ct.POINTER(i32), ct.POINTER(vp), ct.POINTER(vp),
                                      ct.POINTER(vp), ct.POINTER(vp), ct.POINTER(vp), ct.POINTER(vp), vp, vp, vp, vp]
    L.henry_mlmc_telescope.argtypes = [vp, i32, i32, ct.POINTER(vp), ct.POINTER(vp), ct.POINTER(i32),
                                       ct.POINTER(i64), vp, vp, vp]
    _lib = L
    return L


def strerror(code: int) -> str:
    return lib().henry_strerror(code).decode()


def _chk(rc, what):
    if rc != HENRY_OK:
        raise HenryError(rc, what)


def grids(solves) -> ct.Array:
    """[(nx, ny, nsteps), ...] -> henry_grid_t array."""
    arr = (Grid * len(solves))()
    for k, s in enumerate(solves):
        arr[k].nx, arr[k].ny, arr[k].nsteps, arr[k].reserved = int(s[0]), int(s[1]), int(s[2]), 0
    return arr


def opts_default() -> Opts:
    o = Opts()
    lib().henry_opts_default(ct.byref(o))
    return o


def make_opts(**kw) -> Opts:
    o = opts_default()
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def henry_sample_xi(seed: int, level: int, first: int, count: int, dim: int = 3):
    import numpy as np
    out = np.empty((count, dim), np.float64)
    _chk(lib().henry_sample_xi(seed, level, first, count, dim, out.ctypes.data_as(ct.POINTER(ct.c_double))),
         "henry_sample_xi")
    return out


def henry_qmc_points(first: int, count: int, dim: int = 3, shift=None):
    """Halton points 2 frac(phi(first + k) + shift) - 1, [count][dim] on the host."""
    import numpy as np
    out = np.empty((max(count, 0), max(dim, 0)), np.float64)
    sh = None
    if shift is not None:
        sh = np.ascontiguousarray(shift, dtype=np.float64)
        if sh.shape != (max(dim, 0),):
            raise ValueError(f"shift must have {dim} entries")
    _chk(lib().henry_qmc_points(first, count, dim, None if sh is None else sh.ctypes.data_as(ct.POINTER(ct.c_double)),
                                out.ctypes.data_as(ct.POINTER(ct.c_double))), "henry_qmc_points")
    return out


def henry_sample_xi_kl(seed: int, level: int, first: int, count: int):
    import numpy as np
    out = np.empty((count, 41), np.float64)
    _chk(lib().henry_sample_xi_kl(seed, level, first, count, out.ctypes.data_as(ct.POINTER(ct.c_double))),
         "henry_sample_xi_kl")
    return out


def henry_kl_basis(nx: int, ny: int, nmodes: int = 20, corr_len: float = 0.3, nquad: int = 200):
    """(lam[nmodes], modes[nmodes][ny][nx]) on the host."""
    import numpy as np
    lam = np.empty(nmodes, np.float64)
    modes = np.empty((nmodes, ny, nx), np.float64)
    dp = ct.POINTER(ct.c_double)
    _chk(lib().henry_kl_basis(nx, ny, nmodes, corr_len, nquad, lam.ctypes.data_as(dp), modes.ctypes.data_as(dp)),
         "henry_kl_basis")
    return lam, modes


def henry_workspace_bytes(solves, opts: Opts | None = None, ctx=None) -> int:
    g = grids(solves)
    n = ct.c_size_t()
    _chk(lib().henry_workspace_bytes(ctx, g, len(solves), ct.byref(opts) if opts else None, ct.byref(n)),
         "henry_workspace_bytes")
    return n.value


class Context:
    """Owns a henry_ctx (plans, tuned choices) bound to one device."""

    def __init__(self, phys: dict, device: int = 0):
        self.handle = ct.c_void_p()
        p = Phys(**{name: float(phys[name]) for name, _ in Phys._fields_})
        _chk(lib().henry_ctx_create(ct.byref(self.handle), ct.byref(p), device), "henry_ctx_create")
        self.device = device
        self.phys = {name: float(phys[name]) for name, _ in Phys._fields_}
        self.kl = {}  # grid width -> set_kl arguments (to rebuild a context with other constants)

    def set_kl(self, nx: int, ny: int, corr_len: float = 0.3, sigma_phi: float = 0.1, sigma_logk: float = 0.5):
        """Upload the KL basis used by FIELD_KL41 solves on nx x ny grids."""
        _chk(lib().henry_ctx_set_kl(self.handle, nx, ny, corr_len, sigma_phi, sigma_logk), "henry_ctx_set_kl")
        self.kl[nx] = (nx, ny, corr_len, sigma_phi, sigma_logk)

    def close(self):
        if self.handle:
            lib().henry_ctx_destroy(self.handle)
            self.handle = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _need(t, n, dtype, what, device=None, optional=False):
    """Check a caller's tensor before its pointer crosses the ABI: at least
    n elements of `dtype`, contiguous, on the context's GPU.  The library
    sees only the pointer, so a short buffer would be written past its end."""
    import torch
    if t is None:
        if optional:
            return
        raise ValueError(f"{what} is required")
    if t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, not {t.dtype}")
    if not t.is_cuda or (device is not None and t.device.index != device):
        raise ValueError(f"{what} must be on cuda:{device}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.numel() < n:
        raise ValueError(f"{what} has {t.numel()} elements, needs {n}")


def _f64t():
    import torch
    return torch.float64


def _i32t():
    import torch
    return torch.int32


def _stream_of(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


def _check_solve_args(ctx, solves, field, xi, phi, logk, qin, c0, c_out, p_out, qoi_out, status, iters):
    n = len(solves)
    cells = sum(int(s[0]) * int(s[1]) for s in solves)
    f64, i32, d = _f64t(), _i32t(), ctx.device
    if field in (FIELD_CLOSED3, FIELD_TWOLAYER3, FIELD_KL41):
        _need(xi, n * (41 if field == FIELD_KL41 else 3), f64, "xi", d)
    elif field == FIELD_EXPLICIT:
        _need(phi, cells, f64, "phi", d)
        _need(logk, cells, f64, "logk", d)
        _need(qin, n, f64, "qin", d)
    _need(c0, cells, f64, "c0", d, optional=True)
    _need(c_out, cells, f64, "c_out", d)
    _need(p_out, cells, f64, "p_out", d, optional=True)
    _need(qoi_out, n, f64, "qoi_out", d)
    _need(status, n, i32, "status", d)
    _need(iters, n, i32, "iters", d, optional=True)


def henry_solve_batch(ctx: Context, solves, field, xi=None, phi=None, logk=None, qin=None, c0=None,
                      opts: Opts | None = None, c_out=None, p_out=None, qoi_out=None, status=None, iters=None,
                      workspace=None, stream=None):
    """Thin wrapper: tensors are device tensors owned by the caller."""
    g = grids(solves)
    _check_solve_args(ctx, solves, field, xi, phi, logk, qin, c0, c_out, p_out, qoi_out, status, iters)
    rc = lib().henry_solve_batch(ctx.handle, g, len(solves), field, _ptr(xi), _ptr(phi), _ptr(logk), _ptr(qin),
                                 _ptr(c0), ct.byref(opts) if opts else None, _ptr(c_out), _ptr(p_out),
                                 _ptr(qoi_out), _ptr(status), _ptr(iters), _ptr(workspace),
                                 workspace.numel() * workspace.element_size() if workspace is not None else 0,
                                 _stream_of(stream))
    _chk(rc, "henry_solve_batch")


def henry_solve_batch_static(ctx: Context, solves, field, xi=None, phi=None, logk=None, qin=None, c0=None,
                             opts: Opts | None = None, c_out=None, p_out=None, qoi_out=None, status=None, iters=None,
                             stream=None):
    """Thin wrapper of the allocation-free entry point: henry_solve_batch
    with the solves' state in the library's static device buffer (no
    workspace argument; at most STATIC_SCRATCH_BYTES of it)."""
    g = grids(solves)
    _check_solve_args(ctx, solves, field, xi, phi, logk, qin, c0, c_out, p_out, qoi_out, status, iters)
    rc = lib().henry_solve_batch_static(ctx.handle, g, len(solves), field, _ptr(xi), _ptr(phi), _ptr(logk),
                                        _ptr(qin), _ptr(c0), ct.byref(opts) if opts else None, _ptr(c_out),
                                        _ptr(p_out), _ptr(qoi_out), _ptr(status), _ptr(iters), _stream_of(stream))
    _chk(rc, "henry_solve_batch_static")


def henry_solve_batch_trace(ctx: Context, solves, field, xi=None, phi=None, logk=None, qin=None, c0=None,
                            opts: Opts | None = None, nrec=1, points=(), c_fresh=0.012178, trace_out=None, c_out=None,
                            p_out=None, qoi_out=None, status=None, iters=None, workspace=None, stream=None):
    """Thin wrapper: tensors are device tensors owned by the caller; points
    is a host sequence of (x, y)."""
    import numpy as np
    g = grids(solves)
    _check_solve_args(ctx, solves, field, xi, phi, logk, qin, c0, c_out, p_out, qoi_out, status, iters)
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(-1, 2))
    _need(trace_out, len(solves) * int(nrec) * (1 + len(pts)), _f64t(), "trace_out", ctx.device)
    rc = lib().henry_solve_batch_trace(ctx.handle, g, len(solves), field, _ptr(xi), _ptr(phi), _ptr(logk),
                                       _ptr(qin), _ptr(c0), ct.byref(opts) if opts else None, int(nrec), len(pts),
                                       pts.ctypes.data_as(ct.POINTER(ct.c_double)), float(c_fresh), _ptr(trace_out),
                                       _ptr(c_out), _ptr(p_out), _ptr(qoi_out), _ptr(status), _ptr(iters),
                                       _ptr(workspace),
                                       workspace.numel() * workspace.element_size() if workspace is not None else 0,
                                       _stream_of(stream))
    _chk(rc, "henry_solve_batch_trace")


def henry_sample_stats(ctx: Context, x, probs=(), stream=None, x_sub=None):
    """Mean, unbiased variance and type-7 quantiles of each column of the
    device tensor x [nsamples][nvals] (of x - x_sub when x_sub is given);
    returns device tensors (mean [nvals], var [nvals], q [len(probs)][nvals])."""
    import numpy as np
    import torch
    ns, nv = int(x.shape[0]), int(x.shape[1]) if x.dim() > 1 else 1
    f64 = dict(dtype=torch.float64, device=x.device)
    mean, var = torch.empty(nv, **f64), torch.empty(nv, **f64)
    pr = np.ascontiguousarray(probs, dtype=np.float64)
    q = torch.empty((len(pr), nv), **f64)
    if x_sub is not None and tuple(x_sub.shape) != tuple(x.shape):
        raise ValueError("x_sub must have the shape of x")
    _chk(lib().henry_sample_stats(ctx.handle, ns, nv, _ptr(x), _ptr(x_sub), len(pr),
                                  pr.ctypes.data_as(ct.POINTER(ct.c_double)), _ptr(mean), _ptr(var), _ptr(q),
                                  _stream_of(stream)), "henry_sample_stats")
    return mean, var, q


def henry_first_passage(ctx: Context, trace, col, threshold, below=True, stream=None):
    """First record per sample at which column col of trace [nsamples][nrec]
    [stride] falls below (below=True) or rises above threshold, 0 if none,
    and the histogram of those record numbers [nrec + 1]; device tensors."""
    import torch
    ns, nrec, stride = (int(v) for v in trace.shape)
    t = torch.empty(ns, dtype=torch.int32, device=trace.device)
    hist = torch.empty(nrec + 1, dtype=torch.int32, device=trace.device)
    _chk(lib().henry_first_passage(ctx.handle, ns, nrec, stride, int(col), _ptr(trace), float(threshold),
                                   1 if below else 0, _ptr(t), _ptr(hist), _stream_of(stream)), "henry_first_passage")
    return t, hist


def henry_level_smooth(ctx: Context, nx, ny, kind, prec, sweeps, coef, b, x, stream=None):
    """`sweeps` smoothing sweeps of one multigrid level on A x = b (kind 0
    pressure red-black Gauss-Seidel, 1 / 2 transport x- / y-line zebra);
    coef, b, x are device FP64 tensors, x is updated in place."""
    import torch
    elt = 4 if prec == PREC_MIXED else 8
    ws = _aligned_workspace(elt * (10 * nx * ny + 4 * ny), x.device)
    _chk(lib().henry_level_smooth(ctx.handle, nx, ny, kind, prec, sweeps, _ptr(coef), _ptr(b), _ptr(x), _ptr(ws),
                                  ws.numel() * ws.element_size(), _stream_of(stream)), "henry_level_smooth")
    return x


def henry_residual_batch(ctx: Context, solves, field, xi=None, phi=None, logk=None, qin=None, p=None, c=None,
                         cn=None, rp_out=None, rc_out=None, workspace=None, stream=None):
    """Thin wrapper: tensors are device tensors owned by the caller."""
    g = grids(solves)
    rc = lib().henry_residual_batch(ctx.handle, g, len(solves), field, _ptr(xi), _ptr(phi), _ptr(logk), _ptr(qin),
                                    _ptr(p), _ptr(c), _ptr(cn), _ptr(rp_out), _ptr(rc_out), _ptr(workspace),
                                    workspace.numel() * workspace.element_size() if workspace is not None else 0,
                                    _stream_of(stream))
    _chk(rc, "henry_residual_batch")


def residual(ctx: Context, solves, p, c, cn, xi=None, phi=None, logk=None, qin=None, stream=None, model=None):
    """R^p, R^c (packed device tensors) of each solve's discrete equations at
    the state (p, c) with previous time level cn (packed device tensors)."""
    import torch
    dev = torch.device("cuda", ctx.device)
    cells = sum(int(s[0]) * int(s[1]) for s in solves)
    ws_bytes = henry_workspace_bytes(solves)
    ws = torch.empty((ws_bytes + 255) // 256 * 256 // 8 + 32, dtype=torch.float64, device=dev)
    off = (-ws.data_ptr()) % 256 // 8
    ws = ws[off:off + (ws_bytes + 7) // 8]
    rp = torch.empty(cells, dtype=torch.float64, device=dev)
    rc = torch.empty(cells, dtype=torch.float64, device=dev)
    henry_residual_batch(ctx, solves, _field_of(xi, model), xi=xi, phi=phi, logk=logk, qin=qin, p=p, c=c, cn=cn,
                         rp_out=rp, rc_out=rc, workspace=ws, stream=stream)
    return rp, rc


def henry_mlmc_allocate(V, s, eps2):
    """eq:M_ell: (m[l], cost) for variances V[l] and costs s[l] (host)."""
    import numpy as np
    V = np.ascontiguousarray(V, np.float64)
    s = np.ascontiguousarray(s, np.float64)
    m = np.empty(len(V), np.int64)
    cost = ct.c_double()
    dp = lambda a: a.ctypes.data_as(ct.POINTER(ct.c_double))
    _chk(lib().henry_mlmc_allocate(len(V), dp(V), dp(s), float(eps2), m.ctypes.data_as(ct.POINTER(ct.c_int64)),
                                   ct.byref(cost)), "henry_mlmc_allocate")
    return m, cost.value


def henry_mlmc_rates(mean, var, first=1):
    """(alpha, beta, bias of the finest level) from level means and variances."""
    import numpy as np
    mean = np.ascontiguousarray(mean, np.float64)
    var = np.ascontiguousarray(var, np.float64)
    a, b, bias = ct.c_double(), ct.c_double(), ct.c_double()
    dp = lambda x: x.ctypes.data_as(ct.POINTER(ct.c_double))
    _chk(lib().henry_mlmc_rates(len(mean), dp(mean), dp(var), int(first), ct.byref(a), ct.byref(b), ct.byref(bias)),
         "henry_mlmc_rates")
    return a.value, b.value, bias.value


def henry_profile_last(ctx: Context):
    """Per-grid-group HIP-event timings of the last profiled batch."""
    cap = 64
    arr = (GroupTime * cap)()
    n = ct.c_int32()
    _chk(lib().henry_profile_last(ctx.handle, arr, cap, ct.byref(n)), "henry_profile_last")
    return [dict(nx=g.nx, ny=g.ny, nsolves=g.nsolves, launches=g.launches, cell_steps=g.cell_steps, ms=g.ms,
                 threads=g.threads, cluster=g.cluster) for g in arr[:n.value]]


def mlmc_level_estimate(ctx: Context, fine_grids, m, c_fine, c_coarse, q_fine, q_coarse, mean_Y, var_Y, qstats,
                        Ec_finest, var_est, stream=None):
    L = len(fine_grids) - 1
    g = grids(fine_grids)
    f64, d = _f64t(), ctx.device
    for l, fg in enumerate(fine_grids):
        cells, ml = int(fg[0]) * int(fg[1]), int(m[l])
        _need(c_fine[l], ml * cells, f64, f"c_fine[{l}]", d)
        _need(q_fine[l], ml, f64, f"q_fine[{l}]", d)
        if l > 0:
            _need(c_coarse[l], ml * cells // 4, f64, f"c_coarse[{l}]", d)
            _need(q_coarse[l], ml, f64, f"q_coarse[{l}]", d)
        _need(mean_Y[l], cells, f64, f"mean_Y[{l}]", d)
        _need(var_Y[l], cells, f64, f"var_Y[{l}]", d)
    _need(qstats, 2 * (L + 1), f64, "qstats", d)
    _need(Ec_finest, int(fine_grids[-1][0]) * int(fine_grids[-1][1]), f64, "Ec_finest", d)
    _need(var_est, 2, f64, "var_est", d)
    mm = (ct.c_int32 * (L + 1))(*[int(x) for x in m])
    P = ct.c_void_p * (L + 1)
    arr = lambda ts: P(*[(t.data_ptr() if t is not None else None) for t in ts])
    rc = lib().mlmc_level_estimate(ctx.handle, L, g, mm, arr(c_fine), arr(c_coarse), arr(q_fine), arr(q_coarse),
                                   arr(mean_Y), arr(var_Y), _ptr(qstats), _ptr(Ec_finest), _ptr(var_est),
                                   _stream_of(stream))
    _chk(rc, "mlmc_level_estimate")


def henry_mlmc_telescope(ctx: Context, means, vars_=None, m=None, offsets=None, nvals=None, stream=None):
    """Partial sums over levels 0..l of the level means (eq:A) and of
    V_l / m_l, for every l: returns device tensors (pmean [L+1][nvals],
    pvar [L+1][nvals] or None).  means / vars_: per-level device tensors;
    offsets: per-level element offsets (e.g. the cell of a point)."""
    import numpy as np
    import torch
    nl = len(means)
    off = [0] * nl if offsets is None else [int(o) for o in offsets]
    if nvals is None:
        nvals = min(int(t.numel()) - o for t, o in zip(means, off))
    f64, d = _f64t(), ctx.device
    for l in range(nl):
        _need(means[l], off[l] + nvals, f64, f"means[{l}]", d)
        if vars_ is not None:
            _need(vars_[l], off[l] + nvals, f64, f"vars[{l}]", d)
    mm = np.ones(nl, np.int32) if m is None else np.ascontiguousarray(m, dtype=np.int32)
    if len(mm) != nl:
        raise ValueError("one sample count per level")
    P = ct.c_void_p * nl
    dev = torch.device("cuda", ctx.device)
    pm = torch.empty((nl, nvals), dtype=torch.float64, device=dev)
    pv = torch.empty((nl, nvals), dtype=torch.float64, device=dev) if vars_ is not None else None
    offs = np.ascontiguousarray(off, dtype=np.int64)
    rc = lib().henry_mlmc_telescope(ctx.handle, nl, int(nvals), P(*[t.data_ptr() for t in means]),
                                    P(*[t.data_ptr() for t in vars_]) if vars_ is not None else None,
                                    mm.ctypes.data_as(ct.POINTER(ct.c_int32)),
                                    offs.ctypes.data_as(ct.POINTER(ct.c_int64)), _ptr(pm), _ptr(pv),
                                    _stream_of(stream))
    _chk(rc, "henry_mlmc_telescope")
    return pm, pv


def telescoped_q(ctx: Context, qstats, m=None):
    """E[Q] truncated after each level from mlmc_level_estimate's qstats
    ([L+1][2]: mean, variance of Q_l - Q_{l-1}), summed on the device, and
    sum V_l / m_l likewise when m is given; host arrays."""
    L1 = int(qstats.numel()) // 2
    means = [qstats[2 * l:2 * l + 1] for l in range(L1)]
    vars_ = [qstats[2 * l + 1:2 * l + 2] for l in range(L1)] if m is not None else None
    pm, pv = henry_mlmc_telescope(ctx, means, vars_, m, nvals=1)
    return pm[:, 0].cpu().numpy(), (pv[:, 0].cpu().numpy() if pv is not None else None)


# ------------------------------------------------------------------ convenience layer
def _field_of(xi, model=None):
    """HENRY_FIELD_* of a call: no xi -> explicit fields, 41 coefficients ->
    KL, 3 -> the closed-form fields, or with model="two_layer" the two-layer
    porosity model with Kozeny-Carman permeability."""
    if xi is None:
        return FIELD_EXPLICIT
    if xi.shape[-1] == 41:
        return FIELD_KL41
    if model not in (None, "closed", "two_layer"):
        raise ValueError(f"unknown field model {model!r}")
    return FIELD_TWOLAYER3 if model == "two_layer" else FIELD_CLOSED3


def solve(ctx: Context, solves, xi=None, phi=None, logk=None, qin=None, c0=None, opts: Opts | None = None,
          want_p=False, stream=None, model=None, trace=None):
    """Allocate outputs/workspace with torch and run one batch.
    solves: list of (nx, ny, nsteps).  xi [n][3] selects the closed-form
    fields (model="two_layer": the two-layer porosity model), xi [n][41]
    the KL fields (Context.set_kl for every grid), no xi the explicit
    fields.  trace=(nrec, points[, c_fresh]) also records each solve's time
    series (out["trace"], [n][nrec][1 + len(points)]).  Returns dict of
    device tensors."""
    import torch
    dev = torch.device("cuda", ctx.device)
    opts = opts or opts_default()
    cells = sum(int(s[0]) * int(s[1]) for s in solves)
    ws_bytes = henry_workspace_bytes(solves, opts)
    ws = torch.empty((ws_bytes + 255) // 256 * 256 // 8 + 32, dtype=torch.float64, device=dev)
    # 256-byte aligned view
    off = (-ws.data_ptr()) % 256 // 8
    ws = ws[off:off + (ws_bytes + 7) // 8]
    out = dict(c=torch.empty(cells, dtype=torch.float64, device=dev),
               qoi=torch.empty(len(solves), dtype=torch.float64, device=dev),
               status=torch.empty(len(solves), dtype=torch.int32, device=dev),
               iters=torch.empty(len(solves), dtype=torch.int32, device=dev))
    out["p"] = torch.empty(cells, dtype=torch.float64, device=dev) if want_p else None
    field = _field_of(xi, model)
    if trace is None:
        henry_solve_batch(ctx, solves, field, xi=xi, phi=phi, logk=logk, qin=qin, c0=c0, opts=opts, c_out=out["c"],
                          p_out=out["p"], qoi_out=out["qoi"], status=out["status"], iters=out["iters"],
                          workspace=ws, stream=stream)
    else:
        nrec, points = int(trace[0]), list(trace[1])
        c_fresh = float(trace[2]) if len(trace) > 2 else 0.012178
        out["trace"] = torch.empty((len(solves), nrec, 1 + len(points)), dtype=torch.float64, device=dev)
        henry_solve_batch_trace(ctx, solves, field, xi=xi, phi=phi, logk=logk, qin=qin, c0=c0, opts=opts,
                                nrec=nrec, points=points, c_fresh=c_fresh, trace_out=out["trace"], c_out=out["c"],
                                p_out=out["p"], qoi_out=out["qoi"], status=out["status"], iters=out["iters"],
                                workspace=ws, stream=stream)
    out["workspace"] = ws
    return out


def unpack(flat, solves):
    """Split a packed per-solve field into a list of [ny][nx] views."""
    res, off = [], 0
    for s in solves:
        n = int(s[0]) * int(s[1])
        res.append(flat[off:off + n].view(int(s[1]), int(s[0])))
        off += n
    return res


# ------------------------------------------------------------------ discrete adjoint
def henry_adjoint_workspace_bytes(solves, opts: Opts | None = None, ckpt_every: int = 20, ctx=None) -> int:
    g = grids(solves)
    n = ct.c_size_t()
    _chk(lib().henry_adjoint_workspace_bytes(ctx, g, len(solves), ct.byref(opts) if opts else None, ckpt_every,
                                             ct.byref(n)), "henry_adjoint_workspace_bytes")
    return n.value


def henry_adjoint_batch(ctx: Context, solves, field, xi=None, phi=None, logk=None, qin=None,
                        opts: Opts | None = None, ckpt_every=20, adj_tol=1e-10, adj_max_it=60, qoi_out=None,
                        dq_dxi=None, dq_dlogk=None, dq_dphi=None, dq_dq=None, status=None, iters=None,
                        workspace=None, stream=None):
    """Thin wrapper: tensors are device tensors owned by the caller."""
    g = grids(solves)
    n = len(solves)
    cells = sum(int(s[0]) * int(s[1]) for s in solves)
    f64, d = _f64t(), ctx.device
    if field in (FIELD_CLOSED3, FIELD_TWOLAYER3, FIELD_KL41):
        dim = 41 if field == FIELD_KL41 else 3
        _need(xi, n * dim, f64, "xi", d)
        _need(dq_dxi, n * dim, f64, "dq_dxi", d, optional=True)
    elif field == FIELD_EXPLICIT:
        _need(phi, cells, f64, "phi", d)
        _need(logk, cells, f64, "logk", d)
        _need(qin, n, f64, "qin", d)
    _need(qoi_out, n, f64, "qoi_out", d)
    _need(dq_dlogk, cells, f64, "dq_dlogk", d, optional=True)
    _need(dq_dphi, cells, f64, "dq_dphi", d, optional=True)
    _need(dq_dq, n, f64, "dq_dq", d, optional=True)
    _need(status, n, _i32t(), "status", d)
    _need(iters, n, _i32t(), "iters", d, optional=True)
    rc = lib().henry_adjoint_batch(ctx.handle, g, len(solves), field, _ptr(xi), _ptr(phi), _ptr(logk), _ptr(qin),
                                   ct.byref(opts) if opts else None, int(ckpt_every), float(adj_tol),
                                   int(adj_max_it), _ptr(qoi_out), _ptr(dq_dxi), _ptr(dq_dlogk), _ptr(dq_dphi),
                                   _ptr(dq_dq), _ptr(status), _ptr(iters), _ptr(workspace),
                                   workspace.numel() * workspace.element_size() if workspace is not None else 0,
                                   _stream_of(stream))
    _chk(rc, "henry_adjoint_batch")


def aligned_workspace(nbytes, dev):
    """A 256-byte aligned float64 device view of at least nbytes bytes."""
    return _aligned_workspace(nbytes, dev)


def _aligned_workspace(nbytes, dev):
    import torch
    raw = torch.empty(nbytes // 8 + 64, dtype=torch.float64, device=dev)
    off = (-raw.data_ptr()) % 256 // 8
    return raw[off:off + (nbytes + 7) // 8]


def adjoint(ctx: Context, solves, xi=None, phi=None, logk=None, qin=None, opts: Opts | None = None,
            ckpt_every=20, adj_tol=1e-10, adj_max_it=60, stream=None, model=None):
    """Allocate outputs and run the adjoint; returns dict of device tensors
    (qoi, dq_dxi for closed-form fields, dq_dlogk, dq_dphi, dq_dq, status)."""
    import torch
    dev = torch.device("cuda", ctx.device)
    opts = opts or opts_default()
    cells = sum(int(s[0]) * int(s[1]) for s in solves)
    ns = len(solves)
    ws = _aligned_workspace(henry_adjoint_workspace_bytes(solves, opts, ckpt_every), dev)
    f64 = dict(dtype=torch.float64, device=dev)
    out = dict(qoi=torch.empty(ns, **f64), dq_dlogk=torch.empty(cells, **f64), dq_dphi=torch.empty(cells, **f64),
               dq_dq=torch.empty(ns, **f64), status=torch.empty(ns, dtype=torch.int32, device=dev),
               iters=torch.empty(ns, dtype=torch.int32, device=dev))
    field = _field_of(xi, model)
    out["dq_dxi"] = torch.empty((ns, xi.shape[-1]), **f64) if xi is not None else None
    henry_adjoint_batch(ctx, solves, field, xi=xi, phi=phi, logk=logk,
                        qin=qin, opts=opts, ckpt_every=ckpt_every, adj_tol=adj_tol, adj_max_it=adj_max_it,
                        qoi_out=out["qoi"], dq_dxi=out["dq_dxi"], dq_dlogk=out["dq_dlogk"], dq_dphi=out["dq_dphi"],
                        dq_dq=out["dq_dq"], status=out["status"], iters=out["iters"], workspace=ws, stream=stream)
    return out


def _autograd_classes():
    import torch

    class HenryQoI(torch.autograd.Function):
        """Q(xi) for a batch of solves with the closed-form random fields;
        backward runs the discrete adjoint.  Usage:
        HenryQoI.apply(xi, ctx, solves, opts, ckpt_every, adj_tol)."""

        @staticmethod
        def forward(fctx, xi, ctx, solves, opts=None, ckpt_every=20, adj_tol=1e-10):
            xi = xi.detach().contiguous()
            out = solve(ctx, solves, xi=xi, opts=opts)
            fctx.save_for_backward(xi)
            fctx.henry = (ctx, solves, opts, ckpt_every, adj_tol)
            return out["qoi"]

        @staticmethod
        def backward(fctx, gq):
            (xi,) = fctx.saved_tensors
            ctx, solves, opts, ckpt_every, adj_tol = fctx.henry
            a = adjoint(ctx, solves, xi=xi, opts=opts, ckpt_every=ckpt_every, adj_tol=adj_tol)
            return gq[:, None] * a["dq_dxi"], None, None, None, None, None

    class HenryQoILogK(torch.autograd.Function):
        """Q(log K) for caller-provided per-cell fields (packed per solve);
        backward gives dQ/dlog K per cell.  Usage:
        HenryQoILogK.apply(logk, phi, qin, ctx, solves, opts, ckpt_every, adj_tol)."""

        @staticmethod
        def forward(fctx, logk, phi, qin, ctx, solves, opts=None, ckpt_every=20, adj_tol=1e-10):
            logk = logk.detach().contiguous()
            phi = phi.detach().contiguous()
            qin = qin.detach().contiguous()
            out = solve(ctx, solves, phi=phi, logk=logk, qin=qin, opts=opts)
            fctx.save_for_backward(logk, phi, qin)
            fctx.henry = (ctx, solves, opts, ckpt_every, adj_tol)
            return out["qoi"]

        @staticmethod
        def backward(fctx, gq):
            logk, phi, qin = fctx.saved_tensors
            ctx, solves, opts, ckpt_every, adj_tol = fctx.henry
            a = adjoint(ctx, solves, phi=phi, logk=logk, qin=qin, opts=opts, ckpt_every=ckpt_every,
                        adj_tol=adj_tol)
            import torch
            scale = torch.repeat_interleave(gq, torch.tensor([int(s[0]) * int(s[1]) for s in solves],
                                                             device=gq.device))
            return (scale * a["dq_dlogk"], scale * a["dq_dphi"], gq * a["dq_dq"], None, None, None, None,
                    None)

    return HenryQoI, HenryQoILogK


def __getattr__(name):
    if name in ("HenryQoI", "HenryQoILogK"):
        a, b = _autograd_classes()
        globals()["HenryQoI"], globals()["HenryQoILogK"] = a, b
        return globals()[name]
    raise AttributeError(name)


# ------------------------------------------------------------------ autotuning
def henry_tune_set(ctx: Context, nx: int, prec: int, threads: int = 0, cluster: int = 0, stream: int = -1):
    """Store tuned launch choices for grids of width nx (0 / -1: built-in)."""
    _chk(lib().henry_tune_set(ctx.handle, nx, prec, threads, cluster, stream), "henry_tune_set")


def henry_tune_get(ctx: Context, nx: int, prec: int):
    """(threads, cluster, stream) of grids of width nx: the effective
    workgroup size and the stored cluster and stream (0 / -1: built-in)."""
    t, k, st = ct.c_int32(), ct.c_int32(), ct.c_int32()
    _chk(lib().henry_tune_get(ctx.handle, nx, prec, ct.byref(t), ct.byref(k), ct.byref(st)), "henry_tune_get")
    return t.value, k.value, st.value


# The tuner's default candidates.  "halves" (see _plan_streams) is left out:
# on the L = 4 batch it gains 0-2 % on some boxes and loses 1 % on others,
# and its cheap groups' launches stretch to several times their length while
# they wait for CUs (16x8: 26 -> 149 ms), which blurs the per-group timings;
# pass plans=STREAM_PLANS + ("halves",) to include it.
STREAM_PLANS = ("built-in", "one lane", "spread", "serial")
TUNE_FRAC_TARGET = 5


def _plan_streams(plan, grid_costs):
    """Stream of each one-workgroup grid under a named plan: 'built-in'
    leaves the library's plan (-1), 'one lane' puts every such group on
    stream 1 beside the cluster groups, 'halves' the costlier half of them
    (in cost order) on stream 1 and the cheaper half on stream 2, 'spread'
    deals them over streams 1..3 in cost order, 'serial' runs everything on
    stream 0."""
    order = sorted(grid_costs, key=lambda nx: -grid_costs[nx])
    if plan == "built-in":
        return {nx: -1 for nx in order}
    if plan == "one lane":
        return {nx: 1 for nx in order}
    if plan == "halves":
        return {nx: 1 if k < (len(order) + 1) // 2 else 2 for k, nx in enumerate(order)}
    if plan == "spread":
        return {nx: 1 + k % 3 for k, nx in enumerate(order)}
    return {nx: 0 for nx in order}


def _short_batch(solves, target=TUNE_FRAC_TARGET, min_steps=8):
    """The batch shortened by a common factor f that keeps every solve's
    time step (its step count divides by f, the horizon is T / f), with f
    the divisor of the steps' gcd nearest `target` that leaves at least
    `min_steps` steps per solve; (f, shortened solves)."""
    import math
    g = 0
    for s in solves:
        g = math.gcd(g, int(s[2]))
    rmin = min(int(s[2]) for s in solves)
    divs = [d for d in range(1, g + 1) if g % d == 0 and rmin // d >= min_steps] or [1]
    f = min(divs, key=lambda d: (abs(d - target), -d))
    return f, [(int(s[0]), int(s[1]), int(s[2]) // f) for s in solves]


def autotune(ctx: Context, solves, xi, opts: Opts | None = None, tune_steps: int = 8, max_solves: int = 1024,
             candidates=(64, 128, 256, 512, 1024), cache_path: str | None = None, clusters=(1, 2, 4, 8),
             plans=STREAM_PLANS, model=None, reps: int = 2, trial_frac: int = 1):
    """Fill the context's tuning cache for the grids of `solves` by timing
    the candidates on short runs of the caller's own batch:
      1. threads per solve-workgroup, per grid: the first `tune_steps` steps
         of up to `max_solves` solves of that grid alone, HIP-event group
         time on the stream the kernels run on;
      2. workgroups per solve (cluster) for the grids above 2048 cells, one
         grid after another in cost order (eq:workpl: n_l r_l), with at
         most 256 workgroups per group; then the stream plan of the
         one-workgroup groups (STREAM_PLANS); then again every grid's
         workgroup size (half, the same, twice) at its chosen cluster size
         and beside the other groups (a cluster group may run the 512-thread
         build best while 1024 threads won at the built-in cluster size),
         and the stream plan once more at those sizes.  Each candidate times the
         whole batch, between events on the caller's stream, or with
         trial_frac > 1 the batch shortened by about that factor keeping
         every time step (_short_batch).  The whole batch is the default:
         the cluster sizes of the largest grid trade its critical path
         against the CUs left to the other groups, a balance of a few
         percent that the early steps alone misjudge (L = 4 MLMC batch:
         4 against 8 workgroups per 256x128 solve, 411 and 400 ms).
    Each candidate runs `reps` times and its fastest run counts.  The
    choices change no result (bitwise).  With cache_path, choices found
    there are used as they are and new ones are written back.  Returns
    {(nx, prec): (threads, cluster, stream, {candidate: ms})}."""
    import json
    import torch
    opts = opts or opts_default()
    prec = opts.prec
    by_grid = {}
    for k, s in enumerate(solves):
        by_grid.setdefault(int(s[0]), []).append(k)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    result = {}
    keys = {nx: f"{nx}:{prec}" for nx in by_grid}
    if all(k in cache for k in keys.values()):
        for nx, key in keys.items():
            t, kc, st = (int(v) for v in cache[key])
            henry_tune_set(ctx, nx, prec, t, kc, st)
            result[(nx, prec)] = (t, kc, st, {})
        return result
    field = _field_of(xi, model)
    # ---- 1. threads per grid, each grid alone
    tmax = 1024 if prec == PREC_MIXED else 512
    threads = {}
    for nx, ks in sorted(by_grid.items()):
        ks = ks[:max_solves]
        sub = [(int(solves[k][0]), int(solves[k][1]), min(int(solves[k][2]), tune_steps)) for k in ks]
        xs = xi[ks].contiguous()
        cells = nx * (nx // 2)
        times = {}
        for t in candidates:
            if (t > 64 and t > 2 * cells) or t > tmax:
                continue
            o = make_opts(prec=prec, tol=opts.tol, max_outer=opts.max_outer, threads=t, profile=1,
                          predictor=opts.predictor)
            best = None
            for _ in range(reps):
                solve(ctx, sub, xi=xs, opts=o, model=model)
                torch.cuda.synchronize()
                ms = sum(g["ms"] for g in henry_profile_last(ctx))
                best = ms if best is None else min(best, ms)
            times[t] = best
        threads[nx] = (min(times, key=times.get), times)
    # ---- 2. clusters and stream plan on the shortened whole batch
    f, short = _short_batch(solves, target=trial_frac)
    ph = dict(ctx.phys)
    ph["T"] = ph["T"] / f
    tctx = Context(ph, ctx.device)
    for args in ctx.kl.values():
        tctx.set_kl(*args)
    costs = {nx: sum(float(solves[k][0]) * solves[k][1] * solves[k][2] for k in ks) for nx, ks in by_grid.items()}
    choice = {nx: [threads[nx][0], 0, -1] for nx in by_grid}
    o = make_opts(prec=prec, tol=opts.tol, max_outer=opts.max_outer, predictor=opts.predictor)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def trial():
        for nx, (t, kc, st) in choice.items():
            henry_tune_set(tctx, nx, prec, t, kc, st)
        best = None
        for _ in range(reps):
            ev0.record()
            solve(tctx, short, xi=xi, opts=o, model=model)
            ev1.record()
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1)
            best = ms if best is None else min(best, ms)
        return best

    plan_times = {}
    try:
        for nx in sorted(by_grid, key=lambda g: -costs[g]):
            if nx * (nx // 2) <= 2048:
                continue
            ktimes = {}
            for kc in clusters:
                if kc * len(by_grid[nx]) > 256:
                    continue
                choice[nx][1] = kc
                ktimes[kc] = trial()
            choice[nx][1] = min(ktimes, key=ktimes.get)
            threads[nx][1].update({f"cluster {kc}": v for kc, v in ktimes.items()})
        single = {nx: costs[nx] for nx in by_grid
                  if nx * (nx // 2) <= 2048 or choice[nx][1] == 1}
        if single:
            for plan in plans:
                for nx, st in _plan_streams(plan, single).items():
                    choice[nx][2] = st
                plan_times[plan] = trial()
            best_plan = min(plan_times, key=plan_times.get)
            for nx, st in _plan_streams(best_plan, single).items():
                choice[nx][2] = st
        # 3. every grid's workgroup size again (half, the same, twice), in
        # cost order, now with its cluster size and beside the other groups:
        # the sizes of step 1 were timed alone and at the built-in clusters
        for nx in sorted(by_grid, key=lambda g: -costs[g]):
            cells = nx * (nx // 2)
            t0 = choice[nx][0]
            rtimes = {}
            for t in (t0 // 2, t0, 2 * t0):
                if t < 64 or t > tmax or (t > 64 and t > 2 * cells):
                    continue
                choice[nx][0] = t
                rtimes[t] = trial()
            choice[nx][0] = min(rtimes, key=rtimes.get)
            threads[nx][1].update({f"in batch {t}": v for t, v in rtimes.items()})
        # 4. the stream plan again, at these sizes
        if single:
            plan_times = {}
            for plan in plans:
                for nx, st in _plan_streams(plan, single).items():
                    choice[nx][2] = st
                plan_times[plan] = trial()
            best_plan = min(plan_times, key=plan_times.get)
            for nx, st in _plan_streams(best_plan, single).items():
                choice[nx][2] = st
    finally:
        tctx.close()
    for nx in by_grid:
        t, kc, st = choice[nx]
        henry_tune_set(ctx, nx, prec, t, kc, st)
        times = dict(threads[nx][1])
        times.update({f"plan {p}": v for p, v in plan_times.items()})
        result[(nx, prec)] = (t, kc, st, times)
        cache[keys[nx]] = [t, kc, st]
    if cache_path:
        with open(cache_path, "w") as f_:
            json.dump(cache, f_, indent=1, sort_keys=True)
    return result


def mlmc_run(*args, **kwargs):
    """Adaptive MLMC estimate of E[Q] (see paper_2302_07804_amd.mlmc.mlmc_run)."""
    from .mlmc import mlmc_run as run
    return run(*args, **kwargs)


def qmc_run(*args, **kwargs):
    """Randomly shifted Halton estimate of E[Q] and E[c] (see paper_2302_07804_amd.mlmc.qmc_run)."""
    from .mlmc import qmc_run as run
    return run(*args, **kwargs)


def point_cell(*args, **kwargs):
    """Cell index of a point (see paper_2302_07804_amd.mlmc.point_cell)."""
    from .mlmc import point_cell as pc
    return pc(*args, **kwargs)


def telescoped_at(*args, **kwargs):
    """MLMC estimates at a point truncated after each level (see paper_2302_07804_amd.mlmc.telescoped_at)."""
    from .mlmc import telescoped_at as tel
    return tel(*args, **kwargs)


def mlmc_fixed(*args, **kwargs):
    """MLMC estimate with given sample counts (see paper_2302_07804_amd.mlmc.mlmc_fixed)."""
    from .mlmc import mlmc_fixed as run
    return run(*args, **kwargs)


def series_run(*args, **kwargs):
    """Time-series statistics of an ensemble (see paper_2302_07804_amd.mlmc.series_run)."""
    from .mlmc import series_run as run
    return run(*args, **kwargs)


def mlmc_series(*args, **kwargs):
    """MLMC estimate of mean time series (see paper_2302_07804_amd.mlmc.mlmc_series)."""
    from .mlmc import mlmc_series as run
    return run(*args, **kwargs)
