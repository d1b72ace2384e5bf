"""FP64 CPU oracle for the Henry ensemble solves (TEST INFRASTRUCTURE).

Only `tests/`, `__graft_entry__.smoke()` and the benchmark's `cpu_baseline`
leg may import this package.  It wraps the plain C oracle
(`henry_oracle.c`: Newton + exact Jacobian + banded LU, FP64) with ctypes
and adds, in plain numpy / scipy: the MLMC estimator statistics (Sec. 3 of
the paper), a Halton quasi-Monte Carlo rule, the paper's two-layer input
model, the time series and their statistics (Sec. 4), and the multigrid
smoothers on explicitly assembled level operators.  It shares no code with the HIP
library in `paper_2302_07804_amd/`.

Parity status of each function is listed in the module docstrings of the
tests that pin it; every function here is pinned by at least one
`-m "not gpu"` test.
"""
from __future__ import annotations

import concurrent.futures as _cf
import ctypes as _ct
import os as _os
import subprocess as _sp

import numpy as np

_HERE = _os.path.dirname(_os.path.abspath(__file__))
_SRC = _os.path.join(_HERE, "henry_oracle.c")
_LIB_PATH = _os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not _os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        _sp.check_call(["gcc", "-O3", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
                        "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"], cwd=_HERE)
        _os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Phys(_ct.Structure):
    _fields_ = [(k, _ct.c_double) for k in ("rho0", "rho1", "mu", "g", "D", "phi0", "k0", "q_in", "T")]


def phys_struct(phys: dict) -> Phys:
    return Phys(**{name: float(phys[name]) for name, _ in Phys._fields_})


_D = _ct.POINTER(_ct.c_double)
_I32 = _ct.c_int32


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not _os.path.exists(_LIB_PATH):
        build(force=True)
    lib = _ct.CDLL(_LIB_PATH)
    P = _ct.POINTER(Phys)
    lib.oracle_philox4x32_10.argtypes = [_ct.POINTER(_ct.c_uint32)] * 3
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_sample_xi.argtypes = [_ct.c_uint64, _I32, _ct.c_int64, _ct.c_int64, _I32, _D]
    lib.oracle_sample_xi.restype = None
    lib.oracle_fields_closed.argtypes = [P, _I32, _I32, _D, _D, _D, _D]
    lib.oracle_residual.argtypes = [P, _I32, _I32, _I32, _D, _D, _ct.c_double, _D, _D, _D, _D, _D]
    lib.oracle_jacobian_dense.argtypes = [P, _I32, _I32, _I32, _D, _D, _ct.c_double, _D, _D, _D, _D]
    lib.oracle_band_solve_dense.argtypes = [_I32, _I32, _I32, _D, _D, _D, _I32]
    lib.oracle_qoi.argtypes = [P, _I32, _I32, _D, _D]
    lib.oracle_qoi.restype = _ct.c_double
    lib.oracle_solve.argtypes = [P, _I32, _I32, _I32, _D, _D, _ct.c_double, _D, _D, _D, _D,
                                 _ct.POINTER(_I32), _D, _D]
    lib.oracle_adjoint.argtypes = [P, _I32, _I32, _I32, _D, _D, _ct.c_double, _D, _D, _D, _D]
    lib.oracle_tangent.argtypes = [P, _I32, _I32, _I32, _D, _D, _ct.c_double, _D, _D, _ct.c_double,
                                   _D, _D]
    _lib = lib
    return lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


# ---------------------------------------------------------------- sampling
def philox4x32_10(ctr, key):
    lib = _load()
    c = (_ct.c_uint32 * 4)(*ctr)
    k = (_ct.c_uint32 * 2)(*key)
    o = (_ct.c_uint32 * 4)()
    lib.oracle_philox4x32_10(c, k, o)
    return tuple(o)


def sample_xi(seed: int, level: int, first: int, count: int, dim: int = 3) -> np.ndarray:
    lib = _load()
    out = np.empty((count, dim), np.float64)
    lib.oracle_sample_xi(seed, level, first, count, dim, _dp(out))
    return out


def fields_closed(phys, nx, ny, xi):
    lib = _load()
    phi = np.empty((ny, nx)); K = np.empty((ny, nx)); q = np.empty(1)
    _check(lib.oracle_fields_closed(_ct.byref(phys_struct(phys)), nx, ny, _dp(_f64(xi)), _dp(phi), _dp(K),
                                    _dp(q)), "fields")
    return phi, K, float(q[0])


def fields_two_layer(phys, nx, ny, xi):
    """The paper's own random inputs (Sec. 4: eq:poro_2levels,
    eq:poro_2levels_C; Sec. 2.2: e_perm_Kozeny_Carman), at cell centres:
    porosity in two horizontal layers split at y = -0.75, each scaled by its
    own factor C0(xi1); a Kozeny-Carman permeability whose scale makes
    K(phi0) = k0; the recharge with a +-50 % amplitude."""
    h = 1.0 / ny
    x = (np.arange(nx) + 0.5) * h
    y = -1.0 + (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(x, y, indexing="xy")
    x1, x2, x3 = (float(v) for v in xi)
    C0 = np.where(Y < -0.75, 1.0 + 0.2 * x1, 1.0 - 0.2 * x1)
    phi = phys["phi0"] * (1.0 + 0.15 * (x2 * np.cos(np.pi * X / 2) + x2 * np.sin(2 * np.pi * Y)
                                        + x1 * np.cos(2 * np.pi * X))) * C0
    kappa = phys["k0"] * (1.0 - phys["phi0"] ** 2) / phys["phi0"] ** 3
    K = kappa * phi ** 3 / (1.0 - phi ** 2)
    return phi, K, phys["q_in"] * (1.0 + 0.5 * x3)


def field_derivs_two_layer(phys, nx, ny, xi):
    """d(phi)/d(xi_k) and d(K)/d(xi_k) per cell for k = 1, 2 ([2][ny][nx]
    each) and d(q)/d(xi3) of the two-layer model, by the product and chain
    rules on fields_two_layer's formulas."""
    h = 1.0 / ny
    x = (np.arange(nx) + 0.5) * h
    y = -1.0 + (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(x, y, indexing="xy")
    x1, x2 = float(xi[0]), float(xi[1])
    a = np.cos(np.pi * X / 2) + np.sin(2 * np.pi * Y)
    b = np.cos(2 * np.pi * X)
    s = np.where(Y < -0.75, 0.2, -0.2)
    B = 1.0 + 0.15 * (x2 * a + x1 * b)
    C0 = 1.0 + s * x1
    phi0 = phys["phi0"]
    dphi = np.array([phi0 * (0.15 * b * C0 + B * s), phi0 * 0.15 * a * C0])
    phi = phi0 * B * C0
    kappa = phys["k0"] * (1.0 - phi0 ** 2) / phi0 ** 3
    dK_dphi = kappa * (3 * phi ** 2 * (1 - phi ** 2) + 2 * phi ** 4) / (1 - phi ** 2) ** 2
    return dphi, dK_dphi * dphi, phys["q_in"] * 0.5


# ---------------------------------------------------------------- discrete operator
def residual(phys, nsteps, phi, K, q, p, c, cn):
    lib = _load()
    ny, nx = phi.shape
    Rp = np.empty((ny, nx)); Rc = np.empty((ny, nx))
    _check(lib.oracle_residual(_ct.byref(phys_struct(phys)), nx, ny, nsteps, _dp(_f64(phi)), _dp(_f64(K)),
                               float(q), _dp(_f64(p)), _dp(_f64(c)), _dp(_f64(cn)), _dp(Rp), _dp(Rc)), "residual")
    return Rp, Rc


def jacobian_dense(phys, nsteps, phi, K, q, p, c, cn):
    lib = _load()
    ny, nx = phi.shape
    n2 = 2 * nx * ny
    J = np.empty((n2, n2))
    _check(lib.oracle_jacobian_dense(_ct.byref(phys_struct(phys)), nx, ny, nsteps, _dp(_f64(phi)),
                                     _dp(_f64(K)), float(q), _dp(_f64(p)), _dp(_f64(c)), _dp(_f64(cn)),
                                     _dp(J)), "jacobian")
    return J


def band_solve_dense(A, b, kl, ku, trans=False):
    lib = _load()
    A = _f64(A); b = _f64(b)
    x = np.empty_like(b)
    _check(lib.oracle_band_solve_dense(A.shape[0], kl, ku, _dp(A), _dp(b), _dp(x), int(trans)), "band solve")
    return x


def qoi(phys, phi, c):
    lib = _load()
    ny, nx = phi.shape
    return lib.oracle_qoi(_ct.byref(phys_struct(phys)), nx, ny, _dp(_f64(phi)), _dp(_f64(c)))


def cell_to_band(nx, ny):
    """Permutation: band unknown u = 2*(i*ny + j) + v  <->  field index j*nx + i."""
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    return (i * ny + j)  # [ny][nx] -> band cell index


# ---------------------------------------------------------------- solves
def solve(phys, nsteps, phi, K, q, c0=None, trajectory=False):
    """Run the implicit time loop; returns dict(p, c, qoi, iters[, p_traj, c_traj])."""
    lib = _load()
    ny, nx = phi.shape
    p = np.empty((ny, nx)); c = np.empty((ny, nx)); Q = np.empty(1)
    iters = np.zeros(nsteps, np.int32)
    pt = np.empty((nsteps + 1, ny, nx)) if trajectory else None
    ct_ = np.empty((nsteps + 1, ny, nx)) if trajectory else None
    rc = lib.oracle_solve(_ct.byref(phys_struct(phys)), nx, ny, nsteps, _dp(_f64(phi)), _dp(_f64(K)), float(q),
                          _dp(None if c0 is None else _f64(c0)), _dp(p), _dp(c), _dp(Q),
                          iters.ctypes.data_as(_ct.POINTER(_I32)), _dp(pt), _dp(ct_))
    _check(rc, "solve")
    out = dict(p=p, c=c, qoi=float(Q[0]), iters=iters)
    if trajectory:
        out.update(p_traj=pt, c_traj=ct_)
    return out


def solve_xi(phys, nx, ny, nsteps, xi, model=None):
    """Solve with the closed-form fields of xi, or with model="two_layer"
    the two-layer porosity model."""
    fields = fields_two_layer if model == "two_layer" else fields_closed
    phi, K, q = fields(phys, nx, ny, xi)
    return solve(phys, nsteps, phi, K, q)


def solve_many(phys, jobs, threads=None):
    """jobs: list of (nx, ny, nsteps, xi[, model]).  One job per thread
    (ctypes drops the GIL during the C call).  Returns list of result dicts."""
    threads = threads or len(_os.sched_getaffinity(0))
    with _cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda jb: solve_xi(phys, *jb), jobs))


def adjoint(phys, nsteps, phi, K, q):
    """Returns (Q, dQ/dphi [ny][nx], dQ/dK [ny][nx], dQ/dq)."""
    lib = _load()
    ny, nx = phi.shape
    Q = np.empty(1); gphi = np.empty((ny, nx)); gK = np.empty((ny, nx)); gq = np.empty(1)
    _check(lib.oracle_adjoint(_ct.byref(phys_struct(phys)), nx, ny, nsteps, _dp(_f64(phi)), _dp(_f64(K)),
                              float(q), _dp(Q), _dp(gphi), _dp(gK), _dp(gq)), "adjoint")
    return float(Q[0]), gphi, gK, float(gq[0])


def tangent(phys, nsteps, phi, K, q, v_phi, v_K, v_q):
    lib = _load()
    ny, nx = phi.shape
    Q = np.empty(1); dQ = np.empty(1)
    _check(lib.oracle_tangent(_ct.byref(phys_struct(phys)), nx, ny, nsteps, _dp(_f64(phi)), _dp(_f64(K)),
                              float(q), _dp(_f64(v_phi)), _dp(_f64(v_K)), float(v_q), _dp(Q), _dp(dQ)), "tangent")
    return float(Q[0]), float(dQ[0])


def field_derivs_closed(phys, nx, ny, xi):
    """d(phi)/d(xi1) and d(K)/d(xi2) per cell, d(q)/d(xi3): the derivatives
    of the closed-form random fields."""
    h = 1.0 / ny
    x = (np.arange(nx) + 0.5) * h
    y = -1.0 + (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(x, y, indexing="xy")
    dphi = phys["phi0"] * 0.2 * np.cos(np.pi * X / 2) * np.cos(np.pi * Y)
    K = phys["k0"] * np.exp(0.5 * xi[1] * np.sin(np.pi * X / 2))
    dK = K * 0.5 * np.sin(np.pi * X / 2)
    dq = phys["q_in"] * 0.2
    return dphi, dK, dq


def adjoint_xi(phys, nx, ny, nsteps, xi, model=None):
    """Q, dQ/dxi (3,), dQ/dlog K per cell [ny][nx] for the closed-form fields
    (model="two_layer": the two-layer porosity model)."""
    if model == "two_layer":
        phi, K, q = fields_two_layer(phys, nx, ny, xi)
        Q, gphi, gK, gq = adjoint(phys, nsteps, phi, K, q)
        dphi, dK, dq = field_derivs_two_layer(phys, nx, ny, xi)
        g = np.array([(gphi * dphi[k]).sum() + (gK * dK[k]).sum() for k in range(2)] + [gq * dq])
        return Q, g, gK * K
    phi, K, q = fields_closed(phys, nx, ny, xi)
    Q, gphi, gK, gq = adjoint(phys, nsteps, phi, K, q)
    dphi, dK, dq = field_derivs_closed(phys, nx, ny, xi)
    g = np.array([(gphi * dphi).sum(), (gK * dK).sum(), gq * dq])
    return Q, g, gK * K


# ---------------------------------------------------------------- multigrid smoothers
def pressure_operator(te, tn):
    """Sparse matrix of the pressure operator on an [ny][nx] grid (the
    fluid balance's flux form, Sec. 2.3): every interior face couples its
    two cells with its coefficient (east faces te, north faces tn), and the
    last column's te is the seawater face's, on the diagonal only."""
    import scipy.sparse as sp
    ny, nx = te.shape
    rows, cols, vals = [], [], []
    diag = np.zeros(nx * ny)
    for j in range(ny):
        for i in range(nx):
            P = j * nx + i
            if i + 1 < nx:
                E = P + 1
                t = te[j, i]
                rows += [P, E, P, E]; cols += [E, P, P, E]; vals += [-t, -t, t, t]
            else:
                diag[P] += te[j, i]
            if j + 1 < ny:
                N = P + nx
                t = tn[j, i]
                rows += [P, N, P, N]; cols += [N, P, P, N]; vals += [-t, -t, t, t]
    A = sp.coo_matrix((vals, (rows, cols)), shape=(nx * ny, nx * ny)).tocsr()
    return (A + sp.diags(diag)).tocsr()


def transport_operator(acc, mx, my, dx, dy, mr, dr, dl, ml):
    """Sparse matrix of the upwind transport operator on an [ny][nx] grid:
    a cell takes from a neighbour the mass flowing in across their face
    (mx, my: flux leaving the cell east / north) plus the face's diffusion
    (dx, dy); its diagonal is its accumulation plus everything it couples
    to, and on the last and first column the boundary inflow / diffusion
    terms (mr, dr at the sea side, dl, ml at the recharge side)."""
    import scipy.sparse as sp
    ny, nx = acc.shape
    pos = lambda a: max(a, 0.0)
    rows, cols, vals = [], [], []
    for j in range(ny):
        for i in range(nx):
            P = j * nx + i
            d = acc[j, i]
            nb = []
            if i + 1 < nx:
                nb.append((P + 1, pos(-mx[j, i]) + dx[j, i]))
            else:
                d += pos(-mr[j]) + dr[j]
            if i > 0:
                nb.append((P - 1, pos(mx[j, i - 1]) + dx[j, i - 1]))
            else:
                d += dl[j] + ml[j]
            if j + 1 < ny:
                nb.append((P + nx, pos(-my[j, i]) + dy[j, i]))
            if j > 0:
                nb.append((P - nx, pos(my[j - 1, i]) + dy[j - 1, i]))
            for Q, a in nb:
                rows.append(P); cols.append(Q); vals.append(-a)
                d += a
            rows.append(P); cols.append(P); vals.append(d)
    return sp.coo_matrix((vals, (rows, cols)), shape=(nx * ny, nx * ny)).tocsr()


def gauss_seidel_rb(A, b, x, nx, ny, sweeps):
    """Red-black Gauss-Seidel on A x = b: per sweep every red cell
    ((i + j) even) is relaxed, x_P = (b_P - sum_{Q != P} A_PQ x_Q) / A_PP, then
    every black cell with the red values updated."""
    x = np.array(x, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    A = A.tocsr()
    colour = np.add.outer(np.arange(ny), np.arange(nx)).ravel() & 1
    for _ in range(sweeps):
        for col in (0, 1):
            new = x.copy()
            for P in np.flatnonzero(colour == col):
                lo, hi = A.indptr[P], A.indptr[P + 1]
                off = sum(A.data[k] * x[A.indices[k]] for k in range(lo, hi) if A.indices[k] != P)
                new[P] = (b[P] - off) / A[P, P]
            x = new
    return x.reshape(ny, nx)


def zebra_lines(A, b, x, nx, ny, sweeps, ylines=False):
    """Zebra line relaxation on A x = b: per sweep the even lines (rows, or
    columns with ylines), then the odd ones, each solved exactly with the
    other lines held at their current values."""
    x = np.array(x, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    A = A.tocsr()
    nlines = nx if ylines else ny
    for _ in range(sweeps):
        for col in (0, 1):
            for line in range(col, nlines, 2):
                idx = [j * nx + line for j in range(ny)] if ylines else [line * nx + i for i in range(nx)]
                mask = np.zeros(nx * ny, bool)
                mask[idx] = True
                sub = A[idx][:, idx].toarray()
                rhs = b[idx] - A[idx][:, ~mask] @ x[~mask]
                x[idx] = np.linalg.solve(sub, rhs)
    return x.reshape(ny, nx)


# ---------------------------------------------------------------- time series (Sec. 4)
FRESH = 0.012178  # c threshold of the fresh-water indicator in eq:integral_fw


def fresh_area(c, c_fresh=FRESH):
    """eq:integral_fw on the cell grid: the area of the cells with
    c <= c_fresh (cells of area h^2 = 1/ny^2)."""
    ny = c.shape[0]
    return np.count_nonzero(c <= c_fresh) / ny ** 2


def point_value(c, x, y):
    """c [ny][nx] at the point (x, y): the mean over every cell whose closed
    square holds the point (one cell inside, two on a face, four at a
    corner), found by testing each cell, in the cell coordinates
    u = x ny, v = (y + 1) ny."""
    ny, nx = c.shape
    u, v = x * ny, (y + 1.0) * ny
    vals = [c[j, i] for j in range(ny) for i in range(nx) if i <= u <= i + 1 and j <= v <= j + 1]
    return float(np.mean(vals))


def record_steps(nsteps, nrec):
    """Steps after which records k = 1..nrec are taken: the first step at or
    after t = k T / nrec, i.e. ceil(k nsteps / nrec)."""
    return [-(-k * nsteps // nrec) for k in range(1, nrec + 1)]


def trace(phys, nsteps, phi, K, q, nrec, points, c_fresh=FRESH):
    """Time series of one solve: [nrec][1 + len(points)], each record the
    fresh-water area and c at the points, and the solve's result dict."""
    out = solve(phys, nsteps, phi, K, q, trajectory=True)
    rec = []
    for st in record_steps(nsteps, nrec):
        c = out["c_traj"][st]
        rec.append([fresh_area(c, c_fresh)] + [point_value(c, x, y) for x, y in points])
    return np.array(rec), out


def quantile7(x, p):
    """Quantile of Hyndman and Fan's type 7: with the sample sorted
    ascending, x_(lo) + (h - lo)(x_(lo+1) - x_(lo)) at h = (n - 1) p,
    lo = floor(h)."""
    xs = np.sort(np.asarray(x, dtype=np.float64))
    n = len(xs)
    h = (n - 1) * p
    lo = int(np.floor(h))
    hi = min(lo + 1, n - 1)
    return xs[lo] + (h - lo) * (xs[hi] - xs[lo])


def first_passage(series, threshold, below=True):
    """First record k = 1.. of the series below (or above) the threshold;
    0 if none (the first-passage times of Figs. 5 and 7)."""
    for k, a in enumerate(series):
        if (a < threshold) if below else (a > threshold):
            return k + 1
    return 0


# ---------------------------------------------------------------- MLMC statistics (Sec. 3)
def inject(c_coarse, factor):
    """Piecewise-constant injection of a cell field to a grid `factor` times
    finer in each direction: c_fine(f*i + a, f*j + b) = c_coarse(i, j)."""
    return np.repeat(np.repeat(c_coarse, factor, axis=-2), factor, axis=-1)


def level_stats(g_fine, g_coarse=None):
    """Sample mean and unbiased variance of Y_l = g_l - g_{l-1} over the
    first axis (Def. eq:Yell with g_{-1} = 0).  Field-valued coarse samples
    are injected to the fine grid first."""
    g_fine = np.asarray(g_fine, np.float64)
    if g_coarse is None:
        Y = g_fine
    else:
        g_coarse = np.asarray(g_coarse, np.float64)
        if g_fine.ndim == 3:
            Y = g_fine - inject(g_coarse, g_fine.shape[-1] // g_coarse.shape[-1])
        else:
            Y = g_fine - g_coarse
    m = Y.shape[0]
    mean = Y.sum(axis=0) / m
    var = ((Y - mean) ** 2).sum(axis=0) / (m - 1) if m > 1 else np.zeros_like(mean)
    return mean, var


def mlmc_estimate(level_means, level_vars, m):
    """Telescoped E[g_L] = sum_l mean(Y_l) (eq:A), field means injected to
    the finest grid, and the estimator variance sum_l V_l / m_l."""
    L = len(level_means) - 1
    finest = np.asarray(level_means[L])
    if finest.ndim == 2:
        E = np.zeros_like(finest)
        var = np.zeros_like(finest)
        for mean, v, mm in zip(level_means, level_vars, m):
            f = finest.shape[-1] // np.asarray(mean).shape[-1]
            E = E + inject(np.asarray(mean), f)
            var = var + inject(np.asarray(v), f) / mm
    else:
        E = sum(level_means)
        var = sum(np.asarray(v) / mm for v, mm in zip(level_vars, m))
    return E, var


def optimal_samples(V, s, eps2):
    """m_l = ceil(eps^-2 sqrt(V_l/s_l) sum_i sqrt(V_i s_i)) (eq:M_ell) and
    the total cost S = eps^-2 (sum_l sqrt(V_l s_l))^2."""
    V = np.asarray(V, np.float64); s = np.asarray(s, np.float64)
    tot = np.sqrt(V * s).sum()
    m = np.ceil(np.sqrt(V / s) * tot / eps2).astype(np.int64)
    return m, tot * tot / eps2


# ---------------------------------------------------------------- QMC
def radical_inverse(k: int, base: int) -> float:
    """Van der Corput radical inverse: the base-`base` digits of k mirrored
    about the radix point, summed digit by digit (the QMC reference of the
    abstract and of Sec. 4, Fig. 11, whose set-up names Halton points)."""
    f, r = 1.0, 0.0
    while k > 0:
        f /= base
        r += f * (k % base)
        k //= base
    return r


def halton(n: int, dim: int = 3, skip: int = 1) -> np.ndarray:
    """First n Halton points (bases 2, 3, 5, ...) starting at index `skip`."""
    bases = [2, 3, 5, 7, 11, 13][:dim]
    return np.array([[radical_inverse(k, b) for b in bases] for k in range(skip, skip + n)])


def qmc_xi(n: int, dim: int = 3, skip: int = 1, shift=None) -> np.ndarray:
    """Halton points as uniform coefficients on [-1, 1)^dim: each unit-cube
    point rotated by `shift` modulo 1 (a Cranley-Patterson random shift;
    None: no rotation), then mapped by u -> 2u - 1."""
    u = halton(n, dim, skip)
    if shift is not None:
        u = u + np.asarray(shift, dtype=np.float64)
        u = np.where(u >= 1.0, u - 1.0, u)
    return 2.0 * u - 1.0
