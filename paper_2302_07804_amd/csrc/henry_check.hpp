// henry_check.hpp -- one multigrid level's smoothing on a caller's linear
// system: the red-black Gauss-Seidel sweeps of the pressure cycle and the
// zebra line sweeps of the transport cycle, the same device functions the
// solves run inside every V-cycle (Sec. 2.3's multigrid-preconditioned
// iteration, redesigned), exposed so that each can be checked on its own.
#pragma once

#include <hip/hip_runtime.h>

#include "henry_device.hpp"

namespace henry {

// kind 0: pressure RB-GS (te, tn; colour-split layout), 1: transport x-line
// zebra sweeps, 2: transport y-line zebra sweeps.  One workgroup; the
// level's arrays in the inner type T live in `ws` (10 n + 4 ny elements).
template <typename T>
__global__ void __launch_bounds__(sizeof(T) == 4 ? 1024 : 512)
    level_smooth_kernel(int nx, int ny, int kind, int sweeps, const double* coef, const double* b, double* x,
                        T* ws) {
    const int n = nx * ny;
    Level<T> v;
    v.nx = nx; v.ny = ny;
    v.x = ws; v.b = ws + n; v.r = ws + 2 * n; v.te = ws + 3 * n; v.tn = ws + 4 * n;
    v.acc = ws + 5 * n; v.mx = ws + 6 * n; v.my = ws + 7 * n; v.dx = ws + 8 * n; v.dy = ws + 9 * n;
    v.mr = ws + 10 * n; v.dr = v.mr + ny; v.dl = v.dr + ny; v.ml = v.dl + ny;
    for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
        const int i = idx % nx, j = idx / nx;
        if (kind == 0) {
            const int s = pidx(i, j, nx);
            v.x[s] = (T)x[idx];
            v.b[s] = (T)b[idx];
            v.te[s] = (T)coef[idx];
            v.tn[s] = j + 1 < ny ? (T)coef[n + idx] : (T)0;  // no face above the top row
        } else {
            v.x[idx] = (T)x[idx];
            v.b[idx] = (T)b[idx];
            v.acc[idx] = (T)coef[idx];
            v.mx[idx] = (T)coef[n + idx];
            v.my[idx] = (T)coef[2 * n + idx];
            v.dx[idx] = (T)coef[3 * n + idx];
            v.dy[idx] = (T)coef[4 * n + idx];
        }
    }
    if (kind != 0)
        for (int j = threadIdx.x; j < ny; j += blockDim.x) {
            v.mr[j] = (T)coef[5 * n + j];
            v.dr[j] = (T)coef[5 * n + ny + j];
            v.dl[j] = (T)coef[5 * n + 2 * ny + j];
            v.ml[j] = (T)coef[5 * n + 3 * ny + j];
        }
    __syncthreads();
    if (kind == 0) {
        rbgs<T, BlockTeam, 1>(v, sweeps);
    } else {
        for (int s = 0; s < sweeps; ++s) {
            line_smooth<T, false, BlockTeam, 1>(v, kind == 2);
            __syncthreads();
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
        const int i = idx % nx, j = idx / nx;
        x[idx] = (double)v.x[kind == 0 ? pidx(i, j, nx) : idx];
    }
}

}  // namespace henry
