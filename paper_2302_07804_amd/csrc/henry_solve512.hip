// henry_solve512.hip -- the FP32-inner solve kernel built for workgroups of
// at most 512 threads.
//
// The same source as henry::henry_solve_kernel<float> (henry_api.hip),
// compiled here in a namespace of its own with 512-thread launch bounds, so
// that the kernel and every device function it calls (the out-of-line line
// solvers too) get up to 256 VGPRs and spill nothing; in one translation
// unit with the 1024-thread build, the shared out-of-line functions would be
// compiled once, for the tighter budget.  henry_api.hip launches it for the
// groups whose solves are shared by clusters when their workgroups have 512
// threads or fewer.  With the registers to spare, its residual pass forms
// the face coefficients of grids of 512 columns or more from K and phi
// (bandwidth-bound passes; it loads them on the smaller grids, where the
// added divisions would lengthen the latency-bound passes), and its
// transfers between levels gather four cells per thread (1024x512 launch:
// 3.7 % and 7.5 % faster, bitwise the same results).
#include <string.h>

#define HENRY_NS henry512
#define HENRY_FP32_THREADS 512
#define HENRY_SOLVE_KERNEL_ONLY
#define HENRY_RES_FIELDS_NX 512
#define HENRY_TRANSFER_BATCH 4
#include "henry_device.hpp"

// Size of this build's launch record (the same struct as henry::Launch,
// from the same header; checked by the caller before a launch).
size_t henry512_launch_bytes() { return sizeof(henry512::Launch); }

// Launches the 512-thread build on `stream`; `launch` points to a
// henry::Launch.  Returns the launch's hipGetLastError().
hipError_t henry512_launch_solve(dim3 grid, dim3 block, size_t lds, hipStream_t stream, const void* launch) {
    henry512::Launch l;
    memcpy(&l, launch, sizeof(l));
    hipLaunchKernelGGL(henry512::henry_solve_kernel<float>, grid, block, lds, stream, l);
    return hipGetLastError();
}
