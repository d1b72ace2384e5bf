// henry_adjoint.hpp -- discrete adjoint of the batched Henry solves.
//
// For the implicit steps R^n(u^n, c^{n-1}; theta) = 0, n = 1..N, and the
// QoI Q(c^N; phi) (salt mass in x < 1), the gradient is
//   dQ/dtheta = dQ/dtheta|explicit - sum_n (lam^n)^T dR^n/dtheta,
// with (J^N)^T lam^N = (dQ/du^N)^T and
//      (J^n)^T lam^n = -(dR^{n+1}/dc^n)^T lam^{n+1}   (diagonal coupling),
// J^n = dR^n/du^n the exact step Jacobian.  theta: per-cell K (reported as
// d/dlog K), per-cell phi, the recharge q, and through the closed-form
// fields the three xi.
//
// Each transposed system is solved by FP64 defect correction with the exact
// J^T product (hand-derived flux derivatives below).  With E = [[I,0],[-C,I]]
// (C = diag c, the recombination S = R^c - c R^p of the forward solve),
// lam = E^T mu turns J^T lam = b into (E J)^T mu = b, whose diagonal blocks
// are the pressure operator (symmetric) and the non-conservative transport
// operator; they are preconditioned by the forward V-cycles, the transport
// one with the transposed stencil.  The salt block goes first, then the
// pressure block on the recomputed residual.
//
// Time reversal by checkpointing: the forward pass stores its state every
// `ckpt` steps, with the four older states and the counter its
// extrapolated initial guess draws on; each segment is recomputed from its
// checkpoint (bitwise the same states) and then walked backwards.
#pragma once

#include "henry_device.hpp"

namespace henry {

struct AdjLaunch {
    int32_t ckpt;       // checkpoint interval (steps)
    int32_t max_it;     // transposed defect-correction iterations per step
    double tol;         // relative tolerance of the transposed residual
    double* dq_dxi;     // [nsolves][3] or null (closed-form fields)
    double* dq_dlogk;   // packed per cell or null
    double* dq_dphi;    // packed per cell or null
    double* dq_dq;      // [nsolves] or null
};

__host__ __device__ inline int num_ckpts(int nsteps, int k) { return (nsteps + k - 1) / k; }

// Doubles per checkpoint: p, c and the extrapolation history pp, cn, p2,
// c2, p3, c3, p4, c4 (n each), then the converged-state counter (8 doubles).
__host__ __device__ inline int64_t ckpt_doubles(int64_t n) { return 10 * n + 8; }

// FP64 adjoint region: mu_p, mu_c, lam_p, lam_c, dinv_p, dinv_c (inverse
// diagonals of the two blocks at the current step, for the scaled norm),
// b_p, b_c, gK, gphi (n each), the three previous steps' mu (mh: p1, c1,
// p2, c2, p3, c3, n each; the extrapolated start of the transposed
// solves), 8 doubles of scratch, checkpoints (ncp x ckpt_doubles), segment
// states ((k+1) x 2n).
__host__ __device__ inline int64_t adjoint_bytes(int nx, int ny, int nsteps, int k) {
    const int64_t n = (int64_t)nx * ny;
    const int64_t ncp = num_ckpts(nsteps, k);
    return align256(8 * (16 * n + 8 + ncp * ckpt_doubles(n) + (int64_t)(k + 1) * 2 * n));
}

struct Adj {
    double *mu_p, *mu_c, *lam_p, *lam_c, *dinv_p, *dinv_c, *b_p, *b_c, *gK, *gphi, *mh, *scr, *ckpt, *seg;
    int k, ncp;
};

__device__ inline void bind_adj(Adj& A, uint8_t* base, int n, int nsteps, int k) {
    double* f = reinterpret_cast<double*>(base);
    A.mu_p = f; A.mu_c = f + n; A.lam_p = f + 2 * n; A.lam_c = f + 3 * n; A.dinv_p = f + 4 * n;
    A.dinv_c = f + 5 * n;
    A.b_p = f + 6 * n; A.b_c = f + 7 * n; A.gK = f + 8 * n; A.gphi = f + 9 * n; A.mh = f + 10 * n;
    A.scr = f + 16 * n;
    A.k = k;
    A.ncp = num_ckpts(nsteps, k);
    A.ckpt = f + 16 * n + 8;
    A.seg = A.ckpt + (int64_t)A.ncp * ckpt_doubles(n);
}

// ------------------------------------------------------------------ flux derivatives (FP64)
// Derivatives of the flux from cell a to its east (kVertical = false) or
// north (kVertical = true) neighbour b with respect to the states of both
// cells, and with kGrad also to their K and phi; the same flux as the
// residual's (kf = K_f / mu and wf = phi_f D are the precomputed face
// coefficients; K and phi enter only the kGrad derivatives of the harmonic
// means).
struct FaceDer {
    double M, F;
    double Mpa, Mpb, Mca, Mcb;
    double Fpa, Fpb, Fca, Fcb;
    double MKa, MKb, FKa, FKb;
    double Fphia, Fphib;
};

template <bool kVertical, bool kGrad>
__device__ inline FaceDer face_der(const Phys& ph, double h, double pa, double pb, double ca, double cb, double kf,
                                   double wf, double Ka, double Kb, double fa, double fb) {
    FaceDer d;
    const double dr = ph.rho1 - ph.rho0;
    const double rf = 0.5 * (rho_of(ph, ca) + rho_of(ph, cb));
    const double lam = rf * kf, dlam = 0.5 * dr * kf;  // d lam / d c_a = d lam / d c_b
    const double dif = rf * wf, ddif = 0.5 * dr * wf;
    double gr = pb - pa, dgr = 0.0;
    if constexpr (kVertical) {
        gr += rf * ph.g * h;
        dgr = 0.5 * dr * ph.g * h;
    }
    d.M = -lam * gr;
    d.Mpa = lam;
    d.Mpb = -lam;
    d.Mca = -(dlam * gr + lam * dgr);
    d.Mcb = d.Mca;
    const bool upa = d.M >= 0.0;
    const double cup = upa ? ca : cb;
    d.F = d.M * cup - dif * (cb - ca);
    d.Fpa = d.Mpa * cup;
    d.Fpb = d.Mpb * cup;
    d.Fca = d.Mca * cup + (upa ? d.M : 0.0) - ddif * (cb - ca) + dif;
    d.Fcb = d.Mcb * cup + (upa ? 0.0 : d.M) - ddif * (cb - ca) - dif;
    if constexpr (kGrad) {
        const double sK = Ka + Kb, sf = fa + fb;
        const double dKa = 2.0 * Kb * Kb / (sK * sK), dKb = 2.0 * Ka * Ka / (sK * sK);
        d.MKa = -(rf / ph.mu) * gr * dKa;
        d.MKb = -(rf / ph.mu) * gr * dKb;
        d.FKa = d.MKa * cup;
        d.FKb = d.MKb * cup;
        const double dfa = 2.0 * fb * fb / (sf * sf), dfb = 2.0 * fa * fa / (sf * sf);
        d.Fphia = -rf * ph.D * dfa * (cb - ca);
        d.Fphib = -rf * ph.D * dfb * (cb - ca);
    } else {
        d.MKa = d.MKb = d.FKa = d.FKb = d.Fphia = d.Fphib = 0.0;
    }
    return d;
}

// Seawater face (kf = 2 K_P / mu, wf = 2 phi_P D): derivatives with respect
// to the cell's own p, c, and with kGrad K, phi.
struct BndDer { double Mp, Mc, Fp, Fc, MK, FK, Fphi; };

template <bool kGrad>
__device__ inline BndDer right_der(const Phys& ph, double y, double pP, double cP, double kf, double wf) {
    BndDer d;
    const double dr = ph.rho1 - ph.rho0;
    const double rB = 0.5 * (rho_of(ph, cP) + ph.rho1);
    const double lamB = rB * kf;
    const double gB = -ph.rho1 * ph.g * y - pP;
    const double M = -lamB * gB;
    d.Mp = lamB;
    d.Mc = -(0.5 * dr * kf) * gB;
    const bool up = M >= 0.0;
    const double cup = up ? cP : 1.0;
    const double dif = rB * wf, ddif = 0.5 * dr * wf;
    d.Fp = d.Mp * cup;
    d.Fc = d.Mc * cup + (up ? M : 0.0) - ddif * (1.0 - cP) + dif;
    if constexpr (kGrad) {
        d.MK = -(2.0 * rB / ph.mu) * gB;
        d.FK = d.MK * cup;
        d.Fphi = -2.0 * rB * ph.D * (1.0 - cP);
    } else {
        d.MK = d.FK = d.Fphi = 0.0;
    }
    return d;
}

// Recharge face: the mass flux -rho0 q h depends on q only; the salt flux
// 2 rho_B phi D c_P on c and phi.
__device__ inline BndDer left_der(const Phys& ph, double cP, double fP) {
    BndDer d;
    const double dr = ph.rho1 - ph.rho0;
    const double rB = 0.5 * (rho_of(ph, cP) + ph.rho0);
    d.Mp = 0.0; d.Mc = 0.0; d.Fp = 0.0; d.MK = 0.0; d.FK = 0.0;
    d.Fc = dr * fP * ph.D * cP + 2.0 * rB * fP * ph.D;
    d.Fphi = 2.0 * rB * ph.D * cP;
    return d;
}

// ------------------------------------------------------------------ J^T lam and gradients
// kGrad = false: r = b - J^T lam (lam from mu), scaled max norm returned;
//                the inner rhs of the requested block is written to level 0.
// kGrad = true:  gradient accumulation g -= lam^T dR/dtheta and the rhs of
//                the previous step.
// Every operand is loaded from clamped indices first; the interior and the
// boundary form of the east and west faces are both formed and selected.
template <typename T, bool kGrad>
__device__ double jt_pass(const Phys& ph, Solve<T>& S, Adj& A, double* red, int block) {
    const int nx = S.nx, ny = S.ny, n = S.n;
    const double h = S.h, h2t = h * h / S.tau;
    const double dr = ph.rho1 - ph.rho0;
    const double* p = S.p;
    const double* c = S.c;
    const double* lp = A.lam_p;
    const double* lc = A.lam_c;
    Level<T>& L0 = S.lv[0];
    const int sx = log2i(nx);
    double rmax = 0.0;
    const int rk = ClusterTeam::rank(), ts = ClusterTeam::size();
    for (int idx = rk; idx < n; idx += ts) {
        const int i = idx & (nx - 1), j = idx >> sx;
        const Nb q(i, j, nx, ny);
        const double cP = c[idx], cnP = S.cn[idx], fP = S.phi[idx], pP = p[idx];
        const double lpP = lp[idx], lcP = lc[idx];
        const double pE = p[q.e], cE = c[q.e], lpE = lp[q.e], lcE = lc[q.e];
        const double pW = p[q.w], cW = c[q.w], lpW = lp[q.w], lcW = lc[q.w];
        const double pN = p[q.n], cN = c[q.n], lpN = lp[q.n], lcN = lc[q.n];
        const double pS = p[q.s], cS = c[q.s], lpS = lp[q.s], lcS = lc[q.s];
        const double txP = S.tx[idx], wxP = S.wx[idx], tyP = S.ty[idx], wyP = S.wy[idx];
        const double txW = S.tx[q.w], wxW = S.wx[q.w], tyS = S.ty[q.s], wyS = S.wy[q.s];
        double KP = 0.0, KE = 0.0, KW = 0.0, KN = 0.0, KS = 0.0, fE = 0.0, fW = 0.0, fN = 0.0, fS = 0.0;
        if constexpr (kGrad) {
            KP = S.K[idx]; KE = S.K[q.e]; KW = S.K[q.w]; KN = S.K[q.n]; KS = S.K[q.s];
            fE = S.phi[q.e]; fW = S.phi[q.w]; fN = S.phi[q.n]; fS = S.phi[q.s];
        }
        double jp = 0.0, jc = 0.0;       // (J^T lam) at p_P, c_P
        double gK = 0.0, gf = 0.0;       // lam^T dR/dK_P, lam^T dR/dphi_P
        // stored mass
        jc += lpP * h2t * fP * dr + lcP * h2t * fP * (ph.rho0 + 2.0 * dr * cP);
        if constexpr (kGrad)
            gf += lpP * h2t * (rho_of(ph, cP) - rho_of(ph, cnP)) +
                  lcP * h2t * (rho_of(ph, cP) * cP - rho_of(ph, cnP) * cnP);
        // east: P = a, or the seawater face
        {
            const FaceDer d = face_der<false, kGrad>(ph, h, pP, pE, cP, cE, txP, wxP, KP, KE, fP, fE);
            const BndDer b = right_der<kGrad>(ph, -1.0 + (j + 0.5) * h, pP, cP, txP, wxP);
            const double wp = lpP - lpE, wc = lcP - lcE;
            jp += q.he ? wp * d.Mpa + wc * d.Fpa : lpP * b.Mp + lcP * b.Fp;
            jc += q.he ? wp * d.Mca + wc * d.Fca : lpP * b.Mc + lcP * b.Fc;
            if constexpr (kGrad) {
                gK += q.he ? wp * d.MKa + wc * d.FKa : lpP * b.MK + lcP * b.FK;
                gf += q.he ? wc * d.Fphia : lcP * b.Fphi;
            }
        }
        // west: P = b, or the recharge face
        {
            const FaceDer d = face_der<false, kGrad>(ph, h, pW, pP, cW, cP, txW, wxW, KW, KP, fW, fP);
            const BndDer b = left_der(ph, cP, fP);
            const double wp = lpW - lpP, wc = lcW - lcP;
            jp += q.hw ? wp * d.Mpb + wc * d.Fpb : 0.0;
            jc += q.hw ? wp * d.Mcb + wc * d.Fcb : lcP * b.Fc;
            if constexpr (kGrad) {
                gK += q.hw ? wp * d.MKb + wc * d.FKb : 0.0;
                gf += q.hw ? wc * d.Fphib : lcP * b.Fphi;
            }
        }
        // north: P = a (nothing across the top)
        {
            const FaceDer d = face_der<true, kGrad>(ph, h, pP, pN, cP, cN, tyP, wyP, KP, KN, fP, fN);
            const double wp = lpP - lpN, wc = lcP - lcN;
            jp += q.hn ? wp * d.Mpa + wc * d.Fpa : 0.0;
            jc += q.hn ? wp * d.Mca + wc * d.Fca : 0.0;
            if constexpr (kGrad) {
                gK += q.hn ? wp * d.MKa + wc * d.FKa : 0.0;
                gf += q.hn ? wc * d.Fphia : 0.0;
            }
        }
        // south: P = b (nothing across the bottom)
        {
            const FaceDer d = face_der<true, kGrad>(ph, h, pS, pP, cS, cP, tyS, wyS, KS, KP, fS, fP);
            const double wp = lpS - lpP, wc = lcS - lcP;
            jp += q.hs ? wp * d.Mpb + wc * d.Fpb : 0.0;
            jc += q.hs ? wp * d.Mcb + wc * d.Fcb : 0.0;
            if constexpr (kGrad) {
                gK += q.hs ? wp * d.MKb + wc * d.FKb : 0.0;
                gf += q.hs ? wc * d.Fphib : 0.0;
            }
        }
        if constexpr (!kGrad) {
            const double rp = A.b_p[idx] - jp, rc = A.b_c[idx] - jc;
            // norm in units of the local diagonal of each block
            rmax = nanmax(rmax, fabs(rp) * A.dinv_p[idx]);
            rmax = nanmax(rmax, fabs(rc) * A.dinv_c[idx]);
            // the pressure cycle's arrays are colour-split, the transport's natural
            const int at = block == 0 ? pidx(i, j, nx) : idx;
            L0.b[at] = (T)(block == 0 ? rp : rc);
            L0.x[at] = (T)0;
        } else {
            A.gK[idx] -= gK;
            A.gphi[idx] -= gf;
            // rhs of the previous step: -(dR^n/dc^{n-1})^T lam^n
            A.b_p[idx] = 0.0;
            A.b_c[idx] = lpP * h2t * fP * dr + lcP * h2t * fP * (ph.rho0 + 2.0 * dr * cnP);
        }
    }
    if constexpr (!kGrad) {
        double r, unused;
        cluster_max2(rmax, 0.0, red, r, unused);
        return r;
    }
    // lam^T dR/dq: the recharge faces of the first column, summed by the
    // leader in the order of a one-workgroup pass (thread t adds the cells
    // t, t + blockDim, ... in turn), so the sum is the same for every
    // cluster size
    if (g_cl.member == 0) {
        double gq = 0.0;
        for (int j = 0; j < ny; ++j) {
            const int idx = j * nx;
            if ((idx & ((int)blockDim.x - 1)) == (int)threadIdx.x) gq += lp[idx] * (-ph.rho0 * h);
        }
        const double g = block_sum(gq, red);
        if (threadIdx.x == 0) A.scr[0] -= g;
    }
    ClusterTeam::sync();
    return 0.0;
}

// lam = E^T mu: lam_p = mu_p - c mu_c, lam_c = mu_c.
template <typename T>
__device__ void lam_from_mu(Solve<T>& S, Adj& A) {
    for (int idx = ClusterTeam::rank(); idx < S.n; idx += ClusterTeam::size()) {
        A.lam_p[idx] = A.mu_p[idx] - S.c[idx] * A.mu_c[idx];
        A.lam_c[idx] = A.mu_c[idx];
    }
    ClusterTeam::sync();
}

// Start of the next transposed solve: the polynomial extrapolation of order
// `order` (0..3) of mu through the last solves (as the forward steps'
// initial guess), shifting the history.
template <typename T>
__device__ void mu_extrapolate(const Solve<T>& S, Adj& A, int order) {
    const int n = S.n;
    double* h1p = A.mh; double* h1c = A.mh + n;
    double* h2p = A.mh + 2 * n; double* h2c = A.mh + 3 * n;
    double* h3p = A.mh + 4 * n; double* h3c = A.mh + 5 * n;
    for (int idx = ClusterTeam::rank(); idx < n; idx += ClusterTeam::size()) {
        const double p0 = A.mu_p[idx], c0 = A.mu_c[idx];
        const double p1 = h1p[idx], c1 = h1c[idx], p2 = h2p[idx], c2 = h2c[idx];
        if (order == 1) {
            A.mu_p[idx] = 2.0 * p0 - p1;
            A.mu_c[idx] = 2.0 * c0 - c1;
        } else if (order == 2) {
            A.mu_p[idx] = 3.0 * p0 - 3.0 * p1 + p2;
            A.mu_c[idx] = 3.0 * c0 - 3.0 * c1 + c2;
        } else if (order == 3) {
            A.mu_p[idx] = 4.0 * p0 - 6.0 * p1 + 4.0 * p2 - h3p[idx];
            A.mu_c[idx] = 4.0 * c0 - 6.0 * c1 + 4.0 * c2 - h3c[idx];
        }
        h3p[idx] = p2; h3c[idx] = c2;
        h2p[idx] = p1; h2c[idx] = c1;
        h1p[idx] = p0; h1c[idx] = c0;
    }
    ClusterTeam::sync();
}

// One transposed step solve at the state in S (p^n, c^n; c^{n-1} in S.cn)
// for the rhs in A.b; mu holds the previous step's solution as the initial
// guess.  Returns 0 converged, 1 not converged, 2 non-finite.
template <typename T>
__device__ int adjoint_step(const Phys& ph, Solve<T>& S, Adj& A, double* red, int max_it, double tol,
                            double& iters) {
    double np, nc;
    residual_pass(ph, S, 0, red, np, nc);
    coarsen_pressure(S);
    residual_pass(ph, S, 1, red, np, nc);
    coarsen_transport(S);
    // scaled norm of the rhs
    // (and the inverse block diagonals of this step for the norms)
    double bm = 0.0;
    for (int idx = ClusterTeam::rank(); idx < S.n; idx += ClusterTeam::size()) {
        const int i = idx % S.nx, j = idx / S.nx;
        const double ip = 1.0 / (double)pstencil(S.lv[0], NbS(i, j, S.nx, S.ny)).d;
        const double ic = 1.0 / (double)cstencil_t(S.lv[0], Nb(i, j, S.nx, S.ny), j).d;
        A.dinv_p[idx] = ip;
        A.dinv_c[idx] = ic;
        bm = nanmax(bm, fabs(A.b_p[idx]) * ip);
        bm = nanmax(bm, fabs(A.b_c[idx]) * ic);
    }
    {
        double unused;
        cluster_max2(bm, 0.0, red, bm, unused);
    }
    if (!(bm == bm)) return 2;
    int st = 1;
    for (int it = 0; it < max_it; ++it) {
        lam_from_mu(S, A);
        const double rn = jt_pass<T, false>(ph, S, A, red, 1);
        if (!(rn == rn)) { st = 2; break; }
        if (rn <= tol * bm) { st = 0; break; }
        iters += 1.0;
        vcycle<T, true, true>(S);
        for (int idx = ClusterTeam::rank(); idx < S.n; idx += ClusterTeam::size())
            A.mu_c[idx] += (double)S.lv[0].x[idx];
        ClusterTeam::sync();
        lam_from_mu(S, A);
        jt_pass<T, false>(ph, S, A, red, 0);
        vcycle<T, false>(S);
        for (int idx = ClusterTeam::rank(); idx < S.n; idx += ClusterTeam::size())
            A.mu_p[idx] += (double)S.lv[0].x[pidx(idx % S.nx, idx / S.nx, S.nx)];
        ClusterTeam::sync();
    }
    lam_from_mu(S, A);
    return st;
}

template <typename T>
__device__ void save_state(const Solve<T>& S, double* dst) {
    for (int idx = ClusterTeam::rank(); idx < S.n; idx += ClusterTeam::size()) {
        dst[idx] = S.p[idx];
        dst[S.n + idx] = S.c[idx];
    }
    ClusterTeam::sync();
}

// Checkpoint: the state and the extrapolation history before a step, and
// the count of converged states in a row.
template <typename T>
__device__ void save_ckpt(const Solve<T>& S, double* dst, int good) {
    const int n = S.n;
    for (int idx = ClusterTeam::rank(); idx < n; idx += ClusterTeam::size()) {
        dst[idx] = S.p[idx];
        dst[n + idx] = S.c[idx];
        dst[2 * n + idx] = S.pp[idx];
        dst[3 * n + idx] = S.cn[idx];
        dst[4 * n + idx] = S.p2[idx];
        dst[5 * n + idx] = S.c2[idx];
        dst[6 * n + idx] = S.p3[idx];
        dst[7 * n + idx] = S.c3[idx];
        dst[8 * n + idx] = S.p4[idx];
        dst[9 * n + idx] = S.c4[idx];
    }
    if (g_cl.member == 0 && threadIdx.x == 0) dst[10 * n] = (double)good;
    ClusterTeam::sync();
}

template <typename T>
__device__ int load_ckpt(Solve<T>& S, const double* src) {
    const int n = S.n;
    for (int idx = ClusterTeam::rank(); idx < n; idx += ClusterTeam::size()) {
        S.p[idx] = src[idx];
        S.c[idx] = src[n + idx];
        S.pp[idx] = src[2 * n + idx];
        S.cn[idx] = src[3 * n + idx];
        S.p2[idx] = src[4 * n + idx];
        S.c2[idx] = src[5 * n + idx];
        S.p3[idx] = src[6 * n + idx];
        S.c3[idx] = src[7 * n + idx];
        S.p4[idx] = src[8 * n + idx];
        S.c4[idx] = src[9 * n + idx];
    }
    ClusterTeam::sync();
    return (int)src[10 * n];
}

// Extrapolation order of a transposed solve's start after `good` converged
// solutions in a row (polynomials through up to four, mu_extrapolate).
__device__ inline int mu_order(int good) { return good - 1 < 3 ? (good - 1 > 0 ? good - 1 : 0) : 3; }

template <typename T>
__device__ void load_state(Solve<T>& S, const double* src, const double* prev) {
    for (int idx = ClusterTeam::rank(); idx < S.n; idx += ClusterTeam::size()) {
        S.p[idx] = src[idx];
        S.c[idx] = src[S.n + idx];
        if (prev) S.cn[idx] = prev[S.n + idx];
    }
    ClusterTeam::sync();
}

// ------------------------------------------------------------------ the adjoint kernel
template <typename T>
__global__ void __launch_bounds__(512) henry_adjoint_kernel(Launch lp, AdjLaunch al) {
    extern __shared__ __align__(256) uint8_t lds_levels[];
    __shared__ Solve<T> S;
    __shared__ Adj A;
    __shared__ double red[32];
    int cid, member;
    cluster_of_block(lp.cluster, cid, member);
    if (cid >= lp.nsolves) return;
    const SolveDesc d = lp.descs[cid];
    const Phys& ph = lp.ph;
    if (threadIdx.x == 0) {
        bind_solve(S, lp.ws + d.ws_off, d.nx, d.ny, lds_levels, lp.lds_cells, lp.lds_block_cells);
        set_cluster_levels(S, lp.cluster);
        S.nsteps = d.nsteps;
        S.tau = ph.T / d.nsteps;
        S.q = S.scratch[0];
        bind_adj(A, lp.ws + d.adj_off, d.nx * d.ny, d.nsteps, al.ckpt);
    }
    __syncthreads();
    if (lp.cluster > 1) cluster_init(lp.cluster, member, S.scratch, lp.cluster_wait);
    else cluster_init_single();
    // no line staging here: the transposed cycles reuse the LDS levels'
    // coefficients from one cycle to the next, so nothing may overlay them
    if (threadIdx.x == 0) cluster_stage(lds_levels, 0, line_stage_bytes_per_wave<T>());
    const int n = S.n, N = d.nsteps, k = A.k;
    PhaseClock pc;
    pc.init();
    double fiters = 0.0, aiters = 0.0;
    int status = 0;
    // ---- forward pass with checkpoints (each step starts from the same
    // extrapolated guess as the forward solve kernel's)
    const int64_t ck = ckpt_doubles(n);
    const int top = max_order(lp.predictor, N, lp.tol);
    initial_state(ph, S, nullptr);
    ClusterTeam::sync();
    int good = 1;
    for (int s = 0; s < N && !g_cl.failed; ++s) {
        if (s % k == 0) save_ckpt(S, A.ckpt + (int64_t)(s / k) * ck, good);
        const int st = implicit_step(ph, S, red, lp.max_outer, lp.tol, fiters, pc, start_order(good, top));
        if (st == 2) { status = 2; break; }
        if (st == 1 && status == 0) status = 1;
        good = next_good(good, st);
    }
    // (the leader's block reduction, as with one workgroup)
    const double Q = member == 0 ? qoi_of(ph, S, red) : 0.0;
    // ---- adjoint initial conditions: dQ/du^N and the explicit dQ/dphi
    const double h2 = S.h * S.h;
    for (int idx = ClusterTeam::rank(); idx < n; idx += ClusterTeam::size()) {
        const bool left = (idx % S.nx) < S.nx / 2;
        const double cP = S.c[idx];
        A.b_p[idx] = 0.0;
        A.b_c[idx] = left ? h2 * S.phi[idx] * (ph.rho0 + 2.0 * (ph.rho1 - ph.rho0) * cP) : 0.0;
        A.mu_p[idx] = 0.0;
        A.mu_c[idx] = 0.0;
        A.gK[idx] = 0.0;
        A.gphi[idx] = left ? h2 * rho_of(ph, cP) * cP : 0.0;
    }
    if (member == 0 && threadIdx.x == 0) A.scr[0] = 0.0;
    ClusterTeam::sync();
    // ---- reverse sweep over the checkpoint segments (each transposed solve
    // starts from mu extrapolated through the previous solutions; the zero
    // start of the first solve is not one of them)
    int agood = 0;
    for (int seg = A.ncp - 1; seg >= 0 && status != 2 && !g_cl.failed; --seg) {
        const int s0 = seg * k, s1 = min(N, s0 + k);
        int g = load_ckpt(S, A.ckpt + (int64_t)seg * ck);
        save_state(S, A.seg);
        for (int s = s0; s < s1; ++s) {
            double dummy = 0.0;
            const int st = implicit_step(ph, S, red, lp.max_outer, lp.tol, dummy, pc, start_order(g, top));
            g = next_good(g, st);
            save_state(S, A.seg + (int64_t)(s - s0 + 1) * 2 * n);
        }
        for (int m = s1; m > s0; --m) {
            load_state(S, A.seg + (int64_t)(m - s0) * 2 * n, A.seg + (int64_t)(m - 1 - s0) * 2 * n);
            mu_extrapolate(S, A, mu_order(agood));
            const int st = adjoint_step(ph, S, A, red, al.max_it, al.tol, aiters);
            agood = st == 0 ? (agood < 4 ? agood + 1 : 4) : 0;
            if (st == 2) { status = 2; break; }
            if (st == 1 && status == 0) status = 1;
            jt_pass<T, true>(ph, S, A, red, 0);
        }
    }
    // ---- outputs, by the leader alone: its sums take the cells in the
    // order of a one-workgroup solve
    ClusterTeam::sync();
    if (g_cl.failed) status = 3;
    if (member != 0) return;
    const double gq = A.scr[0];
    const double h = S.h;
    double g1 = 0.0, g2 = 0.0;
    const double x1 = lp.field_kind == 3 ? lp.xi[3 * d.index] : 0.0;
    const double x2 = lp.field_kind == 3 ? lp.xi[3 * d.index + 1] : 0.0;
    const double kappa = ph.k0 * (1.0 - ph.phi0 * ph.phi0) / (ph.phi0 * ph.phi0 * ph.phi0);
    for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
        const double KP = S.K[idx];
        if (al.dq_dlogk) al.dq_dlogk[d.field_off + idx] = A.gK[idx] * KP;
        if (al.dq_dphi) al.dq_dphi[d.field_off + idx] = A.gphi[idx];
        if (lp.field_kind == 0) {
            const int i = idx % S.nx, j = idx / S.nx;
            const double x = (i + 0.5) * h, y = -1.0 + (j + 0.5) * h;
            // derivatives of the closed-form fields with respect to xi1, xi2
            g1 += A.gphi[idx] * ph.phi0 * 0.2 * cos(M_PI * x / 2.0) * cos(M_PI * y);
            g2 += A.gK[idx] * KP * 0.5 * sin(M_PI * x / 2.0);
        } else if (lp.field_kind == 3) {
            // two-layer porosity: phi = phi0 B C0 with B = 1 + 0.15 (xi2 a + xi1 b),
            // C0 = 1 +- 0.2 xi1; K = kappa phi^3 / (1 - phi^2), so
            // dK/dphi = kappa phi^2 (3 - phi^2) / (1 - phi^2)^2
            const int i = idx % S.nx, j = idx / S.nx;
            const double x = (i + 0.5) * h, y = -1.0 + (j + 0.5) * h;
            const double a = cos(M_PI * x / 2.0) + sin(2.0 * M_PI * y), b = cos(2.0 * M_PI * x);
            const double sg = y < -0.75 ? 0.2 : -0.2;
            const double B = 1.0 + 0.15 * (x2 * a + x1 * b), C0 = 1.0 + sg * x1;
            const double fP = S.phi[idx], f2 = fP * fP;
            const double gphi = A.gphi[idx] + A.gK[idx] * kappa * f2 * (3.0 - f2) / ((1.0 - f2) * (1.0 - f2));
            g1 += gphi * ph.phi0 * (0.15 * b * C0 + B * sg);
            g2 += gphi * ph.phi0 * 0.15 * a * C0;
        }
    }
    g1 = block_sum(g1, red);
    g2 = block_sum(g2, red);
    if (lp.field_kind == 2 && al.dq_dxi) {
        // KL coefficients: dphi/dxi_k = phi0 s_phi m_k, dK/dxi_{20+k} = K s_K m_k
        for (int k = 0; k < 20; ++k) {
            double ap = 0.0, ak = 0.0;
            for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
                const double m = lp.kl_modes[(size_t)k * n + idx];
                ap += A.gphi[idx] * m;
                ak += A.gK[idx] * S.K[idx] * m;
            }
            ap = block_sum(ap, red);
            ak = block_sum(ak, red);
            if (threadIdx.x == 0) {
                al.dq_dxi[41 * d.index + k] = ap * ph.phi0 * lp.kl_sigma_phi;
                al.dq_dxi[41 * d.index + 20 + k] = ak * lp.kl_sigma_logk;
            }
        }
        if (threadIdx.x == 0) al.dq_dxi[41 * d.index + 40] = gq * ph.q_in * 0.2;
    }
    if (threadIdx.x == 0) {
        lp.qoi_out[d.index] = Q;
        lp.status[d.index] = status;
        if (lp.iters) lp.iters[d.index] = (int32_t)(fiters + aiters);
        if (al.dq_dq) al.dq_dq[d.index] = gq;
        if (al.dq_dxi && (lp.field_kind == 0 || lp.field_kind == 3)) {
            al.dq_dxi[3 * d.index + 0] = g1;
            al.dq_dxi[3 * d.index + 1] = g2;
            al.dq_dxi[3 * d.index + 2] = gq * ph.q_in * (lp.field_kind == 3 ? 0.5 : 0.2);
        }
    }
}

}  // namespace henry
