// Per-node forward recomputation and its vector-Jacobian product (reverse
// mode), for the adjoint of one time step.  Host and device code: the same
// functions run in the adjoint kernels and can be exercised on the CPU.
//
// The node map (Sec. II; the reduced collision of lbm_kernels.h) takes
//   d_i   = f_i - w_i rho_b0        the 27 colour-blind pre-collision deviations,
//   phic  = phi at the node          (Eq. order),
//   xr    = rho_r / rho at the node,
//   g     = (grad phi, grad rho)     the isotropic stencil gradients,
// and returns the colour-blind post-collision populations
//   f'_i = f^(e)_i + F'_i/2 + Delta_i + Omega^(2)_i
// (Eq. EES with Eq. Phi, Eq. ketFd, the relaxed deviatoric central moments
// Delta, Eq. perturb) and the recoloured red and blue populations
//   f^r*_i = xr f'_i + (w_i/|c_i|) c_i . V,   f^b*_i = f'_i - f^r*_i,
//   V = beta xr (1 - xr) rho kappa(alpha_bar) grad phi / |grad phi|   (Eqs. op3r/op3b).
// node_vjp() returns, for cotangents (Lr, Lb) of (f^r*, f^b*), the cotangents
// of d, phic, xr, g and of the perturbation strength A.  Everything is in FP64.
#pragma once
#include "lbm_kernels.h"

#define CG_HD __host__ __device__ __forceinline__

namespace cglbm {

// one-dimensional inverse central-moment basis over c = -1, 0, 1 (index c + 1)
// for shift u; d h0/du = h1 and d h1/du = 2 h2.
struct Basis1 {
    double h0[3], h1[3];
    CG_HD explicit Basis1(double u)
    {
        h0[0] = 0.5 * (u * u - u);
        h0[1] = 1.0 - u * u;
        h0[2] = 0.5 * (u * u + u);
        h1[0] = u - 0.5;
        h1[1] = -2.0 * u;
        h1[2] = u + 0.5;
    }
};
CG_HD constexpr double h2d(int j) { return j == 1 ? -1.0 : 0.5; }  // index j = c + 1

// forward quantities of one node that the reverse sweep needs
struct NodeFwd {
    double m0, rho, u[3], F[3], gp[3], gr[3];
    double hp, nub, s2, abar, kap, om;
    double q[6];   // second central moments of f - f^(e) + F'/2: xx, yy, zz, xy, xz, yz
    double tr;     // (q_xx + q_yy + q_zz) / 3
    double kk[6];  // relaxed and scaled: (1 - s2) q_ab (off-diagonal), (1 - s2)(q_aa - tr)
    double gn;     // |grad phi| (0 when switched off)
    bool on;       // |grad phi|^2 > eps^2
};

CG_HD void node_fwd(const KP& k, const float* d, float phic, const double* g, NodeFwd& f)
{
    double m0 = 0.0, j[3] = {0.0, 0.0, 0.0}, P[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double v = d[i];
        m0 += v;
        j[0] += kCX[i] * v;
        j[1] += kCY[i] * v;
        j[2] += kCZ[i] * v;
        P[0] += kCX[i] * kCX[i] * v;
        P[1] += kCY[i] * kCY[i] * v;
        P[2] += kCZ[i] * kCZ[i] * v;
        P[3] += kCX[i] * kCY[i] * v;
        P[4] += kCX[i] * kCZ[i] * v;
        P[5] += kCY[i] * kCZ[i] * v;
    }
    f.m0 = m0;
    f.rho = (double)k.rho_b0 + m0;
    f.hp = 0.5 * (1.0 + (double)phic);
    f.nub = 1.0 / (f.hp * (double)k.inv_nu_r + (1.0 - f.hp) * (double)k.inv_nu_b);
    f.s2 = 1.0 / (3.0 * f.nub + 0.5);
    f.abar = (double)k.alpha_b + f.hp * (double)k.dalpha;
    f.kap = (27.0 / 19.0) * (1.0 - f.abar);
    f.om = 1.0 - f.s2;
    const double gv[3] = {(double)k.gx, (double)k.gy, (double)k.gz};
    for (int a = 0; a < 3; ++a) {
        f.F[a] = m0 * gv[a];
        f.u[a] = (j[a] + 0.5 * f.F[a]) / f.rho;
        f.gp[a] = g[a];
        f.gr[a] = g[3 + a];
    }
    const double* u = f.u;
    const double* r = f.gr;
    const double* F = f.F;
    const double rho = f.rho, nub = f.nub;
    f.q[0] = P[0] - rho * u[0] * u[0] - 2.0 * nub * u[0] * r[0] + u[0] * F[0];
    f.q[1] = P[1] - rho * u[1] * u[1] - 2.0 * nub * u[1] * r[1] + u[1] * F[1];
    f.q[2] = P[2] - rho * u[2] * u[2] - 2.0 * nub * u[2] * r[2] + u[2] * F[2];
    f.q[3] = P[3] - rho * u[0] * u[1] - nub * (u[0] * r[1] + r[0] * u[1]) + 0.5 * (u[0] * F[1] + u[1] * F[0]);
    f.q[4] = P[4] - rho * u[0] * u[2] - nub * (u[0] * r[2] + r[0] * u[2]) + 0.5 * (u[0] * F[2] + u[2] * F[0]);
    f.q[5] = P[5] - rho * u[1] * u[2] - nub * (u[1] * r[2] + r[1] * u[2]) + 0.5 * (u[1] * F[2] + u[2] * F[1]);
    f.tr = (f.q[0] + f.q[1] + f.q[2]) * (1.0 / 3.0);
    for (int a = 0; a < 3; ++a) f.kk[a] = f.om * (f.q[a] - f.tr);
    for (int a = 3; a < 6; ++a) f.kk[a] = f.om * f.q[a];
    const double G2 = f.gp[0] * f.gp[0] + f.gp[1] * f.gp[1] + f.gp[2] * f.gp[2];
    f.on = G2 > (double)k.eps2;
    f.gn = f.on ? sqrt(G2) : 0.0;
}

// relaxed-moment part Delta of direction (cx, cy, cz)
CG_HD double delta_dir(const NodeFwd& f, const Basis1& bx, const Basis1& by, const Basis1& bz, int cx, int cy,
                       int cz)
{
    const int jx = cx + 1, jy = cy + 1, jz = cz + 1;
    return f.kk[3] * bx.h1[jx] * by.h1[jy] * bz.h0[jz] + f.kk[4] * bx.h1[jx] * by.h0[jy] * bz.h1[jz] +
           f.kk[5] * bx.h0[jx] * by.h1[jy] * bz.h1[jz] + f.kk[0] * h2d(jx) * by.h0[jy] * bz.h0[jz] +
           f.kk[1] * bx.h0[jx] * h2d(jy) * bz.h0[jz] + f.kk[2] * bx.h0[jx] * by.h0[jy] * h2d(jz);
}

// colour-blind post-collision populations f'_i and the recolouring vector V
CG_HD void node_post(const KP& k, const NodeFwd& f, float xr, double* fp, double* V)
{
    const Basis1 bx(f.u[0]), by(f.u[1]), bz(f.u[2]);
    const double u2 = f.u[0] * f.u[0] + f.u[1] * f.u[1] + f.u[2] * f.u[2];
    const double uF = f.u[0] * f.F[0] + f.u[1] * f.F[1] + f.u[2] * f.F[2];
    const double ur = f.u[0] * f.gr[0] + f.u[1] * f.gr[1] + f.u[2] * f.gr[2];
    const double A = k.A;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = kCX[i], cy = kCY[i], cz = kCZ[i];
        const double w = wgtd(i);
        const double cu = cx * f.u[0] + cy * f.u[1] + cz * f.u[2];
        const double cr = cx * f.gr[0] + cy * f.gr[1] + cz * f.gr[2];
        const double cF = cx * f.F[0] + cy * f.F[1] + cz * f.F[2];
        const double cg = cx * f.gp[0] + cy * f.gp[1] + cz * f.gp[2];
        const double poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * u2 + 4.5 * cu * cu * cu - 4.5 * cu * u2;
        double v;
        if (i == 0) {
            v = f.rho * f.abar + w * f.rho * poly - 3.0 * f.nub * ur - 1.5 * w * uF;
            if (f.on) v += A * (10.0 / 27.0) * f.gn;
        } else {
            v = w * (f.rho * f.kap + f.rho * poly + 9.0 * f.nub * cu * cr) + w * (4.5 * cu * cF - 1.5 * uF + 1.5 * cF);
            if (f.on) v += A * w * (cg * cg / f.gn - f.gn);
        }
        fp[i] = v + delta_dir(f, bx, by, bz, cx, cy, cz);
    }
    const double x = xr;
    const double s = f.on ? (double)k.beta * x * (1.0 - x) * f.rho * f.kap / f.gn : 0.0;
    V[0] = s * f.gp[0];
    V[1] = s * f.gp[1];
    V[2] = s * f.gp[2];
}

// recoloured red and blue populations of direction i from f'_i and V
CG_HD void recolour_dir(int i, double xr, double fpi, const double* V, double& fr, double& fb)
{
    double v = xr * fpi;
    if (i != 0) v += wgtd(i) * inv_lend(i) * (kCX[i] * V[0] + kCY[i] * V[1] + kCZ[i] * V[2]);
    fr = v;
    fb = fpi - v;
}

struct NodeAdj {
    double Ld[Q];          // cotangent of d_i
    double Lgp[3], Lgr[3]; // of grad phi, grad rho
    double Lphic, Lxr, LA; // of phi at the node, rho_r / rho, A
};

// reverse sweep of the node map for cotangents Lr (red) and Lb (blue) of the
// post-collision populations; fp are the f'_i of node_post
CG_HD void node_vjp(const KP& k, const NodeFwd& f, float xrf, const double* fp, const float* Lr, const float* Lb,
                    NodeAdj& o)
{
    const double xr = xrf, rho = f.rho, nub = f.nub;
    const double* u = f.u;
    const double* F = f.F;
    const double* gr = f.gr;
    const double* gp = f.gp;
    double L[Q];
    double Lxr = 0.0, LV[3] = {0.0, 0.0, 0.0};
    // recolouring: f^r* = xr f' + W c.V, f^b* = f' - f^r*
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double dl = (double)Lr[i] - (double)Lb[i];
        L[i] = (double)Lb[i] + xr * dl;
        Lxr += dl * fp[i];
        if (i != 0) {
            const double s = dl * wgtd(i) * inv_lend(i);
            LV[0] += kCX[i] * s;
            LV[1] += kCY[i] * s;
            LV[2] += kCZ[i] * s;
        }
    }
    double Lrho = 0.0, Lkap = 0.0, Labar = 0.0, Lnub = 0.0;
    double Lu[3] = {0.0, 0.0, 0.0}, LF[3] = {0.0, 0.0, 0.0}, Lgr[3] = {0.0, 0.0, 0.0}, Lgp[3] = {0.0, 0.0, 0.0};
    const double beta = k.beta;
    if (f.on) {
        const double n[3] = {gp[0] / f.gn, gp[1] / f.gn, gp[2] / f.gn};
        const double LVn = LV[0] * n[0] + LV[1] * n[1] + LV[2] * n[2];
        const double xx = xr * (1.0 - xr);
        const double sV = beta * xx * rho * f.kap;
        Lxr += beta * (1.0 - 2.0 * xr) * rho * f.kap * LVn;
        Lrho += beta * xx * f.kap * LVn;
        Lkap += beta * xx * rho * LVn;
        for (int a = 0; a < 3; ++a) Lgp[a] += sV * (LV[a] - LVn * n[a]) / f.gn;
    }
    // equilibrium, Phi and forcing terms, direction by direction
    const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double su = 0.0, sA = 0.0, S0 = 0.0, M2[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = kCX[i], cy = kCY[i], cz = kCZ[i];
        const double a = L[i] * wgtd(i);
        const double cu = cx * u[0] + cy * u[1] + cz * u[2];
        const double cr = cx * gr[0] + cy * gr[1] + cz * gr[2];
        const double cF = cx * F[0] + cy * F[1] + cz * F[2];
        Lrho += a * (3.0 * cu + 4.5 * cu * cu - 1.5 * u2 + 4.5 * cu * cu * cu - 4.5 * cu * u2);
        su += a * rho * (3.0 + 9.0 * cu);
        sA += a;
        if (i != 0) {
            const double cc = a * (rho * (3.0 + 9.0 * cu + 13.5 * cu * cu - 4.5 * u2) + 9.0 * nub * cr + 4.5 * cF);
            Lu[0] += cx * cc;
            Lu[1] += cy * cc;
            Lu[2] += cz * cc;
            const double cg = a * 9.0 * nub * cu;
            Lgr[0] += cx * cg;
            Lgr[1] += cy * cg;
            Lgr[2] += cz * cg;
            const double cf = a * (4.5 * cu + 1.5);
            LF[0] += cx * cf;
            LF[1] += cy * cf;
            LF[2] += cz * cf;
            Lnub += a * 9.0 * cu * cr;
            S0 += a;
            M2[0] += a * (cx * cx);
            M2[1] += a * (cy * cy);
            M2[2] += a * (cz * cz);
            M2[3] += a * (cx * cy);
            M2[4] += a * (cx * cz);
            M2[5] += a * (cy * cz);
        }
    }
    for (int c = 0; c < 3; ++c) {
        Lu[c] -= su * u[c] + 1.5 * sA * F[c];
        LF[c] -= 1.5 * sA * u[c];
    }
    // rest population: rho alpha_bar and Phi_0 = -3 nu_bar u . grad rho
    const double L0 = L[0];
    Lrho += f.abar * L0;
    Labar += rho * L0;
    Lnub += -3.0 * (u[0] * gr[0] + u[1] * gr[1] + u[2] * gr[2]) * L0;
    for (int c = 0; c < 3; ++c) {
        Lu[c] += -3.0 * nub * L0 * gr[c];
        Lgr[c] += -3.0 * nub * L0 * u[c];
    }
    // moving directions: rho kappa
    Lrho += f.kap * S0;
    Lkap += rho * S0;
    // perturbation (squared projection, prefactor A)
    double LA = 0.0;
    if (f.on) {
        const double A = k.A, gn = f.gn;
        const double Mg[3] = {M2[0] * gp[0] + M2[3] * gp[1] + M2[4] * gp[2],
                              M2[3] * gp[0] + M2[1] * gp[1] + M2[5] * gp[2],
                              M2[4] * gp[0] + M2[5] * gp[1] + M2[2] * gp[2]};
        const double gMg = gp[0] * Mg[0] + gp[1] * Mg[1] + gp[2] * Mg[2];
        LA = gMg / gn - S0 * gn + L0 * (10.0 / 27.0) * gn;
        for (int c = 0; c < 3; ++c)
            Lgp[c] += A * (2.0 * Mg[c] / gn - gMg * gp[c] / (gn * gn * gn) - S0 * gp[c] / gn +
                           L0 * (10.0 / 27.0) * gp[c] / gn);
    }
    // relaxed-moment part: C[a][b][c] = sum_dirs L h_a(cx) h_b(cy) h_c(cz)
    const Basis1 bx(u[0]), by(u[1]), bz(u[2]);
    double X[3][3][3];  // [basis a][jy][jz], contracted over x
#pragma unroll
    for (int jy = 0; jy < 3; ++jy)
#pragma unroll
        for (int jz = 0; jz < 3; ++jz) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int jx = 0; jx < 3; ++jx) {
                const double v = L[dir_of(jx - 1, jy - 1, jz - 1)];
                s0 += v * bx.h0[jx];
                s1 += v * bx.h1[jx];
                s2 += v * h2d(jx);
            }
            X[0][jy][jz] = s0;
            X[1][jy][jz] = s1;
            X[2][jy][jz] = s2;
        }
    double Y[3][3][3];  // [a][b][jz]
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int jz = 0; jz < 3; ++jz) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int jy = 0; jy < 3; ++jy) {
                const double v = X[a][jy][jz];
                s0 += v * by.h0[jy];
                s1 += v * by.h1[jy];
                s2 += v * h2d(jy);
            }
            Y[a][0][jz] = s0;
            Y[a][1][jz] = s1;
            Y[a][2][jz] = s2;
        }
    double C[3][3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int jz = 0; jz < 3; ++jz) {
                const double v = Y[a][b][jz];
                s0 += v * bz.h0[jz];
                s1 += v * bz.h1[jz];
                s2 += v * h2d(jz);
            }
            C[a][b][0] = s0;
            C[a][b][1] = s1;
            C[a][b][2] = s2;
        }
    const double* kk = f.kk;  // xx yy zz xy xz yz
    const double Lk[6] = {C[2][0][0], C[0][2][0], C[0][0][2], C[1][1][0], C[1][0][1], C[0][1][1]};
    Lu[0] += 2.0 * kk[3] * C[2][1][0] + 2.0 * kk[4] * C[2][0][1] + kk[5] * C[1][1][1] + kk[1] * C[1][2][0] +
             kk[2] * C[1][0][2];
    Lu[1] += 2.0 * kk[3] * C[1][2][0] + kk[4] * C[1][1][1] + 2.0 * kk[5] * C[0][2][1] + kk[0] * C[2][1][0] +
             kk[2] * C[0][1][2];
    Lu[2] += kk[3] * C[1][1][1] + 2.0 * kk[4] * C[1][0][2] + 2.0 * kk[5] * C[0][1][2] + kk[0] * C[2][0][1] +
             kk[1] * C[0][2][1];
    // k = (1 - s2) dev(q)
    const double trL = (Lk[0] + Lk[1] + Lk[2]) * (1.0 / 3.0);
    double Lq[6];
    for (int a = 0; a < 3; ++a) Lq[a] = f.om * (Lk[a] - trL);
    for (int a = 3; a < 6; ++a) Lq[a] = f.om * Lk[a];
    double Ls2 = 0.0;
    for (int a = 0; a < 3; ++a) Ls2 -= (f.q[a] - f.tr) * Lk[a];
    for (int a = 3; a < 6; ++a) Ls2 -= f.q[a] * Lk[a];
    // q = P - rho u u^T - nu_bar (u r^T + r u^T) + (u F^T + F u^T)/2, through the symmetric matrix Qm
    const double Qm[3][3] = {{Lq[0], 0.5 * Lq[3], 0.5 * Lq[4]},
                             {0.5 * Lq[3], Lq[1], 0.5 * Lq[5]},
                             {0.5 * Lq[4], 0.5 * Lq[5], Lq[2]}};
    double Qu[3], Qr[3], QF[3];
    for (int a = 0; a < 3; ++a) {
        Qu[a] = Qm[a][0] * u[0] + Qm[a][1] * u[1] + Qm[a][2] * u[2];
        Qr[a] = Qm[a][0] * gr[0] + Qm[a][1] * gr[1] + Qm[a][2] * gr[2];
        QF[a] = Qm[a][0] * F[0] + Qm[a][1] * F[1] + Qm[a][2] * F[2];
    }
    Lrho -= u[0] * Qu[0] + u[1] * Qu[1] + u[2] * Qu[2];
    Lnub -= 2.0 * (u[0] * Qr[0] + u[1] * Qr[1] + u[2] * Qr[2]);
    for (int a = 0; a < 3; ++a) {
        Lu[a] += -2.0 * rho * Qu[a] - 2.0 * nub * Qr[a] + QF[a];
        Lgr[a] += -2.0 * nub * Qu[a];
        LF[a] += Qu[a];
    }
    // interpolated properties
    Labar -= (27.0 / 19.0) * Lkap;
    double Lhp = (double)k.dalpha * Labar;
    Lnub += -3.0 * f.s2 * f.s2 * Ls2;
    Lhp += -nub * nub * ((double)k.inv_nu_r - (double)k.inv_nu_b) * Lnub;
    // u = (j + F/2) / rho, F = m0 g, rho = rho_b0 + m0
    double Lj[3];
    for (int a = 0; a < 3; ++a) {
        Lj[a] = Lu[a] / rho;
        LF[a] += 0.5 * Lu[a] / rho;
    }
    Lrho -= (u[0] * Lu[0] + u[1] * Lu[1] + u[2] * Lu[2]) / rho;
    const double Lm0 = Lrho + (double)k.gx * LF[0] + (double)k.gy * LF[1] + (double)k.gz * LF[2];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = kCX[i], cy = kCY[i], cz = kCZ[i];
        o.Ld[i] = Lm0 + cx * Lj[0] + cy * Lj[1] + cz * Lj[2] + (cx * cx) * Lq[0] + (cy * cy) * Lq[1] +
                  (cz * cz) * Lq[2] + (cx * cy) * Lq[3] + (cx * cz) * Lq[4] + (cy * cz) * Lq[5];
    }
    for (int a = 0; a < 3; ++a) {
        o.Lgp[a] = Lgp[a];
        o.Lgr[a] = Lgr[a];
    }
    o.Lphic = 0.5 * Lhp;
    o.Lxr = Lxr;
    o.LA = LA;
}

}  // namespace cglbm
