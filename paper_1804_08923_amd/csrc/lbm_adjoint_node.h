// Per-node forward recomputation and its vector-Jacobian product (reverse
// mode), for the adjoint of one time step.  Host and device code, templated on
// the arithmetic type R: the adjoint kernels run them in FP32 (the derivative
// coefficients need no cancellation-free sums), a host build runs them in
// FP64 or FP32 for checking.
//
// The node map (Sec. II; the reduced collision of lbm_kernels.h) takes
//   d_i   = f_i - w_i rho_b0        the 27 colour-blind pre-collision deviations
//                                   (through their moments up to second order),
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
// of d, phic, xr, g and of the perturbation strength A.
#pragma once
#include "lbm_kernels.h"

#define CG_HD __host__ __device__ __forceinline__

namespace cglbm {

// one-dimensional inverse central-moment basis over c = -1, 0, 1 (index c + 1)
// for shift u; d h0/du = h1 and d h1/du = 2 h2.
template <class R>
struct Basis1T {
    R h0[3], h1[3];
    CG_HD explicit Basis1T(R u)
    {
        h0[0] = R(0.5) * (u * u - u);
        h0[1] = R(1) - u * u;
        h0[2] = R(0.5) * (u * u + u);
        h1[0] = u - R(0.5);
        h1[1] = R(-2) * u;
        h1[2] = u + R(0.5);
    }
};
template <class R>
CG_HD constexpr R h2r(int j) { return j == 1 ? R(-1) : R(0.5); }  // index j = c + 1

// raw moments of the deviations up to second order
template <class R>
struct MomT {
    R m0 = 0, j[3] = {0, 0, 0}, P[6] = {0, 0, 0, 0, 0, 0};  // P: xx yy zz xy xz yz
    CG_HD void add(int i, R v)
    {
        m0 += v;
        if (kCX[i]) { j[0] += kCX[i] * v; P[0] += v; }
        if (kCY[i]) { j[1] += kCY[i] * v; P[1] += v; }
        if (kCZ[i]) { j[2] += kCZ[i] * v; P[2] += v; }
        if (kCX[i] * kCY[i]) P[3] += (kCX[i] * kCY[i]) * v;
        if (kCX[i] * kCZ[i]) P[4] += (kCX[i] * kCZ[i]) * v;
        if (kCY[i] * kCZ[i]) P[5] += (kCY[i] * kCZ[i]) * v;
    }
};

// forward quantities of one node that the reverse sweep needs
template <class R>
struct NodeFwdT {
    R m0, rho, u[3], F[3], gp[3], gr[3];
    R nub, s2, abar, kap, om;
    R q[6];   // second central moments of f - f^(e) + F'/2: xx, yy, zz, xy, xz, yz
    R tr;     // (q_xx + q_yy + q_zz) / 3
    R kk[6];  // relaxed and scaled: (1 - s2) q_ab (off-diagonal), (1 - s2)(q_aa - tr)
    R gn;     // |grad phi| (0 when switched off)
    R n[3];   // grad phi / |grad phi| (0 when switched off)
    bool on;  // |grad phi|^2 > eps^2
};

template <class R>
CG_HD void node_fwd(const KP& k, const MomT<R>& M, R phic, const double* g, NodeFwdT<R>& f)
{
    f.m0 = M.m0;
    f.rho = (R)k.rho_b0 + M.m0;
    const R hp = R(0.5) * (R(1) + phic);
    f.nub = R(1) / (hp * (R)k.inv_nu_r + (R(1) - hp) * (R)k.inv_nu_b);
    f.s2 = R(1) / (R(3) * f.nub + R(0.5));
    f.abar = (R)k.alpha_b + hp * (R)k.dalpha;
    f.kap = R(27.0 / 19.0) * (R(1) - f.abar);
    f.om = R(1) - f.s2;
    const R gv[3] = {(R)k.gx, (R)k.gy, (R)k.gz};
    const R inv_rho = R(1) / f.rho;
    for (int a = 0; a < 3; ++a) {
        f.F[a] = M.m0 * gv[a];
        f.u[a] = (M.j[a] + R(0.5) * f.F[a]) * inv_rho;
        f.gp[a] = (R)g[a];
        f.gr[a] = (R)g[3 + a];
    }
    const R* u = f.u;
    const R* r = f.gr;
    const R* F = f.F;
    const R rho = f.rho, nub = f.nub;
    f.q[0] = M.P[0] - rho * u[0] * u[0] - R(2) * nub * u[0] * r[0] + u[0] * F[0];
    f.q[1] = M.P[1] - rho * u[1] * u[1] - R(2) * nub * u[1] * r[1] + u[1] * F[1];
    f.q[2] = M.P[2] - rho * u[2] * u[2] - R(2) * nub * u[2] * r[2] + u[2] * F[2];
    f.q[3] = M.P[3] - rho * u[0] * u[1] - nub * (u[0] * r[1] + r[0] * u[1]) + R(0.5) * (u[0] * F[1] + u[1] * F[0]);
    f.q[4] = M.P[4] - rho * u[0] * u[2] - nub * (u[0] * r[2] + r[0] * u[2]) + R(0.5) * (u[0] * F[2] + u[2] * F[0]);
    f.q[5] = M.P[5] - rho * u[1] * u[2] - nub * (u[1] * r[2] + r[1] * u[2]) + R(0.5) * (u[1] * F[2] + u[2] * F[1]);
    f.tr = (f.q[0] + f.q[1] + f.q[2]) * R(1.0 / 3.0);
    for (int a = 0; a < 3; ++a) f.kk[a] = f.om * (f.q[a] - f.tr);
    for (int a = 3; a < 6; ++a) f.kk[a] = f.om * f.q[a];
    const double G2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    f.on = G2 > (double)k.eps2;
    const double gn = f.on ? sqrt(G2) : 0.0, ign = f.on ? 1.0 / gn : 0.0;
    f.gn = (R)gn;
    for (int a = 0; a < 3; ++a) f.n[a] = (R)(g[a] * ign);
}

// colour-blind post-collision population f'_i of direction I
template <class R, int I>
CG_HD R fpost_dir(const KP& k, const NodeFwdT<R>& f, const Basis1T<R>& bx, const Basis1T<R>& by,
                  const Basis1T<R>& bz, R u2, R uF, R ur)
{
    constexpr int cx = kCX[I], cy = kCY[I], cz = kCZ[I];
    constexpr int jx = cx + 1, jy = cy + 1, jz = cz + 1;
    const R w = (R)wgtd(I);
    const R cu = cx * f.u[0] + cy * f.u[1] + cz * f.u[2];
    const R poly = cu * (R(3) + R(4.5) * cu + R(4.5) * cu * cu - R(4.5) * u2) - R(1.5) * u2;
    R v;
    if (I == 0) {
        v = f.rho * f.abar + w * f.rho * poly - R(3) * f.nub * ur - R(1.5) * w * uF;
        if (f.on) v += (R)k.A * R(10.0 / 27.0) * f.gn;
    } else {
        const R cr = cx * f.gr[0] + cy * f.gr[1] + cz * f.gr[2];
        const R cF = cx * f.F[0] + cy * f.F[1] + cz * f.F[2];
        const R cn = cx * f.n[0] + cy * f.n[1] + cz * f.n[2];
        v = w * (f.rho * (f.kap + poly) + R(9) * f.nub * cu * cr + R(4.5) * cu * cF - R(1.5) * uF + R(1.5) * cF);
        if (f.on) v += (R)k.A * w * f.gn * (cn * cn - R(1));
    }
    // relaxed-moment part Delta
    v += f.kk[3] * bx.h1[jx] * by.h1[jy] * bz.h0[jz] + f.kk[4] * bx.h1[jx] * by.h0[jy] * bz.h1[jz] +
         f.kk[5] * bx.h0[jx] * by.h1[jy] * bz.h1[jz] + f.kk[0] * h2r<R>(jx) * by.h0[jy] * bz.h0[jz] +
         f.kk[1] * bx.h0[jx] * h2r<R>(jy) * bz.h0[jz] + f.kk[2] * bx.h0[jx] * by.h0[jy] * h2r<R>(jz);
    return v;
}

template <class R>
struct PostCtx {
    Basis1T<R> bx, by, bz;
    R u2, uF, ur;
    CG_HD explicit PostCtx(const NodeFwdT<R>& f)
        : bx(f.u[0]), by(f.u[1]), bz(f.u[2]),
          u2(f.u[0] * f.u[0] + f.u[1] * f.u[1] + f.u[2] * f.u[2]),
          uF(f.u[0] * f.F[0] + f.u[1] * f.F[1] + f.u[2] * f.F[2]),
          ur(f.u[0] * f.gr[0] + f.u[1] * f.gr[1] + f.u[2] * f.gr[2])
    {
    }
};

template <class R, int I = 0>
CG_HD void fpost_all(const KP& k, const NodeFwdT<R>& f, const PostCtx<R>& c, R* fp)
{
    if constexpr (I < Q) {
        fp[I] = fpost_dir<R, I>(k, f, c.bx, c.by, c.bz, c.u2, c.uF, c.ur);
        fpost_all<R, I + 1>(k, f, c, fp);
    }
}

// colour-blind post-collision populations f'_i and the recolouring vector V
template <class R>
CG_HD void node_post(const KP& k, const NodeFwdT<R>& f, R xr, R* fp, R* V)
{
    const PostCtx<R> c(f);
    fpost_all<R>(k, f, c, fp);
    const R s = f.on ? (R)k.beta * xr * (R(1) - xr) * f.rho * f.kap : R(0);
    for (int a = 0; a < 3; ++a) V[a] = s * f.n[a];
}

// recoloured red and blue populations of direction i from f'_i and V
template <class R>
CG_HD void recolour_dir(int i, R xr, R fpi, const R* V, R& fr, R& fb)
{
    R v = xr * fpi;
    if (i != 0) v += (R)(wgtd(i) * inv_lend(i)) * (kCX[i] * V[0] + kCY[i] * V[1] + kCZ[i] * V[2]);
    fr = v;
    fb = fpi - v;
}

template <class R>
struct NodeAdjT {
    R Lm0, Lj[3], Lq[6];  // cotangents of the raw moments of d: Ld_i = Lm0 + c_i.Lj + c_i c_i : Lq
    R Ld[Q];          // cotangent of d_i
    R Lgp[3], Lgr[3]; // of grad phi, grad rho
    R Lphic, Lxr, LA; // of phi at the node, rho_r / rho, A
};

// first sweep: colour-blind cotangents L'_i = Lb_i + xr (Lr_i - Lb_i) (written
// over Lb), and the cotangents of xr and V through the recolouring
template <class R, int I = 0>
CG_HD void vjp_recolour(const KP& k, const NodeFwdT<R>& f, const PostCtx<R>& c, R xr, const R* Lr, R* L, R& Lxr,
                        R* LV)
{
    if constexpr (I < Q) {
        const R dl = Lr[I] - L[I];
        L[I] += xr * dl;
        Lxr += dl * fpost_dir<R, I>(k, f, c.bx, c.by, c.bz, c.u2, c.uF, c.ur);
        if (I != 0) {
            const R s = dl * (R)(wgtd(I) * inv_lend(I));
            if (kCX[I]) LV[0] += kCX[I] * s;
            if (kCY[I]) LV[1] += kCY[I] * s;
            if (kCZ[I]) LV[2] += kCZ[I] * s;
        }
        vjp_recolour<R, I + 1>(k, f, c, xr, Lr, L, Lxr, LV);
    }
}

// reverse sweep of the node map.  Lr: cotangents of the red post-collision
// populations; LbL: on entry those of the blue ones, overwritten.
template <class R>
CG_HD void node_vjp(const KP& k, const NodeFwdT<R>& f, R xr, const R* Lr, R* LbL, NodeAdjT<R>& o)
{
    const R rho = f.rho, nub = f.nub;
    const R* u = f.u;
    const R* F = f.F;
    const R* gr = f.gr;
    const PostCtx<R> pc(f);
    R* L = LbL;
    R Lxr = 0, LV[3] = {0, 0, 0};
    vjp_recolour<R>(k, f, pc, xr, Lr, L, Lxr, LV);
    R Lrho = 0, Lkap = 0, Labar = 0, Lnub = 0;
    R Lu[3] = {0, 0, 0}, LF[3] = {0, 0, 0}, Lgr[3] = {0, 0, 0}, Lgp[3] = {0, 0, 0};
    const R beta = (R)k.beta;
    if (f.on) {
        const R LVn = LV[0] * f.n[0] + LV[1] * f.n[1] + LV[2] * f.n[2];
        const R xx = xr * (R(1) - xr);
        const R sV = beta * xx * rho * f.kap;
        Lxr += beta * (R(1) - R(2) * xr) * rho * f.kap * LVn;
        Lrho += beta * xx * f.kap * LVn;
        Lkap += beta * xx * rho * LVn;
        const R ig = R(1) / f.gn;
        for (int a = 0; a < 3; ++a) Lgp[a] += sV * (LV[a] - LVn * f.n[a]) * ig;
    }
    // equilibrium, Phi and forcing terms, direction by direction
    const R u2 = pc.u2;
    R su = 0, sA = 0, S0 = 0, M2[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = kCX[i], cy = kCY[i], cz = kCZ[i];
        const R a = L[i] * (R)wgtd(i);
        const R cu = cx * u[0] + cy * u[1] + cz * u[2];
        Lrho += a * (cu * (R(3) + R(4.5) * cu + R(4.5) * cu * cu - R(4.5) * u2) - R(1.5) * u2);
        su += a * (R(3) + R(9) * cu);
        sA += a;
        if (i != 0) {
            const R cr = cx * gr[0] + cy * gr[1] + cz * gr[2];
            const R cF = cx * F[0] + cy * F[1] + cz * F[2];
            const R cc = a * (rho * (R(3) + R(9) * cu + R(13.5) * cu * cu - R(4.5) * u2) + R(9) * nub * cr +
                              R(4.5) * cF);
            const R cg = a * R(9) * nub * cu;
            const R cf = a * (R(4.5) * cu + R(1.5));
            if (cx) { Lu[0] += cx * cc; Lgr[0] += cx * cg; LF[0] += cx * cf; M2[0] += a; }
            if (cy) { Lu[1] += cy * cc; Lgr[1] += cy * cg; LF[1] += cy * cf; M2[1] += a; }
            if (cz) { Lu[2] += cz * cc; Lgr[2] += cz * cg; LF[2] += cz * cf; M2[2] += a; }
            Lnub += a * R(9) * cu * cr;
            S0 += a;
            if (cx * cy) M2[3] += (cx * cy) * a;
            if (cx * cz) M2[4] += (cx * cz) * a;
            if (cy * cz) M2[5] += (cy * cz) * a;
        }
    }
    su *= rho;
    for (int c = 0; c < 3; ++c) {
        Lu[c] -= su * u[c] + R(1.5) * sA * F[c];
        LF[c] -= R(1.5) * sA * u[c];
    }
    // rest population: rho alpha_bar and Phi_0 = -3 nu_bar u . grad rho
    const R L0 = L[0];
    Lrho += f.abar * L0;
    Labar += rho * L0;
    Lnub += R(-3) * pc.ur * L0;
    for (int c = 0; c < 3; ++c) {
        Lu[c] += R(-3) * nub * L0 * gr[c];
        Lgr[c] += R(-3) * nub * L0 * u[c];
    }
    // moving directions: rho kappa
    Lrho += f.kap * S0;
    Lkap += rho * S0;
    // perturbation (squared projection, prefactor A): A |g| [w (c.n)^2 - B]
    R LA = 0;
    if (f.on) {
        const R A = (R)k.A;
        const R* n = f.n;
        const R Mn[3] = {M2[0] * n[0] + M2[3] * n[1] + M2[4] * n[2], M2[3] * n[0] + M2[1] * n[1] + M2[5] * n[2],
                         M2[4] * n[0] + M2[5] * n[1] + M2[2] * n[2]};
        const R nMn = n[0] * Mn[0] + n[1] * Mn[1] + n[2] * Mn[2];
        const R b0 = L0 * R(10.0 / 27.0) - S0;
        LA = f.gn * (nMn + b0);
        for (int c = 0; c < 3; ++c) Lgp[c] += A * (R(2) * Mn[c] + (b0 - nMn) * n[c]);
    }
    // relaxed-moment part: C[a][b][c] = sum over directions of L h_a(cx) h_b(cy) h_c(cz)
    const Basis1T<R>& bx = pc.bx;
    const Basis1T<R>& by = pc.by;
    const Basis1T<R>& bz = pc.bz;
    R X[3][3][3];  // [basis a][jy][jz], contracted over x
#pragma unroll
    for (int jy = 0; jy < 3; ++jy)
#pragma unroll
        for (int jz = 0; jz < 3; ++jz) {
            const R v0 = L[dir_of(-1, jy - 1, jz - 1)], v1 = L[dir_of(0, jy - 1, jz - 1)],
                    v2 = L[dir_of(1, jy - 1, jz - 1)];
            X[0][jy][jz] = v0 * bx.h0[0] + v1 * bx.h0[1] + v2 * bx.h0[2];
            X[1][jy][jz] = v0 * bx.h1[0] + v1 * bx.h1[1] + v2 * bx.h1[2];
            X[2][jy][jz] = R(0.5) * (v0 + v2) - v1;
        }
    R Y[3][3][3];  // [a][b][jz]
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int jz = 0; jz < 3; ++jz) {
            const R v0 = X[a][0][jz], v1 = X[a][1][jz], v2 = X[a][2][jz];
            Y[a][0][jz] = v0 * by.h0[0] + v1 * by.h0[1] + v2 * by.h0[2];
            Y[a][1][jz] = v0 * by.h1[0] + v1 * by.h1[1] + v2 * by.h1[2];
            Y[a][2][jz] = R(0.5) * (v0 + v2) - v1;
        }
    auto Cz = [&](int a, int b, int c) -> R {
        const R v0 = Y[a][b][0], v1 = Y[a][b][1], v2 = Y[a][b][2];
        return c == 0 ? v0 * bz.h0[0] + v1 * bz.h0[1] + v2 * bz.h0[2]
                      : (c == 1 ? v0 * bz.h1[0] + v1 * bz.h1[1] + v2 * bz.h1[2] : R(0.5) * (v0 + v2) - v1);
    };
    const R C200 = Cz(2, 0, 0), C020 = Cz(0, 2, 0), C002 = Cz(0, 0, 2), C110 = Cz(1, 1, 0), C101 = Cz(1, 0, 1),
            C011 = Cz(0, 1, 1), C210 = Cz(2, 1, 0), C201 = Cz(2, 0, 1), C111 = Cz(1, 1, 1), C120 = Cz(1, 2, 0),
            C102 = Cz(1, 0, 2), C021 = Cz(0, 2, 1), C012 = Cz(0, 1, 2);
    const R* kk = f.kk;  // xx yy zz xy xz yz
    const R Lk[6] = {C200, C020, C002, C110, C101, C011};
    Lu[0] += R(2) * kk[3] * C210 + R(2) * kk[4] * C201 + kk[5] * C111 + kk[1] * C120 + kk[2] * C102;
    Lu[1] += R(2) * kk[3] * C120 + kk[4] * C111 + R(2) * kk[5] * C021 + kk[0] * C210 + kk[2] * C012;
    Lu[2] += kk[3] * C111 + R(2) * kk[4] * C102 + R(2) * kk[5] * C012 + kk[0] * C201 + kk[1] * C021;
    // k = (1 - s2) dev(q)
    const R trL = (Lk[0] + Lk[1] + Lk[2]) * R(1.0 / 3.0);
    R Lq[6];
    for (int a = 0; a < 3; ++a) Lq[a] = f.om * (Lk[a] - trL);
    for (int a = 3; a < 6; ++a) Lq[a] = f.om * Lk[a];
    R Ls2 = 0;
    for (int a = 0; a < 3; ++a) Ls2 -= (f.q[a] - f.tr) * Lk[a];
    for (int a = 3; a < 6; ++a) Ls2 -= f.q[a] * Lk[a];
    // q = P - rho u u^T - nu_bar (u r^T + r u^T) + (u F^T + F u^T)/2, through the symmetric matrix Qm
    const R Qm[3][3] = {{Lq[0], R(0.5) * Lq[3], R(0.5) * Lq[4]},
                        {R(0.5) * Lq[3], Lq[1], R(0.5) * Lq[5]},
                        {R(0.5) * Lq[4], R(0.5) * Lq[5], Lq[2]}};
    R Qu[3], Qr[3], QF[3];
    for (int a = 0; a < 3; ++a) {
        Qu[a] = Qm[a][0] * u[0] + Qm[a][1] * u[1] + Qm[a][2] * u[2];
        Qr[a] = Qm[a][0] * gr[0] + Qm[a][1] * gr[1] + Qm[a][2] * gr[2];
        QF[a] = Qm[a][0] * F[0] + Qm[a][1] * F[1] + Qm[a][2] * F[2];
    }
    Lrho -= u[0] * Qu[0] + u[1] * Qu[1] + u[2] * Qu[2];
    Lnub -= R(2) * (u[0] * Qr[0] + u[1] * Qr[1] + u[2] * Qr[2]);
    for (int a = 0; a < 3; ++a) {
        Lu[a] += R(-2) * rho * Qu[a] - R(2) * nub * Qr[a] + QF[a];
        Lgr[a] += R(-2) * nub * Qu[a];
        LF[a] += Qu[a];
    }
    // interpolated properties
    Labar -= R(27.0 / 19.0) * Lkap;
    R Lhp = (R)k.dalpha * Labar;
    Lnub += R(-3) * f.s2 * f.s2 * Ls2;
    Lhp += -nub * nub * ((R)k.inv_nu_r - (R)k.inv_nu_b) * Lnub;
    // u = (j + F/2) / rho, F = m0 g, rho = rho_b0 + m0
    const R inv_rho = R(1) / rho;
    R Lj[3];
    for (int a = 0; a < 3; ++a) {
        Lj[a] = Lu[a] * inv_rho;
        LF[a] += R(0.5) * Lj[a];
    }
    Lrho -= (u[0] * Lu[0] + u[1] * Lu[1] + u[2] * Lu[2]) * inv_rho;
    const R Lm0 = Lrho + (R)k.gx * LF[0] + (R)k.gy * LF[1] + (R)k.gz * LF[2];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = kCX[i], cy = kCY[i], cz = kCZ[i];
        R v = Lm0;
        if (cx) v += cx * Lj[0] + Lq[0];
        if (cy) v += cy * Lj[1] + Lq[1];
        if (cz) v += cz * Lj[2] + Lq[2];
        if (cx * cy) v += (cx * cy) * Lq[3];
        if (cx * cz) v += (cx * cz) * Lq[4];
        if (cy * cz) v += (cy * cz) * Lq[5];
        o.Ld[i] = v;
    }
    o.Lm0 = Lm0;
    for (int a = 0; a < 3; ++a) {
        o.Lj[a] = Lj[a];
        o.Lgp[a] = Lgp[a];
        o.Lgr[a] = Lgr[a];
    }
    for (int a = 0; a < 6; ++a) o.Lq[a] = Lq[a];
    o.Lphic = R(0.5) * Lhp;
    o.Lxr = Lxr;
    o.LA = LA;
}

}  // namespace cglbm
