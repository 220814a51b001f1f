/*
 * cglbm_oracle.c -- plain, slow CPU reference of one time step of the
 * two-colour D3Q27 colour-gradient lattice Boltzmann model with
 * nonorthogonal central moments (Saito et al., arXiv:1804.08923, Sec. II and
 * Appendix A).
 *
 * TEST INFRASTRUCTURE ONLY: called from tests/, the smoke entry point and
 * the CPU-baseline leg of bench.py, never from the product library.  It
 * shares no code with the HIP path.
 *
 * The scheme is evaluated literally, node by node, in the order the paper
 * states it: densities, order parameter, isotropic gradients, interpolated
 * properties, body force and velocity, enhanced equilibrium, forcing
 * populations, the GMRT collision as the matrix chain M^-1 N^-1 K N M with
 * N = T(u) M^-1 (Eq. scoll, Eq. ketF), perturbation (Eq. perturb),
 * recolouring (Eqs. op3r/op3b), streaming (Eq. LBE) and the jet boundaries.
 * Readings of passages that are ambiguous or garbled are marked READING and
 * are listed in the design notes of the repository.
 *
 * Parity status: every function here is pinned by a test in tests/ against
 * values the paper prints (Appendix A matrices) or against closed forms,
 * invariants and special cases.  The jet boundary rules, which the paper
 * gives only in words, are pinned by consequences (tests/test_oracle_jet_bc.py):
 * the free-slip walls against a mirrored periodic lattice (method of images),
 * the inflow against closed-form moments of the inlet equilibrium, fixed
 * points with a closed or resting inlet, the outflow rule at t + 1, and the
 * symmetries of a centred jet.
 */
#include "cglbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#if defined(OR_COMPLEX)
#define RE(x) creal(x)
#define R_SQRT(x) csqrt(x)
#elif defined(OR_FLOAT)
#define RE(x) (x)
#define R_SQRT(x) sqrtf(x)
#else
#define RE(x) (x)
#define R_SQRT(x) sqrt(x)
#endif

/* OR_Q19 builds the same scheme on the D3Q19 subset of the velocity set (the
 * reduced lattice the paper suggests in Sec. II and Sec. IV B as the way to
 * cut the cost, without giving its coefficients).  Its constants are derived
 * below so that every moment the D3Q27 coefficients fix is kept (READING, one
 * note per constant). */
#if defined(OR_Q19)
#define Q 19
#else
#define Q 27
#endif

/* ---- lattice (Eq. velVec; weights below it) -----------------------------
 * The 27 directions in the paper's order; the first 19 (rest, faces, edges)
 * are the D3Q19 subset. */
static const int CX[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1,
                          1, -1, 1, -1, 1, -1, -1, 1};
static const int CY[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 1, -1, 1, -1, 0, 0, 0, 0,
                          1, -1, 1, -1, -1, 1, 1, -1};
static const int CZ[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                          1, -1, -1, 1, 1, -1, 1, -1};

static int csq(int i) { return CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i]; }

/* D3Q27 weights by |c|^2 = 0, 1, 2, 3; D3Q19: the standard weights 1/3,
 * 1/18, 1/36, which keep sum w c c = delta/3 and an isotropic fourth moment */
static double weight(int i)
{
#if defined(OR_Q19)
    switch (csq(i)) {
    case 0: return 1.0 / 3.0;
    case 1: return 1.0 / 18.0;
    default: return 1.0 / 36.0;
    }
#endif
    switch (csq(i)) {
    case 0: return 8.0 / 27.0;
    case 1: return 2.0 / 27.0;
    case 2: return 1.0 / 54.0;
    default: return 1.0 / 216.0;
    }
}

/* perturbation constants B_i (Eq. B_i), c = 1.  On D3Q27 they are B_i = w_i
 * for i > 0 and B_0 = w_0 - 2/3, so that sum B_i = c_s^2 = 1/3 (the operator
 * moves no mass) and sum B_i c c = delta/3.  READING (D3Q19): the same two
 * rules on D3Q19, B_0 = 1/3 - 2/3 = -1/3, B_i = w_i. */
static double bcoef(int i)
{
#if defined(OR_Q19)
    return csq(i) == 0 ? -1.0 / 3.0 : weight(i);
#endif
    switch (csq(i)) {
    case 0: return -10.0 / 27.0;
    case 1: return 2.0 / 27.0;
    case 2: return 1.0 / 54.0;
    default: return 1.0 / 216.0;
    }
}

void or_lattice(int32_t* c, double* w)
{
    for (int i = 0; i < Q; ++i) {
        c[3 * i + 0] = CX[i];
        c[3 * i + 1] = CY[i];
        c[3 * i + 2] = CZ[i];
        w[i] = weight(i);
    }
}

/* ---- moment basis (Eq. momentSet) ----------------------------------------
 * Row j of T(u) is the j-th polynomial of the shifted velocity
 * cbar = c - u; at u = 0 it is the raw-moment matrix M (Eq. M). */
static or_real moment_poly(int j, or_real X, or_real Y, or_real Z)
{
    or_real X2 = X * X, Y2 = Y * Y, Z2 = Z * Z;
    switch (j) {
    case 0: return 1;
    case 1: return X;
    case 2: return Y;
    case 3: return Z;
    case 4: return X * Y;
    case 5: return X * Z;
    case 6: return Y * Z;
    case 7: return X2 - Y2;
    case 8: return X2 - Z2;
    case 9: return X2 + Y2 + Z2;
    case 10: return X * Y2 + X * Z2;
    case 11: return X2 * Y + Y * Z2;
    case 12: return X2 * Z + Y2 * Z;
    case 13: return X * Y2 - X * Z2;
    case 14: return X2 * Y - Y * Z2;
    case 15: return X2 * Z - Y2 * Z;
    case 16: return X * Y * Z;
    case 17: return X2 * Y2 + X2 * Z2 + Y2 * Z2;
    case 18: return X2 * Y2 + X2 * Z2 - Y2 * Z2;
    case 19: return X2 * Y2 - X2 * Z2;
    case 20: return X2 * Y * Z;
    case 21: return X * Y2 * Z;
    case 22: return X * Y * Z2;
    case 23: return X * Y2 * Z2;
    case 24: return X2 * Y * Z2;
    case 25: return X2 * Y2 * Z;
    default: return X2 * Y2 * Z2;
    }
}

/* Row j of the basis in use.  READING (D3Q19): the 19 rows of Eq. momentSet
 * that are not identically zero or dependent on the D3Q19 velocities, that is
 * all but XYZ and the rows of degree 4 and above in which all three
 * components appear: 1, X, Y, Z, the six second-order rows, the six
 * third-order rows without XYZ, and the three rows X2Y2 +/- ... .  Their span is
 * closed under the shift c -> c - u, so N(u) is again unit lower triangular
 * and exact. */
static int basis_row(int j) { return (Q == 19 && j >= 16) ? j + 1 : j; }

void or_moment_matrix(const or_real* u3, or_real* T)
{
    for (int j = 0; j < Q; ++j)
        for (int i = 0; i < Q; ++i)
            T[j * Q + i] = moment_poly(basis_row(j), (or_real)CX[i] - u3[0], (or_real)CY[i] - u3[1],
                                       (or_real)CZ[i] - u3[2]);
}

/* Gauss-Jordan elimination with partial pivoting on |Re|. */
int or_invert(int n, const or_real* A, or_real* Ainv)
{
    or_real* a = (or_real*)malloc(sizeof(or_real) * n * n);
    if (!a) return -1;
    memcpy(a, A, sizeof(or_real) * n * n);
    for (int i = 0; i < n * n; ++i) Ainv[i] = 0;
    for (int i = 0; i < n; ++i) Ainv[i * n + i] = 1;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        double best = fabs((double)RE(a[col * n + col]));
        for (int r = col + 1; r < n; ++r) {
            double v = fabs((double)RE(a[r * n + col]));
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) { free(a); return -2; }
        if (piv != col) {
            for (int k = 0; k < n; ++k) {
                or_real t = a[col * n + k]; a[col * n + k] = a[piv * n + k]; a[piv * n + k] = t;
                t = Ainv[col * n + k]; Ainv[col * n + k] = Ainv[piv * n + k]; Ainv[piv * n + k] = t;
            }
        }
        or_real inv = (or_real)1 / a[col * n + col];
        for (int k = 0; k < n; ++k) { a[col * n + k] *= inv; Ainv[col * n + k] *= inv; }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            or_real fac = a[r * n + col];
            if (RE(fac) == 0 && fac == 0) continue;
            for (int k = 0; k < n; ++k) {
                a[r * n + k] -= fac * a[col * n + k];
                Ainv[r * n + k] -= fac * Ainv[col * n + k];
            }
        }
    }
    free(a);
    return 0;
}

/* M and M^-1 are constants; M^-1 is computed once in double precision from
 * M = T(0) and kept as double (its entries are integers/48, Appendix A). */
static double g_M[Q * Q], g_Minv[Q * Q];
static int g_M_ready = 0;
/* nonzero entries of M^-1 and M as (row, column, value) lists */
static int g_Minv_nnz, g_Minv_k[Q * Q], g_Minv_c[Q * Q];
static double g_Minv_v[Q * Q];
static int g_M_nnz, g_M_r[Q * Q], g_M_c[Q * Q];
static double g_M_v[Q * Q];

static void ensure_M(void)
{
    if (g_M_ready) return;
#pragma omp critical(or_M_init)
    {
        if (!g_M_ready) {
            double a[Q * Q], inv[Q * Q];
            for (int j = 0; j < Q; ++j)
                for (int i = 0; i < Q; ++i) {
                    double X = CX[i], Y = CY[i], Z = CZ[i];
                    /* evaluate the same polynomial rows in double */
                    or_real v = moment_poly(basis_row(j), (or_real)X, (or_real)Y, (or_real)Z);
                    a[j * Q + i] = (double)RE(v);
                }
            memcpy(g_M, a, sizeof(a));
            /* double-precision Gauss-Jordan (same algorithm as or_invert) */
            double w[Q * Q];
            memcpy(w, a, sizeof(a));
            for (int i = 0; i < Q * Q; ++i) inv[i] = 0;
            for (int i = 0; i < Q; ++i) inv[i * Q + i] = 1;
            for (int col = 0; col < Q; ++col) {
                int piv = col;
                for (int r = col + 1; r < Q; ++r)
                    if (fabs(w[r * Q + col]) > fabs(w[piv * Q + col])) piv = r;
                if (piv != col)
                    for (int k = 0; k < Q; ++k) {
                        double t = w[col * Q + k]; w[col * Q + k] = w[piv * Q + k]; w[piv * Q + k] = t;
                        t = inv[col * Q + k]; inv[col * Q + k] = inv[piv * Q + k]; inv[piv * Q + k] = t;
                    }
                double d = 1.0 / w[col * Q + col];
                for (int k = 0; k < Q; ++k) { w[col * Q + k] *= d; inv[col * Q + k] *= d; }
                for (int r = 0; r < Q; ++r) {
                    if (r == col || w[r * Q + col] == 0.0) continue;
                    double fac = w[r * Q + col];
                    for (int k = 0; k < Q; ++k) {
                        w[r * Q + k] -= fac * w[col * Q + k];
                        inv[r * Q + k] -= fac * inv[col * Q + k];
                    }
                }
            }
            /* entries are multiples of 1/48: snap the round-off away */
            for (int i = 0; i < Q * Q; ++i) g_Minv[i] = nearbyint(inv[i] * 48.0) / 48.0;
            g_Minv_nnz = g_M_nnz = 0;
            for (int r = 0; r < Q; ++r)
                for (int c = 0; c < Q; ++c) {
                    if (g_Minv[r * Q + c] != 0.0) {
                        g_Minv_k[g_Minv_nnz] = r; g_Minv_c[g_Minv_nnz] = c;
                        g_Minv_v[g_Minv_nnz++] = g_Minv[r * Q + c];
                    }
                    if (g_M[r * Q + c] != 0.0) {
                        g_M_r[g_M_nnz] = r; g_M_c[g_M_nnz] = c; g_M_v[g_M_nnz++] = g_M[r * Q + c];
                    }
                }
#pragma omp flush
            g_M_ready = 1;
        }
    }
}

/* N = T(u) M^-1 (Appendix A states N = T M^-1); the sum runs over the
 * nonzero entries of the constant M^-1 only. */
void or_shift_matrix(const or_real* u3, or_real* N)
{
    ensure_M();
    or_real T[Q * Q];
    or_moment_matrix(u3, T);
    for (int i = 0; i < Q * Q; ++i) N[i] = 0;
    for (int e = 0; e < g_Minv_nnz; ++e) {
        int k = g_Minv_k[e], c = g_Minv_c[e];
        or_real v = (or_real)g_Minv_v[e];
        for (int r = 0; r < Q; ++r) N[r * Q + c] += T[r * Q + k] * v;
    }
}

/* ---- per-node operators -------------------------------------------------- */

/* varphi_i(alpha_bar), Eq. varphi_ik.  On D3Q27 the moving coefficients are
 * w_i (1 - alpha) / (1 - w_0), so that sum varphi_i = 1 and
 * sum varphi_i c c = (9/19)(1 - alpha) delta.  READING (D3Q19): the same rule,
 * (1 - alpha)/12 on faces and (1 - alpha)/24 on edges, which gives the colour
 * a sound speed squared of (1 - alpha)/2. */
void or_phi_coeffs(or_real ab, or_real* ph)
{
#if defined(OR_Q19)
    for (int i = 0; i < Q; ++i)
        ph[i] = csq(i) == 0 ? ab : csq(i) == 1 ? ((or_real)1 - ab) / (or_real)12
                                                : ((or_real)1 - ab) / (or_real)24;
    return;
#endif
    for (int i = 0; i < Q; ++i) {
        switch (csq(i)) {
        case 0: ph[i] = ab; break;
        case 1: ph[i] = (or_real)2 * ((or_real)1 - ab) / (or_real)19; break;
        case 2: ph[i] = ((or_real)1 - ab) / (or_real)38; break;
        default: ph[i] = ((or_real)1 - ab) / (or_real)152; break;
        }
    }
}

/* isotropic central gradient: grad chi = 3 sum_i w_i chi(x + c_i) c_i
 * (gradient formula at the end of Sec. II, delta_x = delta_t = 1);
 * chi27[i] holds chi(x + c_i). */
void or_gradient(const or_real* chi27, or_real* g3)
{
    or_real gx = 0, gy = 0, gz = 0;
    for (int i = 0; i < Q; ++i) {
        or_real t = (or_real)(3.0 * weight(i)) * chi27[i];
        gx += t * (or_real)CX[i];
        gy += t * (or_real)CY[i];
        gz += t * (or_real)CZ[i];
    }
    g3[0] = gx; g3[1] = gy; g3[2] = gz;
}

/* enhanced equilibrium, Eq. EES with Phi_i of Eq. Phi and the tensor G
 * defined below Eq. order; c = 1.  The D3Q27 Phi_i have sum Phi_i = 0,
 * sum Phi_i c = 0 and sum Phi_i c c = nu_bar [u grad rho + grad rho u +
 * (u . grad rho) I].  READING (D3Q19): Phi_0 = -3 nu_bar u . grad rho as on
 * D3Q27 and Phi_i = m_i nu_bar G' : c_i c_i with G' = 6 G (the symmetric
 * product over 8), m = 2 on faces and 1 on edges: the only such weights
 * with an isotropic fourth moment, and they give the same three moments. */
void or_equilibrium(or_real rho, const or_real* u, or_real ab, or_real nub,
                    const or_real* grho, or_real* feq)
{
    or_real ph[Q];
    or_phi_coeffs(ab, ph);
    or_real u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    /* G = [u (x) grad rho + (u (x) grad rho)^T] / 48 */
    or_real G[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) G[a][b] = (u[a] * grho[b] + u[b] * grho[a]) / (or_real)(Q == 19 ? 8 : 48);
    or_real udr = u[0] * grho[0] + u[1] * grho[1] + u[2] * grho[2];
    for (int i = 0; i < Q; ++i) {
        or_real c[3] = {(or_real)CX[i], (or_real)CY[i], (or_real)CZ[i]};
        or_real cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        or_real poly = (or_real)3 * cu + (or_real)4.5 * cu * cu - (or_real)1.5 * u2
                       + (or_real)4.5 * cu * cu * cu - (or_real)4.5 * cu * u2;
        or_real Phi;
        int k = csq(i);
        if (k == 0) {
            Phi = (or_real)(-3) * nub * udr;
        } else {
            or_real GCC = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) GCC += G[a][b] * c[a] * c[b];
            double m = (Q == 19) ? ((k == 1) ? 2.0 : 1.0) : (k == 1) ? 16.0 : (k == 2) ? 4.0 : 1.0;
            Phi = (or_real)m * nub * GCC;
        }
        feq[i] = rho * (ph[i] + (or_real)weight(i) * poly) + Phi;
    }
}

/* forcing populations F'_i = w_i [3 (c_i - u) + 9 (c_i . u) c_i] . F, Eq. ketFd */
void or_forcing_pop(const or_real* u, const or_real* F, or_real* Fp)
{
    for (int i = 0; i < Q; ++i) {
        or_real c[3] = {(or_real)CX[i], (or_real)CY[i], (or_real)CZ[i]};
        or_real cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        or_real s = 0;
        for (int a = 0; a < 3; ++a) s += ((or_real)3 * (c[a] - u[a]) + (or_real)9 * cu * c[a]) * F[a];
        Fp[i] = (or_real)weight(i) * s;
    }
}

/* y = A x for a dense 27x27 or_real matrix */
static void matvec(const or_real* A, const or_real* x, or_real* y)
{
    for (int r = 0; r < Q; ++r) {
        or_real s = 0;
        for (int c = 0; c < Q; ++c) s += A[r * Q + c] * x[c];
        y[r] = s;
    }
}

/* y = M x and y = M^-1 x over the stored nonzero entries */
static void matvec_M(const or_real* x, or_real* y)
{
    for (int r = 0; r < Q; ++r) y[r] = 0;
    for (int e = 0; e < g_M_nnz; ++e) y[g_M_r[e]] += (or_real)g_M_v[e] * x[g_M_c[e]];
}

static void matvec_Minv(const or_real* x, or_real* y)
{
    for (int r = 0; r < Q; ++r) y[r] = 0;
    for (int e = 0; e < g_Minv_nnz; ++e) y[g_Minv_k[e]] += (or_real)g_Minv_v[e] * x[g_Minv_c[e]];
}

/* x = N^-1 b for the unit lower-triangular shift matrix N (forward
 * substitution; Appendix A gives N lower triangular with unit diagonal). */
static void lower_solve(const or_real* N, const or_real* b, or_real* x)
{
    for (int r = 0; r < Q; ++r) {
        or_real s = b[r];
        for (int c = 0; c < r; ++c) s -= N[r * Q + c] * x[c];
        x[r] = s / N[r * Q + r];
    }
}

/* GMRT single-phase collision plus forcing (Eqs. scoll and ketF):
 *   fdag = f - M^-1 N^-1 K N M (f - feq) + M^-1 N^-1 (I - K/2) N M F'
 * with K = diag[s0, s1 x3, s2nu x5, s2b, s3 x7, s4 x6, s5 x3, s6].
 * READING (D3Q19): K = diag[s0, s1 x3, s2nu x5, s2b, s3 x6, s4 x3], the
 * rates of the rows kept from D3Q27; s5 and s6 have no rows. */
void or_collide(const or_params* p, const or_real* f, const or_real* feq, const or_real* Fp,
                const or_real* u, or_real s2nu, or_real* fdag)
{
    ensure_M();
    or_real N[Q * Q];
    if (p->shift) {
        or_shift_matrix(u, N);
    } else {
        for (int i = 0; i < Q * Q; ++i) N[i] = 0;
        for (int i = 0; i < Q; ++i) N[i * Q + i] = 1;
    }
    or_real K[27];
    K[0] = (or_real)p->rates[0];
    for (int j = 1; j <= 3; ++j) K[j] = (or_real)p->rates[1];
    for (int j = 4; j <= 8; ++j) K[j] = s2nu;
    K[9] = (or_real)p->rates[3];
#if defined(OR_Q19)
    for (int j = 10; j <= 15; ++j) K[j] = (or_real)p->rates[4];
    for (int j = 16; j <= 18; ++j) K[j] = (or_real)p->rates[5];
#else
    for (int j = 10; j <= 16; ++j) K[j] = (or_real)p->rates[4];
    for (int j = 17; j <= 22; ++j) K[j] = (or_real)p->rates[5];
    for (int j = 23; j <= 25; ++j) K[j] = (or_real)p->rates[6];
    K[26] = (or_real)p->rates[7];
#endif

    or_real dif[Q], a[Q], b[Q], c[Q], d[Q], e[Q];
    /* collision term */
    for (int i = 0; i < Q; ++i) dif[i] = f[i] - feq[i];
    matvec_M(dif, a);          /* M (f - feq)           */
    matvec(N, a, b);                /* N M (f - feq)         */
    for (int j = 0; j < Q; ++j) c[j] = K[j] * b[j];
    lower_solve(N, c, d);           /* N^-1 K N M (f - feq)  */
    matvec_Minv(d, e);         /* M^-1 ...              */
    /* forcing term */
    or_real fa[Q], fb[Q], fc[Q], fd[Q], fe[Q];
    matvec_M(Fp, fa);
    matvec(N, fa, fb);
    for (int j = 0; j < Q; ++j) fc[j] = ((or_real)1 - K[j] / (or_real)2) * fb[j];
    lower_solve(N, fc, fd);
    matvec_Minv(fd, fe);
    for (int i = 0; i < Q; ++i) fdag[i] = f[i] - e[i] + fe[i];
}

/* perturbation operator on the colour-blind distribution (Eq. perturb and
 * Eq. B_i).  READING: the projection w_i (c_i . grad phi) / |grad phi|^2 is
 * taken squared, (c_i . grad phi)^2 / |grad phi|^2, which is the continuum-
 * surface-force form the paper cites (the printed linear form does not
 * conserve mass).  READING: the prefactor on the colour-blind f is A, the sum
 * over both colours of A_k/2 with A_r = A_b = A, so that Eq. sigma,
 * sigma = (4/9) A tau, holds.  Switched off where |grad phi| <= grad_eps. */
void or_perturb(const or_params* p, or_real A, const or_real* gphi, or_real* om)
{
    or_real G2 = gphi[0] * gphi[0] + gphi[1] * gphi[1] + gphi[2] * gphi[2];
    if (!(RE(G2) > p->grad_eps * p->grad_eps)) {
        for (int i = 0; i < Q; ++i) om[i] = 0;
        return;
    }
    or_real gn = R_SQRT(G2);
    for (int i = 0; i < Q; ++i) {
        or_real cg = (or_real)CX[i] * gphi[0] + (or_real)CY[i] * gphi[1] + (or_real)CZ[i] * gphi[2];
        om[i] = A * gn * ((or_real)weight(i) * cg * cg / G2 - (or_real)bcoef(i));
    }
}

/* recolouring, Eqs. op3r and op3b, with f^(e)(rho, 0) = rho varphi_i(alpha_bar)
 * (Phi_i vanishes at u = 0) and cos(theta_i) = c_i . grad phi / (|c_i| |grad phi|).
 * READING: cos(theta_0) = 0 (|c_0| = 0), and the beta term is dropped where
 * |grad phi| <= grad_eps. */
void or_recolour(const or_params* p, const or_real* fdag, or_real rho_r, or_real rho_b,
                 or_real ab, const or_real* gphi, or_real* fr, or_real* fb)
{
    or_real rho = rho_r + rho_b;
    or_real ph[Q];
    or_phi_coeffs(ab, ph);
    or_real G2 = gphi[0] * gphi[0] + gphi[1] * gphi[1] + gphi[2] * gphi[2];
    int on = RE(G2) > p->grad_eps * p->grad_eps;
    or_real gn = on ? R_SQRT(G2) : (or_real)1;
    or_real beta = (or_real)p->beta;
    for (int i = 0; i < Q; ++i) {
        or_real cosv = 0;
        if (on && csq(i) > 0) {
            or_real cg = (or_real)CX[i] * gphi[0] + (or_real)CY[i] * gphi[1] + (or_real)CZ[i] * gphi[2];
            cosv = cg / ((or_real)sqrt((double)csq(i)) * gn);
        }
        or_real feq0 = rho * ph[i];
        or_real rec = beta * rho_r * rho_b / (rho * rho) * cosv * feq0;
        fr[i] = rho_r / rho * fdag[i] + rec;
        fb[i] = rho_b / rho * fdag[i] - rec;
    }
}

static double alpha_red(const or_params* p)
{
    /* gamma = rho_r0/rho_b0 = (1 - alpha_b)/(1 - alpha_r) */
    return 1.0 - (1.0 - p->alpha_b) * p->rho_b0 / p->rho_r0;
}

/* one node: everything between streaming steps (Secs. II, Eqs. Momentum to
 * op3b); phi27/rho27 hold the order parameter and density at x + c_i. */
void or_collide_node(const or_params* p, or_real A, const or_real* fr27, const or_real* fb27,
                     const or_real* phi27, const or_real* rho27, or_real* Cr, or_real* Cb)
{
    or_real rho_r = 0, rho_b = 0;
    for (int i = 0; i < Q; ++i) { rho_r += fr27[i]; rho_b += fb27[i]; }
    or_real rho = rho_r + rho_b;
    or_real phi = phi27[0];
    or_real gphi[3], grho[3];
    or_gradient(phi27, gphi);
    or_gradient(rho27, grho);
    double ar = alpha_red(p);
    or_real ab = ((or_real)1 + phi) / (or_real)2 * (or_real)ar
                 + ((or_real)1 - phi) / (or_real)2 * (or_real)p->alpha_b;
    or_real inv_nu = ((or_real)1 + phi) / (or_real)2 / (or_real)p->nu_r
                     + ((or_real)1 - phi) / (or_real)2 / (or_real)p->nu_b;
    or_real nub = (or_real)1 / inv_nu;
    or_real s2nu = p->rates[2] < 0 ? (or_real)1 / ((or_real)3 * nub + (or_real)0.5)
                                   : (or_real)p->rates[2];
    /* body force (Eq. bodyForceJet) and velocity with the half-force term (Eq. Momentum) */
    or_real F[3];
    for (int a = 0; a < 3; ++a) F[a] = (rho - (or_real)p->rho_b0) * (or_real)p->g[a];
    or_real f[Q];
    or_real j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        f[i] = fr27[i] + fb27[i];
        j[0] += f[i] * (or_real)CX[i];
        j[1] += f[i] * (or_real)CY[i];
        j[2] += f[i] * (or_real)CZ[i];
    }
    or_real u[3];
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + F[a] / (or_real)2) / rho;
    or_real feq[Q], Fp[Q], fdag[Q], om[Q];
    or_equilibrium(rho, u, ab, nub, grho, feq);
    or_forcing_pop(u, F, Fp);
    or_collide(p, f, feq, Fp, u, s2nu, fdag);
    or_perturb(p, A, gphi, om);
    for (int i = 0; i < Q; ++i) fdag[i] += om[i];
    or_recolour(p, fdag, rho_r, rho_b, ab, gphi, Cr, Cb);
}

/* ---- whole lattice -------------------------------------------------------- */

static inline int64_t nidx(const or_params* p, int x, int y, int z)
{
    return ((int64_t)z * p->ny + y) * p->nx + x;
}

static inline int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }
static inline int clampi(int a, int n) { return a < 0 ? 0 : (a >= n ? n - 1 : a); }

static int inlet_inside(const or_params* p, int xg, int yg)
{
    if (xg < 0 || xg >= p->nx || yg < 0 || yg >= p->ny) return 0;
    double dx = xg - p->inlet_cx, dy = yg - p->inlet_cy;
    return dx * dx + dy * dy < 0.25 * p->inlet_D * p->inlet_D;
}

/* n-th output (n = 0, 1, ...) of the SplitMix64 generator seeded with `seed`
 * (Steele, Lea and Flood, OOPSLA 2014; finaliser constants of the public
 * reference implementation). */
static uint64_t splitmix64_nth(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + (n + 1u) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* READING (inlet noise, not in the paper): xi in [-1, 1) from the packed
 * counter (t*ny + y)*nx + x. */
double or_noise(uint64_t seed, int64_t t, int32_t x, int32_t y, int32_t nx, int32_t ny)
{
    uint64_t n = ((uint64_t)t * (uint64_t)ny + (uint64_t)y) * (uint64_t)nx + (uint64_t)x;
    uint64_t r = splitmix64_nth(seed, n);
    return (double)(r >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

/* inlet ghost populations at ghost column (xg, yg) for post-collision time t:
 * red equilibrium at rho_r0 with alpha_r, Phi = 0, velocity
 * (u_r e_r, u_z) (Sec. IV A: uniform inflow with the corresponding equilibria). */
static void inlet_ghost(const or_params* p, const or_real* inlet_uz, int xg, int yg, int64_t t,
                        or_real* fe)
{
    double dx = xg - p->inlet_cx, dy = yg - p->inlet_cy;
    double r = sqrt(dx * dx + dy * dy);
    double ur = p->noise_amp * p->inlet_u * or_noise(p->noise_seed, t, xg, yg, p->nx, p->ny);
    or_real u[3];
    u[0] = r > 0 ? (or_real)(ur * dx / r) : (or_real)0;
    u[1] = r > 0 ? (or_real)(ur * dy / r) : (or_real)0;
    u[2] = inlet_uz ? inlet_uz[(int64_t)yg * p->nx + xg] : (or_real)p->inlet_u;
    or_real zero3[3] = {0, 0, 0};
    or_equilibrium((or_real)p->rho_r0, u, (or_real)alpha_red(p), (or_real)1, zero3, fe);
}

/* value of a node field at x + c with the boundary ghost rules:
 * periodic wrap, or (jet) the inlet ghost value inside the circle at z = -1
 * and a mirrored copy (index clamp) across the half-way free-slip walls and
 * at the outlet ghost plane. */
static or_real stencil_get(const or_params* p, const or_real* fld, int x, int y, int z,
                           or_real inlet_value)
{
    if (p->bc == OR_BC_PERIODIC)
        return fld[nidx(p, wrap(x, p->nx), wrap(y, p->ny), wrap(z, p->nz))];
    if (z < 0 && inlet_inside(p, x, y)) return inlet_value;
    return fld[nidx(p, clampi(x, p->nx), clampi(y, p->ny), clampi(z, p->nz))];
}

static int dir_index(int cx, int cy, int cz)
{
    for (int i = 0; i < Q; ++i)
        if (CX[i] == cx && CY[i] == cy && CZ[i] == cz) return i;
    return -1;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* thread count of the parallel loops that follow (n >= 1) */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_step(const or_params* p, const or_real* A, const or_real* inlet_uz, or_real* fr,
            or_real* fb, or_real* hist, int64_t t0, int32_t nsteps)
{
    ensure_M();
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const int64_t N = (int64_t)nx * ny * nz;
    or_real* rr = (or_real*)malloc(sizeof(or_real) * N);
    or_real* rb = (or_real*)malloc(sizeof(or_real) * N);
    or_real* ph = (or_real*)malloc(sizeof(or_real) * N);
    or_real* rt = (or_real*)malloc(sizeof(or_real) * N);
    or_real* Cr = (or_real*)malloc(sizeof(or_real) * Q * N);
    or_real* Cb = (or_real*)malloc(sizeof(or_real) * Q * N);
    if (!rr || !rb || !ph || !rt || !Cr || !Cb) {
        free(rr); free(rb); free(ph); free(rt); free(Cr); free(Cb);
        return -1;
    }
    int mirror[Q][8];
    for (int i = 0; i < Q; ++i)
        for (int m = 0; m < 8; ++m)
            mirror[i][m] = dir_index((m & 1) ? -CX[i] : CX[i], (m & 2) ? -CY[i] : CY[i],
                                     (m & 4) ? -CZ[i] : CZ[i]);

    for (int32_t step = 0; step < nsteps; ++step) {
        const int64_t t = t0 + step;
        /* densities and order parameter (Eq. order) */
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            or_real a = 0, b = 0;
            for (int i = 0; i < Q; ++i) { a += fr[i * N + n]; b += fb[i * N + n]; }
            rr[n] = a; rb[n] = b; rt[n] = a + b;
            or_real sr = a / (or_real)p->rho_r0, sb = b / (or_real)p->rho_b0;
            ph[n] = (sr - sb) / (sr + sb);
        }
        /* collision, perturbation and recolouring at every node */
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
            or_real f1[Q], f2[Q], p27[Q], r27[Q], c1[Q], c2[Q];
            for (int i = 0; i < Q; ++i) {
                f1[i] = fr[i * N + n]; f2[i] = fb[i * N + n];
                p27[i] = stencil_get(p, ph, x + CX[i], y + CY[i], z + CZ[i], (or_real)1);
                r27[i] = stencil_get(p, rt, x + CX[i], y + CY[i], z + CZ[i], (or_real)p->rho_r0);
            }
            or_collide_node(p, A[0], f1, f2, p27, r27, c1, c2);
            for (int i = 0; i < Q; ++i) { Cr[i * N + n] = c1[i]; Cb[i * N + n] = c2[i]; }
        }
        /* streaming (Eq. LBE) with boundary rules */
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
            if (p->bc == OR_BC_JET && z == nz - 1) continue; /* convective outflow below */
            or_real ghost[Q];
            int have_ghost = 0;
            for (int i = 0; i < Q; ++i) {
                int sx = x - CX[i], sy = y - CY[i], sz = z - CZ[i];
                if (p->bc == OR_BC_PERIODIC) {
                    int64_t s = nidx(p, wrap(sx, nx), wrap(sy, ny), wrap(sz, nz));
                    fr[i * N + n] = Cr[i * N + s];
                    fb[i * N + n] = Cb[i * N + s];
                    continue;
                }
                if (sz < 0 && inlet_inside(p, sx, sy)) {
                    /* inflow: populations leave the inlet ghost node (sx, sy, -1) */
                    inlet_ghost(p, inlet_uz, sx, sy, t, ghost);
                    have_ghost = 1;
                    fr[i * N + n] = ghost[i];
                    fb[i * N + n] = 0;
                    continue;
                }
                /* free-slip: specular reflection at the half-way walls x = -1/2,
                 * x = nx - 1/2, y = -1/2, y = ny - 1/2, z = -1/2 (outside the inlet) */
                int m = 0;
                if (sx < 0 || sx >= nx) { m |= 1; sx = x; }
                if (sy < 0 || sy >= ny) { m |= 2; sy = y; }
                if (sz < 0) { m |= 4; sz = z; }
                int ii = mirror[i][m];
                int64_t s = nidx(p, sx, sy, sz);
                fr[i * N + n] = Cr[ii * N + s];
                fb[i * N + n] = Cb[ii * N + s];
            }
            (void)have_ghost;
        }
        if (p->bc == OR_BC_JET) {
            /* convective outflow (Lou et al.): f(N, t+1) = [f(N, t) + lam f(N-1, t+1)]/(1 + lam),
             * lam = U_c = u_z(N-1, t+1).  READING: lam is clamped at 0 (no inflow
             * through the outlet); hist holds f(N, t). */
            const int64_t P = (int64_t)nx * ny;
#pragma omp parallel for schedule(static)
            for (int64_t q = 0; q < P; ++q) {
                int64_t nb = (int64_t)(nz - 2) * P + q, no = (int64_t)(nz - 1) * P + q;
                or_real a = 0, b = 0, jz = 0;
                for (int i = 0; i < Q; ++i) {
                    a += fr[i * N + nb]; b += fb[i * N + nb];
                    jz += (fr[i * N + nb] + fb[i * N + nb]) * (or_real)CZ[i];
                }
                or_real rho = a + b;
                or_real Fz = (rho - (or_real)p->rho_b0) * (or_real)p->g[2];
                or_real uz = (jz + Fz / (or_real)2) / rho;
                or_real lam = RE(uz) > 0 ? uz : (or_real)0;
                for (int i = 0; i < Q; ++i) {
                    or_real vr = (hist[i * P + q] + lam * fr[i * N + nb]) / ((or_real)1 + lam);
                    or_real vb = (hist[(Q + i) * P + q] + lam * fb[i * N + nb]) / ((or_real)1 + lam);
                    fr[i * N + no] = vr; fb[i * N + no] = vb;
                    hist[i * P + q] = vr; hist[(Q + i) * P + q] = vb;
                }
            }
        }
    }
    free(rr); free(rb); free(ph); free(rt); free(Cr); free(Cb);
    return 0;
}

/* per-colour equilibrium from given fields (initial populations):
 * f^k_i = rho_k {varphi_i(alpha_k) + w_i [u terms of Eq. EES]}, Phi = 0 */
void or_init_fields(const or_params* p, const or_real* rho_r, const or_real* rho_b,
                    const or_real* u, or_real* fr, or_real* fb, or_real* hist)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    or_real zero3[3] = {0, 0, 0};
    double ar = alpha_red(p);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        or_real uu[3] = {u ? u[3 * n] : 0, u ? u[3 * n + 1] : 0, u ? u[3 * n + 2] : 0};
        or_real e1[Q], e2[Q];
        or_equilibrium(rho_r[n], uu, (or_real)ar, (or_real)1, zero3, e1);
        or_equilibrium(rho_b[n], uu, (or_real)p->alpha_b, (or_real)1, zero3, e2);
        for (int i = 0; i < Q; ++i) { fr[i * N + n] = e1[i]; fb[i * N + n] = e2[i]; }
    }
    if (p->bc == OR_BC_JET && hist) {
        const int64_t P = (int64_t)p->nx * p->ny;
        for (int64_t q = 0; q < P; ++q)
            for (int i = 0; i < Q; ++i) {
                hist[i * P + q] = fr[i * N + (int64_t)(p->nz - 1) * P + q];
                hist[(Q + i) * P + q] = fb[i * N + (int64_t)(p->nz - 1) * P + q];
            }
    }
}

/* static droplet (Sec. III): rho_r = rho_r0/2 [1 - tanh(2(r - R)/W)],
 * rho_b = rho_b0/2 [1 + tanh(2(r - R)/W)], at rest. */
void or_init_droplet(const or_params* p, double cx, double cy, double cz, double R, double W,
                     or_real* fr, or_real* fb, or_real* hist)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    or_real* a = (or_real*)malloc(sizeof(or_real) * N);
    or_real* b = (or_real*)malloc(sizeof(or_real) * N);
    for (int64_t n = 0; n < N; ++n) {
        int x = (int)(n % p->nx), y = (int)((n / p->nx) % p->ny), z = (int)(n / ((int64_t)p->nx * p->ny));
        double r = sqrt((x - cx) * (x - cx) + (y - cy) * (y - cy) + (z - cz) * (z - cz));
        double th = tanh(2.0 * (r - R) / W);
        a[n] = (or_real)(p->rho_r0 / 2.0 * (1.0 - th));
        b[n] = (or_real)(p->rho_b0 / 2.0 * (1.0 + th));
    }
    or_init_fields(p, a, b, NULL, fr, fb, hist);
    free(a); free(b);
}

void or_macroscopic(const or_params* p, const or_real* fr, const or_real* fb, or_real* rho_r,
                    or_real* rho_b, or_real* u, or_real* phi)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        or_real a = 0, b = 0, j[3] = {0, 0, 0};
        for (int i = 0; i < Q; ++i) {
            a += fr[i * N + n]; b += fb[i * N + n];
            or_real f = fr[i * N + n] + fb[i * N + n];
            j[0] += f * (or_real)CX[i]; j[1] += f * (or_real)CY[i]; j[2] += f * (or_real)CZ[i];
        }
        or_real rho = a + b;
        if (rho_r) rho_r[n] = a;
        if (rho_b) rho_b[n] = b;
        if (u)
            for (int c = 0; c < 3; ++c)
                u[3 * n + c] = (j[c] + (rho - (or_real)p->rho_b0) * (or_real)p->g[c] / (or_real)2) / rho;
        if (phi) {
            or_real sr = a / (or_real)p->rho_r0, sb = b / (or_real)p->rho_b0;
            phi[n] = (sr - sb) / (sr + sb);
        }
    }
}
