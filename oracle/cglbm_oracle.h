/*
 * cglbm_oracle.h -- plain CPU reference (the "oracle") for one time step of
 * the two-colour D3Q27 colour-gradient lattice Boltzmann model with
 * nonorthogonal central moments (Saito, De Rosis, Festuccia, Kaneko, Abe,
 * Koyama, arXiv:1804.08923).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP path; it is
 * never called by the product library.  Only tests/, the smoke entry point
 * and the CPU-baseline leg of bench.py may load it.  It shares no code,
 * tables or headers with the GPU path.
 *
 * One source file is compiled four times:
 *   liboracle.so      real = double          (the FP64 oracle)
 *   liboracle_cs.so   real = double complex  (complex-step tangent-linear)
 *   liboracle_f32.so  real = float           (FP32 floor of the plain scheme)
 *   liboracle_q19.so  real = double, on the D3Q19 subset of the velocity set
 *                     (the reduced lattice of Sec. II; Q = 19 below)
 * Every array argument typed `or_real` takes that build's element type.
 *
 * Population arrays are structure-of-arrays: element (i, node) sits at
 * i*N + node with node = (z*ny + y)*nx + x, i = 0..Q-1 in the order of the
 * paper's velocity set (Eq. velVec); Q = 27, or 19 (rest, faces, edges: the
 * first 19 of that order) in the D3Q19 build.  Sizes written 27 below are Q
 * in the D3Q19 build.
 */
#ifndef CGLBM_ORACLE_H
#define CGLBM_ORACLE_H

#include <stdint.h>

#if defined(OR_COMPLEX)
#include <complex.h>
typedef double _Complex or_real;
#elif defined(OR_FLOAT)
typedef float or_real;
#else
typedef double or_real;
#endif

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_BC_PERIODIC = 0, OR_BC_JET = 1 };

typedef struct or_params {
    int32_t nx, ny, nz;
    int32_t bc;            /* OR_BC_PERIODIC or OR_BC_JET */
    int32_t shift;         /* 1: shift by u (central moments, N(u)); 0: N = I (raw-moment MRT) */
    int32_t pad0;
    double rho_r0, rho_b0; /* phase reference densities; gamma = rho_r0/rho_b0 */
    double alpha_b;        /* alpha of the blue phase; alpha_r follows from gamma */
    double nu_r, nu_b;     /* kinematic viscosities */
    double beta;           /* recolouring parameter */
    double g[3];           /* gravity; body force F = (rho - rho_b0) g */
    double rates[8];       /* s0, s1, s2nu, s2b, s3, s4, s5, s6; s2nu < 0 means "from nu_bar" */
    double grad_eps;       /* |grad phi| <= grad_eps switches perturbation/recolouring term off */
    double inlet_cx, inlet_cy, inlet_D, inlet_u;  /* jet inlet circle and nominal speed */
    double noise_amp;      /* radial inlet noise as a fraction of inlet_u */
    uint64_t noise_seed;
} or_params;

/* lattice tables in the paper's order */
void or_lattice(int32_t* c /* 27x3 */, double* w /* 27 */);

/* moment-basis matrix T(u) of Eq. momentSet evaluated at cbar = c - u; T(0) = M */
void or_moment_matrix(const or_real* u3, or_real* T /* 27x27 row-major */);
/* general inverse by Gauss-Jordan with partial pivoting; returns 0 on success */
int or_invert(int n, const or_real* A, or_real* Ainv);
/* shift matrix N(u) = T(u) M^-1 */
void or_shift_matrix(const or_real* u3, or_real* N);

/* per-node operators (each cites its passage in the source) */
void or_phi_coeffs(or_real alpha_bar, or_real* phi_i);
void or_gradient(const or_real* chi27, or_real* grad3);
void or_equilibrium(or_real rho, const or_real* u, or_real alpha_bar, or_real nu_bar,
                    const or_real* grad_rho, or_real* feq);
void or_forcing_pop(const or_real* u, const or_real* F, or_real* Fp);
void or_collide(const or_params* p, const or_real* f, const or_real* feq, const or_real* Fp,
                const or_real* u, or_real s2nu, or_real* fdag);
void or_perturb(const or_params* p, or_real A, const or_real* grad_phi, or_real* omega2);
void or_recolour(const or_params* p, const or_real* fdag, or_real rho_r, or_real rho_b,
                 or_real alpha_bar, const or_real* grad_phi, or_real* fr, or_real* fb);

/* one full node update from its populations and the 27-point stencils of phi and rho */
void or_collide_node(const or_params* p, or_real A, const or_real* fr27, const or_real* fb27,
                     const or_real* phi27, const or_real* rho27, or_real* Cr, or_real* Cb);

/* whole-lattice operations */
void or_init_fields(const or_params* p, const or_real* rho_r, const or_real* rho_b,
                    const or_real* u /* 3N, xyz interleaved per node */,
                    or_real* fr, or_real* fb, or_real* hist);
void or_init_droplet(const or_params* p, double cx, double cy, double cz, double R, double W,
                     or_real* fr, or_real* fb, or_real* hist);
int or_step(const or_params* p, const or_real* A, const or_real* inlet_uz /* nx*ny or NULL */,
            or_real* fr, or_real* fb, or_real* hist /* 54*nx*ny, jet only */,
            int64_t t0, int32_t nsteps);
void or_macroscopic(const or_params* p, const or_real* fr, const or_real* fb,
                    or_real* rho_r, or_real* rho_b, or_real* u /* 3N */, or_real* phi);
double or_noise(uint64_t seed, int64_t t, int32_t x, int32_t y, int32_t nx, int32_t ny);
int or_num_threads(void);
void or_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
