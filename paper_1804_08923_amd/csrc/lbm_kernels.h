// HIP kernels of the colour-gradient D3Q27 central-moment LBM step for gfx950.
//
// Design (one MI355X, one process):
//  * State: two population buffers (A-B), structure of arrays, 54 planes of
//    N nodes: planes 0..26 hold the colour-blind deviation d_i = f_i - w_i rho_b0,
//    planes 27..53 the red populations f^r_i; blue is f_i - f^r_i.  d is small
//    in both pure phases (rho_r0 varphi_i(alpha_r) = rho_b0 w_i for |c_i| >= 1
//    because gamma = (1 - alpha_b)/(1 - alpha_r)), so FP32 and 16-bit storage
//    keep the momentum sum_i d_i c_i well conditioned.
//  * Pull streaming: a buffer holds post-collision values at their source
//    node; the pre-collision value of direction i at x is read from x - c_i,
//    and the jet boundary rules are applied at that read.  Right after
//    initialisation the buffer holds the pre-collision state itself
//    ("unshifted"), read without a shift.
//  * A step is two kernels: the density pass (writes phi, rho - rho_b0 and
//    rho_r/rho per node) and the fused collide-perturb-recolour-stream
//    kernel, which reads only the 27 colour-blind deviations (the red
//    populations enter only through rho_r/rho), the 27-point stencil of
//    (phi, rho - rho_b0) and writes all 54 post-collision values.
//  * Launch geometry: grid (ceil(nx*ny/256), nz), so z = blockIdx.y is uniform
//    per block and, when nx is a multiple of 64, y is uniform per wavefront;
//    the z and y boundary branches are then taken by whole wavefronts.  Loads
//    and stores use a uniform plane base plus a 32-bit byte offset.
//  * Collision: with s0 = s1 = 0 and s2b = s3..s6 = 1 (Sec. II) the GMRT
//    collision (Eq. scoll) leaves every central moment at its equilibrium
//    value plus half the forcing moment, except the five deviatoric second-
//    order moments, which relax with s2nu.  The kernel therefore needs only
//    the raw moments of d up to second order, uses the closed-form moments of
//    f^(e) and F' (Eq. EES with Eq. Phi; Eq. ketFd) and maps the relaxed
//    deviatoric central moments back to populations through the tensor-product
//    inverse of the one-dimensional central-moment transform.  This equals
//    f^(e) + F'/2 + (1 - s2nu) T(u)^-1 P T(u) (f - f^(e) + F'/2), P the
//    projector on rows 4..8 of Eq. momentSet.
#pragma once
#include "lbm_lattice.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "cglbm.h"

namespace cglbm {

// ---------------------------------------------------------------- storage codecs
struct StF32 {
    typedef float T;
    static __device__ __forceinline__ float dec(T v) { return v; }
    static __device__ __forceinline__ T enc(float v) { return v; }
};
// bfloat16: upper half of the FP32 pattern, encoded round-to-nearest-even
struct StBF16 {
    typedef uint16_t T;
    static __device__ __forceinline__ float dec(T v) { return __uint_as_float((uint32_t)v << 16); }
    static __device__ __forceinline__ T enc(float v)
    {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) return (T)((u >> 16) | 0x40u);
        u += 0x7fffu + ((u >> 16) & 1u);
        return (T)(u >> 16);
    }
};
// IEEE binary16, hardware conversion (round to nearest even)
struct StF16 {
    typedef _Float16 T;
    static __device__ __forceinline__ float dec(T v) { return (float)v; }
    static __device__ __forceinline__ T enc(float v) { return (T)v; }
};

// ---------------------------------------------------------------- parameters
struct KP {
    int nx, ny, nz, N, plane;
    uint32_t nx_mul;   // p / nx = (p * nx_mul) >> nx_sh, exact for p < 2^31
    int nx_sh;
    float rho_r0, rho_b0, alpha_r, alpha_b;
    float dalpha;      // alpha_r - alpha_b
    float a_minus_w0;  // alpha_b - w_0
    float kappa_b_m1;  // 27 (1 - alpha_b) / 19 - 1
    float inv_nu_r, inv_nu_b, A, beta, eps2;
    float gx, gy, gz;
    float inlet_cx, inlet_cy, inlet_r2, inlet_u, noise_amp;
    uint64_t seed;
    long long t;       // time level of the state that is read
    int unshifted;     // state stored without the streaming shift
    const float* inlet_uz;
};

// node coordinates of this thread: z = blockIdx.y, planar index p
struct Node {
    int x, y, z;
    uint32_t n;
    bool valid;
};

__device__ __forceinline__ Node this_node(const KP& k)
{
    Node d;
    const uint32_t p = blockIdx.x * 256u + threadIdx.x;
    d.valid = p < (uint32_t)k.plane;
    d.z = blockIdx.y;
    d.y = (int)(((uint64_t)p * k.nx_mul) >> k.nx_sh);
    d.x = (int)p - d.y * k.nx;
    d.n = (uint32_t)d.z * (uint32_t)k.plane + p;
    return d;
}

// element idx of a plane, addressed as uniform base + 32-bit byte offset
template <class T>
__device__ __forceinline__ T ldp(const T* __restrict__ base, uint32_t idx)
{
    return *(const T*)((const char*)base + (idx * (uint32_t)sizeof(T)));
}
template <class T>
__device__ __forceinline__ void stp(T* __restrict__ base, uint32_t idx, T v)
{
    *(T*)((char*)base + (idx * (uint32_t)sizeof(T))) = v;
}

__device__ __forceinline__ bool inlet_inside(const KP& k, int xg, int yg)
{
    if (xg < 0 || xg >= k.nx || yg < 0 || yg >= k.ny) return false;
    const float dx = (float)xg - k.inlet_cx, dy = (float)yg - k.inlet_cy;
    return dx * dx + dy * dy < k.inlet_r2;
}

// n-th output of SplitMix64 seeded with `seed` (Steele, Lea and Flood 2014)
__device__ __forceinline__ uint64_t splitmix64_nth(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + (n + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// inlet ghost population of direction I leaving ghost column (xg, yg) at
// post-collision time tg: red equilibrium at rho_r0, alpha_r, Phi = 0, with the
// uniform axial inflow plus the radial noise (Sec. IV A).  Returns f^e_I.
template <int I>
__device__ __forceinline__ float inlet_feq_dir(const KP& k, int xg, int yg, long long tg)
{
    const uint64_t cnt = ((uint64_t)tg * (uint64_t)k.ny + (uint64_t)yg) * (uint64_t)k.nx + (uint64_t)xg;
    const uint64_t r = splitmix64_nth(k.seed, cnt);
    const double xi = (double)(r >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    const float ur = (float)((double)k.noise_amp * (double)k.inlet_u * xi);
    const float dx = (float)xg - k.inlet_cx, dy = (float)yg - k.inlet_cy;
    const float rr = sqrtf(dx * dx + dy * dy);
    const float ux = rr > 0.f ? ur * dx / rr : 0.f, uy = rr > 0.f ? ur * dy / rr : 0.f;
    const float uz = k.inlet_uz ? k.inlet_uz[yg * k.nx + xg] : k.inlet_u;
    const float u2 = ux * ux + uy * uy + uz * uz;
    const float cu = kCX[I] * ux + kCY[I] * uy + kCZ[I] * uz;
    const float poly = cu * (3.f + 4.5f * cu + 4.5f * cu * cu - 4.5f * u2) - 1.5f * u2;
    const float kap_r = (27.f / 19.f) * (1.f - k.alpha_r);
    return k.rho_r0 * wgt(I) * (kap_r + poly);  // |c_I| >= 1 here: varphi_I = w_I kappa_r
}

// ---------------------------------------------------------------- pull with boundary rules
// value of direction P (compile-time plane) at source s
template <class S, int P, bool WANT_FR>
__device__ __forceinline__ void load_pair(const typename S::T* __restrict__ src, size_t N, uint32_t s, float& d,
                                          float& fr)
{
    d = S::dec(ldp(src + (size_t)P * N, s));
    if (WANT_FR) fr = S::dec(ldp(src + (size_t)(Q + P) * N, s));
}

// plane of direction I mirrored across the axes in mask M (bit 1: y, bit 2: z)
template <class S, int I, bool WANT_FR>
__device__ __forceinline__ void load_mirrored_yz(const typename S::T* __restrict__ src, size_t N, int m,
                                                 uint32_t s, float& d, float& fr)
{
    switch (m) {
    case 2: load_pair<S, mirror_dir(I, 2), WANT_FR>(src, N, s, d, fr); break;
    case 4: load_pair<S, mirror_dir(I, 4), WANT_FR>(src, N, s, d, fr); break;
    case 6: load_pair<S, mirror_dir(I, 6), WANT_FR>(src, N, s, d, fr); break;
    default: load_pair<S, I, WANT_FR>(src, N, s, d, fr); break;
    }
}

// Reads the pre-collision value of direction I at node nd.
// Periodic: wrap.  Jet: inlet ghost inside the circle at z = -1, specular
// reflection (free slip) at the half-way walls x, y = -1/2, n - 1/2 and
// z = -1/2 elsewhere.  The outlet plane z = nz - 1 is handled separately.
template <int BC, class S, int I, bool WANT_FR>
__device__ __forceinline__ void pull(const typename S::T* __restrict__ src, size_t N, const KP& k, const Node& nd,
                                     float& d, float& fr)
{
    constexpr int cx = kCX[I], cy = kCY[I], cz = kCZ[I];
    if (k.unshifted) {
        load_pair<S, I, WANT_FR>(src, N, nd.n, d, fr);
        return;
    }
    int s = (int)nd.n - cx - cy * k.nx - cz * k.plane;
    if (BC == LBM_BC_PERIODIC) {
        if (cx > 0 && nd.x == 0) s += k.nx;
        if (cx < 0 && nd.x == k.nx - 1) s -= k.nx;
        if (cy > 0 && nd.y == 0) s += k.plane;
        if (cy < 0 && nd.y == k.ny - 1) s -= k.plane;
        if (cz > 0 && nd.z == 0) s += k.N;
        if (cz < 0 && nd.z == k.nz - 1) s -= k.N;
        load_pair<S, I, WANT_FR>(src, N, (uint32_t)s, d, fr);
        return;
    }
    const bool mz = cz > 0 && nd.z == 0;
    if (mz && inlet_inside(k, nd.x - cx, nd.y - cy)) {
        const float fe = inlet_feq_dir<I>(k, nd.x - cx, nd.y - cy, k.t - 1);
        d = fe - wgt(I) * k.rho_b0;
        if (WANT_FR) fr = fe;
        return;
    }
    const bool mx = (cx > 0 && nd.x == 0) || (cx < 0 && nd.x == k.nx - 1);
    const bool my = (cy > 0 && nd.y == 0) || (cy < 0 && nd.y == k.ny - 1);
    if (mx) s += cx;
    if (my) s += cy * k.nx;
    if (mz) s += cz * k.plane;
    const int myz = (my ? 2 : 0) | (mz ? 4 : 0);
    if (cy == 0 && cz <= 0)
        load_pair<S, I, WANT_FR>(src, N, (uint32_t)s, d, fr);
    else
        load_mirrored_yz<S, I, WANT_FR>(src, N, myz, (uint32_t)s, d, fr);
    if (cx != 0 && mx) {
        switch (myz) {
        case 2: load_pair<S, mirror_dir(I, 3), WANT_FR>(src, N, (uint32_t)s, d, fr); break;
        case 4: load_pair<S, mirror_dir(I, 5), WANT_FR>(src, N, (uint32_t)s, d, fr); break;
        case 6: load_pair<S, mirror_dir(I, 7), WANT_FR>(src, N, (uint32_t)s, d, fr); break;
        default: load_pair<S, mirror_dir(I, 1), WANT_FR>(src, N, (uint32_t)s, d, fr); break;
        }
    }
}

template <int BC, class S, bool WANT_FR, int I = 0>
__device__ __forceinline__ void pull_all(const typename S::T* __restrict__ src, size_t N, const KP& k,
                                         const Node& nd, float* d, float* fr)
{
    if constexpr (I < Q) {
        pull<BC, S, I, WANT_FR>(src, N, k, nd, d[I], fr[I]);
        pull_all<BC, S, WANT_FR, I + 1>(src, N, k, nd, d, fr);
    }
}

// Pre-collision state of an outlet node (x, y, nz - 1) by the convective
// condition f(N) = [f_prev(N) + lam f(N - 1)] / (1 + lam), lam = max(0, u_z(N - 1))
// evaluated on the freshly streamed populations of the node below.
template <class S>
__device__ void outlet_state(const typename S::T* __restrict__ src, size_t N, const KP& k,
                             const float* __restrict__ hist, const Node& nd, float* d, float* fr)
{
    Node nb = nd;
    nb.z = k.nz - 2;
    nb.n = nd.n - (uint32_t)k.plane;
    pull_all<LBM_BC_JET, S, true>(src, N, k, nb, d, fr);
    float m0 = 0.f, jz = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        m0 += d[i];
        if (kCZ[i]) jz += kCZ[i] * d[i];
    }
    const float rho = k.rho_b0 + m0;
    const float uz = (jz + 0.5f * m0 * k.gz) / rho;
    const float lam = uz > 0.f ? uz : 0.f;
    const float inv = 1.f / (1.f + lam);
    const uint32_t q = nd.n - (uint32_t)(k.nz - 1) * (uint32_t)k.plane;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        d[i] = (hist[(size_t)i * k.plane + q] + lam * d[i]) * inv;
        fr[i] = (hist[(size_t)(Q + i) * k.plane + q] + lam * fr[i]) * inv;
    }
}

// full pre-collision state (54 values) of any node
template <int BC, class S>
__device__ __forceinline__ void read_state(const typename S::T* __restrict__ src, size_t N, const KP& k,
                                           const float* __restrict__ hist, const Node& nd, float* d, float* fr)
{
    if (BC == LBM_BC_JET && nd.z == k.nz - 1 && !k.unshifted)
        outlet_state<S>(src, N, k, hist, nd, d, fr);
    else
        pull_all<BC, S, true>(src, N, k, nd, d, fr);
}

// ---------------------------------------------------------------- block reduction (FP64 audit)
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int NV>
__device__ void block_partials(double (&v)[NV], double* __restrict__ out, uint32_t slot)
{
    __shared__ double red[NV][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < NV; ++a) {
        const double s = wave_sum(v[a]);
        if (lane == 0) red[a][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int a = threadIdx.x;
        out[(size_t)slot * NV + a] = red[a][0] + red[a][1] + red[a][2] + red[a][3];
    }
}

// ---------------------------------------------------------------- kernels
constexpr int BLOCK = 256;

// Field layout (float): [0, 2N) (phi, rho - rho_b0) pairs per node, [2N, 3N) rho_r / rho.

// Density pass: rho_r = sum f^r, rho - rho_b0 = sum d; phi (Eq. order).
template <int BC, class S>
__global__ __launch_bounds__(BLOCK) void k_density(const typename S::T* __restrict__ src,
                                                    float* __restrict__ fields,
                                                    const float* __restrict__ hist, KP k)
{
    const Node nd = this_node(k);
    if (!nd.valid) return;
    const size_t N = (size_t)k.N;
    float d[Q], fr[Q];
    read_state<BC, S>(src, N, k, hist, nd, d, fr);
    double m0 = 0.0, rr = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        m0 += (double)d[i];
        rr += (double)fr[i];
    }
    const double rho = (double)k.rho_b0 + m0;
    const double rb = rho - rr;
    const double a = rr / (double)k.rho_r0, b = rb / (double)k.rho_b0;
    stp((float2*)fields, nd.n, make_float2((float)((a - b) / (a + b)), (float)m0));
    stp(fields + 2 * N, nd.n, (float)(rr / rho));
}

// offset to neighbour x + c with the ghost rules: periodic wrap, or (jet) a
// mirrored copy (index clamp) at the walls and the outlet ghost plane; returns
// false where the neighbour is the inlet ghost (phi = 1, rho = rho_r0).
template <int BC, int CX, int CY, int CZ>
__device__ __forceinline__ bool neighbour(const KP& k, const Node& nd, int& s)
{
    s = (int)nd.n + CX + CY * k.nx + CZ * k.plane;
    if (BC == LBM_BC_PERIODIC) {
        if (CX < 0 && nd.x == 0) s += k.nx;
        if (CX > 0 && nd.x == k.nx - 1) s -= k.nx;
        if (CY < 0 && nd.y == 0) s += k.plane;
        if (CY > 0 && nd.y == k.ny - 1) s -= k.plane;
        if (CZ < 0 && nd.z == 0) s += k.N;
        if (CZ > 0 && nd.z == k.nz - 1) s -= k.N;
        return true;
    }
    if (CZ < 0 && nd.z == 0) {
        if (inlet_inside(k, nd.x + CX, nd.y + CY)) return false;
        s -= CZ * k.plane;
    }
    if (CZ > 0 && nd.z == k.nz - 1) s -= CZ * k.plane;
    if ((CX < 0 && nd.x == 0) || (CX > 0 && nd.x == k.nx - 1)) s -= CX;
    if ((CY < 0 && nd.y == 0) || (CY > 0 && nd.y == k.ny - 1)) s -= CY * k.nx;
    return true;
}

__host__ __device__ constexpr double wgtd(int i)
{
    return csq(i) == 0 ? 8.0 / 27.0 : csq(i) == 1 ? 2.0 / 27.0 : csq(i) == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
}

template <int BC, int CX, int CY, int CZ>
__device__ __forceinline__ float2 stencil_value(const float2* __restrict__ pd, const KP& k, const Node& nd)
{
    int s;
    if (neighbour<BC, CX, CY, CZ>(k, nd, s)) return ldp(pd, (uint32_t)s);
    return make_float2(1.f, k.rho_r0 - k.rho_b0);
}

// isotropic gradients 3 sum_i w_i chi(x + c_i) c_i of phi and rho - rho_b0,
// accumulated over opposite pairs (i, i + 1) in FP64: g = (dphi[3], drho[3])
template <int BC, int I = 1>
__device__ __forceinline__ void gradients(const float2* __restrict__ pd, const KP& k, const Node& nd,
                                          double (&g)[6])
{
    if constexpr (I < Q) {
        constexpr int cx = kCX[I], cy = kCY[I], cz = kCZ[I];
        const float2 a = stencil_value<BC, cx, cy, cz>(pd, k, nd);
        const float2 b = stencil_value<BC, -cx, -cy, -cz>(pd, k, nd);
        const double dp = (double)a.x - (double)b.x, dr = (double)a.y - (double)b.y;
        constexpr double w3 = 3.0 * wgtd(I);
        if (cx) { g[0] += (w3 * cx) * dp; g[3] += (w3 * cx) * dr; }
        if (cy) { g[1] += (w3 * cy) * dp; g[4] += (w3 * cy) * dr; }
        if (cz) { g[2] += (w3 * cz) * dp; g[5] += (w3 * cz) * dr; }
        gradients<BC, I + 2>(pd, k, nd, g);
    }
}

// one-dimensional inverse central-moment basis: for shift u, the vectors
// h0, h1 (and the constant h2 = (1/2, -1, 1/2)) over c = -1, 0, 1 whose
// central moments sum_c h_a(c) (c - u)^b are delta_ab (a, b = 0, 1, 2).
struct Basis1D {
    float h0[3], h1[3];  // index c + 1
    __device__ __forceinline__ explicit Basis1D(float u)
    {
        h0[1] = 1.f - u * u;
        h0[2] = 0.5f * (u * u + u);
        h0[0] = 0.5f * (u * u - u);
        h1[1] = -2.f * u;
        h1[2] = u + 0.5f;
        h1[0] = u - 0.5f;
    }
};
__device__ __forceinline__ constexpr float h2(int c) { return c == 0 ? -1.f : 0.5f; }

// Collision, perturbation and recolouring of one node from its pre-collision
// colour-blind deviations d, the centre values phic and xr = rho_r/rho and
// the gradients; writes the 54 post-collision values to dst at node n.  The
// scalar part runs in FP64 (cancellation-prone sums and differences), the
// per-direction part in FP32.
template <class S>
__device__ __forceinline__ void collide_store(const KP& k, const float* d, float phic, float xr,
                                              const double (&g)[6], typename S::T* __restrict__ dst, size_t N,
                                              uint32_t n)
{
    // raw moments of d up to second order
    double m0 = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    double pxx = 0.0, pyy = 0.0, pzz = 0.0, pxy = 0.0, pxz = 0.0, pyz = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double v = d[i];
        m0 += v;
        if (kCX[i]) { jx += kCX[i] * v; pxx += v; }
        if (kCY[i]) { jy += kCY[i] * v; pyy += v; }
        if (kCZ[i]) { jz += kCZ[i] * v; pzz += v; }
        if (kCX[i] * kCY[i]) pxy += (kCX[i] * kCY[i]) * v;
        if (kCX[i] * kCZ[i]) pxz += (kCX[i] * kCZ[i]) * v;
        if (kCY[i] * kCZ[i]) pyz += (kCY[i] * kCZ[i]) * v;
    }
    const double rho = (double)k.rho_b0 + m0;
    const double inv_rho = 1.0 / rho;
    // interpolated properties (Sec. II): alpha_bar, harmonic nu_bar, s2nu
    const float hpf = 0.5f * (1.f + phic), hmf = 0.5f * (1.f - phic);
    const float nubf = 1.f / (hpf * k.inv_nu_r + hmf * k.inv_nu_b);
    const float s2 = 1.f / (3.f * nubf + 0.5f);
    const double hp = 0.5 * (1.0 + (double)phic);
    const double abar = (double)k.alpha_b + hp * (double)k.dalpha;
    const double nub = nubf;
    // body force (Eq. bodyForceJet) and velocity with the half-force term (Eq. Momentum)
    const double Fx = m0 * k.gx, Fy = m0 * k.gy, Fz = m0 * k.gz;
    const double ux = (jx + 0.5 * Fx) * inv_rho, uy = (jy + 0.5 * Fy) * inv_rho, uz = (jz + 0.5 * Fz) * inv_rho;
    // first moments of g = f - f^(e) + F'/2 (vanish up to rounding)
    const double Gx = jx + 0.5 * Fx - rho * ux, Gy = jy + 0.5 * Fy - rho * uy, Gz = jz + 0.5 * Fz - rho * uz;
    const double grx = g[3], gry = g[4], grz = g[5];
    // second raw moments of g without their isotropic parts:
    // sum f^(e) c_a c_b = iso + rho u_a u_b + nu_bar (u_a dr_b + dr_a u_b); sum F' c_a c_b = u_a F_b + u_b F_a
    const double qxy = pxy - rho * ux * uy - nub * (ux * gry + grx * uy) + 0.5 * (ux * Fy + uy * Fx);
    const double qxz = pxz - rho * ux * uz - nub * (ux * grz + grx * uz) + 0.5 * (ux * Fz + uz * Fx);
    const double qyz = pyz - rho * uy * uz - nub * (uy * grz + gry * uz) + 0.5 * (uy * Fz + uz * Fy);
    const double qxx = pxx - rho * ux * ux - 2.0 * nub * ux * grx + ux * Fx;
    const double qyy = pyy - rho * uy * uy - 2.0 * nub * uy * gry + uy * Fy;
    const double qzz = pzz - rho * uz * uz - 2.0 * nub * uz * grz + uz * Fz;
    // central moments (shift by u; the zeroth moment of g is exactly 0 here)
    const double cxy = qxy - ux * Gy - uy * Gx, cxz = qxz - ux * Gz - uz * Gx, cyz = qyz - uy * Gz - uz * Gy;
    const double cxx = qxx - 2.0 * ux * Gx, cyy = qyy - 2.0 * uy * Gy, czz = qzz - 2.0 * uz * Gz;
    const double tr3 = (cxx + cyy + czz) * (1.0 / 3.0);
    const double om = 1.0 - (double)s2;
    // relaxed deviatoric central moments, scaled by (1 - s2nu)
    const float kxy = (float)(om * cxy), kxz = (float)(om * cxz), kyz = (float)(om * cyz);
    const float kxx = (float)(om * (cxx - tr3)), kyy = (float)(om * (cyy - tr3)), kzz = (float)(om * (czz - tr3));
    // equilibrium offsets in deviation form: E0 = rho abar - w_0 rho_b0, E1 = rho kappa - rho_b0
    const double kap = (27.0 / 19.0) * (1.0 - abar);
    const double E0 = (double)k.rho_b0 * (hp * (double)k.dalpha + (double)k.a_minus_w0) + m0 * abar;
    const double E1 = (double)k.rho_b0 * (-(27.0 / 19.0) * hp * (double)k.dalpha + (double)k.kappa_b_m1) + m0 * kap;
    const double u2d = ux * ux + uy * uy + uz * uz;
    const double udr = ux * grx + uy * gry + uz * grz;
    const double uFd = ux * Fx + uy * Fy + uz * Fz;

    // FP32 per-direction part
    const float uxf = (float)ux, uyf = (float)uy, uzf = (float)uz, u2 = (float)u2d;
    const float rhof = (float)rho, E1f = (float)E1, uF = (float)uFd;
    const float Fxf = (float)Fx, Fyf = (float)Fy, Fzf = (float)Fz;
    const float grxf = (float)grx, gryf = (float)gry, grzf = (float)grz;
    const float gpx = (float)g[0], gpy = (float)g[1], gpz = (float)g[2];
    // back-projection of the relaxed moments: Delta(c) = sum_a U_a(cy, cz) h_a(cx, ux),
    // contracted axis by axis (z, then y, then x)
    const Basis1D bx(uxf), by(uyf), bz(uzf);
    float U0[3][3], U1[3][3], U2[3][3];
#pragma unroll
    for (int jz2 = 0; jz2 < 3; ++jz2) {
        const float A_ = kxy * bz.h0[jz2], B_ = kxz * bz.h1[jz2], C_ = kyz * bz.h1[jz2];
        const float D_ = kxx * bz.h0[jz2], E_ = kyy * bz.h0[jz2], G_ = kzz * h2(jz2 - 1);
#pragma unroll
        for (int jy2 = 0; jy2 < 3; ++jy2) {
            U1[jy2][jz2] = A_ * by.h1[jy2] + B_ * by.h0[jy2];
            U0[jy2][jz2] = C_ * by.h1[jy2] + E_ * h2(jy2 - 1) + G_ * by.h0[jy2];
            U2[jy2][jz2] = D_ * by.h0[jy2];
        }
    }
    // perturbation (squared projection, prefactor A) and recolouring weights
    const float G2 = gpx * gpx + gpy * gpy + gpz * gpz;
    const bool on = G2 > k.eps2;
    const float gn = on ? sqrtf(G2) : 0.f;
    const float inv_gn = on ? 1.f / gn : 0.f;
    const float Agn = k.A * gn, Aign = k.A * inv_gn;
    const float rec = k.beta * xr * (1.f - xr) * rhof * (float)kap * inv_gn;
    const float nub9 = 9.f * nubf;

    // rest population
    {
        const float w = wgt(0);
        const float de = (float)(E0 - 1.5 * wgtd(0) * rho * u2d - 3.0 * nub * udr);
        const float Fp = -3.f * w * uF;
        const float pert = on ? k.A * (10.f / 27.f) * gn : 0.f;
        const float delta = U0[1][1] * bx.h0[1] + U1[1][1] * bx.h1[1] + U2[1][1] * h2(0);
        const float dd = de + 0.5f * Fp + delta + pert;
        stp(dst, n, S::enc(dd));
        stp(dst + (size_t)Q * N, n, S::enc(xr * (dd + w * k.rho_b0)));
    }
    // opposite pairs (i, i + 1): shared even parts, odd parts change sign
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const int cx = kCX[i], cy = kCY[i], cz = kCZ[i];
        const float w = wgt(i);
        const float cu = cx * uxf + cy * uyf + cz * uzf;
        const float cr = cx * grxf + cy * gryf + cz * grzf;
        const float cF = cx * Fxf + cy * Fyf + cz * Fzf;
        const float cg = cx * gpx + cy * gpy + cz * gpz;
        const float de_e = w * (E1f + rhof * (4.5f * cu * cu - 1.5f * u2) + nub9 * cu * cr);
        const float de_o = w * rhof * cu * (3.f + 4.5f * cu * cu - 4.5f * u2);
        const float fp_e = 0.5f * w * (9.f * cu * cF - 3.f * uF);
        const float fp_o = 1.5f * w * cF;
        const float pert = w * (Aign * cg * cg - Agn);
        const float even = de_e + fp_e + pert;
        const float odd = de_o + fp_o;
        const float rc = rec * w * inv_len(i) * cg;
        // direction i (+c) and i + 1 (-c)
        const float dl_p = U0[cy + 1][cz + 1] * bx.h0[cx + 1] + U1[cy + 1][cz + 1] * bx.h1[cx + 1]
                           + U2[cy + 1][cz + 1] * h2(cx);
        const float dl_m = U0[1 - cy][1 - cz] * bx.h0[1 - cx] + U1[1 - cy][1 - cz] * bx.h1[1 - cx]
                           + U2[1 - cy][1 - cz] * h2(-cx);
        const float dp = even + odd + dl_p;
        const float dm = even - odd + dl_m;
        stp(dst + (size_t)i * N, n, S::enc(dp));
        stp(dst + (size_t)(i + 1) * N, n, S::enc(dm));
        stp(dst + (size_t)(Q + i) * N, n, S::enc(xr * (dp + w * k.rho_b0) + rc));
        stp(dst + (size_t)(Q + i + 1) * N, n, S::enc(xr * (dm + w * k.rho_b0) - rc));
    }
}

template <int BC, class S>
__global__ __launch_bounds__(BLOCK) void k_collide(const typename S::T* __restrict__ src,
                                                    typename S::T* __restrict__ dst,
                                                    const float* __restrict__ fields,
                                                    float* __restrict__ hist, KP k)
{
    const Node nd = this_node(k);
    if (!nd.valid) return;
    const size_t N = (size_t)k.N;
    float d[Q];
    if (BC == LBM_BC_JET && nd.z == k.nz - 1) {
        float fr[Q];
        read_state<BC, S>(src, N, k, hist, nd, d, fr);
        const uint32_t q = nd.n - (uint32_t)(k.nz - 1) * (uint32_t)k.plane;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            hist[(size_t)i * k.plane + q] = d[i];
            hist[(size_t)(Q + i) * k.plane + q] = fr[i];
        }
    } else {
        float unused[Q];
        pull_all<BC, S, false>(src, N, k, nd, d, unused);
    }
    const float2* pd = (const float2*)fields;
    const float phic = ldp(pd, nd.n).x;
    const float xr = ldp(fields + 2 * N, nd.n);
    double g[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    gradients<BC>(pd, k, nd, g);
    collide_store<S>(k, d, phic, xr, g, dst, N, nd.n);
}

// Initial state (unshifted): per-colour equilibria f^k_i = rho_k {varphi_i(alpha_k)
// + w_i [velocity terms of Eq. EES]} of the droplet / jet preset or of caller
// fields, evaluated in FP64 and rounded once to the storage format.
template <class S>
__global__ __launch_bounds__(BLOCK) void k_init(typename S::T* __restrict__ dst, float* __restrict__ hist,
                                                 KP k, int kind, const float* __restrict__ frr,
                                                 const float* __restrict__ frb, const float* __restrict__ fu,
                                                 double dcx, double dcy, double dcz, double R, double W,
                                                 double rho_r0, double rho_b0, double alpha_r, double alpha_b)
{
    const Node nd = this_node(k);
    if (!nd.valid) return;
    const size_t N = (size_t)k.N;
    double rr, rb, ux = 0, uy = 0, uz = 0;
    if (kind == LBM_INIT_DROPLET) {
        const double dx = nd.x - dcx, dy = nd.y - dcy, dz = nd.z - dcz;
        const double th = tanh(2.0 * (sqrt(dx * dx + dy * dy + dz * dz) - R) / W);
        rr = 0.5 * rho_r0 * (1.0 - th);
        rb = 0.5 * rho_b0 * (1.0 + th);
    } else if (kind == LBM_INIT_JET) {
        rr = 0.0;
        rb = rho_b0;
    } else {
        rr = frr[nd.n];
        rb = frb[nd.n];
        if (fu) {
            ux = fu[3 * nd.n];
            uy = fu[3 * nd.n + 1];
            uz = fu[3 * nd.n + 2];
        }
    }
    const double u2 = ux * ux + uy * uy + uz * uz;
    const double kap_r = 27.0 * (1.0 - alpha_r) / 19.0, kap_b = 27.0 * (1.0 - alpha_b) / 19.0;
    const uint32_t q = nd.n - (uint32_t)(k.nz - 1) * (uint32_t)k.plane;
    const bool outlet = hist != nullptr && nd.z == k.nz - 1;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double w = i == 0 ? 8.0 / 27.0 : csq(i) == 1 ? 2.0 / 27.0 : csq(i) == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
        const double cu = kCX[i] * ux + kCY[i] * uy + kCZ[i] * uz;
        const double poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * u2 + 4.5 * cu * cu * cu - 4.5 * cu * u2;
        double fv, fb;
        if (i == 0) {
            fv = rr * (alpha_r + w * poly);
            fb = rb * (alpha_b + w * poly);
        } else {
            fv = rr * w * (kap_r + poly);
            fb = rb * w * (kap_b + poly);
        }
        const double dv = (fv + fb) - w * rho_b0;
        const typename S::T ed = S::enc((float)dv), ef = S::enc((float)fv);
        stp(dst + (size_t)i * N, nd.n, ed);
        stp(dst + (size_t)(Q + i) * N, nd.n, ef);
        if (outlet) {
            hist[(size_t)i * k.plane + q] = S::dec(ed);
            hist[(size_t)(Q + i) * k.plane + q] = S::dec(ef);
        }
    }
}

// set an explicit (fr, fb) FP32 state, unshifted; d is formed in FP64 and
// rounded once
template <class S>
__global__ __launch_bounds__(BLOCK) void k_set_state(typename S::T* __restrict__ dst, float* __restrict__ hist,
                                                      KP k, const float* __restrict__ st, double rho_b0)
{
    const Node nd = this_node(k);
    if (!nd.valid) return;
    const size_t N = (size_t)k.N;
    const uint32_t q = nd.n - (uint32_t)(k.nz - 1) * (uint32_t)k.plane;
    const bool outlet = hist != nullptr && nd.z == k.nz - 1;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double w = i == 0 ? 8.0 / 27.0 : csq(i) == 1 ? 2.0 / 27.0 : csq(i) == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
        const float fr = st[(size_t)i * N + nd.n], fb = st[(size_t)(Q + i) * N + nd.n];
        const double dv = ((double)fr + (double)fb) - w * rho_b0;
        const typename S::T ed = S::enc((float)dv), ef = S::enc(fr);
        stp(dst + (size_t)i * N, nd.n, ed);
        stp(dst + (size_t)(Q + i) * N, nd.n, ef);
        if (outlet) {
            hist[(size_t)i * k.plane + q] = S::dec(ed);
            hist[(size_t)(Q + i) * k.plane + q] = S::dec(ef);
        }
    }
}

// current state as (fr, fb) FP32 (blue formed in FP64, rounded once)
template <int BC, class S>
__global__ __launch_bounds__(BLOCK) void k_get_state(const typename S::T* __restrict__ src,
                                                      const float* __restrict__ hist, KP k,
                                                      float* __restrict__ st, double rho_b0)
{
    const Node nd = this_node(k);
    if (!nd.valid) return;
    const size_t N = (size_t)k.N;
    float d[Q], fr[Q];
    read_state<BC, S>(src, N, k, hist, nd, d, fr);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double w = i == 0 ? 8.0 / 27.0 : csq(i) == 1 ? 2.0 / 27.0 : csq(i) == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
        st[(size_t)i * N + nd.n] = fr[i];
        st[(size_t)(Q + i) * N + nd.n] = (float)(((double)d[i] + w * rho_b0) - (double)fr[i]);
    }
}

// macroscopic fields and FP64 audit partial sums (one slot per block)
template <int BC, class S>
__global__ __launch_bounds__(BLOCK) void k_macro(const typename S::T* __restrict__ src,
                                                  const float* __restrict__ hist, KP k,
                                                  float* __restrict__ o_rr, float* __restrict__ o_rb,
                                                  float* __restrict__ o_u, float* __restrict__ o_phi,
                                                  double* __restrict__ partials)
{
    const Node nd = this_node(k);
    double acc[5] = {0, 0, 0, 0, 0};
    if (nd.valid) {
        const size_t N = (size_t)k.N;
        float d[Q], fr[Q];
        read_state<BC, S>(src, N, k, hist, nd, d, fr);
        float m0 = 0.f, rr = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            m0 += d[i];
            rr += fr[i];
            if (kCX[i]) jx += kCX[i] * d[i];
            if (kCY[i]) jy += kCY[i] * d[i];
            if (kCZ[i]) jz += kCZ[i] * d[i];
        }
        const float rho = k.rho_b0 + m0;
        const float rb = rho - rr;
        const float px = jx + 0.5f * m0 * k.gx, py = jy + 0.5f * m0 * k.gy, pz = jz + 0.5f * m0 * k.gz;
        const uint32_t n = nd.n;
        if (o_rr) o_rr[n] = rr;
        if (o_rb) o_rb[n] = rb;
        if (o_u) {
            o_u[3 * (size_t)n] = px / rho;
            o_u[3 * (size_t)n + 1] = py / rho;
            o_u[3 * (size_t)n + 2] = pz / rho;
        }
        if (o_phi) {
            const float a = rr / k.rho_r0, b = rb / k.rho_b0;
            o_phi[n] = (a - b) / (a + b);
        }
        acc[0] = rr;
        acc[1] = rb;
        acc[2] = px;
        acc[3] = py;
        acc[4] = pz;
    }
    if (partials) block_partials<5>(acc, partials, blockIdx.y * gridDim.x + blockIdx.x);
}

__global__ __launch_bounds__(BLOCK) void k_audit_final(const double* __restrict__ partials, int nblk,
                                                        double* __restrict__ out)
{
    double acc[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += BLOCK)
#pragma unroll
        for (int a = 0; a < 5; ++a) acc[a] += partials[(size_t)b * 5 + a];
    __shared__ double red[5][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        const double s = wave_sum(acc[a]);
        if (lane == 0) red[a][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < 5)
        out[threadIdx.x] = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
}

}  // namespace cglbm
