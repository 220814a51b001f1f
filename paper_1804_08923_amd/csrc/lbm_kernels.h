// HIP kernels of the colour-gradient D3Q27 central-moment LBM step for gfx950.
//
// Design (one MI355X, one process):
//  * Lattice storage is padded by one ghost cell on every side: padded strides
//    px = nx + 2, py = ny + 2, and nz + 2 planes; interior node (x, y, z) sits
//    at ((z + 1) py + y + 1) px + x + 1.  After each pass a small kernel writes
//    into the ghost shell what the boundary rules demand (periodic copies;
//    for the jet, free-slip mirror images, inlet equilibria inside the inlet
//    circle), so the interior kernels pull with one uniform offset per
//    direction and no branches.
//  * Populations: A-B buffers, structure of arrays, planes of NP padded nodes.
//    Planes 0..26 hold the colour-blind deviation d_i = f_i - w_i rho_b0; d is
//    small in both pure phases (rho_r0 varphi_i(alpha_r) = rho_b0 w_i for
//    |c_i| >= 1 because gamma = (1 - alpha_b)/(1 - alpha_r)), so FP32 and
//    16-bit storage keep the momentum sum_i d_i c_i well conditioned.
//  * Colour populations: after recolouring (Eqs. op3r/op3b) with
//    varphi_i = w_i kappa(alpha_bar) for |c_i| >= 1 and cos(theta_i) linear in
//    c_i, the post-collision populations of either colour are
//        f^r*_i = x_r f'_i + (w_i / |c_i|) c_i . V,   f^b*_i = x_b f'_i - (same),
//        x_k = rho_k/rho,  V = beta (rho_r rho_b / rho) kappa grad phi / |grad phi|,
//    affine functions of the colour-blind post-collision f' with four
//    per-node scalars.  The fused kernel therefore stores only d' and the
//    float4 R = (x*, V) of every node, x* the fraction of the kept colour
//    (the one of smaller reference density, see kept_sgn); readers rebuild
//    f^* of direction i at x from d_i and R at the source node x - c_i, and
//    the other colour as f - f^*.  A general state (after initialisation or
//    set_state) keeps the kept colour's populations in planes 27..53 at the
//    node itself ("unshifted") and is read that way by the first step.
//  * A step: density pass (phi, rho - rho_b0, x* per node), ghost fill of
//    those fields, fused collide-perturb-recolour-stream kernel (reads 27
//    deviations and the (phi, rho) stencil, writes 27 deviations and R), ghost
//    fill of the populations.  The jet outlet plane z = nz - 1 (convective
//    condition) is handled inside the density and fused kernels.
//  * Launch geometry: the two stencil kernels take tiles of 128-node x-rows
//    (see "stencil tiles"), z = blockIdx.y + z0; the other kernels a flat
//    grid (ceil(nx*ny/256), planes).
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
#include <type_traits>
#include <stdlib.h>
#include <string.h>

#include "cglbm.h"

namespace cglbm {

// ---------------------------------------------------------------- storage codecs
// kEqRef: the "equilibrium-referenced" 16-bit forms store the moving
// populations relative to a per-node reference equilibrium (see "16-bit
// storage" below) and the rest population exactly, split over two 16-bit
// planes; the plain 16-bit forms store the deviation d_i itself.
struct StF32 {
    typedef float T;
    static constexpr bool kEqRef = false;
    static __device__ __forceinline__ float dec(T v) { return v; }
    static __device__ __forceinline__ T enc(float v) { return v; }
};
// bfloat16: upper half of the FP32 pattern; encoded round-to-nearest-even by
// the gfx950 conversion instruction (v_cvt_pk_bf16_f32)
template <bool EQ>
struct StBF16T {
    typedef uint16_t T;
    static constexpr bool kEqRef = EQ;
    static __device__ __forceinline__ float dec(T v) { return __uint_as_float((uint32_t)v << 16); }
    static __device__ __forceinline__ T enc(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
    static __device__ __forceinline__ float dec_bits(uint32_t b) { return __uint_as_float(b << 16); }
    static __device__ __forceinline__ uint32_t enc_bits(float v) { return enc(v); }
};
// IEEE binary16, hardware conversion (round to nearest even)
template <bool EQ>
struct StF16T {
    typedef _Float16 T;
    static constexpr bool kEqRef = EQ;
    static __device__ __forceinline__ float dec(T v) { return (float)v; }
    static __device__ __forceinline__ T enc(float v) { return (T)v; }
    static __device__ __forceinline__ float dec_bits(uint32_t b)
    {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)b);
    }
    static __device__ __forceinline__ uint32_t enc_bits(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
};
using StBF16 = StBF16T<false>;
using StF16 = StF16T<false>;
using StBF16Eq = StBF16T<true>;
using StF16Eq = StF16T<true>;

// ---------------------------------------------------------------- parameters
struct KP {
    int nx, ny, nz;    // interior lattice
    int px, py;        // padded strides: nx + 2, ny + 2
    uint32_t NP;       // padded node count px * py * (nz + 2)
    uint32_t N;        // interior node count nx * ny * nz
    uint32_t plane;    // nx * ny
    uint32_t nx_mul;   // p / nx = (p * nx_mul) >> nx_sh, exact for p < 2^31
    int nx_sh;
    int ntx;           // stencil tiles (STX wide) along x
    int z0;            // interior plane of blockIdx.y = 0
    float rho_r0, rho_b0, alpha_r, alpha_b;
    float dalpha;      // alpha_r - alpha_b
    float a_minus_w0;  // alpha_b - w_0
    float kappa_b_m1;  // 27 (1 - alpha_b) / 19 - 1
    float inv_nu_r, inv_nu_b, A, beta, eps2;
    float gx, gy, gz;
    float inlet_cx, inlet_cy, inlet_r2, inlet_u, noise_amp;
    uint64_t seed;
    long long t;       // time level of the state that is read
    int unshifted;     // general state (54 planes) stored without the streaming shift
    int xr_tagged;     // adjoint passes: XR holds the tagged minority fraction (else rho_r / rho)
    const float* inlet_uz;
    const float4* R;   // (tagged minority fraction, V) of the state that is read
    const uint4* Qrec; // referenced 16-bit storage: reference record of the state that is read
};

struct MirrorTable {
    int8_t v[Q * 8];
};
constexpr MirrorTable make_mirror()
{
    MirrorTable t{};
    for (int i = 0; i < Q; ++i)
        for (int m = 0; m < 8; ++m) t.v[i * 8 + m] = (int8_t)mirror_dir(i, m);
    return t;
}
// direction i with the components in mask m (bit 0: x, 1: y, 2: z) reversed
__constant__ MirrorTable kMirror = make_mirror();

__device__ __forceinline__ uint32_t pidx(const KP& k, int x, int y, int z)
{
    return ((uint32_t)(z + 1) * (uint32_t)k.py + (uint32_t)(y + 1)) * (uint32_t)k.px + (uint32_t)(x + 1);
}

// padded-index offset of lattice velocity (cx, cy, cz)
__device__ __forceinline__ int doff(const KP& k, int cx, int cy, int cz)
{
    return cx + cy * k.px + cz * k.px * k.py;
}

// interior node of this thread: z = blockIdx.y + z0
struct Node {
    int x, y, z;
    uint32_t n;  // padded index
    uint32_t q;  // y nx + x (index within an interior plane)
    bool valid;
};

__device__ __forceinline__ Node this_node(const KP& k)
{
    Node d;
    const uint32_t p = blockIdx.x * 256u + threadIdx.x;
    d.valid = p < k.plane;
    d.z = (int)blockIdx.y + k.z0;
    d.y = (int)(((uint64_t)p * k.nx_mul) >> k.nx_sh);
    d.x = (int)p - d.y * k.nx;
    d.q = p;
    d.n = pidx(k, d.x, d.y, d.z);
    return d;
}

// element idx of a plane, addressed as uniform base + byte offset (32-bit for
// elements of up to 8 bytes: at most 2^29 padded nodes)
template <class T>
__device__ __forceinline__ T ldp(const T* __restrict__ base, uint32_t idx)
{
    if constexpr (sizeof(T) >= 16)  // 16-byte records: 64-bit offsets (more than 2^28 nodes)
        return *(const T*)((const char*)base + (size_t)idx * sizeof(T));
    else
        return *(const T*)((const char*)base + (idx * (uint32_t)sizeof(T)));
}
template <class T>
__device__ __forceinline__ void stp(T* __restrict__ base, uint32_t idx, T v)
{
    if constexpr (sizeof(T) >= 16)
        *(T*)((char*)base + (size_t)idx * sizeof(T)) = v;
    else
        *(T*)((char*)base + (idx * (uint32_t)sizeof(T))) = v;
}

// Population planes through buffer resources: the plane's base address sits
// in scalar registers and the lane supplies only the byte offset n * sizeof(T)
// (one offset shared by all 27 directions), so a pull costs no per-lane
// address arithmetic.  The resource starts at element -off of the plane (the
// shift of a pull direction) and its record count bounds every access to the
// plane (out-of-range loads read 0 and out-of-range stores are dropped).
template <class T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const T* base, uint32_t elems)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0, (int)(elems * (uint32_t)sizeof(T)),
                                             0x00020000);
}
// element n - off of plane p (2- or 4-byte elements)
template <class T>
__device__ __forceinline__ T ldpl(const T* __restrict__ p, int off, uint32_t NP, uint32_t n)
{
    static_assert(sizeof(T) == 2 || sizeof(T) == 4, "population planes hold 2- or 4-byte values");
    const auto r = plane_rsrc(p - off, NP + (uint32_t)(off < 0 ? -off : off));
    const uint32_t b = n * (uint32_t)sizeof(T);
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, b, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, b, 0, 0));
}
// store v as element n of plane p
template <class T>
__device__ __forceinline__ void stpl(T* __restrict__ p, uint32_t NP, uint32_t n, T v)
{
    const auto r = plane_rsrc(p, NP);
    if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, n * 4u, 0, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, n * 2u, 0, 0);
}

// 16-byte record (R, reference record) of node n, which lies in padded plane
// z + 1 (n or a neighbour in the same row), stored through a buffer resource
// based at that plane: the per-lane offset stays within one plane (32 bits
// for any lattice), so the store needs no 64-bit per-lane address.
template <class T>
__device__ __forceinline__ void st_rec(T* __restrict__ base, const KP& k, int z, uint32_t n, T v)
{
    static_assert(sizeof(T) == 16, "16-byte records");
    const uint32_t pp = (uint32_t)k.px * (uint32_t)k.py, p0 = (uint32_t)(z + 1) * pp;
    const auto r = plane_rsrc(base + p0, pp);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) uint32_t, v), r,
                                           (n - p0) * 16u, 0, 0);
}

// ---------------------------------------------------------------- 16-bit storage
// In the plain 16-bit forms the stored deviation d_i = f_i - w_i rho_b0 of a
// moving direction carries the velocity part of the equilibrium,
// w_i rho (3 c.u + ...), and at interfaces its phase part w_i (rho kappa -
// rho_b0); their 16-bit rounding feeds an O(2^-9 |u|) momentum error into
// every step.  The equilibrium-referenced forms remove both: the collision
// writes, per node, a reference record (rho~, u~, E~) rounded to the storage
// format, E = rho kappa(alpha_bar) - rho_b0, and stores
//   e_i = d'_i - w_i (E~ + rho~ P_i(u~)),
//   P_i(u) = c.u (3 + 4.5 (c.u)^2 - 4.5 u^2) + 4.5 (c.u)^2 - 1.5 u^2;
// readers add the same term computed from the same rounded record, so only
// the rounding of the small remainder e_i is lost.  The rest population (O(1)
// in the red phase) is kept exactly: its FP32 bits are split over plane 0
// (high half) and plane Q (low half; the red planes are used only by a
// general state, never together with this form).
__device__ __forceinline__ float eq_poly(float cu, float u2)
{
    return cu * (3.f + 4.5f * cu * cu - 4.5f * u2) + (4.5f * cu * cu - 1.5f * u2);
}

struct RefRec {
    float rho, ux, uy, uz, e;
};

template <class S>
__device__ __forceinline__ RefRec dec_ref(uint4 q)
{
    RefRec r;
    r.rho = S::dec_bits(q.x & 0xffffu);
    r.ux = S::dec_bits(q.x >> 16);
    r.uy = S::dec_bits(q.y & 0xffffu);
    r.uz = S::dec_bits(q.y >> 16);
    r.e = S::dec_bits(q.z & 0xffffu);
    return r;
}

template <class S>
__device__ __forceinline__ uint4 enc_ref(float rho, float ux, float uy, float uz, float e)
{
    return make_uint4(S::enc_bits(rho) | (S::enc_bits(ux) << 16), S::enc_bits(uy) | (S::enc_bits(uz) << 16),
                      S::enc_bits(e), 0u);
}

// the reference of a ghost cell that mirrors a node across the walls in mask m
__device__ __forceinline__ uint4 mirror_ref(uint4 q, int m)
{
    if (m & 1) q.x ^= 0x80000000u;
    if (m & 2) q.y ^= 0x00008000u;
    if (m & 4) q.y ^= 0x80000000u;
    return q;
}

// deviation d_I = f_I - w_I rho_b0 of direction I stored at padded node
// s = n - off of a post-collision (shifted) state
template <class S, int I>
__device__ __forceinline__ float load_dev(const typename S::T* __restrict__ src, const KP& k, uint32_t n, int off)
{
    if constexpr (!S::kEqRef) {
        return S::dec(ldpl(src + (size_t)I * k.NP, off, k.NP, n));
    } else if constexpr (I == 0) {
        const uint32_t hi = __builtin_bit_cast(uint16_t, ldpl(src, off, k.NP, n));
        const uint32_t lo = __builtin_bit_cast(uint16_t, ldpl(src + (size_t)Q * k.NP, off, k.NP, n));
        return __uint_as_float((hi << 16) | lo);
    } else {
        const RefRec r = dec_ref<S>(ldp(k.Qrec, n - (uint32_t)off));
        const float cu = kCX[I] * r.ux + kCY[I] * r.uy + kCZ[I] * r.uz;
        const float u2 = r.ux * r.ux + r.uy * r.uy + r.uz * r.uz;
        return S::dec(ldpl(src + (size_t)I * k.NP, off, k.NP, n)) + wgt(I) * (r.e + r.rho * eq_poly(cu, u2));
    }
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

// ---------------------------------------------------------------- colour fractions
// The recolouring of a node needs x_r = rho_r/rho and x_b = 1 - x_r.  FP32
// keeps a fraction near 1 only to an absolute 2^-24, which leaves the other
// colour a relative error 2^-24/x, and Eq. order multiplies the error of
// rho_k by rho/rho_k0 (up to gamma where the dense colour dominates).  A node
// therefore keeps the fraction of its minority colour, with full relative
// precision at both ends, and marks which colour that is in the lowest
// mantissa bit: 0 red (the value is x_r), 1 blue (the value is x_b).  The
// mark costs one bit of the fraction: the value is the FP32 number nearest to
// the fraction among those with the right lowest bit (an unbiased rounding to
// a grid of two ulps, so colour masses do not drift).  The other colour is
// always formed as the colour-blind value minus the kept one.
__device__ __forceinline__ uint32_t blue_kept(float s) { return __float_as_uint(s) & 1u; }
__device__ __forceinline__ float frac_tag(double x, uint32_t blue)
{
    const float f = (float)x;
    uint32_t b = __float_as_uint(f);
    if ((b & 1u) != blue) {
        if ((b & 0x7fffffffu) == 0u)
            b |= 1u;  // +-0: the smallest magnitude that carries the mark
        else
            b += fabs(x) > fabs((double)f) ? 1u : 0xffffffffu;  // one ulp towards x (in magnitude)
    }
    return __uint_as_float(b);
}
// the fraction of colour `blue` (0 red, 1 blue) from a tagged value s
__device__ __forceinline__ float frac_of(float s, uint32_t blue) { return blue_kept(s) == blue ? s : 1.f - s; }

// ---------------------------------------------------------------- pull
// Pre-collision value of direction I at padded node n of a post-collision
// (shifted) state: d from plane I at n - c_I (an interior node or a filled
// ghost cell), both colours rebuilt from R there (Eqs. op3r/op3b):
//   f^k*_i = x_k f'_i +- (w_i/|c_i|) c_i . V   (+ red, - blue),
// the kept colour from its fraction, the other as f - f^k (formed in FP64,
// rounded once).
__device__ __forceinline__ float other_colour(const KP& k, int i, float d, float fk)
{
    return (float)(((double)d + wgtd(i) * (double)k.rho_b0) - (double)fk);
}

template <class S, int I, bool WANT_F>
__device__ __forceinline__ void pull_shifted(const typename S::T* __restrict__ src, const KP& k, uint32_t n,
                                             float& d, float& fr, float& fb)
{
    const int off = doff(k, kCX[I], kCY[I], kCZ[I]);
    const uint32_t s = n - (uint32_t)off;
    d = load_dev<S, I>(src, k, n, off);
    if (WANT_F) {
        const float4 r = ldp(k.R, s);
        const float f = d + wgt(I) * k.rho_b0;
        const float vt = I == 0 ? 0.f : (wgt(I) * inv_len(I)) * (kCX[I] * r.y + kCY[I] * r.z + kCZ[I] * r.w);
        const uint32_t bl = blue_kept(r.x);
        const float fk = r.x * f + (bl ? -vt : vt);
        const float fo = other_colour(k, I, d, fk);
        fr = bl ? fo : fk;
        fb = bl ? fk : fo;
    }
}

// value of direction I of a general state stored at node n itself: planes
// Q..2Q-1 hold the populations of the colour the flag of R[n] names
template <class S, int I, bool WANT_F>
__device__ __forceinline__ void pull_general(const typename S::T* __restrict__ src, const KP& k, uint32_t n,
                                             float& d, float& fr, float& fb)
{
    d = S::dec(ldp(src + (size_t)I * k.NP, n));
    if (WANT_F) {
        const float fk = S::dec(ldp(src + (size_t)(Q + I) * k.NP, n));
        const float fo = other_colour(k, I, d, fk);
        const uint32_t bl = blue_kept(ldp(k.R, n).x);
        fr = bl ? fo : fk;
        fb = bl ? fk : fo;
    }
}

template <class S, bool WANT_F, bool SHIFTED, int I = 0>
__device__ __forceinline__ void pull_dirs(const typename S::T* __restrict__ src, const KP& k, uint32_t n, float* d,
                                          float* fr, float* fb)
{
    if constexpr (I < Q) {
        if constexpr (SHIFTED)
            pull_shifted<S, I, WANT_F>(src, k, n, d[I], fr[I], fb[I]);
        else
            pull_general<S, I, WANT_F>(src, k, n, d[I], fr[I], fb[I]);
        pull_dirs<S, WANT_F, SHIFTED, I + 1>(src, k, n, d, fr, fb);
    }
}

// the 27 pre-collision deviations (and colour populations) at padded node n
template <class S, bool WANT_F>
__device__ __forceinline__ void pull_all(const typename S::T* __restrict__ src, const KP& k, uint32_t n, float* d,
                                         float* fr, float* fb)
{
    if (k.unshifted)
        pull_dirs<S, WANT_F, false>(src, k, n, d, fr, fb);
    else
        pull_dirs<S, WANT_F, true>(src, k, n, d, fr, fb);
}

// Pre-collision state of an outlet node (x, y, nz - 1) by the convective
// condition f(N) = [f_prev(N) + lam f(N - 1)] / (1 + lam), lam = max(0, u_z(N - 1))
// evaluated on the freshly streamed populations of the node below; hprev holds
// the outlet plane of the previous step (d, then f^r); blue is formed as f - f^r.
template <class S>
__device__ void outlet_state(const typename S::T* __restrict__ src, const KP& k, const float* __restrict__ hprev,
                             const Node& nd, float* d, float* fr, float* fb)
{
    if (k.unshifted) {
        pull_all<S, true>(src, k, nd.n, d, fr, fb);
        return;
    }
    pull_all<S, true>(src, k, nd.n - (uint32_t)(k.px * k.py), d, fr, fb);
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
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        d[i] = (hprev[(size_t)i * k.plane + nd.q] + lam * d[i]) * inv;
        fr[i] = (hprev[(size_t)(Q + i) * k.plane + nd.q] + lam * fr[i]) * inv;
        fb[i] = other_colour(k, i, d[i], fr[i]);
    }
}

// full pre-collision state (deviations and both colours) of any interior node
template <int BC, class S>
__device__ __forceinline__ void read_state(const typename S::T* __restrict__ src, const KP& k,
                                           const float* __restrict__ hprev, const Node& nd, float* d, float* fr,
                                           float* fb)
{
    if (BC == LBM_BC_JET && nd.z == k.nz - 1)
        outlet_state<S>(src, k, hprev, nd, d, fr, fb);
    else
        pull_all<S, true>(src, k, nd.n, d, fr, fb);
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

constexpr int BLOCK = 256;

// ---------------------------------------------------------------- stencil tiles
// The two stencil kernels (density pass, fused collision) take a tile of
// STX x STY nodes of one plane per block and stage the neighbour data they
// gather 26 times per node (the recolouring float4 R of the density pass, the
// (phi, rho) fields of the gradient) once into LDS: a window of the tile plus a
// one-node rim in x and y, over planes z - 1, z, z + 1, loaded row by row.
constexpr int STX = 128, STY = BLOCK / STX;
// the density pass takes 128 x 4 tiles (512 threads): measured faster than
// 128 x 2 and 128 x 8 (less window rim per node, enough blocks per CU)
constexpr int DTY = 4, DBLOCK = STX * DTY;

template <int TY>
struct TileShape {
    static constexpr int WX = STX + 2, WY = TY + 2, W = 3 * WX * WY, NT = STX * TY;
};
constexpr int SWX = STX + 2, SWY = STY + 2, SW = 3 * SWX * SWY;

struct Tile {
    int x0, y0, z, lx, ly;
    Node nd;
};

template <int TY = STY>
__device__ __forceinline__ Tile this_tile(const KP& k)
{
    Tile t;
    // XCD-aware order: workgroups go round-robin to the 8 XCDs, so a plane's
    // neighbouring tiles would sit on different L2s, each fetching the halo
    // rows they share.  When the plane's tile count T is a multiple of 8, XCD
    // j takes the contiguous band of tiles [j T/8, (j+1) T/8) of every plane
    // (a bijection on the plane's tiles; tile t of planes z and z + 1 still
    // lands on one XCD, as it does in the plain order for such T).
    uint32_t b = blockIdx.x;
    if ((gridDim.x & 7u) == 0) b = (b & 7u) * (gridDim.x >> 3) + (b >> 3);
    const int ty = (int)b / k.ntx, tx = (int)b - ty * k.ntx;
    t.x0 = tx * STX;
    t.y0 = ty * TY;
    t.z = (int)blockIdx.y + k.z0;
    t.lx = (int)threadIdx.x % STX;
    t.ly = (int)threadIdx.x / STX;
    Node& d = t.nd;
    d.x = t.x0 + t.lx;
    d.y = t.y0 + t.ly;
    d.z = t.z;
    d.valid = d.x < k.nx && d.y < k.ny;
    d.q = (uint32_t)d.y * (uint32_t)k.nx + (uint32_t)d.x;
    d.n = pidx(k, d.x, d.y, d.z);
    return t;
}

// window slot of the node at offset (dx, dy, dz) from local node (lx, ly)
template <int TY = STY>
__device__ __forceinline__ int wslot(int lx, int ly, int dx, int dy, int dz)
{
    return ((dz + 1) * TileShape<TY>::WY + (ly + 1 + dy)) * TileShape<TY>::WX + (lx + 1 + dx);
}

// stage field f over the window of tile t (padded cells beyond the ghost
// shell of a ragged last tile are skipped: no valid node reads them).
// BATCH issues all of a lane's loads before its LDS writes: one memory latency
// for the window instead of one per element of the loop.  Measured on the
// 128x128x512 jet: fused kernel 468 -> 464 us (FP32), 322 -> 294 us (BF16),
// adjoint step 1.95 -> 1.73 ms; whole step faster in every storage except
// through the density pass of the equilibrium-referenced forms (3 us slower
// there, so they keep the loop).
template <int TY = STY, bool BATCH = false, class T>
__device__ __forceinline__ void load_window(T* __restrict__ win, const T* __restrict__ f, const KP& k, const Tile& t)
{
    using TS = TileShape<TY>;
    if constexpr (BATCH) {
        constexpr int NIT = (TS::W + TS::NT - 1) / TS::NT;
        T v[NIT];
        bool ok[NIT];
#pragma unroll
        for (int j = 0; j < NIT; ++j) {
            const int w = (int)threadIdx.x + j * TS::NT;
            const int wx = w % TS::WX, r = w / TS::WX;
            const int wy = r % TS::WY, wz = r / TS::WY;
            const int x = t.x0 - 1 + wx, y = t.y0 - 1 + wy;
            ok[j] = w < TS::W && x <= k.nx && y <= k.ny;
            if (ok[j]) v[j] = ldp(f, pidx(k, x, y, t.z - 1 + wz));
        }
#pragma unroll
        for (int j = 0; j < NIT; ++j)
            if (ok[j]) win[(int)threadIdx.x + j * TS::NT] = v[j];
    } else {
        for (int w = threadIdx.x; w < TS::W; w += TS::NT) {
            const int wx = w % TS::WX, r = w / TS::WX;
            const int wy = r % TS::WY, wz = r / TS::WY;
            const int x = t.x0 - 1 + wx, y = t.y0 - 1 + wy;
            if (x <= k.nx && y <= k.ny) win[w] = ldp(f, pidx(k, x, y, t.z - 1 + wz));
        }
    }
}

// ---------------------------------------------------------------- density pass
// n / d for the O(1), positive denominators of the fields (a density, a sum
// of two): the hardware reciprocal refined by two Newton steps and one
// residual correction, a few FP64 ulps from the rounded quotient, which the
// callers then round to FP32.  Saves the scaling and fix-up steps of the IEEE
// division, which these operands need no cover for (no zero, denormal or
// infinite values).
__device__ __forceinline__ double div_fields(double n, double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    const double q = n * r;
    return fma(fma(-d, q, n), r, q);
}

// fields: PD = (phi, rho - rho_b0) per padded node and XR = the minority
// colour's fraction, tagged (see "colour fractions"), from the mass sum
// m0 = rho - rho_b0 and the two colour masses.  phi = (rho_r/rho_r0 -
// rho_b/rho_b0) / (rho_r/rho_r0 + rho_b/rho_b0) (Eq. order) with both
// quotients scaled by rho_r0 rho_b0: one division.
__device__ __forceinline__ float2 store_pd(float2* __restrict__ PD, const KP& k, uint32_t n, double m0, double rr,
                                           double rb)
{
    const double a = rr * (double)k.rho_b0, b = rb * (double)k.rho_r0;
    const float2 v = make_float2((float)div_fields(a - b, a + b), (float)m0);
    stp(PD, n, v);
    return v;
}

__device__ __forceinline__ float2 store_fields_sums(float2* __restrict__ PD, float* __restrict__ XR, const KP& k,
                                                    uint32_t n, double m0, double rr, double rb)
{
    const double rho = (double)k.rho_b0 + m0;
    const float2 v = store_pd(PD, k, n, m0, rr, rb);
    const uint32_t bl = rr > rb;
    stp(XR, n, frac_tag(div_fields(bl ? rb : rr, rho), bl));
    return v;
}

__device__ __forceinline__ float2 store_fields(float2* __restrict__ PD, float* __restrict__ XR, const KP& k,
                                               uint32_t n, const float* d, const float* fr)
{
    double m0 = 0.0, rr = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        m0 += (double)d[i];
        rr += (double)fr[i];
    }
    return store_fields_sums(PD, XR, k, n, m0, rr, (double)k.rho_b0 + m0 - rr);
}

// The (phi, rho - rho_b0) of the ghost shell, written by the node each ghost
// cell images: periodic copies across the wrap, or (jet) mirrored copies
// across the half-way walls and the outlet, and (1, rho_r0 - rho_b0) in the
// inlet circle at z = -1.  Only nodes on a face of the lattice write.
template <int BC>
__device__ __forceinline__ void store_pd_ghosts(float2* __restrict__ PD, const KP& k, int x, int y, int z, float2 v)
{
    const bool yzf = y == 0 || y == k.ny - 1 || z == 0 || z == k.nz - 1;
    if (!yzf) {  // the common case: an x face only (every row has two)
        if (x == 0) stp(PD, pidx(k, BC == LBM_BC_PERIODIC ? k.nx : -1, y, z), v);
        if (x == k.nx - 1) stp(PD, pidx(k, BC == LBM_BC_PERIODIC ? -1 : k.nx, y, z), v);
        return;
    }
    int ix[3] = {x, 0, 0}, iy[3] = {y, 0, 0}, iz[3] = {z, 0, 0};
    int nx = 1, ny = 1, nz = 1;
    if (BC == LBM_BC_PERIODIC) {
        if (x == 0) ix[nx++] = k.nx;
        if (x == k.nx - 1) ix[nx++] = -1;
        if (y == 0) iy[ny++] = k.ny;
        if (y == k.ny - 1) iy[ny++] = -1;
        if (z == 0) iz[nz++] = k.nz;
        if (z == k.nz - 1) iz[nz++] = -1;
    } else {
        if (x == 0) ix[nx++] = -1;
        if (x == k.nx - 1) ix[nx++] = k.nx;
        if (y == 0) iy[ny++] = -1;
        if (y == k.ny - 1) iy[ny++] = k.ny;
        if (z == 0) iz[nz++] = -1;
        if (z == k.nz - 1) iz[nz++] = k.nz;
    }
    if (nx * ny * nz == 1) return;
    for (int c = 0; c < nz; ++c)
        for (int b = 0; b < ny; ++b)
            for (int a = 0; a < nx; ++a) {
                if ((a | b | c) == 0) continue;
                const bool in = BC == LBM_BC_JET && iz[c] < 0 && inlet_inside(k, ix[a], iy[b]);
                stp(PD, pidx(k, ix[a], iy[b], iz[c]), in ? make_float2(1.f, k.rho_r0 - k.rho_b0) : v);
            }
}

__host__ __device__ constexpr double inv_lend(int i)
{
    return csq(i) == 1 ? 1.0 : csq(i) == 2 ? 0.70710678118654752440 : 0.57735026918962576451;
}

// Mass and colour masses of a general state at n.  The mass sum m0 runs in
// FP64 (an exact sum of the stored deviations: mass is conserved up to the
// storage rounding); mk is the mass of the colour the planes Q..2Q-1 hold.
template <class S, int I = 0>
__device__ __forceinline__ void accum_general(const typename S::T* __restrict__ src, const KP& k, uint32_t n,
                                              double& m0, double& mk)
{
    if constexpr (I < Q) {
        m0 += (double)S::dec(ldp(src + (size_t)I * k.NP, n));
        mk += (double)S::dec(ldp(src + (size_t)(Q + I) * k.NP, n));
        accum_general<S, I + 1>(src, k, n, m0, mk);
    }
}

// Mass and minority-colour mass of a shifted state at n, from the pulled
// deviations d and the R of the source nodes in the LDS window.  The colour m
// is the one node n kept in the previous step (its own R, direction 0); its
// mass is written
//   rho_m = x_m(x) rho + sum_{i>=1} [(x_m(x - c_i) - x_m(x)) f_i +- (w_i/|c_i|) c_i . V(x - c_i)],
// an FP64 main term plus FP32 corrections (cf: fractions, cv: recolouring
// vectors, + for red, - for blue) that vanish wherever x_m and V are uniform,
// so pure phases carry no rounding bias.
template <class M, int I = 0>
__device__ __forceinline__ void accum_density_win(const KP& k, const float* d, const float4* __restrict__ win,
                                                  int lx, int ly, M& m0, float& x0, uint32_t& bl, float& cf,
                                                  float& cv)
{
    if constexpr (I < Q) {
        constexpr int cx = kCX[I], cy = kCY[I], cz = kCZ[I];
        const float4 r = win[wslot<DTY>(lx, ly, -cx, -cy, -cz)];
        m0 += (M)d[I];
        if (I == 0) {
            x0 = r.x;
            bl = blue_kept(r.x);
        } else {
            cf += (frac_of(r.x, bl) - x0) * (d[I] + wgt(I) * k.rho_b0);
            cv += (wgt(I) * inv_len(I)) * (cx * r.y + cy * r.z + cz * r.w);
        }
        accum_density_win<M, I + 1>(k, d, win, lx, ly, m0, x0, bl, cf, cv);
    }
}

// Raw moments of the deviations up to second order -- m0, j (3), P (xx, yy,
// zz, xy, xz, yz) -- as 10 planes of N floats at node index nn (z plane + q),
// for the adjoint step; j and P are FP32 sums over opposite pairs.
__device__ __forceinline__ void store_moments(float* __restrict__ MOM, const KP& k, uint32_t nn, float m0,
                                              const float* d)
{
    float jx = 0.f, jy = 0.f, jz = 0.f, pxx = 0.f, pyy = 0.f, pzz = 0.f, pxy = 0.f, pxz = 0.f, pyz = 0.f;
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const float sp = d[i] + d[i + 1], df = d[i] - d[i + 1];
        if (kCX[i]) { jx += kCX[i] * df; pxx += sp; }
        if (kCY[i]) { jy += kCY[i] * df; pyy += sp; }
        if (kCZ[i]) { jz += kCZ[i] * df; pzz += sp; }
        if (kCX[i] * kCY[i]) pxy += (kCX[i] * kCY[i]) * sp;
        if (kCX[i] * kCZ[i]) pxz += (kCX[i] * kCZ[i]) * sp;
        if (kCY[i] * kCZ[i]) pyz += (kCY[i] * kCZ[i]) * sp;
    }
    const float mv[10] = {m0, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz};
    const size_t N = k.N;
#pragma unroll
    for (int a = 0; a < 10; ++a) MOM[(size_t)a * N + nn] = mv[a];
}

// Density pass over the planes of the grid (for the jet all but the outlet
// plane, which k_outlet_density takes: its branch would double this kernel's
// register count and halve its occupancy).  With FP32 storage it also fills
// the field ghost shell; with 16-bit storage k_field_ghosts does (measured:
// the ghost writes cost the shorter 16-bit density pass more than the extra
// launch).
template <class S>
constexpr bool kDensityGhosts = sizeof(typename S::T) == 4;

// Waves per SIMD the density pass is compiled for.  The plain 16-bit forms
// ask for eight (LDS allows four 512-lane blocks per CU): measured 184 -> 177
// us (BF16) and 186 -> 184 us (FP16) on the 128x128x512 jet.  The FP32 and
// referenced forms were slower at eight; a minimum of two leaves their code as
// the compiler chooses for 512-lane blocks.
template <class S>
constexpr int kDensityWaves = (sizeof(typename S::T) == 2 && !S::kEqRef) ? 8 : 2;

// MOMS (the adjoint step from a snapshot): also the raw moments of the pulled
// deviations into MOM.  A compile-time switch: the moment code in the step's
// kernel would raise its registers from 69 to 84 (two blocks per CU instead
// of three), measured 1.85 -> 3.15 ms on the 256x256x1024 jet.
template <int BC, class S, bool MOMS = false>
__global__ __launch_bounds__(DBLOCK) __attribute__((amdgpu_waves_per_eu(kDensityWaves<S>, 8))) void k_density(
    const typename S::T* __restrict__ src, float2* __restrict__ PD, float* __restrict__ XR, KP k,
    float* __restrict__ MOM)
{
    __shared__ float4 win[TileShape<DTY>::W];
    const Tile t = this_tile<DTY>(k);
    const Node& nd = t.nd;
    double m0 = 0.0, mk = 0.0;
    if (k.unshifted) {
        if (!nd.valid) return;
        accum_general<S>(src, k, nd.n, m0, mk);
        const double mo = (double)k.rho_b0 + m0 - mk;
        const bool bl = blue_kept(ldp(k.R, nd.n).x);
        const float2 v = store_fields_sums(PD, XR, k, nd.n, m0, bl ? mo : mk, bl ? mk : mo);
        if constexpr (kDensityGhosts<S>) store_pd_ghosts<BC>(PD, k, nd.x, nd.y, nd.z, v);
        return;
    }
    load_window<DTY, !S::kEqRef>(win, k.R, k, t);
    __syncthreads();
    if (!nd.valid) return;
    float d[Q], unused[Q];
    pull_dirs<S, false, true>(src, k, nd.n, d, unused, unused);
    float x0 = 0.f, cf = 0.f, cv = 0.f;
    uint32_t bl = 0;
    // mass: exact FP64 sum of FP32 deviations; with 16-bit storage an FP32 sum
    // (its rounding is far below the storage rounding, and it is exact in the
    // pure phases, where the deviations vanish)
    using MassT = typename std::conditional<sizeof(typename S::T) == 4, double, float>::type;
    MassT ms = 0;
    accum_density_win(k, d, win, t.lx, t.ly, ms, x0, bl, cf, cv);
    m0 = (double)ms;
    const double rho = (double)k.rho_b0 + m0;
    mk = (double)x0 * rho + (double)(cf + (bl ? -cv : cv));
    const float2 v = store_fields_sums(PD, XR, k, nd.n, m0, bl ? rho - mk : mk, bl ? mk : rho - mk);
    if constexpr (kDensityGhosts<S>) store_pd_ghosts<BC>(PD, k, nd.x, nd.y, nd.z, v);
    if constexpr (MOMS) store_moments(MOM, k, (uint32_t)nd.z * k.plane + nd.q, (float)m0, d);
}

// Jet outlet plane (z = nz - 1): its state by the convective condition,
// recorded in hcur for the collision.  One plane only, so the launch uses
// small blocks (OBLOCK lanes) to spread the latency-bound work over many CUs.
constexpr int OBLOCK = 64;

template <class S>
__global__ __launch_bounds__(OBLOCK) void k_outlet_density(const typename S::T* __restrict__ src,
                                                            float2* __restrict__ PD, float* __restrict__ XR,
                                                            const float* __restrict__ hprev, float* __restrict__ hcur,
                                                            KP k, float* __restrict__ MOM)
{
    const uint32_t q = blockIdx.x * OBLOCK + threadIdx.x;
    if (q >= k.plane) return;
    Node nd;
    nd.z = k.nz - 1;
    nd.y = (int)(((uint64_t)q * k.nx_mul) >> k.nx_sh);
    nd.x = (int)q - nd.y * k.nx;
    nd.q = q;
    nd.valid = true;
    nd.n = pidx(k, nd.x, nd.y, nd.z);
    float d[Q], fr[Q], fb[Q];
    outlet_state<S>(src, k, hprev, nd, d, fr, fb);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        hcur[(size_t)i * k.plane + nd.q] = d[i];
        hcur[(size_t)(Q + i) * k.plane + nd.q] = fr[i];
    }
    const float2 v = store_fields(PD, XR, k, nd.n, d, fr);
    if constexpr (kDensityGhosts<S>) store_pd_ghosts<LBM_BC_JET>(PD, k, nd.x, nd.y, nd.z, v);
    if (MOM) store_moments(MOM, k, (uint32_t)nd.z * k.plane + nd.q, v.y, d);
}


// ---------------------------------------------------------------- ghost shell
// Ghost cell g of the shell: z faces (all x, y incl. ghosts), then y faces
// (z interior), then x faces (y, z interior).
struct Ghost {
    int x, y, z;
    bool valid;
};

__device__ __forceinline__ Ghost shell_cell(const KP& k, uint32_t g)
{
    Ghost c;
    const uint32_t A = (uint32_t)k.px * k.py, B = (uint32_t)k.px * k.nz, C = (uint32_t)k.ny * k.nz;
    c.valid = true;
    if (g < 2 * A) {
        const uint32_t f = g / A, r = g - f * A;
        c.x = (int)(r % k.px) - 1;
        c.y = (int)(r / k.px) - 1;
        c.z = f ? k.nz : -1;
    } else if (g < 2 * A + 2 * B) {
        const uint32_t h = g - 2 * A, f = h / B, r = h - f * B;
        c.x = (int)(r % k.px) - 1;
        c.z = (int)(r / k.px);
        c.y = f ? k.ny : -1;
    } else if (g < 2 * A + 2 * B + 2 * C) {
        const uint32_t h = g - 2 * A - 2 * B, f = h / C, r = h - f * C;
        c.y = (int)(r % k.ny);
        c.z = (int)(r / k.ny);
        c.x = f ? k.nx : -1;
    } else {
        c.valid = false;
        c.x = c.y = c.z = 0;
    }
    return c;
}

__device__ __forceinline__ int wrapc(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }
__device__ __forceinline__ int clampc(int a, int n) { return a < 0 ? 0 : (a >= n ? n - 1 : a); }

// (phi, rho - rho_b0) in the shell: periodic copies, or (jet) mirrored copies
// across the half-way walls and the outlet, and (1, rho_r0 - rho_b0) in the
// inlet circle at z = -1.
template <int BC>
__global__ __launch_bounds__(BLOCK) void k_field_ghosts(float2* __restrict__ PD, KP k, uint32_t ncells)
{
    const uint32_t g = blockIdx.x * BLOCK + threadIdx.x;
    if (g >= ncells) return;
    const Ghost c = shell_cell(k, g);
    if (!c.valid) return;
    const uint32_t dst = pidx(k, c.x, c.y, c.z);
    if (BC == LBM_BC_PERIODIC) {
        PD[dst] = PD[pidx(k, wrapc(c.x, k.nx), wrapc(c.y, k.ny), wrapc(c.z, k.nz))];
        return;
    }
    if (c.z < 0 && inlet_inside(k, c.x, c.y)) {
        PD[dst] = make_float2(1.f, k.rho_r0 - k.rho_b0);
        return;
    }
    PD[dst] = PD[pidx(k, clampc(c.x, k.nx), clampc(c.y, k.ny), clampc(c.z, k.nz))];
}

// Populations and R in the shell cells the fused kernel does not write: every
// shell cell except x-face cells with y and z interior.  A ghost cell g feeds
// direction I of an interior node iff c_I points into the domain along every
// axis on which g lies outside.  Periodic: copy of the wrapped node.  Jet:
// specular reflection, the populations of the clamped node with the outside
// components of c_I reversed and V mirrored alike; inside the inlet circle at
// z = -1 the red inlet equilibrium (d = f^e - w rho_b0, pure red R).
//
// The side of the cell on each axis (0 inside, 1 below, 2 above) selects one of
// 26 compile-time variants, so the directions a cell feeds and their mirror
// images are constants; all loads are issued before the first store (the
// compiler cannot reorder loads past stores to the same array).
template <int SX, int SY, int SZ, int I>
__host__ __device__ constexpr bool ghost_feeds()
{
    return (SX == 0 || (SX == 1 ? kCX[I] > 0 : kCX[I] < 0)) && (SY == 0 || (SY == 1 ? kCY[I] > 0 : kCY[I] < 0)) &&
           (SZ == 0 || (SZ == 1 ? kCZ[I] > 0 : kCZ[I] < 0));
}

template <int BC, class S, int SX, int SY, int SZ, int I = 0>
__device__ __forceinline__ void ghost_gather(const typename S::T* __restrict__ dst, const KP& k, const Ghost& c,
                                             uint32_t wi, bool inlet, typename S::T* v)
{
    if constexpr (I < Q) {
        if constexpr (ghost_feeds<SX, SY, SZ, I>()) {
            constexpr int m = (SX ? 1 : 0) | (SY ? 2 : 0) | (SZ ? 4 : 0);
            constexpr int J = BC == LBM_BC_PERIODIC ? I : mirror_dir(I, m);
            if constexpr (BC == LBM_BC_JET && SZ == 1 && SX == 0 && SY == 0) {
                if (inlet) {
                    v[I] = S::enc(inlet_feq_dir<I>(k, c.x, c.y, k.t) - wgt(I) * k.rho_b0);
                } else {
                    v[I] = ldp(dst + (size_t)J * k.NP, wi);
                }
            } else {
                v[I] = ldp(dst + (size_t)J * k.NP, wi);
            }
        }
        ghost_gather<BC, S, SX, SY, SZ, I + 1>(dst, k, c, wi, inlet, v);
    }
}

template <class S, int SX, int SY, int SZ, int I = 0>
__device__ __forceinline__ void ghost_scatter(typename S::T* __restrict__ dst, const KP& k, uint32_t gi,
                                              const typename S::T* v)
{
    if constexpr (I < Q) {
        if constexpr (ghost_feeds<SX, SY, SZ, I>()) stp(dst + (size_t)I * k.NP, gi, v[I]);
        ghost_scatter<S, SX, SY, SZ, I + 1>(dst, k, gi, v);
    }
}

template <int BC, class S, int SX, int SY, int SZ>
__device__ __forceinline__ void ghost_fill(typename S::T* __restrict__ dst, const KP& k, const Ghost& c,
                                          uint32_t gi, uint32_t wi, bool inlet)
{
    typename S::T v[Q];
    ghost_gather<BC, S, SX, SY, SZ>(dst, k, c, wi, inlet, v);
    ghost_scatter<S, SX, SY, SZ>(dst, k, gi, v);
}

template <int BC, class S>
__device__ __forceinline__ void ghost_dirs(typename S::T* __restrict__ dst, const KP& k, const Ghost& c,
                                           uint32_t gi, uint32_t wi, bool inlet)
{
    const int sx = c.x < 0 ? 1 : (c.x >= k.nx ? 2 : 0);
    const int sy = c.y < 0 ? 1 : (c.y >= k.ny ? 2 : 0);
    const int sz = c.z < 0 ? 1 : (c.z >= k.nz ? 2 : 0);
    switch (sx * 9 + sy * 3 + sz) {
#define CGLBM_GHOST_CASE(X, Y, Z) \
    case X * 9 + Y * 3 + Z: ghost_fill<BC, S, X, Y, Z>(dst, k, c, gi, wi, inlet); break;
        CGLBM_GHOST_CASE(0, 0, 1) CGLBM_GHOST_CASE(0, 0, 2) CGLBM_GHOST_CASE(0, 1, 0) CGLBM_GHOST_CASE(0, 1, 1)
        CGLBM_GHOST_CASE(0, 1, 2) CGLBM_GHOST_CASE(0, 2, 0) CGLBM_GHOST_CASE(0, 2, 1) CGLBM_GHOST_CASE(0, 2, 2)
        CGLBM_GHOST_CASE(1, 0, 0) CGLBM_GHOST_CASE(1, 0, 1) CGLBM_GHOST_CASE(1, 0, 2) CGLBM_GHOST_CASE(1, 1, 0)
        CGLBM_GHOST_CASE(1, 1, 1) CGLBM_GHOST_CASE(1, 1, 2) CGLBM_GHOST_CASE(1, 2, 0) CGLBM_GHOST_CASE(1, 2, 1)
        CGLBM_GHOST_CASE(1, 2, 2) CGLBM_GHOST_CASE(2, 0, 0) CGLBM_GHOST_CASE(2, 0, 1) CGLBM_GHOST_CASE(2, 0, 2)
        CGLBM_GHOST_CASE(2, 1, 0) CGLBM_GHOST_CASE(2, 1, 1) CGLBM_GHOST_CASE(2, 1, 2) CGLBM_GHOST_CASE(2, 2, 0)
        CGLBM_GHOST_CASE(2, 2, 1) CGLBM_GHOST_CASE(2, 2, 2)
#undef CGLBM_GHOST_CASE
    default: break;
    }
}

// The population ghosts launch with one wave per block: few shell cells do
// work (most x-face cells are the fused kernel's), and small blocks spread
// those over more CUs (measured: 3.5 us less per step on the 128x128x512 jet).
constexpr int GBLOCK = 64;

template <int BC, class S>
__global__ __launch_bounds__(GBLOCK) void k_pop_ghosts(typename S::T* __restrict__ dst, float4* __restrict__ Rout,
                                                        uint4* __restrict__ Qout, KP k, uint32_t ncells)
{
    const uint32_t g = blockIdx.x * GBLOCK + threadIdx.x;
    if (g >= ncells) return;
    const Ghost c = shell_cell(k, g);
    if (!c.valid) return;
    // x-face cells of interior rows: written by the fused kernel
    if ((c.x < 0 || c.x >= k.nx) && c.y >= 1 && c.y <= k.ny - 2 && c.z >= 1 && c.z <= k.nz - 2) return;
    if (BC == LBM_BC_JET && c.z >= k.nz) return;  // the outlet plane is never pulled across
    const uint32_t gi = pidx(k, c.x, c.y, c.z);
    if (BC == LBM_BC_PERIODIC) {
        const uint32_t wi = pidx(k, wrapc(c.x, k.nx), wrapc(c.y, k.ny), wrapc(c.z, k.nz));
        ghost_dirs<BC, S>(dst, k, c, gi, wi, false);
        Rout[gi] = Rout[wi];
        if (S::kEqRef) Qout[gi] = Qout[wi];
        return;
    }
    const bool inlet = c.z < 0 && inlet_inside(k, c.x, c.y);
    const int m = ((c.x < 0 || c.x >= k.nx) ? 1 : 0) | ((c.y < 0 || c.y >= k.ny) ? 2 : 0) | (c.z < 0 ? 4 : 0);
    const uint32_t wi = pidx(k, clampc(c.x, k.nx), clampc(c.y, k.ny), clampc(c.z, k.nz));
    ghost_dirs<BC, S>(dst, k, c, gi, wi, inlet);
    if (inlet) {
        Rout[gi] = make_float4(frac_tag(0.0, 1u), 0.f, 0.f, 0.f);  // pure red: x_b = 0
        if (S::kEqRef) Qout[gi] = make_uint4(0u, 0u, 0u, 0u);  // zero record: the stored value is the deviation
    } else {
        const float4 r = Rout[wi];
        Rout[gi] = make_float4(r.x, (m & 1) ? -r.y : r.y, (m & 2) ? -r.z : r.z, (m & 4) ? -r.w : r.w);
        if (S::kEqRef) Qout[gi] = mirror_ref(Qout[wi], m);
    }
}

// ---------------------------------------------------------------- stencil
// isotropic gradients 3 sum_i w_i chi(x + c_i) c_i of phi and rho - rho_b0,
// accumulated over opposite pairs (i, i + 1) in FP64: g = (dphi[3], drho[3])
template <int I = 1>
__device__ __forceinline__ void gradients(const float2* __restrict__ pd, const KP& k, uint32_t n, double (&g)[6])
{
    if constexpr (I < Q) {
        constexpr int cx = kCX[I], cy = kCY[I], cz = kCZ[I];
        const int o = doff(k, cx, cy, cz);
        const float2 a = ldp(pd, n + (uint32_t)o);
        const float2 b = ldp(pd, n - (uint32_t)o);
        const double dp = (double)a.x - (double)b.x, dr = (double)a.y - (double)b.y;
        constexpr double w3 = 3.0 * wgtd(I);
        if (cx) { g[0] += (w3 * cx) * dp; g[3] += (w3 * cx) * dr; }
        if (cy) { g[1] += (w3 * cy) * dp; g[4] += (w3 * cy) * dr; }
        if (cz) { g[2] += (w3 * cz) * dp; g[5] += (w3 * cz) * dr; }
        gradients<I + 2>(pd, k, n, g);
    }
}

// the same gradients in FP32: each pair difference chi(x + c_i) - chi(x - c_i)
// is exact for nearly equal values, the weighted sum of 13 of them is well
// conditioned.  g = (dphi[3], drho[3])
template <int I = 1>
__device__ __forceinline__ void gradients_f(const float2* __restrict__ pd, const KP& k, uint32_t n, float (&g)[6])
{
    if constexpr (I < Q) {
        constexpr int cx = kCX[I], cy = kCY[I], cz = kCZ[I];
        const int o = doff(k, cx, cy, cz);
        const float2 a = ldp(pd, n + (uint32_t)o);
        const float2 b = ldp(pd, n - (uint32_t)o);
        const float dp = a.x - b.x, dr = a.y - b.y;
        constexpr float w3 = 3.0f * wgt(I);
        if (cx) { g[0] += (w3 * cx) * dp; g[3] += (w3 * cx) * dr; }
        if (cy) { g[1] += (w3 * cy) * dp; g[4] += (w3 * cy) * dr; }
        if (cz) { g[2] += (w3 * cz) * dp; g[5] += (w3 * cz) * dr; }
        gradients_f<I + 2>(pd, k, n, g);
    }
}

// the same FP32 gradients from the LDS window of the (phi, rho) fields
template <int I = 1>
__device__ __forceinline__ void gradients_win(const float2* __restrict__ win, int lx, int ly, float (&g)[6])
{
    if constexpr (I < Q) {
        constexpr int cx = kCX[I], cy = kCY[I], cz = kCZ[I];
        const float2 a = win[wslot(lx, ly, cx, cy, cz)];
        const float2 b = win[wslot(lx, ly, -cx, -cy, -cz)];
        const float dp = a.x - b.x, dr = a.y - b.y;
        constexpr float w3 = 3.0f * wgt(I);
        if (cx) { g[0] += (w3 * cx) * dp; g[3] += (w3 * cx) * dr; }
        if (cy) { g[1] += (w3 * cy) * dp; g[4] += (w3 * cy) * dr; }
        if (cz) { g[2] += (w3 * cz) * dp; g[5] += (w3 * cz) * dr; }
        gradients_win<I + 2>(win, lx, ly, g);
    }
}

// ---------------------------------------------------------------- ghost writes of the fused kernel
// A post-collision population J of a boundary node W that would stream out of
// the lattice is what some interior node pulls from a ghost cell.  Periodic:
// the ghost on the opposite side, same direction.  Jet: the ghost W + c_J in the
// plane of J reversed along the wall normal (specular reflection, free slip).
// The fused kernel writes the ghosts of x-wall nodes whose y and z are
// interior (one lane per wavefront, strided cells); k_pop_ghosts fills the
// rest of the shell afterwards.
// the common case: the node lies on an x wall only (y and z interior)
template <int BC, class S, int J>
__device__ __forceinline__ void ghost_pop_x(const KP& k, const Node& nd, typename S::T* __restrict__ dst, float v,
                                            bool xl, bool xh)
{
    constexpr int cx = kCX[J];
    if constexpr (cx != 0) {
        if (cx < 0 ? xl : xh) {
            if (BC == LBM_BC_PERIODIC)
                stp(dst + (size_t)J * k.NP, nd.n - (uint32_t)(cx * k.nx), S::enc(v));
            else
                stp(dst + (size_t)mirror_dir(J, 1) * k.NP, nd.n + (uint32_t)cx, S::enc(v));
        }
    }
}

// R = (x*, V) of the x-wall ghost cell this node feeds: a copy
// (periodic) or with V_x reversed (free slip)
template <int BC>
__device__ __forceinline__ void ghost_R_x(const KP& k, const Node& nd, float4* __restrict__ Rout, float4 r, bool xl,
                                          bool xh)
{
    if (BC == LBM_BC_PERIODIC) {
        if (xh) st_rec(Rout, k, nd.z, nd.n - (uint32_t)k.nx, r);
        if (xl) st_rec(Rout, k, nd.z, nd.n + (uint32_t)k.nx, r);
    } else {
        const float4 m = make_float4(r.x, -r.y, r.z, r.w);
        if (xl) st_rec(Rout, k, nd.z, nd.n - 1u, m);
        if (xh) st_rec(Rout, k, nd.z, nd.n + 1u, m);
    }
}

// the reference record of the same x-wall ghost cell
template <int BC>
__device__ __forceinline__ void ghost_Q_x(const KP& k, const Node& nd, uint4* __restrict__ Qout, uint4 q, bool xl,
                                          bool xh)
{
    if (BC == LBM_BC_PERIODIC) {
        if (xh) st_rec(Qout, k, nd.z, nd.n - (uint32_t)k.nx, q);
        if (xl) st_rec(Qout, k, nd.z, nd.n + (uint32_t)k.nx, q);
    } else {
        const uint4 m = mirror_ref(q, 1);
        if (xl) st_rec(Qout, k, nd.z, nd.n - 1u, m);
        if (xh) st_rec(Qout, k, nd.z, nd.n + 1u, m);
    }
}

template <int BC, class S, int I>
__device__ __forceinline__ void ghost_pair_t(const KP& k, const Node& nd, typename S::T* __restrict__ dst, float vp,
                                             float vm, bool xl, bool xh, bool yz_edge)
{
    if (!yz_edge) {
        ghost_pop_x<BC, S, I>(k, nd, dst, vp, xl, xh);
        ghost_pop_x<BC, S, I + 1>(k, nd, dst, vm, xl, xh);
    }
}

// The x-wall ghost slots that no pull reads (directions that do not point back
// into the lattice) are written too, with zero, so that every cache line of a
// population plane is written whole: a partly written line costs the memory a
// read-modify-write.  A probe of the fused kernel's access pattern on the
// 256x256x1024 lattice: 3.40 ms with the unread slots left alone, 3.16 ms
// with every slot of the row written.
template <class S, int J = 0>
__device__ __forceinline__ void ghost_zero_x(const KP& k, uint32_t n, typename S::T* __restrict__ dst, bool xl,
                                             bool xh)
{
    if constexpr (J < Q) {
        constexpr int cx = kCX[J];
        if (cx <= 0 && xl) stp(dst + (size_t)J * k.NP, n - 1u, S::enc(0.f));
        if (cx >= 0 && xh) stp(dst + (size_t)J * k.NP, n + 1u, S::enc(0.f));
        ghost_zero_x<S, J + 1>(k, n, dst, xl, xh);
    }
}

#define CGLBM_GP(I) \
    case I: ghost_pair_t<BC, S, I>(k, nd, dst, vp, vm, xl, xh, yz_edge); break;
// dispatch on the (unrolled, constant) pair index
template <int BC, class S>
__device__ __forceinline__ void ghost_pair(int i, const KP& k, const Node& nd, typename S::T* __restrict__ dst,
                                           float vp, float vm, bool xl, bool xh, bool yz_edge)
{
    switch (i) {
        CGLBM_GP(1) CGLBM_GP(3) CGLBM_GP(5) CGLBM_GP(7) CGLBM_GP(9) CGLBM_GP(11) CGLBM_GP(13)
        CGLBM_GP(15) CGLBM_GP(17) CGLBM_GP(19) CGLBM_GP(21) CGLBM_GP(23) CGLBM_GP(25)
    default: break;
    }
}
#undef CGLBM_GP

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
// colour-blind deviations d, the centre values phic and xk (the tagged
// minority-colour fraction) and the gradients; writes the 27 post-collision
// colour-blind deviations to dst and (xk, V) of the recolouring to Rout at n.  FP64 only where a
// sum must be exact or an O(1) cancellation happens: the mass m0 and the
// equilibrium offsets E0, E1 (zero in the pure phases).  The momentum and the
// second moments are FP32 sums over opposite pairs (pair differences are exact
// for nearly equal populations, so the momentum of a fluid at rest is exactly
// zero).
template <int BC, class S>
__device__ __forceinline__ void collide_store(const KP& k, const Node& nd, const float* d, float phic, float xk,
                                              const float (&g)[6], typename S::T* __restrict__ dst,
                                              float4* __restrict__ Rout, uint4* __restrict__ Qout)
{
    const size_t N = k.NP;
    const uint32_t n = nd.n;
    // Scalar precision: FP64 for the mass sum and the equilibrium offsets with
    // FP32 storage (exact mass, no rounding bias in the pure phases at the
    // 1e-5 parity level); FP32 with 16-bit storage, whose own rounding is four
    // orders larger (the sum of 27 16-bit values is exact in FP32 but for the
    // widest exponent spreads).  Saves about 70 of the 16-bit kernels' 1 070
    // VALU instructions per wave.
    using H = typename std::conditional<sizeof(typename S::T) == 4, double, float>::type;
    // raw moments of d up to second order
    H m0s = (H)d[0];
    float jx = 0.f, jy = 0.f, jz = 0.f;
    float pxx = 0.f, pyy = 0.f, pzz = 0.f, pxy = 0.f, pxz = 0.f, pyz = 0.f;
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        m0s += (H)d[i] + (H)d[i + 1];
        const float sp = d[i] + d[i + 1], df = d[i] - d[i + 1];
        if (kCX[i]) { jx += kCX[i] * df; pxx += sp; }
        if (kCY[i]) { jy += kCY[i] * df; pyy += sp; }
        if (kCZ[i]) { jz += kCZ[i] * df; pzz += sp; }
        if (kCX[i] * kCY[i]) pxy += (kCX[i] * kCY[i]) * sp;
        if (kCX[i] * kCZ[i]) pxz += (kCX[i] * kCZ[i]) * sp;
        if (kCY[i] * kCZ[i]) pyz += (kCY[i] * kCZ[i]) * sp;
    }
    const H m0d = m0s;
    const float m0 = (float)m0d;
    const float rhof = (float)((H)k.rho_b0 + m0d);
    // hardware reciprocals (1 ulp): the node quantities need no correctly
    // rounded division, and each IEEE division costs about ten instructions
    const float inv_rho = __builtin_amdgcn_rcpf(rhof);
    // interpolated properties (Sec. II): alpha_bar, harmonic nu_bar, s2nu
    const float hpf = 0.5f * (1.f + phic), hmf = 0.5f * (1.f - phic);
    const float nubf = __builtin_amdgcn_rcpf(hpf * k.inv_nu_r + hmf * k.inv_nu_b);
    const float s2 = __builtin_amdgcn_rcpf(3.f * nubf + 0.5f);
    const H hp = (H)0.5 * ((H)1 + (H)phic);
    const H abar = (H)k.alpha_b + hp * (H)k.dalpha;
    const H kap = (H)(27.0 / 19.0) * ((H)1 - abar);
    // equilibrium offsets in deviation form: E0 = rho abar - w_0 rho_b0, E1 = rho kappa - rho_b0
    const H E0 = (H)k.rho_b0 * (hp * (H)k.dalpha + (H)k.a_minus_w0) + m0d * abar;
    const H E1 = (H)k.rho_b0 * (-(H)(27.0 / 19.0) * hp * (H)k.dalpha + (H)k.kappa_b_m1) + m0d * kap;
    // body force (Eq. bodyForceJet) and velocity with the half-force term (Eq. Momentum)
    const float Fxf = m0 * k.gx, Fyf = m0 * k.gy, Fzf = m0 * k.gz;
    const float uxf = (jx + 0.5f * Fxf) * inv_rho, uyf = (jy + 0.5f * Fyf) * inv_rho, uzf = (jz + 0.5f * Fzf) * inv_rho;
    const float grxf = g[3], gryf = g[4], grzf = g[5];
    // second moments of f - f^(e) + F'/2 (its zeroth and first moments vanish, so
    // these are its central moments): sum f^(e) c_a c_b = iso + rho u_a u_b +
    // nu_bar (u_a dr_b + dr_a u_b); sum F' c_a c_b = u_a F_b + u_b F_a
    const float cxy = pxy - rhof * uxf * uyf - nubf * (uxf * gryf + grxf * uyf) + 0.5f * (uxf * Fyf + uyf * Fxf);
    const float cxz = pxz - rhof * uxf * uzf - nubf * (uxf * grzf + grxf * uzf) + 0.5f * (uxf * Fzf + uzf * Fxf);
    const float cyz = pyz - rhof * uyf * uzf - nubf * (uyf * grzf + gryf * uzf) + 0.5f * (uyf * Fzf + uzf * Fyf);
    const float cxx = pxx - rhof * uxf * uxf - 2.f * nubf * uxf * grxf + uxf * Fxf;
    const float cyy = pyy - rhof * uyf * uyf - 2.f * nubf * uyf * gryf + uyf * Fyf;
    const float czz = pzz - rhof * uzf * uzf - 2.f * nubf * uzf * grzf + uzf * Fzf;
    const float tr3 = (cxx + cyy + czz) * (1.f / 3.f);
    const float om = 1.f - s2;
    // relaxed deviatoric central moments, scaled by (1 - s2nu)
    const float kxy = om * cxy, kxz = om * cxz, kyz = om * cyz;
    const float kxx = om * (cxx - tr3), kyy = om * (cyy - tr3), kzz = om * (czz - tr3);
    const float u2 = uxf * uxf + uyf * uyf + uzf * uzf;
    const float udr = uxf * grxf + uyf * gryf + uzf * grzf;
    const float uF = uxf * Fxf + uyf * Fyf + uzf * Fzf;

    // FP32 per-direction part
    const float E1f = (float)E1;
    const float gpx = g[0], gpy = g[1], gpz = g[2];
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
    const float inv_gn = on ? __builtin_amdgcn_rsqf(G2) : 0.f;
    const float gn = G2 * inv_gn;
    const float Agn = k.A * gn, Aign = k.A * inv_gn;
    // recolouring vector V = beta (rho_r rho_b / rho) kappa n (x_r x_b = xk (1 - xk))
    const float rec = k.beta * xk * (1.f - xk) * rhof * (float)kap * inv_gn;
    const float4 rv = make_float4(xk, rec * gpx, rec * gpy, rec * gpz);
    st_rec(Rout, k, nd.z, n, rv);
    const float nub9 = 9.f * nubf;
    const bool xl = nd.x == 0, xh = nd.x == k.nx - 1;
    const bool yz_edge = nd.y == 0 || nd.y == k.ny - 1 || nd.z == 0 || nd.z == k.nz - 1;
    if (!yz_edge) ghost_R_x<BC>(k, nd, Rout, rv, xl, xh);
    // referenced 16-bit storage: reference record of this node, rounded as stored
    float rt = 0.f, uxt = 0.f, uyt = 0.f, uzt = 0.f, et = 0.f;
    if constexpr (S::kEqRef) {
        const uint4 qr = enc_ref<S>(rhof, uxf, uyf, uzf, (float)E1);
        st_rec(Qout, k, nd.z, n, qr);
        if (!yz_edge) ghost_Q_x<BC>(k, nd, Qout, qr, xl, xh);
        const RefRec r = dec_ref<S>(qr);
        rt = r.rho;
        uxt = r.ux;
        uyt = r.uy;
        uzt = r.uz;
        et = r.e;
    }
    const float u2t = uxt * uxt + uyt * uyt + uzt * uzt;

    // rest population
    {
        const float w = wgt(0);
        const float de = (float)E0 - 1.5f * w * rhof * u2 - 3.f * nubf * udr;
        const float Fp = -3.f * w * uF;
        const float pert = on ? k.A * (10.f / 27.f) * gn : 0.f;
        const float delta = U0[1][1] * bx.h0[1] + U1[1][1] * bx.h1[1] + U2[1][1] * h2(0);
        const float dd = de + 0.5f * Fp + delta + pert;
        if constexpr (S::kEqRef) {
            const uint32_t b = __float_as_uint(dd);
            stpl(dst, k.NP, n, __builtin_bit_cast(typename S::T, (uint16_t)(b >> 16)));
            stpl(dst + (size_t)Q * N, k.NP, n, __builtin_bit_cast(typename S::T, (uint16_t)(b & 0xffffu)));
        } else {
            stpl(dst, k.NP, n, S::enc(dd));
        }
    }
    // opposite pairs (i, i + 1): shared even parts, odd parts change sign.
    // Per direction (w_i factored out; cu = c.u, cr = c.grad rho, cF = c.F,
    // cg = c.grad phi):
    //   even = f^(e) even part + F'/2 even part + perturbation
    //        = K0 + cu (4.5 rho cu + 9 nu cr + 4.5 cF) + A/|g| cg^2,
    //          K0 = E1 - 1.5 rho u^2 - 1.5 u.F - A |g|,
    //   odd  = cu (K1 + 4.5 rho cu^2) + 1.5 cF,  K1 = rho (3 - 4.5 u^2)
    const float K0 = E1f - 1.5f * rhof * u2 - 1.5f * uF - Agn;
    const float K1 = rhof * (3.f - 4.5f * u2);
    const float r45 = 4.5f * rhof;
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const int cx = kCX[i], cy = kCY[i], cz = kCZ[i];
        const float w = wgt(i);
        const float cu = cx * uxf + cy * uyf + cz * uzf;
        const float cr = cx * grxf + cy * gryf + cz * grzf;
        const float cF = cx * Fxf + cy * Fyf + cz * Fzf;
        const float cg = cx * gpx + cy * gpy + cz * gpz;
        const float t = r45 * cu + (nub9 * cr + 4.5f * cF);
        const float even = w * (K0 + cu * t + (Aign * cg) * cg);
        const float odd = w * (cu * (K1 + r45 * (cu * cu)) + 1.5f * cF);
        // direction i (+c) and i + 1 (-c)
        const float dl_p = U0[cy + 1][cz + 1] * bx.h0[cx + 1] + U1[cy + 1][cz + 1] * bx.h1[cx + 1]
                           + U2[cy + 1][cz + 1] * h2(cx);
        const float dl_m = U0[1 - cy][1 - cz] * bx.h0[1 - cx] + U1[1 - cy][1 - cz] * bx.h1[1 - cx]
                           + U2[1 - cy][1 - cz] * h2(-cx);
        float dp = even + odd + dl_p;
        float dm = even - odd + dl_m;
        if constexpr (S::kEqRef) {
            // remove the reference's velocity part (even and odd in c)
            const float cut = cx * uxt + cy * uyt + cz * uzt;
            const float re = w * (et + rt * (4.5f * cut * cut - 1.5f * u2t));
            const float ro = w * rt * cut * (3.f + 4.5f * cut * cut - 4.5f * u2t);
            dp -= re + ro;
            dm -= re - ro;
        }
        stpl(dst + (size_t)i * N, k.NP, n, S::enc(dp));
        stpl(dst + (size_t)(i + 1) * N, k.NP, n, S::enc(dm));
        ghost_pair<BC, S>(i, k, nd, dst, dp, dm, xl, xh, yz_edge);
    }
    if (!yz_edge && (xl || xh)) ghost_zero_x<S>(k, n, dst, xl, xh);
}


// ---------------------------------------------------------------- fused collide-recolour-stream
// waves per SIMD, measured on MI355X: four (at most 128 VGPRs) in FP32 and
// the referenced forms, 7 % faster than three in FP32 (five spill there);
// five for plain BF16 and FP16 (96 VGPRs, no spill), up to 9 % faster than
// four.  Jet: the outlet plane's pre-collision state is the one the density
// pass recorded.
template <class S>
constexpr int kCollideWaves = (sizeof(typename S::T) == 2 && !S::kEqRef) ? 5 : 4;

template <int BC, class S>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kCollideWaves<S>, kCollideWaves<S>))) void
k_collide(
    const typename S::T* __restrict__ src, typename S::T* __restrict__ dst, const float2* __restrict__ PD,
    const float* __restrict__ XR, const float* __restrict__ hcur, float4* __restrict__ Rout, uint4* __restrict__ Qout,
    KP k)
{
    // the (phi, rho) stencil from an LDS window (measured faster than through
    // the caches, for the 16-bit forms too at their present occupancy)
    constexpr bool kWin = true;
    __shared__ float2 win[kWin ? SW : 1];
    const Tile t = this_tile(k);
    const Node& nd = t.nd;
    if constexpr (kWin) {
        load_window<STY, true>(win, PD, k, t);
        __syncthreads();
    }
    if (!nd.valid) return;
    float d[Q];
    if (BC == LBM_BC_JET && t.z == k.nz - 1) {
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = hcur[(size_t)i * k.plane + nd.q];
    } else {
        float unused[Q];
        pull_all<S, false>(src, k, nd.n, d, unused, unused);
    }
    const float xk = ldp(XR, nd.n);
    float g[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float phic;
    if constexpr (kWin) {
        phic = win[wslot(t.lx, t.ly, 0, 0, 0)].x;
        gradients_win(win, t.lx, t.ly, g);
    } else {
        phic = ldp(PD, nd.n).x;
        gradients_f(PD, k, nd.n, g);
    }
    collide_store<BC, S>(k, nd, d, phic, xk, g, dst, Rout, Qout);
}


// ---------------------------------------------------------------- state in and out
// Initial state (general form): per-colour equilibria f^k_i = rho_k {varphi_i(alpha_k)
// + w_i [velocity terms of Eq. EES]} of the droplet / jet preset or of caller
// fields (node order), evaluated in FP64 and rounded once to the storage format.
template <class S>
__global__ __launch_bounds__(BLOCK) void k_init(typename S::T* __restrict__ dst, float4* __restrict__ Rw, KP k,
                                                 int kind,
                                                 const float* __restrict__ frr, const float* __restrict__ frb,
                                                 const float* __restrict__ fu, double dcx, double dcy, double dcz,
                                                 double R, double W, double rho_r0, double rho_b0, double alpha_r,
                                                 double alpha_b, double rho_ref)
{
    const Node nd = this_node(k);
    if (!nd.valid) return;
    const size_t NP = k.NP;
    const uint32_t u_idx = (uint32_t)nd.z * k.plane + nd.q;
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
        rr = frr[u_idx];
        rb = frb[u_idx];
        if (fu) {
            ux = fu[3 * (size_t)u_idx];
            uy = fu[3 * (size_t)u_idx + 1];
            uz = fu[3 * (size_t)u_idx + 2];
        }
    }
    const double u2 = ux * ux + uy * uy + uz * uz;
    const double kap_r = 27.0 * (1.0 - alpha_r) / 19.0, kap_b = 27.0 * (1.0 - alpha_b) / 19.0;
    const uint32_t bl = rr > rb;  // planes Q..2Q-1 keep the minority colour
    stp(Rw, nd.n, make_float4(frac_tag(0.0, bl), 0.f, 0.f, 0.f));
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double w = wgtd(i);
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
        const double dv = (fv + fb) - w * rho_ref;  // deviation from the kernels' reference density
        stp(dst + (size_t)i * NP, nd.n, S::enc((float)dv));
        stp(dst + (size_t)(Q + i) * NP, nd.n, S::enc((float)(bl ? fb : fv)));
    }
}

// set an explicit (fr, fb) FP32 state (node order), general form: d formed in
// FP64 and rounded once, and the populations of the node's minority colour
// (flagged in Rw)
template <class S>
__global__ __launch_bounds__(BLOCK) void k_set_state(typename S::T* __restrict__ dst, float4* __restrict__ Rw, KP k,
                                                      const float* __restrict__ st, double rho_b0)
{
    const Node nd = this_node(k);
    if (!nd.valid) return;
    const size_t NP = k.NP, N = k.N;
    const uint32_t u_idx = (uint32_t)nd.z * k.plane + nd.q;
    double rr = 0.0, rb = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        rr += (double)st[(size_t)i * N + u_idx];
        rb += (double)st[(size_t)(Q + i) * N + u_idx];
    }
    const uint32_t bl = rr > rb;
    stp(Rw, nd.n, make_float4(frac_tag(0.0, bl), 0.f, 0.f, 0.f));
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float fr = st[(size_t)i * N + u_idx], fb = st[(size_t)(Q + i) * N + u_idx];
        const double dv = ((double)fr + (double)fb) - wgtd(i) * rho_b0;
        stp(dst + (size_t)i * NP, nd.n, S::enc((float)dv));
        stp(dst + (size_t)(Q + i) * NP, nd.n, S::enc(bl ? fb : fr));
    }
}

// current state as (fr, fb) FP32 in node order
template <int BC, class S>
__global__ __launch_bounds__(BLOCK) void k_get_state(const typename S::T* __restrict__ src,
                                                      const float* __restrict__ hprev, KP k, float* __restrict__ st,
                                                      double rho_b0)
{
    const Node nd = this_node(k);
    if (!nd.valid) return;
    const size_t N = k.N;
    const uint32_t u_idx = (uint32_t)nd.z * k.plane + nd.q;
    float d[Q], fr[Q], fb[Q];
    read_state<BC, S>(src, k, hprev, nd, d, fr, fb);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        st[(size_t)i * N + u_idx] = fr[i];
        st[(size_t)(Q + i) * N + u_idx] = fb[i];
    }
}

// macroscopic fields (node order) and FP64 audit partial sums (one slot per block)
template <int BC, class S>
__global__ __launch_bounds__(BLOCK) void k_macro(const typename S::T* __restrict__ src,
                                                  const float* __restrict__ hprev, KP k, float* __restrict__ o_rr,
                                                  float* __restrict__ o_rb, float* __restrict__ o_u,
                                                  float* __restrict__ o_phi, double* __restrict__ partials)
{
    const Node nd = this_node(k);
    double acc[5] = {0, 0, 0, 0, 0};
    if (nd.valid) {
        float d[Q], fr[Q], fb[Q];
        read_state<BC, S>(src, k, hprev, nd, d, fr, fb);
        double m0 = 0.0, rr = 0.0, rb = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            m0 += (double)d[i];
            rr += (double)fr[i];
            rb += (double)fb[i];
            if (kCX[i]) jx += kCX[i] * (double)d[i];
            if (kCY[i]) jy += kCY[i] * (double)d[i];
            if (kCZ[i]) jz += kCZ[i] * (double)d[i];
        }
        const double rho = (double)k.rho_b0 + m0;
        const double px = jx + 0.5 * m0 * k.gx, py = jy + 0.5 * m0 * k.gy, pz = jz + 0.5 * m0 * k.gz;
        const size_t n = (size_t)nd.z * k.plane + nd.q;
        if (o_rr) o_rr[n] = (float)rr;
        if (o_rb) o_rb[n] = (float)rb;
        if (o_u) {
            o_u[3 * n] = (float)(px / rho);
            o_u[3 * n + 1] = (float)(py / rho);
            o_u[3 * n + 2] = (float)(pz / rho);
        }
        if (o_phi) {
            const double a = rr / k.rho_r0, b = rb / k.rho_b0;
            o_phi[n] = (float)((a - b) / (a + b));
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
