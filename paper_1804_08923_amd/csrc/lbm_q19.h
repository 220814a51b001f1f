// The step on the D3Q19 velocity set: the reduced lattice that Sec. II and
// Sec. IV B suggest as the way to cut the cost of the scheme, which the paper
// leaves without coefficients.  The coefficients keep every moment that the
// D3Q27 ones fix:
//   weights      1/3, 1/18 (faces), 1/36 (edges);
//   varphi_i     alpha at rest, w_i (1 - alpha) / (1 - w_0) = 1.5 w_i (1 - alpha)
//                otherwise (Eq. varphi_ik): sound speed squared (1 - alpha)/2;
//   Phi_i        -3 nu_bar u . grad rho at rest, m_i nu_bar (c.u)(c.grad rho)/4
//                with m = 2 on faces and 1 on edges (Eq. Phi): the second moment
//                nu_bar [u grad rho + grad rho u + (u . grad rho) I] of D3Q27;
//   B_i          -1/3 at rest, w_i otherwise (Eq. B_i): sum B_i = 1/3;
//   moments      the 19 rows of Eq. momentSet that are independent on D3Q19,
//                relaxed with s0, s1, s2nu, s2b, s3, s4 (Eq. scoll).
// Periodic and jet lattices, FP32 storage; the arithmetic is FP64 (the kernels are
// bound by memory traffic, and FP32 arithmetic would add about 1e-5 of the
// spurious velocity of a resting droplet to the FP32 storage floor).  Node
// index n = (z ny + y) nx + x with no padding; the periodic wrap is taken on
// the index.
//
// Reduced collision.  With the paper's rates (s0 = s1 = 0, s2b = s3 = s4 = 1)
// the GMRT collision plus forcing, f - T^-1 K T (f - feq) + T^-1 (I - K/2) T F'
// with T = N(u) M, is
//     fdag = feq + F'/2 + (1 - s2nu) T(u)^-1 P T(u) g,   g = f - feq + F'/2,
// where P keeps the five deviatoric second-order central moments.  g has no
// mass and no momentum, so its central second moments are its raw ones, Pi^g.
// T(u)^-1 of a vector of second-order central moments is taken through the
// monomial moments: the central moments kappa_ab of c - u give the raw ones by
// the binomial shift (the 19 monomials x^a y^b z^c with at most two exponents
// nonzero and each <= 2 form a set closed under the shift), and the raw
// monomial moments give the populations in closed form on D3Q19.
//
// Two state forms share one buffer of N-float planes:
//   general  planes 0..18 the colour-blind deviations d_i = f_i - w_i rho_b0
//            after streaming at x, 19..37 the populations of the node's
//            minority colour, 38 its tag (0: red, 1: blue); the majority colour
//            is f_i minus the minority one (written by init and set_state, read
//            by the first step);
//   shifted  planes 0..18 the deviations d_i = fdag_i - w_i rho_b0 at the node
//            that produced them, then (from byte align256(76 N)) four planes
//            of the record (x, V_x, V_y, V_z) per node, V = beta (rho_r rho_b / rho)
//            (1 - alpha_bar) grad phi / |grad phi|: the red population pulled
//            from x - c_i is (rho_r / rho) f_i + varphi-weighted c_i . V (Eqs.
//            op3r/op3b), so both colours are rebuilt from 23 floats.  x holds
//            the minority colour's fraction, rho_r / rho with the sign bit clear
//            or -rho_b / rho with it set.
// Both forms keep the minority colour without the cancellation f - f^major:
// its FP32 error inside a phase would leave a noisy grad phi for the
// perturbation to turn into velocity.
#pragma once
#include "lbm_diag.h"
#include "lbm_kernels.h"

namespace cglbm {
namespace q19 {

constexpr int Q19 = 19;  // directions 0..18 of the paper's order: rest, faces, edges
constexpr int GEN_PLANES = 2 * Q19 + 1;

__host__ __device__ constexpr double w19(int i)
{
    return csq(i) == 0 ? 1.0 / 3.0 : csq(i) == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
}

// varphi_i / ((1 - alpha) |c_i|): the recolouring weight of c_i . V
__host__ __device__ constexpr double krec(int i)
{
    return csq(i) == 1 ? 1.0 / 12.0 : 0.029462782549439480;  // 1 / (24 sqrt 2)
}

// byte offset of the records in the shifted form
__host__ __device__ inline uint64_t rec_offset(uint64_t N) { return (76ull * N + 255ull) & ~255ull; }

// buffer bytes: the larger of the two forms
__host__ inline uint64_t pop_bytes(uint64_t N)
{
    const uint64_t general = (uint64_t)GEN_PLANES * N * 4ull, shifted = rec_offset(N) + 16ull * N;
    return general > shifted ? general : shifted;
}

// This thread's node and the wrapped neighbour coordinates.  Blocks are handed
// to the 8 XCDs round-robin (block b of a plane goes to XCD b mod 8 when a
// plane has a multiple of 8 blocks); the plane's blocks are permuted so that
// each XCD takes a contiguous band of them, whose y- and z-neighbour rows are
// then fetched into that XCD's L2 only, instead of into three.
constexpr uint32_t kXcds = 8;

struct Site {
    uint32_t n;                    // node index
    uint32_t q;                    // y nx + x
    int x, y, z;
    uint32_t xs[3], ys[3], zs[3];  // periodic: x - 1, x, x + 1; (y - 1, y, y + 1) nx; (z - 1, z, z + 1) nx ny
    bool valid;
};

__device__ __forceinline__ Site site(const KP& k, int zoff = 0)
{
    Site s;
    const uint32_t B = gridDim.x, b = blockIdx.x;
    const uint32_t pb = (B % kXcds == 0) ? (b % kXcds) * (B / kXcds) + b / kXcds : b;
    const uint32_t p = pb * (uint32_t)BLOCK + threadIdx.x;
    s.valid = p < k.plane;
    const int z = (int)blockIdx.y + zoff;
    const int y = (int)(((uint64_t)p * k.nx_mul) >> k.nx_sh);
    const int x = (int)p - y * k.nx;
    s.xs[0] = x == 0 ? k.nx - 1 : x - 1;
    s.xs[1] = x;
    s.xs[2] = x == k.nx - 1 ? 0 : x + 1;
    s.ys[0] = (uint32_t)(y == 0 ? k.ny - 1 : y - 1) * k.nx;
    s.ys[1] = (uint32_t)y * k.nx;
    s.ys[2] = (uint32_t)(y == k.ny - 1 ? 0 : y + 1) * k.nx;
    s.zs[0] = (uint32_t)(z == 0 ? k.nz - 1 : z - 1) * k.plane;
    s.zs[1] = (uint32_t)z * k.plane;
    s.zs[2] = (uint32_t)(z == k.nz - 1 ? 0 : z + 1) * k.plane;
    s.n = s.zs[1] + p;
    s.q = p;
    s.x = x;
    s.y = y;
    s.z = z;
    return s;
}

// node at offset (dx, dy, dz) in {-1, 0, 1}^3
__device__ __forceinline__ uint32_t at(const Site& s, int dx, int dy, int dz)
{
    return s.zs[dz + 1] + s.ys[dy + 1] + s.xs[dx + 1];
}

// the recolouring record of the shifted form: four planes of N floats, the
// minority fraction x, then V_x, V_y, V_z
__device__ __forceinline__ const float* records(const float* pop, uint64_t N)
{
    return (const float*)((const char*)pop + rec_offset(N));
}

// red part of a population of value f pulled from node src along lattice
// direction i (whose velocity, reflected at walls, is (ex, ey, ez)): only the
// V components along which c_i is nonzero are read
__device__ __forceinline__ double red_part(const float* __restrict__ R, size_t N, uint32_t src, int i, double f,
                                           double ex, double ey, double ez)
{
    const float x = R[src];
    double cv = 0.0;
    if (kCX[i]) cv += ex * (double)R[N + src];
    if (kCY[i]) cv += ey * (double)R[2 * N + src];
    if (kCZ[i]) cv += ez * (double)R[3 * N + src];
    const double rec = i ? krec(i) * cv : 0.0;
    return signbit(x) ? f - (-(double)x * f - rec) : (double)x * f + rec;
}

// Jet boundaries (Sec. IV A), with the rules the D3Q27 path uses: a circular
// inlet at z = -1/2 whose ghost cells hold the red equilibrium of the inflow
// (with the seeded radial noise of the time level the populations left it),
// half-way free-slip walls at x, y = -1/2, n - 1/2 and z = -1/2 (specular
// reflection: the population of the clamped node with the outside components
// reversed), and the convective outflow of the top plane.

// inlet ghost population of direction i leaving ghost column (xg, yg) at
// post-collision time tg: red equilibrium at rho_r0, alpha_r, Phi = 0
__device__ __forceinline__ double inlet_feq19(const KP& k, int i, int xg, int yg, long long tg)
{
    const uint64_t cnt = ((uint64_t)tg * (uint64_t)k.ny + (uint64_t)yg) * (uint64_t)k.nx + (uint64_t)xg;
    const uint64_t r = splitmix64_nth(k.seed, cnt);
    const double xi = (double)(r >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    const double ur = (double)k.noise_amp * (double)k.inlet_u * xi;
    const double dx = (double)xg - (double)k.inlet_cx, dy = (double)yg - (double)k.inlet_cy;
    const double rr = sqrt(dx * dx + dy * dy);
    const double ux = rr > 0.0 ? ur * dx / rr : 0.0, uy = rr > 0.0 ? ur * dy / rr : 0.0;
    const double uz = k.inlet_uz ? (double)k.inlet_uz[yg * k.nx + xg] : (double)k.inlet_u;
    const double u2 = ux * ux + uy * uy + uz * uz;
    const double cu = kCX[i] * ux + kCY[i] * uy + kCZ[i] * uz;
    const double poly = cu * (3.0 + 4.5 * cu + 4.5 * cu * cu - 4.5 * u2) - 1.5 * u2;
    const double ph = i == 0 ? (double)k.alpha_r : 1.5 * w19(i) * (1.0 - (double)k.alpha_r);
    return (double)k.rho_r0 * (ph + w19(i) * poly);
}

// colour of population j of the shifted form at node src (Eqs. op3r/op3b)
__device__ __forceinline__ void shifted_pop(const float* __restrict__ pop, const KP& k, int j, uint32_t src,
                                            double& d, double& fr)
{
    const size_t N = k.N;
    d = (double)pop[(size_t)j * N + src];
    fr = red_part(records(pop, N), N, src, j, d + w19(j) * k.rho_b0, kCX[j], kCY[j], kCZ[j]);
}

// Population i streamed into node (x, y, z) of the shifted form: its deviation
// d and its red part fr (the blue part is d + w_i rho_b0 - fr).  Not for the
// jet's outlet plane, which the convective rule fills.
// BOT: the node may lie on the bottom plane z = 0 (the only plane that sees
// the inlet and the bottom wall); false lets the compiler drop that code
template <int BC, bool BOT = true>
__device__ __forceinline__ void pull_at(const float* __restrict__ pop, const KP& k, const Site& s, int i, double& d,
                                        double& fr)
{
    if constexpr (BC == LBM_BC_PERIODIC) {
        shifted_pop(pop, k, i, at(s, -kCX[i], -kCY[i], -kCZ[i]), d, fr);
    } else {
        const int cx = kCX[i], cy = kCY[i], cz = kCZ[i];
        // the source x - c_i lies outside along an axis: reflect there (the
        // walls act per axis; selects, no branch, so the loads of the 19
        // directions issue together)
        const bool ox = cx > 0 ? s.x == 0 : (cx < 0 ? s.x == k.nx - 1 : false);
        const bool oy = cy > 0 ? s.y == 0 : (cy < 0 ? s.y == k.ny - 1 : false);
        const bool oz = BOT && cz > 0 && s.z == 0;
        if (BOT && oz && inlet_inside(k, s.x - cx, s.y - cy)) {  // only on the bottom plane
            fr = inlet_feq19(k, i, s.x - cx, s.y - cy, k.t - 1);  // left the inlet at the previous time level
            d = fr - w19(i) * k.rho_b0;
            return;
        }
        const int m = (ox ? 1 : 0) | (oy ? 2 : 0) | (oz ? 4 : 0);
        const int j = m == 0 ? i : m == 1 ? mirror_dir(i, 1) : m == 2 ? mirror_dir(i, 2) : m == 3 ? mirror_dir(i, 3)
                    : m == 4 ? mirror_dir(i, 4) : m == 5 ? mirror_dir(i, 5) : m == 6 ? mirror_dir(i, 6)
                    : mirror_dir(i, 7);
        const int off = (ox ? 0 : cx) + (oy ? 0 : cy) * k.nx + (oz ? 0 : cz) * (int)k.plane;
        const uint32_t src = (uint32_t)((int)s.n - off);
        const size_t N = k.N;
        d = (double)pop[(size_t)j * N + src];
        // c_j: the components of c_i, reversed along the reflecting axes
        fr = red_part(records(pop, N), N, src, i, d + w19(i) * k.rho_b0, ox ? -cx : cx, oy ? -cy : cy,
                      oz ? -cz : cz);
    }
}

// general form at the node
__device__ __forceinline__ void general_pop(const float* __restrict__ pop, const KP& k, uint32_t n, int i, double& d,
                                            double& fr)
{
    const size_t N = k.N;
    d = (double)pop[(size_t)i * N + n];
    const double mn = (double)pop[(size_t)(Q19 + i) * N + n];
    const bool blue_min = pop[(size_t)(2 * Q19) * N + n] != 0.f;
    fr = blue_min ? d + w19(i) * k.rho_b0 - mn : mn;
}

// The jet's outlet plane after streaming by the convective rule (Lou et al.):
// f(N, t) = [f(N, t - 1) + lam f(N - 1, t)] / (1 + lam), lam = max(0, u_z(N - 1, t))
// with u_z of the freshly streamed plane below (half-force term included);
// hist holds f(N, t - 1) as (d, fr) planes.  Both colours.
__device__ __forceinline__ void outlet_rule(const float* __restrict__ pop, const float* __restrict__ hist,
                                            const KP& k, const Site& s, double (&d)[Q19], double (&fr)[Q19])
{
    Site below = s;  // the plane under the outlet
    below.z = k.nz - 2;
    below.n = s.n - k.plane;
    double m = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < Q19; ++i) {
        pull_at<LBM_BC_JET, false>(pop, k, below, i, d[i], fr[i]);
        m += d[i];
        if (kCZ[i]) jz += kCZ[i] * d[i];
    }
    const double uz = (jz + 0.5 * m * k.gz) / (k.rho_b0 + m);
    const double lam = uz > 0.0 ? uz : 0.0, il = 1.0 / (1.0 + lam);
    const size_t P = k.plane;
#pragma unroll
    for (int i = 0; i < Q19; ++i) {
        d[i] = ((double)hist[(size_t)i * P + s.q] + lam * d[i]) * il;
        fr[i] = ((double)hist[(size_t)(Q19 + i) * P + s.q] + lam * fr[i]) * il;
    }
}

// The state at this node: the populations after streaming, (d_i, fr_i), of
// either form; the jet's outlet plane from the general form, or by the rule.
template <bool GEN, int BC>
__device__ __forceinline__ void node_state(const float* __restrict__ pop, const float* __restrict__ hist, const KP& k,
                                           const Site& s, double (&d)[Q19], double (&fr)[Q19])
{
    if (GEN) {
#pragma unroll
        for (int i = 0; i < Q19; ++i) general_pop(pop, k, s.n, i, d[i], fr[i]);
    } else if (BC == LBM_BC_JET && s.z == k.nz - 1) {
        outlet_rule(pop, hist, k, s, d, fr);
    } else {
#pragma unroll
        for (int i = 0; i < Q19; ++i) pull_at<BC>(pop, k, s, i, d[i], fr[i]);
    }
}

// Per-node fields F (field buffer, two float2 arrays): F[n] = (phi, rho - rho_b0),
// which the collision gathers from the 18 neighbours, and F[N + n] =
// (rho_r, rho_b), which it reads at the node only.
__device__ __forceinline__ void store_fields(float2* __restrict__ F, const KP& k, uint32_t n, double rr, double rb,
                                             double m)
{
    const double a = rr / k.rho_r0, b = rb / k.rho_b0;
    F[n] = make_float2((float)((a - b) / (a + b)), (float)m);
    F[(size_t)k.N + n] = make_float2((float)rr, (float)rb);
}

template <bool GEN, int BC, bool BOT>
__device__ __forceinline__ void density_sums(const float* __restrict__ pop, const KP& k, const Site& s, double& rr,
                                             double& rb, double& m)
{
#pragma unroll
    for (int i = 0; i < Q19; ++i) {
        double d, fr;
        if (GEN)
            general_pop(pop, k, s.n, i, d, fr);
        else
            pull_at<BC, BOT>(pop, k, s, i, d, fr);
        m += d;
        rr += fr;
        rb += d + w19(i) * k.rho_b0 - fr;
    }
}

// Density pass (Eq. order): the fields F of every node, on the
// planes below the jet's outlet (all planes when periodic).
template <bool GEN, int BC>
__global__ __launch_bounds__(BLOCK) void k19_density(const float* __restrict__ pop, float2* __restrict__ F, KP k)
{
    const Site s = site(k);
    if (!s.valid) return;
    double rr = 0.0, rb = 0.0, m = 0.0;
    if (BC == LBM_BC_JET && s.z == 0)  // block-uniform
        density_sums<GEN, BC, true>(pop, k, s, rr, rb, m);
    else
        density_sums<GEN, BC, false>(pop, k, s, rr, rb, m);
    store_fields(F, k, s.n, rr, rb, m);
}

// The jet's outlet plane (one plane, blockIdx.y = 0): its populations after
// streaming (general form, or the convective rule from hprev) go to hcur as
// (d, fr), where the collision and the next step's rule read them, and its
// fields to F.
template <bool GEN>
__global__ __launch_bounds__(BLOCK) void k19_outlet(const float* __restrict__ pop, float2* __restrict__ F,
                                                    const float* __restrict__ hprev, float* __restrict__ hcur, KP k)
{
    const Site s = site(k, k.nz - 1);
    if (!s.valid) return;
    double d[Q19], fr[Q19];
    node_state<GEN, LBM_BC_JET>(pop, hprev, k, s, d, fr);
    double rr = 0.0, rb = 0.0, m = 0.0;
    const size_t P = k.plane;
#pragma unroll
    for (int i = 0; i < Q19; ++i) {
        m += d[i];
        rr += fr[i];
        rb += d[i] + w19(i) * k.rho_b0 - fr[i];
        hcur[(size_t)i * P + s.q] = (float)d[i];
        hcur[(size_t)(Q19 + i) * P + s.q] = (float)fr[i];
    }
    store_fields(F, k, s.n, rr, rb, m);
}

// (phi, rho - rho_b0) of the neighbour at offset (dx, dy, dz): periodic wrap,
// or (jet) (1, rho_r0 - rho_b0) in the inlet circle at z = -1 and the clamped
// node elsewhere outside (the mirrored field of the half-way walls and outlet)
template <int BC, bool BOT = true>
__device__ __forceinline__ float2 field_at(const float2* __restrict__ F, const KP& k, const Site& s, int dx, int dy,
                                           int dz)
{
    if constexpr (BC == LBM_BC_PERIODIC) {
        return F[at(s, dx, dy, dz)];
    } else {
        if (BOT && dz < 0 && s.z == 0 && inlet_inside(k, s.x + dx, s.y + dy))  // bottom plane only
            return make_float2(1.f, k.rho_r0 - k.rho_b0);
        // clamp per axis (selects)
        const int ex = (s.x + dx < 0 || s.x + dx >= k.nx) ? 0 : dx;
        const int ey = (s.y + dy < 0 || s.y + dy >= k.ny) ? 0 : dy;
        const int ez = (s.z + dz < 0 || s.z + dz >= k.nz) ? 0 : dz;
        return F[(uint32_t)((int)s.n + ex + ey * k.nx + ez * (int)k.plane)];
    }
}

// isotropic gradients of phi and rho, 3 sum_i w_i chi(x + c_i) c_i, summed
// over the opposite pairs (i, i + 1) as differences: exactly zero on a
// uniform field, which keeps the recolouring off there
template <int BC, bool BOT>
__device__ __forceinline__ void gradients(const float2* __restrict__ F, const KP& k, const Site& s, double& gpx,
                                          double& gpy, double& gpz, double& grx, double& gry, double& grz)
{
#pragma unroll
    for (int i = 1; i < Q19; i += 2) {
        const float2 qp = field_at<BC, BOT>(F, k, s, kCX[i], kCY[i], kCZ[i]);
        const float2 qm = field_at<BC, BOT>(F, k, s, -kCX[i], -kCY[i], -kCZ[i]);
        const double tp = 3.0 * w19(i) * ((double)qp.x - (double)qm.x);
        const double tr = 3.0 * w19(i) * ((double)qp.y - (double)qm.y);
        if (kCX[i]) { gpx += kCX[i] * tp; grx += kCX[i] * tr; }
        if (kCY[i]) { gpy += kCY[i] * tp; gry += kCY[i] * tr; }
        if (kCZ[i]) { gpz += kCZ[i] * tp; grz += kCZ[i] * tr; }
    }
}

// Collision, perturbation, recolouring and the store of the shifted form at the
// node itself (the next step pulls from it), Sec. II: Eqs. Momentum to op3b.
template <bool GEN, int BC>
__global__ __launch_bounds__(BLOCK) void k19_collide(const float* __restrict__ src, float* __restrict__ dst,
                                                     const float2* __restrict__ F, const float* __restrict__ hcur,
                                                     KP k)
{
    const Site s = site(k);
    if (!s.valid) return;
    const size_t N = k.N;
    float d[Q19];
    if (BC == LBM_BC_JET && s.z == k.nz - 1) {  // the outlet plane: the density pass wrote it to hcur
#pragma unroll
        for (int i = 0; i < Q19; ++i) d[i] = hcur[(size_t)i * k.plane + s.q];
    } else if (GEN) {
#pragma unroll
        for (int i = 0; i < Q19; ++i) d[i] = src[(size_t)i * N + s.n];
    } else if (BC == LBM_BC_JET && s.z == 0) {  // block-uniform
#pragma unroll
        for (int i = 0; i < Q19; ++i) {
            double dd, fr;
            pull_at<BC, true>(src, k, s, i, dd, fr);
            d[i] = (float)dd;
        }
    } else {
#pragma unroll
        for (int i = 0; i < Q19; ++i) {
            double dd, fr;
            pull_at<BC, false>(src, k, s, i, dd, fr);
            d[i] = (float)dd;
        }
    }
    const float2 P = F[s.n], Q = F[(size_t)k.N + s.n];
    const double phi = P.x, m = P.y, rr = Q.x, rb = Q.y;
    double gpx = 0, gpy = 0, gpz = 0, grx = 0, gry = 0, grz = 0;
    if (BC == LBM_BC_JET && s.z == 0)  // block-uniform
        gradients<BC, true>(F, k, s, gpx, gpy, gpz, grx, gry, grz);
    else
        gradients<BC, false>(F, k, s, gpx, gpy, gpz, grx, gry, grz);
    // interpolated properties, body force, velocity (Eqs. bodyForceJet, Momentum)
    const double rho = k.rho_b0 + m;
    const double hp = 0.5 * (1.0 + phi);
    const double ab = (double)k.alpha_b + hp * (double)k.dalpha;
    const double amw = (double)k.a_minus_w0 + hp * (double)k.dalpha;  // alpha_bar - 1/3
    const double nub = 1.0 / (hp * (double)k.inv_nu_r + (1.0 - hp) * (double)k.inv_nu_b);
    const double s2 = 1.0 / (3.0 * nub + 0.5);
    const double Fx = m * k.gx, Fy = m * k.gy, Fz = m * k.gz;
    double jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 1; i < Q19; ++i) {
        if (kCX[i]) jx += kCX[i] * (double)d[i];
        if (kCY[i]) jy += kCY[i] * (double)d[i];
        if (kCZ[i]) jz += kCZ[i] * (double)d[i];
    }
    const double irho = 1.0 / rho;
    const double ux = (jx + 0.5 * Fx) * irho, uy = (jy + 0.5 * Fy) * irho, uz = (jz + 0.5 * Fz) * irho;
    const double u2 = ux * ux + uy * uy + uz * uz;
    const double udr = ux * grx + uy * gry + uz * grz;
    const double uF = ux * Fx + uy * Fy + uz * Fz;
    const double kap = 1.5 * (1.0 - ab) * m - 1.5 * amw * k.rho_b0;  // 1.5 (1 - ab) rho - rho_b0
    // e_i = feq_i - w_i rho_b0 (Eq. EES, Eq. Phi) plus half the forcing
    // population (Eq. ketFd): the post-collision value without the
    // non-equilibrium part
    auto eq_half_force = [&](int i) -> double {
        const double cu = kCX[i] * ux + kCY[i] * uy + kCZ[i] * uz;
        const double cF = kCX[i] * Fx + kCY[i] * Fy + kCZ[i] * Fz;
        const double poly = cu * (3.0 + 4.5 * cu - 4.5 * u2 + 4.5 * cu * cu) - 1.5 * u2;
        double e;
        if (i == 0) {
            e = rho * amw + m * (1.0 / 3.0) + rho * w19(0) * poly - 3.0 * nub * udr;
        } else {
            const double cg = kCX[i] * grx + kCY[i] * gry + kCZ[i] * grz;
            const double mi = csq(i) == 1 ? 0.5 : 0.25;  // m_i / 4
            e = w19(i) * (kap + rho * poly) + mi * nub * cu * cg;
        }
        return e + 0.5 * w19(i) * (3.0 * (cF - uF) + 9.0 * cu * cF);
    };
    // Pi^g of g = f - feq + F'/2 from closed forms of the moments of feq and F'
    // (both lattices' coefficients give them): sum feq c c = rho [(1 - ab)/2 I
    // + u u] + nu_bar [u grad rho + grad rho u + (u . grad rho) I] (Eqs. EES,
    // Phi), sum F' c c = u F + F u (Eq. ketFd), sum w_i rho_b0 c c = rho_b0/3 I.
    // Only the deviatoric part is used, so the isotropic terms are left out:
    // dev Pi^g = dev [sum d c c - rho u u - nu_bar (u grad rho + grad rho u)
    //                 + (u F + F u)/2]
    double pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
#pragma unroll
    for (int i = 1; i < Q19; ++i) {
        const double g = (double)d[i];
        if (kCX[i]) pxx += g;
        if (kCY[i]) pyy += g;
        if (kCZ[i]) pzz += g;
        if (kCX[i] && kCY[i]) pxy += kCX[i] * kCY[i] * g;
        if (kCX[i] && kCZ[i]) pxz += kCX[i] * kCZ[i] * g;
        if (kCY[i] && kCZ[i]) pyz += kCY[i] * kCZ[i] * g;
    }
    pxx += -rho * ux * ux - 2.0 * nub * ux * grx + ux * Fx;
    pyy += -rho * uy * uy - 2.0 * nub * uy * gry + uy * Fy;
    pzz += -rho * uz * uz - 2.0 * nub * uz * grz + uz * Fz;
    pxy += -rho * ux * uy - nub * (ux * gry + uy * grx) + 0.5 * (ux * Fy + uy * Fx);
    pxz += -rho * ux * uz - nub * (ux * grz + uz * grx) + 0.5 * (ux * Fz + uz * Fx);
    pyz += -rho * uy * uz - nub * (uy * grz + uz * gry) + 0.5 * (uy * Fz + uz * Fy);
    // (1 - s2nu) times the deviatoric central second moments
    const double om = 1.0 - s2, tr3 = (pxx + pyy + pzz) * (1.0 / 3.0);
    const double k200 = om * (pxx - tr3), k020 = om * (pyy - tr3), k002 = om * (pzz - tr3);
    const double k110 = om * pxy, k101 = om * pxz, k011 = om * pyz;
    // raw monomial moments of h = T(u)^-1 of them (binomial shift)
    const double m210 = uy * k200 + 2.0 * ux * k110, m120 = ux * k020 + 2.0 * uy * k110;
    const double m201 = uz * k200 + 2.0 * ux * k101, m102 = ux * k002 + 2.0 * uz * k101;
    const double m021 = uz * k020 + 2.0 * uy * k011, m012 = uy * k002 + 2.0 * uz * k011;
    const double m220 = uy * uy * k200 + ux * ux * k020 + 4.0 * ux * uy * k110;
    const double m202 = uz * uz * k200 + ux * ux * k002 + 4.0 * ux * uz * k101;
    const double m022 = uz * uz * k020 + uy * uy * k002 + 4.0 * uy * uz * k011;
    // perturbation (Eq. perturb, Eq. B_i) and recolouring record (Eqs. op3r/op3b)
    const double G2 = gpx * gpx + gpy * gpy + gpz * gpz;
    const bool on = G2 > (double)k.eps2;
    const double gn = on ? sqrt(G2) : 0.0;
    const double Ag = on ? k.A * gn : 0.0;  // A |grad phi|
    const double iG2 = on ? 1.0 / G2 : 0.0;
    const double rc = rr + rb;
    const double vs = on ? k.beta * rr * rb / rc * (1.0 - ab) / gn : 0.0;
#pragma unroll
    for (int i = 0; i < Q19; ++i) {
        const int cx = kCX[i], cy = kCY[i], cz = kCZ[i];
        double h;
        if (cx && cy)
            h = 0.25 * (m220 + cx * m120 + cy * m210 + cx * cy * k110);
        else if (cx && cz)
            h = 0.25 * (m202 + cx * m102 + cz * m201 + cx * cz * k101);
        else if (cy && cz)
            h = 0.25 * (m022 + cy * m012 + cz * m021 + cy * cz * k011);
        else if (cx)
            h = 0.5 * ((k200 - m220 - m202) - cx * (m120 + m102));
        else if (cy)
            h = 0.5 * ((k020 - m220 - m022) - cy * (m210 + m012));
        else if (cz)
            h = 0.5 * ((k002 - m202 - m022) - cz * (m201 + m021));
        else
            h = (m220 + m202 + m022) - (k200 + k020 + k002);
        const double cgp = cx * gpx + cy * gpy + cz * gpz;
        const double Bi = i == 0 ? -1.0 / 3.0 : w19(i);
        const double pert = Ag * (w19(i) * cgp * cgp * iG2 - Bi);
        dst[(size_t)i * N + s.n] = (float)(eq_half_force(i) + h + pert);
    }
    // minority fraction: rho_r / rho, or -rho_b / rho (sign bit set, also for 0)
    const float xm = rr <= rb ? (float)(rr / rc) : -(float)(rb / rc);
    float* R = (float*)((char*)dst + rec_offset(N));
    R[s.n] = xm;
    R[N + s.n] = (float)(vs * gpx);
    R[2 * N + s.n] = (float)(vs * gpy);
    R[3 * N + s.n] = (float)(vs * gpz);
}

// Macroscopic fields (node order) and FP64 audit partial sums, one slot per block.
template <bool GEN, int BC>
__global__ __launch_bounds__(BLOCK) void k19_macro(const float* __restrict__ pop, const float* __restrict__ hist, KP k,
                                                   float* __restrict__ o_rr, float* __restrict__ o_rb,
                                                   float* __restrict__ o_u, float* __restrict__ o_phi,
                                                   double* __restrict__ partials)
{
    const Site s = site(k);
    double acc[5] = {0, 0, 0, 0, 0};
    if (s.valid) {
        double d[Q19], fv[Q19];
        node_state<GEN, BC>(pop, hist, k, s, d, fv);
        double m0 = 0.0, rr = 0.0, rb = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int i = 0; i < Q19; ++i) {
            m0 += d[i];
            rr += fv[i];
            rb += d[i] + w19(i) * k.rho_b0 - fv[i];
            if (kCX[i]) jx += kCX[i] * d[i];
            if (kCY[i]) jy += kCY[i] * d[i];
            if (kCZ[i]) jz += kCZ[i] * d[i];
        }
        const double rho = (double)k.rho_b0 + m0;
        const double px = jx + 0.5 * m0 * k.gx, py = jy + 0.5 * m0 * k.gy, pz = jz + 0.5 * m0 * k.gz;
        const size_t n = s.n;
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

// the state fr[i N + n], fb[(19 + i) N + n] of either form
template <bool GEN, int BC>
__global__ __launch_bounds__(BLOCK) void k19_get_state(const float* __restrict__ pop, const float* __restrict__ hist,
                                                       KP k, float* __restrict__ st)
{
    const Site s = site(k);
    if (!s.valid) return;
    const size_t N = k.N;
    double d[Q19], fr[Q19];
    node_state<GEN, BC>(pop, hist, k, s, d, fr);
#pragma unroll
    for (int i = 0; i < Q19; ++i) {
        st[(size_t)i * N + s.n] = (float)fr[i];
        st[(size_t)(Q19 + i) * N + s.n] = (float)(d[i] + w19(i) * k.rho_b0 - fr[i]);
    }
}

// Jet diagnostics (Sec. IV C), first pass on D3Q19: the order parameter of the
// current state binarised (phi as lbm_macroscopic returns it), labels and
// counters; the union-find passes that follow are those of the D3Q27 path.
template <bool GEN, int BC>
__global__ __launch_bounds__(BLOCK) void k19_diag_init(const float* __restrict__ pop, const float* __restrict__ hist,
                                                       KP k, DiagWork w)
{
    const Site s = site(k);
    bool fg = false;
    if (s.valid) {
        double d[Q19], fr[Q19];
        node_state<GEN, BC>(pop, hist, k, s, d, fr);
        double rr = 0.0, rb = 0.0;
#pragma unroll
        for (int i = 0; i < Q19; ++i) {
            rr += fr[i];
            rb += d[i] + w19(i) * k.rho_b0 - fr[i];
        }
        const double a = rr / k.rho_r0, b = rb / k.rho_b0;
        fg = (float)((a - b) / (a + b)) > 0.f;
        w.label[s.n] = fg ? (int)s.n : -1;
        w.count[s.n] = 0;
        w.column[s.n] = 0;
    }
    const unsigned long long m = __ballot(fg);
    const int zmax = wave_max_int(fg ? s.z : -1);
    if ((threadIdx.x & 63) == 0 && m) {
        atomicAdd(&w.hdr->jet_nodes, (unsigned long long)__popcll(m));
        atomicMax(&w.hdr->front_z, zmax);
    }
}

// general form of one node from FP64 colour populations: the deviations rounded
// once, the minority colour kept as given
__device__ __forceinline__ void put_general(float* __restrict__ dst, const KP& k, uint32_t n, const double (&fr)[Q19],
                                            const double (&fb)[Q19])
{
    const size_t N = k.N;
    double rr = 0.0, rb = 0.0;
#pragma unroll
    for (int i = 0; i < Q19; ++i) {
        rr += fr[i];
        rb += fb[i];
    }
    const bool blue_min = rr > rb;
#pragma unroll
    for (int i = 0; i < Q19; ++i) {
        dst[(size_t)i * N + n] = (float)(fr[i] + fb[i] - w19(i) * k.rho_b0);
        dst[(size_t)(Q19 + i) * N + n] = (float)(blue_min ? fb[i] : fr[i]);
    }
    dst[(size_t)(2 * Q19) * N + n] = blue_min ? 1.f : 0.f;
}

// a caller state (lbm_get_state layout) into the general form
__global__ __launch_bounds__(BLOCK) void k19_set_state(float* __restrict__ dst, KP k, const float* __restrict__ st)
{
    const Site s = site(k);
    if (!s.valid) return;
    const size_t N = k.N;
    double fr[Q19], fb[Q19];
#pragma unroll
    for (int i = 0; i < Q19; ++i) {
        fr[i] = st[(size_t)i * N + s.n];
        fb[i] = st[(size_t)(Q19 + i) * N + s.n];
    }
    put_general(dst, k, s.n, fr, fb);
}

// Initial state (general form): per-colour equilibria rho_k {varphi_i(alpha_k) +
// w_i [velocity terms of Eq. EES]} of the droplet preset or of caller fields,
// in FP64.
__global__ __launch_bounds__(BLOCK) void k19_init(float* __restrict__ dst, KP k, int kind,
                                                  const float* __restrict__ frr, const float* __restrict__ frb,
                                                  const float* __restrict__ fu, double dcx, double dcy, double dcz,
                                                  double R, double W, double rho_r0, double rho_b0, double alpha_r,
                                                  double alpha_b)
{
    const Site s = site(k);
    if (!s.valid) return;
    const uint32_t z = s.zs[1] / k.plane, p = s.n - s.zs[1];
    const uint32_t y = p / (uint32_t)k.nx, x = p - y * (uint32_t)k.nx;
    double rr, rb, ux = 0, uy = 0, uz = 0;
    if (kind == LBM_INIT_DROPLET) {
        const double dx = x - dcx, dy = y - dcy, dz = z - dcz;
        const double th = tanh(2.0 * (sqrt(dx * dx + dy * dy + dz * dz) - R) / W);
        rr = 0.5 * rho_r0 * (1.0 - th);
        rb = 0.5 * rho_b0 * (1.0 + th);
    } else if (kind == LBM_INIT_JET) {
        rr = 0.0;
        rb = rho_b0;
    } else {
        rr = frr[s.n];
        rb = frb[s.n];
        if (fu) {
            ux = fu[3 * (size_t)s.n];
            uy = fu[3 * (size_t)s.n + 1];
            uz = fu[3 * (size_t)s.n + 2];
        }
    }
    const double u2 = ux * ux + uy * uy + uz * uz;
    double fr[Q19], fb[Q19];
#pragma unroll
    for (int i = 0; i < Q19; ++i) {
        const double cu = kCX[i] * ux + kCY[i] * uy + kCZ[i] * uz;
        const double wp = w19(i) * (3.0 * cu + 4.5 * cu * cu - 1.5 * u2 + 4.5 * cu * cu * cu - 4.5 * cu * u2);
        const double phr = i == 0 ? alpha_r : 1.5 * w19(i) * (1.0 - alpha_r);
        const double phb = i == 0 ? alpha_b : 1.5 * w19(i) * (1.0 - alpha_b);
        fr[i] = rr * (phr + wp);
        fb[i] = rb * (phb + wp);
    }
    put_general(dst, k, s.n, fr, fb);
}

}  // namespace q19
}  // namespace cglbm
