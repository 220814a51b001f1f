// Reverse (adjoint) step of the colour-gradient LBM update.
//
// The step maps the state x_t = (f^r, f^b) (54 values per node) to x_{t+1}.
// For a cotangent lambda_{t+1} of x_{t+1} the adjoint step returns
// lambda_t = (d x_{t+1} / d x_t)^T lambda_{t+1} and adds lambda_{t+1} . d x_{t+1}/dA
// and lambda_{t+1} . d x_{t+1}/d u_in (the inlet axial-velocity profile) to the
// caller's gradient accumulators.  The forward quantities of step t are
// recomputed from x_t (no tape).  Passes:
//   1. densities of x_t -> (phi, rho - rho_b0), rho_r/rho per padded node, and the
//      raw moments of the colour-blind deviations up to second order; ghost shell
//   2. (jet) outlet: the convective condition of the outlet plane depends on the
//      streamed populations of the plane below; its adjoint is formed first
//      from a forward recomputation of the three top planes
//   3. per node: reverse streaming (gather of lambda_{t+1} from x + c_i, with the
//      reflections, inlet absorption and outlet rules of the forward step),
//      then the node vector-Jacobian product (lbm_adjoint_node.h); writes the
//      cotangents of the 10 raw moments (the cotangent of deviation i is their
//      quadratic polynomial in c_i), 8 stencil/centre cotangents and a block
//      partial of dJ/dA
//   4. ghost shell of the stencil cotangents (periodic copies; jet: zero,
//      plus the sums that the mirrored ghost fields route back to the wall nodes)
//   5. per node: transpose of the gradient stencil, chain rule through
//      phi(rho_r, rho_b), rho and rho_r/rho, and the red/blue cotangents
//   6. (jet) dJ/du_in over the inlet circle; dJ/dA reduction.
#pragma once
#include "lbm_adjoint_node.h"

namespace cglbm {

// ---------------------------------------------------------------- work buffer
struct AdjWork {
    float* MOM;     // raw moments m0, j (3), P (xx yy zz xy xz yz) of the deviations [10][N]
    float* LC;      // their cotangents [10][N]
    float4* AG0;    // (L grad phi, L phi_centre) per padded node
    float4* AG1;    // (L grad rho, L rho_r/rho) per padded node
    float2* GH;     // jet: stencil cotangents gathered at ghost cells (phi, rho)
    float* PS;      // jet: post-collision populations of the top three planes [54][3][plane]
    float* ML;      // jet: cotangent of the streamed plane nz - 2 incl. the outlet condition [54][plane]
    float* DL;      // jet: direct outlet term of lambda_t at plane nz - 1 [54][plane]
    float* ST;      // jet, state from a snapshot: the outlet plane of x_t as (d, f^r) [54][plane]
    double* AP;     // dJ/dA block partials
};

inline uint64_t align256(uint64_t b) { return (b + 255) & ~(uint64_t)255; }

inline uint64_t adjoint_layout(uint64_t NP, uint64_t N, uint64_t plane, uint64_t nblk, char* base, AdjWork* w)
{
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    char* mom = take(N * 10 * 4);
    char* lc = take(N * 10 * 4);
    char* a0 = take(NP * 16);
    char* a1 = take(NP * 16);
    char* gh = take(NP * 8);
    char* ps = take(2ull * Q * 3 * plane * 4);
    char* ml = take(2ull * Q * plane * 4);
    char* dl = take(2ull * Q * plane * 4);
    char* sp = take(2ull * Q * plane * 4);
    char* ap = take((nblk + 1) * 8);
    if (w) {
        w->MOM = (float*)mom;
        w->LC = (float*)lc;
        w->AG0 = (float4*)a0;
        w->AG1 = (float4*)a1;
        w->GH = (float2*)gh;
        w->PS = (float*)ps;
        w->ML = (float*)ml;
        w->DL = (float*)dl;
        w->ST = (float*)sp;
        w->AP = (double*)ap;
    }
    return off;
}

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ uint32_t nidx(const KP& k, int x, int y, int z)
{
    return ((uint32_t)z * (uint32_t)k.ny + (uint32_t)y) * (uint32_t)k.nx + (uint32_t)x;
}

// 1. densities and raw moments of the deviations d_i = f^r_i + f^b_i - w_i rho_b0
// of an FP32 state (fr planes, then fb), accumulated in FP64
__global__ __launch_bounds__(BLOCK) void k_adj_density(const float* __restrict__ st, float2* __restrict__ PD,
                                                        float* __restrict__ XR, float* __restrict__ MOM, KP k)
{
    const Node nd = this_node(k);
    if (!nd.valid) return;
    const size_t N = k.N;
    const uint32_t n = nidx(k, nd.x, nd.y, nd.z);
    double rr = 0.0;
    MomT<double> M;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double a = st[(size_t)i * N + n], b = st[(size_t)(Q + i) * N + n];
        rr += a;
        M.add(i, (a + b) - wgtd(i) * (double)k.rho_b0);
    }
    // the adjoint passes keep the red fraction x_r = rho_r/rho in XR
    const double rho = (double)k.rho_b0 + M.m0;
    store_pd(PD, k, nd.n, M.m0, rr, rho - rr);
    stp(XR, nd.n, (float)(rr / rho));
    const double mv[10] = {M.m0, M.j[0], M.j[1], M.j[2], M.P[0], M.P[1], M.P[2], M.P[3], M.P[4], M.P[5]};
#pragma unroll
    for (int a = 0; a < 10; ++a) MOM[(size_t)a * N + n] = (float)mv[a];
}

// forward node quantities of node nd from its moments and the field stencil
__device__ __forceinline__ void adj_node_fwd(const KP& k, const float* __restrict__ MOM,
                                             const float2* __restrict__ PD, const float* __restrict__ XR,
                                             const Node& nd, NodeFwdT<float>& f, float& xr)
{
    const size_t N = k.N;
    const uint32_t n = nidx(k, nd.x, nd.y, nd.z);
    MomT<float> M;
    M.m0 = MOM[n];
    for (int a = 0; a < 3; ++a) M.j[a] = MOM[(size_t)(1 + a) * N + n];
    for (int a = 0; a < 6; ++a) M.P[a] = MOM[(size_t)(4 + a) * N + n];
    const float phic = ldp(PD, nd.n).x;
    xr = ldp(XR, nd.n);
    if (k.xr_tagged) xr = frac_of(xr, 0u);
    double g[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    gradients(PD, k, nd.n, g);
    node_fwd<float>(k, M, phic, g, f);
}

// 2a. (jet) post-collision populations of planes nz - 3 .. nz - 1 (z0 = nz - 3)
__global__ __launch_bounds__(BLOCK) void k_adj_top_post(const float* __restrict__ MOM, const float2* __restrict__ PD,
                                                         const float* __restrict__ XR, float* __restrict__ PS, KP k)
{
    const Node nd = this_node(k);
    if (!nd.valid) return;
    NodeFwdT<float> f;
    float xr;
    adj_node_fwd(k, MOM, PD, XR, nd, f, xr);
    float fp[Q], V[3];
    node_post<float>(k, f, xr, fp, V);
    const int zz = nd.z - k.z0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        float fr, fb;
        recolour_dir<float>(i, xr, fp[i], V, fr, fb);
        PS[((size_t)i * 3 + zz) * k.plane + nd.q] = fr;
        PS[((size_t)(Q + i) * 3 + zz) * k.plane + nd.q] = fb;
    }
}

// 2b. (jet) outlet condition f(N) = [h + lam y] / (1 + lam), lam = max(0, u_z(y)),
// y = the streamed populations of plane nz - 2, h = the state's plane nz - 1.
// Writes ML = cotangent of y (lambda of plane nz - 2 plus the outlet terms) and
// DL = lambda of plane nz - 1 / (1 + lam) (the direct dependence on h).
// h comes as (f^r, f^b) planes of stride hs (dfr = 0) or as the (d, f^r)
// planes of stride plane that the density pass of a snapshot wrote (dfr = 1).
__device__ __forceinline__ double top_value(const KP& k, const float* __restrict__ h, size_t hs, int dfr, int j,
                                            uint32_t q)
{
    if (!dfr) return h[(size_t)j * hs + q];
    if (j < Q) return h[(size_t)(Q + j) * k.plane + q];
    const int i = j - Q;
    return ((double)h[(size_t)i * k.plane + q] + wgtd(i) * (double)k.rho_b0) - (double)h[(size_t)(Q + i) * k.plane + q];
}

__global__ __launch_bounds__(BLOCK) void k_adj_outlet(const float* __restrict__ htop, size_t hs, int dfr,
                                                       const float* __restrict__ lam_in,
                                                       const float* __restrict__ PS, float* __restrict__ ML,
                                                       float* __restrict__ DL, KP k)
{
    const uint32_t q = blockIdx.x * BLOCK + threadIdx.x;
    if (q >= k.plane) return;
    const int y = (int)(q / (uint32_t)k.nx), x = (int)(q - (uint32_t)y * k.nx);
    const int zb = k.nz - 2, zt = k.nz - 3;
    const size_t N = k.N, P = k.plane;
    float yv[2 * Q];
    double rho = 0.0, jz = 0.0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        int sx = x - kCX[j], sy = y - kCY[j], m = 0;
        if (sx < 0 || sx >= k.nx) { m |= 1; sx = x; }
        if (sy < 0 || sy >= k.ny) { m |= 2; sy = y; }
        const int jj = kMirror.v[j * 8 + m];
        const int zz = zb - kCZ[j] - zt;
        const uint32_t s = (uint32_t)sy * k.nx + (uint32_t)sx;
        yv[j] = PS[((size_t)jj * 3 + zz) * P + s];
        yv[Q + j] = PS[((size_t)(Q + jj) * 3 + zz) * P + s];
        const double f = (double)yv[j] + (double)yv[Q + j];
        rho += f;
        jz += kCZ[j] * f;
    }
    const double uz = (jz + 0.5 * (rho - (double)k.rho_b0) * (double)k.gz) / rho;
    const double lam = uz > 0.0 ? uz : 0.0;
    const double inv = 1.0 / (1.0 + lam);
    const size_t ntop = (size_t)(k.nz - 1) * P + q, nbot = (size_t)zb * P + q;
    double Llam = 0.0;
#pragma unroll
    for (int j = 0; j < 2 * Q; ++j) {
        const double L1 = lam_in[(size_t)j * N + ntop];
        const double h = top_value(k, htop, hs, dfr, j, q);
        Llam += L1 * ((double)yv[j] - h) * inv * inv;
    }
    const double Luz = uz > 0.0 ? Llam : 0.0;
#pragma unroll
    for (int j = 0; j < 2 * Q; ++j) {
        const int i = j < Q ? j : j - Q;
        const double L1 = lam_in[(size_t)j * N + ntop];
        const double L2 = lam_in[(size_t)j * N + nbot];
        ML[(size_t)j * P + q] = (float)(L2 + L1 * lam * inv + Luz * ((double)kCZ[i] + 0.5 * (double)k.gz - uz) / rho);
        DL[(size_t)j * P + q] = (float)(L1 * inv);
    }
}

// 3. reverse streaming and node VJP
// direction I with the components in mask m reversed, by selects (m varies per lane)
template <int I>
__device__ __forceinline__ int mirror_sel(int m)
{
    constexpr int t0 = mirror_dir(I, 0), t1 = mirror_dir(I, 1), t2 = mirror_dir(I, 2), t3 = mirror_dir(I, 3);
    constexpr int t4 = mirror_dir(I, 4), t5 = mirror_dir(I, 5), t6 = mirror_dir(I, 6), t7 = mirror_dir(I, 7);
    return (m & 4) ? ((m & 2) ? ((m & 1) ? t7 : t6) : ((m & 1) ? t5 : t4))
                   : ((m & 2) ? ((m & 1) ? t3 : t2) : ((m & 1) ? t1 : t0));
}

// cotangents of the post-collision populations of this node: those of the
// populations they become after streaming (x + c_i, reversed on every axis
// that leaves the lattice), zero where the forward step overwrites them
template <int BC, int I = 0>
__device__ __forceinline__ void adj_gather(const KP& k, const float* __restrict__ lam, const float* __restrict__ ML,
                                           const Node& nd, float* Lr, float* Lb)
{
    if constexpr (I < Q) {
        const size_t N = k.N;
        constexpr int cx = kCX[I], cy = kCY[I], cz = kCZ[I];
        int dx = nd.x + cx, dy = nd.y + cy, dz = nd.z + cz;
        float vr = 0.f, vb = 0.f;
        if (BC == LBM_BC_PERIODIC) {
            if (cx) dx = wrapc(dx, k.nx);
            if (cy) dy = wrapc(dy, k.ny);
            if (cz) dz = wrapc(dz, k.nz);
            const size_t n = nidx(k, dx, dy, dz);
            vr = lam[(size_t)I * N + n];
            vb = lam[(size_t)(Q + I) * N + n];
        } else {
            int m = 0;
            bool lost = false;
            if (cx && (dx < 0 || dx >= k.nx)) { m |= 1; dx = nd.x; }
            if (cy && (dy < 0 || dy >= k.ny)) { m |= 2; dy = nd.y; }
            if (cz < 0 && dz < 0) {
                // the ghost below this node is an inlet cell: overwritten by the inflow
                if (m == 0 && inlet_inside(k, nd.x, nd.y)) lost = true;
                m |= 4;
                dz = nd.z;
            }
            if (cz > 0 && dz >= k.nz - 1) lost = true;   // replaced by the convective condition
            if (cz == 0 && dz == k.nz - 1) lost = true;
            if (!lost) {
                const int j = cx || cy || cz < 0 ? mirror_sel<I>(m) : I;
                if (dz == k.nz - 2) {
                    const size_t q = (size_t)dy * k.nx + dx;
                    vr = ML[(size_t)j * k.plane + q];
                    vb = ML[(size_t)(Q + j) * k.plane + q];
                } else {
                    const size_t n = nidx(k, dx, dy, dz);
                    vr = lam[(size_t)j * N + n];
                    vb = lam[(size_t)(Q + j) * N + n];
                }
            }
        }
        Lr[I] = vr;
        Lb[I] = vb;
        adj_gather<BC, I + 1>(k, lam, ML, nd, Lr, Lb);
    }
}

template <int BC>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_adj_node(
    const float* __restrict__ MOM, const float* __restrict__ lam_in, const float* __restrict__ ML,
    const float2* __restrict__ PD, const float* __restrict__ XR, float* __restrict__ LC, float4* __restrict__ AG0,
    float4* __restrict__ AG1, double* __restrict__ AP, KP k)
{
    // the (phi, rho) stencil from the caches: an LDS window with its barrier
    // measured slower at this kernel's two waves per SIMD
    const Node nd = this_node(k);
    double acc[1] = {0.0};
    if (nd.valid) {
        NodeFwdT<float> f;
        float xr;
        adj_node_fwd(k, MOM, PD, XR, nd, f, xr);
        float Lr[Q], Lb[Q];
        adj_gather<BC>(k, lam_in, ML, nd, Lr, Lb);
        NodeAdjT<float> o;
        node_vjp<float>(k, f, xr, Lr, Lb, o);
        const size_t N = k.N;
        const uint32_t n = nidx(k, nd.x, nd.y, nd.z);
        const float lc[10] = {o.Lm0, o.Lj[0], o.Lj[1], o.Lj[2], o.Lq[0], o.Lq[1], o.Lq[2], o.Lq[3], o.Lq[4], o.Lq[5]};
#pragma unroll
        for (int a = 0; a < 10; ++a) LC[(size_t)a * N + n] = lc[a];
        stp(AG0, nd.n, make_float4(o.Lgp[0], o.Lgp[1], o.Lgp[2], o.Lphic));
        stp(AG1, nd.n, make_float4(o.Lgr[0], o.Lgr[1], o.Lgr[2], o.Lxr));
        acc[0] = (double)o.LA;
    }
    block_partials<1>(acc, AP, blockIdx.y * gridDim.x + blockIdx.x);
}

// 4. ghost shell of the stencil cotangents.  Periodic: copies of the wrapped
// nodes.  Jet: zero (the transpose gather then sees only interior nodes), and
// GH = the stencil cotangent that reads this ghost cell's mirrored field
// value, to be routed to the wall node it copies (zero in the inlet circle,
// where the ghost fields are constants).
template <int BC>
__global__ __launch_bounds__(BLOCK) void k_adj_ghosts(float4* __restrict__ AG0, float4* __restrict__ AG1,
                                                       float2* __restrict__ GH, KP k, uint32_t ncells)
{
    const uint32_t gidx = blockIdx.x * BLOCK + threadIdx.x;
    if (gidx >= ncells) return;
    const Ghost c = shell_cell(k, gidx);
    if (!c.valid) return;
    const uint32_t gi = pidx(k, c.x, c.y, c.z);
    if (BC == LBM_BC_PERIODIC) {
        const uint32_t wi = pidx(k, wrapc(c.x, k.nx), wrapc(c.y, k.ny), wrapc(c.z, k.nz));
        AG0[gi] = AG0[wi];
        AG1[gi] = AG1[wi];
        return;
    }
    float sp = 0.f, sr = 0.f;
    if (!(c.z < 0 && inlet_inside(k, c.x, c.y))) {
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int x = c.x - kCX[i], y = c.y - kCY[i], z = c.z - kCZ[i];
            if (x < 0 || x >= k.nx || y < 0 || y >= k.ny || z < 0 || z >= k.nz) continue;
            const uint32_t s = pidx(k, x, y, z);
            const float4 a0 = AG0[s], a1 = AG1[s];
            const float w3 = 3.f * wgt(i);
            sp += w3 * (kCX[i] * a0.x + kCY[i] * a0.y + kCZ[i] * a0.z);
            sr += w3 * (kCX[i] * a1.x + kCY[i] * a1.y + kCZ[i] * a1.z);
        }
    }
    GH[gi] = make_float2(sp, sr);
    // only interior cells are read above, only ghost cells are written here
    AG0[gi] = make_float4(0.f, 0.f, 0.f, 0.f);
    AG1[gi] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// 5. transpose of the gradient stencil and the red / blue cotangents
template <int BC>
__global__ __launch_bounds__(BLOCK) void k_adj_fields(const float4* __restrict__ AG0, const float4* __restrict__ AG1,
                                                       const float2* __restrict__ GH, const float2* __restrict__ PD,
                                                       const float* __restrict__ XR, const float* __restrict__ DL,
                                                       const float* __restrict__ LC, float* __restrict__ lam_out, KP k)
{
    // the stencil cotangents of the tile and its rim from LDS windows
    __shared__ float4 w0[SW], w1[SW];
    const Tile t = this_tile(k);
    const Node& nd = t.nd;
    // batched staging (all loads before the LDS writes): 1.95 -> 1.73 ms per
    // adjoint step on the 128x128x512 jet
    load_window<STY, true>(w0, AG0, k, t);
    load_window<STY, true>(w1, AG1, k, t);
    __syncthreads();
    if (!nd.valid) return;
    float Lphi = w0[wslot(t.lx, t.ly, 0, 0, 0)].w, Lrf = 0.f;
    const float Lxr = w1[wslot(t.lx, t.ly, 0, 0, 0)].w;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int ws = wslot(t.lx, t.ly, -kCX[i], -kCY[i], -kCZ[i]);
        const float4 a0 = w0[ws], a1 = w1[ws];
        const float w3 = 3.f * wgt(i);
        Lphi += w3 * (kCX[i] * a0.x + kCY[i] * a0.y + kCZ[i] * a0.z);
        Lrf += w3 * (kCX[i] * a1.x + kCY[i] * a1.y + kCZ[i] * a1.z);
    }
    if (BC == LBM_BC_JET) {
        // ghost cells whose mirrored field value is this node's
        const int lx = nd.x == 0 ? -1 : 0, hx = nd.x == k.nx - 1 ? 1 : 0;
        const int ly = nd.y == 0 ? -1 : 0, hy = nd.y == k.ny - 1 ? 1 : 0;
        const int lz = nd.z == 0 ? -1 : 0, hz = nd.z == k.nz - 1 ? 1 : 0;
        if (lx | hx | ly | hy | lz | hz) {
            for (int sz = lz; sz <= hz; ++sz)
                for (int sy = ly; sy <= hy; ++sy)
                    for (int sx = lx; sx <= hx; ++sx) {
                        if (!(sx | sy | sz)) continue;
                        const float2 gh = GH[pidx(k, nd.x + sx, nd.y + sy, nd.z + sz)];
                        Lphi += gh.x;
                        Lrf += gh.y;
                    }
        }
    }
    // phi = (a - b)/(a + b), a = rho_r/rho_r0, b = rho_b/rho_b0; rho_r/rho; rho
    const float2 pd = ldp(PD, nd.n);
    const double rho = (double)k.rho_b0 + (double)pd.y;
    const float xrn = k.xr_tagged ? frac_of(ldp(XR, nd.n), 0u) : ldp(XR, nd.n);
    const double rr = (double)xrn * rho, rb = rho - rr;
    const double a = rr / (double)k.rho_r0, b = rb / (double)k.rho_b0;
    const double ab2 = (a + b) * (a + b);
    const float Lrr = (float)(Lphi * 2.0 * b / (ab2 * (double)k.rho_r0) + Lrf + Lxr * rb / (rho * rho));
    const float Lrb = (float)(-Lphi * 2.0 * a / (ab2 * (double)k.rho_b0) + Lrf - Lxr * rr / (rho * rho));
    const size_t N = k.N;
    const uint32_t n = nidx(k, nd.x, nd.y, nd.z);
    float lc[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) lc[c] = LC[(size_t)c * N + n];
    const bool top = BC == LBM_BC_JET && nd.z == k.nz - 1;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = kCX[i], cy = kCY[i], cz = kCZ[i];
        float Ld = lc[0];
        if (cx) Ld += cx * lc[1] + lc[4];
        if (cy) Ld += cy * lc[2] + lc[5];
        if (cz) Ld += cz * lc[3] + lc[6];
        if (cx * cy) Ld += (cx * cy) * lc[7];
        if (cx * cz) Ld += (cx * cz) * lc[8];
        if (cy * cz) Ld += (cy * cz) * lc[9];
        float r = Ld + Lrr, bl = Ld + Lrb;
        if (top) {
            r += DL[(size_t)i * k.plane + nd.q];
            bl += DL[(size_t)(Q + i) * k.plane + nd.q];
        }
        lam_out[(size_t)i * N + n] = r;
        lam_out[(size_t)(Q + i) * N + n] = bl;
    }
}

// 6a. (jet) dJ/du_in: the inlet ghost column (gx, gy) feeds the red populations
// with c_z = +1 of the nodes (gx + c_x, gy + c_y, 0) with its equilibrium.
template <int I = 0>
__device__ __forceinline__ void inlet_grad_dirs(const KP& k, const float* __restrict__ lam, int gx, int gy,
                                                const double (&u)[3], double& acc)
{
    if constexpr (I < Q) {
        if constexpr (kCZ[I] == 1) {
            const int x = gx + kCX[I], y = gy + kCY[I];
            if (x >= 0 && x < k.nx && y >= 0 && y < k.ny) {
                const double cu = kCX[I] * u[0] + kCY[I] * u[1] + u[2];
                const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                const double dfe = (double)k.rho_r0 * wgtd(I) *
                                   ((3.0 + 9.0 * cu + 13.5 * cu * cu - 4.5 * u2) - (3.0 + 9.0 * cu) * u[2]);
                acc += (double)lam[(size_t)I * k.N + (size_t)y * k.nx + x] * dfe;
            }
        }
        inlet_grad_dirs<I + 1>(k, lam, gx, gy, u, acc);
    }
}

__global__ __launch_bounds__(BLOCK) void k_adj_inlet(const float* __restrict__ lam_in, float* __restrict__ dJ_du,
                                                      KP k)
{
    const uint32_t q = blockIdx.x * BLOCK + threadIdx.x;
    if (q >= k.plane) return;
    const int gy = (int)(q / (uint32_t)k.nx), gx = (int)(q - (uint32_t)gy * k.nx);
    if (!inlet_inside(k, gx, gy)) return;
    // inflow velocity of this column at time t (same construction as the forward step)
    const uint64_t cnt = ((uint64_t)k.t * (uint64_t)k.ny + (uint64_t)gy) * (uint64_t)k.nx + (uint64_t)gx;
    const uint64_t r = splitmix64_nth(k.seed, cnt);
    const double xi = (double)(r >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    const float ur = (float)((double)k.noise_amp * (double)k.inlet_u * xi);
    const float dx = (float)gx - k.inlet_cx, dy = (float)gy - k.inlet_cy;
    const float rr = sqrtf(dx * dx + dy * dy);
    double u[3];
    u[0] = rr > 0.f ? ur * dx / rr : 0.f;
    u[1] = rr > 0.f ? ur * dy / rr : 0.f;
    u[2] = k.inlet_uz ? k.inlet_uz[q] : k.inlet_u;
    double acc = 0.0;
    inlet_grad_dirs(k, lam_in, gx, gy, u, acc);
    dJ_du[q] += (float)acc;
}

// 6b. dJ/dA += sum of the block partials (one block of 1024 threads)
constexpr int SUM_BLOCK = 1024;
__global__ __launch_bounds__(SUM_BLOCK) void k_adj_sumA(const double* __restrict__ AP, int nblk,
                                                         double* __restrict__ out)
{
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int b = threadIdx.x;
    for (; b + 3 * SUM_BLOCK < nblk; b += 4 * SUM_BLOCK) {
        a0 += AP[b];
        a1 += AP[b + SUM_BLOCK];
        a2 += AP[b + 2 * SUM_BLOCK];
        a3 += AP[b + 3 * SUM_BLOCK];
    }
    for (; b < nblk; b += SUM_BLOCK) a0 += AP[b];
    __shared__ double red[SUM_BLOCK / 64];
    const double s = wave_sum((a0 + a1) + (a2 + a3));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < SUM_BLOCK / 64; ++w) t += red[w];
        out[0] += t;
    }
}

}  // namespace cglbm
