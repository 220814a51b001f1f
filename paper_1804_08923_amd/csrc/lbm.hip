// C ABI of liblbm.so (declared in include/cglbm.h): validation, buffer
// sizing, handle state and kernel launches.  Device memory is owned by the
// caller; this file never allocates it.
#include <stdarg.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "lbm_adjoint.h"
#include "lbm_diag.h"
#include "lbm_kernels.h"
#include "lbm_q19.h"

using namespace cglbm;

// Work memory of lbm_jet_diagnostics_static (the union-find labels, counts,
// column marks and fragment volumes of diag_layout) for lattices of up to
// kStaticDiagNodes nodes, held by the library on every GPU it runs on until
// the process ends.  Host code reaches it only through the device address
// hipGetSymbolAddress returns for the current device (g_scratch below).
constexpr uint64_t kStaticDiagNodes = 1ull << 22;
constexpr uint64_t kStaticDiagBytes = diag_bytes(kStaticDiagNodes);
static __device__ __align__(256) unsigned char scratch[kStaticDiagBytes];

// One complete state: population planes (shifted form, or the general form
// of 54 planes), the recolouring records R, the reference records of the
// referenced 16-bit forms, and (jet) the outlet plane the next step's
// convective condition starts from.
struct StateSet {
    void* pop;
    float4* R;
    uint4* Q;
    float* hist;
};

struct lbm_handle {
    lbm_params p;
    int q19;            // D3Q19 lattice (lbm_q19.h): own buffers only, no snapshots or adjoint
    KP k;
    StateSet own[2];    // the handle's A and B sets (caller buffers given to lbm_init)
    StateSet ext;       // a caller snapshot that lbm_step_into made current
    int cs;             // current set: 0 or 1 (own), 2 (ext)
    float2* PD;         // (phi, rho - rho_b0) per padded node
    float* XR;          // tagged minority-colour fraction per padded node
    float2* F2;         // D3Q19: (phi, rho - rho_b0) per node, then (rho_r, rho_b) per node
    double* audit;
    void* adjoint;
    hipStream_t stream;
    int device;         // the HIP device current at lbm_init (its scratch address is g_scratch[device])
    long long t;        // time level of the current state
    int unshifted;      // current buffer holds a general state at the node itself
    dim3 grid_all;      // every interior plane
    dim3 grid_tiles;    // stencil tiles of the fused collision
    dim3 grid_dtiles;   // stencil tiles of the density pass
    dim3 grid_plane;    // one plane
    dim3 grid_shell;    // ghost shell cells
    uint32_t ncells;    // ghost shell cell count
    int nblk;           // blocks of grid_all (audit partial slots)
    // instrumentation: events around the kernel groups of each step
    int profiling;
    std::vector<hipEvent_t> ev;  // pool, 5 per recorded step
    size_t ev_used;
};

namespace {

thread_local char g_err[512] = "";

// device address of `scratch` on each device, looked up once per device
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_CHECK(expr)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail(LBM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define LAUNCH_CHECK()                                                                    \
    do {                                                                                  \
        hipError_t e_ = hipGetLastError();                                                \
        if (e_ != hipSuccess) return fail(LBM_ERR_HIP, "kernel launch: %s", hipGetErrorString(e_)); \
    } while (0)

size_t elem_bytes(int storage) { return storage == LBM_STORAGE_FP32 ? 4 : 2; }

bool eq_ref(int storage) { return storage == LBM_STORAGE_BF16_EQ || storage == LBM_STORAGE_FP16_EQ; }

// floats per padded node of the field buffer: R (x2), [reference records (x2)], PD, XR
uint64_t field_floats(int storage) { return eq_ref(storage) ? 19 : 11; }

uint64_t padded_nodes(const lbm_params* p)
{
    return (uint64_t)(p->nx + 2) * (uint64_t)(p->ny + 2) * (uint64_t)(p->nz + 2);
}

bool is_q19(const lbm_params* p) { return p->lattice == 19; }

int validate(const lbm_params* p)
{
    if (!p) return fail(LBM_ERR_INVALID_ARG, "params is NULL");
    if (p->lattice != 0 && p->lattice != 27 && p->lattice != 19)
        return fail(LBM_ERR_INVALID_ARG, "unknown lattice %d (19 or 27)", p->lattice);
    if (is_q19(p)) {
        if (p->storage != LBM_STORAGE_FP32)
            return fail(LBM_ERR_UNSUPPORTED, "the D3Q19 lattice is implemented with FP32 storage only");
        if ((uint64_t)p->nx * p->ny * p->nz > (1ull << 31))
            return fail(LBM_ERR_UNSUPPORTED, "the D3Q19 lattice holds at most 2^31 nodes");
    }
    if (p->bc != LBM_BC_PERIODIC && p->bc != LBM_BC_JET) return fail(LBM_ERR_INVALID_ARG, "unknown bc %d", p->bc);
    if (p->storage < LBM_STORAGE_FP32 || p->storage > LBM_STORAGE_FP16_EQ)
        return fail(LBM_ERR_INVALID_ARG, "unknown storage %d", p->storage);
    const int minn = p->bc == LBM_BC_JET ? 3 : 1;
    if (p->nx < minn || p->ny < minn || p->nz < minn)
        return fail(LBM_ERR_INVALID_ARG, "lattice %dx%dx%d too small (min %d)", p->nx, p->ny, p->nz, minn);
    if (p->nx > 65535 || p->ny > 65535 || p->nz > 65535)
        return fail(LBM_ERR_UNSUPPORTED, "a lattice dimension above 65535");
    // 32-bit byte offsets of a float2 per padded node
    if ((double)padded_nodes(p) * 8.0 > 4294967295.0)
        return fail(LBM_ERR_UNSUPPORTED, "more than 2^29 padded nodes");
    if (!(p->nu_r > 0) || !(p->nu_b > 0)) return fail(LBM_ERR_INVALID_ARG, "viscosities must be > 0");
    if (!(p->rho_r0 > 0) || !(p->rho_b0 > 0)) return fail(LBM_ERR_INVALID_ARG, "reference densities must be > 0");
    if (!(p->alpha_b > 0 && p->alpha_b < 1)) return fail(LBM_ERR_INVALID_ARG, "alpha_b must lie in (0, 1)");
    const double ar = 1.0 - (1.0 - p->alpha_b) * p->rho_b0 / p->rho_r0;
    if (!(ar >= 0 && ar < 1)) return fail(LBM_ERR_INVALID_ARG, "alpha_r = %g outside [0, 1)", ar);
    if (!(p->beta >= 0 && p->beta <= 1)) return fail(LBM_ERR_INVALID_ARG, "beta must lie in [0, 1]");
    if (!std::isfinite(p->A) || !std::isfinite(p->g[0]) || !std::isfinite(p->g[1]) || !std::isfinite(p->g[2]))
        return fail(LBM_ERR_INVALID_ARG, "A and g must be finite");
    if (p->s_b != 1.0 || p->s3 != 1.0 || p->s4 != 1.0 || p->s5 != 1.0 || p->s6 != 1.0)
        return fail(LBM_ERR_UNSUPPORTED, "only s2b = s3 = s4 = s5 = s6 = 1 (the paper's rates) are implemented");
    if (!(p->grad_eps >= 0)) return fail(LBM_ERR_INVALID_ARG, "grad_eps must be >= 0");
    if (p->init < LBM_INIT_FIELDS || p->init > LBM_INIT_JET) return fail(LBM_ERR_INVALID_ARG, "unknown init %d", p->init);
    if (p->bc == LBM_BC_JET) {
        if (!(p->inlet_D >= 0) || !std::isfinite(p->inlet_u) || !(p->noise_amp >= 0) ||
            !std::isfinite(p->inlet_cx) || !std::isfinite(p->inlet_cy) || !std::isfinite(p->inlet_D))
            return fail(LBM_ERR_INVALID_ARG, "bad inlet parameters");
        // the inlet circle must not reach the outermost rows and columns
        const double r = 0.5 * p->inlet_D;
        const int x0 = std::max(0, (int)std::floor(p->inlet_cx - r)), x1 = std::min(p->nx - 1, (int)std::ceil(p->inlet_cx + r));
        const int y0 = std::max(0, (int)std::floor(p->inlet_cy - r)), y1 = std::min(p->ny - 1, (int)std::ceil(p->inlet_cy + r));
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                const double dx = x - p->inlet_cx, dy = y - p->inlet_cy;
                if (dx * dx + dy * dy < r * r && (x == 0 || y == 0 || x == p->nx - 1 || y == p->ny - 1))
                    return fail(LBM_ERR_INVALID_ARG, "the inlet circle touches a side wall at (%d, %d)", x, y);
            }
    }
    if (p->init == LBM_INIT_DROPLET && !(p->drop_W > 0))
        return fail(LBM_ERR_INVALID_ARG, "droplet interface width must be > 0");
    return LBM_OK;
}

void fill_kp(const lbm_params* p, const float* inlet, KP* k)
{
    k->nx = p->nx;
    k->ny = p->ny;
    k->nz = p->nz;
    k->px = p->nx + 2;
    k->py = p->ny + 2;
    k->NP = (uint32_t)padded_nodes(p);
    k->plane = (uint32_t)p->nx * (uint32_t)p->ny;
    k->N = k->plane * (uint32_t)p->nz;
    // p / nx = (p * m) >> (31 + L) with L = ceil(log2 nx), m = ceil(2^(31+L) / nx):
    // exact for p < 2^31 and m < 2^32
    int L = 0;
    while ((1u << L) < (unsigned)p->nx) ++L;
    const unsigned long long two = 1ull << (31 + L);
    k->nx_mul = (uint32_t)((two + (unsigned long long)p->nx - 1) / (unsigned long long)p->nx);
    k->nx_sh = 31 + L;
    k->z0 = 0;
    k->ntx = (p->nx + STX - 1) / STX;
    const double ar = 1.0 - (1.0 - p->alpha_b) * p->rho_b0 / p->rho_r0;
    k->rho_r0 = (float)p->rho_r0;
    k->rho_b0 = (float)p->rho_b0;
    k->alpha_r = (float)ar;
    k->alpha_b = (float)p->alpha_b;
    k->dalpha = (float)(ar - p->alpha_b);
    k->a_minus_w0 = (float)(p->alpha_b - (is_q19(p) ? 1.0 / 3.0 : 8.0 / 27.0));
    k->kappa_b_m1 = (float)(27.0 * (1.0 - p->alpha_b) / 19.0 - 1.0);
    k->inv_nu_r = (float)(1.0 / p->nu_r);
    k->inv_nu_b = (float)(1.0 / p->nu_b);
    k->A = (float)p->A;
    k->beta = (float)p->beta;
    k->eps2 = (float)(p->grad_eps * p->grad_eps);
    k->gx = (float)p->g[0];
    k->gy = (float)p->g[1];
    k->gz = (float)p->g[2];
    k->inlet_cx = (float)p->inlet_cx;
    k->inlet_cy = (float)p->inlet_cy;
    k->inlet_r2 = (float)(0.25 * p->inlet_D * p->inlet_D);
    k->inlet_u = (float)p->inlet_u;
    k->noise_amp = (float)p->noise_amp;
    k->seed = p->noise_seed;
    k->t = 0;
    k->unshifted = 1;
    k->xr_tagged = 0;
    k->inlet_uz = inlet;
    k->R = nullptr;
}

template <int V>
struct IntC {
    static constexpr int value = V;
};

// the device address of the static scratch on device dev (current)
int scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_ERR_UNSUPPORTED, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev]) return LBM_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(LBM_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch[dev] = ptr;
    return LBM_OK;
}

void* scratch_of(int dev)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[dev];
}

// call f(IntC<bc>, Storage) for the handle's configuration
template <class F>
int dispatch(int bc, int storage, F&& f)
{
    if (bc == LBM_BC_PERIODIC) {
        if (storage == LBM_STORAGE_FP32) return f(IntC<LBM_BC_PERIODIC>{}, StF32{});
        if (storage == LBM_STORAGE_BF16) return f(IntC<LBM_BC_PERIODIC>{}, StBF16{});
        if (storage == LBM_STORAGE_FP16) return f(IntC<LBM_BC_PERIODIC>{}, StF16{});
        if (storage == LBM_STORAGE_BF16_EQ) return f(IntC<LBM_BC_PERIODIC>{}, StBF16Eq{});
        return f(IntC<LBM_BC_PERIODIC>{}, StF16Eq{});
    }
    if (storage == LBM_STORAGE_FP32) return f(IntC<LBM_BC_JET>{}, StF32{});
    if (storage == LBM_STORAGE_BF16) return f(IntC<LBM_BC_JET>{}, StBF16{});
    if (storage == LBM_STORAGE_FP16) return f(IntC<LBM_BC_JET>{}, StF16{});
    if (storage == LBM_STORAGE_BF16_EQ) return f(IntC<LBM_BC_JET>{}, StBF16Eq{});
    return f(IntC<LBM_BC_JET>{}, StF16Eq{});
}

bool aligned(const void* ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

// parameters for reading the current state
const StateSet& cur_set(const lbm_handle* h) { return h->cs == 2 ? h->ext : h->own[h->cs]; }

// the own set a step may write: the one not holding the current state
int free_own(const lbm_handle* h) { return h->cs == 0 ? 1 : 0; }

// parameters for reading the current state
KP read_kp(const lbm_handle* h)
{
    const StateSet& c = cur_set(h);
    KP k = h->k;
    k.t = h->t;
    k.unshifted = h->unshifted;
    k.R = c.R;
    k.Qrec = c.Q;
    k.z0 = 0;
    return k;
}

// Layout of a state snapshot (a shifted state, as a step leaves it): the
// population planes 0..26 (0..27 in the referenced 16-bit forms, whose rest
// population also uses plane 27) with the plane stride of the population
// buffers, the recolouring records R, the reference records (referenced
// forms), and the jet's outlet plane (54 floats per (x, y)); each part
// 256-byte aligned.  Returns the byte count; with base != NULL fills *s.
uint64_t snap_layout(const lbm_params* p, char* base, StateSet* s)
{
    const uint64_t NP = padded_nodes(p), plane = (uint64_t)p->nx * p->ny;
    const uint64_t planes = eq_ref(p->storage) ? Q + 1 : Q;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        char* q = base ? base + off : nullptr;
        off += align256(bytes);
        return q;
    };
    char* pop = take(planes * NP * elem_bytes(p->storage));
    char* R = take(NP * 16);
    char* Qr = eq_ref(p->storage) ? take(NP * 16) : nullptr;
    char* hist = p->bc == LBM_BC_JET ? take(2ull * Q * plane * sizeof(float)) : nullptr;
    if (s) {
        s->pop = pop;
        s->R = (float4*)R;
        s->Q = (uint4*)Qr;
        s->hist = (float*)hist;
    }
    return off;
}

// bytes of the parts of a shifted state (what a snapshot holds)
struct SnapBytes {
    size_t pop, rec, hist;
};
SnapBytes snap_bytes_of(const lbm_params* p)
{
    const uint64_t NP = padded_nodes(p), plane = (uint64_t)p->nx * p->ny;
    SnapBytes b;
    b.pop = (size_t)((eq_ref(p->storage) ? Q + 1 : Q) * NP * elem_bytes(p->storage));
    b.rec = (size_t)(NP * 16);
    b.hist = p->bc == LBM_BC_JET ? (size_t)(2ull * Q * plane * sizeof(float)) : 0;
    return b;
}

}  // namespace

extern "C" {

int lbm_query_sizes(const lbm_params* p, lbm_sizes* out)
{
    int rc = validate(p);
    if (rc != LBM_OK) return rc;
    if (!out) return fail(LBM_ERR_INVALID_ARG, "sizes is NULL");
    const uint64_t N = (uint64_t)p->nx * p->ny * p->nz;
    const uint64_t NP = padded_nodes(p);
    const uint64_t plane = (uint64_t)p->nx * p->ny;
    const uint64_t nblk = ((plane + BLOCK - 1) / BLOCK) * (uint64_t)p->nz;
    out->n_nodes = N;
    if (is_q19(p)) {
        out->pop_bytes = q19::pop_bytes(N);
        out->field_bytes = 16ull * N;
        out->hist_bytes = p->bc == LBM_BC_JET ? 2ull * 2ull * q19::Q19 * plane * sizeof(float) : 0;
        out->audit_bytes = (nblk + 1) * 5 * sizeof(double);
        out->inlet_bytes = plane * sizeof(float);
        out->adjoint_bytes = 0;
        out->state_bytes = 2ull * q19::Q19 * N * sizeof(float);
        out->snap_bytes = 0;
        return LBM_OK;
    }
    out->pop_bytes = 2ull * Q * NP * elem_bytes(p->storage);
    out->field_bytes = field_floats(p->storage) * NP * sizeof(float);
    out->hist_bytes = p->bc == LBM_BC_JET ? 2ull * 2ull * Q * plane * sizeof(float) : 0;
    out->audit_bytes = (nblk + 1) * 5 * sizeof(double);
    out->inlet_bytes = plane * sizeof(float);
    out->adjoint_bytes = adjoint_layout(NP, N, plane, nblk, nullptr, nullptr);
    out->state_bytes = 2ull * Q * N * sizeof(float);
    out->snap_bytes = snap_layout(p, nullptr, nullptr);
    return LBM_OK;
}

int lbm_init(lbm_handle** h, const lbm_params* p, const lbm_buffers* buf, const float* rho_r,
             const float* rho_b, const float* u, void* hip_stream)
{
    if (!h) return fail(LBM_ERR_INVALID_ARG, "handle pointer is NULL");
    *h = nullptr;
    int rc = validate(p);
    if (rc != LBM_OK) return rc;
    if (!buf || !buf->pop_a || !buf->pop_b || !buf->fields || !buf->audit)
        return fail(LBM_ERR_INVALID_ARG, "population, field and audit buffers are required");
    if (p->bc == LBM_BC_JET && !buf->hist) return fail(LBM_ERR_INVALID_ARG, "the jet needs the outlet history buffer");
    if (!aligned(buf->pop_a, 256) || !aligned(buf->pop_b, 256) || !aligned(buf->fields, 16) ||
        !aligned(buf->audit, 8) || (buf->hist && !aligned(buf->hist, 16)) ||
        (buf->adjoint && !aligned(buf->adjoint, 256)))
        return fail(LBM_ERR_INVALID_ARG, "misaligned buffer");
    if (buf->pop_a == buf->pop_b) return fail(LBM_ERR_INVALID_ARG, "population buffers must differ");
    if (p->init == LBM_INIT_FIELDS && (!rho_r || !rho_b))
        return fail(LBM_ERR_INVALID_ARG, "init from fields needs rho_r and rho_b");
    int dev = -1;
    HIP_CHECK(hipGetDevice(&dev));
    rc = scratch_setup(dev);
    if (rc != LBM_OK) return rc;
    lbm_handle* H = new (std::nothrow) lbm_handle();
    if (!H) return fail(LBM_ERR_INVALID_ARG, "out of host memory");
    H->p = *p;
    H->q19 = is_q19(p);
    fill_kp(p, buf->inlet_uz, &H->k);
    const size_t NP = H->k.NP;
    H->own[0].pop = buf->pop_a;
    H->own[1].pop = buf->pop_b;
    H->cs = 0;
    H->ext = StateSet{nullptr, nullptr, nullptr, nullptr};
    H->own[0].R = (float4*)buf->fields;
    H->own[1].R = (float4*)(buf->fields + 4 * NP);
    const size_t qf = eq_ref(p->storage) ? 8 * NP : 0;  // records after R, 16-byte aligned
    H->own[0].Q = eq_ref(p->storage) ? (uint4*)(buf->fields + 8 * NP) : nullptr;
    H->own[1].Q = eq_ref(p->storage) ? (uint4*)(buf->fields + 12 * NP) : nullptr;
    H->PD = (float2*)(buf->fields + 8 * NP + qf);
    H->XR = buf->fields + 10 * NP + qf;
    const size_t hplane = 2 * (size_t)Q * H->k.plane;
    H->own[0].hist = p->bc == LBM_BC_JET ? buf->hist : nullptr;
    H->own[1].hist = p->bc == LBM_BC_JET ? buf->hist + hplane : nullptr;
    H->audit = buf->audit;
    H->adjoint = buf->adjoint;
    H->stream = (hipStream_t)hip_stream;
    H->device = dev;
    H->t = 0;
    H->unshifted = 1;
    const unsigned bx = (H->k.plane + BLOCK - 1) / BLOCK;
    H->grid_all = dim3(bx, p->nz);
    H->grid_plane = dim3(bx, 1);
    H->grid_tiles = dim3((unsigned)(H->k.ntx * ((p->ny + STY - 1) / STY)), p->nz);
    H->grid_dtiles = dim3((unsigned)(H->k.ntx * ((p->ny + DTY - 1) / DTY)), p->nz);
    const uint64_t cells = 2ull * H->k.px * H->k.py + 2ull * H->k.px * p->nz + 2ull * p->ny * p->nz;
    H->ncells = (uint32_t)cells;
    H->grid_shell = dim3((unsigned)((cells + BLOCK - 1) / BLOCK));
    H->nblk = (int)(H->grid_all.x * H->grid_all.y);
    if (H->q19) {
        H->F2 = (float2*)buf->fields;
        H->PD = nullptr;
        H->XR = nullptr;
        H->own[0].R = H->own[1].R = nullptr;
        H->own[0].Q = H->own[1].Q = nullptr;
        H->own[0].hist = p->bc == LBM_BC_JET ? buf->hist : nullptr;
        H->own[1].hist = p->bc == LBM_BC_JET ? buf->hist + 2 * (size_t)q19::Q19 * H->k.plane : nullptr;
        const double ar = 1.0 - (1.0 - p->alpha_b) * p->rho_b0 / p->rho_r0;
        hipLaunchKernelGGL(q19::k19_init, H->grid_all, dim3(BLOCK), 0, H->stream, (float*)H->own[0].pop, H->k,
                           p->init, rho_r, rho_b, u, p->drop_cx, p->drop_cy, p->drop_cz, p->drop_R, p->drop_W,
                           p->rho_r0, p->rho_b0, ar, p->alpha_b);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            delete H;
            return fail(LBM_ERR_HIP, "kernel launch: %s", hipGetErrorString(e));
        }
        *h = H;
        return LBM_OK;
    }
    rc = dispatch(p->bc, p->storage, [&](auto bc, auto st) -> int {
        using S = decltype(st);
        (void)bc;
        const double ar = 1.0 - (1.0 - p->alpha_b) * p->rho_b0 / p->rho_r0;
        hipLaunchKernelGGL(k_init<S>, H->grid_all, dim3(BLOCK), 0, H->stream, (typename S::T*)H->own[0].pop, H->own[0].R, H->k,
                           p->init, rho_r, rho_b, u, p->drop_cx, p->drop_cy, p->drop_cz, p->drop_R, p->drop_W,
                           p->rho_r0, p->rho_b0, ar, p->alpha_b, (double)H->k.rho_b0);
        LAUNCH_CHECK();
        return LBM_OK;
    });
    if (rc != LBM_OK) {
        delete H;
        return rc;
    }
    *h = H;
    return LBM_OK;
}

}  // extern "C"

namespace {

// One full time step from the current state into the state set dst, which
// becomes the current state.
template <int BC>
int q19_launch(lbm_handle* h, const StateSet& dst_set, hipEvent_t* e)
{
    const KP k = read_kp(h);
    const float* src = (const float*)cur_set(h).pop;
    float* dst = (float*)dst_set.pop;
    const float* hprev = cur_set(h).hist;
    float* hcur = dst_set.hist;
    // jet: the planes below the outlet, then the outlet plane by its own kernel
    const dim3 gd = BC == LBM_BC_JET ? dim3(h->grid_all.x, (unsigned)(h->p.nz - 1)) : h->grid_all;
    if (h->unshifted)
        hipLaunchKernelGGL((q19::k19_density<true, BC>), gd, dim3(BLOCK), 0, h->stream, src, h->F2, k);
    else
        hipLaunchKernelGGL((q19::k19_density<false, BC>), gd, dim3(BLOCK), 0, h->stream, src, h->F2, k);
    LAUNCH_CHECK();
    if (BC == LBM_BC_JET) {
        if (h->unshifted)
            hipLaunchKernelGGL(q19::k19_outlet<true>, h->grid_plane, dim3(BLOCK), 0, h->stream, src, h->F2, hprev,
                               hcur, k);
        else
            hipLaunchKernelGGL(q19::k19_outlet<false>, h->grid_plane, dim3(BLOCK), 0, h->stream, src, h->F2, hprev,
                               hcur, k);
        LAUNCH_CHECK();
    }
    if (e) {
        HIP_CHECK(hipEventRecord(e[1], h->stream));
        HIP_CHECK(hipEventRecord(e[2], h->stream));
    }
    if (h->unshifted)
        hipLaunchKernelGGL((q19::k19_collide<true, BC>), h->grid_all, dim3(BLOCK), 0, h->stream, src, dst, h->F2,
                           hcur, k);
    else
        hipLaunchKernelGGL((q19::k19_collide<false, BC>), h->grid_all, dim3(BLOCK), 0, h->stream, src, dst, h->F2,
                           hcur, k);
    LAUNCH_CHECK();
    return LBM_OK;
}

int q19_step(lbm_handle* h, const StateSet& dst_set, int dst_cs)
{
    hipEvent_t* e = nullptr;
    if (h->profiling) {
        while (h->ev.size() < h->ev_used + 5) {
            hipEvent_t x;
            HIP_CHECK(hipEventCreate(&x));
            h->ev.push_back(x);
        }
        e = &h->ev[h->ev_used];
        h->ev_used += 5;
        HIP_CHECK(hipEventRecord(e[0], h->stream));
    }
    const int rc = h->p.bc == LBM_BC_JET ? q19_launch<LBM_BC_JET>(h, dst_set, e)
                                         : q19_launch<LBM_BC_PERIODIC>(h, dst_set, e);
    if (rc != LBM_OK) return rc;
    if (e) {
        HIP_CHECK(hipEventRecord(e[3], h->stream));
        HIP_CHECK(hipEventRecord(e[4], h->stream));
    }
    h->cs = dst_cs;
    h->t += 1;
    h->unshifted = 0;
    return LBM_OK;
}

int step_once(lbm_handle* h, const StateSet& dst_set, int dst_cs)
{
    if (h->q19) return q19_step(h, dst_set, dst_cs);
    return dispatch(h->p.bc, h->p.storage, [&](auto bc, auto st) -> int {
        using S = decltype(st);
        using T = typename S::T;
        constexpr int BC = decltype(bc)::value;
        constexpr bool jet = BC == LBM_BC_JET;
        const StateSet& cur = cur_set(h);
        KP k = read_kp(h);
        const T* src = (const T*)cur.pop;
        T* dst = (T*)dst_set.pop;
        float4* Rout = dst_set.R;
        uint4* Qout = dst_set.Q;
        float* hprev = cur.hist;
        float* hcur = dst_set.hist;
        hipEvent_t* e = nullptr;
        if (h->profiling) {
            while (h->ev.size() < h->ev_used + 5) {
                hipEvent_t x;
                HIP_CHECK(hipEventCreate(&x));
                h->ev.push_back(x);
            }
            e = &h->ev[h->ev_used];
            h->ev_used += 5;
            HIP_CHECK(hipEventRecord(e[0], h->stream));
        }
        // density pass (jet: the outlet plane by the convective condition)
        if (jet) {
            const dim3 gi(h->grid_dtiles.x, (unsigned)(h->p.nz - 1));
            const dim3 go((unsigned)((h->k.plane + OBLOCK - 1) / OBLOCK));
            hipLaunchKernelGGL((k_density<BC, S>), gi, dim3(DBLOCK), 0, h->stream, src, h->PD, h->XR, k,
                               (float*)nullptr);
            LAUNCH_CHECK();
            hipLaunchKernelGGL((k_outlet_density<S>), go, dim3(OBLOCK), 0, h->stream, src, h->PD, h->XR, hprev,
                               hcur, k, (float*)nullptr);
        } else {
            hipLaunchKernelGGL((k_density<BC, S>), h->grid_dtiles, dim3(DBLOCK), 0, h->stream, src, h->PD, h->XR,
                               k, (float*)nullptr);
        }
        LAUNCH_CHECK();
        if (e) HIP_CHECK(hipEventRecord(e[1], h->stream));
        if (!kDensityGhosts<S>) {  // FP32: the density kernels fill the field ghost shell
            hipLaunchKernelGGL(k_field_ghosts<BC>, h->grid_shell, dim3(BLOCK), 0, h->stream, h->PD, k, h->ncells);
            LAUNCH_CHECK();
        }
        if (e) HIP_CHECK(hipEventRecord(e[2], h->stream));
        // fused collide-perturb-recolour-stream
        hipLaunchKernelGGL((k_collide<BC, S>), h->grid_tiles, dim3(BLOCK), 0, h->stream, src, dst, h->PD, h->XR,
                           hcur, Rout, Qout, k);
        LAUNCH_CHECK();
        if (e) HIP_CHECK(hipEventRecord(e[3], h->stream));
        hipLaunchKernelGGL((k_pop_ghosts<BC, S>), dim3((h->ncells + GBLOCK - 1) / GBLOCK), dim3(GBLOCK), 0,
                           h->stream, dst, Rout, Qout, k, h->ncells);
        LAUNCH_CHECK();
        if (e) HIP_CHECK(hipEventRecord(e[4], h->stream));
        if (dst_cs == 2) h->ext = dst_set;
        h->cs = dst_cs;
        h->t += 1;
        h->unshifted = 0;
        return LBM_OK;
    });
}

// the snapshot at snap, checked for alignment
int snap_set(const lbm_handle* h, const void* snap, StateSet* s)
{
    if (!snap) return fail(LBM_ERR_INVALID_ARG, "snapshot pointer is NULL");
    if (!aligned(snap, 256)) return fail(LBM_ERR_INVALID_ARG, "snapshot must be 256-byte aligned");
    snap_layout(&h->p, (char*)snap, s);
    return LBM_OK;
}

// copy the shifted state src into dst (device to device, on the stream)
int copy_state(const lbm_handle* h, const StateSet& dst, const StateSet& src)
{
    const SnapBytes b = snap_bytes_of(&h->p);
    if (dst.pop != src.pop) HIP_CHECK(hipMemcpyAsync(dst.pop, src.pop, b.pop, hipMemcpyDeviceToDevice, h->stream));
    if (dst.R != src.R) HIP_CHECK(hipMemcpyAsync(dst.R, src.R, b.rec, hipMemcpyDeviceToDevice, h->stream));
    if (src.Q && dst.Q != src.Q)
        HIP_CHECK(hipMemcpyAsync(dst.Q, src.Q, b.rec, hipMemcpyDeviceToDevice, h->stream));
    if (b.hist && dst.hist != src.hist)
        HIP_CHECK(hipMemcpyAsync(dst.hist, src.hist, b.hist, hipMemcpyDeviceToDevice, h->stream));
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_step(lbm_handle* h, int32_t n_steps)
{
    if (!h) return fail(LBM_ERR_STATE, "handle is NULL");
    if (n_steps < 0) return fail(LBM_ERR_INVALID_ARG, "n_steps < 0");
    for (int s = 0; s < n_steps; ++s) {
        const int d = free_own(h);
        const int rc = step_once(h, h->own[d], d);
        if (rc != LBM_OK) return rc;
    }
    return LBM_OK;
}

int lbm_step_into(lbm_handle* h, void* snap)
{
    if (!h) return fail(LBM_ERR_STATE, "handle is NULL");
    if (h->q19) return fail(LBM_ERR_UNSUPPORTED, "snapshots need the D3Q27 lattice");
    StateSet s;
    int rc = snap_set(h, snap, &s);
    if (rc != LBM_OK) return rc;
    const StateSet& c = cur_set(h);
    if (s.pop == c.pop) return fail(LBM_ERR_INVALID_ARG, "the snapshot holds the current state");
    return step_once(h, s, 2);
}

int lbm_snapshot_save(lbm_handle* h, void* snap)
{
    if (!h) return fail(LBM_ERR_STATE, "handle is NULL");
    if (h->q19) return fail(LBM_ERR_UNSUPPORTED, "snapshots need the D3Q27 lattice");
    if (h->unshifted) return fail(LBM_ERR_STATE, "the current state is a general state (after init or set_state)");
    StateSet s;
    int rc = snap_set(h, snap, &s);
    if (rc != LBM_OK) return rc;
    return copy_state(h, s, cur_set(h));
}

int lbm_snapshot_load(lbm_handle* h, const void* snap, int64_t t)
{
    if (!h) return fail(LBM_ERR_STATE, "handle is NULL");
    if (h->q19) return fail(LBM_ERR_UNSUPPORTED, "snapshots need the D3Q27 lattice");
    if (t < 0) return fail(LBM_ERR_INVALID_ARG, "t < 0");
    StateSet s;
    int rc = snap_set(h, snap, &s);
    if (rc != LBM_OK) return rc;
    const int d = h->cs == 2 ? 0 : h->cs;
    rc = copy_state(h, h->own[d], s);
    if (rc != LBM_OK) return rc;
    h->cs = d;
    h->t = t;
    h->unshifted = 0;
    return LBM_OK;
}

int lbm_macroscopic(lbm_handle* h, float* rho_r, float* rho_b, float* u, float* phi, double* audit)
{
    if (!h) return fail(LBM_ERR_STATE, "handle is NULL");
    const KP k = read_kp(h);
    int rc = h->q19 ? [&]() -> int {
        const float* pop = (const float*)cur_set(h).pop;
        const float* hist = cur_set(h).hist;
        double* part = audit ? h->audit : nullptr;
        const bool jet = h->p.bc == LBM_BC_JET;
        if (h->unshifted)
            hipLaunchKernelGGL((q19::k19_macro<true, LBM_BC_PERIODIC>), h->grid_all, dim3(BLOCK), 0, h->stream, pop,
                               hist, k, rho_r, rho_b, u, phi, part);
        else if (jet)
            hipLaunchKernelGGL((q19::k19_macro<false, LBM_BC_JET>), h->grid_all, dim3(BLOCK), 0, h->stream, pop, hist,
                               k, rho_r, rho_b, u, phi, part);
        else
            hipLaunchKernelGGL((q19::k19_macro<false, LBM_BC_PERIODIC>), h->grid_all, dim3(BLOCK), 0, h->stream, pop,
                               hist, k, rho_r, rho_b, u, phi, part);
        LAUNCH_CHECK();
        return LBM_OK;
    }() : dispatch(h->p.bc, h->p.storage, [&](auto bc, auto st) -> int {
        using S = decltype(st);
        constexpr int BC = decltype(bc)::value;
        hipLaunchKernelGGL((k_macro<BC, S>), h->grid_all, dim3(BLOCK), 0, h->stream,
                           (const typename S::T*)cur_set(h).pop, cur_set(h).hist, k, rho_r, rho_b, u, phi,
                           audit ? h->audit : nullptr);
        LAUNCH_CHECK();
        return LBM_OK;
    });
    if (rc != LBM_OK || !audit) return rc;
    double* tot = h->audit + (size_t)h->nblk * 5;
    hipLaunchKernelGGL(k_audit_final, dim3(1), dim3(BLOCK), 0, h->stream, h->audit, h->nblk, tot);
    LAUNCH_CHECK();
    HIP_CHECK(hipMemcpyAsync(audit, tot, 5 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_CHECK(hipStreamSynchronize(h->stream));
    for (int a = 0; a < 5; ++a)
        if (!std::isfinite(audit[a])) return fail(LBM_ERR_NONFINITE, "audit total %d is not finite", a);
    return LBM_OK;
}

int lbm_get_state(lbm_handle* h, float* state)
{
    if (!h) return fail(LBM_ERR_STATE, "handle is NULL");
    if (!state) return fail(LBM_ERR_INVALID_ARG, "state is NULL");
    const KP k = read_kp(h);
    if (h->q19) {
        const float* pop = (const float*)cur_set(h).pop;
        const float* hist = cur_set(h).hist;
        if (h->unshifted)
            hipLaunchKernelGGL((q19::k19_get_state<true, LBM_BC_PERIODIC>), h->grid_all, dim3(BLOCK), 0, h->stream,
                               pop, hist, k, state);
        else if (h->p.bc == LBM_BC_JET)
            hipLaunchKernelGGL((q19::k19_get_state<false, LBM_BC_JET>), h->grid_all, dim3(BLOCK), 0, h->stream, pop,
                               hist, k, state);
        else
            hipLaunchKernelGGL((q19::k19_get_state<false, LBM_BC_PERIODIC>), h->grid_all, dim3(BLOCK), 0, h->stream,
                               pop, hist, k, state);
        LAUNCH_CHECK();
        return LBM_OK;
    }
    return dispatch(h->p.bc, h->p.storage, [&](auto bc, auto st) -> int {
        using S = decltype(st);
        constexpr int BC = decltype(bc)::value;
        hipLaunchKernelGGL((k_get_state<BC, S>), h->grid_all, dim3(BLOCK), 0, h->stream,
                           (const typename S::T*)cur_set(h).pop, cur_set(h).hist, k, state, (double)h->k.rho_b0);
        LAUNCH_CHECK();
        return LBM_OK;
    });
}

int lbm_set_state(lbm_handle* h, const float* state, int64_t t)
{
    if (!h) return fail(LBM_ERR_STATE, "handle is NULL");
    if (!state) return fail(LBM_ERR_INVALID_ARG, "state is NULL");
    if (t < 0) return fail(LBM_ERR_INVALID_ARG, "t < 0");
    // the general state goes into an own set (a current snapshot is not overwritten)
    const int d = h->cs == 2 ? 0 : h->cs;
    const KP k = read_kp(h);
    if (h->q19) {
        hipLaunchKernelGGL(q19::k19_set_state, h->grid_all, dim3(BLOCK), 0, h->stream, (float*)h->own[d].pop, k,
                           state);
        LAUNCH_CHECK();
        h->cs = d;
        h->t = t;
        h->unshifted = 1;
        return LBM_OK;
    }
    int rc = dispatch(h->p.bc, h->p.storage, [&](auto bc, auto st) -> int {
        using S = decltype(st);
        (void)bc;
        hipLaunchKernelGGL(k_set_state<S>, h->grid_all, dim3(BLOCK), 0, h->stream, (typename S::T*)h->own[d].pop,
                           h->own[d].R, k, state, (double)h->k.rho_b0);
        LAUNCH_CHECK();
        return LBM_OK;
    });
    if (rc != LBM_OK) return rc;
    h->cs = d;
    h->t = t;
    h->unshifted = 1;
    return LBM_OK;
}

int64_t lbm_time(const lbm_handle* h) { return h ? (int64_t)h->t : -1; }

}  // extern "C"

namespace {

// Passes 2-6 of the adjoint step (see lbm_adjoint.h) after pass 1 has written
// PD, XR and the raw moments of x_t; htop/hs/dfr give the outlet plane of x_t.
template <int BC>
int adjoint_rest(lbm_handle* h, const KP& k, const AdjWork& w, const float* htop, size_t hs, int dfr,
                 const float* lambda_in, float* lambda_out, double* dJ_dA, float* dJ_du_in)
{
    hipLaunchKernelGGL(k_field_ghosts<BC>, h->grid_shell, dim3(BLOCK), 0, h->stream, h->PD, k, h->ncells);
    LAUNCH_CHECK();
    if (BC == LBM_BC_JET) {
        KP kt = k;
        kt.z0 = h->p.nz - 3;
        hipLaunchKernelGGL(k_adj_top_post, dim3(h->grid_all.x, 3), dim3(BLOCK), 0, h->stream, w.MOM, h->PD, h->XR,
                           w.PS, kt);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_adj_outlet, h->grid_plane, dim3(BLOCK), 0, h->stream, htop, hs, dfr, lambda_in, w.PS,
                           w.ML, w.DL, k);
        LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_adj_node<BC>, h->grid_all, dim3(BLOCK), 0, h->stream, w.MOM, lambda_in, w.ML, h->PD, h->XR,
                       w.LC, w.AG0, w.AG1, w.AP, k);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_adj_ghosts<BC>, h->grid_shell, dim3(BLOCK), 0, h->stream, w.AG0, w.AG1, w.GH, k, h->ncells);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_adj_fields<BC>, h->grid_tiles, dim3(BLOCK), 0, h->stream, w.AG0, w.AG1, w.GH, h->PD, h->XR,
                       w.DL, w.LC, lambda_out, k);
    LAUNCH_CHECK();
    if (BC == LBM_BC_JET && dJ_du_in) {
        hipLaunchKernelGGL(k_adj_inlet, h->grid_plane, dim3(BLOCK), 0, h->stream, lambda_in, dJ_du_in, k);
        LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_adj_sumA, dim3(1), dim3(SUM_BLOCK), 0, h->stream, w.AP, h->nblk, dJ_dA);
    LAUNCH_CHECK();
    return LBM_OK;
}

int adjoint_args(lbm_handle* h, const void* state_t, int64_t t, const float* lambda_in, float* lambda_out,
                 double* dJ_dA)
{
    if (!h) return fail(LBM_ERR_STATE, "handle is NULL");
    if (h->q19) return fail(LBM_ERR_UNSUPPORTED, "the adjoint step needs the D3Q27 lattice");
    if (!h->adjoint) return fail(LBM_ERR_STATE, "no adjoint work buffer was given to lbm_init");
    if (!state_t || !lambda_in || !lambda_out || !dJ_dA)
        return fail(LBM_ERR_INVALID_ARG, "state_t, lambda_in, lambda_out and dJ_dA are required");
    if (lambda_out == lambda_in || (const void*)lambda_out == state_t)
        return fail(LBM_ERR_INVALID_ARG, "lambda_out must not alias lambda_in or state_t");
    if (t < 0) return fail(LBM_ERR_INVALID_ARG, "t < 0");
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_adjoint_step(lbm_handle* h, const float* state_t, int64_t t, const float* lambda_in, float* lambda_out,
                     double* dJ_dA, float* dJ_du_in)
{
    int rc = adjoint_args(h, state_t, t, lambda_in, lambda_out, dJ_dA);
    if (rc != LBM_OK) return rc;
    AdjWork w;
    adjoint_layout(h->k.NP, h->k.N, h->k.plane, (uint64_t)h->nblk, (char*)h->adjoint, &w);
    KP k = h->k;
    k.t = t;
    k.unshifted = 1;
    k.z0 = 0;
    k.R = nullptr;
    hipLaunchKernelGGL(k_adj_density, h->grid_all, dim3(BLOCK), 0, h->stream, state_t, h->PD, h->XR, w.MOM, k);
    LAUNCH_CHECK();
    const float* top = state_t + (size_t)(h->p.nz - 1) * h->k.plane;
    if (h->p.bc == LBM_BC_PERIODIC)
        return adjoint_rest<LBM_BC_PERIODIC>(h, k, w, top, h->k.N, 0, lambda_in, lambda_out, dJ_dA, dJ_du_in);
    return adjoint_rest<LBM_BC_JET>(h, k, w, top, h->k.N, 0, lambda_in, lambda_out, dJ_dA, dJ_du_in);
}

int lbm_adjoint_step_snapshot(lbm_handle* h, const void* snap_t, int64_t t, const float* lambda_in,
                              float* lambda_out, double* dJ_dA, float* dJ_du_in)
{
    int rc = adjoint_args(h, snap_t, t, lambda_in, lambda_out, dJ_dA);
    if (rc != LBM_OK) return rc;
    StateSet s;
    rc = snap_set(h, snap_t, &s);
    if (rc != LBM_OK) return rc;
    AdjWork w;
    adjoint_layout(h->k.NP, h->k.N, h->k.plane, (uint64_t)h->nblk, (char*)h->adjoint, &w);
    KP k = h->k;
    k.t = t;
    k.unshifted = 0;
    k.z0 = 0;
    k.R = s.R;
    k.Qrec = s.Q;
    k.xr_tagged = 1;
    // pass 1 from the snapshot: the forward density pass (pulled deviations,
    // (phi, rho), tagged colour fraction) plus the raw moments
    rc = dispatch(h->p.bc, h->p.storage, [&](auto bc, auto st) -> int {
        using S = decltype(st);
        constexpr int BC = decltype(bc)::value;
        const typename S::T* src = (const typename S::T*)s.pop;
        if (BC == LBM_BC_JET) {
            const dim3 gi(h->grid_dtiles.x, (unsigned)(h->p.nz - 1));
            const dim3 go((unsigned)((h->k.plane + OBLOCK - 1) / OBLOCK));
            hipLaunchKernelGGL((k_density<BC, S, true>), gi, dim3(DBLOCK), 0, h->stream, src, h->PD, h->XR, k, w.MOM);
            LAUNCH_CHECK();
            hipLaunchKernelGGL((k_outlet_density<S>), go, dim3(OBLOCK), 0, h->stream, src, h->PD, h->XR, s.hist,
                               w.ST, k, w.MOM);
        } else {
            hipLaunchKernelGGL((k_density<BC, S, true>), h->grid_dtiles, dim3(DBLOCK), 0, h->stream, src, h->PD,
                               h->XR, k, w.MOM);
        }
        LAUNCH_CHECK();
        return LBM_OK;
    });
    if (rc != LBM_OK) return rc;
    if (h->p.bc == LBM_BC_PERIODIC)
        return adjoint_rest<LBM_BC_PERIODIC>(h, k, w, w.ST, h->k.plane, 1, lambda_in, lambda_out, dJ_dA, dJ_du_in);
    return adjoint_rest<LBM_BC_JET>(h, k, w, w.ST, h->k.plane, 1, lambda_in, lambda_out, dJ_dA, dJ_du_in);
}

int lbm_profile(lbm_handle* h, int enable)
{
    if (!h) return fail(LBM_ERR_STATE, "handle is NULL");
    h->profiling = enable != 0;
    return LBM_OK;
}

int lbm_profile_read(lbm_handle* h, double* ms, int64_t* launches)
{
    if (!h) return fail(LBM_ERR_STATE, "handle is NULL");
    if (!ms || !launches) return fail(LBM_ERR_INVALID_ARG, "output pointers are NULL");
    ms[0] = ms[1] = ms[2] = 0.0;
    launches[0] = launches[1] = launches[2] = 0;
    if (h->ev_used) HIP_CHECK(hipEventSynchronize(h->ev[h->ev_used - 1]));
    for (size_t i = 0; i + 5 <= h->ev_used; i += 5) {
        float a = 0.f, b = 0.f, c = 0.f, d = 0.f;
        HIP_CHECK(hipEventElapsedTime(&a, h->ev[i], h->ev[i + 1]));
        HIP_CHECK(hipEventElapsedTime(&b, h->ev[i + 1], h->ev[i + 2]));
        HIP_CHECK(hipEventElapsedTime(&c, h->ev[i + 2], h->ev[i + 3]));
        HIP_CHECK(hipEventElapsedTime(&d, h->ev[i + 3], h->ev[i + 4]));
        ms[0] += a;
        ms[1] += c;
        ms[2] += b + d;
        launches[0] += 1;
        launches[1] += 1;
        launches[2] += 1;
    }
    h->ev_used = 0;
    return LBM_OK;
}

int lbm_destroy(lbm_handle* h)
{
    if (h)
        for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    delete h;
    return LBM_OK;
}

int lbm_diag_bytes(const lbm_params* p, uint64_t* bytes)
{
    if (!bytes) return fail(LBM_ERR_INVALID_ARG, "bytes is NULL");
    const int rc = validate(p);
    if (rc != LBM_OK) return rc;
    *bytes = diag_bytes((uint64_t)p->nx * p->ny * p->nz);
    return LBM_OK;
}

}  // extern "C"

namespace {

// the diagnostics kernels on work memory w of the handle's lattice; copies the
// statistics and the first min(cap, n_fragments) volumes to the host
int diag_run(lbm_handle* h, void* work, lbm_jet_stats* stats, int64_t* volumes, int64_t cap)
{
    const KP k = read_kp(h);
    const DiagWork w = diag_layout(work, k.N);
    int rc = dispatch(h->p.bc, h->p.storage, [&](auto bc, auto st) -> int {
        using S = decltype(st);
        constexpr int BC = decltype(bc)::value;
        hipLaunchKernelGGL(k_diag_clear, dim3(1), dim3(64), 0, h->stream, w);
        LAUNCH_CHECK();
        const float* hist = cur_set(h).hist;
        if (!h->q19)
            hipLaunchKernelGGL((k_diag_init<BC, S>), h->grid_all, dim3(BLOCK), 0, h->stream,
                               (const typename S::T*)cur_set(h).pop, hist, k, w);
        else if (h->unshifted)
            hipLaunchKernelGGL((q19::k19_diag_init<true, BC>), h->grid_all, dim3(BLOCK), 0, h->stream,
                               (const float*)cur_set(h).pop, hist, k, w);
        else
            hipLaunchKernelGGL((q19::k19_diag_init<false, BC>), h->grid_all, dim3(BLOCK), 0, h->stream,
                               (const float*)cur_set(h).pop, hist, k, w);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_diag_merge, h->grid_all, dim3(BLOCK), 0, h->stream, k, w);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_diag_flatten, h->grid_all, dim3(BLOCK), 0, h->stream, k, w);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_diag_count, h->grid_all, dim3(BLOCK), 0, h->stream, k, w);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_diag_collect, h->grid_all, dim3(BLOCK), 0, h->stream, k, w);
        LAUNCH_CHECK();
        return LBM_OK;
    });
    if (rc != LBM_OK) return rc;
    DiagHeader hd;
    HIP_CHECK(hipMemcpyAsync(&hd, w.hdr, sizeof(hd), hipMemcpyDeviceToHost, h->stream));
    HIP_CHECK(hipStreamSynchronize(h->stream));
    if (hd.overflow) return fail(LBM_ERR_HIP, "connected-component walk exceeded its bound");
    stats->jet_nodes = (int64_t)hd.jet_nodes;
    stats->front_z = hd.front_z;
    stats->column_volume = (int64_t)hd.column_volume;
    stats->n_fragments = hd.n_fragments;
    const int64_t n = std::min<int64_t>(cap, (int64_t)hd.n_fragments);
    if (n > 0) {
        long long* wide = (long long*)w.label;  // 8 N bytes: labels and counts, free after the collection
        hipLaunchKernelGGL(k_diag_widen, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, h->stream, w,
                           (uint32_t)n, wide);
        LAUNCH_CHECK();
        HIP_CHECK(hipMemcpyAsync(volumes, wide, (size_t)n * sizeof(long long), hipMemcpyDeviceToHost, h->stream));
        HIP_CHECK(hipStreamSynchronize(h->stream));
    }
    return LBM_OK;
}

int diag_args(lbm_handle* h, lbm_jet_stats* stats, int64_t* volumes, int64_t cap)
{
    if (!h) return fail(LBM_ERR_STATE, "handle is NULL");
    if (!stats) return fail(LBM_ERR_INVALID_ARG, "stats is required");
    if (cap < 0 || (cap > 0 && !volumes)) return fail(LBM_ERR_INVALID_ARG, "volumes is NULL with cap > 0");
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_jet_diagnostics(lbm_handle* h, void* work, lbm_jet_stats* stats, int64_t* volumes, int64_t cap)
{
    const int rc = diag_args(h, stats, volumes, cap);
    if (rc != LBM_OK) return rc;
    if (!work) return fail(LBM_ERR_INVALID_ARG, "work is required");
    if (!aligned(work, 256)) return fail(LBM_ERR_INVALID_ARG, "work must be 256-byte aligned");
    return diag_run(h, work, stats, volumes, cap);
}

int lbm_jet_diagnostics_static(lbm_handle* h, lbm_jet_stats* stats, int64_t* volumes, int64_t cap)
{
    const int rc = diag_args(h, stats, volumes, cap);
    if (rc != LBM_OK) return rc;
    if ((uint64_t)h->k.N > kStaticDiagNodes)
        return fail(LBM_ERR_UNSUPPORTED, "%u nodes exceed the %llu nodes of the static diagnostics scratch", h->k.N,
                    (unsigned long long)kStaticDiagNodes);
    void* ptr = scratch_of(h->device);
    if (!ptr) return fail(LBM_ERR_STATE, "no scratch address for device %d", h->device);
    return diag_run(h, ptr, stats, volumes, cap);
}

const char* lbm_status_string(int status)
{
    switch (status) {
    case LBM_OK: return "LBM_OK";
    case LBM_ERR_INVALID_ARG: return "LBM_ERR_INVALID_ARG: invalid argument";
    case LBM_ERR_UNSUPPORTED: return "LBM_ERR_UNSUPPORTED: not implemented by this library";
    case LBM_ERR_HIP: return "LBM_ERR_HIP: HIP runtime error";
    case LBM_ERR_NONFINITE: return "LBM_ERR_NONFINITE: non-finite audit total";
    case LBM_ERR_STATE: return "LBM_ERR_STATE: call out of order";
    default: return "unknown status";
    }
}

const char* lbm_last_error(void) { return g_err; }

}  // extern "C"
