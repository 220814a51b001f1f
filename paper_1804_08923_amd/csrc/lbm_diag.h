// Jet diagnostics of Sec. IV C on the current state: the leading edge of the
// jet phase and its fragments.  The paper's fragment procedure: binarise the
// order parameter (1 for the jet phase, 0 elsewhere), take the connected
// components as fragments, measure each one's volume V and convert it to the
// equivalent spherical diameter d = (6 V / pi)^(1/3); the continuous column
// attached to the nozzle is left out.
//
// Readings: the jet phase is phi > 0 (Eq. order); components are face-
// connected (6-neighbourhood) on the lattice without wrap-around; V counts
// nodes (lattice cells of volume 1); the column is every component with a node
// on the inlet plane z = 0; the leading edge is the largest z of a jet node.
//
// Connected components by lock-free union-find over node indices (the label of
// a node is a parent pointer; every union hangs the larger of two roots under
// the smaller with an atomic minimum, so parents always have smaller indices
// and every find terminates): init, merge with the -x, -y, -z neighbours,
// flatten, count per root, collect the roots.
#pragma once

#include "lbm_kernels.h"

namespace cglbm {

// device work buffer: header, then labels, counts, column marks, compacted
// fragment volumes (each N int32)
struct DiagHeader {
    unsigned long long jet_nodes;
    unsigned long long column_volume;
    unsigned int n_fragments;
    int front_z;
    int overflow;  // a union-find loop hit its iteration bound (never expected)
    int pad[9];
};
static_assert(sizeof(DiagHeader) == 64, "diagnostics header layout");

struct DiagWork {
    DiagHeader* hdr;
    int* label;
    int* count;
    int* column;
    int* volume;
};

constexpr uint64_t diag_bytes(uint64_t N) { return 256 + 4 * 4 * N; }

inline DiagWork diag_layout(void* base, uint64_t N)
{
    char* p = (char*)base;
    DiagWork w;
    w.hdr = (DiagHeader*)p;
    w.label = (int*)(p + 256);
    w.count = w.label + N;
    w.column = w.count + N;
    w.volume = w.column + N;
    return w;
}

// Every union-find walk strictly decreases a node index, so it ends within N
// steps; the loops carry that bound (walk) only as a guard against a defect.

__device__ __forceinline__ int diag_load(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int diag_find(const int* __restrict__ L, int x, int walk, int* overflow)
{
    for (int it = 0; it <= walk; ++it) {
        const int p = diag_load(L + x);
        if (p == x) return x;
        x = p;
    }
    *overflow = 1;
    return x;
}

__device__ __forceinline__ void diag_unite(int* __restrict__ L, int a, int b, int walk, int* overflow)
{
    for (int it = 0; it <= walk; ++it) {
        a = diag_find(L, a, walk, overflow);
        b = diag_find(L, b, walk, overflow);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicMin(L + a, b);  // hang root a under b
        if (old == a) return;
        a = old;  // a was hung elsewhere meanwhile: continue from its parent
    }
    *overflow = 1;
}

__device__ __forceinline__ int wave_max_int(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

__global__ void k_diag_clear(DiagWork w)
{
    if (threadIdx.x == 0) {
        w.hdr->jet_nodes = 0;
        w.hdr->column_volume = 0;
        w.hdr->n_fragments = 0;
        w.hdr->front_z = -1;
        w.hdr->overflow = 0;
    }
}

// 1. order parameter of the current state, binarised; labels, counters
template <int BC, class S>
__global__ __launch_bounds__(BLOCK) void k_diag_init(const typename S::T* __restrict__ src,
                                                      const float* __restrict__ hprev, KP k, DiagWork w)
{
    const Node nd = this_node(k);
    bool fg = false;
    if (nd.valid) {
        const uint32_t i = (uint32_t)nd.z * k.plane + nd.q;
        float d[Q], fr[Q], fb[Q];
        read_state<BC, S>(src, k, hprev, nd, d, fr, fb);
        double rr = 0.0, rb = 0.0;
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            rr += (double)fr[j];
            rb += (double)fb[j];
        }
        const double a = rr / k.rho_r0, b = rb / k.rho_b0;
        fg = (float)((a - b) / (a + b)) > 0.f;  // phi as lbm_macroscopic returns it
        w.label[i] = fg ? (int)i : -1;
        w.count[i] = 0;
        w.column[i] = 0;
    }
    const unsigned long long m = __ballot(fg);
    const int zmax = wave_max_int(fg ? nd.z : -1);
    if ((threadIdx.x & 63) == 0 && m) {
        atomicAdd(&w.hdr->jet_nodes, (unsigned long long)__popcll(m));
        atomicMax(&w.hdr->front_z, zmax);
    }
}

// 2. union with the face neighbours at -x, -y, -z
__global__ __launch_bounds__(BLOCK) void k_diag_merge(KP k, DiagWork w)
{
    const Node nd = this_node(k);
    if (!nd.valid) return;
    const int i = (int)((uint32_t)nd.z * k.plane + nd.q);
    if (diag_load(w.label + i) < 0) return;
    const int walk = (int)k.N;
    if (nd.x > 0 && w.label[i - 1] >= 0) diag_unite(w.label, i, i - 1, walk, &w.hdr->overflow);
    if (nd.y > 0 && w.label[i - k.nx] >= 0) diag_unite(w.label, i, i - k.nx, walk, &w.hdr->overflow);
    if (nd.z > 0 && w.label[i - (int)k.plane] >= 0)
        diag_unite(w.label, i, i - (int)k.plane, walk, &w.hdr->overflow);
}

// 3. every jet node points at its root
__global__ __launch_bounds__(BLOCK) void k_diag_flatten(KP k, DiagWork w)
{
    const Node nd = this_node(k);
    if (!nd.valid) return;
    const int i = (int)((uint32_t)nd.z * k.plane + nd.q);
    if (w.label[i] < 0) return;
    w.label[i] = diag_find(w.label, i, (int)k.N, &w.hdr->overflow);
}

// 4. volumes per root; roots of components with a node on z = 0
__global__ __launch_bounds__(BLOCK) void k_diag_count(KP k, DiagWork w)
{
    const Node nd = this_node(k);
    if (!nd.valid) return;
    const int i = (int)((uint32_t)nd.z * k.plane + nd.q);
    const int r = w.label[i];
    if (r < 0) return;
    atomicAdd(w.count + r, 1);
    if (nd.z == 0) w.column[r] = 1;
}

// 5. the column volume and the list of fragment volumes
__global__ __launch_bounds__(BLOCK) void k_diag_collect(KP k, DiagWork w)
{
    const Node nd = this_node(k);
    if (!nd.valid) return;
    const int i = (int)((uint32_t)nd.z * k.plane + nd.q);
    if (w.label[i] != i) return;
    if (w.column[i]) {
        atomicAdd(&w.hdr->column_volume, (unsigned long long)w.count[i]);
    } else {
        const unsigned int slot = atomicAdd(&w.hdr->n_fragments, 1u);
        w.volume[slot] = w.count[i];
    }
}

// 6. the first n fragment volumes widened to int64 into out (the label and
// count arrays, free once the volumes are collected), for the host copy
__global__ __launch_bounds__(BLOCK) void k_diag_widen(DiagWork w, uint32_t n, long long* __restrict__ out)
{
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) out[i] = (long long)w.volume[i];
}

}  // namespace cglbm
