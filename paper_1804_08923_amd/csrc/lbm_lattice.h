// Device-side lattice constants of the D3Q27 velocity set, in the order of the
// paper's Eq. velVec.  Loops over directions are fully unrolled, so every
// access below folds to an immediate.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cglbm {

constexpr int Q = 27;

constexpr int kCX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1,
                        1, -1, 1, -1, 1, -1, -1, 1};
constexpr int kCY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 1, -1, 1, -1, 0, 0, 0, 0,
                        1, -1, 1, -1, -1, 1, 1, -1};
constexpr int kCZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                        1, -1, -1, 1, 1, -1, 1, -1};

__host__ __device__ constexpr int csq(int i) { return kCX[i] * kCX[i] + kCY[i] * kCY[i] + kCZ[i] * kCZ[i]; }

// D3Q27 weights by |c|^2 = 0, 1, 2, 3
__host__ __device__ constexpr float wgt(int i)
{
    return csq(i) == 0 ? 8.0f / 27.0f : csq(i) == 1 ? 2.0f / 27.0f : csq(i) == 2 ? 1.0f / 54.0f : 1.0f / 216.0f;
}

__host__ __device__ constexpr double wgtd(int i)
{
    return csq(i) == 0 ? 8.0 / 27.0 : csq(i) == 1 ? 2.0 / 27.0 : csq(i) == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
}

// 1/|c_i| for i >= 1 (unused for i = 0)
__host__ __device__ constexpr float inv_len(int i)
{
    return csq(i) == 1 ? 1.0f : csq(i) == 2 ? 0.70710678118654752f : 0.57735026918962576f;
}

// index of the direction (cx, cy, cz)
__host__ __device__ constexpr int dir_of(int cx, int cy, int cz)
{
    int r = -1;
    for (int i = 0; i < Q; ++i)
        if (kCX[i] == cx && kCY[i] == cy && kCZ[i] == cz) r = i;
    return r;
}

// direction i with the components selected by mask m (bit 0: x, 1: y, 2: z) negated
__host__ __device__ constexpr int mirror_dir(int i, int m)
{
    return dir_of((m & 1) ? -kCX[i] : kCX[i], (m & 2) ? -kCY[i] : kCY[i], (m & 4) ? -kCZ[i] : kCZ[i]);
}

}  // namespace cglbm
