// Shared machinery of the neighbour loops (density and force kernels).
//
// One wave64 per receiving cell, one receiver per lane. For every task the
// source cell's particles are loaded one per lane, moved into the receiving
// cell's frame with the task's FP32 offset, and culled against the bounding
// box of the receivers that need work, expanded by the search radius. The
// survivors are appended (ballot + prefix count) to a candidate buffer in LDS.
// When the buffer is full (and at the end) every lane tests every buffered
// candidate against its own radius, appending the accepted slots to its own
// list in LDS; the pair arithmetic then runs from those lists, so lanes only
// spend pair arithmetic on actual neighbours.
//
// Each receiver visits its neighbours in a fixed order (task order, then
// source order), so results do not depend on scheduling.
#pragma once

#include "kernel_shapes.h"
#include "sphx_internal.h"

namespace sphx {

// Candidate buffer slots per flush and per-lane list capacity (8-bit slots).
// Each lane's list is contiguous with a stride of kListStride bytes (an odd
// number of dwords, so the 64 lanes' list heads fall in distinct LDS banks)
// and is read 4 entries at a time.
constexpr int kCap = 256;
constexpr int kListMax = 64;
constexpr int kListStride = kListMax + 4;

__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ float wave_minf(float v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_maxf(float v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_sumi(int v)
{
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ int wave_maxi(int v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Number of set lanes of `mask` below this lane.
__device__ __forceinline__ int lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0));
}

// Make this lane's LDS writes visible to the other lanes of its wave (the
// waves of a block run the neighbour loops independently, so no block-wide
// barrier can be used there).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int bcast(int v, int k) { return __builtin_amdgcn_readlane(v, k); }
__device__ __forceinline__ float bcastf(float v, int k)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

// Task records of a wave's range, fetched 64 at a time (one per lane) and
// read back wave-uniformly.
struct TaskRegs {
    int4 a;    // j0, jc, self, j
    float4 b;  // ox, oy, oz, -
    __device__ __forceinline__ void load(const Task *task, int t, bool ok)
    {
        if (ok) {
            const int4 *p = reinterpret_cast<const int4 *>(task + t);
            a = p[0];
            b = __builtin_bit_cast(float4, p[1]);
        } else {
            a = make_int4(0, 0, 0, 0);
            b = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
};

// Squared distance of a pair for the neighbour tests, with one fixed
// association and fused operations, so that the cell-pair loops, the list
// build and the list loops take identical decisions.
__device__ __forceinline__ float dist2(float dx, float dy, float dz)
{
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// Squared distance between the box [lo, hi] and a task's source cell,
// [o, o + e] in the receiving cell's frame (o the task's offset, e the cell's
// FP32 extent). FP32 addition is monotone, so no particle of the cell lies
// closer (box_dist2 of each particle is >= this): skipping a task whose
// distance is >= R^2 drops no particle that the per-particle cull keeps.
__device__ __forceinline__ float task_box_dist2(float ox, float oy, float oz, float4 e, float3 lo,
                                                float3 hi)
{
    const float dx = fmaxf(fmaxf(lo.x - (ox + e.x), ox - hi.x), 0.0f);
    const float dy = fmaxf(fmaxf(lo.y - (oy + e.y), oy - hi.y), 0.0f);
    const float dz = fmaxf(fmaxf(lo.z - (oz + e.z), oz - hi.z), 0.0f);
    return dist2(dx, dy, dz);
}

// Squared distance from p to the box [lo, hi].
__device__ __forceinline__ float box_dist2(float px, float py, float pz, float3 lo, float3 hi)
{
    float dx = fmaxf(fmaxf(lo.x - px, px - hi.x), 0.0f);
    float dy = fmaxf(fmaxf(lo.y - py, py - hi.y), 0.0f);
    float dz = fmaxf(fmaxf(lo.z - pz, pz - hi.z), 0.0f);
    return dist2(dx, dy, dz);
}

}  // namespace sphx
