// Tasks build: for each leaf cell, the self task and the pair tasks with every
// leaf whose bounding box lies within the larger of the two search radii
// (Section 2.2: self and pair tasks; interactions happen at the level whose
// cell size matches the local search radius). The search walks a tree of
// bounding boxes over the Morton-ordered leaves once per rebuild; the
// neighbour loops themselves never walk it.
//
// Slot layout. Each leaf owns a fixed slot of the task array, sized
// kSlotFactor times its task count at the last layout plus 8; its tasks are
// task[slot[I], end[I]). A rebuild walks the leaves straight into their
// slots, so it moves nothing, copies nothing and needs no readback to size
// anything: only a leaf that outgrows its slot forces a new layout (counts,
// a scan of the new slot sizes, one readback, a walk into the new slots).
// The in-place walks are also what a captured step replays: the _async
// entry points below launch the same kernels, each of which returns at once
// when its device gate reads zero, and report an outgrown slot in a device
// flag instead of handling it.
#include <algorithm>
#include <climits>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "sphx_internal.h"

// The walks below must reach identical decisions in every mode and in the
// serial form: keep the compiler from contracting the box-distance
// arithmetic differently in each.
#pragma clang fp contract(off)

namespace sphx {
namespace {

inline unsigned blocks(int64_t n, int t) { return unsigned((n + t - 1) / t); }

// Per-leaf kernels loop over the leaves with a stride of their grid: one
// block per leaf on the host path (the dispatcher balances uneven walks), at
// most kGatedGrid blocks where a captured step launches them behind a gate
// (a gate that reads zero then costs a small launch, not one block per leaf).
constexpr int64_t kGatedGrid = 8192;
inline unsigned leaf_grid(int64_t nl, const int32_t *run)
{
    return unsigned(run ? std::min<int64_t>(nl, kGatedGrid) : nl);
}

// Slot size of a leaf: kSlotFactor times its task count + 8. Roomy slots let
// the growth rebuilds of the h iteration (radii up to twice larger per pass
// in voids) stay in place.
constexpr int kSlotFactor = 4;

__device__ __forceinline__ int lanes_below64(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0));
}

__device__ __forceinline__ float wave_maxf(float v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Levels of the tree over the leaves, for kernels that update its radii.
struct TreeLevels {
    int64_t off[kMaxLevels];
    int n;
};

// Raise the radii of leaf L's ancestors to at least v: an atomic maximum on
// the non-negative floats' bit patterns (which order like the values), up to
// the first ancestor that already holds as much (it and every node above it
// then hold at least v, or will once the thread that raised it gets there).
__device__ __forceinline__ void raise_ancestors(float *__restrict__ node_r, const TreeLevels &lv,
                                                int64_t L, float v)
{
    int64_t c = L;
    for (int l = 1; l < lv.n; ++l) {
        c /= kTreeFan;
        float *a = node_r + lv.off[l] + c;
        if (__hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= v)
            break;
        atomicMax(reinterpret_cast<int *>(a), __float_as_int(v));
    }
}

// Full build: one level of the tree's radii from the level below.
__global__ void k_tree_radius(int64_t cnt_up, int64_t cnt_dn, const float *__restrict__ r_dn,
                              float *__restrict__ r_up, const int32_t *__restrict__ run)
{
    if (run && !*run)
        return;
    int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= cnt_up)
        return;
    int64_t e = (c + 1) * kTreeFan;
    if (e > cnt_dn)
        e = cnt_dn;
    float r = 0.0f;
    for (int64_t k = c * kTreeFan; k < e; ++k)
        r = fmaxf(r, r_dn[k]);
    r_up[c] = r;
}

// Full build: radius = (1 + skin) * gamma_k * max h over the leaf, for every
// leaf, and every leaf marked for the walk (the tree above: k_tree_radius,
// level by level: every leaf raising its ancestors itself would pile
// thousands of atomics onto the few nodes at the top).
// Clears the outgrown-slot flag and the asymmetry flag (a full build lists
// every pair within max(R_I, R_J)).
__global__ __launch_bounds__(64) void k_leaf_radius(int64_t n_leaves,
                                                    const int32_t *__restrict__ leaf_start,
                                                    const float *__restrict__ hs, float scale,
                                                    float *__restrict__ node_r,
                                                    float *__restrict__ radius,
                                                    uint8_t *__restrict__ overflow,
                                                    uint8_t *__restrict__ dirty,
                                                    int64_t *__restrict__ state,
                                                    const int32_t *__restrict__ run)
{
    if (run && !*run)
        return;
    const int lane = threadIdx.x;
    if (blockIdx.x == 0 && lane == 0) {
        state[kTaskOutgrown] = 0;
        state[kTaskAsym] = 0;
    }
    for (int64_t L = blockIdx.x; L < n_leaves; L += gridDim.x) {
        const int32_t s0 = leaf_start[L], cnt = leaf_start[L + 1] - s0;
        float v = lane < cnt ? hs[s0 + lane] : 0.0f;
        v = wave_maxf(v) * scale;
        if (lane == 0) {
            node_r[L] = v;
            radius[L] = v;
            dirty[L] = 1;
            overflow[L] = 0;
        }
    }
}

// Growth rebuild: a leaf is walked again when (1 + skin) gamma_k max h grew
// beyond its list's radius (the radius then grows; it never shrinks here).
// The tree holds the lists' radii: a grown leaf raises its ancestors' radii
// itself, so no per-level pass is needed. Sets the asymmetry flag: a leaf kept
// as it is may miss a pair that only a grown neighbour's radius reaches.
__global__ __launch_bounds__(64) void k_leaf_radius_grow(int64_t n_leaves,
                                                         const int32_t *__restrict__ leaf_start,
                                                         const float *__restrict__ hs,
                                                         float scale, float *__restrict__ node_r,
                                                         float *__restrict__ radius,
                                                         uint8_t *__restrict__ overflow,
                                                         uint8_t *__restrict__ dirty,
                                                         int64_t *__restrict__ state,
                                                         TreeLevels lv,
                                                         const int32_t *__restrict__ run)
{
    if (run && !*run)
        return;
    const int lane = threadIdx.x;
    if (blockIdx.x == 0 && lane == 0) {
        state[kTaskOutgrown] = 0;
        state[kTaskAsym] = 1;
    }
    for (int64_t L = blockIdx.x; L < n_leaves; L += gridDim.x) {
        const int32_t s0 = leaf_start[L], cnt = leaf_start[L + 1] - s0;
        float v = lane < cnt ? hs[s0 + lane] : 0.0f;
        v = wave_maxf(v) * scale;
        if (lane == 0) {
            const bool grow = v > radius[L];
            dirty[L] = grow ? 1 : 0;
            if (grow) {
                radius[L] = v;
                node_r[L] = v;
                overflow[L] = 0;  // the walk decides again
                raise_ancestors(node_r, lv, L, v);
            }
        }
    }
}

struct TreeView {
    const double *lo, *hi;
    const float *r;
    int64_t level_off[kMaxLevels];
    int64_t level_cnt[kMaxLevels];
    int n_levels;
    double L[3];
    int periodic;
    // several particle sets: the first leaf of each set and the set of each
    // leaf (null with one set); a walk stays inside its leaf's set
    const int32_t *set_leaf, *leaf_set;
};

// The leaves [la, lb) a walk from leaf I may pair it with: its own set's.
__device__ __forceinline__ void set_range(const TreeView &T, int64_t I, int64_t &la, int64_t &lb)
{
    la = 0;
    lb = T.level_cnt[0];
    if (T.leaf_set) {
        const int32_t b = T.leaf_set[I];
        la = T.set_leaf[b];
        lb = T.set_leaf[b + 1];
    }
}

// Whether node c of level lev (the leaves [c 8^lev, (c + 1) 8^lev)) holds a
// leaf of [la, lb).
__device__ __forceinline__ bool node_in_range(int lev, int64_t c, int64_t la, int64_t lb)
{
    const int64_t first = c << (3 * lev), end = (c + 1) << (3 * lev);
    return first < lb && end > la;
}

// Gap between [alo, ahi] and [blo, bhi] + s*L along one axis, for the shifts
// s in {-1, 0, 1} (periodic) or {0}.
__device__ __forceinline__ void axis_gaps(double alo, double ahi, double blo, double bhi,
                                          double L, int periodic, double g[3])
{
    for (int k = 0; k < 3; ++k) {
        double sh = double(k - 1) * L;
        if (!periodic && k != 1) {
            g[k] = INFINITY;
            continue;
        }
        double a = blo + sh - ahi, b = alo - (bhi + sh);
        double d = a > b ? a : b;
        g[k] = d > 0.0 ? d : 0.0;
    }
}

// Gaps of `node` to the receiving box per axis and shift; returns whether the
// node can hold a cell within max(R_I, R_node) of the box.
__device__ __forceinline__ bool node_near(const TreeView &T, const double alo[3],
                                          const double ahi[3], float RI, int64_t node,
                                          double g[3][3], double &R)
{
    R = fmax(double(RI), double(T.r[node]));
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        axis_gaps(alo[a], ahi[a], T.lo[3 * node + a], T.hi[3 * node + a], T.L[a], T.periodic,
                  g[a]);
        double m = fmin(g[a][0], fmin(g[a][1], g[a][2]));
        d2 += m * m;
    }
    return d2 < R * R;
}

// Emit the tasks of one cell that passed node_near, in shift order.
template <class Emit>
__device__ __forceinline__ int emit_shifts(const double g[3][3], double R, Emit &&emit)
{
    const double R2 = R * R;
    int n = 0;
    for (int sx = 0; sx < 3; ++sx) {
        if (!(g[0][sx] < R))
            continue;
        for (int sy = 0; sy < 3; ++sy) {
            if (!(g[1][sy] < R))
                continue;
            for (int sz = 0; sz < 3; ++sz) {
                if (!(g[2][sz] < R))
                    continue;
                double dd = g[0][sx] * g[0][sx] + g[1][sy] * g[1][sy] + g[2][sz] * g[2][sz];
                if (dd < R2) {
                    emit(n, sx - 1, sy - 1, sz - 1);
                    ++n;
                }
            }
        }
    }
    return n;
}

// The task record of leaf I's pair with leaf J at shift (sx, sy, sz): the
// offset origin_J + shift - origin_I formed in FP64, stored in FP32.
__device__ __forceinline__ Task make_task(const TreeView &T, const double *__restrict__ org,
                                          const int32_t *__restrict__ leaf_start, int64_t I,
                                          int64_t J, int sx, int sy, int sz)
{
    Task t;
    t.j = int32_t(J);
    t.j0 = leaf_start[J];
    t.jc = leaf_start[J + 1] - t.j0;
    t.self = (J == I && sx == 0 && sy == 0 && sz == 0) ? 1 : 0;
    t.j0b = t.j0;
    t.ox = float(org[3 * J] + double(sx) * T.L[0] - org[3 * I]);
    t.oy = float(org[3 * J + 1] + double(sy) * T.L[1] - org[3 * I + 1]);
    t.oz = float(org[3 * J + 2] + double(sz) * T.L[2] - org[3 * I + 2]);
    return t;
}

// Leaf I's walk found n tasks: its slot keeps min(n, size) of them (the ones
// written), and a leaf over its slot raises the flag.
__device__ __forceinline__ void slot_done(int64_t I, int32_t n, const int32_t *__restrict__ slot,
                                          int32_t *__restrict__ end, int32_t *__restrict__ count,
                                          int64_t *__restrict__ state)
{
    const int32_t size = slot[I + 1] - slot[I];
    count[I] = n;
    end[I] = slot[I] + (n < size ? n : size);
    if (n > size)
        state[kTaskOutgrown] = 1;
}

// Walk the tree for leaf `I`; for every leaf J (ascending) and shift whose box
// gap is below max(R_I, R_J), call emit(J, sx, sy, sz).
template <class Emit>
__device__ void walk(const TreeView &T, int64_t I, Emit &&emit)
{
    const double *ilo = T.lo + 3 * I, *ihi = T.hi + 3 * I;
    const double alo[3] = {ilo[0], ilo[1], ilo[2]}, ahi[3] = {ihi[0], ihi[1], ihi[2]};
    const float RI = T.r[I];
    int64_t la, lb;
    set_range(T, I, la, lb);
    // stack of (level, node) packed as level * 2^40 + node
    int64_t stack[kTreeFan * kMaxLevels + 8];
    int sp = 0;
    const int top = T.n_levels - 1;
    for (int64_t c = T.level_cnt[top] - 1; c >= 0; --c)
        stack[sp++] = (int64_t(top) << 40) | c;
    while (sp > 0) {
        int64_t e = stack[--sp];
        int lev = int(e >> 40);
        int64_t c = e & ((int64_t(1) << 40) - 1);
        int64_t node = T.level_off[lev] + c;
        double R;
        double g[3][3];
        if (!node_in_range(lev, c, la, lb) || !node_near(T, alo, ahi, RI, node, g, R))
            continue;
        if (lev == 0) {
            emit_shifts(g, R, [&](int, int sx, int sy, int sz) { emit(c, sx, sy, sz); });
            continue;
        }
        int64_t b = c * kTreeFan, e2 = b + kTreeFan;
        if (e2 > T.level_cnt[lev - 1])
            e2 = T.level_cnt[lev - 1];
        for (int64_t k = e2 - 1; k >= b; --k)
            stack[sp++] = (int64_t(lev - 1) << 40) | k;
    }
}

// Serial walks (one thread per leaf) of the leaves whose breadth-first
// frontier did not fit in LDS. WRITE = false: count them (for a new layout);
// WRITE: write them into their slots, for the leaves marked in `only`.
template <bool WRITE>
__global__ void k_task_serial(int64_t n_leaves, TreeView T, const double *__restrict__ org,
                              const int32_t *__restrict__ leaf_start,
                              const int32_t *__restrict__ slot, int32_t *__restrict__ end,
                              int32_t *__restrict__ count, const uint8_t *__restrict__ overflow,
                              const uint8_t *__restrict__ only, Task *__restrict__ task,
                              int64_t *__restrict__ state, const int32_t *__restrict__ run)
{
    if (run && !*run)
        return;
    const int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (I >= n_leaves || !overflow[I] || (only && !only[I]))
        return;
    int32_t n = 0;
    if (!WRITE) {
        walk(T, I, [&](int64_t, int, int, int) { ++n; });
        count[I] = n;
        return;
    }
    const int32_t w0 = slot[I], size = slot[I + 1] - w0;
    walk(T, I, [&](int64_t J, int sx, int sy, int sz) {
        if (n < size)
            task[w0 + n] = make_task(T, org, leaf_start, I, J, sx, sy, sz);
        ++n;
    });
    slot_done(I, n, slot, end, count, state);
}

// Sort keys of the launch order: slot i of the padded leaf range belongs to
// XCD range x = i / per; key = (x, ~work), work = sources of all the leaf's
// tasks (padding slots sort last in their range).
__global__ __launch_bounds__(64) void k_leaf_order_keys(int64_t n_leaves, int64_t nbp,
                                                        const int32_t *__restrict__ tbeg,
                                                        const int32_t *__restrict__ tend,
                                                        const Task *__restrict__ task,
                                                        uint64_t *__restrict__ key,
                                                        int32_t *__restrict__ val)
{
    const int64_t i = blockIdx.x;
    if (i >= nbp)
        return;
    const int lane = threadIdx.x;
    const int64_t per = nbp >> 3;
    uint32_t work = 0;
    if (i < n_leaves) {
        const int32_t a = tbeg[i], b = tend[i];
        uint32_t w = 0;
        for (int32_t t = a + lane; t < b; t += 64)
            w += uint32_t(task[t].jc);
        for (int o = 32; o > 0; o >>= 1)
            w += __shfl_xor(w, o, 64);
        work = w + 1;  // every real leaf sorts before the padding
    }
    if (lane == 0) {
        key[i] = (uint64_t(i / per) << 32) | uint64_t(0xffffffffu - work);
        val[i] = int32_t(i);
    }
}

constexpr int kFront = 1024;  // breadth-first frontier capacity (nodes) per cell

// Exclusive prefix sum over the wave of small non-negative counts (< 32),
// built from one ballot per bit; returns the prefix, sets `total`.
__device__ __forceinline__ int wave_prefix_small(int v, int &total)
{
    const uint64_t below = (uint64_t(1) << (threadIdx.x & 63)) - 1;
    int pre = 0;
    total = 0;
    for (int b = 0; b < 5; ++b) {
        const uint64_t m = __ballot((v >> b) & 1);
        pre += __popcll(m & below) << b;
        total += __popcll(m) << b;
    }
    return pre;
}

// One wave per receiving cell: level-by-level walk of the tree, 8 frontier
// nodes x 8 children tested per step by the 64 lanes; survivors keep their
// ascending order, so the cells (and their shifts) come out in the same order
// as in the serial walk. A frontier that would exceed kFront marks the cell
// for the serial walk instead. WRITE = false counts (count[I]); WRITE writes
// the tasks into the cell's slot, as many as fit, and records them
// (slot_done).
template <bool WRITE, typename FT>
__device__ __forceinline__ void bfs_leaf(int64_t I, const TreeView &T,
                                         const double *__restrict__ org,
                                         const int32_t *__restrict__ leaf_start,
                                         const int32_t *__restrict__ slot,
                                         int32_t *__restrict__ end, int32_t *__restrict__ count,
                                         uint8_t *__restrict__ overflow,
                                         Task *__restrict__ task, int64_t *__restrict__ state,
                                         FT (*front)[kFront])
{
    const int lane = threadIdx.x;
    __syncthreads();  // the previous leaf's frontier reads are done
    const double alo[3] = {T.lo[3 * I], T.lo[3 * I + 1], T.lo[3 * I + 2]};
    const double ahi[3] = {T.hi[3 * I], T.hi[3 * I + 1], T.hi[3 * I + 2]};
    const float RI = T.r[I];
    int64_t la, lb;
    set_range(T, I, la, lb);
    const int top = T.n_levels - 1;
    int cur = 0;
    int ncur = int(T.level_cnt[top]);
    if (ncur > kFront) {
        if (lane == 0) {
            overflow[I] = 1;
            if (!WRITE)
                count[I] = 0;
        }
        return;
    }
    for (int k = lane; k < ncur; k += 64)
        front[0][k] = FT(k);
    int emitted = 0;
    const int32_t wbase = WRITE ? slot[I] : 0;
    const int32_t wcap = WRITE ? slot[I + 1] - slot[I] : 0;
    // One wave-wide round of up to 64 candidate leaves, one per lane, in lane
    // order: tasks counted, prefix-summed over the lanes and written.
    auto emit_round = [&](bool cand, int32_t J) __attribute__((always_inline)) {
        int nt = 0;
        double g[3][3], R = 0.0;
        if (cand && node_near(T, alo, ahi, RI, J, g, R))
            nt = emit_shifts(g, R, [](int, int, int, int) {});
        int tot;
        const int pre = wave_prefix_small(nt, tot);
        if (WRITE && nt > 0) {
            emit_shifts(g, R, [&](int k, int sx, int sy, int sz) {
                if (emitted + pre + k < wcap)
                    task[wbase + emitted + pre + k] =
                        make_task(T, org, leaf_start, I, J, sx, sy, sz);
            });
        }
        emitted += tot;
    };
    for (int lev = top; lev >= 0; --lev) {
        __syncthreads();
        if (lev == 0) {
            // a tree of one level: the frontier holds the leaves themselves
            for (int base = 0; base < ncur; base += 64) {
                const int idx = base + lane;
                const int32_t J = idx < ncur ? int32_t(front[cur][idx]) : 0;
                emit_round(idx < ncur && J >= la && J < lb, J);
            }
            break;
        }
        if (lev == 1) {
            // the children are the leaves (level 0 holds them at their own
            // index): emit them straight from this expansion, in the order
            // a leaf frontier would hold them, so the frontier never has to
            // hold the finest level
            const int64_t n0 = T.level_cnt[0];
            for (int base = 0; base < ncur; base += 8) {
                const int k = base + (lane >> 3);
                const int64_t child =
                    k < ncur ? int64_t(front[cur][k]) * kTreeFan + (lane & 7) : n0;
                const bool in = child < n0 && child >= la && child < lb;
                emit_round(in, in ? int32_t(child) : 0);
            }
            break;
        }
        // expand the frontier into the surviving children at level lev - 1
        const int64_t cnt_dn = T.level_cnt[lev - 1];
        const int64_t off_dn = T.level_off[lev - 1];
        int nnext = 0;
        bool over = false;
        for (int base = 0; base < ncur; base += 8) {
            const int k = base + (lane >> 3);
            const int c = lane & 7;
            bool keep = false;
            int64_t child = 0;
            if (k < ncur) {
                child = int64_t(front[cur][k]) * kTreeFan + c;
                if (child < cnt_dn && node_in_range(lev - 1, child, la, lb)) {
                    double g[3][3], R;
                    keep = node_near(T, alo, ahi, RI, off_dn + child, g, R);
                }
            }
            const uint64_t mask = __ballot(keep);
            const int tot = __popcll(mask);
            if (nnext + tot > kFront) {
                over = true;
                break;
            }
            if (keep)
                front[cur ^ 1][nnext + lanes_below64(mask)] = FT(child);
            nnext += tot;
        }
        if (over) {
            if (lane == 0) {
                overflow[I] = 1;
                if (!WRITE)
                    count[I] = 0;
            }
            return;
        }
        cur ^= 1;
        ncur = nnext;
    }
    if (lane == 0) {
        if (WRITE)
            slot_done(I, emitted, slot, end, count, state);
        else
            count[I] = emitted;
    }
}

// The breadth-first walk over the leaves marked in `only` (every leaf when
// null), with a stride of the grid. FT: the frontier's index type, 16 bits
// when every level has at most 2^16 nodes (half the LDS per wave: twice the
// waves per CU for this latency-bound walk), else 32.
template <bool WRITE, typename FT>
__global__ __launch_bounds__(64) void k_task_bfs(int64_t n_leaves, TreeView T,
                                                 const double *__restrict__ org,
                                                 const int32_t *__restrict__ leaf_start,
                                                 const int32_t *__restrict__ slot,
                                                 int32_t *__restrict__ end,
                                                 int32_t *__restrict__ count,
                                                 uint8_t *__restrict__ overflow,
                                                 Task *__restrict__ task,
                                                 const uint8_t *__restrict__ only,
                                                 int64_t *__restrict__ state,
                                                 const int32_t *__restrict__ run)
{
    if (run && !*run)
        return;
    __shared__ FT front[2][kFront];
    for (int64_t I = blockIdx.x; I < n_leaves; I += gridDim.x) {
        if (only && !only[I])
            continue;
        bfs_leaf<WRITE, FT>(I, T, org, leaf_start, slot, end, count, overflow, task, state,
                            front);
    }
}

// Slot sizes of a new layout from the counts of every leaf, never below the
// leaf's slot in the previous layout (prev, if any: slots only grow, so a
// step whose radii rise and fall in a repeating pattern settles on a layout
// that holds all of it); their 64-bit sum goes to state[kTaskSlots] (the
// 32-bit scan of the sizes must not wrap), the counts' sum (the tasks the
// walk into the new slots will write) to state[kTaskTotal].
__global__ void k_slot_sizes(int64_t n_leaves, const int32_t *__restrict__ count,
                             const int32_t *__restrict__ prev, int32_t *__restrict__ sz,
                             int64_t *__restrict__ state)
{
    const int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t v = 0, c = 0;
    if (I < n_leaves) {
        c = count[I];
        v = int64_t(kSlotFactor) * c + 8;
        const int64_t was = prev ? int64_t(prev[I + 1]) - prev[I] : 0;
        v = v > was ? v : was;
        sz[I] = int32_t(v < int64_t(INT_MAX) ? v : int64_t(INT_MAX));
    } else if (I == n_leaves) {
        sz[I] = 0;
    }
    for (int o = 32; o > 0; o >>= 1) {
        v += __shfl_xor(v, o, 64);
        c += __shfl_xor(c, o, 64);
    }
    if ((threadIdx.x & 63) == 0 && v) {
        atomicAdd(reinterpret_cast<unsigned long long *>(state + kTaskSlots),
                  (unsigned long long)v);
        atomicAdd(reinterpret_cast<unsigned long long *>(state + kTaskTotal),
                  (unsigned long long)c);
    }
}

// Empty slots of a new layout (end = slot start) and a cleared flag.
__global__ void k_slots_empty(int64_t n_leaves, const int32_t *__restrict__ slot,
                              int32_t *__restrict__ end, int64_t *__restrict__ state)
{
    const int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (I < n_leaves)
        end[I] = slot[I];
    if (I == 0)
        state[kTaskOutgrown] = 0;
}

__global__ void k_state_clear(int64_t *__restrict__ state)
{
    if (threadIdx.x < kTaskStateWords)
        state[threadIdx.x] = 0;
}

// state[kTaskTotal] = the tasks held, summed over the leaves' slots: each
// block adds its leaves' counts with one atomic (k_task_total_clear first).
constexpr int kTotalThreads = 256;
__global__ void k_task_total_clear(int64_t *__restrict__ state)
{
    if (threadIdx.x == 0)
        state[kTaskTotal] = 0;
}

__global__ __launch_bounds__(kTotalThreads) void k_task_total(int64_t n_leaves,
                                                              const int32_t *__restrict__ slot,
                                                              const int32_t *__restrict__ end,
                                                              int64_t *__restrict__ state)
{
    __shared__ int64_t part[kTotalThreads / 64];
    int64_t v = 0;
    for (int64_t I = int64_t(blockIdx.x) * kTotalThreads + threadIdx.x; I < n_leaves;
         I += int64_t(gridDim.x) * kTotalThreads)
        v += end[I] - slot[I];
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int k = 0; k < kTotalThreads / 64; ++k)
            t += part[k];
        if (t)
            atomicAdd(reinterpret_cast<unsigned long long *>(state + kTaskTotal),
                      (unsigned long long)t);
    }
}

}  // namespace

// state[kTaskTotal] summed over the slots (two launches; capturable).
static sphx_status total_launch(int64_t nl, sphx_tasks *t, hipStream_t s)
{
    k_task_total_clear<<<1, 64, 0, s>>>(t->state);
    SPHX_HIP(hipGetLastError());
    const unsigned nb = unsigned(std::min<int64_t>((nl + kTotalThreads - 1) / kTotalThreads + 1,
                                                    1024));
    k_task_total<<<nb, kTotalThreads, 0, s>>>(nl, t->slot, t->end, t->state);
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

// The tree view of a grid with the periodic box of the context.
static TreeView tree_view(const sphx_ctx *ctx, const sphx_grid *g)
{
    TreeView T;
    T.lo = g->node_lo;
    T.hi = g->node_hi;
    T.r = g->node_r;
    for (int l = 0; l < kMaxLevels; ++l) {
        T.level_off[l] = l < g->n_levels ? g->level_off[l] : 0;
        T.level_cnt[l] = l < g->n_levels ? g->level_cnt[l] : 0;
    }
    T.n_levels = g->n_levels;
    for (int a = 0; a < 3; ++a)
        T.L[a] = ctx->p.box[a];
    T.periodic = ctx->p.periodic;
    T.set_leaf = g->set_leaf;
    T.leaf_set = g->leaf_set;
    return T;
}

// Launches the breadth-first walk with the narrowest frontier index type.
template <bool WRITE>
static void bfs_launch(const sphx_ctx *ctx, const sphx_grid *g, sphx_tasks *t,
                       const uint8_t *only, const int32_t *run, hipStream_t s)
{
    const int64_t nl = g->n_leaves;
    const TreeView T = tree_view(ctx, g);
    const unsigned grid = leaf_grid(nl, run);
    if (nl <= 65536)
        k_task_bfs<WRITE, uint16_t><<<grid, 64, 0, s>>>(nl, T, g->leaf_org, g->leaf_start,
                                                       t->slot, t->end, t->count, t->overflow,
                                                       t->task, only, t->state, run);
    else
        k_task_bfs<WRITE, int32_t><<<grid, 64, 0, s>>>(nl, T, g->leaf_org, g->leaf_start,
                                                      t->slot, t->end, t->count, t->overflow,
                                                      t->task, only, t->state, run);
}

// Leaf radii (a full build: every leaf, marked; a growth rebuild: the grown
// leaves, marked) and the tree's radii above them.
static sphx_status radii_launch(const sphx_ctx *ctx, sphx_grid *g, sphx_tasks *t, bool grow,
                                const int32_t *run, hipStream_t s)
{
    const int64_t nl = g->n_leaves;
    const float scale = float(ctx->p.gamma_k * (1.0 + ctx->p.skin));
    if (grow) {
        // (the grown leaves raise their ancestors themselves)
        TreeLevels lv;
        for (int l = 0; l < kMaxLevels; ++l)
            lv.off[l] = l < g->n_levels ? g->level_off[l] : 0;
        lv.n = g->n_levels;
        k_leaf_radius_grow<<<leaf_grid(nl, run), 64, 0, s>>>(
            nl, g->leaf_start, g->hs, scale, g->node_r, t->radius, t->overflow, t->dirty,
            t->state, lv, run);
        SPHX_HIP(hipGetLastError());
        return SPHX_OK;
    }
    k_leaf_radius<<<leaf_grid(nl, run), 64, 0, s>>>(nl, g->leaf_start, g->hs, scale, g->node_r,
                                                     t->radius, t->overflow, t->dirty, t->state,
                                                     run);
    SPHX_HIP(hipGetLastError());
    for (int l = 0; l + 1 < g->n_levels; ++l) {
        const int64_t up = g->level_cnt[l + 1];
        k_tree_radius<<<blocks(up, 128), 128, 0, s>>>(up, g->level_cnt[l],
                                                        g->node_r + g->level_off[l],
                                                        g->node_r + g->level_off[l + 1], run);
        SPHX_HIP(hipGetLastError());
    }
    return SPHX_OK;
}

// The marked leaves walked into their slots: the breadth-first walk, then the
// serial walk of those whose frontier overflowed.
static sphx_status walk_slots_launch(const sphx_ctx *ctx, const sphx_grid *g, sphx_tasks *t,
                                     const int32_t *run, hipStream_t s)
{
    const int64_t nl = g->n_leaves;
    bfs_launch<true>(ctx, g, t, t->dirty, run, s);
    SPHX_HIP(hipGetLastError());
    k_task_serial<true><<<blocks(nl, 64), 64, 0, s>>>(nl, tree_view(ctx, g), g->leaf_org,
                                                      g->leaf_start, t->slot, t->end, t->count,
                                                      t->overflow, t->dirty, t->task, t->state,
                                                      run);
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

// The task list's device state, read back (synchronises the stream); with
// total, state[kTaskTotal] is summed over the slots first.
static sphx_status read_state(sphx_ctx *ctx, sphx_tasks *t, hipStream_t s,
                              int64_t st[kTaskStateWords], bool total = true)
{
    if (total)
        SPHX_TRY(total_launch(t->grid->n_leaves, t, s));
    int64_t *h = reinterpret_cast<int64_t *>(ctx->h_pinned + kPinnedBytes - 64);
    SPHX_HIP(hipMemcpyAsync(h, t->state, kTaskStateWords * sizeof(int64_t),
                            hipMemcpyDeviceToHost, s));
    SPHX_HIP(wait_stream(ctx, s));
    for (int k = 0; k < kTaskStateWords; ++k)
        st[k] = h[k];
    return SPHX_OK;
}

size_t tasks_bytes(int64_t n, int leaf_max)
{
    // An estimate (the task count depends on the clustering): one leaf per
    // leaf_max / 4 particles (at least 4) with 96 tasks each, held in slots
    // of kSlotFactor tasks per task + 8 (allocated with an eighth of
    // headroom), plus the per-leaf arrays (slot starts and ends, counts,
    // radius, flags, launch order and its sort keys).
    const int64_t leaves = n / std::max(4, leaf_max / 4) + 1;
    const int64_t per_leaf_tasks = 96;
    const int64_t task_slots = kSlotFactor * per_leaf_tasks + 8;
    return size_t(leaves) * (size_t(task_slots + task_slots / 8) * sizeof(Task) + 48) +
           (1 << 20);
}

void tasks_free(sphx_tasks *t)
{
    if (!t)
        return;
    void *ptrs[] = {t->slot, t->end, t->task, t->count, t->radius, t->scan_tmp, t->overflow,
                    t->dirty, t->state};
    for (void *p : ptrs)
        dfree(p, t->stream);
    for (void *p : {(void *)t->order, (void *)t->okey, (void *)t->okey_out, (void *)t->oval,
                    t->sort_tmp})
        dfree(p, t->stream);
    delete t;
}

// Launch order of the per-leaf loops (see sphx_tasks::order). The sort keys
// use 35 bits: the XCD range (0..7) above the 32-bit inverted work.
constexpr unsigned kOrderKeyBits = 35;
static sphx_status leaf_order(sphx_tasks *t, int64_t nl, hipStream_t s)
{
    const int64_t nbp = pad8(nl);
    if (nbp > t->order_cap) {
        for (void *p : {(void *)t->order, (void *)t->okey, (void *)t->okey_out, (void *)t->oval,
                        t->sort_tmp})
            dfree(p, s);
        t->order = nullptr;
        t->okey = t->okey_out = nullptr;
        t->oval = nullptr;
        t->sort_tmp = nullptr;
        t->order_cap = 0;
        size_t tmp = 0;
        SPHX_HIP(rocprim::radix_sort_pairs(nullptr, tmp, (uint64_t *)nullptr, (uint64_t *)nullptr,
                                           (int32_t *)nullptr, (int32_t *)nullptr, size_t(nbp), 0,
                                           kOrderKeyBits, s));
        if (dmalloc((void **)&t->order, size_t(nbp) * sizeof(int32_t), s) != hipSuccess ||
            dmalloc((void **)&t->okey, size_t(nbp) * sizeof(uint64_t), s) != hipSuccess ||
            dmalloc((void **)&t->okey_out, size_t(nbp) * sizeof(uint64_t), s) != hipSuccess ||
            dmalloc((void **)&t->oval, size_t(nbp) * sizeof(int32_t), s) != hipSuccess ||
            dmalloc(&t->sort_tmp, tmp + 16, s) != hipSuccess) {
            set_error("sphx_tasks_build: out of device memory (leaf order)");
            return SPHX_E_OOM;
        }
        t->sort_tmp_bytes = tmp;
        t->order_cap = nbp;
    }
    k_leaf_order_keys<<<unsigned(nbp), 64, 0, s>>>(nl, nbp, t->slot, t->end, t->task, t->okey,
                                                   t->oval);
    SPHX_HIP(hipGetLastError());
    size_t tmp = t->sort_tmp_bytes;
    SPHX_HIP(rocprim::radix_sort_pairs(t->sort_tmp, tmp, t->okey, t->okey_out, t->oval, t->order,
                                       size_t(nbp), 0, kOrderKeyBits, s));
    return SPHX_OK;
}

// A new slot layout at the current radii (every leaf marked): each leaf's
// tasks counted, slots of kSlotFactor count + 8 (or the leaf's previous
// slot, if larger), the task array grown if needed (the old contents are not
// kept), every leaf walked into its slot.
static sphx_status relayout(sphx_ctx *ctx, sphx_grid *g, sphx_tasks *t, hipStream_t s)
{
    const int64_t nl = g->n_leaves;
    bfs_launch<false>(ctx, g, t, nullptr, nullptr, s);
    SPHX_HIP(hipGetLastError());
    k_task_serial<false><<<blocks(nl, 64), 64, 0, s>>>(nl, tree_view(ctx, g), g->leaf_org,
                                                       g->leaf_start, t->slot, t->end, t->count,
                                                       t->overflow, nullptr, t->task, t->state,
                                                       nullptr);
    SPHX_HIP(hipGetLastError());
    k_state_clear<<<1, 64, 0, s>>>(t->state);
    SPHX_HIP(hipGetLastError());
    // the sizes go to `end` (free until the walk below), their scan to `slot`
    k_slot_sizes<<<blocks(nl + 1, 256), 256, 0, s>>>(nl, t->count, t->task ? t->slot : nullptr,
                                                      t->end, t->state);
    SPHX_HIP(hipGetLastError());
    size_t tmp = t->scan_tmp_bytes;
    SPHX_HIP(rocprim::exclusive_scan(t->scan_tmp, tmp, t->end, t->slot, 0, size_t(nl + 1),
                                     rocprim::plus<int32_t>(), s));
    int64_t st[kTaskStateWords];
    SPHX_TRY(read_state(ctx, t, s, st, false));
    if (st[kTaskSlots] > int64_t(INT_MAX)) {
        set_error("sphx_tasks_build: more than 2^31 task slots");
        return SPHX_E_INVALID;
    }
    const int64_t slots = st[kTaskSlots];
    if (slots > t->cap) {
        dfree(t->task, s);
        t->task = nullptr;
        t->cap = 0;
        const int64_t cap = std::min<int64_t>(slots + slots / 8 + 64, int64_t(INT_MAX));
        SPHX_HIP(dmalloc((void **)&t->task, size_t(cap) * sizeof(Task), s));
        t->cap = cap;
    }
    k_slots_empty<<<blocks(nl, 256), 256, 0, s>>>(nl, t->slot, t->end, t->state);
    SPHX_HIP(hipGetLastError());
    t->relayouts++;
    // every slot holds its leaf's count (the walk below finds the same tasks
    // as the count above), so nothing is read back after it
    SPHX_TRY(walk_slots_launch(ctx, g, t, nullptr, s));
    t->n_tasks = st[kTaskTotal];
    return SPHX_OK;
}

sphx_status tasks_build(sphx_ctx *ctx, sphx_grid *g, const sphx_particles *in, hipStream_t s,
                        sphx_tasks **out)
{
    sphx_tasks *t = *out;
    const int64_t nl = g->n_leaves;
    (void)in;
    if (t && t->grid != g) {
        set_error("sphx_tasks_build: task list belongs to another grid");
        return SPHX_E_STATE;
    }
    if (t)
        t->stream = s;
    bool fresh = false;
    if (!t) {
        t = new sphx_tasks();
        t->serial = next_serial();
        t->grid = g;
        t->stream = s;
        fresh = true;
        auto fail = [&](sphx_status st) {
            tasks_free(t);
            return st;
        };
        if (dmalloc((void **)&t->slot, (nl + 1) * sizeof(int32_t), s) != hipSuccess ||
            dmalloc((void **)&t->end, (nl + 1) * sizeof(int32_t), s) != hipSuccess ||
            dmalloc((void **)&t->count, (nl + 1) * sizeof(int32_t), s) != hipSuccess ||
            dmalloc((void **)&t->radius, (nl + 1) * sizeof(float), s) != hipSuccess ||
            dmalloc((void **)&t->overflow, (nl + 1) * sizeof(uint8_t), s) != hipSuccess ||
            dmalloc((void **)&t->dirty, (nl + 1) * sizeof(uint8_t), s) != hipSuccess ||
            dmalloc((void **)&t->state, kTaskStateWords * sizeof(int64_t), s) != hipSuccess) {
            set_error("sphx_tasks_build: out of device memory");
            return fail(SPHX_E_OOM);
        }
        size_t tmp = 0;
        if (rocprim::exclusive_scan(nullptr, tmp, t->count, t->slot, 0, size_t(nl + 1),
                                    rocprim::plus<int32_t>(), s) != hipSuccess ||
            dmalloc(&t->scan_tmp, tmp + 16, s) != hipSuccess) {
            set_error("sphx_tasks_build: scan workspace");
            return fail(SPHX_E_OOM);
        }
        t->scan_tmp_bytes = tmp;
        k_state_clear<<<1, 64, 0, s>>>(t->state);
        if (hipGetLastError() != hipSuccess) {
            set_error("sphx_tasks_build: launch failed");
            return fail(SPHX_E_HIP);
        }
    }
    struct Guard {
        sphx_tasks *t;
        bool fresh;
        bool keep = false;
        ~Guard()
        {
            if (fresh && !keep)
                tasks_free(t);
        }
    } guard{t, fresh};

    if (nl == 0) {
        t->n_tasks = 0;
        t->symmetric = true;
        guard.keep = true;
        *out = t;
        return SPHX_OK;
    }
    SPHX_TRY(radii_launch(ctx, g, t, false, nullptr, s));
    bool fits = false;
    int64_t st[kTaskStateWords];
    if (t->task) {
        // in place: every leaf into its slot of the current layout
        SPHX_TRY(walk_slots_launch(ctx, g, t, nullptr, s));
        SPHX_TRY(read_state(ctx, t, s, st));
        fits = st[kTaskOutgrown] == 0;
    }
    if (fits)
        t->n_tasks = st[kTaskTotal];
    else
        SPHX_TRY(relayout(ctx, g, t, s));
    SPHX_TRY(leaf_order(t, nl, s));
    t->symmetric = true;
    guard.keep = true;
    *out = t;
    return SPHX_OK;
}

sphx_status tasks_grow(sphx_ctx *ctx, sphx_grid *g, const sphx_particles *in, hipStream_t s,
                       sphx_tasks **out)
{
    sphx_tasks *t = *out;
    const int64_t nl = g->n_leaves;
    if (!t || t->grid != g || !t->task || nl == 0)
        return tasks_build(ctx, g, in, s, out);
    t->stream = s;
    SPHX_TRY(radii_launch(ctx, g, t, true, nullptr, s));
    SPHX_TRY(walk_slots_launch(ctx, g, t, nullptr, s));
    int64_t st[kTaskStateWords];
    SPHX_TRY(read_state(ctx, t, s, st));
    if (st[kTaskOutgrown])
        return tasks_build(ctx, g, in, s, out);  // a full build, in a new layout if need be
    t->n_tasks = st[kTaskTotal];
    // (the launch order of the last full build stays: it orders by work,
    // which the few walked leaves hardly move)
    t->symmetric = false;
    return SPHX_OK;
}

sphx_status tasks_grow_async(const sphx_ctx *ctx, sphx_grid *g, sphx_tasks *t,
                             const int32_t *run, hipStream_t s)
{
    if (g->n_leaves == 0)
        return SPHX_OK;
    SPHX_TRY(radii_launch(ctx, g, t, true, run, s));
    return walk_slots_launch(ctx, g, t, run, s);
}

sphx_status tasks_full_async(const sphx_ctx *ctx, sphx_grid *g, sphx_tasks *t,
                             const int32_t *run, hipStream_t s)
{
    if (g->n_leaves == 0)
        return SPHX_OK;
    SPHX_TRY(radii_launch(ctx, g, t, false, run, s));
    return walk_slots_launch(ctx, g, t, run, s);
}

sphx_status tasks_total_async(const sphx_grid *g, sphx_tasks *t, hipStream_t s)
{
    return total_launch(g->n_leaves, t, s);
}

}  // namespace sphx
