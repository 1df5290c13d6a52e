// Tasks build: for each leaf cell, the self task and the pair tasks with every
// leaf whose bounding box lies within the larger of the two search radii
// (Section 2.2: self and pair tasks; interactions happen at the level whose
// cell size matches the local search radius). The search walks a tree of
// bounding boxes over the Morton-ordered leaves once per rebuild; the
// neighbour loops themselves never walk it.
#include <algorithm>
#include <climits>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "sphx_internal.h"

// The count and fill kernels below must reach identical decisions: keep the
// compiler from contracting the box-distance arithmetic differently in each.
#pragma clang fp contract(off)

namespace sphx {
namespace {

inline unsigned blocks(int64_t n, int t) { return unsigned((n + t - 1) / t); }

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

// One wave per leaf: radius = (1 + skin) * gamma_k * max h over the leaf.
__global__ __launch_bounds__(64) void k_leaf_radius(int64_t n_leaves,
                                                    const int32_t *__restrict__ leaf_start,
                                                    const float *__restrict__ hs, float scale,
                                                    float *__restrict__ node_r,
                                                    float *__restrict__ radius)
{
    int64_t L = blockIdx.x;
    if (L >= n_leaves)
        return;
    int lane = threadIdx.x;
    int32_t s0 = leaf_start[L], cnt = leaf_start[L + 1] - s0;
    float v = lane < cnt ? hs[s0 + lane] : 0.0f;
    v = wave_maxf(v) * scale;
    if (lane == 0) {
        node_r[L] = v;
        radius[L] = v;
    }
}

// Growth rebuild: a leaf is walked again when (1 + skin) gamma_k max h grew
// beyond its list's radius (the radius then grows; it never shrinks here) or
// when the serial walk built its list; the tree holds the lists' radii.
__global__ __launch_bounds__(64) void k_leaf_radius_grow(int64_t n_leaves,
                                                         const int32_t *__restrict__ leaf_start,
                                                         const float *__restrict__ hs,
                                                         float scale, float *__restrict__ node_r,
                                                         float *__restrict__ radius,
                                                         uint8_t *__restrict__ overflow,
                                                         uint8_t *__restrict__ dirty)
{
    int64_t L = blockIdx.x;
    if (L >= n_leaves)
        return;
    int lane = threadIdx.x;
    int32_t s0 = leaf_start[L], cnt = leaf_start[L + 1] - s0;
    float v = lane < cnt ? hs[s0 + lane] : 0.0f;
    v = wave_maxf(v) * scale;
    if (lane == 0) {
        const bool grow = v > radius[L];
        const bool d = grow || overflow[L] != 0;
        const float r = grow ? v : radius[L];
        radius[L] = r;
        node_r[L] = r;
        dirty[L] = d ? 1 : 0;
        if (d)
            overflow[L] = 0;  // the walk decides again
    }
}

// Growth rebuild: the leaves kept as they are count their current lists.
__global__ void k_keep_counts(int64_t n_leaves, const uint8_t *__restrict__ dirty,
                              const int32_t *__restrict__ off, int32_t *__restrict__ count)
{
    const int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (I < n_leaves && !dirty[I])
        count[I] = off[I + 1] - off[I];
    else if (I == n_leaves)
        count[I] = 0;
}

// Growth rebuild: the new list from the old one (leaves kept) and from the
// slots of the walked leaves that fitted (the others are written by the
// second walk or the serial fill).
__global__ __launch_bounds__(64) void k_copy_grown(int64_t n_leaves,
                                                   const uint8_t *__restrict__ dirty,
                                                   const uint8_t *__restrict__ overflow,
                                                   const int32_t *__restrict__ off_old,
                                                   const int32_t *__restrict__ off_new,
                                                   const int32_t *__restrict__ soff,
                                                   const int32_t *__restrict__ count,
                                                   const Task *__restrict__ task_old,
                                                   const Task *__restrict__ slack,
                                                   Task *__restrict__ task_new)
{
    const int64_t I = blockIdx.x;
    if (I >= n_leaves)
        return;
    const int32_t n = count[I], b = off_new[I];
    const Task *src;
    if (!dirty[I])
        src = task_old + off_old[I];
    else if (!overflow[I] && n <= soff[I + 1] - soff[I])
        src = slack + soff[I];
    else
        return;
    for (int32_t k = threadIdx.x; k < n; k += 64)
        task_new[b + k] = src[k];
}

__global__ void k_tree_radius(int64_t cnt_up, int64_t cnt_dn, const float *__restrict__ r_dn,
                              float *__restrict__ r_up)
{
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

struct TreeView {
    const double *lo, *hi;
    const float *r;
    int64_t level_off[kMaxLevels];
    int64_t level_cnt[kMaxLevels];
    int n_levels;
    double L[3];
    int periodic;
};

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

// Walk the tree for leaf `I`; for every leaf J (ascending) and shift whose box
// gap is below max(R_I, R_J), call emit(J, sx, sy, sz).
template <class Emit>
__device__ void walk(const TreeView &T, int64_t I, Emit &&emit)
{
    const double *ilo = T.lo + 3 * I, *ihi = T.hi + 3 * I;
    const double alo[3] = {ilo[0], ilo[1], ilo[2]}, ahi[3] = {ihi[0], ihi[1], ihi[2]};
    const float RI = T.r[I];
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
        if (!node_near(T, alo, ahi, RI, node, g, R))
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

// Serial walks (one thread per cell), used for the cells whose breadth-first
// frontier did not fit in LDS.
__global__ void k_task_count(int64_t n_leaves, TreeView T, const uint8_t *__restrict__ overflow,
                             int32_t *__restrict__ count)
{
    int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (I >= n_leaves || !overflow[I])
        return;
    int32_t c = 0;
    walk(T, I, [&](int64_t, int, int, int) { ++c; });
    count[I] = c;
}

__global__ void k_task_fill(int64_t n_leaves, TreeView T, const double *__restrict__ org,
                            const int32_t *__restrict__ leaf_start,
                            const uint8_t *__restrict__ overflow,
                            const int32_t *__restrict__ off, Task *__restrict__ task)
{
    int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (I >= n_leaves || !overflow[I])
        return;
    int32_t w = off[I];
    const int32_t w_end = off[I + 1];
    const double ox = org[3 * I], oy = org[3 * I + 1], oz = org[3 * I + 2];
    walk(T, I, [&](int64_t J, int sx, int sy, int sz) {
        Task t;
        t.j = int32_t(J);
        t.j0 = leaf_start[J];
        t.jc = leaf_start[J + 1] - t.j0;
        t.self = (J == I && sx == 0 && sy == 0 && sz == 0) ? 1 : 0;
        t.j0b = t.j0;
        // origin_j + shift - origin_i, formed in FP64, stored in FP32
        t.ox = float(org[3 * J] + double(sx) * T.L[0] - ox);
        t.oy = float(org[3 * J + 1] + double(sy) * T.L[1] - oy);
        t.oz = float(org[3 * J + 2] + double(sz) * T.L[2] - oz);
        if (w < w_end)
            task[w++] = t;
    });
}

// Sort keys of the launch order: slot i of the padded leaf range belongs to
// XCD range x = i / per; key = (x, ~work), work = sources of all the leaf's
// tasks (padding slots sort last in their range).
__global__ __launch_bounds__(64) void k_leaf_order_keys(int64_t n_leaves, int64_t nbp,
                                                        const int32_t *__restrict__ off,
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
        const int32_t a = off[i], b = off[i + 1];
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
// for the serial walk instead. MODE 0 counts; MODE 1 writes at off[I];
// MODE 2 writes into the cell's slot of the slack layout, at slot[I] up to
// its size slot[I+1] - slot[I], and counts; MODE 3 writes at off[I] the cells
// whose MODE 2 count exceeded their slot (the others return at once).
// FT: the frontier's index type, 16 bits when every level has at most 2^16
// nodes (half the LDS per wave: twice the waves per CU for this
// latency-bound walk), else 32.
template <int MODE, typename FT>
__global__ __launch_bounds__(64) void k_task_bfs(int64_t n_leaves, TreeView T,
                                                 const double *__restrict__ org,
                                                 const int32_t *__restrict__ leaf_start,
                                                 const int32_t *__restrict__ off,
                                                 const int32_t *__restrict__ slot,
                                                 int32_t *__restrict__ count,
                                                 uint8_t *__restrict__ overflow,
                                                 Task *__restrict__ task,
                                                 const uint8_t *__restrict__ only)
{
    const int64_t I = blockIdx.x;
    if (I >= n_leaves || (only && !only[I]))
        return;  // (only: the growth rebuild walks the marked leaves alone)
    constexpr bool COUNT = MODE == 0 || MODE == 2, WRITE = MODE != 0;
    if (!COUNT && overflow[I])
        return;
    if (MODE == 3 && count[I] <= slot[I + 1] - slot[I])
        return;
    const int lane = threadIdx.x;
    __shared__ FT front[2][kFront];
    const double alo[3] = {T.lo[3 * I], T.lo[3 * I + 1], T.lo[3 * I + 2]};
    const double ahi[3] = {T.hi[3 * I], T.hi[3 * I + 1], T.hi[3 * I + 2]};
    const float RI = T.r[I];
    const int top = T.n_levels - 1;
    int cur = 0;
    int ncur = int(T.level_cnt[top]);
    if (ncur > kFront) {
        if (COUNT && lane == 0) {
            overflow[I] = 1;
            count[I] = 0;
        }
        return;
    }
    for (int k = lane; k < ncur; k += 64)
        front[0][k] = FT(k);
    int emitted = 0;
    const int32_t wbase = MODE == 2 ? slot[I] : (WRITE ? off[I] : 0);
    const int32_t wcap = MODE == 2 ? slot[I + 1] - slot[I] : 0x7fffffff;
    const double oxi = org[3 * I], oyi = org[3 * I + 1], ozi = org[3 * I + 2];
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
            const int32_t j0 = leaf_start[J];
            const int32_t jc = leaf_start[J + 1] - j0;
            emit_shifts(g, R, [&](int k, int sx, int sy, int sz) {
                Task t;
                t.j = J;
                t.j0 = j0;
                t.jc = jc;
                t.self = (J == I && sx == 0 && sy == 0 && sz == 0) ? 1 : 0;
                t.ox = float(org[3 * J] + double(sx) * T.L[0] - oxi);
                t.oy = float(org[3 * J + 1] + double(sy) * T.L[1] - oyi);
                t.oz = float(org[3 * J + 2] + double(sz) * T.L[2] - ozi);
                t.j0b = j0;
                if (emitted + pre + k < wcap)
                    task[wbase + emitted + pre + k] = t;
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
                emit_round(idx < ncur, idx < ncur ? int32_t(front[cur][idx]) : 0);
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
                emit_round(child < n0, child < n0 ? int32_t(child) : 0);
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
                if (child < cnt_dn) {
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
            if (COUNT && lane == 0) {
                overflow[I] = 1;
                count[I] = 0;
            }
            return;
        }
        cur ^= 1;
        ncur = nnext;
    }
    if (COUNT && lane == 0)
        count[I] = emitted;
}

// Compaction of the one-walk rebuild: the tasks of each walked cell that fit
// its slack slot, from the slot to the cell's place in the list (the cells
// that did not fit are walked again, straight into the list).
__global__ __launch_bounds__(64) void k_compact_tasks(int64_t n_leaves,
                                                      const int32_t *__restrict__ soff,
                                                      const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ count,
                                                      const uint8_t *__restrict__ overflow,
                                                      const Task *__restrict__ slack,
                                                      Task *__restrict__ task)
{
    const int64_t I = blockIdx.x;
    if (I >= n_leaves || overflow[I])
        return;
    const int32_t n = count[I], a = soff[I], b = off[I];
    if (n > soff[I + 1] - a)
        return;
    for (int32_t k = threadIdx.x; k < n; k += 64)
        task[b + k] = slack[a + k];
}

// Slot size of a cell in the slack layout: kSlackFactor times its task count
// at the last build, + 8. Roomy slots let the rebuilds inside a step (whose
// radii grow, up to twofold per pass in voids) fit in one walk; measured on
// the clustered box, 4 beats count + 25 % by 2 % per step, for ~6 task records
// per particle of device memory.
constexpr int kSlackFactor = 4;

// Slot sizes of the slack layout from the counts of the last build.
__global__ void k_slack_sizes(int64_t n_leaves, const int32_t *__restrict__ count,
                              int32_t *__restrict__ sz)
{
    const int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (I < n_leaves)
        sz[I] = kSlackFactor * count[I] + 8;
    else if (I == n_leaves)
        sz[I] = 0;
}

}  // namespace

// Launches the walk of mode MODE with the narrowest frontier index type.
template <int MODE>
static void walk_launch(int64_t nl, const TreeView &T, const double *org,
                        const int32_t *leaf_start, const int32_t *off, const int32_t *slot,
                        int32_t *count, uint8_t *overflow, Task *task, hipStream_t s,
                        const uint8_t *only = nullptr)
{
    if (nl <= 65536)
        k_task_bfs<MODE, uint16_t><<<unsigned(nl), 64, 0, s>>>(nl, T, org, leaf_start, off, slot,
                                                              count, overflow, task, only);
    else
        k_task_bfs<MODE, int32_t><<<unsigned(nl), 64, 0, s>>>(nl, T, org, leaf_start, off, slot,
                                                             count, overflow, task, only);
}

size_t tasks_bytes(int64_t n, int leaf_max)
{
    // An estimate (the task count depends on the clustering): one leaf per
    // leaf_max / 4 particles (at least 4) with 96 tasks each, held as the
    // list (allocated with a quarter of headroom), the second list of the
    // growth rebuilds (the same) and the slack layout (kSlackFactor tasks per
    // task + 8 per leaf), plus the per-leaf arrays (offsets twice, counts,
    // radius, order and its sort keys, flags).
    const int64_t leaves = n / std::max(4, leaf_max / 4) + 1;
    const int64_t per_leaf_tasks = 96;
    const int64_t task_slots = 2 * (per_leaf_tasks * 5 / 4) + kSlackFactor * per_leaf_tasks + 8;
    return size_t(leaves) * (size_t(task_slots) * sizeof(Task) + 48) + (1 << 20);
}

void tasks_free(sphx_tasks *t)
{
    if (!t)
        return;
    void *ptrs[] = {t->off, t->task, t->count, t->radius, t->scan_tmp, t->overflow,
                    t->task_alt, t->off_alt, t->dirty};
    for (void *p : ptrs)
        dfree(p, t->stream);
    for (void *p : {(void *)t->order, (void *)t->okey, (void *)t->okey_out, (void *)t->oval,
                    t->sort_tmp, (void *)t->slack, (void *)t->soff})
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
    k_leaf_order_keys<<<unsigned(nbp), 64, 0, s>>>(nl, nbp, t->off, t->task, t->okey, t->oval);
    SPHX_HIP(hipGetLastError());
    size_t tmp = t->sort_tmp_bytes;
    SPHX_HIP(rocprim::radix_sort_pairs(t->sort_tmp, tmp, t->okey, t->okey_out, t->oval, t->order,
                                       size_t(nbp), 0, kOrderKeyBits, s));
    return SPHX_OK;
}

sphx_status tasks_build(sphx_ctx *ctx, sphx_grid *g, const sphx_particles *in, hipStream_t s,
                        sphx_tasks **out)
{
    sphx_tasks *t = *out;
    const int64_t nl = g->n_leaves;
    if (t && t->grid != g) {
        set_error("sphx_tasks_build: task list belongs to another grid");
        return SPHX_E_STATE;
    }
    if (t)
        t->stream = s;
    bool fresh = false;
    if (!t) {
        t = new sphx_tasks();
        t->grid = g;
        t->stream = s;
        fresh = true;
        auto fail = [&](sphx_status st) {
            tasks_free(t);
            return st;
        };
        if (dmalloc((void **)&t->off, (nl + 1) * sizeof(int32_t), s) != hipSuccess ||
            dmalloc((void **)&t->count, (nl + 1) * sizeof(int32_t), s) != hipSuccess ||
            dmalloc((void **)&t->radius, (nl + 1) * sizeof(float), s) != hipSuccess ||
            dmalloc((void **)&t->overflow, (nl + 1) * sizeof(uint8_t), s) != hipSuccess ||
            dmalloc((void **)&t->soff, (nl + 1) * sizeof(int32_t), s) != hipSuccess) {
            set_error("sphx_tasks_build: out of device memory");
            return fail(SPHX_E_OOM);
        }
        size_t tmp = 0;
        if (rocprim::exclusive_scan(nullptr, tmp, t->count, t->off, 0, size_t(nl + 1),
                                    rocprim::plus<int32_t>(), s) != hipSuccess ||
            dmalloc(&t->scan_tmp, tmp + 16, s) != hipSuccess) {
            set_error("sphx_tasks_build: scan workspace");
            return fail(SPHX_E_OOM);
        }
        t->scan_tmp_bytes = tmp;
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
        SPHX_HIP(hipMemsetAsync(t->off, 0, sizeof(int32_t), s));
        guard.keep = true;
        *out = t;
        return SPHX_OK;
    }
    const float scale = float(ctx->p.gamma_k * (1.0 + ctx->p.skin));
    (void)in;
    k_leaf_radius<<<unsigned(nl), 64, 0, s>>>(nl, g->leaf_start, g->hs, scale, g->node_r,
                                              t->radius);
    SPHX_HIP(hipGetLastError());
    for (int l = 0; l + 1 < g->n_levels; ++l) {
        int64_t up = g->level_cnt[l + 1];
        k_tree_radius<<<blocks(up, 128), 128, 0, s>>>(up, g->level_cnt[l],
                                                        g->node_r + g->level_off[l],
                                                        g->node_r + g->level_off[l + 1]);
        SPHX_HIP(hipGetLastError());
    }
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

    auto ensure_task_cap = [&](int64_t total) -> sphx_status {
        if (total > t->cap) {
            dfree(t->task, s);
            t->task = nullptr;
            t->cap = 0;
            const int64_t cap = total + total / 4 + 64;
            SPHX_HIP(dmalloc((void **)&t->task, size_t(cap) * sizeof(Task), s));
            t->cap = cap;
        }
        return SPHX_OK;
    };
    size_t tmp = t->scan_tmp_bytes;
    int32_t total = 0;
    SPHX_HIP(hipMemsetAsync(t->count + nl, 0, sizeof(int32_t), s));
    SPHX_HIP(hipMemsetAsync(t->overflow, 0, size_t(nl) * sizeof(uint8_t), s));
    const bool one_walk = t->slack_ok;
    if (one_walk) {
        // One walk: count every cell's tasks and write them into its slot of
        // the slack layout (slots sized from the previous build's counts).
        walk_launch<2>(nl, T, g->leaf_org, g->leaf_start, t->off, t->soff, t->count,
                       t->overflow, t->slack, s);
    } else {
        walk_launch<0>(nl, T, g->leaf_org, g->leaf_start, t->off, t->soff, t->count,
                       t->overflow, t->task, s);
    }
    SPHX_HIP(hipGetLastError());
    k_task_count<<<blocks(nl, 64), 64, 0, s>>>(nl, T, t->overflow, t->count);
    SPHX_HIP(hipGetLastError());
    SPHX_HIP(rocprim::exclusive_scan(t->scan_tmp, tmp, t->count, t->off, 0, size_t(nl + 1),
                                     rocprim::plus<int32_t>(), s));
    int32_t *h_total = reinterpret_cast<int32_t *>(ctx->h_pinned + kPinnedBytes - 64);
    SPHX_HIP(hipMemcpyAsync(h_total, t->off + nl, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SPHX_HIP(wait_stream(ctx, s));
    total = *h_total;
    if (total < 0) {
        set_error("sphx_tasks_build: task count overflow");
        return SPHX_E_INVALID;
    }
    SPHX_TRY(ensure_task_cap(total));
    t->n_tasks = total;
    if (one_walk) {
        // cells that fitted: from the slot into the list; the others (a few
        // cells whose h grew most) are walked again, writing at their place
        k_compact_tasks<<<unsigned(nl), 64, 0, s>>>(nl, t->soff, t->off, t->count, t->overflow,
                                                    t->slack, t->task);
        SPHX_HIP(hipGetLastError());
        walk_launch<3>(nl, T, g->leaf_org, g->leaf_start, t->off, t->soff, t->count,
                       t->overflow, t->task, s);
    } else {
        walk_launch<1>(nl, T, g->leaf_org, g->leaf_start, t->off, t->soff, t->count,
                       t->overflow, t->task, s);
    }
    SPHX_HIP(hipGetLastError());
    k_task_fill<<<blocks(nl, 64), 64, 0, s>>>(nl, T, g->leaf_org, g->leaf_start, t->overflow,
                                              t->off, t->task);
    SPHX_HIP(hipGetLastError());
    // Slots of the slack layout for the next rebuild, from these counts
    // (kSlackFactor count + 8 per cell); the buffer is sized from the host's
    // bound on their sum, so no readback is needed.
    t->slack_ok = false;
    const int64_t bound = kSlackFactor * int64_t(total) + 8 * nl;
    if (bound <= int64_t(INT32_MAX)) {
        if (bound > t->slack_cap) {
            dfree(t->slack, s);
            t->slack = nullptr;
            t->slack_cap = 0;
            const int64_t want = std::min<int64_t>(bound + bound / 8, int64_t(INT32_MAX));
            if (dmalloc((void **)&t->slack, size_t(want) * sizeof(Task), s) == hipSuccess)
                t->slack_cap = want;
            else
                (void)hipGetLastError();  // no slack: rebuilds keep two walks
        }
        if (t->slack && t->slack_cap >= bound) {
            k_slack_sizes<<<blocks(nl + 1, 256), 256, 0, s>>>(nl, t->count, t->count);
            SPHX_HIP(hipGetLastError());
            SPHX_HIP(rocprim::exclusive_scan(t->scan_tmp, tmp, t->count, t->soff, 0,
                                             size_t(nl + 1), rocprim::plus<int32_t>(), s));
            t->slack_ok = true;
        }
    }
    SPHX_TRY(leaf_order(t, nl, s));
    t->symmetric = true;
    guard.keep = true;
    *out = t;
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
    return T;
}

sphx_status tasks_grow(sphx_ctx *ctx, sphx_grid *g, const sphx_particles *in, hipStream_t s,
                       sphx_tasks **out)
{
    sphx_tasks *t = *out;
    const int64_t nl = g->n_leaves;
    if (!t || t->grid != g || !t->slack_ok || nl == 0)
        return tasks_build(ctx, g, in, s, out);
    t->stream = s;
    if (!t->off_alt) {
        if (dmalloc((void **)&t->off_alt, (nl + 1) * sizeof(int32_t), s) != hipSuccess ||
            dmalloc((void **)&t->dirty, (nl + 1) * sizeof(uint8_t), s) != hipSuccess) {
            set_error("sphx_tasks_build: out of device memory (growth rebuild)");
            return SPHX_E_OOM;
        }
    }
    const float scale = float(ctx->p.gamma_k * (1.0 + ctx->p.skin));
    k_leaf_radius_grow<<<unsigned(nl), 64, 0, s>>>(nl, g->leaf_start, g->hs, scale, g->node_r,
                                                   t->radius, t->overflow, t->dirty);
    SPHX_HIP(hipGetLastError());
    for (int l = 0; l + 1 < g->n_levels; ++l) {
        int64_t up = g->level_cnt[l + 1];
        k_tree_radius<<<blocks(up, 128), 128, 0, s>>>(up, g->level_cnt[l],
                                                        g->node_r + g->level_off[l],
                                                        g->node_r + g->level_off[l + 1]);
        SPHX_HIP(hipGetLastError());
    }
    const TreeView T = tree_view(ctx, g);
    // the marked leaves: one walk into their slots, counting; the serial
    // count for those whose frontier overflowed; the others keep theirs
    walk_launch<2>(nl, T, g->leaf_org, g->leaf_start, t->off, t->soff, t->count, t->overflow,
                   t->slack, s, t->dirty);
    SPHX_HIP(hipGetLastError());
    k_task_count<<<blocks(nl, 64), 64, 0, s>>>(nl, T, t->overflow, t->count);
    SPHX_HIP(hipGetLastError());
    k_keep_counts<<<blocks(nl + 1, 256), 256, 0, s>>>(nl, t->dirty, t->off, t->count);
    SPHX_HIP(hipGetLastError());
    size_t tmp = t->scan_tmp_bytes;
    SPHX_HIP(rocprim::exclusive_scan(t->scan_tmp, tmp, t->count, t->off_alt, 0, size_t(nl + 1),
                                     rocprim::plus<int32_t>(), s));
    int32_t *h_total = reinterpret_cast<int32_t *>(ctx->h_pinned + kPinnedBytes - 64);
    SPHX_HIP(hipMemcpyAsync(h_total, t->off_alt + nl, sizeof(int32_t), hipMemcpyDeviceToHost,
                            s));
    SPHX_HIP(wait_stream(ctx, s));
    const int32_t total = *h_total;
    if (total < 0) {
        set_error("sphx_tasks_build: task count overflow");
        return SPHX_E_INVALID;
    }
    if (total > t->cap_alt) {
        dfree(t->task_alt, s);
        t->task_alt = nullptr;
        t->cap_alt = 0;
        const int64_t cap = int64_t(total) + total / 4 + 64;
        SPHX_HIP(dmalloc((void **)&t->task_alt, size_t(cap) * sizeof(Task), s));
        t->cap_alt = cap;
    }
    k_copy_grown<<<unsigned(nl), 64, 0, s>>>(nl, t->dirty, t->overflow, t->off, t->off_alt,
                                             t->soff, t->count, t->task, t->slack, t->task_alt);
    SPHX_HIP(hipGetLastError());
    // marked leaves over their slot: walked again straight into the list;
    // those with an overflowed frontier: the serial fill
    walk_launch<3>(nl, T, g->leaf_org, g->leaf_start, t->off_alt, t->soff, t->count,
                   t->overflow, t->task_alt, s, t->dirty);
    SPHX_HIP(hipGetLastError());
    k_task_fill<<<blocks(nl, 64), 64, 0, s>>>(nl, T, g->leaf_org, g->leaf_start, t->overflow,
                                              t->off_alt, t->task_alt);
    SPHX_HIP(hipGetLastError());
    std::swap(t->task, t->task_alt);
    std::swap(t->cap, t->cap_alt);
    std::swap(t->off, t->off_alt);
    t->n_tasks = total;
    // (the launch order of the last full build stays: it orders by work,
    // which the few walked leaves hardly move)
    t->symmetric = false;
    return SPHX_OK;
}

}  // namespace sphx
