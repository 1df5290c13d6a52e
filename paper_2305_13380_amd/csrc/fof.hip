// Friends-of-friends groups (Section 9.1): pairs of particles closer than the
// linking length b are linked and the groups are the connected components of
// the links, found with union-find. The pair search reuses the cell structure
// of the neighbour loops, built with b as the search radius: every pair within
// b lies in a self or pair task of its cells.
//
// The link test is taken in FP64 on the caller's positions, with exactly the
// operations of the definition: d = x_i - x_j, the minimum image d - L k
// (k = nearest integer of d / L), r^2 = (dx^2 + dy^2) + dz^2 < b^2 (no
// contraction into fused multiply-adds, so every product and sum rounds as
// written). k is the task's own periodic shift, recovered exactly from its
// offset: a task whose shift is not the nearest image puts the pair at least
// L/2 > b apart, so each linked pair is decided, and counted, once.
#include <algorithm>
#include <climits>

#include "sphx_internal.h"

#pragma clang fp contract(off)

namespace sphx {
namespace {

constexpr int kFofThreads = 256;

__device__ __forceinline__ int32_t ld_relaxed(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of i's set, halving the path on the way. A parent is always a smaller
// index than its child (unions hang the larger root under the smaller, the
// halving replaces a parent by the grandparent), so every step moves to a
// smaller index and the walk ends.
__device__ int32_t find_root(int32_t *parent, int32_t i)
{
    for (;;) {
        const int32_t p = ld_relaxed(parent + i);
        if (p == i)
            return i;
        const int32_t g = ld_relaxed(parent + p);
        if (g != p)
            st_relaxed(parent + i, g);
        i = g;
    }
}

// Merge the sets of a and b: the larger root is hung under the smaller by a
// compare-and-swap that succeeds only while it is still a root. A failed swap
// means that root was hung under a smaller index meanwhile; the loop goes
// on from there, so the roots only decrease and the loop ends.
__device__ void unite(int32_t *parent, int32_t a, int32_t b)
{
    for (;;) {
        a = find_root(parent, a);
        b = find_root(parent, b);
        if (a == b)
            return;
        if (a > b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        const int32_t old = atomicCAS(parent + b, b, a);
        if (old == b)
            return;
        b = old;
    }
}

__global__ void k_fill_h(int64_t n, float hv, float *__restrict__ h)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        h[i] = hv;
}

__global__ void k_fof_fill(int64_t n, int32_t *__restrict__ parent, int32_t *__restrict__ minc,
                           int32_t *__restrict__ size)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    parent[i] = int32_t(i);
    minc[i] = INT_MAX;
    size[i] = 0;
}

__global__ void k_fof_zero(int64_t *counts)
{
    if (threadIdx.x < 2)
        counts[threadIdx.x] = 0;
}

// One wave per receiving leaf, one receiver per lane; for every task, the
// source leaf's positions are staged in LDS and every lane tests the sources
// that come after its receiver in sorted order (each unordered pair once).
__global__ __launch_bounds__(64) void k_fof_link(int64_t n_leaves,
                                                const int32_t *__restrict__ leaf_start,
                                                const double *__restrict__ org,
                                                const int32_t *__restrict__ perm,
                                                const double *__restrict__ x,
                                                const double *__restrict__ y,
                                                const double *__restrict__ z, double Lx,
                                                double Ly, double Lz, int periodic, double b2,
                                                const int32_t *__restrict__ tbeg,
    const int32_t *__restrict__ tend,
                                                const Task *__restrict__ task,
                                                int32_t *__restrict__ parent,
                                                unsigned long long *__restrict__ links)
{
    const int64_t L = blockIdx.x;
    if (L >= n_leaves)
        return;
    const int lane = threadIdx.x;
    const int32_t s0 = leaf_start[L], cnt = leaf_start[L + 1] - s0;
    const bool valid = lane < cnt;
    const int32_t si = s0 + (valid ? lane : 0);
    const int32_t ci = perm[si];
    const double xi = x[ci], yi = y[ci], zi = z[ci];
    const double oix = org[3 * L], oiy = org[3 * L + 1], oiz = org[3 * L + 2];
    __shared__ double sx[kLeafMax], sy[kLeafMax], sz[kLeafMax];
    unsigned long long nl = 0;
    const int32_t ta = tbeg[L], tb = tend[L];
    for (int32_t t = ta; t < tb; ++t) {
        const Task tk = task[t];
        // no source after every receiver of this leaf: nothing to test
        if (tk.j0 + tk.jc - 1 <= s0)
            continue;
        // the task's shift in box lengths: offset = org_j + k L - org_i
        double kx = 0.0, ky = 0.0, kz = 0.0;
        if (periodic) {
            kx = rint((double(tk.ox) - (org[3 * tk.j] - oix)) / Lx);
            ky = rint((double(tk.oy) - (org[3 * tk.j + 1] - oiy)) / Ly);
            kz = rint((double(tk.oz) - (org[3 * tk.j + 2] - oiz)) / Lz);
        }
        const double lx = Lx * kx, ly = Ly * ky, lz = Lz * kz;
        __syncthreads();
        if (lane < tk.jc) {
            const int32_t cj = perm[tk.j0 + lane];
            sx[lane] = x[cj];
            sy[lane] = y[cj];
            sz[lane] = z[cj];
        }
        __syncthreads();
        if (!valid)
            continue;
        for (int k = 0; k < tk.jc; ++k) {
            const int32_t sj = tk.j0 + k;
            if (sj <= si)
                continue;
            const double dx = (xi - sx[k]) - lx;
            const double dy = (yi - sy[k]) - ly;
            const double dz = (zi - sz[k]) - lz;
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < b2) {
                ++nl;
                unite(parent, si, sj);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1)
        nl += __shfl_xor(nl, o, 64);
    if (lane == 0 && nl)
        atomicAdd(links, nl);
}

// Every particle points straight at its root; per root, the smallest caller
// index of its members, the member count, and one count per group.
__global__ void k_fof_label(int64_t n, const int32_t *__restrict__ perm,
                            int32_t *__restrict__ parent, int32_t *__restrict__ minc,
                            int32_t *__restrict__ size, unsigned long long *__restrict__ groups)
{
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    const int32_t r = find_root(parent, int32_t(s));
    atomicMin(minc + r, perm[s]);
    atomicAdd(size + r, 1);
    if (r == int32_t(s))
        atomicAdd(groups, 1ull);
}

// Walks to the root again rather than trusting a pointer written in the
// label pass: the path halving of another thread's walk there may read a
// particle's old parent before the particle points at its root and write an
// older ancestor over it afterwards (tried; one particle of 20,000 lost its
// group).
__global__ void k_fof_out(int64_t n, const int32_t *__restrict__ perm,
                          int32_t *__restrict__ parent, const int32_t *__restrict__ minc,
                          const int32_t *__restrict__ size, int32_t *__restrict__ group,
                          int32_t *__restrict__ group_size)
{
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    const int32_t r = find_root(parent, int32_t(s));
    const int32_t i = perm[s];
    group[i] = minc[r];
    if (group_size)
        group_size[i] = size[r];
}

}  // namespace

SearchCells::~SearchCells()
{
    if (t)
        tasks_free(t);
    if (g)
        grid_free(g);
    dfree(h, s);
}

sphx_status search_cells_build(sphx_ctx *ctx, const sphx_particles *in, double radius,
                               hipStream_t s, SearchCells &sc)
{
    const int64_t n = in->n;
    sc.s = s;
    // h such that the search radius gamma_k h covers `radius` (a relative
    // margin of 2^-20 absorbs the FP32 rounding of h)
    const float hv = float(radius / ctx->p.gamma_k * (1.0 + 1.0 / 1048576.0));
    if (dmalloc((void **)&sc.h, size_t(n) * sizeof(float), s) != hipSuccess) {
        (void)hipGetLastError();
        sc.h = nullptr;
        set_error("device allocation failed");
        return SPHX_E_OOM;
    }
    k_fill_h<<<unsigned((n + kFofThreads - 1) / kFofThreads), kFofThreads, 0, s>>>(n, hv, sc.h);
    SPHX_HIP(hipGetLastError());
    sphx_particles tmp = *in;
    tmp.h = sc.h;
    tmp.active = nullptr;  // every particle takes part
    SPHX_TRY(grid_build(ctx, &tmp, s, &sc.g));
    SPHX_TRY(refresh_h(sc.g, &tmp, s));
    return tasks_build(ctx, sc.g, &tmp, s, &sc.t);
}

sphx_status fof_run(sphx_ctx *ctx, const sphx_particles *in, double b, int32_t *group,
                    int32_t *group_size, int64_t *d_counts, hipStream_t s)
{
    const int64_t n = in->n;
    if (d_counts) {
        k_fof_zero<<<1, 64, 0, s>>>(d_counts);
        SPHX_HIP(hipGetLastError());
    }
    if (n == 0)
        return SPHX_OK;
    // one workspace: two count words (used when the caller gives none), then
    // parent, smallest caller index and size per particle
    unsigned char *ws = nullptr;
    if (dmalloc((void **)&ws, 16 + size_t(n) * 3 * sizeof(int32_t), s) != hipSuccess) {
        (void)hipGetLastError();
        set_error("sphx_fof: device allocation failed");
        return SPHX_E_OOM;
    }
    struct Scratch {
        void *a;
        hipStream_t s;
        ~Scratch() { dfree(a, s); }
    } scratch{ws, s};
    unsigned long long *own = reinterpret_cast<unsigned long long *>(ws);
    int32_t *parent = reinterpret_cast<int32_t *>(ws + 16), *minc = parent + n,
            *size = parent + 2 * n;
    const unsigned nb = unsigned((n + kFofThreads - 1) / kFofThreads);
    k_fof_fill<<<nb, kFofThreads, 0, s>>>(n, parent, minc, size);
    SPHX_HIP(hipGetLastError());
    SearchCells sc;
    SPHX_TRY(search_cells_build(ctx, in, b, s, sc));
    const sphx_grid *g = sc.g;
    const sphx_tasks *t = sc.t;

    // group and link counts: into the caller's array, else the private words
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(d_counts);
    if (!cnt) {
        k_fof_zero<<<1, 64, 0, s>>>(reinterpret_cast<int64_t *>(own));
        SPHX_HIP(hipGetLastError());
        cnt = own;
    }
    unsigned long long *groups = cnt, *links = cnt + 1;
    k_fof_link<<<unsigned(g->n_leaves), 64, 0, s>>>(
        g->n_leaves, g->leaf_start, g->leaf_org, g->perm, in->x, in->y, in->z, ctx->p.box[0],
        ctx->p.box[1], ctx->p.box[2], ctx->p.periodic, b * b, t->slot, t->end, t->task, parent,
        links);
    SPHX_HIP(hipGetLastError());
    k_fof_label<<<nb, kFofThreads, 0, s>>>(n, g->perm, parent, minc, size, groups);
    SPHX_HIP(hipGetLastError());
    k_fof_out<<<nb, kFofThreads, 0, s>>>(n, g->perm, parent, minc, size, group, group_size);
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

}  // namespace sphx
