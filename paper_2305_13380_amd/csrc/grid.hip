// Grid build: Morton sort and leaf cells (Section 2.2 nested grids; Section
// 9.1 depth-first binning, here as a radix sort on a 63-bit Morton key, whose
// order is a depth-first order of the octree).
#include <algorithm>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>

#include "pairs.h"

namespace sphx {
namespace {

__device__ __forceinline__ double wrap_coord(double x, double L, int periodic)
{
    if (!periodic)
        return x;
    double w = x - L * floor(x / L);
    return w >= L ? w - L : w;  // floor rounding can leave w == L
}

// Spread the low 21 bits of v so that bit k moves to bit 3k.
__device__ __forceinline__ uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ __forceinline__ uint64_t quantise(double x, double L)
{
    double q = floor(x / L * double(1 << kMortonBits));
    if (!(q >= 0.0))
        q = 0.0;
    const double top = double((1 << kMortonBits) - 1);
    if (q > top)
        q = top;
    return uint64_t(q);
}

// Validate the inputs and compute the Morton keys of the wrapped positions.
__global__ void k_keys(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                       const double *__restrict__ z, const float *__restrict__ h,
                       const float *__restrict__ m, const float *__restrict__ u, float h_max,
                       double Lx, double Ly, double Lz, int periodic, uint64_t *__restrict__ keys,
                       int32_t *__restrict__ idx, int32_t *__restrict__ bad)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    double px = x[i], py = y[i], pz = z[i];
    float hi = h[i], mi = m[i], ui = u[i];
    bool ok = isfinite(px) && isfinite(py) && isfinite(pz) && isfinite(hi) && hi > 0.0f &&
              hi <= h_max &&
              isfinite(mi) && mi > 0.0f && isfinite(ui) && ui >= 0.0f;
    if (!periodic)
        ok = ok && px >= 0.0 && px < Lx && py >= 0.0 && py < Ly && pz >= 0.0 && pz < Lz;
    if (!ok)
        atomicAdd(bad, 1);
    px = wrap_coord(px, Lx, periodic);
    py = wrap_coord(py, Ly, periodic);
    pz = wrap_coord(pz, Lz, periodic);
    uint64_t k = (spread3(quantise(px, Lx)) << 2) | (spread3(quantise(py, Ly)) << 1) |
                 spread3(quantise(pz, Lz));
    keys[i] = k;
    idx[i] = int32_t(i);
}

// Number of leading 3-bit levels two Morton keys share (21 when equal).
__device__ __forceinline__ int common_levels(uint64_t a, uint64_t b)
{
    uint64_t d = a ^ b;
    int c = d ? (__clzll(int64_t(d)) - 1) / 3 : kMortonBits;
    return c > kMortonBits ? kMortonBits : c;
}

// Index of the first position in [lo, hi) whose key prefix (key >> shift) is
// >= p (keys are sorted, so prefixes are non-decreasing).
__device__ __forceinline__ int64_t lower_prefix(const uint64_t *k, int64_t lo, int64_t hi,
                                                uint64_t p, int shift)
{
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((k[mid] >> shift) < p)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Leaf cells are the maximal aligned octree blocks holding <= cap particles.
// Sorted positions s-1 and s share a leaf exactly when their deepest common
// octree block holds <= cap particles; that block's population is measured
// inside a window of 2 cap + 2 sorted keys around s (a population above cap
// always shows as more than cap keys inside the window).
// With several particle sets (set_of non-null) each set is split on its own:
// its first particle starts a leaf and the windows stay inside the set.
__global__ void k_leaf_flags(int64_t n, const uint64_t *__restrict__ k, int cap,
                             uint32_t *__restrict__ flag, const int32_t *__restrict__ set_of,
                             const int32_t *__restrict__ set_start)
{
    int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    int64_t lo_b = 0, hi_b = n;
    if (set_of) {
        const int32_t b = set_of[s];
        lo_b = set_start[b];
        hi_b = set_start[b + 1];
    }
    if (s == lo_b) {
        flag[s] = 1;
        return;
    }
    const uint64_t b = k[s];
    const int shift = 3 * (kMortonBits - common_levels(k[s - 1], b));
    const uint64_t p = b >> shift;
    int64_t wlo = s - 1 - cap;
    if (wlo < lo_b)
        wlo = lo_b;
    int64_t whi = s + cap + 1;
    if (whi > hi_b)
        whi = hi_b;
    int64_t lo = lower_prefix(k, wlo, s, p, shift);
    int64_t hi = lower_prefix(k, s, whi, p + 1, shift);
    flag[s] = (hi - lo > cap) ? 1u : 0u;
}

// leaf_of[s] = inclusive_scan(flag)[s] - 1; leaf_start[leaf] = first s.
__global__ void k_leaf_index(int64_t n, const uint32_t *__restrict__ flag,
                             const uint32_t *__restrict__ incl, int32_t *__restrict__ leaf_of,
                             int32_t *__restrict__ leaf_start, int32_t *__restrict__ n_leaves)
{
    int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    int32_t L = int32_t(incl[s]) - 1;
    leaf_of[s] = L;
    if (flag[s])
        leaf_start[L] = int32_t(s);
    if (s == n - 1) {
        leaf_start[L + 1] = int32_t(n);
        *n_leaves = L + 1;
    }
}

// Start of every octree leaf: oct_start[leaf] = first sorted index.
__global__ void k_oct_index(int64_t n, const uint32_t *__restrict__ flag,
                            const uint32_t *__restrict__ incl, int32_t *__restrict__ oct_start,
                            int32_t *__restrict__ n_oct)
{
    int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    if (flag[s])
        oct_start[incl[s] - 1] = int32_t(s);
    if (s == n - 1) {
        oct_start[incl[s]] = int32_t(n);
        *n_oct = int32_t(incl[s]);
    }
}

// Parent block of every octree leaf: the deeper of the deepest common blocks
// across its two boundaries (both hold more than cap particles; the deeper
// one is the leaf's parent). Level -1: the leaf is the whole set.
__global__ void k_oct_parent(int64_t n, const uint64_t *__restrict__ k,
                             const int32_t *__restrict__ oct_start,
                             const int32_t *__restrict__ n_oct, int32_t *__restrict__ par_lvl,
                             uint64_t *__restrict__ par_pfx, const int32_t *__restrict__ set_of,
                             const int32_t *__restrict__ set_start)
{
    int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= *n_oct)
        return;
    int64_t a = oct_start[q], b = oct_start[q + 1];
    int64_t lo_b = 0, hi_b = n;  // the leaf's set (a set's ends are like the array's)
    if (set_of) {
        const int32_t st = set_of[a];
        lo_b = set_start[st];
        hi_b = set_start[st + 1];
    }
    int lv = -1;
    if (a > lo_b)
        lv = common_levels(k[a - 1], k[a]);
    if (b < hi_b) {
        int l2 = common_levels(k[b - 1], k[b]);
        lv = l2 > lv ? l2 : lv;
    }
    par_lvl[q] = lv;
    par_pfx[q] = lv < 0 ? 0 : (k[a] >> (3 * (kMortonBits - lv)));
}

// Cells: runs of consecutive sibling octree leaves packed greedily up to cap
// particles (siblings share one parent block, so a cell stays compact).
// Leaves of one parent are at most 8, except below the finest key level
// (identical keys), where they are single particles packed by position.
__global__ void k_pack_cells(int64_t n, const uint64_t *__restrict__ k,
                             const int32_t *__restrict__ oct_start,
                             const int32_t *__restrict__ n_oct,
                             const int32_t *__restrict__ par_lvl,
                             const uint64_t *__restrict__ par_pfx,
                             const uint32_t *__restrict__ oct_incl, int cap,
                             uint32_t *__restrict__ cell_flag,
                             const int32_t *__restrict__ set_of,
                             const int32_t *__restrict__ set_start)
{
    int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= *n_oct)
        return;
    const int lv = par_lvl[q];
    const uint64_t pf = par_pfx[q];
    const int32_t my_set = set_of ? set_of[oct_start[q]] : 0;
    bool start;
    if (lv == kMortonBits) {
        // identical keys: leaves are single particles
        int64_t a = oct_start[q];
        int64_t lo = set_of ? set_start[my_set] : 0, hi = a;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (k[mid] < k[a])
                lo = mid + 1;
            else
                hi = mid;
        }
        int64_t run_first_leaf = int64_t(oct_incl[lo]) - 1;
        start = ((q - run_first_leaf) % cap) == 0;
    } else {
        int64_t r = q;
        while (r > 0 && q - r < 8 && par_lvl[r - 1] == lv && par_pfx[r - 1] == pf && lv >= 0 &&
               (!set_of || set_of[oct_start[r - 1]] == my_set))
            --r;
        int acc = 0;
        start = true;
        for (int64_t t = r; t <= q; ++t) {
            int sz = oct_start[t + 1] - oct_start[t];
            if (t == r || acc + sz > cap) {
                acc = sz;
                start = true;
            } else {
                acc += sz;
                start = false;
            }
        }
    }
    cell_flag[oct_start[q]] = start ? 1u : 0u;
}

__device__ __forceinline__ double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// One wave per leaf: FP64 bounding box of the leaf's particles (origin = min
// corner), then each particle's FP32 position relative to that origin and the
// sorted copies of the other inputs.
__global__ __launch_bounds__(64) void k_leaf_setup(
    int64_t n_leaves, const int32_t *__restrict__ leaf_start, const int32_t *__restrict__ perm,
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    const float *__restrict__ vx, const float *__restrict__ vy, const float *__restrict__ vz,
    const float *__restrict__ m, const float *__restrict__ u, const float *__restrict__ av,
    const float *__restrict__ ac, double Lx, double Ly, double Lz, int periodic,
    double *__restrict__ org, double *__restrict__ node_lo, double *__restrict__ node_hi,
    float4 *__restrict__ q0, float4 *__restrict__ q1, float2 *__restrict__ qa,
    float4 *__restrict__ ext)
{
    int64_t L = blockIdx.x;
    if (L >= n_leaves)
        return;
    int lane = threadIdx.x;
    int32_t s0 = leaf_start[L], cnt = leaf_start[L + 1] - s0;
    bool valid = lane < cnt;
    int32_t s = s0 + (valid ? lane : 0);
    int32_t i = perm[s];
    double px = wrap_coord(x[i], Lx, periodic);
    double py = wrap_coord(y[i], Ly, periodic);
    double pz = wrap_coord(z[i], Lz, periodic);
    double lox = wave_min(px), loy = wave_min(py), loz = wave_min(pz);
    double hix = wave_max(px), hiy = wave_max(py), hiz = wave_max(pz);
    if (lane == 0) {
        org[3 * L + 0] = lox;
        org[3 * L + 1] = loy;
        org[3 * L + 2] = loz;
        node_lo[3 * L + 0] = lox;
        node_lo[3 * L + 1] = loy;
        node_lo[3 * L + 2] = loz;
        node_hi[3 * L + 0] = hix;
        node_hi[3 * L + 1] = hiy;
        node_hi[3 * L + 2] = hiz;
    }
    const float fx = float(px - lox), fy = float(py - loy), fz = float(pz - loz);
    if (valid) {
        q0[s] = make_float4(fx, fy, fz, m[i]);
        q1[s] = make_float4(vx[i], vy[i], vz[i], u[i]);
        qa[s] = make_float2(av[i], ac[i]);
    }
    // the cell's extent in its own frame, from the stored FP32 coordinates
    const float ex = wave_maxf(valid ? fx : 0.0f), ey = wave_maxf(valid ? fy : 0.0f),
                ez = wave_maxf(valid ? fz : 0.0f);
    if (lane == 0)
        ext[L] = make_float4(ex, ey, ez, 0.0f);
}

// Tree over the leaves: node c of level l+1 covers nodes [8c, 8c+8) of level l.
__global__ void k_tree_level(int64_t cnt_up, int64_t cnt_dn, const double *__restrict__ lo_dn,
                             const double *__restrict__ hi_dn, double *__restrict__ lo_up,
                             double *__restrict__ hi_up)
{
    int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= cnt_up)
        return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int64_t e = (c + 1) * kTreeFan;
    if (e > cnt_dn)
        e = cnt_dn;
    for (int64_t k = c * kTreeFan; k < e; ++k)
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], lo_dn[3 * k + a]);
            hi[a] = fmax(hi[a], hi_dn[3 * k + a]);
        }
    for (int a = 0; a < 3; ++a) {
        lo_up[3 * c + a] = lo[a];
        hi_up[3 * c + a] = hi[a];
    }
}

// Start of an h iteration: mark the active particles and copy h into sorted
// order (with mark == nullptr only the copy).
// The inverse of the sort's permutation: caller index -> sorted index.
// Set of every sorted particle (sets keep their ranges through the sort):
// the last b with set_start[b] <= s.
__global__ void k_set_of(int64_t n, const int32_t *__restrict__ set_start, int32_t n_sets,
                         int32_t *__restrict__ set_of)
{
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    int32_t lo = 0, hi = n_sets;  // set_start[lo] <= s < set_start[hi]
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (set_start[mid] <= s)
            lo = mid;
        else
            hi = mid;
    }
    set_of[s] = lo;
}

// First leaf of every set (an empty set: the next set's first leaf) and the
// set of every leaf.
__global__ void k_set_leaves(int64_t n, int32_t n_sets, const int32_t *__restrict__ set_start,
                             const int32_t *__restrict__ leaf_of,
                             const int32_t *__restrict__ leaf_start,
                             const int32_t *__restrict__ set_of,
                             const int32_t *__restrict__ n_leaves,
                             int32_t *__restrict__ set_leaf, int32_t *__restrict__ leaf_set)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int32_t nl = *n_leaves;
    if (i <= n_sets)
        set_leaf[i] = set_start[i] < n ? leaf_of[set_start[i]] : nl;
    if (i < nl)
        leaf_set[i] = set_of[leaf_start[i]];
}

__global__ void k_invert(int64_t n, const int32_t *__restrict__ perm, int32_t *__restrict__ inv)
{
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s < n)
        inv[perm[s]] = int32_t(s);
}

__global__ void k_iter_reset(int64_t n, const int32_t *__restrict__ perm,
                             const uint8_t *__restrict__ active, const float *__restrict__ h,
                             uint8_t *__restrict__ need, float *__restrict__ hs,
                             float *__restrict__ hlo, float *__restrict__ hhi)
{
    int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    const int32_t i = perm[s];
    hs[s] = h[i];
    if (need) {
        need[s] = active ? (active[i] ? 1 : 0) : 1;
        hlo[s] = 0.0f;
        hhi[s] = __builtin_inff();
    }
}

template <class T>
sphx_status dalloc(T **p, size_t count, hipStream_t s)
{
    *p = nullptr;
    if (count == 0)
        count = 1;
    SPHX_HIP(dmalloc((void **)p, count * sizeof(T), s));
    return SPHX_OK;
}

inline unsigned blocks(int64_t n, int t) { return unsigned((n + t - 1) / t); }

// A buffer of the grid. With recycle_workspace: a spare of the context
// (freed there on this stream) whose size lies in [bytes, 2 bytes], the
// smallest such, else a new allocation; either way recorded in g->owned.
template <class T>
sphx_status galloc(sphx_grid *g, T **p, size_t count, hipStream_t s)
{
    *p = nullptr;
    if (count == 0)
        count = 1;
    const size_t bytes = count * sizeof(T);
    if (!g->recycle) {
        SPHX_HIP(dmalloc((void **)p, bytes, s));
        return SPHX_OK;
    }
    auto &sp = g->ctx->spare;
    if (s == g->ctx->spare_stream) {
        size_t pick = sp.size();
        for (size_t k = 0; k < sp.size(); ++k) {
            const size_t b = sp[k].second;
            if (b >= bytes && b / 2 <= bytes && (pick == sp.size() || b < sp[pick].second))
                pick = k;
        }
        if (pick < sp.size()) {
            *p = static_cast<T *>(sp[pick].first);
            g->owned.push_back(sp[pick]);
            sp.erase(sp.begin() + pick);
            return SPHX_OK;
        }
    }
    SPHX_HIP(dmalloc((void **)p, bytes, s));
    g->owned.emplace_back(static_cast<void *>(*p), bytes);
    return SPHX_OK;
}

}  // namespace

void release_spares(sphx_ctx *ctx)
{
    for (auto &b : ctx->spare)
        dfree(b.first, ctx->spare_stream);
    ctx->spare.clear();
}

size_t grid_bytes(int64_t n)
{
    // per particle: keys x2, perm/idx, leaf_of, flags x2, q0, q1, qa, need, g0, g1, g2,
    // hs, d0 + d1, hlo + hhi, d2 (pressure-energy)
    size_t per = 8 * 2 + 4 * 2 + 4 + 4 * 2 + 16 * 2 + 8 + 1 + 16 * 3 + 4 + 32 + 8 + 8;
    // per leaf (at most n leaves): start, origin, tree nodes (~8/7 of the
    // leaves: lo, hi, radius), partial sums
    size_t per_leaf = 4 + 24 + 16 + 4 + (48 + 4) * 8 / 7 + 1 + 48;
    size_t sort_tmp = size_t(n) * 16 + (1 << 20);
    return size_t(n) * (per + per_leaf) + sort_tmp + (1 << 16);
}

void grid_free(sphx_grid *g)
{
    if (!g)
        return;
    if (g->recycle) {
        // the grid's own buffers become the context's spares (an older
        // grid's leftovers are freed first); the rest is freed below
        release_spares(g->ctx);
        g->ctx->spare = std::move(g->owned);
        g->ctx->spare_stream = g->stream;
    }
    auto spare = [&](void *p) {
        if (!g->recycle)
            return false;
        for (auto &b : g->ctx->spare)
            if (b.first == p)
                return true;
        return false;
    };
    void *ptrs[] = {g->keys,    g->perm,     g->leaf_of,  g->q0,      g->q1,     g->qa,
                    g->need,    g->g0,       g->g1,       g->g2,       g->leaf_start, g->leaf_org,
                    g->node_lo,
                    g->node_hi, g->node_r,   g->fsum,     g->sort_tmp, g->keys_in, g->idx_in,
                    g->flags,   g->d_status, g->hs,       g->d0,       g->d1,     g->d2,
                    g->lrad,    g->lcnt,     g->lcap,     g->lboff,    g->lst,    g->lscan_tmp,
                    g->leaf_ext, g->leaf_hmax, g->hlo, g->hhi, g->set_start, g->set_of,
                    g->set_leaf, g->leaf_set};
    for (void *p : ptrs)
        if (!spare(p))
            dfree(p, g->stream);
    delete g;
}

sphx_status iter_reset(sphx_grid *g, const sphx_particles *in, hipStream_t s)
{
    if (g->n == 0)
        return SPHX_OK;
    k_iter_reset<<<blocks(g->n, 256), 256, 0, s>>>(g->n, g->perm, in->active, in->h, g->need,
                                                    g->hs, g->hlo, g->hhi);
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

sphx_status refresh_h(sphx_grid *g, const sphx_particles *in, hipStream_t s)
{
    if (g->n == 0)
        return SPHX_OK;
    k_iter_reset<<<blocks(g->n, 256), 256, 0, s>>>(g->n, g->perm, in->active, in->h, nullptr,
                                                    g->hs, nullptr, nullptr);
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

sphx_status grid_build(sphx_ctx *ctx, const sphx_particles *in, hipStream_t s, sphx_grid **out,
                       const int64_t *sets, int32_t n_sets)
{
    const sphx_params &P = ctx->p;
    const int64_t n = in->n;
    sphx_grid *g = new sphx_grid();
    g->serial = next_serial();
    *out = nullptr;
    g->ctx = ctx;
    g->stream = s;
    g->n = n;
    g->n_sets = sets ? n_sets : 1;
    g->recycle = P.recycle_workspace != 0;
    struct Guard {
        sphx_grid *g;
        bool keep = false;
        ~Guard()
        {
            if (!keep)
                grid_free(g);
        }
    } guard{g};

    SPHX_TRY(galloc(g, &g->d_status, 4, s));
    SPHX_HIP(hipMemsetAsync(g->d_status, 0, 4 * sizeof(int32_t), s));
    SPHX_TRY(galloc(g, &g->keys, n, s));
    SPHX_TRY(galloc(g, &g->keys_in, n, s));
    SPHX_TRY(galloc(g, &g->perm, n, s));
    SPHX_TRY(galloc(g, &g->idx_in, n, s));
    SPHX_TRY(galloc(g, &g->leaf_of, n, s));
    SPHX_TRY(galloc(g, &g->flags, 2 * n, s));
    SPHX_TRY(galloc(g, &g->q0, n, s));
    SPHX_TRY(galloc(g, &g->q1, n, s));
    SPHX_TRY(galloc(g, &g->qa, n, s));
    SPHX_TRY(galloc(g, &g->need, n, s));
    SPHX_TRY(galloc(g, &g->g0, n, s));
    SPHX_TRY(galloc(g, &g->g1, n, s));
    SPHX_TRY(galloc(g, &g->g2, n, s));
    SPHX_TRY(galloc(g, &g->hs, n, s));
    SPHX_TRY(galloc(g, &g->hlo, n, s));
    SPHX_TRY(galloc(g, &g->hhi, n, s));
    SPHX_TRY(galloc(g, &g->d0, n, s));
    SPHX_TRY(galloc(g, &g->d1, n, s));
    if (smoothed_pressure(P.flavour))
        SPHX_TRY(galloc(g, &g->d2, n, s));
    if (sets) {
        std::vector<int32_t> h_sets(size_t(n_sets) + 1);
        for (int32_t b = 0; b <= n_sets; ++b)
            h_sets[b] = int32_t(sets[b]);
        SPHX_TRY(galloc(g, &g->set_start, n_sets + 1, s));
        SPHX_TRY(galloc(g, &g->set_leaf, n_sets + 1, s));
        SPHX_HIP(hipMemcpyAsync(g->set_start, h_sets.data(), h_sets.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, s));
        // (the copy reads the host array before this call returns)
        SPHX_HIP(hipStreamSynchronize(s));
    }

    if (n == 0) {
        g->n_leaves = 0;
        g->n_levels = 0;
        SPHX_TRY(galloc(g, &g->leaf_start, 1, s));
        SPHX_HIP(hipMemsetAsync(g->leaf_start, 0, sizeof(int32_t), s));
        if (sets)
            SPHX_HIP(hipMemsetAsync(g->set_leaf, 0, (size_t(n_sets) + 1) * sizeof(int32_t), s));
        SPHX_TRY(galloc(g, &g->fsum, 6 * 128 * int64_t(g->n_sets), s));
        if (g->recycle)
            release_spares(ctx);
        guard.keep = true;
        *out = g;
        return SPHX_OK;
    }

    k_keys<<<blocks(n, 256), 256, 0, s>>>(n, in->x, in->y, in->z, in->h, in->m, in->u,
                                           float(ctx->h_max), P.box[0],
                                           P.box[1], P.box[2], P.periodic, g->keys_in, g->idx_in,
                                           g->d_status);
    SPHX_HIP(hipGetLastError());

    // Stable LSD radix sort of (key, caller index) on the 63 key bits (each
    // set within its own range).
    size_t tmp = 0;
    if (sets)
        SPHX_HIP(rocprim::segmented_radix_sort_pairs(
            nullptr, tmp, g->keys_in, g->keys, g->idx_in, g->perm, unsigned(n), unsigned(n_sets),
            g->set_start, g->set_start + 1, 0, 63, s));
    else
        SPHX_HIP(rocprim::radix_sort_pairs(nullptr, tmp, g->keys_in, g->keys, g->idx_in,
                                           g->perm, size_t(n), 0, 63, s));
    size_t tmp2 = 0;
    SPHX_HIP(rocprim::inclusive_scan(nullptr, tmp2, g->flags, g->flags + n, size_t(n),
                                     rocprim::plus<uint32_t>(), s));
    g->sort_tmp_bytes = tmp > tmp2 ? tmp : tmp2;
    SPHX_TRY(galloc(g, reinterpret_cast<char **>(&g->sort_tmp), g->sort_tmp_bytes, s));
    if (sets) {
        SPHX_HIP(rocprim::segmented_radix_sort_pairs(
            g->sort_tmp, tmp, g->keys_in, g->keys, g->idx_in, g->perm, unsigned(n),
            unsigned(n_sets), g->set_start, g->set_start + 1, 0, 63, s));
        SPHX_TRY(galloc(g, &g->set_of, n, s));
        k_set_of<<<blocks(n, 256), 256, 0, s>>>(n, g->set_start, n_sets, g->set_of);
        SPHX_HIP(hipGetLastError());
    } else {
        SPHX_HIP(rocprim::radix_sort_pairs(g->sort_tmp, tmp, g->keys_in, g->keys, g->idx_in,
                                           g->perm, size_t(n), 0, 63, s));
    }
    // the sort's input indices are not needed again: the inverse goes there
    g->inv = g->idx_in;
    k_invert<<<blocks(n, 256), 256, 0, s>>>(n, g->perm, g->inv);
    SPHX_HIP(hipGetLastError());

    const int cap = P.leaf_max;
    k_leaf_flags<<<blocks(n, 256), 256, 0, s>>>(n, g->keys, cap, g->flags, g->set_of,
                                                g->set_start);
    SPHX_HIP(hipGetLastError());
    SPHX_HIP(rocprim::inclusive_scan(g->sort_tmp, tmp2, g->flags, g->flags + n, size_t(n),
                                     rocprim::plus<uint32_t>(), s));
    // Octree leaves -> parents -> packed cells. flags[0, n) holds the leaf
    // starts, flags[n, 2n) their inclusive scan; the cell starts then reuse
    // flags[0, n) (cleared first) and their scan flags[n, 2n).
    SPHX_TRY(galloc(g, &g->leaf_start, n + 1, s));
    int32_t *par_lvl = nullptr;
    uint64_t *par_pfx = nullptr;
    SPHX_TRY(dalloc(&par_lvl, n, s));
    if (dmalloc((void **)&par_pfx, size_t(n) * sizeof(uint64_t), s) != hipSuccess) {
        dfree(par_lvl, s);
        set_error("sphx_grid_build: out of device memory");
        return SPHX_E_OOM;
    }
    struct Tmp {
        void *a, *b;
        hipStream_t s;
        ~Tmp()
        {
            dfree(a, s);
            dfree(b, s);
        }
    } tmp_guard{par_lvl, par_pfx, s};
    k_oct_index<<<blocks(n, 256), 256, 0, s>>>(n, g->flags, g->flags + n, g->leaf_start,
                                               g->d_status + 2);
    SPHX_HIP(hipGetLastError());
    k_oct_parent<<<blocks(n, 256), 256, 0, s>>>(n, g->keys, g->leaf_start, g->d_status + 2,
                                                par_lvl, par_pfx, g->set_of, g->set_start);
    SPHX_HIP(hipGetLastError());
    // keep the leaf scan for the identical-key case: copy it out of the way
    SPHX_HIP(hipMemcpyAsync(g->keys_in, g->flags + n, size_t(n) * sizeof(uint32_t),
                            hipMemcpyDeviceToDevice, s));
    SPHX_HIP(hipMemsetAsync(g->flags, 0, size_t(n) * sizeof(uint32_t), s));
    k_pack_cells<<<blocks(n, 256), 256, 0, s>>>(n, g->keys, g->leaf_start, g->d_status + 2,
                                                par_lvl, par_pfx,
                                                reinterpret_cast<uint32_t *>(g->keys_in), cap,
                                                g->flags, g->set_of, g->set_start);
    SPHX_HIP(hipGetLastError());
    SPHX_HIP(rocprim::inclusive_scan(g->sort_tmp, tmp2, g->flags, g->flags + n, size_t(n),
                                     rocprim::plus<uint32_t>(), s));
    k_leaf_index<<<blocks(n, 256), 256, 0, s>>>(n, g->flags, g->flags + n, g->leaf_of,
                                                g->leaf_start, g->d_status + 1);
    SPHX_HIP(hipGetLastError());
    int32_t st[2];
    SPHX_HIP(hipMemcpyAsync(st, g->d_status, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SPHX_HIP(hipStreamSynchronize(s));
    if (st[0] != 0) {
        set_error("sphx_grid_build: " + std::to_string(st[0]) +
                  " particles with non-finite or out-of-range x, h (0 < h <= h_max), m or u");
        return SPHX_E_INVALID;
    }
    const int64_t nl = st[1];
    g->n_leaves = nl;

    // Tree levels over the leaves.
    int64_t off = 0, cnt = nl;
    int lev = 0;
    while (true) {
        g->level_off[lev] = off;
        g->level_cnt[lev] = cnt;
        off += cnt;
        ++lev;
        if (cnt <= 1 || lev == kMaxLevels)
            break;
        cnt = (cnt + kTreeFan - 1) / kTreeFan;
    }
    g->n_levels = lev;
    g->n_nodes = off;
    SPHX_TRY(galloc(g, &g->leaf_org, 3 * nl, s));
    SPHX_TRY(galloc(g, &g->leaf_ext, nl, s));
    SPHX_TRY(galloc(g, &g->leaf_hmax, nl, s));
    SPHX_TRY(galloc(g, &g->node_lo, 3 * off, s));
    SPHX_TRY(galloc(g, &g->node_hi, 3 * off, s));
    SPHX_TRY(galloc(g, &g->node_r, off, s));
    // + the parts of each set's reduction of the sums
    SPHX_TRY(galloc(g, &g->fsum, 6 * (nl + 128 * int64_t(g->n_sets)), s));
    if (sets) {
        SPHX_TRY(galloc(g, &g->leaf_set, nl > 0 ? nl : 1, s));
        k_set_leaves<<<blocks(std::max<int64_t>(nl, int64_t(n_sets) + 1), 256), 256, 0, s>>>(
            n, n_sets, g->set_start, g->leaf_of, g->leaf_start, g->set_of, g->d_status + 1,
            g->set_leaf, g->leaf_set);
        SPHX_HIP(hipGetLastError());
    }

    k_leaf_setup<<<unsigned(nl), 64, 0, s>>>(nl, g->leaf_start, g->perm, in->x, in->y, in->z,
                                             in->vx, in->vy, in->vz, in->m, in->u, in->alpha_v,
                                             in->alpha_c, P.box[0], P.box[1], P.box[2],
                                             P.periodic, g->leaf_org, g->node_lo, g->node_hi,
                                             g->q0, g->q1, g->qa, g->leaf_ext);
    SPHX_HIP(hipGetLastError());
    for (int l = 0; l + 1 < g->n_levels; ++l) {
        int64_t up = g->level_cnt[l + 1];
        k_tree_level<<<blocks(up, 128), 128, 0, s>>>(
            up, g->level_cnt[l], g->node_lo + 3 * g->level_off[l], g->node_hi + 3 * g->level_off[l],
            g->node_lo + 3 * g->level_off[l + 1], g->node_hi + 3 * g->level_off[l + 1]);
        SPHX_HIP(hipGetLastError());
    }
    SPHX_TRY(iter_reset(g, in, s));
    if (g->recycle)
        release_spares(ctx);  // the spares this build did not take
    guard.keep = true;
    *out = g;
    return SPHX_OK;
}

}  // namespace sphx
