// Per-receiver neighbour lists for the passes of the h iteration (Section
// 3.1 iterates the density loop until every h satisfies the partition
// condition; after the first pass the h of most particles moves by a few per
// cent, so the neighbours found once within a slightly larger radius serve
// every later pass).
//
// A receiver's list radius is min((1 + skin) H, task radius of its leaf), at
// least H when the task list is current. The build walks the same cell-pair
// tasks as the density loop (pairs.h) twice: once counting each receiver's
// sources within its list radius, once writing them, in the loop's fixed
// order (task order, then source order). The receivers of a 64-block of
// sorted indices share a column-major slab of 64 x (their largest count)
// entries, so that a list pass reads 64 consecutive entries per step.
#include <rocprim/device/device_scan.hpp>

#include "pairs.h"

namespace sphx {
namespace {

// One wave per leaf. FILL = false: list radius and count of each receiver
// (lrad, lcnt written); FILL = true: the entries (lrad, lcnt and lboff read).
template <bool FILL>
__global__ __launch_bounds__(64) void k_list(
    int64_t n_leaves, int64_t nb_padded, const int32_t *__restrict__ order,
    const int32_t *__restrict__ leaf_start,
    const float4 *__restrict__ q0, const uint8_t *__restrict__ need, const float *__restrict__ hs,
    const float *__restrict__ radius, const int32_t *__restrict__ tbeg,
    const int32_t *__restrict__ tend,
    const Task *__restrict__ task, const float4 *__restrict__ ext, float list_scale,
    float *__restrict__ lrad,
    int32_t *__restrict__ lcnt, const int64_t *__restrict__ lboff, uint32_t *__restrict__ lst)
{
    const int64_t L = leaf_of_block(blockIdx.x, nb_padded, order);
    if (L >= n_leaves)
        return;
    const int lane = threadIdx.x;
    const int32_t s0 = leaf_start[L];
    const int32_t cnt = leaf_start[L + 1] - s0;
    const bool valid = lane < cnt;
    const int32_t s = s0 + (valid ? lane : 0);
    const bool act = valid && need[s];
    float Ri = 0.0f;
    if (!FILL) {
        Ri = act ? fminf(list_scale * hs[s], radius[L]) : 0.0f;
        if (valid)
            lrad[s] = Ri;
    } else if (act) {
        Ri = lrad[s];
    }
    if (!__any(act)) {
        if (!FILL && valid)
            lcnt[s] = 0;
        return;
    }

    __shared__ float4 cp[kCap];    // candidate x, y, z in the receiver cell's frame
    __shared__ uint32_t cc[kCap];  // candidate list entry
    __shared__ uint32_t lst_lds[FILL ? kListStride * 16 : 1];
    uint8_t *my_list = reinterpret_cast<uint8_t *>(lst_lds) + (FILL ? lane * kListStride : 0);

    const float4 pi = q0[s];
    const float R2i = act ? Ri * Ri : -1.0f;
    const float inf = __builtin_inff();
    float3 lo = make_float3(act ? pi.x : inf, act ? pi.y : inf, act ? pi.z : inf);
    float3 hb = make_float3(act ? pi.x : -inf, act ? pi.y : -inf, act ? pi.z : -inf);
    lo.x = wave_minf(lo.x);
    lo.y = wave_minf(lo.y);
    lo.z = wave_minf(lo.z);
    hb.x = wave_maxf(hb.x);
    hb.y = wave_maxf(hb.y);
    hb.z = wave_maxf(hb.z);
    const float R = wave_maxf(Ri);
    const float R2 = R * R;

    int nc = 0;        // buffered candidates (wave-uniform)
    int32_t mine = 0;  // entries counted / written so far
    int myn = 0;       // FILL: accepted slots of the current buffer
    const int64_t my_base = FILL && act ? lboff[s >> 6] + (s & 63) : 0;
    // Both passes take the same decisions; the bound only guarantees that no
    // entry lands outside the block's slab.
    const int32_t my_cap = FILL && act ? lcnt[s] : 0;

    auto write_out = [&]() __attribute__((always_inline)) {
        for (int k = 0; __any(k < myn); k += 4) {
            const uint32_t four = *reinterpret_cast<const uint32_t *>(my_list + k);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (k + q < myn && mine < my_cap) {
                    lst[my_base + int64_t(mine) * 64] = cc[(four >> (8 * q)) & 0xffu];
                    ++mine;
                }
        }
        myn = 0;
    };
    auto test = [&](int c, const float4 &p) __attribute__((always_inline)) {
        const bool in = dist2(pi.x - p.x, pi.y - p.y, pi.z - p.z) < R2i;
        if (FILL) {
            if (in) {
                my_list[myn] = uint8_t(c);
                ++myn;
            }
        } else {
            mine += in ? 1 : 0;
        }
    };
    auto flush = [&]() __attribute__((always_inline)) {
        wave_sync();
        int c = 0;
        for (; c + 4 <= nc; c += 4) {
            const float4 p0 = cp[c], p1 = cp[c + 1], p2 = cp[c + 2], p3 = cp[c + 3];
            test(c, p0);
            test(c + 1, p1);
            test(c + 2, p2);
            test(c + 3, p3);
            if (FILL && __any(myn > kListMax - 4))
                write_out();
        }
        for (; c < nc; ++c)
            test(c, cp[c]);
        if (FILL)
            write_out();
        wave_sync();
        nc = 0;
    };
    auto emit = [&](const float4 &p, uint32_t code, bool keep) __attribute__((always_inline)) {
        const uint64_t mask = __ballot(keep);
        if (mask == 0)
            return;
        const int tot = __popcll(mask);
        if (nc + tot > kCap)
            flush();
        const int pos = nc + lanes_below(mask);
        if (keep) {
            cp[pos] = p;
            cc[pos] = code;
        }
        nc += tot;
    };

    const int32_t ta = tbeg[L], tn = tend[L] - ta;
    for (int32_t tb = 0; tb < tn; tb += 64) {
        const int nb = min(64, tn - tb);
        TaskRegs tr;
        tr.load(task, ta + tb + lane, lane < nb);
        if (lane < nb && task_box_dist2(tr.b.x, tr.b.y, tr.b.z, ext[tr.a.w], lo, hb) >= R2)
            tr.a.y = 0;  // whole source cells beyond R of the receivers' box
        for (int u = 0; u < nb; u += 4) {
            int j0[4], jc[4];
            float ox[4], oy[4], oz[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = min(u + q, nb - 1);
                j0[q] = bcast(tr.a.x, k);
                jc[q] = (u + q < nb) ? bcast(tr.a.y, k) : 0;
                ox[q] = bcastf(tr.b.x, k);
                oy[q] = bcastf(tr.b.y, k);
                oz[q] = bcastf(tr.b.z, k);
            }
            float4 p[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                p[q] = lane < jc[q] ? q0[j0[q] + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                p[q].x += ox[q];
                p[q].y += oy[q];
                p[q].z += oz[q];
                const bool keep = lane < jc[q] && box_dist2(p[q].x, p[q].y, p[q].z, lo, hb) < R2;
                emit(p[q], (uint32_t(tb + u + q) << kListCodeShift) | uint32_t(lane), keep);
            }
        }
    }
    if (nc > 0)
        flush();
    if (!FILL && valid)
        lcnt[s] = act ? mine : 0;
}

// 64 x (largest count) of every 64-block of sorted receivers; the extra
// element past the last block is zero, so that the exclusive scan ends with
// the total.
__global__ void k_list_cap(int64_t n, int64_t n_blocks, const int32_t *__restrict__ lcnt,
                           int64_t *__restrict__ cap)
{
    const int64_t b = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b > n_blocks)
        return;
    const int64_t s = b * 64 + lane;
    const int c = wave_maxi(s < n ? lcnt[s] : 0);
    if (lane == 0)
        cap[b] = int64_t(c) * 64;
}

}  // namespace

size_t lists_bytes(int64_t n)
{
    // list radius and count per particle, block offsets, and the entries:
    // about (1 + skin)^3 times the ~58 kernel neighbours, padded to the
    // block's largest count.
    return size_t(n) * (4 + 4 + 1 + 104 * 4) + (1 << 20);
}

sphx_status list_build(const sphx_ctx *ctx, sphx_grid *g, const sphx_tasks *t, hipStream_t s,
                       bool *ok)
{
    *ok = false;
    if (g->n == 0 || t->n_tasks >= kListMaxTasks)
        return SPHX_OK;
    const int64_t n = g->n;
    const int64_t nb = (n + 63) / 64;
    if (!g->lrad) {
        if (dmalloc((void **)&g->lrad, size_t(n) * sizeof(float), s) != hipSuccess ||
            dmalloc((void **)&g->lcnt, size_t(n) * sizeof(int32_t), s) != hipSuccess ||
            dmalloc((void **)&g->lcap, size_t(nb + 1) * sizeof(int64_t), s) != hipSuccess ||
            dmalloc((void **)&g->lboff, size_t(nb + 1) * sizeof(int64_t), s) != hipSuccess) {
            set_error("list build: out of device memory");
            return SPHX_E_OOM;
        }
        size_t tmp = 0;
        SPHX_HIP(rocprim::exclusive_scan(nullptr, tmp, g->lcap, g->lboff, int64_t(0),
                                         size_t(nb + 1), rocprim::plus<int64_t>(), s));
        if (dmalloc(&g->lscan_tmp, tmp + 16, s) != hipSuccess) {
            set_error("list build: out of device memory");
            return SPHX_E_OOM;
        }
        g->lscan_bytes = tmp;
    }
    const int64_t nl = g->n_leaves;
    const int64_t nlp = pad8(nl);
    const float scale = float(ctx->p.gamma_k * (1.0 + ctx->p.skin));
    SPHX_HIP(ctx->prof->begin(3, s));
    k_list<false><<<unsigned(nlp), 64, 0, s>>>(nl, nlp, t->order, g->leaf_start, g->q0, g->need,
                                               g->hs, t->radius, t->slot, t->end, t->task,
                                               g->leaf_ext, scale, g->lrad, g->lcnt, nullptr, nullptr);
    SPHX_HIP(hipGetLastError());
    k_list_cap<<<unsigned((nb + 1 + 3) / 4), 256, 0, s>>>(n, nb, g->lcnt, g->lcap);
    SPHX_HIP(hipGetLastError());
    size_t tmp = g->lscan_bytes;
    SPHX_HIP(rocprim::exclusive_scan(g->lscan_tmp, tmp, g->lcap, g->lboff, int64_t(0),
                                     size_t(nb + 1), rocprim::plus<int64_t>(), s));
    SPHX_HIP(ctx->prof->end(3, s));
    int64_t total = 0;
    SPHX_HIP(hipMemcpyAsync(&total, g->lboff + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPHX_HIP(hipStreamSynchronize(s));
    if (total > g->lst_cap) {
        dfree(g->lst, s);
        g->lst = nullptr;
        g->lst_cap = 0;
        const int64_t cap = total + total / 8 + 64 * 64;
        if (dmalloc((void **)&g->lst, size_t(cap) * sizeof(uint32_t), s) != hipSuccess) {
            // Not enough memory for lists: stay on the cell-pair path.
            (void)hipGetLastError();
            return SPHX_OK;
        }
        g->lst_cap = cap;
    }
    g->lst_total = total;
    SPHX_HIP(ctx->prof->begin(3, s));
    k_list<true><<<unsigned(nlp), 64, 0, s>>>(nl, nlp, t->order, g->leaf_start, g->q0, g->need,
                                              g->hs, t->radius, t->slot, t->end, t->task,
                                              g->leaf_ext, scale, g->lrad, g->lcnt, g->lboff, g->lst);
    SPHX_HIP(hipGetLastError());
    SPHX_HIP(ctx->prof->end(3, s));
    *ok = true;
    return SPHX_OK;
}

}  // namespace sphx
