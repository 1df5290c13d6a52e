// Density pass (Section 3.1): number density, mass density, their
// h-derivatives, neighbour count, and the velocity divergence and curl sums.
//
// Two loops compute the same sums:
// * k_density, over cell pairs: the loop structure (cull, candidate buffer,
//   per-lane lists) is described in pairs.h. A block of NW waves serves one
//   receiving cell: wave w takes the w-th contiguous share of the cell's
//   tasks, and the shares' partial sums are added in wave order at the end (a
//   fixed order, so results stay reproducible).
// * k_dens_list, over per-receiver neighbour lists (built by lists.hip for the
//   later passes of the h iteration): one lane per receiver, 64 consecutive
//   receivers per wave, each lane walking its own list in its fixed order.
#include "pairs.h"

// Measurement builds (SPHX_PROBE=1) count the cell-pair loop's neighbour
// tests: the lane slots the tests occupy, the tests made by lanes that hold a
// receiver, and the accepted pairs; and its per-lane compute loops: the lane
// slots of their rounds and the list entries evaluated; into probe_counts
// (read and cleared by sphx_probe_read). Product builds count nothing.
#ifndef SPHX_PROBE
#define SPHX_PROBE 0
#endif

namespace sphx {

__device__ unsigned long long probe_counts[5];

namespace {

constexpr int kSums = 9;  // Sw, Smw, Sud, Smud, Sdiv, Scx, Scy, Scz, count
// The pressure-energy flavour (Appendix A) adds Smuw = sum m u w and Smuud =
// sum m u u^2 phi for its smoothed pressure and that pressure's h-derivative.
constexpr int kSumsPE = kSums + 2;

// Where a receiver's results go: the caller's arrays (caller order) and the
// sorted-order state the ghost reads.
struct DensOut {
    float *rho, *rho_dh, *n, *n_dh, *div, *cx, *cy, *cz;
    int32_t *nngb;
    float4 *d0, *d1;
    // pressure-energy only: the smoothed pressure and its h-derivative (caller
    // order, may be null), the sorted pair the ghost reads, and gamma - 1
    float *p_hat, *p_hat_dh;
    float2 *d2;
    float gm1;
};

// Contributions of one directed pair; p and v are the source's position (in
// the receiver's frame) and mass, and its velocity. u = r / H, clamped at 1
// (a pair at or beyond the support adds nothing, also where rounding puts an
// accepted edge pair there). MASK: with on = false the pair adds nothing
// (its inputs must be finite) and on counts it; without MASK every pair is
// evaluated and counted by the caller: list entries past a lane's length
// point to a dummy source beyond every support (mass 0, velocity 0), which
// adds exactly zero. Either way the loops evaluate several list entries at
// once without branching.
template <bool MASK, int K, int NS>
__device__ __forceinline__ void dens_pair(float (&S)[NS], const float4 &pi, const float4 &vi,
                                          float invH, const float4 &p, const float4 &v, bool on)
{
    const float dx = pi.x - p.x, dy = pi.y - p.y, dz = pi.z - p.z;
    const float r2 = dx * dx + dy * dy + dz * dz;
    const float u = fminf(fast_sqrt(r2) * invH, 1.0f);
    const float t3 = Kern<K>::phi(u);
    const float wk = (!MASK || on) ? Kern<K>::w(u) : 0.0f;
    const float ud = (!MASK || on) ? u * u * t3 : 0.0f;
    S[0] += wk;
    S[1] += p.w * wk;
    S[2] += ud;
    S[3] += p.w * ud;
    if (MASK)
        S[8] += on ? 1.0f : 0.0f;
    const float dvx = v.x - vi.x, dvy = v.y - vi.y, dvz = v.z - vi.z;
    const float mt3 = (!MASK || on) ? p.w * t3 : 0.0f;
    S[4] += mt3 * (dvx * dx + dvy * dy + dvz * dz);
    S[5] += mt3 * (dy * dvz - dz * dvy);
    S[6] += mt3 * (dz * dvx - dx * dvz);
    S[7] += mt3 * (dx * dvy - dy * dvx);
    if constexpr (NS == kSumsPE) {
        const float mu = p.w * v.w;  // m_j u_j (the dummy source has m = 0)
        S[9] += mu * wk;
        S[10] += mu * ud;
    }
}

// A receiver's results from its sums. Its own particle went through the loop
// as a pair at r = 0: it contributes W(0) to n and rho and nothing to the
// gradient sums; it is not a neighbour.
template <int K, int NS>
__device__ __forceinline__ void dens_finish(const float (&S)[NS], float hi, float invH,
                                            int64_t s, int32_t gi, const DensOut &o)
{
    constexpr float kW = Kern<K>::kW, kD = Kern<K>::kD;
    const float Sw = S[0];
    const float Smw = S[1];
    // W = kW H^-3 w(u); dW/dh = -(H^-3/h)(3 kW w - kD u^2 phi(u));
    // grad_i W = (dW/dr / r) x_ij with dW/dr / r = -kD H^-5 phi(u).
    const float invH3 = invH * invH * invH;
    const float invH5 = invH3 * invH * invH;
    const float ih = fast_rcp(hi);
    const float n_ = kW * invH3 * Sw;
    const float rho = kW * invH3 * Smw;
    const float n_dh = -invH3 * ih * (3.0f * kW * Sw - kD * S[2]);
    const float rho_dh = -invH3 * ih * (3.0f * kW * Smw - kD * S[3]);
    const float dv = -kD * invH5 * S[4];
    const float cx = -kD * invH5 * S[5];
    const float cy = -kD * invH5 * S[6];
    const float cz = -kD * invH5 * S[7];
    // For the ghost, the two ratios it needs in a form free of cancellation:
    // G' = 3 + h n'/n = kD Sud / (kW Sw) and 1 + h rho'/(3 rho) = kD Smud /
    // (3 kW Smw) (the self term cancels exactly in both).
    const float gp = (kD * S[2]) / (kW * Sw);
    const float fden = (kD * S[3]) / (3.0f * kW * Smw);
    o.d0[s] = make_float4(n_, gp, rho, fden);
    o.d1[s] = make_float4(dv, cx, cy, cz);
    o.n[gi] = n_;
    o.rho[gi] = rho;
    o.n_dh[gi] = n_dh;
    o.rho_dh[gi] = rho_dh;
    o.div[gi] = dv;
    o.cx[gi] = cx;
    o.cy[gi] = cy;
    o.cz[gi] = cz;
    o.nngb[gi] = int32_t(S[8]) - 1;
    if constexpr (NS == kSumsPE) {
        // sum m u W, and the numerator of the grad-h term F of the factors
        // f_ij = 1 - F_i / (m_j u_j): F = h P_hat' / ((gamma - 1) 3 n) /
        // (1 + h n'/(3 n)) = (kD Smuud - 3 kW Smuw) / (kW Sw) / G'
        const float Smuw = S[9], Smuud = S[10];
        o.d2[s] = make_float2(kW * invH3 * Smuw, (kD * Smuud - 3.0f * kW * Smuw) / (kW * Sw));
        if (o.p_hat) {
            o.p_hat[gi] = o.gm1 * kW * invH3 * Smuw;
            o.p_hat_dh[gi] = -o.gm1 * invH3 * ih * (3.0f * kW * Smuw - kD * Smuud);
        }
    }
}

// BAL: compute rounds cut the lanes' lists into chunks of one receiver each
// and spread them over the lanes (compute_bal) instead of each lane walking
// its own list.
template <int CAP, int NW, bool BAL, int K, bool PE>
__global__ __launch_bounds__(64 * NW) void k_density(
    int64_t n_leaves, int64_t nb_padded, const int32_t *__restrict__ order,
    const int32_t *__restrict__ leaf_start,
    const int32_t *__restrict__ perm, const float4 *__restrict__ q0,
    const float4 *__restrict__ q1, const uint8_t *__restrict__ need, const float *__restrict__ hs,
    const float *__restrict__ radius, const int32_t *__restrict__ tbeg,
    const int32_t *__restrict__ tend,
    const Task *__restrict__ task, const float4 *__restrict__ ext, float gamma_k, float far,
    const float *__restrict__ lrad, DensOut o, int32_t *__restrict__ counters,
    const int32_t *__restrict__ skip)
{
    if (skip && *skip)
        return;  // a captured pass with nothing left to do
    static_assert(CAP >= 64 && CAP <= 256, "candidate slots: one task's sources, 8-bit slots");
    constexpr int NS = PE ? kSumsPE : kSums;
    const int64_t L = leaf_of_block(blockIdx.x, nb_padded, order);
    if (L >= n_leaves)
        return;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int32_t s0 = leaf_start[L];
    const int32_t cnt = leaf_start[L + 1] - s0;
    const bool valid = lane < cnt;
    const int32_t s = s0 + (valid ? lane : 0);
    const float hi0 = hs[s];
    // With lists, this loop serves only the receivers whose H outgrew theirs.
    const bool act = valid && need[s] && (!lrad || gamma_k * hi0 > lrad[s]);
    if (!__any(act))
        return;  // the same for every wave of the block

    // candidates x, y, z (receiver cell frame), m and vx, vy, vz; slot CAP is
    // the dummy source that list entries past a lane's length point to
    __shared__ float4 cp_all[NW][CAP + 1];
    __shared__ float4 cv_all[NW][CAP + 1];
    __shared__ uint32_t lst_all[NW][kListStride * 16];
    // BAL only: the receivers' positions and (velocity, 1/H), each receiver's
    // first chunk of the round, and the chunks' partial sums ([sum][slot]).
    __shared__ float4 rp_all[NW][BAL ? 64 : 1];
    __shared__ float4 rv_all[NW][BAL ? 64 : 1];
    __shared__ int32_t cb_all[NW][BAL ? 68 : 1];
    __shared__ float pt_all[NW][BAL ? NS * 64 : 1];
    float4 *cp = cp_all[w];
    float4 *cv = cv_all[w];
    uint8_t *lst = reinterpret_cast<uint8_t *>(lst_all[w]);
    uint8_t *my_list = lst + lane * kListStride;

    const float4 pi = q0[s];
    const float4 vi = q1[s];
    const int32_t gi = perm[s];
    const float hi = act ? hi0 : 1.0f;
    const float H = gamma_k * hi;
    const float invH = fast_rcp(H);
    if (w == 0 && act && H > radius[L] && counters)
        atomicAdd(counters + 3, 1);

    // Bounding box of the receivers that need work, and their largest radius.
    const float inf = __builtin_inff();
    float3 lo = make_float3(act ? pi.x : inf, act ? pi.y : inf, act ? pi.z : inf);
    float3 hb = make_float3(act ? pi.x : -inf, act ? pi.y : -inf, act ? pi.z : -inf);
    lo.x = wave_minf(lo.x);
    lo.y = wave_minf(lo.y);
    lo.z = wave_minf(lo.z);
    hb.x = wave_maxf(hb.x);
    hb.y = wave_maxf(hb.y);
    hb.z = wave_maxf(hb.z);
    const float R = wave_maxf(act ? H : 0.0f);
    const float R2 = R * R;

    // Lane replication: with n_act receivers needing work, each gets nrep
    // lanes (the largest power of two with nrep n_act <= 64). Replica j of a
    // receiver tests and sums the candidates whose running index (over the
    // whole loop, not the buffer) is j mod nrep, so a cell with few receivers
    // left runs its tests and pairs nrep times wider; the replicas' partial
    // sums are added by a butterfly over their lanes at the end (a fixed
    // order). The running index does not depend on the buffer size, so
    // neither do the results; nrep = 1 is the plain loop, lane = receiver.
    const uint64_t amask = __ballot(act);
    const int n_act = __popcll(amask);
    int nrep = 1;
    if (!BAL)
        while (2 * nrep * n_act <= 64)
            nrep *= 2;
    __shared__ uint8_t rmap_all[NW][64];
    int src = lane;
    bool ract = act;
    if (nrep > 1) {
        if (act)
            rmap_all[w][lanes_below(amask)] = uint8_t(lane);
        wave_sync();
        const int k = lane / nrep;
        ract = k < n_act;
        src = ract ? int(rmap_all[w][k]) : lane;
    }
    const int rj = lane & (nrep - 1);  // replica index
    // this lane's receiver (the lane's own particle when nrep = 1)
    const float4 pr = nrep > 1 ? make_float4(__shfl(pi.x, src, 64), __shfl(pi.y, src, 64),
                                             __shfl(pi.z, src, 64), __shfl(pi.w, src, 64))
                               : pi;
    const float4 vr = nrep > 1 ? make_float4(__shfl(vi.x, src, 64), __shfl(vi.y, src, 64),
                                             __shfl(vi.z, src, 64), __shfl(vi.w, src, 64))
                               : vi;
    const float h_src = nrep > 1 ? __shfl(hi, src, 64) : hi;  // every lane shuffles
    const float hr = ract ? h_src : 1.0f;
    const float Hr = gamma_k * hr;
    const float H2r = ract ? Hr * Hr : -1.0f;
    const float invHr = nrep > 1 ? fast_rcp(Hr) : invH;
    const int32_t sr = s0 + src;
    const int32_t gr = nrep > 1 ? __shfl(gi, src, 64) : gi;

    float S[NS] = {};
    int gbase = 0;  // candidates of the earlier buffers (wave-uniform)
    int nc = 0;   // buffered candidates (wave-uniform)
    int myn = 0;  // this lane's list length (its own particle is listed too)
    unsigned probe_cslots = 0, probe_cfill = 0;  // compute-loop lane slots, entries
    float4 *rp = rp_all[w];
    float4 *rv = rv_all[w];
    int32_t *cb = cb_all[w];
    float *pt = pt_all[w];
    if (BAL) {
        rp[lane] = pi;
        rv[lane] = make_float4(vi.x, vi.y, vi.z, invH);
    }

    // Four list entries at a time, without branches: entries past a lane's
    // list length read the dummy slot (beyond every support, mass 0: adds
    // exactly nothing); every listed entry is a neighbour, counted at once.
    if (lane == 0) {
        cp[CAP] = make_float4(far, far, far, 0.0f);
        cv[CAP] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    auto compute = [&]() __attribute__((always_inline)) {
        S[8] += float(myn);
        if (SPHX_PROBE)
            probe_cfill += myn;
        for (int k = 0; __any(k < myn); k += 4) {
            if (SPHX_PROBE)
                probe_cslots += 4;
            const uint32_t four = *reinterpret_cast<const uint32_t *>(my_list + k);
            float4 p[4], v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = k + q < myn ? int((four >> (8 * q)) & 0xffu) : CAP;
                p[q] = cp[c];
                v[q] = cv[c];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                dens_pair<false, K>(S, pr, vr, invHr, p[q], v[q], true);
        }
        myn = 0;
    };
    // Balanced round. The lists are cut into chunks of C entries (C a multiple
    // of 4) of one receiver each, numbered receiver by receiver; lane l takes
    // chunk j*64 + l in sub-round j and runs it like compute() with that
    // receiver's data. C is the candidate with the least work (sub-rounds x C)
    // among W/64, W/48, W/32 and the longest list. Each chunk's sums go to an
    // LDS slot; the receiver's lane adds its chunks in chunk order, so the
    // result does not depend on timing.
    auto compute_bal = [&]() __attribute__((always_inline)) {
        wave_sync();  // the other lanes' lists are read below
        const int W = wave_sumi(myn);
        if (W == 0)
            return;  // wave-uniform
        const int mx = wave_maxi(myn);
        int C = 0, T = 0, cost = 0x7fffffff;
        const int cand[4] = {(W + 63) / 64, (W + 47) / 48, (W + 31) / 32, mx};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int Cq = (cand[q] + 3) & ~3;
            const int Tq = wave_sumi((myn + Cq - 1) / Cq);
            const int cq = ((Tq + 63) / 64) * Cq;
            if (cq < cost) {
                cost = cq;
                C = Cq;
                T = Tq;
            }
        }
        const int nch = (myn + C - 1) / C;
        int incl = nch;  // inclusive prefix of the chunk counts
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (lane >= o)
                incl += t;
        }
        cb[lane + 1] = incl;
        if (lane == 0)
            cb[0] = 0;
        wave_sync();
        for (int j0 = 0; j0 < T; j0 += 64) {
            const int id = j0 + lane;
            int r = 0;  // the receiver of chunk id: the last r with cb[r] <= id
#pragma unroll
            for (int step = 32; step > 0; step >>= 1)
                if (cb[r + step] <= id)
                    r += step;
            const int mr = __shfl(myn, r, 64);
            const int k0 = (id - cb[r]) * C;
            const int len = id < T ? min(C, mr - k0) : 0;
            const float4 P = rp[r], V = rv[r];
            const uint8_t *rl = lst + r * kListStride + (id < T ? k0 : 0);
            float Tc[NS] = {};
            for (int k = 0; __any(k < len); k += 4) {
                const uint32_t four = k < len ? *reinterpret_cast<const uint32_t *>(rl + k) : 0u;
                float4 p[4], v[4];
                bool on[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    on[q] = k + q < len;
                    const int c = on[q] ? int((four >> (8 * q)) & 0xffu) : 0;
                    p[q] = cp[c];
                    v[q] = cv[c];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    dens_pair<true, K>(Tc, P, V, V.w, p[q], v[q], on[q]);
            }
#pragma unroll
            for (int k = 0; k < NS; ++k)
                pt[k * 64 + lane] = Tc[k];
            wave_sync();
            const int c0 = max(incl - nch, j0), c1 = min(incl, j0 + 64);
            for (int c = c0; c < c1; ++c)
#pragma unroll
                for (int k = 0; k < NS; ++k)
                    S[k] += pt[k * 64 + (c - j0)];
            wave_sync();
        }
        myn = 0;
    };
    // The slot is always written; it is kept (the length advanced) only
    // when the candidate lies inside H.
    unsigned probe_tests = 0, probe_hits = 0, probe_slots = 0;
    auto accept = [&](int c, const float4 &p, bool ok) __attribute__((always_inline)) {
        const float r2 = dist2(pr.x - p.x, pr.y - p.y, pr.z - p.z);
        my_list[myn] = uint8_t(c);
        const int hit = (ok && r2 < H2r) ? 1 : 0;
        myn += hit;
        if (SPHX_PROBE) {
            probe_slots += 1;
            probe_tests += (ract && c < CAP) ? 1 : 0;
            probe_hits += hit;
        }
    };
    auto flush = [&]() __attribute__((always_inline)) {
        wave_sync();
        if (nrep == 1) {
            int c = 0;
            for (; c + 4 <= nc; c += 4) {
                const float4 p0 = cp[c], p1 = cp[c + 1], p2 = cp[c + 2], p3 = cp[c + 3];
                accept(c, p0, true);
                accept(c + 1, p1, true);
                accept(c + 2, p2, true);
                accept(c + 3, p3, true);
                if (__any(myn > kListMax - 4)) {
                    if (BAL)
                        compute_bal();
                    else
                        compute();
                }
            }
            for (; c < nc; ++c)
                accept(c, cp[c], true);
            if (BAL)
                compute_bal();
            else
                compute();
        } else {
            // replica rj takes the slots c with gbase + c = rj (mod nrep);
            // slots past the buffer read the dummy source, which no test
            // accepts (no branch around the test)
            const int c0 = (rj - (gbase & (nrep - 1))) & (nrep - 1);
            const int m_end = (nc + nrep - 1) / nrep;
            for (int m = 0; m < m_end; m += 4) {
                int cq[4];
                float4 pq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int c = c0 + (m + q) * nrep;
                    cq[q] = c < nc ? c : CAP;
                    pq[q] = cp[cq[q]];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    accept(cq[q], pq[q], true);
                if (__any(myn > kListMax - 4))
                    compute();
            }
            compute();
        }
        gbase += nc;
        wave_sync();
        nc = 0;
    };

    // Append the kept sources of one task to the candidate buffer.
    auto emit = [&](const float4 &p, const float4 &v, bool keep) __attribute__((always_inline)) {
        const uint64_t mask = __ballot(keep);
        if (mask == 0)
            return;
        const int tot = __popcll(mask);
        if (nc + tot > CAP)
            flush();
        const int pos = nc + lanes_below(mask);
        if (keep) {
            cp[pos] = p;
            cv[pos] = v;
        }
        nc += tot;
    };

    // This wave's share of the cell's tasks: those of the source cells J with
    // J mod NW = w. A split by position would move with the list's length,
    // and a list that also holds cells beyond every receiver's reach (one
    // kept through growth rebuilds) would then give other partial sums.
    const int32_t ta = tbeg[L], t_end = tend[L];
    for (int32_t tb = ta; tb < t_end; tb += 64) {
        const int nb = min(64, t_end - tb);
        TaskRegs tr;
        tr.load(task, tb + lane, lane < nb);
        // whole source cells beyond R of the receivers' box are skipped
        if (lane < nb && ((NW > 1 && tr.a.w % NW != w) ||
                          task_box_dist2(tr.b.x, tr.b.y, tr.b.z, ext[tr.a.w], lo, hb) >= R2))
            tr.a.y = 0;
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
            // positions and velocities in one round trip (the velocities of
            // culled sources are read for nothing: the loop is far from
            // bandwidth-bound, and latency-bound here)
            float4 p[4], v[4];
            bool keep[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool in = lane < jc[q];
                p[q] = in ? q0[j0[q] + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
                v[q] = in ? q1[j0[q] + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                p[q].x += ox[q];
                p[q].y += oy[q];
                p[q].z += oz[q];
                keep[q] = lane < jc[q] && box_dist2(p[q].x, p[q].y, p[q].z, lo, hb) < R2;
            }
            emit(p[0], v[0], keep[0]);
            emit(p[1], v[1], keep[1]);
            emit(p[2], v[2], keep[2]);
            emit(p[3], v[3], keep[3]);
        }
    }
    if (nc > 0)
        flush();
    // the replicas' partial sums, by a butterfly: every replica ends with
    // the same total (each addition is commutative)
    for (int o = 1; o < nrep; o <<= 1)
#pragma unroll
        for (int k = 0; k < NS; ++k)
            S[k] += __shfl_xor(S[k], o, 64);
    if (SPHX_PROBE) {
        unsigned long long v[5] = {probe_slots, probe_tests, probe_hits, probe_cslots,
                                   probe_cfill};
        for (int k = 0; k < 5; ++k) {
            for (int o = 32; o > 0; o >>= 1)
                v[k] += __shfl_xor(v[k], o, 64);
            if (lane == 0)
                atomicAdd(probe_counts + k, v[k]);
        }
    }

    if (NW > 1) {
        // Add the other waves' partial sums to wave 0's, in wave order.
        __syncthreads();
        // the other waves' partial sums (own array: small tiles leave too
        // little room in the candidate buffers)
        __shared__ float red[NW > 1 ? (NW - 1) * NS * 64 : 1];
        if (w > 0)
            for (int k = 0; k < NS; ++k)
                red[((w - 1) * NS + k) * 64 + lane] = S[k];
        __syncthreads();
        if (w > 0)
            return;
        for (int w2 = 1; w2 < NW; ++w2)
            for (int k = 0; k < NS; ++k)
                S[k] += red[((w2 - 1) * NS + k) * 64 + lane];
    }
    if (!ract || rj != 0)
        return;
    dens_finish<K>(S, hr, invHr, sr, gr, o);
}

// Grouped rounds (density_balance = 2). The cell's sources are loaded, culled
// against the box of all the receivers that need work and buffered as in
// k_density; at each flush the receivers are taken in groups of up to 16
// consecutive sorted indices (Morton order: each group is spatially compact)
// with precomputed bounding boxes and radii. For each group in turn the
// wave compacts the buffered candidates that lie within the group's radius
// of its box, and tests and sums only those, with nrep = 64 / (group size)
// lanes per receiver (rounded down to a power of two): replica q takes every
// nrep-th candidate of the group's list from q. So a candidate is tested by
// the receivers near it rather than by every receiver of the cell, and each
// receiver's pair work is spread evenly over its replicas. After each
// group's flush the replicas' partial sums are added by a butterfly and
// accumulated per receiver in LDS, in flush order: results are reproducible
// (they depend on the buffer size, which is fixed per instantiation).
constexpr int kGroupMax = 16;  // receivers per group

template <int CAP, int K>
__global__ __launch_bounds__(64) void k_density_grp(
    int64_t n_leaves, int64_t nb_padded, const int32_t *__restrict__ order,
    const int32_t *__restrict__ leaf_start, const int32_t *__restrict__ perm,
    const float4 *__restrict__ q0, const float4 *__restrict__ q1,
    const uint8_t *__restrict__ need, const float *__restrict__ hs,
    const float *__restrict__ radius, const int32_t *__restrict__ tbeg,
    const int32_t *__restrict__ tend,
    const Task *__restrict__ task, const float4 *__restrict__ ext, float gamma_k, float far,
    DensOut o, int32_t *__restrict__ counters, const int32_t *__restrict__ skip)
{
    if (skip && *skip)
        return;  // a captured pass with nothing left to do
    static_assert(CAP >= 64 && CAP <= 256, "candidate slots: one task's sources, 8-bit slots");
    const int64_t L = leaf_of_block(blockIdx.x, nb_padded, order);
    if (L >= n_leaves)
        return;
    const int lane = threadIdx.x;
    const int32_t s0 = leaf_start[L];
    const int32_t cnt = leaf_start[L + 1] - s0;
    const bool valid = lane < cnt;
    const int32_t s = s0 + (valid ? lane : 0);
    const float hi0 = hs[s];
    const bool act = valid && need[s];
    const uint64_t amask = __ballot(act);
    if (amask == 0)
        return;
    const int n_act = __popcll(amask);

    __shared__ float4 cp[CAP + 1];  // candidates: x, y, z (cell frame), m; slot CAP: dummy
    __shared__ float4 cv[CAP + 1];  // vx, vy, vz
    // per-lane lists: a replica sees at most CAP / 4 of a flush's candidates
    // (groups of up to 16 receivers have 4 or more lanes each)
    constexpr int LMAX = CAP / 4 < 32 ? 32 : CAP / 4;
    constexpr int LSTRIDE = LMAX + 4;  // an odd number of dwords
    __shared__ uint32_t lst_w[LSTRIDE * 16];
    __shared__ float4 rtp[64];           // active receivers by rank: position, m
    __shared__ float4 rtv[64];           // velocity, h
    __shared__ uint8_t rts[64];          // rank -> index in the cell
    __shared__ float acc[kSums][64];     // the receivers' sums by rank
    __shared__ float4 gbox[64 / kGroupMax][2];  // group boxes: lo (w = R^2), hi
    __shared__ uint8_t gidx[CAP];        // the current group's candidate slots
    uint8_t *lst = reinterpret_cast<uint8_t *>(lst_w);
    uint8_t *my_list = lst + lane * LSTRIDE;

    const float4 pi = q0[s];
    const float H = gamma_k * (act ? hi0 : 1.0f);
    if (act) {
        const int k = lanes_below(amask);
        const float4 vi = q1[s];
        rtp[k] = pi;
        rtv[k] = make_float4(vi.x, vi.y, vi.z, hi0);
        rts[k] = uint8_t(lane);
        if (H > radius[L] && counters)
            atomicAdd(counters + 3, 1);
    }
#pragma unroll
    for (int k = 0; k < kSums; ++k)
        acc[k][lane] = 0.0f;
    if (lane == 0) {
        cp[CAP] = make_float4(far, far, far, 0.0f);
        cv[CAP] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    // the box of all the active receivers and their largest radius
    const float inf = __builtin_inff();
    float3 lo = make_float3(act ? pi.x : inf, act ? pi.y : inf, act ? pi.z : inf);
    float3 hb = make_float3(act ? pi.x : -inf, act ? pi.y : -inf, act ? pi.z : -inf);
    lo.x = wave_minf(lo.x);
    lo.y = wave_minf(lo.y);
    lo.z = wave_minf(lo.z);
    hb.x = wave_maxf(hb.x);
    hb.y = wave_maxf(hb.y);
    hb.z = wave_maxf(hb.z);
    const float R = wave_maxf(act ? H : 0.0f);
    const float R2 = R * R;
    const int NG = (n_act + kGroupMax - 1) / kGroupMax;
    wave_sync();  // the receiver table
    // each group's box and radius
    for (int g = 0; g < NG; ++g) {
        const int r0 = g * kGroupMax;
        const int kg = min(kGroupMax, n_act - r0);
        const bool mine = lane < kg;
        const float4 p = rtp[r0 + (mine ? lane : 0)];
        const float Hg = mine ? gamma_k * rtv[r0 + (mine ? lane : 0)].w : 0.0f;
        float3 glo = make_float3(mine ? p.x : inf, mine ? p.y : inf, mine ? p.z : inf);
        float3 ghi = make_float3(mine ? p.x : -inf, mine ? p.y : -inf, mine ? p.z : -inf);
        glo.x = wave_minf(glo.x);
        glo.y = wave_minf(glo.y);
        glo.z = wave_minf(glo.z);
        ghi.x = wave_maxf(ghi.x);
        ghi.y = wave_maxf(ghi.y);
        ghi.z = wave_maxf(ghi.z);
        const float Rg = wave_maxf(Hg);
        if (lane == 0) {
            gbox[g][0] = make_float4(glo.x, glo.y, glo.z, Rg * Rg);
            gbox[g][1] = make_float4(ghi.x, ghi.y, ghi.z, 0.0f);
        }
    }
    wave_sync();

    int nc = 0;  // buffered candidates (wave-uniform)
    auto flush = [&]() __attribute__((always_inline)) {
        wave_sync();
        for (int g = 0; g < NG; ++g) {
            const int r0 = g * kGroupMax;
            const int kg = min(kGroupMax, n_act - r0);
            int nrep = 1;
            while (2 * nrep * kg <= 64)
                nrep *= 2;
            const int r = lane / nrep;
            const int q = lane & (nrep - 1);
            const bool ract = r < kg;
            const int rank = r0 + (ract ? r : 0);
            const float4 pr = rtp[rank];
            const float4 vr = rtv[rank];
            const float Hr = gamma_k * vr.w;
            const float H2r = ract ? Hr * Hr : -1.0f;
            const float invHr = fast_rcp(Hr);
            const float4 b0 = gbox[g][0], b1 = gbox[g][1];
            const float3 glo = make_float3(b0.x, b0.y, b0.z);
            const float3 ghi = make_float3(b1.x, b1.y, b1.z);
            // the group's candidates, buffer order kept
            int len = 0;
            for (int c0 = 0; c0 < nc; c0 += 64) {
                const int slot = c0 + lane;
                bool in = false;
                if (slot < nc) {
                    const float4 p = cp[slot];
                    in = box_dist2(p.x, p.y, p.z, glo, ghi) < b0.w;
                }
                const uint64_t m = __ballot(in);
                if (in)
                    gidx[len + lanes_below(m)] = uint8_t(slot);
                len += __popcll(m);
            }
            wave_sync();
            float S[kSums] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            int myn = 0;
            auto compute = [&]() __attribute__((always_inline)) {
                S[8] += float(myn);
                for (int k = 0; __any(k < myn); k += 4) {
                    const uint32_t four = *reinterpret_cast<const uint32_t *>(my_list + k);
                    float4 p[4], v[4];
#pragma unroll
                    for (int qq = 0; qq < 4; ++qq) {
                        const int c = k + qq < myn ? int((four >> (8 * qq)) & 0xffu) : CAP;
                        p[qq] = cp[c];
                        v[qq] = cv[c];
                    }
#pragma unroll
                    for (int qq = 0; qq < 4; ++qq)
                        dens_pair<false, K>(S, pr, vr, invHr, p[qq], v[qq], true);
                }
                myn = 0;
            };
            // replica q takes the group's candidates q, q + nrep, ...; entries
            // past the list read the dummy source, which no test accepts
            const int m_end = (len + nrep - 1) / nrep;
            for (int m = 0; m < m_end; m += 4) {
                int cq[4];
                float4 pq[4];
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) {
                    const int k = q + (m + qq) * nrep;
                    cq[qq] = k < len ? int(gidx[k]) : CAP;
                    pq[qq] = cp[cq[qq]];
                }
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) {
                    const float r2 = dist2(pr.x - pq[qq].x, pr.y - pq[qq].y, pr.z - pq[qq].z);
                    my_list[myn] = uint8_t(cq[qq]);
                    myn += r2 < H2r ? 1 : 0;
                }
                if (__any(myn > LMAX - 4))
                    compute();
            }
            compute();
            // the replicas' sums (butterfly), added to the receiver's
            for (int x = 1; x < nrep; x <<= 1)
#pragma unroll
                for (int k = 0; k < kSums; ++k)
                    S[k] += __shfl_xor(S[k], x, 64);
            if (ract && q == 0)
#pragma unroll
                for (int k = 0; k < kSums; ++k)
                    acc[k][rank] += S[k];
            wave_sync();  // the group list is rewritten by the next group
        }
        nc = 0;
    };

    // Append the kept sources of one task to the candidate buffer.
    auto emit = [&](const float4 &p, const float4 &v, bool keep) __attribute__((always_inline)) {
        const uint64_t mask = __ballot(keep);
        if (mask == 0)
            return;
        const int tot = __popcll(mask);
        if (nc + tot > CAP)
            flush();
        const int pos = nc + lanes_below(mask);
        if (keep) {
            cp[pos] = p;
            cv[pos] = v;
        }
        nc += tot;
    };

    const int32_t ta = tbeg[L], tn = tend[L] - ta;
    for (int32_t tb = ta; tb < ta + tn; tb += 64) {
        const int nb = min(64, ta + tn - tb);
        TaskRegs tr;
        tr.load(task, tb + lane, lane < nb);
        // whole source cells beyond R of the receivers' box are skipped
        if (lane < nb && task_box_dist2(tr.b.x, tr.b.y, tr.b.z, ext[tr.a.w], lo, hb) >= R2)
            tr.a.y = 0;
        for (int u = 0; u < nb; u += 4) {
            int j0[4], jc[4];
            float ox[4], oy[4], oz[4];
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const int k = min(u + qq, nb - 1);
                j0[qq] = bcast(tr.a.x, k);
                jc[qq] = (u + qq < nb) ? bcast(tr.a.y, k) : 0;
                ox[qq] = bcastf(tr.b.x, k);
                oy[qq] = bcastf(tr.b.y, k);
                oz[qq] = bcastf(tr.b.z, k);
            }
            float4 p[4], v[4];
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const bool in = lane < jc[qq];
                p[qq] = in ? q0[j0[qq] + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
                v[qq] = in ? q1[j0[qq] + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
            bool keep[4];
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                p[qq].x += ox[qq];
                p[qq].y += oy[qq];
                p[qq].z += oz[qq];
                keep[qq] = lane < jc[qq] && box_dist2(p[qq].x, p[qq].y, p[qq].z, lo, hb) < R2;
            }
            emit(p[0], v[0], keep[0]);
            emit(p[1], v[1], keep[1]);
            emit(p[2], v[2], keep[2]);
            emit(p[3], v[3], keep[3]);
        }
    }
    if (nc > 0)
        flush();
    wave_sync();
    if (lane < n_act) {
        float T[kSums];
#pragma unroll
        for (int k = 0; k < kSums; ++k)
            T[k] = acc[k][lane];
        const float hr = rtv[lane].w;
        const int32_t sr = s0 + int32_t(rts[lane]);
        dens_finish<K>(T, hr, fast_rcp(gamma_k * hr), sr, perm[sr], o);
    }
}

// List pass: lane = receiver s = 64 b + lane of 64-block b. Entries decode to
// (task, source index in its leaf); the task's offset half gives the source's
// first sorted index and the FP32 offset into the receiver's frame. Entries
// lie within the list radius (>= H); the r < H test is redone here, with
// the same arithmetic as the cell-pair loop.
template <int K>
__global__ __launch_bounds__(256) void k_dens_list(
    int64_t n, int64_t nwg_padded, const uint8_t *__restrict__ need,
    const float *__restrict__ hs, const float *__restrict__ lrad,
    const int32_t *__restrict__ leaf_of, const int32_t *__restrict__ perm,
    const int32_t *__restrict__ tbeg,
    const int32_t *__restrict__ tend, const Task *__restrict__ task,
    const float4 *__restrict__ q0, const float4 *__restrict__ q1,
    const int32_t *__restrict__ lcnt, const int64_t *__restrict__ lboff,
    const uint32_t *__restrict__ lst, float gamma_k, DensOut o)
{
    const int64_t wg = xcd_remap(blockIdx.x, nwg_padded);
    const int lane = threadIdx.x & 63;
    const int64_t b = wg * 4 + (threadIdx.x >> 6);
    const int64_t s_raw = b * 64 + lane;
    const bool valid = s_raw < n;
    const int64_t s = valid ? s_raw : 0;
    const float hi0 = hs[s];
    const bool act = valid && need[s] && gamma_k * hi0 <= lrad[s];
    if (!__any(act))
        return;  // no block-wide barrier in this kernel
    const int len = act ? lcnt[s] : 0;
    const float4 pi = q0[s];
    const float4 vi = q1[s];
    const float hi = act ? hi0 : 1.0f;
    const float H = gamma_k * hi;
    const float H2 = act ? H * H : -1.0f;
    const float invH = fast_rcp(H);
    const int32_t ta = act ? tbeg[leaf_of[s]] : 0;  // task 0 exists whenever n > 0
    const uint32_t *my = lst + lboff[b] + lane;
    const float4 *thalf = reinterpret_cast<const float4 *>(task) + 1;  // stride 2

    float S[kSums] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    constexpr int U = 4;
    for (int k = 0; __any(k < len); k += U) {
        uint32_t e[U];
#pragma unroll
        for (int q = 0; q < U; ++q)
            e[q] = (k + q < len) ? my[int64_t(k + q) * 64] : 0u;
        float4 T[U];
#pragma unroll
        for (int q = 0; q < U; ++q)
            T[q] = thalf[2 * int64_t(ta + int32_t(e[q] >> kListCodeShift))];
        float4 p[U], v[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int32_t j = __float_as_int(T[q].w) + int32_t(e[q] & 63u);
            p[q] = q0[j];
            v[q] = q1[j];
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            p[q].x += T[q].x;
            p[q].y += T[q].y;
            p[q].z += T[q].z;
            const float r2 = dist2(pi.x - p[q].x, pi.y - p[q].y, pi.z - p[q].z);
            dens_pair<true, K>(S, pi, vi, invH, p[q], v[q], k + q < len && r2 < H2);
        }
    }
    if (!act)
        return;
    dens_finish<K>(S, hi, invH, s, perm[s], o);
}

}  // namespace

static DensOut dens_out(const sphx_ctx *ctx, const sphx_grid *g, const sphx_density_out *o)
{
    return DensOut{o->rho,    o->rho_dh, o->n,      o->n_dh,     o->div_sum, o->curl_x,
                   o->curl_y, o->curl_z, o->nngb,   g->d0,       g->d1,      o->P_hat,
                   o->P_hat_dh, g->d2,   float(ctx->p.gamma_gas - 1.0)};
}

// Receivers whose H exceeds their leaf's task radius (the density loop's own
// staleness test), counted before the first pass of a step: a caller's h may
// have outgrown the task list since it was built, and a pass on a stale list
// would be thrown away. Any count > 0 makes the pass return at once.
__global__ __launch_bounds__(256) void k_stale_count(int64_t n, const uint8_t *__restrict__ need,
                                                     const float *__restrict__ hs,
                                                     const int32_t *__restrict__ leaf_of,
                                                     const float *__restrict__ radius,
                                                     float gamma_k, int32_t *__restrict__ stale)
{
    bool st = false;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256)
        st = st || (need[i] && gamma_k * hs[i] > radius[leaf_of[i]]);
    if (__syncthreads_or(st) && threadIdx.x == 0)
        atomicAdd(stale, 1);  // one per block: at most 1024 on one word
}

sphx_status probe_read(unsigned long long out[5], bool clear)
{
    SPHX_HIP(hipMemcpyFromSymbol(out, HIP_SYMBOL(probe_counts), 5 * sizeof(unsigned long long)));
    if (clear) {
        const unsigned long long zero[5] = {0, 0, 0, 0, 0};
        SPHX_HIP(hipMemcpyToSymbol(HIP_SYMBOL(probe_counts), zero, sizeof(zero)));
    }
    return SPHX_PROBE ? SPHX_OK : 1;
}

sphx_status stale_count_launch(const sphx_ctx *ctx, const sphx_grid *g, const sphx_tasks *t,
                               int32_t *stale, hipStream_t s)
{
    if (g->n == 0 || g->n_leaves == 0)
        return SPHX_OK;
    const int64_t nb = (g->n + 255) / 256;
    k_stale_count<<<unsigned(nb < 1024 ? nb : 1024), 256, 0, s>>>(
        g->n, g->need, g->hs, g->leaf_of, t->radius, float(ctx->p.gamma_k), stale);
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

// The loop shapes of one kernel kind. PE (the pressure-energy flavour's two
// extra sums) is built for the plain cell-pair loop only: the balanced,
// grouped and list loops are refused for that flavour when the context is
// made.
template <int K, bool PE>
static void density_shapes(int tile, int waves, int mode, int64_t nbp, const sphx_ctx *ctx,
                           const sphx_grid *g, const sphx_tasks *t, const float *lr,
                           const DensOut &dout, float far, int32_t *counters,
                           const int32_t *skip, hipStream_t s)
{
#define SPHX_DENSITY_LAUNCH(CAP_, NW_, BAL_)                                                   \
    k_density<CAP_, NW_, BAL_, K, PE><<<unsigned(nbp), 64 * NW_, 0, s>>>(                         \
        g->n_leaves, nbp, t->order, g->leaf_start, g->perm, g->q0, g->q1, g->need, g->hs,      \
        t->radius, t->slot, t->end, t->task, g->leaf_ext, float(ctx->p.gamma_k), far, lr,      \
        dout, counters, skip)
#define SPHX_DENSITY_TILES(NW_, BAL_)                                                          \
    do {                                                                                       \
        if (tile == 64)                                                                        \
            SPHX_DENSITY_LAUNCH(64, NW_, BAL_);                                                \
        else if (tile == 128)                                                                  \
            SPHX_DENSITY_LAUNCH(128, NW_, BAL_);                                               \
        else                                                                                   \
            SPHX_DENSITY_LAUNCH(256, NW_, BAL_);                                               \
    } while (0)
    if constexpr (PE) {
        if (waves == 1)
            SPHX_DENSITY_TILES(1, false);
        else
            SPHX_DENSITY_TILES(2, false);
        return;
    } else {
        if (mode == 2 && !lr) {
#define SPHX_DENSITY_GRP(CAP_)                                                                 \
    k_density_grp<CAP_, K><<<unsigned(nbp), 64, 0, s>>>(                                      \
        g->n_leaves, nbp, t->order, g->leaf_start, g->perm, g->q0, g->q1, g->need, g->hs,      \
        t->radius, t->slot, t->end, t->task, g->leaf_ext, float(ctx->p.gamma_k), far, dout,    \
        counters, skip)
            if (tile == 64)
                SPHX_DENSITY_GRP(64);
            else if (tile == 128)
                SPHX_DENSITY_GRP(128);
            else
                SPHX_DENSITY_GRP(256);
#undef SPHX_DENSITY_GRP
            return;
        }
        if (mode == 1)
            SPHX_DENSITY_TILES(1, true);
        else if (waves == 1)
            SPHX_DENSITY_TILES(1, false);
        else
            SPHX_DENSITY_TILES(2, false);
    }
#undef SPHX_DENSITY_TILES
#undef SPHX_DENSITY_LAUNCH
}

sphx_status density_launch(const sphx_ctx *ctx, const sphx_grid *g, const sphx_tasks *t,
                           const sphx_particles *in, const sphx_density_out *o,
                           int32_t *counters, bool use_lists, hipStream_t s, const int32_t *skip)
{
    if (g->n_leaves == 0)
        return SPHX_OK;
    const int64_t nbp = pad8(g->n_leaves);
    const int tile = ctx->p.density_tile ? ctx->p.density_tile : 128;
    const int waves = ctx->p.density_waves ? ctx->p.density_waves : 1;
    const int mode = ctx->p.density_balance;
    const float *lr = use_lists ? g->lrad : nullptr;
    const DensOut dout = dens_out(ctx, g, o);
    // the dummy source: 4 box lengths out, more than 3 box lengths from any
    // receiver (cell-relative coordinates), while every H is below a third
    const float far = float(4.0 * std::max(ctx->p.box[0], std::max(ctx->p.box[1], ctx->p.box[2])));
    SPHX_HIP(ctx->prof->begin(0, s));
    if (smoothed_pressure(ctx->p.flavour)) {
        SPHX_WITH_KERNEL(ctx->p.kernel, (density_shapes<KK, true>(tile, waves, mode, nbp, ctx, g,
                                                                  t, lr, dout, far, counters,
                                                                  skip, s)));
    } else {
        SPHX_WITH_KERNEL(ctx->p.kernel, (density_shapes<KK, false>(tile, waves, mode, nbp, ctx,
                                                                   g, t, lr, dout, far, counters,
                                                                   skip, s)));
    }
    SPHX_HIP(hipGetLastError());
    SPHX_HIP(ctx->prof->end(0, s));
    return SPHX_OK;
}

sphx_status density_list_launch(const sphx_ctx *ctx, const sphx_grid *g, const sphx_tasks *t,
                                const sphx_density_out *o, hipStream_t s)
{
    if (g->n == 0)
        return SPHX_OK;
    const int64_t nwg = (g->n + 255) / 256;
    const int64_t nwgp = pad8(nwg);
    SPHX_HIP(ctx->prof->begin(2, s));
    SPHX_WITH_KERNEL(ctx->p.kernel,
                     (k_dens_list<KK><<<unsigned(nwgp), 256, 0, s>>>(
                         g->n, nwgp, g->need, g->hs, g->lrad, g->leaf_of, g->perm, t->slot, t->end,
                         t->task, g->q0, g->q1, g->lcnt, g->lboff, g->lst,
                         float(ctx->p.gamma_k), dens_out(ctx, g, o))));
    SPHX_HIP(hipGetLastError());
    SPHX_HIP(ctx->prof->end(2, s));
    return SPHX_OK;
}

}  // namespace sphx
