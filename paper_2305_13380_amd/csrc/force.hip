// Force pass (Section 3.2 density-energy equations of motion with the
// Balsara-switched artificial viscosity; Section 3.3 symmetric alpha_ij and
// artificial conduction) and the FP64 global momentum / energy sums.
//
// The loop structure (cull, candidate buffer, per-lane lists) is described in
// pairs.h; the force set of receiver i is every j != i with r_ij < max(H_i, H_j).
#include <mutex>

#include "pairs.h"

namespace sphx {
namespace {


// Source state of the force pass in sorted order, from the caller's arrays:
// (h, rho, P, c) and (f, B, A, 0), with the pressure-energy flavour
// (gm1sq = (gamma - 1)^2 > 0) (f, B, F, (gamma - 1)^2 u / P_hat); with
// skip_active, only for the inactive particles (a step's ghost has written
// the active ones). One thread per caller index: the seven reads are
// coalesced and only the two 16-byte records are scattered (read through the
// permutation, every 4-byte field would cost a cache line of its own).
__global__ void k_force_state(int64_t n, const int32_t *__restrict__ inv,
                              const float *__restrict__ h, const float *__restrict__ rho,
                              const float *__restrict__ P, const float *__restrict__ c,
                              const float *__restrict__ f, const float *__restrict__ B,
                              const float *__restrict__ A, const float *__restrict__ u,
                              float gm1sq, const uint8_t *__restrict__ skip_active,
                              float4 *__restrict__ g0, float4 *__restrict__ g1)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    if (skip_active && skip_active[i])
        return;
    const int32_t s = inv[i];
    g0[s] = make_float4(h[i], rho[i], P[i], c[i]);
    g1[s] = make_float4(f[i], B[i], A[i], gm1sq > 0.0f ? gm1sq * u[i] / P[i] : 0.0f);
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int kFSums = 7;  // ax, ay, az, du, vsig, count, viscous part of du

// CAP >= 64: a task's kept sources (up to 64) always fit after a flush.
// Inside a step the ghost leaves its results in sorted order only, and the
// force kernel writes them to the caller's arrays for its receivers (every
// particle the step finalised): h, f, P, c, B, A from the force state, div,
// curl and the converged flag from g2. h == null: nothing to write.
struct StepOut {
    float *h, *f, *P, *c, *B, *A, *div, *curl;
    uint8_t *conv;
    const float4 *g2;
};

// FLAV: SPHX_FLAVOUR_* (0 density-energy; 1 density-entropy, Section 3.2:
// the particles' u is the adiabat A (their P came from A rho^gamma in the
// ghost), no conduction, and the output rate is dA/dt = (gamma - 1)
// rho^(1 - gamma) du/dt|visc, the FP64 energy sum keeping the internal-energy
// rate; 2 the Phantom-like flavour of Appendix A: conduction with alpha_c = 1
// and the speed sqrt(2 |P_i - P_j| / (rho_i + rho_j)); 3 pressure-energy,
// Appendix A: P is the smoothed pressure and the pressure terms are
// m_j (gamma - 1)^2 u_i u_j (f_ij g_i / P_i + f_ji g_j / P_j) with f_ij = 1 -
// F_i / (m_j u_j), no conduction; per particle the state holds F and Q =
// (gamma - 1)^2 u / P, so that with R = Q F the pair needs only
// g_i (Q_i m_j u_j - R_i) + g_j (Q_j m_j u_i - R_j m_j / m_i); 4 Anarchy-PU,
// Appendix A: 3 plus conduction with the mean alpha_c and the speed c_i +
// c_j + mu, its source alpha_c staged where the other flavours keep P_j); 5
// GDF, Appendix A: f is the geometric-density correction and A holds
// alpha_c; the pressure terms are (P_i + P_j) G / (2 rho_i rho_j) on the mean
// gradient G / 2, du/dt takes P_i alone plus the conduction m_j (alpha_c,i +
// alpha_c,j)(u_i - u_j) G / ((rho_i + rho_j) r), with the density flavours'
// viscosity).
template <int CAP, int NW, int K, int FLAV>
__global__ __launch_bounds__(64 * NW) void k_force(
    int64_t n_leaves, int64_t nb_padded, const int32_t *__restrict__ order,
    const int32_t *__restrict__ leaf_start,
    const int32_t *__restrict__ perm, const float4 *__restrict__ q0,
    const float4 *__restrict__ q1, const float2 *__restrict__ qa, const float4 *__restrict__ g0,
    const float4 *__restrict__ g1, const uint8_t *__restrict__ active,
    const int32_t *__restrict__ tbeg,
    const int32_t *__restrict__ tend, const Task *__restrict__ task,
    const float4 *__restrict__ ext, const float *__restrict__ hmax, float gamma_k, float beta,
    float far,
    float *__restrict__ o_ax, float *__restrict__ o_ay, float *__restrict__ o_az,
    float *__restrict__ o_du, float *__restrict__ o_vsig, int32_t *__restrict__ o_nf,
    double *__restrict__ fsum, const int32_t *__restrict__ gate, StepOut so, float gamma_gas)
{
    if (gate && *gate)
        return;  // a captured step whose iteration is not finished
    static_assert(CAP >= 64 && CAP <= 256, "candidate slots: one task's sources, 8-bit slots");
    const int64_t L = leaf_of_block(blockIdx.x, nb_padded, order);
    if (L >= n_leaves)
        return;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int32_t s0 = leaf_start[L];
    const int32_t cnt = leaf_start[L + 1] - s0;
    const bool valid = lane < cnt;
    const int32_t s = s0 + (valid ? lane : 0);
    const int32_t gi = perm[s];
    const bool act = valid && (active ? active[gi] != 0 : true);
    if (!__any(act)) {
        if (w == 0 && lane < 6)
            fsum[6 * L + lane] = 0.0;
        return;
    }

    // x, y, z (receiver cell frame), H^2; slot CAP is a dummy source beyond
    // every support (H^2 = 0) that the replicated tests read past the buffer
    __shared__ float4 cp_all[NW][CAP + 1];
    __shared__ float4 cv_all[NW][CAP];  // vx, vy, vz, m
    __shared__ float4 ca_all[NW][CAP];  // 1/H, c, rho, P
    __shared__ float4 cb_all[NW][CAP];  // f, A, B, alpha_v
    __shared__ float2 cc_all[NW][CAP];  // alpha_c P, u
    __shared__ uint32_t lst_all[NW][kListStride * 16];
    float4 *cp = cp_all[w], *cv = cv_all[w], *ca = ca_all[w], *cb = cb_all[w];
    if (lane == 0)
        cp[CAP] = make_float4(far, far, far, 0.0f);
    float2 *cc = cc_all[w];
    uint8_t *lst = reinterpret_cast<uint8_t *>(lst_all[w]);
    uint8_t *my_list = lst + lane * kListStride;

    // the box of the receivers, and their largest radius
    const float4 pown = q0[s];
    const float Hown = gamma_k * g0[s].x;
    const float inf = __builtin_inff();
    float3 lo = make_float3(act ? pown.x : inf, act ? pown.y : inf, act ? pown.z : inf);
    float3 hb = make_float3(act ? pown.x : -inf, act ? pown.y : -inf, act ? pown.z : -inf);
    lo.x = wave_minf(lo.x);
    lo.y = wave_minf(lo.y);
    lo.z = wave_minf(lo.z);
    hb.x = wave_maxf(hb.x);
    hb.y = wave_maxf(hb.y);
    hb.z = wave_maxf(hb.z);
    const float R = wave_maxf(act ? Hown : 0.0f);
    const float R2 = R * R;

    // Lane replication, as in the density loop: with n_act receivers, each
    // gets nrep lanes (the largest power of two with nrep n_act <= 64);
    // replica j takes the candidates whose running index is j mod nrep, and
    // the replicas' sums (max for v_sig) are combined by a butterfly at the
    // end. nrep = 1 is the plain loop, lane = receiver.
    const uint64_t amask = __ballot(act);
    const int n_act = __popcll(amask);
    int nrep = 1;
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
        src = ract ? int(rmap_all[w][k]) : 0;
    }
    const int rj = lane & (nrep - 1);  // replica index
    // this lane's receiver (its own particle when nrep = 1; idle lanes read
    // the cell's first particle)
    const int32_t sr = nrep > 1 ? s0 + src : s;
    const int32_t gr = nrep > 1 ? perm[sr] : gi;
    const float4 pi = nrep > 1 ? q0[sr] : pown;
    const float4 vi = q1[sr];  // w = u
    const float2 ai = qa[sr];
    const float4 gi0 = g0[sr];  // h, rho, P, c
    const float4 gi1 = g1[sr];  // f, B, A
    const float Hi = gamma_k * gi0.x;
    const float Hi2 = ract ? Hi * Hi : -1.0f;
    const float invHi = fast_rcp(Hi);
    const float invHi4 = (invHi * invHi) * (invHi * invHi);
    const float rhoi = gi0.y, Pi = gi0.z, ci = gi0.w;
    const float fi = gi1.x, Bi = gi1.y, Ai = gi1.z;
    // pressure-energy: the receiver's Q, R = Q F, u and 1/m (else unused)
    const float Qi = gi1.w, Ri = gi1.w * gi1.z, ui_ = vi.w;
    const float inv_mi = FLAV == 3 || FLAV == 4 ? fast_rcp(pi.w) : 0.0f;
    const float acPi = ai.y * Pi;

    float ax = 0.f, ay = 0.f, az = 0.f, du = 0.f, duv = 0.f;
    float vsig = 2.0f * ci;
    int32_t nf = 0;
    int nc = 0;
    int myn = 0;  // this lane's list length (its own particle is listed too)
    int gbase = 0;  // candidates of the earlier buffers (wave-uniform)

    // One listed pair; with on = false (past the lane's list, which reads
    // slot 0, or its own particle) it adds exactly nothing, without branches.
    auto pair = [&](int c, bool listed) __attribute__((always_inline)) {
        const float4 p = cp[c];
        const float dx = pi.x - p.x, dy = pi.y - p.y, dz = pi.z - p.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const bool on = listed && r2 > 0.0f;
        const float4 v = cv[c];
        const float4 a = ca[c];
        const float4 b = cb[c];
        const float2 c2 = cc[c];
        // 1/r = 0 for entries past the list (slot 0: finite data) and the
        // receiver's own particle: r, both gradients, G and nu are then 0 and
        // every sum below adds exactly zero without a select
        const float rinv = on ? fast_rsq(r2) : 0.0f;
        const float r = r2 * rinv;
        // dW/dr of either end at u clamped to the support (0 beyond it)
        constexpr float kD = Kern<K>::kD;
        const float ui = r * invHi;
        const float gi = -kD * invHi4 * Kern<K>::mdw(fminf(ui, 1.0f));
        const float uj = r * a.x;
        const float ij2 = a.x * a.x;
        const float gj = -kD * (ij2 * ij2) * Kern<K>::mdw(fminf(uj, 1.0f));
        const float ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
        const float dvx = vi.x - v.x, dvy = vi.y - v.y, dvz = vi.z - v.z;
        const float vdote = dvx * ex + dvy * ey + dvz * ez;
        const float mu = vdote < 0.0f ? vdote : 0.0f;
        const float vs = ci + a.y - beta * mu;
        vsig = on ? fmaxf(vsig, vs) : vsig;
        const float alpha = 0.25f * (ai.x + b.w) * (Bi + b.z);
        const float irs = fast_rcp(rhoi + a.z);
        const float nu = -2.0f * alpha * mu * vs * irs;
        // a kernel term outside its own support (or of an entry that is not
        // a pair) is zero, also when f is infinite (a particle alone in its
        // support at a fixed h)
        const bool in_i = on && ui < 1.0f, in_j = on && uj < 1.0f;
        const float fgi = in_i ? fi * gi : 0.0f, fgj = in_j ? b.x * gj : 0.0f;
        const float G = fgi + fgj;
        const float m = v.w;
        // the pressure terms of i and j (pressure-energy: already times m_j,
        // with the source's b.y = m_j Q_j, c2.x = m_j R_j, c2.y = m_j u_j)
        const float Agi =
            in_i ? (FLAV == 3 || FLAV == 4 ? gi * (Qi * c2.y - Ri) : Ai * gi) : 0.0f;
        const float Agj =
            in_j ? (FLAV == 3 || FLAV == 4 ? gj * (b.y * ui_ - c2.x * inv_mi) : b.y * gj) : 0.0f;
        // GDF: P / (rho_i rho_j) on the mean gradient (0 when G is)
        const float pij = FLAV == 5 ? 0.5f * G * fast_rcp(rhoi * a.z) : 0.0f;
        const float macc = FLAV == 5   ? m * ((Pi + a.w) * pij + 0.5f * nu * G)
                           : FLAV >= 3 ? Agi + Agj + m * (0.5f * nu * G)
                                       : m * (Agi + Agj + 0.5f * nu * G);
        const float psum = Pi + a.w;
        const float ac =
            FLAV == 2 ? 1.0f : (psum > 0.0f ? (acPi + c2.x) * fast_rcp(psum) : 0.0f);
        const float vc =
            (FLAV == 2 ? 0.0f : fabsf(vdote)) + fast_sqrt(2.0f * fabsf(Pi - a.w) * irs);
        const float dvi = m * (0.25f * nu * G) * vdote;
        // Anarchy-PU: the mean alpha_c (the source's in a.w) and the speed
        // c_i + c_j + mu, with m_j (u_i - u_j) = m_j u_i - c2.y
        const float cond4 =
            FLAV == 4 ? 0.5f * (ai.y + a.w) * (ci + a.y + mu) * (m * ui_ - c2.y) * G * irs : 0.0f;
        // GDF conduction: alpha_c,i in A_i, alpha_c,j in b.y; 1/r = 0 off the list
        const float dui = FLAV == 5
                              ? m * ((Pi * pij + 0.25f * nu * G) * vdote +
                                     (Ai + b.y) * (vi.w - c2.y) * G * irs * rinv)
                          : FLAV == 4 ? Agi * vdote + dvi + cond4
                          : FLAV == 3 ? Agi * vdote + dvi
                          : FLAV == 1 ? m * Agi * vdote + dvi
                                      : m * (Agi + 0.25f * nu * G) * vdote +
                                            m * ac * vc * (vi.w - c2.y) * G * irs;
        if (FLAV == 1)
            duv += dvi;
        ax -= macc * ex;
        ay -= macc * ey;
        az -= macc * ez;
        du += dui;
    };
    // Every listed entry is a force neighbour (the receiver's own particle
    // too, subtracted at the end): counted at once.
    auto compute = [&]() __attribute__((always_inline)) {
        nf += myn;
        for (int k = 0; __any(k < myn); k += 4) {
            const uint32_t four = *reinterpret_cast<const uint32_t *>(my_list + k);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool listed = k + q < myn;
                pair(listed ? int((four >> (8 * q)) & 0xffu) : 0, listed);
            }
        }
        myn = 0;
    };
    // The slot is always written; it is kept (the length advanced) only
    // when the pair lies inside max(H_i, H_j).
    auto accept = [&](int c, const float4 &p, bool ok) __attribute__((always_inline)) {
        const float dx = pi.x - p.x, dy = pi.y - p.y, dz = pi.z - p.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        my_list[myn] = uint8_t(c);
        myn += (ok && ract && r2 < fmaxf(Hi2, p.w)) ? 1 : 0;
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
                if (__any(myn > kListMax - 4))
                    compute();
            }
            for (; c < nc; ++c)
                accept(c, cp[c], true);
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
        }
        compute();
        gbase += nc;
        wave_sync();
        nc = 0;
    };

    // Append the kept sources of one task to the candidate buffer.
    auto emit = [&](const float4 &p, float Hj, bool keep, int j0) __attribute__((always_inline)) {
        const uint64_t mask = __ballot(keep);
        if (mask == 0)
            return;
        const int tot = __popcll(mask);
        if (nc + tot > CAP)
            flush();
        const int pos = nc + lanes_below(mask);
        if (keep) {
            const int sj = j0 + lane;
            const float4 v = q1[sj];
            const float2 a = qa[sj];
            const float4 h0 = g0[sj];
            const float4 h1 = g1[sj];
            cp[pos] = make_float4(p.x, p.y, p.z, Hj * Hj);
            cv[pos] = make_float4(v.x, v.y, v.z, p.w);
            // (Anarchy-PU keeps alpha_c,j in place of P_j, which its pair
            // terms do not read)
            ca[pos] = make_float4(fast_rcp(Hj), h0.w, h0.y, FLAV == 4 ? a.y : h0.z);
            if (FLAV == 3 || FLAV == 4) {
                // m_j Q_j, m_j R_j = m_j Q_j F_j, m_j u_j
                cb[pos] = make_float4(h1.x, p.w * h1.w, h1.y, a.x);
                cc[pos] = make_float2(p.w * h1.w * h1.z, p.w * v.w);
            } else {
                cb[pos] = make_float4(h1.x, h1.z, h1.y, a.x);
                cc[pos] = make_float2(a.y * h0.z, v.w);
            }
        }
        nc += tot;
    };

    // This wave's share: the tasks of the source cells J with J mod NW = w
    // (a split that the list's length does not move).
    const int32_t ta = tbeg[L], t_end = tend[L];
    for (int32_t tb = ta; tb < t_end; tb += 64) {
        const int nb = min(64, t_end - tb);
        TaskRegs tr;
        tr.load(task, tb + lane, lane < nb);
        // whole source cells beyond max(R, the cell's largest H_j) of the
        // receivers' box are skipped
        if (lane < nb) {
            const float rj = hmax[tr.a.w];
            if ((NW > 1 && tr.a.w % NW != w) ||
                task_box_dist2(tr.b.x, tr.b.y, tr.b.z, ext[tr.a.w], lo, hb) >= fmaxf(R2, rj * rj))
                tr.a.y = 0;
        }
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
            float hj[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool in = lane < jc[q];
                p[q] = in ? q0[j0[q] + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
                hj[q] = in ? g0[j0[q] + lane].x : 0.0f;
            }
            bool keep[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                p[q].x += ox[q];
                p[q].y += oy[q];
                p[q].z += oz[q];
                const float Hj = gamma_k * hj[q];
                hj[q] = Hj;
                keep[q] = lane < jc[q] &&
                          box_dist2(p[q].x, p[q].y, p[q].z, lo, hb) < fmaxf(R2, Hj * Hj);
            }
            emit(p[0], hj[0], keep[0], j0[0]);
            emit(p[1], hj[1], keep[1], j0[1]);
            emit(p[2], hj[2], keep[2], j0[2]);
            emit(p[3], hj[3], keep[3], j0[3]);
        }
    }
    if (nc > 0)
        flush();
    // the replicas' partial results, by a butterfly: every replica ends with
    // the same totals (each addition and max is commutative)
    for (int o = 1; o < nrep; o <<= 1) {
        ax += __shfl_xor(ax, o, 64);
        ay += __shfl_xor(ay, o, 64);
        az += __shfl_xor(az, o, 64);
        du += __shfl_xor(du, o, 64);
        if (FLAV == 1)
            duv += __shfl_xor(duv, o, 64);
        vsig = fmaxf(vsig, __shfl_xor(vsig, o, 64));
        nf += __shfl_xor(nf, o, 64);
    }

    // the receiver's own particle was listed as a pair at r = 0 and counted
    float F[kFSums] = {ax, ay, az, du, vsig, float(nf - (w == 0 && ract ? 1 : 0)), duv};
    if (NW > 1) {
        __syncthreads();
        // the other waves' partial sums (own array: small tiles leave too
        // little room in the candidate buffers)
        __shared__ float red[NW > 1 ? (NW - 1) * kFSums * 64 : 1];
        if (w > 0)
            for (int k = 0; k < kFSums; ++k)
                red[((w - 1) * kFSums + k) * 64 + lane] = F[k];
        __syncthreads();
        if (w > 0)
            return;
        for (int w2 = 1; w2 < NW; ++w2) {
            for (int k = 0; k < 4; ++k)
                F[k] += red[((w2 - 1) * kFSums + k) * 64 + lane];
            F[4] = fmaxf(F[4], red[((w2 - 1) * kFSums + 4) * 64 + lane]);
            F[5] += red[((w2 - 1) * kFSums + 5) * 64 + lane];
            F[6] += red[((w2 - 1) * kFSums + 6) * 64 + lane];
        }
    }
    double m0 = 0, m1 = 0, m2 = 0, e = 0, sa_ = 0, sd = 0;
    if (ract && rj == 0) {
        o_ax[gr] = F[0];
        o_ay[gr] = F[1];
        o_az[gr] = F[2];
        o_du[gr] = FLAV == 1 ? (gamma_gas - 1.0f) * powf(rhoi, 1.0f - gamma_gas) * F[6] : F[3];
        o_vsig[gr] = F[4];
        if (o_nf)
            o_nf[gr] = int32_t(F[5]);
        if (so.h) {
            const float4 e = so.g2[sr];  // div, curl, converged
            so.h[gr] = gi0.x;
            so.f[gr] = gi1.x;
            so.P[gr] = gi0.z;
            so.c[gr] = gi0.w;
            so.B[gr] = gi1.y;
            so.A[gr] = gi1.z;
            so.div[gr] = e.x;
            so.curl[gr] = e.y;
            so.conv[gr] = e.z != 0.0f ? 1 : 0;
        }
        const double mi = pi.w;
        const double dax = F[0], day = F[1], daz = F[2], ddu = F[3];
        m0 = mi * dax;
        m1 = mi * day;
        m2 = mi * daz;
        e = mi * (double(vi.x) * dax + double(vi.y) * day + double(vi.z) * daz + ddu);
        sa_ = mi * sqrt(dax * dax + day * day + daz * daz);
        sd = mi * fabs(ddu);
    }
    m0 = wave_sum(m0);
    m1 = wave_sum(m1);
    m2 = wave_sum(m2);
    e = wave_sum(e);
    sa_ = wave_sum(sa_);
    sd = wave_sum(sd);
    if (lane == 0) {
        double *o = fsum + 6 * L;
        o[0] = m0;
        o[1] = m1;
        o[2] = m2;
        o[3] = e;
        o[4] = sa_;
        o[5] = sd;
    }
}

// One wave per leaf: the largest search radius gamma_k h of the leaf's
// particles in the force-pass state (their final h), which bounds every H_j
// of a source cell more tightly than the task list's radius.
__global__ __launch_bounds__(64) void k_leaf_hmax(int64_t n_leaves,
                                                  const int32_t *__restrict__ leaf_start,
                                                  const float4 *__restrict__ g0, float gamma_k,
                                                  float *__restrict__ hmax,
                                                  const int32_t *__restrict__ gate)
{
    const int64_t L = blockIdx.x;
    if (L >= n_leaves || (gate && *gate))
        return;
    const int lane = threadIdx.x;
    const int32_t s0 = leaf_start[L], cnt = leaf_start[L + 1] - s0;
    float v = lane < cnt ? g0[s0 + lane].x : 0.0f;
    for (int o = 32; o > 0; o >>= 1)
        v = fmaxf(v, __shfl_xor(v, o, 64));
    if (lane == 0)
        hmax[L] = gamma_k * v;
}

// Fixed-order FP64 reduction of the per-leaf partial sums in two levels, per
// particle set: block b of kSumParts sums its contiguous range of the set's
// leaves (threads stride the range, then a tree over the block), and one
// block per set sums its parts in order. A set's sums so do not depend on the
// other sets in the grid.
constexpr int kSumParts = 128;

__global__ __launch_bounds__(256) void k_sum_leaves(int64_t n_leaves,
                                                    const int32_t *__restrict__ set_leaf,
                                                    const double *__restrict__ fsum,
                                                    double *__restrict__ part,
                                                    const int32_t *__restrict__ gate)
{
    if (gate && *gate)
        return;
    __shared__ double red[6][256];
    const int t = threadIdx.x;
    // set blockIdx.y's leaves (all of them with one set)
    const int64_t lo = set_leaf ? set_leaf[blockIdx.y] : 0;
    const int64_t hi = set_leaf ? set_leaf[blockIdx.y + 1] : n_leaves;
    const int64_t per = (hi - lo + kSumParts - 1) / kSumParts;
    const int64_t a0 = lo + int64_t(blockIdx.x) * per;
    const int64_t a1 = min(hi, a0 + per);
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t L = a0 + t; L < a1; L += 256)
        for (int k = 0; k < 6; ++k)
            a[k] += fsum[6 * L + k];
    for (int k = 0; k < 6; ++k)
        red[k][t] = a[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int k = 0; k < 6; ++k)
                red[k][t] += red[k][t + w];
        __syncthreads();
    }
    if (t < 6)
        part[6 * (int64_t(blockIdx.y) * kSumParts + blockIdx.x) + t] = red[t][0];
}

// One block per set: the set's parts summed in order.
__global__ __launch_bounds__(kSumParts) void k_sum_parts(const double *__restrict__ part,
                                                         double *__restrict__ out,
                                                         const int32_t *__restrict__ gate)
{
    if (gate && *gate)
        return;
    __shared__ double red[6][kSumParts];
    const int t = threadIdx.x;
    const double *p = part + 6 * int64_t(blockIdx.x) * kSumParts;
    for (int k = 0; k < 6; ++k)
        red[k][t] = p[6 * t + k];
    __syncthreads();
    for (int w = kSumParts / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int k = 0; k < 6; ++k)
                red[k][t] += red[k][t + w];
        __syncthreads();
    }
    if (t < 6)
        out[6 * blockIdx.x + t] = red[t][0];
}

// Clears the six FP64 sums of every set of an empty grid (a kernel, not a
// memset node, so that the call can be recorded in a graph).
__global__ void k_zero_sums(double *__restrict__ out, int64_t n)
{
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
        out[i] = 0.0;
}

}  // namespace

// Fixed workspace of sphx_force_noalloc: the per-leaf FP64 partial sums of
// the force kernel (6 per leaf) followed by the kSumParts parts of their
// reduction, for at most kNoallocLeaves leaves (25.2 MB). Every device the
// library runs on holds its own copy until the process ends. Every entry
// is written before it is read in each call (each leaf writes its six, the
// reduction its parts), so nothing needs clearing between calls; calls that
// overlap on one device share it and race.
static __device__ __align__(256) double scratch[6 * (kNoallocLeaves + kSumParts)];

sphx_status noalloc_scratch(int device, double **out)
{
    static std::mutex mu;
    static double *ptr[kNoallocMaxDevices] = {};
    if (device < 0 || device >= kNoallocMaxDevices) {
        set_error("fixed workspace: device index out of range");
        return SPHX_E_INVALID;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[device]) {
        // `device` is current: the array's address on it (each device holds
        // its own copy at its own address)
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("fixed workspace: hipGetSymbolAddress: ") +
                      hipGetErrorString(e));
            return SPHX_E_HIP;
        }
        ptr[device] = static_cast<double *>(p);
    }
    *out = ptr[device];
    return SPHX_OK;
}

// The loop shapes of one kernel kind.
template <int K, int FLAV>
static void force_shapes(int tile, int waves, int64_t nbp, const sphx_ctx *ctx,
                         const sphx_grid *g, const sphx_tasks *t, const sphx_particles *in,
                         const sphx_force_out *o, float far, const int32_t *gate,
                         const StepOut &so, double *fsum, hipStream_t s)
{
#define SPHX_FORCE_LAUNCH(CAP_, NW_)                                                           \
    k_force<CAP_, NW_, K, FLAV><<<unsigned(nbp), 64 * NW_, 0, s>>>(                               \
        g->n_leaves, nbp, t->order, g->leaf_start, g->perm, g->q0, g->q1, g->qa, g->g0, g->g1, \
        in->active, t->slot, t->end, t->task, g->leaf_ext, g->leaf_hmax,                       \
        float(ctx->p.gamma_k), float(ctx->p.beta_v), far, o->ax,                               \
        o->ay, o->az, o->du_dt, o->v_sig, o->nforce, fsum, gate, so, float(ctx->p.gamma_gas))
    if (waves == 1) {
        if (tile == 64)
            SPHX_FORCE_LAUNCH(64, 1);
        else
            SPHX_FORCE_LAUNCH(128, 1);
    } else {
        if (tile == 64)
            SPHX_FORCE_LAUNCH(64, 2);
        else
            SPHX_FORCE_LAUNCH(128, 2);
    }
#undef SPHX_FORCE_LAUNCH
}

sphx_status force_launch(const sphx_ctx *ctx, const sphx_grid *g, const sphx_tasks *t,
                         const sphx_particles *in, const sphx_density_out *d,
                         const sphx_ghost_out *gs, const sphx_force_out *o, double *sums6,
                         hipStream_t s, const int32_t *gate, bool state_ready,
                         double *fsum_fixed)
{
    if (g->n_leaves == 0) {
        if (sums6) {
            k_zero_sums<<<1, 64, 0, s>>>(sums6, 6 * int64_t(g->n_sets));
            SPHX_HIP(hipGetLastError());
        }
        return SPHX_OK;
    }
    // the partial sums: the grid's workspace, or the fixed one
    double *fsum = fsum_fixed ? fsum_fixed : g->fsum;
    // (no kernel timing in the fixed-workspace call: creating timing events
    // would allocate)
    Profiler *prof = fsum_fixed ? nullptr : ctx->prof;
    if (!state_ready || in->active) {
        k_force_state<<<unsigned((g->n + 255) / 256), 256, 0, s>>>(
            g->n, g->inv, in->h, d->rho, gs->P, gs->c, gs->f, gs->balsara, gs->A, in->u,
            smoothed_pressure(ctx->p.flavour)
                ? float((ctx->p.gamma_gas - 1.0) * (ctx->p.gamma_gas - 1.0))
                : 0.0f,
            state_ready ? in->active : nullptr, g->g0, g->g1);
        SPHX_HIP(hipGetLastError());
    }
    if (state_ready && ctx->p.flavour == SPHX_FLAVOUR_GDF)
        SPHX_TRY(gdf_step_launch(ctx, g, t, in, gate, s));
    k_leaf_hmax<<<unsigned(g->n_leaves), 64, 0, s>>>(g->n_leaves, g->leaf_start, g->g0,
                                                      float(ctx->p.gamma_k), g->leaf_hmax, gate);
    SPHX_HIP(hipGetLastError());
    const StepOut so = state_ready ? StepOut{in->h,         gs->f, gs->P,      gs->c,
                                             gs->balsara,   gs->A, gs->div_v,  gs->curl_v,
                                             gs->converged, g->g2}
                                   : StepOut{nullptr, nullptr, nullptr, nullptr, nullptr,
                                             nullptr, nullptr, nullptr, nullptr, nullptr};
    // the dummy source: 4 box lengths out, more than 3 box lengths from any
    // receiver (cell-relative coordinates), while every H is below a third
    const float far = float(4.0 * std::max(ctx->p.box[0], std::max(ctx->p.box[1], ctx->p.box[2])));
    const int64_t nbp = pad8(g->n_leaves);
    if (prof)
        SPHX_HIP(prof->begin(1, s));
    const int tile = ctx->p.force_tile ? ctx->p.force_tile : 64;
    const int waves = ctx->p.force_waves ? ctx->p.force_waves : 1;
    if (ctx->p.flavour == SPHX_FLAVOUR_DENSITY_ENTROPY) {
        SPHX_WITH_KERNEL(ctx->p.kernel, (force_shapes<KK, 1>(tile, waves, nbp, ctx, g, t, in, o,
                                                              far, gate, so, fsum, s)));
    } else if (ctx->p.flavour == SPHX_FLAVOUR_PHANTOM) {
        SPHX_WITH_KERNEL(ctx->p.kernel, (force_shapes<KK, 2>(tile, waves, nbp, ctx, g, t, in, o,
                                                              far, gate, so, fsum, s)));
    } else if (ctx->p.flavour == SPHX_FLAVOUR_PRESSURE_ENERGY) {
        SPHX_WITH_KERNEL(ctx->p.kernel, (force_shapes<KK, 3>(tile, waves, nbp, ctx, g, t, in, o,
                                                              far, gate, so, fsum, s)));
    } else if (ctx->p.flavour == SPHX_FLAVOUR_ANARCHY_PU) {
        SPHX_WITH_KERNEL(ctx->p.kernel, (force_shapes<KK, 4>(tile, waves, nbp, ctx, g, t, in, o,
                                                              far, gate, so, fsum, s)));
    } else if (ctx->p.flavour == SPHX_FLAVOUR_GDF) {
        SPHX_WITH_KERNEL(ctx->p.kernel, (force_shapes<KK, 5>(tile, waves, nbp, ctx, g, t, in, o,
                                                              far, gate, so, fsum, s)));
    } else {
        SPHX_WITH_KERNEL(ctx->p.kernel, (force_shapes<KK, 0>(tile, waves, nbp, ctx, g, t, in, o,
                                                              far, gate, so, fsum, s)));
    }
    SPHX_HIP(hipGetLastError());
    if (prof)
        SPHX_HIP(prof->end(1, s));
    if (sums6) {
        // the six sums of every set (one set: of the whole grid)
        double *part = fsum + 6 * g->n_leaves;
        k_sum_leaves<<<dim3(kSumParts, unsigned(g->n_sets)), 256, 0, s>>>(
            g->n_leaves, g->set_leaf, fsum, part, gate);
        SPHX_HIP(hipGetLastError());
        k_sum_parts<<<unsigned(g->n_sets), kSumParts, 0, s>>>(part, sums6, gate);
        SPHX_HIP(hipGetLastError());
    }
    return SPHX_OK;
}

}  // namespace sphx
