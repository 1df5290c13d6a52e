// The rest of SPHENIX (Section 3.3) and the time integration (Sections 2.4
// and 3.4) on the cell structure of a step:
//
// * gradient loop: for every active receiver i over j != i with
//   0 < r_ij < H_i, the Laplacian of u (Brookshaw's second-derivative form)
//   lap_u_i = 2 sum_j (m_j/rho_j)(u_i - u_j) (dW/dr)/r, the conduction speed
//   vc_i = max_j (|v_ij . x_ij|/r_ij + sqrt(2|P_i - P_j|/(rho_i + rho_j))) (for
//   Anarchy-PU, Appendix A: max_j (c_i + c_j + min(0, v_ij . x_ij)/r_ij) with
//   the flavour's sound speed c = sqrt(gamma P / rho)) and the largest
//   alpha_V among i and its neighbours;
// * the conduction parameter over a step: its linear evolution equation
//   with constant coefficients integrated exactly, then the shock limiter
//   (Anarchy-PU: beta_c = 0.01 and only the plain cap);
// * the step size: the CFL step c_cfl H_i / v_sig,i, capped at Delta times
//   the smallest CFL step among the force-loop neighbours (r < max(H_i, H_j)),
//   and the smallest limited step over the active particles;
// * the leapfrog operators: a (half) kick of v and u, a drift of x;
// * the GDF flavour's loop (Appendix A): for every active receiver i over j
//   with r_ij < H_i, the geometric-density correction f_i = (S1 / rho_i) /
//   S2 with S1 = sum_j m_j r^2 W_ij and S2 = sum_j (m_j / rho_j) r^2 W_ij,
//   and the conduction parameter alpha_c,i = C |S| h_i^2 from the
//   trace-free symmetric part S of V_ab = sum_j (v_a,i - v_a,j)(x_b,i -
//   x_b,j) m_j W_ij / (S1 / 3), |S| the square root of its summed squares
//   (f = 1 and alpha_c = 0 for a receiver with no neighbour at r > 0).
//
// The neighbour loops run one wave per receiving cell, with the sources in
// LDS in the receiver cell's FP32 frame. They cull each source against the
// receivers' box and sweep a buffer of survivors with several lanes per
// receiver in sparse cells (the shape is described before the gradient
// loop); the gradient and GDF loops evaluate their pairs over per-lane
// lists, the step limiter (a compare and a minimum per pair) directly.
#include "kernel_shapes.h"
#include "pairs.h"

namespace sphx {
namespace {

constexpr int kElemThreads = 256;

// Sorted source state of the gradient loop: (h, rho, P, alpha_V).
__global__ __launch_bounds__(kElemThreads) void k_grad_state(
    int64_t n, const int32_t *__restrict__ perm, const float *__restrict__ h,
    const float *__restrict__ rho, const float *__restrict__ P, const float *__restrict__ av,
    float4 *__restrict__ st)
{
    const int64_t s = int64_t(blockIdx.x) * kElemThreads + threadIdx.x;
    if (s >= n)
        return;
    const int32_t i = perm[s];
    st[s] = make_float4(h[i], rho[i], P[i], av[i]);
}

// Both neighbour loops below take one wave per receiving cell. The sources
// of each task are culled against the receivers' box grown by their largest
// H and the survivors appended to an LDS candidate buffer of kCandCap slots;
// a full buffer is swept by every lane. With n active receivers, each gets
// nrep lanes (the largest power of two with nrep n <= 64) and replica r
// tests the slots r, r + nrep, ...; the slots that pass its receiver's test
// go to the lane's own list (8-bit slot numbers in LDS), and the pair terms
// are evaluated over the lists, four entries a round, whenever one is
// nearly full and at the end of the sweep (an entry past a lane's list adds
// exactly zero). The replicas' results meet in a butterfly. Slot kCandCap
// holds a source beyond every support (cell-frame coordinates are below the
// box size) that replicas past the buffer read.
constexpr int kCandCap = 128;
constexpr float kFarSource = 1e15f;

// The sources of the tasks [ta, te) that lie within R of the receivers' box
// [lo, hb]: the task records are fetched 64 at a time (one per lane), a
// cell beyond R is dropped as a whole, and the sources of four tasks are
// loaded together; emit(p, keep, sj) takes each task's sources in turn (p in
// the receiving cell's frame, keep: this lane holds a source within R, sj
// its sorted index). Every lane runs emit the same number of times.
template <class Emit>
__device__ __forceinline__ void near_sources(const Task *__restrict__ task, int32_t ta,
                                             int32_t te, const float4 *__restrict__ ext,
                                             const float4 *__restrict__ q0, float3 lo,
                                             float3 hb, float R2, int lane, Emit &&emit)
{
    for (int32_t t0 = ta; t0 < te; t0 += 64) {
        const int nb = min(64, te - t0);
        TaskRegs tr;
        tr.load(task, t0 + lane, lane < nb);
        if (lane < nb &&
            task_box_dist2(tr.b.x, tr.b.y, tr.b.z, ext[tr.a.w], lo, hb) >= R2)
            tr.a.y = 0;
        for (int u = 0; u < nb; u += 4) {
            int j0[4], jc[4];
            float4 p[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = min(u + q, nb - 1);
                j0[q] = bcast(tr.a.x, k);
                jc[q] = (u + q < nb) ? bcast(tr.a.y, k) : 0;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                p[q] = lane < jc[q] ? q0[j0[q] + lane] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = min(u + q, nb - 1);
                p[q].x += bcastf(tr.b.x, k);
                p[q].y += bcastf(tr.b.y, k);
                p[q].z += bcastf(tr.b.z, k);
                const bool keep =
                    lane < jc[q] && box_dist2(p[q].x, p[q].y, p[q].z, lo, hb) < R2;
                emit(p[q], keep, j0[q] + lane);
            }
        }
    }
}

template <int K>
__global__ __launch_bounds__(64) void k_gradient(
    int64_t n_leaves, const int32_t *__restrict__ leaf_start, const int32_t *__restrict__ perm,
    const float4 *__restrict__ q0, const float4 *__restrict__ q1,
    const float4 *__restrict__ st, const uint8_t *__restrict__ active,
    const int32_t *__restrict__ tbeg,
    const int32_t *__restrict__ tend, const Task *__restrict__ task,
    const float4 *__restrict__ ext, float gamma_k, float *__restrict__ lap_u,
    float *__restrict__ vc, float *__restrict__ avmax, float anarchy_gamma)
{
    const int64_t L = blockIdx.x;
    if (L >= n_leaves)
        return;
    const int lane = threadIdx.x;
    const int32_t s0 = leaf_start[L], cnt = leaf_start[L + 1] - s0;
    const bool valid = lane < cnt;
    const int32_t s = s0 + (valid ? lane : 0);
    const bool act = valid && (!active || active[perm[s]] != 0);
    const uint64_t amask = __ballot(act);
    if (amask == 0)
        return;
    const float4 pown = q0[s];
    const float Hown = gamma_k * st[s].x;
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

    const int n_act = __popcll(amask);
    int nrep = 1;
    while (2 * nrep * n_act <= 64)
        nrep *= 2;
    __shared__ uint8_t rmap[64];
    // x, y, z (receiver cell frame), m; vx, vy, vz, u; m / rho, P, alpha_V
    // and Anarchy-PU's sound speed c (the other flavours: rho)
    __shared__ float4 cp[kCandCap + 1], cv[kCandCap + 1], cs[kCandCap + 1];
    __shared__ uint32_t lst[kListStride * 16];
    uint8_t *my_list = reinterpret_cast<uint8_t *>(lst) + lane * kListStride;
    if (act)
        rmap[lanes_below(amask)] = uint8_t(lane);
    if (lane == 0) {
        cp[kCandCap] = make_float4(kFarSource, kFarSource, kFarSource, 0.0f);
        cv[kCandCap] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        cs[kCandCap] = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
    }
    __syncthreads();
    const int k = lane / nrep;
    const bool ract = k < n_act;
    const int32_t sr = s0 + (ract ? int(rmap[k]) : 0);
    const int rj = lane & (nrep - 1);
    const float4 pi = q0[sr];  // x, y, z (cell frame), m
    const float4 vi = q1[sr];  // vx, vy, vz, u
    const float4 si = st[sr];  // h, rho, P, alpha_V
    // Anarchy-PU (anarchy_gamma = the gas gamma, else 0): the sound speed
    const float ci = anarchy_gamma > 0.0f ? sqrtf(anarchy_gamma * si.z / si.y) : 0.0f;
    const float Hi = gamma_k * si.x;
    const float H2 = ract ? Hi * Hi : -1.0f;
    const float invH = fast_rcp(Hi);
    const float invH5 = (invH * invH) * (invH * invH) * invH;
    constexpr float kD = Kern<K>::kD;

    float lap = 0.0f, vcm = 0.0f, avm = si.w;
    int nc = 0;    // candidates in the buffer (wave-uniform)
    int myn = 0;   // this lane's list length
    // One listed pair (on = false: past the list, reading slot 0, adds nothing).
    auto pair = [&](int c, bool on) __attribute__((always_inline)) {
        const float4 p = cp[c];
        const float dx = pi.x - p.x, dy = pi.y - p.y, dz = pi.z - p.z;
        const float r2 = dist2(dx, dy, dz);
        const float4 v = cv[c];
        const float4 sj = cs[c];
        const float rinv = on ? fast_rsq(r2) : 0.0f;
        const float r = r2 * rinv;
        const float u = fminf(r * invH, 1.0f);
        // dW/dr / r = -kD H^-5 phi(u)
        const float wr = -kD * invH5 * Kern<K>::phi(u);
        const float dl = sj.x * (vi.w - v.w) * wr;
        const float vdx = (vi.x - v.x) * dx + (vi.y - v.y) * dy + (vi.z - v.z) * dz;
        const float vcij =
            anarchy_gamma > 0.0f
                ? ci + sj.w + fminf(vdx, 0.0f) * rinv
                : fabsf(vdx) * rinv +
                      fast_sqrt(2.0f * fabsf(si.z - sj.y) * fast_rcp(si.y + sj.w));
        lap += on ? dl : 0.0f;
        vcm = on ? fmaxf(vcm, vcij) : vcm;
        avm = on ? fmaxf(avm, sj.z) : avm;
    };
    auto compute = [&]() __attribute__((always_inline)) {
        for (int k4 = 0; __any(k4 < myn); k4 += 4) {
            const uint32_t four = *reinterpret_cast<const uint32_t *>(my_list + k4);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool listed = k4 + q < myn;
                pair(listed ? int((four >> (8 * q)) & 0xffu) : 0, listed);
            }
        }
        myn = 0;
    };
    auto sweep = [&]() __attribute__((always_inline)) {
        __syncthreads();  // (one wave per block) the candidates are written
        const int m_end = (nc + nrep - 1) / nrep;
        for (int m = 0; m < m_end; m += 4) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c0 = rj + (m + q) * nrep;
                const int c = c0 < nc ? c0 : kCandCap;
                const float4 p = cp[c];
                const float r2 = dist2(pi.x - p.x, pi.y - p.y, pi.z - p.z);
                // j != i, 0 < r < H_i (the receiver itself is at r = 0)
                my_list[myn] = uint8_t(c);
                myn += (r2 < H2 && r2 > 0.0f) ? 1 : 0;
            }
            if (__any(myn > kListMax - 4))
                compute();
        }
        compute();
        __syncthreads();  // the sweep has read the buffer
        nc = 0;
    };

    near_sources(task, tbeg[L], tend[L], ext, q0, lo, hb, R2, lane,
                 [&](const float4 &p, bool keep, int32_t j) __attribute__((always_inline)) {
                     const uint64_t mask = __ballot(keep);
                     if (mask == 0)
                         return;
                     const int tot = __popcll(mask);
                     if (nc + tot > kCandCap)
                         sweep();
                     if (keep) {
                         const int pos = nc + lanes_below(mask);
                         const float4 sj = st[j];
                         cp[pos] = p;
                         cv[pos] = q1[j];
                         cs[pos] = make_float4(
                             p.w / sj.y, sj.z, sj.w,
                             anarchy_gamma > 0.0f ? sqrtf(anarchy_gamma * sj.z / sj.y) : sj.y);
                     }
                     nc += tot;
                 });
    if (nc > 0)
        sweep();
    for (int o = 1; o < nrep; o <<= 1) {
        lap += __shfl_xor(lap, o, 64);
        vcm = fmaxf(vcm, __shfl_xor(vcm, o, 64));
        avm = fmaxf(avm, __shfl_xor(avm, o, 64));
    }
    if (ract && rj == 0) {
        const int32_t gi = perm[sr];
        lap_u[gi] = 2.0f * lap;
        vc[gi] = vcm;
        avmax[gi] = avm;
    }
}

// Sorted (h, rho) of every particle for the GDF loop (z, w unused).
__global__ __launch_bounds__(kElemThreads) void k_hrho_state(int64_t n,
                                                             const int32_t *__restrict__ perm,
                                                             const float *__restrict__ h,
                                                             const float *__restrict__ rho,
                                                             float4 *__restrict__ st)
{
    const int64_t s = int64_t(blockIdx.x) * kElemThreads + threadIdx.x;
    if (s >= n)
        return;
    const int32_t i = perm[s];
    st[s] = make_float4(h[i], rho[i], 0.0f, 0.0f);
}

// The GDF loop. W_ij = W(r_ij, h_i) carries the factor kW H_i^-3 in every
// sum, and it cancels in f and in V / (S1 / 3): the sums take w(u) alone.
// st: sorted (h, rho) of every particle. Outputs for the active receivers:
// f and alpha_c in caller order (f_out, ac_out) and, inside a step, in the
// sorted force state (g1.x = f, g1.z = alpha_c, the flavour's slots of f
// and A); null pointers are not written. gate: a captured step whose
// iteration is not finished returns at once. DET: also the shock detector
// D = 3/2 [n.V.n + max(-tr V / 3, 0)] into D_out (caller order), n along the
// kernel sum of m_j u_j dW/dr x_ij / r_ij (the pressure gradient's
// direction: its positive factors and its sign drop out of n.V.n; n.V.n = 0
// without a gradient). (The loop shape is the gradient loop's.)
template <int K, bool DET>
__global__ __launch_bounds__(64) void k_gdf(
    int64_t n_leaves, const int32_t *__restrict__ leaf_start, const int32_t *__restrict__ perm,
    const float4 *__restrict__ q0, const float4 *__restrict__ q1,
    const float4 *__restrict__ st, const uint8_t *__restrict__ active,
    const int32_t *__restrict__ tbeg, const int32_t *__restrict__ tend,
    const Task *__restrict__ task, const float4 *__restrict__ ext, float gamma_k, float C,
    const int32_t *__restrict__ gate, float *__restrict__ f_out, float *__restrict__ ac_out,
    float4 *__restrict__ g1, float *__restrict__ D_out)
{
    if (gate && *gate)
        return;
    const int64_t L = blockIdx.x;
    if (L >= n_leaves)
        return;
    const int lane = threadIdx.x;
    const int32_t s0 = leaf_start[L], cnt = leaf_start[L + 1] - s0;
    const bool valid = lane < cnt;
    const int32_t s = s0 + (valid ? lane : 0);
    const bool act = valid && (!active || active[perm[s]] != 0);
    const uint64_t amask = __ballot(act);
    if (amask == 0)
        return;

    // the receivers' box and largest H (over the active particles)
    const float4 pown = q0[s];
    const float Hown = gamma_k * st[s].x;
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

    // lanes -> (receiver, replica)
    const int n_act = __popcll(amask);
    int nrep = 1;
    while (2 * nrep * n_act <= 64)
        nrep *= 2;
    __shared__ uint8_t rmap[64];
    // x, y, z (receiver cell frame), m; and vx, vy, vz, m / rho. Slot kCandCap
    // is a source beyond every support that replicas past the buffer read.
    __shared__ float4 cp[kCandCap + 1], cv[kCandCap + 1];
    __shared__ float cu[DET ? kCandCap + 1 : 1];  // m_j u_j
    __shared__ uint32_t lst[kListStride * 16];
    uint8_t *my_list = reinterpret_cast<uint8_t *>(lst) + lane * kListStride;
    if (act)
        rmap[lanes_below(amask)] = uint8_t(lane);
    if (lane == 0) {
        // (finite: its zero weight times its distance stays zero)
        cp[kCandCap] = make_float4(kFarSource, kFarSource, kFarSource, 0.0f);
        cv[kCandCap] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if constexpr (DET)
            cu[kCandCap] = 0.0f;
    }
    __syncthreads();
    const int k = lane / nrep;
    const bool ract = k < n_act;
    const int32_t sr = s0 + (ract ? int(rmap[k]) : 0);
    const int rj = lane & (nrep - 1);
    const float4 pi = q0[sr];  // x, y, z (cell frame), m
    const float4 vi = q1[sr];  // vx, vy, vz, u
    const float4 si = st[sr];  // h, rho
    const float Hi = gamma_k * si.x;
    const float H2 = ract ? Hi * Hi : -1.0f;
    const float invH = fast_rcp(Hi);

    float S1 = 0.0f, S2 = 0.0f;
    float V[3][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
    float gp[3] = {0.0f, 0.0f, 0.0f};  // DET: the pressure gradient's direction
    int nc = 0;   // candidates in the buffer (wave-uniform)
    int myn = 0;  // this lane's list length
    // One listed pair (on = false: past the list, reading slot 0, adds
    // exactly zero: its weight is 0 and every term carries it). The
    // receiver itself, at r = 0, adds exactly zero too.
    auto pair = [&](int c, bool on) __attribute__((always_inline)) {
        const float4 p = cp[c];
        const float d[3] = {pi.x - p.x, pi.y - p.y, pi.z - p.z};
        const float r2 = dist2(d[0], d[1], d[2]);
        const float4 v = cv[c];
        const float u = fminf(fast_sqrt(r2) * invH, 1.0f);
        const float wt = on ? Kern<K>::w(u) : 0.0f;
        const float mw = p.w * wt;
        S1 += mw * r2;
        S2 += v.w * wt * r2;
        const float dv[3] = {vi.x - v.x, vi.y - v.y, vi.z - v.z};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                V[a][b] += dv[a] * (d[b] * mw);
        if constexpr (DET) {
            // m_j u_j (-dW/dr) / r up to positive factors (0 at r = 0 and
            // past the list)
            const float rinv = on && r2 > 0.0f ? fast_rsq(r2) : 0.0f;
            const float gw = cu[c] * Kern<K>::mdw(u) * rinv;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                gp[a] += gw * d[a];
        }
    };
    auto compute = [&]() __attribute__((always_inline)) {
        for (int k4 = 0; __any(k4 < myn); k4 += 4) {
            const uint32_t four = *reinterpret_cast<const uint32_t *>(my_list + k4);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool listed = k4 + q < myn;
                pair(listed ? int((four >> (8 * q)) & 0xffu) : 0, listed);
            }
        }
        myn = 0;
    };
    auto sweep = [&]() __attribute__((always_inline)) {
        __syncthreads();  // (one wave per block) the candidates are written
        const int m_end = (nc + nrep - 1) / nrep;
        for (int m = 0; m < m_end; m += 4) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c0 = rj + (m + q) * nrep;
                const int c = c0 < nc ? c0 : kCandCap;
                const float4 p = cp[c];
                const float r2 = dist2(pi.x - p.x, pi.y - p.y, pi.z - p.z);
                // r < H_i
                my_list[myn] = uint8_t(c);
                myn += r2 < H2 ? 1 : 0;
            }
            if (__any(myn > kListMax - 4))
                compute();
        }
        compute();
        __syncthreads();  // the sweep has read the buffer
        nc = 0;
    };

    near_sources(task, tbeg[L], tend[L], ext, q0, lo, hb, R2, lane,
                 [&](const float4 &p, bool keep, int32_t j) __attribute__((always_inline)) {
                     const uint64_t mask = __ballot(keep);
                     if (mask == 0)
                         return;
                     const int tot = __popcll(mask);
                     if (nc + tot > kCandCap)
                         sweep();
                     if (keep) {
                         const int pos = nc + lanes_below(mask);
                         const float4 v = q1[j];
                         cp[pos] = p;
                         cv[pos] = make_float4(v.x, v.y, v.z, p.w / st[j].y);
                         if constexpr (DET)
                             cu[pos] = p.w * v.w;
                     }
                     nc += tot;
                 });
    if (nc > 0)
        sweep();
    // the replicas' partial sums (every replica ends with the totals)
    for (int o = 1; o < nrep; o <<= 1) {
        S1 += __shfl_xor(S1, o, 64);
        S2 += __shfl_xor(S2, o, 64);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                V[a][b] += __shfl_xor(V[a][b], o, 64);
        if constexpr (DET)
            for (int a = 0; a < 3; ++a)
                gp[a] += __shfl_xor(gp[a], o, 64);
    }
    if (!ract || rj != 0)
        return;
    float f = 1.0f, ac = 0.0f;
    if (S1 > 0.0f && S2 > 0.0f) {
        f = (S1 / si.y) / S2;
        const float k3 = 3.0f / S1;
        const float tr = (V[0][0] + V[1][1] + V[2][2]) * (1.0f / 3.0f);
        float ss = 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const float sab = 0.5f * (V[a][b] + V[b][a]) - (a == b ? tr : 0.0f);
                ss += sab * sab;
            }
        ac = C * (k3 * sqrtf(ss)) * (si.x * si.x);
    }
    const int32_t gi = perm[sr];
    if constexpr (DET) {
        float D = 0.0f;
        if (S1 > 0.0f) {
            const float k3 = 3.0f / S1;
            const float gn2 = gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2];
            float nvn = 0.0f;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    nvn += gp[a] * V[a][b] * gp[b];
            nvn = gn2 > 0.0f ? k3 * nvn / gn2 : 0.0f;
            const float comp = -k3 * (V[0][0] + V[1][1] + V[2][2]) * (1.0f / 3.0f);
            D = 1.5f * (nvn + fmaxf(comp, 0.0f));
        }
        D_out[gi] = D;
    }
    if (f_out)
        f_out[gi] = f;
    if (ac_out)
        ac_out[gi] = ac;
    if (g1) {
        g1[sr].x = f;
        g1[sr].z = ac;
    }
}

// The conduction parameter over a step dt (constants printed in Section 3.3:
// beta_c = 1, alpha_c,min = 0, alpha_c,max = 1, alpha_V,max = 2; Anarchy-PU,
// Appendix A: beta_c = 0.01 and no shock limiter, av_max = +inf).
__global__ __launch_bounds__(kElemThreads) void k_alpha_c(
    int64_t n, const float *__restrict__ lap_u, const float *__restrict__ u,
    const float *__restrict__ h, const float *__restrict__ vc, const float *__restrict__ avmax,
    const uint8_t *__restrict__ active, float dt, float gamma_k, float beta_c, float av_max,
    float *__restrict__ alpha)
{
    const int64_t i = int64_t(blockIdx.x) * kElemThreads + threadIdx.x;
    if (i >= n || (active && !active[i]))
        return;
    constexpr float a_min = 0.0f, a_max = 1.0f;
    const float H = gamma_k * h[i];
    const float ui = u[i];
    const float S = ui > 0.0f ? beta_c * H * lap_u[i] / sqrtf(ui) : 0.0f;
    const float lam = vc[i] / H;
    float a = alpha[i];
    if (lam > 0.0f) {
        // a_inf + (a - a_inf) e^(-lam dt), written as a + (a_inf - a)(1 - e^(-lam dt))
        // with expm1: no cancellation between a_inf and a when lam dt is small
        const float a_inf = a_min + S / lam;
        a = a + (a_inf - a) * (-expm1f(-lam * dt));
    } else {
        a = a + S * dt;
    }
    const float cap = fmaxf(a_max * (1.0f - avmax[i] / av_max), a_min);
    alpha[i] = fmaxf(fminf(a, cap), a_min);
}

// Sorted (h, CFL step) of every particle, from the caller's h and v_sig.
__global__ __launch_bounds__(kElemThreads) void k_dt_state(
    int64_t n, const int32_t *__restrict__ perm, const float *__restrict__ h,
    const float *__restrict__ vsig, float gamma_k, float c_cfl, float4 *__restrict__ st)
{
    const int64_t s = int64_t(blockIdx.x) * kElemThreads + threadIdx.x;
    if (s >= n)
        return;
    const int32_t i = perm[s];
    const float hh = h[i];
    st[s] = make_float4(hh, c_cfl * gamma_k * hh / vsig[i], 0.0f, 0.0f);
}

// Limited step of every active receiver: its CFL step, capped at delta times
// the smallest CFL step of the particles j != i with r_ij < max(H_i, H_j);
// the smallest limited step over the block goes to *dt_min (FP32 bits of a
// positive value order as integers).
__global__ __launch_bounds__(64) void k_dt_limit(
    int64_t n_leaves, const int32_t *__restrict__ leaf_start, const int32_t *__restrict__ perm,
    const float4 *__restrict__ q0, const float4 *__restrict__ st,
    const uint8_t *__restrict__ active, const int32_t *__restrict__ tbeg,
    const int32_t *__restrict__ tend,
    const Task *__restrict__ task, const float4 *__restrict__ ext, const float *__restrict__ hmax,
    float gamma_k, float delta, float *__restrict__ dt_out, int32_t *__restrict__ dt_min)
{
    const int64_t L = blockIdx.x;
    if (L >= n_leaves)
        return;
    const int lane = threadIdx.x;
    const int32_t s0 = leaf_start[L], cnt = leaf_start[L + 1] - s0;
    const bool valid = lane < cnt;
    const int32_t s = s0 + (valid ? lane : 0);
    const bool act = valid && (!active || active[perm[s]] != 0);
    const uint64_t amask = __ballot(act);
    if (amask == 0)
        return;
    const float4 pown = q0[s];
    const float Hown = gamma_k * st[s].x;
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

    const int n_act = __popcll(amask);
    int nrep = 1;
    while (2 * nrep * n_act <= 64)
        nrep *= 2;
    __shared__ uint8_t rmap[64];
    // x, y, z (receiver cell frame), H_j^2; and delta dt_j with the sorted
    // index of a source met in the unshifted self task (else -1)
    __shared__ float4 cp[kCandCap + 1];
    __shared__ float cdt[kCandCap + 1];
    __shared__ int32_t cself[kCandCap + 1];
    if (act)
        rmap[lanes_below(amask)] = uint8_t(lane);
    if (lane == 0) {
        cp[kCandCap] = make_float4(kFarSource, kFarSource, kFarSource, 0.0f);
        cdt[kCandCap] = inf;
        cself[kCandCap] = -1;
    }
    __syncthreads();
    const int k = lane / nrep;
    const bool ract = k < n_act;
    const int32_t sr = s0 + (ract ? int(rmap[k]) : 0);
    const int rj = lane & (nrep - 1);
    const float4 pi = q0[sr];
    const float4 si = st[sr];  // h, CFL step
    const float Hi = gamma_k * si.x;
    const float H2 = ract ? Hi * Hi : -1.0f;

    float lim = si.y;
    int nc = 0;  // candidates in the buffer (wave-uniform)
    auto sweep = [&]() __attribute__((always_inline)) {
        __syncthreads();  // (one wave per block) the candidates are written
        const int m_end = (nc + nrep - 1) / nrep;
        for (int m = 0; m < m_end; ++m) {
            const int c0 = rj + m * nrep;
            const int c = c0 < nc ? c0 : kCandCap;
            const float4 p = cp[c];
            const float r2 = dist2(pi.x - p.x, pi.y - p.y, pi.z - p.z);
            // j != i (the receiver itself, in the unshifted self task) with
            // r < max(H_i, H_j)
            const bool on = cself[c] != sr && r2 < fmaxf(H2, ract ? p.w : -1.0f);
            lim = on ? fminf(lim, cdt[c]) : lim;
        }
        __syncthreads();  // the sweep has read the buffer
        nc = 0;
    };

    // As near_sources, with the cull radius of a source cell max(R, its
    // largest H) and of a source max(R, H_j).
    const int32_t ta = tbeg[L], te = tend[L];
    for (int32_t t0 = ta; t0 < te; t0 += 64) {
        const int nb = min(64, te - t0);
        TaskRegs tr;
        tr.load(task, t0 + lane, lane < nb);
        if (lane < nb) {
            const float hj = hmax[tr.a.w];
            if (task_box_dist2(tr.b.x, tr.b.y, tr.b.z, ext[tr.a.w], lo, hb) >= fmaxf(R2, hj * hj))
                tr.a.y = 0;
        }
        for (int u = 0; u < nb; u += 4) {
            int j0[4], jc[4], self[4];
            float4 p[4];
            float2 sj[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int kk = min(u + q, nb - 1);
                j0[q] = bcast(tr.a.x, kk);
                jc[q] = (u + q < nb) ? bcast(tr.a.y, kk) : 0;
                self[q] = bcast(tr.a.z, kk);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool in = lane < jc[q];
                p[q] = in ? q0[j0[q] + lane] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                const float4 e = in ? st[j0[q] + lane] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                sj[q] = make_float2(e.x, e.y);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int kk = min(u + q, nb - 1);
                p[q].x += bcastf(tr.b.x, kk);
                p[q].y += bcastf(tr.b.y, kk);
                p[q].z += bcastf(tr.b.z, kk);
                const float Hj = gamma_k * sj[q].x;
                const bool keep = lane < jc[q] &&
                                  box_dist2(p[q].x, p[q].y, p[q].z, lo, hb) < fmaxf(R2, Hj * Hj);
                const uint64_t mask = __ballot(keep);
                if (mask == 0)
                    continue;
                const int tot = __popcll(mask);
                if (nc + tot > kCandCap)
                    sweep();
                if (keep) {
                    const int pos = nc + lanes_below(mask);
                    cp[pos] = make_float4(p[q].x, p[q].y, p[q].z, Hj * Hj);
                    cdt[pos] = delta * sj[q].y;
                    cself[pos] = self[q] ? j0[q] + lane : -1;
                }
                nc += tot;
            }
        }
    }
    if (nc > 0)
        sweep();
    for (int o = 1; o < nrep; o <<= 1)
        lim = fminf(lim, __shfl_xor(lim, o, 64));
    if (ract && rj == 0)
        dt_out[perm[sr]] = lim;
    float mn = ract ? lim : inf;
    mn = wave_minf(mn);
    if (lane == 0 && mn < inf)
        atomicMin(dt_min, __float_as_int(mn));
}

__global__ void k_fill_inf(int32_t *p)
{
    if (threadIdx.x == 0)
        *p = __float_as_int(__builtin_inff());
}

// One wave per leaf: the largest gamma_k h of the leaf's particles (from a
// sorted (h, ...) state), for the limiter's source-cell cull.
__global__ __launch_bounds__(64) void k_leaf_hmax_st(int64_t n_leaves,
                                                     const int32_t *__restrict__ leaf_start,
                                                     const float4 *__restrict__ st, float gamma_k,
                                                     float *__restrict__ hmax)
{
    const int64_t L = blockIdx.x;
    if (L >= n_leaves)
        return;
    const int lane = threadIdx.x;
    const int32_t s0 = leaf_start[L], cnt = leaf_start[L + 1] - s0;
    float v = lane < cnt ? st[s0 + lane].x : 0.0f;
    v = wave_maxf(v);
    if (lane == 0)
        hmax[L] = gamma_k * v;
}

// Half kick (or prediction): out = in + d * dt_half for v (3) and u.
__global__ __launch_bounds__(kElemThreads) void k_kick(
    int64_t n, const float *__restrict__ vx, const float *__restrict__ vy,
    const float *__restrict__ vz, const float *__restrict__ u, const float *__restrict__ ax,
    const float *__restrict__ ay, const float *__restrict__ az, const float *__restrict__ du,
    const uint8_t *__restrict__ active, float dt_half, float *vx_o, float *vy_o, float *vz_o,
    float *u_o)
{
    const int64_t i = int64_t(blockIdx.x) * kElemThreads + threadIdx.x;
    if (i >= n || (active && !active[i]))
        return;
    vx_o[i] = vx[i] + ax[i] * dt_half;
    vy_o[i] = vy[i] + ay[i] * dt_half;
    vz_o[i] = vz[i] + az[i] * dt_half;
    u_o[i] = u[i] + du[i] * dt_half;
}

// Drift in FP64: x += v dt, wrapped into [0, L) in a periodic box.
__global__ __launch_bounds__(kElemThreads) void k_drift(
    int64_t n, double *__restrict__ x, double *__restrict__ y, double *__restrict__ z,
    const float *__restrict__ vx, const float *__restrict__ vy, const float *__restrict__ vz,
    double dt, double Lx, double Ly, double Lz, int periodic)
{
    // each operation rounded on its own (no fused multiply-add), so that the
    // positions follow the plain FP64 arithmetic of a drift exactly
#pragma clang fp contract(off)
    const int64_t i = int64_t(blockIdx.x) * kElemThreads + threadIdx.x;
    if (i >= n)
        return;
    double p[3] = {x[i] + double(vx[i]) * dt, y[i] + double(vy[i]) * dt,
                   z[i] + double(vz[i]) * dt};
    const double B[3] = {Lx, Ly, Lz};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (periodic) {
            p[a] -= B[a] * floor(p[a] / B[a]);
            if (p[a] >= B[a])  // a tiny negative coordinate rounds up to L
                p[a] -= B[a];
        }
    x[i] = p[0];
    y[i] = p[1];
    z[i] = p[2];
}

inline unsigned elem_blocks(int64_t n) { return unsigned((n + kElemThreads - 1) / kElemThreads); }

}  // namespace

sphx_status gradient_launch(const sphx_ctx *ctx, sphx_grid *g, const sphx_tasks *t,
                            const sphx_particles *in, const float *rho, const float *P,
                            float *lap_u, float *vc, float *avmax, hipStream_t s)
{
    if (g->n == 0 || g->n_leaves == 0)
        return SPHX_OK;
    k_grad_state<<<elem_blocks(g->n), kElemThreads, 0, s>>>(g->n, g->perm, in->h, rho, P,
                                                           in->alpha_v, g->g2);
    SPHX_HIP(hipGetLastError());
    SPHX_WITH_KERNEL(ctx->p.kernel,
                     (k_gradient<KK><<<unsigned(g->n_leaves), 64, 0, s>>>(
                         g->n_leaves, g->leaf_start, g->perm, g->q0, g->q1, g->g2, in->active,
                         t->slot, t->end, t->task, g->leaf_ext, float(ctx->p.gamma_k), lap_u, vc,
                         avmax,
                         ctx->p.flavour == SPHX_FLAVOUR_ANARCHY_PU ? float(ctx->p.gamma_gas)
                                                                   : 0.0f)));
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

sphx_status gdf_launch(const sphx_ctx *ctx, sphx_grid *g, const sphx_tasks *t,
                       const sphx_particles *in, const float *rho, float *f, float *alpha_c,
                       float *D, hipStream_t s)
{
    if (g->n == 0 || g->n_leaves == 0)
        return SPHX_OK;
    k_hrho_state<<<elem_blocks(g->n), kElemThreads, 0, s>>>(g->n, g->perm, in->h, rho, g->g2);
    SPHX_HIP(hipGetLastError());
    if (D) {
        SPHX_WITH_KERNEL(ctx->p.kernel,
                         (k_gdf<KK, true><<<unsigned(g->n_leaves), 64, 0, s>>>(
                             g->n_leaves, g->leaf_start, g->perm, g->q0, g->q1, g->g2, in->active,
                             t->slot, t->end, t->task, g->leaf_ext, float(ctx->p.gamma_k),
                             float(kGdfC), nullptr, f, alpha_c, nullptr, D)));
    } else {
        SPHX_WITH_KERNEL(ctx->p.kernel,
                         (k_gdf<KK, false><<<unsigned(g->n_leaves), 64, 0, s>>>(
                             g->n_leaves, g->leaf_start, g->perm, g->q0, g->q1, g->g2, in->active,
                             t->slot, t->end, t->task, g->leaf_ext, float(ctx->p.gamma_k),
                             float(kGdfC), nullptr, f, alpha_c, nullptr, nullptr)));
    }
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

sphx_status gdf_step_launch(const sphx_ctx *ctx, const sphx_grid *g, const sphx_tasks *t,
                            const sphx_particles *in, const int32_t *gate, hipStream_t s)
{
    if (g->n == 0 || g->n_leaves == 0)
        return SPHX_OK;
    // (h, rho) of the force state g0 = (h, rho, P, c); f and alpha_c into g1
    SPHX_WITH_KERNEL(ctx->p.kernel,
                     (k_gdf<KK, false><<<unsigned(g->n_leaves), 64, 0, s>>>(
                         g->n_leaves, g->leaf_start, g->perm, g->q0, g->q1, g->g0, in->active,
                         t->slot, t->end, t->task, g->leaf_ext, float(ctx->p.gamma_k),
                         float(kGdfC), gate, nullptr, nullptr, g->g1, nullptr)));
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

sphx_status alpha_c_launch(const sphx_ctx *ctx, int64_t n, const float *lap_u, const float *u,
                           const float *h, const float *vc, const float *avmax,
                           const uint8_t *active, double dt, float *alpha, hipStream_t s)
{
    if (n == 0)
        return SPHX_OK;
    const bool anarchy = ctx->p.flavour == SPHX_FLAVOUR_ANARCHY_PU;
    k_alpha_c<<<elem_blocks(n), kElemThreads, 0, s>>>(
        n, lap_u, u, h, vc, avmax, active, float(dt), float(ctx->p.gamma_k),
        anarchy ? 0.01f : 1.0f, anarchy ? __builtin_inff() : 2.0f, alpha);
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

sphx_status timestep_launch(const sphx_ctx *ctx, sphx_grid *g, const sphx_tasks *t,
                            const sphx_particles *in, const float *vsig, double c_cfl,
                            double delta, float *dt_out, float *dt_min, hipStream_t s)
{
    int32_t *mn = reinterpret_cast<int32_t *>(dt_min);
    if (mn) {
        k_fill_inf<<<1, 64, 0, s>>>(mn);
        SPHX_HIP(hipGetLastError());
    }
    if (g->n == 0 || g->n_leaves == 0)
        return SPHX_OK;
    const float gk = float(ctx->p.gamma_k);
    k_dt_state<<<elem_blocks(g->n), kElemThreads, 0, s>>>(g->n, g->perm, in->h, vsig, gk,
                                                          float(c_cfl), g->g2);
    SPHX_HIP(hipGetLastError());
    k_leaf_hmax_st<<<unsigned(g->n_leaves), 64, 0, s>>>(g->n_leaves, g->leaf_start, g->g2, gk,
                                                        g->leaf_hmax);
    SPHX_HIP(hipGetLastError());
    k_dt_limit<<<unsigned(g->n_leaves), 64, 0, s>>>(
        g->n_leaves, g->leaf_start, g->perm, g->q0, g->g2, in->active, t->slot, t->end, t->task,
        g->leaf_ext, g->leaf_hmax, gk, float(delta), dt_out, mn);
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

sphx_status kick_launch(int64_t n, const float *vx, const float *vy, const float *vz,
                        const float *u, const float *ax, const float *ay, const float *az,
                        const float *du, const uint8_t *active, double dt_half, float *vx_o,
                        float *vy_o, float *vz_o, float *u_o, hipStream_t s)
{
    if (n == 0)
        return SPHX_OK;
    k_kick<<<elem_blocks(n), kElemThreads, 0, s>>>(n, vx, vy, vz, u, ax, ay, az, du, active,
                                                   float(dt_half), vx_o, vy_o, vz_o, u_o);
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

sphx_status drift_launch(const sphx_ctx *ctx, int64_t n, double *x, double *y, double *z,
                         const float *vx, const float *vy, const float *vz, double dt,
                         hipStream_t s)
{
    if (n == 0)
        return SPHX_OK;
    k_drift<<<elem_blocks(n), kElemThreads, 0, s>>>(n, x, y, z, vx, vy, vz, dt, ctx->p.box[0],
                                                    ctx->p.box[1], ctx->p.box[2],
                                                    ctx->p.periodic);
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

}  // namespace sphx
