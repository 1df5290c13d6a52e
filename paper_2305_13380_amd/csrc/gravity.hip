// Short-range softened gravity by direct summation over the self and pair
// tasks of a cell structure built with the summation radius r_p2p as search
// radius (Section 4.1: the C2 softened potential and force; Section 4.4: the
// short-range truncation of the mesh split). For a pair at separation r:
//   phi(r)    = f(r/H) / H inside the softening support H, 1/r beyond,
//               f(u) = -3u^7 + 15u^6 - 28u^5 + 21u^4 - 7u^2 + 3;
//   phi'(r)/r = g(r/H) / H^3 inside, -1/r^3 beyond,
//               g(u) = f'(u)/u = -21u^5 + 90u^4 - 140u^3 + 84u^2 - 14;
//   chi(r)    = erfc(r / (2 r_s)), chi'(r) = -exp(-r^2/(4 r_s^2)) / (sqrt(pi) r_s)
//               (erfc by the rational approximation the paper names);
//   a_i      += G m_j x_ij [phi' chi + phi chi'] / r,  pot_i -= G m_j phi chi,
// over j != i with r_ij < r_p2p. One wave per receiving leaf, one receiver
// per lane; each task's sources are staged in LDS in the receiver cell's
// FP32 frame and the lanes run through them together: a source no lane sums
// is skipped, the others are evaluated by every lane without branches (the
// softened and Newtonian branches are both evaluated and one is selected).
#include "pairs.h"
#include "sphx_internal.h"

namespace sphx {
namespace {

template <bool TRUNC>
__global__ __launch_bounds__(64) void k_gravity(int64_t n_leaves,
                                               const int32_t *__restrict__ leaf_start,
                                               const int32_t *__restrict__ perm,
                                               const float4 *__restrict__ q0,
                                               const int32_t *__restrict__ tbeg,
    const int32_t *__restrict__ tend,
                                               const Task *__restrict__ task,
                                               const float4 *__restrict__ ext, float H, float rp2,
                                               float inv2rs, float cdchi, float G,
                                               float *__restrict__ ax, float *__restrict__ ay,
                                               float *__restrict__ az, float *__restrict__ pot,
                                               unsigned long long *__restrict__ pairs)
{
    const int64_t L = blockIdx.x;
    if (L >= n_leaves)
        return;
    const int lane = threadIdx.x;
    const int32_t s0 = leaf_start[L], cnt = leaf_start[L + 1] - s0;
    const bool valid = lane < cnt;
    const int32_t s = s0 + (valid ? lane : 0);
    const float4 pi = q0[s];  // x, y, z in the cell frame, m
    const float invH = __builtin_amdgcn_rcpf(H);
    const float invH3 = invH * invH * invH;
    __shared__ float4 src[kLeafMax];
    float sx = 0.f, sy = 0.f, sz = 0.f, sp = 0.f;
    unsigned np_ = 0;
    // the box of the receivers (source leaves wholly beyond r_p2p of it are
    // skipped; a pair the box test drops lies at r_p2p to rounding)
    const float inf = __builtin_inff();
    float3 lo = make_float3(valid ? pi.x : inf, valid ? pi.y : inf, valid ? pi.z : inf);
    float3 hb = make_float3(valid ? pi.x : -inf, valid ? pi.y : -inf, valid ? pi.z : -inf);
    lo.x = wave_minf(lo.x);
    lo.y = wave_minf(lo.y);
    lo.z = wave_minf(lo.z);
    hb.x = wave_maxf(hb.x);
    hb.y = wave_maxf(hb.y);
    hb.z = wave_maxf(hb.z);
    const int32_t ta = tbeg[L], tb = tend[L];
    for (int32_t t = ta; t < tb; ++t) {
        const Task tk = task[t];
        if (task_box_dist2(tk.ox, tk.oy, tk.oz, ext[tk.j], lo, hb) >= rp2)
            continue;
        __syncthreads();
        if (lane < tk.jc) {
            float4 p = q0[tk.j0 + lane];
            p.x += tk.ox;
            p.y += tk.oy;
            p.z += tk.oz;
            src[lane] = p;
        }
        __syncthreads();
        // the receiver's own particle: in the unshifted self task, at its slot
        const int own = (tk.self && valid) ? s - tk.j0 : -1;
        for (int k = 0; k < tk.jc; ++k) {
            const float4 p = src[k];
            const float dx = pi.x - p.x, dy = pi.y - p.y, dz = pi.z - p.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            const bool on = valid && k != own && r2 < rp2;
            if (!__any(on))
                continue;  // no lane sums this source
            const float rinv = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
            const float r = r2 * rinv;
            const float u = r * invH;
            const bool in = u < 1.0f;
            const float u2 = u * u;
            const float f = 3.0f + u2 * (-7.0f + u2 * (21.0f + u * (-28.0f + u * (15.0f - 3.0f * u))));
            const float g = -14.0f + u2 * (84.0f + u * (-140.0f + u * (90.0f - 21.0f * u)));
            const float phi = in ? f * invH : rinv;
            const float dphir = in ? g * invH3 : -(rinv * rinv * rinv);
            float chi = 1.0f, k_r = dphir;
            if (TRUNC) {
                // erfc(x), x = r / (2 r_s), by the rational approximation
                // 7.1.26 of Abramowitz & Stegun (absolute error below
                // 1.5e-7), the one the paper's solver uses: a polynomial in
                // t = 1 / (1 + p x) times exp(-x^2), the factor chi' needs too
                const float x = r * inv2rs;
                const float e = expf(-(x * x));
                const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
                const float poly =
                    t * (0.254829592f +
                         t * (-0.284496736f +
                              t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
                chi = poly * e;
                const float dchir = -cdchi * e * rinv;
                k_r = dphir * chi + phi * dchir;
            }
            const float mk = on ? p.w * k_r : 0.0f;
            sx += mk * dx;
            sy += mk * dy;
            sz += mk * dz;
            sp += on ? p.w * (phi * chi) : 0.0f;
            np_ += on ? 1u : 0u;
        }
    }
    if (pairs) {
        unsigned long long t = np_;
        for (int o = 32; o > 0; o >>= 1)
            t += __shfl_xor(t, o, 64);
        if (lane == 0 && t)
            atomicAdd(pairs, t);
    }
    if (valid) {
        const int32_t i = perm[s];
        ax[i] = G * sx;
        ay[i] = G * sy;
        az[i] = G * sz;
        if (pot)
            pot[i] = -G * sp;
    }
}

__global__ void k_zero_pairs(int64_t *p)
{
    if (threadIdx.x == 0)
        *p = 0;
}

}  // namespace

sphx_status gravity_run(sphx_ctx *ctx, const sphx_particles *in, double G, double H, double rs,
                        double rp2p, float *ax, float *ay, float *az, float *pot,
                        int64_t *d_pairs, hipStream_t s)
{
    if (d_pairs) {
        k_zero_pairs<<<1, 64, 0, s>>>(d_pairs);
        SPHX_HIP(hipGetLastError());
    }
    if (in->n == 0)
        return SPHX_OK;
    SearchCells sc;
    SPHX_TRY(search_cells_build(ctx, in, rp2p, s, sc));
    const sphx_grid *g = sc.g;
    const sphx_tasks *t = sc.t;
    const float rp2 = float(rp2p * rp2p);
    const float inv2rs = rs > 0.0 ? float(0.5 / rs) : 0.0f;
    const float cdchi = rs > 0.0 ? float(1.0 / (sqrt(3.14159265358979323846) * rs)) : 0.0f;
    SPHX_HIP(ctx->prof->begin(4, s));
    if (rs > 0.0)
        k_gravity<true><<<unsigned(g->n_leaves), 64, 0, s>>>(
            g->n_leaves, g->leaf_start, g->perm, g->q0, t->slot, t->end, t->task, g->leaf_ext,
            float(H), rp2, inv2rs, cdchi, float(G), ax, ay, az, pot,
            reinterpret_cast<unsigned long long *>(d_pairs));
    else
        k_gravity<false><<<unsigned(g->n_leaves), 64, 0, s>>>(
            g->n_leaves, g->leaf_start, g->perm, g->q0, t->slot, t->end, t->task, g->leaf_ext,
            float(H), rp2, inv2rs, cdchi, float(G), ax, ay, az, pot,
            reinterpret_cast<unsigned long long *>(d_pairs));
    SPHX_HIP(hipGetLastError());
    SPHX_HIP(ctx->prof->end(4, s));
    return SPHX_OK;
}

}  // namespace sphx
