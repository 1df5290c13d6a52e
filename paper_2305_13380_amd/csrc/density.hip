// Density pass (Section 3.1): number density, mass density, their
// h-derivatives, neighbour count, and the velocity divergence and curl sums.
//
// One wave64 per receiving leaf (one particle per lane). Each task's source
// leaf is staged in LDS with the task's FP32 origin offset already applied,
// so every lane works on small cell-relative FP32 coordinates; LDS reads of
// the source particle are wave-uniform (broadcast). Each receiver sums its
// sources in a fixed order (task order, then source order), so results do not
// depend on scheduling.
#include "sphx_internal.h"

namespace sphx {
namespace {

__global__ __launch_bounds__(64) void k_density(
    int64_t n_leaves, int64_t nb_padded, const int32_t *__restrict__ leaf_start,
    const int32_t *__restrict__ perm, const float4 *__restrict__ q0,
    const float4 *__restrict__ q1, const uint8_t *__restrict__ need, const float *__restrict__ h,
    const float *__restrict__ radius, const int32_t *__restrict__ toff,
    const Task *__restrict__ task, float gamma_k, float *__restrict__ o_rho,
    float *__restrict__ o_rho_dh, float *__restrict__ o_n, float *__restrict__ o_n_dh,
    float *__restrict__ o_div, float *__restrict__ o_cx, float *__restrict__ o_cy,
    float *__restrict__ o_cz, int32_t *__restrict__ o_nngb, int32_t *__restrict__ counters)
{
    const int64_t L = xcd_remap(blockIdx.x, nb_padded);
    if (L >= n_leaves)
        return;
    const int lane = threadIdx.x;
    const int32_t s0 = leaf_start[L];
    const int32_t cnt = leaf_start[L + 1] - s0;
    const bool valid = lane < cnt;
    const int32_t s = s0 + (valid ? lane : 0);
    const bool act = valid && need[s];
    if (!__any(act))
        return;

    __shared__ float4 jp[kLeafMax];
    __shared__ float4 jv[kLeafMax];

    const float4 pi = q0[s];
    const float4 vi = q1[s];
    const int32_t gi = perm[s];
    const float hi = act ? h[gi] : 1.0f;
    const float H = gamma_k * hi;
    const float H2 = H * H;
    const float invH = 1.0f / H;
    if (act && H > radius[L] && counters)
        atomicAdd(counters + 3, 1);

    float Sw = 0.f, Smw = 0.f, Sud = 0.f, Smud = 0.f;
    float Sdiv = 0.f, Scx = 0.f, Scy = 0.f, Scz = 0.f;
    int32_t nn = 0;

    const int32_t t0 = toff[L], t1 = toff[L + 1];
    for (int32_t t = t0; t < t1; ++t) {
        const Task T = task[t];
        const int32_t j0 = leaf_start[T.j];
        const int32_t jc = leaf_start[T.j + 1] - j0;
        __syncthreads();
        if (lane < jc) {
            float4 p = q0[j0 + lane];
            jp[lane] = make_float4(p.x + T.ox, p.y + T.oy, p.z + T.oz, p.w);
            jv[lane] = q1[j0 + lane];
        }
        __syncthreads();
        for (int k = 0; k < jc; ++k) {
            const float4 p = jp[k];
            const float dx = pi.x - p.x, dy = pi.y - p.y, dz = pi.z - p.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (act && r2 < H2) {
                const float r = sqrtf(r2);
                const float u = r * invH;
                const float t1u = 1.0f - u;
                const float t2 = t1u * t1u;
                const float t3 = t2 * t1u;
                const float w = t2 * t2 * (1.0f + 4.0f * u);
                const float ud = u * u * t3;
                Sw += w;
                Smw += p.w * w;
                Sud += ud;
                Smud += p.w * ud;
                if (j0 + k != s) {
                    ++nn;
                    const float4 v = jv[k];
                    const float dvx = v.x - vi.x, dvy = v.y - vi.y, dvz = v.z - vi.z;
                    const float mt3 = p.w * t3;
                    Sdiv += mt3 * (dvx * dx + dvy * dy + dvz * dz);
                    Scx += mt3 * (dy * dvz - dz * dvy);
                    Scy += mt3 * (dz * dvx - dx * dvz);
                    Scz += mt3 * (dx * dvy - dy * dvx);
                }
            }
        }
    }
    if (!act)
        return;
    // W = kW H^-3 (1-u)^4 (1+4u); dW/dh = -(H^-3/h)(3 kW w - kD u^2 (1-u)^3);
    // grad_i W = dW/dr x_ij / r with dW/dr / r = -kD H^-5 (1-u)^3.
    const float invH3 = invH * invH * invH;
    const float invH5 = invH3 * invH * invH;
    const float ih = 1.0f / hi;
    o_n[gi] = kW * invH3 * Sw;
    o_rho[gi] = kW * invH3 * Smw;
    o_n_dh[gi] = -invH3 * ih * (3.0f * kW * Sw - kD * Sud);
    o_rho_dh[gi] = -invH3 * ih * (3.0f * kW * Smw - kD * Smud);
    o_div[gi] = -kD * invH5 * Sdiv;
    o_cx[gi] = -kD * invH5 * Scx;
    o_cy[gi] = -kD * invH5 * Scy;
    o_cz[gi] = -kD * invH5 * Scz;
    o_nngb[gi] = nn;
}

}  // namespace

sphx_status density_launch(const sphx_ctx *ctx, const sphx_grid *g, const sphx_tasks *t,
                           const sphx_particles *in, const sphx_density_out *o,
                           int32_t *counters, hipStream_t s)
{
    if (g->n_leaves == 0)
        return SPHX_OK;
    const int64_t nbp = pad8(g->n_leaves);
    SPHX_HIP(ctx->prof->begin(0, s));
    k_density<<<unsigned(nbp), 64, 0, s>>>(
        g->n_leaves, nbp, g->leaf_start, g->perm, g->q0, g->q1, g->need, in->h, t->radius, t->off,
        t->task, float(ctx->p.gamma_k), o->rho, o->rho_dh, o->n, o->n_dh, o->div_sum, o->curl_x,
        o->curl_y, o->curl_z, o->nngb, counters);
    SPHX_HIP(hipGetLastError());
    SPHX_HIP(ctx->prof->end(0, s));
    return SPHX_OK;
}

}  // namespace sphx
