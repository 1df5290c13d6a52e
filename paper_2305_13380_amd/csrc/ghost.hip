// Ghost (Section 3.1 Newton-Raphson on the partition condition, equation of
// state; Section 3.2 f-factor and Balsara switch). One thread per particle
// needing a pass; everything in FP32.
#include "sphx_internal.h"

namespace sphx {
namespace {

__global__ void k_ghost(int64_t n, const int32_t *__restrict__ perm,
                        const int32_t *__restrict__ leaf_of, uint8_t *__restrict__ need,
                        float *__restrict__ h, const float4 *__restrict__ q1,
                        const float *__restrict__ radius, const float *__restrict__ d_rho,
                        const float *__restrict__ d_rho_dh, const float *__restrict__ d_n,
                        const float *__restrict__ d_n_dh, const float *__restrict__ d_div,
                        const float *__restrict__ d_cx, const float *__restrict__ d_cy,
                        const float *__restrict__ d_cz, float eta3, float h_tol, float h_max,
                        float gamma_k, float gamma_gas, float eps_b, int final_pass,
                        float *__restrict__ o_f, float *__restrict__ o_P, float *__restrict__ o_c,
                        float *__restrict__ o_B, float *__restrict__ o_A,
                        float *__restrict__ o_div, float *__restrict__ o_curl,
                        uint8_t *__restrict__ o_conv, int32_t *__restrict__ counters)
{
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n || !need[s])
        return;
    // A density pass that ran with a stale task list is not used.
    if (counters && counters[3] > 0)
        return;
    const int32_t i = perm[s];
    const float hh = h[i];
    const float nd = d_n[i], ndh = d_n_dh[i];
    const float h2 = hh * hh, h3 = h2 * hh;
    const float F = nd * h3 - eta3;
    const float dF = h3 * ndh + 3.0f * h2 * nd;
    float hn;
    const float step = F / dF;
    if (dF > 0.0f && isfinite(step))
        hn = hh - step;
    else
        hn = F < 0.0f ? 2.0f * hh : 0.5f * hh;
    hn = fminf(fmaxf(hn, 0.5f * hh), 2.0f * hh);
    hn = fminf(hn, h_max);
    const bool conv = fabsf(hn - hh) < h_tol * hh;

    if (!conv && !final_pass) {
        h[i] = hn;
        o_conv[i] = 0;
        if (counters) {
            atomicAdd(counters + 0, 1);
            if (gamma_k * hn > radius[leaf_of[s]])
                atomicAdd(counters + 1, 1);
        }
        return;
    }
    // Converged, or out of passes: finalise at the h the sums belong to.
    need[s] = 0;
    o_conv[i] = conv ? 1 : 0;
    if (counters) {
        if (!conv)
            atomicAdd(counters + 0, 1);
        if (hh >= h_max)
            atomicAdd(counters + 2, 1);
    }
    const float rho = d_rho[i];
    const float u = q1[s].w;
    const float P = (gamma_gas - 1.0f) * u * rho;
    const float c = sqrtf(gamma_gas * (gamma_gas - 1.0f) * u);
    const float f = 1.0f / (1.0f + hh * d_rho_dh[i] / (3.0f * rho));
    const float irho = 1.0f / rho;
    const float div = d_div[i] * irho;
    const float cx = d_cx[i], cy = d_cy[i], cz = d_cz[i];
    const float curl = sqrtf(cx * cx + cy * cy + cz * cz) * irho;
    const float ad = fabsf(div);
    o_f[i] = f;
    o_P[i] = P;
    o_c[i] = c;
    o_B[i] = ad / (ad + curl + eps_b * c / hh);
    o_A[i] = f * P * irho * irho;
    o_div[i] = div;
    o_curl[i] = curl;
}

}  // namespace

sphx_status ghost_launch(const sphx_ctx *ctx, sphx_grid *g, const sphx_tasks *t,
                         sphx_particles *in, const sphx_density_out *d, const sphx_ghost_out *o,
                         int32_t *counters, int final_pass, hipStream_t s)
{
    if (g->n == 0)
        return SPHX_OK;
    const sphx_params &P = ctx->p;
    const float eta3 = float(P.eta * P.eta * P.eta);
    k_ghost<<<unsigned((g->n + 255) / 256), 256, 0, s>>>(
        g->n, g->perm, g->leaf_of, g->need, in->h, g->q1, t->radius, d->rho, d->rho_dh, d->n,
        d->n_dh, d->div_sum, d->curl_x, d->curl_y, d->curl_z, eta3, float(P.h_tol),
        float(ctx->h_max), float(P.gamma_k), float(P.gamma_gas), float(P.eps_balsara),
        final_pass, o->f, o->P, o->c, o->balsara, o->A, o->div_v, o->curl_v, o->converged,
        counters);
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

}  // namespace sphx
