// Ghost (Section 3.1 Newton-Raphson on the partition condition, equation of
// state; Section 3.2 f-factor and Balsara switch; Appendix A smoothed
// pressure and grad-h term of the pressure-energy flavour). Particles needing
// a pass, in sorted order (the density kernel leaves its sums in sorted order
// too), over a grid-stride loop; everything in FP32. The iteration's counters are
// reduced per block and added with one atomic per block and counter (atomics
// from every wave on the same few words serialise in L2).
#include <algorithm>

#include "sphx_internal.h"

namespace sphx {
namespace {

constexpr int kGhostThreads = 256;
constexpr int kGhostMaxBlocks = 1024;

__global__ __launch_bounds__(kGhostThreads) void k_ghost(int64_t n, const int32_t *__restrict__ perm,
                        const int32_t *__restrict__ leaf_of, uint8_t *__restrict__ need,
                        float *__restrict__ h, float *__restrict__ hs,
                        float *__restrict__ hlo, float *__restrict__ hhi,
                        const float4 *__restrict__ q1, const float *__restrict__ radius,
                        const float *__restrict__ lrad,
                        const float4 *__restrict__ d0, const float4 *__restrict__ d1, float inv_eta3,
                        float h_tol, float h_max, float gamma_k, float gamma_gas, float eps_b,
                        int final_pass, int step_mode, int flavour,
                        const float2 *__restrict__ d2, float4 *__restrict__ g0,
                        float4 *__restrict__ g1, float4 *__restrict__ g2, const int32_t *__restrict__ nngb,
                        unsigned long long *__restrict__ units, float *__restrict__ o_f,
                        float *__restrict__ o_P,
                        float *__restrict__ o_c, float *__restrict__ o_B,
                        float *__restrict__ o_A, float *__restrict__ o_div,
                        float *__restrict__ o_curl, uint8_t *__restrict__ o_conv,
                        int32_t *__restrict__ counters, const int32_t *__restrict__ skip)
{
    if (skip && *skip)
        return;  // a captured pass with nothing left to do
    // A density pass that ran with a stale task list is not used.
    const bool stale = counters && counters[3] > 0;
    int n_unconv = 0, n_rebuild = 0, n_clamped = 0, n_beyond = 0;
    unsigned long long pairs_cell = 0, pairs_list = 0;  // interactions of this pass, by loop
    const int64_t stride = int64_t(gridDim.x) * kGhostThreads;
    for (int64_t s = int64_t(blockIdx.x) * kGhostThreads + threadIdx.x; s < n; s += stride) {
        if (stale || !need[s])
            continue;
        const float hh = hs[s];
        const float4 a = d0[s];  // n, G' = 3 + h n'/n, rho, 1 + h rho'/(3 rho)
        const float nd = a.x;
        // Newton-Raphson in ln h on G = ln(n h^3 / eta^3), G' = 3 + h n'/n,
        // with the step limited to a factor 2; in base-2 logarithms:
        // log2(h_new / h) = -log2(n h^3 / eta^3) / G'.
        const float G2 = __log2f(nd * (hh * hh * hh) * inv_eta3);
        const float dG = a.y;
        // bracket of the root: the largest h with G < 0, the smallest with G > 0
        float lo = hlo[s], hi = hhi[s];
        if (G2 < 0.0f && hh > lo)
            hlo[s] = lo = hh;
        if (G2 > 0.0f && hh < hi)
            hhi[s] = hi = hh;
        float e = -G2 / dG;
        if (!(dG > 0.0f) || !isfinite(e))
            e = G2 < 0.0f ? 1.0f : -1.0f;
        e = fminf(fmaxf(e, -1.0f), 1.0f);
        float hn = hh * exp2f(e);
        hn = fminf(hn, h_max);
        // a Newton step that would not converge and leaves a known bracket is
        // replaced by its geometric midpoint (a bisection in ln h): no cycling
        // where G is nearly flat (a converging step may round onto an end)
        if (!(fabsf(hn - hh) < h_tol * hh) && lo > 0.0f && hi < __builtin_inff() &&
            !(hn > lo && hn < hi))
            hn = sqrtf(lo * hi);
        const bool conv = fabsf(hn - hh) < h_tol * hh;
        const int32_t i = perm[s];
        n_unconv += conv ? 0 : 1;
        if (units) {
            const int c = nngb[i];
            if (lrad && gamma_k * hh <= lrad[s])
                pairs_list += c;
            else
                pairs_cell += c;
        }
        if (!conv && !final_pass) {
            hs[s] = hn;
            // Inside a step the caller's h and flag are written once, when the
            // particle is finalised (no scattered writes in every pass).
            if (!step_mode) {
                h[i] = hn;
                o_conv[i] = 0;
            }
            n_rebuild += gamma_k * hn > radius[leaf_of[s]] ? 1 : 0;
            // with neighbour lists: the next pass cannot use this one's list
            n_beyond += (lrad && gamma_k * hn > lrad[s]) ? 1 : 0;
        } else {
            // Converged, or out of passes: finalise at the h the sums belong to.
            need[s] = 0;
            n_clamped += hh >= h_max ? 1 : 0;
            const float4 b = d1[s];  // div_sum, curl_x, curl_y, curl_z
            const float rho = a.z;
            const float u = q1[s].w;
            // density-energy: u is the internal energy; density-entropy: the
            // particle carries the adiabat A, and P = A rho^gamma;
            // pressure-energy: the smoothed pressure (gamma - 1) sum m u W
            const bool entropy = flavour == SPHX_FLAVOUR_DENSITY_ENTROPY;
            const bool pe = smoothed_pressure(flavour);
            const float2 sp = pe ? d2[s] : make_float2(0.0f, 0.0f);  // sum m u W, F G'
            const float P = pe ? (gamma_gas - 1.0f) * sp.x
                               : (entropy ? u * powf(rho, gamma_gas)
                                          : (gamma_gas - 1.0f) * u * rho);
            const float c = (entropy || pe) ? sqrtf(gamma_gas * P / rho)
                                            : sqrtf(gamma_gas * (gamma_gas - 1.0f) * u);
            const float f = 1.0f / a.w;
            const float irho = 1.0f / rho;
            const float div = b.x * irho;
            const float curl = sqrtf(b.y * b.y + b.z * b.z + b.w * b.w) * irho;
            const float ad = fabsf(div);
            const float B = ad / (ad + curl + eps_b * c / hh);
            // pressure-energy: A is the grad-h term F of f_ij = 1 - F_i / (m_j
            // u_j), and the force state's fourth slot (gamma - 1)^2 u / P_hat
            const float A = pe ? sp.y / a.y : f * P * irho * irho;
            const float Q = pe ? (gamma_gas - 1.0f) * (gamma_gas - 1.0f) * u / P : 0.0f;
            if (step_mode) {
                // Sorted state only: the force pass's source state (the same
                // values its gather would read from the outputs) and the
                // rest; the force kernel, which every finalised particle of a
                // step receives in, writes the caller's h and outputs.
                g0[s] = make_float4(hh, rho, P, c);
                g1[s] = make_float4(f, B, A, Q);
                g2[s] = make_float4(div, curl, conv ? 1.0f : 0.0f, 0.0f);
            } else {
                o_conv[i] = conv ? 1 : 0;
                o_f[i] = f;
                o_P[i] = P;
                o_c[i] = c;
                o_B[i] = B;
                o_A[i] = A;
                o_div[i] = div;
                o_curl[i] = curl;
            }
        }
    }
    if (!counters && !units)
        return;
    // block reduction: waves by shuffles, then across the block's waves in LDS
    unsigned long long v[6] = {(unsigned long long)n_unconv, (unsigned long long)n_rebuild,
                               (unsigned long long)n_clamped, (unsigned long long)n_beyond,
                               pairs_cell, pairs_list};
#pragma unroll
    for (int k = 0; k < 6; ++k)
        for (int o = 32; o > 0; o >>= 1)
            v[k] += __shfl_xor(v[k], o, 64);
    __shared__ unsigned long long red[kGhostThreads / 64][6];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < 6; ++k)
            red[wv][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        unsigned long long t = 0;
        for (int w2 = 0; w2 < kGhostThreads / 64; ++w2)
            t += red[w2][k];
        if (t) {
            if (k < 4) {
                if (counters)
                    atomicAdd(counters + (k == 3 ? 4 : k), int(t));
            } else if (units) {
                atomicAdd(units + (k - 4), t);
            }
        }
    }
}

}  // namespace

sphx_status ghost_launch(const sphx_ctx *ctx, sphx_grid *g, const sphx_tasks *t,
                         sphx_particles *in, const sphx_density_out *d, const sphx_ghost_out *o,
                         int32_t *counters, int final_pass, bool use_lists,
                         unsigned long long *units, hipStream_t s, const int32_t *skip,
                         bool step_mode)
{
    if (g->n == 0)
        return SPHX_OK;
    const sphx_params &P = ctx->p;
    const float inv_eta3 = float(1.0 / (P.eta * P.eta * P.eta));
    const int64_t nblk = std::min<int64_t>((g->n + kGhostThreads - 1) / kGhostThreads,
                                           kGhostMaxBlocks);
    k_ghost<<<unsigned(nblk), kGhostThreads, 0, s>>>(
        g->n, g->perm, g->leaf_of, g->need, in->h, g->hs, g->hlo, g->hhi, g->q1, t->radius,
        use_lists ? g->lrad : nullptr, g->d0, g->d1, inv_eta3,
        float(P.h_tol),
        float(ctx->h_max), float(P.gamma_k), float(P.gamma_gas), float(P.eps_balsara),
        final_pass, step_mode ? 1 : 0, P.flavour, g->d2, g->g0,
        g->g1, g->g2, d->nngb, units, o->f, o->P, o->c,
        o->balsara, o->A, o->div_v, o->curl_v, o->converged, counters, skip);
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

}  // namespace sphx
