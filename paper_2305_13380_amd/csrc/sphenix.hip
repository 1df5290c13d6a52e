// SPHENIX viscosity switch (Section 3.3), one particle per thread: the
// change of the velocity divergence over the step gives the shock indicator
// S = H^2 max(0, -d(div v)/dt), H = gamma_k h, and the target
// alpha_loc = alpha_max S / (v_sig^2 + S); alpha rises to the target at once
// and otherwise decays towards it as exp(-ell c dt / H). Streams seven FP32
// words per particle (six read, one written): bound by HBM bandwidth.
#include "sphx_internal.h"

namespace sphx {
namespace {

constexpr int kSwitchThreads = 256;

__global__ __launch_bounds__(kSwitchThreads) void k_alpha_v(
    int64_t n, const float *__restrict__ div_old, const float *__restrict__ div_new,
    const float *__restrict__ c, const float *__restrict__ h, const float *__restrict__ vsig,
    float dt, float gamma_k, float alpha_max, float ell, float *__restrict__ alpha)
{
    const int64_t i = int64_t(blockIdx.x) * kSwitchThreads + threadIdx.x;
    if (i >= n)
        return;
    const float H = gamma_k * h[i];
    const float ddiv = (div_new[i] - div_old[i]) / dt;
    const float S = H * H * fmaxf(-ddiv, 0.0f);
    const float vs = vsig[i];
    const float loc = S > 0.0f ? alpha_max * S / (vs * vs + S) : 0.0f;
    const float a = alpha[i];
    alpha[i] = loc > a ? loc : loc + (a - loc) * expf(-ell * c[i] * dt / H);
}

// The GDF flavour's viscosity parameter (Appendix A): dD/dt = (D_new -
// D_old) / dt, A = 2 h^2 B max(-dD/dt, 0), alpha_loc = alpha_max A / (A +
// v_sig^2); alpha rises to it at once, as the SPHENIX switch does, or else
// relaxes towards it as exp(-0.2 c dt / h) (the exact solution over the
// step). Nine FP32 words per particle.
__global__ __launch_bounds__(kSwitchThreads) void k_gdf_alpha_v(
    int64_t n, const float *__restrict__ D_old, const float *__restrict__ D_new,
    const float *__restrict__ c, const float *__restrict__ h, const float *__restrict__ vsig,
    const float *__restrict__ B, const uint8_t *__restrict__ active, float dt, float alpha_max,
    float *__restrict__ alpha)
{
    const int64_t i = int64_t(blockIdx.x) * kSwitchThreads + threadIdx.x;
    if (i >= n || (active && !active[i]))
        return;
    const float hi = h[i];
    const float dD = (D_new[i] - D_old[i]) / dt;
    const float A = 2.0f * hi * hi * B[i] * fmaxf(-dD, 0.0f);
    const float vs = vsig[i];
    const float loc = A > 0.0f ? alpha_max * A / (A + vs * vs) : 0.0f;
    const float a = alpha[i];
    alpha[i] = loc > a ? loc : loc + (a - loc) * expf(-0.2f * c[i] * dt / hi);
}

}  // namespace

sphx_status gdf_alpha_v_launch(int64_t n, const float *D_old, const float *D_new,
                               const float *c, const float *h, const float *vsig,
                               const float *B, const uint8_t *active, double dt, float *alpha,
                               hipStream_t s)
{
    if (n == 0)
        return SPHX_OK;
    const unsigned nb = unsigned((n + kSwitchThreads - 1) / kSwitchThreads);
    // alpha_V,max: SPHENIX's (Section 3.3), which Appendix A does not restate
    k_gdf_alpha_v<<<nb, kSwitchThreads, 0, s>>>(n, D_old, D_new, c, h, vsig, B, active,
                                                float(dt), 2.0f, alpha);
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

sphx_status alpha_v_launch(const sphx_ctx *ctx, int64_t n, const float *div_old,
                           const float *div_new, const float *c, const float *h,
                           const float *vsig, double dt, float *alpha, hipStream_t s)
{
    if (n == 0)
        return SPHX_OK;
    const unsigned nb = unsigned((n + kSwitchThreads - 1) / kSwitchThreads);
    // decay length: 0.05 (SPHENIX, Section 3.3), 0.25 (the Phantom-like and
    // Anarchy-PU flavours, Appendix A)
    const float ell = (ctx->p.flavour == SPHX_FLAVOUR_PHANTOM ||
                       ctx->p.flavour == SPHX_FLAVOUR_ANARCHY_PU)
                          ? 0.25f
                          : 0.05f;
    k_alpha_v<<<nb, kSwitchThreads, 0, s>>>(n, div_old, div_new, c, h, vsig, float(dt),
                                            float(ctx->p.gamma_k), 2.0f, ell, alpha);
    SPHX_HIP(hipGetLastError());
    return SPHX_OK;
}

}  // namespace sphx
