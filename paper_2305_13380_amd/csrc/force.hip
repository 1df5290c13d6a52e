// Force pass (Section 3.2 density-energy equations of motion with the
// Balsara-switched artificial viscosity; Section 3.3 symmetric alpha_ij and
// artificial conduction) and the FP64 global momentum / energy sums.
//
// One wave64 per receiving leaf; each task's source leaf is staged in LDS in
// the receiver leaf's frame together with the per-source quantities every
// pair term needs, so the inner loop reads wave-uniform LDS addresses.
#include "sphx_internal.h"

namespace sphx {
namespace {

// Sorted copies of the ghost state every source needs: (h, rho, P, c) and
// (f, B, A, 0).
__global__ void k_force_state(int64_t n, const int32_t *__restrict__ perm,
                              const float *__restrict__ h, const float *__restrict__ rho,
                              const float *__restrict__ P, const float *__restrict__ c,
                              const float *__restrict__ f, const float *__restrict__ B,
                              const float *__restrict__ A, float4 *__restrict__ g0,
                              float4 *__restrict__ g1)
{
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    const int32_t i = perm[s];
    g0[s] = make_float4(h[i], rho[i], P[i], c[i]);
    g1[s] = make_float4(f[i], B[i], A[i], 0.0f);
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(64) void k_force(
    int64_t n_leaves, int64_t nb_padded, const int32_t *__restrict__ leaf_start,
    const int32_t *__restrict__ perm, const float4 *__restrict__ q0,
    const float4 *__restrict__ q1, const float2 *__restrict__ qa, const float4 *__restrict__ g0,
    const float4 *__restrict__ g1, const uint8_t *__restrict__ active,
    const int32_t *__restrict__ toff, const Task *__restrict__ task, float gamma_k, float beta,
    float *__restrict__ o_ax, float *__restrict__ o_ay, float *__restrict__ o_az,
    float *__restrict__ o_du, float *__restrict__ o_vsig, int32_t *__restrict__ o_nf,
    double *__restrict__ fsum)
{
    const int64_t L = xcd_remap(blockIdx.x, nb_padded);
    if (L >= n_leaves)
        return;
    const int lane = threadIdx.x;
    const int32_t s0 = leaf_start[L];
    const int32_t cnt = leaf_start[L + 1] - s0;
    const bool valid = lane < cnt;
    const int32_t s = s0 + (valid ? lane : 0);
    const int32_t gi = perm[s];
    const bool act = valid && (active ? active[gi] != 0 : true);
    if (!__any(act)) {
        if (lane < 6)
            fsum[6 * L + lane] = 0.0;
        return;
    }

    __shared__ float4 sp[kLeafMax];  // x, y, z (receiver frame), m
    __shared__ float4 sv[kLeafMax];  // vx, vy, vz, H^2
    __shared__ float4 sa[kLeafMax];  // 1/H, c, rho, P
    __shared__ float4 sb[kLeafMax];  // f, A, B, alpha_v
    __shared__ float2 sc[kLeafMax];  // alpha_c P, u

    const float4 pi = q0[s];
    const float4 vi = q1[s];  // w = u
    const float2 ai = qa[s];
    const float4 gi0 = g0[s];  // h, rho, P, c
    const float4 gi1 = g1[s];  // f, B, A
    const float Hi = gamma_k * gi0.x;
    const float Hi2 = Hi * Hi;
    const float invHi = 1.0f / Hi;
    const float invHi4 = (invHi * invHi) * (invHi * invHi);
    const float rhoi = gi0.y, Pi = gi0.z, ci = gi0.w;
    const float fi = gi1.x, Bi = gi1.y, Ai = gi1.z;
    const float acPi = ai.y * Pi;

    float ax = 0.f, ay = 0.f, az = 0.f, du = 0.f;
    float vsig = 2.0f * ci;
    int32_t nf = 0;

    const int32_t t0 = toff[L], t1 = toff[L + 1];
    for (int32_t t = t0; t < t1; ++t) {
        const Task T = task[t];
        const int32_t j0 = leaf_start[T.j];
        const int32_t jc = leaf_start[T.j + 1] - j0;
        __syncthreads();
        if (lane < jc) {
            const int32_t sj = j0 + lane;
            const float4 p = q0[sj];
            const float4 v = q1[sj];
            const float2 a = qa[sj];
            const float4 h0 = g0[sj];
            const float4 h1 = g1[sj];
            const float Hj = gamma_k * h0.x;
            sp[lane] = make_float4(p.x + T.ox, p.y + T.oy, p.z + T.oz, p.w);
            sv[lane] = make_float4(v.x, v.y, v.z, Hj * Hj);
            sa[lane] = make_float4(1.0f / Hj, h0.w, h0.y, h0.z);
            sb[lane] = make_float4(h1.x, h1.z, h1.y, a.x);
            sc[lane] = make_float2(a.y * h0.z, v.w);
        }
        __syncthreads();
        for (int k = 0; k < jc; ++k) {
            const float4 p = sp[k];
            const float dx = pi.x - p.x, dy = pi.y - p.y, dz = pi.z - p.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            const float4 v = sv[k];
            if (act && r2 < fmaxf(Hi2, v.w) && j0 + k != s) {
                ++nf;
                if (r2 > 0.0f) {
                    const float rinv = rsqrtf(r2);
                    const float r = r2 * rinv;
                    const float4 a = sa[k];
                    const float4 b = sb[k];
                    const float2 c2 = sc[k];
                    const float ui = r * invHi;
                    const float ti = fmaxf(1.0f - ui, 0.0f);
                    const float gi = -kD * invHi4 * ui * (ti * ti * ti);
                    const float uj = r * a.x;
                    const float tj = fmaxf(1.0f - uj, 0.0f);
                    const float ij2 = a.x * a.x;
                    const float gj = -kD * (ij2 * ij2) * uj * (tj * tj * tj);
                    const float ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
                    const float dvx = vi.x - v.x, dvy = vi.y - v.y, dvz = vi.z - v.z;
                    const float vdote = dvx * ex + dvy * ey + dvz * ez;
                    const float mu = vdote < 0.0f ? vdote : 0.0f;
                    const float vs = ci + a.y - beta * mu;
                    vsig = fmaxf(vsig, vs);
                    const float alpha = 0.25f * (ai.x + b.w) * (Bi + b.z);
                    const float irs = 1.0f / (rhoi + a.z);
                    const float nu = -2.0f * alpha * mu * vs * irs;
                    const float G = fi * gi + b.x * gj;
                    const float acc = Ai * gi + b.y * gj + 0.5f * nu * G;
                    const float m = p.w;
                    ax -= m * acc * ex;
                    ay -= m * acc * ey;
                    az -= m * acc * ez;
                    du += m * (Ai * gi + 0.25f * nu * G) * vdote;
                    const float psum = Pi + a.w;
                    const float ac = psum > 0.0f ? (acPi + c2.x) / psum : 0.0f;
                    const float vc = fabsf(vdote) + sqrtf(2.0f * fabsf(Pi - a.w) * irs);
                    du += m * ac * vc * (vi.w - c2.y) * G * irs;
                }
            }
        }
    }
    double m0 = 0, m1 = 0, m2 = 0, e = 0, sa_ = 0, sd = 0;
    if (act) {
        o_ax[gi] = ax;
        o_ay[gi] = ay;
        o_az[gi] = az;
        o_du[gi] = du;
        o_vsig[gi] = vsig;
        if (o_nf)
            o_nf[gi] = nf;
        const double mi = pi.w;
        const double dax = ax, day = ay, daz = az, ddu = du;
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

// Fixed-order FP64 reduction of the per-leaf partial sums (one block).
__global__ __launch_bounds__(256) void k_sum_leaves(int64_t n_leaves,
                                                    const double *__restrict__ fsum,
                                                    double *__restrict__ out)
{
    __shared__ double red[6][256];
    const int t = threadIdx.x;
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t L = t; L < n_leaves; L += 256)
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
        out[t] = red[t][0];
}

}  // namespace

sphx_status force_launch(const sphx_ctx *ctx, const sphx_grid *g, const sphx_tasks *t,
                         const sphx_particles *in, const sphx_density_out *d,
                         const sphx_ghost_out *gs, const sphx_force_out *o, double *sums6,
                         hipStream_t s)
{
    if (g->n_leaves == 0) {
        if (sums6)
            SPHX_HIP(hipMemsetAsync(sums6, 0, 6 * sizeof(double), s));
        return SPHX_OK;
    }
    k_force_state<<<unsigned((g->n + 255) / 256), 256, 0, s>>>(g->n, g->perm, in->h, d->rho,
                                                                gs->P, gs->c, gs->f, gs->balsara,
                                                                gs->A, g->g0, g->g1);
    SPHX_HIP(hipGetLastError());
    const int64_t nbp = pad8(g->n_leaves);
    SPHX_HIP(ctx->prof->begin(1, s));
    k_force<<<unsigned(nbp), 64, 0, s>>>(
        g->n_leaves, nbp, g->leaf_start, g->perm, g->q0, g->q1, g->qa, g->g0, g->g1, in->active,
        t->off, t->task, float(ctx->p.gamma_k), float(ctx->p.beta_v), o->ax, o->ay, o->az,
        o->du_dt, o->v_sig, o->nforce, g->fsum);
    SPHX_HIP(hipGetLastError());
    SPHX_HIP(ctx->prof->end(1, s));
    if (sums6) {
        k_sum_leaves<<<1, 256, 0, s>>>(g->n_leaves, g->fsum, sums6);
        SPHX_HIP(hipGetLastError());
    }
    return SPHX_OK;
}

}  // namespace sphx
