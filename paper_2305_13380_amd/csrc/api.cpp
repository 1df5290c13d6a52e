// C-ABI entry points of the sphx library: argument validation, ownership of
// the opaque handles, and the host side of the h iteration.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <string>

#include "kernel_shapes.h"
#include "sphx_internal.h"

uint64_t next_serial()
{
    static std::atomic<uint64_t> counter{0};
    return ++counter;
}

namespace sphx {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

hipError_t Profiler::begin(int k, hipStream_t s)
{
    if (!on)
        return hipSuccess;
    if (used[k] == pool[k].size()) {
        Rec r;
        hipError_t e = hipEventCreate(&r.a);
        if (e != hipSuccess)
            return e;
        e = hipEventCreate(&r.b);
        if (e != hipSuccess)
            return e;
        pool[k].push_back(r);
    }
    return hipEventRecord(pool[k][used[k]].a, s);
}

hipError_t Profiler::end(int k, hipStream_t s)
{
    if (!on)
        return hipSuccess;
    hipError_t e = hipEventRecord(pool[k][used[k]].b, s);
    ++used[k];
    return e;
}

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

static sphx_status check_particles(const sphx_particles *in, bool need_h_write)
{
    if (!in) {
        set_error("particles: NULL");
        return SPHX_E_INVALID;
    }
    if (in->n < 0 || in->n > int64_t(INT32_MAX) - 1) {
        set_error("particles: n must be in [0, 2^31 - 2]");
        return SPHX_E_INVALID;
    }
    if (in->n == 0)
        return SPHX_OK;
    const void *req[] = {in->x, in->y, in->z, in->vx, in->vy, in->vz, in->m, in->u, in->h,
                         in->alpha_v, in->alpha_c};
    for (const void *p : req)
        if (!p) {
            set_error("particles: a required array pointer is NULL");
            return SPHX_E_INVALID;
        }
    (void)need_h_write;
    return SPHX_OK;
}

static sphx_status check_handles(const sphx_ctx *ctx, const sphx_grid *g, const sphx_tasks *t,
                                 const sphx_particles *in)
{
    if (!ctx || !g) {
        set_error("NULL context or grid");
        return SPHX_E_INVALID;
    }
    if (g->ctx != ctx) {
        set_error("grid belongs to another context");
        return SPHX_E_STATE;
    }
    if (t && t->grid != g) {
        set_error("task list belongs to another grid");
        return SPHX_E_STATE;
    }
    if (in && in->n != g->n) {
        set_error("particle count differs from the grid's");
        return SPHX_E_INVALID;
    }
    return SPHX_OK;
}

hipError_t wait_stream(sphx_ctx *ctx, hipStream_t s)
{
    hipError_t e = hipEventRecord(ctx->ev_wait, s);
    if (e != hipSuccess)
        return e;
    while ((e = hipEventQuery(ctx->ev_wait)) == hipErrorNotReady) {
    }
    (void)hipGetLastError();  // the runtime keeps "not ready" as the last error
    return e;
}

}  // namespace sphx

using namespace sphx;

extern "C" {

void sphx_params_default(sphx_params *p)
{
    if (!p)
        return;
    memset(p, 0, sizeof(*p));
    p->box[0] = p->box[1] = p->box[2] = 1.0;
    p->periodic = 1;
    p->max_iter = 30;
    p->gamma_k = sqrt(15.0) / 2.0;
    p->eta = 1.2348;
    p->h_tol = 1e-4;
    p->h_max = 0.0;
    p->gamma_gas = 5.0 / 3.0;
    p->beta_v = 3.0;
    p->eps_balsara = 1e-4;
    p->skin = 0.1;
    p->neighbour_lists = 0;
    p->leaf_max = 64;
    p->density_tile = 0;
    p->density_waves = 0;
    p->force_tile = 0;
    p->force_waves = 0;
    p->graph_passes = 0;
    p->density_balance = 0;
    p->kernel = SPHX_KERNEL_WENDLAND_C2;
    p->flavour = SPHX_FLAVOUR_DENSITY_ENERGY;
    p->recycle_workspace = 0;
}

sphx_status sphx_params_set_kernel(sphx_params *p, int32_t kernel)
{
    // (H/h)^2 for h = twice the kernel's standard deviation: the per-axis
    // variance of each normalised kernel with support 1 is 1/(4 (H/h)^2)
    static const double gamma2[6] = {15.0 / 4.0, 39.0 / 8.0, 6.0,
                                     10.0 / 3.0, 375.0 / 92.0, 135.0 / 28.0};
    if (!p || kernel < 0 || kernel >= sphx::kKernelKinds) {
        set_error("sphx_params_set_kernel: unknown kernel");
        return SPHX_E_INVALID;
    }
    p->kernel = kernel;
    p->gamma_k = sqrt(gamma2[kernel]);
    return SPHX_OK;
}

const char *sphx_last_error(void) { return g_last_error.c_str(); }

sphx_status sphx_ctx_create(const sphx_params *p, int hip_device, sphx_ctx **out)
{
    if (!p || !out) {
        set_error("sphx_ctx_create: NULL argument");
        return SPHX_E_INVALID;
    }
    *out = nullptr;
    for (int a = 0; a < 3; ++a)
        if (!(p->box[a] > 0.0) || !isfinite(p->box[a])) {
            set_error("sphx_ctx_create: box lengths must be positive and finite");
            return SPHX_E_INVALID;
        }
    if (!(p->eta > 0.0) || !(p->h_tol > 0.0) || p->max_iter < 1 || !(p->gamma_k > 0.0) ||
        p->leaf_max < 8 || p->leaf_max > kLeafMax || !(p->skin >= 0.0) || !(p->gamma_gas > 1.0)) {
        set_error("sphx_ctx_create: invalid eta, h_tol, max_iter, gamma_k, gamma_gas, skin or "
                  "leaf_max (8..64)");
        return SPHX_E_INVALID;
    }
    auto one_of = [](int32_t v, int32_t a, int32_t b, int32_t c) {
        return v == 0 || v == a || v == b || v == c;
    };
    if (!one_of(p->density_tile, 64, 128, 256) || !one_of(p->density_waves, 1, 2, 1) ||
        !one_of(p->force_tile, 64, 128, 64) || !one_of(p->force_waves, 1, 2, 1)) {
        set_error("sphx_ctx_create: loop shapes must be 0 or density_tile 64/128/256, "
                  "density_waves 1/2, force_tile 64/128, force_waves 1/2");
        return SPHX_E_INVALID;
    }
    if (p->kernel < 0 || p->kernel >= sphx::kKernelKinds) {
        set_error("sphx_ctx_create: unknown kernel (SPHX_KERNEL_*)");
        return SPHX_E_INVALID;
    }
    if (p->flavour != SPHX_FLAVOUR_DENSITY_ENERGY && p->flavour != SPHX_FLAVOUR_DENSITY_ENTROPY &&
        p->flavour != SPHX_FLAVOUR_PHANTOM && p->flavour != SPHX_FLAVOUR_PRESSURE_ENERGY &&
        p->flavour != SPHX_FLAVOUR_ANARCHY_PU && p->flavour != SPHX_FLAVOUR_GDF) {
        set_error("sphx_ctx_create: unknown flavour (SPHX_FLAVOUR_*)");
        return SPHX_E_INVALID;
    }
    if (sphx::smoothed_pressure(p->flavour) &&
        (p->density_balance != 0 || p->neighbour_lists != 0)) {
        set_error("sphx_ctx_create: the pressure-energy and Anarchy-PU flavours run the plain "
                  "cell-pair density loop only (density_balance 0, neighbour_lists 0)");
        return SPHX_E_INVALID;
    }
    if (p->graph_passes < 0 || p->graph_passes > 64 || p->density_balance < 0 ||
        p->density_balance > 2) {
        set_error("sphx_ctx_create: graph_passes must be 0..64 and density_balance 0, 1 or 2");
        return SPHX_E_INVALID;
    }
    int ndev = 0;
    SPHX_HIP(hipGetDeviceCount(&ndev));
    if (hip_device < 0 || hip_device >= ndev) {
        set_error("sphx_ctx_create: no such HIP device");
        return SPHX_E_INVALID;
    }
    SPHX_HIP(hipSetDevice(hip_device));
    // Grids, task lists and their scratch come stream-ordered from the
    // device's default pool and go back to it when a request is done; by
    // default the pool hands freed memory back to the device at every
    // synchronisation, and the next build maps it again. Keep it cached.
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, hip_device) == hipSuccess && pool) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
    sphx_ctx *c = new sphx_ctx();
    c->prof = new Profiler();
    c->p = *p;
    c->device = hip_device;
    double lmin = fmin(p->box[0], fmin(p->box[1], p->box[2]));
    double auto_max = lmin / (3.0 * p->gamma_k) * (1.0 - 1e-6);
    c->h_max = p->h_max > 0.0 ? fmin(p->h_max, auto_max) : auto_max;
    if (hipMalloc(&c->d_counters, kStepCounterBytes) != hipSuccess ||
        hipMalloc(&c->d_sums, 8 * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void **)&c->h_pinned, kPinnedBytes, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_wait, hipEventDisableTiming) != hipSuccess) {
        (void)hipFree(c->d_counters);
        (void)hipFree(c->d_sums);
        if (c->h_pinned)
            (void)hipHostFree(c->h_pinned);
        (void)hipGetLastError();
        delete c->prof;
        delete c;
        set_error("sphx_ctx_create: out of device memory");
        return SPHX_E_OOM;
    }
    // The fixed workspace of sphx_force_noalloc on this device: its address
    // is looked up here, at set-up, once per device.
    const sphx_status ws = noalloc_scratch(hip_device, &c->noalloc_sums);
    if (ws < 0) {
        const std::string msg = sphx_last_error();
        sphx_ctx_destroy(c);
        set_error("sphx_ctx_create: " + msg);
        return ws;
    }
    *out = c;
    return SPHX_OK;
}

void sphx_ctx_destroy(sphx_ctx *ctx)
{
    if (!ctx)
        return;
    step_graph_free(ctx->graph);
    release_spares(ctx);
    (void)hipFree(ctx->d_counters);
    (void)hipFree(ctx->d_sums);
    (void)hipHostFree(ctx->h_pinned);
    (void)hipEventDestroy(ctx->ev_wait);
    for (auto &v : ctx->prof->pool)
        for (auto &r : v) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
    delete ctx->prof;
    delete ctx;
}

size_t sphx_workspace_bytes(const sphx_params *p, int64_t n)
{
    if (n < 0)
        return 0;
    const int leaf_max = (p && p->leaf_max > 0) ? p->leaf_max : 64;
    return grid_bytes(n) + tasks_bytes(n, leaf_max) +
           ((p && p->neighbour_lists == 0) ? 0 : lists_bytes(n));
}

sphx_status sphx_grid_build(sphx_ctx *ctx, const sphx_particles *in, void *stream,
                            sphx_grid **out)
{
    if (!ctx || !out) {
        set_error("sphx_grid_build: NULL argument");
        return SPHX_E_INVALID;
    }
    SPHX_TRY(check_particles(in, false));
    SPHX_HIP(hipSetDevice(ctx->device));
    return grid_build(ctx, in, as_stream(stream), out);
}

sphx_status sphx_grid_build_sets(sphx_ctx *ctx, const sphx_particles *in,
                                 const int64_t *set_start, int32_t n_sets, void *stream,
                                 sphx_grid **out)
{
    if (!ctx || !out || !set_start) {
        set_error("sphx_grid_build_sets: NULL argument");
        return SPHX_E_INVALID;
    }
    SPHX_TRY(check_particles(in, false));
    if (n_sets < 1 || n_sets > kMaxSets) {
        set_error("sphx_grid_build_sets: n_sets must be 1.." + std::to_string(kMaxSets));
        return SPHX_E_INVALID;
    }
    if (set_start[0] != 0 || set_start[n_sets] != in->n) {
        set_error("sphx_grid_build_sets: set_start must run from 0 to n");
        return SPHX_E_INVALID;
    }
    for (int32_t b = 0; b < n_sets; ++b)
        if (set_start[b + 1] < set_start[b]) {
            set_error("sphx_grid_build_sets: set_start must not decrease");
            return SPHX_E_INVALID;
        }
    SPHX_HIP(hipSetDevice(ctx->device));
    return grid_build(ctx, in, as_stream(stream), out, set_start, n_sets);
}

void sphx_grid_destroy(sphx_grid *grid) { grid_free(grid); }

sphx_status sphx_tasks_build(sphx_ctx *ctx, sphx_grid *grid, const sphx_particles *in,
                             void *stream, sphx_tasks **out)
{
    if (!out) {
        set_error("sphx_tasks_build: NULL argument");
        return SPHX_E_INVALID;
    }
    SPHX_TRY(check_handles(ctx, grid, *out, in));
    SPHX_TRY(check_particles(in, false));
    SPHX_HIP(hipSetDevice(ctx->device));
    SPHX_TRY(refresh_h(grid, in, as_stream(stream)));
    return tasks_build(ctx, grid, in, as_stream(stream), out);
}

void sphx_tasks_destroy(sphx_tasks *tasks) { tasks_free(tasks); }

sphx_status sphx_alpha_v_update(sphx_ctx *ctx, int64_t n, const float *div_old,
                                const float *div_new, const float *c, const float *h,
                                const float *v_sig, double dt, float *alpha_v, void *stream)
{
    if (!ctx || n < 0 || !(dt > 0.0) || !std::isfinite(dt)) {
        set_error("sphx_alpha_v_update: need a context, n >= 0 and a finite dt > 0");
        return SPHX_E_INVALID;
    }
    if (n > 0 && (!div_old || !div_new || !c || !h || !v_sig || !alpha_v)) {
        set_error("sphx_alpha_v_update: NULL array");
        return SPHX_E_INVALID;
    }
    SPHX_HIP(hipSetDevice(ctx->device));
    return alpha_v_launch(ctx, n, div_old, div_new, c, h, v_sig, dt, alpha_v, as_stream(stream));
}

sphx_status sphx_gradient(sphx_ctx *ctx, sphx_grid *grid, const sphx_tasks *tasks,
                          const sphx_particles *in, const float *rho, const float *P,
                          float *lap_u, float *v_c, float *alpha_v_max, void *stream)
{
    SPHX_TRY(check_handles(ctx, grid, tasks, in));
    SPHX_TRY(check_particles(in, false));
    if (!tasks || (in->n && (!rho || !P || !lap_u || !v_c || !alpha_v_max))) {
        set_error("sphx_gradient: NULL task list, state or output array");
        return SPHX_E_INVALID;
    }
    SPHX_HIP(hipSetDevice(ctx->device));
    return gradient_launch(ctx, grid, tasks, in, rho, P, lap_u, v_c, alpha_v_max,
                           as_stream(stream));
}

sphx_status sphx_gdf(sphx_ctx *ctx, sphx_grid *grid, const sphx_tasks *tasks,
                     const sphx_particles *in, const float *rho, float *f, float *alpha_c,
                     float *D, void *stream)
{
    SPHX_TRY(check_handles(ctx, grid, tasks, in));
    SPHX_TRY(check_particles(in, false));
    if (!tasks || (in->n && (!rho || !f || !alpha_c))) {
        set_error("sphx_gdf: NULL task list, rho or output array");
        return SPHX_E_INVALID;
    }
    SPHX_HIP(hipSetDevice(ctx->device));
    return gdf_launch(ctx, grid, tasks, in, rho, f, alpha_c, D, as_stream(stream));
}

sphx_status sphx_gdf_alpha_v_update(sphx_ctx *ctx, int64_t n, const float *D_old,
                                    const float *D_new, const float *c, const float *h,
                                    const float *v_sig, const float *balsara,
                                    const uint8_t *active, double dt, float *alpha_v,
                                    void *stream)
{
    if (!ctx || n < 0 || !(dt > 0.0) || !std::isfinite(dt)) {
        set_error("sphx_gdf_alpha_v_update: need a context, n >= 0 and a finite dt > 0");
        return SPHX_E_INVALID;
    }
    if (n > 0 && (!D_old || !D_new || !c || !h || !v_sig || !balsara || !alpha_v)) {
        set_error("sphx_gdf_alpha_v_update: NULL array");
        return SPHX_E_INVALID;
    }
    SPHX_HIP(hipSetDevice(ctx->device));
    return gdf_alpha_v_launch(n, D_old, D_new, c, h, v_sig, balsara, active, dt, alpha_v,
                              as_stream(stream));
}

sphx_status sphx_alpha_c_update(sphx_ctx *ctx, int64_t n, const float *lap_u, const float *u,
                                const float *h, const float *v_c, const float *alpha_v_max,
                                const uint8_t *active, double dt, float *alpha_c, void *stream)
{
    if (!ctx || n < 0 || !(dt > 0.0) || !std::isfinite(dt)) {
        set_error("sphx_alpha_c_update: need a context, n >= 0 and a finite dt > 0");
        return SPHX_E_INVALID;
    }
    if (n > 0 && (!lap_u || !u || !h || !v_c || !alpha_v_max || !alpha_c)) {
        set_error("sphx_alpha_c_update: NULL array");
        return SPHX_E_INVALID;
    }
    SPHX_HIP(hipSetDevice(ctx->device));
    return alpha_c_launch(ctx, n, lap_u, u, h, v_c, alpha_v_max, active, dt, alpha_c,
                          as_stream(stream));
}

sphx_status sphx_timestep(sphx_ctx *ctx, sphx_grid *grid, const sphx_tasks *tasks,
                          const sphx_particles *in, const float *v_sig, double c_cfl,
                          double delta, float *dt, float *d_dt_min, void *stream)
{
    SPHX_TRY(check_handles(ctx, grid, tasks, in));
    SPHX_TRY(check_particles(in, false));
    if (!(c_cfl > 0.0) || !std::isfinite(c_cfl) || !(delta >= 1.0) || !std::isfinite(delta)) {
        set_error("sphx_timestep: need 0 < c_cfl < inf and 1 <= delta < inf");
        return SPHX_E_INVALID;
    }
    if (!tasks || (in->n && (!v_sig || !dt))) {
        set_error("sphx_timestep: NULL task list, v_sig or dt");
        return SPHX_E_INVALID;
    }
    SPHX_HIP(hipSetDevice(ctx->device));
    return timestep_launch(ctx, grid, tasks, in, v_sig, c_cfl, delta, dt, d_dt_min,
                           as_stream(stream));
}

sphx_status sphx_kick(sphx_ctx *ctx, int64_t n, const float *vx, const float *vy,
                      const float *vz, const float *u, const float *ax, const float *ay,
                      const float *az, const float *du_dt, const uint8_t *active, double dt_half,
                      float *vx_out, float *vy_out, float *vz_out, float *u_out, void *stream)
{
    if (!ctx || n < 0 || !std::isfinite(dt_half)) {
        set_error("sphx_kick: need a context, n >= 0 and a finite dt_half");
        return SPHX_E_INVALID;
    }
    if (n > 0 && (!vx || !vy || !vz || !u || !ax || !ay || !az || !du_dt || !vx_out ||
                  !vy_out || !vz_out || !u_out)) {
        set_error("sphx_kick: NULL array");
        return SPHX_E_INVALID;
    }
    SPHX_HIP(hipSetDevice(ctx->device));
    return kick_launch(n, vx, vy, vz, u, ax, ay, az, du_dt, active, dt_half, vx_out, vy_out,
                       vz_out, u_out, as_stream(stream));
}

sphx_status sphx_drift(sphx_ctx *ctx, int64_t n, double *x, double *y, double *z,
                       const float *vx, const float *vy, const float *vz, double dt,
                       void *stream)
{
    if (!ctx || n < 0 || !std::isfinite(dt)) {
        set_error("sphx_drift: need a context, n >= 0 and a finite dt");
        return SPHX_E_INVALID;
    }
    if (n > 0 && (!x || !y || !z || !vx || !vy || !vz)) {
        set_error("sphx_drift: NULL array");
        return SPHX_E_INVALID;
    }
    SPHX_HIP(hipSetDevice(ctx->device));
    return drift_launch(ctx, n, x, y, z, vx, vy, vz, dt, as_stream(stream));
}

sphx_status sphx_gravity(sphx_ctx *ctx, const sphx_particles *in, double G, double H,
                         double r_s, double r_p2p, float *ax, float *ay, float *az, float *pot,
                         int64_t *d_pairs, void *stream)
{
    if (!ctx || !in) {
        set_error("sphx_gravity: NULL argument");
        return SPHX_E_INVALID;
    }
    sphx_particles chk = *in;
    if (!chk.h)
        chk.h = ax;  // h is not used: the search radius is r_p2p
    SPHX_TRY(check_particles(&chk, false));
    const double lmin = std::min(ctx->p.box[0], std::min(ctx->p.box[1], ctx->p.box[2]));
    if (!(G > 0.0) || !(H > 0.0) || !(r_s >= 0.0) || !(r_p2p > 0.0) ||
        !(r_p2p <= lmin / 3.0 * (1.0 - 1e-5)) || !std::isfinite(G) || !std::isfinite(H) ||
        !std::isfinite(r_s)) {
        set_error("sphx_gravity: need G > 0, H > 0, r_s >= 0 and 0 < r_p2p <= min(box)/3 "
                  "(1 - 1e-5)");
        return SPHX_E_INVALID;
    }
    if (in->n > 0 && (!ax || !ay || !az)) {
        set_error("sphx_gravity: NULL acceleration array");
        return SPHX_E_INVALID;
    }
    SPHX_HIP(hipSetDevice(ctx->device));
    return gravity_run(ctx, in, G, H, r_s, r_p2p, ax, ay, az, pot, d_pairs, as_stream(stream));
}

sphx_status sphx_fof(sphx_ctx *ctx, const sphx_particles *in, double b, int32_t *group,
                     int32_t *group_size, int64_t *d_counts, void *stream)
{
    if (!ctx || !in) {
        set_error("sphx_fof: NULL argument");
        return SPHX_E_INVALID;
    }
    // h is not used (the search radius is b): check the rest with a stand-in
    sphx_particles chk = *in;
    if (!chk.h)
        chk.h = reinterpret_cast<float *>(group);
    SPHX_TRY(check_particles(&chk, false));
    const double lmin = std::min(ctx->p.box[0], std::min(ctx->p.box[1], ctx->p.box[2]));
    if (!(b > 0.0) || !(b <= lmin / 3.0 * (1.0 - 1e-5))) {
        set_error("sphx_fof: the linking length must be in (0, min(box)/3 (1 - 1e-5)]");
        return SPHX_E_INVALID;
    }
    if (in->n > 0 && !group) {
        set_error("sphx_fof: group is NULL");
        return SPHX_E_INVALID;
    }
    SPHX_HIP(hipSetDevice(ctx->device));
    return fof_run(ctx, in, b, group, group_size, d_counts, as_stream(stream));
}

sphx_status sphx_iter_reset(sphx_ctx *ctx, sphx_grid *grid, const sphx_particles *in,
                            void *stream)
{
    SPHX_TRY(check_handles(ctx, grid, nullptr, in));
    SPHX_TRY(check_particles(in, false));
    return iter_reset(grid, in, as_stream(stream));
}

// Every output array a whole step writes (sphx_step, sphx_autotune).
static sphx_status check_step_outputs(const char *who, const sphx_particles *in,
                                      const sphx_density_out *d, const sphx_ghost_out *g,
                                      const sphx_force_out *o)
{
    if (!d || !g || !o ||
        (in->n && (!d->rho || !d->rho_dh || !d->n || !d->n_dh || !d->div_sum || !d->curl_x ||
                   !d->curl_y || !d->curl_z || !d->nngb || !g->f || !g->P || !g->c ||
                   !g->balsara || !g->A || !g->div_v || !g->curl_v || !g->converged || !o->ax ||
                   !o->ay || !o->az || !o->du_dt || !o->v_sig))) {
        set_error(std::string(who) + ": NULL density, ghost or force output array");
        return SPHX_E_INVALID;
    }
    return SPHX_OK;
}

sphx_status sphx_density(sphx_ctx *ctx, const sphx_grid *grid, const sphx_tasks *tasks,
                         const sphx_particles *in, sphx_density_out *out, int32_t *d_counters,
                         void *stream)
{
    SPHX_TRY(check_handles(ctx, grid, tasks, in));
    SPHX_TRY(check_particles(in, false));
    if (!tasks || !out || (in->n && (!out->rho || !out->rho_dh || !out->n || !out->n_dh ||
                                      !out->div_sum || !out->curl_x || !out->curl_y ||
                                      !out->curl_z || !out->nngb))) {
        set_error("sphx_density: NULL task list or output array");
        return SPHX_E_INVALID;
    }
    // the caller may have changed h since the last pass
    SPHX_TRY(refresh_h(const_cast<sphx_grid *>(grid), in, as_stream(stream)));
    return density_launch(ctx, grid, tasks, in, out, d_counters, false, as_stream(stream));
}

sphx_status sphx_ghost(sphx_ctx *ctx, sphx_grid *grid, const sphx_tasks *tasks,
                       sphx_particles *in, const sphx_density_out *dens, sphx_ghost_out *out,
                       int32_t *d_counters, int32_t final_pass, void *stream)
{
    SPHX_TRY(check_handles(ctx, grid, tasks, in));
    SPHX_TRY(check_particles(in, true));
    if (!tasks || !dens || !out ||
        (in->n && (!out->f || !out->P || !out->c || !out->balsara || !out->A || !out->div_v ||
                   !out->curl_v || !out->converged))) {
        set_error("sphx_ghost: NULL task list, density or output array");
        return SPHX_E_INVALID;
    }
    return ghost_launch(ctx, grid, tasks, in, dens, out, d_counters, final_pass, false, nullptr,
                        as_stream(stream));
}

sphx_status sphx_force(sphx_ctx *ctx, const sphx_grid *grid, const sphx_tasks *tasks,
                       const sphx_particles *in, const sphx_density_out *dens,
                       const sphx_ghost_out *gst, sphx_force_out *out, double *d_sums6,
                       void *stream)
{
    SPHX_TRY(check_handles(ctx, grid, tasks, in));
    SPHX_TRY(check_particles(in, false));
    if (!tasks || !dens || !gst || !out ||
        (in->n && (!out->ax || !out->ay || !out->az || !out->du_dt || !out->v_sig || !dens->rho ||
                   !gst->P || !gst->c || !gst->f || !gst->balsara || !gst->A))) {
        set_error("sphx_force: NULL task list, state or output array");
        return SPHX_E_INVALID;
    }
    return force_launch(ctx, grid, tasks, in, dens, gst, out, d_sums6, as_stream(stream));
}

sphx_status sphx_force_noalloc(sphx_ctx *ctx, const sphx_grid *grid, const sphx_tasks *tasks,
                               const sphx_particles *in, const sphx_density_out *dens,
                               const sphx_ghost_out *gst, sphx_force_out *out, double *d_sums6,
                               void *stream)
{
    SPHX_TRY(check_handles(ctx, grid, tasks, in));
    SPHX_TRY(check_particles(in, false));
    if (!tasks || !dens || !gst || !out ||
        (in->n && (!out->ax || !out->ay || !out->az || !out->du_dt || !out->v_sig || !dens->rho ||
                   !gst->P || !gst->c || !gst->f || !gst->balsara || !gst->A))) {
        set_error("sphx_force_noalloc: NULL task list, state or output array");
        return SPHX_E_INVALID;
    }
    if (grid->n_leaves > kNoallocLeaves) {
        set_error("sphx_force_noalloc: the grid has " + std::to_string(grid->n_leaves) +
                  " leaf cells, more than the " + std::to_string(kNoallocLeaves) +
                  " its fixed workspace holds (use sphx_force)");
        return SPHX_E_INVALID;
    }
    if (grid->n_sets > 1) {
        set_error("sphx_force_noalloc: the grid holds several particle sets (its fixed "
                  "workspace holds the reduction of one; use sphx_force)");
        return SPHX_E_INVALID;
    }
    if (!ctx->noalloc_sums) {
        set_error("sphx_force_noalloc: no fixed workspace on this device");
        return SPHX_E_STATE;
    }
    return force_launch(ctx, grid, tasks, in, dens, gst, out, d_sums6, as_stream(stream), nullptr,
                        false, ctx->noalloc_sums);
}

// The step after validation (sphx_step; the autotuner's timed steps).
static sphx_status step_run(sphx_ctx *ctx, sphx_grid *grid, sphx_tasks **tasks,
                            sphx_particles *in, sphx_density_out *dens, sphx_ghost_out *gst,
                            sphx_force_out *out, double *d_sums6, hipStream_t s,
                            sphx_step_info *info)
{
    sphx_step_info local;
    memset(&local, 0, sizeof(local));
    if (!*tasks)
        SPHX_TRY(tasks_build(ctx, grid, in, s, tasks));
    const int64_t relayouts0 = (*tasks)->relayouts;
    unsigned char *h_buf = ctx->h_pinned;  // kStepCounterBytes of it
    memset(h_buf, 0, kStepCounterBytes);
    int32_t h_counters[kStepCounters] = {0, 0, 0, 0, 0, 0, 0, 0};
    int32_t *dc = ctx->d_counters;
    unsigned long long *d_units =
        reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(dc) + kStepUnitsOffset);
    SPHX_HIP(hipMemsetAsync(d_units, 0, 2 * sizeof(unsigned long long), s));
    const int max_iter = ctx->p.max_iter;
    bool want_lists = ctx->p.neighbour_lists != 0;
    int pass = 0;
    // (no captured pass is the final one of max_iter: that one runs here)
    const int graph_passes = std::min(ctx->p.graph_passes, max_iter - 1);
    if (graph_passes > 0 && !want_lists && grid->n_leaves > 0) {
        bool done = false, relayout = false, force_pending = false;
        SPHX_TRY(step_graph_run(ctx, grid, *tasks, in, dens, gst, out, d_sums6, graph_passes, s,
                                &local, &pass, &done, &relayout, &force_pending));
        local.captured_passes = pass;
        if (relayout) {
            // a leaf outgrew its slot inside the graph: a new layout
            SPHX_TRY(tasks_build(ctx, grid, in, s, tasks));
            local.task_rebuilds++;
        }
        if (force_pending)
            SPHX_TRY(force_launch(ctx, grid, *tasks, in, dens, gst, out, d_sums6, s, nullptr,
                                  true));
        if (done || force_pending) {
            local.passes = pass;
            local.n_leaves = grid->n_leaves;
            local.n_tasks = (*tasks)->n_tasks;
            local.task_relayouts = int32_t((*tasks)->relayouts - relayouts0);
            if (info)
                *info = local;
            sphx_status w = SPHX_OK;
            if (local.unconverged)
                w |= SPHX_W_NOT_CONVERGED;
            if (local.clamped)
                w |= SPHX_W_H_CLAMPED;
            return w;
        }
        // The iteration goes on pass by pass from the state the graph left
        // (its last slot rebuilt the list if that pass asked for it).
        unsigned long long u[2] = {(unsigned long long)local.pairs_cellpair,
                                   (unsigned long long)local.pairs_list};
        memcpy(h_buf + kStepUnitsOffset, u, sizeof(u));
    } else {
        SPHX_TRY(iter_reset(grid, in, s));
    }
    // lists: the neighbour lists are current (built on this task list, for
    // the receivers of the current pass); beyond: receivers of the next pass
    // whose H outgrew their list (they take the cell-pair loop).
    bool lists = false;
    int64_t beyond = 0;
    int stale_repeats = 0;
    while (pass < max_iter) {
        SPHX_HIP(hipMemsetAsync(dc, 0, kStepCounters * sizeof(int32_t), s));
        // Before the first pass: an h that outgrew the task list since it was
        // built (the caller's h, or the previous step's list) makes the pass
        // return at once; the list is rebuilt below and the pass repeated.
        const int32_t *skip = nullptr;
        if (pass == 0 && !lists) {
            SPHX_TRY(stale_count_launch(ctx, grid, *tasks, dc + 3, s));
            skip = dc + 3;
        }
        if (!lists || beyond > 0)
            SPHX_TRY(density_launch(ctx, grid, *tasks, in, dens, dc, lists, s, skip));
        if (lists)
            SPHX_TRY(density_list_launch(ctx, grid, *tasks, dens, s));
        const int final_pass = (pass + 1 == max_iter) ? 1 : 0;
        SPHX_TRY(ghost_launch(ctx, grid, *tasks, in, dens, gst, dc, final_pass, lists, d_units,
                              s, nullptr, true));
        SPHX_HIP(hipMemcpyAsync(h_buf, dc, kStepCounterBytes, hipMemcpyDeviceToHost, s));
        SPHX_HIP(wait_stream(ctx, s));
        memcpy(h_counters, h_buf, sizeof(h_counters));
        if (h_counters[3] > 0) {
            // The pass ran on a stale task list and the ghost skipped it.
            if (++stale_repeats > 4) {
                set_error("sphx_step: task list keeps going stale");
                return SPHX_E_STATE;
            }
            SPHX_TRY(tasks_grow(ctx, grid, in, s, tasks));
            local.task_rebuilds++;
            lists = false;
            continue;
        }
        ++pass;
        local.clamped += h_counters[2];
        if (h_counters[0] == 0)
            break;
        if (final_pass) {
            local.unconverged = h_counters[0];
            break;
        }
        if (h_counters[1] > 0) {
            SPHX_TRY(tasks_grow(ctx, grid, in, s, tasks));
            local.task_rebuilds++;
            lists = false;  // list entries name tasks of the old list
        }
        beyond = lists ? h_counters[4] : 0;
        if (lists)
            local.list_fallback += h_counters[4];
        // (Re)build the lists after the first pass, after a task rebuild, and
        // when many receivers have outgrown theirs.
        if (want_lists && (!lists || beyond > h_counters[0] / 4)) {
            bool ok = false;
            SPHX_TRY(list_build(ctx, grid, *tasks, s, &ok));
            lists = ok;
            want_lists = ok;  // no memory or too many tasks: cell-pair loop from here on
            beyond = 0;
            if (ok) {
                local.list_builds++;
                local.list_entries = grid->lst_total;
            }
        }
    }
    local.passes = pass;
    {
        unsigned long long u[2];
        memcpy(u, h_buf + kStepUnitsOffset, sizeof(u));
        local.pairs_cellpair = int64_t(u[0]);
        local.pairs_list = int64_t(u[1]);
    }
    if (!(*tasks)->symmetric) {
        // the growth rebuilds served the density passes; the force pass needs
        // every pair that either side's radius reaches
        SPHX_TRY(tasks_build(ctx, grid, in, s, tasks));
        local.task_rebuilds++;
    }
    SPHX_TRY(force_launch(ctx, grid, *tasks, in, dens, gst, out, d_sums6, s, nullptr, true));
    local.n_leaves = grid->n_leaves;
    local.n_tasks = (*tasks)->n_tasks;
    local.task_relayouts = int32_t((*tasks)->relayouts - relayouts0);
    if (info)
        *info = local;
    sphx_status w = SPHX_OK;
    if (local.unconverged)
        w |= SPHX_W_NOT_CONVERGED;
    if (local.clamped)
        w |= SPHX_W_H_CLAMPED;
    return w;
}

sphx_status sphx_step(sphx_ctx *ctx, sphx_grid *grid, sphx_tasks **tasks, sphx_particles *in,
                      sphx_density_out *dens, sphx_ghost_out *gst, sphx_force_out *out,
                      double *d_sums6, void *stream, sphx_step_info *info)
{
    if (!tasks) {
        set_error("sphx_step: NULL task-list pointer");
        return SPHX_E_INVALID;
    }
    SPHX_TRY(check_handles(ctx, grid, *tasks, in));
    SPHX_TRY(check_particles(in, true));
    SPHX_TRY(check_step_outputs("sphx_step", in, dens, gst, out));
    SPHX_HIP(hipSetDevice(ctx->device));
    return step_run(ctx, grid, tasks, in, dens, gst, out, d_sums6, as_stream(stream), info);
}

sphx_status sphx_autotune(sphx_ctx *ctx, sphx_grid *grid, sphx_tasks *tasks, sphx_particles *in,
                          sphx_density_out *dens, sphx_ghost_out *gst, sphx_force_out *out,
                          int32_t reps, sphx_params *tuned, void *stream)
{
    SPHX_TRY(check_handles(ctx, grid, tasks, in));
    SPHX_TRY(check_particles(in, true));
    if (!tasks || !tuned || reps < 1) {
        set_error("sphx_autotune: NULL task list or result, or reps < 1");
        return SPHX_E_INVALID;
    }
    SPHX_TRY(check_step_outputs("sphx_autotune", in, dens, gst, out));
    hipStream_t s = as_stream(stream);
    SPHX_HIP(hipSetDevice(ctx->device));
    const sphx_params saved = ctx->p;
    struct Events {
        hipEvent_t a = nullptr, b = nullptr;
        ~Events()
        {
            if (a)
                (void)hipEventDestroy(a);
            if (b)
                (void)hipEventDestroy(b);
        }
    } ev;
    SPHX_HIP(hipEventCreate(&ev.a));
    SPHX_HIP(hipEventCreate(&ev.b));
    // Shortest of `reps` timed runs of f (after one untimed run).
    auto timed = [&](auto &&setup, auto &&f, double *ms) -> sphx_status {
        SPHX_TRY(setup());
        SPHX_TRY(f());
        double best = 1e300;
        for (int r = 0; r < reps; ++r) {
            SPHX_TRY(setup());
            SPHX_HIP(hipEventRecord(ev.a, s));
            SPHX_TRY(f());
            SPHX_HIP(hipEventRecord(ev.b, s));
            SPHX_HIP(hipEventSynchronize(ev.b));
            float t = 0.f;
            SPHX_HIP(hipEventElapsedTime(&t, ev.a, ev.b));
            best = std::min(best, double(t));
        }
        *ms = best;
        return SPHX_OK;
    };
    // The timed steps iterate on a copy of h; the caller's h is never written.
    float *h_tmp = nullptr;
    if (in->n > 0)
        SPHX_HIP(dmalloc((void **)&h_tmp, size_t(in->n) * sizeof(float), s));
    struct Scratch {
        float *p;
        hipStream_t s;
        ~Scratch() { dfree(p, s); }
    } scratch{h_tmp, s};
    sphx_particles tmp = *in;
    tmp.h = h_tmp;
    auto reset_h = [&]() -> sphx_status {
        if (in->n > 0)
            SPHX_HIP(hipMemcpyAsync(h_tmp, in->h, size_t(in->n) * sizeof(float),
                                    hipMemcpyDeviceToDevice, s));
        return SPHX_OK;
    };
    sphx_tasks *tl = tasks;
    // Density kernel time of one whole step from the current copy of h: HIP
    // events around each of its density launches (whole-step wall time is too
    // noisy to order shapes a few percent apart), recorded after the
    // context's own kernel statistics and removed again.
    auto step_density_ms = [&](double *ms) -> sphx_status {
        Profiler &P = *ctx->prof;
        const bool was_on = P.on;
        const size_t base = P.used[0];
        P.on = true;
        const sphx_status w = step_run(ctx, grid, &tl, &tmp, dens, gst, out, nullptr, s, nullptr);
        P.on = was_on;
        double t = 0.0;
        hipError_t e = hipSuccess;
        for (size_t k = base; w >= 0 && e == hipSuccess && k < P.used[0]; ++k) {
            e = hipEventSynchronize(P.pool[0][k].b);
            float x = 0.f;
            if (e == hipSuccess)
                e = hipEventElapsedTime(&x, P.pool[0][k].a, P.pool[0][k].b);
            t += x;
        }
        P.used[0] = base;
        if (w < 0)
            return w;
        SPHX_HIP(e);
        *ms = t;
        return SPHX_OK;
    };
    auto run = [&]() -> sphx_status {
        ctx->p.graph_passes = 0;
        // Density shapes (tile, waves, balance) on whole steps from the
        // caller's h: the passes after the first run on ever fewer receivers,
        // and the best shape for the full first pass is not always the best
        // for the step. (The balanced rounds, never measurably faster, are
        // not among the tuned shapes; the grouped rounds are.)
        const int32_t dshape[7][3] = {{128, 1, 0}, {64, 1, 0}, {256, 1, 0}, {128, 2, 0},
                                      {64, 2, 0},  {128, 1, 2}, {256, 1, 2}};
        double best = 1e300;
        int32_t bt = 128, bw = 1, bb = 0;
        for (auto &sh : dshape) {
            if (sh[2] != 0 && sphx::smoothed_pressure(ctx->p.flavour))
                continue;  // built for the plain loop only
            ctx->p.density_tile = sh[0];
            ctx->p.density_waves = sh[1];
            ctx->p.density_balance = sh[2];
            double ms = 1e300, x = 0.0;
            SPHX_TRY(reset_h());
            SPHX_TRY(step_density_ms(&x));  // untimed
            for (int r = 0; r < reps; ++r) {
                SPHX_TRY(reset_h());
                SPHX_TRY(step_density_ms(&x));
                ms = std::min(ms, x);
            }
            if (ms < best) {
                best = ms;
                bt = sh[0];
                bw = sh[1];
                bb = sh[2];
            }
        }
        ctx->p.density_tile = bt;
        ctx->p.density_waves = bw;
        ctx->p.density_balance = bb;
        // Force shapes at the converged state the last step left (h in the
        // copy, density and ghost outputs).
        const int32_t fshape[4][2] = {{64, 1}, {128, 1}, {64, 2}, {128, 2}};
        best = 1e300;
        int32_t ft = 64, fw = 1;
        for (auto &sh : fshape) {
            ctx->p.force_tile = sh[0];
            ctx->p.force_waves = sh[1];
            double ms = 0.0;
            SPHX_TRY(timed([&]() { return SPHX_OK; },
                           [&]() { return force_launch(ctx, grid, tl, &tmp, dens, gst, out,
                                                       nullptr, s); },
                           &ms));
            if (ms < best) {
                best = ms;
                ft = sh[0];
                fw = sh[1];
            }
        }
        *tuned = saved;
        tuned->density_tile = bt;
        tuned->density_waves = bw;
        tuned->density_balance = bb;
        tuned->force_tile = ft;
        tuned->force_waves = fw;
        // the task list as a build at the caller's h leaves it
        ctx->p = saved;
        SPHX_TRY(refresh_h(grid, in, s));
        SPHX_TRY(tasks_build(ctx, grid, in, s, &tl));
        SPHX_HIP(hipStreamSynchronize(s));
        return SPHX_OK;
    };
    const sphx_status st = run();
    ctx->p = saved;
    return st;
}

sphx_status sphx_profile_enable(sphx_ctx *ctx, int32_t enable)
{
    if (!ctx) {
        set_error("sphx_profile_enable: NULL context");
        return SPHX_E_INVALID;
    }
    ctx->prof->on = enable != 0;
    if (enable)
        for (int k = 0; k < Profiler::kKinds; ++k)
            ctx->prof->used[k] = 0;
    return SPHX_OK;
}

sphx_status sphx_profile_read(sphx_ctx *ctx, int32_t kernel, double *total_ms, int64_t *launches)
{
    if (!ctx || kernel < 0 || kernel >= Profiler::kKinds || !total_ms || !launches) {
        set_error("sphx_profile_read: invalid argument");
        return SPHX_E_INVALID;
    }
    double t = 0.0;
    Profiler &P = *ctx->prof;
    for (size_t k = 0; k < P.used[kernel]; ++k) {
        SPHX_HIP(hipEventSynchronize(P.pool[kernel][k].b));
        float ms = 0.f;
        SPHX_HIP(hipEventElapsedTime(&ms, P.pool[kernel][k].a, P.pool[kernel][k].b));
        t += ms;
    }
    *total_ms = t;
    *launches = int64_t(P.used[kernel]);
    return SPHX_OK;
}

sphx_status sphx_probe_read(sphx_ctx *ctx, uint64_t *counts5, int32_t clear)
{
    if (!ctx || !counts5) {
        set_error("sphx_probe_read: NULL argument");
        return SPHX_E_INVALID;
    }
    SPHX_HIP(hipSetDevice(ctx->device));
    unsigned long long v[5] = {0, 0, 0, 0, 0};
    const sphx_status st = probe_read(v, clear != 0);
    for (int k = 0; k < 5; ++k)
        counts5[k] = v[k];
    return st;
}

int64_t sphx_grid_leaves(const sphx_grid *grid) { return grid ? grid->n_leaves : -1; }

int64_t sphx_tasks_count(const sphx_tasks *tasks) { return tasks ? tasks->n_tasks : -1; }

}  // extern "C"
