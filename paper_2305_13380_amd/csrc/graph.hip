// Captured h-iteration step. The passes of the iteration (Section 3.1: the
// density loop and the ghost, repeated until every h has converged) and the
// force loop are recorded once as a HIP graph on a private capture stream and
// replayed on the caller's stream for as long as the grid, task list, arrays
// and loop shapes stay the same. Passes after every particle has converged
// find no receiver and do nothing, so the graph can hold a fixed number of
// them; a log kernel after each pass keeps its counters and stops the later
// passes when the task list needs a rebuild (the graph cannot rebuild it),
// and the force kernels are gated on the log (no pass stopped the graph, and
// the last pass left no particle unconverged). One readback of the log after the
// replay replaces the readback after every pass; if the iteration is not
// finished inside the graph the caller continues it pass by pass from the
// state the graph left. Counters and flags are cleared by kernels: the graph
// holds no memset nodes.
#include <cstring>
#include <vector>

#include "sphx_internal.h"

namespace sphx {
namespace {

__global__ void k_fill_i32(int32_t *__restrict__ p, int n, int32_t v)
{
    const int i = int(blockIdx.x) * int(blockDim.x) + int(threadIdx.x);
    if (i < n)
        p[i] = v;
}

// Pass p's counters into the log, and the flags: gate[1] remembers a pass
// that must not be followed inside the graph (it met a stale task list, or it
// left an h beyond its task radius, so the next pass would: the caller
// rebuilds the list and goes on pass by pass); gate[0] = 0 opens the force
// pass (no such pass, and pass p left no particle unconverged; a final pass
// finalises every particle); gate[2] = 1 makes the remaining passes return at
// once (such a pass, or nothing left).
__global__ void k_log_pass(const int32_t *__restrict__ c, int32_t *__restrict__ log, int p,
                           int final_pass, int32_t *__restrict__ gate)
{
    const int i = threadIdx.x;
    if (i < kStepCounters)
        log[p * kStepCounters + i] = c[i];
    if (i == 0) {
        const int32_t halt = gate[1] | (c[3] > 0 ? 1 : 0) |
                             ((c[1] > 0 && c[0] > 0 && !final_pass) ? 1 : 0);
        gate[1] = halt;
        gate[0] = halt | ((c[0] > 0 && !final_pass) ? 1 : 0);
        gate[2] = halt | (c[0] == 0 ? 1 : 0);
    }
}

}  // namespace

struct StepGraph {
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const void *> key;
    int32_t *d_log = nullptr;   // passes x kStepCounters
    int32_t *d_gate = nullptr;  // [0] force gate, [1] a pass was stale, [2] skip the rest
    int cap_passes = 0;
};

void step_graph_free(StepGraph *g)
{
    if (!g)
        return;
    if (g->exec)
        (void)hipGraphExecDestroy(g->exec);
    if (g->cap)
        (void)hipStreamDestroy(g->cap);
    (void)hipFree(g->d_log);
    (void)hipFree(g->d_gate);
    delete g;
}

static sphx_status record(sphx_ctx *ctx, StepGraph *G, sphx_grid *grid, sphx_tasks *t,
                          const sphx_particles *in, const sphx_density_out *dens,
                          const sphx_ghost_out *gst, const sphx_force_out *out, double *sums6,
                          int passes, unsigned long long *units, hipStream_t cs)
{
    sphx_particles *pin = const_cast<sphx_particles *>(in);
    SPHX_TRY(iter_reset(grid, in, cs));
    k_fill_i32<<<1, 64, 0, cs>>>(G->d_gate, 3, 0);
    SPHX_HIP(hipGetLastError());
    for (int p = 0; p < passes; ++p) {
        const int final_pass = (p + 1 == ctx->p.max_iter) ? 1 : 0;
        k_fill_i32<<<1, 64, 0, cs>>>(ctx->d_counters, kStepCounters, 0);
        SPHX_HIP(hipGetLastError());
        // the first pass returns at once on a stale task list (the log then
        // stops the graph and the caller rebuilds)
        if (p == 0)
            SPHX_TRY(stale_count_launch(ctx, grid, t, ctx->d_counters + 3, cs));
        SPHX_TRY(density_launch(ctx, grid, t, in, dens, ctx->d_counters, false, cs,
                                p == 0 ? ctx->d_counters + 3 : G->d_gate + 2));
        SPHX_TRY(ghost_launch(ctx, grid, t, pin, dens, gst, ctx->d_counters, final_pass, false,
                              units, cs, G->d_gate + 2, true));
        k_log_pass<<<1, 64, 0, cs>>>(ctx->d_counters, G->d_log, p, final_pass, G->d_gate);
        SPHX_HIP(hipGetLastError());
    }
    return force_launch(ctx, grid, t, in, dens, gst, out, sums6, cs, G->d_gate, true);
}

sphx_status step_graph_run(sphx_ctx *ctx, sphx_grid *grid, sphx_tasks *t, const sphx_particles *in,
                           const sphx_density_out *dens, const sphx_ghost_out *gst,
                           const sphx_force_out *out, double *sums6, int passes, hipStream_t s,
                           sphx_step_info *info, int *pass, bool *done, bool *stale,
                           bool *rebuild)
{
    *pass = 0;
    *done = *stale = *rebuild = false;
    StepGraph *G = ctx->graph;
    if (!G) {
        G = new StepGraph();
        ctx->graph = G;
        SPHX_HIP(hipStreamCreateWithFlags(&G->cap, hipStreamNonBlocking));
        SPHX_HIP(hipMalloc((void **)&G->d_gate, 4 * sizeof(int32_t)));
    }
    if (passes > G->cap_passes) {
        (void)hipFree(G->d_log);
        G->d_log = nullptr;
        G->cap_passes = 0;
        SPHX_HIP(hipMalloc((void **)&G->d_log, size_t(passes) * kStepCounters * sizeof(int32_t)));
        G->cap_passes = passes;
        if (G->exec) {
            (void)hipGraphExecDestroy(G->exec);
            G->exec = nullptr;
        }
    }
    unsigned long long *units = reinterpret_cast<unsigned long long *>(
        reinterpret_cast<char *>(ctx->d_counters) + kStepUnitsOffset);
    const std::vector<const void *> key = {
        grid, t, t->task, t->off, t->order, t->radius, in->x, in->y, in->z, in->vx, in->vy, in->vz,
        in->m, in->u, in->h, in->alpha_v, in->alpha_c, in->active, dens->rho, dens->rho_dh,
        dens->n, dens->n_dh, dens->div_sum, dens->curl_x, dens->curl_y, dens->curl_z, dens->nngb,
        gst->f, gst->P, gst->c, gst->balsara, gst->A, gst->div_v, gst->curl_v, gst->converged,
        out->ax, out->ay, out->az, out->du_dt, out->v_sig, out->nforce, sums6,
        reinterpret_cast<const void *>(intptr_t(passes)),
        reinterpret_cast<const void *>(intptr_t(grid->n)),
        reinterpret_cast<const void *>(intptr_t(grid->n_leaves))};
    if (!G->exec || key != G->key) {
        if (G->exec) {
            (void)hipGraphExecDestroy(G->exec);
            G->exec = nullptr;
        }
        const bool prof_on = ctx->prof->on;
        ctx->prof->on = false;  // no event nodes in the graph
        SPHX_HIP(hipStreamBeginCapture(G->cap, hipStreamCaptureModeThreadLocal));
        const sphx_status rs =
            record(ctx, G, grid, t, in, dens, gst, out, sums6, passes, units, G->cap);
        hipGraph_t graph = nullptr;
        const hipError_t ce = hipStreamEndCapture(G->cap, &graph);
        ctx->prof->on = prof_on;
        if (rs != SPHX_OK) {
            if (graph)
                (void)hipGraphDestroy(graph);
            return rs;
        }
        SPHX_HIP(ce);
        const hipError_t ie = hipGraphInstantiate(&G->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        SPHX_HIP(ie);
        G->key = key;
    }
    SPHX_HIP(hipGraphLaunch(G->exec, s));
    std::vector<int32_t> log(size_t(passes) * kStepCounters);
    unsigned long long u[2] = {0, 0};
    SPHX_HIP(hipMemcpyAsync(log.data(), G->d_log, log.size() * sizeof(int32_t),
                            hipMemcpyDeviceToHost, s));
    SPHX_HIP(hipMemcpyAsync(u, units, sizeof(u), hipMemcpyDeviceToHost, s));
    SPHX_HIP(hipStreamSynchronize(s));
    info->pairs_cellpair = int64_t(u[0]);
    info->pairs_list = int64_t(u[1]);
    for (int p = 0; p < passes; ++p) {
        const int32_t *c = log.data() + size_t(p) * kStepCounters;
        if (c[3] > 0) {
            *stale = true;  // this and the later passes changed nothing
            break;
        }
        *pass = p + 1;
        info->clamped += c[2];
        if (c[0] == 0) {
            *done = true;
            break;
        }
        if (p + 1 == ctx->p.max_iter) {
            info->unconverged = c[0];
            *done = true;
            break;
        }
        if (c[1] > 0) {
            *rebuild = true;  // the later passes of the graph returned at once
            break;
        }
    }
    return SPHX_OK;
}

}  // namespace sphx
