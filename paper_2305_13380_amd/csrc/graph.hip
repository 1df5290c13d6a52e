// Captured h-iteration step. The passes of the iteration (Section 3.1: the
// density loop and the ghost, repeated until every h has converged), the
// task rebuilds between them and the force loop are recorded once as a HIP
// graph on a private capture stream and replayed on the caller's stream for
// as long as the grid, task list, arrays and loop shapes stay the same.
// Passes after every particle has converged find no receiver and do nothing,
// so the graph can hold a fixed number of them. After each pass a log kernel
// keeps its counters and decides, on the device, whether the task list must
// be rebuilt before the next one (the pass met a stale list, or left an h
// beyond its leaf's radius); the in-place growth walk that follows runs only
// then (its kernels return at once otherwise). Before the force pass, a full
// walk restores the symmetric list if any growth walk ran. Only a leaf that
// outgrows its slot stops the graph (a new layout needs an allocation): the
// remaining kernels then return at once and the caller takes over. One
// readback of the log after the replay replaces the readback after every
// pass; if the iteration is not finished inside the graph the caller
// continues it pass by pass from the state the graph left. Counters and
// flags are cleared by kernels: the graph holds no memset nodes.
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

// Gate words: [0] force pass closed, [1] stopped (a leaf outgrew its slot),
// [2] the remaining passes return at once, [3] growth walk after this pass,
// [4] full walk before the force pass.
constexpr int kGateWords = 5;
// Per pass slot, after the pass's own counters [0..4]: [5] the slot's pass
// ran, [6] a growth walk followed it, [7] that walk outgrew a slot. After
// the slots: [0] the full walk ran, [1] it outgrew a slot.
constexpr int kLogRan = 5, kLogGrown = 6, kLogOutgrown = 7;

// Slot p's counters into the log, and the gates. A pass that met a stale
// task list (c[3] > 0: the density loop and the ghost returned at once) does
// not count; its slot rebuilds the list and the next slot repeats it.
__global__ void k_log_pass(const int32_t *__restrict__ c, int32_t *__restrict__ log, int p,
                           int32_t *__restrict__ gate)
{
    const int i = threadIdx.x;
    int32_t *L = log + p * kStepCounters;
    if (i < kLogRan)
        L[i] = c[i];
    if (i != 0)
        return;
    L[kLogOutgrown] = 0;
    if (gate[2]) {
        L[kLogRan] = 0;
        L[kLogGrown] = 0;
        gate[3] = 0;
        return;
    }
    L[kLogRan] = 1;
    if (c[3] > 0) {
        gate[0] = 1;
        gate[3] = 1;
    } else if (c[0] == 0) {
        gate[0] = 0;  // every particle finalised: the force pass may run
        gate[2] = 1;
        gate[3] = 0;
    } else {
        gate[0] = 1;
        gate[3] = c[1] > 0 ? 1 : 0;
    }
    L[kLogGrown] = gate[3];
}

// The outcome of slot p's growth walk (gate[3] says it ran): a leaf over its
// slot stops the graph.
__device__ __forceinline__ void grown_check(const int64_t *__restrict__ state,
                                            int32_t *__restrict__ log, int p,
                                            int32_t *__restrict__ gate)
{
    if (!gate[3])
        return;
    gate[3] = 0;
    if (state[kTaskOutgrown]) {
        gate[0] = gate[1] = gate[2] = 1;
        log[p * kStepCounters + kLogOutgrown] = 1;
    }
}

// Start of slot p: the previous slot's growth outcome, the counters cleared.
__global__ void k_slot_start(int32_t *__restrict__ c, const int64_t *__restrict__ state,
                             int32_t *__restrict__ log, int p, int32_t *__restrict__ gate)
{
    const int i = threadIdx.x;
    if (i < kStepCounters)
        c[i] = 0;
    if (i == 0 && p > 0)
        grown_check(state, log, p - 1, gate);
}

// After the last slot (`last`): its growth outcome; then the full walk runs
// when the iteration finished inside the graph (force open) and a growth
// walk left the list not symmetric.
__global__ void k_full_gate(const int64_t *__restrict__ state, int32_t *__restrict__ log,
                            int last, int32_t *__restrict__ gate)
{
    if (threadIdx.x != 0)
        return;
    grown_check(state, log, last, gate);
    gate[4] = (gate[0] == 0 && state[kTaskAsym] != 0) ? 1 : 0;
}

__global__ void k_full_done(const int64_t *__restrict__ state, int32_t *__restrict__ gate,
                            int32_t *__restrict__ tail)
{
    if (threadIdx.x != 0)
        return;
    tail[0] = gate[4];
    tail[1] = 0;
    if (gate[4] && state[kTaskOutgrown]) {
        gate[0] = gate[1] = 1;  // the force pass waits for a new layout
        tail[1] = 1;
    }
    gate[4] = 0;
}

}  // namespace

struct StepGraph {
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const void *> key;
    int32_t *d_log = nullptr;   // passes x kStepCounters, then the full walk's 2 words
    int32_t *d_gate = nullptr;  // kGateWords
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
    int32_t *gate = G->d_gate;
    SPHX_TRY(iter_reset(grid, in, cs));
    k_fill_i32<<<1, 64, 0, cs>>>(gate, kGateWords, 0);
    SPHX_HIP(hipGetLastError());
    for (int p = 0; p < passes; ++p) {
        k_slot_start<<<1, 64, 0, cs>>>(ctx->d_counters, t->state, G->d_log, p, gate);
        SPHX_HIP(hipGetLastError());
        // the first pass returns at once on a stale task list (its slot then
        // rebuilds the list and the next slot repeats the pass)
        if (p == 0)
            SPHX_TRY(stale_count_launch(ctx, grid, t, ctx->d_counters + 3, cs));
        SPHX_TRY(density_launch(ctx, grid, t, in, dens, ctx->d_counters, false, cs,
                                p == 0 ? ctx->d_counters + 3 : gate + 2));
        // (no slot is the final pass: the caller runs that one)
        SPHX_TRY(ghost_launch(ctx, grid, t, pin, dens, gst, ctx->d_counters, 0, false, units,
                              cs, gate + 2, true));
        k_log_pass<<<1, 64, 0, cs>>>(ctx->d_counters, G->d_log, p, gate);
        SPHX_HIP(hipGetLastError());
        SPHX_TRY(tasks_grow_async(ctx, grid, t, gate + 3, cs));
    }
    k_full_gate<<<1, 64, 0, cs>>>(t->state, G->d_log, passes - 1, gate);
    SPHX_HIP(hipGetLastError());
    SPHX_TRY(tasks_full_async(ctx, grid, t, gate + 4, cs));
    k_full_done<<<1, 64, 0, cs>>>(t->state, gate, G->d_log + passes * kStepCounters);
    SPHX_HIP(hipGetLastError());
    SPHX_TRY(tasks_total_async(grid, t, cs));
    return force_launch(ctx, grid, t, in, dens, gst, out, sums6, cs, gate, true);
}

sphx_status step_graph_run(sphx_ctx *ctx, sphx_grid *grid, sphx_tasks *t, const sphx_particles *in,
                           const sphx_density_out *dens, const sphx_ghost_out *gst,
                           const sphx_force_out *out, double *sums6, int passes, hipStream_t s,
                           sphx_step_info *info, int *pass, bool *done, bool *relayout,
                           bool *force_pending)
{
    *pass = 0;
    *done = *relayout = *force_pending = false;
    StepGraph *G = ctx->graph;
    if (!G) {
        G = new StepGraph();
        ctx->graph = G;
        SPHX_HIP(hipStreamCreateWithFlags(&G->cap, hipStreamNonBlocking));
        SPHX_HIP(hipMalloc((void **)&G->d_gate, 8 * sizeof(int32_t)));
    }
    if (passes > G->cap_passes) {
        (void)hipFree(G->d_log);
        G->d_log = nullptr;
        G->cap_passes = 0;
        SPHX_HIP(hipMalloc((void **)&G->d_log,
                           (size_t(passes) * kStepCounters + 8) * sizeof(int32_t)));
        G->cap_passes = passes;
        if (G->exec) {
            (void)hipGraphExecDestroy(G->exec);
            G->exec = nullptr;
        }
    }
    unsigned long long *units = reinterpret_cast<unsigned long long *>(
        reinterpret_cast<char *>(ctx->d_counters) + kStepUnitsOffset);
    const std::vector<const void *> key = {
        grid, t, t->task, t->slot, t->end, t->state, t->order, t->radius, in->x, in->y, in->z,
        in->vx, in->vy, in->vz, in->m, in->u, in->h, in->alpha_v, in->alpha_c, in->active,
        dens->rho, dens->rho_dh, dens->n, dens->n_dh, dens->div_sum, dens->curl_x, dens->curl_y,
        dens->curl_z, dens->nngb, gst->f, gst->P, gst->c, gst->balsara, gst->A, gst->div_v,
        gst->curl_v, gst->converged, out->ax, out->ay, out->az, out->du_dt, out->v_sig,
        out->nforce, sums6, reinterpret_cast<const void *>(intptr_t(passes)),
        reinterpret_cast<const void *>(intptr_t(grid->n)),
        reinterpret_cast<const void *>(intptr_t(grid->n_leaves)),
        reinterpret_cast<const void *>(uintptr_t(grid->serial)),
        reinterpret_cast<const void *>(uintptr_t(t->serial))};
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
    std::vector<int32_t> log(size_t(passes) * kStepCounters + 2);
    unsigned long long u[2] = {0, 0};
    int64_t st[kTaskStateWords];
    SPHX_HIP(hipMemcpyAsync(log.data(), G->d_log, log.size() * sizeof(int32_t),
                            hipMemcpyDeviceToHost, s));
    SPHX_HIP(hipMemcpyAsync(u, units, sizeof(u), hipMemcpyDeviceToHost, s));
    SPHX_HIP(hipMemcpyAsync(st, t->state, sizeof(st), hipMemcpyDeviceToHost, s));
    SPHX_HIP(hipStreamSynchronize(s));
    info->pairs_cellpair = int64_t(u[0]);
    info->pairs_list = int64_t(u[1]);
    t->n_tasks = st[kTaskTotal];
    t->symmetric = st[kTaskAsym] == 0;
    bool converged = false;
    for (int p = 0; p < passes; ++p) {
        const int32_t *c = log.data() + size_t(p) * kStepCounters;
        if (!c[kLogRan])
            break;
        if (c[kLogGrown])
            info->task_rebuilds++;
        if (c[3] == 0) {  // (a stale pass is not counted: the next slot repeats it)
            *pass += 1;
            info->clamped += c[2];
            if (c[0] == 0) {
                converged = true;
                break;
            }
        }
        if (c[kLogOutgrown]) {
            *relayout = true;  // the caller lays the list out anew and goes on
            break;
        }
    }
    const int32_t *tail = log.data() + size_t(passes) * kStepCounters;
    if (tail[0])
        info->task_rebuilds++;
    if (converged) {
        if (tail[1]) {
            *relayout = true;  // the full walk outgrew a slot: no force pass yet
            *force_pending = true;
        } else {
            *done = true;
        }
    }
    return SPHX_OK;
}

}  // namespace sphx
