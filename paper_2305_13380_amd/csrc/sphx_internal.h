// Internal state and helpers of the sphx library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "sphx.h"

// ---------------------------------------------------------------------------
// Error reporting (thread-local message behind sphx_last_error()).
// ---------------------------------------------------------------------------
namespace sphx {

void set_error(const std::string &msg);

#define SPHX_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            ::sphx::set_error(std::string(#call) + ": " + hipGetErrorString(e_));        \
            return e_ == hipErrorOutOfMemory ? SPHX_E_OOM : SPHX_E_HIP;                  \
        }                                                                                \
    } while (0)

#define SPHX_TRY(expr)                                                                   \
    do {                                                                                 \
        sphx_status s_ = (expr);                                                         \
        if (s_ < 0)                                                                      \
            return s_;                                                                   \
    } while (0)

// One wave64 processes one leaf cell of at most kLeafMax particles.
constexpr int kWave = 64;
constexpr int kLeafMax = 64;
// Flavours whose density loop also forms the smoothed pressure (Appendix A).
__host__ __device__ inline bool smoothed_pressure(int flavour)
{
    return flavour == SPHX_FLAVOUR_PRESSURE_ENERGY || flavour == SPHX_FLAVOUR_ANARCHY_PU;
}
// The GDF flavour's conduction constant C of alpha_c = C |S| h^2 (Appendix A).
constexpr double kGdfC = 0.03;
constexpr int kTreeFan = 8;     // tree over leaves: groups of 8 consecutive nodes
constexpr int kMaxLevels = 24;
constexpr int kMortonBits = 21; // bits per axis of the 63-bit Morton key

// Task record: the source cell (its first sorted index and count), whether it
// is the receiving cell itself without a periodic shift, and the FP32 offset
// origin_j + shift - origin_i (formed in FP64). The second half repeats j0, so
// that it alone (16 bytes) locates a source particle in the receiver's frame.
struct alignas(16) Task {
    int32_t j0;
    int32_t jc;
    int32_t self;
    int32_t j;
    float ox, oy, oz;
    int32_t j0b;  // == j0
};

// Neighbour-list entry: (task index - the receiving leaf's first task) << 6 |
// index of the source within its leaf.
constexpr int kListCodeShift = 6;
constexpr int64_t kListMaxTasks = int64_t(1) << 26;  // task counts beyond this: no lists

// Counters of sphx_step's own array: the public four, then [4] receivers whose
// H outgrew their neighbour list; followed (at byte kStepUnitsOffset) by two
// 64-bit sums over the step: density interactions computed by the cell-pair
// loop and by the list loop.
constexpr int kStepCounters = 8;
constexpr size_t kStepUnitsOffset = kStepCounters * sizeof(int32_t);
constexpr size_t kStepCounterBytes = kStepUnitsOffset + 2 * sizeof(unsigned long long);

// Device words of a task list: a walked leaf outgrew its slot (a new layout
// is needed), the tasks held, the list is not symmetric (a growth rebuild
// since the last full build), and the slot total of a new layout.
constexpr int kTaskOutgrown = 0;
constexpr int kTaskTotal = 1;
constexpr int kTaskAsym = 2;
constexpr int kTaskSlots = 3;
constexpr int kTaskStateWords = 4;
// Most particle sets one grid holds (sphx_grid_build_sets).
constexpr int32_t kMaxSets = 1 << 16;

}  // namespace sphx

namespace sphx {
// Event pairs recorded around kernel launches while profiling is enabled.
struct Profiler {
    bool on = false;
    struct Rec {
        hipEvent_t a, b;
    };
    // density cell-pair, force, density list, list build, gravity
    static constexpr int kKinds = 5;
    std::vector<Rec> pool[kKinds];
    size_t used[kKinds] = {0, 0, 0, 0, 0};
    hipError_t begin(int k, hipStream_t s);
    hipError_t end(int k, hipStream_t s);
};
}  // namespace sphx

namespace sphx {
struct StepGraph;
constexpr size_t kPinnedBytes = 256;
}
struct sphx_ctx {
    sphx_params p;
    sphx::Profiler *prof;
    int device;
    double h_max;
    int32_t *d_counters;  // scratch counters used by sphx_step
    double *d_sums;       // scratch FP64 sums used by sphx_step when the caller passes none
    sphx::StepGraph *graph = nullptr;  // captured step (graph_passes > 0)
    // Readbacks inside a step (pass counters, task totals) land in pinned
    // host memory and are waited for by polling an event: a blocking stream
    // synchronisation left the device idle ~40 us per readback.
    unsigned char *h_pinned = nullptr;  // kPinnedBytes
    hipEvent_t ev_wait = nullptr;
    double *noalloc_sums = nullptr;  // this device's fixed workspace (sphx_force_noalloc)
    // recycle_workspace: the buffers (pointer, bytes) of the last destroyed
    // grid, freed on spare_stream unless the next build there takes them
    std::vector<std::pair<void *, size_t>> spare;
    hipStream_t spare_stream = nullptr;
};

// A number no other grid or task list of the process has had (a captured
// step is keyed on it: a new object can reuse a freed one's addresses).
uint64_t next_serial();

struct sphx_grid {
    sphx_ctx *ctx;
    uint64_t serial;
    hipStream_t stream;  // the stream the grid was built on (its memory is freed there)
    // recycle_workspace: the buffers of the build, handed back to the
    // context's spares when the grid is destroyed
    bool recycle = false;
    std::vector<std::pair<void *, size_t>> owned;
    int64_t n;
    int64_t n_leaves;
    int n_levels;
    int64_t level_off[sphx::kMaxLevels];  // node offset of each tree level (level 0 = leaves)
    int64_t level_cnt[sphx::kMaxLevels];
    int64_t n_nodes;

    // per sorted particle
    uint64_t *keys;     // sorted Morton keys
    int32_t *perm;      // sorted index -> caller index
    int32_t *inv;       // caller index -> sorted index (the sort's input array, reused)
    int32_t *leaf_of;   // sorted index -> leaf
    float4 *q0;         // x, y, z relative to the leaf origin; m
    float4 *q1;         // vx, vy, vz, u
    float2 *qa;         // alpha_v, alpha_c
    uint8_t *need;      // 1: needs a density pass
    float *hs;          // h in sorted order (kept equal to the caller's h by iter_reset,
                        // refresh_h and the ghost)
    float *hlo, *hhi;   // per particle, sorted: bracket of the h iteration's root
                        // (largest h with G < 0, smallest with G > 0), reset by iter_reset
    float4 *d0;         // density results in sorted order: n, 3 + h n'/n, rho, 1 + h rho'/(3 rho)
    float4 *d1;         // div_sum, curl_x, curl_y, curl_z
    float2 *d2;         // pressure-energy flavour only (else null): sum m u W and
                        // the grad-h term times 3 + h n'/n
    float4 *g0;         // force-pass state: h, rho, P, c
    float4 *g1;         // force-pass state: f, balsara, A, 0 (pressure-energy:
                        // f, balsara, F, (gamma - 1)^2 u / P_hat)
    float4 *g2;         // inside a step, the rest of the ghost's outputs: div, curl, converged

    // per leaf
    int32_t *leaf_start;  // n_leaves + 1
    double *leaf_org;     // 3 * n_leaves, FP64 origin (minimum corner of the particles' box)
    float4 *leaf_ext;     // n_leaves: largest FP32 cell-relative x, y, z of the leaf's particles
    float *leaf_hmax;     // n_leaves: gamma_k * largest h of the leaf at the force pass

    // per tree node (all levels)
    double *node_lo;    // 3 * n_nodes
    double *node_hi;    // 3 * n_nodes
    float *node_r;      // search radius of the node (max over its leaves), from tasks build

    double *fsum;       // 6 * (n_leaves + 128 n_sets) FP64 partial sums of the force
                        // pass, then the 128 parts of each set's reduction

    // Independent particle sets in one grid (sphx_grid_build_sets): set b is
    // the caller's particles [set_start[b], set_start[b + 1]), sorted within
    // itself; no leaf holds particles of two sets and no task pairs two sets.
    // One set: n_sets = 1 and the arrays below are null.
    int32_t n_sets;
    int32_t *set_start;  // n_sets + 1, device (the caller's offsets)
    int32_t *set_of;     // n: set of each sorted particle
    int32_t *set_leaf;   // n_sets + 1: first leaf of each set
    int32_t *leaf_set;   // n_leaves: set of each leaf

    // Per-receiver neighbour lists of the h iteration (sorted order). The
    // receivers of 64-block b (sorted indices 64b .. 64b+63) own entries
    // lst[lboff[b] + k * 64 + lane], k < lcnt[s]: every j within lrad[s] of s.
    float *lrad;        // n: list radius (0: no list)
    int32_t *lcnt;      // n: entries
    int64_t *lcap;      // n_blocks + 1: 64 * max entries over the block (scratch)
    int64_t *lboff;     // n_blocks + 1: first entry of each block; [n_blocks] = total
    uint32_t *lst;      // lst_cap entries
    int64_t lst_cap;
    int64_t lst_total;
    void *lscan_tmp;
    size_t lscan_bytes;

    // build scratch
    void *sort_tmp;
    size_t sort_tmp_bytes;
    uint64_t *keys_in;
    int32_t *idx_in;
    uint32_t *flags;
    int32_t *d_status;  // [0] invalid-input count, [1] leaf count
};

struct sphx_tasks {
    sphx_grid *grid;
    uint64_t serial;
    hipStream_t stream;  // the stream of the last build (its memory is freed there)
    int64_t n_tasks;     // tasks held (host copy, as of the last build or captured step)
    int64_t cap;         // task records allocated
    int64_t relayouts;   // new slot layouts so far (the first build's included)
    // Slot layout: leaf I's tasks are task[slot[I], end[I]), inside its slot
    // [slot[I], slot[I + 1]) of kSlotFactor times its count at the last
    // layout + 8 records. Rebuilds walk leaves straight into their slots.
    int32_t *slot;      // n_leaves + 1
    int32_t *end;       // n_leaves (+ 1: scratch of a new layout)
    sphx::Task *task;   // cap
    int32_t *count;     // n_leaves: tasks found by each leaf's last walk
    float *radius;      // per leaf: (1 + skin) * max H at build time
    uint8_t *overflow;  // per leaf: 1 when the serial walk built its list
    uint8_t *dirty;     // per leaf: walked by the current rebuild
    int64_t *state;     // kTaskStateWords device words (kTaskOutgrown, ...)
    void *scan_tmp;
    size_t scan_tmp_bytes;
    // Launch order of the per-leaf loops: the leaves are split into 8
    // contiguous ranges (one per XCD, as xcd_remap) and each range is ordered
    // by decreasing work (sources to load), so that the longest cells start
    // first. order[x * (nbp / 8) + k] = k-th leaf of range x (or >= n_leaves).
    int32_t *order;       // nbp = pad8(n_leaves)
    uint64_t *okey;       // nbp, scratch (sort keys)
    uint64_t *okey_out;   // nbp, scratch
    int32_t *oval;        // nbp, scratch
    void *sort_tmp;
    size_t sort_tmp_bytes;
    int64_t order_cap;
    // Growth rebuilds (tasks_grow) walk only the leaves whose radius grew;
    // the others keep their lists. Such lists serve the density loop (each
    // leaf's list covers its own radius) but can miss a pair that a grown
    // neighbour's radius alone reaches: `symmetric` is false (device copy:
    // state[kTaskAsym] = 1) until the next full build, which the force pass
    // requires.
    bool symmetric;
};

namespace sphx {

// Waits, by polling an event recorded on s, until the work queued on s so far
// (a readback into ctx->h_pinned) has finished.
hipError_t wait_stream(sphx_ctx *ctx, hipStream_t s);

// grid.hip
// sets: null (one set), else n_sets + 1 host offsets (validated by the caller).
sphx_status grid_build(sphx_ctx *ctx, const sphx_particles *in, hipStream_t s, sphx_grid **out,
                       const int64_t *sets = nullptr, int32_t n_sets = 1);
void grid_free(sphx_grid *g);
// Frees the context's spare buffers (recycle_workspace) on their stream.
void release_spares(sphx_ctx *ctx);
sphx_status iter_reset(sphx_grid *g, const sphx_particles *in, hipStream_t s);
sphx_status refresh_h(sphx_grid *g, const sphx_particles *in, hipStream_t s);
size_t grid_bytes(int64_t n);

// tasks.hip
sphx_status tasks_build(sphx_ctx *ctx, sphx_grid *g, const sphx_particles *in, hipStream_t s,
                        sphx_tasks **out);
// Growth rebuild of an existing list for the h iteration's density passes:
// the leaves whose (1 + skin) gamma_k max h grew beyond their list's radius
// are walked again at the current radii, in place, the others keep their
// lists; leaves' radii never shrink here. Leaves the list not symmetric (see
// sphx_tasks). Falls back to tasks_build when there is no layout to walk
// into or a leaf outgrew its slot.
sphx_status tasks_grow(sphx_ctx *ctx, sphx_grid *g, const sphx_particles *in, hipStream_t s,
                       sphx_tasks **out);
// The in-place walks of a growth rebuild and of a full build, for a captured
// step: no readback, no allocation; every kernel returns at once while *run
// is zero. A leaf that outgrows its slot sets state[kTaskOutgrown] (its list
// is then cut short: the caller must not run a loop on it before a
// tasks_build). The list must have a layout (a tasks_build before).
sphx_status tasks_grow_async(const sphx_ctx *ctx, sphx_grid *g, sphx_tasks *t,
                             const int32_t *run, hipStream_t s);
sphx_status tasks_full_async(const sphx_ctx *ctx, sphx_grid *g, sphx_tasks *t,
                             const int32_t *run, hipStream_t s);
// state[kTaskTotal] = the tasks the slots hold (capturable).
sphx_status tasks_total_async(const sphx_grid *g, sphx_tasks *t, hipStream_t s);
void tasks_free(sphx_tasks *t);
// A grid and task list over every particle of `in` with a uniform search
// radius (h = radius / gamma_k on a private array): the pair structure of
// friends-of-friends and direct-summation gravity. Released with the struct.
struct SearchCells {
    sphx_grid *g = nullptr;
    sphx_tasks *t = nullptr;
    float *h = nullptr;
    hipStream_t s = nullptr;
    SearchCells() = default;
    SearchCells(const SearchCells &) = delete;
    SearchCells &operator=(const SearchCells &) = delete;
    ~SearchCells();
};
sphx_status search_cells_build(sphx_ctx *ctx, const sphx_particles *in, double radius,
                               hipStream_t s, SearchCells &sc);
// SPHENIX viscosity switch update, elementwise (alpha_max 2, ell 0.05).
sphx_status alpha_v_launch(const sphx_ctx *ctx, int64_t n, const float *div_old,
                           const float *div_new, const float *c, const float *h,
                           const float *vsig, double dt, float *alpha, hipStream_t s);
// Short-range softened gravity over a grid and tasks built at radius rp2p.
sphx_status gravity_run(sphx_ctx *ctx, const sphx_particles *in, double G, double H, double rs,
                        double rp2p, float *ax, float *ay, float *az, float *pot,
                        int64_t *d_pairs, hipStream_t s);
// Friends-of-friends groups over a grid and tasks built at search radius b.
sphx_status fof_run(sphx_ctx *ctx, const sphx_particles *in, double b, int32_t *group,
                    int32_t *group_size, int64_t *d_counts, hipStream_t s);
size_t tasks_bytes(int64_t n, int leaf_max);

// density.hip
// The probe counters of a measurement build (SPHX_PROBE=1): lane slots of the
// cell-pair loop's neighbour tests, tests by lanes holding a receiver,
// accepted pairs, compute-loop lane slots and the entries they evaluated;
// returns 1 (and zeros) in a product build. Synchronous.
sphx_status probe_read(unsigned long long out[5], bool clear);
// Count the receivers that outgrew their leaf's task radius into *stale
// (added to; a density pass given skip = stale then returns at once).
sphx_status stale_count_launch(const sphx_ctx *ctx, const sphx_grid *g, const sphx_tasks *t,
                               int32_t *stale, hipStream_t s);
// Cell-pair density pass over the receivers that need one; with use_lists,
// only over those whose H exceeds their list radius.
sphx_status density_launch(const sphx_ctx *ctx, const sphx_grid *g, const sphx_tasks *t,
                           const sphx_particles *in, const sphx_density_out *out,
                           int32_t *counters, bool use_lists, hipStream_t s,
                           const int32_t *skip = nullptr);
// List density pass over the receivers that need one and fit their lists.
sphx_status density_list_launch(const sphx_ctx *ctx, const sphx_grid *g, const sphx_tasks *t,
                                const sphx_density_out *out, hipStream_t s);

// lists.hip
// Builds the neighbour lists of every receiver that needs a pass (radius
// min((1 + skin) H, leaf task radius)); *ok = false when the task list is too
// large for list entries (the caller stays on the cell-pair path).
sphx_status list_build(const sphx_ctx *ctx, sphx_grid *g, const sphx_tasks *t, hipStream_t s,
                       bool *ok);
size_t lists_bytes(int64_t n);

// ghost.hip
// step_mode (sphx_step): the caller's h and converged flag are written only
// when a particle is finalised, and the finalising pass also writes the force
// pass's sorted source state (force_launch then runs with state_ready).
sphx_status ghost_launch(const sphx_ctx *ctx, sphx_grid *g, const sphx_tasks *t,
                         sphx_particles *in, const sphx_density_out *d, const sphx_ghost_out *o,
                         int32_t *counters, int final_pass, bool use_lists,
                         unsigned long long *units, hipStream_t s,
                         const int32_t *skip = nullptr, bool step_mode = false);

// force.hip
// fsum_fixed: the FP64 partial sums go to this fixed workspace (6 per leaf,
// then the parts of their reduction) instead of the grid's; the launch then
// creates nothing (no timing events).
sphx_status force_launch(const sphx_ctx *ctx, const sphx_grid *g, const sphx_tasks *t,
                         const sphx_particles *in, const sphx_density_out *d,
                         const sphx_ghost_out *gs, const sphx_force_out *o, double *sums6,
                         hipStream_t s, const int32_t *gate = nullptr,
                         bool state_ready = false, double *fsum_fixed = nullptr);
// The fixed workspace of sphx_force_noalloc on `device` (which must be
// current): its address is looked up once per device and kept.
constexpr int64_t kNoallocLeaves = int64_t(1) << 19;
constexpr int kNoallocMaxDevices = 64;
sphx_status noalloc_scratch(int device, double **out);

// integrate.hip: the gradient loop, the conduction parameter, the step size
// and the leapfrog operators (their scratch is the grid's g2 and leaf_hmax).
sphx_status gradient_launch(const sphx_ctx *ctx, sphx_grid *g, const sphx_tasks *t,
                            const sphx_particles *in, const float *rho, const float *P,
                            float *lap_u, float *vc, float *avmax, hipStream_t s);
// The GDF loop: standalone, into caller-order f and alpha_c (from the
// caller's h and rho); inside a step, into the force state g1 (from g0,
// complete for every particle), gated like the force pass.
sphx_status gdf_launch(const sphx_ctx *ctx, sphx_grid *g, const sphx_tasks *t,
                       const sphx_particles *in, const float *rho, float *f, float *alpha_c,
                       float *D, hipStream_t s);
sphx_status gdf_alpha_v_launch(int64_t n, const float *D_old, const float *D_new,
                               const float *c, const float *h, const float *vsig,
                               const float *B, const uint8_t *active, double dt, float *alpha,
                               hipStream_t s);
sphx_status gdf_step_launch(const sphx_ctx *ctx, const sphx_grid *g, const sphx_tasks *t,
                            const sphx_particles *in, const int32_t *gate, hipStream_t s);
sphx_status alpha_c_launch(const sphx_ctx *ctx, int64_t n, const float *lap_u, const float *u,
                           const float *h, const float *vc, const float *avmax,
                           const uint8_t *active, double dt, float *alpha, hipStream_t s);
sphx_status timestep_launch(const sphx_ctx *ctx, sphx_grid *g, const sphx_tasks *t,
                            const sphx_particles *in, const float *vsig, double c_cfl,
                            double delta, float *dt_out, float *dt_min, hipStream_t s);
sphx_status kick_launch(int64_t n, const float *vx, const float *vy, const float *vz,
                        const float *u, const float *ax, const float *ay, const float *az,
                        const float *du, const uint8_t *active, double dt_half, float *vx_o,
                        float *vy_o, float *vz_o, float *u_o, hipStream_t s);
sphx_status drift_launch(const sphx_ctx *ctx, int64_t n, double *x, double *y, double *z,
                         const float *vx, const float *vy, const float *vz, double dt,
                         hipStream_t s);

// graph.hip
// Captured step: the h iteration's first `passes` passes (none of them the
// final pass of max_iter), the task rebuilds between them, the full rebuild
// before the force pass and a gated force pass as one HIP graph, replayed
// while the handles and arrays stay the same. On return *done = true when
// the step is complete (converged) with force and sums computed; otherwise
// *pass is the number of passes applied, *relayout whether a leaf outgrew its
// slot (the caller must tasks_build before the next loop), *force_pending
// whether the iteration is complete and only the force pass is left (after
// that tasks_build), and the caller continues the iteration from there.
struct StepGraph;
void step_graph_free(StepGraph *g);
sphx_status step_graph_run(sphx_ctx *ctx, sphx_grid *grid, sphx_tasks *t, const sphx_particles *in,
                           const sphx_density_out *dens, const sphx_ghost_out *gst,
                           const sphx_force_out *out, double *sums6, int passes, hipStream_t s,
                           sphx_step_info *info, int *pass, bool *done, bool *relayout,
                           bool *force_pending);

// Blocks are dealt round-robin to the 8 XCDs of the MI355X; remap so that each
// XCD works on a contiguous range of leaves (which share neighbour data in
// that XCD's L2).
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nblocks_padded)
{
    const int64_t per = nblocks_padded >> 3;
    return (b & 7) * per + (b >> 3);
}

// The leaf of block b of a per-leaf loop: the XCD's range as xcd_remap, within
// it the leaves in the task list's decreasing-work order.
__device__ __forceinline__ int64_t leaf_of_block(int64_t b, int64_t nblocks_padded,
                                                 const int32_t *__restrict__ order)
{
    return order[xcd_remap(b, nblocks_padded)];
}

inline int64_t pad8(int64_t n) { return (n + 7) & ~int64_t(7); }

// Grids and task lists allocate their workspace stream-ordered on the stream
// they are built on (no device-wide synchronisation, so requests built on
// different streams overlap) and release it on that stream.
inline hipError_t dmalloc(void **p, size_t bytes, hipStream_t s)
{
    return hipMallocAsync(p, bytes ? bytes : 16, s);
}
inline void dfree(void *p, hipStream_t s)
{
    if (p)
        (void)hipFreeAsync(p, s);
}

}  // namespace sphx
