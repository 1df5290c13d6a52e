/*
 * sphx.h -- C-ABI of the SPH neighbour-loop library for AMD MI355X (gfx950).
 *
 * The library evaluates the data-parallel hot path of smoothed particle
 * hydrodynamics as described in Section 3 of Schaller et al., "SWIFT: A
 * modern highly-parallel gravity and smoothed particle hydrodynamics solver"
 * (arXiv 2305.13380), over self and pair tasks of a spatial cell structure
 * (Section 2.2, "nested grids"):
 *
 *   grid build   Morton sort of the particles and leaf cells (<= leaf_max
 *                particles each, aligned octree blocks), Section 2.2 and the
 *                depth-first binning of Section 9.1;
 *   tasks build  self/pair task list of leaf cells whose bounding boxes are
 *                within a search radius, Section 2.2 and 9.1;
 *   density      number density, its h-derivative, mass density and its
 *                h-derivative, neighbour count, velocity divergence and curl
 *                sums (Section 3.1, "Constructing the number density" and
 *                "Creating general smoothed quantities");
 *   ghost        one Newton-Raphson update of h on n (h/eta)^3 = 1 (Section
 *                3.1), then pressure, sound speed, f-factor, Balsara switch
 *                (Section 3.2) for converged particles;
 *   force        accelerations, du/dt and signal velocity of the density-energy
 *                equations of motion with Balsara-switched artificial
 *                viscosity and artificial conduction (Sections 3.2 and 3.3),
 *                plus FP64 global momentum and energy sums.
 *
 * Conventions shared by every call:
 *   - Device pointers. Every particle and output array is a contiguous device
 *     allocation owned by the caller (structure of arrays, one value per
 *     particle, in the caller's particle order). The library owns only the
 *     opaque handles and their device workspace.
 *   - Streams. `stream` is a hipStream_t (NULL = the default stream). Every
 *     call enqueues work asynchronously; only the calls documented as
 *     synchronising wait for the device.
 *   - Status. 0 = OK, negative = error (nothing useful was produced, the
 *     message is in sphx_last_error()), positive = bit set of warnings
 *     (results are valid).
 *   - Inputs are never written, except h, which sphx_ghost and sphx_step
 *     update in place.
 *   - Threading. A context may be used by one host thread at a time.
 */
#ifndef SPHX_H
#define SPHX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sphx_status;

#define SPHX_OK 0
#define SPHX_E_INVALID (-1)       /* bad argument or non-finite / out-of-range input */
#define SPHX_E_OOM (-2)           /* device allocation failed */
#define SPHX_E_HIP (-3)           /* a HIP runtime call failed */
#define SPHX_E_STATE (-4)         /* handle used out of order (e.g. grid of another ctx) */
#define SPHX_W_NOT_CONVERGED 1    /* some h did not converge within max_iter passes */
#define SPHX_W_H_CLAMPED 2        /* some h were limited to h_max */
#define SPHX_W_REBUILD 4          /* an h outgrew its task list; tasks were (or must be) rebuilt */

/* Method parameters. sphx_params_default() fills the paper's values. */
typedef struct sphx_params {
    double box[3];      /* box edge lengths; particles live in [0, box) */
    int32_t periodic;   /* 1: periodic box (minimum image), 0: open */
    int32_t max_iter;   /* max density passes of the h iteration (default 30) */
    double gamma_k;     /* kernel support H = gamma_k h (Wendland C2: sqrt(15)/2) */
    double eta;         /* smoothing scale of n (h/eta)^3 = 1 (Section 3.1) */
    double h_tol;       /* relative NR tolerance (Section 3.1: 1e-4) */
    double h_max;       /* cap on h; <= 0 selects min(box)/(3 gamma_k)(1-1e-6) */
    double gamma_gas;   /* ratio of specific heats (5/3) */
    double beta_v;      /* signal velocity constant beta (Section 3.2: 3) */
    double eps_balsara; /* Balsara switch regulariser (Section 3.2: 1e-4) */
    double skin;        /* relative enlargement of task search radii (default 0.1) */
    int32_t leaf_max;   /* particles per leaf cell, 8..64 (default 64) */
    int32_t neighbour_lists; /* sphx_step: 1 reuses per-receiver neighbour lists within
                                radius (1 + skin) H over the passes after the first; 0
                                (default) runs the cell-pair loop in every pass */
    /* Loop shapes (0 selects the default; sphx_autotune picks them by timing):
     * candidate-buffer slots per wave and waves per cell of the density loop
     * (64, 128 or 256, default 128; 1 or 2, default 1) and of the force loop
     * (64 or 128, default 64; 1 or 2, default 1). Tile sizes do not change
     * results; the wave count changes the FP32 summation order. */
    int32_t density_tile;
    int32_t density_waves;
    int32_t force_tile;
    int32_t force_waves;
    /* sphx_step: > 0 captures up to graph_passes passes of the h iteration
     * (at most max_iter - 1: the final pass runs uncaptured), the task
     * rebuilds between them (in place, decided on the device), the full
     * rebuild before the force pass and the force pass as one HIP graph
     * (replayed while the handles and arrays stay the same; one readback
     * instead of one per pass). The step continues pass by pass when the
     * iteration needs more passes, or after a rebuild that outgrew the task
     * list's layout. Results are identical to graph_passes = 0 (default 0;
     * not combined with neighbour_lists). */
    int32_t graph_passes;
    /* Density loop: 1 spreads each compute round's pair work evenly over the
     * wave's lanes (lists cut into chunks of one receiver each), 0 (default)
     * lets every lane walk its own list; 2 takes the cell's receivers in
     * groups of up to 16 at each flush of the candidate buffer, each group
     * testing only the candidates near its own bounding box with several
     * lanes per receiver (one wave per cell; the tile then changes the FP32
     * summation order too). Changes the FP32 summation order. */
    int32_t density_balance;
    /* Smoothing kernel (Section 3.1 lists them; one smoothing length h for
     * all, cut-off H = gamma_k h): SPHX_KERNEL_*. Default Wendland C2. Set it
     * with sphx_params_set_kernel, which also sets the kernel's gamma_k. */
    int32_t kernel;
    /* SPH flavour (Section 3.2): SPHX_FLAVOUR_DENSITY_ENERGY (default: the
     * particles carry the internal energy u; Balsara-switched viscosity and
     * artificial conduction) or SPHX_FLAVOUR_DENSITY_ENTROPY (the Gadget2
     * solver: the u array holds the adiabat A, P = A rho^gamma, no
     * conduction, and sphx_force_out.du_dt receives dA/dt = (gamma - 1)
     * rho^(1 - gamma) times the viscous heating rate; the FP64 energy sum
     * keeps the internal-energy rate the forces imply) or SPHX_FLAVOUR_PHANTOM
     * (the Phantom-like flavour of Appendix A: density-energy with alpha_c = 1
     * for every particle, conduction speed sqrt(2 |P_i - P_j| / (rho_i +
     * rho_j)), and the viscosity switch of sphx_alpha_v_update decaying with
     * length 0.25 instead of 0.05) or SPHX_FLAVOUR_PRESSURE_ENERGY
     * (pressure-smoothed SPH of Appendix A: the density loop also forms the
     * smoothed pressure P_hat = (gamma - 1) sum_j m_j u_j W_ij; the ghost
     * returns P = P_hat, c = sqrt(gamma P_hat / rho) and, in
     * sphx_ghost_out.A, the grad-h term F_i of the factors f_ij = 1 - F_i /
     * (m_j u_j); the force pass uses the pressure-energy equation of motion
     * with the density flavours' viscosity and no conduction. Every u must be
     * positive. Runs the plain cell-pair density loop only: sphx_ctx_create
     * refuses it with density_balance != 0 or neighbour_lists != 0) or
     * SPHX_FLAVOUR_ANARCHY_PU (Anarchy-PU of Appendix A: the pressure-energy
     * flavour, with its restrictions, plus conduction with the mean
     * (alpha_c,i + alpha_c,j)/2 and the speed c_i + c_j + mu_ij; in
     * sphx_gradient the same pair speed, in sphx_alpha_c_update beta_c =
     * 0.01 and no shock limiter, in sphx_alpha_v_update the length 0.25) or
     * SPHX_FLAVOUR_GDF (the Gasoline-2-like flavour of Appendix A: the
     * geometric density average force, (P_i + P_j) / (rho_i rho_j) on the
     * mean gradient (f_i W'_i + f_j W'_j) / 2 with the correction f of
     * sphx_gdf in sphx_ghost_out.f, du/dt with P_i alone, the density
     * flavours' viscosity, and the conduction m_j (alpha_c,i + alpha_c,j)
     * (u_i - u_j) G / ((rho_i + rho_j) r) with alpha_c = 0.03 |S| h^2 from
     * the trace-free shear S, carried in sphx_ghost_out.A. sphx_force reads
     * f and alpha_c from *gst; sphx_step forms both after the h iteration
     * and returns them there. The alpha_V evolution of the printed scheme
     * is not part of it). */
    int32_t flavour;
    /* 1: a destroyed grid's device buffers stay with its context and serve
     * the context's next grid build on the same stream (a buffer of between
     * the requested size and twice it); what that build does not take is
     * released at its end, and any rest at sphx_ctx_destroy. For runs that
     * build a new grid of one particle set every step, whose builds then
     * allocate little or nothing. Grids built so must be destroyed before
     * their context, and the stream of the last one destroyed must outlive
     * the context (the buffers it leaves are freed on that stream). Default
     * 0: a grid's buffers are released when it is destroyed. */
    int32_t recycle_workspace;
} sphx_params;

#define SPHX_FLAVOUR_DENSITY_ENERGY 0
#define SPHX_FLAVOUR_DENSITY_ENTROPY 1
#define SPHX_FLAVOUR_PHANTOM 2
#define SPHX_FLAVOUR_PRESSURE_ENERGY 3
#define SPHX_FLAVOUR_ANARCHY_PU 4
#define SPHX_FLAVOUR_GDF 5

#define SPHX_KERNEL_WENDLAND_C2 0
#define SPHX_KERNEL_WENDLAND_C4 1
#define SPHX_KERNEL_WENDLAND_C6 2
#define SPHX_KERNEL_CUBIC_SPLINE 3
#define SPHX_KERNEL_QUARTIC_SPLINE 4
#define SPHX_KERNEL_QUINTIC_SPLINE 5

/* Particle-carried inputs (Section 3.1): positions FP64, the rest FP32. */
typedef struct sphx_particles {
    int64_t n;
    const double *x, *y, *z;
    const float *vx, *vy, *vz;
    const float *m;        /* mass */
    const float *u;        /* internal energy per unit mass */
    float *h;              /* smoothing length; read, and updated by ghost/step */
    const float *alpha_v;  /* per-particle viscosity coefficient alpha_V,i */
    const float *alpha_c;  /* per-particle conduction coefficient alpha_c,i */
    const uint8_t *active; /* NULL: all active; else receivers are those with 1 */
} sphx_particles;

/* Density-pass outputs (caller order, FP32 unless noted). Sums include the
 * self term; nngb excludes it. div_sum/curl_* are the raw sums
 * sum_j m_j (v_j - v_i).grad_i W_ij and sum_j m_j grad_i W_ij x (v_j - v_i).
 * P_hat, P_hat_dh: with SPHX_FLAVOUR_PRESSURE_ENERGY, the smoothed pressure
 * (gamma - 1) sum_j m_j u_j W_ij and its h-derivative (Appendix A); NULL:
 * not written (always ignored by the other flavours). */
typedef struct sphx_density_out {
    float *rho, *rho_dh, *n, *n_dh;
    float *div_sum, *curl_x, *curl_y, *curl_z;
    int32_t *nngb;
    float *P_hat, *P_hat_dh;
} sphx_density_out;

/* Ghost outputs (caller order). converged: 1 once h has converged. */
typedef struct sphx_ghost_out {
    float *f, *P, *c, *balsara, *A, *div_v, *curl_v;
    uint8_t *converged;
} sphx_ghost_out;

/* Force outputs (caller order). nforce may be NULL. */
typedef struct sphx_force_out {
    float *ax, *ay, *az, *du_dt, *v_sig;
    int32_t *nforce;
} sphx_force_out;

/* Counters in a caller-provided device array of 4 int32, zeroed by the caller
 * before each density pass: [0] particles still unconverged after the ghost,
 * [1] particles whose new H exceeds their leaf's task radius (rebuild the
 * tasks before the next pass), [2] particles finalised at h_max, [3]
 * receivers of the density pass whose H exceeded the task radius. */
#define SPHX_COUNTERS 4

/* Result of sphx_step. */
typedef struct sphx_step_info {
    int32_t passes;            /* density passes run */
    int32_t task_rebuilds;     /* task-list rebuilds during the iteration */
    int32_t unconverged;       /* particles not converged after max_iter */
    int32_t clamped;           /* particles at h_max */
    int64_t n_leaves;
    int64_t n_tasks;
    int32_t list_builds;       /* neighbour-list builds during the iteration */
    int32_t list_fallback;     /* receiver passes that outgrew their list (cell-pair loop) */
    int64_t list_entries;      /* entries of the last list build (with block padding) */
    int64_t pairs_cellpair;    /* density interactions (self excluded) computed by the
                                  cell-pair loop over all passes */
    int64_t pairs_list;        /* ... and by the neighbour-list loop */
    int32_t captured_passes;   /* passes (of `passes`) run inside the captured graph
                                  (graph_passes > 0); the rest ran pass by pass */
    int32_t task_relayouts;    /* rebuilds (of task_rebuilds) that laid the task
                                  slots out anew: a leaf outgrew its slot */
} sphx_step_info;

typedef struct sphx_ctx sphx_ctx;
typedef struct sphx_grid sphx_grid;
typedef struct sphx_tasks sphx_tasks;

/* Fill *p with the defaults: unit periodic box, Wendland C2 kernel with
 * gamma_k = sqrt(15)/2, eta = 1.2348, h_tol = 1e-4, max_iter = 30,
 * gamma_gas = 5/3, beta_v = 3, eps_balsara = 1e-4, skin = 0.1,
 * leaf_max = 64, h_max automatic. */
void sphx_params_default(sphx_params *p);

/* Select the smoothing kernel `kernel` (SPHX_KERNEL_*, Section 3.1) and set
 * p->gamma_k to its cut-off ratio H/h for h = twice the kernel's standard
 * deviation (the convention that keeps h, and so eta, the same for every
 * kernel): sqrt(15/4), sqrt(39/8), sqrt(6), sqrt(10/3), sqrt(375/92),
 * sqrt(135/28) in the order of the constants. Other fields are left as they
 * are (an automatic h_max follows gamma_k). E_INVALID for an unknown kernel,
 * *p unchanged. */
sphx_status sphx_params_set_kernel(sphx_params *p, int32_t kernel);

/* Create a context on HIP device `hip_device` (makes it current for the
 * calling thread). Validates *p: E_INVALID for non-positive box, eta, h_tol,
 * max_iter, gamma_k, leaf_max outside 8..64, or an unknown kernel. *out is owned by the caller
 * and released with sphx_ctx_destroy. */
sphx_status sphx_ctx_create(const sphx_params *p, int hip_device, sphx_ctx **out);
void sphx_ctx_destroy(sphx_ctx *ctx);

/* Estimate of the device bytes a grid plus its tasks take for n particles
 * (used to admit requests against an HBM budget): one leaf per leaf_max / 4
 * particles with 96 tasks each, held in their slots (four times the count +
 * 8 per leaf). Boxes clustered into far more tasks per particle take more.
 * Host only, no device call. */
size_t sphx_workspace_bytes(const sphx_params *p, int64_t n);

/* Grid build (Section 2.2 cells, Section 9.1 binning): validates the inputs
 * on the device (E_INVALID on non-finite positions, positions outside
 * [0, box) for open boxes, h <= 0, h > h_max or non-finite, m <= 0, u < 0),
 * sorts the
 * particles by 63-bit Morton key of their FP64 position, splits the sorted
 * order into leaf cells (maximal aligned octree blocks with <= leaf_max
 * particles), and stores per leaf its FP64 origin and extent and per
 * particle its FP32 position relative to its leaf origin. Positions,
 * velocities, masses, u and alpha are copied at this point; later changes to
 * them need a new grid. Synchronises the stream (reads back the leaf count).
 * The workspace is allocated stream-ordered on `stream` and released on it
 * by sphx_grid_destroy, which must be called before that stream is destroyed.
 * *out is released with sphx_grid_destroy. */
sphx_status sphx_grid_build(sphx_ctx *ctx, const sphx_particles *in, void *stream,
                            sphx_grid **out);

/* Grid build over several independent particle sets at once, for batching
 * small requests into one step (the serving loop's batches): set b is the
 * particles [set_start[b], set_start[b + 1]) of *in, each set a box of the
 * context's size and periodicity of its own. Each set is sorted and split
 * into leaves on its own (no leaf holds two sets), and tasks built on this
 * grid pair leaves of one set only, so every density, ghost and force output
 * of a set is bitwise the one a grid of that set alone gives. A step's or
 * force pass's d_sums6 then receives 6 sums per set (set b's at
 * d_sums6[6 b]). set_start: host array of n_sets + 1 offsets from 0 to
 * in->n, non-decreasing (empty sets allowed); n_sets 1..65536; read before
 * the call returns. Otherwise as sphx_grid_build; E_INVALID on bad offsets.
 * sphx_force_noalloc refuses such grids with more than one set. */
sphx_status sphx_grid_build_sets(sphx_ctx *ctx, const sphx_particles *in,
                                 const int64_t *set_start, int32_t n_sets, void *stream,
                                 sphx_grid **out);
void sphx_grid_destroy(sphx_grid *grid);

/* Tasks build (Section 2.2 self and pair tasks): for every leaf, the list of
 * leaves (with periodic shift) whose bounding box lies within
 * max(H_i-leaf, H_j-leaf) * (1 + skin) of its own, H taken from the current
 * h. Each task carries the FP32 offset between the two leaf origins, formed
 * in FP64. Each leaf's tasks sit in a slot of its own, sized four times its
 * task count at the last layout + 8; a rebuild walks every leaf into its slot
 * and lays the slots out anew only when a leaf outgrew its own. Synchronises
 * the stream (reads back the task count). *out is released with
 * sphx_tasks_destroy (on the stream of its last build, which must still
 * exist). Calling it again with an existing *out rebuilds in place. */
sphx_status sphx_tasks_build(sphx_ctx *ctx, sphx_grid *grid, const sphx_particles *in,
                             void *stream, sphx_tasks **out);
void sphx_tasks_destroy(sphx_tasks *tasks);

/* Start an h iteration: mark every active particle as needing a density pass
 * and clear each particle's bracket of the root (the safeguard of the
 * Newton-Raphson step in sphx_ghost). sphx_grid_build does this too.
 * Asynchronous. */
sphx_status sphx_iter_reset(sphx_ctx *ctx, sphx_grid *grid, const sphx_particles *in,
                            void *stream);

/* Density pass (Section 3.1) at the current h for every particle marked as
 * needing one: writes the sums of sphx_density_out for those particles only.
 * The task list must cover every marked particle's H (true right after
 * sphx_tasks_build with the current h). A marked particle whose H exceeds its
 * leaf's task radius is counted in d_counters[3] (if d_counters != NULL); its
 * sums are then incomplete and the tasks must be rebuilt. Asynchronous. */
sphx_status sphx_density(sphx_ctx *ctx, const sphx_grid *grid, const sphx_tasks *tasks,
                         const sphx_particles *in, sphx_density_out *out, int32_t *d_counters,
                         void *stream);

/* Ghost (Section 3.1 NR update; Sections 3.1-3.2 EOS, f-factor, Balsara): for
 * every particle marked as needing a pass, one Newton-Raphson step of h on
 * F(h) = n h^3 - eta^3 from the sums of the last sphx_density pass on this
 * grid (the values it wrote to *dens, also kept in the grid's workspace in
 * sorted order, together with the h they were evaluated at); the step is
 * limited to [h/2, 2h] and h_max. A particle whose step is below h_tol*h is
 * converged: it keeps that h, its ghost outputs are written and its mark is
 * cleared. Otherwise its h (caller array) is replaced by the new value,
 * unless final_pass != 0, in which case it keeps its h, its ghost outputs are
 * written and it is reported unconverged. Adds to d_counters (see
 * SPHX_COUNTERS; may be NULL). Does nothing when d_counters[3] > 0 (the
 * preceding density pass ran on a stale task list). Asynchronous. */
sphx_status sphx_ghost(sphx_ctx *ctx, sphx_grid *grid, const sphx_tasks *tasks,
                       sphx_particles *in, const sphx_density_out *dens, sphx_ghost_out *out,
                       int32_t *d_counters, int32_t final_pass, void *stream);

/* Force pass (Sections 3.2-3.3) for every active particle, over all j != i
 * with r_ij < max(H_i, H_j). Reads the ghost state (rho from *dens; f, P, c,
 * balsara from *gst, and A with SPHX_FLAVOUR_PRESSURE_ENERGY, where P is the
 * smoothed pressure and A the grad-h term F) of every particle, including
 * inactive ones. If
 * d_sums6 != NULL it receives, in FP64, sum m a (3), sum m (v.a + du/dt),
 * sum m |a|, sum m |du/dt| over the active particles (per set, 6 each, on a
 * grid of several sets). Asynchronous. */
sphx_status sphx_force(sphx_ctx *ctx, const sphx_grid *grid, const sphx_tasks *tasks,
                       const sphx_particles *in, const sphx_density_out *dens,
                       const sphx_ghost_out *gst, sphx_force_out *out, double *d_sums6,
                       void *stream);

/* sphx_force with no allocation of any kind, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels, arguments, outputs and
 * bits as sphx_force, but the FP64 partial sums of the conservation sums
 * (6 per leaf cell plus 128 parts of their reduction) live in a fixed
 * device array of the library (25.2 MB per device, set aside by the HIP
 * runtime when the library's code is loaded on the device, at the first
 * sphx_ctx_create there, and held until the process ends) instead of the grid's
 * workspace, no kernel timing events are created, and an empty set clears
 * d_sums6 with a kernel (no memset). Limit: grids of at most 524,288 leaf
 * cells (about 20 M particles at the default leaf size); a larger grid is
 * refused with E_INVALID before anything is enqueued. Every call on one
 * device shares that array, so calls that overlap on one device (other
 * streams, other host threads, other contexts) race: serialise them.
 * Asynchronous. */
sphx_status sphx_force_noalloc(sphx_ctx *ctx, const sphx_grid *grid, const sphx_tasks *tasks,
                               const sphx_particles *in, const sphx_density_out *dens,
                               const sphx_ghost_out *gst, sphx_force_out *out, double *d_sums6,
                               void *stream);

/* One step on an existing grid: the h iteration (density + ghost passes
 * until every active particle has converged or max_iter passes ran; the task
 * list is rebuilt in place whenever an h outgrows its task radius, and a
 * density pass that ran on a stale list is repeated), then the force pass and
 * the FP64 sums. *tasks is built first if NULL (release it with
 * sphx_tasks_destroy). Synchronises the stream once per density pass run
 * pass by pass and once per task rebuild there, and once for the captured
 * part (graph_passes). *info may be NULL. Warnings: W_NOT_CONVERGED,
 * W_H_CLAMPED. */
sphx_status sphx_step(sphx_ctx *ctx, sphx_grid *grid, sphx_tasks **tasks, sphx_particles *in,
                      sphx_density_out *dens, sphx_ghost_out *gst, sphx_force_out *out,
                      double *d_sums6, void *stream, sphx_step_info *info);

/* Autotuner: times each density-loop shape (tile x waves with per-lane
 * rounds, and tiles with grouped rounds; the balanced rounds are not among
 * them) over whole steps (as sphx_step, pass
 * by pass, from the particles' current h, iterating on a device copy of h;
 * the time of the step's density launches, HIP events around each), and each
 * force-loop shape on force passes at the converged state; the shortest of
 * reps timed runs (after one untimed run) counts, events on `stream`. The
 * context's kernel statistics (sphx_profile_*) are left as they were.
 * Returns in *tuned the context's parameters with the fastest shapes. The
 * output arrays are overwritten; h is not changed; the task list is left as
 * a build at the current h leaves it. Allocates n floats for the copy of h.
 * Contexts created from *tuned give identical results to each other, so a
 * caller that needs the same results from several contexts (a server's
 * slots) tunes once and creates all of them from *tuned. Synchronises the
 * stream. */
sphx_status sphx_autotune(sphx_ctx *ctx, sphx_grid *grid, sphx_tasks *tasks, sphx_particles *in,
                          sphx_density_out *dens, sphx_ghost_out *gst, sphx_force_out *out,
                          int32_t reps, sphx_params *tuned, void *stream);

/* Friends-of-friends groups (Section 9.1): particles i and j are linked when
 * they lie closer than the linking length b, decided in FP64 on the caller's
 * positions as |x_i - x_j|^2 < b^2 (minimum image in a periodic box; the
 * squared distance formed as (dx dx + dy dy) + dz dz, each operation rounded
 * on its own); groups are the connected components of the links, found by
 * union-find over the self and pair tasks of a cell structure built with b
 * as its search radius (ctx's leaf_max and skin apply).
 *   in         every particle takes part (in->active and in->h are ignored,
 *              h may be NULL); the other per-particle arrays are read by the
 *              cell build but do not change the groups.
 *   b          0 < b <= min(box)/3 (1 - 1e-5), else E_INVALID.
 *   group      device, n int32, caller order: the smallest caller index of
 *              the particle's group (so group[i] == i marks one particle of
 *              each group). Required when n > 0.
 *   group_size device, n int32, or NULL: the number of particles in i's group.
 *   d_counts   device, 2 int64, or NULL: [0] number of groups, [1] number of
 *              linked pairs.
 * Results do not depend on scheduling. Allocates its workspace on `stream`
 * and synchronises once (the task build reads back its size). */
sphx_status sphx_fof(sphx_ctx *ctx, const sphx_particles *in, double b, int32_t *group,
                     int32_t *group_size, int64_t *d_counts, void *stream);

/* Short-range softened gravity by direct summation (Section 4.1: the C2
 * softened potential and force; Section 4.4: the short-range truncation of
 * the mesh split). For a pair at separation r (minimum image):
 *   phi(r) = f(r/H)/H for r < H, else 1/r, with the printed
 *            f(u) = -3u^7 + 15u^6 - 28u^5 + 21u^4 - 7u^2 + 3;
 *   phi'(r)/r = g(r/H)/H^3 for r < H, else -1/r^3, g(u) = f'(u)/u;
 *   chi(r) = erfc(r / (2 r_s)) (1 when r_s = 0: no truncation);
 *   a_i = G sum_j m_j x_ij [phi'(r) chi(r) + phi(r) chi'(r)] / r (the exact
 *   gradient of the truncated potential), pot_i = -G sum_j m_j phi(r) chi(r),
 *   over j != i with r_ij < r_p2p: the pairs a tree code sums directly (the
 *   multipole and mesh parts of the force are not computed here).
 *   G > 0; H > 0 is the softening kernel's support (3 eps_Plummer); r_s >= 0;
 *   0 < r_p2p <= min(box)/3 (1 - 1e-5); else E_INVALID.
 *   ax, ay, az (device, n FP32 each, caller order) required when n > 0;
 *   pot (device, n FP32) or NULL; d_pairs (device, 1 int64) or NULL: the
 *   number of directed pairs summed.
 * Every particle receives (in->active and in->h are ignored, h may be NULL;
 * the other per-particle arrays are read by the cell build). Pair arithmetic
 * in FP32 on cell-relative coordinates; the r < r_p2p test is taken in FP32
 * too. Allocates its workspace on `stream` and synchronises once (the task
 * build reads back its size). */
sphx_status sphx_gravity(sphx_ctx *ctx, const sphx_particles *in, double G, double H,
                         double r_s, double r_p2p, float *ax, float *ay, float *az, float *pot,
                         int64_t *d_pairs, void *stream);

/* SPHENIX viscosity switch (Section 3.3), per particle i < n (caller order,
 * device FP32 arrays of n): from the velocity divergence at the start and at
 * the end of a step of length dt (div_old, div_new, e.g. sphx_ghost_out.div_v
 * of two steps), the shock indicator S = H^2 max(0, -(div_new - div_old)/dt)
 * with H = gamma_k h, and the target alpha_loc = 2 S / (v_sig^2 + S) (0 where
 * S = 0; alpha_max = 2), alpha_v becomes alpha_loc if that is larger, else
 * alpha_loc + (alpha_v - alpha_loc) exp(-ell c dt / H) (decay length ell =
 * 0.05, or 0.25 with the Phantom-like and Anarchy-PU flavours; the printed
 * update is read as this decay towards the target). alpha_v is read and
 * written in place; c is the sound speed (sphx_ghost_out.c), h the
 * smoothing length, v_sig the signal velocity (sphx_force_out.v_sig).
 * dt > 0 and finite, n >= 0, else E_INVALID. Asynchronous on `stream`. */
sphx_status sphx_alpha_v_update(sphx_ctx *ctx, int64_t n, const float *div_old,
                                const float *div_new, const float *c, const float *h,
                                const float *v_sig, double dt, float *alpha_v, void *stream);

/* SPHENIX gradient loop (Section 3.3), after a step on this grid and task
 * list (the tasks must cover every active particle's H, as sphx_step leaves
 * them). For every active particle i, over the particles j != i with
 * 0 < r_ij < H_i (FP32 arithmetic in the cell frame, like the density pass):
 *   lap_u[i]       = 2 sum_j (m_j / rho_j) (u_i - u_j) (dW/dr)(r_ij, h_i) / r_ij,
 *                    the Laplacian of u that drives the conduction parameter
 *                    (Brookshaw's second-derivative estimator; the paper names
 *                    the Laplacian without printing an estimator);
 *   v_c[i]         = max_j |v_ij . x_ij| / r_ij + sqrt(2 |P_i - P_j| / (rho_i + rho_j)),
 *                    the largest pair conduction speed (0 without neighbours;
 *                    SPHX_FLAVOUR_ANARCHY_PU: max_j c_i + c_j + min(0, v_ij .
 *                    x_ij) / r_ij with c = sqrt(gamma P / rho));
 *   alpha_v_max[i] = the largest alpha_V among i and those j (the shock
 *                    limiter's input).
 * Reads positions, velocities, masses and u of the grid (as copied at its
 * build), and h, alpha_v (in), rho, P (device, caller order, n FP32 each:
 * e.g. sphx_density_out.rho and sphx_ghost_out.P) of every particle. Outputs:
 * device FP32 arrays of n in caller order, written for active particles only.
 * Uses the grid's scratch (not safe concurrently with another call on the
 * same grid). Asynchronous. */
sphx_status sphx_gradient(sphx_ctx *ctx, sphx_grid *grid, const sphx_tasks *tasks,
                          const sphx_particles *in, const float *rho, const float *P,
                          float *lap_u, float *v_c, float *alpha_v_max, void *stream);

/* The GDF flavour's per-particle quantities (Appendix A), for every active
 * receiver i over the j with r_ij < H_i (W_ij = W(r_ij, h_i); FP32 arithmetic
 * in the cell frame):
 *   f[i]       = (S1 / rho_i) / S2, S1 = sum_j m_j r_ij^2 W_ij,
 *                S2 = sum_j (m_j / rho_j) r_ij^2 W_ij (the geometric density
 *                average correction of the force law);
 *   alpha_c[i] = 0.03 |S| h_i^2, S the trace-free symmetric part of
 *                V_ab = sum_j (v_a,i - v_a,j)(x_b,i - x_b,j) m_j W_ij / (S1 / 3)
 *                and |S| the square root of its summed squares (the paper
 *                prints the plain sum; the root gives alpha_c the dimension
 *                of a diffusivity).
 * D != NULL also receives the shock detector of the flavour's viscosity switch,
 *   D[i]       = 3/2 [n_i . V_i . n_i + max(-tr V_i / 3, 0)], n_i the direction
 *                of grad P_i = (gamma - 1) sum_j m_j u_j grad_i W_ij (n.V.n = 0
 *                without a gradient; D = 0 without neighbours at r > 0).
 * A receiver with no neighbour at r > 0 gets f = 1 and alpha_c = 0. Reads
 * positions, velocities and masses of the grid (as copied at its build), and
 * h (in) and rho (device, caller order, n FP32: e.g. sphx_density_out.rho)
 * of every particle, and u of the grid for D. Outputs: device FP32 arrays of
 * n in caller order, written for active particles only (for
 * SPHX_FLAVOUR_GDF's force pass, sphx_ghost_out.f and .A). Any flavour may
 * call it. Uses the grid's scratch (not safe concurrently with another call
 * on the same grid). Asynchronous. */
sphx_status sphx_gdf(sphx_ctx *ctx, sphx_grid *grid, const sphx_tasks *tasks,
                     const sphx_particles *in, const float *rho, float *f, float *alpha_c,
                     float *D, void *stream);

/* The GDF flavour's viscosity switch over a step dt (Appendix A), per active
 * particle i < n (active NULL: all): with dD/dt = (D_new - D_old) / dt from
 * the detector of sphx_gdf at the start and end of the step,
 *   A_i = 2 h_i^2 B_i max(-dD/dt, 0),  alpha_loc = 2 A_i / (A_i + v_sig,i^2)
 * (alpha_V,max = 2, SPHENIX's; B the Balsara switch); alpha_v rises to
 * alpha_loc at once where that is larger (as the SPHENIX switch does) and
 * otherwise relaxes towards it by d alpha/dt = 0.2 c_i (alpha_loc - alpha) /
 * h_i, integrated exactly over the step. Device FP32 arrays of n; alpha_v is
 * updated in place. Asynchronous. */
sphx_status sphx_gdf_alpha_v_update(sphx_ctx *ctx, int64_t n, const float *D_old,
                                    const float *D_new, const float *c, const float *h,
                                    const float *v_sig, const float *balsara,
                                    const uint8_t *active, double dt, float *alpha_v,
                                    void *stream);

/* SPHENIX conduction parameter over a step dt (Section 3.3), per active
 * particle i < n (active NULL: all): the evolution equation
 *   d alpha_c / dt = beta_c H lap_u / sqrt(u) - (alpha_c - alpha_c,min) v_c / H
 * (H = gamma_k h; beta_c = 1, alpha_c,min = 0 as printed) has constant
 * coefficients over the step and is integrated exactly (alpha_inf + (alpha -
 * alpha_inf) exp(-v_c dt / H), alpha_inf = alpha_c,min + S H / v_c with
 * S = beta_c H lap_u / sqrt(u); alpha + S dt where v_c = 0), then capped by
 * the shock limiter at alpha_c,max (1 - alpha_v_max / alpha_V,max) (1 and 2
 * as printed) and kept >= 0 (SPHX_FLAVOUR_ANARCHY_PU, Appendix A: beta_c =
 * 0.01 and the plain cap alpha_c <= 1). Inputs from sphx_gradient (lap_u, v_c,
 * alpha_v_max) and the particles (u, h); alpha_c is updated in place.
 * Device FP32 arrays of n, caller order. dt > 0 and finite, n >= 0, else
 * E_INVALID. Asynchronous. */
sphx_status sphx_alpha_c_update(sphx_ctx *ctx, int64_t n, const float *lap_u, const float *u,
                                const float *h, const float *v_c, const float *alpha_v_max,
                                const uint8_t *active, double dt, float *alpha_c, void *stream);

/* Time-step sizes (Section 3.4): every particle's CFL step
 * dt_cfl = c_cfl H / v_sig (H = gamma_k h, v_sig the force pass's signal
 * velocity; the paper names the condition without printing it), then for
 * every active particle the first limiter: dt[i] = min(dt_cfl,i, delta
 * min_j dt_cfl,j) over the particles j != i with r_ij < max(H_i, H_j) (the
 * force-loop neighbours; delta = 4 in the paper). dt (device FP32, n, caller
 * order) is written for active particles; d_dt_min (device, 1 FP32, or NULL)
 * receives the smallest of them (+inf when none is active), the step of a
 * run with one global step. 0 < c_cfl, 1 <= delta, both finite, else
 * E_INVALID. Uses the grid's scratch. Asynchronous. */
sphx_status sphx_timestep(sphx_ctx *ctx, sphx_grid *grid, const sphx_tasks *tasks,
                          const sphx_particles *in, const float *v_sig, double c_cfl,
                          double delta, float *dt, float *d_dt_min, void *stream);

/* Leapfrog half kick (Section 2.4, kick-drift-kick): for every active
 * particle i < n (active NULL: all), v_out = v + a dt_half, u_out = u +
 * du_dt dt_half (device FP32 arrays of n, caller order; the outputs may be
 * the inputs, for an update in place, or other arrays, for the prediction of
 * v and u at the end of a drift). Asynchronous. */
sphx_status sphx_kick(sphx_ctx *ctx, int64_t n, const float *vx, const float *vy,
                      const float *vz, const float *u, const float *ax, const float *ay,
                      const float *az, const float *du_dt, const uint8_t *active, double dt_half,
                      float *vx_out, float *vy_out, float *vz_out, float *u_out, void *stream);

/* Leapfrog drift (Section 2.4): x += v dt for every particle, in FP64 on the
 * caller's position arrays (updated in place), wrapped into [0, box) in a
 * periodic box. A grid built before the drift no longer matches: build a
 * new one. Asynchronous. */
sphx_status sphx_drift(sphx_ctx *ctx, int64_t n, double *x, double *y, double *z,
                       const float *vx, const float *vy, const float *vz, double dt,
                       void *stream);

/* Kernel timing for measurement tools. sphx_profile_enable(ctx, 1) clears the
 * statistics and starts recording a pair of HIP events around every launch of
 * the cell-pair density kernel (kernel 0), the force kernel (kernel 1), the
 * list density kernel (kernel 2), the neighbour-list build (kernel 3: its
 * counting pass with the offset scan, and its filling pass) and the gravity
 * loop of sphx_gravity (kernel 4), on the stream
 * the kernel is launched on; 0 stops recording. sphx_profile_read
 * waits for the recorded events and returns the summed kernel time in
 * milliseconds and the number of launches since the last enable. */
sphx_status sphx_profile_enable(sphx_ctx *ctx, int32_t enable);
sphx_status sphx_profile_read(sphx_ctx *ctx, int32_t kernel, double *total_ms, int64_t *launches);

/* Neighbour-loop counters of a measurement build of the library (built with
 * SPHX_PROBE=1; product builds count nothing and return 1 with zeros): since
 * the last clear, counts5[0] = lane slots taken by the candidate tests of the
 * cell-pair density loop (per-lane rounds), [1] = those tests made by lanes
 * holding a receiver, [2] = accepted pairs (each receiver's own particle
 * included), [3] = lane slots of its per-lane compute loops (64 lanes x 4
 * entries per round), [4] = list entries those loops evaluated. clear != 0
 * zeroes them after reading. Synchronous. */
sphx_status sphx_probe_read(sphx_ctx *ctx, uint64_t *counts5, int32_t clear);

/* Leaf and task counts of a grid / task list (host values). */
int64_t sphx_grid_leaves(const sphx_grid *grid);
int64_t sphx_tasks_count(const sphx_tasks *tasks);

/* Message of the last error on the calling thread ("" if none). */
const char *sphx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPHX_H */
