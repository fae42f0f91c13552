/*
 * dnslab.h - C ABI of an MI355X (gfx950) library for one explicit projection
 * time step of the incompressible Navier-Stokes equations with a passive
 * scalar and a binary immersed-boundary mask, after Korhonen et al.,
 * arXiv 2204.02107 (Sections 2.1, 2.2 and 2.4).
 *
 * What one step computes (Section 2.1 unless noted):
 *   1. dt from a maximum Courant number (Section 2.4), or a fixed dt;
 *   2. classical RK4 of the momentum equation without the pressure gradient,
 *      second-order central differences, skew-symmetric convection, viscous
 *      term, relaxation forcing S (u_set - u)/tau_f and body force b, all
 *      multiplied by the mask beta;
 *   3. the immersed-boundary pressure iteration of Section 2.2: n_piter FFT
 *      solves of  Lap p^{k+1} = div u* + div((1 - beta) grad p^k), warm-started
 *      from the previous step's pressure, with the central-difference symbol
 *      lambda(m) = -sum_a sin^2(2 pi m_a / N_a) / dx_a^2 (zero on the modes
 *      whose every m_a is 0 or N_a/2);
 *   4. the correction u = beta (u* - grad p);
 *   5. classical RK4 of the passive scalar (flux-form convection with the
 *      projected velocity frozen, masked diffusion alpha_c div(beta grad c),
 *      relaxation forcing), then c = beta c;
 *   6. optionally the sixth-order explicit filter f + pi^-6 sum_a delta6_a f on
 *      u, v, w and c, followed by the mask;
 *   7. FP64 diagnostics (kinetic energy, divergence norm, CO2 mass, room-mean
 *      CO2, Courant number).
 *
 * Conventions for every entry point:
 *   - Device pointers are caller-owned, contiguous, structure-of-arrays, x
 *     fastest: cell (i, j, k) is element i + nx*(j + ny*k).
 *   - Field element type ("field type" below): double for DNSLAB_FP64, float
 *     for DNSLAB_FP32_REFINE, for all of u, v, w, p and c.
 *   - All work is enqueued on params.stream (a hipStream_t; NULL = the null
 *     stream) and is asynchronous, except where an entry point says it
 *     synchronises.
 *   - Return value 0 on success, a negative DNSLAB_E* code otherwise.  On an
 *     argument or state error nothing is enqueued.  No C++ exception crosses
 *     this interface.  dnslab_last_error() gives a message.
 *   - One context per stream; a context is not thread-safe.  The context owns
 *     only its workspace, device memory it obtains through params.alloc (the
 *     caller's allocator, e.g. PyTorch's caching allocator) or, when that is
 *     NULL, with hipMalloc; it returns every block through params.free_ (or
 *     hipFree) after synchronising the streams that used it.  The bound state
 *     buffers stay owned by the caller and must outlive the context.
 *   - Units are SI; the scalar is a plain number (ppm in the room cases).
 */
#ifndef DNSLAB_H
#define DNSLAB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DNSLAB_OK            0
#define DNSLAB_EINVAL       -1   /* bad argument (NULL pointer, bad size, bad parameter) */
#define DNSLAB_ENOMEM       -2   /* device allocation failed */
#define DNSLAB_EUNSUPPORTED -3   /* grid size not of the form 2^a 3^b, or too large */
#define DNSLAB_EHIP         -4   /* a HIP runtime call failed */
#define DNSLAB_ESTATE       -5   /* call not valid in the current state */
#define DNSLAB_EAGAIN       -6   /* pool: not enough HBM budget left right now */
#define DNSLAB_ENONFINITE   -7   /* a diagnostic came out NaN or Inf */

typedef enum { DNSLAB_FP64 = 0, DNSLAB_FP32_REFINE = 1 } dnslab_precision;

typedef struct dnslab_ctx dnslab_ctx;     /* opaque */
typedef struct dnslab_pool dnslab_pool;   /* opaque */

/* Case parameters (the paper's case-setup script, Section 2.4). */
typedef struct {
    int32_t nx, ny, nz;     /* cells; nx = 2^a 3^b with a >= 1 and nx >= 4; ny, nz = 1 or
                               2^a 3^b >= 2; nx <= 4096 and ny, nz <= 2048 in FP64
                               (8192 and 4096 in FP32); fewer than 2^31 cells */
    double lx, ly, lz;      /* periodic box lengths [m]; dx = lx/nx etc. */
    double nu;              /* kinematic viscosity [m^2/s] */
    double alpha_c;         /* scalar diffusivity [m^2/s] */
    double tau_f;           /* forcing relaxation time [s] (> 0) */
    double body[3];         /* body-force acceleration b [m/s^2] */
    double cfl;             /* maximum Courant number sum_a |u_a| dt / dx_a */
    double dt_fixed;        /* > 0: fixed time step; otherwise dt from cfl */
    double u_ref;           /* Courant denominator floor u_ref / min(dx) (> 0 if adaptive) */
    int32_t n_piter;        /* immersed-boundary pressure iterations per step (paper: 4) */
    int32_t filter;         /* 1: sixth-order filter at the end of each step */
    int32_t precision;      /* dnslab_precision */
    void* stream;           /* hipStream_t for all work of this context */
    int32_t project_each_stage;  /* 1: project after every RK4 stage as well as at the end of
                               the step (the alternative Section 2.1 mentions and the paper
                               skips for speed: 4 projections per step, fourth order in
                               time); 0: the paper's single projection per step */
    /* Device memory of the context (workspace, list of cells next to a solid,
     * particle-sort scratch, histogram counters).  alloc(bytes, alloc_user)
     * returns a block of at least bytes device bytes, 256-byte aligned, on the
     * current device, or NULL when it cannot (the call then fails with
     * DNSLAB_ENOMEM; a misaligned block is returned through free_ and counts
     * as a failure); free_(ptr, alloc_user) takes it back.  Called only from
     * the thread that calls the library, never from a stream callback.  Both
     * NULL: hipMalloc / hipFree.  One NULL and the other not: DNSLAB_EINVAL. */
    void* (*alloc)(size_t bytes, void* alloc_user);
    void (*free_)(void* ptr, void* alloc_user);
    void* alloc_user;
} dnslab_params;

/* Per-step diagnostics, all FP64. */
typedef struct {
    double t;               /* simulated time after the step */
    double dt;              /* time step taken */
    double ke;              /* 1/2 sum beta |u|^2 dV after the step */
    double div_l2;          /* sqrt(sum (div u)^2 dV) of the projected velocity */
    double co2_mass;        /* sum beta c dV after the step */
    double co2_room_mean;   /* sum_R beta c / sum_R beta (R = room mask, or all cells) */
    double cfl_max;         /* dt * max sum_a |u_a|/dx_a over the start-of-step velocity */
    int64_t step;           /* steps taken since init / set_state */
} dnslab_diag;

/* Bytes of device workspace a context with these parameters allocates (for
 * HBM-budget admission), not counting the list of cells next to a solid that
 * dnslab_init builds from the mask (at most 13 bytes per such cell).
 * Host-only; enqueues nothing. */
int dnslab_workspace_bytes(const dnslab_params* params, size_t* out_bytes);

/* Create a context bound to caller-owned state buffers u, v, w, p, c (device,
 * nx*ny*nz elements each, types per precision).  beta_dev: uint8 mask, 1 fluid,
 * 0 solid (Section 2.1).  The forcing region S (Section 2.1, eq. tanh) is given
 * sparse: n_forced sorted unique flat indices, S in (0, 1], u_set [3*n] as
 * (x,y,z) triples and c_set [n], all device arrays (may be NULL if n_forced is
 * 0).  room_mask_dev: uint8 region of the room-mean diagnostic, NULL = all
 * cells.  The mask and forcing arrays are copied; the state buffers are kept.
 * Synchronises the stream (computes the first time step). */
int dnslab_init(const dnslab_params* params, const uint8_t* beta_dev,
                int64_t n_forced, const int64_t* forced_idx_dev, const double* forced_S_dev,
                const double* forced_uset_dev, const double* forced_cset_dev,
                const uint8_t* room_mask_dev,
                void* u, void* v, void* w, void* p, void* c,
                dnslab_ctx** out);

/* Advance the bound state by nsteps full steps (items 1-7 above).  If diag is
 * non-NULL the call synchronises and fills it with the last step's values;
 * then it returns DNSLAB_ENONFINITE if any diagnostic of the steps is not
 * finite. */
int dnslab_step(dnslab_ctx* ctx, int32_t nsteps, dnslab_diag* diag);

/* Copy the diagnostics of the last n steps (n <= 4096, oldest first) into
 * out[0..n-1].  Synchronises. */
int dnslab_read_diags(dnslab_ctx* ctx, int32_t n, dnslab_diag* out);

/* One FFT solve of the pressure equation of Section 2.2 without the mask
 * term: p = Lap^-1 rhs with the central-difference symbol, null modes set to
 * zero.  rhs_dev and p_dev: device, nx*ny*nz elements of the field type; they
 * may alias. */
int dnslab_poisson(dnslab_ctx* ctx, const void* rhs_dev, void* p_dev);

/* Size of the static device scratch of dnslab_poisson_noalloc (64 MiB). */
#define DNSLAB_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve of
 * dnslab_poisson without a context.  Grid, lengths, precision and stream come
 * from params (which must pass the same checks as for dnslab_init; the other
 * fields are ignored); rhs_dev and p_dev are as for dnslab_poisson and may
 * alias.  The spectrum and the FFT tables (computed on the device each call)
 * live in a static device array of DNSLAB_NOALLOC_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends; the call
 * allocates nothing and synchronises nothing.  A grid whose spectrum and
 * tables exceed that size (the spectrum takes 16 * ceil16(nx/2+1) * ny * nz
 * bytes in FP64, half in FP32: 256x128x192 fits in FP64, 256x256x128 does
 * not) returns DNSLAB_EINVAL before anything is enqueued.  Every call on one GPU uses the
 * same array: calls that overlap on one GPU (other streams, other threads)
 * race and must be ordered by the caller.  Errors are reported through
 * dnslab_last_error(NULL). */
int dnslab_poisson_noalloc(const dnslab_params* params, const void* rhs_dev, void* p_dev);

/* The projection of Section 2.2 applied in place to the velocity u*, v*, w*
 * (device, field type): n_piter immersed-boundary iterations warm-started from
 * the bound pressure p (which is updated), then u = beta (u* - grad p).  In
 * DNSLAB_FP32_REFINE the last pressure solve is refined once in FP64: its
 * residual is formed in FP64 from the FP32 fields, a correction is solved for,
 * and the velocity correction is applied in FP64 arithmetic. */
int dnslab_project(dnslab_ctx* ctx, void* u, void* v, void* w);

/* One RK4 step of the scalar (item 5) of length dt with the bound velocity
 * frozen; updates the bound c in place. */
int dnslab_scalar_step(dnslab_ctx* ctx, double dt);

/* Momentum right-hand side F(u) of item 2 (without pressure), written to
 * fu, fv, fw (device, field type).  Inputs are not modified. */
int dnslab_momentum_rhs(dnslab_ctx* ctx, const void* u, const void* v, const void* w,
                        void* fu, void* fv, void* fw);

/* Scalar right-hand side G(c; u) of item 5 written to out (device, field type). */
int dnslab_scalar_rhs(dnslab_ctx* ctx, const void* c, const void* u, const void* v,
                      const void* w, void* out);

/* Masked sixth-order filter (item 6) of one field: out = beta (f + pi^-6 sum_a
 * delta6_a f).  f and out must not alias. */
int dnslab_filter(dnslab_ctx* ctx, const void* f, void* out);

/* Re-read the bound state after the caller changed it (recomputes the Courant
 * time step; resets t and the step counter to the given values).  Synchronises. */
int dnslab_set_time(dnslab_ctx* ctx, double t, int64_t step);

/* Release the workspace.  Synchronises the stream first.  NULL is a no-op. */
void dnslab_destroy(dnslab_ctx* ctx);

/* Message of the last error on ctx; with ctx = NULL the last error of this
 * thread (for failed dnslab_init calls).  Never NULL. */
const char* dnslab_last_error(const dnslab_ctx* ctx);

/* Lagrangian particles (Section 2.3): drag du_p/dt = (C_d/tau_p)(u_f - u_p) + g
 * with tau_p = rho_p d^2 / (18 rho_f nu) (d the diameter), Re_p = |u_f - u_p| d/nu,
 * C_d = 1 + Re_p^(2/3)/6, one-way coupled to the bound velocity (trilinear
 * interpolation of the cell values, cell (i, j, k) at (i dx, j dy, k dz),
 * periodic).  Implicit Euler with C_d from the start of the step:
 * u_p' = (u_p + dt (C_d/tau_p) u_f + dt g) / (1 + dt C_d/tau_p), x' = x + dt u_p',
 * wrapped into the periodic box. */
typedef struct {
    double rho_p;           /* particle density [kg/m^3] */
    double rho_f;           /* fluid density [kg/m^3] */
    double g[3];            /* gravitational acceleration [m/s^2] */
} dnslab_particle_params;

/* Advance n particles by one step on the context's stream.  pos and vel are
 * device FP64 arrays of 3n values, structure of arrays (x[0..n), y[0..n),
 * z[0..n)), updated in place; diam holds n diameters [m].  dt > 0 is the step;
 * dt <= 0 takes the time step of the last dnslab_step (read on the device, no
 * synchronisation).  Call after dnslab_step to move the particles with the new
 * velocity.  DNSLAB_EINVAL for n < 0, n >= 2^40, NULL arrays with n > 0, or
 * non-positive densities. */
int dnslab_particles_step(dnslab_ctx* ctx, int64_t n, double* pos, double* vel, const double* diam,
                          const dnslab_particle_params* pp, double dt);

/* Reorder n particles (same arrays as dnslab_particles_step; diam is
 * permuted too) by the linear index i + nx (j + ny k) of the cell holding
 * each one, cell (i, j, k) = floor(x / dx) etc. wrapped into the grid, with a
 * stable sort: particles in one cell keep their relative order, so the result
 * is unique.  Particles carry no identity in the model (Section 2.3), so the
 * order is free; sorted particles gather their fluid velocities from
 * neighbouring cells, which the step kernel turns into coalesced reads.  On
 * the context's stream; allocates device scratch on first use and when n
 * grows (then synchronises the stream first).  The sort is a stable radix
 * sort on the bits the cell count needs (8 per pass).  0 <= n <= 2^28, else
 * DNSLAB_EINVAL. */
int dnslab_particles_sort(dnslab_ctx* ctx, int64_t n, double* pos, double* vel, double* diam);

/* CO2 distribution over the room (Section 3.3): counts of the fluid cells of
 * the room region per bin of the bound c, nbins equal bins over [lo, hi)
 * (bin floor((c - lo) / (hi - lo) * nbins) in FP64, clamped into the end
 * bins).  counts_host receives nbins values.  1 <= nbins <= 4096 and lo < hi,
 * else DNSLAB_EINVAL.  Synchronises the stream. */
int dnslab_co2_histogram(dnslab_ctx* ctx, int32_t nbins, double lo, double hi, int64_t* counts_host);

/* Running sums for time averages: sums_dev (FP64 device array of 5 n values,
 * field-major u, v, w, p, c) += the bound fields.  Asynchronous. */
int dnslab_accumulate(dnslab_ctx* ctx, double* sums_dev);

/* Force of the fluid on an obstacle (Section 3.1.1, Table 2: drag
 * coefficient and Strouhal number of the obstacle in the channel), per unit
 * density.  The obstacle is the set of solid cells (beta = 0) inside the index
 * box i0 <= i < i1, j0 <= j < j1, k0 <= k < k1 (box = {i0, i1, j0, j1, k0,
 * k1}, each range non-empty and inside the grid, else DNSLAB_EINVAL).
 * Pressure part: -dV sum over the obstacle cells of the central gradient of
 * P = p / dt (the bound p holds dt times the kinematic pressure, the
 * correction being u = u* - grad p): the obstacle's share of the momentum the
 * pressure gradient takes from the fluid, equal to face pressures averaged
 * over the two cells of each face.  Viscous part: every face between an
 * obstacle cell and a fluid cell adds nu u_f A / dx_a (A the face area), the
 * flux of the masked second difference into the solid cell.  out_dev (device,
 * 8 doubles, caller-owned) receives Fp_x, Fp_y, Fp_z, Fv_x, Fv_y, Fv_z, then
 * the simulated time t and the dt of the last step.  Asynchronous on the
 * stream; one block walks the box, so the sum is reproducible bit for bit and
 * the call suits obstacle-sized boxes. */
int dnslab_body_force(dnslab_ctx* ctx, const int32_t box[6], double* out_dev);

/* Kernel timing for roofline measurements: when enabled, every launch of the
 * named kernel ("mom_stage", "scalar_stage", "fft_x_fwd", "fft_y", "fft_z", "fft_yz",
 * "fft_x_inv", "filter", "filter_c", "correct", "div", "ib_rhs", "advance",
 * "diag", "refine_res", "particles") is bracketed by HIP events on the stream it is
 * launched on, and the total and count accumulate (kernel_name NULL: off).
 * Steps are issued launch by launch while a kernel is profiled.  Read
 * synchronises. */
int dnslab_profile_enable(dnslab_ctx* ctx, const char* kernel_name);
int dnslab_profile_read(dnslab_ctx* ctx, double* total_ms, int64_t* launches);

/* Issue dnslab_step's work as replays of a HIP graph that holds k whole steps
 * (captured on the first call that needs it; steps beyond a multiple of k are
 * issued launch by launch).  The graph's launches are those of k calls of
 * dnslab_step(ctx, 1) and compute the same results bit for bit; replay takes
 * one host call per k steps instead of one per kernel, which matters for small
 * grids.  k = 0 turns it off (the default).  Needs a stream other than the
 * legacy default stream (NULL): returns DNSLAB_EINVAL otherwise, or for k < 0
 * or k > 4096. */
int dnslab_set_graph_steps(dnslab_ctx* ctx, int32_t k);

/* enable = 1 (the default): the scalar half of a step (scalar RK4, its filter
 * and the diagnostics record) runs on a second stream of the context beside
 * the next step's velocity work, as the data dependences allow, except for
 * FP64 grids of 2^26 cells or more, whose steps stay on one stream (there
 * that is faster).  0: every launch of a step runs in order on the context's
 * stream (for timing kernels alone).  Results are bitwise the same either
 * way.  Enqueues any deferred scalar work first.  DNSLAB_EINVAL unless enable
 * is 0 or 1. */
int dnslab_set_overlap(dnslab_ctx* ctx, int32_t enable);

/* RK4 stages two per pass (Section 2.1's stages carry no pressure, so a
 * kernel can evaluate the first stage of a pair on its tile and a one-cell
 * ring and the second on the tile, reading and writing the fields once per
 * pair).  mode -1 (the default): by grid size (where each block's z chunk is
 * long enough to pay for the pipeline's extra planes); 0: never (one kernel
 * per stage); 1: wherever the 64 x 8 tile divides the grid (nx % 64 == 0,
 * ny % 8 == 0).  The scalar's pairs also need the filter on.  Results agree
 * to rounding (every value is computed with the same expressions).  Enqueues
 * any deferred scalar work first.  DNSLAB_EINVAL unless mode is -1, 0 or 1. */
int dnslab_set_stage_pairs(dnslab_ctx* ctx, int32_t mode);

/* Column passes of the FFT solve (Section 2.2) with the next tile's load in
 * flight while the current tile is transformed (each block walks several
 * tiles, moving them into LDS with asynchronous loads).  mode -1 (the
 * default): the library's choice (currently never: one tile per block
 * measured faster on the grids tried); 0: never; 1: wherever the pass
 * applies (row-major spectrum, plain launches, transform lengths 64 to 1024
 * of the form 2^a 3^b with a compiled chain).  Same arithmetic either way:
 * results are bitwise the same.
 * Enqueues any deferred scalar work first.  DNSLAB_EINVAL unless mode is -1,
 * 0 or 1. */
int dnslab_set_fft_pipeline(dnslab_ctx* ctx, int32_t mode);

/* ------------------------------------------------------------------------
 * Serving pool: many scenarios of different grid sizes resident at once,
 * admitted against an HBM budget and advanced together.  Each step of the
 * pool issues, for every kernel of the step sequence, one batched launch over
 * all active scenarios (scenarios with identical launch sequences share a
 * launch); every scenario computes exactly what dnslab_step would compute for
 * it alone, so its result is independent of the mix.  The pool owns the
 * scenarios' device memory.  All pool calls use the pool's stream; a pool is
 * not thread-safe.
 * ------------------------------------------------------------------------ */

/* Create an empty pool with hbm_budget bytes of device memory, all scenarios
 * of the given precision, working on stream.  The budget covers each
 * scenario's state and workspace plus a 64 KiB share of the batched launch
 * tables, and the device staging buffer of admission (kept between
 * admissions, sized for the largest one so far).  alloc, free_, alloc_user:
 * the allocator of every device block the pool and its scenarios use, with
 * the meaning of the dnslab_params fields of the same names (both NULL:
 * hipMalloc / hipFree; the allocators in admitted params are ignored). */
int dnslab_pool_create(size_t hbm_budget, int32_t precision, void* stream, void* (*alloc)(size_t, void*),
                       void (*free_)(void*, void*), void* alloc_user, dnslab_pool** out);

/* Admit a scenario that will run target_steps steps.  All arrays are HOST
 * memory with the layouts of dnslab_init (initial fields in FP64, converted to
 * the pool precision); params->precision must equal the pool's and
 * params->stream is ignored.  Returns DNSLAB_EAGAIN, with nothing allocated,
 * when the scenario's memory does not fit in what is left of the budget.
 * Synchronises the pool's stream.  *slot_out receives the slot id. */
int dnslab_pool_admit(dnslab_pool* pool, const dnslab_params* params, int64_t target_steps,
                      const uint8_t* beta_host, int64_t n_forced, const int64_t* forced_idx_host,
                      const double* forced_S_host, const double* forced_uset_host,
                      const double* forced_cset_host, const uint8_t* room_mask_host,
                      const double* u0_host, const double* v0_host, const double* w0_host,
                      const double* p0_host, const double* c0_host, int32_t* slot_out);

/* Advance every admitted scenario that has not reached its target by up to
 * nsteps steps (asynchronous; scenarios stop at their own target). */
int dnslab_pool_step(dnslab_pool* pool, int32_t nsteps);

/* enable = 1: replay each pool step from a HIP graph of its batched launches,
 * captured again whenever the set of running scenarios changes (same
 * results; one host call per step).  0: launch by launch (the default).
 * Needs a pool stream other than NULL (DNSLAB_EINVAL otherwise). */
int dnslab_pool_set_graph(dnslab_pool* pool, int32_t enable);

/* Progress of a slot: the last step's diagnostics (zeros before the first
 * step), steps taken and whether the target is reached.  Synchronises. */
int dnslab_pool_query(dnslab_pool* pool, int32_t slot, dnslab_diag* last, int64_t* steps_done,
                      int32_t* done);

/* Copy field 0..4 (u, v, w, p, c) of a slot to host memory as FP64
 * (nx*ny*nz values).  Synchronises. */
int dnslab_pool_read_field(dnslab_pool* pool, int32_t slot, int32_t field, double* host_out);

/* Free a slot's memory and return it to the budget.  Synchronises. */
int dnslab_pool_release(dnslab_pool* pool, int32_t slot);

/* Bytes of the budget in use, scenarios still running, scenarios resident. */
int dnslab_pool_usage(dnslab_pool* pool, size_t* bytes_in_use, int32_t* active, int32_t* resident);

/* Message of the last error on pool (NULL: this thread's last error).  Never NULL. */
const char* dnslab_pool_last_error(const dnslab_pool* pool);

/* Release every slot and the pool.  NULL is a no-op. */
void dnslab_pool_destroy(dnslab_pool* pool);

#ifdef __cplusplus
}
#endif
#endif /* DNSLAB_H */
