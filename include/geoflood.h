/*
 * geoflood.h -- C ABI of the MI355X shallow-water patch library.
 *
 * The library advances the 2D shallow-water equations with bathymetry and
 * Manning friction (Kyanjo, Calhoun & George, GeoFlood v1.0.0, Section 3.1,
 * eq. (shallow) and eq. (manning)) by the wave-propagation finite-volume
 * method with an augmented Riemann solver, limited second-order corrections
 * and transverse waves (Section 3.2, eqs. (wpa_update) and
 * (wpa_update_corrections); Section 3.3), on a forest of quadtrees of
 * fixed-size logically Cartesian patches (Section 4), with ghost cells filled
 * from same-level, coarser and finer neighbours (Figure 1).
 *
 * Conventions shared by every entry point
 *   - Every function returns GF_OK (0) or a negative GF_E_* status; a NULL
 *     context gives GF_E_INVALID.  gf_last_error() describes the last failure.
 *   - Host pointers are owned by the caller, read or written before the call
 *     returns, and never kept.  The library owns all device memory it uses.
 *   - All device work runs on the stream given at creation (NULL = the null
 *     stream).  Functions that return host values synchronise that stream.
 *   - One host thread at a time per context.
 *   - Cell arrays are interior cells of one patch, row-major (j outer),
 *     m x m values, FP64 at the ABI; an FP32 context rounds on the way in
 *     (round to nearest even) and widens on the way out.
 *   - Leaves of a scenario are ordered: trees row-major, then Z-order (x the
 *     low bit) of each patch's lower-left corner within its tree.  A leaf is
 *     described by 4 int32: (tree, level, ix, iy), ix, iy < 2^level.
 *   - Fields: 0 depth h, 1 x-momentum hu, 2 y-momentum hv, 3 bed b.
 */
#ifndef GEOFLOOD_H
#define GEOFLOOD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gf_ctx gf_ctx;

enum {
    GF_OK = 0,
    GF_E_INVALID = -1,     /* bad argument or configuration                      */
    GF_E_NOMEM = -2,       /* device or host allocation failed / pool too small  */
    GF_E_HIP = -3,         /* a HIP runtime call failed                           */
    GF_E_STATE = -4,       /* call out of order (e.g. step before bathymetry)    */
    GF_E_CFL = -5,         /* a fixed step exceeded cfl_max; state kept at the last accepted step */
    GF_E_NUMERIC = -6,     /* NaN/Inf produced; state kept at the last accepted step */
    GF_E_UNSUPPORTED = -7  /* option not built (e.g. patch size)                 */
};

enum { GF_FP64 = 0, GF_FP32 = 1 };                     /* arithmetic of a context */
enum { GF_BC_WALL = 0, GF_BC_EXTRAP = 1, GF_BC_INFLOW = 2 };
enum { GF_TAG_PLAIN = 0, GF_TAG_LEARNED = 1 };         /* gf_tag modes */

/* One independent scenario (an ensemble member).  Sides: 0 x-low, 1 x-high,
 * 2 y-low, 3 y-high. */
typedef struct {
    double x0, y0, x1, y1;       /* domain */
    int32_t mi, mj;              /* trees in x and y (Section 4: m_i x m_j blocks) */
    int32_t min_level, max_level;
    double manning_n;            /* eq. (manning); 0 disables friction */
    int32_t bc[4];               /* GF_BC_* per side */
    int32_t inflow_side;         /* side carrying the inflow segment, or -1 */
    double inflow_lo, inflow_hi; /* segment along that side (Section 5.1.1) */
    const double *hydro;         /* n_hydro pairs (t [s], Q [m^3/s]), piecewise linear; copied */
    int32_t n_hydro;             /* <= 16 */
    double tag_h_refine;         /* depth refine threshold H_r [m] */
    double tag_eta_refine;       /* free-surface difference threshold E_r [m] */
    double t_end;                /* stop time; steps are truncated to reach it */
    /* Further refinement criteria of Section 4.1.  A wet cell also meets the
     * refine criteria where its speed max(|u|, |v|) exceeds tag_u_refine
     * (tested as max(|hu|, |hv|) > U h) or max(|hu|, |hv|) exceeds
     * tag_q_refine (velocity-depth product); 0 turns either off.  Arrays are
     * copied at gf_create and may be freed after it. */
    double tag_u_refine;         /* speed threshold [m/s], >= 0 */
    double tag_q_refine;         /* velocity-depth product threshold [m^2/s], >= 0 */
    int32_t n_regions;           /* flood-source regions, <= 4 */
    const double *regions;       /* n_regions x 6: x0 y0 x1 y1 min_level max_level; a leaf
                                  * overlapping a region is refined below its min level,
                                  * never refined at or above its max level, and never
                                  * coarsened at or below its min level (largest over
                                  * the regions it overlaps) */
    int32_t n_grades;            /* flow grades, <= 4 */
    const double *grades;        /* n_grades x 3: quantity (0 depth, 1 speed), threshold,
                                  * level; a leaf with a wet cell above a grade's
                                  * threshold is taken to the largest such level */
} gf_scenario_desc;

typedef struct {
    int32_t precision;           /* GF_FP64 or GF_FP32 */
    int32_t m;                   /* cells per patch side: 16 or 32 */
    double g;                    /* gravity, 9.81 */
    double dry_tol;              /* wet/dry threshold tau: dry iff h <= tau (1e-4 m) */
    double cfl_desired;          /* target Courant number of the adaptive step (0.9) */
    double cfl_max;              /* steps above this Courant number are rejected (1.0) */
    int32_t n_scen;
    const gf_scenario_desc *scen;
    int64_t max_patches;         /* patch pool capacity over all scenarios */
    void *hip_stream;            /* hipStream_t or NULL */
    const char *autotune_cache;  /* nullable: cache file gf_autotune uses when its own path is NULL;
                                  * copied at gf_create */
    int32_t limiter;             /* limiter of the f-wave corrections (Section 3.2, eq.
                                  * (wpa_update_corrections), limiters that keep the scheme
                                  * TVD): GF_LIMITER_MC (0, the default), _MINMOD, _SUPERBEE,
                                  * _VANLEER, or _NONE (first order: no corrections) */
    int32_t transverse;          /* the 2D extension of Section 3.2: GF_TRANSVERSE_CORRECTED
                                  * (0, the default: each cell's net normal increment,
                                  * corrections included, split into the other direction's
                                  * fluxes) or GF_TRANSVERSE_NONE (no transverse terms; stable
                                  * only to a Courant number of about 0.5) */
} gf_config;

enum { GF_LIMITER_MC = 0, GF_LIMITER_MINMOD = 1, GF_LIMITER_SUPERBEE = 2, GF_LIMITER_VANLEER = 3, GF_LIMITER_NONE = 4 };
enum { GF_TRANSVERSE_CORRECTED = 0, GF_TRANSVERSE_NONE = 1 };

typedef struct {
    int64_t steps;               /* accepted steps over all scenarios in this call */
    int64_t rejected;            /* rejected (retried) steps in this call */
    int64_t cell_updates;        /* interior leaf cells x accepted steps */
    double t_min, t_max;         /* scenario times after the call */
    double dt_min, dt_max;       /* next step lengths after the call */
    double cfl_max;              /* largest Courant number of the accepted steps of the call */
    double seconds;              /* wall time of the call, the final synchronisation included */
} gf_step_stats;

/* Create a context: validates the configuration and allocates the patch
 * pool (state double-buffered, bathymetry, halo tables) on the device.
 * Errors: GF_E_INVALID (bad m, levels, domain), GF_E_NOMEM, GF_E_HIP. */
int gf_create(const gf_config *cfg, gf_ctx **out);
void gf_destroy(gf_ctx *ctx);

/* Bathymetry of scenario `scen` from terrain node values at the corners of
 * the level-`dem_level` cells: dem_nodes[j * nx + i], nx = mi*m*2^dem_level+1,
 * ny = mj*m*2^dem_level+1.  Cell values integrate the bilinear interpolant of
 * the nodes (Section 6.2, integral-preserving topography): at levels >=
 * dem_level the interpolant's cell average, below it the mean of the four
 * children.  Errors: GF_E_INVALID on shape mismatch. */
int gf_set_bathymetry(gf_ctx *ctx, int32_t scen, const double *dem_nodes, int64_t nx, int64_t ny,
                      int32_t dem_level);

/* Initial state from a host callback (the initial condition of an IVP on
 * the quadtree, Section 4; Section 5.1 and 6.2 set theirs this way: a dry
 * start, or a reservoir over the terrain).  For every leaf of scenario
 * `scen`, in leaf order, the library calls
 *   ic(user, scen, level, x0, y0, dx, dy, m, m, b, h, hu, hv)
 * with (x0, y0) the leaf's lower-left corner, (dx, dy) its cell size, b its
 * m*m interior bed values as the library holds them (FP32 contexts: the
 * rounded bed, widened), and h, hu, hv m*m arrays (row-major, j outer) that
 * the callback fills; the library then stores them (rounded to nearest even
 * in an FP32 context).  Then, up to max_passes times: the plain criteria
 * tag the scenario's leaves (other scenarios are left alone), the mesh is
 * regridded with those flags, and the callback sets the new leaves again;
 * a pass that changes no leaf ends the loop.  The callback runs on the
 * calling thread and must not call into the library.  Clocks and budgets of
 * the scenario restart at t = 0.
 * Errors: GF_E_INVALID (null callback, max_passes < 0), GF_E_STATE (no
 * bathymetry or leaves), GF_E_NOMEM (pool too small for a pass). */
typedef void (*gf_ic_fn)(void *user, int32_t scen, int32_t level, double x0, double y0, double dx, double dy,
                         int32_t nx, int32_t ny, const double *b, double *h, double *hu, double *hv);
int gf_set_initial(gf_ctx *ctx, int32_t scen, gf_ic_fn ic, void *user, int32_t max_passes);

/* Replace the mesh of a scenario by the given leaves (n rows of 4 int32, any
 * order; stored in leaf order).  The leaves must tile the domain and be 2:1
 * balanced across faces and corners.  State is zeroed; bathymetry is set.
 * Errors: GF_E_INVALID (not a balanced tiling), GF_E_NOMEM (pool), GF_E_STATE
 * (no bathymetry yet). */
int gf_set_leaves(gf_ctx *ctx, int32_t scen, const int32_t *tlxy, int64_t n);
/* Leaves of a scenario in leaf order; *n receives the count (also when cap is
 * too small, which returns GF_E_INVALID). */
int gf_get_leaves(gf_ctx *ctx, int32_t scen, int32_t *tlxy, int64_t cap, int64_t *n);

/* One field of one leaf (interior, m*m values).  Fields 0..2 settable, 0..3
 * readable. */
int gf_set_patch(gf_ctx *ctx, int32_t scen, int64_t leaf, int32_t field, const double *in);
int gf_get_patch(gf_ctx *ctx, int32_t scen, int64_t leaf, int32_t field, double *out);
/* Whole scenario at once: n_leaves x 3 x m x m values (h, hu, hv per leaf). */
int gf_set_state(gf_ctx *ctx, int32_t scen, const double *in);
/* n_leaves x 4 x m x m values (h, hu, hv, b per leaf). */
int gf_get_state(gf_ctx *ctx, int32_t scen, double *out);

/* Fill the ghost layers (2 cells) of every leaf of every scenario at the
 * current time, as the step does internally: same-level copies, averages of
 * finer neighbours, limited interpolation from coarser neighbours, then the
 * physical rules (wall mirror, extrapolation, inflow from eq. (riemann) /
 * eq. (2-shock)).  The result is kept for gf_get_ghosted. */
int gf_fill_ghosts(gf_ctx *ctx);
/* (m+4)^2 values of one field of one leaf after gf_fill_ghosts, row-major,
 * the first row being ghost row -2. */
int gf_get_ghosted(gf_ctx *ctx, int32_t scen, int64_t leaf, int32_t field, double *out);

/* Advance every scenario by nsteps accepted steps (or to its t_end).
 * dt_fixed == NULL: adaptive steps, dt_{n+1} = dt_n cfl_desired / nu_n with
 * nu the largest Courant number over all edges and levels; a step with
 * nu > cfl_max is rejected and retried with dt cfl_desired / nu; the first
 * step of a scenario comes from a speed-only pass.  dt_fixed != NULL: step k
 * of this call uses dt_fixed[k] in every scenario, and nu > cfl_max returns
 * GF_E_CFL.  Ghost filling, the update, friction, positivity and refluxing
 * at coarse/fine faces all run inside.  `out` is nullable. */
int gf_step(gf_ctx *ctx, int32_t nsteps, const double *dt_fixed, gf_step_stats *out);
/* The same steps by the plain path, the comparator for gf_step: per attempt,
 * for every scenario and level one launch filling the ghosted tiles in device
 * memory ((m+4)^2 cells x 4 fields per leaf), one launch updating each patch
 * from its ghosted tile, then the largest Courant number of each scenario
 * read back to the host, which accepts or rejects and chooses dt with the
 * same arithmetic (Sections 3.2-3.3, eq. (wpa_update), eq. (manning)).
 * Results equal gf_step's bit for bit; arguments, statistics and errors are
 * as for gf_step.  The ghosted tiles stay readable with gf_get_ghosted. */
int gf_step_plain(gf_ctx *ctx, int32_t nsteps, const double *dt_fixed, gf_step_stats *out);

/* Local time stepping across levels (the subcycling of ForestClaw, Section
 * 2.1.3, on which GeoFlood builds; the paper gives no scheme, so this is the
 * Berger-Oliger form): nsteps accepted macro steps, each the
 * step of the coarsest level present; level l takes 2^(l - L0) substeps of
 * it, fine ghosts read their coarser neighbours halfway through a coarse step
 * as the mean of the coarse states before and after, fine face fluxes are
 * summed over the substeps for refluxing, and a macro step is rejected (and
 * redone, shorter) when the largest Courant number of any of its substeps
 * exceeds cfl_max.  dt_fixed (nullable) gives each macro step's length.
 * Every kernel of gf_step serves; work per macro step is the sum over leaves
 * of m^2 2^(level - L0) cell updates, which out->cell_updates counts.  Gauges
 * record once per macro step.  Errors as for gf_step (state kept at the last
 * accepted macro step). */
int gf_step_lts(gf_ctx *ctx, int32_t nsteps, const double *dt_fixed, gf_step_stats *out);

/* Refinement flags of every leaf of every scenario, concatenated in scenario
 * then leaf order: +1 refine, -1 coarsen, 0 keep (Section 4.1).
 * mode GF_TAG_PLAIN, the criteria of Section 4.1, in order: the cell
 * criteria (depth, free-surface gradient, advancing front, speed,
 * velocity-depth product) refine at their thresholds and keep at half of
 * them, else the leaf coarsens; flow grades that hold set the leaf's level;
 * flood-source regions force or cap it; the scenario's level limits apply
 * last.  Decided in FP64 with * + - and compares only.
 * mode GF_TAG_LEARNED: the network's flags, as gf_net_predict (needs
 * parameters: GF_E_STATE otherwise).
 * `flags_out` is nullable (the flags are kept for gf_regrid).
 * Errors: GF_E_INVALID (mode, cap < leaf count), GF_E_STATE. */
int gf_tag(gf_ctx *ctx, int32_t mode, int8_t *flags_out, int64_t cap, int64_t *n);

/* Gauges: the time series at control points that Section 5.1 plots.  Point k
 * (scenario scen[k], x = xy[2k], y = xy[2k+1], inside its domain) reads the
 * leaf cell holding it: cell floor((x - x0)/dx), floor((y - y0)/dy) at the
 * leaf's level (the last cell for a point on the far edge), found again after
 * every mesh change.  Each accepted step of gf_step or gf_step_plain appends
 * (t, h, hu, hv, b) of that cell after refluxing, up to `cap` records per
 * gauge; later records are counted, not kept.  Replaces earlier gauges and
 * clears their records; n = 0 removes them.  Errors: GF_E_INVALID (n above
 * 256, a point outside its domain, cap < 1), GF_E_NOMEM/GF_E_HIP. */
int gf_set_gauges(gf_ctx *ctx, int32_t n, const int32_t *scen, const double *xy, int64_t cap);
/* Records of gauge g, oldest first: up to cap_out rows of 5 doubles
 * (t, h, hu, hv, b) into out; *n receives the number of records taken so far
 * (which may exceed what was kept). */
int gf_get_gauges(gf_ctx *ctx, int32_t g, double *out, int64_t cap_out, int64_t *n);

/* Apply flags (NULL: those of the last gf_tag): refine, close under 2:1
 * face+corner balance, coarsen complete families whose parent stays
 * balanced; refinement by one level at a time (Section 4: no skipped
 * levels).  Moves the data conservatively.  *n_leaves (nullable) receives
 * the new total leaf count. */
int gf_regrid(gf_ctx *ctx, const int8_t *flags_in, int64_t *n_leaves);

/* Mass budget of a scenario: water volume sum(h dx dy) (compensated sum in
 * leaf order), the volume added by resetting negative depths to zero, and the
 * net volume that entered through non-wall physical boundaries. */
int gf_mass(gf_ctx *ctx, int32_t scen, double *mass, double *clamp_volume, double *boundary_volume);

/* The same mass budget for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): it
 * calls no hipMalloc, hipFree or other allocating routine.  The per-patch
 * partial volumes and the three results go to a static device array of
 * 65536 + 64 doubles (512.5 KiB), one per GPU, held until the process ends;
 * the sums are formed on the device in the same order and with the same
 * operations as gf_mass, so the results equal gf_mass's bit for bit.  Every
 * call on one GPU uses that GPU's array: calls that overlap on one GPU (other
 * threads, other streams) race and must be serialised by the caller.
 * Errors: GF_E_INVALID (more than 65536 patches over all scenarios of the
 * context, bad scenario), GF_E_STATE (the mesh changed and no entry point has
 * rebuilt its tables since: gf_step, gf_tag or gf_mass do), GF_E_HIP. */
int gf_mass_static(gf_ctx *ctx, int32_t scen, double *mass, double *clamp_volume, double *boundary_volume);

/* Clock of a scenario. */
int gf_time(gf_ctx *ctx, int32_t scen, double *t, double *dt_next, int64_t *steps, int64_t *rejected);
int gf_set_time(gf_ctx *ctx, int32_t scen, double t, double dt_next);

/* Workgroup size of the step kernel (one workgroup per patch).  Built
 * sizes: m = 32: 256, 512 or 1024 threads; m = 16: 64, 128 or 256.  The default is the
 * smaller one; a tuner times the candidates and sets the faster.  Results do
 * not depend on the choice (same arithmetic per cell).
 * Errors: GF_E_UNSUPPORTED for a size that is not built. */
int gf_set_step_threads(gf_ctx *ctx, int32_t nt);
int gf_get_step_threads(gf_ctx *ctx, int32_t *nt);
/* LDS row padding of the step kernel's tile (0 or 1 extra words per row of
 * m+4 cells): a shape the tuner chooses; results do not depend on it.
 * Errors: GF_E_UNSUPPORTED for other values. */
int gf_set_step_pad(gf_ctx *ctx, int32_t pad);
/* Autotuner: time every built step-kernel shape for `steps` steps on the
 * context's current state and restore the state, clocks and budgets after
 * each trial, so the simulation is unchanged.  It keeps the first shape in
 * the order below (fewer threads, no padding, resident grid first) whose
 * time is within 2% of the fastest, so that a near tie resolves the same
 * way from run to run.  Shapes:
 * workgroup size (m = 32: 256, 512, 1024 threads, i.e. 4, 2, 1 cells per
 * thread; m = 16: 64, 128, 256) x LDS row padding (0, 1) x schedule (the
 * resident persistent grid, half of it, one workgroup per patch): 18.
 * cache_path (nullable; NULL takes gf_config.autotune_cache, which may be
 * NULL too): a text file of earlier choices keyed by GPU architecture,
 * precision, patch size and patch count (rounded up to a power of two); a
 * hit skips the timing (us_per_step is then -1), a miss appends the new
 * choice.  Outputs are nullable.
 * Errors: GF_E_INVALID, GF_E_STATE (no bathymetry or leaves), GF_E_HIP. */
int gf_autotune(gf_ctx *ctx, int32_t steps, const char *cache_path, int32_t *threads, int32_t *schedule,
                int32_t *pad, double *us_per_step);
/* The last timed gf_autotune's trials: n rows of (threads, schedule,
 * padding) into shapes (n x 3, nullable) and their us per step into us
 * (nullable); *n receives the count.  Errors: GF_E_INVALID (cap < n). */
int gf_autotune_trials(gf_ctx *ctx, int32_t *shapes, double *us, int64_t cap, int64_t *n);

/* Schedule of the step kernel.  workgroups = -1 (default): as many
 * persistent workgroups as the GPU holds at once, each taking patches of
 * every level and scenario from a device queue until it is empty; k > 0: at
 * most k persistent workgroups; 0: one workgroup per patch.  Results do not
 * depend on the choice.  Errors: GF_E_INVALID for workgroups < -1. */
int gf_set_schedule(gf_ctx *ctx, int32_t workgroups);

/* Time the steps with HIP events on the context stream.  on: bit 0 times
 * steps, bit 1 has the kernels count patches (gf_profile_patches); 0 stops
 * both.  A timed stretch of steps is bracketed by one event before its first
 * launch and one at the next synchronisation of the stream (the end of a
 * gf_step call, or gf_profile_read), so nothing is queued between the
 * kernels; the span includes every launch of the stretch (the dry-patch and
 * full-update kernels of each step, and reflux and gauges where a step has
 * them).  gf_profile_read synchronises and returns the number of steps
 * since the last read and their summed span in ms.  Errors: GF_E_INVALID
 * for on outside 0..3. */
int gf_profile_enable(gf_ctx *ctx, int32_t on);
int gf_profile_read(gf_ctx *ctx, int64_t *launches, double *ms_total);
/* With bit 2 of gf_profile_enable (value 4): an event pair around every
 * launch of the full-update (step) kernel alone, for the duration of that
 * kernel by itself.  gf_profile_kernel synchronises and returns the number
 * of timed launches since the last read and their summed durations in ms.
 * (The event packets between the dry-patch and step kernels add a few
 * microseconds to each step.) */
int gf_profile_kernel(gf_ctx *ctx, int64_t *launches, double *ms_total);
/* Patch counts over the counted steps (since gf_profile_enable with bit 1):
 * patches that went through the full update, and dry patches found stable
 * (both state buffers already holding the dry update's result, so that
 * nothing is read or written for them).  Synchronises the stream. */
int gf_profile_patches(gf_ctx *ctx, int64_t *full_updates, int64_t *stable_dry);

/* ------------------------------------------------------------------------
 * Learned refinement tagger (for callers that regrid less often than they
 * tag): a small convolutional network predicts per patch whether the plain
 * criteria of Section 4.1 will ask to refine (+1), keep (0) or coarsen (-1)
 * it over the next steps.  Features of a leaf at level l: the 24 x 24
 * pixels around it at its level (3 x 3 patch squares, 8 x 8 pixels each, a
 * pixel the area mean over m/8 x m/8 cells of the leaf fields), channels
 * h, hu/10, hv/10, (b - leaf mean b)/10, zero outside the domain; layout
 * [y][x][channel].  Network: 3x3 convolutions 4->16 (stride 1), 16->32
 * (stride 2), 32->32 (stride 2), ReLU after each, mean pooling, fully
 * connected 32->3; BF16 matrix-core products, FP32 accumulation.
 * ------------------------------------------------------------------------ */
#define GF_NET_PARAMS 14579   /* W1[16][3][3][4] b1[16] W2[32][3][3][16] b2[32] W3[32][3][3][32] b3[32] Wf[3][32] bf[3] */
#define GF_NET_FEATURES 2304  /* values per patch: 24 x 24 x 4 */

/* Set the parameters (FP32 master copy; n must be GF_NET_PARAMS) and reset
 * the optimiser.  Errors: GF_E_INVALID, GF_E_NOMEM. */
int gf_net_set_params(gf_ctx *ctx, const double *params, int64_t n);
int gf_net_get_params(gf_ctx *ctx, double *out, int64_t n);
/* Feature tiles of every leaf of every scenario, in leaf order, from the
 * current state: n_leaves x GF_NET_FEATURES values (out nullable to query
 * the count; cap in values).  Errors: GF_E_STATE, GF_E_INVALID (cap),
 * GF_E_UNSUPPORTED (feature images above 2^28 values). */
int gf_net_features(gf_ctx *ctx, double *out, int64_t cap, int64_t *n_leaves);
/* Logits (n x 3) for n feature tiles given on the host (rounded to BF16 on
 * the device). */
int gf_net_forward(gf_ctx *ctx, const double *x, int32_t n, double *logits);
/* One training step on n samples: labels y in {0 coarsen, 1 keep, 2 refine},
 * class weights class_w[3]; loss = sum over samples of
 * class_w[y] (-log softmax[y]) / sum of class_w[y].  Writes the loss and, if
 * grad is not null, the gradient before the Adam update (lr; beta1 0.9,
 * beta2 0.999, eps 1e-8).  Errors: GF_E_STATE (no parameters), GF_E_INVALID. */
int gf_net_train_step(gf_ctx *ctx, const double *x, const int8_t *y, int32_t n, const double *class_w, double lr,
                      double *loss, double *grad);
/* The same training step on a batch already in device memory (a caller's
 * torch tensors): x_bf16 n x GF_NET_FEATURES bfloat16 values (uint16 bit
 * patterns, [sample][y][x][channel]), y n int8 labels.  Both must stay valid
 * until the context stream has run the step; nothing is copied to the host
 * unless loss is requested (then the stream is synchronised).  The class
 * weight sum of the batch is formed on the device; a label outside 0..2
 * counts with weight 0 (no loss, no gradient).  A batch whose weights sum to
 * zero leaves the parameters unchanged and gives loss 0.
 * Errors: GF_E_INVALID (null pointers, n <= 0, lr < 0), GF_E_STATE (no
 * parameters), GF_E_NOMEM, GF_E_HIP. */
int gf_net_train_step_dev(gf_ctx *ctx, const uint16_t *x_bf16, const int8_t *y, int32_t n, const double *class_w,
                          double lr, double *loss);
/* Flags from the network for every leaf (largest logit, kept within each
 * scenario's level limits), in leaf order; they become the flags that
 * gf_regrid(ctx, NULL, ...) applies, as after gf_tag. */
int gf_net_predict(gf_ctx *ctx, int8_t *flags_out, int64_t cap, int64_t *n);

/* One collection window for training the tagger: the feature tiles of the
 * current leaves (n x GF_NET_FEATURES, nullable), then `window` steps with
 * the plain tagger run every `check_every` steps on this leaf set, labels
 * (n, nullable) 2 (refine) if any check asked to refine, 0 (coarsen) if
 * every check asked to coarsen, else 1; then a regrid with those flags.
 * cap counts leaves: features holds cap x GF_NET_FEATURES values, labels
 * cap entries (GF_E_INVALID if n exceeds it; *n is set either way).  window
 * must be a multiple of check_every. */
int gf_net_collect(gf_ctx *ctx, int32_t window, int32_t check_every, double *features, int8_t *labels, int64_t cap,
                   int64_t *n);

/* Adaptive run: `nsteps` steps with regridding.
 *   GF_RUN_PLAIN:   plain tagger and regrid every check_every steps;
 *   GF_RUN_SPARSE:  plain tagger and regrid every regrid_every steps; the
 *                   plain tagger also runs at the checks between (counted
 *                   as misses when it asks to refine, nothing done);
 *   GF_RUN_LEARNED: network flags every regrid_every steps, with every plain
 *                   refine request honoured and coarsening only where the
 *                   plain tagger agrees; at the checks between, a plain
 *                   refine request forces a regrid of those leaves.
 * regrid_every must be a multiple of check_every. */
enum { GF_RUN_PLAIN = 0, GF_RUN_SPARSE = 1, GF_RUN_LEARNED = 2 };
typedef struct {
    int64_t steps;           /* steps taken */
    int64_t regrids;         /* scheduled regrids */
    int64_t forced_regrids;  /* extra regrids forced by the checks (learned mode) */
    int64_t checks;          /* leaves examined at checks */
    int64_t misses;          /* of those, leaves the plain tagger wanted refined */
    int64_t leaf_steps;      /* sum over steps of the leaf count (work) */
    double seconds;          /* wall time of the call */
} gf_run_stats;
int gf_run(gf_ctx *ctx, int32_t nsteps, int32_t mode, int32_t check_every, int32_t regrid_every, gf_run_stats *stats);

/* Description of the last failure on this context (static storage, valid
 * until the next call on it). */
const char *gf_last_error(const gf_ctx *ctx);

/* Achievable HBM bandwidth probe (not a step of the method: the measured
 * denominator beside the spec-sheet peak of the roofline): one launch of a
 * grid-stride triad c[i] = a[i] + s b[i] over n floats (16-byte vector
 * accesses, n a multiple of 4), 12 n bytes moved, on `hip_stream` (NULL: the
 * null stream).  Device pointers, 16-byte aligned, not overlapping.
 * Errors: GF_E_INVALID (null or misaligned pointer, n <= 0 or not a multiple
 * of 4), GF_E_HIP. */
int gf_probe_triad(const float *a, const float *b, float *c, int64_t n, float s, void *hip_stream);

/* Library version string. */
const char *gf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GEOFLOOD_H */
