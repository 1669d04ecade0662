// Internal layout shared by the host core (gf_host.cpp) and the kernels
// (gf_kernels.inc, built once per precision).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/geoflood.h"   // the GF_LIMITER_* and GF_TRANSVERSE_* values

namespace gf {

// Halo regions of a patch (2-cell ghost layer), each fed by one source:
//   0,1 west face (lower, upper half)   2,3 east face
//   4,5 south face (left, right half)   6,7 north face
//   8 SW corner  9 SE corner  10 NW corner  11 NE corner
enum HaloKind : int32_t { HK_SAME = 0, HK_COARSE = 1, HK_FINE = 2, HK_PHYS = 3 };

struct HaloSrc {
    int32_t kind;   // HaloKind
    int32_t slot;   // source patch slot (unused for HK_PHYS)
    int32_t oi, oj; // index offsets, see the kernel's gather
};

// Per leaf work item.  Indices are global at the leaf's level.
struct PatchDesc {
    int32_t slot;
    int32_t scen;
    int32_t level;
    int32_t phys;        // bit s set: side s (0 xlo,1 xhi,2 ylo,3 yhi) is a physical boundary
    int32_t PI, PJ;      // global patch index
    int32_t bc[4];       // boundary type per side (valid where phys bit set)
    int32_t cf_face[4];  // reflux register index of a face touching a different level, or -1
    int32_t cf_role[4];  // 0 none, 1 this patch is the coarse side, 2 the fine side
    double dx, dy;
    double xlo, ylo;     // lower-left corner of the patch
    HaloSrc src[12];
};

// Reflux task: one coarse patch with up to four faces next to finer patches.
struct RefluxTask {
    int32_t slot;         // coarse patch slot
    int32_t scen;
    int32_t reg_c[4];     // register of each coarse face (m entries), -1 if the face is not coarse/fine
    int32_t reg_f[4][2];  // registers of the two fine faces covering the lower/left and upper/right half
    double area;          // coarse cell area
    int32_t level;        // coarse patch level
    int32_t pad;
};

// Per-scenario clock and controller state, device resident.
struct ScenDev {
    double t, dt, t_end;
    double dt_used;          // step length of the last attempt
    double nu_last;
    double nu_max;           // largest Courant number of the accepted steps since the host reset it
    double manning_n;
    double inflow_lo, inflow_hi;
    double x0, y0;           // domain origin (cell centres x0 + (I + 1/2) dx)
    double hydro_t[16], hydro_q[16];
    int32_t n_hydro;
    int32_t inflow_side;
    int32_t cur;             // buffer index holding the current state
    int32_t status;          // 0 ok, else a GF_E_* code
    int64_t steps, rejected, target;
    int32_t accepted_last;   // 1 if the last launch accepted a step
    int32_t nan_flag;
    unsigned long long smax_bits;  // max |s|/dx of the running attempt (double bits); LTS: max Courant number
    // local time stepping (reading R40)
    int32_t lcur[16];        // per level: the buffer holding its current state
    int32_t lcur0[16];       // the same at the start of the macro step
    int32_t L0, L1;          // coarsest and finest level present
    int32_t lts_on;          // taking part in the running macro step
    int32_t lts_fail;        // the macro step is to be undone (rejected or failed)
};

// Refinement rules of one scenario (Section 4.1): thresholds of the cell
// criteria, flood-source regions and flow grades.
constexpr int kMaxRegions = 4, kMaxGrades = 4;
struct TagRules {
    double h, eta, u, q;              // depth, free surface, speed, velocity-depth (u, q: 0 off)
    double region[kMaxRegions][4];    // x0 y0 x1 y1
    double grade_thr[kMaxGrades];
    int32_t lmin, lmax, n_regions, n_grades;
    int32_t region_lev[kMaxRegions][2];  // min, max level inside
    int32_t grade_qty[kMaxGrades];    // 0 depth, 1 speed
    int32_t grade_lev[kMaxGrades];
};

// A gauge: the cell of the current mesh that holds the point.
struct GaugeDev {
    int32_t scen, slot, cell, level;
};

template <typename R>
struct StepArgs {
    const PatchDesc *desc;
    int32_t n_work;
    ScenDev *scen;
    int32_t n_scen;
    R *q0, *q1;              // [3][cap][m*m] per buffer
    const R *b;              // [cap][m*m]
    const R *bg;             // [cap][ring]
    double *clamp_acc0, *clamp_acc1;   // [cap] per buffer
    double *bnd_acc0, *bnd_acc1;       // [cap] per buffer
    R *reg;                  // reflux registers [n_reg][m][3]
    int64_t cap;             // pool capacity (slots)
    double dt_fixed;         // >= 0: use this step length in every scenario
    int32_t mode;            // 0 step, 1 speed-only pass
    double g, cfl_desired, cfl_max;
    R tau;                   // dry iff h <= tau (tau rounded down to R)
    double tau64;
    unsigned int *done_counter;  // [0] groups done; [16 (1 + g)] workgroups done in group g (64 per group)
    unsigned int *queue;         // next work item (persistent form); reset to 0 by the last workgroup
    int32_t persistent;          // 1: resident workgroups take items from the queue
    uint8_t *dry0, *dry1;        // per slot and buffer: 1 iff every interior cell has h <= tau
    int32_t *wet_list;           // work items dry_kernel left for step_kernel
    unsigned int *wet_count;     // their number; reset to 0 by the last workgroup of step_kernel
    // patches dry_kernel found needing the dry update, for dry_update_kernel:
    // kept in wet_list from its far end (entry k at cap - 1 - k; wet and dry
    // entries together are at most the patch count), their number reset with
    // wet_count
    unsigned int *dry_count;
    // per slot: 0 unknown; 1 + 2c: the last update was a full dry update
    // reading buffer c; 4 stable: both buffers hold the same dry state, a
    // fixed point of the dry update (which then writes nothing)
    uint8_t *dstab;
    unsigned long long *stats;   // [0] patches through step_kernel, [1] stable dry patches (or null)
    int32_t lts;                 // local time stepping: the levels starting a substep at `tick` only
    int32_t tick;
    int32_t limiter;             // GF_LIMITER_*: the wave limiter of the corrections
    int32_t transverse;          // GF_TRANSVERSE_*: corrected transverse terms or none
};

struct RefluxArgsBase {
    const RefluxTask *tasks;
    int32_t n_tasks;
    ScenDev *scen;
    int64_t cap;
    double tau64;
    uint8_t *dstab;          // per-slot dry-update state, cleared for corrected patches
    int32_t lts, tick;       // local time stepping: the levels whose step ends at `tick` only
};

}  // namespace gf

// Launchers, one set per precision (defined in gf_kernels_f32.hip / _f64.hip).
#define GF_DECL_LAUNCHERS(SFX, R)                                                                  \
    hipError_t gf_launch_step_##SFX(const gf::StepArgs<R> &a, int m, int nt, int pad, int grid, hipStream_t s); \
    int gf_step_threads_ok_##SFX(int m, int nt);                                                   \
    hipError_t gf_launch_dry_##SFX(const gf::StepArgs<R> &a, int m, hipStream_t s);                \
    int gf_step_resident_##SFX(int m, int nt, int pad);                                            \
    hipError_t gf_launch_dryflag_##SFX(const gf::PatchDesc *d, int n, const gf::ScenDev *scen,     \
                                       const R *q0, const R *q1, uint8_t *f0, uint8_t *f1,         \
                                       uint8_t *dstab, int64_t cap, R tau, int m, hipStream_t s);  \
    hipError_t gf_launch_reflux_##SFX(const gf::RefluxArgsBase &a, R *q0, R *q1, const R *reg,     \
                                      double *ca0, double *ca1, uint8_t *f0, uint8_t *f1, int m,   \
                                      hipStream_t s);                                               \
    hipError_t gf_launch_tag_##SFX(const gf::PatchDesc *d, int n, const gf::ScenDev *scen,         \
                                   const R *q0, const R *q1, const R *b, int64_t cap,              \
                                   const gf::TagRules *rules, double tau64, int8_t *flags, int m,  \
                                   hipStream_t s);                                                 \
    hipError_t gf_launch_gauge_##SFX(const gf::GaugeDev *g, int n, const gf::ScenDev *scen,        \
                                     const R *q0, const R *q1, const R *b, int64_t cap, int m,       \
                                     int64_t rec_cap, double *rec, int64_t *count, int lts,          \
                                     hipStream_t s);                                                 \
    hipError_t gf_launch_lts_scen_##SFX(gf::ScenDev *scen, int n_scen, int phase, hipStream_t s);    \
    hipError_t gf_launch_lts_copy_##SFX(const gf::PatchDesc *d, int n, const gf::ScenDev *scen,     \
                                        R *q0, R *q1, double *ca0, double *ca1, double *ba0,        \
                                        double *ba1, R *snap, double *snap_acc, int64_t cap,         \
                                        int dir, int m, hipStream_t s);                              \
    hipError_t gf_launch_mass_##SFX(const gf::PatchDesc *d, int n, const gf::ScenDev *scen,        \
                                    const R *q0, const R *q1, int64_t cap, double *out, int m,     \
                                    hipStream_t s);                                                 \
    hipError_t gf_launch_transfer_##SFX(const void *tasks, int n, const gf::ScenDev *scen, R *q0, R *q1, \
                                        const R *b, int64_t cap, double tau, int m, hipStream_t s);       \
    hipError_t gf_launch_state_##SFX(int kind, const R *a, const R *b, const int32_t *slots, int n,      \
                                     int64_t fs, R *out, int m, hipStream_t s);                       \
    hipError_t gf_launch_bathy_##SFX(const R *staged, const int32_t *slots, int n, R *b, R *bg, int m,  \
                                     hipStream_t s);                                                  \
    hipError_t gf_launch_ghost_##SFX(const gf::StepArgs<R> &a, const int32_t *items, int n, R *ghost, int m, \
                                     hipStream_t s);                                                  \
    hipError_t gf_launch_plain_##SFX(const gf::StepArgs<R> &a, const int32_t *items, int n, const R *ghost, \
                                     double *pmax, int32_t *pnan, int m, hipStream_t s);              \
    hipError_t gf_launch_cflred_##SFX(const double *pmax, const int32_t *pnan, const int32_t *range, int n_scen, \
                                      double *out, hipStream_t s);

// regrid transfer task (layout shared with the kernels)
namespace gf {
struct XferTaskH {
    int32_t kind, dst, scen, qx, qy, src[4];
};
}

GF_DECL_LAUNCHERS(f32, float)
GF_DECL_LAUNCHERS(f64, double)

// The entry point that allocates nothing (gf_mass_static, gf_static.hip):
// device scratch for the per-patch partials of this many patches at most.
namespace gf {
constexpr int kStaticMassPatches = 1 << 16;
}
// address of this device's copy of the scratch array (call with the device current)
hipError_t gf_static_scratch(double **ptr);
// res[0..2] = volume, clamp volume, boundary volume of scenario `scen`
hipError_t gf_launch_mass_ordered(const double *part, const gf::PatchDesc *d, int nw, int scen, const double *ca,
                                  const double *ba, double clamp_base, double bnd_base, double *res, hipStream_t s);
