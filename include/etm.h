/*
 * etm.h - C ABI of the MI355X (gfx950) transient EM-thermal-mechanical
 * package solver: the data-parallel hot path of arXiv 2603.07038, Sec. II.
 *
 * One plan = one package design: a rectilinear voxel mesh with one material
 * per cell, a material table, port edges with sampled excitations and run
 * options.  The plan marches
 *   1. the EM field by the explicit central-difference update, Eq. (2)-(3),
 *      with sigma(T) from Eq. (6);
 *   2. the Joule source P = D_sigma e^2 (Sec. II-A, below Eq. 4);
 *   3. transient conduction by forward Euler, Eq. (4)-(5), every R EM steps
 *      with the block-mean Joule source (R = 1 is the paper's schedule);
 *   4. the thermoelastic HEX8 system, Eq. (7)-(8), by CG preconditioned with
 *      a geometric multigrid V-cycle (or nodal Jacobi), and the centroid von
 *      Mises stress, Eq. (9);
 * on one GPU.  Device memory is owned by the caller (e.g. a torch tensor)
 * and handed to the plan as one workspace; all GPU work is enqueued on the
 * caller's HIP stream.
 *
 * Conventions
 *  - Every function returns etm_status (ETM_OK = 0, errors < 0) and never
 *    aborts or prints; etm_last_error() gives a thread-local message.
 *  - Host inputs are borrowed for the duration of the call and deep-copied.
 *  - Spatial arrays handed in or out are C-ordered with x fastest in their
 *    natural shapes: cells (nz,ny,nx); nodes (nz+1,ny+1,nx+1); x-edges
 *    (nz+1,ny+1,nx); y-edges (nz+1,ny,nx+1); z-edges (nz,ny+1,nx+1).  The
 *    x-edge (i,j,k) joins nodes (i,j,k) and (i+1,j,k); likewise y and z.
 *  - SI units.  Temperature is carried as the rise theta = T - T0.
 */
#ifndef ETM_H
#define ETM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t etm_status;
enum {
    ETM_OK = 0,
    ETM_E_INVAL = -1,    /* malformed argument, mesh, material, port or option */
    ETM_E_NOMEM = -2,    /* workspace too small / host allocation failed */
    ETM_E_HIP = -3,      /* a HIP runtime call failed */
    ETM_E_UNSTABLE = -4, /* dt above the CFL limit, explicit thermal step unstable, or non-finite field */
    ETM_E_NOCONV = -5,   /* the mechanical CG did not reach its tolerance within cg_maxit */
    ETM_E_STATE = -6     /* call out of order (e.g. advance before bind) */
};

enum { ETM_PMC = 0, ETM_PEC = 1 };                          /* EM face condition */
enum { ETM_MECH_KINEMATIC = 0, ETM_MECH_CLAMP_ZMIN = 1 };   /* mechanical support */
/* Arithmetic of the path.  FP64: the three-level update of Eq. (2)-(3) on
 * (e^n, e^{n-1}) in FP64.  MIXED: the same scheme in its leapfrog form on
 * (e^n, h^{n-1/2}), both stored in FP32 and combined in FP64, with FP64
 * temperature, Joule accumulation and CG refinement. */
enum { ETM_PREC_FP64 = 0, ETM_PREC_MIXED = 1 };
/* Preconditioner of the mechanical CG (Eq. 8): nodal Jacobi, or a geometric
 * multigrid V-cycle with Galerkin coarse operators (the role the paper's
 * algebraic multigrid plays, Sec. IV-A). */
enum { ETM_PRECOND_JACOBI = 0, ETM_PRECOND_MG = 1 };

/* Fields for etm_read / etm_write (always FP64, natural shapes). */
enum {
    ETM_FIELD_EX = 0, ETM_FIELD_EY = 1, ETM_FIELD_EZ = 2,          /* e^n                 */
    ETM_FIELD_EX_PREV = 3, ETM_FIELD_EY_PREV = 4, ETM_FIELD_EZ_PREV = 5, /* e^{n-1}     */
    ETM_FIELD_THETA = 6,   /* temperature rise on nodes                                  */
    ETM_FIELD_PSUM = 7,    /* sum of the Joule power density over the open thermal block */
    ETM_FIELD_UX = 8, ETM_FIELD_UY = 9, ETM_FIELD_UZ = 10,          /* displacement      */
    ETM_FIELD_VM = 11,     /* von Mises stress per cell (read only)                       */
    ETM_FIELD_FX = 12, ETM_FIELD_FY = 13, ETM_FIELD_FZ = 14         /* thermal load (read only) */
};

/* One material (a row of the table indexed by the per-cell id).
 * eps_r relative permittivity; sigma0 conductivity at T0 [S/m]; tcr
 * temperature coefficient of resistance [1/K] (Eq. 6); k thermal
 * conductivity [W/m/K]; rho_cp volumetric heat capacity [J/m^3/K]; E Young's
 * modulus [Pa]; nu Poisson ratio; cte linear expansion [1/K]; is_void != 0
 * marks a cell without stiffness (air). */
typedef struct {
    double eps_r, sigma0, tcr, k, rho_cp, E, nu, cte;
    int32_t is_void;
    int32_t reserved;
} etm_material;

/* Rectilinear mesh: cell widths dx[nx], dy[ny], dz[nz] in metres (all > 0)
 * and one material id per cell, mat[(k*ny + j)*nx + i] < n_mat. */
typedef struct {
    int32_t nx, ny, nz;
    const double *dx, *dy, *dz;
    const uint8_t *mat;
} etm_mesh;

/* A port edge: direction dir (0/1/2 = x/y/z) starting at node (i,j,k).
 * The edge carries the impressed current density weight * J_wave(t) [A/m^2]
 * and the lumped conductance g [S/m] added to its conductivity in the
 * update (the Norton form of a resistive source).  g does not heat. */
typedef struct {
    int32_t dir, i, j, k, wave;
    int32_t reserved;
    double weight, g;
} etm_port;

/* Closed-form excitation waveforms, evaluated on the device at every EM step
 * (the transient excitation scheme of Sec. III-B: a Ricker trigger, a sine
 * "logic noise" and a Gaussian-pulse-train "data burst" on a carrier, each
 * with its own per-port amplitude, width and phase).  A wave is zero outside
 * [t_on, t_off); inside, with u = (t - t0) / width:
 *   ETM_WAVE_RICKER       amp * (1 - 2 u^2) * exp(-u^2)
 *   ETM_WAVE_SINE         amp * sin(2 pi freq (t - t0))
 *   ETM_WAVE_GAUSS_TRAIN  amp * cos(2 pi freq (t - t0)) * sum_p exp(-((t - pulse_t[p]) / width)^2),
 *                         p < n_pulses
 * Times in seconds, freq in Hz; amp in the unit of the port weight's
 * counterpart (A/m^2 for a current port of weight 1, V for a voltage port).
 * Validation at etm_plan_create: kind known, width > 0 where used,
 * 1 <= n_pulses <= ETM_WAVE_MAX_PULSES for trains, t_on <= t_off (an empty
 * window is a wave that is always zero), all values finite; else
 * ETM_E_INVAL. */
enum { ETM_WAVE_RICKER = 1, ETM_WAVE_SINE = 2, ETM_WAVE_GAUSS_TRAIN = 3 };
#define ETM_WAVE_MAX_PULSES 8
typedef struct {
    int32_t kind;
    int32_t n_pulses;
    double amp, t0, width, freq, t_on, t_off;
    double pulse_t[ETM_WAVE_MAX_PULSES];
} etm_wave;

/* Excitations.  Sampled waves: J_half[w*n_samples + s] = J_w((s - 1/2) dt),
 * so EM step n (making e^{n+1}) uses samples n+1 and n; samples beyond the
 * array are taken as zero.  Column 0 (t = -dt/2) is zero for a causal
 * source.  Closed-form waves (analytic, may be null when n_analytic = 0)
 * follow the sampled ones: a port's wave index w < n_waves names sampled
 * wave w, n_waves <= w < n_waves + n_analytic names analytic[w - n_waves],
 * evaluated at t = (n + 1/2) dt and (n - 1/2) dt for step n.  All arrays
 * are copied at etm_plan_create. */
typedef struct {
    int64_t n_ports;
    const etm_port *ports;
    int32_t n_waves;
    int64_t n_samples;
    const double *J_half;
    int32_t n_analytic;
    int32_t reserved;
    const etm_wave *analytic;
} etm_source;

/* Run options.  Fill with etm_opts_default() first. */
typedef struct {
    double dt;                  /* EM step [s]; 0 = cfl * CFL limit */
    double cfl;                 /* Courant number used when dt == 0 (default 0.9) */
    int32_t force_dt;           /* accept dt above the CFL limit (for failure tests) */
    int32_t precision;          /* ETM_PREC_FP64 or ETM_PREC_MIXED */
    int32_t em_bc[6];           /* -x,+x,-y,+y,-z,+z: ETM_PMC or ETM_PEC */
    int32_t em_per_thermal;     /* R: EM steps per thermal step (>= 1) */
    int32_t mech_every_thermal; /* m > 0: mechanical solve after every m-th thermal step; 0: only on request */
    int32_t mech_bc;            /* ETM_MECH_KINEMATIC or ETM_MECH_CLAMP_ZMIN */
    const uint8_t *mech_mask;   /* optional per-node fixed-DOF bits (1=x,2=y,4=z), node shape; overrides mech_bc */
    int32_t cg_maxit;           /* CG iteration limit per solve (default 200000) */
    double cg_rtol;             /* ||f - K u||_2 <= cg_rtol ||f||_2 on the FP64 residual (default 1e-8) */
    int32_t history_stride;     /* record histories every stride EM steps (0 = never) */
    int32_t n_probes;           /* probes[4*p..] = field (0..2 = ex,ey,ez; 3 = theta), i, j, k */
    const int64_t *probes;
    int64_t history_cap;        /* records kept (0 = enough for n_em_steps_hint) */
    int64_t n_em_steps_hint;    /* expected run length (sizes the history) */
    int32_t mech_precond;       /* ETM_PRECOND_MG (default) or ETM_PRECOND_JACOBI */
    int32_t mg_coarse_dofs;     /* multigrid: coarsen until a level has at most this many DOF
                                   (solved with a dense inverse; default 800, range 3..4000) */
    int32_t mg_degree[2];       /* multigrid: Chebyshev smoothing steps before and after the coarse
                                   correction on the finest level and on the coarser levels
                                   (0 = default: 3 on the finest level, 2 below; range 1..4) */
    int32_t em_slabs;           /* temporal blocking of the EM march: 0 or 1 = one launch per step;
                                   S >= 2 = two steps at a time as a wavefront over S z-slabs, the
                                   second step of a slab running right after the first has finished
                                   the slab and its neighbours, so it finds them in the on-chip caches.
                                   Results are bitwise those of one launch per step.  Pairs never
                                   straddle a thermal step or a history record.  Range 0..64. */
    int32_t mech_overlap;       /* 1 (default) = a scheduled mechanical solve runs on a side stream while
                                   the EM steps that follow it in the same etm_advance call (up to the
                                   next thermal step or history record) run on the plan's stream; the
                                   solve reads only the temperature of its own thermal step and the
                                   march never reads the displacement, so results are bitwise those of
                                   the serial order.  0 = serial.  The plan's stream waits for the
                                   solve before any later work. */
} etm_opts;

/* What etm_sync reports. */
typedef struct {
    int64_t step;          /* EM steps done */
    int32_t status;        /* first asynchronous error seen (ETM_OK if none) */
    int32_t cg_iters;      /* iterations of the last mechanical solve (inner, all refinements) */
    int32_t cg_outer;      /* FP64 residual evaluations of the last solve */
    int32_t n_solves;      /* mechanical solves so far */
    double cg_relres;      /* final ||f - K u|| / ||f|| of the last solve */
    double theta_max;      /* max temperature rise */
    double ejoule;         /* dissipated EM energy so far [J] */
    int64_t n_records;     /* history records available */
    int64_t cg_iters_total;/* inner CG iterations over all solves */
    int32_t mg_levels;     /* multigrid levels (0 with Jacobi or before the first solve) */
    int32_t reserved;
} etm_run_info;

typedef struct etm_plan etm_plan;
typedef struct etm_batch etm_batch;

/* Default options: dt auto at CFL 0.9, FP64, all faces PMC, R = 1, no
 * scheduled mechanics, kinematic mount, rtol 1e-8. */
etm_status etm_opts_default(etm_opts *opts);

/* CFL-limited step for a mesh (Eq. 2 is constrained by CFL, Sec. II-A):
 * dt = cfl / (c0 sqrt(1/dx_min^2 + 1/dy_min^2 + 1/dz_min^2)). */
etm_status etm_cfl_dt(const etm_mesh *mesh, double cfl, double *dt);

/* Validate and copy all inputs; derive tables, DOF maps, constraints and the
 * workspace layout.  Host only.  ETM_E_INVAL on malformed input,
 * ETM_E_UNSTABLE when dt exceeds the CFL limit (unless force_dt) or the
 * explicit thermal step R*dt exceeds its forward-Euler bound. */
etm_status etm_plan_create(const etm_mesh *mesh, const etm_material *mats, int32_t n_mat,
                           const etm_source *src, const etm_opts *opts, etm_plan **out);

/* Device bytes the plan needs in its workspace (256-byte aligned start). */
etm_status etm_plan_footprint(const etm_plan *plan, size_t *device_bytes);

/* The EM step in use [s]. */
etm_status etm_plan_dt(const etm_plan *plan, double *dt);

/* DOF counts: EM edges (PEC edges included), thermal nodes, mechanical node DOFs (3 per node). */
etm_status etm_plan_dofs(const etm_plan *plan, int64_t *em, int64_t *thermal, int64_t *mech);

/* Attach caller-owned device memory (>= footprint bytes, 256-byte aligned)
 * and a hipStream_t (NULL = default stream).  Uploads the tables, zeroes the
 * state (e = 0, theta = 0) and enqueues everything on the stream.  May be
 * called again to move the plan to a new workspace (state is reset). */
etm_status etm_plan_bind(etm_plan *plan, void *device_ws, size_t bytes, void *hip_stream);

/* Enqueue n_em_steps coupled steps (EM + Joule + thermal every R steps +
 * histories; a scheduled mechanical solve is enqueued at its thermal step,
 * on the plan's side stream beside the following EM steps when mech_overlap
 * is set).  Returns without waiting for the GPU, except that a scheduled
 * solve first waits for the previous solve of the plan to be decided (it
 * owns the displacement the next one starts from), and the first solve of a
 * plan waits while it builds the multigrid hierarchy.  Asynchronous errors
 * are reported by etm_sync. */
etm_status etm_advance(etm_plan *plan, int64_t n_em_steps);

/* Enqueue a solve of Eq. (8) for the current temperature (warm-started from
 * the last displacement) and the von Mises stress of Eq. (9) on the plan's
 * stream, and return (same waits as above).  The solve's outer loop -- the
 * FP64 residual check, the mixed path's FP32 corrections, the tolerance
 * ||f - K u|| <= cg_rtol ||f|| and the cg_maxit limit -- is decided on the
 * device; the host enqueues passes sized from the previous solve and, if
 * the device has not decided the solve when they end, more passes at the
 * next call that needs the result.  Its outcome (iterations, residual,
 * ETM_E_NOCONV) is reported by etm_sync. */
etm_status etm_mech_solve(etm_plan *plan);

/* Wait for the plan's work (its stream and an enqueued solve); fill info (may
 * be NULL); return the first asynchronous error (ETM_E_UNSTABLE on a
 * non-finite field or temperature, ETM_E_NOCONV when a solve stopped at
 * cg_maxit or made no progress).  etm_read, etm_write, etm_checkpoint and
 * etm_restore also wait for an enqueued solve before they touch the state. */
etm_status etm_sync(etm_plan *plan, etm_run_info *info);

/* Copy a field out as FP64 in its natural shape (bytes must equal the
 * field's size * 8).  dst_is_device != 0: dst is device memory. */
etm_status etm_read(const etm_plan *plan, int32_t field, void *dst, size_t bytes, int32_t dst_is_device);

/* Overwrite a state field (EX..PSUM, UX..UZ) from FP64 natural-shape data.
 * The mixed path advances e with its face field h (leapfrog form), so its
 * e fields (EX..EZ_PREV) are not writable there (ETM_E_INVAL); checkpoints
 * restore them together with h. */
etm_status etm_write(etm_plan *plan, int32_t field, const void *src, size_t bytes, int32_t src_is_device);

/* Histories: rows of [step, W, cumulative Joule energy, max theta, probes...]
 * where W = 1/2 [(e^{n+1}-e^n)^T D_eps (e^{n+1}-e^n)/dt^2 + e^{n+1 T} S e^n]
 * is the discrete energy Eq. (2) conserves without loss or source.
 * *n_rows receives the number of rows copied. */
etm_status etm_read_history(const etm_plan *plan, double *dst, size_t bytes, int64_t *n_rows);

/* Checkpoint / restore the whole march state (step, fields, block sum,
 * Joule energy, displacement) through host memory; a restored plan
 * continues bitwise identically. */
etm_status etm_checkpoint_size(const etm_plan *plan, size_t *bytes);
etm_status etm_checkpoint(const etm_plan *plan, void *dst, size_t bytes);
etm_status etm_restore(etm_plan *plan, const void *src, size_t bytes);

/* Destroy the plan (does not free the caller's workspace). */
void etm_plan_destroy(etm_plan *plan);

/* ---- batched design variants (one launch per step over all variants) ----
 * A batch holds up to max_slots bound plans.  etm_batch_advance enqueues
 * n_em_steps steps of every attached plan on one stream: each EM step is a
 * single launch that walks a (variant, tile) work list, each thermal block a
 * single launch; chunks of steps are captured once in a HIP graph and
 * replayed.  A variant's results are bitwise those of its solo run.
 * tune_json (NULL or "{}": defaults) is the autotuner's table of tile shapes
 * per size class, the class being floor(log2(cells)) of a variant:
 *   {"kchunk": {"<class>": planes, ...}, "layout": {"<class>": 1 | 2, ...},
 *    "kchunk_fp64": {"<class>": planes, ...}}
 * kchunk (1..128) is the z-chunk of the mixed-precision march tiles and
 * kchunk_fp64 that of the FP64 tiles; layout (mixed precision only) makes
 * the waves take runs of 62 nodes over the plane numbered x fastest (1) or
 * 62-node segments of rows, 4 rows per block (2).  A class without an entry
 * takes the chunk the library picks from the variant's tile count.  Entries
 * out of range and malformed text are ignored; no choice changes results.
 * The string is read at creation and not kept. */
etm_status etm_batch_create(int32_t max_slots, const char *tune_json, etm_batch **out);
etm_status etm_batch_attach(etm_batch *batch, etm_plan *plan, int32_t *slot);
etm_status etm_batch_detach(etm_batch *batch, int32_t slot);
etm_status etm_batch_advance(etm_batch *batch, int64_t n_em_steps, void *hip_stream);

/* etm_batch_advance for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, hosts that forbid
 * hipMalloc): the same steps with the same kernels and bitwise the same
 * results, but the variant descriptors, the work list and the step counter
 * live in a fixed 4 MiB array of device memory that the library holds on
 * each GPU until the process ends, the work list is generated on the device,
 * and every step is launched directly (no graphs).  The call makes no
 * hipMalloc / hipFree / graph instantiation; the batch and its plans must
 * already exist and be bound.
 * Limits (ETM_E_INVAL beyond them, nothing enqueued): at most 64 attached
 * variants; at most 259,344 march tiles over all variants (a tile is 62 x 4
 * nodes by one z-chunk in mixed precision, 64 x 4 in FP64); attached plans
 * must not schedule mechanical solves (mech_every_thermal = 0); every plan's
 * workspace must be on the device that was current at etm_batch_create.
 * The array is shared by every call on one GPU and keeps the last call's
 * contents: calls that overlap on one GPU (two batches advanced from
 * different host threads or on unordered streams) race and must be
 * serialised by the caller.  Errors as etm_batch_advance. */
etm_status etm_batch_advance_noalloc(etm_batch *batch, int64_t n_em_steps, void *hip_stream);
void etm_batch_destroy(etm_batch *batch);

const char *etm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ETM_H */
