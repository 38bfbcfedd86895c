/*
 * djtled.h -- C ABI of the MI355X DJ-TLED library (libdjtled.so).
 *
 * Implements the time step of the direct Jacobian total Lagrangian explicit
 * dynamics method (Zhang, arXiv 2106.14189) on one AMD Instinct MI355X
 * (gfx950):
 *   (a) element nodal forces from the precomputed Jacobian constants and the
 *       gathered nodal displacements (Sec. 2.2, Eq. 10; the neo-Hookean,
 *       transversely isotropic, orthotropic and Mooney-Rivlin rows of Table 3;
 *       invariants of Table 1), or, for comparison, the classical TLED force
 *       (Eq. 4),
 *   (b) reduction of the element forces to the nodes (the sum of Eq. 13),
 *   (c) central-difference explicit integration with lumped mass-proportional
 *       damping (Eq. 13) and displacement boundary conditions, under the
 *       critical step of Eq. 14,
 * for one mesh (several load cases per launch if wanted) or for a batch of
 * meshes in one launch.
 *
 * Conventions shared by every entry point
 *   - Host pointers are read during the call only; the library never keeps or
 *     frees caller memory.  Device pointers must be device memory of the
 *     context's GPU (hipMalloc or a framework allocator).
 *   - Node and element indices are the caller's; the library reorders
 *     internally (space-filling-curve order) and permutes at call entry and exit.
 *   - Device vectors of nodal quantities are n_nodes x 3, row-major (x, y, z of
 *     node 0, then node 1, ...), in the context's precision (float for
 *     DJ_FP32, double for DJ_FP64).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - A context (and a batch) owns device buffers that every call on it
 *     uses: calls on one context must not overlap (one host thread at a
 *     time, one call in flight); separate contexts are independent.
 *   - Return codes: DJ_OK (0), DJ_CONVERGED (1, informational), or a negative
 *     DJ_ERR_*.  djtled_last_error() returns a thread-local message for the
 *     last failing call on the calling thread.
 */
#ifndef DJTLED_H
#define DJTLED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DJ_OK 0
#define DJ_CONVERGED 1
#define DJ_ERR_ARG (-1)          /* invalid argument (null pointer, bad size or enum) */
#define DJ_ERR_BAD_MESH (-2)     /* node index out of range, or det(0J) <= 0 (Eq. 3 / Eq. 12) */
#define DJ_ERR_INVERTED (-3)     /* run-time volume ratio J <= 0 (Eq. 12) */
#define DJ_ERR_NONFINITE (-4)    /* a force or displacement became NaN / Inf */
#define DJ_ERR_UNSUPPORTED (-5)  /* element type / model / precision not built */
#define DJ_ERR_UNSTABLE_DT (-6)  /* dt above the critical step of Eq. 14 without override */
#define DJ_ERR_HIP (-7)          /* a HIP runtime call failed (message has the hipError_t) */
#define DJ_ERR_BARRIER (-8)      /* the persistent kernel's grid barrier timed out */

enum { DJ_T4 = 4, DJ_H8 = 8 };                 /* linear tetrahedron, 8-node hexahedron */
enum { DJ_NH = 0, DJ_TI = 1, DJ_OT = 2, DJ_MR = 3 };  /* Table 3 rows: neo-Hookean, transversely isotropic NH,
                                                       orthotropic NH, Mooney-Rivlin */
enum { DJ_FP32 = 0, DJ_FP64 = 1 };
/* Element force: the Jacobian form of Table 3 (the method), or the classical
   TLED form of Eq. 4 (deformation gradient, C^-1 and the second Piola-Kirchhoff
   stress of the same strain energy), kept as a comparison path (FP32 only), or
   the Jacobian form with the average nodal pressure that Sec. 7 names against
   volumetric locking (DJ_NH / DJ_TI, variants 0..3; see djtled_forces_anp for
   the pressure): every time step then makes a J pass over the elements, a grid
   barrier, and the force pass with each element's pressure the mean of its
   nodes' pressures, and djtled_forces returns these forces. */
enum { DJ_FORM_JACOBIAN = 0, DJ_FORM_CLASSICAL = 1, DJ_FORM_NODAL_PRESSURE = 2 };
enum { DJ_RAMP_NONE = 0, DJ_RAMP_LINEAR = 1, DJ_RAMP_SMOOTH = 2 };
enum { DJ_MODE_FIXED = 0, DJ_MODE_RELAX = 1 };

/* Mesh (host memory).  T4 nodes follow h = (1 - xi - eta - zeta, xi, eta,
   zeta) with det(0J) > 0; H8 nodes follow (---, +--, ++-, -+-, --+, +-+, +++,
   -++) in natural coordinates. */
typedef struct {
    int32_t n_nodes;
    int32_t n_elems;
    int32_t elem_type;      /* DJ_T4 or DJ_H8 */
    const double *X;        /* n_nodes x 3 reference coordinates [m] */
    const int32_t *conn;    /* n_elems x elem_type node indices */
} djtled_mesh;

/* Material (host memory).  mu = E / (2 (1 + nu)), kappa = E / (3 (1 - 2 nu)).
   Per-element arrays may be NULL, in which case the *_uniform value is used.
   DJ_MR takes C10 = mu / 2 (as Sec. 5.1 does) and C01 below; its initial
   shear modulus is 2 (C10 + C01). */
typedef struct {
    int32_t model;          /* DJ_NH, DJ_TI, DJ_OT or DJ_MR (Table 3) */
    const double *E;        /* n_elems Young's modulus [Pa] or NULL */
    const double *nu;       /* n_elems Poisson's ratio or NULL */
    double E_uniform, nu_uniform;
    double rho;             /* mass density [kg / m^3] */
    const double *eta_ratio;   /* DJ_TI, DJ_OT: eta_a / mu per element, or NULL */
    double eta_ratio_uniform;
    const double *fibre;    /* DJ_TI, DJ_OT: n_elems x 3 fibre directions a (normalised internally) */
    double hg_kappa;        /* DJ_H8: hourglass coefficient (Flanagan-Belytschko form); <0 -> 0.1 */
    const double *fibre_b;  /* DJ_OT: n_elems x 3 second fibre directions b */
    const double *eta_b_ratio;  /* DJ_OT: eta_b / mu per element, or NULL */
    double eta_b_ratio_uniform;
    const double *c01;      /* DJ_MR: C01 [Pa] per element, or NULL */
    double c01_uniform;
} djtled_material;

/* Solver parameters. */
typedef struct {
    int32_t precision;      /* DJ_FP32 or DJ_FP64 */
    double dt;              /* time step [s]; 0 -> dt_factor x critical step (Eq. 14) */
    double dt_factor;       /* <= 0 -> 0.9 */
    double alpha;           /* mass-proportional damping D = alpha M [1/s] (Eq. 13) */
    int32_t allow_unstable_dt;  /* nonzero: accept dt above the critical step */
    int32_t chunk_elems;    /* elements per workgroup tile; 0 -> automatic */
    int32_t variant;        /* step kernel variant 0..5 (threads, elements per thread, register budget);
                               -1: automatic (FP32 H8: 2, otherwise 0) */
    int32_t device;         /* HIP device ordinal; < 0 -> current device */
    int32_t formulation;    /* DJ_FORM_JACOBIAN (0), DJ_FORM_CLASSICAL or DJ_FORM_NODAL_PRESSURE;
                               batches take 0 only */
} djtled_params;

typedef struct djtled_ctx djtled_ctx;
typedef struct djtled_loadset djtled_loadset;

/*
 * djtled_precompute -- Algorithm 1, pre-computation.
 * Validates the mesh, reorders it, and builds on the GPU (FP64) every
 * per-element constant the run time needs: the Jacobian 0J (Eq. 3) and its
 * inverse, whose columns are the shape-function derivatives dh/dX of Eq. 6,
 * the volume 0V, the constant I1m = 2 0V 0J^-T 0J^-1 (Eq. 37) kept through
 * 0J^-1, for DJ_TI / DJ_OT the unit fibres and moduli behind I4m and I6m
 * (Eqs. 45, 46), for DJ_MR the C01 modulus (I2m of Eqs. 40-41 is kept
 * through 0J^-1 as I1m is); for DJ_H8 the hourglass vectors; the lumped nodal
 * masses and the critical step (Eq. 14).  Variants 4 and 5 are built for
 * DJ_NH and DJ_TI; the classical form for FP32 and variants 0..3.
 * On success *out owns every device buffer of the context.
 * Errors: DJ_ERR_ARG, DJ_ERR_BAD_MESH, DJ_ERR_UNSUPPORTED, DJ_ERR_UNSTABLE_DT, DJ_ERR_HIP.
 */
int djtled_precompute(const djtled_mesh *mesh, const djtled_material *material,
                      const djtled_params *params, djtled_ctx **out);

/* Frees the context and its device memory (waits for the device first). */
int djtled_destroy(djtled_ctx *ctx);

typedef struct {
    int32_t n_nodes, n_elems, elem_type, model, precision;
    double dt, dt_crit, alpha;
    int32_t n_chunks, chunk_elems, n_copies, n_shared_copies, grid_blocks, block_threads, variant;
    double bytes_per_step;     /* algorithmic HBM bytes of one fused step */
    double elem_bytes;         /* per-element part of bytes_per_step */
    double mass_total;         /* sum of lumped masses [kg] */
    int32_t formulation;       /* DJ_FORM_JACOBIAN or DJ_FORM_CLASSICAL */
} djtled_info_t;

/* Fills *out with sizes, the time step and the traffic model. */
int djtled_info(const djtled_ctx *ctx, djtled_info_t *out);

/*
 * djtled_forces -- internal nodal forces sum_e F^(e)(u) (Eq. 13), each element
 * force from Table 3, or from Eq. 4 for the classical form (plus hourglass
 * control for H8).  u_dev, f_dev: device,
 * n_nodes x 3.  No boundary condition is applied.  Asynchronous on stream.
 * Errors: DJ_ERR_ARG, DJ_ERR_HIP.
 */
int djtled_forces(djtled_ctx *ctx, const void *u_dev, void *f_dev, void *stream);

/*
 * djtled_forces_noalloc -- djtled_forces for callers that cannot allocate
 * device memory at call time (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, kernels and
 * result (bit for bit) as djtled_forces, but the per-call scratch -- the
 * node-copy displacement planes and the shared-node partial sums --
 * lives in one fixed device array of DJTLED_NOALLOC_SCRATCH_BYTES per GPU,
 * owned by the library and held until the process ends; the call itself
 * makes no allocation.  The array's address on the context's GPU is looked
 * up when the context is created (djtled_precompute).  The scratch needed is
 * 3 x (copies + max(shared-node partial entries, 1)) values of the context's
 * precision (the node copies are at most n_elems x elem_type); a context
 * needing more is refused with DJ_ERR_UNSUPPORTED and a message giving both
 * sizes.  No part of the array needs clearing: every entry a call reads was
 * written earlier in the same call.  All calls on one GPU share the array:
 * calls that overlap in time on one GPU (any contexts, any streams) race and
 * must be ordered by the caller.
 * Errors: DJ_ERR_ARG, DJ_ERR_UNSUPPORTED, DJ_ERR_HIP.
 */
#define DJTLED_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int djtled_forces_noalloc(djtled_ctx *ctx, const void *u_dev, void *f_dev, void *stream);

/*
 * djtled_forces_anp -- djtled_forces with the average nodal pressure (the
 * remedy for volumetric locking of nearly incompressible tissue that Sec. 7
 * names): the volumetric energy sum_n V_n kappa_n (J_n - 1)^2 / 2 lives on
 * the nodes, V_n = sum_e 0V_e / n_e and J_n, kappa_n the 0V_e / n_e-weighted
 * averages of the element volume ratios (Eq. 12) and bulk moduli around n;
 * each element's pressure kappa (J - 1) in Table 3 is replaced by the mean of
 * its nodes' kappa_n (J_n - 1).  The nodal averages are formed in FP64 with a
 * fixed summation order.  DJ_NH / DJ_TI contexts, Jacobian form, variants
 * 0..3; the first call allocates scratch buffers kept by the context.
 * Errors: DJ_ERR_ARG, DJ_ERR_UNSUPPORTED, DJ_ERR_HIP.
 */
int djtled_forces_anp(djtled_ctx *ctx, const void *u_dev, void *f_dev, void *stream);

/* Loads (host memory): displacement boundary conditions and external forces. */
typedef struct {
    int32_t n_bc;
    const int32_t *bc_node;   /* n_bc node indices */
    const int32_t *bc_mask;   /* n_bc masks: bit k set = component k prescribed */
    const double *bc_target;  /* n_bc x 3 target displacement at the end of the ramp */
    int32_t ramp;             /* DJ_RAMP_* : s(t) = 1, t / t_ramp, or the quintic smoothstep */
    double t_ramp;            /* ramp duration [s] */
    const double *R;          /* n_nodes x 3 external nodal forces [N] (Eq. 13), or NULL */
} djtled_loads;

/* Uploads a load case to the device (synchronous).  The load set belongs to
   the context and is freed with it or by djtled_loadset_destroy. */
int djtled_loadset_create(djtled_ctx *ctx, const djtled_loads *loads, djtled_loadset **out);
int djtled_loadset_destroy(djtled_loadset *ls);

/* Caller-owned explicit state: u^n and u^{n-1} (device, n_nodes x 3) and n. */
typedef struct {
    void *u_cur;
    void *u_prev;
    int64_t step;
} djtled_state;

typedef struct {
    int32_t mode;             /* DJ_MODE_FIXED or DJ_MODE_RELAX (dynamic relaxation) */
    double tol;               /* RELAX: stop when the residual is <= tol */
    int32_t check_every;      /* RELAX: residual period in steps (>= 1) */
} djtled_step_opts;

typedef struct {
    int32_t code;             /* DJ_OK, DJ_CONVERGED or DJ_ERR_* */
    int32_t steps_done;       /* steps completed by this call */
    int64_t error_step;       /* global step of a run-time error, else -1 */
    int32_t error_elem;       /* caller element index of DJ_ERR_INVERTED, else -1 */
    double residual;          /* last residual evaluated (RELAX), else NaN */
    double kernel_ms;         /* device time of the persistent step kernel (HIP events on `stream`) */
} djtled_status;

/*
 * djtled_step -- n_steps explicit steps of Eq. 13 in ONE persistent kernel
 * launch: per step, element forces (Table 3) -> node reduction -> central
 * difference with damping -> displacement BCs, with one grid barrier per step.
 *   u^{n+1} = u^n + B' (u^n - u^{n-1}) + A_i (R_i - F_i(u^n)),
 *   B' = (2 - alpha dt) / (2 + alpha dt),  A_i = 2 dt^2 / ((2 + alpha dt) m_i),
 * then prescribed components are set to s(t_{n+1}) * target.
 * RELAX: every check_every steps, once the ramp is complete, the residual
 * |(F - R)_free|_2 / |F_constrained|_2 of u^n is evaluated and the run stops
 * without advancing when it is <= tol (code DJ_CONVERGED); with no reaction force the residual is taken as
 * infinite (it is relative to the reaction), so a run never stops there.
 * On return state->u_cur / u_prev / step hold the last completed step; on
 * DJ_ERR_INVERTED, and on DJ_ERR_NONFINITE found in an element, that is the
 * step before the failing one.  A non-finite displacement produced at a node
 * shared by several workgroup tiles is found only after the step that made
 * it: that step then counts as done, the state holds the non-finite value and
 * error_step names the step that produced it.  loads may be NULL
 * (free body, no external force).  Synchronises `stream` to read the status.
 */
int djtled_step(djtled_ctx *ctx, djtled_state *state, const djtled_loadset *loads, int32_t n_steps,
                const djtled_step_opts *opts, djtled_status *out, void *stream);

/*
 * djtled_step_multi -- djtled_step for nrhs (1..8) load cases of the same
 * mesh, material and time step in one persistent launch (Eq. 13 for each
 * case): per step the element phase of every case, one grid barrier for all
 * of them, then their shared-node phases.  Each case has its own state,
 * boundary values and node sums, and its result equals a separate
 * djtled_step call bit for bit.
 *   state: u_cur and u_prev each hold nrhs consecutive n_nodes x 3 arrays
 *          (device); one step counter for all cases;
 *   loads: nrhs load sets of this context sharing the ramp kind and
 *          duration, or NULL (no loads for any case).
 * RELAX: the run stops when every case's residual is <= tol.  out->residual
 * is the largest of the cases' last residuals; residuals (nrhs doubles, host,
 * may be NULL) receives each.  An error in any case stops every case at the
 * same step; *error_case (may be NULL) names the case, else -1.
 * Built for FP32 contexts with the Jacobian form and variants 0..3 (nrhs > 1).
 * Errors: as djtled_step; DJ_ERR_ARG for nrhs out of range, missing or
 * mismatched load sets; DJ_ERR_UNSUPPORTED for other contexts.
 */
int djtled_step_multi(djtled_ctx *ctx, int32_t nrhs, djtled_state *state, const djtled_loadset *const *loads,
                      int32_t n_steps, const djtled_step_opts *opts, djtled_status *out, double *residuals,
                      int32_t *error_case, void *stream);

/*
 * djtled_export_constants -- copies per-element constants to host memory in
 * caller element order, in FP64: V[n_elems], dhdX[n_elems x 3 x elem_type]
 * (row i = d h_a / d X_i, Eq. 6), and the lumped masses mass[n_nodes] in
 * caller node order.  Any output pointer may be NULL.  Synchronous.
 */
int djtled_export_constants(djtled_ctx *ctx, double *V, double *dhdX, double *mass);

/* ------------------------------------------------------------------------
 * Batches: many independent meshes ("instances") of uneven sizes advanced
 * together.  Each instance is a mesh + material + load case as above, with its
 * own critical step (dt = dt_factor x its Eq. 14 bound), its own damping and
 * its own ramp; all instances take the same number of steps per run.  The
 * instances of each element kind ((T4 | H8) x (NH | TI)) are laid out side by
 * side, and every run advances all of them with ONE persistent kernel (one
 * grid barrier per step for the whole batch), replayed from a captured
 * hipGraph.  The batch owns the state of every instance (initially u = 0 at
 * step 0).  External forces R are not supported in batches (loads[i].R must be
 * NULL); batches take the DJ_NH and DJ_TI models; all instances of a kind
 * share rho and hg_kappa.  In a batch, a
 * negative loads[i].t_ramp means a ramp of |t_ramp| steps of the instance's
 * own dt.
 * ------------------------------------------------------------------------ */
typedef struct djtled_batch djtled_batch;

typedef struct {
    int32_t autotune;          /* nonzero: choose variant, chunk size and steps per launch by timing
                                  candidates on a sample of the instances */
    int32_t variant;           /* batch kernel variant when not tuning (FP32: 0..8, 4..7 stage element data
                                  in LDS by prefetch, 8 runs two workgroups per compute unit;
                                  FP64: 0); <0 -> default */
    int32_t chunk_elems;       /* elements per workgroup tile when not tuning; 0 -> kernel capacity */
    int32_t steps_per_launch;  /* persistent-launch length inside a run; 0 -> the whole run */
    int32_t use_graph;         /* nonzero: each run replays a captured hipGraph */
    int32_t tune_steps;        /* steps timed per candidate; 0 -> 20 */
} djtled_tune;

typedef struct {
    int32_t n_inst, n_kinds, n_items, grid_blocks, block_threads, variant, chunk_elems, steps_per_launch;
    int32_t graph;             /* 1: the last run replayed a hipGraph */
    int32_t tune_candidates;   /* candidates timed by the autotuner (0: not tuned) */
    int64_t n_elems, n_nodes;  /* totals over the instances */
    double bytes_per_step;     /* algorithmic HBM bytes of one batch step */
    double tune_ms;            /* host wall time spent autotuning */
    int32_t error_inst;        /* instance of the last run-time error, else -1 */
} djtled_batch_info_t;

/*
 * djtled_batch_create -- pre-computation (as djtled_precompute) of n instances
 * and the batch's work list.  meshes/materials/loads: n entries each (host);
 * alpha: n damping coefficients or NULL (-> params->alpha); params: precision,
 * dt_factor (dt must be 0), allow_unstable_dt, device; tune may be NULL.
 * Errors: DJ_ERR_ARG, DJ_ERR_BAD_MESH, DJ_ERR_UNSUPPORTED, DJ_ERR_UNSTABLE_DT, DJ_ERR_HIP.
 */
int djtled_batch_create(int32_t n, const djtled_mesh *meshes, const djtled_material *materials,
                        const djtled_loads *loads, const double *alpha, const djtled_params *params,
                        const djtled_tune *tune, djtled_batch **out);
int djtled_batch_destroy(djtled_batch *b);
int djtled_batch_info(const djtled_batch *b, djtled_batch_info_t *out);

/* Per-instance sizes and step (n_nodes, n_elems, elem_type, model, precision, dt, dt_crit, alpha). */
int djtled_batch_instance(const djtled_batch *b, int32_t inst, djtled_info_t *out);

/*
 * djtled_batch_run -- n_steps explicit steps of Eq. 13 for every instance
 * (forces of Table 3 -> node sums -> central difference with damping -> BCs
 * ramped per instance).  out->kernel_ms: device time of the run;
 * out->error_elem: caller element (within djtled_batch_info's error_inst) of a
 * DJ_ERR_INVERTED.  On an error every instance stops at the last completed
 * step.  Synchronises `stream`.
 */
int djtled_batch_run(djtled_batch *b, int32_t n_steps, djtled_status *out, void *stream);

/* Device time from the start of the last run to the end of each instance's
   last step (instance order), from per-workgroup time stamps [ms]. */
int djtled_batch_stats(const djtled_batch *b, double *inst_ms);

/* Copy the state (u^n, u^{n-1}; device, n_nodes x 3 of the instance, caller
   node order, batch precision) of one instance out of / into the batch.
   u_prev may be NULL (read: skipped; write: u^{n-1} = u^n).  Asynchronous. */
int djtled_batch_read(djtled_batch *b, int32_t inst, void *u_cur, void *u_prev, void *stream);
int djtled_batch_write(djtled_batch *b, int32_t inst, const void *u_cur, const void *u_prev, void *stream);

/* Every instance back to u = 0 at step 0. */
int djtled_batch_reset(djtled_batch *b, void *stream);

/* Thread-local description of the last error on this thread ("" if none). */
const char *djtled_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DJTLED_H */
