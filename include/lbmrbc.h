/*
 * lbmrbc.h -- C ABI of the MI355X (gfx950) reactive lattice Boltzmann library.
 *
 * One fused time step advances two coupled lattices on one GPU:
 *   - a fluid population f_i: BGK collision with the second-order equilibrium
 *     (Weinmiller et al., Sec. 2.1, eqs. fluid_BGK, fluid_Equilib,
 *     fluid_BGK_visc), halfway bounce-back at solid neighbours, Guo body force;
 *   - a solute population g_i: advection-diffusion BGK with the linear
 *     equilibrium g_eq = C w_i (1 + u.e_i / c_s^2), u taken from the fluid at
 *     the same node and step (Sec. 2.1, eqs. solute_BGK,
 *     solute_equilibrium_function, solute_diffu), with the rest-fraction
 *     weights (Sec. 2.2, eqs. RestFraction, RestFractionCs2), on the fluid's
 *     velocity set or on the paper's reduced D2Q5 / D3Q7 (appendix, velocity
 *     sets; params.solute_q);
 *   - the general reactive boundary condition on every link that enters a
 *     fluid node from a solid node (Sec. 2.3, eq. general_RBC with the k_i of
 *     eqs. k_i_S_Ve, k_i_S2, k_i_S_New and gamma of eq. gammaAppendix);
 *   - the solid-fraction update of each interface node from the mass that
 *     crossed its reactive links (Sec. 2.4, eq. solidFractionUpdate), in FP64,
 *     and the phase-change thresholds phi = 0 / phi = 1 (Sec. 2.4).
 *
 * Conventions
 *   - Nodes are indexed n = x + nx*(y + ny*z) (x fastest).  2D uses nz = 1.
 *   - All array arguments are DEVICE pointers unless stated otherwise, and are
 *     owned by the caller.  The library never frees them.  The only device
 *     memory the library uses is the caller's workspaces (lbm_create,
 *     lbm_record) and one static array per GPU (lbm_record_static).
 *   - All device work is enqueued, in order, on the HIP stream given to
 *     lbm_create (NULL = the legacy default stream).  Only lbm_get_diag,
 *     lbm_set_geometry and lbm_create synchronise that stream.
 *   - Every function returns an lbm_status.  Errors never cross the ABI as
 *     exceptions.  An argument error leaves the context unchanged; the text of
 *     the last error is available from lbm_last_error.
 *   - Not thread-safe per context.  Distinct contexts are independent.
 */
#ifndef LBMRBC_H
#define LBMRBC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* invalid argument or parameter                      */
    LBM_ENOMEM = -2,     /* workspace too small                                */
    LBM_EDEVICE = -3,    /* HIP runtime error (message names the call)         */
    LBM_ESTATE = -4,     /* call out of order (e.g. step before set_geometry)  */
    LBM_ENUMERIC = -5,   /* non-finite population detected                     */
    LBM_ECAPACITY = -6   /* reactive links exceed params.max_links             */
} lbm_status;

/* precision: storage and arithmetic of the populations */
#define LBM_FP64 0       /* FP64 populations                                    */
#define LBM_FP32_DEV 1   /* FP32 deviations f - w_i rho0, g - w_i C_ref; the
                            solid fraction and the mass sums stay FP64        */

/* source population of the reactive boundary condition (the paper's g~_i) */
#define LBM_PRECOLL 0    /* pre-collision population at the fluid boundary node,
                            streamed toward the wall this step (default)      */
#define LBM_POSTCOLL 1   /* the node's own post-collision population that
                            streamed into the wall (halfway, link-wise)       */

/* collision operator of both lattices */
#define LBM_BGK 0        /* single relaxation time (Sec. 2.1, eqs. fluid_BGK,
                            solute_BGK)                                       */
#define LBM_TRT 1        /* two relaxation times with the magic parameter 3/16
                            (Sec. 2.1, eqs. fluid_TRT, solute_TRT): fluid even
                            parts relax with tau_ns, odd parts with tau-; the
                            solute's odd parts with tau_ad, even parts with
                            tau-; the Guo force term is split the same way
                            (the adjoint transposes either operator).      */

/* k_i of the reactive boundary condition */
#define LBM_SNEW 0       /* c_s^-2 gamma k_r (e.n)   -- the paper's new scheme  */
#define LBM_SV 1         /* c_s^-2 k_r (e.n)         -- Verhaeghe              */
#define LBM_SPJ 2        /* c_s^-2 gamma k_r / (e.n) -- Patel / Ju             */
#define LBM_ABB 3        /* k_i = infinity: anti-bounce-back with C_eq at solid
                            nodes with k_r > 0 (k_r = 0: bounce-back)          */

typedef struct {
    int32_t dim;              /* 2 or 3                                            */
    int32_t nx, ny, nz;       /* lattice size; nz = 1 when dim = 2                 */
    int32_t fluid_q;          /* 9 (D2Q9) or 19 (D3Q19)                            */
    int32_t solute_q;         /* fluid_q, or 5 (D2Q5, with D2Q9) / 7 (D3Q7, with
                                 D3Q19): the solute's velocity set.  D2Q5 is the
                                 rest vector and the four axis vectors in the
                                 paper's appendix order; D3Q7 the rest vector,
                                 +x, +y, +z, -x, -y, -z.  On these sets w_0 = J0,
                                 w_i = c_s^2/2, c_s^2 = (1 - J0)/dim (J0 = 1/3
                                 resp. 1/4 when j0 < 0), and reactive links exist
                                 along their directions only.                   */
    int32_t precision;        /* LBM_FP64 | LBM_FP32_DEV                           */
    int32_t rbc_mechanics;    /* LBM_PRECOLL | LBM_POSTCOLL                        */
    int32_t rbc_scheme;       /* LBM_SNEW | LBM_SV | LBM_SPJ | LBM_ABB             */
    double tau_ns;            /* fluid relaxation time, > 1/2                      */
    double tau_ad;            /* solute relaxation time, > 1/2                     */
    double j0;                /* rest fraction in [0,1); < 0: standard weights.  On
                                 D2Q9 / D3Q19 w_0 = J0 and the moving weights
                                 and c_s^2 scale by (1 - J0)/(1 - w_0,std)     */
    double force[3];          /* body force on the fluid (lattice units)           */
    double rho0;              /* FP32_DEV reference density (ignored in FP64)      */
    double c_ref;             /* FP32_DEV reference concentration (ignored in FP64)*/
    double c_eq;              /* equilibrium concentration of the reaction         */
    double k_r;               /* uniform rate constant (when no per-node field)    */
    double v_m;               /* dimensionless molar volume                         */
    double a_m;               /* specific surface area (the paper uses 1)          */
    int32_t periodic[3];      /* fluid periodicity per axis                        */
    int32_t xwrap_shift_y;    /* site (x+nx, y) is site (x, y+shift); needs
                                 periodic[0] and periodic[1]                        */
    int32_t inlet_axis;       /* -1: none; else the solute sees this axis as
                                 non-periodic with a fixed-concentration inlet at
                                 coordinate 0 and a zero-gradient outlet at n-1    */
    double c_in;              /* inlet concentration                                */
    int32_t phase_change;     /* 1: apply the phi thresholds after each step
                                 (Sec. 2.4; single-lattice contexts; lbm_step
                                 then queues up to 32 steps at a time, the
                                 steps after one that crossed a threshold doing
                                 nothing, and synchronises once per batch and
                                 after every event pass).  One pass
                                 takes at most 65536 events (and as many nodes
                                 pushed over a threshold by earlier events of
                                 the pass); beyond that lbm_step returns
                                 ECAPACITY                                   */
    int32_t collision;        /* LBM_BGK | LBM_TRT                                 */
    int64_t max_links;        /* capacity for reactive links; <= 0 selects
                                 max(4096, N*(Q-1)/4)                              */
    int32_t fluid_open;       /* 1: open channel along inlet_axis (Sec. 3.3's
                                 channel flow; needs inlet_axis >= 0 and that axis
                                 not periodic): at the inlet face an incoming
                                 fluid population is the node's own opposite one
                                 plus 2 w_i rho_out (e_i.u_in)/c_s^2 (a wall
                                 moving with the plug velocity), at the outlet
                                 face minus that one plus 2 w_i rho_out (density
                                 rho_out, O(u^2) terms dropped).  0: the box faces
                                 of that axis are bounce-back walls            */
    int32_t ceq_field;        /* 1: the equilibrium concentration of the reaction
                                 varies per solid node, given by lbm_set_ceq
                                 (8 B per node and ts per link of workspace);
                                 0: c_eq everywhere                              */
    double u_in;              /* plug velocity along +inlet_axis                   */
    double rho_out;           /* outlet density (> 0)                              */
} lbm_params;

typedef struct {
    int64_t step;             /* steps taken since lbm_init_fields                 */
    int64_t n_events;         /* phase-change events applied                       */
    int64_t n_links;          /* reactive links of the current geometry            */
    int64_t n_solid_iface;    /* solid nodes with at least one reactive link       */
    int64_t n_fluid;          /* fluid nodes                                       */
    int64_t n_fluid_iface;    /* fluid nodes with at least one reactive link       */
    double mass_c;            /* sum of C over fluid nodes (FP64)                  */
    double phi_sum;           /* sum of phi over all nodes (FP64)                  */
    double wall_exchange;     /* cumulative mass entering the fluid over reactive
                                 links since lbm_init_fields (FP64)               */
    int32_t nan_flag;         /* 1 if any population is non-finite                 */
    int32_t reserved0;
    double inlet_exchange;    /* cumulative mass entering the fluid across the
                                 inlet plane since lbm_init_fields: per step and
                                 inlet link the incoming equilibrium value minus
                                 the node's own population leaving along the
                                 opposite direction (FP64; 0 without an inlet) */
    double outlet_exchange;   /* the same across the outlet plane (the
                                 zero-gradient copy minus the population leaving);
                                 negative when mass leaves.  With no events,
                                 sum C + sum phi / (V_m a_m) changes by exactly
                                 inlet_exchange + outlet_exchange (Sec. 2.4,
                                 eq. solidFractionUpdate); a batch reports the
                                 totals over its domains                      */
    int64_t n_tasks;          /* wavefront tasks of the fused step (each up to 64
                                 consecutive fluid nodes)                      */
    int64_t n_row_words;      /* 64-node row words of the geometry (the step
                                 reads them to find its neighbours)           */
} lbm_diag;

/* Workspace size in bytes for these parameters (host call, no device work).
 * EINVAL on invalid parameters. */
lbm_status lbm_workspace_bytes(const lbm_params *params, size_t *bytes);

/* Create a context on the current HIP device.  dev_workspace: device memory of
 * at least lbm_workspace_bytes, 256-byte aligned, owned by the caller and kept
 * alive until lbm_destroy.  hip_stream: a hipStream_t (NULL = default).
 * EINVAL: bad parameters; ENOMEM: workspace too small. */
lbm_status lbm_create(const lbm_params *params, void *dev_workspace, size_t bytes,
                      void *hip_stream, lbm_ctx **out);

/* Batches (many independent domains advanced by the same launches).
 * The domains share dim, lattice and precision; everything else (size,
 * relaxation times, rest fraction, force, rate constants, boundary settings)
 * is per domain.  All per-node arrays of a batch context (geometry, fields,
 * populations [Q][N], exchange [N][Q]) are the domains' arrays concatenated in
 * domain order; lbm_batch_offsets gives the first node of each domain.  A
 * single-domain context is a batch of one.  Phase change is not available in
 * a batch (EINVAL). */
lbm_status lbm_batch_workspace_bytes(const lbm_params *per_domain, int32_t n, size_t *bytes);
lbm_status lbm_create_batch(const lbm_params *per_domain, int32_t n, void *dev_workspace,
                            size_t bytes, void *hip_stream, lbm_ctx **out);
/* node_off: host array of n + 1 entries (the last is the total node count) */
lbm_status lbm_batch_offsets(const lbm_ctx *ctx, int64_t *node_off);

/* Geometry prep (per geometry, not per step): node classes, reactive link
 * list with k_i per link (Sec. 2.3), solid-side link lists.
 *   solid   [N]    uint8, nonzero = solid (required)
 *   normals [N][3] FP64 unit normals pointing from solid into fluid, read at
 *                  solid nodes (NULL: lattice-gradient normals of the solid
 *                  indicator)
 *   k_r     [N]    FP64 rate constant per solid node (NULL: params.k_r)
 *   phi0    [N]    FP64 initial solid fraction (NULL: 1 at solid, 0 at fluid)
 * Synchronises the stream.  ECAPACITY if the links exceed max_links (the
 * message gives the count needed). */
/* Per-node equilibrium concentration of the reaction (contexts created with
 * ceq_field = 1; EINVAL otherwise): c_eq [N] FP64 device, the value at each
 * solid node is the C_eq of eq. general_RBC on that node's reactive links
 * (fluid entries are ignored).  Copied into the workspace by an asynchronous
 * copy on the context stream (c_eq must stay valid until the stream reaches
 * it; lbm_set_geometry, which synchronises, is the next call in the usual
 * order); takes effect at the next lbm_set_geometry (call it first) and in
 * every relink after phase change.  Until it is called, params.c_eq holds
 * everywhere.  The per-node field is not part of a saved state.  Not with
 * lbm_record / lbm_adjoint. */
lbm_status lbm_set_ceq(lbm_ctx *ctx, const double *c_eq);

lbm_status lbm_set_geometry(lbm_ctx *ctx, const uint8_t *solid, const double *normals,
                            const double *k_r, const double *phi0);

/* Equilibrium initial state of (rho, u, C) at every fluid node, written as the
 * post-collision populations.  rho [N], u [N][3], c [N] FP64; NULL = 1, 0, 0.
 * Resets the step counter and the cumulative exchange. */
lbm_status lbm_init_fields(lbm_ctx *ctx, const double *rho, const double *u,
                           const double *c);

/* Advance nsteps fused time steps (asynchronous; with phase_change = 1 it
 * synchronises once per batch of up to 32 steps and after each event pass,
 * which it runs after the step that crossed a threshold, Sec. 2.4). */
lbm_status lbm_step(lbm_ctx *ctx, int32_t nsteps);

/* lbm_step with per-kernel timing, for measurement: runs nsteps exactly like
 * lbm_step, records a HIP event pair around every kernel launch on the
 * context stream, synchronises, and writes the summed kernel durations in
 * milliseconds: ms[0] the fused step kernel, ms[1] the solid-fraction kernel
 * (host array of 2).  Results are identical to lbm_step. */
lbm_status lbm_step_timed(lbm_ctx *ctx, int32_t nsteps, double *ms);

/* Launch configuration of the step (a performance choice only: every
 * configuration gives bit-identical populations and solid fractions).
 *   wg_waves    tasks (wavefronts of up to 64 fluid nodes) per workgroup:
 *               1, 2, 4 or 8 (default 4); contexts with fluid_open or
 *               ceq_field always run 4 (the autotuner tries no other)
 *   xcd_remap   1: consecutive tiles of tasks run on one XCD, so that the rows
 *               they share stay in one L2 (default 1); 0: plain order
 *   graph_steps 0: lbm_step issues two kernel launches per step (default);
 *               > 0: lbm_step replays a HIP graph holding graph_steps steps
 *               (rounded up to even), built on first use and rebuilt after a
 *               geometry or configuration change; remaining steps run as
 *               plain launches.  Graph objects are the only device-side
 *               allocation the library makes (besides the static array of
 *               lbm_record_static); lbm_destroy frees them.
 *   overlap     1: the solid-side solid-fraction kernel of a step runs on a
 *               second stream of the library, concurrently with the next
 *               step's fused kernel (two exchange buffers); every lbm_step
 *               call still ends ordered on the context stream.  0: both
 *               kernels on the context stream (default).  Ignored with
 *               phase_change = 1. */
typedef struct lbm_launch_config {
    int32_t wg_waves;
    int32_t xcd_remap;
    int32_t graph_steps;
    int32_t overlap;
} lbm_launch_config;

/* EINVAL for values outside the ranges above. */
lbm_status lbm_set_launch_config(lbm_ctx *ctx, const lbm_launch_config *cfg);
lbm_status lbm_get_launch_config(const lbm_ctx *ctx, lbm_launch_config *cfg);

/* Autotuner: times every (wg_waves, xcd_remap) pair over trial_steps plain
 * steps, then overlap on and off for the best pair, then graph replay at
 * graph_steps in {16, 64, 256} (each <= 4 * trial_steps) against plain
 * launches, with HIP events on the
 * context stream, and keeps the fastest configuration.  The trial steps are
 * real steps of the simulation (the step counter advances by the number
 * written to *steps_run); results do not depend on the configuration.
 * best (host, may be NULL) receives the chosen configuration and ms_per_step
 * (host, may be NULL) its time per step.  Synchronises. */
lbm_status lbm_autotune(lbm_ctx *ctx, int32_t trial_steps, lbm_launch_config *best,
                        double *ms_per_step, int64_t *steps_run);

/* Adjoint (reverse-mode gradient) of a loss on the final concentrations with
 * respect to the rate constants k_r of the solid nodes (Sec. 2.3: k enters
 * every reactive link through eqs. k_i_S_Ve, k_i_S2, k_i_S_New and
 * eq. general_RBC).  The fluid does not depend on k_r; the adjoint covers a
 * fluid at rest (pure reaction-diffusion): single-lattice contexts with no
 * body force, inlet_axis = -1, phase_change = 0 and a uniform c_eq (EINVAL
 * otherwise, and
 * lbm_record checks that no fluid node carries momentum).
 *
 * lbm_adjoint_workspace_bytes: device bytes that lbm_record needs for nsteps
 *   steps with a solute checkpoint every ckpt_every steps (1 <= ckpt_every <=
 *   nsteps) on the current geometry: ceil(nsteps/ckpt_every) + 4 solute
 *   states, ckpt_every per-link source values (one storage element per
 *   reactive link and step of a segment; twice that when the run has more
 *   than one segment, so that lbm_adjoint recomputes the next segment on a
 *   second stream while it applies the transposed steps of the current one)
 *   and 8 B per reactive link of capacity.
 * lbm_record: runs nsteps steps exactly as lbm_step does and keeps the
 *   checkpoints in dev_workspace (caller-owned, 256-byte aligned, untouched
 *   by anything else until lbm_adjoint has run).
 * lbm_adjoint: dL_dC [N] FP64 device, dL/dC_T at every node (C_T the final
 *   concentration, sum of the post-collision populations; solid entries are
 *   ignored); writes grad_k [N] FP64 device, dL/dk_r at every solid node that
 *   has a reactive link (0 elsewhere).  ESTATE unless the context is exactly
 *   at the end of the recorded run with the same geometry.  The state is not
 *   changed; the call is asynchronous on the context stream. */
lbm_status lbm_adjoint_workspace_bytes(const lbm_ctx *ctx, int32_t nsteps, int32_t ckpt_every,
                                       size_t *bytes);
lbm_status lbm_record(lbm_ctx *ctx, int32_t nsteps, int32_t ckpt_every, void *dev_workspace,
                      size_t bytes);
lbm_status lbm_adjoint(lbm_ctx *ctx, const double *dL_dC, double *grad_k);

/* lbm_adjoint with per-kernel timing, for measurement: the same gradient
 * (bit for bit), with a HIP event pair around every kernel launch of the
 * backward pass; synchronises after each.  ms (host array of 3) receives the
 * summed durations in milliseconds of the segment recomputation (solute-only
 * forward steps), of the transposed steps, and of the per-segment folds of
 * the transposed steps' dL/dbeta terms into the FP64 totals. */
lbm_status lbm_adjoint_timed(lbm_ctx *ctx, const double *dL_dC, double *grad_k, double *ms);

/* lbm_record without a workspace, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The checkpoints and the adjoint's working arrays live in
 * a device array inside the library, LBM_STATIC_SCRATCH_BYTES per GPU, held
 * from the library's load until the process ends.  Same run, same results
 * and same lbm_adjoint as lbm_record; the steps run as plain kernel launches
 * on the context stream (no graph, no second stream), and nothing is
 * allocated.
 *   ENOMEM if lbm_adjoint_workspace_bytes(ctx, nsteps, ckpt_every) exceeds
 *   LBM_STATIC_SCRATCH_BYTES (the message gives both sizes); the other
 *   errors as lbm_record.
 * One array per GPU, shared by every context on it: each call overwrites the
 * previous call's contents, and lbm_adjoint of a context whose static record
 * has since been overwritten returns ESTATE.  Calls on one GPU (and their
 * lbm_adjoint) must not overlap in time: concurrent use of the array races. */
#define LBM_STATIC_SCRATCH_BYTES (64ull << 20)
lbm_status lbm_record_static(lbm_ctx *ctx, int32_t nsteps, int32_t ckpt_every);

/* Macroscopic fields of the current state (asynchronous; NULL skips a field):
 * rho = sum f, u = (sum e f - F/2)/rho, C = sum g (the values that entered
 * the last collision), phi, type (1 = solid).  rho/c/phi [N], u [N][3] FP64,
 * type [N] uint8.  Solid nodes read rho = u = C = 0. */
lbm_status lbm_get_fields(lbm_ctx *ctx, double *rho, double *u, double *c, double *phi,
                          uint8_t *type);

/* Post-collision populations as absolute FP64 values (NULL skips): f
 * [fluid_q][N] in the fluid set's order, g [solute_q][N] in the solute set's
 * order. */
lbm_status lbm_get_pops(lbm_ctx *ctx, double *f, double *g);

/* Mass that crossed each reactive link in the last step, scattered to a dense
 * [N][fluid_q] FP64 array indexed by fluid direction (zero where there is no
 * link, e.g. along a direction outside a reduced solute set; all zero after a
 * step whose phase change rebuilt the link list). */
lbm_status lbm_get_exchange(lbm_ctx *ctx, double *q);

/* FP64 reductions of the current state (host struct; synchronises).
 * Returns ENUMERIC when a non-finite population is present. */
lbm_status lbm_get_diag(lbm_ctx *ctx, lbm_diag *out);

/* Full state (populations, phi, geometry arrays, counters) to/from a caller
 * device buffer of lbm_state_bytes. */
lbm_status lbm_state_bytes(const lbm_ctx *ctx, size_t *bytes);
lbm_status lbm_save_state(lbm_ctx *ctx, void *dev_buf, size_t bytes);
lbm_status lbm_load_state(lbm_ctx *ctx, const void *dev_buf, size_t bytes);

/* Text of the last error on this context (valid until the next call on it);
 * with ctx = NULL, the last error of a failed lbm_create. */
const char *lbm_last_error(const lbm_ctx *ctx);

/* Release host state.  The caller's workspace is not touched. */
void lbm_destroy(lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBMRBC_H */
