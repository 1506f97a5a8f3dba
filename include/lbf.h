/*
 * lbf.h -- C ABI of the MI355X lattice-Boltzmann library for flow and
 * advection-diffusion-reaction (ADR) through 2D cross-sections of catalytic
 * fibres.
 *
 * The method is the hybrid scheme of Sitaru & Gekle, "Analytical and
 * computational study of cascade reaction processes in catalytic fibrous
 * membranes" (arXiv 2109.04455):
 *   1. a stationary flow field from a lattice-Boltzmann Navier-Stokes solve
 *      (Sec. "Lattice-Boltzmann for the Navier-Stokes equation", Eq. LBE),
 *      here a D2Q9 BGK channel with a parabolic Zou-He velocity inlet, a
 *      Zou-He pressure outlet (rho = 1) and half-way bounce-back at solids;
 *   2. a D2Q5 BGK lattice-Boltzmann ADR solve on the frozen, linearly scaled
 *      velocity (Sec. "Lattice-Boltzmann for Advection-Diffusion-Reaction",
 *      Eqs. LBE_ADE, BGK, the second-order equilibrium, Diffusion_LBM), with
 *      first-order A->B and B->C sources (Eq. source_lbm) applied only to the
 *      populations that stream into a catalytic node;
 *   3. anti-bounce-back inlet (C_A = c_in; bounce-back for B and C) and
 *      zero-gradient outlet (C_w = C_b), Eq. BC, and the outlet fluxes through
 *      the face between columns flux_col and flux_col + 1 (Sec. "Boundary
 *      conditions and flux computation in ADE");
 *   4. the efficiency eps = N_B/(N_A+N_B) or N_C/(N_A+N_B+N_C) (Eq. A-B).
 *
 * Conventions
 *   - Grid x in [0,nx), y in [0,ny), row-major [ny][nx] with x fastest.
 *     Rows y = 0 and y = ny-1 must be solid (channel walls).
 *   - node_type: 0 fluid, 1 inert solid, 2 catalyst type 1 (A->B),
 *     3 catalyst type 2 (B->C).  With nspecies = 2 type-3 nodes are inert.
 *   - Every function returns an lbf_status; no C++ exception crosses the ABI.
 *   - Device pointers are owned by the caller (e.g. allocated by PyTorch);
 *     the library never allocates or frees device memory itself: all its
 *     buffers live in the caller's workspace (lbf_bind) or adjoint scratch.
 *   - All device work is enqueued on the stream given to lbf_bind.  Calls that
 *     return host values synchronise that stream.  A context is not
 *     thread-safe; distinct contexts are independent.
 *   - "Real" is float when real_bytes = 4 and double when real_bytes = 8.
 *   - A step of the library advances the pre-collision state by one time
 *     step: stream (with boundary rules) then collide and react.  After n
 *     steps the observables (fluxes, concentrations) are those of the state
 *     reached after n full time steps of the paper's scheme.
 */
#ifndef LBF_H
#define LBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBF_OK = 0,
    LBF_EINVAL = -1,     /* invalid argument (see lbf_last_error)                  */
    LBF_ENOMEM = -2,     /* workspace too small                                    */
    LBF_EHIP = -3,       /* HIP runtime error (message in lbf_last_error)          */
    LBF_ENOTCONV = -4,   /* step budget exhausted before the tolerance; state valid */
    LBF_EDIVERGED = -5,  /* non-finite flux or velocity detected                   */
    LBF_ESTATE = -6      /* call out of order (e.g. no step taken yet)             */
} lbf_status;

typedef struct lbf_ctx_s *lbf_ctx;

typedef struct {
    int nx, ny;          /* lattice size incl. wall rows; nx >= 8, ny >= 3           */
    int real_bytes;      /* 4 (FP32 state, FP64 reductions) or 8 (FP64)              */
    int nspecies;        /* 2: A->B, 3: cascade A->B->C                              */
    int reaction_mode;   /* 0: link reaction (only the population streaming into a
                            catalytic node reacts, rate of that node);  1: the
                            node variant compared in Sec. "Lattice-Boltzmann for
                            Advection-Diffusion-Reaction": every population of a
                            fluid node next to catalysts reacts, with the mean rate
                            of its catalytic neighbours of each type               */
    double tau_f;        /* D2Q9 relaxation time, > 0.5                              */
    double u0;           /* inlet centre-line velocity of the flow, |u0| < 0.3       */
    double tau_g;        /* D2Q5 relaxation time, > 0.5; D = (tau_g - 1/2)/3         */
    double c_in;         /* inlet concentration of A                                 */
    double vel_scale;    /* ADR velocity = vel_scale * flow velocity (linear scaling) */
    int flux_col;        /* outlet flux face between flux_col and flux_col+1; -1: nx-3 */
    int tile_x, tile_y;  /* thread-block shape (threads) of the ADR step; 0: default */
    int variant;         /* ADR kernel: 0 auto (one node per thread in FP32, 16-byte
                            vectors of 2 nodes in FP64), 1 one node per thread,
                            2 16-byte vectors (4 FP32 or 2 FP64 nodes per thread)   */
    int flags;           /* bit 0: disable the XCD-aware block order; bit 1: cached
                            instead of streaming (non-temporal) population accesses;
                            bit 2: store species A unshifted in FP32 (rejected
                            together with bit 4, LBF_EINVAL: the A field error
                            then reaches ~2e-4 of its maximum on a 512 x 128
                            cascade, against ~1e-6 shifted); bit 3 (batch):
                            one-step ADR launches take one block per tile instead
                            of the persistent tile walk (the batched flow always
                            takes one block per tile);
                            bit 4: FP32 arithmetic for FP32 storage (default: each
                            node update computes in FP64, rounding once per store);
                            bit 5: FP32 arithmetic in the flow step only.
                            Bits 4 and 5 are experimental: both stay within 1e-4
                            of the FP64 oracle over a few thousand steps but not
                            at a steady state (2048 x 512 cascade converged: bit 4
                            eps error 2.9e-3 and field error 2.0e-3, bit 5 field
                            error 1.2e-4; the default FP64 arithmetic 5e-8 and
                            4.5e-6);
                            bit 6: streaming accesses even when the lattice fits
                            the 256 MiB last-level cache (default there: cached);
                            bit 7: 64-bit population offsets in the flow and ADR
                            node updates (default: 32-bit offsets through buffer
                            descriptors while the 9-plane flow lattice is below
                            4 GiB, 64-bit beyond; results are identical);
                            bit 8: one ADR step per launch (default: steps of a
                            link-reaction channel run two per launch, the
                            intermediate state kept in LDS; the last step of
                            every block is a single one); the adjoint's steps
                            likewise, and the flow's (default: two per launch
                            on lattices of at least 2^18 nodes with FP64
                            arithmetic, an odd block ending in a single step;
                            results equal to one step per launch bit for bit);
                            bit 9: untraced two-step launches by wavefronts that
                            march along y with the intermediate rows in
                            registers instead of the LDS tile (FP32 storage with
                            FP64 arithmetic; results identical, slower on this
                            part) */
    int boundary;        /* 0: channel (solid rows 0 and ny-1, inlet at x = 0,
                            outlet at x = nx-1); 1: box periodic in x and y with no
                            inlet or outlet (ADR only: no flow solve, no fluxes,
                            no adjoint; the velocity comes from lbf_set_velocity) */
} lbf_params;

/* Fill *p with defaults for an nx x ny lattice (FP32, 3 species, link
 * reactions, channel, tau_f 0.8, u0 0.05, tau_g 0.8, c_in 1, vel_scale 1,
 * flux_col -1, default tiles (256x1 nodes, 64x4 for vectors), automatic
 * kernel variant, automatic streaming/cached accesses, XCD-aware block
 * order). */
lbf_status lbf_params_default(lbf_params *p, int nx, int ny);

/* Validate the parameters (host only, no HIP call) and create a context. */
lbf_status lbf_create(const lbf_params *p, lbf_ctx *out);

/* Device workspace the context needs (host arithmetic only). */
lbf_status lbf_workspace_bytes(lbf_ctx ctx, size_t *bytes);

/* Attach a caller-owned device workspace (>= lbf_workspace_bytes, 256-byte
 * aligned) and the hipStream_t on which all work is enqueued (may be NULL,
 * the legacy default stream).  The context keeps both until lbf_destroy. */
lbf_status lbf_bind(lbf_ctx ctx, void *workspace_dev, size_t bytes, void *hip_stream);

/* node_type_dev: device uint8 [ny][nx] (copied).  Builds the per-node link
 * masks on the device and the list of fluid nodes next to catalytic nodes.
 * In a channel rows 0 and ny-1 must be solid (LBF_EINVAL otherwise); a
 * periodic box wraps the links instead.  Synchronises. */
lbf_status lbf_set_geometry(lbf_ctx ctx, const uint8_t *node_type_dev);

/* k_dev: device double [ny][nx] (copied); rate of each catalytic node (read
 * at node types 2 and 3).  Values must lie in [0, 1] (LBF_EINVAL).  Syncs. */
lbf_status lbf_set_rates(lbf_ctx ctx, const double *k_dev);

/* Flow (Sec. "Lattice-Boltzmann for the Navier-Stokes equation", Eq. LBE,
 * with a velocity inlet and a pressure outlet in place of the paper's body
 * force): initial state f = f_eq(rho = 1, u = (u_in(y), 0)) with the parabola
 * u_in(y) = 4 u0 (y - 1/2)(ny - 3/2 - y)/(ny - 2)^2.  Channel only
 * (LBF_EINVAL for a periodic box). */
lbf_status lbf_flow_init(lbf_ctx ctx);
/* Advance the flow by exactly nsteps D2Q9 BGK steps (Eq. LBE; asynchronous). */
lbf_status lbf_flow_run(lbf_ctx ctx, long nsteps);
/* Advance until max |u(t) - u(t - check_every)| <= tol * u0 over fluid nodes,
 * or max_steps (then LBF_ENOTCONV): the steady Stokes flow the paper solves
 * once per geometry and scales.  tol <= 0: run exactly max_steps.
 * Synchronises; *steps_done and *residual (max |du|) may be NULL. */
lbf_status lbf_flow_steady(lbf_ctx ctx, long max_steps, int check_every, double tol,
                           long *steps_done, double *residual);
/* Flow velocity of the last flow step (zero at solids), Real [ny][nx]. */
lbf_status lbf_get_velocity(lbf_ctx ctx, void *ux_dev, void *uy_dev);
/* Import a flow velocity, Real [ny][nx] (replaces the flow solve). */
lbf_status lbf_set_velocity(lbf_ctx ctx, const void *ux_dev, const void *uy_dev);

/* ADR (Sec. "Lattice-Boltzmann for Advection-Diffusion-Reaction"): species A
 * at equilibrium with C = c_in and u = vel_scale * u_flow at every fluid
 * node, B and C zero.  Resets the step counter. */
lbf_status lbf_adr_init(lbf_ctx ctx);
/* Advance up to max_steps of the ADR step (Eqs. LBE_ADE, BGK, source_lbm,
 * boundary rules of Eq. BC).  Every check_every steps of the call compute the
 * outlet fluxes and eps (Eq. A-B) and stop at a steady check: eps moved by at
 * most tol of itself since the call's previous check, the outflux of the
 * last species is positive and N_A + ... + N_last balances the inflow of A
 * within 1e-3 of it (LBF_ENOTCONV when max_steps is reached first; a call's
 * first check has no previous eps).  tol <= 0: run exactly max_steps
 * (asynchronous unless checks are requested).  check_every must be >= 1.
 * *steps_done may be NULL.  A periodic box has no eps: it takes tol <= 0 only
 * (LBF_EINVAL otherwise). */
lbf_status lbf_adr_run(lbf_ctx ctx, long max_steps, int check_every, double tol,
                       long *steps_done);
/* Outlet fluxes N[0..nspecies) of the last step (FP64 sums over the rows
 * where both face nodes are fluid), the inflow of A, and eps (Eq. A-B).
 * Requires at least one step (LBF_ESTATE); eps is NaN when sum N = 0.
 * Any output pointer may be NULL.  Channel only.  Synchronises. */
lbf_status lbf_efficiency(lbf_ctx ctx, double *eps, double *N, double *inflow_A);
/* Concentration of one species after the last step (zero at solids), Real
 * [ny][nx].  Requires at least one step. */
lbf_status lbf_get_concentration(lbf_ctx ctx, int species, void *out_dev);
/* Total amount of each species, totals[0..nspecies) (host double), after the
 * last step: the FP64 sum of the concentration over the fluid nodes, with a
 * fixed summation order (bit-reproducible).  In a periodic box with inert
 * walls sum(totals) is conserved and totals[nspecies-1] measures the
 * conversion of the time-dependent problem.  Requires at least one step
 * (LBF_ESTATE).  Synchronises. */
lbf_status lbf_adr_totals(lbf_ctx ctx, double *totals);
/* Production of the reactions: the amount each converts in the next step
 * from the current state (the source term of Eq. source_lbm summed over the
 * lattice, FP64, fixed summation order), rates[0] for A -> B and, with three
 * species, rates[1] for B -> C (host double, nspecies - 1 values).  Link
 * reactions take k of the catalytic node times w_i times the fluid node's
 * concentration per link; the all-populations variant the mean neighbour
 * rate times the concentration per reacting node.  In a periodic box with
 * inert walls, the next step changes the totals of A, B, C by exactly
 * -rates[0], rates[0] - rates[1], rates[1] (up to rounding).  Requires at
 * least one step (LBF_ESTATE).  Synchronises. */
lbf_status lbf_adr_production(lbf_ctx ctx, double *rates);
/* Number of ADR steps taken since lbf_adr_init. */
lbf_status lbf_adr_steps(lbf_ctx ctx, long *steps);

/* Adjoint (reverse-mode) gradient of eps with respect to the rate k(x): the
 * exact derivative of the forward scheme (Eq. source_lbm supplies the only
 * dependence on k), not a method of the paper.
 * Objective: eps after T further steps from the current state, the current
 * pre-collision populations held fixed: the window's first collision and
 * reaction use the rates set at the call (the current post-collision lattice
 * is recomputed from the previous one), so eps_out and the gradient describe
 * the same function of k also after lbf_set_rates.  On return the context has advanced
 * T steps exactly as lbf_adr_run(T) would, *eps_out holds eps, and
 * grad_k_dev (device double [ny][nx]) holds d eps / d k at catalytic nodes
 * and 0 elsewhere.  The forward pass stores the full state every ckpt_every
 * steps and, in reverse, recomputes each segment to record the concentrations
 * the gradient needs; keep_trace = 1 records them for all T steps in the
 * forward pass instead (no recomputation).  adj_ws: caller-owned device
 * scratch of lbf_adjoint_workspace_bytes bytes.  Requires at least one step
 * taken.  Synchronises. */
lbf_status lbf_adjoint_workspace_bytes(lbf_ctx ctx, long T, int ckpt_every, int keep_trace,
                                       size_t *bytes);
lbf_status lbf_adr_adjoint(lbf_ctx ctx, long T, int ckpt_every, int keep_trace, void *adj_ws,
                           size_t adj_bytes, double *eps_out, double *grad_k_dev);

/* Steady-state adjoint: d eps / d k of the steady efficiency, for a context
 * whose ADR state has converged (the caller's responsibility; the current
 * state is taken as the fixed point).  Iterates the adjoint step with the
 * steady concentrations until max |nu| <= tol * max |nu_0| (checked every
 * check_every iterations), summing the gradient of every iteration: the
 * Neumann series of (I - A^T)^-1.  No forward steps, no checkpoints; the
 * ADR state is not modified.  adj_ws: lbf_adjoint_workspace_bytes(ctx, 1, 1,
 * 1, &b) bytes.  LBF_ENOTCONV when max_iters is reached first (gradient of
 * the partial sum still written).  Synchronises. */
lbf_status lbf_adr_adjoint_steady(lbf_ctx ctx, long max_iters, int check_every, double tol,
                                  void *adj_ws, size_t adj_bytes, double *eps_out,
                                  double *grad_k_dev, long *iters_done);

/* Checkpoint / resume of the ADR state (bit-exact). */
lbf_status lbf_state_bytes(lbf_ctx ctx, size_t *bytes);
lbf_status lbf_get_state(lbf_ctx ctx, void *dst_dev);
lbf_status lbf_set_state(lbf_ctx ctx, const void *src_dev);

/* Capture and instantiate the HIP graphs that lbf_adr_run and
 * lbf_time_adr_steps replay for a block of nsteps ADR steps (blocks are at
 * most 1000 steps), from either lattice, without running them: a timed or
 * latency-critical loop then pays no capture cost.  Needs the geometry set
 * and a bound workspace; the graphs are dropped by lbf_bind and
 * lbf_set_geometry.  Host and driver work only. */
lbf_status lbf_prepare_adr_steps(lbf_ctx ctx, long nsteps);

/* Timing helper: enqueue exactly nsteps ADR steps between two HIP events
 * recorded on the bound stream and return the elapsed milliseconds (the
 * average duration of one step kernel is ms / nsteps).  Synchronises. */
lbf_status lbf_time_adr_steps(lbf_ctx ctx, long nsteps, double *ms);
/* Same for the flow kernel. */
lbf_status lbf_time_flow_steps(lbf_ctx ctx, long nsteps, double *ms);

const char *lbf_status_str(lbf_status s);
/* Last error message of the context (never NULL). */
const char *lbf_last_error(lbf_ctx ctx);
void lbf_destroy(lbf_ctx ctx);
int lbf_version(void);

/* Device copy of nbytes from src_dev to dst_dev on hip_stream, timed with
 * HIP events (practical bandwidth ceiling and counter calibration).
 * Synchronises; *ms may be NULL. */
lbf_status lbf_probe_copy(const void *src_dev, void *dst_dev, size_t nbytes, void *hip_stream,
                          double *ms);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc) and hold no
 * context: the outlet fluxes N[0..nspecies), the inflow of A and eps of an
 * ADR state blob, as lbf_efficiency returns them for the context the blob
 * came from.  p: the lattice's parameters (nx, ny, real_bytes, nspecies,
 * c_in, flux_col, flags bit 2 are used; the rest is validated as by
 * lbf_create).  state_dev: device blob as lbf_get_state writes it (two
 * lattices and the header; caller-owned, read only).  node_type_dev: device
 * uint8 [ny][nx] of the same lattice (0 = fluid).  hip_stream: the stream to
 * use; the current device must be the stream's.  Output pointers are host
 * memory and may be NULL.  The library's scratch for the reduction is a
 * file-scope device array of 128 KiB + 32 B on each GPU it runs on (kept
 * until the process ends): no hipMalloc, hipFree or allocating library call.
 * Lattices of more than 262144 rows exceed it: LBF_ENOMEM.  LBF_EINVAL for
 * bad parameters, a periodic box or a blob whose header does not match p;
 * LBF_ESTATE for a blob with no step taken; LBF_EDIVERGED for non-finite
 * fluxes.  Calls on one GPU share its scratch and overlapping calls race:
 * serialise them (one stream, or synchronisation between streams).
 * Synchronises the stream. */
lbf_status lbf_efficiency_noalloc(const lbf_params *p, const void *state_dev,
                                  const uint8_t *node_type_dev, void *hip_stream, double *eps,
                                  double *N, double *inflow_A);

/* ---- batched Pe x Da sweep --------------------------------------------- *
 * n independent instances (own geometry, size, tau_g, vel_scale, rates) run
 * together: one kernel launch per time step covers the tiles of every active
 * instance, and blocks of steps are replayed as a captured HIP graph.
 * Instance i uses params[i] (all must share real_bytes, nspecies, tau_f, u0,
 * c_in, reaction_mode).  node_type and k are the instances' [ny_i][nx_i]
 * arrays concatenated in order. */
typedef struct lbf_batch_s *lbf_batch;
lbf_status lbf_batch_create(int n, const lbf_params *params, lbf_batch *out);
lbf_status lbf_batch_workspace_bytes(lbf_batch b, size_t *bytes);
lbf_status lbf_batch_bind(lbf_batch b, void *workspace_dev, size_t bytes, void *hip_stream);
lbf_status lbf_batch_set_geometry(lbf_batch b, const uint8_t *node_type_concat_dev,
                                  const double *k_concat_dev);
/* Flow for every instance: fixed max_steps when tol <= 0, else until each
 * instance meets the flow tolerance (converged instances stop stepping). */
lbf_status lbf_batch_flow(lbf_batch b, long max_steps, int check_every, double tol);
/* ADR for every instance from its initial state (Sec. "Lattice-Boltzmann
 * for Advection-Diffusion-Reaction", eps per Eq. A-B); every check_every
 * steps of the run each active instance's steady-state test is applied
 * (eps moved by at most tol of itself since its previous check, positive
 * product outflux, outlet fluxes balancing the inflow of A within 1e-3) and
 * converged instances are dropped from the tile list.  tol <= 0: exactly
 * max_steps for all.  Outputs (host arrays of n): eps, product flux (N of
 * the last species), steps taken by each instance.  LBF_ENOTCONV when
 * tol > 0 and some instance is still active after max_steps (the outputs
 * are written). */
lbf_status lbf_batch_run(lbf_batch b, long max_steps, int check_every, double tol,
                         double *eps_host, double *product_flux_host, long *steps_host);
/* Continue the current run by more_steps steps with the same active set and
 * the same check schedule (checks every check_every steps counted from the
 * start of the run; a call ending between two checks only observes): a run
 * split into resumed calls whose lengths are multiples of check_every stops
 * every instance at the same step as one call.  Outputs and LBF_ENOTCONV as
 * for lbf_batch_run.  LBF_ESTATE when no run was started, or after
 * lbf_batch_set_geometry, lbf_batch_flow or lbf_batch_time_steps. */
lbf_status lbf_batch_resume(lbf_batch b, long more_steps, int check_every, double tol,
                            double *eps_host, double *product_flux_host, long *steps_host);
/* Concentration of one species of instance i (Real [ny_i][nx_i]). */
lbf_status lbf_batch_get_concentration(lbf_batch b, int instance, int species, void *out_dev);
lbf_status lbf_batch_time_steps(lbf_batch b, long nsteps, double *ms);
const char *lbf_batch_last_error(lbf_batch b);
void lbf_batch_destroy(lbf_batch b);

#ifdef __cplusplus
}
#endif
#endif /* LBF_H */
