/*
 * lbf3d.h -- C ABI of the 3D lattice-Boltzmann flow + advection-diffusion-
 * reaction path: membranes of randomly oriented, capped fibres (Sitaru &
 * Gekle, arXiv 2109.04455, Sec. "System geometry: Cascade reaction" and Sec.
 * "Membrane generation").
 *
 *   1. flow: D3Q19 BGK in a box periodic in x, y and z, driven by a uniform
 *      body force along x (the paper's set-up, Sec. "Lattice-Boltzmann for the
 *      Navier-Stokes equation"), the force entered by Guo's scheme, half-way
 *      bounce-back at solid nodes;
 *   2. ADR: D3Q7 BGK (w0 = 1/4, w1..6 = 1/8, cs^2 = 1/4, D = (tau_g - 1/2)/4)
 *      with the second-order equilibrium on the linearly scaled flow velocity
 *      (Eqs. LBE_ADE, BGK, Diffusion_LBM), link reactions A->B / B->C at
 *      catalytic nodes (Eq. source_lbm); inlet x = 0 (anti-bounce-back with
 *      C_w = c_in for A, bounce-back for B, C) and outlet x = nx-1 (C_w = C_b),
 *      Eq. BC; periodic in y and z;
 *   3. outlet fluxes through the face between x = flux_col and flux_col + 1,
 *      summed over (y, z), and eps (Eq. A-B).
 *
 * Conventions as in lbf.h: every call returns an lbf_status; device pointers
 * are caller-owned; the library allocates no device memory (all buffers live
 * in the bound workspace); work is enqueued on the bound stream; calls that
 * return host values synchronise it.  Fields are [nz][ny][nx], x fastest.
 * node_type: 0 fluid, 1 inert solid, 2 catalyst type 1 (A->B), 3 catalyst
 * type 2 (B->C; inert with two species).  "Real" is float when
 * real_bytes = 4 and double when 8; FP32 storage computes each node update in
 * FP64 unless flags bit 4 is set.
 */
#ifndef LBF3D_H
#define LBF3D_H

#include "lbf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbf3_ctx_s *lbf3_ctx;

typedef struct {
    int nx, ny, nz;      /* lattice; nx >= 8, ny >= 2, nz >= 2                  */
    int real_bytes;      /* 4 or 8                                              */
    int nspecies;        /* 2: A->B, 3: cascade A->B->C                         */
    double tau_f;        /* D3Q19 relaxation time, > 0.5                        */
    double force_x;      /* body force along x driving the flow, |F| <= 1e-3    */
    double tau_g;        /* D3Q7 relaxation time, > 0.5                         */
    double c_in;         /* inlet concentration of A                            */
    double vel_scale;    /* ADR velocity = vel_scale * flow velocity, >= 0      */
    int flux_col;        /* flux face between flux_col and flux_col+1; -1: nx-3 */
    int tile_x, tile_y;  /* thread block: tile_x nodes along x times tile_y rows
                            (y, z lines); 0: 64 x 4.  tile_x * tile_y must be a
                            multiple of 64 and <= 1024                          */
    int flags;           /* bit 0: no XCD-aware block order; bit 1: cached
                            population accesses; bit 4: FP32 arithmetic;
                            bit 6: streaming accesses even when the lattices
                            fit the last-level cache                            */
} lbf3_params;

/* Defaults for an nx x ny x nz lattice: FP32, 3 species, tau_f 0.8,
 * force 1e-6, tau_g 0.8, c_in 1, vel_scale 1, flux_col -1, tiles 64 x 4,
 * flags 0. */
lbf_status lbf3_params_default(lbf3_params *p, int nx, int ny, int nz);
/* Validate (host only) and create; a context is returned even on
 * LBF_EINVAL so that lbf3_last_error can explain. */
lbf_status lbf3_create(const lbf3_params *p, lbf3_ctx *out);
lbf_status lbf3_workspace_bytes(lbf3_ctx ctx, size_t *bytes);
/* Caller-owned 256-byte aligned device workspace and hipStream_t (may be
 * NULL); kept until lbf3_destroy. */
lbf_status lbf3_bind(lbf3_ctx ctx, void *workspace_dev, size_t bytes, void *hip_stream);
/* node_type_dev: device uint8 [nz][ny][nx] (copied), values 0..3.  Builds the
 * D3Q19 and D3Q7 link masks.  Synchronises. */
lbf_status lbf3_set_geometry(lbf3_ctx ctx, const uint8_t *node_type_dev);
/* k_dev: device double [nz][ny][nx], read at catalytic nodes, in [0, 1]. */
lbf_status lbf3_set_rates(lbf3_ctx ctx, const double *k_dev);

/* Flow: rest fluid (rho = 1) at t = 0; exactly nsteps forced steps. */
lbf_status lbf3_flow_init(lbf3_ctx ctx);
lbf_status lbf3_flow_run(lbf3_ctx ctx, long nsteps);
/* Advance until max|u(t) - u(t - check_every)| <= tol * max|u(t)| over fluid
 * nodes (LBF_ENOTCONV after max_steps).  tol <= 0: exactly max_steps.
 * *steps_done, *residual (max|du|) may be NULL.  Synchronises. */
lbf_status lbf3_flow_steady(lbf3_ctx ctx, long max_steps, int check_every, double tol,
                            long *steps_done, double *residual);
/* Physical flow velocity u = (sum c f + F/2)/rho of the last step, Real
 * [nz][ny][nx] each (zero at solids). */
lbf_status lbf3_get_velocity(lbf3_ctx ctx, void *ux_dev, void *uy_dev, void *uz_dev);
/* Import a velocity field (replaces the flow solve). */
lbf_status lbf3_set_velocity(lbf3_ctx ctx, const void *ux_dev, const void *uy_dev,
                             const void *uz_dev);

/* ADR: A at equilibrium with C = c_in and u = vel_scale * u_flow, B = C = 0. */
lbf_status lbf3_adr_init(lbf3_ctx ctx);
/* As lbf_adr_run: up to max_steps, stopping at a steady check (eps moved by
 * at most tol of itself since the call's previous check, positive outflux of
 * the last species, outlet fluxes balancing the inflow of A within 1e-3;
 * tol <= 0: exactly max_steps). */
lbf_status lbf3_adr_run(lbf3_ctx ctx, long max_steps, int check_every, double tol,
                        long *steps_done);
/* Outlet fluxes N[0..nspecies), inflow of A and eps of the last step (FP64
 * sums in a fixed order).  Requires one step (LBF_ESTATE).  Synchronises. */
lbf_status lbf3_efficiency(lbf3_ctx ctx, double *eps, double *N, double *inflow_A);
/* Concentration of one species after the last step, Real [nz][ny][nx]. */
lbf_status lbf3_get_concentration(lbf3_ctx ctx, int species, void *out_dev);
/* FP64 totals of every species over the fluid nodes (host double[nspecies]). */
lbf_status lbf3_adr_totals(lbf3_ctx ctx, double *totals);
/* Enqueue exactly nsteps steps between two HIP events on the bound stream;
 * *ms receives the elapsed time.  Synchronises. */
lbf_status lbf3_time_adr_steps(lbf3_ctx ctx, long nsteps, double *ms);
lbf_status lbf3_time_flow_steps(lbf3_ctx ctx, long nsteps, double *ms);
const char *lbf3_last_error(lbf3_ctx ctx);
void lbf3_destroy(lbf3_ctx ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBF3D_H */
