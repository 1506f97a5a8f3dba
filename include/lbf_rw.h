/*
 * lbf_rw.h -- C ABI of the GPU random-walk particle tracker, the paper's
 * second method for the same advection-diffusion-reaction problem (Sitaru &
 * Gekle, arXiv 2109.04455, Sec. "Random walk").
 *
 * Model (2D channel, the lattice geometry of lbf.h):
 *   - advection by the bilinearly interpolated lattice velocity
 *     (vel_scale * u), explicit Euler step dt; with wall_mode 1 a solid corner
 *     of the interpolation cell carries minus the value of the fluid corner(s)
 *     next to it, so the interpolant vanishes on the half-way walls;
 *   - diffusion by a step of length sqrt(4 D dt) in a uniformly random
 *     direction;
 *   - specular reflection at solid cells (unit squares centred on solid nodes;
 *     rows outside [0, ny) are solid, columns outside [0, nx) are open);
 *   - reaction within `zone` of a catalytic face: a particle of the source
 *     species turns into the product with probability k(sigma) rate_w dt / zone
 *     (faces tried in the order +x, +y, -x, -y);
 *   - a reservoir strip x in [-1.5, -0.5) refilled every step to `density`
 *     particles of A per unit area; B and C reflect at x = -0.5; particles
 *     leave at x >= nx - 0.5;
 *   - N_s = net crossings of x = xf + 1/2 per unit time while measuring.
 * Random numbers: splitmix64 (Steele, Lea & Flood 2014) as a counter-based
 * generator: draw d of step t of particle `id` is output 8 t + d + 1 of
 * splitmix64 started from seed ^ mix(id) (mix: the splitmix64 output
 * function).  Ids: the j-th initial particle of fluid cell c is c * 256 + j
 * (the cell's count floor(density + U) uses id 2^63 + c); the j-th reservoir
 * particle inserted at step t is 2^62 + t * 2^24 + j.  Results are therefore
 * independent of the particle order in memory.
 *
 * Conventions as in lbf.h (caller-owned workspace and stream, no device
 * allocation by the library, host-returning calls synchronise).
 */
#ifndef LBF_RW_H
#define LBF_RW_H

#include "lbf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbf_rw_s *lbf_rw;

typedef struct {
    int nx, ny;          /* lattice incl. wall rows; nx >= 8, ny >= 3           */
    int nspecies;        /* 2 or 3                                              */
    int xf;              /* measuring plane x = xf + 1/2; -1: nx - 3            */
    int wall_mode;       /* 0: u = 0 at solid nodes; 1: mirrored (see above)    */
    double D;            /* diffusion coefficient; sqrt(4 D dt) < 0.9           */
    double dt;           /* time step, > 0                                       */
    double zone;         /* reactive zone width, (0, 1]                          */
    double rate_w;       /* surface rate per unit length = k * rate_w            */
    double density;      /* particles of A per unit area, (0, 200]               */
    double vel_scale;    /* velocity = vel_scale * field, >= 0                   */
    uint64_t seed;
    long capacity;       /* maximum number of particles held (the particles that
                            left stay in the arrays until the next compaction,
                            at most min(64, nx / 8) steps' worth, about an
                            eighth of the particles the domain holds)          */
} lbf_rw_params;

lbf_status lbf_rw_params_default(lbf_rw_params *p, int nx, int ny);
lbf_status lbf_rw_create(const lbf_rw_params *p, lbf_rw *out);
lbf_status lbf_rw_workspace_bytes(lbf_rw rw, size_t *bytes);
lbf_status lbf_rw_bind(lbf_rw rw, void *workspace_dev, size_t bytes, void *hip_stream);
/* Geometry and fields (device arrays [ny][nx], copied): node_type u8 with
 * values 0..3, flow velocity ux, uy and rates k as double.  Rows 0 and ny-1
 * must be solid (LBF_EINVAL otherwise).  The copy interleaves ux and uy and
 * keeps per cell the types of the 5 x 5 cells around it, so a particle step
 * reads each corner velocity, and every cell type it needs, in one load. */
lbf_status lbf_rw_set_fields(lbf_rw rw, const uint8_t *node_type_dev, const double *ux_dev,
                             const double *uy_dev, const double *k_dev);
/* Uniform A at `density` in every fluid cell; resets the step and the
 * crossing counters.  Synchronises. */
lbf_status lbf_rw_fill(lbf_rw rw);
/* Advance nsteps steps (refill, move, react, count if measure != 0).
 * Asynchronous; LBF_ENOMEM from lbf_rw_counts if the capacity was hit. */
lbf_status lbf_rw_run(lbf_rw rw, long nsteps, int measure);
/* N[0..nspecies) = net crossings per unit time over the measured steps,
 * *nparticles = the particles the last step moved (those inside the domain
 * at its start plus the reservoir refill), *steps (all may be NULL).
 * Synchronises. */
lbf_status lbf_rw_counts(lbf_rw rw, double *N, long *nparticles, long *steps);
/* Trajectory mode: advance np caller-owned particles (device arrays ids u64,
 * x, y double, species u8, updated in place) through steps t0 .. t0+steps-1
 * with no insertion, removal or counting. */
lbf_status lbf_rw_walk(lbf_rw rw, long np, const uint64_t *ids_dev, double *x_dev, double *y_dev,
                       uint8_t *species_dev, long t0, long steps);
/* nsteps steps between two HIP events; *ms elapsed.  Synchronises. */
lbf_status lbf_rw_time_steps(lbf_rw rw, long nsteps, int measure, double *ms);
const char *lbf_rw_last_error(lbf_rw rw);
void lbf_rw_destroy(lbf_rw rw);

#ifdef __cplusplus
}
#endif

#endif /* LBF_RW_H */
