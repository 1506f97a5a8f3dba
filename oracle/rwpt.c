/*
 * rwpt.c -- an independent random-walk particle tracker for the 2D
 * advection-diffusion-reaction problem (paper Sec. "Random walk").
 *
 * TEST INFRASTRUCTURE ONLY: it is the oracle's own cross-check and shares
 * nothing with the lattice-Boltzmann code (neither the oracle's nor the GPU
 * library's).
 *
 * Model, following the paper's description:
 *   - advection by the bilinearly interpolated lattice velocity field, explicit
 *     Euler step dt (0.5 in the paper);
 *   - diffusion by a step of fixed length sqrt(4 D dt) in a uniformly random
 *     direction;
 *   - elastic (specular) reflection at solid cells; the solid geometry is the
 *     union of unit squares centred on solid lattice nodes, so walls sit
 *     half-way between nodes as with lattice bounce-back;
 *   - reaction inside a zone of width `zone` next to each catalytic face: a
 *     particle of the source species reacts with probability rate*dt/zone per
 *     step, where `rate` is the surface rate per unit face length;
 *   - a reservoir strip in front of the inlet is refilled to a uniform density
 *     of species A every step (Dirichlet inlet); B and C are reflected at the
 *     inlet plane; particles leave through the outlet plane;
 *   - N_s = net number of crossings of the plane xf + 1/2 per unit time.
 * Random numbers: splitmix64 (Steele, Lea & Flood, 2014) used as a
 * counter-based generator: every particle has a 64-bit id, and draw d of step
 * t is output n = 8 t + d + 1 of splitmix64 started from the state
 * seed ^ mix(id).  A particle's path therefore depends only on its id, its
 * state and the step, not on the order in which particles are processed.
 * Ids: the j-th particle of the initial fill of fluid cell c is c * 256 + j
 * (the count of cell c is drawn from id 2^63 + c); the j-th reservoir particle
 * inserted at step t is 2^62 + t * 2^24 + j.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static uint64_t mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* draw d of step t of particle id, uniform in [0, 1) */
static double draw(uint64_t seed, uint64_t id, uint64_t t, unsigned d)
{
    uint64_t state = seed ^ mix(id);
    uint64_t n = 8 * t + d + 1;
    return (double)(mix(state + n * 0x9e3779b97f4a7c15ULL) >> 11) * (1.0 / 9007199254740992.0);
}

#define ID_INSERT (1ULL << 62)
#define ID_COUNT (1ULL << 63)

typedef struct {
    int nx, ny;
    const uint8_t *type;
    const double *ux, *uy, *k;
    double vel_scale, h;
} geom_t;

/* solid test for the cell of node (cx, cy); cells left of the inlet and right
 * of the outlet are open */
static int solid(const geom_t *g, int cx, int cy)
{
    if (cy < 0 || cy >= g->ny) return 1;
    if (cx < 0 || cx >= g->nx) return 0;
    return g->type[(size_t)cy * g->nx + cx] != 0;
}

static int cell(double p) { return (int)floor(p + 0.5); }

static double node_u(const geom_t *g, const double *u, int x, int y)
{
    if (y < 0 || y >= g->ny) return 0.0;
    if (x < 0) x = 0;
    if (x >= g->nx) x = g->nx - 1;
    return u[(size_t)y * g->nx + x];
}

/* bilinear interpolation of a nodal field at (px, py).  wall_mode 0: solid
 * nodes carry u = 0 (plain interpolation of the lattice field); wall_mode 1:
 * a solid corner carries minus the value of the fluid corner(s) next to it
 * in the cell, so the interpolant vanishes on the wall half-way between the
 * nodes, where the lattice's bounce-back puts the no-slip wall. */
static double interp(const geom_t *g, const double *u, double px, double py, int wall_mode)
{
    int x0 = (int)floor(px), y0 = (int)floor(py);
    double fx = px - x0, fy = py - y0;
    double v[2][2];
    int sol[2][2];
    for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 2; ++i) {
            sol[j][i] = solid(g, x0 + i, y0 + j);
            v[j][i] = sol[j][i] ? 0.0 : node_u(g, u, x0 + i, y0 + j);
        }
    if (wall_mode == 1) {
        double w[2][2];
        for (int j = 0; j < 2; ++j)
            for (int i = 0; i < 2; ++i) {
                w[j][i] = v[j][i];
                if (!sol[j][i]) continue;
                double sum = 0;
                int n = 0;
                if (!sol[j][1 - i]) { sum -= v[j][1 - i]; ++n; }  /* across a wall normal to x */
                if (!sol[1 - j][i]) { sum -= v[1 - j][i]; ++n; }  /* across a wall normal to y */
                if (n == 0 && !sol[1 - j][1 - i]) { sum -= v[1 - j][1 - i]; n = 1; }
                w[j][i] = n ? sum / n : 0.0;
            }
        for (int j = 0; j < 2; ++j)
            for (int i = 0; i < 2; ++i) v[j][i] = w[j][i];
    }
    return (1 - fx) * (1 - fy) * v[0][0] + fx * (1 - fy) * v[0][1] + (1 - fx) * fy * v[1][0] +
           fx * fy * v[1][1];
}

/* move from (px,py) to (*qx,*qy) with specular reflection at solid faces */
static void reflect(const geom_t *g, double px, double py, double *qx, double *qy)
{
    int ox = cell(px), oy = cell(py);
    int nxc = cell(*qx), nyc = cell(*qy);
    if (!solid(g, nxc, nyc)) return;
    int done = 0;
    if (nxc != ox && solid(g, nxc, oy)) {
        double face = nxc > ox ? ox + 0.5 : ox - 0.5;
        *qx = 2.0 * face - *qx;
        done = 1;
    }
    if (nyc != oy && solid(g, ox, nyc)) {
        double face = nyc > oy ? oy + 0.5 : oy - 0.5;
        *qy = 2.0 * face - *qy;
        done = 1;
    }
    if (!done) { /* corner: only the diagonal cell is solid */
        double fx = nxc > ox ? ox + 0.5 : ox - 0.5;
        double fy = nyc > oy ? oy + 0.5 : oy - 0.5;
        *qx = 2.0 * fx - *qx;
        *qy = 2.0 * fy - *qy;
    }
    if (solid(g, cell(*qx), cell(*qy))) { /* give up on this move */
        *qx = px;
        *qy = py;
    }
}

/*
 * Run the tracker.  Returns 0, or -1 on bad arguments / particle overflow.
 *   c_density   reservoir particles per unit area of species A
 *   zone        reactive zone width next to a catalytic face (<= 1)
 *   rate_w      surface rate per unit length = k(sigma) * rate_w
 *   out[0..ns)  net crossings of xf + 1/2 per unit time over the measurement
 *   out[ns]     number of particles in the domain at the end
 *   wall_mode   velocity interpolation next to solids (see interp)
 */
/* One step of one particle (advect, diffuse, reflect, inlet rule, crossing
 * count, reaction).  Returns 1 if it left through the outlet.  *cross_ds
 * receives the signed crossing of the measuring plane (+1, -1 or 0). */
static int move_particle(const geom_t *g, int ns, uint64_t seed, uint64_t id, uint64_t t,
                         double dt, double step_len, double zone, double rate_w, double buf_hi,
                         double plane, int wall_mode, double *px, double *py, uint8_t *sp,
                         int *cross_ds)
{
    static const int DX[4] = {1, 0, -1, 0}, DY[4] = {0, 1, 0, -1};
    const int nx = g->nx, ny = g->ny;
    double x0 = *px, y0 = *py;
    double u = g->vel_scale * interp(g, g->ux, x0, y0, wall_mode);
    double v = g->vel_scale * interp(g, g->uy, x0, y0, wall_mode);
    double th = 2.0 * M_PI * draw(seed, id, t, 0);
    double x1 = x0 + u * dt + step_len * cos(th);
    double y1 = y0 + v * dt + step_len * sin(th);
    reflect(g, x0, y0, &x1, &y1);
    int s = *sp;
    if (x1 < buf_hi && x0 >= buf_hi && s != 0) /* B, C: reflect at the inlet */
        x1 = 2.0 * buf_hi - x1;
    *cross_ds = (x0 < plane && x1 >= plane) ? 1 : ((x0 >= plane && x1 < plane) ? -1 : 0);
    /* reaction next to catalytic faces of the current cell */
    int cx = cell(x1), cy = cell(y1);
    if (cx >= 0 && cx < nx && cy >= 0 && cy < ny && g->type[(size_t)cy * nx + cx] == 0) {
        for (int d = 0; d < 4; ++d) {
            int sx = cx + DX[d], sy = cy + DY[d];
            if (sx < 0 || sx >= nx || sy < 0 || sy >= ny) continue;
            int ty = g->type[(size_t)sy * nx + sx];
            int src = ty == 2 ? 0 : (ty == 3 && ns == 3 ? 1 : -1);
            if (src != s) continue;
            double dist = d == 0 ? cx + 0.5 - x1 : d == 1 ? cy + 0.5 - y1
                        : d == 2 ? x1 - (cx - 0.5) : y1 - (cy - 0.5);
            if (dist >= zone) continue;
            double p = g->k[(size_t)sy * nx + sx] * rate_w * dt / zone;
            if (draw(seed, id, t, 1 + d) < p) {
                *sp = (uint8_t)(src + 1);
                break;
            }
        }
    }
    *px = x1;
    *py = y1;
    return x1 >= nx - 0.5;
}

/*
 * Run the tracker.  Returns 0, or -1 on bad arguments / particle overflow.
 *   c_density   reservoir particles per unit area of species A (<= 200)
 *   zone        reactive zone width next to a catalytic face (<= 1)
 *   rate_w      surface rate per unit length = k(sigma) * rate_w
 *   out[0..ns)  net crossings of xf + 1/2 per unit time over the measurement
 *   out[ns]     number of particles in the domain at the end
 *   wall_mode   velocity interpolation next to solids (see interp)
 */
int rwpt_run(int nx, int ny, int ns, const uint8_t *type, const double *ux, const double *uy,
             double vel_scale, double D, const double *k, double rate_w, double c_density,
             double dt, double zone, int xf, long burn_steps, long meas_steps, uint64_t seed,
             long max_particles, int wall_mode, double *out)
{
    geom_t g = {nx, ny, type, ux, uy, k, vel_scale, 0.0};
    double step_len = sqrt(4.0 * D * dt);
    if (ns < 2 || ns > 3 || zone <= 0 || zone > 1 || step_len >= 0.9 || c_density > 200)
        return -1;
    double *px = malloc(sizeof(double) * max_particles);
    double *py = malloc(sizeof(double) * max_particles);
    uint8_t *sp = malloc(max_particles);
    uint64_t *pid = malloc(sizeof(uint64_t) * max_particles);
    long np = 0;
    const double buf_lo = -1.5, buf_hi = -0.5; /* reservoir strip */
    const double ylo = 0.5, yhi = ny - 1.5;    /* fluid band between wall rows */
    long buf_count = lround(c_density * (buf_hi - buf_lo) * (yhi - ylo));
    const double plane = xf + 0.5;
    double cross[3] = {0, 0, 0};
    int status = 0;

    /* start from a uniform field of A in every fluid cell */
    for (int y = 0; y < ny && status == 0; ++y)
        for (int x = 0; x < nx; ++x) {
            uint64_t c = (uint64_t)y * nx + x;
            if (type[c] != 0) continue;
            long n = (long)floor(c_density + draw(seed, ID_COUNT + c, 0, 0));
            for (long j = 0; j < n; ++j) {
                if (np >= max_particles) { status = -1; break; }
                uint64_t id = c * 256 + (uint64_t)j;
                px[np] = x - 0.5 + draw(seed, id, 0, 6);
                py[np] = y - 0.5 + draw(seed, id, 0, 7);
                sp[np] = 0;
                pid[np] = id;
                ++np;
            }
        }
    for (long t = 0; t < burn_steps + meas_steps && status == 0; ++t) {
        int measuring = t >= burn_steps;
        /* refill the reservoir: drop its particles, place a fresh uniform set */
        for (long j = 0; j < np;) {
            if (px[j] < buf_hi) {
                --np;
                px[j] = px[np]; py[j] = py[np]; sp[j] = sp[np]; pid[j] = pid[np];
            } else {
                ++j;
            }
        }
        for (long j = 0; j < buf_count; ++j) {
            if (np >= max_particles) { status = -1; break; }
            uint64_t id = ID_INSERT + ((uint64_t)t << 24) + (uint64_t)j;
            px[np] = buf_lo + (buf_hi - buf_lo) * draw(seed, id, 0, 6);
            py[np] = ylo + (yhi - ylo) * draw(seed, id, 0, 7);
            sp[np] = 0;
            pid[np] = id;
            ++np;
        }
        for (long j = 0; j < np;) {
            int ds = 0, s = sp[j];
            int gone = move_particle(&g, ns, seed, pid[j], (uint64_t)t, dt, step_len, zone, rate_w,
                                     buf_hi, plane, wall_mode, &px[j], &py[j], &sp[j], &ds);
            if (measuring) cross[s] += ds;
            if (gone) { /* left through the outlet */
                --np;
                px[j] = px[np]; py[j] = py[np]; sp[j] = sp[np]; pid[j] = pid[np];
                continue;
            }
            ++j;
        }
    }
    for (int s = 0; s < ns; ++s) out[s] = cross[s] / (meas_steps * dt);
    out[ns] = (double)np;
    free(px);
    free(py);
    free(sp);
    free(pid);
    return status;
}

/* Trajectory mode: advance np given particles (ids, positions, species) by
 * steps t0 .. t0+steps-1 with no insertion and no removal (a particle past
 * the outlet keeps moving).  Returns 0. */
int rwpt_walk(int nx, int ny, int ns, const uint8_t *type, const double *ux, const double *uy,
              double vel_scale, double D, const double *k, double rate_w, double dt, double zone,
              int wall_mode, uint64_t seed, long np, const uint64_t *id, double *px, double *py,
              uint8_t *sp, long t0, long steps)
{
    geom_t g = {nx, ny, type, ux, uy, k, vel_scale, 0.0};
    double step_len = sqrt(4.0 * D * dt);
    for (long j = 0; j < np; ++j)
        for (long t = t0; t < t0 + steps; ++t) {
            int ds;
            move_particle(&g, ns, seed, id[j], (uint64_t)t, dt, step_len, zone, rate_w, -0.5,
                          nx + 10.0, wall_mode, &px[j], &py[j], &sp[j], &ds);
        }
    return 0;
}
