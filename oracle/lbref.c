/*
 * lbref.c -- the oracle: a plain, slow, obviously-correct FP64 CPU reference of
 * the hybrid lattice-Boltzmann scheme of Sitaru & Gekle, "Analytical and
 * computational study of cascade reaction processes in catalytic fibrous
 * membranes" (arXiv 2109.04455).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file.  It shares no code, header,
 * table or constant with the GPU library; it is single-threaded, unblocked and
 * follows the paper's order of operations.
 *
 * Conventions
 *   grid  x in [0,nx), y in [0,ny), linear index y*nx + x (x fastest)
 *   node_type: 0 fluid, 1 inert solid, 2 catalyst type 1 (A->B),
 *              3 catalyst type 2 (B->C)
 *   populations [q][ny][nx]; species populations [s][5][ny][nx]
 *   The state held between steps is the PRE-collision population set.
 *   One step = collide (+ react) at every fluid node, then stream with
 *   boundary conditions (paper Sec. "Lattice-Boltzmann for the Navier-Stokes
 *   equation", Eq. LBE; Sec. "Lattice-Boltzmann for Advection-Diffusion-
 *   Reaction", Eq. LBE_ADE).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- velocity sets ------------------------------------------------------ */
/* D2Q9: rest, E, N, W, S, NE, NW, SW, SE */
static const int D9X[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int D9Y[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int D9OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static double d9w(int i) { return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }

/* D2Q5: rest, E, N, W, S.  w0 = 1/3, w1..4 = 1/6 gives cs^2 = 1/3 as in the
 * equilibrium of the ADE section, so D = (tau_g - 1/2)/3 (Eq. Diffusion_LBM). */
static const int D5X[5] = {0, 1, 0, -1, 0};
static const int D5Y[5] = {0, 0, 1, 0, -1};
static const int D5OPP[5] = {0, 3, 4, 1, 2};
static double d5w(int i) { return i == 0 ? 1.0 / 3.0 : 1.0 / 6.0; }

enum { E = 1, N = 2, W = 3, S = 4, NE = 5, NW = 6, SW = 7, SE = 8 };

/* ---- flow: D2Q9 BGK -------------------------------------------------------- */

/* Second-order equilibrium, cs^2 = 1/3. */
static double feq9(int i, double rho, double ux, double uy)
{
    double cu = D9X[i] * ux + D9Y[i] * uy;
    return d9w(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy));
}

/* Parabolic inlet profile: no-slip walls half-way between the solid rows
 * y = 0, ny-1 and the first fluid rows, centre-line velocity u0. */
double ref_inlet_velocity(int ny, double u0, int y)
{
    double h = ny - 2.0;
    return 4.0 * u0 * (y - 0.5) * (ny - 1.5 - y) / (h * h);
}

void ref_flow_init(int nx, int ny, const uint8_t *type, double u0, double *f)
{
    size_t n = (size_t)nx * ny;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t id = (size_t)y * nx + x;
            double ux = ref_inlet_velocity(ny, u0, y);
            for (int i = 0; i < 9; ++i)
                f[i * n + id] = type[id] == 0 ? feq9(i, 1.0, ux, 0.0) : 0.0;
        }
}

/* One step.  f: pre-collision state (read), fout: next pre-collision state,
 * post: scratch [9][ny][nx]. */
static void flow_step(int nx, int ny, const uint8_t *type, double tau, double u0,
                      const double *f, double *fout, double *post)
{
    size_t n = (size_t)nx * ny;
    /* collide */
    for (size_t id = 0; id < n; ++id) {
        if (type[id] != 0) continue;
        double rho = 0, jx = 0, jy = 0;
        for (int i = 0; i < 9; ++i) {
            rho += f[i * n + id];
            jx += D9X[i] * f[i * n + id];
            jy += D9Y[i] * f[i * n + id];
        }
        double ux = jx / rho, uy = jy / rho;
        for (int i = 0; i < 9; ++i)
            post[i * n + id] = f[i * n + id] - (f[i * n + id] - feq9(i, rho, ux, uy)) / tau;
    }
    /* stream: each population arrives from x - c_i; a solid source means the
     * population that left towards the solid comes back reversed (half-way
     * bounce-back); a source outside [0,nx) is an open boundary, filled below. */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t id = (size_t)y * nx + x;
            if (type[id] != 0) {
                for (int i = 0; i < 9; ++i) fout[i * n + id] = 0.0;
                continue;
            }
            for (int i = 0; i < 9; ++i) {
                int sx = x - D9X[i], sy = y - D9Y[i];
                if (sx < 0 || sx >= nx) {
                    fout[i * n + id] = NAN; /* unknown: open boundary */
                } else if (sy < 0 || sy >= ny || type[(size_t)sy * nx + sx] != 0) {
                    fout[i * n + id] = post[D9OPP[i] * n + id];
                } else {
                    fout[i * n + id] = post[i * n + (size_t)sy * nx + sx];
                }
            }
            double *F[9];
            for (int i = 0; i < 9; ++i) F[i] = &fout[i * n + id];
            if (x == 0) {
                /* Zou-He velocity inlet: u = (u_in(y), 0); unknown E, NE, SE */
                double ux = ref_inlet_velocity(ny, u0, y);
                double rho = (*F[0] + *F[N] + *F[S] + 2.0 * (*F[W] + *F[NW] + *F[SW])) / (1.0 - ux);
                *F[E] = *F[W] + 2.0 / 3.0 * rho * ux;
                *F[NE] = *F[SW] - 0.5 * (*F[N] - *F[S]) + rho * ux / 6.0;
                *F[SE] = *F[NW] + 0.5 * (*F[N] - *F[S]) + rho * ux / 6.0;
            } else if (x == nx - 1) {
                /* Zou-He pressure outlet, rho = 1, u_y = 0; unknown W, NW, SW */
                double ux = -1.0 + (*F[0] + *F[N] + *F[S] + 2.0 * (*F[E] + *F[NE] + *F[SE]));
                *F[W] = *F[E] - 2.0 / 3.0 * ux;
                *F[NW] = *F[SE] - 0.5 * (*F[N] - *F[S]) - ux / 6.0;
                *F[SW] = *F[NE] + 0.5 * (*F[N] - *F[S]) - ux / 6.0;
            }
        }
}

void ref_flow_run(int nx, int ny, const uint8_t *type, double tau, double u0,
                  double *f, long nsteps)
{
    size_t bytes = sizeof(double) * 9 * (size_t)nx * ny;
    double *tmp = (double *)malloc(bytes), *post = (double *)calloc(1, bytes);
    for (long t = 0; t < nsteps; ++t) {
        flow_step(nx, ny, type, tau, u0, f, tmp, post);
        memcpy(f, tmp, bytes);
    }
    free(tmp);
    free(post);
}

/* Velocity = first moment / zeroth moment of the pre-collision populations;
 * zero at solid nodes. */
void ref_flow_velocity(int nx, int ny, const uint8_t *type, const double *f,
                       double *ux, double *uy, double *rho_out)
{
    size_t n = (size_t)nx * ny;
    for (size_t id = 0; id < n; ++id) {
        double rho = 0, jx = 0, jy = 0;
        if (type[id] == 0)
            for (int i = 0; i < 9; ++i) {
                rho += f[i * n + id];
                jx += D9X[i] * f[i * n + id];
                jy += D9Y[i] * f[i * n + id];
            }
        ux[id] = type[id] == 0 ? jx / rho : 0.0;
        uy[id] = type[id] == 0 ? jy / rho : 0.0;
        if (rho_out) rho_out[id] = rho;
    }
}

/* ---- advection-diffusion-reaction: D2Q5 BGK ------------------------------- */

/* boundary flags */
#define REF_PERIODIC_X 1
#define REF_PERIODIC_Y 2
/* reaction modes */
#define REF_LINK 0 /* only populations streaming into a catalytic node react */
#define REF_NODE 1 /* every population of a fluid node reacts (rates k, k2 at the node) */
#define REF_NODE_AT_CATALYST 2 /* the paper's comparison variant: every population of a
                                * fluid node next to a catalyst reacts, with the mean rate
                                * of that node's catalytic neighbours of each type */

static double geq5(int i, double c, double ux, double uy)
{
    double cu = D5X[i] * ux + D5Y[i] * uy;
    return d5w(i) * c * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy));
}

/* Initial state: species A at equilibrium with C = c_in and the imposed
 * velocity vel_scale*u at every fluid node, B and C absent. */
void ref_adr_init(int nx, int ny, int ns, const uint8_t *type, const double *ux,
                  const double *uy, double vel_scale, double c_in, double *g)
{
    size_t n = (size_t)nx * ny;
    for (int s = 0; s < ns; ++s)
        for (int i = 0; i < 5; ++i)
            for (size_t id = 0; id < n; ++id) {
                double v = 0.0;
                if (s == 0 && type[id] == 0)
                    v = geq5(i, c_in, vel_scale * ux[id], vel_scale * uy[id]);
                g[((size_t)s * 5 + i) * n + id] = v;
            }
}

static int wrap(int a, int m) { return ((a % m) + m) % m; }

/* One step of the ADR lattice Boltzmann scheme.
 *   g    pre-collision state [ns][5][ny][nx] (read)
 *   gout next pre-collision state
 *   post scratch for the post-collision populations
 *   k    link mode: rate at catalytic solid nodes; node mode: A->B rate at
 *        fluid nodes.  k2: node mode B->C rate (may be NULL).
 *   conc optional [ns][ny][nx] output: pre-collision concentration this step
 */
static void adr_step(int nx, int ny, int ns, const uint8_t *type, const double *k,
                     const double *k2, const double *ux, const double *uy,
                     double vel_scale, double tau, double c_in, int mode, int bc,
                     const double *g, double *gout, double *post, double *conc)
{
    size_t n = (size_t)nx * ny;
#define G(arr, s, i, id) arr[((size_t)(s) * 5 + (i)) * n + (id)]
    /* collide and react at every fluid node */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t id = (size_t)y * nx + x;
            if (type[id] != 0) continue;
            double u = vel_scale * ux[id], v = vel_scale * uy[id];
            double c[3] = {0, 0, 0};
            for (int s = 0; s < ns; ++s)
                for (int i = 0; i < 5; ++i) c[s] += G(g, s, i, id);
            if (conc)
                for (int s = 0; s < ns; ++s) conc[(size_t)s * n + id] = c[s];
            /* BGK collision, Eq. BGK with the second-order equilibrium */
            for (int s = 0; s < ns; ++s)
                for (int i = 0; i < 5; ++i)
                    G(post, s, i, id) = G(g, s, i, id) - (G(g, s, i, id) - geq5(i, c[s], u, v)) / tau;
            /* reaction source, Eq. source_lbm */
            if (mode == REF_LINK) {
                /* only the population heading into a catalytic node reacts;
                 * its rate is the rate of that node; the concentration is the
                 * fluid node's pre-collision one */
                for (int i = 1; i < 5; ++i) {
                    int nxx = x + D5X[i], nyy = y + D5Y[i];
                    if (bc & REF_PERIODIC_X) nxx = wrap(nxx, nx);
                    if (bc & REF_PERIODIC_Y) nyy = wrap(nyy, ny);
                    if (nxx < 0 || nxx >= nx || nyy < 0 || nyy >= ny) continue;
                    size_t sid = (size_t)nyy * nx + nxx;
                    int src, prod;
                    if (type[sid] == 2) {
                        src = 0; prod = 1;
                    } else if (type[sid] == 3 && ns == 3) {
                        src = 1; prod = 2;
                    } else {
                        continue;
                    }
                    double r = k[sid] * d5w(i) * c[src];
                    G(post, src, i, id) -= r;
                    G(post, prod, i, id) += r;
                }
            } else if (mode == REF_NODE_AT_CATALYST) {
                double ksum[2] = {0, 0};
                int kcnt[2] = {0, 0};
                for (int i = 1; i < 5; ++i) {
                    int nxx = x + D5X[i], nyy = y + D5Y[i];
                    if (bc & REF_PERIODIC_X) nxx = wrap(nxx, nx);
                    if (bc & REF_PERIODIC_Y) nyy = wrap(nyy, ny);
                    if (nxx < 0 || nxx >= nx || nyy < 0 || nyy >= ny) continue;
                    size_t sid = (size_t)nyy * nx + nxx;
                    if (type[sid] == 2) { ksum[0] += k[sid]; kcnt[0]++; }
                    if (type[sid] == 3 && ns == 3) { ksum[1] += k[sid]; kcnt[1]++; }
                }
                for (int q = 0; q < 2; ++q) {
                    if (kcnt[q] == 0) continue;
                    int src = q, prod = q + 1;
                    double kk = ksum[q] / kcnt[q];
                    for (int i = 0; i < 5; ++i) {
                        double r = kk * d5w(i) * c[src];
                        G(post, src, i, id) -= r;
                        G(post, prod, i, id) += r;
                    }
                }
            } else {
                for (int i = 0; i < 5; ++i) {
                    double r1 = k[id] * d5w(i) * c[0];
                    G(post, 0, i, id) -= r1;
                    if (ns >= 2) G(post, 1, i, id) += r1;
                    if (ns == 3 && k2) {
                        double r2 = k2[id] * d5w(i) * c[1];
                        G(post, 1, i, id) -= r2;
                        G(post, 2, i, id) += r2;
                    }
                }
            }
        }
    /* stream with boundary conditions */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t id = (size_t)y * nx + x;
            for (int s = 0; s < ns; ++s) {
                if (type[id] != 0) {
                    for (int i = 0; i < 5; ++i) G(gout, s, i, id) = 0.0;
                    continue;
                }
                G(gout, s, 0, id) = G(post, s, 0, id);
                for (int i = 1; i < 5; ++i) {
                    int sx = x - D5X[i], sy = y - D5Y[i];
                    if (bc & REF_PERIODIC_X) sx = wrap(sx, nx);
                    if (bc & REF_PERIODIC_Y) sy = wrap(sy, ny);
                    double val;
                    if (sx < 0) {
                        /* inlet (only i = E reaches here): anti-bounce-back
                         * with C_w = c_in for A (Eq. BC); bounce-back for B, C */
                        if (s == 0)
                            val = -G(post, s, W, id) + 2.0 * d5w(E) * c_in;
                        else
                            val = G(post, s, W, id);
                    } else if (sx >= nx) {
                        /* outlet (only i = W): anti-bounce-back with C_w = C_b,
                         * C_b the concentration of the boundary node itself */
                        double cb = 0.0;
                        for (int j = 0; j < 5; ++j) cb += G(post, s, j, id);
                        val = -G(post, s, E, id) + 2.0 * d5w(W) * cb;
                    } else if (sy < 0 || sy >= ny || type[(size_t)sy * nx + sx] != 0) {
                        val = G(post, s, D5OPP[i], id); /* bounce-back */
                    } else {
                        val = G(post, s, i, (size_t)sy * nx + sx);
                    }
                    G(gout, s, i, id) = val;
                }
            }
        }
#undef G
}

/* Run nsteps steps in place on g.  If conc_trace is non-NULL it receives, for
 * step t (0-based), the pre-collision concentration field [ns][ny][nx] at
 * offset t*ns*nx*ny. */
void ref_adr_run(int nx, int ny, int ns, const uint8_t *type, const double *k,
                 const double *k2, const double *ux, const double *uy, double vel_scale,
                 double tau, double c_in, int mode, int bc, double *g, long nsteps,
                 double *conc_trace)
{
    size_t n = (size_t)nx * ny;
    size_t bytes = sizeof(double) * (size_t)ns * 5 * n;
    double *tmp = (double *)malloc(bytes), *post = (double *)calloc(1, bytes);
    for (long t = 0; t < nsteps; ++t) {
        adr_step(nx, ny, ns, type, k, k2, ux, uy, vel_scale, tau, c_in, mode, bc, g, tmp, post,
                 conc_trace ? conc_trace + (size_t)t * ns * n : NULL);
        memcpy(g, tmp, bytes);
    }
    free(tmp);
    free(post);
}

/* Outlet fluxes after at least one step: N_s is the net number of particles
 * of species s that crossed the face between columns xf and xf+1 in the last
 * streaming (right-moving minus left-moving populations, summed over the rows
 * where both nodes are fluid).  inflow is the net flux of A through the inlet
 * face in the last streaming. */
void ref_adr_observe(int nx, int ny, int ns, const uint8_t *type, const double *g,
                     double c_in, int xf, double *flux, double *inflow)
{
    size_t n = (size_t)nx * ny;
    for (int s = 0; s < ns; ++s) {
        double sum = 0.0;
        for (int y = 0; y < ny; ++y) {
            size_t a = (size_t)y * nx + xf, b = a + 1;
            if (type[a] != 0 || type[b] != 0) continue;
            sum += g[((size_t)s * 5 + E) * n + b] - g[((size_t)s * 5 + W) * n + a];
        }
        flux[s] = sum;
    }
    double in = 0.0;
    for (int y = 0; y < ny; ++y) {
        size_t a = (size_t)y * nx;
        if (type[a] != 0) continue;
        in += 2.0 * g[(size_t)E * n + a] - 2.0 * d5w(E) * c_in;
    }
    *inflow = in;
}

/* Concentration C = sum of populations (pre-collision), zero at solids. */
void ref_adr_concentration(int nx, int ny, int ns, const uint8_t *type, const double *g,
                           double *conc)
{
    size_t n = (size_t)nx * ny;
    for (int s = 0; s < ns; ++s)
        for (size_t id = 0; id < n; ++id) {
            double c = 0.0;
            if (type[id] == 0)
                for (int i = 0; i < 5; ++i) c += g[((size_t)s * 5 + i) * n + id];
            conc[(size_t)s * n + id] = c;
        }
}

/* Total amount of each species over the fluid nodes (pre-collision). */
/* Amount each reaction converts in the next step from the pre-collision
 * state g (Eq. source_lbm summed over the lattice): rate[0] A -> B and, with
 * three species, rate[1] B -> C.  Same reaction modes, rates and boundary
 * wrapping as adr_step: the concentration is the fluid node's pre-collision
 * one, summed over every reacting population. */
void ref_adr_production(int nx, int ny, int ns, const uint8_t *type, const double *k,
                        const double *k2, int mode, int bc, const double *g, double *rate)
{
    size_t n = (size_t)nx * ny;
    rate[0] = rate[1] = 0.0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t id = (size_t)y * nx + x;
            if (type[id] != 0) continue;
            double c[3] = {0, 0, 0};
            for (int s = 0; s < ns; ++s)
                for (int i = 0; i < 5; ++i) c[s] += g[((size_t)s * 5 + i) * n + id];
            if (mode == REF_LINK || mode == REF_NODE_AT_CATALYST) {
                double ksum[2] = {0, 0};
                int kcnt[2] = {0, 0};
                for (int i = 1; i < 5; ++i) {
                    int nxx = x + D5X[i], nyy = y + D5Y[i];
                    if (bc & REF_PERIODIC_X) nxx = wrap(nxx, nx);
                    if (bc & REF_PERIODIC_Y) nyy = wrap(nyy, ny);
                    if (nxx < 0 || nxx >= nx || nyy < 0 || nyy >= ny) continue;
                    size_t sid = (size_t)nyy * nx + nxx;
                    int q = type[sid] == 2 ? 0 : (type[sid] == 3 && ns == 3 ? 1 : -1);
                    if (q < 0) continue;
                    if (mode == REF_LINK)
                        rate[q] += k[sid] * d5w(i) * c[q];
                    else {
                        ksum[q] += k[sid];
                        kcnt[q]++;
                    }
                }
                if (mode == REF_NODE_AT_CATALYST)
                    for (int q = 0; q < 2; ++q)
                        if (kcnt[q])
                            for (int i = 0; i < 5; ++i) rate[q] += ksum[q] / kcnt[q] * d5w(i) * c[q];
            } else {
                for (int i = 0; i < 5; ++i) {
                    rate[0] += k[id] * d5w(i) * c[0];
                    if (ns == 3 && k2) rate[1] += k2[id] * d5w(i) * c[1];
                }
            }
        }
}

void ref_adr_totals(int nx, int ny, int ns, const uint8_t *type, const double *g, double *tot)
{
    size_t n = (size_t)nx * ny;
    for (int s = 0; s < ns; ++s) {
        double t = 0.0;
        for (size_t id = 0; id < n; ++id)
            if (type[id] == 0)
                for (int i = 0; i < 5; ++i) t += g[((size_t)s * 5 + i) * n + id];
        tot[s] = t;
    }
}
