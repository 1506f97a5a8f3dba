/*
 * lbref3d.c -- the oracle for the 3D form of the hybrid lattice-Boltzmann
 * scheme of Sitaru & Gekle, "Analytical and computational study of cascade
 * reaction processes in catalytic fibrous membranes" (arXiv 2109.04455):
 * the randomly oriented fibre membranes of Sec. "System geometry: Cascade
 * reaction" and Sec. "Membrane generation".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file.  It shares no code, header,
 * table or constant with the GPU library; plain FP64 loops in the paper's order
 * of operations (collide (+ react), then stream with boundary conditions).
 *
 * Conventions
 *   grid  x in [0,nx), y in [0,ny), z in [0,nz); linear index (z*ny + y)*nx + x
 *   node_type: 0 fluid, 1 inert solid, 2 catalyst type 1 (A->B),
 *              3 catalyst type 2 (B->C)
 *   flow populations [19][nz][ny][nx]; species populations [s][7][nz][ny][nx]
 *   The state held between steps is the PRE-collision population set.
 *
 * Flow (Sec. "Lattice-Boltzmann for the Navier-Stokes equation", Eq. LBE): the
 * paper drives a flow periodic in every direction with a uniform body force;
 * here D3Q19 BGK with that force entered by Guo's forcing scheme (Guo, Zheng
 * & Shi, Phys. Rev. E 65, 046308 (2002)): physical velocity
 * u = (sum c f + F/2)/rho, equilibrium at u, and the source
 * (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i.u) c_i].F added after collision.
 * Half-way bounce-back at solid nodes.
 *
 * ADR (Sec. "Lattice-Boltzmann for Advection-Diffusion-Reaction", Eqs.
 * LBE_ADE, BGK, the second-order equilibrium, source_lbm): D3Q7 with
 * w0 = 1/4, w1..6 = 1/8, so cs^2 = 1/4 and D = (tau_g - 1/2)/4; equilibrium
 * w_i C (1 + c.u/cs^2 + (c.u)^2/(2 cs^4) - u.u/(2 cs^2)).  Link reactions as in
 * 2D; inlet x = 0 and outlet x = nx-1 as in Eq. BC; periodic in y and z (the
 * paper leaves its other boundaries periodic).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- D3Q19: rest, 6 faces, 12 edges; opposite of i is i^1 for i >= 1 when
 * the list is ordered in (+, -) pairs. */
static const int Q19X[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int Q19Y[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int Q19Z[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static int q19opp(int i) { return i == 0 ? 0 : (i % 2 == 1 ? i + 1 : i - 1); }
static double q19w(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

/* ---- D3Q7: rest, +x, -x, +y, -y, +z, -z */
static const int Q7X[7] = {0, 1, -1, 0, 0, 0, 0};
static const int Q7Y[7] = {0, 0, 0, 1, -1, 0, 0};
static const int Q7Z[7] = {0, 0, 0, 0, 0, 1, -1};
static int q7opp(int i) { return i == 0 ? 0 : (i % 2 == 1 ? i + 1 : i - 1); }
static double q7w(int i) { return i == 0 ? 0.25 : 0.125; }

static int wrap(int a, int m) { return ((a % m) + m) % m; }

#define REF3_PERIODIC_X 1 /* ADR: periodic in x too (pins); y and z are always periodic */
#define REF3_LINK 0
#define REF3_NODE 1 /* every population of a fluid node reacts, rates k, k2 at the node (pins) */

/* ---------------------------------------------------------------- flow ---- */

static double feq19(int i, double rho, double ux, double uy, double uz)
{
    double cu = Q19X[i] * ux + Q19Y[i] * uy + Q19Z[i] * uz;
    return q19w(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy + uz * uz));
}

/* Initial state: rest fluid, rho = 1. */
void ref3_flow_init(int nx, int ny, int nz, const uint8_t *type, double *f)
{
    size_t n = (size_t)nx * ny * nz;
    for (int i = 0; i < 19; ++i)
        for (size_t id = 0; id < n; ++id) f[i * n + id] = type[id] == 0 ? q19w(i) : 0.0;
}

/* Physical velocity and density of a pre-collision state under the force. */
static void moments19(const double *f, size_t n, size_t id, const double F[3], double *rho,
                      double u[3])
{
    double r = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < 19; ++i) {
        double v = f[i * n + id];
        r += v;
        j[0] += Q19X[i] * v;
        j[1] += Q19Y[i] * v;
        j[2] += Q19Z[i] * v;
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / r;
}

static void flow_step(int nx, int ny, int nz, const uint8_t *type, double tau, const double F[3],
                      const double *f, double *fout, double *post)
{
    size_t n = (size_t)nx * ny * nz;
    for (size_t id = 0; id < n; ++id) {
        if (type[id] != 0) continue;
        double rho, u[3];
        moments19(f, n, id, F, &rho, u);
        for (int i = 0; i < 19; ++i) {
            double c[3] = {Q19X[i], Q19Y[i], Q19Z[i]};
            double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
            double src = 0.0;
            for (int a = 0; a < 3; ++a) src += (3.0 * (c[a] - u[a]) + 9.0 * cu * c[a]) * F[a];
            src *= (1.0 - 0.5 / tau) * q19w(i);
            post[i * n + id] = f[i * n + id] - (f[i * n + id] - feq19(i, rho, u[0], u[1], u[2])) / tau + src;
        }
    }
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t id = ((size_t)z * ny + y) * nx + x;
                for (int i = 0; i < 19; ++i) {
                    if (type[id] != 0) {
                        fout[i * n + id] = 0.0;
                        continue;
                    }
                    int sx = wrap(x - Q19X[i], nx), sy = wrap(y - Q19Y[i], ny), sz = wrap(z - Q19Z[i], nz);
                    size_t sid = ((size_t)sz * ny + sy) * nx + sx;
                    fout[i * n + id] = type[sid] != 0 ? post[q19opp(i) * n + id] : post[i * n + sid];
                }
            }
}

void ref3_flow_run(int nx, int ny, int nz, const uint8_t *type, double tau, double fx, double fy,
                   double fz, double *f, long nsteps)
{
    size_t bytes = sizeof(double) * 19 * (size_t)nx * ny * nz;
    double *tmp = (double *)malloc(bytes), *post = (double *)calloc(1, bytes);
    const double F[3] = {fx, fy, fz};
    for (long t = 0; t < nsteps; ++t) {
        flow_step(nx, ny, nz, type, tau, F, f, tmp, post);
        memcpy(f, tmp, bytes);
    }
    free(tmp);
    free(post);
}

/* Velocity (u = (sum c f + F/2)/rho) and density; zero at solid nodes. */
void ref3_flow_velocity(int nx, int ny, int nz, const uint8_t *type, const double *f, double fx,
                        double fy, double fz, double *ux, double *uy, double *uz, double *rho_out)
{
    size_t n = (size_t)nx * ny * nz;
    const double F[3] = {fx, fy, fz};
    for (size_t id = 0; id < n; ++id) {
        double rho = 0.0, u[3] = {0, 0, 0};
        if (type[id] == 0) moments19(f, n, id, F, &rho, u);
        ux[id] = u[0];
        uy[id] = u[1];
        uz[id] = u[2];
        if (rho_out) rho_out[id] = rho;
    }
}

/* ----------------------------------------------------------------- ADR ---- */

static double geq7(int i, double c, double ux, double uy, double uz)
{
    double cu = Q7X[i] * ux + Q7Y[i] * uy + Q7Z[i] * uz;
    return q7w(i) * c * (1.0 + 4.0 * cu + 8.0 * cu * cu - 2.0 * (ux * ux + uy * uy + uz * uz));
}

/* Species A at equilibrium with C = c_in and the velocity vel_scale*u at
 * every fluid node; B and C absent. */
void ref3_adr_init(int nx, int ny, int nz, int ns, const uint8_t *type, const double *ux,
                   const double *uy, const double *uz, double vel_scale, double c_in, double *g)
{
    size_t n = (size_t)nx * ny * nz;
    for (int s = 0; s < ns; ++s)
        for (int i = 0; i < 7; ++i)
            for (size_t id = 0; id < n; ++id) {
                double v = 0.0;
                if (s == 0 && type[id] == 0)
                    v = geq7(i, c_in, vel_scale * ux[id], vel_scale * uy[id], vel_scale * uz[id]);
                g[((size_t)s * 7 + i) * n + id] = v;
            }
}

#define G(arr, s, i, id) arr[((size_t)(s) * 7 + (i)) * n + (id)]

static void adr_step(int nx, int ny, int nz, int ns, const uint8_t *type, const double *k,
                     const double *k2, const double *ux, const double *uy, const double *uz,
                     double vel_scale, double tau, double c_in, int mode, int bc, const double *g,
                     double *gout, double *post)
{
    size_t n = (size_t)nx * ny * nz;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t id = ((size_t)z * ny + y) * nx + x;
                if (type[id] != 0) continue;
                double u = vel_scale * ux[id], v = vel_scale * uy[id], w = vel_scale * uz[id];
                double c[3] = {0, 0, 0};
                for (int s = 0; s < ns; ++s)
                    for (int i = 0; i < 7; ++i) c[s] += G(g, s, i, id);
                for (int s = 0; s < ns; ++s)
                    for (int i = 0; i < 7; ++i)
                        G(post, s, i, id) = G(g, s, i, id) - (G(g, s, i, id) - geq7(i, c[s], u, v, w)) / tau;
                if (mode == REF3_LINK) {
                    /* the population heading into a catalytic node reacts with
                     * that node's rate and the fluid node's concentration */
                    for (int i = 1; i < 7; ++i) {
                        int xx = x + Q7X[i];
                        if (bc & REF3_PERIODIC_X) xx = wrap(xx, nx);
                        if (xx < 0 || xx >= nx) continue;
                        size_t sid = ((size_t)wrap(z + Q7Z[i], nz) * ny + wrap(y + Q7Y[i], ny)) * nx + xx;
                        int src, prod;
                        if (type[sid] == 2) {
                            src = 0;
                            prod = 1;
                        } else if (type[sid] == 3 && ns == 3) {
                            src = 1;
                            prod = 2;
                        } else {
                            continue;
                        }
                        double r = k[sid] * q7w(i) * c[src];
                        G(post, src, i, id) -= r;
                        G(post, prod, i, id) += r;
                    }
                } else {
                    for (int i = 0; i < 7; ++i) {
                        double r1 = k[id] * q7w(i) * c[0];
                        G(post, 0, i, id) -= r1;
                        if (ns >= 2) G(post, 1, i, id) += r1;
                        if (ns == 3 && k2) {
                            double r2 = k2[id] * q7w(i) * c[1];
                            G(post, 1, i, id) -= r2;
                            G(post, 2, i, id) += r2;
                        }
                    }
                }
            }
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t id = ((size_t)z * ny + y) * nx + x;
                for (int s = 0; s < ns; ++s) {
                    if (type[id] != 0) {
                        for (int i = 0; i < 7; ++i) G(gout, s, i, id) = 0.0;
                        continue;
                    }
                    G(gout, s, 0, id) = G(post, s, 0, id);
                    for (int i = 1; i < 7; ++i) {
                        int sx = x - Q7X[i];
                        if (bc & REF3_PERIODIC_X) sx = wrap(sx, nx);
                        double val;
                        if (sx < 0) {
                            /* inlet, Eq. BC: anti-bounce-back with C_w = c_in for
                             * A, bounce-back for B and C */
                            val = s == 0 ? -G(post, s, 2, id) + 2.0 * q7w(1) * c_in : G(post, s, 2, id);
                        } else if (sx >= nx) {
                            /* outlet: anti-bounce-back with C_w = C_b of the node */
                            double cb = 0.0;
                            for (int j = 0; j < 7; ++j) cb += G(post, s, j, id);
                            val = -G(post, s, 1, id) + 2.0 * q7w(2) * cb;
                        } else {
                            size_t sid = ((size_t)wrap(z - Q7Z[i], nz) * ny + wrap(y - Q7Y[i], ny)) * nx + sx;
                            val = type[sid] != 0 ? G(post, s, q7opp(i), id) : G(post, s, i, sid);
                        }
                        G(gout, s, i, id) = val;
                    }
                }
            }
}

void ref3_adr_run(int nx, int ny, int nz, int ns, const uint8_t *type, const double *k,
                  const double *k2, const double *ux, const double *uy, const double *uz,
                  double vel_scale, double tau, double c_in, int mode, int bc, double *g,
                  long nsteps)
{
    size_t n = (size_t)nx * ny * nz;
    size_t bytes = sizeof(double) * (size_t)ns * 7 * n;
    double *tmp = (double *)malloc(bytes), *post = (double *)calloc(1, bytes);
    for (long t = 0; t < nsteps; ++t) {
        adr_step(nx, ny, nz, ns, type, k, k2, ux, uy, uz, vel_scale, tau, c_in, mode, bc, g, tmp,
                 post);
        memcpy(g, tmp, bytes);
    }
    free(tmp);
    free(post);
}

/* Net flux of each species through the face between x = xf and xf + 1 in the
 * last streaming, summed over (y, z) where both nodes are fluid; inflow of A
 * through the inlet face. */
void ref3_adr_observe(int nx, int ny, int nz, int ns, const uint8_t *type, const double *g,
                      double c_in, int xf, double *flux, double *inflow)
{
    size_t n = (size_t)nx * ny * nz;
    for (int s = 0; s < ns; ++s) {
        double sum = 0.0;
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y) {
                size_t a = ((size_t)z * ny + y) * nx + xf, b = a + 1;
                if (type[a] != 0 || type[b] != 0) continue;
                sum += G(g, s, 1, b) - G(g, s, 2, a);
            }
        flux[s] = sum;
    }
    double in = 0.0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
            size_t a = ((size_t)z * ny + y) * nx;
            if (type[a] != 0) continue;
            in += 2.0 * G(g, 0, 1, a) - 2.0 * q7w(1) * c_in;
        }
    *inflow = in;
}

void ref3_adr_concentration(int nx, int ny, int nz, int ns, const uint8_t *type, const double *g,
                            double *conc)
{
    size_t n = (size_t)nx * ny * nz;
    for (int s = 0; s < ns; ++s)
        for (size_t id = 0; id < n; ++id) {
            double c = 0.0;
            if (type[id] == 0)
                for (int i = 0; i < 7; ++i) c += G(g, s, i, id);
            conc[(size_t)s * n + id] = c;
        }
}

#undef G

/* Total amount of each species over the fluid nodes (pre-collision). */
void ref3_adr_totals(int nx, int ny, int nz, int ns, const uint8_t *type, const double *g,
                     double *tot)
{
    size_t n = (size_t)nx * ny * nz;
    for (int s = 0; s < ns; ++s) {
        double t = 0.0;
        for (size_t id = 0; id < n; ++id)
            if (type[id] == 0)
                for (int i = 0; i < 7; ++i) t += g[((size_t)s * 7 + i) * n + id];
        tot[s] = t;
    }
}
