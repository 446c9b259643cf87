/*
 * FP64 CPU oracle for one time step of the 2-D shallow-water model (2DSW).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg may build, load or call this file. It shares no
 * code, header or constant with the HIP path.
 *
 * What the paper fixes (Sect. 6.2, "Test Case 1: 2-D Shallow Water Model"): the
 * model is a time loop that calls a predictor ("dyn") and a first-order Shapiro
 * filter ("shapiro") and then updates the velocity. It gives no equations, so
 * the discretisation below is a reading of that description:
 *
 *  - Arakawa C grid on a closed basin with a static land mask. Every field is a
 *    row-major [ny][nx] array; u[j][i] lives on the east face of cell (j,i),
 *    v[j][i] on its north face. A face is active when both cells it joins are
 *    water; inactive faces carry exactly zero.
 *  - dyn, part 1 (momentum predictor, pressure gradient only):
 *        us = u - (g dt/dx) (eta_E - eta),   vs = v - (g dt/dy) (eta_N - eta)
 *  - dyn, part 2 (free surface from the flux divergence, forward-backward in
 *    time: the fluxes use the predicted velocities and the total depth
 *    h = H + eta of the old surface, upwinded by the sign of the face velocity):
 *        es = eta - (dt/dx)(Fx_e - Fx_w) - (dt/dy)(Fy_n - Fy_s)
 *  - shapiro (first-order, five-point, only across active faces):
 *        eta' = es + (eps/4) * sum over water neighbours (es_nb - es)
 *  - velocity update: u' = us, v' = vs.
 *  - model variants (flags; a reading of the textbook family the paper's model comes
 *    from, none of them in the paper): quadratic bottom friction on the predictor,
 *        us = (u - (g dt/dx)(eta_E - eta)) / (1 + dt cd |u| / h_face),
 *    h_face = mean total depth of the face's two cells (old surface, old |u|), vs
 *    likewise; and the Shapiro filter applied to the predicted velocities as well,
 *        u' = us + (eps/4) * sum over active neighbouring u faces (us_nb - us)
 *    (neighbours east, west, north, south), v' likewise, after the surface update
 *    used the unfiltered us, vs; and nonlinear momentum advection, first-order upwind,
 *        us -= dt (u du/dx + vbar du/dy),  vs -= dt (ubar dv/dx + v dv/dy),
 *    each derivative a one-sided difference on the upstream side of its advecting
 *    velocity, vbar the mean of the four v faces around the u face and ubar likewise,
 *    neighbours off the grid or on inactive faces counted as 0.
 *  - wetting and drying (variant): a water cell is wet while its total depth
 *    H + eta exceeds a threshold hmin (a choice of the caller; the datum may sit above
 *    the still-water level, so ground that can flood is a water cell with a small or
 *    zero total depth). A face between two water cells carries flow when both cells
 *    are wet, or when one is wet and its surface stands higher than the other's, so
 *    the pressure gradient pushes water into the dry cell; otherwise its predicted
 *    velocity is 0. Every water cell takes the flux divergence; the Shapiro filter
 *    acts on wet cells only and exchanges with wet neighbours only (a dry cell keeps
 *    its predicted surface). Wet flags come from the old surface.
 *  - Per-step folds: V_disp = dx dy sum_wet eta', V_tot = dx dy sum_wet (H + eta'),
 *    max|u'|, max|v'|. The paper's compiler turns loop nests into maps and
 *    these reductions into folds (Sect. 4.3).
 *
 * Plain loops, one full-size array per intermediate, no blocking or fusion.
 * Rows are independent in every stage, so OpenMP over rows changes no result.
 * Build: gcc -O3 -march=native -fopenmp -ffp-contract=off (no fast-math).
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(a, j, i) ((a)[(size_t)(j) * (size_t)nx + (size_t)(i)])

static int is_wet(const unsigned char *mask, int nx, int ny, int j, int i) {
    if (i < 0 || j < 0 || i >= nx || j >= ny) return 0;
    return AT(mask, j, i) != 0;
}

#define SW2D_ORACLE_FRICTION 1
#define SW2D_ORACLE_FILTER_UV 2
#define SW2D_ORACLE_ADVECTION 4
#define SW2D_ORACLE_WETDRY 8

/* wet/dry variant: a water cell takes part in the dynamics while its total depth
 * exceeds hmin; land is never wet */
static int wet_now(const double *H, const double *eta, const unsigned char *mask, int nx, int ny,
                   int j, int i, double hmin) {
    return is_wet(mask, nx, ny, j, i) && AT(H, j, i) + AT(eta, j, i) > hmin;
}

/* wet/dry variant: a face between cells a and b (both water) passes flow when both are
 * wet, or when one of them is wet and its surface stands above the other's */
static int face_open(int wa, int wb, double ea, double eb) {
    return (wa && wb) || (wa && ea > eb) || (wb && eb > ea);
}

/* the neighbours the surface filter exchanges with: water cells, or, with wetting and
 * drying, wet cells */
static int filter_nb(const double *H, const double *eta, const unsigned char *mask, int nx, int ny,
                     int j, int i, int wd, double hmin) {
    return wd ? wet_now(H, eta, mask, nx, ny, j, i, hmin) : is_wet(mask, nx, ny, j, i);
}

/* a face value, 0 off the grid */
static double face_at(const double *a, int nx, int ny, int j, int i) {
    if (i < 0 || j < 0 || i >= nx || j >= ny) return 0.0;
    return AT(a, j, i);
}

/* first-order upwind advection of the u face (j,i): u du/dx + vbar du/dy */
static double advect_u(const double *u, const double *v, int nx, int ny, int j, int i, double dx, double dy) {
    const double c = AT(u, j, i);
    const double vbar = 0.25 * ((face_at(v, nx, ny, j, i) + face_at(v, nx, ny, j, i + 1)) +
                                (face_at(v, nx, ny, j - 1, i) + face_at(v, nx, ny, j - 1, i + 1)));
    const double ax = c > 0.0 ? c * (c - face_at(u, nx, ny, j, i - 1)) / dx
                              : c * (face_at(u, nx, ny, j, i + 1) - c) / dx;
    const double ay = vbar > 0.0 ? vbar * (c - face_at(u, nx, ny, j - 1, i)) / dy
                                 : vbar * (face_at(u, nx, ny, j + 1, i) - c) / dy;
    return ax + ay;
}

/* first-order upwind advection of the v face (j,i): ubar dv/dx + v dv/dy */
static double advect_v(const double *u, const double *v, int nx, int ny, int j, int i, double dx, double dy) {
    const double c = AT(v, j, i);
    const double ubar = 0.25 * ((face_at(u, nx, ny, j, i) + face_at(u, nx, ny, j, i - 1)) +
                                (face_at(u, nx, ny, j + 1, i) + face_at(u, nx, ny, j + 1, i - 1)));
    const double bx = ubar > 0.0 ? ubar * (c - face_at(v, nx, ny, j, i - 1)) / dx
                                 : ubar * (face_at(v, nx, ny, j, i + 1) - c) / dx;
    const double by = c > 0.0 ? c * (c - face_at(v, nx, ny, j - 1, i)) / dy
                              : c * (face_at(v, nx, ny, j + 1, i) - c) / dy;
    return bx + by;
}

/* active u face (east face of cell j,i) and active v face (north face) */
static int u_face(const unsigned char *mask, int nx, int ny, int j, int i) {
    return is_wet(mask, nx, ny, j, i) && is_wet(mask, nx, ny, j, i + 1);
}
static int v_face(const unsigned char *mask, int nx, int ny, int j, int i) {
    return is_wet(mask, nx, ny, j, i) && is_wet(mask, nx, ny, j + 1, i);
}

/* Shapiro smoothing of face values a (active where act() says so) into out */
static void filter_faces(int nx, int ny, double e4, const unsigned char *mask, const double *a, double *out,
                         int (*act)(const unsigned char *, int, int, int, int)) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            double o = 0.0;
            if (act(mask, nx, ny, j, i)) {
                double c = AT(a, j, i);
                double s = 0.0;
                if (act(mask, nx, ny, j, i + 1)) s += AT(a, j, i + 1) - c;
                if (act(mask, nx, ny, j, i - 1)) s += AT(a, j, i - 1) - c;
                if (act(mask, nx, ny, j + 1, i)) s += AT(a, j + 1, i) - c;
                if (act(mask, nx, ny, j - 1, i)) s += AT(a, j - 1, i) - c;
                o = c + e4 * s;
            }
            AT(out, j, i) = o;
        }
    }
}

/* One step. scratch holds 3*nx*ny doubles (Fx, Fy, es). flags: SW2D_ORACLE_FRICTION
 * (quadratic bottom friction with coefficient cd), SW2D_ORACLE_FILTER_UV,
 * SW2D_ORACLE_ADVECTION, SW2D_ORACLE_WETDRY (threshold hmin). Returns 0, or 1 if a
 * water cell has non-positive total depth H + eta without SW2D_ORACLE_WETDRY.
 * wd_margin, if not NULL, holds 2 doubles that are lowered to this step's smallest
 * distance of a wet/dry decision from its threshold: [0] |H + eta - hmin| over water
 * cells, [1] |eta_a - eta_b| over faces between a wet and a dry water cell. */
int sw2d_oracle_step(int nx, int ny, double dx, double dy, double g, double dt, double eps,
                     const double *H, const unsigned char *mask,
                     const double *eta, const double *u, const double *v,
                     double *eta_out, double *u_out, double *v_out,
                     double *scratch, int nthreads, int flags, double cd, double hmin,
                     double *wd_margin) {
    const double cx = g * dt / dx, cy = g * dt / dy;
    const double kf = dt * cd;
    const double rx = dt / dx, ry = dt / dy;
    const double e4 = eps / 4.0;
    double *Fx = scratch;
    double *Fy = scratch + (size_t)nx * ny;
    double *es = scratch + 2 * (size_t)nx * ny;
    const int wd = (flags & SW2D_ORACLE_WETDRY) != 0;
    int dry = 0;
    double mh = INFINITY, me = INFINITY;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

    /* dyn, part 1: predicted face velocities; then the upwinded face fluxes. */
#pragma omp parallel for schedule(static) reduction(| : dry) reduction(min : mh, me)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            int w = is_wet(mask, nx, ny, j, i);
            if (w && !wd && !(AT(H, j, i) + AT(eta, j, i) > 0.0)) dry = 1;
            int au = w && is_wet(mask, nx, ny, j, i + 1);
            int av = w && is_wet(mask, nx, ny, j + 1, i);
            if (wd && w) {
                const int d = wet_now(H, eta, mask, nx, ny, j, i, hmin);
                const int dE = wet_now(H, eta, mask, nx, ny, j, i + 1, hmin);
                const int dN = wet_now(H, eta, mask, nx, ny, j + 1, i, hmin);
                mh = fmin(mh, fabs(AT(H, j, i) + AT(eta, j, i) - hmin));
                if (au && d != dE) me = fmin(me, fabs(AT(eta, j, i) - AT(eta, j, i + 1)));
                if (av && d != dN) me = fmin(me, fabs(AT(eta, j, i) - AT(eta, j + 1, i)));
                au = au && face_open(d, dE, AT(eta, j, i), AT(eta, j, i + 1));
                av = av && face_open(d, dN, AT(eta, j, i), AT(eta, j + 1, i));
            }
            double us = 0.0, vs = 0.0, fx = 0.0, fy = 0.0;
            if (au) {
                us = AT(u, j, i) - cx * (AT(eta, j, i + 1) - AT(eta, j, i));
                if (flags & SW2D_ORACLE_ADVECTION) us = us - dt * advect_u(u, v, nx, ny, j, i, dx, dy);
                if (flags & SW2D_ORACLE_FRICTION) {
                    double hf = 0.5 * ((AT(H, j, i) + AT(eta, j, i)) + (AT(H, j, i + 1) + AT(eta, j, i + 1)));
                    us = us / (1.0 + kf * fabs(AT(u, j, i)) / hf);
                }
                double h_up = us > 0.0 ? AT(H, j, i) + AT(eta, j, i)
                                       : AT(H, j, i + 1) + AT(eta, j, i + 1);
                fx = us * h_up;
            }
            if (av) {
                vs = AT(v, j, i) - cy * (AT(eta, j + 1, i) - AT(eta, j, i));
                if (flags & SW2D_ORACLE_ADVECTION) vs = vs - dt * advect_v(u, v, nx, ny, j, i, dx, dy);
                if (flags & SW2D_ORACLE_FRICTION) {
                    double hf = 0.5 * ((AT(H, j, i) + AT(eta, j, i)) + (AT(H, j + 1, i) + AT(eta, j + 1, i)));
                    vs = vs / (1.0 + kf * fabs(AT(v, j, i)) / hf);
                }
                double h_up = vs > 0.0 ? AT(H, j, i) + AT(eta, j, i)
                                       : AT(H, j + 1, i) + AT(eta, j + 1, i);
                fy = vs * h_up;
            }
            AT(u_out, j, i) = us;
            AT(v_out, j, i) = vs;
            AT(Fx, j, i) = fx;
            AT(Fy, j, i) = fy;
        }
    }

    /* dyn, part 2: free surface from the divergence of the fluxes. */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            double e = 0.0;
            if (is_wet(mask, nx, ny, j, i)) {
                double fw = i > 0 ? AT(Fx, j, i - 1) : 0.0;
                double fs = j > 0 ? AT(Fy, j - 1, i) : 0.0;
                e = AT(eta, j, i) - rx * (AT(Fx, j, i) - fw) - ry * (AT(Fy, j, i) - fs);
            }
            AT(es, j, i) = e;
        }
    }

    /* shapiro: five-point smoothing that only exchanges across water neighbours. */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            double out = 0.0;
            if (is_wet(mask, nx, ny, j, i)) {
                double c = AT(es, j, i);
                double s = 0.0;
                if (filter_nb(H, eta, mask, nx, ny, j, i + 1, wd, hmin)) s += AT(es, j, i + 1) - c;
                if (filter_nb(H, eta, mask, nx, ny, j, i - 1, wd, hmin)) s += AT(es, j, i - 1) - c;
                if (filter_nb(H, eta, mask, nx, ny, j + 1, i, wd, hmin)) s += AT(es, j + 1, i) - c;
                if (filter_nb(H, eta, mask, nx, ny, j - 1, i, wd, hmin)) s += AT(es, j - 1, i) - c;
                /* with wetting and drying a dry cell keeps its predicted surface */
                out = (wd && !wet_now(H, eta, mask, nx, ny, j, i, hmin)) ? c : c + e4 * s;
            }
            AT(eta_out, j, i) = out;
        }
    }

    /* variant: the velocity update filters the predicted velocities (Fx, Fy are free now) */
    if (flags & SW2D_ORACLE_FILTER_UV) {
        filter_faces(nx, ny, e4, mask, u_out, Fx, u_face);
        filter_faces(nx, ny, e4, mask, v_out, Fy, v_face);
        memcpy(u_out, Fx, sizeof(double) * (size_t)nx * ny);
        memcpy(v_out, Fy, sizeof(double) * (size_t)nx * ny);
    }
    if (wd_margin) {
        wd_margin[0] = fmin(wd_margin[0], mh);
        wd_margin[1] = fmin(wd_margin[1], me);
    }
    return dry;
}

/* Folds over one state: out[0] = V_tot, out[1] = V_disp, out[2] = max|u|, out[3] = max|v|.
 * Sums run row by row; the row sums are then added in row order, so the result does
 * not depend on the thread count. rowbuf holds 2*ny doubles. */
void sw2d_oracle_reduce(int nx, int ny, double dx, double dy, const double *H,
                        const unsigned char *mask, const double *eta, const double *u,
                        const double *v, double *out, double *rowbuf) {
    double *row_tot = rowbuf, *row_disp = rowbuf + ny;
    double mu = 0.0, mv = 0.0;
#pragma omp parallel for schedule(static) reduction(max : mu, mv)
    for (int j = 0; j < ny; ++j) {
        double st = 0.0, sd = 0.0;
        for (int i = 0; i < nx; ++i) {
            if (AT(mask, j, i)) {
                st += AT(H, j, i) + AT(eta, j, i);
                sd += AT(eta, j, i);
            }
            double au = fabs(AT(u, j, i)), av = fabs(AT(v, j, i));
            if (au > mu) mu = au;
            if (av > mv) mv = av;
        }
        row_tot[j] = st;
        row_disp[j] = sd;
    }
    double st = 0.0, sd = 0.0;
    for (int j = 0; j < ny; ++j) {
        st += row_tot[j];
        sd += row_disp[j];
    }
    out[0] = dx * dy * st;
    out[1] = dx * dy * sd;
    out[2] = mu;
    out[3] = mv;
}

/* nsteps steps in place on (eta, u, v). red, if not NULL, receives 4 doubles per step
 * (the folds of the state after that step); wd_margin as for one step, over all steps.
 * Returns 0, 1 if a water cell dried (without wetting and drying), or 2 if memory ran out. */
int sw2d_oracle_run(int nx, int ny, double dx, double dy, double g, double dt, double eps,
                    const double *H, const unsigned char *mask,
                    double *eta, double *u, double *v, int nsteps, double *red, int nthreads, int flags,
                    double cd, double hmin, double *wd_margin) {
    size_t n = (size_t)nx * ny;
    double *buf = (double *)malloc(sizeof(double) * (6 * n + 2 * (size_t)ny));
    if (!buf) return 2;
    double *e2 = buf, *u2 = buf + n, *v2 = buf + 2 * n, *scratch = buf + 3 * n;
    double *rowbuf = buf + 6 * n;
    double *ce = eta, *cu = u, *cv = v, *ne = e2, *nu = u2, *nv = v2;
    int rc = 0;
    for (int s = 0; s < nsteps && rc == 0; ++s) {
        rc = sw2d_oracle_step(nx, ny, dx, dy, g, dt, eps, H, mask, ce, cu, cv, ne, nu, nv,
                              scratch, nthreads, flags, cd, hmin, wd_margin);
        if (red) sw2d_oracle_reduce(nx, ny, dx, dy, H, mask, ne, nu, nv, red + 4 * (size_t)s, rowbuf);
        double *t;
        t = ce; ce = ne; ne = t;
        t = cu; cu = nu; nu = t;
        t = cv; cv = nv; nv = t;
    }
    if (ce != eta) {
        memcpy(eta, ce, sizeof(double) * n);
        memcpy(u, cu, sizeof(double) * n);
        memcpy(v, cv, sizeof(double) * n);
    }
    free(buf);
    return rc;
}

int sw2d_oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
