/* sor_oracle.c - FP64 reference of red-black successive over-relaxation for the
 * pressure Poisson equation (TEST INFRASTRUCTURE ONLY: used by tests/, the package smoke
 * check and the benchmark's CPU-baseline leg; shares no code with the HIP path).
 *
 * The paper's second workload (Sect. 6.3) solves a Poisson equation for the pressure with
 * successive over-relaxation, 50 iterations on a 300 x 300 x 90 grid. It gives no
 * discretisation; the reading implemented here:
 *   - cells (i, j, k), arrays [nz][ny][nx] row-major; the outermost layer of cells holds
 *     fixed (Dirichlet) values that are read but never written;
 *   - the 7-point Laplacian L p = cx (pE + pW - 2p) + cy (pN + pS - 2p) + cz (pU + pD - 2p),
 *     cx = 1/dx^2, cy = 1/dy^2, cz = 1/dz^2, and the equation L p = f on interior cells;
 *   - one iteration = a sweep over the red cells ((i + j + k) even), then one over the black
 *     cells, each cell set to p + omega (g - p) with the Gauss-Seidel value
 *     g = (cx (pE + pW) + cy (pN + pS) + cz (pU + pD) - f) / (2 (cx + cy + cz));
 *   - after every iteration the residual r = f - L p over the interior cells is folded into
 *     its sum of squares (fixed order: k, then j, then i) and its largest magnitude.
 * Plain loops over the whole grid per sweep, in that order.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#define IX(i, j, k) (((size_t)(k) * (size_t)ny + (size_t)(j)) * (size_t)nx + (size_t)(i))

static void sweep(int nx, int ny, int nz, double cx, double cy, double cz, double omega, int color, double* p,
                  const double* f) {
    const double diag = 2.0 * (cx + cy + cz);
#pragma omp parallel for schedule(static)
    for (int k = 1; k < nz - 1; ++k)
        for (int j = 1; j < ny - 1; ++j)
            for (int i = 1; i < nx - 1; ++i) {
                if (((i + j + k) & 1) != color) continue;
                const double nb = cx * (p[IX(i + 1, j, k)] + p[IX(i - 1, j, k)]) +
                                  cy * (p[IX(i, j + 1, k)] + p[IX(i, j - 1, k)]) +
                                  cz * (p[IX(i, j, k + 1)] + p[IX(i, j, k - 1)]);
                const double g = (nb - f[IX(i, j, k)]) / diag;
                const double old = p[IX(i, j, k)];
                p[IX(i, j, k)] = old + omega * (g - old);
            }
}

/* r = f - L p on the interior; sum of r^2 (k, j, i order) and max |r| */
static void residual(int nx, int ny, int nz, double cx, double cy, double cz, const double* p, const double* f,
                     double* sum_r2, double* max_abs_r) {
    double s = 0.0, m = 0.0;
    for (int k = 1; k < nz - 1; ++k)
        for (int j = 1; j < ny - 1; ++j)
            for (int i = 1; i < nx - 1; ++i) {
                const double c = p[IX(i, j, k)];
                const double lap = cx * (p[IX(i + 1, j, k)] + p[IX(i - 1, j, k)] - 2.0 * c) +
                                   cy * (p[IX(i, j + 1, k)] + p[IX(i, j - 1, k)] - 2.0 * c) +
                                   cz * (p[IX(i, j, k + 1)] + p[IX(i, j, k - 1)] - 2.0 * c);
                const double r = f[IX(i, j, k)] - lap;
                s += r * r;
                if (fabs(r) > m) m = fabs(r);
            }
    *sum_r2 = s;
    *max_abs_r = m;
}

/* Run iters iterations on p (in place). res[2 n] = sum r^2, res[2 n + 1] = max |r| after
 * iteration n + 1. Returns 0, or -1 for an invalid argument. */
int sor_oracle_run(int nx, int ny, int nz, double dx, double dy, double dz, double omega, int iters, double* p,
                   const double* f, double* res) {
    if (nx < 3 || ny < 3 || nz < 3 || iters < 0 || !(dx > 0.0) || !(dy > 0.0) || !(dz > 0.0) || !p || !f)
        return -1;
    const double cx = 1.0 / (dx * dx), cy = 1.0 / (dy * dy), cz = 1.0 / (dz * dz);
    for (int n = 0; n < iters; ++n) {
        sweep(nx, ny, nz, cx, cy, cz, omega, 0, p, f);
        sweep(nx, ny, nz, cx, cy, cz, omega, 1, p, f);
        if (res) residual(nx, ny, nz, cx, cy, cz, p, f, &res[2 * n], &res[2 * n + 1]);
    }
    return 0;
}

/* The residual alone (sum r^2, max |r|) of a state. */
int sor_oracle_residual(int nx, int ny, int nz, double dx, double dy, double dz, const double* p, const double* f,
                        double* out2) {
    if (nx < 3 || ny < 3 || nz < 3 || !p || !f || !out2) return -1;
    residual(nx, ny, nz, 1.0 / (dx * dx), 1.0 / (dy * dy), 1.0 / (dz * dz), p, f, &out2[0], &out2[1]);
    return 0;
}
