/* Sanitizer driver for the C oracle (built with -fsanitize=address,undefined
 * by tests/test_sanitizers_cpu.py): every exported routine on small 2D and
 * 3D grids, both time schemes, the line solve over a range of sizes and
 * stiffnesses, and the series bookkeeping.  Exit 0 when every call succeeds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

uint64_t orc_splitmix64(uint64_t seed, uint64_t k);
void orc_init_field(int dim, const int32_t *n, double c0, double noise, uint64_t seed, double *C);
double orc_exact_sum(const double *x, int64_t m);
void orc_laplacian(int dim, const int32_t *n, const double *L, const double *f, double *out);
void orc_cross(int dim, const int32_t *n, const double *L, const double *f, double *out);
int orc_cyclic_penta_solve(int64_t n, double rho, const double *f, double *y);
int orc_step_theta(int dim, const int32_t *n, const double *L, double gamma, double dt, double theta,
                   double *C, int64_t nsteps);
double orc_energy(int dim, const int32_t *n, const double *L, double gamma, int conv, const double *C);
double orc_mean(int dim, const int32_t *n, const double *C);
double orc_dFdt_identity(int dim, const int32_t *n, const double *L, double gamma, const double *C);
int64_t orc_run_series_theta(int dim, const int32_t *n, const double *L, double gamma, double dt, double theta,
                             int conv, int32_t K, int64_t nsteps, double *C, double *out, int64_t cap);

static int grid_case(int dim, int32_t nx, int32_t ny, int32_t nz, double theta)
{
    const int32_t n[3] = {nx, ny, nz};
    const double L[3] = {6.283185307179586, 5.0, 4.0};
    const int64_t S = (int64_t)nx * ny * nz;
    double *C = malloc(sizeof(double) * S), *out = malloc(sizeof(double) * S);
    double series[6 * 4];
    orc_init_field(dim, n, 0.1, 0.1, 7, C);
    orc_laplacian(dim, n, L, C, out);
    orc_cross(dim, n, L, C, out);
    if (orc_step_theta(dim, n, L, 0.01, 1e-4, theta, C, 3) != 0) return 1;
    const double F = orc_energy(dim, n, L, 0.01, 0, C) + orc_energy(dim, n, L, 0.01, 1, C);
    const double m = orc_mean(dim, n, C), g = orc_dFdt_identity(dim, n, L, 0.01, C);
    if (orc_run_series_theta(dim, n, L, 0.01, 1e-4, theta, 0, 4, 12, C, series, 4) != 4) return 1;
    free(C);
    free(out);
    return !(isfinite(F) && isfinite(m) && isfinite(g));
}

int main(void)
{
    int bad = 0;
    (void)orc_splitmix64(1234567, 1);
    const int sizes[] = {1, 2, 3, 4, 5, 8, 13, 64, 100};
    const double rhos[] = {1e-3, 1.0, 441.0, 1764.0, 1e6};
    for (unsigned a = 0; a < sizeof sizes / sizeof *sizes; ++a)
        for (unsigned b = 0; b < sizeof rhos / sizeof *rhos; ++b) {
            const int n = sizes[a];
            double *f = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * n);
            for (int i = 0; i < n; ++i) f[i] = sin(1.0 + i);
            if (n >= 5) bad |= orc_cyclic_penta_solve(n, rhos[b], f, y) != 0;
            (void)orc_exact_sum(f, n);
            free(f);
            free(y);
        }
    bad |= grid_case(2, 16, 8, 1, 1.0);
    bad |= grid_case(2, 16, 8, 1, 0.5);
    bad |= grid_case(2, 8, 8, 1, 0.5);
    bad |= grid_case(3, 8, 12, 10, 1.0);
    printf(bad ? "oracle driver: FAILED\n" : "oracle driver: ok\n");
    return bad;
}
