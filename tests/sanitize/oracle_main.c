/* Driver for the sanitizer build of the C oracles (test infrastructure).  Built with gcc
 * -fsanitize=address,undefined by tests/test_sanitize_cpu.py and linked with
 * oracle/lbm3_oracle.c and oracle/lbm3_oracle3d.c.  It runs every entry point on small and
 * degenerate periodic lattices (1x1 up to 13x7, zero and tiny densities), every segregation
 * law and both forcings, so that an out-of-bounds access, a use of freed memory or undefined
 * integer or float behaviour in the oracles aborts the run.  Exit status 0: all calls ran and
 * every result was finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int32_t nx, ny;
    double rho0[3];
    double sigma[3];
    double tau[3];
    double beta0;
    int32_t beta_law;
    int32_t forcing;
} oracle_problem;

void oracle_init(const oracle_problem *p, const double *rho, const double *u, double *f);
int oracle_step(const oracle_problem *p, const double *f, double *fnew);
int oracle_run(const oracle_problem *p, double *f, int64_t nsteps);
int oracle_fields(const oracle_problem *p, const double *f, double *rho, double *u, double *F,
                  double *tau);
int oracle_observables(const oracle_problem *p, const double *f, double *out);
int oracle_step_nodes(const oracle_problem *p, const double *f, int32_t count, const int32_t *xs,
                      const int32_t *ys, double *out);
void oracle_gradient(int32_t nx, int32_t ny, const double *phi, double *dx, double *dy);
void oracle_set_num_threads(int n);
int oracle3d_init(const oracle_problem *p, int32_t nz, int32_t q, const double *rho, double *f);
int oracle3d_run(const oracle_problem *p, int32_t nz, int32_t q, double *f, int64_t nsteps);
int oracle3d_observables(const oracle_problem *p, int32_t nz, int32_t q, const double *f, double *out);

static uint64_t state = 0x9e3779b97f4a7c15ull;
static double uniform(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * 0x1.0p-53;
}

/* densities with zero and tiny entries; one fluid of every node holds at least 0.5 */
static void mixture(double *rho, size_t n)
{
    for (size_t j = 0; j < n; ++j) {
        for (int k = 0; k < 3; ++k) {
            const double r = uniform();
            rho[k * n + j] = r < 0.2 ? 0.0 : (r < 0.3 ? 1e-9 * r : 0.2 * r);
        }
        rho[(j % 3) * n + j] += 0.5 + 0.5 * uniform();
    }
}

static int check(const char *what, const double *v, size_t n)
{
    for (size_t j = 0; j < n; ++j)
        if (!isfinite(v[j])) {
            fprintf(stderr, "%s: value %zu is not finite\n", what, j);
            return 1;
        }
    return 0;
}

int main(void)
{
    static const int shapes[][2] = {{1, 1}, {1, 5}, {3, 2}, {2, 1}, {8, 8}, {13, 7}};
    int bad = 0;
    oracle_set_num_threads(2);
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s)
        for (int law = 0; law < 4; ++law)
            for (int forcing = 0; forcing < 2; ++forcing) {
                oracle_problem p = {shapes[s][0], shapes[s][1], {1.0, 0.9, 1.1}, {0.011, 0.013, 0.017},
                                    {0.7, 1.0, 1.3}, 0.7, law, forcing};
                const size_t n = (size_t)p.nx * p.ny;
                double *rho = malloc(3 * n * sizeof(double)), *u = malloc(2 * n * sizeof(double));
                double *f = malloc(27 * n * sizeof(double)), *g = malloc(27 * n * sizeof(double));
                double *fr = malloc(3 * n * sizeof(double)), *fu = malloc(2 * n * sizeof(double));
                double *fF = malloc(2 * n * sizeof(double)), *ftau = malloc(n * sizeof(double));
                double *dx = malloc(n * sizeof(double));
                double *dy = malloc(n * sizeof(double)), obs[8];
                mixture(rho, n);
                for (size_t j = 0; j < 2 * n; ++j) u[j] = 0.02 * (uniform() - 0.5);
                oracle_init(&p, rho, u, f);
                bad |= oracle_step(&p, f, g) != 0;
                bad |= oracle_run(&p, g, 4) != 0;
                bad |= oracle_fields(&p, g, fr, fu, fF, ftau) != 0;
                bad |= oracle_observables(&p, g, obs) != 0;
                oracle_gradient(p.nx, p.ny, fr, dx, dy);
                int32_t xs[4] = {0, p.nx - 1, p.nx / 2, 0}, ys[4] = {0, p.ny - 1, p.ny / 2, p.ny - 1};
                double out[4 * 27];
                bad |= oracle_step_nodes(&p, g, 4, xs, ys, out) != 0;
                bad |= check("state", g, 27 * n) | check("fields", fu, 2 * n) | check("tau", ftau, n) | check("nodes", out, 4 * 27) |
                       check("gradient", dx, n);
                free(rho), free(u), free(f), free(g), free(fr), free(fu), free(fF), free(ftau), free(dx),
                    free(dy);
            }
    static const int shapes3[][3] = {{1, 2, 3}, {2, 1, 1}, {4, 3, 5}};
    for (int q = 19; q <= 27; q += 8)
    for (size_t s = 0; s < sizeof shapes3 / sizeof shapes3[0]; ++s)
        for (int law = 0; law < 4; ++law) {
            oracle_problem p = {shapes3[s][0], shapes3[s][1], {1.0, 1.0, 1.0}, {0.011, 0.013, 0.017},
                                {0.7, 1.0, 1.3}, 0.7, law, 0};
            const int nz = shapes3[s][2];
            const size_t n = (size_t)p.nx * p.ny * nz;
            double *rho = malloc(3 * n * sizeof(double)), *f = malloc(3 * q * n * sizeof(double)), obs[8];
            mixture(rho, n);
            bad |= oracle3d_init(&p, nz, q, rho, f) != 0;
            bad |= oracle3d_run(&p, nz, q, f, 4) != 0;
            bad |= oracle3d_observables(&p, nz, q, f, obs) != 0;
            bad |= check("state3d", f, 3 * q * n);
            free(rho), free(f);
        }
    printf(bad ? "FAILED\n" : "ok\n");
    return bad;
}
