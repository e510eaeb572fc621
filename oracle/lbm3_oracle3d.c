/*
 * lbm3_oracle3d.c -- plain FP64 CPU oracle for the three-dimensional (D3Q19 and D3Q27) form
 * of the ternary colour-gradient step of Yu, Liu, Liang and Zhang (arXiv:1808.08555).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite loads this library.  It shares no code,
 * header or table with the HIP library.  It is compiled together with lbm3_oracle.c, whose
 * segregation law (Eqs. 18-20 and the comparison laws) and local relaxation time
 * (Eqs. 10-11) do not depend on the lattice and are called from here.
 *
 * The paper states its model for DmQn lattices (Sec. 2) and gives the lattice constants
 * for D2Q9.  Readings for three dimensions: the standard D3Q19 lattice (c_s^2 = 1/3,
 * w_0 = 1/3, w = 1/18 on the 6 axis links, 1/36 on the 12 edge links) or the standard D3Q27
 * lattice (c_s^2 = 1/3, w_0 = 8/27, 2/27 on the axis links, 1/54 on the edge links, 1/216
 * on the 8 corner links); Eq. (12), the force of Eq. (7) (stress pair sum, 3 x 3), Guo's
 * term of Eq. (8), the velocity of Eq. (9), the equilibrium of Eq. (3) and the recolouring
 * of Eq. (13) with these constants; streaming as Eq. (22).  Only the paper's forcing (the
 * perturbation operator's B_i are given for D2Q9 only).
 *
 * Conventions: fluids k = 0, 1, 2; q = 19 or 27 links; state f[k][i][z][y][x] (3q planes),
 * x fastest, periodic in x, y and z; the post-streaming distribution, as in the
 * two-dimensional oracle.  Every entry point returns -1 for another q.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* the two-dimensional oracle's problem description and its lattice-independent parts */
typedef struct {
    int32_t nx, ny;
    double rho0[3];
    double sigma[3];
    double tau[3];
    double beta0;
    int32_t beta_law;
    int32_t forcing;
} oracle_problem;
double oracle_beta(const oracle_problem *p, int k, int l, const double *rho);
double oracle_local_tau(const oracle_problem *p, const double *rho);

/* e_0 = 0; axis links 1-6; edge links 7-18 (the D3Q19 lattice ends here); corner links
 * 19-26 (D3Q27); i odd and i + 1 are opposite */
static const int E3[27][3] = {{0, 0, 0},   {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                              {0, 0, 1},   {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                              {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                              {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
                              {1, 1, 1},   {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
                              {1, -1, 1},  {-1, 1, -1}, {-1, 1, 1},  {1, -1, -1}};
static double w3(int q, int i)
{
    if (q == 19) return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
    return i == 0 ? 8.0 / 27.0 : (i <= 6 ? 2.0 / 27.0 : (i <= 18 ? 1.0 / 54.0 : 1.0 / 216.0));
}
static int valid_q(int q) { return q == 19 || q == 27; }

#define GUARD_G 1e-12

static inline int wrap(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

static double sigma_of(const oracle_problem *p, int k, int l)
{
    int a = k < l ? k : l, b = k < l ? l : k;
    if (a == 0 && b == 1) return p->sigma[0];
    if (a == 0 && b == 2) return p->sigma[1];
    return p->sigma[2];
}

int oracle3d_lattice(int32_t q, int32_t *e, double *w)
{
    if (!valid_q(q)) return -1;
    for (int i = 0; i < q; ++i) {
        for (int a = 0; a < 3; ++a) e[3 * i + a] = E3[i][a];
        w[i] = w3(q, i);
    }
    return 0;
}

typedef struct {
    int nx, ny, nz, q;
    size_t N;
} grid;

static size_t idx(const grid *g, int x, int y, int z)
{
    return ((size_t)wrap(z, g->nz) * g->ny + wrap(y, g->ny)) * g->nx + wrap(x, g->nx);
}

/* Eq. (12) in three dimensions: d_a phi = (1/c_s^2) sum_i w_i phi(x + e_i) e_{i a}, taken
 * over the pairs of opposite links as w_i e_{i a} [phi(x + e_i) - phi(x - e_i)]. */
static void gradient3(const grid *g, const double *phi, double *d /* [3][N] */)
{
    for (int z = 0; z < g->nz; ++z)
        for (int y = 0; y < g->ny; ++y)
            for (int x = 0; x < g->nx; ++x) {
                double s[3] = {0.0, 0.0, 0.0};
                for (int i = 1; i < g->q; i += 2) {
                    double fw = phi[idx(g, x + E3[i][0], y + E3[i][1], z + E3[i][2])];
                    double bw = phi[idx(g, x - E3[i][0], y - E3[i][1], z - E3[i][2])];
                    for (int a = 0; a < 3; ++a) s[a] += w3(g->q, i) * E3[i][a] * (fw - bw);
                }
                size_t j = idx(g, x, y, z);
                for (int a = 0; a < 3; ++a) d[a * g->N + j] = 3.0 * s[a];
            }
}

/* Eq. (6) */
static double concentration_factor(const oracle_problem *p, const double *rho_k, int k, int l)
{
    double v = 1e6 * rho_k[k] * rho_k[l] / (p->rho0[k] * p->rho0[l]);
    return v < 1.0 ? v : 1.0;
}

/* G_kl = c_l grad c_k - c_k grad c_l; returns |G| and n (zero at or below the guard) */
static double colour_gradient3(const double *c, const double (*gc)[3], int k, int l, double *G, double *n)
{
    for (int a = 0; a < 3; ++a) G[a] = c[l] * gc[k][a] - c[k] * gc[l][a];
    double m = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
    for (int a = 0; a < 3; ++a) n[a] = m > GUARD_G ? G[a] / m : 0.0;
    return m;
}

/* The fields of a post-streaming state that the step needs: densities rho[3][N], totals
 * ft[q][N] (may be NULL), concentration gradients gc[k][a][N] (Eq. 12), the stress of
 * Eq. (7) summed as printed over ordered pairs, S = sum (sigma C / 2) |G| (I - n n), and
 * the force F_b = sum_a d_a S_ab.  c, S, d are scratch. */
static void field_pass(const oracle_problem *p, const grid *g, const double *f, double *rho, double *ft,
                       double *c, double *gc, double *S, double *F, double *d)
{
    const size_t N = g->N;
    const int Q = g->q;
    for (size_t j = 0; j < N; ++j) {
        if (ft)
            for (int i = 0; i < Q; ++i) ft[i * N + j] = 0.0;
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
            for (int i = 0; i < Q; ++i) {
                double v = f[(size_t)(k * Q + i) * N + j];
                s += v;
                if (ft) ft[i * N + j] += v;
            }
            rho[k * N + j] = s;
        }
    }
    for (int k = 0; k < 3; ++k) {
        for (size_t j = 0; j < N; ++j) c[j] = rho[k * N + j] / (rho[j] + rho[N + j] + rho[2 * N + j]);
        gradient3(g, c, gc + (size_t)3 * k * N);
    }
    for (size_t j = 0; j < N; ++j) {
        double rk[3] = {rho[j], rho[N + j], rho[2 * N + j]};
        double r = rk[0] + rk[1] + rk[2], cc[3] = {rk[0] / r, rk[1] / r, rk[2] / r};
        double gg[3][3];
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a) gg[k][a] = gc[(size_t)(3 * k + a) * N + j];
        double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) {
                if (l == k) continue;
                double G[3], n[3];
                double m = colour_gradient3(cc, gg, k, l, G, n);
                if (!(m > GUARD_G)) continue;
                double a = 0.5 * sigma_of(p, k, l) * concentration_factor(p, rk, k, l) * m;
                for (int u = 0; u < 3; ++u)
                    for (int v = 0; v < 3; ++v) s[3 * u + v] += a * ((u == v ? 1.0 : 0.0) - n[u] * n[v]);
            }
        for (int q = 0; q < 9; ++q) S[q * N + j] = s[q];
    }
    for (size_t q = 0; q < 3 * N; ++q) F[q] = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            gradient3(g, S + (size_t)(3 * a + b) * N, d);
            for (size_t j = 0; j < N; ++j) F[b * N + j] += d[a * N + j];
        }
}

/* One step: collision (Eqs. 1-3, 8-11), recolouring (Eqs. 13, 19-20), streaming (Eq. 22) */
int oracle3d_step(const oracle_problem *p, int32_t nz, int32_t q, const double *f, double *fnew)
{
    if (!valid_q(q)) return -1;
    grid g = {p->nx, p->ny, nz, q, (size_t)p->nx * p->ny * nz};
    const size_t N = g.N;
    const int Q = q;
    double *rho = malloc(sizeof(double) * 3 * N), *ft = malloc(sizeof(double) * Q * N);
    double *c = malloc(sizeof(double) * N), *gc = malloc(sizeof(double) * 9 * N);
    double *S = malloc(sizeof(double) * 9 * N), *F = malloc(sizeof(double) * 3 * N);
    double *d = malloc(sizeof(double) * 3 * N);
    if (!rho || !ft || !c || !gc || !S || !F || !d) {
        free(rho), free(ft), free(c), free(gc), free(S), free(F), free(d);
        return -1;
    }
    field_pass(p, &g, f, rho, ft, c, gc, S, F, d);
    /* collision, recolouring, streaming */
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < g.ny; ++y)
            for (int x = 0; x < g.nx; ++x) {
                size_t j = idx(&g, x, y, z);
                double rk[3] = {rho[j], rho[N + j], rho[2 * N + j]};
                double r = rk[0] + rk[1] + rk[2];
                double m[3] = {0, 0, 0}, Fv[3] = {F[j], F[N + j], F[2 * N + j]};
                for (int i = 0; i < Q; ++i)
                    for (int a = 0; a < 3; ++a) m[a] += ft[i * N + j] * E3[i][a];
                double u[3], uu = 0.0, uF = 0.0;
                for (int a = 0; a < 3; ++a) {
                    u[a] = (m[a] + 0.5 * Fv[a]) / r;
                    uu += u[a] * u[a];
                    uF += u[a] * Fv[a];
                }
                double tau = oracle_local_tau(p, rk);
                double fdag[27];
                for (int i = 0; i < Q; ++i) {
                    double eu = 0.0, eF = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        eu += E3[i][a] * u[a];
                        eF += E3[i][a] * Fv[a];
                    }
                    double feq = w3(Q, i) * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
                    double phi = w3(Q, i) * (1.0 - 1.0 / (2.0 * tau)) * (3.0 * (eF - uF) + 9.0 * eu * eF);
                    double fi = ft[i * N + j];
                    fdag[i] = fi - (fi - feq) / tau + phi;
                }
                double cc[3] = {rk[0] / r, rk[1] / r, rk[2] / r}, gg[3][3];
                for (int k = 0; k < 3; ++k)
                    for (int a = 0; a < 3; ++a) gg[k][a] = gc[(size_t)(3 * k + a) * N + j];
                for (int k = 0; k < 3; ++k) {
                    double out[27];
                    for (int i = 0; i < Q; ++i) out[i] = cc[k] * fdag[i];
                    for (int l = 0; l < 3; ++l) {
                        if (l == k) continue;
                        double G[3], n[3];
                        colour_gradient3(cc, gg, k, l, G, n);
                        double a = oracle_beta(p, k, l, rk) * rk[k] * rk[l] / r;
                        for (int i = 0; i < Q; ++i)
                            out[i] += a * w3(Q, i) * (n[0] * E3[i][0] + n[1] * E3[i][1] + n[2] * E3[i][2]);
                    }
                    for (int i = 0; i < Q; ++i)
                        fnew[(size_t)(k * Q + i) * N + idx(&g, x + E3[i][0], y + E3[i][1], z + E3[i][2])] = out[i];
                }
            }
    free(rho), free(ft), free(c), free(gc), free(S), free(F), free(d);
    return 0;
}

int oracle3d_run(const oracle_problem *p, int32_t nz, int32_t q, double *f, int64_t nsteps)
{
    if (!valid_q(q)) return -1;
    size_t n = (size_t)3 * q * p->nx * p->ny * nz;
    double *tmp = malloc(sizeof(double) * n);
    if (!tmp) return -1;
    for (int64_t s = 0; s < nsteps; ++s) {
        if (oracle3d_step(p, nz, q, f, tmp)) {
            free(tmp);
            return -1;
        }
        memcpy(f, tmp, sizeof(double) * n);
    }
    free(tmp);
    return 0;
}

/* f_{i,k} = w_i rho_k (fluid at rest) */
int oracle3d_init(const oracle_problem *p, int32_t nz, int32_t q, const double *rho, double *f)
{
    if (!valid_q(q)) return -1;
    size_t N = (size_t)p->nx * p->ny * nz;
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < q; ++i)
            for (size_t j = 0; j < N; ++j) f[(size_t)(k * q + i) * N + j] = w3(q, i) * rho[k * N + j];
    return 0;
}

/* masses (3), momentum sum rho u (3), kinetic energy, max |u|, with the velocity of Eq. (9) */
int oracle3d_observables(const oracle_problem *p, int32_t nz, int32_t q, const double *f, double *out)
{
    if (!valid_q(q)) return -1;
    grid g = {p->nx, p->ny, nz, q, (size_t)p->nx * p->ny * nz};
    const size_t N = g.N;
    /* the velocity of Eq. (9) needs the force: the same field pass as the step */
    double *rho = malloc(sizeof(double) * 3 * N), *c = malloc(sizeof(double) * N);
    double *gc = malloc(sizeof(double) * 9 * N), *S = malloc(sizeof(double) * 9 * N);
    double *F = malloc(sizeof(double) * 3 * N), *d = malloc(sizeof(double) * 3 * N);
    int rc = -1;
    if (!rho || !c || !gc || !S || !F || !d) goto done;
    field_pass(p, &g, f, rho, NULL, c, gc, S, F, d);
    for (int q = 0; q < 8; ++q) out[q] = 0.0;
    for (size_t j = 0; j < N; ++j) {
        double r = 0.0, m[3] = {0, 0, 0};
        for (int k = 0; k < 3; ++k) {
            out[k] += rho[k * N + j];
            r += rho[k * N + j];
        }
        for (int k = 0; k < 3; ++k)
            for (int i = 0; i < q; ++i)
                for (int a = 0; a < 3; ++a) m[a] += f[(size_t)(k * q + i) * N + j] * E3[i][a];
        double uu = 0.0;
        for (int a = 0; a < 3; ++a) {
            double ua = (m[a] + 0.5 * F[a * N + j]) / r;
            out[3 + a] += r * ua;
            uu += ua * ua;
        }
        out[6] += 0.5 * r * uu;
        if (sqrt(uu) > out[7]) out[7] = sqrt(uu);
    }
    rc = 0;
done:
    free(rho), free(c), free(gc), free(S), free(F), free(d);
    return rc;
}
