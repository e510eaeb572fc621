/*
 * lbm3_oracle.c -- plain FP64 CPU oracle for one time step of the ternary
 * colour-gradient lattice Boltzmann model of Yu, Liu, Liang and Zhang,
 * "A versatile lattice Boltzmann model for immiscible ternary fluid flows"
 * (arXiv:1808.08555).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or helper with the HIP library; it is written to be read
 * side by side with Sec. 2 of the paper, not to be fast.
 *
 * Conventions
 *   fluids k = 0, 1, 2 are the paper's red, green, blue (fluid 1, 2, 3);
 *   sigma[0] = sigma_rg (12), sigma[1] = sigma_rb (13), sigma[2] = sigma_gb (23);
 *   every field is stored [component][y][x] with x fastest, periodic in x and y;
 *   the state is the post-streaming distribution f[k][i][y][x] (27 planes).
 *
 * Where the paper leaves a choice open, the choice taken here is stated at the
 * point of use (marked "reading").  Equation numbers follow the order of the
 * numbered displays in the paper: (1) collision, (2) BGK, (3) equilibrium,
 * (4)-(5) perturbation operator, (6) concentration factor, (7) interfacial
 * force, (8) Guo forcing, (9) velocity, (10) viscosity mean, (11) relaxation
 * time, (12) isotropic difference, (13) recolouring, (14) Neumann angle,
 * (15)-(17) earlier segregation laws, (18)-(20) proposed segregation law,
 * (22) streaming.
 *
 * The printed constants that no closed form fixes (the 35 of C_t in Eq. (19),
 * the 10^6 of C_kl in Eq. (6), the comparison laws and the perturbation
 * operator) are pinned by node-level checks where C_t and C_kl are below
 * saturation and by agreement, to round-off, with a second transcription of
 * the step written apart from this one (numpy_step.py).  Parity unpinned:
 * exact steady-state fields and spurious-velocity values, which the paper does
 * not print in a form a step-level oracle can reproduce.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* D2Q9 lattice (Sec. 2, text after Eq. 3): e_0 = 0, e_{1,3} = (+-1, 0),     */
/* e_{2,4} = (0, +-1), e_{5,7} = (+-1, +-1), e_{6,8} = (-+1, +-1);           */
/* w_0 = 4/9, w_{1-4} = 1/9, w_{5-8} = 1/36; c = 1, c_s^2 = 1/3.              */
/* ------------------------------------------------------------------------ */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* 1/c_s^2 = 3, 1/(2 c_s^4) = 9/2, 1/(2 c_s^2) = 3/2, 1/c_s^4 = 9 */
#define INV_CS2 3.0
#define INV_2CS4 4.5
#define INV_2CS2 1.5
#define INV_CS4 9.0

/* Threshold below which |G_kl| is treated as zero, so that n_kl = G/|G| is
 * never formed from round-off (reading: the paper does not define n_kl where
 * the colour gradient vanishes; n_kl = 0 and the stress term is 0 there). */
#define GUARD_G 1e-12

#define ORACLE_PI 3.14159265358979323846

typedef struct {
    int32_t nx, ny;
    double rho0[3];  /* pure-fluid densities rho_k^0, Eq. (6) */
    double sigma[3]; /* sigma_rg, sigma_rb, sigma_gb */
    double tau[3];   /* per-fluid relaxation times tau_k */
    double beta0;    /* reference segregation parameter beta^0 */
    int32_t beta_law; /* 0 proposed law, Eqs. (18)-(20); 1 Spencer, Eq. (15);
                         2 Leclaire, Eq. (16); 3 constant beta, Eq. (17) */
    int32_t forcing;  /* 0 the force of Eq. (7) with Guo's term, Eqs. (8)-(9);
                         1 the perturbation operator of Eqs. (4)-(5) */
} oracle_problem;

void oracle_lattice(int32_t *ex, int32_t *ey, double *w)
{
    for (int i = 0; i < 9; ++i) {
        ex[i] = EX[i];
        ey[i] = EY[i];
        w[i] = W[i];
    }
}

static inline int wrap(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

/* sigma_kl for k != l (symmetric) */
static double sigma_of(const oracle_problem *p, int k, int l)
{
    int a = k < l ? k : l, b = k < l ? l : k;
    if (a == 0 && b == 1) return p->sigma[0];
    if (a == 0 && b == 2) return p->sigma[1];
    return p->sigma[2];
}

/* ------------------------------------------------------------------------ */
/* Proposed segregation law, Sec. 2, Eqs. (18)-(20).                         */
/* ------------------------------------------------------------------------ */

/* X_kl of Eq. (18); m is the third fluid (reading: the law-of-cosines cosine
 * of the Neumann-triangle angle opposite sigma_kl, as in Eq. (14)). */
double oracle_X(const oracle_problem *p, int k, int l)
{
    int m = 3 - k - l;
    double smk = sigma_of(p, m, k), sml = sigma_of(p, m, l), skl = sigma_of(p, k, l);
    return (smk * smk + sml * sml - skl * skl) / (2.0 * smk * sml);
}

/* g(X) of Eq. (20).  Reading: where |X| is within 1e-12 of 1 it is taken as
 * exactly +-1 (the branch value there is -1 for X -> 1 and +1 for X -> -1);
 * elsewhere the printed branches are used literally. */
double oracle_g(double X)
{
    if (X >= 1.0 - 1e-12) return -1.0;
    if (X <= -1.0 + 1e-12) return 1.0;
    if (X < 0.0) return 1.0 - sin(acos(X));
    return sin(acos(X)) - 1.0;
}

/* ------------------------------------------------------------------------ */
/* Earlier segregation laws the paper compares against, Eqs. (15)-(17).      */
/* ------------------------------------------------------------------------ */

/* phi_kl of Eq. (14): the Neumann-triangle angle opposite sigma_kl.  Reading:
 * where no triangle exists the cosine is clamped to [-1, 1]. */
static double neumann_phi(const oracle_problem *p, int k, int l)
{
    double c = oracle_X(p, k, l);
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    return acos(c);
}

/* Reading: the Neumann triangle exists when every cosine of Eq. (14) is below 1
 * in magnitude by more than 1e-12 (the tolerance of g(X) above), so that the
 * critical states (a degenerate triangle) count as having none. */
static int neumann_triangle_exists(const oracle_problem *p)
{
    return fabs(oracle_X(p, 0, 1)) < 1.0 - 1e-12 && fabs(oracle_X(p, 0, 2)) < 1.0 - 1e-12 &&
           fabs(oracle_X(p, 1, 2)) < 1.0 - 1e-12;
}

/* Eq. (15), as printed: beta_rg = beta0, beta_rb takes sin(phi_gb) and beta_gb
 * takes sin(phi_rb), with the factor 27 rho_r rho_g rho_b / rho^3. */
static double beta_spencer(const oracle_problem *p, int k, int l, const double *rho)
{
    double r = rho[0] + rho[1] + rho[2];
    double s = 27.0 * rho[0] * rho[1] * rho[2] / (r * r * r);
    if (k == 0 && l == 1) return p->beta0;
    if (k == 0 && l == 2) return p->beta0 * (1.0 + s * (sin(neumann_phi(p, 1, 2)) - 1.0));
    return p->beta0 * (1.0 + s * (sin(neumann_phi(p, 0, 2)) - 1.0));
}

/* Eq. (16): beta0 for the pair with the largest phi (reading: the first of
 * equal maxima in the order rg, rb, gb), beta0 + beta0 C_t [sin(pi - phi_max -
 * phi_kl) - 1] for the others; beta0 everywhere without a Neumann triangle. */
static double beta_leclaire(const oracle_problem *p, int k, int l, const double *rho)
{
    if (!neumann_triangle_exists(p)) return p->beta0;
    const int pk[3] = {0, 0, 1}, pl[3] = {1, 2, 2};
    int kmax = 0, lmax = 1;
    double phimax = neumann_phi(p, 0, 1);
    for (int q = 1; q < 3; ++q) {
        double ph = neumann_phi(p, pk[q], pl[q]);
        if (ph > phimax) {
            phimax = ph;
            kmax = pk[q];
            lmax = pl[q];
        }
    }
    if (k == kmax && l == lmax) return p->beta0;
    double r = rho[0] + rho[1] + rho[2];
    double ct = 35.0 * rho[0] * rho[1] * rho[2] / (r * r * r);
    if (ct > 1.0) ct = 1.0;
    return p->beta0 + p->beta0 * ct * (sin(ORACLE_PI - phimax - neumann_phi(p, k, l)) - 1.0);
}

/* beta_kl = beta_lk at a node with densities rho[3]: Eq. (19) for the proposed
 * law, else the comparison law selected by p->beta_law. */
double oracle_beta(const oracle_problem *p, int k, int l, const double *rho)
{
    if (k > l) {
        int t = k;
        k = l;
        l = t;
    }
    if (p->beta_law == 1) return beta_spencer(p, k, l, rho);
    if (p->beta_law == 2) return beta_leclaire(p, k, l, rho);
    if (p->beta_law == 3) return p->beta0; /* Eq. (17) */
    double r = rho[0] + rho[1] + rho[2];
    double ct = 35.0 * rho[0] * rho[1] * rho[2] / (r * r * r);
    if (ct > 1.0) ct = 1.0;
    return p->beta0 + p->beta0 * ct * oracle_g(oracle_X(p, k, l));
}

/* ------------------------------------------------------------------------ */
/* Node-local pieces of the step.                                            */
/* ------------------------------------------------------------------------ */

/* Equilibrium, Eq. (3). */
void oracle_feq(double rho, double ux, double uy, double *feq)
{
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        double eu = EX[i] * ux + EY[i] * uy;
        feq[i] = W[i] * rho * (1.0 + eu * INV_CS2 + eu * eu * INV_2CS4 - uu * INV_2CS2);
    }
}

/* Guo forcing term, Eq. (8), with delta_t = 1. */
void oracle_guo(double tau, double ux, double uy, double Fx, double Fy, double *phi)
{
    for (int i = 0; i < 9; ++i) {
        double eu = EX[i] * ux + EY[i] * uy;
        double ax = (EX[i] - ux) * INV_CS2 + eu * INV_CS4 * EX[i];
        double ay = (EY[i] - uy) * INV_CS2 + eu * INV_CS4 * EY[i];
        phi[i] = W[i] * (1.0 - 1.0 / (2.0 * tau)) * (ax * Fx + ay * Fy);
    }
}

/* Local relaxation time from the harmonic viscosity mean, Eqs. (10)-(11):
 * rho/nu = sum_k rho_k/nu_k, nu_k = (tau_k - 1/2) c_s^2, tau = nu/c_s^2 + 1/2. */
double oracle_local_tau(const oracle_problem *p, const double *rho)
{
    double r = rho[0] + rho[1] + rho[2];
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        double nu_k = (p->tau[k] - 0.5) / INV_CS2;
        s += rho[k] / nu_k;
    }
    double nu = r / s;
    return nu * INV_CS2 + 0.5;
}

/* Collision of the total distribution at one node, Eqs. (1), (2), (3), (8),
 * (9): f_dag_i = f_i - (f_i - f_eq_i)/tau + Phi_i, with the velocity of Eq. (9)
 * rho u = sum_i f_i e_i + F/2.  Returns u in u_out (may be NULL). */
void oracle_collide_node(const oracle_problem *p, const double *rho_k, const double *f,
                         double Fx, double Fy, double *fdag, double *u_out)
{
    double rho = rho_k[0] + rho_k[1] + rho_k[2];
    double mx = 0.0, my = 0.0;
    for (int i = 0; i < 9; ++i) {
        mx += f[i] * EX[i];
        my += f[i] * EY[i];
    }
    double ux = (mx + 0.5 * Fx) / rho;
    double uy = (my + 0.5 * Fy) / rho;
    double tau = oracle_local_tau(p, rho_k);
    double feq[9], phi[9];
    oracle_feq(rho, ux, uy, feq);
    oracle_guo(tau, ux, uy, Fx, Fy, phi);
    for (int i = 0; i < 9; ++i) {
        double omega = -(f[i] - feq[i]) / tau;
        fdag[i] = f[i] + omega + phi[i];
    }
    if (u_out) {
        u_out[0] = ux;
        u_out[1] = uy;
    }
}

/* Colour gradient G_kl = c_l grad c_k - c_k grad c_l (Sec. 2, after Eq. 5),
 * c_k = rho_k/rho; returns |G_kl| and writes n_kl (zero below GUARD_G). */
static double colour_gradient(const double *c, const double *gx, const double *gy, int k, int l,
                              double *G, double *n)
{
    G[0] = c[l] * gx[k] - c[k] * gx[l];
    G[1] = c[l] * gy[k] - c[k] * gy[l];
    double mag = sqrt(G[0] * G[0] + G[1] * G[1]);
    if (mag > GUARD_G) {
        n[0] = G[0] / mag;
        n[1] = G[1] / mag;
    } else {
        n[0] = 0.0;
        n[1] = 0.0;
    }
    return mag;
}

/* Generalized recolouring at one node, Eq. (13):
 * f_ddag_{i,k} = (rho_k/rho) f_dag_i + sum_{l != k} beta_kl w_i (rho_k rho_l / rho) n_kl . e_i.
 * c, gx, gy: concentrations c_k and their gradients at the node.
 * out[k*9 + i]. */
void oracle_recolour_node(const oracle_problem *p, const double *rho_k, const double *gx,
                          const double *gy, const double *fdag, double *out)
{
    double rho = rho_k[0] + rho_k[1] + rho_k[2];
    double c[3] = {rho_k[0] / rho, rho_k[1] / rho, rho_k[2] / rho};
    for (int k = 0; k < 3; ++k) {
        for (int i = 0; i < 9; ++i) out[k * 9 + i] = c[k] * fdag[i];
        for (int l = 0; l < 3; ++l) {
            if (l == k) continue;
            double G[2], n[2];
            colour_gradient(c, gx, gy, k, l, G, n);
            double beta = oracle_beta(p, k, l, rho_k);
            double a = beta * rho_k[k] * rho_k[l] / rho;
            for (int i = 0; i < 9; ++i) out[k * 9 + i] += a * W[i] * (n[0] * EX[i] + n[1] * EY[i]);
        }
    }
}

/* Concentration factor, Eq. (6). */
static double concentration_factor(const oracle_problem *p, const double *rho_k, int k, int l)
{
    double v = 1e6 * rho_k[k] * rho_k[l] / (p->rho0[k] * p->rho0[l]);
    return v < 1.0 ? v : 1.0;
}

/* Interfacial stress at one node, the bracket of Eq. (7) summed as printed:
 * S = sum_k sum_{l != k} (sigma_kl C_kl / 2) |G_kl| (I - n_kl n_kl).
 * S[0] = S_xx, S[1] = S_xy, S[2] = S_yx, S[3] = S_yy. */
void oracle_stress_node(const oracle_problem *p, const double *rho_k, const double *gx,
                        const double *gy, double *S)
{
    double rho = rho_k[0] + rho_k[1] + rho_k[2];
    double c[3] = {rho_k[0] / rho, rho_k[1] / rho, rho_k[2] / rho};
    S[0] = S[1] = S[2] = S[3] = 0.0;
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
            if (l == k) continue;
            double G[2], n[2];
            double mag = colour_gradient(c, gx, gy, k, l, G, n);
            if (!(mag > GUARD_G)) continue;
            double a = 0.5 * sigma_of(p, k, l) * concentration_factor(p, rho_k, k, l) * mag;
            S[0] += a * (1.0 - n[0] * n[0]);
            S[1] += a * (0.0 - n[0] * n[1]);
            S[2] += a * (0.0 - n[1] * n[0]);
            S[3] += a * (1.0 - n[1] * n[1]);
        }
}

/* Perturbation operator of Eqs. (4)-(5), the comparison forcing: at one node
 * Phi_i = sum_k sum_{l != k} (A_kl C_kl / 2) |G_kl| [w_i (e_i . G_kl)^2 / |G_kl|^2 - B_i]
 * with B_0 = -4/27, B_1-4 = 2/27, B_5-8 = 5/108 (the values the paper quotes).
 * Reading: A_kl = A_lk = 9 sigma_kl / (2 tau), from sigma_kl = (A_kl + A_lk) tau / 9,
 * with tau the node's relaxation time of Eqs. (10)-(11); pairs with |G_kl| at or below
 * the guard add nothing (the term vanishes with |G_kl| anyway). */
void oracle_perturbation_node(const oracle_problem *p, const double *rho_k, const double *gx,
                              const double *gy, double *phi)
{
    static const double B[9] = {-4.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0,
                                5.0 / 108.0, 5.0 / 108.0, 5.0 / 108.0, 5.0 / 108.0};
    double rho = rho_k[0] + rho_k[1] + rho_k[2];
    double c[3] = {rho_k[0] / rho, rho_k[1] / rho, rho_k[2] / rho};
    double tau = oracle_local_tau(p, rho_k);
    for (int i = 0; i < 9; ++i) phi[i] = 0.0;
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
            if (l == k) continue;
            double G[2], n[2];
            double mag = colour_gradient(c, gx, gy, k, l, G, n);
            if (!(mag > GUARD_G)) continue;
            double A = 9.0 * sigma_of(p, k, l) / (2.0 * tau);
            double a = 0.5 * A * concentration_factor(p, rho_k, k, l) * mag;
            for (int i = 0; i < 9; ++i) {
                double eG = EX[i] * G[0] + EY[i] * G[1];
                phi[i] += a * (W[i] * eG * eG / (mag * mag) - B[i]);
            }
        }
}

/* ------------------------------------------------------------------------ */
/* Grid-wide pieces.                                                         */
/* ------------------------------------------------------------------------ */

/* Isotropic difference, Eq. (12): d_alpha phi(x) = (1/c_s^2) sum_i w_i phi(x + e_i) e_{i alpha},
 * periodic in x and y.  Reading: the sum is taken over the four pairs of opposite
 * directions (i, -i), i = 1, 2, 5, 6, as w_i e_{i alpha} [phi(x + e_i) - phi(x - e_i)]
 * (algebraically the same sum, since w_{-i} = w_i and e_{-i} = -e_i); data that are
 * mirror-symmetric about x then give an exactly zero derivative. */
void oracle_gradient(int32_t nx, int32_t ny, const double *phi, double *dx, double *dy)
{
    static const int PAIR_DIR[4] = {1, 2, 5, 6};
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double sx = 0.0, sy = 0.0;
            for (int q = 0; q < 4; ++q) {
                int i = PAIR_DIR[q];
                double fwd = phi[(size_t)wrap(y + EY[i], ny) * nx + wrap(x + EX[i], nx)];
                double bwd = phi[(size_t)wrap(y - EY[i], ny) * nx + wrap(x - EX[i], nx)];
                sx += W[i] * EX[i] * (fwd - bwd);
                sy += W[i] * EY[i] * (fwd - bwd);
            }
            dx[(size_t)y * nx + x] = INV_CS2 * sx;
            dy[(size_t)y * nx + x] = INV_CS2 * sy;
        }
}

/* Macroscopic fields of a post-streaming state: rho_k = sum_i f_{i,k} (text
 * after Eq. 22), the gradients of c_k, and the interfacial force of Eq. (7)
 * whose divergence is taken with the difference of Eq. (12):
 * F_beta = d_x S_{x beta} + d_y S_{y beta}. */
typedef struct {
    double *rho;  /* [3][N] */
    double *ftot; /* [9][N] */
    double *gx;   /* [3][N] */
    double *gy;   /* [3][N] */
    double *S;    /* [4][N] */
    double *F;    /* [2][N] */
    double *tmp;  /* [2][N] */
} fields;

static int fields_alloc(fields *w, size_t N)
{
    w->rho = malloc(sizeof(double) * 3 * N);
    w->ftot = malloc(sizeof(double) * 9 * N);
    w->gx = malloc(sizeof(double) * 3 * N);
    w->gy = malloc(sizeof(double) * 3 * N);
    w->S = malloc(sizeof(double) * 4 * N);
    w->F = malloc(sizeof(double) * 2 * N);
    w->tmp = malloc(sizeof(double) * 2 * N);
    return w->rho && w->ftot && w->gx && w->gy && w->S && w->F && w->tmp;
}

static void fields_free(fields *w)
{
    free(w->rho);
    free(w->ftot);
    free(w->gx);
    free(w->gy);
    free(w->S);
    free(w->F);
    free(w->tmp);
}

static void compute_fields(const oracle_problem *p, const double *f, fields *w)
{
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t j = (size_t)y * nx + x;
            for (int i = 0; i < 9; ++i) w->ftot[i * N + j] = 0.0;
            for (int k = 0; k < 3; ++k) {
                double s = 0.0;
                for (int i = 0; i < 9; ++i) {
                    double v = f[(size_t)(k * 9 + i) * N + j];
                    s += v;
                    w->ftot[i * N + j] += v;
                }
                w->rho[k * N + j] = s;
            }
        }
    /* c_k and its gradient */
    double *c = malloc(sizeof(double) * N);
    for (int k = 0; k < 3; ++k) {
        for (size_t j = 0; j < N; ++j)
            c[j] = w->rho[k * N + j] / (w->rho[j] + w->rho[N + j] + w->rho[2 * N + j]);
        oracle_gradient(nx, ny, c, w->gx + k * N, w->gy + k * N);
    }
    free(c);
    /* stress at every node */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t j = (size_t)y * nx + x;
            double rk[3] = {w->rho[j], w->rho[N + j], w->rho[2 * N + j]};
            double gx[3] = {w->gx[j], w->gx[N + j], w->gx[2 * N + j]};
            double gy[3] = {w->gy[j], w->gy[N + j], w->gy[2 * N + j]};
            double S[4];
            oracle_stress_node(p, rk, gx, gy, S);
            for (int a = 0; a < 4; ++a) w->S[a * N + j] = S[a];
        }
    /* F_x = d_x S_xx + d_y S_yx ; F_y = d_x S_xy + d_y S_yy */
    double *dx = w->tmp, *dy = w->tmp + N;
    oracle_gradient(nx, ny, w->S + 0 * N, dx, dy); /* S_xx */
    for (size_t j = 0; j < N; ++j) w->F[j] = dx[j];
    oracle_gradient(nx, ny, w->S + 2 * N, dx, dy); /* S_yx */
    for (size_t j = 0; j < N; ++j) w->F[j] += dy[j];
    oracle_gradient(nx, ny, w->S + 1 * N, dx, dy); /* S_xy */
    for (size_t j = 0; j < N; ++j) w->F[N + j] = dx[j];
    oracle_gradient(nx, ny, w->S + 3 * N, dx, dy); /* S_yy */
    for (size_t j = 0; j < N; ++j) w->F[N + j] += dy[j];
    /* with the perturbation operator no body force acts: u = sum_i f_i e_i / rho and no
       Guo term */
    if (p->forcing == 1)
        for (size_t j = 0; j < 2 * N; ++j) w->F[j] = 0.0;
}

/* One full time step: collision (Eqs. 1-3, 8-11, or Eqs. 1-5 with the
 * perturbation operator), recolouring (Eqs. 13, 19, 20) and streaming (Eq. 22),
 * from the post-streaming state f to fnew. */
int oracle_step(const oracle_problem *p, const double *f, double *fnew)
{
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    fields w;
    if (!fields_alloc(&w, N)) {
        fields_free(&w);
        return -1;
    }
    compute_fields(p, f, &w);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t j = (size_t)y * nx + x;
            double rk[3] = {w.rho[j], w.rho[N + j], w.rho[2 * N + j]};
            double gx[3] = {w.gx[j], w.gx[N + j], w.gx[2 * N + j]};
            double gy[3] = {w.gy[j], w.gy[N + j], w.gy[2 * N + j]};
            double fi[9], fdag[9], fdd[27];
            for (int i = 0; i < 9; ++i) fi[i] = w.ftot[i * N + j];
            oracle_collide_node(p, rk, fi, w.F[j], w.F[N + j], fdag, NULL);
            if (p->forcing == 1) { /* Eq. (1) with the operator of Eqs. (4)-(5) */
                double phi[9];
                oracle_perturbation_node(p, rk, gx, gy, phi);
                for (int i = 0; i < 9; ++i) fdag[i] += phi[i];
            }
            oracle_recolour_node(p, rk, gx, gy, fdag, fdd);
            /* streaming, Eq. (22): f_{i,k}(x + e_i, t + 1) = f_ddag_{i,k}(x, t) */
            for (int k = 0; k < 3; ++k)
                for (int i = 0; i < 9; ++i) {
                    size_t d = (size_t)wrap(y + EY[i], ny) * nx + wrap(x + EX[i], nx);
                    fnew[(size_t)(k * 9 + i) * N + d] = fdd[k * 9 + i];
                }
        }
    fields_free(&w);
    return 0;
}

/* nsteps steps in place. */
int oracle_run(const oracle_problem *p, double *f, int64_t nsteps)
{
    const size_t M = (size_t)27 * p->nx * p->ny;
    double *g = malloc(sizeof(double) * M);
    if (!g) return -1;
    for (int64_t t = 0; t < nsteps; ++t) {
        if (oracle_step(p, f, g)) {
            free(g);
            return -1;
        }
        memcpy(f, g, sizeof(double) * M);
    }
    free(g);
    return 0;
}

/* Initial populations.  Reading: the paper does not print them; with u = 0
 * the rest equilibrium is split by colour, f_{i,k} = w_i rho_k; with a given
 * velocity, f_{i,k} = (rho_k/rho) f_eq_i(rho, u) of Eq. (3). */
void oracle_init(const oracle_problem *p, const double *rho, const double *u, double *f)
{
    const size_t N = (size_t)p->nx * p->ny;
    for (size_t j = 0; j < N; ++j) {
        double r = rho[j] + rho[N + j] + rho[2 * N + j];
        double feq[9];
        if (u) oracle_feq(r, u[j], u[N + j], feq);
        for (int k = 0; k < 3; ++k)
            for (int i = 0; i < 9; ++i)
                f[(size_t)(k * 9 + i) * N + j] =
                    u ? (rho[k * N + j] / r) * feq[i] : W[i] * rho[k * N + j];
    }
}

/* Macroscopic output of a state: rho_k, the velocity of Eq. (9), the force of
 * Eq. (7) and the local tau of Eq. (11).  Any output pointer may be NULL. */
int oracle_fields(const oracle_problem *p, const double *f, double *rho, double *u, double *F,
                  double *tau)
{
    const size_t N = (size_t)p->nx * p->ny;
    fields w;
    if (!fields_alloc(&w, N)) {
        fields_free(&w);
        return -1;
    }
    compute_fields(p, f, &w);
    for (size_t j = 0; j < N; ++j) {
        double rk[3] = {w.rho[j], w.rho[N + j], w.rho[2 * N + j]};
        double r = rk[0] + rk[1] + rk[2];
        double mx = 0.0, my = 0.0;
        for (int i = 0; i < 9; ++i) {
            mx += w.ftot[i * N + j] * EX[i];
            my += w.ftot[i * N + j] * EY[i];
        }
        if (rho)
            for (int k = 0; k < 3; ++k) rho[k * N + j] = rk[k];
        if (u) {
            u[j] = (mx + 0.5 * w.F[j]) / r;
            u[N + j] = (my + 0.5 * w.F[N + j]) / r;
        }
        if (F) {
            F[j] = w.F[j];
            F[N + j] = w.F[N + j];
        }
        if (tau) tau[j] = oracle_local_tau(p, rk);
    }
    fields_free(&w);
    return 0;
}

/* Observables: per-fluid mass, total momentum sum(rho u), kinetic energy
 * sum(rho |u|^2 / 2) and max |u| (the quantity of Table 2).  Sums are
 * compensated (Kahan) in node order.  out = {M1, M2, M3, Px, Py, KE, umax}. */
static void kahan_add(double *s, double *c, double v)
{
    double y = v - *c;
    double t = *s + y;
    *c = (t - *s) - y;
    *s = t;
}

int oracle_observables(const oracle_problem *p, const double *f, double *out)
{
    const size_t N = (size_t)p->nx * p->ny;
    double *rho = malloc(sizeof(double) * 3 * N), *u = malloc(sizeof(double) * 2 * N);
    if (!rho || !u || oracle_fields(p, f, rho, u, NULL, NULL)) {
        free(rho);
        free(u);
        return -1;
    }
    double s[6] = {0}, c[6] = {0}, umax = 0.0;
    for (size_t j = 0; j < N; ++j) {
        double r = rho[j] + rho[N + j] + rho[2 * N + j];
        for (int k = 0; k < 3; ++k) kahan_add(&s[k], &c[k], rho[k * N + j]);
        kahan_add(&s[3], &c[3], r * u[j]);
        kahan_add(&s[4], &c[4], r * u[N + j]);
        double uu = u[j] * u[j] + u[N + j] * u[N + j];
        kahan_add(&s[5], &c[5], 0.5 * r * uu);
        double um = sqrt(uu);
        if (um > umax || um != um) umax = um;
    }
    for (int a = 0; a < 6; ++a) out[a] = s[a];
    out[6] = umax;
    free(rho);
    free(u);
    return 0;
}

/* One step evaluated only at selected nodes: out[q*27 + k*9 + i] is the
 * post-streaming f_{i,k}(x_q, y_q) after one step of the state f.  The value
 * at a node depends on the state within three nodes of it (streaming reaches
 * one node, the force divergence one more, the colour gradient one more and
 * the densities are local), so the full step is taken on the periodic 7x7
 * window centred on the node and the centre is read back. */
int oracle_step_nodes(const oracle_problem *p, const double *f, int32_t count,
                      const int32_t *xs, const int32_t *ys, double *out)
{
    const size_t N = (size_t)p->nx * p->ny;
    const int R = 3, Wd = 2 * R + 1;
    oracle_problem q = *p;
    q.nx = Wd;
    q.ny = Wd;
    double *win = malloc(sizeof(double) * 27 * Wd * Wd);
    double *nxt = malloc(sizeof(double) * 27 * Wd * Wd);
    if (!win || !nxt) {
        free(win);
        free(nxt);
        return -1;
    }
    for (int32_t s = 0; s < count; ++s) {
        for (int a = 0; a < 27; ++a)
            for (int wy = 0; wy < Wd; ++wy)
                for (int wx = 0; wx < Wd; ++wx) {
                    size_t src = (size_t)wrap(ys[s] + wy - R, p->ny) * p->nx +
                                 wrap(xs[s] + wx - R, p->nx);
                    win[((size_t)a * Wd + wy) * Wd + wx] = f[(size_t)a * N + src];
                }
        if (oracle_step(&q, win, nxt)) {
            free(win);
            free(nxt);
            return -1;
        }
        for (int a = 0; a < 27; ++a) out[(size_t)s * 27 + a] = nxt[((size_t)a * Wd + R) * Wd + R];
    }
    free(win);
    free(nxt);
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the OpenMP loops from now on (for the single-thread baseline). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
