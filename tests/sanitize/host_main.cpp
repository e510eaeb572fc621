// Driver for the sanitizer build of the library's host code (test infrastructure).  Built by
// tests/test_sanitize_cpu.py: the library's sources compiled with hipcc and a host-only
// address and undefined-behaviour sanitizer, linked with this file.  Nothing here touches a
// GPU: it runs the host-side parts (parameter validation and the derived constants of
// Eqs. 6, 10-11 and 18-20, density checks, tile plans with their XCD ordering and row
// choice, the adjoint's slot rule) over ranges of valid, degenerate and invalid inputs, so
// that an out-of-bounds access or undefined behaviour in them aborts the run.
#include <cmath>
#include <cstdio>
#include <vector>

#include "lbm3_handle.h"

using namespace tcg;

static lbm3_params params(int nx, int ny, int law, int forcing, int precision)
{
    lbm3_params p{};
    p.nx = nx;
    p.ny = ny;
    p.rho0[0] = p.rho0[1] = p.rho0[2] = 1.0;
    p.sigma[0] = 0.01;
    p.sigma[1] = 0.03;  // the critical state, |X| = 1
    p.sigma[2] = 0.02;
    p.tau[0] = 0.7;
    p.tau[1] = 1.0;
    p.tau[2] = 1.3;
    p.beta0 = 0.7;
    p.beta_law = law;
    p.forcing = forcing;
    p.precision = precision;
    return p;
}

int main()
{
    int bad = 0;
    // validation and derived constants, valid and invalid parameters
    for (int law = -1; law <= 4; ++law)
        for (int forcing = -1; forcing <= 2; ++forcing)
            for (int prec = -1; prec <= 3; ++prec)
                for (int nx : {0, 1, 7, 65535, 65536})
                    for (int ny : {-1, 1, 5}) {
                        lbm3_params p = params(nx, ny, law, forcing, prec);
                        double X[3], g[3], nu[3];
                        const int rc = lbm3_derived(&p, X, g, nu);
                        if (rc == LBM3_OK) {
                            KParams kp{};
                            derive(&p, &kp, X, g, nu);
                            for (int q = 0; q < 3; ++q) bad |= !std::isfinite(X[q]) || !std::isfinite(nu[q]);
                        }
                    }
    for (double s : {0.0, -1.0, (double)NAN, (double)INFINITY, 1e-300, 1e300}) {
        lbm3_params p = params(8, 8, 0, 0, 0);
        p.sigma[1] = s;
        (void)validate_params(&p);
        p = params(8, 8, 0, 0, 0);
        p.tau[2] = s;
        (void)validate_params(&p);
        p = params(8, 8, 0, 0, 0);
        p.beta0 = s;
        (void)validate_params(&p);
    }
    (void)validate_params(nullptr);
    // density checks
    std::vector<double> rho(3 * 6, 1.0), u(2 * 6, 0.0);
    bad |= check_rho_fields(rho.data(), u.data(), 6) != LBM3_OK;
    rho[7] = -1.0;
    bad |= check_rho_fields(rho.data(), u.data(), 6) == LBM3_OK;
    rho[7] = NAN;
    bad |= check_rho_fields(rho.data(), nullptr, 6) == LBM3_OK;
    // tile plans: every node of the lattice in exactly one tile, widths within the workgroup
    for (int nx : {1, 2, 5, 63, 64, 65, 250, 256, 300, 1024, 4096, 65535})
        for (int ny : {1, 3, 17, 1000})
            for (int threads : {64, 128, 256, 512})
                for (int halo : {3, 6})
                    for (int eb : {4, 8}) {
                        if (threads - 2 * halo < 1 || (halo == 6 && threads > 256)) continue;
                        const int rows = auto_rows(nx, ny, threads, 256 * (halo == 6 ? 1 : 2), eb, halo);
                        std::vector<Tile> L;
                        plan_lattice(3, nx, ny, threads, rows, eb, L, halo);
                        std::vector<unsigned char> hit((size_t)nx * ny, 0);
                        for (const Tile& t : L) {
                            bad |= t.inst != 3 || t.cols < 1 || t.cols > threads - 2 * halo || t.rows < 1;
                            for (int y = t.y0; y < t.y0 + t.rows; ++y)
                                for (int x = t.x0; x < t.x0 + t.cols; ++x) ++hit[(size_t)(y % ny) * nx + x % nx];
                        }
                        for (unsigned char h : hit) bad |= h != 1;
                        std::vector<Tile> P = xcd_order(L, 8);
                        bad |= P.size() != L.size();
                        int tp = 0, tr = 0;
                        default_tile(KParams{}, Prec::F64, &tp, &tr);
                    }
    // block plans (the step's 28 x 12 and the adjoint's 28 x 12 and 30 x 6): every node in
    // exactly one block of at most cmax x rmax
    const int shapes[][2] = {{kBlockCols, kBlockRows}, {30, 6}};
    for (const auto& cr : shapes)
    for (int nx : {1, 2, 27, 28, 29, 31, 57, 256, 1000, 65535})
        for (int ny : {1, 5, 6, 7, 11, 12, 13, 100, 1024}) {
            const int cmax = cr[0], rmax = cr[1];
            std::vector<Tile> L;
            plan_blocks(2, nx, ny, cmax, rmax, L);
            std::vector<unsigned char> hit((size_t)nx * ny, 0);
            for (const Tile& t : L) {
                bad |= t.inst != 2 || t.cols < 1 || t.cols > cmax || t.rows < 1 || t.rows > rmax;
                bad |= t.x0 < 0 || t.y0 < 0 || t.x0 + t.cols > nx || t.y0 + t.rows > ny;
                for (int y = t.y0; y < t.y0 + t.rows; ++y)
                    for (int x = t.x0; x < t.x0 + t.cols; ++x) ++hit[(size_t)y * nx + x];
            }
            for (unsigned char h : hit) bad |= h != 1;
        }
    // the adjoint's two-slot rule
    for (int64_t nodes : {(int64_t)1, (int64_t)1 << 21, (int64_t)1 << 22})
        for (uint64_t free_b : {0ull, 1ull << 20, 1ull << 40})
            for (uint64_t held : {0ull, 1ull << 30}) {
                const int s = lbm3_adjoint_pipeline_slots(nodes, 1ull << 31, held, free_b);
                bad |= s != 1 && s != 2;
            }
    std::printf(bad ? "FAILED\n" : "ok\n");
    return bad;
}
