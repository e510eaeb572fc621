// Host-side tile plans for the fused step (shared by the plain and batched forms).
#include <algorithm>

#include "lbm3_internal.h"

namespace tcg {

void plan_lattice(int inst, int nx, int ny, int threads, int rows, int elem_bytes,
                  std::vector<Tile>& out)
{
    const int wmax = threads - 6;
    const int nseg = std::max(1, (ny + std::max(rows, 1) - 1) / std::max(rows, 1));
    // Line-aligned strips: widths in units of A elements (one 128-byte line) and strips
    // starting at x = 3 (mod A), so that lane 0 of every wavefront (column x0 - 3 + 64 w) sits
    // on a line boundary and unshifted loads cover whole lines.  Used when nx is a multiple
    // of A and a unit-aligned strip width fits the workgroup.
    const int A = 128 / elem_bytes;
    const int wA = wmax / A * A;
    const bool aligned = nx % A == 0 && wA >= A && nx > 6;
    const int nstrips = aligned ? (nx / A + wA / A - 1) / (wA / A) : (nx + wmax - 1) / wmax;
    int x0 = aligned ? 3 : 0;
    for (int sx = 0; sx < nstrips; ++sx) {
        const int cols = aligned ? ((nx / A) / nstrips + (sx < (nx / A) % nstrips ? 1 : 0)) * A
                                 : nx / nstrips + (sx < nx % nstrips ? 1 : 0);
        int y0 = 0;
        for (int sy = 0; sy < nseg; ++sy) {
            const int r = ny / nseg + (sy < ny % nseg ? 1 : 0);
            if (r > 0 && cols > 0) {
                Tile t{};
                t.inst = inst;
                t.x0 = x0;
                t.y0 = y0;
                t.rows = r;
                t.cols = cols;
                out.push_back(t);
            }
            y0 += r;
        }
        x0 += cols;
    }
}

std::vector<Tile> xcd_order(const std::vector<Tile>& L, int nxcd)
{
    const int T = (int)L.size();
    std::vector<Tile> out(T);
    std::vector<int> start(nxcd + 1, 0);
    for (int x = 0; x < nxcd; ++x) start[x + 1] = start[x] + (T - x + nxcd - 1) / nxcd;
    for (int b = 0; b < T; ++b) {
        const int x = b % nxcd, k = b / nxcd;
        out[b] = L[start[x] + k];
    }
    return out;
}

int auto_rows(int nx, int ny, int threads, int slots, int elem_bytes)
{
    std::vector<Tile> probe;
    plan_lattice(0, nx, 1, threads, 1, elem_bytes, probe);
    const int nstrips = (int)probe.size();
    if (slots < 1) slots = 1;
    // time ~ rounds * (rows per segment + 6 warm-up rows: the pipeline is two rows deep
    // and the factored pull starts two source rows further down); fewest rounds, then rows
    double best = 1e300;
    int best_rows = std::min(ny, 64);
    for (int nseg = 1; nseg <= ny; ++nseg) {
        const int rows = (ny + nseg - 1) / nseg;
        if (rows < 2 && nseg > 1) break;
        if (rows > 512) continue;
        const long tiles = (long)nstrips * nseg;
        const long rounds = (tiles + slots - 1) / slots;
        const double cost = (double)rounds * (rows + 6) * (1.0 + 1e-9 * nseg);
        if (cost < best) {
            best = cost;
            best_rows = rows;
        }
    }
    return best_rows;
}

int device_slots(Prec prec, int threads)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return blocks_per_cu(prec, threads) * cus;
}

}  // namespace tcg
