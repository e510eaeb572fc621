// Host-side tile plans for the fused step (shared by the plain and batched forms).
#include <algorithm>

#include "lbm3_internal.h"

namespace tcg {

void plan_lattice(int inst, int nx, int ny, int threads, int rows, int elem_bytes,
                  std::vector<Tile>& out, int halo)
{
    const int wmax = threads - 2 * halo;
    const int nseg = std::max(1, (ny + std::max(rows, 1) - 1) / std::max(rows, 1));
    // Aligned strips: widths in units of A elements and strips starting at x = halo (mod A), so
    // that lane 0 of every wavefront (column x0 - halo + 64 w) sits on a unit boundary.  Used
    // when nx is a multiple of A and a unit-aligned strip width fits the workgroup.  The
    // single step takes 128-byte units (one cache line).  The two-step pass (halo 6) takes
    // units of four columns (32 bytes in FP64, 16 in FP32), which lets the strips fill the
    // device: at 4096 columns 17 strips of 240-244 columns give 255 workgroups for 256 CUs
    // (one per CU), where line-aligned strips of at most 240 columns need 18 strips and leave
    // 252 (measured: FP64 3.7% faster; FP32 storage 7% and FP32 5% faster than with
    // eight-column units).
    const int A = halo == 6 ? 4 : 128 / elem_bytes;
    const int wA = wmax / A * A;
    const bool aligned = nx % A == 0 && wA >= A && nx > 2 * halo;
    const int nstrips = aligned ? (nx / A + wA / A - 1) / (wA / A) : (nx + wmax - 1) / wmax;
    // strips (x0, cols) and segments (y0, rows)
    std::vector<int> sx0(nstrips), scols(nstrips), sy0(nseg), srows(nseg);
    int x0 = aligned ? halo : 0;
    for (int sx = 0; sx < nstrips; ++sx) {
        scols[sx] = aligned ? ((nx / A) / nstrips + (sx < (nx / A) % nstrips ? 1 : 0)) * A
                            : nx / nstrips + (sx < nx % nstrips ? 1 : 0);
        sx0[sx] = x0;
        x0 += scols[sx];
    }
    int y0 = 0;
    for (int sy = 0; sy < nseg; ++sy) {
        srows[sy] = ny / nseg + (sy < ny % nseg ? 1 : 0);
        sy0[sy] = y0;
        y0 += srows[sy];
    }
    // row of tiles after row of tiles: side-by-side tiles march the same rows at the same
    // time, so the halo columns they share are still in L2 when the second one reads them
    for (int sy = 0; sy < nseg; ++sy)
        for (int sx = 0; sx < nstrips; ++sx)
            if (srows[sy] > 0 && scols[sx] > 0) {
                Tile t{};
                t.inst = inst;
                t.x0 = sx0[sx];
                t.y0 = sy0[sy];
                t.rows = srows[sy];
                t.cols = scols[sx];
                out.push_back(t);
            }
}

void plan_blocks(int inst, int nx, int ny, int cmax, int rmax, std::vector<Tile>& out)
{
    const int nbx = (nx + cmax - 1) / cmax, nby = (ny + rmax - 1) / rmax;
    int y0 = 0;
    for (int by = 0; by < nby; ++by) {
        const int rows = ny / nby + (by < ny % nby ? 1 : 0);
        int x0 = 0;
        for (int bx = 0; bx < nbx; ++bx) {
            const int cols = nx / nbx + (bx < nx % nbx ? 1 : 0);
            Tile t{};
            t.inst = inst;
            t.x0 = x0;
            t.y0 = y0;
            t.rows = rows;
            t.cols = cols;
            out.push_back(t);
            x0 += cols;
        }
        y0 += rows;
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

// A step reads one state buffer and writes the other at the same offsets at the same time.
// With the two an even number of MiB apart (what two separate allocations of a size that is
// a multiple of 2 MiB give), the FP64 two-step pass ran at 29.0k MLUPS at 4096^2; an odd
// number of MiB apart, at 30.0k, in every run (measured with distances of the buffer size
// plus 0, 64 KiB, 1, 2 and 3 MiB): the concurrent read and write streams then fall on
// different HBM channels.
hipError_t alloc_state_pair(size_t bytes, void* buf[2])
{
    constexpr size_t MiB = (size_t)1 << 20;
    const size_t off = (bytes + 2 * MiB - 1) / (2 * MiB) * (2 * MiB) + MiB;
    buf[0] = buf[1] = nullptr;
    void* base = nullptr;
    hipError_t e = hipMalloc(&base, off + bytes);
    if (e != hipSuccess) return e;
    buf[0] = base;
    buf[1] = (char*)base + off;
    return hipSuccess;
}

void free_state_pair(void* buf[2])
{
    if (buf[0]) (void)hipFree(buf[0]);
    buf[0] = buf[1] = nullptr;
}

int auto_rows(int nx, int ny, int threads, int slots, int elem_bytes, int halo)
{
    std::vector<Tile> probe;
    plan_lattice(0, nx, 1, threads, 1, elem_bytes, probe, halo);
    const int nstrips = (int)probe.size();
    if (slots < 1) slots = 1;
    // time ~ rounds * (rows per segment + 2 halo warm-up rows: a step's pipeline is two
    // rows deep and its factored pull starts two source rows further down, six rows in
    // all, twelve for the two-step pass); fewest rounds, then fewest rows
    double best = 1e300;
    int best_rows = std::min(ny, 64);
    for (int nseg = 1; nseg <= ny; ++nseg) {
        const int rows = (ny + nseg - 1) / nseg;
        if (rows < 2 && nseg > 1) break;
        if (rows > 512) continue;
        const long tiles = (long)nstrips * nseg;
        const long rounds = (tiles + slots - 1) / slots;
        const double cost = (double)rounds * (rows + 2 * halo) * (1.0 + 1e-9 * nseg);
        if (cost < best) {
            best = cost;
            best_rows = rows;
        }
    }
    return best_rows;
}

static int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

int device_slots(Prec prec, int threads) { return blocks_per_cu(prec, threads) * device_cus(); }

int device_slots_pair(Prec prec, int threads)
{
    int per_cu = 0;
    if (prec == Prec::F64) per_cu = tiles_f64_pair_occupancy(threads);
    if (prec == Prec::F32) per_cu = tiles_f32_pair_occupancy(threads);
    if (prec == Prec::F32S) per_cu = tiles_f32s_pair_occupancy(threads);
    return per_cu * device_cus();
}

}  // namespace tcg
