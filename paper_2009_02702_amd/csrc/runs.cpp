// Runs of equal node IDs along the rows of each mip level (host side).
//
// Footprint assembly (Sec. "Fast Sub-Volume Queries") adds 8^l for every cube
// of a box's footprint to the cube's node. Within one row of a level, a run of
// k consecutive cubes on one node adds k 8^l to it at once, so a row segment of
// a footprint slab can be summed from the row's runs instead of cube by cube:
// the same integer counts, reached with work proportional to the runs the
// segment crosses. Rows are taken along x (row (y, z): index y + Y z, the
// x-fastest map) and along y (row (z, x): index z + Z x, the y-fastest map),
// the two contiguous orientations the query kernels read slabs in.
//
// Per level and orientation: row_ptr[r] = first run of row r (row_ptr[rows] =
// runs), runs[j] = (end << 32) | node with `end` the exclusive end of run j
// along the row, and skip[r * chunks + c] = index of the run that holds cell
// 64 c of row r (a segment starting at cell f begins its walk at most 63 cells
// before f; the row's last run ends at the row's end, so a walk that stops at
// the segment's end never leaves the row). Built only where the runs are at
// most a quarter of the level's cells (long runs).
#include <algorithm>
#include <thread>
#include <vector>

#include "mg_internal.hpp"

namespace mg {
namespace {

constexpr uint32_t kMinRunLength = 4; // average run length below which a level keeps no runs

template <class Fn>
void parallel_for(uint32_t n, unsigned nt, Fn fn)
{
    const unsigned k = std::max(1u, std::min<unsigned>(nt, n));
    std::vector<std::thread> th;
    for (unsigned t = 0; t < k; ++t)
        th.emplace_back(fn, uint32_t(uint64_t(n) * t / k), uint32_t(uint64_t(n) * (t + 1) / k));
    for (auto &x : th) x.join();
}

// row_ptr from per-row run counts; false if the runs are too many to pay.
bool finish_counts(const std::vector<uint32_t> &cnt, LevelRuns *out)
{
    uint64_t total = 0;
    out->row_ptr.assign(cnt.size() + 1, 0);
    for (size_t r = 0; r < cnt.size(); ++r) {
        out->row_ptr[r] = uint32_t(total);
        total += cnt[r];
        if (total > 0xFFFFFFFFull) return false;
    }
    out->row_ptr[cnt.size()] = uint32_t(total);
    if (total * kMinRunLength > uint64_t(out->rows) * out->len) return false;  // short runs: not worth it
    out->runs.assign(total, 0);
    out->skip.assign(uint64_t(out->rows) * out->chunks, 0);
    return true;
}

// Rows along x of one level (X x Y x Z, x fastest): row y + Y z is contiguous.
bool build_x(const uint32_t *m, uint32_t X, uint32_t Y, uint32_t Z, unsigned nt, LevelRuns *out)
{
    out->rows = Y * Z, out->len = X, out->chunks = (X + kRunSkipCells - 1) / kRunSkipCells;
    std::vector<uint32_t> cnt(out->rows, 0);
    parallel_for(out->rows, nt, [&](uint32_t r0, uint32_t r1) {
        for (uint32_t r = r0; r < r1; ++r) {
            const uint32_t *p = m + uint64_t(X) * r;
            uint32_t k = 1;
            for (uint32_t i = 1; i < X; ++i) k += p[i] != p[i - 1];
            cnt[r] = k;
        }
    });
    if (!finish_counts(cnt, out)) return false;
    parallel_for(out->rows, nt, [&](uint32_t r0, uint32_t r1) {
        for (uint32_t r = r0; r < r1; ++r) {
            const uint32_t *p = m + uint64_t(X) * r;
            uint64_t *o = out->runs.data() + out->row_ptr[r];
            uint32_t *sk = out->skip.data() + uint64_t(r) * out->chunks;
            uint32_t j = 0;
            for (uint32_t i = 0; i < X; ++i) {
                if (i > 0 && p[i] != p[i - 1]) o[j++] = (uint64_t(i) << 32) | p[i - 1];
                if (i % kRunSkipCells == 0) sk[i / kRunSkipCells] = out->row_ptr[r] + j;
            }
            o[j] = (uint64_t(X) << 32) | p[X - 1];
        }
    });
    return true;
}

// Rows along y (row z + Z x: cells x + X (y + Y z), y = 0 .. Y-1). Each z-slice
// is read in x-fastest order with per-x state, so the maps stream once.
bool build_y(const uint32_t *m, uint32_t X, uint32_t Y, uint32_t Z, unsigned nt, LevelRuns *out)
{
    out->rows = Z * X, out->len = Y, out->chunks = (Y + kRunSkipCells - 1) / kRunSkipCells;
    std::vector<uint32_t> cnt(out->rows, 0);
    parallel_for(Z, nt, [&](uint32_t z0, uint32_t z1) {
        for (uint32_t z = z0; z < z1; ++z) {
            const uint32_t *s = m + uint64_t(X) * Y * z;
            for (uint32_t x = 0; x < X; ++x) cnt[z + uint64_t(Z) * x] = 1;
            for (uint32_t y = 1; y < Y; ++y)
                for (uint32_t x = 0; x < X; ++x)
                    cnt[z + uint64_t(Z) * x] += s[x + uint64_t(X) * y] != s[x + uint64_t(X) * (y - 1)];
        }
    });
    if (!finish_counts(cnt, out)) return false;
    parallel_for(Z, nt, [&](uint32_t z0, uint32_t z1) {
        std::vector<uint32_t> j(X);
        for (uint32_t z = z0; z < z1; ++z) {
            const uint32_t *s = m + uint64_t(X) * Y * z;
            std::fill(j.begin(), j.end(), 0u);
            for (uint32_t y = 0; y < Y; ++y)
                for (uint32_t x = 0; x < X; ++x) {
                    const uint64_t r = z + uint64_t(Z) * x;
                    const uint32_t v = s[x + uint64_t(X) * y];
                    if (y > 0 && v != s[x + uint64_t(X) * (y - 1)])
                        out->runs[out->row_ptr[r] + j[x]++] = (uint64_t(y) << 32) | s[x + uint64_t(X) * (y - 1)];
                    if (y % kRunSkipCells == 0) out->skip[r * out->chunks + y / kRunSkipCells] = out->row_ptr[r] + j[x];
                }
            for (uint32_t x = 0; x < X; ++x) {
                const uint64_t r = z + uint64_t(Z) * x;
                out->runs[out->row_ptr[r] + j[x]] = (uint64_t(Y) << 32) | s[x + uint64_t(X) * (Y - 1)];
            }
        }
    });
    return true;
}

}  // namespace

void ensure_runs(const Graph &g)
{
    if (g.runs_ready) return;
    g.runs.assign(2 * size_t(g.n_levels), LevelRuns());
    g.runs_ready = true;
    if (g.maps.size() != g.lev_off[g.n_levels]) return;  // maps only on the device: no runs
    const unsigned nt = resolve_threads(0);
    for (uint32_t l = 0; l < g.n_levels; ++l) {
        const uint32_t X = g.lev_dims[3 * l], Y = g.lev_dims[3 * l + 1], Z = g.lev_dims[3 * l + 2];
        const uint32_t *m = g.maps.data() + g.lev_off[l];
        // rows along x (row y + Y z) and along y (row z + Z x)
        if (uint64_t(Y) * Z < 0xFFFFFFFFull && !build_x(m, X, Y, Z, nt, &g.runs[2 * l])) g.runs[2 * l] = LevelRuns();
        if (uint64_t(Z) * X < 0xFFFFFFFFull && !build_y(m, X, Y, Z, nt, &g.runs[2 * l + 1]))
            g.runs[2 * l + 1] = LevelRuns();
    }
}

}  // namespace mg
