/*
 * ORACLE (test infrastructure only; not part of the product path).
 *
 * O1: the plain definition of a box histogram (Sec. "Fast Sub-Volume Queries"):
 * for every box, the number of level-0 voxels carrying each segment, found by
 * visiting every voxel of the box. No mipmap, no footprint, no graph.
 *
 *   vol[x + nx*(y + ny*z)]   compacted segment index in [0, nseg)
 *   boxes[6*q .. 6*q+5]      (x0, y0, z0, dx, dy, dz), half-open extents;
 *                            the upper end is clipped to the volume and an
 *                            origin at or beyond the volume gives an empty box
 *   counts[q*nseg + s]       uint64 voxel count of segment s in box q
 *   probs[q*nseg + s]        counts / (voxels in the clipped box), fp64;
 *                            all zeros for an empty box (may be NULL)
 *
 * Parallel over boxes with OpenMP; `threads` <= 0 keeps the OpenMP default.
 * Returns 0, or -1 on a bad argument, -2 if a voxel holds an index >= nseg.
 */
#include <omp.h>
#include <stdint.h>
#include <string.h>

static inline int64_t clip_hi(int64_t lo, int64_t ext, int64_t dim)
{
    int64_t hi = lo + ext;
    return hi < dim ? hi : dim;
}

int o1_box_counts(const uint32_t *vol, int64_t nx, int64_t ny, int64_t nz, int64_t nseg,
                  const uint32_t *boxes, int64_t nbox, uint64_t *counts, double *probs, int threads)
{
    if (!vol || !boxes || !counts || nx <= 0 || ny <= 0 || nz <= 0 || nseg <= 0 || nbox < 0) return -1;
    if (threads > 0) omp_set_num_threads(threads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nbox; ++q) {
        uint64_t *c = counts + q * nseg;
        memset(c, 0, sizeof(uint64_t) * (size_t)nseg);
        const int64_t x0 = boxes[6 * q], y0 = boxes[6 * q + 1], z0 = boxes[6 * q + 2];
        const int64_t x1 = clip_hi(x0, boxes[6 * q + 3], nx);
        const int64_t y1 = clip_hi(y0, boxes[6 * q + 4], ny);
        const int64_t z1 = clip_hi(z0, boxes[6 * q + 5], nz);
        int64_t n = 0;
        for (int64_t z = z0; z < z1; ++z)
            for (int64_t y = y0; y < y1; ++y) {
                const uint32_t *row = vol + nx * (y + ny * z);
                for (int64_t x = x0; x < x1; ++x) {
                    const uint32_t s = row[x];
                    if ((int64_t)s >= nseg) {
#pragma omp atomic write
                        bad = 1;
                        continue;
                    }
                    c[s] += 1;
                    ++n;
                }
            }
        if (probs) {
            double *p = probs + q * nseg;
            for (int64_t s = 0; s < nseg; ++s) p[s] = n > 0 ? (double)c[s] / (double)n : 0.0;
        }
    }
    return bad ? -2 : 0;
}

/*
 * Compaction of a label volume to segment indices (the distinct IDs in
 * increasing order are numbered 0, 1, ...): lut[max_id + 1] must be zeroed by
 * the caller; on return lut[id] is 1 + the index of every present ID (0 for
 * absent ones) and out[i] the index of vol[i]. Returns the number of distinct
 * IDs, or -1 if a voxel holds an ID above max_id.
 */
int64_t o1_compact(const uint32_t *vol, int64_t n, uint32_t max_id, uint32_t *lut, uint32_t *out, int threads)
{
    if (threads > 0) omp_set_num_threads(threads);
    int bad = 0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (vol[i] > max_id) {
#pragma omp atomic write
            bad = 1;
            continue;
        }
#pragma omp atomic write
        lut[vol[i]] = 1u;
    }
    if (bad) return -1;
    int64_t k = 0;
    for (int64_t v = 0; v <= (int64_t)max_id; ++v)
        if (lut[v]) lut[v] = (uint32_t)(++k);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = lut[vol[i]] - 1u;
    return k;
}

int o1_max_threads(void) { return omp_get_max_threads(); }
