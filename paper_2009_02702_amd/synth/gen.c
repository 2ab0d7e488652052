/*
 * Seeded synthetic segmentation volumes (input generation only).
 *
 * This file draws no random numbers and computes nothing of the Mixture
 * Graph method: the caller (synth/__init__.py) draws seed points and shape
 * parameters from a seeded PCG64 stream and passes them in; this code only
 * rasterises them into a uint32 label volume, x fastest:
 *   index(x, y, z) = x + nx * (y + ny * z).
 *
 *  - synth_voronoi:  label = base + argmin_k |c(v) - s_k|^2 over seed points
 *    s_k, with c(v) = (x + 1/2, y + 1/2, z + 1/2) and the z difference scaled
 *    by zscale (anisotropic distance). Ties go to the lower k, exactly as a
 *    brute-force scan in increasing k with a strict '<' would.
 *  - synth_cell_sums: per-label sums of voxel centres, for one Lloyd step.
 *  - synth_cylinders: capsules painted in order (later ones overwrite): a
 *    voxel centre within r_k of the segment [p_k, q_k] gets label k + 1.
 *
 * Built with gcc -O3 -fopenmp; results do not depend on the thread count
 * because every voxel is computed independently (Voronoi) or every z slice is
 * owned by one thread that paints all capsules in order (cylinders).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline double sqr(double v) { return v * v; }

/* Exact argmin over a candidate superset: the candidates of a block are all
 * seeds whose distance to the block's bounding box of voxel centres is within
 * the smallest "farthest-corner" distance of any seed, widened by a relative
 * margin so that rounding can only add candidates, never drop the winner. */
int synth_voronoi(uint32_t *out, int64_t nx, int64_t ny, int64_t nz,
                  const double *seeds, int64_t k, double zscale, uint32_t base,
                  int64_t bx, int64_t by, int64_t bz)
{
    if (!out || !seeds || k <= 0 || nx <= 0 || ny <= 0 || nz <= 0) return -1;
    if (bx <= 0 || by <= 0 || bz <= 0) return -1;
    const int64_t gx = (nx + bx - 1) / bx, gy = (ny + by - 1) / by, gz = (nz + bz - 1) / bz;
    const int64_t nblocks = gx * gy * gz;
    int failed = 0;
#pragma omp parallel
    {
        int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
        if (!cand) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 4)
        for (int64_t b = 0; b < nblocks; ++b) {
            if (!cand) continue;
            const int64_t ix = b % gx, iy = (b / gx) % gy, iz = b / (gx * gy);
            const int64_t x0 = ix * bx, y0 = iy * by, z0 = iz * bz;
            const int64_t x1 = x0 + bx < nx ? x0 + bx : nx;
            const int64_t y1 = y0 + by < ny ? y0 + by : ny;
            const int64_t z1 = z0 + bz < nz ? z0 + bz : nz;
            /* bounding box of voxel centres, z in scaled units */
            const double lx = x0 + 0.5, hx = x1 - 0.5;
            const double ly = y0 + 0.5, hy = y1 - 0.5;
            const double lz = (z0 + 0.5) * zscale, hz = (z1 - 0.5) * zscale;
            double best = INFINITY;
            for (int64_t s = 0; s < k; ++s) {
                const double sx = seeds[3 * s], sy = seeds[3 * s + 1], sz = seeds[3 * s + 2] * zscale;
                const double fx = fmax(fabs(sx - lx), fabs(sx - hx));
                const double fy = fmax(fabs(sy - ly), fabs(sy - hy));
                const double fz = fmax(fabs(sz - lz), fabs(sz - hz));
                const double d = fx * fx + fy * fy + fz * fz;
                if (d < best) best = d;
            }
            const double lim = best * (1.0 + 1e-9) + 1e-9;
            int64_t nc = 0;
            for (int64_t s = 0; s < k; ++s) {
                const double sx = seeds[3 * s], sy = seeds[3 * s + 1], sz = seeds[3 * s + 2] * zscale;
                const double dx = sx < lx ? lx - sx : (sx > hx ? sx - hx : 0.0);
                const double dy = sy < ly ? ly - sy : (sy > hy ? sy - hy : 0.0);
                const double dz = sz < lz ? lz - sz : (sz > hz ? sz - hz : 0.0);
                if (dx * dx + dy * dy + dz * dz <= lim) cand[nc++] = s;
            }
            for (int64_t z = z0; z < z1; ++z)
                for (int64_t y = y0; y < y1; ++y)
                    for (int64_t x = x0; x < x1; ++x) {
                        const double cx = x + 0.5, cy = y + 0.5, cz = z + 0.5;
                        double bd = INFINITY;
                        int64_t bs = 0;
                        for (int64_t c = 0; c < nc; ++c) {
                            const int64_t s = cand[c];
                            const double d = sqr(cx - seeds[3 * s]) + sqr(cy - seeds[3 * s + 1]) +
                                             sqr((cz - seeds[3 * s + 2]) * zscale);
                            if (d < bd) { bd = d; bs = s; }
                        }
                        out[x + nx * (y + ny * z)] = base + (uint32_t)bs;
                    }
        }
        free(cand);
    }
    return failed ? -2 : 0;
}

/* Brute force over all seeds, for testing the accelerated scan. */
int synth_voronoi_brute(uint32_t *out, int64_t nx, int64_t ny, int64_t nz,
                        const double *seeds, int64_t k, double zscale, uint32_t base)
{
    if (!out || !seeds || k <= 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const double cx = x + 0.5, cy = y + 0.5, cz = z + 0.5;
                double bd = INFINITY;
                int64_t bs = 0;
                for (int64_t s = 0; s < k; ++s) {
                    const double d = sqr(cx - seeds[3 * s]) + sqr(cy - seeds[3 * s + 1]) +
                                     sqr((cz - seeds[3 * s + 2]) * zscale);
                    if (d < bd) { bd = d; bs = s; }
                }
                out[x + nx * (y + ny * z)] = base + (uint32_t)bs;
            }
    return 0;
}

/* sums[3*(label-base)+c] += centre coordinate c, counts[label-base] += 1 */
int synth_cell_sums(const uint32_t *lab, int64_t nx, int64_t ny, int64_t nz,
                    uint32_t base, int64_t k, double *sums, int64_t *counts)
{
    if (!lab || !sums || !counts || k <= 0) return -1;
    memset(sums, 0, sizeof(double) * 3 * (size_t)k);
    memset(counts, 0, sizeof(int64_t) * (size_t)k);
    int bad = 0;
#pragma omp parallel
    {
        double *ls = (double *)calloc(3 * (size_t)k, sizeof(double));
        int64_t *lc = (int64_t *)calloc((size_t)k, sizeof(int64_t));
        if (!ls || !lc) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(static)
        for (int64_t z = 0; z < nz; ++z) {
            if (!ls || !lc) continue;
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    const uint32_t v = lab[x + nx * (y + ny * z)];
                    if (v < base || (int64_t)(v - base) >= k) continue;
                    const int64_t s = v - base;
                    ls[3 * s] += x + 0.5;
                    ls[3 * s + 1] += y + 0.5;
                    ls[3 * s + 2] += z + 0.5;
                    lc[s] += 1;
                }
        }
#pragma omp critical
        {
            if (ls && lc)
                for (int64_t s = 0; s < k; ++s) {
                    sums[3 * s] += ls[3 * s];
                    sums[3 * s + 1] += ls[3 * s + 1];
                    sums[3 * s + 2] += ls[3 * s + 2];
                    counts[s] += lc[s];
                }
        }
        free(ls);
        free(lc);
    }
    return bad ? -2 : 0;
}

/* Squared distance from point c to the segment [p, q]. */
static inline double seg_dist2(const double *c, const double *p, const double *q)
{
    const double ux = q[0] - p[0], uy = q[1] - p[1], uz = q[2] - p[2];
    const double wx = c[0] - p[0], wy = c[1] - p[1], wz = c[2] - p[2];
    const double uu = ux * ux + uy * uy + uz * uz;
    double t = uu > 0 ? (wx * ux + wy * uy + wz * uz) / uu : 0.0;
    t = t < 0 ? 0 : (t > 1 ? 1 : t);
    return sqr(wx - t * ux) + sqr(wy - t * uy) + sqr(wz - t * uz);
}

/* params[8*i .. 8*i+7] = (px, py, pz, qx, qy, qz, r, unused).
 * Every z slice is painted by one thread, capsules in increasing i, so the
 * last capsule covering a voxel wins regardless of the thread count. The
 * per-row x range is a conservative interval from the capsule's bounding box
 * clipped by its distance to the infinite axis line; each voxel in it is
 * tested with the exact predicate. */
int synth_cylinders(uint32_t *out, int64_t nx, int64_t ny, int64_t nz,
                    const double *params, int64_t k)
{
    if (!out || !params || k < 0) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t z = 0; z < nz; ++z) {
        for (int64_t i = 0; i < k; ++i) {
            const double *p = params + 8 * i, *q = params + 8 * i + 3;
            const double r = params[8 * i + 6];
            const double r2 = r * r;
            const double zc = z + 0.5;
            const double zlo = fmin(p[2], q[2]) - r, zhi = fmax(p[2], q[2]) + r;
            if (zc < zlo || zc > zhi) continue;
            int64_t ylo = (int64_t)floor(fmin(p[1], q[1]) - r - 0.5) - 1;
            int64_t yhi = (int64_t)ceil(fmax(p[1], q[1]) + r - 0.5) + 1;
            int64_t xlo0 = (int64_t)floor(fmin(p[0], q[0]) - r - 0.5) - 1;
            int64_t xhi0 = (int64_t)ceil(fmax(p[0], q[0]) + r - 0.5) + 1;
            if (ylo < 0) ylo = 0;
            if (yhi > ny - 1) yhi = ny - 1;
            if (xlo0 < 0) xlo0 = 0;
            if (xhi0 > nx - 1) xhi0 = nx - 1;
            const double ux = q[0] - p[0], uy = q[1] - p[1], uz = q[2] - p[2];
            const double L2 = ux * ux + uy * uy + uz * uz;
            for (int64_t y = ylo; y <= yhi; ++y) {
                const double yc = y + 0.5;
                int64_t xlo = xlo0, xhi = xhi0;
                if (L2 > 0) {
                    /* distance^2 from (x, yc, zc) to the axis line is a
                     * quadratic A x^2 + B x + C; keep x where it is <= r^2 */
                    const double e[3] = {1.0, 0.0, 0.0};
                    const double w0[3] = {0.0 - p[0], yc - p[1], zc - p[2]};
                    const double eu = (e[0] * ux) / L2;
                    const double wu = (w0[0] * ux + w0[1] * uy + w0[2] * uz) / L2;
                    /* residual r(x) = w0 + x e - (wu + x eu) u */
                    const double ax = e[0] - eu * ux, ay = -eu * uy, az = -eu * uz;
                    const double bx0 = w0[0] - wu * ux, by0 = w0[1] - wu * uy, bz0 = w0[2] - wu * uz;
                    const double A = ax * ax + ay * ay + az * az;
                    const double B = 2 * (ax * bx0 + ay * by0 + az * bz0);
                    const double C = bx0 * bx0 + by0 * by0 + bz0 * bz0 - r2;
                    if (A > 1e-12) {
                        const double disc = B * B - 4 * A * C;
                        if (disc < 0) continue;
                        const double sq = sqrt(disc);
                        const double xa = (-B - sq) / (2 * A), xb = (-B + sq) / (2 * A);
                        const int64_t l = (int64_t)floor(xa - 0.5) - 1;
                        const int64_t h = (int64_t)ceil(xb - 0.5) + 1;
                        if (l > xlo) xlo = l;
                        if (h < xhi) xhi = h;
                    } else if (C > 1e-9 * (1.0 + r2)) {
                        continue; /* axis parallel to x and row farther than r */
                    }
                }
                for (int64_t x = xlo; x <= xhi; ++x) {
                    const double c[3] = {x + 0.5, yc, zc};
                    if (seg_dist2(c, p, q) <= r2) out[x + nx * (y + ny * z)] = (uint32_t)(i + 1);
                }
            }
        }
    }
    return 0;
}

/* Brute-force painter for testing the row intervals above. */
int synth_cylinders_brute(uint32_t *out, int64_t nx, int64_t ny, int64_t nz,
                          const double *params, int64_t k)
{
    if (!out || !params || k < 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const double c[3] = {x + 0.5, y + 0.5, z + 0.5};
                for (int64_t i = 0; i < k; ++i) {
                    const double *p = params + 8 * i, *q = params + 8 * i + 3;
                    if (seg_dist2(c, p, q) <= params[8 * i + 6] * params[8 * i + 6])
                        out[x + nx * (y + ny * z)] = (uint32_t)(i + 1);
                }
            }
    return 0;
}
