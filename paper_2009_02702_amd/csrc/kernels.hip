// HIP kernels for gfx950 (MI355X): box-histogram queries over the Mixture
// Graph, the naive level-0 range scan, transfer-function propagation, and the
// device side of upload / workspaces / timing.
//
// Box decomposition (Sec. "Fast Sub-Volume Queries" and the appendix
// algorithm "Footprint assembly in 3D"). The footprint of a box is the set of
// maximal aligned mipmap cubes inside it. Per axis and level l, the level-l
// cells fully inside [x0, x1) are [a_l, b_l) with a_l = ceil(x0 / 2^l) and
// b_l = floor(x1 / 2^l); the cells of that range not covered by a level-(l+1)
// cell inside the box are the (at most two) 1D footprint steps of level l.
// The tensor product of the 1D step lists, tessellated by cubes of the
// smallest level, groups by level into a hollow shell: the outer block
// [a_l, b_l)^3 minus the inner block [2 a_{l+1}, 2 b_{l+1})^3, i.e. at most
// six slabs one cell thick. The kernels enumerate those <= 6 slabs per level
// instead of the up to (2 log2 D)^3 rectangles; the cube set is the same.
// Slabs that are one cell thick along x are read from a transposed copy of
// the level's node map (y fastest) so that every slab streams contiguous rows.
//
// Each cube contributes its 8^l voxels to the node its mip voxel holds
// ("denormalized" samples). Cubes whose node is a source add straight to the
// segment's integer count; other nodes collect integer counts in a per-query
// hash table, then their mass is pushed down the DAG step by step in reverse
// order (node n = (1 - w_n) a_n + w_n b_n gives a the share 1 - w_n and b the
// share w_n). Mass is fp32 with a two-sum compensation term per entry; the
// final per-segment count is summed in fp64 and divided by the box volume.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mg_internal.hpp"

namespace mg {
namespace {

constexpr int kBlock = 256;                    // plain / fallback / naive workgroup size
constexpr int kBlockBig = 512;                 // big-box tier workgroup size
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kMaxLevelsDev = 16;          // dims up to 32768 per axis
constexpr int kMaxSlabs = 6 * kMaxLevelsDev;
constexpr uint32_t kHashPlain = 2048;         // per-box hash slots in LDS, plain kernel
constexpr uint32_t kHashSmall = 256;          // small-box tier (per-source arrays in LDS)
constexpr uint32_t kHashBig = 2048;           // big-box tier (per-source arrays in LDS)
constexpr uint32_t kHashSmallSparse = 2048;   // small-box tier, sources as table entries
constexpr uint32_t kHashBigSparse = 4096;     // big-box tier, sources as table entries
constexpr uint32_t kHashRetry = 8192;         // boxes that overflowed a tier table
constexpr uint32_t kBigLog2 = 14;             // boxes of >= 2^14 cubes go to the big tier
constexpr uint32_t kHashGlobal = 1u << 16;    // fewest per-worker hash slots in the fallback tables
constexpr uint32_t kSegLdsMax = 2048;         // sources kept in LDS
constexpr uint32_t kFallbackWorkers = 128;    // workers of the final global-table launch (budget)
constexpr uint32_t kRunSeg = 256;             // cells of a row one thread sums from the runs
constexpr int kRunBatch = 4;                   // runs a thread loads at once per segment
constexpr uint32_t kRunMinRow = 128;           // rows shorter than this stream cube by cube (default)
constexpr uint32_t kTfPlanes = 4;             // transfer functions per thread of a propagation step
constexpr uint32_t kTfTailPairs = 4096;        // steps of at most this many node x TF pairs may share a launch
constexpr uint32_t kTfTailSteps = 16;          // at most this many of them
constexpr uint32_t kTfTailBlock = 1024;        // threads of that launch (one workgroup)
constexpr uint32_t kMidWorkers = 256;         // workers of the mid-size global-table launch
constexpr uint32_t kQueues = 8;                // work queues per tier
constexpr uint32_t kQueueStride = 64;          // u32 between queue counters (256 bytes)
constexpr int kUnroll = 4;                     // node-ID loads in flight per lane (plain, fallback)
constexpr uint32_t kMaxSteps = 64;              // graph depth the step table holds
constexpr uint32_t kDeferSlots = 128;           // per-wave ring of deferred internal-node runs (dense state)

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            *err = std::string(#expr) + ": " + hipGetErrorString(e_);                  \
            return MG_EDEVICE;                                                         \
        }                                                                              \
    } while (0)

// ---------------------------------------------------------------- constants

struct LevelTable {
    uint32_t n_levels;
    uint32_t vol[3];
    uint32_t dims[MG_MAX_LEVELS][3];
    uint64_t off[MG_MAX_LEVELS];     // element offset of each level in maps
    uint64_t total;                  // elements of one full copy (maps_t starts here)
    // 16-bit copy of level 0 (both orientations), rows padded to an even length:
    // x-fastest index x + pitch_x (y + Y z), then at total16 the y-fastest index
    // y + pitch_y (z + Z x); used when `use16` (dense mode, sources < 65535)
    uint32_t use16;
    uint32_t pitch_x, pitch_y;
    uint64_t total16;
    // row runs (kind-2 slabs): bit 2 l + o set where level l has runs along x (o = 0)
    // or y (o = 1) and the launch reads them; slabs whose rows are at least run_min
    // cubes long are summed from runs
    uint32_t runs_mask;
    uint32_t run_min;
};

// Row runs of one level and orientation as the kernels read them (the device copy
// of the host's LevelRuns): runs[j] = exclusive end << 32 | node; skip[r][c] =
// index of the run holding cell 64 c of row r.
struct RunLevel {
    const uint32_t *skip;      // [rows][chunks]
    const uint64_t *runs;      // [n_runs]
    uint32_t rows, chunks, n_runs;
};

// A slab of cubes at one level, as the query kernels read it: e2 slices (slow
// axis, the thinnest) of e1 rows (mid axis) of e0 cubes (fast axis, the
// contiguous axis of the chosen copy: x in maps, y in maps_t), read as `units`
// 4-byte units per row: one 32-bit node ID per cube (kind 0), or, from the
// 16-bit level-0 copy, aligned pairs of source IDs (kind 1; a row whose first
// cube is at an odd position starts one element early, `odd`); or, kind 2, each
// row segment summed from the row runs of its level and orientation (base, s1b,
// s2b, units unused).
struct Slab {
    uint64_t base;         // byte offset of the first unit in its buffer (maps or maps16)
    uint32_t e0, e1, e2;   // cubes along the fast, mid and slow axes
    uint32_t s1b, s2b;     // bytes between rows / slices (0 where the extent is 1)
    uint32_t units;        // 4-byte units per row
    uint32_t bx, by, bz;   // first cube, level coordinates
    uint8_t level;
    uint8_t kind;          // 0: 32-bit node IDs, 1: pairs of 16-bit level-0 source IDs, 2: row runs
    uint8_t axes;          // fast | mid << 2 | slow << 4 (0 = x, 1 = y, 2 = z)
    uint8_t odd;           // kind 1: the row's first unit starts one element before the slab
};
static_assert(sizeof(Slab) == 48, "Slab layout");

__host__ __device__ inline uint32_t slab_count(const Slab &sl) { return sl.e0 * sl.e1 * sl.e2; }

// Level coordinates of the cube at (fast, mid, slow) offsets (i0, i1, i2).
__host__ __device__ inline void slab_coords(const Slab &sl, uint32_t i0, uint32_t i1, uint32_t i2, uint32_t *x,
                                            uint32_t *y, uint32_t *z)
{
    // selects, not an indexed local array (which the device code would keep in scratch)
    const uint32_t f = sl.axes & 3, m = (sl.axes >> 2) & 3, w = (sl.axes >> 4) & 3;
    *x = sl.bx + (f == 0 ? i0 : 0u) + (m == 0 ? i1 : 0u) + (w == 0 ? i2 : 0u);
    *y = sl.by + (f == 1 ? i0 : 0u) + (m == 1 ? i1 : 0u) + (w == 1 ? i2 : 0u);
    *z = sl.bz + (f == 2 ? i0 : 0u) + (m == 2 ? i1 : 0u) + (w == 2 ? i2 : 0u);
}

// Clipped box: half-open ranges; returns false for an empty box.
__host__ __device__ inline bool clip_box(const uint32_t *b, const LevelTable &lt, uint32_t lo[3], uint32_t hi[3])
{
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        const uint64_t l = b[a], h = uint64_t(b[a]) + b[3 + a];
        lo[a] = uint32_t(l < lt.vol[a] ? l : lt.vol[a]);
        hi[a] = uint32_t(h < lt.vol[a] ? h : lt.vol[a]);
        ok = ok && lo[a] < hi[a];
    }
    return ok;
}

// The slab of level `lev` covering cells [x0, x1) x [y0, y1) x [z0, z1): the
// fast axis is x (rows from maps) unless the block is thinner in x than in y
// (rows along y from maps_t); of the other two, the thinner is the slow axis.
// Level 0 uses the 16-bit copy when lt.use16.
template <bool WRITE>
__host__ __device__ inline void put_slab(Slab *out, int *n, const LevelTable &lt, uint32_t lev, uint32_t x0,
                                         uint32_t x1, uint32_t y0, uint32_t y1, uint32_t z0, uint32_t z1)
{
    if (x1 <= x0 || y1 <= y0 || z1 <= z0) return;
    if (!WRITE) {
        ++*n;
        return;
    }
    const uint32_t ex = x1 - x0, ey = y1 - y0, ez = z1 - z0;
    Slab s;
    s.level = uint8_t(lev);
    s.bx = x0, s.by = y0, s.bz = z0;
    // fast axis f (x unless the block is thinner in x than in y), then mid m and slow w
    const uint32_t f = ex < ey ? 1u : 0u, ef = f ? ey : ex;
    uint32_t m, w, em, ew;
    if (f) {
        if (ez >= ex) m = 2, em = ez, w = 0, ew = ex;
        else m = 0, em = ex, w = 2, ew = ez;
    } else {
        if (ey >= ez) m = 1, em = ey, w = 2, ew = ez;
        else m = 2, em = ez, w = 1, ew = ey;
    }
    s.axes = uint8_t(f | (m << 2) | (w << 4));
    s.e0 = ef, s.e1 = em, s.e2 = ew;
    // rows from the runs (while the slab's (row, segment) items fit 32 bits)
    if (ef >= lt.run_min && ((lt.runs_mask >> (2 * lev + f)) & 1u) &&
        uint64_t(em) * ew * ((ef + kRunSeg - 1) / kRunSeg) < (1ull << 30)) {
        s.kind = 2, s.odd = 0, s.base = 0, s.s1b = s.s2b = 0, s.units = ef;
        out[(*n)++] = s;
        return;
    }
    // element strides of the mid and slow axes in the chosen copy, and the first element
    const uint32_t X = lt.dims[lev][0], Y = lt.dims[lev][1], Z = lt.dims[lev][2];
    const bool pairs = lev == 0 && lt.use16;
    const uint32_t px = pairs ? lt.pitch_x : X, py = pairs ? lt.pitch_y : Y;
    s.kind = pairs ? 1 : 0;
    uint64_t sm, sw, first;
    if (f) {  // y fastest: element y + py (z + Z x)
        const uint64_t sz = py, sx = uint64_t(py) * Z;
        sm = m == 2 ? sz : sx, sw = m == 2 ? sx : sz;
        first = (pairs ? lt.total16 : lt.total + lt.off[lev]) + y0 + uint64_t(py) * (z0 + uint64_t(Z) * x0);
    } else {  // x fastest: element x + px (y + Y z)
        const uint64_t sy = px, sz = uint64_t(px) * Y;
        sm = m == 1 ? sy : sz, sw = m == 1 ? sz : sy;
        first = (pairs ? 0 : lt.off[lev]) + x0 + uint64_t(px) * (y0 + uint64_t(Y) * z0);
    }
    const uint32_t odd = pairs ? ((f == 1 ? y0 : x0) & 1u) : 0u;
    const uint32_t esz = pairs ? 2u : 4u;
    s.odd = uint8_t(odd);
    s.base = esz * (first - odd);
    s.s1b = em > 1 ? uint32_t(esz * sm) : 0u;  // < 2^32 whenever the extent is above 1
    s.s2b = ew > 1 ? uint32_t(esz * sw) : 0u;
    s.units = pairs ? (ef + odd + 1) >> 1 : ef;
    out[(*n)++] = s;
}

// Slabs of level `lev` of the box's footprint (at most 6), written to out[0..]
// when WRITE. Returns their count.
template <bool WRITE>
__host__ __device__ inline int level_slabs(const LevelTable &lt, const uint32_t lo[3], const uint32_t hi[3],
                                           uint32_t lev, Slab *out)
{
    uint32_t a[3], b[3], ia[3], ib[3];
    bool outer = true, inner = true;
    for (int d = 0; d < 3; ++d) {
        const uint64_t one = uint64_t(1) << lev;
        a[d] = uint32_t((uint64_t(lo[d]) + one - 1) >> lev);
        b[d] = hi[d] >> lev;
        outer = outer && a[d] < b[d];
        const uint32_t pa = uint32_t((uint64_t(lo[d]) + 2 * one - 1) >> (lev + 1));
        const uint32_t pb = hi[d] >> (lev + 1);
        inner = inner && pa < pb;
        ia[d] = 2 * pa;
        ib[d] = 2 * pb;
    }
    int n = 0;
    if (!outer) return 0;
    if (!inner) {
        put_slab<WRITE>(out, &n, lt, lev, a[0], b[0], a[1], b[1], a[2], b[2]);
        return n;
    }
    put_slab<WRITE>(out, &n, lt, lev, a[0], ia[0], a[1], b[1], a[2], b[2]);       // x low face
    put_slab<WRITE>(out, &n, lt, lev, ib[0], b[0], a[1], b[1], a[2], b[2]);       // x high face
    put_slab<WRITE>(out, &n, lt, lev, ia[0], ib[0], a[1], ia[1], a[2], b[2]);     // y low face
    put_slab<WRITE>(out, &n, lt, lev, ia[0], ib[0], ib[1], b[1], a[2], b[2]);     // y high face
    put_slab<WRITE>(out, &n, lt, lev, ia[0], ib[0], ia[1], ib[1], a[2], ia[2]);   // z low face
    put_slab<WRITE>(out, &n, lt, lev, ia[0], ib[0], ia[1], ib[1], ib[2], b[2]);   // z high face
    return n;
}

// Wave 0 fills the slab table of one box in LDS; returns via LDS the slab
// count. Lane l handles level l. Must be called by all threads of the block
// (contains no barrier itself).
__device__ inline void build_slabs(const LevelTable &lt, const uint32_t lo[3], const uint32_t hi[3], Slab *slabs,
                                   int *n_slabs)
{
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 64) {
        const int k = lane < int(lt.n_levels) ? level_slabs<false>(lt, lo, hi, uint32_t(lane), nullptr) : 0;
        // exclusive prefix over lanes of k
        int incl = k;
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off, 64);
            if (lane >= off) incl += v;
        }
        if (k) level_slabs<true>(lt, lo, hi, uint32_t(lane), slabs + (incl - k));
        if (lane == 63) *n_slabs = incl;
    }
}

// ---------------------------------------------------------------- per-query state

// Per-query accumulators. Internal nodes of rank >= 3 live in an
// open-addressing table (key, mass, compensation); nodes of rank 1 (both
// predecessors are sources) and rank 2 (predecessors of rank <= 1) never enter
// it: their mass goes straight to the sources, in at most two hops. Sources keep an exact integer count (cubes whose node is a
// source) plus pushed fp32 mass with its compensation term: in dense mode in
// per-source arrays [S], in sparse mode (many sources) as entries of the same
// table. Pointers are into LDS or into a global per-worker region; the same
// code serves both (the compiler resolves the address space after inlining).
struct QueryState {
    uint32_t *keys;     // [cap] node ID or kEmpty
    uint32_t *cnt;      // [cap] exact integer counts of source entries (sparse mode)
    float *hi, *lo;     // [cap] mass and its compensation
    uint32_t *used;     // [cap] slots in insertion order
    uint32_t *n_used;   // scalar
    uint32_t *flags;    // scalar: bit 0 = overflow
    uint32_t *max_key;  // scalar: largest node ID inserted
    uint32_t cap;       // power of two
    uint32_t limit;     // load-factor cap on n_used
    uint32_t *seg_cnt;  // [S] exact integer counts (dense mode)
    float *seg_hi, *seg_lo;  // [S] pushed mass and its compensation (dense mode)
    Slab *slabs;        // [6 * levels] the box's slabs (LDS)
    float *seg_var;     // [S] accumulated variance per source (uncertainty queries), or null
};

struct GraphView {
    const NodeTriple *__restrict__ nodes;
    uint32_t nseg;     // sources are IDs [0, nseg)
    uint32_t r1_end;   // rank-1 nodes are IDs [nseg, r1_end)
    uint32_t r2_end;   // rank-2 nodes are IDs [r1_end, r2_end)
};

// Loads of per-query state written by other threads of the block: relaxed
// agent-scope atomics, so that the global-memory variant reads L2 rather than
// a possibly stale L1 line (in LDS these are plain ds_read).
template <class T>
__device__ inline T ld(const T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint32_t hash_node(uint32_t k)
{
    k ^= k >> 16;
    k *= 0x7feb352dU;
    k ^= k >> 15;
    k *= 0x846ca68bU;
    k ^= k >> 16;
    return k;
}

// Slot of node `key`, inserting it if absent. Returns kEmpty on overflow.
__device__ inline uint32_t table_slot(const QueryState &st, uint32_t key)
{
    const uint32_t mask = st.cap - 1;
    uint32_t slot = hash_node(key) & mask;
    for (uint32_t probe = 0; probe < st.cap; ++probe) {
        const uint32_t k = ld(&st.keys[slot]);
        if (k == key) return slot;
        if (k == kEmpty) {
            const uint32_t old = atomicCAS(&st.keys[slot], kEmpty, key);
            if (old == kEmpty) {
                const uint32_t idx = atomicAdd(st.n_used, 1u);
                st.used[idx] = slot;
                atomicMax(st.max_key, key);
                if (idx >= st.limit) atomicOr(st.flags, 1u);
                return slot;
            }
            if (old == key) return slot;
        }
        slot = (slot + 1) & mask;
    }
    atomicOr(st.flags, 1u);
    return kEmpty;
}

// Compensated accumulation: the atomic returns the value it added to, so the
// exact rounding error of that addition is recovered with two-sum and
// accumulated, with the incoming compensation, in the second word.
__device__ inline void add_mass_at(float *hi, float *lo, float h, float l)
{
    const float old = atomicAdd(hi, h);
    const float s = old + h;
    const float bp = s - old;
    const float e = (old - (s - bp)) + (h - bp);
    atomicAdd(lo, e + l);
}

// w * (h + l) as an unevaluated pair: exact product error via fma, plus w * l.
__device__ inline void scale_pair(float w, float h, float l, float *oh, float *ol)
{
    const float p = w * h;
    *oh = p;
    *ol = fmaf(w, h, -p) + w * l;
}

template <bool SPARSE>
__device__ inline void add_source_count(const QueryState &st, uint32_t s, uint32_t c)
{
    if (SPARSE) {
        const uint32_t slot = table_slot(st, s);
        if (slot != kEmpty) atomicAdd(&st.cnt[slot], c);
    } else {
        atomicAdd(&st.seg_cnt[s], c);
    }
}

template <bool SPARSE>
__device__ inline void add_source_mass(const QueryState &st, uint32_t s, float h, float l)
{
    if (SPARSE) {
        const uint32_t slot = table_slot(st, s);
        if (slot != kEmpty) add_mass_at(&st.hi[slot], &st.lo[slot], h, l);
    } else {
        add_mass_at(&st.seg_hi[s], &st.seg_lo[s], h, l);
    }
}

// Mass (h, l) on a rank-1 node with predecessors (a, b), both sources.
template <bool SPARSE>
__device__ inline void push_pair(const QueryState &st, const NodeTriple &t, float h, float l)
{
    float ah, al, bh, bl;
    scale_pair(1.0f - t.w, h, l, &ah, &al);
    scale_pair(t.w, h, l, &bh, &bl);
    add_source_mass<SPARSE>(st, t.a, ah, al);
    add_source_mass<SPARSE>(st, t.b, bh, bl);
}

// Mass (h, l) on a rank-2 node: each predecessor is a source or a rank-1 node,
// so it is pushed to the sources at once (at most two hops), without a table entry.
template <bool SPARSE>
__device__ inline void push_rank2(const QueryState &st, const GraphView &gv, const NodeTriple &t, float h, float l)
{
    float ah, al, bh, bl;
    scale_pair(1.0f - t.w, h, l, &ah, &al);
    scale_pair(t.w, h, l, &bh, &bl);
    // both predecessors' triples in flight before the first addition
    const bool na = t.a >= gv.nseg, nb = t.b >= gv.nseg;
    NodeTriple ta = {0u, 0u, 0.0f}, tb = {0u, 0u, 0.0f};
    if (na) ta = gv.nodes[t.a];
    if (nb) tb = gv.nodes[t.b];
    if (na) push_pair<SPARSE>(st, ta, ah, al);
    else add_source_mass<SPARSE>(st, t.a, ah, al);
    if (nb) push_pair<SPARSE>(st, tb, bh, bl);
    else add_source_mass<SPARSE>(st, t.b, bh, bl);
}

// Mass pushed into `node` during the reverse push. Nodes of rank <= 2 go straight
// to the sources; only nodes of rank >= 3 accumulate in the table.
template <bool SPARSE>
__device__ inline void route_mass(const QueryState &st, const GraphView &gv, uint32_t node, float h, float l)
{
    if (node < gv.nseg) {
        add_source_mass<SPARSE>(st, node, h, l);
    } else if (node < gv.r1_end) {
        push_pair<SPARSE>(st, gv.nodes[node], h, l);
    } else if (node < gv.r2_end) {
        push_rank2<SPARSE>(st, gv, gv.nodes[node], h, l);
    } else {
        const uint32_t slot = table_slot(st, node);
        if (slot != kEmpty) add_mass_at(&st.hi[slot], &st.lo[slot], h, l);
    }
}

// Integer voxel count c (< 2^32) scattered onto `node` by cubes.
template <bool SPARSE>
__device__ inline void scatter_count(const QueryState &st, const GraphView &gv, uint32_t node, uint32_t c)
{
    if (node < gv.nseg) {
        add_source_count<SPARSE>(st, node, c);
        return;
    }
    const float h = float(c & 0xFFFFFF00u), l = float(c & 0xFFu);  // both exact in fp32
    if (node < gv.r1_end) {
        push_pair<SPARSE>(st, gv.nodes[node], h, l);
    } else if (node < gv.r2_end) {
        push_rank2<SPARSE>(st, gv, gv.nodes[node], h, l);
    } else {
        const uint32_t slot = table_slot(st, node);
        if (slot != kEmpty) add_mass_at(&st.hi[slot], &st.lo[slot], h, l);
    }
}

__device__ inline uint64_t lane_above_mask()
{
    const uint32_t lane = threadIdx.x & 63;
    return lane == 63 ? 0 : (~uint64_t(0) << (lane + 1));
}

// Run starts of a wave: lane 0, and every lane whose value differs from lane
// i-1's (DPP wave shift right by one lane; the shift fills lane 0 with 0, and
// lane 0 is a start regardless). Returned as the wave mask of start lanes,
// taken straight from the vector compare.
__device__ inline uint64_t run_starts(uint32_t v, uint32_t *prev_out)
{
    const uint32_t prev = uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x138, 0xF, 0xF, true));
    *prev_out = prev;
    return __builtin_amdgcn_uicmp(v, prev, 33 /* ne */) | 1u;
}

// Distance from this lane to the next run start above it (64 if none):
// the length of the run this lane starts. `above` = lane_above_mask().
__device__ inline uint32_t run_len(uint64_t starts, uint64_t above, uint32_t lane)
{
    const uint64_t m = starts & above;
    return (m ? uint32_t(__builtin_ctzll(m)) : 64u) - lane;
}

// Run-length merge of equal neighbours in a wave: true at the start lane of a
// run of a real value (not kEmpty), with the run's length in *len.
__device__ inline bool run_head(uint32_t v, uint64_t above, uint32_t *len)
{
    const uint32_t lane = threadIdx.x & 63;
    uint32_t prev;
    const uint64_t starts = run_starts(v, &prev);
    *len = run_len(starts, above, lane);
    return (v != prev || lane == 0) && v != kEmpty;
}

__device__ inline uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------- tiled slab walk
//
// A slab is read as e2 slices of e1 rows of `units` 4-byte units (32-bit node
// IDs, or aligned pairs of 16-bit level-0 IDs). A wave covers a tile of 2^ltx
// units x 2^(6 - ltx) rows (lane (lx, ly) = (lane mod 2^ltx, lane / 2^ltx)),
// and a block is UNROLL tiles stacked along the rows, so a lane's UNROLL loads
// are independent and all in flight together. Blocks (t0, rb, k2) are dealt
// to the waves round-robin. The row of tile u is a wave-uniform pointer (scalar
// registers): the block's first row plus u row steps; a lane adds its 32-bit
// byte offset. Row tiles that start past the slab's last row are not consumed
// (the wave-uniform bound n_u) and load from the last tile that starts inside
// it; lanes outside the slab read their tile's first unit (inside the slab) and
// see kEmpty, so every load stays inside the slab. The same helpers give the
// addresses to the kernels and to the host-side replay (mg_check_load_addresses).

struct TileWalk {
    uint32_t units, e1, e2;   // units per row, rows per slice, slices
    uint32_t s1b;             // bytes between rows
    uint64_t s2b;             // bytes between slices
    uint32_t ltx, lty, ty;    // tile: 2^ltx units x ty = 2^lty rows
    uint32_t rows;            // rows per block (ty * UNROLL)
    uint32_t n_t0, n_rb, n_blk;
    uint64_t row_step;        // bytes between the rows of tiles u and u + 1
};

__host__ __device__ inline TileWalk tile_walk(uint32_t units, uint32_t e1, uint32_t e2, uint32_t s1b, uint64_t s2b,
                                              uint32_t unroll)
{
    TileWalk w;
    w.units = units, w.e1 = e1, w.e2 = e2, w.s1b = s1b, w.s2b = s2b;
    uint32_t ltx = 0;
    while (ltx < 6 && (1u << ltx) < units) ++ltx;   // smallest power of two >= units, at most 64
    if (s1b >= (1u << 26)) ltx = 6;                 // one row per tile: lane offsets stay below 2^32
    w.ltx = ltx;
    w.lty = 6u - ltx;
    w.ty = 1u << w.lty;
    w.rows = w.ty * unroll;
    w.n_t0 = (units + (1u << ltx) - 1) >> ltx;
    w.n_rb = (e1 + w.rows - 1) / w.rows;
    w.n_blk = w.n_t0 * w.n_rb * e2;
    w.row_step = uint64_t(w.ty) * s1b;
    return w;
}

// Byte offset, from the slab's first unit, of block (t0, rb, k2)'s first row.
__host__ __device__ inline uint64_t tile_block_offset(const TileWalk &w, uint32_t t0, uint32_t rb, uint32_t k2)
{
    return uint64_t(rb) * w.rows * w.s1b + uint64_t(k2) * w.s2b + (uint64_t(t0) << w.ltx) * 4u;
}

// Row tiles of block row rb that start inside the slab (>= 1 for rb < n_rb).
__host__ __device__ inline uint32_t tile_n_u(const TileWalk &w, uint32_t rb, uint32_t unroll)
{
    const uint32_t n = (w.e1 - rb * w.rows + w.ty - 1) >> w.lty;
    return n < unroll ? n : unroll;
}

// A lane's byte offset inside its tile (< 2^32: ly < 64 and s1b < 2^26 unless ly == 0).
__host__ __device__ inline uint32_t tile_lane_bytes(const TileWalk &w, uint32_t lane)
{
    return (lane >> w.ltx) * w.s1b + (lane & ((1u << w.ltx) - 1)) * 4u;
}

// Its unit index along the row in tile column t0.
__host__ __device__ inline uint32_t tile_unit(const TileWalk &w, uint32_t t0, uint32_t lane)
{
    return (t0 << w.ltx) + (lane & ((1u << w.ltx) - 1));
}

// Row tiles of block (t0, rb) in which the lane's unit lies inside the slab (<= n_u).
__host__ __device__ inline uint32_t tile_n_ok(const TileWalk &w, uint32_t t0, uint32_t rb, uint32_t lane)
{
    const uint32_t row0 = rb * w.rows + (lane >> w.ltx);
    return (tile_unit(w, t0, lane) < w.units && row0 < w.e1) ? ((w.e1 - row0 + w.ty - 1) >> w.lty) : 0u;
}

// The byte offset of load u of a lane in block (t0, rb, k2): the tile row stays on
// tile n_u - 1 past it, and lanes outside the slab read the tile's first unit.
__host__ __device__ inline uint64_t tile_load_offset(const TileWalk &w, uint64_t blk, uint32_t u, uint32_t n_u,
                                                     uint32_t n_ok, uint32_t lane_bytes)
{
    return blk + uint64_t(u < n_u ? u : n_u - 1) * w.row_step + (u < n_ok ? lane_bytes : 0u);
}

// Which elements of a 16-bit pair unit lie in the slab (bit 0: low, bit 1: high); the
// row's first unit starts one element early when `odd`.
__host__ __device__ inline uint32_t pair_bits(uint32_t unit, uint32_t e0, uint32_t odd)
{
    return ((unit > 0 || odd == 0) ? 1u : 0u) | ((2 * unit + 1 < e0 + odd) ? 2u : 0u);
}

// The naive scan's walk of a clipped box: level 0 as one slab of ez slices of ey rows,
// from the 16-bit x-fastest copy (pairs; *odd = parity of the first x) or the 32-bit
// map; *base = byte offset of the first unit.
__host__ __device__ inline TileWalk naive_walk(const LevelTable &lt, const uint32_t lo[3], const uint32_t hi[3],
                                               bool use16, uint32_t unroll, uint64_t *base, uint32_t *odd)
{
    const uint32_t ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
    if (use16) {
        const uint64_t px = lt.pitch_x, pxy = px * lt.vol[1];
        *odd = lo[0] & 1u;
        *base = 2 * (lo[0] - *odd + px * lo[1] + pxy * lo[2]);
        return tile_walk((ex + *odd + 1) >> 1, ey, ez, ey > 1 ? uint32_t(2 * px) : 0u, ez > 1 ? 2 * pxy : 0u, unroll);
    }
    const uint64_t X = lt.vol[0], XY = X * lt.vol[1];
    *odd = 0;
    *base = 4 * (lo[0] + X * lo[1] + XY * lo[2]);
    return tile_walk(ex, ey, ez, ey > 1 ? uint32_t(4 * X) : 0u, ez > 1 ? 4 * XY : 0u, unroll);
}

// Streams a slab of 32-bit node IDs; `use(v)` consumes each of a block's n_u
// values (every lane calls it, kEmpty outside the slab). The next block's loads
// are in flight while a block is consumed. Blocks are dealt round-robin to the
// waves starting at wave `first`. Returns false if `stop()` became true
// (checked every 8 blocks).
template <int UNROLL, int WAVES, class Use, class Stop>
__device__ inline bool stream_slab(const char *__restrict__ p, const TileWalk &tw, uint32_t first, Use use,
                                   Stop stop)
{
    const uint32_t lane = threadIdx.x & 63, wave = uni(threadIdx.x >> 6);  // the wave index is uniform
    const uint32_t lane_bytes = tile_lane_bytes(tw, lane);
    uint32_t fb = (wave + WAVES - first) % WAVES;
    if (fb >= tw.n_blk) return true;
    // block fb < WAVES as (t0, rb, k2), by subtraction (no division)
    uint32_t t0 = fb, rb = 0, k2 = 0;
    while (t0 >= tw.n_t0) {
        t0 -= tw.n_t0;
        if (++rb == tw.n_rb) rb = 0, ++k2;
    }
    auto load = [&](uint32_t (&v)[UNROLL], uint32_t &n_u, uint32_t &n_ok, uint32_t bt0, uint32_t brb,
                    uint32_t bk2) {
        n_u = tile_n_u(tw, brb, UNROLL);
        __builtin_assume(n_u >= 1);  // brb < n_rb: the block's first tile starts inside the slab
        n_ok = tile_n_ok(tw, bt0, brb, lane);
        const char *blk = p + tile_block_offset(tw, bt0, brb, bk2);
        const char *row = blk;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            if (u > 0 && uint32_t(u) < n_u) row += tw.row_step;  // stays on tile n_u - 1 after it
            v[u] = *reinterpret_cast<const uint32_t *>(row + (uint32_t(u) < n_ok ? lane_bytes : 0u));
        }
    };
    uint32_t v[UNROLL], n_u, n_ok;
    load(v, n_u, n_ok, t0, rb, k2);
    uint32_t iter = 0;
    for (; fb < tw.n_blk; fb += WAVES) {
        if ((++iter & 7u) == 0 && stop()) return false;
        // this wave's next block; after its last one, the current block again (loaded, unused)
        uint32_t nt0 = t0 + WAVES, nrb = rb, nk2 = k2;
        while (nt0 >= tw.n_t0) {
            nt0 -= tw.n_t0;
            if (++nrb == tw.n_rb) nrb = 0, ++nk2;
        }
        const bool more = fb + WAVES < tw.n_blk;
        if (!more) nt0 = t0, nrb = rb, nk2 = k2;
        uint32_t w[UNROLL], w_n_u, w_n_ok;
        load(w, w_n_u, w_n_ok, nt0, nrb, nk2);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
            if (uint32_t(u) < n_u) use(uint32_t(u) < n_ok ? v[u] : kEmpty);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) v[u] = w[u];
        n_u = w_n_u, n_ok = w_n_ok;
        t0 = nt0, rb = nrb, k2 = nk2;
    }
    return true;
}

// Streams a slab of the 16-bit level-0 copy, two elements per unit; `use(lo, hi)`
// gets kEmpty for elements outside the slab (e0 elements per row, the row's first
// unit one element early when `odd`). Three blocks in flight (level 0 is most of
// the cubes, and its 32-bit words leave registers to spare): a block past the
// wave's last one is replaced by the block before it (valid addresses, never consumed).
template <int UNROLL, int WAVES, class Use>
__device__ inline void stream_pairs(const char *__restrict__ p, const TileWalk &tw, uint32_t e0, uint32_t odd,
                                    uint32_t first, Use use)
{
    const uint32_t lane = threadIdx.x & 63, wave = uni(threadIdx.x >> 6);
    const uint32_t lane_bytes = tile_lane_bytes(tw, lane);
    uint32_t fb = (wave + WAVES - first) % WAVES;
    if (fb >= tw.n_blk) return;
    uint32_t t0 = fb, rb = 0, k2 = 0;
    while (t0 >= tw.n_t0) {
        t0 -= tw.n_t0;
        if (++rb == tw.n_rb) rb = 0, ++k2;
    }
    // n_lo / n_hi: row tiles in which this lane's low / high element is inside the slab
    auto load = [&](uint32_t (&v)[UNROLL], uint32_t &n_u, uint32_t &n_lo, uint32_t &n_hi, uint32_t bt0,
                    uint32_t brb, uint32_t bk2) {
        n_u = tile_n_u(tw, brb, UNROLL);
        __builtin_assume(n_u >= 1);
        const uint32_t n_ok = tile_n_ok(tw, bt0, brb, lane);
        const uint32_t pb = pair_bits(tile_unit(tw, bt0, lane), e0, odd);
        n_lo = (pb & 1u) ? n_ok : 0u;
        n_hi = (pb & 2u) ? n_ok : 0u;
        const char *blk = p + tile_block_offset(tw, bt0, brb, bk2);
        const char *row = blk;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            if (u > 0 && uint32_t(u) < n_u) row += tw.row_step;
            v[u] = *reinterpret_cast<const uint32_t *>(row + (uint32_t(u) < n_ok ? lane_bytes : 0u));
        }
    };
    auto advance = [&](uint32_t &bt0, uint32_t &brb, uint32_t &bk2) {
        bt0 += WAVES;
        while (bt0 >= tw.n_t0) {
            bt0 -= tw.n_t0;
            if (++brb == tw.n_rb) brb = 0, ++bk2;
        }
    };
    uint32_t v[UNROLL], n_u, n_lo, n_hi;
    load(v, n_u, n_lo, n_hi, t0, rb, k2);
    uint32_t t1 = t0, rb1 = rb, k21 = k2;
    if (fb + WAVES < tw.n_blk) advance(t1, rb1, k21);
    uint32_t w[UNROLL], w_n_u, w_n_lo, w_n_hi;
    load(w, w_n_u, w_n_lo, w_n_hi, t1, rb1, k21);
    for (; fb < tw.n_blk; fb += WAVES) {
        uint32_t t2 = t1, rb2 = rb1, k22 = k21;
        if (fb + 2 * WAVES < tw.n_blk) advance(t2, rb2, k22);
        uint32_t x[UNROLL], x_n_u, x_n_lo, x_n_hi;
        load(x, x_n_u, x_n_lo, x_n_hi, t2, rb2, k22);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
            if (uint32_t(u) < n_u)
                use(uint32_t(u) < n_lo ? (v[u] & 0xFFFFu) : kEmpty, uint32_t(u) < n_hi ? (v[u] >> 16) : kEmpty);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) v[u] = w[u], w[u] = x[u];
        n_u = w_n_u, n_lo = w_n_lo, n_hi = w_n_hi;
        w_n_u = x_n_u, w_n_lo = x_n_lo, w_n_hi = x_n_hi;
        t1 = t2, rb1 = rb2, k21 = k22;
    }
}

// Counts a wave's 128 level-0 elements (lane l holds elements 2l and 2l+1) into
// integer per-source counters: a run of equal sources over elements a..b adds
// -a at its start element and b+1 at its end element (uint32 wrap-around).
__device__ inline void count_pairs(uint32_t *cnt, uint32_t lo, uint32_t hi, uint32_t lane)
{
    const uint32_t prev_hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(hi), 0x138, 0xF, 0xF, true));
    const uint32_t next_lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(lo), 0x130, 0xF, 0xF, true));
    const bool s_lo = lo != prev_hi || lane == 0;   // element 2l starts a run
    const bool e_lo = lo != hi;                     // element 2l ends one, 2l+1 starts one
    const bool e_hi = hi != next_lo || lane == 63;  // element 2l+1 ends one
    if (lo != kEmpty && (s_lo || e_lo)) atomicAdd(&cnt[lo], (s_lo ? 0u - 2 * lane : 0u) + (e_lo ? 2 * lane + 1 : 0u));
    if (hi != kEmpty && (e_lo || e_hi))
        atomicAdd(&cnt[hi], (e_lo ? 0u - (2 * lane + 1) : 0u) + (e_hi ? 2 * lane + 2 : 0u));
}

// Kind-2 slab: every row segment is summed from its row's runs. The block's
// threads take (row, segment) items, a segment being at most kRunSeg cells of
// one row, one at a time: the skip entry of its 64-cell chunk gives the
// run holding the chunk's first cell (runs before the segment end at or before
// its first cell and add nothing); runs are loaded kRunBatch at a time, and
// each adds (cells of it inside the segment) x 8^level to its node. A row's
// last run ends at the row's end, so a walk never passes it; run loads are also
// clamped to the array. (Two or four segments per thread in flight, or the
// wave's first runs merged per node before their atomics, measured slower:
// the tier kernels then need more registers.)
// A load through a pointer that was itself read from memory (the run table): the
// cast tells the compiler it is global memory, so it issues a global load rather
// than a flat one.
template <class T>
__device__ inline T load_global(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)(p);
}

// Segments per row of a kind-2 slab, as log2 of the power of two >= ceil(e0 / kRunSeg).
__host__ __device__ inline uint32_t run_lseg(uint32_t e0)
{
    uint32_t lseg = 0;
    while ((kRunSeg << lseg) < e0) ++lseg;
    return lseg;
}

// Item `it` of a kind-2 slab: its row index r in the level's runs of orientation
// f and its cells [p0, p1) along the row; false for a padding item past the row.
__host__ __device__ inline bool run_item(const Slab &sp, const LevelTable &lt, uint32_t f, uint32_t lseg,
                                         uint32_t it, uint32_t *r, uint32_t *p0, uint32_t *p1)
{
    const uint32_t c = it & ((1u << lseg) - 1), row = it >> lseg;
    const uint32_t i2 = sp.e2 == 1 ? 0u : row / sp.e1, i1 = row - i2 * sp.e1;
    uint32_t x, y, z;
    slab_coords(sp, 0, i1, i2, &x, &y, &z);
    const uint32_t fa = f == 0 ? x : y;
    *p0 = fa + c * kRunSeg;
    *p1 = min(*p0 + kRunSeg, fa + sp.e0);
    *r = f == 0 ? y + lt.dims[sp.level][1] * z : z + lt.dims[sp.level][2] * x;
    return *p0 < *p1;
}

// Runs of cubes on internal nodes (dense state), deferred per wave: entries (node,
// run length | level << 9) in a ring in LDS, resolved 64 at a time, one per lane.
// Resolving one loads the node's (a, b, w) triple (and, at rank 2, its
// predecessors'), so the load chains of 64 runs are in flight together instead
// of one chain in nearly every step of a slab walk. At most 63 entries wait
// after an append; the ring holds those plus the 64 one append can add.
struct DeferRing {
    uint32_t *node;  // [waves][kDeferSlots]
    uint16_t *code;  // [waves][kDeferSlots]
    uint32_t wbase;  // this wave's ring (wave-uniform, as head and tail)
    uint32_t head;   // entries resolved
    uint32_t tail;   // entries appended
};

// A run of `len` cubes of level `lev` on internal node `node` (dense state). The
// node on a cube stands for the cube's own mixture, so the weight of a rank-1 or
// rank-2 node there is (voxels on the b side) / 8^lev: when w 8^lev is an integer
// k (levels <= 7, where the product is exact in fp32), the run's voxels split
// exactly into len (8^lev - k) on the a side and len k on the b side. A side that
// is a source takes its voxels as an integer count; a side that is a rank-1 node
// (rank 2 only) splits its n voxels per cube by its own weight w': n w' is a
// whole number of voxels (w' is a ratio of voxel counts of the mixtures the node
// serves) up to the fp32 rounding of w', which a distance to the nearest integer
// of at most n 2^-22 bounds, and that integer is the split. Any other weight (as
// in a quantized graph) pushes the mass instead. Ranks 1 and 2 share one triple
// load; a rank-2 node's two predecessor triples are loaded together.
template <bool SPARSE>
__device__ inline void resolve_count(const QueryState &st, const GraphView &gv, uint32_t node, uint32_t len,
                                     uint32_t lev)
{
    if (!SPARSE && node < gv.r2_end) {
        const NodeTriple t = gv.nodes[node];
        const uint32_t c = len << (3u * lev);
        const uint32_t cube = 1u << (3u * lev);
        const float kf = t.w * float(cube);  // exact: a power-of-two scale
        const uint32_t k = uint32_t(kf);
        if (node >= gv.r1_end) {
            if (!(lev <= 7u && float(k) == kf && k <= cube)) {
                push_rank2<SPARSE>(st, gv, t, float(c & 0xFFFFFF00u), float(c & 0xFFu));
                return;
            }
            const bool na = t.a >= gv.nseg, nb = t.b >= gv.nseg;
            NodeTriple ta = {0u, 0u, 0.0f}, tb = {0u, 0u, 0.0f};
            if (na) ta = gv.nodes[t.a];
            if (nb) tb = gv.nodes[t.b];
            // n voxels per cube on one side: to a source, or split by a rank-1 node
            auto side = [&](uint32_t s, bool isnode, const NodeTriple &u, uint32_t n) {
                if (n == 0u) return;
                if (!isnode) {
                    atomicAdd(&st.seg_cnt[s], len * n);
                    return;
                }
                const float mf = u.w * float(n), m = rintf(mf);
                if (fabsf(mf - m) <= float(n) * 0x1p-22f && m >= 0.0f && m <= float(n)) {
                    atomicAdd(&st.seg_cnt[u.a], len * (n - uint32_t(m)));
                    atomicAdd(&st.seg_cnt[u.b], len * uint32_t(m));
                    return;
                }
                const uint32_t cs = len * n;
                push_pair<SPARSE>(st, u, float(cs & 0xFFFFFF00u), float(cs & 0xFFu));
            };
            side(t.a, na, ta, cube - k);
            side(t.b, nb, tb, k);
            return;
        }
        if (lev <= 7u && float(k) == kf && k <= cube) {
            atomicAdd(&st.seg_cnt[t.a], len * (cube - k));
            atomicAdd(&st.seg_cnt[t.b], len * k);
            return;
        }
        push_pair<SPARSE>(st, t, float(c & 0xFFFFFF00u), float(c & 0xFFu));
        return;
    }
    scatter_count<SPARSE>(st, gv, node, len << (3u * lev));
}

// Resolves the n <= 64 oldest entries. Every lane of the wave must call.
template <bool SPARSE>
__device__ inline void ring_resolve(DeferRing &q, const QueryState &st, const GraphView &gv, uint32_t n)
{
    const uint32_t lane = threadIdx.x & 63;
    __builtin_amdgcn_wave_barrier();
    if (lane < n) {
        const uint32_t k = q.wbase + ((q.head + lane) & (kDeferSlots - 1));
        const uint32_t code = q.code[k];
        resolve_count<SPARSE>(st, gv, q.node[k], code & 511u, code >> 9);
    }
    q.head += n;
    __builtin_amdgcn_wave_barrier();
}

// Appends a run of `len` (<= 256) cubes of level `lev` on `node` from each lane
// with `want`; resolves 64 entries once 64 wait. Every lane of the wave must call.
template <bool SPARSE>
__device__ inline void ring_put(DeferRing &q, const QueryState &st, const GraphView &gv, bool want, uint32_t node,
                                uint32_t len, uint32_t lev)
{
    const uint64_t put = __builtin_amdgcn_ballot_w64(want);
    if (put == 0) return;
    if (want) {
        const uint32_t below =
            __builtin_amdgcn_mbcnt_hi(uint32_t(put >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(put), 0u));
        const uint32_t k = q.wbase + ((q.tail + below) & (kDeferSlots - 1));
        q.node[k] = node;
        q.code[k] = uint16_t(len | (lev << 9));
    }
    q.tail += uint32_t(__builtin_popcountll(put));
    if (q.tail - q.head >= 64u) ring_resolve<SPARSE>(q, st, gv, 64u);
}

// A kind-2 slab: each lane sums one (row, segment) item from the row runs. In
// dense mode the loops are wave-uniform (lanes whose segment is done idle), so
// that internal-node runs can go to the wave's ring; in sparse mode each lane
// walks its items on its own.
template <int BLOCK, bool SPARSE>
__device__ inline void scatter_runs(const Slab &sp, const RunLevel &rl, const LevelTable &lt, const QueryState &st,
                                    const GraphView &gv, DeferRing &dq)
{
    const uint32_t f = uni(sp.axes) & 3u, lev = uni(sp.level), lw8 = 3 * lev;
    const uint32_t lseg = run_lseg(uni(sp.e0));
    const uint32_t items = (uni(sp.e1) * uni(sp.e2)) << lseg;
    const uint32_t top = rl.n_runs - 1;
    const uint32_t lane = threadIdx.x & 63;
    // runs v[0 .. kRunBatch): each adds its cells in [pos, p1)
    auto consume = [&](const uint64_t *v, uint32_t &pos, uint32_t p1) {
#pragma unroll
        for (int q = 0; q < kRunBatch; ++q) {
            const uint32_t end = uint32_t(v[q] >> 32), node = uint32_t(v[q]);
            const bool act = pos < p1 && end > pos;
            const uint32_t hi = min(end, p1);
            if (SPARSE) {
                if (act) scatter_count<SPARSE>(st, gv, node, (hi - pos) << lw8);
            } else {
                if (act && node < gv.nseg) atomicAdd(&st.seg_cnt[node], (hi - pos) << lw8);
                ring_put<SPARSE>(dq, st, gv, act && node >= gv.nseg, node, hi - pos, lev);
            }
            if (act) pos = hi;
        }
    };
    if constexpr (SPARSE) {  // no ring: each lane walks its own items
        for (uint32_t it = threadIdx.x; it < items; it += BLOCK) {
            uint32_t r, p0, p1;
            if (!run_item(sp, lt, f, lseg, it, &r, &p0, &p1)) continue;
            uint32_t j = load_global(rl.skip + uint64_t(r) * rl.chunks + p0 / kRunSkipCells);
            uint64_t v[kRunBatch];
#pragma unroll
            for (int q = 0; q < kRunBatch; ++q) v[q] = load_global(rl.runs + min(j + q, top));
            uint32_t pos = p0;
            consume(v, pos, p1);
            while (pos < p1) {  // segments that cross more runs
                j += kRunBatch;
                uint64_t w[kRunBatch];
#pragma unroll
                for (int q = 0; q < kRunBatch; ++q) w[q] = load_global(rl.runs + min(j + q, top));
                consume(w, pos, p1);
            }
        }
        return;
    }
    for (uint32_t b0 = uni(threadIdx.x - lane); b0 < items; b0 += BLOCK) {
        const uint32_t it = b0 + lane;
        uint32_t r, p0 = 0, p1 = 0, j = 0;
        if (!(it < items && run_item(sp, lt, f, lseg, it, &r, &p0, &p1))) p0 = p1 = 0;
        uint64_t v[kRunBatch] = {};
        if (p0 < p1) {
            j = load_global(rl.skip + uint64_t(r) * rl.chunks + p0 / kRunSkipCells);
#pragma unroll
            for (int q = 0; q < kRunBatch; ++q) v[q] = load_global(rl.runs + min(j + q, top));
        }
        uint32_t pos = p0;
        consume(v, pos, p1);
        while (__builtin_amdgcn_ballot_w64(pos < p1) != 0) {  // segments that cross more runs
            uint64_t w[kRunBatch] = {};
            if (pos < p1) {
                j += kRunBatch;
#pragma unroll
                for (int q = 0; q < kRunBatch; ++q) w[q] = load_global(rl.runs + min(j + q, top));
            }
            consume(w, pos, p1);
        }
    }
}

// Scatter: every cube of every slab adds 8^level to its node. Neighbouring
// lanes usually hold the same node (mixtures are spatially coherent), so a run
// of equal nodes in a wave adds its total once. Runs on sources add to an
// integer counter through their two end lanes (start: -a 8^l, end: (b+1) 8^l
// for lanes a..b), which needs no run length; runs on internal nodes take a
// branch that the whole wave skips when no lane needs it, where each start lane
// hands (node, run length, level) to the wave's deferral ring (dense state) or
// scatters run length * 8^level at once (sparse state). Level-0 slabs of the
// 16-bit copy (kind 1) hold two sources per unit (count_pairs).
template <int BLOCK, int UNROLL, bool SPARSE>
__device__ __attribute__((always_inline)) inline void scatter_slabs(
    const Slab *slabs, int n_slabs, const char *__restrict__ maps, const char *__restrict__ maps16,
    const RunLevel *runs, const LevelTable &lt, const QueryState &st, const GraphView &gv, const uint32_t *flags_lds)
{
    constexpr uint32_t kWaves = BLOCK / 64;
    const uint32_t nseg = gv.nseg;
    const uint64_t above = lane_above_mask();
    const uint32_t lane = threadIdx.x & 63;
    // Runs on internal nodes met while streaming the 32-bit levels (dense state) are
    // deferred to a per-wave ring in LDS, (node, run length | level << 7), and resolved
    // 64 at a time, one per lane: resolving one loads the node's (a, b, w) triple (and,
    // at rank 2, its predecessors'), so the load chains of 64 runs are in flight together
    // instead of one chain in nearly every wave step. At most 63 entries wait after a
    // step; the ring holds those plus the 64 a step can add.
    __shared__ uint32_t dq_node[kWaves * (SPARSE ? 1u : kDeferSlots)];
    __shared__ uint16_t dq_code[kWaves * (SPARSE ? 1u : kDeferSlots)];
    DeferRing dq{dq_node, dq_code, uni(threadIdx.x >> 6) * kDeferSlots, 0u, 0u};
    for (int si = 0; si < n_slabs; ++si) {
        const Slab &sp = slabs[si];
        if (uni(*flags_lds) & 1u) return;  // overflowed: the box goes to the retry launch
        if (uni(sp.kind) == 2) {
            scatter_runs<BLOCK, SPARSE>(sp, runs[2 * uni(sp.level) + (uni(sp.axes) & 3u)], lt, st, gv, dq);
            continue;
        }
        const uint64_t base = (uint64_t(uni(uint32_t(sp.base >> 32))) << 32) | uni(uint32_t(sp.base));
        const TileWalk tw = tile_walk(uni(sp.units), uni(sp.e1), uni(sp.e2), uni(sp.s1b), uni(sp.s2b), UNROLL);
        if (!SPARSE && uni(sp.kind) == 1) {
            // level 0: every node is a source; two cubes per unit
            stream_pairs<UNROLL, kWaves>(maps16 + base, tw, uni(sp.e0), uni(sp.odd), uint32_t(si) % kWaves,
                                         [&](uint32_t lo, uint32_t hi) { count_pairs(st.seg_cnt, lo, hi, lane); });
            continue;
        }
        const uint32_t lev = uni(sp.level), lw8 = 3 * lev;
        // a run of lanes [a, b] on one source adds (b + 1 - a) 8^l as -a 8^l at its start lane
        // and (b + 1) 8^l at its end lane (uint32 wrap-around; the counts stay below 2^32)
        const uint32_t w_start = 0u - (lane << lw8), w_end = (lane + 1) << lw8;
        const bool go = stream_slab<UNROLL, kWaves>(
            maps + base, tw, uint32_t(si) % kWaves,
            [&](uint32_t v) {
                if (SPARSE) {
                    uint32_t len;
                    if (run_head(v, above, &len)) scatter_count<SPARSE>(st, gv, v, len << lw8);
                    return;
                }
                // neighbours by DPP wave shifts (lane 0 / lane 63 read 0 and are a start / an end)
                const uint32_t prev = uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x138, 0xF, 0xF, true));
                const uint32_t next = uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x130, 0xF, 0xF, true));
                const bool start = v != prev || lane == 0;
                const bool end = v != next || lane == 63;
                if (v < nseg) {  // a source (kEmpty is not)
                    if (start) atomicAdd(&st.seg_cnt[v], w_start);
                    if (end) atomicAdd(&st.seg_cnt[v], w_end);
                }
                // runs on internal nodes: a branch the wave skips unless a lane needs it
                // (wave masks straight from the vector compares: every lane is active here)
                const bool isint = v - nseg < kEmpty - nseg;
                const uint64_t internal = __builtin_amdgcn_uicmp(v - nseg, kEmpty - nseg, 36 /* ult */);
                if (__builtin_expect(internal != 0, 0)) {
                    const uint64_t put = internal & (__builtin_amdgcn_uicmp(v, prev, 33 /* ne */) | 1u);
                    const uint64_t ends = __builtin_amdgcn_uicmp(v, next, 33 /* ne */) | (1ull << 63);
                    if (start && isint) {
                        // the run ends at the first end lane at or above this one
                        const uint32_t len = uint32_t(__builtin_ctzll(ends >> lane)) + 1u;
                        const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                            uint32_t(put >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(put), 0u));
                        const uint32_t k = dq.wbase + ((dq.tail + below) & (kDeferSlots - 1));
                        dq_node[k] = v;
                        dq_code[k] = uint16_t(len | (lev << 9));
                    }
                    dq.tail += uint32_t(__builtin_popcountll(put));
                    if (dq.tail - dq.head >= 64u) ring_resolve<SPARSE>(dq, st, gv, 64u);
                }
            },
            [&]() { return (uni(*flags_lds) & 1u) != 0; });
        if (!go) return;
    }
    if (!SPARSE && dq.tail != dq.head) ring_resolve<SPARSE>(dq, st, gv, dq.tail - dq.head);
}

// Reverse push through the nodes of rank >= 3 in the table, rank by rank from
// the highest present. All threads of the block must call.
template <int BLOCK, bool SPARSE>
__device__ inline void push_mass(const QueryState &st, const GraphView &gv, const uint32_t *rank_ptr_lds,
                                 uint32_t depth)
{
    const uint32_t nu = ld(st.n_used);
    if (nu == 0 || (ld(st.flags) & 1u)) return;  // uniform
    const uint32_t top_key = ld(st.max_key);
    if (top_key < gv.r2_end) return;  // only sources in the table: nothing to push
    uint32_t r = depth;
    while (r > 3 && rank_ptr_lds[r] > top_key) --r;
    for (; r >= 3; --r) {  // ranks <= 2 never enter the table
        const uint32_t lo_id = rank_ptr_lds[r], hi_id = rank_ptr_lds[r + 1];
        const uint32_t n_now = ld(st.n_used);
        __syncthreads();  // every thread has read n_now before any insert of this rank
        for (uint32_t i = threadIdx.x; i < n_now; i += BLOCK) {
            const uint32_t slot = ld(&st.used[i]);
            const uint32_t key = ld(&st.keys[slot]);
            if (key < lo_id || key >= hi_id) continue;
            const float mh = ld(&st.hi[slot]), ml = ld(&st.lo[slot]);
            const NodeTriple t = gv.nodes[key];
            float ah, al, bh, bl;
            scale_pair(1.0f - t.w, mh, ml, &ah, &al);
            scale_pair(t.w, mh, ml, &bh, &bl);
            route_mass<SPARSE>(st, gv, t.a, ah, al);
            route_mass<SPARSE>(st, gv, t.b, bh, bl);
        }
        __syncthreads();
    }
}

struct QueryArgs {
    LevelTable lt;
    const uint32_t *boxes;
    float *out;                   // dense output [n][S], or nullptr for sparse output
    uint32_t *sp_index;           // sparse output: [n][2] (first entry, entries) per box
    uint32_t *sp_seg;             // sparse output: source of each entry
    float *sp_val;                // sparse output: fraction of each entry
    uint32_t sp_cap;              // entries sp_seg / sp_val hold
    uint32_t *sp_total;           // entries produced (may exceed sp_cap: then the rest are dropped)
    const uint32_t *maps;         // maps then maps_t
    const uint16_t *maps16;       // level 0 as 16-bit IDs (both orientations), if lt.use16
    const RunLevel *runs;         // [2 l + o] row runs of level l along x / y, where lt.runs_mask says
    GraphView gv;
    const uint32_t *rank_ptr;     // [depth + 2]
    uint32_t depth;
    uint32_t n;
    const uint32_t *order;        // query order (batched) or nullptr (identity)
    uint32_t *counters;           // [0] next big-tier box, [1] boxes in list 1, [2] next box of the
                                  // final global tables, [3] next small-tier box, [4] next retry
                                  // box, [5] boxes in list 2, [6] boxes in list 3, [7] next box of
                                  // the mid-size global tables, [8] number of big-tier boxes
    uint32_t table_cap;           // LDS hash slots of this launch
    uint32_t chunk;               // small tier: boxes per dequeue (0: automatic)
    uint32_t g_slots;             // hash slots of each fallback worker's global table
    uint32_t *queues;             // tier work queues: counter of queue j at [j * kQueueStride]
    uint32_t *overflow;           // list 1: boxes whose tier table overflowed
    uint32_t *overflow2;          // list 2: boxes whose retry table overflowed too
    const uint32_t *g_list;       // global-table launches: the boxes they answer,
    uint32_t g_count_idx;         // counters[] entry holding how many,
    uint32_t g_next_idx;          // and the one they dequeue with
    uint32_t *ovf_out;            // where this launch reports overflowed boxes (nullptr: mark NaN)
    uint32_t ovf_out_idx;         // counters[] entry that counts them
    uint32_t stats_tag;           // OR-ed into stats[q][1]: which launch answered the box
    uint32_t *stats;              // optional [n][2]: cubes, table entries (graph nodes) touched
    const uint64_t *lut_ptr;      // mixture lookup table rows: expand instead of push (nullptr: push)
    const uint32_t *lut_seg;
    const float *lut_val;
    const float *lut_err;         // propagated uncertainty of each row entry (uncertainty queries)
    float *out_err;               // [n][S] uncertainty of each fraction, or null (dense output only)
    // fallback global regions (per worker)
    uint32_t *g_keys, *g_cnt, *g_used;
    float *g_hi, *g_lo;
    uint32_t *g_seg_cnt;
    float *g_seg_hi, *g_seg_lo, *g_seg_var;
};

// Mixture lookup expansion (the paper's query through per-node mixtures):
// every graph node in the table adds its mass times its mixture row to the
// sources. Groups of 8 lanes take one node each, lanes over the row's entries.
// Replaces the rank-by-rank push; all threads of the block must call.
template <int BLOCK, bool SPARSE, bool ERR>
__device__ inline void expand_lut(const QueryArgs &A, const QueryState &st)
{
    constexpr uint32_t kGroup = 8;
    const uint32_t nu = ld(st.n_used);
    if (nu == 0 || (ld(st.flags) & 1u)) return;  // uniform
    const uint32_t g = threadIdx.x & (kGroup - 1);
    for (uint32_t i = threadIdx.x / kGroup; i < nu; i += BLOCK / kGroup) {
        const uint32_t slot = ld(&st.used[i]);
        const uint32_t key = ld(&st.keys[slot]);
        if (key < A.gv.r1_end) continue;  // a source (sparse mode); rank-1 nodes never enter the table
        const float mh = ld(&st.hi[slot]), ml = ld(&st.lo[slot]);
        const uint64_t e = A.lut_ptr[key + 1];
        for (uint64_t j = A.lut_ptr[key] + g; j < e; j += kGroup) {
            float ph, pl;
            scale_pair(A.lut_val[j], mh, ml, &ph, &pl);
            add_source_mass<SPARSE>(st, A.lut_seg[j], ph, pl);
            if (ERR) {  // uncertainty: the node's count times its row's, added in quadrature
                const float d = (mh + ml) * A.lut_err[j];
                atomicAdd(&st.seg_var[A.lut_seg[j]], d * d);
            }
        }
    }
}

// LDS bytes of the query kernels' dynamic shared memory.
// Dynamic LDS of the query kernels: per-source arrays (dense mode) and the table,
// then the slab list (6 per level) at a 16-byte aligned offset.
__host__ __device__ inline uint32_t lds_state_bytes(uint32_t nseg, uint32_t cap, bool sparse)
{
    return ((sparse ? cap * 20u : nseg * 12u + cap * 16u) + 15u) & ~15u;
}
__host__ __device__ inline uint32_t lds_bytes(uint32_t nseg, uint32_t cap, bool sparse, uint32_t n_levels,
                                              bool err = false)
{
    return lds_state_bytes(nseg, cap, sparse) + 6u * n_levels * uint32_t(sizeof(Slab)) + (err ? 4u * nseg : 0u);
}

struct QueryShared {
    uint32_t rank_ptr[kMaxSteps + 2];
    int n_slabs;
    uint32_t n_used;
    uint32_t flags;
    uint32_t max_key;
    uint32_t q;
    uint32_t nnz;    // sparse output: entries of this box
    uint32_t base;   // sparse output: first entry of this box
};

// Fraction of voxels of each source of one box, written to the dense row or
// appended to the sparse output. All threads of the block must call.
template <int BLOCK, bool SPARSE, bool ERR>
__device__ inline void write_result(const QueryArgs &A, QueryShared &sh, const QueryState &st, uint32_t q,
                                    bool nonempty, double vol)
{
    const uint32_t nseg = A.gv.nseg;
    if (!SPARSE && !A.out) {
        // per-source arrays, sparse output (the global-table launches): count the box's
        // non-zero sources, reserve their entries with one global atomic, write them
        if (threadIdx.x == 0) sh.nnz = 0;
        __syncthreads();
        // a source got voxels iff any of its three words is non-zero (mass below 256 voxels
        // can sit in the compensation word alone; an untouched source is exactly zero)
        uint32_t mine = 0;
        for (uint32_t s = threadIdx.x; s < nseg; s += BLOCK)
            mine += (ld(&st.seg_cnt[s]) | __float_as_uint(ld(&st.seg_hi[s])) | __float_as_uint(ld(&st.seg_lo[s]))) !=
                    0u;
        if (mine) atomicAdd(&sh.nnz, mine);
        __syncthreads();
        if (threadIdx.x == 0) {
            sh.base = sh.nnz ? atomicAdd(A.sp_total, sh.nnz) : 0u;
            A.sp_index[2 * uint64_t(q)] = sh.base;
            A.sp_index[2 * uint64_t(q) + 1] = sh.nnz;
            sh.nnz = 0;
        }
        __syncthreads();
        for (uint32_t s = threadIdx.x; s < nseg; s += BLOCK) {
            const uint32_t c_int = ld(&st.seg_cnt[s]);
            const float h = ld(&st.seg_hi[s]), l = ld(&st.seg_lo[s]);
            if ((c_int | __float_as_uint(h) | __float_as_uint(l)) == 0u) continue;
            const double c = double(c_int) + double(h) + double(l);
            const uint32_t pos = sh.base + atomicAdd(&sh.nnz, 1u);
            if (pos < A.sp_cap) {
                A.sp_seg[pos] = s;
                A.sp_val[pos] = float(c / vol);
            }
        }
        return;
    }
    if (!SPARSE) {
        float *o = A.out + uint64_t(q) * nseg;
        for (uint32_t s = threadIdx.x; s < nseg; s += BLOCK) {
            const double c = double(ld(&st.seg_cnt[s])) + double(ld(&st.seg_hi[s])) + double(ld(&st.seg_lo[s]));
            o[s] = nonempty ? float(c / vol) : 0.0f;
        }
        if (ERR) {
            float *e = A.out_err + uint64_t(q) * nseg;
            for (uint32_t s = threadIdx.x; s < nseg; s += BLOCK)
                e[s] = nonempty ? float(sqrt(double(ld(&st.seg_var[s]))) / vol) : 0.0f;
        }
        return;
    }
    const uint32_t nu = min(sh.n_used, st.cap);
    if (A.out) {
        float *o = A.out + uint64_t(q) * nseg;
        for (uint32_t s = threadIdx.x; s < nseg; s += BLOCK) o[s] = 0.0f;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < nu; i += BLOCK) {
            const uint32_t slot = ld(&st.used[i]);
            const uint32_t key = ld(&st.keys[slot]);
            if (key >= nseg) continue;
            const double c = double(ld(&st.cnt[slot])) + double(ld(&st.hi[slot])) + double(ld(&st.lo[slot]));
            o[key] = float(c / vol);
        }
        return;
    }
    if (threadIdx.x == 0) sh.nnz = 0;
    __syncthreads();
    uint32_t mine = 0;
    for (uint32_t i = threadIdx.x; i < nu; i += BLOCK) mine += ld(&st.keys[ld(&st.used[i])]) < nseg;
    if (mine) atomicAdd(&sh.nnz, mine);
    __syncthreads();
    if (threadIdx.x == 0) {
        sh.base = sh.nnz ? atomicAdd(A.sp_total, sh.nnz) : 0u;
        A.sp_index[2 * uint64_t(q)] = sh.base;
        A.sp_index[2 * uint64_t(q) + 1] = sh.nnz;
        sh.nnz = 0;
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nu; i += BLOCK) {
        const uint32_t slot = ld(&st.used[i]);
        const uint32_t key = ld(&st.keys[slot]);
        if (key >= nseg) continue;
        const double c = double(ld(&st.cnt[slot])) + double(ld(&st.hi[slot])) + double(ld(&st.lo[slot]));
        const uint32_t pos = sh.base + atomicAdd(&sh.nnz, 1u);
        if (pos < A.sp_cap) {
            A.sp_seg[pos] = key;
            A.sp_val[pos] = float(c / vol);
        }
    }
}

// Marks a box that no table could hold: NaN row (dense) or a NaN entry count.
template <int BLOCK>
__device__ inline void write_failure(const QueryArgs &A, uint32_t q)
{
    if (A.out) {
        float *o = A.out + uint64_t(q) * A.gv.nseg;
        for (uint32_t s = threadIdx.x; s < A.gv.nseg; s += BLOCK) o[s] = __builtin_nanf("");
    } else if (threadIdx.x == 0) {
        A.sp_index[2 * uint64_t(q)] = 0xFFFFFFFFu;
        A.sp_index[2 * uint64_t(q) + 1] = 0xFFFFFFFFu;
    }
}

// One query, by the whole block. `st` must be clean (keys empty, values 0).
// ERR: lookup-table expansion that also accumulates uncertainties (dense output).
// (always inlined: each query kernel is one function, whatever the inliner's size limit)
template <int BLOCK, int UNROLL, bool SPARSE, bool ERR>
__device__ __attribute__((always_inline)) inline void run_query(const QueryArgs &A, QueryShared &sh,
                                                                const QueryState &st, uint32_t q,
                                                                bool report_overflow)
{
    uint32_t lo[3], hi[3];
    const bool nonempty = clip_box(A.boxes + 6 * uint64_t(q), A.lt, lo, hi);
    if (threadIdx.x == 0) {
        sh.n_used = 0;
        sh.flags = 0;
        sh.max_key = 0;
        sh.n_slabs = 0;
    }
    __syncthreads();
    if (nonempty) build_slabs(A.lt, lo, hi, st.slabs, &sh.n_slabs);
    __syncthreads();
    scatter_slabs<BLOCK, UNROLL, SPARSE>(st.slabs, sh.n_slabs, reinterpret_cast<const char *>(A.maps),
                                         reinterpret_cast<const char *>(A.maps16), A.runs, A.lt, st, A.gv,
                                         &sh.flags);
    __syncthreads();
    if (ERR || A.lut_ptr)
        expand_lut<BLOCK, SPARSE, ERR>(A, st);
    else
        push_mass<BLOCK, SPARSE>(st, A.gv, sh.rank_ptr, A.depth);
    __syncthreads();
    const bool overflow = (sh.flags & 1u) != 0;
    if (A.stats && threadIdx.x == 0 && (!overflow || !report_overflow)) {
        uint32_t cubes = 0;
        for (int i = 0; i < sh.n_slabs; ++i) cubes += slab_count(st.slabs[i]);
        A.stats[2 * uint64_t(q)] = cubes;
        // bit 30: answered by the retry launch, bit 31: by the global-table fallback
        A.stats[2 * uint64_t(q) + 1] = sh.n_used | A.stats_tag;
    }
    const uint32_t nseg = A.gv.nseg;
    if (!overflow) {
        const double vol = nonempty ? double(hi[0] - lo[0]) * double(hi[1] - lo[1]) * double(hi[2] - lo[2]) : 0.0;
        write_result<BLOCK, SPARSE, ERR>(A, sh, st, q, nonempty, vol);
    } else if (report_overflow) {
        if (threadIdx.x == 0) {
            const uint32_t k = atomicAdd(&A.counters[A.ovf_out_idx], 1u);
            A.ovf_out[k] = q;
        }
    } else {
        write_failure<BLOCK>(A, q);  // even the per-worker global table overflowed
    }
    __syncthreads();
    // restore a clean state for the next query
    const uint32_t nu = min(sh.n_used, st.cap);
    for (uint32_t i = threadIdx.x; i < nu; i += BLOCK) {
        const uint32_t slot = ld(&st.used[i]);
        st.keys[slot] = kEmpty;
        st.hi[slot] = 0.f;
        st.lo[slot] = 0.f;
        if (SPARSE) st.cnt[slot] = 0;
    }
    if (!SPARSE)
        for (uint32_t s = threadIdx.x; s < nseg; s += BLOCK) {
            st.seg_cnt[s] = 0;
            st.seg_hi[s] = 0.f;
            st.seg_lo[s] = 0.f;
            if (ERR) st.seg_var[s] = 0.f;
        }
    __syncthreads();
}

template <int BLOCK>
__device__ inline void load_rank_ptr(const QueryArgs &A, QueryShared &sh)
{
    for (uint32_t i = threadIdx.x; i < A.depth + 2; i += BLOCK) sh.rank_ptr[i] = A.rank_ptr[i];
}

template <bool SPARSE>
__device__ inline QueryState lds_state(char *dyn, QueryShared &sh, uint32_t nseg, uint32_t cap, uint32_t n_levels,
                                      bool err)
{
    QueryState st;
    st.slabs = reinterpret_cast<Slab *>(dyn + lds_state_bytes(nseg, cap, SPARSE));
    st.seg_var = err ? reinterpret_cast<float *>(dyn + lds_state_bytes(nseg, cap, SPARSE) +
                                                 6u * n_levels * uint32_t(sizeof(Slab)))
                     : nullptr;
    uint32_t *t = reinterpret_cast<uint32_t *>(dyn);
    if (SPARSE) {
        st.seg_cnt = nullptr;
        st.seg_hi = st.seg_lo = nullptr;
        st.cnt = t + 4 * cap;
    } else {
        st.seg_cnt = t;
        st.seg_hi = reinterpret_cast<float *>(t + nseg);
        st.seg_lo = reinterpret_cast<float *>(t + 2 * nseg);
        t += 3 * nseg;
        st.cnt = nullptr;
    }
    st.keys = t;
    st.hi = reinterpret_cast<float *>(t + cap);
    st.lo = reinterpret_cast<float *>(t + 2 * cap);
    st.used = t + 3 * cap;
    st.cap = cap;
    st.limit = cap / 4 * 3;
    st.n_used = &sh.n_used;
    st.flags = &sh.flags;
    st.max_key = &sh.max_key;
    return st;
}

template <int BLOCK, bool SPARSE, bool ERR>
__device__ inline void clear_lds_state(const QueryState &st, uint32_t nseg)
{
    for (uint32_t i = threadIdx.x; i < st.cap; i += BLOCK) {
        st.keys[i] = kEmpty;
        st.hi[i] = 0.f;
        st.lo[i] = 0.f;
        if (SPARSE) st.cnt[i] = 0;
    }
    if (!SPARSE)
        for (uint32_t s = threadIdx.x; s < nseg; s += BLOCK) {
            st.seg_cnt[s] = 0;
            st.seg_hi[s] = 0.f;
            st.seg_lo[s] = 0.f;
            if (ERR) st.seg_var[s] = 0.f;
        }
}

// Plain: one block per query in input order, state in LDS.
template <bool SPARSE>
__global__ __launch_bounds__(kBlock) void query_plain_kernel(QueryArgs A)
{
    extern __shared__ __align__(16) char dyn[];
    __shared__ QueryShared sh;
    const QueryState st = lds_state<SPARSE>(dyn, sh, A.gv.nseg, A.table_cap, A.lt.n_levels, false);
    load_rank_ptr<kBlock>(A, sh);
    clear_lds_state<kBlock, SPARSE, false>(st, A.gv.nseg);
    __syncthreads();
    run_query<kBlock, kUnroll, SPARSE, false>(A, sh, st, blockIdx.x, A.ovf_out != nullptr);
}

// Batched tiers: persistent blocks take queries from the largest-first order.
// BIG: positions [0, counters[8]); otherwise [counters[8], n).
template <int BLOCK, bool BIG, int UNROLL, bool SPARSE, bool ERR>
// Six waves per SIMD (24 per CU: 1536 threads): the register budget the kernel is
// tuned for (at most 80 VGPRs), so that the memory latency of the streamed node
// IDs stays hidden.
__global__ __launch_bounds__(BLOCK, 1536 / BLOCK) void query_tier_kernel(QueryArgs A)
{
    extern __shared__ __align__(16) char dyn[];
    __shared__ QueryShared sh;
    const QueryState st = lds_state<SPARSE>(dyn, sh, A.gv.nseg, A.table_cap, A.lt.n_levels, ERR);
    load_rank_ptr<BLOCK>(A, sh);
    clear_lds_state<BLOCK, SPARSE, ERR>(st, A.gv.nseg);
    const uint32_t split = ld(&A.counters[8]);
    const uint32_t begin = BIG ? 0u : split, end = BIG ? split : A.n;
    // Work queues: a single counter that every workgroup increments serialises
    // at one L2 atomic unit (about 12 ns per box), so the tier's positions of
    // the largest-first order are dealt to kQueues interleaved queues (queue j:
    // positions begin + j, begin + j + kQueues, ...), each with its own counter
    // on its own 256-byte line; workgroup b serves queue b mod kQueues. Each
    // queue is still largest-first. A dequeue takes `chunk` positions (small
    // tier only; 1 by default).
    // (fewer queues when the grid is smaller, so that every queue has a workgroup)
    const uint32_t nq = min(kQueues, gridDim.x);
    const uint32_t qn = blockIdx.x % nq;
    uint32_t *const qc = A.queues + qn * kQueueStride + (BIG ? 0u : 16u);
    const uint32_t chunk = BIG ? 1u : (A.chunk ? A.chunk : 1u);
    for (;;) {
        if (threadIdx.x == 0) sh.q = atomicAdd(qc, chunk);
        __syncthreads();
        const uint32_t i0 = sh.q;
        if (i0 >= end) break;  // uniform; keeps begin + qn + i0 * nq below 2^32
        const uint32_t k0 = begin + qn + i0 * nq;
        if (k0 >= end) break;  // uniform
        // run_query ends with a barrier, so thread 0 rewrites sh.q only after every thread read it
        for (uint32_t i = 0; i < chunk; ++i) {
            const uint32_t k = k0 + i * nq;
            if (k >= end) break;
            run_query<BLOCK, UNROLL, SPARSE, ERR>(A, sh, st, A.order[k], A.ovf_out != nullptr);
        }
    }
}

// Retry of boxes whose tier table overflowed (list 1), with a larger LDS table;
// what overflows again goes to list 2.
template <int BLOCK, int UNROLL, bool SPARSE, bool ERR>
__global__ __launch_bounds__(BLOCK) void query_retry_kernel(QueryArgs A)
{
    extern __shared__ __align__(16) char dyn[];
    __shared__ QueryShared sh;
    const QueryState st = lds_state<SPARSE>(dyn, sh, A.gv.nseg, A.table_cap, A.lt.n_levels, ERR);
    load_rank_ptr<BLOCK>(A, sh);
    clear_lds_state<BLOCK, SPARSE, ERR>(st, A.gv.nseg);
    const uint32_t n_list = ld(&A.counters[1]);
    for (;;) {
        if (threadIdx.x == 0) sh.q = atomicAdd(&A.counters[4], 1u);
        __syncthreads();
        const uint32_t k = sh.q;
        if (k >= n_list) break;  // uniform
        run_query<BLOCK, UNROLL, SPARSE, ERR>(A, sh, st, A.overflow[k], true);
    }
}

// Boxes that overflowed every LDS table, answered with per-worker tables and
// source arrays in the workspace (global memory): first by many workers with
// mid-size tables (list 2; what overflows those goes to list 3), then by a few
// workers whose tables hold every node of the graph (list 3, or list 2 when
// the graph is small enough for those tables alone). Sources always have
// per-worker arrays here (dense state, whatever the output): a cube run on a
// source is one global atomic add without a returned value, where a table
// entry would take a probe round trip.
// Boxes that overflowed every LDS table, in per-worker global-memory tables (node
// table and per-source arrays): each workgroup takes boxes from list A.g_list.
template <bool ERR>
__global__ __launch_bounds__(kBlock) void query_fallback_kernel(QueryArgs A)
{
    extern __shared__ __align__(16) char dyn[];
    __shared__ QueryShared sh;
    QueryState st;
    const uint64_t w = blockIdx.x;
    const uint64_t gs = A.g_slots;
    st.keys = A.g_keys + w * gs;
    st.cnt = A.g_cnt + w * gs;
    st.hi = A.g_hi + w * gs;
    st.lo = A.g_lo + w * gs;
    st.used = A.g_used + w * gs;
    st.cap = A.g_slots;
    st.slabs = reinterpret_cast<Slab *>(dyn);  // the only dynamic LDS of this kernel
    st.limit = st.cap / 4 * 3;
    st.n_used = &sh.n_used;
    st.flags = &sh.flags;
    st.max_key = &sh.max_key;
    st.seg_cnt = A.g_seg_cnt + w * A.gv.nseg;
    st.seg_hi = A.g_seg_hi + w * A.gv.nseg;
    st.seg_lo = A.g_seg_lo + w * A.gv.nseg;
    st.seg_var = ERR ? A.g_seg_var + w * A.gv.nseg : nullptr;
    load_rank_ptr<kBlock>(A, sh);
    __syncthreads();
    const uint32_t n_over = ld(&A.counters[A.g_count_idx]);
    for (;;) {
        if (threadIdx.x == 0) sh.q = atomicAdd(&A.counters[A.g_next_idx], 1u);
        __syncthreads();
        const uint32_t k = sh.q;
        if (k >= n_over) break;  // uniform
        run_query<kBlock, kUnroll, false, ERR>(A, sh, st, A.g_list[k], A.ovf_out != nullptr);
    }
}

// Per-block histogram of 32 buckets, merged with one global atomic per
// non-empty bucket (instead of one contended atomic per box). Every thread of
// the block must call it.
__device__ inline void block_histogram_add(uint32_t bkt, uint32_t *bucket_count)
{
    __shared__ uint32_t h[32];
    if (threadIdx.x < 32) h[threadIdx.x] = 0;
    __syncthreads();
    if (bkt < 32) atomicAdd(&h[bkt], 1u);
    __syncthreads();
    if (threadIdx.x < 32 && h[threadIdx.x]) atomicAdd(&bucket_count[threadIdx.x], h[threadIdx.x]);
}

// Per-query work estimate (cubes) and log2 bucket for the largest-first order.
__global__ void query_size_kernel(LevelTable lt, const uint32_t *boxes, uint32_t n, uint32_t *bucket_of,
                                  uint32_t *bucket_count)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t lo[3], hi[3];
    uint64_t cubes = 0;
    if (q < n && clip_box(boxes + 6 * uint64_t(q), lt, lo, hi)) {
        for (uint32_t l = 0; l < lt.n_levels; ++l) {
            uint64_t outer = 1, inner = 1;
            for (int d = 0; d < 3; ++d) {
                const uint64_t one = uint64_t(1) << l;
                const uint64_t a = (uint64_t(lo[d]) + one - 1) >> l, b = hi[d] >> l;
                const uint64_t pa = (uint64_t(lo[d]) + 2 * one - 1) >> (l + 1), pb = hi[d] >> (l + 1);
                outer *= b > a ? b - a : 0;
                inner *= pb > pa ? 2 * (pb - pa) : 0;
            }
            cubes += outer - inner;
        }
    }
    // 32 buckets, largest work first: bucket 0 holds >= 2^31 cubes
    const uint32_t lg = cubes ? 63 - __clzll(cubes) : 0;
    const uint32_t bkt = q < n ? 31 - min(lg, 31u) : 32u;
    if (q < n) bucket_of[q] = bkt;
    block_histogram_add(bkt, bucket_count);  // every thread, one call site: the barriers match
}

__global__ void query_order_kernel(const uint32_t *bucket_of, uint32_t n, uint32_t *bucket_count, uint32_t *order)
{
    // bucket_count[32 + b] holds, on entry, the first free position of bucket b;
    // each block reserves one range per bucket and ranks its boxes inside it
    __shared__ uint32_t h[32], base[32];
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (threadIdx.x < 32) h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t bkt = q < n ? bucket_of[q] : 32u;
    const uint32_t local = bkt < 32 ? atomicAdd(&h[bkt], 1u) : 0u;
    __syncthreads();
    if (threadIdx.x < 32 && h[threadIdx.x]) base[threadIdx.x] = atomicAdd(&bucket_count[32 + threadIdx.x], h[threadIdx.x]);
    __syncthreads();
    if (bkt < 32) order[base[bkt] + local] = q;
}

__global__ void bucket_scan_kernel(uint32_t *bucket_count, uint32_t *counters)
{
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int b = 0; b < 32; ++b) {
            if (b == 31 - int(kBigLog2) + 1) counters[8] = acc;  // boxes of >= 2^kBigLog2 cubes come first
            bucket_count[32 + b] = acc;
            acc += bucket_count[b];
        }
    }
}

__global__ void reset_counters_kernel(uint32_t *c, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0;
}

// ---------------------------------------------------------------- naive scan

struct NaiveArgs {
    LevelTable lt;
    const uint32_t *boxes;
    float *out;
    const uint32_t *map0;
    const uint16_t *map16;        // 16-bit level 0 (x-fastest, row pitch lt.pitch_x), if lt.use16
    uint32_t nseg;
    uint32_t n;
};

// Naive range query: every level-0 voxel of the box is read and counted
// (same wave-level run merging and unconditional loads as the graph path).
template <int UNROLL>
__global__ __launch_bounds__(kBlock) void naive_kernel(NaiveArgs A)
{
    extern __shared__ __align__(16) char dyn[];
    uint32_t *cnt = reinterpret_cast<uint32_t *>(dyn);
    const uint32_t q = blockIdx.x;
    for (uint32_t s = threadIdx.x; s < A.nseg; s += kBlock) cnt[s] = 0;
    uint32_t lo[3], hi[3];
    const bool nonempty = clip_box(A.boxes + 6 * uint64_t(q), A.lt, lo, hi);
    __syncthreads();
    if (nonempty) {
        uint64_t base;
        uint32_t odd;
        const TileWalk tw = naive_walk(A.lt, lo, hi, A.lt.use16 != 0, UNROLL, &base, &odd);
        const uint32_t lane = threadIdx.x & 63;
        if (A.lt.use16) {
            stream_pairs<UNROLL, kBlock / 64>(reinterpret_cast<const char *>(A.map16) + base, tw, hi[0] - lo[0], odd,
                                              0u, [&](uint32_t a, uint32_t b) { count_pairs(cnt, a, b, lane); });
        } else {
            // runs of equal IDs: -start lane at the start, end lane + 1 at the end (see scatter_slabs)
            const uint32_t w_start = 0u - lane, w_end = lane + 1;
            stream_slab<UNROLL, kBlock / 64>(
                reinterpret_cast<const char *>(A.map0) + base, tw, 0u,
                [&](uint32_t v) {
                    const uint32_t prev = uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x138, 0xF, 0xF, true));
                    const uint32_t next = uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x130, 0xF, 0xF, true));
                    if (v != kEmpty) {
                        if (v != prev || lane == 0) atomicAdd(&cnt[v], w_start);
                        if (v != next || lane == 63) atomicAdd(&cnt[v], w_end);
                    }
                },
                []() { return false; });
        }
    }
    __syncthreads();
    const double vol = nonempty ? double(hi[0] - lo[0]) * double(hi[1] - lo[1]) * double(hi[2] - lo[2]) : 0.0;
    float *o = A.out + uint64_t(q) * A.nseg;
    for (uint32_t s = threadIdx.x; s < A.nseg; s += kBlock) o[s] = nonempty ? float(double(cnt[s]) / vol) : 0.0f;
}

// ---------------------------------------------------------------- footprint (test view)

__global__ __launch_bounds__(kBlock) void footprint_kernel(LevelTable lt, const uint32_t *boxes, uint32_t n,
                                                           const uint32_t *maps, uint32_t *level_counts,
                                                           uint32_t *cubes, uint32_t cap, uint32_t *count)
{
    __shared__ Slab slabs[kMaxSlabs];
    __shared__ int n_slabs;
    __shared__ uint32_t per_level[MG_MAX_LEVELS];
    const uint32_t q = blockIdx.x;
    if (threadIdx.x == 0) n_slabs = 0;
    if (threadIdx.x < MG_MAX_LEVELS) per_level[threadIdx.x] = 0;
    uint32_t lo[3], hi[3];
    const bool nonempty = clip_box(boxes + 6 * uint64_t(q), lt, lo, hi);
    __syncthreads();
    if (nonempty) build_slabs(lt, lo, hi, slabs, &n_slabs);
    __syncthreads();
    for (int si = 0; si < n_slabs; ++si) {
        const Slab sl = slabs[si];
        if (threadIdx.x == 0) atomicAdd(&per_level[sl.level], slab_count(sl));
        if (!cubes) continue;
        for (uint32_t r = threadIdx.x; r < slab_count(sl); r += kBlock) {
            const uint32_t i0 = r % sl.e0, i1 = (r / sl.e0) % sl.e1, i2 = r / (sl.e0 * sl.e1);
            uint32_t x, y, z;
            slab_coords(sl, i0, i1, i2, &x, &y, &z);
            // kind-0 slab (the table is built without the 16-bit copy): 4-byte units
            const uint32_t node = maps[sl.base / 4 + i0 + uint64_t(i1) * (sl.s1b / 4) + uint64_t(i2) * (sl.s2b / 4)];
            const uint32_t k = atomicAdd(count, 1u);
            if (k < cap) {
                uint32_t *c = cubes + 6 * uint64_t(k);
                c[0] = q, c[1] = sl.level, c[2] = x, c[3] = y, c[4] = z, c[5] = node;
            }
        }
    }
    __syncthreads();
    for (uint32_t l = threadIdx.x; l < lt.n_levels; l += kBlock) level_counts[uint64_t(q) * lt.n_levels + l] = per_level[l];
}

// ---------------------------------------------------------------- sparse-output sizing

// Upper bound on the non-zero segments of each box (sizes the sparse output).
// The clipped box lies inside the cells it touches at any level; at the finest
// level where it touches at most 64 cells, one lane per cell reads the cell's
// node, and the bound is the sum of mixlen over the distinct nodes, capped by
// the source count and the box volume. That needs every finer cube's mixture
// to lie inside its enclosing cell's, which holds for exact weights; graphs
// with quantized (merged) weights get the source count and volume cap only.
// One wave per box.
__global__ __launch_bounds__(kBlock) void nnz_bound_kernel(LevelTable lt, const uint32_t *boxes, uint32_t n,
                                                           const uint32_t *__restrict__ maps,
                                                           const uint32_t *__restrict__ mixlen, uint32_t nseg,
                                                           uint32_t exact, uint32_t *bound)
{
    const uint32_t q = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63;
    if (q >= n) return;  // whole waves leave together
    uint32_t lo[3], hi[3];
    if (!clip_box(boxes + 6 * uint64_t(q), lt, lo, hi)) {
        if (lane == 0) bound[q] = 0;
        return;
    }
    // cells touched at level `lane` (levels past the last count as too many)
    uint64_t cells = ~uint64_t(0);
    if (lane < lt.n_levels) {
        cells = 1;
        for (int d = 0; d < 3; ++d) cells *= uint64_t(((hi[d] - 1) >> lane) - (lo[d] >> lane) + 1);
    }
    const uint64_t fits = __ballot(cells <= 64);  // the top level (one cell) always fits
    const uint32_t l = uint32_t(__builtin_ctzll(fits));
    uint32_t c0[3], ext[3];
    for (int d = 0; d < 3; ++d) {
        c0[d] = lo[d] >> l;
        ext[d] = ((hi[d] - 1) >> l) - c0[d] + 1;
    }
    const uint32_t ncell = ext[0] * ext[1] * ext[2];
    uint32_t node = kEmpty, m = 0;
    if (lane < ncell) {
        const uint32_t x = c0[0] + lane % ext[0], y = c0[1] + (lane / ext[0]) % ext[1],
                       z = c0[2] + lane / (ext[0] * ext[1]);
        node = maps[lt.off[l] + x + uint64_t(lt.dims[l][0]) * (y + uint64_t(lt.dims[l][1]) * z)];
        m = mixlen[node];
    }
    // count each distinct node once: drop a lane whose node a lower lane holds
    bool dup = false;
    for (uint32_t j = 0; j < ncell; ++j) {
        const uint32_t v = uint32_t(__shfl(int(node), int(j), 64));
        dup = dup || (j < lane && v == node);
    }
    uint32_t sum = dup ? 0u : m;
    for (int off = 32; off > 0; off >>= 1) sum += uint32_t(__shfl_down(int(sum), off, 64));
    if (lane == 0) {
        const uint64_t vol = uint64_t(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
        bound[q] = uint32_t(std::min<uint64_t>(std::min<uint64_t>(exact ? sum : nseg, nseg), vol));
    }
}

// ---------------------------------------------------------------- TF propagation

// A source's colour under transfer function t: its RGBA8 entry scaled to [0, 1],
// each channel one rounded product (never contracted into a later subtraction, so
// a step that reads it here computes exactly what it computes from the stored value).
__device__ inline float4 tf_source_colour(const uchar4 *tf, uint32_t nseg, uint32_t t, uint32_t src)
{
#pragma clang fp contract(off)
    const uchar4 c = tf[uint64_t(t) * nseg + src];
    const float k = 1.0f / 255.0f;
    return make_float4(float(c.x) * k, float(c.y) * k, float(c.z) * k, float(c.w) * k);
}

// A node's colour from its predecessors' colours va, vb and its weight w: one
// fma per channel, v_a + w (v_b - v_a) (every thread that computes a node's
// colour evaluates exactly this, so a value rebuilt elsewhere is bit-identical).
__device__ inline float4 tf_lerp(float w, float4 va, float4 vb)
{
#pragma clang fp contract(off)
    float4 r;
    r.x = fmaf(w, vb.x - va.x, va.x);
    r.y = fmaf(w, vb.y - va.y, va.y);
    r.z = fmaf(w, vb.z - va.z, va.z);
    r.w = fmaf(w, vb.w - va.w, va.w);
    return r;
}

// The entry of position i of a propagation order: with RANKS the nodes in ID
// order (IDs are sorted by rank, so a rank is a contiguous ID range and node i's
// triple is nodes[i]); else the deferred step schedule's entry sched[i].
template <bool RANKS>
__device__ inline SchedNode tf_entry(const NodeTriple *__restrict__ nodes, const SchedNode *__restrict__ sched,
                                     uint32_t i)
{
    if (RANKS) {
        const NodeTriple t = nodes[i];
        return SchedNode{t.a, t.b, t.w, i};
    }
    return sched[i];
}

// One step of the order (a rank, or a step of the deferred schedule): thread
// (x, y) computes the node at position lo_i + x for the transfer functions
// P y .. P y + P - 1 (grid.y = ceil(T / P)): it loads the node's entry and both
// predecessors' colours in all P planes before it stores any, so 2 P gathers
// per thread are in flight together. Lanes of a wave take consecutive entries
// (coalesced entry reads and, nodes being numbered by rank, contiguous stores).
// FIRST: the first launch: the nodes of the first step (every predecessor a
// source) and, in rank order, those of rank 2 too (every predecessor a source or
// a rank-1 node). It reads source colours from the transfer functions
// themselves and rebuilds a rank-1 predecessor's colour from that node's own two
// sources by the same expression the rank-1 node's thread evaluates (so bit for
// bit the value that thread stores), instead of waiting for it in a launch of
// its own; threads x >= hi_i - lo_i write the sources' own colours (the same
// values), so the frame needs no separate source pass.
template <int P, bool FIRST, bool RANKS>
__global__ void tf_step_kernel(const NodeTriple *__restrict__ nodes, const SchedNode *__restrict__ sched,
                               uint32_t lo_i, uint32_t hi_i, uint32_t n_nodes, uint32_t T,
                               const uchar4 *__restrict__ tf, uint32_t nseg, float4 *out)
{
#pragma clang fp contract(off)
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t p0 = blockIdx.y * P;
    const uint32_t n_step = hi_i - lo_i;
    if (x >= n_step) {
        if (!FIRST || x - n_step >= nseg) return;
        const uint32_t src = x - n_step;
#pragma unroll
        for (int p = 0; p < P; ++p)
            if (P == 1 || p0 + p < T) out[uint64_t(p0 + p) * n_nodes + src] = tf_source_colour(tf, nseg, p0 + p, src);
        return;
    }
    const SchedNode t = tf_entry<RANKS>(nodes, sched, lo_i + x);
    NodeTriple ta{0u, 0u, 0.0f}, tb{0u, 0u, 0.0f};  // a rank-1 predecessor's own triple
    if (FIRST) {
        if (t.a >= nseg) ta = nodes[t.a];
        if (t.b >= nseg) tb = nodes[t.b];
    }
    float4 va[P], vb[P];
#pragma unroll
    for (int p = 0; p < P; ++p)
        if (P == 1 || p0 + p < T) {
            if (FIRST) {
                va[p] = t.a < nseg ? tf_source_colour(tf, nseg, p0 + p, t.a)
                                   : tf_lerp(ta.w, tf_source_colour(tf, nseg, p0 + p, ta.a),
                                             tf_source_colour(tf, nseg, p0 + p, ta.b));
                vb[p] = t.b < nseg ? tf_source_colour(tf, nseg, p0 + p, t.b)
                                   : tf_lerp(tb.w, tf_source_colour(tf, nseg, p0 + p, tb.a),
                                             tf_source_colour(tf, nseg, p0 + p, tb.b));
            } else {
                const float4 *o = out + uint64_t(p0 + p) * n_nodes;
                va[p] = o[t.a];
                vb[p] = o[t.b];
            }
        }
#pragma unroll
    for (int p = 0; p < P; ++p)
        if (P == 1 || p0 + p < T) out[uint64_t(p0 + p) * n_nodes + t.id] = tf_lerp(t.w, va[p], vb[p]);
}

// The last steps of the schedule when each is small (at most kTfTailPairs node x
// transfer-function pairs): one workgroup runs them in order, a block barrier
// between steps (all its waves share one CU and its L1, so the stores of a step
// are visible to the loads of the next), instead of one launch per step.
struct TfTail {
    uint32_t n_steps;
    uint32_t lo[kTfTailSteps + 1];  // step k: schedule entries lo[k] .. lo[k + 1]
};

template <bool RANKS>
__global__ __launch_bounds__(kTfTailBlock) void tf_tail_kernel(const NodeTriple *__restrict__ nodes,
                                                               const SchedNode *__restrict__ sched, TfTail tail,
                                                               uint32_t n_nodes, uint32_t T, float4 *out)
{
    for (uint32_t k = 0; k < tail.n_steps; ++k) {
        const uint32_t lo = tail.lo[k], n = tail.lo[k + 1] - lo;
        for (uint32_t j = threadIdx.x; j < n * T; j += kTfTailBlock) {  // plane-major: lanes take consecutive nodes
            const uint32_t t = j / n;
            const SchedNode e = tf_entry<RANKS>(nodes, sched, lo + j % n);
            float4 *o = out + uint64_t(t) * n_nodes;
            o[e.id] = tf_lerp(e.w, o[e.a], o[e.b]);
        }
        __syncthreads();
    }
}

// Mean colour of a box under one propagated palette: every footprint cube adds
// its 8^l voxels times the palette entry of its node, divided by the box
// volume. One workgroup of kColourBlock threads per box; sums in fp64. Boxes
// whose palette index is kEmpty get zeros. The level table carries no 16-bit
// copy and no row runs, so every slab is read as 32-bit node IDs. A thread
// walks its cubes of a slab kColourBlock apart, its (fast, mid, slow) offsets
// advanced by carries rather than divided out, kColourUnroll node IDs and then
// their palette entries in flight at a time.
constexpr int kColourBlock = 1024;
constexpr int kColourUnroll = 8;
__global__ __launch_bounds__(kColourBlock) void box_colour_kernel(LevelTable lt, const uint32_t *boxes, uint32_t n,
                                                                  const uint32_t *__restrict__ maps,
                                                                  const float4 *__restrict__ palette, uint32_t T,
                                                                  uint32_t n_nodes, const uint32_t *pal_of_box,
                                                                  float4 *out)
{
    __shared__ Slab slabs[kMaxSlabs];
    __shared__ int n_slabs;
    __shared__ double part[kColourBlock / 64][4];
    const uint32_t q = blockIdx.x;
    const uint32_t t = pal_of_box[q];
    uint32_t lo[3], hi[3];
    const bool nonempty = clip_box(boxes + 6 * uint64_t(q), lt, lo, hi) && t < T;
    if (threadIdx.x == 0) n_slabs = 0;
    __syncthreads();
    if (nonempty) build_slabs(lt, lo, hi, slabs, &n_slabs);
    __syncthreads();
    const float4 *pal = palette + uint64_t(t < T ? t : 0) * n_nodes;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int si = 0; si < n_slabs; ++si) {
        const Slab sl = slabs[si];
        const double w = double(uint64_t(1) << (3 * sl.level));
        const uint32_t c = slab_count(sl);
        if (threadIdx.x >= c) continue;
        // this thread's first cube, and the step of kColourBlock cubes, as (fast, mid, slow) offsets
        const uint32_t e01 = sl.e0 * sl.e1;
        uint32_t i0 = threadIdx.x % sl.e0, i1 = (threadIdx.x / sl.e0) % sl.e1, i2 = threadIdx.x / e01;
        const uint32_t d0 = uint32_t(kColourBlock) % sl.e0, d1 = (uint32_t(kColourBlock) / sl.e0) % sl.e1,
                       d2 = uint32_t(kColourBlock) / e01;
        const uint32_t *slab = maps + sl.base / 4;
        const uint64_t s1 = sl.s1b / 4, s2 = sl.s2b / 4;
        for (uint32_t r = threadIdx.x; r < c; r += kColourBlock * kColourUnroll) {
            uint32_t node[kColourUnroll];
#pragma unroll
            for (int u = 0; u < kColourUnroll; ++u) {
                // cube r + u kColourBlock, if inside the slab
                node[u] = r + uint32_t(u) * kColourBlock < c ? slab[i0 + i1 * s1 + i2 * s2] : kEmpty;
                i0 += d0;
                const uint32_t c0 = i0 >= sl.e0 ? 1u : 0u;
                i0 -= c0 ? sl.e0 : 0u;
                i1 += d1 + c0;
                const uint32_t c1 = i1 >= sl.e1 ? 1u : 0u;
                i1 -= c1 ? sl.e1 : 0u;
                i2 += d2 + c1;
            }
            float4 v[kColourUnroll];
#pragma unroll
            for (int u = 0; u < kColourUnroll; ++u)
                v[u] = node[u] != kEmpty ? pal[node[u]] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int u = 0; u < kColourUnroll; ++u)
                acc[0] += w * v[u].x, acc[1] += w * v[u].y, acc[2] += w * v[u].z, acc[3] += w * v[u].w;
        }
    }
    for (int k = 0; k < 4; ++k)
        for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_down(acc[k], off, 64);
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 4; ++k) part[threadIdx.x >> 6][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        for (int wv = 0; wv < kColourBlock / 64; ++wv)
            for (int k = 0; k < 4; ++k) s[k] += part[wv][k];
        const double vol = nonempty ? double(hi[0] - lo[0]) * double(hi[1] - lo[1]) * double(hi[2] - lo[2]) : 1.0;
        out[q] = nonempty ? make_float4(float(s[0] / vol), float(s[1] / vol), float(s[2] / vol), float(s[3] / vol))
                          : make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// ---------------------------------------------------------------- upload helpers

// Palette fetch: the node of each voxel at one level indexes the palette.
__global__ void palette_fetch_kernel(const float4 *__restrict__ palette, uint32_t T, uint32_t n_nodes,
                                     const uint32_t *__restrict__ map, uint32_t X, uint32_t Y, uint32_t Z,
                                     const uint32_t *__restrict__ xyz, uint32_t n, float4 *__restrict__ out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t x = xyz[3 * uint64_t(i)], y = xyz[3 * uint64_t(i) + 1], z = xyz[3 * uint64_t(i) + 2];
    const bool in = x < X && y < Y && z < Z;
    const uint32_t node = in ? map[x + uint64_t(X) * (y + uint64_t(Y) * z)] : 0u;
    for (uint32_t t = 0; t < T; ++t)
        out[uint64_t(t) * n + i] = in ? palette[uint64_t(t) * n_nodes + node] : make_float4(0.f, 0.f, 0.f, 0.f);
}

// The voxel data (A) of a graph stream (Table "bitstream"): per level, voxel by
// voxel (x fastest), the node ID minus i_min(l) in r(l) bits, least significant
// bit first. One thread per voxel: the field is read from the two 32-bit words
// that hold it; level-0 IDs are sources, the others are renumbered by `perm`.
// An ID out of range sets *bad and writes node 0.
struct StreamLevels {
    uint32_t n_levels;
    uint32_t nseg, n_nodes;
    uint64_t off[MG_MAX_LEVELS + 1];     // first voxel of each level
    uint64_t bit[MG_MAX_LEVELS];         // bit of its first field, from the first word
    uint32_t r[MG_MAX_LEVELS], lo[MG_MAX_LEVELS];
};

__global__ void unpack_maps_kernel(StreamLevels sl, const uint32_t *__restrict__ words,
                                   const uint32_t *__restrict__ perm, uint32_t *__restrict__ maps, uint32_t *bad)
{
    const uint64_t total = sl.off[sl.n_levels];
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += stride) {
        uint32_t l = 0;
        while (i >= sl.off[l + 1]) ++l;
        const uint32_t r = sl.r[l];
        const uint64_t b = sl.bit[l] + (i - sl.off[l]) * r;
        const uint64_t w = b >> 5;
        const uint64_t two = (uint64_t(words[w + 1]) << 32) | words[w];
        const uint64_t field = r ? (two >> (b & 31)) & ((uint64_t(1) << r) - 1) : 0;
        const uint64_t id = sl.lo[l] + field;
        const uint64_t limit = l == 0 ? sl.nseg : sl.n_nodes;
        uint32_t node = 0;
        if (id < limit) node = l == 0 ? uint32_t(id) : perm[id];
        else atomicOr(bad, 1u);
        maps[i] = node;
    }
}

// 16-bit copies of level 0: x-fastest with row pitch px, and y-fastest (y + py (z + Z x))
// with row pitch py; padding elements hold 0xFFFF.
__global__ void pack16_kernel(const uint32_t *__restrict__ map0, uint16_t *__restrict__ out, uint32_t X, uint32_t Y,
                              uint32_t Z, uint32_t px, uint32_t py, uint64_t total16, uint64_t total16t)
{
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < total16) {  // x-fastest copy: element i = x + px (y + Y z)
        const uint32_t x = uint32_t(i % px);
        const uint64_t yz = i / px;
        out[i] = x < X ? uint16_t(map0[x + uint64_t(X) * yz]) : uint16_t(0xFFFF);
    }
    if (i < total16t) {  // y-fastest copy: element i = y + py (z + Z x)
        const uint32_t y = uint32_t(i % py);
        const uint64_t zx = i / py;
        const uint32_t z = uint32_t(zx % Z), x = uint32_t(zx / Z);
        out[total16 + i] = y < Y ? uint16_t(map0[x + uint64_t(X) * (y + uint64_t(Y) * z)]) : uint16_t(0xFFFF);
    }
}

__global__ void transpose_level_kernel(const uint32_t *src, uint32_t *dst, uint32_t X, uint32_t Y, uint32_t Z)
{
    // dst[y + Y (z + Z x)] = src[x + X (y + Y z)]
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t total = uint64_t(X) * Y * Z;
    if (i >= total) return;
    const uint32_t x = uint32_t(i % X);
    const uint64_t yz = i / X;
    const uint32_t y = uint32_t(yz % Y), z = uint32_t(yz / Y);
    dst[y + uint64_t(Y) * (z + uint64_t(Z) * x)] = src[i];
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t n, uint32_t v)
{
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Levels, offsets and the 16-bit copy's pitches of a volume (the graph's own
// level table for its dims; the host-side address check builds one from dims).
LevelTable level_table_dims(const uint32_t dims[3])
{
    LevelTable lt;
    std::memset(&lt, 0, sizeof(lt));
    std::vector<uint32_t> ld;
    level_dims(dims, &ld);
    lt.n_levels = uint32_t(ld.size() / 3);
    for (int a = 0; a < 3; ++a) lt.vol[a] = dims[a];
    uint64_t off = 0;
    for (uint32_t l = 0; l < lt.n_levels && l < MG_MAX_LEVELS; ++l) {
        for (int a = 0; a < 3; ++a) lt.dims[l][a] = ld[3 * l + a];
        lt.off[l] = off;
        off += uint64_t(ld[3 * l]) * ld[3 * l + 1] * ld[3 * l + 2];
    }
    lt.total = off;
    lt.pitch_x = dims[0] + (dims[0] & 1u);
    lt.pitch_y = dims[1] + (dims[1] & 1u);
    lt.total16 = uint64_t(lt.pitch_x) * dims[1] * dims[2];
    lt.use16 = 0;  // set per launch where the 16-bit copy is used
    lt.runs_mask = 0, lt.run_min = 0xFFFFFFFFu;  // and where row runs are read
    return lt;
}

LevelTable level_table(const Graph &g) { return level_table_dims(g.dims); }

// ---------------------------------------------------------------- workspace layout

// Per-worker global-memory tables of one global-table launch.
struct GlobalPool {
    uint32_t workers, slots;
    uint32_t *keys, *cnt, *used;
    float *hi, *lo;
    uint32_t *seg_cnt;
    float *seg_hi, *seg_lo, *seg_var;
};

struct Workspace {
    uint32_t *counters;   // 64 u32
    uint32_t *queues;     // kQueues * kQueueStride u32: per-queue counters of the two tiers
    uint32_t *buckets;    // 64 u32
    uint32_t *bucket_of;  // [max_boxes]
    uint32_t *order;      // [max_boxes]
    uint32_t *overflow;   // [max_boxes] list 1: overflowed a tier table
    uint32_t *overflow2;  // [max_boxes] list 2: overflowed the retry table too
    uint32_t *overflow3;  // [max_boxes] list 3: overflowed a mid-size global table too
    GlobalPool fin;       // tables that hold every node of the graph
    GlobalPool mid;       // many workers with mid-size tables (workers 0: none)
    uint64_t bytes;
    uint32_t max_boxes;
};

inline uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

// Global fallback tables: each worker's table holds every node of the graph below
// its 3/4 load limit (a box touches a node at most once), so no box can overflow
// it, with at least 2^16 and at most 2^26 slots; the workers share a budget of
// 128 x 2^16 slots (fewer workers for larger graphs, at least 16).
inline uint32_t fallback_slots(const Graph &g)
{
    const uint64_t need = uint64_t(g.n_nodes) * 4 / 3 + 2;
    uint64_t cap = kHashGlobal;
    while (cap < need && cap < (uint64_t(1) << 26)) cap <<= 1;
    return uint32_t(cap);
}
inline uint32_t fallback_workers(const Graph &g)
{
    return std::max<uint32_t>(16u, uint32_t(uint64_t(kFallbackWorkers) * kHashGlobal / fallback_slots(g)));
}
// Mid-size global tables: kMidWorkers workers of kHashGlobal slots each, for
// boxes that overflow every LDS table but touch fewer than 3/4 x kHashGlobal
// nodes (the largest boxes of the 15,917-capsule volume touch ~30,000). Only
// where the final tables are larger than that.
inline uint32_t mid_workers(const Graph &g) { return fallback_slots(g) > kHashGlobal ? kMidWorkers : 0u; }

// Carves the workspace for `fin_workers` workers of the final tables (0:
// fallback_workers(g)) and `mid_workers` of the mid-size ones (~0u: mid_workers(g));
// with base == nullptr only computes the size.
Workspace carve(const Graph &g, char *base, uint32_t max_boxes, uint32_t fin_workers = 0,
                uint32_t n_mid = ~0u)
{
    Workspace w;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    auto pool = [&](GlobalPool &p, uint32_t workers, uint32_t slots) {
        p.workers = workers, p.slots = slots;
        const uint64_t hs = uint64_t(workers) * slots;
        p.keys = reinterpret_cast<uint32_t *>(take(hs * 4));
        p.cnt = reinterpret_cast<uint32_t *>(take(hs * 4));
        p.used = reinterpret_cast<uint32_t *>(take(hs * 4));
        p.hi = reinterpret_cast<float *>(take(hs * 4));
        p.lo = reinterpret_cast<float *>(take(hs * 4));
        const uint64_t ss = uint64_t(workers) * g.nseg;
        p.seg_cnt = reinterpret_cast<uint32_t *>(take(ss * 4));
        p.seg_hi = reinterpret_cast<float *>(take(ss * 4));
        p.seg_lo = reinterpret_cast<float *>(take(ss * 4));
        p.seg_var = reinterpret_cast<float *>(take(ss * 4));
    };
    // fixed-size part first, so that its layout does not depend on max_boxes
    w.counters = reinterpret_cast<uint32_t *>(take(64 * 4));
    w.buckets = reinterpret_cast<uint32_t *>(take(64 * 4));
    w.queues = reinterpret_cast<uint32_t *>(take(uint64_t(kQueues) * kQueueStride * 4));
    pool(w.fin, fin_workers ? fin_workers : fallback_workers(g), fallback_slots(g));
    pool(w.mid, n_mid == ~0u ? mid_workers(g) : n_mid, kHashGlobal);
    w.bucket_of = reinterpret_cast<uint32_t *>(take(uint64_t(max_boxes) * 4));
    w.order = reinterpret_cast<uint32_t *>(take(uint64_t(max_boxes) * 4));
    w.overflow = reinterpret_cast<uint32_t *>(take(uint64_t(max_boxes) * 4));
    w.overflow2 = reinterpret_cast<uint32_t *>(take(uint64_t(max_boxes) * 4));
    w.overflow3 = reinterpret_cast<uint32_t *>(take(uint64_t(max_boxes) * 4));
    w.bytes = off;
    w.max_boxes = max_boxes;
    return w;
}

int check_device(Graph *g, std::string *err)
{
    if (g->dev.device < 0) {
        *err = "graph is not on a device: call mg_upload first";
        return MG_ESTATE;
    }
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != g->dev.device) HIP_TRY(hipSetDevice(g->dev.device));
    return MG_OK;
}

struct DeviceGuard {
    int prev = -1;
    DeviceGuard() { (void)hipGetDevice(&prev); }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int timing_begin(Graph *g, hipStream_t s, std::string *err)
{
    DeviceState &d = g->dev;
    if (!d.timing) return MG_OK;
    if (d.ev_used >= d.ev_start.size()) {
        hipEvent_t a, b;
        HIP_TRY(hipEventCreate(&a));
        HIP_TRY(hipEventCreate(&b));
        d.ev_start.push_back(a);
        d.ev_stop.push_back(b);
    }
    HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(d.ev_start[d.ev_used]), s));
    return MG_OK;
}

int timing_end(Graph *g, hipStream_t s, std::string *err)
{
    DeviceState &d = g->dev;
    if (!d.timing) return MG_OK;
    HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(d.ev_stop[d.ev_used]), s));
    d.ev_used++;
    return MG_OK;
}

using QueryKernel = void (*)(QueryArgs);
using NaiveKernel = void (*)(NaiveArgs);

template <int BLOCK, bool BIG, bool SPARSE, bool ERR>
QueryKernel tier_kernel(uint32_t unroll)
{
    if constexpr (ERR) {
        return query_tier_kernel<BLOCK, BIG, 8, SPARSE, true>;  // one unroll for uncertainty queries
    } else {
        switch (unroll) {
        case 4: return query_tier_kernel<BLOCK, BIG, 4, SPARSE, false>;
        case 8: return query_tier_kernel<BLOCK, BIG, 8, SPARSE, false>;
        default: return query_tier_kernel<BLOCK, BIG, 16, SPARSE, false>;
        }
    }
}

NaiveKernel naive_variant(uint32_t unroll)
{
    switch (unroll) {
    case 4: return naive_kernel<4>;
    case 8: return naive_kernel<8>;
    default: return naive_kernel<16>;
    }
}

bool valid_unroll(uint32_t u) { return u == 4 || u == 8 || u == 16; }

// Blocks per CU of a kernel variant (queried once, cached per device); also
// raises the kernel's dynamic LDS limit.
// Static LDS of a kernel (its __shared__ variables), as the code object states it.
int static_lds(const void *k, uint32_t *out, std::string *err)
{
    hipFuncAttributes fa{};
    HIP_TRY(hipFuncGetAttributes(&fa, k));
    *out = uint32_t(fa.sharedSizeBytes);
    return MG_OK;
}

int occupancy(DeviceState &d, const void *k, int block, uint32_t dyn, int *out, std::string *err)
{
    for (const auto &e : d.occupancy)
        if (e.kernel == k && e.dyn == dyn) {
            *out = e.blocks;
            return MG_OK;
        }
    uint32_t stat = 0;
    if (int rc = static_lds(k, &stat, err)) return rc;
    if (uint64_t(dyn) + stat > uint64_t(d.lds_max)) {
        *err = "kernel state of " + std::to_string(uint64_t(dyn) + stat) + " bytes exceeds the " +
               std::to_string(d.lds_max) + " bytes of LDS per workgroup";
        return MG_ELIMIT;
    }
    // the attribute is the largest dynamic LDS any launch of this kernel uses
    uint32_t dmax = dyn;
    for (const auto &e : d.occupancy)
        if (e.kernel == k) dmax = std::max(dmax, e.dyn);
    HIP_TRY(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(dmax)));
    int occ = 1;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, block, dyn));
    d.occupancy.push_back(DeviceState::Occ{k, dyn, std::max(occ, 1)});
    *out = std::max(occ, 1);
    return MG_OK;
}

// ---------------------------------------------------------------- no-allocation scratch

// The workspace of mg_query_boxes_noalloc: one array per device, held from the
// module's load until the process ends. Host code never passes `scratch`
// itself to a kernel (in host code the name is a stand-in, not a device
// address); it uses the address hipGetSymbolAddress returns for each device.
constexpr uint64_t kScratchBytes = uint64_t(MG_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) char scratch[kScratchBytes];

struct ScratchSlot {
    char *ptr = nullptr;                // device address of `scratch` on this device
    uint64_t layout[3] = {0, 0, 0};     // (sources, fallback slots, workers) last cleared; 0: never
};
std::mutex g_scratch_mu;
std::vector<ScratchSlot> g_scratch;      // per device ordinal

// The device address of the scratch array on the current device (looked up once per device).
int scratch_slot(int device, ScratchSlot **out, std::string *err)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0) {
        *err = "no device";
        return MG_ESTATE;
    }
    if (g_scratch.size() <= size_t(device)) g_scratch.resize(size_t(device) + 1);
    ScratchSlot &sl = g_scratch[size_t(device)];
    if (!sl.ptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return MG_EDEVICE;
        }
        sl.ptr = static_cast<char *>(p);
    }
    *out = &sl;
    return MG_OK;
}

}  // namespace

// ---------------------------------------------------------------- host-side address check

// Every load the query kernels (and, if naive, the naive scan) issue for these
// boxes, replayed on the host with the kernels' own slab builder and tile-walk
// helpers, UNROLL loads per block. counts: [0] boxes, [1] slabs, [2] lane
// loads checked, [3] cubes read.
int check_load_addresses(const uint32_t dims[3], bool use16, bool naive, bool runs, uint32_t run_min,
                         const uint32_t *boxes, uint32_t n, uint32_t unroll, uint64_t counts[4], std::string *err)
{
    LevelTable lt = level_table_dims(dims);
    if (lt.n_levels > kMaxLevelsDev) {
        *err = "more than " + std::to_string(kMaxLevelsDev) + " mip levels";
        return MG_ELIMIT;
    }
    lt.use16 = use16 ? 1u : 0u;
    if (runs) {  // row runs at every level and orientation whose rows the run builder accepts
        lt.run_min = run_min ? run_min : kRunMinRow;
        for (uint32_t l = 0; l < lt.n_levels && 2 * l + 1 < 32; ++l) {
            const uint64_t X = lt.dims[l][0], Y = lt.dims[l][1], Z = lt.dims[l][2];
            if (Y * Z < 0xFFFFFFFFull) lt.runs_mask |= 1u << (2 * l);
            if (Z * X < 0xFFFFFFFFull) lt.runs_mask |= 1u << (2 * l + 1);
        }
    }
    const uint64_t bytes32 = 2 * lt.total * 4;  // maps then maps_t
    const uint64_t n16t = uint64_t(lt.pitch_y) * dims[2] * dims[0];
    const uint64_t bytes16 = (lt.total16 + n16t) * 2;
    for (int k = 0; k < 4; ++k) counts[k] = 0;
    std::vector<Slab> slabs(kMaxSlabs);
    std::string where;
    // Replays every load of a tile walk (all UNROLL loads of every block, consumed or
    // not) and hands each consumed in-slab unit to unit(t, row, slice, pair bits).
    auto replay = [&](const TileWalk &tw, uint64_t base, uint64_t buf, uint32_t e0, uint32_t odd, bool pairs,
                      auto unit) -> bool {
        const uint64_t extent = uint64_t(tw.e2 - 1) * tw.s2b + uint64_t(tw.e1 - 1) * tw.s1b + 4ull * tw.units;
        if (base % 4 != 0) {
            where = "unaligned slab base";
            return false;
        }
        uint64_t seen = 0;
        for (uint32_t b = 0; b < tw.n_blk; ++b) {
            const uint32_t t0 = b % tw.n_t0, rb = (b / tw.n_t0) % tw.n_rb, k2 = b / (tw.n_t0 * tw.n_rb);
            const uint64_t blk = tile_block_offset(tw, t0, rb, k2);
            const uint32_t n_u = tile_n_u(tw, rb, unroll);
            if (n_u < 1) {
                where = "a block without a row tile";
                return false;
            }
            for (uint32_t lane = 0; lane < 64; ++lane) {
                const uint32_t lane_bytes = tile_lane_bytes(tw, lane);
                const uint32_t n_ok = tile_n_ok(tw, t0, rb, lane);
                if (uint64_t((lane >> tw.ltx)) * tw.s1b + (lane & ((1u << tw.ltx) - 1)) * 4ull >= (1ull << 32)) {
                    where = "lane offset does not fit 32 bits";
                    return false;
                }
                const uint32_t x = tile_unit(tw, t0, lane);
                const uint32_t pb = pairs ? pair_bits(x, e0, odd) : 1u;
                for (uint32_t u = 0; u < unroll; ++u) {
                    const uint64_t off = tile_load_offset(tw, blk, u, n_u, n_ok, lane_bytes);
                    ++counts[2];
                    if (off + 4 > extent) {
                        where = "load past the slab";
                        return false;
                    }
                    if (base + off + 4 > buf) {
                        where = "load past the buffer";
                        return false;
                    }
                    if (u < n_u && u < n_ok) {  // consumed, inside the slab
                        const uint32_t row = rb * tw.rows + u * tw.ty + (lane >> tw.ltx);
                        if (off != uint64_t(k2) * tw.s2b + uint64_t(row) * tw.s1b + 4ull * x) {
                            where = "load is not its unit";
                            return false;
                        }
                        ++seen;
                        if (!unit(x, row, k2, pb)) return false;
                    }
                }
            }
        }
        if (seen != uint64_t(tw.units) * tw.e1 * tw.e2) {
            where = "units read " + std::to_string(seen) + " of " + std::to_string(uint64_t(tw.units) * tw.e1 * tw.e2);
            return false;
        }
        return true;
    };
    for (uint32_t q = 0; q < n; ++q) {
        uint32_t lo[3], hi[3];
        if (!clip_box(boxes + 6 * uint64_t(q), lt, lo, hi)) continue;
        ++counts[0];
        int ns = 0;
        uint64_t cubes_closed = 0;
        for (uint32_t l = 0; l < lt.n_levels; ++l) {
            const int k = level_slabs<false>(lt, lo, hi, l, nullptr);
            if (k > 6) {  // the LDS slab table holds 6 per level
                *err = "box " + std::to_string(q) + ": more than 6 slabs at one level";
                return MG_ELIMIT;
            }
            level_slabs<true>(lt, lo, hi, l, slabs.data() + ns);
            ns += k;
            uint64_t outer = 1, inner = 1;
            for (int d = 0; d < 3; ++d) {
                const uint64_t one = uint64_t(1) << l;
                const uint64_t a = (uint64_t(lo[d]) + one - 1) >> l, b = hi[d] >> l;
                const uint64_t pa = (uint64_t(lo[d]) + 2 * one - 1) >> (l + 1), pb = hi[d] >> (l + 1);
                outer *= b > a ? b - a : 0;
                inner *= pb > pa ? 2 * (pb - pa) : 0;
            }
            cubes_closed += outer - inner;
        }
        uint64_t cubes = 0;
        for (int i = 0; i < ns; ++i) {
            const Slab &sl = slabs[i];
            ++counts[1];
            const uint32_t L = sl.level;
            if (sl.kind == 2) {  // row runs: every item's row and skip entry, its cells inside the box
                const uint32_t f = sl.axes & 3u, lseg = run_lseg(sl.e0);
                const uint64_t len = lt.dims[L][f], rows = f == 0 ? uint64_t(lt.dims[L][1]) * lt.dims[L][2]
                                                                 : uint64_t(lt.dims[L][2]) * lt.dims[L][0];
                const uint64_t chunks = (len + kRunSkipCells - 1) / kRunSkipCells;
                const uint64_t items = (uint64_t(sl.e1) * sl.e2) << lseg;
                if (f > 1 || items >= (1ull << 32)) where = "run slab orientation or size";
                for (uint64_t it = 0; where.empty() && it < items; ++it) {
                    uint32_t r, p0, p1;
                    if (!run_item(sl, lt, f, lseg, uint32_t(it), &r, &p0, &p1)) continue;
                    ++counts[2];
                    if (r >= rows || uint64_t(r) * chunks + p0 / kRunSkipCells >= rows * chunks || p1 > len) {
                        where = "run row or skip entry out of range";
                        break;
                    }
                    // the segment's first and last cube, and the row they lie on
                    const uint32_t row = uint32_t(it >> lseg);
                    const uint32_t i2 = sl.e2 == 1 ? 0u : row / sl.e1, i1 = row - i2 * sl.e1;
                    const uint32_t fa = f == 0 ? sl.bx : sl.by;
                    for (const uint32_t i0 : {p0 - fa, p1 - 1 - fa}) {
                        uint32_t cx, cy, cz;
                        slab_coords(sl, i0, i1, i2, &cx, &cy, &cz);
                        const uint32_t cc[3] = {cx, cy, cz};
                        for (int d = 0; d < 3; ++d)
                            if ((uint64_t(cc[d]) + 1) << L > hi[d] || uint64_t(cc[d]) << L < lo[d])
                                where = "run segment outside the box";
                        if ((f == 0 ? cy + uint64_t(lt.dims[L][1]) * cz : cz + uint64_t(lt.dims[L][2]) * cx) != r)
                            where = "run segment is not on its row";
                    }
                    cubes += p1 - p0;
                }
                if (!where.empty()) {
                    *err = "box " + std::to_string(q) + " level " + std::to_string(L) + " run slab " +
                           std::to_string(sl.e0) + "x" + std::to_string(sl.e1) + "x" + std::to_string(sl.e2) + ": " +
                           where;
                    return MG_ELIMIT;
                }
                continue;
            }
            const TileWalk tw = tile_walk(sl.units, sl.e1, sl.e2, sl.s1b, sl.s2b, unroll);
            const bool tr = (sl.axes & 3) == 1;
            const uint32_t X = lt.dims[L][0], Y = lt.dims[L][1], Z = lt.dims[L][2];
            auto unit = [&](uint32_t x, uint32_t row, uint32_t k2, uint32_t pb) -> bool {
                for (uint32_t h = 0; h < (sl.kind ? 2u : 1u); ++h) {
                    if (!((pb >> h) & 1u)) continue;
                    const uint32_t i0 = sl.kind ? 2 * x + h - sl.odd : x;
                    uint32_t cx, cy, cz;
                    slab_coords(sl, i0, row, k2, &cx, &cy, &cz);
                    const uint32_t cc[3] = {cx, cy, cz};
                    for (int d = 0; d < 3; ++d)
                        if ((uint64_t(cc[d]) + 1) << L > hi[d] || uint64_t(cc[d]) << L < lo[d]) {
                            where = "cube outside the box";
                            return false;
                        }
                    uint64_t el;
                    if (sl.kind) el = tr ? lt.total16 + cy + uint64_t(lt.pitch_y) * (cz + uint64_t(Z) * cx)
                                         : cx + uint64_t(lt.pitch_x) * (cy + uint64_t(Y) * cz);
                    else el = tr ? lt.total + lt.off[L] + cy + uint64_t(Y) * (cz + uint64_t(Z) * cx)
                                 : lt.off[L] + cx + uint64_t(X) * (cy + uint64_t(Y) * cz);
                    const uint64_t byte = sl.base + uint64_t(k2) * sl.s2b + uint64_t(row) * sl.s1b + 4ull * x;
                    const uint64_t at = sl.kind ? byte / 2 + h : byte / 4;
                    if (el != at) {
                        where = "address is not the cube's element";
                        return false;
                    }
                    ++cubes;
                }
                return true;
            };
            if (!replay(tw, sl.base, sl.kind ? bytes16 : bytes32, sl.e0, sl.odd, sl.kind != 0, unit)) {
                *err = "box " + std::to_string(q) + " level " + std::to_string(L) + " slab " + std::to_string(sl.e0) +
                       "x" + std::to_string(sl.e1) + " kind " + std::to_string(sl.kind) + ": " + where;
                return MG_ELIMIT;
            }
        }
        if (cubes != cubes_closed) {
            *err = "box " + std::to_string(q) + ": " + std::to_string(cubes) + " cubes read, the footprint has " +
                   std::to_string(cubes_closed);
            return MG_ELIMIT;
        }
        counts[3] += cubes;
        if (naive) {  // the naive scan reads level 0 of the box from the x-fastest copy
            uint64_t base;
            uint32_t odd;
            const TileWalk tw = naive_walk(lt, lo, hi, use16, unroll, &base, &odd);
            uint64_t vox = 0;
            auto unit = [&](uint32_t x, uint32_t row, uint32_t k2, uint32_t pb) -> bool {
                for (uint32_t h = 0; h < (use16 ? 2u : 1u); ++h) {
                    if (!((pb >> h) & 1u)) continue;
                    const uint32_t cx = lo[0] + (use16 ? 2 * x + h - odd : x), cy = lo[1] + row, cz = lo[2] + k2;
                    if (cx >= hi[0] || cy >= hi[1] || cz >= hi[2]) {
                        where = "voxel outside the box";
                        return false;
                    }
                    const uint64_t el = use16 ? cx + uint64_t(lt.pitch_x) * (cy + uint64_t(dims[1]) * cz)
                                              : cx + uint64_t(dims[0]) * (cy + uint64_t(dims[1]) * cz);
                    const uint64_t off = base + uint64_t(k2) * tw.s2b + uint64_t(row) * tw.s1b + 4ull * x;
                    if (el != (use16 ? off / 2 + h : off / 4)) {
                        where = "address is not the voxel's element";
                        return false;
                    }
                    ++vox;
                }
                return true;
            };
            const uint64_t vox0 = uint64_t(dims[0]) * dims[1] * dims[2];  // level 0 of the 32-bit maps
            if (!replay(tw, base, use16 ? lt.total16 * 2 : vox0 * 4, hi[0] - lo[0], odd, use16, unit)) {
                *err = "box " + std::to_string(q) + " naive scan: " + where;
                return MG_ELIMIT;
            }
            if (vox != uint64_t(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2])) {
                *err = "box " + std::to_string(q) + " naive scan: voxels read " + std::to_string(vox);
                return MG_ELIMIT;
            }
        }
    }
    return MG_OK;
}

// ---------------------------------------------------------------- entry points

// Byte offsets of the graph's device arrays inside one buffer (each 256-byte
// aligned): what mg_device_bytes sizes and mg_bind_device fills.
struct DeviceLayout {
    uint64_t nodes, sched, rank_ptr, mixlen, maps, maps16;
    uint64_t n16, n16t;   // elements of the two 16-bit level-0 copies (0 if none)
    uint64_t run_table;   // RunLevel [2 n_levels]
    std::vector<uint64_t> run_sk, run_rn;  // per level and orientation: skip, runs
    uint64_t bytes;
};

DeviceLayout device_layout(const Graph &g)
{
    DeviceLayout L;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = off;
        off += align256(bytes);
        return at;
    };
    const uint64_t nmap = g.lev_off[g.n_levels];
    L.nodes = take(uint64_t(g.n_nodes) * sizeof(NodeTriple));
    L.sched = take(uint64_t(g.n_nodes) * sizeof(SchedNode));
    L.rank_ptr = take(g.rank_ptr.size() * 4);
    L.mixlen = take(uint64_t(g.n_nodes) * 4);
    L.maps = take(2 * nmap * 4);  // x-fastest copy, then the y-fastest one
    L.n16 = L.n16t = 0;
    if (g.nseg < 0xFFFFu) {       // 16-bit level 0 for the hot path when every source ID fits
        const LevelTable lt = level_table(g);
        L.n16 = lt.total16;
        L.n16t = uint64_t(lt.pitch_y) * g.dims[2] * g.dims[0];
    }
    L.maps16 = take((L.n16 + L.n16t) * sizeof(uint16_t));
    // row runs of every level and orientation that has them (built from the host maps)
    ensure_runs(g);
    L.run_table = take(2 * uint64_t(g.n_levels) * sizeof(RunLevel));
    for (const LevelRuns &r : g.runs) {
        L.run_sk.push_back(r.rows ? take(r.skip.size() * 4) : 0);
        L.run_rn.push_back(r.rows ? take(r.runs.size() * 8) : 0);
    }
    L.bytes = off;
    return L;
}

// Fills `base` (device memory of layout.bytes bytes on `device`) with the
// graph's arrays and derived copies, enqueued on `stream`, then waits for
// them; the graph then reads only this memory. owned: mg_free releases it.
// Where a graph's maps come from when they are not on the host: its stream.
struct StreamSrc {
    const uint8_t *buf;
    uint64_t size;
    const StreamMaps *sm;
};

// Decodes the stream's voxel data into d.maps (x fastest, every level) on `s`;
// waits for it and checks every node ID.
int decode_stream_maps(Graph *g, const StreamSrc &src, hipStream_t s, std::string *err)
{
    const StreamMaps &sm = *src.sm;
    DeviceState &d = g->dev;
    StreamLevels lv;
    std::memset(&lv, 0, sizeof(lv));
    lv.n_levels = g->n_levels;
    lv.nseg = g->nseg;
    lv.n_nodes = g->n_nodes;
    // the staged words start at the 32-bit word holding (A)'s first bit
    const uint64_t first_byte = (sm.a_bit >> 5) * 4;
    const uint64_t lead = sm.a_bit - first_byte * 8;
    uint64_t bits = 0;
    for (uint32_t l = 0; l < g->n_levels; ++l) {
        lv.off[l] = g->lev_off[l];
        lv.bit[l] = lead + sm.bit_off[l];
        lv.r[l] = sm.r[l];
        lv.lo[l] = sm.lo[l];
        bits = sm.bit_off[l] + uint64_t(sm.r[l]) * (g->lev_off[l + 1] - g->lev_off[l]);
    }
    lv.off[g->n_levels] = g->lev_off[g->n_levels];
    // every field lies in the staged words; one zero word past the last field
    const uint64_t words = (lead + bits + 31) / 32 + 1;
    const uint64_t avail = src.size > first_byte ? std::min<uint64_t>(src.size - first_byte, words * 4) : 0;
    void *stage = nullptr, *perm = nullptr, *bad = nullptr;
    const uint64_t perm_bytes = std::max<uint64_t>(sm.perm.size(), 1) * 4;
    if (hipMalloc(&stage, words * 4) != hipSuccess || hipMalloc(&perm, perm_bytes) != hipSuccess ||
        hipMalloc(&bad, 4) != hipSuccess) {
        (void)hipGetLastError();
        if (stage) (void)hipFree(stage);
        if (perm) (void)hipFree(perm);
        *err = "device allocation for decoding the graph stream failed";
        return MG_ENOMEM;
    }
    int rc = MG_OK;
    uint32_t flag = 0;
    auto run = [&]() -> int {
        HIP_TRY(hipMemcpyAsync(stage, src.buf + first_byte, avail, hipMemcpyHostToDevice, s));
        if (avail < words * 4)  // the stream ends inside the last words: zero the rest
            hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, s,
                               static_cast<uint32_t *>(stage) + avail / 4, words - avail / 4, 0u);
        if (avail % 4) {       // a partial last word: its bytes past the stream read as zero
            uint32_t tail = 0;
            std::memcpy(&tail, src.buf + first_byte + (avail / 4) * 4, avail % 4);
            HIP_TRY(hipMemcpyAsync(static_cast<uint32_t *>(stage) + avail / 4, &tail, 4, hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));  // `tail` lives on this stack frame
        }
        if (!sm.perm.empty())
            HIP_TRY(hipMemcpyAsync(perm, sm.perm.data(), sm.perm.size() * 4, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, s, static_cast<uint32_t *>(bad), uint64_t(1), 0u);
        const uint64_t total = g->lev_off[g->n_levels];
        const uint32_t blocks = uint32_t(std::min<uint64_t>((total + 255) / 256, 65536));
        hipLaunchKernelGGL(unpack_maps_kernel, dim3(blocks), dim3(256), 0, s, lv,
                           static_cast<const uint32_t *>(stage), static_cast<const uint32_t *>(perm), d.maps,
                           static_cast<uint32_t *>(bad));
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&flag, bad, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return MG_OK;
    };
    rc = run();
    (void)hipFree(stage);
    (void)hipFree(perm);
    (void)hipFree(bad);
    if (rc) return rc;
    if (flag) {
        *err = "graph stream: voxel node ID out of range";
        return MG_EFORMAT;
    }
    return MG_OK;
}

int dev_bind(Graph *g, int device, void *base, uint64_t bytes, hipStream_t s, bool owned, std::string *err,
             const StreamSrc *src = nullptr)
{
    DeviceState &d = g->dev;
    const DeviceLayout L = device_layout(*g);
    if (bytes < L.bytes) {
        *err = "device buffer of " + std::to_string(bytes) + " bytes; the graph needs " + std::to_string(L.bytes);
        return MG_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(base) % 256 != 0) {
        *err = "device buffer must be 256-byte aligned";
        return MG_EINVAL;
    }
    char *b = static_cast<char *>(base);
    const uint64_t nmap = g->lev_off[g->n_levels];
    std::vector<NodeTriple> nodes(g->n_nodes);
    for (uint32_t n = 0; n < g->n_nodes; ++n) nodes[n] = NodeTriple{g->child_a[n], g->child_b[n], g->alpha[n]};
    std::vector<SchedNode> sched(g->n_nodes);
    for (uint32_t i = 0; i < g->n_nodes; ++i) {
        const uint32_t n = g->sched[i];
        sched[i] = SchedNode{g->child_a[n], g->child_b[n], g->alpha[n], n};
    }
    // sources in a node's mixture, bounded by the sum over its two predecessors (IDs are
    // sorted by rank, so predecessors come first); exact when the two are disjoint
    std::vector<uint32_t> mixlen(g->n_nodes, 1u);
    for (uint32_t n = g->nseg; n < g->n_nodes; ++n)
        mixlen[n] = uint32_t(std::min<uint64_t>(g->nseg, uint64_t(mixlen[g->child_a[n]]) + mixlen[g->child_b[n]]));
    d.base = base;
    d.owned = owned;
    d.device = device;
    d.bytes = L.bytes;
    d.nodes = reinterpret_cast<NodeTriple *>(b + L.nodes);
    d.sched = reinterpret_cast<SchedNode *>(b + L.sched);
    d.rank_ptr = reinterpret_cast<uint32_t *>(b + L.rank_ptr);
    d.mixlen = reinterpret_cast<uint32_t *>(b + L.mixlen);
    d.maps = reinterpret_cast<uint32_t *>(b + L.maps);
    d.maps_t = d.maps + nmap;
    d.maps16 = L.n16 ? reinterpret_cast<uint16_t *>(b + L.maps16) : nullptr;
    HIP_TRY(hipMemcpyAsync(d.nodes, nodes.data(), nodes.size() * sizeof(NodeTriple), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d.sched, sched.data(), sched.size() * sizeof(SchedNode), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d.rank_ptr, g->rank_ptr.data(), g->rank_ptr.size() * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d.mixlen, mixlen.data(), mixlen.size() * 4, hipMemcpyHostToDevice, s));
    if (src) {
        if (int rc = decode_stream_maps(g, *src, s, err)) return rc;
    } else {
        HIP_TRY(hipMemcpyAsync(d.maps, g->maps.data(), nmap * 4, hipMemcpyHostToDevice, s));
    }
    for (uint32_t l = 0; l < g->n_levels; ++l) {
        const uint32_t X = g->lev_dims[3 * l], Y = g->lev_dims[3 * l + 1], Z = g->lev_dims[3 * l + 2];
        const uint64_t cnt = uint64_t(X) * Y * Z;
        const uint32_t blocks = uint32_t((cnt + 255) / 256);
        hipLaunchKernelGGL(transpose_level_kernel, dim3(blocks), dim3(256), 0, s, d.maps + g->lev_off[l],
                           d.maps_t + g->lev_off[l], X, Y, Z);
        HIP_TRY(hipGetLastError());
    }
    if (L.n16) {
        const LevelTable lt = level_table(*g);
        const uint64_t n = std::max(L.n16, L.n16t);
        hipLaunchKernelGGL(pack16_kernel, dim3(uint32_t((n + 255) / 256)), dim3(256), 0, s, d.maps, d.maps16,
                           g->dims[0], g->dims[1], g->dims[2], lt.pitch_x, lt.pitch_y, L.n16, L.n16t);
        HIP_TRY(hipGetLastError());
    }
    // row runs and their table
    std::vector<RunLevel> table(2 * size_t(g->n_levels));
    d.runs_mask = 0;
    for (size_t k = 0; k < g->runs.size() && k < table.size(); ++k) {
        const LevelRuns &r = g->runs[k];
        RunLevel &t = table[k];
        t = RunLevel{nullptr, nullptr, 0, 0, 0};
        if (!r.rows || r.runs.empty()) continue;
        t.skip = reinterpret_cast<const uint32_t *>(b + L.run_sk[k]);
        t.runs = reinterpret_cast<const uint64_t *>(b + L.run_rn[k]);
        t.rows = r.rows, t.chunks = r.chunks, t.n_runs = uint32_t(r.runs.size());
        HIP_TRY(hipMemcpyAsync(b + L.run_sk[k], r.skip.data(), r.skip.size() * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(b + L.run_rn[k], r.runs.data(), r.runs.size() * 8, hipMemcpyHostToDevice, s));
        if (k < 32) d.runs_mask |= 1u << k;
    }
    d.run_table = b + L.run_table;
    if (!table.empty())
        HIP_TRY(hipMemcpyAsync(d.run_table, table.data(), table.size() * sizeof(RunLevel), hipMemcpyHostToDevice, s));
    // the host staging vectors above die with this call
    HIP_TRY(hipStreamSynchronize(s));
    // set-up of the no-allocation path on this device (the scratch array's address)
    ScratchSlot *sl = nullptr;
    if (int rc = scratch_slot(device, &sl, err)) return rc;
    if (!g->lut_ptr.empty()) return dev_upload_lut(g, err);
    return MG_OK;
}

uint64_t dev_device_bytes(const Graph &g) { return device_layout(g).bytes; }

int dev_bind_device(Graph *g, int device, void *base, uint64_t bytes, void *stream, std::string *err)
{
    if (g->maps_on_device) {
        *err = "the graph's node maps exist only on its device (decoded from a stream there)";
        return MG_ESTATE;
    }
    DeviceGuard guard;
    if (g->dev.device >= 0) dev_free(g);
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) {
        *err = "device " + std::to_string(device) + " does not exist";
        return MG_EINVAL;
    }
    HIP_TRY(hipSetDevice(device));
    const int rc = dev_bind(g, device, base, bytes, static_cast<hipStream_t>(stream), false, err);
    if (rc) dev_free(g);
    return rc;
}

int upload_with(Graph *g, int device, const StreamSrc *src, std::string *err)
{
    DeviceGuard guard;
    if (g->dev.device >= 0) dev_free(g);
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device >= ndev) {
        *err = "mg_upload: device " + std::to_string(device) + " does not exist";
        return MG_EINVAL;
    }
    HIP_TRY(hipSetDevice(device));
    const uint64_t bytes = device_layout(*g).bytes;
    void *base = nullptr;
    if (hipMalloc(&base, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *err = "mg_upload: device allocation of " + std::to_string(bytes) + " bytes failed";
        return MG_ENOMEM;
    }
    const int rc = dev_bind(g, device, base, bytes, nullptr, true, err, src);
    if (rc) {
        if (g->dev.base != base) (void)hipFree(base);  // not recorded yet: release it here
        dev_free(g);
    }
    return rc;
}

int dev_upload(Graph *g, int device, std::string *err)
{
    if (g->maps_on_device) {
        *err = "the graph's node maps exist only on its device (decoded from a stream there)";
        return MG_ESTATE;
    }
    return upload_with(g, device, nullptr, err);
}

int dev_upload_stream(Graph *g, const uint8_t *buf, uint64_t size, const StreamMaps &sm, int device,
                      std::string *err)
{
    const StreamSrc src{buf, size, &sm};
    return upload_with(g, device, &src, err);
}

int dev_export_map(const Graph &g, uint32_t level, uint32_t *out, std::string *err)
{
    if (g.dev.device < 0 || !g.dev.maps) {
        *err = "the graph is not on a device";
        return MG_ESTATE;
    }
    DeviceGuard guard;
    HIP_TRY(hipSetDevice(g.dev.device));
    const uint64_t n = g.lev_off[level + 1] - g.lev_off[level];
    HIP_TRY(hipMemcpy(out, g.dev.maps + g.lev_off[level], n * 4, hipMemcpyDeviceToHost));
    return MG_OK;
}

int dev_upload_lut(Graph *g, std::string *err)
{
    DeviceGuard guard;
    DeviceState &d = g->dev;
    if (d.device < 0) {
        *err = "graph not on a device";
        return MG_ESTATE;
    }
    HIP_TRY(hipSetDevice(d.device));
    if (d.lut_ptr) (void)hipFree(d.lut_ptr);
    if (d.lut_seg) (void)hipFree(d.lut_seg);
    if (d.lut_val) (void)hipFree(d.lut_val);
    if (d.lut_err) (void)hipFree(d.lut_err);
    d.lut_ptr = nullptr, d.lut_seg = nullptr, d.lut_val = nullptr, d.lut_err = nullptr;
    const uint64_t bp = g->lut_ptr.size() * sizeof(uint64_t), nnz = g->lut_seg.size();
    if (hipMalloc(&d.lut_ptr, bp) != hipSuccess || hipMalloc(&d.lut_seg, nnz * 4) != hipSuccess ||
        hipMalloc(&d.lut_val, nnz * 4) != hipSuccess) {
        (void)hipGetLastError();
        if (d.lut_ptr) (void)hipFree(d.lut_ptr);
        if (d.lut_seg) (void)hipFree(d.lut_seg);
        d.lut_ptr = nullptr, d.lut_seg = nullptr, d.lut_val = nullptr;
        *err = "mixture lookup table: device allocation failed";
        return MG_ENOMEM;
    }
    HIP_TRY(hipMemcpy(d.lut_ptr, g->lut_ptr.data(), bp, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d.lut_seg, g->lut_seg.data(), nnz * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d.lut_val, g->lut_val.data(), nnz * 4, hipMemcpyHostToDevice));
    d.bytes += bp + 8 * nnz;
    if (g->lut_err.size() == nnz && nnz) {
        if (hipMalloc(&d.lut_err, nnz * 4) != hipSuccess) {
            (void)hipGetLastError();
            d.lut_err = nullptr;
            *err = "mixture lookup table: device allocation failed (uncertainties)";
            return MG_ENOMEM;
        }
        HIP_TRY(hipMemcpy(d.lut_err, g->lut_err.data(), nnz * 4, hipMemcpyHostToDevice));
        d.bytes += 4 * nnz;
    }
    return MG_OK;
}

int dev_palette_fetch(Graph *g, const float *palette, uint32_t T, uint32_t level, const uint32_t *xyz, uint32_t n,
                      float *out, void *stream, std::string *err)
{
    DeviceGuard guard;
    int rc = check_device(g, err);
    if (rc) return rc;
    const uint32_t X = g->lev_dims[3 * level], Y = g->lev_dims[3 * level + 1], Z = g->lev_dims[3 * level + 2];
    hipLaunchKernelGGL(palette_fetch_kernel, dim3((n + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                       reinterpret_cast<const float4 *>(palette), T, g->n_nodes, g->dev.maps + g->lev_off[level], X,
                       Y, Z, xyz, n, reinterpret_cast<float4 *>(out));
    HIP_TRY(hipGetLastError());
    return MG_OK;
}

int dev_box_colour(Graph *g, const float *palette, uint32_t T, const uint32_t *boxes, uint32_t n,
                   const uint32_t *pal_of_box, float *out, void *stream, std::string *err)
{
    DeviceGuard guard;
    int rc = check_device(g, err);
    if (rc) return rc;
    if (g->n_levels > kMaxLevelsDev) {
        *err = "more than " + std::to_string(kMaxLevelsDev) + " mip levels";
        return MG_ELIMIT;
    }
    const LevelTable lt = level_table(*g);
    hipLaunchKernelGGL(box_colour_kernel, dim3(n), dim3(kColourBlock), 0, static_cast<hipStream_t>(stream), lt, boxes, n,
                       g->dev.maps, reinterpret_cast<const float4 *>(palette), T, g->n_nodes, pal_of_box,
                       reinterpret_cast<float4 *>(out));
    HIP_TRY(hipGetLastError());
    return MG_OK;
}

void dev_free(Graph *g)
{
    DeviceState &d = g->dev;
    if (d.device < 0 && !d.base) return;
    DeviceGuard guard;
    if (d.device >= 0) (void)hipSetDevice(d.device);
    if (d.base && d.owned) (void)hipFree(d.base);
    if (d.lut_ptr) (void)hipFree(d.lut_ptr);
    if (d.lut_seg) (void)hipFree(d.lut_seg);
    if (d.lut_val) (void)hipFree(d.lut_val);
    if (d.lut_err) (void)hipFree(d.lut_err);
    for (void *e : d.ev_start) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
    for (void *e : d.ev_stop) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
    d = DeviceState();
}

uint64_t dev_workspace_bytes(const Graph &g, uint32_t max_boxes)
{
    return carve(g, nullptr, std::max<uint32_t>(max_boxes, 1)).bytes;
}

// The global fallback tables of a workspace in their clean state (empty keys,
// zero counts and mass), by fill kernels on `s` (no memset: callers may
// capture the stream into a graph).
void clear_pool(const Graph &g, const GlobalPool &p, hipStream_t s)
{
    const uint64_t hs = uint64_t(p.workers) * p.slots;
    if (hs) {
        hipLaunchKernelGGL(fill_u32_kernel, dim3(1024), dim3(256), 0, s, p.keys, hs, kEmpty);
        hipLaunchKernelGGL(fill_u32_kernel, dim3(1024), dim3(256), 0, s, p.cnt, hs, 0u);
        hipLaunchKernelGGL(fill_u32_kernel, dim3(1024), dim3(256), 0, s, reinterpret_cast<uint32_t *>(p.hi), hs, 0u);
        hipLaunchKernelGGL(fill_u32_kernel, dim3(1024), dim3(256), 0, s, reinterpret_cast<uint32_t *>(p.lo), hs, 0u);
    }
    const uint64_t ss = uint64_t(p.workers) * g.nseg;
    if (!ss) return;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(256), dim3(256), 0, s, p.seg_cnt, ss, 0u);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(256), dim3(256), 0, s, reinterpret_cast<uint32_t *>(p.seg_hi), ss, 0u);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(256), dim3(256), 0, s, reinterpret_cast<uint32_t *>(p.seg_lo), ss, 0u);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(256), dim3(256), 0, s, reinterpret_cast<uint32_t *>(p.seg_var), ss, 0u);
}

void clear_fallback_tables(const Graph &g, const Workspace &w, hipStream_t s)
{
    clear_pool(g, w.fin, s);
    clear_pool(g, w.mid, s);
}

int dev_workspace_init(Graph *g, void *work, uint64_t bytes, void *stream, std::string *err)
{
    int rc = check_device(g, err);
    if (rc) return rc;
    // the fixed-size part (counters, queues, fallback tables) comes first, so its
    // layout does not depend on the box capacity
    Workspace w = carve(*g, static_cast<char *>(work), 1);
    if (bytes < w.bytes) {
        *err = "workspace smaller than mg_workspace_bytes(g, 1)";
        return MG_EINVAL;
    }
    clear_fallback_tables(*g, w, static_cast<hipStream_t>(stream));
    HIP_TRY(hipGetLastError());
    return MG_OK;
}

template <bool SPARSE, bool ERR>
int launch_query(Graph *g, QueryArgs &A, const Workspace &w, const LevelTable &lt, uint32_t n, hipStream_t s,
                 int variant, std::string *err)
{
    int rc = MG_OK;
    DeviceState &d = g->dev;
    const int bbig = d.cfg.block_big == 256 ? 256 : kBlockBig;    // threads per big-tier box
    const QueryKernel kbig = bbig == 256 ? tier_kernel<256, true, SPARSE, ERR>(d.cfg.unroll_big)
                                         : tier_kernel<kBlockBig, true, SPARSE, ERR>(d.cfg.unroll_big);
    const int bsmall = d.cfg.block_small == 256 ? kBlock : 128;  // threads per small-tier box
    const QueryKernel ksmall = bsmall == 128 ? tier_kernel<128, false, SPARSE, ERR>(d.cfg.unroll_small)
                                             : tier_kernel<kBlock, false, SPARSE, ERR>(d.cfg.unroll_small);
    const QueryKernel kplain = query_plain_kernel<SPARSE>;
    const uint32_t cap_big = d.cfg.table_big ? d.cfg.table_big : (SPARSE ? kHashBigSparse : kHashBig);
    const uint32_t cap_small = d.cfg.table_small ? d.cfg.table_small : (SPARSE ? kHashSmallSparse : kHashSmall);
    const uint32_t L = g->n_levels;
    constexpr bool E = ERR;
    const uint32_t dyn_big = lds_bytes(g->nseg, cap_big, SPARSE, L, E),
                   dyn_small = lds_bytes(g->nseg, cap_small, SPARSE, L, E),
                   dyn_plain = lds_bytes(g->nseg, kHashPlain, SPARSE, L, E);
    int occ_big = 1, occ_small = 1, occ_plain = 1;
    if ((rc = occupancy(d, reinterpret_cast<const void *>(kbig), bbig, dyn_big, &occ_big, err)) ||
        (rc = occupancy(d, reinterpret_cast<const void *>(ksmall), bsmall, dyn_small, &occ_small, err)) ||
        (rc = occupancy(d, reinterpret_cast<const void *>(kplain), kBlock, dyn_plain, &occ_plain, err)))
        return rc;
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, w.counters, 64u);
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(256), 0, s, w.queues, kQueues * kQueueStride);
    A.queues = w.queues;
    if (A.sp_total) hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, A.sp_total, 1u);
    if (variant == kQueryBatched || variant == kQueryLut) {
        hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, w.buckets, 64u);
        const uint32_t blocks = (n + 255) / 256;
        hipLaunchKernelGGL(query_size_kernel, dim3(blocks), dim3(256), 0, s, lt, A.boxes, n, w.bucket_of, w.buckets);
        hipLaunchKernelGGL(bucket_scan_kernel, dim3(1), dim3(64), 0, s, w.buckets, w.counters);
        hipLaunchKernelGGL(query_order_kernel, dim3(blocks), dim3(256), 0, s, w.bucket_of, n, w.buckets, w.order);
        A.order = w.order;
        const uint32_t wbig = std::max(1u, std::min<uint32_t>(n, uint32_t(d.ncu) * uint32_t(occ_big)));
        const uint32_t wsmall = std::max(1u, std::min<uint32_t>(n, uint32_t(d.ncu) * uint32_t(occ_small)));
        rc = timing_begin(g, s, err);
        if (rc) return rc;
        A.table_cap = cap_big;
        hipLaunchKernelGGL(kbig, dim3(wbig), dim3(bbig), dyn_big, s, A);
        HIP_TRY(hipGetLastError());
        A.table_cap = cap_small;
        A.chunk = d.cfg.chunk_small;
        hipLaunchKernelGGL(ksmall, dim3(wsmall), dim3(bsmall), dyn_small, s, A);
        HIP_TRY(hipGetLastError());
    } else {
        A.table_cap = kHashPlain;
        rc = timing_begin(g, s, err);
        if (rc) return rc;
        hipLaunchKernelGGL(kplain, dim3(n), dim3(kBlock), dyn_plain, s, A);
        HIP_TRY(hipGetLastError());
    }
    // boxes whose table overflowed: once more with a larger LDS table, then in global memory
    const QueryKernel kretry = query_retry_kernel<kBlockBig, 8, SPARSE, ERR>;
    uint32_t cap_retry = d.cfg.table_retry;
    if (!cap_retry) {  // the largest table up to kHashRetry that fits the LDS of a workgroup
        uint32_t stat = 0;
        if ((rc = static_lds(reinterpret_cast<const void *>(kretry), &stat, err))) return rc;
        cap_retry = kHashRetry;
        while (cap_retry > kHashBigSparse &&
               uint64_t(lds_bytes(g->nseg, cap_retry, SPARSE, L, E)) + stat > uint64_t(d.lds_max))
            cap_retry /= 2;
    }
    const uint32_t dyn_retry = lds_bytes(g->nseg, cap_retry, SPARSE, L, E);
    int occ_retry = 1;
    if ((rc = occupancy(d, reinterpret_cast<const void *>(kretry), kBlockBig, dyn_retry, &occ_retry, err)))
        return rc;
    A.table_cap = cap_retry;
    A.stats_tag = 0x40000000u;
    A.ovf_out = w.overflow2;
    A.ovf_out_idx = 5;
    hipLaunchKernelGGL(kretry, dim3(uint32_t(d.ncu) * uint32_t(occ_retry)), dim3(kBlockBig), dyn_retry, s, A);
    HIP_TRY(hipGetLastError());
    // boxes that overflowed every LDS table: global-memory tables, first many workers with
    // mid-size tables (overflow: list 3), then the few whose tables hold the whole graph
    A.stats_tag = 0x80000000u;
    const QueryKernel kfallback = query_fallback_kernel<ERR>;
    const uint32_t dyn_fb = 6u * L * uint32_t(sizeof(Slab));
    auto use_pool = [&](const GlobalPool &p) {
        A.g_slots = p.slots;
        A.g_keys = p.keys, A.g_cnt = p.cnt, A.g_used = p.used, A.g_hi = p.hi, A.g_lo = p.lo;
        A.g_seg_cnt = p.seg_cnt, A.g_seg_hi = p.seg_hi, A.g_seg_lo = p.seg_lo, A.g_seg_var = p.seg_var;
    };
    if (w.mid.workers) {
        use_pool(w.mid);
        A.g_list = w.overflow2, A.g_count_idx = 5, A.g_next_idx = 7;
        A.ovf_out = w.overflow3;
        A.ovf_out_idx = 6;
        hipLaunchKernelGGL(kfallback, dim3(w.mid.workers), dim3(kBlock), dyn_fb, s, A);
        HIP_TRY(hipGetLastError());
        A.g_list = w.overflow3, A.g_count_idx = 6;
    } else {
        A.g_list = w.overflow2, A.g_count_idx = 5;
    }
    use_pool(w.fin);
    A.g_next_idx = 2;
    A.ovf_out = nullptr;
    hipLaunchKernelGGL(kfallback, dim3(w.fin.workers), dim3(kBlock), dyn_fb, s, A);
    HIP_TRY(hipGetLastError());
    // the timed region: every kernel that answers boxes (tiers or plain, retry, fallback)
    return timing_end(g, s, err);
}

namespace {

// The query path on a carved workspace (the caller's or the library's scratch).
int query_in(Graph *g, const uint32_t *boxes, uint32_t n, float *out, const SparseOut *sp, const Workspace &w,
             hipStream_t s, int variant, uint32_t *stats, std::string *err, float *out_err)
{
    int rc = MG_OK;
    if (g->depth > kMaxSteps) {
        *err = "graph depth " + std::to_string(g->depth) + " beyond the kernels' step table (" +
               std::to_string(kMaxSteps) + ")";
        return MG_ELIMIT;
    }
    if (g->n_levels > kMaxLevelsDev) {
        *err = "more than " + std::to_string(kMaxLevelsDev) + " mip levels";
        return MG_ELIMIT;
    }
    const LevelTable lt = level_table(*g);
    if (!g->dev.launch_ready) {
        HIP_TRY(hipDeviceGetAttribute(&g->dev.lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, g->dev.device));
        HIP_TRY(hipDeviceGetAttribute(&g->dev.ncu, hipDeviceAttributeMultiprocessorCount, g->dev.device));
        g->dev.launch_ready = true;
    }

    if (variant == kQueryNaive) {
        if (g->nseg > 16384) {
            *err = "naive scan keeps per-source counts in LDS: at most 16384 sources";
            return MG_ELIMIT;
        }
        if (sp) {
            *err = "the naive scan writes dense output only";
            return MG_EINVAL;
        }
        NaiveArgs A;
        A.lt = lt;
        A.boxes = boxes;
        A.out = out;
        A.map0 = g->dev.maps;
        A.map16 = g->dev.maps16;
        A.lt.use16 = g->dev.maps16 ? 1u : 0u;
        A.nseg = g->nseg;
        A.n = n;
        rc = timing_begin(g, s, err);
        if (rc) return rc;
        hipLaunchKernelGGL(naive_variant(g->dev.cfg.unroll_naive), dim3(n), dim3(kBlock), g->nseg * 4, s, A);
        HIP_TRY(hipGetLastError());
        return timing_end(g, s, err);
    }

    QueryArgs A;
    std::memset(&A, 0, sizeof(A));
    A.lt = lt;
    A.boxes = boxes;
    A.out = sp ? nullptr : out;
    if (sp) {
        A.sp_index = sp->index;
        A.sp_seg = sp->seg;
        A.sp_val = sp->val;
        A.sp_cap = sp->cap;
        A.sp_total = sp->total;
    }
    A.maps = g->dev.maps;
    A.maps16 = g->dev.maps16;
    A.gv.nodes = g->dev.nodes;
    A.gv.nseg = g->nseg;
    A.gv.r1_end = g->depth >= 1 ? g->rank_ptr[2] : g->nseg;
    A.gv.r2_end = g->depth >= 2 ? g->rank_ptr[3] : A.gv.r1_end;
    A.rank_ptr = g->dev.rank_ptr;
    A.depth = g->depth;
    A.n = n;
    A.counters = w.counters;
    A.overflow = w.overflow;
    A.overflow2 = w.overflow2;
    A.ovf_out = w.overflow;
    A.ovf_out_idx = 1;
    A.stats = stats;
    if (variant == kQueryLut || variant == kQueryLutErr) {
        if (!g->dev.lut_ptr) {
            *err = "the mixture lookup table is not on the device (mg_lut_build)";
            return MG_ESTATE;
        }
        A.lut_ptr = g->dev.lut_ptr;
        A.lut_seg = g->dev.lut_seg;
        A.lut_val = g->dev.lut_val;
    }
    if (variant == kQueryLutErr) {
        if (!g->dev.lut_err) {
            *err = "uncertainties need a graph with quantized weights (mg_quantize) and its lookup table";
            return MG_ESTATE;
        }
        if (sp || g->nseg > kSegLdsMax) {
            *err = "uncertainty queries keep per-source arrays in LDS: at most " + std::to_string(kSegLdsMax) +
                   " sources, dense output";
            return MG_ELIMIT;
        }
        A.lut_err = g->dev.lut_err;
        A.out_err = out_err;
        // every internal node is a table entry, so each node's count meets its row's uncertainty once
        A.gv.r1_end = A.gv.r2_end = g->nseg;
        variant = kQueryLut;
    }
    // sources in LDS arrays while they fit, else as table entries (sparse mode)
    const bool sparse = sp != nullptr || g->nseg > kSegLdsMax;
    A.lt.use16 = (!sparse && g->dev.maps16) ? 1u : 0u;
    // row runs where the graph has them, for slabs whose rows are long enough
    const uint32_t run_min = g->dev.cfg.run_min_row ? g->dev.cfg.run_min_row : kRunMinRow;
    A.lt.runs_mask = run_min == 0xFFFFFFFFu ? 0u : g->dev.runs_mask;
    A.lt.run_min = run_min;
    A.runs = static_cast<const RunLevel *>(g->dev.run_table);
    if (A.out_err) return launch_query<false, true>(g, A, w, lt, n, s, variant, err);
    return sparse ? launch_query<true, false>(g, A, w, lt, n, s, variant, err)
                  : launch_query<false, false>(g, A, w, lt, n, s, variant, err);
}

}  // namespace

int dev_query(Graph *g, const uint32_t *boxes, uint32_t n, float *out, const SparseOut *sp, void *work,
              uint64_t bytes, void *stream, int variant, uint32_t *stats, std::string *err, float *out_err)
{
    DeviceGuard guard;
    int rc = check_device(g, err);
    if (rc) return rc;
    const uint64_t need = dev_workspace_bytes(*g, n);
    if (bytes < need) {
        *err = "workspace of " + std::to_string(bytes) + " bytes is smaller than the " + std::to_string(need) +
               " bytes that " + std::to_string(n) + " boxes need";
        return MG_EINVAL;
    }
    const Workspace w = carve(*g, static_cast<char *>(work), n);
    return query_in(g, boxes, n, out, sp, w, static_cast<hipStream_t>(stream), variant, stats, err, out_err);
}

int dev_query_noalloc(Graph *g, const uint32_t *boxes, uint32_t n, float *out, void *stream, std::string *err)
{
    DeviceGuard guard;
    int rc = check_device(g, err);
    if (rc) return rc;
    ScratchSlot *sl = nullptr;
    if ((rc = scratch_slot(g->dev.device, &sl, err))) return rc;
    // as many workers of the final global tables as fit beside the per-box arrays (at least
    // one), none with mid-size tables (a speed-up only: every box fits the final tables)
    uint32_t workers = fallback_workers(*g);
    while (workers > 1 && carve(*g, nullptr, n, workers, 0).bytes > kScratchBytes) --workers;
    const Workspace probe = carve(*g, nullptr, n, workers, 0);
    if (probe.bytes > kScratchBytes) {
        const uint64_t fixed = carve(*g, nullptr, 1, 1, 0).bytes;
        *err = fixed > kScratchBytes
                   ? "mg_query_boxes_noalloc: the graph's global fallback table (" + std::to_string(fixed) +
                         " bytes for " + std::to_string(g->n_nodes) + " nodes) exceeds the " +
                         std::to_string(kScratchBytes) + "-byte scratch"
                   : "mg_query_boxes_noalloc: " + std::to_string(n) + " boxes exceed the " +
                         std::to_string(kScratchBytes) + "-byte scratch (at most " +
                         std::to_string((kScratchBytes - fixed) / 20) + " boxes on this graph)";
        return MG_ELIMIT;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Workspace w = carve(*g, sl->ptr, n, workers, 0);
    // the scratch keeps the last call's contents; every query leaves the fallback
    // tables clean, so they are cleared only when their layout changes
    const uint64_t layout[3] = {g->nseg, fallback_slots(*g), workers};
    if (std::memcmp(layout, sl->layout, sizeof(layout)) != 0) {
        clear_fallback_tables(*g, w, s);
        HIP_TRY(hipGetLastError());
        std::memcpy(sl->layout, layout, sizeof(layout));
    }
    const bool timing = g->dev.timing;
    g->dev.timing = false;  // no events are created on this path
    rc = query_in(g, boxes, n, out, nullptr, w, s, kQueryBatched, nullptr, err, nullptr);
    g->dev.timing = timing;
    return rc;
}

int dev_footprint(Graph *g, const uint32_t *boxes, uint32_t n, uint32_t *level_counts, uint32_t *cubes, uint32_t cap,
                  uint32_t *count, void *stream, std::string *err)
{
    DeviceGuard guard;
    int rc = check_device(g, err);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const LevelTable lt = level_table(*g);
    hipLaunchKernelGGL(footprint_kernel, dim3(n), dim3(kBlock), 0, s, lt, boxes, n, g->dev.maps, level_counts, cubes,
                       cap, count);
    HIP_TRY(hipGetLastError());
    return MG_OK;
}

int dev_nnz_bound(Graph *g, const uint32_t *boxes, uint32_t n, uint32_t *bound, void *stream, std::string *err)
{
    DeviceGuard guard;
    int rc = check_device(g, err);
    if (rc) return rc;
    const LevelTable lt = level_table(*g);
    const uint32_t per = kBlock / 64;
    hipLaunchKernelGGL(nnz_bound_kernel, dim3((n + per - 1) / per), dim3(kBlock), 0, static_cast<hipStream_t>(stream),
                       lt, boxes, n, g->dev.maps, g->dev.mixlen, g->nseg, g->quant_bits == 0 ? 1u : 0u, bound);
    HIP_TRY(hipGetLastError());
    return MG_OK;
}

int dev_propagate_tf(Graph *g, const uint8_t *tf, uint32_t T, float *out, void *stream, std::string *err)
{
    DeviceGuard guard;
    int rc = check_device(g, err);
    if (rc) return rc;
    if (T > 65535) {
        *err = "at most 65535 transfer functions per call";
        return MG_ELIMIT;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    float4 *o = reinterpret_cast<float4 *>(out);
    // the timed region is the whole frame: sources, then every step
    rc = timing_begin(g, s, err);
    if (rc) return rc;
    const uint32_t tb = g->dev.cfg.tf_block;
    const uint32_t P = std::min<uint32_t>(g->dev.cfg.tf_planes ? g->dev.cfg.tf_planes : kTfPlanes, T);
    const uint32_t P2 = P >= 8 ? 8u : P >= 4 ? 4u : P >= 2 ? 2u : 1u;  // planes per thread
    using StepKernel = void (*)(const NodeTriple *, const SchedNode *, uint32_t, uint32_t, uint32_t, uint32_t,
                                const uchar4 *, uint32_t, float4 *);
    // the order: ranks (default) or the graph's deferred step schedule
    const bool ranks = g->dev.cfg.tf_schedule == 0;
    const std::vector<uint32_t> &ptr = ranks ? g->rank_ptr : g->step_ptr;
    auto pick = [&](bool first) -> StepKernel {
#define MG_TF_STEP(F, R)                                                                                       \
    (P2 == 8 ? tf_step_kernel<8, F, R> : P2 == 4 ? tf_step_kernel<4, F, R> : P2 == 2 ? tf_step_kernel<2, F, R> \
                                                                           : tf_step_kernel<1, F, R>)
        if (ranks) return first ? MG_TF_STEP(true, true) : MG_TF_STEP(false, true);
        return first ? MG_TF_STEP(true, false) : MG_TF_STEP(false, false);
#undef MG_TF_STEP
    };
    const uchar4 *tf4 = reinterpret_cast<const uchar4 *>(tf);
    const uint32_t D = g->depth;
    auto step_size = [&](uint32_t st) { return ptr[st + 1] - ptr[st]; };
    // the first launch takes steps 1 .. first_end - 1: in rank order ranks 1 and 2
    const uint32_t first_end = (ranks && D >= 2) ? 3u : 2u;
    // trailing small steps (two or more) go to the one-workgroup kernel
    uint32_t tail0 = D + 1;
    while (tail0 > first_end && D + 2 - tail0 <= kTfTailSteps && uint64_t(step_size(tail0 - 1)) * T <= kTfTailPairs)
        --tail0;
    if (D + 1 - tail0 < 2) tail0 = D + 1;
    // the first launch (possibly empty) with the sources' colours, then the other steps
    const uint32_t n1 = D >= 1 ? ptr[first_end] - ptr[1] : 0u;
    hipLaunchKernelGGL(pick(true), dim3((n1 + g->nseg + tb - 1) / tb, (T + P2 - 1) / P2), dim3(tb), 0, s,
                       g->dev.nodes, g->dev.sched, g->nseg, g->nseg + n1, g->n_nodes, T, tf4, g->nseg, o);
    HIP_TRY(hipGetLastError());
    for (uint32_t st = first_end; st < tail0; ++st) {
        const uint32_t lo = ptr[st], hi = ptr[st + 1];
        if (hi <= lo) continue;
        hipLaunchKernelGGL(pick(false), dim3((hi - lo + tb - 1) / tb, (T + P2 - 1) / P2), dim3(tb), 0, s,
                           g->dev.nodes, g->dev.sched, lo, hi, g->n_nodes, T, tf4, g->nseg, o);
        HIP_TRY(hipGetLastError());
    }
    if (tail0 <= D) {
        TfTail tail;
        tail.n_steps = D + 1 - tail0;
        for (uint32_t k = 0; k <= tail.n_steps; ++k) tail.lo[k] = ptr[tail0 + k];
        hipLaunchKernelGGL(ranks ? tf_tail_kernel<true> : tf_tail_kernel<false>, dim3(1), dim3(kTfTailBlock), 0, s,
                           g->dev.nodes, g->dev.sched, tail, g->n_nodes, T, o);
        HIP_TRY(hipGetLastError());
    }
    return timing_end(g, s, err);
}

int dev_set_launch(Graph *g, const mg_launch_cfg *cfg, std::string *err)
{
    if (cfg->chunk_small > 64) {
        *err = "mg_set_launch: chunk_small must be in [0, 64]";
        return MG_EINVAL;
    }
    if (!(cfg->block_small == 0 || cfg->block_small == 128 || cfg->block_small == 256) ||
        !(cfg->block_big == 0 || cfg->block_big == 256 || cfg->block_big == 512)) {
        *err = "mg_set_launch: block_small must be 0, 128 or 256 and block_big 0, 256 or 512";
        return MG_EINVAL;
    }
    for (uint32_t t : {cfg->table_big, cfg->table_small, cfg->table_retry})
        if (t != 0 && (t < 64 || t > 8192 || (t & (t - 1)) != 0)) {
            *err = "mg_set_launch: table sizes must be 0 or a power of two in [64, 8192]";
            return MG_EINVAL;
        }
    if (!(cfg->tf_planes == 0 || cfg->tf_planes == 1 || cfg->tf_planes == 2 || cfg->tf_planes == 4 ||
          cfg->tf_planes == 8) || cfg->tf_schedule > 1) {
        *err = "mg_set_launch: tf_planes must be 0, 1, 2, 4 or 8 and tf_schedule 0 or 1";
        return MG_EINVAL;
    }
    const uint32_t tb = cfg->tf_block;
    if (!valid_unroll(cfg->unroll_big) || !valid_unroll(cfg->unroll_small) || !valid_unroll(cfg->unroll_naive) ||
        !(tb == 64 || tb == 128 || tb == 256 || tb == 512 || tb == 1024)) {
        *err = "mg_set_launch: unroll must be 4, 8 or 16 and tf_block a power of two in [64, 1024]";
        return MG_EINVAL;
    }
    g->dev.cfg = *cfg;
    return MG_OK;
}

int dev_autotune(Graph *g, const uint32_t *boxes, uint32_t n, float *out, void *work, uint64_t bytes, uint32_t reps,
                 void *stream, mg_launch_cfg *chosen, std::string *err)
{
    DeviceGuard guard;
    int rc = check_device(g, err);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const mg_launch_cfg saved = g->dev.cfg;
    const bool timing = g->dev.timing;
    g->dev.timing = false;
    auto time_variant = [&](int variant, float *best_ms) -> int {
        float best = 1e30f;
        for (uint32_t r = 0; r <= reps; ++r) {  // the first run warms up
            HIP_TRY(hipEventRecord(e0, s));
            int rc2 = dev_query(g, boxes, n, out, nullptr, work, bytes, stream, variant, nullptr, err);
            if (rc2) return rc2;
            HIP_TRY(hipEventRecord(e1, s));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (r > 0) best = std::min(best, ms);
        }
        *best_ms = best;
        return MG_OK;
    };
    const uint32_t us[3] = {4, 8, 16};
    mg_launch_cfg best_cfg = saved;
    float best = 1e30f;
    for (uint32_t ub : us)
        for (uint32_t usm : us) {
            g->dev.cfg.unroll_big = ub;
            g->dev.cfg.unroll_small = usm;
            float ms = 0;
            if ((rc = time_variant(kQueryBatched, &ms))) break;
            if (ms < best) best = ms, best_cfg.unroll_big = ub, best_cfg.unroll_small = usm;
        }
    // table sizes (LDS per workgroup, hence occupancy), one tier at a time
    const uint32_t tb[3] = {1024, 2048, 4096}, ts[3] = {256, 512, 1024};
    for (uint32_t bbg : {512u, 256u})
        for (uint32_t t : tb) {
            if (rc) break;
            g->dev.cfg = best_cfg;
            g->dev.cfg.table_big = t;
            g->dev.cfg.block_big = bbg;
            float ms = 0;
            if ((rc = time_variant(kQueryBatched, &ms))) break;
            if (ms < best) best = ms, best_cfg.table_big = t, best_cfg.block_big = bbg;
        }
    for (uint32_t bsm : {128u, 256u})
        for (uint32_t t : ts) {
            if (rc) break;
            g->dev.cfg = best_cfg;
            g->dev.cfg.table_small = t;
            g->dev.cfg.block_small = bsm;
            float ms = 0;
            if ((rc = time_variant(kQueryBatched, &ms))) break;
            if (ms < best) best = ms, best_cfg.table_small = t, best_cfg.block_small = bsm;
        }
    for (uint32_t c : {0u, 2u, 4u}) {
        if (rc) break;
        g->dev.cfg = best_cfg;
        g->dev.cfg.chunk_small = c;
        float ms = 0;
        if ((rc = time_variant(kQueryBatched, &ms))) break;
        if (ms < best) best = ms, best_cfg.chunk_small = c;
    }
    // shortest row summed from runs (where the graph keeps runs)
    for (uint32_t m : {64u, 256u}) {
        if (rc || !g->dev.runs_mask) break;
        g->dev.cfg = best_cfg;
        g->dev.cfg.run_min_row = m;
        float ms = 0;
        if ((rc = time_variant(kQueryBatched, &ms))) break;
        if (ms < best) best = ms, best_cfg.run_min_row = m;
    }
    float best_naive = 1e30f;
    for (uint32_t u : us) {
        if (rc) break;
        g->dev.cfg = best_cfg;
        g->dev.cfg.unroll_naive = u;
        float ms = 0;
        if ((rc = time_variant(kQueryNaive, &ms))) break;
        if (ms < best_naive) best_naive = ms, best_cfg.unroll_naive = u;
    }
    g->dev.timing = timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g->dev.cfg = rc ? saved : best_cfg;
    if (!rc && chosen) *chosen = best_cfg;
    return rc;
}

int dev_timing_enable(Graph *g, int enable, std::string *err)
{
    (void)err;
    g->dev.timing = enable != 0;
    return MG_OK;
}

int dev_timing_read(Graph *g, double *ms, uint32_t *launches, std::string *err)
{
    DeviceGuard guard;
    int rc = check_device(g, err);
    if (rc) return rc;
    double tot = 0;
    DeviceState &d = g->dev;
    for (uint32_t i = 0; i < d.ev_used; ++i) {
        HIP_TRY(hipEventSynchronize(static_cast<hipEvent_t>(d.ev_stop[i])));
        float t = 0;
        HIP_TRY(hipEventElapsedTime(&t, static_cast<hipEvent_t>(d.ev_start[i]), static_cast<hipEvent_t>(d.ev_stop[i])));
        tot += t;
    }
    *ms = tot;
    *launches = d.ev_used;
    d.ev_used = 0;
    return MG_OK;
}

int dev_check_load_addresses(const uint32_t dims[3], uint32_t flags, const uint32_t *boxes, uint32_t n,
                              uint32_t unroll, uint64_t counts[4], std::string *err)
{
    return check_load_addresses(dims, (flags & 1u) != 0, (flags & 2u) != 0, (flags & 4u) != 0, flags >> 8, boxes, n,
                                unroll, counts, err);
}

}  // namespace mg
