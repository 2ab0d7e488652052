// CPU construction of the Mixture Graph from a uint32 segment-ID volume.
//
// Paper sections followed (Al-Thelaya, Agus, Schneider, "The Mixture Graph"):
//  * Sec. "Normalized Histogram Mipmap", Eq. (mip): levels halve every axis
//    (rounding up) down to 1^3. A mip voxel holds the normalized histogram of
//    its level-0 support; here it is kept as integer counts reduced by their
//    gcd, so mixtures are compared exactly (border voxels are weighted by
//    their level-0 voxel counts).
//  * Sec. "Factorization": a mixture with k > 1 non-zero entries becomes
//    binary linear interpolations whose leaves are the segments (sources);
//    Sec. "Compression": identical nodes are re-used, which needs equal
//    mixtures, i.e. equal ratios. Every distinct mixture here is one node and
//    nodes are deduplicated on their exact reduced count vector.
//  * Sec. "Implementation Details": (i, j, w) and (j, i, 1 - w) are the same
//    interpolation; the orientation with w <= 1/2 is stored (the heavier part
//    is child a), ties broken by the lower node ID.
//  * Sec. "Reconstruction": topological level = 1 + max of the two
//    predecessors' levels (one linear scan, since predecessors are created
//    first); deferred scheduling of nodes whose successors are all at least
//    two levels up, filling each step to at least ceil(N / depth) nodes.
//
// How a mixture is split differs from the paper's greedy pair search (max
// occurrence / max reduction over all mixtures): the segments of a mixture,
// in increasing segment order, are halved recursively, so every node's
// sub-tree has exactly k - 1 internal nodes and depth ceil(log2 k). This keeps
// the graph shallow (fewer synchronisation steps, smaller fp32 error in the
// push) and the closure of any node exactly its own sub-tree.
//
// Mip voxels are not materialised as mixtures: a voxel whose children all
// hold the same node holds that node too (a sum of proportional count
// vectors is proportional); only voxels with differing children merge their
// children's reduced count vectors, scaled back to voxel counts.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <functional>
#include <numeric>
#include <thread>
#include <unordered_map>
#include <cmath>

#include "mg_internal.hpp"

namespace mg {

unsigned resolve_threads(uint32_t t)
{
    unsigned hw = std::thread::hardware_concurrency();
    if (hw == 0) hw = 1;
    return t == 0 ? hw : std::min<unsigned>(t, 4 * hw);
}

namespace {

constexpr uint32_t kMixed = 0xFFFFFFFFu;

// Run fn(begin, end, worker) over [0, n) in `nt` contiguous chunks, in order.
void parallel_chunks(uint64_t n, unsigned nt, const std::function<void(uint64_t, uint64_t, unsigned)> &fn)
{
    if (n == 0) return;
    if (nt <= 1 || n < 4096) {
        fn(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    const uint64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        const uint64_t b = t * chunk, e = std::min<uint64_t>(n, b + chunk);
        if (b >= e) break;
        th.emplace_back(fn, b, e, t);
    }
    for (auto &x : th) x.join();
}

inline uint64_t mix64(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}

uint64_t hash_mixture(const uint32_t *seg, const uint64_t *cnt, uint32_t k)
{
    uint64_t h = 0x9E3779B97F4A7C15ULL ^ k;
    for (uint32_t i = 0; i < k; ++i) {
        h = mix64(h ^ (uint64_t(seg[i]) * 0x100000001B3ULL));
        h = mix64(h ^ cnt[i]);
    }
    return h | 1;  // 0 marks an empty hash slot
}

uint64_t gcd64(uint64_t a, uint64_t b)
{
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Node store during construction: reduced mixtures, DAG edges, and a hash
// index from mixture to node ID. Sources are nodes 0 .. S-1.
class NodeStore {
public:
    explicit NodeStore(uint32_t nseg)
    {
        off_.reserve(nseg + 1);
        off_.push_back(0);
        for (uint32_t s = 0; s < nseg; ++s) {
            seg_.push_back(s);
            cnt_.push_back(1);
            off_.push_back(seg_.size());
            total_.push_back(1);
            a_.push_back(s);
            b_.push_back(s);
            wn_.push_back(0);
            wd_.push_back(1);
        }
        rehash(1024);
    }

    uint32_t size() const { return uint32_t(total_.size()); }
    uint64_t total(uint32_t n) const { return total_[n]; }
    uint32_t len(uint32_t n) const { return uint32_t(off_[n + 1] - off_[n]); }
    const uint32_t *seg(uint32_t n) const { return seg_.data() + off_[n]; }
    const uint64_t *cnt(uint32_t n) const { return cnt_.data() + off_[n]; }

    // Node of a reduced, segment-sorted count vector, or kMixed if absent (read only).
    uint32_t find(const uint32_t *s, const uint64_t *c, uint32_t k, uint64_t h) const
    {
        if (k == 1) return s[0];
        const uint64_t mask = hkey_.size() - 1;
        for (uint64_t i = h & mask;; i = (i + 1) & mask) {
            if (hkey_[i] == 0) return kMixed;
            if (hkey_[i] == h) {
                const uint32_t n = hval_[i];
                if (len(n) == k && std::equal(s, s + k, seg(n)) && std::equal(c, c + k, cnt(n))) return n;
            }
        }
    }

    // Node of a reduced, segment-sorted count vector; factor it if new.
    uint32_t get(const uint32_t *s, const uint64_t *c, uint32_t k)
    {
        if (k == 1) return s[0];
        const uint64_t h = hash_mixture(s, c, k);
        const uint32_t f = find(s, c, k, h);
        if (f != kMixed) return f;
        return make(s, c, k, h);
    }

    uint64_t nbytes_mix() const { return seg_.size() * 12; }

    std::vector<uint32_t> a_, b_;
    std::vector<uint64_t> wn_, wd_;

private:
    // Split the k >= 2 entries into the first floor(k/2) and the rest.
    uint32_t make(const uint32_t *s, const uint64_t *c, uint32_t k, uint64_t h)
    {
        // own copies: the recursion below may grow storage that s / c point into
        const std::vector<uint32_t> ss(s, s + k);
        const std::vector<uint64_t> cc(c, c + k);
        const uint32_t hl = k / 2, hr = k - hl;
        uint64_t tl = 0, tr = 0, gl = 0, gr = 0;
        for (uint32_t i = 0; i < hl; ++i) tl += cc[i], gl = gcd64(gl, cc[i]);
        for (uint32_t i = hl; i < k; ++i) tr += cc[i], gr = gcd64(gr, cc[i]);
        std::vector<uint64_t> red(k);
        for (uint32_t i = 0; i < hl; ++i) red[i] = cc[i] / gl;
        for (uint32_t i = hl; i < k; ++i) red[i] = cc[i] / gr;
        const uint32_t nl = get(ss.data(), red.data(), hl);
        const uint32_t nr = get(ss.data() + hl, red.data() + hl, hr);
        uint32_t a, b;
        uint64_t wn;
        if (tl > tr || (tl == tr && nl < nr)) {
            a = nl, b = nr, wn = tr;
        } else {
            a = nr, b = nl, wn = tl;
        }
        const uint64_t wd = tl + tr;
        const uint64_t g = gcd64(wn, wd);
        const uint32_t id = size();
        seg_.insert(seg_.end(), ss.begin(), ss.end());
        cnt_.insert(cnt_.end(), cc.begin(), cc.end());
        off_.push_back(seg_.size());
        total_.push_back(wd);
        a_.push_back(a);
        b_.push_back(b);
        wn_.push_back(wn / g);
        wd_.push_back(wd / g);
        insert(h, id);
        return id;
    }

    void insert(uint64_t h, uint32_t id)
    {
        if (2 * (++used_) > hkey_.size()) rehash(hkey_.size() * 2);
        const uint64_t mask = hkey_.size() - 1;
        uint64_t i = h & mask;
        while (hkey_[i] != 0) i = (i + 1) & mask;
        hkey_[i] = h;
        hval_[i] = id;
    }

    void rehash(uint64_t cap)
    {
        std::vector<uint64_t> ok;
        std::vector<uint32_t> ov;
        ok.swap(hkey_);
        ov.swap(hval_);
        hkey_.assign(cap, 0);
        hval_.assign(cap, 0);
        const uint64_t mask = cap - 1;
        for (uint64_t j = 0; j < ok.size(); ++j) {
            if (ok[j] == 0) continue;
            uint64_t i = ok[j] & mask;
            while (hkey_[i] != 0) i = (i + 1) & mask;
            hkey_[i] = ok[j];
            hval_[i] = ov[j];
        }
    }

    std::vector<uint32_t> seg_;
    std::vector<uint64_t> cnt_;
    std::vector<uint64_t> off_;
    std::vector<uint64_t> total_;
    std::vector<uint64_t> hkey_;
    std::vector<uint32_t> hval_;
    uint64_t used_ = 0;
};

// Distinct IDs in increasing order and the compacted level-0 map.
int compact_ids(const uint32_t *ids, uint64_t nvox, unsigned nt, std::vector<uint32_t> *seg_ids,
                uint32_t *map0, std::string *err)
{
    uint32_t maxid = 0;
    {
        std::vector<uint32_t> mx(nt, 0);
        parallel_chunks(nvox, nt, [&](uint64_t b, uint64_t e, unsigned t) {
            uint32_t m = 0;
            for (uint64_t i = b; i < e; ++i) m = std::max(m, ids[i]);
            mx[t] = m;
        });
        for (uint32_t m : mx) maxid = std::max(maxid, m);
    }
    if (maxid < (1u << 26)) {
        // direct table
        std::vector<std::atomic<uint8_t>> seen(uint64_t(maxid) + 1);
        for (auto &s : seen) s.store(0, std::memory_order_relaxed);
        parallel_chunks(nvox, nt, [&](uint64_t b, uint64_t e, unsigned) {
            uint32_t last = 0xFFFFFFFFu;
            for (uint64_t i = b; i < e; ++i) {
                if (ids[i] == last) continue;
                last = ids[i];
                seen[last].store(1, std::memory_order_relaxed);
            }
        });
        std::vector<uint32_t> lut(uint64_t(maxid) + 1, 0);
        seg_ids->clear();
        for (uint64_t v = 0; v <= maxid; ++v)
            if (seen[v].load(std::memory_order_relaxed)) {
                lut[v] = uint32_t(seg_ids->size());
                seg_ids->push_back(uint32_t(v));
            }
        parallel_chunks(nvox, nt, [&](uint64_t b, uint64_t e, unsigned) {
            for (uint64_t i = b; i < e; ++i) map0[i] = lut[ids[i]];
        });
        return MG_OK;
    }
    // sparse IDs: per-chunk sorted distinct lists, merged; then binary search
    std::vector<std::vector<uint32_t>> parts(nt);
    parallel_chunks(nvox, nt, [&](uint64_t b, uint64_t e, unsigned t) {
        std::vector<uint32_t> v;
        uint32_t last = 0;
        bool have = false;
        for (uint64_t i = b; i < e; ++i) {
            if (have && ids[i] == last) continue;
            last = ids[i];
            have = true;
            v.push_back(last);
            if (v.size() > (1u << 20)) {
                std::sort(v.begin(), v.end());
                v.erase(std::unique(v.begin(), v.end()), v.end());
            }
        }
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        parts[t].swap(v);
    });
    seg_ids->clear();
    for (auto &p : parts) seg_ids->insert(seg_ids->end(), p.begin(), p.end());
    std::sort(seg_ids->begin(), seg_ids->end());
    seg_ids->erase(std::unique(seg_ids->begin(), seg_ids->end()), seg_ids->end());
    const std::vector<uint32_t> &sid = *seg_ids;
    parallel_chunks(nvox, nt, [&](uint64_t b, uint64_t e, unsigned) {
        for (uint64_t i = b; i < e; ++i)
            map0[i] = uint32_t(std::lower_bound(sid.begin(), sid.end(), ids[i]) - sid.begin());
    });
    (void)err;
    return MG_OK;
}

inline uint64_t extent(uint64_t i, unsigned lev, uint64_t dim)
{
    const uint64_t lo = i << lev, hi = std::min<uint64_t>((i + 1) << lev, dim);
    return hi - lo;
}

}  // namespace

void level_dims(const uint32_t dims[3], std::vector<uint32_t> *out)
{
    out->clear();
    uint32_t d[3] = {dims[0], dims[1], dims[2]};
    for (;;) {
        out->insert(out->end(), d, d + 3);
        if (d[0] <= 1 && d[1] <= 1 && d[2] <= 1) break;
        for (int a = 0; a < 3; ++a) d[a] = (d[a] + 1) / 2;
    }
}

// Topological levels (Sec. "Reconstruction"), the deferred step schedule, IDs
// renumbered by (rank, creation order) with sources fixed, and the mip voxels
// of levels >= 1 remapped to the new IDs (level 0 holds sources only).
int finalize_dag(const RawDag &d, bool defer, uint32_t max_depth, unsigned nt, Graph *g, std::string *err,
                 std::vector<uint32_t> *perm_out)
{
    const uint32_t N = uint32_t(d.a.size());
    std::vector<uint32_t> rank(N, 0);
    uint32_t depth = 0;
    for (uint32_t n = d.nseg; n < N; ++n) {
        rank[n] = std::max(rank[d.a[n]], rank[d.b[n]]) + 1;
        depth = std::max(depth, rank[n]);
    }
    if (max_depth && depth > max_depth) {
        *err = "graph depth " + std::to_string(depth) + " exceeds max_depth " + std::to_string(max_depth);
        return MG_EDEPTH;
    }
    uint32_t maxmix = 1;
    for (uint32_t n = d.nseg; n < N; ++n) maxmix = std::max(maxmix, d.mix[n]);
    // ---- step schedule
    std::vector<uint32_t> step(N, 0);
    if (defer && depth > 1) {
        std::vector<uint32_t> last(N, depth);  // sinks may run as late as the last step
        for (uint32_t n = d.nseg; n < N; ++n) {
            last[d.a[n]] = std::min(last[d.a[n]], rank[n] - 1);
            last[d.b[n]] = std::min(last[d.b[n]], rank[n] - 1);
        }
        // bucket[r][d]: not yet scheduled nodes of rank r whose window ends at d
        std::vector<std::vector<uint32_t>> by_rank(depth + 1);
        for (uint32_t n = d.nseg; n < N; ++n) by_rank[rank[n]].push_back(n);
        std::vector<std::vector<uint32_t>> pool(depth + 1);  // indexed by window end
        std::vector<size_t> head(depth + 1, 0);
        const uint64_t target = (uint64_t(N - d.nseg) + depth - 1) / depth;
        for (uint32_t s = 1; s <= depth; ++s) {
            for (uint32_t n : by_rank[s]) pool[last[n]].push_back(n);
            uint64_t taken = 0;
            for (uint32_t d = s; d <= depth; ++d) {
                auto &pl = pool[d];
                while (head[d] < pl.size() && (d == s || taken < target)) {
                    step[pl[head[d]++]] = s;
                    ++taken;
                }
                if (taken >= target && d > s) break;
            }
        }
    } else {
        for (uint32_t n = d.nseg; n < N; ++n) step[n] = rank[n];
    }

    // ---- renumber by (rank, creation order); sources keep 0 .. S-1. Nodes whose
    // predecessors are both sources (rank 1) are then one contiguous ID range.
    std::vector<uint32_t> cnt(depth + 2, 0);
    for (uint32_t n = d.nseg; n < N; ++n) cnt[rank[n]]++;
    g->rank_ptr.assign(depth + 2, 0);
    g->rank_ptr[0] = 0;
    g->rank_ptr[1] = d.nseg;
    for (uint32_t r = 1; r <= depth; ++r) g->rank_ptr[r + 1] = g->rank_ptr[r] + cnt[r];
    std::vector<uint32_t> pos(g->rank_ptr.begin(), g->rank_ptr.end());
    std::vector<uint32_t> perm(N);
    for (uint32_t n = 0; n < d.nseg; ++n) perm[n] = n;
    for (uint32_t n = d.nseg; n < N; ++n) perm[n] = pos[rank[n]]++;

    g->n_nodes = N;
    g->depth = depth;
    g->max_mixture = maxmix;
    g->child_a.assign(N, 0);
    g->child_b.assign(N, 0);
    g->alpha.assign(N, 0.f);
    g->wnum.assign(N, 0);
    g->wden.assign(N, 1);
    g->rank.assign(N, 0);
    g->step.assign(N, 0);
    for (uint32_t n = 0; n < N; ++n) {
        const uint32_t p = perm[n];
        g->child_a[p] = perm[d.a[n]];
        g->child_b[p] = perm[d.b[n]];
        g->wnum[p] = d.wn[n];
        g->wden[p] = d.wd[n];
        g->alpha[p] = n < d.nseg ? 0.f : (d.alpha.empty() ? float(double(d.wn[n]) / double(d.wd[n])) : d.alpha[n]);
        g->rank[p] = rank[n];
        g->step[p] = step[n];
    }
    g->node_sigma.clear();
    if (!d.sigma.empty()) {
        g->node_sigma.assign(N, 0.f);
        for (uint32_t n = 0; n < N; ++n) g->node_sigma[perm[n]] = d.sigma[n];
    }
    g->node_code.clear();
    if (!d.code.empty()) {
        g->node_code.assign(N, 0);
        for (uint32_t n = 0; n < N; ++n) g->node_code[perm[n]] = d.code[n];
    }
    // ---- execution order of the step schedule: sources, then step 1, 2, ...
    std::vector<uint32_t> scnt(depth + 2, 0);
    for (uint32_t n = d.nseg; n < N; ++n) scnt[g->step[n]]++;
    g->step_ptr.assign(depth + 2, 0);
    g->step_ptr[1] = d.nseg;
    for (uint32_t s = 1; s <= depth; ++s) g->step_ptr[s + 1] = g->step_ptr[s] + scnt[s];
    std::vector<uint32_t> spos(g->step_ptr.begin(), g->step_ptr.end());
    g->sched.assign(N, 0);
    for (uint32_t n = 0; n < d.nseg; ++n) g->sched[n] = n;
    for (uint32_t n = d.nseg; n < N; ++n) g->sched[spos[g->step[n]]++] = n;
    const uint64_t total = g->maps.size();
    if (total == g->lev_off[g->n_levels] && total > g->lev_off[1]) {  // maps on the host: renumber
        uint32_t *mp = g->maps.data();
        const uint64_t first_internal = g->lev_off[1];
        parallel_chunks(total - first_internal, nt, [&](uint64_t b, uint64_t e, unsigned) {
            for (uint64_t i = b; i < e; ++i) mp[first_internal + i] = perm[mp[first_internal + i]];
        });
    }
    if (perm_out) *perm_out = std::move(perm);
    return MG_OK;
}

int build_graph(const uint32_t *ids, const mg_build_opts *o, Graph *g, std::string *err)
{
    const uint64_t nx = o->nx, ny = o->ny, nz = o->nz;
    const uint64_t nvox = nx * ny * nz;
    const unsigned nt = resolve_threads(o->threads);
    g->dims[0] = o->nx, g->dims[1] = o->ny, g->dims[2] = o->nz;
    level_dims(g->dims, &g->lev_dims);
    g->n_levels = uint32_t(g->lev_dims.size() / 3);
    if (g->n_levels > MG_MAX_LEVELS) {
        *err = "too many mip levels";
        return MG_ELIMIT;
    }
    g->lev_off.assign(g->n_levels + 1, 0);
    for (uint32_t l = 0; l < g->n_levels; ++l)
        g->lev_off[l + 1] = g->lev_off[l] +
                            uint64_t(g->lev_dims[3 * l]) * g->lev_dims[3 * l + 1] * g->lev_dims[3 * l + 2];
    try {
        g->maps.assign(g->lev_off[g->n_levels], 0);
    } catch (...) {
        *err = "host allocation of the node maps failed";
        return MG_ENOMEM;
    }
    int rc = compact_ids(ids, nvox, nt, &g->seg_ids, g->maps.data(), err);
    if (rc) return rc;
    g->nseg = uint32_t(g->seg_ids.size());

    NodeStore store(g->nseg);

    for (uint32_t l = 1; l < g->n_levels; ++l) {
        const uint64_t px = g->lev_dims[3 * (l - 1)], py = g->lev_dims[3 * (l - 1) + 1],
                       pz = g->lev_dims[3 * (l - 1) + 2];
        const uint64_t cx = g->lev_dims[3 * l], cy = g->lev_dims[3 * l + 1], cz = g->lev_dims[3 * l + 2];
        const uint32_t *prev = g->maps.data() + g->lev_off[l - 1];
        uint32_t *cur = g->maps.data() + g->lev_off[l];
        const uint64_t ncur = cx * cy * cz;

        // pass A: voxels whose children share one node inherit it
        std::vector<std::vector<uint64_t>> mixed_parts(nt);
        parallel_chunks(ncur, nt, [&](uint64_t b, uint64_t e, unsigned t) {
            auto &mp = mixed_parts[t];
            for (uint64_t v = b; v < e; ++v) {
                const uint64_t x = v % cx, y = (v / cx) % cy, z = v / (cx * cy);
                uint32_t first = kMixed;
                bool same = true;
                for (int dz = 0; dz < 2 && same; ++dz) {
                    const uint64_t zz = 2 * z + dz;
                    if (zz >= pz) break;
                    for (int dy = 0; dy < 2 && same; ++dy) {
                        const uint64_t yy = 2 * y + dy;
                        if (yy >= py) break;
                        for (int dx = 0; dx < 2; ++dx) {
                            const uint64_t xx = 2 * x + dx;
                            if (xx >= px) break;
                            const uint32_t n = prev[xx + px * (yy + py * zz)];
                            if (first == kMixed) first = n;
                            else if (n != first) { same = false; break; }
                        }
                    }
                }
                if (same) cur[v] = first;
                else { cur[v] = kMixed; mp.push_back(v); }
            }
        });
        std::vector<uint64_t> mixed;
        for (auto &p : mixed_parts) mixed.insert(mixed.end(), p.begin(), p.end());
        mixed_parts.clear();
        if (mixed.empty()) continue;

        // pass B: reduced count vector of every mixed voxel (read-only on the store)
        struct Rec { uint64_t off; uint32_t k; uint64_t h; };
        const unsigned nparts = std::min<unsigned>(nt, unsigned((mixed.size() + 1023) / 1024));
        std::vector<std::vector<uint32_t>> bseg(std::max(1u, nparts));
        std::vector<std::vector<uint64_t>> bcnt(std::max(1u, nparts));
        std::vector<Rec> recs(mixed.size());
        std::vector<uint32_t> part_of(mixed.size());
        parallel_chunks(mixed.size(), std::max(1u, nparts), [&](uint64_t b, uint64_t e, unsigned t) {
            std::vector<std::pair<uint32_t, uint64_t>> acc;
            auto &S = bseg[t];
            auto &C = bcnt[t];
            for (uint64_t i = b; i < e; ++i) {
                const uint64_t v = mixed[i];
                const uint64_t x = v % cx, y = (v / cx) % cy, z = v / (cx * cy);
                uint32_t cn[8];
                uint64_t cw[8];
                int nc = 0;
                for (int dz = 0; dz < 2; ++dz) {
                    const uint64_t zz = 2 * z + dz;
                    if (zz >= pz) break;
                    for (int dy = 0; dy < 2; ++dy) {
                        const uint64_t yy = 2 * y + dy;
                        if (yy >= py) break;
                        for (int dx = 0; dx < 2; ++dx) {
                            const uint64_t xx = 2 * x + dx;
                            if (xx >= px) break;
                            const uint32_t n = prev[xx + px * (yy + py * zz)];
                            const uint64_t nvx = extent(xx, l - 1, nx) * extent(yy, l - 1, ny) * extent(zz, l - 1, nz);
                            int j = 0;
                            while (j < nc && cn[j] != n) ++j;
                            if (j == nc) { cn[nc] = n; cw[nc] = 0; ++nc; }
                            cw[j] += nvx;
                        }
                    }
                }
                acc.clear();
                for (int j = 0; j < nc; ++j) {
                    const uint32_t n = cn[j];
                    const uint64_t scale = cw[j] / store.total(n);  // voxels / reduced total
                    const uint32_t k = store.len(n);
                    const uint32_t *sg = store.seg(n);
                    const uint64_t *ct = store.cnt(n);
                    for (uint32_t q = 0; q < k; ++q) acc.emplace_back(sg[q], ct[q] * scale);
                }
                std::sort(acc.begin(), acc.end());
                const uint64_t off = S.size();
                uint64_t gg = 0;
                for (size_t q = 0; q < acc.size();) {
                    size_t r = q;
                    uint64_t s = 0;
                    while (r < acc.size() && acc[r].first == acc[q].first) s += acc[r++].second;
                    S.push_back(acc[q].first);
                    C.push_back(s);
                    gg = gcd64(gg, s);
                    q = r;
                }
                const uint32_t k = uint32_t(S.size() - off);
                for (uint32_t q = 0; q < k; ++q) C[off + q] /= gg;
                recs[i] = Rec{off, k, hash_mixture(S.data() + off, C.data() + off, k)};
                part_of[i] = t;
            }
        });

        // pass C1: parallel lookup of mixtures that already have a node
        parallel_chunks(mixed.size(), nt, [&](uint64_t b, uint64_t e, unsigned) {
            for (uint64_t i = b; i < e; ++i) {
                const Rec &r = recs[i];
                const unsigned t = part_of[i];
                cur[mixed[i]] = store.find(bseg[t].data() + r.off, bcnt[t].data() + r.off, r.k, r.h);
            }
        });
        // pass C2: create the missing ones in voxel order (deterministic IDs)
        for (uint64_t i = 0; i < mixed.size(); ++i) {
            if (cur[mixed[i]] != kMixed) continue;
            const Rec &r = recs[i];
            const unsigned t = part_of[i];
            cur[mixed[i]] = store.get(bseg[t].data() + r.off, bcnt[t].data() + r.off, r.k);
        }
    }

    if (o->factorizer != MG_FACTOR_HALVING) {
        // the distinct mixtures the maps hold, in scanline order of first
        // appearance (level by level, x fastest), refactored greedily
        const uint32_t S = g->nseg;
        std::vector<uint32_t> slot(store.size(), kMixed);
        std::vector<std::vector<std::pair<uint32_t, uint64_t>>> mix;
        uint32_t *mp = g->maps.data();
        const uint64_t first_internal = g->lev_off[1], total = g->maps.size();
        for (uint64_t i = first_internal; i < total; ++i) {
            const uint32_t n = mp[i];
            if (n < S || slot[n] != kMixed) continue;
            slot[n] = uint32_t(mix.size());
            std::vector<std::pair<uint32_t, uint64_t>> h(store.len(n));
            for (uint32_t q = 0; q < store.len(n); ++q) h[q] = {store.seg(n)[q], store.cnt(n)[q]};
            mix.push_back(std::move(h));
        }
        RawDag dag;
        std::vector<uint32_t> root;
        if (int rc = greedy_factorize(S, mix, o->factorizer, o->tau, &dag, &root, err)) return rc;
        parallel_chunks(total - first_internal, nt, [&](uint64_t b, uint64_t e, unsigned) {
            for (uint64_t i = first_internal + b; i < first_internal + e; ++i)
                if (mp[i] >= S) mp[i] = root[slot[mp[i]]];
        });
        return finalize_dag(dag, o->defer != 0, o->max_depth, nt, g, err);
    }

    // ---- ranks, step schedule, numbering by rank, remapped mip voxels
    RawDag dag;
    dag.nseg = g->nseg;
    const uint32_t N = store.size();
    dag.a.assign(store.a_.begin(), store.a_.begin() + N);
    dag.b.assign(store.b_.begin(), store.b_.begin() + N);
    dag.wn.assign(store.wn_.begin(), store.wn_.begin() + N);
    dag.wd.assign(store.wd_.begin(), store.wd_.begin() + N);
    dag.mix.resize(N);
    for (uint32_t n = 0; n < N; ++n) dag.mix[n] = n < g->nseg ? 1u : store.len(n);
    if (int rc = finalize_dag(dag, o->defer != 0, o->max_depth, nt, g, err)) return rc;
    return MG_OK;
}

// The exact fraction of an fp32 weight: c = fr 2^e with a 24-bit fr.
void weight_fraction(float c, uint64_t *num, uint64_t *den)
{
    int e = 0;
    const float fr = std::frexp(c, &e);  // c = fr 2^e, fr in [1/2, 1)
    uint64_t n = uint64_t(std::ldexp(double(fr), 24)), d = uint64_t(1) << (24 - e);
    while (n % 2 == 0 && d > 1) n /= 2, d /= 2;
    *num = n, *den = d;
}

// Scalar quantization of the interpolation weights (Sec. "Compression": the
// open range (0, 1) is cut into 2^b equal bins, each represented by one
// codeword, with the empirical standard deviation of the weights in the bin
// kept for error estimates; Sec. "Implementation Details": both w and 1 - w
// are quantized and the orientation with the smaller error is kept). The
// codebook is learned from the graph's weights (w <= 1/2); a codeword is the
// mean of its bin's weights, an empty bin gets its midpoint and the standard
// deviation of a uniform bin; codewords and sigmas are then rounded to the
// 20-bit fields the graph stream stores them in (Table "bitstream", C). Nodes
// are visited children first; a node whose two (merged) predecessors coincide
// becomes that predecessor, and nodes with the same predecessors and codeword
// are merged (re-use, Sec. "Compression").
int quantize_graph(const Graph &src, uint32_t bits, uint32_t threads, Graph *dst, std::string *err)
{
    if (bits < 1 || bits > kMaxQuantBits) {
        *err = "quantizer bit rate must be in [1, " + std::to_string(kMaxQuantBits) + "]";
        return MG_EINVAL;
    }
    const uint32_t S = src.nseg, N = src.n_nodes, B = 1u << bits;
    auto bin = [&](double w) { return std::min<uint32_t>(uint32_t(w * B), B - 1); };
    std::vector<double> sum(B, 0.0), dev2(B, 0.0);
    std::vector<uint64_t> cnt(B, 0);
    for (uint32_t n = S; n < N; ++n) {
        const double w = double(src.wnum[n]) / double(src.wden[n]);
        const uint32_t k = bin(w);
        sum[k] += w, cnt[k]++;
    }
    for (uint32_t n = S; n < N; ++n) {  // second pass: squared deviations from the bin mean
        const double w = double(src.wnum[n]) / double(src.wden[n]);
        const uint32_t k = bin(w);
        const double dv = w - sum[k] / double(cnt[k]);
        dev2[k] += dv * dv;
    }
    // codewords and sigmas at the stream's 20-bit resolution: a codeword is the
    // nearest multiple of 2^-20 inside (0, 1); a sigma the nearest multiple of
    // sigma_max / (2^20 - 1), sigma_max being the largest sigma rounded to fp32
    const double scale = double(1u << kCodeBits), smax_q = double((1u << kCodeBits) - 1);
    std::vector<float> code(B), sig(B);
    std::vector<double> sd(B);
    for (uint32_t k = 0; k < B; ++k) {
        double mean;
        if (cnt[k]) {
            mean = sum[k] / double(cnt[k]);
            sd[k] = std::sqrt(dev2[k] / double(cnt[k]));
        } else {
            mean = (k + 0.5) / B;
            sd[k] = 1.0 / B / std::sqrt(12.0);
        }
        const double m = std::min(std::max(std::floor(mean * scale + 0.5), 1.0), scale - 1.0);
        code[k] = float(m / scale);
    }
    const float sigma_max = float(*std::max_element(sd.begin(), sd.end()));
    for (uint32_t k = 0; k < B; ++k) {
        const double m = sigma_max > 0.f ? std::min(std::floor(sd[k] / double(sigma_max) * smax_q + 0.5), smax_q) : 0.0;
        sig[k] = code_sigma_value(sigma_max, uint32_t(m));
    }
    RawDag d;
    d.nseg = S;
    std::vector<uint32_t> rep(N);
    for (uint32_t s = 0; s < S; ++s) {
        rep[s] = s;
        d.a.push_back(s), d.b.push_back(s), d.wn.push_back(0), d.wd.push_back(1), d.mix.push_back(1);
        d.alpha.push_back(0.f), d.sigma.push_back(0.f), d.code.push_back(0);
    }
    struct Key {
        uint32_t a, b, w;
        bool operator==(const Key &o) const { return a == o.a && b == o.b && w == o.w; }
    };
    struct KeyHash {
        size_t operator()(const Key &k) const
        {
            return size_t((uint64_t(k.a) * 0x9E3779B97F4A7C15ull) ^ (uint64_t(k.b) * 0xC2B2AE3D27D4EB4Full) ^ k.w);
        }
    };
    std::unordered_map<Key, uint32_t, KeyHash> made;
    for (uint32_t n = S; n < N; ++n) {  // IDs are sorted by rank: predecessors first
        const uint32_t x = rep[src.child_a[n]], y = rep[src.child_b[n]];
        if (x == y) {
            rep[n] = x;
            continue;
        }
        const double w = double(src.wnum[n]) / double(src.wden[n]);
        const uint32_t k1 = bin(w), k2 = bin(1.0 - w);
        const bool flip = std::fabs((1.0 - w) - code[k2]) < std::fabs(w - code[k1]);
        const uint32_t k = flip ? k2 : k1;
        uint32_t first = flip ? y : x, second = flip ? x : y;  // node = (1 - c) first + c second
        float c = code[k];
        if (c > 0.5f) std::swap(first, second), c = 1.0f - c;  // stored with w <= 1/2 (exact in fp32)
        uint32_t cbits;
        std::memcpy(&cbits, &c, 4);
        const Key key{first, second, cbits};
        auto it = made.find(key);
        if (it != made.end()) {
            rep[n] = it->second;
            continue;
        }
        const uint32_t id = uint32_t(d.a.size());
        made.emplace(key, id);
        rep[n] = id;
        uint64_t num = 0, den = 1;
        weight_fraction(c, &num, &den);
        d.a.push_back(first), d.b.push_back(second), d.wn.push_back(num), d.wd.push_back(den);
        d.mix.push_back(d.mix[first] + d.mix[second]);
        d.alpha.push_back(c), d.sigma.push_back(sig[k]), d.code.push_back(k);
    }
    dst->dims[0] = src.dims[0], dst->dims[1] = src.dims[1], dst->dims[2] = src.dims[2];
    dst->nseg = S;
    dst->n_levels = src.n_levels;
    dst->lev_dims = src.lev_dims;
    dst->lev_off = src.lev_off;
    dst->seg_ids = src.seg_ids;
    dst->maps = src.maps;
    const unsigned nt = resolve_threads(threads);
    uint32_t *mp = dst->maps.data();
    const uint64_t first_internal = dst->lev_off[1];
    parallel_chunks(dst->maps.size() - first_internal, nt, [&](uint64_t b, uint64_t e, unsigned) {
        for (uint64_t i = b; i < e; ++i) mp[first_internal + i] = rep[mp[first_internal + i]];
    });
    // the schedule of the source graph: deferred if its steps differ from its ranks
    const bool defer = src.step != src.rank;
    if (int rc = finalize_dag(d, defer, 0, nt, dst, err)) return rc;
    dst->quant_bits = bits;
    dst->codebook = std::move(code);
    dst->code_sigma = std::move(sig);
    return MG_OK;
}

int validate_graph(const Graph &g, std::string *err)
{
    const uint32_t N = g.n_nodes, S = g.nseg;
    if (S == 0 || N < S || g.child_a.size() != N || g.child_b.size() != N || g.alpha.size() != N ||
        g.wnum.size() != N || g.wden.size() != N || g.rank.size() != N || g.step.size() != N ||
        g.step_ptr.size() != size_t(g.depth) + 2 || g.seg_ids.size() != S) {
        *err = "graph arrays have inconsistent sizes";
        return MG_EFORMAT;
    }
    if (g.rank_ptr.size() != size_t(g.depth) + 2 || g.sched.size() != N) {
        *err = "rank_ptr / sched have inconsistent sizes";
        return MG_EFORMAT;
    }
    for (const std::vector<uint32_t> *ptr : {&g.step_ptr, &g.rank_ptr}) {
        const std::vector<uint32_t> &p = *ptr;
        if (p[0] != 0 || p[1] != S || p[g.depth + 1] != N) {
            *err = "step_ptr / rank_ptr do not delimit the nodes";
            return MG_EFORMAT;
        }
        for (uint32_t s = 0; s <= g.depth; ++s)
            if (p[s] > p[s + 1]) {
                *err = "step_ptr / rank_ptr are not monotone";
                return MG_EFORMAT;
            }
    }
    for (uint32_t s = 1; s < S; ++s)
        if (g.seg_ids[s] <= g.seg_ids[s - 1]) {
            *err = "segment IDs are not increasing";
            return MG_EFORMAT;
        }
    uint32_t rk = 1;
    for (uint32_t n = S; n < N; ++n) {
        while (n >= g.rank_ptr[rk + 1]) ++rk;
        const uint32_t a = g.child_a[n], b = g.child_b[n];
        if (a >= n || b >= n || a == b) {
            *err = "node " + std::to_string(n) + " has a predecessor that is not an earlier node";
            return MG_EFORMAT;
        }
        if (g.rank[n] != rk || g.rank[n] != std::max(g.rank[a], g.rank[b]) + 1) {
            *err = "node " + std::to_string(n) + " has an inconsistent topological level";
            return MG_EFORMAT;
        }
        if (g.step[n] < g.rank[n] || g.step[n] > g.depth || g.step[a] >= g.step[n] || g.step[b] >= g.step[n]) {
            *err = "node " + std::to_string(n) + " runs before one of its predecessors";
            return MG_EFORMAT;
        }
        if (g.wnum[n] == 0 || 2 * g.wnum[n] > g.wden[n]) {
            *err = "node " + std::to_string(n) + " has a weight outside (0, 1/2]";
            return MG_EFORMAT;
        }
        if (g.alpha[n] != float(double(g.wnum[n]) / double(g.wden[n]))) {
            *err = "node " + std::to_string(n) + " has an fp32 weight that does not match its ratio";
            return MG_EFORMAT;
        }
    }
    {
        std::vector<uint8_t> seen(N, 0);
        for (uint32_t st = 0; st <= g.depth; ++st)
            for (uint32_t i = g.step_ptr[st]; i < g.step_ptr[st + 1]; ++i) {
                const uint32_t n = g.sched[i];
                if (n >= N || seen[n] || (st == 0 ? n >= S : (n < S || g.step[n] != st))) {
                    *err = "sched is not the step order of the nodes";
                    return MG_EFORMAT;
                }
                seen[n] = 1;
            }
    }
    std::vector<uint32_t> ld;
    level_dims(g.dims, &ld);
    if (ld != g.lev_dims || g.n_levels != ld.size() / 3 || g.lev_off.size() != g.n_levels + 1 ||
        (!g.maps_on_device && g.maps.size() != g.lev_off[g.n_levels])) {
        *err = "level dimensions do not match the volume";
        return MG_EFORMAT;
    }
    if (g.maps_on_device) return MG_OK;  // the GPU decoder checks every voxel's node ID
    for (uint64_t i = 0; i < g.lev_off[1]; ++i)
        if (g.maps[i] >= S) {
            *err = "a level-0 voxel does not hold a source";
            return MG_EFORMAT;
        }
    for (uint64_t i = g.lev_off[1]; i < g.maps.size(); ++i)
        if (g.maps[i] >= N) {
            *err = "a mip voxel holds an out-of-range node";
            return MG_EFORMAT;
        }
    return MG_OK;
}

// Mixture lookup table (Sec. "Decoder", mixture lookup; used by range queries in
// Sec. "Range queries"): the mixture of every node over the segments, found by
// carrying the unit vector of each source through the interpolations in rank
// order, mu_n = (1 - w_n) mu_a + w_n mu_b, in fp64 from the exact rational
// weights, then stored as fp32. Rows list sources in increasing order. The
// paper also carries a variance per entry for quantized weights; the weights
// here are exact, so the variance would be zero and is not stored.
int build_lut(Graph *g, uint32_t threads, std::string *err)
{
    const uint32_t S = g->nseg, N = g->n_nodes;
    const unsigned nt = resolve_threads(threads);
    std::vector<uint64_t> ptr(uint64_t(N) + 1, 0);
    std::vector<uint32_t> seg(S);
    std::vector<double> val(S, 1.0);
    // propagated uncertainty of each entry (Sec. "Error Propagation", Eq. (error)):
    // with quantized weights, component i of node (1 - w) a + w b has
    // dmu_i = mu_i sqrt((da_i / a_i)^2 + (db_i / b_i)^2 + 2 (dw / w)^2), sources are
    // certain, and a term whose component is absent from a child counts zero
    const bool with_err = !g->node_sigma.empty();
    std::vector<double> unc(with_err ? S : 0, 0.0);
    for (uint32_t s = 0; s < S; ++s) {
        ptr[s] = s;
        seg[s] = s;
    }
    ptr[S] = S;
    const uint64_t kMaxEntries = uint64_t(1) << 34;
    for (uint32_t r = 1; r <= g->depth; ++r) {
        const uint32_t lo = g->rank_ptr[r], hi = g->rank_ptr[r + 1];
        std::vector<uint64_t> len(hi - lo);
        // entries of each row: the union of its two predecessors' rows (children have lower rank)
        parallel_chunks(hi - lo, nt, [&](uint64_t b, uint64_t e, unsigned) {
            for (uint64_t i = b; i < e; ++i) {
                const uint32_t n = lo + uint32_t(i);
                uint64_t pa = ptr[g->child_a[n]], ea = ptr[g->child_a[n] + 1];
                uint64_t pb = ptr[g->child_b[n]], eb = ptr[g->child_b[n] + 1];
                uint64_t k = 0;
                while (pa < ea || pb < eb) {
                    if (pb == eb || (pa < ea && seg[pa] < seg[pb])) ++pa;
                    else if (pa == ea || seg[pb] < seg[pa]) ++pb;
                    else ++pa, ++pb;
                    ++k;
                }
                len[i] = k;
            }
        });
        for (uint32_t i = 0; i < hi - lo; ++i) ptr[lo + i + 1] = ptr[lo + i] + len[i];
        if (ptr[hi] > kMaxEntries) {
            *err = "mixture lookup table beyond 2^34 entries";
            return MG_ELIMIT;
        }
        seg.resize(ptr[hi]);
        val.resize(ptr[hi]);
        if (with_err) unc.resize(ptr[hi]);
        parallel_chunks(hi - lo, nt, [&](uint64_t b, uint64_t e, unsigned) {
            for (uint64_t i = b; i < e; ++i) {
                const uint32_t n = lo + uint32_t(i);
                const double wb = double(g->wnum[n]) / double(g->wden[n]);
                const double wa = double(g->wden[n] - g->wnum[n]) / double(g->wden[n]);
                uint64_t pa = ptr[g->child_a[n]], ea = ptr[g->child_a[n] + 1];
                uint64_t pb = ptr[g->child_b[n]], eb = ptr[g->child_b[n] + 1];
                const double rw = with_err ? double(g->node_sigma[n]) / wb : 0.0;  // dw / w
                uint64_t k = ptr[n];
                while (pa < ea || pb < eb) {
                    double ra = 0.0, rb = 0.0;  // relative uncertainties of the children's components
                    if (pb == eb || (pa < ea && seg[pa] < seg[pb])) {
                        seg[k] = seg[pa];
                        val[k] = wa * val[pa];
                        if (with_err) ra = unc[pa] / val[pa];
                        ++pa;
                    } else if (pa == ea || seg[pb] < seg[pa]) {
                        seg[k] = seg[pb];
                        val[k] = wb * val[pb];
                        if (with_err) rb = unc[pb] / val[pb];
                        ++pb;
                    } else {
                        seg[k] = seg[pa];
                        val[k] = wa * val[pa] + wb * val[pb];
                        if (with_err) ra = unc[pa] / val[pa], rb = unc[pb] / val[pb];
                        ++pa, ++pb;
                    }
                    if (with_err) unc[k] = val[k] * std::sqrt(ra * ra + rb * rb + 2.0 * rw * rw);
                    ++k;
                }
            }
        });
    }
    g->lut_val.resize(val.size());
    for (size_t i = 0; i < val.size(); ++i) g->lut_val[i] = float(val[i]);
    g->lut_err.assign(unc.size(), 0.f);
    for (size_t i = 0; i < unc.size(); ++i) g->lut_err[i] = float(unc[i]);
    g->lut_seg = std::move(seg);
    g->lut_ptr = std::move(ptr);
    return MG_OK;
}

}  // namespace mg
