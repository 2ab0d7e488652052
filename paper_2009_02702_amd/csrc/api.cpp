// C ABI entry points (host side): argument checks, error strings, build,
// export, save/load. GPU work is delegated to kernels.hip.
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "mg_internal.hpp"

struct mg_graph {
    mg::Graph g;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int done(int code, const std::string &msg)
{
    if (code != MG_OK) g_err = msg;
    return code;
}

// ---- save / load: "MGRAPH01" + header + arrays, each followed by FNV-1a 64
constexpr char kMagic[8] = {'M', 'G', 'R', 'A', 'P', 'H', '0', '3'};

uint64_t fnv(const void *p, size_t n, uint64_t h = 0xcbf29ce484222325ULL)
{
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 0x100000001b3ULL;
    return h;
}

bool wr(FILE *f, const void *p, size_t n)
{
    return n == 0 || fwrite(p, 1, n, f) == n;
}

template <class T>
bool wr_vec(FILE *f, const std::vector<T> &v)
{
    const uint64_t n = v.size();
    const uint64_t h = fnv(v.data(), n * sizeof(T));
    return wr(f, &n, 8) && wr(f, v.data(), n * sizeof(T)) && wr(f, &h, 8);
}

bool rd(FILE *f, void *p, size_t n)
{
    return n == 0 || fread(p, 1, n, f) == n;
}

template <class T>
int rd_vec(FILE *f, std::vector<T> *v, uint64_t limit)
{
    uint64_t n = 0, h = 0;
    if (!rd(f, &n, 8)) return MG_EIO;
    if (n > limit) return MG_EFORMAT;
    try {
        v->resize(n);
    } catch (...) {
        return MG_ENOMEM;
    }
    if (!rd(f, v->data(), n * sizeof(T)) || !rd(f, &h, 8)) return MG_EIO;
    if (h != fnv(v->data(), n * sizeof(T))) return MG_EFORMAT;
    return MG_OK;
}

}  // namespace

extern "C" {

const char *mg_last_error(void) { return g_err.c_str(); }

int mg_build(const uint32_t *ids, const mg_build_opts *opts, mg_graph **out)
{
    if (!ids || !opts || !out) return fail(MG_EINVAL, "mg_build: null argument");
    *out = nullptr;
    if (opts->nx == 0 || opts->ny == 0 || opts->nz == 0) return fail(MG_EINVAL, "mg_build: zero dimension");
    const uint64_t nvox = uint64_t(opts->nx) * opts->ny * opts->nz;
    if (nvox >= (1ull << 31))
        return fail(MG_ELIMIT, "mg_build: volumes of 2^31 voxels or more are not supported (31-bit offsets)");
    for (uint32_t r : opts->reserved)
        if (r) return fail(MG_EINVAL, "mg_build: reserved fields must be 0");
    if (opts->defer > 1) return fail(MG_EINVAL, "mg_build: defer must be 0 or 1");
    if (opts->factorizer > MG_FACTOR_GREEDY_OCCURRENCE) return fail(MG_EINVAL, "mg_build: unknown factorizer");
    mg_graph *h = new (std::nothrow) mg_graph;
    if (!h) return fail(MG_ENOMEM, "mg_build: out of host memory");
    std::string err;
    int rc;
    try {
        rc = mg::build_graph(ids, opts, &h->g, &err);
    } catch (const std::bad_alloc &) {
        rc = MG_ENOMEM, err = "mg_build: out of host memory";
    } catch (const std::exception &e) {
        rc = MG_EINVAL, err = std::string("mg_build: ") + e.what();
    }
    if (rc != MG_OK) {
        delete h;
        return fail(rc, err);
    }
    *out = h;
    return MG_OK;
}

int mg_quantize(const mg_graph *h, uint32_t bits, uint32_t threads, mg_graph **out)
{
    if (!h || !out) return fail(MG_EINVAL, "mg_quantize: null argument");
    if (h->g.quant_bits) return fail(MG_EINVAL, "mg_quantize: the graph is already quantized");
    if (h->g.maps_on_device) return fail(MG_ESTATE, "mg_quantize: the node maps exist only on the device");
    *out = nullptr;
    mg_graph *q = new (std::nothrow) mg_graph;
    if (!q) return fail(MG_ENOMEM, "mg_quantize: out of host memory");
    std::string err;
    int rc;
    try {
        rc = mg::quantize_graph(h->g, bits, threads, &q->g, &err);
    } catch (const std::bad_alloc &) {
        rc = MG_ENOMEM, err = "mg_quantize: out of host memory";
    }
    if (rc != MG_OK) {
        delete q;
        return fail(rc, err);
    }
    *out = q;
    return MG_OK;
}

int mg_export_codebook(const mg_graph *h, float *codeword, float *sigma, float *node_sigma, uint32_t *node_code)
{
    if (!h) return fail(MG_EINVAL, "mg_export_codebook: null graph");
    const mg::Graph &g = h->g;
    if (!g.quant_bits) return fail(MG_ESTATE, "mg_export_codebook: the graph has exact weights (mg_quantize)");
    if (codeword) std::memcpy(codeword, g.codebook.data(), g.codebook.size() * sizeof(float));
    if (sigma) std::memcpy(sigma, g.code_sigma.data(), g.code_sigma.size() * sizeof(float));
    if (node_sigma) std::memcpy(node_sigma, g.node_sigma.data(), g.node_sigma.size() * sizeof(float));
    if (node_code) std::memcpy(node_code, g.node_code.data(), g.node_code.size() * sizeof(uint32_t));
    return MG_OK;
}

int mg_info(const mg_graph *h, mg_info_t *out)
{
    if (!h || !out) return fail(MG_EINVAL, "mg_info: null argument");
    const mg::Graph &g = h->g;
    std::memset(out, 0, sizeof(*out));
    out->nseg = g.nseg;
    out->n_nodes = g.n_nodes;
    out->depth = g.depth;
    out->n_levels = g.n_levels;
    for (uint32_t l = 0; l < g.n_levels; ++l)
        for (int a = 0; a < 3; ++a) out->dims[l][a] = g.lev_dims[3 * l + a];
    out->map_voxels = g.lev_off.empty() ? 0 : g.lev_off[g.n_levels];
    out->device_bytes = g.dev.bytes;
    out->device = g.dev.device;
    out->max_mixture = g.max_mixture;
    out->quant_bits = g.quant_bits;
    out->runs_mask = g.dev.runs_mask;
    return MG_OK;
}

int mg_export_dag(const mg_graph *h, uint32_t *child_a, uint32_t *child_b, float *alpha, uint64_t *wnum,
                  uint64_t *wden, uint32_t *rank, uint32_t *rank_ptr, uint32_t *step, uint32_t *sched,
                  uint32_t *step_ptr)
{
    if (!h) return fail(MG_EINVAL, "mg_export_dag: null graph");
    const mg::Graph &g = h->g;
    const size_t n = g.n_nodes;
    if (child_a) std::memcpy(child_a, g.child_a.data(), n * 4);
    if (child_b) std::memcpy(child_b, g.child_b.data(), n * 4);
    if (alpha) std::memcpy(alpha, g.alpha.data(), n * 4);
    if (wnum) std::memcpy(wnum, g.wnum.data(), n * 8);
    if (wden) std::memcpy(wden, g.wden.data(), n * 8);
    if (rank) std::memcpy(rank, g.rank.data(), n * 4);
    if (step) std::memcpy(step, g.step.data(), n * 4);
    if (rank_ptr) std::memcpy(rank_ptr, g.rank_ptr.data(), g.rank_ptr.size() * 4);
    if (sched) std::memcpy(sched, g.sched.data(), n * 4);
    if (step_ptr) std::memcpy(step_ptr, g.step_ptr.data(), g.step_ptr.size() * 4);
    return MG_OK;
}

int mg_export_map(const mg_graph *h, uint32_t level, uint32_t *out)
{
    if (!h || !out) return fail(MG_EINVAL, "mg_export_map: null argument");
    const mg::Graph &g = h->g;
    if (level >= g.n_levels) return fail(MG_EINVAL, "mg_export_map: level out of range");
    if (g.maps_on_device) {  // decoded on the GPU: copied back from there
        std::string err;
        return done(mg::dev_export_map(g, level, out, &err), "mg_export_map: " + err);
    }
    std::memcpy(out, g.maps.data() + g.lev_off[level], (g.lev_off[level + 1] - g.lev_off[level]) * 4);
    return MG_OK;
}

int mg_segment_ids(const mg_graph *h, uint32_t *out)
{
    if (!h || !out) return fail(MG_EINVAL, "mg_segment_ids: null argument");
    std::memcpy(out, h->g.seg_ids.data(), h->g.seg_ids.size() * 4);
    return MG_OK;
}

int mg_upload(mg_graph *h, int device)
{
    if (!h) return fail(MG_EINVAL, "mg_upload: null graph");
    if (device < 0) return fail(MG_EINVAL, "mg_upload: negative device");
    std::string err;
    return done(mg::dev_upload(&h->g, device, &err), err);
}

int mg_device_bytes(const mg_graph *h, uint64_t *bytes)
{
    if (!h || !bytes) return fail(MG_EINVAL, "mg_device_bytes: null argument");
    *bytes = mg::dev_device_bytes(h->g);
    return MG_OK;
}

int mg_bind_device(mg_graph *h, int device, void *d_buf, uint64_t bytes, void *stream)
{
    if (!h || !d_buf) return fail(MG_EINVAL, "mg_bind_device: null argument");
    std::string err;
    return done(mg::dev_bind_device(&h->g, device, d_buf, bytes, stream, &err), "mg_bind_device: " + err);
}

int mg_query_nnz_bound(mg_graph *h, const uint32_t *d_boxes, uint32_t n, uint32_t *d_bound, void *stream)
{
    if (!h) return fail(MG_EINVAL, "mg_query_nnz_bound: null graph");
    if (n == 0) return MG_OK;
    if (!d_boxes || !d_bound) return fail(MG_EINVAL, "mg_query_nnz_bound: null buffer");
    std::string err;
    return done(mg::dev_nnz_bound(&h->g, d_boxes, n, d_bound, stream, &err), err);
}

int mg_workspace_bytes(const mg_graph *h, uint32_t max_boxes, uint64_t *bytes)
{
    if (!h || !bytes) return fail(MG_EINVAL, "mg_workspace_bytes: null argument");
    *bytes = mg::dev_workspace_bytes(h->g, max_boxes);
    return MG_OK;
}

int mg_workspace_init(mg_graph *h, void *d_work, uint64_t work_bytes, void *stream)
{
    if (!h || !d_work) return fail(MG_EINVAL, "mg_workspace_init: null argument");
    std::string err;
    return done(mg::dev_workspace_init(&h->g, d_work, work_bytes, stream, &err), err);
}

static int query_common(mg_graph *h, const uint32_t *boxes, uint32_t n, float *out, void *work,
                        uint64_t bytes, void *stream, int variant, const char *name, uint32_t *stats = nullptr)
{
    if (!h) return fail(MG_EINVAL, std::string(name) + ": null graph");
    if (n == 0) return MG_OK;
    if (!boxes || !out || !work) return fail(MG_EINVAL, std::string(name) + ": null buffer");
    std::string err;
    return done(mg::dev_query(&h->g, boxes, n, out, nullptr, work, bytes, stream, variant, stats, &err), err);
}

int mg_query_boxes(mg_graph *h, const uint32_t *d_boxes, uint32_t n, float *d_out, void *d_work,
                   uint64_t work_bytes, void *stream)
{
    return query_common(h, d_boxes, n, d_out, d_work, work_bytes, stream, mg::kQueryBatched, "mg_query_boxes");
}

int mg_query_boxes_plain(mg_graph *h, const uint32_t *d_boxes, uint32_t n, float *d_out, void *d_work,
                         uint64_t work_bytes, void *stream)
{
    return query_common(h, d_boxes, n, d_out, d_work, work_bytes, stream, mg::kQueryPlain,
                        "mg_query_boxes_plain");
}

int mg_query_boxes_stats(mg_graph *h, const uint32_t *d_boxes, uint32_t n, float *d_out, uint32_t *d_stats,
                         void *d_work, uint64_t work_bytes, void *stream)
{
    if (n && !d_stats) return fail(MG_EINVAL, "mg_query_boxes_stats: null stats buffer");
    return query_common(h, d_boxes, n, d_out, d_work, work_bytes, stream, mg::kQueryBatched,
                        "mg_query_boxes_stats", d_stats);
}

int mg_query_boxes_sparse(mg_graph *h, const uint32_t *d_boxes, uint32_t n, uint32_t *d_index, uint32_t *d_seg,
                          float *d_val, uint32_t capacity, uint32_t *d_total, void *d_work, uint64_t work_bytes,
                          void *stream)
{
    if (!h) return fail(MG_EINVAL, "mg_query_boxes_sparse: null graph");
    if (n == 0) return MG_OK;
    if (!d_boxes || !d_index || !d_total || !d_work || (capacity && (!d_seg || !d_val)))
        return fail(MG_EINVAL, "mg_query_boxes_sparse: null buffer");
    mg::SparseOut sp{d_index, d_seg, d_val, capacity, d_total};
    std::string err;
    return done(mg::dev_query(&h->g, d_boxes, n, nullptr, &sp, d_work, work_bytes, stream, mg::kQueryBatched, nullptr,
                              &err),
                err);
}

int mg_query_boxes_noalloc(mg_graph *h, const uint32_t *d_boxes, uint32_t n, float *d_out, void *stream)
{
    if (!h) return fail(MG_EINVAL, "mg_query_boxes_noalloc: null graph");
    if (n == 0) return MG_OK;
    if (!d_boxes || !d_out) return fail(MG_EINVAL, "mg_query_boxes_noalloc: null buffer");
    std::string err;
    return done(mg::dev_query_noalloc(&h->g, d_boxes, n, d_out, stream, &err), err);
}

int mg_check_load_addresses(uint32_t nx, uint32_t ny, uint32_t nz, uint32_t flags, const uint32_t *boxes,
                            uint32_t n, uint32_t unroll, uint64_t *counts)
{
    if (!counts || (n && !boxes)) return fail(MG_EINVAL, "mg_check_load_addresses: null argument");
    if (!nx || !ny || !nz || uint64_t(nx) * ny * nz >= (1ull << 31))
        return fail(MG_EINVAL, "mg_check_load_addresses: dimensions must be >= 1 with fewer than 2^31 voxels");
    if (!(unroll == 4 || unroll == 8 || unroll == 16))
        return fail(MG_EINVAL, "mg_check_load_addresses: unroll must be 4, 8 or 16");
    const uint32_t dims[3] = {nx, ny, nz};
    std::string err;
    if (flags & 0xF8u) return fail(MG_EINVAL, "mg_check_load_addresses: unknown flags");
    return done(mg::dev_check_load_addresses(dims, flags, boxes, n, unroll, counts, &err), err);
}

int mg_naive_boxes(mg_graph *h, const uint32_t *d_boxes, uint32_t n, float *d_out, void *d_work,
                   uint64_t work_bytes, void *stream)
{
    return query_common(h, d_boxes, n, d_out, d_work, work_bytes, stream, mg::kQueryNaive, "mg_naive_boxes");
}

int mg_footprint(mg_graph *h, const uint32_t *d_boxes, uint32_t n, uint32_t *d_level_counts, uint32_t *d_cubes,
                 uint32_t cap, uint32_t *d_count, void *stream)
{
    if (!h) return fail(MG_EINVAL, "mg_footprint: null graph");
    if (n == 0) return MG_OK;
    if (!d_boxes || !d_level_counts) return fail(MG_EINVAL, "mg_footprint: null buffer");
    if (d_cubes && !d_count) return fail(MG_EINVAL, "mg_footprint: d_cubes needs d_count");
    std::string err;
    return done(mg::dev_footprint(&h->g, d_boxes, n, d_level_counts, d_cubes, cap, d_count, stream, &err), err);
}

int mg_propagate_tf(mg_graph *h, const uint8_t *d_tf, uint32_t T, float *d_node_rgba, void *stream)
{
    if (!h) return fail(MG_EINVAL, "mg_propagate_tf: null graph");
    if (T == 0) return MG_OK;
    if (!d_tf || !d_node_rgba) return fail(MG_EINVAL, "mg_propagate_tf: null buffer");
    std::string err;
    return done(mg::dev_propagate_tf(&h->g, d_tf, T, d_node_rgba, stream, &err), err);
}

int mg_palette_fetch(mg_graph *h, const float *d_palette, uint32_t T, uint32_t level, const uint32_t *d_xyz,
                     uint32_t n, float *d_out, void *stream)
{
    if (!h) return fail(MG_EINVAL, "mg_palette_fetch: null graph");
    if (level >= h->g.n_levels)
        return fail(MG_EINVAL, "mg_palette_fetch: level " + std::to_string(level) + " of a graph with " +
                                   std::to_string(h->g.n_levels) + " levels");
    if (T == 0 || n == 0) return MG_OK;
    if (!d_palette || !d_xyz || !d_out) return fail(MG_EINVAL, "mg_palette_fetch: null buffer");
    std::string err;
    return done(mg::dev_palette_fetch(&h->g, d_palette, T, level, d_xyz, n, d_out, stream, &err), err);
}

int mg_box_colour(mg_graph *h, const float *d_palette, uint32_t T, const uint32_t *d_boxes, uint32_t n,
                  const uint32_t *d_pal_of_box, float *d_out, void *stream)
{
    if (!h) return fail(MG_EINVAL, "mg_box_colour: null graph");
    if (n == 0) return MG_OK;
    if (!d_palette || !d_boxes || !d_pal_of_box || !d_out) return fail(MG_EINVAL, "mg_box_colour: null buffer");
    std::string err;
    return done(mg::dev_box_colour(&h->g, d_palette, T, d_boxes, n, d_pal_of_box, d_out, stream, &err), err);
}

int mg_lut_build(mg_graph *h, uint32_t threads, uint64_t *out_nnz)
{
    if (!h) return fail(MG_EINVAL, "mg_lut_build: null graph");
    std::string err;
    int rc = mg::build_lut(&h->g, threads, &err);
    if (rc == MG_OK && h->g.dev.device >= 0) rc = mg::dev_upload_lut(&h->g, &err);
    if (rc == MG_OK && out_nnz) *out_nnz = h->g.lut_ptr.back();
    return done(rc, err);
}

int mg_export_lut(const mg_graph *h, uint64_t *ptr, uint32_t *seg, float *val, float *err)
{
    if (!h || !ptr) return fail(MG_EINVAL, "mg_export_lut: null argument");
    const mg::Graph &g = h->g;
    if (g.lut_ptr.empty()) return fail(MG_ESTATE, "mg_export_lut: the lookup table was not built (mg_lut_build)");
    std::memcpy(ptr, g.lut_ptr.data(), g.lut_ptr.size() * sizeof(uint64_t));
    if (seg) std::memcpy(seg, g.lut_seg.data(), g.lut_seg.size() * sizeof(uint32_t));
    if (val) std::memcpy(val, g.lut_val.data(), g.lut_val.size() * sizeof(float));
    if (err) {
        if (g.lut_err.size() == g.lut_val.size())
            std::memcpy(err, g.lut_err.data(), g.lut_err.size() * sizeof(float));
        else
            std::memset(err, 0, g.lut_val.size() * sizeof(float));
    }
    return MG_OK;
}

int mg_query_boxes_lut(mg_graph *h, const uint32_t *d_boxes, uint32_t n, float *d_out, void *d_work,
                       uint64_t work_bytes, void *stream)
{
    return query_common(h, d_boxes, n, d_out, d_work, work_bytes, stream, mg::kQueryLut, "mg_query_boxes_lut");
}

int mg_query_boxes_err(mg_graph *h, const uint32_t *d_boxes, uint32_t n, float *d_out, float *d_err, void *d_work,
                       uint64_t work_bytes, void *stream)
{
    if (!h) return fail(MG_EINVAL, "mg_query_boxes_err: null graph");
    if (n == 0) return MG_OK;
    if (!d_boxes || !d_out || !d_err || !d_work) return fail(MG_EINVAL, "mg_query_boxes_err: null buffer");
    std::string err;
    return done(mg::dev_query(&h->g, d_boxes, n, d_out, nullptr, d_work, work_bytes, stream, mg::kQueryLutErr,
                              nullptr, &err, d_err),
                err);
}

int mg_pack(const mg_graph *h, uint8_t *buf, uint64_t capacity, uint64_t *size)
{
    if (!h || !size) return fail(MG_EINVAL, "mg_pack: null argument");
    if (h->g.maps_on_device) return fail(MG_ESTATE, "mg_pack: the node maps exist only on the device");
    std::vector<uint8_t> s;
    std::string err;
    if (int rc = mg::pack_graph(h->g, &s, &err)) return fail(rc, "mg_pack: " + err);
    *size = s.size();
    if (!buf) return MG_OK;
    if (capacity < s.size())
        return fail(MG_ELIMIT, "mg_pack: the stream needs " + std::to_string(s.size()) + " bytes, capacity is " +
                                   std::to_string(capacity));
    std::memcpy(buf, s.data(), s.size());
    return MG_OK;
}

int mg_unpack(const uint8_t *buf, uint64_t size, uint32_t threads, mg_graph **out)
{
    if (!buf || !out) return fail(MG_EINVAL, "mg_unpack: null argument");
    *out = nullptr;
    mg_graph *h = new (std::nothrow) mg_graph;
    if (!h) return fail(MG_ENOMEM, "mg_unpack: out of host memory");
    std::string err;
    if (int rc = mg::unpack_graph(buf, size, threads, &h->g, &err)) {
        delete h;
        return fail(rc, "mg_unpack: " + err);
    }
    *out = h;
    return MG_OK;
}

int mg_unpack_device(const uint8_t *buf, uint64_t size, uint32_t threads, int device, mg_graph **out)
{
    if (!buf || !out) return fail(MG_EINVAL, "mg_unpack_device: null argument");
    if (device < 0) return fail(MG_EINVAL, "mg_unpack_device: negative device");
    *out = nullptr;
    mg_graph *h = new (std::nothrow) mg_graph;
    if (!h) return fail(MG_ENOMEM, "mg_unpack_device: out of host memory");
    std::string err;
    mg::StreamMaps sm;
    int rc;
    try {
        rc = mg::unpack_graph(buf, size, threads, &h->g, &err, &sm);
        if (rc == MG_OK) rc = mg::dev_upload_stream(&h->g, buf, size, sm, device, &err);
    } catch (const std::bad_alloc &) {
        rc = MG_ENOMEM, err = "out of host memory";
    }
    if (rc != MG_OK) {
        delete h;
        return fail(rc, "mg_unpack_device: " + err);
    }
    *out = h;
    return MG_OK;
}

int mg_get_launch(const mg_graph *h, mg_launch_cfg *out)
{
    if (!h || !out) return fail(MG_EINVAL, "mg_get_launch: null argument");
    *out = h->g.dev.cfg;
    return MG_OK;
}

int mg_set_launch(mg_graph *h, const mg_launch_cfg *cfg)
{
    if (!h || !cfg) return fail(MG_EINVAL, "mg_set_launch: null argument");
    std::string err;
    return done(mg::dev_set_launch(&h->g, cfg, &err), err);
}

int mg_autotune(mg_graph *h, const uint32_t *d_boxes, uint32_t n, float *d_out, void *d_work, uint64_t work_bytes,
                uint32_t reps, void *stream, mg_launch_cfg *chosen)
{
    if (!h) return fail(MG_EINVAL, "mg_autotune: null graph");
    if (n == 0 || !d_boxes || !d_out || !d_work) return fail(MG_EINVAL, "mg_autotune: needs boxes, output, workspace");
    std::string err;
    return done(mg::dev_autotune(&h->g, d_boxes, n, d_out, d_work, work_bytes, reps ? reps : 3, stream, chosen, &err),
                err);
}

int mg_timing_enable(mg_graph *h, int enable)
{
    if (!h) return fail(MG_EINVAL, "mg_timing_enable: null graph");
    std::string err;
    return done(mg::dev_timing_enable(&h->g, enable, &err), err);
}

int mg_timing_read(mg_graph *h, double *ms, uint32_t *launches)
{
    if (!h || !ms || !launches) return fail(MG_EINVAL, "mg_timing_read: null argument");
    std::string err;
    return done(mg::dev_timing_read(&h->g, ms, launches, &err), err);
}

int mg_save(const mg_graph *h, const char *path)
{
    if (!h || !path) return fail(MG_EINVAL, "mg_save: null argument");
    const mg::Graph &g = h->g;
    if (g.maps_on_device) return fail(MG_ESTATE, "mg_save: the node maps exist only on the device");
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(MG_EIO, std::string("mg_save: cannot open ") + path);
    uint32_t hdr[9] = {g.dims[0], g.dims[1], g.dims[2], g.nseg, g.n_nodes, g.depth, g.n_levels, g.max_mixture,
                       g.quant_bits};
    bool ok = wr(f, kMagic, 8) && wr(f, hdr, sizeof(hdr)) && wr_vec(f, g.seg_ids) && wr_vec(f, g.child_a) &&
              wr_vec(f, g.child_b) && wr_vec(f, g.alpha) && wr_vec(f, g.wnum) && wr_vec(f, g.wden) &&
              wr_vec(f, g.rank) && wr_vec(f, g.step) && wr_vec(f, g.rank_ptr) && wr_vec(f, g.sched) &&
              wr_vec(f, g.step_ptr) && wr_vec(f, g.lev_off) && wr_vec(f, g.maps) && wr_vec(f, g.codebook) &&
              wr_vec(f, g.code_sigma) && wr_vec(f, g.node_sigma) && wr_vec(f, g.node_code);
    ok = (std::fclose(f) == 0) && ok;
    return ok ? MG_OK : fail(MG_EIO, std::string("mg_save: write failed for ") + path);
}

int mg_load(const char *path, mg_graph **out)
{
    if (!path || !out) return fail(MG_EINVAL, "mg_load: null argument");
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(MG_EIO, std::string("mg_load: cannot open ") + path);
    mg_graph *h = new (std::nothrow) mg_graph;
    if (!h) {
        std::fclose(f);
        return fail(MG_ENOMEM, "mg_load: out of host memory");
    }
    mg::Graph &g = h->g;
    char magic[8];
    uint32_t hdr[9];
    int rc = MG_OK;
    if (!rd(f, magic, 8) || !rd(f, hdr, sizeof(hdr))) rc = MG_EIO;
    else if (std::memcmp(magic, kMagic, 8) != 0) rc = MG_EFORMAT;
    if (rc == MG_OK) {
        g.dims[0] = hdr[0], g.dims[1] = hdr[1], g.dims[2] = hdr[2];
        g.nseg = hdr[3], g.n_nodes = hdr[4], g.depth = hdr[5], g.n_levels = hdr[6], g.max_mixture = hdr[7];
        g.quant_bits = hdr[8];
        const uint64_t nvox = uint64_t(g.dims[0]) * g.dims[1] * g.dims[2];
        const uint64_t N = g.n_nodes, lim_maps = 2 * nvox + 64;
        if (g.dims[0] == 0 || g.dims[1] == 0 || g.dims[2] == 0 || nvox >= (1ull << 31) ||
            g.n_levels > MG_MAX_LEVELS || g.quant_bits > mg::kMaxQuantBits)
            rc = MG_EFORMAT;
        if (rc == MG_OK) rc = rd_vec(f, &g.seg_ids, N);
        if (rc == MG_OK) rc = rd_vec(f, &g.child_a, N);
        if (rc == MG_OK) rc = rd_vec(f, &g.child_b, N);
        if (rc == MG_OK) rc = rd_vec(f, &g.alpha, N);
        if (rc == MG_OK) rc = rd_vec(f, &g.wnum, N);
        if (rc == MG_OK) rc = rd_vec(f, &g.wden, N);
        if (rc == MG_OK) rc = rd_vec(f, &g.rank, N);
        if (rc == MG_OK) rc = rd_vec(f, &g.step, N);
        if (rc == MG_OK) rc = rd_vec(f, &g.rank_ptr, uint64_t(g.depth) + 2);
        if (rc == MG_OK) rc = rd_vec(f, &g.sched, N);
        if (rc == MG_OK) rc = rd_vec(f, &g.step_ptr, uint64_t(g.depth) + 2);
        if (rc == MG_OK) rc = rd_vec(f, &g.lev_off, uint64_t(MG_MAX_LEVELS) + 1);
        if (rc == MG_OK) rc = rd_vec(f, &g.maps, lim_maps);
        const uint64_t nb = g.quant_bits ? (uint64_t(1) << g.quant_bits) : 0, nn = g.quant_bits ? N : 0;
        if (rc == MG_OK) rc = rd_vec(f, &g.codebook, nb);
        if (rc == MG_OK) rc = rd_vec(f, &g.code_sigma, nb);
        if (rc == MG_OK) rc = rd_vec(f, &g.node_sigma, nn);
        if (rc == MG_OK) rc = rd_vec(f, &g.node_code, nn);
        if (rc == MG_OK && (g.codebook.size() != nb || g.code_sigma.size() != nb || g.node_sigma.size() != nn ||
                            g.node_code.size() != nn))
            rc = MG_EFORMAT;
        if (rc == MG_OK)
            for (uint32_t k : g.node_code)
                if (k >= nb && nb) rc = MG_EFORMAT;
        if (rc == MG_OK) mg::level_dims(g.dims, &g.lev_dims);
    }
    std::fclose(f);
    std::string err;
    if (rc == MG_OK) rc = mg::validate_graph(g, &err);
    else err = rc == MG_EIO ? "mg_load: read failed" : "mg_load: corrupt or incompatible file";
    if (rc != MG_OK) {
        delete h;
        return fail(rc, err.empty() ? "mg_load: invalid graph" : "mg_load: " + err);
    }
    *out = h;
    return MG_OK;
}

void mg_free(mg_graph *h)
{
    if (!h) return;
    mg::dev_free(&h->g);
    delete h;
}

}  // extern "C"
