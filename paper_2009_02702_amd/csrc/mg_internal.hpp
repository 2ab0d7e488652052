// Internal types shared by the host builder (builder.cpp), the C ABI
// (api.cpp) and the HIP launchers (kernels.hip). Not installed.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "mg.h"

namespace mg {

// One internal node as the GPU reads it: node = (1 - w) * a + w * b.
// 12 bytes, read with one dwordx3 load per visited node.
struct NodeTriple {
    uint32_t a;
    uint32_t b;
    float w;
};
static_assert(sizeof(NodeTriple) == 12, "NodeTriple must stay 12 bytes");

// A node in step-schedule order, for the propagation kernel (16 bytes).
struct SchedNode {
    uint32_t a;
    uint32_t b;
    float w;
    uint32_t id;
};

struct DeviceState {
    int device = -1;
    void *base = nullptr;          // the one buffer holding every array below (except the table)
    bool owned = false;            // base was allocated by mg_upload (else bound by the caller)
    NodeTriple *nodes = nullptr;   // [n_nodes]
    uint32_t *mixlen = nullptr;    // [n_nodes] bound on the sources in each node's mixture
    uint32_t *rank_ptr = nullptr;  // [depth + 2]
    SchedNode *sched = nullptr;    // [n_nodes] in step order
    uint32_t *maps = nullptr;      // all levels, x fastest
    uint32_t *maps_t = nullptr;    // all levels, y fastest then z then x
    uint16_t *maps16 = nullptr;    // level 0 as 16-bit IDs, both orientations (rows padded to even)
    void *run_table = nullptr;     // row runs per level and orientation (RunLevel [2 n_levels])
    uint32_t runs_mask = 0;        // bit 2 l + o: level l has runs along x (o = 0) / y (o = 1)
    uint64_t *lut_ptr = nullptr;   // [n_nodes + 1] mixture lookup table rows (optional)
    uint32_t *lut_seg = nullptr;   // [lut nnz]
    float *lut_val = nullptr;      // [lut nnz]
    float *lut_err = nullptr;      // [lut nnz] propagated uncertainty (quantized graphs)
    uint64_t bytes = 0;
    // launch parameters, queried once per device and graph
    bool launch_ready = false;
    int ncu = 0, lds_max = 0;
    struct Occ {
        const void *kernel;
        uint32_t dyn;   // dynamic LDS bytes of the launch
        int blocks;     // blocks per CU
    };
    std::vector<Occ> occupancy;  // per kernel variant and LDS size
    mg_launch_cfg cfg = {16, 8, 16, 256, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    bool timing = false;
    std::vector<void *> ev_start, ev_stop;  // hipEvent_t pairs recorded around the dominant kernel
    uint32_t ev_used = 0;
};

// Runs of equal node IDs along the rows of one level in one orientation
// (runs.cpp): row_ptr[rows + 1] into runs, runs[j] = (exclusive end along the
// row) << 32 | node, skip[rows][chunks] = index of the run holding cell 64 c of
// row r. Empty (rows == 0) where the level keeps no runs.
constexpr uint32_t kRunSkipCells = 64;  // cells of a row per skip entry
struct LevelRuns {
    uint32_t rows = 0, len = 0, chunks = 0;
    std::vector<uint32_t> row_ptr;
    std::vector<uint64_t> runs;
    std::vector<uint32_t> skip;
};

struct Graph {
    uint32_t dims[3] = {0, 0, 0};
    uint32_t nseg = 0;
    uint32_t n_nodes = 0;
    uint32_t depth = 0;
    uint32_t n_levels = 0;
    uint32_t max_mixture = 1;
    std::vector<uint32_t> lev_dims;   // 3 per level
    std::vector<uint64_t> lev_off;    // n_levels + 1 offsets into maps
    std::vector<uint32_t> maps;       // node ID per mip voxel, all levels, x fastest (empty when
                                      // maps_on_device: decoded on the GPU from a graph stream)
    bool maps_on_device = false;
    std::vector<uint32_t> seg_ids;    // source -> original volume ID
    std::vector<uint32_t> child_a, child_b, rank, step;  // [n_nodes]
    std::vector<float> alpha;                            // [n_nodes]
    std::vector<uint64_t> wnum, wden;                    // [n_nodes]
    std::vector<uint32_t> rank_ptr;                      // [depth + 2] IDs of each rank
    std::vector<uint32_t> step_ptr;                      // [depth + 2] into sched
    std::vector<uint32_t> sched;                         // [n_nodes] IDs in step order
    // mixture lookup table (optional, built by build_lut): row n = the sources of
    // node n's mixture, increasing, with their fractions
    std::vector<uint64_t> lut_ptr;                       // [n_nodes + 1], empty if not built
    std::vector<uint32_t> lut_seg;
    std::vector<float> lut_val;
    std::vector<float> lut_err;                          // propagated uncertainty (quantized graphs)
    // scalar-quantized weights (quantize_graph); quant_bits == 0: exact weights
    uint32_t quant_bits = 0;
    std::vector<float> codebook, code_sigma;             // [2^bits] codeword and sigma of each bin
    std::vector<float> node_sigma;                       // [n_nodes] sigma of each node's weight
    std::vector<uint32_t> node_code;                     // [n_nodes] codebook index of each node's weight
    // row runs of every level, [2 l] along x and [2 l + 1] along y: derived from
    // the host maps on first use (ensure_runs), a cache of the graph's own data
    mutable std::vector<LevelRuns> runs;
    mutable bool runs_ready = false;
    DeviceState dev;
};

// Fills g.runs from the host maps once (no runs for graphs whose maps are only on
// the device). Not safe against a concurrent first call on the same graph.
void ensure_runs(const Graph &g);

// A DAG in creation order (children before parents; sources 0 .. nseg-1 have
// a = b = n): what finalize_dag turns into a Graph's node arrays.
struct RawDag {
    uint32_t nseg = 0;
    std::vector<uint32_t> a, b;    // predecessors
    std::vector<uint64_t> wn, wd;  // weight of b as an exact fraction
    std::vector<uint32_t> mix;     // segments in the node's mixture
    std::vector<float> alpha;      // fp32 weights if given, else RN(wn / wd)
    std::vector<float> sigma;      // uncertainty of each weight, if any
    std::vector<uint32_t> code;    // codebook index of each weight (quantized graphs), if any
};

// Codewords and their standard deviations are 20-bit fields of the graph
// stream (Table "bitstream", C): codewords are multiples of 2^-20 in (0, 1),
// sigmas multiples of sigma_max / (2^20 - 1).
constexpr uint32_t kCodeBits = 20;
constexpr uint32_t kMaxQuantBits = 16;  // the stream's 4-bit bit-rate field
// sigma of a bin as stored: sigma_max * m / (2^20 - 1), rounded to fp32
inline float code_sigma_value(float sigma_max, uint32_t m)
{
    return float(double(sigma_max) * double(m) / double((1u << kCodeBits) - 1));
}
// The exact fraction num / den of an fp32 weight in (0, 1).
void weight_fraction(float c, uint64_t *num, uint64_t *den);

// Host builder (builder.cpp). Returns MG_OK or an MG_E* code with *err set.
int build_graph(const uint32_t *ids, const mg_build_opts *opts, Graph *g, std::string *err);
// Mixture lookup table of every node, in fp64 through the DAG, stored fp32.
int build_lut(Graph *g, uint32_t threads, std::string *err);
// A copy of `src` with weights scalar-quantized to 2^bits bins and nodes merged.
int quantize_graph(const Graph &src, uint32_t bits, uint32_t threads, Graph *dst, std::string *err);
// Ranks, step schedule and rank-sorted IDs of a DAG in creation order; the maps
// already in g (levels >= 1) are renumbered with the nodes.
// perm (if given) receives each creation-order ID's new ID.
int finalize_dag(const RawDag &d, bool defer, uint32_t max_depth, unsigned nt, Graph *g, std::string *err,
                 std::vector<uint32_t> *perm = nullptr);
// Greedy factorization (Sec. "Compression") of mixtures given as sorted
// (source, count) vectors, in scanline order; appends the sources and the
// interpolation nodes to d and returns each mixture's node in root. Consumes mix.
int greedy_factorize(uint32_t nseg, std::vector<std::vector<std::pair<uint32_t, uint64_t>>> &mix, uint32_t strategy,
                     uint32_t tau, RawDag *d, std::vector<uint32_t> *root, std::string *err);
// Worker threads for a request (0: all hardware threads).
unsigned resolve_threads(uint32_t t);
// Bit-packed graph stream (Table "bitstream"); quantized graphs only.
int pack_graph(const Graph &g, std::vector<uint8_t> *out, std::string *err);
// Where a stream's voxel data (A) lies, for decoding it on the GPU: bit offset
// of (A) in the stream, per level the offset of its first voxel from there,
// r(l) and i_min(l), and the renumbering of the stream's node IDs.
struct StreamMaps {
    uint64_t a_bit = 0;
    std::vector<uint64_t> bit_off;
    std::vector<uint32_t> r, lo;
    std::vector<uint32_t> perm;   // stream (creation-order) ID -> graph ID
};
// dev == nullptr: the maps are decoded on the host; else (A) is skipped, the
// graph gets maps_on_device, and *dev describes (A) for dev_upload_stream.
int unpack_graph(const uint8_t *buf, uint64_t size, uint32_t threads, Graph *g, std::string *err,
                 StreamMaps *dev = nullptr);
// Structural validation of a graph's host arrays (used by mg_load).
int validate_graph(const Graph &g, std::string *err);
// Level dimensions: halve with rounding up until 1^3.
void level_dims(const uint32_t dims[3], std::vector<uint32_t> *out);

// Device side (kernels.hip). All return MG_OK or an MG_E* code with *err set.
int dev_upload(Graph *g, int device, std::string *err);
// A graph whose maps are still in its stream: device buffer allocated as by
// dev_upload, the voxel data (A) decoded on the GPU into the node maps.
int dev_upload_stream(Graph *g, const uint8_t *buf, uint64_t size, const StreamMaps &sm, int device,
                      std::string *err);
// Host copy of one level of the device maps.
int dev_export_map(const Graph &g, uint32_t level, uint32_t *out, std::string *err);
uint64_t dev_device_bytes(const Graph &g);
int dev_bind_device(Graph *g, int device, void *base, uint64_t bytes, void *stream, std::string *err);
int dev_nnz_bound(Graph *g, const uint32_t *boxes, uint32_t n, uint32_t *bound, void *stream, std::string *err);
int dev_upload_lut(Graph *g, std::string *err);
void dev_free(Graph *g);
uint64_t dev_workspace_bytes(const Graph &g, uint32_t max_boxes);
int dev_workspace_init(Graph *g, void *work, uint64_t bytes, void *stream, std::string *err);
struct SparseOut {
    uint32_t *index;   // [n][2] first entry, entries
    uint32_t *seg;     // [cap]
    float *val;        // [cap]
    uint32_t cap;
    uint32_t *total;   // device counter
};
int dev_query(Graph *g, const uint32_t *boxes, uint32_t n, float *out, const SparseOut *sp, void *work,
              uint64_t bytes, void *stream, int variant, uint32_t *stats, std::string *err,
              float *out_err = nullptr);
// mg_query_boxes on the library's static device scratch (allocates nothing).
int dev_query_noalloc(Graph *g, const uint32_t *boxes, uint32_t n, float *out, void *stream, std::string *err);
// Replays on the host every load the query kernels issue for these boxes.
int dev_check_load_addresses(const uint32_t dims[3], uint32_t flags, const uint32_t *boxes, uint32_t n,
                              uint32_t unroll, uint64_t counts[4], std::string *err);
int dev_footprint(Graph *g, const uint32_t *boxes, uint32_t n, uint32_t *level_counts, uint32_t *cubes,
                  uint32_t cap, uint32_t *count, void *stream, std::string *err);
int dev_propagate_tf(Graph *g, const uint8_t *tf, uint32_t T, float *out, void *stream, std::string *err);
int dev_palette_fetch(Graph *g, const float *palette, uint32_t T, uint32_t level, const uint32_t *xyz, uint32_t n,
                      float *out, void *stream, std::string *err);
int dev_box_colour(Graph *g, const float *palette, uint32_t T, const uint32_t *boxes, uint32_t n,
                   const uint32_t *pal_of_box, float *out, void *stream, std::string *err);
int dev_timing_enable(Graph *g, int enable, std::string *err);
int dev_set_launch(Graph *g, const mg_launch_cfg *cfg, std::string *err);
int dev_autotune(Graph *g, const uint32_t *boxes, uint32_t n, float *out, void *work, uint64_t bytes, uint32_t reps,
                 void *stream, mg_launch_cfg *chosen, std::string *err);
int dev_timing_read(Graph *g, double *ms, uint32_t *launches, std::string *err);

enum QueryVariant { kQueryBatched = 0, kQueryPlain = 1, kQueryNaive = 2, kQueryLut = 3, kQueryLutErr = 4 };

}  // namespace mg
