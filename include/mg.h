/*
 * mg.h -- C ABI of the MI355X (gfx950) Mixture Graph library (libmg.so).
 *
 * The Mixture Graph (Al-Thelaya, Agus, Schneider, IEEE VIS 2020) factors the
 * normalized histogram mipmap of a segmentation volume into a DAG of binary
 * linear interpolations. This library builds that graph on the CPU and runs
 * its data-parallel hot path on the GPU:
 *
 *   - box-histogram queries: every box is cut into maximal aligned mipmap
 *     cubes, each cube's voxel count is scattered onto the graph node that
 *     holds its mixture, and that mass is pushed down the DAG in reverse
 *     topological order to per-segment counts;
 *   - transfer-function propagation: one colour per segment carried from the
 *     sources to every node in topological order.
 *
 * Conventions for every entry point:
 *   - Return value: MG_OK (0) or a negative MG_E* code; mg_last_error() then
 *     holds a message for the calling thread. No entry point throws, aborts
 *     or exits.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory on the graph's device (e.g. from torch tensors). The
 *     caller owns every input and output buffer and keeps device buffers alive
 *     until the work queued on `stream` has finished.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Query and propagation calls only enqueue work and never allocate; errors
 *     of the queued kernels surface at the next synchronisation.
 *   - Volumes are x fastest: voxel (x, y, z) is element x + nx*(y + ny*z).
 *   - Boxes are uint32 rows (x0, y0, z0, dx, dy, dz): the half-open range
 *     [x0, x0+dx) x [y0, y0+dy) x [z0, z0+dz), clipped to the volume; an
 *     origin at or past the volume or a zero extent is an empty box (all-zero
 *     histogram), never an error.
 *   - Segments: the distinct IDs of the volume, in increasing order, are the
 *     graph's sources 0 .. S-1; mg_segment_ids() maps them back.
 *   - Calls that share a graph and a workspace must not overlap in time (use
 *     one stream, or one workspace per stream).
 */
#ifndef MG_H
#define MG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MG_OK 0
#define MG_EINVAL (-1)    /* bad argument (null pointer, size, flag)              */
#define MG_ENOMEM (-2)    /* host or device allocation failed                      */
#define MG_EDEVICE (-3)   /* HIP runtime error (message has the HIP error string)  */
#define MG_ESTATE (-4)    /* call out of order (e.g. query before mg_upload)       */
#define MG_EDEPTH (-5)    /* graph deeper than mg_build_opts.max_depth             */
#define MG_EIO (-6)       /* file error in mg_save / mg_load                        */
#define MG_EFORMAT (-7)   /* corrupt or incompatible graph file or graph arrays    */
#define MG_ELIMIT (-8)    /* a size beyond what this library supports (message says) */

typedef struct mg_graph mg_graph; /* opaque; owned by the library, freed by mg_free */

typedef struct {
    uint32_t nx, ny, nz;   /* level-0 dimensions, each >= 1, nx*ny*nz < 2^31       */
    uint32_t defer;        /* 1: deferred, load-balanced step schedule (Sec.
                              "Reconstruction"); 0: one step per topological level */
    uint32_t max_depth;    /* 0: no cap; else fail with MG_EDEPTH beyond it         */
    uint32_t threads;      /* CPU threads for the build; 0 = all hardware threads   */
    uint32_t factorizer;   /* MG_FACTOR_*: how mixtures become interpolations       */
    uint32_t tau;          /* greedy factorizers: mixtures with more than tau
                              components go through the global maximum search,
                              the rest are factorized in scanline order (Sec.
                              "Implementation Details"); 0 or 1: all global      */
    uint32_t reserved[2];  /* must be 0                                             */
} mg_build_opts;

/* Factorizers (mg_build_opts.factorizer). HALVING: each distinct mip-voxel
 * mixture is split into its first and second half of segments, recursively,
 * and equal sub-mixtures are shared (exact counts). GREEDY_REDUCTION /
 * GREEDY_OCCURRENCE: the paper's greedy pair picks (Sec. "Compression", Eq.
 * greedy2 max-reduction phi2, Eq. greedy1 max-occurrence phi1) over the
 * distinct mip-voxel mixtures, in exact integer ratios, with the two-stage
 * cutoff tau; ties between pairs go to the smallest (i, j). */
#define MG_FACTOR_HALVING 0
#define MG_FACTOR_GREEDY_REDUCTION 1
#define MG_FACTOR_GREEDY_OCCURRENCE 2

#define MG_MAX_LEVELS 24

typedef struct {
    uint32_t nseg;          /* S: number of sources (distinct IDs)                   */
    uint32_t n_nodes;       /* sources + internal nodes                              */
    uint32_t depth;         /* topological depth = number of steps                   */
    uint32_t n_levels;      /* mip levels (level 0 .. n_levels-1, last is 1^3)        */
    uint32_t dims[MG_MAX_LEVELS][3]; /* per level (nx, ny, nz)                       */
    uint64_t map_voxels;    /* total mip voxels over all levels                      */
    uint64_t device_bytes;  /* device memory held after mg_upload (0 before)         */
    int32_t device;         /* device ordinal after mg_upload, else -1                */
    uint32_t max_mixture;   /* largest number of segments in one node's mixture      */
    uint32_t quant_bits;    /* 0: exact weights; else the quantizer's bit rate       */
    uint32_t runs_mask;     /* after mg_upload: bit 2 l + o set where level l keeps
                               row runs along x (o = 0) or y (o = 1)                  */
} mg_info_t;

/* Build a graph from a host uint32 ID volume (CPU; Sec. "Normalized Histogram
 * Mipmap" Eq. (mip), Sec. "Factorization", Sec. "Compression", Sec.
 * "Reconstruction"). Mip levels halve each axis rounding up down to 1^3; every
 * mip voxel's mixture is the exact normalized histogram of its level-0 support.
 * Each distinct mixture becomes one node, factored into binary lerps
 * n = (1 - w) a + w b with exact rational w in (0, 1/2]; nodes are numbered by
 * topological level (sources first). On success *out owns host copies of the DAG
 * and of one node ID per mip voxel. `ids` is read only during the call.
 * Volumes of 2^31 voxels or more give MG_ELIMIT. */
int mg_build(const uint32_t *ids, const mg_build_opts *opts, mg_graph **out);

int mg_info(const mg_graph *g, mg_info_t *out);

/* A lossy copy of a graph with scalar-quantized weights (Sec. "Compression":
 * the open range (0, 1) is cut into 2^bits equal bins, one codeword and the
 * empirical standard deviation of the weights per bin; Sec. "Implementation
 * Details": w and 1 - w are both quantized and the orientation with the
 * smaller error is kept). The codebook is learned from the graph's weights; a
 * codeword is the mean of its bin's weights (an empty bin: its midpoint and the
 * standard deviation of a uniform bin), rounded to the 20-bit field the graph
 * stream stores it in (Table "bitstream", C): the nearest multiple of 2^-20 in
 * (0, 1); sigmas to the nearest multiple of sigma_max / (2^20 - 1), sigma_max
 * being the largest bin sigma in fp32. Nodes are visited predecessors first;
 * nodes with equal (merged) predecessors and codeword are merged, and a node
 * whose two predecessors merged becomes that predecessor. The copy supports
 * every entry point of an exact graph (its queries return the quantized
 * histograms) and mg_export_codebook; its lookup table also carries the
 * propagated uncertainty (mg_lut_build, mg_query_boxes_err) and can be
 * written as a bit-packed stream (mg_pack). bits in [1, 16] (the stream's
 * 4-bit bit-rate field), else MG_EINVAL; MG_EINVAL for a quantized graph. */
int mg_quantize(const mg_graph *g, uint32_t bits, uint32_t threads, mg_graph **out);

/* Codebook of a quantized graph: codeword and sigma host fp32 [2^bits]; node_sigma
 * host fp32 [n_nodes], the sigma of each node's weight (0 for sources); node_code
 * host u32 [n_nodes], the bin of each node's weight (the stored weight is the
 * codeword or 1 - codeword; 0 for sources). NULL skips an array; MG_ESTATE for a
 * graph with exact weights. */
int mg_export_codebook(const mg_graph *g, float *codeword, float *sigma, float *node_sigma, uint32_t *node_code);

/* Host copies of the DAG (NULL skips an array). Per node (n_nodes entries):
 * child_a/child_b are its two predecessors and w[n] = wnum[n]/wden[n] the
 * weight of child_b (n = (1 - w) a + w b), alpha[n] = w rounded to fp32;
 * sources have a = b = n, w = 0. rank[n] is the topological level (Sec.
 * "Reconstruction"); node IDs are sorted by rank, and rank_ptr (depth + 2
 * entries) delimits them: rank r holds IDs [rank_ptr[r], rank_ptr[r+1]).
 * step[n] is the step the deferred schedule runs n in (Sec.
 * "Reconstruction"); sched (n_nodes entries) lists the IDs in execution order
 * and step_ptr (depth + 2 entries) delimits each step in it, step 0 holding
 * the sources. */
int mg_export_dag(const mg_graph *g, uint32_t *child_a, uint32_t *child_b, float *alpha,
                  uint64_t *wnum, uint64_t *wden, uint32_t *rank, uint32_t *rank_ptr,
                  uint32_t *step, uint32_t *sched, uint32_t *step_ptr);

/* Host copy of level `level`'s node IDs, x fastest, dims[level] voxels. */
int mg_export_map(const mg_graph *g, uint32_t level, uint32_t *out);

/* Original volume ID of each source, S entries (host). */
int mg_segment_ids(const mg_graph *g, uint32_t *out);

/* Put the graph on a GPU, in device memory the caller owns (e.g. a torch
 * tensor), so that the library holds no device allocation of its own:
 * mg_device_bytes gives the size of one buffer that holds every array the GPU
 * path reads (the DAG's (a, b, w) triples in node order and in step order, the
 * rank table, a per-node bound on its mixture's sources, the node-ID maps of
 * every level x fastest and y fastest, and 16-bit copies of level 0 when the
 * sources fit); mg_bind_device fills `d_buf` (device memory on `device`, at
 * least that many bytes, 256-byte aligned) with them, enqueued on `stream`,
 * and waits for that work before it returns. The caller keeps d_buf alive
 * and unchanged until mg_free, another bind or mg_upload; the library never
 * frees it. The mixture lookup table (mg_lut_build, optional) is still
 * allocated by the library. MG_EINVAL for a small or misaligned buffer or a
 * device that does not exist. Must precede every GPU entry point (or
 * mg_upload). */
int mg_device_bytes(const mg_graph *g, uint64_t *bytes);
int mg_bind_device(mg_graph *g, int device, void *d_buf, uint64_t bytes, void *stream);

/* mg_bind_device into a buffer the library allocates (hipMalloc) on `device`
 * and frees in mg_free; the current device is restored. */
int mg_upload(mg_graph *g, int device);

/* Bytes of device workspace that query calls of up to `max_boxes` boxes need. */
int mg_workspace_bytes(const mg_graph *g, uint32_t max_boxes, uint64_t *bytes);

/* Prepare a workspace once after allocating it (enqueued on `stream`). */
int mg_workspace_init(mg_graph *g, void *d_work, uint64_t work_bytes, void *stream);

/* Box histograms, the batched path (Sec. "Fast Sub-Volume Queries"; the
 * decomposition of the appendix algorithm "Footprint assembly in 3D").
 *   d_boxes  device uint32 [n][6]
 *   d_out    device fp32 [n][S]: fraction of each segment's voxels in the
 *            clipped box (counts divided by the box volume in fp64, rounded
 *            to fp32); all zeros for an empty box. Counts from cubes whose
 *            node is a source are exact integers; mass pushed through the DAG
 *            is accumulated in fp32 with compensated (two-sum) updates.
 *   d_work   workspace of mg_workspace_bytes(g, n) bytes, initialised once.
 * Boxes whose nodes overflow the per-box LDS tables are redone with a larger
 * LDS table, then in global-memory tables: first many workers' tables of
 * 65,536 slots, then (for what overflows those) tables that hold every node
 * of graphs of up to 50,331,647 nodes; only on larger graphs can a box still
 * overflow, and its row is then all NaN.
 */
int mg_query_boxes(mg_graph *g, const uint32_t *d_boxes, uint32_t n, float *d_out,
                   void *d_work, uint64_t work_bytes, void *stream);

/* The same results by one plain workgroup per box, in input order: the
 * straightforward GPU kernel the batched path is measured against. */
int mg_query_boxes_plain(mg_graph *g, const uint32_t *d_boxes, uint32_t n, float *d_out,
                         void *d_work, uint64_t work_bytes, void *stream);

/* mg_query_boxes that also reports the work of each box, for roofline
 * accounting: d_stats device uint32 [n][2]. [q][0] = cubes in box q's
 * footprint. [q][1] bits 0..29 = entries the box's node table held: the
 * distinct internal nodes of rank >= 3 it scattered onto or reached by the
 * push, plus, for graphs with more sources than the LDS source arrays hold,
 * the distinct sources it touched (a source in those arrays takes no entry).
 * Nodes of rank 1 and 2 (every predecessor a source, or a source or a rank-1
 * node) pass their mass straight to the sources and take no entry, so they
 * are not counted: the figure is a lower bound on the number of internal
 * nodes in the closure of the box's cubes. Bit 30 = the box was answered by
 * the retry launch, bit 31 = by a global-memory launch. */
int mg_query_boxes_stats(mg_graph *g, const uint32_t *d_boxes, uint32_t n, float *d_out,
                         uint32_t *d_stats, void *d_work, uint64_t work_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * mg_query_boxes with the library's own workspace instead of d_work, so the
 * call allocates nothing. The workspace is one static device array of
 * MG_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, which the library's code object
 * holds from its first use on that GPU (mg_upload looks up its address) until
 * the process ends. Same arguments, kernels and results as mg_query_boxes
 * (boxes, output layout, clipping); the global fallback tables get as many
 * workers as fit beside the per-box arrays.
 * Boxes that overflow every LDS table go straight to the tables that hold
 * the whole graph (no mid-size tables).
 * Limits (MG_ELIMIT, the message states the limit for this graph): 20 bytes
 * of scratch per box, and one worker's fallback table (20 bytes per slot,
 * slots >= 4/3 x n_nodes rounded up to a power of two) must fit, i.e. graphs
 * of up to about 1.5 M nodes.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap in time on one GPU (other streams, other
 * threads, other graphs) race; order them on one stream or synchronise. */
#define MG_NOALLOC_SCRATCH_BYTES (64u << 20)
int mg_query_boxes_noalloc(mg_graph *g, const uint32_t *d_boxes, uint32_t n, float *d_out, void *stream);

/* Box histograms with sparse output, for many segments: the same path, with
 * each box's non-zero segments appended to one entry buffer.
 *   d_index  device uint32 [n][2]: first entry of the box and its number of
 *            entries (its non-zero segments, in no particular order)
 *   d_seg    device uint32 [capacity]: segment (source) of each entry
 *   d_val    device fp32 [capacity]: fraction of the box's voxels
 *   d_total  device uint32: reset by the call, then the entries produced. If
 *            it exceeds `capacity` after the stream completes, entries at or
 *            beyond `capacity` were not written (call again with more room).
 * A box that no table could hold (possible only on graphs of more than
 * 50,331,647 nodes) gets 0xFFFFFFFF in both index fields. */
int mg_query_boxes_sparse(mg_graph *g, const uint32_t *d_boxes, uint32_t n, uint32_t *d_index,
                          uint32_t *d_seg, float *d_val, uint32_t capacity, uint32_t *d_total,
                          void *d_work, uint64_t work_bytes, void *stream);

/* Upper bound on the non-zero segments of each box, for sizing the sparse
 * output before the query (Sec. "Fast Sub-Volume Queries": how many segments a
 * box holds is not known in advance). d_boxes device uint32 [n][6] as for
 * mg_query_boxes; d_bound device uint32 [n]. A box lies inside the mip cells
 * it touches at any level; at the finest level where it touches at most 64
 * cells, the bound is the sum of the sources of those cells' distinct nodes'
 * mixtures, capped by the number of sources and the box volume (graphs with
 * quantized weights: the cap alone); 0 for an empty box. A sparse query whose
 * capacity is the sum of the bounds never truncates. Enqueued on `stream`. */
int mg_query_nnz_bound(mg_graph *g, const uint32_t *d_boxes, uint32_t n, uint32_t *d_bound, void *stream);

/* Competitor: the naive range query (Sec. "Results", range queries): every
 * level-0 voxel of the box is read and counted. Same output as above. */
int mg_naive_boxes(mg_graph *g, const uint32_t *d_boxes, uint32_t n, float *d_out,
                   void *d_work, uint64_t work_bytes, void *stream);

/* Host-side check of the query kernels' load addresses (no GPU needed): for
 * boxes (host uint32 [n][6]) on a volume of nx x ny x nz voxels, replays every
 * load the batched query kernels issue (all `unroll` loads of every block, 4, 8
 * or 16), with the kernels' own slab builder and tile-walk helpers. flags: bit
 * 0 = level 0 from the 16-bit copy, bit 1 = also the naive scan's loads, bit 2
 * = slabs with rows of at least run_min cubes summed from row runs (every level
 * and orientation the run builder accepts), bits 8..31 = run_min (0: the
 * default of mg_launch_cfg.run_min_row). Checks that each load lies inside its
 * slab and inside the map buffer, that each consumed load reads exactly the
 * element of a footprint cube (or voxel) of the box, for run slabs that each
 * row segment lies in the box on its row and indexes its row and skip entry in
 * range (run loads are clamped to the run array by the kernel), and that every
 * cube of the footprint is read once. counts host uint64 [4]: boxes, slabs,
 * lane loads (run segments for run slabs), cubes. MG_ELIMIT with the first
 * violation in the message. */
int mg_check_load_addresses(uint32_t nx, uint32_t ny, uint32_t nz, uint32_t flags, const uint32_t *boxes,
                            uint32_t n, uint32_t unroll, uint64_t *counts);

/* Footprint of each box as seen by the GPU decomposition: d_level_counts
 * device uint32 [n][n_levels] cubes per level. If d_cubes is not NULL, also
 * appends every cube as uint32 (box, level, cx, cy, cz, node) at slot
 * atomicAdd(d_count, 1) while the slot is below `cap` (d_count device uint32,
 * zeroed by the caller); order is unspecified. */
int mg_footprint(mg_graph *g, const uint32_t *d_boxes, uint32_t n, uint32_t *d_level_counts,
                 uint32_t *d_cubes, uint32_t cap, uint32_t *d_count, void *stream);

/* Transfer-function propagation (Sec. "Reconstruction", colour palette of
 * Sec. "Rendering"): d_tf device uint8 [T][S][4] RGBA8; source s of TF t gets
 * byte/255 per channel, every internal node v_n = v_a + w_n (v_b - v_a) in
 * fp32, step by step. d_node_rgba device fp32 [T][n_nodes][4]. */
int mg_propagate_tf(mg_graph *g, const uint8_t *d_tf, uint32_t T, float *d_node_rgba,
                    void *stream);

/* Per-voxel palette fetch (Sec. "Rendering": a voxel's node ID indexes the
 * colour lookup table, like a paletted texture; the same fetch on a
 * propagated visibility channel gives the visible fraction used for empty
 * space skipping). d_palette device fp32 [T][n_nodes][4] as written by
 * mg_propagate_tf; d_xyz device uint32 [n][3] voxel coordinates at mip
 * `level`; d_out device fp32 [T][n][4] = palette of the voxel's node.
 * Coordinates outside the level's dimensions give (0, 0, 0, 0).
 * MG_EINVAL for level >= n_levels. */
int mg_palette_fetch(mg_graph *g, const float *d_palette, uint32_t T, uint32_t level,
                     const uint32_t *d_xyz, uint32_t n, float *d_out, void *stream);

/* Mean colour of each box under a propagated palette (Sec. "Rendering": the
 * node of a mip voxel indexes the colour table; Sec. "Fast Sub-Volume
 * Queries": a box is the disjoint union of its footprint cubes, each holding
 * 8^l voxels of its node's mixture). d_palette device fp32 [T][n_nodes][4] as
 * written by mg_propagate_tf; d_boxes device uint32 [n][6]; d_pal_of_box device
 * uint32 [n], the palette (< T) each box is coloured with, or 0xFFFFFFFF for
 * none; d_out device fp32 [n][4] = sum over the box's cubes of 8^l times the
 * palette entry of the cube's node, divided by the box volume (fp64 sums), i.e.
 * the TF colours averaged over the box's voxels. Empty boxes and boxes without
 * a palette get zeros. */
int mg_box_colour(mg_graph *g, const float *d_palette, uint32_t T, const uint32_t *d_boxes, uint32_t n,
                  const uint32_t *d_pal_of_box, float *d_out, void *stream);

/* Mixture lookup table (Sec. "Decoder": one mixture per node, found by
 * carrying each source's unit vector through the interpolations; Sec.
 * "Range queries" answers boxes from it). Built on the host in fp64 from the
 * exact weights and stored fp32; uploaded now if the graph is on a device,
 * otherwise by mg_upload. `threads` 0 = all cores. *out_nnz (may be NULL)
 * receives the number of entries. MG_ELIMIT beyond 2^34 entries. */
int mg_lut_build(mg_graph *g, uint32_t threads, uint64_t *out_nnz);

/* Host copy of the lookup table: ptr host uint64 [n_nodes + 1]; row n is
 * seg/val[ptr[n] .. ptr[n+1]), sources in increasing order, fractions fp32;
 * err (same length) the propagated uncertainty of each fraction (Sec. "Error
 * Propagation", Eq. (error); zero for exact weights). seg, val and err may be
 * NULL (then only ptr is written). MG_ESTATE if the table was not built. */
int mg_export_lut(const mg_graph *g, uint64_t *ptr, uint32_t *seg, float *val, float *err);

/* Box histograms answered from the mixture lookup table (the paper's own
 * query, Sec. "Range queries"): the same footprint and scatter as
 * mg_query_boxes, then every scattered graph node adds count * mixture row
 * to the segments, instead of the rank-by-rank push. Same arguments and
 * output as mg_query_boxes; MG_ESTATE unless mg_lut_build ran. */
int mg_query_boxes_lut(mg_graph *g, const uint32_t *d_boxes, uint32_t n, float *d_out,
                       void *d_work, uint64_t work_bytes, void *stream);

/* Box histograms with uncertainties, for graphs with quantized weights (Sec.
 * "Error Propagation": the uncertainty of range queries; Sec. "Range
 * queries"): the lookup-table query, with every scattered graph node's count
 * c_n applied to its row once, and per segment d_err = sqrt(sum_n (c_n
 * dmu_n)^2) / |box| (the sum rule of error propagation over the nodes' terms).
 *   d_out  device fp32 [n][S] fractions (as mg_query_boxes_lut)
 *   d_err  device fp32 [n][S] their uncertainties
 * Needs mg_quantize'd graph and mg_lut_build (else MG_ESTATE) and S <= 2048
 * (MG_ELIMIT). */
int mg_query_boxes_err(mg_graph *g, const uint32_t *d_boxes, uint32_t n, float *d_out, float *d_err,
                       void *d_work, uint64_t work_bytes, void *stream);

/* Launch configuration of the GPU kernels (per graph, after mg_upload).
 * Defaults: 16, 8, 16, 256, then zeros (sizes chosen per mode). */
typedef struct {
    uint32_t unroll_big;    /* node-ID loads in flight per lane, boxes of >= 2^14 cubes: 4, 8 or 16 */
    uint32_t unroll_small;  /* the same for smaller boxes: 4, 8 or 16 */
    uint32_t unroll_naive;  /* level-0 loads in flight per lane of the naive scan: 4, 8 or 16 */
    uint32_t tf_block;      /* threads per workgroup of the propagation kernel: 64, 128, 256, 512, 1024 */
    uint32_t table_big;     /* per-box LDS hash slots, big-box tier (0: default, see below)     */
    uint32_t table_small;   /* small-box tier (0: default)                                      */
    uint32_t table_retry;   /* retry of overflowed boxes (0: the largest of 8192 that fits)     */
    uint32_t block_small;   /* threads per box in the small-box tier: 0 (128), 128 or 256       */
    uint32_t block_big;     /* threads per box in the big-box tier: 0 (512), 256 or 512.
                               Table sizes are 0 or powers of two in [64, 8192] (0: 2048 big,
                               256 small with per-source arrays; 4096 and 2048 when sources are
                               table entries); boxes that overflow every LDS table are answered
                               from global memory, so smaller tables change speed, never
                               results                                                        */
    uint32_t chunk_small;   /* boxes a small-tier workgroup takes per dequeue from its work
                               queue: 0 (one) or 1..64                                          */
    uint32_t tf_planes;     /* transfer functions per thread of the propagation kernel (their
                               gathers in flight together): 0 (default: 4), 1, 2, 4 or 8     */
    uint32_t tf_schedule;   /* order of the propagation launches: 0 (default) rank by rank, the
                               nodes in ID order; 1 the graph's step schedule (deferred when
                               built with defer = 1). Same colours either way                  */
    uint32_t run_min_row;   /* footprint slabs whose rows are at least this many cubes long are
                               summed from the rows' runs of equal node IDs where the graph
                               has them; shorter rows stream cube by cube. 0: default (128);
                               0xFFFFFFFF: never (every slab streams)                          */
} mg_launch_cfg;

int mg_get_launch(const mg_graph *g, mg_launch_cfg *out);
int mg_set_launch(mg_graph *g, const mg_launch_cfg *cfg); /* MG_EINVAL for unsupported values */

/* Autotuner: runs mg_query_boxes and mg_naive_boxes on the caller's boxes with
 * every supported unroll choice, then the table sizes and threads per box of
 * each tier one tier at a time, `reps` timed repetitions each (HIP events on
 * `stream`), keeps the fastest configuration in the graph and returns it in
 * *chosen. Synchronises `stream`; d_out and d_work as for mg_query_boxes. */
int mg_autotune(mg_graph *g, const uint32_t *d_boxes, uint32_t n, float *d_out, void *d_work,
                uint64_t work_bytes, uint32_t reps, void *stream, mg_launch_cfg *chosen);

/* Persist / restore the host graph (raw arrays with a header and checksums,
 * the quantizer's codebook included). mg_load validates the arrays (IDs in
 * range, children before parents, weights in (0, 1/2]) and returns
 * MG_EFORMAT on any mismatch. */
int mg_save(const mg_graph *g, const char *path);
int mg_load(const char *path, mg_graph **out);

/* The bit-packed graph stream of Sec. "Compression" (Table "bitstream"), for a
 * quantized graph (else MG_ESTATE). Header: sources (32 bits), fractional-input
 * flag (1, always 0), bits per node minus 1 (6), sigma_max (32, fp32 bits),
 * level-0 resolution (3 x 32), quantizer bit rate minus 1 (4), internal nodes
 * (bits per node); per level r(l) and i_min(l) (bits per node each). Bulk: per
 * level and voxel (x fastest) its node ID - i_min(l) at r(l) bits; per internal
 * node (first, second, codebook index) at 2 x bits per node + bit rate bits,
 * node = (1 - code) first + code second; per bin codeword x 2^20 and
 * sigma / sigma_max x (2^20 - 1) at 20 bits each; then (an addition) the input
 * label of each source at 32 bits. Bits per node = ceil(log2 #nodes), r(l) =
 * ceil(log2(i_max(l) - i_min(l) + 1)). Fields are unsigned, least significant
 * bit first; bit i of the stream is bit i mod 8 of byte i / 8; zero bits pad
 * the last byte.
 * mg_pack: *size = the stream's bytes; with buf == NULL only the size is
 * returned; MG_ELIMIT if capacity < *size. Host memory, caller-owned.
 * mg_unpack: a new host graph from a stream (nodes renumbered by rank as
 * mg_build does, deferred step schedule); MG_EFORMAT on any malformed or
 * truncated field. unpack(pack(g)) has g's maps, nodes, weights and codebook. */
int mg_pack(const mg_graph *g, uint8_t *buf, uint64_t capacity, uint64_t *size);
int mg_unpack(const uint8_t *buf, uint64_t size, uint32_t threads, mg_graph **out);

/* mg_unpack straight onto a GPU: the host reads the header, the node triples,
 * the codebook and the labels; the voxel data (A), r(l) bits per voxel, is
 * copied to `device` as it is and decoded there by a HIP kernel (one thread
 * per voxel) into the node maps, renumbered like mg_unpack's. The new graph is
 * on `device` as after mg_upload (library-allocated) and gives the same
 * results; its maps are never expanded in host memory, so mg_export_map copies
 * them back from the device, and mg_save, mg_pack, mg_quantize, mg_upload and
 * mg_bind_device return MG_ESTATE for it. A stored node ID out of range is
 * MG_EFORMAT (checked on the device for every voxel). `buf` is host memory,
 * read during the call only. */
int mg_unpack_device(const uint8_t *buf, uint64_t size, uint32_t threads, int device, mg_graph **out);

/* Kernel timing: when enabled, the dominant kernel of each query /
 * propagation call is bracketed by HIP events on the call's stream;
 * mg_timing_read synchronises those events and returns the summed
 * milliseconds and the number of launches since the last read. */
int mg_timing_enable(mg_graph *g, int enable);
int mg_timing_read(mg_graph *g, double *ms, uint32_t *launches);

const char *mg_last_error(void);
void mg_free(mg_graph *g);

#ifdef __cplusplus
}
#endif
#endif /* MG_H */
