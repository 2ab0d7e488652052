// Bit-packed graph stream (Sec. "Compression", Table "bitstream"): the saved
// form of a graph with quantized weights.
//
// Fields are written in the table's order, each as an unsigned integer of the
// stated width, least significant bit first, into a byte string whose bit i is
// bit (i mod 8) of byte i / 8; the stream ends with zero bits up to a byte.
//   (1) sources, 32 bits            (2) fractional input, 1 bit (always 0)
//   (3) bits per node minus 1, 6    (4) sigma_max, 32 (IEEE fp32 bits)
//   (5) level-0 resolution, 3 x 32  (6) quantizer bit rate minus 1, 4
//   (7) internal nodes, (3) bits
//   per level: (8) voxel bits r(l), (9) i_min(l), (3) bits each
//   (A) per level, per voxel (x fastest): node ID - i_min(l), r(l) bits
//   (B) per internal node, in ID order: first, second ((3) bits each) and the
//       codebook index (b bits): node = (1 - code) first + code second
//   (C) per codebook bin: codeword * 2^20 and sigma / sigma_max * (2^20 - 1),
//       20 bits each
//   (D) per source: its label in the input volume, 32 bits (the paper's
//       sources are the input IDs themselves; here sources are the distinct
//       labels, numbered in increasing order)
// Bits per node = ceil(log2(#nodes)) (at least 1); r(l) = ceil(log2(i_max(l) -
// i_min(l) + 1)) with i_min / i_max the smallest / largest node ID of level l.
// The number of levels follows from the resolution (halving until 1^3).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mg_internal.hpp"

namespace mg {
namespace {

uint32_t ceil_log2(uint64_t v)  // smallest r with 2^r >= v (v >= 1)
{
    uint32_t r = 0;
    while ((uint64_t(1) << r) < v) ++r;
    return r;
}

class BitWriter {
  public:
    explicit BitWriter(std::vector<uint8_t> *out) : out_(out) {}
    void put(uint64_t v, uint32_t bits)
    {
        for (uint32_t i = 0; i < bits;) {  // up to 8 bits at a time, into the current byte
            const uint32_t bit = uint32_t(pos_ & 7), take = std::min(8 - bit, bits - i);
            if (bit == 0) out_->push_back(0);
            out_->back() |= uint8_t(((v >> i) & ((1u << take) - 1)) << bit);
            pos_ += take, i += take;
        }
    }
    uint64_t bits() const { return pos_; }

  private:
    std::vector<uint8_t> *out_;
    uint64_t pos_ = 0;
};

class BitReader {
  public:
    BitReader(const uint8_t *p, uint64_t size) : p_(p), nbits_(size * 8) {}
    // false when the stream ends before the field does
    bool get(uint32_t bits, uint64_t *v)
    {
        if (bits > nbits_ - std::min(pos_, nbits_)) return false;
        uint64_t r = 0;
        for (uint32_t i = 0; i < bits;) {
            const uint32_t bit = uint32_t(pos_ & 7), take = std::min(8 - bit, bits - i);
            r |= uint64_t((p_[pos_ >> 3] >> bit) & ((1u << take) - 1)) << i;
            pos_ += take, i += take;
        }
        *v = r;
        return true;
    }
    uint64_t pos() const { return pos_; }
    void skip(uint64_t bits) { pos_ += bits; }

  private:
    const uint8_t *p_;
    uint64_t nbits_, pos_ = 0;
};

}  // namespace

int pack_graph(const Graph &g, std::vector<uint8_t> *out, std::string *err)
{
    const uint32_t S = g.nseg, N = g.n_nodes, b = g.quant_bits;
    if (!b || g.node_code.size() != N || g.codebook.size() != (size_t(1) << b)) {
        *err = "the graph stream stores quantized weights: quantize the graph first (mg_quantize)";
        return MG_ESTATE;
    }
    const uint32_t bpn = std::max<uint32_t>(1, ceil_log2(N));
    const uint32_t B = 1u << b;
    const float sigma_max = *std::max_element(g.code_sigma.begin(), g.code_sigma.end());
    const double scale = double(1u << kCodeBits), smax_q = double((1u << kCodeBits) - 1);
    for (float c : g.codebook)
        if (!(c > 0.f && c < 1.f) || std::floor(double(c) * scale) != double(c) * scale) {
            *err = "graph stream: a codeword is not a 20-bit fraction in (0, 1)";
            return MG_ESTATE;
        }
    // per level: smallest and largest node ID
    std::vector<uint32_t> lo(g.n_levels), r(g.n_levels);
    for (uint32_t l = 0; l < g.n_levels; ++l) {
        const auto first = g.maps.begin() + int64_t(g.lev_off[l]), last = g.maps.begin() + int64_t(g.lev_off[l + 1]);
        const auto mm = std::minmax_element(first, last);
        lo[l] = *mm.first;
        r[l] = ceil_log2(uint64_t(*mm.second) - *mm.first + 1);
    }
    out->clear();
    try {
        uint64_t total = 32 + 1 + 6 + 32 + 96 + 4 + bpn + uint64_t(g.n_levels) * 2 * bpn;
        for (uint32_t l = 0; l < g.n_levels; ++l) total += uint64_t(r[l]) * (g.lev_off[l + 1] - g.lev_off[l]);
        total += uint64_t(N - S) * (2 * bpn + b) + uint64_t(B) * 2 * kCodeBits + 32ull * S;
        out->reserve((total + 7) / 8);
    } catch (...) {
        *err = "host allocation of the graph stream failed";
        return MG_ENOMEM;
    }
    BitWriter w(out);
    uint32_t smax_bits;
    std::memcpy(&smax_bits, &sigma_max, 4);
    w.put(S, 32);
    w.put(0, 1);
    w.put(bpn - 1, 6);
    w.put(smax_bits, 32);
    for (int a = 0; a < 3; ++a) w.put(g.dims[a], 32);
    w.put(b - 1, 4);
    w.put(N - S, bpn);
    for (uint32_t l = 0; l < g.n_levels; ++l) w.put(r[l], bpn), w.put(lo[l], bpn);
    for (uint32_t l = 0; l < g.n_levels; ++l)
        for (uint64_t i = g.lev_off[l]; i < g.lev_off[l + 1]; ++i) w.put(g.maps[i] - lo[l], r[l]);
    for (uint32_t n = S; n < N; ++n) {
        const uint32_t k = g.node_code[n];
        // stored weights are <= 1/2: the codeword itself, or 1 - codeword with the predecessors swapped
        const bool same = g.alpha[n] == g.codebook[k];
        w.put(same ? g.child_a[n] : g.child_b[n], bpn);
        w.put(same ? g.child_b[n] : g.child_a[n], bpn);
        w.put(k, b);
    }
    for (uint32_t k = 0; k < B; ++k) {
        w.put(uint64_t(double(g.codebook[k]) * scale), kCodeBits);
        const double m = sigma_max > 0.f ? std::floor(double(g.code_sigma[k]) / double(sigma_max) * smax_q + 0.5) : 0.0;
        w.put(uint64_t(std::min(m, smax_q)), kCodeBits);
    }
    for (uint32_t s = 0; s < S; ++s) w.put(g.seg_ids[s], 32);
    return MG_OK;
}

int unpack_graph(const uint8_t *buf, uint64_t size, uint32_t threads, Graph *g, std::string *err, StreamMaps *dev)
{
    BitReader rd(buf, size);
    uint64_t v = 0;
    auto fail = [&](const char *what) {
        *err = std::string("graph stream: ") + what;
        return MG_EFORMAT;
    };
#define MG_GET(bits, what)                  \
    do {                                    \
        if (!rd.get((bits), &v)) return fail(what); \
    } while (0)
    MG_GET(32, "truncated header");
    const uint32_t S = uint32_t(v);
    MG_GET(1, "truncated header");
    if (v) return fail("fractional input volumes are not supported");
    MG_GET(6, "truncated header");
    const uint32_t bpn = uint32_t(v) + 1;
    MG_GET(32, "truncated header");
    const uint32_t smax_bits = uint32_t(v);
    float sigma_max;
    std::memcpy(&sigma_max, &smax_bits, 4);
    for (int a = 0; a < 3; ++a) {
        MG_GET(32, "truncated header");
        g->dims[a] = uint32_t(v);
    }
    MG_GET(4, "truncated header");
    const uint32_t b = uint32_t(v) + 1;
    MG_GET(bpn, "truncated header");
    const uint64_t n_int = v;
    const uint64_t nvox = uint64_t(g->dims[0]) * g->dims[1] * g->dims[2];
    if (S == 0 || nvox == 0 || nvox >= (1ull << 31)) return fail("bad source count or resolution");
    if (bpn > 32 || uint64_t(S) + n_int > 0xFFFFFFFFull) return fail("node count out of range");
    const uint32_t N = uint32_t(S + n_int);
    if (bpn != std::max<uint32_t>(1, ceil_log2(N))) return fail("bits per node do not match the node count");
    if (!(sigma_max >= 0.f) || !std::isfinite(sigma_max)) return fail("bad sigma_max");
    level_dims(g->dims, &g->lev_dims);
    g->n_levels = uint32_t(g->lev_dims.size() / 3);
    if (g->n_levels > MG_MAX_LEVELS) return fail("too many mip levels");
    g->lev_off.assign(g->n_levels + 1, 0);
    for (uint32_t l = 0; l < g->n_levels; ++l)
        g->lev_off[l + 1] =
            g->lev_off[l] + uint64_t(g->lev_dims[3 * l]) * g->lev_dims[3 * l + 1] * g->lev_dims[3 * l + 2];
    std::vector<uint32_t> r(g->n_levels), lo(g->n_levels);
    for (uint32_t l = 0; l < g->n_levels; ++l) {
        MG_GET(bpn, "truncated level table");
        r[l] = uint32_t(v);
        MG_GET(bpn, "truncated level table");
        lo[l] = uint32_t(v);
        if (r[l] > 32 || lo[l] >= N) return fail("bad level table");
    }
    // (A) before anything large is allocated, check that the stream can hold it
    uint64_t need = 0;
    for (uint32_t l = 0; l < g->n_levels; ++l) need += uint64_t(r[l]) * (g->lev_off[l + 1] - g->lev_off[l]);
    need += n_int * (2 * bpn + b) + (uint64_t(1) << b) * 2 * kCodeBits + 32ull * S;
    if (rd.pos() + need > size * 8) return fail("truncated bulk data");
    if (dev) {  // (A) stays in the stream, to be decoded on the GPU
        dev->a_bit = rd.pos();
        dev->r = r;
        dev->lo = lo;
        dev->bit_off.assign(g->n_levels, 0);
        uint64_t off = 0;
        for (uint32_t l = 0; l < g->n_levels; ++l) {
            dev->bit_off[l] = off;
            off += uint64_t(r[l]) * (g->lev_off[l + 1] - g->lev_off[l]);
        }
        rd.skip(off);
        g->maps.clear();
        g->maps_on_device = true;
    } else {
        try {
            g->maps.assign(g->lev_off[g->n_levels], 0);
        } catch (...) {
            *err = "host allocation of the node maps failed";
            return MG_ENOMEM;
        }
        for (uint32_t l = 0; l < g->n_levels; ++l) {
            const uint64_t limit = l == 0 ? S : N;  // level-0 voxels are sources
            for (uint64_t i = g->lev_off[l]; i < g->lev_off[l + 1]; ++i) {
                MG_GET(r[l], "truncated voxel data");
                const uint64_t id = uint64_t(lo[l]) + v;
                if (id >= limit) return fail("voxel node ID out of range");
                g->maps[i] = uint32_t(id);
            }
        }
    }
    // (B) nodes, then (C) the codebook they index
    std::vector<uint32_t> first(n_int), second(n_int), code(n_int);
    for (uint64_t j = 0; j < n_int; ++j) {
        MG_GET(bpn, "truncated node data");
        first[j] = uint32_t(v);
        MG_GET(bpn, "truncated node data");
        second[j] = uint32_t(v);
        MG_GET(b, "truncated node data");
        code[j] = uint32_t(v);
        if (first[j] >= S + j || second[j] >= S + j || first[j] == second[j])
            return fail("a node's predecessor is not an earlier node");
    }
    const uint32_t B = 1u << b;
    std::vector<float> cw(B), sg(B);
    for (uint32_t k = 0; k < B; ++k) {
        MG_GET(kCodeBits, "truncated codebook");
        if (v == 0) return fail("a codeword is 0");
        cw[k] = float(double(v) / double(1u << kCodeBits));
        MG_GET(kCodeBits, "truncated codebook");
        sg[k] = code_sigma_value(sigma_max, uint32_t(v));
    }
    g->seg_ids.assign(S, 0);
    for (uint32_t s = 0; s < S; ++s) {
        MG_GET(32, "truncated segment labels");
        g->seg_ids[s] = uint32_t(v);
    }
#undef MG_GET
    RawDag d;
    d.nseg = S;
    for (uint32_t s = 0; s < S; ++s) {
        d.a.push_back(s), d.b.push_back(s), d.wn.push_back(0), d.wd.push_back(1), d.mix.push_back(1);
        d.alpha.push_back(0.f), d.sigma.push_back(0.f), d.code.push_back(0);
    }
    for (uint64_t j = 0; j < n_int; ++j) {
        uint32_t x = first[j], y = second[j];
        float c = cw[code[j]];
        if (c > 0.5f) std::swap(x, y), c = 1.0f - c;  // stored with w <= 1/2 (exact in fp32)
        uint64_t num = 0, den = 1;
        weight_fraction(c, &num, &den);
        d.a.push_back(x), d.b.push_back(y), d.wn.push_back(num), d.wd.push_back(den);
        d.mix.push_back(d.mix[x] + d.mix[y]);
        d.alpha.push_back(c), d.sigma.push_back(sg[code[j]]), d.code.push_back(code[j]);
    }
    g->nseg = S;
    if (int rc = finalize_dag(d, true, 0, resolve_threads(threads), g, err, dev ? &dev->perm : nullptr)) return rc;
    g->quant_bits = b;
    g->codebook = std::move(cw);
    g->code_sigma = std::move(sg);
    return validate_graph(*g, err);
}

}  // namespace mg
