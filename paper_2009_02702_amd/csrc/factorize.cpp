// Greedy factorization of the mixtures into linear interpolations (Sec.
// "Compression", Eqs. greedy1 / greedy2; Sec. "Implementation Details",
// maximum search with the two-stage cutoff tau).
//
// A mixture is a sparse vector of integer counts over node IDs (initially the
// sources). Factoring the pair (i, j) out of a mixture h replaces components i
// and j by one component: the node lambda = (h_i e_i + h_j e_j) / (h_i + h_j),
// with count h_i + h_j. lambda is re-used whenever another mixture factors the
// same pair in the same ratio. Stage 1 takes the mixtures with more than tau
// components and repeatedly picks the pair of largest score phi over them
// (ties: the smallest (i, j)), factoring it out of every stage-1 mixture that
// holds both; a mixture leaves stage 1 once it has tau components or fewer.
// Stage 2 visits the remaining mixtures in scanline order and factors each
// down to one component, taking its pair of largest score over the mixtures
// not yet finished.
//   phi1 (max-occurrence): number of mixtures holding both i and j;
//   phi2 (max-reduction): per mixture holding both, ||h||_0 - 1 if that is
//   above 2, else 2.
#include <algorithm>
#include <cstdint>
#include <queue>
#include <string>
#include <unordered_map>
#include <vector>

#include "mg_internal.hpp"

namespace mg {
namespace {

using Comp = std::pair<uint32_t, uint64_t>;  // (node, count)

inline uint64_t pair_key(uint32_t i, uint32_t j)
{
    return i < j ? (uint64_t(i) << 32) | j : (uint64_t(j) << 32) | i;
}

uint64_t gcd_u64(uint64_t a, uint64_t b)
{
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

struct Entry {
    int64_t score;
    uint64_t key;
    // priority: larger score first, then the smaller pair
    bool operator<(const Entry &o) const { return score != o.score ? score < o.score : key > o.key; }
};

struct NodeKey {
    uint32_t a, b;
    uint64_t wn, wd;
    bool operator==(const NodeKey &o) const { return a == o.a && b == o.b && wn == o.wn && wd == o.wd; }
};
struct NodeKeyHash {
    size_t operator()(const NodeKey &k) const
    {
        uint64_t h = (uint64_t(k.a) << 32 | k.b) * 0x9E3779B97F4A7C15ull;
        h ^= k.wn * 0xC2B2AE3D27D4EB4Full;
        h ^= k.wd * 0x165667B19E3779F9ull;
        return size_t(h ^ (h >> 29));
    }
};

class Greedy {
public:
    Greedy(uint32_t strategy, RawDag *d) : strategy_(strategy), d_(d) {}

    int64_t weight(size_t n) const
    {
        if (n < 2) return 0;
        if (strategy_ == MG_FACTOR_GREEDY_OCCURRENCE) return 1;
        return n > 2 ? int64_t(n) - 1 : 2;
    }

    // Add (sign +1) or remove (-1) the score contributions of one mixture.
    void account(std::unordered_map<uint64_t, int64_t> &score, const std::vector<Comp> &h, int sign) const
    {
        const int64_t w = weight(h.size()) * sign;
        if (!w) return;
        for (size_t x = 0; x < h.size(); ++x)
            for (size_t y = x + 1; y < h.size(); ++y) score[pair_key(h[x].first, h[y].first)] += w;
    }

    // The node (c_i e_i + c_j e_j) / (c_i + c_j): heavier part first (ties:
    // lower ID), weight of the other part as a reduced fraction; created once.
    uint32_t node(uint32_t i, uint64_t ci, uint32_t j, uint64_t cj)
    {
        uint32_t a = i, b = j;
        uint64_t wn = cj;
        if (ci < cj || (ci == cj && j < i)) a = j, b = i, wn = ci;
        uint64_t wd = ci + cj;
        const uint64_t g = gcd_u64(wn, wd);
        wn /= g, wd /= g;
        const NodeKey k{a, b, wn, wd};
        auto it = nodes_.find(k);
        if (it != nodes_.end()) return it->second;
        const uint32_t id = uint32_t(d_->a.size());
        d_->a.push_back(a), d_->b.push_back(b), d_->wn.push_back(wn), d_->wd.push_back(wd);
        d_->mix.push_back(d_->mix[a] + d_->mix[b]);
        nodes_.emplace(k, id);
        return id;
    }

    // Replace components i and j of h by their node; returns the node.
    uint32_t factor(std::vector<Comp> &h, uint32_t i, uint32_t j)
    {
        auto fi = std::lower_bound(h.begin(), h.end(), Comp{i, 0});
        const uint64_t ci = fi->second;
        h.erase(fi);
        auto fj = std::lower_bound(h.begin(), h.end(), Comp{j, 0});
        const uint64_t cj = fj->second;
        h.erase(fj);
        const uint32_t n = node(i, ci, j, cj);
        const Comp c{n, ci + cj};
        h.insert(std::lower_bound(h.begin(), h.end(), c), c);
        return n;
    }

private:
    uint32_t strategy_;
    RawDag *d_;
    std::unordered_map<NodeKey, uint32_t, NodeKeyHash> nodes_;
};

bool holds(const std::vector<Comp> &h, uint32_t n)
{
    auto it = std::lower_bound(h.begin(), h.end(), Comp{n, 0});
    return it != h.end() && it->first == n;
}

}  // namespace

int greedy_factorize(uint32_t nseg, std::vector<std::vector<std::pair<uint32_t, uint64_t>>> &mix, uint32_t strategy,
                     uint32_t tau, RawDag *d, std::vector<uint32_t> *root, std::string *err)
{
    if (strategy != MG_FACTOR_GREEDY_REDUCTION && strategy != MG_FACTOR_GREEDY_OCCURRENCE) {
        *err = "unknown factorizer";
        return MG_EINVAL;
    }
    d->nseg = nseg;
    for (uint32_t s = 0; s < nseg; ++s)
        d->a.push_back(s), d->b.push_back(s), d->wn.push_back(0), d->wd.push_back(1), d->mix.push_back(1);
    Greedy G(strategy, d);
    const size_t M = mix.size();
    for (auto &h : mix) std::sort(h.begin(), h.end());

    // ---- stage 1: mixtures with more than tau components, global maximum search
    std::vector<uint8_t> in1(M, 0);
    std::vector<std::vector<uint32_t>> holders(nseg);  // node -> stage-1 mixtures that received it
    std::unordered_map<uint64_t, int64_t> score;
    for (size_t m = 0; m < M; ++m) {
        if (mix[m].size() < 2 || mix[m].size() <= tau) continue;
        in1[m] = 1;
        G.account(score, mix[m], +1);
        for (const Comp &c : mix[m]) holders[c.first].push_back(uint32_t(m));
    }
    std::priority_queue<Entry> pq;
    for (const auto &kv : score)
        if (kv.second > 0) pq.push(Entry{kv.second, kv.first});
    std::vector<uint32_t> both;
    while (!pq.empty()) {
        const Entry top = pq.top();
        pq.pop();
        auto it = score.find(top.key);
        const int64_t cur = it == score.end() ? 0 : it->second;
        if (cur != top.score) {  // stale: scores only fall without a new entry
            if (cur > 0) pq.push(Entry{cur, top.key});
            continue;
        }
        const uint32_t i = uint32_t(top.key >> 32), j = uint32_t(top.key & 0xFFFFFFFFu);
        const std::vector<uint32_t> &hi = holders[i], &hj = holders[j];
        const std::vector<uint32_t> &shorter = hi.size() <= hj.size() ? hi : hj;
        both.clear();
        for (uint32_t m : shorter)
            if (in1[m] && holds(mix[m], i) && holds(mix[m], j)) both.push_back(m);
        std::sort(both.begin(), both.end());
        both.erase(std::unique(both.begin(), both.end()), both.end());
        for (uint32_t m : both) {
            std::vector<Comp> &h = mix[m];
            G.account(score, h, -1);
            const uint32_t n = G.factor(h, i, j);
            if (n >= holders.size()) holders.resize(size_t(n) + 1);
            if (h.size() > tau && h.size() >= 2) {
                holders[n].push_back(m);
                G.account(score, h, +1);
                for (const Comp &c : h)  // pairs with the new component may have grown
                    if (c.first != n) {
                        const uint64_t k = pair_key(c.first, n);
                        pq.push(Entry{score[k], k});
                    }
            } else {
                in1[m] = 0;
            }
        }
        if (score[top.key] != 0) {
            *err = "greedy factorization: pair score out of step";
            return MG_EFORMAT;
        }
    }

    // ---- stage 2: the rest in scanline order, each mixture down to one component
    score.clear();
    for (size_t m = 0; m < M; ++m)
        if (mix[m].size() >= 2) G.account(score, mix[m], +1);
    for (size_t m = 0; m < M; ++m) {
        std::vector<Comp> &h = mix[m];
        while (h.size() >= 2) {
            Entry best{-1, 0};
            for (size_t x = 0; x < h.size(); ++x)
                for (size_t y = x + 1; y < h.size(); ++y) {
                    const uint64_t k = pair_key(h[x].first, h[y].first);
                    const Entry e{score[k], k};
                    if (best < e) best = e;
                }
            G.account(score, h, -1);
            G.factor(h, uint32_t(best.key >> 32), uint32_t(best.key & 0xFFFFFFFFu));
            G.account(score, h, +1);
        }
    }
    root->resize(M);
    for (size_t m = 0; m < M; ++m) {
        if (mix[m].size() != 1) {
            *err = "greedy factorization left an empty mixture";
            return MG_EFORMAT;
        }
        (*root)[m] = mix[m][0].first;
    }
    return MG_OK;
}

}  // namespace mg
