// Cluster tree and block tree of the H-matrix (Section "Compression").
//
// The matrix is viewed as a hierarchy of blocks of interactions between
// clusters of points; a block is compressed when the clusters are well
// separated, max(R1, R2) < eta * dist, and kept dense when the leaves are
// reached.  Choices made where the paper is silent:
//   - a cluster is split at the midpoint of its tight bounding box along the
//     longest axis (ties: lowest axis); points on the plane go to the lower
//     child; each child keeps the parent's order; leaves hold <= leaf_size
//     points;
//   - R is half the diagonal of the tight bounding box and dist the gap
//     between the two boxes, so touching clusters are never admissible; the
//     test is R^2 < eta^2 dist^2 in FP64, evaluated without contraction
//     (this file is compiled with -ffp-contract=off) so the decision is
//     reproducible;
//   - the mirrored term of a reflective wall is singular at the mirror image
//     of the target, which is never closer to a source box than the target
//     box itself (both lie on the same side of the wall), so the same test
//     covers it;
//   - a block whose storage break-even rank floor(m n / (m + n)) is below
//     kMinLowRank is treated as not admissible (it is split or kept dense):
//     measured on the cube workloads, nearly all such blocks reach that rank
//     in the ACA and fall back to dense storage after the ACA's work;
//   - when one side of a non-admissible block is a leaf, the other is split.
#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

#include "rte_internal.h"

namespace rte {

namespace {

struct Builder {
    const std::vector<double> &pts;
    int leaf;
    ClusterTree &T;
    std::vector<int64_t> tmp;

    int build(int64_t start, int64_t stop) {
        ClusterNode nd;
        nd.start = start;
        nd.stop = stop;
        for (int a = 0; a < 3; ++a) {
            nd.bmin[a] = pts[3 * T.perm[start] + a];
            nd.bmax[a] = nd.bmin[a];
        }
        for (int64_t k = start; k < stop; ++k)
            for (int a = 0; a < 3; ++a) {
                double v = pts[3 * T.perm[k] + a];
                nd.bmin[a] = std::min(nd.bmin[a], v);
                nd.bmax[a] = std::max(nd.bmax[a], v);
            }
        int id = (int)T.nodes.size();
        T.nodes.push_back(nd);
        if (stop - start <= leaf) {
            T.leaves.push_back(id);
            return id;
        }
        int axis = 0;
        double ext = nd.bmax[0] - nd.bmin[0];
        for (int a = 1; a < 3; ++a) {
            double e = nd.bmax[a] - nd.bmin[a];
            if (e > ext) { ext = e; axis = a; }
        }
        double mid = 0.5 * (nd.bmin[axis] + nd.bmax[axis]);
        tmp.clear();
        int64_t w = start;
        for (int64_t k = start; k < stop; ++k) {
            int64_t p = T.perm[k];
            if (pts[3 * p + axis] <= mid) T.perm[w++] = p;
            else tmp.push_back(p);
        }
        std::copy(tmp.begin(), tmp.end(), T.perm.begin() + w);
        int64_t cut = w;
        if (cut == start || cut == stop) throw Error(RTE_E_INTERNAL, "cluster split produced an empty child");
        int c0 = build(start, cut);
        int c1 = build(cut, stop);
        T.nodes[id].child[0] = c0;
        T.nodes[id].child[1] = c1;
        return id;
    }
};

constexpr int64_t kMinLowRank = 24;

bool separated(const double tmin[3], const double tmax[3], const double smin[3], const double smax[3], double eta) {
    double ht[3], hs[3], g[3];
    for (int a = 0; a < 3; ++a) {
        ht[a] = 0.5 * (tmax[a] - tmin[a]);
        hs[a] = 0.5 * (smax[a] - smin[a]);
        double g1 = smin[a] - tmax[a], g2 = tmin[a] - smax[a];
        g[a] = std::max(0.0, std::max(g1, g2));
    }
    double rt2 = ht[0] * ht[0] + ht[1] * ht[1] + ht[2] * ht[2];
    double rs2 = hs[0] * hs[0] + hs[1] * hs[1] + hs[2] * hs[2];
    double d2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    double lhs = std::max(rt2, rs2);
    double rhs = (eta * eta) * d2;
    return lhs < rhs;
}

bool admissible(const ClusterNode &t, const ClusterNode &s, double eta) {
    const int64_t m = t.stop - t.start, n = s.stop - s.start;
    if (m * n / (m + n) < kMinLowRank) return false;
    return separated(t.bmin, t.bmax, s.bmin, s.bmax, eta);
}

struct BlockBuilder {
    const ClusterTree &T, &S;
    double eta;
    bool compress;
    Plan &P;
    void rec(int t, int s) {
        const ClusterNode &a = T.nodes[t], &b = S.nodes[s];
        bool tl = a.child[0] < 0, sl = b.child[0] < 0;
        if (compress && admissible(a, b, eta)) {
            P.lowrank.push_back({a.start, a.stop, b.start, b.stop});
        } else if (tl && sl) {
            P.dense.push_back({a.start, a.stop, b.start, b.stop});
        } else if (tl) {
            for (int c : b.child) rec(t, c);
        } else if (sl) {
            for (int c : a.child) rec(c, s);
        } else {
            for (int c : a.child)
                for (int d : b.child) rec(c, d);
        }
    }
};

}  // namespace

ClusterTree build_cluster_tree(const std::vector<double> &pts, int leaf_size) {
    ClusterTree T;
    int64_t n = (int64_t)pts.size() / 3;
    T.perm.resize(n);
    for (int64_t k = 0; k < n; ++k) T.perm[k] = k;
    if (n == 0) return T;
    Builder b{pts, leaf_size, T, {}};
    b.build(0, n);
    return T;
}

void validate_opts(const Mesh &m, const rte_hmat_opts_t &o) {
    RTE_REQUIRE(o.kind == RTE_VOLUME || o.kind == RTE_SURFACE, "opts.kind must be RTE_VOLUME or RTE_SURFACE");
    RTE_REQUIRE(o.leaf_size >= 1 && o.leaf_size <= 1024, "opts.leaf_size must be in [1, 1024]");
    RTE_REQUIRE(o.dense || (o.eta > 0 && std::isfinite(o.eta)), "opts.eta must be > 0");
    RTE_REQUIRE(o.dense || (o.aca_eps > 0 && o.aca_eps < 1), "opts.aca_eps must be in (0, 1)");
    RTE_REQUIRE(o.recompress == 0 || o.recompress == 1, "opts.recompress must be 0 or 1");
    RTE_REQUIRE(o.aca_hits >= 0 && o.aca_hits <= 2, "opts.aca_hits must be 0, 1 or 2");
    RTE_REQUIRE(o.precision == RTE_FP64 || o.precision == RTE_FP32 || o.precision == RTE_MIXED_BF16,
                "opts.precision must be RTE_FP64, RTE_FP32 or RTE_MIXED_BF16");
    if (o.kind == RTE_SURFACE) RTE_REQUIRE(m.L > 0, "surface matrix: the mesh has no emitting face");
}

std::unique_ptr<Plan> build_plan(const Mesh &m, const rte_hmat_opts_t &o) {
    validate_opts(m, o);
    auto P = std::make_unique<Plan>();
    P->opts = o;
    auto pts = m.positions();
    P->tgt = build_cluster_tree(pts, o.leaf_size);
    P->tgt_nat = P->tgt.perm;
    if (o.kind == RTE_VOLUME) {
        P->src = P->tgt;
        P->src_nat = P->tgt_nat;
    } else {
        P->src = build_cluster_tree(m.emitting_positions(), o.leaf_size);
        P->src_nat.resize(P->src.perm.size());
        for (size_t k = 0; k < P->src.perm.size(); ++k) P->src_nat[k] = m.emitting[P->src.perm[k]];
    }
    BlockBuilder bb{P->tgt, P->src, o.eta, !o.dense, *P};
    bb.rec(0, 0);
    for (int id : P->tgt.leaves) P->tgt_leaves.push_back({P->tgt.nodes[id].start, P->tgt.nodes[id].stop});
    P->leaf_start.push_back(0);
    for (auto &lf : P->tgt_leaves) {
        P->leaf_start.back() = lf.first;
        P->leaf_start.push_back(lf.second);
    }
    P->row_leaf.resize(P->tgt_nat.size());
    for (size_t li = 0; li < P->tgt_leaves.size(); ++li)
        for (int64_t r = P->tgt_leaves[li].first; r < P->tgt_leaves[li].second; ++r) P->row_leaf[(size_t)r] = (int32_t)li;
    return P;
}

struct PlanCache {
    std::mutex mu;
    std::map<std::tuple<int, int, int, double>, std::shared_ptr<const Plan>> plans;
};

std::shared_ptr<PlanCache> new_plan_cache() { return std::make_shared<PlanCache>(); }

std::shared_ptr<const Plan> mesh_plan(const Mesh &m, const rte_hmat_opts_t &o) {
    validate_opts(m, o);
    RTE_REQUIRE(m.plans != nullptr, "mesh_plan: mesh without a plan cache");
    const auto key = std::make_tuple((int)o.kind, (int)(o.dense != 0), (int)o.leaf_size, o.dense ? 0.0 : o.eta);
    PlanCache &C = *m.plans;
    {
        std::lock_guard<std::mutex> g(C.mu);
        auto it = C.plans.find(key);
        if (it != C.plans.end()) return it->second;
    }
    std::shared_ptr<const Plan> P = build_plan(m, o);   // outside the lock: G and S build theirs concurrently
    std::lock_guard<std::mutex> g(C.mu);
    if (C.plans.size() >= 16) C.plans.clear();   // a bound, not a policy: a handful of option sets in practice
    auto ins = C.plans.emplace(key, P);
    return ins.first->second;
}

}  // namespace rte
