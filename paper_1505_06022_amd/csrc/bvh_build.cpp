// Host construction of the multiple-threaded BVH (Sec. 3.1).
//
// 1. Top-down SAH build with binned centroids (bins per axis, leaves of at
//    most max_leaf triangles; a node larger than max_leaf is always split).
//    Optionally with spatial splits as well (Stich, Friedrich and Dietrich,
//    "Spatial splits in bounding volume hierarchies", HPG 2009): where the
//    best object split leaves children whose boxes overlap by more than
//    split_alpha of the scene box's area, planes through the node's box are
//    also tried, each straddling triangle clipped to both sides; a triangle
//    may then sit in several leaves, each time with the box of its part.
// 2. Threading: for each of the six principal directions the tree is walked
//    in preorder with, at every inner node, the child whose box centre comes
//    first along that direction visited first.  Each node stores its skip
//    ("miss") link; the "hit" link of an inner node is implicitly the next
//    node of that preorder, so a hit walks forward through memory.
// 3. Packing into 16-byte nodes (box quantised outward to a 16-bit scene
//    grid, one copy per direction) and 48-byte triangles in leaf order.
#include "bvh_build.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <future>
#include <thread>

namespace pm {
namespace {

struct Box {
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    void grow(const Box &b) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], b.lo[a]);
            hi[a] = std::max(hi[a], b.hi[a]);
        }
    }
    void grow(const float *p) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], p[a]);
            hi[a] = std::max(hi[a], p[a]);
        }
    }
    double area() const {
        double d[3];
        for (int a = 0; a < 3; ++a) d[a] = hi[a] >= lo[a] ? (double)hi[a] - lo[a] : 0.0;
        return 2.0 * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0]);
    }
};

struct TNode {
    Box box;
    int32_t left = -1, right = -1;  // left < 0: leaf
    int32_t start = 0, count = 0;
};

struct Builder {
    const float *V;
    int64_t n;
    int bins, max_leaf;
    double trav_cost;
    std::vector<Box> tb;
    std::vector<float> cen;
    std::vector<int32_t> idx;
    int par_depth;

    int32_t build(int32_t start, int32_t count, int depth, std::vector<TNode> &out) {
        int32_t ni = (int32_t)out.size();
        out.emplace_back();
        Box nb, cb;
        for (int32_t i = start; i < start + count; ++i) {
            nb.grow(tb[idx[i]]);
            cb.grow(&cen[3 * (size_t)idx[i]]);
        }
        out[ni].box = nb;
        auto make_leaf = [&]() {
            out[ni].left = out[ni].right = -1;
            out[ni].start = start;
            out[ni].count = count;
            return ni;
        };
        if (count == 1) return make_leaf();

        // binned SAH over the three axes
        double best_cost = INFINITY;
        int best_axis = -1, best_split = -1;
        const int B = bins;
        std::vector<Box> bb(B);
        std::vector<int32_t> bc(B);
        std::vector<double> rarea(B);
        std::vector<int32_t> rcnt(B);
        for (int a = 0; a < 3; ++a) {
            float ext = cb.hi[a] - cb.lo[a];
            if (!(ext > 0.0f)) continue;
            double scale = (double)B / (double)ext;
            for (int b = 0; b < B; ++b) { bb[b] = Box(); bc[b] = 0; }
            for (int32_t i = start; i < start + count; ++i) {
                int32_t t = idx[i];
                int b = (int)(((double)cen[3 * (size_t)t + a] - cb.lo[a]) * scale);
                b = std::min(std::max(b, 0), B - 1);
                bb[b].grow(tb[t]);
                bc[b]++;
            }
            Box acc;
            int32_t c = 0;
            for (int b = B - 1; b > 0; --b) {
                acc.grow(bb[b]);
                c += bc[b];
                rarea[b] = acc.area();
                rcnt[b] = c;
            }
            acc = Box();
            c = 0;
            for (int b = 0; b < B - 1; ++b) {
                acc.grow(bb[b]);
                c += bc[b];
                int32_t cr = rcnt[b + 1];
                if (c == 0 || cr == 0) continue;
                double cost = acc.area() * c + rarea[b + 1] * cr;
                if (cost < best_cost) {
                    best_cost = cost;
                    best_axis = a;
                    best_split = b;
                }
            }
        }
        double parea = nb.area();
        double split_cost = best_axis >= 0 ? trav_cost + (parea > 0 ? best_cost / parea : 0.0) : INFINITY;
        if (count <= max_leaf && (double)count <= split_cost) return make_leaf();

        int32_t nl;
        if (best_axis < 0) {
            if (count <= max_leaf) return make_leaf();
            nl = count / 2;  // coincident centroids: split the index range
        } else {
            int a = best_axis;
            float ext = cb.hi[a] - cb.lo[a];
            double scale = (double)B / (double)ext;
            auto mid = std::partition(idx.begin() + start, idx.begin() + start + count, [&](int32_t t) {
                int b = (int)(((double)cen[3 * (size_t)t + a] - cb.lo[a]) * scale);
                b = std::min(std::max(b, 0), B - 1);
                return b <= best_split;
            });
            nl = (int32_t)(mid - (idx.begin() + start));
            if (nl == 0 || nl == count) nl = count / 2;
        }
        int32_t l, r;
        if (depth < par_depth && count > 50000) {
            std::vector<TNode> right_nodes;
            auto fut = std::async(std::launch::async, [&]() {
                return build(start + nl, count - nl, depth + 1, right_nodes);
            });
            l = build(start, nl, depth + 1, out);
            fut.get();
            int32_t off = (int32_t)out.size();
            for (auto &nd : right_nodes) {
                if (nd.left >= 0) {
                    nd.left += off;
                    nd.right += off;
                }
                out.push_back(nd);
            }
            r = off;
        } else {
            l = build(start, nl, depth + 1, out);
            r = build(start + nl, count - nl, depth + 1, out);
        }
        out[ni].left = l;
        out[ni].right = r;
        out[ni].start = out[ni].count = 0;
        return ni;
    }
};

// Spatial-split build.  A reference is a triangle with the box of its part
// inside the region it was clipped to.  Boxes are float, rounded outward from
// the double clipping, so each contains the exact part: the union of a
// triangle's leaf boxes covers it.
struct Ref {
    int32_t tri;
    Box box;
};

// A convex polygon in double: a triangle clipped by the six planes of a box
// has at most 9 vertices, and each cut by one more plane adds at most one.
struct Poly {
    double v[12][3];
    int n = 0;
};

// The part of p on one side of the plane x_a = pl (below: x_a <= pl).
void clip_plane(const Poly &p, int a, double pl, bool below, Poly &out) {
    out.n = 0;
    for (int i = 0; i < p.n; ++i) {
        const double *u = p.v[i], *w = p.v[(i + 1) % p.n];
        const bool uin = below ? u[a] <= pl : u[a] >= pl, win = below ? w[a] <= pl : w[a] >= pl;
        if (uin) std::memcpy(out.v[out.n++], u, sizeof(double) * 3);
        if (uin != win) {
            const double f = (pl - u[a]) / (w[a] - u[a]);
            for (int c = 0; c < 3; ++c) out.v[out.n][c] = u[c] + f * (w[c] - u[c]);
            out.v[out.n][a] = pl;
            ++out.n;
        }
    }
}

// The polygon of triangle t inside the region [rlo, rhi].
Poly tri_in_box(const float *V, int32_t t, const double rlo[3], const double rhi[3]) {
    Poly p, q;
    p.n = 3;
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a) p.v[k][a] = V[9 * (size_t)t + 3 * k + a];
    for (int a = 0; a < 3 && p.n; ++a) {
        double lo = p.v[0][a], hi = lo;
        for (int i = 1; i < p.n; ++i) lo = std::min(lo, p.v[i][a]), hi = std::max(hi, p.v[i][a]);
        if (lo < rlo[a]) {  // only planes that cut the polygon
            clip_plane(p, a, rlo[a], false, q);
            p = q;
        }
        if (hi > rhi[a]) {
            clip_plane(p, a, rhi[a], true, q);
            p = q;
        }
    }
    return p;
}

// The box of p within the region [rlo, rhi], rounded outward to float (so it
// contains the exact part); empty if p is.
Box poly_box(const Poly &p, const double rlo[3], const double rhi[3]) {
    Box b;
    if (p.n == 0) return b;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < p.n; ++i)
        for (int a = 0; a < 3; ++a) {
            const double x = std::min(std::max(p.v[i][a], rlo[a]), rhi[a]);
            lo[a] = std::min(lo[a], x);
            hi[a] = std::max(hi[a], x);
        }
    for (int a = 0; a < 3; ++a) {  // rounding is monotone: round the extremes outward
        float l = (float)lo[a], h = (float)hi[a];
        if ((double)l > lo[a]) l = std::nextafter(l, -INFINITY);
        if ((double)h < hi[a]) h = std::nextafter(h, INFINITY);
        b.lo[a] = l;
        b.hi[a] = h;
    }
    return b;
}

// Box of the part of triangle t inside region [rlo, rhi] (clipped in double,
// rounded outward to float); empty if none.
Box clip_tri(const float *V, int32_t t, const double rlo[3], const double rhi[3]) {
    return poly_box(tri_in_box(V, t, rlo, rhi), rlo, rhi);
}

double overlap_area(const Box &a, const Box &b) {
    Box r;
    for (int k = 0; k < 3; ++k) {
        r.lo[k] = std::max(a.lo[k], b.lo[k]);
        r.hi[k] = std::min(a.hi[k], b.hi[k]);
        if (!(r.lo[k] <= r.hi[k])) return 0.0;
    }
    return r.area();
}

struct SplitBuilder {
    const float *V;
    int bins, max_leaf;
    double trav_cost, min_overlap;  // split_alpha x the scene box's area
    int par_depth;

    // Builds the subtree of refs into out (node indices local to out) with its
    // leaves' triangle indices appended to leaf (leaf starts local to leaf).
    // budget: references this subtree may add by spatial splits (its share of
    // the whole build's allowance, so the result does not depend on threads)
    int32_t build(std::vector<Ref> &refs, int depth, int64_t budget, std::vector<TNode> &out,
                  std::vector<int32_t> &leaf) {
        int32_t ni = (int32_t)out.size();
        out.emplace_back();
        const int32_t count = (int32_t)refs.size();
        Box nb, cb;
        for (const Ref &r : refs) {
            nb.grow(r.box);
            float c[3];
            for (int a = 0; a < 3; ++a) c[a] = 0.5f * (r.box.lo[a] + r.box.hi[a]);
            cb.grow(c);
        }
        out[ni].box = nb;
        auto make_leaf = [&]() {
            out[ni].left = out[ni].right = -1;
            out[ni].start = (int32_t)leaf.size();
            out[ni].count = count;
            for (const Ref &r : refs) leaf.push_back(r.tri);
            std::vector<Ref>().swap(refs);
            return ni;
        };
        if (count == 1) return make_leaf();

        const int B = bins;
        std::vector<Box> bb(B), rb(B);
        std::vector<int32_t> bc(B), ec(B), rc(B);
        // object split: binned centroids, as in Builder
        double best_cost = INFINITY;
        int best_axis = -1, best_split = -1;
        Box best_l, best_r;
        for (int a = 0; a < 3; ++a) {
            const float ext = cb.hi[a] - cb.lo[a];
            if (!(ext > 0.0f)) continue;
            const double scale = (double)B / (double)ext;
            for (int b = 0; b < B; ++b) bb[b] = Box(), bc[b] = 0;
            for (const Ref &r : refs) {
                int b = (int)(((double)(0.5f * (r.box.lo[a] + r.box.hi[a])) - cb.lo[a]) * scale);
                b = std::min(std::max(b, 0), B - 1);
                bb[b].grow(r.box);
                bc[b]++;
            }
            Box acc;
            int32_t c = 0;
            for (int b = B - 1; b > 0; --b) acc.grow(bb[b]), c += bc[b], rb[b] = acc, rc[b] = c;
            acc = Box();
            c = 0;
            for (int b = 0; b < B - 1; ++b) {
                acc.grow(bb[b]);
                c += bc[b];
                if (c == 0 || rc[b + 1] == 0) continue;
                const double cost = acc.area() * c + rb[b + 1].area() * rc[b + 1];
                if (cost < best_cost) best_cost = cost, best_axis = a, best_split = b, best_l = acc, best_r = rb[b + 1];
            }
        }
        // spatial split: planes at B - 1 bin boundaries of the node's box per
        // axis; a reference enters the bins its box spans, with the box of its
        // part in each (clipped), and is counted entering its first bin and
        // leaving its last
        double sbest = INFINITY;
        int saxis = -1;
        double splane = 0.0;
        if (budget > 0 && best_axis >= 0 && overlap_area(best_l, best_r) > min_overlap) {
            for (int a = 0; a < 3; ++a) {
                const double lo = nb.lo[a], ext = (double)nb.hi[a] - lo;
                if (!(ext > 0.0)) continue;
                auto plane = [&](int k) { return k == B ? (double)nb.hi[a] : lo + ext * k / B; };
                for (int b = 0; b < B; ++b) bb[b] = Box(), bc[b] = 0, ec[b] = 0;
                for (const Ref &r : refs) {
                    int b0 = (int)(((double)r.box.lo[a] - lo) * B / ext), b1 = (int)(((double)r.box.hi[a] - lo) * B / ext);
                    b0 = std::min(std::max(b0, 0), B - 1);
                    b1 = std::min(std::max(b1, b0), B - 1);
                    bc[b0]++;
                    ec[b1]++;
                    if (b0 == b1) {
                        bb[b0].grow(r.box);
                        continue;
                    }
                    // the triangle's part in the reference's box, cut at each bin boundary in turn
                    double rlo[3], rhi[3];
                    for (int k = 0; k < 3; ++k) rlo[k] = r.box.lo[k], rhi[k] = r.box.hi[k];
                    Poly rest = tri_in_box(V, r.tri, rlo, rhi), part, next;
                    for (int b = b0; b <= b1 && rest.n; ++b) {
                        rlo[a] = std::max((double)r.box.lo[a], plane(b));
                        rhi[a] = std::min((double)r.box.hi[a], plane(b + 1));
                        if (b == b1) {
                            bb[b].grow(poly_box(rest, rlo, rhi));
                            break;
                        }
                        clip_plane(rest, a, rhi[a], true, part);
                        clip_plane(rest, a, rhi[a], false, next);
                        bb[b].grow(poly_box(part, rlo, rhi));
                        rest = next;
                    }
                }
                Box acc;
                int32_t c = 0;
                for (int b = B - 1; b > 0; --b) acc.grow(bb[b]), c += ec[b], rb[b] = acc, rc[b] = c;
                acc = Box();
                c = 0;
                for (int b = 0; b < B - 1; ++b) {
                    acc.grow(bb[b]);
                    c += bc[b];
                    if (c == 0 || rc[b + 1] == 0) continue;
                    const double cost = acc.area() * c + rb[b + 1].area() * rc[b + 1];
                    if (cost < sbest) sbest = cost, saxis = a, splane = plane(b + 1);
                }
            }
        }
        const double parea = nb.area();
        const double bc_min = std::min(best_cost, sbest);
        const double split_cost = bc_min < INFINITY ? trav_cost + (parea > 0 ? bc_min / parea : 0.0) : INFINITY;
        if (count <= max_leaf && (double)count <= split_cost) return make_leaf();

        std::vector<Ref> L, R;
        if (!(sbest < best_cost)) saxis = -1;
        if (saxis >= 0) {
            const int a = saxis;
            for (const Ref &r : refs) {
                if ((double)r.box.hi[a] <= splane) {
                    L.push_back(r);
                } else if ((double)r.box.lo[a] >= splane) {
                    R.push_back(r);
                } else {
                    double rlo[3], rhi[3];
                    for (int k = 0; k < 3; ++k) rlo[k] = r.box.lo[k], rhi[k] = r.box.hi[k];
                    rhi[a] = splane;
                    const Box bl = clip_tri(V, r.tri, rlo, rhi);
                    rhi[a] = r.box.hi[a];
                    rlo[a] = splane;
                    const Box br = clip_tri(V, r.tri, rlo, rhi);
                    if (bl.lo[0] <= bl.hi[0]) L.push_back({r.tri, bl});
                    if (br.lo[0] <= br.hi[0]) R.push_back({r.tri, br});
                }
            }
            // a spatial split must shrink both sides and stay within the budget, or the object split is taken
            if (L.empty() || R.empty() || (int32_t)L.size() == count || (int32_t)R.size() == count ||
                (int64_t)(L.size() + R.size()) - count > budget) {
                L.clear();
                R.clear();
                saxis = -1;
            }
        }
        if (saxis < 0) {
            if (best_axis < 0) {
                if (count <= max_leaf) return make_leaf();
                L.assign(refs.begin(), refs.begin() + count / 2);  // coincident centroids
                R.assign(refs.begin() + count / 2, refs.end());
            } else {
                const int a = best_axis;
                const double scale = (double)B / (double)(cb.hi[a] - cb.lo[a]);
                for (const Ref &r : refs) {
                    int b = (int)(((double)(0.5f * (r.box.lo[a] + r.box.hi[a])) - cb.lo[a]) * scale);
                    b = std::min(std::max(b, 0), B - 1);
                    (b <= best_split ? L : R).push_back(r);
                }
                if (L.empty() || R.empty()) {
                    L.assign(refs.begin(), refs.begin() + count / 2);
                    R.assign(refs.begin() + count / 2, refs.end());
                }
            }
        }
        // the budget left is shared by the children in proportion to their sizes
        const int64_t left_budget = budget - std::max<int64_t>(0, (int64_t)(L.size() + R.size()) - count);
        const int64_t bl = left_budget * (int64_t)L.size() / (int64_t)(L.size() + R.size()), br = left_budget - bl;
        std::vector<Ref>().swap(refs);
        int32_t l, r;
        if (depth < par_depth && count > 50000) {
            std::vector<TNode> right_nodes;
            std::vector<int32_t> right_leaf;
            auto fut =
                std::async(std::launch::async, [&]() { return build(R, depth + 1, br, right_nodes, right_leaf); });
            l = build(L, depth + 1, bl, out, leaf);
            fut.get();
            const int32_t off = (int32_t)out.size(), loff = (int32_t)leaf.size();
            for (auto &nd : right_nodes) {
                if (nd.left >= 0) {
                    nd.left += off;
                    nd.right += off;
                } else {
                    nd.start += loff;
                }
                out.push_back(nd);
            }
            leaf.insert(leaf.end(), right_leaf.begin(), right_leaf.end());
            r = off;
        } else {
            l = build(L, depth + 1, bl, out, leaf);
            r = build(R, depth + 1, br, out, leaf);
        }
        out[ni].left = l;
        out[ni].right = r;
        out[ni].start = out[ni].count = 0;
        return ni;
    }
};

// Spatial splits may add at most this many references per triangle in all.
constexpr int64_t kMaxExtraRefs = 7;

inline uint32_t fbits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}

}  // namespace

bool build_bvh_host(const float *verts, const uint32_t *mats, int64_t n_tri, const BuildOptions &opt, HostBvh &out,
                    std::string &err) {
    auto t0 = std::chrono::steady_clock::now();
    if (n_tri < 1 || n_tri >= (int64_t(1) << 28)) {
        err = "n_tri must be in [1, 2^28)";
        return false;
    }
    if (opt.bins < 2 || opt.bins > 256 || opt.max_leaf < 1 || opt.max_leaf > 7 || !(opt.trav_cost > 0.0) ||
        opt.trav_cost > 64.0) {
        err = "bins must be in [2,256], max_leaf in [1,7] and trav_cost in (0,64]";
        return false;
    }
    if (!(opt.split_alpha >= 0.0 && opt.split_alpha <= 1.0)) {
        err = "split_alpha must be in [0, 1]";
        return false;
    }
    for (int64_t i = 0; i < 9 * n_tri; ++i)
        if (!std::isfinite(verts[i])) {
            err = "non-finite vertex coordinate at triangle " + std::to_string(i / 9);
            return false;
        }
    unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    int nth = opt.n_threads > 0 ? opt.n_threads : (int)std::min(hw, 16u);
    int par_depth = 0;
    while ((1 << par_depth) < nth) par_depth++;
    Builder b;
    b.V = verts;
    b.n = n_tri;
    b.bins = opt.bins;
    b.max_leaf = opt.max_leaf;
    b.trav_cost = opt.trav_cost;
    b.par_depth = par_depth;
    b.tb.resize((size_t)n_tri);
    b.cen.resize(3 * (size_t)n_tri);
    b.idx.resize((size_t)n_tri);
    Box scene;
    for (int64_t i = 0; i < n_tri; ++i) {
        Box t;
        for (int k = 0; k < 3; ++k) t.grow(verts + 9 * i + 3 * k);
        b.tb[i] = t;
        scene.grow(t);
        for (int a = 0; a < 3; ++a) b.cen[3 * i + a] = 0.5f * (t.lo[a] + t.hi[a]);
        b.idx[i] = (int32_t)i;
    }
    std::vector<TNode> tree;
    tree.reserve((size_t)(2 * n_tri));
    // leaf order: the triangle of each record (with spatial splits a triangle
    // can appear more than once)
    std::vector<int32_t> &order = b.idx;
    if (opt.split_alpha > 0.0) {
        SplitBuilder sb;
        sb.V = verts;
        sb.bins = opt.bins;
        sb.max_leaf = opt.max_leaf;
        sb.trav_cost = opt.trav_cost;
        sb.min_overlap = opt.split_alpha * scene.area();
        sb.par_depth = par_depth;
        std::vector<Ref> refs((size_t)n_tri);
        for (int64_t i = 0; i < n_tri; ++i) refs[i] = Ref{(int32_t)i, b.tb[i]};
        order.clear();
        order.reserve((size_t)(n_tri + n_tri / 2));
        sb.build(refs, 0, kMaxExtraRefs * n_tri, tree, order);
        if ((int64_t)order.size() >= (int64_t(1) << 28)) {
            err = "spatial splits made 2^28 or more triangle records: raise split_alpha";
            return false;
        }
    } else {
        b.build(0, (int32_t)n_tri, 0, tree);
    }
    const int64_t nn = (int64_t)tree.size();
    const int64_t n_rec = (int64_t)order.size();

    // statistics: depth, leaves, SAH cost
    std::vector<int32_t> dep((size_t)nn, 0), size((size_t)nn, 1);
    double root_area = tree[0].box.area();
    double sah = 0.0;
    int64_t leaves = 0;
    int32_t maxdep = 0;
    for (int64_t i = 0; i < nn; ++i) {
        const TNode &t = tree[i];
        double rel = root_area > 0 ? t.box.area() / root_area : 1.0;
        if (t.left >= 0) {
            dep[t.left] = dep[i] + 1;
            dep[t.right] = dep[i] + 1;
            sah += rel * opt.trav_cost;
        } else {
            leaves++;
            sah += rel * t.count;
        }
        maxdep = std::max(maxdep, dep[i]);
    }
    for (int64_t i = nn - 1; i >= 0; --i)
        if (tree[i].left >= 0) size[i] = 1 + size[tree[i].left] + size[tree[i].right];

    // box padding: it covers the absolute parts of the error bounds that keep
    // the slab test conservative (2u ext for the plane distances, 22u L for
    // the point of an accepted triangle hit, L <= sqrt(3) ext; u = 2^-24)
    // more than ten times over; the relative parts are the slab test's slack
    float ext = 0.0f;
    for (int a = 0; a < 3; ++a) ext = std::max(ext, scene.hi[a] - scene.lo[a]);
    float mag = 0.0f;
    for (int a = 0; a < 3; ++a) mag = std::max(mag, std::max(std::fabs(scene.lo[a]), std::fabs(scene.hi[a])));
    const double pad = std::max((double)ext * 0x1p-15, (double)mag * 0x1p-20) + 1e-30;

    // 16-bit quantisation grid over the padded scene box: a node's box is
    // rounded outward to grid lines, so the stored box contains the padded one
    float qlo[3], qstep[3];
    for (int a = 0; a < 3; ++a) {
        double lo = (double)scene.lo[a] - pad, hi = (double)scene.hi[a] + pad;
        float l = (float)lo;
        if ((double)l > lo) l = std::nextafter(l, -INFINITY);
        double st = (hi - (double)l) / 65535.0;
        float sf = (float)st;
        while ((double)l + 65535.0 * (double)sf < hi) sf = std::nextafter(sf, INFINITY);
        qlo[a] = l;
        qstep[a] = sf;
    }
    auto q_down = [&](int a, double x) -> uint32_t {
        double q = std::floor((x - (double)qlo[a]) / (double)qstep[a]);
        q = std::min(std::max(q, 0.0), 65535.0);
        while (q > 0.0 && (double)qlo[a] + q * (double)qstep[a] > x) q -= 1.0;
        return (uint32_t)q;
    };
    auto q_up = [&](int a, double x) -> uint32_t {
        double q = std::ceil((x - (double)qlo[a]) / (double)qstep[a]);
        q = std::min(std::max(q, 0.0), 65535.0);
        while (q < 65535.0 && (double)qlo[a] + q * (double)qstep[a] < x) q += 1.0;
        return (uint32_t)q;
    };

    out.n_tri = n_tri;
    out.n_refs = n_rec;
    out.n_nodes = nn;
    out.n_leaves = leaves;
    out.depth = maxdep;
    out.max_leaf = opt.max_leaf;
    out.sah_cost = sah;
    for (int a = 0; a < 3; ++a) {
        out.lo[a] = scene.lo[a];
        out.hi[a] = scene.hi[a];
        out.qlo[a] = qlo[a];
        out.qstep[a] = qstep[a];
    }
    // quantised boxes once per node (shared by the six orders)
    std::vector<uint32_t> qbox((size_t)nn * 3);
    for (int64_t v = 0; v < nn; ++v) {
        const Box &bx = tree[v].box;
        uint32_t lo3[3], hi3[3];
        for (int a = 0; a < 3; ++a) {
            lo3[a] = q_down(a, (double)bx.lo[a] - pad);
            hi3[a] = q_up(a, (double)bx.hi[a] + pad);
        }
        for (int a = 0; a < 3; ++a) qbox[3 * v + a] = lo3[a] | (hi3[a] << 16);
    }
    out.nodes.assign((size_t)kLinkSets * nn * kNodeWords, 0u);
    auto thread_set = [&](int s) {
        const int axis = s >> 1;
        const bool neg = s & 1;
        std::vector<int32_t> stack;
        stack.reserve(256);
        stack.push_back(0);
        int64_t pre = 0;
        uint32_t *base = out.nodes.data() + (size_t)s * nn * kNodeWords;
        while (!stack.empty()) {
            int32_t v = stack.back();
            stack.pop_back();
            const TNode &t = tree[v];
            uint32_t *w = base + (size_t)pre * kNodeWords;
            w[0] = qbox[3 * (size_t)v];
            w[1] = qbox[3 * (size_t)v + 1];
            w[2] = qbox[3 * (size_t)v + 2];
            w[3] = t.left < 0 ? (0x80000000u | ((uint32_t)t.start << 3) | (uint32_t)t.count) : (uint32_t)(pre + size[v]);
            pre++;
            if (t.left >= 0) {
                const Box &L = tree[t.left].box, &R = tree[t.right].box;
                float kl = L.lo[axis] + L.hi[axis], kr = R.lo[axis] + R.hi[axis];
                bool right_first = neg ? (kr > kl) : (kr < kl);
                int32_t first = right_first ? t.right : t.left;
                int32_t second = right_first ? t.left : t.right;
                stack.push_back(second);
                stack.push_back(first);
            }
        }
    };
    std::vector<std::thread> th;
    for (int s = 0; s < kLinkSets; ++s) th.emplace_back(thread_set, s);
    for (auto &x : th) x.join();

    out.tris.assign((size_t)n_rec * kTriWords, 0u);
    for (int64_t k = 0; k < n_rec; ++k) {
        int32_t t = order[k];
        const float *v = verts + 9 * (size_t)t;
        uint32_t *w = out.tris.data() + (size_t)k * kTriWords;
        for (int a = 0; a < 3; ++a) {
            w[a] = fbits(v[a]);
            w[3 + a] = fbits(v[3 + a]);
            w[6 + a] = fbits(v[6 + a]);
        }
        w[9] = (uint32_t)t;
        w[10] = mats ? mats[t] : 0u;
        w[11] = 0u;
    }
    out.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return true;
}

}  // namespace pm
