// Host construction of the multiple-threaded BVH (Sec. 3.1).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace pm {

struct BuildOptions {
    int bins = 32;
    int max_leaf = 4;
    int n_threads = 0;
};

// Device layout (words are 32-bit):
//   nodes: 6 link sets x n_nodes x 8 words.  Set s lists the nodes in the
//          preorder whose children are visited along direction s
//          (0:+x 1:-x 2:+y 3:-y 4:+z 5:-z).  Node = lo.xyz, hi.xyz (padded
//          AABB), skip (preorder index after the subtree = the "miss" link;
//          n_nodes terminates), leaf word (0 inner; first_tri << 3 | count).
//          The "hit" link of an inner node is the next node (i + 1); a leaf's
//          hit link equals its miss link.
//   tris:  n_tri x 12 words in leaf order: v0.xyz, e1 = v1-v0, e2 = v2-v0,
//          original triangle index, material id, 0.
struct HostBvh {
    int64_t n_tri = 0, n_nodes = 0, n_leaves = 0;
    int32_t depth = 0, max_leaf = 0;
    double sah_cost = 0.0, build_ms = 0.0;
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};  // scene bounds (unpadded)
    std::vector<uint32_t> nodes;
    std::vector<uint32_t> tris;
};

constexpr int kNodeWords = 8;
constexpr int kTriWords = 12;
constexpr int kLinkSets = 6;

bool build_bvh_host(const float *verts, const uint32_t *mats, int64_t n_tri, const BuildOptions &opt, HostBvh &out,
                    std::string &err);

}  // namespace pm
