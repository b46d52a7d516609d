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
    double trav_cost = 1.0;  // SAH: node visit cost relative to a triangle test
    int builder = 0;         // PM_BUILD_HOST_SAH or PM_BUILD_GPU_LBVH
    double split_alpha = 0;  // spatial splits where children overlap by more than this x scene area; 0 = none
};

// Device layout (words are 32-bit):
//   nodes: 6 link sets x n_nodes x 4 words.  Set s lists the nodes in the
//          preorder whose children are visited along direction s
//          (0:+x 1:-x 2:+y 3:-y 4:+z 5:-z).  Node = padded AABB quantised
//          outward to a 16-bit grid over the scene (lo.x|lo.y<<16,
//          lo.z|hi.x<<16, hi.y|hi.z<<16; coordinate = qlo + q * qstep) and a
//          link word: inner node -> skip (preorder index after its subtree,
//          the "miss" link; n_nodes terminates); leaf -> bit 31 set,
//          first_tri << 3 | count.  The "hit" link of an inner node is the
//          next node (i + 1); a leaf occupies one slot, so both of its links
//          are i + 1.
//   tris:  n_refs x 12 words in leaf order: v0.xyz, v1.xyz, v2.xyz (float32,
//          as given), original triangle index, material id, 0.  n_refs =
//          n_tri unless spatial splits put a triangle in several leaves.
struct HostBvh {
    int64_t n_tri = 0, n_refs = 0, n_nodes = 0, n_leaves = 0;
    int32_t depth = 0, max_leaf = 0;
    double sah_cost = 0.0, build_ms = 0.0;
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};  // scene bounds (unpadded)
    float qlo[3] = {0, 0, 0}, qstep[3] = {1, 1, 1};  // node quantisation grid
    std::vector<uint32_t> nodes;
    std::vector<uint32_t> tris;
};

constexpr int kNodeWords = 4;
constexpr int kTriWords = 12;
constexpr int kLinkSets = 6;

bool build_bvh_host(const float *verts, const uint32_t *mats, int64_t n_tri, const BuildOptions &opt, HostBvh &out,
                    std::string &err);

}  // namespace pm
