// Level-restricted adaptive octree over Morton-sorted points, with the
// neighbour structures the DMK passes need (Sec. "The DMK method", Step 1).
#pragma once

#include <cstdint>
#include <vector>

namespace dmk {

constexpr int kMaxLevel = 19;   // Morton keys carry 3 * 19 bits below the root
constexpr int kKeyBits = 19;

struct Box {
    int level;
    int64_t ix, iy, iz;   // integer coordinates at its level, in [0, 2^level)
    int parent;
    int child[8];         // child index 4*bx + 2*by + bz, -1 if absent
    int64_t start, end;   // range in the sorted point order
    bool leaf;
};

// One near-field interaction: all points of leaf `src` act on the target leaf
// through the residual kernel at level `lambda`, source images shifted by
// `shift` unit cells (periodic only).
struct NearEntry {
    int src;
    int8_t sx, sy, sz;
    int8_t lambda;
};

// One far-field difference-kernel interaction at the receiver's level: the
// colleague `src` sits at offset (ox,oy,oz) box lengths from the receiver.
struct FarEntry {
    int src;
    int8_t ox, oy, oz;
};

struct Tree {
    bool periodic = false;
    int64_t n = 0;
    int max_level = 0;
    std::vector<Box> boxes;                    // ordered by level, Morton order within a level
    std::vector<int> level_start;              // boxes of level l: [level_start[l], level_start[l+1])
    std::vector<std::vector<FarEntry>> colleagues;  // per box, incl. itself (offset 0)
    // near lists, per non-empty leaf
    std::vector<int> leaves;                   // non-empty leaves
    std::vector<std::vector<NearEntry>> near;  // parallel to `leaves`
    // difference-kernel exchange lists (leaf/non-leaf rule), per non-empty box
    std::vector<std::vector<FarEntry>> incoming;
    // statistics
    int64_t n_near_pairs = 0;                  // sum over near entries of |T| * |S|
};

// Builds the tree from Morton keys sorted ascending (keys use 3 bits per
// level, level-1 digit most significant, digit = 4 bx + 2 by + bz).
// Splits a box while it holds more than `ns` points (up to kMaxLevel), then
// refines until adjacent leaves (sharing a boundary point, through the
// periodic wrap when `periodic`) differ by at most one level.
void build_tree(const uint64_t* sorted_keys, int64_t n, int ns, bool periodic, Tree* T);

// Joins the trees of independent problems into one forest.  Problem t's
// points occupy [offsets[t], offsets[t+1]) of the sorted order.  Boxes are
// ordered by level (problem order within a level); every index is remapped;
// lists never cross problems.  roots[t] receives the index of problem t's root.
void merge_forest(std::vector<Tree>& parts, const std::vector<int64_t>& offsets, Tree* out, std::vector<int>* roots);

}  // namespace dmk
