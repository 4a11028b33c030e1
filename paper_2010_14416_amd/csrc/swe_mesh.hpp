// Host-side mesh preparation for the shallow-water step: validation,
// counter-clockwise orientation, unique edges with their unit normals,
// cell geometry (area, inscribed radius), a space-filling-curve cell order,
// and the per-block edge lists the fused step kernel consumes.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace swe {

constexpr uint32_t kSideLocal = 0x80000000u;
constexpr uint32_t kSideBoundary = 0x40000000u;

// Device-facing mesh in the internal (locality) cell order.
struct BlockMesh {
    int64_t n_nodes = 0, n_cells = 0, n_edges = 0, n_bnd_edges = 0;
    int32_t block_cells = 256;
    int32_t n_blocks = 0;
    int32_t max_block_edges = 0;
    double min_inradius = 0.0, total_area = 0.0;

    // cell order: internal_of_user[u] = i, user_of_internal[i] = u
    std::vector<int32_t> internal_of_user, user_of_internal;

    // per internal cell
    std::vector<double> area, inradius;

    // per block: [blk_cell[b], blk_cell[b+1]) cells,
    //            [blk_edge[b], blk_edge[b+1]) block-edge records
    std::vector<int32_t> blk_cell, blk_edge;

    // per block-edge record: the edge's left side (be_a) and right side
    // (be_b), each coded as
    //   kSideLocal | k << 12 | c : cell c of the block (local index), whose
    //                              local side k is this edge
    //   i (>= 0, < 2^30)         : internal index of a cell of another block
    //   kSideBoundary | s        : boundary slot s (right side only)
    // and the unit normal from left to right (outward on the boundary).
    std::vector<int32_t> be_a, be_b;
    std::vector<double> be_nx, be_ny, be_len;

    // tag of each boundary slot; slots are numbered in block order. Block b
    // holds the blk_bnd[4b+2] slots from blk_bnd[4b] on, whose records are
    // consecutive from record blk_bnd[4b+1] on (after the edges to other
    // blocks); blk_bnd[4b+3] = 0 pads the entry to 16 bytes.
    std::vector<int32_t> bnd_tag;
    std::vector<int32_t> blk_bnd;

    // total boundary length per tag (inflow discharge per unit length)
    std::vector<double> tag_length;
};

// Edges given by the caller instead of discovered from the triangles:
// n edges, nodes[2e], nodes[2e+1] (either order), cells[2e], cells[2e+1]
// (the one or two triangles on the edge, in either slot; -1 in the other
// slot on the boundary), tag[e] (boundary edges, in [0, max_tag); 0 on
// interior edges; tag null = all 0).
struct EdgeInput {
    int64_t n = 0;
    const int32_t *nodes = nullptr;
    const int32_t *cells = nullptr;
    const int32_t *tag = nullptr;
};

// Builds the block mesh. Returns false and sets err on an invalid mesh.
// With edges non-null, the edge table and the boundary tags are taken from
// it (validated against the triangles) and the segments are not used.
// With reorder, cells follow a Hilbert curve through their centroids; with
// group (one value per cell, or null) too, cells are ordered by group first
// and along the curve within a group. With wet_band >= 0, group is instead
// a wet mask and the groups are: wet cells, dry cells at most wet_band
// edge-steps from a wet cell, the other dry cells.
bool build_block_mesh(int64_t n_nodes, const double *xy, int64_t n_cells,
                      const int32_t *tri, int64_t n_bnd,
                      const int32_t *bnd_nodes, const int32_t *bnd_tag,
                      int32_t block_cells, bool reorder,
                      const uint8_t *group, int32_t wet_band,
                      int32_t max_tag, BlockMesh &out, std::string &err,
                      const EdgeInput *edges = nullptr);

}  // namespace swe
