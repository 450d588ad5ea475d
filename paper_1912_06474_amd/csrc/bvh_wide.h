// Widening of the per-cell binary BVHs into 4-wide nodes (bvh_wide.hip).
//
// Both builders (host binned SAH, device radix tree) emit binary nodes, two
// 16 B child records each, stored breadth-first per cell.  The traversal
// kernel reads 4-wide nodes: every binary node at even depth becomes one
// 4-wide node whose records are those of its grandchildren (for an inner
// child) or the child itself (a leaf), copied unchanged, since all records of
// a cell share the cell's lattice.  Unused slots are empty records.  The
// even-depth nodes keep their breadth-first order, which is the 4-wide tree's
// breadth-first order, so a cell's first nodes are still its top levels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace sdd {

struct WidenBufs {
    int n2;             // binary node slots (slots outside every cell's range are ignored)
    const uint4* nodes2;
    const int* cell_root;   // [G] binary root slot of each cell
    const int* cell_nodes;  // [G] binary nodes of each cell, slots [root, root + nodes)
    int G;
    int max_cell_nodes;     // largest cell_nodes (grid of the marking kernel)
    int* anc[2];            // [n2] ancestor pointers (pointer jumping)
    int* dist[2];           // [n2] distance to that ancestor; -1 for slots of no cell
    int* flag;              // [n2 + 1] 1 for a binary node at even depth
    int* idx;               // [n2 + 1] exclusive prefix of flag: 4-wide index; idx[n2] = total
    void* tmp;              // scan scratch
    size_t tmp_bytes;
};

// With tmp == nullptr only sets tmp_bytes.  Otherwise computes every node's
// depth and the 4-wide index of the even-depth ones (idx[n2] = their count).
hipError_t widen_mark(WidenBufs& b, hipStream_t st);
// The 4-wide nodes ([4 * total] records) and each cell's root and node count.
hipError_t widen_emit(const WidenBufs& b, uint4* nodes4, int* cell_root4, int* cell_nodes4, hipStream_t st);

}  // namespace sdd
