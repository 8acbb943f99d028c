// Patch plan: element order, per-patch distinct nodes and LDS slots, and the
// shared-node gather lists (see patch.cpp).
#pragma once
#include <stdint.h>

#include <vector>

namespace fepa {

struct PatchRec {
    int elem_begin;  // first element (patch order) of the patch
    int count;       // elements in the patch
    int pn_off;      // offset of its distinct-node list
    int U;           // distinct nodes
    int P;           // of which private (listed first)
    int sh_off;      // offset of its shared-node partials
};

struct PatchPlan {
    std::vector<int32_t> perm;     // patch-order element -> caller element
    std::vector<int32_t> map_int;  // [E][D^3] node ids in patch order
    std::vector<uint16_t> slot;    // [E][D^3] LDS slot of each element node
    std::vector<int32_t> pn;       // distinct nodes of every patch
    std::vector<PatchRec> patch;
    std::vector<int32_t> sh_node, sh_ptr, sh_idx;  // shared-node gather (CSR)
    std::vector<int32_t> orphans;  // nodes no element references (outputs set to 0)
    int n_entries = 0;             // shared partial entries
    int umax_used = 0;
};

// map: [E][(p+1)^3] node ids in [0, N); x0: host [3][N].
PatchPlan build_patch_plan(int E, int p, int N, const int32_t *map, const double *x0, int B,
                           int umax);

// Appends the plan of another mesh of the same order behind dst: its elements
// follow dst's, its element ids (perm) are shifted by perm_base, and its patch
// rows and shared-node lists are re-based onto dst's arrays. Node ids must
// already be global (meshes own disjoint node ranges), so no patch spans two
// meshes and the kernels treat the result as one mesh.
void append_plan(PatchPlan &dst, const PatchPlan &src, int32_t perm_base);

}  // namespace fepa
