// Host-side view of the LST-built graph and its components (lst_graph.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lst_host.h"

namespace lst {

struct GraphArgs {
    const float *x, *y, *z;
    const int32_t *sensor;
    const int2 *md_hits, *ls_md;
    const ModConst *mod;
    int64_t n_md, n_ls;
    float *feat;                 // [n_md][7]
    int32_t *src, *dst;          // [n_ls]
};

struct ComponentsArgs {
    const int32_t *src, *dst;
    const float *scores;
    int64_t n_nodes, n_edges;
    float threshold;
    int32_t min_mds;
    int32_t *par;                // [n_nodes] workspace
    int32_t *size;               // [n_nodes] workspace
    int32_t *labels;             // [n_nodes]
    int64_t *n_tc;               // [1]
    int64_t *err;                // [1] workspace: bit 0 an id out of range
};

hipError_t run_md_graph(const GraphArgs &a, hipStream_t stream);
// Workspace of the components (parents, sizes, error word) and its carving.
size_t components_workspace(int64_t n_nodes);
ComponentsArgs components_layout(char *ws, int64_t n_nodes);
hipError_t run_components(const ComponentsArgs &a, hipStream_t stream);

}  // namespace lst
