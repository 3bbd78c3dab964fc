// The LST-built graph of Sec. 4 and its track candidates: MDs as nodes, LSs
// as edges, and connected components of the edges the classifier keeps.
//
// Node features (seven per MD, all local to the MD, FP32): r_A / 100,
// phi_A / pi, z_A / 100, 10 alpha (alpha = angle from the radial direction at
// the chord midpoint to the chord, in the transverse plane: the MD's bend),
// eta_MD = asinh(dz / dr) of the chord clipped to [-5, 5], is_endcap,
// layer / 11. Edges: LS (inner a, outer b) becomes b -> a, so the edges
// entering a node are the segments that start at it, already contiguous and
// in order in the build's LS list (the layout the edge classifier needs).
//
// Components: one union-find pass over the kept edges (score >= threshold)
// that always hooks the larger root under the smaller with a compare-and-swap,
// so every root is the smallest node of its tree and the final labels (each
// node's root after a path-compressing find) are the smallest node index of
// each component whatever the order the edges are processed in.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lst_graph.h"

namespace lst {
namespace {

constexpr int kGBlock = 256;
constexpr int kGMaxGrid = 8192;

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

inline int grid_of(int64_t n) {
    int64_t g = (n + kGBlock - 1) / kGBlock;
    return (int)(g < 1 ? 1 : (g > kGMaxGrid ? kGMaxGrid : g));
}

__global__ void k_md_graph(GraphArgs a) {
    for (int64_t i = gtid(); i < a.n_md; i += gstride()) {
        const int2 h = a.md_hits[i];
        const float xa = a.x[h.x], ya = a.y[h.x], za = a.z[h.x];
        const float xo = a.x[h.y], yo = a.y[h.y], zo = a.z[h.y];
        const float ra = sqrtf(xa * xa + ya * ya), ro = sqrtf(xo * xo + yo * yo);
        const float mx = 0.5f * (xa + xo), my = 0.5f * (ya + yo);
        const float dx = xo - xa, dy = yo - ya;
        const float alpha = atan2f(mx * dy - my * dx, mx * dx + my * dy);
        // r_O - r_A without the cancellation of two rounded radii (the
        // coordinate differences of the two hits are exact in FP32)
        const float dr = (dx * (xo + xa) + dy * (yo + ya)) / (ro + ra), dz = zo - za;
        float eta;
        if (dr == 0.0f) eta = dz == 0.0f ? 0.0f : copysignf(5.0f, dz);
        else eta = fminf(5.0f, fmaxf(-5.0f, asinhf(dz / dr)));
        const int32_t m = a.sensor[h.x] >> 1;
        const ModConst mc = a.mod[m];
        float *f = a.feat + 7 * i;
        f[0] = ra / 100.0f;
        f[1] = atan2f(ya, xa) / 3.14159265f;
        f[2] = za / 100.0f;
        f[3] = 10.0f * alpha;
        f[4] = eta;
        f[5] = mc.kind != 0 ? 1.0f : 0.0f;
        f[6] = (float)mc.layer / 11.0f;
    }
    for (int64_t e = gtid(); e < a.n_ls; e += gstride()) {
        const int2 l = a.ls_md[e];
        a.src[e] = l.y;
        a.dst[e] = l.x;
    }
}

// Parent pointers are read and written at device scope (past the per-CU
// caches): every pointer goes to a smaller node, so any value read is an
// ancestor and every walk ends.
__device__ __forceinline__ int32_t ld_par(int32_t *par, int32_t v) {
    return __hip_atomic_load(&par[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t find_root(int32_t *par, int32_t v) {
    int32_t p = ld_par(par, v);
    while (p != v) {
        const int32_t g = ld_par(par, p);
        if (g != p) __hip_atomic_store(&par[v], g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);   // path halving
        v = p;
        p = ld_par(par, v);
    }
    return v;
}

__global__ void k_cc_init(int32_t *par, int64_t n) {
    for (int64_t v = gtid(); v < n; v += gstride()) par[v] = (int32_t)v;
}

__global__ void k_cc_union(ComponentsArgs a) {
    for (int64_t e = gtid(); e < a.n_edges; e += gstride()) {
        if (!(a.scores[e] >= a.threshold)) continue;
        const int32_t s = a.src[e], d = a.dst[e];
        if ((uint64_t)(uint32_t)s >= (uint64_t)a.n_nodes || (uint64_t)(uint32_t)d >= (uint64_t)a.n_nodes) {
            atomicOr((unsigned long long *)a.err, 1ull);     // an id out of range: reported, edge skipped
            continue;
        }
        int32_t u = find_root(a.par, s), v = find_root(a.par, d);
        while (u != v) {
            if (u < v) { const int32_t t = u; u = v; v = t; }     // u > v: hook u under v
            const int32_t old = atomicCAS(&a.par[u], u, v);
            if (old == u) break;
            u = find_root(a.par, old);
            v = find_root(a.par, v);
        }
    }
}

__global__ void k_cc_label(ComponentsArgs a) {
    for (int64_t v = gtid(); v < a.n_nodes; v += gstride()) {
        const int32_t r = find_root(a.par, (int32_t)v);
        a.labels[v] = r;
        atomicAdd(&a.size[r], 1);
    }
}

__global__ void k_cc_zero(ComponentsArgs a) {
    for (int64_t v = gtid(); v < a.n_nodes; v += gstride()) a.size[v] = 0;
    if (gtid() == 0) {
        *a.n_tc = 0;
        *a.err = 0;
    }
}

__global__ void k_cc_count(ComponentsArgs a) {
    __shared__ unsigned long long blk;
    if (threadIdx.x == 0) blk = 0;
    __syncthreads();
    unsigned long long c = 0;
    for (int64_t v = gtid(); v < a.n_nodes; v += gstride())
        if (a.labels[v] == v && a.size[v] >= a.min_mds) ++c;
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(&blk, c);
    __syncthreads();
    if (threadIdx.x == 0 && blk) atomicAdd((unsigned long long *)a.n_tc, blk);
}

}  // namespace

hipError_t run_md_graph(const GraphArgs &a, hipStream_t st) {
    const int64_t n = a.n_md > a.n_ls ? a.n_md : a.n_ls;
    hipLaunchKernelGGL(k_md_graph, dim3(grid_of(n)), dim3(kGBlock), 0, st, a);
    return hipGetLastError();
}

size_t components_workspace(int64_t n_nodes) {
    return (size_t)(4 * (n_nodes + 1) + 255) / 256 * 256 * 2 + 256;
}

ComponentsArgs components_layout(char *ws, int64_t n_nodes) {
    ComponentsArgs a{};
    const size_t s = (size_t)(4 * (n_nodes + 1) + 255) / 256 * 256;
    a.par = (int32_t *)ws;
    a.size = (int32_t *)(ws + s);
    a.err = (int64_t *)(ws + 2 * s);
    return a;
}

hipError_t run_components(const ComponentsArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(k_cc_init, dim3(grid_of(a.n_nodes)), dim3(kGBlock), 0, st, a.par, a.n_nodes);
    hipLaunchKernelGGL(k_cc_zero, dim3(grid_of(a.n_nodes)), dim3(kGBlock), 0, st, a);
    hipLaunchKernelGGL(k_cc_union, dim3(grid_of(a.n_edges)), dim3(kGBlock), 0, st, a);
    hipLaunchKernelGGL(k_cc_label, dim3(grid_of(a.n_nodes)), dim3(kGBlock), 0, st, a);
    hipLaunchKernelGGL(k_cc_count, dim3(grid_of(a.n_nodes)), dim3(kGBlock), 0, st, a);
    return hipGetLastError();
}

}  // namespace lst
