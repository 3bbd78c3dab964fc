// Edge classifier on an LST object graph (the GNN the paper proposes in
// Sec. 4; its architecture is not given there, so this is an interaction
// network): node encoder 7 -> 64 -> 64, edge init 128 -> 64, two
// message-passing steps (edge update 192 -> 64 -> 64 with a residual, sum of
// incoming edge states, node update 128 -> 64 -> 64 with a residual), edge
// head 64 -> 32 -> 1 with a sigmoid.
//
// Dense layers run on the matrix cores (v_mfma_f32_16x16x32_bf16, BF16
// operands rounded to nearest even, FP32 accumulation); node and edge states
// are kept in FP32. A wavefront takes 32 rows (two 16-row blocks) per step
// and computes transposed products D^T = W . X^T, so one lane holds, for
// row l % 16, the output units 16 mb + 4 g + j (g = lane / 16, j = 0..3).
// Every 64-wide input is consumed in the matching K order: K chunk ks, slot
// i of lane group g is unit 32 ks + 16 (i / 4) + 4 g + (i % 4). With that
// order (a permutation of a summed index, so exact) a layer's accumulators
// are the next layer's B operand, and an FP32 row loaded as four float4 per
// lane is at once the B operand and the residual in accumulator layout: no
// LDS traffic between layers. Weights are pre-arranged on the host in
// A-operand fragment order (one 16-byte fragment per lane per (m block, K
// chunk)) and staged in LDS once per block.
//
// Five kernels: encode; edge init fused with the step-0 edge update;
// incoming sums over the dst-sorted edge list (no atomics, edge order);
// step-0 node update; step-1 edge update fused with the head. The step-1 node update is not
// computed: no output depends on it.
#include <hip/hip_runtime.h>

#include "lst_internal.h"

namespace lst {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kGnnThreads = 256;
constexpr int kGnnWaves = kGnnThreads / 64;
constexpr int kNB = 2;                         // 16-row blocks per wave step
constexpr int kRowsPerWave = 16 * kNB;
constexpr int kGnnMaxBlocks = 1024;

__device__ __forceinline__ int64_t g_tid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t g_stride() { return (int64_t)gridDim.x * blockDim.x; }

// copy n 16-byte fragments and nb floats of bias into LDS
__device__ __forceinline__ void stage(uint4 *Lf, const uint4 *frag, int n, float *Lb, const float *bias, int nb) {
    for (int i = threadIdx.x; i < n; i += kGnnThreads) Lf[i] = frag[i];
    for (int i = threadIdx.x; i < nb; i += kGnnThreads) Lb[i] = bias[i];
}

// D[mb][nb] = sum over K chunks of A(mb, ks) . B[ks][nb]
template <int MB, int KS>
__device__ __forceinline__ void layer(const uint4 *Lf, const bf16x8 (*B)[kNB], f32x4 (&D)[MB][kNB]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) D[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const bf16x8 a = __builtin_bit_cast(bf16x8, Lf[(mb * KS + ks) * 64 + lane]);
#pragma unroll
            for (int nb = 0; nb < kNB; ++nb)
                D[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, B[ks][nb], D[mb][nb], 0, 0, 0);
        }
        // keep one K chunk of weight fragments live at a time (otherwise the
        // scheduler hoists every fragment of the layer and occupancy drops to
        // one wave per SIMD)
        __builtin_amdgcn_sched_barrier(0);
    }
}

// FP32 values in accumulator layout (units 16 q + 4 g + j) -> two B chunks
__device__ __forceinline__ void r_to_b(const float (&R)[4][4], bf16x8 *B2 /* [2] (stride kNB) */, int nb) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int i = 0; i < 8; ++i) B2[ks * kNB + nb][i] = (__bf16)R[2 * ks + (i >> 2)][i & 3];
}

// R = D + bias (optionally relu), accumulator layout
template <bool kRelu>
__device__ __forceinline__ void bias_act(const f32x4 (&D)[4][kNB], const float *Lb, int g, int nb, float (&R)[4][4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 b = *reinterpret_cast<const float4 *>(Lb + 16 * q + 4 * g);
        const float bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float v = D[q][nb][j] + bv[j];
            R[q][j] = kRelu ? fmaxf(v, 0.0f) : v;
        }
    }
}

__device__ __forceinline__ void load_row(const float *row, int g, bool ok, float (&R)[4][4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 v = ok ? *reinterpret_cast<const float4 *>(row + 16 * q + 4 * g) : make_float4(0.f, 0.f, 0.f, 0.f);
        R[q][0] = v.x; R[q][1] = v.y; R[q][2] = v.z; R[q][3] = v.w;
    }
}

__device__ __forceinline__ void store_row(float *row, int g, const float (&R)[4][4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
        *reinterpret_cast<float4 *>(row + 16 * q + 4 * g) = make_float4(R[q][0], R[q][1], R[q][2], R[q][3]);
}

__device__ __forceinline__ int64_t clamp_id(int32_t v, int64_t n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

// ------------------------------------------------------------ checks

__global__ void k_gnn_check(const int32_t *src, const int32_t *dst, int64_t n_nodes, int64_t n_edges,
                            int64_t *err) {
    bool bad = false;
    for (int64_t i = g_tid(); i < n_edges; i += g_stride()) {
        const int32_t s = src[i], d = dst[i];
        if (s < 0 || s >= n_nodes || d < 0 || d >= n_nodes) bad = true;
        if (i > 0 && dst[i - 1] > d) bad = true;
    }
    if (bad) atomicOr((unsigned long long *)err, 1ull);
}

// off[v] = first edge with dst >= v, v = 0..n_nodes (dst sorted ascending)
__global__ void k_gnn_offsets(const int32_t *dst, int64_t n_nodes, int64_t n_edges, int64_t *off) {
    for (int64_t v = g_tid(); v <= n_nodes; v += g_stride()) {
        int64_t lo = 0, hi = n_edges;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)dst[mid] < v) lo = mid + 1; else hi = mid;
        }
        off[v] = lo;
    }
}

__global__ void k_gnn_zero(int64_t *p) { if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0; }

// ------------------------------------------------------------ encoder

__global__ __launch_bounds__(kGnnThreads) void k_gnn_encode(GnnDev m, const float *x, int64_t n, float *h0) {
    __shared__ uint4 Lf1[4 * 1 * 64], Lf2[4 * 2 * 64];
    __shared__ float Lb1[64], Lb2[64];
    stage(Lf1, m.frag + m.foff[kGEnc1], 4 * 1 * 64, Lb1, m.bias + m.boff[kGEnc1], 64);
    stage(Lf2, m.frag + m.foff[kGEnc2], 4 * 2 * 64, Lb2, m.bias + m.boff[kGEnc2], 64);
    __syncthreads();
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    const int64_t wave = g_tid() >> 6, nwave = g_stride() >> 6;
    for (int64_t base = wave * kRowsPerWave; base < n; base += nwave * kRowsPerWave) {
        bf16x8 B1[1][kNB];
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            const int64_t row = base + nb * 16 + c;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int k = 8 * g + i;
                B1[0][nb][i] = (__bf16)((row < n && k < 7) ? x[row * 7 + k] : 0.0f);
            }
        }
        f32x4 D[4][kNB];
        layer<4, 1>(Lf1, B1, D);
        bf16x8 B2[2][kNB];
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            float R[4][4];
            bias_act<true>(D, Lb1, g, nb, R);
            r_to_b(R, &B2[0][0], nb);
        }
        layer<4, 2>(Lf2, B2, D);
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            const int64_t row = base + nb * 16 + c;
            float R[4][4];
            bias_act<true>(D, Lb2, g, nb, R);
            if (row < n) store_row(h0 + row * 64, g, R);
        }
    }
}

// ------------------------------------------ edge init + step-0 edge update

__global__ __launch_bounds__(kGnnThreads) void k_gnn_edge_first(GnnDev m, const float *h0, const int32_t *src,
                                                                const int32_t *dst, int64_t n_nodes,
                                                                int64_t n_edges, float *e1) {
    __shared__ uint4 Lfi[4 * 4 * 64], Lfa[4 * 6 * 64], Lfb[4 * 2 * 64];
    __shared__ float Lbi[64], Lba[64], Lbb[64];
    stage(Lfi, m.frag + m.foff[kGInit], 4 * 4 * 64, Lbi, m.bias + m.boff[kGInit], 64);
    stage(Lfa, m.frag + m.foff[kGEdgeA0], 4 * 6 * 64, Lba, m.bias + m.boff[kGEdgeA0], 64);
    stage(Lfb, m.frag + m.foff[kGEdgeB0], 4 * 2 * 64, Lbb, m.bias + m.boff[kGEdgeB0], 64);
    __syncthreads();
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    const int64_t wave = g_tid() >> 6, nwave = g_stride() >> 6;
    for (int64_t base = wave * kRowsPerWave; base < n_edges; base += nwave * kRowsPerWave) {
        bf16x8 Bin[6][kNB];
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            const int64_t row = base + nb * 16 + c;
            const bool ok = row < n_edges;
            const int64_t s = ok ? clamp_id(src[row], n_nodes) : 0, d = ok ? clamp_id(dst[row], n_nodes) : 0;
            float Rs[4][4], Rd[4][4];
            load_row(h0 + s * 64, g, ok, Rs);
            load_row(h0 + d * 64, g, ok, Rd);
            r_to_b(Rs, &Bin[0][0], nb);
            r_to_b(Rd, &Bin[2][0], nb);
        }
        f32x4 D[4][kNB];
        layer<4, 4>(Lfi, Bin, D);
        float Re[kNB][4][4];
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            bias_act<true>(D, Lbi, g, nb, Re[nb]);
            r_to_b(Re[nb], &Bin[4][0], nb);
        }
        layer<4, 6>(Lfa, Bin, D);
        bf16x8 Bh[2][kNB];
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            float R[4][4];
            bias_act<true>(D, Lba, g, nb, R);
            r_to_b(R, &Bh[0][0], nb);
        }
        layer<4, 2>(Lfb, Bh, D);
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            const int64_t row = base + nb * 16 + c;
            float R[4][4];
            bias_act<false>(D, Lbb, g, nb, R);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int j = 0; j < 4; ++j) R[q][j] += Re[nb][q][j];
            if (row < n_edges) store_row(e1 + row * 64, g, R);
        }
    }
}

// ------------------------------------------------- step-0 node update

// m[v] = sum of the states of the edges entering v, in edge order (dst-sorted
// list); one thread per (node, 4-unit slice), so the per-node loops of many
// nodes are in flight at once
__global__ __launch_bounds__(256) void k_gnn_msum(const float *e, const int64_t *in_off, int64_t n_nodes, float *m) {
    const int64_t n = n_nodes * 16;
    for (int64_t t = g_tid(); t < n; t += g_stride()) {
        const int64_t v = t >> 4;
        const int q = (int)(t & 15);
        const int64_t j0 = in_off[v], j1 = in_off[v + 1];
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        int64_t j = j0;
        // four rows in flight, summed in edge order
        for (; j + 4 <= j1; j += 4) {
            float4 x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) x[u] = reinterpret_cast<const float4 *>(e + (j + u) * 64)[q];
#pragma unroll
            for (int u = 0; u < 4; ++u) { acc.x += x[u].x; acc.y += x[u].y; acc.z += x[u].z; acc.w += x[u].w; }
        }
        for (; j < j1; ++j) {
            const float4 x = reinterpret_cast<const float4 *>(e + j * 64)[q];
            acc.x += x.x; acc.y += x.y; acc.z += x.z; acc.w += x.w;
        }
        reinterpret_cast<float4 *>(m + v * 64)[q] = acc;
    }
}

__global__ __launch_bounds__(kGnnThreads) void k_gnn_node(GnnDev m, int lay_a, int lay_b, const float *h,
                                                          const float *msg, int64_t n_nodes, float *h_out) {
    __shared__ uint4 Lfa[4 * 4 * 64], Lfb[4 * 2 * 64];
    __shared__ float Lba[64], Lbb[64];
    stage(Lfa, m.frag + m.foff[lay_a], 4 * 4 * 64, Lba, m.bias + m.boff[lay_a], 64);
    stage(Lfb, m.frag + m.foff[lay_b], 4 * 2 * 64, Lbb, m.bias + m.boff[lay_b], 64);
    __syncthreads();
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    const int64_t wave = g_tid() >> 6, nwave = g_stride() >> 6;
    for (int64_t base = wave * kRowsPerWave; base < n_nodes; base += nwave * kRowsPerWave) {
        bf16x8 Bin[4][kNB];
        float Rh[kNB][4][4];
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            const int64_t v = base + nb * 16 + c;
            const bool ok = v < n_nodes;
            load_row(h + v * 64, g, ok, Rh[nb]);
            float M[4][4];
            load_row(msg + v * 64, g, ok, M);
            r_to_b(Rh[nb], &Bin[0][0], nb);
            r_to_b(M, &Bin[2][0], nb);
        }
        f32x4 D[4][kNB];
        layer<4, 4>(Lfa, Bin, D);
        bf16x8 Bh[2][kNB];
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            float R[4][4];
            bias_act<true>(D, Lba, g, nb, R);
            r_to_b(R, &Bh[0][0], nb);
        }
        layer<4, 2>(Lfb, Bh, D);
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            const int64_t v = base + nb * 16 + c;
            float R[4][4];
            bias_act<false>(D, Lbb, g, nb, R);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int j = 0; j < 4; ++j) R[q][j] += Rh[nb][q][j];
            if (v < n_nodes) store_row(h_out + v * 64, g, R);
        }
    }
}

// ------------------------------------- step-1 edge update + edge head

__global__ __launch_bounds__(kGnnThreads) void k_gnn_edge_last(GnnDev m, const float *h1, const float *e1,
                                                               const int32_t *src, const int32_t *dst,
                                                               int64_t n_nodes, int64_t n_edges, float *score) {
    __shared__ uint4 Lfa[4 * 6 * 64], Lfb[4 * 2 * 64], Lfh[2 * 2 * 64];
    __shared__ float Lba[64], Lbb[64], Lbh[32], Lw2[32];
    stage(Lfa, m.frag + m.foff[kGEdgeA1], 4 * 6 * 64, Lba, m.bias + m.boff[kGEdgeA1], 64);
    stage(Lfb, m.frag + m.foff[kGEdgeB1], 4 * 2 * 64, Lbb, m.bias + m.boff[kGEdgeB1], 64);
    stage(Lfh, m.frag + m.foff[kGHead1], 2 * 2 * 64, Lbh, m.bias + m.boff[kGHead1], 32);
    for (int i = threadIdx.x; i < 32; i += kGnnThreads) Lw2[i] = m.wh2[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    const int64_t wave = g_tid() >> 6, nwave = g_stride() >> 6;
    for (int64_t base = wave * kRowsPerWave; base < n_edges; base += nwave * kRowsPerWave) {
        bf16x8 Bin[6][kNB];
        float Re[kNB][4][4];
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            const int64_t row = base + nb * 16 + c;
            const bool ok = row < n_edges;
            const int64_t s = ok ? clamp_id(src[row], n_nodes) : 0, d = ok ? clamp_id(dst[row], n_nodes) : 0;
            float Rs[4][4], Rd[4][4];
            load_row(h1 + s * 64, g, ok, Rs);
            load_row(h1 + d * 64, g, ok, Rd);
            load_row(e1 + row * 64, g, ok, Re[nb]);
            r_to_b(Rs, &Bin[0][0], nb);
            r_to_b(Rd, &Bin[2][0], nb);
            r_to_b(Re[nb], &Bin[4][0], nb);
        }
        f32x4 D[4][kNB];
        layer<4, 6>(Lfa, Bin, D);
        bf16x8 Bh[2][kNB];
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            float R[4][4];
            bias_act<true>(D, Lba, g, nb, R);
            r_to_b(R, &Bh[0][0], nb);
        }
        layer<4, 2>(Lfb, Bh, D);
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            float R[4][4];
            bias_act<false>(D, Lbb, g, nb, R);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int j = 0; j < 4; ++j) R[q][j] += Re[nb][q][j];
            r_to_b(R, &Bh[0][0], nb);          // e2 (no activation) feeds the head
        }
        f32x4 H[2][kNB];
        layer<2, 2>(Lfh, Bh, H);
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            float part = 0.0f;
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int u = 16 * q + 4 * g + j;
                    part = __builtin_fmaf(Lw2[u], fmaxf(H[q][nb][j] + Lbh[u], 0.0f), part);
                }
            part += __shfl_xor(part, 16, 64);
            part += __shfl_xor(part, 32, 64);
            const int64_t row = base + nb * 16 + c;
            if (g == 0 && row < n_edges) score[row] = 1.0f / (1.0f + expf(-(part + m.bh2)));
        }
    }
}

static inline int gnn_blocks(int64_t rows) {
    int64_t b = (rows + kGnnWaves * kRowsPerWave - 1) / (kGnnWaves * kRowsPerWave);
    if (b < 1) b = 1;
    if (b > kGnnMaxBlocks) b = kGnnMaxBlocks;
    return (int)b;
}

hipError_t run_gnn(const GnnDev &m, const float *x, int64_t n_nodes, const int32_t *src, const int32_t *dst,
                   int64_t n_edges, float *score, const GnnWork &w, hipStream_t st) {
    hipLaunchKernelGGL(k_gnn_zero, dim3(1), dim3(64), 0, st, w.err);
    if (n_edges > 0) {
        int gb = (int)((n_edges + 255) / 256 < 4096 ? (n_edges + 255) / 256 : 4096);
        hipLaunchKernelGGL(k_gnn_check, dim3(gb), dim3(256), 0, st, src, dst, n_nodes, n_edges, w.err);
    }
    int ob = (int)((n_nodes + 256) / 256 < 4096 ? (n_nodes + 256) / 256 : 4096);
    hipLaunchKernelGGL(k_gnn_offsets, dim3(ob), dim3(256), 0, st, dst, n_nodes, n_edges, w.in_off);
    hipLaunchKernelGGL(k_gnn_encode, dim3(gnn_blocks(n_nodes)), dim3(kGnnThreads), 0, st, m, x, n_nodes, w.h0);
    if (n_edges == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_gnn_edge_first, dim3(gnn_blocks(n_edges)), dim3(kGnnThreads), 0, st, m, (const float *)w.h0,
                       src, dst, n_nodes, n_edges, w.e1);
    {
        int64_t mb = (n_nodes * 16 + 255) / 256;
        hipLaunchKernelGGL(k_gnn_msum, dim3((int)(mb < 16384 ? mb : 16384)), dim3(256), 0, st, (const float *)w.e1,
                           (const int64_t *)w.in_off, n_nodes, w.msg);
    }
    hipLaunchKernelGGL(k_gnn_node, dim3(gnn_blocks(n_nodes)), dim3(kGnnThreads), 0, st, m, (int)kGNodeA0,
                       (int)kGNodeB0, (const float *)w.h0, (const float *)w.msg, n_nodes, w.h1);
    hipLaunchKernelGGL(k_gnn_edge_last, dim3(gnn_blocks(n_edges)), dim3(kGnnThreads), 0, st, m, (const float *)w.h1,
                       (const float *)w.e1, src, dst, n_nodes, n_edges, score);
    return hipGetLastError();
}

}  // namespace lst
