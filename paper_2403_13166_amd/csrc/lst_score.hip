// T5-DNN scoring (paper Sec. 2: 42 inputs -> 32 -> 32 -> 1, ReLU hidden
// layers, sigmoid output) over dense feature rows.
//
// BF16 path: a block stages a tile of 256 contiguous rows in LDS with 16-byte
// coalesced loads; one wavefront then scores 64 of them on the matrix cores with
// v_mfma_f32_16x16x32_bf16, computing the transposed products
//   H1^T [32 x 64] = W1 [32 x 64(K, 42 padded)] . Xs^T [64 x 64]
//   H2^T [32 x 64] = W2 [32 x 32]               . relu(H1^T)
// so that each lane's accumulator rows of layer 1 are exactly the B operand
// of layer 2 once the K index of W2 is permuted accordingly (K is a summed
// index, so any consistent permutation is exact): no LDS round trip between
// the layers. Inputs are standardised in FP32 and rounded to BF16 (RNE);
// accumulation is FP32; the 32 -> 1 layer and the sigmoid run on the VALU.
//
// MFMA 16x16x32 lane layout (wave64, l = lane, g = l / 16):
//   A (16 x 32):  lane l holds A[l % 16][8 g + i], i = 0..7
//   B (32 x 16):  lane l holds B[8 g + i][l % 16], i = 0..7
//   D (16 x 16):  lane l holds D[4 g + j][l % 16], j = 0..3
#include <hip/hip_runtime.h>

#include "lst_internal.h"

namespace lst {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

template <int DT>
__device__ __forceinline__ float load_x(const void *X, int64_t i) {
    if (DT == 0) return ((const float *)X)[i];
    return bf16_to_f32(((const uint16_t *)X)[i]);
}

// FP32 vector-ALU scoring, one row per thread.
template <int DT>
__global__ __launch_bounds__(256) void k_score_f32(ModelDev m, const void *X, const int64_t *n_dev,
                                                   int64_t n_cap, float *out) {
    int64_t n = n_dev ? (*n_dev < n_cap ? *n_dev : n_cap) : n_cap;
    for (int64_t r = gtid(); r < n; r += gstride()) {
        float x[kNFeat];
#pragma unroll
        for (int k = 0; k < kNFeat; ++k) x[k] = load_x<DT>(X, r * kNFeat + k);
        out[r] = mlp_f32(m, x);
    }
}

// Hidden unit carried by B-operand slot i of lane group g in layer 2.
__device__ __forceinline__ int perm_unit(int g, int i) { return i < 4 ? 4 * g + i : 16 + 4 * g + (i - 4); }

constexpr int kScoreTile = 256;   // rows per block tile (4 wavefronts x 64 rows)

// One block tile of rows is a contiguous chunk of X (256 x 42 features); the
// block copies it to LDS with 16-byte coalesced loads (converting BF16 input
// to FP32), then every wavefront builds its MFMA operands from LDS.
template <int DT>
__device__ __forceinline__ void stage_rows(float *sx, const void *X, int64_t row0, int nrows) {
    const int nel = nrows * kNFeat;
    if (DT == 0) {
        const float *src = (const float *)X + row0 * kNFeat;
        const bool vec = ((uintptr_t)src & 15) == 0;
        const int n4 = vec ? nel / 4 : 0;
        for (int i = threadIdx.x; i < n4; i += 256)
            reinterpret_cast<float4 *>(sx)[i] = reinterpret_cast<const float4 *>(src)[i];
        for (int i = 4 * n4 + threadIdx.x; i < nel; i += 256) sx[i] = src[i];
    } else {
        const uint16_t *src = (const uint16_t *)X + row0 * kNFeat;
        const bool vec = ((uintptr_t)src & 15) == 0;
        const int n8 = vec ? nel / 8 : 0;
        for (int i = threadIdx.x; i < n8; i += 256) {
            const uint4 u = reinterpret_cast<const uint4 *>(src)[i];
            const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                sx[8 * i + 2 * k] = __uint_as_float(w[k] << 16);
                sx[8 * i + 2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
            }
        }
        for (int i = 8 * n8 + threadIdx.x; i < nel; i += 256) sx[i] = bf16_to_f32(src[i]);
    }
}

template <int DT>
__global__ __launch_bounds__(256) void k_score_mfma(ModelDev m, const void *X, const int64_t *n_dev,
                                                    int64_t n_cap, float *out) {
    __shared__ float sx[kScoreTile * kNFeat];
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15, wv = threadIdx.x >> 6;
    const int64_t n = n_dev ? (*n_dev < n_cap ? *n_dev : n_cap) : n_cap;
    // weights as A operands (kept in registers for the whole kernel)
    bf16x8 w1[2][2], w2[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                int k = ks * 32 + 8 * g + i;
                w1[mb][ks][i] = (__bf16)(k < kNFeat ? m.W1[(mb * 16 + c) * kNFeat + k] : 0.0f);
            }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) w2[mb][i] = (__bf16)m.W2[(mb * 16 + c) * kH1 + perm_unit(g, i)];
    }
    // per-lane standardisation constants of the features this lane loads
    float mu[2][8], isd[2][8];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int k = ks * 32 + 8 * g + i;
            mu[ks][i] = k < kNFeat ? m.mu[k] : 0.0f;
            isd[ks][i] = k < kNFeat ? 1.0f / m.sd[k] : 0.0f;
        }
    float b1v[2][4], b2v[2][4], w3v[2][4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            b1v[mb][j] = m.b1[mb * 16 + 4 * g + j];
            b2v[mb][j] = m.b2[mb * 16 + 4 * g + j];
            w3v[mb][j] = m.w3[mb * 16 + 4 * g + j];
        }
    for (int64_t row0 = (int64_t)blockIdx.x * kScoreTile; row0 < n; row0 += (int64_t)gridDim.x * kScoreTile) {
        const int nrows = n - row0 < kScoreTile ? (int)(n - row0) : kScoreTile;
        __syncthreads();                                   // the previous tile is consumed
        stage_rows<DT>(sx, X, row0, nrows);
        __syncthreads();
        const int base = wv * 64;                          // this wavefront's rows in the tile
        f32x4 acc1[2][4];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc1[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const int r = base + nb * 16 + c;
            const bool ok = r < nrows;
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                bf16x8 xb;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    int k = ks * 32 + 8 * g + i;
                    float v = (ok && k < kNFeat) ? (sx[r * kNFeat + k] - mu[ks][i]) * isd[ks][i] : 0.0f;
                    xb[i] = (__bf16)v;
                }
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
                    acc1[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1[mb][ks], xb, acc1[mb][nb], 0, 0, 0);
            }
        }
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            bf16x8 hb;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                hb[j] = (__bf16)fmaxf(acc1[0][nb][j] + b1v[0][j], 0.0f);
                hb[4 + j] = (__bf16)fmaxf(acc1[1][nb][j] + b1v[1][j], 0.0f);
            }
            float part = 0.0f;
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) {
                f32x4 a2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2[mb], hb, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
                for (int j = 0; j < 4; ++j) part = __builtin_fmaf(w3v[mb][j], fmaxf(a2[j] + b2v[mb][j], 0.0f), part);
            }
            part += __shfl_xor(part, 16, 64);
            part += __shfl_xor(part, 32, 64);
            const int r = base + nb * 16 + c;
            if (g == 0 && r < nrows) out[row0 + r] = 1.0f / (1.0f + expf(-(part + m.b3)));
        }
    }
}

static inline int blocks_for(int64_t n, int rows_per_block) {
    int64_t b = (n + rows_per_block - 1) / rows_per_block;
    if (b < 1) b = 1;
    if (b > 2048) b = 2048;
    return (int)b;
}

hipError_t run_score(const ModelDev &m, const void *X, int dtype, int64_t n, float *out, int precision,
                     hipStream_t st) {
    if (precision == 1) {
        if (dtype == 0)
            hipLaunchKernelGGL(k_score_mfma<0>, dim3(blocks_for(n, 256)), dim3(256), 0, st, m, X,
                               (const int64_t *)nullptr, n, out);
        else
            hipLaunchKernelGGL(k_score_mfma<1>, dim3(blocks_for(n, 256)), dim3(256), 0, st, m, X,
                               (const int64_t *)nullptr, n, out);
    } else {
        if (dtype == 0)
            hipLaunchKernelGGL(k_score_f32<0>, dim3(blocks_for(n, 256)), dim3(256), 0, st, m, X,
                               (const int64_t *)nullptr, n, out);
        else
            hipLaunchKernelGGL(k_score_f32<1>, dim3(blocks_for(n, 256)), dim3(256), 0, st, m, X,
                               (const int64_t *)nullptr, n, out);
    }
    return hipGetLastError();
}

}  // namespace lst
