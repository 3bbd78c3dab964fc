// T5-DNN scoring (paper Sec. 2: 42 inputs -> 32 -> 32 -> 1, ReLU hidden
// layers, sigmoid output) over dense feature rows given by the caller.
//
// BF16 path: a block stages a tile of 256 contiguous rows with 16-byte
// coalesced loads, standardising each value in FP32 and storing it as BF16
// (round to nearest even) in an LDS tile; the tile is then scored on the
// matrix cores (lst_mlp_tile.h, shared with the fused scoring of the build).
// FP32 path: one row per thread on the vector ALU.
#include <hip/hip_runtime.h>

#include "lst_internal.h"
#include "lst_mlp_tile.h"

namespace lst {

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

// Stage rows [row0, row0 + nrows) of X (row-major, kNFeat values per row) into
// the tile, standardised and rounded to BF16. Thread t takes the 16-byte
// chunks t, t + 256, ...; a chunk's values may straddle two rows.
template <int DT>
__device__ __forceinline__ void stage_rows_bf16(uint16_t *tile, const float *s_mu, const float *s_isd,
                                                const void *X, int64_t row0, int nrows) {
    const int nel = nrows * kNFeat;
    constexpr int kPerChunk = DT == 0 ? 4 : 8;
    const uint8_t *src = (const uint8_t *)X + row0 * kNFeat * (DT == 0 ? 4 : 2);
    const bool vec = ((uintptr_t)src & 15) == 0;
    const int nch = vec ? nel / kPerChunk : 0;
    auto put = [&](int idx, float x) {
        const int r = (idx * 24967) >> 20;           // idx / 42, exact for idx < 2^14
        const int k = idx - r * kNFeat;
        const __bf16 v = (__bf16)((x - s_mu[k]) * s_isd[k]);
        tile[r * kRowStride + k] = __builtin_bit_cast(uint16_t, v);
    };
    for (int c = threadIdx.x; c < nch; c += kTileRows) {
        const uint4 u = reinterpret_cast<const uint4 *>(src)[c];
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
        if (DT == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) put(4 * c + j, __uint_as_float(w[j]));
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                put(8 * c + 2 * j, __uint_as_float(w[j] << 16));
                put(8 * c + 2 * j + 1, __uint_as_float(w[j] & 0xffff0000u));
            }
        }
    }
    for (int i = kPerChunk * nch + threadIdx.x; i < nel; i += kTileRows) put(i, load_x<DT>(X, row0 * kNFeat + i));
}

static_assert(kTileRows * kNFeat < (1 << 14), "row index by multiply-shift");

template <int DT>
__global__ __launch_bounds__(kTileRows) void k_score_mfma(ModelDev m, const void *X, const int64_t *n_dev,
                                                          int64_t n_cap, float *out) {
    __shared__ __align__(16) uint16_t tile[kTileRows * kRowStride];
    __shared__ MlpFrags fr;
    __shared__ float s_mu[kNFeat], s_isd[kNFeat];
    mlp_tile_init(&fr, tile, m);
    if (threadIdx.x < kNFeat) {
        s_mu[threadIdx.x] = m.mu[threadIdx.x];
        s_isd[threadIdx.x] = 1.0f / m.sd[threadIdx.x];
    }
    const int64_t n = n_dev ? (*n_dev < n_cap ? *n_dev : n_cap) : n_cap;
    for (int64_t row0 = (int64_t)blockIdx.x * kTileRows; row0 < n; row0 += (int64_t)gridDim.x * kTileRows) {
        const int nrows = n - row0 < kTileRows ? (int)(n - row0) : kTileRows;
        __syncthreads();                                   // the previous tile is consumed
        stage_rows_bf16<DT>(tile, s_mu, s_isd, X, row0, nrows);
        __syncthreads();
        mlp_tile_score(tile, &fr, nrows, m, out + row0);
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
