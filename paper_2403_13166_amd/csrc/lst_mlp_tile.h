// T5-DNN (paper Sec. 2: 42 inputs -> 32 -> 32 -> 1, ReLU hidden layers,
// sigmoid output) on the matrix cores, for a block tile of feature rows held
// in LDS as standardised BF16.
//
// One wavefront scores 64 rows of the tile with v_mfma_f32_16x16x32_bf16,
// computing the transposed products
//   H1^T [32 x 64] = W1 [32 x 64(K, 42 padded)] . Xs^T [64 x 64]
//   H2^T [32 x 64] = W2 [32 x 32]               . relu(H1^T)
// so that each lane's accumulator rows of layer 1 are exactly the B operand
// of layer 2 once the K index of W2 is permuted accordingly (K is a summed
// index, so any consistent permutation is exact). Accumulation is FP32; the
// 32 -> 1 layer and the sigmoid run on the vector ALU.
//
// MFMA 16x16x32 lane layout (wave64, l = lane, g = l / 16):
//   A (16 x 32):  lane l holds A[l % 16][8 g + i], i = 0..7
//   B (32 x 16):  lane l holds B[8 g + i][l % 16], i = 0..7
//   D (16 x 16):  lane l holds D[4 g + j][l % 16], j = 0..3
#pragma once
#include <hip/hip_runtime.h>

#include "lst_device.h"

namespace lst {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTileRows = 256;    // rows of a block tile (4 wavefronts x 64 rows)
// BF16 values per tile row: 42 features, zeros up to the padded K of 64, and 8
// more so that consecutive rows start 4 LDS banks apart (16-byte reads of 8
// consecutive rows then touch 32 distinct banks)
constexpr int kRowStride = 72;

// Weights in MFMA A-fragment order (each lane's 8 BF16 values contiguous).
struct MlpFrags {
    bf16x8 w1[2][2][64];   // [16-unit block of layer 1][32-feature K chunk][lane]
    bf16x8 w2[2][64];      // [16-unit block of layer 2][lane]
};

// Hidden unit of layer 1 carried by B-operand slot i of lane group g in layer 2.
__device__ __forceinline__ int mlp_perm_unit(int g, int i) { return i < 4 ? 4 * g + i : 16 + 4 * g + (i - 4); }

// Fill the fragments (256 threads) and zero the K padding of every tile row.
// The caller synchronises the block before the first use.
__device__ __forceinline__ void mlp_tile_init(MlpFrags *fr, uint16_t *tile, const ModelDev &m) {
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15, j = threadIdx.x >> 6;
    const int mb = j >> 1, ks = j & 1;
    bf16x8 a;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = ks * 32 + 8 * g + i;
        a[i] = (__bf16)(k < kNFeat ? m.W1[(mb * 16 + c) * kNFeat + k] : 0.0f);
    }
    fr->w1[mb][ks][lane] = a;
    if (j < 2) {
        bf16x8 b;
#pragma unroll
        for (int i = 0; i < 8; ++i) b[i] = (__bf16)m.W2[(j * 16 + c) * kH1 + mlp_perm_unit(g, i)];
        fr->w2[j][lane] = b;
    }
    // K padding: BF16 columns 42..63 of each row (32-bit words 21..31)
    uint32_t *t32 = reinterpret_cast<uint32_t *>(tile);
    for (int i = threadIdx.x; i < kTileRows * 11; i += blockDim.x)
        t32[(i / 11) * (kRowStride / 2) + 21 + i % 11] = 0u;
}

// Standardise one row of FP32 features and store it as BF16 (round to nearest
// even) in row r of the tile.
__device__ __forceinline__ void mlp_tile_store_row(uint16_t *tile, int r, const float *ft, const ModelDev &m) {
    uint32_t *dst = reinterpret_cast<uint32_t *>(tile + r * kRowStride);
#pragma unroll
    for (int k = 0; k < kNFeat; k += 2) {
        const __bf16 lo = (__bf16)((ft[k] - ld_scalar(m.mu + k)) * (1.0f / ld_scalar(m.sd + k)));
        const __bf16 hi = (__bf16)((ft[k + 1] - ld_scalar(m.mu + k + 1)) * (1.0f / ld_scalar(m.sd + k + 1)));
        dst[k / 2] = (uint32_t)__builtin_bit_cast(uint16_t, lo) | ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
    }
}

// Score the first `nrows` rows of the tile into out[0 .. nrows).
__device__ __forceinline__ void mlp_tile_score(const uint16_t *tile, const MlpFrags *fr, int nrows,
                                               const ModelDev &m, float *out) {
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15, wv = threadIdx.x >> 6;
    const int base = wv * 64;                  // this wavefront's rows in the tile
    if (base >= nrows) return;
    f32x4 acc1[2][4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc1[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        const bf16x8 a0 = fr->w1[0][ks][lane], a1 = fr->w1[1][ks][lane];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const int r = base + nb * 16 + c;
            const bf16x8 xb = *reinterpret_cast<const bf16x8 *>(tile + r * kRowStride + ks * 32 + 8 * g);
            acc1[0][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, xb, acc1[0][nb], 0, 0, 0);
            acc1[1][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, xb, acc1[1][nb], 0, 0, 0);
        }
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
    const bf16x8 w20 = fr->w2[0][lane], w21 = fr->w2[1][lane];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        bf16x8 hb;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            hb[j] = (__bf16)fmaxf(acc1[0][nb][j] + b1v[0][j], 0.0f);
            hb[4 + j] = (__bf16)fmaxf(acc1[1][nb][j] + b1v[1][j], 0.0f);
        }
        const f32x4 z = f32x4{0.f, 0.f, 0.f, 0.f};
        const f32x4 h0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w20, hb, z, 0, 0, 0);
        const f32x4 h1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w21, hb, z, 0, 0, 0);
        float part = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) part = __builtin_fmaf(w3v[0][j], fmaxf(h0[j] + b2v[0][j], 0.0f), part);
#pragma unroll
        for (int j = 0; j < 4; ++j) part = __builtin_fmaf(w3v[1][j], fmaxf(h1[j] + b2v[1][j], 0.0f), part);
        part += __shfl_xor(part, 16, 64);
        part += __shfl_xor(part, 32, 64);
        const int r = base + nb * 16 + c;
        if (g == 0 && r < nrows) out[r] = 1.0f / (1.0f + expf(-(part + m.b3)));
    }
}

}  // namespace lst
