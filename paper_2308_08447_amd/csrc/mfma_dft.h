// mfma_dft.h -- 16-point DFTs as split-precision BF16 matrix products on the
// gfx950 matrix cores (v_mfma_f32_32x32x16_bf16).
//
// A batch of 32 sixteen-point DFTs y_n = F x_n (F_mr = exp(DIR 2 pi i m r/16)) is
// the real product
//     [Re Y; Im Y] (32 x 32 butterflies) = [[Fr, -Fi], [Fi, Fr]] (32 x 32) [Re X; Im X]
// taken as two 32x32x16 MFMA steps, one over the real and one over the imaginary
// parts of the inputs.  Both operands are split into BF16 terms,
//     v = v0 + v1 (+ v2),  v0 = bf16(v),  v1 = bf16(v - v0),  v2 = bf16(v - v0 - v1),
// each difference exact in FP32, and the products of the leading terms are
// accumulated in FP32: MF = 3 takes F0X0 + F0X1 + F1X0 + F0X2 + F1X1 + F2X0 (6
// products per step).  The library builds MF = 3 only: the two-term form
// (first three products) misses rel-L2 2e-5 where the field is small against
// the largest spectral values.  BF16 has FP32's exponent range, so
// no per-line scaling is needed for field values.
//
// Lane layout of the 32x32x16 MFMA (wave64; lane l, n = l % 32, h = l / 32):
//   A operand: row n, columns 8h .. 8h+7;   B operand: rows 8h .. 8h+7, column n;
//   result: acc[q] = D[8 (q/4) + 4h + q%4][n], q < 16.
// Butterfly n of a batch therefore lives in lanes n and n + 32: lane half h
// supplies inputs r = 8h .. 8h+7 and receives the outputs m = 4h .. 4h+3 and
// 8+4h .. 8+4h+3 (out_index).  F's column order is chosen to match: in the step
// over real parts column 8h + c multiplies Re x_{8h+c}, in the step over
// imaginary parts Im x_{8h+c}, so no lane exchange is needed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dm {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));

// round-to-nearest-even FP32 -> BF16 bits (finite inputs)
__device__ __forceinline__ uint32_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t b) { return __uint_as_float(b << 16); }

// Splits 8 FP32 values into MF BF16 operand vectors (leading term first).
template <int MF>
__device__ __forceinline__ void split_bf16(const float (&v)[8], bf16x8_t (&out)[MF]) {
    u16x8_t p[MF];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        float r = v[c];
#pragma unroll
        for (int s = 0; s < MF; ++s) {
            uint32_t b = bf16_bits(r);
            p[s][c] = (unsigned short)b;
            r = r - bf16_value(b);   // exact: the leading bits cancel
        }
    }
#pragma unroll
    for (int s = 0; s < MF; ++s) out[s] = __builtin_bit_cast(bf16x8_t, p[s]);
}

// cos(2 pi k / 16), k < 16
__device__ __forceinline__ float cos16(int k) {
    constexpr float c1 = 0.92387953251128676f, s1 = 0.38268343236508977f, h = 0.70710678118654752f;
    switch (k & 15) {
        case 0: return 1.f;
        case 1: case 15: return c1;
        case 2: case 14: return h;
        case 3: case 13: return s1;
        case 4: case 12: return 0.f;
        case 5: case 11: return -s1;
        case 6: case 10: return -h;
        case 7: case 9: return -c1;
        default: return -1.f;
    }
}

// The lane's slice of the DFT matrix, split once per transform: a[s][0] for the
// step over real parts, a[s][1] for the step over imaginary parts.
template <int MF>
struct Dft16Matrix {
    bf16x8_t a[MF][2];
    template <int DIR>
    __device__ __forceinline__ void init() {
        const int lane = threadIdx.x & 63, m = lane & 31, h = lane >> 5;
        float re[8], im[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            int r = 8 * h + c;
            int k = ((m & 15) * r) & 15;
            float fr = cos16(k), fi = DIR * cos16(k + 12);   // sin(x) = cos(x - pi/2)
            re[c] = m < 16 ? fr : fi;      // coefficient of Re x_r in Re y_m / Im y_m
            im[c] = m < 16 ? -fi : fr;     // coefficient of Im x_r
        }
        bf16x8_t t[MF];
        split_bf16<MF>(re, t);
#pragma unroll
        for (int s = 0; s < MF; ++s) a[s][0] = t[s];
        split_bf16<MF>(im, t);
#pragma unroll
        for (int s = 0; s < MF; ++s) a[s][1] = t[s];
    }
};
template <>
struct Dft16Matrix<0> {
    template <int DIR>
    __device__ __forceinline__ void init() {}
};

// Output index held in slot c (< 8) of lane half h.
__device__ __forceinline__ int out_index(int h, int c) { return (c < 4 ? 4 * h + c : 4 + 4 * h + c); }

// y = F x for the wave's 32 butterflies: x holds this lane's inputs 8h .. 8h+7
// (twiddles applied), y receives its outputs in out_index order.  Must be
// reached by all 64 lanes of the wave (lanes without a butterfly pass zeros).
template <int MF>
__device__ __forceinline__ void mfma_dft16(const Dft16Matrix<MF>& F, const float2 (&x)[8],
                                           float2 (&y)[8]) {
    float re[8], im[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        re[c] = x[c].x;
        im[c] = x[c].y;
    }
    bf16x8_t xr[MF], xi[MF];
    split_bf16<MF>(re, xr);
    split_bf16<MF>(im, xi);
    f32x16_t acc = {};
    // smallest products first
#define DM_MFMA_TERM(SA, SB)                                                             \
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.a[SA][0], xr[SB], acc, 0, 0, 0);    \
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.a[SA][1], xi[SB], acc, 0, 0, 0);
    if constexpr (MF >= 3) {
        DM_MFMA_TERM(2, 0)
        DM_MFMA_TERM(1, 1)
        DM_MFMA_TERM(0, 2)
    }
    DM_MFMA_TERM(1, 0)
    DM_MFMA_TERM(0, 1)
    DM_MFMA_TERM(0, 0)
#undef DM_MFMA_TERM
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        y[c] = make_float2(acc[c], acc[8 + c]);
        y[4 + c] = make_float2(acc[4 + c], acc[12 + c]);
    }
}

}  // namespace dm
