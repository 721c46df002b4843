// stage_common.h -- shared pieces of the five FFT stages of the demagnetizing-field convolution on gfx950.
//
// Order (App. A execution order, single GPU, no transfers):
//   x R2C   M[3][nz][ny][nx] (f32)        -> S1[3][nz][X1][ny] (c64, written transposed)
//   y FFT   S1                            -> S2[3][nz][X1][Ny] (c64)
//   z conv  S2 in place: z FFT, H^ = K M^ (6 real symmetric components), z IFFT
//   y IFFT  S2                            -> S1 (first ny outputs only)
//   x C2R   S1                            -> H[3][nz][ny][nx] (first nx outputs only)
//
// Zero padding is never stored.  A length-2n transform whose upper n inputs are
// zero splits into two length-n transforms: the even outputs are the DFT of x[t],
// the odd outputs the DFT of x[t] W_2n^t.  Symmetrically, only the first n
// outputs of a length-2n inverse are kept: y[t] = IE[t] + W_2n^-t IO[t], with IE
// and IO the inverses of the even and odd inputs.  Along x two real rows are
// packed into one complex line (z = a + i b) and separated afterwards through
// Hermitian symmetry, so every x transform does half the work of a complex one.
#pragma once

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "engine.h"
#include "fft_lds.h"

namespace dm {

constexpr int NT = 256;

// The two rows of a packed pair are adjacent in S1 (y fastest): move them as one
// 16-byte access when both exist (rows are even then, so the address is aligned).
__device__ __forceinline__ void store_pair(float2* d, float2 a, float2 b, int left) {
    if (left >= 2) *reinterpret_cast<float4*>(d) = make_float4(a.x, a.y, b.x, b.y);
    else if (left == 1) d[0] = a;
}
__device__ __forceinline__ void load_pair(const float2* s, float2& a, float2& b, int left) {
    if (left >= 2) {
        float4 v = *reinterpret_cast<const float4*>(s);
        a = make_float2(v.x, v.y);
        b = make_float2(v.z, v.w);
    } else {
        a = left == 1 ? s[0] : make_float2(0.f, 0.f);
        b = make_float2(0.f, 0.f);
    }
}

// A batched launch covers several independent work items (requests); item r
// owns blocks [start[r], start[r+1]) of the (XCD-renumbered) grid.
template <class B>
__device__ __forceinline__ int batch_item(const B& b, int gid) {
    int r = 0;
    while (r + 1 < b.count && gid >= b.start[r + 1]) ++r;
    return r;
}

// Copies n table entries into LDS (issued with the block's data loads; the
// block's first barrier makes them visible).
__device__ __forceinline__ void stage_table(float2* dst, const float2* __restrict__ src, int n) {
    for (int i = threadIdx.x; i < n; i += NT) dst[i] = src[i];
}

// ============================================================================ launchers
// Each stage has NVARIANTS tile shapes (more rows/lines/columns per block as the
// variant index grows); every variant computes bit-identical results because
// the per-line arithmetic does not depend on how many lines share a block.
namespace {

// x: rows per block (TY) = 4, 8, 16, capped so a block's LDS stays modest for
// long rows (the inverse holds two row buffers)
template <int L, int V, bool INV>
struct XTile {
    static constexpr int CAP = (INV ? 8192 : 16384) / L < 2 ? 2 : (INV ? 8192 : 16384) / L;
    static constexpr int TY = (4 << V) < CAP ? (4 << V) : CAP;
};
// x inverse, register form (variants 1 and 2): rows per block 4 and 8, capped so
// the parked even outputs and the prefetched odd inputs stay within registers
template <int L, int V>
struct XRegTile {
    static constexpr int CAP = 8192 / L < 2 ? 2 : 8192 / L;
    static constexpr int T0 = V <= 1 ? 4 : 8;
    static constexpr int TY = T0 < CAP ? T0 : CAP;
};
// y: padded elements per block 1024, 2048, 4096 -> lines per block
template <int L, int V>
struct YTile { static constexpr int LPB = 2 * L >= (1024 << V) ? 1 : (1024 << V) / (2 * L); };
// z: NZ * TH = 256, 512, 1024
template <int NZ, int V>
struct ZTile { static constexpr int TH = (256 << V) / NZ < 1 ? 1 : (256 << V) / NZ; };
// lean z kernel (512 threads): folded ky per tile = 512 / NZ, x2, x4, within 2 .. 32
template <int NZ, int V>
struct LeanZTile {
    static constexpr int T0 = (512 << V) / NZ;
    static constexpr int TH = T0 < 2 ? 2 : (T0 > 32 ? 32 : T0);
};

// Calls f with the MF form as a compile-time constant (0 for variants other than
// 1): 0 (FP32) or 3 (three-term split BF16 products).
template <int V, class F>
void mf_dispatch(int mf, F&& f) {
    if constexpr (V == 1) {
        if (mf == 3) f(std::integral_constant<int, 3>{});
        else f(std::integral_constant<int, 0>{});
    } else {
        f(std::integral_constant<int, 0>{});
    }
}

template <class B>
int finish_batch(B& b) {  // prefix sums already in start[]; returns the grid size
    return b.start[b.count];
}

}  // namespace

#define DM_POW2_CASES(MACRO) \
    MACRO(2) MACRO(4) MACRO(8) MACRO(16) MACRO(32) MACRO(64) MACRO(128) MACRO(256) MACRO(512) \
    MACRO(1024) MACRO(2048)
// Mesh sizes F 2^j (F = 3, 5, 15, j >= 1) along x and y: FP32, one tile shape.
#define DM_MIXED_CASES(MACRO)                                                                 \
    MACRO(6) MACRO(12) MACRO(24) MACRO(48) MACRO(96) MACRO(192) MACRO(384) MACRO(768)         \
    MACRO(1536) MACRO(10) MACRO(20) MACRO(40) MACRO(80) MACRO(160) MACRO(320) MACRO(640)      \
    MACRO(1280) MACRO(30) MACRO(60) MACRO(120) MACRO(240) MACRO(480) MACRO(960) MACRO(1920)

// The split-precision MFMA form (mf = 3) is built for the middle tile
// variant only; plans that use them always run variant 1.
#define DM_VARIANTS(BODY)        \
    if (mf) variant = 1;         \
    switch (variant) {           \
        case 0: BODY(0) break;   \
        case 1: BODY(1) break;   \
        default: BODY(2) break;  \
    }
#define DM_MF_DISPATCH(V, LAUNCH)                                                   \
    {                                                                               \
        mf_dispatch<V>(mf, [&](auto mfc) { constexpr int MFv = decltype(mfc)::value; LAUNCH }); \
    }

}  // namespace dm
