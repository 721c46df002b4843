// stages.hip -- the five FFT stages of the demagnetizing-field convolution on gfx950.
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
#include <algorithm>
#include <cmath>

#include "engine.h"
#include "fft_lds.h"

namespace dm {

constexpr int NT = 256;

// Workgroups are dispatched to the 8 XCDs round-robin.  Renumber them so that
// every XCD works on one contiguous range of tiles: neighbouring tiles, which
// share cache lines of their partial-line segments (transposed rows, kernel
// rows), then meet in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int B) {
    constexpr int NXCD = 8;
    int x = b % NXCD, i = b / NXCD;
    int q = B / NXCD, r = B % NXCD;
    return x * q + (x < r ? x : r) + i;
}

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

// ============================================================================ x
// One block: component c, plane z, rows y0 .. y0+TY-1 (TY/2 packed pairs).
// Forward: each pair z = a + i b is transformed twice (even outputs: DFT of z,
// odd outputs: DFT of z W_2L^t); the first pass reads the rows straight from M,
// the last pass leaves the spectrum in LDS in natural order, from where the
// Hermitian separation writes S1 transposed (consecutive threads, consecutive y).
template <int L, int TY>
__global__ __launch_bounds__(NT) void x_forward_kernel(const XBatch b,
                                                       const float2* __restrict__ tw_all) {
    constexpr int NP = TY / 2;
    constexpr int LS = lpad_c(L) + 1;  // odd stride: the pairs of one frequency hit distinct banks
    __shared__ float2 buf[NP * LS];
    __shared__ float2 twL[L];
    const float2* tw2L = tw_all + 2 * L;
    stage_table(twL, tw_all + L, L);
    const int tid = threadIdx.x;
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    const float* __restrict__ M = b.d[item].M;
    float2* __restrict__ S1 = b.d[item].S1;
    const int ny = b.d[item].ny, nz = b.d[item].nz;
    const float scale = b.d[item].scale;
    const int nyt = (ny + TY - 1) / TY;
    const int id = gid - b.start[item];
    const int y0 = (id % nyt) * TY, z = (id / nyt) % nz, c = id / (nyt * nz);
    const int rows = min(TY, ny - y0);
    const float* src = M + ((size_t)(c * nz + z) * ny + y0) * L;
    float2* dst = S1 + (size_t)(c * nz + z) * (L + 1) * ny + y0;

    auto pair = [&](int p, int t) {
        float a = (2 * p < rows) ? src[(size_t)(2 * p) * L + t] : 0.f;
        float b = (2 * p + 1 < rows) ? src[(size_t)(2 * p + 1) * L + t] : 0.f;
        return make_float2(a * scale, b * scale);
    };
    auto pair_odd = [&](int p, int t) { return cmul(pair(p, t), tw2L[t]); };
    auto to_lds = [&](int p, int k, float2 v) { buf[p * LS + lpad(k)] = v; };
    using Rows = RowLines<LS>;

    fft_io<L, -1, NP, NT, Rows, false, false, true>(buf, twL, pair, to_lds);
    __syncthreads();
    // even frequencies kx = 2m, m = 0..L/2: Z[2m] = E[m], Z[2L-2m] = E[(L-m) mod L]
    for (int it = tid; it < (L / 2 + 1) * NP; it += NT) {
        int p = it % NP, m = it / NP;
        float2 Zk = buf[p * LS + lpad(m)];
        float2 Zn = cconj(buf[p * LS + lpad((L - m) & (L - 1))]);
        float2 Xa = cscale(cadd(Zk, Zn), 0.5f);
        float2 d = csub(Zk, Zn);
        float2 Xb = make_float2(0.5f * d.y, -0.5f * d.x);
        store_pair(dst + (size_t)(2 * m) * ny + 2 * p, Xa, Xb, rows - 2 * p);
    }
    __syncthreads();
    fft_io<L, -1, NP, NT, Rows, false, false, true>(buf, twL, pair_odd, to_lds);
    __syncthreads();
    // odd frequencies kx = 2m+1, m < L/2: Z[2m+1] = O[m], Z[2L-2m-1] = O[L-1-m]
    for (int it = tid; it < (L / 2) * NP; it += NT) {
        int p = it % NP, m = it / NP;
        float2 Zk = buf[p * LS + lpad(m)];
        float2 Zn = cconj(buf[p * LS + lpad(L - 1 - m)]);
        float2 Xa = cscale(cadd(Zk, Zn), 0.5f);
        float2 d = csub(Zk, Zn);
        float2 Xb = make_float2(0.5f * d.y, -0.5f * d.x);
        store_pair(dst + (size_t)(2 * m + 1) * ny + 2 * p, Xa, Xb, rows - 2 * p);
    }
}

// Inverse: the even (odd) inputs Z[2m] (Z[2m+1]) of the packed pair are gathered
// from S1 (consecutive threads, consecutive y) into LDS; the inverse of the even
// part is parked in a second LDS region, and the last pass of the odd part
// combines z[t] = IE[t] + W_2L^-t IO[t] and stores both rows of H directly.
template <int L, int TY>
__global__ __launch_bounds__(NT) void x_inverse_kernel(const XBatch b,
                                                       const float2* __restrict__ tw_all) {
    constexpr int NP = TY / 2;
    constexpr int LS = lpad_c(L) + 1;  // odd stride: the pairs of one frequency hit distinct banks
    __shared__ float2 buf[NP * LS];
    __shared__ float2 ie[NP * LS];
    __shared__ float2 twL[L];
    __shared__ float2 tw2L[L];  // first half of the length-2L table
    stage_table(twL, tw_all + L, L);
    stage_table(tw2L, tw_all + 2 * L, L);
    const int tid = threadIdx.x;
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    const float2* __restrict__ S1 = b.d[item].S1;
    float* __restrict__ H = b.d[item].H;
    const int ny = b.d[item].ny, nz = b.d[item].nz;
    const int nyt = (ny + TY - 1) / TY;
    const int id = gid - b.start[item];
    const int y0 = (id % nyt) * TY, z = (id / nyt) % nz, c = id / (nyt * nz);
    const int rows = min(TY, ny - y0);
    const float2* src = S1 + (size_t)(c * nz + z) * (L + 1) * ny + y0;
    float* dst = H + ((size_t)(c * nz + z) * ny + y0) * L;
    using Rows = RowLines<LS>;

    // Z[k] = Xa[k] + i Xb[k]; for k > L use Hermitian symmetry X[2L-k] = conj(X[k]).
    // The DC and Nyquist bins of a real row are real: their imaginary parts are dropped.
    for (int it = tid; it < (L / 2 + 1) * NP; it += NT) {
        int p = it % NP, m = it / NP, kx = 2 * m;
        float2 Xa, Xb;
        load_pair(src + (size_t)kx * ny + 2 * p, Xa, Xb, rows - 2 * p);
        if (kx == 0 || kx == L) {
            Xa.y = 0.f;
            Xb.y = 0.f;
        }
        buf[p * LS + lpad(m)] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);
        if (kx > 0 && kx < L) buf[p * LS + lpad(L - m)] = make_float2(Xa.x + Xb.y, Xb.x - Xa.y);
    }
    __syncthreads();
    auto from_lds = [&](int p, int t) { return buf[p * LS + lpad(t)]; };
    auto park = [&](int p, int t, float2 v) { ie[p * LS + lpad(t)] = v; };
    fft_io<L, +1, NP, NT, Rows, false, false, true>(buf, twL, from_lds, park);
    __syncthreads();
    // Odd inputs Z[2m+1]: kx = 2m+1 < L direct, and Z[2L-kx] = conj -> slot L-1-m.
    for (int it = tid; it < (L / 2) * NP; it += NT) {
        int p = it % NP, m = it / NP, kx = 2 * m + 1;
        float2 Xa, Xb;
        load_pair(src + (size_t)kx * ny + 2 * p, Xa, Xb, rows - 2 * p);
        buf[p * LS + lpad(m)] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);
        buf[p * LS + lpad(L - 1 - m)] = make_float2(Xa.x + Xb.y, Xb.x - Xa.y);
    }
    __syncthreads();
    auto combine = [&](int p, int t, float2 io) {
        float2 zz = cadd(ie[p * LS + lpad(t)], cmul(cconj(tw2L[t]), io));
        if (2 * p < rows) dst[(size_t)(2 * p) * L + t] = zz.x;
        if (2 * p + 1 < rows) dst[(size_t)(2 * p + 1) * L + t] = zz.y;
    };
    fft_io<L, +1, NP, NT, Rows, false, false, true>(buf, twL, from_lds, combine);
}

// nx == 1: no x transform (N_x = 1); S1[c][z][0][y] = M[c][z][y][0]
__global__ void x_copy_forward_kernel(const float* __restrict__ M, float2* __restrict__ S1,
                                      size_t n, float scale) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) S1[i] = make_float2(M[i] * scale, 0.f);
}
__global__ void x_copy_inverse_kernel(const float2* __restrict__ S1, float* __restrict__ H,
                                      size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) H[i] = S1[i].x;
}

// ============================================================================ y
// The y and z stages run over a chunk of kx planes [k0, k0 + nk) whose spectra
// live in a chunk-sized S2 buffer [3][nz][xc][Ny] (local plane kx - k0).
// One block: LPB lines (consecutive kx) of one (c, z) plane.  Each line is a
// length-Ny = 2L transform whose upper L inputs are zero (forward) or whose
// upper L outputs are dropped (inverse); the first pass reads S1/S2 straight
// into registers and the last pass stores straight from registers.
template <int L, int LPB>
__global__ __launch_bounds__(NT) void y_forward_kernel(const YBatch b,
                                                       const float2* __restrict__ tw_all) {
    constexpr int LN = 2 * L;
    constexpr int LS = lpad_c(LN);
    __shared__ float2 buf[LPB * LS];
    __shared__ float2 tw[LN];
    stage_table(tw, tw_all + LN, LN);
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    const float2* __restrict__ S1 = b.d[item].S1;
    float2* __restrict__ S2 = b.d[item].S2;
    const int X1 = b.d[item].X1, nz = b.d[item].nz, k0 = b.d[item].k0, nk = b.d[item].nk;
    const int xc = b.d[item].xc;
    const int nt = (nk + LPB - 1) / LPB;
    const int id = gid - b.start[item];
    const int kl0 = (id % nt) * LPB, z = (id / nt) % nz, c = id / (nt * nz);
    const int nl = nk - kl0 < LPB ? nk - kl0 : LPB;  // valid lines in this block
    const float2* in = S1 + ((size_t)(c * nz + z) * X1 + k0 + kl0) * L;
    float2* out = S2 + ((size_t)(c * nz + z) * xc + kl0) * LN;
    auto src = [&](int l, int i) { return l < nl ? in[(size_t)l * L + i] : make_float2(0.f, 0.f); };
    auto sink = [&](int l, int k, float2 v) {
        if (l < nl) out[(size_t)l * LN + k] = v;
    };
    fft_io<LN, -1, LPB, NT, RowLines<LS>, true, false, false>(buf, tw, src, sink);
}

template <int L, int LPB>
__global__ __launch_bounds__(NT) void y_inverse_kernel(const YBatch b,
                                                       const float2* __restrict__ tw_all) {
    constexpr int LN = 2 * L;
    constexpr int LS = lpad_c(LN);
    __shared__ float2 buf[LPB * LS];
    __shared__ float2 tw[LN];
    stage_table(tw, tw_all + LN, LN);
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    const float2* __restrict__ S2 = b.d[item].S2;
    float2* __restrict__ S1 = b.d[item].S1;
    const int X1 = b.d[item].X1, nz = b.d[item].nz, k0 = b.d[item].k0, nk = b.d[item].nk;
    const int xc = b.d[item].xc;
    const int nt = (nk + LPB - 1) / LPB;
    const int id = gid - b.start[item];
    const int kl0 = (id % nt) * LPB, z = (id / nt) % nz, c = id / (nt * nz);
    const int nl = nk - kl0 < LPB ? nk - kl0 : LPB;
    const float2* in = S2 + ((size_t)(c * nz + z) * xc + kl0) * LN;
    float2* out = S1 + ((size_t)(c * nz + z) * X1 + k0 + kl0) * L;
    auto src = [&](int l, int i) { return l < nl ? in[(size_t)l * LN + i] : make_float2(0.f, 0.f); };
    auto sink = [&](int l, int k, float2 v) {
        if (l < nl) out[(size_t)l * L + k] = v;
    };
    fft_io<LN, +1, LPB, NT, RowLines<LS>, false, true, false>(buf, tw, src, sink);
}

// ============================================================================ z
// One block: folded ky indices f in [f0, f0 + th) of one kx, each taken together
// with its mirror ky = Ny - f, so that the kernel values K(kx, |ky|, |kz|) are read
// once for both.  The mirror slot of f = 0 (which has no mirror) carries the
// Nyquist column ky = Ny/2 instead.  Column j < TH holds ky = f0 + j, column
// TH + j holds the mirror of f0 + j.  All stored z planes of the 3 components are
// loaded into registers together with the K tile (so every global load of the
// block is in flight at once), then staged in LDS: element (z, c, column) at
// z * 3NC + c * NC + column, i.e. 3NC interleaved lines of length NZ.
template <int NZ, int TH>
__global__ __launch_bounds__(NT) void z_convolve_kernel(const ZBatch b,
                                                        const float2* __restrict__ tw_all) {
    constexpr int NZH = NZ > 1 ? NZ / 2 : 1;   // stored z planes
    constexpr int KT = NZ > 1 ? NZ / 2 + 1 : 1;  // folded kz values
    constexpr int NC = 2 * TH;                   // columns per block
    constexpr int NLN = 3 * NC;
    __shared__ float2 buf[NZ * NLN];
    __shared__ float ks[6 * KT * (TH + 1)];      // [comp][kz][f - f0], slot TH = Nyquist
    __shared__ float2 twZ[NZ];
    stage_table(twZ, tw_all + NZ, NZ);
    const int tid = threadIdx.x;
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    float2* __restrict__ S2 = b.d[item].S2;
    const float* __restrict__ K = b.d[item].K;
    const int X1 = b.d[item].X1, Ny = b.d[item].Ny, Y1 = b.d[item].Y1, Z1 = b.d[item].Z1;
    const int k0 = b.d[item].k0, xc = b.d[item].xc;
    const int ny = Ny > 1 ? Ny / 2 : 1;
    const int th = TH < ny ? TH : ny;
    const int nft = ny / th;
    const int id = gid - b.start[item];
    const int f0 = (id % nft) * th, kl = id / nft, kx = k0 + kl;
    const size_t P = (size_t)xc * Ny;  // complex elements per z plane of the chunk
    const size_t cstride = (size_t)NZH * P;
    float2* col = S2 + (size_t)kl * Ny;
    const bool nyq = (f0 == 0 && Ny > 1);
    auto col_ky = [&](int j) -> int {
        if (j < TH) return j < th ? f0 + j : -1;
        int jj = j - TH;
        if (jj >= th) return -1;
        int f = f0 + jj;
        if (f == 0) return nyq ? Ny / 2 : -1;
        return Ny - f;
    };

    // kernel tile: slot j < TH holds folded ky = f0 + j, slot TH the Nyquist column
    constexpr int NKL = 6 * KT * (TH + 1);
    constexpr int PK = (NKL + NT - 1) / NT;
    float kr[PK];
#pragma unroll
    for (int q = 0; q < PK; ++q) {
        int it = tid + q * NT;
        kr[q] = 0.f;
        if (it < NKL) {
            int j = it % (TH + 1), rest = it / (TH + 1), kz = rest % KT, comp = rest / KT;
            int f = (j < TH) ? (j < th ? f0 + j : -1) : (nyq ? Ny / 2 : -1);
            if (f >= 0) kr[q] = K[(((size_t)comp * Z1 + kz) * X1 + kx) * Y1 + f];
        }
    }
    // LDS line (c, column) = c * NC + column; element z of a line at z * NLN + line
    auto gsrc = [&](int line, int zz) {
        int c = line / NC, j = line - c * NC;
        int ky = col_ky(j);
        return ky >= 0 ? col[c * cstride + zz * P + ky] : make_float2(0.f, 0.f);
    };
    auto lds_sink = [&](int line, int k, float2 v) { buf[k * NLN + line] = v; };
    if constexpr (NZ == 1) {
        for (int line = tid; line < NLN; line += NT) buf[line] = gsrc(line, 0);
    } else {
        fft_io<NZ, -1, NLN, NT, ColLines<NLN>, true, false, true>(buf, twZ, gsrc, lds_sink);
    }
    // the kernel tile goes to LDS only now, so its loads overlapped the transform
#pragma unroll
    for (int q = 0; q < PK; ++q) {
        int it = tid + q * NT;
        if (it < NKL) ks[it] = kr[q];
    }
    __syncthreads();

    for (int it = tid; it < NZ * NC; it += NT) {
        int j = it % NC, kz = it / NC;
        if (col_ky(j) < 0) continue;
        int kzf = kz;
        float sz = 1.f;
        if (2 * kz > NZ) { kzf = NZ - kz; sz = -1.f; }
        int jj = j < TH ? j : j - TH;
        float sy = 1.f;
        int slot = jj;
        if (j >= TH) {
            if (f0 + jj == 0) slot = TH;   // Nyquist column, folded index Ny/2
            else sy = -1.f;
        }
        const float* k0p = ks + kzf * (TH + 1) + slot;
        constexpr int KC = KT * (TH + 1);
        float kxx = k0p[0], kyy = k0p[KC], kzz = k0p[2 * KC];
        float kxy = sy * k0p[3 * KC], kxz = sz * k0p[4 * KC], kyz = sy * sz * k0p[5 * KC];
        float2* p = buf + kz * NLN + j;
        float2 mx = p[0], my = p[NC], mz = p[2 * NC];
        auto dot3 = [](float a, float x, float b, float y, float c, float z) {
            return fmaf(c, z, fmaf(b, y, a * x));
        };
        p[0] = make_float2(dot3(kxx, mx.x, kxy, my.x, kxz, mz.x), dot3(kxx, mx.y, kxy, my.y, kxz, mz.y));
        p[NC] = make_float2(dot3(kxy, mx.x, kyy, my.x, kyz, mz.x), dot3(kxy, mx.y, kyy, my.y, kyz, mz.y));
        p[2 * NC] = make_float2(dot3(kxz, mx.x, kyz, my.x, kzz, mz.x), dot3(kxz, mx.y, kyz, my.y, kzz, mz.y));
    }
    __syncthreads();

    auto lds_src = [&](int line, int zz) { return buf[zz * NLN + line]; };
    auto gsink = [&](int line, int zz, float2 v) {
        int c = line / NC, j = line - c * NC;
        int ky = col_ky(j);
        if (ky >= 0) col[c * cstride + zz * P + ky] = v;
    };
    if constexpr (NZ == 1) {
        for (int line = tid; line < NLN; line += NT) gsink(line, 0, buf[line]);
    } else {
        fft_io<NZ, +1, NLN, NT, ColLines<NLN>, false, true, true>(buf, twZ, lds_src, gsink);
    }
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
// y: padded elements per block 1024, 2048, 4096 -> lines per block
template <int L, int V>
struct YTile { static constexpr int LPB = 2 * L >= (1024 << V) ? 1 : (1024 << V) / (2 * L); };
// z: NZ * TH = 256, 512, 1024
template <int NZ, int V>
struct ZTile { static constexpr int TH = (256 << V) / NZ < 1 ? 1 : (256 << V) / NZ; };

template <class B>
int finish_batch(B& b) {  // prefix sums already in start[]; returns the grid size
    return b.start[b.count];
}

}  // namespace

#define DM_POW2_CASES(MACRO) \
    MACRO(2) MACRO(4) MACRO(8) MACRO(16) MACRO(32) MACRO(64) MACRO(128) MACRO(256) MACRO(512) \
    MACRO(1024) MACRO(2048)

#define DM_VARIANTS(BODY) \
    switch (variant) {    \
        case 0: BODY(0) break; \
        case 1: BODY(1) break; \
        default: BODY(2) break; \
    }

int launch_x_forward(XBatch b, int nx, int variant, const float2* tw, hipStream_t s) {
    if (b.count < 1 || b.count > MAXB) return fail(DEMAG_EINVAL, "x stage: bad batch size");
    if (nx == 1) {
        for (int r = 0; r < b.count; ++r) {
            size_t n = (size_t)3 * b.d[r].nz * b.d[r].ny;
            hipLaunchKernelGGL(x_copy_forward_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                               s, b.d[r].M, b.d[r].S1, n, b.d[r].scale);
        }
        DM_CHECK_LAUNCH();
        return DEMAG_OK;
    }
    switch (nx) {
#define BODY(V)                                                                               \
    {                                                                                         \
        constexpr int TY = XTile<L, V, false>::TY;                                            \
        b.start[0] = 0;                                                                       \
        for (int r = 0; r < b.count; ++r)                                                     \
            b.start[r + 1] = b.start[r] + ((b.d[r].ny + TY - 1) / TY) * b.d[r].nz * 3;       \
        hipLaunchKernelGGL((x_forward_kernel<L, TY>), dim3((unsigned)finish_batch(b)), dim3(NT), \
                           0, s, b, tw);                                                      \
    }
#define CASE(Lv)                    \
    case Lv: {                      \
        constexpr int L = Lv;       \
        DM_VARIANTS(BODY)           \
        break;                      \
    }
        DM_POW2_CASES(CASE)
#undef CASE
#undef BODY
        default: return fail(DEMAG_EUNSUPPORTED, "x stage: unsupported nx");
    }
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

int launch_x_inverse(XBatch b, int nx, int variant, const float2* tw, hipStream_t s) {
    if (b.count < 1 || b.count > MAXB) return fail(DEMAG_EINVAL, "x stage: bad batch size");
    if (nx == 1) {
        for (int r = 0; r < b.count; ++r) {
            size_t n = (size_t)3 * b.d[r].nz * b.d[r].ny;
            hipLaunchKernelGGL(x_copy_inverse_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                               s, b.d[r].S1, b.d[r].H, n);
        }
        DM_CHECK_LAUNCH();
        return DEMAG_OK;
    }
    switch (nx) {
#define BODY(V)                                                                               \
    {                                                                                         \
        constexpr int TY = XTile<L, V, true>::TY;                                             \
        b.start[0] = 0;                                                                       \
        for (int r = 0; r < b.count; ++r)                                                     \
            b.start[r + 1] = b.start[r] + ((b.d[r].ny + TY - 1) / TY) * b.d[r].nz * 3;       \
        hipLaunchKernelGGL((x_inverse_kernel<L, TY>), dim3((unsigned)finish_batch(b)), dim3(NT), \
                           0, s, b, tw);                                                      \
    }
#define CASE(Lv)                    \
    case Lv: {                      \
        constexpr int L = Lv;       \
        DM_VARIANTS(BODY)           \
        break;                      \
    }
        DM_POW2_CASES(CASE)
#undef CASE
#undef BODY
        default: return fail(DEMAG_EUNSUPPORTED, "x stage: unsupported nx");
    }
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

template <bool INVERSE>
static int launch_y(YBatch b, int ny, int variant, const float2* tw, hipStream_t s) {
    if (b.count < 1 || b.count > MAXB) return fail(DEMAG_EINVAL, "y stage: bad batch size");
    if (ny == 1) return DEMAG_OK;  // no y transform (S2 aliases S1)
    switch (ny) {
#define BODY(V)                                                                                 \
    {                                                                                           \
        constexpr int LPB = YTile<L, V>::LPB;                                                   \
        b.start[0] = 0;                                                                         \
        for (int r = 0; r < b.count; ++r)                                                       \
            b.start[r + 1] = b.start[r] + ((b.d[r].nk + LPB - 1) / LPB) * b.d[r].nz * 3;       \
        if (INVERSE)                                                                            \
            hipLaunchKernelGGL((y_inverse_kernel<L, LPB>), dim3((unsigned)finish_batch(b)),     \
                               dim3(NT), 0, s, b, tw);                                          \
        else                                                                                    \
            hipLaunchKernelGGL((y_forward_kernel<L, LPB>), dim3((unsigned)finish_batch(b)),     \
                               dim3(NT), 0, s, b, tw);                                          \
    }
#define CASE(Lv)                    \
    case Lv: {                      \
        constexpr int L = Lv;       \
        DM_VARIANTS(BODY)           \
        break;                      \
    }
        DM_POW2_CASES(CASE)
#undef CASE
#undef BODY
        default: return fail(DEMAG_EUNSUPPORTED, "y stage: unsupported ny");
    }
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

int launch_y_forward(YBatch b, int ny, int variant, const float2* tw, hipStream_t s) {
    return launch_y<false>(b, ny, variant, tw, s);
}
int launch_y_inverse(YBatch b, int ny, int variant, const float2* tw, hipStream_t s) {
    return launch_y<true>(b, ny, variant, tw, s);
}

int launch_z_convolve(ZBatch b, int Nz, int variant, const float2* tw, hipStream_t s) {
    if (b.count < 1 || b.count > MAXB) return fail(DEMAG_EINVAL, "z stage: bad batch size");
    switch (Nz) {
#define BODY(V)                                                                                \
    {                                                                                          \
        constexpr int TH = ZTile<NZ, V>::TH;                                                   \
        b.start[0] = 0;                                                                        \
        for (int r = 0; r < b.count; ++r) {                                                    \
            int ny = b.d[r].Ny > 1 ? b.d[r].Ny / 2 : 1;                                        \
            int th = TH < ny ? TH : ny;                                                        \
            b.start[r + 1] = b.start[r] + (ny / th) * b.d[r].nk;                               \
        }                                                                                      \
        hipLaunchKernelGGL((z_convolve_kernel<NZ, TH>), dim3((unsigned)finish_batch(b)),       \
                           dim3(NT), 0, s, b, tw);                                             \
    }
#define CASE(NZv)                   \
    case NZv: {                     \
        constexpr int NZ = NZv;     \
        DM_VARIANTS(BODY)           \
        break;                      \
    }
        CASE(1) CASE(4) CASE(8) CASE(16) CASE(32) CASE(64) CASE(128) CASE(256)
#undef CASE
#undef BODY
        default: return fail(DEMAG_EUNSUPPORTED, "z stage: unsupported nz");
    }
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

int twiddle_table_length(const Geometry& g) {
    int m = 2;
    m = std::max(m, g.Nx);
    m = std::max(m, g.Ny);
    m = std::max(m, g.Nz);
    return m;
}

void fill_twiddles(float2* host, int Lmax) {
    // table for length L at offset L (L = 1, 2, 4, ..., Lmax): exp(-2 pi i t/L)
    host[0] = make_float2(0.f, 0.f);
    for (int L = 1; L <= Lmax; L *= 2) {
        for (int t = 0; t < L; ++t) {
            long double ang = -2.0L * 3.141592653589793238462643383279502884L * t / L;
            host[L + t] = make_float2((float)cosl(ang), (float)sinl(ang));
        }
    }
}

}  // namespace dm
