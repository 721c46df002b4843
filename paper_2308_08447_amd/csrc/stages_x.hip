// stages_x.hip -- x stages: R2C of packed real row pairs, C2R with the Hermitian combine (see stage_common.h for the stage order).
#include "stage_common.h"

namespace dm {

// Twiddle sources of the x stages: the tables themselves in LDS, or for FP32
// from L = 1024 on coarse x fine pairs (Tw2), so that the row buffers, not the
// tables, set how many blocks a compute unit holds.  (The MFMA forms keep the
// tables: the extra product raised their registers past two waves per SIMD.)
template <int L, int MF>
constexpr bool x_tw2() { return L >= 1024 && MF == 0; }
template <int L, int MF, int NTX = NT>
__device__ __forceinline__ auto x_twiddles(float2* twt, const float2* __restrict__ full) {
    if constexpr (x_tw2<L, MF>()) {
        return stage_tw2<L, NTX>(twt, full);
    } else {
        for (int i = threadIdx.x; i < L; i += NTX) twt[i] = full[i];
        return (const float2*)twt;
    }
}
// entries t < L of the length-2L table (the inverse's odd-part rotation)
template <int L, int MF, bool PX, int NTX = NT>
__device__ __forceinline__ auto x_twiddles_2l(float2* twt, const float2* __restrict__ full) {
    if constexpr (x_tw2<L, MF>()) {
        return stage_tw2<2 * L, NTX>(twt, full);
    } else {
        if constexpr (!PX)
            for (int i = threadIdx.x; i < L; i += NTX) twt[i] = full[i];
        return (const float2*)twt;
    }
}

// LDS stride of the NP packed lines of an x block (in float2): the Hermitian
// separation and the inverse's gather walk element m of all NP lines with
// consecutive threads on consecutive lines, so 16 neighbouring threads touch
// elements (p, m) .. (p + NP - 1, m + 16/NP - 1).  A stride of 16/NP modulo 16
// puts those 16 float2 (128 bytes) on distinct banks; an odd stride made
// (p + 1, m) and (p, m + 1) collide.
template <int L, int NP>
constexpr int x_line_stride() {
    constexpr int base = lpad_c(L) + 1;
    constexpr int want = NP >= 16 ? 1 : 16 / NP;
    return base + ((want - base % 16) + 16) % 16;
}

// ============================================================================ x
// One block: component c, plane z, rows y0 .. y0+TY-1 (TY/2 packed pairs).
// Forward: each pair z = a + i b is transformed twice (even outputs: DFT of z,
// odd outputs: DFT of z W_2L^t); the first pass reads the rows straight from M,
// the last pass leaves the spectrum in LDS in natural order, from where the
// Hermitian separation writes S1 transposed (consecutive threads, consecutive y).
// PX (periodic x, transform length L): the DFT of z alone gives the L/2 + 1
// frequencies, stored at kx = m.
template <int L, int TY, int MF, bool PX = false>
__global__ __launch_bounds__(NT) void x_forward_kernel(const XBatch b,
                                                       const float2* __restrict__ tw_all) {
    constexpr int X1 = PX ? L / 2 + 1 : L + 1;
    constexpr int NP = TY / 2;
    constexpr int LS = x_line_stride<L, NP>();
    __shared__ float2 buf[NP * LS];
    __shared__ float2 twt[x_tw2<L, MF>() ? tw2_entries(L) : L];
    const auto twL = x_twiddles<L, MF>(twt, tw_all + tw_offset(L));
    const float2* tw2L = tw_all + tw_offset(2 * L);
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
    float2* dst = S1 + (size_t)(c * nz + z) * X1 * ny + y0;

    auto pair = [&](int p, int t) {
        float a = (2 * p < rows) ? src[(size_t)(2 * p) * L + t] : 0.f;
        float b = (2 * p + 1 < rows) ? src[(size_t)(2 * p + 1) * L + t] : 0.f;
        return make_float2(a * scale, b * scale);
    };
    auto pair_odd = [&](int p, int t) { return cmul(pair(p, t), tw2L[t]); };
    auto to_lds = [&](int p, int k, float2 v) { buf[p * LS + lpad(k)] = v; };
    using Rows = RowLines<LS>;

    fft_io<L, -1, NP, NT, Rows, false, false, true, MF>(buf, twL, pair, to_lds);
    __syncthreads();
    // even frequencies kx = 2m, m = 0..L/2: Z[2m] = E[m], Z[2L-2m] = E[(L-m) mod L]
    for (int it = tid; it < (L / 2 + 1) * NP; it += NT) {
        int p = it % NP, m = it / NP;
        float2 Zk = buf[p * LS + lpad(m)];
        float2 Zn = cconj(buf[p * LS + lpad(m == 0 ? 0 : L - m)]);
        float2 Xa = cscale(cadd(Zk, Zn), 0.5f);
        float2 d = csub(Zk, Zn);
        float2 Xb = make_float2(0.5f * d.y, -0.5f * d.x);
        store_pair(dst + (size_t)(PX ? m : 2 * m) * ny + 2 * p, Xa, Xb, rows - 2 * p);
    }
    if constexpr (PX) return;
    __syncthreads();
    fft_io<L, -1, NP, NT, Rows, false, false, true, MF>(buf, twL, pair_odd, to_lds);
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

// Register form of the forward (FP32, open x, power-of-two L >= 32): the row
// values the first pass of the even part reads stay in registers and feed the
// first pass of the odd part as well, so M is read from global memory once
// instead of twice.  The arithmetic is that of x_forward_kernel (the odd inputs
// are the same products z[t] W_2L^t), so both give the same bits.  NTX threads
// per block: 512 gives a 16-row tile of 1024 twice the waves of 256 for the
// same LDS (its 70 KB allow two blocks per compute unit).
template <int L, int TY, int NTX = NT>
__global__ __launch_bounds__(NTX) void x_forward_reg_kernel(const XBatch b,
                                                           const float2* __restrict__ tw_all) {
    constexpr int X1 = L + 1;
    constexpr int NP = TY / 2;
    constexpr int LS = x_line_stride<L, NP>();
    __shared__ float2 buf[NP * LS];
    __shared__ float2 twt[x_tw2<L, 0>() ? tw2_entries(L) : L];
    const auto twL = x_twiddles<L, 0, NTX>(twt, tw_all + tw_offset(L));
    const float2* tw2L = tw_all + tw_offset(2 * L);
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
    float2* dst = S1 + (size_t)(c * nz + z) * X1 * ny + y0;
    using Rows = RowLines<LS>;
    constexpr int R0 = head_radix<L>(), PF = head_per<L, NP, NTX>(), NB0 = L / R0;

    float2 raw[PF][R0];
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        const int bb = tid + q * NTX;
        if ((NB0 * NP) % NTX == 0 || bb < NB0 * NP) {
            int p, j;
            Rows::template split<NB0>(bb, p, j);
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int t = j + r * NB0;
                const float a = (2 * p < rows) ? src[(size_t)(2 * p) * L + t] : 0.f;
                const float bv = (2 * p + 1 < rows) ? src[(size_t)(2 * p + 1) * L + t] : 0.f;
                raw[q][r] = make_float2(a * scale, bv * scale);
            }
        }
    }
    auto to_lds = [&](int p, int k, float2 v) { buf[p * LS + lpad(k)] = v; };
    {
        float2 v[PF][R0];
#pragma unroll
        for (int q = 0; q < PF; ++q)
#pragma unroll
            for (int r = 0; r < R0; ++r) v[q][r] = raw[q][r];
        fft_head_regs<L, -1, NP, NTX, Rows>(buf, twL, v);
        last_pass<L, tail_radix<L>(), -1, NP, NTX, Rows, false, true>(buf, twL, to_lds);
    }
    __syncthreads();
    // even frequencies kx = 2m, m = 0..L/2: Z[2m] = E[m], Z[2L-2m] = E[(L-m) mod L]
    for (int it = tid; it < (L / 2 + 1) * NP; it += NTX) {
        int p = it % NP, m = it / NP;
        float2 Zk = buf[p * LS + lpad(m)];
        float2 Zn = cconj(buf[p * LS + lpad(m == 0 ? 0 : L - m)]);
        float2 Xa = cscale(cadd(Zk, Zn), 0.5f);
        float2 d = csub(Zk, Zn);
        float2 Xb = make_float2(0.5f * d.y, -0.5f * d.x);
        store_pair(dst + (size_t)(2 * m) * ny + 2 * p, Xa, Xb, rows - 2 * p);
    }
    __syncthreads();
    {
        float2 v[PF][R0];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int bb = tid + q * NTX;
            int p, j;
            Rows::template split<NB0>(bb, p, j);
#pragma unroll
            for (int r = 0; r < R0; ++r) v[q][r] = cmul(raw[q][r], tw2L[j + r * NB0]);
        }
        fft_head_regs<L, -1, NP, NTX, Rows>(buf, twL, v);
        last_pass<L, tail_radix<L>(), -1, NP, NTX, Rows, false, true>(buf, twL, to_lds);
    }
    __syncthreads();
    // odd frequencies kx = 2m+1, m < L/2: Z[2m+1] = O[m], Z[2L-2m-1] = O[L-1-m]
    for (int it = tid; it < (L / 2) * NP; it += NTX) {
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
// PX (periodic x): the L inputs Z[m] come from kx = m and their inverse is z.
template <int L, int TY, int MF, bool PX = false>
__global__ __launch_bounds__(NT) void x_inverse_kernel(const XBatch b,
                                                       const float2* __restrict__ tw_all) {
    constexpr int X1 = PX ? L / 2 + 1 : L + 1;
    constexpr int NP = TY / 2;
    constexpr int LS = x_line_stride<L, NP>();
    __shared__ float2 buf[NP * LS];
    __shared__ float2 ie[PX ? 1 : NP * LS];
    __shared__ float2 twt[x_tw2<L, MF>() ? tw2_entries(L) : L];
    // first half of the length-2L table
    __shared__ float2 tw2t[PX ? 1 : (x_tw2<L, MF>() ? tw2_entries(2 * L) : L)];
    const auto twL = x_twiddles<L, MF>(twt, tw_all + tw_offset(L));
    const auto tw2L = x_twiddles_2l<L, MF, PX>(tw2t, tw_all + tw_offset(2 * L));
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
    const float2* src = S1 + (size_t)(c * nz + z) * X1 * ny + y0;
    float* dst = H + ((size_t)(c * nz + z) * ny + y0) * L;
    using Rows = RowLines<LS>;

    // Z[k] = Xa[k] + i Xb[k]; for k > L use Hermitian symmetry X[2L-k] = conj(X[k]).
    // The DC and Nyquist bins of a real row are real: their imaginary parts are dropped.
    for (int it = tid; it < (L / 2 + 1) * NP; it += NT) {
        int p = it % NP, m = it / NP, kx = PX ? m : 2 * m;
        float2 Xa, Xb;
        load_pair(src + (size_t)kx * ny + 2 * p, Xa, Xb, rows - 2 * p);
        if (m == 0 || 2 * m == L) {
            Xa.y = 0.f;
            Xb.y = 0.f;
        }
        buf[p * LS + lpad(m)] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);
        if (m > 0 && 2 * m < L) buf[p * LS + lpad(L - m)] = make_float2(Xa.x + Xb.y, Xb.x - Xa.y);
    }
    __syncthreads();
    auto from_lds = [&](int p, int t) { return buf[p * LS + lpad(t)]; };
    if constexpr (PX) {
        auto rows_out = [&](int p, int t, float2 zz) {
            if (2 * p < rows) dst[(size_t)(2 * p) * L + t] = zz.x;
            if (2 * p + 1 < rows) dst[(size_t)(2 * p + 1) * L + t] = zz.y;
        };
        fft_io<L, +1, NP, NT, Rows, false, false, true, MF>(buf, twL, from_lds, rows_out);
        return;
    }
    auto park = [&](int p, int t, float2 v) { ie[p * LS + lpad(t)] = v; };
    fft_io<L, +1, NP, NT, Rows, false, false, true, MF>(buf, twL, from_lds, park);
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
        float2 zz = cmad(cconj(tw2L[t]), io, ie[p * LS + lpad(t)]);
        if (2 * p < rows) dst[(size_t)(2 * p) * L + t] = zz.x;
        if (2 * p + 1 < rows) dst[(size_t)(2 * p + 1) * L + t] = zz.y;
    };
    fft_io<L, +1, NP, NT, Rows, false, false, true, MF>(buf, twL, from_lds, combine);
}

// Register form of the inverse (FP32, open x, power-of-two L >= 32): the last
// pass of the even part leaves IE in the registers of the thread that later runs
// the same butterfly of the odd part's last pass, so IE needs no second LDS
// region (half the LDS of the kernel above, twice the blocks per compute unit),
// and the odd inputs are loaded into registers while the even part is
// transformed.  The arithmetic is that of x_inverse_kernel, so both give the
// same bits.  Registers are held to 128 so that four blocks share a compute
// unit, as many as the LDS of 8 rows of 1024 allows.
template <int L, int TY, int NTX = NT>
__global__ __launch_bounds__(NTX, 4) void x_inverse_reg_kernel(const XBatch b,
                                                           const float2* __restrict__ tw_all) {
    constexpr int X1 = L + 1;
    constexpr int NP = TY / 2;
    constexpr int LS = x_line_stride<L, NP>();
    __shared__ float2 buf[NP * LS];
    __shared__ float2 twt[x_tw2<L, 0>() ? tw2_entries(L) : L];
    __shared__ float2 tw2t[x_tw2<L, 0>() ? tw2_entries(2 * L) : L];
    const auto twL = x_twiddles<L, 0, NTX>(twt, tw_all + tw_offset(L));
    const auto tw2L = x_twiddles_2l<L, 0, false, NTX>(tw2t, tw_all + tw_offset(2 * L));
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
    const float2* src = S1 + (size_t)(c * nz + z) * X1 * ny + y0;
    float* dst = H + ((size_t)(c * nz + z) * ny + y0) * L;
    using Rows = RowLines<LS>;

    for (int it = tid; it < (L / 2 + 1) * NP; it += NTX) {
        int p = it % NP, m = it / NP, kx = 2 * m;
        float2 Xa, Xb;
        load_pair(src + (size_t)kx * ny + 2 * p, Xa, Xb, rows - 2 * p);
        if (m == 0 || 2 * m == L) {
            Xa.y = 0.f;
            Xb.y = 0.f;
        }
        buf[p * LS + lpad(m)] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);
        if (m > 0 && 2 * m < L) buf[p * LS + lpad(L - m)] = make_float2(Xa.x + Xb.y, Xb.x - Xa.y);
    }
    // odd inputs kx = 2m + 1, in flight during the even part's transform
    constexpr int NO = (L / 2) * NP;
    constexpr int PO = (NO + NTX - 1) / NTX;
    float2 oa[PO], ob[PO];
#pragma unroll
    for (int q = 0; q < PO; ++q) {
        const int it = tid + q * NTX;
        if (NO % NTX == 0 || it < NO) {
            const int p = it % NP, m = it / NP;
            load_pair(src + (size_t)(2 * m + 1) * ny + 2 * p, oa[q], ob[q], rows - 2 * p);
        }
    }
    __syncthreads();
    auto from_lds = [&](int p, int t) { return buf[p * LS + lpad(t)]; };
    constexpr int RL = tail_radix<L>(), PER = tail_per<L, NP, NTX>(), NB = L / RL;
    float2 ie[PER][RL];
    fft_head<L, +1, NP, NTX, Rows, false, true>(buf, twL, from_lds);
    fft_tail<L, +1, NP, NTX, Rows>(buf, twL, ie);
    __syncthreads();
    // Z[2m+1] at slot m, and Z[2L-2m-1] = conj -> slot L-1-m
#pragma unroll
    for (int q = 0; q < PO; ++q) {
        const int it = tid + q * NTX;
        if (NO % NTX == 0 || it < NO) {
            const int p = it % NP, m = it / NP;
            const float2 Xa = oa[q], Xb = ob[q];
            buf[p * LS + lpad(m)] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);
            buf[p * LS + lpad(L - 1 - m)] = make_float2(Xa.x + Xb.y, Xb.x - Xa.y);
        }
    }
    __syncthreads();
    float2 io[PER][RL];
    fft_head<L, +1, NP, NTX, Rows, false, true>(buf, twL, from_lds);
    fft_tail<L, +1, NP, NTX, Rows>(buf, twL, io);
    // z[t] = IE[t] + W_2L^-t IO[t]; both rows of the pair go straight to H
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int bb = tid + q * NTX;
        if ((NB * NP) % NTX == 0 || bb < NB * NP) {
            int p, j;
            Rows::template split<NB>(bb, p, j);
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int t = j + r * NB;
                const float2 zz = cmad(cconj(tw2L[t]), io[q][r], ie[q][r]);
                if (2 * p < rows) dst[(size_t)(2 * p) * L + t] = zz.x;
                if (2 * p + 1 < rows) dst[(size_t)(2 * p + 1) * L + t] = zz.y;
            }
        }
    }
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


int launch_x_forward(XBatch b, int nx, int variant, int mf, const float2* tw, hipStream_t s,
                     bool periodic) {
    if (b.count < 1 || b.count > MAXB) return fail(DEMAG_EINVAL, "x stage: bad batch size");
    if (nx == 1) {
        for (int r = 0; r < b.count; ++r) {
            size_t n = (size_t)3 * b.d[r].nz * b.d[r].ny;
            DM_LAUNCH(x_copy_forward_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                      s, b.d[r].M, b.d[r].S1, n, b.d[r].scale);
        }
        DM_CHECK_LAUNCH();
        return DEMAG_OK;
    }
    if (periodic) {
        if (mf) return fail(DEMAG_EUNSUPPORTED, "x stage: periodic transforms are FP32 only");
        switch (nx) {
#define CASE(Lv)                                                                                  \
    case Lv: {                                                                                    \
        constexpr int L = Lv;                                                                     \
        constexpr int TY = XTile<L, 1, false>::TY;                                                  \
        b.start[0] = 0;                                                                           \
        for (int r = 0; r < b.count; ++r)                                                         \
            b.start[r + 1] = b.start[r] + ((b.d[r].ny + TY - 1) / TY) * b.d[r].nz * 3;           \
        DM_LAUNCH((x_forward_kernel<L, TY, 0, true>), dim3((unsigned)finish_batch(b)),           \
                  dim3(NT), 0, s, b, tw);                                                        \
        break;                                                                                    \
    }
            DM_POW2_CASES(CASE)
#undef CASE
            default: return fail(DEMAG_EUNSUPPORTED, "x stage: unsupported nx");
        }
        DM_CHECK_LAUNCH();
        return DEMAG_OK;
    }
    if (!is_pow2c(nx)) {
        if (mf) return fail(DEMAG_EUNSUPPORTED, "x stage: mixed-radix transforms are FP32 only");
        switch (nx) {
#define CASE(Lv)                                                                                  \
    case Lv: {                                                                                    \
        constexpr int L = Lv;                                                                     \
        constexpr int TY = XTile<L, 1, false>::TY;                                                  \
        b.start[0] = 0;                                                                           \
        for (int r = 0; r < b.count; ++r)                                                         \
            b.start[r + 1] = b.start[r] + ((b.d[r].ny + TY - 1) / TY) * b.d[r].nz * 3;           \
        DM_LAUNCH((x_forward_kernel<L, TY, 0, false>), dim3((unsigned)finish_batch(b)),          \
                  dim3(NT), 0, s, b, tw);                                                        \
        break;                                                                                    \
    }
            DM_MIXED_CASES(CASE)
#undef CASE
            default: return fail(DEMAG_EUNSUPPORTED, "x stage: unsupported nx");
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
        if constexpr (npasses(L) >= 2) {                                                      \
            if (mf == 0) {                                                                    \
                /* variant 0: the largest row tile on 512 threads, where its first pass */  \
                /* has a butterfly for each */                                                \
                constexpr int TYW = XTile<L, 2, false>::TY;                                   \
                constexpr int NTW = (TYW / 2) * (L / head_radix<L>()) >= 2 * NT ? 2 * NT : NT; \
                if (V == 0 && NTW > NT) {                                                     \
                    for (int r = 0; r < b.count; ++r)                                         \
                        b.start[r + 1] = b.start[r] + ((b.d[r].ny + TYW - 1) / TYW) * b.d[r].nz * 3; \
                    DM_LAUNCH((x_forward_reg_kernel<L, TYW, NTW>),                                   \
                              dim3((unsigned)finish_batch(b)), dim3(NTW), 0, s, b, tw);              \
                    break;                                                                    \
                }                                                                             \
                DM_LAUNCH((x_forward_reg_kernel<L, TY>),                                      \
                          dim3((unsigned)finish_batch(b)), dim3(NT), 0, s, b, tw);            \
                break;                                                                        \
            }                                                                                 \
        }                                                                                     \
        DM_MF_DISPATCH(V, DM_LAUNCH((x_forward_kernel<L, TY, MFv>),                           \
                  dim3((unsigned)finish_batch(b)), dim3(NT), 0, s, b, tw);)                   \
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

int launch_x_inverse(XBatch b, int nx, int variant, int mf, const float2* tw, hipStream_t s,
                     bool periodic) {
    if (b.count < 1 || b.count > MAXB) return fail(DEMAG_EINVAL, "x stage: bad batch size");
    if (nx == 1) {
        for (int r = 0; r < b.count; ++r) {
            size_t n = (size_t)3 * b.d[r].nz * b.d[r].ny;
            DM_LAUNCH(x_copy_inverse_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                      s, b.d[r].S1, b.d[r].H, n);
        }
        DM_CHECK_LAUNCH();
        return DEMAG_OK;
    }
    if (periodic) {
        if (mf) return fail(DEMAG_EUNSUPPORTED, "x stage: periodic transforms are FP32 only");
        switch (nx) {
#define CASE(Lv)                                                                                  \
    case Lv: {                                                                                    \
        constexpr int L = Lv;                                                                     \
        constexpr int TY = XTile<L, 1, true>::TY;                                                  \
        b.start[0] = 0;                                                                           \
        for (int r = 0; r < b.count; ++r)                                                         \
            b.start[r + 1] = b.start[r] + ((b.d[r].ny + TY - 1) / TY) * b.d[r].nz * 3;           \
        DM_LAUNCH((x_inverse_kernel<L, TY, 0, true>), dim3((unsigned)finish_batch(b)),           \
                  dim3(NT), 0, s, b, tw);                                                        \
        break;                                                                                    \
    }
            DM_POW2_CASES(CASE)
#undef CASE
            default: return fail(DEMAG_EUNSUPPORTED, "x stage: unsupported nx");
        }
        DM_CHECK_LAUNCH();
        return DEMAG_OK;
    }
    if (!is_pow2c(nx)) {
        if (mf) return fail(DEMAG_EUNSUPPORTED, "x stage: mixed-radix transforms are FP32 only");
        switch (nx) {
#define CASE(Lv)                                                                                  \
    case Lv: {                                                                                    \
        constexpr int L = Lv;                                                                     \
        constexpr int TY = XTile<L, 1, true>::TY;                                                  \
        b.start[0] = 0;                                                                           \
        for (int r = 0; r < b.count; ++r)                                                         \
            b.start[r + 1] = b.start[r] + ((b.d[r].ny + TY - 1) / TY) * b.d[r].nz * 3;           \
        DM_LAUNCH((x_inverse_kernel<L, TY, 0, false>), dim3((unsigned)finish_batch(b)),          \
                  dim3(NT), 0, s, b, tw);                                                        \
        break;                                                                                    \
    }
            DM_MIXED_CASES(CASE)
#undef CASE
            default: return fail(DEMAG_EUNSUPPORTED, "x stage: unsupported nx");
        }
        DM_CHECK_LAUNCH();
        return DEMAG_OK;
    }
    switch (nx) {
#define BODY(V)                                                                               \
    {                                                                                         \
        constexpr int TY = XTile<L, V, true>::TY;                                             \
        constexpr int TYR = XRegTile<L, V>::TY;                                               \
        const bool reg = V >= 1 && mf == 0 && npasses(L) >= 2;                                \
        const int ty = reg ? TYR : TY;                                                        \
        b.start[0] = 0;                                                                       \
        for (int r = 0; r < b.count; ++r)                                                     \
            b.start[r + 1] = b.start[r] + ((b.d[r].ny + ty - 1) / ty) * b.d[r].nz * 3;       \
        if constexpr (V >= 1 && npasses(L) >= 2) {                                            \
            if (reg) {                                                                        \
                DM_LAUNCH((x_inverse_reg_kernel<L, TYR>),                                     \
                          dim3((unsigned)finish_batch(b)), dim3(NT), 0, s, b, tw);            \
                break;                                                                        \
            }                                                                                 \
        }                                                                                     \
        DM_MF_DISPATCH(V, DM_LAUNCH((x_inverse_kernel<L, TY, MFv>),                           \
                  dim3((unsigned)finish_batch(b)), dim3(NT), 0, s, b, tw);)                   \
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


}  // namespace dm
