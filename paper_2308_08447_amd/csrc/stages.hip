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

// ============================================================================ x
// One block: component c, plane z, rows y0 .. y0+TY-1 (TY/2 packed pairs).
template <int L, int TY>
__global__ __launch_bounds__(NT) void x_forward_kernel(const float* __restrict__ M,
                                                       float2* __restrict__ S1, int ny, int nz,
                                                       float scale,
                                                       const float2* __restrict__ tw_all) {
    constexpr int NP = TY / 2;
    constexpr int LS = lpad_c(L);
    constexpr int PER = (NP * L + NT - 1) / NT;
    __shared__ float2 buf[NP * LS];
    const float2* twL = tw_all + L;
    const float2* tw2L = tw_all + 2 * L;
    const int tid = threadIdx.x;
    const int y0 = blockIdx.x * TY, z = blockIdx.y, c = blockIdx.z;
    const int rows = min(TY, ny - y0);
    const float* src = M + ((size_t)(c * nz + z) * ny + y0) * L;
    float2* dst = S1 + (size_t)(c * nz + z) * (L + 1) * ny + y0;

    float2 zr[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int e = tid + q * NT;
        if (e < NP * L) {
            int p = e / L, t = e - p * L;
            float a = (2 * p < rows) ? src[(size_t)(2 * p) * L + t] : 0.f;
            float b = (2 * p + 1 < rows) ? src[(size_t)(2 * p + 1) * L + t] : 0.f;
            zr[q] = make_float2(a * scale, b * scale);
            buf[p * LS + lpad(t)] = zr[q];
        }
    }
    __syncthreads();
    lds_fft<L, -1, NP, NT, RowLines<LS>>(buf, twL);

    // even frequencies kx = 2m, m = 0..L/2: Z[2m] = E[m], Z[2L-2m] = E[(L-m) mod L]
    for (int it = tid; it < (L / 2 + 1) * NP; it += NT) {
        int p = it % NP, m = it / NP;
        float2 Zk = buf[p * LS + lpad(m)];
        float2 Zn = cconj(buf[p * LS + lpad((L - m) & (L - 1))]);
        float2 Xa = cscale(cadd(Zk, Zn), 0.5f);
        float2 d = csub(Zk, Zn);
        float2 Xb = make_float2(0.5f * d.y, -0.5f * d.x);
        size_t o = (size_t)(2 * m) * ny + 2 * p;
        if (2 * p < rows) dst[o] = Xa;
        if (2 * p + 1 < rows) dst[o + 1] = Xb;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int e = tid + q * NT;
        if (e < NP * L) {
            int p = e / L, t = e - p * L;
            buf[p * LS + lpad(t)] = cmul(zr[q], tw2L[t]);
        }
    }
    __syncthreads();
    lds_fft<L, -1, NP, NT, RowLines<LS>>(buf, twL);
    // odd frequencies kx = 2m+1, m < L/2: Z[2m+1] = O[m], Z[2L-2m-1] = O[L-1-m]
    for (int it = tid; it < (L / 2) * NP; it += NT) {
        int p = it % NP, m = it / NP;
        float2 Zk = buf[p * LS + lpad(m)];
        float2 Zn = cconj(buf[p * LS + lpad(L - 1 - m)]);
        float2 Xa = cscale(cadd(Zk, Zn), 0.5f);
        float2 d = csub(Zk, Zn);
        float2 Xb = make_float2(0.5f * d.y, -0.5f * d.x);
        size_t o = (size_t)(2 * m + 1) * ny + 2 * p;
        if (2 * p < rows) dst[o] = Xa;
        if (2 * p + 1 < rows) dst[o + 1] = Xb;
    }
}

template <int L, int TY>
__global__ __launch_bounds__(NT) void x_inverse_kernel(const float2* __restrict__ S1,
                                                       float* __restrict__ H, int ny, int nz,
                                                       const float2* __restrict__ tw_all) {
    constexpr int NP = TY / 2;
    constexpr int LS = lpad_c(L);
    constexpr int PER = (NP * L + NT - 1) / NT;
    __shared__ float2 buf[NP * LS];
    const float2* twL = tw_all + L;
    const float2* tw2L = tw_all + 2 * L;
    const int tid = threadIdx.x;
    const int y0 = blockIdx.x * TY, z = blockIdx.y, c = blockIdx.z;
    const int rows = min(TY, ny - y0);
    const float2* src = S1 + (size_t)(c * nz + z) * (L + 1) * ny + y0;
    float* dst = H + ((size_t)(c * nz + z) * ny + y0) * L;

    // Z[k] = Xa[k] + i Xb[k]; for k > L use Hermitian symmetry X[2L-k] = conj(X[k]).
    // The DC and Nyquist bins of a real row are real: their imaginary parts are dropped.
    // Even inputs Z[2m] -> line p, slot m.
    for (int it = tid; it < (L / 2 + 1) * NP; it += NT) {
        int p = it % NP, m = it / NP, kx = 2 * m;
        size_t o = (size_t)kx * ny + 2 * p;
        float2 Xa = (2 * p < rows) ? src[o] : make_float2(0.f, 0.f);
        float2 Xb = (2 * p + 1 < rows) ? src[o + 1] : make_float2(0.f, 0.f);
        if (kx == 0 || kx == L) {
            Xa.y = 0.f;
            Xb.y = 0.f;
        }
        buf[p * LS + lpad(m)] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);
        if (kx > 0 && kx < L) buf[p * LS + lpad(L - m)] = make_float2(Xa.x + Xb.y, Xb.x - Xa.y);
    }
    __syncthreads();
    lds_fft<L, +1, NP, NT, RowLines<LS>>(buf, twL);
    float2 ie[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int e = tid + q * NT;
        if (e < NP * L) {
            int p = e / L, t = e - p * L;
            ie[q] = buf[p * LS + lpad(t)];
        }
    }
    __syncthreads();
    // Odd inputs Z[2m+1]: kx = 2m+1 < L direct, and Z[2L-kx] = conj -> slot L-1-m.
    for (int it = tid; it < (L / 2) * NP; it += NT) {
        int p = it % NP, m = it / NP, kx = 2 * m + 1;
        size_t o = (size_t)kx * ny + 2 * p;
        float2 Xa = (2 * p < rows) ? src[o] : make_float2(0.f, 0.f);
        float2 Xb = (2 * p + 1 < rows) ? src[o + 1] : make_float2(0.f, 0.f);
        buf[p * LS + lpad(m)] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);
        buf[p * LS + lpad(L - 1 - m)] = make_float2(Xa.x + Xb.y, Xb.x - Xa.y);
    }
    __syncthreads();
    lds_fft<L, +1, NP, NT, RowLines<LS>>(buf, twL);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int e = tid + q * NT;
        if (e < NP * L) {
            int p = e / L, t = e - p * L;
            float2 zz = cadd(ie[q], cmul(cconj(tw2L[t]), buf[p * LS + lpad(t)]));
            if (2 * p < rows) dst[(size_t)(2 * p) * L + t] = zz.x;
            if (2 * p + 1 < rows) dst[(size_t)(2 * p + 1) * L + t] = zz.y;
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

// ============================================================================ y
// One block: LPB lines (consecutive kx) of one (c, z) plane; lines [0, LPB) of
// LDS hold the even-output halves, [LPB, 2 LPB) the odd-output halves.
template <int L, int LPB>
__global__ __launch_bounds__(NT) void y_forward_kernel(const float2* __restrict__ S1,
                                                       float2* __restrict__ S2, int X1, int nz,
                                                       const float2* __restrict__ tw_all) {
    constexpr int LS = lpad_c(L);
    __shared__ float2 buf[2 * LPB * LS];
    const float2* twL = tw_all + L;
    const float2* tw2L = tw_all + 2 * L;
    const int tid = threadIdx.x;
    const int kx0 = blockIdx.x * LPB, z = blockIdx.y, c = blockIdx.z;
    const size_t plane = (size_t)(c * nz + z) * X1;
    for (int it = tid; it < LPB * L; it += NT) {
        int l = it / L, t = it - l * L, kx = kx0 + l;
        float2 v = (kx < X1) ? S1[(plane + kx) * L + t] : make_float2(0.f, 0.f);
        buf[l * LS + lpad(t)] = v;
        buf[(LPB + l) * LS + lpad(t)] = cmul(v, tw2L[t]);
    }
    __syncthreads();
    lds_fft<L, -1, 2 * LPB, NT, RowLines<LS>>(buf, twL);
    for (int it = tid; it < LPB * L; it += NT) {
        int l = it / L, m = it - l * L, kx = kx0 + l;
        if (kx < X1) {
            float2 e = buf[l * LS + lpad(m)], o = buf[(LPB + l) * LS + lpad(m)];
            float4* d = reinterpret_cast<float4*>(S2 + (plane + kx) * (2 * L)) + m;
            *d = make_float4(e.x, e.y, o.x, o.y);
        }
    }
}

template <int L, int LPB>
__global__ __launch_bounds__(NT) void y_inverse_kernel(const float2* __restrict__ S2,
                                                       float2* __restrict__ S1, int X1, int nz,
                                                       const float2* __restrict__ tw_all) {
    constexpr int LS = lpad_c(L);
    __shared__ float2 buf[2 * LPB * LS];
    const float2* twL = tw_all + L;
    const float2* tw2L = tw_all + 2 * L;
    const int tid = threadIdx.x;
    const int kx0 = blockIdx.x * LPB, z = blockIdx.y, c = blockIdx.z;
    const size_t plane = (size_t)(c * nz + z) * X1;
    for (int it = tid; it < LPB * L; it += NT) {
        int l = it / L, m = it - l * L, kx = kx0 + l;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (kx < X1) v = reinterpret_cast<const float4*>(S2 + (plane + kx) * (2 * L))[m];
        buf[l * LS + lpad(m)] = make_float2(v.x, v.y);
        buf[(LPB + l) * LS + lpad(m)] = make_float2(v.z, v.w);
    }
    __syncthreads();
    lds_fft<L, +1, 2 * LPB, NT, RowLines<LS>>(buf, twL);
    for (int it = tid; it < LPB * L; it += NT) {
        int l = it / L, t = it - l * L, kx = kx0 + l;
        if (kx < X1) {
            float2 e = buf[l * LS + lpad(t)], o = buf[(LPB + l) * LS + lpad(t)];
            S1[(plane + kx) * L + t] = cadd(e, cmul(cconj(tw2L[t]), o));
        }
    }
}

// ============================================================================ z
// One block: TK consecutive ky of one kx, all stored z planes, 3 components.
// LDS element (z, c, t) at z * 3TK + c * TK + t: 3TK interleaved lines of length NZ.
template <int NZ, int TK>
__global__ __launch_bounds__(NT) void z_convolve_kernel(float2* __restrict__ S2,
                                                        const float* __restrict__ K, int nz,
                                                        int X1, int Ny, int Y1, int Z1,
                                                        const float2* __restrict__ tw_all) {
    constexpr int NLN = 3 * TK;
    __shared__ float2 buf[NZ * NLN];
    const float2* twZ = tw_all + NZ;
    const int tid = threadIdx.x;
    const int ky0 = blockIdx.x * TK, kx = blockIdx.y;
    const size_t P = (size_t)X1 * Ny;  // complex elements per z plane
    const size_t cstride = (size_t)nz * P;
    float2* col = S2 + (size_t)kx * Ny + ky0;

    for (int it = tid; it < 3 * NZ * TK; it += NT) {
        int t = it % TK, rest = it / TK, zz = rest % NZ, c = rest / NZ;
        float2 v = make_float2(0.f, 0.f);
        if (zz < nz && ky0 + t < Ny) v = col[c * cstride + zz * P + t];
        buf[zz * NLN + c * TK + t] = v;
    }
    __syncthreads();
    lds_fft<NZ, -1, NLN, NT, ColLines<NLN>>(buf, twZ);

    const size_t kc = (size_t)Z1 * X1 * Y1;  // floats per K component
    for (int it = tid; it < NZ * TK; it += NT) {
        int t = it % TK, kz = it / TK, ky = ky0 + t;
        if (ky >= Ny) continue;
        int kyf = ky, kzf = kz;
        float sy = 1.f, sz = 1.f;
        if (2 * ky > Ny) { kyf = Ny - ky; sy = -1.f; }
        if (2 * kz > NZ) { kzf = NZ - kz; sz = -1.f; }
        const float* k0 = K + ((size_t)kzf * X1 + kx) * Y1 + kyf;
        float kxx = k0[0], kyy = k0[kc], kzz = k0[2 * kc];
        float kxy = sy * k0[3 * kc], kxz = sz * k0[4 * kc], kyz = sy * sz * k0[5 * kc];
        float2* p = buf + kz * NLN + t;
        float2 mx = p[0], my = p[TK], mz = p[2 * TK];
        p[0] = make_float2(kxx * mx.x + kxy * my.x + kxz * mz.x, kxx * mx.y + kxy * my.y + kxz * mz.y);
        p[TK] = make_float2(kxy * mx.x + kyy * my.x + kyz * mz.x, kxy * mx.y + kyy * my.y + kyz * mz.y);
        p[2 * TK] = make_float2(kxz * mx.x + kyz * my.x + kzz * mz.x, kxz * mx.y + kyz * my.y + kzz * mz.y);
    }
    __syncthreads();
    lds_fft<NZ, +1, NLN, NT, ColLines<NLN>>(buf, twZ);

    for (int it = tid; it < 3 * nz * TK; it += NT) {
        int t = it % TK, rest = it / TK, zz = rest % nz, c = rest / nz;
        if (ky0 + t < Ny) col[c * cstride + zz * P + t] = buf[zz * NLN + c * TK + t];
    }
}

// ============================================================================ launchers
namespace {

constexpr int x_rows(int L) { return L >= 2048 ? 8 : 16; }
constexpr int y_lines(int L) { return L >= 2048 ? 1 : 2048 / L; }
constexpr int z_tile(int NZ) { return NZ >= 128 ? 16 : (2048 / NZ > 64 ? 64 : 2048 / NZ); }

}  // namespace

#define DM_POW2_CASES(MACRO) \
    MACRO(2) MACRO(4) MACRO(8) MACRO(16) MACRO(32) MACRO(64) MACRO(128) MACRO(256) MACRO(512) \
    MACRO(1024) MACRO(2048)

int launch_x_forward(const StageArgs& a, const float* M, float scale) {
    const Geometry& g = *a.g;
    if (g.nx == 1) {
        size_t n = (size_t)3 * g.nz * g.ny;
        hipLaunchKernelGGL(x_copy_forward_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           a.stream, M, a.S1, n, scale);
        DM_CHECK_LAUNCH();
        return DEMAG_OK;
    }
    switch (g.nx) {
#define CASE(L)                                                                              \
    case L: {                                                                                \
        constexpr int TY = x_rows(L);                                                        \
        dim3 grid((g.ny + TY - 1) / TY, g.nz, 3);                                            \
        hipLaunchKernelGGL((x_forward_kernel<L, TY>), grid, dim3(NT), 0, a.stream, M, a.S1, \
                           g.ny, g.nz, scale, a.tw_all);                                     \
        break;                                                                               \
    }
        DM_POW2_CASES(CASE)
#undef CASE
        default: return fail(DEMAG_EUNSUPPORTED, "x stage: unsupported nx");
    }
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

int launch_x_inverse(const StageArgs& a, float* H) {
    const Geometry& g = *a.g;
    if (g.nx == 1) {
        size_t n = (size_t)3 * g.nz * g.ny;
        hipLaunchKernelGGL(x_copy_inverse_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           a.stream, a.S1, H, n);
        DM_CHECK_LAUNCH();
        return DEMAG_OK;
    }
    switch (g.nx) {
#define CASE(L)                                                                              \
    case L: {                                                                                \
        constexpr int TY = x_rows(L);                                                        \
        dim3 grid((g.ny + TY - 1) / TY, g.nz, 3);                                            \
        hipLaunchKernelGGL((x_inverse_kernel<L, TY>), grid, dim3(NT), 0, a.stream, a.S1, H, \
                           g.ny, g.nz, a.tw_all);                                            \
        break;                                                                               \
    }
        DM_POW2_CASES(CASE)
#undef CASE
        default: return fail(DEMAG_EUNSUPPORTED, "x stage: unsupported nx");
    }
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

int launch_y_forward(const StageArgs& a) {
    const Geometry& g = *a.g;
    if (g.ny == 1) return DEMAG_OK;  // S2 aliases S1
    switch (g.ny) {
#define CASE(L)                                                                                \
    case L: {                                                                                  \
        constexpr int LPB = y_lines(L);                                                        \
        dim3 grid((g.X1 + LPB - 1) / LPB, g.nz, 3);                                            \
        hipLaunchKernelGGL((y_forward_kernel<L, LPB>), grid, dim3(NT), 0, a.stream, a.S1, a.S2, \
                           g.X1, g.nz, a.tw_all);                                              \
        break;                                                                                 \
    }
        DM_POW2_CASES(CASE)
#undef CASE
        default: return fail(DEMAG_EUNSUPPORTED, "y stage: unsupported ny");
    }
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

int launch_y_inverse(const StageArgs& a) {
    const Geometry& g = *a.g;
    if (g.ny == 1) return DEMAG_OK;
    switch (g.ny) {
#define CASE(L)                                                                                \
    case L: {                                                                                  \
        constexpr int LPB = y_lines(L);                                                        \
        dim3 grid((g.X1 + LPB - 1) / LPB, g.nz, 3);                                            \
        hipLaunchKernelGGL((y_inverse_kernel<L, LPB>), grid, dim3(NT), 0, a.stream, a.S2, a.S1, \
                           g.X1, g.nz, a.tw_all);                                              \
        break;                                                                                 \
    }
        DM_POW2_CASES(CASE)
#undef CASE
        default: return fail(DEMAG_EUNSUPPORTED, "y stage: unsupported ny");
    }
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

int launch_z_convolve(const StageArgs& a) {
    const Geometry& g = *a.g;
    switch (g.Nz) {
#define CASE(NZv)                                                                             \
    case NZv: {                                                                               \
        constexpr int TK = z_tile(NZv);                                                       \
        dim3 grid((g.Ny + TK - 1) / TK, g.X1);                                                \
        hipLaunchKernelGGL((z_convolve_kernel<NZv, TK>), grid, dim3(NT), 0, a.stream, a.S2, a.K, \
                           g.nz, g.X1, g.Ny, g.Y1, g.Z1, a.tw_all);                           \
        break;                                                                                \
    }
        CASE(1) CASE(4) CASE(8) CASE(16) CASE(32) CASE(64) CASE(128) CASE(256)
#undef CASE
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
