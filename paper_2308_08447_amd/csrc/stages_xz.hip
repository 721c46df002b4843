// stages_xz.hip -- the three-kernel form of the convolution for thin meshes
// (n_z <= 16, n_y <= 512, 32 <= n_x <= 1024).
//
// The z transform moves into the x kernels, where the n_z rows of one (c, y)
// line of cells are all in hand:
//   xz forward   M[3][nz][ny][nx] (f32)  -> T: x R2C of every row, then per kx a
//                length-Nz z FFT in registers (the upper nz inputs are zero)
//   y conv       T in place: per (kz, kx) column a length-Ny y FFT, H^ = K M^
//                (6 real symmetric components), a truncated y IFFT
//   xz inverse   T -> H: per kx the truncated z IFFT in registers, then the x
//                C2R of every row pair, first nx outputs stored
// Every element of T is read and written once per evaluation by each kernel;
// compared with the five-pass order (x, y, z, y^-1, x^-1) the spectra cross HBM
// three times instead of five, at the price of T holding all Nz planes.
//
// T layout: [3][Nz][G][ny][4] complex, G = ceil((nx+1)/4): column kx of plane
// (c, kz) is group kx/4, slot kx%4, so one y column of four consecutive kx is a
// contiguous 32 ny bytes (the y kernel's loads), and the x kernels move each
// (y, kx pair) as one 16-byte access.
#include "stage_common.h"

namespace dm {

constexpr int TKB = 4;  // kx columns per T group

template <int L>
struct XZShape {
    static constexpr int NTA = L / 2 < 64 ? 64 : L / 2;   // thread t owns kx = 2t, 2t+1
    static constexpr int L2 = 2 * L;                      // padded x length
    static constexpr int LS = lpad_c(L2) + 1;
};

template <int NZS>
struct ZShape {
    static constexpr int NZ = NZS > 1 ? 2 * NZS : 1;      // padded z length
    static constexpr int NPAIR = NZS > 1 ? NZS / 2 : 1;   // packed row pairs
};

template <int L, int NZS>
struct XZRounds {
    static constexpr int CAP = 2048 / L > 0 ? 2048 / L : 1;
    static constexpr int NPR = ZShape<NZS>::NPAIR < CAP ? ZShape<NZS>::NPAIR : CAP;  // pairs per round
    static constexpr int NR = ZShape<NZS>::NPAIR / NPR;
};

template <int NTHR>
__device__ __forceinline__ void stage_table_n(float2* dst, const float2* __restrict__ src, int n) {
    for (int i = threadIdx.x; i < n; i += NTHR) dst[i] = src[i];
}

__device__ __forceinline__ size_t t_index(int c, int kz, int NZ, int G, int ny, int kx, int y) {
    return ((((size_t)c * NZ + kz) * G + kx / TKB) * ny + y) * TKB + kx % TKB;
}

// ============================================================================ xz forward
template <int L, int NZS>
__global__ __launch_bounds__(XZShape<L>::NTA) void xz_forward_kernel(const XZBatch b,
                                                                   const float2* __restrict__ tw_all) {
    using S = XZShape<L>;
    using Z = ZShape<NZS>;
    using RR = XZRounds<L, NZS>;
    constexpr int NTA = S::NTA, L2 = S::L2, LS = S::LS, NZ = Z::NZ, NPR = RR::NPR;
    __shared__ float2 buf[NPR * LS];
    __shared__ float2 tw2[L2];
    __shared__ float2 nyq[2 * Z::NPAIR];
    stage_table_n<NTA>(tw2, tw_all + tw_offset(L2), L2);
    const int t = threadIdx.x;
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    const int ny = b.d[item].ny;
    const float scale = b.d[item].scale;
    const int id = gid - b.start[item];
    const int y = id % ny, c = id / ny;
    const int G = (L + 1 + TKB - 1) / TKB;
    const float* __restrict__ rows = b.d[item].M + ((size_t)c * NZS * ny + y) * L;  // row z at + z ny L
    float2* __restrict__ T = b.d[item].T;
    const bool owner = t < L / 2;

    float2 col[2][NZS];  // x spectra of the two owned kx columns, rows 0..nz-1
#pragma unroll
    for (int rd = 0; rd < RR::NR; ++rd) {
        // pair p of this round packs rows 2(rd NPR + p) and 2(rd NPR + p) + 1 as a + i b
        auto src = [&](int p, int i) {
            const int z0 = 2 * (rd * NPR + p);
            float a = rows[(size_t)z0 * ny * L + i];
            float bb = (z0 + 1 < NZS) ? rows[(size_t)(z0 + 1) * ny * L + i] : 0.f;
            return make_float2(a * scale, bb * scale);
        };
        auto to_lds = [&](int p, int k, float2 v) { buf[p * LS + lpad(k)] = v; };
        fft_io<L2, -1, NPR, NTA, RowLines<LS>, true, false, true>(buf, tw2, src, to_lds);
        __syncthreads();
        // Hermitian separation: X_a[k] = (Z[k] + conj Z[2L-k]) / 2, X_b[k] = (Z[k] - conj Z[2L-k]) / 2i
#pragma unroll
        for (int p = 0; p < NPR; ++p) {
            const int z0 = 2 * (rd * NPR + p);
            if (owner) {
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const int kx = 2 * t + s;
                    float2 Zk = buf[p * LS + lpad(kx)];
                    float2 Zn = cconj(buf[p * LS + lpad((L2 - kx) & (L2 - 1))]);
                    float2 d = csub(Zk, Zn);
                    col[s][z0] = cscale(cadd(Zk, Zn), 0.5f);
                    if (z0 + 1 < NZS) col[s][z0 + 1] = make_float2(0.5f * d.y, -0.5f * d.x);
                }
            }
            if (t == 0) {  // kx = L: Z[L] and conj Z[L]
                float2 Zk = buf[p * LS + lpad(L)];
                nyq[z0] = make_float2(Zk.x, 0.f);
                if (z0 + 1 < NZS) nyq[z0 + 1] = make_float2(Zk.y, 0.f);
            }
        }
        __syncthreads();
    }

    // z: length-NZ transform of the NZS stored rows (upper half zero):
    // Y[2m] = DFT(x)[m], Y[2m+1] = DFT(x W_NZ^z)[m]
    const float2* twz = tw_all + tw_offset(NZ);
    if (owner) {
        float2 Y[2][NZ];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if constexpr (NZS == 1) {
                Y[s][0] = col[s][0];
            } else {
                float2 e[NZS], o[NZS];
#pragma unroll
                for (int z = 0; z < NZS; ++z) {
                    e[z] = col[s][z];
                    o[z] = z == 0 ? col[s][0] : cmul(col[s][z], twz[z]);
                }
                dft<NZS, -1>(e);
                dft<NZS, -1>(o);
#pragma unroll
                for (int m = 0; m < NZS; ++m) {
                    Y[s][2 * m] = e[m];
                    Y[s][2 * m + 1] = o[m];
                }
            }
        }
#pragma unroll
        for (int kz = 0; kz < NZ; ++kz) {
            float2* d = T + t_index(c, kz, NZ, G, ny, 2 * t, y);
            *reinterpret_cast<float4*>(d) = make_float4(Y[0][kz].x, Y[0][kz].y, Y[1][kz].x, Y[1][kz].y);
        }
    }
    // kx = L (real rows: its spectrum is real): direct length-NZ DFT, one output per thread
    if (t < NZ) {
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int z = 0; z < NZS; ++z) acc = cadd(acc, cscale(twz[(t * z) & (NZ - 1)], nyq[z].x));
        T[t_index(c, t, NZ, G, ny, L, y)] = acc;
    }
}

// ============================================================================ y convolution
// One block: plane kz, column kx (ny <= 128; longer columns take
// yconv_reg_kernel below).  Its three component lines (length LNY = 2 ny,
// upper half zero) are transformed together in LDS, multiplied there by the
// tensor (each folded value K(kz, kx, f) serves ky = f and its mirror LNY - f),
// and inverse transformed, keeping the first ny outputs.  The column's T
// elements are one 8-byte slot of each 32-byte (y, group) chunk; the blocks of
// the group's other three columns are neighbours in the grid and run on the
// same XCD, so the chunks are fetched from HBM once and shared through L2.
template <int LNY, int NZ>
__global__ __launch_bounds__(NT) void yconv_kernel(const YCBatch b, const float2* __restrict__ tw_all) {
    constexpr int NY = LNY / 2;
    constexpr int LS = lpad_c(LNY);
    using Rows = RowLines<LS>;
    __shared__ float2 buf[3 * LS];
    __shared__ float2 tw[LNY];
    stage_table(tw, tw_all + tw_offset(LNY), LNY);
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    const YCDesc& d = b.d[item];
    const int X1 = d.X1, Y1 = d.Y1, Z1 = d.Z1, G = d.G;
    const int id = gid - b.start[item];
    // Planes kz and NZ - kz share the folded tensor column: their blocks are
    // adjacent in the grid (same XCD, same moment), so the column is fetched
    // from HBM once; pair j = 0 holds the two self-mirrored planes 0 and NZ/2.
    int kx, kz;
    if constexpr (NZ == 1) {
        kx = id;
        kz = 0;
    } else {
        const int member = id & 1, t = id >> 1, j = t / X1;
        kx = t - j * X1;
        kz = j == 0 ? (member ? NZ / 2 : 0) : (member ? NZ - j : j);
    }
    const size_t cstride = (size_t)NZ * G * NY * TKB;  // complex elements per component
    float2* __restrict__ col = d.T + (((size_t)kz * G + kx / TKB) * NY) * TKB + kx % TKB;

    // The column's folded tensor values are loaded first, so that their latency
    // overlaps the forward transform: slot s of a thread holds f = tid + s NT.
    // K folded: ky > ny flips xy and yz, kz > nz flips xz and yz.
    const int kzf = 2 * kz > NZ ? NZ - kz : kz;
    const float sz = 2 * kz > NZ ? -1.f : 1.f;
    const size_t KC = (size_t)Z1 * X1 * Y1;
    const float* kp = d.K + ((size_t)kzf * X1 + kx) * Y1;
    constexpr int NKS = (NY + 1 + NT - 1) / NT;
    float kv[NKS][6];
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
        const int f = threadIdx.x + s * NT;
#pragma unroll
        for (int a = 0; a < 6; ++a) kv[s][a] = f <= NY ? kp[a * KC + f] : 0.f;
    }

    auto src = [&](int c, int yy) { return col[c * cstride + (size_t)yy * TKB]; };
    auto to_lds = [&](int c, int k, float2 v) { buf[c * LS + lpad(k)] = v; };
    fft_io<LNY, -1, 3, NT, Rows, true, false, true>(buf, tw, src, to_lds);
    __syncthreads();

    // H^_a = sum_b K_ab M^_b; each folded value serves ky = f and its mirror LNY - f
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
        const int f = threadIdx.x + s * NT;
        if (f > NY) continue;
        const float kxx = kv[s][0], kyy = kv[s][1], kzz = kv[s][2];
        const float kxy0 = kv[s][3], kxz = sz * kv[s][4], kyz0 = sz * kv[s][5];
        auto apply = [&](int ky, float sy) {
            const float kxy = sy * kxy0, kyz = sy * kyz0;
            float2 mx = buf[lpad(ky)], my = buf[LS + lpad(ky)], mz = buf[2 * LS + lpad(ky)];
            auto dot3 = [](float a, float x, float bb, float yv, float cc, float zv) {
                return fmaf(cc, zv, fmaf(bb, yv, a * x));
            };
            buf[lpad(ky)] = make_float2(dot3(kxx, mx.x, kxy, my.x, kxz, mz.x), dot3(kxx, mx.y, kxy, my.y, kxz, mz.y));
            buf[LS + lpad(ky)] = make_float2(dot3(kxy, mx.x, kyy, my.x, kyz, mz.x), dot3(kxy, mx.y, kyy, my.y, kyz, mz.y));
            buf[2 * LS + lpad(ky)] = make_float2(dot3(kxz, mx.x, kyz, my.x, kzz, mz.x), dot3(kxz, mx.y, kyz, my.y, kzz, mz.y));
        };
        apply(f, 1.f);
        if (f > 0 && f < NY) apply(LNY - f, -1.f);
    }
    __syncthreads();

    auto from_lds = [&](int c, int i) { return buf[c * LS + lpad(i)]; };
    auto sink = [&](int c, int yy, float2 v) { col[c * cstride + (size_t)yy * TKB] = v; };
    fft_io<LNY, +1, 3, NT, Rows, false, true, true>(buf, tw, from_lds, sink);
}

// Same column work for LNY = 2 NT R (ny = 256, 512), with the radices ordered so
// that the tensor product runs in registers: forward passes 16, 16, R and
// inverse passes R, 16, 16.  After the forward last pass thread j holds
// k = j + NT r (r < R) of all three component lines, which is exactly the input
// set of butterfly j of the inverse first pass; the product sits between the
// two in registers, with no LDS round trip.
template <int LNY, int NZ>
__global__ __launch_bounds__(NT) void yconv_reg_kernel(const YCBatch b, const float2* __restrict__ tw_all) {
    constexpr int NY = LNY / 2;
    constexpr int R = LNY / 256;
    static_assert(R >= 2 && LNY / R == NT, "thread j owns k = j + NT r of the three lines");
    constexpr int LS = lpad_c(LNY);
    using Rows = RowLines<LS>;
    __shared__ float2 buf[3 * LS];
    // twiddles as coarse x fine products (Tw2): 26.6 KB of LDS per block, so
    // five blocks share a compute unit instead of four
    __shared__ float2 twt[tw2_entries(LNY)];
    const Tw2 tw = stage_tw2<LNY, NT>(twt, tw_all + tw_offset(LNY));
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    const YCDesc& d = b.d[item];
    const int X1 = d.X1, Y1 = d.Y1, Z1 = d.Z1, G = d.G;
    const int id = gid - b.start[item];
    int kx, kz;
    if constexpr (NZ == 1) {
        kx = id;
        kz = 0;
    } else {
        const int member = id & 1, t = id >> 1, jj = t / X1;
        kx = t - jj * X1;
        kz = jj == 0 ? (member ? NZ / 2 : 0) : (member ? NZ - jj : jj);
    }
    const size_t cstride = (size_t)NZ * G * NY * TKB;
    float2* __restrict__ col = d.T + (((size_t)kz * G + kx / TKB) * NY) * TKB + kx % TKB;
    const int j = threadIdx.x;

    // tensor values of the thread's k = j + NT r, folded to f = min(k, LNY - k)
    const int kzf = 2 * kz > NZ ? NZ - kz : kz;
    const float sz = 2 * kz > NZ ? -1.f : 1.f;
    const size_t KC = (size_t)Z1 * X1 * Y1;
    const float* kp = d.K + ((size_t)kzf * X1 + kx) * Y1;
    float kv[R][6], sy[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int k = j + NT * r;
        const int f = k <= NY ? k : LNY - k;
        sy[r] = k <= NY ? 1.f : -1.f;
#pragma unroll
        for (int a = 0; a < 6; ++a) kv[r][a] = kp[a * KC + f];
    }

    auto src = [&](int c, int yy) { return col[c * cstride + (size_t)yy * TKB]; };
    first_pass<LNY, 16, -1, 3, NT, Rows, true, false, true>(buf, src);
    stockham_pass<LNY, 16, 16, -1, 3, NT, Rows>(buf, tw);
    float2 v[3][R];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[c][r] = buf[c * LS + lpad(j + NT * r)];
#pragma unroll
        for (int r = 1; r < R; ++r) v[c][r] = cmul(v[c][r], tw[j * r]);
        dft<R, -1>(v[c]);
    }
    // H^_a = sum_b K_ab M^_b at k = j + NT r
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float kxx = kv[r][0], kyy = kv[r][1], kzz = kv[r][2];
        const float kxy = sy[r] * kv[r][3], kxz = sz * kv[r][4], kyz = sy[r] * sz * kv[r][5];
        const float2 mx = v[0][r], my = v[1][r], mz = v[2][r];
        auto dot3 = [](float a, float x, float bb, float yv, float cc, float zv) {
            return fmaf(cc, zv, fmaf(bb, yv, a * x));
        };
        v[0][r] = make_float2(dot3(kxx, mx.x, kxy, my.x, kxz, mz.x), dot3(kxx, mx.y, kxy, my.y, kxz, mz.y));
        v[1][r] = make_float2(dot3(kxy, mx.x, kyy, my.x, kyz, mz.x), dot3(kxy, mx.y, kyy, my.y, kyz, mz.y));
        v[2][r] = make_float2(dot3(kxz, mx.x, kyz, my.x, kzz, mz.x), dot3(kxz, mx.y, kyz, my.y, kzz, mz.y));
    }
    // inverse first pass (radix R, sub-size 1: no twiddles), Stockham order j R + r
#pragma unroll
    for (int c = 0; c < 3; ++c) dft<R, +1>(v[c]);
    __syncthreads();   // every thread has read its forward inputs
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < R; ++r) buf[c * LS + lpad(j * R + r)] = v[c][r];
    __syncthreads();
    stockham_pass<LNY, 16, R, +1, 3, NT, Rows>(buf, tw);
    auto sink = [&](int c, int yy, float2 val) { col[c * cstride + (size_t)yy * TKB] = val; };
    last_pass<LNY, 16, +1, 3, NT, Rows, true, false>(buf, tw, sink);
}

// ============================================================================ xz inverse
template <int L, int NZS>
__global__ __launch_bounds__(XZShape<L>::NTA) void xz_inverse_kernel(const XZBatch b,
                                                                   const float2* __restrict__ tw_all) {
    using S = XZShape<L>;
    using Z = ZShape<NZS>;
    using RR = XZRounds<L, NZS>;
    constexpr int NTA = S::NTA, L2 = S::L2, LS = S::LS, NZ = Z::NZ, NPR = RR::NPR;
    __shared__ float2 buf[NPR * LS];
    __shared__ float2 tw2[L2];
    __shared__ float nyq[NZS];
    stage_table_n<NTA>(tw2, tw_all + tw_offset(L2), L2);
    const int t = threadIdx.x;
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    const int ny = b.d[item].ny;
    const int id = gid - b.start[item];
    const int y = id % ny, c = id / ny;
    const int G = (L + 1 + TKB - 1) / TKB;
    const float2* __restrict__ T = b.d[item].T;
    float* __restrict__ rows = b.d[item].H + ((size_t)c * NZS * ny + y) * L;
    const bool owner = t < L / 2;
    const float2* twz = tw_all + tw_offset(NZ);

    // z: truncated inverse, h[z] = IE[z] + W_NZ^-z IO[z] (IE, IO: inverses of the
    // even and odd kz inputs), for the two owned columns
    float2 col[2][NZS];
    if (owner) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int kx = 2 * t + s;
            if constexpr (NZS == 1) {
                col[s][0] = T[t_index(c, 0, NZ, G, ny, kx, y)];
            } else {
                float2 e[NZS], o[NZS];
#pragma unroll
                for (int m = 0; m < NZS; ++m) {
                    e[m] = T[t_index(c, 2 * m, NZ, G, ny, kx, y)];
                    o[m] = T[t_index(c, 2 * m + 1, NZ, G, ny, kx, y)];
                }
                dft<NZS, +1>(e);
                dft<NZS, +1>(o);
#pragma unroll
                for (int z = 0; z < NZS; ++z)
                    col[s][z] = z == 0 ? cadd(e[0], o[0]) : cadd(e[z], cmul(cconj(twz[z]), o[z]));
            }
        }
    }
    // kx = L: direct truncated inverse (only the real part is used: the row is real)
    if (t < NZS) {
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int k = 0; k < NZ; ++k)
            acc = cadd(acc, cmul(cconj(twz[(k * t) & (NZ - 1)]), T[t_index(c, k, NZ, G, ny, L, y)]));
        nyq[t] = acc.x;
    }
    __syncthreads();

#pragma unroll
    for (int rd = 0; rd < RR::NR; ++rd) {
        // Z[k] = X_a[k] + i X_b[k] for k <= L, Z[2L-k] = conj X_a[k] + i conj X_b[k];
        // the imaginary parts of the DC and Nyquist bins of a real row are dropped
#pragma unroll
        for (int p = 0; p < NPR; ++p) {
            const int z0 = 2 * (rd * NPR + p);
            if (owner) {
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const int kx = 2 * t + s;
                    float2 Xa = col[s][z0];
                    float2 Xb = (z0 + 1 < NZS) ? col[s][z0 + 1] : make_float2(0.f, 0.f);
                    if (kx == 0) {
                        Xa.y = 0.f;
                        Xb.y = 0.f;
                    }
                    buf[p * LS + lpad(kx)] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);
                    if (kx > 0) buf[p * LS + lpad(L2 - kx)] = make_float2(Xa.x + Xb.y, Xb.x - Xa.y);
                }
            }
            if (t == 0) buf[p * LS + lpad(L)] = make_float2(nyq[z0], (z0 + 1 < NZS) ? nyq[z0 + 1] : 0.f);
        }
        __syncthreads();
        auto src = [&](int p, int i) { return buf[p * LS + lpad(i)]; };
        auto sink = [&](int p, int n, float2 v) {
            const int z0 = 2 * (rd * NPR + p);
            rows[(size_t)z0 * ny * L + n] = v.x;
            if (z0 + 1 < NZS) rows[(size_t)(z0 + 1) * ny * L + n] = v.y;
        };
        fft_io<L2, +1, NPR, NTA, RowLines<LS>, false, true, true>(buf, tw2, src, sink);
        __syncthreads();
    }
}

// ============================================================================ launchers
bool xz_supported(int nx, int ny, int nz) {
    auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
    return pow2(nx) && pow2(ny) && pow2(nz) && nx >= 32 && nx <= 1024 && ny >= 16 && ny <= 512 &&
           nz <= 16;
}

int xz_groups(int X1) { return (X1 + TKB - 1) / TKB; }

size_t xz_t_elems(int nx, int ny, int nz) {
    const int NZ = nz > 1 ? 2 * nz : 1;
    const int G = (nx + 1 + TKB - 1) / TKB;
    return (size_t)3 * NZ * G * ny * TKB;
}

#define DM_NZS_CASES(MACRO) MACRO(1) MACRO(2) MACRO(4) MACRO(8) MACRO(16)
#define DM_XZ_L_CASES(MACRO) MACRO(32) MACRO(64) MACRO(128) MACRO(256) MACRO(512) MACRO(1024)

template <bool INVERSE>
static int launch_xz(XZBatch b, int nx, int nz, const float2* tw, hipStream_t s) {
    if (b.count < 1 || b.count > MAXB) return fail(DEMAG_EINVAL, "xz stage: bad batch size");
    b.start[0] = 0;
    for (int r = 0; r < b.count; ++r) b.start[r + 1] = b.start[r] + 3 * b.d[r].ny;
    const unsigned grid = (unsigned)b.start[b.count];
    bool done = false;
#define NZS_CASE(NZv)                                                                         \
    if (nz == NZv) {                                                                          \
        constexpr int NZS = NZv;                                                              \
        if (INVERSE)                                                                          \
            hipLaunchKernelGGL((xz_inverse_kernel<L, NZS>), dim3(grid), dim3(XZShape<L>::NTA), \
                               0, s, b, tw);                                                  \
        else                                                                                  \
            hipLaunchKernelGGL((xz_forward_kernel<L, NZS>), dim3(grid), dim3(XZShape<L>::NTA), \
                               0, s, b, tw);                                                  \
        done = true;                                                                          \
    }
#define L_CASE(Lv)                  \
    if (nx == Lv) {                 \
        constexpr int L = Lv;       \
        DM_NZS_CASES(NZS_CASE)      \
    }
    DM_XZ_L_CASES(L_CASE)
#undef L_CASE
#undef NZS_CASE
    if (!done) return fail(DEMAG_EUNSUPPORTED, "xz stage: unsupported mesh");
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

int launch_xz_forward(XZBatch b, int nx, int nz, const float2* tw, hipStream_t s) {
    return launch_xz<false>(b, nx, nz, tw, s);
}
int launch_xz_inverse(XZBatch b, int nx, int nz, const float2* tw, hipStream_t s) {
    return launch_xz<true>(b, nx, nz, tw, s);
}

int launch_yconv(YCBatch b, int ny, int Nz, const float2* tw, hipStream_t s) {
    if (b.count < 1 || b.count > MAXB) return fail(DEMAG_EINVAL, "y conv: bad batch size");
    b.start[0] = 0;
    for (int r = 0; r < b.count; ++r) b.start[r + 1] = b.start[r] + Nz * b.d[r].X1;
    const unsigned grid = (unsigned)b.start[b.count];
    bool done = false;
#define NZ_CASE(NZv)                                                                                 \
    if (Nz == NZv) {                                                                                 \
        if constexpr (LNY >= 2 * NT)                                                                 \
            hipLaunchKernelGGL((yconv_reg_kernel<LNY, NZv>), dim3(grid), dim3(NT), 0, s, b, tw);     \
        else                                                                                         \
            hipLaunchKernelGGL((yconv_kernel<LNY, NZv>), dim3(grid), dim3(NT), 0, s, b, tw);         \
        done = true;                                                                                 \
    }
#define Y_CASE(NYv)                     \
    if (ny == NYv) {                    \
        constexpr int LNY = 2 * NYv;    \
        NZ_CASE(1) NZ_CASE(4) NZ_CASE(8) NZ_CASE(16) NZ_CASE(32) \
    }
    Y_CASE(16) Y_CASE(32) Y_CASE(64) Y_CASE(128) Y_CASE(256) Y_CASE(512)
#undef Y_CASE
#undef NZ_CASE
    if (!done) return fail(DEMAG_EUNSUPPORTED, "y conv: unsupported mesh");
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

}  // namespace dm
