// stages_xz.hip -- the three-kernel form of the convolution for thin meshes
// (n_z <= 16, 16 <= n_y <= 1024, 32 <= n_x <= 1024).
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
    static constexpr int NTA = L < 64 ? 64 : L;           // thread t owns column kx = t
    static constexpr int L2 = 2 * L;                      // padded x length
    static constexpr int LS = lpad_c(L2) + 1;
};

template <int NZS>
struct ZShape {
    static constexpr int NZ = NZS > 1 ? 2 * NZS : 1;      // padded z length
    static constexpr int NPAIR = NZS > 1 ? NZS / 2 : 1;   // packed row pairs
    static constexpr int H = NZS > 1 ? NZS / 2 : 1;       // length of the z sub-transforms
};

// Row pairs transformed together per round (tile variant V = 0, 1, 2): up to
// 8, 4 or 2 pairs (4, 2, 1 at 2L = 2048, where the 1024-thread block also holds
// a 32-row column in registers).  More pairs give every thread a butterfly in
// the radix-16 passes; fewer take less LDS, so more blocks share a compute
// unit.  The per-line arithmetic is the same, so every variant gives the same
// bits.
template <int L, int NZS, int V>
struct XZRounds {
    static constexpr int CAP = (L >= 1024 ? 4 : 8) >> V;
    static constexpr int NPR = ZShape<NZS>::NPAIR < CAP ? ZShape<NZS>::NPAIR : CAP;  // pairs per round
    static constexpr int NR = ZShape<NZS>::NPAIR / NPR;
};

template <int NTHR>
__device__ __forceinline__ void stage_table_n(float2* dst, const float2* __restrict__ src, int n) {
    for (int i = threadIdx.x; i < n; i += NTHR) dst[i] = src[i];
}

// The x transforms' twiddle table held in LDS with one padding entry per 16:
// the middle passes read entries at strides of 8, 16 and 32, which without the
// padding fold onto a few banks.  Same table values, so the same bits.
struct TwPad {
    const float2* p;
    __device__ __forceinline__ float2 operator[](int t) const { return p[t + (t >> 4)]; }
};
constexpr int tw_pad_entries(int n) { return n + n / 16; }
template <int NTHR>
__device__ __forceinline__ TwPad stage_tw_pad(float2* dst, const float2* __restrict__ src, int n) {
    for (int i = threadIdx.x; i < n; i += NTHR) dst[i + (i >> 4)] = src[i];
    return TwPad{dst};
}

__device__ __forceinline__ size_t t_index(int c, int kz, int NZ, int G, int ny, int kx, int y) {
    return ((((size_t)c * NZ + kz) * G + kx / TKB) * ny + y) * TKB + kx % TKB;
}

// ---- z transforms of one kx column in the registers of one thread
// Padded length NZ = 2 NZS, inputs z >= NZS zero.  With H = NZS / 2, writing
// z = z' + H p (p = 0, 1; p = 2, 3 fall in the zero half) and kz = 4 q + r,
//   Y[4q + r] = sum_{z' < H} W_H^{z' q} W_NZ^{r z'} c_r[z'],
//   c_r[z'] = x[z'] + (W_4)^r x[z' + H]                       (W_4 = -i),
// so each class r of outputs is the H-point DFT of c_r weighted by W_NZ^{r z'}:
// plain for r = 0, the exact half-step weights for r = 2 (W_NZ^2 = W_{2H}), and
// table powers W_NZ^{r 2^d} for r = 1, 3.  Classes are produced one at a time,
// so a thread holds its column plus one class.
template <int NZS, class Out>
__device__ __forceinline__ void z_forward(const float2* x, const float2* __restrict__ twz, Out out) {
    using Z = ZShape<NZS>;
    if constexpr (NZS == 1) {
        out(0, x[0]);
    } else {
        constexpr int H = Z::H;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float2 v[H];
#pragma unroll
            for (int z = 0; z < H; ++z) {
                const float2 u = x[z + H];
                const float2 t = r == 0 ? u : r == 1 ? mul_i<-1>(u) : r == 2 ? make_float2(-u.x, -u.y)
                                                                                : mul_i<+1>(u);
                v[z] = cadd(x[z], t);
            }
            if (r == 0) {
                dft2k<H, -1>(v, TwNone{});
            } else if (r == 2) {
                dft2k<H, -1>(v, TwHalf{});
            } else {
                TwRun w;
#pragma unroll
                for (int d = 0; (1 << d) < H; ++d) w.p[d] = twz[r << d];
                dft2k<H, -1>(v, w);
            }
#pragma unroll
            for (int q = 0; q < H; ++q) out(4 * q + r, v[q]);
        }
    }
}

// Truncated inverse of the above: h[z] = sum_kz Y[kz] W_NZ^{-kz z}, z < NZS.
// With the same split, G_r[z'] = sum_q Y[4q + r] W_H^{-q z'} (an H-point
// inverse DFT of class r), t_r = W_NZ^{-r z'} G_r[z'], and
//   h[z'] = sum_r t_r[z'],   h[z' + H] = sum_r (i)^r t_r[z'].
// in(kz) returns Y[kz]; classes are read one at a time.
template <int NZS, class In>
__device__ __forceinline__ void z_inverse(float2* h, const float2* __restrict__ twz, In in) {
    using Z = ZShape<NZS>;
    if constexpr (NZS == 1) {
        h[0] = in(0);
    } else {
        constexpr int H = Z::H;
        // class 0 sets h; classes 1..3 add to it (a rolled loop: the class
        // index only selects table entries and the rotation by i^r, and one
        // class of loads in flight keeps the registers to h plus one class)
#pragma unroll
        for (int q = 0; q < H; ++q) h[q] = in(4 * q);
        dft2k<H, +1>(h, TwNone{});
#pragma unroll
        for (int z = 0; z < H; ++z) h[z + H] = h[z];
#pragma unroll 1
        for (int r = 1; r < 4; ++r) {
            float2 g[H];
#pragma unroll
            for (int q = 0; q < H; ++q) g[q] = in(4 * q + r);
            dft2k<H, +1>(g, TwNone{});
            // rotation of the upper half by i^r: (re, im) -> (sr re - si im, si re + sr im)
            const float sr = r == 2 ? -1.f : 0.f, si = r == 1 ? 1.f : (r == 3 ? -1.f : 0.f);
#pragma unroll
            for (int z = 0; z < H; ++z) {
                const float2 t = z == 0 ? g[0] : cmul(cconj(twz[r * z]), g[z]);
                h[z] = cadd(h[z], t);
                h[z + H] = cadd(h[z + H], make_float2(fmaf(sr, t.x, -(si * t.y)), fmaf(si, t.x, sr * t.y)));
            }
        }
    }
}

// ============================================================================ xz forward
// One block: component c, row y, all nz rows.  Rows are packed in pairs
// (z, z+1) as a + i b, NPR pairs per round go through the length-2L transform
// in LDS (upper half zero), and thread t takes column kx = t of every row out of
// the Hermitian pair; after the last round it runs the z transform of its
// column in registers and stores the Nz values.  The real Nyquist column
// kx = L is transformed by a direct DFT.
template <int L, int NZS, int V>
__global__ __launch_bounds__(XZShape<L>::NTA) void xz_forward_kernel(const XZBatch b,
                                                                   const float2* __restrict__ tw_all) {
    using S = XZShape<L>;
    using Z = ZShape<NZS>;
    using RR = XZRounds<L, NZS, V>;
    constexpr int NTA = S::NTA, L2 = S::L2, LS = S::LS, NZ = Z::NZ, NPR = RR::NPR;
    __shared__ float2 buf[NPR * LS];
    __shared__ float2 tw2s[tw_pad_entries(L2)];
    __shared__ float nyq[NZS];
    const TwPad tw2 = stage_tw_pad<NTA>(tw2s, tw_all + tw_offset(L2), L2);
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
    const bool owner = t < L;

    float2 col[NZS];  // x spectrum of column kx = t, rows 0..nz-1
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
                float2 Zk = buf[p * LS + lpad(t)];
                float2 Zn = cconj(buf[p * LS + lpad((L2 - t) & (L2 - 1))]);
                float2 d = csub(Zk, Zn);
                col[z0] = cscale(cadd(Zk, Zn), 0.5f);
                if (z0 + 1 < NZS) col[z0 + 1] = make_float2(0.5f * d.y, -0.5f * d.x);
            }
            if (t == 0) {  // kx = L: Z[L] and conj Z[L]
                float2 Zk = buf[p * LS + lpad(L)];
                nyq[z0] = Zk.x;
                if (z0 + 1 < NZS) nyq[z0 + 1] = Zk.y;
            }
        }
        __syncthreads();
    }

    const float2* twz = tw_all + tw_offset(NZ);
    if (owner)
        z_forward<NZS>(col, twz, [&](int kz, float2 v) { T[t_index(c, kz, NZ, G, ny, t, y)] = v; });
    // kx = L (real rows: its spectrum is real): direct length-NZ DFT, one output per thread
    if (t < NZ) {
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int z = 0; z < NZS; ++z) acc = cadd(acc, cscale(twz[(t * z) & (NZ - 1)], nyq[z]));
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

// Same column work for LNY = NTY R (ny >= 256 with NTY = 256 threads, ny >= 128
// with 128), with the radices ordered so that the tensor product runs in
// registers: forward passes 16, R1, R and inverse passes R, R1, 16
// (R1 = LNY / (16 R)).  After the forward last pass thread j holds
// k = j + NTY r (r < R) of all three component lines, which is exactly the
// input set of butterfly j of the inverse first pass; the product sits between
// the two in registers, with no LDS round trip.  The thread count fixes the
// radix order (1024 = 16 16 4 with 256 threads, 16 8 8 with 128), so the two
// forms round differently; each is deterministic.
//
// PAIR = false: a block takes one plane; the blocks of the mirror planes kz and
// NZ - kz, which read the same folded tensor column, are adjacent in the grid.
// PAIR = true: a block takes both mirror planes of one kx (0 and NZ/2 for the
// first pair): the tensor values are loaded once for both, and the second
// column's spectra are loaded into registers while the first column's passes
// run (more registers per thread, fewer waves per SIMD).  Same arithmetic.
template <int LNY, int NZ, int NTY, bool PAIR>
__global__ __launch_bounds__(NTY) void yconv_reg_kernel(const YCBatch b, const float2* __restrict__ tw_all) {
    constexpr int NT = NTY;
    constexpr int NY = LNY / 2;
    constexpr int R = LNY / NT;
    constexpr int R1 = LNY / (16 * R);
    static_assert(R >= 2 && R <= 16 && R1 >= 2 && R1 <= 16 && 16 * R1 * R == LNY,
                  "thread j owns k = j + NT r of the three lines");
    constexpr int LS = lpad_c(LNY);
    using Rows = RowLines<LS>;
    __shared__ float2 buf[3 * LS];
    // twiddles as coarse x fine products (Tw2): 26.6 KB of LDS per block at
    // LNY = 1024, so five blocks share a compute unit instead of four
    __shared__ float2 twt[tw2_entries(LNY)];
    const Tw2 tw = stage_tw2<LNY, NT>(twt, tw_all + tw_offset(LNY));
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    const YCDesc& d = b.d[item];
    const int X1 = d.X1, Y1 = d.Y1, Z1 = d.Z1, G = d.G;
    const int id = gid - b.start[item];
    int kx, kzA, kzB;
    if constexpr (NZ == 1) {
        kx = id;
        kzA = kzB = 0;
    } else if constexpr (PAIR) {
        const int jj = id / X1;
        kx = id - jj * X1;
        kzA = jj;
        kzB = jj == 0 ? NZ / 2 : NZ - jj;
    } else {
        const int member = id & 1, t = id >> 1, jj = t / X1;
        kx = t - jj * X1;
        kzA = kzB = jj == 0 ? (member ? NZ / 2 : 0) : (member ? NZ - jj : jj);
    }
    constexpr int NCOL = (NZ == 1 || !PAIR) ? 1 : 2;
    const size_t cstride = (size_t)NZ * G * NY * TKB;
    auto column = [&](int kz) { return d.T + (((size_t)kz * G + kx / TKB) * NY) * TKB + kx % TKB; };
    const int j = threadIdx.x;

    // first-pass inputs (radix 16, upper half of the padded line zero) of one
    // column, held in registers: butterfly bb = j + q NT of line bb / NB
    constexpr int NB = LNY / 16, TOT = 3 * NB, PER = (TOT + NT - 1) / NT;
    float2 pf[PER][8];
    auto load_column = [&](const float2* colp) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int bb = j + q * NT;
            if (TOT % NT == 0 || bb < TOT) {
                const int line = bb / NB, jb = bb - line * NB;
#pragma unroll
                for (int r = 0; r < 8; ++r) pf[q][r] = colp[line * cstride + (size_t)(jb + r * NB) * TKB];
            }
        }
    };
    // tensor values of the thread's k = j + NT r, folded to f = min(k, LNY - k)
    const size_t KC = (size_t)Z1 * X1 * Y1;
    float kv[R][6], sy[R];
    auto load_tensor = [&](int kzf) {
        const float* kp = d.K + ((size_t)kzf * X1 + kx) * Y1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k = j + NT * r;
            const int f = k <= NY ? k : LNY - k;
            sy[r] = k <= NY ? 1.f : -1.f;
#pragma unroll
            for (int a = 0; a < 6; ++a) kv[r][a] = kp[a * KC + f];
        }
    };

    load_column(column(kzA));
    int kzf_loaded = 2 * kzA > NZ ? NZ - kzA : kzA;
    load_tensor(kzf_loaded);
#pragma unroll
    for (int ci = 0; ci < NCOL; ++ci) {
        const int kz = ci == 0 ? kzA : kzB;
        float2* __restrict__ col = column(kz);
        const int kzf = 2 * kz > NZ ? NZ - kz : kz;
        const float sz = 2 * kz > NZ ? -1.f : 1.f;
        if (kzf != kzf_loaded) {  // the first pair's second plane (NZ/2)
            load_tensor(kzf);
            kzf_loaded = kzf;
        }
        // forward first pass from the registers into LDS
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int bb = j + q * NT;
            if (TOT % NT == 0 || bb < TOT) {
                const int line = bb / NB, jb = bb - line * NB;
                float2 v[16];
#pragma unroll
                for (int r = 0; r < 8; ++r) v[r] = pf[q][r];
                dft_half_in<16, -1>(v);
                float2* dst = buf + Rows::idx(line, jb * 16);
#pragma unroll
                for (int r = 0; r < 16; ++r) dst[Rows::template at<true>(jb * 16, r)] = v[r];
            }
        }
        __syncthreads();
        if (ci + 1 < NCOL) load_column(column(kzB));  // in flight during this column's passes
        stockham_pass<LNY, R1, 16, -1, 3, NT, Rows>(buf, tw);
        float2 v[3][R];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[c][r] = buf[c * LS + lpad(j + NT * r)];
            dft_twiddled<R, -1>(v[c], tw, j);
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
        stockham_pass<LNY, R1, R, +1, 3, NT, Rows>(buf, tw);
        auto sink = [&](int c, int yy, float2 val) { col[c * cstride + (size_t)yy * TKB] = val; };
        last_pass<LNY, 16, +1, 3, NT, Rows, true, false>(buf, tw, sink);
        if (ci + 1 < NCOL) __syncthreads();  // the last pass has read LDS before the next first pass writes it
    }
}

// ============================================================================ xz inverse
// One block: component c, row y.  Thread t reads column kx = t of every kz
// plane, runs the truncated z inverse in registers (nz outputs), then NPR row
// pairs per round are rebuilt in LDS as Hermitian-packed length-2L lines
// (Z[k] = X_a[k] + i X_b[k], Z[2L-k] = conj X_a[k] + i conj X_b[k]) and
// inverse transformed, keeping the first L outputs (real part row z, imaginary
// part row z+1).
template <int L, int NZS, int V>
__global__ __launch_bounds__(XZShape<L>::NTA) void xz_inverse_kernel(const XZBatch b,
                                                                   const float2* __restrict__ tw_all) {
    using S = XZShape<L>;
    using Z = ZShape<NZS>;
    using RR = XZRounds<L, NZS, V>;
    constexpr int NTA = S::NTA, L2 = S::L2, LS = S::LS, NZ = Z::NZ, NPR = RR::NPR;
    __shared__ float2 buf[NPR * LS];
    __shared__ float2 tw2s[tw_pad_entries(L2)];
    __shared__ float nyq[NZS];
    const TwPad tw2 = stage_tw_pad<NTA>(tw2s, tw_all + tw_offset(L2), L2);
    const int t = threadIdx.x;
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    const int ny = b.d[item].ny;
    const int id = gid - b.start[item];
    const int y = id % ny, c = id / ny;
    const int G = (L + 1 + TKB - 1) / TKB;
    const float2* __restrict__ T = b.d[item].T;
    float* __restrict__ rows = b.d[item].H + ((size_t)c * NZS * ny + y) * L;
    const bool owner = t < L;
    const float2* twz = tw_all + tw_offset(NZ);

    float2 col[NZS];
    if (owner)
        z_inverse<NZS>(col, twz, [&](int kz) { return T[t_index(c, kz, NZ, G, ny, t, y)]; });
    // kx = L: direct truncated inverse (only the real part is used: the row is real)
    if (t < NZS) {
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int k = 0; k < NZ; ++k)
            acc = cmad(cconj(twz[(k * t) & (NZ - 1)]), T[t_index(c, k, NZ, G, ny, L, y)], acc);
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
                float2 Xa = col[z0];
                float2 Xb = (z0 + 1 < NZS) ? col[z0 + 1] : make_float2(0.f, 0.f);
                if (t == 0) {
                    Xa.y = 0.f;
                    Xb.y = 0.f;
                }
                buf[p * LS + lpad(t)] = make_float2(Xa.x - Xb.y, Xa.y + Xb.x);
                if (t > 0) buf[p * LS + lpad(L2 - t)] = make_float2(Xa.x + Xb.y, Xb.x - Xa.y);
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
    return pow2(nx) && pow2(ny) && pow2(nz) && nx >= 32 && nx <= 1024 && ny >= 16 && ny <= 1024 &&
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
static int launch_xz(XZBatch b, int nx, int nz, int variant, const float2* tw, hipStream_t s) {
    if (b.count < 1 || b.count > MAXB) return fail(DEMAG_EINVAL, "xz stage: bad batch size");
    b.start[0] = 0;
    for (int r = 0; r < b.count; ++r) b.start[r + 1] = b.start[r] + 3 * b.d[r].ny;
    const unsigned grid = (unsigned)b.start[b.count];
    bool done = false;
#define XZ_LAUNCH(V)                                                                               \
    if (INVERSE)                                                                                   \
        DM_LAUNCH((xz_inverse_kernel<L, NZS, V>), dim3(grid), dim3(XZShape<L>::NTA), 0, s,         \
                  b, tw);                                                                          \
    else                                                                                           \
        DM_LAUNCH((xz_forward_kernel<L, NZS, V>), dim3(grid), dim3(XZShape<L>::NTA), 0, s,         \
                  b, tw);
#define NZS_CASE(NZv)                       \
    if (nz == NZv) {                        \
        constexpr int NZS = NZv;            \
        switch (variant) {                  \
            case 0: XZ_LAUNCH(0) break;     \
            case 1: XZ_LAUNCH(1) break;     \
            default: XZ_LAUNCH(2) break;    \
        }                                   \
        done = true;                        \
    }
#define L_CASE(Lv)                  \
    if (nx == Lv) {                 \
        constexpr int L = Lv;       \
        DM_NZS_CASES(NZS_CASE)      \
    }
    DM_XZ_L_CASES(L_CASE)
#undef L_CASE
#undef NZS_CASE
#undef XZ_LAUNCH
    if (!done) return fail(DEMAG_EUNSUPPORTED, "xz stage: unsupported mesh");
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

int launch_xz_forward(XZBatch b, int nx, int nz, int variant, const float2* tw, hipStream_t s) {
    return launch_xz<false>(b, nx, nz, variant, tw, s);
}
int launch_xz_inverse(XZBatch b, int nx, int nz, int variant, const float2* tw, hipStream_t s) {
    return launch_xz<true>(b, nx, nz, variant, tw, s);
}

// Register-product kernel (LNY = 2 ny >= 512): variant 0 = 128 threads, one
// plane per block (radix order 16, R1, R with R = LNY / 128; LNY <= 1024, else
// as variant 1); 1 = 256 threads, one plane per block; 2 = 256 threads, both
// mirror planes per block.  Variants 1 and 2 give the same bits.
static bool yconv_pairs(int ny, int Nz, int variant) {
    return 2 * ny >= 512 && Nz > 1 && variant == 2;
}
int launch_yconv(YCBatch b, int ny, int Nz, int variant, const float2* tw, hipStream_t s) {
    if (b.count < 1 || b.count > MAXB) return fail(DEMAG_EINVAL, "y conv: bad batch size");
    const int planes_per_block = yconv_pairs(ny, Nz, variant) ? 2 : 1;
    b.start[0] = 0;
    for (int r = 0; r < b.count; ++r) b.start[r + 1] = b.start[r] + Nz / planes_per_block * b.d[r].X1;
    const unsigned grid = (unsigned)b.start[b.count];
    bool done = false;
#define NZ_CASE(NZv)                                                                                  \
    if (Nz == NZv) {                                                                                  \
        if constexpr (LNY >= 2 * NT) {                                                                \
            if (LNY <= 1024 && variant == 0)                                                          \
                DM_LAUNCH((yconv_reg_kernel<LNY, NZv, (LNY <= 1024 ? 128 : 256), false>),             \
                          dim3(grid), dim3(LNY <= 1024 ? 128 : 256), 0, s, b, tw);                    \
            else if (variant == 2)                                                                    \
                DM_LAUNCH((yconv_reg_kernel<LNY, NZv, 256, true>), dim3(grid), dim3(256), 0,          \
                          s, b, tw);                                                                  \
            else                                                                                      \
                DM_LAUNCH((yconv_reg_kernel<LNY, NZv, 256, false>), dim3(grid), dim3(256), 0,         \
                          s, b, tw);                                                                  \
        } else {                                                                                      \
            DM_LAUNCH((yconv_kernel<LNY, NZv>), dim3(grid), dim3(NT), 0, s, b, tw);                   \
        }                                                                                             \
        done = true;                                                                                  \
    }
#define Y_CASE(NYv)                     \
    if (ny == NYv) {                    \
        constexpr int LNY = 2 * NYv;    \
        NZ_CASE(1) NZ_CASE(4) NZ_CASE(8) NZ_CASE(16) NZ_CASE(32) \
    }
    Y_CASE(16) Y_CASE(32) Y_CASE(64) Y_CASE(128) Y_CASE(256) Y_CASE(512) Y_CASE(1024)
#undef Y_CASE
#undef NZ_CASE
    if (!done) return fail(DEMAG_EUNSUPPORTED, "y conv: unsupported mesh");
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

}  // namespace dm
