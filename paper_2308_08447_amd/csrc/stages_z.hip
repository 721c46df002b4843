// stages_z.hip -- z stage: z FFT, the packed symmetric tensor product, z IFFT; and the twiddle table.
#include "stage_common.h"

namespace dm {

// ============================================================================ z
// One block: folded ky indices f in [f0, f0 + th) of one kx, each taken together
// with its mirror ky = Ny - f, so that the kernel values K(kx, |ky|, |kz|) are read
// once for both.  The mirror slot of f = 0 (which has no mirror) carries the
// Nyquist column ky = Ny/2 instead.  Column j < TH holds ky = f0 + j, column
// TH + j holds the mirror of f0 + j.  All stored z planes of the 3 components are
// loaded into registers together with the K tile (so every global load of the
// block is in flight at once), then staged in LDS: element (z, c, column) at
// z * 3NC + c * NC + column, i.e. 3NC interleaved lines of length NZ.
// PZ (periodic z): NZ = nz, every z plane is stored and every output kept.
template <int NZ, int TH, int MF, bool PZ = false>
__global__ __launch_bounds__(NT) void z_convolve_kernel(const ZBatch b,
                                                        const float2* __restrict__ tw_all) {
    constexpr int NZH = NZ > 1 ? (PZ ? NZ : NZ / 2) : 1;   // stored z planes
    constexpr int KT = NZ > 1 ? NZ / 2 + 1 : 1;  // folded kz values
    constexpr int NC = 2 * TH;                   // columns per block
    constexpr int NLN = 3 * NC;
    __shared__ float2 buf[NZ * NLN];
    __shared__ float ks[6 * KT * (TH + 1)];      // [comp][kz][f - f0], slot TH = Nyquist
    __shared__ float2 twZ[NZ];
    stage_table(twZ, tw_all + tw_offset(NZ), NZ);
    const int tid = threadIdx.x;
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    float2* __restrict__ S2 = b.d[item].S2;
    const float* __restrict__ K = b.d[item].K;
    const int X1 = b.d[item].X1, Ny = b.d[item].Ny, Y1 = b.d[item].Y1, Z1 = b.d[item].Z1;
    const int k0 = b.d[item].k0, xc = b.d[item].xc;
    const int ny = Ny > 1 ? Ny / 2 : 1;   // folded ky pairs (not a power of two for mixed Ny)
    const int th = TH < ny ? TH : ny;
    const int nft = (ny + th - 1) / th;
    const int id = gid - b.start[item];
    const int f0 = (id % nft) * th, kl = id / nft, kx = k0 + kl;
    const size_t P = (size_t)xc * Ny;  // complex elements per z plane of the chunk
    const size_t cstride = (size_t)NZH * P;
    float2* col = S2 + (size_t)kl * Ny;
    const bool nyq = (f0 == 0 && Ny > 1);
    auto col_ky = [&](int j) -> int {
        if (j < TH) return (j < th && f0 + j < ny) ? f0 + j : -1;
        int jj = j - TH;
        if (jj >= th || f0 + jj >= ny) return -1;
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
            int f = (j < TH) ? ((j < th && f0 + j < ny) ? f0 + j : -1) : (nyq ? Ny / 2 : -1);
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
        fft_io<NZ, -1, NLN, NT, ColLines<NLN>, !PZ, false, true, MF>(buf, twZ, gsrc, lds_sink);
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
        fft_io<NZ, +1, NLN, NT, ColLines<NLN>, false, !PZ, true, MF>(buf, twZ, lds_src, gsink);
    }
}


// Lean form of the same stage for power-of-two N_y and open z in FP32: every
// index is a shift or a mask, global memory is touched only in two coalesced
// loops (consecutive threads on consecutive ky), and the transforms run in LDS
// on line-major rows (RowLines).  A tile pairs the folded ky = f0 .. f0+TH-1
// with the mirrors ky = N_y - f of f = f0+1 .. f0+TH, i.e. the aligned run
// N_y - f0 - TH .. N_y - f0 - 1 (the mirror of f = N_y/2 is the Nyquist column
// itself), so both runs start on a TH-element boundary and every cache line a
// tile touches is used whole; the tensor tile holds f = f0 .. f0+TH.  A block
// takes CPB consecutive tiles of one kx: the next tile's spectra and tensor
// values are loaded into registers while the current tile is transformed.  Per
// column the arithmetic is that of the kernel above, so both give the same
// bits.  Requires N_y / 2 to be a multiple of CPB TH.
constexpr int NTZ = 512;  // threads of the lean z kernel

template <int NZ, int TH, int CPB>
__global__ __launch_bounds__(NTZ) void z_convolve_lean_kernel(const ZBatch b,
                                                             const float2* __restrict__ tw_all) {
    constexpr int NT = NTZ;
    static_assert(NZ >= 2 && (NZ & (NZ - 1)) == 0 && (TH & (TH - 1)) == 0, "powers of two");
    constexpr int NZH = NZ / 2;                  // stored z planes
    constexpr int KT = NZ / 2 + 1;               // folded kz values
    constexpr int NC = 2 * TH;                   // columns per tile (ky and mirrors)
    constexpr int NLN = 3 * NC;                  // lines (component, column)
    constexpr int LS = lpad_c(NZ) + 1;           // line stride in LDS
    constexpr int LNC = ilog2c(NC), LNZH = ilog2c(NZH);
    static_assert(NT % NC == 0, "a thread keeps its column across the I/O loops");
    constexpr int NE = 3 * NZH * NC;             // elements of a tile in one direction
    constexpr int PE = (NE + NT - 1) / NT;
    constexpr int NKL = 6 * KT * TH;             // tensor values f0 .. f0+TH-1 of a tile
    constexpr int PK = (NKL + NT - 1) / NT;
    constexpr int NKN = 6 * KT;                  // and those of f0 + TH
    constexpr int PN = (NKN + NT - 1) / NT;
    using Rows = RowLines<LS>;
    __shared__ float2 buf[NLN * LS];
    __shared__ float ks[6 * KT * (TH + 1)];      // [comp][kz][f - f0]
    __shared__ float2 twZ[NZ];
    for (int i = threadIdx.x; i < NZ; i += NT) twZ[i] = tw_all[tw_offset(NZ) + i];
    const int tid = threadIdx.x;
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    float2* __restrict__ S2 = b.d[item].S2;
    const float* __restrict__ K = b.d[item].K;
    const int X1 = b.d[item].X1, Ny = b.d[item].Ny, Y1 = b.d[item].Y1, Z1 = b.d[item].Z1;
    const int k0 = b.d[item].k0, xc = b.d[item].xc;
    const int nbt = (Ny >> 1) / (TH * CPB);      // blocks per kx
    const int id = gid - b.start[item];
    const int kl = id / nbt, kx = k0 + kl;
    const int fb = (id - kl * nbt) * (TH * CPB);  // first folded ky of the block
    const uint32_t P = (uint32_t)xc * (uint32_t)Ny;   // complex elements per z plane of the chunk
    const uint32_t cstride = (uint32_t)NZH * P;
    float2* __restrict__ col = S2 + (size_t)kl * Ny;
    const float* __restrict__ kcol = K + (size_t)kx * Y1;
    const size_t kplane = (size_t)X1 * Y1;        // tensor values per (comp, kz) plane
    // the column this thread loads and stores: j < TH ky = f0 + j; j = TH + u the
    // mirror run, ky = Ny - f0 - TH + u (folded f = f0 + TH - u)
    const int jt = tid & (NC - 1);
    auto ky_of = [&](int f0) { return jt < TH ? f0 + jt : Ny - f0 - NC + jt; };
    float2 v[PE];
    float kr[PK];
    auto load_tile = [&](int f0) {
        const int ky = ky_of(f0);
#pragma unroll
        for (int i = 0; i < PE; ++i) {
            const int e = tid + i * NT;
            if (NE % NT == 0 || e < NE) {
                const int z = (e >> LNC) & (NZH - 1), c = e >> (LNC + LNZH);
                v[i] = col[c * cstride + (uint32_t)z * P + ky];
            }
        }
#pragma unroll
        for (int q = 0; q < PK; ++q) {
            const int it = tid + q * NT;
            if (NKL % NT == 0 || it < NKL) {
                const int jj = it & (TH - 1), rest = it / TH;   // rest = comp KT + kz
                const int kz = rest % KT, comp = rest / KT;
                kr[q] = kcol[((size_t)comp * Z1 + kz) * kplane + f0 + jj];
            }
        }
    };
    float kn[PN];  // the tile's last tensor values, f = f0 + TH
    auto load_last = [&](int f0) {
#pragma unroll
        for (int q = 0; q < PN; ++q) {
            const int it = tid + q * NT;
            if (NKN % NT == 0 || it < NKN) {
                const int kz = it % KT, comp = it / KT;
                kn[q] = kcol[((size_t)comp * Z1 + kz) * kplane + f0 + TH];
            }
        }
    };
    load_tile(fb);
    load_last(fb);
    auto lds_src = [&](int line, int i) { return buf[line * LS + lpad(i)]; };
    auto lds_sink = [&](int line, int k, float2 w) { buf[line * LS + lpad(k)] = w; };
#pragma unroll
    for (int t = 0; t < CPB; ++t) {
        const int f0 = fb + t * TH;
        const int ky = ky_of(f0);
#pragma unroll
        for (int i = 0; i < PE; ++i) {
            const int e = tid + i * NT;
            if (NE % NT == 0 || e < NE) {
                const int z = (e >> LNC) & (NZH - 1), c = e >> (LNC + LNZH);
                buf[(c * NC + jt) * LS + lpad(z)] = v[i];
            }
        }
#pragma unroll
        for (int q = 0; q < PK; ++q) {
            const int it = tid + q * NT;
            if (NKL % NT == 0 || it < NKL) {
                const int jj = it & (TH - 1), rest = it / TH;
                ks[rest * (TH + 1) + jj] = kr[q];
            }
        }
#pragma unroll
        for (int q = 0; q < PN; ++q) {
            const int it = tid + q * NT;
            if (NKN % NT == 0 || it < NKN) ks[it * (TH + 1) + TH] = kn[q];
        }
        __syncthreads();
        if (t + 1 < CPB) {   // in flight during this tile's transforms
            load_tile(f0 + TH);
            load_last(f0 + TH);
        }

        fft_io<NZ, -1, NLN, NT, Rows, true, false, true>(buf, twZ, lds_src, lds_sink);
        __syncthreads();

        // H^_a = sum_b K_ab M^_b; K folded: ky mirrors flip xy and yz, kz > NZ/2 flips xz and yz
        constexpr int NP = NZ * NC;
#pragma unroll
        for (int it0 = 0; it0 < NP; it0 += NT) {
            const int it = it0 + tid;
            if (NP % NT != 0 && it >= NP) break;
            const int j = it & (NC - 1), kz = it >> LNC;
            const bool mirror = j >= TH;
            const int slot = mirror ? NC - j : j;             // f - f0
            // ky mirrors flip xy and yz, except the Nyquist column (f = Ny/2)
            const float sy = (mirror && 2 * (f0 + slot) != Ny) ? -1.f : 1.f;
            const int kzf = 2 * kz > NZ ? NZ - kz : kz;
            const float sz = 2 * kz > NZ ? -1.f : 1.f;
            constexpr int KC = KT * (TH + 1);
            const float* kp = ks + kzf * (TH + 1) + slot;
            const float kxx = kp[0], kyy = kp[KC], kzz = kp[2 * KC];
            const float kxy = sy * kp[3 * KC], kxz = sz * kp[4 * KC], kyz = sy * sz * kp[5 * KC];
            float2* p = buf + j * LS + lpad(kz);
            const float2 mx = p[0], my = p[NC * LS], mz = p[2 * NC * LS];
            auto dot3 = [](float a, float x, float bb, float y, float cc, float z) {
                return fmaf(cc, z, fmaf(bb, y, a * x));
            };
            p[0] = make_float2(dot3(kxx, mx.x, kxy, my.x, kxz, mz.x), dot3(kxx, mx.y, kxy, my.y, kxz, mz.y));
            p[NC * LS] = make_float2(dot3(kxy, mx.x, kyy, my.x, kyz, mz.x), dot3(kxy, mx.y, kyy, my.y, kyz, mz.y));
            p[2 * NC * LS] = make_float2(dot3(kxz, mx.x, kyz, my.x, kzz, mz.x), dot3(kxz, mx.y, kyz, my.y, kzz, mz.y));
        }
        __syncthreads();
        fft_io<NZ, +1, NLN, NT, Rows, false, true, true>(buf, twZ, lds_src, lds_sink);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PE; ++i) {
            const int e = tid + i * NT;
            if (NE % NT == 0 || e < NE) {
                const int z = (e >> LNC) & (NZH - 1), c = e >> (LNC + LNZH);
                col[c * cstride + (uint32_t)z * P + ky] = buf[(c * NC + jt) * LS + lpad(z)];
            }
        }
        if (t + 1 < CPB) __syncthreads();  // the stores have read LDS before the next tile is written
    }
}

// Register form of the lean stage for N_z = 64, whose FFT plan above is two
// radix-8 passes (R = 8).  The last pass of the forward z FFT leaves butterfly j
// holding X[j + R r] (r < R), and the first pass of the inverse reads exactly
// those elements, so the thread that runs butterfly j of both passes forms the
// tensor product of its R frequencies in registers.  Thread (column, j) thus
// loads its R/2 nonzero inputs z = j + R r of each component from global memory,
// runs the first forward pass in registers, exchanges once through LDS, runs the
// last pass, multiplies, runs the first inverse pass, exchanges once more, runs
// the last inverse pass and stores its R/2 kept outputs: LDS is touched twice per
// element and direction instead of four or more times, and the tensor values
// come straight from global memory (each is used by four threads of the block:
// kz and N_z - kz, ky and its mirror).  Columns are paired as in the lean
// kernel: CB columns per block, CB/2 folded ky and their aligned mirror run.
// The exchanges go one component at a time through two alternating LDS slots, so
// a slot is rewritten only after the barrier that follows its last read.  The
// per-column arithmetic is that of the two kernels above (same passes, same
// twiddle table entries, same product), so all three give the same bits.
// Requires N_y / 2 to be a multiple of CB / 2.
template <int NZ, int CB>
__global__ __launch_bounds__(CB * 8, 4) void z_convolve_sq_kernel(const ZBatch b,
                                                               const float2* __restrict__ tw_all) {
    constexpr int R = 8;
    static_assert(NZ == 64 && radix_of(NZ, 0) == R && radix_of(NZ, 1) == R && npasses(NZ) == 2,
                  "two radix-8 passes");
    constexpr int NT = CB * R;
    constexpr int TH = CB / 2;                   // folded ky per block
    constexpr int RIN = R / 2;                   // nonzero inputs (and kept outputs) per butterfly
    constexpr int NZH = NZ / 2;
    __shared__ float2 ex[2][NZ * CB];            // element e of column c at e * CB + c
    const int tid = threadIdx.x;
    // with 64 columns per block a wave is one butterfly index j: keep it scalar
    const int c = tid % CB;
    const int j = CB == 64 ? __builtin_amdgcn_readfirstlane(tid / CB) : tid / CB;
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    const ZDesc& d = b.d[item];
    const int Ny = d.Ny, Z1 = d.Z1;
    const int nbt = (Ny >> 1) / TH;              // blocks per kx
    const int id = gid - b.start[item];
    const int kl = id / nbt, kx = d.k0 + kl;
    const int f0 = (id - kl * nbt) * TH;
    const uint32_t P = (uint32_t)d.xc * (uint32_t)Ny;   // elements per z plane of the chunk
    const uint32_t cstride = (uint32_t)NZH * P;
    const bool mirror = c >= TH;
    const int ky = mirror ? Ny - f0 - CB + c : f0 + c;
    const int slot = mirror ? CB - c : c;        // folded f - f0
    const float sy = (mirror && 2 * (f0 + slot) != Ny) ? -1.f : 1.f;
    // Global accesses are a block-uniform base plus a 32-bit byte offset (the
    // chunk is at most 128 MB, the tensor below 4 GB).
    char* __restrict__ sb = reinterpret_cast<char*>(d.S2 + (size_t)kl * Ny);
    const uint32_t so = ((uint32_t)ky + (uint32_t)j * P) * 8u;
    auto s2 = [&](int cc, int r) -> float2& {
        return *reinterpret_cast<float2*>(sb + (so + ((uint32_t)cc * cstride + (uint32_t)(R * r) * P) * 8u));
    };
    // tensor value of component q at folded kz: kz = j + R r <= N_z/2 for r < R/2,
    // else N_z - kz = (N_z - R - R r) + (R - j)
    const char* __restrict__ kb = reinterpret_cast<const char*>(d.K + (size_t)kx * d.Y1 + f0);
    const uint32_t kpl = (uint32_t)d.X1 * (uint32_t)d.Y1;
    const uint32_t klo = ((uint32_t)slot + (uint32_t)j * kpl) * 4u;
    const uint32_t khi = ((uint32_t)slot + (uint32_t)(R - j) * kpl) * 4u;
    auto kval = [&](int q, int r) -> float {
        const uint32_t pl = (uint32_t)q * (uint32_t)Z1 + (uint32_t)(r < RIN ? R * r : NZ - R - R * r);
        return *reinterpret_cast<const float*>(kb + ((r < RIN ? klo : khi) + pl * kpl * 4u));
    };

    float2 v[3][R];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
        for (int r = 0; r < RIN; ++r) v[cc][r] = s2(cc, r);
    // With 64 columns per block the tensor loads go out with the spectrum loads,
    // so they are in flight during the forward transforms (48 more registers,
    // within the 128 that two blocks per compute unit allow); with 32 they are
    // issued at the product, where they fit without spilling.
    constexpr bool KEARLY = CB == 64;
    float kv[6][R];
    if constexpr (KEARLY) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int q = 0; q < 6; ++q) kv[q][r] = kval(q, r);
    }
    // the last passes' twiddles W^(j 2^d), W = exp(-2 pi i / N_z), as table entries
    const float2* twz = tw_all + tw_offset(NZ);
    TwRun twf;
#pragma unroll
    for (int dd = 0; (1 << dd) < R; ++dd) twf.p[dd] = twz[j << dd];

    int sl = 0;
    auto exchange = [&](float2* a) {             // a[r] = element j R + r in, j + R r out
        float2* e = ex[sl];
#pragma unroll
        for (int r = 0; r < R; ++r) e[(j * R + r) * CB + c] = a[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = e[(j + R * r) * CB + c];
        sl ^= 1;
    };
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
        dft_half_in<R, -1>(v[cc]);
        exchange(v[cc]);
        dft2k<R, -1>(v[cc], twf);
    }
    // H^_a = sum_b K_ab M^_b; ky mirrors flip xy and yz (not the Nyquist column),
    // kz > N_z/2 flips xz and yz
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int kz = j + R * r;
        const float sz = 2 * kz > NZ ? -1.f : 1.f;
        if constexpr (!KEARLY) {
#pragma unroll
            for (int q = 0; q < 6; ++q) kv[q][r] = kval(q, r);
        }
        const float kxx = kv[0][r], kyy = kv[1][r], kzz = kv[2][r];
        const float kxy = sy * kv[3][r], kxz = sz * kv[4][r], kyz = sy * sz * kv[5][r];
        const float2 mx = v[0][r], my = v[1][r], mz = v[2][r];
        auto dot3 = [](float a, float x, float bb, float y, float cc2, float z) {
            return fmaf(cc2, z, fmaf(bb, y, a * x));
        };
        v[0][r] = make_float2(dot3(kxx, mx.x, kxy, my.x, kxz, mz.x), dot3(kxx, mx.y, kxy, my.y, kxz, mz.y));
        v[1][r] = make_float2(dot3(kxy, mx.x, kyy, my.x, kyz, mz.x), dot3(kxy, mx.y, kyy, my.y, kyz, mz.y));
        v[2][r] = make_float2(dot3(kxz, mx.x, kyz, my.x, kzz, mz.x), dot3(kxz, mx.y, kyz, my.y, kzz, mz.y));
    }
    TwRun twi;
#pragma unroll
    for (int dd = 0; (1 << dd) < R; ++dd) twi.p[dd] = make_float2(twf.p[dd].x, -twf.p[dd].y);
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
        dft<R, +1>(v[cc]);
        exchange(v[cc]);
        dft2k<R, +1>(v[cc], twi);
#pragma unroll
        for (int r = 0; r < RIN; ++r) s2(cc, r) = v[cc][r];
    }
}

int launch_z_convolve(ZBatch b, int Nz, int variant, int mf, const float2* tw, hipStream_t s,
                      bool periodic) {
    if (b.count < 1 || b.count > MAXB) return fail(DEMAG_EINVAL, "z stage: bad batch size");
    if (periodic && Nz > 1) {
        if (mf) return fail(DEMAG_EUNSUPPORTED, "z stage: periodic transforms are FP32 only");
        switch (Nz) {
#define CASE(NZv)                                                                              \
    case NZv: {                                                                                \
        constexpr int NZ = NZv;                                                                \
        constexpr int TH = ZTile<NZ, 1>::TH;                                                   \
        b.start[0] = 0;                                                                        \
        for (int r = 0; r < b.count; ++r) {                                                    \
            int ny = b.d[r].Ny > 1 ? b.d[r].Ny / 2 : 1;                                        \
            int th = TH < ny ? TH : ny;                                                        \
            b.start[r + 1] = b.start[r] + ((ny + th - 1) / th) * b.d[r].nk;                   \
        }                                                                                      \
        DM_LAUNCH((z_convolve_kernel<NZ, TH, 0, true>), dim3((unsigned)finish_batch(b)),       \
                  dim3(NT), 0, s, b, tw);                                                      \
        break;                                                                                 \
    }
            CASE(2) CASE(4) CASE(8) CASE(16) CASE(32) CASE(64) CASE(128)
#undef CASE
            default: return fail(DEMAG_EUNSUPPORTED, "z stage: unsupported nz");
        }
        DM_CHECK_LAUNCH();
        return DEMAG_OK;
    }
    switch (Nz) {
#define BODY(V)                                                                                \
    {                                                                                          \
        constexpr int TH = ZTile<NZ, V>::TH;                                                   \
        constexpr int THL = LeanZTile<NZ, V>::TH;                                              \
        b.start[0] = 0;                                                                        \
        constexpr int CPB = 2;                                                                 \
        bool lean = NZ >= 2 && mf == 0;                                                        \
        for (int r = 0; r < b.count; ++r) {                                                    \
            int ny = b.d[r].Ny > 1 ? b.d[r].Ny / 2 : 1;                                        \
            lean = lean && b.d[r].Ny >= 2 && (b.d[r].Ny & (b.d[r].Ny - 1)) == 0 &&             \
                   ny % (CPB * THL) == 0;                                                      \
        }                                                                                      \
        for (int r = 0; r < b.count; ++r) {                                                    \
            int ny = b.d[r].Ny > 1 ? b.d[r].Ny / 2 : 1;                                        \
            int th = TH < ny ? TH : ny;                                                        \
            b.start[r + 1] = b.start[r] + (lean ? ny / (CPB * THL) : (ny + th - 1) / th) * b.d[r].nk; \
        }                                                                                      \
        if constexpr (NZ == 64) {                                                              \
            /* variants 0 and 2: the register form with 32 or 64 columns per block */        \
            constexpr int CBQ = V == 2 ? 64 : 32;                                              \
            bool sq = V != 1 && mf == 0;                                                       \
            for (int r = 0; r < b.count; ++r)                                                  \
                sq = sq && b.d[r].Ny >= 2 && (b.d[r].Ny & (b.d[r].Ny - 1)) == 0 &&             \
                     (b.d[r].Ny / 2) % (CBQ / 2) == 0;                                         \
            if (sq) {                                                                          \
                for (int r = 0; r < b.count; ++r)                                              \
                    b.start[r + 1] = b.start[r] + (b.d[r].Ny / CBQ) * b.d[r].nk;               \
                DM_LAUNCH((z_convolve_sq_kernel<NZ, CBQ>), dim3((unsigned)finish_batch(b)),    \
                          dim3(CBQ * 8), 0, s, b, tw);                                         \
                break;                                                                         \
            }                                                                                  \
        }                                                                                      \
        if constexpr (NZ >= 2) {                                                               \
            if (lean) {                                                                        \
                DM_LAUNCH((z_convolve_lean_kernel<NZ, THL, CPB>),                              \
                          dim3((unsigned)finish_batch(b)), dim3(NTZ), 0, s, b, tw);            \
                break;                                                                         \
            }                                                                                  \
        }                                                                                      \
        DM_MF_DISPATCH(V, DM_LAUNCH((z_convolve_kernel<NZ, TH, MFv>),                          \
                  dim3((unsigned)finish_batch(b)), dim3(NT), 0, s, b, tw);)                    \
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

void fill_twiddles(float2* host) {
    for (int i = 0; i < TW_ENTRIES; ++i) host[i] = make_float2(0.f, 0.f);
    for (int F : {1, 3, 5, 15}) {
        for (int L = F; L <= TW_LMAX; L *= 2) {
            const int off = tw_offset(L);
            for (int t = 0; t < L; ++t) {
                long double ang = -2.0L * 3.141592653589793238462643383279502884L * t / L;
                host[off + t] = make_float2((float)cosl(ang), (float)sinl(ang));
            }
        }
    }
}


}  // namespace dm
