// dynamics.hip -- exchange + LLG RK4 stage update (Eqs. 4, 5; Sec. III) and the
// atomistic Heun step (Eqs. 7, 9, 10; Sec. IV) on gfx950.
//
// All kernels stream [3][nz][ny][nx] FP32 fields, one thread per cell, x fastest
// so that every component load is a coalesced row.  The RK4 stage reads its
// neighbours along y/z from rows the neighbouring wavefronts also read (L1/L2
// hits); the Heun stages march through z with the plane in LDS (below).
#include "engine.h"

namespace dm {

namespace {

__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return make_float3(fmaf(a.y, b.z, -(a.z * b.y)), fmaf(a.z, b.x, -(a.x * b.z)),
                       fmaf(a.x, b.y, -(a.y * b.x)));
}

// Landau-Lifshitz right-hand side: -gam [m x H + alpha m x (m x H)]
__device__ __forceinline__ float3 ll_rhs(float3 m, float3 H, float gam, float alpha) {
    float3 mxH = cross3(m, H);
    float3 mmH = cross3(m, mxH);
    return make_float3(-gam * fmaf(alpha, mmH.x, mxH.x), -gam * fmaf(alpha, mmH.y, mxH.y),
                       -gam * fmaf(alpha, mmH.z, mxH.z));
}

__device__ __forceinline__ float3 load3(const float* __restrict__ f, size_t i, size_t N) {
    return make_float3(f[i], f[i + N], f[i + 2 * N]);
}
__device__ __forceinline__ void store3(float* __restrict__ f, size_t i, size_t N, float3 v) {
    f[i] = v.x;
    f[i + N] = v.y;
    f[i + 2 * N] = v.z;
}

// ---------------------------------------------------------------- micromagnetic
// Stage s of classic RK4 on m (step start) with stage input ms:
//   k_s = LL(ms, H_d + H_ex(ms) + H_zee)
//   s=0: acc = k1,      out = m + dt/2 k1
//   s=1: acc += 2 k2,   out = m + dt/2 k2
//   s=2: acc += 2 k3,   out = m + dt k3
//   s=3: out = normalise(m + dt/6 (acc + k4))   (out may alias m)
// One launch updates a batch of independent meshes (one descriptor each).
// Blocks take 256-cell tiles of an xy plane with z fastest in the (XCD-renumbered)
// block order, so the blocks of one tile at z-1, z, z+1 run together on one XCD
// and read each other's planes from L2: the z neighbours of the exchange stencil
// then cost no extra HBM traffic.
__global__ __launch_bounds__(256) void llg_stage_kernel(const LLGBatch b, int stage) {
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    int item = 0;
    while (item + 1 < b.count && gid >= b.start[item + 1]) ++item;
    const LLGDesc& a = b.d[item];
    const size_t P = (size_t)a.nx * a.ny;
    const size_t N = P * a.nz;
    const int local = gid - b.start[item];
    const int zt = local % a.nz;
    const size_t p = (size_t)(local / a.nz) * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const size_t i = (size_t)zt * P + p;
    const float* __restrict__ ms = a.ms;
    const int x = (int)(p % a.nx), y = (int)(p / a.nx), z = zt;
    float3 c = load3(ms, i, N);
    // free boundaries: a missing neighbour is replaced by the cell itself; along
    // a periodic axis the first and last cells are neighbours
    float3 lap = make_float3(0.f, 0.f, 0.f);
    auto add_axis = [&](float coef, int pos, int n, size_t stride, bool per) {
        const size_t wrap = (size_t)(n - 1) * stride;
        float3 l = pos > 0 ? load3(ms, i - stride, N) : (per ? load3(ms, i + wrap, N) : c);
        float3 r = pos < n - 1 ? load3(ms, i + stride, N) : (per ? load3(ms, i - wrap, N) : c);
        lap.x = fmaf(coef, (l.x + r.x) - 2.f * c.x, lap.x);
        lap.y = fmaf(coef, (l.y + r.y) - 2.f * c.y, lap.y);
        lap.z = fmaf(coef, (l.z + r.z) - 2.f * c.z, lap.z);
    };
    if (a.nx > 1) add_axis(a.cx, x, a.nx, 1, a.pbc & 1);
    if (a.ny > 1) add_axis(a.cy, y, a.ny, (size_t)a.nx, a.pbc & 2);
    if (a.nz > 1) add_axis(a.cz, z, a.nz, (size_t)a.nx * a.ny, a.pbc & 4);
    float3 hd = load3(a.Hd, i, N);
    float3 H = make_float3(hd.x + lap.x + a.hz[0], hd.y + lap.y + a.hz[1], hd.z + lap.z + a.hz[2]);
    float3 k = ll_rhs(c, H, a.gam, a.alpha);
    float3 m0 = load3(a.m, i, N);
    if (stage == 0) {
        store3(a.acc, i, N, k);
        float h = 0.5f * a.dt;
        store3(a.out, i, N, make_float3(fmaf(h, k.x, m0.x), fmaf(h, k.y, m0.y), fmaf(h, k.z, m0.z)));
    } else if (stage < 3) {
        float3 s = load3(a.acc, i, N);
        store3(a.acc, i, N, make_float3(fmaf(2.f, k.x, s.x), fmaf(2.f, k.y, s.y), fmaf(2.f, k.z, s.z)));
        float h = stage == 1 ? 0.5f * a.dt : a.dt;
        store3(a.out, i, N, make_float3(fmaf(h, k.x, m0.x), fmaf(h, k.y, m0.y), fmaf(h, k.z, m0.z)));
    } else {
        float3 s = load3(a.acc, i, N);
        float h = a.dt / 6.f;
        float3 v = make_float3(fmaf(h, s.x + k.x, m0.x), fmaf(h, s.y + k.y, m0.y), fmaf(h, s.z + k.z, m0.z));
        float inv = rsqrtf(v.x * v.x + v.y * v.y + v.z * v.z);
        store3(a.out, i, N, make_float3(v.x * inv, v.y * inv, v.z * inv));
    }
}

// Sub-step demagnetizing field from the history ring: out = sum_j w_j h_j with
// the weights of the polynomial through the five step-start fields.
struct Extrap5 {
    const float* h[5];
    float w[5];
};
__global__ __launch_bounds__(256) void extrapolate_kernel(float* __restrict__ out, const Extrap5 e,
                                                          size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v = e.w[0] * e.h[0][i];
#pragma unroll
    for (int j = 1; j < 5; ++j) v = fmaf(e.w[j], e.h[j][i], v);
    out[i] = v;
}

// Mean over the cells of each component of a [3][N] field: one 1024-thread block
// per component, FP64 partial sums in a fixed order (strided per thread, then a
// tree in LDS), so the result does not depend on scheduling.
__global__ __launch_bounds__(1024) void field_mean_kernel(const float* __restrict__ v, size_t n,
                                                          float* __restrict__ out) {
    __shared__ double part[1024];
    const int c = blockIdx.x, t = threadIdx.x;
    const float* __restrict__ f = v + (size_t)c * n;
    double acc = 0.0;
    for (size_t i = t; i < n; i += 1024) acc += (double)f[i];
    part[t] = acc;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    if (t == 0) out[c] = (float)(part[0] / (double)n);
}

// ---------------------------------------------------------------- atomistic
// Eq. (9): M = mu_s mu_B/(a^3 N_S) * sum of the unit spins of the macrocell.
// VEC (macro = 4, 16-byte aligned rows): each row of a macrocell is one float4
// per component.
template <bool VEC>
__global__ __launch_bounds__(256) void macro_average_kernel(AtomArgs a, const float* __restrict__ S,
                                                            float* __restrict__ Mm) {
    const int mx = a.nx / a.macro, my = a.ny / a.macro, mz = a.nz / a.macro;
    const size_t Nm = (size_t)mx * my * mz;
    const size_t N = (size_t)a.nx * a.ny * a.nz;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Nm) return;
    int X = (int)(i % mx), Y = (int)((i / mx) % my), Z = (int)(i / ((size_t)mx * my));
    float3 s = make_float3(0.f, 0.f, 0.f);
    if constexpr (VEC) {
        // the spins are added in the same order as in the general loop below
        for (int dz = 0; dz < 4; ++dz)
            for (int dy = 0; dy < 4; ++dy) {
                size_t row = ((size_t)(Z * 4 + dz) * a.ny + (Y * 4 + dy)) * a.nx + X * 4;
                float4 u = *reinterpret_cast<const float4*>(S + row);
                float4 v = *reinterpret_cast<const float4*>(S + N + row);
                float4 w = *reinterpret_cast<const float4*>(S + 2 * N + row);
                s.x += u.x; s.y += v.x; s.z += w.x;
                s.x += u.y; s.y += v.y; s.z += w.y;
                s.x += u.z; s.y += v.z; s.z += w.z;
                s.x += u.w; s.y += v.w; s.z += w.w;
            }
        store3(Mm, i, Nm, make_float3(a.mscale * s.x, a.mscale * s.y, a.mscale * s.z));
        return;
    }
    for (int dz = 0; dz < a.macro; ++dz)
        for (int dy = 0; dy < a.macro; ++dy) {
            size_t row = ((size_t)(Z * a.macro + dz) * a.ny + (Y * a.macro + dy)) * a.nx + X * a.macro;
            for (int dx = 0; dx < a.macro; ++dx) {
                float3 v = load3(S, row + dx, N);
                s.x += v.x;
                s.y += v.y;
                s.z += v.z;
            }
        }
    store3(Mm, i, Nm, make_float3(a.mscale * s.x, a.mscale * s.y, a.mscale * s.z));
}

// ---- Heun stages (Eq. 10 at T = 0 with the field of Eq. 7 + Eq. 9's macrocell H_d)
// H = J/(mu0 mu_B mu_s) sum_nn S_j (open boundaries: a missing neighbour adds
// nothing) + H_d(macrocell) + H_zee.  A block takes a MTX x MTY column tile of
// the lattice and walks through MZC planes of it.  Each plane of the stencil
// field F (S for the predictor, Sp for the corrector) is read from HBM once:
// the thread's own spin goes to an LDS tile whose edge threads add the x/y
// halo, and the z neighbours are the spins the thread itself held one plane
// before and will hold one plane later (no gathers of whole neighbour rows and
// planes).  Neighbours are summed in the order x-1, x+1, y-1, y+1, z-1, z+1.
// Wide, shallow tiles (128 x 2) measured fastest.
constexpr int MTX = 128, MTY = 2, MZC = 16;

struct MarchTile {
    float v[3][MTY + 2][MTX + 2];
};

// The x/y halo values a thread adds to the tile for plane z: an x halo (left
// of the first column or right of the last) and a y halo (above the first row
// or below the last); zero outside the lattice or for threads with no halo.
struct Halo {
    float3 hx, hy;
};
__device__ __forceinline__ Halo march_halo(const AtomArgs& a, const float* __restrict__ F, size_t N, int x0,
                                           int y0, int z) {
    const int tx = threadIdx.x % MTX, ty = threadIdx.x / MTX;
    const size_t pl = (size_t)a.nx * a.ny;
    auto fetch = [&](int gx, int gy) -> float3 {
        if (gx < 0 || gx >= a.nx || gy < 0 || gy >= a.ny || z >= a.nz) return make_float3(0.f, 0.f, 0.f);
        return load3(F, (size_t)z * pl + (size_t)gy * a.nx + gx, N);
    };
    Halo h{make_float3(0.f, 0.f, 0.f), make_float3(0.f, 0.f, 0.f)};
    if (tx == 0) h.hx = fetch(x0 - 1, y0 + ty);
    if (tx == MTX - 1) h.hx = fetch(x0 + MTX, y0 + ty);
    if (ty == 0) h.hy = fetch(x0 + tx, y0 - 1);
    if (ty == MTY - 1) h.hy = fetch(x0 + tx, y0 + MTY);
    return h;
}

__device__ __forceinline__ void march_fill(MarchTile& t, float3 own, bool inside, const Halo& h) {
    const int tx = threadIdx.x % MTX, ty = threadIdx.x / MTX;
    auto put = [&](int lx, int ly, float3 val) {
        t.v[0][ly][lx] = val.x;
        t.v[1][ly][lx] = val.y;
        t.v[2][ly][lx] = val.z;
    };
    put(tx + 1, ty + 1, inside ? own : make_float3(0.f, 0.f, 0.f));
    if (tx == 0) put(0, ty + 1, h.hx);
    if (tx == MTX - 1) put(MTX + 1, ty + 1, h.hx);
    if (ty == 0) put(tx + 1, 0, h.hy);
    if (ty == MTY - 1) put(tx + 1, MTY + 1, h.hy);
}

// exchange sum of the tile cell (tx, ty) with open boundaries, then z neighbours
__device__ __forceinline__ float3 march_sum(const MarchTile& t, const AtomArgs& a, int x, int y, int z,
                                            float3 below, float3 above) {
    const int tx = threadIdx.x % MTX + 1, ty = threadIdx.x / MTX + 1;
    float3 e = make_float3(0.f, 0.f, 0.f);
    auto add = [&](int lx, int ly) {
        e.x += t.v[0][ly][lx];
        e.y += t.v[1][ly][lx];
        e.z += t.v[2][ly][lx];
    };
    if (x > 0) add(tx - 1, ty);
    if (x < a.nx - 1) add(tx + 1, ty);
    if (y > 0) add(tx, ty - 1);
    if (y < a.ny - 1) add(tx, ty + 1);
    if (z > 0) {
        e.x += below.x;
        e.y += below.y;
        e.z += below.z;
    }
    if (z < a.nz - 1) {
        e.x += above.x;
        e.y += above.y;
        e.z += above.z;
    }
    return e;
}

__device__ __forceinline__ float3 march_field(const AtomArgs& a, const float* __restrict__ Hdm, float3 e,
                                              int x, int y, int z) {
    const int mx = a.nx / a.macro, my = a.ny / a.macro, mz = a.nz / a.macro;
    size_t Nm = (size_t)mx * my * mz;
    size_t im = ((size_t)(z / a.macro) * my + (y / a.macro)) * mx + (x / a.macro);
    float3 hd = load3(Hdm, im, Nm);
    return make_float3(a.cex * e.x + hd.x + a.hz[0], a.cex * e.y + hd.y + a.hz[1],
                       a.cex * e.z + hd.z + a.hz[2]);
}

// STAGE 0: predictor (F = S): f0 = f(S), Sp = S + dt f0.
// STAGE 1: corrector (F = Sp): S = normalise(S + dt/2 (f0 + f(Sp))).
// Every global load a plane needs (its z + 1 neighbours, its tile halo and, for
// the corrector, f0 and S) is issued one plane ahead, so a block's loads are in
// flight while it computes the plane before instead of after each barrier.
template <int STAGE>
__global__ __launch_bounds__(MTX * MTY) void heun_march_kernel(AtomArgs a, const float* __restrict__ F,
                                                             const float* __restrict__ Hdm,
                                                             float* __restrict__ f0, float* Sp_or_S) {
    __shared__ MarchTile tile;
    const size_t N = (size_t)a.nx * a.ny * a.nz;
    const size_t pl = (size_t)a.nx * a.ny;
    const int tilesx = (a.nx + MTX - 1) / MTX, tilesy = (a.ny + MTY - 1) / MTY;
    const int b = blockIdx.x;
    const int bx = b % tilesx, by = (b / tilesx) % tilesy, bz = b / (tilesx * tilesy);
    const int x0 = bx * MTX, y0 = by * MTY, z0 = bz * MZC;
    const int x = x0 + threadIdx.x % MTX, y = y0 + threadIdx.x / MTX;
    const bool inside = x < a.nx && y < a.ny;
    const size_t col = (size_t)y * a.nx + x;
    const int zend = min(z0 + MZC, a.nz);
    const float3 zero = make_float3(0.f, 0.f, 0.f);
    auto column = [&](const float* src, int z) {   // this thread's value of plane z, zero outside
        return (inside && z >= 0 && z < a.nz) ? load3(src, (size_t)z * pl + col, N) : zero;
    };
    float3 below = column(F, z0 - 1);
    float3 cur = column(F, z0);
    float3 above = column(F, z0 + 1);
    Halo halo = march_halo(a, F, N, x0, y0, z0);
    float3 g = zero, sv = zero;   // corrector: f0 and S of the current plane
    if constexpr (STAGE == 1) {
        g = column(f0, z0);
        sv = column(Sp_or_S, z0);
    }
    for (int z = z0; z < zend; ++z) {
        // next plane's loads (consumed in the next iteration)
        const bool more = z + 1 < zend;
        const float3 above2 = more ? column(F, z + 2) : zero;
        const Halo halo2 = more ? march_halo(a, F, N, x0, y0, z + 1) : halo;
        float3 g2 = zero, sv2 = zero;
        if constexpr (STAGE == 1) {
            if (more) {
                g2 = column(f0, z + 1);
                sv2 = column(Sp_or_S, z + 1);
            }
        }
        march_fill(tile, cur, inside, halo);
        __syncthreads();
        if (inside) {
            const size_t i = (size_t)z * pl + col;
            float3 H = march_field(a, Hdm, march_sum(tile, a, x, y, z, below, above), x, y, z);
            float3 f = ll_rhs(cur, H, a.gam, a.alpha);
            if constexpr (STAGE == 0) {
                store3(f0, i, N, f);
                store3(Sp_or_S, i, N, make_float3(cur.x + a.dt * f.x, cur.y + a.dt * f.y, cur.z + a.dt * f.z));
            } else {
                float h = 0.5f * a.dt;
                float3 v = make_float3(sv.x + h * (g.x + f.x), sv.y + h * (g.y + f.y), sv.z + h * (g.z + f.z));
                float inv = rsqrtf(v.x * v.x + v.y * v.y + v.z * v.z);
                store3(Sp_or_S, i, N, make_float3(v.x * inv, v.y * inv, v.z * inv));
            }
        }
        __syncthreads();
        below = cur;
        cur = above;
        above = above2;
        halo = halo2;
        g = g2;
        sv = sv2;
    }
}

unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int launch_llg_stage(LLGBatch b, int stage, hipStream_t stream) {
    if (b.count < 1 || b.count > MAXB) return fail(DEMAG_EINVAL, "llg stage: bad batch size");
    b.start[0] = 0;
    for (int r = 0; r < b.count; ++r) {
        size_t P = (size_t)b.d[r].nx * b.d[r].ny;
        b.start[r + 1] = b.start[r] + (int)blocks_for(P) * b.d[r].nz;
    }
    DM_LAUNCH(llg_stage_kernel, dim3((unsigned)b.start[b.count]), dim3(256), 0, stream, b, stage);
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

int launch_extrapolate(float* out, const float* const h[5], const float w[5], size_t n,
                       hipStream_t stream) {
    Extrap5 e;
    for (int j = 0; j < 5; ++j) {
        e.h[j] = h[j];
        e.w[j] = w[j];
    }
    hipLaunchKernelGGL(extrapolate_kernel, dim3(blocks_for(n)), dim3(256), 0, stream, out, e, n);
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

int launch_field_mean(const float* v, size_t n, float* out, hipStream_t stream) {
    hipLaunchKernelGGL(field_mean_kernel, dim3(3), dim3(1024), 0, stream, v, n, out);
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

int launch_macro_average(const AtomArgs& a, const float* S, float* Mm, hipStream_t stream) {
    size_t Nm = (size_t)(a.nx / a.macro) * (a.ny / a.macro) * (a.nz / a.macro);
    const bool vec = a.macro == 4 && a.nx % 4 == 0 && reinterpret_cast<uintptr_t>(S) % 16 == 0;
    if (vec)
        hipLaunchKernelGGL(macro_average_kernel<true>, dim3(blocks_for(Nm)), dim3(256), 0, stream, a, S, Mm);
    else
        hipLaunchKernelGGL(macro_average_kernel<false>, dim3(blocks_for(Nm)), dim3(256), 0, stream, a, S, Mm);
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

static unsigned march_blocks(const AtomArgs& a) {
    return (unsigned)(((a.nx + MTX - 1) / MTX) * ((a.ny + MTY - 1) / MTY) * ((a.nz + MZC - 1) / MZC));
}

int launch_heun_predict(const AtomArgs& a, const float* S, const float* Hdm, float* f0, float* Sp,
                        hipStream_t stream) {
    hipLaunchKernelGGL(heun_march_kernel<0>, dim3(march_blocks(a)), dim3(MTX * MTY), 0, stream, a, S,
                       Hdm, f0, Sp);
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

int launch_heun_correct(const AtomArgs& a, float* S, const float* Sp, const float* f0,
                        const float* Hdm, hipStream_t stream) {
    hipLaunchKernelGGL(heun_march_kernel<1>, dim3(march_blocks(a)), dim3(MTX * MTY), 0, stream, a, Sp,
                       Hdm, const_cast<float*>(f0), S);
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

}  // namespace dm
