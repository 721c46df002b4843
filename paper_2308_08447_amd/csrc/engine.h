// engine.h -- internal declarations shared by the HIP sources of the demag engine.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/demag.h"

namespace dm {

// ---- error reporting --------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
// Evaluate a HIP call; on failure record the message and return DEMAG_EHIP.
#define DM_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::dm::fail(DEMAG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)
#define DM_CHECK_LAUNCH() DM_HIP(hipGetLastError())

// ---- stage timing -----------------------------------------------------------
// While a plan's stage timer is open on this thread, the next kernel started
// through DM_LAUNCH takes the timer's start and stop events
// (hipExtLaunchKernelGGL), so they record the kernel's own start and end
// rather than queue positions around its dispatch.  Otherwise DM_LAUNCH is a
// plain launch.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchEvents g_launch_events;
#define DM_LAUNCH(KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                                     \
    do {                                                                                       \
        const ::dm::LaunchEvents ev_ = ::dm::g_launch_events;                                  \
        ::dm::g_launch_events = ::dm::LaunchEvents{};                                          \
        if (ev_.start)                                                                         \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, ev_.start, ev_.stop, 0u,  \
                                  __VA_ARGS__);                                                \
        else                                                                                   \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);               \
    } while (0)

// ---- geometry ---------------------------------------------------------------
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

struct Geometry {
    int nx, ny, nz;        // cells
    int Nx, Ny, Nz;        // transform lengths: 2n (open axis), n (periodic), 1 when n = 1
    int X1, Y1, Z1;        // distinct folded frequencies: N/2 + 1, or 1
    int pbc = 0;           // periodic axes: bit 0 x, bit 1 y, bit 2 z
    int images = 0;        // periodic images summed on each side of a periodic axis
    int Rx, Ry, Rz;        // tensor octant extents: n (open), n/2 + 1 (periodic)
    bool px() const { return pbc & 1; }
    bool py() const { return (pbc >> 1) & 1; }
    bool pz() const { return (pbc >> 2) & 1; }
    size_t cells() const { return (size_t)nx * ny * nz; }
    size_t s1_elems() const { return (size_t)3 * nz * X1 * ny; }   // complex
    size_t s2_elems() const { return (size_t)3 * nz * X1 * Ny; }   // complex
    size_t k_elems() const { return (size_t)6 * Z1 * X1 * Y1; }    // real
};

// Returns DEMAG_OK or an error code (and message) for a mesh the kernels cannot take.
// pbc: periodic axes (bit 0 x, 1 y, 2 z); images: copies summed on each side.
int make_geometry(int nx, int ny, int nz, int pbc, int images, Geometry* g);

// ---- FFT stage launchers (stages_*.hip) ---------------------------------------
// periodic = true: the axis of the stage is periodic, its transform has the
// mesh length n (no zero padding) and every output is kept; FP32 and the
// middle tile variant only.
// A launch processes a batch of up to MAXB independent work items (one mesh
// each) that share the stage's transform length; the descriptors travel in the
// kernel arguments, so launches need no device-side tables and can be captured
// in graphs.  tw_all: the twiddle table, length-L part at tw_all + tw_offset(L).
constexpr int MAXB = 16;
constexpr int NVARIANTS = 3;

struct XDesc {            // x stages: M -> S1 (forward), S1 -> H (inverse)
    const float* M;
    float* H;
    float2* S1;           // [3][nz][X1][ny]
    int ny, nz;
    float scale;          // forward input scale (Ms for unit-vector input)
};
struct YDesc {            // y stages over kx planes [k0, k0 + nk) of one mesh
    float2* S1;
    float2* S2;           // chunk buffer [3][nz][xc][Ny]
    int X1, nz, k0, nk, xc;
};
struct ZDesc {            // z convolution over kx planes [k0, k0 + nk)
    float2* S2;           // chunk buffer (== S1 with xc = X1 when ny == 1)
    const float* K;       // [6][Z1][X1][Y1]
    int X1, Ny, Y1, Z1, k0, nk, xc;
};
template <class D>
struct StageBatch {
    D d[MAXB];
    int start[MAXB + 1];  // block prefix sums (filled by the launcher)
    int count;
};
// three-kernel form for thin meshes (stages_xz.hip); nx, nz and ny are launch constants
struct XZDesc {
    const float* M;       // xz forward input
    float* H;             // xz inverse output
    float2* T;            // [3][Nz][G][ny][4] spectra
    int ny;
    float scale;          // applied to M
};
struct YCDesc {
    float2* T;
    const float* K;       // [6][Z1][X1][Y1]
    int X1, Y1, Z1, G;
};
using XZBatch = StageBatch<XZDesc>;
using YCBatch = StageBatch<YCDesc>;
using XBatch = StageBatch<XDesc>;
using YBatch = StageBatch<YDesc>;
using ZBatch = StageBatch<ZDesc>;

int launch_x_forward(XBatch b, int nx, int variant, int mf, const float2* tw, hipStream_t s,
                     bool periodic = false);
int launch_x_inverse(XBatch b, int nx, int variant, int mf, const float2* tw, hipStream_t s,
                     bool periodic = false);
int launch_y_forward(YBatch b, int ny, int variant, int mf, const float2* tw, hipStream_t s,
                     bool periodic = false);
int launch_y_inverse(YBatch b, int ny, int variant, int mf, const float2* tw, hipStream_t s,
                     bool periodic = false);
int launch_z_convolve(ZBatch b, int Nz, int variant, int mf, const float2* tw, hipStream_t s,
                      bool periodic = false);
bool xz_supported(int nx, int ny, int nz);
size_t xz_t_elems(int nx, int ny, int nz);
int xz_groups(int X1);  // kx groups of T
// variant: the tile variant of the stage (xz: row pairs per round; y conv: the
// thread count and with it the radix order)
int launch_xz_forward(XZBatch b, int nx, int nz, int variant, const float2* tw, hipStream_t s);
int launch_yconv(YCBatch b, int ny, int Nz, int variant, const float2* tw, hipStream_t s);
int launch_xz_inverse(XZBatch b, int nx, int nz, int variant, const float2* tw, hipStream_t s);
// Twiddle table: exp(-2 pi i t/L), t < L, for every supported length L <= 4096
// (2^k and F 2^k, F = 3, 5, 15), the table of length L at tw_offset(L).  The
// regions are disjoint: 2^k at [2^k, 2^(k+1)), 3 2^k at 8192 + 4 2^k, 5 2^k at
// 16384 + 8 2^k, 15 2^k at 24576 + 16 2^k.
constexpr int TW_LMAX = 4096;
constexpr int TW_ENTRIES = 32768;
constexpr int tw_odd_part(int n) { return (n > 0 && n % 2 == 0) ? tw_odd_part(n / 2) : n; }
constexpr int tw_offset(int L) {
    return tw_odd_part(L) == 1    ? L
           : tw_odd_part(L) == 3 ? 8192 + 4 * (L / 3)
           : tw_odd_part(L) == 5 ? 16384 + 8 * (L / 5)
                                  : 24576 + 16 * (L / 15);
}
// Fills the host table (TW_ENTRIES float2).
void fill_twiddles(float2* host);

// ---- N^ set-up (tensor.hip) ---------------------------------------------------
// Computes the packed FP32 kernel K (device) for the geometry and cell, in FP64.
int compute_kernel(const Geometry& g, double dx, double dy, double dz, int kind, float* K,
                   hipStream_t stream);

// ---- dynamics (dynamics.hip) ----------------------------------------------------
struct LLGDesc {           // one mesh in a batched RK4 stage update
    const float* m;        // step start
    const float* ms;       // stage input
    const float* Hd;       // demagnetizing field of Ms * ms
    float* acc;
    float* out;            // next stage input (may alias m in the last stage)
    int nx, ny, nz;
    float cx, cy, cz;      // 2A/(mu0 Ms h_d^2), 0 for an axis with one cell
    int pbc;               // periodic axes (bit 0 x, 1 y, 2 z): neighbours wrap around
    float hz[3];
    float gam;             // gamma/(1+alpha^2)
    float alpha;
    float dt;
};
using LLGBatch = StageBatch<LLGDesc>;
int launch_llg_stage(LLGBatch b, int stage, hipStream_t stream);
// out = sum_j w[j] h[j] over n floats (polynomial extrapolation of a field)
int launch_extrapolate(float* out, const float* const h[5], const float w[5], size_t n,
                       hipStream_t stream);

// out[c] = mean over the n cells of component c of the [3][n] field v (device)
int launch_field_mean(const float* v, size_t n, float* out, hipStream_t stream);

struct AtomArgs {
    int nx, ny, nz, macro;
    float cex;             // J/(mu0 mu_B mu_s)
    float hz[3];
    float gam, alpha, dt;
    float mscale;          // mu_s mu_B/(a^3 N_S)
};
int launch_macro_average(const AtomArgs& a, const float* S, float* Mm, hipStream_t stream);
int launch_heun_predict(const AtomArgs& a, const float* S, const float* Hdm, float* f0,
                        float* Sp, hipStream_t stream);
int launch_heun_correct(const AtomArgs& a, float* S, const float* Sp, const float* f0,
                        const float* Hdm, hipStream_t stream);

}  // namespace dm
