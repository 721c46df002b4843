// tensor.hip -- the transformed demagnetizing tensor N^ ("convolution kernel" of
// App. A, computed at initialisation as in Sec. II), in FP64 on the GPU.
//
// 1. N(r) on the octant r = (i dx, j dy, k dz), 0 <= i < nx, 0 <= j < ny,
//    0 <= k < nz, in units of h = max(dx, dy, dz):
//    * |r| <= RC h: Newell's closed forms (f for the diagonal, g for the
//      off-diagonal components) through the 27-point second-difference stencil,
//      weights 2 / -1 per axis;
//    * beyond: moment expansion of the cell-pair average,
//        N_ab ~= -V/(4 pi) [phi_ab + sum_d h_d^2/12 phi_abdd + sum_d h_d^4/360 phi_abdddd
//                          + sum_{d<e} h_d^2 h_e^2/144 phi_abddee],   phi = 1/|r|,
//      where the partial derivatives of 1/r come from the recursion obtained by
//      differentiating r^2 d_i phi = -x_i phi (Leibniz rule), order by order.
// 2. The padded tensor (index r mod N_d, entry n_d left 0) is real and has a
//    parity in every axis (diagonal even; N_ab odd in a and b), so its DFT along
//    one axis is a cosine sum (even) or -i times a sine sum (odd) over r >= 0:
//      E(k) = N(0) + 2 sum_{r>=1} N(r) cos(2 pi k r/N_d),
//      O(k) = 2 sum_{r>=1} N(r) sin(2 pi k r/N_d).
//    Each axis pass is a small FP64 matrix product with a trigonometric matrix;
//    three passes give the real transformed components at the (n_d+1) folded
//    frequencies per axis (the y/z symmetry packing of App. A).
// 3. K = -(-1)^{#odd axes/2} ... stored as FP32: K_ab = -N^_ab/(Nx Ny Nz) with
//    the (-i)^2 = -1 of the two odd axes of an off-diagonal component folded in.
// Periodic axes (Sec. II: modified kernel, no padding): the transform length is
// n_d, the octant is r_d <= n_d/2, N is the sum over the periodic images of the
// body (tensor_image_kernel), and r_d = n_d/2, its own mirror, enters the
// cosine sum once; the sine sums vanish there.
#include <cmath>
#include <vector>

#include "engine.h"

namespace dm {

namespace {

constexpr double RC = 16.0;
constexpr double PI = 3.141592653589793238462643383279502884;

__device__ double newell_f(double x, double y, double z) {
    x = fabs(x);
    y = fabs(y);
    z = fabs(z);
    double x2 = x * x, y2 = y * y, z2 = z * z;
    double R = sqrt(x2 + y2 + z2);
    double res = (2.0 * x2 - y2 - z2) * R / 6.0;
    double q = sqrt(x2 + z2);
    if (q > 0.0) res += 0.5 * y * (z2 - x2) * asinh(y / q);
    q = sqrt(x2 + y2);
    if (q > 0.0) res += 0.5 * z * (y2 - x2) * asinh(z / q);
    q = x * R;
    if (q > 0.0) res -= x * y * z * atan(y * z / q);
    return res;
}

__device__ double newell_g(double x, double y, double z) {
    double x2 = x * x, y2 = y * y, z2 = z * z;
    double R = sqrt(x2 + y2 + z2);
    double res = -x * y * R / 3.0;
    double q = sqrt(x2 + y2);
    if (q > 0.0) res += x * y * z * asinh(z / q);
    q = sqrt(y2 + z2);
    if (q > 0.0) res += y / 6.0 * (3.0 * z2 - y2) * asinh(x / q);
    q = sqrt(x2 + z2);
    if (q > 0.0) res += x / 6.0 * (3.0 * z2 - x2) * asinh(y / q);
    q = z * R;
    if (q != 0.0) res -= z2 * z / 6.0 * atan(x * y / q);
    q = y * R;
    if (q != 0.0) res -= z * y2 / 2.0 * atan(x * z / q);
    q = x * R;
    if (q != 0.0) res -= z * x2 / 2.0 * atan(y * z / q);
    return res;
}

// 27-point second-difference stencil of f or g
template <bool DIAG>
__device__ double stencil(double X, double Y, double Z, double hx, double hy, double hz) {
    const double w[3] = {-1.0, 2.0, -1.0};
    double acc = 0.0;
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q)
            for (int s = 0; s < 3; ++s) {
                double a = X + (p - 1) * hx, b = Y + (q - 1) * hy, c = Z + (s - 1) * hz;
                double v = DIAG ? newell_f(a, b, c) : newell_g(a, b, c);
                acc += w[p] * w[q] * w[s] * v;
            }
    return acc;
}

// Index of multi-index (a, b, c), a + b + c <= 6, in a packed table of 84 entries.
__device__ __forceinline__ int midx(int a, int b, int c) {
    // orders are stored by total order n, then a descending, then b descending
    int n = a + b + c;
    int before = n * (n + 1) * (n + 2) / 6;          // entries of lower total order
    int r = n - a;                                   // remaining for b + c
    int within = (n - a) * (n - a + 1) / 2 + (r - b); // a descending, b descending
    return before + within;
}

// All partial derivatives d^a_x d^b_y d^c_z (1/r), a + b + c <= 6, into F[84].
__device__ void inverse_r_derivatives(double x, double y, double z, double* F) {
    const double X[3] = {x, y, z};
    double r2 = x * x + y * y + z * z;
    double inv_r2 = 1.0 / r2;
    F[0] = sqrt(inv_r2);
    for (int n = 1; n <= 6; ++n) {
        for (int a = n; a >= 0; --a) {
            for (int b = n - a; b >= 0; --b) {
                int c = n - a - b;
                int al[3] = {a, b, c};
                int i = (a > 0) ? 0 : ((b > 0) ? 1 : 2);
                int be[3] = {al[0], al[1], al[2]};
                be[i] -= 1;  // beta = alpha - e_i
                // r^2 F[beta+e_i] = -x_i F[beta] - beta_i F[beta-e_i]
                //   - 2 sum_j beta_j x_j F[beta+e_i-e_j] - sum_j beta_j(beta_j-1) F[beta+e_i-2e_j]
                double acc = -X[i] * F[midx(be[0], be[1], be[2])];
                if (be[i] > 0) {
                    int t[3] = {be[0], be[1], be[2]};
                    t[i] -= 1;
                    acc -= be[i] * F[midx(t[0], t[1], t[2])];
                }
                for (int j = 0; j < 3; ++j) {
                    if (be[j] > 0) {
                        int t[3] = {al[0], al[1], al[2]};
                        t[j] -= 1;
                        acc -= 2.0 * be[j] * X[j] * F[midx(t[0], t[1], t[2])];
                    }
                    if (be[j] > 1) {
                        int t[3] = {al[0], al[1], al[2]};
                        t[j] -= 2;
                        acc -= (double)be[j] * (be[j] - 1) * F[midx(t[0], t[1], t[2])];
                    }
                }
                F[midx(a, b, c)] = acc * inv_r2;
            }
        }
    }
}

__device__ void tensor_far(double x, double y, double z, double hx, double hy, double hz,
                           double* out) {
    double F[84];
    inverse_r_derivatives(x, y, z, F);
    const double H[3] = {hx, hy, hz};
    const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
    const double V = hx * hy * hz;
    for (int comp = 0; comp < 6; ++comp) {
        int base[3] = {0, 0, 0};
        base[pa[comp]] += 1;
        base[pb[comp]] += 1;
        double s = F[midx(base[0], base[1], base[2])];
        for (int d = 0; d < 3; ++d) {
            int t2[3] = {base[0], base[1], base[2]};
            t2[d] += 2;
            int t4[3] = {base[0], base[1], base[2]};
            t4[d] += 4;
            double h2 = H[d] * H[d];
            s += h2 / 12.0 * F[midx(t2[0], t2[1], t2[2])];
            s += h2 * h2 / 360.0 * F[midx(t4[0], t4[1], t4[2])];
            for (int e = d + 1; e < 3; ++e) {
                int t[3] = {base[0], base[1], base[2]};
                t[d] += 2;
                t[e] += 2;
                s += h2 * H[e] * H[e] / 144.0 * F[midx(t[0], t[1], t[2])];
            }
        }
        out[comp] = -V / (4.0 * PI) * s;
    }
}

// N at displacement (X, Y, Z) (units of h).  kind 0: the cell-averaged tensor of
// Eq. (1) (Newell near, moment expansion far); kind 1: the point-dipole tensor of
// Eq. (8), V (delta |r|^2 - 3 r r)/(4 pi |r|^5) with N(0) = 0 (site i excluded).
__device__ void tensor_point(double X, double Y, double Z, double hx, double hy, double hz,
                             int kind, double* out) {
    const double r2 = X * X + Y * Y + Z * Z;
    if (kind == 1) {
        const double c = r2 > 0.0 ? hx * hy * hz / (4.0 * PI * r2 * r2 * sqrt(r2)) : 0.0;
        out[0] = c * (r2 - 3.0 * X * X);
        out[1] = c * (r2 - 3.0 * Y * Y);
        out[2] = c * (r2 - 3.0 * Z * Z);
        out[3] = c * (-3.0 * X * Y);
        out[4] = c * (-3.0 * X * Z);
        out[5] = c * (-3.0 * Y * Z);
    } else if (r2 <= RC * RC) {
        double c = 1.0 / (4.0 * PI * hx * hy * hz);
        out[0] = c * stencil<true>(X, Y, Z, hx, hy, hz);
        out[1] = c * stencil<true>(Y, X, Z, hy, hx, hz);
        out[2] = c * stencil<true>(Z, Y, X, hz, hy, hx);
        out[3] = c * stencil<false>(X, Y, Z, hx, hy, hz);
        out[4] = c * stencil<false>(X, Z, Y, hx, hz, hy);
        out[5] = c * stencil<false>(Y, Z, X, hy, hz, hx);
    } else {
        tensor_far(X, Y, Z, hx, hy, hz, out);
    }
}

// N on the octant; T0[6][nz][ny][nx].
__global__ void tensor_octant_kernel(double* __restrict__ T0, int nx, int ny, int nz,
                                     double hx, double hy, double hz, int kind) {
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t n = (size_t)nx * ny * nz;
    if (idx >= n) return;
    int i = (int)(idx % nx);
    int j = (int)((idx / nx) % ny);
    int k = (int)(idx / ((size_t)nx * ny));
    double out[6];
    tensor_point(i * hx, j * hy, k * hz, hx, hy, hz, kind, out);
    for (int comp = 0; comp < 6; ++comp) T0[(size_t)comp * n + idx] = out[comp];
}

// Moment expansion of the cell-pair tensor through its h^2 term,
//   N_ab ~= -V/(4 pi) [phi_ab + sum_d h_d^2/12 phi_abdd],  phi = 1/|r|,
// with the closed forms phi_ab = (3 x_a x_b - delta_ab r^2)/r^5 and
//   sum_d h_d^2 phi_abdd = 105 x_a x_b S/r^9
//       - 15 (delta_ab S + 2 (h_a^2 + h_b^2) x_a x_b + H x_a x_b)/r^7
//       + 3 delta_ab (H + 2 h_a^2)/r^5,   S = sum_d h_d^2 x_d^2, H = sum_d h_d^2
// (the derivative of 1/r of order four contracted over one index pair).  Its
// relative error falls as (h/r)^4: about 1e-8 at r = 64 h.
__device__ void tensor_h2(double x, double y, double z, double hx, double hy, double hz,
                          double* out) {
    const double X[3] = {x, y, z}, H2[3] = {hx * hx, hy * hy, hz * hz};
    const double r2 = x * x + y * y + z * z;
    const double ir2 = 1.0 / r2;
    const double ir5 = ir2 * ir2 * sqrt(ir2);
    const double ir7 = ir5 * ir2, ir9 = ir7 * ir2;
    const double S = H2[0] * x * x + H2[1] * y * y + H2[2] * z * z;
    const double Hs = H2[0] + H2[1] + H2[2];
    const double c = -hx * hy * hz / (4.0 * PI);
    const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
    for (int comp = 0; comp < 6; ++comp) {
        const int a = pa[comp], b = pb[comp];
        const double xab = X[a] * X[b];
        const double d = a == b ? 1.0 : 0.0;
        const double phi = (3.0 * xab - d * r2) * ir5;
        const double t4 = 105.0 * xab * S * ir9 -
                          15.0 * (d * S + 2.0 * (H2[a] + H2[b]) * xab + Hs * xab) * ir7 +
                          3.0 * d * (Hs + 2.0 * H2[a]) * ir5;
        out[comp] = c * (phi + t4 / 12.0);
    }
}

// Periodic image sum on the octant r_d < R_d; T0[6][Rz][Ry][Rx]:
//   N_pbc(r) = sum_m N(r + m_x n_x hx e_x + m_y n_y hy e_y + m_z n_z hz e_z),
// |m_d| <= P_d (P along periodic axes, 0 otherwise).  The image m = 0 is the
// open tensor; the others use it up to RF h and the h^2 expansion beyond.  A
// component odd in a periodic axis is zero at r_d = n_d/2 (the infinite sum is
// odd and periodic there).
constexpr double RF = 64.0;
__global__ void tensor_image_kernel(double* __restrict__ T0, int Rx, int Ry, int Rz, int nx,
                                    int ny, int nz, int pbc, int P, double hx, double hy,
                                    double hz, int kind) {
    const int Px = (pbc & 1) ? P : 0, Py = (pbc & 2) ? P : 0, Pz = (pbc & 4) ? P : 0;
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t n = (size_t)Rx * Ry * Rz;
    if (idx >= n) return;
    const int i = (int)(idx % Rx);
    const int j = (int)((idx / Rx) % Ry);
    const int k = (int)(idx / ((size_t)Rx * Ry));
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int mz = -Pz; mz <= Pz; ++mz)
        for (int my = -Py; my <= Py; ++my)
            for (int mx = -Px; mx <= Px; ++mx) {
                const double X = (i + (double)mx * nx) * hx;
                const double Y = (j + (double)my * ny) * hy;
                const double Z = (k + (double)mz * nz) * hz;
                double out[6];
                const bool centre = mx == 0 && my == 0 && mz == 0;
                if (centre || kind == 1 || X * X + Y * Y + Z * Z <= RF * RF)
                    tensor_point(X, Y, Z, hx, hy, hz, kind, out);
                else
                    tensor_h2(X, Y, Z, hx, hy, hz, out);
                for (int c = 0; c < 6; ++c) acc[c] += out[c];
            }
    // odd components (xy: x, y; xz: x, z; yz: y, z) at the half-period displacement
    const bool hx0 = (pbc & 1) && nx >= 2 && nx % 2 == 0 && i == nx / 2;
    const bool hy0 = (pbc & 2) && ny >= 2 && ny % 2 == 0 && j == ny / 2;
    const bool hz0 = (pbc & 4) && nz >= 2 && nz % 2 == 0 && k == nz / 2;
    if (hx0 || hy0) acc[3] = 0.0;
    if (hx0 || hz0) acc[4] = 0.0;
    if (hy0 || hz0) acc[5] = 0.0;
    for (int c = 0; c < 6; ++c) T0[(size_t)c * n + idx] = acc[c];
}

// C[b][i][j] = scale * sum_r A(b,i,r) B(b,r,j), strided FP64; 64x64 tiles, 16x16 threads.
template <typename TOUT>
__global__ __launch_bounds__(256) void gemm_f64_kernel(
    const double* __restrict__ A, long as_b, long as_i, long as_r,
    const double* __restrict__ B, long bs_b, long bs_r, long bs_j,
    TOUT* __restrict__ C, long cs_b, long cs_i, long cs_j, int M, int N, int K, double scale) {
    __shared__ double As[16][65];
    __shared__ double Bs[16][65];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64, b = blockIdx.z;
    A += b * as_b;
    B += b * bs_b;
    C += b * cs_b;
    double acc[4][4] = {};
    for (int r0 = 0; r0 < K; r0 += 16) {
        for (int e = threadIdx.x; e < 1024; e += 256) {
            int ii = e % 64, rr = e / 64;
            int gi = i0 + ii, gr = r0 + rr;
            As[rr][ii] = (gi < M && gr < K) ? A[gi * as_i + gr * as_r] : 0.0;
            int jj = e % 64;
            int gj = j0 + jj;
            Bs[rr][jj] = (gj < N && gr < K) ? B[gr * bs_r + gj * bs_j] : 0.0;
        }
        __syncthreads();
        for (int rr = 0; rr < 16; ++rr) {
            double a[4], bb[4];
            for (int u = 0; u < 4; ++u) a[u] = As[rr][ty + 16 * u];
            for (int v = 0; v < 4; ++v) bb[v] = Bs[rr][tx + 16 * v];
            for (int u = 0; u < 4; ++u)
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], bb[v], acc[u][v]);
        }
        __syncthreads();
    }
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) {
            int gi = i0 + ty + 16 * u, gj = j0 + tx + 16 * v;
            if (gi < M && gj < N) C[gi * cs_i + gj * cs_j] = (TOUT)(scale * acc[u][v]);
        }
}

template <typename TOUT>
int gemm(const double* A, long as_b, long as_i, long as_r, const double* B, long bs_b, long bs_r,
         long bs_j, TOUT* C, long cs_b, long cs_i, long cs_j, int M, int N, int K, int batch,
         double scale, hipStream_t s) {
    dim3 grid((N + 63) / 64, (M + 63) / 64, batch);
    hipLaunchKernelGGL((gemm_f64_kernel<TOUT>), grid, dim3(256), 0, s, A, as_b, as_i, as_r, B,
                       bs_b, bs_r, bs_j, C, cs_b, cs_i, cs_j, M, N, K, scale);
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

// Trigonometric matrix [D1][R] of one axis for even (cos) or odd (sin) parity,
// over the octant displacements r < R.  Displacement r stands for the transform
// indices r and N_d - r: weight 2, except r = 0 and (periodic axis) r = N_d/2,
// which occur once.
std::vector<double> trig_matrix(int R, int Nd, int D1, bool odd) {
    std::vector<double> T((size_t)D1 * R, 0.0);
    for (int k = 0; k < D1; ++k)
        for (int r = 0; r < R; ++r) {
            if (Nd == 1) {
                T[(size_t)k * R + r] = odd ? 0.0 : 1.0;
                continue;
            }
            long t = ((long)k * r) % Nd;
            long double ang = 2.0L * 3.141592653589793238462643383279502884L * t / Nd;
            double w = (r == 0) ? (odd ? 0.0 : 1.0) : (2 * r == Nd ? 1.0 : 2.0);
            T[(size_t)k * R + r] = w * (double)(odd ? sinl(ang) : cosl(ang));
        }
    return T;
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

int compute_kernel(const Geometry& g, double dx, double dy, double dz, int kind, float* K,
                   hipStream_t stream) {
    // octant extents (n, or n/2 + 1 along a periodic axis)
    const int nx = g.Rx, ny = g.Ry, nz = g.Rz, X1 = g.X1, Y1 = g.Y1, Z1 = g.Z1;
    const double h = std::fmax(dx, std::fmax(dy, dz));
    const size_t n0 = (size_t)nx * ny * nz;
    const size_t n1 = (size_t)nz * X1 * ny;
    const size_t n2 = (size_t)nz * X1 * Y1;
    DevBuf T0, T1, T2, trig;
    DM_HIP(hipMalloc(&T0.p, 6 * n0 * sizeof(double)));
    DM_HIP(hipMalloc(&T1.p, 6 * n1 * sizeof(double)));
    DM_HIP(hipMalloc(&T2.p, 6 * n2 * sizeof(double)));
    // (a failed set-up allocation is reported as DEMAG_EHIP with the HIP error text)

    // trig matrices: [axis][parity] blocks
    std::vector<double> host;
    size_t off[3][2];
    const int ns[3] = {nx, ny, nz}, Ns[3] = {g.Nx, g.Ny, g.Nz}, Ds[3] = {X1, Y1, Z1};
    for (int ax = 0; ax < 3; ++ax)
        for (int odd = 0; odd < 2; ++odd) {
            off[ax][odd] = host.size();
            auto T = trig_matrix(ns[ax], Ns[ax], Ds[ax], odd != 0);
            host.insert(host.end(), T.begin(), T.end());
        }
    DM_HIP(hipMalloc(&trig.p, host.size() * sizeof(double)));
    DM_HIP(hipMemcpyAsync(trig.p, host.data(), host.size() * sizeof(double),
                          hipMemcpyHostToDevice, stream));
    const double* TR = (const double*)trig.p;

    if (g.pbc)
        hipLaunchKernelGGL(tensor_image_kernel, dim3((unsigned)((n0 + 127) / 128)), dim3(128), 0,
                           stream, (double*)T0.p, nx, ny, nz, g.nx, g.ny, g.nz, g.pbc, g.images,
                           dx / h, dy / h, dz / h, kind);
    else
        hipLaunchKernelGGL(tensor_octant_kernel, dim3((unsigned)((n0 + 127) / 128)), dim3(128), 0,
                           stream, (double*)T0.p, nx, ny, nz, dx / h, dy / h, dz / h, kind);
    DM_CHECK_LAUNCH();

    // parity (x, y, z) per component: xx yy zz xy xz yz
    const int par[6][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
    const double norm = 1.0 / ((double)g.Nx * g.Ny * g.Nz);
    for (int c = 0; c < 6; ++c) {
        const double* t0 = (const double*)T0.p + c * n0;
        double* t1 = (double*)T1.p + c * n1;
        double* t2 = (double*)T2.p + c * n2;
        // x: T1[z][kx][y] = sum_r Tx[kx][r] T0[z][y][r]
        int rc = gemm<double>(TR + off[0][par[c][0]], 0, nx, 1, t0, (long)ny * nx, 1, nx, t1,
                              (long)X1 * ny, ny, 1, X1, ny, nx, nz, 1.0, stream);
        if (rc) return rc;
        // y: T2[z][kx][ky] = sum_r T1[z][kx][r] Ty[ky][r]
        rc = gemm<double>(t1, (long)X1 * ny, ny, 1, TR + off[1][par[c][1]], 0, 1, ny, t2,
                          (long)X1 * Y1, Y1, 1, X1, Y1, ny, nz, 1.0, stream);
        if (rc) return rc;
        // z: K[c][kz][kx ky] = s * sum_r Tz[kz][r] T2[r][kx ky]
        bool offdiag = c >= 3;
        double s = offdiag ? norm : -norm;
        rc = gemm<float>(TR + off[2][par[c][2]], 0, nz, 1, t2, 0, (long)X1 * Y1, 1,
                         K + (size_t)c * Z1 * X1 * Y1, 0, (long)X1 * Y1, 1, Z1, X1 * Y1, nz, 1, s,
                         stream);
        if (rc) return rc;
    }
    DM_HIP(hipStreamSynchronize(stream));
    return DEMAG_OK;
}

}  // namespace dm
