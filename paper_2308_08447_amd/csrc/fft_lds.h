// fft_lds.h -- batched complex FFTs held in LDS, for gfx950.
//
// A workgroup transforms NLINES lines of length L that sit in LDS.  Each radix
// pass is a Stockham autosort step: butterfly j (0 <= j < L/R) of the pass with
// current sub-transform size Ns reads x[j + r L/R] (r < R), multiplies element r
// by W^(r (j mod Ns)) with W = exp(-+2 pi i/(Ns R)), does an R-point DFT in
// registers and writes element r to (j/Ns) Ns R + (j mod Ns) + r Ns.  After the
// last pass the line is in natural order.  Power-of-two lengths use radices
// 2..16, chosen so the passes are as even as possible (e.g. 1024 = 16*8*8).
// Lengths F 2^k with F = 3, 5 or 15 (k >= 1) add radix-3 and radix-5 passes
// between a first and a last power-of-two pass (e.g. 960 = 8*3*5*8), so that
// the first pass can skip zero inputs and the last pass drop outputs.
//
// Twiddles come from a table of exp(-2 pi i t/L), t < L, rounded from FP64 on
// the host, so every twiddle is correctly rounded (no recurrence, no
// hardware sin/cos approximation).  The passes take the table through any
// indexable TW: a pointer, or an accessor that forms the value from a smaller
// table (then within a rounding or two of the correctly rounded value).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "mfma_dft.h"

namespace dm {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// Device code is compiled with -ffp-contract=off: every fused multiply-add is
// written out, so the rounding of each line's arithmetic is fixed by the source
// and does not depend on how a kernel instantiation is unrolled or scheduled.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// c + a b in four fused multiply-adds
__device__ __forceinline__ float2 cmad(float2 a, float2 b, float2 c) {
    return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (DIR = -1) or +i (DIR = +1)
template <int DIR>
__device__ __forceinline__ float2 mul_i(float2 a) {
    if constexpr (DIR < 0) return make_float2(a.y, -a.x);
    else return make_float2(-a.y, a.x);
}

constexpr bool is_pow2_radix(int r) { return r >= 2 && r <= 16 && (r & (r - 1)) == 0; }

// exp(DIR * 2 pi i k / 16), k < 8, as literal constants
template <int DIR>
__device__ __forceinline__ float2 w16(int k) {
    constexpr float c1 = 0.92387953251128676f, s1 = 0.38268343236508977f, h = 0.70710678118654752f;
    float2 w;
    switch (k) {
        case 1: w = make_float2(c1, s1); break;
        case 2: w = make_float2(h, h); break;
        case 3: w = make_float2(s1, c1); break;
        case 5: w = make_float2(-s1, c1); break;
        case 6: w = make_float2(-h, h); break;
        case 7: w = make_float2(-c1, s1); break;
        default: w = make_float2(1.f, 0.f); break;
    }
    if constexpr (DIR < 0) w.y = -w.y;
    return w;
}

// exp(DIR 2 pi i k / 16) for any k (reduced mod 16), exact constants
template <int DIR>
__device__ __forceinline__ float2 w16f(int k) {
    k &= 15;
    if (k < 8) return w16<DIR>(k);
    float2 w = w16<DIR>(k - 8);
    return make_float2(-w.x, -w.y);
}

// exp(DIR 2 pi i k / 32) for any k, exact constants (odd k from cos and sin of
// pi/16 and 3 pi/16 by quadrant symmetry)
template <int DIR>
__device__ __forceinline__ float2 w32f(int k) {
    k &= 31;
    if ((k & 1) == 0) return w16f<DIR>(k >> 1);
    constexpr float c1 = 0.98078528040323044f, s1 = 0.19509032201612826f;
    constexpr float c3 = 0.83146961230254524f, s3 = 0.55557023301960222f;
    const int q = k >> 3, j = k & 7;  // k = 8 q + j, angle = q pi/2 + j pi/16
    float2 w = j == 1 ? make_float2(c1, s1) : j == 3 ? make_float2(c3, s3)
             : j == 5 ? make_float2(s3, c3) : make_float2(s1, c1);
    for (int t = 0; t < q; ++t) w = make_float2(-w.y, w.x);  // times i per quarter turn
    if constexpr (DIR < 0) w.y = -w.y;
    return w;
}

// Butterfly (a, b) -> (a + f b, a - f b) in six operations: four fused
// multiply-adds form p = a + f b, and a - f b is taken as 2a - p.
__device__ __forceinline__ void bfly(float2& a, float2& b, float2 f) {
    const float px = fmaf(f.x, b.x, fmaf(-f.y, b.y, a.x));
    const float py = fmaf(f.x, b.y, fmaf(f.y, b.x, a.y));
    b = make_float2(fmaf(2.f, a.x, -px), fmaf(2.f, a.y, -py));
    a = make_float2(px, py);
}
// The same with f = 1 and with f = DIR i (four operations each).
__device__ __forceinline__ void bfly1(float2& a, float2& b) {
    const float2 p = cadd(a, b);
    b = csub(a, b);
    a = p;
}
template <int DIR>
__device__ __forceinline__ void bfly_i(float2& a, float2& b) {
    const float2 t = mul_i<DIR>(b);
    b = csub(a, t);
    a = cadd(a, t);
}

// Twiddle sources of the power-of-two DFT below.  The transform of size R
// (radix-2 decimation in time) combines at depth d sub-transforms of size
// S = R / 2^d with factors g_d omega_S^m (m < S/2, omega_S = exp(DIR 2 pi i/S)):
//   TwNone    g_d = 1: the plain DFT of v;
//   TwHalf    v[r] is weighted by omega_{2R}^r, so the factor is the exact
//             constant omega_{2S}^{2m+1} (the odd outputs of a length-2R DFT
//             whose upper R inputs are zero);
//   TwRun     v[r] is weighted by w^r for a run-time w, g_d = w^(2^d) taken
//             from p[d] (each a table entry, so no power is formed by repeated
//             products).
struct TwNone {};
struct TwHalf {};
struct TwRun {
    float2 p[4];
};

// Factor of combination m at depth D for a transform of size R (S = R >> D),
// applied as a butterfly; the trivial ones (1 and DIR i) skip the products.
template <int R, int D, int DIR, class TWS>
__device__ __forceinline__ void combine(float2& a, float2& b, int m, const TWS& tws) {
    constexpr int S = R >> D;
    if constexpr (std::is_same<TWS, TwNone>::value) {
        if (m == 0) bfly1(a, b);
        else if (4 * m == S) bfly_i<DIR>(a, b);
        else bfly(a, b, w16f<DIR>(m * (16 / S)));
    } else if constexpr (std::is_same<TWS, TwHalf>::value) {
        // omega_{2S}^{2m+1} = w32f((2m+1) 16/S); S = 2 gives omega_4 = DIR i
        if (S == 2) bfly_i<DIR>(a, b);
        else bfly(a, b, w32f<DIR>((2 * m + 1) * (16 / S)));
    } else {
        const float2 g = tws.p[D];
        if (m == 0) {
            bfly(a, b, g);
        } else if (4 * m == S) {
            bfly(a, b, mul_i<DIR>(g));
        } else if (4 * m < S) {
            bfly(a, b, cmul(g, w16f<DIR>(m * (16 / S))));
        } else {  // omega_S^m = DIR i omega_S^(m - S/4): the same product, rotated
            bfly(a, b, mul_i<DIR>(cmul(g, w16f<DIR>((m - S / 4) * (16 / S)))));
        }
    }
}

template <int R, int D, int DIR, class TWS>
__device__ __forceinline__ void dft2k_rec(float2* v, const TWS& tws) {
    constexpr int S = R >> D;
    if constexpr (S >= 2) {
        float2 e[S / 2], o[S / 2];
#pragma unroll
        for (int i = 0; i < S / 2; ++i) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        dft2k_rec<R, D + 1, DIR>(e, tws);
        dft2k_rec<R, D + 1, DIR>(o, tws);
#pragma unroll
        for (int m = 0; m < S / 2; ++m) {
            combine<R, D, DIR>(e[m], o[m], m, tws);
            v[m] = e[m];
            v[m + S / 2] = o[m];
        }
    }
}

// DFT of size R (a power of two <= 16) of v[r] g^r with g given by the twiddle
// source (see above), natural order in and out.
template <int R, int DIR, class TWS>
__device__ __forceinline__ void dft2k(float2* v, const TWS& tws) {
    static_assert(R >= 1 && R <= 16 && (R & (R - 1)) == 0, "power of two <= 16");
    dft2k_rec<R, 0, DIR>(v, tws);
}

// In-register DFT of size R: 3 and 5 by the symmetric-pair formulas, powers of
// two <= 16 by radix-2 decimation in time with multiply-add butterflies.
template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v) {
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 3) {
        // y_{1,2} = x0 - (x1 + x2)/2 +- DIR i sin(2 pi/3) (x1 - x2)
        constexpr float s = 0.86602540378443865f;
        float2 a = cadd(v[1], v[2]);
        float2 d = cscale(mul_i<DIR>(csub(v[1], v[2])), s);
        float2 t = csub(v[0], cscale(a, 0.5f));
        v[0] = cadd(v[0], a);
        v[1] = cadd(t, d);
        v[2] = csub(t, d);
    } else if constexpr (R == 5) {
        // pairs x1 +- x4, x2 +- x3 against cos and sin of 2 pi/5 and 4 pi/5
        constexpr float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
        constexpr float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;
        float2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
        float2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
        float2 x0 = v[0];
        float2 r1 = cadd(x0, cadd(cscale(a1, c1), cscale(a2, c2)));
        float2 r2 = cadd(x0, cadd(cscale(a1, c2), cscale(a2, c1)));
        float2 i1 = mul_i<DIR>(cadd(cscale(b1, s1), cscale(b2, s2)));
        float2 i2 = mul_i<DIR>(csub(cscale(b1, s2), cscale(b2, s1)));
        v[0] = cadd(x0, cadd(a1, a2));
        v[1] = cadd(r1, i1);
        v[4] = csub(r1, i1);
        v[2] = cadd(r2, i2);
        v[3] = csub(r2, i2);
    } else {
        dft2k<R, DIR>(v, TwNone{});
    }
}

// v * exp(DIR 2 pi i k / 16), k < 8
template <int DIR>
__device__ __forceinline__ float2 rot16(int k, float2 v) {
    if (k == 0) return v;
    if (k == 4) return mul_i<DIR>(v);
    return cmul(w16<DIR>(k), v);
}

// DFT of size R whose inputs R/2 .. R-1 are zero: the even outputs are the
// R/2-point DFT of x, the odd outputs the R/2-point DFT of x[r] W_R^r.
template <int R, int DIR>
__device__ __forceinline__ void dft_half_in(float2* v) {
    if constexpr (R <= 2) {
        v[1] = v[0];
    } else {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int r = 0; r < R / 2; ++r) {
            e[r] = v[r];
            o[r] = v[r];
        }
        dft2k<R / 2, DIR>(e, TwNone{});
        dft2k<R / 2, DIR>(o, TwHalf{});
#pragma unroll
        for (int m = 0; m < R / 2; ++m) {
            v[2 * m] = e[m];
            v[2 * m + 1] = o[m];
        }
    }
}

// Twiddled DFT of a Stockham pass: the DFT of v[r] w^r, w = tw[s] (conjugated
// for the inverse, DIR > 0).  Powers of two take w^(2^d) = tw[2^d s] as table
// entries; other radices multiply every input.
template <int R, int DIR, class TW>
__device__ __forceinline__ void dft_twiddled(float2* v, const TW& tw, int s) {
    if constexpr (is_pow2_radix(R)) {
        TwRun t;
#pragma unroll
        for (int d = 0; (1 << d) < R; ++d) {
            float2 w = tw[s << d];
            if constexpr (DIR > 0) w.y = -w.y;
            t.p[d] = w;
        }
        dft2k<R, DIR>(v, t);
    } else {
#pragma unroll
        for (int r = 1; r < R; ++r) {
            float2 w = tw[s * r];
            if constexpr (DIR > 0) w.y = -w.y;
            v[r] = cmul(v[r], w);
        }
        dft<R, DIR>(v);
    }
}

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }
constexpr int odd_part(int n) { return (n > 0 && n % 2 == 0) ? odd_part(n / 2) : n; }
constexpr bool is_pow2c(int n) { return odd_part(n) == 1; }

// Power-of-two passes of 2^k: ceil(k / 4) of them, bits spread evenly; with an
// odd factor at least two (first and last pass even) once k >= 2.
constexpr int pow2_passes(int k, bool mixed) {
    return (mixed && k >= 2 && (k + 3) / 4 < 2) ? 2 : (k + 3) / 4;
}
constexpr int pow2_radix(int k, int P, int q) {
    return P == 0 ? 1 : 1 << (k / P + (q < k % P ? 1 : 0));
}
constexpr int odd_passes(int F) { return F == 15 ? 2 : (F == 1 ? 0 : 1); }

// Radix of pass p for a length-L transform: the first power-of-two pass, then
// the odd radices (3, 5), then the remaining power-of-two passes.
constexpr int radix_of(int L, int p) {
    const int F = odd_part(L), k = ilog2c(L / F), P = pow2_passes(k, F > 1);
    const int no = odd_passes(F);
    if (F == 1) return pow2_radix(k, P, p);
    if (p == 0 && P > 0) return pow2_radix(k, P, 0);
    const int q = P > 0 ? p - 1 : p;           // index among the odd passes
    if (q < no) return F == 15 ? (q == 0 ? 3 : 5) : F;
    return pow2_radix(k, P, q - no + 1);
}
constexpr int npasses(int L) {
    const int F = odd_part(L);
    return pow2_passes(ilog2c(L / F), F > 1) + odd_passes(F);
}

// Radix plan of the split-precision MFMA transforms (MF > 0): every pass is
// radix 16 except a first pass that takes the remaining 2, 4 or 8 (e.g. 2048 =
// 8*16*16); the pass count is the same as above.
template <int MF>
constexpr int radix_at(int L, int p) {
    if constexpr (MF == 0) {
        return radix_of(L, p);
    } else {
        int k = ilog2c(L), rem = k % 4;
        if (k <= 4) return L;
        return (p == 0 && rem != 0) ? (1 << rem) : 16;
    }
}

// exp(-2 pi i t/L) as the product of a coarse entry t / 32 and a fine entry
// t % 32, both correctly rounded: ceil(L/32) + 32 table entries in LDS instead
// of L, for stages whose block count per compute unit the table would limit.
struct Tw2 {
    const float2* c;
    const float2* f;
    __device__ __forceinline__ float2 operator[](int t) const { return cmul(c[t >> 5], f[t & 31]); }
};
constexpr int tw2_entries(int L) { return (L + 31) / 32 + 32; }
// Fills dst[0 .. tw2_entries(L)) from the full table (block-strided, NT threads)
// and returns the accessor; the caller's next barrier publishes the entries.
template <int L, int NT>
__device__ __forceinline__ Tw2 stage_tw2(float2* dst, const float2* __restrict__ full) {
    constexpr int NC = (L + 31) / 32;
    for (int i = threadIdx.x; i < NC + 32; i += NT) dst[i] = i < NC ? full[32 * i] : full[i - NC];
    return Tw2{dst, dst + NC};
}

// LDS index padding: one float2 of padding every 16 elements breaks the
// power-of-two strides of the Stockham writes across banks.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
constexpr int lpad_c(int i) { return i + (i >> 4); }

// Addressing policy for lines laid out contiguously: line l, element i at
// base + l * LS + lpad(i); butterflies are enumerated j-fastest within a line.
// Both policies also give off(n): the LDS distance between elements i and i + n
// of a line for the index patterns of a power-of-two Stockham pass (n a multiple
// of the butterfly stride, i the butterfly's base), which is a compile-time
// constant: with one padding element per 16, i + n never carries past a
// 16-element boundary that n itself does not cross.
// For other lengths the distance depends on i: at<false>(i, n) computes it.
template <int LS>
struct RowLines {
    static __device__ __forceinline__ int idx(int line, int i) { return line * LS + lpad(i); }
    static constexpr int off(int n) { return lpad_c(n); }
    template <bool P2>
    static __device__ __forceinline__ int at(int i, int n) {
        if constexpr (P2) return lpad_c(n);
        else return lpad(i + n) - lpad(i);
    }
    template <int NB>
    static __device__ __forceinline__ void split(int b, int& line, int& j) { line = b / NB; j = b - line * NB; }
};

// Addressing policy for lines interleaved element-major: element i of line l at
// i * NL + l (consecutive lines adjacent); butterflies enumerated line-fastest.
template <int NL>
struct ColLines {
    static __device__ __forceinline__ int idx(int line, int i) { return i * NL + line; }
    static constexpr int off(int n) { return n * NL; }
    template <bool P2>
    static __device__ __forceinline__ int at(int, int n) { return n * NL; }
    template <int NB>
    static __device__ __forceinline__ void split(int b, int& line, int& j) { j = b / NL; line = b - j * NL; }
};

// One Stockham pass (radix R, sub-size NS) over NLINES lines of length L.
template <int L, int R, int NS, int DIR, int NLINES, int NT, class Addr, class TW>
__device__ __forceinline__ void stockham_pass(float2* buf, TW tw) {
    constexpr int NB = L / R;               // butterflies per line
    constexpr int TOT = NB * NLINES;
    constexpr int PER = (TOT + NT - 1) / NT;
    constexpr bool P2 = is_pow2c(L);
    float2 v[PER][R];
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int b = tid + q * NT;
        if (TOT % NT == 0 || b < TOT) {
            int line, j;
            Addr::template split<NB>(b, line, j);
            const float2* src = buf + Addr::idx(line, j);
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = src[Addr::template at<P2>(j, r * NB)];
            if constexpr (NS > 1) dft_twiddled<R, DIR>(v[q], tw, (j % NS) * (L / (NS * R)));
            else dft<R, DIR>(v[q]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int b = tid + q * NT;
        if (TOT % NT == 0 || b < TOT) {
            int line, j;
            Addr::template split<NB>(b, line, j);
            int k = j % NS;
            const int base = (j / NS) * NS * R + k;
            float2* dst = buf + Addr::idx(line, base);
#pragma unroll
            for (int r = 0; r < R; ++r) dst[Addr::template at<P2>(base, r * NS)] = v[q][r];
        }
    }
    __syncthreads();
}

template <int L, int P, int NS, int DIR, int NLINES, int NT, class Addr, class TW>
__device__ __forceinline__ void fft_passes(float2* buf, TW tw) {
    if constexpr (P < npasses(L)) {
        constexpr int R = radix_of(L, P);
        stockham_pass<L, R, NS, DIR, NLINES, NT, Addr>(buf, tw);
        fft_passes<L, P + 1, NS * R, DIR, NLINES, NT, Addr>(buf, tw);
    }
}

// Stockham FFT whose first pass reads its inputs through src(line, i) straight
// into registers and whose last pass hands its outputs to sink(line, k, v)
// straight from registers; only the passes in between exchange through LDS
// (buf, addressed by Addr).  A length-L transform with P passes thus touches LDS
// 2(P-1) times per element instead of 2P + 2.
//   HALF_IN  inputs i >= L/2 are zero: the first pass neither reads nor adds them
//            (the padded transforms of the convolution);
//   SYNC_IO  src or sink touch buf themselves: barriers separate the first pass's
//            reads from its writes and the last pass's reads from the sink.
// Consecutive threads take consecutive butterflies in the first and last passes,
// so for RowLines a global src/sink is coalesced along the line, for ColLines
// across lines.
template <int L, int R, int DIR, int NLINES, int NT, class Addr, bool HALF_IN, bool SYNC_IO,
          bool TO_LDS, class Src>
__device__ __forceinline__ void first_pass(float2* buf, Src& src) {
    constexpr int NB = L / R;
    constexpr int TOT = NB * NLINES;
    constexpr int PER = (TOT + NT - 1) / NT;
    constexpr int RIN = HALF_IN ? R / 2 : R;
    static_assert(!HALF_IN || R % 2 == 0, "a pruned first pass needs an even radix");
    float2 v[PER][R];
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int b = tid + q * NT;
        if (TOT % NT == 0 || b < TOT) {
            int line, j;
            Addr::template split<NB>(b, line, j);
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = r < RIN ? src(line, j + r * NB) : make_float2(0.f, 0.f);
        }
    }
    if constexpr (SYNC_IO) __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int b = tid + q * NT;
        if (TOT % NT == 0 || b < TOT) {
            int line, j;
            Addr::template split<NB>(b, line, j);
            if constexpr (HALF_IN) dft_half_in<R, DIR>(v[q]);
            else dft<R, DIR>(v[q]);
            if constexpr (TO_LDS) {
                float2* dst = buf + Addr::idx(line, j * R);
#pragma unroll
                for (int r = 0; r < R; ++r) dst[Addr::template at<is_pow2c(L)>(j * R, r)] = v[q][r];
            }
        }
    }
    __syncthreads();
}

template <int L, int R, int DIR, int NLINES, int NT, class Addr, bool HALF_OUT, bool SYNC_IO,
          class Sink, class TW>
__device__ __forceinline__ void last_pass(float2* buf, TW tw, Sink& sink) {
    constexpr int NB = L / R;  // == NS of this pass
    constexpr int TOT = NB * NLINES;
    static_assert(!HALF_OUT || R % 2 == 0, "a truncated last pass needs an even radix");
    constexpr int PER = (TOT + NT - 1) / NT;
    float2 v[PER][R];
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int b = tid + q * NT;
        if (TOT % NT == 0 || b < TOT) {
            int line, j;
            Addr::template split<NB>(b, line, j);
            const float2* src = buf + Addr::idx(line, j);
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = src[Addr::template at<is_pow2c(L)>(j, r * NB)];
        }
    }
    if constexpr (SYNC_IO) __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int b = tid + q * NT;
        if (TOT % NT == 0 || b < TOT) {
            int line, j;
            Addr::template split<NB>(b, line, j);
            dft_twiddled<R, DIR>(v[q], tw, j);
            constexpr int ROUT = HALF_OUT ? R / 2 : R;
#pragma unroll
            for (int r = 0; r < ROUT; ++r) sink(line, j + r * NB, v[q][r]);
        }
    }
}

// ---- radix-16 passes on the matrix cores (split-precision BF16, see mfma_dft.h)
// The pass's butterflies are taken 32 at a time by one wave: butterfly
// b = 32 g + n sits in lanes n and n + 32, lane half h holding inputs and
// outputs 8h .. 8h+7 / out_index(h, .).  Batches g are dealt to the NT/64 waves
// round-robin; the batch loop condition is uniform across a wave, so every lane
// reaches each MFMA, and lanes past the last butterfly carry zeros.
template <int TOT, int NT>
struct MfSched {
    static constexpr int NW = NT / 64;
    static constexpr int NG = (TOT + 31) / 32;
    static constexpr int GPW = (NG + NW - 1) / NW;
};

template <int L, int NS, int DIR, int NLINES, int NT, class Addr, int MF, class TW>
__device__ __forceinline__ void mf_stockham_pass(float2* buf, TW tw,
                                                 const Dft16Matrix<MF>& F) {
    constexpr int NB = L / 16;
    constexpr int TOT = NB * NLINES;
    using S = MfSched<TOT, NT>;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, n = lane & 31, h = lane >> 5;
    float2 y[S::GPW][8];
#pragma unroll
    for (int q = 0; q < S::GPW; ++q) {
        const int g = w + q * S::NW;
        if (S::NG % S::NW == 0 || g < S::NG) {
            const int b = 32 * g + n;
            float2 x[8];
            if (TOT % 32 == 0 || b < TOT) {
                int line, j;
                Addr::template split<NB>(b, line, j);
                const int k = j % NS;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int r = 8 * h + c;
                    x[c] = buf[Addr::idx(line, j + r * NB)];
                    if (NS > 1 && r > 0) {
                        float2 tv = tw[k * r * (L / (NS * 16))];
                        if constexpr (DIR > 0) tv.y = -tv.y;
                        x[c] = cmul(x[c], tv);
                    }
                }
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c) x[c] = make_float2(0.f, 0.f);
            }
            mfma_dft16<MF>(F, x, y[q]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < S::GPW; ++q) {
        const int g = w + q * S::NW;
        const int b = 32 * g + n;
        if ((S::NG % S::NW == 0 || g < S::NG) && (TOT % 32 == 0 || b < TOT)) {
            int line, j;
            Addr::template split<NB>(b, line, j);
            const int k = j % NS;
            const int base = (j / NS) * NS * 16 + k;
#pragma unroll
            for (int c = 0; c < 8; ++c) buf[Addr::idx(line, base + out_index(h, c) * NS)] = y[q][c];
        }
    }
    __syncthreads();
}

// First pass (sub-size 1, no twiddles) reading its inputs through src.
template <int L, int DIR, int NLINES, int NT, class Addr, bool HALF_IN, bool SYNC_IO, int MF,
          class Src>
__device__ __forceinline__ void mf_first_pass(float2* buf, Src& src, const Dft16Matrix<MF>& F) {
    constexpr int NB = L / 16;
    constexpr int TOT = NB * NLINES;
    using S = MfSched<TOT, NT>;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, n = lane & 31, h = lane >> 5;
    float2 x[S::GPW][8];
#pragma unroll
    for (int q = 0; q < S::GPW; ++q) {
        const int g = w + q * S::NW;
        const int b = 32 * g + n;
        const bool live = (S::NG % S::NW == 0 || g < S::NG) && (TOT % 32 == 0 || b < TOT);
        int line = 0, j = 0;
        if (live) Addr::template split<NB>(b, line, j);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int r = 8 * h + c;
            x[q][c] = (live && !(HALF_IN && h == 1)) ? src(line, j + r * NB) : make_float2(0.f, 0.f);
        }
    }
    if constexpr (SYNC_IO) __syncthreads();
#pragma unroll
    for (int q = 0; q < S::GPW; ++q) {
        const int g = w + q * S::NW;
        if (S::NG % S::NW == 0 || g < S::NG) {
            float2 y[8];
            mfma_dft16<MF>(F, x[q], y);
            const int b = 32 * g + n;
            if (TOT % 32 == 0 || b < TOT) {
                int line, j;
                Addr::template split<NB>(b, line, j);
#pragma unroll
                for (int c = 0; c < 8; ++c) buf[Addr::idx(line, j * 16 + out_index(h, c))] = y[c];
            }
        }
    }
    __syncthreads();
}

// Last pass (sub-size L/16) handing its outputs to sink.
template <int L, int DIR, int NLINES, int NT, class Addr, bool HALF_OUT, bool SYNC_IO, int MF,
          class Sink, class TW>
__device__ __forceinline__ void mf_last_pass(float2* buf, TW tw, Sink& sink,
                                             const Dft16Matrix<MF>& F) {
    constexpr int NB = L / 16;  // == sub-size of this pass
    constexpr int TOT = NB * NLINES;
    using S = MfSched<TOT, NT>;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, n = lane & 31, h = lane >> 5;
    float2 x[S::GPW][8];
#pragma unroll
    for (int q = 0; q < S::GPW; ++q) {
        const int g = w + q * S::NW;
        const int b = 32 * g + n;
        const bool live = (S::NG % S::NW == 0 || g < S::NG) && (TOT % 32 == 0 || b < TOT);
        int line = 0, j = 0;
        if (live) Addr::template split<NB>(b, line, j);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int r = 8 * h + c;
            x[q][c] = live ? buf[Addr::idx(line, j + r * NB)] : make_float2(0.f, 0.f);
            if (live && r > 0) {
                float2 tv = tw[j * r];
                if constexpr (DIR > 0) tv.y = -tv.y;
                x[q][c] = cmul(x[q][c], tv);
            }
        }
    }
    if constexpr (SYNC_IO) __syncthreads();
#pragma unroll
    for (int q = 0; q < S::GPW; ++q) {
        const int g = w + q * S::NW;
        if (S::NG % S::NW == 0 || g < S::NG) {
            float2 y[8];
            mfma_dft16<MF>(F, x[q], y);
            const int b = 32 * g + n;
            if (TOT % 32 == 0 || b < TOT) {
                int line, j;
                Addr::template split<NB>(b, line, j);
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int m = out_index(h, c);
                    if (!HALF_OUT || m < 8) sink(line, j + m * NB, y[c]);
                }
            }
        }
    }
}

// L == 16: the whole transform as one batch of matrix products, src -> sink.
template <int DIR, int NLINES, int NT, class Addr, bool HALF_IN, bool HALF_OUT, bool SYNC_IO,
          int MF, class Src, class Sink>
__device__ __forceinline__ void mf_single_pass(Src& src, Sink& sink, const Dft16Matrix<MF>& F) {
    constexpr int TOT = NLINES;
    using S = MfSched<TOT, NT>;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, n = lane & 31, h = lane >> 5;
    float2 x[S::GPW][8];
#pragma unroll
    for (int q = 0; q < S::GPW; ++q) {
        const int g = w + q * S::NW;
        const int b = 32 * g + n;
        const bool live = (S::NG % S::NW == 0 || g < S::NG) && (TOT % 32 == 0 || b < TOT);
        int line = 0, j = 0;
        if (live) Addr::template split<1>(b, line, j);
#pragma unroll
        for (int c = 0; c < 8; ++c)
            x[q][c] = (live && !(HALF_IN && h == 1)) ? src(line, 8 * h + c) : make_float2(0.f, 0.f);
    }
    if constexpr (SYNC_IO) __syncthreads();
#pragma unroll
    for (int q = 0; q < S::GPW; ++q) {
        const int g = w + q * S::NW;
        if (S::NG % S::NW == 0 || g < S::NG) {
            float2 y[8];
            mfma_dft16<MF>(F, x[q], y);
            const int b = 32 * g + n;
            if (TOT % 32 == 0 || b < TOT) {
                int line, j;
                Addr::template split<1>(b, line, j);
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int m = out_index(h, c);
                    if (!HALF_OUT || m < 8) sink(line, m, y[c]);
                }
            }
        }
    }
}

template <int L, int P, int NS, int DIR, int NLINES, int NT, class Addr, int MF, class TW>
__device__ __forceinline__ void middle_passes(float2* buf, TW tw,
                                              const Dft16Matrix<MF>& F) {
    if constexpr (P < npasses(L) - 1) {
        constexpr int R = radix_at<MF>(L, P);
        if constexpr (MF > 0 && R == 16) mf_stockham_pass<L, NS, DIR, NLINES, NT, Addr, MF>(buf, tw, F);
        else stockham_pass<L, R, NS, DIR, NLINES, NT, Addr>(buf, tw);
        middle_passes<L, P + 1, NS * R, DIR, NLINES, NT, Addr, MF>(buf, tw, F);
    }
}

// L <= 16: the whole transform in registers, src -> DFT -> sink.
template <int L, int DIR, int NLINES, int NT, class Addr, bool HALF_IN, bool HALF_OUT,
          bool SYNC_IO, class Src, class Sink>
__device__ __forceinline__ void single_pass(Src& src, Sink& sink) {
    constexpr int TOT = NLINES;
    constexpr int PER = (TOT + NT - 1) / NT;
    constexpr int RIN = HALF_IN ? L / 2 : L;
    constexpr int ROUT = HALF_OUT ? L / 2 : L;
    float2 v[PER][L];
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int b = tid + q * NT;
        if (TOT % NT == 0 || b < TOT) {
            int line, j;
            Addr::template split<1>(b, line, j);
#pragma unroll
            for (int r = 0; r < L; ++r) v[q][r] = r < RIN ? src(line, r) : make_float2(0.f, 0.f);
        }
    }
    if constexpr (SYNC_IO) __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int b = tid + q * NT;
        if (TOT % NT == 0 || b < TOT) {
            int line, j;
            Addr::template split<1>(b, line, j);
            if constexpr (HALF_IN && L >= 2) dft_half_in<L, DIR>(v[q]);
            else dft<L, DIR>(v[q]);
#pragma unroll
            for (int r = 0; r < ROUT; ++r) sink(line, r, v[q][r]);
        }
    }
}

// MF selects the arithmetic of the radix-16 passes: 0 = FP32 butterflies on the
// vector ALUs; 2 or 3 = the split-precision BF16 DFT-matrix products on MFMA
// (see mfma_dft16).  Passes of radix < 16 always run in FP32.
template <int L, int DIR, int NLINES, int NT, class Addr, bool HALF_IN, bool HALF_OUT,
          bool SYNC_IO, int MF = 0, class TW, class Src, class Sink>
__device__ __forceinline__ void fft_io(float2* buf, TW tw, Src src, Sink sink) {
    constexpr int P = npasses(L);
    Dft16Matrix<MF> F;
    if constexpr (MF > 0 && L >= 16) F.template init<DIR>();
    if constexpr (P <= 1) {
        if constexpr (MF > 0 && L == 16)
            mf_single_pass<DIR, NLINES, NT, Addr, HALF_IN, HALF_OUT, SYNC_IO, MF>(src, sink, F);
        else
            single_pass<L, DIR, NLINES, NT, Addr, HALF_IN, HALF_OUT, SYNC_IO>(src, sink);
        return;
    } else {
    constexpr int R0 = radix_at<MF>(L, 0);
    if constexpr (MF > 0 && R0 == 16)
        mf_first_pass<L, DIR, NLINES, NT, Addr, HALF_IN, SYNC_IO, MF>(buf, src, F);
    else
        first_pass<L, R0, DIR, NLINES, NT, Addr, HALF_IN, SYNC_IO, true>(buf, src);
    middle_passes<L, 1, R0, DIR, NLINES, NT, Addr, MF>(buf, tw, F);
    constexpr int RL = radix_at<MF>(L, P - 1);
    if constexpr (MF > 0 && RL == 16)
        mf_last_pass<L, DIR, NLINES, NT, Addr, HALF_OUT, SYNC_IO, MF>(buf, tw, sink, F);
    else
        last_pass<L, RL, DIR, NLINES, NT, Addr, HALF_OUT, SYNC_IO>(buf, tw, sink);
    }
}

// The same transform (FP32, at least two passes) split where a caller wants the
// last pass's outputs in registers: fft_head runs the first and middle passes
// (src -> LDS, ending with a barrier); fft_tail runs the last pass from LDS and
// leaves butterfly b = tid + q NT's outputs in v[q][r], r < R, where Addr's
// split of b into (line, j) gives element j + r L/R.  fft_head then fft_tail
// does exactly the arithmetic of fft_io (HALF_OUT only drops outputs there).
template <int L>
constexpr int tail_radix() { return radix_of(L, npasses(L) - 1); }
template <int L, int NLINES, int NT>
constexpr int tail_per() { return (NLINES * (L / tail_radix<L>()) + NT - 1) / NT; }

template <int L, int DIR, int NLINES, int NT, class Addr, bool HALF_IN, bool SYNC_IO, class TW,
          class Src>
__device__ __forceinline__ void fft_head(float2* buf, TW tw, Src src) {
    static_assert(npasses(L) >= 2, "a split transform needs two passes");
    constexpr int R0 = radix_of(L, 0);
    first_pass<L, R0, DIR, NLINES, NT, Addr, HALF_IN, SYNC_IO, true>(buf, src);
    middle_passes<L, 1, R0, DIR, NLINES, NT, Addr, 0>(buf, tw, Dft16Matrix<0>{});
}

// fft_head with the first pass's inputs already in registers: v[q][r] holds
// element j + r L/R0 of the line that Addr's split gives butterfly
// b = tid + q NT (consumed).
template <int L>
constexpr int head_radix() { return radix_of(L, 0); }
template <int L, int NLINES, int NT>
constexpr int head_per() { return (NLINES * (L / head_radix<L>()) + NT - 1) / NT; }

template <int L, int DIR, int NLINES, int NT, class Addr, class TW>
__device__ __forceinline__ void fft_head_regs(float2* buf, TW tw,
                                              float2 (&v)[head_per<L, NLINES, NT>()][head_radix<L>()]) {
    static_assert(npasses(L) >= 2, "a split transform needs two passes");
    constexpr int R = head_radix<L>();
    constexpr int NB = L / R;
    constexpr int TOT = NB * NLINES;
    constexpr int PER = head_per<L, NLINES, NT>();
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int b = tid + q * NT;
        if (TOT % NT == 0 || b < TOT) {
            int line, j;
            Addr::template split<NB>(b, line, j);
            dft<R, DIR>(v[q]);
            float2* dst = buf + Addr::idx(line, j * R);
#pragma unroll
            for (int r = 0; r < R; ++r) dst[Addr::template at<is_pow2c(L)>(j * R, r)] = v[q][r];
        }
    }
    __syncthreads();
    middle_passes<L, 1, R, DIR, NLINES, NT, Addr, 0>(buf, tw, Dft16Matrix<0>{});
}

template <int L, int DIR, int NLINES, int NT, class Addr, class TW>
__device__ __forceinline__ void fft_tail(const float2* buf, TW tw,
                                         float2 (&v)[tail_per<L, NLINES, NT>()][tail_radix<L>()]) {
    constexpr int R = tail_radix<L>();
    constexpr int NB = L / R;
    constexpr int TOT = NB * NLINES;
    constexpr int PER = tail_per<L, NLINES, NT>();
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int b = tid + q * NT;
        if (TOT % NT == 0 || b < TOT) {
            int line, j;
            Addr::template split<NB>(b, line, j);
            const float2* src = buf + Addr::idx(line, j);
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = src[Addr::template at<is_pow2c(L)>(j, r * NB)];
        }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int b = tid + q * NT;
        if (TOT % NT == 0 || b < TOT) {
            int line, j;
            Addr::template split<NB>(b, line, j);
            dft_twiddled<R, DIR>(v[q], tw, j);
        }
    }
}

// In-place FFT of NLINES lines of length L in LDS (caller syncs before; the
// function ends with a barrier).  DIR = -1 forward, +1 inverse (unnormalised).
// tw points at the length-L table exp(-2 pi i t/L), t < L.
template <int L, int DIR, int NLINES, int NT, class Addr, class TW>
__device__ __forceinline__ void lds_fft(float2* buf, TW tw) {
    if constexpr (L > 1) fft_passes<L, 0, 1, DIR, NLINES, NT, Addr>(buf, tw);
}

}  // namespace dm
