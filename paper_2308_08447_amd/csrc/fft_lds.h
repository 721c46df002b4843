// fft_lds.h -- batched power-of-two complex FFTs held in LDS, for gfx950.
//
// A workgroup transforms NLINES lines of length L that sit in LDS.  Each radix
// pass is a Stockham autosort step: butterfly j (0 <= j < L/R) of the pass with
// current sub-transform size Ns reads x[j + r L/R] (r < R), multiplies element r
// by W^(r (j mod Ns)) with W = exp(-+2 pi i/(Ns R)), does an R-point DFT in
// registers and writes element r to (j/Ns) Ns R + (j mod Ns) + r Ns.  After the
// last pass the line is in natural order.  Radices are 2..16, chosen so the
// passes are as even as possible (e.g. 1024 = 16*8*8).
//
// Twiddles come from a table of exp(-2 pi i t/L), t < L, rounded from FP64 on
// the host, so every twiddle is correctly rounded (no recurrence, no
// hardware sin/cos approximation).
#pragma once

#include <hip/hip_runtime.h>

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
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (DIR = -1) or +i (DIR = +1)
template <int DIR>
__device__ __forceinline__ float2 mul_i(float2 a) {
    if constexpr (DIR < 0) return make_float2(a.y, -a.x);
    else return make_float2(-a.y, a.x);
}

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

// In-register DFT of size R (power of two <= 16), radix-2 decimation in time.
template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v) {
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 2) {
        float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        dft<R / 2, DIR>(e);
        dft<R / 2, DIR>(o);
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            float2 t;
            if (k == 0) t = o[0];
            else if (4 * k == R) t = mul_i<DIR>(o[k]);
            else t = cmul(w16<DIR>(k * (16 / R)), o[k]);
            v[k] = cadd(e[k], t);
            v[k + R / 2] = csub(e[k], t);
        }
    }
}

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

// Radix of pass p for a length-L transform: ceil(log2 L / 4) passes, bits spread evenly.
constexpr int radix_of(int L, int p) {
    int k = ilog2c(L);
    int P = (k + 3) / 4;
    if (P == 0) return 1;
    int base = k / P, extra = k % P;
    return 1 << (base + (p < extra ? 1 : 0));
}
constexpr int npasses(int L) { return (ilog2c(L) + 3) / 4; }

// LDS index padding: one float2 of padding every 16 elements breaks the
// power-of-two strides of the Stockham writes across banks.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
constexpr int lpad_c(int i) { return i + (i >> 4); }

// Addressing policy for lines laid out contiguously: line l, element i at
// base + l * LS + lpad(i); butterflies are enumerated j-fastest within a line.
template <int LS>
struct RowLines {
    static __device__ __forceinline__ int idx(int line, int i) { return line * LS + lpad(i); }
    template <int NB>
    static __device__ __forceinline__ void split(int b, int& line, int& j) { line = b / NB; j = b - line * NB; }
};

// Addressing policy for lines interleaved element-major: element i of line l at
// i * NL + l (consecutive lines adjacent); butterflies enumerated line-fastest.
template <int NL>
struct ColLines {
    static __device__ __forceinline__ int idx(int line, int i) { return i * NL + line; }
    template <int NB>
    static __device__ __forceinline__ void split(int b, int& line, int& j) { j = b / NL; line = b - j * NL; }
};

// One Stockham pass (radix R, sub-size NS) over NLINES lines of length L.
template <int L, int R, int NS, int DIR, int NLINES, int NT, class Addr>
__device__ __forceinline__ void stockham_pass(float2* buf, const float2* __restrict__ tw) {
    constexpr int NB = L / R;               // butterflies per line
    constexpr int TOT = NB * NLINES;
    constexpr int PER = (TOT + NT - 1) / NT;
    float2 v[PER][R];
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int b = tid + q * NT;
        if (TOT % NT == 0 || b < TOT) {
            int line, j;
            Addr::template split<NB>(b, line, j);
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[Addr::idx(line, j + r * NB)];
            if constexpr (NS > 1) {
                int k = j % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = tw[k * r * (L / (NS * R))];
                    if constexpr (DIR > 0) w.y = -w.y;
                    v[q][r] = cmul(v[q][r], w);
                }
            }
            dft<R, DIR>(v[q]);
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
            int base = (j / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[Addr::idx(line, base + r * NS)] = v[q][r];
        }
    }
    __syncthreads();
}

template <int L, int P, int NS, int DIR, int NLINES, int NT, class Addr>
__device__ __forceinline__ void fft_passes(float2* buf, const float2* __restrict__ tw) {
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
            dft<R, DIR>(v[q]);
            if constexpr (TO_LDS) {
#pragma unroll
                for (int r = 0; r < R; ++r) buf[Addr::idx(line, j * R + r)] = v[q][r];
            }
        }
    }
    __syncthreads();
}

template <int L, int R, int DIR, int NLINES, int NT, class Addr, bool HALF_OUT, bool SYNC_IO,
          class Sink>
__device__ __forceinline__ void last_pass(float2* buf, const float2* __restrict__ tw, Sink& sink) {
    constexpr int NB = L / R;  // == NS of this pass
    constexpr int TOT = NB * NLINES;
    constexpr int PER = (TOT + NT - 1) / NT;
    float2 v[PER][R];
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int b = tid + q * NT;
        if (TOT % NT == 0 || b < TOT) {
            int line, j;
            Addr::template split<NB>(b, line, j);
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[Addr::idx(line, j + r * NB)];
        }
    }
    if constexpr (SYNC_IO) __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int b = tid + q * NT;
        if (TOT % NT == 0 || b < TOT) {
            int line, j;
            Addr::template split<NB>(b, line, j);
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = tw[j * r];
                if constexpr (DIR > 0) w.y = -w.y;
                v[q][r] = cmul(v[q][r], w);
            }
            dft<R, DIR>(v[q]);
            constexpr int ROUT = HALF_OUT ? R / 2 : R;
#pragma unroll
            for (int r = 0; r < ROUT; ++r) sink(line, j + r * NB, v[q][r]);
        }
    }
}

template <int L, int P, int NS, int DIR, int NLINES, int NT, class Addr>
__device__ __forceinline__ void middle_passes(float2* buf, const float2* __restrict__ tw) {
    if constexpr (P < npasses(L) - 1) {
        constexpr int R = radix_of(L, P);
        stockham_pass<L, R, NS, DIR, NLINES, NT, Addr>(buf, tw);
        middle_passes<L, P + 1, NS * R, DIR, NLINES, NT, Addr>(buf, tw);
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
            dft<L, DIR>(v[q]);
#pragma unroll
            for (int r = 0; r < ROUT; ++r) sink(line, r, v[q][r]);
        }
    }
}

template <int L, int DIR, int NLINES, int NT, class Addr, bool HALF_IN, bool HALF_OUT,
          bool SYNC_IO, class Src, class Sink>
__device__ __forceinline__ void fft_io(float2* buf, const float2* __restrict__ tw, Src src,
                                       Sink sink) {
    constexpr int P = npasses(L);
    if constexpr (P <= 1) {
        single_pass<L, DIR, NLINES, NT, Addr, HALF_IN, HALF_OUT, SYNC_IO>(src, sink);
        return;
    } else {
    constexpr int R0 = radix_of(L, 0);
    first_pass<L, R0, DIR, NLINES, NT, Addr, HALF_IN, SYNC_IO, true>(buf, src);
    middle_passes<L, 1, R0, DIR, NLINES, NT, Addr>(buf, tw);
    last_pass<L, radix_of(L, P - 1), DIR, NLINES, NT, Addr, HALF_OUT, SYNC_IO>(buf, tw, sink);
    }
}

// In-place FFT of NLINES lines of length L in LDS (caller syncs before; the
// function ends with a barrier).  DIR = -1 forward, +1 inverse (unnormalised).
// tw points at the length-L table exp(-2 pi i t/L), t < L.
template <int L, int DIR, int NLINES, int NT, class Addr>
__device__ __forceinline__ void lds_fft(float2* buf, const float2* __restrict__ tw) {
    if constexpr (L > 1) fft_passes<L, 0, 1, DIR, NLINES, NT, Addr>(buf, tw);
}

}  // namespace dm
