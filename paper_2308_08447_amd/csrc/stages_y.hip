// stages_y.hip -- y stages: padded forward and truncated inverse transforms over kx-plane chunks.
#include "stage_common.h"

namespace dm {

// Twiddle source of a length-LN y transform: the table itself in LDS, or from
// LN = 1024 on the coarse x fine pair (Tw2), which keeps a block's LDS at about
// the size of its lines and doubles the blocks a compute unit holds.
template <int LN>
__device__ __forceinline__ auto y_twiddles(float2* twt, const float2* __restrict__ tw_all) {
    if constexpr (LN >= 1024) {
        return stage_tw2<LN, NT>(twt, tw_all + tw_offset(LN));
    } else {
        stage_table(twt, tw_all + tw_offset(LN), LN);
        return (const float2*)twt;
    }
}

// ============================================================================ y
// The y and z stages run over a chunk of kx planes [k0, k0 + nk) whose spectra
// live in a chunk-sized S2 buffer [3][nz][xc][Ny] (local plane kx - k0).
// One block: LPB lines (consecutive kx) of one (c, z) plane.  Each line is a
// length-Ny = 2L transform whose upper L inputs are zero (forward) or whose
// upper L outputs are dropped (inverse); the first pass reads S1/S2 straight
// into registers and the last pass stores straight from registers.  PY
// (periodic y): a plain length-L transform, Ny = L.
template <int L, int LPB, int MF, bool PY = false>
__global__ __launch_bounds__(NT) void y_forward_kernel(const YBatch b,
                                                       const float2* __restrict__ tw_all) {
    constexpr int LN = PY ? L : 2 * L;
    constexpr int LS = lpad_c(LN);
    __shared__ float2 buf[LPB * LS];
    __shared__ float2 twt[LN >= 1024 ? tw2_entries(LN) : LN];
    const auto tw = y_twiddles<LN>(twt, tw_all);
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    const float2* __restrict__ S1 = b.d[item].S1;
    float2* __restrict__ S2 = b.d[item].S2;
    const int X1 = b.d[item].X1, nz = b.d[item].nz, k0 = b.d[item].k0, nk = b.d[item].nk;
    const int xc = b.d[item].xc;
    const int nt = (nk + LPB - 1) / LPB;
    const int id = gid - b.start[item];
    const int kl0 = (id % nt) * LPB, z = (id / nt) % nz, c = id / (nt * nz);
    const int nl = nk - kl0 < LPB ? nk - kl0 : LPB;  // valid lines in this block
    const float2* in = S1 + ((size_t)(c * nz + z) * X1 + k0 + kl0) * L;
    float2* out = S2 + ((size_t)(c * nz + z) * xc + kl0) * LN;
    auto src = [&](int l, int i) { return l < nl ? in[(size_t)l * L + i] : make_float2(0.f, 0.f); };
    auto sink = [&](int l, int k, float2 v) {
        if (l < nl) out[(size_t)l * LN + k] = v;
    };
    fft_io<LN, -1, LPB, NT, RowLines<LS>, !PY, false, false, MF>(buf, tw, src, sink);
}

template <int L, int LPB, int MF, bool PY = false>
__global__ __launch_bounds__(NT) void y_inverse_kernel(const YBatch b,
                                                       const float2* __restrict__ tw_all) {
    constexpr int LN = PY ? L : 2 * L;
    constexpr int LS = lpad_c(LN);
    __shared__ float2 buf[LPB * LS];
    __shared__ float2 twt[LN >= 1024 ? tw2_entries(LN) : LN];
    const auto tw = y_twiddles<LN>(twt, tw_all);
    const int gid = xcd_tile(blockIdx.x, gridDim.x);
    const int item = batch_item(b, gid);
    const float2* __restrict__ S2 = b.d[item].S2;
    float2* __restrict__ S1 = b.d[item].S1;
    const int X1 = b.d[item].X1, nz = b.d[item].nz, k0 = b.d[item].k0, nk = b.d[item].nk;
    const int xc = b.d[item].xc;
    const int nt = (nk + LPB - 1) / LPB;
    const int id = gid - b.start[item];
    const int kl0 = (id % nt) * LPB, z = (id / nt) % nz, c = id / (nt * nz);
    const int nl = nk - kl0 < LPB ? nk - kl0 : LPB;
    const float2* in = S2 + ((size_t)(c * nz + z) * xc + kl0) * LN;
    float2* out = S1 + ((size_t)(c * nz + z) * X1 + k0 + kl0) * L;
    auto src = [&](int l, int i) { return l < nl ? in[(size_t)l * LN + i] : make_float2(0.f, 0.f); };
    auto sink = [&](int l, int k, float2 v) {
        if (l < nl) out[(size_t)l * L + k] = v;
    };
    fft_io<LN, +1, LPB, NT, RowLines<LS>, false, !PY, false, MF>(buf, tw, src, sink);
}


template <bool INVERSE>
static int launch_y(YBatch b, int ny, int variant, int mf, const float2* tw, hipStream_t s,
                    bool periodic) {
    if (b.count < 1 || b.count > MAXB) return fail(DEMAG_EINVAL, "y stage: bad batch size");
    if (ny == 1) return DEMAG_OK;  // no y transform (S2 aliases S1)
    if (periodic) {
        if (mf) return fail(DEMAG_EUNSUPPORTED, "y stage: periodic transforms are FP32 only");
        switch (ny) {
#define CASE(Lv)                                                                              \
    case Lv: {                                                                                \
        constexpr int L = Lv;                                                                 \
        constexpr int LPB = L >= 2048 ? 1 : 2048 / L;                                         \
        b.start[0] = 0;                                                                       \
        for (int r = 0; r < b.count; ++r)                                                     \
            b.start[r + 1] = b.start[r] + ((b.d[r].nk + LPB - 1) / LPB) * b.d[r].nz * 3;     \
        if (INVERSE)                                                                          \
            DM_LAUNCH((y_inverse_kernel<L, LPB, 0, true>),                                    \
                      dim3((unsigned)finish_batch(b)), dim3(NT), 0, s, b, tw);                \
        else                                                                                  \
            DM_LAUNCH((y_forward_kernel<L, LPB, 0, true>),                                    \
                      dim3((unsigned)finish_batch(b)), dim3(NT), 0, s, b, tw);                \
        break;                                                                                \
    }
            DM_POW2_CASES(CASE)
#undef CASE
            default: return fail(DEMAG_EUNSUPPORTED, "y stage: unsupported ny");
        }
        DM_CHECK_LAUNCH();
        return DEMAG_OK;
    }
    if (!is_pow2c(ny)) {
        if (mf) return fail(DEMAG_EUNSUPPORTED, "y stage: mixed-radix transforms are FP32 only");
        switch (ny) {
#define CASE(Lv)                                                                              \
    case Lv: {                                                                                \
        constexpr int L = Lv;                                                                 \
        constexpr int LPB = YTile<L, 1>::LPB;                                                 \
        b.start[0] = 0;                                                                       \
        for (int r = 0; r < b.count; ++r)                                                     \
            b.start[r + 1] = b.start[r] + ((b.d[r].nk + LPB - 1) / LPB) * b.d[r].nz * 3;     \
        if (INVERSE)                                                                          \
            DM_LAUNCH((y_inverse_kernel<L, LPB, 0, false>),                                   \
                      dim3((unsigned)finish_batch(b)), dim3(NT), 0, s, b, tw);                \
        else                                                                                  \
            DM_LAUNCH((y_forward_kernel<L, LPB, 0, false>),                                   \
                      dim3((unsigned)finish_batch(b)), dim3(NT), 0, s, b, tw);                \
        break;                                                                                \
    }
            DM_MIXED_CASES(CASE)
#undef CASE
            default: return fail(DEMAG_EUNSUPPORTED, "y stage: unsupported ny");
        }
        DM_CHECK_LAUNCH();
        return DEMAG_OK;
    }
    switch (ny) {
#define BODY(V)                                                                                 \
    {                                                                                           \
        constexpr int LPB = YTile<L, V>::LPB;                                                   \
        b.start[0] = 0;                                                                         \
        for (int r = 0; r < b.count; ++r)                                                       \
            b.start[r + 1] = b.start[r] + ((b.d[r].nk + LPB - 1) / LPB) * b.d[r].nz * 3;       \
        if (INVERSE)                                                                            \
            DM_MF_DISPATCH(V, DM_LAUNCH((y_inverse_kernel<L, LPB, MFv>),                        \
                      dim3((unsigned)finish_batch(b)), dim3(NT), 0, s, b, tw);)                 \
        else                                                                                    \
            DM_MF_DISPATCH(V, DM_LAUNCH((y_forward_kernel<L, LPB, MFv>),                        \
                      dim3((unsigned)finish_batch(b)), dim3(NT), 0, s, b, tw);)                 \
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
        default: return fail(DEMAG_EUNSUPPORTED, "y stage: unsupported ny");
    }
    DM_CHECK_LAUNCH();
    return DEMAG_OK;
}

int launch_y_forward(YBatch b, int ny, int variant, int mf, const float2* tw, hipStream_t s,
                     bool periodic) {
    return launch_y<false>(b, ny, variant, mf, tw, s, periodic);
}
int launch_y_inverse(YBatch b, int ny, int variant, int mf, const float2* tw, hipStream_t s,
                     bool periodic) {
    return launch_y<true>(b, ny, variant, mf, tw, s, periodic);
}


}  // namespace dm
