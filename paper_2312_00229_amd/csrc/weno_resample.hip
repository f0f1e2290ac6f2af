// Arbitrary resolution (arXiv 2312.00229, Section 3.3): the 1D WENO spline
// w(V, x) (eq. wenoSpline, built on Section 2's eqs. Tocnost ..
// IzrazOmega), the tensor WENO resampler (eq. tensor) and zooming to any
// size by k WD-WENO doublings followed by the resampler.
//
// On [x_i, x_{i+1}], t = (x - x_i)/h: the quadratics p_i (nodes t = -1, 0, 1)
// and p_{i+1} (nodes 0, 1, 2) are blended with the ideal weights
// C_0 = (2 - t)/3, C_1 = (t + 1)/3 (the linear functions that turn the pair
// into the cubic through the four nodes) divided by (eps + SI_s)^beta, where
// SI_s integrates the squared first and second derivatives of the quadratic
// over [x_i, x_{i+1}] (scale h^(2l-1)):
//   p_i     = v_i + a1 t + a2 t^2,      a1 = (v_{i+1} - v_{i-1})/2, a2 = (v_{i+1} - 2v_i + v_{i-1})/2
//   SI_0    = a1^2 + 2 a1 a2 + (16/3) a2^2
//   p_{i+1} = v_{i+1} + b1 s + b2 s^2,  s = t - 1, b1 = (v_{i+2} - v_i)/2, b2 = (v_{i+2} - 2v_{i+1} + v_i)/2
//   SI_1    = b1^2 - 2 b1 b2 + (16/3) b2^2
// Output sample j of an axis of n_out samples sits at x_j = j (n_in - 1)/(n_out - 1)
// (end points aligned), computed in integers so that t is exact to FP32
// rounding; samples on input nodes are copied.  The two passes (rows, then
// columns) go through an FP32 intermediate in the caller's workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "weno_internal.h"
#include "weno_zoom.h"

using namespace wz;

namespace {

// The blend on [x_i, x_{i+1}] with the differences A1 = 2 a1, A2 = 2 a2,
// B1 = 2 b1, B2 = 2 b2 of the header's coefficients:
//   p_i = v_i + (t/2)(A1 + A2 t),   p_{i+1} = v_{i+1} + (s/2)(B1 + B2 s),
//   4 (eps + SI_0) = E_0 = 4 eps + A1^2 + 2 A1 A2 + (16/3) A2^2,
//   4 (eps + SI_1) = E_1 = 4 eps + B1^2 - 2 B1 B2 + (16/3) B2^2,
// and, dividing alpha_0 + alpha_1 by alpha_1,
//   omega_1 = 1 / (1 + (C_0/C_1) (E_1/E_0)^beta),   u = p_i + omega_1 (p_{i+1} - p_i),
// for beta = 2 written E_0^2 / (E_0^2 + k E_1^2) with one reciprocal per
// sample (two for other beta).  E_0, E_1 >= 4 eps > 0 (for beta = 0 the host
// passes eps = 1: the weights are then C_s whatever the indicators).  A node
// (t = 0, wmask = 0) gets omega_1 = 0 (the reciprocal is of a positive finite
// number), so u = p_i = v_i exactly.
template <int BETA>
__device__ __forceinline__ float blend(float vm, float v0, float v1, float v2, float t, float s, float ht, float hs,
                                       float k, float eps4, float beta, float wmask = 1.0f)
{
    const float A1 = v1 - vm;
    const float A2 = __builtin_fmaf(v0, -2.0f, v1 + vm);
    const float B1 = v2 - v0;
    const float B2 = __builtin_fmaf(v1, -2.0f, v2 + v0);
    const float p0 = __builtin_fmaf(ht, __builtin_fmaf(t, A2, A1), v0);
    const float p1 = __builtin_fmaf(hs, __builtin_fmaf(s, B2, B1), v1);
    const float E0 = __builtin_fmaf(A2, __builtin_fmaf(A2, 16.0f / 3.0f, A1 + A1), __builtin_fmaf(A1, A1, eps4));
    const float E1 = __builtin_fmaf(B2, __builtin_fmaf(B2, 16.0f / 3.0f, -(B1 + B1)), __builtin_fmaf(B1, B1, eps4));
    float w1;
    if constexpr (BETA == 2) {
        // 1/(1 + k (E1/E0)^2) = E0^2 / (E0^2 + k E1^2): one reciprocal (the
        // denominator is at least (4 eps)^2; E^2 stays finite for samples
        // below ~4e9 in magnitude)
        const float e0 = E0 * E0;
        w1 = (e0 * wmask) * rcp(__builtin_fmaf(k, E1 * E1, e0));
    } else {
        const float g = __builtin_amdgcn_exp2f(beta * __builtin_amdgcn_logf(E1 * rcp(E0)));
        w1 = rcp(__builtin_fmaf(k, g, 1.0f)) * wmask;
    }
    return __builtin_fmaf(w1, p1 - p0, p0);
}

// Source position of one output sample along an axis: the interval
// [x_i, x_{i+1}], t in (0, 1) and k = C_0(t)/C_1(t), or a copy of node i
// (node = 1, t = 0).
struct SamplePos {
    int32_t i;
    float t;
    float k;
    int32_t node;
};

// Positions j (n_in - 1)/(n_out - 1) = i + t of an axis, one thread each,
// worked out in integers so that nodes are exact; t and k are rounded once
// from exact ratios.
__device__ void sample_position(SamplePos* __restrict__ pos, int j, int n_in, int n_out)
{
    SamplePos p;
    p.i = 0;
    p.t = 0.0f;
    p.k = 2.0f;
    p.node = 1;
    if (n_out > 1 && n_in > 1) {
        const uint64_t num = (uint64_t)j * (uint64_t)(n_in - 1);
        const uint64_t den = (uint64_t)(n_out - 1);
        int i = (int)(num / den);
        const uint64_t rem = num - (uint64_t)i * den;
        if (i > n_in - 2) {
            p.i = n_in - 1;          // the last node
        } else if (rem == 0) {
            p.i = i;                 // a node
        } else {
            p.i = i;
            p.node = 0;
            p.t = (float)((double)rem / (double)den);
            // C_0/C_1 = (2 - t)/(t + 1) = (2 den - rem)/(den + rem)
            p.k = (float)((double)(2 * den - rem) / (double)(den + rem));
        }
    }
    pos[j] = p;
}

// both tables in one launch: rows first, then columns
__global__ __launch_bounds__(256) void positions_kernel(SamplePos* __restrict__ rows, int h_in, int h_out,
                                                        SamplePos* __restrict__ cols, int w_in, int w_out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < h_out) sample_position(rows, j, h_in, h_out);
    else if (j - h_out < w_out) sample_position(cols, j - h_out, w_in, w_out);
}

// Work split of both passes: a wave owns kCpl columns per lane (64 apart, so
// every memory operation of the wave is one coalesced row segment) and a run
// of kRun output rows; setup is paid once per 64 * kCpl * kRun outputs.
constexpr int kCpl = 2;
constexpr int kRun = 16;

// The row pass writes rows of in_w + 3 samples: padded column x holds input
// column clamp(x - 1, 0, in_w - 1), so the column pass finds the taps
// i - 1 .. i + 2 of any interval at padded columns i .. i + 3, unclamped.
constexpr int kPadCols = 3;

struct RowPassArgs {
    const uint8_t* src;       // input planes (any dtype, byte strides below)
    uint8_t* tmp;             // padded float planes
    int64_t s_n, s_c;
    uint32_t s_h, s_w;        // input row and column strides
    uint32_t src_extent;      // bytes spanned by one input plane
    uint32_t t_h;             // padded row pitch (bytes)
    uint32_t t_plane;         // bytes per padded plane
    int32_t C, in_h, in_w, out_h;
    int32_t chunks, runs;     // column chunks of 64 * kCpl padded columns, row runs of kRun
    float eps4, beta;
};

// AXIS 0: output row r of column x <- input rows i - 1 .. i + 2 of r's
// interval.  Every tap row is uniform over the wave.
template <int BETA, bool IN_U8>
__global__ __launch_bounds__(256) void rows_pass_kernel(RowPassArgs a, const SamplePos* __restrict__ pos)
{
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    if (wave >= a.chunks * a.runs) return;
    const int lane = threadIdx.x & 63;
    const int run = wave / a.chunks, chunk = wave - run * a.chunks;
    const int plane = blockIdx.y;
    const int n = plane / a.C, ch = plane - n * a.C;
    const rsrc_t src = make_rsrc(a.src + n * a.s_n + ch * a.s_c, a.src_extent);
    const rsrc_t dst = make_rsrc(a.tmp + (size_t)plane * a.t_plane, a.t_plane);
    const int padded = a.in_w + kPadCols;
    uint32_t vin[kCpl], vout[kCpl];
#pragma unroll
    for (int j = 0; j < kCpl; ++j) {
        const int x = chunk * (64 * kCpl) + lane + 64 * j;
        const int xc = min(max(x - 1, 0), a.in_w - 1);
        vin[j] = x < padded ? (uint32_t)xc * a.s_w : kOob;
        vout[j] = x < padded ? (uint32_t)x * 4u : kOob;
    }
    constexpr float kScale = IN_U8 ? 1.0f / 255.0f : 1.0f;   // the padded planes are on the [0,1] scale of u8
    // raw taps (bytes stay bytes until the row is used, so that no wait
    // follows the loads)
    using raw = typename std::conditional<IN_U8, uint8_t, float>::type;
    auto ld = [&](uint32_t voff, uint32_t soff) -> raw {
        if constexpr (IN_U8) return __builtin_amdgcn_raw_buffer_load_b8(src, (int)voff, (int)soff, 0);
        else return buf_ld_f32(src, voff, soff);
    };
    // the taps of output row r, loaded one row ahead of their use
    struct Taps {
        raw v[4][kCpl];
        float t, k;
    };
    auto load = [&](Taps& T, int r) {
        const SamplePos p = pos[r];
        const uint32_t s0 = (uint32_t)p.i * a.s_h;
        // a node collapses all four taps onto its row: the blend of four equal
        // (finite) values is that value, exactly
        const bool node = p.node != 0;
        const uint32_t sm = node ? s0 : (uint32_t)max(p.i - 1, 0) * a.s_h;
        const uint32_t s1 = node ? s0 : s0 + a.s_h;
        const uint32_t s2 = node ? s0 : (uint32_t)min(p.i + 2, a.in_h - 1) * a.s_h;
#pragma unroll
        for (int j = 0; j < kCpl; ++j) {
            T.v[0][j] = ld(vin[j], sm);
            T.v[1][j] = ld(vin[j], s0);
            T.v[2][j] = ld(vin[j], s1);
            T.v[3][j] = ld(vin[j], s2);
        }
        T.t = p.t;
        T.k = p.k;
    };
    auto emit = [&](const Taps& T, int r) {
        const float t = T.t, s = t - 1.0f, ht = 0.5f * t, hs = 0.5f * s;
        const uint32_t so = (uint32_t)r * a.t_h;
#pragma unroll
        for (int j = 0; j < kCpl; ++j)
            buf_st_f32(blend<BETA>((float)T.v[0][j], (float)T.v[1][j], (float)T.v[2][j], (float)T.v[3][j], t, s, ht,
                                   hs, T.k, a.eps4, a.beta) *
                           kScale,
                       dst, vout[j], so);
    };
    const int r0 = run * kRun, r1 = min(r0 + kRun, a.out_h);
    Taps A, B;
    int r = r0;
    load(A, r);
    for (; r + 2 <= r1; r += 2) {
        load(B, r + 1);
        emit(A, r);
        load(A, min(r + 2, r1 - 1));
        emit(B, r + 1);
    }
    if (r < r1) emit(A, r);
}

struct ColPassArgs {
    const uint8_t* tmp;       // padded float planes
    uint8_t* dst;             // output planes (any dtype, byte strides below)
    int64_t d_n, d_c;
    uint32_t d_h, d_w;
    uint32_t d_extent;        // bytes spanned by one output plane
    uint32_t t_h, t_plane;
    int32_t C, out_h, out_w;
    int32_t chunks, runs;     // column chunks of 64 * kCpl output columns, row runs of kRun
    float eps4, beta;
};

// AXIS 1: output column c of row r <- padded columns i .. i + 3 of row r,
// i the interval of c.  Positions and tap offsets are per lane, loaded once
// per run.
template <int BETA, bool OUT_U8>
__global__ __launch_bounds__(256) void cols_pass_kernel(ColPassArgs a, const SamplePos* __restrict__ pos)
{
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    if (wave >= a.chunks * a.runs) return;
    const int lane = threadIdx.x & 63;
    const int run = wave / a.chunks, chunk = wave - run * a.chunks;
    const int plane = blockIdx.y;
    const int n = plane / a.C, ch = plane - n * a.C;
    const rsrc_t src = make_rsrc(a.tmp + (size_t)plane * a.t_plane, a.t_plane);
    const rsrc_t dst = make_rsrc(a.dst + n * a.d_n + ch * a.d_c, a.d_extent);
    uint32_t vtap[kCpl], vout[kCpl];
    float t[kCpl], s[kCpl], ht[kCpl], hs[kCpl], k[kCpl], wmask[kCpl];
#pragma unroll
    for (int j = 0; j < kCpl; ++j) {
        const int c = chunk * (64 * kCpl) + lane + 64 * j;
        const SamplePos p = pos[min(c, a.out_w - 1)];
        vtap[j] = (uint32_t)p.i * 4u;
        vout[j] = c < a.out_w ? (uint32_t)c * a.d_w : kOob;
        wmask[j] = p.node ? 0.0f : 1.0f;
        t[j] = p.t;
        s[j] = p.t - 1.0f;
        ht[j] = 0.5f * t[j];
        hs[j] = 0.5f * s[j];
        k[j] = p.k;
    }
    struct Taps {
        float v[4][kCpl];
    };
    auto load = [&](Taps& T, int r) {
        const uint32_t si = (uint32_t)r * a.t_h;
#pragma unroll
        for (int j = 0; j < kCpl; ++j)
#pragma unroll
            for (int m = 0; m < 4; ++m) T.v[m][j] = buf_ld_f32(src, vtap[j] + 4u * m, si);
    };
    auto emit = [&](const Taps& T, int r) {
        const uint32_t so = (uint32_t)r * a.d_h;
#pragma unroll
        for (int j = 0; j < kCpl; ++j) {
            const float u = blend<BETA>(T.v[0][j], T.v[1][j], T.v[2][j], T.v[3][j], t[j], s[j], ht[j], hs[j], k[j],
                                        a.eps4, a.beta, wmask[j]);
            if constexpr (OUT_U8) buf_st_u8(quant_u8(u * 255.0f), dst, vout[j], so);
            else buf_st_f32(u, dst, vout[j], so);
        }
    };
    const int r0 = run * kRun, r1 = min(r0 + kRun, a.out_h);
    Taps A, B;
    int r = r0;
    load(A, r);
    for (; r + 2 <= r1; r += 2) {
        load(B, r + 1);
        emit(A, r);
        load(A, min(r + 2, r1 - 1));
        emit(B, r + 1);
    }
    if (r < r1) emit(A, r);
}

// Fused tensor resampler: a block of 256 threads owns a tile of `tw` output
// columns and a run of output rows of one plane.  For each output row it
// first resamples the four input rows of that row's interval at the input
// columns its columns' intervals touch (columns xa .. xa + 256 M - 1, xa =
// i(c0) - 1, clamped), into an LDS row, then resamples that row along the
// columns; the float intermediate of the two-pass form never leaves the CU.
// The arithmetic, operands and their order are those of the two passes, so
// both forms give the same bits.  The host picks M and tw so that a tile's
// span i(c_last) - i(c0) + 4 fits in 256 M samples.
constexpr int kFuseQ = 3;          // output columns per thread at most (tw <= 768)
constexpr int kFuseThreads = 256;  // threads per block (LDS slots per row: kFuseThreads M)
constexpr int kFuseMaxTw = kFuseThreads * kFuseQ;

struct FusedArgs {
    const uint8_t* src;
    uint8_t* dst;
    int64_t s_n, s_c, d_n, d_c;
    uint32_t s_h, s_w, d_h, d_w;
    uint32_t src_extent, d_extent;
    int32_t C, in_h, in_w, out_h, out_w;
    int32_t tw, ctiles, run;          // tile width, tiles per row, rows per run
    float eps4_in, eps4, beta;        // eps4_in in the input's value scale, eps4 on the float scale
};

template <int BETA, int M, bool IN_U8, bool OUT_U8>
__global__ __launch_bounds__(kFuseThreads) void fused_resample_kernel(FusedArgs a,
                                                                      const SamplePos* __restrict__ prow,
                                                                      const SamplePos* __restrict__ pcol)
{
    __shared__ float row_buf[2][kFuseThreads * M];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tile = blockIdx.x;
    const int rr = tile / a.ctiles, ct = tile - rr * a.ctiles;
    const int plane = blockIdx.y;
    const int n = plane / a.C, ch = plane - n * a.C;
    const rsrc_t src = make_rsrc(a.src + n * a.s_n + ch * a.s_c, a.src_extent);
    const rsrc_t dst = make_rsrc(a.dst + n * a.d_n + ch * a.d_c, a.d_extent);
    const int c0 = ct * a.tw, c1 = min(c0 + a.tw, a.out_w);
    const int xa = pcol[c0].i - 1, xb = pcol[c1 - 1].i + 2;   // the tile's span of input columns
    // row phase: the input columns of this thread's LDS slots (slots past the
    // span load nothing: their values are never read)
    uint32_t vin[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int x = xa + tid + kFuseThreads * m;
        vin[m] = x <= xb ? (uint32_t)min(max(x, 0), a.in_w - 1) * a.s_w : kOob;
    }
    // column phase: per output column, the LDS index of its first tap and its weights
    int lb[kFuseQ];
    uint32_t vout[kFuseQ];
    float t[kFuseQ], s[kFuseQ], ht[kFuseQ], hs[kFuseQ], k[kFuseQ], wmask[kFuseQ];
    int live = 0;   // bit q: the wave owns a column of slot q (uniform)
#pragma unroll
    for (int q = 0; q < kFuseQ; ++q) {
        const int c = c0 + tid + kFuseThreads * q;
        live |= (c0 + kFuseThreads * q + 64 * wave < c1) << q;
        const SamplePos p = pcol[min(c, a.out_w - 1)];
        lb[q] = p.i - 1 - xa;
        vout[q] = c < c1 ? (uint32_t)c * a.d_w : kOob;
        t[q] = p.t;
        s[q] = p.t - 1.0f;
        ht[q] = 0.5f * t[q];
        hs[q] = 0.5f * s[q];
        k[q] = p.k;
        wmask[q] = p.node ? 0.0f : 1.0f;
    }
    live = __builtin_amdgcn_readfirstlane(live);
    constexpr float kScale = IN_U8 ? 1.0f / 255.0f : 1.0f;
    using raw = typename std::conditional<IN_U8, uint8_t, float>::type;
    auto ld = [&](uint32_t voff, uint32_t soff) -> raw {
        if constexpr (IN_U8) return __builtin_amdgcn_raw_buffer_load_b8(src, (int)voff, (int)soff, 0);
        else return buf_ld_f32(src, voff, soff);
    };
    // The row phase slides a window of input rows down the run: W holds rows
    // cur - 1 .. cur + 2 (clamped) at this thread's LDS slots.  Output rows
    // advance the interval by d = i(r + 1) - i(r) >= 0 (uniform), so moving
    // to the next row keeps 4 - d rows and loads d of them (all four past 3):
    // about 1.33 loads per output row when downsampling by 4/3, against four.
    raw W[M][4];
    int cur = 0;
    auto row_off = [&](int row) { return (uint32_t)min(max(row, 0), a.in_h - 1) * a.s_h; };
    auto ld_row = [&](int slot, int row) {
        const uint32_t so = row_off(row);
#pragma unroll
        for (int m = 0; m < M; ++m) W[m][slot] = ld(vin[m], so);
    };
    auto advance = [&](int i) {
        const int d = i - cur;
        if (d == 1) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                W[m][0] = W[m][1];
                W[m][1] = W[m][2];
                W[m][2] = W[m][3];
            }
            ld_row(3, i + 2);
        } else if (d == 2) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                W[m][0] = W[m][2];
                W[m][1] = W[m][3];
            }
            ld_row(2, i + 1);
            ld_row(3, i + 2);
        } else if (d == 3) {
#pragma unroll
            for (int m = 0; m < M; ++m) W[m][0] = W[m][3];
            ld_row(1, i);
            ld_row(2, i + 1);
            ld_row(3, i + 2);
        } else if (d != 0) {
            ld_row(0, i - 1);
            ld_row(1, i);
            ld_row(2, i + 1);
            ld_row(3, i + 2);
        }
        cur = i;
    };
    const int r0 = rr * a.run, r1 = min(r0 + a.run, a.out_h);
    SamplePos pc = prow[r0];   // the row being resampled
    cur = pc.i;
    ld_row(0, cur - 1);
    ld_row(1, cur);
    ld_row(2, cur + 1);
    ld_row(3, cur + 2);
    auto step = [&](int r, float* buf) {
        {
            // a node row (t = 0, omega_1 masked) is its own tap W[1], exactly
            const float tt = pc.t, ss = tt - 1.0f, htt = 0.5f * tt, hss = 0.5f * ss;
            const float wm = pc.node ? 0.0f : 1.0f;
#pragma unroll
            for (int m = 0; m < M; ++m)
                buf[tid + kFuseThreads * m] = blend<BETA>((float)W[m][0], (float)W[m][1], (float)W[m][2],
                                                          (float)W[m][3], tt, ss, htt, hss, pc.k, a.eps4_in, a.beta,
                                                          wm) *
                                              kScale;
        }
        __syncthreads();
        pc = prow[min(r + 1, r1 - 1)];
        advance(pc.i);
        // uniform (kept in a scalar register: a buffer store's row offset)
        const uint32_t so = __builtin_amdgcn_readfirstlane((uint32_t)r * a.d_h);
#pragma unroll
        for (int q = 0; q < kFuseQ; ++q) {
            if (!((live >> q) & 1)) continue;
            const float* L = buf + lb[q];
            const float u = blend<BETA>(L[0], L[1], L[2], L[3], t[q], s[q], ht[q], hs[q], k[q], a.eps4, a.beta, wmask[q]);
            if constexpr (OUT_U8) buf_st_u8(quant_u8(u * 255.0f), dst, vout[q], so);
            else buf_st_f32(u, dst, vout[q], so);
        }
    };
    int r = r0;
    for (; r + 2 <= r1; r += 2) {
        step(r, row_buf[0]);
        step(r + 1, row_buf[1]);
    }
    if (r < r1) step(r, row_buf[0]);
}

// bytes of a position table of n entries (256-byte aligned)
size_t positions_bytes(int64_t n) { return (size_t)((n * (int64_t)sizeof(SamplePos) + 255) / 256 * 256); }

int launch_positions(SamplePos* rows, int h_in, int h_out, SamplePos* cols, int w_in, int w_out, hipStream_t st)
{
    hipLaunchKernelGGL(positions_kernel, dim3((h_out + w_out + 255) / 256), dim3(256), 0, st, rows, h_in, h_out, cols,
                       w_in, w_out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? WENO_OK : wz_hip_error(e, "positions_kernel launch");
}

// 4 eps for the kernels' E_s = 4 (eps + SI_s), in the value scale of the pass
// input (u8: 0..255); beta = 0 takes 1, the weights being C_s whatever eps is
float eps4_of(const weno_params_t* p, double h, bool u8)
{
    const double vs = u8 ? 255.0 : 1.0;
    return p->beta == 0.0f ? 1.0f : (float)(4.0 * (double)p->k_eps * h * h * vs * vs);
}

dim3 pass_grid(int chunks, int runs, int planes)
{
    const int64_t waves = (int64_t)chunks * runs;
    return dim3((unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock), (unsigned)planes);
}

// The row pass of src into padded planes at tmp (out_h rows of pitch t_h bytes).
int launch_rows_pass(const weno_tensor_t* src, uint8_t* tmp, uint32_t t_h, int out_h, const weno_params_t* p,
                     double h, const SamplePos* pos, hipStream_t st)
{
    RowPassArgs a;
    const int64_t ei = wz_esize(src->dtype);
    const bool u8 = src->dtype == WENO_U8;
    a.src = (const uint8_t*)src->data;
    a.tmp = tmp;
    a.s_n = src->sn * ei;
    a.s_c = src->sc * ei;
    a.s_h = (uint32_t)(src->sh * ei);
    a.s_w = (uint32_t)(src->sw * ei);
    a.src_extent = (uint32_t)wz_plane_extent(src);
    a.t_h = t_h;
    a.t_plane = (uint32_t)((int64_t)out_h * t_h);
    a.C = src->c;
    a.in_h = src->h;
    a.in_w = src->w;
    a.out_h = out_h;
    a.chunks = (src->w + kPadCols + 64 * kCpl - 1) / (64 * kCpl);
    a.runs = (out_h + kRun - 1) / kRun;
    a.eps4 = eps4_of(p, h, u8);
    a.beta = p->beta;
    const dim3 grid = pass_grid(a.chunks, a.runs, src->n * src->c);
    if (p->beta == 2.0f) {
        if (u8) hipLaunchKernelGGL((rows_pass_kernel<2, true>), grid, dim3(kBlock), 0, st, a, pos);
        else hipLaunchKernelGGL((rows_pass_kernel<2, false>), grid, dim3(kBlock), 0, st, a, pos);
    } else {
        if (u8) hipLaunchKernelGGL((rows_pass_kernel<kBetaGeneral, true>), grid, dim3(kBlock), 0, st, a, pos);
        else hipLaunchKernelGGL((rows_pass_kernel<kBetaGeneral, false>), grid, dim3(kBlock), 0, st, a, pos);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? WENO_OK : wz_hip_error(e, "rows_pass_kernel launch");
}

// The column pass of the padded planes at tmp (dst->h rows of pitch t_h) into dst.
int launch_cols_pass(const uint8_t* tmp, uint32_t t_h, const weno_tensor_t* dst, const weno_params_t* p, double h,
                     const SamplePos* pos, hipStream_t st)
{
    ColPassArgs a;
    const int64_t eo = wz_esize(dst->dtype);
    const bool u8 = dst->dtype == WENO_U8;
    a.tmp = tmp;
    a.dst = (uint8_t*)dst->data;
    a.d_n = dst->sn * eo;
    a.d_c = dst->sc * eo;
    a.d_h = (uint32_t)(dst->sh * eo);
    a.d_w = (uint32_t)(dst->sw * eo);
    a.d_extent = (uint32_t)wz_plane_extent(dst);
    a.t_h = t_h;
    a.t_plane = (uint32_t)((int64_t)dst->h * t_h);
    a.C = dst->c;
    a.out_h = dst->h;
    a.out_w = dst->w;
    a.chunks = (dst->w + 64 * kCpl - 1) / (64 * kCpl);
    a.runs = (dst->h + kRun - 1) / kRun;
    a.eps4 = eps4_of(p, h, false);   // the padded planes are float, on the [0,1] scale for u8 inputs
    a.beta = p->beta;
    const dim3 grid = pass_grid(a.chunks, a.runs, dst->n * dst->c);
    if (p->beta == 2.0f) {
        if (u8) hipLaunchKernelGGL((cols_pass_kernel<2, true>), grid, dim3(kBlock), 0, st, a, pos);
        else hipLaunchKernelGGL((cols_pass_kernel<2, false>), grid, dim3(kBlock), 0, st, a, pos);
    } else {
        if (u8) hipLaunchKernelGGL((cols_pass_kernel<kBetaGeneral, true>), grid, dim3(kBlock), 0, st, a, pos);
        else hipLaunchKernelGGL((cols_pass_kernel<kBetaGeneral, false>), grid, dim3(kBlock), 0, st, a, pos);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? WENO_OK : wz_hip_error(e, "cols_pass_kernel launch");
}

// Launch shape of the fused resampler along a row of n_in -> n_out samples:
// 256 M LDS slots per row and a tile width tw <= 768 whose span fits them,
// ceil((tw - 1)(n_in - 1)/(n_out - 1)) + 4 <= 256 M, with the row's tiles
// balanced.  M = 2 is taken wherever it allows tiles of 64 columns (width
// ratios up to ~7.9): it measured fastest from upsampling by 1.5 to
// downsampling by 1.9, against M = 1 (more tiles, each paying a barrier and
// its pipeline fill per row) and M = 4 (twice the tap registers).  Larger
// ratios take M = 3 or 4; beyond ~16, ok = false and the two passes run.
struct FusedShape {
    bool ok;
    int m, tw, ctiles;
};

FusedShape fused_shape(int n_in, int n_out)
{
    const int64_t num = n_in > 1 ? n_in - 1 : 0, den = n_out > 1 ? n_out - 1 : 1;
    const int64_t min_tw = n_out < 64 ? n_out : 64;
    for (int m = 2; m <= 4; ++m) {
        int64_t twmax = num == 0 ? kFuseMaxTw : ((int64_t)kFuseThreads * m - 4) * den / num + 1;
        if (twmax > kFuseMaxTw) twmax = kFuseMaxTw;
        if (twmax < min_tw) continue;
        const int64_t tiles = (n_out + twmax - 1) / twmax;
        return {true, m, (int)((n_out + tiles - 1) / tiles), (int)tiles};
    }
    return {false, 0, 0, 0};
}

// rows per run of the fused resampler: 8 for small launches, up to 32 once
// there are more than 16 runs' worth of tile rows per compute unit
int fused_run(int out_h, int ctiles, int64_t planes)
{
    const int64_t tile_rows = (int64_t)out_h * ctiles * planes;
    int64_t run = tile_rows / (256 * 16);
    if (run < 8) run = 8;
    if (run > 32) run = 32;
    return (int)run;
}

template <int BETA, int M>
void launch_fused_typed(const FusedArgs& a, bool in_u8, bool out_u8, dim3 grid, const SamplePos* prow,
                        const SamplePos* pcol, hipStream_t st)
{
    if (in_u8 && out_u8)
        hipLaunchKernelGGL((fused_resample_kernel<BETA, M, true, true>), grid, dim3(kFuseThreads), 0, st, a, prow, pcol);
    else if (in_u8)
        hipLaunchKernelGGL((fused_resample_kernel<BETA, M, true, false>), grid, dim3(kFuseThreads), 0, st, a, prow, pcol);
    else if (out_u8)
        hipLaunchKernelGGL((fused_resample_kernel<BETA, M, false, true>), grid, dim3(kFuseThreads), 0, st, a, prow, pcol);
    else
        hipLaunchKernelGGL((fused_resample_kernel<BETA, M, false, false>), grid, dim3(kFuseThreads), 0, st, a, prow, pcol);
}

template <int BETA>
void launch_fused_beta(const FusedArgs& a, int m, bool in_u8, bool out_u8, dim3 grid, const SamplePos* prow,
                       const SamplePos* pcol, hipStream_t st)
{
    switch (m) {
    case 2: launch_fused_typed<BETA, 2>(a, in_u8, out_u8, grid, prow, pcol, st); break;
    case 3: launch_fused_typed<BETA, 3>(a, in_u8, out_u8, grid, prow, pcol, st); break;
    default: launch_fused_typed<BETA, 4>(a, in_u8, out_u8, grid, prow, pcol, st); break;
    }
}

int launch_fused(const weno_tensor_t* src, const weno_tensor_t* dst, const FusedShape& fs, const weno_params_t* p,
                 double h, const SamplePos* prow, const SamplePos* pcol, hipStream_t st)
{
    FusedArgs a;
    const int64_t ei = wz_esize(src->dtype), eo = wz_esize(dst->dtype);
    const bool in_u8 = src->dtype == WENO_U8, out_u8 = dst->dtype == WENO_U8;
    a.src = (const uint8_t*)src->data;
    a.dst = (uint8_t*)dst->data;
    a.s_n = src->sn * ei;
    a.s_c = src->sc * ei;
    a.d_n = dst->sn * eo;
    a.d_c = dst->sc * eo;
    a.s_h = (uint32_t)(src->sh * ei);
    a.s_w = (uint32_t)(src->sw * ei);
    a.d_h = (uint32_t)(dst->sh * eo);
    a.d_w = (uint32_t)(dst->sw * eo);
    a.src_extent = (uint32_t)wz_plane_extent(src);
    a.d_extent = (uint32_t)wz_plane_extent(dst);
    a.C = src->c;
    a.in_h = src->h;
    a.in_w = src->w;
    a.out_h = dst->h;
    a.out_w = dst->w;
    a.tw = fs.tw;
    a.ctiles = fs.ctiles;
    const int64_t planes = (int64_t)src->n * src->c;
    a.run = fused_run(dst->h, fs.ctiles, planes);
    a.eps4_in = eps4_of(p, h, in_u8);
    a.eps4 = eps4_of(p, h, false);
    a.beta = p->beta;
    const int64_t runs = (dst->h + a.run - 1) / a.run;
    const dim3 grid((unsigned)(runs * fs.ctiles), (unsigned)planes);
    if (p->beta == 2.0f) launch_fused_beta<2>(a, fs.m, in_u8, out_u8, grid, prow, pcol, st);
    else launch_fused_beta<kBetaGeneral>(a, fs.m, in_u8, out_u8, grid, prow, pcol, st);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? WENO_OK : wz_hip_error(e, "fused_resample_kernel launch");
}

// row pitch (floats) of workspace planes: a multiple of 4, so that rows are
// 16-byte aligned and the forward kernel stores them with vector stores
int64_t f32_pitch(int64_t w) { return (w + 3) / 4 * 4; }

weno_tensor_t planar_f32(void* data, int n, int c, int h, int w)
{
    weno_tensor_t t;
    t.data = data;
    t.dtype = WENO_F32;
    t.n = n; t.c = c; t.h = h; t.w = w;
    t.sw = 1; t.sh = f32_pitch(w); t.sc = (int64_t)h * t.sh; t.sn = (int64_t)c * t.sc;
    return t;
}

// bytes of planar float planes of h x w (pitched rows), 256-byte aligned
size_t planes_bytes(int64_t planes, int64_t h, int64_t w) { return (size_t)((planes * h * f32_pitch(w) * 4 + 255) / 256 * 256); }

// doublings needed so that 2^k (n - 1) + 1 reaches the target on every axis longer than one sample
int zoom_levels(const weno_tensor_t* src, const weno_tensor_t* dst)
{
    int k = 0;
    while (k < 8 && ((src->h > 1 && ((int64_t)(src->h - 1) << k) + 1 < dst->h) ||
                     (src->w > 1 && ((int64_t)(src->w - 1) << k) + 1 < dst->w)))
        ++k;
    return k;
}

int check_resample_pair(const weno_tensor_t* src, const weno_tensor_t* dst)
{
    int rc = wz_check_tensor(src);
    if (rc) return rc;
    rc = wz_check_tensor(dst);
    if (rc) return rc;
    if (src->n != dst->n || src->c != dst->c) return WENO_EINVAL;
    if ((int64_t)src->n * src->c > 65535) return WENO_EINVAL;
    // offsets within a plane are 32-bit: every plane (and the float
    // intermediate of the row pass) must span less than 2^31 bytes
    if (wz_plane_extent(src) >= (1ll << 31) || wz_plane_extent(dst) >= (1ll << 31)) return WENO_EINVAL;
    if (wz_overlap(src, dst)) return WENO_EOVERLAP;
    return WENO_OK;
}

}  // namespace

// workspace of the resampler: the position tables of the rows and of the
// columns, then (only where the fused kernel does not apply) the row pass's
// padded float planes (dst->h x (in_w + 3))
static size_t resample_bytes(const weno_tensor_t* src, const weno_tensor_t* dst, int64_t in_w)
{
    const size_t tabs = positions_bytes(dst->h) + positions_bytes(dst->w);
    if (fused_shape((int)in_w, dst->w).ok) return tabs;
    return tabs + planes_bytes((int64_t)src->n * src->c, dst->h, in_w + kPadCols);
}

// src (any dtype, in_h x in_w) resampled into dst: the fused kernel, or the
// row pass then the column pass
static int run_resample(const weno_tensor_t* src, const weno_tensor_t* dst, const weno_params_t* p, double h,
                        uint8_t* ws, hipStream_t st)
{
    SamplePos* rows = (SamplePos*)ws;
    SamplePos* cols = (SamplePos*)(ws + positions_bytes(dst->h));
    uint8_t* tmp = ws + positions_bytes(dst->h) + positions_bytes(dst->w);
    const FusedShape fs = fused_shape(src->w, dst->w);
    if (fs.ok) {
        int rc = launch_positions(rows, src->h, dst->h, cols, src->w, dst->w, st);
        if (rc) return rc;
        return launch_fused(src, dst, fs, p, h, rows, cols, st);
    }
    const int64_t pitch = f32_pitch((int64_t)src->w + kPadCols);
    if ((int64_t)dst->h * pitch * 4 >= (1ll << 31)) return WENO_EINVAL;   // 32-bit plane offsets
    weno_tensor_t t = planar_f32(tmp, src->n, src->c, dst->h, src->w + kPadCols);
    if (wz_overlap(&t, src) || wz_overlap(&t, dst)) return WENO_EOVERLAP;
    int rc = launch_positions(rows, src->h, dst->h, cols, src->w, dst->w, st);
    if (rc) return rc;
    rc = launch_rows_pass(src, tmp, (uint32_t)(pitch * 4), dst->h, p, h, rows, st);
    if (rc) return rc;
    return launch_cols_pass(tmp, (uint32_t)(pitch * 4), dst, p, h, cols, st);
}

extern "C" size_t weno_resample_workspace(const weno_tensor_t* src, const weno_tensor_t* dst)
{
    if (check_resample_pair(src, dst) != WENO_OK) return 0;
    return resample_bytes(src, dst, src->w);
}

extern "C" int weno_resample(const weno_tensor_t* src, const weno_tensor_t* dst, const weno_params_t* p,
                             void* d_workspace, size_t ws_bytes, void* hip_stream)
{
    int rc = check_resample_pair(src, dst);
    if (rc) return rc;
    rc = wz_check_params(p);
    if (rc) return rc;
    if (p->boundary != WENO_BOUNDARY_CLAMP) return WENO_EINVAL;   // samples beyond the ends are clamped
    if (!d_workspace || (uintptr_t)d_workspace % 256 != 0) return WENO_EINVAL;   // tables and planes are aligned
    if (ws_bytes < weno_resample_workspace(src, dst)) return WENO_ENOSPC;
    return run_resample(src, dst, p, p->h, (uint8_t*)d_workspace, (hipStream_t)hip_stream);
}

extern "C" size_t weno_zoom_to_workspace(const weno_tensor_t* src, const weno_tensor_t* dst)
{
    if (check_resample_pair(src, dst) != WENO_OK) return 0;
    const int k = zoom_levels(src, dst);
    size_t total = 0;
    int64_t h = src->h, w = src->w;
    for (int l = 0; l < k; ++l) {
        total += planes_bytes((int64_t)src->n * src->c, 2 * h, 2 * w);
        h = 2 * h - 1;
        w = 2 * w - 1;
    }
    return total + resample_bytes(src, dst, w);
}

int wz_launch_fwd(const weno_tensor_t* src, const weno_tensor_t* dst, const weno_params_t* p, hipStream_t st, int rows,
                  int cols, int tail_rows);
void wz_config_for(const weno_tensor_t* src, const weno_tensor_t* dst, int* rows, int* cols, int* tail_rows);

extern "C" int weno_zoom_to(const weno_tensor_t* src, const weno_tensor_t* dst, const weno_params_t* p,
                            void* d_workspace, size_t ws_bytes, void* hip_stream)
{
    int rc = check_resample_pair(src, dst);
    if (rc) return rc;
    rc = wz_check_params(p);
    if (rc) return rc;
    if (p->boundary != WENO_BOUNDARY_CLAMP) return WENO_EINVAL;   // samples beyond the ends are clamped
    if (!d_workspace || (uintptr_t)d_workspace % 256 != 0) return WENO_EINVAL;   // tables and planes are aligned
    if (ws_bytes < weno_zoom_to_workspace(src, dst)) return WENO_ENOSPC;
    hipStream_t st = (hipStream_t)hip_stream;
    const int k = zoom_levels(src, dst);
    const double w0 = wz_nbw(p);
    weno_tensor_t cur = *src;
    uint8_t* ws = (uint8_t*)d_workspace;
    size_t off = 0;
    for (int l = 0; l < k; ++l) {
        weno_tensor_t out = planar_f32(ws + off, src->n, src->c, 2 * cur.h, 2 * cur.w);
        off += planes_bytes((int64_t)src->n * src->c, out.h, out.w);
        if (wz_overlap(&out, src) || wz_overlap(&out, dst)) return WENO_EOVERLAP;
        rc = wz_check_pair(&cur, &out, 2);
        if (rc) return rc;
        weno_params_t lp = *p;
        const double scale = std::ldexp(1.0, -l);
        lp.h = (float)(p->h * scale);
        lp.nbw = (float)(w0 * scale * scale);
        int rows, cols;
        int tail;
        wz_config_for(&cur, &out, &rows, &cols, &tail);
        rc = wz_launch_fwd(&cur, &out, &lp, st, rows, cols, tail);
        if (rc) return rc;
        // the paper's nested grid: the leading (2n - 1) x (2m - 1) samples
        cur = out;
        cur.h = 2 * (cur.h / 2) - 1;
        cur.w = 2 * (cur.w / 2) - 1;
    }
    weno_params_t rp = *p;
    rp.h = (float)(p->h * std::ldexp(1.0, -k));
    return run_resample(&cur, dst, &rp, rp.h, ws + off, st);
}
