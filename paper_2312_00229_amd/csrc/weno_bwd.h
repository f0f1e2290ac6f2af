// Adjoint of the WD-WENO 2x doubling for gfx950: dL/dV from dL/dU.
//
// Reverse-mode differentiation of arXiv 2312.00229, Section 3 (phase 1:
// eqs. p, 2Dsmoothness, 2DsmoothnessFinal, alpha, IzrazOmega2d,
// 2dKombinacija; phase 2: eqs. tezine, IzrazOmega2dRavno,
// 2dKombinacijaRavno).  At a point with candidates p_k, t_k = eps + D_k and
// blend u:
//     du/dp_k = omega_k,   du/dt_k = -beta omega_k (p_k - u) / t_k,
// t_k takes its own indicator with weight 1 and four neighbour indicators of
// the same direction with weight w; a candidate and an indicator of a stencil
// (a, b, c) (nodes -1, 1, 3; g = b - a, dd = a - 2b + c) have
//     p = (a + b)/2 - dd/8,     dp/d(a,b,c) = (3/8, 3/4, -1/8).
// The walk keeps half samples (v/2 of the input and of the x points), so a
// stencil gives gh = g/2, ddh = dd/2 and the midpoint (a + b)/2 = ha + hb in
// one addition, and it carries the indicators scaled by 3/13:
//     SI* = (3/13) SI = gh f + ddh^2 with f = (12/13) gh,
//     dSI*/d(a,b,c) = (ddh - f, f - 2 ddh, ddh),
// so each derivative term is one product (t* = (3/13) t, and the formula
// for du/dt*_k is the same in the scaled variables).
//
// Work decomposition: like the forward, one wave walks a strip of 64 input
// columns (one per lane) down the image; horizontal neighbours come from DPP
// shifts, so every scatter of the adjoint becomes a gather from adjacent
// lanes, with no atomics: each dL/dV element is written by exactly one lane,
// and the result is deterministic.  Iteration s:
//   forward     the forward pipeline (rows up to s+5), blends of A(s), B(s)
//               and x(s+2) keep the weight factors the seeds need (those of
//               x(s+2) wait in LDS until iteration s+4, the diagonal second
//               differences of input row s+4 until iterations s+6, s+7);
//   seeds       phase-2 seeds of A(s), B(s) from dL/dU;
//   p2 adjoint  indicator adjoints of A(s-1) and B(s); stencil adjoints into
//               dL/dx (rows s-2..s+1) and dL/dV (rows s-2..s+1);
//   p1 seeds    dL/dx of row s-2 is complete: seeds of x(s-2);
//   p1 adjoint  indicator adjoints of x(s-3); stencil adjoints into dL/dV
//               rows s-4..s-1 (the slopes from input rows s-3, s-2 held in a
//               register window, the second differences from LDS);
//   output      dL/dV row s-4 is complete: fold clamped rows/columns onto the
//               edge pixels and store.
// Valid lanes shrink with every neighbour access: the dL/dV of lanes 9..54 is
// exact.  A quad reads inputs I-4 .. I+5 and J-4 .. J+5, so clamped reads
// reach four padded columns left of the image and five right of it (rows
// likewise: four above, five below), all folded onto the edge pixels.  The
// first strip of a row starts at lane 13 so that the four padded columns
// left of the image fall in lanes 9..12 and owns 42 columns; the last starts
// at lane 9 and owns at most 41, which leaves lanes up to 54 for the five
// padded columns right of the image; the strips between own all 46 exact
// lanes.  A strip that is both first and last holds at most 37 columns, so
// images 38..42 wide are split into two strips of 21 and the rest.
#pragma once

#include <stdint.h>

#include <type_traits>

#include "weno_fwd.h"

namespace wz {

constexpr int kBwdLane0First = 13; // lane of the first owned column, first strip of a row
constexpr int kBwdLane0 = 9;       // lane of the first owned column, other strips
constexpr int kBwdOwnFirst = 42;   // columns of the first strip of a row (lanes 13..54)
constexpr int kBwdOwnMid = 46;     // columns of a strip between the first and the last (lanes 9..54)
constexpr int kBwdOwnLast = 41;    // at most, in the last strip (its five padded columns take lanes up to 54)
constexpr int kBwdOwnSingle = 37;  // at most, in a strip that is both first and last (lanes 13..49)

// Strip layout along a row of W columns (host and device).  The exact lanes
// of a strip are 9..54.  The first strip owns columns from lane 13 (lanes
// 9..12 carry the four padded columns left of the image), the last owns at
// most 41 so that the five padded columns right of the image fall in lanes up
// to 54, and strips in between own all 46.  A strip that is both first and
// last holds at most 37 columns: widths 38..42 are two strips, 21 and W - 21.
__host__ __device__ inline int bwd_strip_count(int W)
{
    if (W <= kBwdOwnSingle) return 1;
    if (W <= 42) return 2;
    const int R = W - kBwdOwnFirst;   // columns after the first strip
    if (R <= kBwdOwnLast) return 2;
    return 2 + (R - kBwdOwnLast + kBwdOwnMid - 1) / kBwdOwnMid;
}

// first column c0 and width of strip sx of a row of W columns
__host__ __device__ inline void bwd_strip_span(int W, int sx, int& c0, int& width)
{
    if (W <= kBwdOwnSingle) {
        c0 = 0;
        width = W;
        return;
    }
    if (W <= 42) {
        c0 = 21 * sx;
        width = sx == 0 ? 21 : W - 21;
        return;
    }
    if (sx == 0) {
        c0 = 0;
        width = kBwdOwnFirst;
        return;
    }
    const int n = bwd_strip_count(W), mid = n - 2;
    // the last strip takes what the middle ones leave, at least one column
    // (the last middle strip gives up what that needs)
    const int r = W - kBwdOwnFirst - kBwdOwnMid * mid;
    const int last = r < 1 ? 1 : r;
    if (sx == n - 1) {
        c0 = W - last;
        width = last;
        return;
    }
    c0 = kBwdOwnFirst + kBwdOwnMid * (sx - 1);
    width = sx < n - 2 ? kBwdOwnMid : (W - last) - c0;
}

// Iterations before the first exact dL/dV row.  A walk that starts at row a
// (windows holding fill values) has exact V rows from a+5, second differences
// and x-point indicators from a+6, x-point blends from a+7, +-point blends
// from a+9, their adjoint from a+10, complete dL/dx rows from a+11 and the
// x-point adjoint from a+15; that last one feeds dL/dV rows r-1 .. r+2, so
// the first exact dL/dV row is a+14.  The top strip also folds the padded
// rows -4..-1 onto row 0, so it starts 4 rows earlier; the bottom strip walks
// on until dL/dV row H+4, the last padded row a quad of row H-1 reads.
constexpr int kBwdWarm = 14;
constexpr int kBwdWarmTop = 18;
// The first 9 iterations of a walk from row a run the forward pipeline only.
// Their adjoint work would reach dL/dV rows before a+14 alone: the seeds of
// A(a+9) enter the indicator adjoint of B(a+10), which feeds dL/dx row a+11,
// whose phase-1 seed couples into x row a+12 and so into dL/dV row a+14; the
// seeds of row a+8 and earlier stop at dL/dV row a+13.  (Checked bit for bit
// against the full walk on strip heights 4..40, beta 1, 1.5 and 2: a tenth
// forward-only iteration changes the stored rows.)  Forward-only iterations
// run only the stages whose results reach the first full iteration.
constexpr int kBwdForwardOnly = 9;
// Warm-up cost of a strip in full-iteration equivalents, for the launch
// model: the 14 warm-up iterations (9 forward-only with partial stages, then
// full ones without the phase-1 adjoint) together with the fixed cost of
// starting a wave.  Fitted on MI355X: 8 picks the best measured strip height
// on 3x512^2, 1x2048^2, 3x720x1280 and the shapes of the launch-model fit.
constexpr int kBwdWarmCost = 8;

struct BwdCtx {
    rsrc_t x, gy, gx;           // one plane each: forward input, dL/dU (2H x 2W), dL/dV (H x W); float32
    uint32_t x_h, gy_h, gx_h;   // row strides in bytes
    uint32_t x_w, gy_w, gx_w;   // column strides in bytes
    int32_t H, W;
};

__device__ __forceinline__ float nbL(float x) { return from_left(x); }   // value of column J-1
__device__ __forceinline__ float nbR(float x) { return from_right(x); }  // value of column J+1

// blend with the factors of the seeds: om_k = omega_k, dk_k = omega_k (p_k - u) / t_k
template <int BETA>
__device__ __forceinline__ float blend_seed(const float (&t)[4], const float (&p)[4], float beta, float (&om)[4],
                                            float (&dk)[4])
{
    float a[4], r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if constexpr (BETA == 2) {
            r[k] = rcp(t[k]);
            a[k] = r[k] * r[k];
        } else if constexpr (BETA == 1) {
            r[k] = rcp(t[k]);
            a[k] = r[k];
        } else {
            a[k] = __builtin_amdgcn_exp2f(-beta * __builtin_amdgcn_logf(t[k]));
            r[k] = rcp(t[k]);
        }
    }
    const float S = (a[0] + a[1]) + (a[2] + a[3]);
    const float N = __builtin_fmaf(a[3], p[3], __builtin_fmaf(a[2], p[2], __builtin_fmaf(a[1], p[1], a[0] * p[0])));
    const float rS = rcp(S);
    const float u = N * rS;
#pragma unroll
    for (int k = 0; k < 4; ++k) om[k] = a[k] * rS;
    // p_k - u = sum_j omega_j (p_k - p_j): where one direction dominates
    // (omega_k ~ 1, t_k ~ eps) the exact p_k - u is far below the rounding of
    // u itself, while each omega_j (p_k - p_j) keeps its relative precision.
    const float d01 = p[0] - p[1], d02 = p[0] - p[2], d03 = p[0] - p[3];
    const float d12 = p[1] - p[2], d13 = p[1] - p[3], d23 = p[2] - p[3];
    const float e0 = __builtin_fmaf(om[3], d03, __builtin_fmaf(om[2], d02, om[1] * d01));
    const float e1 = __builtin_fmaf(om[3], d13, __builtin_fmaf(om[2], d12, -(om[0] * d01)));
    const float e2 = __builtin_fmaf(om[3], d23, -__builtin_fmaf(om[1], d12, om[0] * d02));
    const float oe0 = om[0] * e0, oe1 = om[1] * e1, oe2 = om[2] * e2;
    // The omega_k (p_k - u) sum to zero (a sum of omega_k omega_j (p_k - p_j)
    // over ordered pairs), so the last is minus the sum of the others.  Its
    // rounding error is ~1e-7 of the largest of them, and it is scaled by
    // 1/t_3 no more than the largest is scaled by its own 1/t_k.
    const float oe3 = -((oe0 + oe1) + oe2);
    dk[0] = oe0 * r[0];
    dk[1] = oe1 * r[1];
    dk[2] = oe2 * r[2];
    dk[3] = oe3 * r[3];
    return u;
}

// slope factor of an indicator in the scale 3/13: f = (12/13) gh
constexpr float kSlopeF = 12.0f / 13.0f;
__device__ __forceinline__ float slope_f(float gh) { return kSlopeF * gh; }
// candidate (a + b)/2 - dd/8 from the midpoint m = ha + hb and ddh = dd/2
__device__ __forceinline__ float cand_h(float ddh, float m) { return __builtin_fmaf(ddh, -0.25f, m); }

// adjoint of the two stencils of one line: the forward one (x0, x1, x2) and
// the backward one (x1, x0, x-1), with slope factor f = (12/13)(x1 - x0)/2
// (the forward stencil's; the backward one's is -f) and their own half second
// differences ddf, ddb.  Returns the gradients at x0 (s0 = ga_f + gb_b), x1
// (s1 = gb_f + ga_b), x2 (cf) and x-1 (cb).  A stencil (a, b, c) with
// candidate seed gp and seed gs of its scaled indicator gives
//   ga = 3/8 gp + gs (ddh - f),  gb = 3/4 gp + gs (f - 2 ddh),  gc = -1/8 gp + gs ddh;
// written per line rather than per stencil, the slope terms of the two
// stencils fold into one product F = f (gs_f + gs_b), and with E = gs ddh
//   s0 = 3/8 gp_f + 3/4 gp_b + E_f - 2 E_b - F
//   s1 = 3/4 gp_f + 3/8 gp_b - 2 E_f + E_b + F
//   cf = -1/8 gp_f + E_f,   cb = -1/8 gp_b + E_b
// (14 operations against 20 for two stencils and the two sums).
__device__ __forceinline__ void line_adj(float gpf, float gsf, float ddf, float gpb, float gsb, float ddb, float f,
                                         float& s0, float& s1, float& cf, float& cb)
{
    const float ef = gsf * ddf, eb = gsb * ddb;
    const float F = (gsf + gsb) * f;
    s0 = __builtin_fmaf(gpf, 0.375f, __builtin_fmaf(gpb, 0.75f, __builtin_fmaf(eb, -2.0f, ef - F)));
    s1 = __builtin_fmaf(gpf, 0.75f, __builtin_fmaf(gpb, 0.375f, __builtin_fmaf(ef, -2.0f, eb + F)));
    cf = __builtin_fmaf(gpf, -0.125f, ef);
    cb = __builtin_fmaf(gpb, -0.125f, eb);
}

typedef float bwd_f32x4 __attribute__((ext_vector_type(4)));

// LDS of one wave: the x-point seed factors, 4 slots (a row each) x
// (omega_k, dk_k) x 64 lanes of 4 floats, then the diagonal second
// differences of the input rows, 8 slots (a row each) x 64 lanes of 4 floats
constexpr int kBwdSeedWords = 4 * 2 * kWave;
constexpr int kBwdRingWords = kBwdSeedWords + 8 * kWave;
typedef float bwd_f32x2 __attribute__((ext_vector_type(2)));

template <int BETA>
__device__ __forceinline__ void bwd_strip(const BwdCtx& cx, const FwdParams& P, int strip_x, int R0, int R1,
                                          bwd_f32x4* __restrict__ ring)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int H = cx.H, W = cx.W;
    int c0, width;
    bwd_strip_span(W, strip_x, c0, width);
    const int lane0 = strip_x == 0 ? kBwdLane0First : kBwdLane0;
    const int J = c0 - lane0 + lane;
    const bool own = lane >= lane0 && lane < lane0 + width && J < W;
    const bool colin = J >= 0 && J < W;
    const int jc = J < 0 ? 0 : (J >= W ? W - 1 : J);
    const uint32_t xoff = (uint32_t)jc * cx.x_w;
    // dL/dU outside the 2H x 2W grid counts as 0: lanes outside the image and
    // rows outside it read through an offset past the end of the buffer, which
    // the buffer unit answers with 0 and no memory access, so the loads need no
    // branch and can be issued a step before their use
    // Lanes outside the image read at column offset kOobCol, rows outside it
    // at row offset kOobRow: either puts the sum at or above every plane
    // extent (< 2^31), and the two together stay below 2^32 (no wrap).  The
    // row offset is uniform, so the choice for a row is a scalar select.
    constexpr uint32_t kOobCol = 0x7fffffffu, kOobRow = 0x80000000u;
    const uint32_t gyoffA = colin ? (uint32_t)(2 * jc) * cx.gy_w : kOobCol;        // column 2J
    const uint32_t gyoffB = colin ? (uint32_t)(2 * jc + 1) * cx.gy_w : kOobCol;    // column 2J+1
    const uint32_t gxoff = (uint32_t)jc * cx.gx_w;
    const bool first_strip = c0 == 0;
    const bool last_strip = c0 + width >= W;
    const bool top = R0 == 0, bottom = R1 == H;
    const float eh = P.eps_hat, w = P.w, beta = P.beta;

    auto ldV = [&](int r) {
        const int rc = r < 0 ? 0 : (r >= H ? H - 1 : r);
        return buf_ld_f32(cx.x, xoff, (uint32_t)rc * cx.x_h);
    };
    auto ldG = [&](int r, uint32_t off) {   // dL/dU element, 0 outside the 2H x 2W grid
        const bool in = r >= 0 && r < 2 * H;
        return buf_ld_f32(cx.gy, off, in ? (uint32_t)r * cx.gy_h : kOobRow);
    };
    auto stG = [&](int r, float val) { buf_st_f32(val, cx.gx, gxoff, (uint32_t)r * cx.gx_h); };

    // ---------------- forward state (rows relative to s) ----------------
    // half samples: V(r) holds v(r)/2, X(r) the x point of row r over 2
    float Vm3 = 0, Vm2 = 0, Vm1 = 0;                    // V(s-3) .. V(s-1)
    float V0 = 0, V1 = 0, V2 = 0, V3 = 0, V4 = 0;       // V(s) .. V(s+4)
    float dd1_3 = 0, dd2s_3 = 0;
    // indicator windows start at 1 so that pipeline-fill blends never divide by zero
    float SX1[4] = {1, 1, 1, 1}, SX2[4] = {1, 1, 1, 1}, PX2[4] = {};
    float X0 = 0, X1 = 0, ddXv0 = 0, ddr0 = 0;
    float SB0[4] = {1, 1, 1, 1}, PB0[4] = {}, hB0[4] = {1, 1, 1, 1}, hAm1[4] = {1, 1, 1, 1};
    // stencil geometry (slope factor f, half second differences per
    // direction) of B(s) and A(s-1)
    float geoB_fv = 0, geoB_ddd = 0, geoB_ddu = 0, geoB_fh = 0, geoB_ddr = 0, geoB_ddl = 0;
    float geoA_fv = 0, geoA_ddd = 0, geoA_ddu = 0, geoA_fh = 0, geoA_ddr = 0, geoA_ddl = 0;
    // The seed factors of x row s+2 (omega_k and omega_k (p_k - u) / t_k),
    // made at step s, are used at step s+4.  They wait in LDS rather than in
    // registers: slot s & 3 holds them from step s until step s+4 reads it
    // and then overwrites it with its own (each lane reads and writes only its
    // own words, so program order is all the ordering needed).
    int s_ref = 0;   // ring slots count steps from s_ref (set before the first full step)
    auto ring_at = [&](int slot, int half) -> bwd_f32x4& { return ring[(slot * 2 + half) * kWave + lane]; };
    // The diagonal second differences of input row r, {dd1, dd2s, dd1s, dd2}
    // (dd1, dd2 centred at (r, J), dd1s, dd2s at (r, J+1)), made when row r
    // enters the pipeline (step r-4) and read by the phase-1 adjoints of
    // steps r+2 (the .zw half) and r+3 (the .xy half); slot r & 7 is next
    // written at step r+4.
    // Slot of row r: (r - s_ref) & 7.  In the interior trips (steps
    // s_ref + 4i + k) a slot m of the trip's first step is m ^ 4 in the next
    // trip, so dd_lo / dd_hi (slots 0..3 / 4..7 of this lane) trade places
    // after every trip and each access is a fixed base and offset.
    bwd_f32x2* const dd_base = reinterpret_cast<bwd_f32x2*>(ring + kBwdSeedWords + lane);
    bwd_f32x2* dd_lo = dd_base;
    bwd_f32x2* dd_hi = dd_base + 4 * 2 * kWave;
    auto dd_at = [&](int r, int half) -> bwd_f32x2& { return dd_base[((r - s_ref) & 7) * 2 * kWave + half]; };
    auto dd_at_m = [&](auto mc, int half) -> bwd_f32x2& {   // interior: slot m of the trip's frame
        constexpr int m = decltype(mc)::value;
        return ((m & 4) ? dd_hi : dd_lo)[(m & 3) * 2 * kWave + half];
    };
    // ---------------- adjoint state ----------------
    float gtA_m1[4] = {}, gpA_m1[4] = {}, qA_m1[4] = {}, qB_m1[4] = {};
    float accX_m2 = 0, accX_m1 = 0, accX_0 = 0;          // dL/dx rows s-2, s-1, s
    float gtX_m4[4] = {}, gtX_m3[4] = {}, gpX_m3[4] = {};
    float accV_m4 = 0, accV_m3 = 0, accV_m2 = 0, accV_m1 = 0, accV_0 = 0;  // dL/dV rows s-4 .. s
    // the phase-1 term of dL/dV row s-1 from column J-2, kept until row s-1 completes
    float dcV_m3 = 0, dcV_m2 = 0, dcV_m1 = 0;
    float fold_top = 0, held = 0;

    // Pacing by wave priority, as in the doubling: waves sharing a SIMD are
    // otherwise served oldest first, so one runs ahead and the SIMD ends its
    // work on a lone latency-bound wave.  A wave starts at the top priority
    // and steps down as it passes each quarter of its full iterations, so
    // the wave that has done less goes first.  Unlike the doubling this pays
    // in launches of several rounds too (16x3x512x512: 303 -> 288 us; 3x1080x1920:
    // 148 -> 137 us).
    __builtin_amdgcn_s_setprio(3);
    const int s_end = bottom ? H + 8 : R1 + 3;   // dL/dV row s - 4 completes at step s
    int s = R0 - (top ? kBwdWarmTop : kBwdWarm);
    // loads run ahead of their use: V two rows, dL/dU one step
    float Q0 = ldV(s + 5), Q1 = ldV(s + 6);
    float nA = 0, nB = 0, nX = 0, nV = 0;
    // D = 0: a full iteration.  D = -9 .. -1: the forward-only iteration
    // a + 9 + D of a walk that starts at row a (the first kBwdForwardOnly
    // iterations only fill the forward pipeline; their adjoint work would
    // reach only rows before R0).  Like the doubling's prologue, each runs only
    // the stages whose results reach the first full iteration: second
    // differences from D = -7, x-point indicators from -6, x-point blends and
    // their seed factors (read four iterations later) from -4, the vertical
    // differences of the + points from -2 and the + points from -1.
    // P1 = false (full iterations only): skip the phase-1 stencil adjoint and
    // the output, which reach only rows this strip never stores
    auto step = [&](const int s, auto dconst, auto p1, auto slotc) {
        constexpr int D = decltype(dconst)::value;
        constexpr bool FULL = D == 0;
        constexpr bool do_dd = FULL || D >= -7, do_sx = FULL || D >= -6, do_x = FULL || D >= -4;
        constexpr bool do_p2dd = FULL || D >= -2, do_p2 = FULL || D >= -1;
        constexpr int P1M = decltype(p1)::value;
        constexpr bool P1 = P1M != 0, INTERIOR = P1M == 2;
        // slot of the seed-factor ring: (s - s_ref) & 3, a constant in the
        // interior trips (their steps are s_ref + 4i + k)
        int slot;
        if constexpr (std::is_integral<decltype(slotc)>::value) slot = (s - s_ref) & 3;
        else slot = decltype(slotc)::value;
        const float V5 = 0.5f * Q0;
        Q0 = Q1;
        Q1 = ldV(s + 7);
        float gA = 0, gB = 0, gXu = 0, gVu = 0;
        bwd_f32x4 omXr = {}, dkXr = {};   // seed factors of x row s-2
        // second differences of input rows s-3 (.xy) and s-2 (.zw) for the
        // phase-1 adjoint, read before this step writes row s+4's slot
        bwd_f32x2 ddm3 = {}, ddm2 = {};
        if constexpr (P1) {
            if constexpr (std::is_integral<decltype(slotc)>::value) {
                ddm3 = dd_at(s - 3, 0);
                ddm2 = dd_at(s - 2, 1);
            } else {
                constexpr int k = decltype(slotc)::value;
                ddm3 = dd_at_m(std::integral_constant<int, (k - 3) & 7>{}, 0);
                ddm2 = dd_at_m(std::integral_constant<int, (k - 2) & 7>{}, 1);
            }
        }
        if constexpr (FULL) {
            omXr = ring_at(slot, 0);
            dkXr = ring_at(slot, 1);
            gA = nA; gB = nB; gXu = nX; gVu = nV;
            nA = ldG(2 * s + 3, gyoffA);
            nB = ldG(2 * s + 2, gyoffB);
            nX = ldG(2 * s - 1, gyoffB);
            nV = ldG(2 * s - 6, gyoffA);
        }
        // ======================= forward =======================
        float dd1_4 = 0.0f, dd2_4 = 0.0f, dd1s_4 = 0.0f, dd2s_4 = 0.0f;
        if constexpr (do_dd) {
            dd1_4 = d2(nbL(V3), V4, nbR(V5));
            dd2_4 = d2(nbR(V3), V4, nbL(V5));
            dd1s_4 = nbR(dd1_4);
            dd2s_4 = nbR(dd2_4);
            if constexpr (std::is_integral<decltype(slotc)>::value) {
                dd_at(s + 4, 0) = bwd_f32x2{dd1_4, dd2s_4};
                dd_at(s + 4, 1) = bwd_f32x2{dd1s_4, dd2_4};
            } else {
                constexpr int k = decltype(slotc)::value;
                dd_at_m(std::integral_constant<int, (k + 4) & 7>{}, 0) = bwd_f32x2{dd1_4, dd2s_4};
                dd_at_m(std::integral_constant<int, (k + 4) & 7>{}, 1) = bwd_f32x2{dd1s_4, dd2_4};
            }
        }
        // x row s+3
        float SX3[4] = {1, 1, 1, 1}, PX3[4] = {};
        if constexpr (do_sx) {
            const float a1 = V3, b1 = nbR(V4), a2 = nbR(V3), b2 = V4;
            const float g1 = b1 - a1, g2 = b2 - a2;
            const float gc1 = __builtin_fmaf(g1, slope_f(g1), eh), gc2 = __builtin_fmaf(g2, slope_f(g2), eh);
            const float m1 = a1 + b1, m2 = a2 + b2;
            SX3[0] = sidx(dd1s_4, gc1);  PX3[0] = cand_h(dd1s_4, m1);
            SX3[2] = sidx(dd1_3, gc1);   PX3[2] = cand_h(dd1_3, m1);
            SX3[1] = sidx(dd2s_3, gc2);  PX3[1] = cand_h(dd2s_3, m2);
            SX3[3] = sidx(dd2_4, gc2);   PX3[3] = cand_h(dd2_4, m2);
        }
        // x row s+2 with its seed factors
        float X2 = 0.0f;
        if constexpr (do_x) {
            float omX2[4], dkX2[4];
            float t[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                // one neighbour shift per addition, so each folds into it (DPP operand)
                const float ns = ((SX1[k] + SX3[k]) + nbL(SX2[k])) + nbR(SX2[k]);
                t[k] = __builtin_fmaf(w, ns, SX2[k]);
            }
            X2 = 0.5f * blend_seed<BETA>(t, PX2, beta, omX2, dkX2);
            // The factors written at iteration s feed the phase-1 seeds of x
            // row s+2 at iteration s+4, which a kept row needs only from the
            // first full iteration's write on (rows s+2 >= R0-3, or >= -7 for
            // the top strip); the first four full iterations read slots the
            // forward-only ones leave unwritten, and their seeds reach only
            // phase-1 adjoints that are skipped.
            if constexpr (FULL) {
                ring_at(slot, 0) = bwd_f32x4{omX2[0], omX2[1], omX2[2], omX2[3]};
                ring_at(slot, 1) = bwd_f32x4{dkX2[0], dkX2[1], dkX2[2], dkX2[3]};
            }
        }
        float ddXv1 = 0.0f, ddr1 = 0.0f;
        if constexpr (do_p2dd) {
            ddXv1 = d2(X0, X1, X2);
            ddr1 = d2(V0, V1, V2);
        }
        // + points: B(s+1) and A(s)
        float SB1[4] = {1, 1, 1, 1}, PB1[4] = {}, hB1[4] = {1, 1, 1, 1};
        float SA0[4] = {1, 1, 1, 1}, PA0[4] = {}, hA0[4] = {1, 1, 1, 1};
        float nB_fv = 0, nB_ddd = 0, nB_ddu = 0, nB_fh = 0, nB_ddr = 0, nB_ddl = 0;   // geometry of B(s+1)
        float nA_fv = 0, nA_ddd = 0, nA_ddu = 0, nA_fh = 0, nA_ddr = 0, nA_ddl = 0;   // geometry of A(s)
        if constexpr (do_p2) {
            const float v1r = nbR(V1);
            const float ddc = d2(nbL(V1), V1, v1r);
            const float x0l = nbL(X0);
            const float ddXh = d2(x0l, X0, nbR(X0));
            // B(s+1)
            const float gBv = X1 - X0, gBh = v1r - V1;
            nB_fv = slope_f(gBv); nB_ddd = ddXv1;  nB_ddu = ddXv0;
            nB_fh = slope_f(gBh); nB_ddr = nbR(ddc); nB_ddl = ddc;
            const float gcv = __builtin_fmaf(gBv, nB_fv, eh), mv = X0 + X1;
            const float gch = __builtin_fmaf(gBh, nB_fh, eh), mh = V1 + v1r;
            SB1[0] = sidx(nB_ddd, gcv); PB1[0] = cand_h(nB_ddd, mv);
            SB1[2] = sidx(nB_ddu, gcv); PB1[2] = cand_h(nB_ddu, mv);
            SB1[1] = sidx(nB_ddr, gch); PB1[1] = cand_h(nB_ddr, mh);
            SB1[3] = sidx(nB_ddl, gch); PB1[3] = cand_h(nB_ddl, mh);
            // A(s)
            const float gAv = V1 - V0, gAh = X0 - x0l;
            nA_fv = slope_f(gAv); nA_ddd = ddr1;  nA_ddu = ddr0;
            nA_fh = slope_f(gAh); nA_ddr = ddXh;  nA_ddl = nbL(ddXh);
            const float gav = __builtin_fmaf(gAv, nA_fv, eh), mav = V0 + V1;
            const float gah = __builtin_fmaf(gAh, nA_fh, eh), mah = x0l + X0;
            SA0[0] = sidx(nA_ddd, gav); PA0[0] = cand_h(nA_ddd, mav);
            SA0[2] = sidx(nA_ddu, gav); PA0[2] = cand_h(nA_ddu, mav);
            SA0[1] = sidx(nA_ddr, gah); PA0[1] = cand_h(nA_ddr, mah);
            SA0[3] = sidx(nA_ddl, gah); PA0[3] = cand_h(nA_ddl, mah);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                hB1[k] = nbL(SB1[k]) + SB1[k];
                hA0[k] = SA0[k] + nbR(SA0[k]);
            }
        }
        // blends of A(s), B(s) with seed factors
        float omA[4] = {}, dkA[4] = {}, omB[4] = {}, dkB[4] = {};
        if constexpr (FULL) {
            float ta[4], tb[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ta[k] = __builtin_fmaf(w, hB0[k] + hB1[k], SA0[k]);
                tb[k] = __builtin_fmaf(w, hAm1[k] + hA0[k], SB0[k]);
            }
            (void)blend_seed<BETA>(ta, PA0, beta, omA, dkA);
            (void)blend_seed<BETA>(tb, PB0, beta, omB, dkB);
        }

        // ======================= phase-2 seeds =======================
        float gtA[4] = {}, gpA[4] = {}, gtB[4] = {}, gpB[4] = {}, qA[4] = {}, qB[4] = {};
        // accumulators start at -0: -0 + x is x for every x, so the first sum is free
        float accX_p1 = -0.0f, accV_p1 = -0.0f;
        float gtX_m2[4] = {}, gpX_m2[4] = {};
        float dcV_0 = 0.0f;
        if constexpr (FULL) {
        // -beta folds into the seed first (exact for beta = 1 and 2)
        const float gAb = -beta * gA, gBb = -beta * gB;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            gpA[k] = gA * omA[k];
            gtA[k] = gAb * dkA[k];
            gpB[k] = gB * omB[k];
            gtB[k] = gBb * dkB[k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            qB[k] = gtB[k] + nbL(gtB[k]);   // gt_B(s, J) + gt_B(s, J-1)
            qA[k] = gtA[k] + nbR(gtA[k]);   // gt_A(s, J) + gt_A(s, J+1)
        }

        // ======================= phase-2 adjoint =======================
        {
            // A(s-1): indicator seeds gS = gt_A(s-1) + w [gt_B box over rows s-1, s, cols J-1, J]
            float gs[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) gs[k] = __builtin_fmaf(w, qB_m1[k] + qB[k], gtA_m1[k]);
            float s0, s1, cf, cb;
            // vertical stencils on V column J: k0 (V(s-1), V(s), V(s+1)), k2 (V(s), V(s-1), V(s-2))
            line_adj(gpA_m1[0], gs[0], geoA_ddd, gpA_m1[2], gs[2], geoA_ddu, geoA_fv, s0, s1, cf, cb);
            accV_m1 += s0;
            accV_0 += s1;
            accV_p1 += cf;
            accV_m2 += cb;
            // horizontal stencils on x row s-1: k1 (x[J-1], x[J], x[J+1]), k3 (x[J], x[J-1], x[J-2])
            line_adj(gpA_m1[1], gs[1], geoA_ddr, gpA_m1[3], gs[3], geoA_ddl, geoA_fh, s0, s1, cf, cb);
            const float u = s0 + nbR(cb);
            accX_m1 += (s1 + nbR(u)) + nbL(cf);
        }
        {
            // B(s): gS = gt_B(s) + w [gt_A box over rows s-1, s, cols J, J+1]
            float gs[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) gs[k] = __builtin_fmaf(w, qA_m1[k] + qA[k], gtB[k]);
            float s0, s1, cf, cb;
            // vertical stencils on x column J: k0 (x(s-1), x(s), x(s+1)), k2 (x(s), x(s-1), x(s-2))
            line_adj(gpB[0], gs[0], geoB_ddd, gpB[2], gs[2], geoB_ddu, geoB_fv, s0, s1, cf, cb);
            accX_m1 += s0;
            accX_0 += s1;
            accX_p1 += cf;
            accX_m2 += cb;
            // horizontal stencils on V row s: k1 (V[J], V[J+1], V[J+2]), k3 (V[J+1], V[J], V[J-1])
            line_adj(gpB[1], gs[1], geoB_ddr, gpB[3], gs[3], geoB_ddl, geoB_fh, s0, s1, cf, cb);
            const float v = s1 + nbL(cf);
            accV_0 += (s0 + nbL(v)) + nbR(cb);
        }

        // ======================= phase-1 seeds at x row s-2 =======================
        const float gXc = accX_m2 + gXu, gXb = -beta * gXc;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            gpX_m2[k] = gXc * omXr[k];
            gtX_m2[k] = gXb * dkXr[k];
        }

        // ======================= phase-1 adjoint at x row r = s-3 =======================
        if constexpr (P1) {
            const float Qv = Vm3, Rv = Vm2;
            const float dd1_r = ddm3.x, dd2s_r = ddm3.y, dd1s_r1 = ddm2.x, dd2_r1 = ddm2.y;
            // slope factors of the forward stencils k0 and k1
            const float f1 = slope_f(nbR(Rv) - Qv);   // from V(r+1)[J+1] - V(r)[J]
            const float f2 = slope_f(nbR(Qv) - Rv);   // from V(r)[J+1] - V(r+1)[J]
            float gs[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                gs[k] = __builtin_fmaf(w, ((gtX_m4[k] + gtX_m2[k]) + nbL(gtX_m3[k])) + nbR(gtX_m3[k]), gtX_m3[k]);
            // k0 (V(r)[J], V(r+1)[J+1], V(r+2)[J+2])   k2 (V(r+1)[J+1], V(r)[J], V(r-1)[J-1])
            // k1 (V(r+1)[J], V(r)[J+1], V(r-1)[J+2])   k3 (V(r)[J+1], V(r+1)[J], V(r+2)[J-1])
            float d0, d1, d0c, d0b, a0, a1, a1c, a1b;
            line_adj(gpX_m3[0], gs[0], dd1s_r1, gpX_m3[2], gs[2], dd1_r, f1, d0, d1, d0c, d0b);   // main diagonal
            line_adj(gpX_m3[1], gs[1], dd2s_r, gpX_m3[3], gs[3], dd2_r1, f2, a0, a1, a1c, a1b);   // anti-diagonal
            // dL/dV row s-4 takes a1c from column J-2 now and d0c from
            // column J-2 three steps ago (kept in dcV_m3): one double shift
            accV_m4 += nbR(d0b) + nbL(nbL(a1c + dcV_m3));
            accV_m3 += d0 + nbL(a1);
            accV_m2 += a0 + nbL(d1);
            accV_m1 += nbR(a1b);
            dcV_0 = d0c;
        }

        // ======================= dL/dV row s-4 is complete =======================
        if constexpr (P1) {
            const int r = s - 4;
            float val = accV_m4 + gVu;
            // clamped columns: padded columns -4..-1 fold onto column 0, W..W+4 onto W-1
            if (first_strip) {
                float p = J < 0 ? val : 0.0f, acc = -0.0f;
#pragma unroll
                for (int k = 0; k < 4; ++k) { p = nbL(p); acc += p; }
                if (J == 0) val += acc;
            }
            if (last_strip) {
                float q = J >= W ? val : 0.0f, acc = -0.0f;
#pragma unroll
                for (int k = 0; k < 5; ++k) { q = nbR(q); acc += q; }
                if (J == W - 1) val += acc;
            }
            // clamped rows: rows -4..-1 fold onto row 0, rows H..H+4 onto row
            // H-1; interior steps store rows in [R0, R1) that fold nothing
            if constexpr (INTERIOR) {
                if (own) stG(r, val);
            } else if (top && r <= 0 && r < H - 1) {
                if (r < 0) {
                    if (r >= -4) fold_top += val;   // padded rows -4..-1; earlier rows are pipeline fill
                } else if (own) {
                    stG(0, val + fold_top);
                }
            } else if (bottom && r >= H - 1) {
                held += (r == H - 1 && top && H == 1) ? val + fold_top : val;
            } else if (r >= R0 && r < R1) {
                if (own) stG(r, val);
            }
        }
        }   // FULL

        // ======================= slide the windows =======================
        Vm3 = Vm2; Vm2 = Vm1; Vm1 = V0;
        V0 = V1; V1 = V2; V2 = V3; V3 = V4; V4 = V5;
        dd1_3 = dd1_4; dd2s_3 = dd2s_4;
        X0 = X1; X1 = X2; ddXv0 = ddXv1; ddr0 = ddr1;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            SX1[k] = SX2[k]; SX2[k] = SX3[k]; PX2[k] = PX3[k];
            SB0[k] = SB1[k]; PB0[k] = PB1[k]; hB0[k] = hB1[k]; hAm1[k] = hA0[k];
            gtA_m1[k] = gtA[k]; gpA_m1[k] = gpA[k]; qA_m1[k] = qA[k]; qB_m1[k] = qB[k];
            gtX_m4[k] = gtX_m3[k]; gtX_m3[k] = gtX_m2[k]; gpX_m3[k] = gpX_m2[k];
        }
        geoB_fv = nB_fv; geoB_ddd = nB_ddd; geoB_ddu = nB_ddu; geoB_fh = nB_fh; geoB_ddr = nB_ddr; geoB_ddl = nB_ddl;
        geoA_fv = nA_fv; geoA_ddd = nA_ddd; geoA_ddu = nA_ddu; geoA_fh = nA_fh; geoA_ddr = nA_ddr; geoA_ddl = nA_ddl;
        accX_m2 = accX_m1; accX_m1 = accX_0; accX_0 = accX_p1;
        accV_m4 = accV_m3; accV_m3 = accV_m2; accV_m2 = accV_m1; accV_m1 = accV_0; accV_0 = accV_p1;
        dcV_m3 = dcV_m2; dcV_m2 = dcV_m1; dcV_m1 = dcV_0;
    };
    using Full = std::integral_constant<int, 0>;
    using No = std::integral_constant<int, 0>;        // no phase-1 adjoint, no output
    using P1All = std::integral_constant<int, 1>;     // phase-1 adjoint, output with the edge folds
    using P1In = std::integral_constant<int, 2>;      // phase-1 adjoint, interior output row
    using K0 = std::integral_constant<int, 0>;
    using K1 = std::integral_constant<int, 1>;
    using K2 = std::integral_constant<int, 2>;
    using K3 = std::integral_constant<int, 3>;
    static_assert(kBwdForwardOnly == 9, "the forward-only iterations are D = -9 .. -1");
    // Interior steps [s_in0, s_in1) store a row of [R0, R1) that takes no
    // fold (rows 1.. of the top strip, up to H-2 in the bottom one); the
    // steps around them run the output with the edge folds.  The rings'
    // slots count from s_in0, fixed before the first step writes them.
    const int s_in0 = min(top ? 5 : R0 + 4, s_end + 1);
    const int s_in1 = max(s_in0, min(bottom ? H + 3 : R1 + 4, s_end + 1));
    s_ref = s_in0;
    {
        const int s0 = s;
        auto fwd_only = [&](auto dconst) {
            constexpr int D = decltype(dconst)::value;
            if (s0 + 9 + D <= s_end) step(s0 + 9 + D, dconst, No{}, 0);
        };
        fwd_only(std::integral_constant<int, -9>{});
        fwd_only(std::integral_constant<int, -8>{});
        fwd_only(std::integral_constant<int, -7>{});
        fwd_only(std::integral_constant<int, -6>{});
        fwd_only(std::integral_constant<int, -5>{});
        fwd_only(std::integral_constant<int, -4>{});
        fwd_only(std::integral_constant<int, -3>{});
        fwd_only(std::integral_constant<int, -2>{});
        fwd_only(std::integral_constant<int, -1>{});
        s = min(s0 + kBwdForwardOnly, s_end + 1);
    }
    nA = ldG(2 * s + 1, gyoffA);   // + point seeds of row s
    nB = ldG(2 * s, gyoffB);
    nX = ldG(2 * s - 3, gyoffB);   // x row s-2
    nV = ldG(2 * s - 8, gyoffA);   // V row s-4
    // The phase-1 adjoint of iteration s feeds dL/dV rows s-4 .. s-1, and its
    // output stores row s-4: until s = R0 + 1 (the top strip: s = -3, for the
    // folded rows -4 .. -1) both reach only rows this strip never stores, so
    // those iterations (the 6 after the forward-only ones) skip them.
    const int s_p1 = min(top ? -3 : R0 + 1, s_end + 1);
    for (; s + 1 < s_p1; s += 2) {
        step(s, Full{}, No{}, 0);
        step(s + 1, Full{}, No{}, 0);
    }
    if (s < s_p1) step(s++, Full{}, No{}, 0);
    for (; s < s_in0; ++s) step(s, Full{}, P1All{}, 0);
    // four rows per trip so that values carried up to four rows are renamed
    // rather than copied
    const int q1 = s + (s_end - s) / 4, q2 = s + (s_end - s) / 2, q3 = s + 3 * (s_end - s) / 4;
    for (; s + 3 < s_in1; s += 4) {
        if (s >= q3) __builtin_amdgcn_s_setprio(0);
        else if (s >= q2) __builtin_amdgcn_s_setprio(1);
        else if (s >= q1) __builtin_amdgcn_s_setprio(2);
        else __builtin_amdgcn_s_setprio(3);
        step(s, Full{}, P1In{}, K0{});
        step(s + 1, Full{}, P1In{}, K1{});
        step(s + 2, Full{}, P1In{}, K2{});
        step(s + 3, Full{}, P1In{}, K3{});
        bwd_f32x2* const t = dd_lo;
        dd_lo = dd_hi;
        dd_hi = t;
    }
    for (; s < s_in1; ++s) step(s, Full{}, P1In{}, 0);
    for (; s <= s_end; ++s) step(s, Full{}, P1All{}, 0);
    if (bottom) {
        const int r = H - 1;
        if (r >= R0 && own) stG(r, held);
    }
}

}  // namespace wz
