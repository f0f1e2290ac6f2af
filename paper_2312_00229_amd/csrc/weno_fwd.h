// Forward WD-WENO 2x kernel body for gfx950 (CDNA4, wave64).
//
// Method: arXiv 2312.00229, Section 3 -- phase 1 (x points, diagonal
// candidates, eqs. Vektor, p, 2Dsmoothness, 2DsmoothnessFinal, alpha,
// IzrazOmega2d, 2dKombinacija) and phase 2 (+ points, axis candidates,
// eqs. tezine, IzrazOmega2dRavno, 2dKombinacijaRavno), fused per output quad.
//
// Work decomposition ("strip walk"): one wave owns a strip of 64*COLS
// consecutive input columns and walks down `rows` input rows.  Lane l holds
// columns Jbase + l*COLS + c (c < COLS); left/right neighbours come from the
// adjacent lane through wave-wide DPP shifts, which the compiler folds into
// the consuming ALU op, so no LDS is needed.  Vertical neighbours live in
// register windows that slide one row per iteration.  The first 4 and the
// last 5..6 columns of a strip are halo (a quad reads columns J-4..J+5); the
// strip walk starts 9 rows above its first output row to fill the pipeline.
//
// Per iteration R (output quad row R) the stages are, in dependency order:
//   load   consume V(R+5) from the two-row prefetch queue, request V(R+7)
//   dd     diagonal second differences at input row R+4
//   sx     phase-1 candidates p and indicators SI of x points at row R+3
//   x      D = SI + w * (4 neighbours) and the blend for x points at row R+2
//   p2     phase-2 candidates/indicators of the + points B(R+1,.) and A(R,.)
//   blend  A(R,.), B(R,.), then the 2x2 quad store of row R.
//
// Arithmetic (all FP32): for a stencil (a, b, c) on nodes -1, 1, 3 the
// candidate is (a+b)/2 - dd/8 with dd = a - 2b + c, and the indicator
// (b-a)^2 + 13/12 dd^2.  The doubling keeps two scaled copies of every sample
// (input rows and x points): h = v/2 and s = kappa v with kappa^2 = 13/48.
// Then (a+b)/2 = h_a + h_b, g = h_b - h_a = (b-a)/2, dds = s_a - 2 s_b + s_c
// = kappa dd, and the kernel carries SI/4 = g^2 + dds^2: neither the 1/2 of
// the mean nor the 13/12 of the indicator costs an instruction.  The common
// factor 1/4 cancels in the normalised weights; eps is folded into every SI/4
// as eps_q = eps / (4 (1 + 4w)), so SI/4_self + w * sum SI/4_nbr = (D + eps)/4.
// (The adjoint carries SI* = (3/13) SI instead, with eps_hat = eps*3/13 /
// (1 + 4w), so that SI*_self + w * sum SI*_nbr = (3/13)(D + eps).)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace wz {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kXcds = 8;  // MI355X: accelerator complex dies, one L2 each

// beta specialisations
constexpr int kBetaGeneral = -1;

// I/O modes of the strip walk.  The two common layouts are fixed at compile
// time so that every row issues the same memory operations, with no branch:
// the compiler can then keep prefetched rows in flight across iterations.
constexpr int kIoGeneric = 0;  // any dtype pair, strides and output scale (runtime flags)
constexpr int kIoF32 = 1;      // f32 -> f32, destination columns contiguous and vector-aligned
constexpr int kIoU8 = 2;       // u8 -> u8, any strides
constexpr int kIoU8F32 = 3;    // u8 -> f32 (x 1/255), destination as for kIoF32
constexpr int kIoF32U8 = 4;    // f32 -> u8 (x 255), any strides
constexpr bool io_in_u8(int io) { return io == kIoU8 || io == kIoU8F32; }
constexpr bool io_out_u8(int io) { return io == kIoU8 || io == kIoF32U8; }
// the output scale is 1 when both ends have the same dtype
constexpr bool io_scaled(int io) { return io == kIoU8F32 || io == kIoF32U8; }

// A buffer offset past every plane extent (planes span less than 2^31 bytes):
// loads through it return 0 and stores through it are dropped by the buffer
// unit's range check, with no memory access.  Row offsets added to it stay
// below 2^32, so the sum cannot wrap back into range.
constexpr uint32_t kOob = 0x80000000u;

struct FwdParams {
    float eps_hat;  // adjoint: eps*3/13 / (1 + 4w), in the kernel's value scale
    float eps_q;    // doubling: eps / (4 (1 + 4w)), in the kernel's value scale
    float w;        // neighbour-indicator weight
    float beta;     // used by the general-beta path
    float out_scale;  // output value = u * out_scale before quantisation
};

// One image (all of its planes) for the forward kernels.
struct FwdJob {
    const uint8_t* src;  // byte pointer to element 0
    uint8_t* dst;
    int32_t H, W, C, planes;          // planes = N * C
    int64_t s_n, s_c, s_h, s_w;       // byte strides of the source
    int64_t d_n, d_c, d_h, d_w;       // byte strides of the destination
    int32_t in_u8, out_u8;            // element types
    int32_t strips_x, strips_y;       // strips per plane (two-column strips only when tail_rows > 0)
    // tail_rows > 0: the columns left of the last two-column strip are
    // walked by one-column strips of tail_rows rows, tail_bands of them per
    // plane (single-image planar launches; zoom2x_kernel)
    int32_t tail_rows, tail_bands;
    int32_t vec;                      // 2: float4 rows, 1: float2 rows, 0: scalar stores
    uint32_t src_extent, dst_extent;  // bytes spanned by one plane (< 2^31)
    int32_t io;                       // I/O mode (kIo*)
    // readable source region: src points at its element (0, 0), which is
    // image element (-src_shift, -src_shift); reads clamp to src_h x src_w
    // (clamp-to-edge: shift 0 and the image; caller ghost samples: shift 4
    // and (H + 9) x (W + 9))
    int32_t src_shift, src_h, src_w;
};

__device__ __forceinline__ float from_left(float x)
{   // lane i receives lane i-1 (wave_shr:1); lane 0 receives 0
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float from_right(float x)
{   // lane i receives lane i+1 (wave_shl:1); lane 63 receives 0
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xF, 0xF, true));
}

// value of column (c - 1) / (c + 1) of a per-lane column array
template <int COLS>
__device__ __forceinline__ float lft(const float (&x)[COLS], int c)
{
    return c > 0 ? x[c - 1] : from_left(x[COLS - 1]);
}
template <int COLS>
__device__ __forceinline__ float rgt(const float (&x)[COLS], int c)
{
    return c < COLS - 1 ? x[c + 1] : from_right(x[0]);
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// alpha_k = 0.5 / t_k^beta (the 0.5 cancels), u = sum alpha_k p_k / sum alpha_k
template <int BETA>
__device__ __forceinline__ float blend4(float t0, float t1, float t2, float t3,
                                        float p0, float p1, float p2, float p3, float beta)
{
    float a0, a1, a2, a3;
    if constexpr (BETA == 2) {
        float r0 = rcp(t0), r1 = rcp(t1), r2 = rcp(t2), r3 = rcp(t3);
        a0 = r0 * r0; a1 = r1 * r1; a2 = r2 * r2; a3 = r3 * r3;
    } else if constexpr (BETA == 1) {
        a0 = rcp(t0); a1 = rcp(t1); a2 = rcp(t2); a3 = rcp(t3);
    } else {
        a0 = __builtin_amdgcn_exp2f(-beta * __builtin_amdgcn_logf(t0));
        a1 = __builtin_amdgcn_exp2f(-beta * __builtin_amdgcn_logf(t1));
        a2 = __builtin_amdgcn_exp2f(-beta * __builtin_amdgcn_logf(t2));
        a3 = __builtin_amdgcn_exp2f(-beta * __builtin_amdgcn_logf(t3));
    }
    float S = (a0 + a1) + (a2 + a3);
    float N = __builtin_fmaf(a3, p3, __builtin_fmaf(a2, p2, __builtin_fmaf(a1, p1, a0 * p0)));
    return N * rcp(S);
}

// scaled indicator: a second difference squared plus the slope term gc
__device__ __forceinline__ float sidx(float dd, float gc) { return __builtin_fmaf(dd, dd, gc); }

// The doubling's scaled copies (see the header comment): h = v/2, s = kappa v
constexpr float kKappa = 0.52041649986653320f;    // sqrt(13/48)
constexpr float kCandS = -0.24019223070763074f;   // -1 / (8 kappa): dd/8 from dds
__device__ __forceinline__ float half_of(float v) { return 0.5f * v; }
__device__ __forceinline__ float kappa_of(float v) { return kKappa * v; }
// candidate m - dd/8 from dds = kappa dd
__device__ __forceinline__ float cand_s(float dds, float m) { return __builtin_fmaf(dds, kCandS, m); }
// g^2 + eps_q from g = (b - a)/2
__device__ __forceinline__ float gterm_q(float g, float eps_q) { return __builtin_fmaf(g, g, eps_q); }
// a - 2b + c
__device__ __forceinline__ float d2(float a, float b, float c) { return __builtin_fmaf(-2.0f, b, a + c); }

template <int COLS>
struct StripState {
    // input rows R .. R+4 (row R+5 is loaded by the iteration): the samples
    // (stored as the quads' originals) and their copies h = v/2, s = kappa v
    float V0[COLS], V1[COLS], V2[COLS], V3[COLS], V4[COLS];
    float H0[COLS], H1[COLS], H2[COLS], H3[COLS], H4[COLS];
    float S0[COLS], S1[COLS], S2[COLS], S3[COLS], S4[COLS];
    // main-diagonal second difference centred at (R+3, J); anti-diagonal at (R+3, J+1)
    float dd1_3[COLS], dd2s_3[COLS];
    // phase-1 scaled indicators at x rows R+1, R+2 and candidates at x row R+2
    float SX1[4][COLS], SX2[4][COLS], PX2[4][COLS];
    // x values at rows R, R+1 and their copies x/2, kappa x
    float X0[COLS], X1[COLS], XH0[COLS], XH1[COLS], XS0[COLS], XS1[COLS];
    // vertical second differences centred at row R: of x (X(R-1)-2X(R)+X(R+1)) and of V
    float ddXv0[COLS], ddr0[COLS];
    // phase-2: B(R) indicators/candidates, B pair sums at row R, A pair sums at row R-1
    float SB0[4][COLS], PB0[4][COLS], hB0[4][COLS], hAm1[4][COLS];
};

// Per-lane geometry of a strip, fixed for the whole walk.
template <int COLS>
struct StripLanes {
    uint32_t src_off[COLS];  // source column byte offsets (columns clamped to the image)
    int J[COLS];             // input column of each of the lane's columns
    bool own[COLS];          // column stored by this strip
    bool own_all;
    uint32_t st_col[COLS];   // kIoU8: destination column offsets, kOob where not owned
    uint32_t st_vec;         // kIoF32: offset of the lane's vector store, kOob unless all its columns are owned
    uint32_t st_half;        // kIoF32, two columns: offset of a 2-float store when only column 0 is owned, else kOob
    bool any_half;           // some lane of the strip needs st_half (odd width, last strip); uniform
};

// Buffer resources (gfx9 family descriptor, raw addressing): the plane base
// and its byte extent sit in SGPRs, the per-lane column offset in a VGPR and
// the uniform row offset in an SGPR, so loads and stores need no VALU address
// arithmetic.  Offsets are 32-bit: the host rejects planes spanning 2^31 bytes
// or more.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRsrcWord3);
}
__device__ __forceinline__ float buf_ld_f32(rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void buf_st_f32(float v, rsrc_t r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, 0);
}
// Cache policy of the vector stores of whole output rows in a launch of one
// round of waves: device scope (the SC1 bit), so the line is written through
// this XCD's L2 rather than held dirty in it.  The output is written once and
// never read back by the launch; held dirty, it is written back only when the
// launch ends, where every XCD's L2 is flushed before a dependent launch may
// start, and that flush of up to 4 MB per XCD is time the launch adds after
// its last wave (1080p RGB float32: 38.7 -> 36.4 us).  Longer launches keep
// the default write-back policy: there the flush is a small part of the
// launch, and a store written through completes later, which delays the
// waits of the loads issued after it (3x4320x7680: 0.524 -> 0.544 ms
// written through).  Byte stores always keep it: their lines are filled in
// pieces by several waves, and writing every piece through costs far more
// than the flush (uint8 HWC 1080p: 69.7 against 43.5 us).
constexpr int kStRows = 16;

template <int POLICY = 0>
__device__ __forceinline__ void buf_st_f32x2(float a, float b, rsrc_t r, uint32_t voff, uint32_t soff)
{
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    u32x2 v = {__builtin_bit_cast(uint32_t, a), __builtin_bit_cast(uint32_t, b)};
    __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)voff, (int)soff, POLICY);
}
template <int POLICY = 0>
__device__ __forceinline__ void buf_st_f32x4(float a, float b, float c, float d, rsrc_t r, uint32_t voff,
                                             uint32_t soff)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 v = {__builtin_bit_cast(uint32_t, a), __builtin_bit_cast(uint32_t, b), __builtin_bit_cast(uint32_t, c),
               __builtin_bit_cast(uint32_t, d)};
    __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)voff, (int)soff, POLICY);
}
__device__ __forceinline__ void buf_st_u8(uint32_t v, rsrc_t r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b8((uint8_t)v, r, (int)voff, (int)soff, 0);
}

struct StripCtx {
    rsrc_t src, dst;          // one plane each
    uint32_t s_h, d_h, d_w;   // byte strides: source rows, destination rows, destination columns
    uint32_t s_w_bytes;       // source column stride
    int32_t H, W;
    int32_t src_shift, src_h, src_w;   // readable source region (FwdJob)
    int32_t in_u8, out_u8, vec;
    float out_scale;
};

// Raw load of input row r (clamped) into a queue slot: f32 bits or a
// zero-extended byte.  The conversion to float happens when the row is
// consumed, two iterations later, so no wait follows the load.
// queue word of an I/O mode: the u8 mode keeps the loaded byte as a byte, so
// that its widening folds into the conversion at the consuming iteration
template <int IO>
using raw_t = typename std::conditional<io_in_u8(IO), uint8_t, uint32_t>::type;

template <int COLS, int IO>
__device__ __forceinline__ void load_row_raw(const StripCtx& cx, const uint32_t (&off)[COLS], int r, raw_t<IO> (&q)[COLS])
{
    const int rs = r + cx.src_shift;
    const int rc = rs < 0 ? 0 : (rs >= cx.src_h ? cx.src_h - 1 : rs);
    const uint32_t soff = (uint32_t)rc * cx.s_h;
    const bool u8 = io_in_u8(IO) || (IO == kIoGeneric && cx.in_u8);
    if (u8) {
#pragma unroll
        for (int c = 0; c < COLS; ++c) q[c] = __builtin_amdgcn_raw_buffer_load_b8(cx.src, (int)off[c], (int)soff, 0);
    } else {
#pragma unroll
        for (int c = 0; c < COLS; ++c) q[c] = __builtin_amdgcn_raw_buffer_load_b32(cx.src, (int)off[c], (int)soff, 0);
    }
}

template <int IO>
__device__ __forceinline__ float raw_value(const StripCtx& cx, raw_t<IO> q)
{
    if constexpr (io_in_u8(IO)) return (float)q;
    else if constexpr (IO != kIoGeneric) {
        // an explicit copy into a register of its own: the slot's register is
        // then free for the row loaded next, so it stays the loop-carried
        // register and is not copied (waiting for that load) at the back edge
        float v;
        asm("v_mov_b32 %0, %1" : "=&v"(v) : "v"(q));
        return v;
    }
    else return cx.in_u8 ? (float)q : __builtin_bit_cast(float, q);
}

// clamp(round-half-even(u), 0, 255), NaN -> 0, in one instruction:
// v_cvt_pk_u8_f32 rounds to nearest even and saturates (checked on the part
// against that definition on every k + 1/2 tie in [-3, 258], both
// neighbouring floats of each, 2e4 values in [-10, 270], +-0, +-inf, +-1e30
// and NaN)
__device__ __forceinline__ uint32_t quant_u8(float u) { return __builtin_amdgcn_cvt_pk_u8_f32(u, 0u, 0u); }

// store the 2x2 quads of row R for this lane's columns: fixed layouts,
// branch-free (lanes that own nothing store through kOob).  Mixed dtypes
// scale by out_scale (255 or 1/255), as the runtime-flag path does.
template <int COLS, int IO, int ST>
__device__ __forceinline__ void store_quads_fixed(const StripCtx& cx, int R, const StripLanes<COLS>& L,
                                                  const float (&o00)[COLS], const float (&o01)[COLS],
                                                  const float (&o10)[COLS], const float (&o11)[COLS])
{
    const uint32_t r0 = (uint32_t)(2 * R) * cx.d_h;
    const uint32_t r1 = r0 + cx.d_h;
    float a[COLS], b[COLS], c[COLS], d[COLS];
#pragma unroll
    for (int k = 0; k < COLS; ++k) {
        if constexpr (io_scaled(IO)) {
            const float s = cx.out_scale;
            a[k] = o00[k] * s; b[k] = o01[k] * s; c[k] = o10[k] * s; d[k] = o11[k] * s;
        } else {
            a[k] = o00[k]; b[k] = o01[k]; c[k] = o10[k]; d[k] = o11[k];
        }
    }
    if constexpr (!io_out_u8(IO)) {
        if constexpr (COLS == 2) {
            buf_st_f32x4<ST>(a[0], b[0], a[1], b[1], cx.dst, L.st_vec, r0);
            buf_st_f32x4<ST>(c[0], d[0], c[1], d[1], cx.dst, L.st_vec, r1);
            if (L.any_half) {
                buf_st_f32x2<ST>(a[0], b[0], cx.dst, L.st_half, r0);
                buf_st_f32x2<ST>(c[0], d[0], cx.dst, L.st_half, r1);
            }
        } else {
            buf_st_f32x2<ST>(a[0], b[0], cx.dst, L.st_vec, r0);
            buf_st_f32x2<ST>(c[0], d[0], cx.dst, L.st_vec, r1);
        }
    } else {  // one byte per output
#pragma unroll
        for (int k = 0; k < COLS; ++k) {
            const uint32_t off0 = L.st_col[k];
            buf_st_u8(quant_u8(a[k]), cx.dst, off0, r0);
            buf_st_u8(quant_u8(b[k]), cx.dst, off0 + cx.d_w, r0);
            buf_st_u8(quant_u8(c[k]), cx.dst, off0, r1);
            buf_st_u8(quant_u8(d[k]), cx.dst, off0 + cx.d_w, r1);
        }
    }
}

// store the 2x2 quads of row R for this lane's columns (any layout)
template <int COLS, int ST>
__device__ __forceinline__ void store_quads(const StripCtx& cx, int R, const int (&J)[COLS], bool own_all,
                                            const bool (&own)[COLS], const float (&o00)[COLS],
                                            const float (&o01)[COLS], const float (&o10)[COLS],
                                            const float (&o11)[COLS])
{
    const uint32_t r0 = (uint32_t)(2 * R) * cx.d_h;
    const uint32_t r1 = r0 + cx.d_h;
    if (!cx.out_u8 && cx.out_scale == 1.0f && COLS == 2 && cx.vec == 2 && own_all) {
        // same dtype in and out: no rescaling
        const uint32_t off = (uint32_t)(2 * J[0]) * 4u;
        buf_st_f32x4<ST>(o00[0], o01[0], o00[COLS - 1], o01[COLS - 1], cx.dst, off, r0);
        buf_st_f32x4<ST>(o10[0], o11[0], o10[COLS - 1], o11[COLS - 1], cx.dst, off, r1);
    } else if (!cx.out_u8) {
        const float s = cx.out_scale;
        if (COLS == 2 && cx.vec == 2 && own_all) {
            const uint32_t off = (uint32_t)(2 * J[0]) * 4u;
            buf_st_f32x4<ST>(o00[0] * s, o01[0] * s, o00[COLS - 1] * s, o01[COLS - 1] * s, cx.dst, off, r0);
            buf_st_f32x4<ST>(o10[0] * s, o11[0] * s, o10[COLS - 1] * s, o11[COLS - 1] * s, cx.dst, off, r1);
        } else if (cx.vec >= 1) {
#pragma unroll
            for (int c = 0; c < COLS; ++c) {
                if (!own[c]) continue;
                const uint32_t off = (uint32_t)(2 * J[c]) * 4u;
                buf_st_f32x2(o00[c] * s, o01[c] * s, cx.dst, off, r0);
                buf_st_f32x2(o10[c] * s, o11[c] * s, cx.dst, off, r1);
            }
        } else {
#pragma unroll
            for (int c = 0; c < COLS; ++c) {
                if (!own[c]) continue;
                const uint32_t off0 = (uint32_t)(2 * J[c]) * cx.d_w;
                buf_st_f32(o00[c] * s, cx.dst, off0, r0);
                buf_st_f32(o01[c] * s, cx.dst, off0 + cx.d_w, r0);
                buf_st_f32(o10[c] * s, cx.dst, off0, r1);
                buf_st_f32(o11[c] * s, cx.dst, off0 + cx.d_w, r1);
            }
        }
    } else {
        const float s = cx.out_scale;
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            if (!own[c]) continue;
            const uint32_t off0 = (uint32_t)(2 * J[c]) * cx.d_w;
            buf_st_u8(quant_u8(o00[c] * s), cx.dst, off0, r0);
            buf_st_u8(quant_u8(o01[c] * s), cx.dst, off0 + cx.d_w, r0);
            buf_st_u8(quant_u8(o10[c] * s), cx.dst, off0, r1);
            buf_st_u8(quant_u8(o11[c] * s), cx.dst, off0 + cx.d_w, r1);
        }
    }
}

// One strip-walk iteration.  D = 0: main loop (every stage runs, quad row R
// is stored); D < 0: prologue iteration R = R0 + D, where each stage only
// runs once its results can feed an output row >= R0.  Q is the queue slot
// holding input row R+5 (loaded two iterations earlier); it is refilled with
// row R+7.  ST: cache policy of the row stores.
template <int COLS, int BETA, int IO, int D, int ST = 0>
__device__ __forceinline__ void strip_step(StripState<COLS>& s, raw_t<IO> (&Q)[COLS], const StripCtx& cx,
                                           const FwdParams& P, const StripLanes<COLS>& L, int R)
{
    constexpr bool FULL = D == 0;
    constexpr bool do_dd = FULL || D >= -7;
    constexpr bool do_sx = FULL || D >= -6;
    constexpr bool do_x = FULL || D >= -4;
    constexpr bool do_p2dd = FULL || D >= -2;
    constexpr bool do_p2 = FULL || D >= -1;
    const float eq = P.eps_q, w = P.w;

    float V5[COLS], H5[COLS], S5[COLS];
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        V5[c] = raw_value<IO>(cx, Q[c]);
        H5[c] = half_of(V5[c]);
        S5[c] = kappa_of(V5[c]);
    }
    load_row_raw<COLS, IO>(cx, L.src_off, R + 7, Q);

    // ---- dd: diagonal second differences (times kappa) centred at (R+4, J) ----
    float dd1_4[COLS] = {}, dd2_4[COLS] = {}, dd1s_4[COLS] = {}, dd2s_4[COLS] = {};
    if constexpr (do_dd) {
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            dd1_4[c] = d2(lft(s.S3, c), s.S4[c], rgt(S5, c));  // (R+3,J-1) (R+4,J) (R+5,J+1)
            dd2_4[c] = d2(rgt(s.S3, c), s.S4[c], lft(S5, c));  // (R+3,J+1) (R+4,J) (R+5,J-1)
        }
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            dd1s_4[c] = rgt(dd1_4, c);
            dd2s_4[c] = rgt(dd2_4, c);
        }
    }

    // ---- sx: phase-1 candidates and indicators of X(R+3, J) ----
    // X(R+3,J) sits at (R+3.5, J+0.5).  Main diagonal line through V(R+3,J),
    // V(R+4,J+1): k0 steps (+1,+1) (dd centred at (R+4,J+1)), k2 steps (-1,-1)
    // (dd centred at (R+3,J)).  Anti-diagonal line through V(R+3,J+1), V(R+4,J):
    // k1 steps (-1,+1) (dd centred at (R+3,J+1)), k3 steps (+1,-1) (dd at (R+4,J)).
    float SX3[4][COLS] = {}, PX3[4][COLS] = {};
    if constexpr (do_sx) {
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            const float a1 = s.H3[c], b1 = rgt(s.H4, c);
            const float a2 = rgt(s.H3, c), b2 = s.H4[c];
            const float gc1 = gterm_q(b1 - a1, eq), gc2 = gterm_q(b2 - a2, eq);
            const float m1 = a1 + b1, m2 = a2 + b2;
            SX3[0][c] = sidx(dd1s_4[c], gc1);   PX3[0][c] = cand_s(dd1s_4[c], m1);
            SX3[2][c] = sidx(s.dd1_3[c], gc1);  PX3[2][c] = cand_s(s.dd1_3[c], m1);
            SX3[1][c] = sidx(s.dd2s_3[c], gc2); PX3[1][c] = cand_s(s.dd2s_3[c], m2);
            SX3[3][c] = sidx(dd2_4[c], gc2);    PX3[3][c] = cand_s(dd2_4[c], m2);
        }
    }

    // ---- x: D over the four same-direction neighbours (I+-1, J), (I, J+-1); blend X(R+2, J) ----
    float X2[COLS] = {}, XH2[COLS] = {}, XS2[COLS] = {};
    if constexpr (do_x) {
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            float t[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                // one neighbour shift per addition, so that with one column per
                // lane each shift folds into its addition as a DPP operand
                float ns = ((s.SX1[k][c] + SX3[k][c]) + lft(s.SX2[k], c)) + rgt(s.SX2[k], c);
                t[k] = __builtin_fmaf(w, ns, s.SX2[k][c]);
            }
            X2[c] = blend4<BETA>(t[0], t[1], t[2], t[3], s.PX2[0][c], s.PX2[1][c], s.PX2[2][c], s.PX2[3][c], P.beta);
            XH2[c] = half_of(X2[c]);
            XS2[c] = kappa_of(X2[c]);
        }
    }

    // ---- vertical second differences centred at row R+1 ----
    float ddXv1[COLS] = {}, ddr1[COLS] = {};
    if constexpr (do_p2dd) {
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            ddXv1[c] = d2(s.XS0[c], s.XS1[c], XS2[c]);
            ddr1[c] = d2(s.S0[c], s.S1[c], s.S2[c]);
        }
    }

    // ---- p2: + points.  Directions k0 (+1,0) down, k1 (0,+1) right, k2 up, k3 left ----
    float SB1[4][COLS] = {}, PB1[4][COLS] = {}, hB1[4][COLS] = {};
    float SA0[4][COLS] = {}, PA0[4][COLS] = {}, hA0[4][COLS] = {};
    if constexpr (do_p2) {
        float h1r[COLS], ddc[COLS], xh0l[COLS], ddXh[COLS];
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            h1r[c] = rgt(s.H1, c);
            ddc[c] = d2(lft(s.S1, c), s.S1[c], rgt(s.S1, c));      // V row R+1, centred at J
            xh0l[c] = lft(s.XH0, c);
            ddXh[c] = d2(lft(s.XS0, c), s.XS0[c], rgt(s.XS0, c));  // X row R, centred at J
        }
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            // B(R+1, J) at (R+1, J+1/2).  Vertical line through X(R,J), X(R+1,J):
            const float gcv = gterm_q(s.XH1[c] - s.XH0[c], eq), mv = s.XH0[c] + s.XH1[c];
            SB1[0][c] = sidx(ddXv1[c], gcv);   PB1[0][c] = cand_s(ddXv1[c], mv);    // X(R), X(R+1), X(R+2)
            SB1[2][c] = sidx(s.ddXv0[c], gcv); PB1[2][c] = cand_s(s.ddXv0[c], mv);  // X(R+1), X(R), X(R-1)
            // horizontal line through V(R+1,J), V(R+1,J+1)
            const float gch = gterm_q(h1r[c] - s.H1[c], eq), mh = s.H1[c] + h1r[c];
            const float ddcs = rgt(ddc, c);                                          // centred at J+1
            SB1[1][c] = sidx(ddcs, gch);       PB1[1][c] = cand_s(ddcs, mh);        // V(R+1,J..J+2)
            SB1[3][c] = sidx(ddc[c], gch);     PB1[3][c] = cand_s(ddc[c], mh);      // V(R+1,J+1..J-1)

            // A(R, J) at (R+1/2, J).  Vertical line through V(R,J), V(R+1,J):
            const float gav = gterm_q(s.H1[c] - s.H0[c], eq), mav = s.H0[c] + s.H1[c];
            SA0[0][c] = sidx(ddr1[c], gav);    PA0[0][c] = cand_s(ddr1[c], mav);    // V(R), V(R+1), V(R+2)
            SA0[2][c] = sidx(s.ddr0[c], gav);  PA0[2][c] = cand_s(s.ddr0[c], mav);  // V(R+1), V(R), V(R-1)
            // horizontal line through X(R,J-1), X(R,J)
            const float gah = gterm_q(s.XH0[c] - xh0l[c], eq), mah = xh0l[c] + s.XH0[c];
            const float ddXhl = lft(ddXh, c);                                        // centred at J-1
            SA0[1][c] = sidx(ddXh[c], gah);    PA0[1][c] = cand_s(ddXh[c], mah);    // X(R,J-1..J+1)
            SA0[3][c] = sidx(ddXhl, gah);      PA0[3][c] = cand_s(ddXhl, mah);      // X(R,J..J-2)
        }
        // pair sums for the combined indicators of eq. (tezine):
        //   D_A(I,J) = SI_A(I,J) + w [SI_B(I,J-1) + SI_B(I,J) + SI_B(I+1,J-1) + SI_B(I+1,J)]
        //   D_B(I,J) = SI_B(I,J) + w [SI_A(I-1,J) + SI_A(I-1,J+1) + SI_A(I,J) + SI_A(I,J+1)]
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int c = 0; c < COLS; ++c) {
                hB1[k][c] = lft(SB1[k], c) + SB1[k][c];
                hA0[k][c] = SA0[k][c] + rgt(SA0[k], c);
            }
        }
    }

    // ---- blend A(R, .), B(R, .) and store quad row R ----
    if constexpr (FULL) {
        float Aq[COLS], Bq[COLS];
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            float ta[4], tb[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ta[k] = __builtin_fmaf(w, s.hB0[k][c] + hB1[k][c], SA0[k][c]);
                tb[k] = __builtin_fmaf(w, s.hAm1[k][c] + hA0[k][c], s.SB0[k][c]);
            }
            Aq[c] = blend4<BETA>(ta[0], ta[1], ta[2], ta[3], PA0[0][c], PA0[1][c], PA0[2][c], PA0[3][c], P.beta);
            Bq[c] = blend4<BETA>(tb[0], tb[1], tb[2], tb[3], s.PB0[0][c], s.PB0[1][c], s.PB0[2][c],
                                 s.PB0[3][c], P.beta);
        }
        if constexpr (IO == kIoGeneric) {
            store_quads<COLS, ST>(cx, R, L.J, L.own_all, L.own, s.V0, Bq, Aq, s.X0);
        } else if constexpr (io_out_u8(IO)) {
            // byte outputs are rounded anyway: the originals and x values are
            // rebuilt from their halves (exact for every normal float), so the
            // raw windows are dead and the kernel keeps three waves per SIMD
            float v0[COLS], x0[COLS];
#pragma unroll
            for (int c = 0; c < COLS; ++c) {
                v0[c] = s.H0[c] + s.H0[c];
                x0[c] = s.XH0[c] + s.XH0[c];
            }
            store_quads_fixed<COLS, IO, ST>(cx, R, L, v0, Bq, Aq, x0);
        } else {
            store_quads_fixed<COLS, IO, ST>(cx, R, L, s.V0, Bq, Aq, s.X0);
        }
    }

    // ---- slide the windows by one row ----
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        s.V0[c] = s.V1[c]; s.V1[c] = s.V2[c]; s.V2[c] = s.V3[c]; s.V3[c] = s.V4[c]; s.V4[c] = V5[c];
        s.H0[c] = s.H1[c]; s.H1[c] = s.H2[c]; s.H2[c] = s.H3[c]; s.H3[c] = s.H4[c]; s.H4[c] = H5[c];
        s.S0[c] = s.S1[c]; s.S1[c] = s.S2[c]; s.S2[c] = s.S3[c]; s.S3[c] = s.S4[c]; s.S4[c] = S5[c];
        s.dd1_3[c] = dd1_4[c]; s.dd2s_3[c] = dd2s_4[c];
        s.X0[c] = s.X1[c]; s.X1[c] = X2[c];
        s.XH0[c] = s.XH1[c]; s.XH1[c] = XH2[c];
        s.XS0[c] = s.XS1[c]; s.XS1[c] = XS2[c];
        s.ddXv0[c] = ddXv1[c]; s.ddr0[c] = ddr1[c];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            s.SX1[k][c] = s.SX2[k][c]; s.SX2[k][c] = SX3[k][c]; s.PX2[k][c] = PX3[k][c];
            s.SB0[k][c] = SB1[k][c]; s.PB0[k][c] = PB1[k][c]; s.hB0[k][c] = hB1[k][c];
            s.hAm1[k][c] = hA0[k][c];
        }
    }
}

// Input columns a strip of COLS quad columns per lane owns (stores): the
// 64*COLS it walks less a halo of 4 on the left and 5 or 6 on the right (a
// quad reads columns J-4 .. J+5); even for COLS = 2 (16-byte stores).
template <int COLS>
constexpr int strip_own() { return COLS == 1 ? kWave - 9 : 2 * kWave - 10; }

// Walk one strip: owned columns [c0, c0 + strip_own), output rows [R0, R1).
// PACED: the launch runs as one round of waves (every wave resident from the
// start): pace the waves that share a SIMD and write whole output rows
// through the L2.
template <int COLS, int BETA, int IO, bool PACED = false>
__device__ __forceinline__ void zoom_strip(const StripCtx& cx, const FwdParams& P, int c0, int R0, int R1)
{
    constexpr int ST = PACED ? kStRows : 0;
    constexpr int HALO_L = 4;
    constexpr int OWN = strip_own<COLS>();
    const int lane = threadIdx.x & (kWave - 1);
    const int Jbase = c0 - HALO_L;
    StripLanes<COLS> L;
    L.own_all = true;
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        const int sidx_ = lane * COLS + c;
        L.J[c] = Jbase + sidx_;
        L.own[c] = (sidx_ >= HALO_L) && (sidx_ < HALO_L + OWN) && (L.J[c] < cx.W);
        L.own_all = L.own_all && L.own[c];
        const int js = L.J[c] + cx.src_shift;
        const int jc = js < 0 ? 0 : (js >= cx.src_w ? cx.src_w - 1 : js);
        L.src_off[c] = (uint32_t)jc * cx.s_w_bytes;
        L.st_col[c] = L.own[c] ? (uint32_t)(2 * L.J[c]) * cx.d_w : kOob;
    }
    // f32 rows: the lane's 2*COLS floats of an output row are contiguous
    L.st_vec = L.own_all ? (uint32_t)(2 * L.J[0]) * 4u : kOob;
    // odd width: the lane holding column W-1 also holds W, past the image
    const bool half = COLS == 2 && L.own[0] && !L.own_all;
    L.st_half = half ? (uint32_t)(2 * L.J[0]) * 4u : kOob;
    L.any_half = COLS == 2 && (cx.W & 1) && cx.W - 1 >= Jbase + HALO_L && cx.W - 1 < Jbase + HALO_L + OWN;

    StripState<COLS> s;
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        s.V0[c] = s.V1[c] = s.V2[c] = s.V3[c] = s.V4[c] = 0.0f;
        s.H0[c] = s.H1[c] = s.H2[c] = s.H3[c] = s.H4[c] = 0.0f;
        s.S0[c] = s.S1[c] = s.S2[c] = s.S3[c] = s.S4[c] = 0.0f;
        s.dd1_3[c] = s.dd2s_3[c] = s.X0[c] = s.X1[c] = s.ddXv0[c] = s.ddr0[c] = 0.0f;
        s.XH0[c] = s.XH1[c] = s.XS0[c] = s.XS1[c] = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            // indicator windows start at 1 so that pipeline-fill blends never divide by zero
            s.SX1[k][c] = s.SX2[k][c] = 1.0f;
            s.PX2[k][c] = 0.0f;
            s.SB0[k][c] = s.hB0[k][c] = s.hAm1[k][c] = 1.0f;
            s.PB0[k][c] = 0.0f;
        }
    }

    // Pacing by wave priority.  In a launch of one round, two or three waves
    // share each SIMD from start to end, and among waves of equal priority the
    // SIMD issues for the oldest whenever it can: left alone, one wave of each
    // pair runs far ahead and finishes early, and the SIMD spends the end of
    // the launch on one latency-bound wave (1080p RGB: half the waves end at
    // 20 us, the rest at 35.7).  A paced wave steps its priority down from 3
    // to 0 as it passes each quarter of its rows, so the wave that has done
    // less goes first and the waves of a SIMD keep pace and end together.
    // Launches of several rounds are not paced: there, waves ending together
    // would leave the next round's waves to start, and run, alone.
    if constexpr (PACED) __builtin_amdgcn_s_setprio(3);

    // two queue slots used in turn, so that a row is read two iterations
    // after its load and a slot is never copied while its load is in flight
    raw_t<IO> QA[COLS], QB[COLS];
    load_row_raw<COLS, IO>(cx, L.src_off, R0 - 4, QA);
    load_row_raw<COLS, IO>(cx, L.src_off, R0 - 3, QB);
    // prologue: rows R0-9 .. R0-1 fill the pipeline (no stores)
    strip_step<COLS, BETA, IO, -9, ST>(s, QA, cx, P, L, R0 - 9);
    strip_step<COLS, BETA, IO, -8, ST>(s, QB, cx, P, L, R0 - 8);
    strip_step<COLS, BETA, IO, -7, ST>(s, QA, cx, P, L, R0 - 7);
    strip_step<COLS, BETA, IO, -6, ST>(s, QB, cx, P, L, R0 - 6);
    strip_step<COLS, BETA, IO, -5, ST>(s, QA, cx, P, L, R0 - 5);
    strip_step<COLS, BETA, IO, -4, ST>(s, QB, cx, P, L, R0 - 4);
    strip_step<COLS, BETA, IO, -3, ST>(s, QA, cx, P, L, R0 - 3);
    strip_step<COLS, BETA, IO, -2, ST>(s, QB, cx, P, L, R0 - 2);
    strip_step<COLS, BETA, IO, -1, ST>(s, QA, cx, P, L, R0 - 1);
    // Main walk, several rows per trip so that values carried from row to row
    // are renamed rather than copied: six rows (the input windows span six
    // rows and the x-point windows three, so all of them rotate by renaming
    // alone), two for the runtime-flag path and for the two-column byte-output
    // kernels (six-row trips would need over 256 VGPRs there: one wave per
    // SIMD).  Measured VALU instructions per quad of the main loop: one
    // column, six-row trips 164-174 against 178-185 for two-row trips.  The
    // first trip is peeled: the loop is then entered only after the memory
    // operations of a whole trip, as on every later trip, so the compiler's
    // wait counts for the queued loads are exact rather than those of the
    // store-free prologue.
    constexpr int TRIP = (IO == kIoGeneric || (COLS == 2 && io_out_u8(IO))) ? 2 : 6;
    int R = R0;
    {
        const int q1 = R0 + (R1 - R0) / 4, q2 = R0 + (R1 - R0) / 2, q3 = R0 + 3 * (R1 - R0) / 4;
        auto prio = [&](int r) {
            if constexpr (PACED) {
                if (r >= q3) __builtin_amdgcn_s_setprio(0);
                else if (r >= q2) __builtin_amdgcn_s_setprio(1);
                else if (r >= q1) __builtin_amdgcn_s_setprio(2);
                else __builtin_amdgcn_s_setprio(3);
            }
        };
        auto trip = [&](int r) {
#pragma unroll
            for (int k = 0; k < TRIP; k += 2) {
                strip_step<COLS, BETA, IO, 0, ST>(s, QB, cx, P, L, r + k);
                strip_step<COLS, BETA, IO, 0, ST>(s, QA, cx, P, L, r + k + 1);
            }
        };
        if (R + TRIP - 1 < R1) {
            prio(R);
            trip(R);
            for (R += TRIP; R + TRIP - 1 < R1; R += TRIP) {
                prio(R);
                trip(R);
            }
        }
#pragma unroll
        for (int k = 2; k < TRIP; k += 2) {
            if (R + 1 < R1) {
                strip_step<COLS, BETA, IO, 0, ST>(s, QB, cx, P, L, R);
                strip_step<COLS, BETA, IO, 0, ST>(s, QA, cx, P, L, R + 1);
                R += 2;
            }
        }
    }
    if (R < R1) strip_step<COLS, BETA, IO, 0, ST>(s, QB, cx, P, L, R);
}

}  // namespace wz
