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
// rounding; samples on input nodes are copied.  One thread per output
// element; the two passes (rows, then columns) go through an FP32
// intermediate in the caller's workspace.
#include <hip/hip_runtime.h>

#include <cmath>

#include "weno_internal.h"
#include "weno_zoom.h"

using namespace wz;

namespace {

struct ResampleArgs {
    const uint8_t* src;
    uint8_t* dst;
    int32_t C;
    int32_t in_h, in_w, out_h, out_w;   // along the resampled axis: in -> out; the other axis is equal
    int64_t s_n, s_c, s_h, s_w;         // byte strides
    int64_t d_n, d_c, d_h, d_w;
    int32_t in_u8, out_u8;
    float eps;        // in the kernel's value scale
    float beta;
    float out_scale;  // output value = u * out_scale
};

template <int BETA>
__device__ __forceinline__ float weno1d(float vm, float v0, float v1, float v2, float t, float eps, float beta)
{
    const float a1 = 0.5f * (v1 - vm);
    const float a2 = 0.5f * ((v1 + vm) - 2.0f * v0);
    const float b1 = 0.5f * (v2 - v0);
    const float b2 = 0.5f * ((v2 + v0) - 2.0f * v1);
    const float s = t - 1.0f;
    const float p0 = __builtin_fmaf(t, __builtin_fmaf(t, a2, a1), v0);
    const float p1 = __builtin_fmaf(s, __builtin_fmaf(s, b2, b1), v1);
    const float si0 = __builtin_fmaf(a1, a1, a2 * __builtin_fmaf(a2, 16.0f / 3.0f, 2.0f * a1));
    const float si1 = __builtin_fmaf(b1, b1, b2 * __builtin_fmaf(b2, 16.0f / 3.0f, -2.0f * b1));
    const float c0 = (2.0f - t) * (1.0f / 3.0f), c1 = (t + 1.0f) * (1.0f / 3.0f);
    float al0, al1;
    if constexpr (BETA == 2) {
        const float r0 = rcp(eps + si0), r1 = rcp(eps + si1);
        al0 = c0 * (r0 * r0);
        al1 = c1 * (r1 * r1);
    } else {
        al0 = c0 * __builtin_amdgcn_exp2f(-beta * __builtin_amdgcn_logf(eps + si0));
        al1 = c1 * __builtin_amdgcn_exp2f(-beta * __builtin_amdgcn_logf(eps + si1));
    }
    // u = p0 + omega_1 (p1 - p0)
    return __builtin_fmaf(al1 * rcp(al0 + al1), p1 - p0, p0);
}

// Source position of one output sample along an axis: the interval
// [x_i, x_{i+1}] and t in (0, 1), or a node copy of sample i (t < 0).
struct SamplePos {
    int32_t i;
    float t;
};

// Positions j (n_in - 1)/(n_out - 1) = i + t of an axis, one thread each,
// worked out in integers so that nodes are exact; t is rem/den rounded once.
__global__ __launch_bounds__(256) void positions_kernel(SamplePos* __restrict__ pos, int n_in, int n_out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_out) return;
    SamplePos p;
    p.i = 0;
    p.t = -1.0f;
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
            p.t = (float)((double)rem / (double)den);
        }
    }
    pos[j] = p;
}

// AXIS 0: resample along the rows (output row r <- input rows of column c),
// AXIS 1: along the columns (output column c <- input columns of row r).
template <int AXIS, int BETA, bool IN_U8, bool OUT_U8>
__global__ __launch_bounds__(256) void resample_kernel(ResampleArgs a, const SamplePos* __restrict__ pos)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (c >= a.out_w) return;
    const int plane = blockIdx.z;
    const int n = plane / a.C, ch = plane - n * a.C;
    const SamplePos p = pos[AXIS == 0 ? r : c];
    const int n_in = AXIS == 0 ? a.in_h : a.in_w;
    // the input line the samples come from and the stride along it; offsets
    // within a plane are 32-bit (planes span less than 2^31 bytes)
    const uint8_t* plane_in = a.src + n * a.s_n + ch * a.s_c;
    const uint32_t line = AXIS == 0 ? (uint32_t)c * (uint32_t)a.s_w : (uint32_t)r * (uint32_t)a.s_h;
    const uint32_t step = (uint32_t)(AXIS == 0 ? a.s_h : a.s_w);
    auto ld = [&](int k) -> float {
        const int kc = k < 0 ? 0 : (k >= n_in ? n_in - 1 : k);
        const uint8_t* q = plane_in + (line + (uint32_t)kc * step);
        if constexpr (IN_U8) return (float)*q;
        else return *(const float*)q;
    };
    float u;
    if (p.t < 0.0f) u = ld(p.i);
    else u = weno1d<BETA>(ld(p.i - 1), ld(p.i), ld(p.i + 1), ld(p.i + 2), p.t, a.eps, a.beta);
    uint8_t* o = a.dst + n * a.d_n + ch * a.d_c + ((uint32_t)r * (uint32_t)a.d_h + (uint32_t)c * (uint32_t)a.d_w);
    if constexpr (OUT_U8) *o = (uint8_t)quant_u8(u * a.out_scale);
    else *(float*)o = u * a.out_scale;
}

template <int AXIS, int BETA>
void launch_typed(const ResampleArgs& a, const SamplePos* pos, dim3 grid, hipStream_t st)
{
    if (a.in_u8 && a.out_u8)
        hipLaunchKernelGGL((resample_kernel<AXIS, BETA, true, true>), grid, dim3(256), 0, st, a, pos);
    else if (a.in_u8)
        hipLaunchKernelGGL((resample_kernel<AXIS, BETA, true, false>), grid, dim3(256), 0, st, a, pos);
    else if (a.out_u8)
        hipLaunchKernelGGL((resample_kernel<AXIS, BETA, false, true>), grid, dim3(256), 0, st, a, pos);
    else
        hipLaunchKernelGGL((resample_kernel<AXIS, BETA, false, false>), grid, dim3(256), 0, st, a, pos);
}

// bytes of a position table of n entries (256-byte aligned)
size_t positions_bytes(int64_t n) { return (size_t)((n * (int64_t)sizeof(SamplePos) + 255) / 256 * 256); }

int launch_positions(SamplePos* pos, int n_in, int n_out, hipStream_t st)
{
    hipLaunchKernelGGL(positions_kernel, dim3((n_out + 255) / 256), dim3(256), 0, st, pos, n_in, n_out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? WENO_OK : wz_hip_error(e, "positions_kernel launch");
}

// One pass along `axis` (0: rows, 1: columns); `pos` holds the positions of
// the resampled axis (dst->h entries for rows, dst->w for columns).
int launch_resample(int axis, const weno_tensor_t* src, const weno_tensor_t* dst, const weno_params_t* p, double h,
                    const SamplePos* pos, hipStream_t st)
{
    ResampleArgs a;
    const int64_t ei = wz_esize(src->dtype), eo = wz_esize(dst->dtype);
    a.src = (const uint8_t*)src->data;
    a.dst = (uint8_t*)dst->data;
    a.C = src->c;
    a.in_h = src->h;
    a.in_w = src->w;
    a.out_h = dst->h;
    a.out_w = dst->w;
    a.s_n = src->sn * ei; a.s_c = src->sc * ei; a.s_h = src->sh * ei; a.s_w = src->sw * ei;
    a.d_n = dst->sn * eo; a.d_c = dst->sc * eo; a.d_h = dst->sh * eo; a.d_w = dst->sw * eo;
    a.in_u8 = src->dtype == WENO_U8;
    a.out_u8 = dst->dtype == WENO_U8;
    const double vs = a.in_u8 ? 255.0 : 1.0;
    a.eps = (float)((double)p->k_eps * h * h * vs * vs);
    a.beta = p->beta;
    a.out_scale = (float)((a.out_u8 ? 255.0 : 1.0) / vs);
    dim3 grid((dst->w + 255) / 256, dst->h, dst->n * dst->c);
    const bool b2 = p->beta == 2.0f;
    if (axis == 0) {
        if (b2) launch_typed<0, 2>(a, pos, grid, st);
        else launch_typed<0, kBetaGeneral>(a, pos, grid, st);
    } else {
        if (b2) launch_typed<1, 2>(a, pos, grid, st);
        else launch_typed<1, kBetaGeneral>(a, pos, grid, st);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wz_hip_error(e, "resample_kernel launch");
    return WENO_OK;
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
    if ((int64_t)src->n * src->c > 65535 || dst->h > 65535) return WENO_EINVAL;
    // offsets within a plane are 32-bit: every plane (and the float
    // intermediate of the row pass) must span less than 2^31 bytes
    if (wz_plane_extent(src) >= (1ll << 31) || wz_plane_extent(dst) >= (1ll << 31)) return WENO_EINVAL;
    if (wz_overlap(src, dst)) return WENO_EOVERLAP;
    return WENO_OK;
}

}  // namespace

// workspace of the resampler: the row pass's float planes (dst->h x src->w),
// then the position tables of the rows and of the columns
static size_t resample_bytes(const weno_tensor_t* src, const weno_tensor_t* dst, int64_t in_w)
{
    return planes_bytes((int64_t)src->n * src->c, dst->h, in_w) + positions_bytes(dst->h) + positions_bytes(dst->w);
}

// the row pass, then the column pass, of src (any dtype, in_h x in_w) into dst
static int run_resample(const weno_tensor_t* src, const weno_tensor_t* dst, const weno_params_t* p, double h,
                        uint8_t* ws, hipStream_t st)
{
    if ((int64_t)dst->h * f32_pitch(src->w) * 4 >= (1ll << 31)) return WENO_EINVAL;   // 32-bit plane offsets
    weno_tensor_t tmp = planar_f32(ws, src->n, src->c, dst->h, src->w);
    if (wz_overlap(&tmp, src) || wz_overlap(&tmp, dst)) return WENO_EOVERLAP;
    uint8_t* tabs = ws + planes_bytes((int64_t)src->n * src->c, dst->h, src->w);
    SamplePos* rows = (SamplePos*)tabs;
    SamplePos* cols = (SamplePos*)(tabs + positions_bytes(dst->h));
    int rc = launch_positions(rows, src->h, dst->h, st);
    if (rc) return rc;
    rc = launch_positions(cols, src->w, dst->w, st);
    if (rc) return rc;
    rc = launch_resample(0, src, &tmp, p, h, rows, st);
    if (rc) return rc;
    return launch_resample(1, &tmp, dst, p, h, cols, st);
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
    if (!d_workspace) return WENO_EINVAL;
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
                  int cols);
void wz_config_for(const weno_tensor_t* src, int* rows, int* cols);

extern "C" int weno_zoom_to(const weno_tensor_t* src, const weno_tensor_t* dst, const weno_params_t* p,
                            void* d_workspace, size_t ws_bytes, void* hip_stream)
{
    int rc = check_resample_pair(src, dst);
    if (rc) return rc;
    rc = wz_check_params(p);
    if (rc) return rc;
    if (!d_workspace) return WENO_EINVAL;
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
        wz_config_for(&cur, &rows, &cols);
        rc = wz_launch_fwd(&cur, &out, &lp, st, rows, cols);
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
