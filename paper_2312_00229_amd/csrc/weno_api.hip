// C ABI of the WD-WENO 2x zoom library (declarations and contracts in
// include/weno_zoom.h).  Host-side validation, launch configuration and the
// forward / batched / cascade kernels; the adjoint lives in weno_bwd.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "weno_zoom.h"
#include "weno_fwd.h"
#include "weno_internal.h"

using namespace wz;

// --------------------------------------------------------------------------
// kernels
// --------------------------------------------------------------------------
namespace {

// per-plane context: buffer resources over the plane's byte extent
__device__ __forceinline__ StripCtx make_ctx(const FwdJob& jb, int n, int c, float out_scale)
{
    StripCtx cx;
    cx.src = make_rsrc(jb.src + n * jb.s_n + c * jb.s_c, jb.src_extent);
    cx.dst = make_rsrc(jb.dst + n * jb.d_n + c * jb.d_c, jb.dst_extent);
    cx.s_h = (uint32_t)jb.s_h;
    cx.s_w_bytes = (uint32_t)jb.s_w;
    cx.d_h = (uint32_t)jb.d_h;
    cx.d_w = (uint32_t)jb.d_w;
    cx.H = jb.H;
    cx.W = jb.W;
    cx.src_shift = jb.src_shift;
    cx.src_h = jb.src_h;
    cx.src_w = jb.src_w;
    cx.in_u8 = jb.in_u8;
    cx.out_u8 = jb.out_u8;
    cx.vec = jb.vec;
    cx.out_scale = out_scale;
    return cx;
}

// TAIL (two columns only): the launch has one-column tail strips
// (jb.tail_rows > 0) and one wave index across the planes
template <int COLS, int BETA, int IO, bool PACED, bool TAIL = false>
__global__ __launch_bounds__(kBlock) void zoom2x_kernel(FwdJob jb, FwdParams P, int rows_per_strip)
{
    // Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.
    // Renumber them so that every XCD gets a contiguous range of strips
    // (whole bands of adjacent rows): the 9 halo rows a strip shares with the
    // strip above are then re-read from the same L2.  A bijection on
    // [0, gridDim.x).  The XCD of a workgroup is its linear index (plane-major)
    // mod 8.  For images whose planes are interleaved (HWC) the host pads
    // gridDim.x to a multiple of 8: the same strip of every plane then runs
    // on the same XCD, and the lines the planes share meet in one L2 instead
    // of reaching HBM once per plane with a third of their bytes each (1080p
    // RGB uint8: writes 3.0x -> 1.0x the output, reads 4.1x -> 1.1x the
    // input).  Otherwise the XCD of a strip rotates from plane to plane,
    // which spreads the planes' workgroups evenly over the XCDs.  With tail
    // strips the grid is one-dimensional and every XCD gets a contiguous
    // range of waves, plane after plane.
    const int nb = gridDim.x, b = blockIdx.x;
    const int xcd = b % kXcds, k = b / kXcds;
    const int logical = xcd * (nb / kXcds) + min(xcd, nb % kXcds) + k;
    // the wave index is the same in every lane; say so, so that strip rows and
    // buffer offsets live in SGPRs
    const int wave = __builtin_amdgcn_readfirstlane(logical * kWavesPerBlock + (threadIdx.x >> 6));
    if constexpr (TAIL) {
        // One wave index across the planes (gridDim.y is 1).  Per plane: the
        // two-column strips, band by band, then the one-column strips of the
        // last columns (no more than a one-column strip owns), whose bands
        // are taller so that each walks about as long as a two-column strip.
        static_assert(COLS == 2, "tail strips follow two-column strips");
        const int n2 = jb.strips_x * jb.strips_y, per_plane = n2 + jb.tail_bands;
        const int plane = wave / per_plane;
        if (plane >= jb.planes) return;  // whole wave
        const int w = wave - plane * per_plane;
        const int n = plane / jb.C, c = plane - n * jb.C;
        const StripCtx cx = make_ctx(jb, n, c, P.out_scale);
        if (w < n2) {
            const int sy = w / jb.strips_x, sx = w - sy * jb.strips_x;
            const int R0 = sy * rows_per_strip;
            zoom_strip<2, BETA, IO, PACED>(cx, P, sx * strip_own<2>(), R0, min(R0 + rows_per_strip, jb.H));
        } else {
            const int R0 = (w - n2) * jb.tail_rows;
            zoom_strip<1, BETA, IO, PACED>(cx, P, jb.strips_x * strip_own<2>(), R0, min(R0 + jb.tail_rows, jb.H));
        }
    } else {
        const int per_plane = jb.strips_x * jb.strips_y;
        if (wave >= per_plane) return;  // whole wave
        const int plane = blockIdx.y;
        const int sy = wave / jb.strips_x;
        const int sx = wave - sy * jb.strips_x;
        const int n = plane / jb.C, c = plane - n * jb.C;
        const StripCtx cx = make_ctx(jb, n, c, P.out_scale);
        const int R0 = sy * rows_per_strip;
        const int R1 = min(R0 + rows_per_strip, jb.H);
        zoom_strip<COLS, BETA, IO, PACED>(cx, P, sx * strip_own<COLS>(), R0, R1);
    }
}

// Persistent kernel over a work queue of strips of many images.  Item i of
// image k covers plane (i / per_plane) and strip (i % per_plane); images are
// stored in the table largest first, so the queue drains big items early.
// The table is read-only during the launch and the queue head is reached
// through its own pointer, so table reads compile to scalar loads.
template <int COLS, int BETA>
__global__ __launch_bounds__(kBlock) void zoom2x_batched_kernel(const BatchTable* __restrict__ tab,
                                                                unsigned long long* __restrict__ counter,
                                                                int rows_per_strip)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int count = tab->count;
    const int64_t total = tab->total_items;
    const FwdJob* __restrict__ jobs = batch_jobs(tab);
    const int64_t* __restrict__ prefix = batch_prefix(tab);
    for (;;) {
        unsigned long long got = 0;
        if (lane == 0) got = atomicAdd(counter, 1ull);
        // broadcast lane 0's ticket as a provably uniform (scalar) value, so the
        // image table is read with scalar loads and the buffer resources stay
        // in SGPRs
        const uint32_t lo32 = __builtin_amdgcn_readfirstlane((uint32_t)got);
        const uint32_t hi32 = __builtin_amdgcn_readfirstlane((uint32_t)(got >> 32));
        const unsigned long long item = ((unsigned long long)hi32 << 32) | lo32;
        if ((int64_t)item >= total) break;  // every wave reaches this exit
        // image k with prefix[k] <= item < prefix[k+1]
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= (int64_t)item) lo = mid; else hi = mid - 1;
        }
        const FwdJob jb = jobs[lo];
        const int64_t local = (int64_t)item - prefix[lo];
        const int per_plane = jb.strips_x * jb.strips_y;
        const int plane = (int)(local / per_plane);
        const int wv = (int)(local - (int64_t)plane * per_plane);
        const int sy = wv / jb.strips_x;
        const int sx = wv - sy * jb.strips_x;
        const int n = plane / jb.C, c = plane - n * jb.C;
        const FwdParams P = batch_params(tab)[lo];
        const StripCtx cx = make_ctx(jb, n, c, P.out_scale);
        const int R0 = sy * rows_per_strip;
        const int R1 = min(R0 + rows_per_strip, jb.H);
        switch (jb.io) {
        case kIoF32: zoom_strip<COLS, BETA, kIoF32>(cx, P, sx * strip_own<COLS>(), R0, R1); break;
        case kIoU8: zoom_strip<COLS, BETA, kIoU8>(cx, P, sx * strip_own<COLS>(), R0, R1); break;
        case kIoU8F32: zoom_strip<COLS, BETA, kIoU8F32>(cx, P, sx * strip_own<COLS>(), R0, R1); break;
        case kIoF32U8: zoom_strip<COLS, BETA, kIoF32U8>(cx, P, sx * strip_own<COLS>(), R0, R1); break;
        default: zoom_strip<COLS, BETA, kIoGeneric>(cx, P, sx * strip_own<COLS>(), R0, R1); break;
        }
    }
}

__global__ void reset_counter_kernel(BatchTable* tab)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) tab->counter = 0ull;
}

}  // namespace

// --------------------------------------------------------------------------
// status / configuration
// --------------------------------------------------------------------------
static thread_local std::string g_status_text;
// 0 / 0 = automatic (chosen per launch from the image size)
static std::atomic<int32_t> g_rows_per_strip{0};
static std::atomic<int32_t> g_cols_per_lane{0};

int wz_hip_error(hipError_t e, const char* what)
{
    g_status_text = std::string(what) + ": " + hipGetErrorString(e);
    return WENO_EHIP;
}

extern "C" const char* weno_status_string(int status)
{
    switch (status) {
    case WENO_OK: return "ok";
    case WENO_EINVAL: return "invalid argument (null pointer, size, shape or parameter)";
    case WENO_EDTYPE: return "unsupported dtype combination";
    case WENO_EOVERLAP: return "output overlaps an input";
    case WENO_ENOSPC: return "workspace too small (weno_zoom2x_batched_noalloc: more images than its fixed scratch holds)";
    case WENO_EHIP:
        if (g_status_text.empty()) return "HIP runtime error";
        return g_status_text.c_str();
    default: return "unknown status";
    }
}

extern "C" const char* weno_version(void) { return "1.0.0"; }

extern "C" weno_params_t weno_default_params(void)
{
    weno_params_t p;
    p.beta = 2.0f;
    p.k_eps = 1e-8f;
    p.h = 1.0f;
    p.nbw = -1.0f;
    p.boundary = WENO_BOUNDARY_CLAMP;
    return p;
}

extern "C" int weno_set_launch_config(int32_t rows_per_strip, int32_t cols_per_lane)
{
    if (rows_per_strip == 0 && cols_per_lane == 0) {  // back to automatic
        g_rows_per_strip.store(0);
        g_cols_per_lane.store(0);
        return WENO_OK;
    }
    if (rows_per_strip < 4 || rows_per_strip > 4096) return WENO_EINVAL;
    if (cols_per_lane != 1 && cols_per_lane != 2) return WENO_EINVAL;
    g_rows_per_strip.store(rows_per_strip);
    g_cols_per_lane.store(cols_per_lane);
    return WENO_OK;
}

extern "C" void weno_get_launch_config(int32_t* rows_per_strip, int32_t* cols_per_lane)
{
    if (rows_per_strip) *rows_per_strip = g_rows_per_strip.load();
    if (cols_per_lane) *cols_per_lane = g_cols_per_lane.load();
}

// --------------------------------------------------------------------------
// validation helpers (shared with the adjoint and the cascade)
// --------------------------------------------------------------------------
int wz_esize(int32_t dtype) { return dtype == WENO_U8 ? 1 : (dtype == WENO_F32 ? 4 : 0); }


int wz_check_tensor(const weno_tensor_t* t)
{
    if (!t || !t->data) return WENO_EINVAL;
    if (wz_esize(t->dtype) == 0) return WENO_EDTYPE;
    if (t->n < 1 || t->c < 1 || t->h < 1 || t->w < 1) return WENO_EINVAL;
    if (t->sn < 0 || t->sc < 0 || t->sh < 0 || t->sw < 0) return WENO_EINVAL;
    return WENO_OK;
}

void wz_byte_range(const weno_tensor_t* t, uintptr_t* lo, uintptr_t* hi)
{
    const int64_t es = wz_esize(t->dtype);
    const int64_t last = ((int64_t)(t->n - 1) * t->sn + (int64_t)(t->c - 1) * t->sc + (int64_t)(t->h - 1) * t->sh +
                          (int64_t)(t->w - 1) * t->sw) * es;
    *lo = (uintptr_t)t->data;
    *hi = (uintptr_t)t->data + (uintptr_t)last + (uintptr_t)es;
}

// bytes spanned by one (h, w) plane of t
int64_t wz_plane_extent(const weno_tensor_t* t)
{
    const int64_t es = wz_esize(t->dtype);
    return ((int64_t)(t->h - 1) * t->sh + (int64_t)(t->w - 1) * t->sw) * es + es;
}

bool wz_overlap(const weno_tensor_t* a, const weno_tensor_t* b)
{
    uintptr_t alo, ahi, blo, bhi;
    wz_byte_range(a, &alo, &ahi);
    wz_byte_range(b, &blo, &bhi);
    return alo < bhi && blo < ahi;
}

int wz_check_params(const weno_params_t* p)
{
    if (!p) return WENO_EINVAL;
    if (!(p->beta >= 0.0f) || !std::isfinite(p->beta) || p->beta > 64.0f) return WENO_EINVAL;
    if (!(p->k_eps >= 0.0f) || !std::isfinite(p->k_eps)) return WENO_EINVAL;
    if (!(p->h > 0.0f) || !std::isfinite(p->h)) return WENO_EINVAL;
    if (!std::isfinite(p->nbw)) return WENO_EINVAL;
    if (p->boundary != WENO_BOUNDARY_CLAMP && p->boundary != WENO_BOUNDARY_EXTERNAL) return WENO_EINVAL;
    const double eps = (double)p->k_eps * (double)p->h * (double)p->h;
    // The kernels weigh with alpha = t^-beta for a scaled t = c (eps + D) on the
    // [0,1] scale (c = 1/4 in the doubling, 3/13 in its adjoint, 1 in the
    // resampler), and sum four of them: keep 4 ((3/13) eps)^-beta below 2^126
    // so that the sum stays finite in FP32 where every indicator vanishes.
    if (p->beta > 0.0f && (eps <= 0.0 || std::log2(eps * (3.0 / 13.0)) * (double)p->beta < -124.0))
        return WENO_EINVAL;
    return WENO_OK;
}

double wz_nbw(const weno_params_t* p) { return p->nbw < 0.0f ? (double)p->h * (double)p->h / 8.0 : (double)p->nbw; }

FwdParams wz_fwd_params(const weno_params_t* p, int in_u8, int out_u8)
{
    const double w = wz_nbw(p);
    const double vs = in_u8 ? 255.0 : 1.0;  // kernel value scale relative to [0,1]
    const double eps = (double)p->k_eps * (double)p->h * (double)p->h * vs * vs;
    FwdParams P;
    // with beta = 0 the weights are t^0 = 1 whatever the indicator, and eps
    // (which may then be 0) only has to keep t away from 0 for log2
    P.eps_hat = p->beta == 0.0f ? 1.0f : (float)(eps * (3.0 / 13.0) / (1.0 + 4.0 * w));
    P.eps_q = p->beta == 0.0f ? 1.0f : (float)(eps / (4.0 * (1.0 + 4.0 * w)));
    P.w = (float)w;
    P.beta = p->beta;
    const double os = out_u8 ? 255.0 : 1.0;
    P.out_scale = (float)(os / vs);
    return P;
}

int wz_beta_mode(float beta)
{
    if (beta == 2.0f) return 2;
    if (beta == 1.0f) return 1;
    return kBetaGeneral;
}

// Fill a FwdJob for src -> dst (shapes already validated).
// The readable source region of src for a boundary mode: src itself, or
// (WENO_BOUNDARY_EXTERNAL) rows -4 .. h+4 and columns -4 .. w+4 around it.
// Returns WENO_EINVAL if that region's start address would wrap.
int wz_source_region(const weno_tensor_t* src, int boundary, weno_tensor_t* region)
{
    *region = *src;
    if (boundary != WENO_BOUNDARY_EXTERNAL) return WENO_OK;
    const int64_t back = (4 * src->sh + 4 * src->sw) * wz_esize(src->dtype);
    if ((uintptr_t)src->data < (uintptr_t)back) return WENO_EINVAL;
    region->data = (void*)((uintptr_t)src->data - (uintptr_t)back);
    region->h = src->h + 9;
    region->w = src->w + 9;
    return WENO_OK;
}

// tail_rows > 0 (two columns only): the last strip column is walked by
// one-column strips of tail_rows rows (zoom2x_kernel)
FwdJob wz_make_job(const weno_tensor_t* src, const weno_tensor_t* dst, int cols, int rows_per_strip, int boundary,
                   int tail_rows)
{
    FwdJob jb;
    const int64_t ei = wz_esize(src->dtype), eo = wz_esize(dst->dtype);
    jb.src = (const uint8_t*)src->data;
    jb.dst = (uint8_t*)dst->data;
    jb.H = src->h;
    jb.W = src->w;
    jb.C = src->c;
    jb.planes = src->n * src->c;
    jb.s_n = src->sn * ei;
    jb.s_c = src->sc * ei;
    jb.s_h = src->sh * ei;
    jb.s_w = src->sw * ei;
    jb.d_n = dst->sn * eo;
    jb.d_c = dst->sc * eo;
    jb.d_h = dst->sh * eo;
    jb.d_w = dst->sw * eo;
    jb.in_u8 = src->dtype == WENO_U8;
    jb.out_u8 = dst->dtype == WENO_U8;
    const int own = cols == 1 ? strip_own<1>() : strip_own<2>();
    jb.strips_x = (src->w + own - 1) / own;
    jb.strips_y = (src->h + rows_per_strip - 1) / rows_per_strip;
    jb.tail_rows = 0;
    jb.tail_bands = 0;
    if (cols == 2 && tail_rows > 0 && jb.strips_x >= 2 && src->w - (jb.strips_x - 1) * own <= strip_own<1>()) {
        jb.strips_x -= 1;
        jb.tail_rows = tail_rows;
        jb.tail_bands = (src->h + tail_rows - 1) / tail_rows;
    }
    // vector stores need contiguous rows and aligned plane/row starts
    const uintptr_t base = (uintptr_t)dst->data;
    int vec = 0;
    if (!jb.out_u8 && dst->sw == 1) {
        const bool a8 = base % 8 == 0 && (jb.d_h % 8 == 0) && (jb.d_n % 8 == 0) && (jb.d_c % 8 == 0);
        const bool a16 = base % 16 == 0 && (jb.d_h % 16 == 0) && (jb.d_n % 16 == 0) && (jb.d_c % 16 == 0);
        vec = a16 ? 2 : (a8 ? 1 : 0);
    }
    jb.vec = vec;
    // fixed-layout I/O modes where the layout allows (float rows need vector
    // stores: contiguous, aligned destination columns)
    const bool vec_rows = cols == 2 ? vec == 2 : vec >= 1;
    if (jb.in_u8 && jb.out_u8) jb.io = kIoU8;
    else if (!jb.in_u8 && jb.out_u8) jb.io = kIoF32U8;
    else if (!vec_rows) jb.io = kIoGeneric;
    else jb.io = jb.in_u8 ? kIoU8F32 : kIoF32;
    jb.dst_extent = (uint32_t)wz_plane_extent(dst);
    weno_tensor_t region;
    wz_source_region(src, boundary, &region);   // validated by the caller
    jb.src = (const uint8_t*)region.data;
    jb.src_extent = (uint32_t)wz_plane_extent(&region);
    jb.src_shift = boundary == WENO_BOUNDARY_EXTERNAL ? 4 : 0;
    jb.src_h = region.h;
    jb.src_w = region.w;
    return jb;
}

// Checks of a doubling's source region beyond wz_check_pair: with caller
// ghost samples, the extended region must span less than 2^31 bytes per
// plane and must not overlap dst.
int wz_check_region(const weno_tensor_t* src, const weno_tensor_t* dst, int boundary)
{
    if (boundary != WENO_BOUNDARY_EXTERNAL) return WENO_OK;
    weno_tensor_t region;
    if (wz_source_region(src, boundary, &region) != WENO_OK) return WENO_EINVAL;
    if (wz_plane_extent(&region) >= (1ll << 31)) return WENO_EINVAL;
    if (wz_overlap(&region, dst)) return WENO_EOVERLAP;
    return WENO_OK;
}

// shape rules of one doubling
int wz_check_pair(const weno_tensor_t* src, const weno_tensor_t* dst, int factor)
{
    int rc = wz_check_tensor(src);
    if (rc) return rc;
    rc = wz_check_tensor(dst);
    if (rc) return rc;
    if (dst->n != src->n || dst->c != src->c) return WENO_EINVAL;
    if ((int64_t)dst->h != (int64_t)src->h * factor || (int64_t)dst->w != (int64_t)src->w * factor) return WENO_EINVAL;
    if ((int64_t)src->n * src->c > 65535) return WENO_EINVAL;
    // buffer offsets are 32-bit: every plane must span less than 2^31 bytes
    if (wz_plane_extent(src) >= (1ll << 31) || wz_plane_extent(dst) >= (1ll << 31)) return WENO_EINVAL;
    if (wz_overlap(src, dst)) return WENO_EOVERLAP;
    return WENO_OK;
}

static int device_cus();

// Workgroups of a kernel that one compute unit holds at once.  Cached per
// kernel: it depends only on the kernel's registers and the architecture,
// and the library is built for one architecture.
template <int COLS, int BETA, int IO>
static int fwd_resident_blocks()
{
    static std::atomic<int> cache{0};
    int v = cache.load();
    if (v == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &v, reinterpret_cast<const void*>(zoom2x_kernel<COLS, BETA, IO, true>), kBlock, 0) != hipSuccess ||
            v <= 0)
            v = 1;
        cache.store(v);
    }
    return v;
}

// Planes of one image interleaved in memory (channels closer together than
// rows, as in HWC): the same strip of its planes touches the same lines.
static bool planes_share_lines(int C, int64_t sc, int64_t sh)
{
    return C > 1 && std::llabs(sc) < std::llabs(sh);
}

// Workgroups along x for a plane of `strips` strips: padded to a multiple of
// the XCD count when the planes share lines (zoom2x_kernel), the padding
// exiting at once.  The busiest XCD then holds planes x grid_x / 8 of them.
static int fwd_grid_x(int64_t strips, bool share)
{
    const int64_t bx = (strips + kWavesPerBlock - 1) / kWavesPerBlock;
    return (int)(share ? (bx + kXcds - 1) / kXcds * kXcds : bx);
}

// A launch whose workgroups all fit on the device at once (one round) is
// paced (zoom_strip); one of several rounds is not.
template <int COLS, int BETA, int IO>
static hipError_t launch_fwd_beta(const FwdJob& jb, const FwdParams& P, int rows, hipStream_t st)
{
    const bool share = planes_share_lines(jb.C, jb.s_c, jb.s_h) || planes_share_lines(jb.C, jb.d_c, jb.d_h);
    dim3 grid(fwd_grid_x((int64_t)jb.strips_x * jb.strips_y, share), jb.planes);
    if constexpr (COLS == 2) {
        if (jb.tail_rows > 0) {  // one wave index across the planes
            const int64_t waves = (int64_t)jb.planes * ((int64_t)jb.strips_x * jb.strips_y + jb.tail_bands);
            grid = dim3((unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock), 1);
            if ((int64_t)grid.x <= (int64_t)fwd_resident_blocks<COLS, BETA, IO>() * device_cus())
                hipLaunchKernelGGL((zoom2x_kernel<COLS, BETA, IO, true, true>), grid, dim3(kBlock), 0, st, jb, P, rows);
            else
                hipLaunchKernelGGL((zoom2x_kernel<COLS, BETA, IO, false, true>), grid, dim3(kBlock), 0, st, jb, P,
                                   rows);
            return hipGetLastError();
        }
    }
    const int64_t blocks = (int64_t)grid.x * grid.y;
    if (blocks <= (int64_t)fwd_resident_blocks<COLS, BETA, IO>() * device_cus())
        hipLaunchKernelGGL((zoom2x_kernel<COLS, BETA, IO, true>), grid, dim3(kBlock), 0, st, jb, P, rows);
    else
        hipLaunchKernelGGL((zoom2x_kernel<COLS, BETA, IO, false>), grid, dim3(kBlock), 0, st, jb, P, rows);
    return hipGetLastError();
}

template <int COLS, int IO>
static hipError_t launch_fwd_io(const FwdJob& jb, const FwdParams& P, int beta_mode, int rows, hipStream_t st)
{
    if (beta_mode == 2) return launch_fwd_beta<COLS, 2, IO>(jb, P, rows, st);
    if (beta_mode == 1) return launch_fwd_beta<COLS, 1, IO>(jb, P, rows, st);
    return launch_fwd_beta<COLS, kBetaGeneral, IO>(jb, P, rows, st);
}

template <int COLS>
static hipError_t launch_fwd_cols(const FwdJob& jb, const FwdParams& P, int beta_mode, int rows, hipStream_t st)
{
    switch (jb.io) {
    case kIoF32: return launch_fwd_io<COLS, kIoF32>(jb, P, beta_mode, rows, st);
    case kIoU8: return launch_fwd_io<COLS, kIoU8>(jb, P, beta_mode, rows, st);
    case kIoU8F32: return launch_fwd_io<COLS, kIoU8F32>(jb, P, beta_mode, rows, st);
    case kIoF32U8: return launch_fwd_io<COLS, kIoF32U8>(jb, P, beta_mode, rows, st);
    default: return launch_fwd_io<COLS, kIoGeneric>(jb, P, beta_mode, rows, st);
    }
}

// compute units of the current device, cached per device
static int device_cus()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int v = cache[dev].load();
    if (v == 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cache[dev].store(v);
    }
    return v;
}

// Automatic launch configuration from a cost model of the strip walk.  Four
// strips (waves) make a workgroup, which runs on one compute unit, one wave
// per SIMD.  A launch whose busiest compute unit runs m workgroups takes about
//   m x (rows + 4) x R(cols, m)  microseconds,
// where rows + 4 are the iterations of one wave plus the fixed cost of
// starting it (its launch and the pipeline fill) and R(cols, m) the time of
// one iteration of one of m waves sharing a SIMD (a compute unit holds three
// two-column or five one-column workgroups at once: up to that, one paced
// round; beyond it, several rounds).  m counts workgroups, not waves: one
// compute unit given one workgroup more than the rest holds up the launch.
// R is fitted (least squares on the log of the time) to 511 timed launches
// on MI355X: 20 shapes from 1x64x64 to 3x2160x3840 and 48x512x512, both
// column counts, the three shortest strips of each m = 1..8.  Candidates
// are, for each column count and m = 1..8, the shortest strips that put at
// most m workgroups on a compute unit; the cheapest wins.  On those shapes
// the pick is within 6.2 % of the best measured launch (1080p RGB: two
// columns, 27-row strips).
static double iteration_cost(int cols, int64_t m)
{
    static const double one[8] = {0.421, 0.348, 0.319, 0.309, 0.302, 0.313, 0.308, 0.306};
    static const double two[8] = {0.708, 0.589, 0.557, 0.581, 0.571, 0.563, 0.562, 0.578};
    return (cols == 1 ? one : two)[m < 8 ? m - 1 : 7];
}
constexpr int kStartCost = 4;

// Tail strips: when the columns left of the last two-column strip fit one
// one-column strip, that strip column can be walked in one-column strips
// (half the work per row) with bands kTailStretch / 4 times as tall, so that
// each walks about as long as a two-column strip (a one-column iteration
// costs ~0.59 of a two-column one in the fit); the launch then numbers its
// waves across the planes.  48x512x512: four two-column strips and 40
// columns per band, 80.1 -> 71.9 predicted.
constexpr int kTailStretch = 7;

void wz_auto_config(int64_t planes, int H, int W, bool share, int* rows, int* cols, int* tail_rows)
{
    const int64_t cus = device_cus();
    double best = 0.0;
    int best_rows = 8, best_cols = 2, best_tail = 0;
    for (int c = 2; c >= 1; --c) {
        const int own = c == 1 ? strip_own<1>() : strip_own<2>();
        const int64_t strips_x = (W + own - 1) / own;
        for (int64_t m = 1; m <= 8; ++m) {
            // the most bands whose workgroups (planes x ceil(strips / 4), padded
            // as the launch pads them) fit m per compute unit
            int64_t per_plane = m * cus / planes;
            if (share) per_plane = per_plane / kXcds * kXcds;
            int64_t bands = kWavesPerBlock * per_plane / strips_x;
            if (bands < 1) bands = 1;
            int r = (int)((H + bands - 1) / bands);
            r = r < 4 ? 4 : (r > 4096 ? 4096 : r);
            const int64_t blocks = planes * fwd_grid_x(strips_x * ((H + r - 1) / r), share);
            const int64_t mm = (blocks + cus - 1) / cus;
            const double cost = (double)mm * (r + kStartCost) * iteration_cost(c, mm);
            if (best == 0.0 || cost < best) {
                best = cost;
                best_rows = r;
                best_cols = c;
                best_tail = 0;
            }
        }
    }
    // two-column strips with a one-column tail strip column (planar only)
    const int64_t sx = (W + strip_own<2>() - 1) / strip_own<2>();
    if (!share && sx >= 2 && W - (sx - 1) * strip_own<2>() <= strip_own<1>()) {
        const int64_t s2 = sx - 1;
        for (int64_t m = 1; m <= 8; ++m) {
            // waves per plane: s2 x bands + tail bands (~ bands x 4 / kTailStretch)
            const int64_t per_plane = kWavesPerBlock * m * cus / planes;
            int64_t bands = per_plane * kTailStretch / (s2 * kTailStretch + 4);
            if (bands < 1) bands = 1;
            int r = (int)((H + bands - 1) / bands);
            r = r < 4 ? 4 : (r > 4096 ? 4096 : r);
            int rt = r * kTailStretch / 4;
            rt = rt > H ? H : rt;
            const int64_t waves = planes * (s2 * ((H + r - 1) / r) + (H + rt - 1) / rt);
            const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
            const int64_t mm = (blocks + cus - 1) / cus;
            const double cost = (double)mm * (r + kStartCost) * iteration_cost(2, mm);
            if (cost < best) {
                best = cost;
                best_rows = r;
                best_cols = 2;
                best_tail = rt;
            }
        }
    }
    *rows = best_rows;
    *cols = best_cols;
    *tail_rows = best_tail;
}

// launch shape of one doubling: the caller's (weno_set_launch_config, never
// with tail strips) or the cost model's
void wz_config_for(const weno_tensor_t* src, const weno_tensor_t* dst, int* rows, int* cols, int* tail_rows)
{
    *rows = g_rows_per_strip.load();
    *cols = g_cols_per_lane.load();
    *tail_rows = 0;
    const bool share = planes_share_lines(src->c, src->sc, src->sh) || planes_share_lines(dst->c, dst->sc, dst->sh);
    if (*rows == 0 || *cols == 0)
        wz_auto_config((int64_t)src->n * src->c, src->h, src->w, share, rows, cols, tail_rows);
}

int wz_launch_fwd(const weno_tensor_t* src, const weno_tensor_t* dst, const weno_params_t* p, hipStream_t st,
                  int rows, int cols, int tail_rows)
{
    const FwdJob jb = wz_make_job(src, dst, cols, rows, p->boundary, tail_rows);
    const FwdParams P = wz_fwd_params(p, jb.in_u8, jb.out_u8);
    const int bm = wz_beta_mode(p->beta);
    const hipError_t e = cols == 1 ? launch_fwd_cols<1>(jb, P, bm, rows, st) : launch_fwd_cols<2>(jb, P, bm, rows, st);
    if (e != hipSuccess) return wz_hip_error(e, "zoom2x_kernel launch");
    return WENO_OK;
}

extern "C" int weno_query_launch_config(const weno_tensor_t* src, const weno_tensor_t* dst, int32_t* rows_per_strip,
                                        int32_t* cols_per_lane, int32_t* tail_rows)
{
    int rc = wz_check_tensor(src);
    if (rc) return rc;
    if (dst) {
        rc = wz_check_tensor(dst);
        if (rc) return rc;
        if (dst->n != src->n || dst->c != src->c || (int64_t)dst->h != 2ll * src->h || (int64_t)dst->w != 2ll * src->w)
            return WENO_EINVAL;
    }
    int rows, cols, tail;
    wz_config_for(src, dst ? dst : src, &rows, &cols, &tail);
    if (rows_per_strip) *rows_per_strip = rows;
    if (cols_per_lane) *cols_per_lane = cols;
    if (tail_rows) *tail_rows = tail;
    return WENO_OK;
}

// --------------------------------------------------------------------------
// single doubling
// --------------------------------------------------------------------------
extern "C" int weno_zoom2x(const weno_tensor_t* src, const weno_tensor_t* dst, const weno_params_t* p,
                           void* hip_stream)
{
    int rc = wz_check_pair(src, dst, 2);
    if (rc) return rc;
    rc = wz_check_params(p);
    if (rc) return rc;
    rc = wz_check_region(src, dst, p->boundary);
    if (rc) return rc;
    int rows, cols, tail;
    wz_config_for(src, dst, &rows, &cols, &tail);
    return wz_launch_fwd(src, dst, p, (hipStream_t)hip_stream, rows, cols, tail);
}

// --------------------------------------------------------------------------
// batched
// --------------------------------------------------------------------------
extern "C" size_t weno_zoom2x_batched_workspace(int32_t count)
{
    if (count < 1) return 0;
    return batch_table_bytes(count);
}

// argument rules of a batched call (host only, nothing is touched on the device)
static int batched_check(const weno_tensor_t* srcs, const weno_tensor_t* dsts, int32_t count, const weno_params_t* p)
{
    if (!srcs || !dsts || count < 1) return WENO_EINVAL;
    int rc = wz_check_params(p);
    if (rc) return rc;
    for (int i = 0; i < count; ++i) {
        rc = wz_check_pair(&srcs[i], &dsts[i], 2);
        if (rc) return rc;
        rc = wz_check_region(&srcs[i], &dsts[i], p->boundary);
        if (rc) return rc;
    }
    // no output may overlap any input or another output: sweep all byte
    // ranges by start address, remembering the furthest end of each kind
    {
        struct Iv { uintptr_t lo, hi; bool out; };
        std::vector<Iv> iv(2 * (size_t)count);
        for (int i = 0; i < count; ++i) {
            weno_tensor_t region;   // what the kernel reads of image i
            wz_source_region(&srcs[i], p->boundary, &region);
            wz_byte_range(&region, &iv[2 * i].lo, &iv[2 * i].hi);
            iv[2 * i].out = false;
            wz_byte_range(&dsts[i], &iv[2 * i + 1].lo, &iv[2 * i + 1].hi);
            iv[2 * i + 1].out = true;
        }
        std::sort(iv.begin(), iv.end(), [](const Iv& a, const Iv& b) { return a.lo < b.lo; });
        uintptr_t end_in = 0, end_out = 0;
        for (const Iv& v : iv) {
            if (v.lo < end_out || (v.out && v.lo < end_in)) return WENO_EOVERLAP;
            if (v.out) end_out = std::max(end_out, v.hi); else end_in = std::max(end_in, v.hi);
        }
    }
    return WENO_OK;
}

extern "C" int weno_zoom2x_batched_plan(const weno_tensor_t* srcs, const weno_tensor_t* dsts, int32_t count,
                                        const weno_params_t* p, void* d_workspace, size_t ws_bytes,
                                        void* hip_stream, weno_batch_plan_t* plan)
{
    if (!srcs || !dsts || !plan || count < 1 || !d_workspace) return WENO_EINVAL;
    int rc = wz_check_params(p);
    if (rc) return rc;
    if ((uintptr_t)d_workspace % 256 != 0) return WENO_EINVAL;
    if (ws_bytes < batch_table_bytes(count)) return WENO_ENOSPC;
    rc = batched_check(srcs, dsts, count, p);
    if (rc) return rc;
    int rows = g_rows_per_strip.load(), cols = g_cols_per_lane.load();
    if (rows == 0 || cols == 0) {  // the queue balances the load: moderate strips, two columns per lane
        rows = 32;
        cols = 2;
    }
    // largest images first
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (int64_t)srcs[a].h * srcs[a].w * srcs[a].n * srcs[a].c >
               (int64_t)srcs[b].h * srcs[b].w * srcs[b].n * srcs[b].c;
    });
    std::vector<uint8_t> host(batch_table_bytes(count), 0);
    BatchTable* tab = (BatchTable*)host.data();
    FwdJob* jobs = (FwdJob*)(host.data() + batch_jobs_offset());
    int64_t* prefix = (int64_t*)(host.data() + batch_prefix_offset(count));
    FwdParams* prm = (FwdParams*)(host.data() + batch_params_offset(count));
    int64_t total = 0;
    for (int k = 0; k < count; ++k) {
        const int i = order[k];
        jobs[k] = wz_make_job(&srcs[i], &dsts[i], cols, rows, p->boundary, 0);
        prm[k] = wz_fwd_params(p, jobs[k].in_u8, jobs[k].out_u8);
        prefix[k] = total;
        total += (int64_t)jobs[k].planes * jobs[k].strips_x * jobs[k].strips_y;
    }
    prefix[count] = total;
    tab->count = count;
    tab->total_items = total;
    tab->counter = 0;
    tab->params_offset = batch_params_offset(count);
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = hipMemcpyAsync(d_workspace, host.data(), host.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return wz_hip_error(e, "batch table copy");
    e = hipStreamSynchronize(st);  // the host table is freed on return
    if (e != hipSuccess) return wz_hip_error(e, "batch table copy");
    plan->d_workspace = d_workspace;
    plan->ws_bytes = ws_bytes;
    plan->total_items = total;
    plan->count = count;
    plan->rows_per_strip = rows;
    plan->cols_per_lane = cols;
    plan->beta_mode = wz_beta_mode(p->beta);
    plan->reserved = 0;
    return WENO_OK;
}

template <int COLS>
static hipError_t launch_batched_cols(const weno_batch_plan_t* plan, hipStream_t st)
{
    const int cus = device_cus();
    const int64_t waves_needed = plan->total_items;
    int64_t blocks = (int64_t)cus * 4;  // up to 4 workgroups (16 waves) per CU
    const int64_t by_work = (waves_needed + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > by_work) blocks = by_work;
    if (blocks < 1) blocks = 1;
    const BatchTable* tab = (const BatchTable*)plan->d_workspace;
    unsigned long long* counter = &((BatchTable*)plan->d_workspace)->counter;
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, (BatchTable*)plan->d_workspace);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (plan->beta_mode == 2)
        hipLaunchKernelGGL((zoom2x_batched_kernel<COLS, 2>), dim3((unsigned)blocks), dim3(kBlock), 0, st, tab,
                           counter, plan->rows_per_strip);
    else if (plan->beta_mode == 1)
        hipLaunchKernelGGL((zoom2x_batched_kernel<COLS, 1>), dim3((unsigned)blocks), dim3(kBlock), 0, st, tab,
                           counter, plan->rows_per_strip);
    else
        hipLaunchKernelGGL((zoom2x_batched_kernel<COLS, kBetaGeneral>), dim3((unsigned)blocks), dim3(kBlock), 0, st,
                           tab, counter, plan->rows_per_strip);
    return hipGetLastError();
}

extern "C" int weno_zoom2x_batched_run(const weno_batch_plan_t* plan, void* hip_stream)
{
    if (!plan || !plan->d_workspace || plan->count < 1 || plan->total_items < 1) return WENO_EINVAL;
    if (plan->cols_per_lane != 1 && plan->cols_per_lane != 2) return WENO_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    const hipError_t e = plan->cols_per_lane == 1 ? launch_batched_cols<1>(plan, st) : launch_batched_cols<2>(plan, st);
    if (e != hipSuccess) return wz_hip_error(e, "zoom2x_batched_kernel launch");
    return WENO_OK;
}

extern "C" int weno_zoom2x_batched(const weno_tensor_t* srcs, const weno_tensor_t* dsts, int32_t count,
                                   const weno_params_t* p, void* d_workspace, size_t ws_bytes, void* hip_stream)
{
    weno_batch_plan_t plan;
    int rc = weno_zoom2x_batched_plan(srcs, dsts, count, p, d_workspace, ws_bytes, hip_stream, &plan);
    if (rc) return rc;
    return weno_zoom2x_batched_run(&plan, hip_stream);
}

// --------------------------------------------------------------------------
// batched, without a caller workspace
// --------------------------------------------------------------------------
// The image table and queue head of weno_zoom2x_batched_noalloc live in this
// file-scope device array (one copy per GPU, alive until the process ends).
// In host code its name is only a stand-in for the symbol: the device
// address comes from hipGetSymbolAddress, once per device, and only that
// address is ever handed to a copy or a kernel.
constexpr size_t kNoAllocScratchBytes = batch_table_bytes(WENO_NOALLOC_MAX_IMAGES);
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];  // device address of `scratch` per device, set on first use

static int noalloc_scratch(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return wz_hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return WENO_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));  // the current device's copy
        if (e != hipSuccess) return wz_hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!ptr || (uintptr_t)ptr % 256 != 0) return wz_hip_error(hipErrorInvalidSymbol, "scratch address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return WENO_OK;
}

extern "C" int weno_zoom2x_batched_noalloc(const weno_tensor_t* srcs, const weno_tensor_t* dsts, int32_t count,
                                           const weno_params_t* p, void* hip_stream)
{
    if (!srcs || !dsts || count < 1) return WENO_EINVAL;
    if (count > WENO_NOALLOC_MAX_IMAGES) return WENO_ENOSPC;
    int rc = batched_check(srcs, dsts, count, p);
    if (rc) return rc;
    void* ws = nullptr;
    rc = noalloc_scratch(&ws);
    if (rc) return rc;
    // the plan validates everything before it writes the table into the
    // scratch (one host-to-device copy, then a wait on the stream); the run
    // clears the queue head with a kernel before the persistent launch
    weno_batch_plan_t plan;
    rc = weno_zoom2x_batched_plan(srcs, dsts, count, p, ws, kNoAllocScratchBytes, hip_stream, &plan);
    if (rc) return rc;
    return weno_zoom2x_batched_run(&plan, hip_stream);
}

// --------------------------------------------------------------------------
// cascade of doublings
// --------------------------------------------------------------------------
// row pitch (floats) of the float intermediates: a multiple of 4, so that
// rows are 16-byte aligned and the forward kernel stores them with vector
// stores (odd input widths would otherwise leave the first level unaligned)
static int64_t cascade_pitch(int64_t w) { return (w + 3) / 4 * 4; }

static void cascade_level_shape(const weno_tensor_t* src, int lvl, int64_t* h, int64_t* w)
{
    *h = (int64_t)src->h << lvl;
    *w = (int64_t)src->w << lvl;
}

extern "C" size_t weno_zoom2x_cascade_workspace(const weno_tensor_t* src, int32_t levels)
{
    if (wz_check_tensor(src) != WENO_OK || levels < 1 || levels > 8) return 0;
    size_t total = 0;
    for (int l = 1; l < levels; ++l) {
        int64_t h, w;
        cascade_level_shape(src, l, &h, &w);
        const size_t bytes = (size_t)src->n * src->c * h * cascade_pitch(w) * 4;
        total += (bytes + 255) / 256 * 256;
    }
    return total == 0 ? 256 : total;
}

extern "C" int weno_zoom2x_cascade(const weno_tensor_t* src, const weno_tensor_t* dst, int32_t levels,
                                   const weno_params_t* p, void* d_workspace, size_t ws_bytes, void* hip_stream)
{
    if (levels < 1 || levels > 8) return WENO_EINVAL;
    int rc = wz_check_tensor(src);
    if (rc) return rc;
    rc = wz_check_tensor(dst);
    if (rc) return rc;
    rc = wz_check_params(p);
    if (rc) return rc;
    // intermediate levels have no caller ghost samples
    if (p->boundary != WENO_BOUNDARY_CLAMP) return WENO_EINVAL;
    if (dst->n != src->n || dst->c != src->c || (int64_t)dst->h != ((int64_t)src->h << levels) ||
        (int64_t)dst->w != ((int64_t)src->w << levels))
        return WENO_EINVAL;
    if (wz_overlap(src, dst)) return WENO_EOVERLAP;
    if (levels > 1) {
        if (!d_workspace || (uintptr_t)d_workspace % 256 != 0) return WENO_EINVAL;
        if (ws_bytes < weno_zoom2x_cascade_workspace(src, levels)) return WENO_ENOSPC;
    }
    weno_tensor_t cur = *src;
    size_t off = 0;
    weno_params_t lp = *p;
    const double w0 = wz_nbw(p);
    for (int l = 0; l < levels; ++l) {
        weno_tensor_t out;
        if (l == levels - 1) {
            out = *dst;
        } else {
            int64_t h, w;
            cascade_level_shape(src, l + 1, &h, &w);
            out.data = (uint8_t*)d_workspace + off;
            out.dtype = WENO_F32;
            out.n = src->n;
            out.c = src->c;
            out.h = (int32_t)h;
            out.w = (int32_t)w;
            out.sw = 1;
            out.sh = cascade_pitch(w);
            out.sc = h * out.sh;
            out.sn = (int64_t)src->c * out.sc;
            const size_t bytes = (size_t)src->n * src->c * h * out.sh * 4;
            off += (bytes + 255) / 256 * 256;
            if (wz_overlap(&out, dst) || wz_overlap(&out, src)) return WENO_EOVERLAP;
        }
        rc = wz_check_pair(&cur, &out, 2);
        if (rc) return rc;
        // level l works on spacing h / 2^l; an explicit neighbour weight scales with h^2
        const double scale = std::ldexp(1.0, -l);
        lp.h = (float)(p->h * scale);
        lp.nbw = (float)(w0 * scale * scale);
        int rows, cols;
        int tail;
        wz_config_for(&cur, &out, &rows, &cols, &tail);
        rc = wz_launch_fwd(&cur, &out, &lp, (hipStream_t)hip_stream, rows, cols, tail);
        if (rc) return rc;
        cur = out;
    }
    return WENO_OK;
}
