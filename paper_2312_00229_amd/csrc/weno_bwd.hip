// Adjoint of the WD-WENO 2x zoom (weno_zoom2x_backward); the kernel body is
// in weno_bwd.h.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

#include "weno_bwd.h"
#include "weno_internal.h"
#include "weno_zoom.h"

using namespace wz;

namespace {

// launch arguments: plane bases and extents (the kernel builds buffer resources per plane)
struct BwdArgs {
    const uint8_t* x_base;
    const uint8_t* gy_base;
    uint8_t* gx_base;
    uint32_t x_extent, gy_extent, gx_extent;
    uint32_t x_h, gy_h, gx_h, x_w, gy_w, gx_w;
    int32_t H, W;
};

template <int BETA>
__global__ __launch_bounds__(kBlock) void zoom2x_bwd_kernel(BwdArgs base, int C, int64_t x_n, int64_t x_c,
                                                            int64_t gy_n, int64_t gy_c, int64_t gx_n, int64_t gx_c,
                                                            int strips_x, int strips_y, int rows, int top_rows,
                                                            FwdParams P)
{
    __shared__ bwd_f32x4 ring[kWavesPerBlock * kBwdRingWords];
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    if (wave >= strips_x * strips_y) return;  // whole wave
    const int plane = blockIdx.y;
    const int n = plane / C, c = plane - n * C;
    const int sy = wave / strips_x, sx = wave - sy * strips_x;
    BwdCtx cx;
    cx.x = make_rsrc(base.x_base + n * x_n + c * x_c, base.x_extent);
    cx.gy = make_rsrc(base.gy_base + n * gy_n + c * gy_c, base.gy_extent);
    cx.gx = make_rsrc(base.gx_base + n * gx_n + c * gx_c, base.gx_extent);
    cx.x_h = base.x_h; cx.gy_h = base.gy_h; cx.gx_h = base.gx_h;
    cx.x_w = base.x_w; cx.gy_w = base.gy_w; cx.gx_w = base.gx_w;
    cx.H = base.H; cx.W = base.W;
    // band 0 holds top_rows rows, the others rows each (the last what is left)
    const int R0 = sy == 0 ? 0 : top_rows + (sy - 1) * rows;
    const int R1 = min(sy == 0 ? top_rows : R0 + rows, cx.H);
    bwd_strip<BETA>(cx, P, sx, R0, R1, ring + (threadIdx.x >> 6) * kBwdRingWords);
}

// Compute units of the current device and blocks of the adjoint kernel one
// of them holds at once (its register use allows two waves per SIMD, i.e. two
// blocks per CU), cached per device.
struct BwdDevice {
    int cus, per_cu;
};

BwdDevice bwd_device()
{
    static std::atomic<int> cache_cus[64], cache_per_cu[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return {256, 2};
    int cus = cache_cus[dev].load();
    if (cus == 0) {
        int per_cu = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(zoom2x_bwd_kernel<2>),
                                                         kBlock, 0) != hipSuccess || per_cu <= 0)
            per_cu = 1;
        cache_per_cu[dev].store(per_cu);
        cache_cus[dev].store(cus);
    }
    int per_cu = cache_per_cu[dev].load();
    return {cus, per_cu > 0 ? per_cu : 1};
}

// Bands of the adjoint: a walk over rows [R0, R1) takes R1 - R0 + 18 steps
// in the middle of a plane, 4 more in the top band (it starts four rows
// earlier to fold the padded rows -4..-1) and 5 more in the bottom one (it
// walks on to fold the padded rows H..H+4).  So the top band is made 4 rows
// shorter than the others and the automatic height leaves the bottom band
// about 5 short, and every band walks about as long.
struct BwdBands {
    int rows, top, count;   // height of the bands after the first, of the first, and their number
};

BwdBands bwd_bands(int H, int rows)
{
    if (rows >= H) return {H, H, 1};
    int top = rows - (kBwdWarmTop - kBwdWarm);
    if (top < 1) top = 1;
    return {rows, top, 1 + (H - top + rows - 1) / rows};
}

// Longest walk of a band layout, in rows plus the extra steps of the top and
// bottom bands (see bwd_bands); the warm-up every band walks is left out.
int bwd_longest_band(int H, const BwdBands& b)
{
    if (b.count == 1) return H + 9;
    const int last = H - b.top - (b.count - 2) * b.rows;
    const int edge = b.top + 4 > last + 5 ? b.top + 4 : last + 5;
    return b.count == 2 || edge > b.rows ? edge : b.rows;
}

// Strip height of the adjoint.  Every strip walks its rows plus kBwdWarm
// steps, the first of them forward only.  The blocks spread evenly over the
// CUs, so the busiest CU holds k = ceil(blocks / CUs) of them and runs them
// two at a time (one at a time where only one fits); a wave that shares its
// SIMD with another takes about 1.5x as long per row as a wave alone on it
// (measured on MI355X: ~1.8 us against ~1.2 us per row), so a launch costs
// about
//   (1.5 x shared rounds + lone rounds) x (longest band walk + kBwdWarmCost).
// Candidates: for each band count b, bands of ceil((H + 9) / b) rows (the
// edge bands then walk about as long as the others) and of ceil(H / b); the
// cheapest layout wins (the first found on a tie).  A launch of just over
// one block per CU thus pays for the pairs it forms: at 3x256x256 the model
// takes all-alone short strips over a layout that puts two blocks on some
// CUs.
int bwd_auto_rows(int H, int strips_x, int64_t planes, BwdDevice dev)
{
    int best_rows = H;
    int64_t best = INT64_MAX;
    const int max_b = H < 1024 ? H : 1024;
    for (int b = 1; b <= max_b; ++b) {
        for (int pass = 0; pass < 2; ++pass) {
            const int rows = b == 1 ? H : (pass == 0 ? (H + 9 + b - 1) / b : (H + b - 1) / b);
            if (rows < 4 && b > 1) continue;
            const BwdBands bands = bwd_bands(H, rows);
            const int64_t blocks = planes * (((int64_t)strips_x * bands.count + kWavesPerBlock - 1) / kWavesPerBlock);
            const int64_t k = (blocks + dev.cus - 1) / dev.cus;
            const int64_t shared = dev.per_cu >= 2 ? k / 2 : 0;
            const int64_t alone = k - 2 * shared;
            const int64_t cost = (3 * shared + 2 * alone) * (bwd_longest_band(H, bands) + kBwdWarmCost);
            if (cost < best) {
                best = cost;
                best_rows = rows;
            }
        }
    }
    return best_rows;
}

}  // namespace

// strip height of the adjoint set by weno_set_backward_launch_config (0 = automatic)
static std::atomic<int32_t> g_bwd_rows{0};

extern "C" int weno_set_backward_launch_config(int32_t rows_per_strip)
{
    if (rows_per_strip != 0 && (rows_per_strip < 4 || rows_per_strip > 4096)) return WENO_EINVAL;
    g_bwd_rows.store(rows_per_strip);
    return WENO_OK;
}

extern "C" void weno_get_backward_launch_config(int32_t* rows_per_strip)
{
    if (rows_per_strip) *rows_per_strip = g_bwd_rows.load();
}

FwdParams wz_fwd_params(const weno_params_t* p, int in_u8, int out_u8);

extern "C" int weno_zoom2x_backward(const weno_tensor_t* x, const weno_tensor_t* grad_y, const weno_tensor_t* grad_x,
                                    const weno_params_t* p, void* hip_stream)
{
    int rc = wz_check_tensor(x);
    if (rc) return rc;
    rc = wz_check_tensor(grad_y);
    if (rc) return rc;
    rc = wz_check_tensor(grad_x);
    if (rc) return rc;
    if (x->dtype != WENO_F32 || grad_y->dtype != WENO_F32 || grad_x->dtype != WENO_F32) return WENO_EDTYPE;
    rc = wz_check_params(p);
    if (rc) return rc;
    // the adjoint folds clamped reads onto the edge pixels; it has no ghost-sample form
    if (p->boundary != WENO_BOUNDARY_CLAMP) return WENO_EINVAL;
    if (grad_y->n != x->n || grad_y->c != x->c || (int64_t)grad_y->h != 2ll * x->h || (int64_t)grad_y->w != 2ll * x->w)
        return WENO_EINVAL;
    if (grad_x->n != x->n || grad_x->c != x->c || grad_x->h != x->h || grad_x->w != x->w) return WENO_EINVAL;
    if ((int64_t)x->n * x->c > 65535) return WENO_EINVAL;
    if (wz_plane_extent(x) >= (1ll << 31) || wz_plane_extent(grad_y) >= (1ll << 31) ||
        wz_plane_extent(grad_x) >= (1ll << 31))
        return WENO_EINVAL;
    if (wz_overlap(grad_x, x) || wz_overlap(grad_x, grad_y)) return WENO_EOVERLAP;

    BwdArgs cx;
    cx.x_base = (const uint8_t*)x->data;
    cx.gy_base = (const uint8_t*)grad_y->data;
    cx.gx_base = (uint8_t*)grad_x->data;
    cx.x_extent = (uint32_t)wz_plane_extent(x);
    cx.gy_extent = (uint32_t)wz_plane_extent(grad_y);
    cx.gx_extent = (uint32_t)wz_plane_extent(grad_x);
    cx.x_h = (uint32_t)(x->sh * 4);
    cx.gy_h = (uint32_t)(grad_y->sh * 4);
    cx.gx_h = (uint32_t)(grad_x->sh * 4);
    cx.x_w = (uint32_t)(x->sw * 4);
    cx.gy_w = (uint32_t)(grad_y->sw * 4);
    cx.gx_w = (uint32_t)(grad_x->sw * 4);
    cx.H = x->h;
    cx.W = x->w;
    const FwdParams P = wz_fwd_params(p, 0, 0);
    const int strips_x = bwd_strip_count(x->w);
    const int64_t planes = (int64_t)x->n * x->c;
    int rows = bwd_auto_rows(x->h, strips_x, planes, bwd_device());
    const int explicit_rows = g_bwd_rows.load();
    if (explicit_rows > 0) rows = explicit_rows;
    const BwdBands bands = bwd_bands(x->h, rows);
    const int strips_y = bands.count;
    dim3 grid((strips_x * strips_y + kWavesPerBlock - 1) / kWavesPerBlock, x->n * x->c);
    hipStream_t st = (hipStream_t)hip_stream;
    const int bm = wz_beta_mode(p->beta);
    if (bm == 2)
        hipLaunchKernelGGL(zoom2x_bwd_kernel<2>, grid, dim3(kBlock), 0, st, cx, x->c, x->sn * 4, x->sc * 4,
                           grad_y->sn * 4, grad_y->sc * 4, grad_x->sn * 4, grad_x->sc * 4, strips_x, strips_y, bands.rows,
                           bands.top, P);
    else if (bm == 1)
        hipLaunchKernelGGL(zoom2x_bwd_kernel<1>, grid, dim3(kBlock), 0, st, cx, x->c, x->sn * 4, x->sc * 4,
                           grad_y->sn * 4, grad_y->sc * 4, grad_x->sn * 4, grad_x->sc * 4, strips_x, strips_y, bands.rows,
                           bands.top, P);
    else
        hipLaunchKernelGGL(zoom2x_bwd_kernel<kBetaGeneral>, grid, dim3(kBlock), 0, st, cx, x->c, x->sn * 4,
                           x->sc * 4, grad_y->sn * 4, grad_y->sc * 4, grad_x->sn * 4, grad_x->sc * 4, strips_x,
                           strips_y, bands.rows, bands.top, P);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wz_hip_error(e, "zoom2x_bwd_kernel launch");
    return WENO_OK;
}
