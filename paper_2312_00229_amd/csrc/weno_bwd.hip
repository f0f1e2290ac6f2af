// Adjoint of the WD-WENO 2x zoom (weno_zoom2x_backward); the kernel body is
// in weno_bwd.h.
#include <hip/hip_runtime.h>

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
                                                            int strips_x, int strips_y, int rows, FwdParams P)
{
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
    const int R0 = sy * rows;
    const int R1 = min(R0 + rows, cx.H);
    bwd_strip<BETA>(cx, P, sx, R0, R1);
}

}  // namespace

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
    const int strips_x = (x->w + kBwdOwn - 1) / kBwdOwn;
    // Bands give about four waves per SIMD (two resident at a time, 232
    // registers each): measured on 16 x 3 x 512^2, two rounds of waves beat a
    // single round of twice-as-tall strips (0.70 ms at 96 rows vs 1.0 ms at
    // 171), and strips shorter than 32 rows pay too much for the 21-row
    // pipeline fill.
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    const int64_t columns = (int64_t)x->n * x->c * strips_x;
    const int64_t target = 4 * 4 * (int64_t)cus;
    int64_t bands = target / columns;
    if (bands < 1) bands = 1;
    int rows = (int)((x->h + bands - 1) / bands);
    if (rows < 32) rows = 32;
    if (wz_explicit_rows() > 0) rows = wz_explicit_rows();
    const int strips_y = (x->h + rows - 1) / rows;
    dim3 grid((strips_x * strips_y + kWavesPerBlock - 1) / kWavesPerBlock, x->n * x->c);
    hipStream_t st = (hipStream_t)hip_stream;
    const int bm = wz_beta_mode(p->beta);
    if (bm == 2)
        hipLaunchKernelGGL(zoom2x_bwd_kernel<2>, grid, dim3(kBlock), 0, st, cx, x->c, x->sn * 4, x->sc * 4,
                           grad_y->sn * 4, grad_y->sc * 4, grad_x->sn * 4, grad_x->sc * 4, strips_x, strips_y, rows, P);
    else if (bm == 1)
        hipLaunchKernelGGL(zoom2x_bwd_kernel<1>, grid, dim3(kBlock), 0, st, cx, x->c, x->sn * 4, x->sc * 4,
                           grad_y->sn * 4, grad_y->sc * 4, grad_x->sn * 4, grad_x->sc * 4, strips_x, strips_y, rows, P);
    else
        hipLaunchKernelGGL(zoom2x_bwd_kernel<kBetaGeneral>, grid, dim3(kBlock), 0, st, cx, x->c, x->sn * 4,
                           x->sc * 4, grad_y->sn * 4, grad_y->sc * 4, grad_x->sn * 4, grad_x->sc * 4, strips_x,
                           strips_y, rows, P);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wz_hip_error(e, "zoom2x_bwd_kernel launch");
    return WENO_OK;
}
