// Adjoint of the WD-WENO 2x zoom (weno_zoom2x_backward).
#include <hip/hip_runtime.h>

#include "weno_internal.h"
#include "weno_zoom.h"

extern "C" int weno_zoom2x_backward(const weno_tensor_t* x, const weno_tensor_t* grad_y, const weno_tensor_t* grad_x,
                                    const weno_params_t* p, void* hip_stream)
{
    (void)x; (void)grad_y; (void)grad_x; (void)p; (void)hip_stream;
    return WENO_EDTYPE;
}
