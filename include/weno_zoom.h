/*
 * weno_zoom.h -- C ABI of the MI355X (gfx950) WD-WENO 2x zoom library.
 *
 * Method: B. Crnkovic, J. Skific, T. Bosner, "WENO based adaptive image
 * zooming algorithm" (arXiv 2312.00229), Section 3: every output pixel of a
 * resolution doubling is a nonlinear blend of four quadratic 1D candidates,
 * along the diagonals for the odd/odd "x" points (phase 1, eqs. Vektor ..
 * 2dKombinacija, algorithm 1) and along the axes for the mixed-parity "+"
 * points (phase 2, eqs. tezine .. 2dKombinacijaRavno, algorithm 2); the
 * weights come from smoothness indicators summed with those of the four
 * nearest points of the same phase.
 *
 * Conventions shared by every entry point
 *   - Pixel (I, J) of a plane owns the 2x2 output quad
 *       out[2I][2J]     = in[I][J]             (original, copied exactly)
 *       out[2I][2J+1]   = "+" point at (I, J + 1/2)
 *       out[2I+1][2J]   = "+" point at (I + 1/2, J)
 *       out[2I+1][2J+1] = "x" point at (I + 1/2, J + 1/2)
 *     so an H x W plane becomes 2H x 2W; the paper's (2H-1) x (2W-1) grid is
 *     the leading crop.  Input samples outside the plane are clamped to the
 *     edge (the paper does not say; callers that want other boundary data
 *     pad the input themselves and crop: a quad reads inputs I-4..I+5,
 *     J-4..J+5).
 *   - Channels and batch images are independent planes.
 *   - Tensors are described by weno_tensor_t: a DEVICE pointer plus shape
 *     and element strides, so NCHW, NHWC and views all work.  Memory is
 *     owned by the caller; the library keeps no pointer after a call
 *     returns.
 *   - Arithmetic is FP32.  uint8 data are read on the [0,1] scale
 *     (value/255) -- the kernels work on the 0..255 scale with eps scaled by
 *     255^2, which gives the same weights -- and written back as
 *     clamp(round-half-even(255 u), 0, 255).
 *   - Every call is asynchronous on the caller's HIP stream (NULL = the
 *     default stream), returns a status code (0 = WENO_OK, negative =
 *     error, text from weno_status_string) and never aborts.  Argument
 *     errors are detected on the host before anything is enqueued.
 *   - Non-finite inputs propagate; they are not checked.
 *   - Float samples are supported up to 1e8 in magnitude at beta <= 2: the
 *     kernels square sums of squared differences in FP32 (the doubling's
 *     weights 1/t^2, the resampler's E0^2 / (E0^2 + k E1^2)), which leave the
 *     FP32 range for samples of about 1e9 and beyond; larger beta narrows
 *     the range (t^-beta underflows where every direction is rough).
 *   - Thread safety: calls may come from several host threads; the only
 *     process-global state is the launch configuration set by
 *     weno_set_launch_config (read at each call).
 */
#ifndef WENO_ZOOM_H
#define WENO_ZOOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define WENO_OK 0
#define WENO_EINVAL (-1)   /* null pointer, bad size, shape mismatch, bad parameter  */
#define WENO_EDTYPE (-2)   /* unsupported dtype combination                           */
#define WENO_EOVERLAP (-3) /* output memory overlaps an input                         */
#define WENO_ENOSPC (-4)   /* caller workspace too small                              */
#define WENO_EHIP (-5)     /* HIP runtime error; see weno_status_string(WENO_EHIP)    */

typedef enum { WENO_U8 = 0, WENO_F32 = 1 } weno_dtype_t;

/* Input samples outside an (h, w) plane, read by quads near its edges. */
typedef enum {
    WENO_BOUNDARY_CLAMP = 0,    /* the nearest edge sample (default)                   */
    WENO_BOUNDARY_EXTERNAL = 1  /* the caller's own data: rows -4 .. h+4 and columns
                                   -4 .. w+4 of every plane, addressed through the
                                   tensor's strides, must be readable memory (src is a
                                   view into a larger array).  The ghost samples of
                                   the paper's function tests (f beyond the domain)
                                   are passed this way, without padding and cropping.
                                   Accepted by weno_zoom2x and the batched entry
                                   points; dst must not overlap the extended region. */
} weno_boundary_t;

typedef struct {
    void* data;              /* device pointer to element [0][0][0][0]              */
    int32_t dtype;           /* weno_dtype_t                                        */
    int32_t n, c, h, w;      /* batch, channels, rows, columns; all >= 1            */
    int64_t sn, sc, sh, sw;  /* strides in ELEMENTS (not bytes), any sign >= 0      */
} weno_tensor_t;

typedef struct {
    float beta;   /* exponent of the nonlinear weights, eq. (alpha); in
                     [0, 64].  The paper's images use 2, its convergence
                     table 1.  With beta > 0, eps = k_eps h^2 must be > 0 and
                     keep the sum of four weights finite in FP32:
                     beta * log2((3/13) eps) >= -124 (WENO_EINVAL otherwise;
                     e.g. beta <= 4 at eps = 1e-8).                           */
    float k_eps;  /* eps_h = k_eps * h^2 (Section 2, eq. IzrazOmega); >= 0,
                     the paper's usual value 1e-8                              */
    float h;      /* input grid spacing (> 0); 1 for images                    */
    float nbw;    /* weight of the four neighbour indicators in D, eqs.
                     (2DsmoothnessFinal) and (tezine).  < 0 selects h^2/8,
                     the value in the proof of Theorem 1 (eq. DDiffOrder)
                     and the one that reproduces row 2 of Table 1; the
                     definitions print h^2/4, which callers may pass
                     explicitly.                                               */
    int32_t boundary; /* weno_boundary_t                                       */
} weno_params_t;

/* Default parameters: beta 2, k_eps 1e-8, h 1, nbw -1 (h^2/8), clamp. */
weno_params_t weno_default_params(void);

/*
 * One WD-WENO doubling (Section 3, phases 1 and 2 fused in one kernel).
 *   src: (n, c, h, w), WENO_U8 or WENO_F32.
 *   dst: (n, c, 2h, 2w), WENO_U8 or WENO_F32 (any combination with src).
 *   dst must not overlap src.
 */
int weno_zoom2x(const weno_tensor_t* src, const weno_tensor_t* dst, const weno_params_t* p,
                void* hip_stream);

/*
 * Many independent images of uneven sizes in ONE persistent launch: the
 * workgroups pull row strips of all images from a shared work queue (images
 * ordered largest first).  The outputs are bit-identical to weno_zoom2x
 * called per image with the same launch configuration.
 *
 * Two steps, so that the launch itself can be captured into a hipGraph:
 *   weno_zoom2x_batched_plan  validates every pair, writes the image table
 *       into the caller's DEVICE workspace (one host-to-device copy on the
 *       stream, after which the call waits for the stream) and fills `plan`;
 *   weno_zoom2x_batched_run   enqueues a one-thread reset of the queue head
 *       and the persistent kernel; it copies nothing and allocates nothing.
 * weno_zoom2x_batched does both.
 *   srcs[i], dsts[i]: HOST arrays of `count` descriptors (device data), each
 *                     pair obeying the rules of weno_zoom2x; no output may
 *                     overlap any input or another output.
 *   d_workspace:      DEVICE memory, 256-byte aligned, at least
 *                     weno_zoom2x_batched_workspace(count) bytes, owned by the
 *                     caller and left untouched between plan and run.  Runs
 *                     that share a workspace must be ordered on one stream.
 */
typedef struct {
    void* d_workspace;
    size_t ws_bytes;
    int64_t total_items;     /* queue length (row strips of all planes) */
    int32_t count;
    int32_t rows_per_strip;  /* launch configuration captured at plan time */
    int32_t cols_per_lane;
    int32_t beta_mode;
    int64_t reserved;
} weno_batch_plan_t;

size_t weno_zoom2x_batched_workspace(int32_t count);
int weno_zoom2x_batched_plan(const weno_tensor_t* srcs, const weno_tensor_t* dsts, int32_t count,
                             const weno_params_t* p, void* d_workspace, size_t ws_bytes, void* hip_stream,
                             weno_batch_plan_t* plan);
int weno_zoom2x_batched_run(const weno_batch_plan_t* plan, void* hip_stream);
int weno_zoom2x_batched(const weno_tensor_t* srcs, const weno_tensor_t* dsts, int32_t count,
                        const weno_params_t* p, void* d_workspace, size_t ws_bytes, void* hip_stream);

/*
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): weno_zoom2x_batched without a caller
 * workspace.  The image table and the queue head live in a fixed device
 * array inside the library, one per GPU, kept until the process ends
 * (about 700 KB).  The call allocates nothing; like weno_zoom2x_batched it
 * copies the table to the device and waits for the stream once before the
 * launch (so it cannot be captured into a graph; use the plan/run pair with a
 * caller workspace for that).
 *   count: 1 .. WENO_NOALLOC_MAX_IMAGES, else WENO_EINVAL (< 1) or
 *          WENO_ENOSPC (more images than the fixed array holds).
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (from several host threads or on several streams without ordering) race
 * and must be serialised by the caller.  Outputs are bit-identical to
 * weno_zoom2x_batched with the same launch configuration.
 */
#define WENO_NOALLOC_MAX_IMAGES 4096
int weno_zoom2x_batched_noalloc(const weno_tensor_t* srcs, const weno_tensor_t* dsts, int32_t count,
                                const weno_params_t* p, void* hip_stream);

/*
 * `levels` successive doublings (eq. zoomfactor), FP32 intermediates in the
 * caller's workspace, the grid spacing halved at each level (h, h/2, ...).
 *   src: (n, c, h, w); dst: (n, c, 2^levels h, 2^levels w); 1 <= levels <= 8.
 *   d_workspace: DEVICE memory, 256-byte aligned (as hipMalloc returns), of
 *                at least weno_zoom2x_cascade_workspace(src, levels) bytes.
 * Only kernels are enqueued (no copies, no allocation), so the call can be
 * captured into a hipGraph and replayed.
 */
size_t weno_zoom2x_cascade_workspace(const weno_tensor_t* src, int32_t levels);
int weno_zoom2x_cascade(const weno_tensor_t* src, const weno_tensor_t* dst, int32_t levels,
                        const weno_params_t* p, void* d_workspace, size_t ws_bytes, void* hip_stream);

/*
 * Tensor-product WENO resampling (Section 3.3, eq. tensor): every plane of
 * src (n, c, h, w) is resampled to dst (n, c, H, W) of ANY size with the 1D
 * WENO spline of Section 2 (eqs. Tocnost .. IzrazOmega; ideal weights
 * C_0 = (2 - t)/3, C_1 = (t + 1)/3 on [x_i, x_{i+1}]) along the rows, then
 * along the columns.  End points are aligned: output sample j of an axis sits
 * at input coordinate j (h_in - 1)/(h_out - 1); samples on input nodes are
 * copied exactly; samples beyond the ends are clamped.  eps = k_eps h^2 as for
 * the doubling (nbw is unused).
 *   d_workspace: DEVICE memory, 256-byte aligned, of at least
 *                weno_resample_workspace(src, dst) bytes: the positions of the H rows and W columns and, only
 *                where (w - 1)/(W - 1) exceeds about 16, an FP32
 *                (n, c, H, w + 3) intermediate.  Kernels only: capturable.
 */
size_t weno_resample_workspace(const weno_tensor_t* src, const weno_tensor_t* dst);
int weno_resample(const weno_tensor_t* src, const weno_tensor_t* dst, const weno_params_t* p, void* d_workspace,
                  size_t ws_bytes, void* hip_stream);

/*
 * Zoom to ANY size (Section 3.3): k WD-WENO doublings, k the least with
 * 2^k (h - 1) + 1 >= H and 2^k (w - 1) + 1 >= W (an axis of one sample is not
 * doubled), each level doubling the paper's (2h'-1) x (2w'-1) grid of the
 * previous level with the spacing halved, then weno_resample of the
 * (2^k (h-1) + 1) x (2^k (w-1) + 1) grid to (H, W).  k = 0 (a target no larger
 * than the source) is plain resampling.
 *   d_workspace: DEVICE memory, 256-byte aligned, of at least
 *                weno_zoom_to_workspace(src, dst) bytes (FP32 intermediates and
 *                the resampler's workspace).  Kernels only: capturable.
 */
size_t weno_zoom_to_workspace(const weno_tensor_t* src, const weno_tensor_t* dst);
int weno_zoom_to(const weno_tensor_t* src, const weno_tensor_t* dst, const weno_params_t* p, void* d_workspace,
                 size_t ws_bytes, void* hip_stream);

/*
 * Adjoint of weno_zoom2x: grad_x = (d out / d x)^T grad_y for the forward
 * input x (clamped reads fold their gradient onto the edge pixels).  The
 * smoothness indicators, weights and blends of both phases are
 * differentiated exactly (du/dp_k = omega_k, du/dt_k = -beta omega_k
 * (p_k - u)/t_k with t_k = eps + D_k).
 *   x:      (n, c, h, w)   WENO_F32, the forward input
 *   grad_y: (n, c, 2h, 2w) WENO_F32
 *   grad_x: (n, c, h, w)   WENO_F32, overwritten (not accumulated)
 * Deterministic: no atomics, every gradient element is written by one thread.
 */
int weno_zoom2x_backward(const weno_tensor_t* x, const weno_tensor_t* grad_y, const weno_tensor_t* grad_x,
                         const weno_params_t* p, void* hip_stream);

/*
 * Launch configuration of the forward kernels (process-global, read at each
 * call; the Python autotuner sets it).
 *   rows_per_strip: output rows one wave walks down, in [4, 4096]
 *   cols_per_lane:  1 or 2 columns of quads per lane
 * (0, 0) selects the automatic choice (the default): the columns per lane and
 * strip height that minimise a cost model of the launch (workgroups per
 * compute unit x iterations per wave x measured time per iteration); e.g.
 * two columns and 27-row strips for a 1920x1080 RGB frame, one column and
 * 4-row strips for a 256x256 one.  For planar images whose last strip column
 * would hold no more than a one-column strip owns (e.g. 512 wide: four
 * two-column strips and 40 columns), the automatic choice may walk that
 * column in one-column strips of taller bands ("tail" strips).  The
 * configuration changes speed only: every configuration produces
 * bit-identical outputs.  Batched plans capture the configuration when they
 * are made (automatic: 32 rows, 2 columns, no tail strips).
 * weno_get_launch_config reports (0, 0) in automatic mode.
 * Returns WENO_EINVAL for values outside these sets.
 */
int weno_set_launch_config(int32_t rows_per_strip, int32_t cols_per_lane);
void weno_get_launch_config(int32_t* rows_per_strip, int32_t* cols_per_lane);

/*
 * The launch shape weno_zoom2x would use for this pair (the configuration
 * set above, else the automatic choice): rows_per_strip, cols_per_lane and
 * tail_rows (rows of the one-column tail strips; 0: none).  dst may be null:
 * an output in src's layout is assumed (only the layouts matter; no memory
 * is touched).  Any of the three out-pointers may be null.  Returns
 * WENO_EINVAL for an invalid src, or a dst whose shape is not src's doubled;
 * calls no HIP function but the current device and its attribute queries.
 */
int weno_query_launch_config(const weno_tensor_t* src, const weno_tensor_t* dst, int32_t* rows_per_strip,
                             int32_t* cols_per_lane, int32_t* tail_rows);

/*
 * Strip height of the adjoint kernel (weno_zoom2x_backward; process-global,
 * read at each call), independent of the forward's configuration.  The
 * adjoint always runs one column per lane.
 *   rows_per_strip: input rows one wave walks, in [4, 4096]; the top band of
 *                   a plane takes 4 rows fewer (at least 1), since it walks
 *                   4 extra steps to fold the padded rows above the image,
 *                   and the bottom band what is left.  0 selects the
 *                   automatic choice (the default): the height that
 *                   minimises the rounds of resident waves times the
 *                   longest band walk.
 * Gradients are bit-identical across strip heights.  Returns WENO_EINVAL for
 * values outside these sets.
 */
int weno_set_backward_launch_config(int32_t rows_per_strip);
void weno_get_backward_launch_config(int32_t* rows_per_strip);

/* Text for a status code; for WENO_EHIP the last HIP error seen by this
 * thread.  The pointer stays valid until the next call on the same thread. */
const char* weno_status_string(int status);

/* Library version, e.g. "1.0.0". */
const char* weno_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WENO_ZOOM_H */
