/*
 * deskew.h -- C ABI of libdeskew.so: on-the-fly deskew of oblique-plane
 * light-sheet stacks and their projections on an MI355X (gfx950).
 *
 * Method (Lamb, Ward & Kaminski, arXiv 2211.00645):
 *   - Eq. 1: consecutive raw images are laterally offset by l = z cos(alpha),
 *     z the scan distance between images and alpha the sheet angle.  In image
 *     pixels of sample-space size p the per-image shift is
 *         s = (z * cos(alpha * pi / 180)) / p          (FP64, this order)
 *     and image n sits at offset o[n] = n * s (or caller-supplied offsets).
 *   - "Physical principles", remap paragraph and Fig. 2c: each raw image is
 *     remapped into a larger image at its accumulated offset.  The larger
 *     image has origin b = floor(min o) and width W = C + ceil(max o) - b.
 *     Output column x' of image n reads raw column x' + b - o[n] by linear
 *     interpolation, zero outside the raw image.  With o[n] - b = k + phi
 *     (k integer, phi in [0,1)):
 *         D[n][r][x'] = (1 - phi) * S[n][r][x' - k] + phi * S[n][r][x' - k - 1]
 *   - Fig. 2d: the maximum over images of D is the mimicked widefield view,
 *         Pmax[r][x'] = max_n D[n][r][x'];  Psum[r][x'] = sum_n D[n][r][x']
 *     (the sum accumulated in FP64, both rounded once to FP32).
 *
 * Conventions for every entry point:
 *   - Array pointers are DEVICE pointers owned by the caller unless a
 *     parameter says "host".  Arrays are dense, C order:
 *       stack  [planes][rows][cols]   (uint16 or float32)
 *       vol    [planes][rows][width]  float32
 *       psum, pmax [rows][width]      float32
 *   - Kernels are enqueued on the caller's stream and the call returns
 *     without waiting; nothing on the per-stack path allocates or
 *     synchronises.
 *   - Arguments are validated before anything is enqueued; on error nothing
 *     is enqueued and a negative dsk_status is returned.  No C++ exception
 *     crosses this boundary.
 *   - Inputs must be finite (a non-finite neighbour with zero weight would
 *     otherwise turn into NaN).  Device offsets must be finite.
 *   - Outputs must not alias inputs.
 */
#ifndef DESKEW_H
#define DESKEW_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DSK_OK = 0,
    DSK_EINVAL = -1,  /* null pointer, dims <= 0, non-finite geometry, pixel <= 0 */
    DSK_ESHAPE = -2,  /* a size does not fit (index range, workspace too small) */
    DSK_EHIP = -3,    /* HIP launch or runtime error */
    DSK_ENOMEM = -4,  /* device or host allocation failed (batch objects only) */
    DSK_EBUDGET = -5  /* request exceeds the serving memory budget */
} dsk_status;

typedef struct {
    int32_t planes, rows, cols;
} dsk_dims;

/* alpha in degrees, scan step z in micrometres (negative reverses the scan),
 * sample-space pixel size p in micrometres (> 0). */
typedef struct {
    double angle_deg, step_um, pixel_um;
} dsk_geom;

/* Launch shape of the forward kernels.  block: threads per workgroup (64,
 * 128 or 256); per_thread: output columns per thread (1, 2, 4 or 8; 4 and 8
 * use the aligned 16-byte vector kernel when the shape allows it);
 * nt_store: 1 streams the volume with non-temporal stores; unroll: planes
 * whose loads are issued together (1, 2 or 4); wg_per_cu: resident
 * workgroups per compute unit for the persistent batch kernel (0 = as many
 * as fit); pace_gbs: plane pacing of the vector kernel -- a wavefront that
 * runs ahead of the schedule "the launch's resident wavefronts move this
 * many GB/s" sleeps briefly, which keeps the wavefronts on neighbouring
 * planes and the write stream local; without a volume, wavefronts whose
 * planes start late wait for their turn (0 = no pacing; pacing only
 * delays, it never waits on another wavefront).  Every shape gives bitwise
 * identical results. */
typedef struct {
    int32_t block, per_thread, nt_store, unroll, wg_per_cu, pace_gbs;
} dsk_tune;

/* Human-readable name of a dsk_status value (static storage). */
const char *dsk_status_string(int status);

/* Bounds checks of debug builds (built with DSK_CHECK_BOUNDS=1: the library
 * libdeskew_bounds.so).  The forward, projections-only, batch and backward
 * kernels of such a build check every global address they read or write
 * against the extent of the buffer their arguments describe (the stack's
 * readable extent, the volume, the projections, the gradient volume and
 * adjoint), count each address outside it on the device, and send that
 * access to the extent's first element instead of out of the buffer.
 * *count (host) receives the count since the last reset; reset != 0 zeroes
 * it.  Returns 1 in a checking build, 0 in any other (*count = 0),
 * DSK_EINVAL for a null count, DSK_EHIP on a HIP error.  Synchronous. */
int dsk_debug_bounds_violations(unsigned long long *count, int reset);

/* Per-image shift in pixels, Eq. 1: s = (z cos(alpha pi/180)) / p in FP64.
 * shift_px: host out.  DSK_EINVAL if a value is non-finite or p <= 0. */
int dsk_shift_px(dsk_geom g, double *shift_px);

/* Shape query for the remap's larger image ("Physical principles", remap
 * paragraph).  offsets_px: host array of d.planes offsets, or NULL for the
 * uniform scan o[n] = n * shift_px.  Writes W to *out_width and b to
 * *origin (host).  Host only; touches no device.  DSK_ESHAPE if W reaches
 * 2^30 (widths and column counts stay below 2^30 everywhere). */
int dsk_plan(dsk_dims d, const double *offsets_px, double shift_px,
             int64_t *out_width, int64_t *origin);

/* Deskew a uint16 stack scanned uniformly with geometry g: o[n] = n * s,
 * origin and width from dsk_plan.  out_width 0 selects W; a positive value
 * clips or zero-pads the grid on the same formula.  vol, psum and pmax may
 * each be NULL (vol NULL is the live-view case); at least one must be set.
 * One fused pass: the volume and both projections come from one read of the
 * stack.  A paced frame with a volume and more column tiles than the device
 * holds at once goes out as bands of rows, one launch each, on `stream`
 * (bitwise the same result). */
int dsk_deskew_u16(const uint16_t *in, dsk_dims d, dsk_geom g, float *vol,
                   float *psum, float *pmax, int64_t out_width,
                   hipStream_t stream);

/* One colour channel of multi-channel camera frames (methods section: each
 * raw image is split into its colour channels and every channel is deskewed
 * on its own), read in place without a split copy.  frames: DEVICE uint16
 * [d.planes][d.rows][frame_cols]; the channel is the column range
 * [col0, col0 + d.cols) of every frame row (the camera's region layout is
 * the caller's: the paper does not fix it).  Geometry, outputs and
 * out_width as dsk_deskew_u16; the result is bitwise that of
 * dsk_deskew_u16 on the channel copied to a dense stack.  DSK_EINVAL if the
 * range leaves the frame.  Launch channels on separate streams to overlap
 * them. */
int dsk_deskew_channel_u16(const uint16_t *frames, int64_t frame_cols,
                           int64_t col0, dsk_dims d, dsk_geom g, float *vol,
                           float *psum, float *pmax, int64_t out_width,
                           hipStream_t stream);

/* As dsk_deskew_u16 with explicit per-image offsets (pixels).  offsets_dev:
 * DEVICE array of d.planes FP64 offsets (scan jitter, autograd).  origin
 * (b) and out_width (> 0) are explicit, so the grid can stay fixed while
 * the offsets change. */
int dsk_deskew_offsets_u16(const uint16_t *in, dsk_dims d,
                           const double *offsets_dev, int64_t origin,
                           float *vol, float *psum, float *pmax,
                           int64_t out_width, hipStream_t stream);

/* Float32 input, same contract as dsk_deskew_offsets_u16. */
int dsk_deskew_offsets_f32(const float *in, dsk_dims d,
                           const double *offsets_dev, int64_t origin,
                           float *vol, float *psum, float *pmax,
                           int64_t out_width, hipStream_t stream);

/* Forward with an explicit launch shape (tune != NULL) -- used by the
 * autotuner and the benchmark; results are bitwise identical for every
 * shape.  in_is_f32 selects the input type (in points to uint16 or float). */
int dsk_deskew_offsets_tuned(const void *in, int in_is_f32, dsk_dims d,
                             const double *offsets_dev, double shift_px,
                             int64_t origin, float *vol, float *psum,
                             float *pmax, int64_t out_width,
                             const dsk_tune *tune, hipStream_t stream);

/* Launch-shape tuner for one frame (the shape a live stream deskews over
 * and over).  Times candidate shapes -- one or two 4-column groups per
 * lane, unpaced and paced at 5000-6000 GB/s with a volume (9000-12000
 * without), and the default -- for `reps`
 * rounds (3..64), a burst of 3 back-to-back launches of each shape per
 * round, round-robin after one untimed round, re-times the front runners
 * in longer back-to-back runs, on the caller's own buffers and stream, and
 * returns in *tune, among the shapes whose mean time per launch is within
 * 0.5% of the fastest, the one paced slowest; with a volume its pace then
 * steps down by at least 100 GB/s and to at most 5800, clear
 * of the pacing cliff (*ms, host, may be NULL: the mean time measured for
 * the returned shape).  Arguments as
 * dsk_deskew_offsets_tuned.  Every trial computes the full result, so the
 * outputs may be written (with the correct values) or, when the choice is
 * already known, left untouched: call the forward with *tune afterwards.
 * The choice is remembered per architecture, input type, dims, out_width,
 * output set and offsets/uniform scan, in the process and, if the
 * environment variable DSK_TUNE_CACHE names a file, in that JSON file; a
 * remembered choice returns at once without launching.  Synchronises the
 * stream while timing.  Errors of the arguments are those of the forward. */
int dsk_deskew_autotune(const void *in, int in_is_f32, dsk_dims d,
                        const double *offsets_dev, double shift_px,
                        int64_t origin, float *vol, float *psum, float *pmax,
                        int64_t out_width, int reps, hipStream_t stream,
                        dsk_tune *tune, double *ms);

/* Adjoint of the remap (its transpose) applied to grad_vol [planes][rows]
 * [out_width], written as a gather with no atomics:
 *   grad_in[n][r][c] = (1-phi) gD[n][r][c+k] + phi gD[n][r][c+k+1],
 * gD read as 0 outside [0, out_width).  grad_in: [planes][rows][cols]. */
int dsk_deskew_adjoint_f32(const float *grad_vol, dsk_dims d,
                           const double *offsets_dev, int64_t origin,
                           int64_t out_width, float *grad_in,
                           hipStream_t stream);

/* Bytes of device workspace dsk_shear_grad_f32 / dsk_backward_f32 need. */
size_t dsk_shear_grad_workspace_bytes(dsk_dims d);

/* Derivative of a loss with respect to each image offset, given
 * grad_vol = dLoss/dD and the float32 stack in:
 *   grad_offsets[n] = sum_{r,x'} gD[n][r][x'] (S[x'-k-1] - S[x'-k])
 * (the right derivative in o[n] where o[n] - b is an integer), summed in
 * FP64 in a fixed order (deterministic).  grad_offsets: DEVICE, planes
 * doubles.  workspace: DEVICE, at least dsk_shear_grad_workspace_bytes(d)
 * bytes, caller-owned, contents need not be initialised. */
int dsk_shear_grad_f32(const float *in, const float *grad_vol, dsk_dims d,
                       const double *offsets_dev, int64_t origin,
                       int64_t out_width, double *grad_offsets,
                       void *workspace, size_t workspace_bytes,
                       hipStream_t stream);

/* Fused backward: grad_in (adjoint) and grad_offsets (shear gradient) from
 * one read of grad_vol.  Either output may be NULL (not both); the
 * workspace is required when grad_offsets is set. */
int dsk_backward_f32(const float *in, const float *grad_vol, dsk_dims d,
                     const double *offsets_dev, int64_t origin,
                     int64_t out_width, float *grad_in, double *grad_offsets,
                     void *workspace, size_t workspace_bytes,
                     hipStream_t stream);

/* dsk_backward_f32 for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no workspace argument; the shear gradient's partial sums go
 * to a library-owned device array of 1 MiB (131072 doubles), one per
 * device, held until the process ends.  It needs
 * dsk_shear_grad_workspace_bytes(d) <= 1048576, i.e.
 * planes * ceil(rows / clamp(8192 / cols, 1, rows)) <= 131072 (the
 * 256 x 512 x 1024 stack needs 16384); beyond that it returns DSK_ESHAPE
 * and enqueues nothing.  The array is looked up once per device (on the
 * first call with grad_offsets set, with that device current) and never
 * needs clearing: every partial is written before it is read.  Calls on one
 * device share its array, so calls that may overlap on one device (two
 * streams, two threads) race: serialise them, or use dsk_backward_f32 with
 * a workspace per stream.  Arguments, outputs and errors otherwise as
 * dsk_backward_f32; results are bitwise identical to it.  Calls no
 * hipMalloc, hipFree or allocating routine. */
int dsk_backward_f32_noalloc(const float *in, const float *grad_vol,
                             dsk_dims d, const double *offsets_dev,
                             int64_t origin, int64_t out_width,
                             float *grad_in, double *grad_offsets,
                             hipStream_t stream);

/* ---------------------------------------------------------------------
 * Ragged batches: many uint16 stacks of different sizes and geometries in
 * one graph launch.  The graph holds either one persistent kernel (one
 * workgroup per compute-unit slot walks a shared list of (stack, row,
 * column-tile) items: no per-launch tails, best for many small stacks) or
 * one plain paced launch per job (each job's wavefronts keep to one
 * schedule: best for large stacks), in the default shape or in each job
 * frame's tuned shape, whichever the autotuner measures faster.  Each job's outputs are bitwise identical to its own
 * dsk_deskew_offsets_u16 / dsk_deskew_u16 call in either mode.
 * ------------------------------------------------------------------- */
enum {
    DSK_BATCH_PERSISTENT = 0,   /* one persistent kernel over all jobs */
    DSK_BATCH_PER_JOB = 1,      /* one plain launch per job, default shape */
    DSK_BATCH_PER_JOB_TUNED = 2 /* one plain launch per job, in the shape
                                   dsk_deskew_autotune picks for its frame */
};

typedef struct {
    const uint16_t *in;         /* device stack [planes][rows][cols] */
    dsk_dims dims;
    const double *offsets_dev;  /* device offsets, or NULL: o[n] = n*shift_px */
    double shift_px;
    int64_t origin;             /* b */
    int64_t out_width;          /* W (> 0) */
    float *vol, *psum, *pmax;   /* device outputs, each may be NULL */
} dsk_job;

typedef struct dsk_batch dsk_batch;

/* Build a batch: validates the jobs, uploads the job table (device memory
 * owned by the batch), picks the execution (tune != NULL: the persistent
 * kernel in that shape; NULL: time the persistent kernel's candidate shapes
 * and the two per-job modes on `stream` -- which runs the jobs, so outputs
 * are then already written; the tuned per-job mode first tunes each job's
 * frame with dsk_deskew_autotune -- and keep the fastest, remembered per
 * batch shape class in the DSK_TUNE_CACHE file when that variable is set),
 * and captures the launch in a HIP graph.  Host call; allocates and
 * synchronises `stream`. */
int dsk_batch_create(const dsk_job *jobs, int n_jobs, const dsk_tune *tune,
                     hipStream_t stream, dsk_batch **out);

/* Replay the captured graph on `stream` (asynchronous). */
int dsk_batch_launch(dsk_batch *batch, hipStream_t stream);

/* The same launches directly, without the graph. */
int dsk_batch_launch_direct(dsk_batch *batch, hipStream_t stream);

/* The persistent kernel's launch shape, and the autotuner's best time (ms,
 * 0 when the shape was given). */
int dsk_batch_get_tune(const dsk_batch *batch, dsk_tune *tune, double *ms);

/* The execution mode the batch uses (DSK_BATCH_PERSISTENT,
 * DSK_BATCH_PER_JOB or DSK_BATCH_PER_JOB_TUNED) into *mode (host). */
int dsk_batch_get_mode(const dsk_batch *batch, int *mode);

int dsk_batch_destroy(dsk_batch *batch);

/* Bytes of device job table dsk_jobs_launch needs for n_jobs jobs. */
size_t dsk_jobs_table_bytes(int n_jobs);

/* One persistent launch over jobs given per call (the serving path).
 * table_host: host buffer of dsk_jobs_table_bytes(n_jobs) bytes, ideally
 * pinned; it is encoded here and copied to table_dev with hipMemcpyAsync on
 * `stream`, so it must stay unchanged until that copy completes (record an
 * event).  table_dev: device buffer of the same size.  tune NULL: the
 * library default, paced only when every job has one frame (dims and
 * out_width), since pacing helps wavefronts that move in lockstep and
 * holds back a grid whose tiles belong to stacks of different sizes. */
int dsk_jobs_launch(const dsk_job *jobs, int n_jobs, void *table_host,
                    void *table_dev, size_t table_bytes, const dsk_tune *tune,
                    hipStream_t stream);

/* ---------------------------------------------------------------------
 * Rolling update (methods section, rolling update mode; Fig. 4a): for dim
 * samples the displayed projection is refreshed after every camera image
 * instead of once per stack.  State (all DEVICE, caller-owned):
 *   vol    [planes][rows][width] float32 -- the current deskewed images;
 *   tree   dsk_rolling_tree_bytes(d, width) bytes -- a max-tree over images
 *          (NULL allowed when planes == 1);
 *   sum64  [rows][width] double -- the running FP64 sum;
 *   psum, pmax [rows][width] float32 -- the displayed projections.
 * dsk_rolling_reset zeroes all of it (an empty stack: every image 0).
 * dsk_rolling_update_u16 remaps raw image n ([rows][cols] uint16, DEVICE)
 * at offset o[n] (offsets_dev, or n * shift_px when NULL) into leaf n,
 * adds (new - old) to sum64 and refreshes the maximum along the tree; psum
 * and pmax then equal the projections of the stack made of the latest image
 * at every index (pmax bitwise; psum equal to a forward pass when each
 * image has been written once, in order).  One kernel per image.
 * ------------------------------------------------------------------- */
size_t dsk_rolling_tree_bytes(dsk_dims d, int64_t out_width);

int dsk_rolling_reset(dsk_dims d, int64_t out_width, float *vol, float *tree,
                      double *sum64, float *psum, float *pmax,
                      hipStream_t stream);

int dsk_rolling_update_u16(const uint16_t *plane, int32_t n, dsk_dims d,
                           const double *offsets_dev, double shift_px,
                           int64_t origin, int64_t out_width, float *vol,
                           float *tree, double *sum64, float *psum,
                           float *pmax, hipStream_t stream);

/* ---------------------------------------------------------------------
 * Shear-warp rotated view (Fig. 3; shear-warp paragraph of "Physical
 * principles"): remapping with a changed per-image shift s' and stretching
 * the projection along the column axis renders the projection seen from
 * another direction.  For a view at angle theta to the optical axis, in the
 * plane of the scan axis and the optical axis (theta = alpha is the plain
 * deskew, theta = 0 looks straight down the optical axis):
 *     s'      = z cos(theta) / (p cos(theta - alpha))   pixels per image
 *     stretch = cos(theta - alpha)
 * A point at scan position Y and height Z lands in view column
 * (Y cos(theta) + Z sin(theta)) / p - stretch * b.  Requires
 * |theta - alpha| < 90 degrees.
 * ------------------------------------------------------------------- */

/* Host-only geometry of the view: shift per image, stretch, the remap frame
 * (proj_width, origin) of the shifted images and the view width
 * floor((proj_width - 1) * stretch) + 1.  Any output pointer may be NULL. */
int dsk_view_plan(dsk_dims d, dsk_geom g, double theta_deg, double *shear_px,
                  double *stretch, int64_t *proj_width, int64_t *origin,
                  int64_t *view_width);

/* Workspace bytes dsk_view_u16 needs: the two [rows][proj_width] float32
 * projections of the shifted images. */
size_t dsk_view_workspace_bytes(dsk_dims d, int64_t proj_width);

/* The view of a uint16 stack: projections of the stack remapped with
 * offsets n * shear_px in the frame (origin, proj_width), then stretched:
 * view column j samples the projection row at x' = j / stretch by linear
 * interpolation, zero outside [0, proj_width).  vsum / vmax are
 * [rows][view_width] float32 (either may be NULL, not both).  workspace:
 * DEVICE, 16-byte aligned, at least dsk_view_workspace_bytes bytes, owned
 * by the caller and overwritten. */
int dsk_view_u16(const uint16_t *in, dsk_dims d, double shear_px,
                 double stretch, int64_t origin, int64_t proj_width,
                 float *vsum, float *vmax, int64_t view_width,
                 void *workspace, size_t workspace_bytes, hipStream_t stream);

/* Columns of a row of width_in stretched by `stretch` (> 0): every output
 * column up to the last input column's position,
 * floor((width_in - 1) * stretch) + 1, into *width_out (host).  Host only;
 * dsk_view_plan's view width is this of the projection width. */
int dsk_stretch_width(int64_t width_in, double stretch, int64_t *width_out);

/* The stretch alone: out[r][j] = linear interpolation of proj[r][.] at
 * j / stretch (zero outside [0, width_in)); proj [rows][width_in], out
 * [rows][width_out], both DEVICE float32. */
int dsk_stretch_f32(const float *proj, int64_t rows, int64_t width_in,
                    double stretch, float *out, int64_t width_out,
                    hipStream_t stream);

/* ---------------------------------------------------------------------
 * Real-space (affine) deskew ("Physical principles", remap paragraph: the
 * affine transformation of the whole stack that the remap is contrasted
 * with).  The stack is resampled onto a Cartesian grid of the sample:
 * X = x p (rows), Z = z p sin(alpha) (raw columns), Y = Y0 + y dy (scan
 * axis, step dy chosen by the caller).  Raw image n, column z images the
 * scan coordinate n * step + z p cos(alpha), so voxel (y, x, z) lies on raw
 * column z between images floor(u) and floor(u) + 1 with
 *     u = (Y0 + y dy - z p cos(alpha)) / step
 * and is their linear interpolation, zero outside the stack.  Output vol
 * [ny][rows][cols] float32.
 * ------------------------------------------------------------------- */

/* Host-only grid of the stack: Y0 = the smallest scan coordinate of the
 * stack's corners, ny = floor((largest - Y0) / dy) + 1.  DSK_EINVAL for a
 * zero step or dy <= 0. */
int dsk_affine_plan(dsk_dims d, dsk_geom g, double dy_um, double *y0_um,
                    int64_t *ny);

/* Resample a uint16 stack (DEVICE) into vol (DEVICE, [ny][rows][cols]
 * float32) on the grid (y0_um, dy_um, ny), e.g. from dsk_affine_plan. */
int dsk_affine_u16(const uint16_t *in, dsk_dims d, dsk_geom g, double dy_um,
                   double y0_um, int64_t ny, float *vol, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* DESKEW_H */
