/*
 * synim.h - C ABI of the MI355X (gfx950) synthetic interaction-matrix library.
 *
 * The library forms synthetic Shack-Hartmann interaction-matrix (IM) columns:
 * every deformable-mirror influence function (IF) is resampled onto the WFS
 * grid by ONE composite affine map with a single bilinear interpolation
 * (SynIM paper, Sec. 2.1 "Geometric Mapping and Single-Step Interpolation"),
 * then turned into per-subaperture x/y slopes by central finite differences
 * at every pupil pixel and a mean over each subaperture on the exactly aligned
 * grid (Sec. 2.2 "Slope Computation").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Coordinates   pixel (row y, column x) has its centre at integer (x, y); a
 *               grid of n pixels has its centre at (n-1)/2.
 * Inverse map   synim_affine holds p_s = A p_o + b: WFS (output) pixel ->
 *               IF (source) pixel, x first.  IF samples outside the IF grid
 *               are zero (the paper leaves this open; zero fill is the
 *               reading taken).  The fused builds count the samples the
 *               slopes read whose source point leaves the grid; the strict
 *               check synim_plan_oob / synim_batch_oob returns SYNIM_E_OOB
 *               when that count is non-zero.
 * Subapertures  the WFS grid is (n_sub_y*p) x (n_sub_x*p) pixels; subaperture
 *               (u, v) covers columns u*p..u*p+p-1, rows v*p..v*p+p-1 and has
 *               row-major id k = v*n_sub_x + u.  valid_idx lists the ids of the
 *               valid subapertures, strictly ascending; N = n_valid.
 * Slopes        for valid subaperture k with n_k pupil pixels,
 *               s_x = sum_{P=1} (phi[y][x+1] - phi[y][x-1]) / (2 n_k), s_y
 *               likewise; units: phase per WFS pixel.
 * IM layout     actuator-major: im[a*2N + i] = s_x of valid subaperture i,
 *               im[a*2N + N + i] = s_y (x block then y block).  This is the
 *               transpose of the paper's 2N x N_modes matrix.
 * Memory        every array argument is a DEVICE pointer unless marked
 *               (host); descriptors (synim_affine, synim_wfs, ...) are host
 *               structs read during the call.  The caller owns all memory.
 *               Entry points taking a workspace never allocate; size it
 *               with the matching *_workspace query.
 * Streams       work is enqueued on the hipStream_t passed as `stream` (NULL =
 *               default stream); calls return after enqueueing.  Argument
 *               errors are reported synchronously; device-side faults surface
 *               as SYNIM_E_HIP from a later synchronising call.
 * Threads       all entry points are re-entrant; the autotune cache is guarded.
 */
#ifndef SYNIM_H
#define SYNIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SYNIM_OK = 0,
  SYNIM_E_NULL = -1,          /* a required pointer is NULL                      */
  SYNIM_E_SHAPE = -2,         /* inconsistent or unsupported sizes               */
  SYNIM_E_PARAM = -3,         /* invalid parameter value (e.g. magnification 0)  */
  SYNIM_E_OOB = -4,           /* strict check: samples fell outside the IF grid  */
  SYNIM_E_WORKSPACE = -5,     /* workspace missing or too small                  */
  SYNIM_E_HIP = -6,           /* a HIP runtime call failed                       */
  SYNIM_E_NOT_CONVERGED = -7, /* Gauss-Newton stopped without converging        */
  SYNIM_E_UNSUPPORTED = -8    /* no kernel variant for this geometry             */
} synim_status;

/* Human-readable name of a status code (static string). */
const char* synim_status_str(int status);
/* Library version, major*10000 + minor*100 + patch. */
int synim_version(void);

/* Inverse affine map p_s = A p_o + b (see Conventions). */
typedef struct {
  double A[2][2];
  double b[2];
} synim_affine;

/* Plain misregistration of a DM seen by a WFS (forward map, about the grid
 * centres c_s, c_o):  p_o = c_o + t + (mag/kappa) R(rot) (p_s - c_s),
 * R(phi) = [[cos, -sin], [sin, cos]] on (x, y); t = (shift_x, shift_y) in WFS px. */
typedef struct {
  double shift_x, shift_y;
  double rot;   /* radians */
  double mag;
} synim_misreg;

/* Composite DM -> WFS geometry (Sec. 2.1: the DM transform, the LGS
 * perspective at the DM altitude and the WFS transform multiplied into one
 * matrix).  Forward chain, each part about its grid centre:
 *   DM placement   v = dm_mag R(dm_rot) u + dm_shift          (DM px)
 *   LGS footprint  w = (v - footprint) / (kappa * cone_scale)  (WFS px)
 *   WFS            p_o - c_o = diag(wfs_mag_x, wfs_mag_y) R(wfs_rot) w + wfs_shift
 * cone_scale = 1 - h/H_LGS; footprint = h*alpha / DM pixel size. */
typedef struct {
  double dm_shift_x, dm_shift_y, dm_rot, dm_mag;
  double cone_scale, footprint_x, footprint_y;
  double wfs_shift_x, wfs_shift_y, wfs_rot, wfs_mag_x, wfs_mag_y;
  double kappa;   /* DM pixels per WFS pixel */
} synim_geometry;

/* Shack-Hartmann WFS description. */
typedef struct {
  int32_t n_sub_x, n_sub_y;   /* subapertures per row / column                */
  int32_t p;                  /* pixels per subaperture side                  */
  int32_t n_valid;            /* N, number of valid subapertures (>= 1)       */
  const int32_t* valid_idx;   /* device [N], ascending row-major ids          */
  const uint8_t* pupil;       /* device [n_sub_y*p][n_sub_x*p], 0/1           */
} synim_wfs;

/* ---------------------------------------------------------------- geometry */

/* Inverse map of a plain misregistration (Sec. 2.1), and optionally the four
 * derivative maps d p_s / d theta_j = dA[j].A p_o + dA[j].b for theta =
 * (shift_x, shift_y, rot, mag).  Grid sizes are those of the IF (in) and WFS
 * (out) grids; kappa = IF pixels per WFS pixel.
 * A (host, out) required; dA (host, out, 4 entries) may be NULL.
 * Errors: SYNIM_E_NULL, SYNIM_E_PARAM (mag or kappa <= 0, sizes < 1). */
int synim_affine_from_misreg(const synim_misreg* theta, int H_in, int W_in, int H_out, int W_out,
                             double kappa, synim_affine* A, synim_affine* dA);

/* Inverse map of a composite geometry (Sec. 2.1, LGS cone effect and
 * off-axis footprint, WFS anamorphosis), composed and inverted in FP64 on the
 * host.  Errors: SYNIM_E_NULL, SYNIM_E_PARAM (singular chain). */
int synim_affine_from_geometry(const synim_geometry* g, int H_in, int W_in, int H_out, int W_out,
                               synim_affine* A);

/* -------------------------------------------------------- standalone steps */

/* Bilinear resampling of n IFs onto the WFS grid with a `halo`-pixel border
 * (Sec. 2.1 single interpolation):
 *   out[i][y+halo][x+halo] = bilinear(ifs[i], A (x, y) + b)
 * for x in [-halo, W_out+halo), y in [-halo, H_out+halo).
 *   ifs   device float32 [n][H_in][W_in], row-major
 *   out   device float32 [n][H_out+2*halo][W_out+2*halo]
 *   oob_count  device int32[1] or NULL: incremented (atomically) by the number
 *         of output pixels of one IF whose source point lies outside
 *         [0, W_in-1] x [0, H_in-1]; the caller zeroes it beforehand.
 * Errors: SYNIM_E_NULL, SYNIM_E_SHAPE (n, sizes < 1, halo < 0 or > 8),
 *         SYNIM_E_HIP. */
int synim_affine_warp(const float* ifs, int n, int H_in, int W_in, const synim_affine* A,
                      int H_out, int W_out, int halo, float* out, int32_t* oob_count, void* stream);

/* Slopes of n haloed phase maps (Sec. 2.2 central differences + subaperture
 * means).
 *   phase  device float32 [n][H+2][W+2] with pixel (x, y) at [y+1][x+1],
 *          H = n_sub_y*p, W = n_sub_x*p
 *   slopes device float32 [n][2N]
 * A listed subaperture with no pupil pixel reads 0 in both components.
 * Errors: SYNIM_E_NULL, SYNIM_E_SHAPE (also p > 256), SYNIM_E_HIP. */
int synim_sa_slopes(const float* phase, int n, const synim_wfs* wfs, float* slopes, void* stream);

/* ------------------------------------------------------------ fused build */

/* Workspace bytes for synim_im_build / synim_im_jacobian / synim_im_vjp on
 * this WFS and map.  `planes` = 1 for the IM, 5 for IM + 4 Jacobian planes.
 * Errors: SYNIM_E_NULL, SYNIM_E_SHAPE, SYNIM_E_UNSUPPORTED (map too strongly
 * magnified for every kernel variant). */
int synim_im_workspace(const synim_wfs* wfs, const synim_affine* A, int planes, size_t* bytes);

/* Interaction matrix of n_act IFs (Sec. 2.1 + 2.2, fused): for every IF the
 * composite-map bilinear resampling, the central differences at pupil pixels
 * and the subaperture means, in one pass over the IF stack.
 *   ifs  device float32 [n_act][H_in][W_in]
 *   im   device float32 [n_act][2N] (IM layout above)
 *   ws   device workspace of at least synim_im_workspace(.., planes=1) bytes
 * The geometry is folded, per valid subaperture, into one dense weight patch
 * computed in FP64 on the device; the IF stack is then streamed once.
 * Errors: SYNIM_E_NULL, SYNIM_E_SHAPE, SYNIM_E_WORKSPACE, SYNIM_E_UNSUPPORTED,
 *         SYNIM_E_HIP. */
int synim_im_build(const float* ifs, int n_act, int H_in, int W_in, const synim_affine* A,
                   const synim_wfs* wfs, float* im, void* ws, size_t ws_bytes, void* stream);

/* Interaction matrix with the telescoping-sum slope engine, the G-tilt
 * comparator of Sec. 2.2: the mean gradient over the pupil pixels of each
 * valid subaperture k written as boundary differences,
 *   s_x[k] = (1/n_k) sum over the rows of k, over the runs [xa, xb] of pupil
 *            pixels of k on the row, of phi(xb + 1/2, y) - phi(xa - 1/2, y),
 * and s_y likewise over columns, where every boundary value phi is ONE
 * bilinear sample of the IF at the boundary point itself through the
 * composite map (zero outside the IF grid).  Same arguments, layout and
 * workspace (synim_im_workspace, planes = 1) as synim_im_build; the IF stack
 * is streamed once through the same kernel.  The out-of-grid count of the
 * plan is not kept (it is defined on the central-difference samples).
 * Errors: as synim_im_build. */
int synim_im_build_tsum(const float* ifs, int n_act, int H_in, int W_in, const synim_affine* A,
                        const synim_wfs* wfs, float* im, void* ws, size_t ws_bytes, void* stream);

/* Interaction matrix of a pre-masked IF stack with edge repair (Sec. 2.3).
 * The IFs were multiplied by a DM-side mask M on the IF grid, so the single
 * bilinear interpolation softens the mask edge and the warped phase collapses
 * towards zero there.  For every haloed WFS sample q (x in [-1, W], y in
 * [-1, H]) the warped mask m(q) = bilinear(M, A q + b) gives:
 *   1. the strict core S = {m >= threshold} (the paper uses 0.999999), whose
 *      phase is kept; every other sample is cleared;
 *   2. the edge ring E = dilate(S) \ S, dilation by the 4-neighbour cross;
 *   3. for e in E and each direction d in {+x, -x, +y, -y} with P1 = e + d in
 *      S: the estimate 2 phi(P1) - phi(P2) if P2 = e + 2d is in S too, else
 *      phi(P1); phi(e) = the mean of the estimates of the valid directions.
 * Samples outside the haloed window count as outside S.  The slopes of the
 * repaired phase then follow as in synim_im_build.  The repair is linear in
 * the phase for a fixed mask, so it is folded into the plan's FP64 weights
 * and the IF stack is still streamed once.
 *   dm_mask   device uint8 [H_in][W_in], 0/1 (M)
 *   threshold in (0, 1]
 *   ws        device workspace of at least synim_im_repaired_workspace bytes
 * Errors: SYNIM_E_NULL, SYNIM_E_SHAPE, SYNIM_E_PARAM (threshold),
 *         SYNIM_E_WORKSPACE, SYNIM_E_UNSUPPORTED, SYNIM_E_HIP. */
int synim_im_repaired_workspace(const synim_wfs* wfs, const synim_affine* A, size_t* bytes);
int synim_im_build_repaired(const float* ifs, int n_act, int H_in, int W_in,
                            const uint8_t* dm_mask, double threshold, const synim_affine* A,
                            const synim_wfs* wfs, float* im, void* ws, size_t ws_bytes,
                            void* stream);

/* Largest plan synim_im_build_noalloc holds: 16 MiB (the 80x80-subaperture
 * ELT build under a +-1 deg map needs 5.1 MB). */
#define SYNIM_NOALLOC_WS_BYTES (16u << 20)

/* synim_im_build for callers that cannot allocate device memory or pass a
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, result and kernels as
 * synim_im_build, without ws / ws_bytes: the plan lives in one fixed device
 * array of SYNIM_NOALLOC_WS_BYTES per GPU, held from the library's first use
 * on that GPU until the process ends.  Allocates nothing (no hipMalloc, no
 * allocating library call).  Every call on one GPU shares that array and
 * overwrites it: calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller; the array's contents
 * after a call are the last call's plan (status words at its start, see
 * synim_plan_status, not reachable through this entry point).
 * Errors: as synim_im_build; SYNIM_E_WORKSPACE when the geometry's plan
 * exceeds SYNIM_NOALLOC_WS_BYTES. */
int synim_im_build_noalloc(const float* ifs, int n_act, int H_in, int W_in, const synim_affine* A,
                           const synim_wfs* wfs, float* im, void* stream);

/* IM and its Jacobian with respect to theta_j (j = 0..3) for the derivative
 * maps dA (from synim_affine_from_misreg):
 *   d phi / d theta_j = grad bilinear(F, p_s) . (dA[j].A p_o + dA[j].b)
 * with the floor-cell (right-continuous) bilinear gradient, then the slope
 * step.  im may be NULL; dim is device float32 [4][n_act][2N].
 * Workspace: synim_im_workspace(.., planes=5). */
int synim_im_jacobian(const float* ifs, int n_act, int H_in, int W_in, const synim_affine* A,
                      const synim_affine* dA, const synim_wfs* wfs, float* im, float* dim,
                      void* ws, size_t ws_bytes, void* stream);

/* Vector-Jacobian product of the IM with respect to theta:
 *   grad_theta[j] = sum_{a,r} grad_im[a][r] * dIM/dtheta_j[a][r]
 * computed without materialising the Jacobian.
 *   grad_im    device float32 [n_act][2N]
 *   grad_theta device float64 [4] (overwritten)
 * Workspace: synim_im_workspace(.., planes=5) + synim_vjp_extra_workspace(). */
int synim_im_vjp(const float* ifs, int n_act, int H_in, int W_in, const synim_affine* A,
                 const synim_affine* dA, const synim_wfs* wfs, const float* grad_im,
                 double* grad_theta, void* ws, size_t ws_bytes, void* stream);

/* --------------------------------------------------- plan / apply split
 * synim_im_build = synim_im_plan + synim_im_apply(plane 0).  Splitting them
 * lets a caller fold the geometry once and stream several IF stacks (or time
 * the streaming kernel alone).  The plan lives in `ws`; apply must be called
 * with the same wfs, A and `planes` as the plan. */

/* Fold the geometry into per-subaperture weight patches in `ws` (FP64 on the
 * device).  planes = 1 (IM) or 5 (IM + 4 Jacobian planes, dA required).
 * H_in, W_in: the IF grid the plan will stream, used only for the
 * out-of-grid sample count (synim_plan_oob); both 0 leave it uncounted.
 * Errors: SYNIM_E_NULL, SYNIM_E_SHAPE, SYNIM_E_PARAM, SYNIM_E_WORKSPACE,
 *         SYNIM_E_UNSUPPORTED, SYNIM_E_HIP. */
int synim_im_plan(const synim_wfs* wfs, const synim_affine* A, const synim_affine* dA, int planes,
                  int H_in, int W_in, void* ws, size_t ws_bytes, void* stream);

/* Stream n_act IFs through plane `plane` (0 = IM, 1..4 = d/dtheta_j) of a plan
 * built by synim_im_plan; out is device float32 [n_act][2N]. */
int synim_im_apply(const float* ifs, int n_act, int H_in, int W_in, const synim_affine* A,
                   const synim_wfs* wfs, int planes, int plane, float* out, const void* ws,
                   size_t ws_bytes, void* stream);

/* ------------------------------------------------------------- autotuner */

/* Time up to max_candidates (variant x tile shape) configurations of the
 * streaming kernel for this geometry on the caller's IF stack and record the
 * fastest in a process-wide cache keyed by the WFS shape and the map's linear
 * part; later plan/apply/build calls with that key use it.  im and ws are
 * overwritten (ws sized by synim_im_workspace, which already covers every
 * candidate).  times_ms (host, [max_candidates]) and n_tried (host) may be
 * NULL.  Synchronises `stream`.  Errors: as synim_im_build. */
int synim_im_autotune(const float* ifs, int n_act, int H_in, int W_in, const synim_affine* A,
                      const synim_wfs* wfs, float* im, void* ws, size_t ws_bytes,
                      int max_candidates, float* times_ms, int* n_tried, void* stream);

/* Ints in one kernel configuration record. */
#define SYNIM_CONFIG_INTS 10

/* The configuration plan/apply would use now: out (host,
 * [SYNIM_CONFIG_INTS]) = block size, lanes per subaperture, patch rows,
 * patch columns, tile width and height in subapertures, pipeline stages,
 * schedule, 16-byte DMA instructions per wave and stage, most actuators one
 * stage holds.  Schedule: 0 = short actuator chunks dealt round-robin to the
 * XCDs; 1 = one chunk per XCD with every tile of it running at once, one
 * tile per workgroup; E >= 2 = as 1, with the tiles of an XCD kept within
 * one block of E actuators of each other. */
int synim_im_config(const synim_wfs* wfs, const synim_affine* A, int* out);

/* The candidate configurations synim_im_autotune tries, in its order (cost
 * model first): out (host, [max_out][SYNIM_CONFIG_INTS]) as
 * synim_im_config; *n_out (host) receives the count written (at most 256). */
int synim_im_candidates(const synim_wfs* wfs, const synim_affine* A, int* out, int max_out,
                        int* n_out);

/* Pin the configuration later plan/apply/build calls use for this geometry
 * (as if the autotuner had picked it): config (host, [SYNIM_CONFIG_INTS]) as
 * synim_im_config, one of synim_im_candidates.  Errors: SYNIM_E_NULL,
 * SYNIM_E_SHAPE, SYNIM_E_UNSUPPORTED (not a candidate for this geometry). */
int synim_im_set_config(const synim_wfs* wfs, const synim_affine* A, const int* config);

/* Forget every autotuned configuration. */
void synim_autotune_clear(void);

/* The autotune cache as a flat int32 record, to keep across processes (the
 * configurations measured fastest, keyed by geometry; the record is tied to
 * this library's kernel-variant table).  out (host, [cap]) may be NULL:
 * *n_ints (host) then receives the length needed.  Errors: SYNIM_E_NULL,
 * SYNIM_E_SHAPE (cap too small). */
int synim_autotune_export(int32_t* out, int cap, int* n_ints);

/* Merge a record written by synim_autotune_export into the cache (entries
 * replace those of the same geometry).  A configuration that is no longer a
 * candidate of its geometry is ignored when looked up.  Errors: SYNIM_E_NULL,
 * SYNIM_E_PARAM (not such a record, or a malformed entry), SYNIM_E_SHAPE
 * (length), SYNIM_E_UNSUPPORTED (written by a library with another variant
 * table), SYNIM_E_WORKSPACE (cache full: 256 geometries). */
int synim_autotune_import(const int32_t* in, int n_ints);

/* Device status word of the last plan built in `ws`: bit 0 a weight patch was
 * too small for the map, bit 1 a tile bounding box overflowed (that tile's
 * slopes are not written), bit 2 a valid subaperture has no pupil pixel (its
 * slopes are 0).  0 means the plan is complete.  Copies 4 bytes to host_out
 * and synchronises `stream`. */
int synim_plan_status(const void* ws, int* host_out, void* stream);

/* Strict check of the out-of-grid reading (Sec. 2.1 leaves interpolation
 * outside the IF grid open; the library zero-fills).  *host_count (host)
 * receives the number of (valid subaperture, sample) pairs of the last plan
 * built in `ws` (by synim_im_build, _jacobian, _vjp, _autotune, or
 * synim_im_plan with a grid size) whose sample has a non-zero
 * central-difference coefficient in that subaperture and a source point
 * outside [0, W_in-1] x [0, H_in-1]; a sample two subapertures read counts
 * twice.  Returns SYNIM_E_OOB when the count is non-zero (the plan and its
 * IM are still complete, with those taps read as zero), SYNIM_OK otherwise.
 * Synchronises `stream`.  Errors: SYNIM_E_NULL, SYNIM_E_HIP. */
int synim_plan_oob(const void* ws, int64_t* host_count, void* stream);

/* ------------------------------------------------------- multi-pair batch
 * Every (WFS, DM) pair of a multi-WFS system (e.g. 6 LGS WFS x 3 DMs) built in
 * one persistent launch (one per patch size for a batch split as described
 * below) - the multi-WFS batch of Sec. 4.2, where each DM's IF
 * stack is fetched once for all the WFS that see it.  For IM batches
 * (planes = 1) the subapertures of every WFS of a DM are packed, in the order
 * of the IF-grid cells their weight patches start in, into full tiles whose
 * staged box fits the stage buffers, and one staging of a tile's IF rows
 * serves every WFS in it.  The tiles' staged boxes overlap by the patch halo,
 * so HBM still reads a DM's stack more than once (about 3 times for the
 * 6 x 3 MCAO system, against 7.7 times with one staging per pair; how many of
 * the repeats the L2 absorbs depends on timing).  Pairs may
 * have their own map (cone effect, off-axis footprint), WFS (uneven
 * valid-subaperture counts) and DM (uneven actuator counts).  The maps live in
 * device memory, so a graph captured by synim_batch_run_graph replays after
 * synim_batch_set_maps without re-capture.  The kernel configuration is chosen
 * at creation from the initial maps; synim_batch_set_maps checks later maps
 * against it.
 *
 * Split by patch size: the one kernel variant of a launch runs, on every
 * lane, the patch of the batch's most demanding pair (the WFS clocking and
 * the cone scale set each pair's patch).  Where grouping the pairs by their
 * own smallest patch cuts those products by at least 15% (weighted by
 * subapertures x actuators), a shared-tile IM batch is split into parts, one
 * per patch size, each with its own variant, tiles and launch, run one after
 * the other on the caller's stream (synim_batch_parts gives their number);
 * each part then stages a DM's rows for its own pairs. */

typedef struct {
  const float* ifs;           /* device [n_act][H_in][W_in]                     */
  int32_t n_act, H_in, W_in;
} synim_dm;

typedef struct {
  int32_t wfs, dm;            /* indices into the WFS and DM arrays             */
  synim_affine A;             /* initial inverse map of the pair                */
  float* im;                  /* device [dm.n_act][2 N(wfs)], IM layout above   */
} synim_pair;

typedef struct synim_batch synim_batch;   /* opaque, owned by the library */

/* Workspace bytes for synim_batch_create (covers every kernel variant the
 * batch autotuner may pick). */
int synim_batch_workspace(const synim_wfs* wfs, int n_wfs, const synim_dm* dms, int n_dm,
                          const synim_pair* pairs, int n_pairs, size_t* bytes);

/* Build the batch's tables in `ws` (device, caller-owned, must outlive the
 * batch) and upload the initial maps; *out receives the handle.  The WFS
 * descriptors, DM stacks and outputs are borrowed.  Synchronises `stream`.
 * Allocates only host-side bookkeeping and a small pinned staging buffer. */
int synim_batch_create(const synim_wfs* wfs, int n_wfs, const synim_dm* dms, int n_dm,
                       const synim_pair* pairs, int n_pairs, void* ws, size_t ws_bytes,
                       void* stream, synim_batch** out);

/* Upload new maps (host [n_pairs], pair order of creation) on `stream`.
 * Each map is checked on the host against the kernel configuration bound at
 * creation: a map whose weight patches outgrow the bound kernel variant
 * returns SYNIM_E_UNSUPPORTED (create a new batch); one whose tiles outgrow
 * their staged-box bound re-binds the pair tables for the new maps (a
 * captured graph is captured again on the next synim_batch_run_graph; the
 * workspace must hold the new layout, else SYNIM_E_WORKSPACE).  Synchronises
 * with the previous upload only.  Errors: SYNIM_E_NULL, SYNIM_E_PARAM
 * (singular map), SYNIM_E_UNSUPPORTED, SYNIM_E_WORKSPACE, SYNIM_E_HIP. */
int synim_batch_set_maps(synim_batch* b, const synim_affine* maps, void* stream);

/* Enqueue the plans and the single stream launch of every pair (one launch
 * per part of a split batch). */
int synim_batch_run(synim_batch* b, void* stream);

/* As synim_batch_run, through a hipGraph captured on the first call (stream
 * must not be NULL) and replayed afterwards (one graph per part). */
int synim_batch_run_graph(synim_batch* b, void* stream);

/* OR of the pairs' plan status words (see synim_plan_status); synchronises. */
int synim_batch_status(synim_batch* b, int* host_out, void* stream);

/* Strict check of the last run (see synim_plan_oob): *host_count (host) =
 * out-of-grid samples summed over the pairs; SYNIM_E_OOB when non-zero.
 * Synchronises `stream`. */
int synim_batch_oob(synim_batch* b, int64_t* host_count, void* stream);

/* Time up to max_variants kernel variants on the batch (each pair with its
 * best tile shape for that variant) and keep the fastest; drops a captured
 * graph.  times_ms (host) and n_tried (host) may be NULL.  A split batch tunes
 * each part on its own; times_ms[r] is then the sum of the parts' r-th
 * variants (a part with fewer adds its last).  Synchronises. */
int synim_batch_autotune(synim_batch* b, int max_variants, float* times_ms, int* n_tried,
                         void* stream);

/* out6 (host) = block size, lanes per subaperture, pipeline stages, grid,
 * 16-byte DMA instructions per wave and stage, most actuators one stage
 * holds; of the first part for a batch split by patch size. */
int synim_batch_config(const synim_batch* b, int* out6);

/* *n_parts (host) = the launches one run of the batch makes: 1, or the number
 * of patch-size parts of a split batch (see synim_batch_create). */
int synim_batch_parts(const synim_batch* b, int* n_parts);

/* Release the handle (the workspace stays the caller's). */
void synim_batch_destroy(synim_batch* b);

/* ------------------------------------------------ tomographic projection
 * P_opt = (P_DM^T P_DM + lambda I)^-1 P_DM^T P_Layer (Sec. 2.5, after Fusco et
 * al.): the DM influence functions and the virtual layers' modes, each on its
 * own grid at its conjugate altitude, sampled over the telescope pupil along
 * every optimisation direction.  Pupil point r (metres from the axis, pupil
 * pixel p_s metres, grid centre at (n-1)/2) reads a component of altitude h
 * and pixel s at grid coordinate c + (r + h theta) / s by one bilinear
 * interpolation (zero outside the grid).  With a binning factor b, a row is a
 * b x b block of pupil pixels (kept if any pixel is in the mask): the mean of
 * the samples at its pupil pixels.  Rows run direction-major, blocks
 * row-major.  Everything is FP64; the products run on the FP64 matrix cores. */
typedef struct {
  const float* basis;          /* device [n][H][W] influence functions or modes */
  int32_t n, H, W;
  double altitude_m;           /* conjugate altitude (m)                        */
  double pixel_m;              /* grid pixel size (m)                            */
} synim_proj_component;

/* Rows of the projection matrices: kept blocks x n_dir (pupil host [Hp][Wp]). */
int synim_proj_rows(const uint8_t* pupil, int Hp, int Wp, int bin, int n_dir, int* n_rows);
/* Workspace bytes of synim_proj_opt (layers may be NULL for synim_proj_matrix). */
int synim_proj_workspace(const synim_proj_component* dms, int n_dm,
                         const synim_proj_component* layers, int n_layer, int n_dir,
                         const uint8_t* pupil, int Hp, int Wp, int bin, size_t* bytes);
/* The projection matrix of components comps (columns in component order),
 * stored transposed: Pt (device float64) [sum n][ld], Pt[col][row], ld >= rows.
 * dirs (host) [n_dir][2] radians; pupil (host) [Hp][Wp] 0/1.  Synchronises.
 * Errors: SYNIM_E_NULL, SYNIM_E_SHAPE (Hp, Wp not multiples of bin, ld),
 *         SYNIM_E_PARAM, SYNIM_E_WORKSPACE, SYNIM_E_HIP. */
int synim_proj_matrix(const synim_proj_component* comps, int n_comp, const double* dirs, int n_dir,
                      const uint8_t* pupil, int Hp, int Wp, double pupil_pixel_m, int bin,
                      double* Pt, long ld, void* ws, size_t ws_bytes, void* stream);
/* P_opt (device float64 [sum n_dm][sum n_layer], row-major).  lambda >= 0.
 * Synchronises.  Errors: as synim_proj_matrix; SYNIM_E_PARAM also when
 * P_DM^T P_DM + lambda I is not positive definite. */
int synim_proj_opt(const synim_proj_component* dms, int n_dm, const synim_proj_component* layers,
                   int n_layer, const double* dirs, int n_dir, const uint8_t* pupil, int Hp,
                   int Wp, double pupil_pixel_m, int bin, double lambda, double* popt, void* ws,
                   size_t ws_bytes, void* stream);
/* Building blocks (device float64, row-major):
 *   C[m][n] = alpha sum_k X(k, m) Y(k, n) + beta C[m][n], X(k, m) = X[k sxk + m sxm],
 *   Y(k, n) = Y[k syk + n syn] (any strides; FP64 MFMA tiles);
 *   lower Cholesky of the lower triangle of A [n][ld] in place (*status
 *   (device int) gets bit 0 when a pivot is not positive; zero it first);
 *   B [n][ldb] <- (L L^T)^-1 B for m right-hand sides. */
int synim_gemm_f64(int M, int N, int K, double alpha, const double* X, long sxk, long sxm,
                   const double* Y, long syk, long syn, double beta, double* C, long ldc,
                   void* stream);
int synim_potrf_f64(double* A, int n, long ld, int* status, void* stream);
int synim_potrs_f64(const double* L, int n, long ld, double* B, int m, long ldb, void* stream);

/* --------------------------------------------------- learned estimator
 * A small MLP x (n_in) -> h1 -> h2 -> n_out (ReLU after the hidden layers),
 * trained with an MSE loss and Adam, for the learned misregistration
 * estimate.  Parameters are one packed FP32 buffer
 *   W1 [h1][n_in], b1 [h1], W2 [h2][h1], b2 [h2], W3 [n_out][h2], b3 [n_out].
 * Inputs are compact: the non-zero inputs of the input layer lie in two column
 * segments, so x is [B][len0 + len1] and compact column c feeds input
 * seg0 + c (c < len0) or seg1 + c - len0; every other input is zero. */
typedef struct {
  int32_t n_in, h1, h2, n_out;
  int32_t seg0, len0, seg1, len1;
} synim_mlp;

/* Number of packed parameters (0 for an invalid description). */
size_t synim_mlp_param_count(const synim_mlp* net);
/* Floats of caller scratch needed for a batch of B (activations kept from the
 * forward pass for the backward pass). */
size_t synim_mlp_scratch_floats(const synim_mlp* net, int B);

/* y [B][n_out] = net(x [B][len0+len1]); scratch keeps the activations. */
int synim_mlp_forward(const synim_mlp* net, const float* params, const float* x, int B,
                      float* scratch, float* y, void* stream);

/* Gradients of mean((y - t)^2) after synim_mlp_forward on the same x and
 * scratch; grads is packed like params and fully overwritten (W1 columns
 * outside the segments get 0); loss (device float, nullable). */
int synim_mlp_backward(const synim_mlp* net, const float* params, const float* x, int B,
                       float* scratch, const float* y, const float* t, float* grads,
                       float* loss, void* stream);

/* One Adam step (bias-corrected, step >= 1) over n parameters, in place:
 *   m <- b1 m + (1-b1) g,  v <- b2 v + (1-b2) g^2,
 *   p <- p - lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).
 * The hyperparameters are double so that 1-b1, 1-b2 and the bias
 * corrections are exact before their single rounding to float.
 * Errors: SYNIM_E_NULL, SYNIM_E_PARAM (step < 1, lr <= 0, b outside [0, 1)). */
int synim_adam_step(float* params, const float* grads, float* m, float* v, size_t n, int step,
                    double lr, double beta1, double beta2, double eps, void* stream);

/* ---------------------------------------------- misregistration estimation
 * Online tracking regenerates IMs from misregistration estimates (Sec. 5).
 * theta = (shift_x px, shift_y px, rot rad, mag) is estimated from measured
 * slopes of n_probe probe phase maps (e.g. Zernike modes fitted by the DM):
 *   S(theta) = slopes of the probes through the map of theta (as
 *              synim_im_build, one row of 2N per probe), J = dS/dtheta;
 *   Gauss-Newton theta <- theta + (J^T J)^-1 J^T (s - S(theta)) from
 *              theta0 = (0, 0, 0, 1), converged when |step / half-range| < tol
 *              (S and J are FP32, which leaves a floor near 1e-7 on the
 *              normalised step: use tol >= 1e-6);
 *   learned:   a synim_mlp (n_in = 2*feat_len -> h1 -> h2 -> 4) on the
 *              standardised features [x slopes | y slopes] (probe-major,
 *              subaperture-minor, each channel zero-padded to feat_len) whose
 *              output y in [-1, 1] maps to lo + (y + 1)(hi - lo)/2.
 * A call handles up to max_batch samples, each its own map, in one multi-pair
 * build per iteration; the loop runs on the device with no host sync. */

#define SYNIM_MISREG_GN 0
#define SYNIM_MISREG_MLP 1
#define SYNIM_MISREG_MLP_GN 2

typedef struct {
  synim_wfs wfs;              /* the WFS (device arrays)                        */
  const float* probes;        /* device [n_probe][H_in][W_in] probe phase maps  */
  int32_t n_probe, H_in, W_in;
  double kappa;               /* IF pixels per WFS pixel                        */
  int32_t max_batch;          /* samples per call, 1..65535                     */
  double theta_lo[4], theta_hi[4];   /* label box; plans are sized for it       */
  int32_t max_iter;           /* Gauss-Newton iterations, 1..100                */
  double tol;
  const float* mlp_params;    /* device packed MLP, or NULL (GN only)           */
  int32_t h1, h2, feat_len;   /* hidden sizes; per-channel input length         */
  const float* feat_mean;     /* device [2 n_probe N] feature mean              */
  const float* feat_std;      /* device [2 n_probe N] feature std (> 0)         */
  int32_t gn_batched;         /* 0: Gauss-Newton in one launch per call when the
                                 WFS is small (n_probe*N <= 65536, p <= 64), else
                                 per iteration through the batched 5-plane build;
                                 1: always the batched build                    */
} synim_misreg_desc;

typedef struct synim_misreg_ctx synim_misreg_ctx;

int synim_misreg_workspace(const synim_misreg_desc* d, size_t* bytes);
/* Borrows the probes, WFS arrays, MLP and feature statistics; synchronises. */
int synim_misreg_create(const synim_misreg_desc* d, void* ws, size_t ws_bytes, void* stream,
                        synim_misreg_ctx** out);
/* Probe slopes S (device [B][n_probe*2N]) and, if jac is not NULL, the
 * Jacobian (device [B][4][n_probe*2N]) at theta (device float64 [B][4]). */
int synim_misreg_slopes(synim_misreg_ctx* c, const double* theta, int B, float* slopes,
                        float* jac, void* stream);
/* Features (device [B][2 n_probe N], compact MLP input) of slopes; standardised
 * with mean/std (device, nullable: raw features). */
int synim_misreg_features(synim_misreg_ctx* c, const float* slopes, int B, const float* mean,
                          const float* std, float* x, void* stream);
/* Estimate theta (device float64 [B][4]) from slopes (device [B][n_probe*2N]).
 * mode: SYNIM_MISREG_GN, _MLP, _MLP_GN (GN started from the MLP estimate).
 * iters (device int32 [B], nullable): GN steps taken (0 for MLP; -1 / -2 flag
 * a probe region beyond the context's bound / a lost workgroup sync, neither
 * expected inside the label box).  iter_cap (<= max_iter, 0 = max_iter)
 * bounds the GN loop.  use_graph: replay a graph captured on `stream` (must
 * not be NULL) per (B, mode, iter_cap) and, on the paths that read the
 * caller's arrays directly (MLP, one-launch Gauss-Newton), per (slopes,
 * theta, iters) addresses; the 16 most recent graphs are kept. */
int synim_misreg_infer(synim_misreg_ctx* c, const float* slopes, int B, int mode, double* theta,
                       int32_t* iters, int iter_cap, int use_graph, void* stream);
/* OR of the plan status words (see synim_plan_status) of the samples of the
 * last synim_misreg_slopes call or batched Gauss-Newton synim_misreg_infer
 * call (0 after an MLP-only or one-launch Gauss-Newton call, which build no
 * plans); synchronises. */
int synim_misreg_status(synim_misreg_ctx* c, int* host_out, void* stream);
/* Gauss-Newton convergence of the last synim_misreg_infer call: *host_n
 * (host) = samples whose loop stopped without meeting tol (the iteration cap
 * was reached, the normal matrix was singular, or the probe region left the
 * context's bound; 0 after an MLP-only call).  Returns SYNIM_E_NOT_CONVERGED
 * when *host_n > 0, SYNIM_OK otherwise; synchronises `stream`.
 * Errors: SYNIM_E_NULL, SYNIM_E_HIP. */
int synim_misreg_unconverged(synim_misreg_ctx* c, int32_t* host_n, void* stream);
void synim_misreg_destroy(synim_misreg_ctx* c);

#ifdef __cplusplus
}
#endif
#endif /* SYNIM_H */
