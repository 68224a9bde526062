/* fmbym.h - C ABI of the MI355X decoupled correlative pose search (Fast-MbyM).
 *
 * The library estimates the SE(2) pose between two Cartesian radar scans f and
 * g, the problem of Section III-A: find theta, t with f(x) ~= g(R(theta) x + t)
 * (Eq. 1).  It follows ScanMatch (Algorithm 1): the heading comes from the
 * circular correlation of polar magnitude spectra along angle (Eq. 5-8), the
 * translation from the 2-D correlation of f with g rotated by that heading
 * (Eq. 9), both through temperature soft-argmaxes (Section III-D), optionally
 * on masked scans f o m_f, g o m_g (Eq. 11).
 *
 * Conventions (shared by every entry point)
 *   - Scans are float32, row-major [n][n]; row i is y = (i - c) delta_xy and
 *     column j is x = (j - c) delta_xy metres with the origin pixel
 *     c = floor(n/2) (n/2 for even n, (n - 1)/2 for the odd sides the paper
 *     measures, Section IV-C); the sensor is pixel (c, c).
 *   - pose[b] = {theta (rad), t_x (m), t_y (m)} satisfies Eq. 1.
 *   - c_theta[b][k] is the heading score of lag l = k - floor(n_theta/2), i.e. of the
 *     candidate theta_l = l pi / n_theta, CENTRED: the mean score over all
 *     lags is subtracted and returned in saved[b][FMBYM_SAVED_THETA_MEAN].  The
 *     scores are sums of products of non-negative magnitudes, so the mean is
 *     orders of magnitude larger than the lag-dependent part that the softmax
 *     sees; computing the centred part without it keeps that part exact to
 *     FP32 rounding of its own size.  c = c_theta + mean recovers the sums.
 *   - c_xy[b][i][j] is the translation score of lag (s_y, s_x) = (i - c, j - c)
 *     pixels, the linear correlation sum_x f_w[x] g'[x + s].
 *   - The Hann window is (1 + cos(2 pi (k - c) / n)) / 2 per axis: the periodic
 *     Hann for even n, symmetric about the origin pixel for odd n.
 *   - Forward DFTs are unnormalised; correlation values equal their defining sums.
 *
 * Memory and errors
 *   - Every array argument is a DEVICE pointer, allocated and owned by the
 *     caller; the library never allocates in the search calls and keeps no
 *     reference after a call returns.  The plan owns only small constant
 *     tables (twiddles, window) allocated by fmbym_plan_create.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL is the null
 *     stream).  Arguments are validated on the host before anything is
 *     enqueued; a call that returns an error has enqueued nothing.
 *   - Return value: FMBYM_OK or a negative FMBYM_E* code.  Nothing throws or
 *     prints.  Non-finite inputs propagate to the outputs.
 *   - Calls on distinct plans/streams may run concurrently from different
 *     threads; a workspace must not be shared by calls in flight.
 */
#ifndef FMBYM_H
#define FMBYM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMBYM_API __attribute__((visibility("default")))

#define FMBYM_OK 0
#define FMBYM_EINVAL (-1)       /* bad parameter or NULL required pointer          */
#define FMBYM_EUNSUPPORTED (-2) /* size or flag combination not implemented        */
#define FMBYM_EWORKSPACE (-3)   /* workspace NULL or smaller than required          */
#define FMBYM_EHIP (-4)         /* HIP runtime error; see fmbym_last_hip_error()    */

/* flags */
#define FMBYM_HANN 1u           /* periodic Hann window on both scans (Algorithm 1) */
#define FMBYM_ANGLE_MARGINAL 2u /* heading scores from the radius-summed polar profiles,
                                   c[l] = (1/n_r) sum_a S_f[a] S_g[a + l] with S = sum over
                                   radii: the marginal reading of Algorithm 1's "Mean over
                                   r" (default: Eq. 8's per-radius correlation, averaged)  */
#define FMBYM_LOGIT_ZSCORE 4u   /* both softmaxes on standardised scores, (c - mean)/std
                                   over the lags (population std): softmax((c - max c) /
                                   (T std)); a reading of the temperature's scale          */
#define FMBYM_XY_UNWINDOWED 8u  /* translation stage on the unwindowed scans        */
#define FMBYM_HARD_ARGMAX 16u   /* hard argmax instead of both soft-argmaxes: theta and t'
                                   are the lags of the first maximum (lowest heading index;
                                   row-major (s_y, s_x) for c_xy), the search of Eq. 2-3
                                   without the soft relaxation                              */
/* The three readings are forward only: the adjoint, the training pair and the
 * one-call vjp return FMBYM_EUNSUPPORTED for a plan with any of them, and so do
 * the full-circle search with FMBYM_LOGIT_ZSCORE or FMBYM_HARD_ARGMAX, odd sides
 * (plan creation) and fmbym_autotune with the adjoint.  Saved slots hold the
 * statistics of the chosen reading (THETA_SUM, XY_SUM with T std as the
 * temperature; THETA_NU 0 under FMBYM_HARD_ARGMAX). */
#define FMBYM_CHECK_FINITE 64u  /* forward calls count each pair's non-finite input
                                   values (f, g and the masks) into
                                   saved[b][FMBYM_SAVED_STATUS]; the search itself
                                   is unchanged (non-finite values still propagate) */

/* floats per pair in the `saved` statistics buffer, and its slots */
#define FMBYM_SAVED 16
#define FMBYM_SAVED_THETA 0       /* heading theta (rad)                                  */
#define FMBYM_SAVED_COS 1         /* cos(theta), sin(theta) as used by Rotate             */
#define FMBYM_SAVED_SIN 2
#define FMBYM_SAVED_THETA_MAX 3   /* max over lags of c_theta (centred scores)            */
#define FMBYM_SAVED_THETA_SUM 4   /* sum_l exp((c_theta[l] - max) / T_theta)             */
#define FMBYM_SAVED_XY_MAX 5      /* max of c_xy                                          */
#define FMBYM_SAVED_XY_SUM 6      /* sum_s exp((c_xy[s] - max) / T_xy)                   */
#define FMBYM_SAVED_TPX 7         /* t' = (t'_x, t'_y) in metres, before t = R(theta) t' */
#define FMBYM_SAVED_TPY 8
#define FMBYM_SAVED_THETA_MEAN 9  /* mean heading score over all lags                     */
#define FMBYM_SAVED_THETA_ARG 10  /* lag l* of the largest heading score (lowest on ties) */
#define FMBYM_SAVED_THETA_NU 11   /* sum_l p_l (l - l*): theta = (l* + nu) pi / n_theta   */
#define FMBYM_SAVED_STATUS 12     /* with FMBYM_CHECK_FINITE: count of non-finite inputs,
                                     else 0; slots 13 .. 15 are reserved and written as 0 */

typedef struct fmbym_plan_s* fmbym_plan;

/* ScanMatch's parameter list (Algorithm 1) plus the band-pass of its stage 1. */
typedef struct {
    int32_t n;          /* scan side: 128, 256 or 512; or the paper's 127, 255 or 511 (forward
                           only: the calls below that need the adjoint, the training pair, the
                           joint and full-circle searches, the autotuner and ragged lists return
                           FMBYM_EUNSUPPORTED or a zero size for them; no FMBYM_CHECK_FINITE)  */
    int32_t n_theta;    /* angle bins over [0, pi), delta_theta = pi/n_theta: a power of two in
                           16..1024, or at the odd sides any count in 16..1024 (the paper's 733) */
    int32_t n_r;        /* polar radii over [0, n/2) frequency bins: 1..4096 (the method uses n) */
    float delta_xy;     /* metres per pixel (> 0)                                         */
    float temp_theta;   /* heading softmax temperature T_theta (> 0)                      */
    float temp_xy;      /* translation softmax temperature T_xy (> 0)                     */
    float band_lo;      /* band-pass: keep lo <= |k|/n <= hi (cycles per pixel) ...       */
    float band_hi;      /* ... disabled when band_hi <= 0                                  */
    uint32_t flags;     /* FMBYM_HANN | FMBYM_XY_UNWINDOWED | FMBYM_CHECK_FINITE |
                           FMBYM_ANGLE_MARGINAL | FMBYM_LOGIT_ZSCORE | FMBYM_HARD_ARGMAX      */
} fmbym_params;

/* Launch choices of a plan: column-tile widths of the column passes (how many
 * float4 columns one block transforms: 4, 8 or 16), the batch split, the rows
 * each line of the two row passes transforms in sequence, and the radix plan
 * of the n-point column lines of stage 1 and of the |F| adjoint.  Widths, split
 * and rows change speed, never results: every choice runs the same arithmetic
 * on every pair, row and column.  The radix plans (radix-8 stages with 8
 * elements per thread, or radix-4 with 4) round differently, so results move
 * by FP32 rounding, within the parity tolerances.  A block may not exceed 1024
 * threads: width * n / radix <= 1024.  A new plan starts from defaults for its
 * n; fmbym_autotune measures and sets the fastest.  Because of the split's
 * stream and events, calls on one plan must not be issued concurrently from
 * several host threads. */
typedef struct {
    int32_t cols1;      /* stage-1 column FFTs and |F|                      */
    int32_t cols2;      /* stage-2 column correlation                       */
    int32_t cols_xy;    /* adjoint of the stage-2 column correlation        */
    int32_t cols_mag;   /* adjoint of |F| and the stage-1 columns            */
    int32_t split;      /* 1, or 2: the search calls run the two halves of a
                           batch concurrently, the second on a stream the plan
                           owns (joined back to the caller's stream by events;
                           still capturable into a graph)                   */
    int32_t rows1;      /* 1 or 2 rows per line in sequence, stage-1 rows    */
    int32_t rows2;      /* 1 or 2 rows per line in sequence, stage-2 rows    */
    int32_t radix1;     /* 8 or 4: radix plan of the stage-1 column lines    */
    int32_t radix_mag;  /* 8 or 4: radix plan of the |F| adjoint's columns   */
} fmbym_tuning;

/* Validate `p` and build a plan (uploads constant tables to the current device;
 * this call allocates).  `max_batch` bounds the batch of later calls (>= 1). */
FMBYM_API int fmbym_plan_create(const fmbym_params* p, int32_t max_batch, fmbym_plan* out);
FMBYM_API int fmbym_plan_destroy(fmbym_plan plan);

/* Bytes of device workspace needed by fmbym_search (with_backward = 0) or by
 * fmbym_search_backward (with_backward = 1) for `batch` pairs; 0 on bad input. */
FMBYM_API size_t fmbym_search_workspace_size(fmbym_plan plan, int32_t batch, int with_backward);

/* Forward search (Algorithm 1 on Eq. 11's masked scans).
 *   f, g      [batch][n][n]     scans (required)
 *   m_f, m_g  [batch][n][n]     masks, or both NULL for the unmasked search
 *   pose      [batch][3]        output (required)
 *   c_theta   [batch][n_theta]  output heading scores, or NULL
 *   c_xy      [batch][n][n]     output translation scores, or NULL
 *   saved     [batch][FMBYM_SAVED]  output softmax statistics, or NULL
 * c_theta, c_xy and saved are required if fmbym_search_backward will be called. */
FMBYM_API int fmbym_search(fmbym_plan plan, int32_t batch, const float* f, const float* g,
                 const float* m_f, const float* m_g, float* pose, float* c_theta, float* c_xy,
                 float* saved, void* workspace, size_t workspace_bytes, void* stream);

/* Adjoint of fmbym_search: given d_pose = dL/dpose [batch][3], writes
 * d_f, d_g (required) and d_m_f, d_m_g (required iff masks were given) as
 * dL/d(input), all [batch][n][n], overwritten.  pose, c_theta, c_xy and saved
 * are the outputs of the forward call on the same inputs.  The spectra are
 * recomputed, not stored. */
FMBYM_API int fmbym_search_backward(fmbym_plan plan, int32_t batch, const float* f, const float* g,
                          const float* m_f, const float* m_g, const float* pose,
                          const float* c_theta, const float* c_xy, const float* saved,
                          const float* d_pose, float* d_f, float* d_g, float* d_m_f, float* d_m_g,
                          void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------- tuning
 *
 * fmbym_plan_get_tuning / fmbym_plan_set_tuning read and replace the plan's
 * launch choices (set: FMBYM_EINVAL unless every width is 4, 8 or 16, split
 * and the rows are 1 or 2, the radix plans 8 or 4, and the blocks fit).
 * Not to be called while searches on the plan are in flight.
 *
 * fmbym_autotune times whole search steps on synthetic inputs it writes into
 * its workspace (fmbym_autotune_workspace_size bytes) and picks the choices one
 * at a time (split over 1, 2, then the widths over 4, 8, 16 in the order cols1,
 * cols2, cols_xy, cols_mag, then rows1, rows2 over 1, 2 and radix1, radix_mag
 * over 8, 4, each with the width it got; with_backward = 0 times the forward
 * alone and leaves the adjoint's choices as they are).  It synchronises `stream`, creates and
 * destroys two HIP events, sets the result on the plan and writes it to *best;
 * ms_per_step (or NULL) receives the best step time.  Results of the searches
 * do not depend on the choice. */
FMBYM_API int fmbym_plan_get_tuning(fmbym_plan plan, fmbym_tuning* out);
FMBYM_API int fmbym_plan_set_tuning(fmbym_plan plan, const fmbym_tuning* t);
FMBYM_API size_t fmbym_autotune_workspace_size(fmbym_plan plan, int32_t batch, int with_backward);
FMBYM_API int fmbym_autotune(fmbym_plan plan, int32_t batch, int with_backward, void* workspace,
                             size_t workspace_bytes, void* stream, fmbym_tuning* best, float* ms_per_step);

/* ---------------------------------------------------------------- training pair
 *
 * A forward that keeps its intermediates for the adjoint: the stage-1 row
 * spectra and magnitudes |F| (Eq. 5-7), the rotated scan g' = Rotate(g_w)
 * with its heading derivative dg'/dtheta, and the stage-2 row spectra (Eq. 9).
 * fmbym_search_backward_state reads them instead of recomputing them, which
 * removes the stage-1 transforms and the rotation from the adjoint.  Results
 * are those of fmbym_search / fmbym_search_backward up to FP32 rounding order.
 *   state  device buffer of fmbym_search_state_size() bytes, owned by the
 *          caller; written by fmbym_search_train, only read by the adjoint (which
 *          may be called on it any number of times); layout private.
 * Same memory, stream and error rules as above; c_theta, c_xy and saved are
 * required. */
FMBYM_API size_t fmbym_search_state_size(fmbym_plan plan, int32_t batch);
FMBYM_API int fmbym_search_train(fmbym_plan plan, int32_t batch, const float* f, const float* g,
                                 const float* m_f, const float* m_g, float* pose, float* c_theta,
                                 float* c_xy, float* saved, void* state, size_t state_bytes,
                                 void* workspace, size_t workspace_bytes, void* stream);
/* Adjoint of fmbym_search_train (same inputs, its outputs and state); the
 * workspace is that of fmbym_search_workspace_size(plan, batch, 1). */
FMBYM_API int fmbym_search_backward_state(fmbym_plan plan, int32_t batch, const float* f,
                                          const float* g, const float* m_f, const float* m_g,
                                          const float* pose, const float* c_theta, const float* c_xy,
                                          const float* saved, const void* state, size_t state_bytes,
                                          const float* d_pose, float* d_f, float* d_g, float* d_m_f,
                                          float* d_m_g, void* workspace, size_t workspace_bytes,
                                          void* stream);

/* Training forward and its adjoint in one call, for an upstream gradient d_pose
 * the caller already holds (a vector-Jacobian product of the search): the
 * results of fmbym_search_train followed by fmbym_search_backward_state on the
 * same buffers, bit for bit.  With the plan's split = 2 each half of the batch
 * runs both passes on its own stream, forked and joined once for the pair
 * (the two calls fork and join twice).  Arguments as for those two calls; the
 * workspace is that of fmbym_search_workspace_size(plan, batch, 1).  d_pose
 * must not depend on this call's pose (for a loss of the pose, use the two
 * calls with the loss in between). */
FMBYM_API int fmbym_search_vjp(fmbym_plan plan, int32_t batch, const float* f, const float* g,
                               const float* m_f, const float* m_g, float* pose, float* c_theta,
                               float* c_xy, float* saved, void* state, size_t state_bytes,
                               const float* d_pose, float* d_f, float* d_g, float* d_m_f, float* d_m_g,
                               void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------- without allocation
 *
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): fmbym_search with its
 * workspace in a static device array of the library, FMBYM_NOALLOC_SCRATCH_BYTES
 * on every GPU the library runs on, held from module load until the process
 * ends.  Arguments are those of fmbym_search without the workspace; the
 * results are fmbym_search's on the same inputs, bit for bit (same kernels).
 * Returns FMBYM_EWORKSPACE, having enqueued nothing, when the batch's forward
 * workspace (fmbym_search_workspace_size(plan, batch, 0)) exceeds the array:
 * at 512 x 512 with 512 angle bins that admits up to 10 pairs, at 256 x 256
 * with 256 bins 42, at 128 x 128 with 128 bins 160.  FMBYM_EINVAL when the
 * current device is not the one the plan was created on.  The first call on a
 * device looks up the array's device address (no allocation); no call
 * allocates, frees or calls an allocating library routine.  Every call on one
 * GPU uses the same array and leaves its contents behind: calls that may
 * overlap on a GPU (several streams or host threads) race, and the caller must
 * serialise them. */
#define FMBYM_NOALLOC_SCRATCH_BYTES (64u << 20)
FMBYM_API int fmbym_search_noalloc(fmbym_plan plan, int32_t batch, const float* f, const float* g,
                                   const float* m_f, const float* m_g, float* pose, float* c_theta,
                                   float* c_xy, float* saved, void* stream);

/* ---------------------------------------------------------------- joint comparator
 *
 * The exhaustive search that the decoupling replaces (Eq. 2-3 with the heading
 * searched by brute force instead of by Eq. 8): for each of n_angles headings
 * theta_k = -pi/2 + k pi / n_angles, the translation stage's correlation at
 * that heading, J_k(s') = sum_x f_w(x) Rotate(g_w, theta_k)(x + s') over the
 * lags s' of c_xy; the pose is the hard argmax over (k, s') (first maximum in
 * k, then row-major s'), with t = R(theta_k) s' delta_xy.  n_angles times the
 * stage-2 work of fmbym_search.
 *   pose  [batch][3] output (required)
 *   peak  [batch][n_angles] output, max over s' of J_k, or NULL
 * Windowing and masks as in fmbym_search; 1 <= n_angles <= 4096. */
FMBYM_API size_t fmbym_joint_workspace_size(fmbym_plan plan, int32_t batch, int32_t n_angles);
FMBYM_API int fmbym_search_joint(fmbym_plan plan, int32_t batch, int32_t n_angles, const float* f,
                                 const float* g, const float* m_f, const float* m_g, float* pose,
                                 float* peak, void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------- full-circle heading
 *
 * The search for an arbitrary rotational offset (metric localisation, which
 * the paper's Conclusion proposes for the decoupled search).  Stage 1 sees
 * magnitude spectra, point symmetric for real scans (Eq. 5-6), so it fixes the
 * heading only modulo pi: fmbym_search returns theta in [-pi/2, pi/2).  This
 * call runs fmbym_search's forward, then the translation stage (Eq. 9) again
 * at theta + pi, and keeps per pair the heading whose c_xy has the larger
 * maximum (the first, theta, on ties).  About twice fmbym_search's stage-2 work.
 *   pose   [batch][3] output (required): theta in [-pi, pi] and the
 *          translation soft-argmax of the kept heading (t = R(theta) t');
 *          theta + pi is written as theta + pi for theta < 0, else theta - pi
 *   peaks  [batch][2] output, max c_xy at theta and at theta + pi, or NULL
 * Windowing, masks, batch split, memory, stream and error rules as in
 * fmbym_search; forward only (no adjoint). */
FMBYM_API size_t fmbym_full_circle_workspace_size(fmbym_plan plan, int32_t batch);
FMBYM_API int fmbym_search_full_circle(fmbym_plan plan, int32_t batch, const float* f, const float* g,
                                       const float* m_f, const float* m_g, float* pose, float* peaks,
                                       void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------- ragged work lists
 *
 * A serving batch whose pairs come at several scan sizes (the method is timed
 * at three resolutions in Section IV-C; an odometry service may receive all
 * three).  Each pair is searched exactly as fmbym_search would search it alone
 * with the plan of its size; the batch runs as ONE replayable launch: pairs are
 * grouped by (n, masked), every group is a batched forward search, and the
 * groups are concurrent branches of a HIP graph captured at creation. */
#define FMBYM_PAIR_NET_MASK 1u   /* masks of this pair come from the mask network (fmbym_mask.h) */

typedef struct {
    int32_t n;          /* scan side of this pair; one of the plans must have this n              */
    uint32_t flags;     /* 0 or FMBYM_PAIR_NET_MASK                                               */
    const float* f;     /* [n][n] device scans (required)                                         */
    const float* g;
    const float* m_f;   /* [n][n] device masks, or both NULL (must be NULL with FMBYM_PAIR_NET_MASK) */
    const float* m_g;
} fmbym_pair;

typedef struct fmbym_ragged_s* fmbym_ragged;
struct fmbym_mask_desc_s;   /* fmbym_mask_desc of fmbym_mask.h */

/* Bytes of device workspace fmbym_ragged_create needs for this work list
 * (pairs is a HOST array of n_pairs entries; net as for create); 0 on bad input. */
FMBYM_API size_t fmbym_ragged_workspace_size(const fmbym_plan* plans, int32_t n_plans,
                                             const fmbym_pair* pairs, int32_t n_pairs,
                                             const struct fmbym_mask_desc_s* net);

/* Build the launch (this call allocates: pointer tables, streams, the graph).
 *   plans     n_plans plans with distinct n; each pair uses the one of its n
 *             (their max_batch does not bound the group sizes)
 *   pairs     HOST array; the device pointers in it are baked into the launch:
 *             every fmbym_ragged_launch reads what they hold at that time
 *   net       mask network for the pairs flagged FMBYM_PAIR_NET_MASK (NULL if
 *             none is): each such group first runs the network in inference
 *             mode (running statistics) on its 2 x count scans, then the search
 *             on the masked scans; the descriptor is copied, the buffers it
 *             points to are read at every launch
 *   pose      [n_pairs][3] device output, in the order of `pairs`
 *   stamps    [n_pairs + 1] device output or NULL: stamps[i] is the device wall
 *             clock when pose[i] was written, stamps[n_pairs] when the launch
 *             started (ticks of hipDeviceAttributeWallClockRate, in kHz)
 *   workspace fmbym_ragged_workspace_size() bytes, owned by the caller, used by
 *             every launch and by nothing else until fmbym_ragged_destroy
 * Plans, the network's buffers, pose, stamps and workspace must outlive the
 * object.  Launches of one object must not overlap (they share the workspace). */
FMBYM_API int fmbym_ragged_create(const fmbym_plan* plans, int32_t n_plans, const fmbym_pair* pairs,
                                  int32_t n_pairs, const struct fmbym_mask_desc_s* net, float* pose,
                                  uint64_t* stamps, void* workspace, size_t workspace_bytes,
                                  fmbym_ragged* out);
/* Enqueue one replay of the whole work list on `stream`. */
FMBYM_API int fmbym_ragged_launch(fmbym_ragged r, void* stream);
FMBYM_API int fmbym_ragged_destroy(fmbym_ragged r);

/* The same work list in one call, without a launch object: validates and
 * groups `pairs` (a HOST array) as fmbym_ragged_create does, copies the
 * per-pair pointer table into the caller's workspace in stream order, and
 * enqueues every group's batched forward search (network-masked groups after
 * their mask network) one after another on `stream`.  Poses and stamps as for
 * fmbym_ragged_create; each pair's pose is bit for bit what fmbym_search gives
 * it alone with the plan of its size.  Allocates no device memory and creates
 * no stream, event or graph; the workspace (fmbym_search_ragged_workspace_size
 * bytes) must not be used by another call in flight. */
FMBYM_API size_t fmbym_search_ragged_workspace_size(const fmbym_plan* plans, int32_t n_plans,
                                                    const fmbym_pair* pairs, int32_t n_pairs,
                                                    const struct fmbym_mask_desc_s* net);
FMBYM_API int fmbym_search_ragged(const fmbym_plan* plans, int32_t n_plans, const fmbym_pair* pairs,
                                  int32_t n_pairs, const struct fmbym_mask_desc_s* net, float* pose,
                                  uint64_t* stamps, void* workspace, size_t workspace_bytes, void* stream);
/* Rate of the device wall clock behind the stamps, in kHz, for the current device. */
FMBYM_API int fmbym_wall_clock_khz(int32_t* khz);

/* Diagnostics: per-kernel timing.  fmbym_profile_enable(capacity) with
 * capacity > 0 pre-creates `capacity` event pairs (it allocates) and brackets
 * every later kernel launch of the library with two events on the launch's
 * stream, until the pool is used up; capacity <= 0 switches timing off and
 * frees the pool.  fmbym_profile_read synchronises the recorded events and
 * fills, per kernel k < returned count: names[k], total_ms[k] (sum of launch
 * durations) and launches[k].  Arrays must hold max_kernels >= 64 entries.
 * Returns the kernel count, FMBYM_EWORKSPACE if the pool overflowed, or an
 * error code.  Not for concurrent use from several threads. */
FMBYM_API int fmbym_profile_enable(int32_t capacity);
FMBYM_API int fmbym_profile_read(int32_t max_kernels, const char** names, double* total_ms,
                                 int32_t* launches);

FMBYM_API const char* fmbym_strerror(int code);
/* hipError_t of the last FMBYM_EHIP returned on this thread (0 if none). */
FMBYM_API int fmbym_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FMBYM_H */
