/*
 * hgf.h -- C ABI of the MI355X (gfx950) hardware-efficient guided filter (HGF)
 * for multi-label cost volumes.
 *
 * Problem (paper: Dai et al., "Hardware-Efficient Guided Image Filtering For
 * Multi-Label Problem", arXiv 1803.00005):
 *   a multi-label system stores the cost of label l at pixel (x, y) in a cost
 *   volume V(x, y, l), filters every label slice under a guidance image and
 *   picks the winner-takes-all label per pixel (Sec. 1).  Each slice Y is
 *   filtered by HGF (Sec. 4): an n-channel polynomial guidance G is
 *   synthesized from the input guidance I (Sec. 4.2), a ridge regression is
 *   fitted in every (2r+1)x(2r+1) window (Eq. 6 / Eq. 2) with the per-pixel
 *   matrix inverted by the recursion of Prop. 1, and the window predictions
 *   are averaged (Eq. 7, Eq. 11).
 *
 * Conventions shared by every call
 *   - Device pointers are plain HIP device addresses (e.g. the data_ptr() of
 *     a torch CUDA tensor).  The caller owns every buffer it passes in;
 *     the library owns hgf_context and hgf_guide objects.
 *   - Layouts (row-major, no padding unless a leading dimension is given):
 *       guide  float32 [m][H][W]           planar channels
 *       cost   float32 or bfloat16 [H][W][ld]   pixel-major, labels contiguous
 *       out    float32 [H][W][ld]          filtered costs Z
 *       labels int32   [H][W]              winner-takes-all label
 *   - Windows are clipped at the image border: the box filter sums the
 *     in-image pixels of the window and the average divides by their count
 *     (the average operator A(X) = B(X) / B(1) of Sec. 4.3).
 *   - All calls are asynchronous on the given hipStream_t (NULL = the null
 *     stream).  Argument errors are detected on the host before anything is
 *     enqueued; launch errors are returned at once; faults inside kernels
 *     surface at the caller's next synchronisation.
 *   - Every call returns an hgf_status; no C++ exception crosses the ABI
 *     (a failed host allocation returns HGF_E_NOMEM).  hgf_last_error()
 *     returns the detail string of the context's last failed call.
 *   - A context must not be used from two host threads at once.  Calls that
 *     use context-owned memory (a NULL workspace, a resident guide) must
 *     not overlap on two streams: they share that memory.
 *   - Results are deterministic: for fixed parameters and tuning table they
 *     do not depend on the stream, on other images in a batch or the served
 *     mix, on how the labels are split into chunks (hgf_guide_filter) or on
 *     the launch-group size (hgf_set_group_bytes).
 *   - Compiled set: n = 1..19 guidance channels, radius 0..9, every cost
 *     dtype, both solve precisions; the ridge form with float32 costs.
 */
#ifndef HGF_H
#define HGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HGF_OK = 0,
  HGF_E_INVALID = -1,     /* an argument is out of range or inconsistent */
  HGF_E_NOMEM = -2,       /* a device allocation failed or would exceed the budget */
  HGF_E_DEVICE = -3,      /* a HIP runtime call or kernel launch failed */
  HGF_E_UNSUPPORTED = -4, /* valid but not compiled in (n, radius, dtype) */
  HGF_E_BUSY = -5         /* the serving queue is full */
} hgf_status;

/* Element types.  Costs may be float32, bfloat16 or float16 (converted to
 * float32 on load; every sum and product runs in float32 or wider).  The
 * per-pixel solve is applied in float32 or float64 (stats_dtype below). */
typedef enum { HGF_F32 = 0, HGF_BF16 = 1, HGF_F16 = 2, HGF_F64 = 3 } hgf_dtype;

/* Polynomial guidance basis (Sec. 4.2).
 *   MONOMIAL: every monomial of total degree 1..d of the m channels, graded
 *             lexicographic with channel 1 first (RGB, d=2: R,G,B,R^2,RG,RB,
 *             G^2,GB,B^2); n = C(m+d, d) - 1.
 *   POWER:    the paper's map G_{(i-1)d+j} = I_i^j, channel-major; n = m d. */
typedef enum { HGF_BASIS_MONOMIAL = 0, HGF_BASIS_POWER = 1 } hgf_basis;

/* Regularisation.
 *   COVARIANCE: the guided-filter form of Sec. 5.1 (Eqs. 12-13): intercept
 *               free, (Sigma_p + eps E) a_p = cov_p(G, Y) on window means.
 *   RIDGE:      the paper's HGF definition, Eq. 6: every coefficient,
 *               intercept included, penalised by lambda on raw window sums,
 *               (lambda E + X^T X) w_p = X^T Y (Eq. 2). */
typedef enum { HGF_REG_COVARIANCE = 0, HGF_REG_RIDGE = 1 } hgf_reg;

typedef struct {
  int32_t height;          /* H >= 1 */
  int32_t width;           /* W >= 1 */
  int32_t guide_channels;  /* m in {1, 2, 3} */
  int32_t degree;          /* d >= 1 */
  int32_t basis;           /* hgf_basis */
  int32_t reg;             /* hgf_reg */
  int32_t radius;          /* r >= 0: window side 2r + 1 */
  int32_t num_labels;      /* L >= 1 */
  double eps;              /* > 0: eps (COVARIANCE) or lambda (RIDGE) */
  int32_t cost_dtype;      /* hgf_dtype of the cost volume: HGF_F32, HGF_BF16 or HGF_F16 */
  int32_t cost_ld;         /* label stride of cost (0 = num_labels) */
  int32_t out_ld;          /* label stride of out  (0 = num_labels) */
  int32_t stats_dtype;     /* precision of the per-pixel solve (a3, a5).  The
                            * guidance window statistics and the inverse are
                            * always computed in float64; then
                            *   HGF_F32 (0): the inverse and window means are
                            *     stored in float32 and the coefficient
                            *     product a = M c runs in float32;
                            *   HGF_F64: they are stored in float64 and c, a
                            *     and b are formed in float64 (for the
                            *     ill-conditioned systems of large n).
                            * The ridge form always uses float64. */
} hgf_params;

typedef struct hgf_context hgf_context;
typedef struct hgf_guide hgf_guide;

/* n, the number of guidance channels the basis synthesizes from m channels
 * at degree d (Sec. 4.2), or -1 if m, d or basis is invalid. Host only. */
int32_t hgf_num_channels(int32_t m, int32_t d, int32_t basis);

/* 1 if (n, radius) has compiled kernels for the given regularisation, else 0. Host only. */
int32_t hgf_is_supported(int32_t n, int32_t radius, int32_t reg);

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * device memory the context allocates for itself (0 = no bound).  Allocates
 * nothing on the device until a call needs library-owned memory. */
hgf_status hgf_create(int32_t device, size_t hbm_budget_bytes, hgf_context** out);
void hgf_destroy(hgf_context* ctx);

/* Bytes of device workspace hgf_filter needs for these parameters, with the
 * label chunks it processes per launch under the default launch-group size.
 * Host only; validates params. */
hgf_status hgf_workspace_size(const hgf_params* params, size_t* bytes);

/* Upper bound of the coefficient workspace of one launch group (the float32
 * coefficients a, b of the labels filtered by one pair of per-label launches,
 * (n + 1) * 256 bytes per pixel and 64-label chunk).  Default 12 GiB; 0
 * restores it.  Labels that do not fit run in further launch groups, one
 * after another; the results do not change.  A smaller bound lowers the
 * workspace a call needs below hgf_workspace_size(). */
hgf_status hgf_set_group_bytes(hgf_context* ctx, size_t bytes);

/* The whole hot path on one image (Fig. 2 of the paper for every slice):
 * guidance synthesis, guidance box statistics, per-pixel inverse (Prop. 1),
 * per-label coefficient box sums and solve (Eq. 5 / Eq. 13), coefficient
 * box filter and output (Eq. 11), winner-takes-all (Sec. 1).
 *   guide      device float32 [m][H][W]
 *   cost       device [H][W][cost_ld] of cost_dtype; labels 0..L-1 used
 *   out        device float32 [H][W][out_ld] or NULL (labels only)
 *   labels     device int32 [H][W] or NULL (no winner-takes-all)
 *   workspace  device buffer of at least hgf_workspace_size() bytes, 256-byte
 *              aligned, or NULL to use context-owned memory
 * Errors: HGF_E_INVALID (bad params, both outputs NULL, small workspace),
 * HGF_E_UNSUPPORTED (n or radius not compiled in), HGF_E_NOMEM, HGF_E_DEVICE. */
hgf_status hgf_filter(hgf_context* ctx, const hgf_params* params,
                      const float* guide, const void* cost,
                      float* out, int32_t* labels,
                      void* workspace, size_t workspace_bytes, void* hip_stream);

/* Two-phase form.  hgf_guide_create computes the guidance part once and keeps
 * it resident on the device (the all-pair box filters of the guidance are
 * computed once and shared by every slice, Sec. 5.3): the synthesized
 * guidance, the window means and the per-pixel inverses.  The guide buffer
 * is read during the call only.  params->num_labels is the total label count
 * of the volume that later chunks belong to. */
hgf_status hgf_guide_create(hgf_context* ctx, const hgf_params* params,
                            const float* guide, void* hip_stream, hgf_guide** out);

/* Filter labels [label_begin, label_begin + label_count) with resident
 * guidance statistics.
 *   cost_chunk  device [H][W][ld] of the params' cost dtype, label_begin at column 0
 *   out_chunk   device float32 [H][W][ld] or NULL
 *   best_cost, labels  device float32 / int32 [H][W] running minimum and
 *               argmin over the labels filtered so far; when label_begin == 0
 *               they are (re)initialised, otherwise merged (lower cost wins,
 *               lower label on ties).  Both NULL: no winner-takes-all.
 *   ld          label stride of cost_chunk and out_chunk (0 = label_count). */
hgf_status hgf_guide_filter(hgf_context* ctx, hgf_guide* guide,
                            const void* cost_chunk, int32_t label_begin,
                            int32_t label_count, int32_t ld, float* out_chunk,
                            float* best_cost, int32_t* labels, void* hip_stream);

/* Device bytes held by a resident guide. */
size_t hgf_guide_bytes(const hgf_guide* guide);
void hgf_guide_destroy(hgf_guide* guide);

/* Copy a resident guide's per-pixel statistics out (for inspection):
 *   mu    device float64 [H][W][n]   window means of the (shifted) guidance
 *   minv  device [H][W][D(D+1)/2] packed upper triangle of the per-pixel
 *         inverse, row by row: D = n and float32 in the covariance form
 *         (computed in float64, stored rounded), D = n + 1 and float64 in
 *         the ridge form
 *   shift device float64 [n] the constant subtracted from each guidance
 *         channel (0 in ridge mode)
 * Any pointer may be NULL. */
hgf_status hgf_guide_export(const hgf_guide* guide, double* mu, void* minv,
                            double* shift, void* hip_stream);

/* Filter `count` images of uneven size and label count (the batched form).
 * Every image runs the whole path of hgf_filter on one of up to four worker
 * streams (largest images first, each to the least-loaded stream), in
 * context-owned workspaces, so images overlap on the device.  The sequence is
 * captured once into a hipGraph (fork from hip_stream, join back to it) and
 * cached with the batch's signature (parameters, buffer addresses, tuning);
 * a later call with the same signature replays it with one graph launch.
 * The graph holds kernel nodes only.  Results equal hgf_filter's bit for bit.
 * Arrays of length count; outs[i] or labels[i] may be NULL (not both), and
 * outs or labels themselves may be NULL.  Errors as hgf_filter, reported for
 * the first bad image before anything is enqueued. */
hgf_status hgf_filter_batch(hgf_context* ctx, int32_t count, const hgf_params* params,
                            const float* const* guides, const void* const* costs,
                            float* const* outs, int32_t* const* labels,
                            void* hip_stream);

/* Autotuner of the strip decomposition of the strip kernels (a2, a4-a7).
 * Times every candidate block count of the guidance moment, coefficient and
 * output kernels on these inputs with HIP events (three passes of the whole
 * path each) and stores the fastest of each kernel in the context's table for
 * the class (kernel, n, radius, solve form, cost dtype, floor(log2 H W)).
 * Later calls of that class use it.  Synchronises hip_stream.  `out` may be
 * NULL; when given it receives valid filtered costs.  Workspace as hgf_filter.
 * A table entry changes the band boundaries of the float32 running sums, so
 * results move at rounding level when the table changes. */
hgf_status hgf_autotune(hgf_context* ctx, const hgf_params* params,
                        const float* guide, const void* cost, float* out,
                        void* workspace, size_t workspace_bytes, void* hip_stream);

/* The tuning table as rows of 7 int32 (kernel 0=coefficients 1=output
 * 2=guidance moment sums, n, radius, solve form 0=covariance with float32
 * solve 1=covariance with float64 solve 2=ridge, cost hgf_dtype, size class,
 * target blocks).  Writes at most
 * max_rows rows (rows may be NULL) and the total row count to *count. */
hgf_status hgf_tune_entries(const hgf_context* ctx, int32_t* rows, int32_t max_rows,
                            int32_t* count);
/* Set one row (7 int32 as above). */
hgf_status hgf_tune_set(hgf_context* ctx, const int32_t* row);
/* Save / load the table as text, one row per line ('#' starts a comment). */
hgf_status hgf_tune_save(const hgf_context* ctx, const char* path);
hgf_status hgf_tune_load(hgf_context* ctx, const char* path);

/* Serving form: requests arrive one at a time and are filtered as soon as
 * device memory allows (continuous batching).
 *   hgf_server_create  allocates an arena of arena_bytes (within the
 *                      context's budget) and `slots` streams (1..16).
 *   hgf_server_submit  queues one request (parameters and buffers as
 *                      hgf_filter; every buffer must stay valid until the
 *                      request completes).  The request waits for the work
 *                      queued on hip_stream before it (its inputs).  It is
 *                      admitted, in strict FIFO order, when its workspace
 *                      (hgf_workspace_size) fits in the arena, and then runs
 *                      on the least-loaded slot stream.  Returns its id.
 *                      HGF_E_BUSY: max_queue requests already wait;
 *                      HGF_E_NOMEM: it can never fit in the arena.
 *   hgf_server_poll    retires finished requests, admits waiting ones and
 *                      returns up to max_done completion records, oldest
 *                      first.  Outputs of a completed request are ready.
 *   hgf_server_drain   blocks until every submitted request has completed.
 * Once hgf_server_submit has set *id the request is queued, even when the
 * call returns an error: submit, poll and drain also launch waiting
 * requests and return the first launch error among them, and poll and
 * drain return the first device error of the requests they retire; every
 * failed request's completion record carries its own status.
 * Completion times are on the device clock in milliseconds since the server
 * was created.  A request computes exactly what hgf_filter computes for the
 * same parameters and tuning table.  A server is used from one host thread
 * at a time. */
typedef struct hgf_server hgf_server;
typedef struct {
  int64_t id;
  int32_t status;    /* hgf_status of the request */
  int32_t slot;      /* stream it ran on */
  double start_ms;   /* device time its first kernel could start */
  double end_ms;     /* device time its last kernel ended */
} hgf_completion;
typedef struct {
  int32_t pending;
  int32_t running;
  int64_t completed;
  size_t arena_bytes;
  size_t arena_in_use;
  size_t arena_peak;
} hgf_server_info;

hgf_status hgf_server_create(hgf_context* ctx, int32_t slots, size_t arena_bytes,
                             int32_t max_queue, hgf_server** out);
void hgf_server_destroy(hgf_server* server);
hgf_status hgf_server_submit(hgf_server* server, const hgf_params* params,
                             const float* guide, const void* cost, float* out,
                             int32_t* labels, void* hip_stream, int64_t* id);
hgf_status hgf_server_poll(hgf_server* server, hgf_completion* done, int32_t max_done,
                           int32_t* count);
hgf_status hgf_server_drain(hgf_server* server);
hgf_status hgf_server_stats(const hgf_server* server, hgf_server_info* out);
/* The device clock now (ms since the server was created): records an event
 * on an idle stream of the server, waits for it and returns its time.  Pairs a host timestamp taken
 * right after the call with the device clock of the completion records. */
hgf_status hgf_server_now(hgf_server* server, double* ms);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): hgf_filter with
 * its workspace in a library-owned static device array of
 * hgf_static_scratch_bytes() bytes (96 MiB) per GPU, held until the process
 * ends; no call allocates or frees memory.  The caller passes inputs and
 * outputs as for hgf_filter (workspace and label-group size as for a
 * one-chunk launch group); the results equal hgf_filter's bit for bit.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (two streams, or two threads) race and give wrong results.  Errors as
 * hgf_filter, and HGF_E_NOMEM when the filter needs more workspace than the
 * array holds (about 30,000 pixels at n = 9); nothing is enqueued then.
 * With stage timing switched on (hgf_set_stage_timing) the context records
 * timing events, creating them on first use; leave it off where nothing may
 * be created. */
hgf_status hgf_filter_static(hgf_context* ctx, const hgf_params* params,
                             const float* guide, const void* cost,
                             float* out, int32_t* labels, void* hip_stream);
size_t hgf_static_scratch_bytes(void);

/* Standalone clipped box sum (Prop. 2) of C float32 images [C][H][W]:
 * out[c][y][x] = sum of in[c] over the clipped (2r+1)^2 window.  in and out
 * must not overlap. */
hgf_status hgf_box_sum(const float* in, float* out, int32_t channels,
                       int32_t height, int32_t width, int32_t radius,
                       void* hip_stream);

/* Batched inverse of `count` symmetric positive definite D x D matrices by
 * the branch-free recursion of Prop. 1 (Sherman-Morrison bordering, no
 * pivoting), in float64.  a: device [count][D][D] (only the upper triangle
 * is read); minv: device [count][D][D] (full symmetric result). 1 <= D <= 20. */
hgf_status hgf_spd_inverse(const double* a, double* minv, int32_t dim,
                           int32_t count, void* hip_stream);

/* Per-stage timing with HIP events, for measurement (off by default).  While
 * enabled, hgf_filter, hgf_guide_create and hgf_guide_filter record an event
 * before and after every kernel launch on the call's stream.
 * hgf_stage_times waits for the recorded events, writes for each stage id
 * s < max_stages the summed milliseconds ms[s] and the launch count
 * launches[s] (either may be NULL), and clears the record.  Stage ids:
 *   0 guidance means        1 guidance synthesis    2 guidance moment sums
 *   3 per-pixel inverse     4 coefficients (a4-a5)  5 output and WTA (a6-a7)
 *   6 WTA key fill/finalise */
#define HGF_NUM_STAGES 7
hgf_status hgf_set_stage_timing(hgf_context* ctx, int32_t enable);
hgf_status hgf_stage_times(hgf_context* ctx, double* ms, int32_t* launches,
                           int32_t max_stages);

const char* hgf_status_string(hgf_status status);
/* Detail string of the last failed call made with this context (NULL: of the
 * last failed call of this thread that took no context, e.g.
 * hgf_workspace_size).  Valid until the next call with the same context. */
const char* hgf_last_error(const hgf_context* ctx);

#ifdef __cplusplus
}
#endif

#endif /* HGF_H */
