/*
 * ct.h - C ABI of the MI355X contourlet transform library (libct.so).
 *
 * The contourlet transform (CT) of CVC: a Laplacian pyramid (LP) whose
 * bandpass image at every level is split by a directional filter bank (DFB)
 * into 2^l wedge-shaped subbands, iterated on the lowpass (paper section 2.1,
 * Fig. 1), with the 9-7 biorthogonal filters for both (section 2.1). The
 * output of a plane is the coarsest lowpass plus the directional subbands of
 * every scale (section 3.3). The lowpass is then normalised to [0, 255]
 * (section 3.4) and every coefficient is divided by a quantisation step and
 * rounded to the nearest integer (sections 3.5, 3.6).
 *
 * Conventions shared by every call
 *   - A "plane" is one H x W float32 image, row major. A batch is B planes
 *     stored back to back ([B][H][W]).
 *   - Coefficients of one plane form a packed float32 vector of `ncoef`
 *     entries ([B][ncoef] for a batch), laid out as described by
 *     ct_layout_query: the lowpass, then levels from coarse to fine, each
 *     level's subbands in direction order.
 *   - Data pointers are DEVICE pointers owned by the caller. The library never
 *     frees or retains them. It allocates no device memory in these calls:
 *     scratch space comes from the caller's workspace `ws` of `ws_bytes`
 *     bytes (at least ct_workspace_bytes()).
 *   - Every compute call only enqueues work on `stream` and returns without
 *     synchronising. Faults inside kernels surface at the caller's next
 *     synchronisation on that stream.
 *   - All argument and geometry validation happens on the host before any
 *     launch, so an error return means nothing was enqueued.
 *   - Return value: CT_OK (0) on success, a negative CT_ERR_* code otherwise.
 *     No call aborts, exits or throws across this boundary.
 *   - Calls are reentrant. Two calls that share output or workspace buffers
 *     must be ordered by the caller (same stream, or events).
 */
#ifndef CT_H_
#define CT_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CT_MAX_LEVELS 6

enum {
    CT_OK = 0,
    CT_ERR_ARG = -1,          /* null pointer, batch < 0, bad sizes          */
    CT_ERR_GEOM = -2,         /* geometry outside the supported range        */
    CT_ERR_WORKSPACE = -3,    /* workspace smaller than ct_workspace_bytes() */
    CT_ERR_HIP = -4,          /* a HIP runtime call failed                   */
    CT_ERR_UNSUPPORTED = -5   /* valid request this build does not serve     */
};

/*
 * Geometry of one plane.
 *   height, width  unpadded plane size (each >= 2^e, see ct_layout).
 *   levels         J, number of LP levels, 1..6 (section 3.3).
 *   dirs[j]        directional subbands at LP level j+1; dirs[0] is the
 *                  finest level. Each a power of two in [4, 64] (2^l wedges
 *                  at DFB level l, section 2.1). Entries at j >= levels are
 *                  ignored.
 *   filters        CT_FILTERS_CDF97 (0): the 9-7 pair of section 2.1 for the
 *                  LP and the fan filters of the DFB. CT_FILTERS_LEGALL53
 *                  (1): the LeGall 5/3 pair in both places, a variant (same
 *                  construction with two zeros at pi instead of four).
 *   recon          CT_RECON_DUAL (0): the dual-frame LP synthesis, which
 *                  removes the part of a bandpass error the lowpass channel
 *                  sees. CT_RECON_BURT_ADELSON (1): x = d + upsampled c, the
 *                  original pyramid's reconstruction, a variant. Both invert
 *                  the forward transform exactly; they differ on quantised
 *                  coefficients. The forward transform ignores `recon`.
 *   A zero-initialised struct with height, width, levels and dirs set is the
 *   paper's transform. Other values of filters or recon are CT_ERR_GEOM.
 */
typedef struct ct_geom {
    int32_t height, width;
    int32_t levels;
    int32_t dirs[CT_MAX_LEVELS];
    int32_t filters;
    int32_t recon;
} ct_geom;

enum {
    CT_FILTERS_CDF97 = 0,
    CT_FILTERS_LEGALL53 = 1,
    CT_RECON_DUAL = 0,
    CT_RECON_BURT_ADELSON = 1
};

/*
 * Derived layout of one plane.
 *   pad_h, pad_w   R, C: the periodic working size. Each side is rounded up
 *                  to a multiple of 2^e, e = max(J, max_j (j + log2 dirs_j - 2)).
 *                  The extra rows/columns mirror the plane about its last
 *                  sample (x[H+i] = x[H-1-i]); the inverse crops them off.
 *   exp2           e.
 *   ncoef          coefficients per plane = sum of all subband sizes.
 *   nsub           1 + sum_j dirs[j] (entry 0 is the lowpass).
 */
typedef struct ct_layout {
    int32_t pad_h, pad_w;
    int32_t exp2;
    int32_t nsub;
    int64_t ncoef;
} ct_layout;

/*
 * One subband of the packed layout.
 *   level      LP level j (1 = finest); the lowpass has level = J + 1.
 *   k          direction index within the level (-1 for the lowpass). Order:
 *              by wedge angle atan2(w1, w2) over (-45, 135) degrees:
 *              horizontal cone (|w2| > |w1|) first, then vertical cone.
 *   rows, cols natural size of the subband array.
 *   offset     first element within the plane's packed vector.
 *   o1, o2     lattice offset of sample (0, 0) in level-j image coordinates.
 *   s1, s2     lattice steps: sample (i, k) is level pixel (o1 + s1 i, o2 + s2 k).
 *   transposed 1 if stored as the transpose of the natural array (row major
 *              cols x rows): the vertical-cone subbands.
 */
typedef struct ct_subband {
    int32_t level, k;
    int32_t rows, cols;
    int64_t offset;
    int32_t o1, o2;
    int32_t s1, s2;
    int32_t transposed;
    int32_t reserved;
} ct_subband;

/*
 * Host-only query of the layout (no GPU needed).
 * Fills *out, and the first min(cap, nsub) entries of `table` (table may be
 * NULL when cap is 0). Returns CT_ERR_ARG for null geom/out, CT_ERR_GEOM for
 * an unsupported geometry.
 */
int ct_layout_query(const ct_geom* geom, ct_layout* out, ct_subband* table, int32_t cap);

/*
 * Workspace needed by ct_forward/ct_inverse/ct_quantize and the adjoints for
 * `batch` planes, in bytes (host only). Writes 0 and returns an error code
 * on bad input.
 */
int ct_workspace_bytes(const ct_geom* geom, int32_t batch, size_t* bytes);

/*
 * Forward CT (encoder, sections 2.1 and 3.3).
 *   planes  [batch][H][W] float32 input.
 *   coeffs  [batch][ncoef] float32 output, packed layout.
 */
int ct_forward(const ct_geom* geom, int32_t batch, const float* planes, float* coeffs,
               void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Inverse CT (decoder): exact inverse of ct_forward on unquantised
 * coefficients; LP reconstruction uses the dual frame (c' = c - H d,
 * x = d + G up(c')).
 *   coeffs  [batch][ncoef] float32 input.
 *   planes  [batch][H][W] float32 output (padding cropped).
 */
int ct_inverse(const ct_geom* geom, int32_t batch, const float* coeffs, float* planes,
               void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Quantise (sections 3.4-3.6). Per plane b:
 *   lowpass (subband 0): mn = min, mx = max over the plane's lowpass;
 *     s = 255/(mx - mn) (s = 0 when mx == mn); q = round(((c - mn) * s) / step[0])
 *   directional subband i >= 1: q = round(c / step[i])
 *   round = nearest, halves away from zero; saturated to int16; NaN -> 0.
 * All arithmetic in IEEE float32, in exactly this order, correctly rounded.
 *   steps       device float32 [batch][steps_stride] step table per plane; entry
 *               i of a row is the step of subband i (ct_subband order). Use
 *               steps_stride = 0 to share one row of nsub steps by all planes.
 *               Steps must be finite and > 0.
 *   idx         [batch][ncoef] int16 output.
 *   side        [batch][2] float32 output: (mn, mx) of each plane's lowpass.
 */
int ct_quantize(const ct_geom* geom, int32_t batch, const float* coeffs, const float* steps,
                int32_t steps_stride, int16_t* idx, float* side,
                void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * ct_quantize without a workspace, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same arguments, arithmetic and results as ct_quantize,
 * minus ws/ws_bytes. Its scratch (the lowpass min/max partials, 2 KiB per
 * plane) is a static device array that each GPU holds until the process
 * ends, sized for at most 1024 planes: a larger batch returns
 * CT_ERR_WORKSPACE with nothing enqueued. The call allocates nothing. Every
 * call on one GPU shares that GPU's array: calls that overlap in time on one
 * GPU (unordered streams) race and must be ordered by the caller.
 */
int ct_quantize_noalloc(const ct_geom* geom, int32_t batch, const float* coeffs,
                        const float* steps, int32_t steps_stride, int16_t* idx, float* side,
                        hipStream_t stream);

/*
 * Dequantise (the decoder side of sections 3.4-3.5):
 *   directional  c = q * step[i]
 *   lowpass      c = mn + (q * step[0]) * ((mx - mn) / 255)
 * float32, in this order.
 */
int ct_dequantize(const ct_geom* geom, int32_t batch, const int16_t* idx, const float* steps,
                  int32_t steps_stride, const float* side, float* coeffs, hipStream_t stream);

/*
 * Fused encoder and decoder: the same computations as ct_forward followed by
 * ct_quantize, and ct_dequantize followed by ct_inverse, with the float
 * coefficients kept out of HBM (paper section 3: the CT feeds the quantiser
 * directly, and the decoder the inverse CT).
 * ct_encode rounds every directional coefficient to its index where the DFB
 * produces it, with the quantiser's float32 operations on the value that
 * ct_forward would store, then quantises the lowpass (which needs its plane
 * min/max first) in two small passes. Its idx and side equal those of
 * ct_forward + ct_quantize bit for bit. `coeffs` may be NULL; when given it
 * also receives the float coefficients of ct_forward.
 * ct_decode dequantises where the inverse CT loads the subbands and the
 * lowpass, with ct_dequantize's float32 operations; its output equals
 * ct_dequantize + ct_inverse bit for bit.
 * Arguments and workspace as for the separate calls.
 */
int ct_encode(const ct_geom* geom, int32_t batch, const float* planes, const float* steps,
              int32_t steps_stride, int16_t* idx, float* side, float* coeffs,
              void* ws, size_t ws_bytes, hipStream_t stream);
int ct_decode(const ct_geom* geom, int32_t batch, const int16_t* idx, const float* steps,
              int32_t steps_stride, const float* side, float* planes,
              void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Fused encoder from 8-bit RGB frames (section 3.1 front end, then section 3
 * as ct_encode): the colour transform of equations (1)-(3) happens where the
 * first LP level loads its rows, so neither the float planes nor the
 * coefficients reach HBM. Results equal ct_rgb_to_ycocg with n = 1 followed
 * by ct_encode on the 3 * frames planes ordered frame by frame as Y,
 * Co + 127, Cg + 127, bit for bit.
 *   frames     F >= 0 frames (3 * F <= 65535, 3 * F * H * W < 2^40), else
 *              CT_ERR_ARG; F = 0 enqueues nothing.
 *   rgb        uint8 [F][H][W][3], R, G, B interleaved (H, W from geom), no
 *              alignment needed.
 *   steps      as ct_encode, for batch 3 * F (steps_stride > 0: one row per
 *              plane, plane 3 f + k is channel k of frame f).
 *   idx, side  as ct_encode: [3 F][ncoef] int16 and [3 F][2] float.
 *   ws         ct_workspace_bytes(geom, 3 * F) bytes.
 * The chroma planes are full size: subsampled chroma (n > 1) goes through
 * ct_rgb_to_ycocg and ct_encode on the smaller planes.
 */
int ct_encode_rgb(const ct_geom* geom, int32_t frames, const uint8_t* rgb, const float* steps,
                  int32_t steps_stride, int16_t* idx, float* side, void* ws, size_t ws_bytes,
                  hipStream_t stream);

/*
 * Transposes for the differentiable form (gradients through the CT).
 * ct_forward_adjoint computes F^T g: gcoeffs [batch][ncoef] -> gplanes [batch][H][W].
 * ct_inverse_adjoint computes S^T g: gplanes [batch][H][W] -> gcoeffs [batch][ncoef].
 * The frame is not tight, so F^T differs from the inverse S.
 */
int ct_forward_adjoint(const ct_geom* geom, int32_t batch, const float* gcoeffs, float* gplanes,
                       void* ws, size_t ws_bytes, hipStream_t stream);
int ct_inverse_adjoint(const ct_geom* geom, int32_t batch, const float* gplanes, float* gcoeffs,
                       void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Batched form: many streams of uneven resolution and LP depth run one pass
 * of the hot path (forward CT, quantise, dequantise, inverse CT) in one graph
 * launch. Each stream is `batch` planes of one geometry with its
 * own caller-owned device buffers:
 *   planes  [batch][H][W] float32 input
 *   coeffs  [batch][ncoef] float32 forward output
 *   idx     [batch][ncoef] int16 quantiser indices
 *   side    [batch][2] float32 lowpass (min, max)
 *   steps   step table as for ct_quantize (steps_stride 0: one shared row)
 *   deq     [batch][ncoef] float32 dequantised coefficients
 *   out     [batch][H][W] float32 reconstruction
 * ct_plan_create validates every stream, allocates the plan's own workspace
 * and stage tables (the only device allocations of this library), and lays
 * the work out in groups: the stages of one type at one chain position of
 * all streams, run by one launch that covers all their tiles. The groups
 * follow in chain order on one stream. With CT_PLAN_GRAPH the group launches
 * are captured into one HIP graph. With CT_PLAN_AUTOTUNE it runs the tuner
 * of ct_autotune on every stream's geometry; without it, a plan takes the
 * choices an earlier tuning in this process made for its shapes, else the
 * defaults.
 * ct_plan_run enqueues one graph launch (or the group launches) on `stream`.
 * ct_plan_run_plain enqueues the same work as separate per-stream,
 * per-stage launches (the unbatched baseline); both give identical results.
 * A plan may not run on two streams at once; buffers are read and written
 * on every run. ct_plan_destroy waits for nothing: synchronise first.
 */
typedef struct ct_stream_desc {
    ct_geom geom;
    int32_t batch;
    const float* planes;
    float* coeffs;
    int16_t* idx;
    float* side;
    const float* steps;
    int32_t steps_stride;
    float* deq;
    float* out;
} ct_stream_desc;

typedef struct ct_plan ct_plan;

typedef struct ct_plan_info_t {
    int32_t streams, stages, work_items, launches;
    int32_t graph, autotuned;
    int32_t levels_paired, levels_single;   /* LP levels with l >= 4 whose deeper tree levels run */
    int32_t levels_triple;                  /* two, one or three per pass (the tuned choice)   */
    int64_t workspace_bytes;
    int32_t levels_short_blocks;            /* LP levels whose split passes aim at twice or half */
    int32_t levels_tall_blocks;             /* the default wavefronts (the tuned choice), or run */
    int32_t levels_sized_blocks;            /* blocks of explicit rows                           */
} ct_plan_info_t;

#define CT_PLAN_GRAPH 1
#define CT_PLAN_AUTOTUNE 2
#define CT_PLAN_FUSED 4     /* fused encoder and decoder (as ct_encode, ct_decode): deq is not
                               written and may be NULL, coeffs only when not NULL */

int ct_plan_create(const ct_stream_desc* streams, int32_t n, int32_t flags, ct_plan** out);
int ct_plan_run(ct_plan* plan, hipStream_t stream);
int ct_plan_run_plain(ct_plan* plan, hipStream_t stream);
int ct_plan_info(const ct_plan* plan, ct_plan_info_t* info);
void ct_plan_destroy(ct_plan* plan);

/*
 * Tile-shape autotuning of the DFB split passes. For every LP level of `geom`
 * with three or more DFB tree levels, times (HIP events on `stream`, waiting
 * for them on the host) the level's split passes, analysis then synthesis, for
 * every combination of tree levels per streaming pass (one, two or three) and
 * row-block height (the default, the heights aiming at twice or half as many
 * wavefronts, and heights that cut the tallest parent channel into 2..10 equal
 * blocks), and keeps the fastest; a choice cached in the JSON file
 * CT_AUTOTUNE_CACHE (default $HOME/.cache/ct_autotune.json) for this device
 * architecture and shape is taken without timing. The choices go into a
 * per-process table, keyed by device, level shape and batch, that later
 * ct_forward, ct_inverse, their adjoints, ct_encode, ct_decode and plans
 * without CT_PLAN_AUTOTUNE read. Every choice computes the same operations in
 * the same order: results are identical with and without tuning.
 *   ws, ws_bytes  a workspace of ct_workspace_bytes(geom, batch), used as
 *                 scratch (its contents are overwritten).
 * Returns CT_OK, CT_ERR_ARG, CT_ERR_GEOM, CT_ERR_WORKSPACE or CT_ERR_HIP.
 * ct_autotune_clear empties the per-process table (the defaults again).
 */
int ct_autotune(const ct_geom* geom, int32_t batch, void* ws, size_t ws_bytes, hipStream_t stream);
int ct_autotune_clear(void);

/*
 * Encoder front end and decoder back end (paper section 2.3, Table I;
 * section 3.1). These calls take sizes instead of a ct_geom; they follow the
 * other conventions above (device pointers owned by the caller, enqueue only,
 * validation before any launch, CT_ERR_* returns) and need no workspace.
 *   batch, height, width  B frames of H x W pixels (B >= 0, H, W >= 1), with
 *                         3 * B * H * W < 2^31, else CT_ERR_ARG.
 *   n                     chroma subsampling factor, 1..CT_MAX_CHROMA_FACTOR
 *                         (1 keeps every sample). Chroma planes are
 *                         Hc x Wc with Hc = ceil(H / n), Wc = ceil(W / n).
 *   rgb (forward)         uint8 [B][H][W][3], R, G, B interleaved, 4-byte
 *                         aligned.
 *   y                     float32 [B][H][W] luminance planes, 16-byte
 *                         aligned: the layout ct_forward / ct_encode take.
 *   co, cg                float32 [B][Hc][Wc] chroma planes.
 * ct_rgb_to_ycocg applies equations (1)-(3) to every pixel, writes Y, and
 * writes Co + 127 and Cg + 127 at the samples (n i, n j) (section 3.1: chroma
 * kept at every n-th row and column and moved into [0, 255] by +127; exactly,
 * equations (2)-(3) reach +-127.5, so values lie in [-0.5, 254.5]). Every
 * result is exact in float32 (quarter integers below 2^10).
 * ct_ycocg_to_rgb is the decoder side: for pixel (r, c) it interpolates each
 * chroma plane bilinearly between samples floor(r / n), floor(c / n) and the
 * next ones (the last sample repeated past the edge) with weights
 * (r mod n) / n and (c mod n) / n, subtracts 127, and applies equations
 * (4)-(6). Output rgb float32 [B][H][W][3] interleaved, 16-byte aligned,
 * neither rounded nor clamped. float32 arithmetic, weights from 1/n rounded
 * to float32.
 */
#define CT_MAX_CHROMA_FACTOR 64
int ct_rgb_to_ycocg(int32_t batch, int32_t height, int32_t width, int32_t n, const uint8_t* rgb,
                    float* y, float* co, float* cg, hipStream_t stream);
int ct_ycocg_to_rgb(int32_t batch, int32_t height, int32_t width, int32_t n, const float* y,
                    const float* co, const float* cg, float* rgb, hipStream_t stream);

/*
 * K-frame lowpass filtering (paper section 3.7), in place on the int16
 * indices of ct_quantize / ct_encode (idx [batch][ncoef], batch * ncoef <
 * 2^31). Only each plane's lowpass (subband 0: rows x cols at offset 0, row
 * major) changes.
 *   inverse = 0  every element below the first row becomes its difference
 *                with the element above it in the input;
 *   inverse != 0 the running sums down every column, undoing the above.
 * Differences and sums wrap modulo 2^16 (two's complement int16), so the
 * pair restores any input exactly; for the quantiser's lowpass indices
 * (0..255) no wrap occurs and the differences are the exact ones.
 */
int ct_lowpass_diff(const ct_geom* geom, int32_t batch, int16_t* idx, int32_t inverse,
                    hipStream_t stream);

/*
 * Full-search block-matching motion estimation on luminance (paper section
 * 3.2). Conventions as above; no workspace.
 *   batch, height, width  B frame pairs of H x W pixels (B >= 0, H, W >= 1,
 *                         B * H * W < 2^31).
 *   w                     search range, 1..16: displacements (dy, dx) with
 *                         |dy|, |dx| <= w, (2w + 1)^2 candidates.
 *   cur, prev             float32 [B][H][W]: plane b of `cur` is matched
 *                         against plane b of `prev` (for a clip of frames
 *                         F, pass F[1:] and F[:-1]). Values are taken on
 *                         the 8-bit scale in steps of 1/4, as
 *                         ct_rgb_to_ycocg produces them: rounded to the
 *                         nearest quarter (halves to even), clamped to
 *                         [0, 255].
 *   mv                    int16 [B][nby][nbx][2] output, nby = ceil(H/16),
 *                         nbx = ceil(W/16): (dy, dx) of each 16 x 16 block
 *                         (edge blocks cropped to the frame). Block (y, x)
 *                         of cur matches the block at (y + dy, x + dx) of
 *                         prev, which lies wholly inside the frame.
 *   ssd                   int32 [B][nby][nbx] output, or NULL: the winning
 *                         sum of squared differences of 4 Y (16 times that
 *                         of Y; the MSE is ssd / (16 * block pixels)).
 * The winner is the smallest sum (equivalently MSE), ties broken by the
 * smallest |dy| + |dx|, then dy, then dx: the result is exact and unique.
 */
int ct_motion_search(int32_t batch, int32_t height, int32_t width, int32_t w, const float* cur,
                     const float* prev, int16_t* mv, int32_t* ssd, hipStream_t stream);

/*
 * Host-only view of ct_motion_search's work layout for search range w
 * (1..16), as the kernel computes it (for inspection and tests).
 *   layout  int32 [6] output: LDS row pitch of the window pairs (words), offset
 *           of the odd-column copy, offset of the block, words per wavefront,
 *           tasks per window row, and 1 if a full block's last pass runs as
 *           half-tasks on lane pairs.
 *   rows,   int32 [cap] outputs: window row and first column offset of the
 *   sa      first cap tasks (a task is the candidates (row, sa) and
 *           (row, sa + 2), the second one only when sa + 2 <= 2w).
 * Returns the number of tasks, or CT_ERR_ARG.
 */
int ct_motion_layout_query(int32_t w, int32_t* layout, int32_t* rows, int32_t* sa, int32_t cap);

/*
 * P-frame components (paper section 3.7): the motion-compensated prediction
 * is made on the quantised CT components, with the luminance motion vectors
 * of ct_motion_search mapped to each component's scale. Conventions as
 * above; no workspace.
 *   cur, prev   int16 [batch][ncoef] indices of the current and previous
 *               frames (ct_quantize / ct_encode layout).
 *   mv, nby,    int16 [ceil(batch / mv_group)][nby][nbx][2] block vectors
 *   nbx,        (dy, dx) of ct_motion_search; plane b uses field
 *   mv_group    b / mv_group (3 for the Y, Co, Cg planes of one frame).
 *   n           chroma subsampling factor of the planes (1 for luminance).
 * A sample (i, k) of a subband of level j with lattice offset (o1, o2) and
 * steps (s1, s2) (ct_subband) sits at luminance pixel
 * n 2^(j-1) (o1 + s1 i, o2 + s2 k), a lowpass sample at n 2^J (i, k); it
 * takes the vector of the 16 x 16 block holding that pixel (the last block
 * row / column for the padding), divided by its sample spacing n 2^(j-1)
 * (s1, s2) (n 2^J for the lowpass) and rounded to the nearest integer,
 * halves away from zero. The prediction is the previous plane's component
 * at the displaced position in its natural orientation, modulo the
 * component's size.
 *   inverse = 0   out = cur - prediction (encoder)
 *   inverse != 0  out = cur + prediction (decoder: cur holds the P-frame
 *                 components, out the frame's indices)
 * Arithmetic modulo 2^16, so the pair is exact on any input. out may be cur
 * (in place), not prev.
 */
int ct_mc_residual(const ct_geom* geom, int32_t batch, int32_t n, const int16_t* cur,
                   const int16_t* prev, const int16_t* mv, int32_t nby, int32_t nbx,
                   int32_t mv_group, int32_t inverse, int16_t* out, hipStream_t stream);

/*
 * Zero-run coding (paper section 3.8) of quantised indices, on the device.
 * Every component is read along its natural rows (image rows; the
 * transposed vertical-cone subbands along their stored columns). In a coded
 * component a non-zero value is one int16 symbol, itself, and a maximal run
 * of n zeros inside a row is the two symbols 0, n. K-frames (p_frame = 0)
 * code the directional subbands and copy the lowpass unchanged; P-frames
 * (p_frame != 0) code every component.
 *   idx       int16 [batch][ncoef] input.
 *   symbols   int16 [batch][2 ncoef] output; plane b's stream starts at
 *             symbols + b 2 ncoef (2 ncoef bounds any stream).
 *   sub_off   int32 [batch][nsub + 1] output: the symbol offset of every
 *             component within its plane's stream, then the plane's count.
 *   ws        workspace of ct_rle_workspace_bytes() bytes.
 * ct_rle_decode_host is the decoder (host code, one plane, host pointers):
 * symbols holds sub_off[nsub] symbols. It checks first that sub_off starts
 * at or above 0 and never decreases, then parses every component's rows, and
 * returns CT_ERR_ARG for offsets or a stream that do not parse to exactly the
 * layout; it reads no symbol outside [sub_off[0], sub_off[nsub]).
 */
int ct_rle_workspace_bytes(const ct_geom* geom, int32_t batch, size_t* bytes);
int ct_rle_encode(const ct_geom* geom, int32_t batch, const int16_t* idx, int32_t p_frame,
                  int16_t* symbols, int32_t* sub_off, void* ws, size_t ws_bytes, hipStream_t stream);
int ct_rle_decode_host(const ct_geom* geom, const int16_t* symbols, const int32_t* sub_off,
                       int32_t p_frame, int16_t* idx);

/*
 * DEFLATE of one plane's symbol stream (paper section 3.9), host code
 * (zlib, compression level 0..9). mode 0 compresses every component on its
 * own (transmission scalability: comp_bytes[s] for each of the nsub
 * components, back to back in out); mode 1 compresses the whole plane at
 * once (CVC-NTS: comp_bytes[0]). The symbols are taken as little-endian
 * int16 bytes. *total receives the bytes written; CT_ERR_WORKSPACE if cap
 * is too small (cap = sum of compressBound over the parts always suffices).
 * ct_inflate_host is the inverse; it needs sub_off to size every part, and
 * `in` holds the sum of comp_bytes over the parts. Both return CT_ERR_ARG
 * when sub_off is negative or decreasing (checked before any access).
 */
int ct_deflate_host(const int16_t* symbols, const int32_t* sub_off, int32_t nsub, int32_t mode,
                    int32_t level, uint8_t* out, size_t cap, uint32_t* comp_bytes, size_t* total);
int ct_inflate_host(const uint8_t* in, const uint32_t* comp_bytes, const int32_t* sub_off,
                    int32_t nsub, int32_t mode, int16_t* symbols);

/*
 * Per-kernel timing (HIP events), for benchmarks and tracing.
 * ct_profile_enable(1) creates a pool of `max_launches` event pairs (0 picks
 * 16384) and makes every later launch record one event before and one after
 * itself on its stream; ct_profile_enable(0) stops recording and releases
 * the pool. Recording adds two event packets per launch and allocates
 * nothing on the device.
 * ct_profile_collect waits for the recorded events, aggregates them by
 * kernel (name, launches, total milliseconds, compulsory bytes = inputs read
 * once + outputs written once, and alg_bytes = the part of those that are the
 * codec's own inputs and outputs: frames, float coefficients when the call
 * writes or reads them, indices; workspace intermediates excluded), writes
 * up to `cap` entries, sets *n to the
 * number of kernels seen, and clears the record. Returns CT_ERR_HIP if an
 * event query fails, CT_ERR_UNSUPPORTED if launches were dropped because
 * the pool ran out.
 */
typedef struct ct_kernel_stat {
    char name[32];
    int64_t launches;
    double total_ms;
    double bytes;
    double alg_bytes;
} ct_kernel_stat;
int ct_profile_enable(int32_t on, int32_t max_launches);
int ct_profile_collect(ct_kernel_stat* out, int32_t cap, int32_t* n);

/* Human-readable text for a CT_ERR_* code (static storage). */
const char* ct_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* CT_H_ */
