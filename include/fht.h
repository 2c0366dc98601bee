/*
 * fht.h -- C ABI of the MI355X (gfx950) Fast Hough Transform library, libfht.so.
 *
 * The transform is Brady's dyadic Fast Hough Transform in the form studied by
 * Aliev, Ershov and Nikolaev (arXiv 1811.06378): sums of an image along all
 * dyadic linear patterns, with the paper's zero extension (section 3.1), the
 * four angle quadrants concatenated into one full Hough image (section 3.3),
 * the angle-range modification that shears the image inside the first
 * iteration (section 4) and the fhtshift regrouping (section 5).
 *
 * Conventions.
 *   Image I: h rows x w columns, element (x, y) at img[y * ld_img + x].
 *   h' = 2^ceil(log2 h), w' = 2^ceil(log2 w), W = w' + h'.  Both sides are
 *   padded with zeros to the next power of two and the image is extended by
 *   h' zero columns (w' for the transposed image), so every quadrant has W
 *   columns and patterns never wrap into the image (section 3.1).
 *   D_n(s, y) is the column offset at row y of the dyadic pattern with shift s
 *   over n rows: the top half uses shift s>>1, the bottom half uses s>>1 and
 *   starts s - (s>>1) columns further (section 2; section 4, Fig. 6).
 *   Quadrant 1 [315;0]:  H1[s,x] = sum_y P [y, (x + D_h'(s,y)) mod W], s < h'
 *   Quadrant 2 [0;45]:   H2[s,x] = sum_y P [y, (x - D_h'(s,y)) mod W], s < h'
 *   Quadrant 3 [45;90]:  H3[s,x] = sum_c Pt[c, (x - D_w'(s,c)) mod W], s < w'
 *   Quadrant 4 [90;135]: H4[s,x] = sum_c Pt[c, (x + D_w'(s,c)) mod W], s < w'
 *   (P = padded I, Pt = padded transpose of I.)
 *   Full image (section 3.3): [flip(H1); H2[1:]; flip(H3)[1:]; H4[1:]], i.e.
 *   2(w'+h')-3 rows of W columns.  Hough cell (x0, r) is at
 *   hough[r * ld_hough + x0].
 *
 * Memory and streams.  Every image, Hough and workspace pointer is a DEVICE
 * pointer owned by the caller; the library never frees or retains it.  Work
 * is enqueued on `stream` (a hipStream_t; NULL = the default stream) and the
 * call returns without synchronising.  No entry point allocates device memory
 * except fht_batch_plan_create.  Scratch space comes from the caller's
 * workspace, sized by the matching *_workspace_size query.
 *
 * Errors.  Every entry point validates its arguments before any HIP call.  On
 * a negative status nothing has been enqueued and nothing written.  A launch
 * failure returns FHT_ERR_HIP.  fht_last_error() returns a per-thread message
 * for the last failure.
 *
 * Element types.  Allowed (input, accumulator) pairs: (FHT_U8, FHT_I32),
 * (FHT_I32, FHT_I32), (FHT_F32, FHT_F32).  Integer results are exact while
 * every partial sum fits in int32 (uint8 input: always, since 255 * 65536 <
 * 2^31).  Float results use only binary32 additions in the stage order of the
 * recurrence, so they are reproducible bit for bit.
 */
#ifndef FHT_H
#define FHT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum fht_status {
    FHT_OK = 0,
    FHT_ERR_INVALID = -1,     /* bad pointer, size, leading dimension or flag */
    FHT_ERR_UNSUPPORTED = -2, /* valid request the library does not implement */
    FHT_ERR_WORKSPACE = -3,   /* workspace missing or smaller than required */
    FHT_ERR_HIP = -4,         /* a HIP runtime call or launch failed */
    FHT_ERR_TIMEOUT = -5      /* fht_engine_status: a bounded dependency wait of the
                                 opt-in persistent engine (FHT_ENGINE=1) gave up */
};

enum fht_dtype { FHT_U8 = 0, FHT_I32 = 1, FHT_F32 = 2 };

/* Quadrant selection.  FHT_FULL (all four bits) produces the merged full image
 * of section 3.3; any other non-empty subset produces the selected quadrants
 * unmerged and unflipped, stacked in increasing quadrant order. */
enum { FHT_Q1 = 1, FHT_Q2 = 2, FHT_Q3 = 4, FHT_Q4 = 8, FHT_FULL = 15 };

/* fht_forward / fht_adjoint flags.
 * FHT_FLAG_SHIFTED: output (forward) or input (adjoint) is fhtshift-ed.
 * FHT_FLAG_MAX (fht_forward only): each Hough cell is the maximum, not the
 *   sum, of the padded image along its pattern; the transform generalises to
 *   any associative, commutative operation (section 1).  Same patterns, same
 *   shapes and layout; the zero padding takes part in the maximum, and on a
 *   0/1 image the result is the logical OR.  Exact in every dtype.  The
 *   adjoint rejects it (FHT_ERR_INVALID). */
enum { FHT_FLAG_SHIFTED = 1, FHT_FLAG_MAX = 2 };

/* Largest supported side (pow2-padded): 65536. */
#define FHT_MAX_SIDE 65536

int fht_version(void);
const char* fht_status_string(int status);
const char* fht_last_error(void);

/*
 * Shape of the Hough image for an h x w image and a quadrant selection
 * (section 3.1 sizes; section 3.3 full size 2(w+h)-3).  Host-only, pure.
 * FULL -> (2(w'+h')-3, W); Q1 or Q2 alone -> (h', W); Q3 or Q4 -> (w', W);
 * other subsets -> the sum of the selected rows, W columns.
 * Returns FHT_ERR_INVALID for w < 1, h < 1, an empty/unknown selection, null
 * outputs or sides above FHT_MAX_SIDE.
 */
int fht_hough_shape(int w, int h, unsigned quads, int64_t* rows, int64_t* cols);

/*
 * Shape of the angle-range transform (section 4): (S+1, W).
 * Requires 0 <= S <= n-1 and |S1| <= n-1, n = h' (w' when transposed).
 */
int fht_range_shape(int w, int h, int S1, int S, int transposed, int64_t* rows, int64_t* cols);

/* Workspace bytes needed by fht_forward / fht_adjoint / fht_range. */
int fht_workspace_size(int w, int h, unsigned quads, int in_t, int acc_t, size_t* bytes);
int fht_range_workspace_size(int w, int h, int S1, int S, int transposed, int in_t, int acc_t,
                             size_t* bytes);
int fht_adjoint_workspace_size(int w, int h, unsigned quads, int t, size_t* bytes);

/*
 * Forward FHT (sections 3.1 and 3.3; fhtshift of section 5 with
 * FHT_FLAG_SHIFTED; the max transform of section 1 with FHT_FLAG_MAX).
 *   img       device, h x w elements of in_t, row pitch ld_img >= w (elements)
 *   hough     device, rows x cols of acc_t from fht_hough_shape, row pitch
 *             ld_hough >= cols; every cell is written
 *   workspace device, >= fht_workspace_size bytes, 256-byte aligned; its
 *             contents on entry are ignored and on exit undefined
 *   stream    hipStream_t or NULL
 * img and hough must not overlap.
 */
int fht_forward(const void* img, int in_t, int w, int h, int64_t ld_img, void* hough, int acc_t,
                int64_t ld_hough, unsigned quads, unsigned flags, void* workspace,
                size_t ws_bytes, void* stream);

/*
 * fht_forward of a stack of n same-size images in one set of launches (the
 * image index runs on the launch grid): image i at img + i * img_stride
 * elements (img_stride >= h * ld_img when n > 1), its Hough image at
 * hough + i * hough_stride elements (hough_stride >= rows * ld_hough when
 * n > 1).  Every other argument as fht_forward; results equal n calls of
 * fht_forward bit for bit.  Images run in groups whose bands fit 8 GiB; the
 * workspace (>= fht_forward_stack_workspace_size, 256-byte aligned) holds
 * one single-image workspace (rounded up to 256 bytes) per image of a group.
 */
int fht_forward_stack_workspace_size(int w, int h, unsigned quads, int in_t, int acc_t, int n, size_t* bytes);
int fht_forward_stack(const void* img, int in_t, int w, int h, int64_t ld_img, int64_t img_stride, int n,
                      void* hough, int acc_t, int64_t ld_hough, int64_t hough_stride, unsigned quads,
                      unsigned flags, void* workspace, size_t ws_bytes, void* stream);

/*
 * Allocation-free forward, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as fht_forward, without
 * the workspace: the scratch (intermediate bands) is a file-scope device
 * array of FHT_NOALLOC_SCRATCH_BYTES that the library's code object holds on
 * every GPU it runs on until the process ends; its address is looked up once
 * per device, on that device's first call.  The call allocates nothing,
 * frees nothing and calls no allocating routine.
 *   Limit: transforms whose fht_workspace_size exceeds
 *   FHT_NOALLOC_SCRATCH_BYTES return FHT_ERR_UNSUPPORTED (the full image of
 *   a 2048 x 1024 image fits, for every dtype; 2048 x 2048 does not).
 *   Sharing: every call on one GPU uses that GPU's one array, whose contents
 *   are left from the last call (no call relies on them).  Calls that overlap
 *   in time on one GPU (two streams, two threads, or a graph replay beside an
 *   eager call) race on it: order them on one stream or use fht_forward.
 */
#define FHT_NOALLOC_SCRATCH_BYTES (64u << 20)
int fht_forward_noalloc(const void* img, int in_t, int w, int h, int64_t ld_img, void* hough, int acc_t,
                        int64_t ld_hough, unsigned quads, unsigned flags, void* stream);

/*
 * Angle-range transform (section 4).  Shifts s = 0..S of quadrant 1 (quadrant
 * 4 of the transposed image when transposed != 0) computed on the image whose
 * row y is read cyclically pre-shifted right by
 *   sigma(y) = floor((2*y*S1 + (n-1)) / (2*(n-1)))   (n = h' or w'),
 * inside the first stage, without a sheared copy.  Row s then holds the sums
 * along patterns of slope (s - S1)/(n-1) columns per row; stages compute only
 * the shifts that some output row s <= S depends on.
 *   hough  device, (S+1) x W of acc_t, pitch ld_hough >= W.
 * Requirements as for fht_range_shape.
 */
int fht_range(const void* img, int in_t, int w, int h, int64_t ld_img, int S1, int S,
              int transposed, void* hough, int acc_t, int64_t ld_hough, void* workspace,
              size_t ws_bytes, void* stream);

/*
 * fhtshift of a full Hough image (section 5), or its inverse.  Row r of local
 * shift s in quadrant q is rolled right cyclically by
 *   q1: floor((h'+s)/2)  q2: floor((h'-s)/2)  q3: floor((w'-s)/2)  q4: floor((w'+s)/2)
 * (left by the same amounts when inverse != 0), which centres each row's
 * meaningful run of w'+s (vertical) or h'+s (horizontal) cells.
 *   in, out  device, (2(w'+h')-3) x W of t (FHT_I32 or FHT_F32), pitches
 *            ld_in, ld_out >= W.  out == in (same pitch) rolls in place and
 *            needs W * 4 <= 163840; other overlaps are invalid.
 */
int fht_shift(const void* in, int64_t ld_in, void* out, int64_t ld_out, int t, int w, int h,
              int inverse, void* stream);

/*
 * Adjoint (transpose) of fht_forward: grad_img = F^T grad_hough, i.e. every
 * Hough cell's value is added back onto the pixels of its pattern (dyadic
 * back-projection), cropped to the h x w image; with FHT_FULL the dropped
 * duplicate junction rows contribute nothing.  Used as the backward of the
 * forward transform.
 *   grad_hough device, shape of fht_hough_shape(w, h, quads) of t, pitch
 *              ld_hough; fhtshift-ed when flags has FHT_FLAG_SHIFTED
 *   grad_img   device, h x w of t, pitch ld_img >= w; fully overwritten (the
 *              first quadrant's contribution is stored, the later ones are
 *              added to it in place, in quadrant order)
 *   t          FHT_I32 or FHT_F32 (the accumulator type of the forward)
 * The workspace holds the intermediate bands.
 */
int fht_adjoint(const void* grad_hough, int t, int64_t ld_hough, void* grad_img, int64_t ld_img,
                int w, int h, unsigned quads, unsigned flags, void* workspace, size_t ws_bytes,
                void* stream);

/*
 * fht_adjoint of a stack of n same-size gradients (the backward of a stack
 * of images): one launch per pass kind covers a whole group of images (as
 * many as keep their bands within 2 GiB, at most 8192), so small images fill
 * the chip together where one alone leaves it mostly idle.
 * Image i's gradient starts grad_stride elements after image i-1's
 * (grad_stride >= rows * ld_hough when n > 1), and its output img_stride
 * elements after (img_stride >= h * ld_img when n > 1).  Every other
 * argument as fht_adjoint; results equal n calls of fht_adjoint bit for bit.
 * The workspace (>= fht_adjoint_stack_workspace_size, 256-byte aligned)
 * holds one single-image workspace (rounded up to 256 bytes) per image of a
 * group.
 */
int fht_adjoint_stack_workspace_size(int w, int h, unsigned quads, int t, int n, size_t* bytes);
int fht_adjoint_stack(const void* grad_hough, int t, int64_t ld_hough, int64_t grad_stride,
                      void* grad_img, int64_t ld_img, int64_t img_stride, int w, int h, int n,
                      unsigned quads, unsigned flags, void* workspace, size_t ws_bytes, void* stream);

/*
 * Angle range of the image scaled along the sheared axis by alpha = num/den
 * (section 4: a scale in the first iteration maps [-arctg(1/alpha); 0] onto
 * [-45; 0], and the shear then selects the range).  The paper fixes no
 * resampling rule; here the scaled image has ceil(alpha * w) columns (rows
 * when transposed) and sample x is the source sample floor(x * den / num)
 * (nearest sample; alpha > 1 repeats samples, alpha < 1 skips them).  The
 * result is fht_range of that scaled image: shape and workspace from the
 * two helpers below, which take the unscaled w, h.  num, den in 1..64.
 * img is the unscaled h x w image; everything else as fht_range.
 */
int fht_range_scaled_shape(int w, int h, int num, int den, int S1, int S, int transposed, int64_t* rows,
                           int64_t* cols);
int fht_range_scaled_workspace_size(int w, int h, int num, int den, int S1, int S, int transposed, int in_t,
                                    int acc_t, size_t* bytes);
int fht_range_scaled(const void* img, int in_t, int w, int h, int64_t ld_img, int num, int den, int S1, int S,
                     int transposed, void* hough, int acc_t, int64_t ld_hough, void* workspace, size_t ws_bytes,
                     void* stream);

/*
 * Adjoint of fht_range (transpose of the angle-range transform of section 4):
 * the gradient of rows 0..S goes back through the transposed stages to the
 * padded source sheared by sigma(y), is read back at the unsheared columns,
 * and is cropped to the image (transposed back when transposed = 1).
 *   grad      device, (S+1) x W of t (FHT_I32 or FHT_F32), row pitch ld_grad
 *   grad_img  device, h x w of t, row pitch ld_img >= w; overwritten
 *   workspace >= fht_range_adjoint_workspace_size bytes, 256-byte aligned
 * Same S1, S, transposed limits as fht_range; grad and grad_img must not
 * overlap.  Integer gradients are exact: <R x, g> = <x, R^T g>.
 */
int fht_range_adjoint_workspace_size(int w, int h, int S1, int S, int transposed, int t, size_t* bytes);
int fht_range_adjoint(const void* grad, int t, int64_t ld_grad, int S1, int S, int transposed, void* grad_img,
                      int64_t ld_img, int w, int h, void* workspace, size_t ws_bytes, void* stream);

/*
 * Batched forward over many images of different sizes (many independent
 * transforms of sections 3.1 and 3.3).  Each image is transformed as by
 * fht_forward(quads, flags = 0) into its own slice of one packed output
 * buffer.  The plan fixes, once, every pass of every quadrant of every image;
 * a call enqueues one small table-resolving kernel and then one launch per
 * (pass, stages, last-pass) class covering every tile of every image in that
 * class.  All work is kernel launches on the caller's stream, so a call can
 * be captured in a hipGraph and replayed.  Images are processed in chunks
 * whose intermediate bands fit 8 GiB, which bounds the workspace.
 *
 * fht_batch_plan_create: ws[i], hs[i] are the n image sizes (host arrays),
 *   any sides from 1 to FHT_MAX_SIDE; quadrants of at most 4 rows run as
 *   one thread per Hough cell inside the same plan.  FHT_ERR_UNSUPPORTED if
 *   one launch class of one chunk would exceed 2^31 work items.  Allocates
 *   the plan's device tables (the only allocating entry point) on the
 *   current device; with up to 2^26 tile items they include an item ->
 *   group map (environment FHT_BATCH_MAP=0 at plan creation leaves it out:
 *   the kernels then search the group table).  *ws_bytes receives the
 *   workspace size, *out_elems the total number of output elements;
 *   out_offsets (host, n entries, may be NULL) receives each image's element
 *   offset in the packed output (each image's Hough image is stored densely,
 *   ld_hough = W_i).
 * fht_batch_forward: imgs is a DEVICE array of n device pointers (image i
 *   dense, ld = w_i); hough is the packed output; workspace is 256-byte
 *   aligned, at least *ws_bytes.  A plan is immutable: concurrent calls on
 *   different streams need their own workspace.
 * fht_batch_forward_stack: as fht_batch_forward for a plan of n equal
 *   sizes (FHT_ERR_INVALID otherwise), with image i dense at base +
 *   i * stride_bytes (stride_bytes >= one image when n > 1): no device
 *   pointer array, so nothing is copied from the host per call.
 * fht_batch_plan_destroy: frees the plan's tables (NULL is a no-op).
 */
typedef struct fht_batch_plan fht_batch_plan;
int fht_batch_plan_create(const int32_t* ws, const int32_t* hs, int n, unsigned quads, int in_t,
                          int acc_t, fht_batch_plan** plan, size_t* ws_bytes, int64_t* out_elems,
                          int64_t* out_offsets);
int fht_batch_forward(const fht_batch_plan* plan, const void* const* imgs, void* hough,
                      void* workspace, size_t ws_bytes, void* stream);
int fht_batch_forward_stack(const fht_batch_plan* plan, const void* base, int64_t stride_bytes, void* hough,
                            void* workspace, size_t ws_bytes, void* stream);
int fht_batch_plan_destroy(fht_batch_plan* plan);

/*
 * From a Hough cell back to the image (sections 3.2 and 3.3), host only.
 * row, x0: a cell of the Hough image of an h x w image with quads = FHT_FULL
 * (row in 0..2(w'+h')-4, attributed to its quadrant by the row order of
 * section 3.3) or a single quadrant (row = shift); shifted = 1 if the image
 * was fhtshift-ed (full image only).  The cell's dyadic pattern is walked row
 * by row on the padded source with cyclic columns (cases a and b of
 * section 3.2); seg[0..3] receive the image coordinates (x, y) of its first
 * and last pixel inside the image and seg[4] the number of such pixels.
 * seg[4] = 0: the pattern lies in the zero extension only (case c, the black
 * zone); seg[0..3] are then 0.  Mostly horizontal quadrants (3, 4) give
 * their pattern along image columns.
 */
int fht_cell_segment(int w, int h, unsigned quads, int64_t row, int64_t x0, int shifted, int32_t* seg);

/*
 * Local maxima of a Hough image (t = FHT_I32 or FHT_F32, rows x cols, pitch
 * ld, device): cells with value > threshold that are the strict maximum of
 * their (2 radius + 1)^2 neighbourhood, cyclic in columns and clipped in
 * rows; equal values are ordered by linear index (row * cols + col), so a
 * plateau yields one cell.  The linear indices of the first max_out maxima
 * found are written to out (device, unordered) and *count (device, unsigned)
 * receives the total number found, which may exceed max_out.  radius in
 * 1..64 and 2 radius + 1 <= cols.  Asynchronous on stream.
 */
int fht_peaks(const void* hough, int t, int64_t rows, int64_t cols, int64_t ld, int radius, double threshold,
              int64_t* out, int max_out, unsigned* count, void* stream);

/*
 * Launch timing (instrumentation, not part of the method).  fht_timing_enable
 * (1) clears previous records and starts recording: every pass kernel the
 * library enqueues afterwards (forward, range, adjoint and batched passes) is
 * bracketed by two HIP events on its launch stream; launches inside a stream
 * capture are not recorded.  fht_timing_enable(0) stops recording.
 * fht_timing_report(index, ...) waits for the recorded events and returns,
 * for the index-th kernel instantiation seen (in first-launch order), its
 * name as "fht::<kernel><template arguments>" (copied into name, at most
 * name_cap bytes with the terminator), the number of launches and their
 * summed elapsed time in milliseconds; FHT_ERR_INVALID past the last one.
 * The device is the one current at fht_timing_enable(1).
 * fht_timing_filter(substr) restricts recording to the kernels whose name
 * contains substr (NULL or "" records every kernel again); the string is
 * copied, at most 255 bytes.  Each pair of events delays the next launch by
 * a few microseconds, so timing only the kernel of interest disturbs the
 * rest of the stream less.
 */
int fht_timing_enable(int on);
int fht_timing_filter(const char* substr);
int fht_timing_report(int index, char* name, int name_cap, int64_t* launches, double* total_ms);

/*
 * Stage-fusion depth.  A quadrant of n = 2^k rows runs its k stages in the
 * fewest passes of at most 6 stages; how the stages are split among the
 * passes is a free choice (each pass 3..6 stages).  By default two passes
 * put as many stages as they can in the first (the second keeps at least 3:
 * 1024 rows run 6+4) and three or more are as even as possible, larger first
 * (8192 rows: 5+4+4).  fht_set_pass_split sets the split used for k from now
 * on by every call in the process (npass = 0 restores the default; npass must
 * be the fewest passes, each entry 3..6, summing to k; k in 3..16).
 * fht_autotune times every candidate split for the stage counts of an h x w
 * full transform (dtype pair in_t/acc_t) with HIP events on `stream`, `reps`
 * calls each, on buffers it allocates and frees itself (it synchronises; not
 * for the hot path), and keeps the fastest with fht_set_pass_split.  Splits
 * change band widths: query workspace sizes after tuning (a call with a
 * short workspace returns FHT_ERR_WORKSPACE).  Results are bit-identical for
 * every split: the additions of each stage do not depend on the grouping.
 */
int fht_set_pass_split(int k, int npass, const int* passes);
int fht_autotune(int w, int h, int in_t, int acc_t, int reps, void* stream);

/*
 * Error state of the opt-in persistent engine (environment FHT_ENGINE=1 at
 * the first call in the process): a forward call run by the engine waits
 * for the tiles of a quadrant's previous pass with a bounded spin
 * (FHT_SPIN_LIMIT iterations, default 2^21) and, if a wait gives up, marks
 * word 1 of its workspace and carries on, so the kernel always ends.  This
 * call waits for `stream` and reads that word for the last engine call on
 * `workspace`: FHT_ERR_TIMEOUT if a wait gave up (that call's results are
 * invalid), FHT_OK otherwise.  It synchronises the stream; not for the hot
 * path.  Without the engine the word is never written.
 */
int fht_engine_status(const void* workspace, void* stream);

/*
 * Tile height of the pass kernels.  A pass runs on tiles of 64 rows (8
 * waves, two workgroups per CU) or, for passes of at most 5 stages, 32 rows
 * (4 waves, half the LDS, four workgroups per CU): twice as many tiles,
 * which fills the chip at sizes whose passes have few tiles.  Results are
 * bit-identical either way (the same additions in the same order).  The
 * default rule is 32 rows for every pass of at most 5 stages.
 * fht_set_tile_rows sets the height used from now on for passes of at most 5
 * stages of quadrants with 2^k rows (rows = 32 or 64; 0 restores the default
 * rule; k in 3..16); passes of 6 stages always use 64.  fht_tile_rows
 * returns the height such passes use for a side.  fht_autotune also picks it.
 */
int fht_set_tile_rows(int k, int rows);
int fht_tile_rows(int side, int* rows);

/* Stage-fusion split chosen for a side (number of passes and stages per pass),
 * for inspection and tests.  passes[] receives up to 4 entries. */
int fht_pass_split(int side, int* npass, int* passes);

#ifdef __cplusplus
}
#endif

#endif /* FHT_H */
