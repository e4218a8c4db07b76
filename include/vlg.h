/*
 * vlg.h -- C ABI of the MI355X spatial model checker.
 *
 * Evaluates SLCS formulas (paper "A spatial model checker in GPU", Sect. 2,
 * Eq. def:syntax) pixel-wise over 2-D images on one AMD Instinct MI355X
 * (gfx950).  Every operator runs in hand-written HIP kernels on 1-bit-packed
 * masks; the host side only parses, plans and launches.
 *
 * Conventions
 *   - Every call returns an int status: VLG_OK (0) or a negative VLG_E* code.
 *     The message of the last failure on the calling thread is returned by
 *     vlg_last_error().  No C++ exception crosses this interface.
 *   - Handles (vlg_ctx, vlg_image, vlg_formula) are owned by the library and
 *     released by the matching *_free / vlg_destroy call.
 *   - A context is bound to one device and one HIP stream and is not
 *     thread-safe.  Formulas are immutable after compilation and may be used
 *     with any image and any context.
 *   - Work is enqueued asynchronously on the context's stream.  Results in
 *     device memory are complete once vlg_sync() returns (or once the caller
 *     synchronises that stream).  Calls that read or write host memory
 *     synchronise the stream before returning.
 *
 * Packed mask format (VLG_PACKED64): row-major uint64 words, wpr =
 * ceil(W/64) words per row, pixel (y, x) is bit (x % 64) of word
 * y*wpr + x/64 (least significant bit first); bits for x >= W are zero.
 * Size: H * wpr * 8 bytes.
 * Byte mask format (VLG_U8MASK): row-major uint8, one byte (0 or 1) per
 * pixel, H * W bytes.
 */
#ifndef VLG_H
#define VLG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define VLG_OK 0
#define VLG_EINVAL (-1)  /* bad argument (null handle, bad enum, index out of range) */
#define VLG_EPARSE (-2)  /* formula text does not parse; message has line and column */
#define VLG_ESHAPE (-3)  /* image shape/channel mismatch or size beyond limits */
#define VLG_ENOMEM (-4)  /* device or host allocation failed */
#define VLG_EHIP (-5)    /* a HIP runtime call failed */
#define VLG_ENOCONV (-6) /* a labelling loop stopped at its iteration cap (see
                            vlg_set_loop_cap); reported by the next call that
                            synchronises the context's stream */

/* ---- enums ---- */
#define VLG_F32 0        /* image pixel types */
#define VLG_U8 1
#define VLG_U16 2        /* the paper's pixel type (Sect. 3: 2-D uint16 images) */
#define VLG_HOST 0       /* where a caller buffer lives */
#define VLG_DEVICE 1
#define VLG_PACKED64 0   /* mask formats, see above */
#define VLG_U8MASK 1

/* Executor modes (vlg_set_mode).
 *   VLG_MODE_PEROP: one kernel launch per operator of the expanded formula,
 *     derived operators (interior, surrounded, grow) expanded into primitive
 *     operators as their definitions read, as the paper's tool schedules them
 *     (Sect. 3, Implementation details).
 *   VLG_MODE_FUSED: the same results with fewer launches and fewer bytes:
 *     all atoms of one channel read the channel once, negations are folded
 *     into the consuming kernel, interior is one erosion kernel, surrounded
 *     and grow run the reachability kernels without materialising their
 *     complemented operands.
 *   VLG_MODE_GRAPH: the fused schedule captured once per (formula, image,
 *     output buffers) as a hipGraph and replayed.  Default. */
#define VLG_MODE_PEROP 0
#define VLG_MODE_FUSED 1
#define VLG_MODE_GRAPH 2

typedef struct vlg_ctx vlg_ctx;
typedef struct vlg_image vlg_image;
typedef struct vlg_formula vlg_formula;

typedef struct vlg_formula_stats {
    int64_t parsed_nodes;   /* operator applications before hash-consing */
    int64_t nodes;          /* distinct DAG nodes after hash-consing: atoms,
                               true/false, !, &, |, N, interior, reach,
                               surrounded, grow each count as one */
    int64_t reach_nodes;    /* reach + surrounded + grow nodes */
    int64_t atoms;          /* threshold atoms (incl. percentile atoms) */
    int64_t outputs;        /* number of `output` statements */
    int64_t steps_perop;    /* kernel steps of the per-operator schedule */
    int64_t steps_fused;    /* kernel steps of the fused schedule */
    int64_t peak_masks;     /* peak live intermediate masks (fused schedule) */
    int64_t launches_fused; /* kernel launches of the fused schedule (batched
                               Boolean and near steps count once) */
    int64_t labellings;     /* connected-component labellings (fused schedule) */
    int64_t labelling_reuse;/* reach-type nodes served by an earlier labelling of
                               the same passable mask */
    int64_t segments;       /* fused segments (runs of Boolean and near steps
                               run by one tile kernel) at the default halo cap */
} vlg_formula_stats;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * enqueue on, or NULL for a stream owned by the context.  The library does not
 * take ownership of a caller stream. */
int vlg_create(vlg_ctx **out, int device, void *hip_stream);
void vlg_destroy(vlg_ctx *ctx);
/* Block until all work enqueued by this context has finished.  Returns
 * VLG_ENOCONV (and clears the condition) when a labelling loop of that work
 * stopped at its iteration cap: the outputs of the work enqueued since the
 * previous synchronisation are then not valid. */
int vlg_sync(vlg_ctx *ctx);
/* Iteration cap of every loop of the labelling kernels (union-find walks,
 * hooks and their retries, the root walks of the flag pass), per walk.  The
 * paper's labelling ends by a termination check after each iteration (Sect. 3,
 * Connected components labelling); here every device loop is bounded instead,
 * so that a labelling fault ends in an error code, never in a hang.  When a
 * walk reaches the cap it stops, the kernel exits normally with every array
 * still readable, and a flag is raised that the next synchronising call
 * (vlg_sync, a call with host outputs, a server request) turns into
 * VLG_ENOCONV.  cap >= 1; 0 restores the default (2^20, far above any walk of
 * a correct labelling). */
int vlg_set_loop_cap(vlg_ctx *ctx, int cap);
/* Select the executor mode (VLG_MODE_*); see above. */
int vlg_set_mode(vlg_ctx *ctx, int mode);

/* Copy an image into a device buffer owned by the library (paper Sect. 3:
 * images stay on the device and values are passed by buffer reference).
 *   data: pixels, channel-planar [channels][height][pitch], in host memory
 *     (where = VLG_HOST) or device memory (VLG_DEVICE, e.g. a torch tensor's
 *     data pointer); pitch_elems >= width is the row stride in elements (0
 *     means width).  dtype is VLG_F32, VLG_U8 or VLG_U16; every pixel type
 *     converts exactly to float32, the type atoms compare in.
 *   channels >= 1, height >= 0, width >= 0; height*width < 2^31.
 * The copy is complete when the call returns (host source) or in stream order
 * (device source): the caller may free a host source at once and a device
 * source after synchronising the context's stream. */
int vlg_load_image(vlg_ctx *ctx, const void *data, int dtype, int channels, int height, int width,
                   int64_t pitch_elems, int where, vlg_image **out);
int vlg_image_free(vlg_image *img);
/* Load a volume (a 3-D image: the logic on volumes, the extension the paper
 * names as its main limitation, Sect. 1, Sect. 3, Sect. 5): data is
 * [channels][depth][height][width], rows of width elements, dtype and
 * `where` as for vlg_load_image.  Formulas evaluate with N over the 26
 * voxels sharing a face, an edge or a vertex (the voxel included) and
 * 26-connected paths; atoms, percentiles and Boolean operators are voxel by
 * voxel.  Output masks of a volume are depth*height rows of packed words
 * (slice after slice), or depth*height*width bytes.  Volumes are evaluated
 * one at a time (vlg_check_batch rejects them), never with fused segments,
 * and label with the voxel union-find whatever VLG_TUNE_CCL_ALGO says.
 * Errors: as vlg_load_image; VLG_ESHAPE when depth*height*width >= 2^31. */
int vlg_load_volume(vlg_ctx *ctx, const void *data, int dtype, int channels, int depth, int height, int width,
                    int where, vlg_image **out);
int vlg_image_shape(const vlg_image *img, int *channels, int *height, int *width);
/* Shape of an image or volume: depth 1 and the image's height for images,
 * slices and rows per slice for volumes (vlg_image_shape reports a volume's
 * height as depth*height). */
int vlg_image_shape3(const vlg_image *img, int *channels, int *depth, int *height, int *width);

/* Parse and compile formula text (ImgQL subset, paper Sect. 3 Syntax):
 *   let NAME = expr | let NAME(p1, ..., pk) = expr | output "name" expr
 *   expr: e | e, e & e, !e, (e), true, false,
 *         intensity(img[, c]) CMP t with CMP one of >. <. >=. <=. and t a
 *         number or percentile(img, c, q),
 *         near(e) (also N(e)), interior(e), reach(a, b) = rho a[b],
 *         surrounded(a, b), grow(a, b), and calls of user macros.
 * Macros are expanded and identical sub-expressions become one DAG node
 * (hash-consing; & and | are commutative), as in the paper's memoised macro
 * expansion into a task DAG (Sect. 3, Implementation details).  On a parse
 * error returns VLG_EPARSE with "line L col C: ..." in vlg_last_error(). */
int vlg_compile_formula(vlg_ctx *ctx, const char *src, vlg_formula **out);
int vlg_formula_info(const vlg_formula *f, vlg_formula_stats *stats);
/* The kernel schedule of every output of f as JSON text (an "explain" of the
 * plan; no device work): mode VLG_MODE_PEROP or VLG_MODE_FUSED, fuse_halo
 * the segment halo cap of the fused schedule (see VLG_TUNE_FUSE_HALO).
 * {"nslots", "npct", "noutputs", "steps": [{"kind", "x"/"y"/"z": [slot, inv],
 * "out", "op", "inv_out", "chan", "user", "group", "seg", "q": [[q, scalar]],
 * "atoms": [[cmp, use_pct, thr, scalar, out]]}], "segments": [{"halo",
 * "nregs", "inputs", "outputs", "ins": [[op, dst, a, b, inv]]}]}; mask slot
 * -1 is the zero mask, slots <= -2 are outputs -2-k.  Writes at most len bytes
 * (NUL included) to buf; *needed (if not NULL) receives the size needed; with
 * len = 0 only the size is reported. */
int vlg_formula_plan(const vlg_formula *f, int mode, int fuse_halo, char *buf, int64_t len, int64_t *needed);
/* Name of output `index` (pointer valid while f lives), or NULL. */
const char *vlg_formula_output_name(const vlg_formula *f, int index);
int vlg_formula_free(vlg_formula *f);

/* Model checking of one formula on one image (paper Sect. 2: the satisfaction
 * relation of Eq. def:syntax, pixel by pixel; Sect. 3: one kernel per
 * operator over whole images, with reachability through connected components;
 * Sect. 4.2, Fig. specification: the saved result is the mask of the pixels
 * that satisfy a formula).
 * Evaluate output `output_index` of f on img and write the mask to `out_mask`
 * (caller-owned, format fmt, in host or device memory).  Only the DAG nodes
 * that output needs are evaluated.  Device outputs complete in the order of
 * the context's stream (work of other streams on the same buffers must be
 * ordered against it by the caller); host outputs are complete on return.
 * Errors: VLG_EINVAL (null handle, bad index, format or memory kind),
 * VLG_ESHAPE (the formula reads a channel the image lacks), VLG_ENOMEM,
 * VLG_EHIP; with host outputs also VLG_ENOCONV (see vlg_sync). */
int vlg_check(vlg_ctx *ctx, const vlg_formula *f, const vlg_image *img, int output_index,
              void *out_mask, int fmt, int where);
/* Evaluate every output of f on img in one pass (shared sub-expressions are
 * evaluated once, as the paper's memoised task DAG does, Sect. 3,
 * Implementation details).  outs[i] receives output i; a NULL entry skips it.
 * Same formats, completion rules and errors as vlg_check. */
int vlg_check_all(vlg_ctx *ctx, const vlg_formula *f, const vlg_image *img, void *const *outs,
                  int fmt, int where);
/* Evaluate every output of f on each of n images (sizes may differ): the
 * satisfaction relation of Sect. 2 per image, as vlg_check_all.
 * outs[i * n_outputs + k] receives output k of image i (NULL skips it).
 * In fused and graph mode the batch runs as one launch per schedule step for
 * all images of a pixel type (persistent kernels over per-image descriptors,
 * each image with its own workspace region); in per-op mode the images are
 * evaluated one after another.  Same completion rules and errors as
 * vlg_check_all. */
int vlg_check_batch(vlg_ctx *ctx, const vlg_formula *f, const vlg_image *const *imgs, int n,
                    void *const *outs, int fmt, int where);

/* Connected-component labelling of a packed device mask (8-connectivity, the
 * labelling the paper uses to compute reachability, Sect. 3).  labels_dev is a
 * device int32 [height][width] array; each foreground pixel receives the
 * smallest row-major index y*width+x of its component, background -1.  Runs on
 * the context's stream. */
int vlg_ccl_labels(vlg_ctx *ctx, const uint64_t *mask_dev, int height, int width,
                   int32_t *labels_dev);

/* For callers that cannot allocate device memory during a call (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same labelling as vlg_ccl_labels, with the same arguments, result and
 * errors, but its labelling arrays live in a fixed device array of
 * VLG_NOALLOC_SCRATCH_BYTES that each GPU holds from the library's load until
 * the process ends; the call allocates nothing.  The array needs
 * 9 * ceil(height/2) * ceil(width/2) bytes plus alignment (4096 x 4096 fits);
 * a larger image fails with VLG_ESHAPE and a message, before any work is
 * enqueued.  Every call on one GPU, from any context or thread, shares that
 * GPU's array and leaves its contents behind (the next call rewrites what it
 * reads): calls that overlap on one GPU race, so the caller orders them (for
 * example on one stream).  The result completes in the order of the
 * context's stream, as with vlg_ccl_labels. */
#define VLG_NOALLOC_SCRATCH_BYTES (40ll << 20)
int vlg_ccl_labels_noalloc(vlg_ctx *ctx, const uint64_t *mask_dev, int height, int width,
                           int32_t *labels_dev);

/* Connected-component labelling of a packed device volume mask of depth
 * slices of height x width (26-connectivity, the labelling behind
 * reachability on volumes).  labels_dev is a device int32
 * [depth][height][width] array; each voxel of the mask receives the
 * smallest linear index (z*height + y)*width + x of its component,
 * background -1.  Runs on the context's stream; VLG_ENOCONV (at vlg_sync)
 * when a union-find walk stopped at the loop cap. */
int vlg_ccl_labels3(vlg_ctx *ctx, const uint64_t *mask_dev, int depth, int height, int width,
                    int32_t *labels_dev);

/* Counters of the last reachability labelling run on ctx (for measurement):
 * union attempts and retry iterations of the cross-tile merge, and the
 * number of kernel launches per labelling. */
typedef struct vlg_ccl_counters {
    int64_t merge_unions;
    int64_t merge_retries;
    int64_t launches_per_ccl;
    /* pointer-jumping labellings (VLG_CCL_POINTER_JUMPING) since the last
     * read: labellings, main iterations, rounds (reconnect + termination
     * check), kernel launches */
    int64_t pj_labellings;
    int64_t pj_main_iterations;
    int64_t pj_rounds;
    int64_t pj_launches;
} vlg_ccl_counters;
int vlg_ccl_read_counters(vlg_ctx *ctx, vlg_ccl_counters *out);

/* The paper's own labelling algorithm (Sect. 3, Alg. CCL, Fig. cc-movie) on
 * a packed device mask: labels are coordinate pairs (row, column) ordered
 * lexicographically; initialization labels each pixel of the mask with its
 * coordinates; a main iteration gives each pixel holding (i', j') the
 * largest label in the Moore neighbourhood of (i', j') (pointer jumping,
 * from one label array into the other); every `reconnect_every` main
 * iterations (1..64; 0 = the context's VLG_TUNE_PJ_RECONNECT, default 16 as
 * in the paper's text; its figure uses 8) a reconnect writes, at the pixel a
 * pixel points to, the largest label around that pixel when it is larger
 * (atomic maximum over the writers), and the termination check looks for
 * two neighbouring pixels of the mask with different labels.  The host
 * waits for the check after every round, as the paper's tool does.
 * labels_dev (device int32 [height][width]) receives, for each pixel of the
 * mask, the row-major index y*width+x of its component's largest pixel, -1
 * for background.  stats (optional) receives the main iterations, rounds
 * and launches.  height and width must be below 65535 (VLG_ESHAPE);
 * VLG_ENOCONV when the check still fails after the context's loop cap of
 * rounds (vlg_set_loop_cap). */
typedef struct vlg_pj_stats {
    int64_t main_iterations;
    int64_t rounds;
    int64_t launches;
} vlg_pj_stats;
int vlg_ccl_labels_pj(vlg_ctx *ctx, const uint64_t *mask_dev, int height, int width, int reconnect_every,
                      int32_t *labels_dev, vlg_pj_stats *stats);

/* Measurement.  Runs the fused schedule of every output of f on img `iters`
 * times, one launch at a time, with a HIP event recorded on the context's
 * stream before and after each step, and reports per kernel kind its number
 * of launches, total time and algorithmic bytes (what the operator must read
 * and write: image channels, input and output masks, labelling arrays).
 * Writes at most max_out entries and the number of kinds to *n_out. */
typedef struct vlg_kernel_time {
    char name[32];   /* "atoms", "logic", "near", "ccl_local", "ccl_merge",
                        "ccl_flag", "ccl_gather", "percentile" */
    int64_t launches;
    double ms;       /* total over all launches */
    double bytes;    /* algorithmic bytes over all launches */
} vlg_kernel_time;
int vlg_profile(vlg_ctx *ctx, const vlg_formula *f, const vlg_image *img, int iters, vlg_kernel_time *out,
                int max_out, int *n_out);
/* The same per-kind table for the batched executor (vlg_check_batch in
 * fused mode, no graph): HIP events around every launch of the batched
 * schedule of every output of f on the n images (one pixel type, no
 * volumes), `iters` times; bytes are the steps' algorithmic bytes summed over
 * the images.  Outputs go to the library's own mask slots.  Synchronises the
 * stream. */
int vlg_profile_batch(vlg_ctx *ctx, const vlg_formula *f, const vlg_image *const *imgs, int n, int iters,
                      vlg_kernel_time *out, int max_out, int *n_out);
/* Measurement of one kernel without per-launch events: enqueues the fused
 * schedule (one labelling at a time) of every output of f on img up to and
 * including its first single (ungrouped) step of `kind` ("atoms", "logic",
 * "near", "ccl_local", "ccl_merge", "ccl_flag", "ccl_gather", "segment" or
 * "arith"), then that step `reps` times back to back between two HIP events
 * on the context's stream.  A merge or flag step repeated alone would find
 * its work done, so for those the repeated unit starts at the labelling's
 * tile-local pass, and the same unit without the step is timed too and
 * subtracted.  *avg_ms receives the mean time of one launch of the step,
 * *bytes its algorithmic bytes (as in vlg_profile).  Synchronises the
 * stream.  VLG_EINVAL when the schedule has no such step or labels with the
 * pointer-jumping schedule. */
int vlg_profile_step(vlg_ctx *ctx, const vlg_formula *f, const vlg_image *img, const char *kind, int reps,
                     double *avg_ms, double *bytes);
/* Measurement: the HBM reference.  Copies `bytes` (a multiple of width) from
 * src_dev to dst_dev (device buffers, not overlapping) in width-byte units
 * (8 or 16), non-temporal loads and stores, once as a warm-up and then
 * `reps` times back to back between two HIP events on the context's stream;
 * *avg_ms receives the mean time of one copy (bytes read + bytes written
 * per copy).  Synchronises the stream. */
int vlg_stream_copy(vlg_ctx *ctx, void *dst_dev, const void *src_dev, int64_t bytes, int width, int reps,
                    double *avg_ms);

/* Tunables of the executor.  Each has a default, may be forced for a
 * context, and is otherwise looked up per image shape class (ceil(log2 H),
 * ceil(log2 W)) in the context's table, which vlg_autotune fills (batches:
 * per batch class, filled by vlg_autotune_batch).
 *   VLG_TUNE_CCL_TILE_ROWS: block rows (2x2 pixels each) per labelling tile:
 *     8, 16 or 32; tiles are 128 pixels wide.  Taller tiles do more work in
 *     LDS and leave fewer tile borders to merge globally.  Default: the
 *     tallest height that leaves at least 1024 tiles (counted over the whole
 *     batch for vlg_check_batch), else 8.
 *   VLG_TUNE_NEAR_ROWS: rows per band of the near kernel: 4, 8, 16 or 32
 *     (default: from the image size).  Taller bands reload fewer halo rows,
 *     shorter ones give more parallel bands.
 *   VLG_TUNE_BATCH_GRID: workgroups of a persistent batched launch: 1024,
 *     2048, 4096 or 8192 (default).
 *   VLG_TUNE_CCL_LANES: labellings run together, 1, 2, 4 or 8 (default 1).
 *     With L > 1 the fused schedule groups up to L independent labellings
 *     that are ready together into one region, each with its own labelling
 *     workspace, and each phase of the union-find labelling (tile-local
 *     pass, merge, flag, gather) runs for all of them in one launch on the
 *     context's stream.  Needs L labelling workspaces.
 *   VLG_TUNE_FUSE_HALO: fused segments of the fused schedule: runs of
 *     consecutive Boolean and near steps that one tile kernel evaluates with
 *     every intermediate mask in LDS, the tile extended by a halo as deep as
 *     the segment's longest chain of near steps.  The value is the largest
 *     halo allowed (2, 4, 8 or 16 rows); 1 (the default) forms no segments:
 *     on the measured workloads segments only paid off where the autotuner
 *     picks them.
 *   VLG_TUNE_CCL_ALGO: the labelling behind reach-type nodes (Sect. 3:
 *     reachability through connected components).  VLG_CCL_UNION_FIND
 *     (default): union-find over 2x2 blocks in fixed launches, no host wait.
 *     VLG_CCL_POINTER_JUMPING: the paper's Alg. CCL as vlg_ccl_labels_pj
 *     runs it, with the host waiting for the termination check after every
 *     round; an evaluation that labels with it is therefore never captured
 *     as a graph (graph mode runs it launch by launch), and images need
 *     rows and columns below 65535.  vlg_check_batch always uses union-find.
 *   VLG_TUNE_PJ_RECONNECT: main iterations between reconnects of the
 *     pointer-jumping labelling, 1..64 (default 16).
 *   VLG_TUNE_ARITH: the kernel of arithmetic atoms.  VLG_ARITH_COMPILED
 *     (default): the programs of a launch compiled with hipRTC into a
 *     straight-line kernel the first time they run (about a second per
 *     distinct group of programs, then kept until the process ends; a group
 *     that does not compile runs on the interpreter).
 *     VLG_ARITH_INTERPRETER: one precompiled kernel that decodes the
 *     programs.  Both give the same bits. */
#define VLG_TUNE_CCL_TILE_ROWS 0
#define VLG_TUNE_NEAR_ROWS 1
#define VLG_TUNE_BATCH_GRID 2
#define VLG_TUNE_CCL_LANES 3
#define VLG_TUNE_FUSE_HALO 4
#define VLG_TUNE_CCL_ALGO 5
#define VLG_TUNE_PJ_RECONNECT 6
#define VLG_TUNE_ARITH 7
#define VLG_CCL_UNION_FIND 1      /* values of VLG_TUNE_CCL_ALGO */
#define VLG_CCL_POINTER_JUMPING 2
#define VLG_ARITH_INTERPRETER 1   /* values of VLG_TUNE_ARITH */
#define VLG_ARITH_COMPILED 2
/* Force `value` for every image (value 0 returns to table/default). */
int vlg_set_tunable(vlg_ctx *ctx, int which, int value);
/* The value used for an image of height x width on this context. */
int vlg_get_tunable(vlg_ctx *ctx, int which, int height, int width, int *value);

typedef struct vlg_tune_report {
    int which;          /* VLG_TUNE_* */
    int best;           /* chosen value, stored for the image's shape class */
    int n;              /* candidates tried */
    int candidates[8];
    double ms[8];       /* mean time of one evaluation of f on img per candidate */
} vlg_tune_report;
/* Autotuner: evaluate every output of f on img `iters` times per candidate
 * value of each tunable that applies (labelling tile rows when f has a
 * reach-type node, near band rows when it has a near step; fused schedule,
 * HIP events on the context's stream), one tunable after the other, and
 * store the fastest value for img's shape class.  Writes one report per
 * tunable tried to out[0 .. max_out-1]; *n_out receives their number. */
int vlg_autotune(vlg_ctx *ctx, const vlg_formula *f, const vlg_image *img, int iters, vlg_tune_report *out,
                 int max_out, int *n_out);
/* Autotuner for batches: evaluate every output of f on the n images with the
 * batched schedule (as vlg_check_batch in fused mode) `iters` times per
 * candidate of the labelling tile rows (when f has a reach-type node) and of
 * the persistent grid size, and store the fastest values for the batch class
 * (ceil(log2 n), ceil(log2 of the mean pixels per image)); vlg_check_batch
 * then uses them for batches of that class (otherwise the tile rows of its
 * largest image's shape class and the default grid).  Outputs go to internal
 * buffers.  Same reports as vlg_autotune. */
int vlg_autotune_batch(vlg_ctx *ctx, const vlg_formula *f, const vlg_image *const *imgs, int n, int iters,
                       vlg_tune_report *out, int max_out, int *n_out);
/* Save / load the context's tuning table as JSON lines
 * {"arch": "gfx950", "tunable": ..., "h_class": ..., "w_class": ..., "value": ...}
 * with tunable "ccl_tile_rows", "near_band_rows" or "batch_grid" (suffix
 * "_batch" for batch classes, whose two class numbers are the batch and
 * mean-image classes); loading keeps only the entries of the context's
 * device architecture. */
int vlg_tune_save(vlg_ctx *ctx, const char *path);
int vlg_tune_load(vlg_ctx *ctx, const char *path);

/* Serving loop: continuous batching of evaluation requests on one device.
 * nslots worker slots each own a context (its own stream); a request
 * (formula, resident image, device output buffers, packed format) is admitted
 * to a free slot in arrival order once its HBM footprint (live masks,
 * labelling and percentile workspace) fits in what remains of
 * hbm_budget_bytes, reserved from one device pool.  Requests admitted to
 * different slots run concurrently on the device.  A request whose footprint
 * exceeds the whole budget completes at once with VLG_ENOMEM.  Functions are
 * thread-safe; submit never blocks on device work. */
typedef struct vlg_server vlg_server;
typedef struct vlg_server_stats {
    int64_t submitted, completed, rejected;
    int64_t max_inflight;        /* most requests running at once */
    int64_t max_queued;          /* most requests waiting for admission */
    int64_t peak_reserved_bytes; /* most pool bytes reserved at once */
    int64_t budget_bytes;
} vlg_server_stats;
int vlg_server_create(vlg_server **out, int device, int nslots, int64_t hbm_budget_bytes);
/* Device workspace one evaluation of every output of f on img needs (the
 * footprint the server reserves at admission), in bytes. */
int vlg_evaluation_bytes(const vlg_formula *f, const vlg_image *img, int64_t *bytes);
/* outs[k]: packed device buffer of output k (NULL skips it); valid until the
 * request completes, and with no write pending on another stream when
 * submitted (slot streams do not wait for other streams).  *request_id
 * identifies the request for vlg_server_wait. */
int vlg_server_submit(vlg_server *s, const vlg_formula *f, const vlg_image *img, void *const *outs,
                      int64_t *request_id);
/* Block until the request completes; returns its status.  queue_ms: submit to
 * admission; run_ms: admission to completion (outputs written).  Each id can
 * be waited for once. */
int vlg_server_wait(vlg_server *s, int64_t request_id, double *queue_ms, double *run_ms);
int vlg_server_read_stats(vlg_server *s, vlg_server_stats *out);
/* Finish every submitted request, stop the slots, release the pool. */
int vlg_server_destroy(vlg_server *s);

/* Message of the last failed call on this thread ("" if none). */
const char *vlg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VLG_H */
