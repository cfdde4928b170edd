/*
 * thin.h -- C ABI of the MI355X (gfx950) lambda-leveling library.
 *
 * The library lowers the lambda-destructible points of a grayscale image
 * until the image is stable: the lambda-leveling loop of Couprie-Bertrand
 * grayscale topological thinning, as defined in section 2.1 of Mahmoudi,
 * Akil and Matas, "Parallel image thinning through topological operators on
 * shared memory parallel machines" (the lambda-destructible point, the
 * lowering target alpha-, and the "repeat until stability" loop of the
 * algorithm box in section 2.2 with the type set lambda-destructible).
 * The same loop with the algorithm box's own type set (lambda-deletable and
 * not lambda-end) gives the lambda-skeleton (thin_skeleton, THIN_OP_SKELETON).
 * thin_gradient computes the gradient image the paper thins in its Fig. 1
 * (a Deriche gradient magnitude), so the whole illustrated pipeline runs on
 * the GPU.
 *
 * Conventions shared by every call:
 *   - An image is a caller-owned DEVICE buffer of h rows by w columns,
 *     row-major, element type uint8 (THIN_U8) or uint16 (THIN_U16), row pitch
 *     `pitch_elems` elements (w when contiguous).  It is processed IN PLACE:
 *     on return it holds the stable image.  The library never frees it.
 *   - Gray levels are the image's own integers (F maps pixels to integers,
 *     section 2.1); lambda is in the same units and any uint32 value is valid.
 *   - Adjacency pair (n, n') for sections and their complements (section 2.1):
 *     THIN_ADJ_8_4 = (8,4), THIN_ADJ_4_8 = (4,8).
 *   - The 1-pixel frame of the image is never modified (the paper's F lives
 *     on Z^2; a finite image needs a border rule, and a read-only frame gives
 *     every processed pixel a full 3x3 neighbourhood inside the image).
 *     Images with h < 3 or w < 3 have no interior: the call returns THIN_OK,
 *     leaves them unchanged and reports passes = 0.
 *   - The order of lowering is fixed (the paper selects a point of minimal
 *     value without a tie-break): pass p visits the parity classes
 *     (i mod 2, j mod 2) = (0,0), (0,1), (1,0), (1,1) in that order on
 *     absolute 0-based (row, column); each class is lowered all at once,
 *     which equals lowering it pixel by pixel because two pixels of one class
 *     are never 8-adjacent.  Stability is a whole pass without lowering.
 *     The result, pass count and lowering count are therefore deterministic
 *     and do not depend on tiling, launch shape or batching.
 *   - Calls are synchronous with respect to the host: they return after the
 *     result is in the caller's buffer.  Work is enqueued on the stream given
 *     in thin_config (NULL = the null stream), so it orders after earlier
 *     work on that stream.
 *   - A context is not thread-safe: use one per host thread.
 *   - Error codes (negative) leave the image untouched for THIN_EINVAL and
 *     THIN_ENOMEM; after THIN_EDEVICE its contents are unspecified; after
 *     THIN_ELIMIT it holds the state after the last complete pass (a valid
 *     resume point: calling again continues to the same final image).
 */
#ifndef THIN_H
#define THIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    THIN_OK = 0,
    THIN_EINVAL = -1,   /* NULL pointer with h*w > 0, negative size, bad dtype, adjacency or
                           operator, pitch < w */
    THIN_ENOMEM = -2,   /* scratch above max_device_bytes, or a device allocation failed */
    THIN_EDEVICE = -3,  /* a HIP call failed */
    THIN_ELIMIT = -4,   /* max_passes reached before stability */
    THIN_EBUSY = -5     /* serving: admission would exceed the device-memory budget */
};

enum { THIN_U8 = 1, THIN_U16 = 2 };
enum { THIN_ADJ_8_4 = 0, THIN_ADJ_4_8 = 1 };

/* Operators (thin_image.op).  Both lower a point of their type set to
 * alpha- until stability, with the same parity-class order (section 2.2). */
enum {
    THIN_OP_LEVELING = 0,   /* lambda-leveling: the lambda-destructible points */
    THIN_OP_SKELETON = 1    /* lambda-skeleton (the algorithm box of section 2.2): the
                               lambda-deletable points that are not lambda-end points
                               (section 2.1: a peak, T+ = 0, is lambda-deletable when
                               F(x) - alpha- <= lambda; an end point, with exactly one
                               n-neighbour in the section at its own level, is lambda-end
                               when F(x) - alpha- > lambda) */
};

/* Engines (thin_config.engine).  All produce bit-identical results. */
enum {
    THIN_ENGINE_AUTO = 0,     /* the tiled engine */
    THIN_ENGINE_TILED = 1,    /* one launch per round of LDS tiles (several parity steps per
                                 residency, stable tiles skipped); the host checks convergence */
    THIN_ENGINE_STEP = 2,     /* one parity step per launch over global memory (simple, slow) */
    /* 3 is not used (permanently unavailable: thin_create refuses it) */
    THIN_ENGINE_COOP = 4,     /* one cooperative launch for the whole run: the tiled engine's
                                 rounds separated by grid-wide barriers; convergence decided
                                 on the device */
    THIN_ENGINE_WORKLIST = 5  /* pixel work lists (the re-examination rule of section 2.2):
                                 one block per image runs every parity step, examining only
                                 the candidates whose 3x3 changed since their last examination
                                 (thin_stats.examinations then equals the sequential
                                 dirty-pixel sweep's count); sides up to 131070 */
};

typedef struct thin_ctx thin_ctx;

typedef struct thin_config {
    int32_t device;             /* HIP device ordinal */
    int32_t engine;             /* THIN_ENGINE_*, 0 = auto */
    void* hip_stream;           /* hipStream_t to enqueue on; NULL = the null stream */
    uint64_t max_device_bytes;  /* cap on device scratch owned by the context; 0 = no cap */
    uint64_t max_passes;        /* per-image pass cap (THIN_ELIMIT when reached); 0 = none */
    int32_t tile;               /* tile side in pixels for the tiled engine; 0 = automatic */
    int32_t steps_per_round;    /* parity steps per tile residency (halo width); 0 = automatic */
    uint32_t flags;             /* THIN_FLAG_* */
    int32_t threads;            /* with tile: threads per tile, 0 = first compiled choice */
    int32_t variant;            /* with tile and threads: residency variant (thin_tune_result) */
    int32_t reserved;
    const char* tune_cache;     /* NULL, or the path of a text file of autotuned shapes: read at
                                   thin_create (entries for this device's architecture only),
                                   and thin_autotune adds or replaces its result there; the
                                   string is copied */
} thin_config;

/* thin_config.flags */
enum {
    THIN_FLAG_PROFILE = 1,      /* time every round kernel with HIP events (see thin_profile) */
    THIN_FLAG_GRAPH = 2,        /* tiled engine: replay chunks of rounds as HIP graphs
                                   (ignored while THIN_FLAG_PROFILE is set) */
    THIN_FLAG_TAIL = 4          /* tiled engine: hand a single image's convergence tail to the
                                   pixel work-list kernel once the image (at most 512x512
                                   pixels) lowers fewer than 2048 pixels per round; results are
                                   identical, and on MI355X it is measured slower than staying
                                   on the tiles, so it is off by default */
};

typedef struct thin_profile_info {
    uint64_t launches;          /* round-kernel launches timed since the last reset */
    double kernel_ms;           /* sum of their durations, from HIP events on the context stream */
    uint64_t tile_rounds;       /* tile residencies they processed */
} thin_profile_info;

typedef struct thin_stats {
    uint64_t passes;       /* passes to stability, including the final pass without lowering */
    uint64_t lowerings;    /* number of lowerings F(x) := alpha- performed */
    uint64_t tile_rounds;  /* tile residencies processed (work done; depends on the engine) */
    uint32_t converged;    /* 1 when stable, 0 when stopped by max_passes */
    uint32_t reserved;
    uint64_t examinations; /* candidates the kernels characterised (work done; depends on the
                              engine: tile halos are characterised by every tile that holds
                              them, and the pixel work-list engine characterises exactly the
                              candidates whose 3x3 changed since their last characterisation) */
} thin_stats;

typedef struct thin_image {
    void* image;           /* caller-owned device buffer, modified in place */
    int64_t h, w;          /* rows, columns */
    int64_t pitch_elems;   /* row pitch in elements; 0 means w */
    int32_t dtype;         /* THIN_U8 or THIN_U16 */
    uint32_t lambda;       /* contrast parameter of the lambda-destructible test */
    int32_t adjacency;     /* THIN_ADJ_8_4 or THIN_ADJ_4_8 */
    int32_t op;            /* THIN_OP_LEVELING (0) or THIN_OP_SKELETON */
} thin_image;

/* Creates a context on cfg->device (cfg may be NULL: device 0, defaults).
 * Uploads the connectivity tables; scratch is allocated on first use and
 * kept.  Returns THIN_OK and *out, or an error (then *out is NULL). */
int thin_create(thin_ctx** out, const thin_config* cfg);

/* Lowers every lambda-destructible point of one image until stability
 * (section 2.2, type set lambda-destructible; section 2.1 for the test and
 * for alpha-).  image: device pointer to h*w contiguous elements.
 * stats may be NULL. */
int thin_run(thin_ctx* ctx, void* image, int64_t h, int64_t w, int32_t dtype,
             uint32_t lambda, int32_t adjacency, thin_stats* stats);

/* thin_run for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, result, statistics and errors as thin_run, but every
 * scratch buffer (the ping-pong twin, per-tile state and change bitmaps,
 * tile queues, counters, the image descriptor) is carved out of a static
 * device array of 64 MiB that the library holds on each GPU it runs on until
 * the process ends, so the call makes no hipMalloc, hipFree or other
 * allocating call (thin_create set up what it needs: the array's device
 * address on the context's device and the host counter snapshots).  An image
 * whose scratch does not fit (its twin plus about a quarter byte per pixel of
 * tile state: square u8 images up to 7296x7296, u16 up to 5453x5453) is
 * refused with THIN_ENOMEM and left untouched.
 * Runs on the tiled engine only (THIN_EINVAL for other engine settings);
 * THIN_FLAG_GRAPH and THIN_FLAG_PROFILE are ignored.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other host
 * threads, other contexts, other streams) race and must be serialised by
 * the caller.  Each call clears the parts of the array that must start at
 * zero. */
int thin_run_noalloc(thin_ctx* ctx, void* image, int64_t h, int64_t w, int32_t dtype,
                     uint32_t lambda, int32_t adjacency, thin_stats* stats);

/* The lambda-skeleton of one image (section 2.2, the algorithm box: lower
 * the lambda-deletable, not lambda-end points until stability; section 2.1
 * for peaks, end points and alpha-).  Arguments, conventions, order of
 * lowering, statistics and errors as for thin_run. */
int thin_skeleton(thin_ctx* ctx, void* image, int64_t h, int64_t w, int32_t dtype,
                  uint32_t lambda, int32_t adjacency, thin_stats* stats);

/* Same as thin_run for n independent images of any sizes, dtypes, lambdas,
 * adjacencies and operators, processed together by one device work list.  Images must
 * not overlap.  stats: NULL or an array of n entries.  Each image's result
 * and statistics equal those of a thin_run call on it alone. */
int thin_run_batch(thin_ctx* ctx, const thin_image* imgs, int32_t n, thin_stats* stats);

/* Serving (continuous batching) of independent images, each lowered exactly
 * as thin_run would lower it alone (section 2.2, lambda-destructible type
 * set; section 2.1 for the test and alpha-).  thin_serve_admit makes an
 * image resident under a caller-chosen tag; it takes part from the next
 * round of thin_serve_step on, each image on its own round clock.  The
 * first admission reserves the serving budget once: max_device_bytes when
 * set, else 1 GiB (twins take about 29/32 of it, per-tile state the rest)
 * and at most 16384 images are resident at a time.  An image whose twin or
 * tile state does not fit next to the resident ones is refused with
 * THIN_EBUSY and nothing is admitted: step and admit again later.  Images
 * smaller than 3x3 retire at the next thin_serve_step unchanged.  The image
 * buffer must stay valid, and untouched by the caller, until its tag is
 * reported.  Serving needs the tiled or cooperative engine setting
 * (THIN_EINVAL otherwise); it always runs the tiled round kernel. */
int thin_serve_admit(thin_ctx* ctx, const thin_image* img, uint64_t tag);

/* Runs `rounds` round launches (each up to steps_per_round parity steps of
 * every active tile) over every resident image, then retires the images that
 * are stable (or reached max_passes): their final values are in their own
 * buffers when the call returns.  rounds may be 0 to only collect reports.
 * Up to `cap` retired tags, oldest first, are written to done_tags (and their
 * statistics to done_stats when not NULL); *n_done (nullable) receives how
 * many were written; the rest are reported by later calls.  *n_resident
 * (nullable) receives the number of images still resident.  Blocks until the
 * launched rounds are done. */
int thin_serve_step(thin_ctx* ctx, int32_t rounds, uint64_t* done_tags, thin_stats* done_stats,
                    int32_t cap, int32_t* n_done, int32_t* n_resident);

/* Result of thin_autotune: the chosen tile shape and its time. */
typedef struct thin_tune_result {
    int32_t tile_h, tile_w;     /* tile interior */
    int32_t steps_per_round;    /* parity steps per residency (halo width) */
    int32_t threads;            /* threads per tile */
    int32_t variant;            /* residency variant (0..4) */
    int32_t candidates;         /* shapes timed */
    double ms;                  /* best wall time of one run over the images, chosen shape */
    double default_ms;          /* the same with the untuned choice */
} thin_tune_result;

/* Tile-shape autotuner for the tiled engine.  Runs the images (copies of
 * them: the caller's buffers are left untouched) once with every compiled
 * tile shape, re-times the fastest few `reps` times, and makes the fastest
 * the context's shape for later work lists of the same size class (total
 * pixels and pixels per image, each rounded down to a power of two).  With
 * thin_config.tune_cache set, the choice is also written to that file under
 * the device's architecture name (e.g. gfx950) and size class, so later
 * contexts on the same architecture start from it.  The
 * results of every shape are identical; only the time differs.  The copies
 * are freed before the call returns.  out may be NULL.  Returns THIN_OK,
 * THIN_EINVAL (bad arguments, nothing to tune), THIN_ENOMEM or
 * THIN_EDEVICE. */
int thin_autotune(thin_ctx* ctx, const thin_image* imgs, int32_t n, int32_t reps,
                  thin_tune_result* out);

/* Gradient front-end: the image the paper thins in its illustration
 * (Fig. 1(a)) is the Deriche gradient of a grayscale image.  Computes, in
 * float32, Deriche's recursive smoothing f(n) = k (a|n| + 1) r^|n| and
 * derivative g(n) = -c n r^|n| (r = exp(-alpha); k gives f unit sum, c gives
 * g unit response to a unit ramp): gx = g along columns of f along rows,
 * gy = g along rows of f along columns, with signals extended by their edge
 * values; stores min(top, rint(sqrt(gx^2 + gy^2) * gain)) into dst (top =
 * 255 for THIN_U8, 65535 for THIN_U16).  src and dst are caller-owned device
 * buffers of h rows and w columns with row pitches in elements (0 = w); dst
 * may be src itself when dtype and pitch match.  magnitude is NULL or a
 * device buffer of h*w floats (contiguous) that receives sqrt(gx^2 + gy^2).
 * Every float operation is rounded on its own in a fixed order, so results
 * are reproducible bit for bit.  The context keeps 32 bytes per pixel of
 * scratch.  Synchronous like thin_run.  Returns THIN_OK, THIN_EINVAL (bad
 * size, dtype or pitch, alpha <= 0, gain < 0 or not finite, NULL buffer with
 * h*w > 0), THIN_ENOMEM or THIN_EDEVICE. */
int thin_gradient(thin_ctx* ctx, const void* src, int64_t h, int64_t w, int64_t src_pitch,
                  int32_t src_dtype, float alpha, float gain, void* dst, int64_t dst_pitch,
                  int32_t dst_dtype, float* magnitude);

/* The 12 float32 coefficients thin_gradient uses for alpha (a0..a3 of the
 * smoothing recursions, d1 and d2 of the derivative ones, the feedback b1 and
 * b2, then the steady states of the causal and anticausal smoothing and
 * derivative recursions for a constant input of 1).  n must be at least 12.
 * Returns THIN_OK or THIN_EINVAL.  Needs no GPU. */
int thin_gradient_coefficients(float alpha, float* out, int32_t n);

/* Releases the context and all scratch it owns (NULL is accepted).
 * Never frees caller images. */
int thin_destroy(thin_ctx* ctx);

/* Static text for an error code. */
const char* thin_strerror(int code);

/* Text of the last error seen by ctx ("" when none; never NULL). */
const char* thin_last_error(const thin_ctx* ctx);

/* Reads (and with reset != 0 clears) the kernel timing gathered while
 * THIN_FLAG_PROFILE is set.  Returns THIN_EINVAL for NULL arguments. */
int thin_profile(thin_ctx* ctx, thin_profile_info* out, int32_t reset);

/* Host-side copy of the connectivity table the kernels use for adjacency
 * `adjacency` and operator `op`: for each upper-neighbour mask m (bit p set
 * when ring neighbour p has F >= F(x); ring order E, NE, N, NW, W, SW, S, SE,
 * rows growing downward), out[2m] holds bit 0 = destructible (T+ = 1 and
 * T-- = 1), bits 4..6 = T--, bits 8..10 = T+, and for THIN_OP_SKELETON
 * bit 1 = peak (T+ = 0) and bit 2 = end point (exactly one n-neighbour in
 * m); out[2m+1] holds, in byte c, the ring mask of the c-th counted lower
 * component (c < T--).  n must be at least 512.  Returns THIN_OK or
 * THIN_EINVAL.  Needs no GPU. */
int thin_topology_table(int32_t adjacency, int32_t op, uint32_t* out, int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* THIN_H */
