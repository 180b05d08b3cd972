/*
 * moa_fft.h -- C ABI of the MI355X (gfx950) dimension-lifted radix-2 FFT.
 *
 * The operation is the complex discrete Fourier transform of a vector of
 * length n = 2^t, t >= 0, as stated by the high-level radix-2 program of
 * Ch. 3 (Fig. vanloan_fft: input x in C^n, output the FFT of x), computed by
 * the cache-optimized ("dimension-lifted") method of Ch. 3-5: the vector is
 * viewed through a lift shape <... r c>, every level's butterflies run inside
 * one level of the GPU memory hierarchy (VGPRs and LDS of one workgroup),
 * and twiddle multiplies and reshape-transposes happen between levels
 * (sections "Cache-Optimized FFT: Key Elements of the New Approach",
 * "The General Algorithm", "Reordering the Data").
 *
 * Conventions, for every entry point:
 *   - FORWARD computes X_k = sum_j x_j exp(-2 pi i j k / n); ADJOINT computes
 *     the conjugate transform Y_j = sum_k y_k exp(+2 pi i j k / n).  Neither
 *     is normalised, so ADJOINT(FORWARD(x)) = n x.
 *   - Complex data are interleaved (re, im) pairs: MOA_C64 = two float32
 *     (the layout of torch.complex64), MOA_C128 = two float64.
 *   - Input and output are in natural order.  Transforms of a batch are
 *     contiguous, one after the other.
 *   - Device pointers are HIP device addresses owned by the caller; the
 *     library never frees them.  The plan owns its twiddle tables and
 *     workspace and releases them in moa_fft_destroy.
 *   - moa_fft_exec is asynchronous on the given HIP stream (NULL = the null
 *     stream) and never synchronises the host.
 *   - Every call returns a status; nothing aborts or throws across the ABI.
 *     Arguments are validated on the host before any HIP call, so invalid
 *     input is reported without touching the GPU.
 *   - A plan is immutable after creation.  Concurrent moa_fft_exec calls on
 *     one plan must be serialised on one stream because they share the
 *     plan's workspace.
 */
#ifndef MOA_FFT_H
#define MOA_FFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct moa_fft_plan_s* moa_fft_plan_t;

typedef enum { MOA_FFT_FORWARD = 0, MOA_FFT_ADJOINT = 1 } moa_fft_dir_t;

typedef enum { MOA_C64 = 0, MOA_C128 = 1 } moa_fft_dtype_t;

/* Arithmetic of the butterflies.  NATIVE: float32 for MOA_C64, float64 for
 * MOA_C128.  SPLIT_BF16 / SPLIT_FP16 (MOA_C64 only): every radix-16 stage is
 * a dense 16-point DFT contraction on the matrix cores with each operand
 * split into a high and a low half-precision part (three products, float32
 * accumulation); the dense radix-n butterfly is the general-radix block of
 * Ch. 1 (Fig. radnbutterfly).  Only levels of 16, 256 or 4096 points run
 * on the matrix cores, and only where one tile gathers 2^11 points or more
 * (a 16-point level of fewer than 128 transforms, a 256-point one of fewer
 * than 8, runs in float32).  Other levels, and all twiddles, stay float32. */
typedef enum {
    MOA_FFT_PREC_NATIVE = 0,
    MOA_FFT_PREC_SPLIT_BF16 = 1,
    MOA_FFT_PREC_SPLIT_FP16 = 2
} moa_fft_prec_t;

typedef enum {
    MOA_OK = 0,
    MOA_ERR_NULL = 1,        /* a required pointer argument is NULL            */
    MOA_ERR_SIZE = 2,        /* n < 1, not a power of two, or above 2^30       */
    MOA_ERR_LIFT = 3,        /* lift shape: product != n, a factor that is not
                                a power of two, rank outside 1..8, or a level
                                longer than one workgroup can hold in LDS      */
    MOA_ERR_BATCH = 4,       /* batch < 1, count < 1, or total size overflow   */
    MOA_ERR_DTYPE = 5,       /* unknown dtype/precision, or SPLIT with C128    */
    MOA_ERR_ALLOC = 6,       /* device or host allocation failed               */
    MOA_ERR_HIP = 7,         /* a HIP runtime call failed                      */
    MOA_ERR_STATE = 8,       /* plan is host-only (cannot execute) or invalid  */
    MOA_ERR_ARG = 9,         /* other invalid argument (direction, flags, len) */
    MOA_ERR_TUNING = 10,     /* tuning parameters outside the kernel's limits  */
    MOA_ERR_SCRATCH = 11     /* moa_fft_exec_noalloc: the plan needs more
                                workspace than MOA_FFT_SCRATCH_BYTES          */
} moa_status_t;

/* Flags for the plan constructors. */
#define MOA_FFT_FLAG_HOST_ONLY 0x1u   /* validate and lower only: no device
                                         resources; describe() works, exec()
                                         returns MOA_ERR_STATE              */
#define MOA_FFT_FLAG_PER_SIZE 0x2u    /* uneven batch: one plain launch per
                                         distinct size instead of one
                                         fused launch                       */
#define MOA_FFT_FLAG_GRAPH 0x4u       /* record the plan's launches for each
                                         (direction, in, out) once as a HIP
                                         graph of kernel nodes and replay it
                                         with one hipGraphLaunch per exec   */
#define MOA_FFT_FLAG_NO_WORKSPACE 0x8u /* allocate no workspace: a plan with
                                         more than one level then runs whole
                                         only through moa_fft_exec_noalloc
                                         (moa_fft_exec returns MOA_ERR_STATE;
                                         moa_fft_exec_level needs none)      */

/* Bytes of the library's static device workspace used by
 * moa_fft_exec_noalloc on each GPU: 64 MiB, the workspace of 2^23 complex64
 * or 2^22 complex128 points. */
#define MOA_FFT_SCRATCH_BYTES ((size_t)64 << 20)

/* Optional launch tuning, one entry per level of the lift (level 0 = the
 * innermost block c, the first pass).  Zero entries select the defaults. */
typedef struct {
    int32_t cols_per_block[8];  /* transforms (columns of the lifted view)
                                   handled by one workgroup in that pass;
                                   a nonzero entry also selects the level
                                   kernel for a short single-level plan,
                                   which by default runs one transform a
                                   workgroup on N/4 threads              */
    int32_t persistent_blocks;  /* uneven batch: workgroups of the fused
                                   launch (0 = one per task; fewer make it
                                   persistent, each workgroup walking the
                                   tasks with a grid stride)               */
    int32_t stream;             /* non-temporal (streaming) access to data a
                                   transform touches once: the first level's
                                   loads of the caller's input; for an
                                   uneven batch its loads and its stores.
                                   0 = when the input is at most 256 MiB
                                   (the Infinity Cache), 1 = always,
                                   -1 = never; other values MOA_ERR_TUNING  */
    uint32_t lg_radix;          /* largest register radix of each level's
                                   stages, 4 bits per level (level l in
                                   bits 4l .. 4l+3): log2 of the radix, 0 =
                                   the default (16, i.e. 4), 2 / 3 / 5 =
                                   radix 4 / 8 / 32 (the general-radix
                                   block of Ch. 1, Fig. radnbutterfly):
                                   stages of that radix, then one with the
                                   remaining radix.  Other radices run the
                                   level kernel (complex64 levels of 2^5 ..
                                   2^14 points, not the split precisions);
                                   radix 32 needs 32 points a thread,
                                   i.e. a level that stores in its load
                                   pattern, with at most 512 threads.
                                   Anything else MOA_ERR_TUNING            */
    int32_t batch_task_lg;      /* uneven batch: log2 of the most points one
                                   task (one workgroup's share) packs from
                                   transforms of 2^13 points or fewer: 11,
                                   12 or 13 (0 = 13); shorter tasks mean
                                   more of them for the dispatcher to
                                   balance.  A longer transform is one
                                   task (a 2^14-point complex64 transform
                                   too).  Anything else MOA_ERR_TUNING     */
    int32_t reserved[4];
} moa_fft_tuning_t;

/*
 * Plan `batch` contiguous transforms of length n.
 *
 * lift_shape / lift_rank: the lift <s_0 ... s_{k-1}> of Ch. 3: the vector is
 * viewed as an s_0 x ... x s_{k-1} array (row-major), s_{k-1} = c is the
 * innermost block handled by the first level, and each further level works
 * on the next axis outwards.  The product must equal n, every factor must
 * be a power of two, and each factor must fit one workgroup (at most 2^14
 * points for MOA_C64, 2^13 for MOA_C128).  NULL/0 selects a default lift
 * (measured on MI355X): one level when n itself fits; for MOA_C64 with
 * 2^19 <= n <= 2^23 in batches of 2^24 points or more, two levels with one
 * of 4096 points, <n/4096 4096> while the batch holds 2^25 points or fewer
 * (and always at 2^23), <4096 n/4096> beyond, except <256 128 256> for
 * n = 2^23 in batches of up to 2^25 points; for MOA_C64 with n >= 2^25 the
 * three levels <256 4096 n/2^20>;
 * for MOA_C128 with 2^23 <= n <= 2^26 the three levels <256 256 n/2^16>;
 * otherwise the fewest levels of near-equal size.  With a SPLIT precision
 * and n <= 2^24 the default takes the fewest levels, cut where it can into
 * 16-, 256- and 4096-point levels for the matrix cores (2^20: <4096 256>),
 * the bits that make no whole radix-16 digit going to the first level.  The
 * paper's uniform blocking by c corresponds to <2^p_max c ... c>.
 *
 * On success *out receives a new plan.  Errors: MOA_ERR_NULL (out NULL, or
 * lift_shape NULL with lift_rank > 0), MOA_ERR_SIZE, MOA_ERR_LIFT,
 * MOA_ERR_BATCH, MOA_ERR_DTYPE, MOA_ERR_ARG (unknown flag bits),
 * MOA_ERR_ALLOC / MOA_ERR_HIP (device resources).  *out is untouched on
 * error.
 */
moa_status_t moa_fft_plan(moa_fft_plan_t* out, int64_t n, int64_t batch,
                          const int64_t* lift_shape, int32_t lift_rank,
                          moa_fft_dtype_t dtype, moa_fft_prec_t prec, uint32_t flags);

/* moa_fft_plan with explicit launch tuning (tuning may be NULL).
 * MOA_ERR_TUNING if a value does not fit the kernel's limits. */
moa_status_t moa_fft_plan_tuned(moa_fft_plan_t* out, int64_t n, int64_t batch,
                                const int64_t* lift_shape, int32_t lift_rank,
                                moa_fft_dtype_t dtype, moa_fft_prec_t prec, uint32_t flags,
                                const moa_fft_tuning_t* tuning);

/*
 * Plan `batch` contiguous multi-dimensional transforms of an array of shape
 * dims[0] x ... x dims[rank-1] (row-major: dims[rank-1] is the contiguous
 * axis): X[k] = sum_j x[j] exp(-2 pi i sum_a j_a k_a / dims[a]) forward, the
 * conjugate transform for ADJOINT, unnormalised.  The multi-dimensional
 * extension of the lifted FFT (Ch. 1, "Conclusions for the General Radix
 * Approach", and Ch. 3, "Conclusions"): the array is the lifted view of its
 * ravel, and the transform is the levels of that lift with no inter-level
 * factor between them and no final digit reversal -- one kernel launch per
 * axis of extent > 1, the contiguous axis first, each a DFT along its axis
 * with the inner axes as the tile.  The first launch reads `in` and writes
 * `out`, the others run in place in `out`, so the plan owns no workspace
 * (in == out is allowed).
 *
 * rank: 1..8.  Every extent must be a power of two of at most one
 * workgroup's block (moa_fft_max_block: 2^14 for MOA_C64, 2^13 for
 * MOA_C128), and their product at most 2^30.  prec as for moa_fft_plan
 * (axes whose length is 16, 256 or 4096 run on the matrix cores with a
 * SPLIT precision).  Errors: MOA_ERR_NULL (out or dims NULL), MOA_ERR_ARG
 * (rank outside 1..8, unknown or PER_SIZE flag), MOA_ERR_SIZE (an extent
 * that is not a power of two, too long, or a product above 2^30),
 * MOA_ERR_BATCH, MOA_ERR_DTYPE, MOA_ERR_LIFT (no kernel takes an axis),
 * MOA_ERR_ALLOC / MOA_ERR_HIP.
 * *out is untouched on error.  moa_fft_num_levels reports the launches;
 * moa_fft_exec_level(l) runs the l-th launch from `in` to `out`.
 */
moa_status_t moa_fft_plan_nd(moa_fft_plan_t* out, int32_t rank, const int64_t* dims, int64_t batch,
                             moa_fft_dtype_t dtype, moa_fft_prec_t prec, uint32_t flags);

/* moa_fft_plan_nd with explicit launch tuning (one cols_per_block entry per
 * launch, in launch order; tuning may be NULL). */
moa_status_t moa_fft_plan_nd_tuned(moa_fft_plan_t* out, int32_t rank, const int64_t* dims, int64_t batch,
                                   moa_fft_dtype_t dtype, moa_fft_prec_t prec, uint32_t flags,
                                   const moa_fft_tuning_t* tuning);

/*
 * Plan an uneven batch: `count` transforms, transform i of length sizes[i]
 * (each a power of two between 1 and 2^14 for MOA_C64, 2^13 for MOA_C128),
 * packed one after the other in input and output (transform i starts at
 * element sum_{j<i} sizes[j]).  The host array `sizes` is copied.  By
 * default all transforms run in one fused launch of one workgroup per task
 * (tasks ordered longest first; a tuned smaller grid makes the launch
 * persistent); with MOA_FFT_FLAG_PER_SIZE they run as one plain launch per
 * distinct size.
 * Errors as moa_fft_plan; MOA_ERR_SIZE names an invalid entry of sizes.
 */
moa_status_t moa_fft_plan_batched(moa_fft_plan_t* out, const int64_t* sizes, int64_t count,
                                  moa_fft_dtype_t dtype, uint32_t flags);

/* moa_fft_plan_batched with explicit tuning (tuning may be NULL). */
moa_status_t moa_fft_plan_batched_tuned(moa_fft_plan_t* out, const int64_t* sizes, int64_t count,
                                        moa_fft_dtype_t dtype, uint32_t flags,
                                        const moa_fft_tuning_t* tuning);

/*
 * Execute a plan in direction dir on device buffers holding batch * n (or
 * sum(sizes)) complex elements.  in == out (in place) is allowed; other
 * overlaps are not.  Asynchronous on `stream` (a hipStream_t, NULL = null
 * stream).  Errors: MOA_ERR_NULL (p, in or out NULL), MOA_ERR_STATE (p is
 * not a live plan, or is host-only), MOA_ERR_ARG (bad dir, or a caller
 * buffer off the 16-byte alignment a paired-column level needs),
 * MOA_ERR_HIP (launch failure).
 */
moa_status_t moa_fft_exec(moa_fft_plan_t p, moa_fft_dir_t dir, const void* in, void* out,
                          void* stream);

/*
 * moa_fft_exec for callers that cannot allocate device memory: code under
 * HIP graph (stream) capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It calls no hipMalloc, hipFree or allocating library routine
 * and builds no HIP graph (a MOA_FFT_FLAG_GRAPH plan's launches are issued
 * directly).  The workspace a plan of several levels needs (batch * n
 * complex elements) is taken from a static device array of
 * MOA_FFT_SCRATCH_BYTES that the library holds on each GPU it runs on until
 * the process ends, instead of the plan's own workspace, so the plan may be
 * made with MOA_FFT_FLAG_NO_WORKSPACE.  Plans of one level (and uneven
 * batches) need none and run exactly as with moa_fft_exec.
 *
 * Every call on one GPU shares that GPU's array: calls whose executions
 * overlap on one GPU (two streams, or two host threads) race and give wrong
 * results; serialise them on one stream.  The array keeps the last call's
 * contents; nothing in it needs to start at zero (the first level of an
 * execution writes all of the workspace before any level reads it).
 *
 * Arguments and result as moa_fft_exec (the buffers stay the caller's).
 * Errors: those of moa_fft_exec, plus MOA_ERR_SCRATCH when the plan needs
 * more than MOA_FFT_SCRATCH_BYTES of workspace (checked on the host before
 * any HIP call), and MOA_ERR_HIP if the array's device address cannot be
 * obtained.
 */
moa_status_t moa_fft_exec_noalloc(moa_fft_plan_t p, moa_fft_dir_t dir, const void* in, void* out,
                                  void* stream);

/*
 * Run only level `level` of a plan (one kernel launch) from `in` to `out`,
 * for timing and inspecting one level of the lift ("The General
 * Algorithm": one level = one pass over memory).  Level l reads `in` in the
 * layout level l - 1 writes and writes `out` in the layout level l + 1
 * reads, so running levels 0..L-1 in order through caller buffers of batch
 * * n elements (level 0 reading x, the last level writing the result) equals
 * moa_fft_exec.  The intermediate layout is the plan's workspace layout
 * (moa_fft_describe: the digit strides of each pass, and the blocked
 * out_layout / in_layout of a paired-column lift): after level 0 of a
 * two-level lift <r c> it holds the length-c DFTs of the r stride-r columns
 * multiplied by the inter-level factor omega_n^(a k), column a, frequency k.
 * in == out is accepted only where the level stores in its load pattern:
 * every level of a multi-dimensional plan, a single-level plan, the middle
 * levels of a lift of three or more levels, and level 0 of a lift whose
 * workspace keeps the digit positions (not the blocked paired-column
 * layout); otherwise MOA_ERR_ARG.  For a multi-dimensional plan level l is
 * the l-th axis launch.  For an uneven batch planned with
 * MOA_FFT_FLAG_PER_SIZE, level g runs the transforms of the g-th distinct
 * length (longest first) from `in` to `out`; for the fused form level 0 is
 * the whole launch.  Needs no workspace.  Errors as moa_fft_exec, plus
 * MOA_ERR_ARG for a level outside 0..L-1.
 */
moa_status_t moa_fft_exec_level(moa_fft_plan_t p, moa_fft_dir_t dir, int32_t level, const void* in,
                                void* out, void* stream);

/* Number of levels (= kernel launches per execution) of a plan; 1 for an
 * uneven batch in one fused launch, the number of distinct lengths for
 * one planned with MOA_FFT_FLAG_PER_SIZE. */
moa_status_t moa_fft_num_levels(moa_fft_plan_t p, int32_t* levels);

/* Bytes of device workspace the plan owns (0 for single-level plans). */
moa_status_t moa_fft_workspace_size(moa_fft_plan_t p, size_t* bytes);

/*
 * Write a NUL-terminated JSON description of the plan into buf (len bytes):
 * the lift, and for every pass the loop bounds and strides of its
 * operational normal form (the DFT axis and each batch axis with its size,
 * input stride and output stride), twiddle root, launch shape and LDS
 * bytes.  Errors: MOA_ERR_NULL (p or buf NULL), MOA_ERR_ARG if len is
 * smaller than moa_fft_describe_size (the text is then truncated and still
 * NUL-terminated when len > 0).
 */
moa_status_t moa_fft_describe(moa_fft_plan_t p, char* buf, size_t len);

/* Bytes (including the NUL) that moa_fft_describe needs for this plan. */
moa_status_t moa_fft_describe_size(moa_fft_plan_t p, size_t* bytes);

/* Release the plan and its device resources.  NULL is accepted (no-op).
 * The library keeps a registry of live plans: destroying a plan twice, or
 * passing any non-NULL handle that is not a live plan to this or any other
 * call, returns MOA_ERR_STATE without touching memory (a NULL handle gives
 * MOA_ERR_NULL, except here).  A handle is the plan's address,
 * so a stale handle that equals a newer plan's address names that plan.
 * Destroying a plan while another thread uses it is the caller's error. */
moa_status_t moa_fft_destroy(moa_fft_plan_t p);

/* Static, NUL-terminated name of a status code ("MOA_OK", ...). */
const char* moa_fft_status_string(moa_status_t s);

/* Largest single-level (in-LDS) transform length for a dtype. */
int64_t moa_fft_max_block(moa_fft_dtype_t dtype);

#ifdef __cplusplus
}
#endif

#endif /* MOA_FFT_H */
