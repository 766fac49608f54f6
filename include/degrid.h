/*
 * degrid.h -- C ABI of the MI355X (gfx950) 3D degridding library.
 *
 * The operation (Section 2 of the paper, "Implementation"): degridding forms
 * each visibility as a weighted sum of regularly sampled values. The inputs
 * are
 *   - an oversampled gridding convolution function (GCF) for the uv plane,
 *     G_uv, with support 8 x 8;
 *   - an oversampled GCF for the w direction, G_w, with support 4;
 *   - a stack of S subgrids of 512 x 512 x 4 complex values;
 *   - for each subgrid, the list of its visibility coordinates [u, v, w].
 * For every visibility the library computes the subgrid point g = [x, y, z]
 * where the weighted sum starts and the positions of its weights inside the
 * oversampled tables, then
 *     V = sum_{tv<8} sum_{tu<8} sum_{tw<4}
 *           G_w[o_w][tw] * G_uv[o_v][o_u][tv][tu] * A_s[y+tv][x+tu][z+tw].
 * grid_adjoint applies the transpose of the same real linear map.
 *
 * Conventions fixed by this library (the paper leaves them open):
 *   - subgrid layout [S][n_v][n_u][n_w], w fastest, complex interleaved
 *     (re, im);
 *   - [u, v, w] are float64 in subgrid cells, origin at cell 0; per axis
 *     k = floor(c * os) of the float64 product (exact when os is a power of
 *     two; for other factors this rounding of the product is the contract),
 *     cell n = floor(k / os), oversample index o = k - n * os, first tap
 *     n - (W/2 - 1);
 *   - subgrids may hold more w planes than the w support (n_w > 4): the
 *     first w tap z = floor(w) - 1 then varies between visibilities;
 *   - G_uv is indexed [o_v][o_u][t_v][t_u], G_w is indexed [o_w][t_w]; both
 *     real;
 *   - a visibility whose neighbourhood leaves the subgrid (or whose
 *     coordinate is NaN or infinite) is out of range: its output is 0 and it
 *     is counted (degrid_oob_count), it is not an error;
 *   - the visibilities of subgrid s are rows vis_offsets[s] ..
 *     vis_offsets[s+1]-1 of uvw and of the output (CSR offsets).
 *
 * Ownership: the caller owns every input and output buffer (device memory,
 * e.g. from torch or hipMalloc). A plan owns its own device scratch (tile
 * queue, queue cursors, out-of-range counter); only degrid_plan,
 * degrid_batch_plan and degrid_tune allocate. degrid_execute, grid_adjoint
 * and degrid_batch_execute allocate nothing and are asynchronous on the
 * stream they are given. A plan or batch must be used by one stream at a
 * time; calls that overlap on two streams race on the plan's scratch.
 * degrid_plan_sort also allocates (the plan's work-order permutation).
 *
 * Errors: every call returns a dg_status. Argument errors are detected on the
 * host before any device work is queued. HIP errors map to DG_ERR_HIP;
 * degrid_last_error() returns a thread-local detail string for the last
 * failing call on the calling thread. No C++ exception crosses this ABI.
 */
#ifndef DEGRID_H
#define DEGRID_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DG_OK = 0,
    DG_ERR_INVALID_ARG = 1,   /* a pointer, size, offset list or descriptor field is invalid */
    DG_ERR_UNSUPPORTED = 2,   /* valid but not implemented (e.g. support other than 8 / 4)   */
    DG_ERR_NOMEM = 3,         /* device or host allocation failed                            */
    DG_ERR_HIP = 4,           /* a HIP runtime call failed (no device, launch failure, ...)  */
    DG_ERR_NOT_READY = 5      /* the object is not in a state that allows the call           */
} dg_status;

/* Storage type of subgrid values. Accumulation is always float32. */
typedef enum {
    DG_GRID_C64 = 0,   /* complex float32, 8 bytes per value            */
    DG_GRID_CBF16 = 1, /* complex bfloat16 (re, im), 4 bytes per value  */
    DG_GRID_CF16 = 2   /* complex float16 (re, im), 4 bytes per value   */
} dg_grid_dtype;

/* Storage type of the G_uv and G_w tables. Any table type goes with any
 * storage type. With DG_GRID_CF16 storage and DG_GCF_F16 tables, or
 * DG_GRID_CBF16 and DG_GCF_BF16, the sums over w run on the packed 16-bit dot
 * products (each product exact in float32, float32 accumulation). */
typedef enum {
    DG_GCF_F32 = 0,
    DG_GCF_F16 = 1,
    DG_GCF_BF16 = 2
} dg_gcf_dtype;

/* Problem descriptor (Section 2: subgrid size, GCF supports and oversampling). */
typedef struct {
    int32_t n_v, n_u, n_w;          /* subgrid size; the paper's is 512, 512, 4; n_w >= 4          */
    int32_t support_uv, support_w;  /* GCF supports; must be 8 and 4 (else DG_ERR_UNSUPPORTED)     */
    int32_t os_uv, os_w;            /* oversampling factors in [1, 64]; tables are                 */
                                    /* G_uv[os_uv][os_uv][8][8] and G_w[os_w][4]                   */
    int32_t grid_dtype;             /* dg_grid_dtype                                               */
    int32_t gcf_dtype;              /* dg_gcf_dtype                                                */
    int32_t n_b;                    /* visibilities per tile in [1, 64]; 0 = library choice        */
    uint32_t flags;                 /* reserved, must be 0                                         */
} dg_desc;

typedef struct dg_plan_* dg_plan;    /* opaque, owned by the library */
typedef struct dg_batch_* dg_batch;  /* opaque, owned by the library */

/* Read-only facts about a plan (for logging and tests). */
typedef struct {
    int64_t n_subgrids;
    int64_t n_vis;          /* vis_offsets[S]                                     */
    int64_t n_tiles;        /* work items in the plan's queue                     */
    int32_t n_b;            /* visibilities per tile actually used                */
    int32_t kernel;         /* index of the gather kernel variant                 */
    int32_t grid_blocks;    /* workgroups of the persistent launch                */
    int32_t block_threads;  /* threads per workgroup                              */
    int32_t n_queues;       /* per-XCD queues of the tile list                    */
    int32_t device;         /* HIP device the plan's scratch lives on             */
    int32_t sorted;         /* 1 if degrid_plan_sort set a work order             */
    int32_t n_kernels;      /* number of gather kernel variants                   */
} dg_plan_info;

/*
 * Build a plan for S = n_subgrids subgrids (Section 2: the inputs are the
 * subgrid stack, the two oversampled GCFs and, for each subgrid, its list of
 * visibility coordinates; a thread block takes N_b visibilities of one
 * subgrid, and Eq. (1) sizes the launch from the largest list; here the
 * N_b-visibility tiles of every subgrid form one queue that a persistent
 * launch drains).
 *   d            descriptor (host); copied.
 *   vis_offsets  host int64[S+1]; offsets[0] == 0, non-decreasing; copied.
 *   stream       stream used for the plan's own uploads (may be NULL).
 *   out          receives the plan; *out is set to NULL on failure.
 * Allocates device scratch on the current HIP device. Synchronises 'stream'.
 * Returns DG_ERR_INVALID_ARG for a bad descriptor or offsets,
 * DG_ERR_UNSUPPORTED for supports other than 8 x 8 and 4, for a subgrid of
 * 2^30 bytes or more, for n_u > 65543 or n_v > 65542 (first taps are
 * packed into 16 bits per axis), for 2^32 or more visibilities, or for more
 * than 2^31 - 1 tiles, DG_ERR_NOMEM or
 * DG_ERR_HIP when the device side cannot be set up. A plan for subgrids with
 * n_w != 4 uses the one kernel variant that reads taps starting at any w
 * (no LDS staging); degrid_plan_set_kernel refuses the others for it, and
 * its adjoint scatters with float32 atomics even after degrid_plan_sort.
 * With d->n_b == 0 the library chooses the tile size and kernel variant: the
 * choice recorded by degrid_tune in the DG_TUNE_CACHE file for this device
 * and problem shape class if there is one; else tiles of 64 visibilities
 * (smaller, a multiple of 8, when the plan has fewer than 16 visibilities per
 * resident wavefront), staged through LDS boxes for complex float32 storage
 * and gathered through the caches for the 16-bit storage types and for plans
 * of at most two resident wavefronts' worth of visibilities.
 */
dg_status degrid_plan(const dg_desc* d, int64_t n_subgrids, const int64_t* vis_offsets,
                      hipStream_t stream, dg_plan* out);

/*
 * Degrid (Section 2; the launch geometry of Eq. (1) is replaced by a
 * persistent, load-balanced tile queue).
 *   subgrids  device [S][n_v][n_u][n_w] complex in the plan's grid dtype.
 *   g_uv      device [os_uv][os_uv][8][8] in the plan's gcf dtype.
 *   g_w       device [os_w][4] in the plan's gcf dtype.
 *   uvw       device float64 [N][3], N = vis_offsets[S].
 *   vis_out   device complex float32 [N]; every entry is written.
 * Asynchronous on 'stream'; allocates nothing. The out-of-range count of this
 * call replaces the plan's previous count.
 * Alignment (every entry point that takes these arrays): each element
 * naturally aligned (subgrids 8 bytes for complex float32, 4 for the 16-bit
 * complex types; g_uv 4 or 2; uvw and complex float32 arrays 8), and g_w on
 * a 4-byte boundary whatever its dtype (its rows are read as whole 32-bit
 * words). A misaligned pointer gives DG_ERR_INVALID_ARG and launches nothing.
 */
dg_status degrid_execute(dg_plan p, const void* subgrids, const void* g_uv, const void* g_w,
                         const double* uvw, void* vis_out, hipStream_t stream);

/*
 * Degrid without a plan, allocating nothing: for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). Same operation, arguments and results as
 * degrid_execute on a plan in input order (degrid_plan without
 * degrid_plan_sort), with the plan's inputs passed directly:
 *   d            descriptor (host), as for degrid_plan; n_b = 0 means 64.
 *   n_subgrids   S, at most 16384.
 *   vis_offsets  host int64[S+1], as for degrid_plan; copied (stream-ordered)
 *                into the library's device scratch before the call returns.
 *   subgrids, g_uv, g_w, uvw, vis_out  device arrays as for degrid_execute.
 *   oob_count    device int64, or NULL: receives this call's out-of-range
 *                count (written by the call's kernels, stream-ordered).
 * The scratch (a tile cursor and count, the offsets and per-subgrid tile
 * offsets: 262 656 bytes) is one static device array per GPU, held until the
 * process ends and shared by every call on that GPU: calls that overlap on
 * one GPU (two streams, or two host threads) race and give wrong results.
 * Calls no hipMalloc or hipFree. Every visibility's result equals
 * degrid_execute's (input-order tiles of n_b visibilities, gathered through
 * the caches). DG_ERR_UNSUPPORTED for more than 16384 subgrids or 2^31 - 1
 * tiles; other argument errors as for degrid_plan and degrid_execute, all
 * detected before any device work. Asynchronous on 'stream'.
 */
dg_status degrid_execute_noalloc(const dg_desc* d, int64_t n_subgrids, const int64_t* vis_offsets,
                                 const void* subgrids, const void* g_uv, const void* g_w, const double* uvw,
                                 void* vis_out, int64_t* oob_count, hipStream_t stream);

/*
 * Gradients with respect to the tables (the chain rule through the weighted
 * sum of Section 2; each visibility is linear in each table). Given the
 * gradient of a real loss L with respect to the visibilities,
 * grad_vis[i] = dL/dRe(V_i) + i dL/dIm(V_i) (device complex float32 [N]):
 *   grad_g_uv[o_v][o_u][t_v][t_u] = sum over in-range i with offsets (o_v, o_u) of
 *       Re(conj(grad_vis[i]) * sum_tw G_w[o_w][t_w] * A[y+t_v][x+t_u][z+t_w]);
 *   grad_g_w[o_w][t_w] = sum over in-range i with offset o_w of
 *       Re(conj(grad_vis[i]) * sum_{t_v,t_u} G_uv[o_v][o_u][t_v][t_u] * A[...]).
 *   grad_g_uv  device float32 [os_uv][os_uv][8][8], or NULL (not computed).
 *   grad_g_w   device float32 [os_w][4], or NULL (not computed).
 *   accumulate 0: the outputs are overwritten; 1: added to.
 * Other arguments as for degrid_execute, in the plan's dtypes. Out-of-range
 * visibilities add nothing. The sums meet in float32 atomics, so the last
 * bits depend on timing. Both outputs 4-byte aligned. Asynchronous on
 * 'stream'; allocates nothing.
 */
dg_status degrid_table_grad(dg_plan p, const void* subgrids, const void* g_uv, const void* g_w, const double* uvw,
                            const void* grad_vis, float* grad_g_uv, float* grad_g_w, int32_t accumulate,
                            hipStream_t stream);

/*
 * Residual and loss in the same pass as the degrid (the imaging major cycle
 * of Section 1 subtracts the model visibilities from the observed ones):
 *   res_out[i] = v_obs[i] - degrid(subgrids)_i   (complex float32 [N]);
 *   *loss_out  = sum over all i of |res_out[i]|^2 (float64, device scalar).
 * An out-of-range visibility has a model of 0, so its residual is v_obs[i].
 * v_obs and res_out are device complex float32 [N] and may be the same
 * buffer (in place). Each tile's float64 partial sum is added in a fixed
 * order, so the loss has the same bits on every call of the same plan (it
 * may differ in the last bits between plans cut into other tiles). With
 * no visibilities the loss is written as 0. Other arguments as for
 * degrid_execute. Asynchronous on 'stream'; allocates nothing.
 */
dg_status degrid_residual(dg_plan p, const void* subgrids, const void* g_uv, const void* g_w, const double* uvw,
                          const void* v_obs, void* res_out, double* loss_out, hipStream_t stream);

/*
 * Adjoint of degrid_execute (gridding; the transpose of the weighted sum of
 * Section 2, which the paper does not implement): scatters G_w * G_uv * V_i
 * onto the 8 x 8 x 4 neighbourhood of every in-range visibility.
 *   vis          device complex float32 [N].
 *   subgrids_out device complex float32 [S][n_v][n_u][n_w] (always float32,
 *                whatever the plan's grid dtype).
 *   accumulate   0: the output is overwritten; 1: contributions are added to
 *                its current contents.
 * On a plan with a work order (degrid_plan_sort), every 16 x 16-cell block
 * of the output is summed by one wavefront in LDS and written once, so the
 * result has the same bits on every call; visibilities whose coordinates
 * moved since the sort are added by a second pass with float32 atomics (so
 * when some moved, their sums' last bits vary from run to run). On
 * a plan in input order the output is zeroed (by a kernel) and contributions
 * are added with float32 atomics, so the last bits vary from run to run.
 * Asynchronous on 'stream'; allocates nothing.
 */
dg_status grid_adjoint(dg_plan p, const void* vis, const void* g_uv, const void* g_w,
                       const double* uvw, void* subgrids_out, int32_t accumulate,
                       hipStream_t stream);

/*
 * Out-of-range visibilities seen by the last degrid_execute, degrid_residual
 * or grid_adjoint of this plan: those whose 8 x 8 x 4 neighbourhood, starting
 * at the point g of Section 2, does not lie inside the subgrid (the paper does
 * not say what happens there; such a visibility's output is 0). 0 before the
 * first call and after a call on a plan without visibilities. Synchronises
 * the stream of the last call.
 */
dg_status degrid_oob_count(dg_plan p, int64_t* count);

/*
 * Reorder the plan's work for locality: within each subgrid, visibilities are
 * processed in the order of a Hilbert curve through the cells that hold
 * (u, v), so a tile holds visibilities that are close in the subgrid and
 * consecutive tiles cover neighbouring regions (Section 2 notes that one grid point may serve
 * several visibilities; this makes that reuse happen in cache).
 *   uvw  device float64 [N][3], the coordinates later calls will use; NULL
 *        drops the work order (back to input order).
 * Every output stays in input order and every result is unchanged (each
 * visibility's sum does not depend on the order); only speed depends on uvw
 * matching the coordinates passed to later calls. Allocates the plan's
 * permutation (4 bytes per visibility) and temporary sort buffers;
 * synchronises 'stream'. DG_ERR_UNSUPPORTED if N >= 2^32.
 * Batches built from this plan before the call must be rebuilt.
 */
dg_status degrid_plan_sort(dg_plan p, const double* uvw, hipStream_t stream);

/* Plan facts; host only, does not touch the device. */
dg_status degrid_plan_get_info(dg_plan p, dg_plan_info* info);

/*
 * Time the gather kernel variants and tile sizes on the given (real) inputs
 * and keep the fastest in the plan (the tile list is rebuilt). Writes the
 * choice to the on-disk cache named by DG_TUNE_CACHE when that is set.
 * Synchronises 'stream'. vis_out is overwritten.
 */
dg_status degrid_tune(dg_plan p, const void* subgrids, const void* g_uv, const void* g_w,
                      const double* uvw, void* vis_out, hipStream_t stream);

/*
 * Choose the gather kernel variant and the tile size by hand (what
 * degrid_tune chooses by timing). kernel: index in [0, number of variants),
 * or -1 to keep the current one; n_b: visibilities per tile in [1, 64], or 0
 * to keep the current one. Variants differ in how much LDS each wavefront
 * uses to stage a tile's cells (variant 0 stages nothing); results are the
 * same for every variant. Rebuilds the tile list (allocates); synchronises
 * 'stream'. Batches built from this plan before the call must be rebuilt.
 */
dg_status degrid_plan_set_kernel(dg_plan p, int32_t kernel, int32_t n_b, hipStream_t stream);

/* Release a plan and its device scratch (synchronises the device). NULL is a no-op. */
dg_status degrid_destroy(dg_plan p);

/*
 * Batch several plans (independent problems with their own S, counts and
 * oversampling, same grid and gcf dtypes) into one persistent launch. (Section
 * 2 warns that uneven visibility counts per subgrid leave most blocks of the
 * Eq. (1) launch idle, and Section 3 measures throughput against the counts;
 * one queue over the tiles of several problems keeps the device full.) The
 * plans must stay alive while the batch exists. The batch runs one gather
 * kernel, that of the plan with the most visibilities (degrid_batch_tune
 * gives every plan the same one); DG_ERR_INVALID_ARG if another plan's tiles
 * are larger than that kernel takes. Allocates the batch's tile list, queue
 * and per-problem argument table. DG_ERR_UNSUPPORTED for more than 65535
 * plans or 2^31 - 1 tiles in all.
 */
dg_status degrid_batch_plan(const dg_plan* plans, int32_t n, dg_batch* out);

/*
 * Degrid every problem of the batch in one launch (Section 2's degridding of
 * each problem, as degrid_execute).
 *   args  host array of 5*n pointers: for problem i,
 *         args[5i+0] subgrids, [5i+1] g_uv, [5i+2] g_w, [5i+3] uvw,
 *         [5i+4] vis_out (all device pointers, as in degrid_execute).
 * The persistent launch is captured into a HIP graph when the batch is
 * planned and replayed on 'stream' by every call; a change of pointers
 * re-uploads the per-problem argument table (a stream-ordered copy from the
 * batch's pinned staging buffer) and keeps the graph.
 */
dg_status degrid_batch_execute(dg_batch b, const void* const* args, hipStream_t stream);
/* (DG_ERR_NOT_READY if one of the plans was re-sorted or re-tuned after the
 * batch was planned.) */

/*
 * Batch autotuner: times every gather kernel variant and tile size on one
 * launch of the whole batch (the given inputs, as for degrid_batch_execute)
 * and leaves every plan set to the fastest choice; a batch planned from
 * these plans afterwards uses it. (The paper picks the visibilities per
 * block, N_b, by measurement, Section 3.) best_kernel and best_n_b, if not
 * NULL, receive the choice. Allocates (rebuilds tile lists and builds
 * trial batches), overwrites the outputs named in args and synchronises the
 * stream. Batches planned from these plans before the call become stale
 * (DG_ERR_NOT_READY).
 */
dg_status degrid_batch_tune(const dg_plan* plans, int32_t n, const void* const* args, hipStream_t stream,
                            int32_t* best_kernel, int32_t* best_n_b);

/* Out-of-range count of the batch's last execute. Synchronises its stream. */
dg_status degrid_batch_oob_count(dg_batch b, int64_t* count);

/* Release a batch (not its plans). NULL is a no-op. */
dg_status degrid_batch_destroy(dg_batch b);

/* Static string naming a status code. */
const char* degrid_status_str(dg_status s);

/* Detail of the last failing call on this thread ("" if none). */
const char* degrid_last_error(void);

/* Library version as major * 10000 + minor * 100 + patch. */
int32_t degrid_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DEGRID_H */
