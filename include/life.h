/*
 * life.h - C ABI of the MI355X (gfx950) library for the hot path of the Linear
 * Fascicle Evaluation (LiFE) method: the two sparse-Tucker-decomposed products
 * that every SBB-NNLS iteration runs, and the iteration itself.
 *
 * Source: Aggarwal & Bondhugula, "Optimizing the Linear Fascicle Evaluation
 * Algorithm for Multi-Core and Many-Core Systems" (arxiv 1905.06234).
 *
 * Model.  The diffusion signal y (N_theta*N_v values) is approximated by M w
 * (Sec. 2.1, eq. 1), with M never formed: for each voxel v, M_v = D Phi_v
 * (eq. 3, with the S0(v) factor folded into the Phi values), i.e. the tensor
 * form Y = Phi x1 D x2 S0 x3 w^T (eq. 4).  Phi is given as one
 * (atom, voxel, fascicle, value) entry per nonzero (Sec. 2.2: the atoms,
 * voxels, fibers and values vectors).
 *
 * Conventions for every call:
 *   - Indices are 0-based.  atom is int16, voxel and fascicle are int32.
 *   - D is N_theta x N_a, stored theta-fastest: D[t + N_theta*a] (the offset
 *     rule "N_theta times the index" of Sec. 4.1).  Signals (y, b, r) are
 *     stored theta-fastest per voxel: y[t + N_theta*v].
 *   - Floating point data are IEEE float32; scalar reductions inside
 *     life_sbbnnls_step are carried in float64.
 *   - "device" pointers are HIP device memory on the device the plan was built
 *     on; "host" pointers are ordinary host memory.
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).
 *     life_dsc, life_wc and life_sbbnnls_step only enqueue work: they never
 *     allocate, free or synchronize.
 *   - Results are deterministic: the same plan and inputs give bitwise equal
 *     outputs on every call (fixed reduction orders, no atomics).
 *   - Workspace: everything a call writes besides its outputs (weights in the
 *     plan's fascicle order, WC pass-1 values, the SBB vectors and partial sums).
 *     A plan owns one, used by the calls that take no scratch argument; calls
 *     that share it must not overlap in time (enqueue them on one stream, or
 *     order the streams).  life_dsc_ws, life_wc_ws and life_sbbnnls_step_ws take
 *     the caller's scratch instead (life_plan_scratch_bytes bytes), so one plan
 *     serves several streams at once, one scratch buffer per stream.  The plan's
 *     own arrays are only read by these calls.
 *   - Every function returns a life_status; on an error nothing is enqueued
 *     and outputs are left untouched unless stated.
 */
#ifndef LIFE_H
#define LIFE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LIFE_OK = 0,
    LIFE_EINVAL = 1,  /* NULL pointer, negative size, dimension out of its limits */
    LIFE_ERANGE = 2,  /* an index outside [0, n), or nnz beyond 2^31 - 2 */
    LIFE_ENOMEM = 3,  /* host or device allocation failed */
    LIFE_EDEVICE = 4  /* HIP runtime error (no device, wrong device, launch failure) */
} life_status;

/* Problem dimensions.  Limits: 1 <= n_theta <= 1024; 1 <= n_atoms <= 32767;
 * n_voxels, n_fascicles >= 0; 0 <= nnz <= 2^31 - 2.  nnz = 0 is legal (M = 0). */
typedef struct {
    int32_t n_theta;      /* N_theta: diffusion directions (rows of D)          */
    int32_t n_atoms;      /* N_a: dictionary atoms (columns of D)                 */
    int32_t n_voxels;     /* N_v                                                  */
    int32_t n_fascicles;  /* N_f: length of w                                     */
    int64_t nnz;          /* N_c: nonzeros of Phi                                 */
} life_dims;

/* Opaque plan: the restructured (sorted) copies of Phi on one device, plus the
 * workspace of the calls below. */
typedef struct life_plan_s *life_plan_t;

/* Device-resident state of SBB-NNLS (Algorithm 1), written by
 * life_sbbnnls_step.  Zero it (all bytes) to start at iteration 0; to resume,
 * keep w and set iter. */
typedef struct {
    int64_t iter;      /* i: the next iteration to run (counted from 0)                */
    double alpha;      /* alpha^(i) used by the last completed iteration               */
    double obj;        /* f(w^(i)) = 1/2 ||M w^(i) - b||^2 (eq. 2) at that iteration   */
    double gt_norm2;   /* ||g~||^2 of the projected gradient at that iteration         */
    double num;        /* numerator of that alpha                                      */
    double den;        /* denominator of that alpha (0 -> alpha = 0, w unchanged)      */
} life_sbb_state;

/* Kernel classes reported by the profiling hooks. */
typedef enum {
    LIFE_K_DSC = 0,        /* y = M w (voxel-segmented)                          */
    LIFE_K_WC_Z = 1,       /* WC pass 1: per-nonzero projections, voxel order     */
    LIFE_K_WC_SUM = 2,     /* WC pass 2: per-fascicle sums                        */
    LIFE_K_MASK = 3,       /* projected gradient g~ and ||g~||^2 partials          */
    LIFE_K_ALPHA = 4,      /* step length from the partial sums                   */
    LIFE_K_UPDATE = 5,     /* w <- [w - alpha g~]_+                               */
    LIFE_K_WC_Z_2ND = 6,   /* WC pass 1 of v'' = M^T v' (SBB, gated by parity)    */
    LIFE_K_WC_SUM_2ND = 7, /* WC pass 2 of v'' (SBB, gated by parity)             */
    LIFE_K_PERMUTE = 8,    /* weights into the plan's fascicle order              */
    LIFE_K_DD = 9,         /* dictionary gradient (per-group partials)            */
    LIFE_K_DD_REDUCE = 10, /* dictionary gradient: sum of the partials            */
    LIFE_K_COUNT = 11
} life_kernel_kind;

/* Human-readable name of a status code (static string; never NULL). */
const char *life_status_str(life_status s);

/* The HIP runtime's message for the last device error that a kernel launch of
 * this library ran into on the calling thread ("" if none): the detail behind a
 * LIFE_EDEVICE (static string; never NULL). */
const char *life_hip_error(void);

/* Restructuring on the host only (no device touched): the data-restructuring
 * step of Sec. 4.1 ("Data Restructuring": voxel-based for DSC; fiber-based,
 * i.e. by fascicle, for WC) as two permutations with their segment offsets.
 * Voxels are processed in a locality order: voxel index order, or, when grid
 * coordinates are given, the Morton (Z-order) sequence of the coordinates (ties
 * by index).  Fascicles are ranked by the Z-order (bit interleave) of the first
 * and last processing positions of the voxels they cross (ties by fascicle index,
 * empty fascicles last), so that fascicles crossing the same voxels have nearby
 * ranks.
 *   atom, voxel, fascicle: host, nnz entries each (input COO order).
 *   voxel_xyz (host, 3*n_voxels, optional): non-negative (x, y, z) grid
 *                                   coordinates of each voxel, or NULL.
 *   dsc_perm  (host, nnz):          input positions in DSC order, the total order
 *                                   (voxel, atom, fascicle, input position).
 *   vox_ptr   (host, n_voxels+1):   voxel v owns DSC positions [vox_ptr[v], vox_ptr[v+1]).
 *   fas_rank  (host, n_fascicles):  processing rank of each fascicle (a permutation).
 *   wc_perm   (host, nnz):          for WC slot j, its position in the DSC order; WC
 *                                   slots follow (fas_rank[fascicle], voxel position,
 *                                   atom, fascicle, input position).
 *   fas_ptr   (host, n_fascicles+1): the fascicle of rank r owns WC slots
 *                                   [fas_ptr[r], fas_ptr[r+1]).
 * Any output may be NULL (not written).  Errors: LIFE_EINVAL (dims or a needed
 * pointer NULL), LIFE_ERANGE (an index or a coordinate out of range), LIFE_ENOMEM. */
life_status life_plan_host(const life_dims *dims, const int16_t *atom, const int32_t *voxel,
                           const int32_t *fascicle, const int16_t *voxel_xyz, int32_t *dsc_perm,
                           int32_t *vox_ptr, int32_t *fas_rank, int32_t *wc_perm, int32_t *fas_ptr);

/* Build a plan on the current HIP device from host COO arrays (Sec. 2.2 Phi
 * vectors; restructuring of Sec. 4.1 done once and amortized over the
 * iterations, as the paper does before SBB-NNLS).  Copies the sorted arrays to
 * the device and allocates the workspace.  Synchronous.  The inputs are not
 * retained.  On success *out owns device memory until life_plan_destroy.
 * Errors: LIFE_EINVAL, LIFE_ERANGE (index checks happen here, once),
 * LIFE_ENOMEM, LIFE_EDEVICE. */
life_status life_plan(const life_dims *dims, const int16_t *atom, const int32_t *voxel,
                      const int32_t *fascicle, const float *phi, life_plan_t *out);

/* life_plan with the voxels' grid coordinates (host, 3*n_voxels, non-negative;
 * NULL = life_plan): the plan then processes voxels in Morton order, so each
 * 64-voxel work chunk is a compact block and the WC gathers stay local (see
 * life_plan_host).  Results are the same products; only summation orders and
 * speed differ.  Errors: as life_plan; LIFE_ERANGE for a negative coordinate. */
life_status life_plan_ex(const life_dims *dims, const int16_t *atom, const int32_t *voxel,
                         const int32_t *fascicle, const float *phi, const int16_t *voxel_xyz,
                         life_plan_t *out);

/* Flags of life_plan_flags. */
enum {
    LIFE_PLAN_DEVICE_INPUT = 1, /* atom, voxel, fascicle, phi are device pointers (else host) */
    LIFE_PLAN_HOST_BUILD = 2    /* restructure on the host (the reference builder; slower)   */
};

/* Words written by life_plan_digest. */
#define LIFE_DIGEST_WORDS 24

/* The general plan builder (life_plan, life_plan_ex and life_plan_batch call it
 * with flags = 0): n_inst = 1 builds a single problem (vox_off, fas_off may then
 * be NULL), n_inst > 1 a batched plan as life_plan_batch.  The restructuring of
 * Sec. 4.1 (the sorts by voxel and by fascicle and the chunked layout derived
 * from them) runs on the device with stable radix sorts, scans and gathers, and
 * gives the same plan, bit for bit, as the host builder (LIFE_PLAN_HOST_BUILD),
 * which stays available as the reference.  With LIFE_PLAN_DEVICE_INPUT the COO
 * arrays are device memory of the current device (not retained; nothing is
 * copied from the host).  The host builder is also used when N_theta > 128 or a
 * voxel crosses more fascicles than a chunk holds (16384 at most).
 * tile_atoms: 0 = the default dictionary tiling (as many atoms per LDS tile as
 * 104 KB holds, then balanced), else at most that many atoms per tile (the
 * tiles are balanced; fewer atoms per tile leave more LDS to the chunk's
 * fascicle list; ignored when N_theta > 128).  Results are the same products for
 * every tiling; summation orders differ.  Synchronous.
 * Errors: as life_plan_batch; LIFE_EINVAL for unknown flags, tile_atoms < 0, or a
 * tiling whose LDS blocks do not fit (checked before any device is touched). */
life_status life_plan_flags(const life_dims *dims, int32_t n_inst, const int32_t *vox_off, const int32_t *fas_off,
                            const int16_t *atom, const int32_t *voxel, const int32_t *fascicle, const float *phi,
                            const int16_t *voxel_xyz, uint32_t flags, int32_t tile_atoms, life_plan_t *out);

/* Atoms per dictionary tile of a plan (host output; 0 for the generic kernels
 * used when N_theta > 128 or a chunk's fascicles overflow). */
life_status life_plan_tile_atoms(life_plan_t plan, int32_t *tile_atoms);

/* Choose the plan's geometry by measurement (the paper picks its kernel
 * variants by timing runs on the input, Sec. 4.1), extended from the schedule
 * to the dictionary tiling: a plan is built (as life_plan_flags, device
 * builder) for each tiling of 3 to 8 balanced tiles that fits the LDS, each
 * times reps DSC+WC pairs on D and fixed pseudo-random w and y, the fastest is
 * kept and life_plan_tune then picks its schedule.  Every candidate computes
 * the same products; only summation orders and speed differ.
 *   flags: 0 or LIFE_PLAN_DEVICE_INPUT (as life_plan_flags).
 *   D: device, the dictionary the plan will be used with (N_theta x N_a).
 *   tile_atoms_out, policy_out (host, optional): the chosen tiling and schedule.
 * Allocates two signals and two weight vectors of scratch for the timing;
 * synchronizes the device.  Errors: as life_plan_flags; LIFE_EINVAL for
 * reps < 1 or a missing D. */
life_status life_plan_autotune(const life_dims *dims, int32_t n_inst, const int32_t *vox_off,
                               const int32_t *fas_off, const int16_t *atom, const int32_t *voxel,
                               const int32_t *fascicle, const float *phi, const int16_t *voxel_xyz, uint32_t flags,
                               const float *D, int32_t reps, int32_t *tile_atoms_out, int32_t *policy_out,
                               life_plan_t *out);

/* Digest of every array of a plan (one 64-bit FNV-1a hash per array, the last
 * word over the layout's sizes), to compare plans bit for bit.  digest: host,
 * LIFE_DIGEST_WORDS entries.  Synchronous.  Errors: LIFE_EINVAL, LIFE_ENOMEM,
 * LIFE_EDEVICE. */
life_status life_plan_digest(life_plan_t plan, uint64_t *digest);

/* A batched plan: n_inst independent problems that share the dictionary D,
 * given as one block-diagonal problem.  The caller concatenates the instances:
 * instance k owns voxels [vox_off[k], vox_off[k+1]) and fascicles
 * [fas_off[k], fas_off[k+1]) of the union (dims describes the union); every
 * nonzero's voxel and fascicle belong to the same instance.  One launch of each
 * product then covers all instances; no work chunk spans two instances, so
 * life_sbbnnls_step_batch can keep separate step lengths.  D, w, y, b and g are
 * the concatenations of the instances' vectors.
 *   vox_off, fas_off (host, n_inst + 1 entries: 0 = first, last = union size).
 *   Other arguments as life_plan_ex (voxel_xyz optional, Morton order inside
 *   each instance).
 * Errors: LIFE_EINVAL (bad offsets, n_inst < 1, N_theta > 128 with n_inst > 1),
 * LIFE_ERANGE (an index out of range or a nonzero that crosses instances),
 * LIFE_ENOMEM, LIFE_EDEVICE. */
life_status life_plan_batch(const life_dims *dims, int32_t n_inst, const int32_t *vox_off, const int32_t *fas_off,
                            const int16_t *atom, const int32_t *voxel, const int32_t *fascicle, const float *phi,
                            const int16_t *voxel_xyz, life_plan_t *out);

/* The restructuring of a batched plan on the host only (no device touched):
 * voxel processing positions (proc_pos, host, n_voxels: instance by instance,
 * each instance's block padded to whole 64-voxel chunks; Morton order inside an
 * instance when voxel_xyz is given, else voxel order), and the permutations and
 * offsets of life_plan_host over the union.  Fascicles are ranked instance by
 * instance (the instance is the major key, so instance k's fascicles take exactly
 * the ranks [fas_off[k], fas_off[k+1])); inside an instance by the Z-order of the
 * first and last processing positions of their voxels (ties by fascicle index),
 * those without nonzeros last.  Arguments and errors as life_plan_batch /
 * life_plan_host; any output may be NULL. */
life_status life_plan_host_batch(const life_dims *dims, int32_t n_inst, const int32_t *vox_off,
                                 const int32_t *fas_off, const int16_t *atom, const int32_t *voxel,
                                 const int32_t *fascicle, const int16_t *voxel_xyz, int32_t *proc_pos,
                                 int32_t *dsc_perm, int32_t *vox_ptr, int32_t *fas_rank, int32_t *wc_perm,
                                 int32_t *fas_ptr);

/* Number of instances of a plan (1 unless built by life_plan_batch). */
life_status life_plan_instances(life_plan_t plan, int32_t *n_inst);

/* Choose the plan's work schedule by measurement (the paper selects its
 * kernels by timing runs on the input, Sec. 4.1): every workgroup-to-chunk
 * schedule (index order; XCD-contiguous ranges of equal count; of equal work)
 * times reps DSC+WC pairs on (D, w, y) and the fastest is kept.  Results do
 * not depend on the schedule.  D, w, y: device inputs as life_dsc/life_wc.
 * policy (host, optional): the chosen schedule (0, 1, 2).  Synchronizes the
 * device; uses the plan's workspace.  The schedule is rewritten in place (same
 * device addresses and launch grids), so graphs captured on the plan before the
 * call stay valid and run the chosen schedule. */
life_status life_plan_tune(life_plan_t plan, const float *D, const float *w, const float *y, int32_t reps,
                           int32_t *policy);

/* Release a plan and its device memory (synchronizes the device first).
 * NULL is accepted and ignored. */
life_status life_plan_destroy(life_plan_t plan);

/* Dimensions the plan was built with (host output). */
life_status life_plan_dims(life_plan_t plan, life_dims *out);

/* Copy the plan's device arrays to host buffers (any may be NULL): the DSC
 * order arrays vox_ptr (n_voxels+1), atom_v, fas_v (fascicle ranks), phi_v
 * (nnz each), fas_rank (n_fascicles) and the WC order arrays fas_ptr
 * (n_fascicles+1) and wc_perm (nnz), as life_plan_host defines them.
 * Synchronous. */
life_status life_plan_export(life_plan_t plan, int32_t *vox_ptr, int16_t *atom_v, int32_t *fas_v,
                             float *phi_v, int32_t *fas_rank, int32_t *fas_ptr, int32_t *wc_perm);

/* DSC, the diffusion signal computation y = M w (eq. 1; Sec. 2.2, the "daxpy"
 * form of the inner loop): y[t + N_theta*v] = sum over nonzeros c of voxel v of
 * D[t + N_theta*atom_c] * phi_c * w[fascicle_c].
 *   D (device, N_theta*N_a), w (device, N_f) are read; y (device, N_theta*N_v) is
 *   overwritten (voxels with no nonzero get 0).  Nonzeros of a zero weight add
 *   nothing (Sec. 2.2): in a 64-voxel chunk where at least 1/8 of the weights are
 *   zero, their products are skipped (the sums of the others keep their order
 *   and value); elsewhere they add an exact zero.
 * Errors: LIFE_EINVAL (NULL plan or pointer with a nonzero size), LIFE_EDEVICE. */
life_status life_dsc(life_plan_t plan, const float *D, const float *w, float *y, void *stream);

/* WC, the weight computation g = M^T y (the transpose product of eq. 6; Sec. 2.2,
 * the "dot-product" form): g[f] = sum over nonzeros c of fascicle f of
 * phi_c * sum_t D[t + N_theta*atom_c] * y[t + N_theta*voxel_c].
 *   D (device), y (device, N_theta*N_v) are read; g (device, N_f) is
 *   overwritten (fascicles with no nonzero get 0).
 * Precision: with N_theta <= 128 the inner products <D[:,a], y[:,v]> are formed
 *   on the matrix cores as exact integer sums of 8-bit digit products: each
 *   column of D and of y is scaled by a power of two and rounded to a 30-bit
 *   integer (to 2^-31 of its largest magnitude), the digit products of weight
 *   2^16 and below are dropped, and the sum is rounded once to float; the sums
 *   over nonzeros are FP32 in a fixed order.  Larger N_theta uses FP32 FMAs.
 * Errors: as life_dsc. */
life_status life_wc(life_plan_t plan, const float *D, const float *y, float *g, void *stream);

/* Bytes of the caller scratch that life_dsc_ws, life_wc_ws and
 * life_sbbnnls_step_ws take (the size of the plan's own workspace).  *bytes
 * (host) is written.  Errors: LIFE_EINVAL (NULL argument). */
life_status life_plan_scratch_bytes(life_plan_t plan, uint64_t *bytes);

/* life_dsc and life_wc with the caller's scratch in place of the plan's
 * workspace.  scratch (device, 256-byte aligned, scratch_bytes >=
 * life_plan_scratch_bytes) is overwritten; it must not be used by another call
 * in flight.  scratch = NULL selects the plan's workspace (same as life_dsc /
 * life_wc).  Results are bitwise the same as those of life_dsc / life_wc.
 * Errors: as life_dsc; LIFE_EINVAL also for a scratch that is too small or
 * misaligned. */
life_status life_dsc_ws(life_plan_t plan, const float *D, const float *w, float *y, void *scratch,
                        uint64_t scratch_bytes, void *stream);
life_status life_wc_ws(life_plan_t plan, const float *D, const float *y, float *g, void *scratch,
                       uint64_t scratch_bytes, void *stream);

/* life_dsc for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and bitwise the same y, with the call's workspace (the weights in the
 * plan's fascicle order, 4 * n_fascicles bytes rounded up to 256) in a static
 * device array of 64 MiB that the library holds on each device it runs on until
 * the process ends.  The call allocates and frees nothing and creates no events
 * (the profiling hooks do not record it).  Every call on one device shares that
 * device's array: calls that overlap in time on one device race (enqueue them on
 * one stream, or order the streams).  Arguments as life_dsc.
 * Errors: as life_dsc; LIFE_ERANGE when the workspace exceeds 64 MiB
 * (n_fascicles above 16,777,216). */
life_status life_dsc_noalloc(life_plan_t plan, const float *D, const float *w, float *y, void *stream);

/* One SBB-NNLS iteration, Algorithm 1 (Sec. 2.1) with eqs. 5-6:
 *   r  = M w - b;   g = M^T r  (the gradient, eq. 6);
 *   g~ = g with g_f set to 0 where w_f = 0 and g_f > 0 (projected gradient);
 *   v' = M g~;
 *   i odd : alpha = <g~,g~> / <v',v'>;
 *   i even: v'' = M^T v';  alpha = <v',v'> / <v'',v''>;
 *   (a zero denominator gives alpha = 0)
 *   w <- [w - alpha g~]_+  (eq. 5; non-positive results become +0).
 * i is state->iter; the call increments it and records alpha, f(w), ||g~||^2,
 * numerator and denominator in *state.  Two DSC and, on even i, two WC (one WC
 * on odd i) run per call: on average 2 and 1.5, as the paper counts.
 *   D (device), b (device, N_theta*N_v) are read; w (device, N_f) is updated in
 *   place; state (device) is read and written.  Everything stays on the device.
 * Errors: as life_dsc. */
life_status life_sbbnnls_step(life_plan_t plan, const float *D, const float *b, float *w,
                              life_sbb_state *state, void *stream);

/* life_sbbnnls_step with the caller's scratch in place of the plan's workspace
 * (arguments as life_dsc_ws: scratch is device memory of at least
 * life_plan_scratch_bytes bytes, 256-byte aligned; NULL = the plan's own).
 * Bitwise the same results as life_sbbnnls_step.  Errors: as life_dsc_ws. */
life_status life_sbbnnls_step_ws(life_plan_t plan, const float *D, const float *b, float *w,
                                 life_sbb_state *state, void *scratch, uint64_t scratch_bytes, void *stream);

/* One SBB-NNLS iteration with the step lengths of eqs. 7-8 as printed, i.e. the
 * classic lagged Barzilai-Borwein form: alpha^(i) is evaluated at q, the
 * projected gradient of the previous iterate (at i = 0, the current one):
 *   r, g, g~ as in life_sbbnnls_step;   v' = M q;
 *   i even: alpha = <q,q> / <v',v'>                                 (eq. 7)
 *   i odd : v'' = M^T v';  alpha = <v',v'> / <v'',v''>               (eq. 8)
 *   (a zero denominator gives alpha = 0);   w <- [w - alpha g~]_+   (eq. 5).
 *   gt_prev (device, N_f, caller's fascicle order): read as q when i > 0 (not
 *   read at i = 0), then overwritten with this iteration's g~, ready for the
 *   next call.  Two DSC and, on odd i, two WC per call.
 *   Other arguments, state and errors as life_sbbnnls_step. */
life_status life_sbbnnls_step_lagged(life_plan_t plan, const float *D, const float *b, float *w,
                                     float *gt_prev, life_sbb_state *state, void *stream);

/* Gradient with respect to the dictionary of the DSC product: with y = M(D) w
 * (eq. 1, M_v = D Phi_v of eq. 3 with S0 folded into Phi; y is linear in D),
 *   dD[t + N_theta*a] = d<ybar, M(D) w>/dD[t, a]
 *                     = sum over nonzeros c with atom_c = a of
 *                       phi_c * w[fascicle_c] * ybar[t + N_theta*voxel_c].
 * With ybar = 2 (M w - y_obs) this is the dictionary gradient of the loss
 * ||y_obs - M(D) w||^2; the weight gradient is life_wc of the same ybar.  The
 * paper fits w only; this call serves dictionary learning over the same encoding.
 *   w (device, N_f) and ybar (device, N_theta*N_v) are read; dD (device,
 *   N_theta*N_a) is overwritten (atoms with no nonzero get 0).  Deterministic.
 * Errors: as life_dsc. */
life_status life_dict_grad(life_plan_t plan, const float *w, const float *ybar, float *dD, void *stream);

/* One SBB-NNLS iteration (Algorithm 1, as life_sbbnnls_step) of every instance
 * of a batched plan, in one pass of each product over all instances.  Each
 * instance k has its own step length and scalars in states[k] (device,
 * n_inst entries); the instances advance together (the second WC runs on the
 * iterations where states[0].iter is even).  D (device), b (device, union
 * signal) are read; w (device, union weights) is updated in place.  A plan with
 * one instance takes the same path (its scalars summed per instance).
 * Errors: as life_sbbnnls_step. */
life_status life_sbbnnls_step_batch(life_plan_t plan, const float *D, const float *b, float *w,
                                    life_sbb_state *states, void *stream);

/* Profiling hooks for the benchmark: when enabled, every kernel the plan
 * launches is bracketed by HIP events on its stream.  The two launches of an
 * SBB step's second WC (v'' = M^T v') are recorded under their own kinds: on
 * the iterations that do not need it they are enqueued but return at once.
 * life_profile_read
 * synchronizes those events, writes per-kind total milliseconds and launch
 * counts (arrays of LIFE_K_COUNT entries, host; either may be NULL) and
 * resets the record. */
life_status life_profile_enable(life_plan_t plan, int enable);
life_status life_profile_read(life_plan_t plan, double *ms, int64_t *count);

#ifdef __cplusplus
}
#endif

#endif /* LIFE_H */
