/*
 * kkt.h -- C ABI of the MI355X (gfx950) segmented block Cholesky KKT solver.
 *
 * Solves Psi x = r (arXiv 2511.00946, Sec. 2, Eq. 2) for block-tridiagonal-arrow
 * SPD matrices Psi (Eq. 3) with uniform stage size b (Sec. 3.1) and a global
 * block of size ng >= 0, for one system or a ragged batch of systems.  The
 * horizon of each system is split into p segments; segments are factored
 * independently (Algorithm 1, parallel phase, Eqs. 4-5), the separator and arrow
 * blocks form a reduced system (Eq. 7) that is factored next (Algorithm 1,
 * sequential phase), and the substitutions sweep the same way (Algorithms 2 and
 * 3, Eqs. 9-12).  p = 1 is the sequential block Cholesky.
 *
 * Precision: FP64 throughout.
 *
 * Memory: every data pointer is a DEVICE pointer owned by the caller.  The
 * library never allocates device memory.  kkt_workspace_init prepares a workspace
 * (and, on its first use on a device, the plan's launch state there: side
 * streams, events, launch shapes) and synchronises the stream; factor and solve
 * calls then only enqueue work -- no allocation, no device query, no host
 * synchronisation -- so they can be captured in a HIP graph, the first call on a
 * workspace included.  When a plan has more than one launch class, the classes
 * of a call run concurrently on streams the plan owns, forked from and joined
 * back into the caller's stream with events: the call stays ordered on the
 * caller's stream.  Scratch lives in the caller's workspace
 * (kkt_plan_info.workspace_bytes, 256-byte aligned).  Calls that share a
 * workspace must not overlap in time; calls of one plan on different workspaces
 * may be made from several host threads (the plan serialises their enqueueing).
 *
 * Data layout (FP64, row-major blocks).  Systems are packed one after another in
 * five pools; kkt_plan_system gives each system's offsets (in doubles):
 *   D      [N, b, b]     D_i   = Psi_{i,i}    (the solver uses (D_i + D_i^T)/2)
 *   C      [N-1, b, b]   C_i   = Psi_{i+1,i}  (Psi_{i,i+1} = C_i^T)
 *   B      [N, ng, b]    B_i   = Psi_{g,i}    (Psi_{i,g} = B_i^T)
 *   corner [ng, ng]      Psi_{g,g}            (the solver uses its symmetric part)
 *   rhs    [N b + ng, nrhs]  stage rows first, g rows last; overwritten by x.
 * With ng = 0 the B and corner pools are empty and may be NULL.
 *
 * Return codes: 0 OK; negative values are launch-time errors (see KKT_E*); on an
 * error nothing of the call runs, except that a launch failure after the first
 * kernel leaves the kernels already queued ordered on the caller's stream.
 * Numerical breakdown is reported per system in the device array info[S]:
 *   0      factorization succeeded;
 *   j > 0  the diagonal block of natural stage j (1-based) met a pivot that is
 *          not positive and finite; j = N + 1 names the corner block.  With
 *          several failures the first in elimination order is reported
 *          (segment stages, then separators, then the corner).
 *   A failed system's solution is set to NaN; other systems are unaffected.
 */
#ifndef KKT_MI355X_H
#define KKT_MI355X_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KKT_OK              0
#define KKT_EDIMS          -1   /* N < 1, b outside 1..48, ng outside 0..16, nrhs outside 1..8,
                                   p > (N+1)/2, or an impossible first-segment length      */
#define KKT_EPOINTER       -2   /* NULL or misaligned pointer                               */
#define KKT_EWORKSPACE     -3   /* workspace not initialised for this plan on the current
                                   device (kkt_workspace_init)                              */
#define KKT_ELAUNCH        -4   /* HIP launch or runtime error                              */
#define KKT_ENOTFACTORED   -5   /* solve before any factorization into this workspace       */
#define KKT_EINTERNAL      -6

#define KKT_MAX_B     48
#define KKT_MAX_NG    16
#define KKT_MAX_NRHS   8
#define KKT_NUM_CLASSES 5       /* padded block sizes 8, 16, 24, 32, 48 */

typedef struct kkt_plan kkt_plan;   /* opaque, host-only */

/* One system's shape.
 *   N   number of stages (diagonal blocks), >= 1
 *   b   stage block size, 1..KKT_MAX_B
 *   ng  global block size, 0..KKT_MAX_NG
 *   p   segments: 1 = sequential method; p >= 2 = segmented method with p
 *       segments (needs N >= 2p - 1); 0 = let the plan's cost model choose.
 *   N1  first-segment length; 0 = the balance rule of Eq. (13): sigma = 19/7
 *       for a given p; for p = 0 the cost model's sigma = t_fill / t_first, the
 *       balance its estimates assume.  Otherwise the other p-1 segments get
 *       (N - N1 - (p-1)) / (p-1) stages, which must be a positive integer.        */
typedef struct {
    int32_t N, b, ng, p, N1;
} kkt_dims;

typedef struct {
    int32_t num_systems;
    int32_t nrhs;
    int32_t num_items;        /* (system, segment) work items                      */
    int32_t num_classes;      /* launch classes (at most 8)                         */
    int64_t D_len, C_len, B_len, corner_len, rhs_len;   /* pool lengths, doubles   */
    int64_t workspace_bytes;
    double  factor_flops;     /* one factorization: standard counts (potrf n^3/3, trsm m n^2,
                                 syrk n^2 k, gemm 2 m n k) of the operations of Algorithm 1 */
    double  solve_flops;      /* one solve, all rhs (trsv n^2, gemv 2 m n; Algorithms 2, 3) */
    int64_t factor_words;     /* |hat L| in doubles, including fill-in             */
    int64_t input_words;      /* |Psi| in doubles (D, C, B, corner pools)           */
} kkt_plan_info;

/* Where one system lives.  Pool offsets in doubles from the pool base; factor
 * offsets in doubles from the workspace's factor region (kkt_plan_factor_offset).
 * The factor is stored block for block in the pattern of the input:
 *   Ld[s]  (b x b, lower)  hat D of segment stages, hat A_k at separators
 *   Lc[s]  (b x b)         the factor block coupling stages s and s+1, oriented as
 *                          in hat L: hat L[s+1, s] (hat E, or hat F_k when s is the
 *                          last stage of segment k), except at a separator s, where
 *                          it is hat L[s, s+1] (hat B^T_{1k}, Eq. 5)
 *   Lb[s]  (ng x b)        hat G of segment stages, hat Q_k at separators
 *   Lg     (ng x ng, lower) hat R
 *   fill   ((N_k - 1) b x b per segment k >= 2) hat B^T_{ik} = hat L[sep_k, (i,k)], i >= 2
 *   H      ((p - 2) b x b) hat H_k = hat L[sep_{k+1}, sep_k], k = 2..p-1        */
typedef struct {
    int32_t N, b, ng, p, N1, Nk;      /* Nk: length of segments 2..p (0 if p = 1) */
    int64_t off_D, off_C, off_B, off_corner, off_rhs;
    int64_t off_Ld, off_Lc, off_Lb, off_Lg, off_fill, off_H;
} kkt_system_layout;

/* Plan a batch of num_systems systems (dims: host array, read during the call),
 * nrhs right-hand sides each.  *plan receives a host object the caller releases
 * with kkt_plan_destroy.  Fails with KKT_EDIMS on an unsupported shape.  Systems
 * with p = 0 get their segment count from the default cost model (below). */
int kkt_plan_create(kkt_plan **plan, int32_t num_systems, const kkt_dims *dims, int32_t nrhs);

/* Cost model used to choose p for systems given with p = 0 (Sec. 3.3: the
 * balance of Eq. 13 and the makespan of Table 1's phases, with measured stage
 * costs).  Per padded block-size class (8, 16, 24, 32, 48): the time of one stage
 * of a first segment (t_first), of a segment carrying fill rows (t_fill,
 * segments 2..p), of one reduced-chain stage (t_red), the fixed cost of an item
 * (t_item), and the number of items the device runs at once, for unsegmented
 * systems (workers) and for the items of segmented ones (workers_seg; 0 = same
 * as workers).  The work of a system counts against the pool its items run in.
 * Units are arbitrary but common.  Segment lengths follow Eq. 13's balance with
 * sigma = t_fill / t_first.  The classes of a batch share the device, so the
 * step is estimated as max(sum over classes of total work / workers, longest
 * item).  The plan searches a bound T on the longest item: every system with
 * p = 0 takes the fewest segments whose longest item stays within T, and the
 * smallest T that the resulting summed work also meets is kept (systems of one
 * class and length get equal p).  Fixed p are honoured and enter the estimate.
 * The default model follows the flop ratios of Table 1 (7/3, 19/3 and 10/3 b^3
 * per stage, t_level = 64 t_first, family 0); a measured one
 * (paper_2511_00946_amd/autotune.py, which also times both families of the 24
 * and 32 classes and keeps the faster) can be passed. */
typedef struct {
    double t_first[KKT_NUM_CLASSES], t_fill[KKT_NUM_CLASSES], t_red[KKT_NUM_CLASSES], t_item[KKT_NUM_CLASSES];
    double workers[KKT_NUM_CLASSES], workers_seg[KKT_NUM_CLASSES];
    double t_level[KKT_NUM_CLASSES];   /* fixed cost of one more level of recursive
                                          segmentation (its extra launches), below */
    double family[KKT_NUM_CLASSES];    /* sweep family of the class (the tile shape):
                                          0 the library's choice, 1 the dense single-wave
                                          sweeps on 32-wide tiles (classes 24 and 32
                                          only), 2 the row-lane sweeps on tiles of the
                                          class's own width                             */
} kkt_cost_model;

int kkt_plan_create_tuned(kkt_plan **plan, int32_t num_systems, const kkt_dims *dims, int32_t nrhs,
                          const kkt_cost_model *model);

/* Recursive (multi-level) segmentation.  Once the segment stages of a system are
 * eliminated, its p - 1 separators carry a reduced system (Sec. 3.2, Eqs. 8-9:
 * diagonal blocks hat A_k, couplings hat H_k between neighbouring separators,
 * arrow blocks hat Q_k, the corner's partial sums) that is itself a
 * block-tridiagonal arrow chain of the same b and ng.  Algorithms 1-3 sweep it
 * sequentially; here it can instead be segmented in turn, and its own reduced
 * chain again, which bounds the sequential depth by the number of levels (the
 * O(log N) method that Sec. 5 names as future work).  p[0] is the segment count
 * of the system's reduced chain, p[1] that of the reduced chain of that chain,
 * and so on; a 0 or 1 ends the recursion (that chain is swept sequentially).
 * Level l needs a chain of M >= 2 p[l] - 1 stages (M = p - 1 for level 0,
 * p[l-1] - 1 below); every level's segments follow Eq. 13's balance.  The
 * factor of a nested system is that of the elimination order the recursion
 * defines: segment stages of the whole chain, then those of the reduced chain,
 * and so on; the separators' blocks live with the reduced systems
 * (kkt_plan_reduced), and info names the first failing block in that order. */
#define KKT_MAX_LEVELS 4
typedef struct {
    int32_t p[KKT_MAX_LEVELS];
    int32_t N1[KKT_MAX_LEVELS];   /* first-segment length of each level's chain, as
                                     kkt_dims.N1 (0: Eq. 13's balance)              */
} kkt_nest;

/* As kkt_plan_create_tuned (model may be NULL: the default model), with nest[s]
 * the recursion of system s (nest may be NULL: none).  nest is read for systems
 * with a given p; for systems with p = 0 the cost model chooses p and the
 * recursion together (a reduced chain of M stages is segmented when the longest
 * path through its levels, t_level each, beats M t_red).  KKT_EDIMS if a level's
 * chain is too short for its segment count. */
int kkt_plan_create_nested(kkt_plan **plan, int32_t num_systems, const kkt_dims *dims, const kkt_nest *nest,
                           int32_t nrhs, const kkt_cost_model *model);

/* Where the reduced chain of system s is factored when it is segmented: *child
 * receives the plan of the reduced systems (owned by plan: do not destroy it),
 * *child_system the index of s's chain in it, and *workspace_offset the byte
 * offset inside plan's workspace of the child's own workspace (its factor region
 * at that offset plus kkt_plan_factor_offset(child)).  The child's systems read
 * their couplings hat H_k from plan's factor region (their off_C is relative to
 * it).  *child is NULL if the chain of s is swept sequentially. */
int kkt_plan_reduced(const kkt_plan *plan, int32_t s, const kkt_plan **child, int32_t *child_system,
                     int64_t *workspace_offset);
/* Releases the plan and its side streams and events.  No call of the plan may be
 * in flight on the host; work already enqueued is unaffected. */
int kkt_plan_destroy(kkt_plan *plan);
int kkt_plan_get_info(const kkt_plan *plan, kkt_plan_info *info);
int kkt_plan_system(const kkt_plan *plan, int32_t s, kkt_system_layout *out);
/* Byte offset of the factor region inside the workspace. */
int64_t kkt_plan_factor_offset(const kkt_plan *plan);

/* Prepare a workspace (device, 256-byte aligned, kkt_plan_info.workspace_bytes
 * bytes) for this plan on the current device: copies the plan's tables into it,
 * on the first workspace of a device also creates the plan's side streams and
 * events there and fixes every launch shape, and synchronises the stream.  Once
 * per workspace before its first use; the plan then forgets any factor it held
 * in this workspace.  Not capturable (it synchronises). */
int kkt_workspace_init(const kkt_plan *plan, void *workspace, hipStream_t stream);

/* Factorization (Algorithm 1).  D, C, B, corner: input pools (device, read
 * only).  info: device int32[S], written per system.  KKT_EWORKSPACE if the
 * workspace was not initialised for this plan on the current device. */
int kkt_factor(const kkt_plan *plan, const double *D, const double *C, const double *B,
               const double *corner, void *workspace, int32_t *info, hipStream_t stream);

/* Forward and backward substitution (Algorithms 2, 3) with a factor already in
 * the workspace; rhs (device, rhs pool layout) is overwritten by x.  Returns
 * KKT_ENOTFACTORED if this plan has not factored into the workspace since its
 * kkt_workspace_init (the same holds for kkt_solve_adjoint). */
int kkt_solve(const kkt_plan *plan, void *workspace, double *rhs, hipStream_t stream);

/* Factorization fused with the forward substitution, then the backward
 * substitution, in one pass over the data: rhs is overwritten by x. */
int kkt_factor_solve(const kkt_plan *plan, const double *D, const double *C, const double *B,
                     const double *corner, void *workspace, double *rhs, int32_t *info,
                     hipStream_t stream);

/* kkt_factor_solve without a caller workspace and without any allocation, for
 * callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, hosts that forbid hipMalloc).  The workspace is a device array
 * inside the library, KKT_NOALLOC_MAX_BYTES bytes on each device it runs on,
 * held until the process ends; plans whose workspace_bytes exceed it get
 * KKT_EWORKSPACE.  The plan's tables are copied into the array (enqueued on
 * stream) whenever it last served another plan.  Every class runs on the
 * caller's stream (no side streams).  All calls on one device share the array:
 * calls that overlap in time on one device race, so the caller orders them
 * (one stream, or events); the factor left in the array is not usable by
 * kkt_solve.  Arguments and results as kkt_factor_solve. */
#define KKT_NOALLOC_MAX_BYTES (32ll << 20)
int kkt_factor_solve_noalloc(const kkt_plan *plan, const double *D, const double *C, const double *B,
                             const double *corner, double *rhs, int32_t *info, hipStream_t stream);

/* Adjoint of x = Psi^{-1} r for a loss L(x) (Psi is symmetric, Eq. 3): given x and
 * gx = dL/dx (rhs pool layout, all nrhs columns), overwrite gx with
 * lambda = Psi^{-1} gx = dL/dr and write the gradients restricted to the block
 * pattern (pools laid out like D, C, B, corner):
 *   dD_i = -sym(lambda_i x_i^T),  dC_i = -(lambda_{i+1} x_i^T + x_{i+1} lambda_i^T),
 *   dB_i = -(lambda_g x_i^T + x_g lambda_i^T),  dcorner = -sym(lambda_g x_g^T),
 * summed over the rhs columns.  Uses the factor in the workspace. */
int kkt_solve_adjoint(const kkt_plan *plan, void *workspace, const double *x, double *gx,
                      double *dD, double *dC, double *dB, double *dcorner, hipStream_t stream);

/* Device-side check of the last call on this workspace: *flag = 0, or
 * KKT_WS_FOREIGN if the workspace held another plan's tables (it was
 * re-initialised by another plan): every kernel of that call then returned
 * without touching its outputs.  Synchronises the stream. */
#define KKT_WS_FOREIGN 2
int kkt_workspace_error(const kkt_plan *plan, const void *workspace, hipStream_t stream, int32_t *flag);

/* Launch class c of the plan (0 <= c < num_classes): padded block size, number
 * of work items, threads per workgroup and LDS bytes of its first launch in the
 * factor-solve mode, and its number of workgroups (as many as fit on the device
 * at once, at most one per item; 0 before kkt_workspace_init on the current
 * device).  Systems are grouped by padded block size (8, 16, 24, 32, 48); in the
 * 16, 24 and 32 groups the unsegmented systems (p = 1) and the segmented ones
 * form two classes (see kkt_plan_class_kind). */
int kkt_plan_class_info(const kkt_plan *plan, int32_t c, int32_t *block_pad, int32_t *num_items,
                        int32_t *threads, int64_t *lds_bytes, int32_t *grid);

/* Kind of launch class c: the row-lane sweeps (one workgroup of one to three
 * 64-lane waves per item, every thread holding one row of a stage's panel:
 * the 8 and 48 groups), whole systems on the dense single-wave sweeps (FP64
 * matrix cores), or segmented systems of the 16/24/32 groups on the dense segment
 * sweeps (their sequential phase, and in the solve-only and adjoint modes the
 * whole class, run on the row-lane sweeps). */
#define KKT_CLASS_ROWLANE          0
#define KKT_CLASS_DENSE            1
#define KKT_CLASS_DENSE_SEGMENTED  2
int kkt_plan_class_kind(const kkt_plan *plan, int32_t c, int32_t *kind);

/* Record start / stop on the class's stream around the launches of class c in
 * every later call (NULL, NULL turns it off).  For measurement: the events are
 * the caller's and must outlive the calls that record them. */
int kkt_plan_set_class_events(kkt_plan *plan, int32_t c, hipEvent_t start, hipEvent_t stop);

const char *kkt_status_string(int status);

/* ---- Non-uniform stage sizes (Sec. 2, Eqs. 1 and 3: stage i of a system has its
 * own size n_i; the method of Sec. 3 assumes one size b).  A system with sizes
 * n_0..n_{N-1} is solved by the plan of the same system with b >= max n_i: each
 * stage is embedded in b x b with the identity on the padded diagonal and zeros in
 * the padded rows and columns of its coupling and arrow blocks, which decouples the
 * padded variables (their solution is 0) and leaves the real ones unchanged (exact).
 * Non-uniform pools, per system, system after system, row-major FP64:
 *   D_i [n_i, n_i], C_i = Psi_{i+1,i} [n_{i+1}, n_i] (i < N-1), B_i [ng, n_i],
 *   corner [ng, ng], rhs [(n_0 + ... + n_{N-1} + ng), nrhs] (stage parts, then g). */
typedef struct kkt_ragged kkt_ragged;   /* opaque: per-stage copy tables on the device */

/* stage_sizes: host array, the N sizes of system 0, then of system 1, ... (plan
 * order); each 1 <= n_i <= b of its system.  Allocates the device tables on the
 * current device (one hipMalloc) and synchronises.  KKT_EDIMS for a size out of
 * range (checked before any device call).  The tables hold offsets only: the plan
 * may be destroyed first. */
int kkt_ragged_create(const kkt_plan *plan, const int32_t *stage_sizes, kkt_ragged **out);
int kkt_ragged_destroy(kkt_ragged *ragged);
/* Lengths (doubles) of the non-uniform pools. */
int kkt_ragged_lengths(const kkt_ragged *ragged, int64_t *D_len, int64_t *C_len, int64_t *B_len,
                       int64_t *corner_len, int64_t *rhs_len);
/* Non-uniform pools (device, read) -> the plan's padded pools (device, written
 * entirely, padding included); enqueued on stream.  Pointers 8-byte aligned; the
 * padded pools are the plan's D/C/B/corner/rhs pools. */
int kkt_ragged_pad(const kkt_ragged *ragged, const double *D, const double *C, const double *B,
                   const double *corner, const double *rhs, double *Dp, double *Cp, double *Bp,
                   double *cornerp, double *rhsp, hipStream_t stream);
/* The real entries of a padded solution (device, the plan's rhs layout) -> x in the
 * non-uniform rhs layout (device); enqueued on stream. */
int kkt_ragged_unpad(const kkt_ragged *ragged, const double *xp, double *x, hipStream_t stream);

/* ---- KKT systems of a multistage QP (Sec. 2, Eq. 1).  The paper takes Psi from
 * the interior-point solver without deriving it; the reading used here is the
 * proximal interior-point Newton system
 *     [ H   A^T   G^T  ] [dx]   [rx]
 *     [ A  -d I    0   ] [dy] = [ry]      H = P + rho I, d = delta > 0, W = diag(w) > 0,
 *     [ G    0   -W^-1 ] [dz]   [rz]
 * (P the Hessian of Eq. 1's cost, A and G its stacked equality and inequality
 * rows), reduced by eliminating dy = (A dx - ry)/d and dz = W (G dx - rz) to
 *     Psi dx = rx + A^T ry / d + G^T W rz,   Psi = P + rho I + A^T A / d + G^T W G,
 * which is SPD with the pattern of Eq. 3.  One interior-point iteration then
 * assembles Psi, factors it once and solves several right-hand sides
 * (kkt_qp_reduce_rhs, kkt_solve, kkt_qp_recover).
 * A system of the plan (N stages of size b, ng globals) gets pe equality and me
 * inequality rows per constraint group (0 <= pe, me <= KKT_QP_MAX_ROWS); group
 * k < N-1 couples x_k, x_{k+1} and g, group N-1 (terminal) x_{N-1} and g.  QP pools,
 * per system, system after system, row-major FP64 (the paper's symbols):
 *   Q  [N, b, b]    Hessian block of x_i (Q_i; Q_N for the last stage)  - the plan's D layout
 *   S  [N-1, b, b]  Hessian block (x_{i+1}, x_i) (S_i)                   - the C layout
 *   T  [N, ng, b]   Hessian block (g, x_i) (T_i; T_N)                   - the B layout
 *   Qg [ng, ng]     Hessian block of g (Q_g)                            - the corner layout
 *   EL [N, pe, b], ER [N-1, pe, b], EG [N, pe, ng]   equality rows of group k on
 *                   x_k (A_k; A_N), on x_{k+1} (B_k), on g (E_k)
 *   IL [N, me, b], IR [N-1, me, b], IG [N, me, ng]   inequality rows (C_k; D_N),
 *                   (D_k), (F_k)
 *   w  [N, me]      positive weights of the inequality rows
 *   ry [N pe, nrhs], rz [N me, nrhs] (and dy, dz)     vectors of the constraint rows
 * rx, dx and the reduced rhs use the plan's rhs layout. */
#define KKT_QP_MAX_ROWS 32
typedef struct kkt_qp kkt_qp;   /* opaque: layouts and device tables */
typedef struct {
    const double *Q, *S, *T, *Qg, *EL, *ER, *EG, *IL, *IR, *IG, *w;   /* device pools */
} kkt_qp_data;

/* n_eq, n_in: host arrays of the plan's S systems (pe, me).  Allocates the device
 * tables and a scratch array on the current device (hipMalloc) and synchronises.
 * KKT_EDIMS for counts out of range (checked before any device call).  Calls on
 * one kkt_qp share its scratch: they must not overlap in time. */
int kkt_qp_create(const kkt_plan *plan, const int32_t *n_eq, const int32_t *n_in, kkt_qp **out);
int kkt_qp_destroy(kkt_qp *qp);
/* Pool lengths (doubles) of the constraint data and vectors (the cost pools have
 * the plan's D, C, B and corner lengths). */
int kkt_qp_lengths(const kkt_qp *qp, int64_t *EL_len, int64_t *ER_len, int64_t *EG_len, int64_t *IL_len,
                   int64_t *IR_len, int64_t *IG_len, int64_t *w_len, int64_t *ry_len, int64_t *rz_len);
/* Offsets (doubles) of system s in those pools, in the order of kkt_qp_lengths. */
int kkt_qp_offsets(const kkt_qp *qp, int32_t s, int64_t offsets[9]);
/* Psi -> the plan's D, C, B, corner pools (device, written entirely); rho >= 0,
 * delta > 0.  D may alias Q (and C S, B T, corner Qg).  Enqueued on stream. */
int kkt_qp_assemble(const kkt_qp *qp, const kkt_qp_data *data, double rho, double delta, double *D, double *C,
                    double *B, double *corner, hipStream_t stream);
/* rhs = rx + A^T ry / delta + G^T W rz (the plan's rhs layout; rhs may alias rx). */
int kkt_qp_reduce_rhs(const kkt_qp *qp, const kkt_qp_data *data, double delta, const double *rx, const double *ry,
                      const double *rz, double *rhs, hipStream_t stream);
/* dy = (A dx - ry) / delta, dz = W (G dx - rz). */
int kkt_qp_recover(const kkt_qp *qp, const kkt_qp_data *data, double delta, const double *dx, const double *ry,
                   const double *rz, double *dy, double *dz, hipStream_t stream);

/* ---- The interior-point loop around these solves (the paper runs its solver
 * inside PIQP and does not describe the iteration; the reading used here): a
 * primal-dual method with Mehrotra's predictor-corrector for
 *     min 1/2 x^T P x + c^T x   s.t.   A x = beq,   G x + s = h,   s >= 0,
 * each of whose Newton systems is the regularised one above with the proximal
 * centres at the current iterate (the regularisation vanishes in the residuals,
 * so the fixed point is the exact KKT point).  Per iteration, per system: the
 * residuals r_d = P x + c + A^T y + G^T z, r_p = A x - beq, r_s = G x + s - h and
 * mu = s^T z / m; a system stops when max |r| <= tol and mu <= tol; otherwise
 * w = z / (s + delta z), Psi is assembled and factored once, and two right-hand
 * sides are solved: the predictor (rx, ry, rz) = (-r_d, -r_p, -r_s + s) and the
 * corrector with rz = -r_s - (-s z + sigma mu - ds_aff dz_aff) / z, sigma =
 * (mu_aff / mu)^3; ds = -r_s - rz - dz / w; the step is min(1, 0.99 times the
 * largest step keeping s, z >= 0).  Start: from x = 0, y = 0, s = z = 1 the full
 * predictor step, then s and z moved into the interior by Mehrotra's heuristic
 * (s += max(-1.5 min s, 0), likewise z, then s += s^T z / (2 sum z), z += s^T z /
 * (2 sum s)); systems without inequality rows start at x = 0.  rho and delta are
 * the regularisation of the start step; iteration k uses them times
 * max(1e-4, 10^-(k+1)) (proximal methods shrink it as they converge).
 * Vectors: c and x in the plan's rhs layout, beq and y in the ry layout, h, z and
 * s in the rz layout (one column: the plan must have nrhs = 1). */
typedef struct kkt_ipm kkt_ipm;   /* opaque: work vectors and per-system state */

/* Allocates the work vectors on the current device (hipMalloc, pinned host word).
 * KKT_EDIMS if the plan has nrhs != 1 or is not qp's plan size.  plan and qp must
 * outlive it. */
int kkt_ipm_create(const kkt_plan *plan, const kkt_qp *qp, kkt_ipm **out);
int kkt_ipm_destroy(kkt_ipm *ipm);
/* Runs the loop on stream (it synchronises once per iteration to test whether
 * any system still runs; not capturable).  workspace: initialised for the plan.
 * data: the QP pools (data->w is not read: the loop keeps its own weights).
 * x, y, z, s (device) receive the iterates; status (device int32[S]) the
 * iterations each system took to converge, -1 if a factorization failed, -2 if it
 * did not converge within max_iter. */
int kkt_ipm_solve(kkt_ipm *ipm, void *workspace, const kkt_qp_data *data, const double *c, const double *beq,
                  const double *h, double rho, double delta, double tol, int32_t max_iter, double *x, double *y,
                  double *z, double *s, int32_t *status, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* KKT_MI355X_H */
