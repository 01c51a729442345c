/*
 * ifgf.h -- C ABI of the MI355X (gfx950) IFGF operator library.
 *
 * The library evaluates the discrete operator of Bauinger and Bruno, "IFGF:
 * Interpolated Factored Green Function method" (arXiv 2010.02857), Sec. 2,
 * eq. (field1) with the Helmholtz kernel of eq. (greensfunction):
 *
 *     I_r(x_l) = sum_{m != l} a_r(x_m) e^{i k |x_l - x_m|} / (4 pi |x_l - x_m|),
 *
 * for N points x_1..x_N that serve as both sources and targets, by the
 * O(N log N) IFGF algorithm of Sec. 3.3 (Algorithm 1): octree of boxes, cone
 * segments per box, leaf-level direct evaluation at the cone interpolation
 * points, child-to-parent Chebyshev interpolation with re-centring by the
 * centred factor, direct near-field sums, and interpolation at the cousin
 * targets of every level.
 *
 * Conventions common to every call:
 *   - Every call returns an ifgf_status; no C++ exception crosses the ABI.
 *     On failure ifgf_last_error() returns a message for the calling thread.
 *   - "device" pointers are HIP device allocations on the GPU that was
 *     current when the plan was created; "host" pointers are ordinary memory.
 *   - Complex arrays are interleaved (re, im).  With precision IFGF_FP64 they
 *     are complex128 (two doubles); with IFGF_MIXED complex64 (two floats).
 *   - A batch of nrhs vectors is laid out [nrhs][n]: vector r occupies
 *     elements r*n .. r*n + n - 1, in the order the points were given.
 *   - `stream` is a hipStream_t passed as void* (NULL: the null stream).  The
 *     apply calls are asynchronous on it; argument errors are reported
 *     synchronously, kernel launch failures as IFGF_E_HIP.  An apply or
 *     gradient call also runs part of its work (near field, cousin
 *     evaluations) on a second stream the plan owns, at default priority:
 *     that stream waits on `stream` for the call's inputs, touches only the
 *     plan's workspaces, and `stream` waits on it before the call's last
 *     kernel, so the call as a whole is ordered on `stream`.
 *     IFGF_SIDE_STREAM=0 in the environment keeps everything on `stream`.
 *   - A plan owns all device memory it allocates (tree, cone tables, cone
 *     value buffers).  It may be used by one stream at a time: its
 *     workspaces are shared, and concurrent calls on one plan race.
 */
#ifndef IFGF_H
#define IFGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ifgf_plan* ifgf_plan_t;

typedef enum {
    IFGF_OK = 0,
    IFGF_E_INVALID_ARG = 1,   /* bad argument (pointer, size, duplicate points) */
    IFGF_E_OUT_OF_MEMORY = 2, /* host or device allocation failed, or the
                                 workspace limit is too small                 */
    IFGF_E_HIP = 3,           /* a HIP runtime call or kernel launch failed   */
    IFGF_E_UNSUPPORTED = 4,   /* valid request the library cannot serve       */
    IFGF_E_INTERNAL = 5
} ifgf_status;

typedef enum {
    IFGF_FP64 = 0,  /* all arithmetic in FP64; complex128 input and output    */
    IFGF_MIXED = 1  /* FP64 for distances, the phase k r and its reduction
                       modulo 2 pi, box centres and the cone-coordinate map
                       (s, theta, phi); FP32 for interpolation, kernel values
                       and accumulation; complex64 input and output           */
} ifgf_precision;

#define IFGF_MAX_LEVELS 24

/* Plan options.  Zero-initialised fields take the defaults noted. */
typedef struct {
    int32_t leaf_ns;         /* radial cone intervals per leaf box, n_{s,D}
                                (0: 1, the paper's choice, Sec. 4)            */
    int32_t leaf_nc;         /* polar cone intervals per leaf box, n_{C,D};
                                there are 2 n_{C,D} azimuthal ones (0: 2)    */
    int32_t precision;       /* ifgf_precision (0: IFGF_FP64)                 */
    int32_t max_nrhs;        /* largest nrhs an apply call may pass; sizes
                                the workspaces (0: 16)                        */
    int32_t store_levels;    /* cone values of every level kept after an
                                apply for ifgf_grad_targets: 1 keep, 0
                                recompute them in the gradient call, -1 keep
                                them if they fit in a quarter of the free
                                device memory                                 */
    int32_t host_only;       /* 1: build the hierarchy on the host only (no
                                GPU use); apply calls return
                                IFGF_E_UNSUPPORTED but ifgf_plan_stats works */
    int32_t no_dilate;       /* 1: mark only the cone a query point falls in;
                                0: also mark the neighbouring cone when the
                                point lies within 1e-10 (local coordinates)
                                of a cone face, so that the GPU's own
                                evaluation of the point's cone always finds
                                computed data                                 */
    int32_t use_graph;       /* 1: ifgf_apply / ifgf_apply_adjoint capture
                                their kernel launches into a HIP graph the
                                first time a (densities, out, nrhs,
                                direction) combination is seen and replay it
                                afterwards (on the caller's stream); at most
                                8 graphs are kept per plan, least recently
                                used dropped.  Ignored while stage profiling
                                is on.  0: launch eagerly                     */
    size_t workspace_limit;  /* device bytes the plan may allocate, 0: none  */
    int32_t leaf_max;        /* adaptive octree (the remedy for uneven point
                                counts per box named in Sec. 4 and Sec. 5):
                                a box of level >= 2 holding at most leaf_max
                                points (sources and distinct targets
                                together) is a leaf and is not split; its
                                sources reach the targets of its neighbour
                                boxes directly on its own level and its
                                relevant cones get their node values
                                directly; boxes below it are no source boxes.
                                0: every leaf on level D (Sec. 3.3.1)        */
} ifgf_options;

/* Per-level counts of a plan; entry d is level d (1-based). */
typedef struct {
    int32_t D;                               /* levels                          */
    int32_t n_points;
    double H1;                               /* root box side                   */
    double x1[3];                            /* root box centre                 */
    double kappa;
    int32_t ps, pang;                        /* node counts per cone direction  */
    int32_t ns[IFGF_MAX_LEVELS + 1];         /* radial intervals n_{s,d}        */
    int32_t nc[IFGF_MAX_LEVELS + 1];         /* polar intervals n_{C,d}         */
    int64_t n_boxes[IFGF_MAX_LEVELS + 1];    /* relevant boxes |R_B^d|          */
    int64_t n_cones[IFGF_MAX_LEVELS + 1];    /* relevant cone segments |R_C^d|  */
    int64_t n_cousin_boxes[IFGF_MAX_LEVELS + 1];  /* sum over source boxes of |M B| */
    int64_t max_cousin_boxes[IFGF_MAX_LEVELS + 1];
    int64_t n_cousin_evals[IFGF_MAX_LEVELS + 1];  /* (target, cousin box) pairs */
    int64_t n_parent_evals[IFGF_MAX_LEVELS + 1];  /* (parent node, child) pairs
                                                     interpolated at level d   */
    int64_t n_leaf_pairs;                    /* (cone node, source) pairs of the
                                                leaf boxes of every level      */
    int64_t n_near_pairs;                    /* directly summed pairs           */
    int64_t n_dilated;                       /* cones marked only by dilation   */
    int64_t n_frames[IFGF_MAX_LEVELS + 1];   /* distinct child-to-parent frames
                                                tabulated for level d (0: the
                                                geometry is computed on the fly) */
    int32_t pairs_tabulated[IFGF_MAX_LEVELS + 1]; /* 1: the cousin-target geometry
                                                of level d is tabulated        */
    int64_t device_bytes;                    /* device memory held by the plan  */
    double t_plan_s;                         /* host seconds to build the plan  */
    int64_t n_sources;                       /* densities per right-hand side   */
    int64_t n_targets;                       /* outputs per right-hand side     */
    int64_t n_src_boxes[IFGF_MAX_LEVELS + 1];  /* boxes of the source tree (all
                                                relevant boxes unless adaptive) */
    int64_t n_leaf_boxes[IFGF_MAX_LEVELS + 1]; /* its leaves on level d        */
} ifgf_stats;

/* Create a plan for the points (Sec. 3.3.2: box octree, relevant boxes,
 * neighbours and cousins, cone segments per level and the relevant ones).
 *   points   host, n x 3 row-major FP64; copied, the caller keeps ownership.
 *            Points must be pairwise different (Sec. 2); two equal points
 *            give IFGF_E_INVALID_ARG.
 *   n        number of points, >= 2.
 *   k        wavenumber kappa >= 0 (0: the Laplace limit 1/(4 pi r)).
 *   levels   number of levels D >= 2, or 0: D = 1 + round(log2(4 H_1 k /
 *            (2 pi))) so that the leaf boxes are about a quarter wavelength
 *            wide (Sec. 4); for k = 0 the smallest D with at most 8 points
 *            per relevant leaf box.
 *   degrees  {P_s, P_ang}: Chebyshev nodes per cone in s and in each angle
 *            (Sec. 3.2, eq. interp_pts); NULL: {3, 5}.  Each in 1..8 (below
 *            1: IFGF_E_INVALID_ARG, above 8: IFGF_E_UNSUPPORTED).  {3,5},
 *            {4,6} and {2,3} run kernels compiled for those counts (matrix
 *            cores, pair tables); other counts run kernels that read them at
 *            run time, with the geometry computed per evaluation.
 *   opt      NULL for defaults.
 *   plan     receives the new plan.                                        */
ifgf_status ifgf_plan_create(const double* points, int64_t n, double k, int32_t levels,
                             const int32_t* degrees, const ifgf_options* opt, ifgf_plan_t* plan);

/* Create a plan with distinct sources and targets (the field of Sec. 2,
 * eq. field1, evaluated at points other than the sources).  The hierarchy is
 * built over the n + m points together, the targets carrying zero density,
 * so the result is the IFGF approximation of sum_m a(x_m) G(y, x_m) at every
 * target y.  All points (sources and targets) must be pairwise different.
 *   sources  host, n x 3 FP64 (copied); targets  host, m x 3 FP64 (copied).
 * With such a plan ifgf_apply maps densities [nrhs][n] to out [nrhs][m],
 * ifgf_apply_adjoint maps [nrhs][m] to [nrhs][n], and ifgf_grad_targets
 * takes densities [nrhs][n] and grad_out [nrhs][m] and writes grad_xyz [m][3]
 * (target coordinates).  Other arguments as for ifgf_plan_create.          */
ifgf_status ifgf_plan_create_targets(const double* sources, int64_t n, const double* targets, int64_t m, double k,
                                     int32_t levels, const int32_t* degrees, const ifgf_options* opt,
                                     ifgf_plan_t* plan);

/* out = IFGF approximation of the operator applied to the densities
 * (Algorithm 1).
 *   densities  device, [nrhs][n_sources] complex (dtype by precision); read
 *              only.
 *   nrhs       1 .. max_nrhs.
 *   out        device, [nrhs][n_targets] complex, overwritten; must not
 *              alias the densities.  (n_sources = n_targets = n unless the
 *              plan has distinct targets; ifgf_plan_stats reports both.)   */
ifgf_status ifgf_apply(ifgf_plan_t plan, const void* densities, int32_t nrhs, void* out, void* stream);

/* out = adjoint operator applied to v: the conjugate transpose of the
 * discrete operator of Sec. 2, eq. (field1),
 *   out_r(x_m) = sum_{l != m} conj(G(x_l, x_m)) v_r(x_l),
 * evaluated by the same hierarchy with the conjugated kernel (k -> -k, which
 * conjugates every factor e^{i k .} while the real interpolation weights are
 * unchanged).  The direction is an explicit argument of the pipeline, never
 * read from the sign of k (at k = 0 the windows still swap).  With distinct
 * targets v is [nrhs][n_targets] and out [nrhs][n_sources].  Otherwise the
 * same layouts and rules as ifgf_apply.                                    */
ifgf_status ifgf_apply_adjoint(ifgf_plan_t plan, const void* v, int32_t nrhs, void* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as ifgf_apply, bit for bit, computed with no allocation at all.
 * The apply's workspaces (densities and output in the plan's point order,
 * two cone-value buffers, cousin-pair values) are carved from a static
 * device array of 256 MiB that the library holds on each GPU it runs on
 * until the process ends; its address is taken when a plan is created on
 * that GPU.  Everything runs on `stream` (no second stream, no events,
 * stage timing off for the call).  The plan's own workspaces and any cone
 * values it stored are left untouched.
 *   Limit: when the workspaces of this plan and nrhs exceed the array,
 *   IFGF_E_INVALID_ARG with the byte counts in ifgf_last_error(), and
 *   nothing is launched.  (N = 6144 at 16 right-hand sides fits; a plan of
 *   393216 points does not.)
 *   Every call on one GPU, from any plan, shares that GPU's array and it
 *   keeps the last call's contents (every part is written before it is
 *   read): calls that overlap on one GPU race, so order them on one stream
 *   or synchronise between them.
 * Arguments and layouts as for ifgf_apply.                                 */
ifgf_status ifgf_apply_noalloc(ifgf_plan_t plan, const void* densities, int32_t nrhs, void* out, void* stream);

/* Gradient of a real loss L(I) with respect to the target coordinates, the
 * sources held fixed:
 *   grad_xyz[l][c] = sum_r Re( conj(g_r(x_l)) * dI_r(x_l)/dx_{l,c} ),
 * where g = dL/dRe(I) + i dL/dIm(I) (PyTorch's convention for complex
 * gradients) and dI/dx differentiates the IFGF approximation: the gradient
 * of the Helmholtz kernel of eq. (greensfunction) in the near field and, at
 * every level, of the centred factor times the Chebyshev interpolant in
 * (s, theta, phi) of Sec. 3.2 (eq. defparametrizationr).  On the polar axis
 * of a box's frame, where phi is undefined, the derivative across the axis
 * is the one-sided one into the half-plane phi = 0 that holds the axis.
 *   densities  device [nrhs][n_sources] complex, the forward input.
 *   grad_out   device [nrhs][n_targets] complex, g.
 *   nrhs       1 .. max_nrhs (passes of 16 right-hand sides are summed).
 *   grad_xyz   device [n_targets][3] FP64, overwritten.
 * The cone values are recomputed from the densities (see
 * ifgf_grad_targets_stored for reusing those of the last apply).           */
ifgf_status ifgf_grad_targets(ifgf_plan_t plan, const void* densities, const void* grad_out,
                              int32_t nrhs, double* grad_xyz, void* stream);

/* As ifgf_grad_targets, but reuses the cone values of every level that the
 * last ifgf_apply of this plan stored (store_levels), when that apply took
 * the same densities pointer and nrhs <= 16.  The caller guarantees that the
 * contents of `densities` have not changed since that apply (the autograd
 * Function of the Python binding does, through PyTorch's version check of
 * saved tensors); the plan compares only pointers and sizes.  Otherwise, or
 * when nothing is stored, the cone values are recomputed as by
 * ifgf_grad_targets.                                                        */
ifgf_status ifgf_grad_targets_stored(ifgf_plan_t plan, const void* densities, const void* grad_out,
                                     int32_t nrhs, double* grad_xyz, void* stream);

/* Per-level counts of the hierarchy (host, no GPU work). */
ifgf_status ifgf_plan_stats(ifgf_plan_t plan, ifgf_stats* out);

/* Synchronises the stream of the plan's last apply or gradient call (and the
 * plan's second stream), not the whole device, and reports how many
 * interpolation queries found no computed cone since the plan was created
 * (must be 0). */
ifgf_status ifgf_plan_check(ifgf_plan_t plan, int64_t* misses);

/* Child-to-parent kernel variants (the interpolation from child to parent
 * cone values, Sec. 3.3, Algorithm 1), for ifgf_plan_kernel_choice.  All
 * compute the same values up to FP rounding order. */
typedef enum {
    IFGF_C2P_GEOMETRY = 0,      /* per point, child-frame geometry in FP64      */
    IFGF_C2P_FRAMES = 1,        /* per point, tabulated frames                  */
    IFGF_C2P_LDS = 2,           /* frames, child cones staged in LDS            */
    IFGF_C2P_MFMA = 3,          /* batched RHS on matrix cores, per slot (FP32
                                   or FP64, 4 or 16 RHS)                      */
    IFGF_C2P_MFMA_GEOMETRY = 4, /* the same without frame tables                */
    IFGF_C2P_BOXES = 5,         /* matrix cores, boxes of one parent cone as
                                   matrix columns (FP32, 1 or 4 RHS per pass) */
    IFGF_C2P_QUADS = 6,         /* vector units, 1 RHS: each child cone value
                                   read from LDS once for up to 4 points (2 in
                                   FP64) of the same child cone               */
    IFGF_C2P_LDS_TILED = 7,     /* IFGF_C2P_LDS visiting the parent slots in
                                   box-tile order (blocks of boxes, one parent
                                   cone after the other), which shares frames
                                   in cache                                   */
    IFGF_C2P_BOX_ACC = 8,       /* matrix cores (FP32 or FP64), boxes of one
                                   parent cone as matrix columns, parent values
                                   accumulated in LDS, weights formed in
                                   registers                                  */
    IFGF_C2P_BOX_ACC_HALF = 9   /* IFGF_C2P_BOX_ACC with 8 complex columns per
                                   pass in one tile, half its LDS (1 or 4 RHS
                                   per pass)                                  */
} ifgf_c2p_variant;

/* Times every applicable child-to-parent variant at every level for nrhs
 * right-hand sides (1, 2-4 and 5-16 share a setting) and keeps the fastest
 * for later apply and gradient calls of that size.  Runs on `stream` with
 * zero densities, synchronously (returns when done); overwrites the plan's
 * workspaces, so cone values stored by an earlier apply are discarded.  Must
 * not be called while a stream capture is active.  Invalidates captured
 * graphs.  IFGF_E_INVALID_ARG for nrhs outside [1, max_nrhs]. */
ifgf_status ifgf_plan_autotune(ifgf_plan_t plan, int32_t nrhs, void* stream);

/* variant[d] (host array of IFGF_MAX_LEVELS + 1 entries) receives the
 * ifgf_c2p_variant used for the child-to-parent step from level d to d - 1
 * for nrhs right-hand sides: the tuned one, or the default rule; -1 where
 * there is no such step (d < 4, d > D, host_only plans). */
ifgf_status ifgf_plan_kernel_choice(ifgf_plan_t plan, int32_t nrhs, int32_t* variant);

/* mask[d] (host array of IFGF_MAX_LEVELS + 1 entries) receives the set of
 * ifgf_c2p_variant values (bit v) that apply to the step from level d to
 * d - 1 for nrhs right-hand sides; 0 where there is no such step. */
ifgf_status ifgf_plan_kernel_candidates(ifgf_plan_t plan, int32_t nrhs, int32_t* mask);

/* Sets the child-to-parent variant per level for nrhs right-hand sides:
 * variant[d] (host array of IFGF_MAX_LEVELS + 1 entries) >= 0 selects that
 * ifgf_c2p_variant for the step from level d to d - 1, -1 restores the
 * default rule.  IFGF_E_INVALID_ARG (and nothing changed) if a variant is
 * given for a level without such a step or does not apply there (e.g. a
 * matrix-core variant on an FP64 plan).  Invalidates captured graphs. */
ifgf_status ifgf_plan_set_kernel_choice(ifgf_plan_t plan, int32_t nrhs, const int32_t* variant);

/* Kernel stages of an apply or gradient call, for ifgf_plan_stage_times. */
typedef enum {
    IFGF_STAGE_PERMUTE_IN = 0,   /* densities to Morton order                  */
    IFGF_STAGE_NEARFIELD = 1,    /* direct sums over leaf neighbourhoods       */
    IFGF_STAGE_LEAF_NODES = 2,   /* F_k^D at the leaf cone interpolation points */
    IFGF_STAGE_COUSIN_EVAL = 3,  /* interpolation at cousin targets, per level */
    IFGF_STAGE_CHILD_TO_PARENT = 4, /* interpolation onto parent cone points   */
    IFGF_STAGE_PERMUTE_OUT = 5,  /* result back to input order                 */
    IFGF_STAGE_NEAR_GRAD = 6,    /* near-field target gradient                 */
    IFGF_STAGE_COUSIN_GRAD = 7,  /* far-field target gradient, per level       */
    IFGF_STAGE_PERMUTE_GRAD = 8, /* gradient back to input order               */
    IFGF_NUM_STAGES = 9
} ifgf_stage;

/* Stage timing with HIP events recorded around every kernel launch, on the
 * stream it runs on (the caller's or the plan's second stream).  enable = 1 starts recording (and clears the totals),
 * enable = 0 stops.  Off by default; recording adds two events per launch. */
ifgf_status ifgf_plan_profile(ifgf_plan_t plan, int32_t enable);

/* Synchronises the plan's streams, then returns per stage the summed kernel
 * milliseconds and the number of launches recorded since profiling was
 * enabled (arrays of IFGF_NUM_STAGES entries, host).  Totals keep
 * accumulating until the next ifgf_plan_profile(plan, 1). */
ifgf_status ifgf_plan_stage_times(ifgf_plan_t plan, double* ms, int64_t* launches);

/* The same totals split by level for one stage (arrays of IFGF_MAX_LEVELS +
 * 1 entries, host): entry d holds the cousin evaluation of level d, the
 * child-to-parent step from level d to d - 1, the leaf values at d = D;
 * stages without a level are reported at entry 0.  Synchronises the plan's
 * streams first. */
ifgf_status ifgf_plan_level_times(ifgf_plan_t plan, int32_t stage, double* ms, int64_t* launches);

/* Releases the plan and all memory it owns.  NULL is accepted. */
ifgf_status ifgf_plan_destroy(ifgf_plan_t plan);

const char* ifgf_status_string(ifgf_status s);
const char* ifgf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IFGF_H */
