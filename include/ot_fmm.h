/*
 * ot_fmm.h -- C ABI of the MI355X octree fast-multipole self-gravity library.
 *
 * The operation is the gravity solve of Octo-Tiger (arXiv 2412.15518): Sec. 4.3
 * ("Octo-Tiger in a Nutshell") describes an FMM gravity solver on an octree
 * whose nodes each hold an 8x8x8-cell sub-grid, and Sec. 5.5 the stencil form
 * of its same-level interactions.  The paper gives no formulas; this library
 * implements the following reading of it, with G the gravitational constant
 * and h the leaf cell width:
 *
 *   phi_i = -G sum_{j != i} m_j / |x_i - x_j|,     g_i = -grad phi at x_i,
 *   m_j = rho_j h^3 at the geometric centre of leaf cell j,
 *
 * evaluated by a Cartesian FMM of total order p = 3 with expansions about
 * geometric cell centres: P2M/M2M moment aggregation, same-level M2L over the
 * parity-aware stencil (a cell pair of level l >= 1 interacts at l when the
 * cells are farther apart than 1/theta cell widths and their parents are not;
 * the root sub-grid takes all its far pairs), exact P2P over every leaf pair
 * whose parents are near, and L2L/L2P back to the leaf centres.  Domain
 * boundaries are isolated (no mass outside the tree).
 *
 * Adaptive trees (leaves on several levels; Sec. 4.3 refines the octree where
 * the solution needs it): a leaf cell of level l is a point mass rho h_l^3 at
 * its centre.  Leaves whose sub-grids touch must lie at most one level apart
 * (2:1 balance).  The same-level rule above then holds at every level between
 * all existing cells, leaves included; a leaf near a refined cell of its
 * level meets that cell's children (leaves one level finer) by exact P2P.
 *
 * The adjoint returns d rho of  sum_i dphi_i phi_i + sum_i dg_i . g_i  through
 * the same discrete operator (its exact transpose).
 *
 * Conventions for every entry point:
 *  - Return 0 (OT_FMM_OK) on success or a negative status; the status string
 *    and ot_fmm_last_error() (a per-thread message) describe the failure.
 *    No entry point aborts or prints.
 *  - Device arrays are caller-owned FP64 device pointers, 8-byte aligned,
 *    densely packed.  A cell field (rho, phi, dphi, drho) holds
 *    N = 512 * n_leaf_nodes values: leaf k of the layout (leaves counted in
 *    node order) owns [512 k, 512 k + 512), x fastest inside the sub-grid.
 *    Vector fields (g, dg) are three such planes (x, y, z) back to back.
 *  - Work is enqueued on the given HIP stream (NULL = the default stream) with
 *    no host synchronisation; results are ready when the stream reaches them.
 *    A plan owns scratch memory and must not run on two streams at once.
 *  - Forward and adjoint allocate nothing: the plan allocates all device
 *    memory at creation.
 */
#ifndef OT_FMM_H
#define OT_FMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define OT_FMM_OK                   0
#define OT_FMM_INVALID_ARGUMENT    -1  /* null/misaligned pointer, bad flag, NaN */
#define OT_FMM_INVALID_LAYOUT      -2  /* not a proper octree (see plan_create) */
#define OT_FMM_UNSUPPORTED_ORDER   -3  /* order other than 3 */
#define OT_FMM_UNSUPPORTED_THETA   -4  /* theta outside (1/3, 1] */
#define OT_FMM_UNSUPPORTED_LAYOUT  -5  /* valid octree this build cannot run (not 2:1 balanced, depth > 6) */
#define OT_FMM_OUT_OF_MEMORY       -6  /* host or device allocation failed */
#define OT_FMM_DEVICE_ERROR        -7  /* a HIP call failed */
#define OT_FMM_NO_DEVICE_STATE     -8  /* plan created with OT_FMM_HOST_ONLY */

/* ---- plan flags -------------------------------------------------------- */
#define OT_FMM_FP64       0u         /* all arithmetic in FP64 (default) */
#define OT_FMM_HOST_ONLY  (1u << 0)  /* validate and build host tables only: no
                                        device memory; plan_info works, forward
                                        and adjoint return OT_FMM_NO_DEVICE_STATE */
#define OT_FMM_M2L_FP32   (1u << 1)  /* M2L (forward and adjoint) in FP32: moments
                                        and derivative tensors rounded to FP32, the
                                        products of each parent offset summed in
                                        FP32 and then added to FP64 accumulators;
                                        every other stage stays FP64.  The paper's
                                        runs are FP64 (its data-set table, Sec. 6.1):
                                        this is an optional lower-precision M2L whose
                                        result differs from the FP64 one by about
                                        1e-7 normwise (bounded by 1e-5 in the tests).
                                        Moments must stay inside the FP32 range. */
#define OT_FMM_AUTOTUNE   (1u << 2)  /* pick the stencil chunk count of each leaf pass
                                        (1, 2, 4 or 8 waves per block of 64 leaf
                                        parents) by timing them at plan creation;
                                        without it the count follows from the tree
                                        size (at least ~16384 waves per launch).
                                        Results of different counts agree to
                                        rounding; a plan keeps its counts, so its
                                        calls repeat bit for bit. */
#define OT_FMM_AM_CORRECTION (1u << 3) /* keep what ot_fmm_am_correction needs
                                        (full moments at every level, order-4
                                        kernel tables, per-level torque
                                        polynomials and a partial-sum buffer of
                                        at most 63 MB); uniform trees only */

typedef struct ot_fmm_plan_s *ot_fmm_plan;   /* opaque */

/* Octree of 8^3-cell sub-grids (paper Sec. 4.3).  Node 0 is the root (level 0,
 * coord (0,0,0), parent -1).  A node of level l has integer sub-grid
 * coordinates in [0, 2^l)^3; its parent has level l-1 and coordinates
 * coord >> 1; a node is either a leaf or has all 8 children.  Leaves may sit
 * on several levels (2:1 balanced).  The cell width of the deepest level L is
 * h_leaf_min; a cell of level l is 2^(L-l) times wider.  origin (the low corner of the root) shifts every position
 * alike and does not change phi or g.  The arrays are read during
 * plan_create only. */
typedef struct {
    int32_t        n_nodes;
    const int32_t *level;     /* [n_nodes] */
    const int32_t *coord;     /* [3 * n_nodes] x, y, z per node */
    const int32_t *parent;    /* [n_nodes] */
    const uint8_t *is_leaf;   /* [n_nodes] 0 or 1 */
    double         h_leaf_min;
    double         origin[3];
    double         G;
} ot_octree_layout;

typedef struct {
    int32_t depth;                 /* L, leaf level */
    int32_t order;                 /* expansion order p */
    double  theta;                 /* opening parameter; near radius 1/theta cells */
    int64_t n_nodes;
    int64_t n_leaf_nodes;
    int64_t n_leaf_cells;          /* 512 * n_leaf_nodes */
    int64_t p2p_pairs;             /* ordered leaf pairs evaluated exactly (both cells in the domain;
                                      adaptive trees: across levels too) */
    int64_t m2l_pairs;             /* ordered M2L pairs over the levels below the leaves (adaptive
                                      trees: below the deepest level, leaf cells included) */
    int64_t m2l_pairs_level[16];   /* per level 0..L-1 */
    double  flops_forward;         /* algorithmic FP64 FLOP per forward (8 per P2P pair, 168 per M2L pair, plus M2M/L2L) */
    double  flops_adjoint;         /* same for the adjoint */
    double  bytes_forward;         /* algorithmic HBM bytes per forward */
    double  bytes_adjoint;
    size_t  device_bytes;          /* device memory owned by the plan */
    int32_t leaf_chunks_forward;   /* stencil chunks (waves per leaf block) of the forward leaf pass
                                      (adaptive trees: of the deepest level's) */
    int32_t leaf_chunks_adjoint;   /* the same for the adjoint */
} ot_fmm_info;

/* Validate `layout`, build the interaction tables and allocate all device
 * scratch on the current HIP device.  theta in (1/3, 1] (0.4 gives the
 * near radius of 2.5 cells), order = 3.  On success *out owns the plan; on
 * failure *out is NULL.  Layout errors (INVALID_LAYOUT): root not node 0, a
 * parent index out of range or at the wrong level, coordinates outside the
 * level or not within the parent, duplicate nodes, an internal node without
 * all 8 children, a leaf with children.  UNSUPPORTED_LAYOUT: deeper than 6
 * levels, or an adaptive tree whose refined sub-grids miss a same-level
 * neighbour (touching leaves more than one level apart).  In adaptive trees
 * every level holding leaves has its own leaf pass, whose chunk count the size
 * rule (or OT_FMM_AUTOTUNE, per level) picks. */
int ot_fmm_plan_create(const ot_octree_layout *layout, double theta, int order,
                       uint32_t flags, ot_fmm_plan *out);

/* phi[N], g[3N] <- FMM of rho[N] (device pointers, layout order). */
int ot_fmm_forward(ot_fmm_plan plan, const double *rho, double *phi, double *g,
                   void *hip_stream);

/* Angular-momentum correction (Sec. 4.3 names it; the formula is this
 * library's reading).  The truncated M2L conserves linear momentum but not
 * angular momentum: for an M2L pair (A <- B), R = z_A - z_B, the particles'
 * torque is R x E/2 per ordered pair, E being the pair energy's derivative in
 * the expansion centre z_A (its terms of total order p + 1).  t[3N] <- the
 * spin torque per unit mass that takes it back:
 *   t_i = -1/2 sum over the M2L pairs (A <- B) of cell i's ancestors of R x e_i,
 * e_i cell i's share of E per unit mass, so that sum_i m_i (x_i x g_i + t_i)
 * = 0 exactly with g from ot_fmm_forward on the same rho; t is linear in rho.
 * Needs a plan created with OT_FMM_AM_CORRECTION (else INVALID_ARGUMENT); runs
 * its own upward pass.  FP64. */
int ot_fmm_am_correction(ot_fmm_plan plan, const double *rho, double *t, void *hip_stream);

/* drho[N] <- transpose of the forward operator applied to (dphi[N], dg[3N]). */
int ot_fmm_adjoint(ot_fmm_plan plan, const double *dphi, const double *dg,
                   double *drho, void *hip_stream);

int ot_fmm_plan_info(ot_fmm_plan plan, ot_fmm_info *info);

/* Set the stencil chunk counts (waves per block of 64 leaf parents, each
 * summing a contiguous part of the parent-offset list) of the forward and
 * adjoint leaf passes, overriding the size rule or the autotuner; each in
 * [1, 8].  Counts outside it are INVALID_ARGUMENT, a host-only plan
 * NO_DEVICE_STATE.  Calls enqueued afterwards use the new counts. */
int ot_fmm_plan_set_leaf_chunks(ot_fmm_plan plan, int forward, int adjoint);

/* Releases the plan and its device memory (the device must be idle for it).
 * NULL is a no-op. */
void ot_fmm_destroy(ot_fmm_plan plan);

const char *ot_fmm_status_string(int status);
const char *ot_fmm_last_error(void);   /* message of this thread's last failure */

/* ---- kernel timing ------------------------------------------------------
 * Between timing_begin and timing_end every forward/adjoint call records HIP
 * events on its stream around each kernel phase (at most max_calls calls are
 * recorded).  timing_end waits for the last event and reports, per phase, the
 * number of timed launches and their summed duration. */
#define OT_FMM_PHASE_UPWARD_LEAF      0   /* P2M + M2M of up to 3 levels above the leaves, forward */
#define OT_FMM_PHASE_M2M              1   /* M2M of the remaining levels, L-5..0 (none at depth <= 4) */
#define OT_FMM_PHASE_M2L              2   /* M2L, all levels, one launch */
#define OT_FMM_PHASE_L2L              3   /* M2L sums + L2L, levels 0..L-2 (level L-1: leaf phase) */
#define OT_FMM_PHASE_LEAF             4   /* leaf P2P + L2P, forward */
#define OT_FMM_PHASE_UPWARD_LEAF_ADJ  5   /* P2M of the dual sources + M2M of up to 3 levels, adjoint */
#define OT_FMM_PHASE_LEAF_ADJ         6
#define OT_FMM_PHASE_TOTAL            7   /* whole forward or adjoint call */
/* Adaptive trees: UPWARD_LEAF(_ADJ) holds the whole upward pass (leaf moments
 * and M2M level by level), M2M is empty, M2L holds its two launches (refined
 * sinks; leaf sinks next to refined cells), L2L the level-by-level L2L, and
 * LEAF(_ADJ) every level's leaf pass and coarse-fine pass. */
#define OT_FMM_NUM_PHASES             8

typedef struct {
    int32_t calls;                          /* calls recorded */
    int64_t launches[OT_FMM_NUM_PHASES];    /* kernel launches per phase */
    int64_t events[OT_FMM_NUM_PHASES];      /* timed intervals per phase */
    double  ms[OT_FMM_NUM_PHASES];          /* summed interval time per phase */
} ot_fmm_timing;

int ot_fmm_timing_begin(ot_fmm_plan plan, int max_calls);
/* Restrict the events of the calls that follow to the phases whose bit
 * (1u << phase) is set in phase_mask; timing_begin selects every phase.  Each
 * recorded phase adds two events to the stream, so timing one phase perturbs
 * the measured calls least.  Needs an active timing_begin; a mask of 0 or
 * with bits beyond OT_FMM_NUM_PHASES is INVALID_ARGUMENT. */
int ot_fmm_timing_phases(ot_fmm_plan plan, uint32_t phase_mask);
int ot_fmm_timing_end(ot_fmm_plan plan, ot_fmm_timing *out);
const char *ot_fmm_phase_name(int phase);

/* ---- batches of independent octrees ---------------------------------------
 * The paper runs many small sub-grid kernels concurrently and fuses them to
 * keep the GPU busy (Sec. 5.3, dynamic work aggregation and the executor
 * pools of its HPX/Kokkos runtime).  A batch does the same for independent
 * plans: one call enqueues the forward (or adjoint) of every plan, spread over
 * a few internal HIP streams so that small trees run side by side, and joins
 * them back into the caller's stream.  The same enqueue sequence can be
 * captured once into a HIP graph and replayed, which removes the per-launch
 * host cost of the many small kernels.
 *
 * A batch does not own its plans: they must outlive it, and no plan may run
 * elsewhere while a batch call or graph replay that uses it is in flight (a
 * plan's scratch is shared by all its calls).  Every plan lives on the same
 * device; a plan appears at most once in a batch. */
typedef struct ot_fmm_batch_s *ot_fmm_batch;   /* opaque */
typedef struct ot_fmm_graph_s *ot_fmm_graph;   /* opaque */

/* n >= 1 plans with device state; n_streams in [1, 16] internal streams (at
 * most n are used; plan i runs on stream i mod n_streams).  The streams and
 * events are created here at default priority. */
int ot_fmm_batch_create(const ot_fmm_plan *plans, int n, int n_streams, ot_fmm_batch *out);

/* Forward of every plan i: rho[i] -> phi[i], g[i] (host arrays of n device
 * pointers, each as in ot_fmm_forward).  Work is ordered after everything
 * enqueued on hip_stream before the call, and everything enqueued on it
 * afterwards waits for all n plans.  Pointers are checked before any work is
 * enqueued. */
int ot_fmm_batch_forward(ot_fmm_batch b, const double *const *rho, double *const *phi, double *const *g,
                         void *hip_stream);
/* Adjoint of every plan i: dphi[i], dg[i] -> drho[i], as in ot_fmm_adjoint. */
int ot_fmm_batch_adjoint(ot_fmm_batch b, const double *const *dphi, const double *const *dg,
                         double *const *drho, void *hip_stream);

/* Capture the batch forward (or adjoint) for these fixed device buffers into
 * an executable HIP graph.  Kernel timing must be off for every plan (no
 * timing_begin without timing_end).  The graph records the buffer addresses:
 * a replay reads and writes the same buffers. */
int ot_fmm_batch_capture_forward(ot_fmm_batch b, const double *const *rho, double *const *phi,
                                 double *const *g, ot_fmm_graph *out);
int ot_fmm_batch_capture_adjoint(ot_fmm_batch b, const double *const *dphi, const double *const *dg,
                                 double *const *drho, ot_fmm_graph *out);

/* Replay a captured graph on hip_stream (NULL = the default stream). */
int ot_fmm_graph_launch(ot_fmm_graph g, void *hip_stream);

/* Release a graph or a batch (NULL is a no-op); the device must be idle for
 * the work they enqueued. */
void ot_fmm_graph_destroy(ot_fmm_graph g);
void ot_fmm_batch_destroy(ot_fmm_batch b);

#ifdef __cplusplus
}
#endif

#endif /* OT_FMM_H */
