// ot_fmm_internal.h -- plan state and kernel launchers of the HIP FMM library.
//
// Storage (all FP64, device-resident, allocated once per plan):
//   A cell c of level l is addressed through its parent q = c >> 1 and its
//   child index b = (c_x & 1) + 2 (c_y & 1) + 4 (c_z & 1).  Every level below
//   the leaves keeps
//     Mr[l]: the M2L's reduced moments over the parent grid padded by a zero
//            halo of hp parents per side (pp = np + 2 hp, np = n_l / 2), in
//            groups of one 16-byte load: [NR/2][8][pp^3][2]; FP32 in M32[l]
//            ([NR/4][8][pp^3][4]) when the M2L runs in FP32,
//     M[l] : the full scaled moments [NC][8][pp^3], only at the levels an M2M
//            launch reads back from memory,
//     C[l] : local coefficients [NC][8][np^3]  (levels below L-1; the leaf
//            pass forms the locals of level L-1 in registers),
//   so the 64 lanes of a wave that handle 64 neighbouring parents read
//   consecutive addresses, and the stencil never needs a bounds check.
//   The leaf sources (masses, or the adjoint's cotangents) are staged in the
//   same padded form, by pairs of children: src[plane][4][ppL^3][2].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "ot_fmm.h"

namespace otfmm {

constexpr int NC = 20;                          // components of orders 0..3
constexpr int NR = 16;                          // components of the reduced M2L form (z-power <= 1)
constexpr int SUB = 8;                          // cells per sub-grid axis
constexpr int OFF_R = 7;                        // offset tables span [-7, 7]^3
constexpr int OFF_W = 2 * OFF_R + 1;
constexpr int OFF_N = OFF_W * OFF_W * OFF_W;    // 3375
constexpr int MAX_LEVELS = 8;                   // per-level arrays in the plan
// deepest supported leaf level.  The M2L forms a level's offsets in 32 bits
// (component group x child x padded parent grid: 1.5e8 at the deepest M2L
// level of depth 6, 1.1e9 at depth 7, with no margin beyond); depth 7 is
// untested and would need about 100 GB of plan memory.
constexpr int MAX_DEPTH = 6;
constexpr int WG = 256;                         // threads per workgroup (4 waves)
constexpr int LEAF_MAX_CHUNKS = 8;              // waves per leaf block (stencil chunks)

__host__ __device__ inline int off_index(int ox, int oy, int oz)
{
    return ((oz + OFF_R) * OFF_W + (oy + OFF_R)) * OFF_W + (ox + OFF_R);
}

// 64 lanes of a wave cover a block of bx*by*bz parents of an np^3 grid:
// rows along x (as long as np allows), or, with subgrid, the 4x4x4 parents of
// one sub-grid (sparse levels of adaptive trees, where rows would hold cells
// of sub-grids that do not exist)
struct Block { int bx, by, bz; };
__host__ __device__ inline Block block_shape(int np, int subgrid = 0)
{
    Block b;
    if (subgrid) {
        b.bx = b.by = b.bz = 4;
        return b;
    }
    b.bx = np < 64 ? np : 64;
    b.by = np < 64 / b.bx ? np : 64 / b.bx;
    b.bz = 64 / (b.bx * b.by);
    return b;
}

struct DevLevel {
    int np;          // parents per axis (n_l / 2)
    int hp;          // halo of the moment array, in parents
    int pp;          // np + 2 hp
    int maxp;        // partial-sum pieces of the M2L per block (see M2LDesc)
    int bx, by, bz;  // M2L block shape (64 parents)
    int nbx, nby;    // blocks per axis in x and y
    double h;        // cell width of this level
    double *M;       // [NC][8][pp^3] full moments; null unless an M2M reads this level from memory
    double *Mr;      // [NR/2][8][pp^3][2] reduced moments, M2L sources (FP64 M2L; else null)
    float *M32;      // [NR/4][8][pp^3][4] the same in FP32 (FP32 M2L; else null)
    double *C;       // [NC][8][np^3] local coefficients (final); null at level L-1
    double *Cp;      // [maxp][NC][8][np^3] M2L partial sums
    double *Mr_ref;          // adaptive trees: the reduced moments of refined cells alone (leaf cells zero),
    float *M32_ref;          //   the sources of the leaf-sink M2L (FP64 or FP32 M2L); else null
    const int32_t *ulist;    // the M2L units computed (a source in the domain and, in an adaptive tree,
                             //   a sink in an existing sub-grid), ascending, as block << 9 | offset
};

// M2L work: a block = 64 sink parents of one level (bx*by*bz parents, lane =
// parent, blocks numbered z-major); a unit = one block and one parent offset
// P of the level's list (the near list, or the whole cube at the root).  The
// units of each level are cut into equal runs, one per resident workgroup,
// and no run crosses a level.  A run [ubeg, uend) (level-local unit indices)
// starts inside block ubeg / nP; a block split over k runs gets k partial
// sums, pieces 0..k-1 of the level's Cp: the run holding the block's first
// unit writes piece 0, the next run piece 1, and so on.  Consumers add the
// pieces in a fixed order, so the result does not depend on timing.
// A unit whose 64 sources all lie outside the domain (in the zero halo)
// contributes nothing: the runs skip it, and are cut at equal counts of the
// other units.  A piece whose run skips all of its block's units stays zero.
struct M2LDesc {
    int level;
    int ubeg, uend;
    int piece0;      // piece of the run's first (possibly partial) block
    int nvalid;      // units of [ubeg, uend) with a source in the domain (the only ones computed)
    int vbeg;        // the first of them in the level's unit list
};

struct DevPlan {
    int L;               // leaf level
    int r2i;             // largest integer k with k <= (1/theta)^2: far iff |o|^2 > r2i
    double hleaf, G, h3;
    int npL, hpL, ppL;   // leaf parents per axis, their halo, padded width
    int sL;              // leaf sub-grids per axis (2^L)
    int64_t n_leaf_cells;
    const int32_t *leaf_slot;   // [sL^3] leaf index in layout order
    double *src;                // [4][4][ppL^3][2]: plane, child pair, padded parent
    const double *Ktab;         // [OFF_N][4]: K0, K1x, K1y, K1z of a leaf pair
    const double *Kst;          // [n_plist_leaf][27][4]: Ktab rows of 2P + e, e in {-1,0,1}^3
    const double *Ksa;          // [4][n_plist_leaf][27]: the same rows plane by plane for the
                                //   adjoint leaf pass: K0, then -K1x, -K1y, -K1z
    const double *Dtab;         // [L][OFF_N][NC]: derivative tensor of -G/r per level
    const float *Dtab32;        // the same in FP32 (FP32 M2L only)
    int m2l_fp32;               // 1: the M2L runs in FP32 with FP64 accumulation
    const char4 *plist_leaf; int n_plist_leaf;   // parent offsets of the leaf P2P
    const char4 *plist_near; int n_plist_near;   // |P| <= 1/theta (levels >= 1)
    const char4 *plist_cube; int n_plist_cube;   // [-3,3]^3 (root level)
    const M2LDesc *mdesc; int n_mdesc;          // one per M2L workgroup
    int n_span; int span_top[MAX_LEVELS], span_n[MAX_LEVELS];   // tree passes over levels 0..L-2
    double e_leaf[NC];   // e_a(h/2, h/2, h/2): L2P shift magnitudes, leaf cell from its parent
    int leaf_chunks[2];  // stencil chunks (waves per block) of the forward and adjoint leaf passes
    // Adaptive trees (leaves on several levels).  The plan keeps one copy of
    // this struct per level that holds leaves (a "view": L is that level and
    // the leaf fields above describe its leaves); the level arrays lev[] are
    // shared.  Uniform trees leave all of these null / 0.
    const double *own_Cp; int own_maxp;  // the leaf-sink M2L's pieces of this level (null if none)
    const uint16_t *own_np;              // pieces per M2L block of this level (0: no unit computed)
    int own_subgrid_blocks;              // those M2L blocks are sub-grids (1) or rows (0)
    const int32_t *blist; int nblist;   // blocks of the leaf pass holding a leaf sub-grid of this level
    const uint8_t *ntype_L;             // kinds of this level's sub-grids (0 none, 1 leaf, 2 refined)
    int leaf_subgrid_blocks;            // blocks of the leaf pass are sub-grids (block_shape)
    const double *src_up, *src_dn;      // source planes of levels L-1 and L+1 (null without leaves there)
    int hp_up, pp_up, hp_dn, pp_dn;
    const double *Kcf_up;        // [n_plist_near][8][4]: kernel rows, child c of a parent to a leaf of level L-1
    const double *Kcf_dn;        // [7^3][8][4]: kernel rows, cell of level L to child c' of the level-L cell
                                 //   at offset o in [-3, 3]^3 (zero rows where o = 0 or |o|^2 > r2i)
    DevLevel lev[MAX_LEVELS];
};

struct TimingState {
    bool active = false;
    int max_calls = 0;
    int calls = 0;
    uint32_t mask = ~0u;               // phases that record events
    std::vector<hipEvent_t> pool;      // pre-created events
    size_t next = 0;
    struct Rec { int phase; int launches; hipEvent_t a, b; };
    std::vector<Rec> recs;
};

}  // namespace otfmm

struct ot_fmm_plan_s {
    int L = 0;
    int order = 3;
    double theta = 0.4;
    double r2 = 6.25;
    uint32_t flags = 0;
    double h = 1.0, G = 1.0;
    int64_t n_nodes = 0, n_leaf_nodes = 0;
    int device = -1;
    bool has_device = false;

    // host tables
    std::vector<int32_t> leaf_slot;
    std::vector<char4> plist_near, plist_cube;
    std::vector<otfmm::M2LDesc> mdesc;
    // adaptive trees
    bool amr = false;
    std::vector<uint8_t> ntype[otfmm::MAX_LEVELS];     // per level and sub-grid: 0 none, 1 leaf, 2 refined
    std::vector<int32_t> lslot[otfmm::MAX_LEVELS];     // per level and sub-grid: leaf index, or -1
    std::vector<int32_t> lnodes[otfmm::MAX_LEVELS];    // leaf sub-grids per level, packed x | y << 10 | z << 20
    std::vector<int32_t> rnodes[otfmm::MAX_LEVELS];    // refined sub-grids per level, packed alike
    std::vector<int32_t> lblk[otfmm::MAX_LEVELS];      // leaf-pass blocks per level
    int lsub[otfmm::MAX_LEVELS] = {};                  // 1: those blocks are sub-grids, 0: rows
    std::vector<double> Kst_l[otfmm::MAX_LEVELS], Ksa_l[otfmm::MAX_LEVELS];
    std::vector<double> Kup_l[otfmm::MAX_LEVELS], Kdn_l[otfmm::MAX_LEVELS];
    otfmm::DevPlan view[otfmm::MAX_LEVELS];            // per level holding leaves
    // the leaf-sink M2L of an adaptive tree: a copy of the plan whose levels
    // read Mr_ref, with its own units, runs and pieces
    otfmm::DevPlan m2l_leaf{};
    bool has_m2l_leaf = false;
    // angular-momentum correction (plan flag OT_FMM_AM_CORRECTION, uniform trees)
    std::vector<double> KX;                            // [L][OFF_N][10][3]
    const double *dev_KX = nullptr;
    double *Pi[otfmm::MAX_LEVELS] = {};                // [3 * NC][8][np^3] per level
    int am_tiled = 0;                                  // the device gives a workgroup 2 AM_TILE_LDS (2), AM_TILE_LDS (1) of LDS
    double *Pi_part = nullptr;                         // partial Pi of the levels whose offsets are split
    const int32_t *dev_lnodes[otfmm::MAX_LEVELS] = {}, *dev_rnodes[otfmm::MAX_LEVELS] = {};
    const uint8_t *dev_ntype[otfmm::MAX_LEVELS] = {};
    std::vector<int32_t> ulist[otfmm::MAX_LEVELS];    // M2L units computed, per level
    std::vector<double> Ktab, Kst, Ksa, Dtab;
    std::vector<float> Dtab32;
    ot_fmm_info info{};

    // device state
    otfmm::DevPlan dp{};
    std::vector<void *> allocations;
    otfmm::TimingState timing;
};

namespace otfmm {

// kernel launchers (ot_fmm_kernels.hip); each returns hipGetLastError()
// P2M into level L-1 fused with the bottom M2M span (or plain P2M at depth <= 1)
hipError_t launch_upward_leaf(const DevPlan &p, const double *rho, hipStream_t s);
hipError_t launch_upward_leaf_adj(const DevPlan &p, const double *w, const double *u, hipStream_t s);
hipError_t launch_m2m_upper(const DevPlan &p, hipStream_t s);      // the M2M spans above the bottom one
hipError_t launch_m2l(const DevPlan &p, hipStream_t s);
hipError_t m2l_blocks_per_cu(int fp32, int *n);   // resident M2L workgroups per CU
hipError_t launch_l2l_span(const DevPlan &p, int span, hipStream_t s);
hipError_t launch_leaf(const DevPlan &p, double *phi, double *g, hipStream_t s);
hipError_t launch_leaf_adj(const DevPlan &p, double *drho, hipStream_t s);
// either leaf pass with an explicit chunk count (1 .. LEAF_MAX_CHUNKS)
hipError_t launch_leaf_chunks(const DevPlan &p, int adj, int nchunk, double *out0, double *out1, hipStream_t s);
// adaptive trees: v is the view of the level named in each comment
//   moments of the n leaf sub-grids of level v.L (M2L sources)
hipError_t launch_amr_leaf_moments(const DevPlan &v, int adj, const int32_t *nodes, int n, const double *a0,
                                   const double *a1, hipStream_t s);
//   moments of the n refined sub-grids of level l (v: view of level l + 1, or
//   any plan whose lev[] is the tree's when level l + 1 holds no leaves)
hipError_t launch_amr_m2m(const DevPlan &v, int adj, int l, const int32_t *nodes, int n, const uint8_t *child_type,
                          const double *a0, const double *a1, hipStream_t s);
// angular-momentum correction of a uniform plan whose levels keep full
// moments (after its upward pass): Pi per level (Pi_host: the device pointers
// of levels 0..L-1), each level's then gaining its parent's, then t[3N]
// (Pi_part: am_split_size(p.L) doubles, used where tiled)
hipError_t launch_am_correction(const DevPlan &p, const double *KX, double *const *Pi_host, double *Pi_part,
                                double *t, int tiled, hipStream_t s);
// LDS bytes of one staging buffer of the tiled Pi kernel (tiled = 1 needs this
// much per workgroup, tiled = 2 twice as much)
constexpr size_t AM_TILE_LDS = (size_t)8 * NC * 64 * sizeof(double);
// The tiled Pi kernel splits the parent offsets of level l into this many
// parts, one workgroup each, where the level's 64-parent blocks alone would
// leave most of the GPU idle (1 block at level 0, 8 at level 1, 64 at level
// 2); the parts' sums are added in part order by a second kernel, whose
// chain of adds caps the parts at 64.
inline int am_split(int l)
{
    const long nblk = (long)(4 << l) * (4 << l) * (4 << l) / 64;
    if (nblk >= 256) return 1;
    return 256 / nblk > 64 ? 64 : (int)(256 / nblk);
}
// doubles of the partial-sum buffer: the largest level that splits
inline size_t am_split_size(int L)
{
    size_t m = 0;
    for (int l = 0; l < L; ++l)
        if (am_split(l) > 1) {
            const size_t np3 = (size_t)(4 << l) * (4 << l) * (4 << l);
            const size_t n = (size_t)am_split(l) * 3 * NC * 8 * np3;
            m = n > m ? n : m;
        }
    return m;
}
//   final local expansions of the n refined sub-grids of level l (p: the plan)
hipError_t launch_amr_l2l(const DevPlan &p, int l, const int32_t *nodes, int n, hipStream_t s);
//   for the leaves of level v.L: their own level's M2L part (below the finest
//   level) and their P2P pairs with leaves one level up or down
hipError_t launch_amr_cf(const DevPlan &v, int adj, double *out0, double *out1, hipStream_t s);

}  // namespace otfmm
