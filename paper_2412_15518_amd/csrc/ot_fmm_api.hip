// ot_fmm_api.hip -- C ABI, plan construction and call orchestration.
//
// plan_create validates the octree, builds the per-level interaction tables
// (parent-offset lists, the derivative tensors of K = -G/r per stencil offset,
// the leaf pair kernel K0/K1) and allocates every device buffer once, so that
// forward and adjoint only enqueue kernels.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_set>
#include <vector>

#include "ot_fmm_internal.h"

using namespace otfmm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(OT_FMM_DEVICE_ERROR, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// derivative tensor of K(r) = -G/|r| at R = (x, y, z), orders 0..3, in the
// kernels' component order (0; x y z; xx xy xz yy yz zz; xxx xxy xxz xyy xyz
// xzz yyy yyz yzz zzz), from the closed forms
//   d_i (1/r)         = -x_i / r^3
//   d_i d_j (1/r)     = 3 x_i x_j / r^5 - delta_ij / r^3
//   d_i d_j d_k (1/r) = -15 x_i x_j x_k / r^7
//                       + 3 (delta_ij x_k + delta_ik x_j + delta_jk x_i) / r^5
// ---------------------------------------------------------------------------
void derivative_tensor(double G, double x, double y, double z, double *D)
{
    const double X[3] = {x, y, z};
    const double r = std::sqrt(x * x + y * y + z * z);
    const double ir = 1.0 / r, ir2 = ir * ir, ir3 = ir * ir2, ir5 = ir3 * ir2, ir7 = ir5 * ir2;
    auto dl = [](int i, int j) { return i == j ? 1.0 : 0.0; };
    D[0] = -G * ir;
    for (int i = 0; i < 3; ++i) D[1 + i] = G * X[i] * ir3;
    static const int two[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    for (int c = 0; c < 6; ++c) {
        const int i = two[c][0], j = two[c][1];
        D[4 + c] = -G * (3.0 * X[i] * X[j] * ir5 - dl(i, j) * ir3);
    }
    static const int three[10][3] = {{0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 1, 1}, {0, 1, 2},
                                     {0, 2, 2}, {1, 1, 1}, {1, 1, 2}, {1, 2, 2}, {2, 2, 2}};
    for (int c = 0; c < 10; ++c) {
        const int i = three[c][0], j = three[c][1], k = three[c][2];
        const double t = -15.0 * X[i] * X[j] * X[k] * ir7 +
                         3.0 * (dl(i, j) * X[k] + dl(i, k) * X[j] + dl(j, k) * X[i]) * ir5;
        D[10 + c] = -G * t;
    }
}

// cells c in [0, n) with c = b (mod 2) whose partner c + o is in [0, n)
int64_t axis_count(int n, int b, int o)
{
    int64_t cnt = 0;
    for (int c = b; c < n; c += 2)
        if (c + o >= 0 && c + o < n) ++cnt;
    return cnt;
}

struct Key {
    int l, x, y, z;
    bool operator==(const Key &o) const { return l == o.l && x == o.x && y == o.y && z == o.z; }
};
struct KeyHash {
    size_t operator()(const Key &k) const
    {
        uint64_t h = (uint64_t)(uint32_t)k.l * 0x9E3779B97F4A7C15ull;
        h ^= (uint64_t)(uint32_t)k.x + 0x7F4A7C15ull + (h << 6) + (h >> 2);
        h ^= (uint64_t)(uint32_t)k.y + 0x9E3779B9ull + (h << 6) + (h >> 2);
        h ^= (uint64_t)(uint32_t)k.z + 0x85EBCA6Bull + (h << 6) + (h >> 2);
        return (size_t)h;
    }
};

int validate_layout(const ot_octree_layout *lay, ot_fmm_plan P)
{
    if (!lay) return fail(OT_FMM_INVALID_ARGUMENT, "layout is NULL");
    const int64_t n = lay->n_nodes;
    if (n < 1) return fail(OT_FMM_INVALID_LAYOUT, "layout has no nodes");
    if (!lay->level || !lay->coord || !lay->parent || !lay->is_leaf)
        return fail(OT_FMM_INVALID_ARGUMENT, "layout array pointer is NULL");
    if (!(lay->h_leaf_min > 0.0) || !std::isfinite(lay->h_leaf_min))
        return fail(OT_FMM_INVALID_ARGUMENT, "h_leaf_min must be finite and > 0");
    if (!std::isfinite(lay->G)) return fail(OT_FMM_INVALID_ARGUMENT, "G must be finite");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(lay->origin[k])) return fail(OT_FMM_INVALID_ARGUMENT, "origin must be finite");
    if (lay->level[0] != 0 || lay->parent[0] != -1 || lay->coord[0] || lay->coord[1] || lay->coord[2])
        return fail(OT_FMM_INVALID_LAYOUT, "node 0 must be the root: level 0, parent -1, coord (0,0,0)");

    std::vector<int> nchild((size_t)n, 0);
    std::unordered_set<Key, KeyHash> seen;
    seen.reserve((size_t)n * 2);
    int L = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int l = lay->level[i];
        const int x = lay->coord[3 * i], y = lay->coord[3 * i + 1], z = lay->coord[3 * i + 2];
        char buf[160];
        if (l < 0 || l > 30) {
            snprintf(buf, sizeof buf, "node %lld: level %d out of range", (long long)i, l);
            return fail(OT_FMM_INVALID_LAYOUT, buf);
        }
        const int m = 1 << l;
        if (x < 0 || y < 0 || z < 0 || x >= m || y >= m || z >= m) {
            snprintf(buf, sizeof buf, "node %lld: coordinates (%d,%d,%d) outside level %d", (long long)i, x, y, z, l);
            return fail(OT_FMM_INVALID_LAYOUT, buf);
        }
        if (lay->is_leaf[i] > 1) {
            snprintf(buf, sizeof buf, "node %lld: is_leaf must be 0 or 1", (long long)i);
            return fail(OT_FMM_INVALID_LAYOUT, buf);
        }
        if (i > 0) {
            const int64_t pa = lay->parent[i];
            if (pa < 0 || pa >= n || pa == i) {
                snprintf(buf, sizeof buf, "node %lld: parent %lld out of range", (long long)i, (long long)pa);
                return fail(OT_FMM_INVALID_LAYOUT, buf);
            }
            if (lay->level[pa] != l - 1) {
                snprintf(buf, sizeof buf, "node %lld: parent %lld is not one level up", (long long)i, (long long)pa);
                return fail(OT_FMM_INVALID_LAYOUT, buf);
            }
            if (lay->coord[3 * pa] != (x >> 1) || lay->coord[3 * pa + 1] != (y >> 1) ||
                lay->coord[3 * pa + 2] != (z >> 1)) {
                snprintf(buf, sizeof buf, "node %lld: coordinates not inside parent %lld", (long long)i, (long long)pa);
                return fail(OT_FMM_INVALID_LAYOUT, buf);
            }
            nchild[(size_t)pa] += 1;
        }
        if (!seen.insert(Key{l, x, y, z}).second) {
            snprintf(buf, sizeof buf, "node %lld: duplicate of an earlier node (level %d, %d,%d,%d)",
                     (long long)i, l, x, y, z);
            return fail(OT_FMM_INVALID_LAYOUT, buf);
        }
        L = std::max(L, l);
    }
    int64_t nleaf = 0;
    for (int64_t i = 0; i < n; ++i) {
        char buf[128];
        if (lay->is_leaf[i]) {
            if (nchild[(size_t)i] != 0) {
                snprintf(buf, sizeof buf, "node %lld: leaf with children", (long long)i);
                return fail(OT_FMM_INVALID_LAYOUT, buf);
            }
            ++nleaf;
        } else if (nchild[(size_t)i] != 8) {
            snprintf(buf, sizeof buf, "node %lld: internal node with %d of 8 children", (long long)i, nchild[(size_t)i]);
            return fail(OT_FMM_INVALID_LAYOUT, buf);
        }
    }
    if (L > MAX_DEPTH)
        return fail(OT_FMM_UNSUPPORTED_LAYOUT, "octree deeper than 6 levels (more than 512^3 leaf cells)");
    bool amr = false;
    for (int64_t i = 0; i < n; ++i) amr = amr || (lay->is_leaf[i] && lay->level[i] != L);
    P->L = L;
    P->n_nodes = n;
    P->n_leaf_nodes = nleaf;
    P->h = lay->h_leaf_min;
    P->G = lay->G;
    if (amr) {
        // Leaves on several levels.  Per level: the sub-grids' kinds and leaf
        // indices; then 2:1 balance: the 26 sub-grids around every refined
        // one exist (so leaves that touch lie at most one level apart)
        P->amr = true;
        for (int l = 0; l <= L; ++l) {
            const size_t m = (size_t)1 << l;
            P->ntype[l].assign(m * m * m, 0);
            P->lslot[l].assign(m * m * m, -1);
        }
        int64_t k = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int l = lay->level[i];
            const int x = lay->coord[3 * i], y = lay->coord[3 * i + 1], z = lay->coord[3 * i + 2];
            const size_t m = (size_t)1 << l, at = ((size_t)z * m + y) * m + x;
            const int32_t packed = x | (y << 10) | (z << 20);
            P->ntype[l][at] = lay->is_leaf[i] ? 1 : 2;
            if (lay->is_leaf[i]) {
                P->lslot[l][at] = (int32_t)k++;
                P->lnodes[l].push_back(packed);
            } else {
                P->rnodes[l].push_back(packed);
            }
        }
        for (int l = 1; l < L; ++l) {
            const int m = 1 << l;
            for (int32_t pk : P->rnodes[l]) {
                const int x = pk & 1023, y = (pk >> 10) & 1023, z = (pk >> 20) & 1023;
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int qx = x + dx, qy = y + dy, qz = z + dz;
                            if (qx < 0 || qy < 0 || qz < 0 || qx >= m || qy >= m || qz >= m) continue;
                            if (P->ntype[l][((size_t)qz * m + qy) * m + qx] == 0) {
                                char buf[200];
                                snprintf(buf, sizeof buf,
                                         "octree is not 2:1 balanced: refined sub-grid (%d,%d,%d) of level %d has no "
                                         "neighbour at (%d,%d,%d)",
                                         x, y, z, l, qx, qy, qz);
                                return fail(OT_FMM_UNSUPPORTED_LAYOUT, buf);
                            }
                        }
            }
        }
        return OT_FMM_OK;
    }

    // a valid octree whose leaves all sit at level L is the full tree of depth L
    const int sL = 1 << L;
    P->leaf_slot.assign((size_t)sL * sL * sL, -1);
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!lay->is_leaf[i]) continue;
        const int x = lay->coord[3 * i], y = lay->coord[3 * i + 1], z = lay->coord[3 * i + 2];
        P->leaf_slot[((size_t)z * sL + y) * sL + x] = (int32_t)k++;
    }
    return OT_FMM_OK;
}

// shift magnitudes e_a(x, x, x) of the leaf L2P (x = h/2); the sign of a
// component follows the child's octant
void shift_mags(double x, double *e)
{
    const double x2 = 0.5 * x * x;
    const double v[NC] = {1.0, x, x, x, x2, x * x, x * x, x2, x * x, x2,
                          x2 * x / 3.0, x2 * x, x2 * x, x * x2, x * x * x, x * x2,
                          x2 * x / 3.0, x2 * x, x * x2, x2 * x / 3.0};
    for (int k = 0; k < NC; ++k) e[k] = v[k];
}

// The leaf pass reads, per parent offset P of its list, the 27 kernel rows
// of the offsets 2P + e (Kst: K0, K1x, K1y, K1z per row).  The adjoint pass
// streams one source plane at a time: rows of K0, then of -K1x, -K1y, -K1z
// (the transpose flips the sign of the odd part).  The rows of Ktab (cell
// width h) are scaled by s0 (K0) and s1 (K1) for another cell width; with
// near_only, rows of far offsets (|o|^2 > r2i) are zero.
void leaf_tables(const std::vector<double> &Ktab, const std::vector<char4> &pl, double s0, double s1, int r2i,
                 bool near_only, std::vector<double> &Kst, std::vector<double> &Ksa)
{
    const size_t nP = pl.size();
    Kst.assign(nP * 27 * 4, 0.0);
    for (size_t i = 0; i < nP; ++i)
        for (int e = 0; e < 27; ++e) {
            const int ox = 2 * pl[i].x + e % 3 - 1, oy = 2 * pl[i].y + (e / 3) % 3 - 1, oz = 2 * pl[i].z + e / 9 - 1;
            if (near_only && ox * ox + oy * oy + oz * oz > r2i) continue;
            for (int j = 0; j < 4; ++j)
                Kst[(i * 27 + e) * 4 + j] = (j == 0 ? s0 : s1) * Ktab[(size_t)off_index(ox, oy, oz) * 4 + j];
        }
    Ksa.assign(4 * nP * 27, 0.0);
    for (int j = 0; j < 4; ++j)
        for (size_t i = 0; i < nP; ++i)
            for (int e = 0; e < 27; ++e)
                Ksa[((size_t)j * nP + i) * 27 + e] = (j == 0 ? 1.0 : -1.0) * Kst[(i * 27 + e) * 4 + j];
}

// Coarse-fine kernel row (K0, K1x, K1y, K1z) for the source offset
// D = (2 o + sgn (c - 1/2)) h per axis, D = source - sink, c a child index
void cf_row(const int o[3], int c, int sgn, double h, double G, double *row)
{
    double D[3];
    for (int k = 0; k < 3; ++k) D[k] = (2.0 * o[k] + sgn * (((c >> k) & 1) - 0.5)) * h;
    const double r = std::sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    row[0] = -G / r;
    for (int k = 0; k < 3; ++k) row[1 + k] = G * D[k] / (r * r * r);
}

// up: [near offset][child c][4], sink = child c of parent Q, source = cell
// Q + o one level up (sgn = -1)
void cf_table(const std::vector<char4> &pl, double h, double G, int sgn, std::vector<double> &K)
{
    K.assign(pl.size() * 8 * 4, 0.0);
    for (size_t i = 0; i < pl.size(); ++i) {
        if (!pl[i].x && !pl[i].y && !pl[i].z) continue;
        const int o[3] = {pl[i].x, pl[i].y, pl[i].z};
        for (int c = 0; c < 8; ++c) cf_row(o, c, sgn, h, G, &K[(i * 8 + c) * 4]);
    }
}

// down: [o in [-3, 3]^3][child c][4], sink = a cell B, source = child c of
// the cell B + o one level down (sgn = +1); zero unless 0 < |o|^2 <= r2i
void cf_table_down(int r2i, double h, double G, std::vector<double> &K)
{
    K.assign(343 * 8 * 4, 0.0);
    for (int i = 0; i < 343; ++i) {
        const int o[3] = {i % 7 - 3, (i / 7) % 7 - 3, i / 49 - 3};
        const int o2 = o[0] * o[0] + o[1] * o[1] + o[2] * o[2];
        if (o2 == 0 || o2 > r2i) continue;
        for (int c = 0; c < 8; ++c) cf_row(o, c, +1, h, G, &K[((size_t)i * 8 + c) * 4]);
    }
}

// Block shape of an adaptive tree's level l (np = 4 << l parents per axis,
// the grid of its M2L and of its leaf pass): one sub-grid per block from 16
// parents per axis on (levels 2 and deeper), so that a block's sinks are all
// leaves or all refined cells of one sub-grid; rows at levels 0 and 1
Block amr_block(int l) { return block_shape(4 << l, (4 << l) >= 16); }

// Angular-momentum correction table, per level l < L and offset o (source
// minus sink, R = -o h_l): KX[c][j] = -1/2 (R x K^(c+e))_j for the 10
// order-3 components c, K = -G/r, from the closed form of the fourth
// derivatives of 1/r:
//   d_ijkl (1/r) = 105 x_i x_j x_k x_l / r^9
//                  - 15 (d_ij x_k x_l + 5 more pairings) / r^7 + 3 (d_ij d_kl + 2 more) / r^5
void am_table(ot_fmm_plan P)
{
    const int L = P->L;
    static const int three[10][3] = {{0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 1, 1}, {0, 1, 2},
                                     {0, 2, 2}, {1, 1, 1}, {1, 1, 2}, {1, 2, 2}, {2, 2, 2}};
    auto dl = [](int i, int j) { return i == j ? 1.0 : 0.0; };
    P->KX.assign((size_t)std::max(L, 1) * OFF_N * 30, 0.0);
    for (int l = 0; l < L; ++l) {
        const double hl = P->h * (double)(1 << (L - l));
        for (int oz = -OFF_R; oz <= OFF_R; ++oz)
            for (int oy = -OFF_R; oy <= OFF_R; ++oy)
                for (int ox = -OFF_R; ox <= OFF_R; ++ox) {
                    if (!ox && !oy && !oz) continue;
                    const double X[3] = {-ox * hl, -oy * hl, -oz * hl};
                    const double r2 = X[0] * X[0] + X[1] * X[1] + X[2] * X[2], r = std::sqrt(r2);
                    const double i5 = 1.0 / (r2 * r2 * r), i7 = i5 / r2, i9 = i7 / r2;
                    auto K4 = [&](int i, int j, int k, int m) {
                        const double t = 105.0 * X[i] * X[j] * X[k] * X[m] * i9 -
                                         15.0 * (dl(i, j) * X[k] * X[m] + dl(i, k) * X[j] * X[m] +
                                                 dl(i, m) * X[j] * X[k] + dl(j, k) * X[i] * X[m] +
                                                 dl(j, m) * X[i] * X[k] + dl(k, m) * X[i] * X[j]) * i7 +
                                         3.0 * (dl(i, j) * dl(k, m) + dl(i, k) * dl(j, m) + dl(i, m) * dl(j, k)) * i5;
                        return -P->G * t;
                    };
                    double *row = &P->KX[((size_t)l * OFF_N + off_index(ox, oy, oz)) * 30];
                    for (int c = 0; c < 10; ++c) {
                        const int i = three[c][0], j = three[c][1], k = three[c][2];
                        double Ke[3];
                        for (int e = 0; e < 3; ++e) Ke[e] = K4(i, j, k, e);
                        row[3 * c + 0] = -0.5 * (X[1] * Ke[2] - X[2] * Ke[1]);
                        row[3 * c + 1] = -0.5 * (X[2] * Ke[0] - X[0] * Ke[2]);
                        row[3 * c + 2] = -0.5 * (X[0] * Ke[1] - X[1] * Ke[0]);
                    }
                }
    }
}

// Blocks (64 parents of shape bs) of level l that hold a parent of a listed
// sub-grid's cells
std::vector<int32_t> blocks_of(int l, const std::vector<int32_t> &nodes, Block bs)
{
    const int np = 4 << l;
    const int bx = bs.bx, by = bs.by, bz = bs.bz;
    const int nbx = np / bx, nby = np / by;
    std::vector<int32_t> out;
    for (int32_t pk : nodes) {
        const int x = pk & 1023, y = (pk >> 10) & 1023, z = (pk >> 20) & 1023;
        for (int qz = 4 * z; qz < 4 * z + 4; ++qz)
            for (int qy = 4 * y; qy < 4 * y + 4; ++qy)
                for (int qx = 4 * x; qx < 4 * x + 4; ++qx)
                    out.push_back(((qz / bz) * nby + qy / by) * nbx + qx / bx);
    }
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
    return out;
}

// per level holding leaves of an adaptive tree: blocks and kernel tables
void build_amr_tables(ot_fmm_plan P)
{
    const int L = P->L, r2i = P->dp.r2i;
    for (int l = 1; l <= L; ++l) {
        P->lblk[l].clear();
        if (P->lnodes[l].empty()) continue;
        // the leaf pass's blocks (64 parents each): rows where at least 3/4 of
        // the rows' parents lie in leaf sub-grids of this level (rows load
        // contiguously), else one sub-grid per block
        P->lsub[l] = 0;
        P->lblk[l] = blocks_of(l, P->lnodes[l], block_shape(4 << l));
        if ((int64_t)P->lnodes[l].size() * 4 < (int64_t)P->lblk[l].size() * 3) {
            P->lsub[l] = 1;
            P->lblk[l] = blocks_of(l, P->lnodes[l], block_shape(4 << l, 1));
        }
        const double hl = P->h * (double)(1 << (L - l)), r = P->h / hl;
        leaf_tables(P->Ktab, P->plist_near, r, r * r, r2i, false, P->Kst_l[l], P->Ksa_l[l]);
        P->Kup_l[l].clear();
        P->Kdn_l[l].clear();
        if (!P->lnodes[l - 1].empty()) cf_table(P->plist_near, hl, P->G, -1, P->Kup_l[l]);
        if (l < L && !P->lnodes[l + 1].empty()) cf_table_down(r2i, 0.5 * hl, P->G, P->Kdn_l[l]);
    }
}

void build_tables(ot_fmm_plan P)
{
    const int L = P->L;
    const double r2 = P->r2;
    // integer r2i: |o|^2 > r2i  <=>  (double)|o|^2 > r2
    int r2i = 0;
    while ((double)(r2i + 1) <= r2) ++r2i;
    P->dp.r2i = r2i;

    P->plist_near.clear();
    P->plist_cube.clear();
    for (int z = -3; z <= 3; ++z)
        for (int y = -3; y <= 3; ++y)
            for (int x = -3; x <= 3; ++x) {
                char4 c;
                c.x = (signed char)x; c.y = (signed char)y; c.z = (signed char)z; c.w = 0;
                P->plist_cube.push_back(c);
                if (x * x + y * y + z * z <= r2i) P->plist_near.push_back(c);
            }

    // leaf pair kernel, source offset o = c_source - c_sink:
    //   phi += K0 m, g += K1 m with K0 = -G/(h|o|), K1 = G o / (h^2 |o|^3)
    const double h = P->h, G = P->G;
    P->Ktab.assign((size_t)OFF_N * 4, 0.0);
    for (int z = -OFF_R; z <= OFF_R; ++z)
        for (int y = -OFF_R; y <= OFF_R; ++y)
            for (int x = -OFF_R; x <= OFF_R; ++x) {
                if (!x && !y && !z) continue;
                const double d = std::sqrt((double)(x * x + y * y + z * z));
                double *K = &P->Ktab[(size_t)off_index(x, y, z) * 4];
                K[0] = -G / (h * d);
                const double c = G / (h * h * d * d * d);
                K[1] = c * x; K[2] = c * y; K[3] = c * z;
            }

    const std::vector<char4> &pl = (L == 0) ? P->plist_cube : P->plist_near;
    leaf_tables(P->Ktab, pl, 1.0, 1.0, r2i, false, P->Kst, P->Ksa);

    // tree passes over the levels 0..L-2 in spans of at most three levels,
    // aligned to the bottom: [L-4, L-2], [L-7, L-5], ... and a shorter top span
    P->dp.n_span = 0;
    {
        int top = L - 1, spans[MAX_LEVELS][2], n = 0;
        while (top > 0) {
            const int lo = std::max(0, top - 3);
            spans[n][0] = lo;
            spans[n][1] = top - lo;
            ++n;
            top = lo;
        }
        for (int i = 0; i < n; ++i) {        // top-down order
            P->dp.span_top[i] = spans[n - 1 - i][0];
            P->dp.span_n[i] = spans[n - 1 - i][1];
        }
        P->dp.n_span = n;
    }

    shift_mags(0.5 * h, P->dp.e_leaf);

    // derivative tensors per level l < L at R = z_sink - z_source = -o h_l
    const int nlev = std::max(L, 1);
    P->Dtab.assign((size_t)nlev * OFF_N * NC, 0.0);
    for (int l = 0; l < L; ++l) {
        const double hl = h * (double)(1 << (L - l));
        for (int z = -OFF_R; z <= OFF_R; ++z)
            for (int y = -OFF_R; y <= OFF_R; ++y)
                for (int x = -OFF_R; x <= OFF_R; ++x) {
                    if (!x && !y && !z) continue;
                    derivative_tensor(G, -x * hl, -y * hl, -z * hl,
                                      &P->Dtab[((size_t)l * OFF_N + off_index(x, y, z)) * NC]);
                }
    }

}

// Whether M2L unit (block blk, parent offset P) of a level with np parents
// per axis has a source in the domain: the block's parents shifted by P
// overlap [0, np) on every axis.  The blocks are those of the kernels: 64
// parents, bx * by * bz, numbered x fastest.
bool unit_has_sources(int np, int blk, char4 P, Block bs)
{
    const int bx = bs.bx, by = bs.by, bz = bs.bz;
    const int nbx = np / bx, nby = np / by;
    const int x0 = (blk % nbx) * bx, y0 = ((blk / nbx) % nby) * by, z0 = (blk / (nbx * nby)) * bz;
    auto overlap = [np](int a0, int n, int o) { return a0 + o < np && a0 + n - 1 + o >= 0; };
    return overlap(x0, bx, P.x) && overlap(y0, by, P.y) && overlap(z0, bz, P.z);
}

// Cut each level's M2L units into runs, G workgroups in all, in proportion
// to the level's computed units (a source in the domain and, in an adaptive
// tree, a block with cells of existing sub-grids; at least one run per
// level); runs are balanced in those units and skip the others.  Records
// per level the list of computed units and how many partial sums a block can
// receive.
struct M2LSched {
    std::vector<M2LDesc> mdesc;
    std::vector<int32_t> ulist[MAX_LEVELS];
    int maxp[MAX_LEVELS] = {};
    std::vector<uint16_t> npieces[MAX_LEVELS];     // per block: its pieces, 0 if no unit of it is computed
};

// Whether unit (block blk, parent offset P) of level l reads a cell of a
// refined sub-grid: the block's parents shifted by P cover sub-grids (parent
// >> 2) of which one is refined
bool unit_reads_refined(ot_fmm_plan P_, int l, int blk, char4 P, Block bs)
{
    const int np = 4 << l, m = 1 << l;
    const int nbx = np / bs.bx, nby = np / bs.by;
    const int x0 = (blk % nbx) * bs.bx + P.x, y0 = ((blk / nbx) % nby) * bs.by + P.y,
              z0 = (blk / (nbx * nby)) * bs.bz + P.z;
    auto lo = [](int a) { return std::max(a, 0) >> 2; };
    auto hi = [np](int a) { return std::min(a, np - 1) >> 2; };
    for (int z = lo(z0); z <= hi(z0 + bs.bz - 1); ++z)
        for (int y = lo(y0); y <= hi(y0 + bs.by - 1); ++y)
            for (int x = lo(x0); x <= hi(x0 + bs.bx - 1); ++x)
                if (x < m && y < m && z < m && P_->ntype[l][((size_t)z * m + y) * m + x] == 2) return true;
    return false;
}

// live_nodes (per level, or null): only blocks holding cells of these sub-grids;
// refined_sources: only units that read a cell of a refined sub-grid
void build_m2l_schedule(ot_fmm_plan P, int G, const std::vector<int32_t> *live_nodes, M2LSched &S,
                        bool refined_sources = false)
{
    S.mdesc.clear();
    const int L = P->L;
    for (int l = 0; l < MAX_LEVELS; ++l) {
        S.maxp[l] = 0;
        S.ulist[l].clear();
        S.npieces[l].clear();
    }
    if (L < 1) return;
    std::vector<std::vector<int64_t>> pos(L);     // each level's computed units, in order
    std::vector<int64_t> U(L), V(L);
    int64_t Vtot = 0;
    for (int l = 0; l < L; ++l) {
        const int np = 4 << l;
        const std::vector<char4> &pl = (l == 0) ? P->plist_cube : P->plist_near;
        const int nP = (int)pl.size();
        U[l] = (int64_t)np * np * np / 64 * nP;
        // adaptive trees: only blocks that hold cells of the listed sub-grids
        std::vector<char> live;
        if (live_nodes) {
            live.assign((size_t)(U[l] / nP), 0);
            for (int32_t b : blocks_of(l, live_nodes[l], amr_block(l))) live[(size_t)b] = 1;
        }
        const Block bs = P->amr ? amr_block(l) : block_shape(np);
        for (int64_t u = 0; u < U[l]; ++u)
            if (unit_has_sources(np, (int)(u / nP), pl[u % nP], bs) && (live.empty() || live[(size_t)(u / nP)]) &&
                (!refined_sources || unit_reads_refined(P, l, (int)(u / nP), pl[u % nP], bs))) {
                pos[l].push_back(u);
            }
        V[l] = (int64_t)pos[l].size();
        Vtot += V[l];
    }
    std::vector<int> Gl(L);
    int used = 0;
    for (int l = 0; l < L; ++l) {
        // at least one run per level, and runs of at least 8 units (32 tiles)
        Gl[l] = (int)std::max<int64_t>(1, std::min<int64_t>(V[l] / 8, (int64_t)G * V[l] / Vtot));
        used += Gl[l];
    }
    // hand any remainder to the deepest level
    if (used < G) Gl[L - 1] = (int)std::max<int64_t>(1, std::min<int64_t>(V[L - 1] / 8, Gl[L - 1] + (G - used)));
    for (int l = L - 1; l >= 0; --l) {
        const int nP = (l == 0) ? (int)P->plist_cube.size() : (int)P->plist_near.size();
        const int g = Gl[l];
        // run r covers raw units [b[r], b[r + 1]): from its first computed unit
        // (run 0 from unit 0) up to the next run's
        std::vector<int64_t> b(g + 1);
        for (int r = 0; r < g; ++r) b[r] = (r == 0) ? 0 : pos[l][(size_t)((int64_t)r * V[l] / g)];
        b[g] = U[l];
        auto run_of = [&](int64_t u) {        // run of this level whose range holds unit u
            return (int)(std::upper_bound(b.begin(), b.end(), u) - b.begin()) - 1;
        };
        for (int r = 0; r < g; ++r) {
            M2LDesc d{};
            d.level = l;
            d.ubeg = (int)b[r];
            d.uend = (int)b[r + 1];
            d.nvalid = (int)((int64_t)(r + 1) * V[l] / g - (int64_t)r * V[l] / g);
            d.vbeg = (int)((int64_t)r * V[l] / g);
            const int64_t first = (int64_t)(d.ubeg / nP) * nP;
            d.piece0 = (d.ubeg == first) ? 0 : r - run_of(first);
            S.mdesc.push_back(d);
        }
        S.ulist[l].resize(pos[l].size());          // block << 9 | parent offset (nP <= 343)
        for (size_t k = 0; k < pos[l].size(); ++k)
            S.ulist[l][k] = (int32_t)(((pos[l][k] / nP) << 9) | (pos[l][k] % nP));
        int maxp = 0;
        for (int64_t blk = 0; blk < U[l] / nP; ++blk)
            maxp = std::max(maxp, run_of(blk * nP + nP - 1) - run_of(blk * nP) + 1);
        S.maxp[l] = maxp;
        // a block's pieces are numbered from the run holding its first unit
        std::vector<char> has((size_t)(U[l] / nP), 0);
        for (int64_t u : pos[l]) has[(size_t)(u / nP)] = 1;
        S.npieces[l].assign(has.size(), 0);
        for (size_t blk = 0; blk < has.size(); ++blk)
            if (has[blk])
                S.npieces[l][blk] = (uint16_t)(run_of((int64_t)blk * nP + nP - 1) - run_of((int64_t)blk * nP) + 1);
    }
}

// Adaptive trees: ordered pairs by enumeration over the cells of every
// existing sub-grid.  M2L pairs per level (existing sink and source); P2P
// pairs: leaf pairs of one level (near ones, and at the finest level the far
// stencil too, which its leaf pass sums directly) and the coarse-fine pairs.
void fill_info_amr(ot_fmm_plan P)
{
    ot_fmm_info &I = P->info;
    const int L = P->L, r2i = P->dp.r2i;
    auto kind = [&](int l, int x, int y, int z) -> int {
        const int n = 8 << l;
        if (l < 0 || l > L || x < 0 || y < 0 || z < 0 || x >= n || y >= n || z >= n) return 0;
        const size_t m = (size_t)1 << l;
        return P->ntype[l][((size_t)(z >> 3) * m + (y >> 3)) * m + (x >> 3)];
    };
    auto near = [&](int dx, int dy, int dz) { return dx * dx + dy * dy + dz * dz <= r2i; };
    int64_t p2p = 0, m2l = 0;
    for (int l = 0; l <= L; ++l) {
        int64_t cnt_m2l = 0, cnt_p2p = 0;
        std::vector<int32_t> all(P->lnodes[l]);
        all.insert(all.end(), P->rnodes[l].begin(), P->rnodes[l].end());
        for (int32_t pk : all) {
            const int sx = pk & 1023, sy = (pk >> 10) & 1023, sz = (pk >> 20) & 1023;
            const bool leaf = kind(l, 8 * sx, 8 * sy, 8 * sz) == 1;
            for (int k = 0; k < 512; ++k) {
                const int x = 8 * sx + (k & 7), y = 8 * sy + ((k >> 3) & 7), z = 8 * sz + (k >> 6);
                // same-level stencil: the children of the parents near the
                // cell's parent (the whole root sub-grid at the root)
                const int r = (int)std::sqrt((double)r2i);
                const std::vector<char4> &pl = (l == 0) ? P->plist_cube : P->plist_near;
                for (size_t ip = 0; ip < pl.size() * 8; ++ip) {
                            const char4 Pc = pl[ip >> 3];
                            const int bp = (int)(ip & 7);
                            const int bx = 2 * ((x >> 1) + Pc.x) + (bp & 1), by = 2 * ((y >> 1) + Pc.y) + ((bp >> 1) & 1),
                                      bz = 2 * ((z >> 1) + Pc.z) + (bp >> 2);
                            const int dx = bx - x, dy = by - y, dz = bz - z;
                            const int t = kind(l, bx, by, bz);
                            if (!t || (!dx && !dy && !dz)) continue;
                            if (near(dx, dy, dz)) {
                                if (leaf && t == 1) ++cnt_p2p;
                                else if (leaf && t == 2) cnt_p2p += 8;       // the refined cell's children
                                continue;
                            }
                            if (l > 0 && !near((bx >> 1) - (x >> 1), (by >> 1) - (y >> 1), (bz >> 1) - (z >> 1)))
                                continue;
                            if (leaf && t == 1) ++cnt_p2p;      // two leaves: the leaf pass sums them directly
                            else ++cnt_m2l;
                        }
                // a leaf's coarse-fine pairs with the leaves near its parent
                if (leaf && l > 0)
                    for (int dz = -r; dz <= r; ++dz)
                        for (int dy = -r; dy <= r; ++dy)
                            for (int dx = -r; dx <= r; ++dx)
                                if ((dx || dy || dz) && near(dx, dy, dz) &&
                                    kind(l - 1, (x >> 1) + dx, (y >> 1) + dy, (z >> 1) + dz) == 1)
                                    ++cnt_p2p;
            }
        }
        if (l < L) I.m2l_pairs_level[l] = cnt_m2l;
        m2l += cnt_m2l;
        p2p += cnt_p2p;
    }
    I.p2p_pairs = p2p;
    I.m2l_pairs = m2l;
    int64_t refined_cells = 0;
    for (int l = 1; l < L; ++l) refined_cells += 512 * (int64_t)P->rnodes[l].size();
    const double N = (double)I.n_leaf_cells;
    const double tree = 2.0 * 84.0 * 2.0 * (double)refined_cells;
    I.flops_forward = 8.0 * (double)p2p + 168.0 * (double)m2l + tree + 2.0 * (20.0 + 50.0) * N;
    I.flops_adjoint = 8.0 * (double)p2p + 168.0 * (double)m2l + tree + 2.0 * (50.0 + 20.0) * N;
    int64_t cells = 0;
    for (int l = 0; l < L; ++l) cells += 512 * (int64_t)(P->rnodes[l].size() + P->lnodes[l].size());
    I.bytes_forward = 8.0 * N + 32.0 * N + 4.0 * NC * 8.0 * (double)cells;
    I.bytes_adjoint = 32.0 * N + 8.0 * N + 4.0 * NC * 8.0 * (double)cells;
}

// ordered pairs and algorithmic work of the plan
void fill_info(ot_fmm_plan P)
{
    ot_fmm_info &I = P->info;
    std::memset(&I, 0, sizeof I);
    const int L = P->L;
    const int r2i = P->dp.r2i;
    I.depth = L;
    I.order = P->order;
    I.theta = P->theta;
    I.n_nodes = P->n_nodes;
    I.n_leaf_nodes = P->n_leaf_nodes;
    I.n_leaf_cells = P->n_leaf_nodes * 512;

    auto parity_sum = [&](int n, bool far) {
        // sum over sink parities b, near parent offsets P and source children b'
        int64_t tot = 0;
        for (int b = 0; b < 8; ++b)
            for (const char4 &Pc : P->plist_near)
                for (int bp = 0; bp < 8; ++bp) {
                    const int o[3] = {2 * Pc.x + (bp & 1) - (b & 1), 2 * Pc.y + ((bp >> 1) & 1) - ((b >> 1) & 1),
                                      2 * Pc.z + (bp >> 2) - (b >> 2)};
                    const int o2 = o[0] * o[0] + o[1] * o[1] + o[2] * o[2];
                    if (o2 == 0 || (far && o2 <= r2i)) continue;
                    tot += axis_count(n, b & 1, o[0]) * axis_count(n, (b >> 1) & 1, o[1]) *
                           axis_count(n, b >> 2, o[2]);
                }
        return tot;
    };
    auto root_far = [&]() {
        int64_t tot = 0;
        for (int a = 0; a < 512; ++a)
            for (int c = 0; c < 512; ++c) {
                const int dx = (c & 7) - (a & 7), dy = ((c >> 3) & 7) - ((a >> 3) & 7), dz = (c >> 6) - (a >> 6);
                if (dx * dx + dy * dy + dz * dz > r2i) ++tot;
            }
        return tot;
    };

    if (P->amr) {
        fill_info_amr(P);
        return;
    }
    const int64_t N = I.n_leaf_cells;
    I.p2p_pairs = (L == 0) ? (int64_t)512 * 511 : parity_sum(8 << L, false);
    int64_t m2l = 0;
    for (int l = 0; l < L; ++l) {
        I.m2l_pairs_level[l] = (l == 0) ? root_far() : parity_sum(8 << l, true);
        m2l += I.m2l_pairs_level[l];
    }
    I.m2l_pairs = m2l;

    // algorithmic FLOP: 8 per P2P pair, 168 per M2L pair; M2M/L2L 84 FMA per
    // cell of levels 1..L-1; leaves: 20 FMA into the first moments, 50 FMA
    // of L2P (potential + gradient); adjoint leaves 50 (monopole + dipole)
    // and 20 (potential).
    int64_t internal_below_root = 0;
    for (int l = 1; l < L; ++l) internal_below_root += (int64_t)(8 << l) * (8 << l) * (8 << l);
    const double tree = 2.0 * 84.0 * 2.0 * (double)internal_below_root;   // M2M + L2L
    const double lf = (L >= 1) ? 1.0 : 0.0;
    I.flops_forward = 8.0 * (double)I.p2p_pairs + 168.0 * (double)m2l + tree + lf * 2.0 * (20.0 + 50.0) * (double)N;
    I.flops_adjoint = 8.0 * (double)I.p2p_pairs + 168.0 * (double)m2l + tree + lf * 2.0 * (50.0 + 20.0) * (double)N;
    // algorithmic bytes: leaf inputs and outputs once, plus every internal
    // cell's moments and locals written once and read once
    int64_t internal = 0;
    for (int l = 0; l < L; ++l) internal += (int64_t)(8 << l) * (8 << l) * (8 << l);
    const double tree_bytes = 4.0 * NC * 8.0 * (double)internal;
    I.bytes_forward = 8.0 * N + 32.0 * N + tree_bytes;
    I.bytes_adjoint = 32.0 * N + 8.0 * N + tree_bytes;
}

template <typename T>
int dev_alloc(ot_fmm_plan P, T **ptr, size_t count, bool zero)
{
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(OT_FMM_OUT_OF_MEMORY, std::string("hipMalloc of ") + std::to_string(bytes) +
                                              " bytes failed: " + hipGetErrorString(e));
    }
    P->allocations.push_back(p);
    P->info.device_bytes += bytes;
    if (zero) {
        e = hipMemset(p, 0, bytes);
        if (e != hipSuccess) return hip_fail(e, "hipMemset");
    }
    *ptr = static_cast<T *>(p);
    return OT_FMM_OK;
}

template <typename T>
int dev_upload(ot_fmm_plan P, const T **dst, const std::vector<T> &src)
{
    T *p = nullptr;
    int rc = dev_alloc(P, &p, src.size(), false);
    if (rc) return rc;
    if (!src.empty()) {
        hipError_t e = hipMemcpy(p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    }
    *dst = p;
    return OT_FMM_OK;
}

void free_device(ot_fmm_plan P)
{
    for (void *p : P->allocations) (void)hipFree(p);
    P->allocations.clear();
    for (hipEvent_t ev : P->timing.pool) (void)hipEventDestroy(ev);
    P->timing.pool.clear();
}

// Time each leaf pass of d (the plan, or one level's view of an adaptive
// tree) with 1, 2, 4 and 8 stencil chunks (a warm-up launch, then the best of
// three single launches, on the plan's zeroed scratch and temporary outputs)
// and keep the fastest count.
int autotune_leaf(ot_fmm_plan P, DevPlan &d)
{
    const size_t N = (size_t)d.n_leaf_cells;
    double *o0 = nullptr, *o1 = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipMalloc(&o0, N * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&o1, 3 * N * sizeof(double));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    for (int adj = 0; adj < 2 && e == hipSuccess; ++adj) {
        float best = 0.0f;
        for (int c = 1; c <= LEAF_MAX_CHUNKS && e == hipSuccess; c *= 2) {
            float tmin = 0.0f;
            for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
                if ((e = hipEventRecord(ev[0], st)) != hipSuccess) break;
                if ((e = launch_leaf_chunks(d, adj, c, o0, o1, st)) != hipSuccess) break;
                if ((e = hipEventRecord(ev[1], st)) != hipSuccess) break;
                if ((e = hipEventSynchronize(ev[1])) != hipSuccess) break;
                float ms = 0.0f;
                if ((e = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess) break;
                if (rep > 0 && (rep == 1 || ms < tmin)) tmin = ms;     // launch 0 warms up
            }
            if (e == hipSuccess && (c == 1 || tmin < best)) {
                best = tmin;
                d.leaf_chunks[adj] = c;
            }
        }
    }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (st) (void)hipStreamDestroy(st);
    if (o1) (void)hipFree(o1);
    if (o0) (void)hipFree(o0);
    return e == hipSuccess ? OT_FMM_OK : hip_fail(e, "leaf autotuning");
}

// stencil chunks of a leaf pass over nblk blocks: the smallest power of two
// that gives a launch of at least 16384 waves (see setup_device)
int chunk_rule(int64_t nblk)
{
    int c = 1;
    while (c < LEAF_MAX_CHUNKS && nblk * c < 16384) c *= 2;
    return c;
}

// Adaptive trees: node kinds and lists on the device, and one view of the
// plan per level that holds leaves (its leaf pass and coarse-fine pass)
int setup_amr_views(ot_fmm_plan P, int G)
{
    DevPlan &d = P->dp;
    const int L = P->L;
    int rc;
    // The leaf-sink M2L: for the leaf sub-grids next to a refined one of their
    // level (the far stencil reaches at most 5 cells, inside the 26
    // neighbours), the M2L from the refined cells alone; a leaf's far pairs
    // with leaves are P2P pairs of its leaf pass.
    std::vector<int32_t> iface[MAX_LEVELS];
    for (int l = 1; l < L; ++l) {
        const int m = 1 << l;
        for (int32_t pk : P->lnodes[l]) {
            const int x = pk & 1023, y = (pk >> 10) & 1023, z = (pk >> 20) & 1023;
            bool any = false;
            for (int e = 0; e < 27 && !any; ++e) {
                const int qx = x + e % 3 - 1, qy = y + (e / 3) % 3 - 1, qz = z + e / 9 - 1;
                if (qx < 0 || qy < 0 || qz < 0 || qx >= m || qy >= m || qz >= m) continue;
                any = P->ntype[l][((size_t)qz * m + qy) * m + qx] == 2;
            }
            if (any) iface[l].push_back(pk);
        }
    }
    M2LSched S;
    build_m2l_schedule(P, G, iface, S, true);
    int64_t nunits = 0;
    for (int l = 0; l < L; ++l) nunits += (int64_t)S.ulist[l].size();
    P->has_m2l_leaf = nunits > 0;
    double *cpB[MAX_LEVELS] = {};
    for (int l = 0; l < L; ++l) {
        DevLevel &v = d.lev[l];
        const size_t pp3 = (size_t)v.pp * v.pp * v.pp, np3 = (size_t)v.np * v.np * v.np;
        v.Mr_ref = nullptr;
        v.M32_ref = nullptr;
        if (!P->has_m2l_leaf || P->rnodes[l].empty()) continue;
        if (d.m2l_fp32) {
            if ((rc = dev_alloc(P, &v.M32_ref, (size_t)NR * 8 * pp3, true))) return rc;
        } else if ((rc = dev_alloc(P, &v.Mr_ref, (size_t)NR * 8 * pp3, true))) {
            return rc;
        }
        if (!S.ulist[l].empty() && (rc = dev_alloc(P, &cpB[l], (size_t)std::max(S.maxp[l], 1) * NC * 8 * np3, true)))
            return rc;
    }
    if (P->has_m2l_leaf) {
        DevPlan &b = P->m2l_leaf;
        b = d;
        for (int l = 0; l < L; ++l) {
            DevLevel &v = b.lev[l];
            v.Mr = v.Mr_ref;
            v.M32 = v.M32_ref;
            v.Cp = cpB[l];
            v.maxp = S.maxp[l];
            v.ulist = nullptr;
            if ((rc = dev_upload(P, &v.ulist, S.ulist[l]))) return rc;
        }
        const M2LDesc *md = nullptr;
        if ((rc = dev_upload(P, &md, S.mdesc))) return rc;
        b.mdesc = md;
        b.n_mdesc = (int)S.mdesc.size();
    }
    for (int l = 0; l <= L; ++l) {
        const uint8_t *nt = nullptr;
        if ((rc = dev_upload(P, &nt, P->ntype[l]))) return rc;
        P->dev_ntype[l] = nt;
        if ((rc = dev_upload(P, &P->dev_lnodes[l], P->lnodes[l]))) return rc;
        if ((rc = dev_upload(P, &P->dev_rnodes[l], P->rnodes[l]))) return rc;
    }
    double *srcs[MAX_LEVELS] = {};
    for (int l = 1; l <= L; ++l) {
        if (P->lnodes[l].empty()) continue;
        DevPlan &v = P->view[l];
        v = d;
        const double hl = P->h * (double)(1 << (L - l));
        v.L = l;
        v.hleaf = hl;
        v.h3 = hl * hl * hl;
        v.sL = 1 << l;
        v.npL = 4 << l;
        v.hpL = 2;
        v.ppL = v.npL + 2 * v.hpL;
        if ((rc = dev_upload(P, &v.leaf_slot, P->lslot[l]))) return rc;
        if ((rc = dev_upload(P, &v.Kst, P->Kst_l[l]))) return rc;
        if ((rc = dev_upload(P, &v.Ksa, P->Ksa_l[l]))) return rc;
        v.plist_leaf = d.plist_near;
        v.n_plist_leaf = d.n_plist_near;
        shift_mags(0.5 * hl, v.e_leaf);
        const size_t pp3 = (size_t)v.ppL * v.ppL * v.ppL;
        if ((rc = dev_alloc(P, &srcs[l], 4 * 8 * pp3, true))) return rc;
        v.src = srcs[l];
        v.own_Cp = (l < L && cpB[l]) ? cpB[l] : nullptr;
        v.own_maxp = (l < L) ? S.maxp[l] : 0;
        v.own_np = nullptr;
        v.own_subgrid_blocks = (4 << l) >= 16 ? 1 : 0;      // the M2L's blocks at this level (amr_block)
        if (v.own_Cp && (rc = dev_upload(P, &v.own_np, S.npieces[l]))) return rc;
        v.ntype_L = P->dev_ntype[l];
        v.leaf_subgrid_blocks = P->lsub[l];
        if ((rc = dev_upload(P, &v.blist, P->lblk[l]))) return rc;
        v.nblist = (int)P->lblk[l].size();
        v.Kcf_up = v.Kcf_dn = nullptr;
        if (!P->Kup_l[l].empty() && (rc = dev_upload(P, &v.Kcf_up, P->Kup_l[l]))) return rc;
        if (!P->Kdn_l[l].empty() && (rc = dev_upload(P, &v.Kcf_dn, P->Kdn_l[l]))) return rc;
        v.leaf_chunks[0] = v.leaf_chunks[1] = chunk_rule(v.nblist);
    }
    for (int l = 1; l <= L; ++l) {
        if (P->lnodes[l].empty()) continue;
        DevPlan &v = P->view[l];
        v.src_up = v.Kcf_up ? srcs[l - 1] : nullptr;
        v.hp_up = 2;
        v.pp_up = (4 << (l - 1)) + 4;
        v.src_dn = v.Kcf_dn ? srcs[l + 1] : nullptr;
        v.hp_dn = 2;
        v.pp_dn = (4 << (l + 1)) + 4;
    }
    return OT_FMM_OK;
}

int setup_device(ot_fmm_plan P)
{
    hipError_t e = hipGetDevice(&P->device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    DevPlan &d = P->dp;
    const int L = P->L;
    d.L = L;
    d.hleaf = P->h;
    d.G = P->G;
    d.h3 = P->h * P->h * P->h;
    d.sL = 1 << L;
    d.npL = 4 << L;
    d.hpL = (L == 0) ? 3 : 2;
    d.ppL = d.npL + 2 * d.hpL;
    d.n_leaf_cells = P->n_leaf_nodes * 512;
    int rc;
    if ((rc = dev_upload(P, &d.leaf_slot, P->leaf_slot))) return rc;
    if ((rc = dev_upload(P, &d.Ktab, P->Ktab))) return rc;
    if ((rc = dev_upload(P, &d.Kst, P->Kst))) return rc;
    if ((rc = dev_upload(P, &d.Ksa, P->Ksa))) return rc;
    if ((rc = dev_upload(P, &d.Dtab, P->Dtab))) return rc;
    d.m2l_fp32 = (P->flags & OT_FMM_M2L_FP32) ? 1 : 0;
    d.Dtab32 = nullptr;
    if (d.m2l_fp32) {
        P->Dtab32.assign(P->Dtab.begin(), P->Dtab.end());    // rounded to nearest
        if ((rc = dev_upload(P, &d.Dtab32, P->Dtab32))) return rc;
    }
    if ((rc = dev_upload(P, &d.plist_near, P->plist_near))) return rc;
    if ((rc = dev_upload(P, &d.plist_cube, P->plist_cube))) return rc;
    int ncu = 0, per_cu = 0;
    if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, P->device)) != hipSuccess)
        return hip_fail(e, "hipDeviceGetAttribute");
    if ((e = m2l_blocks_per_cu(d.m2l_fp32, &per_cu)) != hipSuccess) return hip_fail(e, "occupancy of the M2L kernel");
    const int G = std::max(1, ncu * std::max(1, per_cu));
    {
        // adaptive trees: the M2L of refined sinks (the leaf sinks next to
        // refined cells get a second, leaf-sink M2L; see setup_amr_views)
        M2LSched S;
        build_m2l_schedule(P, G, P->amr ? P->rnodes : nullptr, S);
        P->mdesc = S.mdesc;
        for (int l = 0; l < MAX_LEVELS; ++l) {
            P->ulist[l] = S.ulist[l];
            d.lev[l].maxp = S.maxp[l];
        }
    }
    if ((rc = dev_upload(P, &d.mdesc, P->mdesc))) return rc;
    d.n_plist_near = (int)P->plist_near.size();
    d.n_plist_cube = (int)P->plist_cube.size();
    d.plist_leaf = (L == 0) ? d.plist_cube : d.plist_near;
    d.n_plist_leaf = (L == 0) ? d.n_plist_cube : d.n_plist_near;
    d.n_mdesc = (int)P->mdesc.size();
    const size_t ppL3 = (size_t)d.ppL * d.ppL * d.ppL;
    d.src = nullptr;
    if (!P->amr && (rc = dev_alloc(P, &d.src, 4 * 8 * ppL3, true))) return rc;
    for (int l = 0; l < L; ++l) {
        DevLevel &v = d.lev[l];
        v.np = 4 << l;
        v.hp = (l == 0) ? 3 : 2;
        v.pp = v.np + 2 * v.hp;
        v.h = P->h * (double)(1 << (L - l));
        const Block bs = P->amr ? amr_block(l) : block_shape(v.np);
        v.bx = bs.bx;
        v.by = bs.by;
        v.bz = bs.bz;
        v.nbx = v.np / v.bx;
        v.nby = v.np / v.by;
        const size_t pp3 = (size_t)v.pp * v.pp * v.pp, np3 = (size_t)v.np * v.np * v.np;
        // full moments where an M2M launch reads them back from memory: the
        // top level of every span below another span (the bottom span forms
        // level L-1 itself, from the leaf sources)
        bool full = false;
        for (int i = 1; i < d.n_span; ++i) full = full || (l == d.span_top[i]);
        if (P->amr) full = l >= 1 && !P->rnodes[l].empty();     // the M2M of level l - 1 reads them
        if (P->flags & OT_FMM_AM_CORRECTION) full = true;       // the correction reads every level's
        v.M = nullptr;
        v.Mr = nullptr;
        v.M32 = nullptr;
        if (full && (rc = dev_alloc(P, &v.M, (size_t)NC * 8 * pp3, true))) return rc;
        if (d.m2l_fp32) {
            if ((rc = dev_alloc(P, &v.M32, (size_t)NR * 8 * pp3, true))) return rc;
        } else if ((rc = dev_alloc(P, &v.Mr, (size_t)NR * 8 * pp3, true))) {
            return rc;
        }
        if (l < L - 1 && (rc = dev_alloc(P, &v.C, (size_t)NC * 8 * np3, true))) return rc;
        if ((rc = dev_upload(P, &v.ulist, P->ulist[l]))) return rc;
        // pieces a block never receives stay zero: the schedule is fixed per plan
        if ((rc = dev_alloc(P, &v.Cp, (size_t)std::max(v.maxp, 1) * NC * 8 * np3, true))) return rc;
    }
    if (P->amr && (rc = setup_amr_views(P, G))) return rc;
    if (P->flags & OT_FMM_AM_CORRECTION) {
        am_table(P);
        if ((rc = dev_upload(P, &P->dev_KX, P->KX))) return rc;
        for (int l = 0; l < L; ++l) {
            const size_t np3 = (size_t)d.lev[l].np * d.lev[l].np * d.lev[l].np;
            if ((rc = dev_alloc(P, &P->Pi[l], (size_t)3 * NC * 8 * np3, true))) return rc;
        }
        int lds = 0;
        if ((e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device)) != hipSuccess)
            return hip_fail(e, "hipDeviceGetAttribute");
        P->am_tiled = (size_t)lds >= 2 * AM_TILE_LDS ? 2 : (size_t)lds >= AM_TILE_LDS ? 1 : 0;
        const size_t nsplit = am_split_size(L);
        if (P->am_tiled && nsplit && (rc = dev_alloc(P, &P->Pi_part, nsplit, false))) return rc;
    }
    // stencil chunks of the leaf passes: the smallest power of two that gives
    // a launch at least 16384 waves (four rounds of the 4096 wave slots the
    // leaf kernels' registers leave), at most LEAF_MAX_CHUNKS per block.  The
    // timing tuner picks the same counts at depths 1..4 (8, 8, 8, 4) and at
    // depth 5 (1) for the adjoint.
    d.leaf_chunks[0] = d.leaf_chunks[1] = chunk_rule((int64_t)d.npL * d.npL * d.npL / 64);
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize after plan setup");
    if (P->flags & OT_FMM_AUTOTUNE) {
        if (!P->amr) {
            if ((rc = autotune_leaf(P, d))) return rc;
        } else {
            for (int l = 1; l <= L; ++l)
                if (!P->lnodes[l].empty() && (rc = autotune_leaf(P, P->view[l]))) return rc;
        }
    }
    P->has_device = true;
    return OT_FMM_OK;
}

bool misaligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) != 0; }


// --------------------------------------------------------------------------
// timing of kernel phases with events on the call's stream
// --------------------------------------------------------------------------
struct Phase {
    ot_fmm_plan P;
    hipStream_t s;
    int phase;
    int launches;
    hipEvent_t a = nullptr, b = nullptr;
    Phase(ot_fmm_plan P_, hipStream_t s_, int phase_, int launches_) : P(P_), s(s_), phase(phase_), launches(launches_)
    {
        TimingState &T = P->timing;
        if (!T.active || T.calls >= T.max_calls || T.next + 2 > T.pool.size() || !((T.mask >> phase) & 1u)) return;
        a = T.pool[T.next++];
        b = T.pool[T.next++];
        (void)hipEventRecord(a, s);
    }
    void end()
    {
        if (!a) return;
        (void)hipEventRecord(b, s);
        P->timing.recs.push_back(TimingState::Rec{phase, launches, a, b});
    }
};

struct DeviceGuard {
    int prev = -1;
    bool switched = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) switched = (hipSetDevice(dev) == hipSuccess);
    }
    ~DeviceGuard()
    {
        if (switched) (void)hipSetDevice(prev);
    }
};

// the M2M spans above the bottom one (the bottom span runs fused with the
// P2M), the M2L of every level, and the L2L down to level L-2; the forward
// and the adjoint share them (the leaf stages differ)
hipError_t tree_passes(ot_fmm_plan P, hipStream_t s)
{
    const DevPlan &d = P->dp;
    hipError_t e = hipSuccess;
    if (d.n_span > 1) {
        Phase ph(P, s, OT_FMM_PHASE_M2M, d.n_span - 1);
        if ((e = launch_m2m_upper(d, s)) != hipSuccess) return e;
        ph.end();
    }
    if (P->L >= 1) {
        Phase ph(P, s, OT_FMM_PHASE_M2L, 1);
        if ((e = launch_m2l(d, s)) != hipSuccess) return e;
        ph.end();
    }
    if (d.n_span > 0) {
        Phase ph(P, s, OT_FMM_PHASE_L2L, d.n_span);
        for (int i = 0; i < d.n_span; ++i)
            if ((e = launch_l2l_span(d, i, s)) != hipSuccess) return e;
        ph.end();
    }
    return e;
}

// Adaptive trees, forward (adj 0: rho -> phi, g) or adjoint (adj 1: dphi, dg
// -> drho): leaf moments and M2M level by level, the M2L of every level, the
// L2L spans, then per level holding leaves its leaf pass and its coarse-fine
// pairs.
int amr_run(ot_fmm_plan P, int adj, const double *a0, const double *a1, double *out0, double *out1, hipStream_t s)
{
    const DevPlan &d = P->dp;
    const int L = P->L;
    hipError_t e;
    {
        int nl = 0;
        for (int l = 0; l <= L; ++l) nl += (l >= 1 && l < L && !P->lnodes[l].empty()) + !P->rnodes[l].empty();
        Phase ph(P, s, adj ? OT_FMM_PHASE_UPWARD_LEAF_ADJ : OT_FMM_PHASE_UPWARD_LEAF, nl);
        for (int l = 1; l < L; ++l)
            if (!P->lnodes[l].empty() &&
                (e = launch_amr_leaf_moments(P->view[l], adj, P->dev_lnodes[l], (int)P->lnodes[l].size(), a0, a1,
                                             s)) != hipSuccess)
                return hip_fail(e, "launch of the leaf moments");
        for (int l = L - 1; l >= 0; --l) {
            const DevPlan &v = P->lnodes[l + 1].empty() ? d : P->view[l + 1];
            if ((e = launch_amr_m2m(v, adj, l, P->dev_rnodes[l], (int)P->rnodes[l].size(), P->dev_ntype[l + 1], a0,
                                    a1, s)) != hipSuccess)
                return hip_fail(e, "launch of an M2M level");
        }
        ph.end();
    }
    {
        Phase ph(P, s, OT_FMM_PHASE_M2L, 1 + P->has_m2l_leaf);
        if ((e = launch_m2l(d, s)) != hipSuccess) return hip_fail(e, "launch m2l");
        if (P->has_m2l_leaf && (e = launch_m2l(P->m2l_leaf, s)) != hipSuccess)
            return hip_fail(e, "launch of the leaf-sink m2l");
        ph.end();
    }
    if (L >= 2) {
        // level by level over the refined sub-grids (a leaf cell's final
        // local has no reader); levels 0 .. L-2, the leaf passes form L-1
        Phase ph(P, s, OT_FMM_PHASE_L2L, L - 1);
        for (int l = 0; l <= L - 2; ++l)
            if ((e = launch_amr_l2l(d, l, P->dev_rnodes[l], (int)P->rnodes[l].size(), s)) != hipSuccess)
                return hip_fail(e, "launch of an L2L level");
        ph.end();
    }
    {
        int nl = 0;
        for (int l = 1; l <= L; ++l)
            nl += P->lnodes[l].empty() ? 0 : 1 + (P->view[l].own_Cp || P->view[l].src_up || P->view[l].src_dn);
        Phase ph(P, s, adj ? OT_FMM_PHASE_LEAF_ADJ : OT_FMM_PHASE_LEAF, nl);
        for (int l = 1; l <= L; ++l) {
            if (P->lnodes[l].empty()) continue;
            const DevPlan &v = P->view[l];
            if ((e = launch_leaf_chunks(v, adj, v.leaf_chunks[adj], out0, out1, s)) != hipSuccess)
                return hip_fail(e, "launch of a leaf pass");
        }
        for (int l = 1; l <= L; ++l)
            if (!P->lnodes[l].empty() && (e = launch_amr_cf(P->view[l], adj, out0, out1, s)) != hipSuccess)
                return hip_fail(e, "launch of a coarse-fine pass");
        ph.end();
    }
    return OT_FMM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// batches of independent plans: a fork over a few internal streams and a join
// back into the caller's stream, enqueued eagerly or captured into a graph
// ---------------------------------------------------------------------------
struct ot_fmm_batch_s {
    std::vector<ot_fmm_plan> plans;
    int device = -1;
    std::vector<hipStream_t> streams;   // internal, default priority
    hipEvent_t fork = nullptr;          // recorded on the caller's stream
    std::vector<hipEvent_t> join;       // one per internal stream
};

struct ot_fmm_graph_s {
    int device = -1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int BATCH_MAX_STREAMS = 16;

void release_batch(ot_fmm_batch B)
{
    for (hipStream_t s : B->streams) (void)hipStreamDestroy(s);
    for (hipEvent_t ev : B->join) (void)hipEventDestroy(ev);
    if (B->fork) (void)hipEventDestroy(B->fork);
    delete B;
}

// every pointer of the n argument triples present and 8-byte aligned
int check_batch_args(ot_fmm_batch B, const void *const *a, const void *const *b, const void *const *c)
{
    if (!B) return fail(OT_FMM_INVALID_ARGUMENT, "batch is NULL");
    if (!a || !b || !c) return fail(OT_FMM_INVALID_ARGUMENT, "NULL pointer array");
    for (size_t i = 0; i < B->plans.size(); ++i) {
        if (!a[i] || !b[i] || !c[i]) return fail(OT_FMM_INVALID_ARGUMENT, "NULL device pointer in a batch");
        if (misaligned(a[i]) || misaligned(b[i]) || misaligned(c[i]))
            return fail(OT_FMM_INVALID_ARGUMENT, "device pointers must be 8-byte aligned");
    }
    return OT_FMM_OK;
}

// fork from s, run plan i on internal stream i mod n_streams, join into s.
// The join is enqueued even after a failed launch, so that a capture stays
// well formed; the first failure is returned.
template <typename F>
int batch_enqueue(ot_fmm_batch B, hipStream_t s, F run_plan)
{
    const size_t ns = B->streams.size();
    hipError_t e = hipEventRecord(B->fork, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord (batch fork)");
    for (size_t k = 0; k < ns; ++k)
        if ((e = hipStreamWaitEvent(B->streams[k], B->fork, 0)) != hipSuccess)
            return hip_fail(e, "hipStreamWaitEvent (batch fork)");
    int rc = OT_FMM_OK;
    for (size_t i = 0; i < B->plans.size() && rc == OT_FMM_OK; ++i) rc = run_plan(i, B->streams[i % ns]);
    for (size_t k = 0; k < ns; ++k) {
        if ((e = hipEventRecord(B->join[k], B->streams[k])) != hipSuccess ||
            (e = hipStreamWaitEvent(s, B->join[k], 0)) != hipSuccess) {
            if (rc == OT_FMM_OK) rc = hip_fail(e, "batch join");
        }
    }
    return rc;
}

// capture one enqueue of the batch into an executable graph, on a stream of
// its own
template <typename F>
int batch_capture(ot_fmm_batch B, F enqueue, ot_fmm_graph *out)
{
    for (ot_fmm_plan P : B->plans)
        if (P->timing.active)
            return fail(OT_FMM_INVALID_ARGUMENT, "kernel timing is active on a plan of the batch; end it before capturing");
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags (capture)");
    ot_fmm_graph G = new (std::nothrow) ot_fmm_graph_s();
    if (!G) {
        (void)hipStreamDestroy(cs);
        return fail(OT_FMM_OUT_OF_MEMORY, "host allocation of the graph failed");
    }
    G->device = B->device;
    int rc = OT_FMM_OK;
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        rc = hip_fail(e, "hipStreamBeginCapture");
    } else {
        rc = enqueue(cs);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        if (rc == OT_FMM_OK && e != hipSuccess) rc = hip_fail(e, "hipStreamEndCapture");
        G->graph = g;
        if (rc == OT_FMM_OK && (e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0)) != hipSuccess)
            rc = hip_fail(e, "hipGraphInstantiate");
    }
    (void)hipStreamDestroy(cs);
    if (rc != OT_FMM_OK) {
        if (G->exec) (void)hipGraphExecDestroy(G->exec);
        if (G->graph) (void)hipGraphDestroy(G->graph);
        delete G;
        return rc;
    }
    *out = G;
    return OT_FMM_OK;
}

}  // namespace

extern "C" {

const char *ot_fmm_status_string(int s)
{
    switch (s) {
    case OT_FMM_OK: return "OT_FMM_OK";
    case OT_FMM_INVALID_ARGUMENT: return "OT_FMM_INVALID_ARGUMENT";
    case OT_FMM_INVALID_LAYOUT: return "OT_FMM_INVALID_LAYOUT";
    case OT_FMM_UNSUPPORTED_ORDER: return "OT_FMM_UNSUPPORTED_ORDER";
    case OT_FMM_UNSUPPORTED_THETA: return "OT_FMM_UNSUPPORTED_THETA";
    case OT_FMM_UNSUPPORTED_LAYOUT: return "OT_FMM_UNSUPPORTED_LAYOUT";
    case OT_FMM_OUT_OF_MEMORY: return "OT_FMM_OUT_OF_MEMORY";
    case OT_FMM_DEVICE_ERROR: return "OT_FMM_DEVICE_ERROR";
    case OT_FMM_NO_DEVICE_STATE: return "OT_FMM_NO_DEVICE_STATE";
    default: return "OT_FMM_UNKNOWN_STATUS";
    }
}

const char *ot_fmm_last_error(void) { return g_err.c_str(); }

const char *ot_fmm_phase_name(int phase)
{
    static const char *names[OT_FMM_NUM_PHASES] = {"upward_leaf", "m2m", "m2l", "l2l",
                                                   "leaf", "upward_leaf_adj", "leaf_adj", "total"};
    return (phase >= 0 && phase < OT_FMM_NUM_PHASES) ? names[phase] : "unknown";
}

int ot_fmm_plan_create(const ot_octree_layout *layout, double theta, int order, uint32_t flags,
                       ot_fmm_plan *out)
{
    if (!out) return fail(OT_FMM_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    if (flags & ~(OT_FMM_HOST_ONLY | OT_FMM_M2L_FP32 | OT_FMM_AUTOTUNE | OT_FMM_AM_CORRECTION))
        return fail(OT_FMM_INVALID_ARGUMENT, "unknown flag bits");
    if (!std::isfinite(theta) || theta <= 0.0) return fail(OT_FMM_INVALID_ARGUMENT, "theta must be finite and > 0");
    if (!(theta > 1.0 / 3.0 && theta <= 1.0))
        return fail(OT_FMM_UNSUPPORTED_THETA, "theta must lie in (1/3, 1] (near radius 1/theta in [1, 3) cells)");
    if (order != 3) return fail(OT_FMM_UNSUPPORTED_ORDER, "only expansion order 3 is implemented");
    ot_fmm_plan P = new (std::nothrow) ot_fmm_plan_s();
    if (!P) return fail(OT_FMM_OUT_OF_MEMORY, "host allocation of the plan failed");
    P->theta = theta;
    P->order = order;
    P->flags = flags;
    const double rn = 1.0 / theta;
    P->r2 = rn * rn;
    int rc = validate_layout(layout, P);
    if (rc) { delete P; return rc; }
    if (P->amr && (flags & OT_FMM_AM_CORRECTION)) {
        delete P;
        return fail(OT_FMM_UNSUPPORTED_LAYOUT, "the angular-momentum correction is built for uniform trees only");
    }
    try {
        build_tables(P);
        if (P->amr) build_amr_tables(P);
        fill_info(P);
    } catch (const std::bad_alloc &) {
        delete P;
        return fail(OT_FMM_OUT_OF_MEMORY, "host allocation of the tables failed");
    }
    if (!(flags & OT_FMM_HOST_ONLY)) {
        rc = setup_device(P);
        if (rc) {
            free_device(P);
            delete P;
            return rc;
        }
    }
    *out = P;
    return OT_FMM_OK;
}

int ot_fmm_plan_info(ot_fmm_plan P, ot_fmm_info *info)
{
    if (!P || !info) return fail(OT_FMM_INVALID_ARGUMENT, "plan or info is NULL");
    *info = P->info;
    const DevPlan &lp = P->amr ? P->view[P->L] : P->dp;     // adaptive trees: the deepest level's pass
    info->leaf_chunks_forward = P->has_device ? lp.leaf_chunks[0] : 0;
    info->leaf_chunks_adjoint = P->has_device ? lp.leaf_chunks[1] : 0;
    return OT_FMM_OK;
}

int ot_fmm_plan_set_leaf_chunks(ot_fmm_plan P, int forward, int adjoint)
{
    if (!P) return fail(OT_FMM_INVALID_ARGUMENT, "plan is NULL");
    if (forward < 1 || forward > LEAF_MAX_CHUNKS || adjoint < 1 || adjoint > LEAF_MAX_CHUNKS)
        return fail(OT_FMM_INVALID_ARGUMENT, "leaf chunk counts must lie in [1, 8]");
    if (!P->has_device) return fail(OT_FMM_NO_DEVICE_STATE, "plan was created with OT_FMM_HOST_ONLY");
    P->dp.leaf_chunks[0] = forward;
    P->dp.leaf_chunks[1] = adjoint;
    for (int l = 0; l < MAX_LEVELS; ++l) {      // adaptive trees: every level's leaf pass
        P->view[l].leaf_chunks[0] = forward;
        P->view[l].leaf_chunks[1] = adjoint;
    }
    return OT_FMM_OK;
}

void ot_fmm_destroy(ot_fmm_plan P)
{
    if (!P) return;
    if (P->has_device) {
        DeviceGuard g(P->device);
        free_device(P);
    }
    delete P;
}

int ot_fmm_forward(ot_fmm_plan P, const double *rho, double *phi, double *g, void *hip_stream)
{
    if (!P) return fail(OT_FMM_INVALID_ARGUMENT, "plan is NULL");
    if (!P->has_device) return fail(OT_FMM_NO_DEVICE_STATE, "plan was created with OT_FMM_HOST_ONLY");
    if (!rho || !phi || !g) return fail(OT_FMM_INVALID_ARGUMENT, "NULL device pointer");
    if (misaligned(rho) || misaligned(phi) || misaligned(g))
        return fail(OT_FMM_INVALID_ARGUMENT, "device pointers must be 8-byte aligned");
    DeviceGuard guard(P->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const DevPlan &d = P->dp;
    hipError_t e;
    Phase total(P, s, OT_FMM_PHASE_TOTAL, 0);
    if (P->amr) {
        const int rc = amr_run(P, 0, rho, nullptr, phi, g, s);
        if (rc) return rc;
        total.end();
        if (P->timing.active && P->timing.calls < P->timing.max_calls) P->timing.calls++;
        return OT_FMM_OK;
    }
    {
        Phase ph(P, s, OT_FMM_PHASE_UPWARD_LEAF, 1);
        if ((e = launch_upward_leaf(d, rho, s)) != hipSuccess) return hip_fail(e, "launch upward_leaf");
        ph.end();
    }
    if ((e = tree_passes(P, s)) != hipSuccess) return hip_fail(e, "launch of a tree pass");
    {
        Phase ph(P, s, OT_FMM_PHASE_LEAF, 1);
        if ((e = launch_leaf(d, phi, g, s)) != hipSuccess) return hip_fail(e, "launch leaf");
        ph.end();
    }
    total.end();
    if (P->timing.active && P->timing.calls < P->timing.max_calls) P->timing.calls++;
    return OT_FMM_OK;
}

int ot_fmm_am_correction(ot_fmm_plan P, const double *rho, double *t, void *hip_stream)
{
    if (!P) return fail(OT_FMM_INVALID_ARGUMENT, "plan is NULL");
    if (!P->has_device) return fail(OT_FMM_NO_DEVICE_STATE, "plan was created with OT_FMM_HOST_ONLY");
    if (!(P->flags & OT_FMM_AM_CORRECTION))
        return fail(OT_FMM_INVALID_ARGUMENT, "plan was created without OT_FMM_AM_CORRECTION");
    if (!rho || !t) return fail(OT_FMM_INVALID_ARGUMENT, "NULL device pointer");
    if (misaligned(rho) || misaligned(t)) return fail(OT_FMM_INVALID_ARGUMENT, "device pointers must be 8-byte aligned");
    DeviceGuard guard(P->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const DevPlan &d = P->dp;
    hipError_t e;
    if ((e = launch_upward_leaf(d, rho, s)) != hipSuccess) return hip_fail(e, "launch upward_leaf");
    if ((e = launch_m2m_upper(d, s)) != hipSuccess) return hip_fail(e, "launch of the upper M2M spans");
    if ((e = launch_am_correction(d, P->dev_KX, P->Pi, P->Pi_part, t, P->am_tiled, s)) != hipSuccess)
        return hip_fail(e, "launch of the angular-momentum correction");
    return OT_FMM_OK;
}

int ot_fmm_adjoint(ot_fmm_plan P, const double *dphi, const double *dg, double *drho, void *hip_stream)
{
    if (!P) return fail(OT_FMM_INVALID_ARGUMENT, "plan is NULL");
    if (!P->has_device) return fail(OT_FMM_NO_DEVICE_STATE, "plan was created with OT_FMM_HOST_ONLY");
    if (!dphi || !dg || !drho) return fail(OT_FMM_INVALID_ARGUMENT, "NULL device pointer");
    if (misaligned(dphi) || misaligned(dg) || misaligned(drho))
        return fail(OT_FMM_INVALID_ARGUMENT, "device pointers must be 8-byte aligned");
    DeviceGuard guard(P->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const DevPlan &d = P->dp;
    hipError_t e;
    Phase total(P, s, OT_FMM_PHASE_TOTAL, 0);
    if (P->amr) {
        const int rc = amr_run(P, 1, dphi, dg, drho, nullptr, s);
        if (rc) return rc;
        total.end();
        if (P->timing.active && P->timing.calls < P->timing.max_calls) P->timing.calls++;
        return OT_FMM_OK;
    }
    {
        Phase ph(P, s, OT_FMM_PHASE_UPWARD_LEAF_ADJ, 1);
        if ((e = launch_upward_leaf_adj(d, dphi, dg, s)) != hipSuccess) return hip_fail(e, "launch upward_leaf_adj");
        ph.end();
    }
    if ((e = tree_passes(P, s)) != hipSuccess) return hip_fail(e, "launch of a tree pass");
    {
        Phase ph(P, s, OT_FMM_PHASE_LEAF_ADJ, 1);
        if ((e = launch_leaf_adj(d, drho, s)) != hipSuccess) return hip_fail(e, "launch leaf_adj");
        ph.end();
    }
    total.end();
    if (P->timing.active && P->timing.calls < P->timing.max_calls) P->timing.calls++;
    return OT_FMM_OK;
}

int ot_fmm_timing_begin(ot_fmm_plan P, int max_calls)
{
    if (!P || max_calls < 1) return fail(OT_FMM_INVALID_ARGUMENT, "plan is NULL or max_calls < 1");
    if (!P->has_device) return fail(OT_FMM_NO_DEVICE_STATE, "plan was created with OT_FMM_HOST_ONLY");
    DeviceGuard guard(P->device);
    TimingState &T = P->timing;
    for (hipEvent_t ev : T.pool) (void)hipEventDestroy(ev);
    T = TimingState{};
    const size_t need = (size_t)max_calls * 2 * OT_FMM_NUM_PHASES;
    T.pool.reserve(need);
    for (size_t i = 0; i < need; ++i) {
        hipEvent_t ev;
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            for (hipEvent_t x : T.pool) (void)hipEventDestroy(x);
            T.pool.clear();
            return hip_fail(e, "hipEventCreate");
        }
        T.pool.push_back(ev);
    }
    T.active = true;
    T.max_calls = max_calls;
    return OT_FMM_OK;
}

int ot_fmm_timing_phases(ot_fmm_plan P, uint32_t phase_mask)
{
    if (!P) return fail(OT_FMM_INVALID_ARGUMENT, "plan is NULL");
    if (!P->timing.active) return fail(OT_FMM_INVALID_ARGUMENT, "no active timing_begin");
    if (phase_mask == 0 || (phase_mask >> OT_FMM_NUM_PHASES) != 0)
        return fail(OT_FMM_INVALID_ARGUMENT, "phase mask selects no phase or an unknown one");
    P->timing.mask = phase_mask;
    return OT_FMM_OK;
}

int ot_fmm_timing_end(ot_fmm_plan P, ot_fmm_timing *out)
{
    if (!P || !out) return fail(OT_FMM_INVALID_ARGUMENT, "plan or out is NULL");
    if (!P->has_device) return fail(OT_FMM_NO_DEVICE_STATE, "plan was created with OT_FMM_HOST_ONLY");
    DeviceGuard guard(P->device);
    TimingState &T = P->timing;
    std::memset(out, 0, sizeof *out);
    out->calls = T.calls;
    int rc = OT_FMM_OK;
    for (const auto &r : T.recs) {
        hipError_t e = hipEventSynchronize(r.b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) { rc = hip_fail(e, "timing events"); break; }
        out->ms[r.phase] += ms;
        out->events[r.phase] += 1;
        out->launches[r.phase] += r.launches;
    }
    for (hipEvent_t ev : T.pool) (void)hipEventDestroy(ev);
    T = TimingState{};
    return rc;
}

int ot_fmm_batch_create(const ot_fmm_plan *plans, int n, int n_streams, ot_fmm_batch *out)
{
    if (!out) return fail(OT_FMM_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    if (!plans || n < 1) return fail(OT_FMM_INVALID_ARGUMENT, "a batch needs at least one plan");
    if (n_streams < 1 || n_streams > BATCH_MAX_STREAMS)
        return fail(OT_FMM_INVALID_ARGUMENT, "n_streams must lie in [1, 16]");
    std::unordered_set<const void *> seen;
    for (int i = 0; i < n; ++i) {
        if (!plans[i]) return fail(OT_FMM_INVALID_ARGUMENT, "NULL plan in a batch");
        if (!plans[i]->has_device) return fail(OT_FMM_NO_DEVICE_STATE, "a plan of the batch was created with OT_FMM_HOST_ONLY");
        if (plans[i]->device != plans[0]->device) return fail(OT_FMM_INVALID_ARGUMENT, "the plans of a batch live on different devices");
        if (!seen.insert(plans[i]).second) return fail(OT_FMM_INVALID_ARGUMENT, "a plan appears twice in a batch");
    }
    ot_fmm_batch B = new (std::nothrow) ot_fmm_batch_s();
    if (!B) return fail(OT_FMM_OUT_OF_MEMORY, "host allocation of the batch failed");
    try {
        B->plans.assign(plans, plans + n);
    } catch (const std::bad_alloc &) {
        delete B;
        return fail(OT_FMM_OUT_OF_MEMORY, "host allocation of the batch failed");
    }
    B->device = plans[0]->device;
    DeviceGuard guard(B->device);
    const int ns = std::min(n, n_streams);
    hipError_t e = hipEventCreateWithFlags(&B->fork, hipEventDisableTiming);
    for (int k = 0; k < ns && e == hipSuccess; ++k) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) break;
        B->streams.push_back(st);
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) break;
        B->join.push_back(ev);
    }
    if (e != hipSuccess) {
        release_batch(B);
        return hip_fail(e, "batch streams and events");
    }
    *out = B;
    return OT_FMM_OK;
}

int ot_fmm_batch_forward(ot_fmm_batch B, const double *const *rho, double *const *phi, double *const *g,
                         void *hip_stream)
{
    int rc = check_batch_args(B, (const void *const *)rho, (const void *const *)phi, (const void *const *)g);
    if (rc) return rc;
    DeviceGuard guard(B->device);
    return batch_enqueue(B, static_cast<hipStream_t>(hip_stream), [&](size_t i, hipStream_t st) {
        return ot_fmm_forward(B->plans[i], rho[i], phi[i], g[i], st);
    });
}

int ot_fmm_batch_adjoint(ot_fmm_batch B, const double *const *dphi, const double *const *dg,
                         double *const *drho, void *hip_stream)
{
    int rc = check_batch_args(B, (const void *const *)dphi, (const void *const *)dg, (const void *const *)drho);
    if (rc) return rc;
    DeviceGuard guard(B->device);
    return batch_enqueue(B, static_cast<hipStream_t>(hip_stream), [&](size_t i, hipStream_t st) {
        return ot_fmm_adjoint(B->plans[i], dphi[i], dg[i], drho[i], st);
    });
}

int ot_fmm_batch_capture_forward(ot_fmm_batch B, const double *const *rho, double *const *phi,
                                 double *const *g, ot_fmm_graph *out)
{
    if (!out) return fail(OT_FMM_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    int rc = check_batch_args(B, (const void *const *)rho, (const void *const *)phi, (const void *const *)g);
    if (rc) return rc;
    DeviceGuard guard(B->device);
    return batch_capture(B, [&](hipStream_t cs) {
        return batch_enqueue(B, cs, [&](size_t i, hipStream_t st) {
            return ot_fmm_forward(B->plans[i], rho[i], phi[i], g[i], st);
        });
    }, out);
}

int ot_fmm_batch_capture_adjoint(ot_fmm_batch B, const double *const *dphi, const double *const *dg,
                                 double *const *drho, ot_fmm_graph *out)
{
    if (!out) return fail(OT_FMM_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    int rc = check_batch_args(B, (const void *const *)dphi, (const void *const *)dg, (const void *const *)drho);
    if (rc) return rc;
    DeviceGuard guard(B->device);
    return batch_capture(B, [&](hipStream_t cs) {
        return batch_enqueue(B, cs, [&](size_t i, hipStream_t st) {
            return ot_fmm_adjoint(B->plans[i], dphi[i], dg[i], drho[i], st);
        });
    }, out);
}

int ot_fmm_graph_launch(ot_fmm_graph G, void *hip_stream)
{
    if (!G || !G->exec) return fail(OT_FMM_INVALID_ARGUMENT, "graph is NULL");
    DeviceGuard guard(G->device);
    hipError_t e = hipGraphLaunch(G->exec, static_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? OT_FMM_OK : hip_fail(e, "hipGraphLaunch");
}

void ot_fmm_graph_destroy(ot_fmm_graph G)
{
    if (!G) return;
    DeviceGuard guard(G->device);
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;
}

void ot_fmm_batch_destroy(ot_fmm_batch B)
{
    if (!B) return;
    DeviceGuard guard(B->device);
    release_batch(B);
}

}  // extern "C"
