// ot_fmm_kernels.hip -- gfx950 kernels of the octree FMM gravity solve.
//
// Expansion algebra (order p = 3, 20 components each, expansions about
// geometric cell centres; the paper, Sec. 4.3, names an FMM on 8^3 sub-grids
// and Sec. 5.5 its same-level stencil, without formulas):
//   scaled moments    Mt_A^a = sum_i m_i (z_A - x_i)^a / a!
//   local coefficients C_A^a = d^a phi at z_A  (Taylor coefficients times a!)
//   e_a(x) = x^a / a!  (component order below)
//   M2M   Mt_P^a += sum_{b <= a} e_{a-b}(z_P - z_c) Mt_c^b
//   M2L   C_A^a  += sum_{|a|+|b| <= 3} D^{a+b}(z_A - z_B) Mt_B^b,
//         D = derivative tensor of K(r) = -G/|r|, evaluated in the reduced
//         form below (16 source and 16 sink components, 70 FMA per pair)
//   L2L   C_c^a  += sum_{|a|+|g| <= 3} e_g(z_c - z_P) C_P^{a+g}
//   L2P   phi = C^0, g = -C^{e_k} at the leaf centre
//   P2P   phi_i += K0(o) m_{i+o}, g_i += K1(o) m_{i+o} for every leaf pair whose
//         parents are near (the far children of near parents included: with
//         point-mass leaves both evaluations are exact and coincide).
// The adjoint runs the same pipeline on dual sources.  Transposed stage by
// stage, the forward chain becomes: L2P^T puts a monopole w and a scaled
// dipole +u at each leaf centre; L2L^T is the scaled M2M; M2L^T is the same
// M2L kernel, since D^{a+b}(-R) = (-1)^{|a|+|b|} D^{a+b}(R) and the factors
// (-1)^{|a|}, (-1)^{|b|} are absorbed into the dual variables (which is why
// the dipole enters as +u); M2M^T is the L2L; P2M^T is the potential-only L2P
// times h^3.  So only the leaf stages differ.
//
// Work mapping: a lane owns one parent cell q of the level and the children
// 2q + b of it, so every stencil offset o = 2P + b' - b is uniform across a
// wave (P from the parent-offset list, b' the source child, b the sink child):
// the tables K(o) and D(o) arrive through scalar loads, and the moments of
// the 64 neighbouring parents are contiguous in memory.
#include <hip/hip_runtime.h>

#include <utility>

#include "ot_fmm_internal.h"

namespace otfmm {

// ------------------------------------------------------------------------
// component order: by total order, then x-power descending, then y-power
// ------------------------------------------------------------------------
struct MIdx { int t, u, v; };
constexpr MIdx kMI[NC] = {
    {0, 0, 0},
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
    {2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2},
    {3, 0, 0}, {2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {1, 1, 1}, {1, 0, 2},
    {0, 3, 0}, {0, 2, 1}, {0, 1, 2}, {0, 0, 3}};

constexpr int comp_of(int t, int u, int v)
{
    for (int k = 0; k < NC; ++k)
        if (kMI[k].t == t && kMI[k].u == u && kMI[k].v == v) return k;
    return -1;
}
constexpr int order_of(int k) { return kMI[k].t + kMI[k].u + kMI[k].v; }

struct Term { int i, j, k; };
template <int N>
struct Terms { Term t[N]; int n; };

// (a, b, a+b) with |a| + |b| <= 3: M2L  C[a] += D[a+b] M[b];
//                                   L2L  C[a] += e[b] Cp[a+b]
constexpr Terms<84> make_sum_terms()
{
    Terms<84> T{};
    T.n = 0;
    for (int a = 0; a < NC; ++a)
        for (int b = 0; b < NC; ++b)
            if (order_of(a) + order_of(b) <= 3)
                T.t[T.n++] = {a, b, comp_of(kMI[a].t + kMI[b].t, kMI[a].u + kMI[b].u, kMI[a].v + kMI[b].v)};
    return T;
}

// (a, b, a-b) with b <= a componentwise: M2M  Mp[a] += e[a-b] Mc[b]
constexpr Terms<84> make_sub_terms()
{
    Terms<84> T{};
    T.n = 0;
    for (int a = 0; a < NC; ++a)
        for (int b = 0; b < NC; ++b)
            if (kMI[b].t <= kMI[a].t && kMI[b].u <= kMI[a].u && kMI[b].v <= kMI[a].v)
                T.t[T.n++] = {a, b, comp_of(kMI[a].t - kMI[b].t, kMI[a].u - kMI[b].u, kMI[a].v - kMI[b].v)};
    return T;
}

// (a, k, a - e_k) with a_k >= 1: dipole source  Mp[a] += u_k e[a - e_k]
constexpr Terms<30> make_dipole_terms()
{
    Terms<30> T{};
    T.n = 0;
    for (int a = 0; a < NC; ++a)
        for (int k = 0; k < 3; ++k) {
            int t = kMI[a].t - (k == 0), u = kMI[a].u - (k == 1), v = kMI[a].v - (k == 2);
            if (t >= 0 && u >= 0 && v >= 0) T.t[T.n++] = {a, k, comp_of(t, u, v)};
        }
    return T;
}

// (k, g, g + e_k) with |g| <= 2: gradient of the local expansion at the leaf
//   dphi/dx_k = sum_g e[g] C[g + e_k]
constexpr Terms<30> make_grad_terms()
{
    Terms<30> T{};
    T.n = 0;
    for (int k = 0; k < 3; ++k)
        for (int g = 0; g < NC; ++g)
            if (order_of(g) <= 2)
                T.t[T.n++] = {k, g, comp_of(kMI[g].t + (k == 0), kMI[g].u + (k == 1), kMI[g].v + (k == 2))};
    return T;
}

static_assert(make_sum_terms().n == 84, "84 terms of total order <= 3");
static_assert(make_sub_terms().n == 84, "84 shift terms");
static_assert(make_dipole_terms().n == 30, "30 dipole terms");
static_assert(make_grad_terms().n == 30, "30 gradient terms");

// ------------------------------------------------------------------------
// Reduced form of the M2L.  K = -G/r is harmonic away from the origin, so its
// derivative tensors are traceless: D^{c+2x} + D^{c+2y} + D^{c+2z} = 0 for
// every c.  A component k with a z-power of 2 or more (zz, xzz, yzz, zzz) is
// then D^k = -D^{k-2z+2x} - D^{k-2z+2y}, two components of lower z-power.
// Substituting this on both sides of the contraction gives:
//   sources: sum_b D^{a+b} Mt^b = sum over the 16 kept b of D^{a+b} R^b with
//            R^c = Mt^c - Mt^{c-2x+2z} [c_x >= 2] - Mt^{c-2y+2z} [c_y >= 2]
//            (formed once per cell when its moments are stored);
//   sinks:   the M2L's share of C^k for the 4 dropped k follows from the kept
//            ones, C^k = -C^{k-2z+2x} - C^{k-2z+2y} (formed once per stored
//            partial sum).
// Kept are the 16 components with z-power <= 1, in the order of kMI.  A pair
// costs 70 FMA over 16 source values instead of 84 over 20; the operator is
// the same up to rounding.
// ------------------------------------------------------------------------
struct RedTab {
    int full[NR];                  // kept component r -> its index in kMI
    int red_of[NC];                // index in kMI -> kept component, or -1
    int sub1[NR], sub2[NR];        // R^r = Mt^full - Mt^sub1 - Mt^sub2 (-1: no term)
    int dep1[NC], dep2[NC];        // dropped k: C^k = -C^dep1 - C^dep2 (kept indices)
};
constexpr RedTab make_red()
{
    RedTab R{};
    int n = 0;
    for (int k = 0; k < NC; ++k) {
        R.red_of[k] = -1;
        if (kMI[k].v < 2) {
            R.full[n] = k;
            R.red_of[k] = n++;
        }
    }
    for (int r = 0; r < NR; ++r) {
        const MIdx c = kMI[R.full[r]];
        R.sub1[r] = c.t >= 2 ? comp_of(c.t - 2, c.u, c.v + 2) : -1;
        R.sub2[r] = c.u >= 2 ? comp_of(c.t, c.u - 2, c.v + 2) : -1;
    }
    for (int k = 0; k < NC; ++k) {
        const MIdx c = kMI[k];
        R.dep1[k] = c.v >= 2 ? R.red_of[comp_of(c.t + 2, c.u, c.v - 2)] : -1;
        R.dep2[k] = c.v >= 2 ? R.red_of[comp_of(c.t, c.u + 2, c.v - 2)] : -1;
    }
    return R;
}
constexpr bool red_ok()
{
    const RedTab R = make_red();
    int n = 0;
    for (int k = 0; k < NC; ++k) n += R.red_of[k] >= 0;
    for (int k = 0; k < NC; ++k)
        if (R.red_of[k] < 0 && (R.dep1[k] < 0 || R.dep2[k] < 0)) return false;
    return n == NR;
}
static_assert(red_ok(), "16 kept components; every dropped one has its two kept partners");

// (a, b, a+b) over kept a, b with |a| + |b| <= 3, ordered by source b: every
// R[b] is consumed right after it is read, by all sinks at once.  The D index
// a+b is in kMI order (the derivative rows keep all 20 components).
constexpr Terms<70> make_red_terms_by_source()
{
    const RedTab R = make_red();
    Terms<70> T{};
    T.n = 0;
    for (int b = 0; b < NR; ++b)
        for (int a = 0; a < NR; ++a) {
            const MIdx x = kMI[R.full[a]], y = kMI[R.full[b]];
            if (x.t + x.u + x.v + y.t + y.u + y.v <= 3) T.t[T.n++] = {a, b, comp_of(x.t + y.t, x.u + y.u, x.v + y.v)};
        }
    return T;
}
static_assert(make_red_terms_by_source().n == 70, "70 terms of the reduced M2L");

constexpr int terms_of_source(int b)      // b: kept component
{
    const int o = order_of(make_red().full[b]);
    return (o == 0) ? 16 : (o == 1) ? 9 : (o == 2) ? 4 : 1;
}
constexpr int source_begin(int b)
{
    int n = 0;
    for (int j = 0; j < b; ++j) n += terms_of_source(j);
    return n;
}
static_assert(source_begin(NR) == 70, "source-major term ranges");

// one sink:  C[a] += D[a+b] m  for the terms of kept source component b
template <int B, int... I>
__device__ __forceinline__ void m2l1_component(double *C, const double *D, double m, std::integer_sequence<int, I...>)
{
    constexpr Terms<70> T = make_red_terms_by_source();
    constexpr int o = source_begin(B);
    ((C[T.t[o + I].i] = fma(D[T.t[o + I].k], m, C[T.t[o + I].i])), ...);
}

template <int K>
__device__ __forceinline__ double comp_or_zero(const double *M)
{
    if constexpr (K >= 0) return M[K];
    else return 0.0;
}

// reduced component R of the full scaled moments M
template <int R>
__device__ __forceinline__ double reduced(const double *M)
{
    constexpr RedTab T = make_red();
    return M[T.full[R]] - comp_or_zero<T.sub1[R]>(M) - comp_or_zero<T.sub2[R]>(M);
}
// The reduced moments are stored in groups of one 16-byte load: FP64 pairs
// [NR/2][8][pp^3] double2, FP32 quads [NR/4][8][pp^3] float4; out points at
// the cell's group 0, groups are cs apart.
template <int... G>
__device__ __forceinline__ void store_reduced(double2 *out, int64_t cs, const double *M, std::integer_sequence<int, G...>)
{
    ((out[G * cs] = make_double2(reduced<2 * G>(M), reduced<2 * G + 1>(M))), ...);
}
template <int... G>
__device__ __forceinline__ void store_reduced(float4 *out, int64_t cs, const double *M, std::integer_sequence<int, G...>)
{
    ((out[G * cs] = make_float4((float)reduced<4 * G>(M), (float)reduced<4 * G + 1>(M), (float)reduced<4 * G + 2>(M),
                                (float)reduced<4 * G + 3>(M))),
     ...);
}

// the 20 local coefficients of an M2L sum from its 16 kept ones
template <int K>
__device__ __forceinline__ double expand_one(const double *Cr)
{
    constexpr RedTab T = make_red();
    if constexpr (T.red_of[K] >= 0) return Cr[T.red_of[K]];
    else return -(Cr[T.dep1[K]] + Cr[T.dep2[K]]);
}
template <int... K>
__device__ __forceinline__ void expand_locals(double *Cf, const double *Cr, std::integer_sequence<int, K...>)
{
    ((Cf[K] = expand_one<K>(Cr)), ...);
}

// Cc[a] += e[g] Cp[a+g]
template <int... I>
__device__ __forceinline__ void l2l_terms(double *Cc, const double *e, const double *Cp,
                                          std::integer_sequence<int, I...>)
{
    constexpr Terms<84> T = make_sum_terms();
    ((Cc[T.t[I].i] = fma(e[T.t[I].j], Cp[T.t[I].k], Cc[T.t[I].i])), ...);
}
__device__ __forceinline__ void l2l_apply(double *Cc, const double *e, const double *Cp)
{
    l2l_terms(Cc, e, Cp, std::make_integer_sequence<int, 84>{});
}

// Mp[a] += e[a-b] Mc[b]
template <int... I>
__device__ __forceinline__ void m2m_terms(double *Mp, const double *e, const double *Mc,
                                          std::integer_sequence<int, I...>)
{
    constexpr Terms<84> T = make_sub_terms();
    ((Mp[T.t[I].i] = fma(e[T.t[I].k], Mc[T.t[I].j], Mp[T.t[I].i])), ...);
}
__device__ __forceinline__ void m2m_apply(double *Mp, const double *e, const double *Mc)
{
    m2m_terms(Mp, e, Mc, std::make_integer_sequence<int, 84>{});
}

// Mp[a] += u[k] e[a - e_k]
template <int... I>
__device__ __forceinline__ void dipole_terms(double *Mp, const double *e, const double *u,
                                             std::integer_sequence<int, I...>)
{
    constexpr Terms<30> T = make_dipole_terms();
    ((Mp[T.t[I].i] = fma(u[T.t[I].j], e[T.t[I].k], Mp[T.t[I].i])), ...);
}
__device__ __forceinline__ void dipole_apply(double *Mp, const double *e, const double *u)
{
    dipole_terms(Mp, e, u, std::make_integer_sequence<int, 30>{});
}

// e_a(x) = x^a / a!
__device__ __forceinline__ void taylor(double x, double y, double z, double *e)
{
    const double x2 = 0.5 * x * x, y2 = 0.5 * y * y, z2 = 0.5 * z * z;
    e[0] = 1.0;
    e[1] = x; e[2] = y; e[3] = z;
    e[4] = x2; e[5] = x * y; e[6] = x * z; e[7] = y2; e[8] = y * z; e[9] = z2;
    e[10] = x2 * x * (1.0 / 3.0); e[11] = x2 * y; e[12] = x2 * z; e[13] = x * y2; e[14] = x * y * z;
    e[15] = x * z2; e[16] = y2 * y * (1.0 / 3.0); e[17] = y2 * z; e[18] = y * z2; e[19] = z2 * z * (1.0 / 3.0);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2);
// renumbering them this way gives each XCD a contiguous run of work items,
// so neighbouring items that share data share an L2.  The grid is a
// multiple of 8.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks)
{
    const int per = (nblocks + 7) >> 3;          // items per XCD
    return (bid & 7) * per + (bid >> 3);
}

// ------------------------------------------------------------------------
// P2M and the first M2M, for one leaf parent Q (a cell of level L-1): stages
// Q's 8 leaf sources into the padded source planes and returns Q's scaled
// moments.  Forward: point masses m = rho h^3.  Adjoint: the dual sources, a
// monopole w and a scaled dipole +u at each leaf centre.
// ------------------------------------------------------------------------
// The same P2M one leaf child at a time (adaptive trees' M2M, a lane per
// child).  LeafQ: where the leaf children of Q sit: their sub-grid's first leaf
// index, Q's padded source-plane index, the children's first coordinates in the
// sub-grid
struct LeafQ {
    int64_t base, padQ, ppL3, N;
    double hh;
    int lx0, ly0, lz0;
};
__device__ __forceinline__ LeafQ leaf_q(const DevPlan &p, int Qx, int Qy, int Qz)
{
    LeafQ q;
    q.padQ = ((int64_t)(Qz + p.hpL) * p.ppL + (Qy + p.hpL)) * p.ppL + (Qx + p.hpL);
    q.base = (int64_t)p.leaf_slot[((int64_t)(Qz >> 2) * p.sL + (Qy >> 2)) * p.sL + (Qx >> 2)] * 512;
    q.lx0 = (2 * Qx) & 7; q.ly0 = (2 * Qy) & 7; q.lz0 = (2 * Qz) & 7;
    q.ppL3 = (int64_t)p.ppL * p.ppL * p.ppL;
    q.N = p.n_leaf_cells;
    q.hh = 0.5 * p.hleaf;
    return q;
}

// leaf child b of Q (its x, y, z bits: b & 1, (b >> 1) & 1, b >> 2): stage its
// sources and add its moments about Q's centre to Mq
template <bool ADJ>
__device__ __forceinline__ void leaf_p2m_child(const DevPlan &p, const double *__restrict__ a0,
                                               const double *__restrict__ a1, const LeafQ &q, int b, double *Mq)
{
    const int64_t ppL3 = q.ppL3, N = q.N;
    const double hh = q.hh;
    const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
    const int64_t idx = q.base + ((q.lz0 + bz) * 8 + (q.ly0 + by)) * 8 + (q.lx0 + bx);
    double e[NC];
    taylor(bx ? -hh : hh, by ? -hh : hh, bz ? -hh : hh, e);    // e(z_Q - z_child)
    // source planes [plane][child pair][parent][2]: one 16-byte load of
    // 64 neighbouring parents reads 1 KB of contiguous memory
    const int64_t sp = ((b >> 1) * ppL3 + q.padQ) * 2 + (b & 1);
    if (!ADJ) {
        const double m = a0[idx] * p.h3;
        p.src[sp] = m;
#pragma unroll
        for (int k = 0; k < NC; ++k) Mq[k] = fma(e[k], m, Mq[k]);
    } else {
        const double w = a0[idx];
        double u[3] = {a1[idx], a1[N + idx], a1[2 * N + idx]};
        p.src[sp] = w;
        p.src[8 * ppL3 + sp] = u[0];
        p.src[16 * ppL3 + sp] = u[1];
        p.src[24 * ppL3 + sp] = u[2];
#pragma unroll
        for (int k = 0; k < NC; ++k) Mq[k] = fma(e[k], w, Mq[k]);
        dipole_apply(Mq, e, u);
    }
}

template <bool ADJ>
__device__ __forceinline__ void leaf_p2m(const DevPlan &p, const double *__restrict__ a0,
                                         const double *__restrict__ a1, int Qx, int Qy, int Qz, double *Mq)
{
    const int64_t ppL3 = (int64_t)p.ppL * p.ppL * p.ppL;
    const int64_t padQ = ((int64_t)(Qz + p.hpL) * p.ppL + (Qy + p.hpL)) * p.ppL + (Qx + p.hpL);
    const int sx = Qx >> 2, sy = Qy >> 2, sz = Qz >> 2;
    const int64_t base = (int64_t)p.leaf_slot[((int64_t)sz * p.sL + sy) * p.sL + sx] * 512;
    const int lx0 = (2 * Qx) & 7, ly0 = (2 * Qy) & 7, lz0 = (2 * Qz) & 7;
    const int64_t N = p.n_leaf_cells;
    const double hh = 0.5 * p.hleaf;
#pragma unroll
    for (int k = 0; k < NC; ++k) Mq[k] = 0.0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
        const int64_t idx = base + ((lz0 + bz) * 8 + (ly0 + by)) * 8 + (lx0 + bx);
        double e[NC];
        taylor(bx ? -hh : hh, by ? -hh : hh, bz ? -hh : hh, e);    // e(z_Q - z_child)
        // source planes [plane][child pair][parent][2]: one 16-byte load of
        // 64 neighbouring parents reads 1 KB of contiguous memory
        const int64_t sp = ((b >> 1) * ppL3 + padQ) * 2 + (b & 1);
        if (!ADJ) {
            const double m = a0[idx] * p.h3;
            p.src[sp] = m;
#pragma unroll
            for (int k = 0; k < NC; ++k) Mq[k] = fma(e[k], m, Mq[k]);
        } else {
            const double w = a0[idx];
            double u[3] = {a1[idx], a1[N + idx], a1[2 * N + idx]};
            p.src[sp] = w;
            p.src[8 * ppL3 + sp] = u[0];
            p.src[16 * ppL3 + sp] = u[1];
            p.src[24 * ppL3 + sp] = u[2];
#pragma unroll
            for (int k = 0; k < NC; ++k) Mq[k] = fma(e[k], w, Mq[k]);
            dipole_apply(Mq, e, u);
        }
    }
}

// store the moments of cell c of level l (kept under its parent c >> 1):
// always the reduced form the M2L reads (FP64, or FP32 for the FP32 M2L),
// and the full moments when an M2M launch reads this level back (full)
__device__ __forceinline__ void store_moments(const DevLevel &D, int cx, int cy, int cz, const double *Mq, bool full,
                                              bool refined = false)
{
    const int bs = (cx & 1) + 2 * (cy & 1) + 4 * (cz & 1);
    const int64_t pp = D.pp, pp3 = pp * pp * pp;
    const int64_t pad = ((int64_t)((cz >> 1) + D.hp) * pp + ((cy >> 1) + D.hp)) * pp + ((cx >> 1) + D.hp);
    const int64_t at = (int64_t)bs * pp3 + pad, cs = 8 * pp3;
    if (full) {
#pragma unroll
        for (int k = 0; k < NC; ++k) D.M[at + k * cs] = Mq[k];
    }
    if (D.M32)
        store_reduced(reinterpret_cast<float4 *>(D.M32) + at, cs, Mq, std::make_integer_sequence<int, NR / 4>{});
    else
        store_reduced(reinterpret_cast<double2 *>(D.Mr) + at, cs, Mq, std::make_integer_sequence<int, NR / 2>{});
    if (refined && D.Mr_ref)        // adaptive trees: the moments of refined cells alone
        store_reduced(reinterpret_cast<double2 *>(D.Mr_ref) + at, cs, Mq, std::make_integer_sequence<int, NR / 2>{});
    if (refined && D.M32_ref)
        store_reduced(reinterpret_cast<float4 *>(D.M32_ref) + at, cs, Mq, std::make_integer_sequence<int, NR / 4>{});
}

// P2M + M2M into level L-1 when no level lies between it and the root
// (depth 0 and 1): lane = one leaf parent Q
template <bool ADJ>
__global__ __launch_bounds__(WG) void k_upward_leaf(const DevPlan p, const double *__restrict__ a0,
                                                    const double *__restrict__ a1)
{
    const int npL = p.npL;
    const int64_t nQ = (int64_t)npL * npL * npL;
    const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (t >= nQ) return;
    const int Qx = (int)(t % npL), Qy = (int)((t / npL) % npL), Qz = (int)(t / ((int64_t)npL * npL));
    double Mq[NC];
    leaf_p2m<ADJ>(p, a0, a1, Qx, Qy, Qz, Mq);
    if (p.L >= 1) store_moments(p.lev[p.L - 1], Qx, Qy, Qz, Mq, p.lev[p.L - 1].M != nullptr);
}

typedef __attribute__((address_space(1))) double gdouble;   // global memory
typedef __attribute__((address_space(1))) void gvoid;
typedef __attribute__((address_space(3))) void lvoid;       // LDS
// s_waitcnt immediate of gfx9 that waits for vmcnt = 0 only (expcnt and
// lgkmcnt at their maxima): the vector memory operations of this wave,
// loads into LDS included, are complete
constexpr int WAIT_VMCNT0 = 0x0F70;

// C[k] += sum over the pieces of cp[(piece * NC + k) * cs], in piece order.
// The loads of U pieces are issued before the first of their adds, so a
// cell with many pieces waits U times less often.
template <int U>
__device__ __forceinline__ void add_pieces(double *C, const double *cp, int64_t cs, int maxp)
{
    int piece = 0;
    for (; piece + U <= maxp; piece += U) {
        double t[U][NC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double *pc = cp + (piece + u) * NC * cs;
            asm volatile("" : "+v"(pc));     // one address per piece, not one induction pointer per component
            const gdouble *g = (const gdouble *)pc;
#pragma unroll
            for (int k = 0; k < NC; ++k) t[u][k] = g[k * cs];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < NC; ++k) C[k] += t[u][k];
    }
    for (; piece < maxp; ++piece) {
        const double *pc = cp + piece * NC * cs;
        asm volatile("" : "+v"(pc));
        const gdouble *g = (const gdouble *)pc;
        double t[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) t[k] = g[k * cs];
#pragma unroll
        for (int k = 0; k < NC; ++k) C[k] += t[k];
    }
}

// ------------------------------------------------------------------------
// Tree passes over a span of levels [t, t + n), n <= 3, in one launch: a
// workgroup owns one cell A of level t and its descendants down to level
// t + n - 1 (1 + 8 + 64 cells).  The cells of the span at depth j are
// numbered by their path from A, three bits (the child index) per level.
// ------------------------------------------------------------------------
__device__ __forceinline__ void span_cell(int ax, int ay, int az, int j, int idx, int &cx, int &cy, int &cz)
{
    cx = ax; cy = ay; cz = az;
    for (int i = j - 1; i >= 0; --i) {
        const int b = (idx >> (3 * i)) & 7;
        cx = 2 * cx + (b & 1);
        cy = 2 * cy + ((b >> 1) & 1);
        cz = 2 * cz + (b >> 2);
    }
}

// M2M, deepest level of the span first.  Thread t = (cell ci, child b) of a
// step shifts the moments of child b to the centre of cell ci; the 8
// children of a cell sit in 8 consecutive lanes and are summed by shuffles
// in a fixed order.  The children of the deepest cells come from memory
// (SRC = 0), or, for the bottom span, are the leaf parents themselves, whose
// moments thread t forms by P2M from the leaf sources and stores (SRC = 1:
// the masses of the forward pass, SRC = 2: the adjoint's dual sources); the
// other steps take their children from the previous step through LDS.
constexpr int M2M_SPAN_WG = 512;

// four waves per SIMD (at most 128 registers): two 8-wave workgroups per CU,
// so the 512 workgroups of depth 4 run in one round
template <int SRC>
__global__ __launch_bounds__(M2M_SPAN_WG) __attribute__((amdgpu_waves_per_eu(4)))
void k_m2m_span(const DevPlan p, const double *__restrict__ a0, const double *__restrict__ a1, int ltop, int nlev)
{
    __shared__ double Ms[2][64][NC];      // moments of the span's cells at depths 1 and 2
    const int n = 8 << ltop;
    const int a = xcd_remap(blockIdx.x, gridDim.x);
    if (a >= n * n * n) return;
    const int ax = a % n, ay = (a / n) % n, az = a / (n * n);
    const int t = threadIdx.x;
    const int b = t & 7, ci = t >> 3;
    for (int j = nlev - 1; j >= 0; --j) {
        const int lv = ltop + j;
        const bool act = ci < (1 << (3 * j));
        int cx, cy, cz;
        span_cell(ax, ay, az, j, ci, cx, cy, cz);
        double Mc[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) Mc[k] = 0.0;
        if (act) {
            if (j == nlev - 1 && SRC >= 1) {
                // the child is a leaf parent: P2M from its leaf sources, stored for the M2L
                const int Qx = 2 * cx + (b & 1), Qy = 2 * cy + ((b >> 1) & 1), Qz = 2 * cz + (b >> 2);
                leaf_p2m<SRC == 2>(p, a0, a1, Qx, Qy, Qz, Mc);
                store_moments(p.lev[lv + 1], Qx, Qy, Qz, Mc, p.lev[lv + 1].M != nullptr);
            } else if (j == nlev - 1) {
                // the children of c are stored under c in level lv + 1
                const DevLevel &Dc = p.lev[lv + 1];
                const int64_t pp = Dc.pp, pp3 = pp * pp * pp;
                const int64_t pad = ((int64_t)(cz + Dc.hp) * pp + (cy + Dc.hp)) * pp + (cx + Dc.hp);
#pragma unroll
                for (int k = 0; k < NC; ++k) Mc[k] = Dc.M[(k * 8 + b) * pp3 + pad];
            } else {
#pragma unroll
                for (int k = 0; k < NC; ++k) Mc[k] = Ms[(j + 1) & 1][ci * 8 + b][k];
            }
        }
        const double hh = 0.5 * p.lev[lv + 1].h;
        double e[NC], Mp[NC];
        taylor((b & 1) ? -hh : hh, ((b >> 1) & 1) ? -hh : hh, (b >> 2) ? -hh : hh, e);   // e(z_c - z_child)
#pragma unroll
        for (int k = 0; k < NC; ++k) Mp[k] = 0.0;
        m2m_apply(Mp, e, Mc);
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            Mp[k] += __shfl_down(Mp[k], 4, 8);
            Mp[k] += __shfl_down(Mp[k], 2, 8);
            Mp[k] += __shfl_down(Mp[k], 1, 8);
        }
        if (act && b == 0) {
            if (j > 0) {
#pragma unroll
                for (int k = 0; k < NC; ++k) Ms[j & 1][ci][k] = Mp[k];
            }
            store_moments(p.lev[lv], cx, cy, cz, Mp, p.lev[lv].M != nullptr);   // full: read by the span above
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------
// M2L
// ------------------------------------------------------------------------
constexpr int M2L_TBP = 2;                       // source children per tile

// M2L over every level below the leaves in one launch.
//
// Exactly one workgroup (8 waves) per resident slot; workgroup g walks its
// run of units (block, P) of one level in order, 8 / M2L_TBP tiles of M2L_TBP
// source children per unit.  Wave w handles sink child b = w of its lane's
// parent, so a lane keeps 16 accumulators (the reduced form) and a wave one
// derivative row (20 scalars): few registers, eight waves per SIMD to hide
// the scalar and LDS latencies.  The tile of reduced source moments (2
// children x 16 components x 64 parents) is loaded once per workgroup,
// straight from global memory into LDS (16 bytes per lane, no registers),
// and read two components per 16-byte LDS read.  It is double-buffered:
// tile k+1 is in flight while tile k is consumed.  Sums stay in registers
// while the block is the same and are stored as a partial sum (piece) when
// it changes.
constexpr int M2L_WG = 512;                       // 8 waves, one per sink child

typedef const __attribute__((address_space(4))) int32_t cint32;

// unit k of a level's list of computed units, stored as block << 9 | parent
// offset.  The list is never written by a kernel; read through the constant
// address space, its entries arrive by scalar loads.
__device__ __forceinline__ void unit_at(const int32_t *list, int k, int &blk, int &i)
{
    const int u = ((const cint32 *)list)[k];
    blk = u >> 9;
    i = u & 511;
}

template <int PAIR, int... I>
__device__ __forceinline__ void m2l1_pair(double *C, const double *D, double2 m, std::integer_sequence<int, I...>)
{
    m2l1_component<2 * PAIR>(C, D, m.x, std::make_integer_sequence<int, terms_of_source(2 * PAIR)>{});
    m2l1_component<2 * PAIR + 1>(C, D, m.y, std::make_integer_sequence<int, terms_of_source(2 * PAIR + 1)>{});
}

// one source child of a tile: rows[pair * 64 + lane] = components
// (2 pair, 2 pair + 1) of the lane's source.  Six LDS reads go out before the
// first product (one wait covers them and the derivative row), the last two
// while the first three component pairs are being consumed: a wave has only
// two waits per pair, and at most six reads (24 registers) in flight.
__device__ __forceinline__ void m2l1_child(double *C, const double *D, const double2 *rows, int lane)
{
    static_assert(NR / 2 == 8, "eight component pairs");
    constexpr std::integer_sequence<int> none{};
    const double2 m0 = rows[0 * 64 + lane], m1 = rows[1 * 64 + lane], m2 = rows[2 * 64 + lane];
    const double2 m3 = rows[3 * 64 + lane], m4 = rows[4 * 64 + lane], m5 = rows[5 * 64 + lane];
    __builtin_amdgcn_sched_barrier(0);
    m2l1_pair<0>(C, D, m0, none);
    m2l1_pair<1>(C, D, m1, none);
    m2l1_pair<2>(C, D, m2, none);
    __builtin_amdgcn_sched_barrier(0);
    const double2 m6 = rows[6 * 64 + lane], m7 = rows[7 * 64 + lane];
    __builtin_amdgcn_sched_barrier(0);
    m2l1_pair<3>(C, D, m3, none);
    m2l1_pair<4>(C, D, m4, none);
    m2l1_pair<5>(C, D, m5, none);
    __builtin_amdgcn_sched_barrier(0);
    m2l1_pair<6>(C, D, m6, none);
    m2l1_pair<7>(C, D, m7, none);
}

__global__ __launch_bounds__(M2L_WG) __attribute__((amdgpu_waves_per_eu(8)))
void k_m2l(const DevPlan p, const double *__restrict__ Dtab, const char4 *__restrict__ near,
           const char4 *__restrict__ cube, const M2LDesc *__restrict__ descs)
{
    // two tile buffers [child of the tile][component pair][lane] -> 2 components,
    // separate arrays so that reads of one and loads into the other are
    // visibly independent
    __shared__ double2 tile0[M2L_TBP][NR / 2][64], tile1[M2L_TBP][NR / 2][64];
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    if (g >= p.n_mdesc) return;
    const M2LDesc d = descs[g];
    const int lev = d.level;
    const DevLevel &D = p.lev[lev];
    const int lane = threadIdx.x & 63;
    const int b = uniform(threadIdx.x >> 6);        // this wave's sink child
    const int r2i = p.r2i;
    const int nP = lev == 0 ? p.n_plist_cube : p.n_plist_near;
    const char4 *__restrict__ plist = lev == 0 ? cube : near;
    const double *__restrict__ Dl = Dtab + (size_t)lev * OFF_N * NC;
    const double2 *__restrict__ Mr = reinterpret_cast<const double2 *>(D.Mr);
    const int np = D.np, pp = D.pp, hp = D.hp;
    const int pp3 = pp * pp * pp, np3 = np * np * np;
    const int lx = lane & (D.bx - 1), ly = (lane / D.bx) & (D.by - 1), lz = lane / (D.bx * D.by);
    auto lane_xyz = [&](int blk, int &qx, int &qy, int &qz) {
        qx = (blk % D.nbx) * D.bx + lx;
        qy = ((blk / D.nbx) % D.nby) * D.by + ly;
        qz = (blk / (D.nbx * D.nby)) * D.bz + lz;
    };
    auto lane_q = [&](int blk) {
        int qx, qy, qz;
        lane_xyz(blk, qx, qy, qz);
        return (qz * np + qy) * np + qx;
    };
    auto lane_mq = [&](int blk) {
        int qx, qy, qz;
        lane_xyz(blk, qx, qy, qz);
        return ((qz + hp) * pp + (qy + hp)) * pp + (qx + hp);
    };
    constexpr int TPP = 8 / M2L_TBP;                // tiles per unit
    constexpr int ROWS = M2L_TBP * NR / 2;          // 16-byte rows of 64 lanes per tile
    static_assert(ROWS % 8 == 0, "each wave loads the same number of rows");
    const int ntiles = d.nvalid * TPP;
    if (ntiles == 0) return;                       // the whole workgroup

    // fetch cursor: block fb, parent offset fi, tile ft.  Wave w loads rows
    // r = w + 8 j of the next tile (component pair r % 8 of tile child r / 8)
    // straight from global memory into LDS, 16 bytes per lane.
    // the run's units are entries vbeg .. vbeg + nvalid - 1 of the level's list
    int fk = d.vbeg, fb, fi, ft = 0;
    unit_at(D.ulist, fk, fb, fi);
    int fmq = lane_mq(fb);
    auto fetch = [&](double2 (*t)[NR / 2][64]) {
        const char4 P = plist[fi];
        const double2 *src = Mr + (fmq + ft * M2L_TBP * pp3 + (P.z * pp + P.y) * pp + P.x);
#pragma unroll
        for (int j = 0; j < ROWS / 8; ++j) {
            const int r = b + 8 * j, i = r / (NR / 2), k = r % (NR / 2);
            __builtin_amdgcn_global_load_lds((gvoid *)(src + (k * 8 + i) * pp3), (lvoid *)&t[i][k][0], 16, 0, 0);
        }
    };
    // the loads of this wave have reached LDS; with the barrier after it,
    // those of every wave
    auto loads_done = [&]() { __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0); };

    // compute cursor; the run's first raw block takes piece piece0, a block
    // that starts inside the run piece 0
    int ck = d.vbeg, cb = fb, ci = fi, ct = 0;
    int piece = (cb == d.ubeg / nP) ? d.piece0 : 0;

    double C[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) C[k] = 0.0;
    auto flush = [&]() {
        double *out = D.Cp + (size_t)piece * NC * 8 * np3 + lane_q(cb);
        double Cf[NC];
        expand_locals(Cf, C, std::make_integer_sequence<int, NC>{});
#pragma unroll
        for (int k = 0; k < NC; ++k) out[(size_t)(k * 8 + b) * np3] = Cf[k];
#pragma unroll
        for (int k = 0; k < NR; ++k) C[k] = 0.0;
    };

    // one tile: start loading the next one into nxt, consume cur
    auto step = [&](int k, double2 (*cur)[NR / 2][64], double2 (*nxt)[NR / 2][64]) {
        if (k + 1 < ntiles) {
            if (++ft == TPP) {
                ft = 0;
                const int ob = fb;
                unit_at(D.ulist, ++fk, fb, fi);
                if (fb != ob) fmq = lane_mq(fb);
            }
            fetch(nxt);
        }
        const char4 P = plist[ci];
        const int bp0 = ct * M2L_TBP;
#pragma unroll
        for (int i = 0; i < M2L_TBP; ++i) {
            const int bp = bp0 + i;
            const int ox = 2 * P.x + (bp & 1) - (b & 1), oy = 2 * P.y + ((bp >> 1) & 1) - ((b >> 1) & 1),
                      oz = 2 * P.z + (bp >> 2) - (b >> 2);
            if (ox * ox + oy * oy + oz * oz <= r2i) continue;       // near: handled one level down
            const double *Dr = Dl + off_index(ox, oy, oz) * NC;
            double Dv[NC];
#pragma unroll
            for (int q = 0; q < NC; ++q) Dv[q] = Dr[q];
            m2l1_child(C, Dv, &cur[i][0][0], lane);
        }
        if (++ct == TPP && k + 1 < ntiles) {
            ct = 0;
            int nb, ni;
            unit_at(D.ulist, ++ck, nb, ni);
            if (nb != cb) {                     // block done in this run: store its piece
                flush();
                piece = 0;
            }
            cb = nb;
            ci = ni;
        }
        loads_done();
        __syncthreads();
    };

    fetch(tile0);
    loads_done();
    __syncthreads();
    for (int k = 0; k < ntiles; k += 2) {
        step(k, tile0, tile1);
        if (k + 1 < ntiles) step(k + 1, tile1, tile0);
    }
    flush();                                    // the run's last block
}

// M2L in FP32 (plan flag OT_FMM_M2L_FP32).  The schedule, the work mapping
// and the partial sums are those of k_m2l; the moments and derivative rows
// are FP32, the LDS tile holds four components per 16-byte read, and the 70
// products of a pair are accumulated in FP32 over one parent offset (the 8
// source children of a unit) and then added to FP64 accumulators, which the
// pieces receive.
template <int B, int... I>
__device__ __forceinline__ void m2l1f_component(float *C, const float *D, float m, std::integer_sequence<int, I...>)
{
    constexpr Terms<70> T = make_red_terms_by_source();
    constexpr int o = source_begin(B);
    ((C[T.t[o + I].i] = fmaf(D[T.t[o + I].k], m, C[T.t[o + I].i])), ...);
}

template <int Q>
__device__ __forceinline__ void m2l1f_quad(float *C, const float *D, float4 m)
{
    m2l1f_component<4 * Q>(C, D, m.x, std::make_integer_sequence<int, terms_of_source(4 * Q)>{});
    m2l1f_component<4 * Q + 1>(C, D, m.y, std::make_integer_sequence<int, terms_of_source(4 * Q + 1)>{});
    m2l1f_component<4 * Q + 2>(C, D, m.z, std::make_integer_sequence<int, terms_of_source(4 * Q + 2)>{});
    m2l1f_component<4 * Q + 3>(C, D, m.w, std::make_integer_sequence<int, terms_of_source(4 * Q + 3)>{});
}

template <int... Q>
__device__ __forceinline__ void m2l1f_child(float *C, const float *D, const float4 *rows, int lane,
                                            std::integer_sequence<int, Q...>)
{
    // rows[q * 64 + lane] = components 4q .. 4q + 3 of the lane's source
    (m2l1f_quad<Q>(C, D, rows[Q * 64 + lane]), ...);
}

constexpr int M2LF_QUADS = M2L_TBP * NR / 4;                  // (child, 4 components) rows per tile
static_assert(M2LF_QUADS == 8, "one quad row per wave");

// one quad row (16 bytes per lane) per wave and tile
static_assert(M2L_TBP * NR / 4 == 8, "one quad row per wave");

// six waves per SIMD (at most 80 registers); eight would spill
__global__ __launch_bounds__(M2L_WG) __attribute__((amdgpu_waves_per_eu(6)))
void k_m2l_f32(const DevPlan p, const float *__restrict__ Dtab32, const char4 *__restrict__ near,
               const char4 *__restrict__ cube, const M2LDesc *__restrict__ descs)
{
    // two tile buffers [child of the tile][component quad][lane] -> 4 components
    __shared__ float4 tile0[M2L_TBP][NR / 4][64], tile1[M2L_TBP][NR / 4][64];
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    if (g >= p.n_mdesc) return;
    const M2LDesc d = descs[g];
    const int lev = d.level;
    const DevLevel &D = p.lev[lev];
    const int lane = threadIdx.x & 63;
    const int b = uniform(threadIdx.x >> 6);        // this wave's sink child
    const int r2i = p.r2i;
    const int nP = lev == 0 ? p.n_plist_cube : p.n_plist_near;
    const char4 *__restrict__ plist = lev == 0 ? cube : near;
    const float *__restrict__ Dl = Dtab32 + (size_t)lev * OFF_N * NC;
    const float4 *__restrict__ M32 = reinterpret_cast<const float4 *>(D.M32);
    const int np = D.np, pp = D.pp, hp = D.hp;
    const int pp3 = pp * pp * pp, np3 = np * np * np;
    const int lx = lane & (D.bx - 1), ly = (lane / D.bx) & (D.by - 1), lz = lane / (D.bx * D.by);
    auto lane_xyz = [&](int blk, int &qx, int &qy, int &qz) {
        qx = (blk % D.nbx) * D.bx + lx;
        qy = ((blk / D.nbx) % D.nby) * D.by + ly;
        qz = (blk / (D.nbx * D.nby)) * D.bz + lz;
    };
    auto lane_q = [&](int blk) {
        int qx, qy, qz;
        lane_xyz(blk, qx, qy, qz);
        return (qz * np + qy) * np + qx;
    };
    auto lane_mq = [&](int blk) {
        int qx, qy, qz;
        lane_xyz(blk, qx, qy, qz);
        return ((qz + hp) * pp + (qy + hp)) * pp + (qx + hp);
    };
    constexpr int TPP = 8 / M2L_TBP;                // tiles per unit
    const int ntiles = d.nvalid * TPP;
    if (ntiles == 0) return;                       // the whole workgroup

    // fetch cursor as in k_m2l; wave w loads quad row w of the next tile
    // (tile child w / 4, reduced components 4 (w % 4) .. + 3) into LDS
    int fk = d.vbeg, fb, fi, ft = 0;               // as in k_m2l
    unit_at(D.ulist, fk, fb, fi);
    int fmq = lane_mq(fb);
    const int ti = b / (NR / 4), tq = b % (NR / 4);
    auto fetch = [&](float4 (*t)[NR / 4][64]) {
        const char4 P = plist[fi];
        const float4 *src = M32 + (fmq + ft * M2L_TBP * pp3 + (P.z * pp + P.y) * pp + P.x);
        __builtin_amdgcn_global_load_lds((gvoid *)(src + (tq * 8 + ti) * pp3), (lvoid *)&t[ti][tq][0], 16, 0, 0);
    };
    auto loads_done = [&]() { __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0); };

    int ck = d.vbeg, cb = fb, ci = fi, ct = 0;
    int piece = (cb == d.ubeg / nP) ? d.piece0 : 0;

    double C[NR];           // FP64 accumulators of the block
    float Cf[NR];           // FP32 sum of the current parent offset
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        C[k] = 0.0;
        Cf[k] = 0.0f;
    }
    auto fold = [&]() {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            C[k] += (double)Cf[k];
            Cf[k] = 0.0f;
        }
    };
    auto flush = [&]() {
        fold();
        double *out = D.Cp + (size_t)piece * NC * 8 * np3 + lane_q(cb);
        double Cx[NC];
        expand_locals(Cx, C, std::make_integer_sequence<int, NC>{});
#pragma unroll
        for (int k = 0; k < NC; ++k) out[(size_t)(k * 8 + b) * np3] = Cx[k];
#pragma unroll
        for (int k = 0; k < NR; ++k) C[k] = 0.0;
    };

    auto step = [&](int k, float4 (*cur)[NR / 4][64], float4 (*nxt)[NR / 4][64]) {
        if (k + 1 < ntiles) {
            if (++ft == TPP) {
                ft = 0;
                const int ob = fb;
                unit_at(D.ulist, ++fk, fb, fi);
                if (fb != ob) fmq = lane_mq(fb);
            }
            fetch(nxt);
        }
        const char4 P = plist[ci];
        const int bp0 = ct * M2L_TBP;
#pragma unroll
        for (int i = 0; i < M2L_TBP; ++i) {
            const int bp = bp0 + i;
            const int ox = 2 * P.x + (bp & 1) - (b & 1), oy = 2 * P.y + ((bp >> 1) & 1) - ((b >> 1) & 1),
                      oz = 2 * P.z + (bp >> 2) - (b >> 2);
            if (ox * ox + oy * oy + oz * oz <= r2i) continue;       // near: handled one level down
            const float *Dr = Dl + off_index(ox, oy, oz) * NC;
            float Dv[NC];
#pragma unroll
            for (int q = 0; q < NC; ++q) Dv[q] = Dr[q];
            m2l1f_child(Cf, Dv, &cur[i][0][0], lane, std::make_integer_sequence<int, NR / 4>{});
        }
        if (++ct == TPP) {
            ct = 0;
            fold();                             // one parent offset done
            if (k + 1 < ntiles) {
                int nb, ni;
                unit_at(D.ulist, ++ck, nb, ni);
                if (nb != cb) {                 // block done in this run: store its piece
                    flush();
                    piece = 0;
                }
                cb = nb;
                ci = ni;
            }
        }
        loads_done();
        __syncthreads();
    };

    fetch(tile0);
    loads_done();
    __syncthreads();
    for (int k = 0; k < ntiles; k += 2) {
        step(k, tile0, tile1);
        if (k + 1 < ntiles) step(k + 1, tile1, tile0);
    }
    flush();                                    // the run's last block
}

// L2L over a span, top level first.  Thread groups: t = 0 the cell A,
// t in [1, 9) its children, t in [9, 73) its grandchildren.  Every thread
// first adds the M2L pieces of its cell (they do not depend on the parents),
// then, level by level, the shift of its parent's final expansion (from
// memory for A, from LDS below it).
constexpr int L2L_SPAN_WG = 128;

__global__ __launch_bounds__(L2L_SPAN_WG) void k_l2l_span(const DevPlan p, int ltop, int nlev)
{
    __shared__ double Cs0[NC], Cs1[8][NC];
    const int n = 8 << ltop;
    const int a = xcd_remap(blockIdx.x, gridDim.x);
    if (a >= n * n * n) return;
    const int ax = a % n, ay = (a / n) % n, az = a / (n * n);
    const int t = threadIdx.x;
    const int j = (t == 0) ? 0 : (t < 9 ? 1 : 2);
    const int ci = (t == 0) ? 0 : (t < 9 ? t - 1 : t - 9);
    const bool act = t < 73 && j < nlev;
    const int lv = ltop + j;
    int cx, cy, cz;
    span_cell(ax, ay, az, j, ci, cx, cy, cz);

    const int bs = (cx & 1) + 2 * (cy & 1) + 4 * (cz & 1);
    double C[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) C[k] = 0.0;
    int64_t np3 = 0, q = 0;
    if (act) {
        const DevLevel &D = p.lev[lv];
        const int64_t np = D.np;
        np3 = np * np * np;
        q = ((int64_t)(cz >> 1) * np + (cy >> 1)) * np + (cx >> 1);
        add_pieces<4>(C, D.Cp + bs * np3 + q, 8 * np3, D.maxp);
    }
    for (int st = 0; st < nlev; ++st) {
        if (act && j == st) {
            double Cp[NC];
            bool shift = true;
            if (st == 0) {
                if (ltop > 0) {          // parent R = c >> 1 of level ltop - 1, final
                    const DevLevel &Dp = p.lev[ltop - 1];
                    const int Rx = cx >> 1, Ry = cy >> 1, Rz = cz >> 1;
                    const int bR = (Rx & 1) + 2 * (Ry & 1) + 4 * (Rz & 1);
                    const int64_t npp = Dp.np, npp3 = npp * npp * npp;
                    const int64_t qR = ((int64_t)(Rz >> 1) * npp + (Ry >> 1)) * npp + (Rx >> 1);
#pragma unroll
                    for (int k = 0; k < NC; ++k) Cp[k] = Dp.C[(k * 8 + bR) * npp3 + qR];
                } else {
                    shift = false;
#pragma unroll
                    for (int k = 0; k < NC; ++k) Cp[k] = 0.0;
                }
            } else if (st == 1) {
#pragma unroll
                for (int k = 0; k < NC; ++k) Cp[k] = Cs0[k];
            } else {
#pragma unroll
                for (int k = 0; k < NC; ++k) Cp[k] = Cs1[ci >> 3][k];
            }
            if (shift) {
                const double hh = 0.5 * p.lev[lv].h;
                double e[NC];
                taylor((cx & 1) ? hh : -hh, (cy & 1) ? hh : -hh, (cz & 1) ? hh : -hh, e);   // e(z_c - z_parent)
                l2l_apply(C, e, Cp);
            }
            if (st == 0 && nlev > 1) {
#pragma unroll
                for (int k = 0; k < NC; ++k) Cs0[k] = C[k];
            } else if (st == 1 && nlev > 2) {
#pragma unroll
                for (int k = 0; k < NC; ++k) Cs1[ci][k] = C[k];
            }
            double *out = p.lev[lv].C;
#pragma unroll
            for (int k = 0; k < NC; ++k) out[(k * 8 + bs) * np3 + q] = C[k];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------
// Leaf pass: local expansion of the leaf parent, L2P, then P2P over the
// leaf stencil.
//
// A wave owns 64 leaf parents Q (lane = Q) and all 8 children of each.
// The local expansion of Q (level L-1) is its M2L pieces plus the shift of
// its parent's, formed in registers; it is evaluated at the 8 children
// first, so it is dead before the pair loop starts.  For a parent offset P
// the 64 child pairs (b', b) use the 27 offsets 2P + e, e = b' - b in
// {-1,0,1}^3; the stream tables hold, per step, those 27 kernel rows, read
// through scalar loads, each serving every pair with that e.  The forward
// pass takes one source plane (the mass) and four accumulators per child;
// the adjoint takes four planes (w, u) and one accumulator, and runs the
// planes one after the other, so the sources in flight at a time are a
// single plane, whose neighbourhood stays in L2.  The sources of the next
// step are loaded while the current ones are consumed.
// ------------------------------------------------------------------------

// octant sign of e_a at child b: along an axis whose bit is 0 the child
// centre lies at -x from its parent
constexpr bool neg_of(int b, int a)
{
    return ((kMI[a].t * (1 - (b & 1)) + kMI[a].u * (1 - ((b >> 1) & 1)) + kMI[a].v * (1 - (b >> 2))) & 1) != 0;
}

// potential of the local expansion C at child B: sum_a e_a C[a]
template <int B, int... A>
__device__ __forceinline__ double l2p_phi(const double *C, const double *em, std::integer_sequence<int, A...>)
{
    double s = 0.0;
    ((s = fma(neg_of(B, A) ? -em[A] : em[A], C[A], s)), ...);
    return s;
}

// gradient at child B: gr[k] += e_g C[g + e_k], |g| <= 2
template <int B, int... I>
__device__ __forceinline__ void l2p_grad(double *gr, const double *C, const double *em,
                                         std::integer_sequence<int, I...>)
{
    constexpr Terms<30> T = make_grad_terms();
    ((gr[T.t[I].i] = fma(neg_of(B, T.t[I].j) ? -em[T.t[I].j] : em[T.t[I].j], C[T.t[I].k], gr[T.t[I].i])), ...);
}

template <bool ADJ, int NA, int... B>
__device__ __forceinline__ void leaf_l2p(double (&acc)[8][NA], const double *C, const double *em,
                                         std::integer_sequence<int, B...>)
{
    ((acc[B][0] = l2p_phi<B>(C, em, std::make_integer_sequence<int, NC>{})), ...);
    if constexpr (!ADJ) {
        auto grad = [&](auto bc) {
            constexpr int b = decltype(bc)::value;
            double gr[3] = {0.0, 0.0, 0.0};
            l2p_grad<b>(gr, C, em, std::make_integer_sequence<int, 30>{});
            acc[b][1 % NA] = -gr[0];
            acc[b][2 % NA] = -gr[1];
            acc[b][3 % NA] = -gr[2];
        };
        (grad(std::integral_constant<int, B>{}), ...);
    }
}

// local expansion of leaf parent Q (a cell of level L-1): its M2L pieces
// plus the L2L shift of its parent's final expansion (level L-2)
__device__ __forceinline__ void leaf_parent_local(const DevPlan &p, int Qx, int Qy, int Qz, double *C)
{
#pragma unroll
    for (int k = 0; k < NC; ++k) C[k] = 0.0;
    if (p.L < 1) return;
    const DevLevel &D = p.lev[p.L - 1];
    const int bQ = (Qx & 1) + 2 * (Qy & 1) + 4 * (Qz & 1);
    const int64_t nq = D.np, nq3 = nq * nq * nq;
    const int64_t q = ((int64_t)(Qz >> 1) * nq + (Qy >> 1)) * nq + (Qx >> 1);
    add_pieces<1>(C, D.Cp + bQ * nq3 + q, 8 * nq3, D.maxp);
    if (p.L < 2) return;
    const DevLevel &Dp = p.lev[p.L - 2];
    const int Rx = Qx >> 1, Ry = Qy >> 1, Rz = Qz >> 1;
    const int bR = (Rx & 1) + 2 * (Ry & 1) + 4 * (Rz & 1);
    const int64_t nr = Dp.np, nr3 = nr * nr * nr;
    const int64_t r = ((int64_t)(Rz >> 1) * nr + (Ry >> 1)) * nr + (Rx >> 1);
    double CR[NC], e[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) CR[k] = Dp.C[(k * 8 + bR) * nr3 + r];
    const double hh = p.hleaf;                  // half the width of a leaf parent
    taylor((Qx & 1) ? hh : -hh, (Qy & 1) ? hh : -hh, (Qz & 1) ? hh : -hh, e);   // e(z_Q - z_R)
    l2l_apply(C, e, CR);
}

// Stencil chunks: the workgroup of block blk has nchunk waves; wave c sums
// the c-th part of the parent-offset list (forward) or of the (plane, offset)
// steps (adjoint) for the same 64 leaf parents, wave 0 also the L2P, and the
// partial sums meet in LDS in the fixed order ((w1 + w2) + ...) + w0.  Small
// trees get more waves this way; a given chunk count gives the same bits on
// every call.
// steps of the P2P loop that wave 0's prologue (the pieces, the L2L from the
// parent and the L2P) is worth: wave 0 takes that many fewer steps (forward
// steps of 256 FMA, adjoint steps of 64)
constexpr int LEAF_LEAD = 4, LEAF_LEAD_ADJ = 16;
template <bool ADJ>
__global__ __launch_bounds__(LEAF_MAX_CHUNKS * 64) void k_leaf(const DevPlan p, const double *__restrict__ Ks,
                                                              const char4 *__restrict__ plist,
                                                              double *__restrict__ out0, double *__restrict__ out1,
                                                              int nchunk)
{
    const int npL = p.npL;
    const Block bs = block_shape(npL, p.leaf_subgrid_blocks);
    const int nbx = npL / bs.bx, nby = npL / bs.by, nbz = npL / bs.bz;
    const int bi = xcd_remap(blockIdx.x, gridDim.x);
    const int blk = p.blist ? (bi < p.nblist ? p.blist[bi] : -1) : bi;
    if (blk < 0 || blk >= nbx * nby * nbz) return;  // the whole workgroup: no barrier is skipped
    const int chunk = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int Qx = (blk % nbx) * bs.bx + lane % bs.bx;
    const int Qy = ((blk / nbx) % nby) * bs.by + (lane / bs.bx) % bs.by;
    const int Qz = (blk / (nbx * nby)) * bs.bz + lane / (bs.bx * bs.by);
    const int64_t pp = p.ppL;
    const int64_t ppL3 = pp * pp * pp;
    // this lane's parent in the source planes [plane][child pair][parent][2]
    const double2 *__restrict__ S =
        reinterpret_cast<const double2 *>(p.src) + ((Qz + p.hpL) * pp + (Qy + p.hpL)) * pp + (Qx + p.hpL);

    constexpr int NA = ADJ ? 1 : 4;     // accumulators per sink child
    double acc[8][NA];
    if (chunk == 0) {
        double C[NC];
        leaf_parent_local(p, Qx, Qy, Qz, C);
        leaf_l2p<ADJ, NA>(acc, C, p.e_leaf, std::make_integer_sequence<int, 8>{});
    } else {
#pragma unroll
        for (int b = 0; b < 8; ++b)
#pragma unroll
            for (int a = 0; a < NA; ++a) acc[b][a] = 0.0;
    }

    // The fetch of the next step is unconditional (the last step re-reads a
    // valid entry): a conditional one would merge the wait counts of both
    // paths and make every step wait for its own prefetch.  A scheduling
    // barrier keeps the loads ahead of the step's arithmetic, and the
    // prefetched values pass through an empty asm after it, so the compiler
    // cannot fold the rotation into a load at the top of the loop.
    const int nP = p.n_plist_leaf;
    if constexpr (!ADJ) {
        double cur[8], nxt[8];
        auto fetch = [&](int pi, double *dst) {
            const char4 P = plist[pi];
            const double2 *src = S + ((int64_t)P.z * pp + P.y) * pp + P.x;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double2 v = src[c * ppL3];
                dst[2 * c] = v.x;
                dst[2 * c + 1] = v.y;
            }
        };
        // wave 0 also forms the local expansion and its L2P: it takes LEAF_LEAD
        // fewer steps, the others share them
        auto pbound = [&](int c) {
            if (c == 0) return 0;
            if (c >= nchunk) return nP;
            const int v = (int)((int64_t)c * (nP + LEAF_LEAD) / nchunk) - LEAF_LEAD;
            return v < 0 ? 0 : v;
        };
        const int p0 = pbound(chunk), p1 = pbound(chunk + 1);
        fetch(p0 < nP ? p0 : nP - 1, cur);
        for (int pi = p0; pi < p1; ++pi) {
            fetch(pi + 1 < p1 ? pi + 1 : pi, nxt);
            __builtin_amdgcn_sched_barrier(0);      // keep the prefetch ahead of the arithmetic
            const double *__restrict__ K = Ks + (size_t)pi * 27 * 4;
#pragma unroll
            for (int e = 0; e < 27; ++e) {
                const int ex = e % 3 - 1, ey = (e / 3) % 3 - 1, ez = e / 9 - 1;
                const double k0 = K[4 * e], k1 = K[4 * e + 1], k2 = K[4 * e + 2], k3 = K[4 * e + 3];
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const int bx = (b & 1) + ex, by = ((b >> 1) & 1) + ey, bz = (b >> 2) + ez;
                    if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
                    const double m = cur[bx + 2 * by + 4 * bz];
                    acc[b][0] = fma(k0, m, acc[b][0]);
                    acc[b][1 % NA] = fma(k1, m, acc[b][1 % NA]);
                    acc[b][2 % NA] = fma(k2, m, acc[b][2 % NA]);
                    acc[b][3 % NA] = fma(k3, m, acc[b][3 % NA]);
                }
            }
#pragma unroll
            for (int bp = 0; bp < 8; ++bp) {
                asm("" : "+v"(nxt[bp]));
                cur[bp] = nxt[bp];
            }
        }
    } else {
        // Steps run over (plane j, list entry i), plane-major, 27 rows of Ks
        // each.  A step has a quarter of the forward's arithmetic, so the
        // sources travel in a ring of four register sets, fetched three
        // steps before use; the loop is unrolled by four (4 nP steps), so the
        // ring needs no register copies.
        auto fetch = [&](int j, int pi, double *dst) {
            const char4 P = plist[pi];
            const double2 *src = S + (int64_t)j * 4 * ppL3 + ((int64_t)P.z * pp + P.y) * pp + P.x;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double2 v = src[c * ppL3];
                dst[2 * c] = v.x;
                dst[2 * c + 1] = v.y;
            }
        };
        // this chunk's steps [s0, s1): multiples of four, as the ring needs
        const int nst = 4 * nP;
        auto bound = [&](int c) {
            if (c == 0) return 0;
            if (c >= nchunk) return nst;
            const int v = ((int)((int64_t)c * (nst + LEAF_LEAD_ADJ) / nchunk) - LEAF_LEAD_ADJ) & ~3;
            return v < 0 ? 0 : v;
        };
        const int s0 = bound(chunk), s1 = bound(chunk + 1);
        int fj = s0 / nP, fi = s0 % nP;  // plane and entry of the next fetch
        auto fetch_next = [&](double *dst) {    // wraps to the start after the last step
            fetch(fj, fi, dst);
            if (++fi == nP) {
                fi = 0;
                fj = (fj == 3) ? 0 : fj + 1;
            }
        };
        auto step = [&](int st, const double *src) {
            const double *__restrict__ K = Ks + (size_t)st * 27;
#pragma unroll
            for (int e = 0; e < 27; ++e) {
                const int ex = e % 3 - 1, ey = (e / 3) % 3 - 1, ez = e / 9 - 1;
                const double k = K[e];
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const int bx = (b & 1) + ex, by = ((b >> 1) & 1) + ey, bz = (b >> 2) + ez;
                    if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
                    acc[b][0] = fma(k, src[bx + 2 * by + 4 * bz], acc[b][0]);
                }
            }
        };
        double r0[8], r1[8], r2[8], r3[8];
        // issue order r0..r3 here as in the loop, so the wait counts agree
        fetch_next(r0);
        __builtin_amdgcn_sched_barrier(0);
        fetch_next(r1);
        __builtin_amdgcn_sched_barrier(0);
        fetch_next(r2);
        __builtin_amdgcn_sched_barrier(0);
        fetch_next(r3);
        __builtin_amdgcn_sched_barrier(0);
        for (int st = s0; st < s1; st += 4) {
            step(st, r0);
            fetch_next(r0);
            __builtin_amdgcn_sched_barrier(0);
            step(st + 1, r1);
            fetch_next(r1);
            __builtin_amdgcn_sched_barrier(0);
            step(st + 2, r2);
            fetch_next(r2);
            __builtin_amdgcn_sched_barrier(0);
            step(st + 3, r3);
            fetch_next(r3);
            __builtin_amdgcn_sched_barrier(0);
            asm volatile("" ::: "memory");      // no folding of the ring into loads at the loop head
        }
    }

    if (nchunk > 1) {
        extern __shared__ double red[];     // [8 * NA][64] running sum of waves 1 .. c
        for (int c = 1; c < nchunk; ++c) {
            if (chunk == c) {
#pragma unroll
                for (int b = 0; b < 8; ++b)
#pragma unroll
                    for (int a = 0; a < NA; ++a) {
                        double *r = &red[(b * NA + a) * 64 + lane];
                        *r = (c == 1) ? acc[b][a] : *r + acc[b][a];
                    }
            }
            __syncthreads();
        }
        if (chunk != 0) return;
#pragma unroll
        for (int b = 0; b < 8; ++b)
#pragma unroll
            for (int a = 0; a < NA; ++a) acc[b][a] += red[(b * NA + a) * 64 + lane];
    }

    const int sgx = Qx >> 2, sgy = Qy >> 2, sgz = Qz >> 2;
    const int32_t slot = p.leaf_slot[((int64_t)sgz * p.sL + sgy) * p.sL + sgx];
    if (slot < 0) return;          // adaptive tree: this parent's children are not leaves of this level
    const int64_t base = (int64_t)slot * 512;
    const int lx0 = (2 * Qx) & 7, ly0 = (2 * Qy) & 7, lz0 = (2 * Qz) & 7;
    const int64_t N = p.n_leaf_cells;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int64_t idx = base + ((lz0 + (b >> 2)) * 8 + (ly0 + ((b >> 1) & 1))) * 8 + (lx0 + (b & 1));
        if constexpr (!ADJ) {
            out0[idx] = acc[b][0];
            out1[idx] = acc[b][1 % NA];
            out1[N + idx] = acc[b][2 % NA];
            out1[2 * N + idx] = acc[b][3 % NA];
        } else {
            out0[idx] = p.h3 * acc[b][0];
        }
    }
}

// ------------------------------------------------------------------------
// Adaptive trees.  Every level keeps the dense arrays of a uniform tree; the
// cells of sub-grids that do not exist stay zero.  A leaf cell of a level
// below the finest one is an M2L source and sink of its level; its near pairs
// are P2P pairs with the leaves of its level, with the children of near
// refined cells (leaves one level finer) and with the leaves near its parent
// (one level coarser).
// ------------------------------------------------------------------------

// cell (x, y, z) of sub-grid `packed` (x | y << 10 | z << 20), k = local index
__device__ __forceinline__ void amr_cell(int32_t packed, int k, int &x, int &y, int &z)
{
    x = 8 * (packed & 1023) + (k & 7);
    y = 8 * ((packed >> 10) & 1023) + ((k >> 3) & 7);
    z = 8 * ((packed >> 20) & 1023) + (k >> 6);
}

// moments of the leaf cells of level p.L (p: that level's view), stored as
// M2L sources: the point mass, or the dual source (a monopole w and a
// dipole u at the cell centre)
template <bool ADJ>
__global__ __launch_bounds__(WG) void k_amr_leaf_moments(const DevPlan p, const int32_t *__restrict__ nodes,
                                                         int n, const double *__restrict__ a0,
                                                         const double *__restrict__ a1)
{
    const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (t >= (int64_t)n * 512) return;
    const int32_t nd = nodes[t >> 9];
    const int k = (int)(t & 511);
    int x, y, z;
    amr_cell(nd, k, x, y, z);
    const int64_t idx = (int64_t)p.leaf_slot[((int64_t)(z >> 3) * p.sL + (y >> 3)) * p.sL + (x >> 3)] * 512 + k;
    double Mq[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) Mq[c] = 0.0;
    if (!ADJ) {
        Mq[0] = a0[idx] * p.h3;
    } else {
        const int64_t N = p.n_leaf_cells;
        double e[NC];
        const double u[3] = {a1[idx], a1[N + idx], a1[2 * N + idx]};
        taylor(0.0, 0.0, 0.0, e);
        Mq[0] = a0[idx];
        dipole_apply(Mq, e, u);
    }
    store_moments(p.lev[p.L], x, y, z, Mq, false);
}

// Sums v over the S lanes l0 + STRIDE j (j < S, S a power of two, l0 < STRIDE)
// with a fixed xor butterfly, for 8 lanes ((v0 + v1) + (v2 + v3)) +
// ((v4 + v5) + (v6 + v7)); every lane of a group ends with the same bits,
// since the partner lane adds the same two values in swapped order.
template <int S, int STRIDE = 1>
__device__ __forceinline__ void lane_sum(double *v)
{
#pragma unroll
    for (int off = STRIDE; off < S * STRIDE; off <<= 1)
#pragma unroll
        for (int k = 0; k < NC; ++k) v[k] += __shfl_xor(v[k], off, 64);
}

// moments of the cells of the n refined sub-grids of level l from their
// children: the M2M of the refined child sub-grid's full moments, or, when the
// child sub-grid is a leaf, the P2M of its leaf cells, whose sources it stages
// for the leaf pass (p is the view of level l + 1).  Eight lanes per cell,
// lane b = child b; their shifted moments are summed by lane_sum<8>.
template <bool ADJ>
__global__ __launch_bounds__(WG) void k_amr_m2m(const DevPlan p, int l, const int32_t *__restrict__ nodes, int n,
                                                const uint8_t *__restrict__ child_type, const double *__restrict__ a0,
                                                const double *__restrict__ a1)
{
    const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (t >= (int64_t)n * 4096) return;          // whole waves: n * 4096 is a multiple of WG
    const int64_t c = t >> 3;
    const int b = (int)(t & 7);
    int x, y, z;
    amr_cell(nodes[c >> 9], (int)(c & 511), x, y, z);
    const int64_t mc = (int64_t)2 << l;                   // sub-grids per axis one level down
    const uint8_t ct = child_type[((int64_t)(z >> 2) * mc + (y >> 2)) * mc + (x >> 2)];
    double Mq[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) Mq[k] = 0.0;
    if (ct == 1) {
        leaf_p2m_child<ADJ>(p, a0, a1, leaf_q(p, x, y, z), b, Mq);
    } else {
        const DevLevel &Dc = p.lev[l + 1];
        const int64_t pp = Dc.pp, pp3 = pp * pp * pp;
        const int64_t pad = ((int64_t)(z + Dc.hp) * pp + (y + Dc.hp)) * pp + (x + Dc.hp);
        const double hh = 0.5 * Dc.h;
        double Mc[NC], e[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) Mc[k] = Dc.M[(k * 8 + b) * pp3 + pad];
        taylor((b & 1) ? -hh : hh, ((b >> 1) & 1) ? -hh : hh, (b >> 2) ? -hh : hh, e);   // e(z_cell - z_child)
        m2m_apply(Mq, e, Mc);
    }
    lane_sum<8>(Mq);
    if (b == 0) store_moments(p.lev[l], x, y, z, Mq, p.lev[l].M != nullptr, true);
}

// final local expansions of the cells of the n refined sub-grids of level l:
// their M2L pieces plus the shift of the parent's.  S lanes per cell: a wave
// holds 64 / S consecutive cells, lane s * 64 / S + i sums pieces s, s + S, ...
// of cell i in order (so that the lanes reading one piece read neighbouring
// cells), and lane_sum adds the S lanes' sums.
template <int S>
__global__ __launch_bounds__(WG) void k_amr_l2l(const DevPlan p, int l, const int32_t *__restrict__ nodes, int n)
{
    constexpr int CPW = 64 / S;                  // cells per wave
    const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (t >= (int64_t)n * 512 * S) return;       // whole waves: n * 512 * S is a multiple of WG
    const int wl = (int)(t & 63);
    const int64_t cell = (t >> 6) * CPW + wl % CPW;
    const int ls = wl / CPW;
    int cx, cy, cz;
    amr_cell(nodes[cell >> 9], (int)(cell & 511), cx, cy, cz);
    const DevLevel &D = p.lev[l];
    const int bs = (cx & 1) + 2 * (cy & 1) + 4 * (cz & 1);
    const int64_t np = D.np, np3 = np * np * np, cs = 8 * np3;
    const int64_t q = ((int64_t)(cz >> 1) * np + (cy >> 1)) * np + (cx >> 1);
    double C[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) C[k] = 0.0;
    const double *cp = D.Cp + bs * np3 + q;
    int piece = ls;
    for (; piece + S < D.maxp; piece += 2 * S) {      // two pieces' loads before their adds
        double t0[NC], t1[NC];
        const double *p0 = cp + piece * NC * cs, *p1 = cp + (piece + S) * NC * cs;
        asm volatile("" : "+v"(p0), "+v"(p1));
        const gdouble *g0 = (const gdouble *)p0, *g1 = (const gdouble *)p1;
#pragma unroll
        for (int k = 0; k < NC; ++k) { t0[k] = g0[k * cs]; t1[k] = g1[k * cs]; }
#pragma unroll
        for (int k = 0; k < NC; ++k) C[k] = (C[k] + t0[k]) + t1[k];
    }
    if (piece < D.maxp) {
        const gdouble *g0 = (const gdouble *)(cp + piece * NC * cs);
#pragma unroll
        for (int k = 0; k < NC; ++k) C[k] += g0[k * cs];
    }
    lane_sum<S, CPW>(C);
    if (l > 0) {
        const DevLevel &Dp = p.lev[l - 1];
        const int Rx = cx >> 1, Ry = cy >> 1, Rz = cz >> 1;
        const int bR = (Rx & 1) + 2 * (Ry & 1) + 4 * (Rz & 1);
        const int64_t npp = Dp.np, npp3 = npp * npp * npp;
        const int64_t qR = ((int64_t)(Rz >> 1) * npp + (Ry >> 1)) * npp + (Rx >> 1);
        double Cp[NC], e[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) Cp[k] = Dp.C[(k * 8 + bR) * npp3 + qR];
        const double hh = 0.5 * D.h;
        taylor((cx & 1) ? hh : -hh, (cy & 1) ? hh : -hh, (cz & 1) ? hh : -hh, e);   // e(z_c - z_parent)
        l2l_apply(C, e, Cp);
    }
    if (ls == 0) {
#pragma unroll
        for (int k = 0; k < NC; ++k) D.C[(k * 8 + bs) * np3 + q] = C[k];
    }
}

// source plane value of cell (x, y, z) of a level whose planes are padded by
// hp parents (pp per axis): plane j, cell stored under its parent
__device__ __forceinline__ int64_t src_index(int x, int y, int z, int hp, int pp, int j)
{
    const int64_t pp3 = (int64_t)pp * pp * pp;
    const int b = (x & 1) + 2 * (y & 1) + 4 * (z & 1);
    const int64_t pad = ((int64_t)((z >> 1) + hp) * pp + ((y >> 1) + hp)) * pp + ((x >> 1) + hp);
    return (int64_t)j * 8 * pp3 + ((b >> 1) * pp3 + pad) * 2 + (b & 1);
}

// What the leaf pass of an adaptive tree's level p.L leaves out (p: that
// level's view), added to the outputs it wrote.  Lane = one parent Q of the
// block, its 8 children the sinks.  Next to refined cells of its level: the
// cell's own M2L expansion from those refined cells, at its centre (potential,
// minus the gradient).  Coarse-fine
// P2P, up: the leaves of level L-1 near Q; down: the children (leaves of
// level L+1) of the refined cells near each child.
// A block's CF_WAVES waves split the loops and the pieces and meet in LDS in
// the fixed order ((w1 + w2) + ...) + w0.
constexpr int CF_WAVES = 8;
template <bool ADJ>
__global__ __launch_bounds__(CF_WAVES * 64) void k_amr_cf(const DevPlan p, double *__restrict__ out0,
                                                         double *__restrict__ out1)
{
    const int npL = p.npL;
    const Block bs = block_shape(npL, p.leaf_subgrid_blocks);
    const int nbx = npL / bs.bx, nby = npL / bs.by;
    if ((int)blockIdx.x >= p.nblist) return;        // the whole workgroup
    const int blk = p.blist[blockIdx.x];
    const int lane = threadIdx.x & 63;
    const int wave = uniform(threadIdx.x >> 6);
    const int Qx = (blk % nbx) * bs.bx + lane % bs.bx;
    const int Qy = ((blk / nbx) % nby) * bs.by + (lane / bs.bx) % bs.by;
    const int Qz = (blk / (nbx * nby)) * bs.bz + lane / (bs.bx * bs.by);
    const int32_t slot = p.leaf_slot[((int64_t)(Qz >> 2) * p.sL + (Qy >> 2)) * p.sL + (Qx >> 2)];
    const bool live = slot >= 0;           // lanes of other sub-grids still meet the barriers
    constexpr int NA = ADJ ? 1 : 4;
    double acc[8][NA];
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
        for (int a = 0; a < NA; ++a) acc[b][a] = 0.0;
    if (live && p.own_Cp) {
        // the pieces of Q's M2L block (as many as the block received) are
        // dealt to the waves (piece k to wave k mod CF_WAVES)
        const int64_t nq = p.lev[p.L].np, nq3 = nq * nq * nq;
        const int64_t q = ((int64_t)Qz * nq + Qy) * nq + Qx;
        const Block mb = block_shape(npL, p.own_subgrid_blocks);
        const int mbx = npL / mb.bx, mby = npL / mb.by;
        const int npc = p.own_np[((Qz / mb.bz) * mby + Qy / mb.by) * mbx + Qx / mb.bx];
        for (int piece = wave; piece < npc; piece += CF_WAVES) {
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const double *cp = p.own_Cp + ((int64_t)piece * NC * 8 + b) * nq3 + q;
                acc[b][0] += cp[0];
                if constexpr (!ADJ) {
                    acc[b][1 % NA] -= cp[1 * 8 * nq3];
                    acc[b][2 % NA] -= cp[2 * 8 * nq3];
                    acc[b][3 % NA] -= cp[3 * 8 * nq3];
                }
            }
        }
    }
    const int nP = p.n_plist_near;
    // the 27 sub-grids around this lane's (at level L): which are refined
    // (children that are finer leaves) and which are missing (a coarser leaf
    // covers them); independent loads, then no load decides a branch below
    const int64_t m = p.sL;
    const int sgx = Qx >> 2, sgy = Qy >> 2, sgz = Qz >> 2;
    uint32_t refined = 0, missing = 0;
    for (int e = 0; e < 27 && live; ++e) {
        const int x = sgx + e % 3 - 1, y = sgy + (e / 3) % 3 - 1, z = sgz + e / 9 - 1;
        if (x < 0 || y < 0 || z < 0 || x >= m || y >= m || z >= m) continue;
        const uint8_t t = p.ntype_L[((int64_t)z * m + y) * m + x];
        refined |= (uint32_t)(t == 2) << e;
        missing |= (uint32_t)(t == 0) << e;
    }
    // one pair: kernel row K (K0, K1) against the planes at src index si
    auto pair = [&](double(&ac)[NA], const double *K, const double *src, int64_t si, int64_t pl) {
        if constexpr (!ADJ) {
            const double m = src[si];
            ac[0] = fma(K[0], m, ac[0]);
            ac[1 % NA] = fma(K[1], m, ac[1 % NA]);
            ac[2 % NA] = fma(K[2], m, ac[2 % NA]);
            ac[3 % NA] = fma(K[3], m, ac[3 % NA]);
        } else {
            // transpose: K0 w - K1 . u
            ac[0] = fma(K[0], src[si], ac[0]);
            ac[0] = fma(-K[1], src[si + pl], ac[0]);
            ac[0] = fma(-K[2], src[si + 2 * pl], ac[0]);
            ac[0] = fma(-K[3], src[si + 3 * pl], ac[0]);
        }
    };
    if (p.src_up && missing) {
        const int64_t pl = 8 * (int64_t)p.pp_up * p.pp_up * p.pp_up;
        for (int i = wave * nP / CF_WAVES; i < (wave + 1) * nP / CF_WAVES; ++i) {
            const char4 P = p.plist_near[i];
            if (P.x == 0 && P.y == 0 && P.z == 0) continue;
            const int64_t si = src_index(Qx + P.x, Qy + P.y, Qz + P.z, p.hp_up, p.pp_up, 0);
#pragma unroll
            for (int b = 0; b < 8; ++b) pair(acc[b], p.Kcf_up + ((int64_t)i * 8 + b) * 4, p.src_up, si, pl);
        }
    }
    if (p.src_dn && refined) {
        // the cells A = 2Q + d, d in [-2, 3]^3, around this lane's 8 children
        // B = 2Q + b hold every near partner; where A is refined, its 8
        // children (leaves one level finer) are loaded once and paired with
        // each child B that A is near to (o = A - B)
        const int64_t pp = p.pp_dn, pp3 = pp * pp * pp;
        const double2 *__restrict__ S2 = reinterpret_cast<const double2 *>(p.src_dn);
        constexpr int NPL = ADJ ? 4 : 1;     // source planes
        for (int d = wave * 216 / CF_WAVES; d < (wave + 1) * 216 / CF_WAVES; ++d) {
            const int dx = d % 6 - 2, dy = (d / 6) % 6 - 2, dz = d / 36 - 2;
            const int Ax = 2 * Qx + dx, Ay = 2 * Qy + dy, Az = 2 * Qz + dz;
            const int e = ((Az >> 3) - sgz + 1) * 9 + ((Ay >> 3) - sgy + 1) * 3 + ((Ax >> 3) - sgx + 1);
            if (Ax < 0 || Ay < 0 || Az < 0 || !((refined >> e) & 1u)) continue;
            const int64_t pad = ((int64_t)(Az + p.hp_dn) * pp + (Ay + p.hp_dn)) * pp + (Ax + p.hp_dn);
            double mc[NPL][8];
#pragma unroll
            for (int j = 0; j < NPL; ++j)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double2 v = S2[(int64_t)j * 4 * pp3 + c * pp3 + pad];
                    mc[j][2 * c] = v.x;
                    mc[j][2 * c + 1] = v.y;
                }
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int ox = dx - (b & 1), oy = dy - ((b >> 1) & 1), oz = dz - (b >> 2);
                const int o2 = ox * ox + oy * oy + oz * oz;
                if (o2 == 0 || o2 > p.r2i) continue;
                const double *K = p.Kcf_dn + (int64_t)(((oz + 3) * 7 + (oy + 3)) * 7 + (ox + 3)) * 32;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const double *k = K + 4 * c;
                    if constexpr (!ADJ) {
                        acc[b][0] = fma(k[0], mc[0][c], acc[b][0]);
                        acc[b][1 % NA] = fma(k[1], mc[0][c], acc[b][1 % NA]);
                        acc[b][2 % NA] = fma(k[2], mc[0][c], acc[b][2 % NA]);
                        acc[b][3 % NA] = fma(k[3], mc[0][c], acc[b][3 % NA]);
                    } else {
                        acc[b][0] = fma(k[0], mc[0][c], acc[b][0]);
                        acc[b][0] = fma(-k[1], mc[NPL > 1 ? 1 : 0][c], acc[b][0]);
                        acc[b][0] = fma(-k[2], mc[NPL > 2 ? 2 : 0][c], acc[b][0]);
                        acc[b][0] = fma(-k[3], mc[NPL > 3 ? 3 : 0][c], acc[b][0]);
                    }
                }
            }
        }
    }
    __shared__ double red[8 * NA][64];      // running sum of waves 1 .. c
    for (int c = 1; c < CF_WAVES; ++c) {
        if (wave == c) {
#pragma unroll
            for (int b = 0; b < 8; ++b)
#pragma unroll
                for (int a = 0; a < NA; ++a) red[b * NA + a][lane] = (c == 1) ? acc[b][a] : red[b * NA + a][lane] + acc[b][a];
        }
        __syncthreads();
    }
    if (wave != 0 || !live) return;
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
        for (int a = 0; a < NA; ++a) acc[b][a] += red[b * NA + a][lane];
    const int64_t base = (int64_t)slot * 512;
    const int lx0 = (2 * Qx) & 7, ly0 = (2 * Qy) & 7, lz0 = (2 * Qz) & 7;
    const int64_t N = p.n_leaf_cells;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int64_t idx = base + ((lz0 + (b >> 2)) * 8 + (ly0 + ((b >> 1) & 1))) * 8 + (lx0 + (b & 1));
        if constexpr (!ADJ) {
            out0[idx] += acc[b][0];
            out1[idx] += acc[b][1 % NA];
            out1[N + idx] += acc[b][2 % NA];
            out1[2 * N + idx] += acc[b][3 % NA];
        } else {
            out0[idx] += p.h3 * acc[b][0];
        }
    }
}

// ------------------------------------------------------------------------
// Angular-momentum correction.  For an M2L pair (A <- B), R = z_A - z_B, the
// truncated pair energy depends on the expansion centres through its
// boundary term of total order p + 1 = 4; the correction is the spin torque
// per unit mass t at each leaf cell x_i:
//   t_i,j = sum over i's ancestors A and their M2L partners B of
//           sum_a (x_i - z_A)^a / a! Pi_A^a_j,
//   Pi_A^a_j = sum_B sum_{|a|+|b|=3} KX_j^(a+b)(R) Mt_B^b,
//   KX_j^c = -1/2 (R x K^(c+e))_j = -1/2 eps_jkl R_k K^(c+e_l),
// with Mt the scaled moments sum m (z - x)^b / b! (which carry the sign and
// factorial of the source side) and K = -G/r.  sum_i m_i (x_i x g_i + t_i)
// then vanishes exactly.
// ------------------------------------------------------------------------
struct AMTerm { int a, b, c; };      // sink order a, source order b, c = a + b (total order 3)
struct AMTerms { AMTerm t[56]; int n; };
constexpr AMTerms make_am_terms()
{
    AMTerms T{};
    T.n = 0;
    for (int a = 0; a < NC; ++a)
        for (int b = 0; b < NC; ++b)
            if (order_of(a) + order_of(b) == 3)
                T.t[T.n++] = {a, b, comp_of(kMI[a].t + kMI[b].t, kMI[a].u + kMI[b].u, kMI[a].v + kMI[b].v)};
    return T;
}
static_assert(make_am_terms().n == 56, "56 (a, b) pairs of total order 3");

// Pi of the cells of level l, all three components.  WIDE = false: one
// thread per cell.  WIDE = true (levels with few cells): one wave per cell,
// whose lanes split the partner list; the partial sums meet by shuffles in a
// fixed order.
template <bool WIDE>
__global__ __launch_bounds__(WG) void k_am_pi(const DevPlan p, int l, const double *__restrict__ KX,
                                              double *__restrict__ Pi)
{
    const DevLevel &D = p.lev[l];
    const int n = 2 * D.np;
    const int64_t t = WIDE ? (int64_t)blockIdx.x : (int64_t)blockIdx.x * WG + threadIdx.x;
    if (t >= (int64_t)n * n * n) return;           // WIDE: the whole wave
    const int cx = (int)(t % n), cy = (int)((t / n) % n), cz = (int)(t / ((int64_t)n * n));
    const int b = (cx & 1) + 2 * (cy & 1) + 4 * (cz & 1);
    const int nP = l == 0 ? p.n_plist_cube : p.n_plist_near;
    const char4 *plist = l == 0 ? p.plist_cube : p.plist_near;
    const int64_t pp = D.pp, pp3 = pp * pp * pp, np = D.np, np3 = np * np * np;
    const double *KXl = KX + (int64_t)l * OFF_N * 30;
    double P3[3][NC];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int a = 0; a < NC; ++a) P3[j][a] = 0.0;
    constexpr AMTerms T = make_am_terms();
    const int k0 = WIDE ? (int)threadIdx.x : 0, dk = WIDE ? 64 : 1;
    for (int k = k0; k < nP * 8; k += dk) {
        const char4 P = plist[k >> 3];
        const int bp = k & 7;
        const int ox = 2 * P.x + (bp & 1) - (cx & 1), oy = 2 * P.y + ((bp >> 1) & 1) - (cy & 1),
                  oz = 2 * P.z + (bp >> 2) - (cz & 1);
        if (ox * ox + oy * oy + oz * oz <= p.r2i) continue;          // near: one level down
        const int64_t pad = ((int64_t)((cz >> 1) + P.z + D.hp) * pp + ((cy >> 1) + P.y + D.hp)) * pp +
                            ((cx >> 1) + P.x + D.hp);
        double M[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) M[q] = D.M[(q * 8 + bp) * pp3 + pad];
        const double *K = KXl + (int64_t)off_index(ox, oy, oz) * 30;   // [10 order-3 components][3]
#pragma unroll
        for (int q = 0; q < 56; ++q)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                P3[j][T.t[q].a] = fma(K[3 * (T.t[q].c - 10) + j], M[T.t[q].b], P3[j][T.t[q].a]);
    }
    if constexpr (WIDE) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int a = 0; a < NC; ++a)
                for (int o = 32; o >= 1; o >>= 1) P3[j][a] += __shfl_down(P3[j][a], o, 64);
        if (threadIdx.x != 0) return;
    }
    const int64_t q = ((int64_t)(cz >> 1) * np + (cy >> 1)) * np + (cx >> 1);
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int a = 0; a < NC; ++a) Pi[((int64_t)(j * NC + a) * 8 + b) * np3 + q] = P3[j][a];
}

// Pi of the cells of the deeper levels, organised like the M2L: a workgroup
// of 8 waves owns a block of 64 parents (lane = parent) and wave w its sink
// child w.  For each parent offset P the moments of the 8 source children of
// the 64 parents Q + P are staged once in LDS (wave w loads child w's, one
// offset ahead) for all 8 waves, and the kernel row of a (P, b') pair, which
// depends only on the offset 2P + b' - w, is the same for the whole wave.
constexpr int AM_WG = 512;
// NBUF = 2: two staging buffers (twice the LDS), used by alternate offsets,
// so one barrier per offset suffices: a wave that stores into a buffer has
// passed the barrier that every wave reaches only after its products from
// that buffer two offsets before.
template <int NBUF>
__global__ __launch_bounds__(AM_WG) void k_am_pi_tile(const DevPlan p, int l, const double *__restrict__ KX,
                                                      double *__restrict__ Pi, int split,
                                                      const double *__restrict__ Pup)
{
    extern __shared__ double tiles[];                  // NBUF x [8 source children][NC][64]
    const DevLevel &D = p.lev[l];
    const int np = D.np;
    const Block bs = block_shape(np);
    const int nbx = np / bs.bx, nby = np / bs.by, nbz = np / bs.bz;
    // split > 1: workgroup = (block, part), the part's offsets i0 .. i1 - 1,
    // its sums written to partial buffer `part` (Pi then holds split buffers)
    const int blk = blockIdx.x / split, part = blockIdx.x % split;
    if (blk >= nbx * nby * nbz) return;               // the whole workgroup
    const int lane = threadIdx.x & 63;
    const int w = uniform(threadIdx.x >> 6);           // sink child, and the source child this wave stages
    const int Qx = (blk % nbx) * bs.bx + lane % bs.bx;
    const int Qy = ((blk / nbx) % nby) * bs.by + (lane / bs.bx) % bs.by;
    const int Qz = (blk / (nbx * nby)) * bs.bz + lane / (bs.bx * bs.by);
    const int nP = l == 0 ? p.n_plist_cube : p.n_plist_near;      // level 0: the whole root cube
    const char4 *plist = l == 0 ? p.plist_cube : p.plist_near;
    const int64_t pp = D.pp, pp3 = pp * pp * pp, np3 = (int64_t)np * np * np;
    const double *KXl = KX + (int64_t)l * OFF_N * 30;
    double P3[3][NC];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int a = 0; a < NC; ++a) P3[j][a] = 0.0;
    constexpr AMTerms T = make_am_terms();
    // the moments of offset i + 1 are loaded into registers while offset i's
    // products run, and stored to LDS at the top of the next step
    double nx[NC];
    auto load = [&](int i) {
        const char4 P = plist[i];
        const int64_t pad = ((int64_t)(Qz + P.z + D.hp) * pp + (Qy + P.y + D.hp)) * pp + (Qx + P.x + D.hp);
#pragma unroll
        for (int c = 0; c < NC; ++c) nx[c] = D.M[(c * 8 + w) * pp3 + pad];
    };
    const int i0 = part * nP / split, i1 = (part + 1) * nP / split;
    load(i0);
    for (int i = i0; i < i1; ++i) {
        const char4 P = plist[i];
        double *tile = tiles + (NBUF == 2 ? ((i - i0) & 1) * (8 * NC * 64) : 0);
#pragma unroll
        for (int c = 0; c < NC; ++c) tile[(w * NC + c) * 64 + lane] = nx[c];
        __syncthreads();
        if (i + 1 < i1) load(i + 1);
        for (int bp = 0; bp < 8; ++bp) {
            const int ox = 2 * P.x + (bp & 1) - (w & 1), oy = 2 * P.y + ((bp >> 1) & 1) - ((w >> 1) & 1),
                      oz = 2 * P.z + (bp >> 2) - (w >> 2);
            if (ox * ox + oy * oy + oz * oz <= p.r2i) continue;     // near (wave-uniform): one level down
            const double *K = KXl + (int64_t)off_index(ox, oy, oz) * 30;
            double M[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) M[c] = tile[(bp * NC + c) * 64 + lane];
#pragma unroll
            for (int q = 0; q < 56; ++q)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    P3[j][T.t[q].a] = fma(K[3 * (T.t[q].c - 10) + j], M[T.t[q].b], P3[j][T.t[q].a]);
        }
        if (NBUF == 1) __syncthreads();
    }
    if (Pup) {
        // split == 1, l > 0: fold in the parent's Pi (cell 2Q + w's parent is
        // Q), as k_am_down does
        const int bR = (Qx & 1) + 2 * (Qy & 1) + 4 * (Qz & 1);
        const int64_t npp = p.lev[l - 1].np, npp3 = npp * npp * npp;
        const int64_t qR = ((int64_t)(Qz >> 1) * npp + (Qy >> 1)) * npp + (Qx >> 1);
        double e[NC];
        const double hh = 0.5 * D.h;
        taylor((w & 1) ? hh : -hh, ((w >> 1) & 1) ? hh : -hh, (w >> 2) ? hh : -hh, e);   // e(z_c - z_Q)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double Cp[NC];
#pragma unroll
            for (int a = 0; a < NC; ++a) Cp[a] = Pup[((int64_t)(j * NC + a) * 8 + bR) * npp3 + qR];
            l2l_apply(P3[j], e, Cp);
        }
    }
    const int64_t q = ((int64_t)Qz * np + Qy) * np + Qx;
    double *out = Pi + (int64_t)part * 3 * NC * 8 * np3;
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int a = 0; a < NC; ++a) out[((int64_t)(j * NC + a) * 8 + w) * np3 + q] = P3[j][a];
}

// Pi[e] = the split parts' sums of element e, added in part order
__global__ __launch_bounds__(WG) void k_am_sum(const double *__restrict__ parts, int split, int64_t n,
                                               double *__restrict__ Pi)
{
    const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (t >= n) return;
    double s = parts[t];
#pragma unroll 8
    for (int k = 1; k < split; ++k) s += parts[k * n + t];
    Pi[t] = s;
}

// Pi of level l gains its parent's, re-expanded about the cell's centre (the
// L2L shift of each of the 3 components), so that the Pi of level L-1 holds
// the whole sum over the ancestors.  One thread per cell of level l.
__global__ __launch_bounds__(WG) void k_am_down(const DevPlan p, int l, const double *__restrict__ Pup,
                                                double *__restrict__ Pi)
{
    const DevLevel &D = p.lev[l], &Dp = p.lev[l - 1];
    const int n = 2 * D.np;
    const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (t >= (int64_t)n * n * n) return;
    const int cx = (int)(t % n), cy = (int)((t / n) % n), cz = (int)(t / ((int64_t)n * n));
    const int b = (cx & 1) + 2 * (cy & 1) + 4 * (cz & 1);
    const int64_t np = D.np, np3 = np * np * np;
    const int64_t q = ((int64_t)(cz >> 1) * np + (cy >> 1)) * np + (cx >> 1);
    const int Rx = cx >> 1, Ry = cy >> 1, Rz = cz >> 1;
    const int bR = (Rx & 1) + 2 * (Ry & 1) + 4 * (Rz & 1);
    const int64_t npp = Dp.np, npp3 = npp * npp * npp;
    const int64_t qR = ((int64_t)(Rz >> 1) * npp + (Ry >> 1)) * npp + (Rx >> 1);
    double e[NC];
    const double hh = 0.5 * D.h;
    taylor((cx & 1) ? hh : -hh, (cy & 1) ? hh : -hh, (cz & 1) ? hh : -hh, e);   // e(z_c - z_parent)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double C[NC], Cp[NC];
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            C[a] = Pi[((int64_t)(j * NC + a) * 8 + b) * np3 + q];
            Cp[a] = Pup[((int64_t)(j * NC + a) * 8 + bR) * npp3 + qR];
        }
        l2l_apply(C, e, Cp);
#pragma unroll
        for (int a = 0; a < NC; ++a) Pi[((int64_t)(j * NC + a) * 8 + b) * np3 + q] = C[a];
    }
}

// t at every leaf cell: the Pi of its level-(L-1) ancestor, which holds the
// shifted sum over all its ancestors, evaluated at the cell centre.  A
// workgroup takes an 8 x 8 x 4 brick of leaf cells, a wave one 8 x 8 layer of
// it (one sub-grid's).
__global__ __launch_bounds__(WG) void k_am_leaf(const DevPlan p, const double *__restrict__ Pi,
                                                double *__restrict__ tout)
{
    static_assert(WG == 256, "an 8 x 8 x 4 brick per workgroup");
    const int n = 8 << p.L;
    const int nbx = n / 8, nby = n / 8;
    const int brick = blockIdx.x;
    if (brick >= nbx * nby * (n / 4)) return;
    const int cx = (brick % nbx) * 8 + (threadIdx.x & 7), cy = ((brick / nbx) % nby) * 8 + ((threadIdx.x >> 3) & 7),
              cz = (brick / (nbx * nby)) * 4 + (threadIdx.x >> 6);
    double acc[3] = {0.0, 0.0, 0.0};
    if (p.L > 0) {
        const int l = p.L - 1;
        const int ax = cx >> 1, ay = cy >> 1, az = cz >> 1;
        const DevLevel &D = p.lev[l];
        // leaf centre minus the ancestor's centre
        const double x = (cx + 0.5) * p.hleaf - (ax + 0.5) * D.h, y = (cy + 0.5) * p.hleaf - (ay + 0.5) * D.h,
                     z = (cz + 0.5) * p.hleaf - (az + 0.5) * D.h;
        double e[NC];
        taylor(x, y, z, e);
        const int64_t np = D.np, np3 = np * np * np;
        const int64_t q = ((int64_t)(az >> 1) * np + (ay >> 1)) * np + (ax >> 1);
        const int b = (ax & 1) + 2 * (ay & 1) + 4 * (az & 1);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int a = 0; a < NC; ++a) acc[j] = fma(e[a], Pi[((int64_t)(j * NC + a) * 8 + b) * np3 + q], acc[j]);
    }
    const int64_t slot = p.leaf_slot[((int64_t)(cz >> 3) * p.sL + (cy >> 3)) * p.sL + (cx >> 3)];
    const int64_t idx = slot * 512 + ((cz & 7) * 8 + (cy & 7)) * 8 + (cx & 7);
    const int64_t N = p.n_leaf_cells;
    tout[idx] = acc[0];
    tout[N + idx] = acc[1];
    tout[2 * N + idx] = acc[2];
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
static inline unsigned grid_for(int64_t n) { return (unsigned)((n + WG - 1) / WG); }
static inline unsigned grid_x8(int64_t n) { return (unsigned)((n + 7) / 8 * 8); }

// upward pass up to the bottom M2M span: P2M into level L-1 fused with the
// bottom span (src 1: forward, 2: adjoint).  Depths 0 and 1 have no span and
// run the P2M alone.
static hipError_t launch_upward_leaf(const DevPlan &p, int src, const double *a0, const double *a1, hipStream_t s)
{
    const int last = p.n_span - 1;
    const int64_t nq = (int64_t)p.npL * p.npL * p.npL;
    if (last < 0) {
        if (src == 1)
            hipLaunchKernelGGL(k_upward_leaf<false>, dim3(grid_for(nq)), dim3(WG), 0, s, p, a0, a1);
        else
            hipLaunchKernelGGL(k_upward_leaf<true>, dim3(grid_for(nq)), dim3(WG), 0, s, p, a0, a1);
        return hipGetLastError();
    }
    const int t = p.span_top[last], nl = p.span_n[last];
    const int64_t n = 8 << t;
    const dim3 grid(grid_x8(n * n * n)), block(nl == 3 ? M2M_SPAN_WG : 64);
    if (src == 1)
        hipLaunchKernelGGL(k_m2m_span<1>, grid, block, 0, s, p, a0, a1, t, nl);
    else
        hipLaunchKernelGGL(k_m2m_span<2>, grid, block, 0, s, p, a0, a1, t, nl);
    return hipGetLastError();
}

hipError_t launch_upward_leaf(const DevPlan &p, const double *rho, hipStream_t s)
{
    return launch_upward_leaf(p, 1, rho, nullptr, s);
}

hipError_t launch_upward_leaf_adj(const DevPlan &p, const double *w, const double *u, hipStream_t s)
{
    return launch_upward_leaf(p, 2, w, u, s);
}

// the M2M spans above the bottom one, deepest first
hipError_t launch_m2m_upper(const DevPlan &p, hipStream_t s)
{
    for (int i = p.n_span - 2; i >= 0; --i) {
        const int t = p.span_top[i], nl = p.span_n[i];
        const int64_t n = 8 << t;
        hipLaunchKernelGGL(k_m2m_span<0>, dim3(grid_x8(n * n * n)), dim3(nl == 3 ? M2M_SPAN_WG : 64), 0, s, p,
                           nullptr, nullptr, t, nl);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_m2l(const DevPlan &p, hipStream_t s)
{
    if (p.n_mdesc == 0) return hipSuccess;
    const unsigned grid = (unsigned)(((p.n_mdesc + 7) / 8) * 8);     // whole rounds over the 8 XCDs
    if (p.m2l_fp32)
        hipLaunchKernelGGL(k_m2l_f32, dim3(grid), dim3(M2L_WG), 0, s, p, p.Dtab32, p.plist_near, p.plist_cube,
                           p.mdesc);
    else
        hipLaunchKernelGGL(k_m2l, dim3(grid), dim3(M2L_WG), 0, s, p, p.Dtab, p.plist_near, p.plist_cube, p.mdesc);
    return hipGetLastError();
}

hipError_t m2l_blocks_per_cu(int fp32, int *n)
{
    if (fp32) return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_m2l_f32, M2L_WG, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_m2l, M2L_WG, 0);
}

hipError_t launch_l2l_span(const DevPlan &p, int i, hipStream_t s)
{
    const int t = p.span_top[i], nl = p.span_n[i];
    const int64_t n = 8 << t;
    hipLaunchKernelGGL(k_l2l_span, dim3(grid_x8(n * n * n)), dim3(nl == 3 ? L2L_SPAN_WG : 64), 0, s, p, t, nl);
    return hipGetLastError();
}

// one workgroup of nchunk waves per block of 64 leaf parents
hipError_t launch_leaf_chunks(const DevPlan &p, int adj, int nchunk, double *out0, double *out1, hipStream_t s)
{
    if (nchunk < 1 || nchunk > LEAF_MAX_CHUNKS) return hipErrorInvalidValue;
    const Block bs = block_shape(p.npL, p.leaf_subgrid_blocks);
    const int64_t nblk = p.blist ? (int64_t)p.nblist : ((int64_t)p.npL / bs.bx) * (p.npL / bs.by) * (p.npL / bs.bz);
    if (nblk == 0) return hipSuccess;
    const unsigned grid = (unsigned)((nblk + 7) / 8 * 8);               // whole rounds over the 8 XCDs
    const size_t lds = nchunk > 1 ? (size_t)8 * (adj ? 1 : 4) * 64 * sizeof(double) : 0;
    if (adj)
        hipLaunchKernelGGL(k_leaf<true>, dim3(grid), dim3(64 * nchunk), lds, s, p, p.Ksa, p.plist_leaf, out0,
                           nullptr, nchunk);
    else
        hipLaunchKernelGGL(k_leaf<false>, dim3(grid), dim3(64 * nchunk), lds, s, p, p.Kst, p.plist_leaf, out0,
                           out1, nchunk);
    return hipGetLastError();
}

hipError_t launch_leaf(const DevPlan &p, double *phi, double *g, hipStream_t s)
{
    return launch_leaf_chunks(p, 0, p.leaf_chunks[0], phi, g, s);
}

hipError_t launch_leaf_adj(const DevPlan &p, double *drho, hipStream_t s)
{
    return launch_leaf_chunks(p, 1, p.leaf_chunks[1], drho, nullptr, s);
}

}  // namespace otfmm

namespace otfmm {

hipError_t launch_amr_leaf_moments(const DevPlan &v, int adj, const int32_t *nodes, int n, const double *a0,
                                   const double *a1, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const dim3 grid(grid_for((int64_t)n * 512));
    if (adj)
        hipLaunchKernelGGL(k_amr_leaf_moments<true>, grid, dim3(WG), 0, s, v, nodes, n, a0, a1);
    else
        hipLaunchKernelGGL(k_amr_leaf_moments<false>, grid, dim3(WG), 0, s, v, nodes, n, a0, a1);
    return hipGetLastError();
}

hipError_t launch_amr_m2m(const DevPlan &v, int adj, int l, const int32_t *nodes, int n, const uint8_t *child_type,
                          const double *a0, const double *a1, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const dim3 grid(grid_for((int64_t)n * 4096));
    if (adj)
        hipLaunchKernelGGL(k_amr_m2m<true>, grid, dim3(WG), 0, s, v, l, nodes, n, child_type, a0, a1);
    else
        hipLaunchKernelGGL(k_amr_m2m<false>, grid, dim3(WG), 0, s, v, l, nodes, n, child_type, a0, a1);
    return hipGetLastError();
}

hipError_t launch_amr_l2l(const DevPlan &p, int l, const int32_t *nodes, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    // lanes per cell from the level's pieces per cell: 8 (at most two pieces a
    // lane up to 16 pieces; these launches are short and wait on memory), 32
    // beyond
    const int maxp = p.lev[l].maxp;
    const int64_t cells = (int64_t)n * 512;
    if (maxp > 16)
        hipLaunchKernelGGL(k_amr_l2l<32>, dim3(grid_for(cells * 32)), dim3(WG), 0, s, p, l, nodes, n);
    else
        hipLaunchKernelGGL(k_amr_l2l<8>, dim3(grid_for(cells * 8)), dim3(WG), 0, s, p, l, nodes, n);
    return hipGetLastError();
}

hipError_t launch_amr_cf(const DevPlan &v, int adj, double *out0, double *out1, hipStream_t s)
{
    if (v.nblist <= 0 || (!v.own_Cp && !v.src_up && !v.src_dn)) return hipSuccess;
    if (adj)
        hipLaunchKernelGGL(k_amr_cf<true>, dim3(v.nblist), dim3(CF_WAVES * 64), 0, s, v, out0, out1);
    else
        hipLaunchKernelGGL(k_amr_cf<false>, dim3(v.nblist), dim3(CF_WAVES * 64), 0, s, v, out0, out1);
    return hipGetLastError();
}

}  // namespace otfmm

namespace otfmm {

hipError_t launch_am_correction(const DevPlan &p, const double *KX, double *const *Pi_host, double *Pi_part,
                                double *t, int tiled, hipStream_t s)
{
    for (int l = 0; l < p.L; ++l) {
        const int64_t n = 8 << l;
        // the tiled form, its offsets split over several workgroups at levels
        // 0..2, which have only 1, 8 and 64 blocks.  Without the LDS for it
        // (measured at 128^3): a wave per cell at levels 0 and 1 (81 and 176
        // us), a thread per cell below (0.70 ms at level 2, 2.6 at level 3).
        if (!tiled && l <= 1) {
            hipLaunchKernelGGL(k_am_pi<true>, dim3((unsigned)(n * n * n)), dim3(64), 0, s, p, l, KX, Pi_host[l]);
        } else if (!tiled) {
            hipLaunchKernelGGL(k_am_pi<false>, dim3(grid_for(n * n * n)), dim3(WG), 0, s, p, l, KX, Pi_host[l]);
        } else {
            const int split = am_split(l);
            const unsigned nblk = (unsigned)(n * n * n / 512);
            // tiled = 2: the device gives a workgroup LDS for two staging buffers
            auto tile = [&](unsigned grid, double *out, int parts, const double *up) {
                if (tiled == 2)
                    hipLaunchKernelGGL(k_am_pi_tile<2>, dim3(grid), dim3(AM_WG), 2 * AM_TILE_LDS, s, p, l, KX, out,
                                       parts, up);
                else
                    hipLaunchKernelGGL(k_am_pi_tile<1>, dim3(grid), dim3(AM_WG), AM_TILE_LDS, s, p, l, KX, out, parts,
                                       up);
            };
            if (split == 1) {
                // the parent's Pi folded in by the same launch
                tile(nblk, Pi_host[l], 1, l > 0 ? (const double *)Pi_host[l - 1] : nullptr);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
                continue;
            } else {
                const int64_t ne = 3 * NC * 8 * (n * n * n / 8);
                tile(nblk * split, Pi_part, split, nullptr);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL(k_am_sum, dim3(grid_for(ne)), dim3(WG), 0, s, Pi_part, split, ne, Pi_host[l]);
            }
        }
        if (l > 0)                                 // fold in the ancestors' (final above level l)
            hipLaunchKernelGGL(k_am_down, dim3(grid_for(n * n * n)), dim3(WG), 0, s, p, l, Pi_host[l - 1], Pi_host[l]);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t n = 8 << p.L;
    hipLaunchKernelGGL(k_am_leaf, dim3((unsigned)(n * n * n / 256)), dim3(WG), 0, s, p,
                       p.L > 0 ? Pi_host[p.L - 1] : nullptr, t);
    return hipGetLastError();
}

}  // namespace otfmm
