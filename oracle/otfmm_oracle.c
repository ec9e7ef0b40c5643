/*
 * otfmm_oracle.c -- plain, slow, FP64 CPU oracle for the octree fast-multipole
 * self-gravity solve of Octo-Tiger (paper Sec. 4.3 "Octo-Tiger in a Nutshell":
 * FMM gravity on an adaptive octree of 8x8x8-cell sub-grids; Sec. 5.5: the
 * same-level interactions are a fixed stencil rather than interaction lists).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the GPU
 * path.
 *
 * The paper names the method but gives none of its formulas; this file reads
 * it with geometric expansion centres, total-order truncation and the
 * parity-aware opening rule, all stated below.
 *
 * Geometry (uniform tree of 8^3-cell sub-grids):
 *   level l = 0..L has n_l = 8*2^l cells per axis and cell width h_l = h*2^(L-l);
 *   the centre of cell c is (c + 1/2) h_l (the origin only shifts all positions
 *   and drops out of every difference).  Cell c at level l has the parent c>>1
 *   at level l-1.  Leaf cells (level L) are point masses m = rho h^3 at their
 *   centres; the self pair is excluded; boundaries are isolated (no cells
 *   outside the box).
 *
 * Method (total expansion order p, opening parameter theta, r_n = 1/theta):
 *   P2M  leaf monopole at the cell centre.
 *   M2M  exact moment shift; moments M_A^a = sum_i m_i (x_i - z_A)^a (multi-index
 *        a, no factorial).
 *   Interaction rule: at level l >= 1 an ordered cell pair (A,B), A != B, is an
 *        M2L pair iff |c_B - c_A| > r_n and |c_B>>1 - c_A>>1| <= r_n; at level 0
 *        (the root sub-grid has no parent) iff |c_B - c_A| > r_n.  At the leaf
 *        level the remaining pairs with 0 < |c_B - c_A| <= r_n are P2P.
 *   M2L  C_A^a += sum_{|a|+|b|<=p} ((-1)^|b| / b!) D^(a+b)(z_A - z_B) M_B^b,
 *        D^a = derivatives of K(r) = -G/|r| (total-order truncation).
 *   L2L  exact Taylor re-expansion C_c^a += sum_g (d^g/g!) C_P^(a+g), d = z_c - z_P.
 *   L2P  at leaf centres: phi = C^0, g = -C^(e_k), plus the P2P sums.
 * The adjoint is the literal transpose of that chain.
 *
 * Cartesian derivatives of 1/r come from the McMurchie-Davidson recurrence
 * (McMurchie & Davidson, J. Comput. Phys. 26 (1978) 218), evaluated per pair.
 *
 * Every pass can be restricted to the leaf z-slab [zlo, zhi): a cell of level l
 * is processed when its z-extent overlaps the slab (the upward pass always runs
 * in full).  This only bounds how much work a timing sample does.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* multi-indices a = (t,u,v) with t+u+v <= p, ordered by total order         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int p;
    int n;          /* number of multi-indices */
    int (*a)[3];    /* [n][3] */
    int *lookup;    /* (p+1)^3 -> position, -1 if t+u+v > p */
    int *order;     /* [n] |a| */
    double *ifact;  /* [n] 1/a! */
    int upto[16];   /* number of multi-indices of total order <= o */
} mset;

static double fact(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; }
static double binom(int n, int k) { return fact(n) / (fact(k) * fact(n - k)); }

static int mset_init(mset *s, int p)
{
    memset(s, 0, sizeof(*s));
    if (p < 0 || p > 12) return -1;
    s->p = p;
    s->n = (p + 1) * (p + 2) * (p + 3) / 6;
    s->a = malloc(sizeof(int[3]) * (size_t)s->n);
    s->lookup = malloc(sizeof(int) * (size_t)(p + 1) * (p + 1) * (p + 1));
    s->order = malloc(sizeof(int) * (size_t)s->n);
    s->ifact = malloc(sizeof(double) * (size_t)s->n);
    if (!s->a || !s->lookup || !s->order || !s->ifact) return -1;
    for (int i = 0; i < (p + 1) * (p + 1) * (p + 1); ++i) s->lookup[i] = -1;
    int k = 0;
    for (int order = 0; order <= p; ++order)
        for (int t = order; t >= 0; --t)
            for (int u = order - t; u >= 0; --u) {
                int v = order - t - u;
                s->a[k][0] = t; s->a[k][1] = u; s->a[k][2] = v;
                s->lookup[(t * (p + 1) + u) * (p + 1) + v] = k;
                s->order[k] = order;
                s->ifact[k] = 1.0 / (fact(t) * fact(u) * fact(v));
                ++k;
            }
    for (int o = 0; o <= p; ++o) s->upto[o] = (o + 1) * (o + 2) * (o + 3) / 6;
    return 0;
}

static void mset_free(mset *s) { free(s->a); free(s->lookup); free(s->order); free(s->ifact); }

static int mset_find(const mset *s, int t, int u, int v)
{
    if (t < 0 || u < 0 || v < 0 || t + u + v > s->p) return -1;
    return s->lookup[(t * (s->p + 1) + u) * (s->p + 1) + v];
}

/* x^a for a 3-vector x and multi-index (t,u,v) */
static double mpow(const double x[3], int t, int u, int v)
{
    double r = 1.0;
    for (int i = 0; i < t; ++i) r *= x[0];
    for (int i = 0; i < u; ++i) r *= x[1];
    for (int i = 0; i < v; ++i) r *= x[2];
    return r;
}

/* ------------------------------------------------------------------------ */
/* derivatives of 1/r: out[k] = d^(a_k) (1/r) at (X,Y,Z), all |a_k| <= p.   */
/* McMurchie-Davidson: R^n_000 = (-1)^n (2n-1)!! / r^(2n+1),                */
/*   R^n_{t,u,v} = X R^{n+1}_{t-1,u,v} + (t-1) R^{n+1}_{t-2,u,v}  (likewise  */
/*   in u with Y and in v with Z), and d^(t,u,v)(1/r) = R^0_{t,u,v}.         */
/* R is caller scratch of (p+1)^4 doubles.                                   */
/* ------------------------------------------------------------------------ */
static void inv_r_derivs(const mset *s, double X, double Y, double Z, double *out, double *R)
{
    const int p = s->p, q = p + 1;
#define RR(n, t, u, v) R[(((n) * q + (t)) * q + (u)) * q + (v)]
    const double r2 = X * X + Y * Y + Z * Z;
    const double r = sqrt(r2);
    double dfact = 1.0;                  /* (2n-1)!! */
    double rpow = 1.0 / r;               /* r^-(2n+1) */
    for (int n = 0; n <= p; ++n) {
        RR(n, 0, 0, 0) = ((n & 1) ? -1.0 : 1.0) * dfact * rpow;
        dfact *= (double)(2 * n + 1);
        rpow /= r2;
    }
    for (int order = 1; order <= p; ++order)
        for (int t = order; t >= 0; --t)
            for (int u = order - t; u >= 0; --u) {
                int v = order - t - u;
                for (int n = 0; n + order <= p; ++n) {
                    double val;
                    if (t > 0) {
                        val = X * RR(n + 1, t - 1, u, v);
                        if (t > 1) val += (t - 1) * RR(n + 1, t - 2, u, v);
                    } else if (u > 0) {
                        val = Y * RR(n + 1, t, u - 1, v);
                        if (u > 1) val += (u - 1) * RR(n + 1, t, u - 2, v);
                    } else {
                        val = Z * RR(n + 1, t, u, v - 1);
                        if (v > 1) val += (v - 1) * RR(n + 1, t, u, v - 2);
                    }
                    RR(n, t, u, v) = val;
                }
            }
    for (int k = 0; k < s->n; ++k) out[k] = RR(0, s->a[k][0], s->a[k][1], s->a[k][2]);
#undef RR
}

/* ------------------------------------------------------------------------ */
/* tree geometry                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int L;            /* leaf level */
    double h;         /* leaf cell width */
    double G;
    double r2;        /* (1/theta)^2 */
    int reach;        /* floor(1/theta): max |parent offset| per axis */
    int zlo, zhi;     /* leaf z-slab processed by the restricted passes */
} tree;

static int nlev(int l) { return 8 << l; }
static double hlev(const tree *T, int l) { return T->h * (double)(1 << (T->L - l)); }
static int64_t cid(int n, int x, int y, int z) { return ((int64_t)z * n + y) * n + x; }

static void centre(const tree *T, int l, int x, int y, int z, double out[3])
{
    const double hl = hlev(T, l);
    out[0] = (x + 0.5) * hl; out[1] = (y + 0.5) * hl; out[2] = (z + 0.5) * hl;
}

/* z-range of level-l cells whose leaf extent overlaps the slab */
static int zfirst(const tree *T, int l) { return T->zlo >> (T->L - l); }
static int zend(const tree *T, int l) { return ((T->zhi - 1) >> (T->L - l)) + 1; }

static int is_near(const tree *T, int dx, int dy, int dz)
{
    return (double)(dx * dx + dy * dy + dz * dz) <= T->r2;
}

/* Interaction rule at level l for the ordered pair (sink A, source B). */
static int m2l_rule(const tree *T, int l, const int A[3], const int B[3])
{
    if (A[0] == B[0] && A[1] == B[1] && A[2] == B[2]) return 0;
    if (is_near(T, B[0] - A[0], B[1] - A[1], B[2] - A[2])) return 0;
    if (l == 0) return 1;
    return is_near(T, (B[0] >> 1) - (A[0] >> 1), (B[1] >> 1) - (A[1] >> 1),
                   (B[2] >> 1) - (A[2] >> 1));
}

static int p2p_rule(const tree *T, const int A[3], const int B[3])
{
    if (A[0] == B[0] && A[1] == B[1] && A[2] == B[2]) return 0;
    return is_near(T, B[0] - A[0], B[1] - A[1], B[2] - A[2]);
}

/* Candidate partners of A at level l (clipped to the domain): every cell of
 * the level at level 0, otherwise the children of the parents within `reach`
 * per axis of A's parent.  Every pair the rule accepts lies in this box. */
typedef struct { int lo[3], hi[3]; } box;

static box m2l_candidates(const tree *T, int l, const int A[3])
{
    box b;
    const int n = nlev(l);
    for (int k = 0; k < 3; ++k) {
        if (l == 0) { b.lo[k] = 0; b.hi[k] = n - 1; continue; }
        int q = A[k] >> 1;
        int lo = 2 * (q - T->reach), hi = 2 * (q + T->reach) + 1;
        b.lo[k] = lo < 0 ? 0 : lo;
        b.hi[k] = hi > n - 1 ? n - 1 : hi;
    }
    return b;
}

static box p2p_candidates(const tree *T, const int A[3])
{
    box b;
    const int n = nlev(T->L);
    for (int k = 0; k < 3; ++k) {
        int lo = A[k] - T->reach, hi = A[k] + T->reach;
        b.lo[k] = lo < 0 ? 0 : lo;
        b.hi[k] = hi > n - 1 ? n - 1 : hi;
    }
    return b;
}

static int tree_init(tree *T, int L, double theta, double h, double G)
{
    if (L < 0 || L > 7 || !(theta > 0.0) || !(h > 0.0)) return -1;
    T->L = L; T->h = h; T->G = G;
    const double rn = 1.0 / theta;
    T->r2 = rn * rn;
    T->reach = (int)floor(rn);
    T->zlo = 0; T->zhi = nlev(L);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* expansion operators (unscaled moments, derivative-tensor locals)          */
/* ------------------------------------------------------------------------ */

/* M2L: C_A^a += sum_{|a|+|b|<=p} ((-1)^|b| / b!) D^(a+b)(R) M_B^b with
 * R = z_A - z_B.  `q` is the highest order the source moments can hold
 * (higher ones are zero and are skipped).  D and Rs are scratch. */
static void m2l(const mset *s, double G, const double R[3], const double *MB, int q,
                double *CA, double *D, double *Rs)
{
    inv_r_derivs(s, R[0], R[1], R[2], D, Rs);
    for (int ia = 0; ia < s->n; ++ia) {
        const int *a = s->a[ia];
        const int qb = (s->p - s->order[ia]) < q ? (s->p - s->order[ia]) : q;
        double acc = 0.0;
        for (int ib = 0; ib < s->upto[qb]; ++ib) {
            const int *b = s->a[ib];
            int k = mset_find(s, a[0] + b[0], a[1] + b[1], a[2] + b[2]);
            double sgn = (s->order[ib] & 1) ? -1.0 : 1.0;
            acc += sgn * s->ifact[ib] * (-G * D[k]) * MB[ib];
        }
        CA[ia] += acc;
    }
}

/* M2M: M_P^a += sum_{b<=a} binom(a,b) d^(a-b) M_c^b, d = z_c - z_P. */
static void m2m(const mset *s, const double d[3], const double *Mc, int q, double *MP)
{
    for (int ia = 0; ia < s->n; ++ia) {
        const int *a = s->a[ia];
        double acc = 0.0;
        for (int ib = 0; ib < s->upto[q]; ++ib) {
            const int *b = s->a[ib];
            if (b[0] > a[0] || b[1] > a[1] || b[2] > a[2]) continue;
            double c = binom(a[0], b[0]) * binom(a[1], b[1]) * binom(a[2], b[2]);
            acc += c * mpow(d, a[0] - b[0], a[1] - b[1], a[2] - b[2]) * Mc[ib];
        }
        MP[ia] += acc;
    }
}

/* L2L: C_c^a += sum_{|a+g|<=p} (d^g / g!) C_P^(a+g), d = z_c - z_P. */
static void l2l(const mset *s, const double d[3], const double *CP, double *Cc)
{
    for (int ia = 0; ia < s->n; ++ia) {
        const int *a = s->a[ia];
        double acc = 0.0;
        for (int ig = 0; ig < s->upto[s->p - s->order[ia]]; ++ig) {
            const int *g = s->a[ig];
            int k = mset_find(s, a[0] + g[0], a[1] + g[1], a[2] + g[2]);
            acc += mpow(d, g[0], g[1], g[2]) * s->ifact[ig] * CP[k];
        }
        Cc[ia] += acc;
    }
}

/* P2P: potential and acceleration at x_i of a point mass m_j at x_j. */
static void p2p(double G, const double xi[3], const double xj[3], double mj, double *phi, double g[3])
{
    double r[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double rinv = 1.0 / sqrt(r2);
    double rinv3 = rinv * rinv * rinv;
    *phi += -G * mj * rinv;
    for (int k = 0; k < 3; ++k) g[k] += -G * mj * r[k] * rinv3;
}

/* ------------------------------------------------------------------------ */
/* tree state                                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    tree T;
    mset s;
    double *M[8];   /* [n_l^3][ncomp] moments (or their adjoints) per level */
    double *C[8];   /* [n_l^3][ncomp] local coefficients (or adjoints) per level */
} fmm;

static void fmm_free(fmm *F)
{
    for (int l = 0; l < 8; ++l) { free(F->M[l]); free(F->C[l]); F->M[l] = F->C[l] = NULL; }
    mset_free(&F->s);
}

static int fmm_alloc(fmm *F, int L, int p, double theta, double h, double G)
{
    memset(F, 0, sizeof(*F));
    if (tree_init(&F->T, L, theta, h, G)) return -1;
    if (mset_init(&F->s, p)) return -1;
    for (int l = 0; l <= L; ++l) {
        size_t n3 = (size_t)nlev(l) * nlev(l) * nlev(l);
        F->M[l] = calloc(n3 * F->s.n, sizeof(double));
        F->C[l] = calloc(n3 * F->s.n, sizeof(double));
        if (!F->M[l] || !F->C[l]) return -1;
    }
    return 0;
}

static int set_slab(fmm *F, int zlo, int zhi)
{
    const int n = nlev(F->T.L);
    if (zlo < 0 || zhi > n || zlo >= zhi) return -1;
    F->T.zlo = zlo; F->T.zhi = zhi;
    return 0;
}

static size_t scratch_len(const mset *s) { return (size_t)(s->p + 1) * (s->p + 1) * (s->p + 1) * (s->p + 1); }

/* P2M + M2M upward pass (always the whole tree). Leaf monopole m = rho h^3. */
static void upward(fmm *F, const double *rho)
{
    const tree *T = &F->T;
    const int nc = F->s.n, L = T->L;
    const int n = nlev(L);
    const double h3 = T->h * T->h * T->h;
    for (int64_t i = 0; i < (int64_t)n * n * n; ++i) F->M[L][i * nc + 0] = rho[i] * h3;
    for (int l = L - 1; l >= 0; --l) {
        const int np = nlev(l), nch = nlev(l + 1);
        const int q = (l == L - 1) ? 0 : F->s.p;   /* leaf moments are monopoles */
#pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < np; ++z)
            for (int y = 0; y < np; ++y)
                for (int x = 0; x < np; ++x) {
                    double zP[3], zc[3], d[3];
                    centre(T, l, x, y, z, zP);
                    double *MP = &F->M[l][cid(np, x, y, z) * nc];
                    for (int b = 0; b < 8; ++b) {
                        int cx = 2 * x + (b & 1), cy = 2 * y + ((b >> 1) & 1), cz = 2 * z + (b >> 2);
                        centre(T, l + 1, cx, cy, cz, zc);
                        for (int k = 0; k < 3; ++k) d[k] = zc[k] - zP[k];
                        m2m(&F->s, d, &F->M[l + 1][cid(nch, cx, cy, cz) * nc], q, MP);
                    }
                }
    }
}

/* M2L at every level, the leaf level included (its far pairs act on leaf
 * monopoles); sinks restricted to the slab. */
static void interact(fmm *F)
{
    const tree *T = &F->T;
    const int nc = F->s.n;
    for (int l = 0; l <= T->L; ++l) {
        const int n = nlev(l);
        const int q = (l == T->L) ? 0 : F->s.p;
        const int z0 = zfirst(T, l), z1 = zend(T, l);
#pragma omp parallel
        {
            double *D = malloc(sizeof(double) * nc);
            double *Rs = malloc(sizeof(double) * scratch_len(&F->s));
#pragma omp for collapse(2) schedule(dynamic, 1)
            for (int z = z0; z < z1; ++z)
                for (int y = 0; y < n; ++y)
                    for (int x = 0; x < n; ++x) {
                        const int A[3] = {x, y, z};
                        double zA[3], zB[3], R[3];
                        centre(T, l, x, y, z, zA);
                        double *CA = &F->C[l][cid(n, x, y, z) * nc];
                        box bx = m2l_candidates(T, l, A);
                        for (int bz = bx.lo[2]; bz <= bx.hi[2]; ++bz)
                            for (int by = bx.lo[1]; by <= bx.hi[1]; ++by)
                                for (int bxx = bx.lo[0]; bxx <= bx.hi[0]; ++bxx) {
                                    const int B[3] = {bxx, by, bz};
                                    if (!m2l_rule(T, l, A, B)) continue;
                                    centre(T, l, bxx, by, bz, zB);
                                    for (int k = 0; k < 3; ++k) R[k] = zA[k] - zB[k];
                                    m2l(&F->s, T->G, R, &F->M[l][cid(n, bxx, by, bz) * nc], q, CA, D, Rs);
                                }
                    }
            free(D);
            free(Rs);
        }
    }
}

/* L2L downward pass (levels 1..L), sinks restricted to the slab. */
static void downward(fmm *F)
{
    const tree *T = &F->T;
    const int nc = F->s.n;
    for (int l = 1; l <= T->L; ++l) {
        const int n = nlev(l), np = nlev(l - 1);
        const int z0 = zfirst(T, l), z1 = zend(T, l);
#pragma omp parallel for collapse(2) schedule(static)
        for (int z = z0; z < z1; ++z)
            for (int y = 0; y < n; ++y)
                for (int x = 0; x < n; ++x) {
                    double zc[3], zP[3], d[3];
                    centre(T, l, x, y, z, zc);
                    centre(T, l - 1, x >> 1, y >> 1, z >> 1, zP);
                    for (int k = 0; k < 3; ++k) d[k] = zc[k] - zP[k];
                    l2l(&F->s, d, &F->C[l - 1][cid(np, x >> 1, y >> 1, z >> 1) * nc],
                        &F->C[l][cid(n, x, y, z) * nc]);
                }
    }
}

/* Index of the first-order multi-index e_k. */
static int e_k(const mset *s, int k) { return mset_find(s, k == 0, k == 1, k == 2); }

/* L2P + P2P at the leaves of the slab. */
static void evaluate(fmm *F, const double *rho, double *phi, double *g)
{
    const tree *T = &F->T;
    const int nc = F->s.n, L = T->L, n = nlev(L);
    const int64_t N = (int64_t)n * n * n;
    const double h3 = T->h * T->h * T->h;
    const int p = F->s.p;
    const int ex = e_k(&F->s, 0), ey = e_k(&F->s, 1), ez = e_k(&F->s, 2);
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int z = T->zlo; z < T->zhi; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                const int A[3] = {x, y, z};
                const int64_t i = cid(n, x, y, z);
                const double *C = &F->C[L][i * nc];
                double xi[3], xj[3];
                centre(T, L, x, y, z, xi);
                double ph = C[0];
                double gg[3] = {0.0, 0.0, 0.0};
                if (p >= 1) { gg[0] = -C[ex]; gg[1] = -C[ey]; gg[2] = -C[ez]; }
                box bx = p2p_candidates(T, A);
                for (int bz = bx.lo[2]; bz <= bx.hi[2]; ++bz)
                    for (int by = bx.lo[1]; by <= bx.hi[1]; ++by)
                        for (int bxx = bx.lo[0]; bxx <= bx.hi[0]; ++bxx) {
                            const int B[3] = {bxx, by, bz};
                            if (!p2p_rule(T, A, B)) continue;
                            centre(T, L, bxx, by, bz, xj);
                            p2p(T->G, xi, xj, rho[cid(n, bxx, by, bz)] * h3, &ph, gg);
                        }
                phi[i] = ph;
                g[i] = gg[0]; g[N + i] = gg[1]; g[2 * N + i] = gg[2];
            }
}

/* ------------------------------------------------------------------------ */
/* public entry points (dense grids, x fastest: index (z*n + y)*n + x)       */
/* All return 0 on success, -1 on a bad argument or allocation failure.      */
/* ------------------------------------------------------------------------ */

int oracle_ncomp(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Multi-index table in this oracle's component order: idx[3k..3k+2] = (t,u,v). */
int oracle_multi_index(int p, int *idx)
{
    mset s;
    if (mset_init(&s, p)) { mset_free(&s); return -1; }
    for (int k = 0; k < s.n; ++k) { idx[3 * k] = s.a[k][0]; idx[3 * k + 1] = s.a[k][1]; idx[3 * k + 2] = s.a[k][2]; }
    mset_free(&s);
    return 0;
}

/* Derivatives of 1/r at R (all orders <= p, oracle component order). */
int oracle_inv_r_derivs(int p, const double *R, double *out)
{
    mset s;
    if (mset_init(&s, p)) { mset_free(&s); return -1; }
    double *Rs = malloc(sizeof(double) * scratch_len(&s));
    inv_r_derivs(&s, R[0], R[1], R[2], out, Rs);
    free(Rs);
    mset_free(&s);
    return 0;
}

/* Direct Newtonian sum over the cell centres of an n^3 grid (i != j).
 * sinks: NULL for all cells (nsink ignored), else nsink dense cell indices.
 * phi[nsink], g[3*nsink] (three planes). */
int oracle_direct(int n, double h, double G, const double *rho, int64_t nsink,
                  const int64_t *sinks, double *phi, double *g)
{
    if (n <= 0 || !(h > 0.0)) return -1;
    const int64_t N = (int64_t)n * n * n;
    const double h3 = h * h * h;
    if (!sinks) nsink = N;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < nsink; ++s) {
        const int64_t i = sinks ? sinks[s] : s;
        const int ix = (int)(i % n), iy = (int)((i / n) % n), iz = (int)(i / ((int64_t)n * n));
        const double xi[3] = {(ix + 0.5) * h, (iy + 0.5) * h, (iz + 0.5) * h};
        double ph = 0.0, gg[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            const int jx = (int)(j % n), jy = (int)((j / n) % n), jz = (int)(j / ((int64_t)n * n));
            const double xj[3] = {(jx + 0.5) * h, (jy + 0.5) * h, (jz + 0.5) * h};
            p2p(G, xi, xj, rho[j] * h3, &ph, gg);
        }
        phi[s] = ph;
        g[s] = gg[0]; g[nsink + s] = gg[1]; g[2 * nsink + s] = gg[2];
    }
    return 0;
}

/* FMM forward on a uniform tree with leaf level L (n = 8*2^L cells per axis),
 * outputs written for the leaves of the slab [zlo, zhi) only. */
int oracle_fmm_slab(int L, int p, double theta, double h, double G, const double *rho,
                    int zlo, int zhi, double *phi, double *g)
{
    fmm F;
    if (fmm_alloc(&F, L, p, theta, h, G) || set_slab(&F, zlo, zhi)) { fmm_free(&F); return -1; }
    upward(&F, rho);
    interact(&F);
    downward(&F);
    evaluate(&F, rho, phi, g);
    fmm_free(&F);
    return 0;
}

int oracle_fmm(int L, int p, double theta, double h, double G, const double *rho,
               double *phi, double *g)
{
    return oracle_fmm_slab(L, p, theta, h, G, rho, 0, nlev(L < 0 ? 0 : L), phi, g);
}

/* FMM forward evaluated only at the given leaf cells: for each sink, the P2P
 * sum plus, for every ancestor A_l (l = 0..L), the M2L sum over A_l's
 * interaction list, re-expanded exactly from z_{A_l} to the sink centre. */
int oracle_fmm_sinks(int L, int p, double theta, double h, double G, const double *rho,
                     int64_t nsink, const int64_t *sinks, double *phi, double *g)
{
    fmm F;
    if (fmm_alloc(&F, L, p, theta, h, G)) { fmm_free(&F); return -1; }
    const tree *T = &F.T;
    const int nc = F.s.n, n = nlev(L);
    const double h3 = h * h * h;
    upward(&F, rho);
    const int ex = e_k(&F.s, 0), ey = e_k(&F.s, 1), ez = e_k(&F.s, 2);
#pragma omp parallel
    {
        double *D = malloc(sizeof(double) * nc);
        double *Rs = malloc(sizeof(double) * scratch_len(&F.s));
        double *CA = malloc(sizeof(double) * nc);
        double *Ci = malloc(sizeof(double) * nc);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < nsink; ++s) {
            const int64_t i = sinks[s];
            const int ix = (int)(i % n), iy = (int)((i / n) % n), iz = (int)(i / ((int64_t)n * n));
            double xi[3], zA[3], zB[3], R[3], d[3];
            centre(T, L, ix, iy, iz, xi);
            memset(Ci, 0, sizeof(double) * nc);
            for (int l = 0; l <= L; ++l) {
                const int nl = nlev(l), sh = L - l;
                const int q = (l == L) ? 0 : p;
                const int A[3] = {ix >> sh, iy >> sh, iz >> sh};
                centre(T, l, A[0], A[1], A[2], zA);
                memset(CA, 0, sizeof(double) * nc);
                box bx = m2l_candidates(T, l, A);
                for (int bz = bx.lo[2]; bz <= bx.hi[2]; ++bz)
                    for (int by = bx.lo[1]; by <= bx.hi[1]; ++by)
                        for (int bxx = bx.lo[0]; bxx <= bx.hi[0]; ++bxx) {
                            const int B[3] = {bxx, by, bz};
                            if (!m2l_rule(T, l, A, B)) continue;
                            centre(T, l, bxx, by, bz, zB);
                            for (int k = 0; k < 3; ++k) R[k] = zA[k] - zB[k];
                            m2l(&F.s, G, R, &F.M[l][cid(nl, bxx, by, bz) * nc], q, CA, D, Rs);
                        }
                for (int k = 0; k < 3; ++k) d[k] = xi[k] - zA[k];
                l2l(&F.s, d, CA, Ci);
            }
            double ph = Ci[0], gg[3] = {0.0, 0.0, 0.0};
            if (p >= 1) { gg[0] = -Ci[ex]; gg[1] = -Ci[ey]; gg[2] = -Ci[ez]; }
            const int A[3] = {ix, iy, iz};
            double xj[3];
            box bx = p2p_candidates(T, A);
            for (int bz = bx.lo[2]; bz <= bx.hi[2]; ++bz)
                for (int by = bx.lo[1]; by <= bx.hi[1]; ++by)
                    for (int bxx = bx.lo[0]; bxx <= bx.hi[0]; ++bxx) {
                        const int B[3] = {bxx, by, bz};
                        if (!p2p_rule(T, A, B)) continue;
                        centre(T, L, bxx, by, bz, xj);
                        p2p(G, xi, xj, rho[cid(n, bxx, by, bz)] * h3, &ph, gg);
                    }
            phi[s] = ph;
            g[s] = gg[0]; g[nsink + s] = gg[1]; g[2 * nsink + s] = gg[2];
        }
        free(D); free(Rs); free(CA); free(Ci);
    }
    fmm_free(&F);
    return 0;
}

/* Adjoint: drho = F^T (w, u) for the loss sum_i w_i phi_i + u_i . g_i, as the
 * literal transpose of the forward chain, in reverse order:
 *   (L2P, P2P)^T -> L2L^T (upward) -> M2L^T -> M2M^T (downward) -> P2M^T.
 * F.C holds the adjoints of the local coefficients, F.M those of the moments.
 * drho is written for the leaves of the slab [zlo, zhi) only. */
int oracle_fmm_adjoint_slab(int L, int p, double theta, double h, double G, const double *w,
                            const double *u, int zlo, int zhi, double *drho)
{
    fmm F;
    if (fmm_alloc(&F, L, p, theta, h, G) || set_slab(&F, zlo, zhi)) { fmm_free(&F); return -1; }
    const tree *T = &F.T;
    const mset *s = &F.s;
    const int nc = s->n, n = nlev(L);
    const int64_t N = (int64_t)n * n * n;
    const double h3 = h * h * h;
    const int ex = e_k(s, 0), ey = e_k(s, 1), ez = e_k(s, 2);

    /* L2P^T: phi = C^0 and g_k = -C^(e_k) at every leaf */
    for (int64_t i = 0; i < N; ++i) {
        double *C = &F.C[L][i * nc];
        C[0] = w[i];
        if (p >= 1) { C[ex] = -u[i]; C[ey] = -u[N + i]; C[ez] = -u[2 * N + i]; }
    }

    /* L2L^T: C_P^(a+g) += (d^g / g!) C_c^a over the children c, levels L..1
     * (the whole tree: every parent's adjoint feeds the slab's M2L^T) */
    for (int l = L; l >= 1; --l) {
        const int nch = nlev(l), np = nlev(l - 1);
#pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < np; ++z)
            for (int y = 0; y < np; ++y)
                for (int x = 0; x < np; ++x) {
                    double zP[3], zc[3], d[3];
                    centre(T, l - 1, x, y, z, zP);
                    double *CP = &F.C[l - 1][cid(np, x, y, z) * nc];
                    for (int b = 0; b < 8; ++b) {
                        int cx = 2 * x + (b & 1), cy = 2 * y + ((b >> 1) & 1), cz = 2 * z + (b >> 2);
                        centre(T, l, cx, cy, cz, zc);
                        for (int k = 0; k < 3; ++k) d[k] = zc[k] - zP[k];
                        const double *Cc = &F.C[l][cid(nch, cx, cy, cz) * nc];
                        const int qa = (l == L) ? (p >= 1 ? 1 : 0) : p;  /* leaf adjoints: orders 0, 1 */
                        for (int ia = 0; ia < s->upto[qa]; ++ia)
                            for (int ig = 0; ig < s->upto[p - s->order[ia]]; ++ig) {
                                const int *a = s->a[ia], *gm = s->a[ig];
                                int k = mset_find(s, a[0] + gm[0], a[1] + gm[1], a[2] + gm[2]);
                                CP[k] += mpow(d, gm[0], gm[1], gm[2]) * s->ifact[ig] * Cc[ia];
                            }
                    }
                }
    }

    /* M2L^T: M_B^b += ((-1)^|b| / b!) D^(a+b)(z_A - z_B) C_A^a over the pairs
     * (A,B) the interaction rule accepts, gathered at the source B. */
    for (int l = 0; l <= L; ++l) {
        const int nl = nlev(l);
        const int qa = (l == L) ? (p >= 1 ? 1 : 0) : p;
        /* a leaf holds only a monopole moment, so only its adjoint is live */
        const int nb = (l == L) ? 1 : nc;
        const int z0 = zfirst(T, l), z1 = zend(T, l);
#pragma omp parallel
        {
            double *D = malloc(sizeof(double) * nc);
            double *Rs = malloc(sizeof(double) * scratch_len(s));
#pragma omp for collapse(2) schedule(dynamic, 1)
            for (int z = z0; z < z1; ++z)
                for (int y = 0; y < nl; ++y)
                    for (int x = 0; x < nl; ++x) {
                        const int B[3] = {x, y, z};
                        double zA[3], zB[3], R[3];
                        centre(T, l, x, y, z, zB);
                        double *MB = &F.M[l][cid(nl, x, y, z) * nc];
                        box bx = m2l_candidates(T, l, B);
                        for (int az = bx.lo[2]; az <= bx.hi[2]; ++az)
                            for (int ay = bx.lo[1]; ay <= bx.hi[1]; ++ay)
                                for (int axx = bx.lo[0]; axx <= bx.hi[0]; ++axx) {
                                    const int A[3] = {axx, ay, az};
                                    if (!m2l_rule(T, l, A, B)) continue;
                                    centre(T, l, axx, ay, az, zA);
                                    for (int k = 0; k < 3; ++k) R[k] = zA[k] - zB[k];
                                    inv_r_derivs(s, R[0], R[1], R[2], D, Rs);
                                    const double *CA = &F.C[l][cid(nl, axx, ay, az) * nc];
                                    for (int ib = 0; ib < nb; ++ib) {
                                        const int *b = s->a[ib];
                                        const double sgn = (s->order[ib] & 1) ? -1.0 : 1.0;
                                        const int qmax = (p - s->order[ib]) < qa ? (p - s->order[ib]) : qa;
                                        double acc = 0.0;
                                        for (int ia = 0; ia < s->upto[qmax]; ++ia) {
                                            const int *a = s->a[ia];
                                            int k = mset_find(s, a[0] + b[0], a[1] + b[1], a[2] + b[2]);
                                            acc += sgn * s->ifact[ib] * (-G * D[k]) * CA[ia];
                                        }
                                        MB[ib] += acc;
                                    }
                                }
                    }
            free(D);
            free(Rs);
        }
    }

    /* M2M^T: M_c^b += binom(a,b) d^(a-b) M_P^a, levels 0..L-1 downward */
    for (int l = 0; l < L; ++l) {
        const int np = nlev(l), nch = nlev(l + 1);
        const int qb = (l + 1 == L) ? 0 : p;   /* leaf moments: only the monopole is live */
        const int z0 = zfirst(T, l + 1), z1 = zend(T, l + 1);
#pragma omp parallel for collapse(2) schedule(static)
        for (int z = z0; z < z1; ++z)
            for (int y = 0; y < nch; ++y)
                for (int x = 0; x < nch; ++x) {
                    double zP[3], zc[3], d[3];
                    centre(T, l + 1, x, y, z, zc);
                    centre(T, l, x >> 1, y >> 1, z >> 1, zP);
                    for (int k = 0; k < 3; ++k) d[k] = zc[k] - zP[k];
                    const double *MP = &F.M[l][cid(np, x >> 1, y >> 1, z >> 1) * nc];
                    double *Mc = &F.M[l + 1][cid(nch, x, y, z) * nc];
                    for (int ib = 0; ib < s->upto[qb]; ++ib)
                        for (int ia = 0; ia < nc; ++ia) {
                            const int *a = s->a[ia], *b = s->a[ib];
                            if (b[0] > a[0] || b[1] > a[1] || b[2] > a[2]) continue;
                            double c = binom(a[0], b[0]) * binom(a[1], b[1]) * binom(a[2], b[2]);
                            Mc[ib] += c * mpow(d, a[0] - b[0], a[1] - b[1], a[2] - b[2]) * MP[ia];
                        }
                }
    }

    /* (P2P)^T gathered at the source j, then P2M^T: drho_j = h^3 (M_j^0 + mhat_j) */
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int z = T->zlo; z < T->zhi; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                const int Bj[3] = {x, y, z};
                const int64_t j = cid(n, x, y, z);
                double xj[3], xi[3];
                centre(T, L, x, y, z, xj);
                double mh = 0.0;
                box bx = p2p_candidates(T, Bj);
                for (int iz = bx.lo[2]; iz <= bx.hi[2]; ++iz)
                    for (int iy = bx.lo[1]; iy <= bx.hi[1]; ++iy)
                        for (int ix = bx.lo[0]; ix <= bx.hi[0]; ++ix) {
                            const int Ai[3] = {ix, iy, iz};
                            if (!p2p_rule(T, Ai, Bj)) continue;
                            centre(T, L, ix, iy, iz, xi);
                            /* d phi_i / d m_j and d g_i / d m_j of the P2P term */
                            double ph = 0.0, gg[3] = {0.0, 0.0, 0.0};
                            p2p(G, xi, xj, 1.0, &ph, gg);
                            const int64_t i = cid(n, ix, iy, iz);
                            mh += ph * w[i] + gg[0] * u[i] + gg[1] * u[N + i] + gg[2] * u[2 * N + i];
                        }
                drho[j] = h3 * (F.M[L][j * nc + 0] + mh);
            }
    fmm_free(&F);
    return 0;
}

int oracle_fmm_adjoint(int L, int p, double theta, double h, double G, const double *w,
                       const double *u, double *drho)
{
    return oracle_fmm_adjoint_slab(L, p, theta, h, G, w, u, 0, nlev(L < 0 ? 0 : L), drho);
}

/* Moments of every cell at `level` after the upward pass: out[k*n_l^3 + cell]. */
int oracle_moments(int L, int p, double h, const double *rho, int level, double *out)
{
    fmm F;
    if (level < 0 || level > L) return -1;
    if (fmm_alloc(&F, L, p, 1.0, h, 1.0)) { fmm_free(&F); return -1; }
    upward(&F, rho);
    const int64_t n3 = (int64_t)nlev(level) * nlev(level) * nlev(level);
    for (int64_t i = 0; i < n3; ++i)
        for (int k = 0; k < F.s.n; ++k) out[k * n3 + i] = F.M[level][i * F.s.n + k];
    fmm_free(&F);
    return 0;
}

/* Ordered-pair counts by brute-force enumeration of the interaction rule over
 * the slab's sinks: *p2p_out = leaf P2P pairs, m2l_out[l] = M2L pairs at level
 * l (l = 0..L; the leaf level's far pairs are in m2l_out[L]). */
int oracle_pair_counts_slab(int L, double theta, int zlo, int zhi, int64_t *p2p_out, int64_t *m2l_out)
{
    tree T;
    if (tree_init(&T, L, theta, 1.0, 1.0)) return -1;
    if (zlo < 0 || zhi > nlev(L) || zlo >= zhi) return -1;
    T.zlo = zlo; T.zhi = zhi;
    int64_t pc = 0;
    for (int l = 0; l <= L; ++l) {
        const int n = nlev(l);
        const int z0 = zfirst(&T, l), z1 = zend(&T, l);
        int64_t cnt = 0;
#pragma omp parallel for collapse(2) reduction(+ : cnt) schedule(static)
        for (int z = z0; z < z1; ++z)
            for (int y = 0; y < n; ++y)
                for (int x = 0; x < n; ++x) {
                    const int A[3] = {x, y, z};
                    box bx = m2l_candidates(&T, l, A);
                    for (int bz = bx.lo[2]; bz <= bx.hi[2]; ++bz)
                        for (int by = bx.lo[1]; by <= bx.hi[1]; ++by)
                            for (int bxx = bx.lo[0]; bxx <= bx.hi[0]; ++bxx) {
                                const int B[3] = {bxx, by, bz};
                                cnt += m2l_rule(&T, l, A, B);
                            }
                }
        m2l_out[l] = cnt;
    }
    const int n = nlev(L);
#pragma omp parallel for collapse(2) reduction(+ : pc) schedule(static)
    for (int z = zlo; z < zhi; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                const int A[3] = {x, y, z};
                box bx = p2p_candidates(&T, A);
                for (int bz = bx.lo[2]; bz <= bx.hi[2]; ++bz)
                    for (int by = bx.lo[1]; by <= bx.hi[1]; ++by)
                        for (int bxx = bx.lo[0]; bxx <= bx.hi[0]; ++bxx) {
                            const int B[3] = {bxx, by, bz};
                            pc += p2p_rule(&T, A, B);
                        }
            }
    *p2p_out = pc;
    return 0;
}

int oracle_pair_counts(int L, double theta, int64_t *p2p_out, int64_t *m2l_out)
{
    return oracle_pair_counts_slab(L, theta, 0, nlev(L < 0 ? 0 : L), p2p_out, m2l_out);
}

/* ======================================================================== */
/* Adaptive octrees: leaf sub-grids on several levels                        */
/* ======================================================================== */
/*
 * Nodes are 8^3-cell sub-grids given as (level, coordinates, leaf flag), node
 * 0 the root and every internal node with its 8 children (Sec. 4.3: the octree
 * is refined where the solution needs it).  The finest level Lmax has cell
 * width h, level l has h_l = h 2^(Lmax - l), and a leaf cell is a point mass
 * m = rho h_l^3 at its centre.  Leaf cell k of leaf node j (j-th leaf in
 * layout order) has index 512 j + k, x fastest inside the sub-grid.
 *
 * The paper names the adaptive tree but not the treatment where refinement
 * changes.  Reading used here:
 *   - leaf sub-grids that touch (across a face, an edge or a corner) lie at
 *     most one level apart (2:1 balance);
 *   - at each level l the same-level rule of the uniform tree holds between
 *     all cells that exist at l, leaves and refined cells alike: (A, B) is an
 *     M2L pair when B is far from A and their parents are near (at the root:
 *     when B is far);
 *   - a near pair at level l of two leaves is a P2P pair; a near pair of a
 *     leaf and a refined cell is a P2P pair between the leaf and each child of
 *     the refined cell (those children are leaves under 2:1 balance); a near
 *     pair of two refined cells passes to their children.
 * Every ordered pair of distinct leaf cells is then accounted for once: the
 * first level at which their ancestors are far gives the M2L pair, and
 * ancestors that stay near down to the coarser leaf give a P2P pair.
 */
typedef struct {
    int Lmax;
    double h, G, r2;
    int reach;
    int64_t nn;
    const int32_t *lvl, *crd;
    const uint8_t *leaf;
    int32_t *nid[8];       /* per level: node at sub-grid coordinates, or -1 */
    int64_t *first;        /* per node: index of its first leaf cell, -1 if internal */
    int64_t *leaf_node;    /* per leaf sub-grid in layout order: its node */
    int64_t ncell;
    double *M;             /* [nn * 512][nc]: moments of every cell of every node */
    mset s;
} amr;

static double amr_h(const amr *A, int l) { return A->h * (double)(1 << (A->Lmax - l)); }

static void amr_free(amr *A)
{
    for (int l = 0; l < 8; ++l) { free(A->nid[l]); A->nid[l] = NULL; }
    free(A->first); free(A->leaf_node); free(A->M);
    A->first = NULL; A->leaf_node = NULL; A->M = NULL;
    mset_free(&A->s);
}

static int amr_init(amr *A, int64_t nn, const int32_t *lvl, const int32_t *crd, const uint8_t *leaf,
                    int p, double theta, double h, double G)
{
    memset(A, 0, sizeof(*A));
    if (nn < 1 || !(theta > 0.0) || !(h > 0.0) || mset_init(&A->s, p)) return -1;
    A->nn = nn; A->lvl = lvl; A->crd = crd; A->leaf = leaf;
    A->h = h; A->G = G;
    const double rn = 1.0 / theta;
    A->r2 = rn * rn;
    A->reach = (int)floor(rn);
    int Lmax = 0;
    for (int64_t i = 0; i < nn; ++i) {
        if (lvl[i] < 0 || lvl[i] > 7) return -1;
        if (lvl[i] > Lmax) Lmax = lvl[i];
    }
    A->Lmax = Lmax;
    for (int l = 0; l <= Lmax; ++l) {
        const int64_t m = (int64_t)1 << l;
        A->nid[l] = malloc(sizeof(int32_t) * (size_t)(m * m * m));
        if (!A->nid[l]) return -1;
        for (int64_t k = 0; k < m * m * m; ++k) A->nid[l][k] = -1;
    }
    A->first = malloc(sizeof(int64_t) * (size_t)nn);
    A->leaf_node = malloc(sizeof(int64_t) * (size_t)nn);
    if (!A->first || !A->leaf_node) return -1;
    int64_t nleaf = 0;
    for (int64_t i = 0; i < nn; ++i) {
        const int l = lvl[i];
        const int64_t m = (int64_t)1 << l;
        const int x = crd[3 * i], y = crd[3 * i + 1], z = crd[3 * i + 2];
        if (x < 0 || y < 0 || z < 0 || x >= m || y >= m || z >= m) return -1;
        A->nid[l][(z * m + y) * m + x] = (int32_t)i;
        if (leaf[i]) A->leaf_node[nleaf] = i;
        A->first[i] = leaf[i] ? 512 * nleaf++ : -1;
    }
    A->ncell = 512 * nleaf;
    A->M = calloc((size_t)nn * 512 * (size_t)A->s.n, sizeof(double));
    return A->M ? 0 : -1;
}

/* node holding cell (x, y, z) of level l, or -1 where the level has no cell */
static int64_t amr_node(const amr *A, int l, int x, int y, int z)
{
    if (l < 0 || l > A->Lmax) return -1;
    const int n = 8 << l;
    if (x < 0 || y < 0 || z < 0 || x >= n || y >= n || z >= n) return -1;
    const int64_t m = (int64_t)1 << l;
    return A->nid[l][((int64_t)(z >> 3) * m + (y >> 3)) * m + (x >> 3)];
}

static int64_t amr_slot(int x, int y, int z) { return ((int64_t)(z & 7) * 8 + (y & 7)) * 8 + (x & 7); }

/* 0: no such cell, 1: leaf cell, 2: refined cell */
static int amr_type(const amr *A, int l, int x, int y, int z)
{
    const int64_t nd = amr_node(A, l, x, y, z);
    if (nd < 0) return 0;
    return A->leaf[nd] ? 1 : 2;
}

static const double *amr_moments(const amr *A, int l, int x, int y, int z)
{
    return &A->M[((size_t)amr_node(A, l, x, y, z) * 512 + (size_t)amr_slot(x, y, z)) * (size_t)A->s.n];
}

static double amr_mass(const amr *A, const double *rho, int l, int x, int y, int z)
{
    const double hl = amr_h(A, l);
    return rho[A->first[amr_node(A, l, x, y, z)] + amr_slot(x, y, z)] * hl * hl * hl;
}

static void amr_centre(const amr *A, int l, int x, int y, int z, double out[3])
{
    const double hl = amr_h(A, l);
    out[0] = (x + 0.5) * hl; out[1] = (y + 0.5) * hl; out[2] = (z + 0.5) * hl;
}

/* P2M at every leaf cell, M2M into every refined cell, finest level first */
static void amr_upward(amr *A, const double *rho)
{
    const int nc = A->s.n;
    for (int l = A->Lmax; l >= 0; --l) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t i = 0; i < A->nn; ++i) {
            if (A->lvl[i] != l) continue;
            const int bx = 8 * A->crd[3 * i], by = 8 * A->crd[3 * i + 1], bz = 8 * A->crd[3 * i + 2];
            const double hl = amr_h(A, l), h3 = hl * hl * hl;
            for (int k = 0; k < 512; ++k) {
                const int x = bx + (k & 7), y = by + ((k >> 3) & 7), z = bz + (k >> 6);
                double *Mc = &A->M[((size_t)i * 512 + (size_t)k) * (size_t)nc];
                if (A->leaf[i]) {
                    Mc[0] = rho[A->first[i] + k] * h3;
                    continue;
                }
                double zc[3], zk[3], d[3];
                amr_centre(A, l, x, y, z, zc);
                for (int b = 0; b < 8; ++b) {
                    const int cx = 2 * x + (b & 1), cy = 2 * y + ((b >> 1) & 1), cz = 2 * z + (b >> 2);
                    amr_centre(A, l + 1, cx, cy, cz, zk);
                    for (int t = 0; t < 3; ++t) d[t] = zk[t] - zc[t];
                    m2m(&A->s, d, amr_moments(A, l + 1, cx, cy, cz), A->s.p, Mc);
                }
            }
        }
    }
}

static int amr_near(const amr *A, int dx, int dy, int dz) { return (double)(dx * dx + dy * dy + dz * dz) <= A->r2; }

static int amr_m2l_rule(const amr *A, int l, const int a[3], const int b[3])
{
    if (a[0] == b[0] && a[1] == b[1] && a[2] == b[2]) return 0;
    if (amr_near(A, b[0] - a[0], b[1] - a[1], b[2] - a[2])) return 0;
    if (l == 0) return 1;
    return amr_near(A, (b[0] >> 1) - (a[0] >> 1), (b[1] >> 1) - (a[1] >> 1), (b[2] >> 1) - (a[2] >> 1));
}

/* Every partner of one leaf cell (level li, cell c): fn(kind, l, B, arg) is
 * called once per M2L partner (kind 0: cell B of level l) and once per P2P
 * partner (kind 1: leaf cell B of level l).  Returns -2 when a near refined
 * cell has a child that is not a leaf (the tree is not 2:1 balanced). */
typedef void (*amr_visit)(int kind, int l, const int B[3], void *arg);

static int amr_partners(const amr *A, int li, const int c[3], amr_visit fn, void *arg)
{
    for (int l = 0; l <= li; ++l) {
        const int sh = li - l, n = 8 << l;
        const int a[3] = {c[0] >> sh, c[1] >> sh, c[2] >> sh};
        int lo[3], hi[3];
        for (int t = 0; t < 3; ++t) {
            if (l == 0) { lo[t] = 0; hi[t] = n - 1; continue; }
            const int q = a[t] >> 1;
            lo[t] = 2 * (q - A->reach); hi[t] = 2 * (q + A->reach) + 1;
            if (lo[t] < 0) lo[t] = 0;
            if (hi[t] > n - 1) hi[t] = n - 1;
        }
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) {
                    const int B[3] = {x, y, z};
                    if (amr_type(A, l, x, y, z) && amr_m2l_rule(A, l, a, B)) fn(0, l, B, arg);
                }
    }
    /* near cells of the sink's own level, and of its parent's level */
    for (int up = 0; up <= 1 && up <= li; ++up) {
        const int l = li - up;
        const int a[3] = {c[0] >> up, c[1] >> up, c[2] >> up};
        for (int z = a[2] - A->reach; z <= a[2] + A->reach; ++z)
            for (int y = a[1] - A->reach; y <= a[1] + A->reach; ++y)
                for (int x = a[0] - A->reach; x <= a[0] + A->reach; ++x) {
                    if (x == a[0] && y == a[1] && z == a[2]) continue;
                    if (!amr_near(A, x - a[0], y - a[1], z - a[2])) continue;
                    const int t = amr_type(A, l, x, y, z);
                    const int B[3] = {x, y, z};
                    if (t == 1) {
                        fn(1, l, B, arg);              /* same-level leaf, or a coarser leaf near the parent */
                    } else if (t == 2 && up == 0) {    /* refined near cell: its children */
                        for (int b = 0; b < 8; ++b) {
                            const int Bc[3] = {2 * x + (b & 1), 2 * y + ((b >> 1) & 1), 2 * z + (b >> 2)};
                            if (amr_type(A, l + 1, Bc[0], Bc[1], Bc[2]) != 1) return -2;
                            fn(1, l + 1, Bc, arg);
                        }
                    }
                }
    }
    return 0;
}

typedef struct {
    const amr *A;
    const double *rho;
    int li, c[3];
    double xi[3];
    double *Ci, *CA, *D, *Rs;
    double phi, g[3];
} amr_eval;

static void amr_eval_visit(int kind, int l, const int B[3], void *arg)
{
    amr_eval *E = arg;
    const amr *A = E->A;
    double zB[3];
    amr_centre(A, l, B[0], B[1], B[2], zB);
    if (kind == 1) {
        p2p(A->G, E->xi, zB, amr_mass(A, E->rho, l, B[0], B[1], B[2]), &E->phi, E->g);
        return;
    }
    /* M2L from B into the sink's ancestor of level l, re-expanded exactly to the sink centre */
    const int sh = E->li - l;
    const int c[3] = {E->c[0] >> sh, E->c[1] >> sh, E->c[2] >> sh};
    double zA[3], R[3], d[3];
    amr_centre(A, l, c[0], c[1], c[2], zA);
    for (int t = 0; t < 3; ++t) { R[t] = zA[t] - zB[t]; d[t] = E->xi[t] - zA[t]; }
    memset(E->CA, 0, sizeof(double) * (size_t)A->s.n);
    m2l(&A->s, A->G, R, amr_moments(A, l, B[0], B[1], B[2]), A->s.p, E->CA, E->D, E->Rs);
    l2l(&A->s, d, E->CA, E->Ci);
}

/* leaf cell index -> (level, cell coordinates) */
static int amr_locate(const amr *A, int64_t cell, int *li, int c[3])
{
    if (cell < 0 || cell >= A->ncell) return -1;
    const int64_t i = A->leaf_node[cell / 512], k = cell % 512;
    *li = A->lvl[i];
    c[0] = 8 * A->crd[3 * i] + (int)(k & 7);
    c[1] = 8 * A->crd[3 * i + 1] + (int)((k >> 3) & 7);
    c[2] = 8 * A->crd[3 * i + 2] + (int)(k >> 6);
    return 0;
}

/* FMM forward on an adaptive octree, evaluated per sink (leaf cell indices):
 * phi[s] and g[k * nsink + s]. */
int oracle_amr_sinks(int64_t nn, const int32_t *lvl, const int32_t *crd, const uint8_t *leaf, int p,
                     double theta, double h, double G, const double *rho, int64_t nsink, const int64_t *sinks,
                     double *phi, double *g)
{
    amr A;
    if (amr_init(&A, nn, lvl, crd, leaf, p, theta, h, G)) { amr_free(&A); return -1; }
    amr_upward(&A, rho);
    const int nc = A.s.n, ex = e_k(&A.s, 0), ey = e_k(&A.s, 1), ez = e_k(&A.s, 2);
    int rc = 0;
#pragma omp parallel
    {
        amr_eval E;
        E.A = &A; E.rho = rho;
        E.Ci = malloc(sizeof(double) * nc); E.CA = malloc(sizeof(double) * nc);
        E.D = malloc(sizeof(double) * nc); E.Rs = malloc(sizeof(double) * scratch_len(&A.s));
#pragma omp for schedule(dynamic, 4)
        for (int64_t s = 0; s < nsink; ++s) {
            int *c = E.c;
            if (amr_locate(&A, sinks[s], &E.li, c)) {
#pragma omp atomic write
                rc = -1;
                continue;
            }
            amr_centre(&A, E.li, c[0], c[1], c[2], E.xi);
            memset(E.Ci, 0, sizeof(double) * nc);
            E.phi = 0.0; E.g[0] = E.g[1] = E.g[2] = 0.0;
            if (amr_partners(&A, E.li, c, amr_eval_visit, &E)) {
#pragma omp atomic write
                rc = -2;
                continue;
            }
            phi[s] = E.Ci[0] + E.phi;
            g[s] = E.g[0] - (p >= 1 ? E.Ci[ex] : 0.0);
            g[nsink + s] = E.g[1] - (p >= 1 ? E.Ci[ey] : 0.0);
            g[2 * nsink + s] = E.g[2] - (p >= 1 ? E.Ci[ez] : 0.0);
        }
        free(E.Ci); free(E.CA); free(E.D); free(E.Rs);
    }
    amr_free(&A);
    return rc;
}

/* Direct Newtonian sum over all leaf cells of an adaptive octree (point
 * masses rho h_l^3 at the cell centres, i != j), at the given sinks. */
int oracle_amr_direct(int64_t nn, const int32_t *lvl, const int32_t *crd, const uint8_t *leaf, double h,
                      double G, const double *rho, int64_t nsink, const int64_t *sinks, double *phi, double *g)
{
    amr A;
    if (amr_init(&A, nn, lvl, crd, leaf, 0, 1.0, h, G)) { amr_free(&A); return -1; }
    double *pos = malloc(sizeof(double) * 3 * (size_t)A.ncell), *mass = malloc(sizeof(double) * (size_t)A.ncell);
    if (!pos || !mass) { free(pos); free(mass); amr_free(&A); return -1; }
    for (int64_t i = 0; i < nn; ++i) {
        if (!leaf[i]) continue;
        const int l = lvl[i];
        const double hl = amr_h(&A, l);
        for (int k = 0; k < 512; ++k) {
            const int64_t j = A.first[i] + k;
            amr_centre(&A, l, 8 * crd[3 * i] + (k & 7), 8 * crd[3 * i + 1] + ((k >> 3) & 7), 8 * crd[3 * i + 2] + (k >> 6),
                       &pos[3 * j]);
            mass[j] = rho[j] * hl * hl * hl;
        }
    }
    int rc = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < nsink; ++s) {
        const int64_t i = sinks[s];
        if (i < 0 || i >= A.ncell) {
#pragma omp atomic write
            rc = -1;
            continue;
        }
        double ph = 0.0, gg[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < A.ncell; ++j)
            if (j != i) p2p(G, &pos[3 * i], &pos[3 * j], mass[j], &ph, gg);
        phi[s] = ph;
        g[s] = gg[0]; g[nsink + s] = gg[1]; g[2 * nsink + s] = gg[2];
    }
    free(pos); free(mass);
    amr_free(&A);
    return rc;
}

/* Pair cover of one sink: mult[j] = how many times the sink's partners
 * account for leaf cell j (an M2L partner accounts for every leaf cell under
 * it).  Exact cover: 1 for every j other than the sink, 0 for the sink. */
typedef struct { const amr *A; int32_t *mult; } amr_cov;

static void amr_mark(const amr *A, int l, int x, int y, int z, int32_t *mult)
{
    const int64_t nd = amr_node(A, l, x, y, z);
    if (nd < 0) return;
    if (A->leaf[nd]) { mult[A->first[nd] + amr_slot(x, y, z)] += 1; return; }
    for (int b = 0; b < 8; ++b) amr_mark(A, l + 1, 2 * x + (b & 1), 2 * y + ((b >> 1) & 1), 2 * z + (b >> 2), mult);
}

static void amr_cover_visit(int kind, int l, const int B[3], void *arg)
{
    amr_cov *V = arg;
    (void)kind;
    amr_mark(V->A, l, B[0], B[1], B[2], V->mult);
}

int oracle_amr_cover(int64_t nn, const int32_t *lvl, const int32_t *crd, const uint8_t *leaf, double theta,
                     int64_t sink, int32_t *mult)
{
    amr A;
    if (amr_init(&A, nn, lvl, crd, leaf, 0, theta, 1.0, 1.0)) { amr_free(&A); return -1; }
    int li, c[3];
    int rc = amr_locate(&A, sink, &li, c);
    if (!rc) {
        memset(mult, 0, sizeof(int32_t) * (size_t)A.ncell);
        amr_cov V = {&A, mult};
        rc = amr_partners(&A, li, c, amr_cover_visit, &V);
    }
    amr_free(&A);
    return rc;
}

/* ======================================================================== */
/* Angular-momentum correction (spin torque per unit mass)                   */
/* ======================================================================== */
/*
 * Sec. 4.3 names an angular-momentum-conserving correction of the FMM without
 * its formula.  Reading used here.  For one ordered M2L pair (A <- B) with
 * R = z_A - z_B, the truncated pair energy depends on the fixed expansion
 * centres, and its derivative in z_A is the boundary term of total order p+1:
 *   E_k = sum_{|a|+|b|=p} (1/a!) M_A^a ((-1)^|b| / b!) K^(a+b+e_k)(R) M_B^b,
 * K = -G/r.  The particles' total orbital torque equals 1/2 the sum over
 * ordered pairs of R x E.  E splits over A's members i as m_i e_i with
 *   e_i,k = sum_{|a|+|b|=p} (1/a!) (x_i - z_A)^a ((-1)^|b| / b!) K^(a+b+e_k)(R) M_B^b,
 * so the spin torque per unit mass
 *   t_i = -1/2 sum over the M2L pairs (A <- B) of i's ancestors A of R x e_i
 * makes sum_i m_i (x_i x g_i + t_i) vanish exactly, pair by pair, and is
 * linear in rho like g.  Leaf pairs of monopoles carry no such term (every
 * product above has a factor of order >= 1 that vanishes for them).
 * Uniform trees; t[k * nsink + s] at the given leaf cells (dense indices).
 */
int oracle_amcorr_sinks(int L, int p, double theta, double h, double G, const double *rho, int64_t nsink,
                        const int64_t *sinks, double *t)
{
    fmm F;
    mset s1;
    if (fmm_alloc(&F, L, p, theta, h, G) || mset_init(&s1, p + 1)) { fmm_free(&F); return -1; }
    const tree *T = &F.T;
    const mset *s = &F.s;
    const int nc = s->n, n = nlev(L);
    upward(&F, rho);
#pragma omp parallel
    {
        double *D = malloc(sizeof(double) * (size_t)s1.n);
        double *Rs = malloc(sizeof(double) * scratch_len(&s1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < nsink; ++q) {
            const int64_t i = sinks[q];
            const int ix = (int)(i % n), iy = (int)((i / n) % n), iz = (int)(i / ((int64_t)n * n));
            double xi[3], zA[3], zB[3], R[3], d[3], tt[3] = {0.0, 0.0, 0.0};
            centre(T, L, ix, iy, iz, xi);
            for (int l = 0; l < L; ++l) {
                const int nl = nlev(l), sh = L - l;
                const int A[3] = {ix >> sh, iy >> sh, iz >> sh};
                centre(T, l, A[0], A[1], A[2], zA);
                for (int k = 0; k < 3; ++k) d[k] = xi[k] - zA[k];
                box bx = m2l_candidates(T, l, A);
                for (int bz = bx.lo[2]; bz <= bx.hi[2]; ++bz)
                    for (int by = bx.lo[1]; by <= bx.hi[1]; ++by)
                        for (int bxx = bx.lo[0]; bxx <= bx.hi[0]; ++bxx) {
                            const int B[3] = {bxx, by, bz};
                            if (!m2l_rule(T, l, A, B)) continue;
                            centre(T, l, bxx, by, bz, zB);
                            for (int k = 0; k < 3; ++k) R[k] = zA[k] - zB[k];
                            inv_r_derivs(&s1, R[0], R[1], R[2], D, Rs);
                            const double *MB = &F.M[l][cid(nl, bxx, by, bz) * nc];
                            double e[3] = {0.0, 0.0, 0.0};
                            for (int ia = 0; ia < nc; ++ia)
                                for (int ib = 0; ib < nc; ++ib) {
                                    if (s->order[ia] + s->order[ib] != p) continue;
                                    const int *a = s->a[ia], *b = s->a[ib];
                                    const double sgn = (s->order[ib] & 1) ? -1.0 : 1.0;
                                    const double c = mpow(d, a[0], a[1], a[2]) * s->ifact[ia] * sgn * s->ifact[ib] * MB[ib];
                                    for (int k = 0; k < 3; ++k)
                                        e[k] += c * (-G) * D[mset_find(&s1, a[0] + b[0] + (k == 0), a[1] + b[1] + (k == 1),
                                                                      a[2] + b[2] + (k == 2))];
                                }
                            tt[0] += -0.5 * (R[1] * e[2] - R[2] * e[1]);
                            tt[1] += -0.5 * (R[2] * e[0] - R[0] * e[2]);
                            tt[2] += -0.5 * (R[0] * e[1] - R[1] * e[0]);
                        }
            }
            t[q] = tt[0]; t[nsink + q] = tt[1]; t[2 * nsink + q] = tt[2];
        }
        free(D); free(Rs);
    }
    mset_free(&s1);
    fmm_free(&F);
    return 0;
}
