/*
 * Plain FP64 CPU reference ("oracle") for the IFGF operator of Bauinger and
 * Bruno, "IFGF: Interpolated Factored Green Function method" (arXiv
 * 2010.02857).
 *
 * TEST INFRASTRUCTURE ONLY.  It is written to be read against the paper, not
 * to be fast: every loop follows the order of Algorithm 1 (Sec. 3.3.3), every
 * formula cites the equation it restates, and OpenMP only splits the outer
 * box loops (with atomic accumulation) so that the larger test problems finish
 * in seconds.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library; the GPU library shares no code with
 * it and never calls it.
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * design notes of the repository):
 *   R1  Chebyshev coefficients (Sec. 3.2, eq. defchebyshevcoeffsandpoints):
 *       the printed weights mix endpoint-grid weights with first-kind nodes
 *       and do not reproduce constants; the standard first-kind discrete
 *       transform a_i = 2/(b_i n) sum_k u(t_k) T_i(t_k) is used.
 *   R2  Nodes are first-kind Chebyshev nodes t_k = cos((2k+1) pi / (2n)).
 *   R3  P_s, P_ang are node counts per direction (accuracy orders).
 *   R4  The factor 1/(4 pi) lives in the centred factor only (eq. factored_f);
 *       eq. factor_r's extra 1/(4 pi) is not used.
 *   R5  Cone refinement multiplies the interval counts going up the tree:
 *       n_{.,d-1} = a_d n_{.,d} with a_d = 2 iff 2 kappa H_d > 1 (Sec. 3.3.1).
 *   R6  Root box: centre = bounding-box midpoint, side = largest extent, the
 *       box bounding the sources and any distinct targets; box indices are
 *       clamped to the last box on the upper faces.
 *   R7  Cone index = the half-open interval of eq. (defconedomain) holding
 *       the coordinate: floor(coordinate / interval length), where a value
 *       within 1e-10 (in interval units) below a boundary counts as on it
 *       and so falls in the interval above; clamped to the last interval;
 *       phi = atan2(y, x) shifted into [0, 2 pi) and wrapped at 2 pi.
 *   R8  Relevance rule (ii) marks the child cones containing the nodes of the
 *       parent's relevant cones (the node-based narrative of Sec. 3.3.2).
 *   R9  The self term is skipped by index.
 *   R10 Levels: D = 1 + round(log2(4 H_1 / lambda)) so that H_D ~ lambda/4
 *       (Sec. 4); for kappa = 0 the smallest D >= 2 with at most 8 points per
 *       relevant leaf box.
 *   R16 Adaptive octree (named in Sec. 4 and Sec. 5 as the remedy for uneven
 *       point counts per box, with no algorithm given): with leaf_max > 0 a
 *       box of level d >= 2 holding at most leaf_max points (sources and
 *       distinct targets together) is a leaf and is split no further; the
 *       boxes below it take no part as sources.  Its sources reach the
 *       targets of its neighbour boxes on its own level directly, its
 *       relevant cones (rules (i) and (ii) as for any box) get their node
 *       values directly from its sources, and from there on it is treated
 *       like any box of its level.  Targets keep their boxes on every level,
 *       so that the cousin relation of eq. (defcousinboxes) stays as it is.
 *       leaf_max = 0 is the tree of Sec. 3.3.1 (every leaf on level D).
 */
#include "ifgf_oracle.h"

#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cplx;

static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------ kernel */

static double norm3(const double* v) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

static double dist3(const double* a, const double* b)
{
    double v[3] = {a[0] - b[0], a[1] - b[1], a[2] - b[2]};
    return norm3(v);
}

/* G(x, x') = e^{i kappa r} / (4 pi r), r = |x - x'|  (eq. greensfunction). */
static cplx green_r(double kappa, double r)
{
    return (cos(kappa * r) + I * sin(kappa * r)) / (4.0 * PI * r);
}

/* Analytic factor centred at c (eq. factored_f with x_S = c):
 *   g_c(x, y) = |x - c| / |x - y| * exp(i kappa (|x - y| - |x - c|)).
 * The difference of the two radii is formed as
 *   (|y - c|^2 - 2 (x - c).(y - c)) / (|x - y| + |x - c|),
 * which is the same number in exact arithmetic and keeps its relative accuracy
 * when x lies far from c (small s).                                        */
static cplx analytic_factor(double kappa, const double* c, const double* x, const double* y)
{
    double u[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    double w[3] = {y[0] - c[0], y[1] - c[1], y[2] - c[2]};
    double ru = norm3(u);
    double rxy = dist3(x, y);
    double num = (w[0] * w[0] + w[1] * w[1] + w[2] * w[2]) - 2.0 * (u[0] * w[0] + u[1] * w[1] + u[2] * w[2]);
    double diff = num / (rxy + ru);
    return (ru / rxy) * (cos(kappa * diff) + I * sin(kappa * diff));
}

void oracle_green(double kappa, const double* x, const double* y, double* out)
{
    cplx g = green_r(kappa, dist3(x, y));
    out[0] = creal(g);
    out[1] = cimag(g);
}

void oracle_analytic_factor(double kappa, const double* c, const double* x, const double* y, double* out)
{
    cplx g = analytic_factor(kappa, c, x, y);
    out[0] = creal(g);
    out[1] = cimag(g);
}

/* ---------------------------------------------------------- direct O(N^2) */

/* eq. (field1): out_r[i] = sum_{j != skip[i]} a_r[j] G(t_i, x_j). */
int oracle_direct(const double* pts, int64_t n, const double* dens, int32_t nrhs, double kappa,
                  const double* tpos, const int64_t* skip, int64_t m, double* out)
{
    if (!pts || !dens || !tpos || !out || n < 1 || m < 0 || nrhs < 1) return -1;
    const cplx* a = (const cplx*)dens;
    cplx* o = (cplx*)out;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        for (int32_t r = 0; r < nrhs; ++r) {
            cplx acc = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                if (skip && skip[i] == j) continue;
                acc += a[(int64_t)r * n + j] * green_r(kappa, dist3(&tpos[3 * i], &pts[3 * j]));
            }
            o[(int64_t)r * m + i] = acc;
        }
    }
    return 0;
}

/* grad_t G(t, x) = G (i kappa - 1/r) (t - x) / r. */
static void green_grad(double kappa, const double* t, const double* x, cplx* g)
{
    double v[3] = {t[0] - x[0], t[1] - x[1], t[2] - x[2]};
    double r = norm3(v);
    cplx f = green_r(kappa, r) * (I * kappa - 1.0 / r) / r;
    g[0] = f * v[0];
    g[1] = f * v[1];
    g[2] = f * v[2];
}

int oracle_direct_grad(const double* pts, int64_t n, const double* dens, int32_t nrhs, double kappa,
                       const double* tpos, const int64_t* skip, int64_t m, double* grad)
{
    if (!pts || !dens || !tpos || !grad || n < 1 || m < 0 || nrhs < 1) return -1;
    const cplx* a = (const cplx*)dens;
    cplx* o = (cplx*)grad;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        for (int32_t r = 0; r < nrhs; ++r) {
            cplx acc[3] = {0.0, 0.0, 0.0};
            for (int64_t j = 0; j < n; ++j) {
                if (skip && skip[i] == j) continue;
                cplx g[3];
                green_grad(kappa, &tpos[3 * i], &pts[3 * j], g);
                for (int c = 0; c < 3; ++c) acc[c] += a[(int64_t)r * n + j] * g[c];
            }
            for (int c = 0; c < 3; ++c) o[((int64_t)r * m + i) * 3 + c] = acc[c];
        }
    }
    return 0;
}

/* ------------------------------------------------------------- Chebyshev */

/* First-kind nodes x_k = cos((2k+1) pi / (2n)) (Sec. 3.2). */
void oracle_cheb_nodes(int32_t n, double* t)
{
    for (int32_t k = 0; k < n; ++k) t[k] = cos((2.0 * k + 1.0) * PI / (2.0 * n));
}

/* T_0..T_{n-1} at t and their derivatives, by the three-term recurrence. */
static void cheb_T(int n, double t, double* T, double* dT)
{
    T[0] = 1.0;
    if (dT) dT[0] = 0.0;
    if (n > 1) {
        T[1] = t;
        if (dT) dT[1] = 1.0;
    }
    for (int i = 2; i < n; ++i) {
        T[i] = 2.0 * t * T[i - 1] - T[i - 2];
        if (dT) dT[i] = 2.0 * T[i - 1] + 2.0 * t * dT[i - 1] - dT[i - 2];
    }
}

/* One-dimensional discrete Chebyshev transform (reading R1):
 *   a_i = 2/(b_i n) sum_k u(x_k) T_i(x_k),  b_0 = 2, b_i = 1 otherwise,
 * with T_i(x_k) = cos(i (2k+1) pi / (2n)).  u and a have stride `st`. */
static void cheb_coeffs_1d(int n, const cplx* u, int st, cplx* a)
{
    for (int i = 0; i < n; ++i) {
        cplx acc = 0.0;
        for (int k = 0; k < n; ++k) acc += u[k * st] * cos(i * (2.0 * k + 1.0) * PI / (2.0 * n));
        a[i * st] = acc * (2.0 / ((i == 0 ? 2.0 : 1.0) * n));
    }
}

/* Coefficients of the tensor interpolant through values u[a][b][c] on the
 * ps x pang x pang node grid: the three-dimensional problem is solved as a
 * sequence of one-dimensional problems along s, theta and phi (Sec. 3.2). */
static void cheb_coeffs_3d(int ps, int pa, const cplx* u, cplx* A)
{
    int P = ps * pa * pa;
    cplx* t1 = (cplx*)malloc(sizeof(cplx) * P);
    cplx* t2 = (cplx*)malloc(sizeof(cplx) * P);
    /* along phi (innermost index, stride 1) */
    for (int a = 0; a < ps; ++a)
        for (int b = 0; b < pa; ++b) cheb_coeffs_1d(pa, &u[(a * pa + b) * pa], 1, &t1[(a * pa + b) * pa]);
    /* along theta (stride pa) */
    for (int a = 0; a < ps; ++a)
        for (int c = 0; c < pa; ++c) cheb_coeffs_1d(pa, &t1[a * pa * pa + c], pa, &t2[a * pa * pa + c]);
    /* along s (stride pa*pa) */
    for (int b = 0; b < pa; ++b)
        for (int c = 0; c < pa; ++c) cheb_coeffs_1d(ps, &t2[b * pa + c], pa * pa, &A[b * pa + c]);
    free(t1);
    free(t2);
}

/* Evaluation sum_{i,j,l} A_ijl T_i(ts) T_j(tt) T_l(tp) (eq.
 * defchebyshevinterpooperator in each variable); with dA != NULL also the
 * three partial derivatives with respect to (ts, tt, tp). */
static cplx cheb_eval_3d(int ps, int pa, const cplx* A, int stride, const double* loc, cplx* dA)
{
    double Ts[16], Tt[16], Tp[16], dTs[16], dTt[16], dTp[16];
    cheb_T(ps, loc[0], Ts, dTs);
    cheb_T(pa, loc[1], Tt, dTt);
    cheb_T(pa, loc[2], Tp, dTp);
    cplx v = 0.0, d0 = 0.0, d1 = 0.0, d2 = 0.0;
    for (int i = 0; i < ps; ++i)
        for (int j = 0; j < pa; ++j)
            for (int l = 0; l < pa; ++l) {
                cplx c = A[((i * pa + j) * pa + l) * stride];
                v += c * Ts[i] * Tt[j] * Tp[l];
                if (dA) {
                    d0 += c * dTs[i] * Tt[j] * Tp[l];
                    d1 += c * Ts[i] * dTt[j] * Tp[l];
                    d2 += c * Ts[i] * Tt[j] * dTp[l];
                }
            }
    if (dA) {
        dA[0] = d0;
        dA[1] = d1;
        dA[2] = d2;
    }
    return v;
}

void oracle_cheb_interp3(int32_t ps, int32_t pang, const double* u, double ts, double tt, double tp,
                         double* out)
{
    int P = ps * pang * pang;
    cplx* A = (cplx*)malloc(sizeof(cplx) * P);
    cheb_coeffs_3d(ps, pang, (const cplx*)u, A);
    double loc[3] = {ts, tt, tp};
    cplx v = cheb_eval_3d(ps, pang, A, 1, loc, NULL);
    out[0] = creal(v);
    out[1] = cimag(v);
    free(A);
}

/* ----------------------------------------------------------- cone geometry */

/* eta = sqrt(3)/3: targets at least one box side away from the box have
 * s <= eta (Sec. 3.1). */
static double eta_const(void) { return sqrt(3.0) / 3.0; }

/* Spherical coordinates of x about centre c (eq. defparametrizationr) in the
 * singularity-resolving variable s = h / r, h = sqrt(3) H / 2 (eqs.
 * defparametrizationins, def_eps), the cone (eqs. defconedomain,
 * defconedomainproduct) that contains them and the local coordinates in
 * [-1, 1] of the point inside that cone. */
void oracle_cone_coords(const double* c, double H, int32_t ns, int32_t nc, const double* x, int32_t* idx,
                        double* loc, double* sth)
{
    double v[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    double r = norm3(v);
    double h = sqrt(3.0) * H / 2.0;
    double s = h / r;
    double theta = atan2(sqrt(v[0] * v[0] + v[1] * v[1]), v[2]);
    double phi = atan2(v[1], v[0]);
    if (phi < 0.0) phi += 2.0 * PI;
    double ds = eta_const() / ns, dth = PI / nc, dph = PI / nc;
    /* Interval index of coordinate / interval length q.  The intervals of
     * eq. (defconedomain) are half-open, so a point on a boundary belongs to
     * the interval above it; q within 1e-10 below an integer counts as on
     * that boundary (reading R7).  phi wraps around at 2 pi. */
    const double tie = 1e-10;
    double qs = s / ds, qt = theta / dth, qp = phi / dph;
    int32_t is = (int32_t)floor(qs + tie), it = (int32_t)floor(qt + tie), ip = (int32_t)floor(qp + tie);
    if (ip >= 2 * nc) {
        ip -= 2 * nc;
        qp -= 2 * nc;
    }
    if (is > ns - 1) is = ns - 1;
    if (it > nc - 1) it = nc - 1;
    if (ip > 2 * nc - 1) ip = 2 * nc - 1;
    if (is < 0) is = 0;
    if (it < 0) it = 0;
    if (ip < 0) ip = 0;
    idx[0] = is;
    idx[1] = it;
    idx[2] = ip;
    loc[0] = 2.0 * (qs - is) - 1.0;
    loc[1] = 2.0 * (qt - it) - 1.0;
    loc[2] = 2.0 * (qp - ip) - 1.0;
    if (sth) {
        sth[0] = s;
        sth[1] = theta;
        sth[2] = phi;
    }
}

/* x = c + x^d(s, theta, phi) for the point with local coordinates loc in cone
 * idx (eqs. defparametrizationr, parametrizationleveldependent, interp_pts). */
void oracle_cone_point(const double* c, double H, int32_t ns, int32_t nc, const int32_t* idx,
                       const double* loc, double* x)
{
    double h = sqrt(3.0) * H / 2.0;
    double ds = eta_const() / ns, dth = PI / nc, dph = PI / nc;
    double s = ds * (idx[0] + 0.5 * (loc[0] + 1.0));
    double th = dth * (idx[1] + 0.5 * (loc[1] + 1.0));
    double ph = dph * (idx[2] + 0.5 * (loc[2] + 1.0));
    double r = h / s;
    x[0] = c[0] + r * sin(th) * cos(ph);
    x[1] = c[1] + r * sin(th) * sin(ph);
    x[2] = c[2] + r * cos(th);
}

static int64_t cone_id(const int32_t* idx, int nc) { return ((int64_t)idx[0] * nc + idx[1]) * (2 * nc) + idx[2]; }

static void cone_idx(int64_t id, int nc, int32_t* idx)
{
    idx[2] = (int32_t)(id % (2 * nc));
    idx[1] = (int32_t)((id / (2 * nc)) % nc);
    idx[0] = (int32_t)(id / (2 * (int64_t)nc * nc));
}

/* --------------------------------------------------------- box hierarchy */

typedef struct {
    double H;            /* box side H_d (eq. defboxsizesandcenters)            */
    int64_t nbox;        /* relevant boxes R_B^d                                */
    uint64_t* key;       /* sorted packed multi-indices (0-based)               */
    int64_t* src_off;    /* CSR: sources in each box                            */
    int64_t* src;
    int64_t* tgt_off;    /* CSR: targets in each box                            */
    int64_t* tgt;
    int64_t* parent;     /* P B (index at level d-1)                            */
    int64_t* chl_off;    /* Q B (indices at level d+1)                          */
    int64_t* chl;
    int64_t* nbr_off;    /* N B, including B itself                             */
    int64_t* nbr;
    int64_t* cou_off;    /* M B (eq. defcousinboxes)                            */
    int64_t* cou;
    int ns, nc;          /* cone intervals n_{s,d}, n_{C,d}                     */
    int64_t* cone_off;   /* R_C B: sorted relevant cone ids per box             */
    int64_t* cone;
    uint8_t* active;     /* the box is part of the (adaptive) source tree       */
    uint8_t* leaf;       /* an active box that is not split further             */
} level_t;

static uint64_t pack3(const int64_t* k) { return ((uint64_t)k[0] << 42) | ((uint64_t)k[1] << 21) | (uint64_t)k[2]; }

static void unpack3(uint64_t key, int64_t* k)
{
    k[0] = (int64_t)(key >> 42);
    k[1] = (int64_t)((key >> 21) & ((1u << 21) - 1));
    k[2] = (int64_t)(key & ((1u << 21) - 1));
}

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

static int cmp_i64(const void* a, const void* b)
{
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

static int64_t find_key(const level_t* L, uint64_t key)
{
    int64_t lo = 0, hi = L->nbox - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (L->key[mid] == key) return mid;
        if (L->key[mid] < key) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

/* Level-d multi-index of x: integer part of (x - corner) / H_d, clamped to the
 * 2^{d-1} boxes per axis (Sec. 3.3.2 and reading R6). */
static void box_of(const double* x, const double* corner, double H, int64_t nb, int64_t* k)
{
    for (int a = 0; a < 3; ++a) {
        double q = floor((x[a] - corner[a]) / H);
        int64_t v = (int64_t)q;
        if (q < 0.0) v = 0;
        if (v > nb - 1) v = nb - 1;
        k[a] = v;
    }
}

/* Box centre x_k^d = x_1^1 - H_1/2 + H_d/2 (2k - 1) with 1-based k, i.e.
 * (2 k0 + 1) with the 0-based k0 stored here (eq. defboxsizesandcenters). */
static void box_centre(const double* x1, double H1, double Hd, uint64_t key, double* c)
{
    int64_t k[3];
    unpack3(key, k);
    for (int a = 0; a < 3; ++a) c[a] = x1[a] - H1 / 2.0 + Hd / 2.0 * (2.0 * k[a] + 1.0);
}

static int64_t* csr_from_owner(const int64_t* owner, int64_t cnt, int64_t nbox, int64_t** off_out)
{
    int64_t* off = (int64_t*)calloc(nbox + 1, sizeof(int64_t));
    int64_t* list = (int64_t*)malloc(sizeof(int64_t) * (cnt > 0 ? cnt : 1));
    for (int64_t i = 0; i < cnt; ++i) off[owner[i] + 1]++;
    for (int64_t b = 0; b < nbox; ++b) off[b + 1] += off[b];
    int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (nbox + 1));
    memcpy(pos, off, sizeof(int64_t) * (nbox + 1));
    for (int64_t i = 0; i < cnt; ++i) list[pos[owner[i]]++] = i;
    free(pos);
    *off_out = off;
    return list;
}

static void free_level(level_t* L)
{
    free(L->key);
    free(L->src_off);
    free(L->src);
    free(L->tgt_off);
    free(L->tgt);
    free(L->parent);
    free(L->chl_off);
    free(L->chl);
    free(L->nbr_off);
    free(L->nbr);
    free(L->cou_off);
    free(L->cou);
    free(L->cone_off);
    free(L->cone);
    free(L->active);
    free(L->leaf);
}

/* Slot of cone `id` of box b: position of id in the sorted list R_C B. */
static int64_t find_cone(const level_t* L, int64_t b, int64_t id)
{
    int64_t lo = L->cone_off[b], hi = L->cone_off[b + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (L->cone[mid] == id) return mid;
        if (L->cone[mid] < id) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

static uint64_t mix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static void atomic_add_c(double* p, cplx v)
{
#pragma omp atomic
    p[0] += creal(v);
#pragma omp atomic
    p[1] += cimag(v);
}

/* Node (a, b, c) of a ps x pang x pang grid: local coordinates of the
 * first-kind Chebyshev nodes in (s, theta, phi) (eq. interp_pts). */
static void node_loc(int pa, int nu, const double* ts, const double* ta, double* loc)
{
    int a = nu / (pa * pa), b = (nu / pa) % pa, c = nu % pa;
    loc[0] = ts[a];
    loc[1] = ta[b];
    loc[2] = ta[c];
}

/* ------------------------------------------------------------- the method */

/* The node values F_k^d (eq. I_k) of every relevant cone of box b of level
 * Ld, summed directly over the box's sources, into vals[slot][node][rhs]. */
static void direct_node_values(const level_t* Ld, int64_t b, const double* x1, double H1, int P, int pang,
                               const double* tsn, const double* tan_, const double* pts, int64_t n,
                               const cplx* a, int32_t nrhs, double kappa, cplx* vals)
{
    double ctr[3];
    box_centre(x1, H1, Ld->H, Ld->key[b], ctr);
    for (int64_t gi = Ld->cone_off[b]; gi < Ld->cone_off[b + 1]; ++gi) {
        int32_t idx[3];
        cone_idx(Ld->cone[gi], Ld->nc, idx);
        for (int nu = 0; nu < P; ++nu) {
            double loc[3], x[3];
            node_loc(pang, nu, tsn, tan_, loc);
            oracle_cone_point(ctr, Ld->H, Ld->ns, Ld->nc, idx, loc, x);
            for (int32_t r = 0; r < nrhs; ++r) {
                cplx F = 0.0;
                for (int64_t si = Ld->src_off[b]; si < Ld->src_off[b + 1]; ++si) {
                    int64_t j = Ld->src[si];
                    F += a[(int64_t)r * n + j] * analytic_factor(kappa, ctr, x, &pts[3 * j]);
                }
                vals[((size_t)gi * P + nu) * nrhs + r] = F;
            }
        }
    }
}

int oracle_ifgf(const double* pts, int64_t n, const double* dens, int32_t nrhs, double kappa, int32_t levels,
                int32_t ps, int32_t pang, int32_t leaf_ns, int32_t leaf_nc, const double* tpos,
                const int64_t* skip_in, int64_t m, double* out, double* grad, uint64_t* sig,
                oracle_stats* stats)
{
    return oracle_ifgf_ex(pts, n, dens, nrhs, kappa, levels, ps, pang, leaf_ns, leaf_nc, 0, tpos, skip_in, m,
                          out, grad, sig, stats);
}

int oracle_ifgf_ex(const double* pts, int64_t n, const double* dens, int32_t nrhs, double kappa, int32_t levels,
                   int32_t ps, int32_t pang, int32_t leaf_ns, int32_t leaf_nc, int32_t leaf_max,
                   const double* tpos, const int64_t* skip_in, int64_t m, double* out, double* grad,
                   uint64_t* sig, oracle_stats* stats)
{
    if (!pts || !dens || !out || n < 2 || nrhs < 1 || ps < 1 || pang < 1 || ps > 16 || pang > 16 ||
        leaf_ns < 1 || leaf_nc < 1 || levels < 0 || levels > ORACLE_MAX_LEVELS || leaf_max < 0)
        return -1;
    const int distinct_targets = tpos != NULL;
    int64_t* skip_own = NULL;
    const int64_t* skip = skip_in;
    if (!tpos) {
        tpos = pts;
        m = n;
        skip_own = (int64_t*)malloc(sizeof(int64_t) * n);
        for (int64_t i = 0; i < n; ++i) skip_own[i] = i;
        skip = skip_own;
    }
    const cplx* a = (const cplx*)dens;
    const int P = ps * pang * pang;
    const double t_start = omp_get_wtime();   /* T_pre: the hierarchy below */

    /* Root box B_1^1 containing Gamma_N (eq. deffirstbox; reading R6): every
     * point the operator involves, i.e. the sources and, when they are given
     * apart, the targets as well. */
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) lo[c] = hi[c] = pts[c];
    for (int64_t i = 1; i < n; ++i)
        for (int c = 0; c < 3; ++c) {
            if (pts[3 * i + c] < lo[c]) lo[c] = pts[3 * i + c];
            if (pts[3 * i + c] > hi[c]) hi[c] = pts[3 * i + c];
        }
    if (distinct_targets)
        for (int64_t i = 0; i < m; ++i)
            for (int c = 0; c < 3; ++c) {
                if (tpos[3 * i + c] < lo[c]) lo[c] = tpos[3 * i + c];
                if (tpos[3 * i + c] > hi[c]) hi[c] = tpos[3 * i + c];
            }
    double x1[3], H1 = 0.0;
    for (int c = 0; c < 3; ++c) {
        x1[c] = 0.5 * (lo[c] + hi[c]);
        if (hi[c] - lo[c] > H1) H1 = hi[c] - lo[c];
    }
    if (!(H1 > 0.0)) {
        free(skip_own);
        return -2;
    }
    double corner[3] = {x1[0] - H1 / 2.0, x1[1] - H1 / 2.0, x1[2] - H1 / 2.0};

    /* Number of levels (reading R10). */
    int D = levels;
    if (D == 0) {
        if (kappa != 0.0) {
            double lambda = 2.0 * PI / fabs(kappa);
            D = 1 + (int)floor(log2(4.0 * H1 / lambda) + 0.5);
            if (D < 2) D = 2;
            if (D > ORACLE_MAX_LEVELS) D = ORACLE_MAX_LEVELS;
        } else {
            for (D = 2; D < ORACLE_MAX_LEVELS; ++D) {
                double Hd = ldexp(H1, -(D - 1));
                int64_t nb = (int64_t)1 << (D - 1);
                uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * n);
                for (int64_t i = 0; i < n; ++i) {
                    int64_t k[3];
                    box_of(&pts[3 * i], corner, Hd, nb, k);
                    keys[i] = pack3(k);
                }
                qsort(keys, n, sizeof(uint64_t), cmp_u64);
                int64_t nu = 0;
                for (int64_t i = 0; i < n; ++i)
                    if (i == 0 || keys[i] != keys[i - 1]) ++nu;
                free(keys);
                if ((double)n / (double)nu <= 8.0) break;
            }
        }
    }
    if (D < 2) D = 2;

    level_t* L = (level_t*)calloc(D + 2, sizeof(level_t));

    /* Relevant boxes of every level: boxes holding a source or a target
     * (with targets equal to the sources this is R_B^d of Sec. 3.3.1). */
    for (int d = 1; d <= D; ++d) {
        level_t* Ld = &L[d];
        Ld->H = ldexp(H1, -(d - 1));
        int64_t nb = (int64_t)1 << (d - 1);
        uint64_t* sk = (uint64_t*)malloc(sizeof(uint64_t) * n);
        uint64_t* tk = (uint64_t*)malloc(sizeof(uint64_t) * (m > 0 ? m : 1));
        for (int64_t i = 0; i < n; ++i) {
            int64_t k[3];
            box_of(&pts[3 * i], corner, Ld->H, nb, k);
            sk[i] = pack3(k);
        }
        for (int64_t i = 0; i < m; ++i) {
            int64_t k[3];
            box_of(&tpos[3 * i], corner, Ld->H, nb, k);
            tk[i] = pack3(k);
        }
        uint64_t* all = (uint64_t*)malloc(sizeof(uint64_t) * (n + m));
        memcpy(all, sk, sizeof(uint64_t) * n);
        memcpy(all + n, tk, sizeof(uint64_t) * m);
        qsort(all, n + m, sizeof(uint64_t), cmp_u64);
        int64_t nu = 0;
        for (int64_t i = 0; i < n + m; ++i)
            if (i == 0 || all[i] != all[nu - 1]) all[nu++] = all[i];
        Ld->nbox = nu;
        Ld->key = all;
        int64_t* own = (int64_t*)malloc(sizeof(int64_t) * (n > m ? n : m) + 8);
        for (int64_t i = 0; i < n; ++i) own[i] = find_key(Ld, sk[i]);
        Ld->src = csr_from_owner(own, n, nu, &Ld->src_off);
        for (int64_t i = 0; i < m; ++i) own[i] = find_key(Ld, tk[i]);
        Ld->tgt = csr_from_owner(own, m, nu, &Ld->tgt_off);
        free(own);
        free(sk);
        free(tk);
    }

    /* Parents P B and children Q B. */
    for (int d = 1; d <= D; ++d) {
        level_t* Ld = &L[d];
        Ld->parent = (int64_t*)malloc(sizeof(int64_t) * Ld->nbox);
        for (int64_t b = 0; b < Ld->nbox; ++b) {
            if (d == 1) {
                Ld->parent[b] = -1;
                continue;
            }
            int64_t k[3];
            unpack3(Ld->key[b], k);
            for (int c = 0; c < 3; ++c) k[c] /= 2;
            Ld->parent[b] = find_key(&L[d - 1], pack3(k));
        }
    }
    for (int d = 1; d <= D; ++d) {
        level_t* Ld = &L[d];
        if (d < D) {
            Ld->chl = csr_from_owner(L[d + 1].parent, L[d + 1].nbox, Ld->nbox, &Ld->chl_off);
        } else {
            Ld->chl_off = (int64_t*)calloc(Ld->nbox + 1, sizeof(int64_t));
            Ld->chl = (int64_t*)malloc(sizeof(int64_t));
        }
    }

    /* Neighbours N B: relevant boxes a with |a - k|_inf <= 1. */
    for (int d = 1; d <= D; ++d) {
        level_t* Ld = &L[d];
        Ld->nbr_off = (int64_t*)calloc(Ld->nbox + 1, sizeof(int64_t));
        int64_t* tmp = (int64_t*)malloc(sizeof(int64_t) * 27 * Ld->nbox);
        int64_t cnt = 0;
        int64_t nb = (int64_t)1 << (d - 1);
        for (int64_t b = 0; b < Ld->nbox; ++b) {
            int64_t k[3];
            unpack3(Ld->key[b], k);
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        int64_t q[3] = {k[0] + dx, k[1] + dy, k[2] + dz};
                        if (q[0] < 0 || q[1] < 0 || q[2] < 0 || q[0] >= nb || q[1] >= nb || q[2] >= nb) continue;
                        int64_t j = find_key(Ld, pack3(q));
                        if (j >= 0) tmp[cnt++] = j;
                    }
            Ld->nbr_off[b + 1] = cnt;
        }
        Ld->nbr = tmp;
    }

    /* Cousins M B = (R_B^d \ N B) ∩ Q N P B (eq. defcousinboxes). */
    for (int d = 1; d <= D; ++d) {
        level_t* Ld = &L[d];
        Ld->cou_off = (int64_t*)calloc(Ld->nbox + 1, sizeof(int64_t));
        int64_t cap = 64, cnt = 0;
        int64_t* tmp = (int64_t*)malloc(sizeof(int64_t) * cap);
        for (int64_t b = 0; b < Ld->nbox; ++b) {
            if (d >= 2) {
                int64_t k[3];
                unpack3(Ld->key[b], k);
                const level_t* Lp = &L[d - 1];
                int64_t p = Ld->parent[b];
                for (int64_t qi = Lp->nbr_off[p]; qi < Lp->nbr_off[p + 1]; ++qi) {
                    int64_t q = Lp->nbr[qi];
                    for (int64_t ci = Lp->chl_off[q]; ci < Lp->chl_off[q + 1]; ++ci) {
                        int64_t c = Lp->chl[ci], kc[3];
                        unpack3(Ld->key[c], kc);
                        int64_t dmax = 0;
                        for (int e = 0; e < 3; ++e) {
                            int64_t dd = llabs(kc[e] - k[e]);
                            if (dd > dmax) dmax = dd;
                        }
                        if (dmax <= 1) continue;
                        if (cnt == cap) {
                            cap *= 2;
                            tmp = (int64_t*)realloc(tmp, sizeof(int64_t) * cap);
                        }
                        tmp[cnt++] = c;
                    }
                }
            }
            Ld->cou_off[b + 1] = cnt;
        }
        Ld->cou = tmp;
    }

    /* The source tree (reading R16): the root is split; below it a box is
     * active when its parent is active and not a leaf, and an active box is
     * a leaf on level D or when it holds at most leaf_max points. */
    for (int d = 1; d <= D; ++d) {
        level_t* Ld = &L[d];
        Ld->active = (uint8_t*)calloc(Ld->nbox + 1, 1);
        Ld->leaf = (uint8_t*)calloc(Ld->nbox + 1, 1);
        for (int64_t b = 0; b < Ld->nbox; ++b) {
            if (d == 1) {
                Ld->active[b] = 1;
                continue;
            }
            int64_t p = Ld->parent[b];
            Ld->active[b] = L[d - 1].active[p] && !L[d - 1].leaf[p];
            int64_t cnt = Ld->src_off[b + 1] - Ld->src_off[b];
            if (distinct_targets) cnt += Ld->tgt_off[b + 1] - Ld->tgt_off[b];
            Ld->leaf[b] = Ld->active[b] && (d == D || (leaf_max > 0 && cnt <= leaf_max));
        }
    }

    /* Cone intervals per level (reading R5). */
    L[D].ns = leaf_ns;
    L[D].nc = leaf_nc;
    for (int d = D; d >= 2; --d) {
        int ad = (2.0 * fabs(kappa) * L[d].H > 1.0) ? 2 : 1;
        L[d - 1].ns = ad * L[d].ns;
        L[d - 1].nc = ad * L[d].nc;
    }

    double tsn[16], tan_[16];
    oracle_cheb_nodes(ps, tsn);
    oracle_cheb_nodes(pang, tan_);

    /* Relevant cone segments, one sweep d = 3..D (Sec. 3.3.2, eq.
     * defallrelevantconesegments; none at d = 1, 2). */
    for (int d = 1; d <= D; ++d) {
        L[d].cone_off = (int64_t*)calloc(L[d].nbox + 1, sizeof(int64_t));
        L[d].cone = (int64_t*)malloc(sizeof(int64_t));
    }
    for (int d = 3; d <= D; ++d) {
        level_t* Ld = &L[d];
        const level_t* Lp = &L[d - 1];
        int64_t** lists = (int64_t**)calloc(Ld->nbox, sizeof(int64_t*));
        int64_t* lens = (int64_t*)calloc(Ld->nbox, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = 0; b < Ld->nbox; ++b) {
            if (!Ld->active[b]) continue;   /* not a source box: no cones */
            double ctr[3];
            box_centre(x1, H1, Ld->H, Ld->key[b], ctr);
            int64_t cap = 64, cnt = 0;
            int64_t* lst = (int64_t*)malloc(sizeof(int64_t) * cap);
            /* (i) cones containing a cousin target point */
            for (int64_t ci = Ld->cou_off[b]; ci < Ld->cou_off[b + 1]; ++ci) {
                int64_t c = Ld->cou[ci];
                for (int64_t ti = Ld->tgt_off[c]; ti < Ld->tgt_off[c + 1]; ++ti) {
                    int64_t t = Ld->tgt[ti];
                    int32_t idx[3];
                    double loc[3];
                    oracle_cone_coords(ctr, Ld->H, Ld->ns, Ld->nc, &tpos[3 * t], idx, loc, NULL);
                    if (cnt == cap) {
                        cap *= 2;
                        lst = (int64_t*)realloc(lst, sizeof(int64_t) * cap);
                    }
                    lst[cnt++] = cone_id(idx, Ld->nc);
                }
            }
            /* (ii) cones containing an interpolation point of a relevant cone
             * of the parent box (reading R8) */
            if (d >= 4) {
                int64_t p = Ld->parent[b];
                double pctr[3];
                box_centre(x1, H1, Lp->H, Lp->key[p], pctr);
                for (int64_t gi = Lp->cone_off[p]; gi < Lp->cone_off[p + 1]; ++gi) {
                    int32_t pidx[3];
                    cone_idx(Lp->cone[gi], Lp->nc, pidx);
                    for (int nu = 0; nu < P; ++nu) {
                        double ploc[3], x[3], loc[3];
                        int32_t idx[3];
                        node_loc(pang, nu, tsn, tan_, ploc);
                        oracle_cone_point(pctr, Lp->H, Lp->ns, Lp->nc, pidx, ploc, x);
                        oracle_cone_coords(ctr, Ld->H, Ld->ns, Ld->nc, x, idx, loc, NULL);
                        if (cnt == cap) {
                            cap *= 2;
                            lst = (int64_t*)realloc(lst, sizeof(int64_t) * cap);
                        }
                        lst[cnt++] = cone_id(idx, Ld->nc);
                    }
                }
            }
            qsort(lst, cnt, sizeof(int64_t), cmp_i64);
            int64_t nu = 0;
            for (int64_t i = 0; i < cnt; ++i)
                if (i == 0 || lst[i] != lst[nu - 1]) lst[nu++] = lst[i];
            lists[b] = lst;
            lens[b] = nu;
        }
        int64_t tot = 0;
        for (int64_t b = 0; b < Ld->nbox; ++b) {
            Ld->cone_off[b] = tot;
            tot += lens[b];
        }
        Ld->cone_off[Ld->nbox] = tot;
        free(Ld->cone);
        Ld->cone = (int64_t*)malloc(sizeof(int64_t) * (tot > 0 ? tot : 1));
        for (int64_t b = 0; b < Ld->nbox; ++b) {
            if (lens[b]) memcpy(&Ld->cone[Ld->cone_off[b]], lists[b], sizeof(int64_t) * lens[b]);
            free(lists[b]);
        }
        free(lists);
        free(lens);
    }

    /* ------------------------------------------------ operator evaluation */
    const double t_eval = omp_get_wtime();   /* T_acc: from here on */
    /* Output and gradient accumulate as [target][rhs] (interleaved complex);
     * they are transposed to [rhs][target] at the end. */
    double* acc = (double*)calloc((size_t)2 * m * nrhs + 2, sizeof(double));
    double* gacc = grad ? (double*)calloc((size_t)6 * m * nrhs + 6, sizeof(double)) : NULL;
    uint64_t* sg = (uint64_t*)calloc(m + 1, sizeof(uint64_t));
    int64_t near_pairs = 0;
    int bad = 0; /* set if a query ever misses its relevant cone (must not happen) */
    int64_t far_pairs[ORACLE_MAX_LEVELS + 1] = {0}, cousin_evals[ORACLE_MAX_LEVELS + 1] = {0},
            parent_evals[ORACLE_MAX_LEVELS + 1] = {0};

    /* Direct evaluations (Algorithm 1, first box loop): the sources of every
     * leaf box at the targets of its neighbourhood U B, on the leaf's own
     * level (level D only, unless the tree is adaptive). */
    int64_t np_acc = 0;
    for (int d = 2; d <= D; ++d) {
        const level_t* Ld = &L[d];
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : np_acc)
        for (int64_t b = 0; b < Ld->nbox; ++b) {
            if (!Ld->leaf[b]) continue;
            for (int64_t qi = Ld->nbr_off[b]; qi < Ld->nbr_off[b + 1]; ++qi) {
                int64_t q = Ld->nbr[qi];
                for (int64_t ti = Ld->tgt_off[q]; ti < Ld->tgt_off[q + 1]; ++ti) {
                    int64_t t = Ld->tgt[ti];
                    const double* xt = &tpos[3 * t];
                    for (int32_t r = 0; r < nrhs; ++r) {
                        cplx v = 0.0, gv[3] = {0.0, 0.0, 0.0};
                        for (int64_t si = Ld->src_off[b]; si < Ld->src_off[b + 1]; ++si) {
                            int64_t j = Ld->src[si];
                            if (skip && skip[t] == j) continue;
                            v += a[(int64_t)r * n + j] * green_r(kappa, dist3(xt, &pts[3 * j]));
                            if (gacc) {
                                cplx g[3];
                                green_grad(kappa, xt, &pts[3 * j], g);
                                for (int c = 0; c < 3; ++c) gv[c] += a[(int64_t)r * n + j] * g[c];
                            }
                            if (r == 0) np_acc++;
                        }
                        atomic_add_c(&acc[2 * (t * nrhs + r)], v);
                        if (gacc)
                            for (int c = 0; c < 3; ++c) atomic_add_c(&gacc[2 * ((t * nrhs + r) * 3 + c)], gv[c]);
                    }
                    if (sig && Ld->src_off[b + 1] > Ld->src_off[b]) {
                        uint64_t h = mix64(((uint64_t)d << 56) ^ Ld->key[b] ^ 0x5555ull);
#pragma omp atomic
                        sg[t] += h;
                    }
                }
            }
        }
    }
    near_pairs = np_acc;

    /* Node values of level D; the levels above receive theirs from their
     * children (pvals below). */
    cplx* coef = (cplx*)calloc((size_t)L[D].cone_off[L[D].nbox] * P * nrhs + 1, sizeof(cplx));

    /* Interpolation, d = D..3 (Algorithm 1, second loop). */
    for (int d = D; d >= 3; --d) {
        const level_t* Ld = &L[d];
        const level_t* Lp = &L[d - 1];
        /* F_k^d at all interpolation points of the relevant cones of the leaf
         * boxes of level d, directly from their sources (eq. I_k) */
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t b = 0; b < Ld->nbox; ++b)
            if (Ld->leaf[b])
                direct_node_values(Ld, b, x1, H1, P, pang, tsn, tan_, pts, n, a, nrhs, kappa, coef);
        /* interpolants of level d: node values -> Chebyshev coefficients */
        const int64_t ncd = Ld->cone_off[Ld->nbox];
#pragma omp parallel for schedule(static)
        for (int64_t gi = 0; gi < ncd; ++gi) {
            cplx u[16 * 16 * 16], A[16 * 16 * 16];
            for (int32_t r = 0; r < nrhs; ++r) {
                for (int nu = 0; nu < P; ++nu) u[nu] = coef[((size_t)gi * P + nu) * nrhs + r];
                cheb_coeffs_3d(ps, pang, u, A);
                for (int nu = 0; nu < P; ++nu) coef[((size_t)gi * P + nu) * nrhs + r] = A[nu];
            }
        }
        int64_t ncp = (d > 3) ? Lp->cone_off[Lp->nbox] : 0;
        double* pvals = (d > 3) ? (double*)calloc((size_t)2 * ncp * P * nrhs + 2, sizeof(double)) : NULL;
        int64_t fp = 0, ce = 0, pe = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : fp, ce, pe)
        for (int64_t b = 0; b < Ld->nbox; ++b) {
            if (!Ld->active[b]) continue;   /* not a source box */
            double ctr[3];
            box_centre(x1, H1, Ld->H, Ld->key[b], ctr);
            int64_t nsrc = Ld->src_off[b + 1] - Ld->src_off[b];
            /* I_k^d at cousin targets: interpolate F_k^d, times G(x, x_k^d) */
            for (int64_t ci = Ld->cou_off[b]; ci < Ld->cou_off[b + 1]; ++ci) {
                int64_t c = Ld->cou[ci];
                for (int64_t ti = Ld->tgt_off[c]; ti < Ld->tgt_off[c + 1]; ++ti) {
                    int64_t t = Ld->tgt[ti];
                    const double* xt = &tpos[3 * t];
                    int32_t idx[3];
                    double loc[3], sth[3];
                    oracle_cone_coords(ctr, Ld->H, Ld->ns, Ld->nc, xt, idx, loc, sth);
                    int64_t id = cone_id(idx, Ld->nc);
                    int64_t slot = find_cone(Ld, b, id);
                    if (slot < 0) {
#pragma omp atomic write
                        bad = 1;
                        continue;
                    }
                    double r0 = dist3(xt, ctr);
                    cplx Gc = green_r(kappa, r0);
                    ce++;
                    fp += nsrc;
                    for (int32_t r = 0; r < nrhs; ++r) {
                        cplx dP[3];
                        cplx F = cheb_eval_3d(ps, pang, &coef[(size_t)slot * P * nrhs + r], nrhs, loc,
                                              gacc ? dP : NULL);
                        atomic_add_c(&acc[2 * (t * nrhs + r)], Gc * F);
                        if (gacc) {
                            /* grad [G(x, x_k) P(s, theta, phi)] = P grad G + G grad P, with
                             * grad s = -(s/r) v/r, grad theta = theta_hat / r,
                             * grad phi = phi_hat / (r sin theta), and d loc / d(s, theta, phi)
                             * = 2 / (interval length).
                             * On the polar axis of the box's frame (rho = 0) phi is undefined
                             * and the interpolant in (s, theta, phi) is differentiable along
                             * the axis but not across it.  There the gradient is the
                             * derivative along the axis plus, across it, the one-sided
                             * derivative into the half-plane phi = 0 to which the axis belongs
                             * (atan2(0, 0) = 0): grad theta = theta_hat(theta, phi = 0) / r =
                             * (cos theta, 0, 0) / r, and no phi term (phi is constant on that
                             * half-plane). */
                            double v[3] = {xt[0] - ctr[0], xt[1] - ctr[1], xt[2] - ctr[2]};
                            double rho = sqrt(v[0] * v[0] + v[1] * v[1]);
                            double r2 = r0 * r0;
                            double gs[3] = {-sth[0] * v[0] / r2, -sth[0] * v[1] / r2, -sth[0] * v[2] / r2};
                            double gt[3], gp[3];
                            if (rho > 0.0) {
                                gt[0] = v[0] * v[2] / (rho * r2);
                                gt[1] = v[1] * v[2] / (rho * r2);
                                gt[2] = -rho / r2;
                                gp[0] = -v[1] / (rho * rho);
                                gp[1] = v[0] / (rho * rho);
                                gp[2] = 0.0;
                            } else {
                                gt[0] = v[2] / r2;
                                gt[1] = gt[2] = 0.0;
                                gp[0] = gp[1] = gp[2] = 0.0;
                            }
                            double ds = eta_const() / Ld->ns, dth = PI / Ld->nc;
                            cplx gG[3];
                            green_grad(kappa, xt, ctr, gG);
                            for (int e = 0; e < 3; ++e) {
                                cplx gP = dP[0] * (2.0 / ds) * gs[e] + dP[1] * (2.0 / dth) * gt[e] +
                                          dP[2] * (2.0 / dth) * gp[e];
                                atomic_add_c(&gacc[2 * ((t * nrhs + r) * 3 + e)], F * gG[e] + Gc * gP);
                            }
                        }
                    }
                    if (sig) {
                        uint64_t h = mix64(((uint64_t)d << 56) ^ (Ld->key[b] * 0x100000001b3ull) ^ mix64((uint64_t)id));
#pragma omp atomic
                        sg[t] += h;
                    }
                }
            }
            /* F_j^{d-1} at the parent's interpolation points: interpolate F_k^d
             * and re-centre by G(x, x_k^d) / G(x, x_j^{d-1}) */
            if (d > 3) {
                int64_t p = Ld->parent[b];
                double pctr[3];
                box_centre(x1, H1, Lp->H, Lp->key[p], pctr);
                for (int64_t gi = Lp->cone_off[p]; gi < Lp->cone_off[p + 1]; ++gi) {
                    int32_t pidx[3];
                    cone_idx(Lp->cone[gi], Lp->nc, pidx);
                    for (int nu = 0; nu < P; ++nu) {
                        double ploc[3], x[3], loc[3];
                        int32_t idx[3];
                        node_loc(pang, nu, tsn, tan_, ploc);
                        oracle_cone_point(pctr, Lp->H, Lp->ns, Lp->nc, pidx, ploc, x);
                        oracle_cone_coords(ctr, Ld->H, Ld->ns, Ld->nc, x, idx, loc, NULL);
                        int64_t slot = find_cone(Ld, b, cone_id(idx, Ld->nc));
                        if (slot < 0) {
#pragma omp atomic write
                            bad = 1;
                            continue;
                        }
                        /* G(x, x_k) / G(x, x_j) = g_{x_j}(x, x_k) by eq. (factor) */
                        cplx ratio = analytic_factor(kappa, pctr, x, ctr);
                        pe++;
                        for (int32_t r = 0; r < nrhs; ++r) {
                            cplx F = cheb_eval_3d(ps, pang, &coef[(size_t)slot * P * nrhs + r], nrhs, loc, NULL);
                            atomic_add_c(&pvals[2 * (((size_t)gi * P + nu) * nrhs + r)], F * ratio);
                        }
                    }
                }
            }
        }
        far_pairs[d] = fp;
        cousin_evals[d] = ce;
        parent_evals[d] = pe;
        free(coef);
        coef = (cplx*)pvals;   /* node values of level d - 1 (NULL after level 3) */
    }
    free(coef);

    for (int64_t t = 0; t < m; ++t)
        for (int32_t r = 0; r < nrhs; ++r) {
            out[2 * ((int64_t)r * m + t)] = acc[2 * (t * nrhs + r)];
            out[2 * ((int64_t)r * m + t) + 1] = acc[2 * (t * nrhs + r) + 1];
            if (grad)
                for (int e = 0; e < 6; ++e) grad[6 * ((int64_t)r * m + t) + e] = gacc[6 * (t * nrhs + r) + e];
        }
    if (sig)
        for (int64_t t = 0; t < m; ++t) sig[t] = sg[t];
    const double t_end = omp_get_wtime();

    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->t_pre = t_eval - t_start;
        stats->t_acc = t_end - t_eval;
        stats->D = D;
        stats->H1 = H1;
        for (int c = 0; c < 3; ++c) stats->x1[c] = x1[c];
        stats->n_near_pairs = near_pairs;
        for (int d = 1; d <= D; ++d) {
            stats->ns[d] = L[d].ns;
            stats->nc[d] = L[d].nc;
            stats->n_boxes[d] = L[d].nbox;
            stats->n_cones[d] = L[d].cone_off[L[d].nbox];
            /* cousins of the source boxes (every box unless adaptive) */
            int64_t mx = 0;
            for (int64_t b = 0; b < L[d].nbox; ++b) {
                if (!L[d].active[b]) continue;
                stats->n_cousin_boxes[d] += L[d].cou_off[b + 1] - L[d].cou_off[b];
                if (L[d].cou_off[b + 1] - L[d].cou_off[b] > mx) mx = L[d].cou_off[b + 1] - L[d].cou_off[b];
            }
            stats->max_cousin_boxes[d] = mx;
            stats->n_cousin_evals[d] = cousin_evals[d];
            stats->n_parent_evals[d] = parent_evals[d];
            stats->n_far_pairs[d] = far_pairs[d];
            for (int64_t b = 0; b < L[d].nbox; ++b) {
                stats->n_src_boxes[d] += L[d].active[b];
                stats->n_leaf_boxes[d] += L[d].leaf[b];
            }
        }
    }

    for (int d = 1; d <= D; ++d) free_level(&L[d]);
    free(L);
    free(acc);
    free(gacc);
    free(sg);
    free(skip_own);
    return bad ? -3 : 0;
}
