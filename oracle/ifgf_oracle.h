/*
 * Plain FP64 CPU reference ("oracle") for the IFGF operator of Bauinger and
 * Bruno, "IFGF: Interpolated Factored Green Function method" (arXiv
 * 2010.02857).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against the paper.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * Conventions shared by every entry point:
 *   - points are FP64, row-major [n][3];
 *   - complex arrays are interleaved (re, im) FP64;
 *   - a batch of right-hand sides is laid out [nrhs][n] (one vector after the
 *     other), outputs likewise [nrhs][m];
 *   - the functions return 0 on success and a negative code on bad input.
 */
#ifndef IFGF_ORACLE_H
#define IFGF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_MAX_LEVELS 24

/* Per-level counts of the hierarchy that the IFGF oracle built; index d is
 * level d (1-based, entry 0 unused). */
typedef struct {
    int32_t D;                                /* number of levels            */
    double H1;                                /* root box side               */
    double x1[3];                             /* root box centre             */
    int32_t ns[ORACLE_MAX_LEVELS + 1];        /* radial intervals n_{s,d}    */
    int32_t nc[ORACLE_MAX_LEVELS + 1];        /* polar intervals n_{C,d}     */
    int64_t n_boxes[ORACLE_MAX_LEVELS + 1];   /* relevant boxes |R_B^d|      */
    int64_t n_cones[ORACLE_MAX_LEVELS + 1];   /* relevant cones |R_C^d|      */
    int64_t n_cousin_boxes[ORACLE_MAX_LEVELS + 1];  /* sum_k |M B_k| over the
                                                       source boxes          */
    int64_t max_cousin_boxes[ORACLE_MAX_LEVELS + 1];/* max_k |M B_k|         */
    int64_t n_cousin_evals[ORACLE_MAX_LEVELS + 1];  /* sum_k |V B_k ∩ targets|*/
    int64_t n_parent_evals[ORACLE_MAX_LEVELS + 1];  /* child->parent node evals*/
    int64_t n_far_pairs[ORACLE_MAX_LEVELS + 1];     /* (target, source) pairs
                                                       covered at level d    */
    int64_t n_near_pairs;                     /* pairs summed directly       */
    int64_t n_src_boxes[ORACLE_MAX_LEVELS + 1];     /* boxes of the source tree*/
    int64_t n_leaf_boxes[ORACLE_MAX_LEVELS + 1];    /* its leaves on level d   */
    double t_pre;                             /* seconds: hierarchy and
                                                 relevant cones (T_pre)      */
    double t_acc;                             /* seconds: operator
                                                 evaluation (T_acc)          */
} oracle_stats;

/* Direct O(N^2) sum of Sec. 2, eq. (field1) with the Helmholtz kernel of
 * eq. (greensfunction): out_r[i] = sum_{j != skip[i]} a_r[j] G(t_i, x_j).
 *   pts   [n][3] source points, dens [nrhs][n] complex
 *   tpos  [m][3] target positions, skip[m] source index to leave out (-1: none)
 *   out   [nrhs][m] complex                                                  */
int oracle_direct(const double* pts, int64_t n, const double* dens, int32_t nrhs,
                  double kappa, const double* tpos, const int64_t* skip, int64_t m,
                  double* out);

/* Gradient of the direct sum with respect to the target position:
 * grad[r][i][c] = d/d t_{i,c} sum_{j != skip[i]} a_r[j] G(t_i, x_j), complex,
 * laid out [nrhs][m][3].                                                     */
int oracle_direct_grad(const double* pts, int64_t n, const double* dens, int32_t nrhs,
                       double kappa, const double* tpos, const int64_t* skip, int64_t m,
                       double* grad);

/* Plain FP64 IFGF (Sec. 3.3, Algorithm 1).
 *   levels  D >= 2, or 0 to choose H_D about a quarter wavelength (Sec. 4);
 *   ps, pang  Chebyshev node counts per cone in s and in each angle;
 *   leaf_ns, leaf_nc  cone counts n_{s,D}, n_{C,D} of the leaf level;
 *   tpos/skip/m  target override (NULL tpos: targets are the sources and
 *               skip[i] = i);
 *   out     [nrhs][m] complex;
 *   grad    optional [nrhs][m][3] complex derivative of the IFGF output with
 *           respect to the target position (NULL: not computed);
 *   sig     optional [m] signature of every discrete choice made for each
 *           target (its boxes and the cone it falls in for every cousin box);
 *           two targets with equal signatures were treated by the same
 *           piecewise-smooth branch of the method;
 *   stats   optional.                                                       */
int oracle_ifgf(const double* pts, int64_t n, const double* dens, int32_t nrhs,
                double kappa, int32_t levels, int32_t ps, int32_t pang,
                int32_t leaf_ns, int32_t leaf_nc,
                const double* tpos, const int64_t* skip, int64_t m,
                double* out, double* grad, uint64_t* sig, oracle_stats* stats);

/* oracle_ifgf on an adaptive octree (the reading of Sec. 4 and Sec. 5 stated
 * in the source as R16): leaf_max > 0 stops splitting a box of level >= 2
 * that holds at most leaf_max points (sources plus distinct targets);
 * leaf_max = 0 gives oracle_ifgf exactly.                                   */
int oracle_ifgf_ex(const double* pts, int64_t n, const double* dens, int32_t nrhs,
                   double kappa, int32_t levels, int32_t ps, int32_t pang,
                   int32_t leaf_ns, int32_t leaf_nc, int32_t leaf_max,
                   const double* tpos, const int64_t* skip, int64_t m,
                   double* out, double* grad, uint64_t* sig, oracle_stats* stats);

/* The pieces of the method, exposed so that tests can pin them one by one. */

/* Green function G(x, y) of eq. (greensfunction) and analytic factor
 * g_c(x, y) of eq. (factored_f) centred at c; each writes one complex.     */
void oracle_green(double kappa, const double* x, const double* y, double* out);
void oracle_analytic_factor(double kappa, const double* c, const double* x,
                            const double* y, double* out);

/* First-kind Chebyshev nodes on [-1, 1] (Sec. 3.2). */
void oracle_cheb_nodes(int32_t n, double* t);

/* Tensor Chebyshev interpolant through values u[a][b][c] given at the nodes
 * (t_a, t_b, t_c) of a ps x pang x pang grid, evaluated at (ts, tt, tp). */
void oracle_cheb_interp3(int32_t ps, int32_t pang, const double* u, double ts,
                         double tt, double tp, double* out);

/* Cone coordinates of x seen from box centre c at a level with box side H,
 * ns radial and nc polar intervals: idx = (i_s, i_theta, i_phi), loc = local
 * coordinates in [-1, 1]^3, sth = (s, theta, phi).                        */
void oracle_cone_coords(const double* c, double H, int32_t ns, int32_t nc,
                        const double* x, int32_t* idx, double* loc, double* sth);

/* Position of the point with local coordinates loc in cone idx. */
void oracle_cone_point(const double* c, double H, int32_t ns, int32_t nc,
                       const int32_t* idx, const double* loc, double* x);

#ifdef __cplusplus
}
#endif
#endif
