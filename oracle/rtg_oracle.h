/*
 * rtg_oracle.h -- CPU oracle for all-pairs r-nearest-neighbours by randomly
 * transformed grids (RTG).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously correct FP64
 * implementation of what the GPU library computes.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library, and the
 * library never calls it.
 *
 * What it follows (Kleinbort, Salzman & Halperin, "Efficient high-quality
 * motion planning by fast all-pairs r-nearest-neighbors"):
 *   - the problem (Sec. I): report every pair p,q of P with ||p-q|| <= r;
 *   - Randomly Shifted Grids (Sec. III, Alg. "Randomly Shifted Grids"): for
 *     each of m grids of cell side c = c~ * r draw a uniform shift, put every
 *     point into the cell that contains it, test every pair of points that
 *     share a cell and report it when its distance is at most r;
 *   - the random-orientation variant (Sec. III and III-B): each grid also gets
 *     a uniformly random orientation;
 *   - pairs reported by several grids are reported once (Sec. III-B), and
 *     every pair is stored in both orientations so that the per-point
 *     neighbour lists answer multiple r-NN queries (Sec. III-B);
 *   - the MR-metric of the multi-robot experiments (Sec. IV-C) as an
 *     alternative pair test on the same Euclidean grids.
 *
 * Parameter names: the paper's m (number of grids) is `k` here and its
 * cell-size factor c~ is `alpha`; the grid cell side is alpha * r.
 *
 * Readings where the paper is silent:
 *   - "at most r" is taken literally: a pair is reported iff d^2 <= r*r, with
 *     d^2 summed in FP64 from the FP32 coordinates in axis order, no FMA;
 *   - a cell is half-open: kappa_j = floor(y_j);
 *   - a transform maps p to y = (R p) / c + u: rotate, scale to cell units,
 *     then shift by u in [0,1)^d cell units;
 *   - the shift is uniform, the orientation is Haar on O(d) (Gaussian rows,
 *     modified Gram-Schmidt in index order);
 *   - random numbers come from SplitMix64 (Steele, Lea & Flood, 2014):
 *     transform t draws from the stream started at the (t+1)-th SplitMix64
 *     output of `seed`; it first draws the d shifts, then the d*d Gaussians
 *     of its rotation (Marsaglia's polar method, pairs in row-major order),
 *     whose rows are orthonormalised by modified Gram-Schmidt applied twice;
 *   - pairs are by index; coincident points are reported (distance 0) and a
 *     point is never paired with itself;
 *   - the output is a canonical CSR: rows ascending, columns ascending;
 *   - the MR-metric's robots are equal blocks of consecutive axes, and the
 *     grids stay Euclidean: only the pair test changes (the paper names the
 *     metric but not how the grids treat it).
 */
#ifndef RTG_ORACLE_H
#define RTG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORACLE_OK = 0,
  ORACLE_EINVAL = -1,
  ORACLE_ENOMEM = -2,
  ORACLE_ERANGE = -3
};

enum {
  ORACLE_NO_ROTATE = 1u,  /* shift-only grids (the paper's first algorithm) */
  ORACLE_UPPER_ONLY = 2u  /* store (i,j) in row i only, j > i              */
};

/* The MR-metric of Sec. IV-C: ORACLE_ROBOTS(b) in flags, b in [2, d] dividing
 * d, splits a configuration into b robots of d / b consecutive axes each and
 * measures the distance of two configurations as the sum of the robots'
 * Euclidean displacements (each an FP64 square root of the robot's squared
 * displacement summed in axis order); a pair is within r iff that sum <= r.
 * The grids stay those of the Euclidean method.  b = 0 or 1: Euclidean. */
#define ORACLE_ROBOTS_SHIFT 8
#define ORACLE_ROBOTS_MASK 0xFF00u
#define ORACLE_ROBOTS(b) ((uint32_t)(b) << ORACLE_ROBOTS_SHIFT)

/* A neighbour list in CSR form, owned by the oracle (free with
 * oracle_result_free).  row_ptr has n+1 entries, col has nnz entries. */
typedef struct {
  int64_t n;
  int64_t nnz;
  int64_t *row_ptr;
  int32_t *col;
} oracle_result;

/* SplitMix64: advance the state by the golden gamma and return the mixed
 * output. */
uint64_t oracle_splitmix64_next(uint64_t *state);

/* Uniform double in [0,1) from the top 53 bits of one SplitMix64 output. */
double oracle_uniform01(uint64_t *state);

/* Two independent standard normals by Marsaglia's polar method. */
void oracle_gaussian_pair(uint64_t *state, double *g0, double *g1);

/* The k seeded transforms: R is [k][d][d] row-major (rows orthonormal), u is
 * [k][d] in [0,1).  With ORACLE_NO_ROTATE, R is the identity. */
int oracle_make_transforms(uint64_t seed, int32_t k, int32_t d, uint32_t flags,
                           double *R, double *u);

/* Integer cell coordinates of every point under one transform:
 * kappa[i*d + j] = floor(((R_j0 p_0 + R_j1 p_1) + ...) * inv_c + u_j).
 * Returns ORACLE_ERANGE if some |y_j| >= 2^31. */
int oracle_cell_coords(const float *points, int64_t n, int32_t d,
                       const double *R, const double *u, double inv_c,
                       int64_t *kappa);

/* Pairs (i<j) reported by ONE transform, written to pairs[2*p], pairs[2*p+1],
 * sorted by (i,j).  *npairs receives the count; the array is malloc'd and is
 * released with oracle_free. */
int oracle_transform_pairs(const float *points, int64_t n, int32_t d, double r,
                           double alpha, const double *R, const double *u,
                           int64_t **pairs, int64_t *npairs);

/* Full RTG with caller-given transforms (R [k][d][d], u [k][d]).  flags:
 * ORACLE_UPPER_ONLY, ORACLE_ROBOTS(b) (NO_ROTATE is not used: R is given). */
int oracle_rtg_with_transforms(const float *points, int64_t n, int32_t d,
                               double r, int32_t k, double alpha,
                               const double *R, const double *u, uint32_t flags,
                               oracle_result **out);

/* Full RTG with transforms drawn from `seed`. */
int oracle_rtg(const float *points, int64_t n, int32_t d, double r, int32_t k,
               double alpha, uint64_t seed, uint32_t flags,
               oracle_result **out);

/* The rows `rows[0..nrows)` of the symmetric RTG neighbour list, computed one
 * by one: q is a neighbour of row s iff q != s, some transform puts q and s
 * in the same cell, and q is within r of s (the metric of flags).  Same
 * transforms as oracle_rtg_with_transforms; result rows follow the order of
 * `rows`.  flags: ORACLE_ROBOTS(b). */
int oracle_rtg_rows(const float *points, int64_t n, int32_t d, double r,
                    int32_t k, double alpha, const double *R, const double *u,
                    uint32_t flags, const int64_t *rows, int64_t nrows,
                    oracle_result **out);

/* Query mode: the same grids answer r-NN queries for new points.  Row s of
 * the result lists, ascending and once each, the indexed points p_i with
 * ||p_i - q_s|| <= r (FP64, axis order, as for pairs) that share a cell with
 * q_s under some transform -- q_s takes the role of one more point of the
 * set (a query equal to p_i reports i).  Transforms as in
 * oracle_rtg_with_transforms; flags: ORACLE_ROBOTS(b) (the distance test is
 * then the MR-metric's).  ORACLE_ERANGE if a cell coordinate of a point or a
 * query has |y| >= 2^31. */
int oracle_rtg_query(const float *points, int64_t n, int32_t d,
                     const float *queries, int64_t m, double r, int32_t k,
                     double alpha, const double *R, const double *u,
                     uint32_t flags, oracle_result **out);

/* Exact all-pairs r-NN by testing every pair (the set RTG approximates).
 * flags: ORACLE_UPPER_ONLY, ORACLE_ROBOTS(b). */
int oracle_bruteforce(const float *points, int64_t n, int32_t d, double r,
                      uint32_t flags, oracle_result **out);

void oracle_result_free(oracle_result *res);
void oracle_free(void *p);

#ifdef __cplusplus
}
#endif

#endif /* RTG_ORACLE_H */
