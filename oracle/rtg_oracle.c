/*
 * rtg_oracle.c -- CPU oracle for all-pairs r-NN by randomly transformed grids.
 *
 * TEST INFRASTRUCTURE ONLY (see rtg_oracle.h): plain C, FP64, no FMA
 * contraction (built with -ffp-contract=off), sums taken left to right.  It
 * follows the paper's steps in its order and does no blocking, fusion or
 * reordering: per grid, put each point in its cell, group equal cells, test
 * every same-cell pair; then take the union over the grids and lay the pairs
 * out as a symmetric neighbour list.
 */
#define _GNU_SOURCE
#include "rtg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Random numbers: SplitMix64 (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).                             */

#define SPLITMIX_GAMMA 0x9E3779B97F4A7C15ull

uint64_t oracle_splitmix64_next(uint64_t *state) {
  uint64_t z;
  *state = *state + SPLITMIX_GAMMA;
  z = *state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double oracle_uniform01(uint64_t *state) {
  uint64_t x = oracle_splitmix64_next(state);
  return (double)(x >> 11) * (1.0 / 9007199254740992.0); /* 2^-53 */
}

/* Marsaglia & Bray (1964), the polar form of Box-Muller: draw (a,b) uniform
 * in the square [-1,1)^2 until it falls strictly inside the unit disc, then
 * scale both by sqrt(-2 ln s / s). */
void oracle_gaussian_pair(uint64_t *state, double *g0, double *g1) {
  double a, b, s, f;
  do {
    a = 2.0 * oracle_uniform01(state) - 1.0;
    b = 2.0 * oracle_uniform01(state) - 1.0;
    s = a * a + b * b;
  } while (s >= 1.0 || s == 0.0);
  f = sqrt(-2.0 * log(s) / s);
  *g0 = a * f;
  *g1 = b * f;
}

/* ------------------------------------------------------------------------ */
/* Transforms: the random shift of each grid (Alg. Randomly Shifted Grids,
 * "choose a random shift") and the random orientation of the second variant
 * (Sec. III).                                                                */

int oracle_make_transforms(uint64_t seed, int32_t k, int32_t d, uint32_t flags,
                           double *R, double *u) {
  int32_t t, i, j, l;
  double *G;
  if (k < 1 || d < 1 || d > 64 || R == NULL || u == NULL) return ORACLE_EINVAL;
  G = (double *)malloc(sizeof(double) * (size_t)d * (size_t)d);
  if (G == NULL) return ORACLE_ENOMEM;

  for (t = 0; t < k; ++t) {
    double *Rt = R + (size_t)t * d * d;
    double *ut = u + (size_t)t * d;
    /* The stream of transform t starts at the (t+1)-th output of seed's own
     * SplitMix64 stream, so transform t does not depend on k. */
    uint64_t parent = seed;
    uint64_t st = 0;
    for (i = 0; i <= t; ++i) st = oracle_splitmix64_next(&parent);

    /* Shift: d uniforms in [0,1), in cell units. */
    for (j = 0; j < d; ++j) ut[j] = oracle_uniform01(&st);

    if (flags & ORACLE_NO_ROTATE) {
      for (i = 0; i < d; ++i)
        for (j = 0; j < d; ++j) Rt[i * d + j] = (i == j) ? 1.0 : 0.0;
      continue;
    }

    /* Orientation: a d x d matrix of standard normals, filled row-major two
     * at a time; the rows are then orthonormalised in index order by modified
     * Gram-Schmidt.  A Gaussian matrix orthonormalised this way is Haar
     * distributed on O(d). */
    for (i = 0; i < d * d; i += 2) {
      double g0, g1;
      oracle_gaussian_pair(&st, &g0, &g1);
      G[i] = g0;
      if (i + 1 < d * d) G[i + 1] = g1;
    }
    for (i = 0; i < d; ++i) {
      double *v = G + (size_t)i * d;
      double nrm2 = 0.0, nrm;
      int pass;
      /* Two sweeps of projections against the earlier rows: one sweep of
       * modified Gram-Schmidt loses orthogonality in proportion to the
       * conditioning of G; a second sweep restores it to rounding level
       * ("twice is enough", Giraud, Langou & Rozloznik, 2005). */
      for (pass = 0; pass < 2; ++pass)
        for (j = 0; j < i; ++j) {
          const double *q = Rt + (size_t)j * d;
          double dot = 0.0;
          for (l = 0; l < d; ++l) dot = dot + v[l] * q[l];
          for (l = 0; l < d; ++l) v[l] = v[l] - dot * q[l];
        }
      for (l = 0; l < d; ++l) nrm2 = nrm2 + v[l] * v[l];
      nrm = sqrt(nrm2);
      if (!(nrm > 0.0)) {
        free(G);
        return ORACLE_ERANGE;
      }
      for (l = 0; l < d; ++l) Rt[(size_t)i * d + l] = v[l] / nrm;
    }
  }
  free(G);
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Cells: "compute the grid cell u that p lies in" (Alg. Randomly Shifted
 * Grids).  In cell units the transformed point is y = (R p) * (1/c) + u and
 * its cell is the integer vector floor(y).                                  */

int oracle_cell_coords(const float *points, int64_t n, int32_t d,
                       const double *R, const double *u, double inv_c,
                       int64_t *kappa) {
  int64_t i;
  int32_t j, l;
  for (i = 0; i < n; ++i) {
    const float *p = points + (size_t)i * d;
    for (j = 0; j < d; ++j) {
      double z = R[(size_t)j * d + 0] * (double)p[0];
      double y;
      for (l = 1; l < d; ++l) z = z + R[(size_t)j * d + l] * (double)p[l];
      y = z * inv_c + u[j];
      if (!(fabs(y) < 2147483648.0)) return ORACLE_ERANGE;
      kappa[(size_t)i * d + j] = (int64_t)floor(y);
    }
  }
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* The pair test.
 *   Euclidean metric (Sec. I): s = sum over axes, in axis order, of
 *   ((double)p_l - (double)q_l)^2; the pair is within r iff s <= r*r.
 *   MR-metric (Sec. IV-C, several robots moving at once): the configuration
 *   holds `robots` robots of d / robots consecutive axes each, and the
 *   distance is the sum, in robot order, of every robot's own Euclidean
 *   displacement -- the FP64 square root of that robot's squared displacement,
 *   summed in axis order as above; the pair is within r iff the sum <= r. */
typedef struct {
  double r, r2;
  int32_t d;
  int32_t sub; /* axes per robot; 0: the Euclidean metric */
} pair_metric;

/* The metric that `flags` selects (ORACLE_ROBOTS(b), b >= 2, dividing d). */
static int make_metric(double r, int32_t d, uint32_t flags, pair_metric *mt) {
  uint32_t robots = (flags & ORACLE_ROBOTS_MASK) >> ORACLE_ROBOTS_SHIFT;
  mt->r = r;
  mt->r2 = r * r;
  mt->d = d;
  mt->sub = 0;
  if (robots <= 1) return ORACLE_OK;
  if (robots > (uint32_t)d || d % (int32_t)robots != 0) return ORACLE_EINVAL;
  mt->sub = d / (int32_t)robots;
  return ORACLE_OK;
}

static int within_metric(const pair_metric *mt, const float *pa,
                         const float *pb) {
  double s = 0.0;
  int32_t l, b;
  if (mt->sub == 0) {
    for (l = 0; l < mt->d; ++l) {
      double delta = (double)pa[l] - (double)pb[l];
      s = s + delta * delta;
    }
    return s <= mt->r2;
  }
  for (b = 0; b < mt->d; b += mt->sub) {
    double t = 0.0;
    for (l = b; l < b + mt->sub; ++l) {
      double delta = (double)pa[l] - (double)pb[l];
      t = t + delta * delta;
    }
    s = s + sqrt(t);
  }
  return s <= mt->r;
}

static int within_r(const pair_metric *mt, const float *points, int64_t a,
                    int64_t b) {
  return within_metric(mt, points + (size_t)a * mt->d,
                       points + (size_t)b * mt->d);
}

/* Growable array of (i,j) index pairs. */
typedef struct {
  int64_t *v; /* 2 entries per pair */
  int64_t n, cap;
} pair_vec;

static int pv_push(pair_vec *pv, int64_t i, int64_t j) {
  if (pv->n == pv->cap) {
    int64_t nc = pv->cap ? pv->cap * 2 : 1024;
    int64_t *nv = (int64_t *)realloc(pv->v, sizeof(int64_t) * 2 * (size_t)nc);
    if (nv == NULL) return ORACLE_ENOMEM;
    pv->v = nv;
    pv->cap = nc;
  }
  pv->v[2 * pv->n] = i;
  pv->v[2 * pv->n + 1] = j;
  pv->n++;
  return ORACLE_OK;
}

static int cmp_pair(const void *a, const void *b) {
  const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
  if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
  if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
  return 0;
}

/* Sort pairs by (i,j) and drop repeats. */
static void sort_unique(pair_vec *pv) {
  int64_t w = 0, q;
  if (pv->n == 0) return;
  qsort(pv->v, (size_t)pv->n, 2 * sizeof(int64_t), cmp_pair);
  for (q = 0; q < pv->n; ++q) {
    if (w > 0 && pv->v[2 * (w - 1)] == pv->v[2 * q] &&
        pv->v[2 * (w - 1) + 1] == pv->v[2 * q + 1])
      continue;
    pv->v[2 * w] = pv->v[2 * q];
    pv->v[2 * w + 1] = pv->v[2 * q + 1];
    ++w;
  }
  pv->n = w;
}

/* Order point indices by their cell vector (lexicographic), ties by index. */
typedef struct {
  const int64_t *kappa;
  int32_t d;
} cell_order;

static int cmp_by_cell(const void *a, const void *b, void *ctx) {
  const cell_order *co = (const cell_order *)ctx;
  int64_t ia = *(const int64_t *)a, ib = *(const int64_t *)b;
  const int64_t *ka = co->kappa + (size_t)ia * co->d;
  const int64_t *kb = co->kappa + (size_t)ib * co->d;
  int32_t j;
  for (j = 0; j < co->d; ++j)
    if (ka[j] != kb[j]) return ka[j] < kb[j] ? -1 : 1;
  if (ia != ib) return ia < ib ? -1 : 1;
  return 0;
}

static int same_cell(const int64_t *kappa, int32_t d, int64_t a, int64_t b) {
  int32_t j;
  for (j = 0; j < d; ++j)
    if (kappa[(size_t)a * d + j] != kappa[(size_t)b * d + j]) return 0;
  return 1;
}

/* One grid of Alg. Randomly Shifted Grids: cells of every point, then every
 * pair inside each non-empty cell; reported pairs are appended to pv. */
static int one_grid(const float *points, int64_t n, int32_t d,
                    const pair_metric *mt, double inv_c, const double *R,
                    const double *u, pair_vec *pv) {
  int64_t *kappa, *order, g0, g1, a, b;
  cell_order co;
  int rc;
  kappa = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * (size_t)d);
  order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (kappa == NULL || order == NULL) {
    free(kappa);
    free(order);
    return ORACLE_ENOMEM;
  }
  rc = oracle_cell_coords(points, n, d, R, u, inv_c, kappa);
  if (rc != ORACLE_OK) goto done;

  /* U: the non-empty cells, found by sorting the points by cell vector. */
  for (a = 0; a < n; ++a) order[a] = a;
  co.kappa = kappa;
  co.d = d;
  qsort_r(order, (size_t)n, sizeof(int64_t), cmp_by_cell, &co);

  /* Each run [g0,g1) of equal cell vectors is one cell; test all its pairs. */
  for (g0 = 0; g0 < n; g0 = g1) {
    g1 = g0 + 1;
    while (g1 < n && same_cell(kappa, d, order[g0], order[g1])) ++g1;
    for (a = g0; a < g1; ++a)
      for (b = a + 1; b < g1; ++b) {
        int64_t i = order[a], j = order[b]; /* i < j: ties sorted by index */
        if (within_r(mt, points, i, j)) {
          rc = pv_push(pv, i, j);
          if (rc != ORACLE_OK) goto done;
        }
      }
  }
done:
  free(kappa);
  free(order);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Argument checks shared by the entry points (same rules as the library).   */

static int check_points(const float *points, int64_t n, int32_t d) {
  int64_t q;
  if (d < 1 || d > 64 || n < 0 || n >= ((int64_t)1 << 31)) return ORACLE_EINVAL;
  if (n > 0 && points == NULL) return ORACLE_EINVAL;
  for (q = 0; q < n * (int64_t)d; ++q)
    if (!isfinite(points[q])) return ORACLE_EINVAL;
  return ORACLE_OK;
}

static int check_radius(double r) {
  return (isfinite(r) && r > 0.0) ? ORACLE_OK : ORACLE_EINVAL;
}

/* ------------------------------------------------------------------------ */
/* Storing every pair twice (Sec. III-B): build the directed list (i,j) and
 * (j,i), sort it by (row, column), and count rows.                          */

static int make_csr(const pair_vec *pv, int64_t n, uint32_t flags,
                    oracle_result **out) {
  int both = !(flags & ORACLE_UPPER_ONLY);
  int64_t m = pv->n * (both ? 2 : 1), q;
  int64_t *dir = NULL;
  oracle_result *res = (oracle_result *)calloc(1, sizeof(oracle_result));
  if (res == NULL) return ORACLE_ENOMEM;
  res->n = n;
  res->nnz = m;
  res->row_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  res->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  dir = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)(m > 0 ? m : 1));
  if (res->row_ptr == NULL || res->col == NULL || dir == NULL) {
    free(dir);
    oracle_result_free(res);
    return ORACLE_ENOMEM;
  }
  for (q = 0; q < pv->n; ++q) {
    int64_t i = pv->v[2 * q], j = pv->v[2 * q + 1];
    int64_t w = both ? 2 * q : q;
    dir[2 * w] = i;
    dir[2 * w + 1] = j;
    if (both) {
      dir[2 * w + 2] = j;
      dir[2 * w + 3] = i;
    }
  }
  if (m > 0) qsort(dir, (size_t)m, 2 * sizeof(int64_t), cmp_pair);
  for (q = 0; q < m; ++q) {
    res->row_ptr[dir[2 * q] + 1] += 1;
    res->col[q] = (int32_t)dir[2 * q + 1];
  }
  for (q = 0; q < n; ++q) res->row_ptr[q + 1] += res->row_ptr[q];
  free(dir);
  *out = res;
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */

int oracle_transform_pairs(const float *points, int64_t n, int32_t d, double r,
                           double alpha, const double *R, const double *u,
                           int64_t **pairs, int64_t *npairs) {
  pair_vec pv = {NULL, 0, 0};
  int rc = check_points(points, n, d);
  if (rc == ORACLE_OK) rc = check_radius(r);
  if (rc == ORACLE_OK && !(isfinite(alpha) && alpha > 0.0)) rc = ORACLE_EINVAL;
  if (rc != ORACLE_OK) return rc;
  if (n >= 2) {
    double c = alpha * r;
    pair_metric mt;
    make_metric(r, d, 0u, &mt);
    rc = one_grid(points, n, d, &mt, 1.0 / c, R, u, &pv);
    if (rc != ORACLE_OK) {
      free(pv.v);
      return rc;
    }
  }
  sort_unique(&pv); /* one grid never repeats a pair; this only sorts */
  *pairs = pv.v;
  *npairs = pv.n;
  return ORACLE_OK;
}

int oracle_rtg_with_transforms(const float *points, int64_t n, int32_t d,
                               double r, int32_t k, double alpha,
                               const double *R, const double *u, uint32_t flags,
                               oracle_result **out) {
  pair_vec pv = {NULL, 0, 0};
  pair_metric mt;
  int32_t t;
  int rc = check_points(points, n, d);
  if (rc == ORACLE_OK) rc = check_radius(r);
  if (rc == ORACLE_OK && (k < 1 || !(isfinite(alpha) && alpha > 0.0)))
    rc = ORACLE_EINVAL;
  if (rc == ORACLE_OK) rc = make_metric(r, d, flags, &mt);
  if (rc != ORACLE_OK) return rc;
  if (n >= 2) {
    double c = alpha * r;
    double inv_c = 1.0 / c;
    for (t = 0; t < k; ++t) {
      rc = one_grid(points, n, d, &mt, inv_c, R + (size_t)t * d * d,
                    u + (size_t)t * d, &pv);
      if (rc != ORACLE_OK) {
        free(pv.v);
        return rc;
      }
    }
  }
  /* Union over the grids: each neighbouring pair is reported once. */
  sort_unique(&pv);
  rc = make_csr(&pv, n, flags, out);
  free(pv.v);
  return rc;
}

int oracle_rtg(const float *points, int64_t n, int32_t d, double r, int32_t k,
               double alpha, uint64_t seed, uint32_t flags,
               oracle_result **out) {
  double *R, *u;
  int rc = check_points(points, n, d);
  if (rc == ORACLE_OK) rc = check_radius(r);
  if (rc == ORACLE_OK && (k < 1 || !(isfinite(alpha) && alpha > 0.0)))
    rc = ORACLE_EINVAL;
  if (rc != ORACLE_OK) return rc;
  R = (double *)malloc(sizeof(double) * (size_t)k * d * d);
  u = (double *)malloc(sizeof(double) * (size_t)k * d);
  if (R == NULL || u == NULL) {
    free(R);
    free(u);
    return ORACLE_ENOMEM;
  }
  rc = oracle_make_transforms(seed, k, d, flags, R, u);
  if (rc == ORACLE_OK)
    rc = oracle_rtg_with_transforms(points, n, d, r, k, alpha, R, u, flags, out);
  free(R);
  free(u);
  return rc;
}

int oracle_rtg_rows(const float *points, int64_t n, int32_t d, double r,
                    int32_t k, double alpha, const double *R, const double *u,
                    uint32_t flags, const int64_t *rows, int64_t nrows,
                    oracle_result **out) {
  pair_vec pv = {NULL, 0, 0};
  pair_metric mt;
  int64_t *kappa = NULL;
  int64_t q, s;
  int32_t t;
  int rc = check_points(points, n, d);
  if (rc == ORACLE_OK) rc = check_radius(r);
  if (rc == ORACLE_OK && (k < 1 || !(isfinite(alpha) && alpha > 0.0) || nrows < 0))
    rc = ORACLE_EINVAL;
  if (rc == ORACLE_OK) rc = make_metric(r, d, flags, &mt);
  for (s = 0; rc == ORACLE_OK && s < nrows; ++s)
    if (rows[s] < 0 || rows[s] >= n) rc = ORACLE_EINVAL;
  if (rc != ORACLE_OK) return rc;
  if (n >= 2 && nrows > 0) {
    double inv_c = 1.0 / (alpha * r);
    kappa = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * (size_t)d);
    if (kappa == NULL) return ORACLE_ENOMEM;
    for (t = 0; t < k; ++t) {
      rc = oracle_cell_coords(points, n, d, R + (size_t)t * d * d,
                              u + (size_t)t * d, inv_c, kappa);
      if (rc != ORACLE_OK) goto fail;
      for (s = 0; s < nrows; ++s)
        for (q = 0; q < n; ++q)
          if (q != rows[s] && same_cell(kappa, d, rows[s], q) &&
              within_r(&mt, points, rows[s], q)) {
            rc = pv_push(&pv, s, q); /* (output row, neighbour) */
            if (rc != ORACLE_OK) goto fail;
          }
    }
  }
  sort_unique(&pv); /* a neighbour found by several grids is kept once */
  rc = make_csr(&pv, nrows, ORACLE_UPPER_ONLY, out);
  free(kappa);
  free(pv.v);
  return rc;
fail:
  free(kappa);
  free(pv.v);
  return rc;
}

int oracle_rtg_query(const float *points, int64_t n, int32_t d,
                     const float *queries, int64_t m, double r, int32_t k,
                     double alpha, const double *R, const double *u,
                     uint32_t flags, oracle_result **out) {
  pair_vec pv = {NULL, 0, 0};
  pair_metric mt;
  int64_t *kp = NULL, *kq = NULL;
  int64_t s, i;
  int32_t t, j;
  int rc = check_points(points, n, d);
  if (rc == ORACLE_OK) rc = check_points(queries, m, d);
  if (rc == ORACLE_OK) rc = check_radius(r);
  if (rc == ORACLE_OK && (k < 1 || !(isfinite(alpha) && alpha > 0.0)))
    rc = ORACLE_EINVAL;
  if (rc == ORACLE_OK) rc = make_metric(r, d, flags, &mt);
  if (rc != ORACLE_OK) return rc;
  if (n >= 1 && m >= 1) {
    double inv_c = 1.0 / (alpha * r);
    kp = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * (size_t)d);
    kq = (int64_t *)malloc(sizeof(int64_t) * (size_t)m * (size_t)d);
    if (kp == NULL || kq == NULL) {
      rc = ORACLE_ENOMEM;
      goto done;
    }
    for (t = 0; t < k; ++t) {
      /* the cell of every point and of every query under transform t */
      rc = oracle_cell_coords(points, n, d, R + (size_t)t * d * d,
                              u + (size_t)t * d, inv_c, kp);
      if (rc == ORACLE_OK)
        rc = oracle_cell_coords(queries, m, d, R + (size_t)t * d * d,
                                u + (size_t)t * d, inv_c, kq);
      if (rc != ORACLE_OK) goto done;
      for (s = 0; s < m; ++s)
        for (i = 0; i < n; ++i) {
          int same = 1;
          for (j = 0; j < d && same; ++j)
            same = kq[(size_t)s * d + j] == kp[(size_t)i * d + j];
          if (same && within_metric(&mt, queries + (size_t)s * d,
                                    points + (size_t)i * d)) {
            rc = pv_push(&pv, s, i); /* (query row, indexed point) */
            if (rc != ORACLE_OK) goto done;
          }
        }
    }
  }
  sort_unique(&pv); /* a point found by several grids is kept once */
  rc = make_csr(&pv, m, ORACLE_UPPER_ONLY, out);
done:
  free(kp);
  free(kq);
  free(pv.v);
  return rc;
}

int oracle_bruteforce(const float *points, int64_t n, int32_t d, double r,
                      uint32_t flags, oracle_result **out) {
  pair_vec pv = {NULL, 0, 0};
  pair_metric mt;
  int64_t i, j;
  int rc = check_points(points, n, d);
  if (rc == ORACLE_OK) rc = check_radius(r);
  if (rc == ORACLE_OK) rc = make_metric(r, d, flags, &mt);
  if (rc != ORACLE_OK) return rc;
  for (i = 0; i < n; ++i)
    for (j = i + 1; j < n; ++j)
      if (within_r(&mt, points, i, j)) {
        rc = pv_push(&pv, i, j);
        if (rc != ORACLE_OK) {
          free(pv.v);
          return rc;
        }
      }
  rc = make_csr(&pv, n, flags, out);
  free(pv.v);
  return rc;
}

void oracle_result_free(oracle_result *res) {
  if (res == NULL) return;
  free(res->row_ptr);
  free(res->col);
  free(res);
}

void oracle_free(void *p) { free(p); }
