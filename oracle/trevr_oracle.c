/*
 * trevr_oracle.c -- reference oracle for the TREVR per-sink radiation field.
 *
 * Grond, Woods, Wadsley & Couchman (2019), "TREVR: A general N log^2 N
 * radiative transfer algorithm", MNRAS.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product
 * library neither links nor calls it, and the two share no source.
 *
 * This is a plain, slow, obviously-correct transcription of the method:
 * recursive tree build, recursive source walk, recursive refinement, all in
 * IEEE binary64 (no FMA contraction: build with -ffp-contract=off).  Where the
 * paper is silent the reading taken is stated at the spot.
 *
 * Paper sections followed:
 *   Sec. 2.1, eqs. (dtau), (ient), (simpflux), (simpint): I = L e^-tau/(4 pi s^2)
 *   Sec. 2.2 / 2.3: space-filling binary tree, longest-axis bisection, buckets
 *                   of at most N_B particles, separate radiation tree
 *   Sec. 2.2.1, eq. (openangle): merge at the centre of luminosity when
 *                   theta_open > l/r
 *   Sec. 2.2.2, eqs. (taui), (tausum) and the algorithm figure: walk the ray
 *                   up from the sink bucket and from the source cell, using a
 *                   chain cell's own average away from its child
 *   Sec. 2.2.3, eq. (refcrit): refine where tau_ref < (alpha_max-alpha_min) l;
 *                   directional alpha_min / alpha_max built bottom-up
 *   Sec. 2.3:       volume-weighted cell density sum(m)/sum(m/rho)
 *   Sec. 2.2.4 (background shell): merged background sources on the sphere
 *   Sec. 2.3, 3 (walk variants): a per-bucket opening test, Gasoline's opening
 *                   radius, a top-down ray walk, early termination past tau_max
 *   Sec. 2.2.3 and 2.3 (sub-bucket refinement): below a bucket, an SPH-style
 *                   particle trace, tau = sum_j m_j kappa_j (integral of the
 *                   smoothing kernel along the ray), the receiver excluded
 * The adjoint (gradients of a flux loss) is not in the paper; it is the exact
 * derivative of the forward above with every discrete decision held fixed.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define DMAX 63 /* deepest level: 63 path bits fit a 64-bit key */

typedef struct {
  int64_t first, count; /* range in the sorted particle order */
  int depth, leaf;
  int64_t parent, right, skip; /* left child is always self+1 (pre-order) */
  uint64_t key;                /* path bits, depth-0 decision at bit 62 */
  double lo[3], hi[3], split;  /* space-filling box, split plane */
  double A, B, SL, SLx[3];     /* sum m kappa, sum m/rho, sum L, sum L x */
  double alpha, amin[3], amax[3], alpha_min, alpha_max, dalpha;
  double xl[3], lc, lfar; /* centre of luminosity, luminosity, far vertex */
  /* values as the walk sees them: binary64, or rounded to binary32 */
  double t_lo[3], t_hi[3], t_split, t_xl[3], t_lc, t_lfar, t_alpha, t_dalpha;
} onode;

typedef struct {
  int64_t n, m, cap;
  int nb, mirror32;
  int axis[DMAX + 1];
  double rlo[3], rhi[3];
  double *x, *mass, *rho, *kappa, *lum; /* x is [3n], particle-major */
  uint64_t *pkey;
  int64_t *perm, *leaf_of;
  onode *nd;
  /* bands (oracle_set_bands): transport alpha per band and the band-maximum
   * transport spread, which takes the refinement decisions */
  int nbands;
  double *band_alpha; /* [nbands][m] */
  double *band_dalpha; /* [m] */
  /* sub-bucket particle trace (oracle_set_sph): smoothing lengths, m kappa,
   * each bucket's transport particle spread (-1 for other cells) and the
   * absorbers whose kernel support reaches the bucket's box (CSR by cell) */
  int sph;
  double *sph_h, *sph_mk, *sph_dp, *sph_hmax;
  int64_t *nb_off, *nb_idx;
  /* background shell (oracle_set_background): per cell, whether all of its
   * luminous particles are background sources, and then its merged source
   * moved onto the sphere (transport precision) */
  int bg;
  unsigned char *bg_cell;
  double *bg_pos; /* [m][3] */
} otree;

/* The mirror of binary32 transport: every value the walk reads is rounded
 * once to binary32, and the ray's geometry (direction, 1/d, r^2, r, plane
 * crossings, piece lengths) is computed in binary32, which tr() gives here by
 * rounding each binary64 operation on binary32 operands: for +, -, *, / and
 * sqrt that equals the correctly rounded binary32 operation, since binary64
 * carries more than twice binary32's precision plus two bits.  The products
 * alpha l and (alpha_max - alpha_min) l of two binary32 values, and the sums
 * of tau and the flux, are exact or binary64 in both modes. */
static double tr(const otree *t, double v) {
  return t->mirror32 ? (double)(float)v : v;
}

/* ---------------------------------------------------------------- tree ---- */

/* Split axis per depth: bisect the longest axis of the current cell shape
 * (Sec. 2.3).  All cells at one depth share one shape, so the axis depends on
 * the depth only.  Ties go to the lowest axis index (reading: paper silent). */
static void level_axes(otree *t) {
  double w[3];
  for (int a = 0; a < 3; ++a) w[a] = t->rhi[a] - t->rlo[a];
  for (int d = 0; d <= DMAX; ++d) {
    int a = 0;
    if (w[1] > w[a]) a = 1;
    if (w[2] > w[a]) a = 2;
    t->axis[d] = a;
    w[a] *= 0.5;
  }
}

/* A particle's path: at each level the cell is cut at the midpoint of its
 * split axis; a point on the plane goes to the upper (right) child. */
static uint64_t path_key(const otree *t, const double *x) {
  double lo[3], hi[3];
  uint64_t k = 0;
  memcpy(lo, t->rlo, sizeof lo);
  memcpy(hi, t->rhi, sizeof hi);
  for (int d = 0; d < DMAX; ++d) {
    int a = t->axis[d];
    double s = 0.5 * (lo[a] + hi[a]);
    if (x[a] >= s) {
      k |= (uint64_t)1 << (62 - d);
      lo[a] = s;
    } else {
      hi[a] = s;
    }
  }
  return k;
}

static const uint64_t *g_sort_keys; /* qsort has no context argument */
static int cmp_key_index(const void *pa, const void *pb) {
  int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
  uint64_t ka = g_sort_keys[a], kb = g_sort_keys[b];
  if (ka != kb) return ka < kb ? -1 : 1;
  return a < b ? -1 : (a > b);
}

static int64_t new_node(otree *t) {
  if (t->m == t->cap) {
    t->cap = t->cap ? 2 * t->cap : 1024;
    t->nd = (onode *)realloc(t->nd, (size_t)t->cap * sizeof(onode));
  }
  memset(&t->nd[t->m], 0, sizeof(onode));
  return t->m++;
}

/* Nodes are numbered in depth-first pre-order, left before right.  A cell
 * with more than N_B particles (and depth below DMAX) gets both children even
 * when one is empty: the radiation tree must fill space (Sec. 2.2.2, 2.3). */
static int64_t build_node(otree *t, int64_t b, int64_t e, int depth,
                          uint64_t prefix, const double lo[3],
                          const double hi[3], int64_t parent) {
  int64_t id = new_node(t);
  onode *p = &t->nd[id];
  p->first = b;
  p->count = e - b;
  p->depth = depth;
  p->parent = parent;
  p->key = prefix;
  memcpy(p->lo, lo, 3 * sizeof(double));
  memcpy(p->hi, hi, 3 * sizeof(double));
  if (e - b > t->nb && depth < DMAX) {
    int a = t->axis[depth];
    double s = 0.5 * (lo[a] + hi[a]);
    int64_t mid = b;
    while (mid < e && !((t->pkey[t->perm[mid]] >> (62 - depth)) & 1)) ++mid;
    double lhi[3], rlo[3];
    memcpy(lhi, hi, sizeof lhi);
    memcpy(rlo, lo, sizeof rlo);
    lhi[a] = s;
    rlo[a] = s;
    build_node(t, b, mid, depth + 1, prefix, lo, lhi, id);
    int64_t r = build_node(t, mid, e, depth + 1,
                           prefix | ((uint64_t)1 << (62 - depth)), rlo, hi, id);
    p = &t->nd[id]; /* the array may have moved */
    p->leaf = 0;
    p->split = s;
    p->right = r;
  } else {
    p->leaf = 1;
    p->right = -1;
    p->split = 0.0;
    for (int64_t k = b; k < e; ++k) t->leaf_of[t->perm[k]] = id;
  }
  t->nd[id].skip = t->m;
  return id;
}

/* Cell properties (Sec. 2.2.1, 2.2.3, 2.3). */
static void cell_properties(otree *t) {
  /* sums, bottom-up: children have larger pre-order indices than parents */
  for (int64_t id = t->m - 1; id >= 0; --id) {
    onode *p = &t->nd[id];
    if (p->leaf) {
      for (int64_t k = p->first; k < p->first + p->count; ++k) {
        int64_t q = t->perm[k];
        if (t->mass[q] > 0) {
          p->A += t->mass[q] * t->kappa[q];
          p->B += t->mass[q] / t->rho[q];
        }
        p->SL += t->lum[q];
        for (int a = 0; a < 3; ++a) p->SLx[a] += t->lum[q] * t->x[3 * q + a];
      }
    } else {
      const onode *l = &t->nd[id + 1], *r = &t->nd[p->right];
      p->A = l->A + r->A;
      p->B = l->B + r->B;
      p->SL = l->SL + r->SL;
      for (int a = 0; a < 3; ++a) p->SLx[a] = l->SLx[a] + r->SLx[a];
    }
  }
  /* absorption coefficient alpha = kappa rho_cell with the volume-weighted
   * density; a cell with no absorbing mass takes its parent's value (reading:
   * paper silent), top-down */
  for (int64_t id = 0; id < t->m; ++id) {
    onode *p = &t->nd[id];
    if (p->B > 0)
      p->alpha = p->A / p->B;
    else
      p->alpha = (p->parent < 0) ? 0.0 : t->nd[p->parent].alpha;
  }
  /* directional bounds, bottom-up: along the split axis a ray crosses both
   * children, so their optical depths add and the sum is divided by the
   * parent width (children have equal widths: the mean); across it a ray
   * sees one child or the other (min / max). */
  for (int64_t id = t->m - 1; id >= 0; --id) {
    onode *p = &t->nd[id];
    if (p->leaf) {
      for (int b = 0; b < 3; ++b) p->amin[b] = p->amax[b] = p->alpha;
    } else {
      const onode *l = &t->nd[id + 1], *r = &t->nd[p->right];
      int s = t->axis[p->depth];
      for (int b = 0; b < 3; ++b) {
        if (b == s) {
          p->amin[b] = 0.5 * (l->amin[b] + r->amin[b]);
          p->amax[b] = 0.5 * (l->amax[b] + r->amax[b]);
        } else {
          p->amin[b] = l->amin[b] < r->amin[b] ? l->amin[b] : r->amin[b];
          p->amax[b] = l->amax[b] > r->amax[b] ? l->amax[b] : r->amax[b];
        }
      }
    }
    double mn = p->amin[0], mx = p->amax[0];
    for (int b = 1; b < 3; ++b) {
      if (p->amin[b] < mn) mn = p->amin[b];
      if (p->amax[b] > mx) mx = p->amax[b];
    }
    p->alpha_min = mn;
    p->alpha_max = mx;
    p->dalpha = mx - mn;
  }
  /* merged source: centre of luminosity and the distance from it to the
   * furthest vertex of the (space-filling) cell */
  for (int64_t id = 0; id < t->m; ++id) {
    onode *p = &t->nd[id];
    if (p->SL > 0) {
      p->lc = p->SL;
      for (int a = 0; a < 3; ++a) p->xl[a] = p->SLx[a] / p->SL;
      double far2 = 0.0;
      for (int v = 0; v < 8; ++v) {
        double dv[3];
        for (int a = 0; a < 3; ++a)
          dv[a] = ((v >> a) & 1 ? p->hi[a] : p->lo[a]) - p->xl[a];
        double q = (dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2];
        if (q > far2) far2 = q;
      }
      p->lfar = sqrt(far2);
    }
  }
  for (int64_t id = 0; id < t->m; ++id) {
    onode *p = &t->nd[id];
    for (int a = 0; a < 3; ++a) {
      p->t_lo[a] = tr(t, p->lo[a]);
      p->t_hi[a] = tr(t, p->hi[a]);
      p->t_xl[a] = tr(t, p->xl[a]);
    }
    p->t_split = tr(t, p->split);
    p->t_lc = tr(t, p->lc);
    p->t_lfar = tr(t, p->lfar);
    p->t_alpha = tr(t, p->alpha);
    p->t_dalpha = tr(t, p->dalpha);
  }
}

/* Cell alpha and spread for one opacity field kap (per particle), with the
 * same sums, inheritance and directional bounds as cell_properties. */
static void band_properties(const otree *t, const double *kap, double *alpha, double *dalpha) {
  double *A = (double *)calloc((size_t)t->m, sizeof(double));
  double *amin = (double *)malloc(3 * (size_t)t->m * sizeof(double));
  double *amax = (double *)malloc(3 * (size_t)t->m * sizeof(double));
  for (int64_t id = t->m - 1; id >= 0; --id) {
    const onode *p = &t->nd[id];
    if (p->leaf) {
      for (int64_t k = p->first; k < p->first + p->count; ++k) {
        int64_t q = t->perm[k];
        if (t->mass[q] > 0) A[id] += t->mass[q] * kap[q];
      }
    } else {
      A[id] = A[id + 1] + A[p->right];
    }
  }
  for (int64_t id = 0; id < t->m; ++id) {
    const onode *p = &t->nd[id];
    if (p->B > 0)
      alpha[id] = A[id] / p->B;
    else
      alpha[id] = (p->parent < 0) ? 0.0 : alpha[p->parent];
  }
  for (int64_t id = t->m - 1; id >= 0; --id) {
    const onode *p = &t->nd[id];
    double *mn = &amin[3 * id], *mx = &amax[3 * id];
    if (p->leaf) {
      for (int b = 0; b < 3; ++b) mn[b] = mx[b] = alpha[id];
    } else {
      const double *lmn = &amin[3 * (id + 1)], *lmx = &amax[3 * (id + 1)];
      const double *rmn = &amin[3 * p->right], *rmx = &amax[3 * p->right];
      int s = t->axis[p->depth];
      for (int b = 0; b < 3; ++b) {
        if (b == s) {
          mn[b] = 0.5 * (lmn[b] + rmn[b]);
          mx[b] = 0.5 * (lmx[b] + rmx[b]);
        } else {
          mn[b] = lmn[b] < rmn[b] ? lmn[b] : rmn[b];
          mx[b] = lmx[b] > rmx[b] ? lmx[b] : rmx[b];
        }
      }
    }
    double lo = mn[0], hi = mx[0];
    for (int b = 1; b < 3; ++b) {
      if (mn[b] < lo) lo = mn[b];
      if (mx[b] > hi) hi = mx[b];
    }
    dalpha[id] = hi - lo;
  }
  free(A);
  free(amin);
  free(amax);
}

/* Several opacity bands on one traversal (a reading: the paper's method
 * carries one opacity): band b's cell alpha comes from kappa_b exactly as the
 * tree's own alpha comes from kappa; a piece is refined where any band's
 * criterion asks for it, (max_b spread_b) l > tau_ref, so every band meets
 * eq. (refcrit).  kappa_bands: [k][n], k <= 8. */
int oracle_set_bands(void *h, int k, const double *kappa_bands) {
  otree *t = (otree *)h;
  if (k < 1 || k > 8) return -1;
  free(t->band_alpha);
  free(t->band_dalpha);
  t->nbands = k;
  t->band_alpha = (double *)malloc((size_t)k * (size_t)t->m * sizeof(double));
  t->band_dalpha = (double *)calloc((size_t)t->m, sizeof(double));
  double *da = (double *)malloc((size_t)t->m * sizeof(double));
  for (int b = 0; b < k; ++b) {
    double *al = t->band_alpha + (size_t)b * (size_t)t->m;
    band_properties(t, kappa_bands + (size_t)b * (size_t)t->n, al, da);
    for (int64_t id = 0; id < t->m; ++id) {
      al[id] = tr(t, al[id]);
      const double d = tr(t, da[id]);
      if (d > t->band_dalpha[id]) t->band_dalpha[id] = d;
    }
  }
  free(da);
  return 0;
}

void oracle_free(void *h) {
  otree *t = (otree *)h;
  if (!t) return;
  free(t->x);
  free(t->mass);
  free(t->rho);
  free(t->kappa);
  free(t->lum);
  free(t->pkey);
  free(t->perm);
  free(t->leaf_of);
  free(t->nd);
  free(t->band_alpha);
  free(t->band_dalpha);
  free(t->sph_h);
  free(t->sph_mk);
  free(t->sph_dp);
  free(t->sph_hmax);
  free(t->nb_off);
  free(t->nb_idx);
  free(t->bg_cell);
  free(t->bg_pos);
  free(t);
}

/* Build the tree and its properties.  mass may be NULL (all ones).  Returns
 * NULL on invalid input (particle outside [lo, hi), non-positive density of
 * an absorber, negative opacity or luminosity, N_B < 1). */
void *oracle_build(int64_t n, const double *x, const double *y,
                   const double *z, const double *mass, const double *rho,
                   const double *kappa, const double *lum, const double *lo,
                   const double *hi, int nb, int mirror32) {
  if (n < 0 || nb < 1) return NULL;
  otree *t = (otree *)calloc(1, sizeof(otree));
  t->n = n;
  t->nb = nb;
  t->mirror32 = mirror32;
  for (int a = 0; a < 3; ++a) {
    t->rlo[a] = lo[a];
    t->rhi[a] = hi[a];
    if (!(hi[a] > lo[a])) {
      oracle_free(t);
      return NULL;
    }
  }
  size_t nn = (size_t)(n > 0 ? n : 1);
  t->x = (double *)malloc(3 * nn * sizeof(double));
  t->mass = (double *)malloc(nn * sizeof(double));
  t->rho = (double *)malloc(nn * sizeof(double));
  t->kappa = (double *)malloc(nn * sizeof(double));
  t->lum = (double *)malloc(nn * sizeof(double));
  t->pkey = (uint64_t *)malloc(nn * sizeof(uint64_t));
  t->perm = (int64_t *)malloc(nn * sizeof(int64_t));
  t->leaf_of = (int64_t *)malloc(nn * sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]};
    for (int a = 0; a < 3; ++a) {
      if (!(p[a] >= lo[a] && p[a] < hi[a])) {
        oracle_free(t);
        return NULL;
      }
      t->x[3 * i + a] = tr(t, p[a]);
    }
    t->mass[i] = mass ? mass[i] : 1.0;
    t->rho[i] = rho[i];
    t->kappa[i] = kappa[i];
    t->lum[i] = tr(t, lum[i]);
    if (!(t->mass[i] >= 0) || !(t->kappa[i] >= 0) || !(t->lum[i] >= 0) ||
        (t->mass[i] > 0 && !(t->rho[i] > 0)) || !isfinite(t->rho[i]) ||
        !isfinite(t->kappa[i]) || !isfinite(t->lum[i]) ||
        !isfinite(t->mass[i])) {
      oracle_free(t);
      return NULL;
    }
  }
  level_axes(t);
  for (int64_t i = 0; i < n; ++i) {
    t->pkey[i] = path_key(t, &t->x[3 * i]);
    t->perm[i] = i;
  }
  g_sort_keys = t->pkey;
  qsort(t->perm, (size_t)n, sizeof(int64_t), cmp_key_index);
  build_node(t, 0, n, 0, 0, t->rlo, t->rhi, -1);
  cell_properties(t);
  return t;
}

int64_t oracle_num_nodes(void *h) { return ((otree *)h)->m; }
int oracle_axis(void *h, int depth) { return ((otree *)h)->axis[depth]; }

/* Node export.  node_i: 8 per node {first, count, depth, leaf, parent, right,
 * skip, axis-of-depth}.  node_f: ORACLE_NF per node, see the order below. */
#define ORACLE_NF 22
int oracle_export(void *h, int64_t *perm, int64_t *leaf_of, int64_t *node_i,
                  uint64_t *node_key, double *node_f) {
  otree *t = (otree *)h;
  for (int64_t i = 0; i < t->n; ++i) {
    if (perm) perm[i] = t->perm[i];
    if (leaf_of) leaf_of[i] = t->leaf_of[i];
  }
  for (int64_t id = 0; id < t->m; ++id) {
    const onode *p = &t->nd[id];
    if (node_i) {
      int64_t *o = node_i + 8 * id;
      o[0] = p->first;
      o[1] = p->count;
      o[2] = p->depth;
      o[3] = p->leaf;
      o[4] = p->parent;
      o[5] = p->right;
      o[6] = p->skip;
      o[7] = t->axis[p->depth];
    }
    if (node_key) node_key[id] = p->key;
    if (node_f) {
      double *o = node_f + ORACLE_NF * id;
      for (int a = 0; a < 3; ++a) {
        o[0 + a] = p->lo[a];
        o[3 + a] = p->hi[a];
        o[10 + a] = p->SLx[a];
        o[17 + a] = p->xl[a];
      }
      o[6] = p->split;
      o[7] = p->A;
      o[8] = p->B;
      o[9] = p->SL;
      o[13] = p->alpha;
      o[14] = p->alpha_min;
      o[15] = p->alpha_max;
      o[16] = p->dalpha;
      o[20] = p->lc;
      o[21] = p->lfar;
    }
  }
  return 0;
}

/* Export of the values the walk reads (the transport copy): binary64, or, in
 * mirror mode, each rounded once to binary32 from its binary64 value.
 * ORACLE_NT per node: lo[3], hi[3], split, x_L[3], L_C, l_far, alpha,
 * alpha_max - alpha_min.  pos receives the particle positions and lum the
 * luminosities the walk reads (input order, 3 and 1 per particle). */
#define ORACLE_NT 14
int oracle_export_transport(void *h, double *node_t, double *pos, double *lum) {
  const otree *t = (const otree *)h;
  for (int64_t id = 0; id < t->m && node_t; ++id) {
    const onode *p = &t->nd[id];
    double *o = node_t + ORACLE_NT * id;
    for (int a = 0; a < 3; ++a) {
      o[0 + a] = p->t_lo[a];
      o[3 + a] = p->t_hi[a];
      o[7 + a] = p->t_xl[a];
    }
    o[6] = p->t_split;
    o[10] = p->t_lc;
    o[11] = p->t_lfar;
    o[12] = p->t_alpha;
    o[13] = p->t_dalpha;
  }
  for (int64_t i = 0; i < t->n; ++i) {
    if (pos)
      for (int a = 0; a < 3; ++a) pos[3 * i + a] = t->x[3 * i + a];
    if (lum) lum[i] = t->lum[i];
  }
  return 0;
}

/* ------------------------------------------------------------ the walk ---- */

typedef struct {
  int64_t node;      /* cell whose alpha multiplies this piece */
  double ta, tb;     /* piece of the ray, parameter t in [0,1] from the sink */
  int taga, tagb;    /* axis of the plane that produced ta / tb, -1 if none */
  double alpha, len; /* alpha used and the length r (tb - ta) */
} oseg;

typedef struct {
  double d[3], inv[3], r2, r;
  double tau;
  double tau_b[8]; /* per band (band mode) */
  int nseg, cap;
  oseg *seg;
} oray;

typedef struct {
  const otree *t;
  int64_t i, S;
  double xi[3];
  double theta2, tau_ref;
  double F, G;
  double Fv[3]; /* vector flux: sum of f times the unit vector from source to sink */
  double Pm[6]; /* second moment: sum of f n_a n_b (xx, yy, zz, xy, xz, yz) */
  int bands;     /* band mode: per-band tau and flux, band-maximum spread */
  int sph;       /* sub-bucket particle trace below the buckets */
  int bg;        /* merged background sources on the sphere */
  /* walk variants: opening test 0 eq. (openangle) at the sink point, 1 at the
   * sink's bucket box, 2 Gasoline's opening radius about x_L; ray walk 0 up
   * the tree (Sec. 2.2.2), 1 top down from the meeting cell; rays with
   * tau > tau_max contribute nothing (early termination) */
  int open_mode, ray_mode;
  double tau_max;
  double Fb[8];
  int64_t n_open, n_rays, n_psrc, n_seg, n_trace;
  /* adjoint accumulators (NULL in a forward pass) */
  double w;
  double *abar, *lbar, *xbar, *direct;
  /* optional piece log of one ray (ray number piece_ray of the walk) */
  int64_t piece_ray, piece_n, piece_cap;
  int64_t *piece_node;
  double *piece_t; /* ta, tb, alpha, len per piece */
  /* optional ray log */
  int64_t log_n, log_cap;
  int64_t *log_C, *log_src;
  double *log_y, *log_L, *log_tau, *log_f;
} osink;

/* the spread (alpha_max - alpha_min) that takes a cell's refinement decision */
static double spread(const osink *c, int64_t X) {
  return c->bands ? c->t->band_dalpha[X] : c->t->nd[X].t_dalpha;
}

/* ---------------------------------------------- sub-bucket particle trace ---- */

/* The M4 cubic spline kernel with support 2h, W(r, h) = w(r/h) / (pi h^3),
 * normalised so that its volume integral is one. */
static double w_m4(double q) {
  if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
  if (q < 2.0) {
    double u = 2.0 - q;
    return 0.25 * u * u * u;
  }
  return 0.0;
}

/* The integrand of the line integral in units of h: w(sqrt(beta^2 + s^2)). */
static double w_line(double beta, double s) { return w_m4(sqrt(beta * beta + s * s)); }

/* Five-point Gauss-Legendre rule on [a, b] (nodes and weights from their
 * closed forms: 0, +-sqrt(5 -+ 2 sqrt(10/7)) / 3). */
static double gl5(double beta, double a, double b) {
  const double x1 = sqrt(5.0 - 2.0 * sqrt(10.0 / 7.0)) / 3.0;
  const double x2 = sqrt(5.0 + 2.0 * sqrt(10.0 / 7.0)) / 3.0;
  const double w0 = 128.0 / 225.0;
  const double w1 = (322.0 + 13.0 * sqrt(70.0)) / 900.0;
  const double w2 = (322.0 - 13.0 * sqrt(70.0)) / 900.0;
  const double c = 0.5 * (a + b), hw = 0.5 * (b - a);
  double sum = w0 * w_line(beta, c);
  sum += w1 * (w_line(beta, c - hw * x1) + w_line(beta, c + hw * x1));
  sum += w2 * (w_line(beta, c - hw * x2) + w_line(beta, c + hw * x2));
  return hw * sum;
}

/* Adaptive quadrature: the rule on [a, b] against the rule on its halves,
 * to 1e-15 per unit length (w <= 1, so rounding stays below that). */
static double gl5_adapt(double beta, double a, double b, double whole, int depth) {
  double m = 0.5 * (a + b);
  double left = gl5(beta, a, m), right = gl5(beta, m, b);
  double two = left + right;
  if (depth >= 40 || fabs(two - whole) <= 1e-15 * (b - a)) return two;
  return gl5_adapt(beta, a, m, left, depth + 1) + gl5_adapt(beta, m, b, right, depth + 1);
}

/* Integral of W(sqrt(b^2 + u^2), h) over u in [u0, u1] (u0 <= u1): the
 * plain definition, by adaptive quadrature on the pieces between the points
 * where the kernel's formula changes (q = 1, 2) and the closest approach. */
double oracle_sph_line(double b, double h, double u0, double u1) {
  if (!(h > 0) || !(u1 > u0)) return 0.0;
  double beta = b / h, s0 = u0 / h, s1 = u1 / h;
  if (beta >= 2.0) return 0.0;
  double e2 = sqrt(4.0 - beta * beta);
  double cuts[7];
  int nc = 0;
  cuts[nc++] = -e2;
  if (beta < 1.0) cuts[nc++] = -sqrt(1.0 - beta * beta);
  cuts[nc++] = 0.0;
  if (beta < 1.0) cuts[nc++] = sqrt(1.0 - beta * beta);
  cuts[nc++] = e2;
  double total = 0.0;
  for (int k = 0; k + 1 < nc; ++k) {
    double a = cuts[k] > s0 ? cuts[k] : s0;
    double e = cuts[k + 1] < s1 ? cuts[k + 1] : s1;
    if (e > a) total += gl5_adapt(beta, a, e, gl5(beta, a, e), 0);
  }
  return total / (M_PI * h * h);
}

/* Optical depth of the ray piece [ta, tb] inside bucket X, Sec. 2.3: each
 * absorber j whose kernel reaches the bucket adds m_j kappa_j times the
 * kernel's integral over the piece; the receiving particle does not absorb
 * its own radiation. */
static double sph_piece(const osink *c, const oray *ry, int64_t X, double ta, double tb) {
  const otree *t = c->t;
  double tau = 0.0;
  for (int64_t k = t->nb_off[X]; k < t->nb_off[X + 1]; ++k) {
    int64_t j = t->nb_idx[k];
    if (j == c->i) continue;
    const double *xj = &t->x[3 * j];
    double dl[3], p[3];
    for (int a = 0; a < 3; ++a) dl[a] = xj[a] - c->xi[a];
    /* closest approach to the ray's line at parameter ts */
    double ts = ((dl[0] * ry->d[0] + dl[1] * ry->d[1]) + dl[2] * ry->d[2]) / ry->r2;
    for (int a = 0; a < 3; ++a) p[a] = dl[a] - ts * ry->d[a];
    double b = sqrt((p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]);
    tau += t->sph_mk[j] * oracle_sph_line(b, t->sph_h[j], (ta - ts) * ry->r, (tb - ts) * ry->r);
  }
  return tau;
}

/* the absorbers whose kernel support (radius 2 h) reaches box [lo, hi], by a
 * query down the tree; each cell carries the largest h of its absorbers */
static void sph_query(const otree *t, int64_t C, const double *lo, const double *hi,
                      int64_t *out, int64_t *n, int count_only) {
  const onode *p = &t->nd[C];
  if (!(t->sph_hmax[C] > 0)) return;
  double g2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    double g = p->lo[a] - hi[a];
    double g1 = lo[a] - p->hi[a];
    if (g1 > g) g = g1;
    if (g > 0) g2 += g * g;
  }
  if (!(g2 < 4.0 * t->sph_hmax[C] * t->sph_hmax[C])) return;
  if (p->leaf) {
    for (int64_t k = p->first; k < p->first + p->count; ++k) {
      int64_t j = t->perm[k];
      if (!(t->sph_mk[j] > 0)) continue;
      double d2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        double v = t->x[3 * j + a];
        double g = lo[a] - v > v - hi[a] ? lo[a] - v : v - hi[a];
        if (g > 0) d2 += g * g;
      }
      if (d2 < 4.0 * t->sph_h[j] * t->sph_h[j]) {
        if (!count_only) out[*n] = j;
        ++*n;
      }
    }
    return;
  }
  sph_query(t, C + 1, lo, hi, out, n, count_only);
  sph_query(t, p->right, lo, hi, out, n, count_only);
}

/* Smoothing lengths h (input order, > 0) for the sub-bucket particle trace.
 * A bucket's refinement decision uses the spread of its particles' absorption
 * coefficients kappa rho (those with mass), in the transport precision. */
int oracle_set_sph(void *hd, const double *h) {
  otree *t = (otree *)hd;
  for (int64_t i = 0; i < t->n; ++i)
    if (!(h[i] > 0) || !isfinite(h[i])) return -1;
  size_t nn = (size_t)(t->n > 0 ? t->n : 1), mm = (size_t)t->m;
  free(t->sph_h);
  free(t->sph_mk);
  free(t->sph_dp);
  free(t->sph_hmax);
  free(t->nb_off);
  free(t->nb_idx);
  t->sph_h = (double *)malloc(nn * sizeof(double));
  t->sph_mk = (double *)malloc(nn * sizeof(double));
  t->sph_dp = (double *)malloc(mm * sizeof(double));
  t->sph_hmax = (double *)calloc(mm, sizeof(double));
  t->nb_off = (int64_t *)calloc(mm + 1, sizeof(int64_t));
  for (int64_t i = 0; i < t->n; ++i) {
    t->sph_h[i] = tr(t, h[i]);
    t->sph_mk[i] = t->mass[i] > 0 ? t->mass[i] * t->kappa[i] : 0.0;
  }
  for (int64_t id = t->m - 1; id >= 0; --id) {
    const onode *p = &t->nd[id];
    t->sph_dp[id] = -1.0;
    if (p->leaf) {
      double lo = INFINITY, hi = -INFINITY, hm = 0.0;
      for (int64_t k = p->first; k < p->first + p->count; ++k) {
        int64_t j = t->perm[k];
        if (t->mass[j] > 0) {
          double a = t->kappa[j] * t->rho[j];
          if (a < lo) lo = a;
          if (a > hi) hi = a;
        }
        if (t->sph_mk[j] > 0 && t->sph_h[j] > hm) hm = t->sph_h[j];
      }
      t->sph_dp[id] = hi >= lo ? tr(t, hi - lo) : 0.0;
      t->sph_hmax[id] = hm;
    } else {
      double a = t->sph_hmax[id + 1], b = t->sph_hmax[p->right];
      t->sph_hmax[id] = a > b ? a : b;
    }
  }
  for (int64_t id = 0; id < t->m; ++id) {
    int64_t cnt = 0;
    if (t->nd[id].leaf) sph_query(t, 0, t->nd[id].lo, t->nd[id].hi, NULL, &cnt, 1);
    t->nb_off[id + 1] = t->nb_off[id] + cnt;
  }
  t->nb_idx = (int64_t *)malloc((size_t)(t->nb_off[t->m] > 0 ? t->nb_off[t->m] : 1) *
                                sizeof(int64_t));
  for (int64_t id = 0; id < t->m; ++id) {
    int64_t cnt = 0;
    if (t->nd[id].leaf)
      sph_query(t, 0, t->nd[id].lo, t->nd[id].hi, t->nb_idx + t->nb_off[id], &cnt, 0);
  }
  t->sph = 1;
  return 0;
}

/* A bucket's absorbers (input indices, tree order); returns their number. */
int64_t oracle_sph_neighbours(void *hd, int64_t node, int64_t cap, int64_t *out) {
  const otree *t = (const otree *)hd;
  if (!t->sph || node < 0 || node >= t->m) return -1;
  int64_t n = t->nb_off[node + 1] - t->nb_off[node];
  for (int64_t k = 0; k < n && k < cap; ++k) out[k] = t->nb_idx[t->nb_off[node] + k];
  return n;
}

/* Each cell's sub-bucket decision spread (-1 for cells that are not buckets). */
int oracle_sph_spread(void *hd, double *dp) {
  const otree *t = (const otree *)hd;
  if (!t->sph) return -1;
  for (int64_t id = 0; id < t->m; ++id) dp[id] = t->sph_dp[id];
  return 0;
}

/* one alpha * l term of eq. (tausum) */
static void add_piece(osink *c, oray *ry, int64_t node, double ta, int taga,
                      double tb, int tagb, double l) {
  double alpha = c->t->nd[node].t_alpha;
  if (l > 0) c->n_seg++;
  if (c->sph && c->t->nd[node].leaf && c->t->sph_dp[node] * l > c->tau_ref)
    ry->tau += sph_piece(c, ry, node, ta, tb); /* refinement below the bucket */
  else
    ry->tau += alpha * l;
  if (c->bands)
    for (int b = 0; b < c->t->nbands; ++b)
      ry->tau_b[b] += c->t->band_alpha[(size_t)b * (size_t)c->t->m + (size_t)node] * l;
  if (c->abar || (c->piece_node && c->log_n == c->piece_ray)) {
    if (ry->nseg == ry->cap) {
      ry->cap = ry->cap ? 2 * ry->cap : 32;
      ry->seg = (oseg *)realloc(ry->seg, (size_t)ry->cap * sizeof(oseg));
    }
    oseg *s = &ry->seg[ry->nseg++];
    s->node = node;
    s->ta = ta;
    s->tb = tb;
    s->taga = taga;
    s->tagb = tagb;
    s->alpha = alpha;
    s->len = l;
  }
}

/* Refinement (Sec. 2.2.3): use cell X's average on [ta, tb] unless
 * tau_ref < (alpha_max - alpha_min) l, in which case the cell's children
 * are used instead, recursively.  Buckets are not refined further (the
 * sub-bucket particle trace is a separate step). */
static void refine(osink *c, oray *ry, int64_t X, double ta, int taga,
                   double tb, int tagb) {
  const otree *t = c->t;
  const onode *p = &t->nd[X];
  double l = tr(t, ry->r * tr(t, tb - ta));
  c->n_trace++;
  if (p->leaf || !(spread(c, X) * l > c->tau_ref)) {
    add_piece(c, ry, X, ta, taga, tb, tagb, l);
    return;
  }
  int ax = t->axis[p->depth];
  double s = p->t_split;
  int64_t L = X + 1, R = p->right;
  if (ry->d[ax] == 0.0) { /* ray parallel to the plane: one side only */
    refine(c, ry, c->xi[ax] >= s ? R : L, ta, taga, tb, tagb);
    return;
  }
  double ts = tr(t, tr(t, s - c->xi[ax]) * ry->inv[ax]);
  int64_t nearc = ry->d[ax] > 0 ? L : R;
  int64_t farc = ry->d[ax] > 0 ? R : L;
  double t1 = tb;
  int g1 = tagb;
  if (ts < tb) {
    t1 = ts;
    g1 = ax;
  }
  if (t1 > ta) refine(c, ry, nearc, ta, taga, t1, g1);
  double t0 = ta;
  int g0 = taga;
  if (ts > ta) {
    t0 = ts;
    g0 = ax;
  }
  if (tb > t0) refine(c, ry, farc, t0, g0, tb, tagb);
}

/* A piece of the ray inside chain cell P but outside P's child on the path,
 * i.e. inside the sibling X.  The chain cell's own average is used there
 * (the ray walks up the tree: lowest resolution mid-ray); if P fails the
 * refinement test the sibling is refined instead. */
static void chain_piece(osink *c, oray *ry, int64_t P, int64_t X, double ta,
                        int taga, double tb, int tagb) {
  double l = tr(c->t, ry->r * tr(c->t, tb - ta));
  c->n_trace++;
  if (spread(c, P) * l > c->tau_ref) {
    refine(c, ry, X, ta, taga, tb, tagb);
    return;
  }
  add_piece(c, ry, P, ta, taga, tb, tagb, l);
}

static int key_bit(uint64_t k, int depth) { return (int)((k >> (62 - depth)) & 1); }

/* Reverse ray trace from the sink (t = 0) to a source at y in cell C (t = 1).
 * Eqs. (taui), (tausum); the flux contribution is eq. (simpint). */
static void trace_ray(osink *c, int64_t C, const double y[3], double L,
                      int64_t src) {
  const otree *t = c->t;
  oray ry;
  memset(&ry, 0, sizeof ry);
  for (int a = 0; a < 3; ++a) {
    ry.d[a] = tr(t, y[a] - c->xi[a]);
    ry.inv[a] = ry.d[a] != 0.0 ? tr(t, 1.0 / ry.d[a]) : 0.0;
  }
  ry.r2 = tr(t, tr(t, tr(t, ry.d[0] * ry.d[0]) + tr(t, ry.d[1] * ry.d[1])) +
                    tr(t, ry.d[2] * ry.d[2]));
  ry.r = tr(t, sqrt(ry.r2));
  const int64_t S = c->S;
  if (C == S) {
    c->n_trace++;
    add_piece(c, &ry, S, 0.0, -1, 1.0, -1, ry.r * (1.0 - 0.0));
  } else {
    uint64_t kS = t->nd[S].key, kC = t->nd[C].key;
    int a = __builtin_clzll(kS ^ kC) - 1; /* depth of the meeting cell */
    int64_t A = S;
    while (t->nd[A].depth > a) A = t->nd[A].parent;
    if (c->ray_mode == 1) {
      /* top down (Sec. 3 discussion of other walks): the meeting cell holds
       * the whole ray; refine it from there by eq. (refcrit) alone */
      refine(c, &ry, A, 0.0, -1, 1.0, -1);
      goto done;
    }
    int axA = t->axis[a];
    double sA = t->nd[A].t_split;
    int sr = key_bit(kS, a), cr = key_bit(kC, a);
    double tA;
    int gA;
    if (ry.d[axA] != 0.0) {
      tA = tr(t, tr(t, sA - c->xi[axA]) * ry.inv[axA]);
      gA = axA;
      if (tA < 0.0) {
        tA = 0.0;
        gA = -1;
      }
      if (tA > 1.0) {
        tA = 1.0;
        gA = -1;
      }
    } else { /* ray in the plane: it belongs to the upper side */
      tA = sr ? 1.0 : 0.0;
      gA = -1;
    }
    /* sink side: [0, tA] lies in A's child toward S; walk down to S */
    double tP = tA;
    int gP = gA;
    int64_t P = sr ? t->nd[A].right : A + 1;
    for (int dd = a + 1; dd < t->nd[S].depth; ++dd) {
      int b = key_bit(kS, dd);
      int ax = t->axis[dd];
      int64_t child = b ? t->nd[P].right : P + 1;
      int64_t sib = b ? P + 1 : t->nd[P].right;
      double dax = ry.d[ax];
      if (dax != 0.0 && ((!b && dax > 0) || (b && dax < 0))) {
        double tc = tr(t, tr(t, t->nd[P].t_split - c->xi[ax]) * ry.inv[ax]);
        int gc = ax;
        if (tc < 0.0) {
          tc = 0.0;
          gc = -1;
        }
        if (tc < tP) {
          chain_piece(c, &ry, P, sib, tc, gc, tP, gP);
          tP = tc;
          gP = gc;
        }
      }
      P = child;
    }
    c->n_trace++;
    add_piece(c, &ry, S, 0.0, -1, tP, gP, tr(t, ry.r * tr(t, tP - 0.0)));
    /* source side: [tA, 1] lies in A's child toward C; walk down to C */
    double tQ = tA;
    int gQ = gA;
    int64_t Q = cr ? t->nd[A].right : A + 1;
    for (int dd = a + 1; dd < t->nd[C].depth; ++dd) {
      int b = key_bit(kC, dd);
      int ax = t->axis[dd];
      int64_t child = b ? t->nd[Q].right : Q + 1;
      int64_t sib = b ? Q + 1 : t->nd[Q].right;
      double dax = ry.d[ax];
      if (dax != 0.0 && ((b && dax > 0) || (!b && dax < 0))) {
        double tc = tr(t, tr(t, t->nd[Q].t_split - c->xi[ax]) * ry.inv[ax]);
        int gc = ax;
        if (tc > 1.0) {
          tc = 1.0;
          gc = -1;
        }
        if (tc > tQ) {
          chain_piece(c, &ry, Q, sib, tQ, gQ, tc, gc);
          tQ = tc;
          gQ = gc;
        }
      }
      Q = child;
    }
    refine(c, &ry, C, tQ, gQ, 1.0, -1);
  }
done:;
  /* a merged cell of background sources radiates from its point on the
   * sphere (Sec. 2.2.4); tau still runs to x_L, inside the cell */
  double r2f = ry.r2;
  if (c->bg && src < 0 && t->bg_cell[C]) {
    double e[3];
    for (int a = 0; a < 3; ++a) e[a] = t->bg_pos[3 * C + a] - c->xi[a];
    r2f = (e[0] * e[0] + e[1] * e[1]) + e[2] * e[2];
  }
  /* early termination: a ray past tau_max contributes nothing */
  double f = ry.tau > c->tau_max ? 0.0 : (L * exp(-ry.tau)) / ((4.0 * M_PI) * r2f);
  c->F += f;
  c->G += f * ry.tau;
  if (c->bands)
    for (int b = 0; b < t->nbands; ++b)
      c->Fb[b] += (L * exp(-ry.tau_b[b])) / ((4.0 * M_PI) * ry.r2);
  /* the ray's direction of travel at the sink, (x_i - y) / r */
  double nv[3];
  for (int a = 0; a < 3; ++a) {
    nv[a] = -ry.d[a] / ry.r;
    c->Fv[a] += f * nv[a];
  }
  c->Pm[0] += f * (nv[0] * nv[0]);
  c->Pm[1] += f * (nv[1] * nv[1]);
  c->Pm[2] += f * (nv[2] * nv[2]);
  c->Pm[3] += f * (nv[0] * nv[1]);
  c->Pm[4] += f * (nv[0] * nv[2]);
  c->Pm[5] += f * (nv[1] * nv[2]);
  if (c->log_C && c->log_n < c->log_cap) {
    int64_t k = c->log_n;
    c->log_C[k] = C;
    c->log_src[k] = src;
    for (int a = 0; a < 3; ++a) c->log_y[3 * k + a] = y[a];
    c->log_L[k] = L;
    c->log_tau[k] = ry.tau;
    c->log_f[k] = f;
  }
  if (c->piece_node && c->log_n == c->piece_ray) {
    for (int k = 0; k < ry.nseg && k < c->piece_cap; ++k) {
      c->piece_node[k] = ry.seg[k].node;
      c->piece_t[4 * k + 0] = ry.seg[k].ta;
      c->piece_t[4 * k + 1] = ry.seg[k].tb;
      c->piece_t[4 * k + 2] = ry.seg[k].alpha;
      c->piece_t[4 * k + 3] = ry.seg[k].len;
    }
    c->piece_n = ry.nseg;
  }
  c->log_n++;
  if (c->abar) {
    /* adjoint of this ray with decisions held fixed */
    double g = c->w * f;
    for (int k = 0; k < ry.nseg; ++k) c->abar[ry.seg[k].node] -= g * ry.seg[k].len;
    if (src >= 0) {
      c->direct[src] += g / L;
    } else {
      /* d tau / d y: the length scales with r, each plane crossing
       * t = (s - x_a)/d_a moves with d tau_b / d y_a = -t / d_a */
      double dtdy[3];
      for (int a = 0; a < 3; ++a) dtdy[a] = (ry.tau / ry.r) * (ry.d[a] / ry.r);
      for (int k = 0; k < ry.nseg; ++k) {
        const oseg *s = &ry.seg[k];
        if (s->tagb >= 0)
          dtdy[s->tagb] += ry.r * s->alpha * (-s->tb * ry.inv[s->tagb]);
        if (s->taga >= 0)
          dtdy[s->taga] -= ry.r * s->alpha * (-s->ta * ry.inv[s->taga]);
      }
      c->lbar[C] += g / L;
      for (int a = 0; a < 3; ++a)
        c->xbar[3 * C + a] += g * (-2.0 * ry.d[a] / ry.r2 - dtdy[a]);
    }
  }
  free(ry.seg);
}

/* Source walk (Sec. 2.2.1): depth-first from the root, left before right;
 * cells without luminosity are skipped; a cell is merged at its centre of
 * luminosity when theta_open > l / r, l = distance from the centre of
 * luminosity to the furthest vertex, r = distance from the sink to the
 * closest point of the cell (strict, compared squared). */
static void walk(osink *c, int64_t id) {
  const otree *t = c->t;
  const onode *p = &t->nd[id];
  if (p->t_lc == 0.0) return;
  c->n_open++;
  double dd[3];
  for (int a = 0; a < 3; ++a) {
    double u = p->t_lo[a] - c->xi[a];
    double v = c->xi[a] - p->t_hi[a];
    double g = u > v ? u : v;
    dd[a] = g > 0.0 ? g : 0.0;
  }
  double r2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2];
  int accept = p->t_lfar * p->t_lfar < c->theta2 * r2;
  if (c->open_mode == 1) {
    /* per bucket: r from the sink's bucket box to the cell's box, so that
     * every sink of a bucket takes the same decision */
    const onode *b = &t->nd[c->S];
    double g2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      double u = p->t_lo[a] - b->t_hi[a];
      double v = b->t_lo[a] - p->t_hi[a];
      double g = u > v ? u : v;
      if (g > 0.0) g2 += g * g;
    }
    accept = p->t_lfar * p->t_lfar < c->theta2 * g2;
  } else if (c->open_mode == 2) {
    /* Gasoline (Sec. 2.3): opened inside r_open = 2 B_max / (sqrt(3) theta)
     * about the centre (here x_L; B_max the distance to the furthest vertex,
     * l_far), i.e. accepted where 3 theta^2 d^2 > 4 l_far^2; a cell holding
     * the sink is always opened */
    double e[3];
    for (int a = 0; a < 3; ++a) e[a] = c->xi[a] - p->t_xl[a];
    double d2 = (e[0] * e[0] + e[1] * e[1]) + e[2] * e[2];
    accept = r2 > 0.0 && 3.0 * c->theta2 * d2 > 4.0 * (p->t_lfar * p->t_lfar);
  }
  if (accept) {
    c->n_rays++;
    trace_ray(c, id, p->t_xl, p->t_lc, -1);
    return;
  }
  if (p->leaf) {
    for (int64_t k = p->first; k < p->first + p->count; ++k) {
      int64_t j = t->perm[k];
      const double *xj = &t->x[3 * j];
      if (!(t->lum[j] > 0) || j == c->i) continue;
      if (xj[0] == c->xi[0] && xj[1] == c->xi[1] && xj[2] == c->xi[2]) continue;
      c->n_rays++;
      c->n_psrc++;
      trace_ray(c, id, xj, t->lum[j], j);
    }
    return;
  }
  walk(c, id + 1);
  walk(c, p->right);
}

static void sink_init(osink *c, const otree *t, int64_t i, double theta,
                      double tau_ref) {
  memset(c, 0, sizeof *c);
  c->t = t;
  c->i = i;
  c->S = t->leaf_of[i];
  for (int a = 0; a < 3; ++a) c->xi[a] = t->x[3 * i + a];
  c->theta2 = theta * theta;
  c->tau_ref = tau_ref;
  c->tau_max = INFINITY;
}

/* Flux (angle-summed intensity, eq. simpint summed over sources) at each
 * sink.  sinks == NULL means every particle, in index order.  counters, if
 * given, receive 5 per sink: n_open, n_rays, n_psrc, n_seg, n_trace.  G, if
 * given, receives sum over rays of f * tau. */
int oracle_flux(void *h, double theta, double tau_ref, const int64_t *sinks,
                int64_t ns, int nthreads, double *F, int64_t *counters,
                double *G) {
  const otree *t = (const otree *)h;
  if (!(theta >= 0)) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t q = 0; q < ns; ++q) {
    int64_t i = sinks ? sinks[q] : q;
    osink c;
    sink_init(&c, t, i, theta, tau_ref);
    walk(&c, 0);
    F[q] = c.F;
    if (G) G[q] = c.G;
    if (counters) {
      counters[5 * q + 0] = c.n_open;
      counters[5 * q + 1] = c.n_rays;
      counters[5 * q + 2] = c.n_psrc;
      counters[5 * q + 3] = c.n_seg;
      counters[5 * q + 4] = c.n_trace;
    }
  }
  return 0;
}

/* Net radiation flux, eq. (simpflux): each ray's L exp(-tau)/(4 pi r^2) along
 * the unit vector from the source point to the sink, summed over the sink's
 * rays in walk order.  Fv receives 3 per sink (x, y, z).
 * F receives the scalar flux as in oracle_flux. */
int oracle_flux_vec(void *h, double theta, double tau_ref, const int64_t *sinks,
                    int64_t ns, int nthreads, double *F, double *Fv) {
  const otree *t = (const otree *)h;
  if (!(theta >= 0)) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t q = 0; q < ns; ++q) {
    int64_t i = sinks ? sinks[q] : q;
    osink c;
    sink_init(&c, t, i, theta, tau_ref);
    walk(&c, 0);
    F[q] = c.F;
    for (int a = 0; a < 3; ++a) Fv[3 * q + a] = c.Fv[a];
  }
  return 0;
}

/* Second moment of the intensity (the radiation pressure tensor times c; the
 * paper notes that such moments follow by simple sums, Sec. 2.1): for each
 * sink the sum over its rays, in walk order, of f n_a n_b with n the unit
 * vector from the source point to the sink.  Pm receives 6 per sink (xx, yy,
 * zz, xy, xz, yz); F and Fv as in oracle_flux_vec. */
int oracle_flux_moments(void *h, double theta, double tau_ref, const int64_t *sinks,
                        int64_t ns, int nthreads, double *F, double *Fv, double *Pm) {
  const otree *t = (const otree *)h;
  if (!(theta >= 0)) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t q = 0; q < ns; ++q) {
    int64_t i = sinks ? sinks[q] : q;
    osink c;
    sink_init(&c, t, i, theta, tau_ref);
    walk(&c, 0);
    F[q] = c.F;
    for (int a = 0; a < 3; ++a) Fv[3 * q + a] = c.Fv[a];
    for (int a = 0; a < 6; ++a) Pm[6 * q + a] = c.Pm[a];
  }
  return 0;
}

/* Flux per band (oracle_set_bands first): Fb receives nbands per sink; the
 * counters are those of the band traversal. */
int oracle_flux_bands(void *h, double theta, double tau_ref, const int64_t *sinks,
                      int64_t ns, int nthreads, double *Fb, int64_t *counters) {
  const otree *t = (const otree *)h;
  if (!(theta >= 0) || t->nbands < 1) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t q = 0; q < ns; ++q) {
    int64_t i = sinks ? sinks[q] : q;
    osink c;
    sink_init(&c, t, i, theta, tau_ref);
    c.bands = 1;
    walk(&c, 0);
    for (int b = 0; b < t->nbands; ++b) Fb[(size_t)t->nbands * (size_t)q + b] = c.Fb[b];
    if (counters) {
      counters[5 * q + 0] = c.n_open;
      counters[5 * q + 1] = c.n_rays;
      counters[5 * q + 2] = c.n_psrc;
      counters[5 * q + 3] = c.n_seg;
      counters[5 * q + 4] = c.n_trace;
    }
  }
  return 0;
}

/* Flux with the sub-bucket particle trace (oracle_set_sph first): as
 * oracle_flux, but a ray piece in a bucket whose particle spread fails the
 * refinement test, spread * l > tau_ref, takes the particle trace. */
int oracle_flux_sph(void *h, double theta, double tau_ref, const int64_t *sinks, int64_t ns,
                    int nthreads, double *F, int64_t *counters) {
  const otree *t = (const otree *)h;
  if (!(theta >= 0) || !t->sph) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t q = 0; q < ns; ++q) {
    int64_t i = sinks ? sinks[q] : q;
    osink c;
    sink_init(&c, t, i, theta, tau_ref);
    c.sph = 1;
    walk(&c, 0);
    F[q] = c.F;
    if (counters) {
      counters[5 * q + 0] = c.n_open;
      counters[5 * q + 1] = c.n_rays;
      counters[5 * q + 2] = c.n_psrc;
      counters[5 * q + 3] = c.n_seg;
      counters[5 * q + 4] = c.n_trace;
    }
  }
  return 0;
}

/* oracle_ray_log with the sub-bucket particle trace. */
int64_t oracle_ray_log_sph(void *h, double theta, double tau_ref, int64_t sink, int64_t cap,
                           int64_t *C, int64_t *src, double *y, double *L, double *tau,
                           double *f) {
  const otree *t = (const otree *)h;
  if (!t->sph) return -1;
  osink c;
  sink_init(&c, t, sink, theta, tau_ref);
  c.sph = 1;
  c.log_cap = cap;
  c.log_C = C;
  c.log_src = src;
  c.log_y = y;
  c.log_L = L;
  c.log_tau = tau;
  c.log_f = f;
  walk(&c, 0);
  return c.log_n;
}

/* Flux with the walk variants (open_mode 0, 1, 2; ray_mode 0, 1; tau_max,
 * +infinity for none), otherwise as oracle_flux. */
int oracle_flux_variant(void *h, double theta, double tau_ref, int open_mode, int ray_mode,
                        double tau_max, const int64_t *sinks, int64_t ns, int nthreads,
                        double *F, int64_t *counters) {
  const otree *t = (const otree *)h;
  if (!(theta >= 0) || open_mode < 0 || open_mode > 2 || ray_mode < 0 || ray_mode > 1 ||
      !(tau_max > 0))
    return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t q = 0; q < ns; ++q) {
    int64_t i = sinks ? sinks[q] : q;
    osink c;
    sink_init(&c, t, i, theta, tau_ref);
    c.open_mode = open_mode;
    c.ray_mode = ray_mode;
    c.tau_max = tau_max;
    walk(&c, 0);
    F[q] = c.F;
    if (counters) {
      counters[5 * q + 0] = c.n_open;
      counters[5 * q + 1] = c.n_rays;
      counters[5 * q + 2] = c.n_psrc;
      counters[5 * q + 3] = c.n_seg;
      counters[5 * q + 4] = c.n_trace;
    }
  }
  return 0;
}

/* oracle_ray_log with the walk variants. */
int64_t oracle_ray_log_variant(void *h, double theta, double tau_ref, int open_mode,
                               int ray_mode, int64_t sink, int64_t cap, int64_t *C,
                               int64_t *src, double *y, double *L, double *tau, double *f) {
  const otree *t = (const otree *)h;
  osink c;
  sink_init(&c, t, sink, theta, tau_ref);
  c.open_mode = open_mode;
  c.ray_mode = ray_mode;
  c.log_cap = cap;
  c.log_C = C;
  c.log_src = src;
  c.log_y = y;
  c.log_L = L;
  c.log_tau = tau;
  c.log_f = f;
  walk(&c, 0);
  return c.log_n;
}

/* Background shell (Sec. 2.2.4): flags[n] marks the background sources
 * (input order), which lie on the sphere of the given centre and radius.  A
 * cell whose luminous particles are all background sources has its merged
 * source moved radially onto the sphere, y' = c + R (x_L - c) / |x_L - c|
 * (the paper's remedy for merged centres of luminosity that fall inside the
 * sphere); a ray from it keeps its optical depth to x_L and takes
 * L e^-tau / (4 pi |y' - x_i|^2). */
int oracle_set_background(void *h, const double *centre, double radius,
                          const unsigned char *flags) {
  otree *t = (otree *)h;
  if (!(radius > 0) || !isfinite(radius)) return -1;
  free(t->bg_cell);
  free(t->bg_pos);
  t->bg_cell = (unsigned char *)calloc((size_t)(t->m > 0 ? t->m : 1), 1);
  t->bg_pos = (double *)calloc(3 * (size_t)(t->m > 0 ? t->m : 1), sizeof(double));
  for (int64_t id = 0; id < t->m; ++id) {
    const onode *p = &t->nd[id];
    if (!(p->t_lc > 0)) continue;
    int only = 1;
    for (int64_t k = p->first; k < p->first + p->count; ++k) {
      int64_t j = t->perm[k];
      if (t->lum[j] > 0 && !flags[j]) only = 0;
    }
    if (!only) continue;
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = p->t_xl[a] - centre[a];
    double len = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    t->bg_cell[id] = 1;
    for (int a = 0; a < 3; ++a)
      t->bg_pos[3 * id + a] = tr(t, len > 0 ? centre[a] + radius * (v[a] / len) : p->t_xl[a]);
  }
  t->bg = 1;
  return 0;
}

/* Flux with the background shell's merged sources on the sphere. */
int oracle_flux_background(void *h, double theta, double tau_ref, const int64_t *sinks,
                           int64_t ns, int nthreads, double *F, int64_t *counters) {
  const otree *t = (const otree *)h;
  if (!(theta >= 0) || !t->bg) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t q = 0; q < ns; ++q) {
    int64_t i = sinks ? sinks[q] : q;
    osink c;
    sink_init(&c, t, i, theta, tau_ref);
    c.bg = 1;
    walk(&c, 0);
    F[q] = c.F;
    if (counters) {
      counters[5 * q + 0] = c.n_open;
      counters[5 * q + 1] = c.n_rays;
      counters[5 * q + 2] = c.n_psrc;
      counters[5 * q + 3] = c.n_seg;
      counters[5 * q + 4] = c.n_trace;
    }
  }
  return 0;
}

/* The cells moved onto the sphere (flag) and their points, [m][3]. */
int oracle_background_cells(void *h, unsigned char *flag, double *pos) {
  const otree *t = (const otree *)h;
  if (!t->bg) return -1;
  for (int64_t id = 0; id < t->m; ++id) {
    flag[id] = t->bg_cell[id];
    for (int a = 0; a < 3; ++a) pos[3 * id + a] = t->bg_pos[3 * id + a];
  }
  return 0;
}

/* Every ray of one sink, in walk order.  Returns the number of rays (the
 * arrays hold the first cap of them).  src = -1 for a merged cell. */
int64_t oracle_ray_log(void *h, double theta, double tau_ref, int64_t sink,
                       int64_t cap, int64_t *C, int64_t *src, double *y,
                       double *L, double *tau, double *f) {
  const otree *t = (const otree *)h;
  osink c;
  sink_init(&c, t, sink, theta, tau_ref);
  c.log_cap = cap;
  c.log_C = C;
  c.log_src = src;
  c.log_y = y;
  c.log_L = L;
  c.log_tau = tau;
  c.log_f = f;
  walk(&c, 0);
  return c.log_n;
}

/* The pieces (cell, ta, tb, alpha, length) of ray number ray_index of one
 * sink's walk, in the order they were added.  Returns the piece count. */
int64_t oracle_ray_pieces(void *h, double theta, double tau_ref, int64_t sink,
                          int64_t ray_index, int64_t cap, int64_t *node,
                          double *tparams) {
  const otree *t = (const otree *)h;
  osink c;
  sink_init(&c, t, sink, theta, tau_ref);
  c.piece_ray = ray_index;
  c.piece_cap = cap;
  c.piece_node = node;
  c.piece_t = tparams;
  walk(&c, 0);
  return c.piece_n;
}

/* Gradient of sum_i gradF_i F_i with respect to every particle's rho, kappa
 * and L, with the traversal (every accept / open / refine decision and every
 * piece's cell) held fixed.  alpha = A/B gives
 *   d alpha / d kappa_p = m_p / B,  d alpha / d rho_p = alpha m_p / (B rho_p^2)
 * for every cell holding p; a cell without absorbing mass took its parent's
 * alpha, so its adjoint goes to the parent.  A merged source has
 * L_C = sum L_j and x_L = sum L_j x_j / L_C, so
 *   dL_C/dL_j = 1,  dx_L/dL_j = (x_j - x_L) / L_C. */
int oracle_adjoint(void *h, double theta, double tau_ref, const int64_t *sinks,
                   int64_t ns, const double *gradF, int nthreads,
                   double *grad_rho, double *grad_kappa, double *grad_lum) {
  const otree *t = (const otree *)h;
  int64_t m = t->m, n = t->n;
  int nt = 1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  nt = omp_get_max_threads();
#endif
  size_t per = (size_t)(5 * m + n);
  double *acc = (double *)calloc((size_t)nt * per, sizeof(double));
#ifdef _OPENMP
#pragma omp parallel
#endif
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double *mine = acc + (size_t)tid * per;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int64_t q = 0; q < ns; ++q) {
      int64_t i = sinks ? sinks[q] : q;
      osink c;
      sink_init(&c, t, i, theta, tau_ref);
      c.w = gradF[q];
      c.abar = mine;
      c.lbar = mine + m;
      c.xbar = mine + 2 * m;
      c.direct = mine + 5 * m;
      walk(&c, 0);
    }
  }
  double *abar = acc, *lbar = acc + m, *xbar = acc + 2 * m, *direct = acc + 5 * m;
  for (int k = 1; k < nt; ++k) {
    const double *o = acc + (size_t)k * per;
    for (size_t e = 0; e < per; ++e) acc[e] += o[e];
  }
  for (int64_t id = m - 1; id > 0; --id)
    if (!(t->nd[id].B > 0)) abar[t->nd[id].parent] += abar[id];
  for (int64_t p = 0; p < n; ++p) {
    double gk = 0.0, gr = 0.0, gl = direct[p];
    for (int64_t id = t->leaf_of[p]; id >= 0; id = t->nd[id].parent) {
      const onode *c = &t->nd[id];
      if (c->B > 0 && t->mass[p] > 0) {
        gk += abar[id] * t->mass[p] / c->B;
        gr += abar[id] * c->alpha * t->mass[p] / (c->B * t->rho[p] * t->rho[p]);
      }
      if (c->lc > 0) {
        double dot = 0.0;
        for (int a = 0; a < 3; ++a)
          dot += xbar[3 * id + a] * (t->x[3 * p + a] - c->xl[a]);
        gl += lbar[id] + dot / c->lc;
      }
    }
    grad_rho[p] = gr;
    grad_kappa[p] = gk;
    grad_lum[p] = gl;
  }
  free(acc);
  return 0;
}
