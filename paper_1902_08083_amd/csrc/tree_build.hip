// Radiation-tree build on gfx950 (Sec. 2.2 and 2.3 of the TREVR paper).
//
//  1. k_keys: per particle, validate the inputs and compute its 63-level path
//     through midpoint bisections of the level axes (binary64 compares).
//  2. Stable radix sort of (path, index) -- and, for several boxes, a second
//     stable sort by box -- gives the particle order (box, path, index).
//  3. Level by level: every cell with more than N_B particles (depth < 63)
//     splits at the first particle whose path bit at this depth is set, and
//     both halves are kept (space-filling tree).
//  4. Subtree sizes bottom-up, depth-first indices top-down, then every cell
//     writes its record at its depth-first index.
//  5. Cell properties in binary64 with a fixed summation order: bucket sums in
//     particle order, parent = lower + upper child; alpha top-down; the
//     directional alpha bounds bottom-up; centre of luminosity and
//     far-vertex distance; finally the transport records.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>
#include <cmath>

#include "trevr_internal.h"

namespace trevr {

enum : int { ERR_RANGE = 1, ERR_NONFINITE = 2, ERR_VALUE = 4, ERR_MOVED = 8 };

template <typename T>
struct PartIn {
  const T *x, *y, *z, *mass, *rho, *kappa, *lum;
};

__device__ inline int box_of(const int64_t *off, int nbox, int64_t i) {
  int lo = 0, hi = nbox;  // off[lo] <= i < off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= i)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <typename T>
__global__ void k_keys(PartIn<T> in, int64_t n, const int64_t *box_off, int nbox,
                       const double *box_lo, const double *box_hi, const int8_t *axis_tab,
                       uint64_t *keys, int32_t *vals, uint32_t *bkey, int *err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int b = box_of(box_off, nbox, i);
  double p[3] = {(double)in.x[i], (double)in.y[i], (double)in.z[i]};
  double m = in.mass ? (double)in.mass[i] : 1.0;
  double rho = (double)in.rho[i], kap = (double)in.kappa[i], L = (double)in.lum[i];
  int e = 0;
  if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2]) || !isfinite(m) ||
      !isfinite(kap) || !isfinite(L) || (m > 0 && !isfinite(rho)))
    e |= ERR_NONFINITE;
  else if (m < 0 || kap < 0 || L < 0 || (m > 0 && !(rho > 0)))
    e |= ERR_VALUE;
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = box_lo[3 * b + a];
    hi[a] = box_hi[3 * b + a];
    if (!(p[a] >= lo[a] && p[a] < hi[a])) e |= ERR_RANGE;
  }
  if (e) atomicOr(err, e);
  uint64_t k = 0;
  const int8_t *ax = axis_tab + 64 * b;
  for (int d = 0; d < kDmax; ++d) {
    int a = ax[d];
    double s = 0.5 * (lo[a] + hi[a]);
    double pa = a == 0 ? p[0] : (a == 1 ? p[1] : p[2]);
    if (pa >= s) {
      k |= 1ull << (62 - d);
      if (a == 0) lo[0] = s; else if (a == 1) lo[1] = s; else lo[2] = s;
    } else {
      if (a == 0) hi[0] = s; else if (a == 1) hi[1] = s; else hi[2] = s;
    }
  }
  keys[i] = k;
  vals[i] = (int32_t)i;
  if (bkey) bkey[i] = (uint32_t)b;
}

__global__ void k_gather_box(const int32_t *perm, const int64_t *box_off, int nbox, int64_t n,
                             uint32_t *bkey) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) bkey[k] = (uint32_t)box_of(box_off, nbox, perm[k]);
}

__global__ void k_gather_keys(const int32_t *perm, const uint64_t *keys, int64_t n,
                              uint64_t *skeys) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) skeys[k] = keys[perm[k]];
}

__global__ void k_roots(BfsNode *lvl, int nbox, const int64_t *box_off, const double *box_lo,
                        const double *box_hi) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbox) return;
  BfsNode r;
  r.first = (int32_t)box_off[b];
  r.count = (int32_t)(box_off[b + 1] - box_off[b]);
  r.box = b;
  r.parent = -1;
  r.child = -1;
  r.size = 1;
  r.pre = 0;
  r.pad = 0;
  r.prefix = 0;
  for (int a = 0; a < 3; ++a) {
    r.lo[a] = box_lo[3 * b + a];
    r.hi[a] = box_hi[3 * b + a];
  }
  lvl[b] = r;
}

__global__ void k_split_flags(const BfsNode *lvl, int cnt, int nb, int depth, int32_t *flag) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < cnt) flag[j] = (lvl[j].count > nb && depth < kDmax) ? 1 : 0;
}

__global__ void k_split_emit(BfsNode *lvl, int cnt, BfsNode *next, const int32_t *flag,
                             const int32_t *scan, const uint64_t *skeys, int depth,
                             const int8_t *axis_tab) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  BfsNode nd = lvl[j];
  if (!flag[j]) {
    lvl[j].child = -1;
    return;
  }
  int c = 2 * scan[j];
  lvl[j].child = c;
  int a = axis_tab[64 * nd.box + depth];
  double s = 0.5 * (nd.lo[a] + nd.hi[a]);
  // first particle of the range whose path bit at this depth is set
  const uint64_t bit = 1ull << (62 - depth);
  int lo = nd.first, hi = nd.first + nd.count;
  while (lo < hi) {
    int mid = lo + ((hi - lo) >> 1);
    if (skeys[mid] & bit)
      hi = mid;
    else
      lo = mid + 1;
  }
  BfsNode l = nd, r = nd;
  l.count = lo - nd.first;
  r.first = lo;
  r.count = nd.first + nd.count - lo;
  l.parent = r.parent = j;
  l.child = r.child = -1;
  l.size = r.size = 1;
  r.prefix = nd.prefix | bit;
  l.hi[a] = s;
  r.lo[a] = s;
  next[c] = l;
  next[c + 1] = r;
}

__global__ void k_total(const int32_t *flag, const int32_t *scan, int cnt, int32_t *out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = scan[cnt - 1] + flag[cnt - 1];
}

__global__ void k_sizes(BfsNode *lvl, int cnt, const BfsNode *next) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  int c = lvl[j].child;
  lvl[j].size = c < 0 ? 1 : 1 + next[c].size + next[c + 1].size;
}

__global__ void k_root_pre(BfsNode *lvl, int nbox, int32_t *box_root) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t acc = 0;
  for (int b = 0; b < nbox; ++b) {
    lvl[b].pre = acc;
    box_root[b] = acc;
    acc += lvl[b].size;
  }
}

__global__ void k_child_pre(const BfsNode *lvl, int cnt, BfsNode *next) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  int c = lvl[j].child;
  if (c < 0) return;
  int32_t p = lvl[j].pre;
  next[c].pre = p + 1;
  next[c + 1].pre = p + 1 + next[c].size;
}

struct NodeOut {
  int32_t *first, *count, *depth, *parent, *right, *skip, *box;
  int8_t *axis;
  uint64_t *key;
  double *lo, *hi, *split;  // lo/hi: [3][m]
  int32_t *leaf_sorted;
  int64_t m;
};

__global__ void k_write_nodes(const BfsNode *lvl, int cnt, const BfsNode *prev,
                              const BfsNode *next, int depth, const int8_t *axis_tab,
                              NodeOut o) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  BfsNode nd = lvl[j];
  int32_t p = nd.pre;
  o.first[p] = nd.first;
  o.count[p] = nd.count;
  o.depth[p] = depth;
  o.parent[p] = nd.parent < 0 ? -1 : prev[nd.parent].pre;
  o.right[p] = nd.child < 0 ? -1 : next[nd.child + 1].pre;
  o.skip[p] = p + nd.size;
  o.box[p] = nd.box;
  int a = axis_tab[64 * nd.box + depth];
  o.axis[p] = (int8_t)a;
  o.key[p] = nd.prefix;
  for (int q = 0; q < 3; ++q) {
    o.lo[q * o.m + p] = nd.lo[q];
    o.hi[q * o.m + p] = nd.hi[q];
  }
  o.split[p] = nd.child < 0 ? 0.0 : 0.5 * (nd.lo[a] + nd.hi[a]);
  if (nd.child < 0)
    for (int k = nd.first; k < nd.first + nd.count; ++k) o.leaf_sorted[k] = p;
}

// ---- properties ----------------------------------------------------------

struct Props {
  double *A, *B, *SL, *SLx, *alpha, *amin, *amax, *alpha_min, *alpha_max, *dalpha, *xl, *lc,
      *lfar;
  const int32_t *first, *count, *right, *parent, *depth;
  const int8_t *axis;
  const double *lo, *hi;
  int64_t m;
};

template <typename T>
__global__ void k_bucket_sums(const BfsNode *lvl, int cnt, PartIn<T> in, const int32_t *perm,
                              Props P) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  const BfsNode nd = lvl[j];
  if (nd.child >= 0) return;
  double A = 0, B = 0, SL = 0, Sx = 0, Sy = 0, Sz = 0;
  for (int k = nd.first; k < nd.first + nd.count; ++k) {
    int q = perm[k];
    double m = in.mass ? (double)in.mass[q] : 1.0;
    double L = (double)in.lum[q];
    if (m > 0) {
      A += m * (double)in.kappa[q];
      B += m / (double)in.rho[q];
    }
    SL += L;
    Sx += L * (double)in.x[q];
    Sy += L * (double)in.y[q];
    Sz += L * (double)in.z[q];
  }
  int p = nd.pre;
  P.A[p] = A;
  P.B[p] = B;
  P.SL[p] = SL;
  P.SLx[p] = Sx;
  P.SLx[P.m + p] = Sy;
  P.SLx[2 * P.m + p] = Sz;
}

__global__ void k_internal_sums(const BfsNode *lvl, int cnt, Props P) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  const BfsNode nd = lvl[j];
  if (nd.child < 0) return;
  int p = nd.pre, l = p + 1, r = P.right[p];
  P.A[p] = P.A[l] + P.A[r];
  P.B[p] = P.B[l] + P.B[r];
  P.SL[p] = P.SL[l] + P.SL[r];
  for (int a = 0; a < 3; ++a) P.SLx[a * P.m + p] = P.SLx[a * P.m + l] + P.SLx[a * P.m + r];
}

__global__ void k_alpha(const BfsNode *lvl, int cnt, Props P) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  int p = lvl[j].pre;
  double B = P.B[p];
  int par = P.parent[p];
  P.alpha[p] = B > 0 ? P.A[p] / B : (par < 0 ? 0.0 : P.alpha[par]);
}

__global__ void k_bounds(const BfsNode *lvl, int cnt, Props P) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  int p = lvl[j].pre;
  double mn[3], mx[3];
  if (lvl[j].child < 0) {
    for (int b = 0; b < 3; ++b) mn[b] = mx[b] = P.alpha[p];
  } else {
    int l = p + 1, r = P.right[p], s = P.axis[p];
    for (int b = 0; b < 3; ++b) {
      double ln = P.amin[b * P.m + l], rn = P.amin[b * P.m + r];
      double lx = P.amax[b * P.m + l], rx = P.amax[b * P.m + r];
      if (b == s) {  // both children crossed: tau adds, width doubles
        mn[b] = 0.5 * (ln + rn);
        mx[b] = 0.5 * (lx + rx);
      } else {  // one child or the other
        mn[b] = ln < rn ? ln : rn;
        mx[b] = lx > rx ? lx : rx;
      }
    }
  }
  double lo = mn[0], hi = mx[0];
  for (int b = 0; b < 3; ++b) {
    P.amin[b * P.m + p] = mn[b];
    P.amax[b * P.m + p] = mx[b];
    if (mn[b] < lo) lo = mn[b];
    if (mx[b] > hi) hi = mx[b];
  }
  P.alpha_min[p] = lo;
  P.alpha_max[p] = hi;
  P.dalpha[p] = hi - lo;
}

template <typename T>
__global__ void k_finish(Props P, WalkRecT<T> *W, TraceRecT<T> *TR) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P.m) return;
  const int64_t m = P.m;
  double SL = P.SL[p];
  double xl[3] = {0, 0, 0}, lc = 0, lfar = 0;
  if (SL > 0) {
    lc = SL;
    double far2 = 0;
    double part[3];
    for (int a = 0; a < 3; ++a) {
      xl[a] = P.SLx[a * m + p] / SL;
      double dl = P.lo[a * m + p] - xl[a];
      double dh = P.hi[a * m + p] - xl[a];
      double ql = dl * dl, qh = dh * dh;
      part[a] = ql > qh ? ql : qh;  // furthest vertex: per-axis maxima
    }
    far2 = (part[0] + part[1]) + part[2];
    lfar = sqrt(far2);
  }
  for (int a = 0; a < 3; ++a) P.xl[a * m + p] = xl[a];
  P.lc[p] = lc;
  P.lfar[p] = lfar;
  int32_t r = P.right[p];
  int32_t ra = (r < 0 ? 0 : r) | ((int32_t)P.axis[p] << 30);
  WalkRecT<T> w;
  for (int a = 0; a < 3; ++a) {
    w.lo[a] = (T)P.lo[a * m + p];
    w.hi[a] = (T)P.hi[a * m + p];
    w.xl[a] = (T)xl[a];
  }
  w.L = (T)lc;
  w.lfar = (T)lfar;
  w.skip = 0;  // written by k_skip
  w.right_ax = ra;
  w.first = P.first[p];
  w.count = P.count[p];
  w.depth = P.depth[p];
  W[p] = w;
  TraceRecT<T> t;
  t.split = 0;
  t.alpha = (T)P.alpha[p];
  t.dalpha = (T)P.dalpha[p];
  t.right_ax = ra;
  TR[p] = t;
}

template <typename T>
__global__ void k_finish2(const int32_t *skip, const double *split, int64_t m, WalkRecT<T> *W,
                          TraceRecT<T> *TR) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  W[p].skip = skip[p];
  TR[p].split = (T)split[p];
}

template <typename T>
__global__ void k_particles(PartIn<T> in, const int32_t *perm, int64_t n, P4<T> *ps,
                            int32_t *inv, T *pmass, T *prho, T *pkappa) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int q = perm[k];
  P4<T> v;
  v.x = in.x[q];
  v.y = in.y[q];
  v.z = in.z[q];
  v.L = in.lum[q];
  ps[k] = v;
  inv[q] = (int32_t)k;
  pmass[k] = in.mass ? in.mass[q] : (T)1;
  prho[k] = in.rho[q];
  pkappa[k] = in.kappa[q];
}

__global__ void k_sorted_box(const int32_t *perm, const int64_t *box_off, int nbox, int64_t n,
                             int32_t *pbox) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) pbox[k] = box_of(box_off, nbox, perm[k]);
}

static inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// Cell properties (a2) on the tree's topology: bucket and internal sums,
// alpha, directional bounds, the transport records, and the particles in
// sorted order.  Shared by the build and the refit.
template <typename T>
static int cell_props(trevr_tree *t, const PartIn<T> &in, int64_t n, int64_t m, int nbox,
                      hipStream_t s) {
  const size_t mm = (size_t)m, nn = (size_t)(n > 0 ? n : 1);
  const int nlev = (int)t->level_cnt.size();
  const BfsNode *bfs = t->bfs.as<BfsNode>();
  const int32_t *perm = t->perm.as<int32_t>();
  DevBuf *props[] = {&t->n_A, &t->n_B, &t->n_SL, &t->n_alpha, &t->n_alpha_min, &t->n_alpha_max,
                     &t->n_dalpha, &t->n_lc, &t->n_lfar};
  for (DevBuf *b : props) TREVR_HIP(b->ensure(8 * mm));
  TREVR_HIP(t->n_SLx.ensure(24 * mm));
  TREVR_HIP(t->n_amin.ensure(24 * mm));
  TREVR_HIP(t->n_amax.ensure(24 * mm));
  TREVR_HIP(t->n_xl.ensure(24 * mm));
  Props P{t->n_A.as<double>(),         t->n_B.as<double>(),         t->n_SL.as<double>(),
          t->n_SLx.as<double>(),       t->n_alpha.as<double>(),     t->n_amin.as<double>(),
          t->n_amax.as<double>(),      t->n_alpha_min.as<double>(), t->n_alpha_max.as<double>(),
          t->n_dalpha.as<double>(),    t->n_xl.as<double>(),        t->n_lc.as<double>(),
          t->n_lfar.as<double>(),      t->n_first.as<int32_t>(),    t->n_count.as<int32_t>(),
          t->n_right.as<int32_t>(),    t->n_parent.as<int32_t>(),   t->n_depth.as<int32_t>(),
          t->n_axis.as<int8_t>(),      t->n_lo.as<double>(),        t->n_hi.as<double>(),
          m};
  for (int d = nlev - 1; d >= 0; --d) {
    const BfsNode *lvl = bfs + t->level_off[d];
    int c = (int)t->level_cnt[d];
    k_bucket_sums<T><<<nblk(c), 256, 0, s>>>(lvl, c, in, perm, P);
    k_internal_sums<<<nblk(c), 256, 0, s>>>(lvl, c, P);
  }
  for (int d = 0; d < nlev; ++d)
    k_alpha<<<nblk(t->level_cnt[d]), 256, 0, s>>>(bfs + t->level_off[d], (int)t->level_cnt[d],
                                                   P);
  for (int d = nlev - 1; d >= 0; --d)
    k_bounds<<<nblk(t->level_cnt[d]), 256, 0, s>>>(bfs + t->level_off[d], (int)t->level_cnt[d],
                                                    P);
  TREVR_HIP(t->walk.ensure(sizeof(WalkRecT<T>) * mm));
  TREVR_HIP(t->trace.ensure(sizeof(TraceRecT<T>) * mm));
  k_finish<T><<<nblk(m), 256, 0, s>>>(P, t->walk.as<WalkRecT<T>>(), t->trace.as<TraceRecT<T>>());
  k_finish2<T><<<nblk(m), 256, 0, s>>>(t->n_skip.as<int32_t>(), t->n_split.as<double>(), m,
                                       t->walk.as<WalkRecT<T>>(), t->trace.as<TraceRecT<T>>());

  TREVR_HIP(t->psrc.ensure(sizeof(P4<T>) * nn));
  TREVR_HIP(t->inv.ensure(4 * nn));
  TREVR_HIP(t->pbox.ensure(4 * nn));
  TREVR_HIP(t->pmass.ensure(sizeof(T) * nn));
  TREVR_HIP(t->prho.ensure(sizeof(T) * nn));
  TREVR_HIP(t->pkappa.ensure(sizeof(T) * nn));
  if (n > 0) {
    k_particles<T><<<nblk(n), 256, 0, s>>>(in, perm, n, t->psrc.as<P4<T>>(), t->inv.as<int32_t>(),
                                           t->pmass.as<T>(), t->prho.as<T>(),
                                           t->pkappa.as<T>());
    k_sorted_box<<<nblk(n), 256, 0, s>>>(perm, t->box_off.as<int64_t>(), nbox, n,
                                         t->pbox.as<int32_t>());
  }
  TREVR_HIP(hipGetLastError());
  return TREVR_OK;
}

template <typename T>
static int build_typed(trevr_tree *t, const trevr_particles *p, hipStream_t s) {
  const int64_t n = p->n;
  const int nbox = p->n_boxes;
  PartIn<T> in{(const T *)p->x, (const T *)p->y, (const T *)p->z, (const T *)p->mass,
               (const T *)p->rho, (const T *)p->kappa, (const T *)p->lum};

  // per-box tables (host): offsets, corners, level axes (longest current width,
  // ties to the lowest axis; all cells of one depth share one shape)
  std::vector<int64_t> off(nbox + 1);
  if (p->box_offsets) {
    for (int b = 0; b <= nbox; ++b) off[b] = p->box_offsets[b];
  } else {
    off[0] = 0;
    off[1] = n;
  }
  std::vector<int8_t> axes(64 * nbox);
  for (int b = 0; b < nbox; ++b) {
    double w[3];
    for (int a = 0; a < 3; ++a) w[a] = p->box_hi[3 * b + a] - p->box_lo[3 * b + a];
    for (int d = 0; d < 64; ++d) {
      int a = 0;
      if (w[1] > w[a]) a = 1;
      if (w[2] > w[a]) a = 2;
      axes[64 * b + d] = (int8_t)a;
      w[a] *= 0.5;
    }
  }
  std::vector<uint64_t> axm(3 * nbox, 0);
  for (int b = 0; b < nbox; ++b)
    for (int d = 0; d < kDmax; ++d) axm[3 * b + axes[64 * b + d]] |= 1ull << (62 - d);
  TREVR_HIP(t->axmask.ensure(sizeof(uint64_t) * 3 * nbox));
  TREVR_HIP(hipMemcpyAsync(t->axmask.p, axm.data(), sizeof(uint64_t) * 3 * nbox,
                           hipMemcpyHostToDevice, s));
  TREVR_HIP(t->box_off.ensure(sizeof(int64_t) * (nbox + 1)));
  TREVR_HIP(t->box_lo.ensure(sizeof(double) * 3 * nbox));
  TREVR_HIP(t->box_hi.ensure(sizeof(double) * 3 * nbox));
  TREVR_HIP(t->axis_tab.ensure(64 * nbox));
  TREVR_HIP(t->box_root.ensure(sizeof(int32_t) * nbox));
  TREVR_HIP(hipMemcpyAsync(t->box_off.p, off.data(), sizeof(int64_t) * (nbox + 1),
                           hipMemcpyHostToDevice, s));
  TREVR_HIP(hipMemcpyAsync(t->box_lo.p, p->box_lo, sizeof(double) * 3 * nbox,
                           hipMemcpyHostToDevice, s));
  TREVR_HIP(hipMemcpyAsync(t->box_hi.p, p->box_hi, sizeof(double) * 3 * nbox,
                           hipMemcpyHostToDevice, s));
  TREVR_HIP(hipMemcpyAsync(t->axis_tab.p, axes.data(), 64 * nbox, hipMemcpyHostToDevice, s));
  t->h_box_off = off;
  t->h_box_lo.assign(p->box_lo, p->box_lo + 3 * nbox);
  t->h_box_hi.assign(p->box_hi, p->box_hi + 3 * nbox);

  const size_t nn = (size_t)(n > 0 ? n : 1);
  TREVR_HIP(t->keys_in.ensure(8 * nn));
  TREVR_HIP(t->keys_out.ensure(8 * nn));
  TREVR_HIP(t->vals_in.ensure(4 * nn));
  TREVR_HIP(t->vals_out.ensure(4 * nn));
  TREVR_HIP(t->box_key.ensure(8 * nn));  // two u32 arrays
  TREVR_HIP(t->skeys.ensure(8 * nn));
  TREVR_HIP(t->err.ensure(64));
  TREVR_HIP(t->small.ensure(64));
  TREVR_HIP(hipMemsetAsync(t->err.p, 0, 4, s));

  uint64_t *keys = t->keys_in.as<uint64_t>();
  int32_t *vals = t->vals_in.as<int32_t>();
  uint32_t *bk0 = t->box_key.as<uint32_t>();
  uint32_t *bk1 = bk0 + nn;
  if (n > 0)
    k_keys<T><<<nblk(n), 256, 0, s>>>(in, n, t->box_off.as<int64_t>(), nbox,
                                      t->box_lo.as<double>(), t->box_hi.as<double>(),
                                      t->axis_tab.as<int8_t>(), keys, vals, nullptr,
                                      t->err.as<int>());
  TREVR_HIP(hipGetLastError());

  // stable sorts: by path (63 bits), then by box
  int32_t *perm = vals;
  if (n > 1) {
    size_t tmp = 0;
    TREVR_HIP(rocprim::radix_sort_pairs(nullptr, tmp, keys, t->keys_out.as<uint64_t>(), vals,
                                        t->vals_out.as<int32_t>(), (size_t)n, 0, 63, s));
    size_t tmp2 = 0;
    if (nbox > 1)
      TREVR_HIP(rocprim::radix_sort_pairs(nullptr, tmp2, bk0, bk1, t->vals_out.as<int32_t>(),
                                          vals, (size_t)n, 0, 32, s));
    TREVR_HIP(t->sort_tmp.ensure(std::max(tmp, tmp2)));
    tmp = t->sort_tmp.bytes;
    TREVR_HIP(rocprim::radix_sort_pairs(t->sort_tmp.p, tmp, keys, t->keys_out.as<uint64_t>(),
                                        vals, t->vals_out.as<int32_t>(), (size_t)n, 0, 63, s));
    perm = t->vals_out.as<int32_t>();
    if (nbox > 1) {
      int nbits = 1;
      while ((1 << nbits) < nbox) ++nbits;
      k_gather_box<<<nblk(n), 256, 0, s>>>(perm, t->box_off.as<int64_t>(), nbox, n, bk0);
      tmp2 = t->sort_tmp.bytes;
      TREVR_HIP(rocprim::radix_sort_pairs(t->sort_tmp.p, tmp2, bk0, bk1, perm, vals, (size_t)n,
                                          0, nbits, s));
      perm = vals;
    }
  }
  // keep the permutation in its own buffer
  TREVR_HIP(t->perm.ensure(4 * nn));
  if (n > 0)
    TREVR_HIP(hipMemcpyAsync(t->perm.p, perm, 4 * n, hipMemcpyDeviceToDevice, s));
  perm = t->perm.as<int32_t>();
  uint64_t *skeys = t->skeys.as<uint64_t>();
  if (n > 0) k_gather_keys<<<nblk(n), 256, 0, s>>>(perm, keys, n, skeys);

  // ---- level-by-level construction --------------------------------------
  t->level_off.clear();
  t->level_cnt.clear();
  int64_t cap = 2 * (n / (p->bucket_size + 1)) + 2 * nbox + 64;
  TREVR_HIP(t->bfs.ensure(sizeof(BfsNode) * (size_t)cap));
  BfsNode *bfs = t->bfs.as<BfsNode>();
  k_roots<<<nblk(nbox), 256, 0, s>>>(bfs, nbox, t->box_off.as<int64_t>(),
                                     t->box_lo.as<double>(), t->box_hi.as<double>());
  int64_t total = nbox, cnt = nbox;
  int depth = 0;
  int32_t *hsplits = nullptr;
  TREVR_HIP(hipHostMalloc((void **)&hsplits, sizeof(int32_t)));
  struct Guard {
    int32_t *h;
    ~Guard() { (void)hipHostFree(h); }
  } guard{hsplits};
  while (cnt > 0) {
    t->level_off.push_back(total - cnt);
    t->level_cnt.push_back(cnt);
    // room for up to 2 cnt children
    int64_t need = total + 2 * cnt;
    if (need > cap) {
      int64_t ncap = std::max(need, 2 * cap);
      DevBuf nb;
      TREVR_HIP(nb.ensure(sizeof(BfsNode) * (size_t)ncap));
      TREVR_HIP(hipMemcpyAsync(nb.p, t->bfs.p, sizeof(BfsNode) * total,
                               hipMemcpyDeviceToDevice, s));
      TREVR_HIP(hipStreamSynchronize(s));
      t->bfs.release();
      t->bfs = nb;
      nb.p = nullptr;
      nb.bytes = 0;
      cap = ncap;
      bfs = t->bfs.as<BfsNode>();
    }
    BfsNode *lvl = bfs + (total - cnt);
    BfsNode *next = bfs + total;
    TREVR_HIP(t->flags.ensure(4 * (size_t)cnt));
    TREVR_HIP(t->scan.ensure(4 * (size_t)cnt));
    int32_t *flag = t->flags.as<int32_t>(), *scan = t->scan.as<int32_t>();
    k_split_flags<<<nblk(cnt), 256, 0, s>>>(lvl, (int)cnt, p->bucket_size, depth, flag);
    size_t tmp = 0;
    TREVR_HIP(rocprim::exclusive_scan(nullptr, tmp, flag, scan, 0, (size_t)cnt,
                                      rocprim::plus<int32_t>(), s));
    if (tmp > t->sort_tmp.bytes) TREVR_HIP(t->sort_tmp.ensure(tmp));
    tmp = t->sort_tmp.bytes;
    TREVR_HIP(rocprim::exclusive_scan(t->sort_tmp.p, tmp, flag, scan, 0, (size_t)cnt,
                                      rocprim::plus<int32_t>(), s));
    k_total<<<1, 64, 0, s>>>(flag, scan, (int)cnt, t->small.as<int32_t>());
    k_split_emit<<<nblk(cnt), 256, 0, s>>>(lvl, (int)cnt, next, flag, scan, skeys, depth,
                                           t->axis_tab.as<int8_t>());
    TREVR_HIP(hipGetLastError());
    TREVR_HIP(hipMemcpyAsync(hsplits, t->small.p, 4, hipMemcpyDeviceToHost, s));
    TREVR_HIP(hipStreamSynchronize(s));
    if (depth == 0) {  // the inputs were validated by k_keys: report now
      int herr = 0;
      TREVR_HIP(hipMemcpy(&herr, t->err.p, 4, hipMemcpyDeviceToHost));
      if (herr & ERR_NONFINITE) return fail(TREVR_E_NONFINITE, "non-finite input value");
      if (herr & ERR_VALUE)
        return fail(TREVR_E_VALUE, "negative mass/opacity/luminosity or density <= 0");
      if (herr & ERR_RANGE) return fail(TREVR_E_RANGE, "particle outside its box [lo, hi)");
    }
    cnt = 2 * (int64_t)(*hsplits);
    total += cnt;
    if (total >= (1 << 30) - 1) return fail(TREVR_E_CAPACITY, "more than 2^30 - 2 tree cells");
    // the walk addresses trace records with 32-bit byte offsets
    if ((uint64_t)total * sizeof(TraceRecT<T>) > ((uint64_t)1 << 32))
      return fail(TREVR_E_CAPACITY,
                  "trace records beyond 4 GiB (2^28 cells in binary32, 2^27 in binary64)");
    ++depth;
  }
  const int nlev = (int)t->level_cnt.size();
  const int64_t m = total;
  t->max_depth = nlev - 1;

  for (int d = nlev - 1; d >= 0; --d) {
    BfsNode *lvl = bfs + t->level_off[d];
    BfsNode *next = d + 1 < nlev ? bfs + t->level_off[d + 1] : bfs;
    k_sizes<<<nblk(t->level_cnt[d]), 256, 0, s>>>(lvl, (int)t->level_cnt[d], next);
  }
  k_root_pre<<<1, 64, 0, s>>>(bfs, nbox, t->box_root.as<int32_t>());
  for (int d = 0; d + 1 < nlev; ++d)
    k_child_pre<<<nblk(t->level_cnt[d]), 256, 0, s>>>(bfs + t->level_off[d],
                                                       (int)t->level_cnt[d],
                                                       bfs + t->level_off[d + 1]);

  // ---- cell arrays ---------------------------------------------------------
  const size_t mm = (size_t)m;
  TREVR_HIP(t->n_first.ensure(4 * mm));
  TREVR_HIP(t->n_count.ensure(4 * mm));
  TREVR_HIP(t->n_depth.ensure(4 * mm));
  TREVR_HIP(t->n_parent.ensure(4 * mm));
  TREVR_HIP(t->n_right.ensure(4 * mm));
  TREVR_HIP(t->n_skip.ensure(4 * mm));
  TREVR_HIP(t->n_box.ensure(4 * mm));
  TREVR_HIP(t->n_axis.ensure(mm));
  TREVR_HIP(t->key.ensure(8 * mm));
  TREVR_HIP(t->n_lo.ensure(24 * mm));
  TREVR_HIP(t->n_hi.ensure(24 * mm));
  TREVR_HIP(t->n_split.ensure(8 * mm));
  TREVR_HIP(t->leaf.ensure(4 * nn));
  NodeOut o{t->n_first.as<int32_t>(), t->n_count.as<int32_t>(), t->n_depth.as<int32_t>(),
            t->n_parent.as<int32_t>(), t->n_right.as<int32_t>(), t->n_skip.as<int32_t>(),
            t->n_box.as<int32_t>(), t->n_axis.as<int8_t>(), t->key.as<uint64_t>(),
            t->n_lo.as<double>(), t->n_hi.as<double>(), t->n_split.as<double>(),
            t->leaf.as<int32_t>(), m};
  for (int d = 0; d < nlev; ++d) {
    const BfsNode *prev = d > 0 ? bfs + t->level_off[d - 1] : bfs;
    const BfsNode *next = d + 1 < nlev ? bfs + t->level_off[d + 1] : bfs;
    k_write_nodes<<<nblk(t->level_cnt[d]), 256, 0, s>>>(bfs + t->level_off[d],
                                                         (int)t->level_cnt[d], prev, next, d,
                                                         t->axis_tab.as<int8_t>(), o);
  }
  TREVR_HIP(hipGetLastError());

  {
    int rc = cell_props<T>(t, in, n, m, nbox, s);
    if (rc != TREVR_OK) return rc;
  }
  t->h_box_root.resize(nbox);
  TREVR_HIP(hipMemcpyAsync(t->h_box_root.data(), t->box_root.p, 4 * nbox, hipMemcpyDeviceToHost,
                           s));
  TREVR_HIP(hipStreamSynchronize(s));
  t->n = n;
  t->m = m;
  t->n_boxes = nbox;
  t->nb = p->bucket_size;
  t->prec = p->prec;
  t->built = true;
  return TREVR_OK;
}

// ---- opacity bands ----------------------------------------------------------
// Band b's cell alpha and spread come from its opacity field exactly as the
// tree's own do from kappa (the same sums in the same order, B = sum m/rho
// shared); a trace record copy carries the largest band spread, which takes
// the refinement decisions.
template <typename T>
__global__ void k_band_bucket(const BfsNode *lvl, int cnt, const T *pmass, const T *kap,
                              const int32_t *perm, double *A) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  const BfsNode nd = lvl[j];
  if (nd.child >= 0) return;
  double a = 0;
  for (int k = nd.first; k < nd.first + nd.count; ++k) {
    double m = (double)pmass[k];
    if (m > 0) a += m * (double)kap[perm[k]];
  }
  A[nd.pre] = a;
}

__global__ void k_band_internal(const BfsNode *lvl, int cnt, const int32_t *right, double *A) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  const BfsNode nd = lvl[j];
  if (nd.child < 0) return;
  int p = nd.pre;
  A[p] = A[p + 1] + A[right[p]];
}

// band_alpha is [m][4]: a cell's bands side by side (one 16-byte load in
// binary32), unused bands zero.
template <typename T>
__global__ void k_band_pack(const double *alpha, const double *dalpha, int64_t m, int first,
                            int band, T *band_alpha, double *dmax) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  if (first)
    for (int b = 0; b < 4; ++b) band_alpha[4 * p + b] = (T)0;
  band_alpha[4 * p + band] = (T)alpha[p];
  const double d = (double)(T)dalpha[p];
  dmax[p] = first || d > dmax[p] ? d : dmax[p];
}

template <typename T>
__global__ void k_band_records(const TraceRecT<T> *TR, const double *dmax, int64_t m,
                               TraceRecT<T> *out) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  TraceRecT<T> r = TR[p];
  r.dalpha = (T)dmax[p];
  out[p] = r;
}

template <typename T>
__global__ void k_band_check(const T *kap, int64_t count, int *err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double k = (double)kap[i];
  if (!isfinite(k))
    atomicOr(err, ERR_NONFINITE);
  else if (k < 0)
    atomicOr(err, ERR_VALUE);
}

template <typename T>
static int bands_typed(trevr_tree *t, int nb, const T *kb, hipStream_t s) {
  const int64_t n = t->n, m = t->m;
  const size_t mm = (size_t)(m > 0 ? m : 1);
  TREVR_HIP(hipMemsetAsync(t->err.p, 0, 4, s));
  if (n > 0) k_band_check<T><<<nblk(n * nb), 256, 0, s>>>(kb, n * nb, t->err.as<int>());
  TREVR_HIP(hipGetLastError());
  int herr = 0;
  TREVR_HIP(hipMemcpyAsync(&herr, t->err.p, 4, hipMemcpyDeviceToHost, s));
  TREVR_HIP(hipStreamSynchronize(s));
  if (herr & ERR_NONFINITE) return fail(TREVR_E_NONFINITE, "non-finite band opacity");
  if (herr & ERR_VALUE) return fail(TREVR_E_VALUE, "negative band opacity");
  TREVR_HIP(t->band_alpha.ensure(sizeof(T) * mm * 4));
  TREVR_HIP(t->band_dmax.ensure(8 * mm));
  TREVR_HIP(t->band_trace.ensure(sizeof(TraceRecT<T>) * mm));
  DevBuf *scr[] = {&t->bs_A, &t->bs_alpha, &t->bs_amin_d, &t->bs_amax_d, &t->bs_dalpha};
  for (DevBuf *b : scr) TREVR_HIP(b->ensure(8 * mm));
  TREVR_HIP(t->bs_amin.ensure(24 * mm));
  TREVR_HIP(t->bs_amax.ensure(24 * mm));
  // the build's topology and B; band scratch for everything kappa touches
  Props P{t->bs_A.as<double>(),     t->n_B.as<double>(),      nullptr,
          nullptr,                  t->bs_alpha.as<double>(), t->bs_amin.as<double>(),
          t->bs_amax.as<double>(),  t->bs_amin_d.as<double>(), t->bs_amax_d.as<double>(),
          t->bs_dalpha.as<double>(), nullptr,                  nullptr,
          nullptr,                  t->n_first.as<int32_t>(), t->n_count.as<int32_t>(),
          t->n_right.as<int32_t>(), t->n_parent.as<int32_t>(), t->n_depth.as<int32_t>(),
          t->n_axis.as<int8_t>(),   t->n_lo.as<double>(),     t->n_hi.as<double>(),
          m};
  const int nlev = (int)t->level_cnt.size();
  const BfsNode *bfs = t->bfs.as<BfsNode>();
  for (int b = 0; b < nb; ++b) {
    const T *kap = kb + (size_t)b * (size_t)n;
    for (int d = nlev - 1; d >= 0; --d) {
      const BfsNode *lvl = bfs + t->level_off[d];
      int c = (int)t->level_cnt[d];
      k_band_bucket<T><<<nblk(c), 256, 0, s>>>(lvl, c, t->pmass.as<T>(), kap,
                                               t->perm.as<int32_t>(), P.A);
      k_band_internal<<<nblk(c), 256, 0, s>>>(lvl, c, P.right, P.A);
    }
    for (int d = 0; d < nlev; ++d)
      k_alpha<<<nblk(t->level_cnt[d]), 256, 0, s>>>(bfs + t->level_off[d],
                                                     (int)t->level_cnt[d], P);
    for (int d = nlev - 1; d >= 0; --d)
      k_bounds<<<nblk(t->level_cnt[d]), 256, 0, s>>>(bfs + t->level_off[d],
                                                      (int)t->level_cnt[d], P);
    k_band_pack<T><<<nblk(m), 256, 0, s>>>(P.alpha, P.dalpha, m, b == 0, b,
                                           t->band_alpha.as<T>(), t->band_dmax.as<double>());
  }
  k_band_records<T><<<nblk(m), 256, 0, s>>>(t->trace.as<TraceRecT<T>>(),
                                            t->band_dmax.as<double>(), m,
                                            t->band_trace.as<TraceRecT<T>>());
  TREVR_HIP(hipGetLastError());
  TREVR_HIP(hipStreamSynchronize(s));
  t->n_bands = nb;
  return TREVR_OK;
}

int bands_impl(trevr_tree *t, int nb, const void *kb, hipStream_t s) {
  t->n_bands = 0;
  if (t->prec == TREVR_F64) return bands_typed<double>(t, nb, (const double *)kb, s);
  return bands_typed<float>(t, nb, (const float *)kb, s);
}

// ---- sub-bucket particle trace (Sec. 2.2.3, 2.3) --------------------------
//
// Below a bucket the ray meets particles: each absorber j adds m_j kappa_j
// times its smoothing kernel's integral along the piece.  The set-up keeps,
// in sorted order, every particle's position and h and its m kappa; per
// bucket the spread of kappa rho over its particles (the refinement decision
// at that level); and per bucket the absorbers whose kernel support (radius
// 2h) reaches its box, found by a query down the tree with the largest h of
// each cell's absorbers.
template <typename T>
__global__ void k_sph_particles(const T *h, const int32_t *perm, const P4<T> *ps,
                                const T *pmass, const T *pkappa, int64_t n, P4<T> *pos,
                                double *mk, int *err) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const T hv = h[perm[k]];
  const double hd = (double)hv;
  if (!isfinite(hd))
    atomicOr(err, ERR_NONFINITE);
  else if (!(hd > 0))
    atomicOr(err, ERR_VALUE);
  P4<T> v = ps[k];
  v.L = hv;
  pos[k] = v;
  const double m = (double)pmass[k];
  mk[k] = m > 0 ? m * (double)pkappa[k] : 0.0;
}

template <typename T>
__global__ void k_sph_bucket(const BfsNode *lvl, int cnt, const T *pmass, const T *pkappa,
                             const T *prho, const P4<T> *pos, const double *mk, T *dp,
                             double *hmax) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  const BfsNode nd = lvl[j];
  if (nd.child >= 0) {
    dp[nd.pre] = (T)-1;
    return;
  }
  double lo = INFINITY, hi = -INFINITY, hm = 0.0;
  for (int k = nd.first; k < nd.first + nd.count; ++k) {
    if ((double)pmass[k] > 0) {
      const double a = (double)pkappa[k] * (double)prho[k];
      lo = a < lo ? a : lo;
      hi = a > hi ? a : hi;
    }
    const double h = (double)pos[k].L;
    if (mk[k] > 0 && h > hm) hm = h;
  }
  dp[nd.pre] = hi >= lo ? (T)(hi - lo) : (T)0;
  hmax[nd.pre] = hm;
}

__global__ void k_sph_internal(const BfsNode *lvl, int cnt, const int32_t *right,
                               double *hmax) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  const BfsNode nd = lvl[j];
  if (nd.child < 0) return;
  const int p = nd.pre;
  const double a = hmax[p + 1], b = hmax[right[p]];
  hmax[p] = a > b ? a : b;
}

// One thread per cell; a bucket walks its box's tree in depth-first order,
// skipping subtrees whose absorbers cannot reach it.  Without `off` it counts
// its absorbers, with it writes them (sorted indices, ascending).
template <typename T>
__global__ void k_sph_lists(int64_t m, const int32_t *right, const int32_t *skip,
                            const int32_t *first, const int32_t *count, const int32_t *nbox,
                            const int32_t *box_root, const double *lo, const double *hi,
                            const double *hmax, const P4<T> *pos, const double *mk,
                            const int64_t *off, int32_t *cnt, int32_t *out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  if (right[p] >= 0) {
    if (!off) cnt[p] = 0;
    return;
  }
  double blo[3], bhi[3];
  for (int a = 0; a < 3; ++a) {
    blo[a] = lo[a * m + p];
    bhi[a] = hi[a * m + p];
  }
  const int root = box_root[nbox[p]];
  const int end = skip[root];
  const int64_t w = off ? off[p] : 0;
  int found = 0;
  for (int c = root; c < end;) {
    const double hm = hmax[c];
    double g2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      double g = lo[a * m + c] - bhi[a];
      const double g1 = blo[a] - hi[a * m + c];
      if (g1 > g) g = g1;
      if (g > 0) g2 += g * g;
    }
    if (!(hm > 0) || !(g2 < 4.0 * hm * hm)) {
      c = skip[c];
      continue;
    }
    if (right[c] >= 0) {
      ++c;
      continue;
    }
    for (int k = first[c]; k < first[c] + count[c]; ++k) {
      if (!(mk[k] > 0)) continue;
      const P4<T> v = pos[k];
      const double x[3] = {(double)v.x, (double)v.y, (double)v.z};
      double d2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        const double g = blo[a] - x[a] > x[a] - bhi[a] ? blo[a] - x[a] : x[a] - bhi[a];
        if (g > 0) d2 += g * g;
      }
      const double h = (double)v.L;
      if (d2 < 4.0 * h * h) {
        if (off) out[w + found] = k;
        ++found;
      }
    }
    c = skip[c];
  }
  if (!off) cnt[p] = found;
}

// The walk's trace records with each bucket's particle spread in its spread
// field (a bucket's own spread is never used to split it).
template <typename T>
__global__ void k_sph_records(const TraceRecT<T> *TR, const T *dp, int64_t m, TraceRecT<T> *out) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  TraceRecT<T> r = TR[p];
  if (rax_right(r.right_ax) == 0) r.dalpha = dp[p];
  out[p] = r;
}

__global__ void k_sph_total(const int32_t *cnt, const int64_t *off, int64_t m, int64_t *tot) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    tot[0] = m > 0 ? off[m - 1] + (int64_t)cnt[m - 1] : 0;
}

template <typename T>
static int sph_typed(trevr_tree *t, const T *h, hipStream_t s) {
  const int64_t n = t->n, m = t->m;
  const size_t mm = (size_t)(m > 0 ? m : 1), nn = (size_t)(n > 0 ? n : 1);
  TREVR_HIP(t->sph_pos.ensure(sizeof(P4<T>) * nn));
  TREVR_HIP(t->sph_mk.ensure(8 * nn));
  TREVR_HIP(t->sph_dp.ensure(sizeof(T) * mm));
  TREVR_HIP(t->sph_hmax.ensure(8 * mm));
  TREVR_HIP(t->sph_cnt.ensure(4 * mm));
  TREVR_HIP(t->sph_off.ensure(8 * (mm + 1)));
  TREVR_HIP(t->sph_trace.ensure(sizeof(TraceRecT<T>) * mm));
  TREVR_HIP(hipMemsetAsync(t->err.p, 0, 4, s));
  if (n > 0)
    k_sph_particles<T><<<nblk(n), 256, 0, s>>>(
        h, t->perm.as<int32_t>(), t->psrc.as<P4<T>>(), t->pmass.as<T>(), t->pkappa.as<T>(), n,
        t->sph_pos.as<P4<T>>(), t->sph_mk.as<double>(), t->err.as<int>());
  TREVR_HIP(hipGetLastError());
  int herr = 0;
  TREVR_HIP(hipMemcpyAsync(&herr, t->err.p, 4, hipMemcpyDeviceToHost, s));
  TREVR_HIP(hipStreamSynchronize(s));
  if (herr & ERR_NONFINITE) return fail(TREVR_E_NONFINITE, "non-finite smoothing length");
  if (herr & ERR_VALUE) return fail(TREVR_E_VALUE, "smoothing length not positive");
  const BfsNode *bfs = t->bfs.as<BfsNode>();
  for (int d = (int)t->level_cnt.size() - 1; d >= 0; --d) {
    const BfsNode *lvl = bfs + t->level_off[d];
    const int c = (int)t->level_cnt[d];
    k_sph_bucket<T><<<nblk(c), 256, 0, s>>>(lvl, c, t->pmass.as<T>(), t->pkappa.as<T>(),
                                            t->prho.as<T>(), t->sph_pos.as<P4<T>>(),
                                            t->sph_mk.as<double>(), t->sph_dp.as<T>(),
                                            t->sph_hmax.as<double>());
    k_sph_internal<<<nblk(c), 256, 0, s>>>(lvl, c, t->n_right.as<int32_t>(),
                                           t->sph_hmax.as<double>());
  }
  auto lists = [&](const int64_t *off, int32_t *out) {
    k_sph_lists<T><<<nblk(m, 128), 128, 0, s>>>(
        m, t->n_right.as<int32_t>(), t->n_skip.as<int32_t>(), t->n_first.as<int32_t>(),
        t->n_count.as<int32_t>(), t->n_box.as<int32_t>(), t->box_root.as<int32_t>(),
        t->n_lo.as<double>(), t->n_hi.as<double>(), t->sph_hmax.as<double>(),
        t->sph_pos.as<P4<T>>(), t->sph_mk.as<double>(), off, t->sph_cnt.as<int32_t>(), out);
  };
  if (m > 0) {
    k_sph_records<T><<<nblk(m), 256, 0, s>>>(t->trace.as<TraceRecT<T>>(), t->sph_dp.as<T>(), m,
                                             t->sph_trace.as<TraceRecT<T>>());
    lists(nullptr, nullptr);
  }
  int32_t *cnt = t->sph_cnt.as<int32_t>();
  int64_t *off = t->sph_off.as<int64_t>();
  size_t tmp = 0;
  TREVR_HIP(rocprim::exclusive_scan(nullptr, tmp, cnt, off, (int64_t)0, (size_t)m,
                                    rocprim::plus<int64_t>(), s));
  if (tmp > t->sort_tmp.bytes) TREVR_HIP(t->sort_tmp.ensure(tmp));
  tmp = t->sort_tmp.bytes;
  TREVR_HIP(rocprim::exclusive_scan(t->sort_tmp.p, tmp, cnt, off, (int64_t)0, (size_t)m,
                                    rocprim::plus<int64_t>(), s));
  k_sph_total<<<1, 64, 0, s>>>(cnt, off, m, off + m);
  TREVR_HIP(hipGetLastError());
  int64_t total = 0;
  TREVR_HIP(hipMemcpyAsync(&total, off + m, 8, hipMemcpyDeviceToHost, s));
  TREVR_HIP(hipStreamSynchronize(s));
  {  // the lists must fit in the free device memory (beyond what they hold now)
    size_t free_b = 0, total_b = 0;
    TREVR_HIP(hipMemGetInfo(&free_b, &total_b));
    if ((double)total * 4.0 > 0.9 * (double)(free_b + t->sph_nb.bytes))
      return fail(TREVR_E_CAPACITY,
                  "absorber lists (" + std::to_string(total) +
                      " entries) exceed the free device memory: smoothing lengths too large");
  }
  TREVR_HIP(t->sph_nb.ensure(4 * (size_t)(total > 0 ? total : 1)));
  if (m > 0) lists(off, t->sph_nb.as<int32_t>());
  TREVR_HIP(hipGetLastError());
  TREVR_HIP(hipStreamSynchronize(s));
  t->sph_entries = total;
  t->sph_ok = true;
  return TREVR_OK;
}

int sph_impl(trevr_tree *t, const void *h, hipStream_t s) {
  t->sph_ok = false;
  if (t->prec == TREVR_F64) return sph_typed<double>(t, (const double *)h, s);
  return sph_typed<float>(t, (const float *)h, s);
}

// The absorber lists (input indices) and each cell's decision spread, to host
// memory; with offsets == NULL only the number of list entries.
int export_sph_impl(const trevr_tree *t, int64_t *n_entries, int64_t *offsets,
                    int64_t *neighbours, double *spread, hipStream_t s) {
  *n_entries = t->sph_entries;
  if (!offsets) return TREVR_OK;
  const int64_t m = t->m, e = t->sph_entries;
  std::vector<int32_t> nb((size_t)(e > 0 ? e : 1)), perm((size_t)(t->n > 0 ? t->n : 1));
  TREVR_HIP(hipMemcpyAsync(offsets, t->sph_off.p, 8 * (size_t)(m + 1), hipMemcpyDeviceToHost, s));
  if (e > 0) TREVR_HIP(hipMemcpyAsync(nb.data(), t->sph_nb.p, 4 * (size_t)e, hipMemcpyDeviceToHost, s));
  if (t->n > 0)
    TREVR_HIP(hipMemcpyAsync(perm.data(), t->perm.p, 4 * (size_t)t->n, hipMemcpyDeviceToHost, s));
  std::vector<double> dp((size_t)(m > 0 ? m : 1));
  if (t->prec == TREVR_F64) {
    if (m > 0) TREVR_HIP(hipMemcpyAsync(dp.data(), t->sph_dp.p, 8 * (size_t)m, hipMemcpyDeviceToHost, s));
    TREVR_HIP(hipStreamSynchronize(s));
  } else {
    std::vector<float> f((size_t)(m > 0 ? m : 1));
    if (m > 0) TREVR_HIP(hipMemcpyAsync(f.data(), t->sph_dp.p, 4 * (size_t)m, hipMemcpyDeviceToHost, s));
    TREVR_HIP(hipStreamSynchronize(s));
    for (int64_t p = 0; p < m; ++p) dp[(size_t)p] = (double)f[(size_t)p];
  }
  for (int64_t k = 0; k < e; ++k) neighbours[k] = perm[(size_t)nb[(size_t)k]];
  if (spread)
    for (int64_t p = 0; p < m; ++p) spread[p] = dp[(size_t)p];
  return TREVR_OK;
}

// ---- background shell (Sec. 2.2.4) -----------------------------------------
//
// Background sources sit on a sphere at the edge of the volume.  A merged
// cell of them has its centre of luminosity inside the sphere, which
// over-estimates the flux near the shell; such a cell (every luminous particle
// in it a background source) is given the point where the ray from the centre
// through its x_L meets the sphere, y' = c + R (x_L - c) / |x_L - c|.
template <typename T>
__global__ void k_bg_bucket(const BfsNode *lvl, int cnt, const P4<T> *ps, const int32_t *perm,
                            const uint8_t *flags, const int32_t *right, int32_t *nonbg) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  const BfsNode nd = lvl[j];
  const int p = nd.pre;
  if (nd.child >= 0) {
    nonbg[p] = nonbg[p + 1] | nonbg[right[p]];
    return;
  }
  int any = 0;
  for (int k = nd.first; k < nd.first + nd.count; ++k)
    if (ps[k].L > (T)0 && !flags[perm[k]]) any = 1;
  nonbg[p] = any;
}

template <typename T>
__global__ void k_bg_cells(const WalkRecT<T> *W, const int32_t *nonbg, int64_t m, double c0,
                           double c1, double c2, double radius, P4<T> *out) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  const WalkRecT<T> w = W[p];
  P4<T> o;
  o.x = w.xl[0];
  o.y = w.xl[1];
  o.z = w.xl[2];
  o.L = (T)0;
  if (w.L > (T)0 && !nonbg[p]) {
    const double c[3] = {c0, c1, c2};
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = (double)w.xl[a] - c[a];
    const double len = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    if (len > 0) {
      o.x = (T)(c[0] + radius * (v[0] / len));
      o.y = (T)(c[1] + radius * (v[1] / len));
      o.z = (T)(c[2] + radius * (v[2] / len));
    }
    o.L = (T)1;
  }
  out[p] = o;
}

template <typename T>
static int background_typed(trevr_tree *t, const double *centre, double radius,
                            const uint8_t *flags, hipStream_t s) {
  const int64_t m = t->m;
  const size_t mm = (size_t)(m > 0 ? m : 1);
  TREVR_HIP(t->bg_pos.ensure(sizeof(P4<T>) * mm));
  TREVR_HIP(t->bg_nonbg.ensure(4 * mm));
  const BfsNode *bfs = t->bfs.as<BfsNode>();
  for (int d = (int)t->level_cnt.size() - 1; d >= 0; --d) {  // children first
    const int c = (int)t->level_cnt[d];
    k_bg_bucket<T><<<nblk(c), 256, 0, s>>>(bfs + t->level_off[d], c, t->psrc.as<P4<T>>(),
                                           t->perm.as<int32_t>(), flags,
                                           t->n_right.as<int32_t>(), t->bg_nonbg.as<int32_t>());
  }
  if (m > 0)
    k_bg_cells<T><<<nblk(m), 256, 0, s>>>(t->walk.as<WalkRecT<T>>(), t->bg_nonbg.as<int32_t>(),
                                          m, centre[0], centre[1], centre[2], radius,
                                          t->bg_pos.as<P4<T>>());
  TREVR_HIP(hipGetLastError());
  TREVR_HIP(hipStreamSynchronize(s));
  t->bg_ok = true;
  return TREVR_OK;
}

int background_impl(trevr_tree *t, const double *centre, double radius, const uint8_t *flags,
                    hipStream_t s) {
  t->bg_ok = false;
  if (t->prec == TREVR_F64) return background_typed<double>(t, centre, radius, flags, s);
  return background_typed<float>(t, centre, radius, flags, s);
}

// Refit: new mass, rho, kappa and lum on the positions of the build.  Each
// particle's position must equal, value for value, the one the tree was built
// from (then every key, and the whole topology, is unchanged); the values are
// validated as in the build.
template <typename T>
__global__ void k_refit_check(PartIn<T> in, int64_t n, const int32_t *inv, const P4<T> *ps,
                              int *err) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const P4<T> v = ps[inv[q]];
  double m = in.mass ? (double)in.mass[q] : 1.0;
  double rho = (double)in.rho[q], kap = (double)in.kappa[q], L = (double)in.lum[q];
  int e = 0;
  if (!(in.x[q] == v.x && in.y[q] == v.y && in.z[q] == v.z)) e |= ERR_MOVED;
  if (!isfinite(m) || !isfinite(kap) || !isfinite(L) || (m > 0 && !isfinite(rho)))
    e |= ERR_NONFINITE;
  else if (m < 0 || kap < 0 || L < 0 || (m > 0 && !(rho > 0)))
    e |= ERR_VALUE;
  if (e) atomicOr(err, e);
}

template <typename T>
static int refit_typed(trevr_tree *t, const trevr_particles *p, hipStream_t s) {
  const int64_t n = t->n;
  PartIn<T> in{(const T *)p->x, (const T *)p->y, (const T *)p->z, (const T *)p->mass,
               (const T *)p->rho, (const T *)p->kappa, (const T *)p->lum};
  TREVR_HIP(hipMemsetAsync(t->err.p, 0, 4, s));
  if (n > 0)
    k_refit_check<T><<<nblk(n), 256, 0, s>>>(in, n, t->inv.as<int32_t>(),
                                             t->psrc.as<P4<T>>(), t->err.as<int>());
  TREVR_HIP(hipGetLastError());
  int herr = 0;
  TREVR_HIP(hipMemcpyAsync(&herr, t->err.p, 4, hipMemcpyDeviceToHost, s));
  TREVR_HIP(hipStreamSynchronize(s));
  if (herr & ERR_MOVED) return fail(TREVR_E_ARG, "a position differs from the build's");
  if (herr & ERR_NONFINITE) return fail(TREVR_E_NONFINITE, "non-finite input value");
  if (herr & ERR_VALUE)
    return fail(TREVR_E_VALUE, "negative mass/opacity/luminosity or density <= 0");
  t->built = false;
  int rc = cell_props<T>(t, in, n, t->m, t->n_boxes, s);
  if (rc != TREVR_OK) return rc;
  TREVR_HIP(hipStreamSynchronize(s));
  t->built = true;
  return TREVR_OK;
}

int refit_tree_impl(trevr_tree *t, const trevr_particles *p, hipStream_t s) {
  t->tape_ok = false;
  t->n_bands = 0;
  t->sph_ok = false;
  t->bg_ok = false;
  if (t->prec == TREVR_F64) return refit_typed<double>(t, p, s);
  return refit_typed<float>(t, p, s);
}

int build_tree_impl(trevr_tree *t, const trevr_particles *p, hipStream_t s) {
  t->built = false;
  t->tape_ok = false;
  t->n_bands = 0;
  t->sph_ok = false;
  t->bg_ok = false;
  if (p->prec == TREVR_F64) return build_typed<double>(t, p, s);
  return build_typed<float>(t, p, s);
}

// ---- export ---------------------------------------------------------------

template <typename U>
static int dl(std::vector<U> &h, const DevBuf &b, size_t count, hipStream_t s) {
  h.resize(count);
  if (count)
    TREVR_HIP(hipMemcpyAsync(h.data(), b.p, sizeof(U) * count, hipMemcpyDeviceToHost, s));
  return TREVR_OK;
}

int export_tree_impl(const trevr_tree *t, int64_t *perm, int64_t *leaf_of, int64_t *node_i,
                     uint64_t *node_key, double *node_f, hipStream_t s) {
  const size_t n = (size_t)t->n, m = (size_t)t->m;
  std::vector<int32_t> hp, hl, first, count, depth, parent, right, skip;
  std::vector<int8_t> axis;
  std::vector<uint64_t> key;
  std::vector<double> lo, hi, split, A, B, SL, SLx, alpha, amin, amax, dal, xl, lc, lfar;
  int rc;
#define DL(h, b, c) \
  if ((rc = dl(h, t->b, c, s)) != TREVR_OK) return rc
  DL(hp, perm, n);
  DL(hl, leaf, n);
  DL(first, n_first, m);
  DL(count, n_count, m);
  DL(depth, n_depth, m);
  DL(parent, n_parent, m);
  DL(right, n_right, m);
  DL(skip, n_skip, m);
  DL(axis, n_axis, m);
  DL(key, key, m);
  DL(lo, n_lo, 3 * m);
  DL(hi, n_hi, 3 * m);
  DL(split, n_split, m);
  DL(A, n_A, m);
  DL(B, n_B, m);
  DL(SL, n_SL, m);
  DL(SLx, n_SLx, 3 * m);
  DL(alpha, n_alpha, m);
  DL(amin, n_alpha_min, m);
  DL(amax, n_alpha_max, m);
  DL(dal, n_dalpha, m);
  DL(xl, n_xl, 3 * m);
  DL(lc, n_lc, m);
  DL(lfar, n_lfar, m);
#undef DL
  TREVR_HIP(hipStreamSynchronize(s));
  for (size_t k = 0; k < n; ++k) {
    if (perm) perm[k] = hp[k];
    if (leaf_of) leaf_of[hp[k]] = hl[k];
  }
  for (size_t p = 0; p < m; ++p) {
    if (node_i) {
      int64_t *o = node_i + 8 * p;
      o[0] = first[p];
      o[1] = count[p];
      o[2] = depth[p];
      o[3] = right[p] < 0 ? 1 : 0;
      o[4] = parent[p];
      o[5] = right[p];
      o[6] = skip[p];
      o[7] = axis[p];
    }
    if (node_key) node_key[p] = key[p];
    if (node_f) {
      double *o = node_f + 22 * p;
      for (int a = 0; a < 3; ++a) {
        o[0 + a] = lo[a * m + p];
        o[3 + a] = hi[a * m + p];
        o[10 + a] = SLx[a * m + p];
        o[17 + a] = xl[a * m + p];
      }
      o[6] = split[p];
      o[7] = A[p];
      o[8] = B[p];
      o[9] = SL[p];
      o[13] = alpha[p];
      o[14] = amin[p];
      o[15] = amax[p];
      o[16] = dal[p];
      o[20] = lc[p];
      o[21] = lfar[p];
    }
  }
  return TREVR_OK;
}

}  // namespace trevr
