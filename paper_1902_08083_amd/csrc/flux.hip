// Per-sink radiation field on gfx950 (Sec. 2.1-2.2.3 of the TREVR paper) and
// its adjoint.
//
// One wavefront evaluates 64 sinks that are adjacent in tree order, so their
// source walks (Sec. 2.2.1) visit nearly the same cells.  The walk is done
// once per wave: each visited cell is read with wave-uniform (scalar) loads,
// every lane applies the opening test (eq. openangle) for its own sink, the
// accepting lanes trace their ray at once, and the wave descends into a cell
// if any lane opened it.  Lanes that accepted an ancestor are masked off in
// its subtree; the per-depth masks live in LDS.
//
// A ray (Sec. 2.2.2-2.2.3) is traced by its own lane: split at the meeting
// cell A of the sink bucket S and the source cell C, walk down from A toward
// S and toward C, and wherever the ray lies in a chain cell's other half use
// that chain cell's average unless (alpha_max - alpha_min) l > tau_ref, in
// which case the other half is refined recursively (eq. refcrit).  The ray's
// geometry (direction, 1/d, r^2, r, plane crossings t, piece lengths l) is
// computed in the transport precision T, binary32 or binary64, each operation
// correctly rounded and none contracted; the refinement criterion's product
// and each term alpha l are exact binary64 products of T values, and tau and
// the flux are summed in binary64.  Cell data come from the transport records.
//
// The tracer hands every piece (cell, alpha, length, end points) to a policy:
// the forward sums tau; the adjoint, which re-runs the identical tracer,
// scatters d(loss)/d(alpha) to the cells and accumulates d tau / d y.
//
// Work distribution: a persistent grid; each wave takes chunks of 64 sinks
// from an atomic queue.  Workgroups are dealt round-robin to the 8 XCDs, so
// the queue is split into 8 contiguous ranges (one per XCD, taken by
// blockIdx % 8) and a wave steals from the next range once its own is empty:
// each XCD's L2 then sees a compact region of the tree.
#include <cmath>
#include <type_traits>

#include "trevr_internal.h"

namespace trevr {

constexpr int kXcd = 8;

template <typename T>
struct FluxArgs {
  const WalkRecT<T> *__restrict__ W;
  const TraceRecT<T> *__restrict__ TR;
  const uint64_t *__restrict__ key;
  const int32_t *__restrict__ ndepth;
  const P4<T> *__restrict__ ps;
  const int32_t *__restrict__ perm;
  const int32_t *__restrict__ inv;
  const int32_t *__restrict__ leaf;
  const int32_t *__restrict__ pbox;
  const int32_t *__restrict__ box_root;
  const uint64_t *__restrict__ axmask;  // per box: 3 masks of path-bit positions
  const int32_t *__restrict__ sinks;
  int64_t n_sinks;
  int64_t n;         // particles
  int32_t n_chunks;  // work-queue grabs
  int32_t group;     // 64-sink groups per grab
  double theta2, tau_ref;
  T *flux;
  T *flux_vec;  // [3][n_sinks]: the vector flux (kernels with MOM >= 1)
  T *flux_mom;  // [6][n_sinks]: the second moment xx, yy, zz, xy, xz, yz (MOM == 2)
  // opacity bands (kernels with NBND > 0): a.TR then carries the largest band
  // spread; a cell's alpha per band is band_alpha[cell][b] (4 per cell)
  const T *__restrict__ band_alpha;
  int32_t n_bands;
  T *flux_bands;  // [n_bands][n_sinks]
  // sub-bucket particle trace (kernels with SPH; a.TR then carries each
  // bucket's particle spread): per bucket its absorbers (sorted indices,
  // int64 offsets by cell), per particle x, y, z, h and m kappa
  const int64_t *__restrict__ sph_off;
  const int32_t *__restrict__ sph_nb;
  const P4<T> *__restrict__ sph_pos;
  const double *__restrict__ sph_mk;
  // walk variants (kernels with VAR): opening test 0 at the sink point,
  // 1 at the sink's bucket box, 2 Gasoline's opening radius about x_L; ray
  // walk 0 up the tree, 1 top down from the meeting cell; rays past tau_max
  // contribute nothing (and stop being traced)
  int32_t variant, open_mode, ray_mode;
  double tau_max;
  // background shell (kernels with VAR): per cell, x, y, z of its merged
  // source on the sphere and L = 1 where that applies, else null
  const P4<T> *__restrict__ bg_pos;
  int32_t *counters;
  int32_t *queue;  // kXcd counters
  // Tape of per-ray optical depths: one block of 64 per round, the blocks of
  // one 64-sink set chained in round order.  Mode 1 (flux) writes it, mode 2
  // (adjoint) reads it instead of tracing each ray for tau a first time, and
  // takes its rounds from the recorded ray lists instead of walking again.
  double *tape;        // [tape_cap][64]
  uint32_t *tape_src;  // [tape_cap][64] the ray's queue entry (its source)
  uint8_t *tape_own;   // [tape_cap][64] the ray's owning lane (its sink)
  uint8_t *tape_nb;    // [tape_cap] rays in the block's round (1..64)
  int32_t *tape_next;  // [tape_cap] the set's next block, -1 after its last
  int32_t *tape_head;  // [64-sink sets] the set's first block, -1 if it has none
  int32_t *tape_ctr;   // blocks taken; above tape_cap the tape is incomplete
  int32_t tape_cap;
  int32_t tape_mode;   // 0 none, 1 record, 2 replay
  int32_t tape_chunk;  // record: blocks a wave takes from the counter at once
  // adjoint
  const T *__restrict__ grad_flux;
  double *abar;    // [m]  d loss / d alpha
  double *lbar;    // [m]  d loss / d L_C
  double *xbar;    // [3][m] d loss / d x_L
  double *direct;  // [n]  d loss / d L_j (rays from single particles), sorted order
  int64_t m;
};

// v[a] for a in {0, 1, 2} as two selects: the three values are passed
// separately so that the ray's per-axis arrays stay in registers.
template <typename G>
__device__ __forceinline__ G pick3(int a, G v0, G v1, G v2) {
  const G v01 = a == 0 ? v0 : v1;
  return a == 2 ? v2 : v01;
}
#define sel3(v, a) pick3((a), (v)[0], (v)[1], (v)[2])

// A trace record as one 16-byte buffer load (two in binary64): tr_fetch
// issues it, tr_open unpacks the fields.  The buffer resource spans the
// record array from its base with 32-bit byte offsets (the build keeps the
// records within 4 GiB); a buffer-load intrinsic is never split into
// dependent loads of the fields that each branch uses, and its offset costs
// one shift instead of 64-bit address arithmetic.
template <typename T>
struct TrRaw;
template <>
struct TrRaw<float> {
  uint4 u;
};
template <>
struct TrRaw<double> {
  uint4 u, w;
};
// Raw buffer (stride 0), no range limit, gfx9 data format word.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tr_rsrc(const void *TR) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(TR), (short)0, -1, 0x00020000);
}
typedef __attribute__((ext_vector_type(4))) unsigned u32x4;
__device__ __forceinline__ TrRaw<float> tr_fetch(const TraceRecT<float> *TR, int i) {
  const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(tr_rsrc(TR), (unsigned)i * 16u, 0, 0);
  return TrRaw<float>{make_uint4(v.x, v.y, v.z, v.w)};
}
__device__ __forceinline__ TrRaw<double> tr_fetch(const TraceRecT<double> *TR, int i) {
  const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(tr_rsrc(TR), (unsigned)i * 32u, 0, 0);
  const u32x4 w =
      __builtin_amdgcn_raw_buffer_load_b128(tr_rsrc(TR), (unsigned)i * 32u + 16u, 0, 0);
  return TrRaw<double>{make_uint4(v.x, v.y, v.z, v.w), make_uint4(w.x, w.y, w.z, w.w)};
}
__device__ __forceinline__ TraceRecT<float> tr_open(TrRaw<float> v) {
  TraceRecT<float> r;
  r.split = __uint_as_float(v.u.x);
  r.alpha = __uint_as_float(v.u.y);
  r.dalpha = __uint_as_float(v.u.z);
  r.right_ax = (int32_t)v.u.w;
  return r;
}
__device__ __forceinline__ TraceRecT<double> tr_open(TrRaw<double> v) {
  TraceRecT<double> r;
  r.split = __hiloint2double((int)v.u.y, (int)v.u.x);
  r.alpha = __hiloint2double((int)v.u.w, (int)v.u.z);
  r.dalpha = __hiloint2double((int)v.w.y, (int)v.w.x);
  r.right_ax = (int32_t)v.w.z;
  r.pad = 0;
  return r;
}
template <typename T>
__device__ __forceinline__ TraceRecT<T> load_tr(const TraceRecT<T> *TR, int i) {
  return tr_open(tr_fetch(TR, i));
}

typedef __attribute__((address_space(3))) int32_t lds_i32;
typedef __attribute__((address_space(3))) double lds_d;

// Atomic adds with an explicit address space: LDS accumulators through
// ds_add_f64, device memory through global_atomic_add_f64 (never FLAT).
typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(1))) double gbl_f64;
__device__ __forceinline__ void lds_add(double *p, double v) {
  __builtin_amdgcn_ds_atomic_fadd_f64((lds_f64 *)p, v);
}
__device__ __forceinline__ void gbl_add(double *p, double v) {
  (void)__builtin_amdgcn_global_atomic_fadd_f64((gbl_f64 *)p, v);
}

// Orders a wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// The ray, in the geometry precision G (the transport precision).
template <typename G>
struct RayCtx {
  G xi[3], d[3], inv[3];
  G r, r2;
  double tau_ref;
  int n_seg, n_trace;
  int pm;  // per axis a: bit a set if d_a == 0, bit a + 4 if d_a <= 0 (near half upper)
  // the lane's refinement stack in LDS (stride 64): kr entries, deeper ones
  // spill to private memory.  An entry is a pending cell | (tag + 1) << 30
  // and its exit parameter: in binary32 both in one 8-byte word (st), in
  // binary64 in two arrays (stn, stb).
  int32_t *stn;
  double *stb;
  uint64_t *st;
  int kr;
};

// The deeper part of the lane's stack, in private memory, in the LDS part's
// format: binary32 entries packed in 8 bytes, binary64 ones in 12.
template <typename G>
struct StackSpill;
template <>
struct StackSpill<float> {
  uint64_t e[kRefineStack];
};
template <>
struct StackSpill<double> {
  uint32_t n[kRefineStack];
  double t[kRefineStack];
};
__device__ __forceinline__ void spill_write(StackSpill<float> &o, int i, uint32_t e, float t) {
  o.e[i] = (uint64_t)e | ((uint64_t)__float_as_uint(t) << 32);
}
__device__ __forceinline__ void spill_write(StackSpill<double> &o, int i, uint32_t e, double t) {
  o.n[i] = e;
  o.t[i] = t;
}
__device__ __forceinline__ void spill_read(const StackSpill<float> &o, int i, uint32_t &e,
                                           float &t) {
  const uint64_t v = o.e[i];
  e = (uint32_t)v;
  t = __uint_as_float((uint32_t)(v >> 32));
}
__device__ __forceinline__ void spill_read(const StackSpill<double> &o, int i, uint32_t &e,
                                           double &t) {
  e = o.n[i];
  t = o.t[i];
}

// A stack entry whose cell is kMark opens a deferred refinement job: its tag
// and parameter are the job's entry crossing; the entry below it holds the
// cell and the exit.  Cell indices stay below kMark (the build checks).
constexpr int kMark = 0x3fffffff;

typedef __attribute__((address_space(3))) uint64_t lds_u64;
// LDS slot k of the lane's stack: write an entry (e = cell | (tag + 1) << 30)
// and read one back.
__device__ __forceinline__ void st_write(const RayCtx<float> &c, int k, uint32_t e, float t) {
  ((lds_u64 *)c.st)[k * kWave] = (uint64_t)e | ((uint64_t)__float_as_uint(t) << 32);
}
__device__ __forceinline__ void st_write(const RayCtx<double> &c, int k, uint32_t e, double t) {
  ((lds_i32 *)c.stn)[k * kWave] = (int32_t)e;
  ((lds_d *)c.stb)[k * kWave] = t;
}
__device__ __forceinline__ void st_read(const RayCtx<float> &c, int k, uint32_t &e, float &t) {
  const uint64_t v = ((lds_u64 *)c.st)[k * kWave];
  e = (uint32_t)v;
  t = __uint_as_float((uint32_t)(v >> 32));
}
__device__ __forceinline__ void st_read(const RayCtx<double> &c, int k, uint32_t &e, double &t) {
  e = (uint32_t)((lds_i32 *)c.stn)[k * kWave];
  t = ((lds_d *)c.stb)[k * kWave];
}
template <typename G>
__device__ __forceinline__ void stack_push(RayCtx<G> &c, StackSpill<G> &ovf, int k, int node,
                                           int tag, G t) {
  const uint32_t e = (uint32_t)node | ((uint32_t)(tag + 1) << 30);
  if (k < c.kr)
    st_write(c, k, e, t);
  else
    spill_write(ovf, k - c.kr, e, t);
}
template <typename G>
__device__ __forceinline__ void stack_pop(const RayCtx<G> &c, const StackSpill<G> &ovf, int k,
                                          int &node, int &tag, G &t) {
  uint32_t e;
  if (k < c.kr)
    st_read(c, k, e, t);
  else
    spill_read(ovf, k - c.kr, e, t);
  node = (int)(e & 0x3fffffffu);
  tag = (int)(e >> 30) - 1;
}

// A policy receives each piece as (cell, alpha, length, entry t and plane,
// exit t and plane, spread) -- spread: for a bucket, its record's
// spread field (the particle spread in the particle-trace kernel's records),
// -1 for other cells.  Its traits shape the tracer at compile time: kLight
// picks the form of the refinement step (see refine_branchy); kVar enables
// the walk variants' top-down walk and early stop (a stop() member); kCount
// keeps the per-ray counters of pieces and steps; kTags carries the planes
// that bound each piece through the stack (the entry and exit plane
// arguments are -1 or stale without it).
// Forward policy: tau = sum alpha l (eq. tausum).
struct TauSum {
  static constexpr bool kLight = false;
  static constexpr bool kVar = false;   // walk variants: top-down walk, early stop
  static constexpr bool kCount = true;  // per-ray counters of pieces and steps
  static constexpr bool kTags = false;  // the planes that bound each piece (adjoint scatter)
  double tau = 0.0;
  __device__ __forceinline__ void operator()(int, double alpha, double l, double, int, double,
                                             int, double) {
    tau += alpha * l;
  }
};

// The same sum without the counters (a flux call that asks for none).
struct TauSumNC : TauSum {
  static constexpr bool kCount = false;
};

// The same sum in the adjoint's first pass.
struct TauSumA : TauSum {
  static constexpr bool kLight = true;
  static constexpr bool kCount = false;
};

// The sum of the walk variants: the tracer stops once tau passes tau_max
// (pieces add non-negative terms, so the ray's full tau would too).
template <bool C = true>
struct TauVar : TauSum {
  static constexpr bool kVar = true;
  static constexpr bool kCount = C;
  double tau_max;
  __device__ __forceinline__ bool stop() const { return tau > tau_max; }
};

// Band policy: one tau per opacity band; a piece's alpha is that band's cell
// value (the record's own alpha is not used).
constexpr int kMaxBands = 4;
template <typename T, bool C = true>
struct BandSum {
  static constexpr bool kLight = false;
  static constexpr bool kVar = false;
  static constexpr bool kCount = C;
  static constexpr bool kTags = false;
  const T *ba;  // [cell][4]
  int nb;
  double tau[kMaxBands] = {0.0, 0.0, 0.0, 0.0};
  __device__ __forceinline__ void operator()(int node, double, double l, double, int, double,
                                             int, double) {
    T v[kMaxBands];
    if constexpr (sizeof(T) == 4) {  // the cell's bands in one 16-byte load
      const float4 q = reinterpret_cast<const float4 *>(ba)[node];
      v[0] = q.x;
      v[1] = q.y;
      v[2] = q.z;
      v[3] = q.w;
    } else {
      for (int b = 0; b < kMaxBands; ++b) v[b] = ba[(int64_t)kMaxBands * node + b];
    }
    for (int b = 0; b < kMaxBands; ++b)
      if (b < nb) tau[b] += (double)v[b] * l;
  }
};

// The M4 cubic spline (support 2h, W = w(r/h) / (pi h^3)) integrated along a
// line at impact parameter b, in units of h: G(beta, s) is the integral of
// w(sqrt(beta^2 + u^2)) over u in [0, s], s >= 0.  w is a polynomial in q on
// q < 1 and on 1 <= q < 2, and along the line the integrals of q^0 and q^2 are
// polynomials in u, those of q and q^3 closed forms with asinh(u / beta),
// taken as log(s + q) - log(beta) (lnb: log(beta), shared by a line's
// evaluations; the term is scaled by beta^2, so the difference's rounding
// stays at the level of the other terms').
// in_out: the inner and the outer polynomial's primitive at s (q = |(beta, s)|).
__device__ __forceinline__ void m4_prims(double beta, double b2, double lnb, double s,
                                         double &p_in, double &p_out) {
  const double q = sqrt(b2 + s * s);
  const double as = beta > 0.0 ? log(s + q) - lnb : 0.0;
  const double i1 = 0.5 * (s * q + b2 * as);
  const double i2 = b2 * s + (s * s * s) / 3.0;
  const double i3 = 0.125 * (s * q * (2.0 * s * s + 5.0 * b2)) + 0.375 * (b2 * b2) * as;
  p_in = s - 1.5 * i2 + 0.75 * i3;
  p_out = 2.0 * s - 3.0 * i1 + 1.5 * i2 - 0.25 * i3;
}
// G at |v|, with the sign of v (G is odd in s); s1, s2: where q = 1, 2 along
// the line (s1 = 0 when beta >= 1), k_io = inner - outer primitive at s1.
__device__ __forceinline__ double m4_g(double beta, double b2, double lnb, double v, double s1,
                                       double s2, double k_io) {
  double s = fabs(v);
  s = s < s2 ? s : s2;
  double p_in, p_out;
  m4_prims(beta, b2, lnb, s, p_in, p_out);
  const double g = s <= s1 ? p_in : k_io + p_out;
  return v < 0.0 ? -g : g;
}
// Integral of W(sqrt(b^2 + u^2), h) over u in [u0, u1].
__device__ __forceinline__ double m4_line(double b, double h, double u0, double u1) {
  const double beta = b / h;
  if (!(beta < 2.0)) return 0.0;
  const double b2 = beta * beta;
  const double s2 = sqrt(4.0 - b2);
  const double v0 = u0 / h, v1 = u1 / h;
  if (v0 >= s2 || v1 <= -s2) return 0.0;  // the piece misses the support
  const double lnb = beta > 0.0 ? log(beta) : 0.0;
  double s1 = 0.0, k_io = 0.0;
  if (b2 < 1.0) {
    s1 = sqrt(1.0 - b2);
    double p_in, p_out;
    m4_prims(beta, b2, lnb, s1, p_in, p_out);
    k_io = p_in - p_out;
  }
  const double g =
      m4_g(beta, b2, lnb, v1, s1, s2, k_io) - m4_g(beta, b2, lnb, v0, s1, s2, k_io);
  return g / (M_PI * h * h);
}

// Sub-bucket policy (Sec. 2.2.3, 2.3): a piece in a bucket whose particle
// spread fails the refinement test, spread * l > tau_ref, takes the particle
// trace -- each of the bucket's absorbers but the receiving particle adds
// m kappa times its kernel's integral over the piece; every other piece adds
// alpha l as in eq. (tausum).  Few pieces take the particle trace, each with a
// list of a few hundred absorbers, so a lane leaves its first kSphJobs such
// pieces as jobs that the whole wave runs after the round's trace (sph_jobs);
// further ones it traces itself.
constexpr int kSphJobs = 4;

// The ray for absorber terms: binary64, and binary32 for the rejection test.
struct SphRay {
  double xi[3], d[3], r, r2;
  float xf[3], df[3], inv_r2f, inv_rf;
  float slack;  // 4e-6 of the magnitude of the ray's coordinates (and of its length)
  int self;     // the receiving particle (sorted index)
  __device__ __forceinline__ void finish() {
    double mag = r;
    for (int a = 0; a < 3; ++a) {
      xf[a] = (float)xi[a];
      df[a] = (float)d[a];
      const double a0 = fabs(xi[a]), a1 = fabs(xi[a] + d[a]);
      mag = fmax(mag, fmax(a0, a1) + r);
    }
    inv_r2f = (float)(1.0 / r2);
    inv_rf = (float)(1.0 / r);
    slack = (float)(4e-6 * mag);
  }
  // whether absorber j's support may reach the piece (never false for one
  // whose term is not zero; false for the receiver)
  template <typename T>
  __device__ __forceinline__ bool reaches(const P4<T> *pos, int j, float taf, float tbf) const {
    if (j == self) return false;
    const P4<T> pj = pos[j];
    // Rejection in binary32: the absorber's distance to the line, or its
    // closest approach beyond the piece's ends, exceeds 2h (1 + 1e-3) + slack.
    // The binary32 error of both, in length, is below 1e-6 of the
    // coordinates' magnitude, which slack covers four times over, so a
    // rejected absorber's term is exactly zero in binary64 as well.
    const float ex = (float)pj.x - xf[0], ey = (float)pj.y - xf[1], ez = (float)pj.z - xf[2];
    const float tsf = ((ex * df[0] + ey * df[1]) + ez * df[2]) * inv_r2f;
    const float px = ex - tsf * df[0], py = ey - tsf * df[1], pz = ez - tsf * df[2];
    const float reach = 2.002f * (float)pj.L + slack;
    if ((px * px + py * py) + pz * pz >= reach * reach) return false;
    const float win = reach * inv_rf;
    return !(tsf <= taf - win || tsf >= tbf + win);
  }
  // absorber j's term m kappa (integral of W along the piece), binary64
  template <typename T>
  __device__ __forceinline__ double exact(const P4<T> *pos, const double *mk, int j, double ta,
                                          double tb) const {
    const P4<T> pj = pos[j];
    const double dl0 = (double)pj.x - xi[0], dl1 = (double)pj.y - xi[1],
                 dl2 = (double)pj.z - xi[2];
    const double ts = ((dl0 * d[0] + dl1 * d[1]) + dl2 * d[2]) / r2;  // closest approach
    const double p0 = dl0 - ts * d[0], p1 = dl1 - ts * d[1], p2 = dl2 - ts * d[2];
    const double b = sqrt((p0 * p0 + p1 * p1) + p2 * p2);
    return mk[j] * m4_line(b, (double)pj.L, (ta - ts) * r, (tb - ts) * r);
  }
};

// A bucket piece traced by its own lane (a ray's jobs beyond kSphJobs; rare).
// Out of line, so that the tracer's many emit sites stay small; the ray comes
// by value.
template <typename T>
__device__ __attribute__((noinline)) double sph_piece_lane(
    const int64_t *off, const int32_t *nb, const P4<T> *pos, const double *mk, int node,
    double ta, double tb, double x0, double x1, double x2, double d0, double d1, double d2,
    double r, double r2, int self) {
  SphRay g;
  g.xi[0] = x0;
  g.xi[1] = x1;
  g.xi[2] = x2;
  g.d[0] = d0;
  g.d[1] = d1;
  g.d[2] = d2;
  g.r = r;
  g.r2 = r2;
  g.self = self;
  g.finish();
  const int64_t e = off[node + 1];
  const float taf = (float)ta, tbf = (float)tb;
  double tau = 0.0;
  for (int64_t k = off[node]; k < e; ++k) {
    const int j = nb[k];
    if (g.reaches(pos, j, taf, tbf)) tau += g.exact(pos, mk, j, ta, tb);
  }
  return tau;
}

template <typename T, bool C = true>
struct SphSum {
  static constexpr bool kLight = false;
  static constexpr bool kVar = false;
  static constexpr bool kCount = C;
  static constexpr bool kTags = false;
  const int64_t *off;
  const int32_t *nb;
  const P4<T> *pos;
  const double *mk;
  const RayCtx<T> *c;  // the lane's ray (xi, d, r, r2)
  double tau_ref;
  int self;  // the receiving particle (sorted index)
  double tau = 0.0;
  int nj = 0;  // jobs left for the wave: bucket, piece ends
  int jn[kSphJobs];
  double jta[kSphJobs], jtb[kSphJobs];

  __device__ __forceinline__ void operator()(int node, double alpha, double l, double ta, int,
                                             double tb, int, double spread) {
    if (!(spread >= 0.0 && spread * l > tau_ref)) {
      tau += alpha * l;
      return;
    }
    if (nj < kSphJobs) {  // selects keep the job slots in registers
      for (int q = 0; q < kSphJobs; ++q)
        if (q == nj) {
          jn[q] = node;
          jta[q] = ta;
          jtb[q] = tb;
        }
      ++nj;
      return;
    }
    tau += sph_piece_lane<T>(off, nb, pos, mk, node, ta, tb, c->xi[0], c->xi[1], c->xi[2],
                             c->d[0], c->d[1], c->d[2], c->r, c->r2, self);
  }
};

// The jobs of every lane's SphSum, one at a time, by the whole wave.  The
// lanes test the bucket's absorbers 64 at a time and pack those that reach
// the piece into an LDS buffer of the wave (kSphBuf entries; the refinement
// stack's, which is free between rays); the packed ones are then evaluated
// in binary64, lane i taking entries i, i + 64, ...  The terms are summed in a
// fixed order (per lane, then a butterfly over the wave) and the sum is added
// to the job's lane.  Called by all lanes of the wave together; c is the
// lane's ray.
constexpr int kSphBuf = 1024;
template <typename T, bool C>
__device__ __forceinline__ void sph_jobs(SphSum<T, C> &ss, const RayCtx<T> &c, int lane,
                                         int32_t *buf) {
  const uint64_t below = (1ull << lane) - 1;
  lds_i32 *lb = (lds_i32 *)buf;
  for (int q = 0; q < kSphJobs; ++q) {
    uint64_t pend = __ballot(ss.nj > q);
    while (pend) {
      const int L = __ffsll((unsigned long long)pend) - 1;
      pend &= pend - 1;
      int node = 0;
      double ta = 0.0, tb = 0.0;
      for (int u = 0; u < kSphJobs; ++u)
        if (u == q) {
          node = ss.jn[u];
          ta = ss.jta[u];
          tb = ss.jtb[u];
        }
      node = __shfl(node, L);
      ta = __shfl(ta, L);
      tb = __shfl(tb, L);
      SphRay g;  // the job lane's ray
      for (int a = 0; a < 3; ++a) {
        g.xi[a] = (double)__shfl(c.xi[a], L);
        g.d[a] = (double)__shfl(c.d[a], L);
      }
      g.r = (double)__shfl(c.r, L);
      g.r2 = (double)__shfl(c.r2, L);
      g.self = __shfl(ss.self, L);
      g.finish();
      const float taf = (float)ta, tbf = (float)tb;
      const int64_t b0 = ss.off[node], e = ss.off[node + 1];
      double part = 0.0;
      int nbuf = 0;
      for (int64_t k0 = b0; k0 < e; k0 += 64) {
        const int64_t k = k0 + lane;
        int j = 0;
        bool hit = false;
        if (k < e) {
          j = ss.nb[k];
          hit = g.reaches(ss.pos, j, taf, tbf);
        }
        const uint64_t bm = __ballot(hit);
        if (hit) lb[nbuf + __popcll(bm & below)] = j;
        nbuf += __popcll(bm);
        if (nbuf > kSphBuf - 64 || k0 + 64 >= e) {
          wave_sync();
          for (int i = lane; i < nbuf; i += 64) part += g.exact(ss.pos, ss.mk, lb[i], ta, tb);
          wave_sync();
          nbuf = 0;
        }
      }
      part = wave_sum(part);
      if (lane == L) ss.tau += part;
    }
  }
}

// Adjoint policy: d loss / d alpha_cell += -g l, and d tau / d y gets
// r alpha (d tb/dy - d ta/dy) with d t/d y_a = -t / d_a for a plane crossing:
// per axis a the sums of alpha t over the crossings of that axis (entries
// minus exits) are kept in u, and d tau / d y_a += r u_a / d_a once per ray.
struct Scatter {
  static constexpr bool kLight = true;
  static constexpr bool kVar = false;
  static constexpr bool kCount = false;
  static constexpr bool kTags = true;
  double g;        // weight * flux contribution of the ray
  double dtdy[3];  // d tau / d y
  double u[3];     // per axis: sum of alpha t over entry crossings minus exit crossings
  double r;
  double inv[3];
  double *abar;
  int32_t *hk;  // per-wave LDS table of cells: keys (-1: free) ...
  double *hv;   // ... and their sums, written out after each round
  int hmask;    // table slots - 1 (a power of two minus one)
  // Every piece goes to the table, at the slot of its cell's number modulo
  // the table size: a round's rays share most of their cells, so the round's
  // sums reach device memory as about one atomic per distinct cell, and the
  // cells of a round are numbered close together (depth-first order), so
  // neighbours take neighbouring slots.  One compare-and-swap claims a free
  // slot or finds the cell's own.  A cell whose slot holds another cell
  // takes it over: the slot's old sum goes to device memory, so the table
  // keeps the cells the round is working on.  Of several lanes of one call
  // that would take the same slot, one does (a compare-and-swap on the key it
  // saw); the others send their own sum to device memory.  The call's hits
  // land before any slot changes hands.  (Measured at 2^20: 111.2 -> 109.0 ms
  // against two probes at two multiplicative hashes.)
  __device__ __forceinline__ void pool(int node, double v) {
    const int sl = (int)((uint32_t)node & (uint32_t)hmask);
    int k = -1;  // the slot's key before: free (now ours), this cell, or another
    __hip_atomic_compare_exchange_strong((lds_i32 *)hk + sl, &k, node, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    const bool hit = k == -1 || k == node;
    if (hit) lds_add(&hv[sl], v);
    // The two branches exclude each other per lane, so without this the
    // compiler may order a take-over before another lane's hit on that slot.
    wave_sync();
    if (!hit) {
      int kk = k;
      __hip_atomic_compare_exchange_strong((lds_i32 *)hk + sl, &kk, node, __ATOMIC_RELAXED,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      if (kk == k) {
        const double old = __hip_atomic_exchange((lds_d *)hv + sl, v, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WAVEFRONT);
        gbl_add(&abar[k], old);
      } else {
        gbl_add(&abar[node], v);
      }
    }
  }
  __device__ __forceinline__ void operator()(int node, double alpha, double l, double ta, int ga,
                                             double tb, int gb, double) {
    pool(node, -(g * l));

    // Each crossing goes to its axis's sum by an FMA with a coefficient of 1,
    // -1 or 0 (a select of the high word only): cheaper than selecting the
    // binary64 terms themselves.
    const double xb = alpha * tb, xa = alpha * ta;
    u[0] = fma(ga == 0 ? 1.0 : 0.0, xa, u[0]);
    u[1] = fma(ga == 1 ? 1.0 : 0.0, xa, u[1]);
    u[2] = fma(ga == 2 ? 1.0 : 0.0, xa, u[2]);
    u[0] = fma(gb == 0 ? -1.0 : 0.0, xb, u[0]);
    u[1] = fma(gb == 1 ? -1.0 : 0.0, xb, u[1]);
    u[2] = fma(gb == 2 ? -1.0 : 0.0, xb, u[2]);
  }
};

// Refinement of cell X on [ta, tb]: the cell's own average unless it is not a
// bucket and (alpha_max - alpha_min) l > tau_ref; then the near and far
// halves in ray order (an explicit stack replaces the recursion).  A ray in
// the split plane lies in the upper half only.  The lane's stack holds sp0
// entries, deferred jobs (a marker over a cell); those above depth base are
// refined after X, those below are left for a later call.
//
// Two forms of one step, with identical arithmetic and emit order.  The
// branching form takes either the split or the emit-and-pop path and leaves
// the loop at one place, after the next record is requested (a finished lane
// requests its last cell again); the light form evaluates the split on every
// lane, writes the free slot above the stack top and reads the two top slots
// unconditionally, and selects the next state.  Measured on this hardware,
// the light form is the faster one in the adjoint kernel (both passes), the
// branching form in the forward kernel.
template <typename T, typename Emit>
__device__ void refine_branchy(const TraceRecT<T> *__restrict__ TR, int X, T ta,
                               int ga, T tb, int gb, RayCtx<T> &c, StackSpill<T> &ovf, int sp0,
                               int base, Emit &emit) {
  int sp = sp0;
  int cur = X;
  T cta = ta, ctb = tb;
  int cga = ga, cgb = gb;
  TrRaw<T> raw = tr_fetch(TR, cur);
  bool go = true;
  do {
    const TraceRecT<T> rec = tr_open(raw);
    const T l = c.r * (ctb - cta);
    if constexpr (Emit::kCount) c.n_trace++;
    const int right = rax_right(rec.right_ax);
    const bool split_it = (right != 0) & ((double)rec.dalpha * (double)l > c.tau_ref);
    int ncur = cur;
    if (!split_it) {
      if constexpr (Emit::kCount) c.n_seg += l > 0;
      emit(cur, (double)rec.alpha, (double)l, (double)cta, cga,
           (double)ctb, cgb, right == 0 ? (double)rec.dalpha : -1.0);
      go = sp > base;
      if constexpr (Emit::kVar) go = go && !emit.stop();
      if (go) {
        int nd, tg;
        T tt;
        stack_pop(c, ovf, --sp, nd, tg, tt);
        if (nd == kMark) {  // a deferred job: its entry, then its cell and exit
          cta = tt;
          cga = tg;
          stack_pop(c, ovf, --sp, nd, tg, tt);
        } else {
          cta = ctb;
          cga = cgb;
        }
        ncur = nd;
        ctb = tt;
        cgb = tg;
      }
    } else {
      const int ax = rax_axis(rec.right_ax);
      const T s = rec.split;
      const T xax = sel3(c.xi, ax);
      const T ts = (s - xax) * sel3(c.inv, ax);
      const bool up = (c.pm >> (ax + 4)) & 1;  // near half is the upper child
      const int nearc = up ? right : cur + 1;
      const int farc = up ? cur + 1 : right;
      const bool cut_b = ts < ctb;      // the plane ends the near part
      const bool cut_a = !(ts <= cta);  // the plane starts the far part (also for NaN)
      const T t1 = cut_b ? ts : ctb;
      const int g1 = cut_b ? ax : cgb;
      const T t0 = cut_a ? ts : cta;
      const int g0 = cut_a ? ax : cga;
      const bool has_near = t1 > cta;
      const bool has_far = ctb > t0;
      if (has_near && has_far) stack_push(c, ovf, sp++, farc, Emit::kTags ? cgb : -1, ctb);
      go = has_near || has_far;  // one of them: refinement's intervals are never empty
      ncur = has_near ? nearc : farc;
      cta = has_near ? cta : t0;
      cga = has_near ? cga : g0;
      ctb = has_near ? t1 : ctb;
      cgb = has_near ? g1 : cgb;
    }
    cur = ncur;
    raw = tr_fetch(TR, cur);
  } while (go);
}
template <typename T, typename Emit>
__device__ void refine_light(const TraceRecT<T> *__restrict__ TR, int X, T ta,
                             int ga, T tb, int gb, RayCtx<T> &c, StackSpill<T> &ovf, int sp0,
                             int base, Emit &emit) {
  int sp = sp0;
  int cur = X;
  T cta = ta, ctb = tb;
  int cga = ga, cgb = gb;
  TrRaw<T> raw = tr_fetch(TR, cur);
  for (;;) {
    const TraceRecT<T> rec = tr_open(raw);
    const T l = c.r * (ctb - cta);
    if constexpr (Emit::kCount) c.n_trace++;
    const int right = rax_right(rec.right_ax);
    const bool split_it = (right != 0) & ((double)rec.dalpha * (double)l > c.tau_ref);
    // Every lane evaluates the split; the next state is selected below.
    const int ax = rax_axis(rec.right_ax);
    const T s = rec.split;
    const T xax = sel3(c.xi, ax);
    const T ts = (s - xax) * sel3(c.inv, ax);
    const bool up = (c.pm >> (ax + 4)) & 1;  // near half is the upper child
    const bool cut_b = ts < ctb;             // the plane ends the near part
    const bool cut_a = !(ts <= cta);         // the plane starts the far part (also for NaN)
    const T t1 = cut_b ? ts : ctb;
    const T t0 = cut_a ? ts : cta;
    const bool has_near = t1 > cta;
    const bool has_far = ctb > t0;
    const int nearc = up ? right : cur + 1;
    const int farc = up ? cur + 1 : right;
    const bool push = split_it & has_near & has_far;
    const bool pop = !split_it & (sp > base);
    // The slot above the top is free, so the LDS part is written whether or
    // not the lane pushes; reads of the two top slots are clamped in range.
    {
      const int tg = Emit::kTags ? cgb : -1;
      const uint32_t e = (uint32_t)farc | ((uint32_t)(tg + 1) << 30);
      if (sp < c.kr)
        st_write(c, sp, e, ctb);
      else if (push)
        spill_write(ovf, sp - c.kr, e, ctb);
    }
    int nd1, tg1, nd2, tg2;
    T tt1, tt2;
    {
      const int k1 = sp - 1, k2 = sp - 2;
      const int r1 = k1 < 0 ? 0 : k1 < c.kr ? k1 : c.kr - 1;
      const int r2 = k2 < 0 ? 0 : k2 < c.kr ? k2 : c.kr - 1;
      uint32_t e1, e2;
      st_read(c, r1, e1, tt1);
      st_read(c, r2, e2, tt2);
      if (pop && k1 >= c.kr) spill_read(ovf, k1 - c.kr, e1, tt1);
      nd1 = (int)(e1 & 0x3fffffffu);
      tg1 = (int)(e1 >> 30) - 1;
      if (pop && nd1 == kMark && k2 >= c.kr) spill_read(ovf, k2 - c.kr, e2, tt2);
      nd2 = (int)(e2 & 0x3fffffffu);
      tg2 = (int)(e2 >> 30) - 1;
    }
    const bool job = pop & (nd1 == kMark);  // a deferred job: its entry, then its cell and exit
    const bool done = split_it ? !(has_near | has_far) : !pop;
    int ncur;
    T ncta, nctb;
    int ncga, ncgb;
    if (split_it) {
      ncur = has_near ? nearc : farc;
      ncta = has_near ? cta : t0;
      ncga = has_near ? cga : (cut_a ? ax : cga);
      nctb = has_near ? t1 : ctb;
      ncgb = has_near ? (cut_b ? ax : cgb) : cgb;
    } else {
      ncur = job ? nd2 : nd1;
      ncta = job ? tt1 : ctb;
      ncga = job ? tg1 : cgb;
      nctb = job ? tt2 : tt1;
      ncgb = job ? tg2 : tg1;
    }
    sp += push ? 1 : job ? -2 : pop ? -1 : 0;
    // The next record is requested before the piece is emitted (an emit that
    // writes device memory then does not delay it).
    raw = tr_fetch(TR, done ? cur : ncur);
    if (!split_it) {
      if constexpr (Emit::kCount) c.n_seg += l > 0;
      emit(cur, (double)rec.alpha, (double)l, (double)cta, cga,
           (double)ctb, cgb, right == 0 ? (double)rec.dalpha : -1.0);
    }
    if (done) return;  // no entry left
    cur = ncur;
    cta = ncta;
    ctb = nctb;
    cga = ncga;
    cgb = ncgb;
  }
}
template <typename T, typename Emit>
__device__ __forceinline__ void refine(const TraceRecT<T> *__restrict__ TR, int X, T ta, int ga,
                                       T tb, int gb, RayCtx<T> &c,
                                       StackSpill<T> &ovf, int sp0, int base, Emit &emit) {
  if constexpr (Emit::kLight)
    refine_light<T>(TR, X, ta, ga, tb, gb, c, ovf, sp0, base, emit);
  else
    refine_branchy<T>(TR, X, ta, ga, tb, gb, c, ovf, sp0, base, emit);
}
// A piece of the ray in chain cell P but outside P's child on the path: P's
// own average, or, if P fails the refinement test, the sibling X to be
// refined later -- a job (X on [ta, tb]) is left on the lane's stack, so
// that all of a ray's refinement runs in one loop after its chains.
template <typename T, typename Emit>
__device__ __forceinline__ void chain_piece(const TraceRecT<T> *__restrict__ TR,
                                            const TraceRecT<T> &rP, int P, int X, T ta, int ga,
                                            T tb, int gb, RayCtx<T> &c,
                                            StackSpill<T> &ovf, int &sp, Emit &emit) {
  const T l = c.r * (tb - ta);
  if constexpr (Emit::kCount) c.n_trace++;
  if ((double)rP.dalpha * (double)l > c.tau_ref) {
    if (sp + 2 <= c.kr - 2) {  // room in the LDS part, two entries kept for refinement
      stack_push(c, ovf, sp++, X, Emit::kTags ? gb : -1, tb);
      stack_push(c, ovf, sp++, kMark, Emit::kTags ? ga : -1, ta);
    } else {
      refine<T>(TR, X, ta, ga, tb, gb, c, ovf, sp, sp, emit);
    }
    return;
  }
  if constexpr (Emit::kCount) c.n_seg += l > 0;
  emit(P, (double)rP.alpha, (double)l, (double)ta, ga, (double)tb, gb, -1.0);
}

// The sink's bucket and where its ancestors are kept: depths <= dpre are
// shared by the wave (LDS `pre`), the deepest ks depths above the bucket sit
// in the lane's LDS window (stride 64; slot = depth - depthS + ks), and the
// rare depths in between are found again by descending from the shared part.
struct SinkCtx {
  int S;
  uint64_t keyS;
  int depthS;
  double alphaS;
  double spreadS;  // the bucket's particle spread (particle-trace kernel), else 0
  uint64_t axm[3];  // the box's split axis masks over path-bit positions
  int root;
  int dpre;
  int ks;
  const int32_t *pre;
  int32_t *win;
};

template <typename T>
__device__ __forceinline__ int sink_anc(const TraceRecT<T> *__restrict__ TR, const SinkCtx &sk,
                                        int dd) {
  if (dd <= sk.dpre) return ((const lds_i32 *)sk.pre)[dd];
  const int slot = dd - sk.depthS + sk.ks;
  if (slot >= 0) return ((const lds_i32 *)sk.win)[slot * kWave];
  int node = sk.dpre >= 0 ? ((const lds_i32 *)sk.pre)[sk.dpre] : sk.root;
  for (int j = sk.dpre > 0 ? sk.dpre : 0; j < dd; ++j)
    node = ((sk.keyS >> (62 - j)) & 1) ? rax_right(load_tr(TR, node).right_ax) : node + 1;
  return node;
}

template <typename G>
__device__ __forceinline__ void ray_setup(RayCtx<G> &c, G y0, G y1, G y2) {
  c.d[0] = y0 - c.xi[0];
  c.d[1] = y1 - c.xi[1];
  c.d[2] = y2 - c.xi[2];
  // 1/d_a, and -infinity where the ray is parallel to the axis's planes: the
  // refinement step's crossing is then -inf, +inf or NaN (sink below, above
  // or on the plane) and its comparisons send the whole interval to the
  // child on the sink's side, the upper one on the plane
  for (int q = 0; q < 3; ++q) c.inv[q] = c.d[q] != G(0) ? G(1) / c.d[q] : -G(INFINITY);
  c.r2 = (c.d[0] * c.d[0] + c.d[1] * c.d[1]) + c.d[2] * c.d[2];
  c.r = sqrt(c.r2);
  c.pm = 0;
  for (int q = 0; q < 3; ++q)
    c.pm |= (c.d[q] == G(0) ? 1 << q : 0) | (c.d[q] <= G(0) ? 16 << q : 0);
}

// Reverse ray trace from the sink (t = 0) to the source in cell C (t = 1),
// handing every piece to `emit` in a fixed order: sink chain (from the
// meeting cell down), the sink's bucket, source chain, the source cell.
template <typename T, typename Emit>
__device__ void trace_pieces(const FluxArgs<T> &a, int C, uint64_t keyC, int depthC,
                             const SinkCtx &sk, RayCtx<T> &c, Emit &emit) {
  if (C == sk.S) {
    if constexpr (Emit::kCount) c.n_trace++;
    const T l = c.r * (T(1) - T(0));
    if constexpr (Emit::kCount) c.n_seg += l > 0;
    emit(sk.S, sk.alphaS, (double)l, 0.0, -1, 1.0, -1, sk.spreadS);
    return;
  }
  StackSpill<T> ovf;
  int sp = 0;  // deferred refinement jobs on the lane's stack
  const int ad = __clzll((long long)(sk.keyS ^ keyC)) - 1;  // depth of the meeting cell
  const int A = sink_anc<T>(a.TR, sk, ad);
  if constexpr (Emit::kVar) {
    if (a.ray_mode == 1) {  // top down: the meeting cell holds the whole ray
      refine<T>(a.TR, A, T(0), -1, T(1), -1, c, ovf, 0, 0, emit);
      return;
    }
  }
  const TraceRecT<T> rA = load_tr(a.TR, A);
  const int axA = rax_axis(rA.right_ax);
  const int sr = (int)((sk.keyS >> (62 - ad)) & 1);
  const T dA = sel3(c.d, axA);
  T tA;
  int gA = -1;
  if (dA != T(0)) {
    tA = (rA.split - sel3(c.xi, axA)) * sel3(c.inv, axA);
    gA = axA;
    if (tA < T(0)) {
      tA = T(0);
      gA = -1;
    }
    if (tA > T(1)) {
      tA = T(1);
      gA = -1;
    }
  } else {
    tA = sr ? T(1) : T(0);  // ray in the plane: it belongs to the upper side
  }
  // Chain levels where the ray crosses into (sink side) or arrives from
  // (source side) the other half.  The split axis depends on the depth only,
  // so per axis a mask of path-bit positions (bit 62 - depth) selects them:
  // moving up axis a the other half of a lower-half sink chain is upper, etc.
  uint64_t mS = 0, mC = 0;
  for (int q = 0; q < 3; ++q) {
    const uint64_t axm = sk.axm[q];
    if (c.d[q] > T(0)) {
      mS |= axm & ~sk.keyS;
      mC |= axm & keyC;
    } else if (c.d[q] < T(0)) {
      mS |= axm & sk.keyS;
      mC |= axm & ~keyC;
    }
  }
  // depths ad+1 .. depth-1 are path-bit positions 63-depth .. 61-ad
  const uint64_t below_A = (1ull << (62 - ad)) - 1;
  mS &= below_A & ~((1ull << (63 - sk.depthS)) - 1);
  mC &= below_A & ~((1ull << (63 - depthC)) - 1);
  // sink side, [0, tP], shallowest level first
  T tP = tA;
  int gP = gA;
  while (mS) {
    if constexpr (Emit::kVar)
      if (emit.stop()) return;
    const int pos = 63 - __clzll((long long)mS);
    mS &= ~(1ull << pos);
    const int dd = 62 - pos;
    const int P = sink_anc<T>(a.TR, sk, dd);
    const TraceRecT<T> rP = load_tr(a.TR, P);
    const int b = (int)((sk.keyS >> (62 - dd)) & 1);
    const int ax = rax_axis(rP.right_ax);
    T tc = (rP.split - sel3(c.xi, ax)) * sel3(c.inv, ax);
    int gc = ax;
    if (tc < T(0)) {
      tc = T(0);
      gc = -1;
    }
    if (tc < tP) {
      const int sib = b ? P + 1 : rax_right(rP.right_ax);
      chain_piece<T>(a.TR, rP, P, sib, tc, gc, tP, gP, c, ovf, sp, emit);
      tP = tc;
      gP = gc;
    }
  }
  {
    if constexpr (Emit::kCount) c.n_trace++;
    const T l = c.r * (tP - T(0));
    if constexpr (Emit::kCount) c.n_seg += l > 0;
    emit(sk.S, sk.alphaS, (double)l, 0.0, -1, (double)tP, gP, sk.spreadS);
  }
  // source side, [tQ, 1]: C's ancestors below A are found walking down from
  // A along C's path bits.  A lower child is the next cell in depth-first
  // order, so only the levels where the path turns to the upper child, or
  // where the ray crosses, need their record.
  T tQ = tA;
  int gQ = gA;
  uint64_t stops = (keyC & below_A & ~((1ull << (63 - depthC)) - 1)) | mC;
  int Q = ((keyC >> (62 - ad)) & 1) ? rax_right(rA.right_ax) : A + 1;  // at depth ad + 1
  int dq = ad + 1;
  while (stops) {
    if constexpr (Emit::kVar)
      if (emit.stop()) return;
    const int pos = 63 - __clzll((long long)stops);
    stops &= ~(1ull << pos);
    const int dd = 62 - pos;
    Q += dd - dq;  // lower children in between
    const TraceRecT<T> rQ = load_tr(a.TR, Q);
    const int b = (int)((keyC >> (62 - dd)) & 1);
    if ((mC >> pos) & 1) {
      const int ax = rax_axis(rQ.right_ax);
      T tc = (rQ.split - sel3(c.xi, ax)) * sel3(c.inv, ax);
      int gc = ax;
      if (tc > T(1)) {
        tc = T(1);
        gc = -1;
      }
      if (tc > tQ) {
        const int sib = b ? Q + 1 : rax_right(rQ.right_ax);
        chain_piece<T>(a.TR, rQ, Q, sib, tQ, gQ, tc, gc, c, ovf, sp, emit);
        tQ = tc;
        gQ = gc;
      }
    }
    Q = b ? rax_right(rQ.right_ax) : Q + 1;
    dq = dd + 1;
  }
  if constexpr (Emit::kVar)
    if (emit.stop()) return;
  int X0 = C, ga0 = gQ, gb0 = -1;
  T ta0 = tQ, tb0 = T(1);
  if (!(T(1) > tQ)) {
    // The source point lies on the meeting cell's plane, so C's interval is
    // empty.  C's steps are taken here (each counted; a zero-length piece at
    // the first cell that does not split; a plane parallel to the ray passes
    // the interval to the child on the sink's side, the upper one on the
    // plane), and the refinement starts from the top job instead, with the
    // rest of the jobs under it.  Refinement thus only ever sees non-empty
    // intervals, which the parallel-plane form of its step relies on.
    for (int X = C;;) {  // a plane parallel to the ray passes the interval to one child
      const TraceRecT<T> rX = load_tr(a.TR, X);
      if constexpr (Emit::kCount) c.n_trace++;
      const int right = rax_right(rX.right_ax);
      if (!((right != 0) & ((double)rX.dalpha * 0.0 > c.tau_ref))) {
        emit(X, (double)rX.alpha, 0.0, (double)tQ, gQ, 1.0, -1,
             right == 0 ? (double)rX.dalpha : -1.0);
        break;
      }
      const int ax = rax_axis(rX.right_ax);
      if (!((c.pm >> ax) & 1)) break;  // a crossing plane: both parts are empty
      X = sel3(c.xi, ax) >= rX.split ? right : X + 1;
    }
    if (sp == 0) return;
    int mark;
    stack_pop(c, ovf, --sp, mark, ga0, ta0);  // the job's marker: its entry
    stack_pop(c, ovf, --sp, X0, gb0, tb0);    // its cell and exit
  }
  refine<T>(a.TR, X0, ta0, ga0, tb0, gb0, c, ovf, sp, 0, emit);
}

__device__ __forceinline__ int wave_take(int32_t *queue, int n_chunks) {
  // contiguous range per XCD, then steal from the following ranges
  const int x0 = (int)(blockIdx.x % kXcd);
  const int per = (n_chunks + kXcd - 1) / kXcd;
  for (int k = 0; k < kXcd; ++k) {
    const int x = (x0 + k) % kXcd;
    const int lo = x * per;
    const int hi = min(n_chunks, lo + per);
    if (lo >= hi) continue;
    int got = 0;
    if ((threadIdx.x & 63) == 0) got = atomicAdd(&queue[x], 1);
    got = __shfl(got, 0);
    if (lo + got < hi) return lo + got;
  }
  return -1;
}

// LDS per wave, 8-byte items first: open masks (64 x u64), the adjoint's
// table (hn x (f64 + i32)), the refinement stacks (kr entries x 64 lanes; an
// entry is 8 bytes for binary32, f64 + i32 for binary64), the ray queue
// (kQueue x (i32 + u8)), the per-sink counts of traced pieces and steps
// (2 x 64 x i32, a forward that keeps counters), the sink-ancestor windows
// (ks x 64 lanes x i32) and the shared sink-chain prefix (kPre x i32).  The
// adjoint's replay instance (ADJ with TAPE) walks no tree: it has no open
// masks, and its queue holds one round.
constexpr int kQueue = 128;       // ray queue slots per wave (a power of two)
// Depths of the wave-shared sink-chain prefix: deeper shared levels (trees
// deeper than the headline's 29) are found by descending from its last one.
constexpr int kPre = 32;
constexpr int kQueueReplay = 64;  // the same in the replay instance
template <bool ADJ, typename T, bool CNT = true, bool TAPE = false>
__host__ __device__ constexpr size_t lds_per_wave(int ks, int kr, int hn) {
  return (ADJ && TAPE ? 0 : (size_t)64 * 8) + (ADJ ? (size_t)hn * 12 : 0) +
         (size_t)kr * 64 * (sizeof(T) == 4 ? 8 : 12) +
         (size_t)(ADJ && TAPE ? kQueueReplay : kQueue) * 5 + (ADJ || !CNT ? 0 : 2 * 64 * 4) +
         (size_t)ks * 64 * 4 + kPre * 4;
}

// Window depth, stack entries and table slots per occupancy variant (waves
// per SIMD), chosen so that that many waves fit the CU's 160 KiB of LDS.  The
// adjoint spends its LDS on the table first: a round's rays touch about 175
// distinct cells at the headline workload, and a table much under that
// sends most pieces to device-memory atomics.
__host__ __device__ constexpr int occ_ks(int wps, bool adj, bool f32) {
  if (wps <= 3) return adj ? (f32 ? 3 : 2) : (f32 ? 6 : 14);
  // binary32 4-wave forward: the prefix's freed 128 bytes and the slack make
  // a 5th window level (173.1 -> 171.9 ms at the headline, 15 stack entries)
  if (wps == 4) return adj ? 3 : (f32 ? 5 : 4);
  if (wps == 5) return adj ? 3 : 5;
  return wps <= 7 ? (adj ? (f32 ? 3 : 4) : 3) : (adj ? 3 : 2);
}
__host__ __device__ constexpr int occ_kr(int wps, bool adj, bool f32, bool cnt) {
  if (f32) {
    if (wps <= 3) return adj ? 16 : cnt ? 19 : 20;
    if (wps == 4) return adj ? 12 : cnt ? 14 : 15;  // one more without the per-sink counts
    if (wps == 5) return adj ? 8 : 9;
    return wps <= 7 ? 7 : 4;
  }
  if (wps <= 3) return adj ? 11 : 10;
  if (wps == 4) return adj ? 8 : 9;
  if (wps == 5) return adj ? 5 : 6;
  return wps <= 7 ? (adj ? 4 : 5) : (adj ? 2 : 3);
}
// adjoint: slots of the per-wave table of d loss / d alpha (a power of two)
__host__ __device__ constexpr int occ_hn(int wps, bool adj) {
  return !adj ? 0 : wps <= 3 ? 256 : wps <= 5 ? 128 : 64;
}
// The replay instance spends the walk's LDS (open masks, half the queue:
// 832 bytes), as measured for the taped adjoint at 2^20: at 4 waves per SIMD
// on two more stack entries (one in binary64), 117.9 -> 113.1 ms against
// three more window levels; elsewhere on three more window levels (768
// bytes), at 3 waves 113.5 -> 110.8 ms, where a 17th stack entry and a 4th
// level gave 111.8 ms.
__host__ __device__ constexpr int occ_ks_t(int wps, bool adj, bool f32, bool tape) {
  return occ_ks(wps, adj, f32) + (adj && tape && wps != 4 ? 3 : 0);
}
__host__ __device__ constexpr int occ_kr_t(int wps, bool adj, bool f32, bool cnt, bool tape) {
  return occ_kr(wps, adj, f32, cnt) + (adj && tape && wps == 4 ? (f32 ? 2 : 1) : 0);
}
template <bool ADJ, typename T, bool CNT, bool TAPE = false>
__host__ __device__ constexpr size_t occ_lds(int wps) {
  constexpr bool f32 = sizeof(T) == 4;
  return lds_per_wave<ADJ, T, CNT, TAPE>(occ_ks_t(wps, ADJ, f32, TAPE),
                                         occ_kr_t(wps, ADJ, f32, CNT, TAPE), occ_hn(wps, ADJ));
}
constexpr size_t kLdsPerCu = 160 * 1024;
// wps workgroups of 4 waves per CU.  A workgroup's LDS is taken in granules:
// measured at 3 workgroups per CU, 4 x 13,440 bytes fit and 4 x 13,504 did
// not; at 4, 4 x 10,240 fit.  A 2,560-byte granule fits every measured case.
constexpr size_t kLdsGranule = 2560;
constexpr bool lds_fits(size_t per_wave, int wps) {
  return (per_wave * 4 + kLdsGranule - 1) / kLdsGranule * kLdsGranule * wps <= kLdsPerCu;
}
template <typename T>
constexpr bool occ_fits(int wps) {
  return lds_fits(occ_lds<false, T, true>(wps), wps) &&
         lds_fits(occ_lds<false, T, false>(wps), wps) &&
         lds_fits(occ_lds<true, T, false>(wps), wps) &&
         lds_fits(occ_lds<true, T, false, true>(wps), wps);
}
static_assert(occ_fits<float>(3) && occ_fits<float>(4) && occ_fits<float>(5) &&
                  occ_fits<float>(6) && occ_fits<float>(8), "");
static_assert(occ_fits<double>(3) && occ_fits<double>(4) && occ_fits<double>(5) &&
                  occ_fits<double>(6) && occ_fits<double>(8), "");

constexpr uint32_t kQParticle = 0x80000000u;  // queue entry: a particle source, not a cell

// The source walk of 64 sinks, one per lane, shared by the wave (Sec. 2.2.1).
// The rays it produces go, in walk order, into one queue per wave: at each
// visited cell the accepting sinks' rays (in lane order), then for an opened
// bucket each (sink, particle) pair (particle-major).  Whenever 64 rays are
// queued they are traced as one round, one ray per lane, and what is left at
// the end of a box is traced in shorter rounds.  Rays of consecutive cells are
// alike, so a round's lanes run for similar times.  A tracing lane takes the
// owning sink's context by lane shuffles; each owner adds its results in
// queue order, so a sink's sum is in its own walk order whatever the other
// sinks of the wave are.
// TAPE: the tape's instances.  In the forward, the recording flux (tape mode
// 1), so that the plain flux carries none of the tape's code; in the adjoint,
// the replay of a complete recording (tape mode 2), which walks no tree.
template <typename T, bool ADJ, int KS, int KR, int HN, int MOM = 0, int NBND = 0, int SPH = 0,
          int VAR = 0, bool CNT = true, bool TAPE = false>
__device__ __forceinline__ void walk_body(const FluxArgs<T> &a) {
  constexpr bool REC = !ADJ && TAPE;
  constexpr bool RPL = ADJ && TAPE;
  constexpr int QN = RPL ? kQueueReplay : kQueue;
  // The adjoint from a tape is launched as a pair: the replay instance runs
  // when the recording is complete, the walking one (which traces each ray
  // twice) when it is not, and each returns at once in the other case.
  if constexpr (ADJ)
    if (a.tape_mode == 2 && (*a.tape_ctr <= a.tape_cap) != RPL) return;
  extern __shared__ unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1;  // the lanes below this one
  unsigned char *base = smem + wv * lds_per_wave<ADJ, T, CNT, TAPE>(KS, KR, HN);
  uint64_t *s_open = reinterpret_cast<uint64_t *>(base);
  if (!RPL) base += 64 * 8;
  double *s_hv = reinterpret_cast<double *>(base);  // adjoint table: sums, then keys
  if (ADJ) base += HN * 8;
  int32_t *s_hk = reinterpret_cast<int32_t *>(base);
  if (ADJ) base += HN * 4;
  double *s_stb = reinterpret_cast<double *>(base);  // the stack: 8-byte entries or t ...
  base += KR * 64 * 8;
  int32_t *s_stn = reinterpret_cast<int32_t *>(base);  // ... and cells (binary64)
  if (sizeof(T) == 8) base += KR * 64 * 4;
  lds_i32 *s_qe = (lds_i32 *)reinterpret_cast<int32_t *>(base);  // entry: cell or particle
  base += QN * 4;
  int32_t *s_cnt = reinterpret_cast<int32_t *>(base);  // forward: pieces, steps per sink
  if (!ADJ && CNT) base += 2 * 64 * 4;
  int32_t *s_anc = reinterpret_cast<int32_t *>(base);
  base += KS * 64 * 4;
  int32_t *s_pre = reinterpret_cast<int32_t *>(base);
  uint8_t *s_qo = reinterpret_cast<uint8_t *>(s_pre + kPre);  // entry's owning lane
  if (ADJ) {
    for (int j = lane; j < HN; j += 64) {
      s_hk[j] = -1;
      s_hv[j] = 0.0;
    }
  }
  RayCtx<T> c;
  c.tau_ref = a.tau_ref;
  c.stn = s_stn + lane;
  c.stb = s_stb + lane;
  c.st = reinterpret_cast<uint64_t *>(s_stb) + lane;
  c.kr = KR;
  constexpr bool replay = RPL;  // rounds from the recording's ray lists
  int chunk = -1, sub = a.group;
  int tc_next = 0, tc_end = 0;  // recording: the wave's blocks not yet used
  for (;;) {
    if (sub == a.group) {
      chunk = wave_take(a.queue, a.n_chunks);
      if (chunk < 0) break;
      sub = 0;
    }
    const int64_t set = (int64_t)chunk * a.group + sub;  // the 64-sink set
    const int64_t q = ((int64_t)chunk * a.group + sub++) * 64 + lane;
    if (__ballot(q < a.n_sinks) == 0) {
      sub = a.group;
      continue;
    }
    const bool in_list = q < a.n_sinks;
    bool bad = false;  // a sink index outside [0, n)
    int k = 0;
    if (in_list) {
      if (a.sinks) {
        const int32_t si = a.sinks[q];
        bad = si < 0 || (int64_t)si >= a.n;
        if (!bad) k = a.inv[si];
      } else {
        k = (int)q;
      }
    }
    const bool valid = in_list && !bad;
    // this lane's sink: it owns the opening tests and the sums of its rays
    const P4<T> me = a.ps[k];
    const double xo[3] = {(double)me.x, (double)me.y, (double)me.z};
    SinkCtx sk;
    sk.S = a.leaf[k];
    sk.keyS = a.key[sk.S];
    sk.depthS = a.ndepth[sk.S];
    sk.alphaS = (double)a.TR[sk.S].alpha;
    double bb_lo[3] = {0.0, 0.0, 0.0}, bb_hi[3] = {0.0, 0.0, 0.0};  // (VAR) the bucket's box
    if (VAR > 0) {
      const WalkRecT<T> &wb = a.W[sk.S];
      for (int q3 = 0; q3 < 3; ++q3) {
        bb_lo[q3] = (double)wb.lo[q3];
        bb_hi[q3] = (double)wb.hi[q3];
      }
    }
    sk.spreadS = SPH > 0 ? (double)a.TR[sk.S].dalpha : 0.0;
    const int my_box = a.pbox[k];
    const int my_root = a.box_root[my_box];
    sk.axm[0] = a.axmask[3 * my_box + 0];
    sk.axm[1] = a.axmask[3 * my_box + 1];
    sk.axm[2] = a.axmask[3 * my_box + 2];
    const uint64_t vmask = __ballot(valid);
    const int lead0 = vmask ? __ffsll((unsigned long long)vmask) - 1 : 0;
    // Sink-chain depths whose cell is the same for every valid lane: same box
    // and path bits above that depth, and not below any lane's bucket.
    int d_common;
    {
      const uint64_t keyL = __shfl(sk.keyS, lead0);
      const int rootL = __shfl(my_root, lead0);
      int dc = kDmax;
      if (valid) {
        const uint64_t x = sk.keyS ^ keyL;
        dc = x ? __clzll((long long)x) - 1 : kDmax;
        if (sk.depthS < dc) dc = sk.depthS;
        if (my_root != rootL) dc = -1;
      }
      for (int o = 32; o > 0; o >>= 1) {
        const int other = __shfl_xor(dc, o);
        dc = other < dc ? other : dc;
      }
      d_common = vmask ? (dc < kPre - 1 ? dc : kPre - 1) : -1;
    }
    sk.root = my_root;
    sk.dpre = d_common;
    sk.ks = KS;
    sk.pre = s_pre;
    sk.win = s_anc + lane;
    {  // the ancestors of the sink's bucket, by depth, into the LDS tables
      int node = my_root;
      for (int dd = 0; dd <= sk.depthS; ++dd) {
        if (dd <= d_common && lane == lead0) s_pre[dd] = node;
        if (dd == sk.depthS) break;
        const int slot = dd - sk.depthS + KS;
        if (slot >= 0) sk.win[slot * kWave] = node;
        const int right = rax_right(load_tr(a.TR, node).right_ax);
        node = ((sk.keyS >> (62 - dd)) & 1) ? right : node + 1;
      }
    }
    if (!ADJ && CNT) {
      s_cnt[lane] = 0;
      s_cnt[64 + lane] = 0;
    }
    wave_sync();
    double wgt = 0.0;
    // grad_flux is indexed like flux: by list position, or by particle
    if (ADJ && valid) wgt = (double)a.grad_flux[a.sinks ? q : (int64_t)a.perm[k]];
    double F = 0.0;
    double FV[3] = {0.0, 0.0, 0.0};            // vector flux (MOM >= 1)
    double FP[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // second moment (MOM == 2)
    double FB[kMaxBands] = {0.0, 0.0, 0.0, 0.0};      // flux per band (NBND > 0)
    int n_open = 0, n_rays = 0, n_psrc = 0;
    int qh = 0, qn = 0;  // the queue: first entry, entries (wave-uniform)
    int tprev = -1;      // recording: the set's last block
    int tcur = -1;       // replay: the set's next block
    if (REC && lane == 0) a.tape_head[set] = -1;
    if (replay) tcur = a.tape_head[set];

    // One round: the first min(qn, 64) queued rays, one per lane.
    auto round = [&]() {
      wave_sync();
      const int nb = qn < 64 ? qn : 64;
      const bool busy = lane < nb;
      uint32_t e = 0;
      int owner = 0;
      if (busy) {
        const int slot = (qh + lane) & (QN - 1);
        e = (uint32_t)s_qe[slot];
        owner = s_qo[slot];
      }
      qh = (qh + nb) & (QN - 1);
      qn -= nb;
      // the owner's sink
      const T ox = __shfl(me.x, owner), oy = __shfl(me.y, owner), oz = __shfl(me.z, owner);
      SinkCtx tk;
      tk.S = __shfl(sk.S, owner);
      tk.keyS = __shfl(sk.keyS, owner);
      tk.depthS = __shfl(sk.depthS, owner);
      tk.alphaS = __shfl(sk.alphaS, owner);
      tk.spreadS = SPH > 0 ? __shfl(sk.spreadS, owner) : 0.0;
      tk.axm[0] = __shfl(sk.axm[0], owner);
      tk.axm[1] = __shfl(sk.axm[1], owner);
      tk.axm[2] = __shfl(sk.axm[2], owner);
      tk.root = __shfl(sk.root, owner);
      tk.dpre = d_common;
      tk.ks = KS;
      tk.pre = s_pre;
      tk.win = s_anc + owner;
      const double wg = ADJ ? __shfl(wgt, owner) : 0.0;
      const int self_k = SPH > 0 ? __shfl(k, owner) : 0;  // the receiving particle
      double f = 0.0;
      double fv[3] = {0.0, 0.0, 0.0};  // f along the ray's direction of travel n
      double fp[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // f n_a n_b
      double fb[kMaxBands] = {0.0, 0.0, 0.0, 0.0};      // f per band
      int tblk = -1;     // this round's tape block
      bool rp = false;   // tau from the tape
      if constexpr (REC) {
        // Blocks come from one counter, tape_chunk at a time per wave, so
        // that few atomics meet on it; the numbers a wave takes increase (the
        // wave's last unused ones are left over).
        if (tc_next == tc_end) {
          int c0 = 0;
          if (lane == 0) c0 = atomicAdd(a.tape_ctr, a.tape_chunk);
          tc_next = __builtin_amdgcn_readfirstlane(c0);
          tc_end = tc_next + a.tape_chunk;
        }
        const int b = tc_next++;
        if (b < a.tape_cap) {  // blocks come in increasing order, so a full tape stays full
          if (lane == 0) {
            if (tprev < 0)
              a.tape_head[set] = b;
            else
              a.tape_next[tprev] = b;
            a.tape_next[b] = -1;
          }
          tblk = b;
        }
        tprev = b;
      }
      double tau_rec = 0.0;
      // adjoint: the ray's terms for its source (d loss / d L, and d loss / d x_L
      // of a cell), summed over the round's rays of one source before the atomics
      double sv[4] = {0.0, 0.0, 0.0, 0.0};
      if (replay && tcur >= 0) {
        rp = true;
        tblk = tcur;
        if (busy) tau_rec = a.tape[(int64_t)tblk * 64 + lane];
        tcur = a.tape_next[tblk];
      }
      SphSum<T, CNT> ss;  // (SPH) the particle trace, with its jobs for the wave
      double sph_L = 0.0;
      ss.off = a.sph_off;
      ss.nb = a.sph_nb;
      ss.pos = a.sph_pos;
      ss.mk = a.sph_mk;
      if (busy) {
        const bool psrc = (e & kQParticle) != 0;
        const int id = (int)(e & ~kQParticle);
        int C;
        T yx, yy, yz, L;
        if (psrc) {
          const P4<T> pj = a.ps[id];
          C = a.leaf[id];
          yx = pj.x;
          yy = pj.y;
          yz = pj.z;
          L = pj.L;
        } else {
          C = id;
          yx = a.W[id].xl[0];
          yy = a.W[id].xl[1];
          yz = a.W[id].xl[2];
          L = a.W[id].L;
        }
        const uint64_t keyC = a.key[C];
        const int depthC = a.ndepth[C];
        c.xi[0] = ox;
        c.xi[1] = oy;
        c.xi[2] = oz;
        c.n_seg = 0;
        c.n_trace = 0;
        ray_setup(c, yx, yy, yz);
        std::conditional_t<ADJ, TauSumA, std::conditional_t<CNT, TauSum, TauSumNC>> ts;
        if constexpr (SPH > 0) {  // particle trace below the buckets
          ss.c = &c;
          ss.tau_ref = c.tau_ref;
          ss.self = self_k;
          trace_pieces<T>(a, C, keyC, depthC, tk, c, ss);
          ts.tau = ss.tau;
          sph_L = (double)L;
        } else if constexpr (NBND > 0) {  // one traversal, one tau per band
          BandSum<T, CNT> bsum;
          bsum.ba = a.band_alpha;
          bsum.nb = a.n_bands;
          trace_pieces<T>(a, C, keyC, depthC, tk, c, bsum);
          for (int b = 0; b < kMaxBands; ++b)
            if (b < a.n_bands)
              fb[b] = ((double)L * exp(-bsum.tau[b])) / ((4.0 * M_PI) * (double)c.r2);
        } else if constexpr (VAR > 0) {  // walk variants, with the early stop
          TauVar<CNT> tv;
          tv.tau_max = a.tau_max;
          trace_pieces<T>(a, C, keyC, depthC, tk, c, tv);
          ts.tau = tv.tau;
        } else if (rp) {
          ts.tau = tau_rec;
        } else {
          trace_pieces<T>(a, C, keyC, depthC, tk, c, ts);
        }
        if (REC && tblk >= 0) {  // lane 0 is busy in every round
          const int64_t r = (int64_t)tblk * 64 + lane;
          a.tape[r] = ts.tau;
          a.tape_src[r] = e;
          a.tape_own[r] = (uint8_t)owner;
          if (lane == 0) a.tape_nb[tblk] = (uint8_t)nb;
        }
        f = ((double)L * exp(-ts.tau)) / ((4.0 * M_PI) * (double)c.r2);
        if constexpr (VAR > 0) {
          if (a.bg_pos && !psrc) {  // a merged background cell radiates from the sphere
            const P4<T> b = a.bg_pos[id];
            if (b.L != (T)0) {
              const double e0 = (double)b.x - (double)c.xi[0],
                           e1 = (double)b.y - (double)c.xi[1],
                           e2 = (double)b.z - (double)c.xi[2];
              const double r2f = (e0 * e0 + e1 * e1) + e2 * e2;
              f = ((double)L * exp(-ts.tau)) / ((4.0 * M_PI) * r2f);
            }
          }
          if (ts.tau > a.tau_max) f = 0.0;  // early termination
        }
        if (MOM >= 1) {
          double nv[3];
          for (int q3 = 0; q3 < 3; ++q3) {
            nv[q3] = -(double)c.d[q3] / (double)c.r;
            fv[q3] = f * nv[q3];
          }
          if (MOM == 2) {
            fp[0] = f * (nv[0] * nv[0]);
            fp[1] = f * (nv[1] * nv[1]);
            fp[2] = f * (nv[2] * nv[2]);
            fp[3] = f * (nv[0] * nv[1]);
            fp[4] = f * (nv[0] * nv[2]);
            fp[5] = f * (nv[1] * nv[2]);
          }
        }
        if (!ADJ) {
          if (CNT) {
            __hip_atomic_fetch_add(&s_cnt[owner], c.n_seg, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WAVEFRONT);
            __hip_atomic_fetch_add(&s_cnt[64 + owner], c.n_trace, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WAVEFRONT);
          }
        } else {
          Scatter sc;
          sc.g = wg * f;
          for (int q3 = 0; q3 < 3; ++q3)
            sc.dtdy[q3] = psrc ? 0.0 : (ts.tau / (double)c.r) * ((double)c.d[q3] / (double)c.r);
          sc.r = (double)c.r;
          sc.inv[0] = (double)c.inv[0];
          sc.inv[1] = (double)c.inv[1];
          sc.inv[2] = (double)c.inv[2];
          sc.abar = a.abar;
          sc.hk = s_hk;
          sc.hv = s_hv;
          sc.hmask = HN - 1;
          sc.u[0] = sc.u[1] = sc.u[2] = 0.0;
          trace_pieces<T>(a, C, keyC, depthC, tk, c, sc);
          for (int q3 = 0; q3 < 3; ++q3)  // no crossings (u = 0) along an axis with d = 0
            if (!((c.pm >> q3) & 1)) sc.dtdy[q3] += (double)c.r * (double)c.inv[q3] * sc.u[q3];
          sv[0] = sc.g / (double)L;  // d loss / d L of the source
          if (!psrc)                 // d loss / d x_L of the cell
            for (int q3 = 0; q3 < 3; ++q3)
              sv[1 + q3] = sc.g * (-2.0 * (double)c.d[q3] / (double)c.r2 - sc.dtdy[q3]);
        }
      }
      if constexpr (SPH > 0) {  // the round's particle-trace jobs, by the whole wave
        const bool had = ss.nj > 0;
        static_assert(SPH == 0 || KR * 64 * 8 >= kSphBuf * 4, "job buffer in the stack's LDS");
        sph_jobs<T, CNT>(ss, c, lane, reinterpret_cast<int32_t *>(s_stb));
        if (had) f = (sph_L * exp(-ss.tau)) / ((4.0 * M_PI) * (double)c.r2);
      }
      if (ADJ) {
        // Rays of one source are adjacent in the queue (a visited cell's
        // accepting sinks; an opened bucket's particle, sink by sink), so the
        // round's lanes form runs of one source: a segmented sum over each
        // run, then one set of device atomics per run.
        const uint32_t key = busy ? e : 0xffffffffu;
        const uint32_t prev = __shfl_up(key, 1);
        const bool head = lane == 0 || prev != key;
        const uint64_t hm = __ballot(head);
        const int start = 63 - __clzll(hm & ((2ull << lane) - 1));  // the run's first lane
        for (int o = 1; o < 64; o <<= 1) {
          const bool take = lane - o >= start;
          for (int q3 = 0; q3 < 4; ++q3) {
            const double t = __shfl_up(sv[q3], o);
            if (take) sv[q3] += t;
          }
        }
        const bool tail = busy && (lane == nb - 1 || (lane < 63 && ((hm >> (lane + 1)) & 1)));
        if (tail) {
          const int id = (int)(e & ~kQParticle);
          if (e & kQParticle) {
            gbl_add(&a.direct[id], sv[0]);
          } else {
            gbl_add(&a.lbar[id], sv[0]);
            gbl_add(&a.xbar[id], sv[1]);
            gbl_add(&a.xbar[a.m + id], sv[2]);
            gbl_add(&a.xbar[2 * a.m + id], sv[3]);
          }
        }
      }
      if (ADJ) {  // write the round's table out to device memory and clear it
        wave_sync();
        for (int j = lane; j < HN; j += 64) {
          const int key = s_hk[j];
          if (key != -1) {
            gbl_add(&a.abar[key], s_hv[j]);
            s_hk[j] = -1;
            s_hv[j] = 0.0;
          }
        }
        wave_sync();
      }
      if (!ADJ) {  // each owner adds its rays' fluxes in queue order
        // Runs: stretches of lanes with strictly increasing owners (a visited
        // cell's accepting sinks, an opened bucket's particle for each opening
        // sink).  An owner has at most one ray in a run, so one forward
        // permute per run hands every ray's flux to its owner.
        const int prev_o = __shfl_up(owner, 1);
        uint64_t rs = __ballot(busy && (lane == 0 || owner <= prev_o));
        if (__popcll(rs) <= 24) {
          while (rs) {
            const int r0 = __ffsll((unsigned long long)rs) - 1;
            rs &= rs - 1;
            const int r1 = rs ? __ffsll((unsigned long long)rs) - 1 : nb;
            const bool in = lane >= r0 && lane < r1;
            // lanes outside the run push nothing useful, to lane 63
            const int to = (in ? owner : 63) * 4;
            const int hi = __builtin_amdgcn_ds_permute(to, in ? __double2hiint(f) : 0);
            const int lo = __builtin_amdgcn_ds_permute(to, in ? __double2loint(f) : 0);
            const int got = __builtin_amdgcn_ds_permute(to, in ? 1 : 0);
            double fj = __hiloint2double(hi, lo);
            double fvj[3] = {0.0, 0.0, 0.0};
            if (MOM >= 1)
              for (int q3 = 0; q3 < 3; ++q3)
                fvj[q3] = __hiloint2double(
                    __builtin_amdgcn_ds_permute(to, in ? __double2hiint(fv[q3]) : 0),
                    __builtin_amdgcn_ds_permute(to, in ? __double2loint(fv[q3]) : 0));
            double fbj[kMaxBands] = {0.0, 0.0, 0.0, 0.0};
            if (NBND > 0)
              for (int b = 0; b < kMaxBands; ++b)
                fbj[b] = __hiloint2double(
                    __builtin_amdgcn_ds_permute(to, in ? __double2hiint(fb[b]) : 0),
                    __builtin_amdgcn_ds_permute(to, in ? __double2loint(fb[b]) : 0));
            double fpj[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            if (MOM == 2)
              for (int q6 = 0; q6 < 6; ++q6)
                fpj[q6] = __hiloint2double(
                    __builtin_amdgcn_ds_permute(to, in ? __double2hiint(fp[q6]) : 0),
                    __builtin_amdgcn_ds_permute(to, in ? __double2loint(fp[q6]) : 0));
            bool has = got != 0;
            // a later lane outside the run can overwrite lane 63's value
            const uint64_t m63 = __ballot(in && owner == 63);
            if (m63) {
              const int j63 = __ffsll((unsigned long long)m63) - 1;
              const double f63 =
                  __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(f), j63),
                                   __builtin_amdgcn_readlane(__double2loint(f), j63));
              if (lane == 63) {
                has = true;
                fj = f63;
              }
              if (MOM >= 1)
                for (int q3 = 0; q3 < 3; ++q3) {
                  const double v63 =
                      __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(fv[q3]), j63),
                                       __builtin_amdgcn_readlane(__double2loint(fv[q3]), j63));
                  if (lane == 63) fvj[q3] = v63;
                }
              if (NBND > 0)
                for (int b = 0; b < kMaxBands; ++b) {
                  const double v63 =
                      __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(fb[b]), j63),
                                       __builtin_amdgcn_readlane(__double2loint(fb[b]), j63));
                  if (lane == 63) fbj[b] = v63;
                }
              if (MOM == 2)
                for (int q6 = 0; q6 < 6; ++q6) {
                  const double v63 =
                      __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(fp[q6]), j63),
                                       __builtin_amdgcn_readlane(__double2loint(fp[q6]), j63));
                  if (lane == 63) fpj[q6] = v63;
                }
            }
            if (has) {
              F += fj;
              if (MOM >= 1)
                for (int q3 = 0; q3 < 3; ++q3) FV[q3] += fvj[q3];
              if (MOM == 2)
                for (int q6 = 0; q6 < 6; ++q6) FP[q6] += fpj[q6];
              if (NBND > 0)
                for (int b = 0; b < kMaxBands; ++b) FB[b] += fbj[b];
            }
          }
        } else {
          for (int j = 0; j < nb; ++j) {
            const int oj = __builtin_amdgcn_readlane(owner, j);
            const double fj =
                __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(f), j),
                                 __builtin_amdgcn_readlane(__double2loint(f), j));
            if (lane == oj) F += fj;
            if (MOM >= 1)
              for (int q3 = 0; q3 < 3; ++q3) {
                const double vj =
                    __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(fv[q3]), j),
                                     __builtin_amdgcn_readlane(__double2loint(fv[q3]), j));
                if (lane == oj) FV[q3] += vj;
              }
            if (NBND > 0)
              for (int b = 0; b < kMaxBands; ++b) {
                const double vj =
                    __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(fb[b]), j),
                                     __builtin_amdgcn_readlane(__double2loint(fb[b]), j));
                if (lane == oj) FB[b] += vj;
              }
            if (MOM == 2)
              for (int q6 = 0; q6 < 6; ++q6) {
                const double vj =
                    __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(fp[q6]), j),
                                     __builtin_amdgcn_readlane(__double2loint(fp[q6]), j));
                if (lane == oj) FP[q6] += vj;
              }
          }
        }
      }
    };

    uint64_t pending = vmask;
    while (pending) {
      const int lead = __ffsll((unsigned long long)pending) - 1;
      const int root = __shfl(my_root, lead);
      const uint64_t group = __ballot(valid && my_root == root);
      pending &= ~group;
      const int end = a.W[root].skip;
      int n = root;
      uint64_t active = group;
      bool from_skip = false;
      for (; !replay;) {  // a replay takes its rays from the tape below
        const WalkRecT<T> w = a.W[n];
        const int depth = w.depth;
        if (from_skip) active = s_open[depth - 1];
        const bool mine = (active >> lane) & 1;
        uint64_t openm = 0;
        if (w.L != (T)0) {
          bool acc = false;
          if (mine) {
            if (CNT) n_open++;
            double g[3];
            for (int q3 = 0; q3 < 3; ++q3) {
              const double u = (double)w.lo[q3] - xo[q3];
              const double v = xo[q3] - (double)w.hi[q3];
              const double gg = u > v ? u : v;
              g[q3] = gg > 0.0 ? gg : 0.0;
            }
            const double r2 = (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
            const double lf = (double)w.lfar;
            acc = lf * lf < a.theta2 * r2;
            if constexpr (VAR > 0) {
              if (a.open_mode == 1) {  // r from the sink's bucket box
                for (int q3 = 0; q3 < 3; ++q3) {
                  const double u = (double)w.lo[q3] - bb_hi[q3];
                  const double v = bb_lo[q3] - (double)w.hi[q3];
                  const double gg = u > v ? u : v;
                  g[q3] = gg > 0.0 ? gg : 0.0;
                }
                const double rb2 = (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
                acc = lf * lf < a.theta2 * rb2;
              } else if (a.open_mode == 2) {  // outside r_open about x_L, sink outside
                const double e0 = xo[0] - (double)w.xl[0], e1 = xo[1] - (double)w.xl[1],
                             e2 = xo[2] - (double)w.xl[2];
                const double d2 = (e0 * e0 + e1 * e1) + e2 * e2;
                acc = r2 > 0.0 && (3.0 * a.theta2) * d2 > 4.0 * (lf * lf);
              }
            }
          }
          const uint64_t accm = __ballot(acc);
          openm = active & ~accm;
          // queue invariant: qn < 64 here, so a visit's cell rays fit
          if (acc) {
            if (CNT) n_rays++;
            const int slot = (qh + qn + __popcll(accm & below)) & (QN - 1);
            s_qe[slot] = n;
            s_qo[slot] = (uint8_t)lane;
          }
          qn += __popcll(accm);
          if (qn >= 64) round();
          if (openm && rax_right(w.right_ax) == 0) {  // bucket: its particles one by one
            const bool op = (openm >> lane) & 1;
            for (int kk = w.first; kk < w.first + w.count; ++kk) {
              const P4<T> pj = a.ps[kk];
              const bool use = op && pj.L > (T)0 && kk != k &&
                               !(pj.x == me.x && pj.y == me.y && pj.z == me.z);
              const uint64_t um = __ballot(use);
              if (use) {
                if (CNT) {
                  n_rays++;
                  n_psrc++;
                }
                const int slot = (qh + qn + __popcll(um & below)) & (QN - 1);
                s_qe[slot] = (int32_t)((uint32_t)kk | kQParticle);
                s_qo[slot] = (uint8_t)lane;
              }
              qn += __popcll(um);
              if (qn >= 64) round();
            }
          }
        }
        if (openm && rax_right(w.right_ax) != 0) {
          s_open[depth] = openm;
          active = openm;
          n = n + 1;
          from_skip = false;
          continue;
        }
        n = w.skip;
        if (n >= end) break;
        from_skip = true;
      }
      // The rest of this box's rays.  A replay walks no tree: the recording's
      // rounds come back block by block from their ray lists, the same rays
      // in the same rounds and order as the recording's walk made them.
      for (;;) {
        if (replay && qn == 0 && tcur >= 0) {
          const int nbt = a.tape_nb[tcur];
          if (lane < nbt) {
            const int64_t r = (int64_t)tcur * 64 + lane;
            const int slot = (qh + lane) & (QN - 1);
            s_qe[slot] = (int32_t)a.tape_src[r];
            s_qo[slot] = a.tape_own[r];
          }
          qn = nbt;
        }
        if (qn == 0) break;
        round();
      }
    }
    if (!ADJ) {
      wave_sync();
      if (in_list) {
        const int64_t out = a.sinks ? q : (int64_t)a.perm[k];
        if (NBND == 0) a.flux[out] = bad ? (T)NAN : (T)F;  // the band kernel has no flux
        if (MOM >= 1)
          for (int q3 = 0; q3 < 3; ++q3)
            a.flux_vec[q3 * a.n_sinks + out] = bad ? (T)NAN : (T)FV[q3];
        if (MOM == 2)
          for (int q6 = 0; q6 < 6; ++q6)
            a.flux_mom[q6 * a.n_sinks + out] = bad ? (T)NAN : (T)FP[q6];
        if (NBND > 0)
          for (int b = 0; b < kMaxBands; ++b)
            if (b < a.n_bands) a.flux_bands[b * a.n_sinks + out] = bad ? (T)NAN : (T)FB[b];
        if (CNT && a.counters) {
          int32_t *o = a.counters + 5 * out;
          o[0] = bad ? -1 : n_open;
          o[1] = bad ? -1 : n_rays;
          o[2] = bad ? -1 : n_psrc;
          o[3] = bad ? -1 : s_cnt[lane];
          o[4] = bad ? -1 : s_cnt[64 + lane];
        }
      }
    }
  }
}

// The walk at the LDS split of an occupancy variant (waves per SIMD).
template <typename T, bool ADJ, int WPS, int MOM, int NBND, int SPH, int VAR, bool CNT,
          bool TAPE = false>
__device__ __forceinline__ void walk_at(const FluxArgs<T> &a) {
  constexpr bool f32 = sizeof(T) == 4;
  walk_body<T, ADJ, occ_ks_t(WPS, ADJ, f32, TAPE), occ_kr_t(WPS, ADJ, f32, CNT, TAPE),
            occ_hn(WPS, ADJ), MOM, NBND, SPH, VAR, CNT, TAPE>(a);
}

// The walk kernel at several register budgets: with fewer VGPRs more waves
// share a SIMD (better latency hiding) at the price of spills; the launch
// shape picks one (waves per SIMD = workgroups per CU x waves per workgroup
// / 4, at least 3).
template <typename T, bool ADJ, bool CNT, bool TAPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_walk(
    FluxArgs<T> a) {
  walk_at<T, ADJ, 3, 0, 0, 0, 0, CNT, TAPE>(a);
}
template <typename T, bool ADJ, bool CNT, bool TAPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_walk4(
    FluxArgs<T> a) {
  walk_at<T, ADJ, 4, 0, 0, 0, 0, CNT, TAPE>(a);
}
// The flux with the vector flux, at the 4-wave budget.
template <typename T, bool CNT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_walk4v(
    FluxArgs<T> a) {
  walk_at<T, false, 4, 1, 0, 0, 0, CNT>(a);
}
// The flux per opacity band, at the 4-wave budget.
template <typename T, bool CNT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_walk4b(
    FluxArgs<T> a) {
  walk_at<T, false, 4, 0, kMaxBands, 0, 0, CNT>(a);
}
// The flux with the walk variants, at the 4-wave budget.
template <typename T, bool CNT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_walk4x(
    FluxArgs<T> a) {
  walk_at<T, false, 4, 0, 0, 0, 1, CNT>(a);
}
// The flux with the sub-bucket particle trace, with the 3-wave LDS split at
// 2 waves per SIMD: its binary64 kernel integrals need the registers (862.6
// -> 805.3 ms at 2^21, where 2 waves made the other walk modes 36-43 %
// slower).
template <typename T, bool CNT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_walk3s(
    FluxArgs<T> a) {
  walk_at<T, false, 3, 0, 0, 1, 0, CNT>(a);
}
// The flux with the vector flux and the second moment, at the 4-wave budget.
// The band, variant and moment kernels use up to 164 VGPRs without spills at
// 3 waves per SIMD; at 4, with spills, they ran 3-14 % faster at 2^21.
template <typename T, bool CNT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_walk4m(
    FluxArgs<T> a) {
  walk_at<T, false, 4, 2, 0, 0, 0, CNT>(a);
}
template <typename T, bool ADJ, bool CNT, bool TAPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_walk5(
    FluxArgs<T> a) {
  walk_at<T, ADJ, 5, 0, 0, 0, 0, CNT, TAPE>(a);
}
template <typename T, bool ADJ, bool CNT, bool TAPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_walk6(
    FluxArgs<T> a) {
  walk_at<T, ADJ, 6, 0, 0, 0, 0, CNT, TAPE>(a);
}
template <typename T, bool ADJ, bool CNT, bool TAPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_walk8(
    FluxArgs<T> a) {
  walk_at<T, ADJ, 8, 0, 0, 0, 0, CNT, TAPE>(a);
}

__global__ void k_zero_i32(int32_t *p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_zero_f64(double *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// Totals of the per-sink counters: a grid-stride sum per thread, a wave sum,
// one 64-bit atomic per wave and counter.  Invalid sinks (-1) are skipped.
__global__ void k_zero_i64(int64_t *p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}
__global__ void k_sum_counters(const int32_t *c, int64_t n, int64_t *tot) {
  int64_t s[5] = {0, 0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (c[5 * i] >= 0)
      for (int k = 0; k < 5; ++k) s[k] += c[5 * i + k];
  for (int k = 0; k < 5; ++k) {
    for (int o = 32; o > 0; o >>= 1) s[k] += __shfl_xor(s[k], o);
    if ((threadIdx.x & 63) == 0 && s[k] != 0)
      atomicAdd((unsigned long long *)&tot[k], (unsigned long long)s[k]);
  }
}

// A cell without absorbing mass took its parent's alpha: its adjoint goes to
// the parent (one level, deepest first).
__global__ void k_adj_empty_up(const BfsNode *lvl, int cnt, const double *B,
                               const int32_t *parent, double *abar) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  const int p = lvl[j].pre;
  const int par = parent[p];
  if (par >= 0 && !(B[p] > 0)) gbl_add(&abar[par], abar[p]);
}

// Per particle: sum over the cells holding it (bucket up to the root) of
//   d alpha / d kappa_p = m_p / B,  d alpha / d rho_p = alpha m_p / (B rho_p^2),
//   d L_C / d L_p = 1,  d x_L / d L_p = (x_p - x_L) / L_C.
template <typename T>
__global__ void k_adj_particles(int64_t n, int64_t m, const int32_t *perm, const int32_t *leaf,
                                const int32_t *parent, const double *B, const double *alpha,
                                const double *lc, const double *xl, const P4<T> *ps,
                                const T *pmass, const T *prho, const double *abar,
                                const double *lbar, const double *xbar, const double *direct,
                                T *grad_rho, T *grad_kappa, T *grad_lum) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const P4<T> p = ps[k];
  const double x[3] = {(double)p.x, (double)p.y, (double)p.z};
  const double mp = (double)pmass[k], rp = (double)prho[k];
  double gk = 0.0, gr = 0.0, gl = direct[k];
  for (int id = leaf[k]; id >= 0; id = parent[id]) {
    const double Bc = B[id];
    if (Bc > 0 && mp > 0) {
      gk += abar[id] * mp / Bc;
      gr += abar[id] * alpha[id] * mp / (Bc * rp * rp);
    }
    const double L = lc[id];
    if (L > 0) {
      double dot = 0.0;
      for (int q = 0; q < 3; ++q) dot += xbar[q * m + id] * (x[q] - xl[q * m + id]);
      gl += lbar[id] + dot / L;
    }
  }
  const int i = perm[k];
  grad_rho[i] = (T)gr;
  grad_kappa[i] = (T)gk;
  grad_lum[i] = (T)gl;
}

static inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

template <typename T, bool ADJ>
static FluxArgs<T> make_args(const trevr_tree *t, double theta, double tau_ref,
                             const int32_t *sinks, int64_t n_sinks) {
  FluxArgs<T> a{};
  a.W = static_cast<const WalkRecT<T> *>(t->walk.p);
  a.TR = static_cast<const TraceRecT<T> *>(t->trace.p);
  a.key = t->key.as<uint64_t>();
  a.ndepth = t->n_depth.as<int32_t>();
  a.ps = static_cast<const P4<T> *>(t->psrc.p);
  a.perm = t->perm.as<int32_t>();
  a.inv = t->inv.as<int32_t>();
  a.leaf = t->leaf.as<int32_t>();
  a.pbox = t->pbox.as<int32_t>();
  a.box_root = t->box_root.as<int32_t>();
  a.axmask = t->axmask.as<uint64_t>();
  a.sinks = sinks;
  a.n_sinks = n_sinks;
  a.n = t->n;
  a.group = (ADJ ? t->launch_adj : t->launch).chunk / 64;
  a.n_chunks = (int32_t)((n_sinks + 64 * a.group - 1) / (64 * a.group));
  a.theta2 = theta * theta;
  a.tau_ref = tau_ref;
  a.queue = t->queue.as<int32_t>();
  a.m = t->m;
  return a;
}

// The walk kernel of an occupancy variant (waves per SIMD).
template <typename T, bool ADJ, bool CNT, bool TAPE>
static void walk_kernel(int wps, int64_t blocks, int threads, size_t shmem, const FluxArgs<T> &a,
                        hipStream_t s) {
  if (wps == 8)
    k_walk8<T, ADJ, CNT, TAPE><<<(unsigned)blocks, threads, shmem, s>>>(a);
  else if (wps == 6)
    k_walk6<T, ADJ, CNT, TAPE><<<(unsigned)blocks, threads, shmem, s>>>(a);
  else if (wps == 5)
    k_walk5<T, ADJ, CNT, TAPE><<<(unsigned)blocks, threads, shmem, s>>>(a);
  else if (wps == 4)
    k_walk4<T, ADJ, CNT, TAPE><<<(unsigned)blocks, threads, shmem, s>>>(a);
  else
    k_walk<T, ADJ, CNT, TAPE><<<(unsigned)blocks, threads, shmem, s>>>(a);
}

template <typename T, bool ADJ>
static int launch_walk(const trevr_tree *t, const FluxArgs<T> &a, hipStream_t s) {
  k_zero_i32<<<1, 64, 0, s>>>(a.queue, kXcd);
  const trevr_launch &L = ADJ ? t->launch_adj : t->launch;
  const int waves = L.waves_per_block > 4 ? 4 : L.waves_per_block;
  const int threads = 64 * waves;
  int64_t blocks = (int64_t)L.blocks_per_cu * t->num_cu;
  const int64_t need = (a.n_chunks + waves - 1) / waves;
  if (blocks > need) blocks = need;
  if constexpr (!ADJ) {
    if (a.flux_bands) {  // the bands: the 4-wave kernel, at most 4 waves per SIMD
      const int bpc = L.blocks_per_cu * waves > 16 ? 16 / waves : L.blocks_per_cu;
      int64_t vb = (int64_t)bpc * t->num_cu;
      if (vb > need) vb = need;
      if (a.counters)
        k_walk4b<T, true><<<(unsigned)vb, threads, waves * occ_lds<false, T, true>(4), s>>>(a);
      else
        k_walk4b<T, false><<<(unsigned)vb, threads, waves * occ_lds<false, T, false>(4), s>>>(a);
      TREVR_HIP(hipGetLastError());
      return TREVR_OK;
    }
    if (a.variant) {  // the walk variants: the 4-wave kernel, at most 4 waves per SIMD
      const int bpc = L.blocks_per_cu * waves > 16 ? 16 / waves : L.blocks_per_cu;
      int64_t vb = (int64_t)bpc * t->num_cu;
      if (vb > need) vb = need;
      if (a.counters)
        k_walk4x<T, true><<<(unsigned)vb, threads, waves * occ_lds<false, T, true>(4), s>>>(a);
      else
        k_walk4x<T, false><<<(unsigned)vb, threads, waves * occ_lds<false, T, false>(4), s>>>(a);
      TREVR_HIP(hipGetLastError());
      return TREVR_OK;
    }
    if (a.sph_nb) {  // the particle trace: the 2-wave kernel, at most 2 waves per SIMD
      const int bpc = L.blocks_per_cu * waves > 8 ? 8 / waves : L.blocks_per_cu;
      int64_t vb = (int64_t)bpc * t->num_cu;
      if (vb > need) vb = need;
      if (a.counters)
        k_walk3s<T, true><<<(unsigned)vb, threads, waves * occ_lds<false, T, true>(3), s>>>(a);
      else
        k_walk3s<T, false><<<(unsigned)vb, threads, waves * occ_lds<false, T, false>(3), s>>>(a);
      TREVR_HIP(hipGetLastError());
      return TREVR_OK;
    }
    if (a.flux_mom) {  // the moments: the 4-wave kernel, at most 4 waves per SIMD
      const int bpc = L.blocks_per_cu * waves > 16 ? 16 / waves : L.blocks_per_cu;
      int64_t vb = (int64_t)bpc * t->num_cu;
      if (vb > need) vb = need;
      if (a.counters)
        k_walk4m<T, true><<<(unsigned)vb, threads, waves * occ_lds<false, T, true>(4), s>>>(a);
      else
        k_walk4m<T, false><<<(unsigned)vb, threads, waves * occ_lds<false, T, false>(4), s>>>(a);
      TREVR_HIP(hipGetLastError());
      return TREVR_OK;
    }
    if (a.flux_vec) {  // the vector flux: the 4-wave kernel, at most 4 waves per SIMD
      const int bpc = L.blocks_per_cu * waves > 16 ? 16 / waves : L.blocks_per_cu;
      int64_t vb = (int64_t)bpc * t->num_cu;
      if (vb > need) vb = need;
      if (a.counters)
        k_walk4v<T, true><<<(unsigned)vb, threads, waves * occ_lds<false, T, true>(4), s>>>(a);
      else
        k_walk4v<T, false><<<(unsigned)vb, threads, waves * occ_lds<false, T, false>(4), s>>>(a);
      TREVR_HIP(hipGetLastError());
      return TREVR_OK;
    }
  }
  const int per_simd = (L.blocks_per_cu * waves + 3) / 4;
  const int wps = per_simd >= 8 ? 8 : per_simd >= 6 ? 6 : per_simd == 5 ? 5 : per_simd == 4 ? 4 : 3;
  // waves per workgroup <= 4 x wps, so the workgroup fits the CU's LDS
  // per-sink counters only when asked for (the adjoint never keeps them)
  const bool cnt = !ADJ && a.counters;
  const size_t shmem = (size_t)waves * (cnt ? occ_lds<ADJ, T, true>(wps)
                                            : occ_lds<ADJ, T, false>(wps));
  if (shmem > kLdsPerCu) return fail(TREVR_E_ARG, "launch shape needs more LDS than a CU has");
  if constexpr (ADJ) {
    if (a.tape_mode == 2) {  // the replay; the walking instance below only if it was short
      const size_t shmem_r = (size_t)waves * occ_lds<true, T, false, true>(wps);
      walk_kernel<T, true, false, true>(wps, blocks, threads, shmem_r, a, s);
      k_zero_i32<<<1, 64, 0, s>>>(a.queue, kXcd);
    }
    walk_kernel<T, true, false, false>(wps, blocks, threads, shmem, a, s);
  } else {
    const bool rec = a.tape_mode == 1;
    if (cnt && rec)
      walk_kernel<T, false, true, true>(wps, blocks, threads, shmem, a, s);
    else if (cnt)
      walk_kernel<T, false, true, false>(wps, blocks, threads, shmem, a, s);
    else if (rec)
      walk_kernel<T, false, false, true>(wps, blocks, threads, shmem, a, s);
    else
      walk_kernel<T, false, false, false>(wps, blocks, threads, shmem, a, s);
  }
  TREVR_HIP(hipGetLastError());
  return TREVR_OK;
}

// A tape of per-ray optical depths: the tree's own, or one laid out in a
// caller's scratch buffer.
struct TapeBufs {
  double *tape;     // [cap][64]
  uint32_t *src;    // [cap][64]
  uint8_t *own;     // [cap][64]
  uint8_t *nb;      // [cap]
  int32_t *next;    // [cap]
  int32_t *head;    // [64-sink sets]
  int32_t *ctr;     // blocks taken
  int64_t cap;      // blocks
};
static TapeBufs tree_tape(const trevr_tree *t) {
  return TapeBufs{t->tape.as<double>(),       t->tape_src.as<uint32_t>(),
                  t->tape_own.as<uint8_t>(),    t->tape_nb.as<uint8_t>(),
                  t->tape_next.as<int32_t>(),   t->tape_head.as<int32_t>(),
                  t->tape_ctr.as<int32_t>(),    t->tape_cap};
}

template <typename T>
static void set_tape(FluxArgs<T> &a, int mode, const TapeBufs *tb) {
  a.tape_mode = mode;
  if (mode == 0) return;
  a.tape = tb->tape;
  a.tape_src = tb->src;
  a.tape_own = tb->own;
  a.tape_nb = tb->nb;
  a.tape_next = tb->next;
  a.tape_head = tb->head;
  a.tape_ctr = tb->ctr;
  a.tape_cap = (int32_t)tb->cap;
  a.tape_chunk = 1;
}

// Blocks per counter atomic of a recording: 8 when the tape has room for
// eight left over per wave many times over (the last recording's count plus a
// quarter sizes it), else 1.
static int32_t tape_chunk(const trevr_tree *t, int64_t cap) {
  const trevr_launch &L = t->launch;
  const int64_t waves = (int64_t)t->num_cu * L.blocks_per_cu *
                        (L.waves_per_block > 4 ? 4 : L.waves_per_block);
  return cap >= 16 * 8 * waves ? 8 : 1;
}

template <typename T>
static int flux_typed(const trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
                      int64_t n_sinks, void *flux, int32_t *counters, int tape_mode,
                      const TapeBufs *tb, hipStream_t s, void *flux_vec = nullptr,
                      void *flux_mom = nullptr) {
  if (n_sinks == 0) return TREVR_OK;
  FluxArgs<T> a = make_args<T, false>(t, theta, tau_ref, sinks, n_sinks);
  a.flux = static_cast<T *>(flux);
  a.flux_vec = static_cast<T *>(flux_vec);
  a.flux_mom = static_cast<T *>(flux_mom);
  a.counters = counters;
  set_tape<T>(a, tape_mode, tb);
  if (tape_mode == 1) a.tape_chunk = tape_chunk(t, tb->cap);
  return launch_walk<T, false>(t, a, s);
}

int flux_impl(const trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
              int64_t n_sinks, void *flux, int32_t *counters, hipStream_t s) {
  if (t->prec == TREVR_F64)
    return flux_typed<double>(t, theta, tau_ref, sinks, n_sinks, flux, counters, 0, nullptr, s);
  return flux_typed<float>(t, theta, tau_ref, sinks, n_sinks, flux, counters, 0, nullptr, s);
}

template <typename T>
static int flux_bands_typed(const trevr_tree *t, double theta, double tau_ref,
                            const int32_t *sinks, int64_t n_sinks, void *flux_bands,
                            int32_t *counters, hipStream_t s) {
  if (n_sinks == 0) return TREVR_OK;
  FluxArgs<T> a = make_args<T, false>(t, theta, tau_ref, sinks, n_sinks);
  a.TR = static_cast<const TraceRecT<T> *>(t->band_trace.p);  // largest band spread
  a.band_alpha = t->band_alpha.as<T>();
  a.n_bands = t->n_bands;
  a.flux_bands = static_cast<T *>(flux_bands);
  a.counters = counters;
  return launch_walk<T, false>(t, a, s);
}

int flux_bands_impl(const trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
                    int64_t n_sinks, void *flux_bands, int32_t *counters, hipStream_t s) {
  if (t->prec == TREVR_F64)
    return flux_bands_typed<double>(t, theta, tau_ref, sinks, n_sinks, flux_bands, counters, s);
  return flux_bands_typed<float>(t, theta, tau_ref, sinks, n_sinks, flux_bands, counters, s);
}

template <typename T>
static int flux_sph_typed(const trevr_tree *t, double theta, double tau_ref,
                          const int32_t *sinks, int64_t n_sinks, void *flux, int32_t *counters,
                          hipStream_t s) {
  if (n_sinks == 0) return TREVR_OK;
  FluxArgs<T> a = make_args<T, false>(t, theta, tau_ref, sinks, n_sinks);
  a.TR = static_cast<const TraceRecT<T> *>(t->sph_trace.p);  // buckets: particle spread
  a.sph_off = t->sph_off.as<int64_t>();
  a.sph_nb = t->sph_nb.as<int32_t>();
  a.sph_pos = t->sph_pos.as<P4<T>>();
  a.sph_mk = t->sph_mk.as<double>();
  a.flux = static_cast<T *>(flux);
  a.counters = counters;
  return launch_walk<T, false>(t, a, s);
}

int flux_sph_impl(const trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
                  int64_t n_sinks, void *flux, int32_t *counters, hipStream_t s) {
  if (t->prec == TREVR_F64)
    return flux_sph_typed<double>(t, theta, tau_ref, sinks, n_sinks, flux, counters, s);
  return flux_sph_typed<float>(t, theta, tau_ref, sinks, n_sinks, flux, counters, s);
}

template <typename T>
static int flux_variant_typed(const trevr_tree *t, double theta, double tau_ref, int open_mode,
                              int ray_mode, double tau_max, const int32_t *sinks,
                              int64_t n_sinks, void *flux, int32_t *counters, hipStream_t s) {
  if (n_sinks == 0) return TREVR_OK;
  FluxArgs<T> a = make_args<T, false>(t, theta, tau_ref, sinks, n_sinks);
  a.variant = 1;
  a.open_mode = open_mode;
  a.ray_mode = ray_mode;
  a.tau_max = tau_max;
  a.flux = static_cast<T *>(flux);
  a.counters = counters;
  return launch_walk<T, false>(t, a, s);
}

int flux_variant_impl(const trevr_tree *t, double theta, double tau_ref, int open_mode,
                      int ray_mode, double tau_max, const int32_t *sinks, int64_t n_sinks,
                      void *flux, int32_t *counters, hipStream_t s) {
  if (t->prec == TREVR_F64)
    return flux_variant_typed<double>(t, theta, tau_ref, open_mode, ray_mode, tau_max, sinks,
                                      n_sinks, flux, counters, s);
  return flux_variant_typed<float>(t, theta, tau_ref, open_mode, ray_mode, tau_max, sinks,
                                   n_sinks, flux, counters, s);
}

template <typename T>
static int flux_background_typed(const trevr_tree *t, double theta, double tau_ref,
                                 const int32_t *sinks, int64_t n_sinks, void *flux,
                                 int32_t *counters, hipStream_t s) {
  if (n_sinks == 0) return TREVR_OK;
  FluxArgs<T> a = make_args<T, false>(t, theta, tau_ref, sinks, n_sinks);
  a.variant = 1;  // the variants' kernel with its default modes
  a.tau_max = INFINITY;
  a.bg_pos = static_cast<const P4<T> *>(t->bg_pos.p);
  a.flux = static_cast<T *>(flux);
  a.counters = counters;
  return launch_walk<T, false>(t, a, s);
}

int flux_background_impl(const trevr_tree *t, double theta, double tau_ref,
                         const int32_t *sinks, int64_t n_sinks, void *flux, int32_t *counters,
                         hipStream_t s) {
  if (t->prec == TREVR_F64)
    return flux_background_typed<double>(t, theta, tau_ref, sinks, n_sinks, flux, counters, s);
  return flux_background_typed<float>(t, theta, tau_ref, sinks, n_sinks, flux, counters, s);
}

int flux_vec_impl(const trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
                  int64_t n_sinks, void *flux, void *flux_vec, void *flux_mom,
                  int32_t *counters, hipStream_t s) {
  if (t->prec == TREVR_F64)
    return flux_typed<double>(t, theta, tau_ref, sinks, n_sinks, flux, counters, 0, nullptr, s,
                              flux_vec, flux_mom);
  return flux_typed<float>(t, theta, tau_ref, sinks, n_sinks, flux, counters, 0, nullptr, s,
                           flux_vec, flux_mom);
}

// Blocks for the next recording: what trevr_reserve_tape set, else the last
// recording's count plus a quarter (and one per set), else a first guess of
// 1024 rays per sink.
static int64_t tape_want(const trevr_tree *t, int64_t n_sinks) {
  const int64_t sets = (n_sinks + 63) / 64;
  const int64_t used = t->tape_used_h ? *(volatile int32_t *)t->tape_used_h : 0;
  int64_t cap = t->tape_reserve > 0 ? t->tape_reserve
                                    : used > 0 ? used + used / 4 + sets : sets * 1024 + sets;
  if (cap > INT32_MAX - 65536) cap = INT32_MAX - 65536;
  return cap < 1 ? 1 : cap;
}
// Bytes per tape block (64 rays): taus, sources, owners, the ray count and
// the link to the set's next block.
constexpr size_t kTapeBlockBytes =
    64 * sizeof(double) + 64 * sizeof(uint32_t) + 64 * sizeof(uint8_t) + sizeof(uint8_t) +
    sizeof(int32_t);
// The same, cut to what fits in half the free device memory (beyond what the
// tree's tape already holds); `fits` tells whether it was cut.
static int tape_blocks(trevr_tree *t, int64_t n_sinks, int64_t &cap, bool &fits) {
  cap = tape_want(t, n_sinks);
  size_t free_b = 0, total_b = 0;
  TREVR_HIP(hipMemGetInfo(&free_b, &total_b));
  const size_t held = t->tape.bytes + t->tape_src.bytes + t->tape_own.bytes + t->tape_nb.bytes +
                      t->tape_next.bytes;
  const int64_t fit = (int64_t)((free_b / 2 + held) / kTapeBlockBytes);
  fits = cap <= fit;
  if (!fits && t->tape_reserve <= 0) cap = fit;
  if (cap < 1) cap = 1;
  return TREVR_OK;
}

// A recording flux into the tape `tb`: the block counter is cleared by a
// kernel (capturable), then the walk records one tau per ray.
static int record_into(const trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
                       int64_t n_sinks, void *flux, int32_t *counters, const TapeBufs &tb,
                       hipStream_t s) {
  k_zero_i32<<<1, 64, 0, s>>>(tb.ctr, 1);
  return t->prec == TREVR_F64
             ? flux_typed<double>(t, theta, tau_ref, sinks, n_sinks, flux, counters, 1, &tb, s)
             : flux_typed<float>(t, theta, tau_ref, sinks, n_sinks, flux, counters, 1, &tb, s);
}

// The recording flux on the tree's tape: sizes it (the last recording's block
// count plus a quarter, or a first guess of 1024 rays per sink within half the
// free memory), then records.  A recording that outgrows its tape is left
// incomplete; the adjoint then traces twice, and the next recording is sized
// from this one's count, which reaches the host asynchronously.
int flux_taped_impl(trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
                    int64_t n_sinks, void *flux, int32_t *counters, hipStream_t s) {
  t->tape_ok = false;
  if (!t->tape_used_h) {
    TREVR_HIP(hipHostMalloc((void **)&t->tape_used_h, sizeof(int32_t), hipHostMallocDefault));
    *t->tape_used_h = 0;
  }
  const int64_t sets = (n_sinks + 63) / 64;
  int64_t cap = 0;
  bool fits = true;
  {
    int rc = tape_blocks(t, n_sinks, cap, fits);
    if (rc != TREVR_OK) return rc;
  }
  (void)fits;  // a short tape only makes the taped adjoint trace twice
  TREVR_HIP(t->tape.ensure((size_t)cap * 64 * sizeof(double)));
  TREVR_HIP(t->tape_src.ensure((size_t)cap * 64 * sizeof(uint32_t)));
  TREVR_HIP(t->tape_own.ensure((size_t)cap * 64 * sizeof(uint8_t)));
  TREVR_HIP(t->tape_nb.ensure((size_t)cap * sizeof(uint8_t)));
  TREVR_HIP(t->tape_next.ensure((size_t)cap * sizeof(int32_t)));
  TREVR_HIP(t->tape_head.ensure((size_t)(sets > 0 ? sets : 1) * sizeof(int32_t)));
  TREVR_HIP(t->tape_ctr.ensure(sizeof(int32_t)));
  t->tape_cap = cap;
  int rc = record_into(t, theta, tau_ref, sinks, n_sinks, flux, counters, tree_tape(t), s);
  if (rc != TREVR_OK) return rc;
  TREVR_HIP(hipMemcpyAsync(t->tape_used_h, t->tape_ctr.p, sizeof(int32_t),
                           hipMemcpyDeviceToHost, s));
  t->tape_ok = true;
  t->tape_theta = theta;
  t->tape_tau_ref = tau_ref;
  t->tape_sinks = sinks;
  t->tape_n_sinks = n_sinks;
  return TREVR_OK;
}

// The adjoint's accumulators: per cell d loss / d alpha, d loss / d L_C and
// d loss / d x_L (5 m doubles), per particle d loss / d L of single sources.
struct AdjBufs {
  double *node;  // [5][m]
  double *part;  // [n]
};

template <typename T>
static int adjoint_typed(const trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
                         int64_t n_sinks, const void *grad_flux, void *grad_rho,
                         void *grad_kappa, void *grad_lum, int tape_mode, const TapeBufs *tb,
                         const AdjBufs &ab, hipStream_t s) {
  const int64_t m = t->m, n = t->n;
  double *abar = ab.node;
  double *lbar = abar + m, *xbar = abar + 2 * m;
  double *direct = ab.part;
  k_zero_f64<<<nblk(5 * m), 256, 0, s>>>(abar, 5 * m);
  if (n > 0) k_zero_f64<<<nblk(n), 256, 0, s>>>(direct, n);
  if (n_sinks > 0) {
    FluxArgs<T> a = make_args<T, true>(t, theta, tau_ref, sinks, n_sinks);
    a.grad_flux = static_cast<const T *>(grad_flux);
    a.abar = abar;
    a.lbar = lbar;
    a.xbar = xbar;
    a.direct = direct;
    set_tape<T>(a, tape_mode, tb);
    int rc = launch_walk<T, true>(t, a, s);
    if (rc != TREVR_OK) return rc;
  }
  const BfsNode *bfs = t->bfs.as<BfsNode>();
  for (int d = (int)t->level_cnt.size() - 1; d >= 1; --d)
    k_adj_empty_up<<<nblk(t->level_cnt[d]), 256, 0, s>>>(
        bfs + t->level_off[d], (int)t->level_cnt[d], t->n_B.as<double>(),
        t->n_parent.as<int32_t>(), abar);
  if (n > 0)
    k_adj_particles<T><<<nblk(n), 256, 0, s>>>(
        n, m, t->perm.as<int32_t>(), t->leaf.as<int32_t>(), t->n_parent.as<int32_t>(),
        t->n_B.as<double>(), t->n_alpha.as<double>(), t->n_lc.as<double>(),
        t->n_xl.as<double>(), static_cast<const P4<T> *>(t->psrc.p),
        static_cast<const T *>(t->pmass.p), static_cast<const T *>(t->prho.p), abar, lbar, xbar,
        direct, static_cast<T *>(grad_rho), static_cast<T *>(grad_kappa),
        static_cast<T *>(grad_lum));
  TREVR_HIP(hipGetLastError());
  return TREVR_OK;
}

static int adjoint_dispatch(const trevr_tree *t, double theta, double tau_ref,
                            const int32_t *sinks, int64_t n_sinks, const void *grad_flux,
                            void *grad_rho, void *grad_kappa, void *grad_lum, int tape_mode,
                            const TapeBufs *tb, const AdjBufs &ab, hipStream_t s) {
  if (t->prec == TREVR_F64)
    return adjoint_typed<double>(t, theta, tau_ref, sinks, n_sinks, grad_flux, grad_rho,
                                 grad_kappa, grad_lum, tape_mode, tb, ab, s);
  return adjoint_typed<float>(t, theta, tau_ref, sinks, n_sinks, grad_flux, grad_rho, grad_kappa,
                              grad_lum, tape_mode, tb, ab, s);
}

static int tree_adj_bufs(trevr_tree *t, AdjBufs &ab) {
  const int64_t m = t->m, n = t->n;
  TREVR_HIP(t->adj_node.ensure(sizeof(double) * 5 * (size_t)(m > 0 ? m : 1)));
  TREVR_HIP(t->adj_part.ensure(sizeof(double) * (size_t)(n > 0 ? n : 1)));
  ab.node = t->adj_node.as<double>();
  ab.part = t->adj_part.as<double>();
  return TREVR_OK;
}

// Caller scratch layout, each part 256-byte aligned: the accumulators
// (5 m + n doubles); in store mode then the recording's flux (n_sinks of the
// tree's precision), the tape's per-set heads (4 B per 64 sinks), its block
// counter, and the tape itself, cap blocks of kTapeBlockBytes (64 taus, 64
// sources, 64 owners, the ray count and the link), each array on its own.
static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }
static size_t adj_part_bytes(const trevr_tree *t) {
  return al256(sizeof(double) * 5 * (size_t)(t->m > 0 ? t->m : 1)) +
         al256(sizeof(double) * (size_t)(t->n > 0 ? t->n : 1));
}
static size_t store_fixed_bytes(const trevr_tree *t, int64_t n_sinks) {
  const size_t elem = t->prec == TREVR_F64 ? sizeof(double) : sizeof(float);
  const int64_t sets = (n_sinks + 63) / 64;
  return al256(elem * (size_t)(n_sinks > 0 ? n_sinks : 1)) +
         al256(sizeof(int32_t) * (size_t)(sets > 0 ? sets : 1)) + 256;
}
static size_t store_block_bytes(int64_t cap) {
  const size_t c = (size_t)cap;
  return al256(c * 64 * sizeof(double)) + al256(c * 64 * sizeof(uint32_t)) +
         al256(c * 64 * sizeof(uint8_t)) + al256(c * sizeof(uint8_t)) +
         al256(c * sizeof(int32_t));
}

int adjoint_scratch_size_impl(const trevr_tree *t, int mode, int64_t n_sinks, size_t *bytes) {
  if (mode == TREVR_ADJ_AUTO) {
    *bytes = 0;
  } else if (mode == TREVR_ADJ_RECOMPUTE) {
    *bytes = adj_part_bytes(t);
  } else {
    const int64_t sets = (n_sinks + 63) / 64;
    int64_t cap = tape_want(t, n_sinks);
    if (cap < sets) cap = sets;
    *bytes = adj_part_bytes(t) + store_fixed_bytes(t, n_sinks) + store_block_bytes(cap);
  }
  return TREVR_OK;
}

// Carve the caller's scratch; returns false if it is too small.
static bool carve(const trevr_tree *t, int mode, int64_t n_sinks, void *scratch, size_t bytes,
                  AdjBufs &ab, TapeBufs &tb, void *&flux_tmp) {
  char *p = static_cast<char *>(scratch);
  const size_t need_adj = adj_part_bytes(t);
  if (bytes < need_adj) return false;
  ab.node = reinterpret_cast<double *>(p);
  ab.part = reinterpret_cast<double *>(p + al256(sizeof(double) * 5 * (size_t)(t->m > 0 ? t->m : 1)));
  if (mode != TREVR_ADJ_STORE) return true;
  p += need_adj;
  size_t left = bytes - need_adj;
  const size_t fixed = store_fixed_bytes(t, n_sinks);
  if (left < fixed) return false;
  const size_t elem = t->prec == TREVR_F64 ? sizeof(double) : sizeof(float);
  const int64_t sets = (n_sinks + 63) / 64;
  flux_tmp = p;
  p += al256(elem * (size_t)(n_sinks > 0 ? n_sinks : 1));
  tb.head = reinterpret_cast<int32_t *>(p);
  p += al256(sizeof(int32_t) * (size_t)(sets > 0 ? sets : 1));
  tb.ctr = reinterpret_cast<int32_t *>(p);
  p += 256;
  left -= fixed;
  // the largest cap whose blocks fit
  int64_t cap = (int64_t)(left / kTapeBlockBytes);
  while (cap > 0 && store_block_bytes(cap) > left) --cap;
  if (cap > INT32_MAX - 65536) cap = INT32_MAX - 65536;
  if (cap < (sets > 0 ? sets : 1)) return false;
  const size_t c = (size_t)cap;
  tb.tape = reinterpret_cast<double *>(p);
  p += al256(c * 64 * sizeof(double));
  tb.src = reinterpret_cast<uint32_t *>(p);
  p += al256(c * 64 * sizeof(uint32_t));
  tb.own = reinterpret_cast<uint8_t *>(p);
  p += al256(c * 64 * sizeof(uint8_t));
  tb.nb = reinterpret_cast<uint8_t *>(p);
  p += al256(c * sizeof(uint8_t));
  tb.next = reinterpret_cast<int32_t *>(p);
  tb.cap = cap;
  return true;
}

// The adjoint.  AUTO (tree-owned scratch): while the tree holds no recording
// of the caller's, a recording flux and the taped adjoint (each ray traced
// once for tau, once for the scatter, in two kernels) when the tape fits in
// half the free device memory; else one kernel that traces every ray twice;
// a recording of the caller's is left as it is.  RECOMPUTE: that one kernel.
// STORE: the recording flux and the taped adjoint, on the tree's tape (which
// then no longer holds a recording of the caller's) or on one in the
// caller's scratch.  With caller scratch nothing is allocated, nothing waits,
// and every step is a kernel launch (graph-capturable).
int adjoint_impl(trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
                 int64_t n_sinks, const void *grad_flux, void *grad_rho, void *grad_kappa,
                 void *grad_lum, int mode, void *scratch, size_t scratch_bytes, hipStream_t s) {
  if (scratch) {
    AdjBufs ab{};
    TapeBufs tb{};
    void *flux_tmp = nullptr;
    if (!carve(t, mode, n_sinks, scratch, scratch_bytes, ab, tb, flux_tmp))
      return fail(TREVR_E_CAPACITY, "scratch smaller than trevr_adjoint_scratch_size");
    if (mode == TREVR_ADJ_STORE && n_sinks > 0) {
      int rc = record_into(t, theta, tau_ref, sinks, n_sinks, flux_tmp, nullptr, tb, s);
      if (rc != TREVR_OK) return rc;
      return adjoint_dispatch(t, theta, tau_ref, sinks, n_sinks, grad_flux, grad_rho, grad_kappa,
                              grad_lum, 2, &tb, ab, s);
    }
    return adjoint_dispatch(t, theta, tau_ref, sinks, n_sinks, grad_flux, grad_rho, grad_kappa,
                            grad_lum, 0, nullptr, ab, s);
  }
  bool store = mode == TREVR_ADJ_STORE;
  if (mode == TREVR_ADJ_AUTO && n_sinks > 0 && !t->tape_ok) {
    int64_t cap = 0;
    bool fits = false;
    int rc = tape_blocks(t, n_sinks, cap, fits);
    if (rc != TREVR_OK) return rc;
    store = fits;
  }
  if (store && n_sinks > 0) {
    const size_t elem = t->prec == TREVR_F64 ? sizeof(double) : sizeof(float);
    TREVR_HIP(t->adj_flux.ensure(elem * (size_t)n_sinks));
    int rc = flux_taped_impl(t, theta, tau_ref, sinks, n_sinks, t->adj_flux.p, nullptr, s);
    if (rc == TREVR_OK) rc = adjoint_taped_impl(t, grad_flux, grad_rho, grad_kappa, grad_lum, s);
    t->tape_ok = false;  // the tape served as scratch
    return rc;
  }
  AdjBufs ab{};
  int rc = tree_adj_bufs(t, ab);
  if (rc != TREVR_OK) return rc;
  return adjoint_dispatch(t, theta, tau_ref, sinks, n_sinks, grad_flux, grad_rho, grad_kappa,
                          grad_lum, 0, nullptr, ab, s);
}

int sum_counters_impl(const int32_t *counters, int64_t n_sinks, int64_t *totals,
                      hipStream_t s) {
  k_zero_i64<<<1, 64, 0, s>>>(totals, 5);
  if (n_sinks > 0) {
    int64_t blocks = (n_sinks + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_sum_counters<<<(unsigned)blocks, 256, 0, s>>>(counters, n_sinks, totals);
  }
  TREVR_HIP(hipGetLastError());
  return TREVR_OK;
}

int adjoint_taped_impl(trevr_tree *t, const void *grad_flux, void *grad_rho, void *grad_kappa,
                       void *grad_lum, hipStream_t s) {
  AdjBufs ab{};
  int rc = tree_adj_bufs(t, ab);
  if (rc != TREVR_OK) return rc;
  const TapeBufs tb = tree_tape(t);
  return adjoint_dispatch(t, t->tape_theta, t->tape_tau_ref, t->tape_sinks, t->tape_n_sinks,
                          grad_flux, grad_rho, grad_kappa, grad_lum, 2, &tb, ab, s);
}

}  // namespace trevr
