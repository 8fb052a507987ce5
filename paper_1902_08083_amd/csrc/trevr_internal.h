// Internal layouts of the TREVR gfx950 library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "trevr.h"

namespace trevr {

constexpr int kDmax = 63;           // deepest level; 63 path bits per key
constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kRefineStack = 64;    // refinement recursion never exceeds the depth

// ---- transport records (what the kernels read in the hot loops) ----------
//
// Source-walk record, one per cell in depth-first order.  Read wave-uniformly
// (scalar loads) by the opening test; 64 B in binary32, 128 B in binary64.
template <typename T>
struct WalkRecT;
template <>
struct alignas(64) WalkRecT<float> {
  float lo[3], hi[3];  // space-filling box
  float xl[3];         // centre of luminosity
  float L;             // luminosity (0: no sources below)
  float lfar;          // centre of luminosity -> furthest vertex
  int32_t skip;        // next cell after this subtree
  int32_t right_ax;    // upper child (0 at a leaf) | split axis << 30
  int32_t first;       // first particle (sorted order)
  int32_t count;       // particles in the cell
  int32_t depth;
};
template <>
struct alignas(64) WalkRecT<double> {
  double lo[3], hi[3];
  double xl[3];
  double L;
  double lfar;
  int32_t skip, right_ax, first, count, depth;
  int32_t pad[5];
};
static_assert(sizeof(WalkRecT<float>) == 64, "walk record layout");
static_assert(sizeof(WalkRecT<double>) == 128, "walk record layout");

// Ray-trace record: what a chain step or a refinement step reads.
template <typename T>
struct TraceRecT;
template <>
struct alignas(16) TraceRecT<float> {
  float split, alpha, dalpha;
  int32_t right_ax;
};
template <>
struct alignas(32) TraceRecT<double> {
  double split, alpha, dalpha;
  int32_t right_ax, pad;
};
static_assert(sizeof(TraceRecT<float>) == 16, "trace record layout");
static_assert(sizeof(TraceRecT<double>) == 32, "trace record layout");

// Particle in sorted order: position and luminosity.
template <typename T>
struct P4;
template <>
struct alignas(16) P4<float> {
  float x, y, z, L;
};
template <>
struct alignas(32) P4<double> {
  double x, y, z, L;
};

__host__ __device__ inline int rax_right(int32_t ra) { return ra & 0x3fffffff; }
__host__ __device__ inline int rax_axis(int32_t ra) { return (int)((uint32_t)ra >> 30); }

// Level-order (breadth-first) cell record used while building.
struct BfsNode {
  int32_t first, count, box, parent;  // parent: index in the previous level
  int32_t child;                      // index of the lower child in the next level, -1 leaf
  int32_t size;                       // cells in the subtree
  int32_t pre;                        // depth-first index
  int32_t pad;
  uint64_t prefix;                    // path bits
  double lo[3], hi[3];
};

// ---- device buffers -------------------------------------------------------
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t need) {
    if (need <= bytes && p) return hipSuccess;
    if (p) {
      hipError_t e = hipFree(p);
      p = nullptr;
      bytes = 0;
      if (e != hipSuccess) return e;
    }
    size_t want = need < 256 ? 256 : need;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) bytes = want;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename U>
  U *as() const {
    return static_cast<U *>(p);
  }
};

}  // namespace trevr

// The tree handle.
struct trevr_tree {
  bool built = false;
  int64_t n = 0, m = 0;
  trevr_prec prec = TREVR_F32;
  int32_t nb = 8;
  int32_t n_boxes = 0;
  int32_t max_depth = 0;
  int device = 0;
  int num_cu = 256;
  trevr_launch launch{4, 4, 64};      // flux kernel
  trevr_launch launch_adj{3, 4, 64};  // adjoint kernel

  // transport
  trevr::DevBuf walk, trace, key, psrc;
  // particles in sorted order
  trevr::DevBuf perm, inv, leaf, pbox, pmass, prho, pkappa;
  // per box
  trevr::DevBuf box_root, box_off, box_lo, box_hi, axis_tab;
  trevr::DevBuf axmask;  // per box: 3 u64, bit (62 - depth) set where that depth splits axis a
  std::vector<int32_t> h_box_root;
  std::vector<int64_t> h_box_off;
  std::vector<double> h_box_lo, h_box_hi;
  // binary64 cell data (build, export, adjoint)
  trevr::DevBuf n_first, n_count, n_depth, n_parent, n_right, n_skip, n_box, n_axis;
  trevr::DevBuf n_lo, n_hi, n_split, n_A, n_B, n_SL, n_SLx, n_alpha, n_amin, n_amax;
  trevr::DevBuf n_alpha_min, n_alpha_max, n_dalpha, n_xl, n_lc, n_lfar;
  // build scratch
  trevr::DevBuf keys_in, keys_out, vals_in, vals_out, sort_tmp, bfs, flags, scan, err;
  trevr::DevBuf box_key, skeys, small;
  std::vector<int64_t> level_off, level_cnt;
  // work queue (one counter per XCD) and adjoint scratch
  trevr::DevBuf queue;
  trevr::DevBuf adj_node, adj_part, adj_heap, adj_flux;
  // opacity bands (trevr_set_bands): per band cell alpha [n_bands][m] in the
  // transport precision, the largest band spread, trace records carrying it
  int32_t n_bands = 0;
  trevr::DevBuf band_alpha, band_dmax, band_trace;
  trevr::DevBuf bs_A, bs_alpha, bs_amin, bs_amax, bs_amin_d, bs_amax_d, bs_dalpha;
  // sub-bucket particle trace (trevr_set_sph), sorted order: per particle
  // x, y, z, h (P4 with h in place of L) and m kappa; per cell the decision
  // spread (-1 but at buckets) and the largest h of its absorbers; per bucket
  // the absorbers whose kernel reaches its box (int64 offsets by cell); trace
  // records whose buckets carry their particle spread
  bool sph_ok = false;
  int64_t sph_entries = 0;
  trevr::DevBuf sph_pos, sph_mk, sph_dp, sph_hmax, sph_cnt, sph_off, sph_nb, sph_trace;
  // background shell (trevr_set_background): per cell whose luminous
  // particles are all background sources, its merged source on the sphere
  // (x, y, z; L = 1 for such a cell, 0 otherwise)
  bool bg_ok = false;
  trevr::DevBuf bg_pos, bg_nonbg;
  // tape of per-ray optical depths (and each round's ray list) from the last
  // recording flux call
  trevr::DevBuf tape, tape_src, tape_own, tape_nb, tape_next, tape_head, tape_ctr;
  int64_t tape_cap = 0;             // blocks of 64
  int64_t tape_reserve = 0;         // blocks for later recordings, 0 = sized automatically
  int32_t *tape_used_h = nullptr;   // pinned: blocks the last recording took
  bool tape_ok = false;             // a recording exists for the arguments below
  double tape_theta = 0.0, tape_tau_ref = 0.0;
  const int32_t *tape_sinks = nullptr;
  int64_t tape_n_sinks = 0;

  ~trevr_tree();
};

namespace trevr {
// error reporting (per host thread)
int fail(int status, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

int build_tree_impl(trevr_tree *t, const trevr_particles *p, hipStream_t s);
int refit_tree_impl(trevr_tree *t, const trevr_particles *p, hipStream_t s);
int bands_impl(trevr_tree *t, int nb, const void *kappa_bands, hipStream_t s);
int flux_bands_impl(const trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
                    int64_t n_sinks, void *flux_bands, int32_t *counters, hipStream_t s);
int flux_variant_impl(const trevr_tree *t, double theta, double tau_ref, int open_mode,
                      int ray_mode, double tau_max, const int32_t *sinks, int64_t n_sinks,
                      void *flux, int32_t *counters, hipStream_t s);
int sph_impl(trevr_tree *t, const void *h, hipStream_t s);
int background_impl(trevr_tree *t, const double *centre, double radius, const uint8_t *flags,
                    hipStream_t s);
int flux_background_impl(const trevr_tree *t, double theta, double tau_ref,
                         const int32_t *sinks, int64_t n_sinks, void *flux, int32_t *counters,
                         hipStream_t s);
int export_sph_impl(const trevr_tree *t, int64_t *n_entries, int64_t *offsets,
                    int64_t *neighbours, double *spread, hipStream_t s);
int flux_sph_impl(const trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
                  int64_t n_sinks, void *flux, int32_t *counters, hipStream_t s);
int export_tree_impl(const trevr_tree *t, int64_t *perm, int64_t *leaf_of, int64_t *node_i,
                     uint64_t *node_key, double *node_f, hipStream_t s);
int flux_impl(const trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
              int64_t n_sinks, void *flux, int32_t *counters, hipStream_t s);
int adjoint_impl(trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
                 int64_t n_sinks, const void *grad_flux, void *grad_rho, void *grad_kappa,
                 void *grad_lum, int mode, void *scratch, size_t scratch_bytes, hipStream_t s);
int adjoint_scratch_size_impl(const trevr_tree *t, int mode, int64_t n_sinks, size_t *bytes);
int sum_counters_impl(const int32_t *counters, int64_t n_sinks, int64_t *totals, hipStream_t s);
int noalloc_setup(int device);  // the no-allocation adjoint's scratch, per device
int flux_vec_impl(const trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
                  int64_t n_sinks, void *flux, void *flux_vec, void *flux_mom,
                  int32_t *counters, hipStream_t s);
int flux_taped_impl(trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
                    int64_t n_sinks, void *flux, int32_t *counters, hipStream_t s);
int adjoint_taped_impl(trevr_tree *t, const void *grad_flux, void *grad_rho, void *grad_kappa,
                       void *grad_lum, hipStream_t s);
}  // namespace trevr

#define TREVR_HIP(call)                                      \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return ::trevr::hip_fail(e_, #call); \
  } while (0)
