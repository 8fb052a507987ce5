// C ABI entry points: argument validation, error reporting, dispatch.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "trevr_internal.h"

namespace trevr {

static thread_local std::string g_last_error;

int fail(int status, const std::string &msg) {
  g_last_error = msg;
  return status;
}

int hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string("HIP error ") + hipGetErrorName(e) + " (" + hipGetErrorString(e) +
                 ") in " + what;
  return TREVR_E_HIP;
}

static int check_particles(const trevr_particles *p) {
  if (!p) return fail(TREVR_E_ARG, "particles is NULL");
  if (p->n < 0) return fail(TREVR_E_ARG, "n < 0");
  if (p->n >= (int64_t)1 << 31) return fail(TREVR_E_CAPACITY, "more than 2^31 - 1 particles");
  if (p->prec != TREVR_F32 && p->prec != TREVR_F64) return fail(TREVR_E_ARG, "bad precision");
  if (p->n_boxes < 1) return fail(TREVR_E_ARG, "n_boxes < 1");
  if (p->bucket_size < 1) return fail(TREVR_E_ARG, "bucket_size < 1");
  if (!p->box_lo || !p->box_hi) return fail(TREVR_E_ARG, "box corners are NULL");
  if (p->n_boxes > 1 && !p->box_offsets) return fail(TREVR_E_ARG, "box_offsets is NULL");
  if (p->n > 0 && (!p->x || !p->y || !p->z || !p->rho || !p->kappa || !p->lum))
    return fail(TREVR_E_ARG, "a particle array is NULL");
  for (int b = 0; b < 3 * p->n_boxes; ++b) {
    if (!std::isfinite(p->box_lo[b]) || !std::isfinite(p->box_hi[b]))
      return fail(TREVR_E_NONFINITE, "non-finite box corner");
    if (!(p->box_hi[b] > p->box_lo[b])) return fail(TREVR_E_ARG, "box with hi <= lo");
  }
  if (p->box_offsets) {
    if (p->box_offsets[0] != 0 || p->box_offsets[p->n_boxes] != p->n)
      return fail(TREVR_E_ARG, "box_offsets must run from 0 to n");
    for (int b = 0; b < p->n_boxes; ++b)
      if (p->box_offsets[b + 1] < p->box_offsets[b])
        return fail(TREVR_E_ARG, "box_offsets must not decrease");
  }
  return TREVR_OK;
}

// The walk's arguments; those that need no tree are checked first (so that
// they can be tested without a device).
static int check_walk_args(double theta, double tau_ref, int64_t n_sinks) {
  if (!(theta >= 0) || !std::isfinite(theta)) return fail(TREVR_E_ARG, "theta_open must be >= 0");
  if (std::isnan(tau_ref)) return fail(TREVR_E_ARG, "tau_ref is NaN");
  if (n_sinks < 0) return fail(TREVR_E_ARG, "n_sinks < 0");
  if (n_sinks >= (int64_t)1 << 31) return fail(TREVR_E_CAPACITY, "too many sinks");
  return TREVR_OK;
}
static int check_walk(const trevr_tree *t, double theta, double tau_ref, const int32_t *sinks,
                      int64_t n_sinks) {
  const int rc = check_walk_args(theta, tau_ref, n_sinks);
  if (rc != TREVR_OK) return rc;
  if (!t) return fail(TREVR_E_ARG, "tree is NULL");
  if (!t->built) return fail(TREVR_E_STATE, "tree holds no built tree");
  if (!sinks && n_sinks != t->n && n_sinks != 0)
    return fail(TREVR_E_ARG, "sinks NULL needs n_sinks == n");
  return TREVR_OK;
}

}  // namespace trevr

trevr_tree::~trevr_tree() {
  trevr::DevBuf *all[] = {&walk, &trace, &key, &psrc, &perm, &inv, &leaf, &pbox, &pmass, &prho,
                          &box_root, &box_off, &box_lo, &box_hi, &axis_tab, &axmask, &n_first, &n_count,
                          &n_depth, &n_parent, &n_right, &n_skip, &n_box, &n_axis, &n_lo,
                          &n_hi, &n_split, &n_A, &n_B, &n_SL, &n_SLx, &n_alpha, &n_amin,
                          &n_amax, &n_alpha_min, &n_alpha_max, &n_dalpha, &n_xl, &n_lc,
                          &n_lfar, &keys_in, &keys_out, &vals_in, &vals_out, &sort_tmp, &bfs,
                          &flags, &scan, &err, &box_key, &skeys, &small, &queue, &adj_node,
                          &adj_part, &adj_heap, &adj_flux, &tape, &tape_src, &tape_own, &tape_nb,
                          &tape_next, &tape_head, &tape_ctr,
                          &band_alpha, &band_dmax, &band_trace, &bs_A, &bs_alpha, &bs_amin,
                          &bs_amax, &bs_amin_d, &bs_amax_d, &bs_dalpha, &pkappa, &sph_pos,
                          &sph_mk, &sph_dp, &sph_hmax, &sph_cnt, &sph_off, &sph_nb,
                          &sph_trace, &bg_pos, &bg_nonbg};
  for (auto *b : all) b->release();
  if (tape_used_h) (void)hipHostFree(tape_used_h);
}

extern "C" {

const char *trevr_status_string(int status) {
  switch (status) {
    case TREVR_OK: return "ok";
    case TREVR_E_ARG: return "invalid argument";
    case TREVR_E_RANGE: return "particle outside its box";
    case TREVR_E_NONFINITE: return "non-finite input";
    case TREVR_E_VALUE: return "invalid input value";
    case TREVR_E_STATE: return "tree not built";
    case TREVR_E_CAPACITY: return "size beyond the layout's capacity";
    case TREVR_E_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char *trevr_last_error(void) { return trevr::g_last_error.c_str(); }

int trevr_tree_create(trevr_tree **out) {
  if (!out) return trevr::fail(TREVR_E_ARG, "out is NULL");
  trevr_tree *t = new (std::nothrow) trevr_tree();
  if (!t) return trevr::fail(TREVR_E_ARG, "out of host memory");
  hipError_t e = hipGetDevice(&t->device);
  if (e != hipSuccess) {
    delete t;
    return trevr::hip_fail(e, "hipGetDevice");
  }
  int cu = 0;
  e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, t->device);
  if (e != hipSuccess) {
    delete t;
    return trevr::hip_fail(e, "hipDeviceGetAttribute");
  }
  t->num_cu = cu > 0 ? cu : 256;
  {  // this device's copy of the no-allocation adjoint's scratch, once per device
    const int rc = trevr::noalloc_setup(t->device);
    if (rc != TREVR_OK) {
      delete t;
      return rc;
    }
  }
  e = t->queue.ensure(256);
  if (e != hipSuccess) {
    delete t;
    return trevr::hip_fail(e, "hipMalloc(queue)");
  }
  *out = t;
  return TREVR_OK;
}

void trevr_tree_destroy(trevr_tree *tree) { delete tree; }

int trevr_build_tree(trevr_tree *tree, const trevr_particles *p, hipStream_t stream) {
  int rc = trevr::check_particles(p);  // host-side fields first
  if (rc != TREVR_OK) return rc;
  if (!tree) return trevr::fail(TREVR_E_ARG, "tree is NULL");
  return trevr::build_tree_impl(tree, p, stream);
}

int trevr_set_bands(trevr_tree *tree, int32_t n_bands, const void *kappa_bands,
                    hipStream_t stream) {
  if (!tree) return trevr::fail(TREVR_E_ARG, "tree is NULL");
  if (!tree->built) return trevr::fail(TREVR_E_STATE, "tree holds no built tree");
  if (n_bands < 1 || n_bands > 4) return trevr::fail(TREVR_E_ARG, "n_bands must be 1..4");
  if (tree->n > 0 && !kappa_bands) return trevr::fail(TREVR_E_ARG, "kappa_bands is NULL");
  return trevr::bands_impl(tree, n_bands, kappa_bands, stream);
}

int trevr_compute_flux_bands(const trevr_tree *tree, double theta_open, double tau_ref,
                             const int32_t *sinks, int64_t n_sinks, void *flux_bands,
                             int32_t *counters, hipStream_t stream) {
  int rc = trevr::check_walk(tree, theta_open, tau_ref, sinks, n_sinks);
  if (rc != TREVR_OK) return rc;
  if (tree->n_bands < 1) return trevr::fail(TREVR_E_STATE, "no bands set on this tree");
  if (n_sinks > 0 && !flux_bands) return trevr::fail(TREVR_E_ARG, "flux_bands is NULL");
  return trevr::flux_bands_impl(tree, theta_open, tau_ref, sinks, n_sinks, flux_bands, counters,
                                stream);
}

int trevr_compute_flux_variant(const trevr_tree *tree, double theta_open, double tau_ref,
                               int32_t open_mode, int32_t ray_mode, double tau_max,
                               const int32_t *sinks, int64_t n_sinks, void *flux,
                               int32_t *counters, hipStream_t stream) {
  if (open_mode < 0 || open_mode > 2) return trevr::fail(TREVR_E_ARG, "open_mode must be 0, 1 or 2");
  if (ray_mode < 0 || ray_mode > 1) return trevr::fail(TREVR_E_ARG, "ray_mode must be 0 or 1");
  if (!(tau_max > 0)) return trevr::fail(TREVR_E_ARG, "tau_max must be > 0 (or +infinity)");
  int rc = trevr::check_walk(tree, theta_open, tau_ref, sinks, n_sinks);
  if (rc != TREVR_OK) return rc;
  if (n_sinks > 0 && !flux) return trevr::fail(TREVR_E_ARG, "flux is NULL");
  return trevr::flux_variant_impl(tree, theta_open, tau_ref, open_mode, ray_mode, tau_max, sinks,
                                  n_sinks, flux, counters, stream);
}

int trevr_set_background(trevr_tree *tree, const double *centre, double radius,
                         const uint8_t *flags, hipStream_t stream) {
  if (!tree) return trevr::fail(TREVR_E_ARG, "tree is NULL");
  if (!tree->built) return trevr::fail(TREVR_E_STATE, "tree holds no built tree");
  if (!centre || (tree->n > 0 && !flags)) return trevr::fail(TREVR_E_ARG, "centre or flags is NULL");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(centre[a])) return trevr::fail(TREVR_E_ARG, "centre is not finite");
  if (!(radius > 0) || !std::isfinite(radius))
    return trevr::fail(TREVR_E_ARG, "radius must be finite and > 0");
  return trevr::background_impl(tree, centre, radius, flags, stream);
}

int trevr_compute_flux_background(const trevr_tree *tree, double theta_open, double tau_ref,
                                  const int32_t *sinks, int64_t n_sinks, void *flux,
                                  int32_t *counters, hipStream_t stream) {
  int rc = trevr::check_walk(tree, theta_open, tau_ref, sinks, n_sinks);
  if (rc != TREVR_OK) return rc;
  if (!tree->bg_ok) return trevr::fail(TREVR_E_STATE, "no background shell set on this tree");
  if (n_sinks > 0 && !flux) return trevr::fail(TREVR_E_ARG, "flux is NULL");
  return trevr::flux_background_impl(tree, theta_open, tau_ref, sinks, n_sinks, flux, counters,
                                     stream);
}

int trevr_set_sph(trevr_tree *tree, const void *h, hipStream_t stream) {
  if (!tree) return trevr::fail(TREVR_E_ARG, "tree is NULL");
  if (!tree->built) return trevr::fail(TREVR_E_STATE, "tree holds no built tree");
  if (tree->n > 0 && !h) return trevr::fail(TREVR_E_ARG, "h is NULL");
  return trevr::sph_impl(tree, h, stream);
}

int trevr_compute_flux_sph(const trevr_tree *tree, double theta_open, double tau_ref,
                           const int32_t *sinks, int64_t n_sinks, void *flux, int32_t *counters,
                           hipStream_t stream) {
  int rc = trevr::check_walk(tree, theta_open, tau_ref, sinks, n_sinks);
  if (rc != TREVR_OK) return rc;
  if (!tree->sph_ok) return trevr::fail(TREVR_E_STATE, "no smoothing lengths set on this tree");
  if (n_sinks > 0 && !flux) return trevr::fail(TREVR_E_ARG, "flux is NULL");
  return trevr::flux_sph_impl(tree, theta_open, tau_ref, sinks, n_sinks, flux, counters, stream);
}

int trevr_export_sph(const trevr_tree *tree, int64_t *n_entries, int64_t *offsets,
                     int64_t *neighbours, double *spread, hipStream_t stream) {
  if (!tree || !n_entries) return trevr::fail(TREVR_E_ARG, "tree or n_entries is NULL");
  if (!tree->built || !tree->sph_ok)
    return trevr::fail(TREVR_E_STATE, "no smoothing lengths set on this tree");
  if (offsets && tree->sph_entries > 0 && !neighbours)
    return trevr::fail(TREVR_E_ARG, "neighbours is NULL");
  return trevr::export_sph_impl(tree, n_entries, offsets, neighbours, spread, stream);
}

int trevr_refit_tree(trevr_tree *tree, const trevr_particles *p, hipStream_t stream) {
  int rc = trevr::check_particles(p);  // host-side fields first
  if (rc != TREVR_OK) return rc;
  if (!tree) return trevr::fail(TREVR_E_ARG, "tree is NULL");
  if (!tree->built) return trevr::fail(TREVR_E_STATE, "tree holds no built tree");
  if (p->n != tree->n || p->prec != tree->prec || p->n_boxes != tree->n_boxes ||
      p->bucket_size != tree->nb)
    return trevr::fail(TREVR_E_ARG, "n, precision, boxes or bucket size differ from the build");
  for (int b = 0; b <= p->n_boxes; ++b) {
    const int64_t o = p->box_offsets ? p->box_offsets[b] : (b == 0 ? 0 : p->n);
    if (o != tree->h_box_off[b]) return trevr::fail(TREVR_E_ARG, "box offsets differ");
  }
  for (int b = 0; b < 3 * p->n_boxes; ++b)
    if (p->box_lo[b] != tree->h_box_lo[b] || p->box_hi[b] != tree->h_box_hi[b])
      return trevr::fail(TREVR_E_ARG, "box corners differ from the build");
  return trevr::refit_tree_impl(tree, p, stream);
}

int trevr_tree_info(const trevr_tree *tree, trevr_tree_info_t *info) {
  if (!tree || !info) return trevr::fail(TREVR_E_ARG, "NULL argument");
  if (!tree->built) return trevr::fail(TREVR_E_STATE, "tree holds no built tree");
  info->n = tree->n;
  info->m = tree->m;
  info->n_boxes = tree->n_boxes;
  info->max_depth = tree->max_depth;
  info->prec = tree->prec;
  info->bucket_size = tree->nb;
  return TREVR_OK;
}

int trevr_compute_flux(const trevr_tree *tree, double theta_open, double tau_ref,
                       const int32_t *sinks, int64_t n_sinks, void *flux, int32_t *counters,
                       hipStream_t stream) {
  int rc = trevr::check_walk(tree, theta_open, tau_ref, sinks, n_sinks);
  if (rc != TREVR_OK) return rc;
  if (n_sinks > 0 && !flux) return trevr::fail(TREVR_E_ARG, "flux is NULL");
  return trevr::flux_impl(tree, theta_open, tau_ref, sinks, n_sinks, flux, counters, stream);
}

int trevr_compute_flux_vector(const trevr_tree *tree, double theta_open, double tau_ref,
                              const int32_t *sinks, int64_t n_sinks, void *flux, void *flux_vec,
                              int32_t *counters, hipStream_t stream) {
  int rc = trevr::check_walk(tree, theta_open, tau_ref, sinks, n_sinks);
  if (rc != TREVR_OK) return rc;
  if (n_sinks > 0 && (!flux || !flux_vec))
    return trevr::fail(TREVR_E_ARG, "flux or flux_vec is NULL");
  return trevr::flux_vec_impl(tree, theta_open, tau_ref, sinks, n_sinks, flux, flux_vec,
                              nullptr, counters, stream);
}

int trevr_compute_flux_moments(const trevr_tree *tree, double theta_open, double tau_ref,
                               const int32_t *sinks, int64_t n_sinks, void *flux,
                               void *flux_vec, void *flux_mom, int32_t *counters,
                               hipStream_t stream) {
  int rc = trevr::check_walk(tree, theta_open, tau_ref, sinks, n_sinks);
  if (rc != TREVR_OK) return rc;
  if (n_sinks > 0 && (!flux || !flux_vec || !flux_mom))
    return trevr::fail(TREVR_E_ARG, "flux, flux_vec or flux_mom is NULL");
  return trevr::flux_vec_impl(tree, theta_open, tau_ref, sinks, n_sinks, flux, flux_vec,
                              flux_mom, counters, stream);
}

int trevr_compute_flux_taped(trevr_tree *tree, double theta_open, double tau_ref,
                             const int32_t *sinks, int64_t n_sinks, void *flux,
                             int32_t *counters, hipStream_t stream) {
  int rc = trevr::check_walk(tree, theta_open, tau_ref, sinks, n_sinks);
  if (rc != TREVR_OK) return rc;
  if (n_sinks > 0 && !flux) return trevr::fail(TREVR_E_ARG, "flux is NULL");
  return trevr::flux_taped_impl(tree, theta_open, tau_ref, sinks, n_sinks, flux, counters,
                                stream);
}

int trevr_compute_flux_adjoint_taped(trevr_tree *tree, const void *grad_flux, void *grad_rho,
                                     void *grad_kappa, void *grad_lum, hipStream_t stream) {
  if (!tree) return trevr::fail(TREVR_E_ARG, "tree is NULL");
  if (!tree->built) return trevr::fail(TREVR_E_STATE, "tree holds no built tree");
  if (!tree->tape_ok) return trevr::fail(TREVR_E_STATE, "no recording flux call on this tree");
  if (tree->n > 0 && (!grad_rho || !grad_kappa || !grad_lum))
    return trevr::fail(TREVR_E_ARG, "a gradient output is NULL");
  if (tree->tape_n_sinks > 0 && !grad_flux) return trevr::fail(TREVR_E_ARG, "grad_flux is NULL");
  return trevr::adjoint_taped_impl(tree, grad_flux, grad_rho, grad_kappa, grad_lum, stream);
}

int trevr_reserve_tape(trevr_tree *tree, int64_t blocks) {
  if (!tree) return trevr::fail(TREVR_E_ARG, "tree is NULL");
  if (blocks < 0 || blocks > INT32_MAX - 65536)
    return trevr::fail(TREVR_E_ARG, "blocks must be 0..2^31 - 65537");
  tree->tape_reserve = blocks;
  return TREVR_OK;
}

int trevr_compute_flux_adjoint(trevr_tree *tree, double theta_open, double tau_ref,
                               const int32_t *sinks, int64_t n_sinks, const void *grad_flux,
                               void *grad_rho, void *grad_kappa, void *grad_lum, int32_t mode,
                               void *scratch, size_t scratch_bytes, hipStream_t stream) {
  if (mode < TREVR_ADJ_AUTO || mode > TREVR_ADJ_STORE)
    return trevr::fail(TREVR_E_ARG, "mode must be TREVR_ADJ_AUTO, _RECOMPUTE or _STORE");
  if (scratch && mode == TREVR_ADJ_AUTO)
    return trevr::fail(TREVR_E_ARG, "TREVR_ADJ_AUTO takes no caller scratch");
  if (scratch && ((uintptr_t)scratch & 7u))
    return trevr::fail(TREVR_E_ARG, "scratch must be 8-byte aligned");
  int rc = trevr::check_walk_args(theta_open, tau_ref, n_sinks);
  if (rc != TREVR_OK) return rc;
  if (n_sinks > 0 && !grad_flux) return trevr::fail(TREVR_E_ARG, "grad_flux is NULL");
  rc = trevr::check_walk(tree, theta_open, tau_ref, sinks, n_sinks);
  if (rc != TREVR_OK) return rc;
  if (tree->n > 0 && (!grad_rho || !grad_kappa || !grad_lum))
    return trevr::fail(TREVR_E_ARG, "a gradient output is NULL");
  return trevr::adjoint_impl(tree, theta_open, tau_ref, sinks, n_sinks, grad_flux, grad_rho,
                             grad_kappa, grad_lum, mode, scratch, scratch_bytes, stream);
}

int trevr_adjoint_scratch_size(const trevr_tree *tree, int32_t mode, int64_t n_sinks,
                               size_t *bytes) {
  if (!tree || !bytes) return trevr::fail(TREVR_E_ARG, "tree or bytes is NULL");
  if (!tree->built) return trevr::fail(TREVR_E_STATE, "tree holds no built tree");
  if (mode < TREVR_ADJ_AUTO || mode > TREVR_ADJ_STORE)
    return trevr::fail(TREVR_E_ARG, "mode must be TREVR_ADJ_AUTO, _RECOMPUTE or _STORE");
  if (n_sinks < 0 || n_sinks >= (int64_t)1 << 31) return trevr::fail(TREVR_E_ARG, "bad n_sinks");
  return trevr::adjoint_scratch_size_impl(tree, mode, n_sinks, bytes);
}

int trevr_sum_counters(const int32_t *counters, int64_t n_sinks, int64_t *totals,
                       hipStream_t stream) {
  if (n_sinks < 0 || !totals || (n_sinks > 0 && !counters))
    return trevr::fail(TREVR_E_ARG, "NULL array or negative n_sinks");
  return trevr::sum_counters_impl(counters, n_sinks, totals, stream);
}

static int check_launch(const trevr_launch *cfg) {
  if (!cfg) return trevr::fail(TREVR_E_ARG, "NULL argument");
  if (cfg->blocks_per_cu < 1 || cfg->blocks_per_cu > 32)
    return trevr::fail(TREVR_E_ARG, "blocks_per_cu must be 1..32");
  if (cfg->waves_per_block < 1 || cfg->waves_per_block > 16)
    return trevr::fail(TREVR_E_ARG, "waves_per_block must be 1..16");
  if (cfg->chunk < 64 || cfg->chunk % 64 != 0 || cfg->chunk > 4096)
    return trevr::fail(TREVR_E_ARG, "chunk must be a multiple of 64 in 64..4096");
  return TREVR_OK;
}
static int set_launch_checked(trevr_tree *tree, const trevr_launch *cfg, trevr_launch *dst) {
  int rc = check_launch(cfg);  // the shape first
  if (rc != TREVR_OK) return rc;
  if (!tree) return trevr::fail(TREVR_E_ARG, "NULL argument");
  *dst = *cfg;
  return TREVR_OK;
}

int trevr_set_launch(trevr_tree *tree, const trevr_launch *cfg) {
  return set_launch_checked(tree, cfg, tree ? &tree->launch : nullptr);
}

int trevr_get_launch(const trevr_tree *tree, trevr_launch *cfg) {
  if (!tree || !cfg) return trevr::fail(TREVR_E_ARG, "NULL argument");
  *cfg = tree->launch;
  return TREVR_OK;
}

int trevr_set_adjoint_launch(trevr_tree *tree, const trevr_launch *cfg) {
  return set_launch_checked(tree, cfg, tree ? &tree->launch_adj : nullptr);
}

int trevr_get_adjoint_launch(const trevr_tree *tree, trevr_launch *cfg) {
  if (!tree || !cfg) return trevr::fail(TREVR_E_ARG, "NULL argument");
  *cfg = tree->launch_adj;
  return TREVR_OK;
}

int trevr_export_tree(const trevr_tree *tree, int64_t *perm, int64_t *leaf_of, int64_t *node_i,
                      uint64_t *node_key, double *node_f, hipStream_t stream) {
  if (!tree) return trevr::fail(TREVR_E_ARG, "tree is NULL");
  if (!tree->built) return trevr::fail(TREVR_E_STATE, "tree holds no built tree");
  return trevr::export_tree_impl(tree, perm, leaf_of, node_i, node_key, node_f, stream);
}

}  // extern "C"
