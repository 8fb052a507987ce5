/*
 * trevr.h -- C ABI of the MI355X (gfx950) TREVR radiation-field library.
 *
 * TREVR (Grond, Woods, Wadsley & Couchman 2019, "TREVR: A general N log^2 N
 * radiative transfer algorithm") evaluates, at every sink, the angle-summed
 * intensity of point sources attenuated along straight rays:
 *
 *     F_i = sum over rays of  L exp(-tau) / (4 pi r^2)           (Sec. 2.1)
 *
 * Sources are merged on a space-filling binary tree with the opening-angle
 * criterion (Sec. 2.2.1), and each ray's optical depth tau = sum alpha l is
 * accumulated over tree cells, refining a cell only where its spread of
 * optical depth exceeds tau_ref (Sec. 2.2.2-2.2.3).
 *
 * Conventions shared by every entry point:
 *  - Every array argument named as "device" is a device pointer owned by the
 *    caller; the library never frees or retains it beyond the call, except
 *    where stated.  Host arrays are read during the call only.
 *  - Floating-point arrays are float (TREVR_F32) or double (TREVR_F64) as
 *    the particle set's precision says.  In TREVR_F32 ("binary32
 *    transport") the tree stores its cell data rounded to binary32 from the
 *    binary64 build values, each ray's geometry (direction, 1/d, r^2, r, plane
 *    crossings, piece lengths) is binary32, the refinement test and every
 *    alpha l term are exact binary64 products, and optical depths and fluxes
 *    are summed in binary64.  TREVR_F64 is binary64 throughout.
 *  - Every function returns a trevr_status (0 = success).  On failure a
 *    message is available from trevr_last_error() (per host thread).  The
 *    library never aborts and never prints.
 *  - Calls that take a stream enqueue their work on it and return without
 *    waiting, except the set-up and export calls (trevr_build_tree,
 *    trevr_refit_tree, trevr_set_bands, trevr_set_sph, trevr_set_background,
 *    trevr_export_tree, trevr_export_sph), which wait on their stream.
 *  - Calls on one tree handle must not overlap in time.
 *
 * Entry points: the tree (create, build, refit, info, export); the flux and
 * its counters; the adjoint, plain and from a recording flux (tape); the
 * vector flux and the second moment; several opacity bands on one
 * traversal; the particle trace below the buckets; the walk variants
 * (per-bucket or Gasoline opening, top-down ray walk, early termination);
 * the background shell; one step of photoionisation equilibrium; launch
 * shapes of the walk kernels.
 */
#ifndef TREVR_H
#define TREVR_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { TREVR_F32 = 0, TREVR_F64 = 1 } trevr_prec;

typedef enum {
  TREVR_OK = 0,
  TREVR_E_ARG = -1,       /* invalid argument (NULL pointer, bad size, ...) */
  TREVR_E_RANGE = -2,     /* a particle lies outside its box [lo, hi)       */
  TREVR_E_NONFINITE = -3, /* NaN or infinity in an input array               */
  TREVR_E_VALUE = -4,     /* negative mass, opacity or luminosity, or a
                             non-positive density where the mass is > 0     */
  TREVR_E_STATE = -5,     /* the tree handle holds no (suitable) tree        */
  TREVR_E_CAPACITY = -6,  /* more nodes or particles than the layout holds   */
  TREVR_E_HIP = -100      /* a HIP runtime call failed                        */
} trevr_status;

/* The particle set: one or more independent boxes ("a forest").  Box b holds
 * the particles [box_offsets[b], box_offsets[b+1]) of the arrays below and
 * its own space-filling tree over [box_lo[3b..3b+2], box_hi[3b..3b+2]).
 * One particle set carries every role (Sec. 2.2): a particle with L > 0 is a
 * source, every particle may be a sink, and a particle with mass > 0 is an
 * absorber with absorption coefficient kappa rho.  */
typedef struct {
  int64_t n;                   /* total particles over all boxes, >= 0        */
  trevr_prec prec;             /* element type of every float array below     */
  const void *x, *y, *z;       /* device, n each: positions inside their box  */
  const void *mass;            /* device, n, or NULL (all 1); mass >= 0       */
  const void *rho;             /* device, n: density, > 0 where mass > 0      */
  const void *kappa;           /* device, n: opacity, >= 0                    */
  const void *lum;             /* device, n: luminosity, >= 0                 */
  int32_t n_boxes;             /* >= 1                                        */
  const int64_t *box_offsets;  /* host, n_boxes + 1 (NULL allowed if 1 box)   */
  const double *box_lo;        /* host, 3 n_boxes: lower corners               */
  const double *box_hi;        /* host, 3 n_boxes: upper corners (exclusive)  */
  int32_t bucket_size;         /* N_B >= 1: most particles per leaf (Sec. 2.2) */
} trevr_particles;

/* Launch knobs of the flux kernel and, separately, of the adjoint kernel
 * (set by the autotuner; a new tree starts at {4, 4, 64} for the flux and
 * {3, 4, 64} for the adjoint, the faster shapes measured on MI355X).  Waves
 * per SIMD, ceil(blocks_per_cu x min(waves_per_block, 4) / 4), pick the
 * kernel's register budget. */
typedef struct {
  int32_t blocks_per_cu;   /* persistent workgroups per compute unit, 1..32   */
  int32_t waves_per_block; /* 1..16 accepted; at most 4 wavefronts are used   */
  int32_t chunk;           /* sinks per work-queue grab, a multiple of 64      */
} trevr_launch;

typedef struct {
  int64_t n;          /* particles                                          */
  int64_t m;          /* tree cells (all boxes)                             */
  int32_t n_boxes;
  int32_t max_depth;  /* deepest cell                                       */
  trevr_prec prec;
  int32_t bucket_size;
} trevr_tree_info_t;

typedef struct trevr_tree trevr_tree; /* opaque handle */

const char *trevr_status_string(int status);
const char *trevr_last_error(void);

/* Create an empty tree handle.  Its device buffers are allocated by
 * trevr_build_tree and grow as needed; trevr_tree_destroy frees them. */
int trevr_tree_create(trevr_tree **out);
void trevr_tree_destroy(trevr_tree *tree);

/* (Re)build the radiation tree and its cell properties (Sec. 2.2, 2.3):
 *  - each box is bisected at the midpoint of its longest axis (ties to the
 *    lowest axis index), recursively; a point on a plane goes to the upper
 *    half; a cell with more than bucket_size particles gets both halves even
 *    if one is empty (the tree fills space); depth is capped at 63;
 *  - cells are numbered depth-first, lower half first; particles are ordered
 *    by their 63-level path, ties by input index;
 *  - per cell: alpha = sum(m kappa) / sum(m / rho) (the volume-weighted
 *    density times the mass-weighted opacity; a cell without absorbing mass
 *    takes its parent's), directional alpha_min / alpha_max combined
 *    bottom-up (Sec. 2.2.3), luminosity, centre of luminosity and the
 *    distance from it to the furthest vertex (Sec. 2.2.1).
 * The tree copies what it needs from the particle arrays.  Waits on
 * `stream`.  Errors: TREVR_E_ARG, _RANGE, _NONFINITE, _VALUE, _CAPACITY
 * (n >= 2^31 particles, more than 2^30 - 2 cells, or trace records beyond
 * 4 GiB: more than 2^28 cells in binary32, 2^27 in binary64), _HIP; on error
 * the handle holds no tree. */
int trevr_build_tree(trevr_tree *tree, const trevr_particles *p, hipStream_t stream);

/* Refit: recompute every cell property of the built tree (alpha, the
 * directional alpha bounds, L_C, x_L, l_far; Sec. 2.2.1, 2.2.3) from new
 * mass, rho, kappa and lum, keeping its topology.  The particles must be the
 * build's: same n, precision, boxes (offsets and corners) and bucket size,
 * and every position equal, value for value, to the one the tree was built
 * from (checked on the device); the tree then equals a fresh build from the
 * same arrays.  Invalidates the tape of trevr_compute_flux_taped.  Waits on
 * `stream`.  Errors: TREVR_E_ARG (another particle set, or a moved position),
 * _STATE, _NONFINITE, _VALUE, _HIP; after a validation error the tree keeps
 * its previous properties, after a later one it holds no tree. */
int trevr_refit_tree(trevr_tree *tree, const trevr_particles *p, hipStream_t stream);

int trevr_tree_info(const trevr_tree *tree, trevr_tree_info_t *info);

/* Radiation field at the sinks (Sec. 2.1-2.2.3): for each sink a depth-first
 * source walk merges every luminous cell whose centre-of-luminosity to
 * furthest-vertex distance l satisfies l < theta_open r (r = distance from
 * the sink to the closest point of the cell, eq. openangle), else opens it
 * (a bucket then gives its particles, other than the sink and points at the
 * sink's position, as individual sources); each ray's optical depth is
 * summed over cells walking up from the sink's bucket and the source cell
 * (Sec. 2.2.2), refining where (alpha_max - alpha_min) l > tau_ref
 * (eq. refcrit); flux += L exp(-tau) / (4 pi r^2).
 *   theta_open >= 0; tau_ref any (negative: refine to buckets always,
 *   +infinity: never refine).
 *   sinks: device, n_sinks particle indices, or NULL for every particle (then
 *   n_sinks must equal n and flux[i] belongs to particle i); n_sinks = 0 is
 *   an empty evaluation whatever sinks is.  An index
 *   outside [0, n) is not evaluated: its flux is NaN and its counters -1
 *   (in the adjoint it contributes nothing).
 *   flux: device, n_sinks, precision of the tree.
 *   counters: device int32 [n_sinks][5] or NULL: cells tested for opening,
 *   rays, rays from single particles, pieces with positive length, cell
 *   records read by the ray trace.
 * Asynchronous; allocates nothing (graph-capturable) once the tree is built.
 * Errors: TREVR_E_ARG, _STATE, _HIP. */
int trevr_compute_flux(const trevr_tree *tree, double theta_open, double tau_ref,
                       const int32_t *sinks, int64_t n_sinks, void *flux, int32_t *counters,
                       hipStream_t stream);

/* How the adjoint meets the forward's rays (none stores segment lists):
 *   TREVR_ADJ_RECOMPUTE: one kernel traces every ray twice, once for its
 *     optical depth and once to scatter d loss / d alpha over its pieces
 *     (segments recomputed, nothing stored per ray);
 *   TREVR_ADJ_STORE: a recording flux stores each ray's optical depth and
 *     each round's list of rays (13 B per ray), then the adjoint replays the
 *     rounds without walking the tree and traces each ray once, for the
 *     scatter (a recording that outgrew its tape is traced twice instead);
 *   TREVR_ADJ_AUTO: STORE while the tree holds no recording of the caller's
 *     (trevr_compute_flux_taped) and the tape fits in half the free device
 *     memory, else RECOMPUTE; scratch owned by the tree. */
typedef enum { TREVR_ADJ_AUTO = 0, TREVR_ADJ_RECOMPUTE = 1, TREVR_ADJ_STORE = 2 } trevr_adjoint_mode;

/* Gradient of  sum_k grad_flux[k] * flux[k]  (flux as trevr_compute_flux
 * returns it for the same arguments) with respect to every particle's rho,
 * kappa and lum, with every accept / open / refine decision of the forward
 * held fixed (Sec. 2.2.1-2.2.3: alpha = sum m kappa / sum m/rho of each
 * piece's cell, the merged sources' L_C and centre of luminosity).  Merged
 * sources contribute through their luminosity and their centre of
 * luminosity.
 *   grad_flux: device, n_sinks.  grad_rho, grad_kappa, grad_lum: device, n
 *   each (overwritten; zero for massless particles' rho and kappa).
 *   mode: a trevr_adjoint_mode.
 *   scratch: NULL, or device memory of scratch_bytes >= what
 *   trevr_adjoint_scratch_size returns for this mode and n_sinks, 8-byte
 *   aligned, owned by the caller and not retained.  With caller scratch the
 *   call allocates nothing, never waits and only launches kernels (it can be
 *   captured in a HIP graph); STORE then keeps its tape in the scratch and
 *   leaves the tree's recording as it is.  With scratch NULL the tree's own
 *   scratch is used, allocated on first use and when the tape grows (such a
 *   call is not capturable); STORE then uses the tree's tape and drops a
 *   recording of the caller's.  AUTO takes no caller scratch.
 * Asynchronous.  Errors: TREVR_E_ARG (mode out of range, scratch with AUTO or
 * misaligned), TREVR_E_CAPACITY (scratch_bytes too small), _STATE, _HIP. */
int trevr_compute_flux_adjoint(trevr_tree *tree, double theta_open, double tau_ref,
                               const int32_t *sinks, int64_t n_sinks, const void *grad_flux,
                               void *grad_rho, void *grad_kappa, void *grad_lum, int32_t mode,
                               void *scratch, size_t scratch_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * trevr_compute_flux_adjoint in TREVR_ADJ_RECOMPUTE mode, with its scratch
 * (8 (5 m + n) bytes: the per-cell and per-particle accumulators) in a
 * device buffer of the library's own, 64 MiB per GPU, looked up when the
 * first tree is created on that GPU and held until the process ends.  The
 * call allocates nothing and frees nothing; the accumulators are cleared by
 * kernels at the start of every call.  Arguments and results as
 * trevr_compute_flux_adjoint.  The buffer is shared by every call on one
 * GPU: calls that overlap in time on one GPU (on different streams, or from
 * different host threads) race, and must be ordered by the caller.  The tree
 * must live on the current device.  Asynchronous.  Errors: TREVR_E_CAPACITY
 * (the tree needs more than 64 MiB: about 1.6 million cells with as many
 * particles), TREVR_E_ARG (as trevr_compute_flux_adjoint, or the tree's
 * device is not the current one), _STATE, _HIP. */
int trevr_compute_flux_adjoint_noalloc(trevr_tree *tree, double theta_open, double tau_ref,
                                       const int32_t *sinks, int64_t n_sinks,
                                       const void *grad_flux, void *grad_rho, void *grad_kappa,
                                       void *grad_lum, hipStream_t stream);

/* Device scratch that trevr_compute_flux_adjoint needs in `mode` for
 * n_sinks sinks on the built tree: RECOMPUTE 8 (5 m + n) bytes (per cell
 * d loss / d alpha, d loss / d L_C and d loss / d x_L; per particle the
 * single sources' d loss / d L), STORE that plus the recording's flux, the
 * tape's per-set heads and a tape of 837 B per 64 rays, sized as the tree
 * sizes its own (the last recording's block count plus a quarter, or 1024
 * rays per sink); AUTO 0 (it takes none).  A smaller STORE scratch that still
 * holds one tape block per 64 sinks is accepted: a recording that outgrows
 * it makes the adjoint trace each ray twice (same result).  Host, no wait.
 * Errors: TREVR_E_ARG, _STATE. */
int trevr_adjoint_scratch_size(const trevr_tree *tree, int32_t mode, int64_t n_sinks,
                               size_t *bytes);

/* Totals of per-sink counters (as trevr_compute_flux writes them, [n_sinks][5])
 * over the sinks, skipping invalid sinks (-1): totals, device int64 [5],
 * overwritten.  cell visits = totals[0] + totals[4].  Asynchronous, allocates
 * nothing.  Errors: TREVR_E_ARG, _HIP. */
int trevr_sum_counters(const int32_t *counters, int64_t n_sinks, int64_t *totals,
                       hipStream_t stream);

/* Flux and net radiation flux at the sinks (Sec. 2.1, eq. simpflux):
 * everything trevr_compute_flux computes, and in addition the vector sum over
 * the sink's rays, in walk order, of L exp(-tau) / (4 pi r^2) n, with n the
 * unit vector from the source point y (a particle, or a merged cell's centre
 * of luminosity) to the sink x.  It is the first moment of the intensity,
 * from which the radiation pressure follows.
 *   flux_vec: device, 3 x n_sinks, [component][sink] (x block, y block, z
 *   block), precision of the tree; NaN for an invalid sink index.
 * Runs the 4-wave kernel whatever the launch shape (at most 4 waves per
 * SIMD).  Asynchronous, allocates nothing.  Errors: as trevr_compute_flux. */
int trevr_compute_flux_vector(const trevr_tree *tree, double theta_open, double tau_ref,
                              const int32_t *sinks, int64_t n_sinks, void *flux, void *flux_vec,
                              int32_t *counters, hipStream_t stream);

/* Flux, net flux and the second moment of the intensity at the sinks: what
 * trevr_compute_flux_vector computes, and in addition the sum over the sink's
 * rays, in walk order, of L exp(-tau) / (4 pi r^2) n_a n_b (n as above): the
 * radiation pressure tensor times c (Sec. 2.1 notes that such higher moments
 * follow by simple sums).  Its trace is the flux.
 *   flux_mom: device, 6 x n_sinks, [component][sink] with components xx, yy,
 *   zz, xy, xz, yz; precision of the tree; NaN for an invalid sink index.
 * Runs a 3-wave kernel whatever the launch shape (at most 3 waves per SIMD).
 * Asynchronous, allocates nothing.  Errors: as trevr_compute_flux. */
int trevr_compute_flux_moments(const trevr_tree *tree, double theta_open, double tau_ref,
                               const int32_t *sinks, int64_t n_sinks, void *flux,
                               void *flux_vec, void *flux_mom, int32_t *counters,
                               hipStream_t stream);

/* Several opacity bands on one traversal (a reading: the paper carries one
 * opacity; this is the frequency-band extension of the same walk).  Band b's
 * cell alpha and directional spread come from its opacity field exactly as
 * the tree's own come from kappa (Sec. 2.2.3, eqs. for alpha and the spread;
 * the density weights are the tree's).  A piece is refined where the largest
 * band spread asks for it, (max_b (alpha_max - alpha_min)_b) l > tau_ref
 * (eq. refcrit), so every band meets the criterion; each band sums its own
 * tau_b and flux L exp(-tau_b) / (4 pi r^2).  One band equal to the tree's
 * kappa gives trevr_compute_flux's result up to summation order.
 * trevr_set_bands: kappa_bands device [n_bands][n], per particle in input
 * order, precision of the tree, finite and >= 0; 1 <= n_bands <= 4.  Waits on
 * `stream`.  Errors: TREVR_E_ARG, _STATE, _NONFINITE, _VALUE, _HIP.  A build
 * or a refit drops the bands.
 * trevr_compute_flux_bands: flux_bands device [n_bands][n_sinks], precision
 * of the tree (NaN for an invalid sink index); counters as trevr_compute_flux
 * (of the band traversal).  Runs a 3-wave kernel whatever the launch shape.
 * Asynchronous, allocates nothing.  Errors: as trevr_compute_flux, and
 * TREVR_E_STATE if no bands are set. */
int trevr_set_bands(trevr_tree *tree, int32_t n_bands, const void *kappa_bands,
                    hipStream_t stream);
int trevr_compute_flux_bands(const trevr_tree *tree, double theta_open, double tau_ref,
                             const int32_t *sinks, int64_t n_sinks, void *flux_bands,
                             int32_t *counters, hipStream_t stream);

/* Walk variants the paper proposes (each a separate mode; 0 / 0 / +infinity
 * is exactly trevr_compute_flux's traversal):
 *   open_mode 0: eq. openangle at the sink point (the default);
 *             1: per bucket -- r is the distance from the sink's bucket box
 *                to the cell's box, so every sink of a bucket opens and merges
 *                the same cells (the interaction list of Gasoline's bucket
 *                walk);
 *             2: Gasoline's opening radius (Sec. 2.3): a cell is merged when
 *                the sink lies farther than r_open = 2 B_max / (sqrt(3) theta)
 *                from its centre of luminosity (B_max: the distance from it
 *                to the cell's furthest vertex) and outside the cell;
 *   ray_mode  0: up the tree from the sink's bucket and the source cell
 *                (Sec. 2.2.2, the default);
 *             1: top down -- the meeting cell holds the whole ray, which is
 *                refined from there by eq. refcrit alone (the more aggressive
 *                walk Sec. 3 discusses);
 *   tau_max:  early termination (Sec. 4) -- a ray whose optical depth exceeds
 *             tau_max contributes nothing and is traced no further once its
 *             partial sum passes it; +infinity for none.
 * Arguments and results as trevr_compute_flux; with tau_max finite the
 * counters count the pieces actually traced.  Runs a 3-wave kernel whatever
 * the launch shape.  Asynchronous, allocates nothing.  Errors: as
 * trevr_compute_flux, and TREVR_E_ARG for a mode out of range or
 * tau_max <= 0 (NaN). */
int trevr_compute_flux_variant(const trevr_tree *tree, double theta_open, double tau_ref,
                               int32_t open_mode, int32_t ray_mode, double tau_max,
                               const int32_t *sinks, int64_t n_sinks, void *flux,
                               int32_t *counters, hipStream_t stream);

/* Background radiation from a shell of sources (Sec. 2.2.4): background
 * sources are ordinary particles with luminosity (typically massless) placed
 * on a sphere at the edge of the volume, e.g. on a golden-angle spiral.  A
 * merged cell whose luminous particles are all background sources would
 * radiate from its centre of luminosity, which lies inside the sphere and so
 * over-estimates the flux near the shell; here it radiates from the point
 * where the ray from the centre through x_L meets the sphere,
 * y' = centre + radius (x_L - centre) / |x_L - centre|.  The ray's optical
 * depth still runs to x_L (inside the cell); the flux term is
 * L_C e^-tau / (4 pi |y' - x_i|^2).  At the shell's centre an optically thin
 * flux is then exactly L / (4 pi R^2) at any theta_open.
 * trevr_set_background: centre host double[3], radius > 0 (finite), flags
 * device uint8 [n] (input order; non-zero marks a background source).  Waits
 * on `stream`.  Errors: TREVR_E_ARG, _STATE, _HIP.  A build or a refit drops
 * it.
 * trevr_compute_flux_background: as trevr_compute_flux with that change.
 * Runs the 3-wave kernel of the walk variants.  Asynchronous, allocates
 * nothing.  Errors: as trevr_compute_flux, and TREVR_E_STATE without a
 * background set. */
int trevr_set_background(trevr_tree *tree, const double *centre, double radius,
                         const uint8_t *flags, hipStream_t stream);
int trevr_compute_flux_background(const trevr_tree *tree, double theta_open, double tau_ref,
                                  const int32_t *sinks, int64_t n_sinks, void *flux,
                                  int32_t *counters, hipStream_t stream);

/* Ionisation-equilibrium coupling (the Stromgren test of Sec. 3.3 run to its
 * fixed point): one damped step of on-the-spot photoionisation equilibrium
 * per particle.  With rate sigma F and recombination alpha_B n_H (1 - x)^2
 * for neutral fraction x, equilibrium solves x q = (1 - x)^2 with
 * q = sigma F / (alpha_B n_H); its root in [0, 1] is taken in the form
 * x_eq = 2 / ((2 + q) + sqrt((2 + q)^2 - 4)).  Then x <- (1 - damping) x +
 * damping x_eq and kappa = sigma x (the opacity per unit mass for the next
 * flux, e.g. through trevr_refit_tree).
 *   flux: device [n], the flux at each particle (input order); n_h: device
 *   [n] hydrogen number density, or NULL for 1; x: device [n], read and
 *   written; kappa: device [n], written; all of precision prec.
 *   dx_max: device, one double: receives max_i |x_eq - x_old|.
 * With flux NULL only kappa = sigma x is written (x unchanged, dx_max 0):
 * the opacity of a first flux from given fractions.
 * sigma >= 0, alpha_B > 0, 0 < damping <= 1.  Asynchronous, allocates
 * nothing.  Errors: TREVR_E_ARG, _HIP. */
int trevr_ionisation_update(int64_t n, trevr_prec prec, const void *flux, const void *n_h,
                            double sigma, double alpha_b, double damping, void *x, void *kappa,
                            double *dx_max, hipStream_t stream);

/* Refinement below the buckets: a particle trace in the manner of SPHRay
 * (Sec. 2.2.3 and the ray-tracing passage of Sec. 2.3).  Where refinement
 * reaches a bucket and the bucket's own spread still fails the criterion,
 * spread * l > tau_ref (eq. refcrit; the spread is max - min of kappa rho over
 * the bucket's particles with mass), the piece's optical depth is, instead of
 * alpha_bucket l, the sum over the absorbers whose kernel support reaches the
 * bucket's box of m_j kappa_j times the integral of their smoothing kernel
 * along the piece (the paper's tau = (m int W) kappa ds); the receiving
 * particle never absorbs its own radiation.  The kernel is the M4 cubic
 * spline with support 2h, W(r, h) = w(r / h) / (pi h^3), integrated in closed
 * form (binary64).  tau_ref = infinity gives trevr_compute_flux's result.
 * trevr_set_sph: h device [n], smoothing lengths per particle in input order,
 * precision of the tree, finite and > 0.  Builds, on the device, each
 * bucket's absorber list (4 B per entry, typically 100-200 entries per bucket)
 * and per-particle and per-cell data (24-40 B per particle, 12-16 B per cell),
 * owned by the tree.  Waits on `stream`.  Errors: TREVR_E_ARG, _STATE,
 * _NONFINITE, _VALUE, _CAPACITY (the lists would not fit in the free device
 * memory), _HIP.  A build or a refit drops the smoothing lengths.
 * trevr_compute_flux_sph: as trevr_compute_flux (arguments, counters, NaN for
 * an invalid sink index), with the particle trace below the buckets.  Runs a
 * 3-wave kernel whatever the launch shape.  Asynchronous, allocates nothing.
 * Errors: as trevr_compute_flux, and TREVR_E_STATE without smoothing lengths.
 * trevr_export_sph: the absorber lists to host memory: *n_entries receives the
 * total entries; if offsets is not NULL, offsets [m + 1] (per cell, in the
 * depth-first order of trevr_export_tree; empty but at buckets), neighbours
 * [n_entries] (input indices, ascending tree order within a list) and, if not
 * NULL, spread [m] (the decision spread, -1 for cells that are not buckets).
 * Waits on `stream`.  Errors: TREVR_E_ARG, _STATE, _HIP. */
int trevr_set_sph(trevr_tree *tree, const void *h, hipStream_t stream);
int trevr_compute_flux_sph(const trevr_tree *tree, double theta_open, double tau_ref,
                           const int32_t *sinks, int64_t n_sinks, void *flux, int32_t *counters,
                           hipStream_t stream);
int trevr_export_sph(const trevr_tree *tree, int64_t *n_entries, int64_t *offsets,
                     int64_t *neighbours, double *spread, hipStream_t stream);

/* The flux and its adjoint with the traversal recorded once.  The recording
 * flux computes exactly what trevr_compute_flux computes (same arguments and
 * errors) and in addition stores every ray's optical depth tau (binary64)
 * and each round's list of rays (source and sink) in a tape owned by the
 * tree: 13 B per ray in blocks of 64; the taped adjoint computes what
 * trevr_compute_flux_adjoint computes for the arguments of the last
 * recording call on this tree, taking its rays from the tape instead of
 * walking the tree again and each ray's tau from it, so each ray is traced
 * once (for the scatter of Sec. 2.2.3's pieces) instead of twice.  The sink array of the recording call must be unchanged until
 * the taped adjoint has run, and both run on one stream (or are ordered).
 * Tape size: the last recording's block count plus a quarter, a first guess
 * of 1024 rays per sink within half the free device memory, or what
 * trevr_reserve_tape set.  A recording that outgrows its tape is incomplete:
 * the taped adjoint then traces every ray twice (same result, checked on the
 * device, no host synchronisation), and the next recording is sized from the
 * count.  The recording call allocates (not graph-capturable).  Errors: as
 * trevr_compute_flux; the taped adjoint: TREVR_E_STATE (no recording since
 * the tree was built), _ARG, _HIP. */
int trevr_compute_flux_taped(trevr_tree *tree, double theta_open, double tau_ref,
                             const int32_t *sinks, int64_t n_sinks, void *flux,
                             int32_t *counters, hipStream_t stream);
int trevr_compute_flux_adjoint_taped(trevr_tree *tree, const void *grad_flux, void *grad_rho,
                                     void *grad_kappa, void *grad_lum, hipStream_t stream);
/* Tape capacity of later recordings in blocks (one block per round of up to
 * 64 rays); 0 restores automatic sizing.  Errors: TREVR_E_ARG. */
int trevr_reserve_tape(trevr_tree *tree, int64_t blocks);

/* Launch knobs for later flux calls on this tree (autotuning).  Errors:
 * TREVR_E_ARG (NULL, or a field out of the ranges trevr_launch states). */
int trevr_set_launch(trevr_tree *tree, const trevr_launch *cfg);
int trevr_get_launch(const trevr_tree *tree, trevr_launch *cfg);

/* The same for later adjoint calls on this tree. */
int trevr_set_adjoint_launch(trevr_tree *tree, const trevr_launch *cfg);
int trevr_get_adjoint_launch(const trevr_tree *tree, trevr_launch *cfg);

/* Copy the tree to host memory for inspection (all host pointers, any may be
 * NULL):
 *   perm[n]: particle index at each sorted position;
 *   leaf_of[n]: leaf cell of each particle;
 *   node_i[m][8]: first, count, depth, leaf (0/1), parent (-1 at a root),
 *                 upper child (-1 at a leaf), next cell after the subtree,
 *                 split axis of the cell's depth;
 *   node_key[m]: path bits, the depth-0 choice at bit 62;
 *   node_f[m][22]: binary64 lo[3], hi[3], split plane, sum m kappa,
 *                 sum m / rho, sum L, sum L x[3], alpha, alpha_min,
 *                 alpha_max, alpha_max - alpha_min, centre of luminosity[3],
 *                 luminosity, far-vertex distance.
 * Waits on `stream`.  Errors: TREVR_E_ARG, _STATE, _HIP. */
int trevr_export_tree(const trevr_tree *tree, int64_t *perm, int64_t *leaf_of, int64_t *node_i,
                      uint64_t *node_key, double *node_f, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* TREVR_H */
