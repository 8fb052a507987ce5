/* Drives the oracle's OpenMP loops on several threads for ThreadSanitizer
 * (test infrastructure, built and run by tests/test_sanitizers.py): the flux,
 * the vector flux, bands, the particle trace, a walk variant, the background
 * shell and the adjoint, on a seeded random particle set.  Exits 0 if every
 * call returns 0 and the flux is finite and positive. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void *oracle_build(int64_t n, const double *x, const double *y, const double *z,
                   const double *mass, const double *rho, const double *kappa, const double *lum,
                   const double *lo, const double *hi, int nb, int mirror32);
void oracle_free(void *h);
int oracle_flux(void *h, double theta, double tau_ref, const int64_t *sinks, int64_t ns,
                int nthreads, double *F, int64_t *counters, double *G);
int oracle_flux_vec(void *h, double theta, double tau_ref, const int64_t *sinks, int64_t ns,
                    int nthreads, double *F, double *Fv);
int oracle_set_bands(void *h, int k, const double *kappa_bands);
int oracle_flux_bands(void *h, double theta, double tau_ref, const int64_t *sinks, int64_t ns,
                      int nthreads, double *Fb, int64_t *counters);
int oracle_set_sph(void *h, const double *hsm);
int oracle_flux_sph(void *h, double theta, double tau_ref, const int64_t *sinks, int64_t ns,
                    int nthreads, double *F, int64_t *counters);
int oracle_flux_variant(void *h, double theta, double tau_ref, int open_mode, int ray_mode,
                        double tau_max, const int64_t *sinks, int64_t ns, int nthreads,
                        double *F, int64_t *counters);
int oracle_set_background(void *h, const double *centre, double radius,
                          const unsigned char *flags);
int oracle_flux_background(void *h, double theta, double tau_ref, const int64_t *sinks,
                           int64_t ns, int nthreads, double *F, int64_t *counters);
int oracle_adjoint(void *h, double theta, double tau_ref, const int64_t *sinks, int64_t ns,
                   const double *gradF, int nthreads, double *grad_rho, double *grad_kappa,
                   double *grad_lum);

static uint64_t s = 88172645463325252ull; /* xorshift64 */
static double rnd(void) {
  s ^= s << 13;
  s ^= s >> 7;
  s ^= s << 17;
  return (double)(s >> 11) * (1.0 / 9007199254740992.0);
}

int main(int argc, char **argv) {
  const int64_t n = argc > 1 ? atoll(argv[1]) : 1500;
  const int nt = argc > 2 ? atoi(argv[2]) : 4;
  double *x = malloc(n * sizeof(double)), *y = malloc(n * sizeof(double));
  double *z = malloc(n * sizeof(double)), *m = malloc(n * sizeof(double));
  double *rho = malloc(n * sizeof(double)), *kap = malloc(n * sizeof(double));
  double *lum = malloc(n * sizeof(double)), *hsm = malloc(n * sizeof(double));
  double *kb = malloc(2 * n * sizeof(double)), *F = malloc(n * sizeof(double));
  double *Fv = malloc(3 * n * sizeof(double)), *Fb = malloc(2 * n * sizeof(double));
  double *gr = malloc(n * sizeof(double)), *gk = malloc(n * sizeof(double));
  double *gl = malloc(n * sizeof(double)), *w = malloc(n * sizeof(double));
  int64_t *C = malloc(5 * n * sizeof(int64_t));
  unsigned char *flags = malloc(n);
  for (int64_t i = 0; i < n; ++i) {
    x[i] = rnd();
    y[i] = rnd();
    z[i] = i % 7 == 0 ? 0.5 : rnd(); /* a plane of points */
    m[i] = i % 11 == 0 ? 0.0 : 0.5 + rnd();
    rho[i] = exp(rnd() - 0.5);
    kap[i] = 0.2 + 3.0 * rnd();
    lum[i] = i % 3 == 0 ? pow(10.0, rnd() - 0.5) : 0.0;
    hsm[i] = 0.05 + 0.05 * rnd();
    kb[i] = kap[i];
    kb[n + i] = 0.5 * kap[i];
    flags[i] = i % 5 == 0;
    w[i] = rnd() - 0.5;
  }
  const double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, c[3] = {0.5, 0.5, 0.5};
  const int64_t n_few = n < 96 ? n : 96; /* the particle trace on a few sinks */
  int64_t few[96];
  for (int64_t i = 0; i < n_few; ++i) few[i] = (i * 37) % n;
  int bad = 0;
  for (int mirror = 0; mirror < 2; ++mirror) {
    void *t = oracle_build(n, x, y, z, m, rho, kap, lum, lo, hi, 6, mirror);
    if (!t) return 2;
    bad |= oracle_flux(t, 0.75, 0.1, NULL, n, nt, F, C, NULL);
    for (int64_t i = 0; i < n; ++i) bad |= !(F[i] >= 0 && isfinite(F[i]));
    bad |= oracle_flux_vec(t, 0.5, -1.0, NULL, n, nt, F, Fv);
    bad |= oracle_set_bands(t, 2, kb);
    bad |= oracle_flux_bands(t, 0.75, 0.1, NULL, n, nt, Fb, C);
    bad |= oracle_flux_variant(t, 0.75, 0.1, 1, 1, 5.0, NULL, n, nt, F, C);
    bad |= oracle_set_sph(t, hsm);
    bad |= oracle_flux_sph(t, 0.75, 0.05, few, n_few, nt, F, C);
    bad |= oracle_set_background(t, c, 0.45, flags);
    bad |= oracle_flux_background(t, 1.0, 0.1, NULL, n, nt, F, C);
    bad |= oracle_adjoint(t, 0.75, 0.1, NULL, n, w, nt, gr, gk, gl);
    oracle_free(t);
  }
  printf("driver done: %s\n", bad ? "ERROR" : "ok");
  return bad ? 1 : 0;
}
