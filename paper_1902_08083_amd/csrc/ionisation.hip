// Ionisation-equilibrium coupling around the flux: one damped step of
// on-the-spot photoionisation equilibrium per particle (the Stromgren test of
// Sec. 3.3 run to its fixed point).  With photoionisation rate sigma F and
// recombination alpha_B n_H (1 - x)^2 per neutral fraction x, equilibrium is
// x q = (1 - x)^2 with q = sigma F / (alpha_B n_H), whose root in [0, 1] is
// x_eq = 2 / ((2 + q) + sqrt((2 + q)^2 - 4)) (the product of the two roots is
// one; this form has no cancellation at large q).  The opacity per unit mass
// of the next flux is kappa = sigma x.
#include <cmath>

#include "trevr_internal.h"

namespace trevr {

template <typename T>
__global__ void k_ion_update(int64_t n, const T *flux, const T *n_h, double sigma, double alpha_b,
                             double damping, T *x, T *kappa, double *dx_max) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double dx = 0.0;
  if (i < n) {
    const double nh = n_h ? (double)n_h[i] : 1.0;
    const double q = sigma * (double)flux[i] / (alpha_b * nh);
    const double b = 2.0 + q;
    const double xe = 2.0 / (b + sqrt(b * b - 4.0));
    const double x0 = (double)x[i];
    const double x1 = (1.0 - damping) * x0 + damping * xe;
    dx = fabs(xe - x0);
    x[i] = (T)x1;
    kappa[i] = (T)(sigma * (double)(T)x1);
  }
  // wave maximum, then one atomic per wave (dx >= 0: the bit pattern orders)
  for (int o = 32; o > 0; o >>= 1) {
    const double v = __shfl_xor(dx, o);
    dx = v > dx ? v : dx;
  }
  if ((threadIdx.x & 63) == 0 && dx > 0.0)
    atomicMax((unsigned long long *)dx_max, (unsigned long long)__double_as_longlong(dx));
}

__global__ void k_ion_zero(double *p) { *p = 0.0; }

// kappa = sigma x only (the opacity of a first flux from given fractions).
template <typename T>
__global__ void k_ion_kappa(int64_t n, double sigma, const T *x, T *kappa) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) kappa[i] = (T)(sigma * (double)x[i]);
}

}  // namespace trevr

int trevr_ionisation_update(int64_t n, trevr_prec prec, const void *flux, const void *n_h,
                            double sigma, double alpha_b, double damping, void *x, void *kappa,
                            double *dx_max, hipStream_t stream) {
  if (n < 0 || (n > 0 && (!x || !kappa)) || !dx_max)
    return trevr::fail(TREVR_E_ARG, "NULL array or negative n");
  if (prec != TREVR_F32 && prec != TREVR_F64) return trevr::fail(TREVR_E_ARG, "bad precision");
  if (!(sigma >= 0) || !std::isfinite(sigma) || !(alpha_b > 0) || !std::isfinite(alpha_b) ||
      !(damping > 0 && damping <= 1))
    return trevr::fail(TREVR_E_ARG, "sigma >= 0, alpha_B > 0 and 0 < damping <= 1 required");
  trevr::k_ion_zero<<<1, 1, 0, stream>>>(dx_max);
  if (n > 0 && !flux) {  // kappa = sigma x only
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (prec == TREVR_F64)
      trevr::k_ion_kappa<double><<<blocks, 256, 0, stream>>>(n, sigma, (const double *)x,
                                                             (double *)kappa);
    else
      trevr::k_ion_kappa<float><<<blocks, 256, 0, stream>>>(n, sigma, (const float *)x,
                                                            (float *)kappa);
  } else if (n > 0) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (prec == TREVR_F64)
      trevr::k_ion_update<double><<<blocks, 256, 0, stream>>>(
          n, (const double *)flux, (const double *)n_h, sigma, alpha_b, damping, (double *)x,
          (double *)kappa, dx_max);
    else
      trevr::k_ion_update<float><<<blocks, 256, 0, stream>>>(
          n, (const float *)flux, (const float *)n_h, sigma, alpha_b, damping, (float *)x,
          (float *)kappa, dx_max);
  }
  TREVR_HIP(hipGetLastError());
  return TREVR_OK;
}
