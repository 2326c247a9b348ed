// Chebyshev expansion of the orbital propagator exp(-i A dt) (Sec. II.C,
// Eq. exponential_integrator): the coefficients of the series in the shifted
// and scaled operator (A - c) / r, shared by the step kernels of every model
// kind (device code).
#pragma once

#include "iesh_internal.hpp"

namespace iesh {

// Bessel J_k(rho), k = 0..K, by Miller's downward recurrence normalised with
// J_0 + 2 sum_{k>=1} J_{2k} = 1.
__device__ inline void bessel_j(int K, double rho, double* J) {
  for (int k = 0; k <= K; ++k) J[k] = 0.0;
  if (rho < 1e-300) {
    J[0] = 1.0;
    return;
  }
  const int base = (K > (int)rho ? K : (int)rho);
  int m = base + 30 + (int)sqrt(40.0 * (base + 1));
  m += (m & 1);
  double jp1 = 0.0, jk = 1e-280, norm = 0.0;
  for (int k = m; k > 0; --k) {
    const double jm1 = (2.0 * k / rho) * jk - jp1;  // J_{k-1}
    jp1 = jk;
    jk = jm1;
    if (fabs(jk) > 1e250) {
      jk *= 1e-250;
      jp1 *= 1e-250;
      norm *= 1e-250;
      for (int q = 0; q <= K; ++q) J[q] *= 1e-250;
    }
    const int km1 = k - 1;
    if (km1 <= K) J[km1] = jk;
    if (km1 > 0 && (km1 & 1) == 0) norm += 2.0 * jk;
  }
  norm += jk;  // J_0
  const double inv = 1.0 / norm;
  for (int k = 0; k <= K; ++k) J[k] *= inv;
}

// Number of Chebyshev terms so that the tail sum_{k>K} 2|J_k(rho)| < tol,
// bounding |J_k(rho)| by (rho/2)^k / k!.
__device__ inline int cheb_terms(double rho, double tol) {
  const double h = 0.5 * rho;
  double term = 1.0;  // (rho/2)^k / k!
  for (int k = 0; k < kMaxCheb - 1; ++k) {
    const double next = term * h / (k + 1);  // bound of |J_{k+1}|
    if (k + 2 > h) {
      const double tail = 2.0 * next / (1.0 - h / (k + 2));
      if (tail < tol) return k > 0 ? k : 1;
    }
    term = next;
  }
  return -1;
}

// Chebyshev block of one trajectory for a propagator over dte whose
// Hermitian matrix has its spectrum in [lo, hi] (Gershgorin bounds): centre,
// 1/radius, number of terms K and the coefficients
//   c_k = e^{-i c dte} (2 - delta_k0) (-i)^k J_k(r dte).
// Counts the terms in the work counters, the context's and (cls_work, may be
// null) the class's (count_step: also one trajectory-step).  J: scratch of kMaxCheb doubles.  Returns K, or -1 when
// the series would need more than kMaxCheb terms.
__device__ inline int write_cheb(double* cb, double lo, double hi, double dte, int precision,
                                 Counters* cnt, bool count_step, double* J, int64_t* cls_work) {
  const double cc = 0.5 * (lo + hi);
  const double rr = fmax(0.5 * (hi - lo), 1e-300);
  const double rho = rr * dte;
  // truncation: the tail bound stays under about two units of FP64 rounding,
  // or a quarter of one unit of FP32 rounding (2^-26) for the FP32 series
  const int K = cheb_terms(rho, precision == IESH_FP64 ? 2e-16 : 0x1p-26);
  if (K < 0) return -1;
  bessel_j(K, rho, J);
  double sn, cs;
  sincos(cc * dte, &sn, &cs);
  // e^{-i c dt} * (2 - delta_k0) * (-i)^k * J_k
  for (int k = 0; k <= K; ++k) {
    const double a = (k ? 2.0 : 1.0) * J[k];
    double ar, ai;  // (-i)^k * a
    switch (k & 3) {
      case 0: ar = a; ai = 0.0; break;
      case 1: ar = 0.0; ai = -a; break;
      case 2: ar = -a; ai = 0.0; break;
      default: ar = 0.0; ai = a; break;
    }
    cb[CHEB_COEF + 2 * k] = cs * ar + sn * ai;
    cb[CHEB_COEF + 2 * k + 1] = cs * ai - sn * ar;
  }
  cb[CHEB_C] = cc;
  cb[CHEB_INVR] = 1.0 / rr;
  cb[CHEB_K] = (double)K;
  cb[CHEB_RHO] = rho;
  // work counters (integer sums: independent of the order of the adds)
  atomicAdd((unsigned long long*)&cnt->sum_cheb, (unsigned long long)K);
  if (count_step) atomicAdd((unsigned long long*)&cnt->traj_steps, 1ull);
  atomicMax((unsigned long long*)&cnt->max_cheb, (unsigned long long)K);
  if (cls_work) {  // the same two sums for the trajectory's class
    atomicAdd((unsigned long long*)&cls_work[0], (unsigned long long)K);
    if (count_step) atomicAdd((unsigned long long*)&cls_work[1], 1ull);
  }
  return K;
}

}  // namespace iesh
