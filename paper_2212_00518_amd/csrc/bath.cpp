// Bath discretisation of Appendix A (host code).
//
// Trapezoid: eps_k = a + (k-1)(b-a)/M, w_k = (b-a)/M (left-endpoint grid as
// printed); midpoint variant eps_k = a + (k-1/2)(b-a)/M.
// Gauss-Legendre: M/2 nodes on [a, eps_f] and M/2 on [eps_f, b], each an
// affine map of the Legendre nodes x_i on [-1, 1] with weights scaled by
// half the interval length.  Nodes are found by Newton's method on P_m with
// the three-term recurrence (m + 1) P_{m+1} = (2m + 1) x P_m - m P_{m-1},
// started from the asymptotic guesses cos(pi (i - 1/4) / (m + 1/2)); the
// weights are 2 / ((1 - x^2) P_m'(x)^2).

#include <cmath>
#include <vector>

#include "iesh_internal.hpp"

namespace iesh {

static void legendre_nodes(int m, std::vector<double>& x, std::vector<double>& w) {
  x.assign(m, 0.0);
  w.assign(m, 0.0);
  for (int i = 0; i < m; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (m + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < m; ++k) {
        const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      const double pm = (m == 0) ? 1.0 : p1;
      const double pm1 = (m == 1) ? 1.0 : p0;
      // P_m'(z) = m (z P_m - P_{m-1}) / (z^2 - 1)
      dp = m * (z * pm - pm1) / (z * z - 1.0);
      const double dz = pm / dp;
      z -= dz;
      if (std::fabs(dz) <= 1e-16 * std::fabs(z) + 1e-300) {
        // one more evaluation for the weight at the converged node
        p0 = 1.0;
        p1 = z;
        for (int k = 1; k < m; ++k) {
          const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
          p0 = p1;
          p1 = p2;
        }
        dp = m * (z * p1 - ((m == 1) ? 1.0 : p0)) / (z * z - 1.0);
        break;
      }
    }
    // ascending order
    x[m - 1 - i] = z;
    w[m - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

int discretize(int kind, int M, double a, double b, double eps_f, double* eps, double* w) {
  if (M < 1 || !(b > a) || !eps || !w) return IESH_EINVAL;
  if (kind == IESH_BATH_TRAPEZOID || kind == IESH_BATH_TRAPEZOID_MIDPOINT) {
    const double off = (kind == IESH_BATH_TRAPEZOID) ? 0.0 : 0.5;
    for (int k = 0; k < M; ++k) {
      eps[k] = a + (k + off) * (b - a) / M;
      w[k] = (b - a) / M;
    }
    return IESH_OK;
  }
  if (kind == IESH_BATH_GAUSS_LEGENDRE) {
    if (M % 2 || !(eps_f > a && eps_f < b)) return IESH_EINVAL;
    const int m = M / 2;
    std::vector<double> x, wt;
    legendre_nodes(m, x, wt);
    for (int i = 0; i < m; ++i) {
      eps[i] = 0.5 * (eps_f - a) * x[i] + 0.5 * (a + eps_f);
      w[i] = 0.5 * (eps_f - a) * wt[i];
      eps[m + i] = 0.5 * (b - eps_f) * x[i] + 0.5 * (eps_f + b);
      w[m + i] = 0.5 * (b - eps_f) * wt[i];
    }
    return IESH_OK;
  }
  return IESH_EINVAL;
}

// Bath of a workload: the band placed for the chemical potential, one or two
// leads on one grid, and the number of levels below mu.
int bath_levels(const iesh_bath_desc& d, double* eps, double* w, int32_t* lead,
                int32_t* n_below) {
  if (!eps || !w || !(d.W > 0.0) || !std::isfinite(d.W) || !std::isfinite(d.mu)) return IESH_EINVAL;
  if (d.n_leads != 1 && d.n_leads != 2) return IESH_EINVAL;
  if (d.M < d.n_leads || d.M % d.n_leads) return IESH_EINVAL;
  if (d.placement != IESH_BAND_CENTRED && d.placement != IESH_BAND_FIXED) return IESH_EINVAL;
  const double centre = d.placement == IESH_BAND_CENTRED ? d.mu : 0.0;
  const double a = centre - 0.5 * d.W, b = centre + 0.5 * d.W;
  const int Mg = d.M / d.n_leads;  // levels of the shared grid
  std::vector<double> ge(Mg), gw(Mg);
  const int rc = discretize(d.kind, Mg, a, b, d.mu, ge.data(), gw.data());
  if (rc) return rc;
  int below = 0;
  for (int k = 0; k < Mg; ++k)
    for (int l = 0; l < d.n_leads; ++l) {
      // each lead couples with Gamma / n_leads: every grid level appears once
      // per lead with that share of its weight, lead 0 first
      const int q = k * d.n_leads + l;
      eps[q] = ge[k];
      w[q] = gw[k] / d.n_leads;
      if (lead) lead[q] = l;
      below += ge[k] < d.mu ? 1 : 0;
    }
  if (n_below) *n_below = below;
  return IESH_OK;
}

}  // namespace iesh
