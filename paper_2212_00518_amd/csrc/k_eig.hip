// Arrowhead eigen-solver, couplings, Chebyshev set-up and velocity Verlet.
//
// The one-electron Hamiltonian of the Newns-Anderson model (Sec. II.B) is a
// symmetric arrowhead matrix: h on [0][0], the bath energies eps_k on the
// diagonal and the couplings V_k in row and column 0.  Its eigenvalues are
// the roots of the secular function
//     f(lambda) = lambda - h + sum_k V_k^2 / (eps_k - lambda),
// one below eps_0, one between each pair of neighbouring bath levels and one
// above eps_{M-1} (strict interlacing when every V_k != 0 and the levels are
// distinct; equal levels are deflated first, see ModelDev).  Each root is
// found relative to its nearest pole, tau = lambda - eps_o, so that the
// differences lambda_j - eps_k stay accurate for closely spaced levels; the
// iteration fits a two-pole rational model to f and f' at the current point
// (quadratic convergence) inside a bisection bracket.  Only the impurity
// components q0_j of the eigenvectors are kept, since every quantity of the
// step is a function of (lambda, q0) alone; q0_j^2 = 1 / f'(lambda_j) comes
// with the root's last secular evaluation (the bath components, which the
// lead weights of a biased start need, use couplings recomputed from the
// roots by the Loewner formula, for which the computed roots are exact):
//   G_jk = (Q^T dH/dx Q)_jk = q0_j q0_k (h' + rho (lambda_j + lambda_k - 2h)),
// with V_k(x) = Vbar_k f(x) and rho = f'/f (row 0 of the eigen-equation gives
// sum_k V_k Q_kj = (lambda_j - h) q0_j).
//
// One work-group per trajectory; 256 threads; every array lives in LDS.

#include "iesh_cheb.hpp"
#include "iesh_internal.hpp"

namespace iesh {
namespace {

constexpr int kEigThreads = 256;
static_assert(kEigThreads % 64 == 0, "whole waves: the secular solve relies on it");
// Register budget of the step kernels: 5 waves per SIMD (at most 96 VGPRs)
// fit without spills; the LDS of a work-group would allow 7.
constexpr int kEigWavesPerSimd = 5;
constexpr double kEps = 2.220446049250313e-16;

struct EigLds {
  double e[kMaxStates];      // bath energies
  double V2[kMaxStates];     // V_k(x)^2
  double tau[kMaxStates];    // root relative to its origin pole
  double Vh2[kMaxStates];    // Loewner couplings squared
  double q0[kMaxStates];     // impurity amplitudes
  double lam[kMaxStates];    // eigenvalues (eps_o + tau)
  double eo[kMaxStates];     // origin pole energy eps_o of each state (coupling build)
  double red[kEigThreads];   // reductions
  double red2[kEigThreads];
  int org[kMaxStates];       // origin pole index of each root
  int fail;
  int count;
  double sc[16];             // scalars
  double J[kMaxCheb];        // Bessel values J_0..J_K of the propagator
  double nuc[4][kMaxDof];    // half-step velocity, new, frozen-propagator geometry, force
};

// 1/d from the hardware reciprocal estimate and two Newton steps
// r <- r + r (1 - d r) (each squares the relative error).  Measured on gfx950
// over 4M values spanning 1e-9 .. 5e8: the estimate is within 4.7e-8, one
// step within 2.2e-15, two steps within 1.2e-16 (one unit in the last place).
// d != 0 at every call (poles are excluded from the root brackets, the
// secular poles are distinct and the roots interlace them strictly).
__device__ inline double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// The same with one Newton step (within 2.2e-15): the secular sums.
__device__ inline double rcp_nr1(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  return fma(r, fma(-d, r, 1.0), r);
}

// f and its split derivative at tau (origin eo); terms with k < j are left
// of the root.  j0 is the same for all lanes of the wave and no lane's j lies
// outside [j0, j0 + 64), so poles below j0 are left of every lane's root and
// poles from j0 + 64 on right of it: only the 64 poles between need the
// per-lane split.  Every point evaluated lies inside the root's gap, so a
// left term V_k^2 / (eps_k - lambda) is negative and a right one positive,
// and the sum of their moduli (for the rounding bound err) is the right sum
// minus the left sum outside the per-lane range.  Each term carries the
// one-step reciprocal's 2.2e-15, so f is known to about 3e-15 of that sum;
// err = 16 eps of it.  A root accurate to that is accurate to about 3e-15
// relative to its distance from the nearest pole.
// The same for a root whose pole sum is shared by a group of G lanes (G a
// power of two, the group's lanes adjacent and G > 1): lane g of the group
// sums the poles k = g, g + G, ... with the per-lane left/right split, and the
// group combines its partial sums (every lane of it gets the totals).  It
// serves the last, partly filled wave of roots, whose idle lanes would
// otherwise cost as many instructions as a full wave.
__device__ inline void secular_eval_group(int j, int g, int G, int M, const double* e,
                                          const double* V2, double eo, double emh, double tau,
                                          double& f, double& dl, double& dr, double& err) {
  double pl = 0.0, pr = 0.0, l = 0.0, r = 0.0;
  for (int k = g; k < M; k += G) {
    const double d = (e[k] - eo) - tau;
    const double inv = rcp_nr1(d);
    const double t = V2[k] * inv;
    if (k < j) {
      pl += t;
      l = fma(t, inv, l);
    } else {
      pr += t;
      r = fma(t, inv, r);
    }
  }
  for (int sh = 1; sh < G; sh <<= 1) {
    pl += __shfl_xor(pl, sh);
    pr += __shfl_xor(pr, sh);
    l += __shfl_xor(l, sh);
    r += __shfl_xor(r, sh);
  }
  f = emh + tau + (pl + pr);
  dl = l;
  dr = r;
  err = 16.0 * kEps * (fabs(emh) + fabs(tau) + (pr - pl));
}

__device__ inline void secular_eval(int j, int j0, int M, const double* e, const double* V2,
                                    double eo, double emh, double tau, double& f, double& dl,
                                    double& dr, double& err, int g = 0, int G = 1) {
  if (G > 1) {
    secular_eval_group(j, g, G, M, e, V2, eo, emh, tau, f, dl, dr, err);
    return;
  }
  double pl = 0.0, pm = 0.0, pr = 0.0, am = 0.0, l = 0.0, r = 0.0;
  const int k1 = min(j0, M), k2 = min(j0 + 64, M);
#pragma unroll 4
  for (int k = 0; k < k1; ++k) {
    const double d = (e[k] - eo) - tau;  // eps_k - lambda < 0
    const double inv = rcp_nr1(d);
    const double t = V2[k] * inv;
    pl += t;
    l = fma(t, inv, l);
  }
#pragma unroll 2
  for (int k = k1; k < k2; ++k) {
    const double d = (e[k] - eo) - tau;
    const double inv = rcp_nr1(d);
    const double t = V2[k] * inv;
    pm += t;
    am += fabs(t);
    if (k < j)
      l = fma(t, inv, l);
    else
      r = fma(t, inv, r);
  }
#pragma unroll 4
  for (int k = k2; k < M; ++k) {
    const double d = (e[k] - eo) - tau;  // eps_k - lambda > 0
    const double inv = rcp_nr1(d);
    const double t = V2[k] * inv;
    pr += t;
    r = fma(t, inv, r);
  }
  f = emh + tau + ((pl + pm) + pr);
  dl = l;
  dr = r;
  err = 16.0 * kEps * (fabs(emh) + fabs(tau) + ((pr - pl) + am));
}

// Root of a2 eta^2 + a1 eta + a0 inside (alpha, beta).
__device__ inline double quad_root_in(double a2, double a1, double a0, double alpha, double beta) {
  if (a2 == 0.0) return -a0 / a1;
  const double sq = sqrt(fmax(a1 * a1 - 4.0 * a2 * a0, 0.0));
  const double q = -0.5 * (a1 + copysign(sq, a1));
  const double r1 = q / a2;
  const double r2 = (q != 0.0) ? a0 / q : 0.0;
  const bool in1 = r1 > alpha && r1 < beta;
  const bool in2 = r2 > alpha && r2 < beta;
  if (in1 && in2) return fabs(r1) < fabs(r2) ? r1 : r2;
  if (in1) return r1;
  if (in2) return r2;
  return fabs(r1) < fabs(r2) ? r1 : r2;
}

// A step of the iteration shorter than this, relative to the new point, ends
// it without evaluating f there: near the root the error falls quadratically
// (the next error is about the step squared over the distance to the nearest
// pole, far below rounding), and f' at the accepted point differs from f' at
// the last evaluated one by about twice the step over that distance.
constexpr double kStepAccept = 1e-13;
// The same on the mixed path's step solves: the accepted root is still
// accurate to about the step squared (1e-18 relative), and f' (so Q0) to
// about 2e-9, far below the FP32 propagation's rounding; it saves the last
// evaluation of most roots.
constexpr double kStepAcceptMixed = 1e-9;

// Root j (0..M) of the secular function; j0 as in secular_eval.  Returns 1
// on convergence.  Warm start (dlt >= 0): the root is known to lie within dlt
// of lam_g (the same root of a nearby geometry, see solve_arrowhead); the
// bracket shrinks to that interval (intersected with the root's gap) and the
// iteration starts at the predicted root lam_s when that lies strictly inside
// it.  The origin pole is the near one when the interval lies on one side of
// the gap's midpoint, else the one on the predicted root's side: the root is
// then within dlt of the midpoint, about half a gap from either pole, and
// both origins give the differences eps_k - lambda to full relative accuracy.
// dsum_out: sum_k V_k^2 / (eps_k - lambda)^2 at the last point evaluated
// (within a relative 2 kStepAccept of the returned root, so f' there is f' at
// the root to about 1e-13).
__device__ int secular_root(int j, int j0, int M, const double* e, const double* V2, double h,
                            double vnorm, int max_it, double accept, double lam_g, double dlt, double lam_s,
                            double& tau_out, int& org_out, double& dsum_out, int g = 0, int G = 1) {
  int o;
  double lo, hi, tau, f = 0.0, dl = 0.0, dr = 0.0, err = 0.0;
  bool have_f = false;
  bool warm = dlt >= 0.0;
  if (warm && j > 0 && j < M) {
    const double mid = e[j - 1] + 0.5 * (e[j] - e[j - 1]);
    if (lam_g + dlt < mid) {
      o = j - 1;
      lo = fmax(0.0, (lam_g - dlt) - e[o]);
      hi = fmin(0.5 * (e[j] - e[j - 1]), (lam_g + dlt) - e[o]);
    } else if (lam_g - dlt > mid) {
      o = j;
      lo = fmax(-0.5 * (e[j] - e[j - 1]) * (1.0 + 4.0 * kEps), (lam_g - dlt) - e[o]);
      hi = fmin(0.0, (lam_g + dlt) - e[o]);
    } else if (lam_s < mid) {
      // the root may sit on either side of the midpoint; the gap's far pole
      // stays outside the bracket (the rounded pole difference is within half
      // a unit of the exact one)
      o = j - 1;
      lo = fmax(0.0, (lam_g - dlt) - e[o]);
      hi = fmin((e[j] - e[o]) * (1.0 - 4.0 * kEps), (lam_g + dlt) - e[o]);
    } else {
      o = j;
      lo = fmax((e[j - 1] - e[o]) * (1.0 - 4.0 * kEps), (lam_g - dlt) - e[o]);
      hi = fmin(0.0, (lam_g + dlt) - e[o]);
    }
  }
  if (warm && (j == 0 || j == M)) {
    o = (j == 0) ? 0 : M - 1;
    if (j == 0) {
      lo = fmax((fmin(h, e[0]) - vnorm) - e[0], (lam_g - dlt) - e[0]);
      hi = fmin(0.0, (lam_g + dlt) - e[0]);
    } else {
      lo = fmax(0.0, (lam_g - dlt) - e[M - 1]);
      hi = fmin((fmax(h, e[M - 1]) + vnorm) - e[M - 1], (lam_g + dlt) - e[M - 1]);
    }
  }
  if (warm) {
    // an empty interval (it cannot happen while the bound holds) falls back.
    // The start lies strictly inside the bracket: one end may be the origin
    // pole itself (tau = 0), where f is not defined, and a predicted start
    // can overshoot onto it near an avoided crossing; the previous root, else
    // the bracket's middle, replaces such a start.
    if (!(lo < hi)) {
      warm = false;
    } else {
      double t0 = lam_s - e[o];
      if (!(t0 > lo && t0 < hi)) t0 = lam_g - e[o];
      if (!(t0 > lo && t0 < hi)) t0 = 0.5 * (lo + hi);
      tau = t0;
    }
  }
  if (warm) {
  } else if (j == 0) {
    o = 0;
    lo = (fmin(h, e[0]) - vnorm) - e[0];
    hi = 0.0;
    tau = lo;
  } else if (j == M) {
    o = M - 1;
    lo = 0.0;
    hi = (fmax(h, e[M - 1]) + vnorm) - e[M - 1];
    tau = hi;
  } else {
    const double gap = e[j] - e[j - 1];
    const double half = 0.5 * gap;
    secular_eval(j, j0, M, e, V2, e[j - 1], e[j - 1] - h, half, f, dl, dr, err, g, G);
    if (f >= 0.0) {
      o = j - 1;
      lo = 0.0;
      hi = half;
      tau = half;
      have_f = true;
    } else {
      o = j;
      lo = -half * (1.0 + 4.0 * kEps);
      hi = 0.0;
      tau = lo;
    }
  }
  const double eo = e[o];
  const double emh = eo - h;
  int ok = 0;
  for (int it = 0; it < max_it; ++it) {
    if (!have_f) secular_eval(j, j0, M, e, V2, eo, emh, tau, f, dl, dr, err, g, G);
    have_f = false;
    dsum_out = dl + dr;
    if (f == 0.0 || fabs(f) <= err) {
      ok = 1;
      break;
    }
    if (f < 0.0)
      lo = tau;
    else
      hi = tau;
    double eta;
    if (j > 0 && j < M) {
      const double alpha = (e[j - 1] - eo) - tau;
      const double beta = (e[j] - eo) - tau;
      double s1, s2;
      if (o == j - 1) {
        s1 = alpha * alpha * dl;
        s2 = beta * beta * (dr + 1.0);
      } else {
        s1 = alpha * alpha * (dl + 1.0);
        s2 = beta * beta * dr;
      }
      const double c = f - s1 / alpha - s2 / beta;
      eta = quad_root_in(c, -(c * (alpha + beta) + s1 + s2), alpha * beta * f, alpha, beta);
    } else if (j == 0) {
      const double beta = -tau;
      const double s = V2[0];
      const double L = 1.0 + (dr - s / (beta * beta));
      const double c0 = f - s / beta;
      const double B = L * beta - c0;
      const double sq = sqrt(fmax(B * B + 4.0 * L * beta * f, 0.0));
      eta = (B > 0.0) ? (-2.0 * beta * f / (B + sq)) : ((B - sq) / (2.0 * L));
    } else {
      const double alpha = -tau;
      const double s = V2[M - 1];
      const double L = 1.0 + (dl - s / (alpha * alpha));
      const double c0 = f - s / alpha;
      const double B = L * alpha - c0;
      const double sq = sqrt(fmax(B * B + 4.0 * L * alpha * f, 0.0));
      eta = (B < 0.0) ? (2.0 * alpha * f / (sq - B)) : ((B + sq) / (2.0 * L));
    }
    double tn = tau + eta;
    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    if (fabs(tn - tau) <= accept * fabs(tn) ||
        hi - lo <= 2.0 * kEps * fmax(fabs(lo), fabs(hi))) {
      tau = tn;
      ok = 1;
      break;
    }
    tau = tn;
  }
  tau_out = tau;
  org_out = o;
  return ok;
}

// Roots of a trajectory's last arrowhead solve (per secular root, before
// the deflated states are placed) and that solve's geometry, to start the
// next solve from (keyed by the trajectory's home index).
struct RootStore {
  double* tau;     // [n_pad] root relative to its origin pole
  double* q0;      // [n_pad] impurity component of the root's eigenvector
  int32_t* org;    // [n_pad] origin pole
  double* geo;     // [4]: h, f, valid (1), unused
};

__device__ inline RootStore root_store(const ClassDev& c, int t) {
  const size_t hm = (size_t)c.home[t], np = c.md.n_pad;
  return RootStore{c.root_tau + hm * 2 * np, c.root_tau + hm * 2 * np + np, c.root_org + hm * np,
                   c.root_geo + 4 * hm};
}

// Solve the arrowhead problem of geometry x; fills lam, tau, org, q0 in LDS
// (entries n..n_pad-1 of lam/q0 set to 0).  Returns model scalars.
// The eigenvector of root lambda_j is proportional to (1, V_k / (lambda_j -
// eps_k)), so its impurity component is q0_j = f'(lambda_j)^(-1/2), read off
// the secular iteration's last evaluation; the pole-relative differences it
// sums are the same ones the root was found from.  kLoewner also leaves the
// Loewner couplings (the couplings for which the computed roots are exact,
// which give the bath components of the eigenvectors) in L.Vh2.
// rs (may be null): warm = start every root from the stored one of the last
// solve, store = keep this solve's roots there.  By Weyl's inequality each
// eigenvalue moves by at most ||H' - H||_2 <= |dh| + ||dV|| between the two
// geometries (the bath energies are fixed and V = Vbar f(x), so
// ||dV|| = |df| ||Vbar||); with that bound, doubled, every root gets a bracket
// that contains it, and the safeguarded iteration converges in a couple of
// steps instead of starting from the gap.
template <bool kLoewner = false>
__device__ ModelAt solve_arrowhead(const ModelDev& md, const double* __restrict__ vbar,
                                   const double* x, EigLds& L, RootStore rs = RootStore{},
                                   bool warm = false, bool store = false,
                                   double accept = kStepAccept) {
  // the secular problem over the distinct bath energies (M = M_red poles,
  // M + 1 roots); repeated energies are expanded into deflated states below
  const int M = md.M_red, n = M + 1, tid = threadIdx.x;
  const ModelAt ma = model_at(md, x);
  for (int k = tid; k < M; k += kEigThreads) {
    const double V = vbar[k] * ma.f;
    L.V2[k] = V * V;
  }
  __syncthreads();
  // ||V||^2 (fixed-order reduction)
  double part = 0.0;
  for (int k = tid; k < M; k += kEigThreads) part += L.V2[k];
  L.red[tid] = part;
  __syncthreads();
  for (int s = kEigThreads / 2; s > 0; s >>= 1) {
    if (tid < s) L.red[tid] += L.red[tid + s];
    __syncthreads();
  }
  const double vnorm = sqrt(L.red[0]);
  __syncthreads();
  // warm start: the bound on how far every root moved since the stored solve,
  // and the first-order move of each (q_j^T (H' - H) q_j with the stored
  // vectors: dh q0_j^2 + 2 q0_j^2 (lambda_j - h) df / f, since
  // sum_k V_k Q_kj = (lambda_j - h) q0_j) as the starting point
  double dlt = -1.0, dh0 = 0.0, dfr = 0.0, h0 = 0.0;
  if (rs.geo && warm && rs.geo[2] == 1.0) {
    h0 = rs.geo[0];
    dh0 = ma.h - h0;
    const double df = ma.f - rs.geo[1];
    dfr = rs.geo[1] != 0.0 ? df / rs.geo[1] : 0.0;  // f = 0: no coupling, no move from V
    const double bound = fabs(dh0) + fabs(df) * (vnorm / ma.f);
    dlt = 2.0 * bound + 64.0 * kEps * (fabs(ma.h) + vnorm + fabs(L.e[0]) + fabs(L.e[M - 1]));
  }
  // A wave solves the 64 consecutive roots from jb.  In the last, partly
  // filled wave (T < 64 roots) groups of G lanes share a root's pole sums,
  // G the largest power of two with G T <= 64; lane g == 0 of a group keeps
  // the result.
  const int lane = tid & 63;
  for (int jb = tid - lane; jb < n; jb += kEigThreads) {
    const int T = min(64, n - jb);
    int G = 1;
    while (2 * G * T <= 64) G *= 2;
    const int j = jb + lane / G, g = lane & (G - 1);
    if (j >= jb + T) continue;
    double tau;
    int o;
    double lam_g = 0.0, lam_s = 0.0;
    if (dlt >= 0.0) {
      lam_g = L.e[rs.org[j]] + rs.tau[j];
      const double q2 = rs.q0[j] * rs.q0[j];
      lam_s = lam_g + q2 * (dh0 + 2.0 * (lam_g - h0) * dfr);
    }
    double dsum = 0.0;
    const int ok = secular_root(j, jb, M, L.e, L.V2, ma.h, vnorm, md.eig_iter, accept, lam_g, dlt, lam_s, tau,
                                o, dsum, g, G);
    if (g == 0) {
      L.tau[j] = tau;
      L.org[j] = o;
      L.lam[j] = L.e[o] + tau;
      L.q0[j] = 1.0 / sqrt(1.0 + dsum);
      if (!ok) atomicOr(&L.fail, 1);
      if (rs.geo && store) {
        rs.tau[j] = tau;
        rs.q0[j] = L.q0[j];
        rs.org[j] = o;
      }
    }
  }
  __syncthreads();
  if (rs.geo && store && tid == 0) {
    rs.geo[0] = ma.h;
    rs.geo[1] = ma.f;
    rs.geo[2] = L.fail ? 0.0 : 1.0;
  }
  // Loewner couplings: Vh_k^2 = -prod_j (e_k - lambda_j) / prod_{l != k} (e_k - e_l),
  // factors paired so that each ratio stays near 1.
  // The factors are taken in the order of l; as in the secular sums, only the
  // 64 indices l inside the wave's own range [k0, k0 + 64) need the per-lane
  // choice between the two forms.
  if constexpr (kLoewner) {
  for (int k = tid; k < M; k += kEigThreads) {
    const int k0 = __builtin_amdgcn_readfirstlane(k - (tid & 63));
    const int l1 = min(k0, M), l2 = min(k0 + 64, M);
    const double ek = L.e[k];
    const double dk = (ek - L.e[L.org[k]]) - L.tau[k];            // e_k - lambda_k  > 0
    const double dk1 = (ek - L.e[L.org[k + 1]]) - L.tau[k + 1];   // e_k - lambda_k+1 < 0
    double prod = dk * (-dk1);
    for (int l = 0; l < l1; ++l)
      prod *= ((ek - L.e[L.org[l]]) - L.tau[l]) * rcp_nr(ek - L.e[l]);
    for (int l = l1; l < l2; ++l) {
      if (l < k) {
        prod *= ((ek - L.e[L.org[l]]) - L.tau[l]) * rcp_nr(ek - L.e[l]);
      } else if (l > k) {
        prod *= ((L.e[L.org[l + 1]] - ek) + L.tau[l + 1]) * rcp_nr(L.e[l] - ek);
      }
    }
    for (int l = l2; l < M; ++l)
      prod *= ((L.e[L.org[l + 1]] - ek) + L.tau[l + 1]) * rcp_nr(L.e[l] - ek);
    L.Vh2[k] = prod;
  }
  }
  for (int j = md.n + tid; j < md.n_pad; j += kEigThreads) {
    L.q0[j] = 0.0;
    L.lam[j] = 0.0;
  }
  __syncthreads();
  if (md.expand) {
    // deflation: adiabatic state j is secular root r = expand[j] or, for
    // expand[j] = -(m + 1), the eigenstate at pole m with no impurity part
    constexpr int kPer = (kMaxStates + kEigThreads - 1) / kEigThreads;
    double tq[kPer], tt[kPer];
    int to[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int j = tid + i * kEigThreads;
      tq[i] = 0.0;
      tt[i] = 0.0;
      to[i] = 0;
      if (j < md.n) {
        const int r = md.expand[j];
        if (r >= 0) {
          tq[i] = L.q0[r];
          tt[i] = L.tau[r];
          to[i] = L.org[r];
        } else {
          to[i] = -r - 1;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int j = tid + i * kEigThreads;
      if (j < md.n) {
        L.q0[j] = tq[i];
        L.tau[j] = tt[i];
        L.org[j] = to[i];
        L.lam[j] = L.e[to[i]] + tt[i];
      }
    }
    __syncthreads();
  }
  return ma;
}

// lambda_k - lambda_j from the pole-relative representation.
__device__ inline double lam_diff(const EigLds& L, int k, int j) {
  return (L.e[L.org[k]] - L.e[L.org[j]]) + (L.tau[k] - L.tau[j]);
}

__device__ void write_model_geo(double* geo, const ModelAt& ma) {
  geo[GEO_H] = ma.h;
  geo[GEO_DH] = ma.dh;
  geo[GEO_RHO] = ma.rho;
  geo[GEO_U0] = ma.U0;
  geo[GEO_DU0] = ma.dU0;
}

// Hellmann-Feynman force of the occupied set at the geometry held in L.
__device__ double hf_force(const ModelDev& md, const ModelAt& ma, const int32_t* occ, EigLds& L) {
  const int tid = threadIdx.x;
  double part = 0.0;
  if (tid < md.N) {
    const int a = occ[tid];
    part = L.q0[a] * L.q0[a] * (ma.dh + 2.0 * ma.rho * (L.lam[a] - ma.h));
  }
  L.red2[tid] = part;
  __syncthreads();
  for (int s = kEigThreads / 2; s > 0; s >>= 1) {
    if (tid < s) L.red2[tid] += L.red2[tid + s];
    __syncthreads();
  }
  const double F = -ma.dU0 - L.red2[0];
  __syncthreads();
  return F;
}

// Hellmann-Feynman force on every coordinate of the multi-coordinate model at
// geometry x (held in L): F_nu = -dU0/dR_nu - sum_occ q0^2 (dh_nu + 2 rho_nu (lambda - h)),
// into F[0 .. ndof) (every thread gets the same values).
__device__ void hf_force_multi(const ModelDev& md, const ModelAt& ma, const double* x,
                               const int32_t* occ, EigLds& L, double* F) {
  const int tid = threadIdx.x;
  double p1 = 0.0, p2 = 0.0;
  if (tid < md.N) {
    const int a = occ[tid];
    const double q2 = L.q0[a] * L.q0[a];
    p1 = q2;
    p2 = q2 * (L.lam[a] - ma.h);
  }
  L.red[tid] = p1;
  L.red2[tid] = p2;
  __syncthreads();
  for (int s = kEigThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      L.red[tid] += L.red[tid + s];
      L.red2[tid] += L.red2[tid + s];
    }
    __syncthreads();
  }
  const double s1 = L.red[0], s2 = L.red2[0];
  __syncthreads();
  for (int nu = 0; nu < md.ndof; ++nu) {
    double dh, rho, dU0;
    multi_dof_grad(md, x, nu, dh, rho, dU0);
    F[nu] = -dU0 - dh * s1 - 2.0 * rho * s2;
  }
}

// Per-coordinate gradients into geo (coordinate 0 also in the scalar slots)
// and, with several coordinates, v.grad h and v.grad f / f for the velocity v.
__device__ void write_geo_grads(double* geo, const ModelDev& md, const ModelAt& ma, const double* x,
                                const double* v) {
  if (md.kind == IESH_MODEL_MULTI_DOF) {
    double vdh = 0.0, vrho = 0.0;
    for (int nu = 0; nu < md.ndof; ++nu) {
      multi_dof_grad(md, x, nu, geo[GEO_DHV + nu], geo[GEO_RHOV + nu], geo[GEO_DU0V + nu]);
      vdh += v[nu] * geo[GEO_DHV + nu];
      vrho += v[nu] * geo[GEO_RHOV + nu];
    }
    geo[GEO_VDH] = vdh;
    geo[GEO_VRHO] = vrho;
  } else {
    geo[GEO_DHV] = ma.dh;
    geo[GEO_RHOV] = ma.rho;
    geo[GEO_DU0V] = ma.dU0;
  }
}

__device__ void load_bath(const ClassDev& c, EigLds& L) {
  for (int k = threadIdx.x; k < c.md.M_red; k += kEigThreads) L.e[k] = c.eps[k];
  if (threadIdx.x == 0) {
    L.fail = 0;
    L.count = 0;
  }
  __syncthreads();
}

// One step for one trajectory up to (not including) the propagation.
// sub = -1: the whole step (midpoint geometry for the propagator, then the
// end point); sub = j in [0, nsub): only the propagator of electronic
// sub-step j, frozen at x_n + (j + 1/2)/nsub (x_{n+1} - x_n) for dt/nsub;
// sub = -2: only the end point (after the sub-steps).
__device__ void eig_step_one(const ClassDev& c, int t, double dt_run, int precision, Counters* cnt,
                             int sub, int nsub, EigLds& L) {
  const int tid = threadIdx.x;
  if (t >= live_slots(c) || (c.status[t] & kFreezeMask)) return;
  const double dt = c.clock ? c.clock[2 * (size_t)t] : dt_run;  // this trajectory's step
  const ModelDev& md = c.md;
  load_bath(c, L);
  const int nd = md.ndof;
  if (tid < nd) {
    const int nu = tid;
    double vh, xn, x;
    if (c.path) {
      // prescribed path (one coordinate): v over the step from the two end points
      const double* pp = c.path + (size_t)c.gtraj[t] * c.path_len + c.path_n;
      x = pp[0];
      xn = pp[1];
      vh = (xn - x) / dt;
    } else {
      x = c.x[(size_t)t * nd + nu];
      const double v = c.v[(size_t)t * nd + nu], F = c.F[(size_t)t * nd + nu];
      vh = v + 0.5 * dt * F / md.mass_dof[nu];
      xn = x + dt * vh;
    }
    L.nuc[0][nu] = vh;
    L.nuc[1][nu] = xn;
    L.nuc[2][nu] = (sub >= 0) ? x + ((sub + 0.5) / nsub) * (xn - x) : 0.5 * (x + xn);
  }
  __syncthreads();
  const double vh = L.nuc[0][0];
  const double dte = (sub >= 0) ? dt / nsub : dt;  // electronic step of this propagator

  const int n = md.n, n_pad = md.n_pad, RT = n_pad / 16;
  if (sub != -2) {
  // ---- midpoint geometry: couplings for the propagator
  // warm starts from the trajectory's previous solve (not along prescribed
  // paths, whose backward pass revisits steps out of order)
  const bool warm = c.root_tau && !c.path;
  // the mixed path's step solves stop the secular iteration earlier (not
  // along prescribed paths, whose gradients are FP64)
  const double accept = (precision == IESH_FP64 || c.path) ? kStepAccept : kStepAcceptMixed;
  RootStore rs{};
  if (warm) rs = root_store(c, t);
  ModelAt mm = solve_arrowhead(md, c.vbar, L.nuc[2], L, rs, warm, warm, accept);
  double vfac = vh;
  if (nd > 1) {
    // v . D over the coordinates: the gradients enter through v.grad h and v.grad f / f
    double dhe = 0.0, rhoe = 0.0;
    for (int nu = 0; nu < nd; ++nu) {
      double dh, rho, dU0;
      multi_dof_grad(md, L.nuc[2], nu, dh, rho, dU0);
      dhe += L.nuc[0][nu] * dh;
      rhoe += L.nuc[0][nu] * rho;
    }
    mm.dh = dhe;
    mm.rho = rhoe;
    vfac = 1.0;
  }
  double* Bt = c.Bt + (size_t)t * n_pad * n_pad;
  float* Bt32 = c.Bt32 ? c.Bt32 + (size_t)t * n_pad * n_pad : nullptr;
  double lo_part = 1e300, hi_part = -1e300;
  for (int k = tid; k < n; k += kEigThreads) L.eo[k] = L.e[L.org[k]];
  __syncthreads();
  for (int j = tid; j < n_pad; j += kEigThreads) {
    const int lane_off = ((j >> 4) << 6) + (j & 15);
    // v D[j][k] = q0_k (a_j + b_j (lambda_k - h)) / (lambda_k - lambda_j) with
    // a_j = v q0_j (h' + rho (lambda_j - h)) and b_j = v q0_j rho, since
    // G_jk = q0_j q0_k (h' + rho (lambda_j + lambda_k - 2h)); q0 = 0 on the
    // padding rows.  Zero where the numerator vanishes: deflated states (no
    // impurity part), possibly degenerate with each other.
    const double q0j = L.q0[j];
    const double aj = vfac * q0j * (mm.dh + mm.rho * (L.lam[j] - mm.h));
    const double bj = vfac * q0j * mm.rho;
    const double eoj = (j < n) ? L.eo[j] : 0.0, tj = (j < n) ? L.tau[j] : 0.0;
    double rsum = 0.0;
    for (int k = 0; k < n_pad; ++k) {
      double val = 0.0;
      if (k < n) {
        const double num = L.q0[k] * fma(bj, L.lam[k] - mm.h, aj);
        const double dif = (L.eo[k] - eoj) + (L.tau[k] - tj);  // lambda_k - lambda_j
        val = (num == 0.0 || k == j) ? 0.0 : num * rcp_nr1(dif);
      }
      rsum += fabs(val);
      // element (j, k) of the tile-ordered matrix: the part set by k is the
      // same for every lane, so the stores take a uniform base and a fixed
      // per-lane offset (n_pad^2 < 2^31)
      const int koff = (((k >> 2) * RT) << 6) + ((k & 3) << 4);
      if (precision == IESH_FP64)
        (Bt + koff)[lane_off] = val;
      else
        (Bt32 + koff)[lane_off] = (float)val;
    }
    if (j < n) {
      lo_part = fmin(lo_part, L.lam[j] - rsum);
      hi_part = fmax(hi_part, L.lam[j] + rsum);
    }
    c.lam_mid[(size_t)t * n_pad + j] = (j < n) ? L.lam[j] : 0.0;
  }
  L.red[tid] = lo_part;
  L.red2[tid] = hi_part;
  __syncthreads();
  for (int s = kEigThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      L.red[tid] = fmin(L.red[tid], L.red[tid + s]);
      L.red2[tid] = fmax(L.red2[tid], L.red2[tid + s]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    double* cb = c.cheb + (size_t)t * kChebStride;
    if (write_cheb(cb, L.red[0], L.red2[0], dte, precision, cnt, sub <= 0, L.J, c.work) < 0)
      atomicOr(&L.fail, 2);
  }
  __syncthreads();
  }
  if (sub >= 0) {
    // a sub-step's failure freezes the trajectory before its propagation
    if (tid == 0 && L.fail) c.status[t] |= IESH_TRAJ_NONCONV;
    return;
  }

  // ---- end-point geometry: energies, amplitudes, forces
  const bool warm_end = c.root_tau && !c.path;
  RootStore rse{};
  if (warm_end) rse = root_store(c, t);
  const ModelAt mn = solve_arrowhead(md, c.vbar, L.nuc[1], L, rse, warm_end, warm_end,
                                     (precision == IESH_FP64 || c.path) ? kStepAccept : kStepAcceptMixed);
  for (int j = tid; j < n_pad; j += kEigThreads) {
    c.lam[(size_t)t * n_pad + j] = L.lam[j];
    c.q0[(size_t)t * n_pad + j] = L.q0[j];
  }
  double Fv[kMaxDof];
  if (nd == 1)
    Fv[0] = hf_force(md, mn, c.occ + (size_t)t * md.N, L);
  else
    hf_force_multi(md, mn, L.nuc[1], c.occ + (size_t)t * md.N, L, Fv);
  if (tid == 0) {
    double* geo = c.geo + (size_t)t * kGeoStride;
    write_model_geo(geo, mn);
    int st = c.status[t];
    double vnv[kMaxDof];
    for (int nu = 0; nu < nd; ++nu) {
      const double xn = L.nuc[1][nu];
      const double vn = L.nuc[0][nu] + 0.5 * dt * Fv[nu] / md.mass_dof[nu];
      vnv[nu] = vn;
      c.x[(size_t)t * nd + nu] = xn;
      c.v[(size_t)t * nd + nu] = vn;
      c.F[(size_t)t * nd + nu] = Fv[nu];
      if (!isfinite(xn) || !isfinite(vn)) st |= IESH_TRAJ_NONFINITE;
    }
    write_geo_grads(geo, md, mn, L.nuc[1], vnv);
    if (L.fail & 1) st |= IESH_TRAJ_NONCONV;
    if (L.fail & 2) st |= IESH_TRAJ_NONCONV;
    c.status[t] = st;
  }
}

__global__ __launch_bounds__(kEigThreads) __attribute__((amdgpu_waves_per_eu(kEigWavesPerSimd))) void k_eig_step(ClassDev c, double dt_run, int precision,
                                                           Counters* cnt, int sub, int nsub) {
  __shared__ EigLds L;
  eig_step_one(c, blockIdx.x, dt_run, precision, cnt, sub, nsub, L);
}

// The same step for several arrowhead classes in one launch: block b works
// on slot b - first[k] of class k (first[k] <= b < first[k + 1]).  The classes
// come largest first, so the dispatcher hands out the long work-groups
// first and the small classes fill the compute units behind them.
__global__ __launch_bounds__(kEigThreads) __attribute__((amdgpu_waves_per_eu(kEigWavesPerSimd))) void k_eig_fused(ClassSet set, double dt_run, int precision,
                                                            Counters* cnt, int sub, int nsub) {
  __shared__ EigLds L;
  const int b = blockIdx.x;
  int k = 0;
  while (k + 1 < set.n && b >= set.first[k + 1]) ++k;
  eig_step_one(set.c[k], b - set.first[k], dt_run, precision, cnt, sub, nsub, L);
}

// Eigen-solve at the current x (no dynamics): energies, amplitudes, model
// scalars; mode 1 also refreshes the force of the current occupations.
__global__ __launch_bounds__(kEigThreads) void k_eig_query(ClassDev c, int t0, int mode) {
  __shared__ EigLds L;
  const int t = t0 + blockIdx.x;
  const int tid = threadIdx.x;
  const ModelDev& md = c.md;
  load_bath(c, L);
  const int nd = md.ndof;
  if (tid < nd) L.nuc[1][tid] = c.x[(size_t)t * nd + tid];
  __syncthreads();
  // a state upload (mode 1) keeps the roots for the warm start of the first
  // step; a plain query leaves the stored ones, so queries do not change the
  // dynamics
  RootStore rs{};
  const bool store = mode == 1 && c.root_tau && !c.path;
  if (store) rs = root_store(c, t);
  const ModelAt ma = solve_arrowhead(md, c.vbar, L.nuc[1], L, rs, false, store);
  for (int j = tid; j < md.n_pad; j += kEigThreads) {
    c.lam[(size_t)t * md.n_pad + j] = L.lam[j];
    c.q0[(size_t)t * md.n_pad + j] = L.q0[j];
  }
  if (tid == 0) {
    write_model_geo(c.geo + (size_t)t * kGeoStride, ma);
    write_geo_grads(c.geo + (size_t)t * kGeoStride, md, ma, L.nuc[1], c.v + (size_t)t * nd);
  }
  if (mode == 1) {
    double Fv[kMaxDof];
    if (nd == 1)
      Fv[0] = hf_force(md, ma, c.occ + (size_t)t * md.N, L);
    else
      hf_force_multi(md, ma, L.nuc[1], c.occ + (size_t)t * md.N, L, Fv);
    if (tid == 0) {
      for (int nu = 0; nu < nd; ++nu) c.F[(size_t)t * nd + nu] = Fv[nu];
      if (L.fail) c.status[t] |= IESH_TRAJ_NONCONV;
    }
  }
}

__device__ inline double fermi_fn(double e, double mu, double kT) {
  const double z = (e - mu) / kT;
  return (z > 0.0) ? exp(-z) / (1.0 + exp(-z)) : 1.0 / (1.0 + exp(z));
}

// Occupation probability of orbital a at chemical potential mu: one Fermi
// function, or with a bias V the weighted mix of the impurity (mu) and the
// two leads (mu +- V/2); w0 = lead-0 weight of the orbital.
__device__ inline double occ_prob(const EigLds& L, int a, double mu, double kT, double bias) {
  if (bias == 0.0) return fermi_fn(L.lam[a], mu, kT);
  const double q2 = L.q0[a] * L.q0[a], w0 = L.V2[a], w1 = 1.0 - q2 - w0;
  return q2 * fermi_fn(L.lam[a], mu, kT) + w0 * fermi_fn(L.lam[a], mu + 0.5 * bias, kT) +
         w1 * fermi_fn(L.lam[a], mu - 0.5 * bias, kT);
}

// Lead-0 weight of every adiabatic state into L.V2 (free after the solve):
// a secular root j has bath components Vh_m q0_j / (lambda_j - e_m) on the
// coupled combination of pole m, of which the share lead0[m] lies on lead 0;
// a deflated state at pole m takes lead0[M_red + m].
__device__ void lead_weights(const ModelDev& md, EigLds& L) {
  const int Mr = md.M_red;
  for (int j = threadIdx.x; j < md.n; j += kEigThreads) {
    const int r = md.expand ? md.expand[j] : j;
    double w0;
    if (r < 0) {
      w0 = md.lead0[Mr - r - 1];
    } else {
      const double eo = L.e[L.org[j]], tj = L.tau[j];
      double s = 0.0;
      for (int m = 0; m < Mr; ++m) {
        const double id = rcp_nr((L.e[m] - eo) - tj);
        s += md.lead0[m] * L.Vh2[m] * (id * id);
      }
      w0 = L.q0[j] * L.q0[j] * s;
    }
    L.V2[j] = w0;
  }
  __syncthreads();
}

// Initial occupations at kT (fixed N) and unit-vector orbitals.
__global__ __launch_bounds__(kEigThreads) void k_init_thermal(ClassDev c, double kT, double bias,
                                                              uint64_t seed) {
  __shared__ EigLds L;
  const int t = blockIdx.x;
  const int tid = threadIdx.x;
  const ModelDev& md = c.md;
  const int n = md.n, N = md.N;
  load_bath(c, L);
  if (tid < md.ndof) L.nuc[1][tid] = c.x[(size_t)t * md.ndof + tid];
  __syncthreads();
  RootStore rs{};
  const bool store = c.root_tau && !c.path;
  if (store) rs = root_store(c, t);
  const ModelAt ma = solve_arrowhead<true>(md, c.vbar, L.nuc[1], L, rs, false, store);
  int32_t* occ = c.occ + (size_t)t * N;
  __shared__ int chosen[kMaxStates];
  bool done = false;
  if (kT > 0.0) {
    if (bias != 0.0) lead_weights(md, L);
    // chemical potential by bisection on sum_a f_a = N
    double lo = L.lam[0] - 50.0 * kT - 1.0 - fabs(bias);
    double hi = L.lam[n - 1] + 50.0 * kT + 1.0 + fabs(bias);
    for (int it = 0; it < 200; ++it) {
      const double mu = 0.5 * (lo + hi);
      double part = 0.0;
      for (int a = tid; a < n; a += kEigThreads) part += occ_prob(L, a, mu, kT, bias);
      L.red[tid] = part;
      __syncthreads();
      for (int s = kEigThreads / 2; s > 0; s >>= 1) {
        if (tid < s) L.red[tid] += L.red[tid + s];
        __syncthreads();
      }
      if (L.red[0] > (double)N)
        hi = mu;
      else
        lo = mu;
      __syncthreads();
    }
    const double mu = 0.5 * (lo + hi);
    const uint32_t gt = (uint32_t)c.gtraj[t];
    for (int attempt = 0; attempt < 4096 && !done; ++attempt) {
      int cnt = 0;
      for (int a = tid; a < n; a += kEigThreads) {
        const double fa = occ_prob(L, a, mu, kT, bias);
        const double u = philox_uniform(seed, gt, (uint64_t)attempt * n + a, 1u);
        chosen[a] = (u < fa) ? 1 : 0;
        cnt += chosen[a];
      }
      L.red[tid] = (double)cnt;
      __syncthreads();
      for (int s = kEigThreads / 2; s > 0; s >>= 1) {
        if (tid < s) L.red[tid] += L.red[tid + s];
        __syncthreads();
      }
      done = ((int)L.red[0] == N);
      __syncthreads();
    }
  }
  if (tid == 0) {
    int r = 0;
    for (int a = 0; a < n; ++a) {
      if (done ? chosen[a] : (a < N)) occ[r++] = a;
    }
  }
  __syncthreads();
  // orbitals: column j = unit vector of occ[j]
  for (int idx = tid; idx < N * md.n_pad; idx += kEigThreads) {
    const int j = idx / md.n_pad, i = idx % md.n_pad;
    const double val = (i == occ[j]) ? 1.0 : 0.0;
    if (c.C64) {
      c.C64[((size_t)t * N * md.n_pad + idx) * 2] = val;
      c.C64[((size_t)t * N * md.n_pad + idx) * 2 + 1] = 0.0;
    }
    if (c.C32) {
      c.C32[((size_t)t * N * md.n_pad + idx) * 2] = (float)val;
      c.C32[((size_t)t * N * md.n_pad + idx) * 2 + 1] = 0.0f;
    }
  }
  for (int j = tid; j < md.n_pad; j += kEigThreads) {
    c.lam[(size_t)t * md.n_pad + j] = L.lam[j];
    c.q0[(size_t)t * md.n_pad + j] = L.q0[j];
  }
  const int nd = md.ndof;
  double Fv[kMaxDof];
  if (nd == 1)
    Fv[0] = hf_force(md, ma, occ, L);
  else
    hf_force_multi(md, ma, L.nuc[1], occ, L, Fv);
  if (tid == 0) {
    write_model_geo(c.geo + (size_t)t * kGeoStride, ma);
    write_geo_grads(c.geo + (size_t)t * kGeoStride, md, ma, L.nuc[1], c.v + (size_t)t * nd);
    for (int nu = 0; nu < nd; ++nu) c.F[(size_t)t * nd + nu] = Fv[nu];
    c.status[t] = L.fail ? IESH_TRAJ_NONCONV : 0;
  }
}

// ---------------------------------------------------------------------------
// Reverse mode through the eigen-solve (adjoint along prescribed paths;
// harmonic model: V_k constant, rho = 0).  With the gauge q0_j > 0 the
// impurity amplitude is a function of the root alone, q0_j = f'(lambda_j)^{-1/2}
// with f'(l) = 1 + sum_k V_k^2 / (l - eps_k)^2, and the roots follow from
// f(lambda_j) = 0 by the implicit function theorem:
//   d lambda_j / dh = q0_j^2,  d lambda_j / dV_k = 2 V_k q0_j^2 / (lambda_j - eps_k),
//   d lambda_j / d eps_k = V_k^2 q0_j^2 / (lambda_j - eps_k)^2.
// So cotangents (lbar, qbar) of (lambda, q0) map to (h, V, eps) in O(n M).
// Gradient layout per trajectory: [eps_d, Gamma, eps_1 .. eps_M, omega, g, dG].

struct AdjLds {
  EigLds L;
  double lbar[kMaxStates];
  double qbar[kMaxStates];
  double fb[kMaxStates];  // cotangent of f'(lambda_j)
  double red3[kEigThreads];
};

// lambda_j - eps_k from the pole-relative representation.
__device__ inline double lam_minus_eps(const EigLds& L, int j, int k) {
  return -((L.e[k] - L.e[L.org[j]]) - L.tau[j]);
}

__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = kEigThreads / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Accumulate into grad the parameter cotangents of one eigen-solve at x whose
// (lambda, q0) cotangents are in A.lbar, A.qbar, plus hpbar for h' = dh/dx.
__device__ void eig_backprop(const ModelDev& md, const ModelAt& ma, double x, AdjLds& A,
                             double hpbar, double* grad) {
  const EigLds& L = A.L;
  const int n = md.n, M = md.M, tid = threadIdx.x;
  // f' cotangent and the total lambda cotangent
  for (int j = tid; j < n; j += kEigThreads) {
    double s3 = 0.0;
    for (int k = 0; k < M; ++k) {
      const double d = lam_minus_eps(L, j, k);
      s3 += L.V2[k] / (d * d * d);
    }
    const double q = L.q0[j];
    const double fb = -0.5 * A.qbar[j] * q * q * q;
    A.fb[j] = fb;
    A.lbar[j] += fb * (-2.0 * s3);
  }
  __syncthreads();
  double hpart = 0.0;
  for (int j = tid; j < n; j += kEigThreads) hpart += A.lbar[j] * L.q0[j] * L.q0[j];
  const double hbar = block_sum(hpart, A.red3);
  double gpart = 0.0;
  for (int k = tid; k < M; k += kEigThreads) {
    const double V = sqrt(L.V2[k]);
    double vb = 0.0, eb = 0.0;
    for (int j = 0; j < n; ++j) {
      const double d = lam_minus_eps(L, j, k);
      const double q2 = L.q0[j] * L.q0[j];
      const double lb = A.lbar[j], fb = A.fb[j];
      vb += lb * 2.0 * V * q2 / d + fb * 2.0 * V / (d * d);
      eb += lb * L.V2[k] * q2 / (d * d) + fb * 2.0 * L.V2[k] / (d * d * d);
    }
    grad[2 + k] += eb;
    gpart += vb * V / (2.0 * md.Gamma);
  }
  const double Gbar = block_sum(gpart, A.red3);
  if (tid == 0) {
    const double omega = md.p[0], g = md.p[1], m = md.mass;
    grad[0] += hbar;
    grad[1] += Gbar;
    grad[2 + M] += hbar * m * omega * (g * g - 2.0 * g * x) + hpbar * (-2.0 * m * omega * g);
    grad[3 + M] += hbar * m * omega * omega * (g - x) + hpbar * (-m * omega * omega);
    grad[4 + M] += hbar;
  }
  __syncthreads();
}

// Explicit terms of the loss at x_s (end of step s - 1, s = 1 .. T) for one
// trajectory: Gh += w c_P q0 z^T / T (z = C^T q0) and, at s = T,
// w c_E diag(lambda) C; the force term adds to the q0 and h' cotangents, the
// hop term's (q0, lambda, h') cotangents come in through hopbar (may be
// null); all of them go through the eigen-solve into grad.
__global__ __launch_bounds__(kEigThreads) void k_adj_explicit(ClassDev c, const double* Cs,
                                                              double* Gh, const double* weights,
                                                              const double* hopbar, AdjTerms wt,
                                                              double* grads, int gstride, int s,
                                                              int T) {
  __shared__ AdjLds A;
  __shared__ double zr[kMaxElec], zi[kMaxElec];
  EigLds& L = A.L;
  const int t = blockIdx.x, tid = threadIdx.x;
  const ModelDev& md = c.md;
  const int n = md.n, n_pad = md.n_pad, N = md.N;
  const double w = weights[c.gtraj[t]];
  const double x = c.path[(size_t)c.gtraj[t] * c.path_len + s];
  load_bath(c, L);
  const ModelAt ma = solve_arrowhead(md, c.vbar, &x, L);
  const double* C = Cs + (size_t)t * N * n_pad * 2;
  double* G = Gh + (size_t)t * N * n_pad * 2;
  // z_o = sum_a q0_a C[o][a], one wave per orbital
  const int lane = tid & 63, wv = tid >> 6;
  for (int o = wv; o < N; o += kEigThreads / 64) {
    double ar = 0.0, ai = 0.0;
    for (int a = lane; a < n; a += 64) {
      ar += L.q0[a] * C[((size_t)o * n_pad + a) * 2];
      ai += L.q0[a] * C[((size_t)o * n_pad + a) * 2 + 1];
    }
    for (int m = 32; m > 0; m >>= 1) {
      ar += __shfl_xor(ar, m);
      ai += __shfl_xor(ai, m);
    }
    if (lane == 0) {
      zr[o] = ar;
      zi[o] = ai;
    }
  }
  __syncthreads();
  const bool last = (s == T);
  const double invT = 1.0 / T;
  const double omega = md.p[0], gg = md.p[1], m = md.mass;
  const double hp = -m * omega * omega * gg;
  const double* hb = hopbar ? hopbar + (size_t)t * (2 * n_pad + 1) : nullptr;
  // Gh update; qbar_a = (2/T) sum_o Re(C[o][a] conj(z_o)); at T, lbar_a = rho_a - n0_a
  for (int a = tid; a < n; a += kEigThreads) {
    double qb = 0.0, rho = 0.0;
    for (int o = 0; o < N; ++o) {
      const size_t e = ((size_t)o * n_pad + a) * 2;
      const double cr = C[e], ci = C[e + 1];
      qb += cr * zr[o] + ci * zi[o];
      rho += cr * cr + ci * ci;
      double gr = wt.cP * invT * L.q0[a] * zr[o], gi = wt.cP * invT * L.q0[a] * zi[o];
      if (last) {
        gr += wt.cE * L.lam[a] * cr;
        gi += wt.cE * L.lam[a] * ci;
      }
      G[e] += w * gr;
      G[e + 1] += w * gi;
    }
    bool occ = false;
    for (int r = 0; r < N; ++r) occ |= (c.occ[(size_t)t * N + r] == a);
    double qbar = wt.cP * 2.0 * invT * qb;
    // force term: F = -m omega^2 x - h' sum_occ q0^2
    if (occ) qbar -= wt.cF * invT * hp * 2.0 * L.q0[a];
    double lb = last ? wt.cE * (rho - (occ ? 1.0 : 0.0)) : 0.0;
    A.qbar[a] = w * qbar + (hb ? hb[a] : 0.0);
    A.lbar[a] = w * lb + (hb ? hb[n_pad + a] : 0.0);
  }
  // h' cotangent: force term and hop term
  double hpart = 0.0;
  for (int r = tid; r < N; r += kEigThreads) {
    const double q = L.q0[c.occ[(size_t)t * N + r]];
    hpart -= wt.cF * invT * q * q;
  }
  const double hpbar = w * block_sum(hpart, A.red3) + (hb ? hb[2 * n_pad] : 0.0);
  double* gr = grads + (size_t)c.gtraj[t] * gstride;
  if (tid == 0 && wt.cF != 0.0) gr[2 + md.M] += -w * wt.cF * invT * 2.0 * m * omega * x;
  __syncthreads();
  eig_backprop(md, ma, x, A, hpbar, gr);
}

// Midpoint of step s: from Phi = dL/dAt (ImPhi [n_pad][n_pad], ReD = Re diag)
// with At = (A - c)/r, A = diag(lambda) - i v D, D_jk = h' q0_j q0_k /
// (lambda_k - lambda_j): lbar_j = (2/r) Re Phi_jj, Dbar = (2 v / r) Im Phi,
// then through D to (lambda, q0, h') and through the eigen-solve.
__global__ __launch_bounds__(kEigThreads) void k_adj_mid(ClassDev c, const double* imphi,
                                                         const double* rediag, double* grads,
                                                         int gstride, int s, double dt) {
  __shared__ AdjLds A;
  EigLds& L = A.L;
  const int t = blockIdx.x, tid = threadIdx.x;
  const ModelDev& md = c.md;
  const int n = md.n, n_pad = md.n_pad;
  const double* pp = c.path + (size_t)c.gtraj[t] * c.path_len + s;
  const double x0 = pp[0], x1 = pp[1];
  const double xm = 0.5 * (x0 + x1), v = (x1 - x0) / dt;
  const double r = 1.0 / c.cheb[(size_t)t * kChebStride + CHEB_INVR];
  load_bath(c, L);
  const ModelAt ma = solve_arrowhead(md, c.vbar, &xm, L);
  const double hp = ma.dh;
  const double* P = imphi + (size_t)t * n_pad * n_pad;
  const double sc = 2.0 * v / r;  // Dbar = sc * Im Phi
  double hpart = 0.0;
  for (int m = tid; m < n; m += kEigThreads) {
    double qb = 0.0, lb = 0.0;
    for (int k = 0; k < n; ++k) {
      if (k == m) continue;
      const double dkm = lam_diff(L, k, m);  // lambda_k - lambda_m
      const double Dmk = hp * L.q0[m] * L.q0[k] / dkm;
      const double Dkm = -Dmk;
      const double bmk = sc * P[(size_t)m * n_pad + k], bkm = sc * P[(size_t)k * n_pad + m];
      qb += hp * L.q0[k] * (bmk - bkm) / dkm;
      lb += (bmk * Dmk + bkm * Dkm) / dkm;
      hpart += bmk * L.q0[m] * L.q0[k] / dkm;
    }
    A.qbar[m] = qb;
    A.lbar[m] = lb + 2.0 / r * rediag[(size_t)t * n_pad + m];
  }
  const double hpbar = block_sum(hpart, A.red3);
  eig_backprop(md, ma, xm, A, hpbar, grads + (size_t)c.gtraj[t] * gstride);
}

// Chebyshev block with conjugated coefficients (the adjoint series).
__global__ void k_conj_cheb(ClassDev c, double* out) {
  const int t = blockIdx.x;
  const double* in = c.cheb + (size_t)t * kChebStride;
  double* o = out + (size_t)t * kChebStride;
  for (int e = threadIdx.x; e < kChebStride; e += blockDim.x) {
    const bool imag = e >= CHEB_COEF && ((e - CHEB_COEF) & 1);
    o[e] = imag ? -in[e] : in[e];
  }
}

}  // namespace

hipError_t launch_eig_step(const ClassDev& c, double dt, Counters* cnt, hipStream_t s, int sub,
                           int nsub) {
  const int precision = c.C64 ? IESH_FP64 : IESH_MIXED;
  if (c.n_live < 1) return hipSuccess;
  hipLaunchKernelGGL(k_eig_step, dim3(c.n_live), dim3(kEigThreads), 0, s, c, dt, precision, cnt, sub,
                     nsub);
  return hipGetLastError();
}

hipError_t launch_eig_fused(const ClassSet& set, double dt, int precision, Counters* cnt, hipStream_t s,
                            int sub, int nsub) {
  if (set.n < 1 || set.first[set.n] < 1) return hipSuccess;
  hipLaunchKernelGGL(k_eig_fused, dim3(set.first[set.n]), dim3(kEigThreads), 0, s, set, dt, precision, cnt,
                     sub, nsub);
  return hipGetLastError();
}

hipError_t launch_eig_query(const ClassDev& c, int t0, int nt, hipStream_t s) {
  hipLaunchKernelGGL(k_eig_query, dim3(nt), dim3(kEigThreads), 0, s, c, t0, 0);
  return hipGetLastError();
}

hipError_t launch_forces(const ClassDev& c, hipStream_t s) {
  hipLaunchKernelGGL(k_eig_query, dim3(c.n_traj), dim3(kEigThreads), 0, s, c, 0, 1);
  return hipGetLastError();
}

hipError_t launch_init_thermal(const ClassDev& c, double kT, double bias, uint64_t seed,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_init_thermal, dim3(c.n_traj), dim3(kEigThreads), 0, s, c, kT, bias, seed);
  return hipGetLastError();
}

hipError_t launch_adj_explicit(const ClassDev& c, const double* Cs, double* Gh, const double* weights,
                               const double* hopbar, const AdjTerms& w, double* grads, int gstride,
                               int s, int T, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_explicit, dim3(c.n_traj), dim3(kEigThreads), 0, st, c, Cs, Gh, weights,
                     hopbar, w, grads, gstride, s, T);
  return hipGetLastError();
}

hipError_t launch_adj_mid(const ClassDev& c, const double* imphi, const double* rediag, double* grads,
                          int gstride, int s, double dt, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_mid, dim3(c.n_traj), dim3(kEigThreads), 0, st, c, imphi, rediag, grads,
                     gstride, s, dt);
  return hipGetLastError();
}

hipError_t launch_conj_cheb(const ClassDev& c, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_conj_cheb, dim3(c.n_traj), dim3(64), 0, st, c, out);
  return hipGetLastError();
}

}  // namespace iesh
