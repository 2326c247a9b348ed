// Internal declarations shared by the HIP translation units of libiesh.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/iesh.h"

namespace iesh {

constexpr int kMaxStates = IESH_MAX_STATES;  // n = M + 1
constexpr int kMaxElec = IESH_MAX_ELEC;      // N
constexpr int kMaxDof = IESH_MAX_DOF;        // nuclear coordinates
constexpr int kMaxCheb = 64;                 // Chebyshev terms per step
constexpr int kChebStride = 2 * kMaxCheb + 8;
constexpr int kGeoStride = 32;
// The no-hop bound assumes the stored orbitals are orthonormal up to a
// defect ||C^H C - I|| <= delta.  On the mixed path delta is the larger of a
// floor and this multiple of the defect the last Loewdin step measured (the
// growth over one period, before its correction).
constexpr double kDefectSafety = 4.0;
constexpr double kDeltaFP64 = 1e-8;
constexpr double kDeltaMixed = 1e-3;

// Status bits that stop a trajectory.
constexpr int kFreezeMask = IESH_TRAJ_EXITED | IESH_TRAJ_NONCONV | IESH_TRAJ_NONFINITE |
                            IESH_TRAJ_STEPCAP;

// Per-trajectory scalars at the most recent geometry (layout of geo[]):
// h, dh/dx, rho = f'/f, U0, dU0/dx of coordinate 0; v.grad h and
// v.grad f / f with the current velocity (several coordinates); then the
// gradients of every coordinate (dh/dR_nu, rho_nu, dU0/dR_nu) at GEO_DHV,
// GEO_RHOV, GEO_DU0V.
enum GeoSlot {
  GEO_H = 0, GEO_DH = 1, GEO_RHO = 2, GEO_U0 = 3, GEO_DU0 = 4, GEO_VDH = 5, GEO_VRHO = 6,
  GEO_DHV = 8, GEO_RHOV = 8 + kMaxDof, GEO_DU0V = 8 + 2 * kMaxDof
};

// Chebyshev parameter block (layout of cheb[]): [0] centre c, [1] 1/radius,
// [2] number of terms K (as double), [3] radius*dt, then K complex
// coefficients (re, im) starting at [8].
enum ChebSlot { CHEB_C = 0, CHEB_INVR = 1, CHEB_K = 2, CHEB_RHO = 3, CHEB_COEF = 8 };

// Model constants passed by value to kernels.
struct ModelDev {
  int kind;
  int M;       // bath levels
  int M_red;   // distinct bath energies (poles of the secular function); M without repeats
  int eig_iter;  // secular iterations allowed per root
  int n;       // M + 1
  int n_pad;   // n rounded up to 16
  int N;       // electrons
  int ndof;    // nuclear coordinates
  double mass;
  double Gamma;
  double p[16];
  double mass_dof[kMaxDof];  // mass of each coordinate (mass_dof[0] = mass for one coordinate)
  double dofp[kMaxDof][6];   // IESH_MODEL_MULTI_DOF: D, a, r, g, c, s per coordinate
  // Repeated bath energies (deflation): the levels of a group of g equal
  // energies couple to the impurity only through one combination, which
  // keeps a pole of the secular function with the summed weight; the g - 1
  // orthogonal combinations are eigenstates at that energy with no impurity
  // component.  expand[j] (j < n, nullptr without repeats) names adiabatic
  // state j: r >= 0 is root r of the secular function over the M_red
  // distinct poles, -(m + 1) a deflated state at pole m.  Deflated states lie
  // between roots m and m + 1, so the energies stay ascending.
  const int32_t* expand;
  // Two leads (nullptr for one): lead0[m] is the share of pole m's squared
  // coupling that belongs to lead 0, lead0[M_red + m] the lead-0 weight of
  // each deflated state at pole m (their mean over the degenerate subspace).
  const double* lead0;
};

// Device state of one bath-size class.
struct ClassDev {
  ModelDev md;
  int n_traj;           // trajectories in this class (allocated slots)
  int n_live;           // host: slots a launch covers (the class size, except while autotuning)
  int64_t* work = nullptr;  // [2] device: Chebyshev terms summed, trajectory-steps (this class)
  int32_t* live = nullptr;  // [1] device: leading slots the step kernels visit (the
                            // others hold frozen trajectories); lowered by the
                            // compaction kernels without a host round trip
  int traj_offset;      // first global trajectory index of this class
  int nct_max;          // column tiles per propagation work-group
  int n_slabs;          // propagation work-groups per trajectory
  // [T][ceil(N / 8)][n_pad]: for propagation slab s of trajectory t, the
  // squared norms over the slab's orbitals of every row of C after the last
  // propagation (sum_j |C[i][j]|^2), read by the no-hop bound
  double* rown = nullptr;
  int hop_groups = 0;   // work-groups of a persistent ratio-kernel launch (0: one per slot)
  int exit_dof = 0;     // coordinate compared with the exit distance
  int exact_hops = 0;   // 1: determinant ratios at every step (no-hop bound unused)
  // step clock: [T][2] = (dt of the next step, elapsed time); the step kernels
  // take dt from it.  dt_levels > 0 adapts dt to the hop probabilities.
  double* clock = nullptr;
  double dt0 = 0.0;     // largest step (the run's dt)
  double gmax = 0.0;    // bound on the rescaled hop-probability total per step
  int dt_levels = 0;    // halvings allowed (0: fixed step)
  // device arrays (class-local trajectory index t)
  double* eps = nullptr;    // [M]
  double* vbar = nullptr;   // [M]  sqrt(Gamma w / 2 pi)
  double* x = nullptr;      // [T][ndof]
  double* v = nullptr;      // [T][ndof]
  double* F = nullptr;      // [T][ndof]
  int32_t* occ = nullptr;   // [T][N]
  int32_t* status = nullptr;  // [T]
  int32_t* gtraj = nullptr;   // [T] global trajectory index
  int32_t* home = nullptr;    // [T] class-local index of the trajectory held in this slot
  int64_t* nsteps = nullptr;  // [T] steps taken
  int64_t* stepcap = nullptr;  // [T] freeze after this many steps (0: no own cap)
  double* C64 = nullptr;    // [T][N][n_pad] complex (re, im)
  float* C32 = nullptr;     // [T][N][n_pad] complex (re, im), mixed path
  double* lam = nullptr;    // [T][n_pad] energies at the current geometry
  double* q0 = nullptr;     // [T][n_pad] impurity amplitudes
  double* lam_mid = nullptr;  // [T][n_pad]
  double* geo = nullptr;    // [T][kGeoStride]
  double* cheb = nullptr;   // [T][kChebStride]
  double* Bt = nullptr;     // [T][n_pad/4][n_pad/16][64] v*D at the midpoint, MFMA A-tile order
  float* Bt32 = nullptr;    // same in FP32 (mixed path)
  double* gbuf = nullptr;   // [T][N][n_pad] hop probabilities (query mode)
  double* obs = nullptr;    // [records][T][IESH_N_OBS] (class-local records)
  double2* low = nullptr;   // Loewdin scratch (mixed path)
  // [T] by home index (mixed path): ||C^H C - I||_F before the last Loewdin
  // correction (0 before the first); the no-hop bound allows a defect of
  // max(delta floor, kDefectSafety * this) for the stored orbitals
  double* defect = nullptr;
  // dense model kind (H(x) = H0 + x H1): [n_pad][n_pad] each, zero-padded,
  // shared by the class; Gd [T][n_pad][n_pad] = Q^T H1 Q at the last solve
  // (ascending, sign-fixed basis), read by the hop kernels
  const double* H0 = nullptr;
  const double* H1 = nullptr;
  double* Gd = nullptr;
  // arrowhead classes, by home index: the secular roots of the trajectory's
  // last solve ([T][2][n_pad]: relative to their origin poles, then the
  // impurity components q0; [T][n_pad] the poles) and its geometry ([T][4]:
  // h, f, valid), the warm start of the next
  double* root_tau = nullptr;
  int32_t* root_org = nullptr;
  double* root_geo = nullptr;
  double* Qw = nullptr;  // [T][n_pad][n_pad] by home index: eigenvectors of the
                         // trajectory's last solve (warm start of the next)
  int32_t* hopq = nullptr;  // [3 + T] queue for the determinant-ratio kernel: count, -, done, list
  double2* hopx = nullptr;  // [T][N][N] inverse of S (shapes whose registers cannot hold it)
  // prescribed nuclear path (adjoint): x of trajectory g at step n is
  // path[g * path_len + n]; the step kernels follow it when path != nullptr
  const double* path = nullptr;
  int path_len = 0;
  int path_n = 0;
};

struct Counters {
  int64_t step;          // global step counter (hop uniform counter)
  int64_t run_step0;     // first step of the current iesh_run call
  int64_t n_events;      // events recorded
  int64_t record_every;
  int64_t sum_cheb;      // Chebyshev terms summed over propagated trajectory-steps
  int64_t traj_steps;    // trajectory-steps taken
  int64_t hop_evals;     // trajectory-steps that needed the determinant ratios
  int64_t max_cheb;      // largest number of Chebyshev terms used
  // orthonormality defect ||C^H C - I||_F measured by the Loewdin steps: the
  // largest one (bit pattern of a non-negative double, which orders like the
  // value) and the number of measurements above the no-hop bound's allowance
  // for the period before them
  uint64_t defect_max_bits;
  int64_t defect_violations;
};

// -------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), host and device.
struct Philox4 {
  uint32_t v[4];
};

__host__ __device__ inline uint32_t mulhi32(uint32_t a, uint32_t b) {
  return (uint32_t)(((uint64_t)a * (uint64_t)b) >> 32);
}

__host__ __device__ inline Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                  uint32_t c3, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    uint32_t lo0 = M0 * c0, hi0 = mulhi32(M0, c0);
    uint32_t lo1 = M1 * c2, hi1 = mulhi32(M1, c2);
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  Philox4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

// Uniform in [0, 1) for (seed, trajectory, counter, stream).
__host__ __device__ inline double philox_uniform(uint64_t seed, uint32_t traj, uint64_t counter,
                                                 uint32_t stream) {
  Philox4 w = philox4x32_10((uint32_t)counter, (uint32_t)(counter >> 32), traj, stream,
                            (uint32_t)seed, (uint32_t)(seed >> 32));
  uint64_t u = ((uint64_t)w.v[1] << 32) | (uint64_t)w.v[0];
  return (double)(u >> 11) * (1.0 / 9007199254740992.0);
}

// -------------------------------------------------------------------------
// Model scalars at the geometry x[0 .. ndof).  Couplings factor as
// V_k(x) = Vbar_k f(x); rho = f'/f.  dU0, dh and rho are those of coordinate
// 0; model_grad gives them for any coordinate.
struct ModelAt {
  double U0, dU0, h, dh, f, rho;
};

// dh/dR_nu, rho_nu = (df/dR_nu)/f and dU0/dR_nu of the multi-coordinate model.
__host__ __device__ inline void multi_dof_grad(const ModelDev& md, const double* x, int nu,
                                               double& dh, double& rho, double& dU0) {
  const double D = md.dofp[nu][0], a = md.dofp[nu][1], r = md.dofp[nu][2];
  const double g = md.dofp[nu][3], cc = md.dofp[nu][4], s = md.dofp[nu][5];
  const double e = exp(-a * (x[nu] - r));
  dU0 = 2.0 * D * a * e * (1.0 - e);
  dh = g;
  rho = -(x[nu] - cc) / (2.0 * s * s);
}

__host__ __device__ inline ModelAt model_at(const ModelDev& md, const double* xv) {
  ModelAt r;
  const double x = xv[0];
  if (md.kind == IESH_MODEL_MULTI_DOF) {
    double U0 = 0.0, hs = md.p[0] + md.p[1], lf = 0.0;
    for (int nu = 0; nu < md.ndof; ++nu) {
      const double D = md.dofp[nu][0], a = md.dofp[nu][1], rr = md.dofp[nu][2];
      const double g = md.dofp[nu][3], cc = md.dofp[nu][4], s = md.dofp[nu][5];
      const double e = exp(-a * (xv[nu] - rr));
      U0 += D * (1.0 - e) * (1.0 - e);
      hs += g * (xv[nu] - rr);
      lf -= (xv[nu] - cc) * (xv[nu] - cc) / (4.0 * s * s);
    }
    r.U0 = U0;
    r.h = hs;
    r.f = exp(lf);
    multi_dof_grad(md, xv, 0, r.dh, r.rho, r.dU0);
  } else if (md.kind == IESH_MODEL_HARMONIC) {
    const double omega = md.p[0], g = md.p[1], dG = md.p[2], eps_d = md.p[3];
    const double k = md.mass * omega * omega;
    r.U0 = 0.5 * k * x * x;
    r.dU0 = k * x;
    const double U1 = 0.5 * k * (x - g) * (x - g) + dG;
    r.h = U1 - r.U0 + eps_d;
    r.dh = -k * g;
    r.f = 1.0;
    r.rho = 0.0;
  } else {
    const double De = md.p[0], x0 = md.p[1], a = md.p[2], D1 = md.p[3], D2 = md.p[4];
    const double ap = md.p[5], Vinf = md.p[6], q = md.p[7], at = md.p[8], xt = md.p[9];
    const double c = md.p[10], eps_d = md.p[11];
    const double e = exp(-a * (x - x0));
    r.U0 = De * (e - 1.0) * (e - 1.0) + c;
    r.dU0 = -2.0 * De * a * e * (e - 1.0);
    const double e1 = exp(-ap * (x - x0));
    const double U1 = D1 * e1 * e1 - D2 * e1 + Vinf;
    const double dU1 = -2.0 * ap * D1 * e1 * e1 + ap * D2 * e1;
    r.h = U1 - r.U0 + eps_d;
    r.dh = dU1 - r.dU0;
    const double t = tanh((x - xt) / at);
    r.f = 0.5 * (1.0 - q) * (1.0 - t) + q;
    const double df = -0.5 * (1.0 - q) * (1.0 - t * t) / at;
    r.rho = df / r.f;
  }
  return r;
}

// Leading slots of a class that the step kernels visit.
__device__ inline int live_slots(const ClassDev& c) { return c.live ? *c.live : c.n_live; }

// Several classes for one launch (kernel argument: up to kFuseMax classes);
// block b belongs to class k for first[k] <= b < first[k + 1].
constexpr int kFuseMax = 4;
struct ClassSet {
  ClassDev c[kFuseMax];
  int first[kFuseMax + 1];
  int n;
};

// Spare copies of the state that moves with a trajectory (compaction).
// Step clock after a step whose hop probabilities total g_total: the next
// step is the largest dt0 / 2^k (k <= dt_levels) for which g_total rescaled
// from the current step to it stays at or below gmax (Sec. II.C bounds the
// step by the hopping probabilities; they are proportional to the step).
__device__ inline void advance_clock(const ClassDev& c, int t, double g_total) {
  double* ck = c.clock + 2 * (size_t)t;
  const double dtc = ck[0];
  double dtn = c.dt0;
  for (int k = 0; k < c.dt_levels && g_total * (dtn / dtc) > c.gmax; ++k) dtn = 0.5 * dtn;
  ck[0] = dtn;
  ck[1] += dtc;
}

struct CompactBufs {
  double* x = nullptr;
  double* v = nullptr;
  double* F = nullptr;
  int32_t* status = nullptr;
  int32_t* gtraj = nullptr;
  int32_t* home = nullptr;
  int64_t* nsteps = nullptr;
  int64_t* stepcap = nullptr;
  int32_t* occ = nullptr;  // [T][N]
  double* clock = nullptr;  // [T][2]
  void* C = nullptr;       // [T][N][n_pad] complex, element type of the orbitals
  int32_t* dst = nullptr;  // [T] destination slot of each live slot
  int32_t* n_active = nullptr;  // [1]
};

// -------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).
// sub: -1 whole step, j >= 0 propagator of electronic sub-step j of nsub, -2 end point only.
hipError_t launch_eig_step(const ClassDev& c, double dt, Counters* cnt, hipStream_t s, int sub = -1,
                           int nsub = 1);
hipError_t launch_eig_query(const ClassDev& c, int t0, int nt, hipStream_t s);
// the step of several arrowhead classes in one launch
hipError_t launch_eig_fused(const ClassSet& set, double dt, int precision, Counters* cnt, hipStream_t s,
                            int sub = -1, int nsub = 1);
hipError_t launch_init_thermal(const ClassDev& c, double kT, double bias, uint64_t seed,
                               hipStream_t s);
// dense symmetric eigen-decomposition (k_jacobi.hip)
size_t jacobi_work_elems(int n, int batch);  // doubles of global workspace (0: all in LDS)
hipError_t launch_jacobi(const double* H, int n, int batch, double* lam, double* Q, int32_t* sweeps,
                         double* work, hipStream_t s);
hipError_t launch_forces(const ClassDev& c, hipStream_t s);
// dense model kind (k_dense.hip)
size_t dense_lds_size(int n_pad);
hipError_t launch_dense_step(const ClassDev& c, double dt, Counters* cnt, hipStream_t s, int sub = -1,
                             int nsub = 1);
hipError_t launch_dense_query(const ClassDev& c, int t0, int nt, int mode, hipStream_t s);
hipError_t launch_dense_init_thermal(const ClassDev& c, double kT, uint64_t seed, hipStream_t s);
hipError_t launch_prop(const ClassDev& c, int precision, hipStream_t s);
hipError_t launch_prop_taps(const ClassDev& c, int mode, double* taps, int tap_k, hipStream_t s);
int prop_max_col_tiles(int precision);
int hop_resident_groups(const ClassDev& c, int precision, int n_cu);
int prop_max_tiles_per_wave(int precision);
hipError_t prop_prepare(const ClassDev& c, int precision);
size_t prop_lds_bytes(const ClassDev& c, int precision);
hipError_t launch_hop(const ClassDev& c, double dt, uint64_t seed, Counters* cnt,
                      iesh_event* events, int query_mode, int t0, int nt, int record,
                      int exit_enabled, double exit_x, int64_t max_steps, int precision,
                      hipStream_t s);
bool hop_needs_scratch(const ClassDev& c);
// the no-hop bound of several classes of one kind in one launch
hipError_t launch_filter_fused(const ClassSet& set, double dt, uint64_t seed, Counters* cnt, int record,
                               int exit_enabled, double exit_x, int64_t max_steps, int precision,
                               hipStream_t s);
hipError_t launch_lowdin(const ClassDev& c, Counters* cnt, int every, double2* scratch,
                         hipStream_t s);
size_t lowdin_scratch_elems(const ClassDev& c);
hipError_t launch_advance(Counters* cnt, hipStream_t s);
hipError_t launch_fill(double* p, size_t count, double value, hipStream_t s);
// Adjoint along prescribed paths (k_eig.hip, k_adjoint.hip).
struct AdjTerms {
  double cP, cE, cG, cF;  // weights of the population, excitation, hop and force terms
};
hipError_t launch_adj_loss(const ClassDev& c, double* loss, int s, int T, const AdjTerms& w,
                          hipStream_t st);
size_t adj_hop_scratch_elems(const ClassDev& c);
hipError_t launch_adj_hop(const ClassDev& c, const double* Cs, double* Gh, double* scr,
                          const double* weights, double* loss, double* hopbar, int s, int T,
                          double dt, double cG, int reverse, hipStream_t st);
hipError_t launch_adj_explicit(const ClassDev& c, const double* Cs, double* Gh, const double* weights,
                               const double* hopbar, const AdjTerms& w, double* grads, int gstride,
                               int s, int T, hipStream_t st);
hipError_t launch_adj_mid(const ClassDev& c, const double* imphi, const double* rediag, double* grads,
                          int gstride, int s, double dt, hipStream_t st);
hipError_t launch_conj_cheb(const ClassDev& c, double* out, hipStream_t st);
hipError_t launch_adj_phi(const ClassDev& c, const double* taps_s, const double* taps_t, int tap_k,
                          double* imphi, double* rediag, hipStream_t st);
hipError_t launch_compact_rank(const ClassDev& c, int32_t* dst, int32_t* n_active, hipStream_t s);
hipError_t launch_compact_move(const ClassDev& c, const int32_t* dst, const CompactBufs& b,
                               int precision, hipStream_t s);
hipError_t launch_compact(const ClassDev& c, const CompactBufs& b, int precision, hipStream_t s);

// Reason of the last failed context-free call on this thread (api.cpp):
// what iesh_last_error(NULL) returns.
void set_call_error(const std::string& why);

// Host-side bath discretisation (bath.cpp).
int discretize(int kind, int M, double a, double b, double eps_f, double* eps, double* w);
int bath_levels(const iesh_bath_desc& d, double* eps, double* w, int32_t* lead, int32_t* n_below);

}  // namespace iesh
