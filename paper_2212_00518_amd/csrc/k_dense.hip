// Step kernels for a one-electron Hamiltonian of any symmetric structure,
// affine in one nuclear coordinate: H(x) = H0 + x H1, dH/dx = H1 (Eq.
// single_electron_discrete_electronic_hamiltonian without the arrowhead
// structure; the couplings of Sec. II.B, G = Q^T (dH/dx) Q,
// D_jk = G_jk / (lambda_k - lambda_j), and the Hellmann-Feynman force of
// Eq. classical_hamiltonian, F = -U0' - sum_{a in s} G_aa).
//
// One work-group (8 waves) per trajectory.  The eigen-decomposition of
// H(x) runs in LDS: two matrices padded to n_pad = n rounded up to 16 with a
// row stride of n_pad + 1 doubles (2 n_pad (n_pad + 1) doubles, which bounds
// n at IESH_DENSE_MAX_N, 96).  A warm solve starts from the trajectory's
// previous eigenvectors and refines them by first-order perturbation updates
// whose products run on the FP64 matrix cores (see perturb_refine); a cold
// solve, and the fallback of a warm one, is the cyclic two-sided Jacobi
// method (Golub and Van Loan): every sweep visits each index pair once in
// m - 1 rounds of m/2 disjoint pairs (round-robin over m = n rounded up to
// even), so the rotations of a round are independent and one pass rotates
// rows, a second columns; a pair is skipped once |a_pq| <= eps
// sqrt(|a_pp a_qq|) (the relative stopping rule of Demmel and Veselic).
// Eigenvalues are ranked ascending; each eigenvector's first nonzero
// component (the impurity component, generically) is made positive.
//
// The projection G = V^T (H1 V) is two dense products of order n_pad on the
// FP64 matrix cores (16x16x4 instructions, see mm_tiles): T = H1 V overwrites
// the diagonalised matrix in LDS, then G = V^T T (on and above the diagonal,
// mirrored) is written to the trajectory's block of Gd in the ranked,
// sign-fixed basis.  The midpoint solve turns G into B = v D in
// the propagation kernel's tile order with the Gershgorin interval of
// A = diag(lambda) - i B and the Chebyshev block; the end-point solve leaves
// lambda, Q[0, :] and G for the hop kernels and completes velocity Verlet.

#include "iesh_cheb.hpp"
#include "iesh_internal.hpp"

namespace iesh {
namespace {

constexpr int kDenThreads = 512;
constexpr int kDenWaves = kDenThreads / 64;
constexpr int kJacobiSweeps = 60;
constexpr int64_t kDenseColdEvery = 256;  // steps between cold eigen-solves of a trajectory
constexpr double kEpsD = 2.220446049250313e-16;
// A sweep whose rotations all have |tan| below this ends the iteration: the
// off-diagonal elements it leaves are about the square of its largest
// rotation relative to the level gaps, so the next sweep would rotate by
// angles near rounding (the confirming sweep without rotations is skipped).
constexpr double kJacobiSmallRot = 1e-8;
// Rotations a wave applies per round and columns (rows) a lane covers, for
// n <= IESH_DENSE_MAX_N.
constexpr int kPairsPerWave = (IESH_DENSE_MAX_N / 2 + kDenWaves - 1) / kDenWaves;
constexpr int kColsPerLane = (IESH_DENSE_MAX_N + 63) / 64;
static_assert(IESH_DENSE_MAX_N / 16 <= kDenWaves, "the coupling rows take one wave per 16 rows");

typedef double v4d __attribute__((ext_vector_type(4)));

// Views of the dynamic LDS of one work-group (np = n_pad, ld = np + 1).
struct DenLds {
  double* A;     // [np][ld]: H(x), rotated to diagonal form; then T = H1 V
  double* V;     // [np][ld]: accumulated rotations, eigenvectors in columns
  double* lam;   // [np]: eigenvalues, ascending
  double* q0;    // [np]: impurity components (ascending order, sign-fixed)
  double* dj;    // [np]: eigenvalue of Jacobi column j
  double* sg;    // [np]: sign applied to Jacobi column j
  double* rs;    // [np]: row sums of |B| (the Gershgorin interval)
  double* red;   // [2 kDenWaves]: per-wave partial results
  double* J;     // [kMaxCheb]: Bessel values
  double* nuc;   // [4]: half-step velocity, new position, propagator position, force
  int* rank;     // [np]: position of Jacobi column j in ascending order
  int* pq;       // [np]: the pairs of a round
  int* flag;     // [5]: rotation happened, failure bits, unused, unused, a large rotation
                 // in this sweep
};

__host__ __device__ inline size_t dense_lds_bytes(int np) {
  const size_t ld = np + 1;
  return sizeof(double) * (2 * (size_t)np * ld + 4 * (size_t)np + (size_t)np + 2 * kDenWaves +
                           kMaxCheb + 4) +
         sizeof(int) * (2 * (size_t)np + 5);
}

__device__ __forceinline__ DenLds dense_lds(double* sm, int np) {
  DenLds L;
  const size_t ld = np + 1;
  L.A = sm;
  L.V = L.A + (size_t)np * ld;
  L.lam = L.V + (size_t)np * ld;
  L.q0 = L.lam + np;
  L.dj = L.q0 + np;
  L.sg = L.dj + np;
  L.rs = L.sg + np;
  L.red = L.rs + np;
  L.J = L.red + 2 * kDenWaves;
  L.nuc = L.J + kMaxCheb;
  L.rank = reinterpret_cast<int*>(L.nuc + 4);
  L.pq = L.rank + np;
  L.flag = L.pq + np;
  return L;
}

// Value of lane `src` (wave-uniform) of a per-lane double.
__device__ __forceinline__ double lane_value(double v, int src) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)u, src);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum of v over the work-group (every thread gets it).
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
  const int tid = threadIdx.x;
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kDenWaves; ++w) s += red[w];
  __syncthreads();
  return s;
}

__device__ __forceinline__ double block_min(double v, double* red) {
  for (int m = 32; m > 0; m >>= 1) v = fmin(v, __shfl_xor(v, m));
  const int tid = threadIdx.x;
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < kDenWaves; ++w) s = fmin(s, red[w]);
  __syncthreads();
  return s;
}

__device__ __forceinline__ double block_max(double v, double* red) { return -block_min(-v, red); }

// A copy of a wave-uniform int that the compiler cannot see through: the
// addresses computed from it in one stage of the eigen-solve are neither
// shared with nor hoisted into earlier stages (the two solves of a step and
// the updates of the refinement would otherwise keep them all live at once).
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return __builtin_amdgcn_readfirstlane(v);
}

// 16x16 output tiles a wave takes in a product of order n_pad.
constexpr int kTilesPerWave =
    ((IESH_DENSE_MAX_N / 16) * (IESH_DENSE_MAX_N / 16) + kDenWaves - 1) / kDenWaves;

// Row and column block of the u-th 16x16 output tile of a wave: tiles
// wave, wave + kDenWaves, ... of the RT x RT blocks (row-major), or of the
// RT (RT + 1) / 2 blocks on and above the diagonal when kUpper.
template <bool kUpper>
__device__ __forceinline__ bool tile_of(int wave, int u, int RT, int& rt, int& ct) {
  int t = wave + u * kDenWaves;
  if (!kUpper) {
    rt = t / RT;
    ct = t - rt * RT;
    return t < RT * RT;
  }
  rt = 0;
  while (rt < RT && t >= RT - rt) {
    t -= RT - rt;
    ++rt;
  }
  ct = rt + t;
  return rt < RT;
}

// Element (i, k) of a matrix operand at p[i * rs + k * cs] (LDS or global).
struct MatView {
  const double* p;
  int rs, cs;
};

// Products a wave forms in one pass of mm_tiles.
enum MmMode { kOne, kTwoX, kTwoY };

// acc1[u] = the u-th 16x16 tile of this wave (tile_of) of X1 Y1, n_pad =
// 16 RT; with kTwoX also acc2[u] of X2 Y1 (one B operand serves both), with
// kTwoY acc2[u] of X1 Y2 (one A operand serves both).  Lane (lr, lk) holds
// rows lk + 4 r, column lr of a tile (16x16x4 layout).  The operands of the
// next k-block of every tile are requested before the products of the
// current one, and a wave's tiles beyond its share load those of tile 0 and
// skip the products, so no load waits behind a branch.
template <bool kUpper, MmMode kMode>
__device__ __forceinline__ void mm_tiles(v4d (&acc1)[kTilesPerWave], v4d (&acc2)[kTilesPerWave], int RT,
                                         int wave, int lane, MatView X1, MatView X2, MatView Y1,
                                         MatView Y2) {
  const int lr = lane & 15, lk = lane >> 4, KB = 4 * RT;
  const double* x1p[kTilesPerWave];
  const double* x2p[kTilesPerWave];
  const double* y1p[kTilesPerWave];
  const double* y2p[kTilesPerWave];
  bool on[kTilesPerWave];
#pragma unroll
  for (int u = 0; u < kTilesPerWave; ++u) {
    int rt, ct;
    on[u] = tile_of<kUpper>(wave, u, RT, rt, ct);
    if (!on[u]) rt = ct = 0;
    x1p[u] = X1.p + (rt * 16 + lr) * X1.rs + lk * X1.cs;
    x2p[u] = X2.p + (rt * 16 + lr) * X2.rs + lk * X2.cs;
    y1p[u] = Y1.p + lk * Y1.rs + (ct * 16 + lr) * Y1.cs;
    y2p[u] = Y2.p + lk * Y2.rs + (ct * 16 + lr) * Y2.cs;
    acc1[u] = v4d{0.0, 0.0, 0.0, 0.0};
    acc2[u] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  const int sx1 = 4 * X1.cs, sx2 = 4 * X2.cs, sy1 = 4 * Y1.rs, sy2 = 4 * Y2.rs;
  // software pipelined: the operands of k-block kb + 1 are requested before
  // the products of k-block kb (the last request repeats k-block KB - 1)
  double a1[kTilesPerWave], a2[kTilesPerWave], b1[kTilesPerWave], b2[kTilesPerWave];
  const auto fetch = [&](int kb, double* f1, double* f2, double* g1, double* g2) {
#pragma unroll
    for (int u = 0; u < kTilesPerWave; ++u) {
      f1[u] = x1p[u][kb * sx1];
      if constexpr (kMode == kTwoX) f2[u] = x2p[u][kb * sx2];
      g1[u] = y1p[u][kb * sy1];
      if constexpr (kMode == kTwoY) g2[u] = y2p[u][kb * sy2];
    }
  };
  fetch(0, a1, a2, b1, b2);
#pragma unroll 2
  for (int kb = 0; kb < KB; ++kb) {
    double n1[kTilesPerWave], n2[kTilesPerWave], m1[kTilesPerWave], m2[kTilesPerWave];
    fetch(kb + 1 < KB ? kb + 1 : kb, n1, n2, m1, m2);
#pragma unroll
    for (int u = 0; u < kTilesPerWave; ++u) {
      if (on[u]) {
        acc1[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], b1[u], acc1[u], 0, 0, 0);
        if constexpr (kMode == kTwoX)
          acc2[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[u], b1[u], acc2[u], 0, 0, 0);
        if constexpr (kMode == kTwoY)
          acc2[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], b2[u], acc2[u], 0, 0, 0);
      }
    }
#pragma unroll
    for (int u = 0; u < kTilesPerWave; ++u) {
      a1[u] = n1[u];
      if constexpr (kMode == kTwoX) a2[u] = n2[u];
      b1[u] = m1[u];
      if constexpr (kMode == kTwoY) b2[u] = m2[u];
    }
  }
}

// T = Hx V on the matrix cores, Hx = H(x) (symmetric, n_pad x n_pad in
// global memory, read by columns: 16 consecutive doubles per row of four
// lanes), V in LDS; T stored at out[i * os + j].
__device__ __forceinline__ void hv_product(const double* Hx, const DenLds& L, int np, int ld, double* out,
                                           int os) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4, RT = np / 16;
  v4d acc[kTilesPerWave], acc2[kTilesPerWave];
  const MatView h{Hx, 1, np}, v{L.V, ld, 1};
  mm_tiles<false, kOne>(acc, acc2, RT, wave, lane, h, h, v, v);
#pragma unroll
  for (int u = 0; u < kTilesPerWave; ++u) {
    int rt, ct;
    if (!tile_of<false>(wave, u, RT, rt, ct)) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) out[(rt * 16 + lk + 4 * r) * os + ct * 16 + lr] = acc[u][r];
  }
}

// A = V^T Hx V in full into L.A (for the Jacobi sweeps), through T = Hx V in
// the scratch block tmp.
__device__ __forceinline__ void full_rayleigh(const ClassDev& c, const double* Hx, DenLds& L, double* tmp) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int np = opaque(c.md.n_pad), ld = np + 1, RT = np / 16;
  hv_product(Hx, L, np, ld, tmp, np);
  __syncthreads();  // T complete (work-group visibility of the global writes)
  v4d acc[kTilesPerWave], acc2[kTilesPerWave];
  const MatView vt{L.V, 1, ld}, t{tmp, np, 1};
  mm_tiles<true, kOne>(acc, acc2, RT, wave, lane, vt, vt, t, t);
#pragma unroll
  for (int u = 0; u < kTilesPerWave; ++u) {
    int rt, ct;
    if (!tile_of<true>(wave, u, RT, rt, ct)) continue;
    const int j = ct * 16 + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = rt * 16 + lk + 4 * r;
      if (i <= j) {
        L.A[i * ld + j] = acc[u][r];
        L.A[j * ld + i] = acc[u][r];
      }
    }
  }
  __syncthreads();
}

// Perturbative refinement of a warm start.  V starts as W, the eigenvectors
// of the trajectory's previous solve (the geometry has moved by half a step):
// A = V^T H V is nearly diagonal and E = V^T V - I nearly zero.  One update
// V <- V (I + X) with
//   X_ij = (A_ij - A_jj E_ij) / (A_jj - A_ii)  (i != j),  X_ii = -E_ii / 2
// removes, to first order, both A's off-diagonal part and E (X + X^T = -E,
// and (I + X)^T A (I + X) has no first-order off-diagonal part), so every
// update squares both relative to the level gaps: the quadratic convergence
// of the Jacobi method without its n - 1 rounds of rotations per sweep, and
// orthonormality restored at each update instead of carried (no exponential
// series is needed).  A and E are recomputed from the current V each time.
// The update whose largest |X_ij| is below kPertDone is the last (what it
// leaves is below FP64 rounding relative to the gaps, as after the last
// Jacobi sweep; on the mixed path kPertDoneMixed, which leaves eigenvector
// errors of a few 1e-10, far below the FP32 propagation's rounding and its
// 2^-26 series truncation); the eigenvalues then follow from A, E and that last X to second
// order, without a last product H V.  An update whose Frobenius norm
// exceeds kPertMax (close levels, a poor start) or kPertUpdates updates
// without convergence (fewer when the run caps the eigen-solve's
// iterations, eig_max_iter) hand over to the Jacobi sweeps.
constexpr int kPertUpdates = 6;
constexpr double kPertDone = 1e-8;
constexpr double kPertDoneMixed = 1e-5;
constexpr double kPertMax = 0.1;

// Refines V (in L.V) for Hx = H(x) (n_pad x n_pad, global); L.A and L.dj
// are its working space, tmp a scratch block of n_pad^2 doubles.  True:
// L.A's diagonal holds the eigenvalues (Jacobi order of L.V).  False: a
// start for the sweeps, which keep V's orthonormality as they find it: the
// warm start itself, L.A = W^T H W, when the first update is refused; else
// (the updates leave V orthonormal only once they converge) the cold start,
// L.A = H(x) and V = I.
__device__ __forceinline__ bool perturb_refine(const ClassDev& c, const double* Hx, DenLds& L, double* tmp,
                                               double done) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int n = c.md.n, RT = c.md.n_pad / 16;
  // the strides are made opaque at the start of every stage (see opaque)
  int np = c.md.n_pad, ld = np + 1;
  const auto fresh = [&] {
    np = opaque(np);
    ld = opaque(ld);
  };
  double* T = L.A;  // H V, then X
  double* const Xm = L.A;
  double* V = L.V;
  v4d acc[kTilesPerWave], acc2[kTilesPerWave];
  fresh();
  hv_product(Hx, L, np, ld, T, ld);
  __syncthreads();
  const int max_upd = min(kPertUpdates, c.md.eig_iter);
  int applied = 0;  // updates applied to V
  for (int upd = 0; upd < max_upd; ++upd) {
    // A = V^T T and E + I = V^T V on and above the diagonal (registers); the
    // diagonal of A to L.dj.  The first update takes E = 0: W is orthonormal
    // to rounding (the last update of the previous solve converged, or the
    // sweeps produced it), and the next update measures what it leaves
    fresh();
    {
      const MatView vt{V, 1, ld}, tv{T, ld, 1};
      if (upd == 0)
        mm_tiles<true, kOne>(acc, acc2, RT, wave, lane, vt, vt, tv, tv);
      else
        mm_tiles<true, kTwoY>(acc, acc2, RT, wave, lane, vt, vt, tv, MatView{V, ld, 1});
    }
#pragma unroll
    for (int u = 0; u < kTilesPerWave; ++u) {
      int rt, ct;
      if (!tile_of<true>(wave, u, RT, rt, ct) || rt != ct) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (lk + 4 * r == lr) L.dj[rt * 16 + lr] = acc[u][r];
    }
    __syncthreads();  // diagonal complete, every wave done reading T
    // X into L.A, its largest element and Frobenius norm
    fresh();
    double xmax = 0.0, xsq = 0.0;
#pragma unroll
    for (int u = 0; u < kTilesPerWave; ++u) {
      int rt, ct;
      if (!tile_of<true>(wave, u, RT, rt, ct)) continue;
      const int j = ct * 16 + lr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = rt * 16 + lk + 4 * r;
        if (i > j) continue;
        const double a = acc[u][r];
        const double e = (upd == 0) ? 0.0 : acc2[u][r] - (i == j ? 1.0 : 0.0);
        double xij = 0.0, xji = 0.0;
        if (j < n) {
          if (i == j) {
            xij = xji = -0.5 * e;
          } else {
            const double di = L.dj[i], dj = L.dj[j];
            const double nij = a - dj * e, nji = a - di * e;
            if (nij != 0.0) xij = nij / (dj - di);
            if (nji != 0.0) xji = nji / (di - dj);
          }
        }
        Xm[i * ld + j] = xij;
        Xm[j * ld + i] = xji;
        xmax = fmax(xmax, fmax(fabs(xij), fabs(xji)));
        xsq += (i == j) ? xij * xij : xij * xij + xji * xji;
      }
    }
    // the wave's largest element and sum of squares to L.red; the barrier
    // publishes them with X
    for (int m = 32; m > 0; m >>= 1) {
      xmax = fmax(xmax, __shfl_xor(xmax, m));
      xsq += __shfl_xor(xsq, m);
    }
    if (lane == 0) {
      L.red[wave] = xmax;
      L.red[kDenWaves + wave] = xsq;
    }
    __syncthreads();
    xmax = L.red[0];
    xsq = L.red[kDenWaves];
    for (int w = 1; w < kDenWaves; ++w) {
      xmax = fmax(xmax, L.red[w]);
      xsq += L.red[kDenWaves + w];
    }
    const double f = sqrt(xsq);
    if (!(f <= kPertMax)) break;  // also a gap of zero (inf) or NaN
    // V <- V + V X
    fresh();
    {
      const MatView v{V, ld, 1}, x{Xm, ld, 1};
      mm_tiles<false, kOne>(acc, acc2, RT, wave, lane, v, v, x, x);
    }
    __syncthreads();  // every wave done reading V, X and L.red
    fresh();
#pragma unroll
    for (int u = 0; u < kTilesPerWave; ++u) {
      int rt, ct;
      if (!tile_of<false>(wave, u, RT, rt, ct)) continue;
      const int j = ct * 16 + lr;
#pragma unroll
      for (int r = 0; r < 4; ++r) V[(rt * 16 + lk + 4 * r) * ld + j] += acc[u][r];
    }
    ++applied;
    if (xmax <= done) {
      // eigenvalues of the updated V to second order in X (the first-order
      // relation A_kj = X_kj (A_jj - A_kk) + A_jj E_kj, E_jj = -2 X_jj):
      //   lambda_j = A_jj (1 + 2 X_jj) + sum_{k != j} X_kj^2 (A_jj - A_kk),
      // the neglected terms are of order |X|^3 and E_jj^2 (the E X terms
      // cancel against the normalisation): below 1e-20 relative after
      // kPertDone, 1e-12 after kPertDoneMixed; thread
      // j reads column j of X only and leaves lambda_j on L.A's diagonal
      fresh();
      for (int j = tid; j < n; j += kDenThreads) {
        const double dj = L.dj[j];
        double s2 = 0.0;
        for (int k = 0; k < n; ++k) {
          const double xk = Xm[k * ld + j];
          if (k != j) s2 += xk * xk * (dj - L.dj[k]);
        }
        Xm[j * ld + j] = dj * (1.0 + 2.0 * Xm[j * ld + j]) + s2;
      }
      __syncthreads();
      return true;
    }
    __syncthreads();
    fresh();
    hv_product(Hx, L, np, ld, T, ld);
    __syncthreads();
  }
  if (applied == 0) {
    full_rayleigh(c, Hx, L, tmp);
  } else {
    fresh();
    for (int idx = tid; idx < np * np; idx += kDenThreads) {
      const int i = idx / np, j = idx - i * np;
      L.A[i * ld + j] = Hx[idx];
      V[i * ld + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
  }
  return false;
}

// Eigen-decomposition of H(x) = H0 + x H1 in LDS, cold (Jacobi sweeps from
// H(x) and the identity) or warm (W != nullptr: perturbative refinement of
// the eigenvectors W of the previous solve, whose block then holds H(x), with
// the sweeps as fallback; tmp a scratch block of n_pad^2 doubles); afterwards
// L.lam, L.q0 hold the ascending eigenvalues and impurity components,
// L.dj / L.sg / L.rank the Jacobi-order eigenvalues, signs and ranks, L.V the
// eigenvectors (Jacobi order, unsigned).  Returns false when the sweeps did
// not converge.
__device__ __forceinline__ bool dense_eigen(const ClassDev& c, double x, DenLds& L, double* W = nullptr,
                                            double* tmp = nullptr, double done = kPertDone) {
  const int tid = threadIdx.x;
  const int n = c.md.n, np = c.md.n_pad, ld = np + 1;
  const int m = n + (n & 1), half = m / 2;
  bool converged = false;
  if (W) {
    // V = W; W's block then holds H(x) until save_basis (H0 and H1 are
    // symmetric, so H(x) is exactly symmetric)
    for (int idx = tid; idx < np * np; idx += kDenThreads) {
      const int i = idx / np, j = idx - i * np;
      L.V[(size_t)i * ld + j] = W[idx];
      W[idx] = c.H0[idx] + x * c.H1[idx];
    }
    __syncthreads();  // (work-group visibility of the global writes)
    converged = perturb_refine(c, W, L, tmp, done);
  } else {
    const double* H0 = c.H0;
    const double* H1 = c.H1;
    for (int idx = tid; idx < np * np; idx += kDenThreads) {
      const int i = idx / np, j = idx - i * np;
      L.A[(size_t)i * ld + j] = H0[idx] + x * H1[idx];  // zero outside n x n
      L.V[(size_t)i * ld + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
  }
  for (int sweep = 0; !converged && sweep < kJacobiSweeps; ++sweep) {
    if (tid == 0) {
      L.flag[0] = 0;
      L.flag[4] = 0;
    }
    __syncthreads();
    // the pairs of a round are disjoint, so a wave takes pairs wave, wave + 8,
    // ... (its lane i computes the rotation of the i-th) and a lane columns
    // (rows) lane and lane + 64; the rotations need no exchange between
    // waves, and a round costs two barriers
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    for (int r = 0; r < m - 1; ++r) {
      int pl = 0, ql = 0;
      double cl = 1.0, sl = 0.0;
      {
        const int k = wave + kDenWaves * lane;
        if (lane < kPairsPerWave && k < half) {
          int p, q;
          if (k == 0) {
            p = r;
            q = m - 1;
          } else {
            p = (r + k) % (m - 1);
            q = (r - k + (m - 1)) % (m - 1);
          }
          if (p > q) {
            const int tmp = p;
            p = q;
            q = tmp;
          }
          pl = p;
          ql = q;
          if (q < n) {
            const double apq = L.A[p * ld + q];
            const double app = L.A[p * ld + p], aqq = L.A[q * ld + q];
            // |a_pq| > eps sqrt(|a_pp a_qq|), squared
            if (apq != 0.0 && apq * apq > (kEpsD * kEpsD) * fabs(app * aqq)) {
              // t = tan of the rotation angle, the smaller root of
              // t^2 + 2 tau t - 1 = 0, tau = (a_qq - a_pp) / (2 a_pq)
              const double d = aqq - app;
              const double tt = (d >= 0.0 ? 2.0 : -2.0) * apq / (fabs(d) + sqrt(d * d + 4.0 * apq * apq));
              cl = 1.0 / sqrt(1.0 + tt * tt);
              sl = tt * cl;
              L.flag[0] = 1;
              if (fabs(tt) > kJacobiSmallRot) L.flag[4] = 1;
            }
          }
        }
      }
      int pp[kPairsPerWave], qq[kPairsPerWave];
      double cc[kPairsPerWave], ss[kPairsPerWave];
#pragma unroll
      for (int i = 0; i < kPairsPerWave; ++i) {
        pp[i] = __builtin_amdgcn_readlane(pl, i);
        qq[i] = __builtin_amdgcn_readlane(ql, i);
        cc[i] = lane_value(cl, i);
        ss[i] = lane_value(sl, i);  // 0: nothing to apply (uniform)
      }
      {
        double ap[kPairsPerWave][kColsPerLane], aq[kPairsPerWave][kColsPerLane];
#pragma unroll
        for (int i = 0; i < kPairsPerWave; ++i)
#pragma unroll
          for (int u = 0; u < kColsPerLane; ++u) {
            const int j = lane + 64 * u;
            if (ss[i] != 0.0 && j < m) {
              ap[i][u] = L.A[pp[i] * ld + j];
              aq[i][u] = L.A[qq[i] * ld + j];
            }
          }
#pragma unroll
        for (int i = 0; i < kPairsPerWave; ++i)
#pragma unroll
          for (int u = 0; u < kColsPerLane; ++u) {
            const int j = lane + 64 * u;
            if (ss[i] != 0.0 && j < m) {
              L.A[pp[i] * ld + j] = cc[i] * ap[i][u] - ss[i] * aq[i][u];
              L.A[qq[i] * ld + j] = ss[i] * ap[i][u] + cc[i] * aq[i][u];
            }
          }
      }
      __syncthreads();
      {
        double ap[kPairsPerWave][kColsPerLane], aq[kPairsPerWave][kColsPerLane];
        double vp[kPairsPerWave][kColsPerLane], vq[kPairsPerWave][kColsPerLane];
#pragma unroll
        for (int i = 0; i < kPairsPerWave; ++i)
#pragma unroll
          for (int u = 0; u < kColsPerLane; ++u) {
            const int j = lane + 64 * u;
            if (ss[i] != 0.0 && j < m) {
              ap[i][u] = L.A[j * ld + pp[i]];
              aq[i][u] = L.A[j * ld + qq[i]];
              vp[i][u] = L.V[j * ld + pp[i]];
              vq[i][u] = L.V[j * ld + qq[i]];
            }
          }
#pragma unroll
        for (int i = 0; i < kPairsPerWave; ++i)
#pragma unroll
          for (int u = 0; u < kColsPerLane; ++u) {
            const int j = lane + 64 * u;
            if (ss[i] != 0.0 && j < m) {
              L.A[j * ld + pp[i]] = (j == qq[i]) ? 0.0 : cc[i] * ap[i][u] - ss[i] * aq[i][u];
              L.A[j * ld + qq[i]] = (j == pp[i]) ? 0.0 : ss[i] * ap[i][u] + cc[i] * aq[i][u];
              L.V[j * ld + pp[i]] = cc[i] * vp[i][u] - ss[i] * vq[i][u];
              L.V[j * ld + qq[i]] = ss[i] * vp[i][u] + cc[i] * vq[i][u];
            }
          }
      }
      __syncthreads();
    }
    const int any = L.flag[0], large = L.flag[4];
    __syncthreads();
    if (!any || !large) {
      converged = true;
      break;
    }
  }
  // rank (ascending, ties by index) and sign (first nonzero component > 0)
  for (int j = tid; j < np; j += kDenThreads) L.dj[j] = (j < n) ? L.A[(size_t)j * ld + j] : 0.0;
  __syncthreads();
  for (int j = tid; j < n; j += kDenThreads) {
    const double d = L.dj[j];
    int rk = 0;
    for (int i = 0; i < n; ++i) {
      const double di = L.dj[i];
      rk += (di < d || (di == d && i < j)) ? 1 : 0;
    }
    double sgn = 1.0;
    for (int i = 0; i < n; ++i) {
      const double v = L.V[(size_t)i * ld + j];
      if (v != 0.0) {
        sgn = v < 0.0 ? -1.0 : 1.0;
        break;
      }
    }
    L.rank[j] = rk;
    L.sg[j] = sgn;
    L.lam[rk] = d;
    L.q0[rk] = sgn * L.V[j];
  }
  for (int j = n + tid; j < np; j += kDenThreads) {
    L.rank[j] = j;
    L.sg[j] = 0.0;  // padding columns carry no state
    L.lam[j] = 0.0;
    L.q0[j] = 0.0;
  }
  __syncthreads();
  return converged;
}

// The eigenvectors of the last solve (Jacobi order) into the trajectory's
// warm-start block.
__device__ __forceinline__ void save_basis(const ClassDev& c, const DenLds& L, double* W) {
  const int np = c.md.n_pad, ld = np + 1;
  for (int idx = threadIdx.x; idx < np * np; idx += kDenThreads) {
    const int i = idx / np, j = idx - i * np;
    W[idx] = L.V[(size_t)i * ld + j];
  }
}

// G = V^T H1 V on the matrix cores into Gd (ranked, sign-fixed basis; rows
// and columns n .. n_pad - 1 untouched; G on and above the diagonal,
// mirrored below), and the same n x n block into L.A (row stride
// n_pad + 1) for the couplings; T = H1 V passes through L.A before.
__device__ __forceinline__ void dense_project(const ClassDev& c, DenLds& L, double* Gd) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int n = c.md.n, np = opaque(c.md.n_pad), ld = np + 1, RT = np / 16;
  v4d acc[kTilesPerWave], acc2[kTilesPerWave];
  // T = H1 V (the diagonalised matrix in L.A is no longer needed)
  {
    const MatView h{c.H1, 1, np}, v{L.V, ld, 1};
    mm_tiles<false, kOne>(acc, acc2, RT, wave, lane, h, h, v, v);
  }
#pragma unroll
  for (int u = 0; u < kTilesPerWave; ++u) {
    int rt, ct;
    if (!tile_of<false>(wave, u, RT, rt, ct)) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) L.A[(size_t)(rt * 16 + lk + 4 * r) * ld + ct * 16 + lr] = acc[u][r];
  }
  __syncthreads();
  // G = V^T T, scattered to the ranked basis with the column signs
  {
    const MatView vt{L.V, 1, ld}, t{L.A, ld, 1};
    mm_tiles<true, kOne>(acc, acc2, RT, wave, lane, vt, vt, t, t);
  }
  __syncthreads();  // every wave done reading T
#pragma unroll
  for (int u = 0; u < kTilesPerWave; ++u) {
    int rt, ct;
    if (!tile_of<true>(wave, u, RT, rt, ct)) continue;
    const int b = ct * 16 + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = rt * 16 + lk + 4 * r;
      if (a <= b && b < n) {
        const double g = L.sg[a] * L.sg[b] * acc[u][r];
        const int ra = L.rank[a], rb = L.rank[b];
        Gd[(size_t)ra * np + rb] = g;
        Gd[(size_t)rb * np + ra] = g;
        L.A[ra * ld + rb] = g;
        L.A[rb * ld + ra] = g;
      }
    }
  }
  __syncthreads();  // Gd complete (work-group visibility of the global writes)
}

// D_jk = G_jk / (lambda_k - lambda_j) with G from L.A (left there by
// dense_project); zero on the diagonal and between states whose energies
// agree to 1e-12 of the largest |lambda|.
__device__ __forceinline__ double dense_D(const DenLds& L, int ld, double tol, int j, int k) {
  const double diff = L.lam[k] - L.lam[j];
  return (j == k || fabs(diff) <= tol) ? 0.0 : L.A[j * ld + k] / diff;
}

__device__ __forceinline__ double lam_tol(const DenLds& L, int n) {
  return 1e-12 * fmax(fabs(L.lam[0]), fabs(L.lam[n - 1]));
}

// Hellmann-Feynman force of the occupied set: -U0'(x) - sum_{a in s} G_aa.
__device__ __forceinline__ double dense_force(const ClassDev& c, const double* Gd, const int32_t* occ, double x,
                              DenLds& L) {
  const int np = c.md.n_pad;
  double part = 0.0;
  for (int r = threadIdx.x; r < c.md.N; r += kDenThreads) {
    const int a = occ[r];
    part += Gd[(size_t)a * np + a];
  }
  const double s = block_sum(part, L.red);
  const double k = c.md.mass * c.md.p[0] * c.md.p[0];
  return -k * (x - c.md.p[1]) - s;
}

__device__ __forceinline__ void dense_geo(double* geo, const ModelDev& md, double x) {
  const double k = md.mass * md.p[0] * md.p[0];
  const double u = x - md.p[1];
  geo[GEO_U0] = 0.5 * k * u * u;
  geo[GEO_DU0] = k * u;
  geo[GEO_DU0V] = k * u;
  geo[GEO_H] = 0.0;
  geo[GEO_DH] = 0.0;
  geo[GEO_RHO] = 0.0;
}

// One step of one trajectory up to the propagation (sub as in k_eig_step:
// -1 the whole step, j >= 0 the propagator of electronic sub-step j of nsub,
// -2 the end point only).
__global__ __launch_bounds__(kDenThreads) void k_dense_step(ClassDev c, double dt_run, int precision,
                                                             Counters* cnt, int sub, int nsub) {
  extern __shared__ double sm[];
  const int t = blockIdx.x, tid = threadIdx.x;
  if (t >= live_slots(c) || (c.status[t] & kFreezeMask)) return;
  const ModelDev& md = c.md;
  const int n = md.n, np = md.n_pad, RT = np / 16;
  DenLds L = dense_lds(sm, np);
  const double dt = c.clock ? c.clock[2 * (size_t)t] : dt_run;
  if (tid == 0) {
    const double x = c.x[t], v = c.v[t], F = c.F[t];
    const double vh = v + 0.5 * dt * F / md.mass;
    const double xn = x + dt * vh;
    L.nuc[0] = vh;
    L.nuc[1] = xn;
    L.nuc[2] = (sub >= 0) ? x + ((sub + 0.5) / nsub) * (xn - x) : 0.5 * (x + xn);
    L.flag[1] = 0;
  }
  __syncthreads();
  const double vh = L.nuc[0];
  const double dte = (sub >= 0) ? dt / nsub : dt;
  double* Gd = c.Gd + (size_t)t * np * np;
  // warm starts from the previous solve of this trajectory (its block is
  // keyed by the home index, so it needs no move when slots are compacted);
  // every kDenseColdEvery steps the midpoint solve starts cold (a bound on
  // how long a trajectory's solves depend on a carried basis; the refinement
  // itself restores orthonormality at every update), and the end-point solve
  // always starts from the midpoint solve of its own step
  double* W = c.Qw + (size_t)c.home[t] * np * np;
  const bool warm = (c.nsteps[t] % kDenseColdEvery) != 0;
  const double done = (precision == IESH_FP64) ? kPertDone : kPertDoneMixed;
  if (sub != -2) {
    // ---- propagator geometry: B = v D in the propagation's tile order
    if (!dense_eigen(c, L.nuc[2], L, warm ? W : nullptr, Gd, done) && tid == 0) L.flag[1] |= 1;
    save_basis(c, L, W);
    dense_project(c, L, Gd);
    const double tol = lam_tol(L, n);
    double* Bt = c.Bt ? c.Bt + (size_t)t * np * np : nullptr;
    float* Bt32 = c.Bt32 ? c.Bt32 + (size_t)t * np * np : nullptr;
    // a thread per (row j, quarter of the columns): rows rt*16 .. rt*16 + 15
    // of wave rt, quarter (lane >> 4); the quarters' sums of |B_jk| meet by
    // lane exchanges (a fixed order, so the interval is reproducible)
    {
      const int lane = tid & 63, rt = tid >> 6, lane_lo = lane & 15, qtr = lane >> 4;
      const int j = rt * 16 + lane_lo, kq = np / 4;
      double rsum = 0.0;
      if (rt < RT) {
        for (int k = qtr * kq; k < (qtr + 1) * kq; ++k) {
          const double val = (j < n && k < n) ? vh * dense_D(L, np + 1, tol, j, k) : 0.0;
          rsum += fabs(val);
          const size_t off = ((size_t)((k >> 2) * RT + rt) << 6) + lane_lo + ((k & 3) << 4);
          if (precision == IESH_FP64)
            Bt[off] = val;
          else
            Bt32[off] = (float)val;
        }
      }
      rsum += __shfl_xor(rsum, 16);
      rsum += __shfl_xor(rsum, 32);
      if (rt < RT && qtr == 0) L.rs[j] = rsum;
    }
    __syncthreads();
    double lo_part = 1e300, hi_part = -1e300;
    for (int j = tid; j < np; j += kDenThreads) {
      if (j < n) {
        lo_part = fmin(lo_part, L.lam[j] - L.rs[j]);
        hi_part = fmax(hi_part, L.lam[j] + L.rs[j]);
      }
      c.lam_mid[(size_t)t * np + j] = L.lam[j];
    }
    const double lo = block_min(lo_part, L.red), hi = block_max(hi_part, L.red);
    if (tid == 0) {
      double* cb = c.cheb + (size_t)t * kChebStride;
      if (write_cheb(cb, lo, hi, dte, precision, cnt, sub <= 0, L.J, c.work) < 0) L.flag[1] |= 2;
    }
    __syncthreads();
    if (sub >= 0) {
      if (tid == 0 && L.flag[1]) c.status[t] |= IESH_TRAJ_NONCONV;
      return;
    }
  }
  // ---- end point: energies, amplitudes, couplings for the hop, forces
  const double xn = L.nuc[1];
  if (!dense_eigen(c, xn, L, W, Gd, done) && tid == 0) L.flag[1] |= 1;
  save_basis(c, L, W);
  dense_project(c, L, Gd);
  for (int j = tid; j < np; j += kDenThreads) {
    c.lam[(size_t)t * np + j] = L.lam[j];
    c.q0[(size_t)t * np + j] = L.q0[j];
  }
  const double F = dense_force(c, Gd, c.occ + (size_t)t * md.N, xn, L);
  if (tid == 0) {
    double* geo = c.geo + (size_t)t * kGeoStride;
    dense_geo(geo, md, xn);
    int st = c.status[t];
    const double vn = vh + 0.5 * dt * F / md.mass;
    c.x[t] = xn;
    c.v[t] = vn;
    c.F[t] = F;
    if (!isfinite(xn) || !isfinite(vn)) st |= IESH_TRAJ_NONFINITE;
    if (L.flag[1]) st |= IESH_TRAJ_NONCONV;
    c.status[t] = st;
  }
}

// Eigen-solve and couplings at the current x (no dynamics); mode 1 also
// refreshes the force of the current occupations.
__global__ __launch_bounds__(kDenThreads) void k_dense_query(ClassDev c, int t0, int mode) {
  extern __shared__ double sm[];
  const int t = t0 + blockIdx.x, tid = threadIdx.x;
  const ModelDev& md = c.md;
  const int np = md.n_pad;
  DenLds L = dense_lds(sm, np);
  const double x = c.x[t];
  const bool ok = dense_eigen(c, x, L);
  // a state upload (mode 1) sets the warm-start basis; a plain query leaves
  // it, so that queries do not change the dynamics
  if (mode == 1) save_basis(c, L, c.Qw + (size_t)c.home[t] * np * np);
  double* Gd = c.Gd + (size_t)t * np * np;
  dense_project(c, L, Gd);
  for (int j = tid; j < np; j += kDenThreads) {
    c.lam[(size_t)t * np + j] = L.lam[j];
    c.q0[(size_t)t * np + j] = L.q0[j];
  }
  if (tid == 0) dense_geo(c.geo + (size_t)t * kGeoStride, md, x);
  if (mode == 1) {
    const double F = dense_force(c, Gd, c.occ + (size_t)t * md.N, x, L);
    if (tid == 0) {
      c.F[t] = F;
      if (!ok) c.status[t] |= IESH_TRAJ_NONCONV;
    }
  }
}

__device__ __forceinline__ double fermi_d(double e, double mu, double kT) {
  const double z = (e - mu) / kT;
  return (z > 0.0) ? exp(-z) / (1.0 + exp(-z)) : 1.0 / (1.0 + exp(z));
}

// Initial occupations at kT (fixed N: chemical potential by bisection, one
// uniform per level and attempt from Philox stream 1, the lowest N after
// 4096 failed attempts or at kT = 0) and unit-vector orbitals, as for the
// other model kinds.
__global__ __launch_bounds__(kDenThreads) void k_dense_init_thermal(ClassDev c, double kT,
                                                                     uint64_t seed) {
  extern __shared__ double sm[];
  const int t = blockIdx.x, tid = threadIdx.x;
  const ModelDev& md = c.md;
  const int n = md.n, np = md.n_pad, N = md.N;
  DenLds L = dense_lds(sm, np);
  const double x = c.x[t];
  const bool ok = dense_eigen(c, x, L);
  save_basis(c, L, c.Qw + (size_t)c.home[t] * np * np);
  double* Gd = c.Gd + (size_t)t * np * np;
  dense_project(c, L, Gd);
  int32_t* occ = c.occ + (size_t)t * N;
  // the chosen levels reuse the rank array (no longer needed)
  int* chosen = L.rank;
  bool done = false;
  if (kT > 0.0) {
    double lo = L.lam[0] - 50.0 * kT - 1.0, hi = L.lam[n - 1] + 50.0 * kT + 1.0;
    for (int it = 0; it < 200; ++it) {
      const double mu = 0.5 * (lo + hi);
      double part = 0.0;
      for (int a = tid; a < n; a += kDenThreads) part += fermi_d(L.lam[a], mu, kT);
      if (block_sum(part, L.red) > (double)N)
        hi = mu;
      else
        lo = mu;
    }
    const double mu = 0.5 * (lo + hi);
    const uint32_t gt = (uint32_t)c.gtraj[t];
    for (int attempt = 0; attempt < 4096 && !done; ++attempt) {
      int cntl = 0;
      for (int a = tid; a < n; a += kDenThreads) {
        const double u = philox_uniform(seed, gt, (uint64_t)attempt * n + a, 1u);
        chosen[a] = (u < fermi_d(L.lam[a], mu, kT)) ? 1 : 0;
        cntl += chosen[a];
      }
      done = ((int)block_sum((double)cntl, L.red) == N);
    }
  }
  __syncthreads();
  if (tid == 0) {
    int r = 0;
    for (int a = 0; a < n; ++a)
      if (done ? chosen[a] : (a < N)) occ[r++] = a;
  }
  __syncthreads();
  for (int idx = tid; idx < N * np; idx += kDenThreads) {
    const int j = idx / np, i = idx % np;
    const double val = (i == occ[j]) ? 1.0 : 0.0;
    if (c.C64) {
      c.C64[((size_t)t * N * np + idx) * 2] = val;
      c.C64[((size_t)t * N * np + idx) * 2 + 1] = 0.0;
    }
    if (c.C32) {
      c.C32[((size_t)t * N * np + idx) * 2] = (float)val;
      c.C32[((size_t)t * N * np + idx) * 2 + 1] = 0.0f;
    }
  }
  for (int j = tid; j < np; j += kDenThreads) {
    c.lam[(size_t)t * np + j] = L.lam[j];
    c.q0[(size_t)t * np + j] = L.q0[j];
  }
  const double F = dense_force(c, Gd, occ, x, L);
  if (tid == 0) {
    dense_geo(c.geo + (size_t)t * kGeoStride, md, x);
    c.F[t] = F;
    c.status[t] = ok ? 0 : IESH_TRAJ_NONCONV;
  }
}

hipError_t set_lds(const void* fn, size_t bytes) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

size_t dense_lds_size(int n_pad) { return dense_lds_bytes(n_pad); }

hipError_t launch_dense_step(const ClassDev& c, double dt, Counters* cnt, hipStream_t s, int sub,
                             int nsub) {
  const int precision = c.C64 ? IESH_FP64 : IESH_MIXED;
  if (c.n_live < 1) return hipSuccess;
  const size_t lds = dense_lds_bytes(c.md.n_pad);
  hipError_t e = set_lds((const void*)k_dense_step, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dense_step, dim3(c.n_live), dim3(kDenThreads), lds, s, c, dt, precision, cnt,
                     sub, nsub);
  return hipGetLastError();
}

hipError_t launch_dense_query(const ClassDev& c, int t0, int nt, int mode, hipStream_t s) {
  if (nt < 1) return hipSuccess;
  const size_t lds = dense_lds_bytes(c.md.n_pad);
  hipError_t e = set_lds((const void*)k_dense_query, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dense_query, dim3(nt), dim3(kDenThreads), lds, s, c, t0, mode);
  return hipGetLastError();
}

hipError_t launch_dense_init_thermal(const ClassDev& c, double kT, uint64_t seed, hipStream_t s) {
  if (c.n_traj < 1) return hipSuccess;
  const size_t lds = dense_lds_bytes(c.md.n_pad);
  hipError_t e = set_lds((const void*)k_dense_init_thermal, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dense_init_thermal, dim3(c.n_traj), dim3(kDenThreads), lds, s, c, kT, seed);
  return hipGetLastError();
}

}  // namespace iesh
