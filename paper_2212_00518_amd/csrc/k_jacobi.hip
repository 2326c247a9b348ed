// Batched eigen-decomposition of general dense symmetric matrices by cyclic
// two-sided Jacobi rotations: the fallback for a one-electron Hamiltonian
// that is not an arrowhead (the arrowhead case has its own secular solver).
//
// One work-group per matrix; the matrix A and the accumulated rotations V
// live in LDS for orders up to IESH_JACOBI_LDS_N, beyond that in a global
// workspace (same code, generic pointers).  A sweep visits every index
// pair once in m - 1 rounds of m/2 disjoint pairs (round-robin schedule over
// m = n rounded up to even; pairs with the padding index are skipped), so
// the rotations of a round are independent, and A <- J^T A J takes one pass
// over 2x2 blocks (rows of one pair, columns of another), each a function of
// itself alone, so a round touches A by rows only and in place.  In the
// global workspace V is kept transposed (row j holds eigenvector j), so its
// update walks rows too.  The rotation of pair (p, q)
// annihilates a_pq (Golub and Van Loan, symmetric Schur decomposition):
//   tau = (a_qq - a_pp) / (2 a_pq),  t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1 / sqrt(1 + t^2),  s = t c,  A <- J^T A J,  V <- V J,
// with J the identity except J_pp = J_qq = c, J_pq = s, J_qp = -s.  A pair is
// skipped once |a_pq| <= eps sqrt(|a_pp a_qq|) (eps the FP64 unit roundoff
// times 2; the relative-accuracy stopping rule of Demmel and Veselic) or
// a_pq = 0; the iteration ends after a sweep without rotations or whose
// rotations were all below kSmallRot (or reports non-convergence after
// max_sweeps).

#include "iesh_internal.hpp"

namespace iesh {
namespace {

constexpr int kJacThreads = 1024;
constexpr int kJacWaves = kJacThreads / 64;
// A sweep whose rotations all have |tan| below this ends the iteration: the
// off-diagonal elements it leaves are about the square of its largest
// rotation relative to the gaps, so the next sweep would only rotate by
// angles near rounding.
constexpr double kSmallRot = 1e-8;

// LDS bytes: A and V (when in LDS), the rotations of a round and the pairs.
size_t jacobi_lds(int n, bool in_lds) {
  const int m = n + (n & 1);
  return sizeof(double) * ((in_lds ? 2 * (size_t)m * (m + 1) : 0) + m) + sizeof(int) * (m + 4);
}

template <bool kLds>
__global__ __launch_bounds__(kJacThreads) void k_jacobi(const double* __restrict__ H, int n,
                                                       double* __restrict__ lam,
                                                       double* __restrict__ Q, int32_t* sweeps_out,
                                                       int max_sweeps, double* work) {
  extern __shared__ double sm[];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int m = n + (n & 1), half = m / 2;
  const int ld = m + 1;             // row stride: a column walk spreads over the LDS banks
  double* A = kLds ? sm : work + (size_t)b * 2 * m * ld;  // [m][ld]
  double* V = A + (size_t)m * ld;   // [m][ld]: V, transposed in the workspace
  // element (i, j) of V: row-major in LDS, column-major in the workspace
  const auto vix = [ld](int i, int j) { return kLds ? i * ld + j : j * ld + i; };
  double* cs = kLds ? V + (size_t)m * ld : sm;  // [half] cosines of the round
  double* sn = cs + half;           // [half] sines
  int* pq = reinterpret_cast<int*>(sn + half);  // [m]: p, q of each pair
  int* flag = pq + m;               // [2]: a rotation, a rotation above kSmallRot in this sweep

  const double* Hb = H + (size_t)b * n * n;
  for (int idx = tid; idx < m * m; idx += kJacThreads) {
    const int i = idx / m, j = idx - i * m;
    A[(size_t)i * ld + j] = (i < n && j < n) ? Hb[(size_t)i * n + j] : 0.0;
    V[vix(i, j)] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();

  int sweep = 0;
  bool converged = false;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) {
      flag[0] = 0;
      flag[1] = 0;
    }
    __syncthreads();
    for (int r = 0; r < m - 1; ++r) {
      // the pairs of round r and their rotations
      for (int k = tid; k < half; k += kJacThreads) {
        int p, q;
        if (k == 0) {
          p = r;
          q = m - 1;
        } else {
          p = (r + k) % (m - 1);
          q = (r - k + (m - 1)) % (m - 1);
        }
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[(size_t)p * ld + q];
          const double app = A[(size_t)p * ld + p], aqq = A[(size_t)q * ld + q];
          if (apq != 0.0 && fabs(apq) > 2.220446049250313e-16 * sqrt(fabs(app) * fabs(aqq))) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = copysign(1.0, tau) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            flag[0] = 1;
            if (fabs(t) > kSmallRot) flag[1] = 1;
          }
        }
        pq[2 * k] = p;
        pq[2 * k + 1] = q;
        cs[k] = c;
        sn[k] = s;
      }
      __syncthreads();
      // A <- J^T A J in one pass: the 2x2 block of rows (p_a, q_a) and
      // columns (p_b, q_b) becomes J_a^T B J_b and depends on that block
      // only, so a lane reads and then writes its own four elements (a wave
      // takes row pairs a = wave, wave + 16, ..., a lane column pairs
      // b = lane, lane + 64, ...; blocks of two pairs without rotation stay).
      // V <- V J_a in the same pass (columns p_a, q_a of V).
      for (int a = wave; a < half; a += kJacWaves) {
        const int pa = pq[2 * a], qa = pq[2 * a + 1];
        const double ca = cs[a], sa = sn[a];
        double* rp = A + (size_t)pa * ld;
        double* rq = A + (size_t)qa * ld;
#pragma unroll 1
        for (int bb = lane; bb < half; bb += 64) {
          const double sb = sn[bb];
          if (sa == 0.0 && sb == 0.0) continue;
          const int pb = pq[2 * bb], qb = pq[2 * bb + 1];
          const double cb = cs[bb];
          const double a_pp = rp[pb], a_pq = rp[qb], a_qp = rq[pb], a_qq = rq[qb];
          // rows: J_a^T B
          const double xpp = ca * a_pp - sa * a_qp, xpq = ca * a_pq - sa * a_qq;
          const double xqp = sa * a_pp + ca * a_qp, xqq = sa * a_pq + ca * a_qq;
          // columns: (J_a^T B) J_b; the annihilated pair is set to zero
          rp[pb] = cb * xpp - sb * xpq;
          rp[qb] = (bb == a) ? 0.0 : sb * xpp + cb * xpq;
          rq[pb] = (bb == a) ? 0.0 : cb * xqp - sb * xqq;
          rq[qb] = sb * xqp + cb * xqq;
        }
        if (sa != 0.0) {
#pragma unroll 1
          for (int j = lane; j < m; j += 64) {
            const double vp = V[vix(j, pa)], vq = V[vix(j, qa)];
            V[vix(j, pa)] = ca * vp - sa * vq;
            V[vix(j, qa)] = sa * vp + ca * vq;
          }
        }
      }
      __syncthreads();
    }
    const int any = flag[0], large = flag[1];
    __syncthreads();
    if (!any || !large) {
      converged = true;
      break;
    }
  }

  // ascending order (ties by index) and the phase: the first component of
  // each eigenvector above 1e-12 of its largest is made positive
  int* rank = pq;  // reuse: [m]
  for (int j = tid; j < n; j += kJacThreads) {
    const double dj = A[(size_t)j * ld + j];
    int rk = 0;
    for (int i = 0; i < n; ++i) {
      const double di = A[(size_t)i * ld + i];
      rk += (di < dj || (di == dj && i < j)) ? 1 : 0;
    }
    rank[j] = rk;
  }
  __syncthreads();
  for (int j = tid; j < n; j += kJacThreads) {
    double vmax = 0.0;
    for (int i = 0; i < n; ++i) vmax = fmax(vmax, fabs(V[vix(i, j)]));
    double sgn = 1.0;
    for (int i = 0; i < n; ++i) {
      const double v = V[vix(i, j)];
      if (fabs(v) > 1e-12 * vmax) {
        sgn = v < 0.0 ? -1.0 : 1.0;
        break;
      }
    }
    const int rk = rank[j];
    lam[(size_t)b * n + rk] = A[(size_t)j * ld + j];
    double* Qb = Q + (size_t)b * n * n;
    for (int i = 0; i < n; ++i) Qb[(size_t)i * n + rk] = sgn * V[vix(i, j)];
  }
  if (tid == 0 && sweeps_out) sweeps_out[b] = converged ? sweep + 1 : -1;
}

}  // namespace

size_t jacobi_work_elems(int n, int batch) {
  if (n <= IESH_JACOBI_LDS_N) return 0;
  const size_t m = n + (n & 1);
  return (size_t)batch * 2 * m * (m + 1);
}

hipError_t launch_jacobi(const double* H, int n, int batch, double* lam, double* Q, int32_t* sweeps,
                         double* work, hipStream_t s) {
  const bool in_lds = n <= IESH_JACOBI_LDS_N;
  const size_t lds = jacobi_lds(n, in_lds);
  const void* fn = in_lds ? (const void*)k_jacobi<true> : (const void*)k_jacobi<false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (in_lds)
    hipLaunchKernelGGL(k_jacobi<true>, dim3(batch), dim3(kJacThreads), lds, s, H, n, lam, Q, sweeps, 60,
                       work);
  else
    hipLaunchKernelGGL(k_jacobi<false>, dim3(batch), dim3(kJacThreads), lds, s, H, n, lam, Q, sweeps, 60,
                       work);
  return hipGetLastError();
}

}  // namespace iesh
