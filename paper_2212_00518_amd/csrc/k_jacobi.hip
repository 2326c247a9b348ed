// Batched eigen-decomposition of general dense symmetric matrices by cyclic
// two-sided Jacobi rotations: the fallback for a one-electron Hamiltonian
// that is not an arrowhead (the arrowhead case has its own secular solver).
//
// One work-group per matrix; the matrix A and the accumulated rotations V
// live in LDS for orders up to IESH_JACOBI_LDS_N, beyond that in a global
// workspace (same code, generic pointers).  A sweep visits every index
// pair once in m - 1 rounds of m/2 disjoint pairs (round-robin schedule over
// m = n rounded up to even; pairs with the padding index are skipped), so
// the rotations of a round are independent: one pass rotates the rows of
// every pair, a second the columns of A and V.  In the global workspace V is
// kept transposed (row j holds eigenvector j), so its update walks rows and
// only A's column update reads one cache line per element.  The rotation of
// pair (p, q)
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

constexpr int kJacThreads = 256;
constexpr int kJacWaves = kJacThreads / 64;
constexpr int kChunk = 2;  // pairs a wave rotates per batch of loads
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
      // rows p, q of every pair: rows <- J^T rows.  A wave takes pairs wave,
      // wave + 4, ... (kChunk at a time) and a lane columns lane, lane + 64,
      // ...; the elements of a chunk are all loaded before any is stored.
      for (int k0 = wave; k0 < half; k0 += kJacWaves * kChunk) {
        int pp[kChunk], qq[kChunk];
        double cc[kChunk], ss[kChunk];
#pragma unroll
        for (int i = 0; i < kChunk; ++i) {
          const int k = k0 + kJacWaves * i, kk = (k < half) ? k : 0;
          ss[i] = (k < half) ? sn[kk] : 0.0;  // 0: nothing to apply (uniform)
          cc[i] = cs[kk];
          pp[i] = pq[2 * kk];
          qq[i] = pq[2 * kk + 1];
        }
#pragma unroll 1
        for (int j = lane; j < m; j += 64) {
          double ap[kChunk], aq[kChunk];
#pragma unroll
          for (int i = 0; i < kChunk; ++i)
            if (ss[i] != 0.0) {
              ap[i] = A[pp[i] * ld + j];
              aq[i] = A[qq[i] * ld + j];
            }
#pragma unroll
          for (int i = 0; i < kChunk; ++i)
            if (ss[i] != 0.0) {
              A[pp[i] * ld + j] = cc[i] * ap[i] - ss[i] * aq[i];
              A[qq[i] * ld + j] = ss[i] * ap[i] + cc[i] * aq[i];
            }
        }
      }
      __syncthreads();
      // columns p, q of A and V: columns <- columns J (a lane per row)
      for (int k0 = wave; k0 < half; k0 += kJacWaves * kChunk) {
        int pp[kChunk], qq[kChunk];
        double cc[kChunk], ss[kChunk];
#pragma unroll
        for (int i = 0; i < kChunk; ++i) {
          const int k = k0 + kJacWaves * i, kk = (k < half) ? k : 0;
          ss[i] = (k < half) ? sn[kk] : 0.0;
          cc[i] = cs[kk];
          pp[i] = pq[2 * kk];
          qq[i] = pq[2 * kk + 1];
        }
#pragma unroll 1
        for (int j = lane; j < m; j += 64) {
          double ap[kChunk], aq[kChunk], vp[kChunk], vq[kChunk];
#pragma unroll
          for (int i = 0; i < kChunk; ++i)
            if (ss[i] != 0.0) {
              ap[i] = A[j * ld + pp[i]];
              aq[i] = A[j * ld + qq[i]];
              vp[i] = V[vix(j, pp[i])];
              vq[i] = V[vix(j, qq[i])];
            }
#pragma unroll
          for (int i = 0; i < kChunk; ++i)
            if (ss[i] != 0.0) {
              // the annihilated pair (rows p and q of columns q and p) is set to zero
              A[j * ld + pp[i]] = (j == qq[i]) ? 0.0 : cc[i] * ap[i] - ss[i] * aq[i];
              A[j * ld + qq[i]] = (j == pp[i]) ? 0.0 : ss[i] * ap[i] + cc[i] * aq[i];
              V[vix(j, pp[i])] = cc[i] * vp[i] - ss[i] * vq[i];
              V[vix(j, qq[i])] = ss[i] * vp[i] + cc[i] * vq[i];
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
