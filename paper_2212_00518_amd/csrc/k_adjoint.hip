// Path loss and the contraction of the adjoint Chebyshev vectors (adjoint
// pattern along prescribed nuclear paths).
//
// Loss of one path (impurity population and electronic excitation energy of
// the Newns-Anderson model, Sec. II.B and III.B):
//   L = (1/T) sum_{s=1..T} P(s) + E_exc(T),  P(s) = sum_o |sum_a q0_a(x_s) C_ao(s)|^2,
//   E_exc = sum_a lambda_a(x_T) (rho_a - n0_a),  rho_a = sum_o |C_ao(T)|^2.
//
// Reverse mode through one propagation y = sum_k c_k T_k(At) x with output
// cotangent g: the cotangent of x is the same series with conjugated
// coefficients applied to g (its Clenshaw vectors s_k, k = K .. 1), and the
// derivative with respect to At is
//   Phi = sum_{k=1..K} w_k conj(s_k) t_{k-1}^T,  w_1 = 1, w_k = 2 (k > 1),
// with the Chebyshev vectors t_k = T_k(At) x.  Only Im Phi and the real
// diagonal are needed (A = diag(lambda) - i v D with real lambda, D).

#include "iesh_internal.hpp"

namespace iesh {
namespace {

constexpr int kLossThreads = 256;
constexpr int kPhiThreads = 256;
constexpr int kPhiChunk = 8;  // orbitals staged per LDS chunk
constexpr int kMaxRT = (kMaxStates + 15) / 16;

// loss[g] += P(s+1) / T (and E_exc at the last step), with lambda, q0 at the
// end point of step s and the propagated orbitals.
__global__ __launch_bounds__(kLossThreads) void k_adj_loss(ClassDev c, double* loss, int s, int T) {
  __shared__ double red[kLossThreads];
  const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = c.md.n, n_pad = c.md.n_pad, N = c.md.N;
  const double* C = c.C64 + (size_t)t * N * n_pad * 2;
  const double* q0 = c.q0 + (size_t)t * n_pad;
  const double* lam = c.lam + (size_t)t * n_pad;
  double part = 0.0;
  for (int o = wv; o < N; o += kLossThreads / 64) {
    double zr = 0.0, zi = 0.0;
    for (int a = lane; a < n; a += 64) {
      zr += q0[a] * C[((size_t)o * n_pad + a) * 2];
      zi += q0[a] * C[((size_t)o * n_pad + a) * 2 + 1];
    }
    for (int m = 32; m > 0; m >>= 1) {
      zr += __shfl_xor(zr, m);
      zi += __shfl_xor(zi, m);
    }
    if (lane == 0) part += (zr * zr + zi * zi) / T;
  }
  if (s == T - 1) {
    for (int a = tid; a < n; a += kLossThreads) {
      double rho = 0.0;
      for (int o = 0; o < N; ++o) {
        const double cr = C[((size_t)o * n_pad + a) * 2], ci = C[((size_t)o * n_pad + a) * 2 + 1];
        rho += cr * cr + ci * ci;
      }
      bool occ = false;
      for (int r = 0; r < N; ++r) occ |= (c.occ[(size_t)t * N + r] == a);
      part += lam[a] * (rho - (occ ? 1.0 : 0.0));
    }
  }
  red[tid] = part;
  __syncthreads();
  for (int st = kLossThreads / 2; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) loss[c.gtraj[t]] += red[0];
}

// Work-group (trajectory t, row tile rt): rows i = 16 rt + ti, columns
// l = tg + 16 cl; Im Phi[i][l] and Re Phi[i][i].
__global__ __launch_bounds__(kPhiThreads) void k_adj_phi(ClassDev c, const double* taps_s,
                                                         const double* taps_t, int tap_k,
                                                         double* imphi, double* rediag) {
  __shared__ double2 ts[kPhiChunk][kMaxStates];  // t_{k-1}[o][l]
  __shared__ double2 ss[kPhiChunk][16];          // s_k[o][i]
  const int RT = c.md.n_pad / 16;
  const int t = blockIdx.x / RT, rt = blockIdx.x % RT;
  const int tid = threadIdx.x, ti = tid & 15, tg = tid >> 4;
  const int n_pad = c.md.n_pad, N = c.md.N;
  const int K = (int)c.cheb[(size_t)t * kChebStride + CHEB_K];
  const size_t per_k = (size_t)N * n_pad * 2;
  const double* S = taps_s + (size_t)t * tap_k * per_k;
  const double* Tt = taps_t + (size_t)t * tap_k * per_k;
  const int i = 16 * rt + ti;
  double acc[kMaxRT];
#pragma unroll
  for (int cl = 0; cl < kMaxRT; ++cl) acc[cl] = 0.0;
  double dg = 0.0;
  for (int k = 1; k <= K; ++k) {
    const double w = (k == 1) ? 1.0 : 2.0;
    const double* sk = S + (size_t)(k - 1) * per_k;
    const double* tk = Tt + (size_t)(k - 1) * per_k;
    for (int o0 = 0; o0 < N; o0 += kPhiChunk) {
      const int no = min(kPhiChunk, N - o0);
      __syncthreads();
      for (int e = tid; e < no * n_pad; e += kPhiThreads) {
        const int oo = e / n_pad, l = e - oo * n_pad;
        const size_t off = ((size_t)(o0 + oo) * n_pad + l) * 2;
        ts[oo][l] = make_double2(tk[off], tk[off + 1]);
      }
      for (int e = tid; e < no * 16; e += kPhiThreads) {
        const int oo = e >> 4, ii = e & 15;
        const size_t off = ((size_t)(o0 + oo) * n_pad + 16 * rt + ii) * 2;
        ss[oo][ii] = make_double2(w * sk[off], w * sk[off + 1]);
      }
      __syncthreads();
      for (int oo = 0; oo < no; ++oo) {
        const double2 sv = ss[oo][ti];
#pragma unroll
        for (int cl = 0; cl < kMaxRT; ++cl) {
          const int l = tg + 16 * cl;
          if (cl < RT) {
            const double2 tv = ts[oo][l];
            acc[cl] += sv.x * tv.y - sv.y * tv.x;  // Im(conj(s) t)
          }
        }
        if (tg == ti) {  // the thread whose column set holds l = i (cl = rt)
          const double2 tv = ts[oo][i];
          dg += sv.x * tv.x + sv.y * tv.y;
        }
      }
    }
  }
  double* P = imphi + (size_t)t * n_pad * n_pad;
#pragma unroll
  for (int cl = 0; cl < kMaxRT; ++cl) {
    const int l = tg + 16 * cl;
    if (cl < RT) P[(size_t)i * n_pad + l] = acc[cl];
  }
  if (tg == ti) rediag[(size_t)t * n_pad + i] = dg;
}

}  // namespace

hipError_t launch_adj_loss(const ClassDev& c, double* loss, int s, int T, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_loss, dim3(c.n_traj), dim3(kLossThreads), 0, st, c, loss, s, T);
  return hipGetLastError();
}

hipError_t launch_adj_phi(const ClassDev& c, const double* taps_s, const double* taps_t, int tap_k,
                          double* imphi, double* rediag, hipStream_t st) {
  const int RT = c.md.n_pad / 16;
  hipLaunchKernelGGL(k_adj_phi, dim3(c.n_traj * RT), dim3(kPhiThreads), 0, st, c, taps_s, taps_t,
                     tap_k, imphi, rediag);
  return hipGetLastError();
}

}  // namespace iesh
