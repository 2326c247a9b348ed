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

// Im Phi and Re diag(Phi) as one real product per trajectory on the matrix
// cores.  With the flat orbital index f = (k - 1) N + o over the K N stored
// vectors (the tap layout [k-1][o][i] is contiguous in f), inner rows
// q = 2 f + part and
//   A[q][i] = w_k (Re s, -Im s)[part],   Bm[q][l] = (Im t, Re t)[part],
// Im Phi = A^T Bm.  Chunks of 4 orbitals (8 inner rows, two 16x16x4 FP64
// steps) are staged in LDS through registers: the global loads of chunk c+1
// are in flight while the waves multiply chunk c.  Element e of a chunk is
// the flat complex index c n_el + e of the stored vectors (n_el = 4 n_pad),
// so a thread's elements keep their LDS positions from chunk to chunk.  A
// work-group owns the rows [16 r0, 16 (r0 + nr)) of one trajectory's Phi
// (nr RT <= 64 tiles, contiguous row-major ranges per wave); the diagonal of
// its rows comes from the staged elements directly.
constexpr int kPhiWaves = 8;
constexpr int kPhiThreads = kPhiWaves * 64;
constexpr int kPhiOrb = 4;                        // orbitals per chunk
constexpr int kPhiMaxTiles = 64;                  // output tiles per work-group
constexpr int kPhiPer = (kPhiOrb * kMaxStates + kPhiThreads - 1) / kPhiThreads;

typedef double v4d __attribute__((ext_vector_type(4)));

// Row stride of an LDS panel of width 16 m: 16 mod 32 doubles, so the rows
// of one operand read start 32 banks apart.
__host__ __device__ constexpr int panel_ld(int m) { return 16 * m + ((m & 1) ? 0 : 16); }

__host__ __device__ inline int phi_rows_per_group(int RT) {
  const int nr = kPhiMaxTiles / RT;
  return nr < RT ? nr : RT;
}

struct PhiJob {
  double* As;  // LDS A panel [8][lda]
  double* Bs;  // LDS B panel [8][ldb]
  const double2* S;
  const double2* Tt;
  int lda, ldb, r0, RT, n_pad, N, i0, wa, n_el, n_chunks;
  size_t F_el;  // K N n_pad: stored complex elements of the trajectory
};

template <int NQ>
__device__ void phi_run(const PhiJob& J, int p0, double* Pm, double* rediag_t) {
  const int tid = threadIdx.x, lane = tid & 63, lrow = lane & 15, lk = lane >> 4;
  const size_t wN = (size_t)J.N * J.n_pad;  // elements of the k = 1 vectors (weight 1)
  // this thread's elements: LDS offsets and whether they fall in the A rows
  int offB[kPhiPer], offA[kPhiPer];
  bool inA[kPhiPer], live[kPhiPer];
#pragma unroll
  for (int r = 0; r < kPhiPer; ++r) {
    const int e = tid + r * kPhiThreads;
    const int ff = e / J.n_pad, i = e - ff * J.n_pad;
    live[r] = e < J.n_el;
    inA[r] = live[r] && i >= J.i0 && i < J.i0 + J.wa;
    offB[r] = 2 * ff * J.ldb + i;
    offA[r] = 2 * ff * J.lda + i - J.i0;
  }
  double2 sv[kPhiPer], tv[kPhiPer];
  double dsum[kPhiPer];
#pragma unroll
  for (int r = 0; r < kPhiPer; ++r) dsum[r] = 0.0;
  auto fetch = [&](int ch) {
#pragma unroll
    for (int r = 0; r < kPhiPer; ++r) {
      const size_t g = (size_t)ch * J.n_el + tid + r * kPhiThreads;
      sv[r] = make_double2(0.0, 0.0);
      tv[r] = make_double2(0.0, 0.0);
      if (live[r] && g < J.F_el) {
        tv[r] = J.Tt[g];
        if (inA[r]) {
          sv[r] = J.S[g];
          if (g >= wN) sv[r] = make_double2(2.0 * sv[r].x, 2.0 * sv[r].y);
        }
      }
    }
  };
  v4d acc[NQ > 0 ? NQ : 1];
  int ra[NQ > 0 ? NQ : 1], cb[NQ > 0 ? NQ : 1];
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
    const int p = p0 + u, pr = p / J.RT, pc = p - pr * J.RT;
    ra[u] = lk * J.lda + 16 * pr + lrow;
    cb[u] = lk * J.ldb + 16 * pc + lrow;
  }
  if (J.n_chunks > 0) fetch(0);
  for (int ch = 0; ch < J.n_chunks; ++ch) {
    __syncthreads();  // the previous chunk's operands are consumed
#pragma unroll
    for (int r = 0; r < kPhiPer; ++r) {
      if (live[r]) {
        J.Bs[offB[r]] = tv[r].y;
        J.Bs[offB[r] + J.ldb] = tv[r].x;
      }
      if (inA[r]) {
        J.As[offA[r]] = sv[r].x;
        J.As[offA[r] + J.lda] = -sv[r].y;
        dsum[r] += sv[r].x * tv[r].x + sv[r].y * tv[r].y;
      }
    }
    __syncthreads();
    if (ch + 1 < J.n_chunks) fetch(ch + 1);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int u = 0; u < NQ; ++u) {
        const double a = J.As[ra[u] + 4 * j * J.lda];
        const double b = J.Bs[cb[u] + 4 * j * J.ldb];
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    const int p = p0 + u, pr = p / J.RT, pc = p - pr * J.RT;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      Pm[(size_t)(16 * (J.r0 + pr) + lk + 4 * r) * J.n_pad + 16 * pc + lrow] = acc[u][r];
  }
  // diagonal: per-element partial sums to LDS (over the B panel), then the
  // sum over the 4 orbitals of a chunk position
  __syncthreads();
  double* dp = J.Bs;  // [4][n_pad] fits in [8][ldb]
#pragma unroll
  for (int r = 0; r < kPhiPer; ++r)
    if (live[r]) dp[tid + r * kPhiThreads] = dsum[r];
  __syncthreads();
  for (int i = J.i0 + tid; i < J.i0 + J.wa; i += kPhiThreads) {
    double d = 0.0;
    for (int ff = 0; ff < kPhiOrb; ++ff) d += dp[ff * J.n_pad + i];
    rediag_t[i] = d;
  }
}

__global__ __launch_bounds__(kPhiThreads) void k_adj_phi(ClassDev c, const double* taps_s,
                                                         const double* taps_t, int tap_k,
                                                         double* imphi, double* rediag) {
  extern __shared__ double phi_smem[];
  const int n_pad = c.md.n_pad, N = c.md.N, RT = n_pad >> 4;
  const int nr_max = phi_rows_per_group(RT);
  const int n_blk = (RT + nr_max - 1) / nr_max;
  // blocks of one trajectory on one XCD (they share the Chebyshev vectors in L2)
  const int b = blockIdx.x, xcd = b & 7, local = b >> 3;
  const int blk = local % n_blk;
  const int t = (local / n_blk) * 8 + xcd;
  if (t >= c.n_live) return;
  PhiJob J;
  J.r0 = blk * nr_max;
  const int nr = min(nr_max, RT - J.r0);
  J.RT = RT;
  J.n_pad = n_pad;
  J.N = N;
  J.i0 = 16 * J.r0;
  J.wa = 16 * nr;
  J.lda = panel_ld(nr);
  J.ldb = panel_ld(RT);
  J.As = phi_smem;
  J.Bs = phi_smem + 8 * J.lda;
  const int K = (int)c.cheb[(size_t)t * kChebStride + CHEB_K];
  J.n_el = kPhiOrb * n_pad;
  J.F_el = (size_t)K * N * n_pad;
  J.n_chunks = (K * N + kPhiOrb - 1) / kPhiOrb;
  const size_t per_traj = (size_t)tap_k * N * n_pad * 2;
  J.S = reinterpret_cast<const double2*>(taps_s + (size_t)t * per_traj);
  J.Tt = reinterpret_cast<const double2*>(taps_t + (size_t)t * per_traj);
  // wave's tiles: contiguous row-major range of the nr x RT tiles
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int P = nr * RT;
  const int base_q = P / kPhiWaves, rem_q = P % kPhiWaves;
  const int nq = base_q + (wave < rem_q ? 1 : 0);
  const int p0 = wave * base_q + (wave < rem_q ? wave : rem_q);
  double* Pm = imphi + (size_t)t * n_pad * n_pad;
  double* rd = rediag + (size_t)t * n_pad;
  switch (nq) {
    case 0: phi_run<0>(J, p0, Pm, rd); break;
    case 1: phi_run<1>(J, p0, Pm, rd); break;
    case 2: phi_run<2>(J, p0, Pm, rd); break;
    case 3: phi_run<3>(J, p0, Pm, rd); break;
    case 4: phi_run<4>(J, p0, Pm, rd); break;
    case 5: phi_run<5>(J, p0, Pm, rd); break;
    case 6: phi_run<6>(J, p0, Pm, rd); break;
    case 7: phi_run<7>(J, p0, Pm, rd); break;
    default: phi_run<8>(J, p0, Pm, rd); break;
  }
}

}  // namespace

hipError_t launch_adj_loss(const ClassDev& c, double* loss, int s, int T, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_loss, dim3(c.n_traj), dim3(kLossThreads), 0, st, c, loss, s, T);
  return hipGetLastError();
}

hipError_t launch_adj_phi(const ClassDev& c, const double* taps_s, const double* taps_t, int tap_k,
                          double* imphi, double* rediag, hipStream_t st) {
  if (c.n_live < 1) return hipSuccess;
  const int RT = c.md.n_pad / 16;
  const int nr = phi_rows_per_group(RT);
  const int n_blk = (RT + nr - 1) / nr;
  const size_t lds = sizeof(double) * 8 * (panel_ld(nr) + panel_ld(RT));
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_adj_phi,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int n_traj_pad = (c.n_live + 7) / 8 * 8;
  hipLaunchKernelGGL(k_adj_phi, dim3(n_traj_pad * n_blk), dim3(kPhiThreads), lds, st, c, taps_s,
                     taps_t, tap_k, imphi, rediag);
  return hipGetLastError();
}

}  // namespace iesh
