// Path loss, its hop-probability term, and the contraction of the adjoint
// Chebyshev vectors (adjoint pattern along prescribed nuclear paths).
//
// Loss of one path with term weights (c_P, c_E, c_G, c_F), at x_s (s = 1..T):
//   L = c_P (1/T) sum_s P(s) + c_E E_exc(T) + c_G (1/T) sum_s G(s) + c_F (1/T) sum_s F(s),
//   P(s) = sum_o |sum_a q0_a C_ao(s)|^2            (impurity population, Sec. III.B),
//   E_exc = sum_a lambda_a(x_T) (rho_a - n0_a),     rho_a = sum_o |C_ao(T)|^2,
//   G(s) = sum_{a occupied, b not} g_ab,  g_ab = max(-2 dt v D_ba Re W_b,r(a), 0),
//          W = C_U S^-1 (Eqs. hopping_probability and hopping_rate),
//   F(s) = -dU0/dx - h' sum_{a occupied} q0_a^2     (Eq. classical_hamiltonian),
// occupations held at their initial values, v = (x_s - x_{s-1}) / dt.
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
constexpr int kHopAdjThreads = 256;

// loss[g] += the P, F terms at x_{s+1} (and E_exc at the last step), with
// lambda, q0 at the end point of step s and the propagated orbitals.
__global__ __launch_bounds__(kLossThreads) void k_adj_loss(ClassDev c, double* loss, int s, int T,
                                                           AdjTerms w) {
  __shared__ double red[kLossThreads];
  const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = c.md.n, n_pad = c.md.n_pad, N = c.md.N;
  const double* C = c.C64 + (size_t)t * N * n_pad * 2;
  const double* q0 = c.q0 + (size_t)t * n_pad;
  const double* lam = c.lam + (size_t)t * n_pad;
  const int32_t* occ = c.occ + (size_t)t * N;
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
    if (lane == 0) part += w.cP * (zr * zr + zi * zi) / T;
  }
  if (w.cF != 0.0) {
    // Hellmann-Feynman force on the held occupations (harmonic model)
    const double omega = c.md.p[0], g = c.md.p[1], m = c.md.mass;
    const double x = c.path[(size_t)c.gtraj[t] * c.path_len + s + 1];
    const double hp = -m * omega * omega * g;
    for (int r = tid; r < N; r += kLossThreads) {
      const double q = q0[occ[r]];
      part -= w.cF * hp * q * q / T;
    }
    if (tid == 0) part -= w.cF * m * omega * omega * x / T;
  }
  if (s == T - 1) {
    for (int a = tid; a < n; a += kLossThreads) {
      double rho = 0.0;
      for (int o = 0; o < N; ++o) {
        const double cr = C[((size_t)o * n_pad + a) * 2], ci = C[((size_t)o * n_pad + a) * 2 + 1];
        rho += cr * cr + ci * ci;
      }
      bool oc = false;
      for (int r = 0; r < N; ++r) oc |= (occ[r] == a);
      part += w.cE * lam[a] * (rho - (oc ? 1.0 : 0.0));
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

// Hop-probability term at x_s for one trajectory (one work-group).
// S = C[occupied rows] is inverted in place by Gauss-Jordan elimination with
// partial (row) pivoting, the row interchanges undone as column interchanges
// at the end; the N x N matrix lives in LDS when it fits the work-group's
// dynamic LDS, else in the trajectory's scratch block.  W = C_U X, the pair
// probabilities g_ab and (forward) their sum into the loss.  Reverse: with
// R_br = dL/dRe W_br = c [g_ab > 0] (-2 dt v D_ba) and Dbar_ba = c [g_ab > 0]
// (-2 dt v Re W_br) (c = weight c_G / T), the orbital cotangents are
//   Gbar_U = R X^H,  Gbar_S = -W^H Gbar_U   (added as halves to the Wirtinger
// cotangent Gh), and D_ba = h' q0_b q0_a / (lambda_a - lambda_b) passes Dbar
// to (q0, lambda, h'), written to hopbar = [qbar (n_pad) | lbar (n_pad) | hpbar]
// for the reverse of the end-point eigen-solve.  Sums run in a fixed order.
// Scratch per trajectory (doubles): S 2 N^2, W and Gbar_U 2 n_pad N each,
// R and Dbar n_pad N each.
__host__ __device__ inline size_t hop_adj_scratch(int n_pad, int N) {
  return (size_t)2 * N * N + (size_t)6 * n_pad * N;
}

// Dynamic LDS of the hop-term kernel: the N x N inverse when it fits.
constexpr size_t kHopAdjLdsMax = 128 * 1024;
inline size_t hop_adj_lds(int N) {
  const size_t b = (size_t)N * N * sizeof(double2);
  return b <= kHopAdjLdsMax ? b : 0;
}

// kLds: the inverse lives in LDS, known at compile time so that its accesses
// are LDS instructions (a pointer that may point either way compiles to flat
// accesses, which take the memory path even for LDS).
template <bool kLds>
__global__ __launch_bounds__(kHopAdjThreads) void k_adj_hop(ClassDev c, const double* Cs, double* Gh,
                                                            double* scr, const double* weights,
                                                            double* loss, double* hopbar, int s,
                                                            int T, double dt, double cG, int reverse) {
  __shared__ int mark[kMaxStates];
  __shared__ int uidx[kMaxStates];
  __shared__ double2 fcol[kMaxElec];
  __shared__ double red[kHopAdjThreads];
  __shared__ int redi[kHopAdjThreads];
  __shared__ double qb[kMaxStates], lb[kMaxStates];
  __shared__ int sing;
  __shared__ int piv[kMaxElec];
  extern __shared__ double2 hop_smem[];
  const int t = blockIdx.x, tid = threadIdx.x;
  if (t >= live_slots(c)) return;
  const int n = c.md.n, n_pad = c.md.n_pad, N = c.md.N, nU = n - N;
  const double* C = Cs + (size_t)t * N * n_pad * 2;
  const double* lam = c.lam + (size_t)t * n_pad;
  const double* q0 = c.q0 + (size_t)t * n_pad;
  const int32_t* occ = c.occ + (size_t)t * N;
  const int g = c.gtraj[t];
  const double* pp = c.path + (size_t)g * c.path_len + s;
  const double v = (pp[0] - pp[-1]) / dt;
  const double omega = c.md.p[0], gg = c.md.p[1];
  const double hp = -c.md.mass * omega * omega * gg;
  double* base = scr + (size_t)t * hop_adj_scratch(n_pad, N);
  // X: [N][N] (S in, S^-1 out), in LDS when the launch gave it room
  double2* Mg = kLds ? hop_smem : reinterpret_cast<double2*>(base);
  double2* Wg = reinterpret_cast<double2*>(base + 2 * N * N);  // [nU][N]
  double2* Gu = Wg + (size_t)n_pad * N;                        // [nU][N]
  double* Rg = reinterpret_cast<double*>(Gu + (size_t)n_pad * N);  // [nU][N]
  double* Db = Rg + (size_t)n_pad * N;                         // [nU][N]

  for (int a = tid; a < n; a += kHopAdjThreads) mark[a] = 0;
  if (tid == 0) sing = 0;
  __syncthreads();
  for (int r = tid; r < N; r += kHopAdjThreads) mark[occ[r]] = 1;
  __syncthreads();
  if (tid == 0) {
    int j = 0;
    for (int a = 0; a < n; ++a)
      if (!mark[a]) uidx[j++] = a;
  }
  // S[r][o] = C[o][occ[r]]
  for (int e = tid; e < N * N; e += kHopAdjThreads) {
    const int r = e / N, col = e - r * N;
    const size_t off = ((size_t)col * n_pad + occ[r]) * 2;
    Mg[e] = make_double2(C[off], C[off + 1]);
  }
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    // pivot: largest |M[r][k]|, r >= k, smallest r among equals
    double best = -1.0;
    int bi = N;
    for (int r = k + tid; r < N; r += kHopAdjThreads) {
      const double2 m = Mg[(size_t)r * N + k];
      const double mag = m.x * m.x + m.y * m.y;
      if (mag > best) {
        best = mag;
        bi = r;
      }
    }
    // wave reduction by lane swaps, then the four wave results in a fixed order
    for (int m = 32; m > 0; m >>= 1) {
      const double o = __shfl_xor(best, m);
      const int oi = __shfl_xor(bi, m);
      if (o > best || (o == best && oi < bi)) {
        best = o;
        bi = oi;
      }
    }
    if ((tid & 63) == 0) {
      red[tid >> 6] = best;
      redi[tid >> 6] = bi;
    }
    __syncthreads();
    best = red[0];
    bi = redi[0];
    for (int q = 1; q < kHopAdjThreads / 64; ++q)
      if (red[q] > best || (red[q] == best && redi[q] < bi)) {
        best = red[q];
        bi = redi[q];
      }
    const int p = bi;
    if (!(best > 0.0)) {
      if (tid == 0) sing = 1;
      break;  // uniform: every thread read the same reduction result
    }
    if (tid == 0) piv[k] = p;
    if (p != k) {
      for (int col = tid; col < N; col += kHopAdjThreads) {
        const double2 a = Mg[(size_t)k * N + col], b = Mg[(size_t)p * N + col];
        Mg[(size_t)k * N + col] = b;
        Mg[(size_t)p * N + col] = a;
      }
    }
    __syncthreads();
    for (int r = tid; r < N; r += kHopAdjThreads) fcol[r] = Mg[(size_t)r * N + k];
    __syncthreads();
    const double2 pv = fcol[k];
    const double den = pv.x * pv.x + pv.y * pv.y;
    const double ir = pv.x / den, ii = -pv.y / den;  // 1 / pivot
    // row k: M[k][j] / pivot for j != k, 1 / pivot at j = k
    for (int col = tid; col < N; col += kHopAdjThreads) {
      const double2 a = (col == k) ? make_double2(1.0, 0.0) : Mg[(size_t)k * N + col];
      Mg[(size_t)k * N + col] = make_double2(a.x * ir - a.y * ii, a.x * ii + a.y * ir);
    }
    __syncthreads();
    // other rows: M[r][j] -= f_r M[k][j] (j != k), M[r][k] = -f_r M[k][k]
    for (int e = tid; e < N * N; e += kHopAdjThreads) {
      const int r = e / N, col = e - r * N;
      if (r == k) continue;
      const double2 f = fcol[r], a = Mg[(size_t)k * N + col];
      double2 m = (col == k) ? make_double2(0.0, 0.0) : Mg[e];
      m.x -= f.x * a.x - f.y * a.y;
      m.y -= f.x * a.y + f.y * a.x;
      Mg[e] = m;
    }
    __syncthreads();
  }
  __syncthreads();
  // undo the row interchanges as column interchanges, last first
  if (!sing) {
    for (int k = N - 1; k >= 0; --k) {
      const int p = piv[k];
      if (p != k) {
        for (int r = tid; r < N; r += kHopAdjThreads) {
          const double2 a = Mg[(size_t)r * N + k], b = Mg[(size_t)r * N + p];
          Mg[(size_t)r * N + k] = b;
          Mg[(size_t)r * N + p] = a;
        }
      }
      __syncthreads();
    }
  }
  const bool singular = sing != 0;
  const double wt = reverse ? weights[g] : 1.0;
  const double sc = wt * cG / T;
  // W = C_U X (X[o][r] = M[o][r]), pair probabilities
  double gsum = 0.0;
  if (!singular) {
    for (int e = tid; e < nU * N; e += kHopAdjThreads) {
      const int r = e / nU, j = e - r * nU;  // element [r][j]: consecutive threads, consecutive b
      const int b = uidx[j], a = occ[r];
      double wr = 0.0, wi = 0.0;
      for (int o = 0; o < N; ++o) {
        const size_t off = ((size_t)o * n_pad + b) * 2;
        const double cr = C[off], ci = C[off + 1];
        const double2 x = Mg[(size_t)o * N + r];
        wr += cr * x.x - ci * x.y;
        wi += cr * x.y + ci * x.x;
      }
      const double D = hp * q0[b] * q0[a] / (lam[a] - lam[b]);
      const double y = -2.0 * dt * v * D * wr;
      if (reverse) {
        const bool on = y > 0.0;
        Wg[e] = make_double2(wr, wi);
        Rg[e] = on ? sc * (-2.0 * dt * v * D) : 0.0;
        Db[e] = on ? sc * (-2.0 * dt * v * wr) : 0.0;
      } else {
        gsum += fmax(y, 0.0);
      }
    }
  }
  if (!reverse) {
    red[tid] = gsum;
    __syncthreads();
    for (int st = kHopAdjThreads / 2; st > 0; st >>= 1) {
      if (tid < st) red[tid] += red[tid + st];
      __syncthreads();
    }
    if (tid == 0) loss[g] += sc * red[0];
    return;
  }
  double* hb = hopbar + (size_t)t * (2 * n_pad + 1);
  if (singular) {
    for (int a = tid; a < 2 * n_pad + 1; a += kHopAdjThreads) hb[a] = 0.0;
    return;
  }
  __syncthreads();
  // (q0, lambda, h') cotangents of the couplings D_ba, b unoccupied, a occupied
  double hpart = 0.0;
  for (int j = tid; j < nU; j += kHopAdjThreads) {
    const int b = uidx[j];
    double qs = 0.0, ls = 0.0;
    for (int r = 0; r < N; ++r) {
      const int a = occ[r];
      const double d = lam[a] - lam[b];
      const double db = Db[(size_t)r * nU + j];
      qs += db * hp * q0[a] / d;
      ls += db * hp * q0[b] * q0[a] / (d * d);  // dD_ba/dlambda_b = D_ba / d
      hpart += db * q0[b] * q0[a] / d;
    }
    qb[b] = qs;
    lb[b] = ls;
  }
  for (int r = tid; r < N; r += kHopAdjThreads) {
    const int a = occ[r];
    double qs = 0.0, ls = 0.0;
    for (int j = 0; j < nU; ++j) {
      const int b = uidx[j];
      const double d = lam[a] - lam[b];
      const double db = Db[(size_t)r * nU + j];
      qs += db * hp * q0[b] / d;
      ls -= db * hp * q0[b] * q0[a] / (d * d);  // dD_ba/dlambda_a = -D_ba / d
    }
    qb[a] = qs;
    lb[a] = ls;
  }
  red[tid] = hpart;
  __syncthreads();
  for (int st = kHopAdjThreads / 2; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  for (int a = tid; a < n_pad; a += kHopAdjThreads) {
    hb[a] = a < n ? qb[a] : 0.0;
    hb[n_pad + a] = a < n ? lb[a] : 0.0;
  }
  if (tid == 0) hb[2 * n_pad] = red[0];
  // Gbar_U[j][o] = sum_r R[j][r] conj(X[o][r]), stored [o][j]
  for (int e = tid; e < nU * N; e += kHopAdjThreads) {
    const int o = e / nU, j = e - o * nU;
    double gr = 0.0, gi = 0.0;
    for (int r = 0; r < N; ++r) {
      const double rv = Rg[(size_t)r * nU + j];
      const double2 x = Mg[(size_t)o * N + r];
      gr += rv * x.x;
      gi -= rv * x.y;
    }
    Gu[e] = make_double2(gr, gi);
  }
  __syncthreads();
  double* G = Gh + (size_t)t * N * n_pad * 2;
  for (int e = tid; e < nU * N; e += kHopAdjThreads) {
    const int o = e / nU, j = e - o * nU;
    const size_t off = ((size_t)o * n_pad + uidx[j]) * 2;
    G[off] += 0.5 * Gu[e].x;
    G[off + 1] += 0.5 * Gu[e].y;
  }
  // Gbar_S[r][o] = -sum_j conj(W[j][r]) Gbar_U[j][o]
  for (int e = tid; e < N * N; e += kHopAdjThreads) {
    const int r = e / N, o = e - r * N;
    double gr = 0.0, gi = 0.0;
    for (int j = 0; j < nU; ++j) {
      const double2 wv = Wg[(size_t)r * nU + j], gu = Gu[(size_t)o * nU + j];
      gr -= wv.x * gu.x + wv.y * gu.y;
      gi -= wv.x * gu.y - wv.y * gu.x;
    }
    const size_t off = ((size_t)o * n_pad + occ[r]) * 2;
    G[off] += 0.5 * gr;
    G[off + 1] += 0.5 * gi;
  }
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
  if (t >= live_slots(c)) return;
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

hipError_t launch_adj_loss(const ClassDev& c, double* loss, int s, int T, const AdjTerms& w,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_adj_loss, dim3(c.n_traj), dim3(kLossThreads), 0, st, c, loss, s, T, w);
  return hipGetLastError();
}

size_t adj_hop_scratch_elems(const ClassDev& c) {
  return (size_t)c.n_traj * hop_adj_scratch(c.md.n_pad, c.md.N);
}

hipError_t launch_adj_hop(const ClassDev& c, const double* Cs, double* Gh, double* scr,
                          const double* weights, double* loss, double* hopbar, int s, int T,
                          double dt, double cG, int reverse, hipStream_t st) {
  if (c.n_live < 1) return hipSuccess;
  const size_t lds = hop_adj_lds(c.md.N);
  if (lds == 0) {
    hipLaunchKernelGGL(k_adj_hop<false>, dim3(c.n_live), dim3(kHopAdjThreads), 0, st, c, Cs, Gh, scr,
                       weights, loss, hopbar, s, T, dt, cG, reverse);
    return hipGetLastError();
  }
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_adj_hop<true>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_adj_hop<true>, dim3(c.n_live), dim3(kHopAdjThreads), lds, st, c, Cs, Gh, scr,
                     weights, loss, hopbar, s, T, dt, cG, reverse);
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
