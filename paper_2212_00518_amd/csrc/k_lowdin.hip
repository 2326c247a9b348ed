// FP64 Loewdin re-orthonormalisation of FP32 orbitals (mixed precision).
//
// Propagation in FP32 lets the orbital overlap matrix C^H C drift away from
// the identity by rounding.  Every L steps the orbitals are replaced by
// their symmetric orthonormalisation C (C^H C)^{-1/2}, computed in FP64.
// With E = C^H C - I (of the order of the FP32 rounding accumulated over L
// steps), (I + E)^{-1/2} = I - E/2 + 3/8 E^2 + O(E^3), which is exact to FP64
// rounding for |E| ~ 1e-5.  The symmetric choice keeps each orbital as close
// as possible to its unorthonormalised self, so the correction does not
// bias any particular orbital.
//
// One work-group of 1024 threads per trajectory at a time (a persistent grid
// walks the trajectories).  Thread (ti, tj), tid = ti + 32 tj, accumulates
// rows ti + 32 ri and columns jb + tj + 32 cj (jb a group of 64 columns) of
// each product in registers; the
// operands are staged through LDS in chunks of 16 along the contracted index:
//   1. G = C^H C over chunks of 16 states, E = G - I to the work-group's
//      scratch;
//   2. E^2 over chunks of 16 rows of E (E is Hermitian, so a row chunk also
//      gives the column chunk), X = I - E/2 + 3/8 E^2 to scratch;
//   3. C X over chunks of 16 orbitals, for the states in passes of 128; a
//      pass is staged in scratch and written back (as FP32) after all its
//      reads of the old orbitals.

#include "iesh_internal.hpp"

namespace iesh {
namespace {

constexpr int kLowThreads = 1024;
constexpr int kPassSlots = 4;  // 32-state row slots per pass of the C X product

struct LowLds {
  double2 a[16][kMaxStates];  // chunk of 16 states (all orbitals) or 16 orbitals (all states)
  double2 b[16][kMaxElec];    // chunk of 16 rows of E or X
};

__device__ inline double2 cmad(double2 acc, double2 a, double2 b) {  // acc + a b
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}

__device__ inline double2 conj2(double2 a) { return make_double2(a.x, -a.y); }

template <int kRI>
__global__ __launch_bounds__(kLowThreads) void k_lowdin(ClassDev c, Counters* cnt,
                                                         int every, double2* scratch) {
  // 32-row slots covering the N orbitals; columns in groups of kCJ slots
  constexpr int kCJ = kRI < 2 ? kRI : 2;
  const int64_t step = cnt->step;     // step just completed
  if (every <= 0 || (step + 1) % every != 0) return;
  __shared__ LowLds L;
  __shared__ double defect_part[kLowThreads / 64];
  const int N = c.md.N, n_pad = c.md.n_pad, n = c.md.n;
  double2* E = scratch + (size_t)blockIdx.x * ((2 * (size_t)N + 32 * kPassSlots) * N);
  double2* X = E + (size_t)N * N;
  double2* Y = X + (size_t)N * N;  // [N][32 kPassSlots]: a state pass of the new orbitals
  const int tid = threadIdx.x, ti = tid & 31, tj = tid >> 5;

  for (int t = blockIdx.x; t < live_slots(c); t += gridDim.x) {
    if (c.status[t] & kFreezeMask) continue;  // uniform
    float2* C = reinterpret_cast<float2*>(c.C32) + (size_t)t * N * n_pad;  // C[j][s]

    // ---- 1. G[i][j] = sum_s conj(C[i][s]) C[j][s]; ||E||_F^2 on the way
    double e2 = 0.0;
    for (int jb = 0; jb < N; jb += 32 * kCJ) {
    double2 acc[kRI][kCJ];
#pragma unroll
    for (int ri = 0; ri < kRI; ++ri)
#pragma unroll
      for (int cj = 0; cj < kCJ; ++cj) acc[ri][cj] = make_double2(0.0, 0.0);
    for (int s0 = 0; s0 < n; s0 += 16) {
      __syncthreads();
      for (int e = tid; e < 16 * N; e += kLowThreads) {
        const int j = e >> 4, kk = e & 15;
        const int sidx = s0 + kk;
        const float2 z = (sidx < n) ? C[(size_t)j * n_pad + sidx] : make_float2(0.f, 0.f);
        L.a[kk][j] = make_double2((double)z.x, (double)z.y);
      }
      __syncthreads();
      const int nk = min(16, n - s0);
#pragma unroll 1
      for (int kk = 0; kk < nk; ++kk) {
        double2 ai[kRI], bj[kCJ];
#pragma unroll
        for (int ri = 0; ri < kRI; ++ri) ai[ri] = conj2(L.a[kk][ti + 32 * ri]);
#pragma unroll
        for (int cj = 0; cj < kCJ; ++cj) bj[cj] = L.a[kk][jb + tj + 32 * cj];
#pragma unroll
        for (int ri = 0; ri < kRI; ++ri)
#pragma unroll
          for (int cj = 0; cj < kCJ; ++cj) acc[ri][cj] = cmad(acc[ri][cj], ai[ri], bj[cj]);
      }
    }
#pragma unroll
    for (int ri = 0; ri < kRI; ++ri)
#pragma unroll
      for (int cj = 0; cj < kCJ; ++cj) {
        const int i = ti + 32 * ri, j = jb + tj + 32 * cj;
        if (i < N && j < N) {
          const double2 e = make_double2(acc[ri][cj].x - (i == j ? 1.0 : 0.0), acc[ri][cj].y);
          E[(size_t)i * N + j] = e;
          e2 += e.x * e.x + e.y * e.y;
        }
      }
    }
    // the defect this period left, before the correction: it sets the no-hop
    // bound's allowance for the next period; a defect above the allowance of
    // the period just ended is counted
    for (int m = 32; m > 0; m >>= 1) e2 += __shfl_xor(e2, m);
    if ((tid & 63) == 0) defect_part[tid >> 6] = e2;
    __syncthreads();  // E complete (block-scope visibility of the global writes)
    if (tid == 0) {
      double tot = 0.0;
      for (int w = 0; w < kLowThreads / 64; ++w) tot += defect_part[w];
      const double d = sqrt(tot);
      double* dp = c.defect + c.home[t];
      const double allowed = fmax(kDeltaMixed, kDefectSafety * *dp);
      if (d > allowed) atomicAdd((unsigned long long*)&cnt->defect_violations, 1ull);
      *dp = d;
      atomicMax((unsigned long long*)&cnt->defect_max_bits,
                (unsigned long long)__double_as_longlong(d));
    }

    // ---- 2. X = I - E/2 + 3/8 E^2, E^2[i][j] = sum_k conj(E[k][i]) E[k][j]
    for (int jb = 0; jb < N; jb += 32 * kCJ) {
    double2 acc[kRI][kCJ];
#pragma unroll
    for (int ri = 0; ri < kRI; ++ri)
#pragma unroll
      for (int cj = 0; cj < kCJ; ++cj) acc[ri][cj] = make_double2(0.0, 0.0);
    for (int k0 = 0; k0 < N; k0 += 16) {
      __syncthreads();
      for (int e = tid; e < 16 * N; e += kLowThreads) {
        const int kk = e / N, j = e - kk * N;
        L.b[kk][j] = (k0 + kk < N) ? E[(size_t)(k0 + kk) * N + j] : make_double2(0.0, 0.0);
      }
      __syncthreads();
      const int nk = min(16, N - k0);
#pragma unroll 1
      for (int kk = 0; kk < nk; ++kk) {
        double2 ai[kRI], bj[kCJ];
#pragma unroll
        for (int ri = 0; ri < kRI; ++ri) {
          const int i = ti + 32 * ri;
          ai[ri] = (i < N) ? conj2(L.b[kk][i]) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int cj = 0; cj < kCJ; ++cj) {
          const int j = jb + tj + 32 * cj;
          bj[cj] = (j < N) ? L.b[kk][j] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int ri = 0; ri < kRI; ++ri)
#pragma unroll
          for (int cj = 0; cj < kCJ; ++cj) acc[ri][cj] = cmad(acc[ri][cj], ai[ri], bj[cj]);
      }
    }
#pragma unroll
    for (int ri = 0; ri < kRI; ++ri)
#pragma unroll
      for (int cj = 0; cj < kCJ; ++cj) {
        const int i = ti + 32 * ri, j = jb + tj + 32 * cj;
        if (i < N && j < N) {
          const double2 e = E[(size_t)i * N + j];
          X[(size_t)i * N + j] = make_double2((i == j ? 1.0 : 0.0) - 0.5 * e.x + 0.375 * acc[ri][cj].x,
                                              -0.5 * e.y + 0.375 * acc[ri][cj].y);
        }
      }
    }
    __syncthreads();

    // ---- 3. C'[j][s] = sum_k C[k][s] X[k][j], states in passes of 32 kPassSlots
    // and column groups of 32 kCJ; a pass writes its states back only after
    // all its column groups have read them
    for (int p0 = 0; p0 < n; p0 += 32 * kPassSlots) {
      const int ns = min(32 * kPassSlots, n - p0);
      for (int jb = 0; jb < N; jb += 32 * kCJ) {
        double2 y[kPassSlots][kCJ];
#pragma unroll
        for (int rs = 0; rs < kPassSlots; ++rs)
#pragma unroll
          for (int cj = 0; cj < kCJ; ++cj) y[rs][cj] = make_double2(0.0, 0.0);
        for (int k0 = 0; k0 < N; k0 += 16) {
          __syncthreads();
          for (int e = tid; e < 16 * N; e += kLowThreads) {
            const int kk = e / N, j = e - kk * N;
            L.b[kk][j] = (k0 + kk < N) ? X[(size_t)(k0 + kk) * N + j] : make_double2(0.0, 0.0);
          }
          for (int e = tid; e < 16 * ns; e += kLowThreads) {
            const int kk = e / ns, sl = e - kk * ns;
            const float2 z = (k0 + kk < N) ? C[(size_t)(k0 + kk) * n_pad + p0 + sl] : make_float2(0.f, 0.f);
            L.a[kk][sl] = make_double2((double)z.x, (double)z.y);
          }
          __syncthreads();
          const int nk = min(16, N - k0);
#pragma unroll 1
          for (int kk = 0; kk < nk; ++kk) {
            double2 as[kPassSlots], bj[kCJ];
#pragma unroll
            for (int rs = 0; rs < kPassSlots; ++rs) {
              const int sl = ti + 32 * rs;
              as[rs] = (sl < ns) ? L.a[kk][sl] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int cj = 0; cj < kCJ; ++cj) {
              const int j = jb + tj + 32 * cj;
              bj[cj] = (j < N) ? L.b[kk][j] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int rs = 0; rs < kPassSlots; ++rs)
#pragma unroll
              for (int cj = 0; cj < kCJ; ++cj) y[rs][cj] = cmad(y[rs][cj], as[rs], bj[cj]);
          }
        }
        // results wait in the work-group's scratch until every column group
        // of the pass has read the old states
#pragma unroll
        for (int rs = 0; rs < kPassSlots; ++rs)
#pragma unroll
          for (int cj = 0; cj < kCJ; ++cj) {
            const int sl = ti + 32 * rs, j = jb + tj + 32 * cj;
            if (sl < ns && j < N) Y[(size_t)j * (32 * kPassSlots) + sl] = y[rs][cj];
          }
      }
      __syncthreads();  // every read of this pass's states is done
      for (int e = tid; e < N * ns; e += kLowThreads) {
        const int j = e / ns, sl = e - j * ns;
        const double2 v = Y[(size_t)j * (32 * kPassSlots) + sl];
        C[(size_t)j * n_pad + p0 + sl] = make_float2((float)v.x, (float)v.y);
      }
    }
    __syncthreads();
  }
}

}  // namespace

int lowdin_blocks(const ClassDev& c) { return c.n_traj < 512 ? c.n_traj : 512; }

size_t lowdin_scratch_elems(const ClassDev& c) {
  const size_t N = c.md.N;
  return (size_t)lowdin_blocks(c) * ((2 * N + 32 * kPassSlots) * N);
}

hipError_t launch_lowdin(const ClassDev& c, Counters* cnt, int every, double2* scratch,
                         hipStream_t s) {
  const int nb = lowdin_blocks(c);
  if (nb <= 0) return hipSuccess;
  const int ri = (c.md.N + 31) / 32;
  if (ri <= 1)
    hipLaunchKernelGGL(k_lowdin<1>, dim3(nb), dim3(kLowThreads), 0, s, c, cnt, every, scratch);
  else if (ri <= 2)
    hipLaunchKernelGGL(k_lowdin<2>, dim3(nb), dim3(kLowThreads), 0, s, c, cnt, every, scratch);
  else if (ri <= 3)
    hipLaunchKernelGGL(k_lowdin<3>, dim3(nb), dim3(kLowThreads), 0, s, c, cnt, every, scratch);
  else if (ri <= 4)
    hipLaunchKernelGGL(k_lowdin<4>, dim3(nb), dim3(kLowThreads), 0, s, c, cnt, every, scratch);
  else if (ri <= 5)
    hipLaunchKernelGGL(k_lowdin<5>, dim3(nb), dim3(kLowThreads), 0, s, c, cnt, every, scratch);
  else
    hipLaunchKernelGGL(k_lowdin<6>, dim3(nb), dim3(kLowThreads), 0, s, c, cnt, every, scratch);
  return hipGetLastError();
}

}  // namespace iesh
