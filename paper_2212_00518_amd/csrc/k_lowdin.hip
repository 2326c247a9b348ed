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
// Persistent grid: each work-group processes trajectories t = blockIdx.x +
// k * gridDim.x with scratch (E, X, Y) private to the work-group.

#include "iesh_internal.hpp"

namespace iesh {
namespace {

constexpr int kLowThreads = 256;

__global__ __launch_bounds__(kLowThreads) void k_lowdin(ClassDev c, const Counters* cnt,
                                                         int every, double2* scratch) {
  const int64_t step = cnt->step;  // step just completed
  if (every <= 0 || (step + 1) % every != 0) return;
  const int N = c.md.N, n_pad = c.md.n_pad, n = c.md.n;
  double2* E = scratch + (size_t)blockIdx.x * (2 * N * N + (size_t)N * n_pad);
  double2* X = E + (size_t)N * N;
  double2* Y = X + (size_t)N * N;
  const int tid = threadIdx.x;
  for (int t = blockIdx.x; t < c.n_traj; t += gridDim.x) {
    if (c.status[t] & kFreezeMask) continue;
    const float2* C = reinterpret_cast<const float2*>(c.C32) + (size_t)t * N * n_pad;
    // E = C^H C - I   (C[j][i] = coefficient of state i in orbital j)
    for (int idx = tid; idx < N * N; idx += kLowThreads) {
      const int i = idx / N, j = idx % N;
      double sr = 0.0, si = 0.0;
      for (int k = 0; k < n; ++k) {
        const float2 a = C[(size_t)i * n_pad + k], b = C[(size_t)j * n_pad + k];
        // conj(a) * b
        sr += (double)a.x * b.x + (double)a.y * b.y;
        si += (double)a.x * b.y - (double)a.y * b.x;
      }
      E[idx] = make_double2(sr - (i == j ? 1.0 : 0.0), si);
    }
    __syncthreads();
    // X = I - E/2 + 3/8 E^2
    for (int idx = tid; idx < N * N; idx += kLowThreads) {
      const int i = idx / N, j = idx % N;
      double sr = 0.0, si = 0.0;
      for (int k = 0; k < N; ++k) {
        const double2 a = E[(size_t)i * N + k], b = E[(size_t)k * N + j];
        sr += a.x * b.x - a.y * b.y;
        si += a.x * b.y + a.y * b.x;
      }
      const double2 e = E[idx];
      X[idx] = make_double2((i == j ? 1.0 : 0.0) - 0.5 * e.x + 0.375 * sr, -0.5 * e.y + 0.375 * si);
    }
    __syncthreads();
    // Y[j] = sum_k C[k] X[k][j]  (orbital j of the new set)
    for (int idx = tid; idx < N * n_pad; idx += kLowThreads) {
      const int j = idx / n_pad, i = idx % n_pad;
      double sr = 0.0, si = 0.0;
      if (i < n) {
        for (int k = 0; k < N; ++k) {
          const float2 a = C[(size_t)k * n_pad + i];
          const double2 b = X[(size_t)k * N + j];
          sr += (double)a.x * b.x - (double)a.y * b.y;
          si += (double)a.x * b.y + (double)a.y * b.x;
        }
      }
      Y[idx] = make_double2(sr, si);
    }
    __syncthreads();
    float2* Cw = reinterpret_cast<float2*>(c.C32) + (size_t)t * N * n_pad;
    for (int idx = tid; idx < N * n_pad; idx += kLowThreads) {
      const double2 y = Y[idx];
      Cw[idx] = make_float2((float)y.x, (float)y.y);
    }
    __syncthreads();
  }
}

}  // namespace

int lowdin_blocks(const ClassDev& c) { return c.n_traj < 512 ? c.n_traj : 512; }

size_t lowdin_scratch_elems(const ClassDev& c) {
  const size_t N = c.md.N, n_pad = c.md.n_pad;
  return (size_t)lowdin_blocks(c) * (2 * N * N + N * n_pad);
}

hipError_t launch_lowdin(const ClassDev& c, const Counters* cnt, int every, double2* scratch,
                         hipStream_t s) {
  const int nb = lowdin_blocks(c);
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lowdin, dim3(nb), dim3(kLowThreads), 0, s, c, cnt, every, scratch);
  return hipGetLastError();
}

}  // namespace iesh
