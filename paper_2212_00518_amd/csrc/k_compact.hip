// Compaction of frozen trajectories (exited, at the step cap, non-finite).
//
// Trajectories stop at different times (a scattering trajectory leaves once
// it has rebounded past the exit distance).  Every few hundred steps the live
// slots [0, live) of a class are permuted stably so that the active
// trajectories come first; the step kernels then visit only the leading
// active slots.  Per-trajectory state that outlives a step moves with the
// trajectory: position, velocity, force, status, global index, step count,
// step cap, home index (the slot it was uploaded to, which keys its
// observable records, its orthonormality defect and its warm-start basis),
// occupations and orbitals.  Everything else is recomputed at the start of
// the next step.  The hop uniforms are keyed by the global index, so a
// trajectory's dynamics do not depend on where it sits.
//
// The whole compaction runs on the device, four launches per class: rank
// (destinations and the active count), move (live slots to the spare
// arrays), back (spare arrays to the live slots), commit (the live count
// becomes the active count).  The live count is read from device memory by
// every kernel, so a captured graph replays compaction and steps with no
// host round trip and no re-capture.

#include <algorithm>

#include "iesh_internal.hpp"

namespace iesh {
namespace {

constexpr int kRankThreads = 1024;
constexpr int kMoveThreads = 256;

// dst[t] for t < n_live: active slots keep their order at the front, frozen
// ones follow in order.  n_active_out[0] = number of active slots.
__global__ __launch_bounds__(kRankThreads) void k_compact_rank(ClassDev c, int32_t* dst,
                                                                int32_t* n_active_out) {
  __shared__ int part[kRankThreads];
  const int tid = threadIdx.x, nl = live_slots(c);
  const int per = (nl + kRankThreads - 1) / kRankThreads;
  const int lo = min(nl, tid * per), hi = min(nl, lo + per);
  int mine = 0;
  for (int t = lo; t < hi; ++t) mine += (c.status[t] & kFreezeMask) ? 0 : 1;
  part[tid] = mine;
  __syncthreads();
  // inclusive scan of the per-thread counts (Hillis-Steele)
  for (int off = 1; off < kRankThreads; off <<= 1) {
    const int add = (tid >= off) ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += add;
    __syncthreads();
  }
  const int total = part[kRankThreads - 1];
  int before = part[tid] - mine;  // active slots before lo
  for (int t = lo; t < hi; ++t) {
    const bool active = !(c.status[t] & kFreezeMask);
    dst[t] = active ? before : total + (t - before);
    before += active ? 1 : 0;
  }
  if (tid == 0) n_active_out[0] = total;
}

template <typename CT>
__global__ __launch_bounds__(kMoveThreads) void k_compact_move(ClassDev c, const int32_t* dst,
                                                                CompactBufs b, const CT* C,
                                                                CT* Cs) {
  const int t = blockIdx.x;
  if (t >= live_slots(c)) return;
  const int d = dst[t];
  const int N = c.md.N, n_pad = c.md.n_pad, nd = c.md.ndof;
  if (threadIdx.x < nd) {
    const int nu = threadIdx.x;
    b.x[(size_t)d * nd + nu] = c.x[(size_t)t * nd + nu];
    b.v[(size_t)d * nd + nu] = c.v[(size_t)t * nd + nu];
    b.F[(size_t)d * nd + nu] = c.F[(size_t)t * nd + nu];
  }
  if (threadIdx.x == 0) {
    b.status[d] = c.status[t];
    b.gtraj[d] = c.gtraj[t];
    b.home[d] = c.home[t];
    b.nsteps[d] = c.nsteps[t];
    b.stepcap[d] = c.stepcap[t];
  }
  if (c.clock && threadIdx.x < 2) b.clock[2 * (size_t)d + threadIdx.x] = c.clock[2 * (size_t)t + threadIdx.x];
  for (int r = threadIdx.x; r < N; r += kMoveThreads) b.occ[(size_t)d * N + r] = c.occ[(size_t)t * N + r];
  const size_t len = (size_t)N * n_pad * 2;
  const CT* src = C + (size_t)t * len;
  CT* out = Cs + (size_t)d * len;
  for (size_t e = threadIdx.x; e < len; e += kMoveThreads) out[e] = src[e];
}

// Spare slot t back into live slot t (slots below the live count before the
// commit).
template <typename CT>
__global__ __launch_bounds__(kMoveThreads) void k_compact_back(ClassDev c, CompactBufs b, CT* C,
                                                                const CT* Cs) {
  const int t = blockIdx.x;
  if (t >= live_slots(c)) return;
  const int N = c.md.N, n_pad = c.md.n_pad, nd = c.md.ndof;
  if (threadIdx.x < nd) {
    const int nu = threadIdx.x;
    c.x[(size_t)t * nd + nu] = b.x[(size_t)t * nd + nu];
    c.v[(size_t)t * nd + nu] = b.v[(size_t)t * nd + nu];
    c.F[(size_t)t * nd + nu] = b.F[(size_t)t * nd + nu];
  }
  if (threadIdx.x == 0) {
    c.status[t] = b.status[t];
    c.gtraj[t] = b.gtraj[t];
    c.home[t] = b.home[t];
    c.nsteps[t] = b.nsteps[t];
    c.stepcap[t] = b.stepcap[t];
  }
  if (c.clock && threadIdx.x < 2) c.clock[2 * (size_t)t + threadIdx.x] = b.clock[2 * (size_t)t + threadIdx.x];
  for (int r = threadIdx.x; r < N; r += kMoveThreads) c.occ[(size_t)t * N + r] = b.occ[(size_t)t * N + r];
  const size_t len = (size_t)N * n_pad * 2;
  const CT* src = Cs + (size_t)t * len;
  CT* out = C + (size_t)t * len;
  for (size_t e = threadIdx.x; e < len; e += kMoveThreads) out[e] = src[e];
}

__global__ void k_compact_commit(ClassDev c, const int32_t* n_active) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c.live = *n_active;
}

__global__ __launch_bounds__(256) void k_fill(double* p, size_t count, double value) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (size_t)gridDim.x * 256)
    p[e] = value;
}

}  // namespace

hipError_t launch_fill(double* p, size_t count, double value, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

hipError_t launch_compact_rank(const ClassDev& c, int32_t* dst, int32_t* n_active, hipStream_t s) {
  hipLaunchKernelGGL(k_compact_rank, dim3(1), dim3(kRankThreads), 0, s, c, dst, n_active);
  return hipGetLastError();
}

hipError_t launch_compact_move(const ClassDev& c, const int32_t* dst, const CompactBufs& b,
                               int precision, hipStream_t s) {
  if (c.n_live < 1) return hipSuccess;
  if (precision == IESH_FP64)
    hipLaunchKernelGGL(k_compact_move<double>, dim3(c.n_live), dim3(kMoveThreads), 0, s, c, dst, b,
                       (const double*)c.C64, (double*)b.C);
  else
    hipLaunchKernelGGL(k_compact_move<float>, dim3(c.n_live), dim3(kMoveThreads), 0, s, c, dst, b,
                       (const float*)c.C32, (float*)b.C);
  return hipGetLastError();
}

// The device-side compaction of one class (c.live must be set): rank, move,
// back, commit.
hipError_t launch_compact(const ClassDev& c, const CompactBufs& b, int precision, hipStream_t s) {
  if (c.n_live < 1 || !b.dst || !c.live) return hipSuccess;
  hipError_t e = launch_compact_rank(c, b.dst, b.n_active, s);
  if (e == hipSuccess) e = launch_compact_move(c, b.dst, b, precision, s);
  if (e != hipSuccess) return e;
  if (precision == IESH_FP64)
    hipLaunchKernelGGL(k_compact_back<double>, dim3(c.n_live), dim3(kMoveThreads), 0, s, c, b, c.C64,
                       (const double*)b.C);
  else
    hipLaunchKernelGGL(k_compact_back<float>, dim3(c.n_live), dim3(kMoveThreads), 0, s, c, b, c.C32,
                       (const float*)b.C);
  hipLaunchKernelGGL(k_compact_commit, dim3(1), dim3(64), 0, s, c, b.n_active);
  return hipGetLastError();
}

}  // namespace iesh
