// Orbital propagation C <- exp(-i A dt) C with A = diag(lambda) - i B,
// B = v D (Sec. II.C, Eq. exponential_integrator; propagator frozen at the
// step midpoint).  A is Hermitian, so exp(-i A dt) is expanded in Chebyshev
// polynomials of the shifted and scaled operator At = (A - c)/r whose
// spectrum lies in [-1, 1] (Gershgorin bounds computed with B):
//   exp(-i A dt) = sum_k c_k T_k(At),  c_k = e^{-i c dt} (2 - delta_k0) (-i)^k J_k(r dt),
// summed with Clenshaw's backward recurrence
//   b_k = c_k X + 2 At b_{k+1} - b_{k+2},  result = c_0 X + At b_1 - b_2,
// which needs no running sum.
// The number of terms comes from a tail bound of the Bessel coefficients and
// reaches FP64 (or FP32) rounding.
//
// Each application of At is one real matrix product B [Re X | Im X] on the
// matrix cores plus diagonal terms:
//   (A X)_re = lambda X_re + B X_im,   (A X)_im = lambda X_im - B X_re.
//
// Work decomposition: one work-group (8 waves) per (trajectory, slab of
// orbitals).  A slab holds up to kMaxColTiles 16-column tiles; each tile
// carries 8 orbitals as [Re of 8 | Im of 8], so the real and imaginary part
// of an orbital sit in lanes l and l^8 of the same MFMA tile and meet through
// one lane swap.  b_{k+1} of the slab lives in LDS (B operand).  The
// accumulator row held by a lane differs between the FP64 (row lk + 4 r) and
// FP32 (row 4 lk + r) 16x16x4 matrix instructions.  The
// coupling matrix B is streamed from memory through a double-buffered LDS
// stage of two 4-column blocks (A operand), so every wave reads it from LDS.
// The output tiles (row tile, column tile) of the slab are dealt to the
// waves round-robin, which balances the four SIMDs for any tile count; each
// wave keeps b_{k+2}, its component of the input X and the product of its
// tiles in registers.  The number
// of tiles of a wave is a template parameter (wave-uniform dispatch), so the
// matrix-core chains carry no predication.  Work-group ids are mapped so
// that the slabs of one trajectory land on the same XCD and share B in L2.

#include "iesh_internal.hpp"

namespace iesh {
namespace {

constexpr int kPropWaves = 8;
constexpr int kPropThreads = kPropWaves * 64;
constexpr int kStageKB = 2;  // k-blocks (of 4 columns of B) per LDS stage
constexpr int kPre = (kStageKB * (kMaxStates / 16) * 64 + kPropThreads - 1) / kPropThreads;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct PropCfg;

template <>
struct PropCfg<double> {
  typedef v4d acc_t;
  static constexpr int kMaxColTiles = 3;
  static constexpr int kMaxPairs = 6;  // ceil(14 * 3 / 8)
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of accumulator element r held by lane group lk (measured on gfx950)
  __device__ static constexpr int out_row(int lk, int r) { return lk + 4 * r; }
  __device__ static inline double* C(const ClassDev& c) { return c.C64; }
  __device__ static inline const double* B(const ClassDev& c) { return c.Bt; }
};

template <>
struct PropCfg<float> {
  typedef v4f acc_t;
  static constexpr int kMaxColTiles = 5;
  static constexpr int kMaxPairs = 9;  // ceil(14 * 5 / 8)
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int out_row(int lk, int r) { return 4 * lk + r; }
  __device__ static inline float* C(const ClassDev& c) { return c.C32; }
  __device__ static inline const float* B(const ClassDev& c) { return c.Bt32; }
};

// Geometry of one work-group's slab, shared by all waves.
template <typename T>
struct Slab {
  T* X;         // LDS [n_pad][ldx]: b_{k+1}, finally the result
  T* lam;       // LDS [n_pad]: lambda - c
  T* stage;     // LDS 2 x [kStageKB][RT][64]
  const T* Bt;  // memory [KB][RT][64]
  const T* Cg;  // memory [N][n_pad] complex: the input orbitals
  const double* cb;
  int n_pad, N, RT, KB, ldx, tile0, nct, stage_elems, n_stages, K;
  T invr;
};

// The Clenshaw loop for a wave that owns NQ output tiles.
template <typename T, int NQ>
__device__ void clenshaw_tiles(const Slab<T>& s, int wave, int tid) {
  typedef PropCfg<T> Cfg;
  typedef typename Cfg::acc_t acc_t;
  constexpr int NQ1 = NQ > 0 ? NQ : 1;
  const int lane = tid & 63;
  const int lrow = lane & 15;  // output column within a tile / A row
  const int lk = lane >> 4;    // k index within a block / output row group
  const bool is_re = lrow < 8;
  int prow[NQ1], pcol[NQ1];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int p = wave + kPropWaves * q;
    prow[q] = p / s.nct;
    pcol[q] = p - prow[q] * s.nct;
  }
  acc_t Bq[NQ1];  // b_{k+2}
  acc_t Xq[NQ1];  // this lane's component of the input X
#pragma unroll
  for (int q = 0; q < NQ1; ++q) {
    Bq[q] = acc_t{0, 0, 0, 0};
    Xq[q] = acc_t{0, 0, 0, 0};
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int o = s.tile0 * 8 + pcol[q] * 8 + (lrow & 7);
    if (o < s.N) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        Xq[q][r] = s.Cg[((size_t)o * s.n_pad + prow[q] * 16 + Cfg::out_row(lk, r)) * 2 + (is_re ? 0 : 1)];
    }
  }

  for (int k = s.K - 1; k >= 0; --k) {
    acc_t Y[NQ1];
#pragma unroll
    for (int q = 0; q < NQ1; ++q) Y[q] = acc_t{0, 0, 0, 0};

    // Y = B b_{k+1}, B streamed through two LDS stages
    for (int e = tid; e < s.stage_elems; e += kPropThreads)
      s.stage[e] = (e / (s.RT * 64) < s.KB) ? s.Bt[e] : (T)0;
    __syncthreads();
    for (int st = 0; st < s.n_stages; ++st) {
      T pre[kPre];
      const bool more = st + 1 < s.n_stages;
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        const int e = tid + u * kPropThreads;
        const int kb_abs = (st + 1) * kStageKB + e / (s.RT * 64);
        pre[u] = (more && e < s.stage_elems && kb_abs < s.KB)
                     ? s.Bt[(size_t)(st + 1) * s.stage_elems + e]
                     : (T)0;
      }
      const T* sb = s.stage + (st & 1) * s.stage_elems;
#pragma unroll
      for (int kk = 0; kk < kStageKB; ++kk) {
        const int kb = st * kStageKB + kk;
        if (kb < s.KB) {  // uniform
          const T* xrow = s.X + (kb * 4 + lk) * s.ldx + lrow;
          const T* arow = sb + kk * s.RT * 64 + lane;
#pragma unroll
          for (int q = 0; q < NQ; ++q) Y[q] = Cfg::mma(arow[prow[q] << 6], xrow[pcol[q] * 16], Y[q]);
        }
      }
      if (more) {
        T* nb = s.stage + ((st + 1) & 1) * s.stage_elems;
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
          const int e = tid + u * kPropThreads;
          if (e < s.stage_elems) nb[e] = pre[u];
        }
      }
      __syncthreads();
    }

    // b_k = c_k X + 2 At b_{k+1} - b_{k+2}   (k >= 1)
    // out = c_0 X +   At b_1     - b_2       (k == 0)
    const T cr = (T)s.cb[CHEB_COEF + 2 * k], ci = (T)s.cb[CHEB_COEF + 2 * k + 1];
    const T scale = ((k == 0) ? (T)1 : (T)2) * s.invr;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = prow[q] * 16 + Cfg::out_row(lk, r);
        const T x = Xq[q][r];
        const T xp = __shfl_xor(x, 8);
        const T cx = is_re ? (cr * x - ci * xp) : (cr * x + ci * xp);
        const T b1 = s.X[row * s.ldx + pcol[q] * 16 + lrow];
        const T yp = __shfl_xor(Y[q][r], 8);
        const T atb = s.lam[row] * b1 + (is_re ? yp : -yp);
        Y[q][r] = cx + scale * atb - Bq[q][r];  // b_k, stored after the barrier
        Bq[q][r] = b1;
      }
    }
    __syncthreads();  // every wave has read b_{k+1}
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        s.X[(prow[q] * 16 + Cfg::out_row(lk, r)) * s.ldx + pcol[q] * 16 + lrow] = Y[q][r];
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kPropThreads) void k_prop(ClassDev c) {
  typedef PropCfg<T> Cfg;
  extern __shared__ unsigned char smem_raw[];

  // XCD-aware id mapping: blocks b, b+8, b+16, ... share an XCD.
  const int b = blockIdx.x;
  const int xcd = b & 7;
  const int local = b >> 3;
  const int slab = local % c.n_slabs;
  const int t = (local / c.n_slabs) * 8 + xcd;
  if (t >= c.n_traj) return;
  if (c.status[t] & kFreezeMask) return;

  const ModelDev& md = c.md;
  Slab<T> s;
  s.n_pad = md.n_pad;
  s.N = md.N;
  s.RT = s.n_pad >> 4;
  s.KB = s.n_pad >> 2;
  const int tiles_total = (s.N + 7) >> 3;
  const int base = tiles_total / c.n_slabs, rem = tiles_total % c.n_slabs;
  s.tile0 = slab * base + (slab < rem ? slab : rem);
  s.nct = base + (slab < rem ? 1 : 0);
  s.ldx = 16 * s.nct + 2;
  s.X = reinterpret_cast<T*>(smem_raw);
  s.lam = s.X + (size_t)s.n_pad * s.ldx;
  s.stage = s.lam + s.n_pad;
  s.stage_elems = kStageKB * s.RT * 64;
  s.n_stages = (s.KB + kStageKB - 1) / kStageKB;
  s.Bt = Cfg::B(c) + (size_t)t * s.n_pad * s.n_pad;
  T* Cg = Cfg::C(c) + (size_t)t * s.N * s.n_pad * 2;
  s.Cg = Cg;
  s.cb = c.cheb + (size_t)t * kChebStride;
  s.K = (int)s.cb[CHEB_K];
  s.invr = (T)s.cb[CHEB_INVR];
  const T cc = (T)s.cb[CHEB_C];

  const int tid = threadIdx.x;
  for (int i = tid; i < s.n_pad; i += kPropThreads)
    s.lam[i] = (T)c.lam_mid[(size_t)t * s.n_pad + i] - cc;

  // b_K = c_K X into LDS: X[i][lt*16 + (o&7)] = Re, X[i][lt*16 + 8 + (o&7)] = Im
  const int n_orb = s.nct * 8;
  {
    const T cr = (T)s.cb[CHEB_COEF + 2 * s.K], ci = (T)s.cb[CHEB_COEF + 2 * s.K + 1];
    for (int idx = tid; idx < n_orb * s.n_pad; idx += kPropThreads) {
      const int ol = idx / s.n_pad, i = idx - ol * s.n_pad;
      const int o = s.tile0 * 8 + ol;
      T re = 0, im = 0;
      if (o < s.N) {
        re = Cg[((size_t)o * s.n_pad + i) * 2];
        im = Cg[((size_t)o * s.n_pad + i) * 2 + 1];
      }
      const int col = (ol >> 3) * 16 + (ol & 7);
      s.X[i * s.ldx + col] = cr * re - ci * im;
      s.X[i * s.ldx + col + 8] = cr * im + ci * re;
    }
  }
  __syncthreads();

  // tiles p = wave + 8 q, q < nq; dispatch on the (wave-uniform) count
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int P = s.RT * s.nct;
  const int nq = (P > wave) ? (P - wave + kPropWaves - 1) / kPropWaves : 0;
  switch (nq) {
    case 0: clenshaw_tiles<T, 0>(s, wave, tid); break;
    case 1: clenshaw_tiles<T, 1>(s, wave, tid); break;
    case 2: clenshaw_tiles<T, 2>(s, wave, tid); break;
    case 3: clenshaw_tiles<T, 3>(s, wave, tid); break;
    case 4: clenshaw_tiles<T, 4>(s, wave, tid); break;
    case 5: clenshaw_tiles<T, 5>(s, wave, tid); break;
    case 6: clenshaw_tiles<T, 6>(s, wave, tid); break;
    case 7: if constexpr (Cfg::kMaxPairs >= 7) clenshaw_tiles<T, 7>(s, wave, tid); break;
    case 8: if constexpr (Cfg::kMaxPairs >= 8) clenshaw_tiles<T, 8>(s, wave, tid); break;
    default: if constexpr (Cfg::kMaxPairs >= 9) clenshaw_tiles<T, 9>(s, wave, tid); break;
  }

  // result (in LDS) to memory, coalesced
  for (int idx = tid; idx < n_orb * s.n_pad; idx += kPropThreads) {
    const int ol = idx / s.n_pad, i = idx - ol * s.n_pad;
    const int o = s.tile0 * 8 + ol;
    if (o < s.N) {
      const int col = (ol >> 3) * 16 + (ol & 7);
      Cg[((size_t)o * s.n_pad + i) * 2] = s.X[i * s.ldx + col];
      Cg[((size_t)o * s.n_pad + i) * 2 + 1] = s.X[i * s.ldx + col + 8];
    }
  }
}

template <typename T>
size_t lds_bytes_t(const ClassDev& c) {
  const size_t n_pad = c.md.n_pad, RT = n_pad / 16;
  return sizeof(T) * (n_pad * (16 * c.nct_max + 2) + n_pad + 2 * kStageKB * RT * 64);
}

template <typename T>
hipError_t launch_prop_t(const ClassDev& c, dim3 grid, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_prop<T>, grid, dim3(kPropThreads), lds, s, c);
  return hipGetLastError();
}

}  // namespace

int prop_max_col_tiles(int precision) {
  return precision == IESH_FP64 ? PropCfg<double>::kMaxColTiles : PropCfg<float>::kMaxColTiles;
}

size_t prop_lds_bytes(const ClassDev& c, int precision) {
  return precision == IESH_FP64 ? lds_bytes_t<double>(c) : lds_bytes_t<float>(c);
}

// Allow the propagation kernels the LDS they need (above the 64 KB default).
hipError_t prop_prepare(const ClassDev& c, int precision) {
  const size_t lds = prop_lds_bytes(c, precision);
  if (lds <= 64 * 1024) return hipSuccess;
  const void* fn = (precision == IESH_FP64) ? (const void*)k_prop<double> : (const void*)k_prop<float>;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_prop(const ClassDev& c, int precision, hipStream_t s) {
  const int n_traj_pad = (c.n_traj + 7) / 8 * 8;
  const dim3 grid(n_traj_pad * c.n_slabs);
  const size_t lds = prop_lds_bytes(c, precision);
  if (precision == IESH_FP64) return launch_prop_t<double>(c, grid, lds, s);
  return launch_prop_t<float>(c, grid, lds, s);
}

}  // namespace iesh
