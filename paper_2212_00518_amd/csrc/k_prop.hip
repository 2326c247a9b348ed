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
// FP32 (row 4 lk + r) 16x16x4 matrix instructions.  The output tiles (row
// tile, column tile) of the slab are split into contiguous row-major ranges,
// one per wave; each wave streams its own A-operand fragments of the
// coupling matrix B from memory through a buffer resource, kDepth k-blocks
// ahead in registers, and keeps its component of the input X and the product
// of its tiles in registers.  The number of tiles of a wave is a template
// parameter (wave-uniform dispatch), so the matrix-core chains carry no
// predication.  Work-group ids are mapped so that the slabs of one
// trajectory land on the same XCD and share B in L2.

#include "iesh_internal.hpp"

namespace iesh {
namespace {

constexpr int kPropWaves = 8;
constexpr int kPropThreads = kPropWaves * 64;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct PropCfg;

template <>
struct PropCfg<double> {
  typedef v4d acc_t;
  // k-blocks of A operands in flight per wave (the k-block count is a
  // multiple); two suffice for the 64-cycle FP64 products and keep the
  // widest register tier free of spills
  static constexpr int kDepth = 2;
  static constexpr int kMaxColTiles = 3;
  static constexpr int kMaxPairs = 6;  // output tiles per wave (the slab width is capped to fit)
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
  static constexpr int kDepth = 4;  // two-tile waves; wider ones use 2
  static constexpr int kMaxColTiles = 5;
  static constexpr int kMaxPairs = 9;  // output tiles per wave (the slab width is capped to fit)
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int out_row(int lk, int r) { return 4 * lk + r; }
  __device__ static inline float* C(const ClassDev& c) { return c.C32; }
  __device__ static inline const float* B(const ClassDev& c) { return c.Bt32; }
};

// One element per lane of an A-operand fragment through a buffer resource.
template <typename T>
__device__ inline T load_frag(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ inline double load_frag<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ inline float load_frag<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// Value of lane l ^ 8 (the other half of the real/imaginary pair): within a
// row of 16 lanes that is a rotation by 8, one DPP register move (row_ror:8)
// instead of a permute through the LDS crossbar.
__device__ inline float swap8(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x128, 0xf, 0xf, false));
}
__device__ inline double swap8(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, 0x128, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), 0x128, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Row stride (elements) of the LDS slab: 16 nct, plus 16 when nct is even, so
// the stride is 16 mod 32 elements.  The rows of one 16x16x4 B operand then
// start 32 (FP64) or 16 (FP32) four-byte words apart modulo 64 and a read
// serves its lanes from disjoint banks.
__host__ __device__ constexpr int slab_ld(int nct) { return 16 * nct + ((nct & 1) ? 0 : 16); }

// Geometry of one work-group's slab, shared by all waves.
template <typename T>
struct Slab {
  T* X0;        // LDS [n_pad][ldx]: b_j for even j, finally the result
  T* X1;        // LDS [n_pad][ldx]: b_j for odd j
  T* lam;       // LDS [n_pad]: lambda - c
  const T* Bt;  // memory [n_pad / 4][RT][64]; the first KB k-blocks enter the product
  const T* Cg;  // memory [N][n_pad] complex: the input orbitals
  const double* cb;
  T* tap;       // memory [K][N][n_pad] complex (tap modes), this trajectory
  int n_pad, N, RT, KB, ldx, tile0, nct, K;
  T invr;
};

// Kernel modes.  kPropagate: C <- sum_k c_k T_k(At) C (Clenshaw).  kClenshawTaps:
// the same, and b_k for k = K .. 1 is stored at tap[k - 1] (run on a cotangent
// with conjugated coefficients it gives the adjoint vectors of the series).
// kForwardTaps: the Chebyshev vectors t_k = T_k(At) C for k = 0 .. K-1 are
// stored at tap[k] and C is left unchanged.
enum PropMode { kPropagate = 0, kClenshawTaps = 1, kForwardTaps = 2 };

// Store the element of a lane's accumulator tile (orbital o, row) at tap[k].
template <typename T>
__device__ inline void tap_store(const Slab<T>& s, int k, int o, int row, bool is_re, T val) {
  if (o < s.N) s.tap[(((size_t)k * s.N + o) * s.n_pad + row) * 2 + (is_re ? 0 : 1)] = val;
}

// The Clenshaw loop for a wave that owns NQ output tiles: the contiguous
// range [t0, t0 + NQ) of the slab's tiles in row-major order, so
// consecutive tiles mostly share their row tile of B (repeated fragment
// loads of a wave hit the L1 cache).  Each wave streams its A operands
// (fragments of B) from memory itself, kDepth k-blocks ahead.  The k-block
// loop has no barriers; b_{k+1} is read from LDS.
template <typename T, int NQ, int kMode>
__device__ void clenshaw_tiles(const Slab<T>& s, int t0, int tid) {
  typedef PropCfg<T> Cfg;
  typedef typename Cfg::acc_t acc_t;
  constexpr int NQ1 = NQ > 0 ? NQ : 1;
  // ring depth: the deeper FP32 ring only where its registers cost no occupancy
  constexpr int kDepth = (NQ <= 2) ? Cfg::kDepth : 2;
  const int lane = tid & 63;
  const int lrow = lane & 15;  // output column within a tile / A row
  const int lk = lane >> 4;    // k index within a block / output row group
  const bool is_re = lrow < 8;
  int prow[NQ1], pcol[NQ1];
#pragma unroll
  for (int q = 0; q < NQ1; ++q) {
    const int p = t0 + q;
    prow[q] = p / s.nct;
    pcol[q] = p - prow[q] * s.nct;
  }
  acc_t Xq[NQ1];  // this lane's component of the input X
#pragma unroll
  for (int q = 0; q < NQ1; ++q) Xq[q] = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int o = s.tile0 * 8 + pcol[q] * 8 + (lrow & 7);
    if (o < s.N) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        Xq[q][r] = s.Cg[((size_t)o * s.n_pad + prow[q] * 16 + Cfg::out_row(lk, r)) * 2 + (is_re ? 0 : 1)];
    }
  }
  // A operands through a buffer resource over this trajectory's B: the
  // per-tile offset (lane and row tile) is a register fixed for the whole
  // loop, the k-block offset is one scalar shared by the wave's tiles.
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)s.Bt, (short)0, (int)(sizeof(T) * s.n_pad * s.n_pad), 0x00020000);
  const unsigned kb_bytes = s.RT * 64 * sizeof(T);
  unsigned voff[NQ1];
#pragma unroll
  for (int q = 0; q < NQ1; ++q) voff[q] = (unsigned)(lane + prow[q] * 64) * sizeof(T);

  // Y = B b_{k+1}: A fragments from memory through a ring of kDepth k-blocks
  // in registers.  B is the same in every term, so the ring wraps around: the
  // loads issued during the last k-blocks of a term fetch the first k-blocks
  // of the next, and no term starts or ends waiting for memory.
  T a[kDepth][NQ1];
  // issue order = order of use, so the waits at the loop head stay partial
#pragma unroll
  for (int d = 0; d < kDepth; ++d)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      a[d][q] = load_frag<T>(rsrc, voff[q], d * kb_bytes);
      __builtin_amdgcn_sched_barrier(0);
    }
  const unsigned atotal = (unsigned)s.KB * kb_bytes;
  unsigned aoff = (kDepth * kb_bytes) % atotal;

  // Clenshaw: k = K-1 .. 0 produces b_k.  Forward recurrence: k = K-1 .. 1
  // produces t_{K-k} (the loop index only sets the buffer parity).
  const int k_end = (kMode == kForwardTaps) ? 1 : 0;
  for (int k = s.K - 1; k >= k_end; --k) {
    acc_t Y[NQ1];
#pragma unroll
    for (int q = 0; q < NQ1; ++q) Y[q] = acc_t{0, 0, 0, 0};

    const T* b1buf = (k & 1) ? s.X0 : s.X1;
    T* b2buf = (k & 1) ? s.X1 : s.X0;  // holds b_{k+2}, receives b_k

    // B operands from LDS one k-block ahead; the index past the last k-block
    // is clamped (a harmless reread), so the loop body has no branches.
    T xv[2][NQ1];
#pragma unroll
    for (int q = 0; q < NQ; ++q) xv[0][q] = b1buf[lk * s.ldx + pcol[q] * 16 + lrow];
    // B operands likewise: a per-tile LDS address plus a scalar k-block
    // offset, one block ahead of the loop index.
    const T* xq[NQ1];
#pragma unroll
    for (int q = 0; q < NQ1; ++q) xq[q] = b1buf + lk * s.ldx + pcol[q] * 16 + lrow;
    const unsigned xstep = 4u * s.ldx * sizeof(T), xlast = (unsigned)(s.KB - 1) * xstep;
    unsigned xoff = min(xstep, xlast);
    for (int kb0 = 0; kb0 < s.KB; kb0 += kDepth) {
#pragma unroll
      for (int d = 0; d < kDepth; ++d) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          xv[(d + 1) & 1][q] = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(xq[q]) + xoff);
        xoff = min(xoff + xstep, xlast);
        // the scheduling barriers keep the LDS reads of block kb + 1 ahead of
        // the products of block kb (left alone, the scheduler sinks them to
        // their use and each block waits a full LDS round trip)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) Y[q] = Cfg::mma(a[d][q], xv[d & 1][q], Y[q]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) a[d][q] = load_frag<T>(rsrc, voff[q], aoff);
        aoff = (aoff + kb_bytes == atotal) ? 0u : aoff + kb_bytes;
      }
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
        const T xp = swap8(x);
        const T cx = is_re ? (cr * x - ci * xp) : (cr * x + ci * xp);
        const int e = row * s.ldx + pcol[q] * 16 + lrow;
        const T b1 = b1buf[e];
        const T yp = swap8(Y[q][r]);
        const T atb = s.lam[row] * b1 + (is_re ? yp : -yp);
        if (kMode == kForwardTaps) {
          // t_{j+1} = 2 At t_j - t_{j-1} (t_1 = At t_0) replaces t_{j-1}
          const int j = s.K - 1 - k;
          const T tn = ((j == 0) ? s.invr : (T)2 * s.invr) * atb - b2buf[e];
          b2buf[e] = tn;
          tap_store(s, j + 1, s.tile0 * 8 + pcol[q] * 8 + (lrow & 7), row, is_re, tn);
        } else {
          // b_k replaces b_{k+2}: the element belongs to this lane alone
          const T bk = cx + scale * atb - b2buf[e];
          b2buf[e] = bk;
          if (kMode == kClenshawTaps && k >= 1)
            tap_store(s, k - 1, s.tile0 * 8 + pcol[q] * 8 + (lrow & 7), row, is_re, bk);
        }
      }
    }
    // b_k complete before anyone reads it; b_{k+1} free to be overwritten
    __syncthreads();
  }
}

// kQ: the most output tiles any wave of the launch owns.  Instantiated for a
// few tiers so that narrow slabs get a kernel with fewer registers (more
// work-groups per CU).
template <typename T, int kMode, int kQ>
__device__ void prop_item(const ClassDev& c, T* taps, int tap_k, int b, unsigned char* smem_raw) {
  typedef PropCfg<T> Cfg;

  // XCD-aware id mapping: blocks b, b+8, b+16, ... share an XCD.
  const int xcd = b & 7;
  const int local = b >> 3;
  const int slab = local % c.n_slabs;
  const int t = (local / c.n_slabs) * 8 + xcd;
  if (t >= live_slots(c)) return;
  if (c.status[t] & kFreezeMask) return;

  const ModelDev& md = c.md;
  Slab<T> s;
  s.n_pad = md.n_pad;
  s.N = md.N;
  s.RT = s.n_pad >> 4;
  // k-blocks of the product: rows past n of B and of the slab are zero, so
  // the sum stops at ceil(n / 4) blocks, rounded up to the prefetch ring
  s.KB = ((((md.n + 3) >> 2) + Cfg::kDepth - 1) / Cfg::kDepth) * Cfg::kDepth;
  const int tiles_total = (s.N + 7) >> 3;
  const int base = tiles_total / c.n_slabs, rem = tiles_total % c.n_slabs;
  s.tile0 = slab * base + (slab < rem ? slab : rem);
  s.nct = base + (slab < rem ? 1 : 0);
  s.ldx = slab_ld(s.nct);
  s.X0 = reinterpret_cast<T*>(smem_raw);
  s.X1 = s.X0 + (size_t)s.n_pad * s.ldx;
  s.lam = s.X1 + (size_t)s.n_pad * s.ldx;
  s.Bt = Cfg::B(c) + (size_t)t * s.n_pad * s.n_pad;
  T* Cg = Cfg::C(c) + (size_t)t * s.N * s.n_pad * 2;
  s.Cg = Cg;
  s.cb = c.cheb + (size_t)t * kChebStride;
  s.K = (int)s.cb[CHEB_K];
  s.invr = (T)s.cb[CHEB_INVR];
  s.tap = taps ? taps + (size_t)t * tap_k * s.N * s.n_pad * 2 : nullptr;
  const T cc = (T)s.cb[CHEB_C];

  const int tid = threadIdx.x;
  for (int i = tid; i < s.n_pad; i += kPropThreads)
    s.lam[i] = (T)c.lam_mid[(size_t)t * s.n_pad + i] - cc;

  // b_K = c_K X into the buffer of its parity: row i, column
  // lt*16 + (o&7) = Re, lt*16 + 8 + (o&7) = Im; b_{K+1} = 0 into the other
  const int n_orb = s.nct * 8;
  {
    T* bk = (s.K & 1) ? s.X1 : s.X0;
    T* bk1 = (s.K & 1) ? s.X0 : s.X1;
    for (int idx = tid; idx < s.n_pad * s.ldx; idx += kPropThreads) bk1[idx] = (T)0;
    // the forward recurrence starts from t_0 = X
    const T cr = (kMode == kForwardTaps) ? (T)1 : (T)s.cb[CHEB_COEF + 2 * s.K];
    const T ci = (kMode == kForwardTaps) ? (T)0 : (T)s.cb[CHEB_COEF + 2 * s.K + 1];
    for (int idx = tid; idx < n_orb * s.n_pad; idx += kPropThreads) {
      const int ol = idx / s.n_pad, i = idx - ol * s.n_pad;
      const int o = s.tile0 * 8 + ol;
      T re = 0, im = 0;
      if (o < s.N) {
        re = Cg[((size_t)o * s.n_pad + i) * 2];
        im = Cg[((size_t)o * s.n_pad + i) * 2 + 1];
      }
      const int col = (ol >> 3) * 16 + (ol & 7);
      const T vre = cr * re - ci * im, vim = cr * im + ci * re;
      bk[i * s.ldx + col] = vre;
      bk[i * s.ldx + col + 8] = vim;
      if (kMode != kPropagate) {
        const int kt = (kMode == kForwardTaps) ? 0 : s.K - 1;
        tap_store(s, kt, o, i, true, vre);
        tap_store(s, kt, o, i, false, vim);
      }
    }
  }
  __syncthreads();

  // tiles [t0, t0 + nq) of the P row-major tiles; dispatch on the
  // (wave-uniform) count
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int P = s.RT * s.nct;
  const int base_q = P / kPropWaves, rem_q = P % kPropWaves;
  const int nq = base_q + (wave < rem_q ? 1 : 0);
  const int t0 = wave * base_q + (wave < rem_q ? wave : rem_q);
  switch (nq) {
    case 0: clenshaw_tiles<T, 0, kMode>(s, t0, tid); break;
    case 1: clenshaw_tiles<T, 1, kMode>(s, t0, tid); break;
    case 2: clenshaw_tiles<T, 2, kMode>(s, t0, tid); break;
    case 3: if constexpr (kQ >= 3) clenshaw_tiles<T, 3, kMode>(s, t0, tid); break;
    case 4: if constexpr (kQ >= 4) clenshaw_tiles<T, 4, kMode>(s, t0, tid); break;
    case 5: if constexpr (kQ >= 5) clenshaw_tiles<T, 5, kMode>(s, t0, tid); break;
    case 6: if constexpr (kQ >= 6) clenshaw_tiles<T, 6, kMode>(s, t0, tid); break;
    case 7: if constexpr (kQ >= 7) clenshaw_tiles<T, 7, kMode>(s, t0, tid); break;
    case 8: if constexpr (kQ >= 8) clenshaw_tiles<T, 8, kMode>(s, t0, tid); break;
    default: if constexpr (kQ >= 9) clenshaw_tiles<T, 9, kMode>(s, t0, tid); break;
  }

  // result (in LDS) to memory, coalesced
  if (kMode == kForwardTaps) return;
  for (int idx = tid; idx < n_orb * s.n_pad; idx += kPropThreads) {
    const int ol = idx / s.n_pad, i = idx - ol * s.n_pad;
    const int o = s.tile0 * 8 + ol;
    if (o < s.N) {
      const int col = (ol >> 3) * 16 + (ol & 7);
      Cg[((size_t)o * s.n_pad + i) * 2] = s.X0[i * s.ldx + col];
      Cg[((size_t)o * s.n_pad + i) * 2 + 1] = s.X0[i * s.ldx + col + 8];
    }
  }
  // squared row norms over the slab's orbitals (of the stored values, summed
  // in FP64 in orbital order), so that the no-hop bound need not read C again
  if (kMode == kPropagate && c.rown) {
    double* rn = c.rown + ((size_t)t * ((s.N + 7) >> 3) + slab) * s.n_pad;
    for (int i = tid; i < s.n_pad; i += kPropThreads) {
      double acc = 0.0;
      for (int ol = 0; ol < n_orb && s.tile0 * 8 + ol < s.N; ++ol) {
        const int col = (ol >> 3) * 16 + (ol & 7);
        const double re = (double)s.X0[i * s.ldx + col], im = (double)s.X0[i * s.ldx + col + 8];
        acc = fma(re, re, acc);
        acc = fma(im, im, acc);
      }
      rn[i] = acc;
    }
  }
}

// One work-group per (trajectory, slab) item; items of slots past the live
// count (read from the device) end at once.
template <typename T, int kMode, int kQ>
__global__ __launch_bounds__(kPropThreads) void k_prop(ClassDev c, T* taps, int tap_k) {
  extern __shared__ unsigned char smem_raw[];
  prop_item<T, kMode, kQ>(c, taps, tap_k, blockIdx.x, smem_raw);
}

template <typename T>
size_t lds_bytes_t(const ClassDev& c) {
  const size_t n_pad = c.md.n_pad;
  int ld = 0;
  for (int nct = 1; nct <= c.nct_max; ++nct) ld = ld > slab_ld(nct) ? ld : slab_ld(nct);
  return sizeof(T) * (2 * n_pad * ld + n_pad);
}

// Register tiers of the kernel: the smallest tier that holds the launch's
// largest per-wave tile count is used.
template <typename T>
struct Tiers;
template <>
struct Tiers<double> {
  static constexpr int q[4] = {2, 3, 4, 6};
};
template <>
struct Tiers<float> {
  static constexpr int q[4] = {2, 3, 6, 9};
};

template <typename T, int kMode>
const void* prop_fn(int tier) {
  switch (tier) {
    case 0: return (const void*)k_prop<T, kMode, Tiers<T>::q[0]>;
    case 1: return (const void*)k_prop<T, kMode, Tiers<T>::q[1]>;
    case 2: return (const void*)k_prop<T, kMode, Tiers<T>::q[2]>;
    default: return (const void*)k_prop<T, kMode, Tiers<T>::q[3]>;
  }
}

template <typename T>
int prop_tier(const ClassDev& c) {
  const int q = ((c.md.n_pad / 16) * c.nct_max + kPropWaves - 1) / kPropWaves;
  int tier = 0;
  while (tier < 3 && Tiers<T>::q[tier] < q) ++tier;
  return tier;
}

template <typename T, int kMode>
hipError_t launch_prop_t(const ClassDev& c, dim3 grid, size_t lds, hipStream_t s, T* taps,
                         int tap_k) {
  switch (prop_tier<T>(c)) {
    case 0:
      hipLaunchKernelGGL((k_prop<T, kMode, Tiers<T>::q[0]>), grid, dim3(kPropThreads), lds, s, c, taps,
                         tap_k);
      break;
    case 1:
      hipLaunchKernelGGL((k_prop<T, kMode, Tiers<T>::q[1]>), grid, dim3(kPropThreads), lds, s, c, taps,
                         tap_k);
      break;
    case 2:
      hipLaunchKernelGGL((k_prop<T, kMode, Tiers<T>::q[2]>), grid, dim3(kPropThreads), lds, s, c, taps,
                         tap_k);
      break;
    default:
      hipLaunchKernelGGL((k_prop<T, kMode, Tiers<T>::q[3]>), grid, dim3(kPropThreads), lds, s, c, taps,
                         tap_k);
      break;
  }
  return hipGetLastError();
}

}  // namespace

int prop_max_col_tiles(int precision) {
  return precision == IESH_FP64 ? PropCfg<double>::kMaxColTiles : PropCfg<float>::kMaxColTiles;
}

int prop_max_tiles_per_wave(int precision) {
  return precision == IESH_FP64 ? PropCfg<double>::kMaxPairs : PropCfg<float>::kMaxPairs;
}

size_t prop_lds_bytes(const ClassDev& c, int precision) {
  return precision == IESH_FP64 ? lds_bytes_t<double>(c) : lds_bytes_t<float>(c);
}

// Allow the propagation kernels the LDS they need (above the 64 KB default).
hipError_t prop_prepare(const ClassDev& c, int precision) {
  const size_t lds = prop_lds_bytes(c, precision);
  if (lds <= 64 * 1024) return hipSuccess;
  for (int tier = 0; tier < 4; ++tier) {
    const void* fns[3] = {nullptr, nullptr, nullptr};
    if (precision == IESH_FP64) {
      fns[0] = prop_fn<double, kPropagate>(tier);
      fns[1] = prop_fn<double, kClenshawTaps>(tier);
      fns[2] = prop_fn<double, kForwardTaps>(tier);
    } else {
      fns[0] = prop_fn<float, kPropagate>(tier);
    }
    for (const void* fn : fns) {
      if (!fn) continue;
      const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_prop(const ClassDev& c, int precision, hipStream_t s) {
  if (c.n_live < 1) return hipSuccess;
  const int n_traj_pad = (c.n_live + 7) / 8 * 8;
  const dim3 grid(n_traj_pad * c.n_slabs);
  const size_t lds = prop_lds_bytes(c, precision);
  if (precision == IESH_FP64) return launch_prop_t<double, kPropagate>(c, grid, lds, s, nullptr, 0);
  return launch_prop_t<float, kPropagate>(c, grid, lds, s, nullptr, 0);
}

// FP64 tap modes for the adjoint: mode 1 stores the Clenshaw vectors b_K .. b_1
// of the series applied to c.C64, mode 2 the Chebyshev vectors t_0 .. t_{K-1}
// of c.C64 (left unchanged); taps: [trajectory][tap_k][N][n_pad] complex.
hipError_t launch_prop_taps(const ClassDev& c, int mode, double* taps, int tap_k, hipStream_t s) {
  if (c.n_live < 1) return hipSuccess;
  const int n_traj_pad = (c.n_live + 7) / 8 * 8;
  const dim3 grid(n_traj_pad * c.n_slabs);
  const size_t lds = prop_lds_bytes(c, IESH_FP64);
  if (mode == kClenshawTaps) return launch_prop_t<double, kClenshawTaps>(c, grid, lds, s, taps, tap_k);
  return launch_prop_t<double, kForwardTaps>(c, grid, lds, s, taps, tap_k);
}

}  // namespace iesh
