// Hop probabilities from determinant ratios, hop selection, rescaling,
// occupation update and observables (Sec. II.B, Eqs. hopping_probability and
// hopping_rate; the Slater-determinant overlaps <k|psi> = det S).
//
// For the occupied set s (sorted) the overlap matrix is S = C[s, :].  Moving
// one electron from orbital a (row r of S) to orbital b replaces row r of S
// by row b of C, and by the matrix determinant lemma
//     <j|psi> / <k|psi> = (C S^-1)[b][r] = W[b][r],
// so every hop probability follows from one inverse of S:
//     g(a -> b) = max(-2 dt v D[b][a] Re W[b][r], 0).
// The inverse comes from Gauss-Jordan elimination with column pivoting on S
// alone, done in place: processing row r of S picks the unused column p of
// largest modulus; afterwards the array X satisfies
//     X[q][c] = (S^-1)[perm[q]][perm^-1[c]],   perm[r] = pivot column of row r,
// so with Y = C_U[:, perm] X the ratios are W[b][r] = Y[b][perm[r]].  Only
// Re W enters g, so Y is accumulated as a real product over the 2N real and
// imaginary parts.
//
// One 512-thread work-group per trajectory that the exact no-hop bound could
// not settle, taken in order from a per-class queue filled by the bound
// kernel.  Thread (ti, tj), tid =
// ti + 16 tj, owns rows ti + 16 ri and columns tj + 32 cj of X and rows
// ti + 16 rb (positions in the unoccupied list) and columns tj + 32 cj of Y in
// registers (the slot counts are template parameters sized to the problem).
// A row of X and the pivot column are exchanged through LDS, and every wave
// chooses the pivot redundantly from the same LDS data.  Y is accumulated
// over chunks of 8 rows of X staged in LDS with the matching orbitals of C_U;
// when X and Y together would not fit in registers, X goes to the
// trajectory's scratch after the inversion and the chunks are read from there.

#include "iesh_internal.hpp"

namespace iesh {
namespace {

constexpr int kHopThreads = 512;
constexpr int kRowLanes = 16;  // threads along the rows

constexpr int kElecPad = (kMaxElec + 31) / 32 * 32;  // columns covered by the 32-wide slots

struct HopLds {
  double2 rowbuf[2][kElecPad];   // row r of X (pivot search and elimination factors)
  double2 colbuf[2][kElecPad];   // scaled pivot column of X
  double2 xs[8][kElecPad];       // chunk of 8 rows of X
  double2 cu[8][kMaxStates];     // C[u_bi][perm[q]] for the chunk's rows q
  double lam[kMaxStates];
  double q0[kMaxStates];
  double rowsum[kMaxElec];
  double grow[kMaxStates];       // g of the selected row, by unoccupied position
  double zz[kMaxElec];
  int occflag[kMaxStates];
  int uocc[kMaxStates];          // unoccupied states, ascending
  int perm[kMaxElec];
  int invperm[kMaxElec];
  int occ[kMaxElec];
  unsigned long long wkey[2][kHopThreads / 64];  // per-wave pivot keys, by row parity
  int singular;
  int sc_occ_changed;
  double sc_xi;
  double sc_v;
  double sc_ekin;
  double dofv[kMaxDof];  // velocity per coordinate (thread 0 of the hop)
  double dofd[kMaxDof];  // rescaling direction per coordinate
};

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Element i of orbital j of trajectory t, widened to FP64.
template <bool kF32>
__device__ inline double2 orb(const ClassDev& c, size_t base, int n_pad, int j, int i) {
  if (kF32) {
    const float2 f = reinterpret_cast<const float2*>(c.C32)[base + (size_t)j * n_pad + i];
    return make_double2((double)f.x, (double)f.y);
  }
  return reinterpret_cast<const double2*>(c.C64)[base + (size_t)j * n_pad + i];
}

// X and Y in registers together, or X through scratch for the product.
template <int kRS, int kRB>
constexpr bool x_via_scratch() {
  return 4 * kRS * ((kRS + 1) / 2) + 2 * kRB * ((kRS + 1) / 2) > 170;
}

// Everything the step needs for trajectory t (all threads of the work-group).
// kDense: couplings from the stored G = Q^T dH/dx Q of the dense model kind
// instead of the (lambda, q0) closed form.
template <bool kF32, int kRS, int kRB, bool kDense>
__device__ void hop_one(const ClassDev& c, int t, double dt_run, uint64_t seed, Counters* cnt,
                        iesh_event* events, int query_mode, int record, int exit_enabled,
                        double exit_x, int64_t max_steps, HopLds& L, double2* xscr) {
  const double dt = c.clock ? c.clock[2 * (size_t)t] : dt_run;  // this trajectory's step
  constexpr int kCS = (kRS + 1) / 2;  // 32-column slots covering 16 kRS columns
  constexpr bool kXS = x_via_scratch<kRS, kRB>();
  const int tid = threadIdx.x;
  const int ti = tid & 15, tj = tid >> 4;
  const int lane = tid & 63;
  const ModelDev& md = c.md;
  const int n = md.n, n_pad = md.n_pad, N = md.N, nU = n - N;
  if (!query_mode && (c.status[t] & kFreezeMask)) return;  // uniform
  const size_t base = (size_t)t * N * n_pad;
  if (!query_mode && tid == 0) atomicAdd((unsigned long long*)&cnt->hop_evals, 1ull);
  __syncthreads();  // the previous trajectory of this work-group is done with L

  for (int k = tid; k < n_pad; k += kHopThreads) {
    L.lam[k] = c.lam[(size_t)t * n_pad + k];
    L.q0[k] = c.q0[(size_t)t * n_pad + k];
    L.occflag[k] = 0;
  }
  if (tid == 0) L.singular = 0;
  __syncthreads();
  for (int r = tid; r < N; r += kHopThreads) {
    const int a = c.occ[(size_t)t * N + r];
    L.occ[r] = a;
    L.occflag[a] = 1;
  }
  __syncthreads();
  // unoccupied list: b sits at position b - #{occupied < b}
  for (int b = tid; b < n; b += kHopThreads) {
    if (L.occflag[b]) continue;
    int lo = 0, hi = N;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (L.occ[mid] < b)
        lo = mid + 1;
      else
        hi = mid;
    }
    L.uocc[b - lo] = b;
  }

  // ---- impurity amplitude of every orbital, sum_i q0_i C[i][j] (observable)
  if (record && !query_mode) {
    const int wv = tid >> 6;
    for (int j = wv; j < N; j += kHopThreads / 64) {
      double zr = 0.0, zi = 0.0;
      for (int i = lane; i < n_pad; i += 64) {
        const double2 z = orb<kF32>(c, base, n_pad, j, i);
        zr += L.q0[i] * z.x;
        zi += L.q0[i] * z.y;
      }
      for (int m = 32; m > 0; m >>= 1) {
        zr += __shfl_xor(zr, m);
        zi += __shfl_xor(zi, m);
      }
      if (lane == 0) L.zz[j] = zr * zr + zi * zi;
    }
  }

  // ---- S = C[s, :] into registers: x[ri][cj] = S[ti + 16 ri][tj + 32 cj]
  double2 x[kRS][kCS];
#pragma unroll
  for (int ri = 0; ri < kRS; ++ri) {
#pragma unroll
    for (int cj = 0; cj < kCS; ++cj) {
      const int i = ti + 16 * ri, j = tj + 32 * cj;
      x[ri][cj] = (i < N && j < N) ? orb<kF32>(c, base, n_pad, j, L.occ[i]) : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();

  // ---- in-place Gauss-Jordan inversion with column pivoting
  // The pivot of row r is the largest of keys that hold |X[r][j]|^2 in their
  // high bits (the bit pattern of a non-negative double orders like the
  // value) and 255 - j in the low 8 bits, so equal moduli go to the smallest
  // column; moduli within a relative 2^-44 of each other count as equal.
  // When the owners of row r publish it (right after their update of the
  // previous step) each wave reduces its owners' keys to one slot.
  static_assert(kMaxElec <= 256, "pivot keys hold 256 columns");
  constexpr int kWaves = kHopThreads / 64;
  unsigned used = 0u;  // bit cj: this thread's column tj + 32 cj has been a pivot
  auto publish_row = [&](int r) {
    const int ri0 = r >> 4, buf = r & 1;
    unsigned long long k = 0ull;
    if (ti == (r & 15)) {
      // one uniform branch per register row; the empty asm keeps the stores
      // in their branches (merged, they would need a run-time register index)
#pragma unroll
      for (int ri = 0; ri < kRS; ++ri) {
        if (ri == ri0) {
#pragma unroll
          for (int cj = 0; cj < kCS; ++cj) {
            const int j = tj + 32 * cj;
            if (j < N) {
              const double2 z = x[ri][cj];
              L.rowbuf[buf][j] = z;
              const double m = z.x * z.x + z.y * z.y;
              if (!((used >> cj) & 1u) && m > 0.0 && m < INFINITY) {
                const unsigned long long kj =
                    ((unsigned long long)__double_as_longlong(m) & ~0xFFull) | (unsigned long long)(255 - j);
                k = kj > k ? kj : k;
              }
            }
          }
          asm volatile("" ::: "memory");
        }
      }
    }
    // the owners of a wave are lanes l, l ^ 16, l ^ 32, l ^ 48
    unsigned long long o = __shfl_xor(k, 16);
    k = o > k ? o : k;
    o = __shfl_xor(k, 32);
    k = o > k ? o : k;
    if (lane == (r & 15)) L.wkey[buf][tid >> 6] = k;
  };
  // entries of the row and column buffers past N stay zero, so the update
  // needs no bounds selects
  for (int e = tid; e < 2 * kElecPad; e += kHopThreads) {
    L.rowbuf[e / kElecPad][e % kElecPad] = make_double2(0.0, 0.0);
    L.colbuf[e / kElecPad][e % kElecPad] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  publish_row(0);
  __syncthreads();
  for (int r = 0; r < N; ++r) {
    const int buf = r & 1;
    unsigned long long kr = 0ull;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const unsigned long long kw = L.wkey[buf][w];
      kr = kw > kr ? kw : kr;
    }
    // no finite nonzero candidate (singular S): the remaining steps are
    // no-ops; the decision is uniform
    const bool bad = (kr == 0ull);
    const int p = bad ? 0 : 255 - (int)(kr & 0xFFull);
    if (!bad && tj == (p & 31)) used |= 1u << (p >> 5);
    const double2 piv = L.rowbuf[buf][p];
    const double best = piv.x * piv.x + piv.y * piv.y;
    const double inv_m = bad ? 0.0 : 1.0 / best;
    const double2 pinv = make_double2(piv.x * inv_m, -piv.y * inv_m);  // 1 / piv
    if (tid == 0) {
      L.perm[r] = p;
      if (bad) L.singular = 1;
    }
    // owners of column p publish it scaled by 1/piv, with 1/piv in row r
    // (before row r is cleared below)
    if (!bad && tj == (p & 31)) {
      const int cj0 = p >> 5;
#pragma unroll
      for (int cj = 0; cj < kCS; ++cj) {
        if (cj == cj0) {
#pragma unroll
          for (int ri = 0; ri < kRS; ++ri) {
            const int ii = ti + 16 * ri;
            if (ii < N) L.colbuf[buf][ii] = (ii == r) ? pinv : cmul(x[ri][cj], pinv);
          }
          asm volatile("" ::: "memory");
        }
      }
    }
    // row r is cleared by its owners (the update then leaves -X[r][j] / piv
    // in it)
    if (!bad && ti == (r & 15)) {
      const int ri0 = r >> 4;
#pragma unroll
      for (int ri = 0; ri < kRS; ++ri)
        if (ri == ri0)
#pragma unroll
          for (int cj = 0; cj < kCS; ++cj) x[ri][cj] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    // every column j: X[:, j] -= X[r][j] * (published column); column p is
    // then replaced by the published column itself
    if (!bad) {  // uniform
      double2 rb[kCS];
#pragma unroll
      for (int cj = 0; cj < kCS; ++cj) rb[cj] = L.rowbuf[buf][tj + 32 * cj];
#pragma unroll
      for (int ri = 0; ri < kRS; ++ri) {
        const double2 cbv = L.colbuf[buf][ti + 16 * ri];
#pragma unroll
        for (int cj = 0; cj < kCS; ++cj) {
          x[ri][cj].x = fma(-rb[cj].x, cbv.x, x[ri][cj].x);
          x[ri][cj].x = fma(rb[cj].y, cbv.y, x[ri][cj].x);
          x[ri][cj].y = fma(-rb[cj].x, cbv.y, x[ri][cj].y);
          x[ri][cj].y = fma(-rb[cj].y, cbv.x, x[ri][cj].y);
        }
      }
    }
    if (!bad && tj == (p & 31)) {
      const int cj0 = p >> 5;
#pragma unroll
      for (int cj = 0; cj < kCS; ++cj) {
        if (cj == cj0) {
#pragma unroll
          for (int ri = 0; ri < kRS; ++ri) {
            const int ii = ti + 16 * ri;
            if (ii < N) x[ri][cj] = L.colbuf[buf][ii];
          }
        }
      }
    }
    if (r + 1 < N) publish_row(r + 1);
    __syncthreads();
  }
  __syncthreads();
  const bool singular = L.singular != 0;
  if (!singular) {
    for (int r = tid; r < N; r += kHopThreads) L.invperm[L.perm[r]] = r;
  }

  // ---- Y[bi][c] = Re sum_q C[u_bi][perm[q]] X[q][c], chunks of 8 rows q
  if (kXS) {
#pragma unroll
    for (int ri = 0; ri < kRS; ++ri)
#pragma unroll
      for (int cj = 0; cj < kCS; ++cj) {
        const int i = ti + 16 * ri, j = tj + 32 * cj;
        if (i < N && j < N) xscr[(size_t)i * N + j] = x[ri][cj];
      }
  }
  double y[kRB][kCS];
#pragma unroll
  for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
    for (int cj = 0; cj < kCS; ++cj) y[rb][cj] = 0.0;
#pragma unroll
  for (int ri = 0; ri < kRS; ++ri) {
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int q0 = 16 * ri + 8 * hh;
      if (q0 < N) {  // uniform
        __syncthreads();  // the previous chunk has been consumed (X in scratch is complete)
        if (kXS) {
          for (int e = tid; e < 8 * N; e += kHopThreads) {
            const int qq = e / N, j = e - qq * N;
            L.xs[qq][j] = (q0 + qq < N) ? xscr[(size_t)(q0 + qq) * N + j] : make_double2(0.0, 0.0);
          }
        } else if ((ti >> 3) == hh) {
#pragma unroll
          for (int cj = 0; cj < kCS; ++cj) {
            const int j = tj + 32 * cj;
            if (j < N) L.xs[ti & 7][j] = x[ri][cj];
          }
        }
        const int nq = min(8, N - q0);
        for (int e = tid; e < nq * nU; e += kHopThreads) {
          const int qq = e / nU, bi = e - qq * nU;
          L.cu[qq][bi] = orb<kF32>(c, base, n_pad, L.perm[q0 + qq], L.uocc[bi]);
        }
        __syncthreads();
        for (int qq = 0; qq < nq; ++qq) {
          double2 xv[kCS];
#pragma unroll
          for (int cj = 0; cj < kCS; ++cj) xv[cj] = L.xs[qq][tj + 32 * cj];
#pragma unroll
          for (int rb = 0; rb < kRB; ++rb) {
            const int bi = ti + 16 * rb;
            const double2 cv = (bi < nU) ? L.cu[qq][bi] : make_double2(0.0, 0.0);
#pragma unroll
            for (int cj = 0; cj < kCS; ++cj) y[rb][cj] += cv.x * xv[cj].x - cv.y * xv[cj].y;
          }
        }
      }
    }
  }
  __syncthreads();

  const double* geo = c.geo + (size_t)t * kGeoStride;
  const int nd = md.ndof;
  const double h = geo[GEO_H];
  // v.D from the coordinate gradients: with several coordinates the sums
  // v.grad h and v.grad f / f replace (dh, rho) and the velocity factor is 1
  const bool multi = nd > 1;
  const double dh = multi ? geo[GEO_VDH] : geo[GEO_DH];
  const double rho = multi ? geo[GEO_VRHO] : geo[GEO_RHO];
  const double v = multi ? 1.0 : c.v[(size_t)t * nd];
  // dense model kind: G = Q^T dH/dx Q from memory, and D = 0 between states
  // whose energies agree to 1e-12 of the largest |lambda|
  const double* Gd = kDense ? c.Gd + (size_t)t * n_pad * n_pad : nullptr;
  const double gtol = kDense ? 1e-12 * fmax(fabs(L.lam[0]), fabs(L.lam[n - 1])) : 0.0;
  auto coupling = [&](int b, int a) -> double {  // G[b][a]
    if constexpr (kDense) return fabs(L.lam[a] - L.lam[b]) <= gtol ? 0.0 : Gd[(size_t)b * n_pad + a];
    return L.q0[b] * L.q0[a] * (dh + rho * ((L.lam[b] - h) + (L.lam[a] - h)));
  };

  // ---- hop probabilities, formed on the fly from the owned elements of Y
  auto gval = [&](int rb, int cj) -> double {
    const int bi = ti + 16 * rb, j = tj + 32 * cj;
    if (singular || bi >= nU || j >= N) return 0.0;
    const int bb = L.uocc[bi];
    const int a = L.occ[L.invperm[j]];
    const double gab = coupling(bb, a);
    // v <b|d/dx a>.  A deflated state (no impurity part) gives gab = 0: an
    // exact 0 unless two deflated states share their energy (three or more
    // equal bath levels), where 0/0 is NaN and the fmax below (maxNum: the
    // non-NaN operand) returns 0.  No branch here: it costs registers.
    const double vD = v * gab / (L.lam[a] - L.lam[bb]);
    return fmax(-2.0 * dt * vD * y[rb][cj], 0.0);
  };

  if (query_mode) {
    double* go = c.gbuf + (size_t)t * N * n_pad;
    for (int e = tid; e < N * n_pad; e += kHopThreads) go[e] = 0.0;
    __syncthreads();
    if (!singular) {
#pragma unroll
      for (int rb = 0; rb < kRB; ++rb) {
#pragma unroll
        for (int cj = 0; cj < kCS; ++cj) {
          const int bi = ti + 16 * rb, j = tj + 32 * cj;
          if (bi < nU && j < N) go[(size_t)L.invperm[j] * n_pad + L.uocc[bi]] = gval(rb, cj);
        }
      }
    }
    if (singular && tid == 0) c.status[t] |= IESH_TRAJ_SINGULAR_S;
    return;
  }

  // ---- row totals (fixed-order reduction over the owned rows)
#pragma unroll
  for (int cj = 0; cj < kCS; ++cj) {
    double s = 0.0;
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb) s += gval(rb, cj);
    for (int m = kRowLanes / 2; m > 0; m >>= 1) s += __shfl_xor(s, m, kRowLanes);
    const int j = tj + 32 * cj;
    if (ti == 0 && j < N && !singular) L.rowsum[L.invperm[j]] = s;
  }
  __syncthreads();

  const int64_t step = cnt->step;
  __shared__ int sel_r;
  __shared__ double sel_prev, sel_margin, sel_total;
  if (tid == 0) {
    sel_r = -1;
    sel_margin = 1e300;
    sel_total = 0.0;
    if (!singular) {
      const double xi = philox_uniform(seed, (uint32_t)c.gtraj[t], (uint64_t)step, 0u);
      double cum = 0.0, margin = 1e300;
      for (int r = 0; r < N; ++r) {
        const double prev = cum;
        cum = cum + L.rowsum[r];
        margin = fmin(margin, fabs(cum - xi));
        if (sel_r < 0 && cum > xi) {
          sel_r = r;
          sel_prev = prev;
          break;
        }
      }
      double tot = 0.0;
      for (int r = 0; r < N; ++r) tot += L.rowsum[r];
      sel_total = tot;
      sel_margin = margin;
      L.sc_xi = xi;
    }
  }
  __syncthreads();
  const int rsel = sel_r;
  if (rsel >= 0) {
    const int csel = L.perm[rsel];
    if (tj == (csel & 31)) {
      const int cj0 = csel >> 5;
#pragma unroll
      for (int cj = 0; cj < kCS; ++cj) {
        if (cj == cj0) {
#pragma unroll
          for (int rb = 0; rb < kRB; ++rb) {
            const int bi = ti + 16 * rb;
            if (bi < nU) L.grow[bi] = gval(rb, cj);
          }
          asm volatile("" ::: "memory");
        }
      }
    }
  }
  __syncthreads();

  if (tid == 0) {
    double* vv = L.dofv;
    for (int nu = 0; nu < nd; ++nu) vv[nu] = c.v[(size_t)t * nd + nu];
    int32_t st = c.status[t];
    if (singular) st |= IESH_TRAJ_SINGULAR_S;
    int occ_changed = 0;
    if (rsel >= 0) {
      const double xi = L.sc_xi;
      double acc = sel_prev, margin = sel_margin;
      int bsel = -1;
      for (int bi = 0; bi < nU; ++bi) {  // b ascending over the unoccupied states
        const double g = L.grow[bi];
        if (g == 0.0) continue;
        acc = acc + g;
        margin = fmin(margin, fabs(acc - xi));
        if (acc > xi) {
          bsel = L.uocc[bi];
          break;
        }
      }
      if (bsel < 0) {
        for (int bi = nU - 1; bi >= 0; --bi)
          if (L.grow[bi] > 0.0) {
            bsel = L.uocc[bi];
            break;
          }
        margin = 0.0;
      }
      const int a = L.occ[rsel];
      // rescale along d_nu = <b|d/dR_nu a> (momentum change gamma d)
      double* dv = L.dofd;
      for (int nu = 0; nu < nd; ++nu) {
        const double dhn = geo[GEO_DHV + nu], rhon = geo[GEO_RHOV + nu];
        const double gba = kDense ? coupling(bsel, a)
                                  : L.q0[bsel] * L.q0[a] * (dhn + rhon * ((L.lam[bsel] - h) + (L.lam[a] - h)));
        dv[nu] = gba == 0.0 ? 0.0 : gba / (L.lam[a] - L.lam[bsel]);
      }
      const double dE = L.lam[bsel] - L.lam[a];
      double A2 = dv[0] * dv[0] / (2.0 * md.mass_dof[0]);
      double B1 = vv[0] * dv[0];
      for (int nu = 1; nu < nd; ++nu) {
        A2 += dv[nu] * dv[nu] / (2.0 * md.mass_dof[nu]);
        B1 += vv[nu] * dv[nu];
      }
      const double disc = B1 * B1 - 4.0 * A2 * dE;
      int accepted = 0;
      if (A2 != 0.0 && disc >= 0.0) {
        const double root = sqrt(disc);
        const double q = B1 + (B1 >= 0.0 ? root : -root);
        const double gamma = (q != 0.0) ? 2.0 * dE / q : 0.0;
        for (int nu = 0; nu < nd; ++nu) vv[nu] = vv[nu] - gamma * dv[nu] / md.mass_dof[nu];
        accepted = 1;
        // occupation update, keep sorted
        int* o = L.occ;
        o[rsel] = bsel;
        int r = rsel;
        while (r > 0 && o[r - 1] > o[r]) {
          const int tmp = o[r - 1];
          o[r - 1] = o[r];
          o[r] = tmp;
          --r;
        }
        while (r < N - 1 && o[r + 1] < o[r]) {
          const int tmp = o[r + 1];
          o[r + 1] = o[r];
          o[r] = tmp;
          ++r;
        }
        occ_changed = 1;
      }
      const int64_t slot = atomicAdd((unsigned long long*)&cnt->n_events, 1ull);
      if (slot < IESH_EVENT_CAP) {
        iesh_event* ev = events + slot;
        ev->step = step;
        ev->traj = c.gtraj[t];
        ev->a = a;
        ev->b = bsel;
        ev->accepted = accepted;
        ev->margin = margin;
        ev->g_total = sel_total;
      }
    }
    // force refresh for the (possibly new) occupations
    if (occ_changed) {
      for (int nu = 0; nu < nd; ++nu) {
        const double dhn = geo[GEO_DHV + nu], rhon = geo[GEO_RHOV + nu];
        double s = 0.0;
        for (int r = 0; r < N; ++r) {
          const int a = L.occ[r];
          s += kDense ? Gd[(size_t)a * n_pad + a] : L.q0[a] * L.q0[a] * (dhn + 2.0 * rhon * (L.lam[a] - h));
        }
        c.F[(size_t)t * nd + nu] = -geo[GEO_DU0V + nu] - s;
        c.v[(size_t)t * nd + nu] = vv[nu];
      }
    }
    const int64_t ns = c.nsteps[t] + 1;
    c.nsteps[t] = ns;
    const double x = c.x[(size_t)t * nd + c.exit_dof];
    if (exit_enabled && x > exit_x) st |= IESH_TRAJ_EXITED;
    if ((max_steps > 0 && ns >= max_steps) || (c.stepcap[t] > 0 && ns >= c.stepcap[t]))
      st |= IESH_TRAJ_STEPCAP;
    double ekin = 0.0;
    for (int nu = 0; nu < nd; ++nu) {
      if (!isfinite(vv[nu])) st |= IESH_TRAJ_NONFINITE;
      ekin += 0.5 * md.mass_dof[nu] * vv[nu] * vv[nu];
    }
    c.status[t] = st;
    if (c.clock) advance_clock(c, t, sel_total);
    L.sc_occ_changed = occ_changed;
    L.sc_ekin = ekin;
  }
  __syncthreads();
  if (L.sc_occ_changed) {
    for (int r = tid; r < N; r += kHopThreads) c.occ[(size_t)t * N + r] = L.occ[r];
  }
  if (record && tid == 0) {
    const int64_t rel = step - cnt->run_step0 + 1;
    if (cnt->record_every > 0 && rel % cnt->record_every == 0) {
      const int64_t rec = rel / cnt->record_every - 1;
      double pds = 0.0, elam = 0.0, pdw = 0.0;
      for (int r = 0; r < N; ++r) {
        const int a = L.occ[r];
        pds += L.q0[a] * L.q0[a];
        elam += L.lam[a];
        pdw += L.zz[r];
      }
      const double ekin = L.sc_ekin;
      const double epot = geo[GEO_U0] + elam;
      double* o = c.obs + ((size_t)rec * c.n_traj + c.home[t]) * IESH_N_OBS;
      o[IESH_OBS_PD_SURF] = pds;
      o[IESH_OBS_PD_WF] = pdw;
      o[IESH_OBS_EKIN] = ekin;
      o[IESH_OBS_EPOT] = epot;
      o[IESH_OBS_ETOT] = ekin + epot;
    }
  }
}


// Work-group b takes entries b, b + G, ... (G the grid) of the class queue
// hopq = [count, unused, done, list...] that the bound kernel fills; the
// last work-group to finish resets the queue for the next step.  In query
// mode work-group b handles trajectory t0 + b.
template <bool kF32, int kRS, int kRB, bool kDense>
__global__ __launch_bounds__(kHopThreads) void k_hop(ClassDev c, double dt, uint64_t seed,
                                                     Counters* cnt, iesh_event* events,
                                                     int query_mode, int t0, int record,
                                                     int exit_enabled, double exit_x,
                                                     int64_t max_steps) {
  __shared__ HopLds L;
  int32_t* q = c.hopq;
  const int b = blockIdx.x;
  // persistent: entries b, b + G, b + 2G, ... of the queue (G the grid)
  const int n_items = query_mode ? 1 : q[0];
  for (int e = query_mode ? 0 : b; e < n_items; e += gridDim.x) {
    const int t = query_mode ? t0 + b : q[3 + e];
    double2* xscr = x_via_scratch<kRS, kRB>() ? c.hopx + (size_t)t * c.md.N * c.md.N : nullptr;
    hop_one<kF32, kRS, kRB, kDense>(c, t, dt, seed, cnt, events, query_mode, record, exit_enabled,
                                    exit_x, max_steps, L, xscr);
  }
  if (!query_mode && threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&q[2], 1) == (int)gridDim.x - 1) {
      q[0] = 0;
      q[2] = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Exact hop filter.  For orbitals with orthonormal columns, S^H S =
// I - C_U^H C_U, so sigma_min(S)^2 >= 1 - ||C_U||_F^2 - delta, where delta
// bounds the orthonormality defect ||C^H C - I|| of the stored orbitals
// (FP64: a fixed 1e-8; mixed: the larger of 1e-3 and four times the defect
// the last Loewdin step measured before correcting, i.e. the growth over one
// Loewdin period; the mixed path without Loewdin steps never measures it and
// runs without the filter).  Row b of the ratios, W[b][:] = C_U[b, :] S^-1,
// has norm ||W[b][:]|| <= ||C_U[b, :]|| / sigma_min(S), and g <= 2 dt
// |v D[b][s_r]| |W[b][r]|, so by Cauchy-Schwarz over r the total hop
// probability of the step is bounded by
//   sum_{r, b} g <= 2 dt sum_b ||C_U[b, :]|| (sum_r |v D[b][s_r]|^2)^(1/2) / sigma_min(S).
// When that bound does not exceed the step's uniform xi, no pair can be
// selected and the step ends without a hop: the filter completes such
// trajectories (counters, exit checks, observables) and the determinant-ratio
// kernel runs only for the others.  No factorisation is needed for the bound:
// it costs one pass over C and one coupling per (occupied, unoccupied) pair.
constexpr int kFltThreads = 256;

struct FltLds {
  double lam[kMaxStates];
  double q0[kMaxStates];
  double rn[kMaxStates];  // ||C[b, :]||
  double red[kFltThreads];
  double red2[kFltThreads];
  double zz[kMaxElec];
  int occflag[kMaxStates];
  int occ[kMaxElec];
};

template <bool kF32, bool kDense>
__device__ void filter_one(const ClassDev& c, int t, double dt_run, uint64_t seed, Counters* cnt,
                           int record, int exit_enabled, double exit_x, int64_t max_steps,
                           double delta, FltLds& L) {
  const int tid = threadIdx.x;
  const ModelDev& md = c.md;
  const int n = md.n, n_pad = md.n_pad, N = md.N;
  if (t >= live_slots(c) || (c.status[t] & kFreezeMask)) return;
  const double dt = c.clock ? c.clock[2 * (size_t)t] : dt_run;  // this trajectory's step
  for (int k = tid; k < n_pad; k += kFltThreads) {
    L.lam[k] = c.lam[(size_t)t * n_pad + k];
    L.q0[k] = c.q0[(size_t)t * n_pad + k];
    L.occflag[k] = 0;
  }
  __syncthreads();
  for (int r = tid; r < N; r += kFltThreads) {
    const int a = c.occ[(size_t)t * N + r];
    L.occ[r] = a;
    L.occflag[a] = 1;
  }
  __syncthreads();
  // row norms of C (state b over all orbitals); ||C_U||_F^2 over unoccupied b
  const size_t base = (size_t)t * N * n_pad;
  double fro_part = 0.0;
  for (int b = tid; b < n_pad; b += kFltThreads) {
    double s2 = 0.0;
    for (int j = 0; j < N; ++j) {
      double re, im;
      if (kF32) {
        const float2 z = reinterpret_cast<const float2*>(c.C32)[base + (size_t)j * n_pad + b];
        re = z.x;
        im = z.y;
      } else {
        const double2 z = reinterpret_cast<const double2*>(c.C64)[base + (size_t)j * n_pad + b];
        re = z.x;
        im = z.y;
      }
      s2 += re * re + im * im;
    }
    L.rn[b] = sqrt(s2);
    if (b < n && !L.occflag[b]) fro_part += s2;
  }
  __syncthreads();
  // sum_b ||C_U[b]|| (sum_r |v D[b][s_r]|^2)^(1/2)
  const double* geo = c.geo + (size_t)t * kGeoStride;
  const int nd = md.ndof;
  const double h = geo[GEO_H];
  const bool multi = nd > 1;
  const double dh = multi ? geo[GEO_VDH] : geo[GEO_DH];
  const double rho = multi ? geo[GEO_VRHO] : geo[GEO_RHO];
  const double v = multi ? 1.0 : c.v[(size_t)t * nd];
  const double* Gd = kDense ? c.Gd + (size_t)t * n_pad * n_pad : nullptr;
  const double gtol = kDense ? 1e-12 * fmax(fabs(L.lam[0]), fabs(L.lam[n - 1])) : 0.0;
  double bnd_part = 0.0;
  for (int b = tid; b < n; b += kFltThreads) {
    if (L.occflag[b]) continue;
    double s = 0.0;
    for (int r = 0; r < N; ++r) {
      const int a = L.occ[r];
      const double gab = kDense ? (fabs(L.lam[a] - L.lam[b]) <= gtol ? 0.0 : Gd[(size_t)b * n_pad + a])
                                : L.q0[b] * L.q0[a] * (dh + rho * ((L.lam[b] - h) + (L.lam[a] - h)));
      if (gab != 0.0) {
        const double d = v * gab / (L.lam[a] - L.lam[b]);
        s = fma(d, d, s);
      }
    }
    bnd_part += L.rn[b] * sqrt(s);
  }
  L.red[tid] = fro_part;
  L.red2[tid] = bnd_part;
  __syncthreads();
  for (int st = kFltThreads / 2; st > 0; st >>= 1) {
    if (tid < st) {
      L.red[tid] += L.red[tid + st];
      L.red2[tid] += L.red2[tid + st];
    }
    __syncthreads();
  }
  const double fro2 = L.red[0], S1 = L.red2[0];
  const int64_t step = cnt->step;
  const double xi = philox_uniform(seed, (uint32_t)c.gtraj[t], (uint64_t)step, 0u);
  const double smin2 = 1.0 - fro2 - (c.defect ? fmax(delta, kDefectSafety * c.defect[c.home[t]]) : delta);
  // no hop when the bound on the total lies below the uniform; an adaptive
  // step also needs the bound to keep the next step at its largest (the
  // total, at most the bound, then selects dt0 exactly)
  const double bound = smin2 > 0.0 ? (1.0 + 1e-10) * 2.0 * dt * S1 / sqrt(smin2) : 0.0;
  const bool no_hop = !c.exact_hops && smin2 > 0.0 && bound <= xi &&
                      (c.dt_levels == 0 || bound * (c.dt0 / dt) <= c.gmax);
  __syncthreads();
  if (!no_hop) {
    if (tid == 0) c.hopq[3 + atomicAdd(&c.hopq[0], 1)] = t;
    return;
  }
  // impurity amplitude of every orbital (observable), one wave per orbital
  if (record) {
    const int lane = tid & 63, wv = tid >> 6;
    for (int j = wv; j < N; j += kFltThreads / 64) {
      double zr = 0.0, zi = 0.0;
      for (int i = lane; i < n_pad; i += 64) {
        double re, im;
        if (kF32) {
          const float2 z = reinterpret_cast<const float2*>(c.C32)[base + (size_t)j * n_pad + i];
          re = z.x;
          im = z.y;
        } else {
          const double2 z = reinterpret_cast<const double2*>(c.C64)[base + (size_t)j * n_pad + i];
          re = z.x;
          im = z.y;
        }
        zr += L.q0[i] * re;
        zi += L.q0[i] * im;
      }
      for (int m = 32; m > 0; m >>= 1) {
        zr += __shfl_xor(zr, m);
        zi += __shfl_xor(zi, m);
      }
      if (lane == 0) L.zz[j] = zr * zr + zi * zi;
    }
    __syncthreads();
  }
  if (tid == 0) {
    int32_t st = c.status[t];
    const int64_t ns = c.nsteps[t] + 1;
    c.nsteps[t] = ns;
    if (exit_enabled && c.x[(size_t)t * nd + c.exit_dof] > exit_x) st |= IESH_TRAJ_EXITED;
    if ((max_steps > 0 && ns >= max_steps) || (c.stepcap[t] > 0 && ns >= c.stepcap[t]))
      st |= IESH_TRAJ_STEPCAP;
    double ekin = 0.0;
    for (int nu = 0; nu < nd; ++nu) {
      const double vn = c.v[(size_t)t * nd + nu];
      if (!isfinite(vn)) st |= IESH_TRAJ_NONFINITE;
      ekin += 0.5 * md.mass_dof[nu] * vn * vn;
    }
    c.status[t] = st;
    if (c.clock) advance_clock(c, t, 0.0);  // the bound kept the step at dt0
    if (record) {
      const int64_t rel = step - cnt->run_step0 + 1;
      if (cnt->record_every > 0 && rel % cnt->record_every == 0) {
        const int64_t rec = rel / cnt->record_every - 1;
        double pds = 0.0, elam = 0.0, pdw = 0.0;
        for (int r = 0; r < N; ++r) {
          const int a = L.occ[r];
          pds += L.q0[a] * L.q0[a];
          elam += L.lam[a];
          pdw += L.zz[r];
        }
        const double epot = geo[GEO_U0] + elam;
        double* o = c.obs + ((size_t)rec * c.n_traj + c.home[t]) * IESH_N_OBS;
        o[IESH_OBS_PD_SURF] = pds;
        o[IESH_OBS_PD_WF] = pdw;
        o[IESH_OBS_EKIN] = ekin;
        o[IESH_OBS_EPOT] = epot;
        o[IESH_OBS_ETOT] = ekin + epot;
      }
    }
  }
}

// The bound for several classes (all of one kind) in one launch: block b
// works on slot b - first[k] of class k, classes largest first.
template <bool kF32, bool kDense>
__global__ __launch_bounds__(kFltThreads) void k_filter_fused(ClassSet set, double dt_run, uint64_t seed,
                                                              Counters* cnt, int record, int exit_enabled,
                                                              double exit_x, int64_t max_steps, double delta) {
  __shared__ FltLds L;
  const int b = blockIdx.x;
  int k = 0;
  while (k + 1 < set.n && b >= set.first[k + 1]) ++k;
  filter_one<kF32, kDense>(set.c[k], b - set.first[k], dt_run, seed, cnt, record, exit_enabled, exit_x,
                           max_steps, delta, L);
}

__global__ void k_advance(Counters* cnt) {
  if (threadIdx.x == 0 && blockIdx.x == 0) cnt->step = cnt->step + 1;
}

}  // namespace

// Register slots: RS rows of 16 for the N x N inverse (N <= 16 RS), RB rows
// of 16 for the n - N unoccupied states.  Buckets that cannot occur with
// n <= IESH_MAX_STATES are not instantiated.
constexpr int rs_floor(int rs) { return rs == 2 ? 0 : rs == 4 ? 2 : rs == 7 ? 4 : rs == 10 ? 7 : 10; }
constexpr int rb_floor(int rb) {
  return rb == 2 ? 0 : rb == 4 ? 2 : rb == 7 ? 4 : rb == 11 ? 7 : rb == 14 ? 11 : 14;
}
template <int RS, int RB>
constexpr bool bucket_possible(int max_states = kMaxStates) {
  return 16 * rs_floor(RS) + 1 + 16 * rb_floor(RB) + 1 <= max_states;
}

template <bool F32, int RS, int RB>
static void launch_hop_t(const ClassDev& c, dim3 grid, double dt, uint64_t seed, Counters* cnt,
                         iesh_event* events, int query_mode, int t0, int record,
                         int exit_enabled, double exit_x, int64_t max_steps, hipStream_t s) {
  if (c.Gd) {
    // the dense model kind: n <= IESH_DENSE_MAX_N
    if constexpr (bucket_possible<RS, RB>(IESH_DENSE_MAX_N))
      hipLaunchKernelGGL((k_hop<F32, RS, RB, true>), grid, dim3(kHopThreads), 0, s, c, dt, seed, cnt,
                         events, query_mode, t0, record, exit_enabled, exit_x, max_steps);
    return;
  }
  if constexpr (bucket_possible<RS, RB>())
    hipLaunchKernelGGL((k_hop<F32, RS, RB, false>), grid, dim3(kHopThreads), 0, s, c, dt, seed, cnt,
                       events, query_mode, t0, record, exit_enabled, exit_x, max_steps);
}

template <bool F32, int RS, int RB>
static const void* hop_fn_t(bool dense) {
  if (dense) {
    if constexpr (bucket_possible<RS, RB>(IESH_DENSE_MAX_N)) return (const void*)k_hop<F32, RS, RB, true>;
    return nullptr;
  }
  if constexpr (bucket_possible<RS, RB>()) return (const void*)k_hop<F32, RS, RB, false>;
  return nullptr;
}

template <bool F32, int RS>
static const void* hop_fn_rs(const ClassDev& c) {
  const int rb = (c.md.n - c.md.N + 15) / 16;
  const bool d = c.Gd != nullptr;
  if (rb <= 2) return hop_fn_t<F32, RS, 2>(d);
  if (rb <= 4) return hop_fn_t<F32, RS, 4>(d);
  if (rb <= 7) return hop_fn_t<F32, RS, 7>(d);
  if (rb <= 11) return hop_fn_t<F32, RS, 11>(d);
  if (rb <= 14) return hop_fn_t<F32, RS, 14>(d);
  return hop_fn_t<F32, RS, 21>(d);
}

template <bool F32>
static const void* hop_fn_p(const ClassDev& c) {
  const int rs = (c.md.N + 15) / 16;
  if (rs <= 2) return hop_fn_rs<F32, 2>(c);
  if (rs <= 4) return hop_fn_rs<F32, 4>(c);
  if (rs <= 7) return hop_fn_rs<F32, 7>(c);
  if (rs <= 10) return hop_fn_rs<F32, 10>(c);
  return hop_fn_rs<F32, 11>(c);
}

static const void* hop_fn(const ClassDev& c, int precision) {
  return precision == IESH_FP64 ? hop_fn_p<false>(c) : hop_fn_p<true>(c);
}

template <bool F32, int RS>
static void launch_hop_rs(const ClassDev& c, dim3 grid, double dt, uint64_t seed,
                          Counters* cnt, iesh_event* events, int query_mode, int t0,
                          int record, int exit_enabled, double exit_x, int64_t max_steps,
                          hipStream_t s) {
  const int rb = (c.md.n - c.md.N + 15) / 16;
#define IESH_HOP_RB(RBV)                                                                      \
  launch_hop_t<F32, RS, RBV>(c, grid, dt, seed, cnt, events, query_mode, t0, record,          \
                             exit_enabled, exit_x, max_steps, s)
  if (rb <= 2)
    IESH_HOP_RB(2);
  else if (rb <= 4)
    IESH_HOP_RB(4);
  else if (rb <= 7)
    IESH_HOP_RB(7);
  else if (rb <= 11)
    IESH_HOP_RB(11);
  else if (rb <= 14)
    IESH_HOP_RB(14);
  else
    IESH_HOP_RB(21);
#undef IESH_HOP_RB
}

template <bool F32>
static void launch_hop_p(const ClassDev& c, dim3 grid, double dt, uint64_t seed, Counters* cnt,
                         iesh_event* events, int query_mode, int t0, int record,
                         int exit_enabled, double exit_x, int64_t max_steps, hipStream_t s) {
  const int rs = (c.md.N + 15) / 16;
#define IESH_HOP_RS(RSV)                                                                      \
  launch_hop_rs<F32, RSV>(c, grid, dt, seed, cnt, events, query_mode, t0, record,             \
                          exit_enabled, exit_x, max_steps, s)
  if (rs <= 2)
    IESH_HOP_RS(2);
  else if (rs <= 4)
    IESH_HOP_RS(4);
  else if (rs <= 7)
    IESH_HOP_RS(7);
  else if (rs <= 10)
    IESH_HOP_RS(10);
  else
    IESH_HOP_RS(11);
#undef IESH_HOP_RS
}

// Work-groups of the ratio kernel resident at once (one trajectory each).
int hop_resident_groups(const ClassDev& c, int precision, int n_cu) {
  // every instantiation has 512 threads and the same static LDS; registers
  // differ by shape, so take the occupancy of the class's own kernel
  int per_cu = 0;
  const void* fn = hop_fn(c, precision);
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kHopThreads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return per_cu * n_cu;
}

bool hop_needs_scratch(const ClassDev& c) {
  const int rs = (c.md.N + 15) / 16, rb = (c.md.n - c.md.N + 15) / 16;
  const int RS = rs <= 2 ? 2 : rs <= 4 ? 4 : rs <= 7 ? 7 : rs <= 10 ? 10 : 11;
  const int RB = rb <= 2 ? 2 : rb <= 4 ? 4 : rb <= 7 ? 7 : rb <= 11 ? 11 : rb <= 14 ? 14 : 21;
  const int CS = (RS + 1) / 2;
  return 4 * RS * CS + 2 * RB * CS > 170;
}

hipError_t launch_hop(const ClassDev& c, double dt, uint64_t seed, Counters* cnt,
                      iesh_event* events, int query_mode, int t0, int nt, int record,
                      int exit_enabled, double exit_x, int64_t max_steps, int precision,
                      hipStream_t s) {
  if (!query_mode && c.n_live < 1) return hipSuccess;
  const int full = c.hop_groups > 0 && c.hop_groups < c.n_live ? c.hop_groups : c.n_live;
  const dim3 grid(query_mode ? nt : full);
  const int t0e = query_mode ? t0 : 0;
  if (precision == IESH_FP64)
    launch_hop_p<false>(c, grid, dt, seed, cnt, events, query_mode, t0e, record, exit_enabled,
                        exit_x, max_steps, s);
  else
    launch_hop_p<true>(c, grid, dt, seed, cnt, events, query_mode, t0e, record, exit_enabled,
                       exit_x, max_steps, s);
  return hipGetLastError();
}

hipError_t launch_filter_fused(const ClassSet& set, double dt, uint64_t seed, Counters* cnt, int record,
                               int exit_enabled, double exit_x, int64_t max_steps, int precision,
                               hipStream_t s) {
  if (set.n < 1 || set.first[set.n] < 1) return hipSuccess;
  const double delta = (precision == IESH_FP64) ? kDeltaFP64 : kDeltaMixed;
  const bool dense = set.c[0].Gd != nullptr;
  const dim3 grid(set.first[set.n]);
#define IESH_FUSED(F32, DENSE)                                                                           \
  hipLaunchKernelGGL((k_filter_fused<F32, DENSE>), grid, dim3(kFltThreads), 0, s, set, dt, seed, cnt, record, \
                     exit_enabled, exit_x, max_steps, delta)
  if (precision == IESH_FP64) {
    if (dense)
      IESH_FUSED(false, true);
    else
      IESH_FUSED(false, false);
  } else {
    if (dense)
      IESH_FUSED(true, true);
    else
      IESH_FUSED(true, false);
  }
#undef IESH_FUSED
  return hipGetLastError();
}

hipError_t launch_advance(Counters* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, cnt);
  return hipGetLastError();
}

}  // namespace iesh
