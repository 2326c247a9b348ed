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
// Two kernels evaluate these ratios, one 512-thread work-group per
// trajectory that the exact no-hop bound could not settle, taken in order
// from a per-class queue filled by the bound kernel: for N <= kMmCols the
// matrix-core kernel further below (panels of rows, rank-kPanel updates and
// the product Y on the FP64 matrix instructions); for wider occupied sets the
// register kernel described here.  Thread (ti, tj), tid =
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

// Hop selection (Sec. II.B: one uniform per trajectory and step, pairs in
// canonical order): the occupied row r from the cumulative row totals
// L.rowsum, whose entry is the first total above the step's uniform.
// Returns r (-1: no hop); sel_prev = cumulative total before row r,
// sel_margin = smallest |cumulative - xi| seen, sel_total = sum of all rows.
template <class LDS>
__device__ __forceinline__ int hop_select(const ClassDev& c, int t, uint64_t seed, Counters* cnt, bool singular, int N,
                          LDS& L, double& sel_prev_out, double& sel_margin_out, double& sel_total_out) {
  const int tid = threadIdx.x;
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
  sel_prev_out = sel_prev;
  sel_margin_out = sel_margin;
  sel_total_out = sel_total;
  const int r = sel_r;
  __syncthreads();  // every thread has read the selection before it is reused
  return r;
}

// The rest of the step once L.grow holds g of the selected row rsel by
// unoccupied position: the target b from the cumulative sum continued within
// the row, momentum rescaling along d = <b|d/dR a> (frustrated when the
// kinetic energy along d is too small), the occupation update, the force of
// the new occupations, the hop event, the step's status checks and the
// observable record.
template <bool kDense, class LDS>
__device__ __forceinline__ void hop_apply(const ClassDev& c, int t, Counters* cnt, iesh_event* events, int record,
                          int exit_enabled, double exit_x, int64_t max_steps, bool singular, int rsel,
                          double sel_prev, double sel_margin, double sel_total, LDS& L) {
  const int tid = threadIdx.x;
  const ModelDev& md = c.md;
  const int n = md.n, n_pad = md.n_pad, N = md.N, nU = n - N;
  const int nd = md.ndof;
  const double* geo = c.geo + (size_t)t * kGeoStride;
  const double h = geo[GEO_H];
  const double* Gd = kDense ? c.Gd + (size_t)t * n_pad * n_pad : nullptr;
  const double gtol = kDense ? 1e-12 * fmax(fabs(L.lam[0]), fabs(L.lam[n - 1])) : 0.0;
  auto coupling = [&](int b, int a) -> double {  // G[b][a]
    if constexpr (kDense) return fabs(L.lam[a] - L.lam[b]) <= gtol ? 0.0 : Gd[(size_t)b * n_pad + a];
    return 0.0;
  };
  const int64_t step = cnt->step;
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
    for (int r = tid; r < N; r += blockDim.x) c.occ[(size_t)t * N + r] = L.occ[r];
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

  double sel_prev = 0.0, sel_margin = 0.0, sel_total = 0.0;
  const int rsel = hop_select(c, t, seed, cnt, singular, N, L, sel_prev, sel_margin, sel_total);
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

  hop_apply<kDense>(c, t, cnt, events, record, exit_enabled, exit_x, max_steps, singular, rsel,
                    sel_prev, sel_margin, sel_total, L);
}

// ---------------------------------------------------------------------------
// Ratio kernel on the matrix cores (N <= kMmCols).  The same in-place
// Gauss-Jordan inversion with column pivoting, taken kPanel rows at a time.
// For the rows R of a panel, elimination of those rows alone (their pivots
// chosen one after another by the rule above) gives their final values
// P = [A^-1 | -A^-1 B] in the layout of the in-place array, where A = X[R][Q]
// and B = X[R][others] for the panel's pivot columns Q, and every other row
// then becomes
//     X[i][:] += X[i][Q] E,   E = P - I_Q  (I_Q: ones at (k, Q_k)),
// a rank-kPanel complex update on the FP64 matrix instructions; the panel
// rows take P.  The pivots come out as in the register kernel up to the
// pivot keys' resolution (13 significant bits of |X|^2 here), so the two
// kernels agree to rounding.  Wave 0 eliminates (lane l holds columns l and
// l + 64 of the panel rows: no barrier inside a panel) while waves 1..7, which hold column
// tiles 0..6 of X, apply the previous panel's update: the row tile of the
// next panel first, then, beside the elimination of that panel, the others.
// A panel costs three barriers.  X lives in the accumulator layout of the
// 16x16x4 FP64 instruction (lane l, element e: row lk + 4 e, column lr of the
// tile, with lr = l & 15, lk = l >> 4).  Element e of an accumulator tile is
// also the B operand of k-block e of the product Y = C_U[:, perm] X, whose
// A operand comes from LDS, 16 unoccupied states at a time (the next block
// loaded while the current one is multiplied); g goes to the trajectory's g
// buffer and the row totals are reduced inside the owning wave.
constexpr int kMmThreads = 512;
constexpr int kMmTiles = kMmThreads / 64 - 1;  // column tiles of X (waves 1..7)
constexpr int kMmCols = 16 * kMmTiles;         // N limit of the matrix-core path
constexpr int kPanel = 4;                      // rows per panel (a multiple of 4 dividing 16)
static_assert(kPanel % 4 == 0 && 16 % kPanel == 0, "panel rows");
static_assert(kMmCols <= 112, "panel columns: two per lane of the eliminating wave, 127 - j > 0 in the pivot keys");
constexpr int kCuLoads = (16 * kMmCols + kMmThreads - 1) / kMmThreads;  // C_U elements per thread

struct HopMmLds {
  double2 pan[kPanel][kMmCols];        // rows of the next panel before their elimination
  double2 ebuf[2][kPanel][kMmCols];    // E of a panel (by panel parity)
  double2 gq[2][kMmCols][kPanel + 1];  // X[:, Q] of a panel before its update
  double2 cu[2][16][kMmCols + 1];      // C[perm[q]][u_b] for 16 unoccupied states
  int qk[2][kPanel];                   // pivot columns of a panel (-1: none)
  double lam[kMaxStates];
  double q0[kMaxStates];
  double rowsum[kMaxElec];
  double grow[kMaxStates];  // g of the selected row, by unoccupied position
  double zz[kMaxElec];
  int occflag[kMaxStates];
  int uocc[kMaxStates];  // unoccupied states, ascending
  int perm[kMaxElec];
  int invperm[kMaxElec];
  int occ[kMaxElec];
  int singular;
  int sc_occ_changed;
  double sc_xi;
  double sc_ekin;
  double dofv[kMaxDof];
  double dofd[kMaxDof];
};

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline v4d mfma64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Value of lane `src` (wave-uniform) of a per-lane double.
__device__ inline double lane_value(double v, int src) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)u, src);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// 1/d for a normal d > 0: the hardware estimate and two Newton steps
// (each squares the relative error; the estimate is good to about 2^-23).
__device__ inline double rcp_pos(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// Maximum of a 32-bit key over the wave (wave-uniform result): within each
// row of 16 lanes by two quad permutations and two row rotations (every lane
// ends with its row's maximum), then across the four rows.
template <int kCtrl>
__device__ inline unsigned dpp_u32(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, 0xf, 0xf, false);
}
__device__ inline unsigned wave_max_u32(unsigned k) {
  k = max(k, dpp_u32<0xB1>(k));   // quad_perm [1, 0, 3, 2]
  k = max(k, dpp_u32<0x4E>(k));   // quad_perm [2, 3, 0, 1]
  k = max(k, dpp_u32<0x124>(k));  // row_ror:4
  k = max(k, dpp_u32<0x128>(k));  // row_ror:8
  const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)k, 0);
  const unsigned b = (unsigned)__builtin_amdgcn_readlane((int)k, 16);
  const unsigned c2 = (unsigned)__builtin_amdgcn_readlane((int)k, 32);
  const unsigned d = (unsigned)__builtin_amdgcn_readlane((int)k, 48);
  return max(max(a, b), max(c2, d));
}

// Elimination of the panel rows held in L.pan (rows < rows) among the
// columns not yet used (bit s of `used`: column l + 64 s), final values
// minus I_Q into L.ebuf[buf], pivots into L.qk[buf].  One wave; returns false
// when no finite nonzero pivot is left (S singular).  Pivot: the largest
// |X[i][j]|^2 to 13 significant bits (the high word of the double with its
// low 7 bits replaced by 127 - j: the bit pattern of a non-negative double
// orders like its value), ties to the smallest j; any pivot within a
// relative 2^-13 of the largest is as stable.
__device__ bool panel_eliminate(HopMmLds& L, int buf, int rows, int N, unsigned& used) {
  const int l = threadIdx.x & 63;
  double2 P[kPanel][2];
#pragma unroll
  for (int i = 0; i < kPanel; ++i) {
    P[i][0] = L.pan[i][l];
    P[i][1] = (l + 64 < kMmCols) ? L.pan[i][l + 64] : make_double2(0.0, 0.0);
  }
  bool ok = true;
  int qk[kPanel];
#pragma unroll
  for (int i = 0; i < kPanel; ++i) {
    qk[i] = -1;
    if (i < rows && ok) {  // uniform
      unsigned k = 0u;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int col = l + 64 * s;
        const double m = P[i][s].x * P[i][s].x + P[i][s].y * P[i][s].y;
        const unsigned kj = ((unsigned)(__double_as_longlong(m) >> 32) & ~0x7Fu) | (unsigned)(127 - col);
        const bool cand = col < N && !((used >> s) & 1u) && m > 0.0 && m < INFINITY;
        k = cand ? max(k, kj) : k;
      }
      k = wave_max_u32(k);
      if (k == 0u) {
        ok = false;  // no finite nonzero candidate
      } else {
        const int pc = 127 - (int)(k & 0x7Fu);
        const int owner = pc & 63, ps = pc >> 6;
        if (l == owner) used |= 1u << ps;
        const double2 pv = ps ? P[i][1] : P[i][0];
        const double2 piv = make_double2(lane_value(pv.x, owner), lane_value(pv.y, owner));
        const double mp = piv.x * piv.x + piv.y * piv.y;
        const double inv_m = mp > 1e-290 ? rcp_pos(mp) : 1.0 / mp;  // uniform
        const double2 pinv = make_double2(piv.x * inv_m, -piv.y * inv_m);
        const double2 rv0 = P[i][0], rv1 = P[i][1];
        P[i][0] = make_double2(0.0, 0.0);
        P[i][1] = make_double2(0.0, 0.0);
#pragma unroll
        for (int i2 = 0; i2 < kPanel; ++i2) {
          if (i2 < rows) {  // uniform
            double2 f;
            if (i2 == i) {
              f = pinv;
            } else {
              const double2 cv = ps ? P[i2][1] : P[i2][0];
              f = cmul(make_double2(lane_value(cv.x, owner), lane_value(cv.y, owner)), pinv);
            }
            // X[i2][j] -= X[i][j] f for every column (the pivot column then
            // takes f)
            P[i2][0].x = fma(-rv0.x, f.x, P[i2][0].x);
            P[i2][0].x = fma(rv0.y, f.y, P[i2][0].x);
            P[i2][0].y = fma(-rv0.x, f.y, P[i2][0].y);
            P[i2][0].y = fma(-rv0.y, f.x, P[i2][0].y);
            P[i2][1].x = fma(-rv1.x, f.x, P[i2][1].x);
            P[i2][1].x = fma(rv1.y, f.y, P[i2][1].x);
            P[i2][1].y = fma(-rv1.x, f.y, P[i2][1].y);
            P[i2][1].y = fma(-rv1.y, f.x, P[i2][1].y);
            if (l == owner) {
              if (ps)
                P[i2][1] = f;
              else
                P[i2][0] = f;
            }
          }
        }
        qk[i] = pc;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kPanel; ++i) {
    double2 e0v = P[i][0], e1v = P[i][1];
    if (!ok || qk[i] < 0) {
      e0v = make_double2(0.0, 0.0);
      e1v = make_double2(0.0, 0.0);
    } else {
      if (qk[i] == l) e0v.x -= 1.0;
      if (qk[i] == l + 64) e1v.x -= 1.0;
    }
    L.ebuf[buf][i][l] = e0v;
    if (l + 64 < kMmCols) L.ebuf[buf][i][l + 64] = e1v;
    if (l == 0) L.qk[buf][i] = ok ? qk[i] : -1;
  }
  return ok;
}

template <bool kF32, bool kDense>
__device__ __forceinline__ void hop_one_mm(const ClassDev& c, int t, double dt_run, uint64_t seed,
                                           Counters* cnt, iesh_event* events, int query_mode, int record,
                                           int exit_enabled, double exit_x, int64_t max_steps, HopMmLds& L) {
  const double dt = c.clock ? c.clock[2 * (size_t)t] : dt_run;  // this trajectory's step
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
  const ModelDev& md = c.md;
  const int n = md.n, n_pad = md.n_pad, N = md.N, nU = n - N;
  const int RT = (N + 15) >> 4;
  const int ct = w - 1;                       // this wave's column tile of X
  const bool owns = w >= 1 && ct < RT;        // uniform
  const int col = 16 * ct + lr;               // this lane's column of X (owners)
  if (!query_mode && (c.status[t] & kFreezeMask)) return;  // uniform
  const size_t base = (size_t)t * N * n_pad;
  if (!query_mode && tid == 0) atomicAdd((unsigned long long*)&cnt->hop_evals, 1ull);
  __syncthreads();  // the previous trajectory of this work-group is done with L

  for (int k = tid; k < n_pad; k += kMmThreads) {
    L.lam[k] = c.lam[(size_t)t * n_pad + k];
    L.q0[k] = c.q0[(size_t)t * n_pad + k];
    L.occflag[k] = 0;
  }
  if (tid == 0) L.singular = 0;
  __syncthreads();
  for (int r = tid; r < N; r += kMmThreads) {
    const int a = c.occ[(size_t)t * N + r];
    L.occ[r] = a;
    L.occflag[a] = 1;
  }
  __syncthreads();
  // unoccupied list: b sits at position b - #{occupied < b}
  for (int b = tid; b < n; b += kMmThreads) {
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
  // impurity amplitude of every orbital, sum_i q0_i C[i][j] (observable)
  if (record && !query_mode) {
    for (int j = w; j < N; j += kMmThreads / 64) {
      double zr = 0.0, zi = 0.0;
      for (int i = l; i < n_pad; i += 64) {
        const double2 z = orb<kF32>(c, base, n_pad, j, i);
        zr += L.q0[i] * z.x;
        zi += L.q0[i] * z.y;
      }
      for (int m = 32; m > 0; m >>= 1) {
        zr += __shfl_xor(zr, m);
        zi += __shfl_xor(zi, m);
      }
      if (l == 0) L.zz[j] = zr * zr + zi * zi;
    }
  }
  // columns of the panel rows that no wave holds stay zero
  for (int e = tid; e < kPanel * kMmCols; e += kMmThreads) {
    if (e % kMmCols >= 16 * RT) L.pan[e / kMmCols][e % kMmCols] = make_double2(0.0, 0.0);
  }
  __syncthreads();

  // ---- X = S = C[s, :]: xr/xi[it] is tile (it, ct)
  // (every load in bounds and unconditional, so that they are all in flight
  // at once; elements outside S are then set to zero)
  v4d xr[kMmTiles], xi[kMmTiles];
#pragma unroll
  for (int it = 0; it < kMmTiles; ++it) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 16 * it + lk + 4 * e;
      const bool in = owns && row < N && col < N;
      const double2 z = orb<kF32>(c, base, n_pad, in ? col : 0, L.occ[in ? row : 0]);
      xr[it][e] = in ? z.x : 0.0;
      xi[it][e] = in ? z.y : 0.0;
    }
  }

  // update of tile it by panel pp (buffer pb), then the panel's own rows take P
  auto update_tile = [&](v4d& tr, v4d& ti, int it, int pp) {
    const int pb = pp & 1;
#pragma unroll
    for (int kb = 0; kb < kPanel / 4; ++kb) {
      const double2 eb = L.ebuf[pb][4 * kb + lk][col];
      const double2 ga = L.gq[pb][16 * it + lr][4 * kb + lk];
      tr = mfma64(ga.x, eb.x, tr);
      tr = mfma64(-ga.y, eb.y, tr);
      ti = mfma64(ga.x, eb.y, ti);
      ti = mfma64(ga.y, eb.x, ti);
    }
    if (it == (kPanel * pp) >> 4) {
      // selects, not conditional stores: merged stores would index the
      // register tile at run time
      const int e0 = ((kPanel * pp) & 15) >> 2;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool in = e >= e0 && e < e0 + kPanel / 4;
        const int i = in ? lk + 4 * (e - e0) : 0;
        const double2 ev = L.ebuf[pb][i][col];
        const double nx = ev.x + (L.qk[pb][i] == col ? 1.0 : 0.0);
        tr[e] = in ? nx : tr[e];
        ti[e] = in ? ev.y : ti[e];
      }
    }
  };
  // rows of panel pp (before elimination) to L.pan
  auto panel_rows = [&](const v4d& tr, const v4d& ti, int pp) {
    const int e0 = ((kPanel * pp) & 15) >> 2;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (e >= e0 && e < e0 + kPanel / 4) L.pan[lk + 4 * (e - e0)][col] = make_double2(tr[e], ti[e]);
  };
  // pivot columns of X for panel pp (buffer pb) to L.gq, before its update:
  // the lanes whose column is a pivot write it, all pivots at once
  auto gather_q = [&](int pp) {
    const int pb = pp & 1;
    int kk = -1;
#pragma unroll
    for (int k = 0; k < kPanel; ++k)
      if (L.qk[pb][k] == col) kk = k;
    if (owns && kk >= 0) {
#pragma unroll
      for (int it = 0; it < kMmTiles; ++it)
#pragma unroll
        for (int e = 0; e < 4; ++e) L.gq[pb][16 * it + lk + 4 * e][kk] = make_double2(xr[it][e], xi[it][e]);
    }
#pragma unroll
    for (int k = 0; k < kPanel; ++k) {
      const int q = L.qk[pb][k];
      if (q < 0) {
        // no pivot (rows past N, or S singular): a zero column
        for (int row = tid; row < kMmCols; row += kMmThreads) L.gq[pb][row][k] = make_double2(0.0, 0.0);
      } else if (tid == 0) {
        L.perm[kPanel * pp + k] = q;
      }
    }
  };

  // ---- panels
  unsigned used = 0u;  // wave 0: bit s, column l + 64 s has been a pivot
  const int n_panels = (N + kPanel - 1) / kPanel;
  if (owns) panel_rows(xr[0], xi[0], 0);
  __syncthreads();
  if (w == 0 && !panel_eliminate(L, 0, min(kPanel, N), N, used) && l == 0) L.singular = 1;
  __syncthreads();
  gather_q(0);
  __syncthreads();
  for (int p = 0; p < n_panels; ++p) {
    const bool next = p + 1 < n_panels;
    const int itn = (kPanel * (p + 1)) >> 4;  // row tile of the next panel
    // (a) the next panel's row tile first, and its rows to L.pan
    if (owns && next) {
#pragma unroll
      for (int it = 0; it < kMmTiles; ++it) {
        if (it == itn) {
          update_tile(xr[it], xi[it], it, p);
          panel_rows(xr[it], xi[it], p + 1);
        }
      }
    }
    __syncthreads();
    // (b) wave 0 eliminates the next panel while the others finish the update
    if (w == 0) {
      if (next && !panel_eliminate(L, (p + 1) & 1, min(kPanel, N - kPanel * (p + 1)), N, used) && l == 0)
        L.singular = 1;
    } else if (owns) {
#pragma unroll
      for (int it = 0; it < kMmTiles; ++it)
        if (it < RT && !(next && it == itn)) update_tile(xr[it], xi[it], it, p);
    }
    __syncthreads();
    // (c) the next panel's pivot columns
    if (next) gather_q(p + 1);
    __syncthreads();
  }
  const bool singular = L.singular != 0;
  if (!singular) {
    for (int r = tid; r < N; r += kMmThreads) L.invperm[L.perm[r]] = r;
  }
  double* gout = c.gbuf + (size_t)t * N * n_pad;
  if (query_mode) {
    for (int e = tid; e < N * n_pad; e += kMmThreads) gout[e] = 0.0;
  }
  __syncthreads();

  // ---- Y[b][c] = Re sum_q C[perm[q]][u_b] X[q][c], 16 unoccupied states at a
  // time, and g of every (occupied, unoccupied) pair
  const double* geo = c.geo + (size_t)t * kGeoStride;
  const int nd = md.ndof;
  const double h = geo[GEO_H];
  const bool multi = nd > 1;
  const double dh = multi ? geo[GEO_VDH] : geo[GEO_DH];
  const double rho = multi ? geo[GEO_VRHO] : geo[GEO_RHO];
  const double v = multi ? 1.0 : c.v[(size_t)t * nd];
  const double* Gd = kDense ? c.Gd + (size_t)t * n_pad * n_pad : nullptr;
  const double gtol = kDense ? 1e-12 * fmax(fabs(L.lam[0]), fabs(L.lam[n - 1])) : 0.0;
  // element e = tid + kMmThreads j of a block: unoccupied position 16 bt + e % 16, column e / 16
  auto load_cu = [&](int bt, double2* r) {
#pragma unroll
    for (int j = 0; j < kCuLoads; ++j) {
      const int e = tid + kMmThreads * j;
      const int bi = 16 * bt + (e & 15), q = e >> 4;
      const bool in = e < 16 * kMmCols && q < N && bi < nU && !singular;
      // (perm is complete only when S is not singular: index 0 otherwise)
      const int orbital = in ? L.perm[q] : 0, state = in ? L.uocc[bi] : 0;
      const double2 z = orb<kF32>(c, base, n_pad, orbital, state);
      r[j] = in ? z : make_double2(0.0, 0.0);
    }
  };
  auto store_cu = [&](int buf, const double2* r) {
#pragma unroll
    for (int j = 0; j < kCuLoads; ++j) {
      const int e = tid + kMmThreads * j;
      if (e < 16 * kMmCols) L.cu[buf][e & 15][e >> 4] = r[j];
    }
  };
  double rsum = 0.0;
  const int r_own = (owns && col < N && !singular) ? L.invperm[col] : 0;
  const int a_own = L.occ[r_own];
  const int BT = (nU + 15) >> 4;
  double2 pre[kCuLoads];
  load_cu(0, pre);
  store_cu(0, pre);
  __syncthreads();
  for (int bt = 0; bt < BT; ++bt) {
    const int cb = bt & 1;
    if (bt + 1 < BT) load_cu(bt + 1, pre);
    if (owns) {
      v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int qt = 0; qt < kMmTiles; ++qt) {
        if (qt < RT) {
#pragma unroll
          for (int kb = 0; kb < 4; ++kb) {
            const double2 av = L.cu[cb][lr][16 * qt + 4 * kb + lk];
            acc = mfma64(av.x, xr[qt][kb], acc);
            acc = mfma64(-av.y, xi[qt][kb], acc);
          }
        }
      }
      if (col < N && !singular) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int bi = 16 * bt + lk + 4 * e;
          if (bi < nU) {
            const int bb = L.uocc[bi];
            const double gab =
                kDense ? (fabs(L.lam[a_own] - L.lam[bb]) <= gtol ? 0.0 : Gd[(size_t)bb * n_pad + a_own])
                       : L.q0[bb] * L.q0[a_own] * (dh + rho * ((L.lam[bb] - h) + (L.lam[a_own] - h)));
            // v <b|d/dx a> (the deflated cases as in the register kernel)
            const double vD = v * gab / (L.lam[a_own] - L.lam[bb]);
            const double g = fmax(-2.0 * dt * vD * acc[e], 0.0);
            rsum += g;
            gout[(size_t)r_own * n_pad + bb] = g;
          }
        }
      }
    }
    if (bt + 1 < BT) store_cu(cb ^ 1, pre);
    __syncthreads();
  }
  // row totals: the four lanes of a column hold its rows lk + 4 e
  rsum += __shfl_xor(rsum, 16);
  rsum += __shfl_xor(rsum, 32);
  if (owns && lk == 0 && col < N && !singular) L.rowsum[r_own] = rsum;
  __syncthreads();
  if (query_mode) {
    if (singular && tid == 0) c.status[t] |= IESH_TRAJ_SINGULAR_S;
    return;
  }
  double sel_prev = 0.0, sel_margin = 0.0, sel_total = 0.0;
  const int rsel = hop_select(c, t, seed, cnt, singular, N, L, sel_prev, sel_margin, sel_total);
  if (rsel >= 0) {
    for (int bi = tid; bi < nU; bi += kMmThreads) L.grow[bi] = gout[(size_t)rsel * n_pad + L.uocc[bi]];
  }
  __syncthreads();
  hop_apply<kDense>(c, t, cnt, events, record, exit_enabled, exit_x, max_steps, singular, rsel,
                    sel_prev, sel_margin, sel_total, L);
}

template <bool kF32, bool kDense>
__global__ __launch_bounds__(kMmThreads) void k_hop_mm(ClassDev c, double dt, uint64_t seed, Counters* cnt,
                                                       iesh_event* events, int query_mode, int t0,
                                                       int record, int exit_enabled, double exit_x,
                                                       int64_t max_steps) {
  __shared__ HopMmLds L;
  int32_t* q = c.hopq;
  const int b = blockIdx.x;
  const int n_items = query_mode ? 1 : q[0];
  for (int e = query_mode ? 0 : b; e < n_items; e += gridDim.x) {
    const int t = query_mode ? t0 + b : q[3 + e];
    hop_one_mm<kF32, kDense>(c, t, dt, seed, cnt, events, query_mode, record, exit_enabled, exit_x,
                             max_steps, L);
  }
  if (!query_mode && threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&q[2], 1) == (int)gridDim.x - 1) {
      q[0] = 0;
      q[2] = 0;
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
  // row norms of C (state b over all orbitals); ||C_U||_F^2 over unoccupied b.
  // The propagation leaves the squared norms per slab of orbitals (c.rown);
  // without them the orbitals are read here.
  const size_t base = (size_t)t * N * n_pad;
  double fro_part = 0.0;
  const int slabs_max = (N + 7) >> 3;
  for (int b = tid; b < n_pad; b += kFltThreads) {
    double s2 = 0.0;
    if (c.rown) {
      for (int sl = 0; sl < c.n_slabs; ++sl) s2 += c.rown[((size_t)t * slabs_max + sl) * n_pad + b];
    } else {
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

// The matrix-core kernel serves N <= kMmCols; wider occupied sets keep the
// register kernel.
static bool hop_mm(const ClassDev& c) { return c.md.N <= kMmCols; }

static const void* hop_mm_fn(const ClassDev& c, int precision) {
  const bool d = c.Gd != nullptr;
  if (precision == IESH_FP64) return d ? (const void*)k_hop_mm<false, true> : (const void*)k_hop_mm<false, false>;
  return d ? (const void*)k_hop_mm<true, true> : (const void*)k_hop_mm<true, false>;
}

static const void* hop_fn(const ClassDev& c, int precision) {
  if (hop_mm(c)) return hop_mm_fn(c, precision);
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
  // registers and LDS differ by kernel and shape, so take the occupancy of
  // the class's own kernel
  int per_cu = 0;
  const void* fn = hop_fn(c, precision);
  const int threads = hop_mm(c) ? kMmThreads : kHopThreads;
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return per_cu * n_cu;
}

bool hop_needs_scratch(const ClassDev& c) {
  if (hop_mm(c)) return false;
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
  if (hop_mm(c)) {
    const bool d = c.Gd != nullptr;
#define IESH_MM(F32, DENSE)                                                                        \
  hipLaunchKernelGGL((k_hop_mm<F32, DENSE>), grid, dim3(kMmThreads), 0, s, c, dt, seed, cnt, events, \
                     query_mode, t0e, record, exit_enabled, exit_x, max_steps)
    if (precision == IESH_FP64) {
      if (d)
        IESH_MM(false, true);
      else
        IESH_MM(false, false);
    } else {
      if (d)
        IESH_MM(true, true);
      else
        IESH_MM(true, false);
    }
#undef IESH_MM
    return hipGetLastError();
  }
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
