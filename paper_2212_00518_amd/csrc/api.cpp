// C ABI of libiesh: context, device memory, state transfer, step loop.

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "iesh_internal.hpp"

using namespace iesh;

struct iesh_ctx {
  std::vector<ClassDev> cls;
  std::vector<int32_t> traj_class;  // global trajectory -> class
  std::vector<int32_t> traj_local;  // global trajectory -> home index inside its class
  std::vector<std::vector<int32_t>> members;    // per class: home index -> global trajectory
  std::vector<std::vector<int32_t>> slot_home;  // per class: slot -> home index
  std::vector<std::vector<int32_t>> home_slot;  // per class: home index -> slot
  std::vector<CompactBufs> spare;               // per class, when compaction is enabled
  std::vector<std::vector<int64_t>> caps_home;  // per class: step cap by home index
  iesh_run_desc run{};
  hipStream_t stream = nullptr;
  bool own_stream = false;  // created here when the caller passes none
  int device = 0;
  Counters* cnt = nullptr;
  iesh_event* events = nullptr;
  int n_max = 0, N_max = 0;
  int ndof = 1;  // nuclear coordinates per trajectory (all models)
  int n_cu = 256;  // compute units of the device
  int64_t step = 0;
  size_t device_bytes = 0;
  std::string err;
  std::vector<std::pair<void*, size_t>> allocations;  // (pointer, bytes)
  // graph cache for iesh_run: one step, and the device-side compaction
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_record = -1;
  hipGraphExec_t compact_exec = nullptr;
  hipGraph_t compact_graph = nullptr;
  std::vector<int> live_host;  // live slots per class at the last refresh
  int64_t obs_records = 0;  // capacity of the class observable buffers
  // per-kernel timing with HIP events (diagnostic)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_marks;  // (timer, index of the start event)
  // adjoint along prescribed paths: buffers of the last forward pass
  struct AdjClass {
    double* ckpt = nullptr;    // [n_ckpt][T][N][n_pad] complex: C at the segment starts
    double* snap = nullptr;    // [seg + 1][T][N][n_pad] complex: C inside one segment
    double* Gh = nullptr;      // [T][N][n_pad] complex: cotangent of C (Wirtinger, dL/d conj C)
    double* taps_s = nullptr;  // [T][tap_k][N][n_pad] complex: adjoint Clenshaw vectors
    double* taps_t = nullptr;  // [T][tap_k][N][n_pad] complex: Chebyshev vectors
    double* imphi = nullptr;   // [T][n_pad][n_pad]
    double* rediag = nullptr;  // [T][n_pad]
    double* chebc = nullptr;   // [T][kChebStride] conjugated series
    double* hopscr = nullptr;  // hop-term scratch (S | I, W, Gbar_U, R, Dbar per trajectory)
    double* hopbar = nullptr;  // [T][2 n_pad + 1] hop-term cotangents of (q0, lambda, h')
  };
  std::vector<AdjClass> adj;
  std::vector<void*> adj_allocs;
  double* adj_path = nullptr;  // [n_traj][n_steps + 1]
  double* adj_loss = nullptr;  // [n_traj]
  double* adj_w = nullptr;     // [n_traj]
  double* adj_grad = nullptr;  // [n_traj][n_max + 4]
  int adj_steps = 0, adj_ckpt = 0, adj_tap_k = 0;
  AdjTerms adj_terms{1.0, 1.0, 0.0, 0.0};
  bool adj_forward_done = false, adj_backward_bufs = false;
};

namespace {

int fail(iesh_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

#define HIPTRY(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, IESH_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

template <typename T>
int dalloc(iesh_ctx* ctx, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return IESH_OK;
  void* q = nullptr;
  const size_t bytes = count * sizeof(T);
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) return fail(ctx, IESH_ENOMEM, "hipMalloc failed: " + std::to_string(bytes) + " bytes");
  ctx->allocations.push_back({q, bytes});
  if (hipMemsetAsync(q, 0, bytes, ctx->stream) != hipSuccess)
    return fail(ctx, IESH_EDEVICE, "hipMemsetAsync failed");
  ctx->device_bytes += bytes;
  *p = reinterpret_cast<T*>(q);
  return IESH_OK;
}

// Free one allocation made by dalloc (after the stream has drained).
template <typename T>
void dfree(iesh_ctx* ctx, T*& p) {
  if (!p) return;
  for (size_t i = 0; i < ctx->allocations.size(); ++i)
    if (ctx->allocations[i].first == (void*)p) {
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipFree(p);
      ctx->device_bytes -= ctx->allocations[i].second;
      ctx->allocations.erase(ctx->allocations.begin() + i);
      break;
    }
  p = nullptr;
}

void free_graph(iesh_ctx* ctx) {
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  if (ctx->compact_exec) (void)hipGraphExecDestroy(ctx->compact_exec);
  if (ctx->compact_graph) (void)hipGraphDestroy(ctx->compact_graph);
  ctx->graph_exec = nullptr;
  ctx->graph = nullptr;
  ctx->graph_record = -1;
  ctx->compact_exec = nullptr;
  ctx->compact_graph = nullptr;
}

int round16(int v) { return (v + 15) / 16 * 16; }

// Propagation work split: column tiles of 8 orbitals, up to
// prop_max_col_tiles per work-group, limited by the LDS footprint.
hipEvent_t next_event(iesh_ctx* ctx);

// Largest slab width (16-column tiles per propagation work-group) whose LDS
// fits and whose output tiles (row tiles x slab width, dealt to 8 waves) stay
// within the per-wave tile count the kernel is compiled for, not above `limit`.
int widest_slab(ClassDev& c, int precision, int limit) {
  const size_t lds_budget = 160 * 1024;
  const int tiles = (c.md.N + 7) / 8;
  const int RT = c.md.n_pad / 16;
  int nct = std::min(std::min(prop_max_col_tiles(precision), tiles), limit);
  for (; nct > 1; --nct) {
    c.nct_max = nct;
    const bool fits_waves = (RT * nct + 7) / 8 <= prop_max_tiles_per_wave(precision);
    if (fits_waves && prop_lds_bytes(c, precision) <= lds_budget) break;
  }
  return std::max(nct, 1);
}

// Split the orbital tiles into slabs of at most nct tiles, balanced.
void set_slabs(ClassDev& c, int nct) {
  const int tiles = (c.md.N + 7) / 8;
  c.n_slabs = (tiles + nct - 1) / nct;
  c.nct_max = (tiles + c.n_slabs - 1) / c.n_slabs;
}

void choose_slabs(ClassDev& c, int precision) { set_slabs(c, widest_slab(c, precision, 1 << 20)); }

// Time the propagation kernel for every slab width on a sample of slots
// (K = 12 terms, zero data: the time depends on the shapes only) and keep the
// fastest per trajectory.  Results do not depend on the choice: every output
// tile accumulates its k-blocks in the same order.
int autotune_slabs(iesh_ctx* ctx, ClassDev& c) {
  const int prec = ctx->run.precision;
  const int widest = widest_slab(c, prec, 1 << 20);
  if (widest <= 1 || c.n_traj < 64) {
    set_slabs(c, widest);
    return IESH_OK;
  }
  const int sample = std::min(c.n_traj, 4 * ctx->n_cu);
  std::vector<double> cb(kChebStride, 0.0);
  cb[CHEB_K] = 12.0;
  cb[CHEB_INVR] = 1.0;
  for (int t = 0; t < sample; ++t)
    HIPTRY(ctx, hipMemcpyAsync(c.cheb + (size_t)t * kChebStride, cb.data(), cb.size() * sizeof(double),
                               hipMemcpyHostToDevice, ctx->stream));
  hipEvent_t e0 = next_event(ctx), e1 = next_event(ctx);
  if (!e0 || !e1) return fail(ctx, IESH_EDEVICE, "event creation failed");
  const int saved_live = c.n_live;
  int32_t* saved_dev_live = c.live;
  c.n_live = sample;
  c.live = nullptr;  // the timing launches cover the sample slots
  int best = widest;
  float best_ms = 1e30f;
  std::vector<int> seen;
  for (int nct = 1; nct <= widest; ++nct) {
    set_slabs(c, nct);
    if (std::find(seen.begin(), seen.end(), c.nct_max) != seen.end()) continue;
    seen.push_back(c.nct_max);
    HIPTRY(ctx, prop_prepare(c, prec));
    float ms_min = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      HIPTRY(ctx, hipEventRecord(e0, ctx->stream));
      HIPTRY(ctx, launch_prop(c, prec, ctx->stream));
      HIPTRY(ctx, hipEventRecord(e1, ctx->stream));
      HIPTRY(ctx, hipEventSynchronize(e1));
      float ms = 0.0f;
      HIPTRY(ctx, hipEventElapsedTime(&ms, e0, e1));
      ms_min = std::min(ms_min, ms);
    }
    if (ms_min < best_ms) {
      best_ms = ms_min;
      best = c.nct_max;
    }
  }
  ctx->ev_used = 0;
  c.n_live = saved_live;
  c.live = saved_dev_live;
  set_slabs(c, best);
  HIPTRY(ctx, prop_prepare(c, prec));
  HIPTRY(ctx, hipMemsetAsync(c.cheb, 0, (size_t)sample * kChebStride * sizeof(double), ctx->stream));
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  return IESH_OK;
}

int model_ndof(const iesh_model_desc& m) { return m.n_dof < 1 ? 1 : m.n_dof; }

// Distinct bath energies of a model with their summed weights, the map from
// adiabatic index to secular root or deflated state (ModelDev::expand), and
// the lead-0 shares of two-lead models (ModelDev::lead0).
struct BathPoles {
  std::vector<double> eps, w, lead0;
  std::vector<int32_t> expand;
};

BathPoles bath_poles(const iesh_model_desc& d) {
  BathPoles b;
  std::vector<int> size;        // levels per pole
  std::vector<double> w0;       // lead-0 weight per pole
  std::vector<int> n0;          // lead-0 levels per pole
  for (int k = 0; k < d.n_bath; ++k) {
    const bool l0 = d.lead && d.lead[k] == 0;
    if (k == 0 || d.eps[k] != d.eps[k - 1]) {
      b.eps.push_back(d.eps[k]);
      b.w.push_back(0.0);
      size.push_back(0);
      w0.push_back(0.0);
      n0.push_back(0);
    }
    b.w.back() += d.w[k];
    size.back() += 1;
    if (l0) {
      w0.back() += d.w[k];
      n0.back() += 1;
    }
  }
  const int Mr = (int)b.eps.size();
  // root 0, then per pole m its g_m - 1 deflated states and root m + 1
  b.expand.push_back(0);
  for (int m = 0; m < Mr; ++m) {
    for (int q = 1; q < size[m]; ++q) b.expand.push_back(-(m + 1));
    b.expand.push_back(m + 1);
  }
  if (d.lead) {
    b.lead0.assign(2 * Mr, 0.0);
    for (int m = 0; m < Mr; ++m) {
      const double phi = w0[m] / b.w[m];
      b.lead0[m] = phi;
      // the deflated states of a pole carry the pole's levels minus the
      // coupled combination; each gets the mean over them
      b.lead0[Mr + m] = size[m] > 1 ? (n0[m] - phi) / (size[m] - 1) : 0.0;
    }
  }
  return b;
}

int validate_dense(const iesh_model_desc& m, std::string& why) {
  if (m.n_dof > 1) {
    why = "IESH_MODEL_DENSE has one coordinate";
    return 0;
  }
  if (m.n_bath < 1 || m.n_bath + 1 > IESH_DENSE_MAX_N) {
    why = "IESH_MODEL_DENSE: n = n_bath + 1 out of range [2, IESH_DENSE_MAX_N]";
    return 0;
  }
  if (m.n_elec < 1 || m.n_elec > m.n_bath) {
    why = "n_elec out of range";
    return 0;
  }
  if (!m.dense) {
    why = "IESH_MODEL_DENSE needs the matrices H0 and H1 (dense)";
    return 0;
  }
  const int n = m.n_bath + 1;
  for (int h = 0; h < 2; ++h) {
    const double* H = m.dense + (size_t)h * n * n;
    double big = 0.0;
    for (int q = 0; q < n * n; ++q) {
      if (!std::isfinite(H[q])) {
        why = "IESH_MODEL_DENSE: non-finite matrix element";
        return 0;
      }
      big = std::max(big, std::fabs(H[q]));
    }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j)
        if (std::fabs(H[(size_t)i * n + j] - H[(size_t)j * n + i]) > 1e-14 * big) {
          why = h ? "IESH_MODEL_DENSE: H1 is not symmetric" : "IESH_MODEL_DENSE: H0 is not symmetric";
          return 0;
        }
  }
  if (!(m.mass > 0.0) || !std::isfinite(m.params[0]) || !std::isfinite(m.params[1])) {
    why = "mass must be > 0 and omega, x_c finite";
    return 0;
  }
  if (m.lead) {
    why = "IESH_MODEL_DENSE has no leads";
    return 0;
  }
  return 1;
}

int validate_model(const iesh_model_desc& m, std::string& why) {
  if (m.kind == IESH_MODEL_DENSE) return validate_dense(m, why);
  if (m.kind != IESH_MODEL_HARMONIC && m.kind != IESH_MODEL_MORSE_TANH &&
      m.kind != IESH_MODEL_MULTI_DOF) {
    why = "unknown model kind";
    return 0;
  }
  if (m.kind != IESH_MODEL_MULTI_DOF && model_ndof(m) != 1) {
    why = "only IESH_MODEL_MULTI_DOF has several coordinates";
    return 0;
  }
  if (m.kind == IESH_MODEL_MULTI_DOF) {
    if (m.n_dof < 1 || m.n_dof > IESH_MAX_DOF || !m.dof) {
      why = "n_dof out of range [1, IESH_MAX_DOF] or dof missing";
      return 0;
    }
    for (int nu = 0; nu < m.n_dof; ++nu) {
      const double* r = m.dof + 7 * nu;
      for (int q = 0; q < 7; ++q)
        if (!std::isfinite(r[q])) {
          why = "non-finite coordinate constant";
          return 0;
        }
      if (!(r[0] > 0.0) || !(r[6] > 0.0)) {
        why = "coordinate mass and Gaussian width must be > 0";
        return 0;
      }
    }
  }
  if (m.n_bath < 1 || m.n_bath + 1 > IESH_MAX_STATES) {
    why = "n_bath out of range [1, IESH_MAX_STATES-1]";
    return 0;
  }
  if (m.n_elec < 1 || m.n_elec > m.n_bath || m.n_elec > IESH_MAX_ELEC) {
    why = "n_elec out of range";
    return 0;
  }
  if (!m.eps || !m.w) {
    why = "eps and w must be given";
    return 0;
  }
  for (int k = 0; k < m.n_bath; ++k) {
    if (!(m.w[k] > 0.0) || !std::isfinite(m.eps[k])) {
      why = "bath weights must be > 0 and energies finite";
      return 0;
    }
    if (k && !(m.eps[k] >= m.eps[k - 1])) {
      why = "bath energies must be ascending";
      return 0;
    }
    if (m.lead && m.lead[k] != 0 && m.lead[k] != 1) {
      why = "lead labels must be 0 or 1";
      return 0;
    }
  }
  if ((m.kind != IESH_MODEL_MULTI_DOF && !(m.mass > 0.0)) || !(m.Gamma > 0.0)) {
    why = "mass and Gamma must be > 0";
    return 0;
  }
  return 1;
}

int upload_state(iesh_ctx* ctx, const double* x, const double* v, const double* C,
                 const int32_t* occ) {
  const int T = ctx->run.n_traj;
  for (size_t ci = 0; ci < ctx->cls.size(); ++ci) {
    ClassDev& c = ctx->cls[ci];
    const int Tc = c.n_traj, N = c.md.N, n = c.md.n, n_pad = c.md.n_pad, nd = ctx->ndof;
    std::vector<double> hx((size_t)Tc * nd), hv((size_t)Tc * nd);
    std::vector<int32_t> hocc((size_t)Tc * N);
    std::vector<double> hC;
    std::vector<float> hC32;
    const bool f64 = ctx->run.precision == IESH_FP64;
    if (C) {
      if (f64)
        hC.assign((size_t)Tc * N * n_pad * 2, 0.0);
      else
        hC32.assign((size_t)Tc * N * n_pad * 2, 0.0f);
    }
    int tl = 0;
    for (int t = 0; t < T; ++t) {
      if (ctx->traj_class[t] != (int)ci) continue;
      for (int nu = 0; nu < nd; ++nu) {
        hx[(size_t)tl * nd + nu] = x[(size_t)t * nd + nu];
        hv[(size_t)tl * nd + nu] = v[(size_t)t * nd + nu];
      }
      if (occ) {
        for (int r = 0; r < N; ++r) {
          const int a = occ[(size_t)t * ctx->N_max + r];
          if (a < 0 || a >= n || (r && a <= occ[(size_t)t * ctx->N_max + r - 1]))
            return fail(ctx, IESH_EINVAL, "occupations must be sorted, distinct, in [0, n)");
          hocc[(size_t)tl * N + r] = a;
        }
      }
      if (C) {
        const double* src = C + (size_t)t * ctx->n_max * ctx->N_max * 2;
        for (int j = 0; j < N; ++j)
          for (int i = 0; i < n; ++i) {
            const size_t d = (((size_t)tl * N + j) * n_pad + i) * 2;
            const size_t s = ((size_t)j * n + i) * 2;
            if (f64) {
              hC[d] = src[s];
              hC[d + 1] = src[s + 1];
            } else {
              hC32[d] = (float)src[s];
              hC32[d + 1] = (float)src[s + 1];
            }
          }
      }
      ++tl;
    }
    HIPTRY(ctx, hipMemcpyAsync(c.x, hx.data(), hx.size() * sizeof(double), hipMemcpyHostToDevice,
                               ctx->stream));
    HIPTRY(ctx, hipMemcpyAsync(c.v, hv.data(), hv.size() * sizeof(double), hipMemcpyHostToDevice,
                               ctx->stream));
    if (occ)
      HIPTRY(ctx, hipMemcpyAsync(c.occ, hocc.data(), hocc.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, ctx->stream));
    if (C) {
      if (f64)
        HIPTRY(ctx, hipMemcpyAsync(c.C64, hC.data(), hC.size() * sizeof(double),
                                   hipMemcpyHostToDevice, ctx->stream));
      else
        HIPTRY(ctx, hipMemcpyAsync(c.C32, hC32.data(), hC32.size() * sizeof(float),
                                   hipMemcpyHostToDevice, ctx->stream));
    }
    HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  }
  return IESH_OK;
}

int reset_traj_words(iesh_ctx* ctx) {
  for (auto& c : ctx->cls) {
    HIPTRY(ctx, hipMemsetAsync(c.status, 0, c.n_traj * sizeof(int32_t), ctx->stream));
    HIPTRY(ctx, hipMemsetAsync(c.nsteps, 0, c.n_traj * sizeof(int64_t), ctx->stream));
    if (c.defect) HIPTRY(ctx, hipMemsetAsync(c.defect, 0, c.n_traj * sizeof(double), ctx->stream));
  }
  HIPTRY(ctx, hipMemsetAsync(&ctx->cnt->n_events, 0, sizeof(int64_t), ctx->stream));
  HIPTRY(ctx, hipMemsetAsync(&ctx->cnt->defect_max_bits, 0, 2 * sizeof(int64_t), ctx->stream));
  return IESH_OK;
}

// Slots back in upload order (slot = home index), every slot live.
int reset_perm(iesh_ctx* ctx) {
  for (size_t ci = 0; ci < ctx->cls.size(); ++ci) {
    ClassDev& c = ctx->cls[ci];
    auto& sh = ctx->slot_home[ci];
    auto& hs = ctx->home_slot[ci];
    for (int s = 0; s < c.n_traj; ++s) sh[s] = hs[s] = s;
    if (c.n_traj) {
      HIPTRY(ctx, hipMemcpyAsync(c.home, sh.data(), c.n_traj * sizeof(int32_t),
                                 hipMemcpyHostToDevice, ctx->stream));
      HIPTRY(ctx, hipMemcpyAsync(c.stepcap, ctx->caps_home[ci].data(), c.n_traj * sizeof(int64_t),
                                 hipMemcpyHostToDevice, ctx->stream));
      // every trajectory restarts its clock at the largest step
      std::vector<double> ck(2 * (size_t)c.n_traj);
      for (int s = 0; s < c.n_traj; ++s) {
        ck[2 * (size_t)s] = c.dt0;
        ck[2 * (size_t)s + 1] = 0.0;
      }
      HIPTRY(ctx, hipMemcpyAsync(c.clock, ck.data(), ck.size() * sizeof(double), hipMemcpyHostToDevice,
                                 ctx->stream));
      HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
    }
    if (c.live) {
      const int32_t nl = c.n_traj;
      HIPTRY(ctx, hipMemcpyAsync(c.live, &nl, sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
      HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
    }
    c.n_live = c.n_traj;
    ctx->live_host[ci] = c.n_traj;
  }
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  return IESH_OK;
}

// Slot order and live counts of the classes after device-side compaction
// (for the calls that address trajectories by their global index).
int refresh_perm(iesh_ctx* ctx) {
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  for (size_t ci = 0; ci < ctx->cls.size(); ++ci) {
    ClassDev& c = ctx->cls[ci];
    if (!c.n_traj || !ctx->spare[ci].dst) continue;
    int32_t nl = 0;
    HIPTRY(ctx, hipMemcpy(&nl, c.live, sizeof(int32_t), hipMemcpyDeviceToHost));
    auto& sh = ctx->slot_home[ci];
    HIPTRY(ctx, hipMemcpy(sh.data(), c.home, c.n_traj * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int sl = 0; sl < c.n_traj; ++sl) ctx->home_slot[ci][sh[sl]] = sl;
    ctx->live_host[ci] = nl;
  }
  return IESH_OK;
}

// The non-empty classes of one kind (arrowhead or dense) in sets of at most
// kFuseMax for the fused launches, largest first in each set; block ranges
// cover every slot of a class (the kernels skip slots past the live count).
std::vector<ClassSet> class_sets(const iesh_ctx* ctx, bool dense) {
  std::vector<int> idx;
  for (size_t ci = 0; ci < ctx->cls.size(); ++ci)
    if (ctx->cls[ci].n_traj && ((ctx->cls[ci].Gd != nullptr) == dense)) idx.push_back((int)ci);
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int a, int b) { return ctx->cls[a].md.n_pad > ctx->cls[b].md.n_pad; });
  std::vector<ClassSet> sets;
  for (size_t i = 0; i < idx.size(); i += kFuseMax) {
    ClassSet set{};
    set.n = 0;
    set.first[0] = 0;
    for (size_t j = i; j < idx.size() && j < i + kFuseMax; ++j) {
      set.c[set.n] = ctx->cls[idx[j]];
      set.first[set.n + 1] = set.first[set.n] + ctx->cls[idx[j]].n_live;
      ++set.n;
    }
    sets.push_back(set);
  }
  return sets;
}

// Device-side compaction of every class that has spare arrays.
int enqueue_compact(iesh_ctx* ctx) {
  for (size_t ci = 0; ci < ctx->cls.size(); ++ci) {
    ClassDev& c = ctx->cls[ci];
    if (!c.n_traj || !ctx->spare[ci].dst) continue;
    HIPTRY(ctx, launch_compact(c, ctx->spare[ci], ctx->run.precision, ctx->stream));
  }
  return IESH_OK;
}

int set_counters(iesh_ctx* ctx, int64_t run_step0, int64_t record_every) {
  // step, run_step0 are the first two fields; record_every the fourth
  const int64_t head[2] = {ctx->step, run_step0};
  HIPTRY(ctx, hipMemcpyAsync(ctx->cnt, head, sizeof(head), hipMemcpyHostToDevice, ctx->stream));
  HIPTRY(ctx, hipMemcpyAsync(&ctx->cnt->record_every, &record_every, sizeof(int64_t),
                             hipMemcpyHostToDevice, ctx->stream));
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  return IESH_OK;
}

hipEvent_t next_event(iesh_ctx* ctx) {
  if (ctx->ev_used == ctx->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->ev_pool.push_back(e);
  }
  return ctx->ev_pool[ctx->ev_used++];
}

// Launch `fn` bracketed by timing events when timing is on.
template <typename F>
hipError_t timed(iesh_ctx* ctx, int timer, F fn) {
  if (!ctx->timing) return fn();
  const size_t i0 = ctx->ev_used;
  hipEvent_t a = next_event(ctx);
  if (!a) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, ctx->stream);
  if (e != hipSuccess) return e;
  e = fn();
  if (e != hipSuccess) return e;
  hipEvent_t b = next_event(ctx);
  if (!b) return hipErrorOutOfMemory;
  e = hipEventRecord(b, ctx->stream);
  ctx->ev_marks.push_back({timer, i0});
  return e;
}

// Kernel sequence of one step for every class.  The eigen-solves of the
// arrowhead classes run in one launch whose blocks cover every class, largest
// class first, so that the small classes fill the compute units behind the
// large ones; so does the no-hop bound.  Propagation, ratios and Loewdin
// steps are per class (their register and LDS shapes depend on n and N).
// Every kernel reads the live-slot count of its class from the device.
int enqueue_step(iesh_ctx* ctx, int record) {
  const iesh_run_desc& r = ctx->run;
  hipStream_t s = ctx->stream;
  Counters* cnt = ctx->cnt;
  const int S = r.elec_substeps;
  const std::vector<ClassSet> arrow = class_sets(ctx, false), dense = class_sets(ctx, true);
  auto eig = [&](int sub, int nsub) -> int {
    for (const ClassSet& set : arrow)
      HIPTRY(ctx, timed(ctx, IESH_TIMER_EIG,
                        [&] { return launch_eig_fused(set, r.dt, r.precision, cnt, s, sub, nsub); }));
    for (auto& c : ctx->cls)
      if (c.n_traj && c.Gd)
        HIPTRY(ctx, timed(ctx, IESH_TIMER_EIG, [&] { return launch_dense_step(c, r.dt, cnt, s, sub, nsub); }));
    return IESH_OK;
  };
  auto prop = [&]() -> int {
    for (auto& c : ctx->cls)
      if (c.n_traj) HIPTRY(ctx, timed(ctx, IESH_TIMER_PROP, [&] { return launch_prop(c, r.precision, s); }));
    return IESH_OK;
  };
  int rc;
  if (S <= 1) {
    if ((rc = eig(-1, 1)) || (rc = prop())) return rc;
  } else {
    // electronic sub-steps: a propagator and a propagation each, then the end point
    for (int j = 0; j < S; ++j)
      if ((rc = eig(j, S)) || (rc = prop())) return rc;
    if ((rc = eig(-2, S))) return rc;
  }
  for (const auto* sets : {&arrow, &dense})
    for (const ClassSet& set : *sets)
      HIPTRY(ctx, timed(ctx, IESH_TIMER_FILTER, [&] {
               return launch_filter_fused(set, r.dt, r.seed, cnt, record, r.exit_enabled, r.exit_x,
                                          r.max_steps, r.precision, s);
             }));
  for (auto& c : ctx->cls) {
    if (c.n_traj == 0) continue;
    HIPTRY(ctx, timed(ctx, IESH_TIMER_HOP, [&] {
             return launch_hop(c, r.dt, r.seed, cnt, ctx->events, 0, 0, c.n_traj, record,
                               r.exit_enabled, r.exit_x, r.max_steps, r.precision, s);
           }));
    if (r.precision == IESH_MIXED && r.lowdin_every > 0)
      HIPTRY(ctx, timed(ctx, IESH_TIMER_LOWDIN,
                        [&] { return launch_lowdin(c, cnt, r.lowdin_every, c.low, s); }));
  }
  HIPTRY(ctx, launch_advance(ctx->cnt, ctx->stream));
  return IESH_OK;
}

// ---- adjoint along prescribed paths ----------------------------------------
template <typename T>
int adj_alloc(iesh_ctx* ctx, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return IESH_OK;
  void* q = nullptr;
  const size_t bytes = count * sizeof(T);
  if (hipMalloc(&q, bytes) != hipSuccess)
    return fail(ctx, IESH_ENOMEM, "hipMalloc failed (adjoint): " + std::to_string(bytes) + " bytes");
  ctx->adj_allocs.push_back(q);
  if (hipMemsetAsync(q, 0, bytes, ctx->stream) != hipSuccess)
    return fail(ctx, IESH_EDEVICE, "hipMemsetAsync failed");
  *p = reinterpret_cast<T*>(q);
  return IESH_OK;
}

void adj_release(iesh_ctx* ctx) {
  (void)hipStreamSynchronize(ctx->stream);
  for (void* p : ctx->adj_allocs) (void)hipFree(p);
  ctx->adj_allocs.clear();
  ctx->adj.assign(ctx->cls.size(), iesh_ctx::AdjClass{});
  ctx->adj_path = ctx->adj_loss = ctx->adj_w = ctx->adj_grad = nullptr;
  ctx->adj_forward_done = ctx->adj_backward_bufs = false;
}

// The class with the prescribed path attached, at step n.
ClassDev on_path(const iesh_ctx* ctx, const ClassDev& c, int n) {
  ClassDev cc = c;
  cc.path = ctx->adj_path;
  cc.path_len = ctx->adj_steps + 1;
  cc.path_n = n;
  return cc;
}

// One forward step along the path: eigen-solves, propagation of cc.C64.
int adj_step(iesh_ctx* ctx, const ClassDev& cc) {
  HIPTRY(ctx, timed(ctx, IESH_TIMER_ADJ_EIG,
                    [&] { return launch_eig_step(cc, ctx->run.dt, ctx->cnt, ctx->stream); }));
  HIPTRY(ctx, timed(ctx, IESH_TIMER_ADJ_PROP, [&] { return launch_prop(cc, IESH_FP64, ctx->stream); }));
  return IESH_OK;
}

}  // namespace

extern "C" {

int iesh_version(int* major, int* minor, int* patch) {
  if (major) *major = 0;
  if (minor) *minor = 1;
  if (patch) *patch = 0;
  return IESH_OK;
}

// reason of the last failed iesh_create on this thread (no context exists then)
thread_local std::string g_create_err;

const char* iesh_last_error(const iesh_ctx* ctx) {
  if (ctx) return ctx->err.c_str();
  return g_create_err.empty() ? "null context" : g_create_err.c_str();
}

int iesh_eigh_batched(const double* H, int32_t n, int32_t batch, double* lam, double* Q,
                      int32_t* sweeps, int32_t mem_kind, void* hip_stream) {
  g_create_err.clear();
  auto bad = [](const char* why) {
    g_create_err = why;
    return IESH_EINVAL;
  };
  if (n < 1 || n > IESH_JACOBI_MAX_N) return bad("eigh: n out of range [1, IESH_JACOBI_MAX_N]");
  if (batch < 0) return bad("eigh: batch must be >= 0");
  if (mem_kind != IESH_MEM_HOST && mem_kind != IESH_MEM_DEVICE) return bad("eigh: unknown mem_kind");
  if (batch == 0) return IESH_OK;
  if (!H || !lam || !Q) return bad("eigh: H, lam and Q must be given");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  auto dev_err = [](const std::string& why) {
    g_create_err = "eigh: " + why;
    return IESH_EDEVICE;
  };
  // global workspace for orders beyond the LDS limit
  const size_t nwork = jacobi_work_elems(n, batch);
  double* work = nullptr;
  if (nwork && hipMalloc(&work, nwork * sizeof(double)) != hipSuccess) {
    g_create_err = "eigh: device allocation failed";
    return IESH_ENOMEM;
  }
  if (mem_kind == IESH_MEM_DEVICE) {
    hipError_t e = launch_jacobi(H, n, batch, lam, Q, sweeps, work, st);
    if (e == hipSuccess && work) e = hipStreamSynchronize(st);
    (void)hipFree(work);
    if (e != hipSuccess) return dev_err(hipGetErrorString(e));
    return IESH_OK;
  }
  // host arrays: device copies for the call
  const size_t nm = (size_t)batch * n * n, nl = (size_t)batch * n;
  double *dH = nullptr, *dlam = nullptr, *dQ = nullptr;
  int32_t* dsw = nullptr;
  auto release = [&] {
    (void)hipFree(dH);
    (void)hipFree(dlam);
    (void)hipFree(dQ);
    (void)hipFree(dsw);
    (void)hipFree(work);
  };
  if (hipMalloc(&dH, nm * sizeof(double)) != hipSuccess ||
      hipMalloc(&dlam, nl * sizeof(double)) != hipSuccess ||
      hipMalloc(&dQ, nm * sizeof(double)) != hipSuccess ||
      (sweeps && hipMalloc(&dsw, batch * sizeof(int32_t)) != hipSuccess)) {
    release();
    g_create_err = "eigh: device allocation failed";
    return IESH_ENOMEM;
  }
  hipError_t e = hipMemcpyAsync(dH, H, nm * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_jacobi(dH, n, batch, dlam, dQ, dsw, work, st);
  if (e == hipSuccess) e = hipMemcpyAsync(lam, dlam, nl * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(Q, dQ, nm * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && sweeps)
    e = hipMemcpyAsync(sweeps, dsw, batch * sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  release();
  if (e != hipSuccess) return dev_err(hipGetErrorString(e));
  return IESH_OK;
}

int iesh_discretize(int32_t kind, int32_t M, double a, double b, double eps_f, double* eps,
                    double* w) {
  return discretize(kind, M, a, b, eps_f, eps, w);
}

int iesh_bath(const iesh_bath_desc* desc, double* eps, double* w, int32_t* lead, int32_t* n_below) {
  if (!desc) return IESH_EINVAL;
  return bath_levels(*desc, eps, w, lead, n_below);
}

int iesh_destroy(iesh_ctx* ctx) {
  if (!ctx) return IESH_OK;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  free_graph(ctx);
  for (auto& a : ctx->allocations) (void)hipFree(a.first);
  for (void* p : ctx->adj_allocs) (void)hipFree(p);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return IESH_OK;
}

int iesh_create(const iesh_model_desc* models, int32_t n_models, const int32_t* traj_model,
                const iesh_run_desc* run, void* hip_stream, iesh_ctx** out) {
  if (!out) return IESH_EINVAL;
  *out = nullptr;
  if (!models || n_models < 1 || !run) return IESH_EINVAL;
  iesh_ctx* ctx = new (std::nothrow) iesh_ctx();
  if (!ctx) return IESH_ENOMEM;
  g_create_err.clear();
  auto bail = [&](int code) {
    // keep the message for iesh_last_error(NULL)
    g_create_err = ctx->err;
    iesh_destroy(ctx);
    std::fprintf(stderr, "iesh_create: %s\n", g_create_err.c_str());
    return code;
  };
  ctx->run = *run;
  const iesh_run_desc& r = ctx->run;
  // every argument check comes before the first device call
  if (r.n_traj < 1) return (fail(ctx, IESH_EINVAL, "n_traj must be >= 1"), bail(IESH_EINVAL));
  if (!(r.dt > 0.0)) return (fail(ctx, IESH_EINVAL, "dt must be > 0"), bail(IESH_EINVAL));
  if (!(r.kT >= 0.0)) return (fail(ctx, IESH_EINVAL, "kT must be >= 0"), bail(IESH_EINVAL));
  if (r.precision != IESH_FP64 && r.precision != IESH_MIXED)
    return (fail(ctx, IESH_EINVAL, "unknown precision"), bail(IESH_EINVAL));
  if (r.lowdin_every < 0 || r.record_every < 0)
    return (fail(ctx, IESH_EINVAL, "negative cadence"), bail(IESH_EINVAL));
  for (int m = 0; m < n_models; ++m) {
    std::string why;
    if (!validate_model(models[m], why))
      return (fail(ctx, IESH_EINVAL, "model " + std::to_string(m) + ": " + why), bail(IESH_EINVAL));
  }
  if (r.compact_every < 0) return (fail(ctx, IESH_EINVAL, "negative cadence"), bail(IESH_EINVAL));
  if (r.elec_substeps < 0 || r.elec_substeps > 64)
    return (fail(ctx, IESH_EINVAL, "elec_substeps out of range [0, 64]"), bail(IESH_EINVAL));
  if (ctx->run.elec_substeps == 0) ctx->run.elec_substeps = 1;
  if (r.eig_max_iter < 0 || r.eig_max_iter > 128)
    return (fail(ctx, IESH_EINVAL, "eig_max_iter out of range [0, 128]"), bail(IESH_EINVAL));
  if (r.dt_levels < 0 || r.dt_levels > 30)
    return (fail(ctx, IESH_EINVAL, "dt_levels out of range [0, 30]"), bail(IESH_EINVAL));
  if (r.dt_levels > 0 && !(r.hop_gmax > 0.0 && std::isfinite(r.hop_gmax)))
    return (fail(ctx, IESH_EINVAL, "an adaptive step needs hop_gmax > 0"), bail(IESH_EINVAL));
  if (!std::isfinite(r.bias))
    return (fail(ctx, IESH_EINVAL, "bias must be finite"), bail(IESH_EINVAL));
  if (r.bias != 0.0) {
    if (!(r.kT > 0.0))
      return (fail(ctx, IESH_EINVAL, "a bias needs kT > 0"), bail(IESH_EINVAL));
    for (int m = 0; m < n_models; ++m)
      if (!models[m].lead)
        return (fail(ctx, IESH_EINVAL, "a bias needs lead labels in every model"), bail(IESH_EINVAL));
  }
  ctx->traj_class.assign(r.n_traj, 0);
  ctx->traj_local.assign(r.n_traj, 0);
  std::vector<int> count(n_models, 0);
  for (int t = 0; t < r.n_traj; ++t) {
    const int m = traj_model ? traj_model[t] : 0;
    if (m < 0 || m >= n_models)
      return (fail(ctx, IESH_EINVAL, "traj_model out of range"), bail(IESH_EINVAL));
    ctx->traj_class[t] = m;
    ctx->traj_local[t] = count[m]++;
  }
  const int ndof0 = model_ndof(models[0]);
  for (int m = 1; m < n_models; ++m)
    if (model_ndof(models[m]) != ndof0)
      return (fail(ctx, IESH_EINVAL, "all models of a context need the same n_dof"), bail(IESH_EINVAL));
  if (r.exit_dof < 0 || r.exit_dof >= ndof0)
    return (fail(ctx, IESH_EINVAL, "exit_dof out of range [0, n_dof)"), bail(IESH_EINVAL));
  if (r.hop_filter_off != 0 && r.hop_filter_off != 1)
    return (fail(ctx, IESH_EINVAL, "hop_filter_off must be 0 or 1"), bail(IESH_EINVAL));

  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (!ctx->stream) {
    // the step loop is captured into a graph, which needs a non-null stream
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess)
      return (fail(ctx, IESH_EDEVICE, "stream creation failed"), bail(IESH_EDEVICE));
    ctx->own_stream = true;
  }
  (void)hipGetDevice(&ctx->device);
  if (hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device) !=
          hipSuccess ||
      ctx->n_cu < 1)
    ctx->n_cu = 256;
  int rc = dalloc(ctx, &ctx->cnt, 1);
  if (rc) return bail(rc);
  rc = dalloc(ctx, &ctx->events, (size_t)IESH_EVENT_CAP);
  if (rc) return bail(rc);
  ctx->live_host.assign(n_models, 0);
  ctx->cls.resize(n_models);
  ctx->members.assign(n_models, {});
  ctx->slot_home.assign(n_models, {});
  ctx->home_slot.assign(n_models, {});
  ctx->spare.assign(n_models, CompactBufs{});
  ctx->caps_home.assign(n_models, {});
  for (int t = 0; t < r.n_traj; ++t) ctx->members[ctx->traj_class[t]].push_back(t);
  for (int m = 0; m < n_models; ++m) {
    const iesh_model_desc& d = models[m];
    ClassDev& c = ctx->cls[m];
    c.md.kind = d.kind;
    c.md.M = d.n_bath;
    c.md.M_red = d.n_bath;
    c.md.eig_iter = r.eig_max_iter > 0 ? r.eig_max_iter : 128;
    c.md.expand = nullptr;
    c.md.lead0 = nullptr;
    c.md.n = d.n_bath + 1;
    c.md.n_pad = round16(c.md.n);
    c.md.N = d.n_elec;
    c.md.mass = d.mass;
    c.md.Gamma = d.Gamma;
    for (int q = 0; q < 16; ++q) c.md.p[q] = d.params[q];
    c.md.ndof = model_ndof(d);
    if (m == 0) ctx->ndof = c.md.ndof;
    if (c.md.ndof != ctx->ndof)
      return (fail(ctx, IESH_EINVAL, "all models of a context need the same n_dof"), bail(IESH_EINVAL));
    for (int nu = 0; nu < kMaxDof; ++nu) {
      c.md.mass_dof[nu] = 0.0;
      for (int q = 0; q < 6; ++q) c.md.dofp[nu][q] = 0.0;
    }
    if (d.kind == IESH_MODEL_MULTI_DOF) {
      c.md.mass = d.dof[0];
      for (int nu = 0; nu < c.md.ndof; ++nu) {
        c.md.mass_dof[nu] = d.dof[7 * nu];
        for (int q = 0; q < 6; ++q) c.md.dofp[nu][q] = d.dof[7 * nu + 1 + q];
      }
    } else {
      c.md.mass_dof[0] = d.mass;
    }
    c.exit_dof = r.exit_dof;
    // the mixed path measures the orthonormality defect the no-hop bound
    // needs only at its Loewdin steps: without them it evaluates the ratios
    // at every step
    c.exact_hops = r.hop_filter_off || (r.precision == IESH_MIXED && r.lowdin_every == 0);
    c.dt0 = r.dt;
    c.gmax = r.hop_gmax;
    c.dt_levels = r.dt_levels;
    c.n_traj = count[m];
    c.n_live = count[m];
    ctx->slot_home[m].assign(count[m], 0);
    ctx->home_slot[m].assign(count[m], 0);
    ctx->caps_home[m].assign(count[m], 0);
    ctx->n_max = std::max(ctx->n_max, c.md.n);
    ctx->N_max = std::max(ctx->N_max, c.md.N);
    choose_slabs(c, r.precision);
    const int T = c.n_traj, n_pad = c.md.n_pad, N = c.md.N, M = c.md.M;
    if (T == 0) continue;
    const int nd = c.md.ndof;
    const bool dense = d.kind == IESH_MODEL_DENSE;
    if ((rc = dalloc(ctx, &c.eps, M)) || (rc = dalloc(ctx, &c.vbar, M)) ||
        (rc = dalloc(ctx, &c.x, (size_t)T * nd)) || (rc = dalloc(ctx, &c.v, (size_t)T * nd)) ||
        (rc = dalloc(ctx, &c.F, (size_t)T * nd)) ||
        (rc = dalloc(ctx, &c.occ, (size_t)T * N)) || (rc = dalloc(ctx, &c.status, T)) ||
        (rc = dalloc(ctx, &c.gtraj, T)) || (rc = dalloc(ctx, &c.nsteps, T)) ||
        (rc = dalloc(ctx, &c.home, T)) || (rc = dalloc(ctx, &c.stepcap, T)) ||
        (rc = dalloc(ctx, &c.lam, (size_t)T * n_pad)) || (rc = dalloc(ctx, &c.q0, (size_t)T * n_pad)) ||
        (rc = dalloc(ctx, &c.lam_mid, (size_t)T * n_pad)) ||
        (rc = dalloc(ctx, &c.geo, (size_t)T * kGeoStride)) ||
        (rc = dalloc(ctx, &c.cheb, (size_t)T * kChebStride)) ||
        (rc = dalloc(ctx, &c.gbuf, (size_t)T * N * n_pad)) ||
        (rc = dalloc(ctx, &c.rown, (size_t)T * ((N + 7) / 8) * n_pad)) ||
        (rc = dalloc(ctx, &c.clock, (size_t)2 * T)) ||
        (rc = dalloc(ctx, &c.hopq, (size_t)3 + T)) || (rc = dalloc(ctx, &c.live, 1)) ||
        (rc = dalloc(ctx, &c.work, 2)))
      return bail(rc);
    if (hop_needs_scratch(c) && (rc = dalloc(ctx, &c.hopx, (size_t)T * N * N)))
      return bail(rc);
    if (!dense && ((rc = dalloc(ctx, &c.root_tau, (size_t)T * 2 * n_pad)) ||
                   (rc = dalloc(ctx, &c.root_org, (size_t)T * n_pad)) ||
                   (rc = dalloc(ctx, &c.root_geo, (size_t)T * 4))))
      return bail(rc);
    if (dense) {
      double *h0 = nullptr, *h1 = nullptr;
      if ((rc = dalloc(ctx, &h0, (size_t)n_pad * n_pad)) || (rc = dalloc(ctx, &h1, (size_t)n_pad * n_pad)) ||
          (rc = dalloc(ctx, &c.Gd, (size_t)T * n_pad * n_pad)) ||
          (rc = dalloc(ctx, &c.Qw, (size_t)T * n_pad * n_pad)))
        return bail(rc);
      const int n = c.md.n;
      // padded to n_pad and symmetrised (validation bounds the asymmetry by
      // 1e-14 of the largest element): the kernels read either triangle
      std::vector<double> pad((size_t)2 * n_pad * n_pad, 0.0);
      for (int h = 0; h < 2; ++h) {
        const double* H = d.dense + (size_t)h * n * n;
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j)
            pad[(size_t)h * n_pad * n_pad + (size_t)i * n_pad + j] =
                0.5 * (H[(size_t)i * n + j] + H[(size_t)j * n + i]);
      }
      if (hipMemcpyAsync(h0, pad.data(), (size_t)n_pad * n_pad * sizeof(double), hipMemcpyHostToDevice,
                         ctx->stream) != hipSuccess ||
          hipMemcpyAsync(h1, pad.data() + (size_t)n_pad * n_pad, (size_t)n_pad * n_pad * sizeof(double),
                         hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
          hipStreamSynchronize(ctx->stream) != hipSuccess)
        return (fail(ctx, IESH_EDEVICE, "upload of the dense model failed"), bail(IESH_EDEVICE));
      c.H0 = h0;
      c.H1 = h1;
    }
    if (r.compact_every > 0) {
      CompactBufs& b = ctx->spare[m];
      const size_t csz = (size_t)T * N * n_pad * 2;
      if ((rc = dalloc(ctx, &b.x, (size_t)T * nd)) || (rc = dalloc(ctx, &b.v, (size_t)T * nd)) ||
          (rc = dalloc(ctx, &b.F, (size_t)T * nd)) ||
          (rc = dalloc(ctx, &b.status, T)) || (rc = dalloc(ctx, &b.gtraj, T)) ||
          (rc = dalloc(ctx, &b.home, T)) || (rc = dalloc(ctx, &b.nsteps, T)) ||
          (rc = dalloc(ctx, &b.stepcap, T)) ||
          (rc = dalloc(ctx, &b.occ, (size_t)T * N)) || (rc = dalloc(ctx, &b.dst, T)) ||
          (rc = dalloc(ctx, &b.clock, (size_t)2 * T)) ||
          (rc = dalloc(ctx, &b.n_active, 1)))
        return bail(rc);
      if (r.precision == IESH_FP64) {
        double* p = nullptr;
        if ((rc = dalloc(ctx, &p, csz))) return bail(rc);
        b.C = p;
      } else {
        float* p = nullptr;
        if ((rc = dalloc(ctx, &p, csz))) return bail(rc);
        b.C = p;
      }
    }
    if (r.precision == IESH_FP64) {
      if ((rc = dalloc(ctx, &c.C64, (size_t)T * N * n_pad * 2)) ||
          (rc = dalloc(ctx, &c.Bt, (size_t)T * n_pad * n_pad)))
        return bail(rc);
    } else {
      if ((rc = dalloc(ctx, &c.C32, (size_t)T * N * n_pad * 2)) ||
          (rc = dalloc(ctx, &c.Bt32, (size_t)T * n_pad * n_pad)) ||
          (rc = dalloc(ctx, &c.low, lowdin_scratch_elems(c))) ||
          (rc = dalloc(ctx, &c.defect, (size_t)T)))
        return bail(rc);
    }
    if (hipError_t e = prop_prepare(c, r.precision); e != hipSuccess)
      return (fail(ctx, IESH_EDEVICE, std::string("propagation LDS attribute: ") +
                                         hipGetErrorString(e)),
              bail(IESH_EDEVICE));
    std::vector<int32_t> gt;
    for (int t = 0; t < r.n_traj; ++t)
      if (ctx->traj_class[t] == m) gt.push_back(t);
    if (dense) {  // no bath poles: the eigen-solve is the dense one
      if (hipMemcpyAsync(c.gtraj, gt.data(), T * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream) ||
          hipStreamSynchronize(ctx->stream))
        return (fail(ctx, IESH_EDEVICE, "upload of model data failed"), bail(IESH_EDEVICE));
      continue;
    }
    // poles of the secular function: groups of equal bath energies, each
    // with the summed weight (V^2 of the coupled combination)
    const BathPoles bp = bath_poles(d);
    const int Mr = (int)bp.eps.size();
    std::vector<double> vb(Mr);
    for (int q = 0; q < Mr; ++q) vb[q] = std::sqrt(d.Gamma * bp.w[q] / (2.0 * M_PI));
    int32_t* expand = nullptr;
    double* lead0 = nullptr;
    if (Mr < M && (rc = dalloc(ctx, &expand, (size_t)c.md.n))) return bail(rc);
    if (d.lead && (rc = dalloc(ctx, &lead0, (size_t)2 * Mr))) return bail(rc);
    if (hipMemcpyAsync(c.eps, bp.eps.data(), Mr * sizeof(double), hipMemcpyHostToDevice, ctx->stream) ||
        hipMemcpyAsync(c.vbar, vb.data(), Mr * sizeof(double), hipMemcpyHostToDevice, ctx->stream) ||
        hipMemcpyAsync(c.gtraj, gt.data(), T * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream) ||
        (expand && hipMemcpyAsync(expand, bp.expand.data(), c.md.n * sizeof(int32_t),
                                  hipMemcpyHostToDevice, ctx->stream)) ||
        (lead0 && hipMemcpyAsync(lead0, bp.lead0.data(), 2 * Mr * sizeof(double),
                                 hipMemcpyHostToDevice, ctx->stream)) ||
        hipStreamSynchronize(ctx->stream))
      return (fail(ctx, IESH_EDEVICE, "upload of model data failed"), bail(IESH_EDEVICE));
    c.md.M_red = Mr;
    c.md.expand = expand;
    c.md.lead0 = lead0;
  }
  if (hipStreamSynchronize(ctx->stream) != hipSuccess)
    return (fail(ctx, IESH_EDEVICE, "device synchronisation failed"), bail(IESH_EDEVICE));
  for (auto& c : ctx->cls)
    if (c.n_traj && autotune_slabs(ctx, c)) return bail(IESH_EDEVICE);
  // the ratio kernel is persistent over its queue: as many work-groups as
  // are resident at once
  for (auto& c : ctx->cls)
    if (c.n_traj) c.hop_groups = hop_resident_groups(c, r.precision, ctx->n_cu);
  if (set_counters(ctx, 0, 0)) return bail(IESH_EDEVICE);
  if (reset_perm(ctx)) return bail(IESH_EDEVICE);
  *out = ctx;
  return IESH_OK;
}

int iesh_set_step_caps(iesh_ctx* ctx, const int64_t* caps) {
  if (!ctx || !caps) return IESH_EINVAL;
  for (size_t ci = 0; ci < ctx->cls.size(); ++ci) {
    ClassDev& c = ctx->cls[ci];
    if (!c.n_traj) continue;
    std::vector<int64_t> h(c.n_traj);
    for (int hm = 0; hm < c.n_traj; ++hm) {
      const int64_t v = caps[ctx->members[ci][hm]];
      if (v < 0) return fail(ctx, IESH_EINVAL, "negative step cap");
      h[ctx->home_slot[ci][hm]] = v;
      ctx->caps_home[ci][hm] = v;
    }
    HIPTRY(ctx, hipMemcpyAsync(c.stepcap, h.data(), h.size() * sizeof(int64_t),
                               hipMemcpyHostToDevice, ctx->stream));
  }
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  return IESH_OK;
}

int iesh_class_info(const iesh_ctx* ctx, int32_t cls, int32_t* info) {
  if (!ctx || !info || cls < 0 || cls >= (int)ctx->cls.size()) return IESH_EINVAL;
  const ClassDev& c = ctx->cls[cls];
  info[0] = c.n_traj;
  info[1] = ctx->live_host[cls];
  info[2] = c.md.n;
  info[3] = c.md.N;
  info[4] = c.nct_max;
  info[5] = c.n_slabs;
  info[6] = c.md.n_pad;
  info[7] = 0;
  return IESH_OK;
}

int iesh_query_sizes(const iesh_ctx* ctx, iesh_sizes* out) {
  if (!ctx || !out) return IESH_EINVAL;
  out->n_traj = ctx->run.n_traj;
  out->n_models = (int32_t)ctx->cls.size();
  out->n_max = ctx->n_max;
  out->N_max = ctx->N_max;
  out->n_dof = ctx->ndof;
  out->reserved = 0;
  out->device_bytes = (int64_t)ctx->device_bytes;
  return IESH_OK;
}

int iesh_set_step(iesh_ctx* ctx, int64_t step) {
  if (!ctx || step < 0) return IESH_EINVAL;
  ctx->step = step;
  return set_counters(ctx, step, 0);
}

int iesh_get_step(const iesh_ctx* ctx, int64_t* step) {
  if (!ctx || !step) return IESH_EINVAL;
  *step = ctx->step;
  return IESH_OK;
}

static std::vector<double> host_copy_d(iesh_ctx* ctx, const double* p, size_t count, int mem_kind) {
  std::vector<double> h(count);
  if (mem_kind == IESH_MEM_DEVICE) {
    (void)hipMemcpy(h.data(), p, count * sizeof(double), hipMemcpyDeviceToHost);
  } else {
    std::memcpy(h.data(), p, count * sizeof(double));
  }
  (void)ctx;
  return h;
}

int iesh_set_state(iesh_ctx* ctx, const double* x, const double* v, const double* C,
                   const int32_t* occ, int32_t mem_kind) {
  if (!ctx || !x || !v || !C || !occ) return fail(ctx, IESH_EINVAL, "null state pointer");
  if (mem_kind != IESH_MEM_HOST && mem_kind != IESH_MEM_DEVICE)
    return fail(ctx, IESH_EINVAL, "mem_kind");
  const int T = ctx->run.n_traj;
  std::vector<double> hx, hv, hC;
  std::vector<int32_t> hocc;
  const size_t csize = (size_t)T * ctx->n_max * ctx->N_max * 2;
  if (mem_kind == IESH_MEM_DEVICE) {
    hx = host_copy_d(ctx, x, (size_t)T * ctx->ndof, mem_kind);
    hv = host_copy_d(ctx, v, (size_t)T * ctx->ndof, mem_kind);
    hC = host_copy_d(ctx, C, csize, mem_kind);
    hocc.resize((size_t)T * ctx->N_max);
    HIPTRY(ctx, hipMemcpy(hocc.data(), occ, hocc.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    x = hx.data();
    v = hv.data();
    C = hC.data();
    occ = hocc.data();
  }
  int rc = reset_perm(ctx);
  if (rc) return rc;
  if ((rc = upload_state(ctx, x, v, C, occ))) return rc;
  if ((rc = reset_traj_words(ctx))) return rc;
  for (auto& c : ctx->cls)
    if (c.n_traj)
      HIPTRY(ctx, c.Gd ? launch_dense_query(c, 0, c.n_traj, 1, ctx->stream) : launch_forces(c, ctx->stream));
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  return IESH_OK;
}

int iesh_init_thermal(iesh_ctx* ctx, const double* x, const double* v) {
  if (!ctx || !x || !v) return fail(ctx, IESH_EINVAL, "null pointer");
  int rc = reset_perm(ctx);
  if (rc) return rc;
  if ((rc = upload_state(ctx, x, v, nullptr, nullptr))) return rc;
  if ((rc = reset_traj_words(ctx))) return rc;
  for (auto& c : ctx->cls)
    if (c.n_traj)
      HIPTRY(ctx, c.Gd ? launch_dense_init_thermal(c, ctx->run.kT, ctx->run.seed, ctx->stream)
                       : launch_init_thermal(c, ctx->run.kT, ctx->run.bias, ctx->run.seed, ctx->stream));
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  return IESH_OK;
}

int iesh_get_state(iesh_ctx* ctx, double* x, double* v, double* C, int32_t* occ,
                   int32_t mem_kind) {
  if (!ctx) return IESH_EINVAL;
  if (mem_kind != IESH_MEM_HOST && mem_kind != IESH_MEM_DEVICE)
    return fail(ctx, IESH_EINVAL, "mem_kind");
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  const int T = ctx->run.n_traj;
  const size_t csize = (size_t)T * ctx->n_max * ctx->N_max * 2;
  const int nd = ctx->ndof;
  std::vector<double> hx((size_t)T * nd), hv((size_t)T * nd), hC(C ? csize : 0, 0.0);
  std::vector<int32_t> hocc(occ ? (size_t)T * ctx->N_max : 0, -1);
  for (size_t ci = 0; ci < ctx->cls.size(); ++ci) {
    ClassDev& c = ctx->cls[ci];
    const int Tc = c.n_traj, N = c.md.N, n = c.md.n, n_pad = c.md.n_pad;
    if (!Tc) continue;
    std::vector<double> cx((size_t)Tc * nd), cv((size_t)Tc * nd);
    std::vector<int32_t> cocc((size_t)Tc * N);
    HIPTRY(ctx, hipMemcpy(cx.data(), c.x, cx.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIPTRY(ctx, hipMemcpy(cv.data(), c.v, cv.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIPTRY(ctx, hipMemcpy(cocc.data(), c.occ, cocc.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<double> cC;
    if (C) {
      cC.resize((size_t)Tc * N * n_pad * 2);
      if (ctx->run.precision == IESH_FP64) {
        HIPTRY(ctx, hipMemcpy(cC.data(), c.C64, cC.size() * sizeof(double), hipMemcpyDeviceToHost));
      } else {
        std::vector<float> f(cC.size());
        HIPTRY(ctx, hipMemcpy(f.data(), c.C32, f.size() * sizeof(float), hipMemcpyDeviceToHost));
        for (size_t q = 0; q < f.size(); ++q) cC[q] = f[q];
      }
    }
    for (int sl = 0; sl < Tc; ++sl) {
      const int t = ctx->members[ci][ctx->slot_home[ci][sl]];
      const int tl = sl;
      for (int nu = 0; nu < nd; ++nu) {
        hx[(size_t)t * nd + nu] = cx[(size_t)tl * nd + nu];
        hv[(size_t)t * nd + nu] = cv[(size_t)tl * nd + nu];
      }
      if (occ)
        for (int r = 0; r < N; ++r) hocc[(size_t)t * ctx->N_max + r] = cocc[(size_t)tl * N + r];
      if (C) {
        double* dst = hC.data() + (size_t)t * ctx->n_max * ctx->N_max * 2;
        for (int j = 0; j < N; ++j)
          for (int i = 0; i < n; ++i) {
            const size_t s = (((size_t)tl * N + j) * n_pad + i) * 2;
            dst[((size_t)j * n + i) * 2] = cC[s];
            dst[((size_t)j * n + i) * 2 + 1] = cC[s + 1];
          }
      }
    }
  }
  auto put = [&](void* dst, const void* src, size_t bytes) -> int {
    if (!dst) return IESH_OK;
    if (mem_kind == IESH_MEM_DEVICE) {
      HIPTRY(ctx, hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    } else {
      std::memcpy(dst, src, bytes);
    }
    return IESH_OK;
  };
  int rc;
  if ((rc = put(x, hx.data(), hx.size() * sizeof(double)))) return rc;
  if ((rc = put(v, hv.data(), hv.size() * sizeof(double)))) return rc;
  if ((rc = put(C, hC.data(), hC.size() * sizeof(double)))) return rc;
  if ((rc = put(occ, hocc.data(), hocc.size() * sizeof(int32_t)))) return rc;
  return IESH_OK;
}

int iesh_step(iesh_ctx* ctx) {
  if (!ctx) return IESH_EINVAL;
  int rc = enqueue_step(ctx, 0);
  if (rc) return rc;
  ctx->step += 1;
  return IESH_OK;
}

int iesh_sync(iesh_ctx* ctx) {
  if (!ctx) return IESH_EINVAL;
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  return IESH_OK;
}

int iesh_run(iesh_ctx* ctx, int64_t n_steps, double* obs_out) {
  if (!ctx || n_steps < 0) return IESH_EINVAL;
  const iesh_run_desc& r = ctx->run;
  const int record = (obs_out && r.record_every > 0) ? 1 : 0;
  const int64_t n_rec = record ? n_steps / r.record_every : 0;
  if (record && n_rec > ctx->obs_records) {
    free_graph(ctx);  // observable pointers are captured in the graph
    for (auto& c : ctx->cls) {
      if (!c.n_traj) continue;
      dfree(ctx, c.obs);
      int rc = dalloc(ctx, &c.obs, (size_t)n_rec * c.n_traj * IESH_N_OBS);
      if (rc) return rc;
    }
    ctx->obs_records = n_rec;
  }
  if (record) {
    // records of trajectories that are frozen when they fall due stay NaN
    for (auto& c : ctx->cls)
      if (c.n_traj)
        HIPTRY(ctx, launch_fill(c.obs, (size_t)n_rec * c.n_traj * IESH_N_OBS, NAN, ctx->stream));
  }
  int rc = set_counters(ctx, ctx->step, record ? r.record_every : 0);
  if (rc) return rc;
  if (n_steps == 0) return IESH_OK;
  // chunks end where compaction is due
  int64_t left = n_steps;
  while (left > 0) {
    const int64_t chunk = r.compact_every > 0 ? std::min<int64_t>(left, r.compact_every) : left;
    if (ctx->timing) {
      // eager launches so that every kernel is bracketed by its own events
      for (int64_t k = 0; k < chunk; ++k) {
        rc = enqueue_step(ctx, record);
        if (rc) return rc;
        ctx->step += 1;
      }
    } else {
      if (ctx->graph_record != record) {
        free_graph(ctx);
        HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
        HIPTRY(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
        rc = enqueue_step(ctx, record);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->stream, &g);
        if (rc) {
          if (g) (void)hipGraphDestroy(g);
          return rc;
        }
        if (e != hipSuccess)
          return fail(ctx, IESH_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        ctx->graph = g;
        HIPTRY(ctx, hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0));
        ctx->graph_record = record;
      }
      for (int64_t k = 0; k < chunk; ++k) HIPTRY(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream));
      ctx->step += chunk;
    }
    left -= chunk;
    if (r.compact_every > 0) {
      // compaction on the device: no host round trip, no re-capture
      if (ctx->timing) {
        if ((rc = enqueue_compact(ctx))) return rc;
      } else {
        if (!ctx->compact_exec) {
          HIPTRY(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
          rc = enqueue_compact(ctx);
          hipGraph_t g = nullptr;
          hipError_t e = hipStreamEndCapture(ctx->stream, &g);
          if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
          }
          if (e != hipSuccess)
            return fail(ctx, IESH_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
          ctx->compact_graph = g;
          HIPTRY(ctx, hipGraphInstantiate(&ctx->compact_exec, g, nullptr, nullptr, 0));
        }
        HIPTRY(ctx, hipGraphLaunch(ctx->compact_exec, ctx->stream));
      }
    }
  }
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  if (r.compact_every > 0 && (rc = refresh_perm(ctx))) return rc;
  if (record) {
    const int T = r.n_traj;
    for (size_t ci = 0; ci < ctx->cls.size(); ++ci) {
      ClassDev& c = ctx->cls[ci];
      if (!c.n_traj) continue;
      std::vector<double> h((size_t)n_rec * c.n_traj * IESH_N_OBS);
      HIPTRY(ctx, hipMemcpy(h.data(), c.obs, h.size() * sizeof(double), hipMemcpyDeviceToHost));
      int tl = 0;
      for (int t = 0; t < T; ++t) {
        if (ctx->traj_class[t] != (int)ci) continue;
        for (int64_t q = 0; q < n_rec; ++q)
          for (int o = 0; o < IESH_N_OBS; ++o)
            obs_out[((size_t)q * T + t) * IESH_N_OBS + o] =
                h[((size_t)q * c.n_traj + tl) * IESH_N_OBS + o];
        ++tl;
      }
    }
  }
  return IESH_OK;
}

int iesh_hop_probs(iesh_ctx* ctx, int32_t traj0, int32_t ntraj, double* g_out, int32_t mem_kind) {
  if (!ctx || !g_out || traj0 < 0 || ntraj < 1 || traj0 + ntraj > ctx->run.n_traj)
    return fail(ctx, IESH_EINVAL, "trajectory range");
  const int stride = ctx->n_max * ctx->N_max;
  std::vector<double> host((size_t)ntraj * stride, 0.0);
  for (int q = 0; q < ntraj; ++q) {
    const int t = traj0 + q;
    ClassDev& c = ctx->cls[ctx->traj_class[t]];
    const int tl = ctx->home_slot[ctx->traj_class[t]][ctx->traj_local[t]];
    HIPTRY(ctx, c.Gd ? launch_dense_query(c, tl, 1, 0, ctx->stream) : launch_eig_query(c, tl, 1, ctx->stream));
    HIPTRY(ctx, launch_hop(c, ctx->run.dt, ctx->run.seed, ctx->cnt, ctx->events, 1, tl, 1, 0, 0,
                           0.0, 0, ctx->run.precision, ctx->stream));
    const int N = c.md.N, n = c.md.n, n_pad = c.md.n_pad;
    std::vector<double> g((size_t)N * n_pad);
    HIPTRY(ctx, hipMemcpyAsync(g.data(), c.gbuf + (size_t)tl * N * n_pad, g.size() * sizeof(double),
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int rr = 0; rr < N; ++rr)
      for (int b = 0; b < n; ++b) host[(size_t)q * stride + (size_t)rr * n + b] = g[(size_t)rr * n_pad + b];
  }
  if (mem_kind == IESH_MEM_DEVICE) {
    HIPTRY(ctx, hipMemcpy(g_out, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice));
  } else {
    std::memcpy(g_out, host.data(), host.size() * sizeof(double));
  }
  return IESH_OK;
}

int iesh_adiabatic(iesh_ctx* ctx, int32_t traj0, int32_t ntraj, double* lam_out, double* q0_out) {
  if (!ctx || traj0 < 0 || ntraj < 1 || traj0 + ntraj > ctx->run.n_traj)
    return fail(ctx, IESH_EINVAL, "trajectory range");
  for (int q = 0; q < ntraj; ++q) {
    const int t = traj0 + q;
    ClassDev& c = ctx->cls[ctx->traj_class[t]];
    const int tl = ctx->home_slot[ctx->traj_class[t]][ctx->traj_local[t]];
    HIPTRY(ctx, c.Gd ? launch_dense_query(c, tl, 1, 0, ctx->stream) : launch_eig_query(c, tl, 1, ctx->stream));
    const int n = c.md.n, n_pad = c.md.n_pad;
    std::vector<double> l(n_pad), qq(n_pad);
    HIPTRY(ctx, hipMemcpyAsync(l.data(), c.lam + (size_t)tl * n_pad, n_pad * sizeof(double),
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPTRY(ctx, hipMemcpyAsync(qq.data(), c.q0 + (size_t)tl * n_pad, n_pad * sizeof(double),
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int j = 0; j < n; ++j) {
      if (lam_out) lam_out[(size_t)q * ctx->n_max + j] = l[j];
      if (q0_out) q0_out[(size_t)q * ctx->n_max + j] = qq[j];
    }
  }
  return IESH_OK;
}

int iesh_traj_status(iesh_ctx* ctx, int32_t* status_out) {
  if (!ctx || !status_out) return IESH_EINVAL;
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  for (size_t ci = 0; ci < ctx->cls.size(); ++ci) {
    ClassDev& c = ctx->cls[ci];
    if (!c.n_traj) continue;
    std::vector<int32_t> s(c.n_traj);
    HIPTRY(ctx, hipMemcpy(s.data(), c.status, s.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int sl = 0; sl < c.n_traj; ++sl) status_out[ctx->members[ci][ctx->slot_home[ci][sl]]] = s[sl];
  }
  return IESH_OK;
}

int iesh_traj_clock(iesh_ctx* ctx, double* time_out, double* dt_out) {
  if (!ctx || (!time_out && !dt_out)) return IESH_EINVAL;
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  for (size_t ci = 0; ci < ctx->cls.size(); ++ci) {
    ClassDev& c = ctx->cls[ci];
    if (!c.n_traj) continue;
    std::vector<double> ck(2 * (size_t)c.n_traj);
    HIPTRY(ctx, hipMemcpy(ck.data(), c.clock, ck.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int sl = 0; sl < c.n_traj; ++sl) {
      const int g = ctx->members[ci][ctx->slot_home[ci][sl]];
      if (dt_out) dt_out[g] = ck[2 * (size_t)sl];
      if (time_out) time_out[g] = ck[2 * (size_t)sl + 1];
    }
  }
  return IESH_OK;
}

int iesh_events(iesh_ctx* ctx, iesh_event* out, int64_t cap, int64_t* count) {
  if (!ctx || !count || cap < 0) return IESH_EINVAL;
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  int64_t n = 0;
  HIPTRY(ctx, hipMemcpy(&n, &ctx->cnt->n_events, sizeof(int64_t), hipMemcpyDeviceToHost));
  *count = n;
  int64_t have = std::min<int64_t>(n, IESH_EVENT_CAP);
  if (out && cap > 0 && have > 0) {
    std::vector<iesh_event> ev(have);
    HIPTRY(ctx, hipMemcpy(ev.data(), ctx->events, have * sizeof(iesh_event), hipMemcpyDeviceToHost));
    std::sort(ev.begin(), ev.end(), [](const iesh_event& a, const iesh_event& b) {
      return a.step != b.step ? a.step < b.step : a.traj < b.traj;
    });
    if (n > IESH_EVENT_CAP) {
      // which events of the step that overflowed the log got a slot depends
      // on the order of the work-groups: drop that whole step
      const int64_t last = ev.back().step;
      while (have > 0 && ev[have - 1].step == last) --have;
    }
    const int64_t m = std::min(have, cap);
    if (m > 0) std::memcpy(out, ev.data(), m * sizeof(iesh_event));
  }
  return IESH_OK;
}

int iesh_clear_events(iesh_ctx* ctx) {
  if (!ctx) return IESH_EINVAL;
  HIPTRY(ctx, hipMemsetAsync(&ctx->cnt->n_events, 0, sizeof(int64_t), ctx->stream));
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  return IESH_OK;
}

int iesh_timing(iesh_ctx* ctx, int32_t enable) {
  if (!ctx) return IESH_EINVAL;
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  ctx->timing = enable != 0;
  ctx->ev_used = 0;
  ctx->ev_marks.clear();
  const int64_t zero[3] = {0, 0, 0};
  HIPTRY(ctx, hipMemcpy(&ctx->cnt->sum_cheb, zero, sizeof(zero), hipMemcpyHostToDevice));
  for (auto& c : ctx->cls)
    if (c.work) HIPTRY(ctx, hipMemcpy(c.work, zero, 2 * sizeof(int64_t), hipMemcpyHostToDevice));
  return IESH_OK;
}

int iesh_class_work(iesh_ctx* ctx, int32_t cls, int64_t* sum_cheb_terms, int64_t* traj_steps) {
  if (!ctx || cls < 0 || cls >= (int)ctx->cls.size() || !sum_cheb_terms || !traj_steps)
    return fail(ctx, IESH_EINVAL, "class index or null pointer");
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  int64_t w[2] = {0, 0};
  if (ctx->cls[cls].work)
    HIPTRY(ctx, hipMemcpy(w, ctx->cls[cls].work, sizeof(w), hipMemcpyDeviceToHost));
  *sum_cheb_terms = w[0];
  *traj_steps = w[1];
  return IESH_OK;
}

int iesh_timing_read(iesh_ctx* ctx, double* ms, int64_t* launches) {
  if (!ctx || !ms || !launches) return IESH_EINVAL;
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < IESH_N_TIMERS; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  for (const auto& m : ctx->ev_marks) {
    float t = 0.0f;
    HIPTRY(ctx, hipEventElapsedTime(&t, ctx->ev_pool[m.second], ctx->ev_pool[m.second + 1]));
    ms[m.first] += t;
    launches[m.first] += 1;
  }
  ctx->ev_used = 0;
  ctx->ev_marks.clear();
  return IESH_OK;
}

int iesh_work(iesh_ctx* ctx, int64_t* sum_cheb_terms, int64_t* traj_steps) {
  if (!ctx || !sum_cheb_terms || !traj_steps) return IESH_EINVAL;
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  int64_t w[2];
  HIPTRY(ctx, hipMemcpy(w, &ctx->cnt->sum_cheb, sizeof(w), hipMemcpyDeviceToHost));
  *sum_cheb_terms = w[0];
  *traj_steps = w[1];
  return IESH_OK;
}

int iesh_orthonormality_defect(iesh_ctx* ctx, double* per_traj, double* max_seen,
                               int64_t* violations) {
  if (!ctx) return IESH_EINVAL;
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  uint64_t w[2] = {0, 0};
  HIPTRY(ctx, hipMemcpy(w, &ctx->cnt->defect_max_bits, sizeof(w), hipMemcpyDeviceToHost));
  if (max_seen) std::memcpy(max_seen, &w[0], sizeof(double));
  if (violations) *violations = (int64_t)w[1];
  if (per_traj) {
    for (size_t ci = 0; ci < ctx->cls.size(); ++ci) {
      const ClassDev& c = ctx->cls[ci];
      if (!c.n_traj) continue;
      std::vector<double> d(c.n_traj, 0.0);
      if (c.defect)
        HIPTRY(ctx, hipMemcpy(d.data(), c.defect, d.size() * sizeof(double), hipMemcpyDeviceToHost));
      for (int hm = 0; hm < c.n_traj; ++hm) per_traj[ctx->members[ci][hm]] = d[hm];
    }
  }
  return IESH_OK;
}

int iesh_hop_evals(iesh_ctx* ctx, int64_t* full_evals) {
  if (!ctx || !full_evals) return IESH_EINVAL;
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  HIPTRY(ctx, hipMemcpy(full_evals, &ctx->cnt->hop_evals, sizeof(int64_t), hipMemcpyDeviceToHost));
  return IESH_OK;
}


int iesh_adjoint_forward(iesh_ctx* ctx, const double* path, int32_t n_steps, int32_t ckpt_every,
                         const double* terms, double* loss_out) {
  if (!ctx || !path || n_steps < 1 || ckpt_every < 1)
    return fail(ctx, IESH_EINVAL, "adjoint: path, n_steps >= 1 and ckpt_every >= 1 required");
  AdjTerms tw{1.0, 1.0, 0.0, 0.0};
  if (terms) {
    tw = AdjTerms{terms[0], terms[1], terms[2], terms[3]};
    if (!std::isfinite(tw.cP) || !std::isfinite(tw.cE) || !std::isfinite(tw.cG) ||
        !std::isfinite(tw.cF))
      return fail(ctx, IESH_EINVAL, "adjoint: non-finite loss term weight");
  }
  if (ctx->run.precision != IESH_FP64)
    return fail(ctx, IESH_ENOTSUP, "adjoint: FP64 contexts only");
  if (ctx->run.elec_substeps > 1)
    return fail(ctx, IESH_ENOTSUP, "adjoint: one electronic step per nuclear step only");
  for (const auto& c : ctx->cls)
    if (c.n_traj && c.md.kind != IESH_MODEL_HARMONIC)
      return fail(ctx, IESH_ENOTSUP, "adjoint: harmonic (double-well) models only");
  for (const auto& c : ctx->cls)
    if (c.n_traj && c.md.M_red != c.md.M)
      return fail(ctx, IESH_ENOTSUP, "adjoint: distinct bath energies only");
  if (ctx->run.dt_levels > 0) return fail(ctx, IESH_ENOTSUP, "adjoint: fixed time step only");
  const int T = ctx->run.n_traj;
  for (size_t q = 0; q < (size_t)T * (n_steps + 1); ++q)
    if (!std::isfinite(path[q])) return fail(ctx, IESH_EINVAL, "adjoint: non-finite path");
  adj_release(ctx);
  ctx->adj_terms = tw;
  ctx->adj_steps = n_steps;
  ctx->adj_ckpt = std::min(ckpt_every, n_steps);
  const int n_ckpt = (n_steps + ctx->adj_ckpt - 1) / ctx->adj_ckpt;
  int rc;
  if ((rc = adj_alloc(ctx, &ctx->adj_path, (size_t)T * (n_steps + 1))) ||
      (rc = adj_alloc(ctx, &ctx->adj_loss, (size_t)T)))
    return rc;
  HIPTRY(ctx, hipMemcpyAsync(ctx->adj_path, path, (size_t)T * (n_steps + 1) * sizeof(double),
                             hipMemcpyHostToDevice, ctx->stream));
  for (size_t ci = 0; ci < ctx->cls.size(); ++ci) {
    const ClassDev& c = ctx->cls[ci];
    if (!c.n_traj) continue;
    if ((rc = adj_alloc(ctx, &ctx->adj[ci].ckpt, (size_t)n_ckpt * c.n_traj * c.md.N * c.md.n_pad * 2)))
      return rc;
    if (tw.cG != 0.0 && (rc = adj_alloc(ctx, &ctx->adj[ci].hopscr, adj_hop_scratch_elems(c))))
      return rc;
  }
  // start: x = path[.][0], v = 0, the N lowest adiabatic orbitals occupied
  std::vector<double> x0(T), v0(T, 0.0);
  for (int t = 0; t < T; ++t) x0[t] = path[(size_t)t * (n_steps + 1)];
  if ((rc = reset_perm(ctx)) || (rc = upload_state(ctx, x0.data(), v0.data(), nullptr, nullptr)) ||
      (rc = reset_traj_words(ctx)))
    return rc;
  const int64_t zero = 0;
  HIPTRY(ctx, hipMemcpyAsync(&ctx->cnt->max_cheb, &zero, sizeof(zero), hipMemcpyHostToDevice,
                             ctx->stream));
  for (auto& c : ctx->cls)
    if (c.n_traj) HIPTRY(ctx, launch_init_thermal(c, 0.0, 0.0, ctx->run.seed, ctx->stream));
  for (int n = 0; n < n_steps; ++n) {
    for (size_t ci = 0; ci < ctx->cls.size(); ++ci) {
      const ClassDev& c = ctx->cls[ci];
      if (!c.n_traj) continue;
      const size_t csz = (size_t)c.n_traj * c.md.N * c.md.n_pad * 2;
      if (n % ctx->adj_ckpt == 0)
        HIPTRY(ctx, hipMemcpyAsync(ctx->adj[ci].ckpt + (size_t)(n / ctx->adj_ckpt) * csz, c.C64,
                                   csz * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
      const ClassDev cc = on_path(ctx, c, n);
      if ((rc = adj_step(ctx, cc))) return rc;
      HIPTRY(ctx, timed(ctx, IESH_TIMER_ADJ_EIG,
                        [&] { return launch_adj_loss(cc, ctx->adj_loss, n, n_steps, tw, ctx->stream); }));
      if (tw.cG != 0.0)
        HIPTRY(ctx, timed(ctx, IESH_TIMER_ADJ_HOP, [&] {
                 return launch_adj_hop(cc, c.C64, nullptr, ctx->adj[ci].hopscr, nullptr, ctx->adj_loss,
                                       nullptr, n + 1, n_steps, ctx->run.dt, tw.cG, 0, ctx->stream);
               }));
    }
  }
  int64_t kmax = 0;
  HIPTRY(ctx, hipMemcpyAsync(&kmax, &ctx->cnt->max_cheb, sizeof(int64_t), hipMemcpyDeviceToHost,
                             ctx->stream));
  if (loss_out)
    HIPTRY(ctx, hipMemcpyAsync(loss_out, ctx->adj_loss, T * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  ctx->adj_tap_k = (int)std::max<int64_t>(kmax, 1);
  ctx->step += n_steps;
  ctx->adj_forward_done = true;
  return IESH_OK;
}

int iesh_adjoint_backward(iesh_ctx* ctx, const double* dloss, double* grad_out) {
  if (!ctx || !dloss || !grad_out) return fail(ctx, IESH_EINVAL, "adjoint: null pointer");
  if (!ctx->adj_forward_done)
    return fail(ctx, IESH_ESTATE, "adjoint: iesh_adjoint_forward must come first");
  const int T = ctx->run.n_traj, nst = ctx->adj_steps, seg = ctx->adj_ckpt;
  const int gstride = ctx->n_max + 4;
  int rc;
  if (!ctx->adj_backward_bufs) {
    if ((rc = adj_alloc(ctx, &ctx->adj_w, (size_t)T)) ||
        (rc = adj_alloc(ctx, &ctx->adj_grad, (size_t)T * gstride)))
      return rc;
    for (size_t ci = 0; ci < ctx->cls.size(); ++ci) {
      const ClassDev& c = ctx->cls[ci];
      if (!c.n_traj) continue;
      auto& a = ctx->adj[ci];
      const size_t csz = (size_t)c.n_traj * c.md.N * c.md.n_pad * 2;
      if ((rc = adj_alloc(ctx, &a.snap, (size_t)(seg + 1) * csz)) ||
          (rc = adj_alloc(ctx, &a.Gh, csz)) ||
          (rc = adj_alloc(ctx, &a.taps_s, (size_t)ctx->adj_tap_k * csz)) ||
          (rc = adj_alloc(ctx, &a.taps_t, (size_t)ctx->adj_tap_k * csz)) ||
          (rc = adj_alloc(ctx, &a.imphi, (size_t)c.n_traj * c.md.n_pad * c.md.n_pad)) ||
          (rc = adj_alloc(ctx, &a.rediag, (size_t)c.n_traj * c.md.n_pad)) ||
          (rc = adj_alloc(ctx, &a.chebc, (size_t)c.n_traj * kChebStride)))
        return rc;
      if (ctx->adj_terms.cG != 0.0 &&
          (rc = adj_alloc(ctx, &a.hopbar, (size_t)c.n_traj * (2 * c.md.n_pad + 1))))
        return rc;
    }
    ctx->adj_backward_bufs = true;
  }
  HIPTRY(ctx, hipMemcpyAsync(ctx->adj_w, dloss, T * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIPTRY(ctx, hipMemsetAsync(ctx->adj_grad, 0, (size_t)T * gstride * sizeof(double), ctx->stream));
  for (size_t ci = 0; ci < ctx->cls.size(); ++ci) {
    const ClassDev& c = ctx->cls[ci];
    if (!c.n_traj) continue;
    const size_t csz = (size_t)c.n_traj * c.md.N * c.md.n_pad * 2;
    HIPTRY(ctx, hipMemsetAsync(ctx->adj[ci].Gh, 0, csz * sizeof(double), ctx->stream));
  }
  const int n_ckpt = (nst + seg - 1) / seg;
  for (int sg = n_ckpt - 1; sg >= 0; --sg) {
    const int a0 = sg * seg, b0 = std::min(a0 + seg, nst);
    for (size_t ci = 0; ci < ctx->cls.size(); ++ci) {
      const ClassDev& c = ctx->cls[ci];
      if (!c.n_traj) continue;
      auto& a = ctx->adj[ci];
      const size_t csz = (size_t)c.n_traj * c.md.N * c.md.n_pad * 2;
      auto snap = [&](int j) { return a.snap + (size_t)j * csz; };
      // orbitals C_{a0} .. C_{b0} of the segment, recomputed from its checkpoint
      HIPTRY(ctx, hipMemcpyAsync(snap(0), a.ckpt + (size_t)sg * csz, csz * sizeof(double),
                                 hipMemcpyDeviceToDevice, ctx->stream));
      for (int n = a0; n < b0; ++n) {
        HIPTRY(ctx, hipMemcpyAsync(snap(n - a0 + 1), snap(n - a0), csz * sizeof(double),
                                   hipMemcpyDeviceToDevice, ctx->stream));
        ClassDev cc = on_path(ctx, c, n);
        cc.C64 = snap(n - a0 + 1);
        if ((rc = adj_step(ctx, cc))) return rc;
      }
      // reverse sweep over the segment
      for (int n = b0 - 1; n >= a0; --n) {
        ClassDev cc = on_path(ctx, c, n);
        const hipStream_t st = ctx->stream;
        HIPTRY(ctx, timed(ctx, IESH_TIMER_ADJ_EIG,
                          [&] { return launch_eig_step(cc, ctx->run.dt, ctx->cnt, st); }));
        // explicit loss terms at x_{n+1}: cotangent of C_{n+1}
        const AdjTerms& tw = ctx->adj_terms;
        if (tw.cG != 0.0)
          HIPTRY(ctx, timed(ctx, IESH_TIMER_ADJ_HOP, [&] {
                   return launch_adj_hop(cc, snap(n - a0 + 1), a.Gh, a.hopscr, ctx->adj_w, nullptr,
                                         a.hopbar, n + 1, nst, ctx->run.dt, tw.cG, 1, st);
                 }));
        HIPTRY(ctx, timed(ctx, IESH_TIMER_ADJ_EIG, [&] {
                 return launch_adj_explicit(cc, snap(n - a0 + 1), a.Gh, ctx->adj_w,
                                            tw.cG != 0.0 ? a.hopbar : nullptr, tw, ctx->adj_grad,
                                            gstride, n + 1, nst, st);
               }));
        // Chebyshev vectors of C_n under this step's propagator
        ClassDev cf = cc;
        cf.C64 = snap(n - a0);
        HIPTRY(ctx, timed(ctx, IESH_TIMER_ADJ_PROP,
                          [&] { return launch_prop_taps(cf, 2, a.taps_t, ctx->adj_tap_k, st); }));
        // cotangent of C_n = U^H (cotangent of C_{n+1}), keeping the adjoint vectors
        HIPTRY(ctx, launch_conj_cheb(cc, a.chebc, st));
        ClassDev cg = cc;
        cg.C64 = a.Gh;
        cg.cheb = a.chebc;
        HIPTRY(ctx, timed(ctx, IESH_TIMER_ADJ_PROP,
                          [&] { return launch_prop_taps(cg, 1, a.taps_s, ctx->adj_tap_k, st); }));
        // through the propagator matrix into the midpoint eigen-solve
        HIPTRY(ctx, timed(ctx, IESH_TIMER_ADJ_PHI, [&] {
                 return launch_adj_phi(cc, a.taps_s, a.taps_t, ctx->adj_tap_k, a.imphi, a.rediag, st);
               }));
        HIPTRY(ctx, timed(ctx, IESH_TIMER_ADJ_EIG, [&] {
                 return launch_adj_mid(cc, a.imphi, a.rediag, ctx->adj_grad, gstride, n,
                                       ctx->run.dt, st);
               }));
      }
    }
  }
  HIPTRY(ctx, hipMemcpyAsync(grad_out, ctx->adj_grad, (size_t)T * gstride * sizeof(double),
                             hipMemcpyDeviceToHost, ctx->stream));
  HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
  return IESH_OK;
}

}  // extern "C"

namespace iesh {
void set_call_error(const std::string& why) { g_create_err = why; }
}  // namespace iesh
