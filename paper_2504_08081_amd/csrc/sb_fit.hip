// Fit-step kernel of the serving loop (gfx950).
//
// One workgroup of NW waves advances one resident fit by up to `iters`
// Levenberg-Marquardt iterations.  Each evaluation runs the bandflux pipeline of
// sb_device.h in FIT mode (row projections for the flux, d/dx1 and d/dc; d/dt0
// comes from the phase-weight derivatives and d/d ln x0 equals the flux), and
// accumulates chi2, J^T W J and J^T W r over the fit's observations with a
// fixed-order workgroup reduction whose result every thread receives.  Every
// thread then holds an identical copy of the LM state and takes the same 4x4
// damped step, so the iteration loop has no thread-dependent branch around its
// barriers.  The fit's state is read from and written back to its slot, so a
// fit gives the same result however its iterations are split over launches and
// whichever other fits share the launch.
#include <climits>
#include <mutex>

#include "sb_device.h"
#include "sb_lbfgsb.h"

namespace sbk {

struct FitShared {
  unsigned mask[2];
  int rlo[SB_MAX_BANDS];
  int rhi[SB_MAX_BANDS];
  int slot_of[SB_MAX_BANDS];
  int slot_ok[BAND_GROUP];
  float red[red_floats(16, MAX_NW)];
  FitSlot lb;      // L-BFGS-B: the fit's state, updated by thread 0 between evaluations
  int lb_go;       // L-BFGS-B: thread 0 planned another evaluation
};

// chi2, H (packed) and g at parameters q = (t0, ln x0, x1, c); every thread gets them.
struct FitObs {
  const float* t;
  const int* band;
  const float* data;
  const float* w;
  int n;
};

template <int NW>
__device__ void fit_eval(const KModel& m, const KTables& tb, const KFit& F, const FitObs& O, double s64,
                         const float* q, const Lds& L, FitShared& S, float (&out)[15]) {
  constexpr int NT = NW * WAVE;
  const int tid = threadIdx.x;
  const float t0 = q[0], x0 = expf(q[1]), x1 = q[2], c = q[3];
  const float s = (float)s64;
  const float A = (float)((double)x0 * s64);
  reset_scan(S.mask, S.rlo, S.rhi, S.slot_of);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 15; ++k) out[k] = 0.f;
  for (int i = tid; i < O.n; i += NT) {
    const int bd = O.band[i];
    const PhaseCell pc = phase_cell(O.t[i], t0, s64, m);
    if ((unsigned)bd >= (unsigned)m.n_bands || pc.nan) {
      // only device-resident batches can hold these (the server checks its requests)
      if ((unsigned)bd >= (unsigned)m.n_bands) atomicOr(F.err, EFLAG_BAND);
      out[14] = __builtin_nanf("");
      continue;
    }
    if (!pc.in) {
      const float r = O.data[i];
      out[14] = fmaf(r * r, O.w[i], out[14]);
      continue;
    }
    atomicMin(&S.rlo[bd], pc.r0);
    atomicMax(&S.rhi[bd], pc.r1);
    atomicOr(&S.mask[bd >> 5], 1u << (bd & 31));
  }
  __syncthreads();
  constexpr int NR = ModeInfo<FIT>::NR;
  unsigned rem0 = (unsigned)uni((int)S.mask[0]), rem1 = (unsigned)uni((int)S.mask[1]);
  while (rem0 | rem1) {
    unsigned g0, g1;
    take_group(rem0, rem1, g0, g1, ModeInfo<FIT>::GROUP);
    group_rows<FIT, NW>(m, tb, g0, g1, s64, c, x1, S.rlo, S.rhi, S.slot_of, S.slot_ok, L, F.err);
    __syncthreads();
    for (int i = tid; i < O.n; i += NT) {
      const int bd = O.band[i];
      if ((unsigned)bd >= (unsigned)m.n_bands) continue;
      const int slot = S.slot_of[bd];
      if (slot < 0) continue;
      const PhaseCell pc = phase_cell(O.t[i], t0, s64, m);
      if (!pc.in || pc.nan) continue;
      const int rlo = S.rlo[bd], rhi = S.rhi[bd];
      const float* Rb = L.R + (size_t)slot * m.n_phase * NR;
      float J[4], f;
      if (!S.slot_ok[slot]) {
        f = __builtin_nanf("");
        J[0] = J[1] = J[2] = J[3] = f;
      } else {
        float wp[4], dw[4];
        cr_weights(pc.x, pc.edge, wp);
        cr_dweights(pc.x, pc.edge, dw);
        // all four taps (an edge cell's outer weights are zero and add exact zeros), unrolled
        float Sx = 0.f, Sp = 0.f, S1 = 0.f, Sc = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const float* r = Rb + row_clamp(pc.a - 1 + t, rlo, rhi) * NR;
          Sx = fmaf(wp[t], r[0], Sx);
          Sp = fmaf(dw[t], r[0], Sp);
          S1 = fmaf(wp[t], r[1], S1);
          Sc = fmaf(wp[t], r[2], Sc);
        }
        f = A * Sx;
        J[0] = -A * s * Sp * m.inv_dphase;   // d/dt0
        J[1] = f;                            // d/d ln x0
        J[2] = A * S1;                       // d/dx1
        J[3] = A * Sc;                       // d/dc
      }
      const float wi = O.w[i];
      const float r = O.data[i] - f;
      int k = 0;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const float wa = wi * J[a];
#pragma unroll
        for (int bb = a; bb < 4; ++bb) {
          out[k] = fmaf(wa, J[bb], out[k]);
          ++k;
        }
        out[10 + a] = fmaf(wa, r, out[10 + a]);
      }
      out[14] = fmaf(r * r, wi, out[14]);
    }
    __syncthreads();
    for (int h = 0; h < 2; ++h) {
      unsigned gm = h ? g1 : g0;
      while (gm) {
        const int bd = h * 32 + __ffs(gm) - 1;
        gm &= gm - 1;
        if (tid == 0) S.slot_of[bd] = -1;
      }
    }
  }
  block_sum<15, NW>(out, S.red);
}

// Solve (H + lambda diag H) d = g by Cholesky over the free parameters (free_mask
// bit i set): a held parameter's row and column become those of the identity and
// its right-hand side 0, which decouples it with d_i = 0 and leaves the free block
// as it was.  False if a pivot is not positive.
__device__ bool damped_solve(const float* H, const float* g, float lambda, int free_mask, float* d) {
  float a[4][4];
  float rhs[4];
  int k = 0;
  for (int i = 0; i < 4; ++i)
    for (int j = i; j < 4; ++j) {
      const bool keep = ((free_mask >> i) & 1) && ((free_mask >> j) & 1);
      const float v = keep ? H[k] : (i == j ? 1.f : 0.f);
      a[i][j] = v;
      a[j][i] = v;
      ++k;
    }
  for (int i = 0; i < 4; ++i) {
    const bool fr = (free_mask >> i) & 1;
    if (fr) a[i][i] = fmaf(lambda, a[i][i], a[i][i]);
    rhs[i] = fr ? g[i] : 0.f;
  }
  // L L^T with the pivots' reciprocal square roots kept (inv[i] = 1 / L_ii), so
  // every division is a multiplication: the step is a descent direction whose
  // trial point is evaluated before it is accepted, so the hardware reciprocal
  // square root's last-bit error is harmless
  float l[4][4] = {};
  float inv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      float sum = a[i][j];
#pragma unroll
      for (int p = 0; p < j; ++p) sum = fmaf(-l[i][p], l[j][p], sum);
      if (i == j) {
        if (!(sum > 0.f) || !isfinite(sum)) return false;
        inv[i] = __builtin_amdgcn_rsqf(sum);
        l[i][i] = sum * inv[i];
      } else {
        l[i][j] = sum * inv[j];
      }
    }
  }
  float y[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float sum = rhs[i];
#pragma unroll
    for (int p = 0; p < i; ++p) sum = fmaf(-l[i][p], y[p], sum);
    y[i] = sum * inv[i];
  }
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    float sum = y[i];
#pragma unroll
    for (int p = i + 1; p < 4; ++p) sum = fmaf(-l[p][i], d[p], sum);
    d[i] = sum * inv[i];
  }
  for (int i = 0; i < 4; ++i)
    if (!isfinite(d[i])) return false;
  return true;
}

// Where a fit starts: its observations, redshift, starting point, free mask and
// (L-BFGS-B) bounds of q, from the admission header or the caller's batch arrays.
struct FitStart {
  float z;
  float q[4];
  float lo[4], hi[4];
  int free_mask;
  bool bad;          // malformed offsets or bounds: nothing to fit
};

// Bounds of q = (t0, ln x0, x1, c) from bounds of (t0, x0, x1, c) (null: none); an x0 bound
// <= 0 is no lower bound; false if a bound is NaN, an upper x0 bound is <= 0 or lo > hi.
__device__ inline bool q_bounds(const float* lower, const float* upper, float* lo, float* hi) {
  const float inf = __builtin_inff();
  bool ok = true;
  for (int i = 0; i < 4; ++i) {
    float a = lower ? lower[i] : -inf, b = upper ? upper[i] : inf;
    if (i == 1) {
      a = a > 0.f ? (float)log((double)a) : -inf;
      if (upper) {
        ok = ok && b > 0.f;
        b = b > 0.f ? (float)log((double)b) : -inf;
      }
    }
    ok = ok && !(a != a) && !(b != b) && a <= b;
    lo[i] = a;
    hi[i] = b;
  }
  return ok;
}

// The L-BFGS-B iterations of one fit (sb_lbfgsb.h): thread 0 keeps the state in
// LDS and plans each evaluation; every thread evaluates chi2 and its gradient
// at the planned point.
template <int NW>
__device__ void fit_lbfgsb(const KModel& m, const KTables& tb, const KFit& F, const FitObs& O, int obs_off,
                           bool start, const FitStart& fs, FitSlot* sl, int f, const Lds& L, FitShared& S) {
  const int tid = threadIdx.x;
  FitSlot& st = S.lb;
  if (tid == 0) {
    if (start) {
      st = FitSlot{};
      st.obs_off = obs_off;
      st.n_obs = O.n;
      st.iter = -1;
      st.status = SB_OK;
      st.free_mask = fs.free_mask;
      st.z = fs.z;
      for (int i = 0; i < 4; ++i) {
        const bool fr = (fs.free_mask >> i) & 1;
        st.lb_lo[i] = fr ? fs.lo[i] : fs.q[i];
        st.lb_hi[i] = fr ? fs.hi[i] : fs.q[i];
        st.q[i] = fminf(fmaxf(fs.q[i], st.lb_lo[i]), st.lb_hi[i]);
      }
      st.lb_phase = LB_NEED_DIR;
      st.lb_first = 1;
      if (fs.bad) {
        st.chi2 = __builtin_nanf("");
        st.iter = 0;
        st.status = SB_FIT_DIVERGED;
      }
    } else {
      st = *sl;
    }
  }
  __syncthreads();
  const double s64 = 1.0 / (1.0 + (double)uni_f(S.lb.z));
  float out[15];
  if (uni(S.lb.iter < 0 ? 1 : 0)) {
    float q[4] = {S.lb.q[0], S.lb.q[1], S.lb.q[2], S.lb.q[3]};
    fit_eval<NW>(m, tb, F, O, s64, q, L, S, out);
    if (tid == 0) {
      st.chi2 = out[14];
      if (isfinite(out[14])) {
        for (int i = 0; i < 4; ++i) st.g[i] = out[10 + i];
        st.iter = 0;
      } else {
        st.status = SB_FIT_DIVERGED;
      }
    }
  }
  for (int it = 0; it < F.iters; ++it) {
    if (tid == 0) S.lb_go = lb_plan(st, F.fit_iters) ? 1 : 0;
    __syncthreads();
    if (!uni(S.lb_go)) break;
    float q[4] = {S.lb.lb_trial[0], S.lb.lb_trial[1], S.lb.lb_trial[2], S.lb.lb_trial[3]};
    fit_eval<NW>(m, tb, F, O, s64, q, L, S, out);
    if (tid == 0) lb_after_eval(st, out[14], out + 10, F.lbfgs_m);
  }
  if (tid == 0) {
    *sl = st;
    if (F.b_off) {
      if (F.b_last) {
        sb_fit_out r;
        r.t0 = st.q[0];
        r.x0 = (st.free_mask & SB_FREE_X0) ? expf(st.q[1]) : F.b_x0[f];
        r.x1 = st.q[2];
        r.c = st.q[3];
        r.chi2 = st.chi2;
        r.status = st.status;
        r.iters = st.iter < 0 ? 0 : st.iter;
        r.n_accept = st.n_accept;
        F.b_out[f] = r;
      }
    } else {
      const int oi = F.out_idx[f];
      if (oi >= 0) F.results[oi] = st;
    }
  }
}

template <int NW>
__global__ __launch_bounds__(NW * WAVE) void k_fit(KModel m, KTables tb, KFit F) {
  constexpr int NT = NW * WAVE;
  extern __shared__ __align__(16) char smem[];
  __shared__ FitShared S;
  const Lds L = lds_carve<FIT, NW>(smem, m, tb, uni((int)(threadIdx.x / WAVE)));
  // no band's point data in this launch's scratch yet (read after the first barrier)
  if ((threadIdx.x & (WAVE - 1)) == 0) L.tag[0] = -1;
  const int tid = threadIdx.x;
  const bool batch = F.b_off != nullptr;
  const int f = blockIdx.x;
  FitSlot* sl = F.slots + (batch ? f : F.active[f]);
  const int adm = batch ? -1 : uni(F.admit[f]);
  const bool start = batch ? (F.b_first != 0) : (adm >= 0);
  FitObs O;
  int obs_off = 0;
  FitStart fs{};
  if (start) {
    if (batch) {
      // first launch of a batch fit: its observations are the caller's CSR range
      int lo = F.b_off[f], hi = F.b_off[f + 1];
      fs.bad = lo < 0 || hi < lo || hi > F.b_n_obs;
      if (fs.bad) {
        if (tid == 0) atomicOr(F.err, EFLAG_CSR);
        lo = hi = 0;
      }
      O.t = F.b_t + lo;
      O.band = F.b_band + lo;
      O.data = F.b_data + lo;
      O.w = F.b_w + lo;
      O.n = hi - lo;
      obs_off = lo;
      fs.z = F.b_z[f];
      fs.q[0] = F.b_t0[f];
      fs.q[1] = (float)log((double)F.b_x0[f]);
      fs.q[2] = F.b_x1[f];
      fs.q[3] = F.b_c[f];
      const int fm = F.b_free ? (int)(F.b_free[f] & (unsigned)SB_FREE_ALL) : 0;
      fs.free_mask = fm == 0 ? SB_FREE_ALL : fm;
      if (!q_bounds(F.b_lower ? F.b_lower + 4 * f : nullptr, F.b_upper ? F.b_upper + 4 * f : nullptr, fs.lo, fs.hi))
        fs.bad = true;
    } else {
      // first launch of a served fit: move its observations from the inbox to the arena
      const AdmitHeader h = F.hdr[adm];
      for (int i = tid; i < h.n_obs; i += NT) {
        F.t[h.arena_off + i] = F.in_t[h.src_off + i];
        F.band[h.arena_off + i] = F.in_band[h.src_off + i];
        F.data[h.arena_off + i] = F.in_data[h.src_off + i];
        F.w[h.arena_off + i] = F.in_w[h.src_off + i];
      }
      // this launch reads the inbox copy; the arena copy serves the later launches
      O.t = F.in_t + h.src_off;
      O.band = F.in_band + h.src_off;
      O.data = F.in_data + h.src_off;
      O.w = F.in_w + h.src_off;
      O.n = h.n_obs;
      obs_off = h.arena_off;
      fs.z = h.z;
      fs.q[0] = h.t0;
      fs.q[1] = h.lnx0;
      fs.q[2] = h.x1;
      fs.q[3] = h.c;
      fs.free_mask = h.free_mask;
      for (int i = 0; i < 4; ++i) {
        fs.lo[i] = h.lo[i];
        fs.hi[i] = h.hi[i];
      }
    }
  } else {
    obs_off = sl->obs_off;
    O.t = (batch ? F.b_t : F.t) + obs_off;
    O.band = (batch ? F.b_band : F.band) + obs_off;
    O.data = (batch ? F.b_data : F.data) + obs_off;
    O.w = (batch ? F.b_w : F.w) + obs_off;
    O.n = sl->n_obs;
  }
  if (uni(F.solver) == SB_SOLVER_LBFGSB) {
    fit_lbfgsb<NW>(m, tb, F, O, obs_off, start, fs, sl, f, L, S);
    return;
  }

  // Levenberg-Marquardt: the state in registers; every thread holds the same values
  float z;
  float q[4], H[10], g[4], lambda, chi2;
  int iter, n_acc, status, free_mask;
  if (start) {
    z = fs.z;
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = fs.q[k];
    free_mask = fs.free_mask;
#pragma unroll
    for (int k = 0; k < 10; ++k) H[k] = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = 0.f;
    lambda = F.lambda0;
    chi2 = 0.f;
    iter = -1;
    n_acc = 0;
    status = SB_OK;
    if (uni(fs.bad ? 1 : 0)) {
      // malformed offsets: no observations to fit
      chi2 = __builtin_nanf("");
      iter = 0;
      status = SB_FIT_DIVERGED;
    }
  } else {
    z = sl->z;
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = sl->q[k];
#pragma unroll
    for (int k = 0; k < 10; ++k) H[k] = sl->H[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = sl->g[k];
    lambda = sl->lambda;
    chi2 = sl->chi2;
    iter = sl->iter;
    n_acc = sl->n_accept;
    status = sl->status;
    free_mask = sl->free_mask;
  }
  const double s64 = 1.0 / (1.0 + (double)z);
  float out[15];
  if (uni(iter < 0 ? 1 : 0)) {
    fit_eval<NW>(m, tb, F, O, s64, q, L, S, out);
    if (uni(isfinite(out[14]) ? 1 : 0)) {
#pragma unroll
      for (int k = 0; k < 10; ++k) H[k] = out[k];
#pragma unroll
      for (int k = 0; k < 4; ++k) g[k] = out[10 + k];
      chi2 = out[14];
      iter = 0;
      lambda = F.lambda0;
    } else {
      chi2 = out[14];
      status = SB_FIT_DIVERGED;
    }
  }
  for (int it = 0; it < F.iters; ++it) {
    if (uni((status != SB_OK || iter >= F.fit_iters) ? 1 : 0)) break;
    float d[4];
    const int solved = uni(damped_solve(H, g, lambda, free_mask, d) ? 1 : 0);
    if (!solved) {
      lambda = fminf(lambda * 10.f, 1e9f);
      iter += 1;
      continue;
    }
    float qt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) qt[k] = q[k] + d[k];
    fit_eval<NW>(m, tb, F, O, s64, qt, L, S, out);
    if (uni((isfinite(out[14]) && out[14] < chi2) ? 1 : 0)) {
#pragma unroll
      for (int k = 0; k < 4; ++k) q[k] = qt[k];
#pragma unroll
      for (int k = 0; k < 10; ++k) H[k] = out[k];
#pragma unroll
      for (int k = 0; k < 4; ++k) g[k] = out[10 + k];
      chi2 = out[14];
      lambda = fmaxf(lambda * 0.1f, 1e-9f);
      n_acc += 1;
    } else {
      lambda = fminf(lambda * 10.f, 1e9f);
    }
    iter += 1;
  }
  if (tid == 0) {
    FitSlot st{};
    st.obs_off = obs_off;
    st.n_obs = O.n;
    st.iter = iter;
    st.n_accept = n_acc;
    st.status = status;
    st.free_mask = free_mask;
    st.z = z;
    for (int k = 0; k < 4; ++k) st.q[k] = q[k];
    st.lambda = lambda;
    st.chi2 = chi2;
    for (int k = 0; k < 10; ++k) st.H[k] = H[k];
    for (int k = 0; k < 4; ++k) st.g[k] = g[k];
    *sl = st;
    if (batch) {
      if (F.b_last) {
        sb_fit_out r;
        r.t0 = q[0];
        r.x0 = (free_mask & SB_FREE_X0) ? expf(q[1]) : F.b_x0[f];
        r.x1 = q[2];
        r.c = q[3];
        r.chi2 = chi2;
        r.status = status;
        r.iters = iter < 0 ? 0 : iter;
        r.n_accept = n_acc;
        F.b_out[f] = r;
      }
    } else {
      const int oi = F.out_idx[f];
      if (oi >= 0) F.results[oi] = st;
    }
  }
}

size_t fit_lds_bytes(const KModel& m, int max_pts, int jcap) {
  return lds_layout_bytes<FIT>(m.n_phase, max_pts, jcap, 1);
}

template <int NW>
static hipError_t launch_fit_nw(const KModel& m, const KTables& tb, const KFit& f, size_t lds, hipStream_t st) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_fit<NW>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_fit<NW>, dim3(f.n_active), dim3(NW * WAVE), lds, st, m, tb, f);
  return hipGetLastError();
}

// The preferred number of waves per fit when its LDS fits, else one.
hipError_t launch_fit(const KModel& m, const KTables& tb, const KFit& f, hipStream_t st) {
  if (f.n_active <= 0) return hipSuccess;
  constexpr int NW = ModeInfo<FIT>::NW;
  const size_t lds = lds_layout_bytes<FIT>(m.n_phase, tb.max_pts, tb.jcap, NW);
  if (lds <= (size_t)tb.lds_limit) return launch_fit_nw<NW>(m, tb, f, lds, st);
  return launch_fit_nw<1>(m, tb, f, fit_lds_bytes(m, tb.max_pts, tb.jcap), st);
}

// ------------------------------------------------------------ allocation-free batch fits
//
// The per-fit state of sb_fit_batch_noalloc lives in this fixed device array
// (one copy per GPU, held until the process ends).  Host code never passes the
// array's name to a kernel: the name is a host-side stand-in, and the device
// address comes from hipGetSymbolAddress, taken once per device at context
// creation with that device current.
static __device__ __align__(256) FitSlot scratch[SB_FIT_NOALLOC_MAX];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
FitSlot* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t fit_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = (FitSlot*)p;
  return hipSuccess;
}

FitSlot* fit_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

// Batch fits run two waves per fit (one if that LDS does not fit): a batch has
// enough fits to fill the GPU, and at 163 VGPRs a CU holds twelve waves, so
// smaller workgroups keep more fits in flight (4,096 fits: 3.4 ms per LM call
// against 7.6 ms with the server's eight waves, 3.7 against 9.3 ms for L-BFGS-B).
// Every fit of every batch call gets the same shape, so a fit's result does not
// depend on the rest of its batch.
constexpr int BATCH_FIT_NW = 2;

hipError_t launch_fit_batch(const KModel& m, const KTables& tb, KFit f, int n_fit, int fit_iters, int iters_per_tick,
                            hipStream_t st) {
  if (n_fit <= 0) return hipSuccess;
  const int n_launch = fit_iters <= 0 ? 1 : (fit_iters + iters_per_tick - 1) / iters_per_tick;
  const size_t lds = lds_layout_bytes<FIT>(m.n_phase, tb.max_pts, tb.jcap, BATCH_FIT_NW);
  const bool two = lds <= (size_t)tb.lds_limit;
  f.n_active = n_fit;
  f.fit_iters = fit_iters;
  f.iters = iters_per_tick;
  for (int l = 0; l < n_launch; ++l) {
    f.b_first = l == 0;
    f.b_last = l == n_launch - 1;
    const hipError_t e = two ? launch_fit_nw<BATCH_FIT_NW>(m, tb, f, lds, st)
                             : launch_fit_nw<1>(m, tb, f, fit_lds_bytes(m, tb.max_pts, tb.jcap), st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace sbk
