// Device-side building blocks of the bandflux pipeline (gfx950, wave64).
//
// The bandflux of observation i of supernova s in band b (bandflux equation,
// trapezoid rule) is
//     f_i = A * sum_k W_k E_k I(p_i, mu_k),   W_k = w_k lam_k T_k / (hc),
//     E_k = exp(c CL(mu_k)),  mu_k = lam_k s,  I = M0 + x1 M1 interpolated.
// The bicubic is separable, I(p, mu) = sum_a wp_a(p) sum_j wl_j(mu) M[a, j],
// so every observation of the same (supernova, band) shares the wavelength
// half of the work:
//     G(j)  = sum_k W_k E_k wl_j(mu_k)                  (per band, per supernova)
//     R(a)  = sum_j G(j) (M0 + x1 M1)[a, j]             (one row projection per row)
//     f_i   = A * sum_a wp_a(p_i) R(a)                  (4 taps per observation)
// This is the same sum as the definition, only reassociated.  The adjoint
// needs more weight vectors and projections (colour, wavelength derivative,
// M1 alone), which reuse the same surface reads.
//
// Precision: storage, weights and every sum are FP32.  The grid coordinates
// (s = 1/(1+z), the phase, the rest wavelengths mu_k) are formed in FP64 and
// split into an integer cell and an FP32 fraction, so their rounding does not
// move the evaluation point.  The wavelength derivative of the Catmull-Rom
// interpolant is evaluated on first differences D(j) = M(j+1) - M(j) of the
// nodes (exact in FP32 for neighbouring values), with the weights
// e_t = -(dw_0 + ... + dw_t); the same derivative written with the derivative
// weights dw_t directly would cancel column by column.
#pragma once

#include "sb_internal.h"

namespace sbk {

// A value every lane of the workgroup holds equally (read from LDS after a
// barrier, or from a kernel argument), made visibly uniform to the compiler.
// Every loop bound, early exit or branch that encloses a barrier goes through
// it, so the compiler keeps those exits uniform and never splits a wave
// around a barrier.
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Which row projections a pass computes.
//   FWD: Rx                       (flux)
//   FIT: Rx, R1, Rc               (flux, d/dx1, d/dc; d/dt0 from the phase weights)
//   VJP: Rx, R1, Rc, Rl           (all five partials, including z)
enum Mode { FWD = 0, FIT = 1, VJP = 2 };

// NP per-point arrays, NG weight vectors, NR row projections.
//   FWD: P                                   | G               | Rx
//   FIT: P, Pc                               | G, Gc           | Rx, R1, Rc
//   VJP: P, Pc, Plc (4 taps), Pd (3 taps)    | G, Gc, Glc, Gd  | Rx, R1, Rc, Rl
template <int MODE> struct ModeInfo;
template <> struct ModeInfo<FWD> { static constexpr int NP = 4, NG = 1, NR = 1; };
template <> struct ModeInfo<FIT> { static constexpr int NP = 8, NG = 2, NR = 3; };
template <> struct ModeInfo<VJP> { static constexpr int NP = 15, NG = 4, NR = 4; };

// Catmull-Rom (Keys a = -1/2) weights of the four nodes a-1..a+2 at fraction x of
// cell a; linear weights (nodes a, a+1 only) in the first and last cell.
__device__ inline void cr_weights(float x, bool edge, float w[4]) {
  if (edge) {
    w[0] = 0.f; w[1] = 1.f - x; w[2] = x; w[3] = 0.f;
    return;
  }
  const float x2 = x * x, x3 = x2 * x;
  w[0] = -0.5f * x3 + x2 - 0.5f * x;
  w[1] = 1.5f * x3 - 2.5f * x2 + 1.f;
  w[2] = -1.5f * x3 + 2.f * x2 + 0.5f * x;
  w[3] = 0.5f * x3 - 0.5f * x2;
}

// d(weights)/dx of cr_weights.
__device__ inline void cr_dweights(float x, bool edge, float d[4]) {
  if (edge) {
    d[0] = 0.f; d[1] = -1.f; d[2] = 1.f; d[3] = 0.f;
    return;
  }
  const float x2 = x * x;
  d[0] = -1.5f * x2 + 2.f * x - 0.5f;
  d[1] = 4.5f * x2 - 5.f * x;
  d[2] = -4.5f * x2 + 4.f * x + 0.5f;
  d[3] = 1.5f * x2 - x;
}

// The same derivative on first differences: sum_t dw_t M(a-1+t) equals
// sum_{t<3} e_t D(a-1+t) with D(j) = M(j+1) - M(j) and e_t = -(dw_0 + .. + dw_t).
// Edge cells (linear): the derivative is D(a).
__device__ inline void cr_diff_weights(float x, bool edge, float e[3]) {
  if (edge) {
    e[0] = 0.f; e[1] = 1.f; e[2] = 0.f;
    return;
  }
  const float x2 = x * x;
  e[0] = 1.5f * x2 - 2.f * x + 0.5f;
  e[1] = -3.f * x2 + 3.f * x + 0.5f;
  e[2] = 1.5f * x2 - x;
}

// Phase cell of an observation, from FP64 coordinates.  Written with
// contraction off so that every call site rounds identically (row ranges and
// weights must agree).
struct PhaseCell {
  float p;      // rest phase (t - t0) s
  float x;      // fraction in cell a
  int a;        // cell in [0, n_phase - 2]
  bool edge;    // first or last cell: linear
  bool in;      // inside [phase0, phase_max]
  bool nan;     // non-finite input
  int r0, r1;   // rows with non-zero weight
};

__device__ inline PhaseCell phase_cell(float t, float t0, double s, const KModel& m) {
#pragma clang fp contract(off)
  PhaseCell c;
  const double p = ((double)t - (double)t0) * s;
  const double u = (p - m.phase0_d) * m.inv_dphase_d;
  c.p = (float)p;
  c.nan = !(u == u);
  c.in = (u >= 0.0) && (u <= (double)(m.n_phase - 1));
  const double uu = c.in ? u : 0.0;
  int a = (int)floor(uu);
  a = a < 0 ? 0 : (a > m.n_phase - 2 ? m.n_phase - 2 : a);
  c.a = a;
  c.x = (float)(uu - (double)a);
  c.edge = (a == 0) || (a == m.n_phase - 2);
  c.r0 = c.edge ? a : a - 1;
  c.r1 = c.edge ? a + 1 : a + 2;
  return c;
}

// Colour law CL(mu) and dCL/dmu.
__device__ inline void colour_law(float mu, const KModel& m, float& cl, float& dcl) {
  const float r = (mu - m.cl_b) * m.cl_inv_span;
  float v = 0.f, d = 0.f;
  for (int n = m.cl_deg - 1; n >= 0; --n) {
    v = fmaf(v, r, m.cl[n]);
    d = fmaf(d, r, m.dcl[n]);
  }
  cl = v * r;
  dcl = d * m.cl_inv_span;
}

// Pointers into the dynamic LDS of one workgroup.
struct Lds {
  float* P;    // [NP][max_pts]      point weights per tap
  int* j0;     // [max_pts]          wavelength cell per point
  int* kf;     // [n_wave + 2]       first point of each cell
  float* G;    // [NG][n_wave + 4]   weight vectors over the window
  float* RP;   // [NWAVES][64][NR]   per-wave partial row projections
  float* R;    // [n_phase][NR]      row projections of the current band
  int gstride; // n_wave + 4
};

template <int MODE>
__host__ __device__ inline size_t lds_layout_bytes(int n_phase, int n_wave, int max_pts) {
  constexpr int NP = ModeInfo<MODE>::NP, NG = ModeInfo<MODE>::NG, NR = ModeInfo<MODE>::NR;
  size_t b = 0;
  b += (size_t)NP * max_pts * sizeof(float);
  b += (size_t)max_pts * sizeof(int);
  b += (size_t)(n_wave + 2) * sizeof(int);
  b += (size_t)NG * (n_wave + 4) * sizeof(float);
  b += (size_t)NWAVES * 64 * NR * sizeof(float);
  b += (size_t)n_phase * NR * sizeof(float);
  return b;
}

template <int MODE>
__device__ inline Lds lds_carve(char* base, const KModel& m, int max_pts) {
  constexpr int NP = ModeInfo<MODE>::NP, NG = ModeInfo<MODE>::NG, NR = ModeInfo<MODE>::NR;
  Lds L;
  char* p = base;
  L.P = (float*)p;  p += (size_t)NP * max_pts * sizeof(float);
  L.j0 = (int*)p;   p += (size_t)max_pts * sizeof(int);
  L.kf = (int*)p;   p += (size_t)(m.n_wave + 2) * sizeof(int);
  L.G = (float*)p;  p += (size_t)NG * (m.n_wave + 4) * sizeof(float);
  L.RP = (float*)p; p += (size_t)NWAVES * 64 * NR * sizeof(float);
  L.R = (float*)p;
  L.gstride = m.n_wave + 4;
  return L;
}

// Row projections of one (supernova, band) for rows [rlo, rhi]:
//   R[(a - rlo)*NR + 0] = sum_j G(j)  (M0 + x1 M1)[a, j]
//   R[...+1]            = sum_j G(j)  M1[a, j]                          (FIT, VJP)
//   R[...+2]            = sum_j Gc(j) (M0 + x1 M1)[a, j]                (FIT, VJP)
//   R[...+3]            = sum_j Glc(j) (M0 + x1 M1)[a, j]
//                       + sum_j Gd(j) (D0 + x1 D1)[a, j]                (VJP)
// with om_k = W_k exp(c CL(mu_k)) and
//   G(j)   = sum_k om_k wl_j(mu_k),          Gc(j) = sum_k om_k CL(mu_k) wl_j(mu_k),
//   Glc(j) = sum_k om_k mu_k c CL'(mu_k) wl_j(mu_k),
//   Gd(j)  = sum_k om_k mu_k e_j(mu_k) / dwave   (difference weights, D(j) = M(j+1) - M(j)),
// so that Rl gives sum_k om_k mu_k [dI/dmu + c CL' I] at the phase rows.
// All threads of the workgroup must call it (it holds barriers).  Returns
// false, uniformly, when the band's rest window leaves the wavelength grid.
// *flag is an LDS int used as scratch.
template <int MODE>
__device__ bool band_rows(const KModel& m, const KTables& tb, int bd, double s, float c, float x1,
                          int rlo, int rhi, const Lds& L, int* flag) {
  constexpr int NG = ModeInfo<MODE>::NG, NR = ModeInfo<MODE>::NR;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int np = uni(tb.npts[bd]);
  bd = uni(bd);
  rlo = uni(rlo);
  rhi = uni(rhi);
  const float2* pts = tb.pts + (size_t)bd * SB_MAX_BAND_POINTS;
  const int P = tb.max_pts;

  if (tid == 0) *flag = 0;
  __syncthreads();

  // (1) quadrature points: wavelength cell, tap weights times om_k
  for (int k = tid; k < np; k += WG) {
    const float2 lw = pts[k];
    float x, mu;
    int j0;
    bool ok;
    {
#pragma clang fp contract(off)
      const double mu_d = (double)lw.x * s;
      const double v = (mu_d - m.wave0_d) * m.inv_dwave_d;
      ok = (v >= 0.0) && (v <= (double)(m.n_wave - 1));
      const double vv = ok ? v : 0.0;
      j0 = (int)floor(vv);
      j0 = j0 < 0 ? 0 : (j0 > m.n_wave - 2 ? m.n_wave - 2 : j0);
      x = (float)(vv - (double)j0);
      mu = (float)mu_d;
    }
    if (!ok) *flag = 1;
    const bool edge = (j0 == 0) || (j0 == m.n_wave - 2);
    float cl, dcl;
    colour_law(mu, m, cl, dcl);
    const float om = lw.y * expf(c * cl);
    float w[4];
    cr_weights(x, edge, w);
#pragma unroll
    for (int t = 0; t < 4; ++t) L.P[t * P + k] = om * w[t];
    if (MODE != FWD) {
      const float omc = om * cl;
#pragma unroll
      for (int t = 0; t < 4; ++t) L.P[(4 + t) * P + k] = omc * w[t];
    }
    if (MODE == VJP) {
      float e[3];
      cr_diff_weights(x, edge, e);
      const float omu = om * mu;
      const float omlc = omu * (c * dcl);
      const float omd = omu * m.inv_dwave;
#pragma unroll
      for (int t = 0; t < 4; ++t) L.P[(8 + t) * P + k] = omlc * w[t];
#pragma unroll
      for (int t = 0; t < 3; ++t) L.P[(12 + t) * P + k] = omd * e[t];
    }
    L.j0[k] = j0;
  }
  __syncthreads();
  if (uni(*flag)) return false;

  // (2) first point of every wavelength cell touched (cells are non-decreasing in k)
  const int j0f = uni(L.j0[0]), j0l = uni(L.j0[np - 1]);
  const int ncell = j0l - j0f + 1;
  for (int k = tid; k < np; k += WG) {
    // the clamps only keep every index in bounds
    const int cur = min(max(L.j0[k] - j0f, 0), ncell - 1);
    const int prev = (k == 0) ? -1 : min(max(L.j0[k - 1] - j0f, -1), ncell - 1);
    for (int q = prev + 1; q <= cur; ++q) L.kf[q] = k;
  }
  if (tid == 0) L.kf[ncell] = np;
  __syncthreads();

  // (3) weight vectors over the window of columns [j_lo, j_hi]; node tap t and
  //     difference tap t of a point in cell j0 both land on column j0 - 1 + t
  const int j_lo = j0f - 1 < 0 ? 0 : j0f - 1;
  const int j_hi = j0l + 2 > m.n_wave - 1 ? m.n_wave - 1 : j0l + 2;
  const int J = j_hi - j_lo + 1;
  for (int col = tid; col < J; col += WG) {
    const int j = j_lo + col;
    float g[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) g[q] = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int q = j - t + 1 - j0f;   // cell whose tap t lands on column j
      if (q < 0 || q >= ncell) continue;
      const int k1 = min(L.kf[q + 1], np);
      for (int k = max(L.kf[q], 0); k < k1; ++k) {
        g[0] += L.P[t * P + k];
        if (MODE != FWD) g[1] += L.P[(4 + t) * P + k];
        if (MODE == VJP) {
          g[2] += L.P[(8 + t) * P + k];
          if (t < 3) g[3] += L.P[(12 + t) * P + k];
        }
      }
    }
#pragma unroll
    for (int h = 0; h < NG; ++h) L.G[h * L.gstride + col] = g[h];
  }
  __syncthreads();

  // (4) row projections: lanes over rows, waves over quarters of the window
  const int nrow = rhi - rlo + 1;
  const int qc = (J + NWAVES - 1) / NWAVES;
  const int c0 = min(wv * qc, J), c1 = min(c0 + qc, J);
  for (int rb = 0; rb < nrow; rb += 64) {
    const int a = rlo + rb + lane;
    const int a_ld = a < m.n_phase - 1 ? a : m.n_phase - 1;
    const float2* colp = tb.surf + a_ld;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    if (MODE == VJP) {
      // carries the next column for the first differences (clamped at the grid end,
      // where its difference weight is zero)
      float2 cur = colp[(size_t)min(j_lo + c0, m.n_wave - 1) * m.row_pad];
#pragma unroll 4
      for (int cc = c0; cc < c1; ++cc) {
        const float2 nxt = colp[(size_t)min(j_lo + cc + 1, m.n_wave - 1) * m.row_pad];
        const float mx = fmaf(x1, cur.y, cur.x);
        const float dx = fmaf(x1, nxt.y - cur.y, nxt.x - cur.x);
        const float g = L.G[cc];
        acc[0] = fmaf(g, mx, acc[0]);
        acc[1] = fmaf(g, cur.y, acc[1]);
        acc[2] = fmaf(L.G[L.gstride + cc], mx, acc[2]);
        acc[3] = fmaf(L.G[2 * L.gstride + cc], mx, acc[3]);
        acc[3] = fmaf(L.G[3 * L.gstride + cc], dx, acc[3]);
        cur = nxt;
      }
    } else {
      const float2* cp = colp + (size_t)(j_lo + c0) * m.row_pad;
      int cc = c0;
      for (; cc + 4 <= c1; cc += 4) {
        float2 mm[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) mm[u] = cp[(size_t)(cc - c0 + u) * m.row_pad];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float g = L.G[cc + u];
          const float mx = fmaf(x1, mm[u].y, mm[u].x);
          acc[0] = fmaf(g, mx, acc[0]);
          if (MODE == FIT) {
            acc[1] = fmaf(g, mm[u].y, acc[1]);
            acc[2] = fmaf(L.G[L.gstride + cc + u], mx, acc[2]);
          }
        }
      }
      for (; cc < c1; ++cc) {
        const float2 mm = cp[(size_t)(cc - c0) * m.row_pad];
        const float g = L.G[cc];
        const float mx = fmaf(x1, mm.y, mm.x);
        acc[0] = fmaf(g, mx, acc[0]);
        if (MODE == FIT) {
          acc[1] = fmaf(g, mm.y, acc[1]);
          acc[2] = fmaf(L.G[L.gstride + cc], mx, acc[2]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) L.RP[(wv * 64 + lane) * NR + r] = acc[r];
    __syncthreads();
    if (tid < 64 * NR) {
      const int row = tid / NR, r = tid - row * NR;
      if (rb + row < nrow) {
        float v = L.RP[(0 * 64 + row) * NR + r];
#pragma unroll
        for (int w2 = 1; w2 < NWAVES; ++w2) v += L.RP[(w2 * 64 + row) * NR + r];
        L.R[(rb + row) * NR + r] = v;
      }
    }
    __syncthreads();
  }
  return true;
}

// Index of surface row a in the row projections of [rlo, rhi] (clamped into range).
__device__ inline int row_index(int a, int rlo, int rhi) {
  return min(max(a, rlo), rhi) - rlo;
}

// Sum of N values over the workgroup in a fixed order; every thread gets the
// same result (each thread adds the four per-wave partials in wave order).
template <int N>
__device__ inline void block_sum(float (&v)[N], float* red) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    float x = v[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    v[q] = x;
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) red[wv * N + q] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < N; ++q) {
    float x = red[q];
#pragma unroll
    for (int w2 = 1; w2 < NWAVES; ++w2) x += red[w2 * N + q];
    v[q] = x;
  }
  __syncthreads();
}

// Branch-free reset of the per-band scan state (every thread stores the same
// values), so no lane-dependent branch sits in loops that hold barriers.
__device__ inline void reset_scan(unsigned* mask, int* rlo, int* rhi) {
  const int tid = threadIdx.x;
  rlo[tid & (SB_MAX_BANDS - 1)] = 0x7fffffff;
  rhi[tid & (SB_MAX_BANDS - 1)] = -1;
  mask[tid & 1] = 0u;
}

}  // namespace sbk
