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
__device__ inline float uni_f(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }

// Which row projections a pass computes.
//   FWD: Rx                       (flux)
//   FIT: Rx, R1, Rc               (flux, d/dx1, d/dc; d/dt0 from the phase weights)
//   VJP: Rx, R1, Rc, Rl, Rd       (all five partials, including z; Rd projects the phase
//                                  first differences of the nodes, for d/dt0 and d/dz)
enum Mode { FWD = 0, FIT = 1, VJP = 2 };

// Per mode: NG weight vectors, interleaved per point tap and per window column
// as one vector type (float / float2 / float4), and NR row projections.
//   FWD: G                  | Rx
//   FIT: G, Gc              | Rx, R1, Rc
//   VJP: G, Gc, Glc, Gd     | Rx, R1, Rc, Rl, Rd
template <int MODE> struct ModeInfo;
// A workgroup of NW waves (fewer if the LDS for NW waves does not fit; see the
// launches) evaluates one supernova; the bands of a group are
// handed to the waves in turn (wave w takes the group's bands w, w + NW, ...),
// each wave building its bands' weight vectors in its own LDS scratch.  GROUP
// bands have their row projections held in LDS at once, and the observations
// of those bands are finished in one pass by the whole workgroup (an extra group
// costs one more scan of the band ids).  The adjoint's three waves and six-band
// groups give a supernova of five or six bands two bands per wave in one group
// (3-4% faster on 4,096 supernovae than two waves over groups of four, whose
// second group left one wave idle; four waves over eight bands were slower).
// CW is the column chunk of the row projections (columns whose surface loads
// are in flight together).
template <> struct ModeInfo<FWD> { static constexpr int NG = 1, NR = 1, NW = 2, GROUP = 8, CW = 4; typedef float V; };
template <> struct ModeInfo<FIT> { static constexpr int NG = 2, NR = 3, NW = 8, GROUP = 8, CW = 4; typedef float2 V; };
template <> struct ModeInfo<VJP> { static constexpr int NG = 4, NR = 5, NW = 3, GROUP = 6, CW = 4; typedef float4 V; };

// Largest group over the modes (sizes the per-slot flags).
constexpr int BAND_GROUP = 8;

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

// The colour law's coefficients spread over the lanes of a wave: lane n holds
// a_(n+1) in .x and (n+1) a_(n+1) in .y (zero past the degree), so that the
// Horner steps read them with readlane instead of waiting on memory.
__device__ inline float2 colour_coefs(const KModel& m) {
  const int lane = threadIdx.x & (WAVE - 1);
  float2 q = make_float2(0.f, 0.f);
#pragma unroll
  for (int n = 0; n < SB_MAX_CL_DEGREE; ++n)
    if (lane == n) q = make_float2(m.cl[n], m.dcl[n]);
  return q;
}

__device__ inline float lane_f(float v, int n) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), n));
}

// Colour law CL(mu) and dCL/dmu (coefficients q from colour_coefs).
__device__ inline void colour_law(float mu, const KModel& m, float2 q, float& cl, float& dcl) {
  const float r = (mu - m.cl_b) * m.cl_inv_span;
  float v = 0.f, d = 0.f;
  for (int n = m.cl_deg - 1; n >= 0; --n) {
    v = fmaf(v, r, lane_f(q.x, n));
    d = fmaf(d, r, lane_f(q.y, n));
  }
  cl = v * r;
  dcl = d * m.cl_inv_span;
}

// Ordering point for LDS traffic among the lanes of one wave: the wave's LDS
// operations complete in issue order, so only the compiler must not move
// accesses across it.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pointers into the dynamic LDS of one workgroup (one supernova): the calling
// wave's scratch, and the group's row projections shared by the workgroup.
struct Lds {
  void* P;     // [max_pts] of V             weight factors per quadrature point
  float* x;    // [max_pts]                  fraction in the point's wavelength cell
  int* kf;     // [jcap + 2]                 first point of each cell
  int* tag;    // [4] after kf               fit mode: band held in P, x, kf (-1: none), j0f, j0l, np
  void* G;     // [jcap] of V                weight vectors over the window
  float* R;    // [GROUP][n_phase][NR]       row projections of the bands of a group
};

// Bytes of one wave's scratch (16-byte multiple).
template <int MODE>
__host__ __device__ inline size_t wave_scratch_bytes(int max_pts, int jcap) {
  typedef typename ModeInfo<MODE>::V V;
  size_t b = 0;
  b += (size_t)max_pts * sizeof(V);
  b += (size_t)max_pts * sizeof(float);
  b += (size_t)(jcap + 2 + 4) * sizeof(int);
  b = (b + 15) & ~(size_t)15;
  b += (size_t)jcap * sizeof(V);
  return (b + 15) & ~(size_t)15;
}

// Dynamic LDS of a workgroup of nw waves.
template <int MODE>
__host__ __device__ inline size_t lds_layout_bytes(int n_phase, int max_pts, int jcap, int nw) {
  return nw * wave_scratch_bytes<MODE>(max_pts, jcap) +
         (size_t)ModeInfo<MODE>::GROUP * n_phase * ModeInfo<MODE>::NR * sizeof(float);
}

template <int MODE, int NW>
__device__ inline Lds lds_carve(char* base, const KModel& m, const KTables& tb, int wave) {
  typedef typename ModeInfo<MODE>::V V;
  const size_t ws = wave_scratch_bytes<MODE>(tb.max_pts, tb.jcap);
  Lds L;
  size_t o = (size_t)wave * ws;
  L.P = base + o;            o += (size_t)tb.max_pts * sizeof(V);
  L.x = (float*)(base + o);  o += (size_t)tb.max_pts * sizeof(float);
  L.kf = (int*)(base + o);   o += (size_t)(tb.jcap + 2) * sizeof(int);
  L.tag = (int*)(base + o);  o += 4 * sizeof(int);
  o = (o + 15) & ~(size_t)15;
  L.G = base + o;
  L.R = (float*)(base + (size_t)NW * ws);
  return L;
}

template <typename V> __device__ inline V vzero();
template <> __device__ inline float vzero<float>() { return 0.f; }
template <> __device__ inline float2 vzero<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ inline float4 vzero<float4>() { return make_float4(0.f, 0.f, 0.f, 0.f); }

// Tap sums of one wavelength cell over its points k in [k0, k1):
//   C[t] = sum_k wl_t(x_k) P_k      (node tap t lands on column cell - 1 + t)
// and, for the adjoint's difference weights (component w), C[t].w = sum_k
// e_t(x_k) P_k.w for t < 3 (difference D(cell - 1 + t)).  MAY_EDGE false: the
// caller knows that the cell is not a first or last cell of the grid.
template <int MODE, bool MAY_EDGE>
__device__ inline void cell_taps(typename ModeInfo<MODE>::V (&C)[4], const Lds& L, int k0, int k1, bool edge_in,
                                 float c) {
  typedef typename ModeInfo<MODE>::V V;
  const V* Pv = (const V*)L.P;
  const bool edge = MAY_EDGE && edge_in;
  for (int k = k0; k < k1; ++k) {
    const float x = L.x[k];
    V p = Pv[k];
    if constexpr (MODE == FIT) {
      // the fit keeps (W_k, CL(mu_k)), which depend on z only; om_k follows the colour
      const float om = p.x * expf(c * p.y);
      p = make_float2(om, om * p.y);
    }
    float w[4];
    cr_weights(x, edge, w);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if constexpr (MODE == FWD) {
        C[t] = fmaf(p, w[t], C[t]);
      } else {
        C[t].x = fmaf(p.x, w[t], C[t].x);
        C[t].y = fmaf(p.y, w[t], C[t].y);
        if constexpr (MODE == VJP) C[t].z = fmaf(p.z, w[t], C[t].z);
      }
    }
    if constexpr (MODE == VJP) {
      float e[3];
      cr_diff_weights(x, edge, e);
#pragma unroll
      for (int t = 0; t < 3; ++t) C[t].w = fmaf(p.w, e[t], C[t].w);
    }
  }
}

// v plus w of the next lane down: lane L adds lane L - 1's w, lane 0 adds 0 (one DPP wave
// shift fused into the add).
__device__ inline float add_up1(float v, float w) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(w), 0x138, 0xF, 0xF, true));
}
__device__ inline float2 add_up1(float2 v, float2 w) { return make_float2(add_up1(v.x, w.x), add_up1(v.y, w.y)); }
__device__ inline float4 add_up1(float4 v, float4 w) {
  return make_float4(add_up1(v.x, w.x), add_up1(v.y, w.y), add_up1(v.z, w.z), add_up1(v.w, w.w));
}

// Surface nodes (M0, M1) of the lane's row in CW consecutive columns: buffer
// loads with the lane's row offset loff in a vector register and the column's
// byte offset col (uniform) in a scalar register, so no vector address
// arithmetic is spent.  The resource's size bounds every read: lanes past the
// last row pass loff = BUF_OFF_NONE, read zeros and fetch nothing.
template <int CW>
__device__ inline void load_cols(float2 (&v)[CW], __amdgpu_buffer_rsrc_t rs, unsigned loff, int col, int cstride) {
#pragma unroll
  for (int u = 0; u < CW; ++u)
    v[u] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)loff, col + u * cstride, 0));
}

// One window column of the forward / fit row projections: node mc = (M0, M1)
// of the lane's row, weight vector g.
template <int MODE>
__device__ inline void col_step(float (&acc)[5], typename ModeInfo<MODE>::V g, float2 mc, float x1) {
  const float mx = fmaf(x1, mc.y, mc.x);
  if constexpr (MODE == FWD) {
    acc[0] = fmaf(g, mx, acc[0]);
  } else {
    acc[0] = fmaf(g.x, mx, acc[0]);
    acc[1] = fmaf(g.x, mc.y, acc[1]);
    acc[2] = fmaf(g.y, mx, acc[2]);
  }
}

// CW columns held in v; column u goes to chain u mod 4.
template <int MODE, int CW>
__device__ inline void chunk_cols(float (&acc)[4][5], const typename ModeInfo<MODE>::V* g, const float2 (&v)[CW],
                                  float x1) {
#pragma unroll
  for (int u = 0; u < CW; ++u) col_step<MODE>(acc[u & 3], g[u], v[u], x1);
}

// The last rem (< CW, uniform) columns, held in v[0..rem-1].
template <int MODE, int CW>
__device__ inline void tail_cols(float (&acc)[4][5], const typename ModeInfo<MODE>::V* g, const float2 (&v)[CW],
                                 int rem, float x1) {
#pragma unroll
  for (int u = 0; u < CW - 1; ++u)
    if (u < rem) col_step<MODE>(acc[u & 3], g[u], v[u], x1);
}

// The combined node of the next row (lane + 1) minus this lane's: one DPP
// wave shift (lane L reads lane L + 1; the last lane reads 0 and its value is
// never used).
__device__ inline float next_row_diff(float mx) {
  const float nx = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(mx), 0x130, 0xF, 0xF, true));
  return nx - mx;
}

// One window column j of the adjoint's row projections from the lane's row
// nodes cur = (M0, M1)(j), with the previous column's combined node prev =
// (M0 + x1 M1)(j-1) and difference weight gdp: the first difference of the
// combined nodes, mx(j) - mx(j-1), is formed here and its term goes to the
// previous column's chain, after that column's own terms, so every chain sums
// in column order.  The phase first difference mx(a+1, j) - mx(a, j) (the next
// row is the next lane) goes to Rd with the flux weight.  Chains are window
// columns mod 4 (U = this one's).
template <int U>
__device__ inline void col_step_d(float (&acc)[4][5], float4 g, float2 cur, float& prev, float& gdp, float x1) {
  constexpr int P = (U + 3) & 3;
  const float mx = fmaf(x1, cur.y, cur.x);
  acc[P][3] = fmaf(gdp, mx - prev, acc[P][3]);
  acc[U][0] = fmaf(g.x, mx, acc[U][0]);
  acc[U][1] = fmaf(g.x, cur.y, acc[U][1]);
  acc[U][2] = fmaf(g.y, mx, acc[U][2]);
  acc[U][3] = fmaf(g.z, mx, acc[U][3]);
  acc[U][4] = fmaf(g.x, next_row_diff(mx), acc[U][4]);
  prev = mx;
  gdp = g.w;
}

template <int CW>
__device__ inline void chunk_cols_d(float (&acc)[4][5], const float4* g, const float2 (&v)[CW], float& prev,
                                    float& gdp, float x1) {
  static_assert(CW == 4, "one chunk is one column per chain");
  col_step_d<0>(acc, g[0], v[0], prev, gdp, x1);
  col_step_d<1>(acc, g[1], v[1], prev, gdp, x1);
  col_step_d<2>(acc, g[2], v[2], prev, gdp, x1);
  col_step_d<3>(acc, g[3], v[3], prev, gdp, x1);
}

// The difference term of the window's last column, on chain P, from the nodes
// of the column after the window, nx.  Its weight is zero; the term is kept so that every chain
// ends as the column loop leaves it.
template <int P>
__device__ inline void close_chain(float (&acc)[4][5], float2 nx, float prev, float gdp, float x1) {
  acc[P][3] = fmaf(gdp, fmaf(x1, nx.y, nx.x) - prev, acc[P][3]);
}

// The last rem (< 4) window columns, held in v[0 .. rem-1], and the closing
// difference term from v[rem] (branches on the uniform rem, static indices only).
__device__ inline void tail_cols_d(float (&acc)[4][5], const float4* g, const float2 (&v)[4], int rem,
                                   float& prev, float& gdp, float x1) {
  if (rem == 0) {
    close_chain<3>(acc, v[0], prev, gdp, x1);
    return;
  }
  col_step_d<0>(acc, g[0], v[0], prev, gdp, x1);
  if (rem == 1) {
    close_chain<0>(acc, v[1], prev, gdp, x1);
    return;
  }
  col_step_d<1>(acc, g[1], v[1], prev, gdp, x1);
  if (rem == 2) {
    close_chain<1>(acc, v[2], prev, gdp, x1);
    return;
  }
  col_step_d<2>(acc, g[2], v[2], prev, gdp, x1);
  close_chain<2>(acc, v[3], prev, gdp, x1);
}

// Rest wavelength mu = lam s of a quadrature point and its wavelength cell j0
// and fraction x, from FP64 coordinates (contraction off, so every call site
// rounds identically).  ok: mu on the wavelength grid.  The cell is
// non-decreasing in lam.
struct WaveCell {
  float x, mu;
  int j0;
  bool ok;
};

__device__ inline WaveCell wave_cell(float lam, double s, const KModel& m) {
#pragma clang fp contract(off)
  WaveCell w;
  const double mu_d = (double)lam * s;
  const double v = (mu_d - m.wave0_d) * m.inv_dwave_d;
  w.ok = (v >= 0.0) && (v <= (double)(m.n_wave - 1));
  const double vv = w.ok ? v : 0.0;
  int j0 = (int)floor(vv);
  j0 = j0 < 0 ? 0 : (j0 > m.n_wave - 2 ? m.n_wave - 2 : j0);
  w.j0 = j0;
  w.x = (float)(vv - (double)j0);
  w.mu = (float)mu_d;
  return w;
}

// Quadrature point k of a band, (lam_k, W_k) = lw, for a supernova with
// s = 1/(1+z) and colour c: its fraction x and weight factors P (om_k = W_k
// exp(c CL(mu_k)), and per mode om_k CL, om_k mu_k c CL', om_k mu_k / dwave;
// the fit stores (W_k, CL(mu_k)) and applies the colour in the weight pass)
// into the wave's scratch, if k < np.  Every lane of the wave calls it (the
// colour law reads its coefficients across lanes).  Returns the point's
// wavelength cell.
template <int MODE>
__device__ inline int point_setup(const KModel& m, double s, float c, float2 clq, float2 lw, int k, int np,
                                  const Lds& L) {
  typedef typename ModeInfo<MODE>::V V;
  const WaveCell w = wave_cell(lw.x, s, m);
  float cl, dcl;
  colour_law(w.mu, m, clq, cl, dcl);
  if constexpr (MODE == FIT) {
    // the colour factor is applied in the weight pass (cell_taps)
    if (k < np) {
      ((V*)L.P)[k] = make_float2(lw.y, cl);
      L.x[k] = w.x;
    }
    return w.j0;
  }
  const float om = lw.y * expf(c * cl);
  if (k < np) {
    V* Pv = (V*)L.P;
    if constexpr (MODE == FWD) {
      Pv[k] = om;
    } else if constexpr (MODE == VJP) {
      const float omu = om * w.mu;
      Pv[k] = make_float4(om, om * cl, omu * (c * dcl), omu * m.inv_dwave);
    }
    L.x[k] = w.x;
  }
  return w.j0;
}

// Row projections of one (supernova, band) for rows [rlo, rhi], written to
// Rb[a*NR + r] for the absolute row a:
//   r=0  sum_j G(j)  (M0 + x1 M1)[a, j]
//   r=1  sum_j G(j)  M1[a, j]                          (FIT, VJP)
//   r=2  sum_j Gc(j) (M0 + x1 M1)[a, j]                (FIT, VJP)
//   r=3  sum_j Glc(j) (M0 + x1 M1)[a, j]
//        + sum_j Gd(j) D[a, j]                         (VJP)
//   r=4  sum_j G(j) ((M0 + x1 M1)[a+1, j] - (M0 + x1 M1)[a, j])   (VJP, rows a < rhi)
// with om_k = W_k exp(c CL(mu_k)) and
//   G(j)   = sum_k om_k wl_j(mu_k),          Gc(j) = sum_k om_k CL(mu_k) wl_j(mu_k),
//   Glc(j) = sum_k om_k mu_k c CL'(mu_k) wl_j(mu_k),
//   Gd(j)  = sum_k om_k mu_k e_j(mu_k) / dwave   (difference weights on the first
//            differences D(j) = (M0 + x1 M1)(j+1) - (M0 + x1 M1)(j) of the combined nodes),
// so that r=3 gives sum_k om_k mu_k [dI/dmu + c CL' I] at the phase rows.
// Every lane of one wave calls it, with that wave's scratch in L; it
// synchronises only within the wave.  Returns false, uniformly, when the band's
// rest window leaves the wavelength grid (or exceeds the window capacity, which
// covers z >= WINDOW_Z_MIN).
template <int MODE>
__device__ bool band_rows(const KModel& m, const KTables& tb, int bd, double s, float c, float x1,
                          int rlo, int rhi, const Lds& L, float* Rb) {
  typedef typename ModeInfo<MODE>::V V;
  constexpr int NR = ModeInfo<MODE>::NR;
  const int lane = threadIdx.x & (WAVE - 1);
  bd = uni(bd);
  rlo = uni(rlo);
  rhi = uni(rhi);
  V* Gv = (V*)L.G;

  // A fit evaluates the same bands at the same redshift in every iteration: the
  // points' cells, fractions, colour law and the cell table depend on z only, so
  // a wave whose scratch already holds this band (tag) goes straight to (3).
  bool cached = false;
  if constexpr (MODE == FIT) cached = uni(L.tag[0] == bd ? 1 : 0) != 0;
  int np, j0f, j0l;
  float2 cur = make_float2(0.f, 0.f);
  const float2* pts = tb.pts + (size_t)bd * SB_MAX_BAND_POINTS;
  if (cached) {
    j0f = uni(L.tag[1]);
    j0l = uni(L.tag[2]);
    np = uni(L.tag[3]);
  } else {
    np = uni(tb.npts[bd]);
    // the first pass's points, and the band's first and last point (lanes 0 and
    // 1 of one load), are requested before anything waits on memory
    cur = lane < np ? pts[lane] : make_float2(0.f, 0.f);
    const float ends = pts[lane == 0 ? 0 : np - 1].x;
    // the window: the cells of the first and last points (cells are non-decreasing
    // in k, so every point is on the grid if these two are)
    const WaveCell wf = wave_cell(lane_f(ends, 0), s, m), wl = wave_cell(lane_f(ends, 1), s, m);
    if (!uni(wf.ok && wl.ok ? 1 : 0)) return false;
    j0f = uni(wf.j0);
    j0l = uni(wl.j0);
  }
  const int ncell = j0l - j0f + 1;
  const int j_lo = j0f - 1 < 0 ? 0 : j0f - 1;
  const int j_hi = j0l + 2 > m.n_wave - 1 ? m.n_wave - 1 : j0l + 2;
  const int J = j_hi - j_lo + 1;
  if (J > tb.jcap) return false;

  // (1) quadrature points: fraction and weight factors into LDS; and (2) the
  //     first point of every cell, kf[q] (cell j0f + q): a point whose cell is
  //     above the previous point's starts the cells in between.  The previous
  //     point's cell comes from the lane below, or for lane 0 from the last
  //     point of the previous pass.  Each pass requests the next pass's points
  //     before it works on its own.
  if (!cached) {
  const float2 clq = colour_coefs(m);
  int carry = j0f - 1;
  for (int k0 = 0; k0 < np; k0 += WAVE) {
    const int k = k0 + lane;
    const float2 nxt = k + WAVE < np ? pts[k + WAVE] : make_float2(0.f, 0.f);
    int j0 = point_setup<MODE>(m, s, c, clq, cur, k, np, L);
    if (k >= np) j0 = j0l;
    cur = nxt;
    int prev = __shfl_up(j0, 1, WAVE);
    if (lane == 0) prev = carry;
    if (k < np)
      for (int q = prev + 1; q <= j0; ++q) L.kf[q - j0f] = k;
    carry = __builtin_amdgcn_readlane(j0, min(np - k0, WAVE) - 1);
  }
  if (lane == 0) {
    L.kf[ncell] = np;
    if (MODE == FIT) {
      L.tag[0] = bd;
      L.tag[1] = j0f;
      L.tag[2] = j0l;
      L.tag[3] = np;
    }
  }
  }
  wave_sync();

  // (3) weight vectors over the window of columns [j_lo, j_hi].  Lane L of a
  //     pass starting at column b takes column b + L and the cell just above
  //     it, j_lo + b + L + 1, and sums the four taps of that cell's points
  //     (each point read once).  Column b + L needs tap t of the cell t below
  //     that one, held by lane L - t: G = C0 + up(C1 + up(C2 + up(C3))), each
  //     "+ up" one DPP-shifted add.  Passes start 3 columns early and advance by WAVE - 3, so every tap a
  //     written column needs comes from a lane of the same pass.
  //     Only a window that reaches the grid's first or last cell can hold an
  //     edge cell, so other windows take the branch without the edge weights.
  const bool win_edge = uni(j0f == 0 || j0l >= m.n_wave - 2 ? 1 : 0);
  for (int b = -3; b + 3 < J; b += WAVE - 3) {
    const int col = b + lane;
    const int cell = j_lo + col + 1;
    const int q = cell - j0f;
    // lanes without a cell of the window run an empty point range (one code path,
    // so the tap sums are zeroed once)
    const bool has = q >= 0 && q < ncell;
    const int qc = has ? q : 0;
    const int k0 = max(L.kf[qc], 0), k1 = has ? min(L.kf[qc + 1], np) : k0;
    V C[4] = {vzero<V>(), vzero<V>(), vzero<V>(), vzero<V>()};
    if (win_edge)
      cell_taps<MODE, true>(C, L, k0, k1, (cell == 0) || (cell == m.n_wave - 2), c);
    else
      cell_taps<MODE, false>(C, L, k0, k1, false, c);
    // lanes 0..2 write nothing, so the zero shifted into lane 0 never reaches a written column
    V g = add_up1(C[2], C[3]);
    g = add_up1(C[1], g);
    g = add_up1(C[0], g);
    if (lane >= 3 && col < J) Gv[col] = g;
  }
  wave_sync();

  // (4) row projections: lanes over rows, the wave over every window column in
  //     chunks of CW columns (4 for the adjoint); the loads of the next chunk are
  //     issued before the current one is summed (two register buffers in turn).
  //     The column address is uniform (scalar) plus the lane's fixed row offset,
  //     and the padding columns after the grid keep every prefetch in bounds.
  const int nrow = rhi - rlo + 1;
  if constexpr (MODE == VJP) {
    // the adjoint reads the node surface like the other modes and forms the
    // first differences of the combined nodes on the way (see col_step_d).  A
    // pass covers 64 rows and advances by 63: the phase difference of a pass's
    // last row needs the row after it, which the next pass holds in its first lane.
    const int cstride = m.row_pad * (int)sizeof(float2);
    const int n4 = J >> 2, rem = J & 3;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)tb.surf, 0, tb.surf_bytes, BUF_RSRC_WORD3);
    for (int rb = 0;; rb += WAVE - 1) {
      const int a = rlo + rb + lane;
      const unsigned loff = rb + lane < nrow ? (unsigned)a * (unsigned)sizeof(float2) : BUF_OFF_NONE;
      const int cb = j_lo * cstride;
      float acc[4][5];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int r = 0; r < 5; ++r) acc[u][r] = 0.f;
      float prev = 0.f;
      float gdp = 0.f;
      float2 A[4], B[4];
      load_cols<4>(A, rs, loff, cb, cstride);
      int c = 0;
      for (; c + 2 <= n4; c += 2) {
        load_cols<4>(B, rs, loff, cb + (4 * c + 4) * cstride, cstride);
        chunk_cols_d<4>(acc, Gv + 4 * c, A, prev, gdp, x1);
        load_cols<4>(A, rs, loff, cb + (4 * c + 8) * cstride, cstride);
        chunk_cols_d<4>(acc, Gv + 4 * c + 4, B, prev, gdp, x1);
      }
      if (c < n4) {
        load_cols<4>(B, rs, loff, cb + (4 * c + 4) * cstride, cstride);
        chunk_cols_d<4>(acc, Gv + 4 * c, A, prev, gdp, x1);
        tail_cols_d(acc, Gv + 4 * c + 4, B, rem, prev, gdp, x1);
      } else {
        tail_cols_d(acc, Gv + 4 * c, A, rem, prev, gdp, x1);
      }
      if (rb + lane < nrow) {
#pragma unroll
        for (int r = 0; r < NR - 1; ++r) Rb[a * NR + r] = (acc[0][r] + acc[1][r]) + (acc[2][r] + acc[3][r]);
      }
      // Rd(a) for a < rhi (the last row has no successor)
      if (lane < WAVE - 1 && rb + lane < nrow - 1)
        Rb[a * NR + 4] = (acc[0][4] + acc[1][4]) + (acc[2][4] + acc[3][4]);
      if (rb + WAVE - 1 >= nrow - 1) break;
    }
    wave_sync();
    return true;
  }
  constexpr int CW = ModeInfo<MODE>::CW;
  const int cstride = m.row_pad * (int)sizeof(float2);
  const int nc = J / CW, rem = J % CW;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)tb.surf, 0, tb.surf_bytes, BUF_RSRC_WORD3);
  for (int rb = 0; rb < nrow; rb += 64) {
    const int a = rlo + rb + lane;
    const unsigned loff = rb + lane < nrow ? (unsigned)a * (unsigned)sizeof(float2) : BUF_OFF_NONE;
    const int cb = j_lo * cstride;
    float acc[4][5];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int r = 0; r < 5; ++r) acc[u][r] = 0.f;
    float2 A[CW], B[CW];
    load_cols<CW>(A, rs, loff, cb, cstride);
    int c = 0;
    for (; c + 2 <= nc; c += 2) {
      load_cols<CW>(B, rs, loff, cb + (CW * c + CW) * cstride, cstride);
      chunk_cols<MODE, CW>(acc, Gv + CW * c, A, x1);
      load_cols<CW>(A, rs, loff, cb + (CW * c + 2 * CW) * cstride, cstride);
      chunk_cols<MODE, CW>(acc, Gv + CW * c + CW, B, x1);
    }
    if (c < nc) {
      load_cols<CW>(B, rs, loff, cb + (CW * c + CW) * cstride, cstride);
      chunk_cols<MODE, CW>(acc, Gv + CW * c, A, x1);
      tail_cols<MODE, CW>(acc, Gv + CW * c + CW, B, rem, x1);
    } else {
      tail_cols<MODE, CW>(acc, Gv + CW * c, A, rem, x1);
    }
    if (rb + lane < nrow) {
#pragma unroll
      for (int r = 0; r < NR; ++r) Rb[a * NR + r] = (acc[0][r] + acc[1][r]) + (acc[2][r] + acc[3][r]);
    }
  }
  wave_sync();
  return true;
}

// Row projections of every band of a group (masks g0, g1; uniform), into the
// slots 0, 1, ... of L.R in ascending band order.  Wave w takes the group's
// bands w, w + NW, ...  Lane 0 of the wave records the band's slot and whether
// its window could be evaluated.  All threads of the workgroup call it; the
// caller synchronises the workgroup before the projections are read.
template <int MODE, int NW>
__device__ void group_rows(const KModel& m, const KTables& tb, unsigned g0, unsigned g1, double s, float c, float x1,
                           const int* rlo, const int* rhi, int* slot_of, int* slot_ok, const Lds& L, int* err) {
  constexpr int NR = ModeInfo<MODE>::NR;
  const int wv = uni((int)(threadIdx.x / WAVE)), lane = threadIdx.x & (WAVE - 1);
  int sl = 0;
  for (int h = 0; h < 2; ++h) {
    unsigned gm = h ? g1 : g0;
    while (gm) {
      const int bd = h * 32 + __ffs(gm) - 1;
      gm &= gm - 1;
      if (sl % NW == wv) {
        const bool ok = band_rows<MODE>(m, tb, bd, s, c, x1, uni(rlo[bd]), uni(rhi[bd]), L,
                                        L.R + (size_t)sl * m.n_phase * NR);
        if (lane == 0) {
          slot_of[bd] = sl;
          slot_ok[sl] = ok ? 1 : 0;
          if (!ok) atomicOr(err, EFLAG_WINDOW);
        }
      }
      ++sl;
    }
  }
}

// Row a clamped into [rlo, rhi] (the rows whose projections were computed).
__device__ inline int row_clamp(int a, int rlo, int rhi) { return min(max(a, rlo), rhi); }

// Next group of up to cap bands, lowest ids first, taken out of the remaining
// band mask (all values uniform).
__device__ inline void take_group(unsigned& rem0, unsigned& rem1, unsigned& g0, unsigned& g1, int cap) {
  g0 = g1 = 0u;
  for (int n = 0; n < cap && (rem0 | rem1); ++n) {
    if (rem0) {
      const unsigned bit = rem0 & (0u - rem0);
      g0 |= bit;
      rem0 &= ~bit;
    } else {
      const unsigned bit = rem1 & (0u - rem1);
      g1 |= bit;
      rem1 &= ~bit;
    }
  }
}

// Sum over the 64 lanes of a wave; every lane receives the same value.  A
// butterfly in ascending distance: distances 1 and 2 are quad permutes, and 4
// and 8 are the row half-mirror and mirror, which pair a lane with a partner
// holding the same partial sum as its xor partner (after the shorter distances
// every lane of a 4- or 8-lane group holds the same bits, float addition being
// commutative); 16 and 32 cross rows through the LDS permute unit.
template <int CTRL>
__device__ inline float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
__device__ inline float wave_sum(float x) {
  x += dpp_mov<0xB1>(x);    // quad_perm [1,0,3,2]: lane ^ 1
  x += dpp_mov<0x4E>(x);    // quad_perm [2,3,0,1]: lane ^ 2
  x += dpp_mov<0x141>(x);   // row_half_mirror: 7 - lane within 8 (same sum as lane ^ 4)
  x += dpp_mov<0x140>(x);   // row_mirror: 15 - lane within 16 (same sum as lane ^ 8)
  x += __shfl_xor(x, 16, WAVE);
  x += __shfl_xor(x, 32, WAVE);
  return x;
}

// Floats of the reduction scratch block_sum<N, NW> needs: the waves'
// partials and the result, each padded to a multiple of 4.
constexpr int red_pad(int n) { return (n + 3) & ~3; }
constexpr int red_floats(int n, int nw) { return (nw + 1) * red_pad(n); }

// Sum of N values over a workgroup of NW waves in a fixed order; every thread
// gets the same result.  Each wave sums its lanes (wave_sum), lane 0 stores the
// wave's partials, thread q < N adds them in wave order, and every thread reads
// the N sums.  red holds red_floats(N, NW) floats.
template <int N, int NW>
__device__ inline void block_sum(float (&v)[N], float* red) {
  constexpr int NP = red_pad(N);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) red[wv * NP + q] = v[q];
  }
  __syncthreads();
  if (tid < N) {
    float x = red[tid];
#pragma unroll
    for (int w2 = 1; w2 < NW; ++w2) x += red[w2 * NP + tid];
    red[NW * NP + tid] = x;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] = red[NW * NP + q];
}

// Branch-free reset of the per-band scan state (every thread stores the same
// values), so no lane-dependent branch sits in loops that hold barriers.
__device__ inline void reset_scan(unsigned* mask, int* rlo, int* rhi, int* slot_of) {
  const int tid = threadIdx.x;
  rlo[tid & (SB_MAX_BANDS - 1)] = 0x7fffffff;
  rhi[tid & (SB_MAX_BANDS - 1)] = -1;
  slot_of[tid & (SB_MAX_BANDS - 1)] = -1;
  mask[tid & 1] = 0u;
}

}  // namespace sbk
