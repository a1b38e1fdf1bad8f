// Bounded limited-memory quasi-Newton fit step (L-BFGS-B) of the fit kernel.
//
// The paper's optimisation example fits x0, x1, t0, c with L-BFGS-B (section
// "Implementation", the example scripts).  The method is that of Byrd, Lu,
// Nocedal and Zhu (SIAM J. Sci. Comput. 16, 1995), here on the four unknowns
// q = (t0, ln x0, x1, c) with bounds lo <= q <= hi and objective chi2(q):
//   - quasi-Newton matrix: B = theta I updated by BFGS with the kept pairs
//     (oldest first), the dense form of their compact representation;
//   - generalized Cauchy point: the first local minimiser of the quadratic model
//     along the projected steepest-descent path, segment by segment between the
//     breakpoints where a variable reaches a bound;
//   - subspace step: the model minimised over the variables not at a bound at
//     the Cauchy point, cut back to the box (direct primal method);
//   - line search along d = xbar - q, step at most the largest feasible one,
//     first trial min(1/|d|, max) after a (re)start and min(1, max) otherwise,
//     ending on chi2(q + a d) <= chi2 + FTOL a g.d and |g(q + a d).d| <= GTOL |g.d|
//     (a bracketing search with safeguarded cubic interpolation);
//   - a new pair (s, y) is kept only if s.y > eps y.y.
// Each kernel iteration is one evaluation of chi2 and its gradient (the fit's
// iteration budget counts evaluations).  One thread runs this logic on the
// state in LDS between evaluations; every thread reads the trial point.
#pragma once

#include "sb_internal.h"

namespace sbk {

constexpr float LB_FTOL = 1e-3f;
constexpr float LB_GTOL = 0.9f;
constexpr int LB_MAX_LS = 20;

enum : int { LB_NEED_DIR = 0, LB_IN_LS = 1, LB_DONE = 2 };

// B = theta I updated by BFGS with the n kept pairs (S[i], Y[i]), oldest first.
__device__ inline void lb_matrix(const FitSlot& st, float B[4][4]) {
  float theta = 1.f;
  if (st.lb_n > 0) {
    const float* s = st.lb_S[st.lb_n - 1];
    const float* y = st.lb_Y[st.lb_n - 1];
    float yy = 0.f, sy = 0.f;
    for (int i = 0; i < 4; ++i) {
      yy = fmaf(y[i], y[i], yy);
      sy = fmaf(s[i], y[i], sy);
    }
    theta = yy / sy;
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) B[i][j] = i == j ? theta : 0.f;
  for (int p = 0; p < st.lb_n; ++p) {
    const float* s = st.lb_S[p];
    const float* y = st.lb_Y[p];
    float Bs[4];
    float sBs = 0.f, ys = 0.f;
    for (int i = 0; i < 4; ++i) {
      float v = 0.f;
      for (int j = 0; j < 4; ++j) v = fmaf(B[i][j], s[j], v);
      Bs[i] = v;
    }
    for (int i = 0; i < 4; ++i) {
      sBs = fmaf(s[i], Bs[i], sBs);
      ys = fmaf(y[i], s[i], ys);
    }
    const float a = 1.f / sBs, b = 1.f / ys;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) B[i][j] = fmaf(y[i] * b, y[j], fmaf(-Bs[i] * a, Bs[j], B[i][j]));
  }
}

__device__ inline float dot4(const float* a, const float* b) {
  float v = 0.f;
  for (int i = 0; i < 4; ++i) v = fmaf(a[i], b[i], v);
  return v;
}

// d^T B v
__device__ inline float quad4(const float B[4][4], const float* d, const float* v) {
  float r = 0.f;
  for (int i = 0; i < 4; ++i) {
    float w = 0.f;
    for (int j = 0; j < 4; ++j) w = fmaf(B[i][j], v[j], w);
    r = fmaf(d[i], w, r);
  }
  return r;
}

// Generalized Cauchy point xc from x with gradient g, bounds lo/hi, matrix B.
__device__ inline void lb_cauchy(const float* x, const float* g, const float* lo, const float* hi, const float B[4][4],
                                 float* xc) {
  const float inf = __builtin_inff();
  float tb[4], d[4], z[4];
  for (int i = 0; i < 4; ++i) {
    tb[i] = g[i] < 0.f ? (x[i] - hi[i]) / g[i] : (g[i] > 0.f ? (x[i] - lo[i]) / g[i] : inf);
    d[i] = tb[i] > 0.f ? -g[i] : 0.f;
    z[i] = 0.f;
  }
  // breakpoints in increasing order (ties by index)
  int ord[4] = {0, 1, 2, 3};
  for (int i = 1; i < 4; ++i)
    for (int j = i; j > 0 && tb[ord[j]] < tb[ord[j - 1]]; --j) {
      const int t = ord[j];
      ord[j] = ord[j - 1];
      ord[j - 1] = t;
    }
  float t_old = 0.f;
  for (int k = 0; k < 4; ++k) {
    const int b = ord[k];
    if (!(tb[b] > 0.f) || !(tb[b] < inf)) continue;
    const float fp = dot4(g, d) + quad4(B, d, z);
    const float fpp = quad4(B, d, d);
    if (fp >= 0.f) {
      for (int i = 0; i < 4; ++i) xc[i] = x[i] + z[i];
      return;
    }
    const float dt = tb[b] - t_old;
    const float dt_min = fpp > 0.f ? -fp / fpp : inf;
    if (dt_min < dt) {
      for (int i = 0; i < 4; ++i) xc[i] = fmaf(dt_min, d[i], x[i] + z[i]);
      return;
    }
    for (int i = 0; i < 4; ++i) z[i] = fmaf(dt, d[i], z[i]);
    z[b] = (d[b] > 0.f ? hi[b] : lo[b]) - x[b];
    d[b] = 0.f;
    t_old = tb[b];
  }
  const float fp = dot4(g, d) + quad4(B, d, z);
  const float fpp = quad4(B, d, d);
  bool any = false;
  for (int i = 0; i < 4; ++i) any |= d[i] != 0.f;
  if (fp >= 0.f || !any) {
    for (int i = 0; i < 4; ++i) xc[i] = x[i] + z[i];
    return;
  }
  const float dt_min = fpp > 0.f ? -fp / fpp : 0.f;
  for (int i = 0; i < 4; ++i) xc[i] = fmaf(dt_min, d[i], x[i] + z[i]);
}

// Subspace step from xc over the variables strictly inside their bounds, cut back
// to the box.  False if the reduced matrix is not positive definite.
__device__ inline bool lb_subspace(const float* x, const float* g, const float* lo, const float* hi,
                                   const float B[4][4], const float* xc, float* xbar) {
  bool fr[4];
  int nf = 0;
  for (int i = 0; i < 4; ++i) {
    fr[i] = xc[i] > lo[i] && xc[i] < hi[i];
    nf += fr[i];
    xbar[i] = xc[i];
  }
  if (nf == 0) return true;
  float dz[4], r[4];
  for (int i = 0; i < 4; ++i) dz[i] = xc[i] - x[i];
  for (int i = 0; i < 4; ++i) {
    float v = g[i];
    for (int j = 0; j < 4; ++j) v = fmaf(B[i][j], dz[j], v);
    r[i] = v;
  }
  // Cholesky of B over the free variables (held rows and columns as the identity's)
  float a[4][4], rhs[4];
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j < 4; ++j) a[i][j] = (fr[i] && fr[j]) ? B[i][j] : (i == j ? 1.f : 0.f);
    rhs[i] = fr[i] ? -r[i] : 0.f;
  }
  float l[4][4] = {};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j <= i; ++j) {
      float s = a[i][j];
      for (int p = 0; p < j; ++p) s = fmaf(-l[i][p], l[j][p], s);
      if (i == j) {
        if (!(s > 0.f) || !isfinite(s)) return false;
        l[i][i] = sqrtf(s);
      } else {
        l[i][j] = s / l[j][j];
      }
    }
  float y[4], dF[4];
  for (int i = 0; i < 4; ++i) {
    float s = rhs[i];
    for (int p = 0; p < i; ++p) s = fmaf(-l[i][p], y[p], s);
    y[i] = s / l[i][i];
  }
  for (int i = 3; i >= 0; --i) {
    float s = y[i];
    for (int p = i + 1; p < 4; ++p) s = fmaf(-l[p][i], dF[p], s);
    dF[i] = s / l[i][i];
  }
  float alpha = 1.f;
  for (int i = 0; i < 4; ++i) {
    if (!fr[i]) continue;
    if (dF[i] > 0.f) alpha = fminf(alpha, (hi[i] - xc[i]) / dF[i]);
    else if (dF[i] < 0.f) alpha = fminf(alpha, (lo[i] - xc[i]) / dF[i]);
  }
  for (int i = 0; i < 4; ++i)
    if (fr[i]) xbar[i] = fmaf(alpha, dF[i], xc[i]);
  return true;
}

// Minimiser of the cubic through (a, fa, ga), (b, fb, gb), kept 0.1 of the
// interval away from its ends; the midpoint if the cubic has none.
__device__ inline float lb_cubic(float a, float fa, float ga, float b, float fb, float gb) {
  const float lo = fminf(a, b), hi = fmaxf(a, b), w = hi - lo;
  const float d1 = ga + gb - 3.f * (fa - fb) / (a - b);
  const float disc = d1 * d1 - ga * gb;
  if (disc < 0.f) return 0.5f * (a + b);
  const float d2 = copysignf(sqrtf(disc), b - a);
  const float den = gb - ga + 2.f * d2;
  if (den == 0.f) return 0.5f * (a + b);
  const float x = b - (b - a) * (gb + d2 - d1) / den;
  return fminf(fmaxf(x, lo + 0.1f * w), hi - 0.1f * w);
}

// The gradient of chi2 at the state's point (the fit keeps g = J^T W r).
__device__ inline void lb_grad(const float* gls, float* gf) {
  for (int i = 0; i < 4; ++i) gf[i] = -2.f * gls[i];
}

// Plans the next evaluation: a new search direction if needed, then the trial
// point into st.lb_trial.  False when the fit has nothing more to evaluate.
__device__ inline bool lb_plan(FitSlot& st, int fit_iters) {
  if (st.status != SB_OK || st.iter >= fit_iters || st.lb_phase == LB_DONE) return false;
  if (st.lb_phase == LB_NEED_DIR) {
    float gf[4], B[4][4], xc[4], xbar[4];
    lb_grad(st.g, gf);
    bool ok = false;
    for (int attempt = 0; attempt < 2 && !ok; ++attempt) {
      lb_matrix(st, B);
      lb_cauchy(st.q, gf, st.lb_lo, st.lb_hi, B, xc);
      const bool sub = lb_subspace(st.q, gf, st.lb_lo, st.lb_hi, B, xc, xbar);
      bool any = false;
      float gd = 0.f;
      for (int i = 0; i < 4; ++i) {
        st.lb_d[i] = xbar[i] - st.q[i];
        any |= st.lb_d[i] != 0.f;
        gd = fmaf(gf[i], st.lb_d[i], gd);
      }
      if (sub && !any) {
        st.lb_phase = LB_DONE;   // projected gradient zero: stationary
        return false;
      }
      if (sub && gd < 0.f) {
        st.lb_gd = gd;
        ok = true;
      } else if (st.lb_n > 0) {
        st.lb_n = 0;             // not a descent direction: restart from steepest descent
        st.lb_first = 1;
      } else {
        break;
      }
    }
    if (!ok) {
      st.lb_phase = LB_DONE;
      return false;
    }
    float amax = __builtin_inff(), dn = 0.f;
    for (int i = 0; i < 4; ++i) {
      if (st.lb_d[i] > 0.f) amax = fminf(amax, (st.lb_hi[i] - st.q[i]) / st.lb_d[i]);
      else if (st.lb_d[i] < 0.f) amax = fminf(amax, (st.lb_lo[i] - st.q[i]) / st.lb_d[i]);
      dn = fmaf(st.lb_d[i], st.lb_d[i], dn);
    }
    st.lb_amax = amax;
    st.lb_a = st.lb_first ? fminf(1.f / sqrtf(dn), amax) : fminf(1.f, amax);
    st.lb_alo = 0.f;
    st.lb_flo = st.chi2;
    st.lb_glo = st.lb_gd;
    st.lb_has_hi = 0;
    st.lb_trials = 0;
    st.lb_phase = LB_IN_LS;
  }
  for (int i = 0; i < 4; ++i) st.lb_trial[i] = fminf(fmaxf(fmaf(st.lb_a, st.lb_d[i], st.q[i]), st.lb_lo[i]), st.lb_hi[i]);
  return true;
}

// The line-search step after the evaluation (chi2 ft, J^T W r gls) at the trial
// point: accept it (new pair, new point) or choose the next trial step.
__device__ inline void lb_after_eval(FitSlot& st, float ft, const float* gls, int m) {
  st.iter += 1;
  st.lb_trials += 1;
  float gt[4];
  lb_grad(gls, gt);
  const float dt = dot4(gt, st.lb_d);
  const float a = st.lb_a;
  bool accept = false;
  if (!isfinite(ft) || ft > fmaf(LB_FTOL * a, st.lb_gd, st.chi2) || ft >= st.lb_flo) {
    st.lb_ahi = a;
    st.lb_fhi = isfinite(ft) ? ft : __builtin_inff();
    st.lb_ghi = isfinite(dt) ? dt : 0.f;
    st.lb_has_hi = 1;
  } else if (fabsf(dt) <= -LB_GTOL * st.lb_gd) {
    accept = true;
  } else {
    if ((!st.lb_has_hi && dt >= 0.f) || (st.lb_has_hi && dt * (st.lb_ahi - st.lb_alo) >= 0.f)) {
      st.lb_ahi = st.lb_alo;
      st.lb_fhi = st.lb_flo;
      st.lb_ghi = st.lb_glo;
      st.lb_has_hi = 1;
    }
    st.lb_alo = a;
    st.lb_flo = ft;
    st.lb_glo = dt;
    if (!st.lb_has_hi && a >= st.lb_amax) accept = true;   // the largest feasible step
  }
  if (accept) {
    float s[4], y[4], gx[4];
    lb_grad(st.g, gx);
    float sy = 0.f, yy = 0.f;
    for (int i = 0; i < 4; ++i) {
      s[i] = st.lb_trial[i] - st.q[i];
      y[i] = gt[i] - gx[i];
      sy = fmaf(s[i], y[i], sy);
      yy = fmaf(y[i], y[i], yy);
    }
    if (sy > __FLT_EPSILON__ * yy) {
      if (st.lb_n == m) {
        for (int p = 1; p < m; ++p)
          for (int i = 0; i < 4; ++i) {
            st.lb_S[p - 1][i] = st.lb_S[p][i];
            st.lb_Y[p - 1][i] = st.lb_Y[p][i];
          }
        st.lb_n -= 1;
      }
      for (int i = 0; i < 4; ++i) {
        st.lb_S[st.lb_n][i] = s[i];
        st.lb_Y[st.lb_n][i] = y[i];
      }
      st.lb_n += 1;
    }
    for (int i = 0; i < 4; ++i) {
      st.q[i] = st.lb_trial[i];
      st.g[i] = gls[i];
    }
    st.chi2 = ft;
    st.n_accept += 1;
    st.lb_first = 0;
    st.lb_phase = LB_NEED_DIR;
    return;
  }
  if (st.lb_trials >= LB_MAX_LS) {
    if (st.lb_n > 0) {
      st.lb_n = 0;               // line search failed: restart from steepest descent
      st.lb_first = 1;
      st.lb_phase = LB_NEED_DIR;
    } else {
      st.lb_phase = LB_DONE;
    }
    return;
  }
  if (!st.lb_has_hi) st.lb_a = fminf(4.f * st.lb_alo, st.lb_amax);
  else if (!isfinite(st.lb_fhi)) st.lb_a = st.lb_alo + 0.5f * (st.lb_ahi - st.lb_alo);
  else st.lb_a = lb_cubic(st.lb_alo, st.lb_flo, st.lb_glo, st.lb_ahi, st.lb_fhi, st.lb_ghi);
}

}  // namespace sbk
