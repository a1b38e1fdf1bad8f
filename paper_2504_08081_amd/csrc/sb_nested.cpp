// Nested-sampling driver (the paper's nested-sampling example) over the
// broadcast chi-square sweep.
//
// Skilling's nested sampling: N live points from the prior; each iteration the
// lowest-likelihood live point becomes a dead point with prior mass
// X_i = exp(-i/N) and weight X_{i-1} - X_i, and is replaced by a draw from the
// prior restricted to L > L*.  The evidence Z = sum L_i w_i and the information H
// accumulate in logs; the live points join with weights X_final / N at the end.
//
// The constrained draws are batched for the GPU: candidates are drawn uniformly
// from the prior inside an enlarged box around the live points in the unit cube,
// a whole batch is evaluated by one broadcast chi-square launch (every candidate
// sees the same observation table), and the candidates above the current L* are
// kept in draw order and consumed while they stay above the rising threshold.
// Draw n's unit-cube coordinates come from the counter-based generator
// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC11 2011) with counter
// (n, d div 4, 0, 0) for coordinate d, so every draw is reproducible by index.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <vector>

#include "sb_ctx.h"

namespace {

constexpr uint64_t KEY1 = 0x5A17BF1A5A17BF1Aull;   // second key word of the draws' generator

void philox_block(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3], k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    const unsigned __int128 p0 = (unsigned __int128)M0 * x0;
    const unsigned __int128 p1 = (unsigned __int128)M1 * x2;
    const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

// Unit-cube coordinates of draw n.
void unit_draw(uint64_t seed, uint64_t n, double u[5]) {
  const uint64_t key[2] = {seed, KEY1};
  uint64_t c0[4] = {n, 0, 0, 0}, c1[4] = {n, 1, 0, 0}, b0[4], b1[4];
  philox_block(c0, key, b0);
  philox_block(c1, key, b1);
  const uint64_t w[5] = {b0[0], b0[1], b0[2], b0[3], b1[0]};
  for (int d = 0; d < 5; ++d) u[d] = ((double)(w[d] >> 11) + 0.5) * 0x1p-53;
}

void prior_transform(const sb_prior* pr, const double u[5], double th[5]) {
  for (int d = 0; d < 5; ++d) {
    const sb_prior& p = pr[d];
    if (p.kind == SB_PRIOR_FIXED) th[d] = p.a;
    else if (p.kind == SB_PRIOR_UNIFORM) th[d] = p.a + (p.b - p.a) * u[d];
    else th[d] = std::exp(std::log(p.a) + (std::log(p.b) - std::log(p.a)) * u[d]);
  }
}

double logaddexp(double a, double b) {
  if (a == -INFINITY) return b;
  if (b == -INFINITY) return a;
  const double m = std::max(a, b);
  return m + std::log1p(std::exp(-std::fabs(a - b)));
}

struct Cand {
  double u[5], th[5], logl;
  int64_t draw;
};

// Device and pinned host buffers of one batch of candidates.
struct Batch {
  int n = 0;
  float* d = nullptr;     // device: z, t0, x0, x1, c [5][n], then chi2 [n]
  float* h = nullptr;     // pinned host, same layout
  ~Batch() {
    if (d) (void)hipFree(d);
    if (h) (void)hipHostFree(h);
  }
};

}  // namespace

extern "C" {

void sb_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) { philox_block(ctr, key, out); }

sb_status sb_nested_sampling(sb_ctx* ctx, const sb_ns_config* cfg, int32_t n_obs, const float* t, const int32_t* band,
                             const float* data, const float* inv_sigma2, double* dead_theta, double* dead_logl,
                             double* dead_logw, int64_t* dead_draw, double* live_theta, double* live_logl,
                             double* live_logw, sb_ns_summary* out, void* hip_stream) {
  using sbh::set_error;
  if (!ctx || !cfg || !out) return set_error(SB_ERR_ARG, "sb_nested_sampling: NULL argument");
  if (ctx->n_bands == 0) return set_error(SB_ERR_STATE, "sb_nested_sampling: no band registered");
  if (n_obs < 0 || (n_obs > 0 && (!t || !band || !data || !inv_sigma2)))
    return set_error(SB_ERR_ARG, "sb_nested_sampling: observation table");
  if (cfg->n_live < 2 || cfg->batch < 1 || cfg->batch > (1 << 24) - 1 || cfg->max_iter < 0 || cfg->max_evals < 0 ||
      !(cfg->enlarge >= 1.0) || !(cfg->dlogz >= 0.0) || !std::isfinite(cfg->log_norm))
    return set_error(SB_ERR_ARG, "sb_nested_sampling: bad configuration");
  for (int d = 0; d < 5; ++d) {
    const sb_prior& p = cfg->prior[d];
    const bool ok = (p.kind == SB_PRIOR_FIXED && std::isfinite(p.a)) ||
                    (p.kind == SB_PRIOR_UNIFORM && std::isfinite(p.a) && std::isfinite(p.b) && p.a < p.b) ||
                    (p.kind == SB_PRIOR_LOG_UNIFORM && p.a > 0 && std::isfinite(p.b) && p.a < p.b);
    if (!ok) return set_error(SB_ERR_ARG, "sb_nested_sampling: bad prior for parameter " + std::to_string(d));
  }
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e = hipSetDevice(ctx->device);
  const int N = cfg->n_live;
  const int bmax = std::max(cfg->batch, N);
  Batch B;
  B.n = bmax;
  if (e == hipSuccess) e = hipMalloc((void**)&B.d, (size_t)6 * bmax * sizeof(float));
  if (e == hipSuccess) e = hipHostMalloc((void**)&B.h, (size_t)6 * bmax * sizeof(float), hipHostMallocDefault);
  if (e != hipSuccess) return set_error(SB_ERR_NOMEM, std::string("sb_nested_sampling: ") + hipGetErrorString(e));

  // ln L of n candidates (their parameters in th[n][5]) by one broadcast chi-square launch;
  // a sample whose band windows leave the surface has chi2 = NaN and ln L = -inf
  std::vector<double> logl_buf(bmax);
  auto evaluate = [&](const std::vector<Cand>& cs, int n) -> sb_status {
    for (int k = 0; k < n; ++k)
      for (int d = 0; d < 5; ++d) B.h[(size_t)d * bmax + k] = (float)cs[k].th[d];
    hipError_t ee = hipMemcpyAsync(B.d, B.h, (size_t)5 * bmax * sizeof(float), hipMemcpyHostToDevice, st);
    sbk::KBatch kb{};
    kb.n_sn = n;
    kb.n_obs = n_obs;
    kb.flags = SB_OBS_BROADCAST | SB_OUT_CHI2;
    kb.z = B.d;
    kb.t0 = B.d + bmax;
    kb.x0 = B.d + 2 * bmax;
    kb.x1 = B.d + 3 * bmax;
    kb.c = B.d + 4 * bmax;
    kb.t = t;
    kb.band = band;
    kb.data = data;
    kb.w = inv_sigma2;
    kb.chi2 = B.d + 5 * bmax;
    kb.err = ctx->d_err;
    if (ee == hipSuccess) ee = sbk::launch_sn(false, ctx->km, ctx->tables(), kb, st);
    if (ee == hipSuccess)
      ee = hipMemcpyAsync(B.h + 5 * bmax, B.d + 5 * bmax, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, st);
    if (ee == hipSuccess) ee = hipStreamSynchronize(st);
    if (ee != hipSuccess) return set_error(SB_ERR_DEVICE, std::string("sb_nested_sampling: ") + hipGetErrorString(ee));
    for (int k = 0; k < n; ++k) {
      const double c2 = (double)B.h[(size_t)5 * bmax + k];
      logl_buf[k] = std::isnan(c2) ? -INFINITY : cfg->log_norm - 0.5 * c2;
    }
    return SB_OK;
  };

  // initial live points: draws 0 .. N-1 over the whole unit cube
  std::vector<Cand> live(N), cand(bmax);
  for (int i = 0; i < N; ++i) {
    unit_draw(cfg->seed, (uint64_t)i, live[i].u);
    prior_transform(cfg->prior, live[i].u, live[i].th);
    live[i].draw = i;
  }
  sb_status s = evaluate(live, N);
  if (s != SB_OK) return s;
  for (int i = 0; i < N; ++i) live[i].logl = logl_buf[i];
  int64_t n_draw = N, n_eval = N, n_batches = 1, n_iter = 0;
  double logz = -INFINITY, H = 0.0, logx = 0.0;
  const double log_shrink = std::log(-std::expm1(-1.0 / N));
  bool stopped_on_evals = false;
  std::deque<Cand> pool;
  auto accumulate = [&](double l, double lw) {
    const double lz_new = logaddexp(logz, l + lw);
    H = std::exp(l + lw - lz_new) * l + (std::isfinite(logz) ? std::exp(logz - lz_new) * (H + logz) : 0.0) - lz_new;
    logz = lz_new;
  };
  while (n_iter < cfg->max_iter) {
    double lmax = -INFINITY;
    int worst = 0;
    for (int i = 0; i < N; ++i) {
      lmax = std::max(lmax, live[i].logl);
      if (live[i].logl < live[worst].logl) worst = i;
    }
    if (std::isfinite(logz) && logaddexp(logz, lmax + logx) - logz < cfg->dlogz) break;
    const double lstar = live[worst].logl;
    const double lw = logx + log_shrink;
    accumulate(lstar, lw);
    if (dead_theta) std::memcpy(dead_theta + 5 * n_iter, live[worst].th, 5 * sizeof(double));
    if (dead_logl) dead_logl[n_iter] = lstar;
    if (dead_logw) dead_logw[n_iter] = lw;
    if (dead_draw) dead_draw[n_iter] = live[worst].draw;
    logx -= 1.0 / N;
    ++n_iter;
    // replacement: the first kept candidate above L*; a new batch when none is left
    for (;;) {
      while (!pool.empty() && !(pool.front().logl > lstar)) pool.pop_front();
      if (!pool.empty()) break;
      if (n_eval >= cfg->max_evals) {
        stopped_on_evals = true;
        break;
      }
      double lo[5], hi[5];
      for (int d = 0; d < 5; ++d) {
        double a = live[0].u[d], b = live[0].u[d];
        for (int i = 1; i < N; ++i) {
          a = std::min(a, live[i].u[d]);
          b = std::max(b, live[i].u[d]);
        }
        const double c = 0.5 * (a + b), h = 0.5 * (b - a) * cfg->enlarge;
        lo[d] = std::max(c - h, 0.0);
        hi[d] = std::min(c + h, 1.0);
      }
      const int nb = cfg->batch;
      for (int k = 0; k < nb; ++k) {
        double v[5];
        unit_draw(cfg->seed, (uint64_t)(n_draw + k), v);
        for (int d = 0; d < 5; ++d) cand[k].u[d] = lo[d] + (hi[d] - lo[d]) * v[d];
        prior_transform(cfg->prior, cand[k].u, cand[k].th);
        cand[k].draw = n_draw + k;
      }
      s = evaluate(cand, nb);
      if (s != SB_OK) return s;
      for (int k = 0; k < nb; ++k) {
        cand[k].logl = logl_buf[k];
        if (cand[k].logl > lstar) pool.push_back(cand[k]);
      }
      n_draw += nb;
      n_eval += nb;
      ++n_batches;
    }
    if (stopped_on_evals) break;
    live[worst] = pool.front();
    pool.pop_front();
  }
  const double lw_live = logx - std::log((double)N);
  for (int i = 0; i < N; ++i) {
    accumulate(live[i].logl, lw_live);
    if (live_theta) std::memcpy(live_theta + 5 * i, live[i].th, 5 * sizeof(double));
    if (live_logl) live_logl[i] = live[i].logl;
    if (live_logw) live_logw[i] = lw_live;
  }
  out->logz = logz;
  out->logz_err = std::sqrt(std::max(H, 0.0) / N);
  out->information = H;
  out->n_iter = n_iter;
  out->n_eval = n_eval;
  out->n_batches = n_batches;
  out->stopped_on_evals = stopped_on_evals ? 1 : 0;
  return SB_OK;
}

}  // extern "C"
