// Host side of the C ABI: context, surfaces, band registry, launch of the
// bandflux / adjoint / sweep kernels, device error flags.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <climits>
#include <cstdio>
#include <cstring>
#include <new>

#include "sb_ctx.h"
#include "sb_server.h"

namespace {
thread_local std::string g_last_error;

// h c with the exact SI values of h (erg s) and c (Angstrom / s): erg Angstrom.
constexpr double H_ERG_S = 6.62607015e-27;
constexpr double HC_ERG_ANGSTROM = H_ERG_S * 2.99792458e18;
// AB reference spectral flux density: m_AB = -2.5 log10(f_nu / (erg s^-1 cm^-2 Hz^-1)) - 48.60 = 0.
const double FNU_AB = std::pow(10.0, -0.4 * 48.60);

bool finite_all(const double* a, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

sb_status hip_fail(hipError_t e, const char* what) {
  return sbh::set_error(SB_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
}  // namespace

namespace sbh {

sb_status set_error(sb_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

double now_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

sb_status build_band_grid(const double* wave, const double* trans, int n, double spacing, int rule,
                          std::vector<double>& lam, std::vector<double>& W, double* zp_ab) {
  if (!wave || !trans || n < 2) return set_error(SB_ERR_ARG, "band: need at least 2 samples");
  if (!(spacing > 0.0) || !std::isfinite(spacing)) return set_error(SB_ERR_ARG, "band: spacing must be > 0");
  if (rule != SB_QUAD_TRAPEZOID && rule != SB_QUAD_MIDPOINT) return set_error(SB_ERR_ARG, "band: unknown rule");
  if (!finite_all(wave, n) || !finite_all(trans, n)) return set_error(SB_ERR_ARG, "band: non-finite sample");
  for (int i = 0; i < n; ++i) {
    if (i > 0 && !(wave[i] > wave[i - 1])) return set_error(SB_ERR_ARG, "band: wavelengths must increase");
    if (trans[i] < 0.0) return set_error(SB_ERR_ARG, "band: negative transmission");
  }
  const double L = wave[0], U = wave[n - 1];
  // N equal intervals no wider than the spacing (tolerant to rounding of an exact ratio)
  const double ratio = (U - L) / spacing;
  if (ratio > 1e7) return set_error(SB_ERR_ARG, "band: too many quadrature nodes");
  long N = (long)std::ceil(ratio - 1e-9);
  if (N < 1) N = 1;
  if (N + 1 > SB_MAX_BAND_POINTS) return set_error(SB_ERR_ARG, "band: more than SB_MAX_BAND_POINTS nodes");
  const double delta = (U - L) / (double)N;
  // trapezoid: the N + 1 interval ends, weights Delta/2 at the ends and Delta inside;
  // midpoint: the N interval midpoints, weight Delta
  const bool mid = rule == SB_QUAD_MIDPOINT;
  const long n_nodes = mid ? N : N + 1;
  lam.assign(n_nodes, 0.0);
  W.assign(n_nodes, 0.0);
  int seg = 0;
  double zp = 0.0;
  for (long k = 0; k < n_nodes; ++k) {
    const double x = mid ? L + delta * ((double)k + 0.5) : ((k == N) ? U : L + delta * (double)k);
    while (seg < n - 2 && x > wave[seg + 1]) ++seg;
    // linear interpolation of the transmission between samples seg and seg+1
    const double slope = (trans[seg + 1] - trans[seg]) / (wave[seg + 1] - wave[seg]);
    const double T = slope * (x - wave[seg]) + trans[seg];
    const double w = (!mid && (k == 0 || k == N)) ? 0.5 * delta : delta;
    lam[k] = x;
    W[k] = w * x * T / HC_ERG_ANGSTROM;
    zp += w * T / x;
  }
  if (zp_ab) *zp_ab = zp * FNU_AB / H_ERG_S;
  return SB_OK;
}

// Two numeric columns per line ('#' comments, blank lines skipped; spaces, tabs or a comma).
sb_status read_band_file(const char* path, std::vector<double>& wave, std::vector<double>& trans) {
  wave.clear();
  trans.clear();
  if (!path) return set_error(SB_ERR_ARG, "band file: NULL path");
  FILE* fh = std::fopen(path, "r");
  if (!fh) return set_error(SB_ERR_ARG, std::string("band file: cannot open ") + path);
  char line[4096];
  int lineno = 0;
  sb_status st = SB_OK;
  while (std::fgets(line, sizeof line, fh)) {
    ++lineno;
    if (!std::strchr(line, '\n') && !std::feof(fh)) {
      st = set_error(SB_ERR_ARG, "band file: line " + std::to_string(lineno) + " too long");
      break;
    }
    if (char* hash = std::strchr(line, '#')) *hash = '\0';
    for (char* c = line; *c; ++c)
      if (*c == ',') *c = ' ';
    char* p = line;
    while (*p == ' ' || *p == '\t' || *p == '\r' || *p == '\n') ++p;
    if (!*p) continue;
    char* end = nullptr;
    const double a = std::strtod(p, &end);
    const bool ok_a = end != p;
    p = end;
    const double b = std::strtod(p, &end);
    const bool ok_b = end != p;
    p = end;
    while (*p == ' ' || *p == '\t' || *p == '\r' || *p == '\n') ++p;
    if (!ok_a || !ok_b || *p) {
      st = set_error(SB_ERR_ARG, "band file: line " + std::to_string(lineno) + " is not two numbers");
      break;
    }
    wave.push_back(a);
    trans.push_back(b);
  }
  std::fclose(fh);
  return st;
}

}  // namespace sbh

using sbh::set_error;

extern "C" {

const char* sb_last_error(void) { return g_last_error.c_str(); }

const char* sb_status_string(sb_status st) {
  switch (st) {
    case SB_OK: return "ok";
    case SB_PENDING: return "pending";
    case SB_CANCELLED: return "cancelled";
    case SB_FIT_DIVERGED: return "fit diverged";
    case SB_ERR_ARG: return "invalid argument";
    case SB_ERR_RANGE: return "out of range (band window, band id or CSR offsets)";
    case SB_ERR_DEVICE: return "device error";
    case SB_ERR_NOMEM: return "out of memory";
    case SB_ERR_BUDGET: return "request exceeds the serving budget";
    case SB_ERR_STATE: return "invalid state";
    case SB_ERR_NOTFOUND: return "unknown ticket";
    default: return "unknown status";
  }
}

void sb_config_default(sb_config* cfg) {
  if (!cfg) return;
  cfg->max_spacing = 5.0;
  cfg->max_obs_per_fit = 256;
  cfg->max_slots = 1024;
  cfg->hbm_budget_bytes = 256ll << 20;
  cfg->iters_per_tick = 5;
  cfg->fit_iters = 50;
  cfg->lm_lambda0 = 1e-3;
  cfg->quad_rule = SB_QUAD_TRAPEZOID;
  cfg->lds_limit_bytes = 0;
  cfg->solver = SB_SOLVER_LM;
  cfg->lbfgs_m = 5;
}

sb_status sb_band_grid(const double* wave, const double* trans, int32_t n, double max_spacing, int32_t rule,
                       int32_t cap,
                       float* lam_out, float* weight_out, int32_t* n_points) {
  if (!n_points) return set_error(SB_ERR_ARG, "sb_band_grid: n_points is NULL");
  std::vector<double> lam, W;
  sb_status st = sbh::build_band_grid(wave, trans, n, max_spacing, rule, lam, W);
  if (st != SB_OK) return st;
  *n_points = (int32_t)lam.size();
  if ((int)lam.size() > cap) return set_error(SB_ERR_ARG, "sb_band_grid: cap too small");
  for (size_t k = 0; k < lam.size(); ++k) {
    if (lam_out) lam_out[k] = (float)lam[k];
    if (weight_out) weight_out[k] = (float)W[k];
  }
  return SB_OK;
}

static void free_ctx(sb_ctx* c) {
  if (!c) return;
  for (auto& kv : c->ws)
    if (kv.second.ptr) (void)hipFree(kv.second.ptr);
  if (c->d_surf) (void)hipFree(c->d_surf);
  if (c->d_pts) (void)hipFree(c->d_pts);
  if (c->d_npts) (void)hipFree(c->d_npts);
  if (c->d_err) (void)hipFree(c->d_err);
  delete c;
}

sb_status sb_create(const sb_model_desc* md, const sb_config* cfg_in, int device, sb_ctx** out) {
  if (!md || !out) return set_error(SB_ERR_ARG, "sb_create: NULL argument");
  *out = nullptr;
  if (md->n_phase < 4 || md->n_phase > sbk::MAX_PHASE || md->n_wave < 4 || md->n_wave > sbk::MAX_WAVE)
    return set_error(SB_ERR_ARG, "sb_create: grid size out of range");
  if (!md->m0 || !md->m1) return set_error(SB_ERR_ARG, "sb_create: NULL surface");
  const double g4[4] = {md->phase0, md->dphase, md->wave0, md->dwave};
  if (!finite_all(g4, 4) || !(md->dphase > 0) || !(md->dwave > 0))
    return set_error(SB_ERR_ARG, "sb_create: bad grid spacing/origin");
  if (md->cl_degree < 0 || md->cl_degree > SB_MAX_CL_DEGREE || (md->cl_degree > 0 && !md->cl_coef))
    return set_error(SB_ERR_ARG, "sb_create: bad colour law degree");
  if (md->cl_degree > 0 && !finite_all(md->cl_coef, md->cl_degree))
    return set_error(SB_ERR_ARG, "sb_create: non-finite colour law");
  if (!std::isfinite(md->cl_wave_b) || !std::isfinite(md->cl_wave_v) || md->cl_wave_v == md->cl_wave_b)
    return set_error(SB_ERR_ARG, "sb_create: colour law reference wavelengths");
  const size_t nsurf = (size_t)md->n_phase * md->n_wave;
  for (size_t i = 0; i < nsurf; ++i)
    if (!std::isfinite(md->m0[i]) || !std::isfinite(md->m1[i]))
      return set_error(SB_ERR_ARG, "sb_create: non-finite surface value");

  sb_config cfg;
  sb_config_default(&cfg);
  if (cfg_in) cfg = *cfg_in;
  if (!(cfg.max_spacing > 0) || cfg.max_obs_per_fit < 1 || cfg.max_obs_per_fit > 1024 || cfg.max_slots < 1 ||
      cfg.max_slots > 65536 || cfg.hbm_budget_bytes < 0 || cfg.iters_per_tick < 1 || cfg.fit_iters < 0 ||
      !(cfg.lm_lambda0 > 0) || cfg.lds_limit_bytes < 0 ||
      (cfg.quad_rule != SB_QUAD_TRAPEZOID && cfg.quad_rule != SB_QUAD_MIDPOINT) ||
      (cfg.solver != SB_SOLVER_LM && cfg.solver != SB_SOLVER_LBFGSB) || cfg.lbfgs_m < 1 ||
      cfg.lbfgs_m > sbk::LB_MAX_M)
    return set_error(SB_ERR_ARG, "sb_create: bad configuration");

  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");

  // the device address of the allocation-free fits' state array, once per device
  e = sbk::fit_scratch_init(device);
  if (e != hipSuccess) return hip_fail(e, "sb_create: hipGetSymbolAddress of the fit state array");

  sb_ctx* c = new (std::nothrow) sb_ctx();
  if (!c) return set_error(SB_ERR_NOMEM, "sb_create: host allocation");
  c->device = device;
  c->cfg = cfg;
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
  // per-workgroup LDS: the opt-in maximum where the device reports one (launches above 64 KiB
  // raise the kernel's limit), capped by the configuration
  size_t dev_lds = prop.sharedMemPerBlock > 0 ? prop.sharedMemPerBlock : 65536;
  if (prop.sharedMemPerBlockOptin > dev_lds) dev_lds = prop.sharedMemPerBlockOptin;
  c->max_lds = cfg.lds_limit_bytes > 0 ? std::min<size_t>(dev_lds, (size_t)cfg.lds_limit_bytes) : dev_lds;

  sbk::KModel& k = c->km;
  k.n_phase = md->n_phase;
  k.n_wave = md->n_wave;
  k.row_pad = (md->n_phase + 15) / 16 * 16;
  k.n_bands = 0;
  k.phase0 = (float)md->phase0;
  k.inv_dphase = (float)(1.0 / md->dphase);
  k.wave0 = (float)md->wave0;
  k.inv_dwave = (float)(1.0 / md->dwave);
  k.phase0_d = md->phase0;
  k.inv_dphase_d = 1.0 / md->dphase;
  k.wave0_d = md->wave0;
  k.inv_dwave_d = 1.0 / md->dwave;
  k.cl_b = (float)md->cl_wave_b;
  k.cl_inv_span = (float)(1.0 / (md->cl_wave_v - md->cl_wave_b));
  k.cl_deg = md->cl_degree;
  for (int n = 0; n < SB_MAX_CL_DEGREE; ++n) {
    k.cl[n] = n < md->cl_degree ? (float)md->cl_coef[n] : 0.f;
    k.dcl[n] = n < md->cl_degree ? (float)((n + 1) * md->cl_coef[n]) : 0.f;
  }
  c->wave_lo = md->wave0;
  c->wave_hi = md->wave0 + (md->n_wave - 1) * md->dwave;

  // surfaces, wavelength-major: node (a, j) -> surf[j * row_pad + a] = (M0, M1), followed by
  // SURF_PAD_COLS zero columns that the row projections may prefetch past the last column
  std::vector<float2> surf((size_t)(k.n_wave + sbk::SURF_PAD_COLS) * k.row_pad, make_float2(0.f, 0.f));
  for (int a = 0; a < k.n_phase; ++a)
    for (int j = 0; j < k.n_wave; ++j) {
      const size_t src = (size_t)a * k.n_wave + j;
      surf[(size_t)j * k.row_pad + a] = make_float2(md->m0[src], md->m1[src]);
    }
  const size_t pts_bytes = (size_t)SB_MAX_BANDS * SB_MAX_BAND_POINTS * sizeof(float2);
  if ((e = hipMalloc(&c->d_surf, surf.size() * sizeof(float2))) != hipSuccess ||
      (e = hipMalloc(&c->d_pts, pts_bytes)) != hipSuccess ||
      (e = hipMalloc(&c->d_npts, SB_MAX_BANDS * sizeof(int))) != hipSuccess ||
      (e = hipMalloc(&c->d_err, sizeof(int))) != hipSuccess) {
    free_ctx(c);
    return set_error(SB_ERR_NOMEM, std::string("sb_create: hipMalloc: ") + hipGetErrorString(e));
  }
  if ((e = hipMemcpy(c->d_surf, surf.data(), surf.size() * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(c->d_pts, 0, pts_bytes)) != hipSuccess ||
      (e = hipMemset(c->d_npts, 0, SB_MAX_BANDS * sizeof(int))) != hipSuccess ||
      (e = hipMemset(c->d_err, 0, sizeof(int))) != hipSuccess) {
    free_ctx(c);
    return hip_fail(e, "sb_create: upload");
  }
  *out = c;
  return SB_OK;
}

sb_status sb_destroy(sb_ctx* ctx) {
  if (!ctx) return set_error(SB_ERR_ARG, "sb_destroy: NULL context");
  (void)hipSetDevice(ctx->device);
  if (ctx->server) {
    delete ctx->server;
    ctx->server = nullptr;
  }
  (void)hipDeviceSynchronize();
  free_ctx(ctx);
  return SB_OK;
}

sb_status sb_add_band(sb_ctx* ctx, const double* wave, const double* trans, int32_t n, int32_t* band_id) {
  if (!ctx || !band_id) return set_error(SB_ERR_ARG, "sb_add_band: NULL argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (ctx->n_bands >= SB_MAX_BANDS) return set_error(SB_ERR_ARG, "sb_add_band: registry full");
  std::vector<double> lam, W;
  double zp_ab = 0.0;
  sb_status st = sbh::build_band_grid(wave, trans, n, ctx->cfg.max_spacing, ctx->cfg.quad_rule, lam, W, &zp_ab);
  if (st != SB_OK) return st;
  const int np = (int)lam.size();
  // surface window of the band for rest wavelengths lam/(1+z), z >= WINDOW_Z_MIN: at most
  // (U - L)/((1 + WINDOW_Z_MIN) dwave) columns plus the stencil
  const double span = wave[n - 1] - wave[0];
  const int jc = (int)std::min<double>(ctx->km.n_wave + 4,
                                       std::ceil(span * ctx->km.inv_dwave_d / (1.0 + sbk::WINDOW_Z_MIN)) + 8);
  const int jcap = std::max(ctx->jcap, jc);
  // the per-supernova pipeline keeps a band's nodes in LDS: check it fits
  const size_t need = std::max(sbk::lds_bytes(ctx->km, std::max(np, ctx->max_pts), jcap, true),
                               sbk::fit_lds_bytes(ctx->km, std::max(np, ctx->max_pts), jcap));
  if (need > ctx->max_lds) return set_error(SB_ERR_ARG, "sb_add_band: band grid too large for LDS");
  std::vector<float2> host(np);
  for (int k = 0; k < np; ++k) host[k] = make_float2((float)lam[k], (float)W[k]);
  hipError_t e = hipSetDevice(ctx->device);
  const int id = ctx->n_bands;
  if (e == hipSuccess)
    e = hipMemcpy(ctx->d_pts + (size_t)id * SB_MAX_BAND_POINTS, host.data(), np * sizeof(float2),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ctx->d_npts + id, &np, sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "sb_add_band: upload");
  ctx->band_lo.push_back(wave[0]);
  ctx->band_hi.push_back(wave[n - 1]);
  ctx->band_zp_ab.push_back(zp_ab);
  ctx->max_pts = std::max(ctx->max_pts, np);
  ctx->jcap = jcap;
  ctx->n_bands = id + 1;
  ctx->km.n_bands = ctx->n_bands;
  *band_id = id;
  return SB_OK;
}

sb_status sb_read_band_file(const char* path, double* wave, double* trans, int32_t cap, int32_t* n) {
  if (!n) return set_error(SB_ERR_ARG, "sb_read_band_file: n is NULL");
  std::vector<double> w, t;
  sb_status st = sbh::read_band_file(path, w, t);
  if (st != SB_OK) return st;
  *n = (int32_t)std::min<size_t>(w.size(), (size_t)INT32_MAX);
  if ((int64_t)w.size() > cap) return set_error(SB_ERR_ARG, "sb_read_band_file: more rows than cap");
  if (!w.empty() && (!wave || !trans)) return set_error(SB_ERR_ARG, "sb_read_band_file: NULL output");
  for (size_t i = 0; i < w.size(); ++i) {
    wave[i] = w[i];
    trans[i] = t[i];
  }
  return SB_OK;
}

sb_status sb_add_band_file(sb_ctx* ctx, const char* path, int32_t* band_id) {
  if (!ctx || !band_id) return set_error(SB_ERR_ARG, "sb_add_band_file: NULL argument");
  std::vector<double> w, t;
  sb_status st = sbh::read_band_file(path, w, t);
  if (st != SB_OK) return st;
  if (w.size() > 65536) return set_error(SB_ERR_ARG, "sb_add_band_file: more than 65,536 rows");
  return sb_add_band(ctx, w.data(), t.data(), (int32_t)w.size(), band_id);
}

sb_status sb_band_zeropoint(sb_ctx* ctx, int32_t band_id, int32_t magsys, double* zp_flux) {
  if (!ctx || !zp_flux) return set_error(SB_ERR_ARG, "sb_band_zeropoint: NULL argument");
  if (magsys != SB_MAGSYS_AB) return set_error(SB_ERR_ARG, "sb_band_zeropoint: unknown magnitude system");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (band_id < 0 || band_id >= ctx->n_bands) return set_error(SB_ERR_ARG, "sb_band_zeropoint: unknown band");
  *zp_flux = ctx->band_zp_ab[band_id];
  return SB_OK;
}

sb_status sb_band_zeropoint_ab(const double* wave, const double* trans, int32_t n, double max_spacing, int32_t rule,
                               double* zp_flux) {
  if (!zp_flux) return set_error(SB_ERR_ARG, "sb_band_zeropoint_ab: NULL output");
  std::vector<double> lam, W;
  return sbh::build_band_grid(wave, trans, n, max_spacing, rule, lam, W, zp_flux);
}

static sb_status check_batch(const sb_ctx* ctx, const sb_batch* b, const char* who) {
  const std::string w(who);
  if (!ctx || !b) return set_error(SB_ERR_ARG, w + ": NULL argument");
  if (b->n_sn < 0 || b->n_obs < 0) return set_error(SB_ERR_ARG, w + ": negative size");
  if (b->n_sn > (1 << 24) - 1) return set_error(SB_ERR_ARG, w + ": more than 2^24 - 1 supernovae in one call");
  if ((b->flags & SB_OBS_BROADCAST) && (int64_t)b->n_sn * b->n_obs > ((int64_t)1 << 40))
    return set_error(SB_ERR_ARG, w + ": broadcast output too large");
  if (b->flags & ~(SB_OBS_BROADCAST | SB_OUT_CHI2 | SB_PERSISTENT)) return set_error(SB_ERR_ARG, w + ": unknown flags");
  if ((b->flags & SB_PERSISTENT) && !(b->flags & SB_OBS_BROADCAST))
    return set_error(SB_ERR_ARG, w + ": SB_PERSISTENT needs SB_OBS_BROADCAST");
  if (ctx->n_bands == 0) return set_error(SB_ERR_STATE, w + ": no band registered");
  if (b->n_sn > 0 && (!b->z || !b->t0 || !b->x0 || !b->x1 || !b->c))
    return set_error(SB_ERR_ARG, w + ": NULL parameter array");
  if (b->n_obs > 0 && (!b->t || !b->band)) return set_error(SB_ERR_ARG, w + ": NULL observation array");
  if (!(b->flags & SB_OBS_BROADCAST) && b->n_sn > 0 && !b->sn_offsets)
    return set_error(SB_ERR_ARG, w + ": NULL sn_offsets");
  if ((b->flags & SB_OUT_CHI2) && b->n_obs > 0 && (!b->data || !b->inv_sigma2))
    return set_error(SB_ERR_ARG, w + ": SB_OUT_CHI2 needs data and inv_sigma2");
  return SB_OK;
}

static sbk::KBatch make_kbatch(sb_ctx* ctx, const sb_batch* b) {
  sbk::KBatch k{};
  k.n_sn = b->n_sn;
  k.n_obs = b->n_obs;
  k.flags = b->flags;
  k.z = b->z; k.t0 = b->t0; k.x0 = b->x0; k.x1 = b->x1; k.c = b->c;
  k.t = b->t; k.band = b->band; k.off = b->sn_offsets;
  k.data = b->data; k.w = b->inv_sigma2;
  k.err = ctx->d_err;
  return k;
}

// The stream's workspace, at least `bytes` long; the caller holds ctx->ws_mu until its
// launches that use the buffer are enqueued (so no other thread can replace the buffer
// in between).  Growing it waits for the stream's earlier work (which may still use the
// old buffer) and allocates, so it is refused while the stream is being captured into a
// graph: one call of the same size before the capture sizes it.
static sb_status stream_workspace(sb_ctx* ctx, hipStream_t st, size_t bytes, void** out) {
  sb_ctx::Workspace& w = ctx->ws[(void*)st];
  if (w.bytes >= bytes) {
    *out = w.ptr;
    return SB_OK;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone)
    return set_error(SB_ERR_STATE, "sb_bandflux_vjp: the stream's workspace must grow, which cannot happen during "
                                   "graph capture: make one call of this size on the stream before capturing");
  if (w.ptr) {
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    (void)hipFree(w.ptr);
    w.ptr = nullptr;
    w.bytes = 0;
  }
  const size_t want = std::max(bytes, (size_t)1 << 16);
  if ((e = hipMalloc(&w.ptr, want)) != hipSuccess) {
    w.ptr = nullptr;
    return set_error(SB_ERR_NOMEM, std::string("sb_bandflux_vjp: workspace: ") + hipGetErrorString(e));
  }
  w.bytes = want;
  *out = w.ptr;
  return SB_OK;
}

static sb_status launch(sb_ctx* ctx, bool adj, sbk::KBatch& kb, hipStream_t st) {
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  const size_t lds = sbk::lds_bytes(ctx->km, ctx->max_pts, ctx->jcap, adj);
  if (lds > ctx->max_lds) return set_error(SB_ERR_ARG, "bands too large for LDS");
  std::unique_lock<std::mutex> lk(ctx->ws_mu, std::defer_lock);
  if (adj && ctx->n_bands <= sbk::BAND_SPLIT_MAX) {
    lk.lock();
    void* p = nullptr;
    const sb_status s = stream_workspace(ctx, st, sbk::band_part_bytes(kb.n_sn, ctx->n_bands), &p);
    if (s != SB_OK) return s;
    kb.part = (float*)p;
  }
  e = sbk::launch_sn(adj, ctx->km, ctx->tables(), kb, st);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return SB_OK;
}

sb_status sb_bandflux(sb_ctx* ctx, const sb_batch* b, float* out, void* hip_stream) {
  sb_status st = check_batch(ctx, b, "sb_bandflux");
  if (st != SB_OK) return st;
  const bool chi2 = (b->flags & SB_OUT_CHI2) != 0;
  const bool any_out = b->n_sn > 0 && (chi2 || b->n_obs > 0);
  if (!any_out) return SB_OK;
  if (!out) return set_error(SB_ERR_ARG, "sb_bandflux: NULL output");
  sbk::KBatch kb = make_kbatch(ctx, b);
  if (chi2) kb.chi2 = out; else kb.flux = out;
  return launch(ctx, false, kb, (hipStream_t)hip_stream);
}

sb_status sb_bandflux_vjp(sb_ctx* ctx, const sb_batch* b, const float* cot, float* grad, float* flux_out,
                          float* jac_out, float* chi2_out, void* hip_stream) {
  sb_status st = check_batch(ctx, b, "sb_bandflux_vjp");
  if (st != SB_OK) return st;
  const bool chi2 = (b->flags & SB_OUT_CHI2) != 0;
  if (b->n_sn == 0) return SB_OK;
  if (!grad) return set_error(SB_ERR_ARG, "sb_bandflux_vjp: NULL grad");
  if (chi2 && cot) return set_error(SB_ERR_ARG, "sb_bandflux_vjp: cotangent must be NULL with SB_OUT_CHI2");
  if (!chi2 && !cot && b->n_obs > 0) return set_error(SB_ERR_ARG, "sb_bandflux_vjp: NULL cotangent");
  if (!chi2 && chi2_out) return set_error(SB_ERR_ARG, "sb_bandflux_vjp: chi2_out needs SB_OUT_CHI2");
  sbk::KBatch kb = make_kbatch(ctx, b);
  kb.cot = cot;
  kb.grad = grad;
  kb.flux = flux_out;
  kb.jac = jac_out;
  kb.chi2 = chi2_out;
  return launch(ctx, true, kb, (hipStream_t)hip_stream);
}

static sb_status check_fit_batch(const sb_ctx* ctx, const sb_fit_batch_desc* b, const void* out, const char* who) {
  const std::string w(who);
  if (!ctx || !b) return set_error(SB_ERR_ARG, w + ": NULL argument");
  if (b->n_fit < 0 || b->n_obs < 0) return set_error(SB_ERR_ARG, w + ": negative size");
  if (b->n_fit > (1 << 24) - 1) return set_error(SB_ERR_ARG, w + ": more than 2^24 - 1 fits in one call");
  if (ctx->n_bands == 0) return set_error(SB_ERR_STATE, w + ": no band registered");
  if (b->n_fit > 0 && (!b->z || !b->t0 || !b->x0 || !b->x1 || !b->c || !b->fit_offsets || !out))
    return set_error(SB_ERR_ARG, w + ": NULL parameter, offset or output array");
  if (b->n_obs > 0 && (!b->t || !b->band || !b->data || !b->inv_sigma2))
    return set_error(SB_ERR_ARG, w + ": NULL observation array");
  if ((b->lower || b->upper) && ctx->cfg.solver != SB_SOLVER_LBFGSB)
    return set_error(SB_ERR_ARG, w + ": bounds need the L-BFGS-B solver (sb_config.solver)");
  return SB_OK;
}

// The fit kernel's arguments for a batch call (state in `slots`).
static sbk::KFit make_kfit_batch(sb_ctx* ctx, const sb_fit_batch_desc* b, sb_fit_out* out, sbk::FitSlot* slots) {
  sbk::KFit f{};
  f.slots = slots;
  f.lambda0 = (float)ctx->cfg.lm_lambda0;
  f.solver = ctx->cfg.solver;
  f.lbfgs_m = ctx->cfg.lbfgs_m;
  f.err = ctx->d_err;
  f.b_off = b->fit_offsets;
  f.b_lower = b->lower;
  f.b_upper = b->upper;
  f.b_z = b->z; f.b_t0 = b->t0; f.b_x0 = b->x0; f.b_x1 = b->x1; f.b_c = b->c;
  f.b_free = b->free_mask;
  f.b_t = b->t; f.b_band = b->band; f.b_data = b->data; f.b_w = b->inv_sigma2;
  f.b_n_obs = b->n_obs;
  f.b_out = out;
  return f;
}

sb_status sb_fit_batch(sb_ctx* ctx, const sb_fit_batch_desc* b, sb_fit_out* out, void* hip_stream) {
  sb_status st = check_fit_batch(ctx, b, out, "sb_fit_batch");
  if (st != SB_OK || b->n_fit == 0) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  // per-fit state between the launches: stream-ordered, so it lives exactly as long as the call's work
  sbk::FitSlot* slots = nullptr;
  e = hipMallocAsync((void**)&slots, (size_t)b->n_fit * sizeof(sbk::FitSlot), s);
  if (e != hipSuccess) return set_error(SB_ERR_NOMEM, std::string("sb_fit_batch: hipMallocAsync: ") + hipGetErrorString(e));
  e = sbk::launch_fit_batch(ctx->km, ctx->tables(), make_kfit_batch(ctx, b, out, slots), b->n_fit, ctx->cfg.fit_iters,
                            ctx->cfg.iters_per_tick, s);
  const hipError_t ef = hipFreeAsync(slots, s);
  if (e != hipSuccess) return hip_fail(e, "sb_fit_batch: launch");
  if (ef != hipSuccess) return hip_fail(ef, "sb_fit_batch: hipFreeAsync");
  return SB_OK;
}

sb_status sb_fit_batch_noalloc(sb_ctx* ctx, const sb_fit_batch_desc* b, sb_fit_out* out, void* hip_stream) {
  sb_status st = check_fit_batch(ctx, b, out, "sb_fit_batch_noalloc");
  if (st != SB_OK || b->n_fit == 0) return st;
  if (b->n_fit > SB_FIT_NOALLOC_MAX)
    return set_error(SB_ERR_ARG, "sb_fit_batch_noalloc: n_fit exceeds SB_FIT_NOALLOC_MAX (" +
                                     std::to_string(SB_FIT_NOALLOC_MAX) + "); split the batch or use sb_fit_batch");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  sbk::FitSlot* slots = sbk::fit_scratch(ctx->device);
  if (!slots) return set_error(SB_ERR_STATE, "sb_fit_batch_noalloc: no state array for this device");
  // every slot the call uses is written by its first launch before any launch reads it
  e = sbk::launch_fit_batch(ctx->km, ctx->tables(), make_kfit_batch(ctx, b, out, slots), b->n_fit,
                            ctx->cfg.fit_iters, ctx->cfg.iters_per_tick, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "sb_fit_batch_noalloc: launch");
  return SB_OK;
}

sb_status sb_peak_probe(int32_t kind, int64_t n, int32_t iters, const void* src, void* dst, double* work,
                        void* hip_stream) {
  if (!work || !dst) return set_error(SB_ERR_ARG, "sb_peak_probe: NULL argument");
  if (n < 1) return set_error(SB_ERR_ARG, "sb_peak_probe: n must be positive");
  if (((uintptr_t)dst & 15) != 0) return set_error(SB_ERR_ARG, "sb_peak_probe: dst must be 16-byte aligned");
  switch (kind) {
    case SB_PROBE_FMA_F32:
    case SB_PROBE_LDS_READ:
      if (iters < 1) return set_error(SB_ERR_ARG, "sb_peak_probe: iters must be positive");
      if (n > (1 << 23)) return set_error(SB_ERR_ARG, "sb_peak_probe: more than 2^23 workgroups");
      break;
    case SB_PROBE_COPY:
      if (!src || ((uintptr_t)src & 15) != 0)
        return set_error(SB_ERR_ARG, "sb_peak_probe: src must be a 16-byte aligned device buffer");
      if (n % 16 != 0) return set_error(SB_ERR_ARG, "sb_peak_probe: copy size must be a multiple of 16 bytes");
      break;
    default:
      return set_error(SB_ERR_ARG, "sb_peak_probe: unknown probe kind");
  }
  const hipError_t e = sbk::launch_probe(kind, n, iters, src, dst, work, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "sb_peak_probe: launch");
  return SB_OK;
}

sb_status sb_device_check(sb_ctx* ctx, void* hip_stream) {
  if (!ctx) return set_error(SB_ERR_ARG, "sb_device_check: NULL context");
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)hip_stream);
  int flags = 0;
  if (e == hipSuccess) e = hipMemcpy(&flags, ctx->d_err, sizeof(int), hipMemcpyDeviceToHost);
  if (e == hipSuccess && flags) e = hipMemset(ctx->d_err, 0, sizeof(int));
  if (e != hipSuccess) return hip_fail(e, "sb_device_check");
  if (flags) {
    std::string m = "device flags:";
    if (flags & sbk::EFLAG_WINDOW) m += " band window outside the surface grid;";
    if (flags & sbk::EFLAG_BAND) m += " band id out of range;";
    if (flags & sbk::EFLAG_CSR) m += " malformed sn_offsets;";
    return set_error(SB_ERR_RANGE, m);
  }
  return SB_OK;
}

}  // extern "C"
