// Context object and host helpers shared by sb_host.cpp and sb_server.cpp.
#pragma once

#include <atomic>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "sb_internal.h"

namespace sbh {

class Server;

sb_status set_error(sb_status st, const std::string& msg);
double now_seconds();

// Quadrature grid of one band (trapezoid or midpoint rule), float64: nodes, and W_k = w_k lam_k T_k / (hc);
// zp_ab (optional) receives the AB zero-point flux sum_k w_k T_k f_nu,AB / (h lam_k).
sb_status build_band_grid(const double* wave, const double* trans, int n, double spacing, int rule,
                          std::vector<double>& lam, std::vector<double>& W, double* zp_ab = nullptr);

// Rows of a two-column bandpass text file.
sb_status read_band_file(const char* path, std::vector<double>& wave, std::vector<double>& trans);

}  // namespace sbh

struct sb_ctx {
  int device = 0;
  sb_config cfg{};
  sbk::KModel km{};
  double wave_lo = 0, wave_hi = 0;     // surface wavelength range (Angstrom)
  float2* d_surf = nullptr;
  float2* d_pts = nullptr;
  int* d_npts = nullptr;
  int* d_err = nullptr;
  int n_bands = 0;
  int max_pts = 0;
  int jcap = 0;
  std::vector<double> band_lo, band_hi; // sample range of each band
  std::vector<double> band_zp_ab;       // AB zero-point flux of each band
  int n_cu = 1;
  size_t max_lds = 65536;
  std::mutex mu;                       // band registration, server start
  sbh::Server* server = nullptr;
  // per-stream device workspace (the adjoint's per-band partial sums): calls on one stream
  // run in order, so each stream keeps one buffer, grown on demand
  struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
  };
  std::mutex ws_mu;
  std::unordered_map<void*, Workspace> ws;

  sbk::KTables tables() const {
    sbk::KTables t;
    t.surf = d_surf;
    t.pts = d_pts;
    t.npts = d_npts;
    t.max_pts = max_pts;
    t.jcap = jcap;
    t.surf_bytes = (int)((size_t)(km.n_wave + sbk::SURF_PAD_COLS) * km.row_pad * sizeof(float2));
    t.lds_limit = (int)max_lds;
    return t;
  }
};
