// Library-internal declarations shared by the host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "saltbf.h"

namespace sbk {

constexpr int WAVE = 64;           // threads per wavefront
constexpr int N_XCD = 8;           // accelerator complex dies (each with its own L2) of an MI355X
constexpr int MAX_NW = 8;          // wavefronts per workgroup, at most (per mode in sb_device.h)
constexpr int MAX_PHASE = 256;     // surface rows supported
constexpr int MAX_WAVE = 8192;     // surface columns supported
constexpr double WINDOW_Z_MIN = -0.05;  // the LDS window capacity covers every z >= this
constexpr int SURF_PAD_COLS = 16;  // zero columns after the last surface column (at least the widest chunk)
constexpr int BUF_RSRC_WORD3 = 0x00020000;  // buffer resource flags word (gfx9 family: raw 32-bit data)
constexpr unsigned BUF_OFF_NONE = 0x40000000u;  // a buffer offset past every resource: the load returns 0

// Sticky device error bits (sb_device_check maps any of them to SB_ERR_RANGE).
enum : int { EFLAG_WINDOW = 1, EFLAG_BAND = 2, EFLAG_CSR = 4 };

// Model constants, passed by value as a kernel argument.
struct KModel {
  int n_phase, n_wave, row_pad, n_bands;
  float phase0, inv_dphase, wave0, inv_dwave;
  double phase0_d, inv_dphase_d, wave0_d, inv_dwave_d;   // grid coordinates are formed in FP64
  float cl_b, cl_inv_span;
  int cl_deg;
  float cl[SB_MAX_CL_DEGREE];    // a_1..a_deg
  float dcl[SB_MAX_CL_DEGREE];   // n * a_n
};

// Device tables owned by the context.
struct KTables {
  const float2* surf;   // [n_wave + SURF_PAD_COLS][row_pad] of (M0, M1): node (a, j) -> surf[j*row_pad + a]
  const float2* pts;    // [n_bands][SB_MAX_BAND_POINTS] of (lam_k, W_k)
  const int* npts;      // [n_bands] node count per band
  int max_pts;          // largest node count over registered bands (sizes the LDS)
  int jcap;             // largest surface window (columns) a band can need for z >= WINDOW_Z_MIN
  int surf_bytes;       // size of surf in bytes
  int lds_limit;        // dynamic LDS bytes a workgroup may use (host side: picks the waves per workgroup)
};

// One bandflux / adjoint launch.
struct KBatch {
  int n_sn, n_obs, flags;
  const float *z, *t0, *x0, *x1, *c;
  const float* t;
  const int* band;
  const int* off;
  const float *data, *w, *cot;
  float *flux, *grad, *jac, *chi2;
  int* err;
  float* part;   // adjoint by band: [n_sn][n_bands][6] partial sums (workspace), or null
};

// The adjoint runs one wave per (supernova, band) and sums the bands' partials in a
// second kernel when at most this many bands are registered (the batch kernel
// launches a workgroup for every registered band of every supernova).
constexpr int BAND_SPLIT_MAX = 8;
constexpr int PART_WORDS = 6;     // per (supernova, band): the five gradient sums and chi2
inline size_t band_part_bytes(int n_sn, int n_bands) {
  return (size_t)n_sn * (size_t)n_bands * PART_WORDS * sizeof(float);
}

// Dynamic LDS bytes of the per-supernova pipeline in its smallest form (one
// wave per workgroup); launches use more waves where they fit in tb.lds_limit.
size_t lds_bytes(const KModel& m, int max_pts, int jcap, bool adj);

// One workgroup per supernova, or per parameter sample when the batch shares
// one observation table (forward, or forward + adjoint).
hipError_t launch_sn(bool adj, const KModel& m, const KTables& tb, const KBatch& b, hipStream_t st);

// ------------------------------------------------------------------ fit server

constexpr int LB_MAX_M = 5;       // L-BFGS-B correction pairs kept, at most

// Per-fit device state; lives in the server's slot array (or the batch fit's
// scratch) between launches.
struct FitSlot {
  int obs_off;      // first observation in the arena (batch fits: in the caller's arrays)
  int n_obs;
  int iter;         // iterations (evaluations) done; -1 = not yet evaluated at the start point
  int n_accept;
  int status;       // SB_OK / SB_FIT_DIVERGED
  int free_mask;    // SB_FREE_* bits of the parameters the fit varies
  int lb_phase;     // L-BFGS-B: needs a direction / in a line search / done
  int lb_n;         // L-BFGS-B: correction pairs kept
  int lb_first;     // L-BFGS-B: first iteration since a (re)start
  int lb_has_hi;    // L-BFGS-B line search: the bracket has an upper end
  int lb_trials;    // L-BFGS-B line search: evaluations in the current search
  int pad_;
  float z;
  float q[4];       // t0, ln x0, x1, c
  float lambda;     // LM damping
  float chi2;
  float H[10];      // LM: J^T W J, packed upper triangle (00 01 02 03 11 12 13 22 23 33)
  float g[4];       // J^T W r at q (chi2's gradient is -2 g)
  // L-BFGS-B (solver SB_SOLVER_LBFGSB)
  float lb_lo[4], lb_hi[4];              // bounds of q
  float lb_S[LB_MAX_M][4], lb_Y[LB_MAX_M][4];   // correction pairs, oldest first
  float lb_d[4], lb_trial[4];            // search direction, trial point
  float lb_gd, lb_a, lb_amax;            // slope along d at q, trial step, largest feasible step
  float lb_alo, lb_flo, lb_glo;          // best step of the search so far (chi2, slope)
  float lb_ahi, lb_fhi, lb_ghi;          // other end of the bracket
};

// A request admitted in this launch: copied from the inbox into its arena range
// and its slot initialised by the workgroup that then runs it.
struct AdmitHeader {
  int slot;
  int arena_off;
  int n_obs;
  int src_off;       // offset of its observations in the inbox arrays
  float z, t0, lnx0, x1, c;
  int free_mask;
  int pad_[2];
  float lo[4], hi[4];   // L-BFGS-B bounds of (t0, ln x0, x1, c); +-inf when none
};

struct KFit {
  FitSlot* slots;
  FitSlot* results;    // finished fits of this launch, at out_idx
  const int* active;   // slot ids of this launch
  const int* out_idx;  // >= 0: this launch finishes the fit, write its state there
  const int* admit;    // >= 0: index of its AdmitHeader (first launch of the fit)
  const AdmitHeader* hdr;
  const float* in_t;   // inbox observation arrays
  const int* in_band;
  const float* in_data;
  const float* in_w;
  int n_active;
  int iters;           // iterations to run this launch
  int fit_iters;       // total per fit
  int solver;          // SB_SOLVER_LM or SB_SOLVER_LBFGSB
  int lbfgs_m;         // L-BFGS-B correction pairs kept (1..LB_MAX_M)
  float lambda0;
  float* t;            // arena [capacity]: observations of resident fits
  int* band;
  float* data;
  float* w;            // 1/sigma^2
  int* err;
  // batch mode (sb_fit_batch): fit f is workgroup f and slot f; its observations are the
  // caller's CSR range; the first launch starts from the caller's arrays, the last one
  // writes the caller's results
  const int* b_off;    // non-null: batch mode
  const float *b_z, *b_t0, *b_x0, *b_x1, *b_c;
  const unsigned* b_free;
  const float *b_lower, *b_upper;   // [n_fit][4] L-BFGS-B bounds of (t0, x0, x1, c), or null
  const float* b_t;
  const int* b_band;
  const float* b_data;
  const float* b_w;
  int b_n_obs;
  int b_first, b_last;
  sb_fit_out* b_out;
};

hipError_t launch_fit(const KModel& m, const KTables& tb, const KFit& f, hipStream_t st);

// Batch fits: the fit kernel over n_fit fits in launches of iters_per_tick iterations, state in
// slots ([n_fit] device FitSlot).
hipError_t launch_fit_batch(const KModel& m, const KTables& tb, KFit f, int n_fit, int fit_iters,
                            int iters_per_tick, hipStream_t st);
size_t fit_lds_bytes(const KModel& m, int max_pts, int jcap);   // smallest form, as lds_bytes

// Peak-rate probes (sb_probe.hip): one launch of probe `kind` (SB_PROBE_*), its FLOPs or bytes in *work.
hipError_t launch_probe(int kind, int64_t n, int iters, const void* src, void* dst, double* work, hipStream_t st);

// The fixed per-device state array of allocation-free batch fits
// (SB_FIT_NOALLOC_MAX slots): fit_scratch_init takes its device address once per
// device (that device current); fit_scratch returns it, or null before.
hipError_t fit_scratch_init(int device);
FitSlot* fit_scratch(int device);

}  // namespace sbk
