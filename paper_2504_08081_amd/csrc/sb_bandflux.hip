// Bandflux, adjoint and sweep kernels (gfx950).
//
// One workgroup of NW waves evaluates one supernova (or one parameter sample
// of a sweep): it scans the supernova's observations for the bands they use
// and the surface rows their phases touch, then, a group of bands at a time,
// its waves build the bands' wavelength weight vectors and row projections
// (sb_device.h, one band per wave at a time) and the whole workgroup finishes
// every observation of the group's bands with a 4-tap phase interpolation.
// The adjoint accumulates sum_i gbar_i d f_i / d theta per thread and reduces
// it over the workgroup in a fixed order, so one writer produces each
// supernova's gradient without atomics.
#include <climits>

#include "sb_device.h"

namespace sbk {

struct SnShared {
  unsigned mask[2];
  int rlo[SB_MAX_BANDS];
  int rhi[SB_MAX_BANDS];
  int slot_of[SB_MAX_BANDS];   // band -> its slot in the current group, -1 otherwise
  int slot_ok[BAND_GROUP];
  float red[red_floats(8, MAX_NW)];
};

// Per-observation outputs of an observation that cannot be evaluated.
template <int MODE>
__device__ inline void write_obs(const KBatch& b, size_t o, float f, const float* d) {
  if (MODE == FWD) {
    if (!(b.flags & SB_OUT_CHI2)) b.flux[o] = f;
  } else {
    if (b.flux) b.flux[o] = f;
    if (b.jac) {
#pragma unroll
      for (int q = 0; q < SB_N_PARAMS; ++q) b.jac[o * SB_N_PARAMS + q] = d[q];
    }
  }
}

// Evaluate supernova (or sample) `sn` with a workgroup of NW waves.  All
// threads of the workgroup call it.
template <int MODE, bool BCAST, int NW>
__device__ void sn_body(const KModel& m, const KTables& tb, const KBatch& b, int sn, const Lds& L,
                        SnShared& S) {
  constexpr int NR = ModeInfo<MODE>::NR, NT = NW * WAVE;
  // The adjoint's observation pass always spreads the observations over the
  // threads of the mode's own wave count, so that each thread's partial sums,
  // and hence the gradient's summation order, do not depend on how many waves
  // built the row projections (extra waves contribute exact zeros).
  constexpr int OBS_NT = MODE == VJP ? (NT < ModeInfo<VJP>::NW * WAVE ? NT : ModeInfo<VJP>::NW * WAVE) : NT;
  const int tid = threadIdx.x;
  const bool chi2 = (b.flags & SB_OUT_CHI2) != 0;
  const float z = b.z[sn], t0 = b.t0[sn], x0 = b.x0[sn], x1 = b.x1[sn], c = b.c[sn];
  const double s64 = 1.0 / (1.0 + (double)z);
  const float s = (float)s64;
  const float A = (float)((double)x0 * s64);
  const float qnan = __builtin_nanf("");

  int lo = 0, hi = b.n_obs;
  bool csr_bad = false;
  if (!BCAST) {
    lo = b.off[sn];
    hi = b.off[sn + 1];
    if (lo < 0 || hi < lo || hi > b.n_obs) {
      csr_bad = true;
      lo = hi = 0;
    }
  }
  const size_t obase = BCAST ? (size_t)sn * (size_t)b.n_obs : 0;

  reset_scan(S.mask, S.rlo, S.rhi, S.slot_of);
  __syncthreads();

  // acc: gradient (z, t0, x0, x1, c) and chi2
  float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (csr_bad) {
    if (tid == 0) atomicOr(b.err, EFLAG_CSR);
#pragma unroll
    for (int q = 0; q < 6; ++q) acc[q] = qnan;
  }

  // scan: bands in use, rows touched; observations with nothing to integrate
  // (their chi-square terms join the threads' partial sums: same layout as below)
  for (int i = lo + tid; tid < OBS_NT && i < hi; i += OBS_NT) {
    const int bd = b.band[i];
    const PhaseCell pc = phase_cell(b.t[i], t0, s64, m);
    const bool bad_band = (unsigned)bd >= (unsigned)m.n_bands;
    if (bad_band || pc.nan) {
      if (bad_band) atomicOr(b.err, EFLAG_BAND);
      const float dn[5] = {qnan, qnan, qnan, qnan, qnan};
      write_obs<MODE>(b, obase + i, qnan, dn);
#pragma unroll
      for (int q = 0; q < 6; ++q) acc[q] = qnan;
      continue;
    }
    if (!pc.in) {
      const float d0[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
      write_obs<MODE>(b, obase + i, 0.f, d0);
      if (chi2) {
        const float r = -b.data[i];
        acc[5] = fmaf(r * r, b.w[i], acc[5]);
      }
      continue;
    }
    atomicMin(&S.rlo[bd], pc.r0);
    atomicMax(&S.rhi[bd], pc.r1);
    atomicOr(&S.mask[bd >> 5], 1u << (bd & 31));
  }
  __syncthreads();

  unsigned rem0 = (unsigned)uni((int)S.mask[0]), rem1 = (unsigned)uni((int)S.mask[1]);
  while (rem0 | rem1) {
    unsigned g0, g1;
    take_group(rem0, rem1, g0, g1, ModeInfo<MODE>::GROUP);
    // row projections of every band of the group, one band per wave at a time
    group_rows<MODE, NW>(m, tb, g0, g1, s64, c, x1, S.rlo, S.rhi, S.slot_of, S.slot_ok, L, b.err);
    __syncthreads();

    // every observation of the group's bands, in one pass
    for (int i = lo + tid; tid < OBS_NT && i < hi; i += OBS_NT) {
      const int bd = b.band[i];
      if ((unsigned)bd >= (unsigned)m.n_bands) continue;
      const int slot = S.slot_of[bd];
      if (slot < 0) continue;
      const PhaseCell pc = phase_cell(b.t[i], t0, s64, m);
      if (!pc.in) continue;
      const int rlo = S.rlo[bd], rhi = S.rhi[bd];
      const float* Rb = L.R + (size_t)slot * m.n_phase * NR;
      float f, dv[5];
      if (!S.slot_ok[slot]) {
        f = qnan;
#pragma unroll
        for (int q = 0; q < 5; ++q) dv[q] = qnan;
      } else {
        float wp[4];
        cr_weights(pc.x, pc.edge, wp);
        // all four taps (an edge cell's outer weights are zero and add exact zeros; the
        // clamped rows are rows the band wrote), so the loop unrolls
        float Sx = 0.f;
        if constexpr (MODE == FWD) {
#pragma unroll
          for (int t = 0; t < 4; ++t) Sx = fmaf(wp[t], Rb[row_clamp(pc.a - 1 + t, rlo, rhi) * NR], Sx);
          f = A * Sx;
        } else {
          float S1 = 0.f, Sc = 0.f, Sl = 0.f, Sp = 0.f;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const float* r = Rb + row_clamp(pc.a - 1 + t, rlo, rhi) * NR;
            Sx = fmaf(wp[t], r[0], Sx);
            S1 = fmaf(wp[t], r[1], S1);
            Sc = fmaf(wp[t], r[2], Sc);
            Sl = fmaf(wp[t], r[3], Sl);
          }
          // the phase derivative on the projected phase differences Rd (rows rlo .. rhi-1):
          // sum_t dw_t R(a-1+t) = sum_{t<3} e_t Rd(a-1+t); edge cells: Rd(a)
          float e[3];
          cr_diff_weights(pc.x, pc.edge, e);
#pragma unroll
          for (int t = 0; t < 3; ++t) Sp = fmaf(e[t], Rb[row_clamp(pc.a - 1 + t, rlo, rhi - 1) * NR + 4], Sp);
          Sp *= m.inv_dphase;
          f = A * Sx;
          const float As = A * s;
          dv[0] = -s * f - As * fmaf(pc.p, Sp, Sl);   // z
          dv[1] = -As * Sp;                           // t0
          dv[2] = s * Sx;                             // x0
          dv[3] = A * S1;                             // x1
          dv[4] = A * Sc;                             // c
        }
      }
      if (MODE == FWD) {
        if (chi2) {
          const float r = f - b.data[i];
          acc[5] = fmaf(r * r, b.w[i], acc[5]);
        } else {
          b.flux[obase + i] = f;
        }
      } else {
        write_obs<MODE>(b, obase + i, f, dv);
        float gbar;
        if (chi2) {
          const float r = f - b.data[i];
          const float wi = b.w[i];
          acc[5] = fmaf(r * r, wi, acc[5]);
          gbar = 2.f * r * wi;
        } else {
          gbar = b.cot[obase + i];
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[q] = fmaf(gbar, dv[q], acc[q]);
      }
    }
    __syncthreads();
    // release the group's slots
    for (int h = 0; h < 2; ++h) {
      unsigned gm = h ? g1 : g0;
      while (gm) {
        const int bd = h * 32 + __ffs(gm) - 1;
        gm &= gm - 1;
        if (tid == 0) S.slot_of[bd] = -1;
      }
    }
  }

  if (MODE == VJP) {
    block_sum<6, NW>(acc, S.red);
    if (tid == 0) {
#pragma unroll
      for (int q = 0; q < 5; ++q) b.grad[(size_t)sn * SB_N_PARAMS + q] = acc[q];
      if (chi2 && b.chi2) b.chi2[sn] = acc[5];
    }
  } else if (chi2) {
    float a1[1] = {acc[5]};
    block_sum<1, NW>(a1, S.red);
    if (tid == 0) b.chi2[sn] = a1[0];
  }
}

// Workgroup `bid` of `n` goes to XCD bid mod N_XCD (the dispatcher hands workgroups
// to the XCDs in turn).  This maps the workgroups so that XCD x takes the
// contiguous items [x q + min(x, r), ...) (q = n div N_XCD, r = n mod N_XCD, the
// first r XCDs one more) in order: neighbouring supernovae share the cache lines
// at the ends of their observation ranges, which are then fetched into one L2
// instead of two.  A bijection of [0, n) for any n.
__device__ inline int xcd_item(int bid, int n) {
  const int q = n / N_XCD, r = n % N_XCD, x = bid % N_XCD;
  return x * q + min(x, r) + bid / N_XCD;
}

template <int MODE, bool BCAST, int NW>
// At most 102 VGPRs (five waves per SIMD): the adjoint then takes 93 without
// spilling, and six of its three-wave workgroups fit a CU's registers and LDS
// (4% faster on 4,096 supernovae than five at 116 VGPRs).  The forward takes 55.
__global__ __launch_bounds__(NW * WAVE) __attribute__((amdgpu_waves_per_eu(5))) void k_sn(KModel m, KTables tb, KBatch b) {
  extern __shared__ __align__(16) char smem[];
  __shared__ SnShared S;
  const Lds L = lds_carve<MODE, NW>(smem, m, tb, uni((int)(threadIdx.x / WAVE)));
  sn_body<MODE, BCAST, NW>(m, tb, b, xcd_item(blockIdx.x, gridDim.x), L, S);
}

// A sweep as a persistent launch: workgroup g evaluates samples g, g + G, ...
// (G = the grid), each exactly as k_sn's workgroup for that sample would; the
// loop bounds are uniform, and a barrier separates one sample's last reads of
// the shared tables from the next sample's scan.
template <int MODE, int NW>
__global__ __launch_bounds__(NW * WAVE) __attribute__((amdgpu_waves_per_eu(5))) void k_sweep(KModel m, KTables tb,
                                                                                           KBatch b) {
  extern __shared__ __align__(16) char smem[];
  __shared__ SnShared S;
  const Lds L = lds_carve<MODE, NW>(smem, m, tb, uni((int)(threadIdx.x / WAVE)));
  const int n = uni(b.n_sn), step = uni((int)gridDim.x);
  for (int s = uni((int)blockIdx.x); s < n; s += step) {
    sn_body<MODE, true, NW>(m, tb, b, s, L, S);
    __syncthreads();
  }
}

// ------------------------------------------------------------ adjoint by band
//
// With few bands registered the adjoint runs one wave per (supernova, band): its
// workgroups are a sixth of a supernova's, so a batch of a few thousand supernovae
// fills the GPU with many short workgroups instead of a few long ones whose last
// round leaves compute units idle.  Wave (s, b) scans supernova s's observations
// for band b (the row range its phases touch, and the first and last such
// observation), builds the band's row projections with band_rows, finishes every
// observation of the band, and writes its six sums (gradient and chi2), summed
// over its lanes in a fixed order, to part[s][b].  k_band_sum then adds the bands'
// sums in band order: one writer per supernova, no float atomics, and every result
// independent of the rest of the batch and of the launch shape.  Observations
// whose band id is out of range are the band-0 wave's (NaN and the range flag).

__device__ inline int wave_min_i(int x) {
  for (int o = 1; o < WAVE; o <<= 1) x = min(x, __shfl_xor(x, o, WAVE));
  return x;
}
__device__ inline int wave_max_i(int x) {
  for (int o = 1; o < WAVE; o <<= 1) x = max(x, __shfl_xor(x, o, WAVE));
  return x;
}

// Dynamic LDS of a band workgroup: one wave's scratch and one band's row projections.
__host__ __device__ inline size_t band_lds_bytes(const KModel& m, int max_pts, int jcap) {
  return wave_scratch_bytes<VJP>(max_pts, jcap) + (size_t)m.n_phase * ModeInfo<VJP>::NR * sizeof(float);
}

template <bool BCAST>
__device__ void band_body(const KModel& m, const KTables& tb, const KBatch& b, int item, int nb, const Lds& L) {
  constexpr int NR = ModeInfo<VJP>::NR;
  const int lane = threadIdx.x & (WAVE - 1);
  const int sn = uni(item / nb), bd = uni(item - sn * nb);
  const bool chi2 = (b.flags & SB_OUT_CHI2) != 0;
  const float z = b.z[sn], t0 = b.t0[sn], x0 = b.x0[sn], x1 = b.x1[sn], c = b.c[sn];
  const double s64 = 1.0 / (1.0 + (double)z);
  const float s = (float)s64;
  const float A = (float)((double)x0 * s64);
  const float qnan = __builtin_nanf("");

  int lo = 0, hi = b.n_obs;
  bool csr_bad = false;
  if (!BCAST) {
    lo = b.off[sn];
    hi = b.off[sn + 1];
    if (lo < 0 || hi < lo || hi > b.n_obs) {
      csr_bad = true;
      lo = hi = 0;
    }
  }
  lo = uni(lo);
  hi = uni(hi);
  const size_t obase = BCAST ? (size_t)sn * (size_t)b.n_obs : 0;

  // the lane's sums start with the scan's chi-square terms (c2) and a NaN for
  // observations that cannot be evaluated (bad); two registers, not six, stay live
  // through band_rows
  float c2 = 0.f;
  bool bad = false;
  if (csr_bad && bd == 0) {
    if (lane == 0) atomicOr(b.err, EFLAG_CSR);
    bad = true;
  }

  // scan: the band's observations, the rows their phases touch; observations with
  // nothing to integrate (their chi-square terms join the lane's sums)
  int rlo = INT_MAX, rhi = -1, first = INT_MAX, last = -1;
  for (int i = lo + lane; i < hi; i += WAVE) {
    const int bi = b.band[i];
    if ((unsigned)bi >= (unsigned)m.n_bands) {
      if (bd == 0) {
        atomicOr(b.err, EFLAG_BAND);
        const float dn[5] = {qnan, qnan, qnan, qnan, qnan};
        write_obs<VJP>(b, obase + i, qnan, dn);
        bad = true;
      }
      continue;
    }
    if (bi != bd) continue;
    const PhaseCell pc = phase_cell(b.t[i], t0, s64, m);
    if (pc.nan) {
      const float dn[5] = {qnan, qnan, qnan, qnan, qnan};
      write_obs<VJP>(b, obase + i, qnan, dn);
      bad = true;
      continue;
    }
    if (!pc.in) {
      const float d0[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
      write_obs<VJP>(b, obase + i, 0.f, d0);
      if (chi2) {
        const float r = -b.data[i];
        c2 = fmaf(r * r, b.w[i], c2);
      }
      continue;
    }
    rlo = min(rlo, pc.r0);
    rhi = max(rhi, pc.r1);
    first = min(first, i);
    last = max(last, i);
  }
  rlo = uni(wave_min_i(rlo));
  rhi = uni(wave_max_i(rhi));
  first = uni(wave_min_i(first));
  last = uni(wave_max_i(last));

  // acc: gradient (z, t0, x0, x1, c) and chi2
  float acc[6];
  if (rhi >= 0) {
    const bool ok = band_rows<VJP>(m, tb, bd, s64, c, x1, rlo, rhi, L, L.R);
#pragma unroll
    for (int q = 0; q < 5; ++q) acc[q] = bad ? qnan : 0.f;
    acc[5] = bad ? qnan : c2;
    if (!ok && lane == 0) atomicOr(b.err, EFLAG_WINDOW);
    const float* Rb = L.R;
    // every observation of the band, between the first and the last one found
    for (int i = first + lane; i <= last; i += WAVE) {
      if (b.band[i] != bd) continue;
      const PhaseCell pc = phase_cell(b.t[i], t0, s64, m);
      if (!pc.in) continue;
      float f, dv[5];
      if (!ok) {
        f = qnan;
#pragma unroll
        for (int q = 0; q < 5; ++q) dv[q] = qnan;
      } else {
        float wp[4];
        cr_weights(pc.x, pc.edge, wp);
        // all four taps, as in sn_body
        float Sx = 0.f, S1 = 0.f, Sc = 0.f, Sl = 0.f, Sp = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const float* r = Rb + row_clamp(pc.a - 1 + t, rlo, rhi) * NR;
          Sx = fmaf(wp[t], r[0], Sx);
          S1 = fmaf(wp[t], r[1], S1);
          Sc = fmaf(wp[t], r[2], Sc);
          Sl = fmaf(wp[t], r[3], Sl);
        }
        // the phase derivative on the projected phase differences Rd (rows rlo .. rhi-1)
        float e[3];
        cr_diff_weights(pc.x, pc.edge, e);
#pragma unroll
        for (int t = 0; t < 3; ++t) Sp = fmaf(e[t], Rb[row_clamp(pc.a - 1 + t, rlo, rhi - 1) * NR + 4], Sp);
        Sp *= m.inv_dphase;
        f = A * Sx;
        const float As = A * s;
        dv[0] = -s * f - As * fmaf(pc.p, Sp, Sl);   // z
        dv[1] = -As * Sp;                           // t0
        dv[2] = s * Sx;                             // x0
        dv[3] = A * S1;                             // x1
        dv[4] = A * Sc;                             // c
      }
      write_obs<VJP>(b, obase + i, f, dv);
      float gbar;
      if (chi2) {
        const float r = f - b.data[i];
        const float wi = b.w[i];
        acc[5] = fmaf(r * r, wi, acc[5]);
        gbar = 2.f * r * wi;
      } else {
        gbar = b.cot[obase + i];
      }
#pragma unroll
      for (int q = 0; q < 5; ++q) acc[q] = fmaf(gbar, dv[q], acc[q]);
    }
  } else {
#pragma unroll
    for (int q = 0; q < 5; ++q) acc[q] = bad ? qnan : 0.f;
    acc[5] = bad ? qnan : c2;
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) acc[q] = wave_sum(acc[q]);
  if (lane == 0) {
    float* p = b.part + (size_t)item * PART_WORDS;
#pragma unroll
    for (int q = 0; q < PART_WORDS; ++q) p[q] = acc[q];
  }
  // the next item's band_rows rewrites the scratch this item's observation pass read
  wave_sync();
}

// Items (supernova, band) = (it div nb, it mod nb) for it = g, g + G, ... (G the grid;
// one item per workgroup unless the launch is persistent), XCD-contiguous.
template <bool BCAST>
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(5))) void k_band(KModel m, KTables tb, KBatch b,
                                                                                       int nb) {
  extern __shared__ __align__(16) char smem[];
  const Lds L = lds_carve<VJP, 1>(smem, m, tb, 0);
  const int n_items = uni(b.n_sn * nb), step = uni((int)gridDim.x);
  for (int it = uni((int)blockIdx.x); it < n_items; it += step)
    band_body<BCAST>(m, tb, b, xcd_item(it, n_items), nb, L);
}

// Component q of supernova s's gradient (q < 5) or its chi2 (q = 5), one thread per
// (s, q): the bands' sums, all loaded at once, added in band order.
__global__ __launch_bounds__(256) void k_band_sum(const float* __restrict__ part, int n_sn, int nb,
                                                  float* __restrict__ grad, float* __restrict__ chi2) {
  const int id = blockIdx.x * 256 + threadIdx.x;
  if (id >= n_sn * PART_WORDS) return;
  const int sn = id / PART_WORDS, q = id - sn * PART_WORDS;
  const float* p = part + (size_t)sn * nb * PART_WORDS + q;
  float v[BAND_SPLIT_MAX];
#pragma unroll
  for (int k = 0; k < BAND_SPLIT_MAX; ++k) v[k] = k < nb ? p[k * PART_WORDS] : 0.f;
  float g = 0.f;
#pragma unroll
  for (int k = 0; k < BAND_SPLIT_MAX; ++k)
    if (k < nb) g += v[k];
  if (q < SB_N_PARAMS)
    grad[(size_t)sn * SB_N_PARAMS + q] = g;
  else if (chi2)
    chi2[sn] = g;
}

size_t lds_bytes(const KModel& m, int max_pts, int jcap, bool adj) {
  return adj ? lds_layout_bytes<VJP>(m.n_phase, max_pts, jcap, 1)
             : lds_layout_bytes<FWD>(m.n_phase, max_pts, jcap, 1);
}

template <typename K>
static hipError_t prep_lds(K kern, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int MODE, bool BCAST, int NW>
static hipError_t launch_nw(const KModel& m, const KTables& tb, const KBatch& b, size_t lds, hipStream_t st) {
  hipError_t e = prep_lds(k_sn<MODE, BCAST, NW>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_sn<MODE, BCAST, NW>), dim3(b.n_sn), dim3(NW * WAVE), lds, st, m, tb, b);
  return hipGetLastError();
}

// The mode's preferred number of waves per workgroup when its LDS fits, else one.
template <int MODE, bool BCAST>
static hipError_t launch_one(const KModel& m, const KTables& tb, const KBatch& b, hipStream_t st) {
  constexpr int NW = ModeInfo<MODE>::NW;
  const size_t lds = lds_layout_bytes<MODE>(m.n_phase, tb.max_pts, tb.jcap, NW);
  if (lds <= (size_t)tb.lds_limit) return launch_nw<MODE, BCAST, NW>(m, tb, b, lds, st);
  return launch_nw<MODE, BCAST, 1>(m, tb, b, lds_layout_bytes<MODE>(m.n_phase, tb.max_pts, tb.jcap, 1), st);
}

// A persistent sweep with k_sn's workgroup shape for the mode (so each sample's
// results are bitwise those of the one-workgroup-per-sample launch), never more
// workgroups than samples.  Samples differ in cost (z sets each band's window),
// so a static stride needs spare workgroups to balance: on 1,048,576 samples
// one workgroup per resident slot took 16.6 ms, PERSIST_ROUNDS = 16 per slot
// 13.5 ms, against 13.2 ms for one workgroup per sample (the hardware
// dispatcher balances dynamically and its per-workgroup cost is small).
constexpr int PERSIST_ROUNDS = 16;

template <int MODE, int NW>
static hipError_t launch_sweep_nw(const KModel& m, const KTables& tb, const KBatch& b, size_t lds, hipStream_t st) {
  hipError_t e = prep_lds(k_sweep<MODE, NW>, lds);
  if (e != hipSuccess) return e;
  int dev = 0, n_cu = 0, per_cu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep<MODE, NW>, NW * WAVE, lds);
  if (e != hipSuccess) return e;
  const long long slots = (long long)(per_cu > 0 ? per_cu : 1) * (n_cu > 0 ? n_cu : 1) * PERSIST_ROUNDS;
  const int grid = (int)(slots < b.n_sn ? slots : b.n_sn);
  hipLaunchKernelGGL((k_sweep<MODE, NW>), dim3(grid), dim3(NW * WAVE), lds, st, m, tb, b);
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch_sweep(const KModel& m, const KTables& tb, const KBatch& b, hipStream_t st) {
  constexpr int NW = ModeInfo<MODE>::NW;
  const size_t lds = lds_layout_bytes<MODE>(m.n_phase, tb.max_pts, tb.jcap, NW);
  if (lds <= (size_t)tb.lds_limit) return launch_sweep_nw<MODE, NW>(m, tb, b, lds, st);
  return launch_sweep_nw<MODE, 1>(m, tb, b, lds_layout_bytes<MODE>(m.n_phase, tb.max_pts, tb.jcap, 1), st);
}

// Forward calls that return fluxes only may use any number of waves per
// supernova: each observation's flux comes from its band's projections, built
// by one wave whatever the workgroup size, so the results are bit for bit the
// same (chi-square, a sum over the waves, keeps the mode's shape).  A few
// supernovae get one wave per band, which shortens the call; larger batches get
// three (two bands per wave for six bands, 2% faster than two waves).
constexpr int FEW_SN = 64;
constexpr int FEW_SN_NW = 8;
constexpr int FLUX_NW = 3;

// An adjoint call on a few supernovae: one wave per band of a group builds the
// row projections; the observation pass keeps the mode's thread layout
// (OBS_NT in sn_body), so every result is bit for bit that of the batch kernel.
constexpr int FEW_SN_VJP_NW = ModeInfo<VJP>::GROUP;

// The adjoint by band (b.part set by the host): k_band over every (supernova, band),
// or a persistent grid of them, then k_band_sum.
template <bool BCAST>
static hipError_t launch_band_t(const KModel& m, const KTables& tb, const KBatch& b, hipStream_t st) {
  const int nb = m.n_bands;
  const int items = b.n_sn * nb;
  const size_t lds = band_lds_bytes(m, tb.max_pts, tb.jcap);
  hipError_t e = prep_lds(k_band<BCAST>, lds);
  if (e != hipSuccess) return e;
  int grid = items;
  if (b.flags & SB_PERSISTENT) {
    int dev = 0, n_cu = 0, per_cu = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_band<BCAST>, WAVE, lds);
    if (e != hipSuccess) return e;
    const long long slots = (long long)(per_cu > 0 ? per_cu : 1) * (n_cu > 0 ? n_cu : 1) * PERSIST_ROUNDS;
    grid = (int)(slots < items ? slots : items);
  }
  hipLaunchKernelGGL((k_band<BCAST>), dim3(grid), dim3(WAVE), lds, st, m, tb, b, nb);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_band_sum, dim3((b.n_sn * PART_WORDS + 255) / 256), dim3(256), 0, st, (const float*)b.part,
                     b.n_sn, nb, b.grad, b.chi2);
  return hipGetLastError();
}

hipError_t launch_sn(bool adj, const KModel& m, const KTables& tb, const KBatch& b, hipStream_t st) {
  const bool bc = (b.flags & SB_OBS_BROADCAST) != 0;
  if (adj && b.part) return bc ? launch_band_t<true>(m, tb, b, st) : launch_band_t<false>(m, tb, b, st);
  if (bc && (b.flags & SB_PERSISTENT)) return adj ? launch_sweep<VJP>(m, tb, b, st) : launch_sweep<FWD>(m, tb, b, st);
  if (adj && !bc && b.n_sn <= FEW_SN) {
    const size_t lds = lds_layout_bytes<VJP>(m.n_phase, tb.max_pts, tb.jcap, FEW_SN_VJP_NW);
    if (lds <= (size_t)tb.lds_limit) return launch_nw<VJP, false, FEW_SN_VJP_NW>(m, tb, b, lds, st);
  }
  if (adj) return bc ? launch_one<VJP, true>(m, tb, b, st) : launch_one<VJP, false>(m, tb, b, st);
  if (!bc && !(b.flags & SB_OUT_CHI2)) {
    if (b.n_sn <= FEW_SN) {
      const size_t lds = lds_layout_bytes<FWD>(m.n_phase, tb.max_pts, tb.jcap, FEW_SN_NW);
      if (lds <= (size_t)tb.lds_limit) return launch_nw<FWD, false, FEW_SN_NW>(m, tb, b, lds, st);
    }
    const size_t lds = lds_layout_bytes<FWD>(m.n_phase, tb.max_pts, tb.jcap, FLUX_NW);
    if (lds <= (size_t)tb.lds_limit) return launch_nw<FWD, false, FLUX_NW>(m, tb, b, lds, st);
  }
  return bc ? launch_one<FWD, true>(m, tb, b, st) : launch_one<FWD, false>(m, tb, b, st);
}

}  // namespace sbk
