// Exercises the saltbf C ABI from plain C++ (no Python, no torch): reads a
// model, bands and a batch from a raw little-endian input file, evaluates the
// bandflux (sb_bandflux) and the cotangent gradient (sb_bandflux_vjp) on
// device buffers it allocates with the HIP runtime, and writes the fluxes and
// gradients to an output file.  Test infrastructure: tests/test_gpu_cabi.py
// writes the input and compares the output with the oracle.
//
// Input layout (all little-endian):
//   int32  n_phase, n_wave, cl_degree, n_bands, n_sn, n_obs
//   double phase0, dphase, wave0, dwave, cl_wave_b, cl_wave_v
//   double cl_coef[cl_degree]
//   float  m0[n_phase * n_wave], m1[n_phase * n_wave]
//   per band: int32 n, double wave[n], double trans[n]
//   float  z[n_sn], t0[n_sn], x0[n_sn], x1[n_sn], c[n_sn]
//   float  t[n_obs]; int32 band[n_obs]; int32 sn_offsets[n_sn + 1]; float cotangent[n_obs]
// Output layout: float flux[n_obs], float grad[n_sn * 5].
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "saltbf.h"

namespace {

bool rd(FILE* f, void* p, size_t bytes) { return bytes == 0 || fread(p, 1, bytes, f) == bytes; }

template <typename T>
bool rdv(FILE* f, std::vector<T>& v, size_t n) {
  v.resize(n);
  return rd(f, v.data(), n * sizeof(T));
}

int fail(const char* what, sb_status st) {
  fprintf(stderr, "%s: %s (%s)\n", what, sb_status_string(st), sb_last_error());
  return 1;
}

template <typename T>
T* upload(const std::vector<T>& h) {
  T* d = nullptr;
  if (hipMalloc(&d, h.size() * sizeof(T) + 16) != hipSuccess) return nullptr;
  if (!h.empty() && hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
  return d;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s input output\n", argv[0]);
    return 2;
  }
  FILE* in = fopen(argv[1], "rb");
  if (!in) return 2;
  int32_t hdr[6];
  double geo[6];
  if (!rd(in, hdr, sizeof hdr) || !rd(in, geo, sizeof geo)) return 2;
  const int n_phase = hdr[0], n_wave = hdr[1], cl_deg = hdr[2], n_bands = hdr[3], n_sn = hdr[4], n_obs = hdr[5];
  std::vector<double> cl;
  std::vector<float> m0, m1;
  if (!rdv(in, cl, cl_deg) || !rdv(in, m0, (size_t)n_phase * n_wave) || !rdv(in, m1, (size_t)n_phase * n_wave))
    return 2;
  sb_model_desc md{n_phase, n_wave, geo[0], geo[1], geo[2], geo[3], m0.data(), m1.data(), cl_deg, cl.data(),
                   geo[4], geo[5]};
  sb_config cfg;
  sb_config_default(&cfg);
  sb_ctx* ctx = nullptr;
  sb_status st = sb_create(&md, &cfg, 0, &ctx);
  if (st != SB_OK) return fail("sb_create", st);
  for (int b = 0; b < n_bands; ++b) {
    int32_t n = 0;
    std::vector<double> w, tr;
    if (!rd(in, &n, sizeof n) || !rdv(in, w, n) || !rdv(in, tr, n)) return 2;
    int32_t id = -1;
    st = sb_add_band(ctx, w.data(), tr.data(), n, &id);
    if (st != SB_OK) return fail("sb_add_band", st);
  }
  std::vector<float> z, t0, x0, x1, c, t, cot;
  std::vector<int32_t> band, off;
  if (!rdv(in, z, n_sn) || !rdv(in, t0, n_sn) || !rdv(in, x0, n_sn) || !rdv(in, x1, n_sn) || !rdv(in, c, n_sn) ||
      !rdv(in, t, n_obs) || !rdv(in, band, n_obs) || !rdv(in, off, (size_t)n_sn + 1) || !rdv(in, cot, n_obs))
    return 2;
  fclose(in);

  sb_batch b{};
  b.n_sn = n_sn;
  b.n_obs = n_obs;
  b.flags = 0;
  b.z = upload(z);
  b.t0 = upload(t0);
  b.x0 = upload(x0);
  b.x1 = upload(x1);
  b.c = upload(c);
  b.t = upload(t);
  b.band = upload(band);
  b.sn_offsets = upload(off);
  const float* d_cot = upload(cot);
  float *d_flux = nullptr, *d_grad = nullptr;
  if (!b.z || !b.t0 || !b.x0 || !b.x1 || !b.c || !b.t || !b.band || !b.sn_offsets || !d_cot ||
      hipMalloc(&d_flux, (size_t)n_obs * sizeof(float) + 16) != hipSuccess ||
      hipMalloc(&d_grad, (size_t)n_sn * 5 * sizeof(float) + 16) != hipSuccess) {
    fprintf(stderr, "device allocation failed\n");
    return 1;
  }
  hipStream_t stream;
  if (hipStreamCreate(&stream) != hipSuccess) return 1;
  st = sb_bandflux(ctx, &b, d_flux, stream);
  if (st != SB_OK) return fail("sb_bandflux", st);
  st = sb_bandflux_vjp(ctx, &b, d_cot, d_grad, nullptr, nullptr, nullptr, stream);
  if (st != SB_OK) return fail("sb_bandflux_vjp", st);
  st = sb_device_check(ctx, stream);
  if (st != SB_OK) return fail("sb_device_check", st);
  std::vector<float> flux(n_obs), grad((size_t)n_sn * 5);
  if ((n_obs && hipMemcpy(flux.data(), d_flux, n_obs * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) ||
      hipMemcpy(grad.data(), d_grad, grad.size() * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return 1;
  FILE* out = fopen(argv[2], "wb");
  if (!out) return 2;
  fwrite(flux.data(), sizeof(float), flux.size(), out);
  fwrite(grad.data(), sizeof(float), grad.size(), out);
  fclose(out);
  (void)hipStreamDestroy(stream);
  for (const void* p : {(const void*)b.z, (const void*)b.t0, (const void*)b.x0, (const void*)b.x1, (const void*)b.c,
                        (const void*)b.t, (const void*)b.band, (const void*)b.sn_offsets, (const void*)d_cot})
    (void)hipFree(const_cast<void*>(p));
  (void)hipFree(d_flux);
  (void)hipFree(d_grad);
  st = sb_destroy(ctx);
  if (st != SB_OK) return fail("sb_destroy", st);
  printf("ok %d obs %d sn\n", n_obs, n_sn);
  return 0;
}
