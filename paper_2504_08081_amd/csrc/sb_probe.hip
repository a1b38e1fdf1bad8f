// Peak-rate probes (gfx950): kernels whose work is known exactly, so that a
// caller timing one launch measures the rate a roofline is quoted against on
// the device at hand, instead of taking a datasheet figure on trust.
//
//   FMA_F32   FP32 fused multiply-adds on the vector ALUs, one per lane per
//             instruction (packed FP32 is switched off in this library, so this
//             is the attainable ceiling of its kernels);
//   LDS_READ  128-bit LDS reads, consecutive lanes at consecutive addresses
//             (no bank conflicts);
//   COPY      a device-to-device copy with 128-bit loads and stores (HBM read +
//             write bytes).
//
// Every result is written out, so nothing can be optimised away, and the
// values follow closed forms the caller can check.
#include <algorithm>

#include "sb_internal.h"

namespace sbk {

constexpr int PROBE_THREADS = 256;
constexpr int FMA_CHAINS = 16;        // independent chains per thread: enough to hide the FMA latency
constexpr int LDS_VEC = 1024;         // float4 entries of the LDS table (16 KiB: eight workgroups fit a CU)

// x <- x * a + b, FMA_CHAINS chains of `iters` steps each; chain j starts at j.
__global__ __launch_bounds__(PROBE_THREADS) void k_probe_fma(float a, float b, int iters, float* out) {
  float x[FMA_CHAINS];
#pragma unroll
  for (int j = 0; j < FMA_CHAINS; ++j) x[j] = (float)j;
  for (int k = 0; k < iters; ++k) {
#pragma unroll
    for (int j = 0; j < FMA_CHAINS; ++j) x[j] = fmaf(x[j], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < FMA_CHAINS; ++j) s += x[j];
  out[(size_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = s;
}

// The table holds T[i] = (i, i + 1/4, i + 1/2, i + 3/4); in sweep k thread t reads
// entries (t xor (k mod 256)) + 256 r, r = 0 .. 3 (the sweep index changes the
// addresses, so no read can be hoisted out of the sweep loop; each group of eight
// lanes still reads eight consecutive-modulo-8 entries, one per bank quad), and
// writes the sum of all components it read.  One address per sweep, the four
// reads at immediate offsets: four adds per 128-bit read.
__global__ __launch_bounds__(PROBE_THREADS) void k_probe_lds(int iters, float* out) {
  __shared__ float4 T[LDS_VEC];
  for (int i = threadIdx.x; i < LDS_VEC; i += PROBE_THREADS)
    T[i] = make_float4((float)i, (float)i + 0.25f, (float)i + 0.5f, (float)i + 0.75f);
  __syncthreads();
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int k = 0; k < iters; ++k) {
    const float4* row = T + (threadIdx.x ^ (unsigned)(k & (PROBE_THREADS - 1)));
#pragma unroll
    for (int r = 0; r < LDS_VEC / PROBE_THREADS; ++r) {
      const float4 v = row[r * PROBE_THREADS];
      acc.x += v.x;
      acc.y += v.y;
      acc.z += v.z;
      acc.w += v.w;
    }
  }
  out[(size_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = (acc.x + acc.y) + (acc.z + acc.w);
}

// dst[i] = src[i] over n 16-byte entries, one per thread (grid-stride beyond 2^30
// workgroups), with non-temporal loads and stores: of the forms measured on a
// 1 GiB copy (grid-stride with 4 or 8 loads in flight per thread, cached or not,
// 2,048-16,384 workgroups; hipMemcpyAsync) this one moved the most bytes.
typedef float v4f __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(PROBE_THREADS) void k_probe_copy(const v4f* __restrict__ src, v4f* __restrict__ dst,
                                                              size_t n) {
  const size_t stride = (size_t)gridDim.x * PROBE_THREADS;
  for (size_t i = (size_t)blockIdx.x * PROBE_THREADS + threadIdx.x; i < n; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_probe(int kind, int64_t n, int iters, const void* src, void* dst, double* work,
                        hipStream_t st) {
  switch (kind) {
    case SB_PROBE_FMA_F32:
      // the multiplier and addend keep every chain bounded: x -> b / (1 - a) = 1
      hipLaunchKernelGGL(k_probe_fma, dim3((unsigned)n), dim3(PROBE_THREADS), 0, st, 0.9990234375f, 0.0009765625f,
                         iters, (float*)dst);
      *work = 2.0 * (double)n * PROBE_THREADS * (double)iters * FMA_CHAINS;
      break;
    case SB_PROBE_LDS_READ:
      hipLaunchKernelGGL(k_probe_lds, dim3((unsigned)n), dim3(PROBE_THREADS), 0, st, iters, (float*)dst);
      *work = (double)n * (double)iters * LDS_VEC * sizeof(float4);
      break;
    case SB_PROBE_COPY: {
      const size_t nv = (size_t)n / sizeof(v4f);
      const unsigned grid = (unsigned)std::min<size_t>((nv + PROBE_THREADS - 1) / PROBE_THREADS, (size_t)1 << 30);
      hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(PROBE_THREADS), 0, st, (const v4f*)src, (v4f*)dst, nv);
      *work = 2.0 * (double)n;
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sbk
