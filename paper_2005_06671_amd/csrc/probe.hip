// Measurement probes (tools, not part of the method).
//
// Gather throughput of the memory system: every lane walks an xorshift
// sequence and sums the floats it addresses, so no index array competes with
// the gathers for bandwidth.  Indices cover the largest power of two <= n
// floats, or a window of `window` floats (a power of two) chosen per lane;
// iters is rounded up to a multiple of 8.
//
// FP32 VALU rate: every lane runs eight independent chains of non-packed FMAs
// (32 per iteration), enough independent work to keep a SIMD issuing.
#include "kernels.h"

namespace ss {

__global__ __launch_bounds__(256) void gather_probe_kernel(const float* __restrict__ src,
                                                           unsigned mask, unsigned wmask,
                                                           unsigned nwin, int iters,
                                                           float* __restrict__ out) {
  const unsigned tid = blockIdx.x * 256u + threadIdx.x;
  unsigned x = tid * 2654435761u + 12345u;
  x ^= x >> 16;
  const unsigned base = wmask ? ((x % nwin) * (wmask + 1u)) : 0u;
  // eight independent loads in flight per lane
  float acc[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  for (int k = 0; k < iters; k += 8) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      x ^= x << 13;
      x ^= x >> 17;
      x ^= x << 5;
      const unsigned idx = wmask ? base + (x & wmask) : (x & mask);
      acc[q] += src[idx];
    }
  }
  out[tid] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

hipError_t launch_gather_probe(const float* src, long long n_floats, long long window, int iters,
                               float* out, long long n_threads, hipStream_t stream) {
  unsigned long long p = 1;
  while (p * 2 <= (unsigned long long)n_floats) p *= 2;
  const unsigned mask = (unsigned)(p - 1);
  const unsigned wmask = window > 0 ? (unsigned)(window - 1) : 0u;
  const unsigned nwin = window > 0 ? (unsigned)(p / (unsigned long long)window) : 1u;
  hipLaunchKernelGGL(gather_probe_kernel, dim3((unsigned)(n_threads / 256)), dim3(256), 0, stream,
                     src, mask, wmask, nwin, iters, out);
  return hipGetLastError();
}

// Coherent gathers, as the shadow rays issue them: the 64 lanes of a
// wavefront read one 8 x 8 patch of a [rows][width] image (lane k: row k / 8,
// column k % 8), the patch origin drawn per wavefront and step from a
// wave-uniform xorshift sequence, eight patches in flight per lane.
__global__ __launch_bounds__(256) void gather_tiles_probe_kernel(const float* __restrict__ src,
                                                                 unsigned width, unsigned span_x,
                                                                 unsigned span_y, int iters,
                                                                 float* __restrict__ out) {
  const unsigned lane = threadIdx.x & 63u;
  const unsigned wave = blockIdx.x * 4u + (threadIdx.x >> 6);
  unsigned x = wave * 2654435761u + 97u;
  x ^= x >> 16;
  const unsigned lx = lane & 7u, ly = lane >> 3;
  float acc[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  for (int k = 0; k < iters; k += 8) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      x ^= x << 13;
      x ^= x >> 17;
      x ^= x << 5;
      const unsigned px = (x & 0xffffu) % span_x, py = (x >> 16) % span_y;
      acc[q] += src[(size_t)(py + ly) * width + px + lx];
    }
  }
  out[blockIdx.x * 256u + threadIdx.x] =
      ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

hipError_t launch_gather_tiles_probe(const float* src, int width, int rows, int iters, float* out,
                                     long long n_threads, hipStream_t stream) {
  hipLaunchKernelGGL(gather_tiles_probe_kernel, dim3((unsigned)(n_threads / 256)), dim3(256), 0,
                     stream, src, (unsigned)width, (unsigned)(width - 7), (unsigned)(rows - 7),
                     iters, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void valu_probe_kernel(int iters, float a, float b,
                                                         float* __restrict__ out) {
  const float x = (float)threadIdx.x * 1e-3f;
  float c0 = x, c1 = x + 1.0f, c2 = x + 2.0f, c3 = x + 3.0f;
  float c4 = x + 4.0f, c5 = x + 5.0f, c6 = x + 6.0f, c7 = x + 7.0f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      c0 = fmaf(c0, a, b);
      c1 = fmaf(c1, a, b);
      c2 = fmaf(c2, a, b);
      c3 = fmaf(c3, a, b);
      c4 = fmaf(c4, a, b);
      c5 = fmaf(c5, a, b);
      c6 = fmaf(c6, a, b);
      c7 = fmaf(c7, a, b);
    }
  }
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = ((c0 + c1) + (c2 + c3)) + ((c4 + c5) + (c6 + c7));
}

hipError_t launch_valu_probe(int iters, long long n_workgroups, float* out, hipStream_t stream) {
  hipLaunchKernelGGL(valu_probe_kernel, dim3((unsigned)n_workgroups), dim3(256), 0, stream, iters,
                     0.999f, 0.001f, out);
  return hipGetLastError();
}

}  // namespace ss
