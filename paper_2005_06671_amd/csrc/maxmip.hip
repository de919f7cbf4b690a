// Maximum mipmap for gfx950 (Sec. 3.2, "Maximum mipmaps").
//
// A 256-thread workgroup reads one 64 x 64 block of the source level with
// coalesced 16-byte loads (each thread a 4 x 4 patch: four rows of float4) and
// writes up to six levels of that block:
//   +1, +2  in registers (2 x 2 and 1 x 1 per thread),
//   +3, +4  by cross-lane max within the wavefront (no LDS),
//   +5, +6  through a 4 x 4 LDS tile.
// Every texel is read from HBM once per launch; levels are written once.
#include "kernels.h"

namespace ss {

struct MipDst {
  int off[6];
  int w[6];
  int h[6];
};

__device__ __forceinline__ float canon(float v) { return v + 0.0f; }  // -0 -> +0

template <int F>
__global__ __launch_bounds__(256) void maxmip_kernel(const float* __restrict__ src, int sw, int sh,
                                                     float* __restrict__ dst, MipDst d, int nbx,
                                                     int vec_ok) {
  __shared__ float lds[4][4];
  const int b = blockIdx.x;
  const int bx = b % nbx, by = b / nbx;
  const int t = threadIdx.x;
  const int c4 = t & 15, rg = t >> 4;
  const int col0 = bx * 64 + c4 * 4, row0 = by * 64 + rg * 4;
  const float NEG = -__builtin_inff();
  float v[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = row0 + r;
    if (row < sh && vec_ok && col0 + 3 < sw) {
      const float4 q = *reinterpret_cast<const float4*>(src + (size_t)row * sw + col0);
      v[r][0] = canon(q.x);
      v[r][1] = canon(q.y);
      v[r][2] = canon(q.z);
      v[r][3] = canon(q.w);
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        v[r][c] = (row < sh && col0 + c < sw) ? canon(src[(size_t)row * sw + col0 + c]) : NEG;
    }
  }
  // level +1: 2 x 2 per thread
  float a[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
      a[r][c] = fmaxf(fmaxf(v[2 * r][2 * c], v[2 * r][2 * c + 1]),
                      fmaxf(v[2 * r + 1][2 * c], v[2 * r + 1][2 * c + 1]));
  {
    const int w1 = d.w[0], h1 = d.h[0];
    float* L1 = dst + d.off[0];
    const int cc = bx * 32 + c4 * 2;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int rr = by * 32 + rg * 2 + r;
      if (rr < h1) {
        if ((w1 & 1) == 0 && cc + 1 < w1) {
          *reinterpret_cast<float2*>(L1 + (size_t)rr * w1 + cc) = make_float2(a[r][0], a[r][1]);
        } else {
          if (cc < w1) L1[(size_t)rr * w1 + cc] = a[r][0];
          if (cc + 1 < w1) L1[(size_t)rr * w1 + cc + 1] = a[r][1];
        }
      }
    }
  }
  if (F == 1) return;
  // level +2: one value per thread
  float b2 = fmaxf(fmaxf(a[0][0], a[0][1]), fmaxf(a[1][0], a[1][1]));
  {
    const int rr = by * 16 + rg, cc = bx * 16 + c4;
    if (rr < d.h[1] && cc < d.w[1]) dst[d.off[1] + (size_t)rr * d.w[1] + cc] = b2;
  }
  if (F == 2) return;
  // level +3: lanes (c4, c4^1) x (rg, rg^1) of the same wavefront
  float b3 = fmaxf(b2, __shfl_xor(b2, 1, 64));
  b3 = fmaxf(b3, __shfl_xor(b3, 16, 64));
  if (((c4 | rg) & 1) == 0) {
    const int rr = by * 8 + (rg >> 1), cc = bx * 8 + (c4 >> 1);
    if (rr < d.h[2] && cc < d.w[2]) dst[d.off[2] + (size_t)rr * d.w[2] + cc] = b3;
  }
  if (F == 3) return;
  // level +4: lanes (c4, c4^2) x (rg, rg^2)
  float b4 = fmaxf(b3, __shfl_xor(b3, 2, 64));
  b4 = fmaxf(b4, __shfl_xor(b4, 32, 64));
  if (((c4 | rg) & 3) == 0) {
    const int rr = by * 4 + (rg >> 2), cc = bx * 4 + (c4 >> 2);
    if (rr < d.h[3] && cc < d.w[3]) dst[d.off[3] + (size_t)rr * d.w[3] + cc] = b4;
    lds[rg >> 2][c4 >> 2] = b4;
  }
  if (F == 4) return;
  __syncthreads();
  if (t < 4) {
    const int r5 = t >> 1, c5 = t & 1;
    const float m5 = fmaxf(fmaxf(lds[2 * r5][2 * c5], lds[2 * r5][2 * c5 + 1]),
                           fmaxf(lds[2 * r5 + 1][2 * c5], lds[2 * r5 + 1][2 * c5 + 1]));
    const int rr = by * 2 + r5, cc = bx * 2 + c5;
    if (rr < d.h[4] && cc < d.w[4]) dst[d.off[4] + (size_t)rr * d.w[4] + cc] = m5;
  }
  if (F == 5) return;
  if (t == 0) {
    float m6 = lds[0][0];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) m6 = fmaxf(m6, lds[r][c]);
    if (by < d.h[5] && bx < d.w[5]) dst[d.off[5] + (size_t)by * d.w[5] + bx] = m6;
  }
}

// Tap-bound level 0: the maximum over the 3 x 3 block around each texel,
// clipped to the tile (repeating the edge row or column gives the same
// maximum), -0 stored as +0.  One thread per column strip of 8 rows: each row's
// 3-wide maximum is loaded once and the 3-row window slides down in registers.
__global__ __launch_bounds__(256) void block3_max_kernel(const float* __restrict__ src, int W, int H,
                                                         float* __restrict__ dst) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y0 = blockIdx.y * 8;
  if (x >= W) return;
  const int xl = max(x - 1, 0), xr = min(x + 1, W - 1);
  auto row_max = [&](int y) {
    const float* p = src + (size_t)y * W;
    return fmaxf(fmaxf(p[xl], p[x]), p[xr]);
  };
  float a = row_max(max(y0 - 1, 0));
  float b = row_max(y0);
  for (int k = 0; k < 8; ++k) {
    const int y = y0 + k;
    if (y >= H) break;
    const float c = row_max(min(y + 1, H - 1));
    dst[(size_t)y * W + x] = canon(fmaxf(fmaxf(a, b), c));
    a = b;
    b = c;
  }
}

hipError_t launch_block3_max(const float* src, int W, int H, float* dst, hipStream_t stream) {
  if (W <= 0 || H <= 0) return hipSuccess;
  dim3 grid((W + 255) / 256, (H + 7) / 8), block(256);
  hipLaunchKernelGGL(block3_max_kernel, grid, block, 0, stream, src, W, H, dst);
  return hipGetLastError();
}

hipError_t launch_maxmip(const float* src, int sw, int sh, float* dst_base, const int* dst_off,
                         const int* dst_w, const int* dst_h, int F, hipStream_t stream) {
  MipDst d;
  for (int k = 0; k < 6; ++k) {
    d.off[k] = k < F ? dst_off[k] : 0;
    d.w[k] = k < F ? dst_w[k] : 0;
    d.h[k] = k < F ? dst_h[k] : 0;
  }
  const int nbx = (sw + 63) / 64, nby = (sh + 63) / 64;
  const int nb = nbx * nby;
  if (nb == 0) return hipSuccess;
  const int vec_ok = ((reinterpret_cast<uintptr_t>(src) & 15) == 0) && (sw % 4 == 0);
  dim3 grid(nb), block(256);
  switch (F) {
    case 1: hipLaunchKernelGGL(maxmip_kernel<1>, grid, block, 0, stream, src, sw, sh, dst_base, d, nbx, vec_ok); break;
    case 2: hipLaunchKernelGGL(maxmip_kernel<2>, grid, block, 0, stream, src, sw, sh, dst_base, d, nbx, vec_ok); break;
    case 3: hipLaunchKernelGGL(maxmip_kernel<3>, grid, block, 0, stream, src, sw, sh, dst_base, d, nbx, vec_ok); break;
    case 4: hipLaunchKernelGGL(maxmip_kernel<4>, grid, block, 0, stream, src, sw, sh, dst_base, d, nbx, vec_ok); break;
    case 5: hipLaunchKernelGGL(maxmip_kernel<5>, grid, block, 0, stream, src, sw, sh, dst_base, d, nbx, vec_ok); break;
    default: hipLaunchKernelGGL(maxmip_kernel<6>, grid, block, 0, stream, src, sw, sh, dst_base, d, nbx, vec_ok); break;
  }
  return hipGetLastError();
}

}  // namespace ss
