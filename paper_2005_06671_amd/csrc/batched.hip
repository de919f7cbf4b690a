// Persistent batched kernel: many suns over tiles of uneven size in one launch.
//
// Items are (tile, sun, group of ray blocks) in tile-major, sun-minor order;
// a workgroup takes the next item from a device counter (one atomic per item,
// issued by one lane and broadcast through LDS) until the queue is empty, so
// every workgroup reaches the exit.  Per-(tile, sun) parameter blocks live in
// the workspace; the item index is wave-uniform, so they are read with scalar
// loads.  Each ray runs the same device code as the per-tile kernel, so the
// outputs are bit-identical to it.
#include "kernels.h"
#include "ray.h"

namespace ss {

__device__ __forceinline__ int pair_of(const long long* __restrict__ start, int n_pairs, long long item) {
  int lo = 0, hi = n_pairs;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= item) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <bool SPHERE, int TW, int MODE>
__global__ __launch_bounds__(256) void batched_kernel(const TileK* __restrict__ pairs,
                                                      float* const* __restrict__ outs,
                                                      const long long* __restrict__ item_start,
                                                      const int* __restrict__ pair_nbx,
                                                      unsigned int* __restrict__ counter,
                                                      long long item_limit, int n_pairs) {
  constexpr int TH = 64 / TW;
  __shared__ unsigned int s_item;
  __shared__ int tab[SS_MAXLEV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
    __syncthreads();
    const long long item = (long long)s_item;
    // every thread is past the previous item here, so the table can be refilled
    const int pair = item < item_limit
                         ? __builtin_amdgcn_readfirstlane(pair_of(item_start, n_pairs, item))
                         : 0;
    if (MODE == SS_MODE_EXACT && item < item_limit) bound_tab_fill(pairs[pair], tab);
    __syncthreads();
    if (item >= item_limit) break;
    const TileK& T = pairs[pair];
    float* out = outs[pair];
    const int nbx = pair_nbx[pair];
    const long long first = (item - item_start[pair]) * SS_ITEM_BLOCKS;
    const long long nblk = (long long)nbx * ((T.RH + 2 * TH - 1) / (2 * TH));
    for (int g = 0; g < SS_ITEM_BLOCKS; ++g) {
      const long long blk = first + g;
      if (blk >= nblk) break;
      const int bxi = (int)(blk % nbx), byi = (int)(blk / nbx);
      const int li = bxi * (2 * TW) + (wave & 1) * TW + lane % TW;
      const int lj = byi * (2 * TH) + (wave >> 1) * TH + lane / TW;
      if (li < T.RW && lj < T.RH) {
        const int i = T.rx0 + li, j = T.ry0 + lj;
        const float hp = T.h[j * T.W + i];
        Ray<SPHERE> r;
        ray_init(T, i, j, hp, r);
        unsigned n_lb = 0, n_smp = 0;
        const float alpha = trace_ray<SPHERE, MODE>(T, r, n_lb, n_smp, tab).alpha;
        out[lj * T.RW + li] = disc_fraction(alpha, T);
      }
    }
  }
}

__global__ void fill_u32_kernel(unsigned int* p, unsigned int v, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

hipError_t launch_fill_u32(unsigned int* p, unsigned int v, int n, hipStream_t stream) {
  hipLaunchKernelGGL(fill_u32_kernel, dim3((n + 63) / 64), dim3(64), 0, stream, p, v, n);
  return hipGetLastError();
}

template <bool SPHERE, int TW, int MODE>
static hipError_t launch_b(const TileK* d_pairs, float* const* d_out, const long long* d_start,
                           const int* d_nbx, unsigned int* d_counter, const BatchDesc& bd,
                           int n_wg, hipStream_t stream) {
  hipLaunchKernelGGL((batched_kernel<SPHERE, TW, MODE>), dim3(n_wg), dim3(256), 0, stream, d_pairs,
                     d_out, d_start, d_nbx, d_counter, bd.item_limit, bd.n_pairs);
  return hipGetLastError();
}

template <bool SPHERE, int MODE>
static hipError_t launch_bm(const TileK* a, float* const* b, const long long* c, const int* d,
                            unsigned int* e, const BatchDesc& bd, int ray_tile, int n_wg,
                            hipStream_t s) {
  switch (ray_tile) {
    case SS_TILE_16x4: return launch_b<SPHERE, 16, MODE>(a, b, c, d, e, bd, n_wg, s);
    case SS_TILE_4x16: return launch_b<SPHERE, 4, MODE>(a, b, c, d, e, bd, n_wg, s);
    case SS_TILE_32x2: return launch_b<SPHERE, 32, MODE>(a, b, c, d, e, bd, n_wg, s);
    default: return launch_b<SPHERE, 8, MODE>(a, b, c, d, e, bd, n_wg, s);
  }
}

template <bool SPHERE>
static hipError_t launch_bs(const TileK* a, float* const* b, const long long* c, const int* d,
                            unsigned int* e, const BatchDesc& bd, int mode, int ray_tile, int n_wg,
                            hipStream_t s) {
  switch (mode) {
    case SS_MODE_UNIFORM: return launch_bm<SPHERE, SS_MODE_UNIFORM>(a, b, c, d, e, bd, ray_tile, n_wg, s);
    case SS_MODE_POINT: return launch_bm<SPHERE, SS_MODE_POINT>(a, b, c, d, e, bd, ray_tile, n_wg, s);
    case SS_MODE_EXACT: return launch_bm<SPHERE, SS_MODE_EXACT>(a, b, c, d, e, bd, ray_tile, n_wg, s);
    default: return launch_bm<SPHERE, SS_MODE_DP>(a, b, c, d, e, bd, ray_tile, n_wg, s);
  }
}

hipError_t launch_batched(const TileK* d_pairs, float* const* d_out_ptrs, const long long* d_item_start,
                          const int* d_pair_nbx, unsigned int* d_counter, const BatchDesc& bd,
                          bool sphere, int mode, int ray_tile, int n_workgroups, hipStream_t stream) {
  if (bd.item_limit <= 0 || n_workgroups <= 0) return hipSuccess;
  if (sphere)
    return launch_bs<true>(d_pairs, d_out_ptrs, d_item_start, d_pair_nbx, d_counter, bd, mode,
                           ray_tile, n_workgroups, stream);
  return launch_bs<false>(d_pairs, d_out_ptrs, d_item_start, d_pair_nbx, d_counter, bd, mode,
                          ray_tile, n_workgroups, stream);
}

template <bool SPHERE, int MODE>
static const void* kernel_of(int tw) {
  switch (tw) {
    case 16: return reinterpret_cast<const void*>(&batched_kernel<SPHERE, 16, MODE>);
    case 4: return reinterpret_cast<const void*>(&batched_kernel<SPHERE, 4, MODE>);
    case 32: return reinterpret_cast<const void*>(&batched_kernel<SPHERE, 32, MODE>);
    default: return reinterpret_cast<const void*>(&batched_kernel<SPHERE, 8, MODE>);
  }
}

template <bool SPHERE>
static const void* kernel_of_mode(int mode, int tw) {
  switch (mode) {
    case SS_MODE_UNIFORM: return kernel_of<SPHERE, SS_MODE_UNIFORM>(tw);
    case SS_MODE_POINT: return kernel_of<SPHERE, SS_MODE_POINT>(tw);
    case SS_MODE_EXACT: return kernel_of<SPHERE, SS_MODE_EXACT>(tw);
    default: return kernel_of<SPHERE, SS_MODE_DP>(tw);
  }
}

// Workgroups that fit on the device at once for the chosen variant.
int batched_workgroups(bool sphere, int mode, int ray_tile) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const int tw = ray_tile == SS_TILE_16x4 ? 16 : ray_tile == SS_TILE_4x16 ? 4 : ray_tile == SS_TILE_32x2 ? 32 : 8;
  const void* fn = sphere ? kernel_of_mode<true>(mode, tw) : kernel_of_mode<false>(mode, tw);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, 0) != hipSuccess || per < 1) per = 1;
  return ncu * per;
}

}  // namespace ss
