// The batched call: many suns over tiles of uneven size in one launch, as a
// flat grid over every ray block of every (tile, sun) pair (flat_kernel, the
// default) or a persistent kernel with per-XCD queues (batched_kernel); and
// the staging of the batch's per-pair set-up into the workspace through kernel
// arguments (stage_kernel, expand_kernel), so the call needs no host buffer,
// no copy and no wait.
//
// Persistent form:
// Items are groups of ray blocks of a (tile, sun) pair.  Each pair's items are
// split into SS_NXCD contiguous row bands, and XCD x has its own queue: band x
// of every pair, pairs in tile-major, sun-minor order.  A workgroup takes the
// next item of its XCD's queue (one atomic per item, issued by one lane and
// broadcast through LDS), so an XCD's rays stay in its bands and reuse its L2,
// as the per-tile kernel's workgroup remap does; when that queue is empty it
// takes items from the other queues in turn, so the launch still ends with one
// tail, and after every queue has run dry once it exits.  The next item is
// claimed while the current one is worked, so no wave waits on the atomic.  Per-(tile, sun)
// parameter blocks live in the workspace; the item index is wave-uniform, so
// they are read with scalar loads.  Each ray runs the same device code as the
// per-tile kernel, so the outputs are bit-identical to it.
#include <stddef.h>
#include <string.h>

#include "kernels.h"
#include "ray.h"

namespace ss {

// Last pair p with row[p] <= q (row: n_pairs + 1 non-decreasing prefix sums).
__device__ __forceinline__ int pair_of(const long long* __restrict__ row, int n_pairs, long long q) {
  int lo = 0, hi = n_pairs;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (row[mid] <= q) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Thread 0's claim of the next item: q (>= 0 when an index was already taken
// from queue (xcd + tried) % SS_NXCD) is resolved to a pair and item; an empty
// queue moves on to the next one.  Returns pair -1 once every queue has run dry.
__device__ __forceinline__ int resolve_claim(const long long* __restrict__ item_start,
                                             const long long* __restrict__ xstart,
                                             unsigned int* __restrict__ counter, int n_pairs,
                                             int xcd, int& tried, long long q, long long& item) {
  while (tried < SS_NXCD) {
    const int x = (xcd + tried) % SS_NXCD;
    const long long* row = xstart + (size_t)x * (n_pairs + 1);
    if (q < 0) q = (long long)atomicAdd(&counter[x], 1u);
    if (q < row[n_pairs]) {
      const int pr = pair_of(row, n_pairs, q);
      const long long n = item_start[pr + 1] - item_start[pr];
      item = item_start[pr] + (long long)x * n / SS_NXCD + (q - row[pr]);
      return pr;
    }
    q = -1;
    ++tried;  // a queue only grows emptier
  }
  return -1;
}

// Occupancy: the stepping modes are held to 8 wavefronts per SIMD (at most 64
// VGPRs; the compiler spills a dword or two, outside the per-run loops), 5%
// faster on the 4096^2 x 8-sun workload than the 7 their free allocation
// gives; the exact mode to 7 (72 VGPRs, no spill), 6% faster than its free 6
// and than 8 (which spills inside the walk).
template <bool SPHERE, int TW, int MODE>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256),
                          amdgpu_waves_per_eu(MODE == SS_MODE_EXACT ? 7 : 8))) void batched_kernel(const TileK* __restrict__ pairs,
                                                      float* const* __restrict__ outs,
                                                      const long long* __restrict__ item_start,
                                                      const long long* __restrict__ xstart,
                                                      const int* __restrict__ pair_nbx,
                                                      unsigned int* __restrict__ counter,
                                                      int n_pairs) {
  constexpr int TH = 64 / TW;
  // two slots: the item being worked and the next one; the next claim's index
  // and the queue search state live here too, so nothing extra stays in
  // registers across the rays
  __shared__ int s_pair[2];
  __shared__ long long s_item[2];
  __shared__ long long s_q;
  __shared__ int s_tried;
  __shared__ int tab[SS_MAXLEV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int xcd = (int)(blockIdx.x % SS_NXCD);
  if (threadIdx.x == 0) {
    int tried = 0;
    long long it = 0;
    s_pair[0] = resolve_claim(item_start, xstart, counter, n_pairs, xcd, tried, -1, it);
    s_item[0] = it;
    s_tried = tried;
  }
  __syncthreads();
  for (int buf = 0;; buf ^= 1) {
    const int pair = __builtin_amdgcn_readfirstlane(s_pair[buf]);
    if (pair < 0) break;  // the same slot for every thread
    const long long item = s_item[buf];
    // claim the next item now; only wave 0 waits for the atomic, the others
    // go on with their rays
    if (threadIdx.x == 0) {
      const int tried = s_tried;
      s_q = tried < SS_NXCD ? (long long)atomicAdd(&counter[(xcd + tried) % SS_NXCD], 1u) : -1;
    }
    if (MODE == SS_MODE_EXACT) {
      // every thread finished the previous item at the barrier ending it
      bound_tab_fill(pairs[pair], tab);
      __syncthreads();
    }
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
    if (threadIdx.x == 0) {
      int tried = s_tried;
      long long it = 0;
      s_pair[buf ^ 1] = resolve_claim(item_start, xstart, counter, n_pairs, xcd, tried, s_q, it);
      s_item[buf ^ 1] = it;
      s_tried = tried;
    }
    __syncthreads();
  }
}

// Flat form: one workgroup per ray block of every pair (grid = all blocks),
// ids remapped as the per-tile kernels remap theirs (groups of one device-full,
// TileK.wg_group, a run per XCD inside each); the pair comes from the block
// prefix sums.  No queue: the hardware deals the workgroups, and the batch
// still ends with one tail.
static_assert(SS_ITEM_BLOCKS == 1, "the flat form reads the item prefix sums as block prefix sums");

template <bool SPHERE, int TW, int MODE>
__global__ __launch_bounds__(256) void flat_kernel(const TileK* __restrict__ pairs,
                                                   float* const* __restrict__ outs,
                                                   const long long* __restrict__ block_start,
                                                   const int* __restrict__ pair_nbx, int n_pairs,
                                                   int n_blocks, int grp) {
  constexpr int TH = 64 / TW;
  __shared__ int tab[SS_MAXLEV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long blk_all = xcd_remap_grouped((int)blockIdx.x, n_blocks, grp);
  const int pair = __builtin_amdgcn_readfirstlane(pair_of(block_start, n_pairs, blk_all));
  const TileK& T = pairs[pair];
  if (MODE == SS_MODE_EXACT) {
    bound_tab_fill(T, tab);
    __syncthreads();
  }
  const int nbx = pair_nbx[pair];
  const long long blk = blk_all - block_start[pair];
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
    outs[pair][lj * T.RW + li] = disc_fraction(alpha, T);
  }
}

template <bool SPHERE, int MODE>
static hipError_t launch_flat_m(const TileK* a, float* const* b, const long long* c, const int* d,
                                int n_pairs, int n_blocks, int grp, int ray_tile, hipStream_t s) {
  const dim3 g((unsigned)n_blocks), t(256);
  switch (ray_tile) {
    case SS_TILE_16x4:
      hipLaunchKernelGGL((flat_kernel<SPHERE, 16, MODE>), g, t, 0, s, a, b, c, d, n_pairs, n_blocks, grp);
      break;
    case SS_TILE_4x16:
      hipLaunchKernelGGL((flat_kernel<SPHERE, 4, MODE>), g, t, 0, s, a, b, c, d, n_pairs, n_blocks, grp);
      break;
    case SS_TILE_32x2:
      hipLaunchKernelGGL((flat_kernel<SPHERE, 32, MODE>), g, t, 0, s, a, b, c, d, n_pairs, n_blocks, grp);
      break;
    default:
      hipLaunchKernelGGL((flat_kernel<SPHERE, 8, MODE>), g, t, 0, s, a, b, c, d, n_pairs, n_blocks, grp);
      break;
  }
  return hipGetLastError();
}

template <bool SPHERE>
static hipError_t launch_flat_s(const TileK* a, float* const* b, const long long* c, const int* d,
                                int n_pairs, int n_blocks, int grp, int mode, int ray_tile,
                                hipStream_t s) {
  switch (mode) {
    case SS_MODE_UNIFORM: return launch_flat_m<SPHERE, SS_MODE_UNIFORM>(a, b, c, d, n_pairs, n_blocks, grp, ray_tile, s);
    case SS_MODE_POINT: return launch_flat_m<SPHERE, SS_MODE_POINT>(a, b, c, d, n_pairs, n_blocks, grp, ray_tile, s);
    case SS_MODE_EXACT: return launch_flat_m<SPHERE, SS_MODE_EXACT>(a, b, c, d, n_pairs, n_blocks, grp, ray_tile, s);
    default: return launch_flat_m<SPHERE, SS_MODE_DP>(a, b, c, d, n_pairs, n_blocks, grp, ray_tile, s);
  }
}

hipError_t launch_batched_flat(const TileK* d_pairs, float* const* d_out_ptrs,
                               const long long* d_block_start, const int* d_pair_nbx,
                               const BatchDesc& bd, int grp, bool sphere, int mode, int ray_tile,
                               hipStream_t stream) {
  if (bd.total_items <= 0) return hipSuccess;
  const int nb = (int)bd.total_items;
  if (sphere)
    return launch_flat_s<true>(d_pairs, d_out_ptrs, d_block_start, d_pair_nbx, bd.n_pairs, nb,
                               grp, mode, ray_tile, stream);
  return launch_flat_s<false>(d_pairs, d_out_ptrs, d_block_start, d_pair_nbx, bd.n_pairs, nb, grp,
                              mode, ray_tile, stream);
}

__global__ void fill_u32_kernel(unsigned int* p, unsigned int v, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

hipError_t launch_fill_u32(unsigned int* p, unsigned int v, int n, hipStream_t stream) {
  hipLaunchKernelGGL(fill_u32_kernel, dim3((n + 63) / 64), dim3(64), 0, stream, p, v, n);
  return hipGetLastError();
}

// ---- staging of the batch tables through kernel arguments ----

#define SS_STAGE_WORDS 500
struct StageChunk {
  unsigned n;
  unsigned w[SS_STAGE_WORDS];
};

__global__ __launch_bounds__(256) void stage_kernel(unsigned* __restrict__ dst, StageChunk c) {
  for (unsigned k = threadIdx.x; k < c.n; k += 256) dst[k] = c.w[k];
}

hipError_t launch_stage(void* d_dst, const void* h_src, size_t bytes, hipStream_t stream) {
  const unsigned* src = static_cast<const unsigned*>(h_src);
  unsigned* dst = static_cast<unsigned*>(d_dst);
  const size_t words = bytes / 4;
  StageChunk c = {};
  for (size_t k = 0; k < words; k += SS_STAGE_WORDS) {
    c.n = (unsigned)(words - k < SS_STAGE_WORDS ? words - k : SS_STAGE_WORDS);
    memcpy(c.w, src + k, c.n * sizeof(unsigned));
    hipLaunchKernelGGL(stage_kernel, dim3(1), dim3(256), 0, stream, dst + k, c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One wavefront per pair: the TileK words come from the tile's template except
// the sun fields (from the pair's record) and the run starts (formed from the
// template's grid indices and the pair's delta/2, as the host set-up forms them).
static_assert(offsetof(TileK, ucap) == offsetof(TileK, Lx) + 11 * sizeof(float),
              "the sun fields of TileK are contiguous");
static_assert(sizeof(TileK) % 4 == 0, "TileK is copied by words");

__global__ __launch_bounds__(64) void expand_kernel(const TileK* __restrict__ tmpl,
                                                    const StageTile* __restrict__ st,
                                                    const StagePair* __restrict__ sp, int n_tiles,
                                                    int n_suns, TileK* __restrict__ pairs,
                                                    float** __restrict__ outs,
                                                    long long* __restrict__ start,
                                                    long long* __restrict__ xstart,
                                                    int* __restrict__ nbx) {
  constexpr int NW = (int)(sizeof(TileK) / 4);
  constexpr int W_SUN = (int)(offsetof(TileK, Lx) / 4);
  constexpr int W_TAU = (int)(offsetof(TileK, tau) / 4);
  const int p = blockIdx.x;
  const int t = p / n_suns, k = p % n_suns;
  const int n_pairs = n_tiles * n_suns;
  const TileK& T = tmpl[t];
  const StagePair& P = sp[p];
  const unsigned* src = reinterpret_cast<const unsigned*>(&T);
  unsigned* dst = reinterpret_cast<unsigned*>(&pairs[p]);
  const int nseg = T.nseg;
  for (int w = threadIdx.x; w < NW; w += 64) {
    unsigned v = src[w];
    if (w >= W_SUN && w < W_SUN + 12) {
      v = __float_as_uint(P.sun[w - W_SUN]);
    } else if (w >= W_TAU && w <= W_TAU + nseg) {
      const int j = w - W_TAU;
      const int a = j < nseg ? T.a0[j] : T.a0[nseg - 1] + (2 << T.m0[nseg - 1]);
      v = __float_as_uint(run_start_len(a, P.half_delta));
    }
    dst[w] = v;
  }
  const long long items = st[t].items;
  if (threadIdx.x == 0) {
    outs[p] = P.out;
    start[p] = st[t].start + (long long)k * items;
    nbx[p] = st[t].nbx;
    if (p == n_pairs - 1) start[n_pairs] = st[n_tiles].start;
  }
  if (xstart && threadIdx.x < SS_NXCD) {
    const int x = threadIdx.x;
    const long long band = (long long)(x + 1) * items / SS_NXCD - (long long)x * items / SS_NXCD;
    long long* row = xstart + (size_t)x * (n_pairs + 1);
    row[p] = st[t].xt[x] + (long long)k * band;
    if (p == n_pairs - 1) row[n_pairs] = st[n_tiles].xt[x];
  }
}

hipError_t launch_expand(const TileK* tmpl, const StageTile* st, const StagePair* sp, int n_tiles,
                         int n_suns, TileK* pairs, float** outs, long long* start,
                         long long* xstart, int* nbx, hipStream_t stream) {
  const long long np = (long long)n_tiles * n_suns;
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(expand_kernel, dim3((unsigned)np), dim3(64), 0, stream, tmpl, st, sp, n_tiles,
                     n_suns, pairs, outs, start, xstart, nbx);
  return hipGetLastError();
}

template <bool SPHERE, int TW, int MODE>
static hipError_t launch_b(const TileK* d_pairs, float* const* d_out, const long long* d_start,
                           const long long* d_xs, const int* d_nbx, unsigned int* d_counter,
                           const BatchDesc& bd, int n_wg, hipStream_t stream) {
  hipLaunchKernelGGL((batched_kernel<SPHERE, TW, MODE>), dim3(n_wg), dim3(256), 0, stream, d_pairs,
                     d_out, d_start, d_xs, d_nbx, d_counter, bd.n_pairs);
  return hipGetLastError();
}

template <bool SPHERE, int MODE>
static hipError_t launch_bm(const TileK* a, float* const* b, const long long* c,
                            const long long* x, const int* d, unsigned int* e, const BatchDesc& bd,
                            int ray_tile, int n_wg, hipStream_t s) {
  switch (ray_tile) {
    case SS_TILE_16x4: return launch_b<SPHERE, 16, MODE>(a, b, c, x, d, e, bd, n_wg, s);
    case SS_TILE_4x16: return launch_b<SPHERE, 4, MODE>(a, b, c, x, d, e, bd, n_wg, s);
    case SS_TILE_32x2: return launch_b<SPHERE, 32, MODE>(a, b, c, x, d, e, bd, n_wg, s);
    default: return launch_b<SPHERE, 8, MODE>(a, b, c, x, d, e, bd, n_wg, s);
  }
}

template <bool SPHERE>
static hipError_t launch_bs(const TileK* a, float* const* b, const long long* c,
                            const long long* x, const int* d, unsigned int* e, const BatchDesc& bd,
                            int mode, int ray_tile, int n_wg, hipStream_t s) {
  switch (mode) {
    case SS_MODE_UNIFORM: return launch_bm<SPHERE, SS_MODE_UNIFORM>(a, b, c, x, d, e, bd, ray_tile, n_wg, s);
    case SS_MODE_POINT: return launch_bm<SPHERE, SS_MODE_POINT>(a, b, c, x, d, e, bd, ray_tile, n_wg, s);
    case SS_MODE_EXACT: return launch_bm<SPHERE, SS_MODE_EXACT>(a, b, c, x, d, e, bd, ray_tile, n_wg, s);
    default: return launch_bm<SPHERE, SS_MODE_DP>(a, b, c, x, d, e, bd, ray_tile, n_wg, s);
  }
}

hipError_t launch_batched(const TileK* d_pairs, float* const* d_out_ptrs, const long long* d_item_start,
                          const long long* d_xstart, const int* d_pair_nbx, unsigned int* d_counter,
                          const BatchDesc& bd, bool sphere, int mode, int ray_tile, int n_workgroups,
                          hipStream_t stream) {
  if (bd.total_items <= 0 || n_workgroups <= 0) return hipSuccess;
  if (sphere)
    return launch_bs<true>(d_pairs, d_out_ptrs, d_item_start, d_xstart, d_pair_nbx, d_counter, bd,
                           mode, ray_tile, n_workgroups, stream);
  return launch_bs<false>(d_pairs, d_out_ptrs, d_item_start, d_xstart, d_pair_nbx, d_counter, bd,
                          mode, ray_tile, n_workgroups, stream);
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
