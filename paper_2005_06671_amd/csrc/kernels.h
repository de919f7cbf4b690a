// Host-side launchers of the gfx950 kernels (internal to libsoftshadow).
#pragma once

#include "../../include/softshadow.h"
#include "common.h"

namespace ss {

#define SS_ITEM_BLOCKS 1  // ray blocks (256 rays each) per queue item of the batched kernel
#define SS_NXCD 8         // XCDs; workgroup ids are dealt round-robin over them

// Maximum mipmap: levels [m_src+1, m_src+F] from level m_src (F <= 6).
hipError_t launch_maxmip(const float* src, int sw, int sh, float* dst_base, const int* dst_off,
                         const int* dst_w, const int* dst_h, int F, hipStream_t stream);

// Tap-bound pyramid level 0: maximum over each texel's 3 x 3 block (clipped).
hipError_t launch_block3_max(const float* src, int W, int H, float* dst, hipStream_t stream);

void grid_for(const TileK& T, int ray_tile, int* nbx, int* nblocks);

// sample != nullptr (and !count): also record each ray's deciding sample index.
hipError_t launch_forward(const TileK& T, bool sphere, int mode, int ray_tile, bool count,
                          float* out, unsigned long long* counter, int* sample,
                          hipStream_t stream);

// Shadow rays from n surface points (float2 continuous texel coordinates);
// img_w > 0: the points are an image of img_w columns, shaded in pixel tiles.
hipError_t launch_points(const TileK& T, bool sphere, int mode, const float* xy, long long n,
                         int img_w, float* out, hipStream_t stream);

// Adjoint of launch_points (points held fixed), same work mapping.
hipError_t launch_points_adjoint(const TileK& T, bool sphere, int mode, double elev, double azim,
                                 const float* xy, long long n, int img_w, const float* gs,
                                 float* gh, double* gsun, hipStream_t stream);

// sample != nullptr: take the deciding samples from there instead of replaying.
// sfwd != nullptr: the forward's shadow factors; rays at 0 or 1 are skipped.
hipError_t launch_adjoint(const TileK& T, bool sphere, int mode, double elev, double azim,
                          const float* gs, const int* sample, const float* sfwd, float* gh,
                          double* gsun, hipStream_t stream);

// Persistent batched launch over (tile, sun, ray block) items.
struct BatchDesc {
  int n_pairs;            // tiles * suns
  int n_tiles, n_suns;
  long long total_items;  // sum over pairs of their items (groups of SS_ITEM_BLOCKS ray blocks)
};
// d_xstart: SS_NXCD rows of n_pairs + 1 prefix sums, row x = the items of band x of
// each pair (band x of a pair: its items [x n / SS_NXCD, (x + 1) n / SS_NXCD));
// d_counter: SS_NXCD queue counters, zero at launch.
hipError_t launch_batched(const TileK* d_pairs, float* const* d_out_ptrs, const long long* d_item_start,
                          const long long* d_xstart, const int* d_pair_nbx, unsigned int* d_counter,
                          const BatchDesc& bd, bool sphere, int mode, int ray_tile, int n_workgroups,
                          hipStream_t stream);
// Flat form of the batched call: one workgroup per ray block of every pair
// (n blocks = bd.total_items with one block per item, below 2^31).
hipError_t launch_batched_flat(const TileK* d_pairs, float* const* d_out_ptrs,
                               const long long* d_block_start, const int* d_pair_nbx,
                               const BatchDesc& bd, int grp, bool sphere, int mode, int ray_tile,
                               hipStream_t stream);
hipError_t launch_fill_u32(unsigned int* p, unsigned int v, int n, hipStream_t stream);

// Compact image of a batch, formed on the host (FP64 set-up) and staged into
// the workspace through kernel arguments (no host buffer outlives the call, no
// host wait, capturable); the expand kernel turns it into the per-pair
// parameter blocks and tables the batched kernels read.
struct StageTile {        // n_tiles + 1 entries; the last holds the totals
  long long items;        // ray blocks of each (tile, sun) pair of this tile
  long long start;        // block index of the tile's first pair
  long long xt[SS_NXCD];  // queue x's index of the tile's first pair (persistent form)
  int nbx, pad;           // ray-block grid width
};
struct StagePair {        // one per (tile, sun) pair, tile-major
  float sun[12];          // the TileK fields Lx .. ucap of this pair
  double half_delta;      // delta/2 in FP64; run starts are run_start_len(a0_j, half_delta)
  float* out;             // its output buffer
};
static_assert(sizeof(StageTile) % 4 == 0 && sizeof(StagePair) % 8 == 0, "word-staged records");
// Copies `bytes` (a multiple of 4) from host memory into device memory by
// kernel arguments, in chunks of about 2 KB.
hipError_t launch_stage(void* d_dst, const void* h_src, size_t bytes, hipStream_t stream);
// pairs[p] = the tile's template with the pair's sun fields and run starts;
// outs, block starts, grid widths and (xstart != nullptr) the per-queue prefix
// sums of every pair, with their totals in entry n_pairs.
hipError_t launch_expand(const TileK* tmpl, const StageTile* st, const StagePair* sp, int n_tiles,
                         int n_suns, TileK* pairs, float** outs, long long* start,
                         long long* xstart, int* nbx, hipStream_t stream);
int batched_workgroups(bool sphere, int mode, int ray_tile);

// View rays (pinhole camera) onto the terrain; the host fills every field.
struct ViewK {
  const float* h;            // heightfield [H][W]
  const float* bnd;          // tap-bound pyramid level 0, [H][W]
  const float* bmm;          // its levels >= 1 at loff[m]
  int W, H, L;
  int lw[SS_MAXLEV], lh[SS_MAXLEV], loff[SS_MAXLEV];
  float inv_pow2[SS_MAXLEV]; // 2^-m
  float texel, invT;         // texel spacing and its inverse
  float R, invR;             // body radius and its inverse (0 on the plane)
  float cx0, cy0;            // W/2, H/2: texel coordinates of the tile centre
  float ex, ey, ez;          // eye, relative to the tile-centre surface point
  float fx, fy, fz, rx, ry, rz, ux, uy, uz;  // pixel ray: f + sx r + sy u
  int img_w, img_h, nbx, nby;
  float inv_w2, inv_h2;      // 2 / img_w, 2 / img_h
  float step, inv_step;      // grid spacing along the ray (m) and its inverse
  float far;                 // last counting ray length (+inf: none)
  float m_abs, m_rel;        // skip margin m_abs + m_rel (|eye| + t), metres
  int max_iter;              // walk iterations per ray (a bound never reached)
  int max_samples;           // samples per ray (a bound never reached)
};
hipError_t launch_view(const ViewK& K, bool sphere, int mode, float* t, float* xy, int* steps,
                       hipStream_t stream);

// Resampling between gnomonic tile frames (FP64 definition, rounded once).
struct ResampleK {
  const float* src;
  float* dst;
  int Ws, Hs, Wd, Hd;
  double R;
  double cd[3], exd[3], eyd[3], oxd, oyd, Dd;  // destination frame
  double cs[3], exs[3], eys[3], oxs, oys, Ds;  // source frame
};
hipError_t launch_resample(const ResampleK& K, hipStream_t stream);

// Gather throughput probe (measurement only).
hipError_t launch_gather_probe(const float* src, long long n_floats, long long window, int iters,
                               float* out, long long n_threads, hipStream_t stream);
hipError_t launch_gather_tiles_probe(const float* src, int width, int rows, int iters, float* out,
                                     long long n_threads, hipStream_t stream);
hipError_t launch_valu_probe(int iters, long long n_workgroups, float* out, hipStream_t stream);

}  // namespace ss
