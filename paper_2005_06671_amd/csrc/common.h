// Parameter block shared by the host set-up and the gfx950 kernels.
//
// The host forms every per-(tile, sun) quantity in FP64 and rounds it once to
// FP32 here; the kernels work in FP32 relative to each ray's origin.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define SS_MAXLEV 18   // supports max(width, rows) <= 65536
#define SS_MAXSEG 48   // concatenated runs per ray

struct TileK {
  const float* h;            // level 0: the heightfield, [H][W]
  const float* mm;           // levels >= 1, packed at loff[m]
  const float* bnd;          // tap-bound pyramid level 0, [H][W] (exact mode only)
  const float* bmm;          // its levels >= 1, packed at loff[m] like mm
  int W, H, L;               // size and number of mip levels (incl. level 0)
  int rx0, ry0, RW, RH;      // ray window: origins (rx0 + x, ry0 + y), x < RW, y < RH
  int lw[SS_MAXLEV], lh[SS_MAXLEV];
  int loff[SS_MAXLEV];       // float offset of level m >= 1 inside mm
  float texel;               // texel spacing on the tangent plane (m)
  float invR;                // 1 / body radius (0 on the plane)
  float Lx, Ly, Lz;          // unit vector toward the sun centre, tile frame
  float half_delta;          // delta/2, delta = texel / cos(elev): first sample and grid step
  float two_over_delta;      // 2 / delta
  float rL, inv_rL;          // sun disc angular radius and its inverse
  float prune_margin;        // safety margin (rad) of the result-invariant exits
  float tan_rL;              // tan(r_L)
  float tan_margin;          // tan(prune_margin)
  float ustep;               // uniform stepping: step in ray length (m)
  float ucap;                // uniform stepping: cap on ray length (m), +inf = tile edge
  int nseg;                  // number of concatenated runs
  int m0[SS_MAXSEG];         // top mip level of run j
  float tau[SS_MAXSEG + 1];  // ray length where run j starts (tau[nseg] = end)
  int a0[SS_MAXSEG];         // grid index of run j's start: tau_j = (a0_j + 1) delta/2
  int prune;                 // 1: result-invariant early exits enabled
  int wg_group;              // per-tile kernels: workgroup ids are remapped within groups of
                             // this many (one device-full, a multiple of 8)
};

// Ray length where the run starting at half-texel grid index a begins:
// tau = (a + 1) delta/2, one FP64 product rounded once to FP32.  The per-tile
// set-up on the host and the batched call's expand kernel on the device both
// form it this way, so their parameter blocks agree bit for bit.
__host__ __device__ inline float run_start_len(int a, double half_delta) {
  return (float)((double)(a + 1) * half_delta);
}

// Ray tile shapes: lanes of one wavefront cover TW x TH texels (TW * TH = 64),
// a 256-thread workgroup covers 2 x 2 wavefront tiles.
enum { SS_TILE_8x8 = 1, SS_TILE_16x4 = 2, SS_TILE_4x16 = 3, SS_TILE_32x2 = 4 };
