// Device helpers: trilinear sampling, finite differences, block reductions.
#pragma once

#include "internal.h"

namespace lddmm {

// Index of voxel (x, y, z) on grid g (every grid has fewer than 2^31 voxels).
__device__ __forceinline__ uint32_t vidx(const Geom& g, int x, int y, int z) {
  return (uint32_t)((z * g.ny + y) * g.nx + x);
}

// Voxel coordinates of linear index i (magic-number division, no hardware divide).
__device__ __forceinline__ void vcoord(const Geom& g, uint32_t i, int& x, int& y, int& z) {
  const uint32_t t = fdiv(i, g.fx);
  const uint32_t zz = fdiv(t, g.fy);
  x = (int)(i - t * (uint32_t)g.nx);
  y = (int)(t - zz * (uint32_t)g.ny);
  z = (int)zz;
}

// ------------------------------------------------------------ buffer access --
// Raw buffer loads/stores address a field through a scalar descriptor and a
// 32-bit byte offset, so no per-lane 64-bit address arithmetic is needed.  An
// offset at or beyond the field's size reads as 0 (and a store there is
// dropped), which gives zero-outside sampling without branches.  Every field
// has fewer than 2^30 voxels, so byte offsets fit in 32 bits.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr uint32_t kOutside = 0x3FFFFFFFu;   // element index that is always out of range

__device__ __forceinline__ rsrc_t rsrc(const float* p, uint32_t count) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(count * 4u), 0x00020000);
}
// The b32 builtins move raw 32-bit words: reinterpret, never convert.
__device__ __forceinline__ float bld(rsrc_t r, uint32_t idx) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, idx * 4u, 0, 0));
}
__device__ __forceinline__ void bst(rsrc_t r, uint32_t idx, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, idx * 4u, 0, 0);
}

// Corner offsets of a trilinear cell (clamped: all 8 inside the grid).
struct Cell {
  uint32_t o[8];
  float fx, fy, fz;
};

__device__ __forceinline__ float lerp_cell(const Cell& c, float v0, float v1, float v2, float v3,
                                           float v4, float v5, float v6, float v7);

// XCD-aware work split of a sweep over n voxels.  Blocks are dealt to the 8 XCDs
// round-robin (block b runs on XCD b mod 8), so the blocks of one XCD take one
// contiguous eighth of the grid -- a slab of whole z-planes -- and stride through
// it together, keeping stencil and gather neighbours of the current window in
// that XCD's L2.  `tile` is the block's index among the `ntiles` (a multiple of
// 8) blocks of this problem; batched launches start every problem's tiles at a
// multiple of 8, so tile mod 8 is still the XCD.
struct XcdRange {
  uint32_t first, end, stride;
};

__device__ __forceinline__ XcdRange xcd_range(uint32_t n, uint32_t tile, uint32_t ntiles) {
  const uint32_t xcd = tile % kXCD, local = tile / kXCD;
  const uint32_t per = ntiles / kXCD;
  const uint32_t chunk = (n + kXCD - 1) / kXCD;
  const uint32_t beg = xcd * chunk;
  const uint32_t end = beg + chunk < n ? beg + chunk : n;
  return XcdRange{beg + local * kBlock + threadIdx.x, end, per * kBlock};
}

// Position y = i + d along one axis of length n, coordinates clamped to [0, n-1]:
// cell c = min(floor(y), n-2), fraction f = y - c.  The fraction is formed from d
// alone (d - floor(d) is exact), so no precision is lost to the integer part.
__device__ __forceinline__ void cell_clamp(int i, float d, int n, int& c, float& f) {
  d = fminf(fmaxf(d, -(float)(n + 2)), (float)(n + 2));   // also maps NaN to a finite value
  const float fl = floorf(d);
  int ci = i + (int)fl;
  float fr = d - fl;
  if (ci < 0) {
    ci = 0;
    fr = 0.f;
  } else if (ci >= n - 1) {
    ci = n - 2;
    fr = 1.f;
  }
  c = ci;
  f = fr;
}

// Same position without clamping (zero-outside sampling decides validity per corner).
__device__ __forceinline__ void cell_free(int i, float d, int n, int& c, float& f) {
  d = fminf(fmaxf(d, -(float)(n + 2)), (float)(n + 2));
  const float fl = floorf(d);
  c = i + (int)fl;
  f = d - fl;
}

__device__ __forceinline__ float lerp8(float v000, float v100, float v010, float v110, float v001,
                                       float v101, float v011, float v111, float fx, float fy,
                                       float fz) {
  const float a = v000 + fx * (v100 - v000);
  const float b = v010 + fx * (v110 - v010);
  const float c = v001 + fx * (v101 - v001);
  const float d = v011 + fx * (v111 - v011);
  const float e = a + fy * (b - a);
  const float f = c + fy * (d - c);
  return e + fz * (f - e);
}

__device__ __forceinline__ float lerp_cell(const Cell& c, float v0, float v1, float v2, float v3,
                                           float v4, float v5, float v6, float v7) {
  return lerp8(v0, v1, v2, v3, v4, v5, v6, v7, c.fx, c.fy, c.fz);
}

// Cell of position (x, y, z) + d with clamped coordinates.
__device__ __forceinline__ Cell make_cell_clamp(const Geom& g, int x, int y, int z, float dx,
                                                float dy, float dz) {
  Cell c;
  int cx, cy, cz;
  cell_clamp(x, dx, g.nx, cx, c.fx);
  cell_clamp(y, dy, g.ny, cy, c.fy);
  cell_clamp(z, dz, g.nz, cz, c.fz);
  const uint32_t sy = (uint32_t)g.nx, sz = (uint32_t)(g.nx * g.ny);
  const uint32_t o = vidx(g, cx, cy, cz);
  c.o[0] = o;
  c.o[1] = o + 1;
  c.o[2] = o + sy;
  c.o[3] = o + sy + 1;
  c.o[4] = o + sz;
  c.o[5] = o + sz + 1;
  c.o[6] = o + sz + sy;
  c.o[7] = o + sz + sy + 1;
  return c;
}

// Cell of position (x, y, z) + d for zero-outside sampling: corners outside the
// grid get the out-of-range offset and read as 0.
__device__ __forceinline__ Cell make_cell_zero(const Geom& g, int x, int y, int z, float dx,
                                               float dy, float dz) {
  Cell c;
  int cx, cy, cz;
  cell_free(x, dx, g.nx, cx, c.fx);
  cell_free(y, dy, g.ny, cy, c.fy);
  cell_free(z, dz, g.nz, cz, c.fz);
  const bool x0 = (unsigned)cx < (unsigned)g.nx, x1 = (unsigned)(cx + 1) < (unsigned)g.nx;
  const bool y0 = (unsigned)cy < (unsigned)g.ny, y1 = (unsigned)(cy + 1) < (unsigned)g.ny;
  const bool z0 = (unsigned)cz < (unsigned)g.nz, z1 = (unsigned)(cz + 1) < (unsigned)g.nz;
  const uint32_t sy = (uint32_t)g.nx, sz = (uint32_t)(g.nx * g.ny);
  const uint32_t o = (uint32_t)((cz * g.ny + cy) * g.nx + cx);   // wraps harmlessly when outside
  c.o[0] = (x0 && y0 && z0) ? o : kOutside;
  c.o[1] = (x1 && y0 && z0) ? o + 1 : kOutside;
  c.o[2] = (x0 && y1 && z0) ? o + sy : kOutside;
  c.o[3] = (x1 && y1 && z0) ? o + sy + 1 : kOutside;
  c.o[4] = (x0 && y0 && z1) ? o + sz : kOutside;
  c.o[5] = (x1 && y0 && z1) ? o + sz + 1 : kOutside;
  c.o[6] = (x0 && y1 && z1) ? o + sz + sy : kOutside;
  c.o[7] = (x1 && y1 && z1) ? o + sz + sy + 1 : kOutside;
  return c;
}

__device__ __forceinline__ float sample(rsrc_t r, const Cell& c) {
  return lerp_cell(c, bld(r, c.o[0]), bld(r, c.o[1]), bld(r, c.o[2]), bld(r, c.o[3]),
                   bld(r, c.o[4]), bld(r, c.o[5]), bld(r, c.o[6]), bld(r, c.o[7]));
}

// np.gradient-stencil derivative along one axis through a buffer.
__device__ __forceinline__ float dstencil_b(rsrc_t f, uint32_t i, int c, int n, uint32_t s,
                                            float inv_h) {
  const uint32_t ip = (c == n - 1) ? i : i + s;
  const uint32_t im = (c == 0) ? i : i - s;
  const float sc = (c == 0 || c == n - 1) ? inv_h : 0.5f * inv_h;
  return (bld(f, ip) - bld(f, im)) * sc;
}

// Neighbour offsets of the periodic 7-point stencil.
struct Nbr {
  uint32_t xm, xp, ym, yp, zm, zp;
};

__device__ __forceinline__ Nbr periodic_nbr(const Geom& g, uint32_t i, int x, int y, int z) {
  const uint32_t sy = (uint32_t)g.nx, sz = (uint32_t)(g.nx * g.ny);
  Nbr b;
  b.xm = (x == 0) ? i + g.nx - 1 : i - 1;
  b.xp = (x == g.nx - 1) ? i - (g.nx - 1) : i + 1;
  b.ym = (y == 0) ? i + (g.ny - 1) * sy : i - sy;
  b.yp = (y == g.ny - 1) ? i - (g.ny - 1) * sy : i + sy;
  b.zm = (z == 0) ? i + (g.nz - 1) * sz : i - sz;
  b.zp = (z == g.nz - 1) ? i - (g.nz - 1) * sz : i + sz;
  return b;
}

// 7-point Laplacian (unit spacing) from the six neighbour values and the centre;
// every caller goes through this one expression, so all give the same bits.
__device__ __forceinline__ float lap7_of(float xm, float xp, float ym, float yp, float zm, float zp,
                                         float center) {
  return (xm + xp) + (ym + yp) + (zm + zp) - 6.f * center;
}

__device__ __forceinline__ float lap7_b(rsrc_t f, const Nbr& b, float center) {
  return lap7_of(bld(f, b.xm), bld(f, b.xp), bld(f, b.ym), bld(f, b.yp), bld(f, b.zm),
                 bld(f, b.zp), center);
}

// Trilinear sample of a field at a clamped cell (all 8 corners inside the grid).
__device__ __forceinline__ float tri_clamped(const float* __restrict__ f, const Geom& g, int cx,
                                             int cy, int cz, float fx, float fy, float fz) {
  const uint32_t sy = (uint32_t)g.nx, sz = (uint32_t)(g.nx * g.ny);
  const uint32_t o = vidx(g, cx, cy, cz);
  return lerp8(f[o], f[o + 1], f[o + sy], f[o + sy + 1], f[o + sz], f[o + sz + 1], f[o + sz + sy],
               f[o + sz + sy + 1], fx, fy, fz);
}

// Trilinear sample with zero outside the grid.
__device__ __forceinline__ float tri_zero(const float* __restrict__ f, const Geom& g, int cx, int cy,
                                          int cz, float fx, float fy, float fz) {
  const bool x0 = (unsigned)cx < (unsigned)g.nx, x1 = (unsigned)(cx + 1) < (unsigned)g.nx;
  const bool y0 = (unsigned)cy < (unsigned)g.ny, y1 = (unsigned)(cy + 1) < (unsigned)g.ny;
  const bool z0 = (unsigned)cz < (unsigned)g.nz, z1 = (unsigned)(cz + 1) < (unsigned)g.nz;
  if (!((x0 || x1) && (y0 || y1) && (z0 || z1))) return 0.f;
  const int ax = x0 ? cx : cx + 1, bx = x1 ? cx + 1 : cx;
  const int ay = y0 ? cy : cy + 1, by = y1 ? cy + 1 : cy;
  const int az = z0 ? cz : cz + 1, bz = z1 ? cz + 1 : cz;
  const uint32_t sy = (uint32_t)g.nx, sz = (uint32_t)(g.nx * g.ny);
  const uint32_t ya = ay * sy, yb = by * sy, za = az * sz, zb = bz * sz;
  auto ld = [&](bool ok, uint32_t off) { return ok ? f[off] : 0.f; };
  const float v000 = ld(x0 && y0 && z0, za + ya + ax);
  const float v100 = ld(x1 && y0 && z0, za + ya + bx);
  const float v010 = ld(x0 && y1 && z0, za + yb + ax);
  const float v110 = ld(x1 && y1 && z0, za + yb + bx);
  const float v001 = ld(x0 && y0 && z1, zb + ya + ax);
  const float v101 = ld(x1 && y0 && z1, zb + ya + bx);
  const float v011 = ld(x0 && y1 && z1, zb + yb + ax);
  const float v111 = ld(x1 && y1 && z1, zb + yb + bx);
  return lerp8(v000, v100, v010, v110, v001, v101, v011, v111, fx, fy, fz);
}

// One-dimensional derivative with the np.gradient stencil: central inside,
// first-order one-sided on the two faces.
__device__ __forceinline__ float dstencil(const float* __restrict__ f, uint32_t i, int c, int n,
                                          uint32_t s, float inv_h) {
  if (c == 0) return (f[i + s] - f[i]) * inv_h;
  if (c == n - 1) return (f[i] - f[i - s]) * inv_h;
  return (f[i + s] - f[i - s]) * (0.5f * inv_h);
}

// Periodic 7-point Laplacian (times h^2) of f at (x, y, z).
__device__ __forceinline__ float lap7(const float* __restrict__ f, const Geom& g, uint32_t i, int x,
                                      int y, int z) {
  const uint32_t sy = (uint32_t)g.nx, sz = (uint32_t)(g.nx * g.ny);
  const uint32_t xm = (x == 0) ? i + g.nx - 1 : i - 1;
  const uint32_t xp = (x == g.nx - 1) ? i - (g.nx - 1) : i + 1;
  const uint32_t ym = (y == 0) ? i + (g.ny - 1) * sy : i - sy;
  const uint32_t yp = (y == g.ny - 1) ? i - (g.ny - 1) * sy : i + sy;
  const uint32_t zm = (z == 0) ? i + (g.nz - 1) * sz : i - sz;
  const uint32_t zp = (z == g.nz - 1) ? i - (g.nz - 1) * sz : i + sz;
  return (f[xm] + f[xp]) + (f[ym] + f[yp]) + (f[zm] + f[zp]) - 6.f * f[i];
}

// Sum over a 256-thread block (deterministic order); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int k = 0; k < kBlock / 64; ++k) t += red[k];
  }
  __syncthreads();
  return t;
}

__device__ __forceinline__ double block_min(double v) {
  __shared__ double red[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    t = red[0];
    for (int k = 1; k < kBlock / 64; ++k) t = fmin(t, red[k]);
  }
  __syncthreads();
  return t;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// Problem of block b in a batched launch (tile offsets are ascending).
__device__ __forceinline__ int batch_pair(const BatchRef& br, int b) {
  int p = 0;
  while (p + 1 < br.np && b >= br.off[p + 1]) ++p;
  return p;
}

}  // namespace lddmm
