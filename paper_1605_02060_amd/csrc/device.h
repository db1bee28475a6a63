// Device helpers: trilinear sampling, finite differences, block reductions.
#pragma once

#include "internal.h"

namespace lddmm {

// Index of voxel (x, y, z) on grid g.
__device__ __forceinline__ long long vidx(const Geom& g, int x, int y, int z) {
  return ((long long)z * g.ny + y) * g.nx + x;
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

// Trilinear sample of a field at a clamped cell (all 8 corners inside the grid).
__device__ __forceinline__ float tri_clamped(const float* __restrict__ f, const Geom& g, int cx,
                                             int cy, int cz, float fx, float fy, float fz) {
  const long long sy = g.nx, sz = (long long)g.nx * g.ny;
  const float* p = f + vidx(g, cx, cy, cz);
  return lerp8(p[0], p[1], p[sy], p[sy + 1], p[sz], p[sz + 1], p[sz + sy], p[sz + sy + 1], fx, fy,
               fz);
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
  const long long sy = g.nx, sz = (long long)g.nx * g.ny;
  const long long ya = ay * sy, yb = by * sy, za = az * sz, zb = bz * sz;
  auto ld = [&](bool ok, long long off) { return ok ? f[off] : 0.f; };
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
__device__ __forceinline__ float dstencil(const float* __restrict__ f, long long i, int c, int n,
                                          long long s, float inv_h) {
  if (c == 0) return (f[i + s] - f[i]) * inv_h;
  if (c == n - 1) return (f[i] - f[i - s]) * inv_h;
  return (f[i + s] - f[i - s]) * (0.5f * inv_h);
}

// Periodic 7-point Laplacian (times h^2) of f at (x, y, z).
__device__ __forceinline__ float lap7(const float* __restrict__ f, const Geom& g, long long i, int x,
                                      int y, int z) {
  const long long sy = g.nx, sz = (long long)g.nx * g.ny;
  const long long xm = (x == 0) ? i + g.nx - 1 : i - 1;
  const long long xp = (x == g.nx - 1) ? i - (g.nx - 1) : i + 1;
  const long long ym = (y == 0) ? i + (long long)(g.ny - 1) * sy : i - sy;
  const long long yp = (y == g.ny - 1) ? i - (long long)(g.ny - 1) * sy : i + sy;
  const long long zm = (z == 0) ? i + (long long)(g.nz - 1) * sz : i - sz;
  const long long zp = (z == g.nz - 1) ? i - (long long)(g.nz - 1) * sz : i + sz;
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

}  // namespace lddmm
