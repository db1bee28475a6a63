// Flow kernels: forward sweep (inverse maps + deformed templates + energy
// partials), backward sweep (forward maps + Jacobian + back-transported
// residual + body force), pyramid transfer, padding, apply and masks.
//
// Discretisation (Methods, Registration; Beg et al. 2005 as cited there):
//   u0_{j+1}(x) = -dt v_j(x) + S_clamp(u0_j; x - dt v_j(x)/h)
//   J0_{j+1}(x) = S_zero(J0; x + u0_{j+1}(x)/h)
//   u1_j(x)     =  dt v_j(x) + S_clamp(u1_{j+1}; x + dt v_j(x)/h)
//   b_j(x)      = (2/sigma^2) det(I + D u1_j) sum_c w_c S_zero(r_c; x + u1_j/h) grad J0c_j
// with u = phi - id in physical units (spacing h), positions in voxels.
#include "device.h"

namespace lddmm {

// Blocks of a sweep kernel: a multiple of the 8 XCDs, at most g_sweep_blocks.
static int g_sweep_blocks = 4096;

void set_sweep_blocks(int b) {
  b = (b + kXCD - 1) / kXCD * kXCD;
  g_sweep_blocks = b < kXCD ? kXCD : (b > kPartMax ? kPartMax : b);
}

int reduce_grid(long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  b = (b + kXCD - 1) / kXCD * kXCD;
  if (b > g_sweep_blocks) b = g_sweep_blocks;
  return (int)(b < kXCD ? kXCD : b);
}

static inline unsigned grid1d(long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  if (b > (1LL << 30)) b = 1LL << 30;
  return (unsigned)(b < 1 ? 1 : b);
}

// ------------------------------------------------------------------ setup ----

__global__ __launch_bounds__(kBlock) void k_pad(const float* __restrict__ src, int Nx, int Ny,
                                                int Nz, float* __restrict__ dst, Geom g) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < g.n;
       i += (long long)gridDim.x * kBlock) {
    int x, y, z;
    vcoord(g, (uint32_t)i, x, y, z);
    float v = 0.f;
    if (x < Nx && y < Ny && z < Nz) v = src[((long long)z * Ny + y) * Nx + x];
    dst[i] = v;
  }
}

void launch_pad(const float* src, int Nx, int Ny, int Nz, float* dst, const Geom& g,
                hipStream_t s) {
  hipLaunchKernelGGL(k_pad, dim3(grid1d(g.n)), dim3(kBlock), 0, s, src, Nx, Ny, Nz, dst, g);
}

// 2x block average, nfields consecutive planes of the fine grid.
__global__ __launch_bounds__(kBlock) void k_down2(const float* __restrict__ src, Geom f,
                                                  float* __restrict__ dst, Geom c, int nfields) {
  const long long total = c.n * nfields;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total;
       i += (long long)gridDim.x * kBlock) {
    const long long fld = i / c.n;
    const long long k = i - fld * c.n;
    const int x = (int)(k % c.nx);
    const long long t = k / c.nx;
    const int y = (int)(t % c.ny);
    const int z = (int)(t / c.ny);
    const float* p = src + fld * f.n + vidx(f, 2 * x, 2 * y, 2 * z);
    const int sy = f.nx, sz = f.nx * f.ny;
    const float s = ((p[0] + p[1]) + (p[sy] + p[sy + 1])) + ((p[sz] + p[sz + 1]) + (p[sz + sy] + p[sz + sy + 1]));
    dst[i] = 0.125f * s;
  }
}

void launch_down2(const float* src, const Geom& fine, float* dst, const Geom& coarse, int nfields,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_down2, dim3(grid1d(coarse.n * nfields)), dim3(kBlock), 0, s, src, fine, dst,
                     coarse, nfields);
}

// Cell-centred 2x trilinear upsample, coordinates clamped: fine i <-> coarse (i + 1/2)/2 - 1/2.
__global__ __launch_bounds__(kBlock) void k_up2(const float* __restrict__ src, Geom c,
                                                float* __restrict__ dst, Geom f, int nfields) {
  const long long total = f.n * nfields;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total;
       i += (long long)gridDim.x * kBlock) {
    const long long fld = i / f.n;
    const long long k = i - fld * f.n;
    const int x = (int)(k % f.nx);
    const long long t = k / f.nx;
    const int y = (int)(t % f.ny);
    const int z = (int)(t / f.ny);
    // coarse position = x/2 - 1/4 = floor(x/2) + d with d = -1/4 (x even) or +1/4 (x odd)
    int cx, cy, cz;
    float fx, fy, fz;
    cell_clamp(x >> 1, (x & 1) ? 0.25f : -0.25f, c.nx, cx, fx);
    cell_clamp(y >> 1, (y & 1) ? 0.25f : -0.25f, c.ny, cy, fy);
    cell_clamp(z >> 1, (z & 1) ? 0.25f : -0.25f, c.nz, cz, fz);
    dst[i] = tri_clamped(src + fld * c.n, c, cx, cy, cz, fx, fy, fz);
  }
}

void launch_up2(const float* src, const Geom& coarse, float* dst, const Geom& fine, int nfields,
                hipStream_t s) {
  hipLaunchKernelGGL(k_up2, dim3(grid1d(fine.n * nfields)), dim3(kBlock), 0, s, src, coarse, dst,
                     fine, nfields);
}

// Mean velocity over one step along the characteristic through grid point
// (x, y, z), with v_j constant in time within the step: the fourth-order
// Runge-Kutta stages of dy/ds = v_j(y) / h taken over the signed step s = +-dt/h
// (k1 = v_j(x), k2 = v_j(x + s/2 k1), k3 = v_j(x + s/2 k2), k4 = v_j(x + s k3),
// trilinear with clamped coordinates), vbar = (k1 + 2 k2 + 2 k3 + k4) / 6.  The
// departure or arrival point is then x + s vbar (the paper's flow integrator).
__device__ __forceinline__ void rk4_mean(rsrc_t V0, rsrc_t V1, rsrc_t V2, const Geom& g, int x,
                                         int y, int z, float s, float& mx, float& my, float& mz) {
  const float k1x = mx, k1y = my, k1z = mz;
  const Cell c2 = make_cell_clamp(g, x, y, z, 0.5f * s * k1x, 0.5f * s * k1y, 0.5f * s * k1z);
  const float k2x = sample(V0, c2), k2y = sample(V1, c2), k2z = sample(V2, c2);
  const Cell c3 = make_cell_clamp(g, x, y, z, 0.5f * s * k2x, 0.5f * s * k2y, 0.5f * s * k2z);
  const float k3x = sample(V0, c3), k3y = sample(V1, c3), k3z = sample(V2, c3);
  const Cell c4 = make_cell_clamp(g, x, y, z, s * k3x, s * k3y, s * k3z);
  const float k4x = sample(V0, c4), k4y = sample(V1, c4), k4z = sample(V2, c4);
  const float sixth = 1.f / 6.f;
  mx = (k1x + 2.f * k2x + 2.f * k3x + k4x) * sixth;
  my = (k1y + 2.f * k2y + 2.f * k3y + k4y) * sixth;
  mz = (k1z + 2.f * k2z + 2.f * k3z + k4z) * sixth;
}

// ---------------------------------------------------------- forward sweep ----

// Buffers of forward step j as raw buffer descriptors.
template <int NC>
struct FwdView {
  rsrc_t V0, V1, V2;            // v_j
  rsrc_t U0, U1, U2;            // u0_j
  rsrc_t W0, W1, W2;            // u0_{j+1}
  rsrc_t T0[NC], T1[NC], OUT[NC];
  rsrc_t IM0, IM1;              // monitored image channel
};

template <int NC, bool LAST>
__device__ __forceinline__ FwdView<NC> fwd_view(const FwdArgs& a) {
  const long long N = a.g.n;
  const uint32_t n = (uint32_t)N;
  FwdView<NC> f;
  const float* vb = (a.st->eval ? a.vB : a.vA) + (long long)a.j * 3 * N;
  f.V0 = rsrc(vb, n);
  f.V1 = rsrc(vb + N, n);
  f.V2 = rsrc(vb + 2 * N, n);
  f.U0 = rsrc(a.u_cur, n);
  f.U1 = rsrc(a.u_cur + N, n);
  f.U2 = rsrc(a.u_cur + 2 * N, n);
  f.W0 = rsrc(a.u_next, n);
  f.W1 = rsrc(a.u_next + N, n);
  f.W2 = rsrc(a.u_next + 2 * N, n);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    f.T0[c] = rsrc(a.J0 + (long long)a.ch[c] * N, n);
    f.T1[c] = rsrc(a.J1 + (long long)a.ch[c] * N, n);
    f.OUT[c] = rsrc((LAST ? a.r : a.J0t_next) + (long long)c * N, n);
  }
  const int ic = a.img_ch >= 0 ? a.img_ch : 0;
  f.IM0 = rsrc(a.J0 + (long long)ic * N, n);
  f.IM1 = rsrc(a.J1 + (long long)ic * N, n);
  return f;
}

// Forward step j at voxel i = (x, y, z): the map step, the deformed templates
// (the residual and the data terms at the last step) and the regulariser term
// |gamma v - alpha Lap v|^2 from v_j = (vx, vy, vz) and its 7-point Laplacians.
// The map u0_j at a clamped position, read from global memory: every traversal's
// sampler gives these bits (the LDS-staged one samples the same 8 corners in the
// same order).
template <int NC>
struct GlobalMapSampler {
  const FwdView<NC>& f;
  const Geom& g;
  __device__ __forceinline__ void operator()(int x, int y, int z, float dx, float dy, float dz,
                                             float out[3]) const {
    const Cell cl = make_cell_clamp(g, x, y, z, dx, dy, dz);
    out[0] = sample(f.U0, cl);
    out[1] = sample(f.U1, cl);
    out[2] = sample(f.U2, cl);
  }
};

// The weighted template channels with zero outside the grid at (x, y, z) + d.
template <int NC>
struct GlobalTemplateSampler {
  const FwdView<NC>& f;
  const Geom& g;
  __device__ __forceinline__ void operator()(int x, int y, int z, float dx, float dy, float dz,
                                             float out[NC]) const {
    const Cell cz = make_cell_zero(g, x, y, z, dx, dy, dz);
#pragma unroll
    for (int c = 0; c < NC; ++c) out[c] = sample(f.T0[c], cz);
  }
};

template <int NC, bool FIRST, bool LAST, bool RK4, class MapSampler, class TemplateSampler>
__device__ __forceinline__ void forward_voxel(const FwdArgs& a, const FwdView<NC>& f, uint32_t i,
                                              int x, int y, int z, float vx, float vy, float vz,
                                              float lapx, float lapy, float lapz, double& accR,
                                              double& accD, double& accI, const MapSampler& ms,
                                              const TemplateSampler& ts) {
  const Geom& g = a.g;
  const float dt = a.dt, ih = g.inv_h;
  const float c2 = a.alpha * ih * ih;
  float mx = vx, my = vy, mz = vz;                    // velocity of the map step
  if (RK4) rk4_mean(f.V0, f.V1, f.V2, g, x, y, z, -dt * ih, mx, my, mz);
  float ux = -dt * mx, uy = -dt * my, uz = -dt * mz;
  if (!FIRST) {
    float gv[3];
    ms(x, y, z, -dt * mx * ih, -dt * my * ih, -dt * mz * ih, gv);
    ux += gv[0];
    uy += gv[1];
    uz += gv[2];
  }
  bst(f.W0, i, ux);
  bst(f.W1, i, uy);
  bst(f.W2, i, uz);
  // deformed templates at t_{j+1}
  {
    float tv[NC];
    ts(x, y, z, ux * ih, uy * ih, uz * ih, tv);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const float val = tv[c];
      if (!LAST) {
        bst(f.OUT[c], i, val);
      } else {
        const float r = val - bld(f.T1[c], i);
        bst(f.OUT[c], i, r);
        accD += (double)a.w[c] * (double)r * (double)r;
        if (a.img_weighted && c == a.img_slot) accI += (double)r * (double)r;
      }
    }
    if (LAST && a.img_ch >= 0 && !a.img_weighted) {
      const Cell cz = make_cell_zero(g, x, y, z, ux * ih, uy * ih, uz * ih);
      const float d = sample(f.IM0, cz) - bld(f.IM1, i);
      accI += (double)d * (double)d;
    }
  }
  // |L v_j|^2 with L = gamma - alpha Lap (periodic 7-point)
  const float lx = a.gamma * vx - c2 * lapx;
  const float ly = a.gamma * vy - c2 * lapy;
  const float lz = a.gamma * vz - c2 * lapz;
  accR += (double)lx * lx + (double)ly * ly + (double)lz * lz;
}

template <bool LAST>
__device__ __forceinline__ void forward_partials(const FwdArgs& a, uint32_t tile, double accR,
                                                 double accD, double accI) {
  const double sR = block_sum(accR);
  if (threadIdx.x == 0) a.partR[tile] = sR;
  if (LAST) {
    const double sD = block_sum(accD);
    const double sI = block_sum(accI);
    if (threadIdx.x == 0) {
      a.partD[tile] = sD;
      a.partI[tile] = sI;
    }
  }
}

// Grid-stride traversal: the XCD slabs of xcd_range, every voxel on its own.
template <int NC, bool FIRST, bool LAST, bool RK4 = false>
__device__ __forceinline__ void forward_body(const FwdArgs& a, uint32_t tile, uint32_t ntiles) {
  if (a.st->mode == MODE_STOPPED) return;
  const Geom g = a.g;
  const FwdView<NC> f = fwd_view<NC, LAST>(a);
  double accR = 0.0, accD = 0.0, accI = 0.0;
  const XcdRange rg = xcd_range((uint32_t)g.n, tile, ntiles);
  for (uint32_t i = rg.first; i < rg.end; i += rg.stride) {
    int x, y, z;
    vcoord(g, i, x, y, z);
    const float vx = bld(f.V0, i), vy = bld(f.V1, i), vz = bld(f.V2, i);
    const Nbr nb = periodic_nbr(g, i, x, y, z);
    forward_voxel<NC, FIRST, LAST, RK4>(a, f, i, x, y, z, vx, vy, vz, lap7_b(f.V0, nb, vx),
                                        lap7_b(f.V1, nb, vy), lap7_b(f.V2, nb, vz), accR, accD,
                                        accI, GlobalMapSampler<NC>{f, g},
                                        GlobalTemplateSampler<NC>{f, g});
  }
  forward_partials<LAST>(a, tile, accR, accD, accI);
}

// Plane-marching traversal.  A tile is kBlock consecutive voxels of an xy plane
// over a run of consecutive planes; each thread walks its column up the run and
// keeps v_j of the planes below, at and above the current one in registers (the
// z terms of the stencil), loading the plane after next one step ahead, so the
// gathers of a step never wait on the load of v.  Tiles go to the XCDs in
// contiguous runs (block b runs on XCD b mod 8), so the rows above and below a
// tile, which the stencil and the gathers read, come from neighbouring tiles of
// the same XCD and its L2.  ntiles is a multiple of 8 and at least the number of
// plane blocks ceil(nx ny / kBlock); tiles past the last run are idle.
template <int NC, bool FIRST, bool LAST, bool RK4 = false>
__device__ __forceinline__ void forward_zmarch_body(const FwdArgs& a, uint32_t tile,
                                                    uint32_t ntiles) {
  if (a.st->mode == MODE_STOPPED) return;
  const Geom g = a.g;
  const FwdView<NC> f = fwd_view<NC, LAST>(a);
  const uint32_t nx = (uint32_t)g.nx, ny = (uint32_t)g.ny, nz = (uint32_t)g.nz;
  const uint32_t nxy = nx * ny;
  const uint32_t nb = (nxy + kBlock - 1) / kBlock;
  uint32_t nzc = ntiles / nb;
  nzc = nzc < 1 ? 1 : (nzc > nz ? nz : nzc);
  const uint32_t run = (nz + nzc - 1) / nzc;
  const uint32_t l = (tile % kXCD) * (ntiles / kXCD) + tile / kXCD;
  const uint32_t zc = l / nb;
  const uint32_t p = (l - zc * nb) * kBlock + threadIdx.x;   // index within the plane
  const uint32_t z0 = zc * run;
  double accR = 0.0, accD = 0.0, accI = 0.0;
  if (p < nxy && z0 < nz) {
    const uint32_t z1 = z0 + run < nz ? z0 + run : nz;
    const uint32_t yq = fdiv(p, g.fx);
    const int x = (int)(p - yq * nx), y = (int)yq;
    // periodic in-plane neighbours as offsets added to i (modulo 2^32)
    const uint32_t dxm = x == 0 ? nx - 1 : 0u - 1u;
    const uint32_t dxp = x == (int)nx - 1 ? 0u - (nx - 1) : 1u;
    const uint32_t dym = y == 0 ? (ny - 1) * nx : 0u - nx;
    const uint32_t dyp = y == (int)ny - 1 ? 0u - (ny - 1) * nx : nx;
    const rsrc_t V[3] = {f.V0, f.V1, f.V2};
    const uint32_t zb = z0 == 0 ? nz - 1 : z0 - 1;
    uint32_t zp = z0 + 1 == nz ? 0 : z0 + 1;
    float vm[3], vc[3], vp[3];                               // v_j at z - 1, z, z + 1
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      vm[c] = bld(V[c], zb * nxy + p);
      vc[c] = bld(V[c], z0 * nxy + p);
      vp[c] = bld(V[c], zp * nxy + p);
    }
    for (uint32_t z = z0; z < z1; ++z) {
      const uint32_t i = z * nxy + p;
      const uint32_t zn = zp + 1 == nz ? 0 : zp + 1;         // the plane after next
      float vn[3] = {0.f, 0.f, 0.f};
      if (z + 1 < z1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) vn[c] = bld(V[c], zn * nxy + p);
      }
      float lap[3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        lap[c] = lap7_of(bld(V[c], i + dxm), bld(V[c], i + dxp), bld(V[c], i + dym),
                         bld(V[c], i + dyp), vm[c], vp[c], vc[c]);
      forward_voxel<NC, FIRST, LAST, RK4>(a, f, i, x, y, (int)z, vc[0], vc[1], vc[2], lap[0],
                                          lap[1], lap[2], accR, accD, accI,
                                          GlobalMapSampler<NC>{f, g},
                                          GlobalTemplateSampler<NC>{f, g});
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        vm[c] = vc[c];
        vc[c] = vp[c];
        vp[c] = vn[c];
      }
      zp = zn;
    }
  }
  forward_partials<LAST>(a, tile, accR, accD, accI);
}

template <int NC, bool FIRST, bool LAST, bool RK4>
__device__ void forward_staged_body(const FwdArgs& a, int block);

// TRAV: 0 grid-stride, 1 plane-marching, 2 LDS-staged (forward_traversal)
template <int NC, bool FIRST, bool LAST, bool RK4, int TRAV>
__global__ __launch_bounds__(kBlock) void k_forward(FwdArgs a) {
  if (TRAV == 2)
    forward_staged_body<NC, FIRST, LAST, RK4>(a, blockIdx.x);
  else if (TRAV == 1)
    forward_zmarch_body<NC, FIRST, LAST, RK4>(a, blockIdx.x, gridDim.x);
  else
    forward_body<NC, FIRST, LAST, RK4>(a, blockIdx.x, gridDim.x);
}

// One launch for every problem of a batch: block b runs tile b - off[p] of problem p.
template <int NC, bool FIRST, bool LAST>
__global__ __launch_bounds__(kBlock) void k_forward_batched(BatchRef br, int j) {
  const int p = batch_pair(br, blockIdx.x);
  const PairTab* t = (const PairTab*)br.tab[p];
  const uint32_t tile = blockIdx.x - br.off[p], ntiles = br.off[p + 1] - br.off[p];
  if (t->fwd[j].staged)
    forward_staged_body<NC, FIRST, LAST, false>(t->fwd[j], (int)tile);
  else if (t->fwd[j].zmarch)
    forward_zmarch_body<NC, FIRST, LAST>(t->fwd[j], tile, ntiles);
  else
    forward_body<NC, FIRST, LAST>(t->fwd[j], tile, ntiles);
}

// Tiles of a plane-marching launch: whole runs of planes for every plane block,
// at most g_fwd_tiles where that allows one run, rounded up to a multiple of 8;
// 0 selects the grid-stride traversal.
static int g_fwd_tiles = 1792;

void set_fwd_tiles(int t) { g_fwd_tiles = t <= 0 ? 0 : (t > kPartMax ? kPartMax : t); }

static long long plane_blocks(const Geom& g) {
  return ((long long)g.nx * g.ny + kBlock - 1) / kBlock;
}

bool forward_zmarch(const Geom& g) {
  return g_fwd_tiles > 0 && plane_blocks(g) <= kPartMax - (kXCD - 1);
}

int forward_staged_blocks(const Geom& g);

int forward_tiles(const Geom& g) {
  if (forward_staged(g)) return forward_staged_blocks(g);
  if (!forward_zmarch(g)) return reduce_grid(g.n);
  const long long nb = plane_blocks(g);
  long long nzc = g_fwd_tiles / nb;                           // runs of planes
  const long long cap = (kPartMax - (kXCD - 1)) / nb;         // so that the tiles fit kPartMax
  if (nzc > cap) nzc = cap;
  if (nzc > g.nz) nzc = g.nz;
  if (nzc < 1) nzc = 1;
  const long long run = (g.nz + nzc - 1) / nzc;
  nzc = (g.nz + run - 1) / run;
  return (int)((nb * nzc + kXCD - 1) / kXCD * kXCD);
}

template <int NC, bool RK4>
static void fwd_dispatch(const FwdArgs& a, hipStream_t s) {
  const int grid = (a.staged || a.zmarch) ? forward_tiles(a.g) : reduce_grid(a.g.n);
  const bool first = (a.j == 0), last = (a.j == a.T - 1);
#define FWD(F, L, Z) \
  hipLaunchKernelGGL((k_forward<NC, F, L, RK4, Z>), dim3(grid), dim3(kBlock), 0, s, a)
  if (a.staged) {
    if (first && last) FWD(true, true, 2); else if (first) FWD(true, false, 2);
    else if (last) FWD(false, true, 2); else FWD(false, false, 2);
  } else if (a.zmarch) {
    if (first && last) FWD(true, true, 1); else if (first) FWD(true, false, 1);
    else if (last) FWD(false, true, 1); else FWD(false, false, 1);
  } else {
    if (first && last) FWD(true, true, 0); else if (first) FWD(true, false, 0);
    else if (last) FWD(false, true, 0); else FWD(false, false, 0);
  }
#undef FWD
}



// --------------------------------------------------------- backward sweep ----

template <int NC, bool HAS_U, bool UZERO, bool HAS_B, bool RK4 = false>
__device__ __forceinline__ void backward_body(const BwdArgs& a, uint32_t tile, uint32_t ntiles) {
  const State* st = a.st;
  if (a.need_mode >= 0 && st->mode != a.need_mode) return;
  const Geom g = a.g;
  const long long N = g.n;
  const uint32_t n = (uint32_t)N;
  const float dt = a.dt, ih = g.inv_h;
  const uint32_t sy = (uint32_t)g.nx, sz = (uint32_t)(g.nx * g.ny);
  const float* vb = (a.vfix ? a.vfix : (st->base ? a.vB : a.vA)) +
                    (long long)(a.j >= 0 ? a.j : 0) * 3 * N;
  const rsrc_t V0 = rsrc(vb, n), V1 = rsrc(vb + N, n), V2 = rsrc(vb + 2 * N, n);
  const float* un = a.u_next ? a.u_next : a.u_cur;   // unused when UZERO and !HAS_B
  const rsrc_t N0 = rsrc(un, n), N1 = rsrc(un + N, n), N2 = rsrc(un + 2 * N, n);
  float* uc = a.u_cur ? a.u_cur : a.b;               // unused when !HAS_U
  const rsrc_t C0 = rsrc(uc, n), C1 = rsrc(uc + N, n), C2 = rsrc(uc + 2 * N, n);
  const rsrc_t B0 = rsrc(a.b, n), B1 = rsrc(a.b + N, n), B2 = rsrc(a.b + 2 * N, n);
  rsrc_t RR[NC], JJ[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    RR[c] = rsrc(a.r + (long long)c * N, n);
    JJ[c] = rsrc(a.J0t + (long long)c * a.cstride, n);
  }
  double mind = 1e300;
  const XcdRange rg = xcd_range(n, tile, ntiles);
  for (uint32_t i = rg.first; i < rg.end; i += rg.stride) {
    int x, y, z;
    vcoord(g, i, x, y, z);
    if (HAS_U) {
      float vx = bld(V0, i), vy = bld(V1, i), vz = bld(V2, i);
      if (RK4) rk4_mean(V0, V1, V2, g, x, y, z, dt * ih, vx, vy, vz);   // vbar replaces v_j(x)
      float ux = dt * vx, uy = dt * vy, uz = dt * vz;
      if (!UZERO) {
        const Cell cl = make_cell_clamp(g, x, y, z, dt * vx * ih, dt * vy * ih, dt * vz * ih);
        ux += sample(N0, cl);
        uy += sample(N1, cl);
        uz += sample(N2, cl);
      }
      bst(C0, i, ux);
      bst(C1, i, uy);
      bst(C2, i, uz);
    }
    if (HAS_B) {
      // Jacobian matrix I + D u of u1 at time jb (rows: component, columns: direction)
      float J[3][3];
      const rsrc_t nr[3] = {N0, N1, N2};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        J[c][0] = dstencil_b(nr[c], i, x, g.nx, 1u, ih);
        J[c][1] = dstencil_b(nr[c], i, y, g.ny, sy, ih);
        J[c][2] = dstencil_b(nr[c], i, z, g.nz, sz, ih);
      }
      J[0][0] += 1.f;
      J[1][1] += 1.f;
      J[2][2] += 1.f;
      const float det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                        J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                        J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      mind = fmin(mind, (double)det);
      const Cell cz = make_cell_zero(g, x, y, z, bld(N0, i) * ih, bld(N1, i) * ih,
                                     bld(N2, i) * ih);
      float bx = 0.f, by = 0.f, bz = 0.f;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const float rw = a.w[c] * sample(RR[c], cz);
        bx += rw * dstencil_b(JJ[c], i, x, g.nx, 1u, ih);
        by += rw * dstencil_b(JJ[c], i, y, g.ny, sy, ih);
        bz += rw * dstencil_b(JJ[c], i, z, g.nz, sz, ih);
      }
      const float s = a.coef * det;
      bst(B0, i, s * bx);
      bst(B1, i, s * by);
      bst(B2, i, s * bz);
    }
  }
  if (HAS_B) {
    const double m = block_min(mind);
    if (threadIdx.x == 0) a.partDet[tile] = m;
  }
}

template <int NC, bool HAS_U, bool UZERO, bool HAS_B, bool RK4>
__global__ __launch_bounds__(kBlock) void k_backward(BwdArgs a) {
  backward_body<NC, HAS_U, UZERO, HAS_B, RK4>(a, blockIdx.x, gridDim.x);
}

template <int NC, bool HAS_U, bool UZERO, bool HAS_B>
__global__ __launch_bounds__(kBlock) void k_backward_batched(BatchRef br, int slot) {
  const int p = batch_pair(br, blockIdx.x);
  const PairTab* t = (const PairTab*)br.tab[p];
  backward_body<NC, HAS_U, UZERO, HAS_B>(t->bwd[slot], blockIdx.x - br.off[p],
                                         br.off[p + 1] - br.off[p]);
}

// ------------------------------------------- backward sweep, LDS-staged ----
// The body-force steps of backward_body, with the gathers and stencils of
// u1_{j+1} and the stencil of the deformed template read from LDS.  A block owns
// a kBX x kBY column of (x, y) and marches up one z-slab, keeping rings of planes
// in LDS and loading one new plane of each per step while the step computes:
//  - u1_{j+1}: planes z - kBH .. z + kBH with an (x, y) halo of kBH, clamped to
//    the grid.  A map gather whose cell leaves this window (|dt v / h| >= kBH)
//    reads global memory;
//  - the deformed template: planes z - 1 .. z + 1, halo 1 (its gradient).
// The residual gather (displacements of many voxels) stays in global memory.
// The arithmetic and its order are those of backward_body, so both give the
// same bits.  The halo is 1: the stencil needs no more, and a map gather of
// less than a voxel per step (the usual case: about 0.3 voxel in the atlas
// workload) stays in the window; filling a halo-2 ring cost more than the
// gathers between one and two voxels it kept in LDS.  The columns are 64 x 4:
// a wavefront then owns one 64-voxel row segment, whose loads touch fewer cache
// lines than the two 32-voxel segments of a 32 x 8 column, which pays for the
// taller halo (66 x 6 against 34 x 10 staged values per 256 voxels).
constexpr int kBX = 64, kBY = 4, kBH = 1;
constexpr int kBRing = 2 * kBH + 1;
constexpr int kBXH = kBX + 2 * kBH, kBYH = kBY + 2 * kBH;     // map window
constexpr int kBXJ = kBX + 2, kBYJ = kBY + 2;                 // halo-1 window
constexpr int kUPlane = 3 * kBYH * kBXH;
constexpr int kURegs = (kUPlane + kBlock - 1) / kBlock;
static_assert(kBX * kBY == kBlock, "one voxel per thread and plane");

struct SweepTiling {
  int ntx, nty, nslab;
};

__host__ __device__ inline SweepTiling sweep_tiling(const Geom& g) {
  SweepTiling t;
  t.ntx = (g.nx + kBX - 1) / kBX;
  t.nty = (g.ny + kBY - 1) / kBY;
  const int per = g.nz / (kXCD * 15);                 // about 15 planes per slab
  t.nslab = kXCD * (per < 1 ? 1 : per);
  return t;
}

// The staged kernel runs when it has at least g_staged_min_blocks blocks (default
// 8 per CU: a block marches a whole slab, so fewer leave the chip idle -- at
// 140 x 80 x 120 it has 400 blocks and ran 1.7x slower than the grid-stride
// kernel), when its blocks fit the partial buffer, and when every byte offset
// into a map (3 n floats) fits 32 bits.  The host decides and passes the
// decision in BwdArgs::staged.
static int g_staged_min_blocks = 2048;

void set_staged_min_blocks(int b) { g_staged_min_blocks = b < 1 ? 1 : b; }

bool backward_staged(const Geom& g) {
  const SweepTiling t = sweep_tiling(g);
  const long long blocks = (long long)t.ntx * t.nty * t.nslab;
  return blocks >= g_staged_min_blocks && blocks <= kPartMax && 3LL * g.n < (1LL << 30);
}

// Blocks (and min-det partials) of one body-force launch of this grid.
int backward_partials(const Geom& g) {
  if (!backward_staged(g)) return reduce_grid(g.n);
  const SweepTiling t = sweep_tiling(g);
  return t.ntx * t.nty * t.nslab;
}

struct SlabTile {
  int x0, y0, zbeg, zend;
};

// Block -> (column, slab).  Blocks run on XCD block mod 8; the slabs of XCD x
// are x, x + 8, ..., so each XCD's L2 serves disjoint z-ranges.
__device__ __forceinline__ SlabTile slab_tile(const Geom& g, int block) {
  const SweepTiling tl = sweep_tiling(g);
  const int ntile = tl.ntx * tl.nty;
  const int xcd = block % kXCD, local = block / kXCD;
  const int slab = xcd + kXCD * (local / ntile), tile = local % ntile;
  SlabTile t;
  t.x0 = (tile % tl.ntx) * kBX;
  t.y0 = (tile / tl.ntx) * kBY;
  t.zbeg = (int)((long long)slab * g.nz / tl.nslab);
  t.zend = (int)((long long)(slab + 1) * g.nz / tl.nslab);
  return t;
}


// Ring of map planes (3 components, halo kBH, clamped) staged through registers.
// Slot-major layout: element e of a staged plane (component, window row, window
// column: the order in which the block's threads load them) sits at s[slot] + e.
// A thread's LDS addresses and in-plane global offsets are then the same on every
// plane of the march and are computed once, before it.
struct MapRing {
  float (*s)[3][kBYH][kBXH];     // [slot][component][row][column]
  float reg[kURegs];
  uint32_t off[kURegs];          // in-plane element offset of element r, component included,
                                 // of the periodic image of its (x, y)
  uint32_t ok;                   // bit r: element r lies in the grid's (x, y) range
  __device__ __forceinline__ void init(const Geom& g, uint32_t n, int x0, int y0) {
    ok = 0u;
#pragma unroll
    for (int r = 0; r < kURegs; ++r) {
      const int e = threadIdx.x + r * kBlock;
      off[r] = 0u;
      if (e < kUPlane) {
        const int c = e / (kBYH * kBXH), rem = e - c * (kBYH * kBXH);
        const int ly = rem / kBXH, lx = rem - ly * kBXH;
        const int gx = x0 - kBH + lx, gy = y0 - kBH + ly;
        const int px = (gx % g.nx + g.nx) % g.nx, py = (gy % g.ny + g.ny) % g.ny;
        off[r] = (uint32_t)c * n + (uint32_t)(py * g.nx + px);
        if ((unsigned)gx < (unsigned)g.nx && (unsigned)gy < (unsigned)g.ny) ok |= 1u << r;
      }
    }
  }
  // Plane p into registers (0 outside the grid).
  __device__ __forceinline__ void fetch(rsrc_t U, const Geom& g, int p) {
    const bool pin = p >= 0 && p < g.nz;
    const uint32_t po = pin ? (uint32_t)p * (uint32_t)(g.nx * g.ny) : 0u;
#pragma unroll
    for (int r = 0; r < kURegs; ++r) reg[r] = (pin && ((ok >> r) & 1u)) ? bld(U, off[r] + po) : 0.f;
  }
  // Plane p (-nz <= p < 2 nz) of a periodic field into registers, the window
  // wrapped around the grid in x, y and z.
  __device__ __forceinline__ void fetch_periodic(rsrc_t U, const Geom& g, int p) {
    const int pw = p < 0 ? p + g.nz : (p >= g.nz ? p - g.nz : p);
    const uint32_t po = (uint32_t)pw * (uint32_t)(g.nx * g.ny);
#pragma unroll
    for (int r = 0; r < kURegs; ++r)
      reg[r] = (threadIdx.x + r * kBlock < kUPlane) ? bld(U, off[r] + po) : 0.f;
  }
  // Plane p >= 0 into slot p mod 2 of a two-slot ring of the same window.
  __device__ __forceinline__ void put2(int p) {
    float* base = &s[p & 1][0][0][0];
#pragma unroll
    for (int r = 0; r < kURegs; ++r) {
      const int e = threadIdx.x + r * kBlock;
      if (e < kUPlane) base[e] = reg[r];
    }
  }
  // Plane p >= -kBRing into slot (p + kBRing) mod kBRing.
  __device__ __forceinline__ void put(int p) {
    float* base = &s[(p + kBRing) % kBRing][0][0][0];
#pragma unroll
    for (int r = 0; r < kURegs; ++r) {
      const int e = threadIdx.x + r * kBlock;
      if (e < kUPlane) base[e] = reg[r];
    }
  }
  // Trilinear sample of all three components at the clamped cell (cx, cy, cz),
  // if its 8 corners are in the window of step z.
  __device__ __forceinline__ bool sample3(int x0, int y0, int z, int cx, int cy, int cz, float fx,
                                          float fy, float fz, float out[3]) const {
    const int wx = cx - (x0 - kBH), wy = cy - (y0 - kBH);
    if (!(wx >= 0 && wx + 1 < kBXH && wy >= 0 && wy + 1 < kBYH && cz >= z - kBH &&
          cz + 1 <= z + kBH))
      return false;
    const int za = cz % kBRing, zb = (cz + 1) % kBRing;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      out[c] = lerp8(s[za][c][wy][wx], s[za][c][wy][wx + 1], s[za][c][wy + 1][wx],
                     s[za][c][wy + 1][wx + 1], s[zb][c][wy][wx], s[zb][c][wy][wx + 1],
                     s[zb][c][wy + 1][wx], s[zb][c][wy + 1][wx + 1], fx, fy, fz);
    return true;
  }
};

// Ring of K-component planes z - 1 .. z + 1 with halo 1 (zero outside the grid),
// slot-major like MapRing.
template <int K>
struct HaloRing {
  static constexpr int kPlane = K * kBYJ * kBXJ;
  static constexpr int kRegs = (kPlane + kBlock - 1) / kBlock;
  float (*s)[K][kBYJ][kBXJ];     // [slot][component][row][column]
  float reg[kRegs];
  uint32_t off[kRegs];           // in-plane element offset of element r
  uint32_t ok, c1;               // bit r: in the grid's (x, y) range / of component 1
  __device__ __forceinline__ void init(const Geom& g, int x0, int y0) {
    ok = 0u;
    c1 = 0u;
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
      const int e = threadIdx.x + r * kBlock;
      off[r] = 0u;
      if (e < kPlane) {
        const int c = e / (kBYJ * kBXJ), rem = e - c * (kBYJ * kBXJ);
        const int ly = rem / kBXJ, lx = rem - ly * kBXJ;
        const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        if ((unsigned)gx < (unsigned)g.nx && (unsigned)gy < (unsigned)g.ny) {
          off[r] = (uint32_t)(gy * g.nx + gx);
          ok |= 1u << r;
          if (c > 0) c1 |= 1u << r;
        }
      }
    }
  }
  // One component: the window is that of a map ring with halo 1, whose element e
  // of component 0 has the same in-plane offset, so its offsets are taken over.
  __device__ __forceinline__ void init_from(const MapRing& m) {
    static_assert(K == 1 && kBH == 1 && kBXJ == kBXH && kBYJ == kBYH && kRegs <= kURegs,
                  "the same window");
    ok = 0u;
    c1 = 0u;
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
      off[r] = m.off[r];
      if (threadIdx.x + r * kBlock < kPlane) ok |= m.ok & (1u << r);
    }
  }
  // Plane p of every component into registers; component c is read through R[c].
  __device__ __forceinline__ void fetch(const rsrc_t* R, const Geom& g, int p) {
    const bool pin = p >= 0 && p < g.nz;
    const uint32_t po = pin ? (uint32_t)p * (uint32_t)(g.nx * g.ny) : 0u;
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
      float val = 0.f;
      if (pin && ((ok >> r) & 1u)) val = bld(R[K > 1 && ((c1 >> r) & 1u) ? 1 : 0], off[r] + po);
      reg[r] = val;
    }
  }
  // Plane p >= -1 into slot (p + 3) mod 3 (the planes outside the grid as zeros).
  __device__ __forceinline__ void put(int p) {
    float* base = &s[(p + 3) % 3][0][0][0];
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
      const int e = threadIdx.x + r * kBlock;
      if (e < kPlane) base[e] = reg[r];
    }
  }
  // Whether the 8 corners of cell (cx, cy, cz) lie in the window of step z:
  // columns x0 - 1 .. x0 + kBX, rows y0 - 1 .. y0 + kBY, planes z - 1 .. z + 1.
  __device__ __forceinline__ static bool covers(int x0, int y0, int z, int cx, int cy, int cz) {
    const int wx = cx - (x0 - 1), wy = cy - (y0 - 1);
    return wx >= 0 && wx + 1 < kBXJ && wy >= 0 && wy + 1 < kBYJ && cz >= z - 1 && cz <= z;
  }
  // Trilinear sample of component c at a covered cell, zero outside the grid (the
  // staged planes hold zeros there), corners in the order of sample().
  __device__ __forceinline__ float lerp(int c, int x0, int y0, int cx, int cy, int cz, float fx,
                                        float fy, float fz) const {
    const int wx = cx - (x0 - 1), wy = cy - (y0 - 1);
    const int za = (cz + 3) % 3, zb = (cz + 4) % 3;
    return lerp8(s[za][c][wy][wx], s[za][c][wy][wx + 1], s[za][c][wy + 1][wx],
                 s[za][c][wy + 1][wx + 1], s[zb][c][wy][wx], s[zb][c][wy][wx + 1],
                 s[zb][c][wy + 1][wx], s[zb][c][wy + 1][wx + 1], fx, fy, fz);
  }
};

__device__ __forceinline__ float dstencil_v(float plus, float minus, float center, int c, int n,
                                            float inv_h) {
  const float vp = (c == n - 1) ? center : plus;
  const float vm = (c == 0) ? center : minus;
  const float sc = (c == 0 || c == n - 1) ? inv_h : 0.5f * inv_h;
  return (vp - vm) * sc;
}

template <int NC, bool HAS_U, bool RK4 = false>
__device__ __forceinline__ void backward_staged_body(const BwdArgs& a, int block) {
  __shared__ float su[kBRing][3][kBYH][kBXH];
  __shared__ float sj[3][NC][kBYJ][kBXJ];
  const State* st = a.st;
  if (a.need_mode >= 0 && st->mode != a.need_mode) return;   // uniform over the grid
  const Geom g = a.g;
  const long long N = g.n;
  const uint32_t n = (uint32_t)N;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const float dt = a.dt, ih = g.inv_h;
  const float* vb = (a.vfix ? a.vfix : (st->base ? a.vB : a.vA)) +
                    (long long)(a.j >= 0 ? a.j : 0) * 3 * N;
  const rsrc_t V0 = rsrc(vb, n), V1 = rsrc(vb + N, n), V2 = rsrc(vb + 2 * N, n);
  const float* un = a.u_next;
  const rsrc_t UN = rsrc(un, 3u * n);                   // all three components
  const rsrc_t N0 = rsrc(un, n), N1 = rsrc(un + N, n), N2 = rsrc(un + 2 * N, n);
  float* uc = a.u_cur ? a.u_cur : a.b;                  // unused when !HAS_U
  const rsrc_t C0 = rsrc(uc, n), C1 = rsrc(uc + N, n), C2 = rsrc(uc + 2 * N, n);
  const rsrc_t B0 = rsrc(a.b, n), B1 = rsrc(a.b + N, n), B2 = rsrc(a.b + 2 * N, n);
  rsrc_t RR[NC], JJ[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    RR[c] = rsrc(a.r + (long long)c * N, n);
    JJ[c] = rsrc(a.J0t + (long long)c * a.cstride, n);
  }
  const SlabTile tt = slab_tile(g, block);
  const int tx = threadIdx.x % kBX, ty = threadIdx.x / kBX;
  const int x = tt.x0 + tx, y = tt.y0 + ty;
  const bool inside = x < nx && y < ny;
  MapRing mu;
  mu.s = su;
  mu.init(g, n, tt.x0, tt.y0);
  HaloRing<NC> rj;
  rj.s = sj;
  rj.init(g, tt.x0, tt.y0);
  for (int p = tt.zbeg - kBH; p < tt.zbeg + kBH; ++p) {
    mu.fetch(UN, g, p);
    mu.put(p);
  }
  rj.fetch(JJ, g, tt.zbeg - 1);
  rj.put(tt.zbeg - 1);
  rj.fetch(JJ, g, tt.zbeg);
  rj.put(tt.zbeg);

  const int lx = tx + kBH, ly = ty + kBH;                    // own position in the map window
  const int jx = tx + 1, jy = ty + 1;
  const uint32_t nxy = (uint32_t)(nx * ny);
  // Residuals sampled at x + u1(x)/h on plane zz, from the staged map (plane zz in the ring).
  auto residuals = [&](int zz, float out[NC]) {
    const int sz = zz % kBRing;
    const Cell czc = make_cell_zero(g, x, y, zz, su[sz][0][ly][lx] * ih, su[sz][1][ly][lx] * ih,
                                    su[sz][2][ly][lx] * ih);
#pragma unroll
    for (int c = 0; c < NC; ++c) out[c] = sample(RR[c], czc);
  };
  // With a map to compute, the residual samples and v of a plane are loaded one
  // step ahead, so their latency overlaps the step before; the first plane's
  // come before the march.  The last step (no map) samples in its own step.
  float rs[NC], vc[3] = {0.f, 0.f, 0.f};
  if (HAS_U) {
    __syncthreads();
    if (inside) {
      residuals(tt.zbeg, rs);
      const uint32_t i0 = (uint32_t)tt.zbeg * nxy + (uint32_t)(y * nx + x);
      vc[0] = bld(V0, i0);
      vc[1] = bld(V1, i0);
      vc[2] = bld(V2, i0);
    }
  }
  mu.fetch(UN, g, tt.zbeg + kBH);
  rj.fetch(JJ, g, tt.zbeg + 1);
  double mind = 1e300;
  for (int z = tt.zbeg; z < tt.zend; ++z) {
    mu.put(z + kBH);
    rj.put(z + 1);
    __syncthreads();
    if (z + 1 < tt.zend) {                                   // in flight during the step
      mu.fetch(UN, g, z + kBH + 1);
      rj.fetch(JJ, g, z + 2);
    }
    if (inside) {
      const uint32_t i = (uint32_t)((z * ny + y) * nx + x);
      const int s0 = z % kBRing;
      const int zn = z + 1 < tt.zend ? z + 1 : z;            // the next plane (the last: again)
      float vn[3] = {0.f, 0.f, 0.f}, rn[NC];
      if (HAS_U) {
        const uint32_t inext = i + (zn > z ? nxy : 0u);
        vn[0] = bld(V0, inext);
        vn[1] = bld(V1, inext);
        vn[2] = bld(V2, inext);
        residuals(zn, rn);
      } else {
        residuals(z, rs);
      }
      if (HAS_U) {
        float vx = vc[0], vy = vc[1], vz = vc[2];
        if (RK4) rk4_mean(V0, V1, V2, g, x, y, z, dt * ih, vx, vy, vz);
        float ux = dt * vx, uy = dt * vy, uz = dt * vz;
        int cx, cy, cz;
        float fx, fy, fz;
        cell_clamp(x, dt * vx * ih, nx, cx, fx);
        cell_clamp(y, dt * vy * ih, ny, cy, fy);
        cell_clamp(z, dt * vz * ih, nz, cz, fz);
        float gv[3];
        if (!mu.sample3(tt.x0, tt.y0, z, cx, cy, cz, fx, fy, fz, gv)) {
          const Cell cl = make_cell_clamp(g, x, y, z, dt * vx * ih, dt * vy * ih, dt * vz * ih);
          gv[0] = sample(N0, cl);
          gv[1] = sample(N1, cl);
          gv[2] = sample(N2, cl);
        }
        ux += gv[0];
        uy += gv[1];
        uz += gv[2];
        bst(C0, i, ux);
        bst(C1, i, uy);
        bst(C2, i, uz);
      }
      // Jacobian matrix I + D u of u1 at time jb (rows: component, columns: direction)
      const int sm1 = (z + kBRing - 1) % kBRing, sp1 = (z + 1) % kBRing;
      float J[3][3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float ce = su[s0][c][ly][lx];
        J[c][0] = dstencil_v(su[s0][c][ly][lx + 1], su[s0][c][ly][lx - 1], ce, x, nx, ih);
        J[c][1] = dstencil_v(su[s0][c][ly + 1][lx], su[s0][c][ly - 1][lx], ce, y, ny, ih);
        J[c][2] = dstencil_v(su[sp1][c][ly][lx], su[sm1][c][ly][lx], ce, z, nz, ih);
      }
      J[0][0] += 1.f;
      J[1][1] += 1.f;
      J[2][2] += 1.f;
      const float det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                        J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                        J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      mind = fmin(mind, (double)det);
      const int j0 = z % 3, jm = (z + 2) % 3, jp = (z + 1) % 3;
      float bx = 0.f, by = 0.f, bz = 0.f;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const float rw = a.w[c] * rs[c];
        const float ce = sj[j0][c][jy][jx];
        bx += rw * dstencil_v(sj[j0][c][jy][jx + 1], sj[j0][c][jy][jx - 1], ce, x, nx, ih);
        by += rw * dstencil_v(sj[j0][c][jy + 1][jx], sj[j0][c][jy - 1][jx], ce, y, ny, ih);
        bz += rw * dstencil_v(sj[jp][c][jy][jx], sj[jm][c][jy][jx], ce, z, nz, ih);
      }
      const float sc = a.coef * det;
      bst(B0, i, sc * bx);
      bst(B1, i, sc * by);
      bst(B2, i, sc * bz);
      if (HAS_U) {
#pragma unroll
        for (int c = 0; c < 3; ++c) vc[c] = vn[c];
#pragma unroll
        for (int c = 0; c < NC; ++c) rs[c] = rn[c];
      }
    }
    __syncthreads();
  }
  const double m = block_min(mind);
  if (threadIdx.x == 0) a.partDet[block] = m;
}

template <int NC, bool HAS_U, bool RK4>
__global__ __launch_bounds__(kBlock) void k_backward_staged(BwdArgs a) {
  backward_staged_body<NC, HAS_U, RK4>(a, blockIdx.x);
}

template <bool RK4>
static void staged_dispatch(const BwdArgs& a, bool hu, hipStream_t s) {
  const dim3 grid(backward_partials(a.g));
  if (a.nch == 2) {
    if (hu)
      hipLaunchKernelGGL((k_backward_staged<2, true, RK4>), grid, dim3(kBlock), 0, s, a);
    else
      hipLaunchKernelGGL((k_backward_staged<2, false, RK4>), grid, dim3(kBlock), 0, s, a);
  } else {
    if (hu)
      hipLaunchKernelGGL((k_backward_staged<1, true, RK4>), grid, dim3(kBlock), 0, s, a);
    else
      hipLaunchKernelGGL((k_backward_staged<1, false, RK4>), grid, dim3(kBlock), 0, s, a);
  }
}

// ------------------------------------------- forward sweep, LDS-staged ----
// The forward step with the map gather of u0_j read from LDS: a block owns a
// kBX x kBY column of (x, y) and marches up one z-slab (the tiles and slabs of
// the staged backward sweep), keeping a ring of u0_j planes z - kBH .. z + kBH
// (halo kBH, clamped) and loading one new plane per step while the step
// computes.  A gather whose cell leaves the window reads global memory.  v_j of
// the planes below, at and above the current one stays in registers (the z
// terms of the stencil); the in-plane neighbours are loads.  The template gather
// (displacements of many voxels) stays in global memory.  The per-voxel
// arithmetic is forward_voxel's with the same 8 corners in the same order, so
// all traversals give the same bits.
static int g_fwd_staged_min_blocks = 2048;

void set_fwd_staged_min_blocks(int b) { g_fwd_staged_min_blocks = b < 1 ? 1 : b; }

bool forward_staged(const Geom& g) {
  const SweepTiling t = sweep_tiling(g);
  const long long blocks = (long long)t.ntx * t.nty * t.nslab;
  return blocks >= g_fwd_staged_min_blocks && blocks <= kPartMax && 3LL * g.n < (1LL << 30);
}

int forward_staged_blocks(const Geom& g) {
  const SweepTiling t = sweep_tiling(g);
  return t.ntx * t.nty * t.nslab;
}

template <int NC>
struct StagedMapSampler {
  const MapRing& mu;
  const FwdView<NC>& f;
  const Geom& g;
  int x0, y0;
  __device__ __forceinline__ void operator()(int x, int y, int z, float dx, float dy, float dz,
                                             float out[3]) const {
    int cx, cy, cz;
    float fx, fy, fz;
    cell_clamp(x, dx, g.nx, cx, fx);
    cell_clamp(y, dy, g.ny, cy, fy);
    cell_clamp(z, dz, g.nz, cz, fz);
    if (!mu.sample3(x0, y0, z, cx, cy, cz, fx, fy, fz, out))
      GlobalMapSampler<NC>{f, g}(x, y, z, dx, dy, dz, out);
  }
};

// The template channels at (x, y, z) + d from the staged template planes
// z - 1 .. z + 1 when the cell lies in the window, else from global memory; the
// same cell, fractions and corner order either way.
template <int NC>
struct StagedTemplateSampler {
  const HaloRing<NC>& rt;
  const FwdView<NC>& f;
  const Geom& g;
  int x0, y0;
  __device__ __forceinline__ void operator()(int x, int y, int z, float dx, float dy, float dz,
                                             float out[NC]) const {
    int cx, cy, cz;
    float fx, fy, fz;
    cell_free(x, dx, g.nx, cx, fx);
    cell_free(y, dy, g.ny, cy, fy);
    cell_free(z, dz, g.nz, cz, fz);
    if (HaloRing<NC>::covers(x0, y0, z, cx, cy, cz)) {
#pragma unroll
      for (int c = 0; c < NC; ++c) out[c] = rt.lerp(c, x0, y0, cx, cy, cz, fx, fy, fz);
    } else {
      GlobalTemplateSampler<NC>{f, g}(x, y, z, dx, dy, dz, out);
    }
  }
};

template <int NC, bool FIRST, bool LAST, bool RK4>
__device__ void forward_staged_body(const FwdArgs& a, int block) {
  // v_j is staged as well: planes z and z + 1 of its periodic extension in two
  // slots, the in-plane neighbours of the 7-point stencil and its z + 1 term
  // (the z - 1 term is the previous step's centre).  The template channel is staged too in the
  // first-order steps that are not the last, with one weighted channel (the last
  // step, the RK4 steps and a second channel hold more live registers, and the
  // ring would cost a wave per SIMD).
  static_assert(kBH == 1, "the v window is the map window");
  constexpr bool TR = NC == 1 && !LAST && !RK4;
  __shared__ float su[kBRing][3][kBYH][kBXH];
  __shared__ float sv[2][3][kBYH][kBXH];
  __shared__ float stp[TR ? 3 : 1][NC][kBYJ][kBXJ];
  if (a.st->mode == MODE_STOPPED) return;                     // uniform over the grid
  const Geom g = a.g;
  const FwdView<NC> f = fwd_view<NC, LAST>(a);
  const uint32_t n = (uint32_t)g.n;
  const int nx = g.nx, ny = g.ny;
  const uint32_t nxy = (uint32_t)(nx * ny);
  const SlabTile tt = slab_tile(g, block);
  const int tx = threadIdx.x % kBX, ty = threadIdx.x / kBX;
  const int x = tt.x0 + tx, y = tt.y0 + ty;
  const bool inside = x < nx && y < ny;
  const int lx = tx + 1, ly = ty + 1;                         // own position in the windows
  MapRing mu, vr;
  mu.s = su;
  vr.s = sv;
  vr.init(g, n, tt.x0, tt.y0);
  const rsrc_t U = rsrc(a.u_cur, 3u * n);
  const float* vb = (a.st->eval ? a.vB : a.vA) + (long long)a.j * 3 * g.n;
  const rsrc_t VA = rsrc(vb, 3u * n);                         // all three components
  if (!FIRST) {
    mu.init(g, n, tt.x0, tt.y0);
    for (int q = tt.zbeg - kBH; q < tt.zbeg + kBH; ++q) {
      mu.fetch(U, g, q);
      mu.put(q);
    }
    mu.fetch(U, g, tt.zbeg + kBH);
  }
  vr.fetch_periodic(VA, g, tt.zbeg);
  vr.put2(tt.zbeg);
  vr.fetch_periodic(VA, g, tt.zbeg + 1);
  float vm[3] = {0.f, 0.f, 0.f};                              // v_j of plane z - 1 at (x, y)
  if (inside) {
    const uint32_t zb = tt.zbeg == 0 ? (uint32_t)g.nz - 1 : (uint32_t)tt.zbeg - 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) vm[c] = bld(VA, (uint32_t)c * n + zb * nxy + (uint32_t)(y * nx + x));
  }
  HaloRing<NC> rt;                                            // template planes z - 1 .. z + 1
  if constexpr (TR) {
    rt.s = stp;
    if constexpr (!FIRST)
      rt.init_from(mu);
    else
      rt.init(g, tt.x0, tt.y0);
    for (int q = tt.zbeg - 1; q <= tt.zbeg; ++q) {
      rt.fetch(f.T0, g, q);
      rt.put(q);
    }
    rt.fetch(f.T0, g, tt.zbeg + 1);
  }
  const uint32_t p = inside ? (uint32_t)(y * nx + x) : 0u;
  const StagedMapSampler<NC> ms{mu, f, g, tt.x0, tt.y0};
  double accR = 0.0, accD = 0.0, accI = 0.0;
  for (int z = tt.zbeg; z < tt.zend; ++z) {
    if (!FIRST) mu.put(z + kBH);
    vr.put2(z + 1);
    if (TR) rt.put(z + 1);
    __syncthreads();
    if (z + 1 < tt.zend) {                                    // in flight during the step
      if (!FIRST) mu.fetch(U, g, z + kBH + 1);
      vr.fetch_periodic(VA, g, z + 2);
      if (TR) rt.fetch(f.T0, g, z + 2);
    }
    if (inside) {
      const uint32_t i = (uint32_t)z * nxy + p;
      const int s0 = z & 1, sp = s0 ^ 1;
      float vc[3], lap[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        vc[c] = sv[s0][c][ly][lx];
        lap[c] = lap7_of(sv[s0][c][ly][lx - 1], sv[s0][c][ly][lx + 1], sv[s0][c][ly - 1][lx],
                         sv[s0][c][ly + 1][lx], vm[c], sv[sp][c][ly][lx], vc[c]);
      }
      if constexpr (TR)
        forward_voxel<NC, FIRST, LAST, RK4>(a, f, i, x, y, z, vc[0], vc[1], vc[2], lap[0], lap[1],
                                            lap[2], accR, accD, accI, ms,
                                            StagedTemplateSampler<NC>{rt, f, g, tt.x0, tt.y0});
      else
        forward_voxel<NC, FIRST, LAST, RK4>(a, f, i, x, y, z, vc[0], vc[1], vc[2], lap[0], lap[1],
                                            lap[2], accR, accD, accI, ms,
                                            GlobalTemplateSampler<NC>{f, g});
#pragma unroll
      for (int c = 0; c < 3; ++c) vm[c] = vc[c];
    }
    __syncthreads();
  }
  forward_partials<LAST>(a, (uint32_t)block, accR, accD, accI);
}

// Batched body-force step: every problem gets backward_partials(g) blocks and
// runs the staged body when its grid allows it.
template <int NC, bool HAS_U>
__global__ __launch_bounds__(kBlock) void k_backward_force_batched(BatchRef br, int slot) {
  const int p = batch_pair(br, blockIdx.x);
  const BwdArgs& a = ((const PairTab*)br.tab[p])->bwd[slot];
  const int tile = blockIdx.x - br.off[p];
  if (a.staged)
    backward_staged_body<NC, HAS_U>(a, tile);
  else
    backward_body<NC, HAS_U, false, true>(a, tile, br.off[p + 1] - br.off[p]);
}

void launch_forward(const FwdArgs& a, hipStream_t s) {
  if (a.rk4) {
    if (a.nch == 2)
      fwd_dispatch<2, true>(a, s);
    else
      fwd_dispatch<1, true>(a, s);
  } else {
    if (a.nch == 2)
      fwd_dispatch<2, false>(a, s);
    else
      fwd_dispatch<1, false>(a, s);
  }
}

template <int NC, bool RK4>
static void bwd_dispatch(const BwdArgs& a, hipStream_t s) {
  const int grid = reduce_grid(a.g.n);
  const bool hu = a.j >= 0, uz = (a.u_next == nullptr), hb = (a.jb >= 0 && a.jb < a.T);
  if (hu && uz && !hb)
    hipLaunchKernelGGL((k_backward<NC, true, true, false, RK4>), dim3(grid), dim3(kBlock), 0, s, a);
  else if (hu && !uz && hb)
    hipLaunchKernelGGL((k_backward<NC, true, false, true, RK4>), dim3(grid), dim3(kBlock), 0, s, a);
  else if (hu && !uz && !hb)
    hipLaunchKernelGGL((k_backward<NC, true, false, false, RK4>), dim3(grid), dim3(kBlock), 0, s, a);
  else if (!hu && hb)
    hipLaunchKernelGGL((k_backward<NC, false, false, true, RK4>), dim3(grid), dim3(kBlock), 0, s, a);
}

void launch_backward(const BwdArgs& a, hipStream_t s) {
  const bool hu = a.j >= 0, uz = (a.u_next == nullptr), hb = (a.jb >= 0 && a.jb < a.T);
  if (hb && !uz && a.staged) {
    if (a.rk4)
      staged_dispatch<true>(a, hu, s);
    else
      staged_dispatch<false>(a, hu, s);
    return;
  }
  if (a.rk4) {
    if (a.nch == 2)
      bwd_dispatch<2, true>(a, s);
    else
      bwd_dispatch<1, true>(a, s);
  } else {
    if (a.nch == 2)
      bwd_dispatch<2, false>(a, s);
    else
      bwd_dispatch<1, false>(a, s);
  }
}

// Batched sweeps: step j of every problem (same T, same channel count).
void launch_forward_batched(const BatchRef& br, int j, int T, int nch, hipStream_t s) {
  const bool first = (j == 0), last = (j == T - 1);
  const dim3 grid(br.off[br.np]);
#define FWDB(NC, F, L) \
  hipLaunchKernelGGL((k_forward_batched<NC, F, L>), grid, dim3(kBlock), 0, s, br, j)
  if (nch == 2) {
    if (first && last) FWDB(2, true, true); else if (first) FWDB(2, true, false);
    else if (last) FWDB(2, false, true); else FWDB(2, false, false);
  } else {
    if (first && last) FWDB(1, true, true); else if (first) FWDB(1, true, false);
    else if (last) FWDB(1, false, true); else FWDB(1, false, false);
  }
#undef FWDB
}

// slot = j + 1 (the table holds the T + 1 backward launches, j = T-1 .. -1)
void launch_backward_batched(const BatchRef& br, int j, int T, int nch, hipStream_t s) {
  const bool hu = j >= 0, uz = (j == T - 1), hb = (j + 1 <= T - 1);
  const dim3 grid(br.off[br.np]);
  const int slot = j + 1;
#define BWDB(NC, A, B, C) \
  hipLaunchKernelGGL((k_backward_batched<NC, A, B, C>), grid, dim3(kBlock), 0, s, br, slot)
#define BWDF(NC, A) \
  hipLaunchKernelGGL((k_backward_force_batched<NC, A>), grid, dim3(kBlock), 0, s, br, slot)
  if (nch == 2) {
    if (hu && uz && !hb) BWDB(2, true, true, false);
    else if (hu && !uz && hb) BWDF(2, true);
    else if (hu && !uz && !hb) BWDB(2, true, false, false);
    else if (!hu && hb) BWDF(2, false);
  } else {
    if (hu && uz && !hb) BWDB(1, true, true, false);
    else if (hu && !uz && hb) BWDF(1, true);
    else if (hu && !uz && !hb) BWDB(1, true, false, false);
    else if (!hu && hb) BWDF(1, false);
  }
#undef BWDB
#undef BWDF
}

// ------------------------------------------------------------ utilities ----

__global__ __launch_bounds__(kBlock) void k_crop3(const float* __restrict__ u, Geom g, int Nx,
                                                  int Ny, int Nz, float* __restrict__ out) {
  const long long N = (long long)Nx * Ny * Nz;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < 3 * N;
       i += (long long)gridDim.x * kBlock) {
    const int c = (int)(i / N);
    const long long k = i - c * N;
    const int x = (int)(k % Nx);
    const long long t = k / Nx;
    const int y = (int)(t % Ny);
    const int z = (int)(t / Ny);
    out[i] = u[c * g.n + vidx(g, x, y, z)];
  }
}

void launch_crop3(const float* u, const Geom& g, int Nx, int Ny, int Nz, float* out,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_crop3, dim3(grid1d(3LL * Nx * Ny * Nz)), dim3(kBlock), 0, s, u, g, Nx, Ny,
                     Nz, out);
}

template <typename TS>
__global__ __launch_bounds__(kBlock) void k_apply(const float* __restrict__ u, Geom g,
                                                  const TS* __restrict__ src, int interp,
                                                  TS* __restrict__ dst) {
  const long long n = g.n;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock) {
    const int x = (int)(i % g.nx);
    const long long t = i / g.nx;
    const int y = (int)(t % g.ny);
    const int z = (int)(t / g.ny);
    const float dx = u[i] * g.inv_h, dy = u[i + n] * g.inv_h, dz = u[i + 2 * n] * g.inv_h;
    if (interp == 0) {
      int cx, cy, cz;
      float fx, fy, fz;
      cell_free(x, dx, g.nx, cx, fx);
      cell_free(y, dy, g.ny, cy, fy);
      cell_free(z, dz, g.nz, cz, fz);
      dst[i] = (TS)tri_zero((const float*)src, g, cx, cy, cz, fx, fy, fz);
    } else {
      // nearest: index floor(y + 1/2) with y = i + d; rounding uses d alone
      int cx, cy, cz;
      float fx, fy, fz;
      cell_free(x, dx + 0.5f, g.nx, cx, fx);
      cell_free(y, dy + 0.5f, g.ny, cy, fy);
      cell_free(z, dz + 0.5f, g.nz, cz, fz);
      const bool ok = (unsigned)cx < (unsigned)g.nx && (unsigned)cy < (unsigned)g.ny &&
                      (unsigned)cz < (unsigned)g.nz;
      dst[i] = ok ? src[vidx(g, cx, cy, cz)] : (TS)0;
    }
  }
}

void launch_apply(const float* u, int Nx, int Ny, int Nz, float inv_h, const void* src, int interp,
                  int dtype, void* dst, hipStream_t s) {
  Geom g{};
  g.nx = Nx;
  g.ny = Ny;
  g.nz = Nz;
  g.n = (long long)Nx * Ny * Nz;
  g.inv_h = inv_h;
  g.h = 1.f / inv_h;
  if (dtype == 1)
    hipLaunchKernelGGL(k_apply<int>, dim3(grid1d(g.n)), dim3(kBlock), 0, s, u, g,
                       (const int*)src, interp, (int*)dst);
  else
    hipLaunchKernelGGL(k_apply<float>, dim3(grid1d(g.n)), dim3(kBlock), 0, s, u, g,
                       (const float*)src, interp, (float*)dst);
}

__global__ __launch_bounds__(kBlock) void k_make_mask(const float* __restrict__ img, long long n,
                                                      float tau, float* __restrict__ m,
                                                      float* __restrict__ mi) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock) {
    const float v = img[i];
    const float k = v > tau ? 1.f : 0.f;
    m[i] = k;
    if (mi) mi[i] = k * v;
  }
}

void launch_make_mask(const float* img, long long n, float tau, float* m, float* mi,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_make_mask, dim3(grid1d(n)), dim3(kBlock), 0, s, img, n, tau, m, mi);
}

__global__ __launch_bounds__(kBlock) void k_fill(float* __restrict__ p, long long n, float val) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    p[i] = val;
}

void launch_fill(float* p, long long n, float val, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(grid1d(n)), dim3(kBlock), 0, s, p, n, val);
}

// Device copy: 16-byte loads and stores when both buffers are 16-byte aligned
// (the tail, and unaligned buffers, element by element); one 16-byte element per
// thread over the whole grid (the loop only covers grids beyond the launch cap).
__global__ __launch_bounds__(kBlock) void k_copy(const float* __restrict__ a, float* __restrict__ b,
                                                 long long n) {
  const long long stride = (long long)gridDim.x * kBlock;
  const long long t0 = (long long)blockIdx.x * kBlock + threadIdx.x;
  long long done = 0;
  if ((((uintptr_t)a | (uintptr_t)b) & 15) == 0) {
    const long long n4 = n >> 2;
    const float4* __restrict__ a4 = reinterpret_cast<const float4*>(a);
    float4* __restrict__ b4 = reinterpret_cast<float4*>(b);
    for (long long i = t0; i < n4; i += stride) b4[i] = a4[i];
    done = n4 << 2;
  }
  for (long long i = done + t0; i < n; i += stride) b[i] = a[i];
}

void launch_copy(const float* src, float* dst, long long n, hipStream_t s) {
  long long blocks = (n / 4 + kBlock - 1) / kBlock;
  blocks = blocks < 1 ? 1 : (blocks > (1LL << 30) ? (1LL << 30) : blocks);
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(kBlock), 0, s, src, dst, n);
}

}  // namespace lddmm
