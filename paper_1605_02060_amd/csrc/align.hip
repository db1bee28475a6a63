// Rigid and affine pre-alignment (Methods, Registration): gradient descent on
// the mean squared error between the template image sampled through an affine
// sampling map S (x = B y + c, physical coordinates, S = R^-1 or R^-1 A^-1) and
// the target image, and the resampling src(S(y + u(y))) that composes the
// alignment with a deformation (phi^-1 = R^-1 A^-1 phi_10).
//
// One descent slot is two launches, so the whole descent runs without a host
// synchronisation:
//   k_align_partials  one pass over the target voxels: each samples the
//                     template at the candidate's S(y) (8 taps, zero outside),
//                     the residual and the exact derivative of the trilinear
//                     interpolant, and accumulates the MSE and its 12 gradient
//                     sums in FP64; per-block partials;
//   k_align_control   one block: totals, the accept / halve guard against the
//                     current iterate, the trace row, and the next candidate
//                     (rigid: B exp(-eps [w]_x) by Rodrigues' formula, so B
//                     stays a rotation; affine: B - eps G_B) in FP64.
// The sampling positions are FP64, evaluated as (B y + c) / h without
// multiply-add fusion (this file is compiled with -ffp-contract=off), and the
// trilinear weights FP32, as in the deformation's samplers.
#include <cfloat>
#include <cmath>

#include "internal.h"
#include "lddmm.h"

namespace lddmm {
namespace {

constexpr int kWaves = kBlock / 64;
constexpr int kParts = 13;              // MSE sum, r g_d p_e (9), r g_d (3)
constexpr int kAlignBlocksMax = 2048;

struct AlignGeom {
  int nx0, ny0, nz0;                    // template grid
  int nx1, ny1, nz1;                    // target grid
  long long n1;                         // < 2^30 (each axis at most LDDMM_MAX_DIM)
  FastDiv fx1, fy1;                     // division by nx1, ny1
  double h0, h1;
  double yc[3];                         // target centre (physical)
  double rho2;                          // mean squared distance of target voxels from yc
};

struct AlignState {
  double S[12];                         // current iterate [B | c], 3 x 4 row-major
  double G[12];                         // its gradient: G_B (3 x 3 row-major), G_c'
  double Sc[12];                        // candidate evaluated by the next partials pass
  double E;                             // MSE of the current iterate
  double eps;                           // translation step
  int halvings;
  int stopped;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline int align_blocks(long long n) {
  long long b = (n + (long long)kBlock * 8 - 1) / ((long long)kBlock * 8);
  b = (b + kXCD - 1) / kXCD * kXCD;
  if (b < kXCD) b = kXCD;
  if (b > kAlignBlocksMax) b = kAlignBlocksMax;
  return (int)b;
}

inline size_t align_state_offset(int nblk) {
  return align256(sizeof(double) * kParts * (size_t)nblk);
}

// Zero-outside trilinear sample of f at index position q, with its index-space
// derivative (cell floor(q), the derivative of the interpolant inside it).
__device__ __forceinline__ void sample_grad(const float* __restrict__ f, int nx, int ny, int nz,
                                            double qx, double qy, double qz, float& v, float& gx,
                                            float& gy, float& gz) {
  const double cxd = floor(qx), cyd = floor(qy), czd = floor(qz);
  v = gx = gy = gz = 0.f;
  if (cxd < -1.0 || cyd < -1.0 || czd < -1.0 || cxd > (double)(nx - 1) ||
      cyd > (double)(ny - 1) || czd > (double)(nz - 1))
    return;
  const int cx = (int)cxd, cy = (int)cyd, cz = (int)czd;
  const float fx = (float)(qx - cxd), fy = (float)(qy - cyd), fz = (float)(qz - czd);
  // corner validity per axis; 32-bit offsets (every grid has fewer than 2^30 voxels)
  const bool vx[2] = {cx >= 0, cx + 1 < nx}, vy[2] = {cy >= 0, cy + 1 < ny},
             vz[2] = {cz >= 0, cz + 1 < nz};
  const int base = (cz * ny + cy) * nx + cx, sy = nx, sz = nx * ny;
  float t[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int bx = k & 1, by = (k >> 1) & 1, bz = k >> 2;
    t[k] = (vx[bx] && vy[by] && vz[bz]) ? f[base + bx + by * sy + bz * sz] : 0.f;
  }
  const float ex = 1.f - fx, ey = 1.f - fy, ez = 1.f - fz;
  v = ez * (ey * (ex * t[0] + fx * t[1]) + fy * (ex * t[2] + fx * t[3])) +
      fz * (ey * (ex * t[4] + fx * t[5]) + fy * (ex * t[6] + fx * t[7]));
  gx = ez * (ey * (t[1] - t[0]) + fy * (t[3] - t[2])) + fz * (ey * (t[5] - t[4]) + fy * (t[7] - t[6]));
  gy = ez * (ex * (t[2] - t[0]) + fx * (t[3] - t[1])) + fz * (ex * (t[6] - t[4]) + fx * (t[7] - t[5]));
  gz = ey * (ex * (t[4] - t[0]) + fx * (t[5] - t[1])) + fy * (ex * (t[6] - t[2]) + fx * (t[7] - t[3]));
}

__device__ __forceinline__ double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

__global__ void k_align_init(const double* __restrict__ S0, double step,
                             AlignState* __restrict__ st) {
  if (threadIdx.x < 12) {
    st->S[threadIdx.x] = S0[threadIdx.x];
    st->Sc[threadIdx.x] = S0[threadIdx.x];
    st->G[threadIdx.x] = 0.0;
  }
  if (threadIdx.x == 0) {
    st->E = INFINITY;
    st->eps = step;
    st->halvings = 0;
    st->stopped = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_align_partials(AlignGeom g, const float* __restrict__ I0,
                                                           const float* __restrict__ I1,
                                                           const AlignState* __restrict__ st,
                                                           double* __restrict__ part) {
  if (st->stopped) return;
  const double* S = st->Sc;
  const double B00 = S[0], B01 = S[1], B02 = S[2], C0 = S[3];
  const double B10 = S[4], B11 = S[5], B12 = S[6], C1 = S[7];
  const double B20 = S[8], B21 = S[9], B22 = S[10], C2 = S[11];
  const double ih0 = 1.0 / g.h0;
  double acc[kParts];
#pragma unroll
  for (int k = 0; k < kParts; ++k) acc[k] = 0.0;
  const uint32_t stride = gridDim.x * kBlock;
  const uint32_t n1 = (uint32_t)g.n1;
  // two voxels per iteration (the second a grid stride further), so that both
  // voxels' gathers are in flight together; a second voxel past the end repeats
  // the first with zero weight
  for (uint32_t i0 = blockIdx.x * kBlock + threadIdx.x; i0 < n1; i0 += 2 * stride) {
    const uint32_t i1 = i0 + stride < n1 ? i0 + stride : i0;
    const double w1 = i0 + stride < n1 ? 1.0 : 0.0;
    double q[2][3], p[2][3];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const uint32_t i = u ? i1 : i0;
      const uint32_t t = fdiv(i, g.fx1), z = fdiv(t, g.fy1);
      const int x = (int)(i - t * (uint32_t)g.nx1), y = (int)(t - z * (uint32_t)g.ny1);
      // template index position (B y + c) / h0, in the definition's order of
      // operations (no multiply-add fusion in this file): positions that are
      // whole numbers stay whole, so the cell, and the one-sided derivative on
      // a cell face, are the definition's
      const double yx = g.h1 * x, yy = g.h1 * y, yz = g.h1 * z;
      q[u][0] = (B00 * yx + B01 * yy + B02 * yz + C0) / g.h0;
      q[u][1] = (B10 * yx + B11 * yy + B12 * yz + C1) / g.h0;
      q[u][2] = (B20 * yx + B21 * yy + B22 * yz + C2) / g.h0;
      p[u][0] = yx - g.yc[0];
      p[u][1] = yy - g.yc[1];
      p[u][2] = yz - g.yc[2];
    }
    float v[2], gx[2], gy[2], gz[2];
    sample_grad(I0, g.nx0, g.ny0, g.nz0, q[0][0], q[0][1], q[0][2], v[0], gx[0], gy[0], gz[0]);
    sample_grad(I0, g.nx0, g.ny0, g.nz0, q[1][0], q[1][1], q[1][2], v[1], gx[1], gy[1], gz[1]);
    const float t0 = I1[i0], t1 = I1[i1];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const double r = (double)(v[u] - (u ? t1 : t0)) * (u ? w1 : 1.0);
      acc[0] += r * r;
      const double rg[3] = {r * gx[u] * ih0, r * gy[u] * ih0, r * gz[u] * ih0};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        acc[1 + 3 * d] += rg[d] * p[u][0];
        acc[2 + 3 * d] += rg[d] * p[u][1];
        acc[3 + 3 * d] += rg[d] * p[u][2];
        acc[10 + d] += rg[d];
      }
    }
  }
  __shared__ double red[kWaves][kParts];
#pragma unroll
  for (int k = 0; k < kParts; ++k) {
    const double s = wave_sum(acc[k]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < kParts) {
    double s = 0.0;
    for (int w = 0; w < kWaves; ++w) s += red[w][threadIdx.x];
    part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

__device__ void rodrigues(const double w[3], double R[9]) {
  const double t2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  double a, b;
  if (t2 < 1e-12) {
    a = 1.0 - t2 / 6.0;
    b = 0.5 - t2 / 24.0;
  } else {
    const double t = sqrt(t2);
    a = sin(t) / t;
    b = (1.0 - cos(t)) / t2;
  }
  const double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double k2 = 0.0;
      for (int l = 0; l < 3; ++l) k2 += K[i * 3 + l] * K[l * 3 + j];
      R[i * 3 + j] = (i == j ? 1.0 : 0.0) + a * K[i * 3 + j] + b * k2;
    }
}

// Next candidate from the current iterate S with gradient G and steps eps_t, eps_l.
__device__ void make_candidate(const double S[12], const double G[12], double eps_t, double eps_l,
                               int mode, const double yc[3], double out[12]) {
  double B[9], cp[3];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) B[i * 3 + j] = S[i * 4 + j];
    cp[i] = B[i * 3] * yc[0] + B[i * 3 + 1] * yc[1] + B[i * 3 + 2] * yc[2] + S[i * 4 + 3];
  }
  double Bn[9];
  if (mode == LDDMM_ALIGN_RIGID) {
    // w_k = <G_B, B [e_k]_x>: the derivative of the MSE along B exp(t [e_k]_x)
    double w[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 3; ++i) {
      const double* Gi = G + i * 3;
      const double* Bi = B + i * 3;
      w[0] += Gi[1] * Bi[2] - Gi[2] * Bi[1];
      w[1] += Gi[2] * Bi[0] - Gi[0] * Bi[2];
      w[2] += Gi[0] * Bi[1] - Gi[1] * Bi[0];
    }
    const double mw[3] = {-eps_l * w[0], -eps_l * w[1], -eps_l * w[2]};
    double R[9];
    rodrigues(mw, R);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        Bn[i * 3 + j] = B[i * 3] * R[j] + B[i * 3 + 1] * R[3 + j] + B[i * 3 + 2] * R[6 + j];
  } else {
    for (int k = 0; k < 9; ++k) Bn[k] = B[k] - eps_l * G[k];
  }
  for (int i = 0; i < 3; ++i) {
    const double cpn = cp[i] - eps_t * G[9 + i];
    for (int j = 0; j < 3; ++j) out[i * 4 + j] = Bn[i * 3 + j];
    out[i * 4 + 3] = cpn - (Bn[i * 3] * yc[0] + Bn[i * 3 + 1] * yc[1] + Bn[i * 3 + 2] * yc[2]);
  }
}

__global__ __launch_bounds__(kBlock) void k_align_control(const double* __restrict__ part, int nblk,
                                                          AlignGeom g, AlignState* __restrict__ st,
                                                          int mode, int slot, int max_halvings,
                                                          double* __restrict__ trace) {
  if (st->stopped) return;
  double loc[kParts];
#pragma unroll
  for (int k = 0; k < kParts; ++k) loc[k] = 0.0;
  for (int j = threadIdx.x; j < nblk; j += kBlock)
#pragma unroll
    for (int k = 0; k < kParts; ++k) loc[k] += part[(size_t)k * nblk + j];
  __shared__ double red[kWaves][kParts];
#pragma unroll
  for (int k = 0; k < kParts; ++k) {
    const double s = wave_sum(loc[k]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double tot[kParts];
  for (int k = 0; k < kParts; ++k) {
    tot[k] = 0.0;
    for (int w = 0; w < kWaves; ++w) tot[k] += red[w][k];
  }
  const double n = (double)g.n1;
  const double E = tot[0] / n;
  double G[12];
  for (int k = 0; k < 12; ++k) G[k] = 2.0 * tot[1 + k] / n;
  double used = st->eps, accepted = 1.0;
  if (slot == 0) {
    st->E = E;
    for (int k = 0; k < 12; ++k) st->G[k] = G[k];
  } else if (E <= st->E) {
    st->E = E;
    for (int k = 0; k < 12; ++k) {
      st->S[k] = st->Sc[k];
      st->G[k] = G[k];
    }
    st->halvings = 0;
  } else {
    st->eps = 0.5 * st->eps;
    st->halvings += 1;
    accepted = 0.0;
  }
  if (trace) {
    double* row = trace + (size_t)slot * LDDMM_ALIGN_TRACE_COLS;
    row[0] = E;
    row[1] = used;
    row[2] = accepted;
    row[3] = (double)st->halvings;
    for (int k = 0; k < 12; ++k) row[4 + k] = st->S[k];
    for (int k = 0; k < 12; ++k) row[16 + k] = st->G[k];
  }
  if (st->halvings > max_halvings) {
    st->stopped = 1;
    return;
  }
  double Sc[12];
  make_candidate(st->S, st->G, st->eps, st->eps / g.rho2, mode, g.yc, Sc);
  for (int k = 0; k < 12; ++k) st->Sc[k] = Sc[k];
}

__global__ void k_align_finish(const AlignState* __restrict__ st, double* __restrict__ S_out) {
  if (threadIdx.x < 12) S_out[threadIdx.x] = st->S[threadIdx.x];
}

struct ApplyAffArgs {
  int nx, ny, nz;                       // destination grid
  long long n;                          // < 2^30
  FastDiv fx, fy;                       // division by nx, ny
  double hd;
  const float* u;                       // [3][n] physical displacement or null
  const double* S;                      // [12]
  int snx, sny, snz;                    // source grid
  double hs;
  const void* src;
  int interp, dtype;
  void* dst;
};

__global__ __launch_bounds__(kBlock) void k_apply_affine(ApplyAffArgs a) {
  const double B00 = a.S[0], B01 = a.S[1], B02 = a.S[2], C0 = a.S[3];
  const double B10 = a.S[4], B11 = a.S[5], B12 = a.S[6], C1 = a.S[7];
  const double B20 = a.S[8], B21 = a.S[9], B22 = a.S[10], C2 = a.S[11];
  const uint32_t stride = gridDim.x * kBlock;
  const uint32_t n = (uint32_t)a.n;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const uint32_t t = fdiv(i, a.fx), z = fdiv(t, a.fy);
    const int x = (int)(i - t * (uint32_t)a.nx), y = (int)(t - z * (uint32_t)a.ny);
    double yx = a.hd * x, yy = a.hd * y, yz = a.hd * z;
    if (a.u) {
      yx += (double)a.u[i];
      yy += (double)a.u[a.n + i];
      yz += (double)a.u[2 * a.n + i];
    }
    const double qx = (B00 * yx + B01 * yy + B02 * yz + C0) / a.hs;
    const double qy = (B10 * yx + B11 * yy + B12 * yz + C1) / a.hs;
    const double qz = (B20 * yx + B21 * yy + B22 * yz + C2) / a.hs;
    if (a.interp == LDDMM_INTERP_LINEAR) {
      float v, gx, gy, gz;
      sample_grad(static_cast<const float*>(a.src), a.snx, a.sny, a.snz, qx, qy, qz, v, gx, gy,
                  gz);
      static_cast<float*>(a.dst)[i] = v;
    } else {
      const double rx = floor(qx + 0.5), ry = floor(qy + 0.5), rz = floor(qz + 0.5);
      const bool ok = rx >= 0.0 && rx < (double)a.snx && ry >= 0.0 && ry < (double)a.sny &&
                      rz >= 0.0 && rz < (double)a.snz;
      const long long j = ok ? ((long long)rz * a.sny + (long long)ry) * a.snx + (long long)rx : 0;
      if (a.dtype == LDDMM_I32)
        static_cast<int32_t*>(a.dst)[i] = ok ? static_cast<const int32_t*>(a.src)[j] : 0;
      else
        static_cast<float*>(a.dst)[i] = ok ? static_cast<const float*>(a.src)[j] : 0.f;
    }
  }
}

inline long long grid_voxels(const lddmm_grid* g) {
  if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nx > LDDMM_MAX_DIM ||
      g->ny > LDDMM_MAX_DIM || g->nz > LDDMM_MAX_DIM || !(g->spacing > 0.0) ||
      !std::isfinite(g->spacing))
    return -1;
  return (long long)g->nx * g->ny * g->nz;
}

AlignGeom make_align_geom(const lddmm_grid* t0, const lddmm_grid* t1) {
  AlignGeom g;
  g.nx0 = t0->nx;
  g.ny0 = t0->ny;
  g.nz0 = t0->nz;
  g.nx1 = t1->nx;
  g.ny1 = t1->ny;
  g.nz1 = t1->nz;
  g.n1 = (long long)t1->nx * t1->ny * t1->nz;
  g.fx1 = make_fastdiv((uint32_t)t1->nx);
  g.fy1 = make_fastdiv((uint32_t)t1->ny);
  g.h0 = t0->spacing;
  g.h1 = t1->spacing;
  g.yc[0] = 0.5 * t1->spacing * (t1->nx - 1);
  g.yc[1] = 0.5 * t1->spacing * (t1->ny - 1);
  g.yc[2] = 0.5 * t1->spacing * (t1->nz - 1);
  g.rho2 = 0.0;
  for (int n : {t1->nx, t1->ny, t1->nz})
    g.rho2 += t1->spacing * t1->spacing * ((double)n * n - 1.0) / 12.0;
  return g;
}

int launch_status() {
  return hipGetLastError() == hipSuccess ? LDDMM_OK : LDDMM_EHIP;
}

}  // namespace
}  // namespace lddmm

using namespace lddmm;

extern "C" {

size_t lddmm_align_workspace_size(const lddmm_grid* target_grid) {
  const long long n1 = grid_voxels(target_grid);
  if (n1 < 0) return 0;
  const int nblk = align_blocks(n1);
  return align_state_offset(nblk) + align256(sizeof(AlignState));
}

int lddmm_align(const lddmm_grid* template_grid, const float* template_image,
                const lddmm_grid* target_grid, const float* target_image,
                const lddmm_align_params* params, double* affine, double* trace, void* workspace,
                size_t workspace_bytes, void* stream) {
  const long long n0 = grid_voxels(template_grid), n1 = grid_voxels(target_grid);
  if (n0 < 0 || n1 < 0 || !template_image || !target_image || !params || !affine || !workspace)
    return LDDMM_EINVAL;
  if (params->mode != LDDMM_ALIGN_RIGID && params->mode != LDDMM_ALIGN_AFFINE) return LDDMM_EINVAL;
  if (n1 < 2 || params->iters < 0 || params->max_halvings < 0 || !(params->step > 0.0) ||
      !std::isfinite(params->step))
    return LDDMM_EINVAL;
  if (workspace_bytes < lddmm_align_workspace_size(target_grid)) return LDDMM_EINVAL;
  const int nblk = align_blocks(n1);
  char* ws = static_cast<char*>(workspace);
  double* part = reinterpret_cast<double*>(ws);
  AlignState* st = reinterpret_cast<AlignState*>(ws + align_state_offset(nblk));
  const AlignGeom g = make_align_geom(template_grid, target_grid);
  hipStream_t s = (hipStream_t)stream;
  (void)hipGetLastError();   // clear an earlier error: the status returned is these launches'
  hipLaunchKernelGGL(k_align_init, dim3(1), dim3(64), 0, s, affine, params->step, st);
  for (int slot = 0; slot <= params->iters; ++slot) {
    {
      ProfScope ps(LDDMM_PROF_ALIGN, n1, s);
      hipLaunchKernelGGL(k_align_partials, dim3(nblk), dim3(kBlock), 0, s, g, template_image,
                         target_image, st, part);
    }
    hipLaunchKernelGGL(k_align_control, dim3(1), dim3(kBlock), 0, s, part, nblk, g, st,
                       (int)params->mode, slot, (int)params->max_halvings, trace);
  }
  hipLaunchKernelGGL(k_align_finish, dim3(1), dim3(64), 0, s, st, affine);
  return launch_status();
}

int lddmm_apply_affine(const lddmm_grid* dst_grid, const float* u, const double* affine,
                       const lddmm_grid* src_grid, const void* src, int32_t interp, int32_t dtype,
                       void* dst, void* stream) {
  const long long nd = grid_voxels(dst_grid), ns = grid_voxels(src_grid);
  if (nd < 0 || ns < 0 || !affine || !src || !dst) return LDDMM_EINVAL;
  if (interp != LDDMM_INTERP_LINEAR && interp != LDDMM_INTERP_NEAREST) return LDDMM_EINVAL;
  if (dtype != LDDMM_F32 && dtype != LDDMM_I32) return LDDMM_EINVAL;
  if (interp == LDDMM_INTERP_LINEAR && dtype != LDDMM_F32) return LDDMM_EINVAL;
  ApplyAffArgs a;
  a.nx = dst_grid->nx;
  a.ny = dst_grid->ny;
  a.nz = dst_grid->nz;
  a.n = nd;
  a.fx = make_fastdiv((uint32_t)dst_grid->nx);
  a.fy = make_fastdiv((uint32_t)dst_grid->ny);
  a.hd = dst_grid->spacing;
  a.u = u;
  a.S = affine;
  a.snx = src_grid->nx;
  a.sny = src_grid->ny;
  a.snz = src_grid->nz;
  a.hs = src_grid->spacing;
  a.src = src;
  a.interp = interp;
  a.dtype = dtype;
  a.dst = dst;
  long long blocks = (nd + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  (void)hipGetLastError();   // clear an earlier error: the status returned is these launches'
  hipLaunchKernelGGL(k_apply_affine, dim3((unsigned)blocks), dim3(kBlock), 0, (hipStream_t)stream,
                     a);
  return launch_status();
}

}  // extern "C"
