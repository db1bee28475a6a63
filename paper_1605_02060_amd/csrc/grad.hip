// Exact gradient of the discrete energy (reverse mode through the forward sweep).
//
// Forward sweep (Methods, Registration, semi-Lagrangian reading):
//   u_{j+1}(x) = -dt v_j(x) + S_clamp(u_j; y_j(x)),   y_j(x) = x - dt v_j(x)/h,
//   E = R(v) + (h^3/sigma^2) sum_c w_c sum_x (S_zero(J0c; x + u_T/h) - J1c)^2.
// Reverse sweep, with ubar_j = dE/du_j:
//   ubar_T  = (2 h^3/sigma^2) sum_c w_c r_c (1/h) grad_y S_zero(J0c; y)|_{y = x + u_T/h}
//   vbar_j  = -dt ubar_{j+1} - (dt/h) (d_y S_clamp(u_j; y_j))^T ubar_{j+1}
//   ubar_j  = S_clamp(.; y_j)^T ubar_{j+1}                       (adjoint of sampling)
//   dE/dv_j = vbar_j + 2 dt h^3 L(L v_j),   L = gamma - alpha Lap (periodic).
// The adjoint of sampling is evaluated as a gather: output voxel z sums the
// contributions of every source x whose clamped cell has z as a corner.  With
// |dt v/h| < Rr along every axis those sources satisfy |x - z| <= Rr, so the
// sum is over a (2 Rr + 1)^3 neighbourhood in a fixed order: deterministic.
#include "device.h"

namespace lddmm {

static inline unsigned grid_for(long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

// ----------------------------------------------------------- d/dy of samplers

// Trilinear interpolant and its derivatives at a cell (corners loaded by caller).
struct TriD {
  float d[3];
};

__device__ __forceinline__ TriD tri_deriv(float v000, float v100, float v010, float v110,
                                          float v001, float v101, float v011, float v111,
                                          float fx, float fy, float fz) {
  const float gx = 1.f - fx, gy = 1.f - fy, gz = 1.f - fz;
  TriD t;
  t.d[0] = gy * gz * (v100 - v000) + fy * gz * (v110 - v010) + gy * fz * (v101 - v001) +
           fy * fz * (v111 - v011);
  t.d[1] = gx * gz * (v010 - v000) + fx * gz * (v110 - v100) + gx * fz * (v011 - v001) +
           fx * fz * (v111 - v101);
  t.d[2] = gx * gy * (v001 - v000) + fx * gy * (v101 - v100) + gx * fy * (v011 - v010) +
           fx * fy * (v111 - v110);
  return t;
}

__device__ __forceinline__ TriD tri_deriv_cell(rsrc_t r, const Cell& c) {
  return tri_deriv(bld(r, c.o[0]), bld(r, c.o[1]), bld(r, c.o[2]), bld(r, c.o[3]), bld(r, c.o[4]),
                   bld(r, c.o[5]), bld(r, c.o[6]), bld(r, c.o[7]), c.fx, c.fy, c.fz);
}

// Axis clamped?  (y outside [0, n-1]; the derivative along it is zero.)
__device__ __forceinline__ bool clamped(int i, float d, int n) {
  d = fminf(fmaxf(d, -(float)(n + 2)), (float)(n + 2));
  const float y = (float)i + d;
  return y < 0.f || y > (float)(n - 1);
}

// ------------------------------------------------------------------ kernels

constexpr int kSplatMaxR = 3;

// ubar_T = coef * sum_c w_c r_c (1/h) grad_y S_zero(J0c; x + u_T/h)
template <int NC>
__global__ __launch_bounds__(kBlock) void k_ubar_init(GradArgs a) {
  const Geom g = a.g;
  const long long N = g.n;
  const uint32_t n = (uint32_t)N;
  const rsrc_t U0 = rsrc(a.u, n), U1 = rsrc(a.u + N, n), U2 = rsrc(a.u + 2 * N, n);
  const rsrc_t O0 = rsrc(a.ub_out, n), O1 = rsrc(a.ub_out + N, n), O2 = rsrc(a.ub_out + 2 * N, n);
  rsrc_t T0[NC], RR[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    T0[c] = rsrc(a.J0 + (long long)a.ch[c] * N, n);
    RR[c] = rsrc(a.r + (long long)c * N, n);
  }
  const float ih = g.inv_h;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    int x, y, z;
    vcoord(g, i, x, y, z);
    const Cell cz = make_cell_zero(g, x, y, z, bld(U0, i) * ih, bld(U1, i) * ih, bld(U2, i) * ih);
    float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const TriD t = tri_deriv_cell(T0[c], cz);
      const float s = a.coef * a.wc[c] * bld(RR[c], i) * ih;
      gx += s * t.d[0];
      gy += s * t.d[1];
      gz += s * t.d[2];
    }
    bst(O0, i, gx);
    bst(O1, i, gy);
    bst(O2, i, gz);
  }
}

// w = L v_j (periodic 7-point Laplacian)
__global__ __launch_bounds__(kBlock) void k_Lv(GradArgs a) {
  const Geom g = a.g;
  const long long N = g.n;
  const uint32_t n = (uint32_t)N;
  const float c2 = a.alpha * g.inv_h * g.inv_h;
  for (int c = 0; c < 3; ++c) {
    const rsrc_t V = rsrc(a.v + c * N, n), W = rsrc(a.w + c * N, n);
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
      int x, y, z;
      vcoord(g, i, x, y, z);
      const Nbr nb = periodic_nbr(g, i, x, y, z);
      const float v0 = bld(V, i);
      bst(W, i, a.gamma * v0 - c2 * lap7_b(V, nb, v0));
    }
  }
}

// dE/dv_j = -dt ubar - (dt/h) (d_y S_clamp(u_j; y_j))^T ubar + reg * L w
__global__ __launch_bounds__(kBlock) void k_coord_grad(GradArgs a) {
  const Geom g = a.g;
  const long long N = g.n;
  const uint32_t n = (uint32_t)N;
  const rsrc_t V0 = rsrc(a.v, n), V1 = rsrc(a.v + N, n), V2 = rsrc(a.v + 2 * N, n);
  const rsrc_t U0 = rsrc(a.u, n), U1 = rsrc(a.u + N, n), U2 = rsrc(a.u + 2 * N, n);
  const rsrc_t B0 = rsrc(a.ub_in, n), B1 = rsrc(a.ub_in + N, n), B2 = rsrc(a.ub_in + 2 * N, n);
  const rsrc_t W0 = rsrc(a.w, n), W1 = rsrc(a.w + N, n), W2 = rsrc(a.w + 2 * N, n);
  const rsrc_t G0 = rsrc(a.grad, n), G1 = rsrc(a.grad + N, n), G2 = rsrc(a.grad + 2 * N, n);
  const float dt = a.dt, ih = g.inv_h;
  const float c2 = a.alpha * ih * ih;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    int x, y, z;
    vcoord(g, i, x, y, z);
    const float dx = -dt * bld(V0, i) * ih, dy = -dt * bld(V1, i) * ih, dz = -dt * bld(V2, i) * ih;
    const Cell cl = make_cell_clamp(g, x, y, z, dx, dy, dz);
    const bool kx = clamped(x, dx, g.nx), ky = clamped(y, dy, g.ny), kz = clamped(z, dz, g.nz);
    const float b0 = bld(B0, i), b1 = bld(B1, i), b2 = bld(B2, i);
    // J[a][b] = d S(u_j[a]) / d y_b ; vbar_b = -dt ub_b - (dt/h) sum_a J[a][b] ub_a
    const TriD t0 = tri_deriv_cell(U0, cl), t1 = tri_deriv_cell(U1, cl), t2 = tri_deriv_cell(U2, cl);
    float vb[3];
    const float bb[3] = {b0, b1, b2};
    const bool kc[3] = {kx, ky, kz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float jt = kc[d] ? 0.f : (t0.d[d] * b0 + t1.d[d] * b1 + t2.d[d] * b2);
      vb[d] = -dt * bb[d] - dt * ih * jt;
    }
    const Nbr nb = periodic_nbr(g, i, x, y, z);
    const float w0 = bld(W0, i), w1 = bld(W1, i), w2 = bld(W2, i);
    bst(G0, i, vb[0] + a.reg * (a.gamma * w0 - c2 * lap7_b(W0, nb, w0)));
    bst(G1, i, vb[1] + a.reg * (a.gamma * w1 - c2 * lap7_b(W1, nb, w1)));
    bst(G2, i, vb[2] + a.reg * (a.gamma * w2 - c2 * lap7_b(W2, nb, w2)));
  }
}

// ubar_j(z) = sum over sources x with z a corner of x's clamped cell of weight * ubar_{j+1}(x)
__global__ __launch_bounds__(kBlock) void k_splat(GradArgs a) {
  const Geom g = a.g;
  const long long N = g.n;
  const uint32_t n = (uint32_t)N;
  const rsrc_t V0 = rsrc(a.v, n), V1 = rsrc(a.v + N, n), V2 = rsrc(a.v + 2 * N, n);
  const rsrc_t B0 = rsrc(a.ub_in, n), B1 = rsrc(a.ub_in + N, n), B2 = rsrc(a.ub_in + 2 * N, n);
  const rsrc_t O0 = rsrc(a.ub_out, n), O1 = rsrc(a.ub_out + N, n), O2 = rsrc(a.ub_out + 2 * N, n);
  int Rr = *a.radius;
  if (Rr > kSplatMaxR) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.overflow = 1;
    Rr = kSplatMaxR;
  }
  const float dt = a.dt, ih = g.inv_h;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    int zx, zy, zz;
    vcoord(g, i, zx, zy, zz);
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
    for (int oz = -Rr; oz <= Rr; ++oz) {
      const int sz = zz + oz;
      if (sz < 0 || sz >= g.nz) continue;
      for (int oy = -Rr; oy <= Rr; ++oy) {
        const int sy = zy + oy;
        if (sy < 0 || sy >= g.ny) continue;
        for (int ox = -Rr; ox <= Rr; ++ox) {
          const int sx = zx + ox;
          if (sx < 0 || sx >= g.nx) continue;
          const uint32_t src = vidx(g, sx, sy, sz);
          int cx, cy, cz;
          float fx, fy, fz;
          cell_clamp(sx, -dt * bld(V0, src) * ih, g.nx, cx, fx);
          cell_clamp(sy, -dt * bld(V1, src) * ih, g.ny, cy, fy);
          cell_clamp(sz, -dt * bld(V2, src) * ih, g.nz, cz, fz);
          const int ex = zx - cx, ey = zy - cy, ez = zz - cz;
          if ((unsigned)ex > 1u || (unsigned)ey > 1u || (unsigned)ez > 1u) continue;
          const float w = (ex ? fx : 1.f - fx) * (ey ? fy : 1.f - fy) * (ez ? fz : 1.f - fz);
          s0 += w * bld(B0, src);
          s1 += w * bld(B1, src);
          s2 += w * bld(B2, src);
        }
      }
    }
    bst(O0, i, s0);
    bst(O1, i, s1);
    bst(O2, i, s2);
  }
}

// Splat radius of step j: Rr = floor(max_x max_axis |dt v_j / h|) + 1, as a device int.
__global__ __launch_bounds__(1024) void k_radius(const float* v, long long N, float scale,
                                                 int* radius) {
  __shared__ float red[1024];
  float m = 0.f;
  for (long long i = threadIdx.x; i < 3 * N; i += blockDim.x) m = fmaxf(m, fabsf(v[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float d = red[0] * scale;
    *radius = (d == d) ? (int)floorf(fminf(d, 1e6f)) + 1 : kSplatMaxR + 1;
  }
}

// ------------------------------------------------------------ launchers

void launch_ubar_init(const GradArgs& a, hipStream_t s) {
  if (a.nch == 2)
    hipLaunchKernelGGL(k_ubar_init<2>, dim3(grid_for(a.g.n)), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_ubar_init<1>, dim3(grid_for(a.g.n)), dim3(kBlock), 0, s, a);
}

void launch_grad_step(const GradArgs& a, hipStream_t s) {
  const unsigned gb = grid_for(a.g.n);
  hipLaunchKernelGGL(k_radius, dim3(1), dim3(1024), 0, s, a.v, a.g.n, a.dt * a.g.inv_h,
                     (int*)a.radius);
  hipLaunchKernelGGL(k_Lv, dim3(gb), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_coord_grad, dim3(gb), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_splat, dim3(gb), dim3(kBlock), 0, s, a);
}

}  // namespace lddmm
