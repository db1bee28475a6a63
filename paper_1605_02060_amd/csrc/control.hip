// Device-side control of gradient descent: energy reductions, the step guard
// and the trace.  Keeping the accept/reject decision on the device lets the
// host enqueue a whole level without synchronising.
#include "device.h"

namespace lddmm {

__global__ void k_level_begin(State* st, double step, int keep_flags) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->mode = (keep_flags && st->nonfinite) ? MODE_STOPPED : MODE_INIT;
  st->base = 0;
  st->eval = 0;
  st->halvings = 0;
  if (!keep_flags) {
    st->row = 0;
    st->stopped_any = 0;
    st->nonfinite = 0;
    st->min_det_final = 1e300;
  }
  st->eps = step;
  st->step0 = step;
  st->min_det = __longlong_as_double(0x7ff8000000000000LL);   // NaN until a gradient is taken
}

void launch_level_begin(State* st, double step, int keep_flags, hipStream_t s) {
  hipLaunchKernelGGL(k_level_begin, dim3(1), dim3(64), 0, s, st, step, keep_flags);
}

// Three sums over one 1024-thread block at once (per-thread values in, totals out
// in every thread): a fixed shuffle tree within each wavefront, then the 16
// wavefront sums in order; red holds at least 3 x 16 doubles.
__device__ void block1024_sum3(double& a, double& b, double& c, double* red) {
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
    c += __shfl_down(c, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) {
    red[wid] = a;
    red[16 + wid] = b;
    red[32 + wid] = c;
  }
  __syncthreads();
  a = red[0];
  b = red[16];
  c = red[32];
  for (int w = 1; w < nw; ++w) {
    a += red[w];
    b += red[16 + w];
    c += red[32 + w];
  }
  __syncthreads();
}

// Minimum of one value per thread over a 1024-thread block (every thread gets it).
__device__ double block1024_min_of(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < nw; ++w) r = fmin(r, red[w]);
  __syncthreads();
  return r;
}

__device__ double block1024_min(const double* p, int count, double* red) {
  double v = 1e300;
  for (int i = threadIdx.x; i < count; i += blockDim.x) v = fmin(v, p[i]);
  return block1024_min_of(v, red);
}

constexpr int kDecideBatch = 16;  // partials of each array in flight per thread in k_decide's pass
constexpr int kDecideData = 4;    // data partials loaded ahead per thread (kPartMax / 1024)

// Reduce the energy of the evaluated velocity and take the guard decision.
//  init = 1 : first evaluation of a level (row 0), no decision.
//  mode GRAD / RETRY : the slot evaluated a trial in buffer 1 - base.
__device__ __forceinline__ void decide_body(State* st, const double* partR, int T,
                                            const double* partD, const double* partI,
                                            const double* partDet, int nfw, int nbw, int has_img,
                                            double dt, double h3, double inv_sigma2, int guard,
                                            double* trace, int init) {
  __shared__ double red[3 * 1024];
  const int mode = st->mode;
  if (mode == MODE_STOPPED) {
    if (threadIdx.x == 0 && !init) {
      double* row = trace + (long long)st->row * 8;
      const double nan = __longlong_as_double(0x7ff8000000000000LL);
      row[0] = nan;
      row[1] = nan;
      row[2] = nan;
      row[3] = st->eps;
      row[4] = st->min_det;
      row[5] = nan;
      row[6] = 0.0;
      row[7] = st->E;
      st->row += 1;
    }
    return;
  }
  // One strided pass over the partials of every time step (the regulariser's,
  // and with a decision the min-det ones), then one reduction tree per quantity;
  // each thread adds its partials in increasing index order and the trees are
  // fixed, so repeated calls give the same bits.  Every round loads
  // kDecideBatch partials of each array before it uses them, and the data
  // partials (at most kDecideData per thread) come before the first round, so
  // their latencies overlap instead of adding up.
  const bool want_det = !init && mode == MODE_GRAD;
  const int step = blockDim.x;
  double d = 0.0, im = 0.0;
  {
    double vd[kDecideData], vi[kDecideData];
#pragma unroll
    for (int u = 0; u < kDecideData; ++u) {
      const int ii = (int)threadIdx.x + u * step;
      vd[u] = ii < nfw ? partD[ii] : 0.0;
      vi[u] = ii < nfw ? partI[ii] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kDecideData; ++u) {
      if ((int)threadIdx.x + u * step < nfw) {
        d += vd[u];
        im += vi[u];
      }
    }
    for (int ii = (int)threadIdx.x + kDecideData * step; ii < nfw; ii += step) {
      d += partD[ii];
      im += partI[ii];
    }
  }
  double r = 0.0, m = 1e300;
  const int nR = T * nfw, nDet = want_det ? T * nbw : 0, nmax = nR > nDet ? nR : nDet;
  for (int i0 = (int)threadIdx.x; i0 < nmax; i0 += kDecideBatch * step) {
    double vr[kDecideBatch], vt[kDecideBatch];
#pragma unroll
    for (int u = 0; u < kDecideBatch; ++u) {
      const int ii = i0 + u * step;
      vr[u] = 0.0;
      vt[u] = 1e300;
      if (ii < nR) {
        const int j = ii / nfw;
        vr[u] = partR[(long long)j * kPartMax + (ii - j * nfw)];
      }
      if (ii < nDet) {
        const int j = ii / nbw;
        vt[u] = partDet[(long long)j * kPartMax + (ii - j * nbw)];
      }
    }
#pragma unroll
    for (int u = 0; u < kDecideBatch; ++u) {
      if (i0 + u * step < nR) r += vr[u];
      m = fmin(m, vt[u]);
    }
  }
  block1024_sum3(r, d, im, red);
  const double R = r, D = d, I = im;
  const double md = want_det ? block1024_min_of(m, red) : 0.0;
  if (threadIdx.x != 0) return;
  const double nan = __longlong_as_double(0x7ff8000000000000LL);
  const double Rt = dt * h3 * R;
  const double Dt = h3 * inv_sigma2 * D;
  const double It = has_img ? h3 * I : nan;
  const double Et = Rt + Dt;
  double* row = trace + (long long)st->row * 8;
  if (init) {
    st->E = Et;
    st->R = Rt;
    st->D = Dt;
    st->img = It;
    row[0] = Et;
    row[1] = Rt;
    row[2] = Dt;
    row[3] = st->step0;
    row[4] = nan;
    row[5] = It;
    row[6] = 1.0;
    row[7] = Et;
    st->row += 1;
    if (!isfinite(Et)) {
      st->nonfinite = 1;
      st->mode = MODE_STOPPED;
    } else {
      st->mode = MODE_GRAD;
      st->eval = 1 - st->base;
    }
    return;
  }
  if (mode == MODE_GRAD) st->min_det = md;
  const double used = st->eps;
  const bool ok = !guard || (Et <= st->E);
  if (ok) {
    st->base = 1 - st->base;
    st->E = Et;
    st->R = Rt;
    st->D = Dt;
    st->img = It;
    st->halvings = 0;
    st->mode = MODE_GRAD;
    if (!isfinite(Et)) {
      st->nonfinite = 1;
      st->mode = MODE_STOPPED;
    }
  } else {
    st->eps = 0.5 * st->eps;
    st->halvings += 1;
    st->mode = MODE_RETRY;
    if (st->halvings >= 10) {
      st->mode = MODE_STOPPED;
      st->stopped_any = 1;
    }
  }
  st->eval = 1 - st->base;
  row[0] = Et;
  row[1] = Rt;
  row[2] = Dt;
  row[3] = used;
  row[4] = st->min_det;
  row[5] = It;
  row[6] = ok ? 1.0 : 0.0;
  row[7] = st->E;
  st->row += 1;
}

__global__ __launch_bounds__(1024) void k_decide(State* st, const double* partR, int T,
                                                 const double* partD, const double* partI,
                                                 const double* partDet, int nfw, int nbw,
                                                 int has_img, double dt, double h3,
                                                 double inv_sigma2, int guard, double* trace,
                                                 int init) {
  decide_body(st, partR, T, partD, partI, partDet, nfw, nbw, has_img, dt, h3, inv_sigma2, guard,
              trace, init);
}

// One block per problem of a batch.
__global__ __launch_bounds__(1024) void k_decide_batched(BatchRef br, int init) {
  const DecideArgs& d = ((const PairTab*)br.tab[blockIdx.x])->dec[init];
  decide_body(d.st, d.partR, d.T, d.partD, d.partI, d.partDet, d.nfw, d.nbw, d.has_img, d.dt, d.h3,
              d.inv_sigma2, d.guard, d.trace, d.init);
}

void launch_decide_batched(const BatchRef& br, int init, hipStream_t s) {
  hipLaunchKernelGGL(k_decide_batched, dim3(br.np), dim3(1024), 0, s, br, init);
}

void launch_decide(State* st, const double* partR, int T, const double* partD, const double* partI,
                   const double* partDet, int nblk_fwd, int nblk_bwd, int has_img, double dt,
                   double h3, double inv_sigma2, int guard, double* trace, int init,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(1024), 0, s, st, partR, T, partD, partI, partDet,
                     nblk_fwd, nblk_bwd, has_img, dt, h3, inv_sigma2, guard, trace, init);
}

// After a rejection: trial <- (base + trial) / 2, i.e. v - eps g with the halved eps.
__device__ __forceinline__ void retry_body(float* vA, float* vB, long long count, const State* st,
                                           long long tile, long long ntiles) {
  if (st->mode != MODE_RETRY) return;
  const float* base = st->base ? vB : vA;
  float* trial = st->base ? vA : vB;
  for (long long i = tile * kBlock + threadIdx.x; i < count; i += ntiles * kBlock)
    trial[i] = 0.5f * (base[i] + trial[i]);
}

__global__ __launch_bounds__(kBlock) void k_retry(float* vA, float* vB, long long count,
                                                  const State* st) {
  retry_body(vA, vB, count, st, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_retry_batched(BatchRef br) {
  const int p = batch_pair(br, blockIdx.x);
  const RetryArgs& r = ((const PairTab*)br.tab[p])->rty;
  retry_body(r.vA, r.vB, r.count, r.st, blockIdx.x - br.off[p], br.off[p + 1] - br.off[p]);
}

void launch_retry_batched(const BatchRef& br, hipStream_t s) {
  hipLaunchKernelGGL(k_retry_batched, dim3(br.off[br.np]), dim3(kBlock), 0, s, br);
}

// Most slots accept their trial and the kernel returns at once, so its cost is
// the dispatch of its blocks: 4096 of them (a grid-stride loop covers the rest)
// take a few microseconds where one block per 256 elements took about 15.
void launch_retry(float* vA, float* vB, long long count, const State* st, hipStream_t s) {
  long long b = (count + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_retry, dim3((unsigned)b), dim3(kBlock), 0, s, vA, vB, count, st);
}

// Min det D phi_{t_j,1} over j < T and the grid, from the body-force steps of a
// backward sweep of the returned velocity (partials of jb = 0 .. T-1).
__global__ __launch_bounds__(1024) void k_final_det(State* st, const double* partDet, int T,
                                                    int nbw) {
  __shared__ double red[1024];
  double md = 1e300;
  for (int j = 0; j < T; ++j) md = fmin(md, block1024_min(partDet + (long long)j * kPartMax, nbw, red));
  if (threadIdx.x == 0) st->min_det_final = md;
}

void launch_final_det(State* st, const double* partDet, int T, int nbw, hipStream_t s) {
  hipLaunchKernelGGL(k_final_det, dim3(1), dim3(1024), 0, s, st, partDet, T, nbw);
}

__global__ void k_energy_out(const State* st, double* out4) {
  if (threadIdx.x == 0) {
    out4[0] = st->E;
    out4[1] = st->R;
    out4[2] = st->D;
    out4[3] = st->img;
  }
}

void launch_energy_out(const State* st, double* out4, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_out, dim3(1), dim3(64), 0, s, st, out4);
}

// As k_energy_out, but E is reported as NaN when the splat radius overflowed.
__global__ void k_energy_out_checked(const State* st, const int* overflow, double* out4) {
  if (threadIdx.x == 0) {
    out4[0] = *overflow ? __longlong_as_double(0x7ff8000000000000LL) : st->E;
    out4[1] = st->R;
    out4[2] = st->D;
    out4[3] = st->img;
  }
}

void launch_energy_out_checked(const State* st, const int* overflow, double* out4, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_out_checked, dim3(1), dim3(64), 0, s, st, overflow, out4);
}

}  // namespace lddmm
