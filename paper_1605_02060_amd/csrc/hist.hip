// Image-LDDMM preprocessing (Methods, Preprocessing): each brain mask is applied
// to its image and the masked template image is histogram-matched to the masked
// target image -- equal-width histograms of the in-mask voxels, matched exactly
// at quantile points and linearly in between.
//
// Five launches, all streaming over the two images:
//   1. per-block in-mask minimum, maximum and count (both images, blockIdx.y);
//   2. one block per image reduces them to lo, hi and the bin scale;
//   3. per-block histograms in LDS (one copy per wavefront, so the LDS atomics
//      of a wavefront only contend with themselves), written out as per-block
//      partial counts: no global atomics and nothing to clear beforehand, and
//      the integer sums do not depend on the order they are added in;
//   4. one block per (bin, image) sums that bin's partial counts (stored
//      bin-major, so each sum reads contiguous memory); then one block walks
//      the cumulative histogram once per image for the quantile points and
//      writes the FP64 point table;
//   5. the map itself, one FP64 polyline evaluation per in-mask voxel.
// The bin decision is taken in float32 (the stored precision); the table and
// the map are FP64 with no multiply-add fusion (this file is compiled with
// -ffp-contract=off), so the arithmetic is the definition's, operation by
// operation.
#include <cfloat>
#include <cmath>

#include "internal.h"
#include "lddmm.h"

namespace lddmm {
namespace {

constexpr int kWaves = kBlock / 64;
constexpr int kHistBlocksMax = 1024;     // partial blocks per image
constexpr int kTablePts = LDDMM_HIST_MAX_POINTS + 2;

struct HistImage {
  const float* I;
  const float* M;
  long long n;
};

struct HistTable {
  double s[kTablePts];         // source points: lo, quantiles, hi
  double r[kTablePts];         // reference points
  double slope[kTablePts];     // (r[k+1] - r[k]) / (s[k+1] - s[k])
  int last;                    // index of the last point (n_points + 1)
  int valid;                   // both masks non-empty
};

struct HistRange {
  float lo, hi, scale, pad;
  unsigned long long n;
  unsigned long long pad2;
};

struct HistLayout {
  size_t plo, phi, pn, range, pcount, totals, table, total;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline int hist_blocks(long long nmax) {
  long long b = (nmax + (long long)kBlock * 32 - 1) / ((long long)kBlock * 32);
  b = (b + kXCD - 1) / kXCD * kXCD;
  if (b < kXCD) b = kXCD;
  if (b > kHistBlocksMax) b = kHistBlocksMax;
  return (int)b;
}

HistLayout hist_layout(int nblk, int nbins) {
  HistLayout L;
  size_t o = 0;
  L.plo = o;    o = align256(o + sizeof(float) * 2 * nblk);
  L.phi = o;    o = align256(o + sizeof(float) * 2 * nblk);
  L.pn = o;     o = align256(o + sizeof(unsigned) * 2 * nblk);
  L.range = o;  o = align256(o + sizeof(HistRange) * 2);
  L.pcount = o; o = align256(o + sizeof(unsigned) * 2 * (size_t)nblk * nbins);
  L.totals = o; o = align256(o + sizeof(unsigned long long) * 2 * nbins);
  L.table = o;  o = align256(o + sizeof(HistTable));
  L.total = o;
  return L;
}

__device__ __forceinline__ bool aligned16(const void* p) {
  return ((uintptr_t)p & 15) == 0;
}

// Block-wide reduction of (lo, hi, count); the result is valid in thread 0.
__device__ void block_minmax(float& lo, float& hi, unsigned& cnt) {
  __shared__ float slo[kWaves], shi[kWaves];
  __shared__ unsigned scnt[kWaves];
  for (int o = 32; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o));
    hi = fmaxf(hi, __shfl_xor(hi, o));
    cnt += __shfl_xor(cnt, o);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    slo[w] = lo;
    shi[w] = hi;
    scnt[w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kWaves; ++k) {
      lo = fminf(lo, slo[k]);
      hi = fmaxf(hi, shi[k]);
      cnt += scnt[k];
    }
  }
}

// Pass 1: in-mask min / max / count per block.
__global__ __launch_bounds__(kBlock) void k_hist_range_part(HistImage a, HistImage b,
                                                            float* __restrict__ plo,
                                                            float* __restrict__ phi,
                                                            unsigned* __restrict__ pn) {
  const HistImage im = blockIdx.y ? b : a;
  float lo = FLT_MAX, hi = -FLT_MAX;
  unsigned cnt = 0;
  const long long stride = (long long)gridDim.x * kBlock;
  const long long t0 = (long long)blockIdx.x * kBlock + threadIdx.x;
  long long done = 0;
  if (aligned16(im.I) && aligned16(im.M)) {
    const long long n4 = im.n >> 2;
    const float4* I4 = reinterpret_cast<const float4*>(im.I);
    const float4* M4 = reinterpret_cast<const float4*>(im.M);
    for (long long i = t0; i < n4; i += stride) {
      const float4 x = I4[i], m = M4[i];
      if (m.x > 0.f) { lo = fminf(lo, x.x); hi = fmaxf(hi, x.x); ++cnt; }
      if (m.y > 0.f) { lo = fminf(lo, x.y); hi = fmaxf(hi, x.y); ++cnt; }
      if (m.z > 0.f) { lo = fminf(lo, x.z); hi = fmaxf(hi, x.z); ++cnt; }
      if (m.w > 0.f) { lo = fminf(lo, x.w); hi = fmaxf(hi, x.w); ++cnt; }
    }
    done = n4 << 2;
  }
  for (long long i = done + t0; i < im.n; i += stride) {
    if (im.M[i] > 0.f) {
      const float x = im.I[i];
      lo = fminf(lo, x);
      hi = fmaxf(hi, x);
      ++cnt;
    }
  }
  block_minmax(lo, hi, cnt);
  if (threadIdx.x == 0) {
    const int o = blockIdx.y * gridDim.x + blockIdx.x;
    plo[o] = lo;
    phi[o] = hi;
    pn[o] = cnt;
  }
}

// Pass 2: one block per image; lo, hi, count and the float32 bin scale.
__global__ __launch_bounds__(kBlock) void k_hist_range_final(const float* __restrict__ plo,
                                                             const float* __restrict__ phi,
                                                             const unsigned* __restrict__ pn,
                                                             int nblk, int nbins,
                                                             HistRange* __restrict__ range) {
  const int img = blockIdx.x;
  float lo = FLT_MAX, hi = -FLT_MAX;
  unsigned long long n = 0;
  for (int k = threadIdx.x; k < nblk; k += kBlock) {
    lo = fminf(lo, plo[img * nblk + k]);
    hi = fmaxf(hi, phi[img * nblk + k]);
    n += pn[img * nblk + k];
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o));
    hi = fmaxf(hi, __shfl_xor(hi, o));
    n += __shfl_xor(n, o);
  }
  __shared__ float slo[kWaves], shi[kWaves];
  __shared__ unsigned long long sn[kWaves];
  if ((threadIdx.x & 63) == 0) {
    slo[threadIdx.x >> 6] = lo;
    shi[threadIdx.x >> 6] = hi;
    sn[threadIdx.x >> 6] = n;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kWaves; ++k) {
      lo = fminf(lo, slo[k]);
      hi = fmaxf(hi, shi[k]);
      n += sn[k];
    }
    HistRange R;
    R.lo = lo;
    R.hi = hi;
    R.scale = (n > 0 && hi > lo) ? (float)nbins / (hi - lo) : 0.f;
    R.pad = 0.f;
    R.n = n;
    R.pad2 = 0;
    range[img] = R;
  }
}

__device__ __forceinline__ void bin_add(unsigned* h, float x, float lo, float scale, int nbins) {
  int b = (int)((x - lo) * scale);
  b = b < 0 ? 0 : (b > nbins - 1 ? nbins - 1 : b);
  atomicAdd(&h[b], 1u);
}

// Pass 3: per-block partial histograms (one LDS copy per wavefront).
__global__ __launch_bounds__(kBlock) void k_hist_count(HistImage a, HistImage b, int nbins,
                                                       const HistRange* __restrict__ range,
                                                       unsigned* __restrict__ pcount) {
  extern __shared__ unsigned hl[];                     // [kWaves][nbins]
  const HistImage im = blockIdx.y ? b : a;
  for (int k = threadIdx.x; k < kWaves * nbins; k += kBlock) hl[k] = 0u;
  __syncthreads();
  const HistRange R = range[blockIdx.y];
  unsigned* h = hl + (threadIdx.x >> 6) * nbins;
  const long long stride = (long long)gridDim.x * kBlock;
  const long long t0 = (long long)blockIdx.x * kBlock + threadIdx.x;
  long long done = 0;
  if (aligned16(im.I) && aligned16(im.M)) {
    const long long n4 = im.n >> 2;
    const float4* I4 = reinterpret_cast<const float4*>(im.I);
    const float4* M4 = reinterpret_cast<const float4*>(im.M);
    for (long long i = t0; i < n4; i += stride) {
      const float4 x = I4[i], m = M4[i];
      if (m.x > 0.f) bin_add(h, x.x, R.lo, R.scale, nbins);
      if (m.y > 0.f) bin_add(h, x.y, R.lo, R.scale, nbins);
      if (m.z > 0.f) bin_add(h, x.z, R.lo, R.scale, nbins);
      if (m.w > 0.f) bin_add(h, x.w, R.lo, R.scale, nbins);
    }
    done = n4 << 2;
  }
  for (long long i = done + t0; i < im.n; i += stride)
    if (im.M[i] > 0.f) bin_add(h, im.I[i], R.lo, R.scale, nbins);
  __syncthreads();
  // bin-major partials: pcount[img][bin][block]
  for (int k = threadIdx.x; k < nbins; k += kBlock) {
    unsigned c = 0;
    for (int w = 0; w < kWaves; ++w) c += hl[w * nbins + k];
    pcount[((size_t)blockIdx.y * nbins + k) * gridDim.x + blockIdx.x] = c;
  }
}

// Quantile points of one histogram, in increasing order of p.  The first bin
// whose cumulative count reaches p n moves forward only, so one walk over the
// bins serves every point.
__device__ void quantile_points(const unsigned long long* cnt, int nbins, const HistRange& R,
                                int npts, double* pts) {
  const double lo = (double)R.lo, hi = (double)R.hi;
  const double width = (hi - lo) / (double)nbins;
  const double n = (double)R.n;
  pts[0] = lo;
  int b = 0;
  unsigned long long before = 0;
  for (int k = 1; k <= npts; ++k) {
    const double p = (double)k / (double)(npts + 1);
    const double need = p * n;
    while (b < nbins && !(cnt[b] > 0 && (double)(before + cnt[b]) >= need)) {
      before += cnt[b];
      ++b;
    }
    if (b == nbins) {
      pts[k] = hi;
    } else {
      pts[k] = lo + ((double)b + (need - (double)before) / (double)cnt[b]) * width;
    }
  }
  pts[npts + 1] = hi;
}

// Pass 4a: one block per (bin, image): the bin's total over the partial blocks.
__global__ __launch_bounds__(kBlock) void k_hist_sum(const unsigned* __restrict__ pcount, int nblk,
                                                     unsigned long long* __restrict__ totals) {
  const int row = blockIdx.y * gridDim.x + blockIdx.x;          // img * nbins + bin
  const unsigned* p = pcount + (size_t)row * nblk;
  unsigned long long c = 0;
  for (int j = threadIdx.x; j < nblk; j += kBlock) c += p[j];
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  __shared__ unsigned long long sc[kWaves];
  if ((threadIdx.x & 63) == 0) sc[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kWaves; ++w) c += sc[w];
    totals[row] = c;
  }
}

// Pass 4b: one block; quantile points and slopes from the bin totals.
__global__ __launch_bounds__(kBlock) void k_hist_table(const unsigned long long* __restrict__ totals,
                                                       int nbins, int npts,
                                                       const HistRange* __restrict__ range,
                                                       HistTable* __restrict__ table,
                                                       double* __restrict__ points,
                                                       long long* __restrict__ counts) {
  extern __shared__ unsigned long long cs[];           // [2][nbins]
  __shared__ double pts[2][kTablePts];
  for (int k = threadIdx.x; k < 2 * nbins; k += kBlock) {
    cs[k] = totals[k];
    if (counts) counts[k] = (long long)totals[k];
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const HistRange R = range[threadIdx.x];
    if (R.n > 0) quantile_points(cs + threadIdx.x * nbins, nbins, R, npts, pts[threadIdx.x]);
  }
  __syncthreads();
  const int valid = range[0].n > 0 && range[1].n > 0;
  const int last = npts + 1;
  for (int k = threadIdx.x; k <= last; k += kBlock) {
    table->s[k] = valid ? pts[0][k] : 0.0;
    table->r[k] = valid ? pts[1][k] : 0.0;
    if (k < last)
      table->slope[k] = valid ? (pts[1][k + 1] - pts[1][k]) / (pts[0][k + 1] - pts[0][k]) : 0.0;
    if (points) {
      points[k] = valid ? pts[0][k] : 0.0;
      points[last + 1 + k] = valid ? pts[1][k] : 0.0;
    }
  }
  if (threadIdx.x == 0) {
    table->last = last;
    table->valid = valid;
  }
}

__device__ __forceinline__ float map_value(float x, float m, const HistTable& T) {
  if (!(m > 0.f) || !T.valid) return 0.f;
  const double xd = (double)x;
  const int last = T.last;
  if (xd >= T.s[last]) return (float)T.r[last];
  int k = 0;
  for (int j = 1; j < last; ++j)
    if (T.s[j] <= xd) k = j;
  return (float)(T.r[k] + (xd - T.s[k]) * T.slope[k]);
}

// Pass 5: out = matched source inside its mask, 0 outside.
__global__ __launch_bounds__(kBlock) void k_hist_apply(HistImage a, const HistTable* __restrict__ table,
                                                       float* __restrict__ out) {
  __shared__ HistTable T;
  if (threadIdx.x == 0) {
    T.last = table->last;
    T.valid = table->valid;
  }
  for (int k = threadIdx.x; k < kTablePts; k += kBlock) {
    T.s[k] = table->s[k];
    T.r[k] = table->r[k];
    T.slope[k] = table->slope[k];
  }
  __syncthreads();
  const long long stride = (long long)gridDim.x * kBlock;
  const long long t0 = (long long)blockIdx.x * kBlock + threadIdx.x;
  long long done = 0;
  if (aligned16(a.I) && aligned16(a.M) && aligned16(out)) {
    const long long n4 = a.n >> 2;
    const float4* I4 = reinterpret_cast<const float4*>(a.I);
    const float4* M4 = reinterpret_cast<const float4*>(a.M);
    float4* O4 = reinterpret_cast<float4*>(out);
    for (long long i = t0; i < n4; i += stride) {
      const float4 x = I4[i], m = M4[i];
      float4 y;
      y.x = map_value(x.x, m.x, T);
      y.y = map_value(x.y, m.y, T);
      y.z = map_value(x.z, m.z, T);
      y.w = map_value(x.w, m.w, T);
      O4[i] = y;
    }
    done = n4 << 2;
  }
  for (long long i = done + t0; i < a.n; i += stride) out[i] = map_value(a.I[i], a.M[i], T);
}

__global__ __launch_bounds__(kBlock) void k_mask_image(const float* __restrict__ I,
                                                       const float* __restrict__ M, long long n,
                                                       float* __restrict__ out) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    out[i] = M[i] > 0.f ? I[i] : 0.f;
}

inline long long grid_voxels(const lddmm_grid* g) {
  if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nx > LDDMM_MAX_DIM ||
      g->ny > LDDMM_MAX_DIM || g->nz > LDDMM_MAX_DIM)
    return -1;
  return (long long)g->nx * g->ny * g->nz;
}

inline unsigned stream_blocks(long long n) {
  long long b = (n / 4 + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  return (unsigned)(b < 1 ? 1 : b);
}

int launch_status() {
  return hipGetLastError() == hipSuccess ? LDDMM_OK : LDDMM_EHIP;
}

}  // namespace
}  // namespace lddmm

using namespace lddmm;

extern "C" {

size_t lddmm_histogram_match_workspace_size(const lddmm_grid* src_grid,
                                            const lddmm_grid* ref_grid, int32_t n_bins) {
  const long long ns = grid_voxels(src_grid), nr = grid_voxels(ref_grid);
  if (ns < 0 || nr < 0 || n_bins < 1 || n_bins > LDDMM_HIST_MAX_BINS) return 0;
  const int nblk = hist_blocks(ns > nr ? ns : nr);
  return hist_layout(nblk, n_bins).total;
}

int lddmm_histogram_match(const lddmm_grid* src_grid, const float* src, const float* src_mask,
                          const lddmm_grid* ref_grid, const float* ref, const float* ref_mask,
                          int32_t n_bins, int32_t n_points, float* out, double* points,
                          int64_t* counts, void* workspace, size_t workspace_bytes,
                          void* stream) {
  const long long ns = grid_voxels(src_grid), nr = grid_voxels(ref_grid);
  if (ns < 0 || nr < 0 || !src || !src_mask || !ref || !ref_mask || !out || !workspace)
    return LDDMM_EINVAL;
  if (n_bins < 1 || n_bins > LDDMM_HIST_MAX_BINS || n_points < 0 ||
      n_points > LDDMM_HIST_MAX_POINTS)
    return LDDMM_EINVAL;
  const int nblk = hist_blocks(ns > nr ? ns : nr);
  const HistLayout L = hist_layout(nblk, n_bins);
  if (workspace_bytes < L.total) return LDDMM_EINVAL;
  char* ws = static_cast<char*>(workspace);
  float* plo = reinterpret_cast<float*>(ws + L.plo);
  float* phi = reinterpret_cast<float*>(ws + L.phi);
  unsigned* pn = reinterpret_cast<unsigned*>(ws + L.pn);
  HistRange* range = reinterpret_cast<HistRange*>(ws + L.range);
  unsigned* pcount = reinterpret_cast<unsigned*>(ws + L.pcount);
  unsigned long long* totals = reinterpret_cast<unsigned long long*>(ws + L.totals);
  HistTable* table = reinterpret_cast<HistTable*>(ws + L.table);
  const HistImage a{src, src_mask, ns}, b{ref, ref_mask, nr};
  hipStream_t s = (hipStream_t)stream;
  (void)hipGetLastError();   // clear an earlier error: the status returned is these launches'
  {
    ProfScope ps(LDDMM_PROF_HIST_RANGE, ns + nr, s);
    hipLaunchKernelGGL(k_hist_range_part, dim3(nblk, 2), dim3(kBlock), 0, s, a, b, plo, phi, pn);
    hipLaunchKernelGGL(k_hist_range_final, dim3(2), dim3(kBlock), 0, s, plo, phi, pn, nblk,
                       (int)n_bins, range);
  }
  {
    ProfScope ps(LDDMM_PROF_HIST_COUNT, ns + nr, s);
    hipLaunchKernelGGL(k_hist_count, dim3(nblk, 2), dim3(kBlock),
                       sizeof(unsigned) * kWaves * n_bins, s, a, b, (int)n_bins, range, pcount);
    hipLaunchKernelGGL(k_hist_sum, dim3(n_bins, 2), dim3(kBlock), 0, s, pcount, nblk, totals);
    hipLaunchKernelGGL(k_hist_table, dim3(1), dim3(kBlock),
                       sizeof(unsigned long long) * 2 * n_bins, s, totals, (int)n_bins,
                       (int)n_points, range, table, points, reinterpret_cast<long long*>(counts));
  }
  {
    ProfScope ps(LDDMM_PROF_HIST_APPLY, ns, s);
    hipLaunchKernelGGL(k_hist_apply, dim3(stream_blocks(ns)), dim3(kBlock), 0, s, a, table, out);
  }
  return launch_status();
}

int lddmm_mask_image(const lddmm_grid* grid, const float* image, const float* mask, float* out,
                     void* stream) {
  const long long n = grid_voxels(grid);
  if (n < 0 || !image || !mask || !out) return LDDMM_EINVAL;
  long long blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  (void)hipGetLastError();   // clear an earlier error: the status returned is these launches'
  hipLaunchKernelGGL(k_mask_image, dim3((unsigned)blocks), dim3(kBlock), 0, (hipStream_t)stream,
                     image, mask, n, out);
  return launch_status();
}

}  // extern "C"
