// Mask generation (Methods, Mask Generation) and the surface metrics of the
// evaluation (Methods, Evaluation), on bit-packed masks.
//
// Layout: a mask is packed 32 voxels per word along x, rows of W = ceil(nx/32)
// words, word (wx, y, z) at (z ny + y) W + wx, bit b = voxel x = 32 wx + b;
// bits past nx are always 0.
//
// Morphology with a ball: the ball of physical radius r is the union, over the
// (dy, dz) with dy^2 + dz^2 <= (r/h)^2, of x-runs of half-width w(dy, dz) =
// max{dx : dx^2 + dy^2 + dz^2 <= (r/h)^2}.  Dilation of a word ORs, over those
// (dy, dz), the row (y+dy, z+dz) dilated along x by w (shifts of the word and
// its two neighbours); erosion ANDs the x-eroded rows.  Outside the grid is
// background for both.  One thread per output word: 32 voxels per thread, and
// the per-word work is independent of how many voxels the ball holds.
//
// Surface distances: S = mask voxels with a face neighbour outside the mask.
// The squared distance (in voxels, exact integers) from every voxel to the
// nearest voxel of the other surface is the separable minimum
//   d2(x, y, z) = min_z' [ min_y' [ g1(x, y', z') + (y - y')^2 ] + (z - z')^2 ],
//   g1(x, y, z) = min over surface voxels x' of row (y, z) of (x - x')^2,
// computed as: the nearest set bit along each x row (bit scans of the packed
// words), a min pass along y for every voxel, and the min along z only at the
// voxels of the first surface, searched outward from the voxel and stopped once
// the squared offset alone reaches the best value found (exact).  The Hausdorff distance takes the largest d2 (atomicMax); the median
// counts every d2 in a histogram over the integers 0 .. max possible (counts in
// LDS for small d2, which hold nearly all of them), and one block finds the
// middle rank(s).  Distances are h sqrt(d2) in FP64.
#include <cfloat>
#include <cmath>

#include "internal.h"
#include "lddmm.h"
#include "lddmm_masks.h"

namespace lddmm {
namespace {

constexpr int kWaves = kBlock / 64;
constexpr int kMaxM = LDDMM_MORPH_MAX_RADIUS_VOXELS + 1;
constexpr int kTable = (2 * kMaxM + 1) * (2 * kMaxM + 1);
constexpr uint32_t kInf = 0x3FFFFFFFu;
constexpr int kLdsBins = 4096;          // squared distances counted in LDS first

struct MGrid {
  int nx, ny, nz, W;                    // W: words per row
  long long nwords;                     // W ny nz
  long long n;                          // nx ny nz
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

MGrid make_mgrid(const lddmm_grid* g) {
  MGrid m;
  m.nx = g->nx;
  m.ny = g->ny;
  m.nz = g->nz;
  m.W = (g->nx + 31) / 32;
  m.nwords = (long long)m.W * g->ny * g->nz;
  m.n = (long long)g->nx * g->ny * g->nz;
  return m;
}

inline long long grid_voxels(const lddmm_grid* g) {
  if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nx > LDDMM_MAX_DIM ||
      g->ny > LDDMM_MAX_DIM || g->nz > LDDMM_MAX_DIM || !(g->spacing > 0.0) ||
      !std::isfinite(g->spacing))
    return -1;
  return (long long)g->nx * g->ny * g->nz;
}

inline unsigned blocks_for(long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  if (b > 65535) b = 65535;
  return (unsigned)(b < 1 ? 1 : b);
}

// ------------------------------------------------------------- packing ----

enum : int { SRC_MASK = 0, SRC_THRESHOLD = 1, SRC_LABELS = 2 };

// One wavefront per row: lanes read 64 consecutive voxels, a ballot packs them.
__global__ __launch_bounds__(64) void k_pack(MGrid g, const void* __restrict__ src, int kind,
                                             float tau, uint32_t* __restrict__ out) {
  const long long row = blockIdx.x;                      // y + ny z
  const long long base = row * g.nx;
  uint32_t* dst = out + row * g.W;
  for (int x0 = 0; x0 < g.nx; x0 += 64) {
    const int x = x0 + threadIdx.x;
    bool on = false;
    if (x < g.nx) {
      if (kind == SRC_LABELS)
        on = static_cast<const int32_t*>(src)[base + x] != 0;
      else if (kind == SRC_THRESHOLD)
        on = static_cast<const float*>(src)[base + x] > tau;
      else
        on = static_cast<const float*>(src)[base + x] > 0.f;
    }
    const unsigned long long bits = __ballot(on);
    if (threadIdx.x == 0) {
      const int w = x0 >> 5;
      dst[w] = (uint32_t)bits;
      if (w + 1 < g.W) dst[w + 1] = (uint32_t)(bits >> 32);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_unpack(MGrid g, const uint32_t* __restrict__ in,
                                                   float* __restrict__ out) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < g.n;
       i += (long long)gridDim.x * kBlock) {
    const long long row = i / g.nx;
    const int x = (int)(i - row * g.nx);
    out[i] = (in[row * g.W + (x >> 5)] >> (x & 31)) & 1u ? 1.f : 0.f;
  }
}

// ---------------------------------------------------------- morphology ----

// Half-widths w(dy, dz) of the ball (-1: no voxel of the ball in that row), the
// same FP64 decision as the definition: dx^2 + dy^2 + dz^2 <= (r/h)^2.
__global__ void k_ball_table(double rho, int m, int8_t* __restrict__ table) {
  const double rr = rho * rho;
  const int side = 2 * m + 1;
  for (int k = threadIdx.x; k < side * side; k += blockDim.x) {
    const int dy = k % side - m, dz = k / side - m;
    int w = -1;
    for (int dx = 0; dx <= m; ++dx)
      if ((double)(dx * dx + dy * dy + dz * dz) <= rr) w = dx;
    table[k] = (int8_t)w;
  }
}

__device__ __forceinline__ uint32_t word_at(const uint32_t* __restrict__ a, const MGrid& g, int wx,
                                            long long rowbase) {
  return (wx >= 0 && wx < g.W) ? a[rowbase + wx] : 0u;
}

__device__ __forceinline__ uint32_t dilate_x(uint32_t prev, uint32_t cur, uint32_t next, int w) {
  uint32_t acc = cur;
  for (int s = 1; s <= w; ++s)
    acc |= (cur << s) | (prev >> (32 - s)) | (cur >> s) | (next << (32 - s));
  return acc;
}

__device__ __forceinline__ uint32_t erode_x(uint32_t prev, uint32_t cur, uint32_t next, int w) {
  uint32_t acc = cur;
  for (int s = 1; s <= w; ++s)
    acc &= ((cur << s) | (prev >> (32 - s))) & ((cur >> s) | (next << (32 - s)));
  return acc;
}

__device__ __forceinline__ uint32_t valid_bits(const MGrid& g, int wx) {
  const int rem = g.nx - 32 * wx;
  return rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
}

// One thread per output word; erode (dilate = 0) or dilate (dilate = 1).
__global__ __launch_bounds__(kBlock) void k_morph(MGrid g, const uint32_t* __restrict__ in,
                                                  uint32_t* __restrict__ out,
                                                  const int8_t* __restrict__ table, int m,
                                                  int dilate) {
  __shared__ int8_t tab[kTable];
  const int side = 2 * m + 1;
  for (int k = threadIdx.x; k < side * side; k += kBlock) tab[k] = table[k];
  __syncthreads();
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < g.nwords;
       i += (long long)gridDim.x * kBlock) {
    const long long row = i / g.W;
    const int wx = (int)(i - row * g.W);
    const int y = (int)(row % g.ny), z = (int)(row / g.ny);
    uint32_t acc = dilate ? 0u : 0xFFFFFFFFu;
    for (int k = 0; k < side * side; ++k) {
      const int w = tab[k];
      if (w < 0) continue;
      const int yy = y + (k % side - m), zz = z + (k / side - m);
      if (yy < 0 || yy >= g.ny || zz < 0 || zz >= g.nz) {
        if (!dilate) {
          acc = 0u;
          break;
        }
        continue;
      }
      const long long rb = ((long long)zz * g.ny + yy) * g.W;
      const uint32_t p = word_at(in, g, wx - 1, rb), c = in[rb + wx], nx = word_at(in, g, wx + 1, rb);
      if (dilate) {
        acc |= dilate_x(p, c, nx, w);
      } else {
        acc &= erode_x(p, c, nx, w);
        if (!acc) break;
      }
    }
    out[i] = acc & valid_bits(g, wx);
  }
}

// --------------------------------------------------------------- surfaces ----

__global__ __launch_bounds__(kBlock) void k_surface(MGrid g, const uint32_t* __restrict__ a,
                                                    uint32_t* __restrict__ s) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < g.nwords;
       i += (long long)gridDim.x * kBlock) {
    const long long row = i / g.W;
    const int wx = (int)(i - row * g.W);
    const int y = (int)(row % g.ny), z = (int)(row / g.ny);
    const uint32_t c = a[i];
    const uint32_t p = word_at(a, g, wx - 1, row * g.W), n = word_at(a, g, wx + 1, row * g.W);
    uint32_t inner = c & ((c << 1) | (p >> 31)) & ((c >> 1) | (n << 31));
    inner &= y > 0 ? a[i - g.W] : 0u;
    inner &= y + 1 < g.ny ? a[i + g.W] : 0u;
    inner &= z > 0 ? a[i - (long long)g.W * g.ny] : 0u;
    inner &= z + 1 < g.nz ? a[i + (long long)g.W * g.ny] : 0u;
    s[i] = c & ~inner;
  }
}

// x pass: squared distance along the row to the nearest surface voxel, one
// thread per voxel: the nearest set bit at or left of x and at or right of x,
// found with count-leading / trailing-zero over the packed words.
__global__ __launch_bounds__(kBlock) void k_edt_x(MGrid g, const uint32_t* __restrict__ s,
                                                  uint32_t* __restrict__ g1) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < g.n;
       i += (long long)gridDim.x * kBlock) {
    const long long row = i / g.nx;
    const int x = (int)(i - row * g.nx);
    const uint32_t* sr = s + row * g.W;
    const int w0 = x >> 5, b = x & 31;
    uint32_t best = kInf;
    // left: bits <= b of word w0, then whole words further left
    uint32_t m = sr[w0] & (b == 31 ? 0xFFFFFFFFu : ((2u << b) - 1u));
    for (int w = w0;;) {
      if (m) {
        const int left = 32 * w + 31 - __clz(m);
        best = (uint32_t)((x - left) * (x - left));
        break;
      }
      if (--w < 0) break;
      m = sr[w];
    }
    // right: bits >= b of word w0, then whole words further right
    m = sr[w0] & ~((1u << b) - 1u);
    for (int w = w0;;) {
      if (m) {
        const int right = 32 * w + __ffs(m) - 1;
        const uint32_t d = (uint32_t)((right - x) * (right - x));
        best = d < best ? d : best;
        break;
      }
      if (++w >= g.W) break;
      m = sr[w];
    }
    g1[i] = best;
  }
}

// y pass for every voxel: g2(x, y, z) = min_y' g1(x, y', z) + (y - y')^2.  A block
// holds a tile of tx x-columns of one z plane in LDS (all y; tx ny <= 16384
// values, 64 KB).
inline int edt_tile_x(int ny) {
  int tx = 16384 / ny;
  return tx > 32 ? 32 : (tx < 1 ? 1 : tx);
}

__global__ __launch_bounds__(kBlock) void k_edt_y(MGrid g, int tx, const uint32_t* __restrict__ g1,
                                                  uint32_t* __restrict__ g2) {
  extern __shared__ uint32_t col[];                       // [ny][tx]
  const int tiles = (g.nx + tx - 1) / tx;
  const int z = blockIdx.x / tiles, x0 = (blockIdx.x % tiles) * tx;
  const long long plane = (long long)z * g.ny * g.nx;
  for (int k = threadIdx.x; k < g.ny * tx; k += kBlock) {
    const int y = k / tx, x = x0 + k % tx;
    col[k] = x < g.nx ? g1[plane + (long long)y * g.nx + x] : kInf;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < g.ny * tx; k += kBlock) {
    const int y = k / tx, xl = k % tx, x = x0 + xl;
    if (x >= g.nx) continue;
    // every row of the column (most columns never meet the surface, so an
    // outward search with early exit does not pay here); kInf + (ny-1)^2 still
    // fits, so no term needs a test, and a result at or above kInf is kInf
    uint32_t best = kInf;
    for (int yp = 0; yp < g.ny; ++yp) {
      const uint32_t e = col[yp * tx + xl] + (uint32_t)((y - yp) * (y - yp));
      best = e < best ? e : best;
    }
    g2[plane + (long long)y * g.nx + x] = best < kInf ? best : kInf;
  }
}

// z pass at the voxels of surface A (one thread per packed word, its set bits
// only): d2 = min_z' g2(x, y, z') + (z - z')^2, searched outward from z until
// (z - z')^2 >= d2; then the Hausdorff maximum and the histogram of d2.
__global__ __launch_bounds__(kBlock) void k_edt_z_collect(MGrid g, const uint32_t* __restrict__ sa,
                                                          const uint32_t* __restrict__ g2,
                                                          uint32_t* __restrict__ hist,
                                                          uint32_t nbins,
                                                          unsigned* __restrict__ scal) {
  __shared__ uint32_t lh[kLdsBins];
  __shared__ unsigned lmax, lcnt;
  for (int k = threadIdx.x; k < kLdsBins; k += kBlock) lh[k] = 0u;
  if (threadIdx.x == 0) {
    lmax = 0u;
    lcnt = 0u;
  }
  __syncthreads();
  const long long plane = (long long)g.nx * g.ny;
  unsigned my_max = 0u, my_cnt = 0u;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < g.nwords;
       i += (long long)gridDim.x * kBlock) {
    uint32_t bits = sa[i];
    if (!bits) continue;
    const long long row = i / g.W;
    const int wx = (int)(i - row * g.W);
    const int y = (int)(row % g.ny), z = (int)(row / g.ny);
    while (bits) {
      const int bit = __ffs(bits) - 1;
      bits &= bits - 1u;
      const int x = 32 * wx + bit;
      const long long xy = (long long)y * g.nx + x;
      uint32_t best = g2[(long long)z * plane + xy];
      for (int d = 1; (uint32_t)(d * d) < best; ++d) {
        const bool lo = z - d >= 0, hi = z + d < g.nz;
        if (!lo && !hi) break;
        const uint32_t a = lo ? g2[(long long)(z - d) * plane + xy] : kInf;
        const uint32_t c = hi ? g2[(long long)(z + d) * plane + xy] : kInf;
        const uint32_t m = a < c ? a : c;
        if (m < kInf) {
          const uint32_t e = m + (uint32_t)(d * d);
          best = e < best ? e : best;
        }
      }
      // the other surface is non-empty whenever the result is used, so best < kInf
      my_max = best > my_max ? best : my_max;
      ++my_cnt;
      if (best < (uint32_t)kLdsBins)
        atomicAdd(&lh[best], 1u);
      else if (best < nbins)
        atomicAdd(&hist[best], 1u);
    }
  }
  if (my_cnt) {
    atomicMax(&lmax, my_max);
    atomicAdd(&lcnt, my_cnt);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kLdsBins && k < (int)nbins; k += kBlock)
    if (lh[k]) atomicAdd(&hist[k], lh[k]);
  if (threadIdx.x == 0 && lcnt) {
    atomicMax(&scal[0], lmax);
    atomicAdd(&scal[1], lcnt);
  }
}

__global__ __launch_bounds__(kBlock) void k_count_bits(const uint32_t* __restrict__ a, long long n,
                                                       unsigned* __restrict__ dst) {
  unsigned c = 0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    c += __popc(a[i]);
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  __shared__ unsigned sw[kWaves];
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned t = 0;
    for (int w = 0; w < kWaves; ++w) t += sw[w];
    if (t) atomicAdd(dst, t);
  }
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t* __restrict__ p, long long n,
                                                     uint32_t v) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    p[i] = v;
}

// Sums of the histogram in tiles of kBlock bins, one block per tile.
__global__ __launch_bounds__(kBlock) void k_tile_sums(const uint32_t* __restrict__ hist,
                                                      uint32_t nbins, uint32_t* __restrict__ tsum) {
  const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
  uint32_t c = k < nbins ? hist[k] : 0u;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  __shared__ uint32_t wsum[kWaves];
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kWaves; ++w) t += wsum[w];
    tsum[blockIdx.x] = t;
  }
}

// One block: Hausdorff distance and the median of the histogram of d2 over both
// directions; out = {d_H, d_M, |S_A|, |S_B|}.  The tile sums (in LDS) locate the
// tiles of the middle rank(s), whose bins are then read into LDS and scanned.
constexpr int kMaxTiles = 12800;        // >= (3 * 1023^2 + 1) / kBlock

__global__ __launch_bounds__(kBlock) void k_surface_final(const uint32_t* __restrict__ hist,
                                                          uint32_t nbins,
                                                          const uint32_t* __restrict__ tsum_g,
                                                          const unsigned* __restrict__ scal,
                                                          double h, double* __restrict__ out) {
  __shared__ uint32_t tsum[kMaxTiles];
  __shared__ uint32_t bins[2][kBlock];
  __shared__ uint32_t tile[2];
  __shared__ unsigned long long before_tile[2];
  const unsigned na = scal[2], nb = scal[3];
  const unsigned long long m = (unsigned long long)scal[1];   // distances counted, both ways
  const uint32_t ntiles = (nbins + kBlock - 1) / kBlock;
  for (uint32_t t = threadIdx.x; t < ntiles; t += kBlock) tsum[t] = tsum_g[t];
  __syncthreads();
  const bool empty = na == 0 || nb == 0 || m == 0;
  // 0-based ranks of the middle value(s) in increasing d2 order
  const unsigned long long ranks[2] = {empty ? 0 : (m - 1) / 2, empty ? 0 : m / 2};
  if (threadIdx.x < 2) {
    unsigned long long before = 0;
    uint32_t t = 0;
    if (!empty)
      while (before + tsum[t] <= ranks[threadIdx.x]) before += tsum[t++];
    tile[threadIdx.x] = t;
    before_tile[threadIdx.x] = before;
  }
  __syncthreads();
  for (int q = 0; q < 2; ++q) {
    const uint32_t k = tile[q] * kBlock + threadIdx.x;
    bins[q][threadIdx.x] = k < nbins ? hist[k] : 0u;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  out[2] = (double)na;
  out[3] = (double)nb;
  if (empty) {
    out[0] = NAN;
    out[1] = NAN;
    return;
  }
  out[0] = h * sqrt((double)scal[0]);
  double v[2];
  for (int q = 0; q < 2; ++q) {
    unsigned long long before = before_tile[q];
    int j = 0;
    for (;; ++j) {
      before += bins[q][j];
      if (before > ranks[q]) break;
    }
    v[q] = h * sqrt((double)(tile[q] * kBlock + j));
  }
  out[1] = (m & 1ull) ? v[0] : (v[0] + v[1]) / 2.0;
}

__global__ __launch_bounds__(kBlock) void k_label_mask(const int32_t* __restrict__ L, long long n,
                                                       float* __restrict__ m) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    m[i] = L[i] != 0 ? 1.f : 0.f;
}

// ------------------------------------------------------------- workspace ----

struct MaskLayout {
  size_t a, b, c, table, g1, g2, hist, tsum, scal, total;
};

MaskLayout mask_layout(const MGrid& g, uint32_t nbins) {
  MaskLayout L;
  size_t o = 0;
  const size_t wb = align256(sizeof(uint32_t) * (size_t)g.nwords);
  L.a = o; o += wb;
  L.b = o; o += wb;
  L.c = o; o += wb;
  L.table = o; o += align256(kTable);
  L.g1 = o; o += align256(sizeof(uint32_t) * (size_t)g.n);
  L.g2 = o; o += align256(sizeof(uint32_t) * (size_t)g.n);
  L.hist = o; o += align256(sizeof(uint32_t) * (size_t)nbins);
  L.tsum = o; o += align256(sizeof(uint32_t) * (size_t)((nbins + kBlock - 1) / kBlock));
  L.scal = o; o += align256(sizeof(unsigned) * 8);
  L.total = o;
  return L;
}

uint32_t dist_bins(const MGrid& g) {
  const long long dx = g.nx - 1, dy = g.ny - 1, dz = g.nz - 1;
  return (uint32_t)(dx * dx + dy * dy + dz * dz + 1);
}

int launch_status() {
  return hipGetLastError() == hipSuccess ? LDDMM_OK : LDDMM_EHIP;
}

// One erosion or dilation of `in` into `out` with the ball of radius rho voxels.
void morph_pass(const MGrid& g, const uint32_t* in, uint32_t* out, int8_t* table, double rho,
                int dilate, hipStream_t s) {
  const int m = (int)floor(rho) + 1;
  hipLaunchKernelGGL(k_ball_table, dim3(1), dim3(kBlock), 0, s, rho, m, table);
  hipLaunchKernelGGL(k_morph, dim3(blocks_for(g.nwords)), dim3(kBlock), 0, s, g, in, out, table,
                     m, dilate);
}

bool radius_ok(double radius, double h) {
  return radius >= 0.0 && std::isfinite(radius) &&
         radius / h < (double)(LDDMM_MORPH_MAX_RADIUS_VOXELS + 1);
}

}  // namespace
}  // namespace lddmm

using namespace lddmm;

extern "C" {

size_t lddmm_masks_workspace_size(const lddmm_grid* grid) {
  if (grid_voxels(grid) < 0) return 0;
  const MGrid g = make_mgrid(grid);
  return mask_layout(g, dist_bins(g)).total;
}

int lddmm_label_mask(const lddmm_grid* grid, const int32_t* labels, float* mask, void* stream) {
  if (grid_voxels(grid) < 0 || !labels || !mask) return LDDMM_EINVAL;
  const MGrid g = make_mgrid(grid);
  (void)hipGetLastError();   // clear an earlier error: the status returned is these launches'
  hipLaunchKernelGGL(k_label_mask, dim3(blocks_for(g.n)), dim3(kBlock), 0, (hipStream_t)stream,
                     labels, g.n, mask);
  return launch_status();
}

int lddmm_morphology(const lddmm_grid* grid, const float* mask, int32_t op, double radius,
                     float* out, void* workspace, size_t workspace_bytes, void* stream) {
  if (grid_voxels(grid) < 0 || !mask || !out || !workspace) return LDDMM_EINVAL;
  if (op < LDDMM_MORPH_ERODE || op > LDDMM_MORPH_CLOSE) return LDDMM_EINVAL;
  if (!radius_ok(radius, grid->spacing)) return LDDMM_EINVAL;
  if (workspace_bytes < lddmm_masks_workspace_size(grid)) return LDDMM_EINVAL;
  const MGrid g = make_mgrid(grid);
  const MaskLayout L = mask_layout(g, dist_bins(g));
  char* ws = static_cast<char*>(workspace);
  uint32_t* a = reinterpret_cast<uint32_t*>(ws + L.a);
  uint32_t* b = reinterpret_cast<uint32_t*>(ws + L.b);
  int8_t* table = reinterpret_cast<int8_t*>(ws + L.table);
  const double rho = radius / grid->spacing;
  hipStream_t s = (hipStream_t)stream;
  (void)hipGetLastError();   // clear an earlier error: the status returned is these launches'
  {
    hipLaunchKernelGGL(k_pack, dim3((unsigned)(g.ny * g.nz)), dim3(64), 0, s, g, mask, (int)SRC_MASK,
                       0.f, a);
    if (op == LDDMM_MORPH_ERODE || op == LDDMM_MORPH_DILATE) {
      morph_pass(g, a, b, table, rho, op == LDDMM_MORPH_DILATE, s);
      hipLaunchKernelGGL(k_unpack, dim3(blocks_for(g.n)), dim3(kBlock), 0, s, g, b, out);
    } else {
      const int first_dilates = op == LDDMM_MORPH_CLOSE;
      morph_pass(g, a, b, table, rho, first_dilates, s);
      morph_pass(g, b, a, table, rho, !first_dilates, s);
      hipLaunchKernelGGL(k_unpack, dim3(blocks_for(g.n)), dim3(kBlock), 0, s, g, a, out);
    }
  }
  return launch_status();
}

int lddmm_target_mask(const lddmm_grid* grid, const float* image, float tau, double open_radius,
                      double close_radius, float* mask, void* workspace, size_t workspace_bytes,
                      void* stream) {
  if (grid_voxels(grid) < 0 || !image || !mask || !workspace) return LDDMM_EINVAL;
  if (!radius_ok(open_radius, grid->spacing) || !radius_ok(close_radius, grid->spacing))
    return LDDMM_EINVAL;
  if (workspace_bytes < lddmm_masks_workspace_size(grid)) return LDDMM_EINVAL;
  const MGrid g = make_mgrid(grid);
  const MaskLayout L = mask_layout(g, dist_bins(g));
  char* ws = static_cast<char*>(workspace);
  uint32_t* a = reinterpret_cast<uint32_t*>(ws + L.a);
  uint32_t* b = reinterpret_cast<uint32_t*>(ws + L.b);
  int8_t* table = reinterpret_cast<int8_t*>(ws + L.table);
  hipStream_t s = (hipStream_t)stream;
  (void)hipGetLastError();   // clear an earlier error: the status returned is these launches'
  {
    hipLaunchKernelGGL(k_pack, dim3((unsigned)(g.ny * g.nz)), dim3(64), 0, s, g, image,
                       (int)SRC_THRESHOLD, tau, a);
    const double ro = open_radius / grid->spacing, rc = close_radius / grid->spacing;
    morph_pass(g, a, b, table, ro, 0, s);        // opening: erode, then dilate
    morph_pass(g, b, a, table, ro, 1, s);
    morph_pass(g, a, b, table, rc, 1, s);        // closing: dilate, then erode
    morph_pass(g, b, a, table, rc, 0, s);
    hipLaunchKernelGGL(k_unpack, dim3(blocks_for(g.n)), dim3(kBlock), 0, s, g, a, mask);
  }
  return launch_status();
}

int lddmm_surface_distance(const lddmm_grid* grid, const float* mask_a, const float* mask_b,
                           double* out, void* workspace, size_t workspace_bytes, void* stream) {
  if (grid_voxels(grid) < 0 || !mask_a || !mask_b || !out || !workspace) return LDDMM_EINVAL;
  if (workspace_bytes < lddmm_masks_workspace_size(grid)) return LDDMM_EINVAL;
  const MGrid g = make_mgrid(grid);
  const uint32_t nbins = dist_bins(g);
  const MaskLayout L = mask_layout(g, nbins);
  char* ws = static_cast<char*>(workspace);
  uint32_t* a = reinterpret_cast<uint32_t*>(ws + L.a);
  uint32_t* b = reinterpret_cast<uint32_t*>(ws + L.b);
  uint32_t* c = reinterpret_cast<uint32_t*>(ws + L.c);
  uint32_t* g1 = reinterpret_cast<uint32_t*>(ws + L.g1);
  uint32_t* g2 = reinterpret_cast<uint32_t*>(ws + L.g2);
  uint32_t* hist = reinterpret_cast<uint32_t*>(ws + L.hist);
  uint32_t* tsum = reinterpret_cast<uint32_t*>(ws + L.tsum);
  unsigned* scal = reinterpret_cast<unsigned*>(ws + L.scal);
  hipStream_t s = (hipStream_t)stream;
  const unsigned rows = (unsigned)(g.ny * g.nz);
  const int tx = edt_tile_x(g.ny);
  const unsigned ytiles = (unsigned)(g.nz * ((g.nx + tx - 1) / tx));
  (void)hipGetLastError();   // clear an earlier error: the status returned is these launches'
  {
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(nbins)), dim3(kBlock), 0, s, hist,
                       (long long)nbins, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kBlock), 0, s, scal, 8ll, 0u);
    hipLaunchKernelGGL(k_pack, dim3(rows), dim3(64), 0, s, g, mask_a, (int)SRC_MASK, 0.f, a);
    hipLaunchKernelGGL(k_pack, dim3(rows), dim3(64), 0, s, g, mask_b, (int)SRC_MASK, 0.f, b);
    hipLaunchKernelGGL(k_surface, dim3(blocks_for(g.nwords)), dim3(kBlock), 0, s, g, a, c);  // S_A
    hipLaunchKernelGGL(k_surface, dim3(blocks_for(g.nwords)), dim3(kBlock), 0, s, g, b, a);  // S_B
    hipLaunchKernelGGL(k_count_bits, dim3(blocks_for(g.nwords)), dim3(kBlock), 0, s, c, g.nwords,
                       scal + 2);
    hipLaunchKernelGGL(k_count_bits, dim3(blocks_for(g.nwords)), dim3(kBlock), 0, s, a, g.nwords,
                       scal + 3);
    for (int dir = 0; dir < 2; ++dir) {
      const uint32_t* from = dir == 0 ? c : a;       // surface whose voxels are measured
      const uint32_t* to = dir == 0 ? a : c;         // surface measured against
      hipLaunchKernelGGL(k_edt_x, dim3(blocks_for(g.n)), dim3(kBlock), 0, s, g, to, g1);
      {
        ProfScope ps(LDDMM_PROF_OTHER, g.n, s);     // the y pass: the dominant kernel
        hipLaunchKernelGGL(k_edt_y, dim3(ytiles), dim3(kBlock), sizeof(uint32_t) * g.ny * tx, s,
                           g, tx, g1, g2);
      }
      hipLaunchKernelGGL(k_edt_z_collect, dim3(blocks_for(g.nwords)), dim3(kBlock), 0, s, g, from,
                         g2, hist, nbins, scal);
    }
    hipLaunchKernelGGL(k_tile_sums, dim3((nbins + kBlock - 1) / kBlock), dim3(kBlock), 0, s, hist,
                       nbins, tsum);
    hipLaunchKernelGGL(k_surface_final, dim3(1), dim3(kBlock), 0, s, hist, nbins, tsum, scal,
                       grid->spacing, out);
  }
  return launch_status();
}

}  // extern "C"
