// Kernels of the warm-start network: 3x3x3 convolutions (forward, input
// gradient, weight gradient) as implicit GEMMs on the bf16 matrix cores, and
// the small elementwise layers around them.  Activations and weights are bf16
// in HBM, every sum accumulates in FP32 (MFMA) or FP64 (losses).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "lddmm_cnn.h"

namespace lddmm_cnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

constexpr int kThreads = 256;     // 4 wavefronts of 64
constexpr int BK = 32;            // K per MFMA step (v_mfma_f32_16x16x32_bf16)
constexpr int LDK = BK + 8;       // LDS row stride in bf16: 80 bytes, 16-byte aligned rows

__device__ __forceinline__ float bf2f(u16 b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}

// Round to nearest bf16, ties to even (NaN stays NaN).
__device__ __forceinline__ u16 f2bf(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u16)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}

enum { OP_FWD = 0, OP_DGRAD = 1, OP_WGRAD = 2 };

// One convolution as C[M x N] = sum_k A[m][k] B[k][n]:
//  forward : m = output voxel, n = output channel, k = (tap, input channel);
//            A = input gathered at s*o + tap - 1, B = w[n][k].
//  dgrad   : m = input voxel, n = input channel, k = (tap, output channel);
//            A = dy at the output voxel o with s*o + tap - 1 = m (if any),
//            B = wt[n][k] (the transposed weight).
//  wgrad   : m = output channel, n = (tap, input channel), k = output voxel;
//            A = dy[k][m], B = input at s*k + tap - 1; the K range is split
//            over blockIdx.z and the partial tiles are reduced afterwards.
struct ConvArgs {
  const u16* x;       // forward / wgrad input; dgrad: dy
  const u16* wb;      // forward: w; dgrad: wt; wgrad: dy
  const float* bias;
  const u16* mask;
  const u16* add;
  void* out;          // forward: y; dgrad: dx; wgrad: FP32 partial tiles
  int n, d, h, w, ci; // input geometry
  int od, oh, ow, co; // output geometry
  int s;
  int M, N, K, kchunk;
  int relu, out_f32, add_stride, add_off;
};

// (b, z, y, x) of voxel index m on an n x d x h x w grid, as (b d + z, y, x).
__device__ __forceinline__ void split_voxel(int m, int d, int h, int w, int& bz, int& y, int& x) {
  x = m % w;
  const int t = m / w;
  y = t % h;
  bz = t / h;
  (void)d;
}

// 8 consecutive bf16 (16 bytes) from p, or zeros.
__device__ __forceinline__ uint4 ld8(const u16* p) { return *(const uint4*)p; }

template <int OP, bool VEC>
__device__ __forceinline__ uint4 load_a_k(const ConvArgs& a, int m, int k, int kend, int bz, int ry,
                                          int rx) {
  // A row m (KCONTIG): 8 consecutive k from k.  bz, ry, rx: the row's voxel.
  uint4 r = make_uint4(0, 0, 0, 0);
  if (m >= a.M) return r;
  if (OP == OP_FWD) {
    const int b = bz / a.od, oz = bz - b * a.od;
    if (VEC) {
      if (k >= kend) return r;
      const int tap = k / a.ci, c0 = k - tap * a.ci;
      const int kz = tap / 9, ky = (tap / 3) % 3, kx = tap % 3;
      const int iz = oz * a.s + kz - 1, iy = ry * a.s + ky - 1, ix = rx * a.s + kx - 1;
      if ((unsigned)iz < (unsigned)a.d && (unsigned)iy < (unsigned)a.h &&
          (unsigned)ix < (unsigned)a.w)
        r = ld8(a.x + ((((long)b * a.d + iz) * a.h + iy) * a.w + ix) * a.ci + c0);
      return r;
    }
    u16 e[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      e[j] = 0;
      const int kk = k + j;
      if (kk < kend) {
        const int tap = kk / a.ci, c = kk - tap * a.ci;
        const int kz = tap / 9, ky = (tap / 3) % 3, kx = tap % 3;
        const int iz = oz * a.s + kz - 1, iy = ry * a.s + ky - 1, ix = rx * a.s + kx - 1;
        if ((unsigned)iz < (unsigned)a.d && (unsigned)iy < (unsigned)a.h &&
            (unsigned)ix < (unsigned)a.w)
          e[j] = a.x[((((long)b * a.d + iz) * a.h + iy) * a.w + ix) * a.ci + c];
      }
    }
    r.x = e[0] | ((uint32_t)e[1] << 16);
    r.y = e[2] | ((uint32_t)e[3] << 16);
    r.z = e[4] | ((uint32_t)e[5] << 16);
    r.w = e[6] | ((uint32_t)e[7] << 16);
    return r;
  } else {  // OP_DGRAD: row = input voxel; dy (in a.x) has the output geometry, a.co channels
    const int b = bz / a.d, iz = bz - b * a.d;
    u16 e[8];
    const int nv = VEC ? 1 : 8;
    for (int j = 0; j < nv; ++j) {
      const int kk = k + j;
      if (!VEC) e[j] = 0;
      if (kk >= kend) continue;
      const int tap = kk / a.co, c = kk - tap * a.co;
      const int kz = tap / 9, ky = (tap / 3) % 3, kx = tap % 3;
      int oz = iz + 1 - kz, oy = ry + 1 - ky, ox = rx + 1 - kx;
      if (a.s == 2) {
        if ((oz | oy | ox) & 1) continue;
        oz >>= 1;
        oy >>= 1;
        ox >>= 1;
      }
      if ((unsigned)oz < (unsigned)a.od && (unsigned)oy < (unsigned)a.oh &&
          (unsigned)ox < (unsigned)a.ow) {
        const u16* p = a.x + ((((long)b * a.od + oz) * a.oh + oy) * a.ow + ox) * a.co + c;
        if (VEC)
          r = ld8(p);
        else
          e[j] = *p;
      }
    }
    if (!VEC) {
      r.x = e[0] | ((uint32_t)e[1] << 16);
      r.y = e[2] | ((uint32_t)e[3] << 16);
      r.z = e[4] | ((uint32_t)e[5] << 16);
      r.w = e[6] | ((uint32_t)e[7] << 16);
    }
    return r;
  }
}

// B row n (KCONTIG, forward / dgrad): 8 consecutive k of the (transposed) weight.
template <bool VEC>
__device__ __forceinline__ uint4 load_b_k(const ConvArgs& a, int n, int k, int kend) {
  uint4 r = make_uint4(0, 0, 0, 0);
  if (n >= a.N) return r;
  const u16* p = a.wb + (long)n * a.K + k;
  if (VEC) {
    if (k < kend) r = ld8(p);
    return r;
  }
  u16 e[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) e[j] = (k + j < kend) ? p[j] : (u16)0;
  r.x = e[0] | ((uint32_t)e[1] << 16);
  r.y = e[2] | ((uint32_t)e[3] << 16);
  r.z = e[4] | ((uint32_t)e[5] << 16);
  r.w = e[6] | ((uint32_t)e[7] << 16);
  return r;
}

// wgrad A (MNCONTIG): dy[k][m .. m+8) at output voxel k.
template <bool VEC>
__device__ __forceinline__ uint4 load_a_mn(const ConvArgs& a, int m, int k, int kend) {
  uint4 r = make_uint4(0, 0, 0, 0);
  if (k >= kend || m >= a.M) return r;
  const u16* p = a.wb + (long)k * a.co + m;
  if (VEC) return ld8(p);
  u16 e[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) e[j] = (m + j < a.M) ? p[j] : (u16)0;
  r.x = e[0] | ((uint32_t)e[1] << 16);
  r.y = e[2] | ((uint32_t)e[3] << 16);
  r.z = e[4] | ((uint32_t)e[5] << 16);
  r.w = e[6] | ((uint32_t)e[7] << 16);
  return r;
}

// wgrad B (MNCONTIG): input at s*o + tap - 1 for columns n .. n+8 = (tap, ci).
template <bool VEC>
__device__ __forceinline__ uint4 load_b_mn(const ConvArgs& a, int n, int k, int kend) {
  uint4 r = make_uint4(0, 0, 0, 0);
  if (k >= kend || n >= a.N) return r;
  int bz, oy, ox;
  split_voxel(k, a.od, a.oh, a.ow, bz, oy, ox);
  const int b = bz / a.od, oz = bz - b * a.od;
  u16 e[8];
  const int nv = VEC ? 1 : 8;
  for (int j = 0; j < nv; ++j) {
    const int nn = n + j;
    if (!VEC) e[j] = 0;
    if (nn >= a.N) continue;
    const int tap = nn / a.ci, c = nn - tap * a.ci;
    const int kz = tap / 9, ky = (tap / 3) % 3, kx = tap % 3;
    const int iz = oz * a.s + kz - 1, iy = oy * a.s + ky - 1, ix = ox * a.s + kx - 1;
    if ((unsigned)iz < (unsigned)a.d && (unsigned)iy < (unsigned)a.h &&
        (unsigned)ix < (unsigned)a.w) {
      const u16* p = a.x + ((((long)b * a.d + iz) * a.h + iy) * a.w + ix) * a.ci + c;
      if (VEC)
        r = ld8(p);
      else
        e[j] = *p;
    }
  }
  if (!VEC) {
    r.x = e[0] | ((uint32_t)e[1] << 16);
    r.y = e[2] | ((uint32_t)e[3] << 16);
    r.z = e[4] | ((uint32_t)e[5] << 16);
    r.w = e[6] | ((uint32_t)e[7] << 16);
  }
  return r;
}

__device__ __forceinline__ void st8_rows(u16* sm, int row, int col, uint4 v) {
  // 8 values of consecutive rows row .. row+7 at column col (transposing store)
  sm[(row + 0) * LDK + col] = (u16)(v.x & 0xffff);
  sm[(row + 1) * LDK + col] = (u16)(v.x >> 16);
  sm[(row + 2) * LDK + col] = (u16)(v.y & 0xffff);
  sm[(row + 3) * LDK + col] = (u16)(v.y >> 16);
  sm[(row + 4) * LDK + col] = (u16)(v.z & 0xffff);
  sm[(row + 5) * LDK + col] = (u16)(v.z >> 16);
  sm[(row + 6) * LDK + col] = (u16)(v.w & 0xffff);
  sm[(row + 7) * LDK + col] = (u16)(v.w >> 16);
}

// Block tile BM x BN over 4 waves arranged WAVES_M x (4 / WAVES_M); each wave owns
// TM x TN MFMA tiles of 16 x 16.  LDS holds A as [BM][BK] and B as [BN][BK]
// (k contiguous), so a lane reads its 8 k-values of one row as one 16-byte load.
// MFMA lane layout (16x16x32): lane l supplies row l%16 of A and column l%16 of B
// with k in 8*(l/16) .. +8 (the same k order for both operands); it receives
// D[4*(l/16) + r][l%16], r = 0..3.
template <int OP, int BM, int BN, int WAVES_M, bool VA, bool VB>
__global__ __launch_bounds__(kThreads) void k_conv_gemm(ConvArgs a) {
  constexpr int WAVES_N = 4 / WAVES_M;
  constexpr int TM = BM / (16 * WAVES_M), TN = BN / (16 * WAVES_N);
  static_assert(TM >= 1 && TN >= 1, "tile");
  constexpr int GA = (OP == OP_WGRAD) ? (BM / 8) * BK : BM * (BK / 8);   // 8-element groups
  constexpr int GB = (OP == OP_WGRAD) ? (BN / 8) * BK : BN * (BK / 8);
  constexpr int RA = (GA + kThreads - 1) / kThreads, RB = (GB + kThreads - 1) / kThreads;
  __shared__ __attribute__((aligned(16))) u16 As[BM * LDK];
  __shared__ __attribute__((aligned(16))) u16 Bs[BN * LDK];

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave % WAVES_M, wn = wave / WAVES_M;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int kbeg = blockIdx.z * a.kchunk;
  const int kend = min(a.K, kbeg + a.kchunk);

  // per-thread voxel of its A rows (forward / dgrad), fixed over the K loop
  int rbz[RA], rry[RA], rrx[RA];
  if (OP != OP_WGRAD) {
#pragma unroll
    for (int i = 0; i < RA; ++i) {
      const int g = t + i * kThreads;
      const int m = m0 + g / (BK / 8);
      rbz[i] = rry[i] = rrx[i] = 0;
      if (g < GA && m < a.M) {
        if (OP == OP_FWD)
          split_voxel(m, a.od, a.oh, a.ow, rbz[i], rry[i], rrx[i]);
        else
          split_voxel(m, a.d, a.h, a.w, rbz[i], rry[i], rrx[i]);
      }
    }
  }

  uint4 ra[RA], rb[RB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < RA; ++i) {
      const int g = t + i * kThreads;
      ra[i] = make_uint4(0, 0, 0, 0);
      if (g < GA) {
        if (OP == OP_WGRAD)
          ra[i] = load_a_mn<VA>(a, m0 + 8 * (g / BK), k0 + (g % BK), kend);
        else
          ra[i] = load_a_k<OP, VA>(a, m0 + g / (BK / 8), k0 + 8 * (g % (BK / 8)), kend, rbz[i],
                                   rry[i], rrx[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int g = t + i * kThreads;
      rb[i] = make_uint4(0, 0, 0, 0);
      if (g < GB) {
        if (OP == OP_WGRAD)
          rb[i] = load_b_mn<VB>(a, n0 + 8 * (g / BK), k0 + (g % BK), kend);
        else
          rb[i] = load_b_k<VB>(a, n0 + g / (BK / 8), k0 + 8 * (g % (BK / 8)), kend);
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < RA; ++i) {
      const int g = t + i * kThreads;
      if (g < GA) {
        if (OP == OP_WGRAD)
          st8_rows(As, 8 * (g / BK), g % BK, ra[i]);
        else
          *(uint4*)&As[(g / (BK / 8)) * LDK + 8 * (g % (BK / 8))] = ra[i];
      }
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int g = t + i * kThreads;
      if (g < GB) {
        if (OP == OP_WGRAD)
          st8_rows(Bs, 8 * (g / BK), g % BK, rb[i]);
        else
          *(uint4*)&Bs[(g / (BK / 8)) * LDK + 8 * (g % (BK / 8))] = rb[i];
      }
    }
  };

  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + BK < kend) fetch(k0 + BK);     // next chunk's global loads overlap the MFMAs
    const int kq = 8 * (lane >> 4), r16 = lane & 15;
    bf16x8 fa[TM], fb[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
      fa[i] = *(const bf16x8*)&As[((wm * TM + i) * 16 + r16) * LDK + kq];
#pragma unroll
    for (int j = 0; j < TN; ++j)
      fb[j] = *(const bf16x8*)&Bs[((wn * TN + j) * 16 + r16) * LDK + kq];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
  }

  // epilogue
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = n0 + (wn * TN + j) * 16 + (lane & 15);
      if (col >= a.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + (wm * TM + i) * 16 + 4 * (lane >> 4) + r;
        if (row >= a.M) continue;
        float v = acc[i][j][r];
        if (OP == OP_WGRAD) {
          ((float*)a.out)[((long)blockIdx.z * a.M + row) * a.N + col] = v;
          continue;
        }
        if (OP == OP_FWD) {
          if (a.bias) v += a.bias[col];
          if (a.relu) v = fmaxf(v, 0.f);
        } else {
          if (a.mask && !(bf2f(a.mask[(long)row * a.N + col]) > 0.f)) v = 0.f;
          if (a.add) v += bf2f(a.add[(long)row * a.add_stride + a.add_off + col]);
        }
        const long o = (long)row * a.N + col;
        if (a.out_f32)
          ((float*)a.out)[o] = v;
        else
          ((u16*)a.out)[o] = f2bf(v);
      }
    }
}

template <int OP, int BM, int BN, int WM>
static void launch_tile(const ConvArgs& a, bool va, bool vb, dim3 grid, hipStream_t s) {
  if (va && vb)
    hipLaunchKernelGGL((k_conv_gemm<OP, BM, BN, WM, true, true>), grid, dim3(kThreads), 0, s, a);
  else if (va)
    hipLaunchKernelGGL((k_conv_gemm<OP, BM, BN, WM, true, false>), grid, dim3(kThreads), 0, s, a);
  else if (vb)
    hipLaunchKernelGGL((k_conv_gemm<OP, BM, BN, WM, false, true>), grid, dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((k_conv_gemm<OP, BM, BN, WM, false, false>), grid, dim3(kThreads), 0, s,
                       a);
}

// Forward and dgrad: M large, N = channels.
template <int OP>
static void launch_mk(const ConvArgs& a, bool va, bool vb, hipStream_t s) {
  if (a.N <= 16) {
    launch_tile<OP, 128, 16, 4>(a, va, vb, dim3((a.M + 127) / 128, 1, 1), s);
  } else if (a.N <= 32) {
    launch_tile<OP, 128, 32, 4>(a, va, vb, dim3((a.M + 127) / 128, 1, 1), s);
  } else {
    launch_tile<OP, 64, 64, 2>(a, va, vb, dim3((a.M + 63) / 64, (a.N + 63) / 64, 1), s);
  }
}

// wgrad tiles: BM from the output channels, BN = 64 columns of (tap, ci).
static int wgrad_bm(int co) { return co <= 16 ? 16 : (co <= 32 ? 32 : 64); }

static void wgrad_split(int M, int N, int K, int* nsplit, int* kchunk) {
  const int bm = wgrad_bm(M);
  const long tiles = (long)((M + bm - 1) / bm) * ((N + 63) / 64);
  long want = std::max(1L, 2048 / std::max(1L, tiles));
  long chunk = (K + want - 1) / want;
  chunk = std::max(256L, (chunk + BK - 1) / BK * BK);
  *kchunk = (int)chunk;
  *nsplit = (int)((K + chunk - 1) / chunk);
}

// ------------------------------------------------------------ small kernels --

__global__ void k_reduce_splits(const float* part, int nsplit, long count, float* out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float v = 0.f;
  for (int s = 0; s < nsplit; ++s) v += part[(long)s * count + i];
  out[i] = v;
}

// Per-block, per-channel partial sums of dy over voxels (rows), fixed order.
__global__ __launch_bounds__(kThreads) void k_bias_partial(const u16* dy, long rows, int co,
                                                           int rows_per_block, float* part) {
  const int c = threadIdx.x % co;           // co <= 256 channels, one thread group per channel
  const int lanes = kThreads / co;          // threads per channel
  const int l = threadIdx.x / co;
  __shared__ float red[kThreads];
  float v = 0.f;
  const long r0 = (long)blockIdx.x * rows_per_block;
  const long r1 = min(rows, r0 + rows_per_block);
  if (l < lanes)
    for (long r = r0 + l; r < r1; r += lanes) v += bf2f(dy[r * co + c]);
  red[threadIdx.x] = (l < lanes) ? v : 0.f;
  __syncthreads();
  if (threadIdx.x < co) {
    float s = 0.f;
    for (int j = 0; j < lanes; ++j) s += red[j * co + threadIdx.x];
    part[(long)blockIdx.x * co + threadIdx.x] = s;
  }
}

__global__ void k_bias_final(const float* part, int nblk, int co, float* db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= co) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += part[(long)b * co + c];
  db[c] = s;
}

__global__ void k_transpose_w(const u16* w, int co, int ci, u16* wt) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;   // index into wt [ci][27][co]
  const long total = (long)co * 27 * ci;
  if (i >= total) return;
  const int o = (int)(i % co);
  const long r = i / co;
  const int tap = (int)(r % 27), c = (int)(r / 27);
  wt[i] = w[((long)o * 27 + tap) * ci + c];
}

__global__ void k_to_bf16(const float* src, long count, u16* dst) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = f2bf(src[i]);
}

__global__ void k_upcat(const u16* coarse, int n, int d, int h, int w, int cc, const u16* skip,
                        int cs, u16* out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int C = cc + cs;
  const long total = (long)n * 8 * d * h * w * C;
  if (i >= total) return;
  const int c = (int)(i % C);
  const long q = i / C;                          // fine voxel
  if (c >= cc) {
    out[i] = skip[q * cs + (c - cc)];
    return;
  }
  const int W2 = 2 * w, H2 = 2 * h, D2 = 2 * d;
  const int x = (int)(q % W2);
  const long t = q / W2;
  const int y = (int)(t % H2);
  const long t2 = t / H2;
  const int z = (int)(t2 % D2);
  const int b = (int)(t2 / D2);
  out[i] = coarse[((((long)b * d + z / 2) * h + y / 2) * w + x / 2) * cc + c];
}

__global__ void k_upcat_bwd(const u16* dcat, int n, int d, int h, int w, int cc, int cs,
                            u16* dco) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)n * d * h * w * cc;
  if (i >= total) return;
  const int c = (int)(i % cc);
  const long p = i / cc;
  const int x = (int)(p % w);
  const long t = p / w;
  const int y = (int)(t % h);
  const long t2 = t / h;
  const int z = (int)(t2 % d);
  const int b = (int)(t2 / d);
  const int C = cc + cs;
  float s = 0.f;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const long q = (((long)b * 2 * d + 2 * z + dz) * 2 * h + 2 * y + dy) * 2 * w + 2 * x + dx;
        s += bf2f(dcat[q * C + c]);
      }
  dco[i] = f2bf(s);
}

__global__ __launch_bounds__(kThreads) void k_mse(const float* out, const float* tgt, long count,
                                                  u16* dout, double* part) {
  __shared__ double red[kThreads];
  double acc = 0.0;
  const double sc = 2.0 / (double)count;
  for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < count;
       i += (long)gridDim.x * kThreads) {
    const double dlt = (double)out[i] - (double)tgt[i];
    acc += dlt * dlt;
    dout[i] = f2bf((float)(sc * dlt));
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kThreads) void k_mse_final(const double* part, int nblk, long count,
                                                        double* loss) {
  __shared__ double red[kThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kThreads) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (double)count;
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, long count, float lr,
                       float b1, float b2, float eps, float c1, float c2, u16* pb) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  p[i] = pi;
  if (pb) pb[i] = f2bf(pi);
}

__global__ void k_pack_masks(const float* M0, const float* M1, long count, u16* x) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  x[2 * i] = f2bf(M0[i]);
  x[2 * i + 1] = f2bf(M1[i]);
}

// label[(z h4 + y) w4 + x][3j + c] = scale * mean over the 4x4x4 block of v[j][c]
__global__ void k_pool_velocity(const float* v, int T, int d, int h, int w, float scale,
                                float* label) {
  const int d4 = d / 4, h4 = h / 4, w4 = w / 4, C = 3 * T;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)d4 * h4 * w4 * C;
  if (i >= total) return;
  const int ch = (int)(i % C);
  const long p = i / C;
  const int x = (int)(p % w4);
  const int y = (int)((p / w4) % h4);
  const int z = (int)(p / ((long)w4 * h4));
  const float* f = v + (long)ch * d * h * w;        // channel 3j + c is plane (j, c)
  float s = 0.f;
  for (int dz = 0; dz < 4; ++dz)
    for (int dy = 0; dy < 4; ++dy)
      for (int dx = 0; dx < 4; ++dx)
        s += f[((long)(4 * z + dz) * h + 4 * y + dy) * w + 4 * x + dx];
  label[i] = scale * s * (1.f / 64.f);
}

static unsigned blocks(long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

static int hip_ok() { return hipGetLastError() == hipSuccess ? LDDMM_OK : LDDMM_EHIP; }

static bool shape_ok(const lddmm_cnn_shape& s) {
  return s.n > 0 && s.d > 0 && s.h > 0 && s.w > 0 && s.c > 0;
}

static long elems(const lddmm_cnn_shape& s) { return (long)s.n * s.d * s.h * s.w * s.c; }

static constexpr long kMaxElems = 0x7fffffffL;

static ConvArgs conv_args(lddmm_cnn_shape xs, int cout, int stride) {
  ConvArgs a{};
  a.n = xs.n;
  a.d = xs.d;
  a.h = xs.h;
  a.w = xs.w;
  a.ci = xs.c;
  a.s = stride;
  a.od = (xs.d - 1) / stride + 1;
  a.oh = (xs.h - 1) / stride + 1;
  a.ow = (xs.w - 1) / stride + 1;
  a.co = cout;
  return a;
}

}  // namespace lddmm_cnn

using namespace lddmm_cnn;

extern "C" {

int lddmm_conv3d_forward(const uint16_t* x, lddmm_cnn_shape xs, const uint16_t* w,
                         const float* bias, int32_t cout, int32_t stride, int32_t relu, void* y,
                         int32_t y_dtype, void* stream) {
  if (!x || !w || !y || !shape_ok(xs) || cout < 1 || (stride != 1 && stride != 2) ||
      (y_dtype != LDDMM_CNN_BF16 && y_dtype != LDDMM_CNN_F32))
    return LDDMM_EINVAL;
  ConvArgs a = conv_args(xs, cout, stride);
  const long M = (long)a.n * a.od * a.oh * a.ow;
  if (elems(xs) > kMaxElems || M * cout > kMaxElems || 27L * xs.c > kMaxElems) return LDDMM_EINVAL;
  a.x = x;
  a.wb = w;
  a.bias = bias;
  a.out = y;
  a.relu = relu ? 1 : 0;
  a.out_f32 = y_dtype == LDDMM_CNN_F32;
  a.M = (int)M;
  a.N = cout;
  a.K = 27 * xs.c;
  a.kchunk = a.K;
  hipGetLastError();
  const bool vec = (xs.c % 8) == 0;
  launch_mk<OP_FWD>(a, vec, vec, (hipStream_t)stream);
  return hip_ok();
}

int lddmm_conv3d_backward_data(const uint16_t* dy, lddmm_cnn_shape xs, int32_t cout,
                               int32_t stride, const uint16_t* wt, const uint16_t* mask,
                               const uint16_t* add, int32_t add_stride, int32_t add_off, void* dx,
                               int32_t dx_dtype, void* stream) {
  if (!dy || !wt || !dx || !shape_ok(xs) || cout < 1 || (stride != 1 && stride != 2) ||
      (dx_dtype != LDDMM_CNN_BF16 && dx_dtype != LDDMM_CNN_F32))
    return LDDMM_EINVAL;
  if (add && (add_off < 0 || add_stride < add_off + xs.c)) return LDDMM_EINVAL;
  ConvArgs a = conv_args(xs, cout, stride);
  const long nvox = (long)xs.n * xs.d * xs.h * xs.w;
  if (elems(xs) > kMaxElems || (long)a.n * a.od * a.oh * a.ow * cout > kMaxElems ||
      (add && nvox * add_stride > kMaxElems))
    return LDDMM_EINVAL;
  a.x = dy;
  a.wb = wt;
  a.mask = mask;
  a.add = add;
  a.add_stride = add_stride;
  a.add_off = add_off;
  a.out = dx;
  a.out_f32 = dx_dtype == LDDMM_CNN_F32;
  a.M = (int)nvox;
  a.N = xs.c;
  a.K = 27 * cout;
  a.kchunk = a.K;
  hipGetLastError();
  const bool vec = (cout % 8) == 0;
  launch_mk<OP_DGRAD>(a, vec, vec, (hipStream_t)stream);
  return hip_ok();
}

size_t lddmm_conv3d_wgrad_workspace(lddmm_cnn_shape xs, int32_t cout, int32_t stride) {
  if (!shape_ok(xs) || cout < 1 || (stride != 1 && stride != 2)) return 0;
  ConvArgs a = conv_args(xs, cout, stride);
  const long K = (long)a.n * a.od * a.oh * a.ow;
  int nsplit, kchunk;
  wgrad_split(cout, 27 * xs.c, (int)std::min(K, kMaxElems), &nsplit, &kchunk);
  const size_t part = (size_t)nsplit * cout * 27 * xs.c * sizeof(float);
  const long rows_per_block = 4096;
  const size_t bias = (size_t)((K + rows_per_block - 1) / rows_per_block) * cout * sizeof(float);
  return (part + 255) / 256 * 256 + bias;
}

int lddmm_conv3d_backward_weight(const uint16_t* dy, const uint16_t* x, lddmm_cnn_shape xs,
                                 int32_t cout, int32_t stride, float* dw, float* db,
                                 void* workspace, size_t workspace_bytes, void* stream) {
  if (!dy || !x || !dw || !workspace || !shape_ok(xs) || cout < 1 || cout > 256 ||
      (stride != 1 && stride != 2))
    return LDDMM_EINVAL;
  ConvArgs a = conv_args(xs, cout, stride);
  const long K = (long)a.n * a.od * a.oh * a.ow;
  if (elems(xs) > kMaxElems || K * cout > kMaxElems) return LDDMM_EINVAL;
  if (workspace_bytes < lddmm_conv3d_wgrad_workspace(xs, cout, stride)) return LDDMM_EINVAL;
  int nsplit, kchunk;
  wgrad_split(cout, 27 * xs.c, (int)K, &nsplit, &kchunk);
  float* part = (float*)workspace;
  const size_t part_bytes = ((size_t)nsplit * cout * 27 * xs.c * sizeof(float) + 255) / 256 * 256;
  a.x = x;
  a.wb = dy;
  a.out = part;
  a.M = cout;
  a.N = 27 * xs.c;
  a.K = (int)K;
  a.kchunk = kchunk;
  hipStream_t s = (hipStream_t)stream;
  hipGetLastError();
  const bool va = (cout % 8) == 0, vb = (xs.c % 8) == 0;
  const dim3 grid((cout + wgrad_bm(cout) - 1) / wgrad_bm(cout), (a.N + 63) / 64, nsplit);
  if (cout <= 16)
    launch_tile<OP_WGRAD, 16, 64, 1>(a, va, vb, grid, s);
  else if (cout <= 32)
    launch_tile<OP_WGRAD, 32, 64, 2>(a, va, vb, grid, s);
  else
    launch_tile<OP_WGRAD, 64, 64, 2>(a, va, vb, grid, s);
  const long count = (long)cout * a.N;
  hipLaunchKernelGGL(k_reduce_splits, dim3(blocks(count)), dim3(256), 0, s, part, nsplit, count,
                     dw);
  if (db) {
    const int rows_per_block = 4096;
    const int nblk = (int)((K + rows_per_block - 1) / rows_per_block);
    float* bpart = (float*)((char*)workspace + part_bytes);
    hipLaunchKernelGGL(k_bias_partial, dim3(nblk), dim3(kThreads), 0, s, dy, K, (int)cout,
                       rows_per_block, bpart);
    hipLaunchKernelGGL(k_bias_final, dim3(blocks(cout)), dim3(256), 0, s, bpart, nblk, (int)cout,
                       db);
  }
  return hip_ok();
}

int lddmm_cnn_transpose_weight(const uint16_t* w, int32_t cout, int32_t cin, uint16_t* wt,
                               void* stream) {
  if (!w || !wt || cout < 1 || cin < 1) return LDDMM_EINVAL;
  const long total = (long)cout * 27 * cin;
  hipGetLastError();
  hipLaunchKernelGGL(k_transpose_w, dim3(blocks(total)), dim3(256), 0, (hipStream_t)stream, w,
                     (int)cout, (int)cin, wt);
  return hip_ok();
}

int lddmm_cnn_to_bf16(const float* src, int64_t count, uint16_t* dst, void* stream) {
  if (!src || !dst || count < 1 || count > kMaxElems) return LDDMM_EINVAL;
  hipGetLastError();
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks(count)), dim3(256), 0, (hipStream_t)stream, src,
                     (long)count, dst);
  return hip_ok();
}

int lddmm_cnn_upcat(const uint16_t* coarse, lddmm_cnn_shape cs, const uint16_t* skip,
                    int32_t skip_c, uint16_t* out, void* stream) {
  if (!coarse || !skip || !out || !shape_ok(cs) || skip_c < 1) return LDDMM_EINVAL;
  const long total = (long)cs.n * 8 * cs.d * cs.h * cs.w * (cs.c + skip_c);
  if (total > kMaxElems) return LDDMM_EINVAL;
  hipGetLastError();
  hipLaunchKernelGGL(k_upcat, dim3(blocks(total)), dim3(256), 0, (hipStream_t)stream, coarse,
                     cs.n, cs.d, cs.h, cs.w, cs.c, skip, (int)skip_c, out);
  return hip_ok();
}

int lddmm_cnn_upcat_backward(const uint16_t* dcat, lddmm_cnn_shape cs, int32_t skip_c,
                             uint16_t* d_coarse, void* stream) {
  if (!dcat || !d_coarse || !shape_ok(cs) || skip_c < 0) return LDDMM_EINVAL;
  const long total = (long)cs.n * 8 * cs.d * cs.h * cs.w * (cs.c + skip_c);
  if (total > kMaxElems) return LDDMM_EINVAL;
  hipGetLastError();
  hipLaunchKernelGGL(k_upcat_bwd, dim3(blocks(elems(cs))), dim3(256), 0, (hipStream_t)stream,
                     dcat, cs.n, cs.d, cs.h, cs.w, cs.c, (int)skip_c, d_coarse);
  return hip_ok();
}

static int mse_blocks(long count) { return (int)std::min(1024L, (count + 4095) / 4096); }

size_t lddmm_cnn_mse_workspace(int64_t count) {
  return count < 1 ? 0 : (size_t)mse_blocks(count) * sizeof(double);
}

int lddmm_cnn_mse(const float* out, const float* target, int64_t count, uint16_t* dout,
                  double* loss, void* workspace, size_t workspace_bytes, void* stream) {
  if (!out || !target || !dout || !loss || !workspace || count < 1 || count > kMaxElems ||
      workspace_bytes < lddmm_cnn_mse_workspace(count))
    return LDDMM_EINVAL;
  const int nb = mse_blocks(count);
  hipStream_t s = (hipStream_t)stream;
  hipGetLastError();
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(kThreads), 0, s, out, target, (long)count, dout,
                     (double*)workspace);
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(kThreads), 0, s, (const double*)workspace, nb,
                     (long)count, loss);
  return hip_ok();
}

int lddmm_cnn_adam(float* p, const float* g, float* m, float* v, int64_t count, int32_t step,
                   float lr, float beta1, float beta2, float eps, uint16_t* p_bf16, void* stream) {
  if (!p || !g || !m || !v || count < 1 || count > kMaxElems || step < 1) return LDDMM_EINVAL;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
  hipGetLastError();
  hipLaunchKernelGGL(k_adam, dim3(blocks(count)), dim3(256), 0, (hipStream_t)stream, p, g, m, v,
                     (long)count, lr, beta1, beta2, eps, c1, c2, p_bf16);
  return hip_ok();
}

int lddmm_cnn_pack_masks(const float* M0, const float* M1, int64_t count, uint16_t* x,
                         void* stream) {
  if (!M0 || !M1 || !x || count < 1 || 2 * count > kMaxElems) return LDDMM_EINVAL;
  hipGetLastError();
  hipLaunchKernelGGL(k_pack_masks, dim3(blocks(count)), dim3(256), 0, (hipStream_t)stream, M0, M1,
                     (long)count, x);
  return hip_ok();
}

int lddmm_cnn_pool_velocity(const float* v, int32_t T, int32_t d, int32_t h, int32_t w,
                            float scale, float* label, void* stream) {
  if (!v || !label || T < 1 || d < 4 || h < 4 || w < 4 || d % 4 || h % 4 || w % 4 ||
      3L * T * d * h * w > kMaxElems)
    return LDDMM_EINVAL;
  const long total = 3L * T * (d / 4) * (h / 4) * (w / 4);
  hipGetLastError();
  hipLaunchKernelGGL(k_pool_velocity, dim3(blocks(total)), dim3(256), 0, (hipStream_t)stream, v,
                     (int)T, (int)d, (int)h, (int)w, scale, label);
  return hip_ok();
}

}  // extern "C"
