// Smoothing by K = (L^dagger L)^-1, L = gamma - alpha Lap (Methods, Registration),
// as a 3D DFT on the computational grid: mixed-radix (2,3,4,5,7,8) Stockham
// transforms staged in LDS, one axis per pass.
//
//   pass x-fwd : real body force b [3][P] -> half spectrum S [3][nz][ny][hs]
//                (hx = nx/2 + 1 used entries per row, rows padded to hs, a
//                multiple of 16 entries, so 128-byte tile segments stay aligned)
//                (two real lines packed into one complex transform)
//   pass y     : transform along y, in place on S
//   pass z+K   : transform along z, multiply by K_hat / |P|, inverse along z
//   pass y-inv : inverse along y
//   pass x-inv : inverse along x (Hermitian extension) + epilogue (update of v)
//
// Inverse transforms use IDFT(X) = conj(DFT(conj(X))) / N with the 1/|P| folded
// into the K_hat multiply.  Twiddles and the Laplacian symbol are generated in
// FP64 on the device and rounded once.
#include "device.h"
#include "dft.h"

namespace lddmm {

// ------------------------------------------------------------------ plans ----

bool make_plan(int n, FFTPlan* p) {
  p->n = n;
  p->nst = 0;
  int m = n, p2 = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++p2;
  }
  int st = 0;
  auto push = [&](int r) {
    if (st >= kMaxStages) return false;
    p->radix[st++] = r;
    return true;
  };
  // powers of two: radix 8 where possible, two radix-4 stages instead of 8 x 2
  while (p2 >= 3 && p2 != 4) {
    if (!push(8)) return false;
    p2 -= 3;
  }
  while (p2 >= 2) {
    if (!push(4)) return false;
    p2 -= 2;
  }
  if (p2 == 1 && !push(2)) return false;
  for (int r : {3, 5, 7}) {
    while (m % r == 0) {
      if (!push(r)) return false;
      m /= r;
    }
  }
  p->nst = st;
  int ns = 1;
  for (int k = 0; k < st; ++k) {
    p->fnb[k] = make_fastdiv((uint32_t)(n / p->radix[k]));
    p->fns[k] = make_fastdiv((uint32_t)ns);
    ns *= p->radix[k];
  }
  return m == 1;
}

__global__ void k_twiddles(float2* tw, int n) {
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < n; m += gridDim.x * blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)m / (double)n, &s, &c);
    tw[m] = make_float2((float)c, (float)-s);     // exp(-2 pi i m / n)
  }
}

void launch_twiddles(float2* tw, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles, dim3((n + 255) / 256), dim3(256), 0, s, tw, n);
}

// lambda_d(k) = (2 - 2 cos(2 pi k / n)) / h^2 : periodic 7-point Laplacian symbol along one axis.
__global__ void k_lambda(double* lam, int n, double h) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    lam[k] = (2.0 - 2.0 * cospi(2.0 * (double)k / (double)n)) / (h * h);
}

void launch_lambda(double* lam, int n, double h, hipStream_t s) {
  hipLaunchKernelGGL(k_lambda, dim3((n + 255) / 256), dim3(256), 0, s, lam, n, h);
}

// -------------------------------------------------------- radix butterflies --
// Forward DFT of R points: y[m] = sum_p x[p] exp(-2 pi i p m / R).

template <int R>
struct Roots;
template <>
struct Roots<2> {
  static constexpr float c[2] = {1.f, -1.f};
  static constexpr float s[2] = {0.f, 0.f};
};
template <>
struct Roots<3> {
  static constexpr float c[3] = {1.f, -0.5f, -0.5f};
  static constexpr float s[3] = {0.f, 0.86602540378443865f, -0.86602540378443865f};
};
template <>
struct Roots<4> {
  static constexpr float c[4] = {1.f, 0.f, -1.f, 0.f};
  static constexpr float s[4] = {0.f, 1.f, 0.f, -1.f};
};
template <>
struct Roots<5> {
  static constexpr float c[5] = {1.f, 0.30901699437494742f, -0.80901699437494742f,
                                 -0.80901699437494742f, 0.30901699437494742f};
  static constexpr float s[5] = {0.f, 0.95105651629515357f, 0.58778525229247313f,
                                 -0.58778525229247313f, -0.95105651629515357f};
};
template <>
struct Roots<7> {
  static constexpr float c[7] = {1.f,
                                 0.62348980185873353f,
                                 -0.22252093395631440f,
                                 -0.90096886790241913f,
                                 -0.90096886790241913f,
                                 -0.22252093395631440f,
                                 0.62348980185873353f};
  static constexpr float s[7] = {0.f,
                                 0.78183148246802981f,
                                 0.97492791218182361f,
                                 0.43388373911755812f,
                                 -0.43388373911755812f,
                                 -0.97492791218182361f,
                                 -0.78183148246802981f};
};
template <>
struct Roots<8> {
  static constexpr float c[8] = {1.f,  0.70710678118654752f,  0.f, -0.70710678118654752f,
                                 -1.f, -0.70710678118654752f, 0.f, 0.70710678118654752f};
  static constexpr float s[8] = {0.f, 0.70710678118654752f,  1.f,  0.70710678118654752f,
                                 0.f, -0.70710678118654752f, -1.f, -0.70710678118654752f};
};

// (a) * (-i)
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

template <int R>
__device__ __forceinline__ void radix_dft(float2 (&v)[R]);

template <>
__device__ __forceinline__ void radix_dft<2>(float2 (&v)[2]) {
  const float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

// 4-point DFT: W4 = -i.
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  const float2 t0 = cadd(x0, x2), t1 = csub(x0, x2);
  const float2 t2 = cadd(x1, x3), t3 = mul_mi(csub(x1, x3));
  x0 = cadd(t0, t2);
  x2 = csub(t0, t2);
  x1 = cadd(t1, t3);
  x3 = csub(t1, t3);
}

template <>
__device__ __forceinline__ void radix_dft<4>(float2 (&v)[4]) {
  dft4(v[0], v[1], v[2], v[3]);
}

// 8-point DFT as two 4-point DFTs (even / odd samples) and W8^k twiddles.
template <>
__device__ __forceinline__ void radix_dft<8>(float2 (&v)[8]) {
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  const float r = 0.70710678118654752f;
  // W8^1 = (1 - i)/sqrt2, W8^2 = -i, W8^3 = -(1 + i)/sqrt2
  const float2 w1 = make_float2(r * (o1.x + o1.y), r * (o1.y - o1.x));
  const float2 w2 = mul_mi(o2);
  const float2 w3 = make_float2(r * (o3.y - o3.x), -r * (o3.x + o3.y));
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, w1);
  v[5] = csub(e1, w1);
  v[2] = cadd(e2, w2);
  v[6] = csub(e2, w2);
  v[3] = cadd(e3, w3);
  v[7] = csub(e3, w3);
}

// Odd R: pair x[p] with x[R-p].  With a_p = x_p + x_{R-p}, b_p = x_p - x_{R-p}:
//   y_m     = x_0 + sum_p a_p cos(2 pi p m / R) - i sum_p b_p sin(2 pi p m / R)
//   y_{R-m} = x_0 + sum_p a_p cos(2 pi p m / R) + i sum_p b_p sin(2 pi p m / R)
template <int R>
__device__ __forceinline__ void radix_dft_odd(float2 (&v)[R]) {
  constexpr int H = (R - 1) / 2;
  float2 a[H], b[H];
#pragma unroll
  for (int p = 1; p <= H; ++p) {
    a[p - 1] = cadd(v[p], v[R - p]);
    b[p - 1] = csub(v[p], v[R - p]);
  }
  const float2 x0 = v[0];
  float2 y0 = x0;
#pragma unroll
  for (int p = 0; p < H; ++p) y0 = cadd(y0, a[p]);
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    float cr = x0.x, ci = x0.y, sr = 0.f, si = 0.f;
#pragma unroll
    for (int p = 1; p <= H; ++p) {
      const int k = (p * m) % R;
      const float c = Roots<R>::c[k], s = Roots<R>::s[k];
      cr += a[p - 1].x * c;
      ci += a[p - 1].y * c;
      sr += b[p - 1].x * s;
      si += b[p - 1].y * s;
    }
    // -i * (sr + i si) = si - i sr
    v[m] = make_float2(cr + si, ci - sr);
    v[R - m] = make_float2(cr - si, ci + sr);
  }
  v[0] = y0;
}

template <>
__device__ __forceinline__ void radix_dft<3>(float2 (&v)[3]) { radix_dft_odd<3>(v); }
template <>
__device__ __forceinline__ void radix_dft<5>(float2 (&v)[5]) { radix_dft_odd<5>(v); }
template <>
__device__ __forceinline__ void radix_dft<7>(float2 (&v)[7]) { radix_dft_odd<7>(v); }

template <int R>
__device__ __forceinline__ void radix_dft(float2 (&v)[R]) {
  float2 out[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    float re = v[0].x, im = v[0].y;
#pragma unroll
    for (int p = 1; p < R; ++p) {
      const int k = (p * m) % R;
      const float c = Roots<R>::c[k], s = -Roots<R>::s[k];
      re += v[p].x * c - v[p].y * s;
      im += v[p].x * s + v[p].y * c;
    }
    out[m] = make_float2(re, im);
  }
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = out[m];
}

// One Stockham stage on nl lines of length N held in LDS (line l at sm + l*ls).
// Ns = product of the radices already applied.  All reads of the stage (and its
// twiddles) happen before the barrier and all writes after it, so the stage
// runs in place.
template <int R, int EMAX>
__device__ __forceinline__ void fft_stage(float2* sm, int N, int ls, int nl, int Ns,
                                          const FastDiv& fnb, const FastDiv& fns,
                                          const float2* __restrict__ tw) {
  constexpr int NB = (EMAX + R - 1) / R;
  const int nb = N / R;
  const int total = nl * nb;
  const int step = N / (Ns * R);
  float2 val[NB][R];
  int line[NB], jq[NB], kk[NB];     // butterfly j = jq Ns + k of line l, kept across the barrier
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int bi = threadIdx.x + t * kBlock;
    line[t] = -1;
    jq[t] = 0;
    kk[t] = 0;
    if (bi < total) {
      const int l = (int)fdiv((uint32_t)bi, fnb);
      const int j = bi - l * nb;
      line[t] = l;
      jq[t] = (int)fdiv((uint32_t)j, fns);
      kk[t] = j - jq[t] * Ns;
      const float2* src = sm + l * ls + j;
#pragma unroll
      for (int q = 0; q < R; ++q) val[t][q] = src[q * nb];
      if (Ns > 1) {
        const int k = kk[t];
#pragma unroll
        for (int q = 1; q < R; ++q) val[t][q] = cmul(val[t][q], tw[q * k * step]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    if (line[t] >= 0) {
      radix_dft<R>(val[t]);
      float2* dst = sm + line[t] * ls + jq[t] * Ns * R + kk[t];
#pragma unroll
      for (int q = 0; q < R; ++q) dst[q * Ns] = val[t][q];
    }
  }
  __syncthreads();
}

// Forward DFT of nl lines of length p.n in LDS (line stride ls; natural order in and out).
// Requires nl * p.n <= 256 * EMAX (each thread holds at most EMAX values per stage).
template <int EMAX>
__device__ __forceinline__ void lds_fft(float2* sm, int ls, int nl, const FFTPlan& p,
                                        const float2* __restrict__ tw) {
  int Ns = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int R = p.radix[s];
    switch (R) {
      case 2: fft_stage<2, EMAX>(sm, p.n, ls, nl, Ns, p.fnb[s], p.fns[s], tw); break;
      case 3: fft_stage<3, EMAX>(sm, p.n, ls, nl, Ns, p.fnb[s], p.fns[s], tw); break;
      case 4: fft_stage<4, EMAX>(sm, p.n, ls, nl, Ns, p.fnb[s], p.fns[s], tw); break;
      case 5: fft_stage<5, EMAX>(sm, p.n, ls, nl, Ns, p.fnb[s], p.fns[s], tw); break;
      case 7: fft_stage<7, EMAX>(sm, p.n, ls, nl, Ns, p.fnb[s], p.fns[s], tw); break;
      default: fft_stage<8, EMAX>(sm, p.n, ls, nl, Ns, p.fnb[s], p.fns[s], tw); break;
    }
    Ns *= R;
  }
}

__device__ __forceinline__ bool gate(const State* st, int need_mode) {
  return need_mode < 0 || st->mode == need_mode;
}

// Tile geometry of one FFT block: `nl` lines of length N, line stride `ls` in LDS.
// Every thread moves at most EMAX elements between HBM and LDS; all of its global
// loads are issued before any LDS write so their latencies overlap.

// Every block first copies the N twiddles of its axis into LDS, after its tile
// (rounded up to 16 elements): each stage reads up to R - 1 twiddles per
// butterfly, and from LDS these no longer put an L2 round trip into every stage.
__device__ __forceinline__ int tw_offset(int tile_elems) { return (tile_elems + 15) & ~15; }

__device__ __forceinline__ const float2* stage_twiddles(float2* sm, int tile_elems,
                                                        const float2* __restrict__ tw, int N) {
  float2* t = sm + tw_offset(tile_elems);
  for (int e = threadIdx.x; e < N; e += kBlock) t[e] = tw[e];
  return t;
}

// ------------------------------------ y and z passes, compile-time plans ----
// A line of length N = N1 N2 is transformed by G = max(N1, N2) threads in two
// steps with one exchange through LDS:
//   x[n1 + N1 n2] --(N2-point DFT over n2, thread n1)--> Y[n1][k2]
//   --(times W_N^(n1 k2))--> --(N1-point DFT over n1, thread k2)--> X[k2 + N2 k1].
// A tile is kCT consecutive kx columns of one (component, plane); thread
// (c, t) = (tid mod kCT, tid / kCT), so the kCT lanes of a row move one
// 128-byte segment.  Each thread loads its N2 values straight from global
// memory and stores its N1 results there; only the exchange goes through LDS
// (line stride N + 1).  The z pass keeps the spectrum in registers between the
// forward transform, the K multiply and the inverse transform; the inverse runs
// the same split the other way round (k2 + N2 k1 -> p1 + N1 p2), which takes the
// forward output order as it is and returns natural order.
// Every index is a compile-time constant or a per-thread offset, so the stages
// spend their instructions on the butterflies.  Lengths without a plan use the
// runtime-planned passes above.

constexpr int kCT = 16;   // kx columns per tile of a compile-time pass

#define LDDMM_CT_PLANS(X) \
  X(240, 16, 15) X(160, 16, 10) X(120, 12, 10) X(80, 10, 8) X(60, 10, 6) X(40, 8, 5) \
  X(32, 8, 4) X(64, 8, 8) X(96, 12, 8) X(128, 16, 8) X(70, 10, 7) X(140, 14, 10) \
  X(72, 12, 6) X(75, 15, 5) X(81, 9, 9) X(84, 12, 7) X(90, 15, 6) X(98, 14, 7) \
  X(100, 10, 10) X(105, 15, 7) X(108, 12, 9) X(112, 16, 7) X(126, 14, 9) X(135, 15, 9) \
  X(144, 12, 12) X(150, 15, 10)

static bool ct_plan(int n, int* n1, int* n2) {
#define LDDMM_CT_CASE(N, A, B) \
  if (n == N) {                \
    *n1 = A;                   \
    *n2 = B;                   \
    return true;               \
  }
  LDDMM_CT_PLANS(LDDMM_CT_CASE)
#undef LDDMM_CT_CASE
  return false;
}

// LDS of one compile-time tile: the exchange, the twiddles and (z pass) the
// K symbol tables.
static size_t ct_lds_bytes(int n) {
  return sizeof(float2) * ((size_t)kCT * (n + 1) + n) + sizeof(float) * ((size_t)n + kCT);
}

// y pass (forward, or inverse through conj(DFT(conj X))) of columns
// bx * kCT .. + kCT - 1 of plane z of component comp.
template <int N1, int N2, bool INV>
__device__ __forceinline__ void ct_y_body(const FftPair& f, int bx, int zslab, int comp) {
  constexpr int N = N1 * N2, LS = N + 1;
  extern __shared__ float2 sm[];
  float2* sx = sm;
  float2* stw = sm + kCT * LS;
  const Geom& g = f.g;
  const int hs = g.hs;
  const int c = threadIdx.x % kCT, t = threadIdx.x / kCT;
  float2* __restrict__ col =
      f.S + (long long)comp * g.nspec + (long long)zslab * g.ny * hs + bx * kCT + c;
  const float2* __restrict__ tw = f.tw[1];
  for (int e = threadIdx.x; e < N; e += blockDim.x) stw[e] = tw[e];
  float2 v[N2];
  if (t < N1) {
#pragma unroll
    for (int q = 0; q < N2; ++q) {
      const float2 a = col[(t + N1 * q) * hs];
      v[q] = INV ? dft::conj(a) : a;
    }
  }
  __syncthreads();
  if (t < N1) {
    dft::dft<N2>(v);
#pragma unroll
    for (int q = 1; q < N2; ++q) v[q] = dft::mul(v[q], stw[t * q]);
#pragma unroll
    for (int q = 0; q < N2; ++q) sx[c * LS + t + N1 * q] = v[q];
  }
  __syncthreads();
  if (t < N2) {
    float2 w[N1];
#pragma unroll
    for (int p = 0; p < N1; ++p) w[p] = sx[c * LS + p + N1 * t];
    dft::dft<N1>(w);
#pragma unroll
    for (int k = 0; k < N1; ++k) col[(t + N2 * k) * hs] = INV ? dft::conj(w[k]) : w[k];
  }
}

// z pass: forward transform, K_hat / |P| (and conj), forward transform of the
// conjugate, conj on the way out: N_z IDFT_z(K_hat X / |P|).
template <int N1, int N2>
__device__ __forceinline__ void ct_zK_body(const FftPair& f, int bx, int ky, int comp) {
  constexpr int N = N1 * N2, LS = N + 1;
  extern __shared__ float2 sm[];
  float2* sx = sm;
  float2* stw = sm + kCT * LS;
  float* saz = reinterpret_cast<float*>(stw + N);
  float* scxy = saz + N;
  const Geom& g = f.g;
  const int hs = g.hs;
  const int zs = g.ny * hs;
  const int c = threadIdx.x % kCT, t = threadIdx.x / kCT;
  float2* __restrict__ col = f.S + (long long)comp * g.nspec + (long long)ky * hs + bx * kCT + c;
  const float2* __restrict__ tw = f.tw[2];
  const double* __restrict__ lamz = f.lam[2];
  for (int e = threadIdx.x; e < N; e += blockDim.x) {
    stw[e] = tw[e];
    saz[e] = (float)(f.alpha * lamz[e]);
  }
  if (threadIdx.x < kCT) {
    const int kx = bx * kCT + (int)threadIdx.x;
    scxy[threadIdx.x] = (float)(f.gamma + f.alpha * (f.lam[0][kx < g.hx ? kx : 0] + f.lam[1][ky]));
  }
  float2 v[N2];
  if (t < N1) {
#pragma unroll
    for (int q = 0; q < N2; ++q) v[q] = col[(t + N1 * q) * zs];
  }
  __syncthreads();
  if (t < N1) {
    dft::dft<N2>(v);
#pragma unroll
    for (int q = 1; q < N2; ++q) v[q] = dft::mul(v[q], stw[t * q]);
#pragma unroll
    for (int q = 0; q < N2; ++q) sx[c * LS + t + N1 * q] = v[q];
  }
  __syncthreads();
  float2 w[N1];
  if (t < N2) {
#pragma unroll
    for (int p = 0; p < N1; ++p) w[p] = sx[c * LS + p + N1 * t];
    dft::dft<N1>(w);
    const float inv_n = (float)(1.0 / ((double)g.nx * (double)g.ny * (double)g.nz));
    const float cxy = scxy[c];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      const float d = cxy + saz[t + N2 * k];
      const float kh = inv_n * __builtin_amdgcn_rcpf(d * d);
      w[k] = make_float2(w[k].x * kh, -w[k].y * kh);          // conj(K_hat X / |P|)
    }
    dft::dft<N1>(w);
#pragma unroll
    for (int p = 1; p < N1; ++p) w[p] = dft::mul(w[p], stw[t * p]);
  }
  __syncthreads();
  if (t < N2) {
#pragma unroll
    for (int p = 0; p < N1; ++p) sx[c * LS + t + N2 * p] = w[p];
  }
  __syncthreads();
  if (t < N1) {
    float2 u[N2];
#pragma unroll
    for (int q = 0; q < N2; ++q) u[q] = sx[c * LS + q + N2 * t];
    dft::dft<N2>(u);
#pragma unroll
    for (int q = 0; q < N2; ++q) col[(t + N1 * q) * zs] = dft::conj(u[q]);
  }
}

template <int N1, int N2, bool INV>
__global__ __launch_bounds__(kCT * (N1 > N2 ? N1 : N2)) void k_fftc_y(FftPair f) {
  if (!gate(f.st, f.need_mode)) return;
  ct_y_body<N1, N2, INV>(f, blockIdx.x, blockIdx.y, blockIdx.z);
}

// XCD-aware tile order as in k_fft_z_K.
template <int N1, int N2>
__global__ __launch_bounds__(kCT * (N1 > N2 ? N1 : N2)) void k_fftc_zK(FftPair f) {
  if (!gate(f.st, f.need_mode)) return;
  const uint32_t total = gridDim.x;
  uint32_t t = blockIdx.x;
  if ((total % kXCD) == 0) t = (t % kXCD) * (total / kXCD) + t / kXCD;
  const int bx = (int)(t % (uint32_t)f.nbx_z), r = (int)(t / (uint32_t)f.nbx_z);
  ct_zK_body<N1, N2>(f, bx, r % f.g.ny, r / f.g.ny);
}

// The compile-time body for this problem's length, if it has one (batched
// launches: 256 threads, kCT x 16, of which the plan uses kCT x G).
template <bool INV>
__device__ __forceinline__ bool ct_y_dispatch(const FftPair& f, int bx, int zslab, int comp) {
  switch (f.g.ny) {
#define LDDMM_CT_CASE(N, A, B)              \
  case N:                                   \
    ct_y_body<A, B, INV>(f, bx, zslab, comp); \
    return true;
    LDDMM_CT_PLANS(LDDMM_CT_CASE)
#undef LDDMM_CT_CASE
    default:
      return false;
  }
}

__device__ __forceinline__ bool ct_zK_dispatch(const FftPair& f, int bx, int ky, int comp) {
  switch (f.g.nz) {
#define LDDMM_CT_CASE(N, A, B)          \
  case N:                               \
    ct_zK_body<A, B>(f, bx, ky, comp); \
    return true;
    LDDMM_CT_PLANS(LDDMM_CT_CASE)
#undef LDDMM_CT_CASE
    default:
      return false;
  }
}

// ------------------------------------------- x passes, compile-time plans ----
// Rows are packed two by two into complex lines as in the runtime-planned x
// passes (3 lines per row pair: bx and by of each row, bz of both).  A block
// holds kXP(G) row pairs, 3 kXP lines of length N = N1 N2, one line per G
// threads.  Loads and stores stay row-contiguous through LDS (line stride N + 1);
// the two factor steps run in registers between them: step A in place (a thread
// reads and writes the same positions), step B through registers.

#define LDDMM_CTX_PLANS(X) LDDMM_CT_PLANS(X) X(280, 20, 14)

// Row pairs per block of a compile-time x pass: as many as fit 256 threads.
__host__ __device__ constexpr int kXP(int G) { return kBlock / (3 * G); }

static bool ctx_plan(int n, int* n1, int* n2) {
#define LDDMM_CT_CASE(N, A, B) \
  if (n == N) {                \
    *n1 = A;                   \
    *n2 = B;                   \
    return true;               \
  }
  LDDMM_CTX_PLANS(LDDMM_CT_CASE)
#undef LDDMM_CT_CASE
  return false;
}

// In-LDS transform of the block's lines: natural order in sx[l LS + x] and out.
template <int N1, int N2, int LPB>
__device__ __forceinline__ void ct_lines(float2* sx, const float2* stw) {
  constexpr int N = N1 * N2, G = N1 > N2 ? N1 : N2, LS = N + 1;
  const int l = threadIdx.x / G, t = threadIdx.x % G;
  if (l < LPB && t < N1) {
    float2 v[N2];
#pragma unroll
    for (int q = 0; q < N2; ++q) v[q] = sx[l * LS + t + N1 * q];
    dft::dft<N2>(v);
#pragma unroll
    for (int q = 1; q < N2; ++q) v[q] = dft::mul(v[q], stw[t * q]);
#pragma unroll
    for (int q = 0; q < N2; ++q) sx[l * LS + t + N1 * q] = v[q];
  }
  __syncthreads();
  float2 w[N1];
  if (l < LPB && t < N2) {
#pragma unroll
    for (int p = 0; p < N1; ++p) w[p] = sx[l * LS + p + N1 * t];
    dft::dft<N1>(w);
  }
  __syncthreads();
  if (l < LPB && t < N2) {
#pragma unroll
    for (int k = 0; k < N1; ++k) sx[l * LS + t + N2 * k] = w[k];
  }
  __syncthreads();
}

// 16-byte global accesses of the x passes when rows allow them: a row of N floats
// (and each component plane) starts on a 16-byte boundary when 4 divides N.
template <int N>
struct XVec {
  static constexpr bool on = (N % 4) == 0;
};

__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ void st4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }

template <int N1, int N2>
__device__ __forceinline__ void ctx_fwd_body(const FftPair& f, int block) {
  constexpr int N = N1 * N2, G = N1 > N2 ? N1 : N2, LS = N + 1, HX = N / 2 + 1;
  constexpr int PPB = kXP(G), LPB = 3 * PPB;
  extern __shared__ float2 sm[];
  float2* sx = sm;
  float2* stw = sm + LPB * LS;
  const float* __restrict__ b = f.b;
  float2* __restrict__ S = f.S;
  const Geom& g = f.g;
  const long long n = g.n;
  const int nrows = g.ny * g.nz, hs = g.hs;
  const int pair0 = block * PPB;
  const float2* __restrict__ tw = f.tw[0];
  for (int e = threadIdx.x; e < N; e += blockDim.x) stw[e] = tw[e];
  // line l of the block: which = l mod 3 picks (bx, by) of row r0, of row r1, or bz of both
  auto row_src = [&](int l, const float*& pa, const float*& pb) {
    const int pp = l / 3, which = l - 3 * pp;
    const int r0 = 2 * (pair0 + pp), r1 = r0 + 1;
    pa = pb = nullptr;
    if (which == 0) {
      if (r0 < nrows) { pa = b + (long long)r0 * N; pb = b + n + (long long)r0 * N; }
    } else if (which == 1) {
      if (r1 < nrows) { pa = b + (long long)r1 * N; pb = b + n + (long long)r1 * N; }
    } else {
      if (r0 < nrows) pa = b + 2 * n + (long long)r0 * N;
      if (r1 < nrows) pb = b + 2 * n + (long long)r1 * N;
    }
  };
  if constexpr (XVec<N>::on) {
    constexpr int N4 = N / 4;
    constexpr int PER = (LPB * N4 + 3 * PPB * G - 1) / (3 * PPB * G);
    float4 ta[PER], tb[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = threadIdx.x + r * blockDim.x;
      ta[r] = tb[r] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < LPB * N4) {
        const int l = e / N4, x4 = e - l * N4;
        const float *pa, *pb;
        row_src(l, pa, pb);
        if (pa) ta[r] = ld4(pa + 4 * x4);
        if (pb) tb[r] = ld4(pb + 4 * x4);
      }
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = threadIdx.x + r * blockDim.x;
      if (e < LPB * N4) {
        const int l = e / N4, x = 4 * (e - l * N4);
        float2* d = sx + l * LS + x;
        d[0] = make_float2(ta[r].x, tb[r].x);
        d[1] = make_float2(ta[r].y, tb[r].y);
        d[2] = make_float2(ta[r].z, tb[r].z);
        d[3] = make_float2(ta[r].w, tb[r].w);
      }
    }
  } else {
    constexpr int PER = (LPB * N + 3 * PPB * G - 1) / (3 * PPB * G);
    float2 tmp[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = threadIdx.x + r * blockDim.x;
      float2 z = make_float2(0.f, 0.f);
      if (e < LPB * N) {
        const int l = e / N, x = e - l * N;
        const float *pa, *pb;
        row_src(l, pa, pb);
        z = make_float2(pa ? pa[x] : 0.f, pb ? pb[x] : 0.f);
      }
      tmp[r] = z;
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = threadIdx.x + r * blockDim.x;
      if (e < LPB * N) {
        const int l = e / N, x = e - l * N;
        sx[l * LS + x] = tmp[r];
      }
    }
  }
  __syncthreads();
  ct_lines<N1, N2, LPB>(sx, stw);
  // Hermitian split: A = (Z[k] + conj Z[N-k]) / 2, B = (Z[k] - conj Z[N-k]) / 2i.
  // With 16-byte stores each thread writes k and k + 1; the pair past HX - 1 lands
  // in the row's padding (hs > HX), which no pass reads.
  auto split = [&](int l, int k, float2& A, float2& B) {
    const float2 zk = sx[l * LS + k];
    const float2 zm = dft::conj(sx[l * LS + (k == 0 ? 0 : N - k)]);
    A = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
    B = make_float2(0.5f * (zk.y - zm.y), -0.5f * (zk.x - zm.x));
  };
  constexpr int KV = XVec<N>::on ? 2 : 1;              // spectrum entries per store
  constexpr int HK = (HX + KV - 1) / KV;
  for (int e = threadIdx.x; e < LPB * HK; e += blockDim.x) {
    const int l = e / HK, k = KV * (e - l * HK);
    const int pp = l / 3, which = l - 3 * pp;
    const int r0 = 2 * (pair0 + pp), r1 = r0 + 1;
    float2 A0, B0, A1, B1;
    split(l, k, A0, B0);
    if (KV == 2) split(l, k + 1, A1, B1);
    auto put = [&](long long at, float2 x0, float2 x1) {
      if (KV == 2)
        *reinterpret_cast<float4*>(S + at) = make_float4(x0.x, x0.y, x1.x, x1.y);
      else
        S[at] = x0;
    };
    if (which == 0) {
      if (r0 < nrows) {
        put((long long)r0 * hs + k, A0, A1);
        put(g.nspec + (long long)r0 * hs + k, B0, B1);
      }
    } else if (which == 1) {
      if (r1 < nrows) {
        put((long long)r1 * hs + k, A0, A1);
        put(g.nspec + (long long)r1 * hs + k, B0, B1);
      }
    } else {
      if (r0 < nrows) put(2 * g.nspec + (long long)r0 * hs + k, A0, A1);
      if (r1 < nrows) put(2 * g.nspec + (long long)r1 * hs + k, B0, B1);
    }
  }
}

template <int N1, int N2>
__device__ __forceinline__ void ctx_inv_body(const FftPair& f, const UpdArgs& u, int block) {
  constexpr int N = N1 * N2, G = N1 > N2 ? N1 : N2, LS = N + 1, HX = N / 2 + 1;
  constexpr int PPB = kXP(G), LPB = 3 * PPB;
  constexpr bool V = XVec<N>::on;
  const State* st = u.st;
  extern __shared__ float2 sm[];
  float2* sx = sm;
  float2* stw = sm + LPB * LS;
  const float2* __restrict__ S = f.S;
  const Geom& g = f.g;
  const long long n = g.n;
  const int nrows = g.ny * g.nz, hs = g.hs;
  const int pair0 = block * PPB;
  const float2* __restrict__ tw = f.tw[0];
  for (int e = threadIdx.x; e < N; e += blockDim.x) stw[e] = tw[e];
  // Each half-spectrum value is read once and written to k and to its mirror N - k,
  // as conj(Z) with Z = A + i B for the forward transform of the inverse; the upper
  // half holds Z[N - k] = conj A[k] + i conj B[k].  With 16-byte loads a thread takes
  // k and k + 1 (the entry past HX - 1 is row padding and is dropped).
  constexpr int KV = V ? 2 : 1;
  constexpr int HK = (HX + KV - 1) / KV;
  constexpr int PER = (LPB * HK + 3 * PPB * G - 1) / (3 * PPB * G);
  float4 tA[PER], tB[PER];          // (A_k, A_k+1), (B_k, B_k+1); .zw unused when KV = 1
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int e = threadIdx.x + r * blockDim.x;
    float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = A;
    if (e < LPB * HK) {
      const int l = e / HK, k = KV * (e - l * HK);
      const int pp = l / 3, which = l - 3 * pp;
      const int r0 = 2 * (pair0 + pp), r1 = r0 + 1;
      auto get = [&](long long at) {
        if (V) return *reinterpret_cast<const float4*>(S + at);
        const float2 z = S[at];
        return make_float4(z.x, z.y, 0.f, 0.f);
      };
      if (which == 0) {
        if (r0 < nrows) {
          A = get((long long)r0 * hs + k);
          B = get(g.nspec + (long long)r0 * hs + k);
        }
      } else if (which == 1) {
        if (r1 < nrows) {
          A = get((long long)r1 * hs + k);
          B = get(g.nspec + (long long)r1 * hs + k);
        }
      } else {
        if (r0 < nrows) A = get(2 * g.nspec + (long long)r0 * hs + k);
        if (r1 < nrows) B = get(2 * g.nspec + (long long)r1 * hs + k);
      }
    }
    tA[r] = A;
    tB[r] = B;
  }
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int e = threadIdx.x + r * blockDim.x;
    if (e < LPB * HK) {
      const int l = e / HK, k0 = KV * (e - l * HK);
#pragma unroll
      for (int q = 0; q < KV; ++q) {
        const int k = k0 + q;
        if (k >= HX) continue;
        const float2 A = q ? make_float2(tA[r].z, tA[r].w) : make_float2(tA[r].x, tA[r].y);
        const float2 B = q ? make_float2(tB[r].z, tB[r].w) : make_float2(tB[r].x, tB[r].y);
        sx[l * LS + k] = make_float2(A.x - B.y, -(A.y + B.x));
        if (k >= 1 && N - k >= HX) sx[l * LS + N - k] = make_float2(A.x + B.y, A.y - B.x);
      }
    }
  }
  __syncthreads();
  ct_lines<N1, N2, LPB>(sx, stw);
  // result z = conj(DFT(conj Z)): real line a = Re z = Re y, b = Im z = -Im y
  float* vA = u.vA;
  float* vB = u.vB;
  const int base = st->base;
  const float eps = (float)st->eps;
  constexpr int XV = V ? 4 : 1;                  // voxels per thread and row
  constexpr int NX = N / XV;
  for (int e = threadIdx.x; e < 2 * PPB * NX; e += blockDim.x) {
    const int q = e / NX, x = XV * (e - q * NX);
    const int pp = q >> 1, half = q & 1;
    const int row = 2 * (pair0 + pp) + half;
    if (row >= nrows) continue;
    float kb0[XV], kb1[XV], kb2[XV];
#pragma unroll
    for (int m = 0; m < XV; ++m) {
      const float2 y01 = sx[(3 * pp + half) * LS + x + m];
      const float2 y2 = sx[(3 * pp + 2) * LS + x + m];
      kb0[m] = y01.x;
      kb1[m] = -y01.y;
      kb2[m] = half ? -y2.y : y2.x;
    }
    const long long i = (long long)row * N + x;
    if (u.kind == UPD_WRITE_KB) {
#pragma unroll
      for (int m = 0; m < XV; ++m) {
        u.out[i + m] = kb0[m];
        u.out[i + n + m] = kb1[m];
        u.out[i + 2 * n + m] = kb2[m];
      }
    } else if (u.kind == UPD_WRITE_G) {
      const float* v = (u.vfix ? u.vfix : (base ? vB : vA)) + (long long)u.j * 3 * n;
      float* o = u.out + (long long)u.j * 3 * n;
#pragma unroll
      for (int m = 0; m < XV; ++m) {
        o[i + m] = 2.f * v[i + m] - kb0[m];
        o[i + n + m] = 2.f * v[i + n + m] - kb1[m];
        o[i + 2 * n + m] = 2.f * v[i + 2 * n + m] - kb2[m];
      }
    } else {
      const float* v = (base ? vB : vA) + (long long)u.j * 3 * n;
      float* vt = (base ? vA : vB) + (long long)u.j * 3 * n;
      if (V) {
        const float4 a0 = ld4(v + i), a1 = ld4(v + i + n), a2 = ld4(v + i + 2 * n);
        auto upd = [&](float4 a, const float* kb) {
          return make_float4(a.x - eps * (2.f * a.x - kb[0]), a.y - eps * (2.f * a.y - kb[1]),
                             a.z - eps * (2.f * a.z - kb[2]), a.w - eps * (2.f * a.w - kb[3]));
        };
        st4(vt + i, upd(a0, kb0));
        st4(vt + i + n, upd(a1, kb1));
        st4(vt + i + 2 * n, upd(a2, kb2));
      } else {
#pragma unroll
        for (int m = 0; m < XV; ++m) {
          const float a0 = v[i + m], a1 = v[i + n + m], a2 = v[i + 2 * n + m];
          vt[i + m] = a0 - eps * (2.f * a0 - kb0[m]);
          vt[i + n + m] = a1 - eps * (2.f * a1 - kb1[m]);
          vt[i + 2 * n + m] = a2 - eps * (2.f * a2 - kb2[m]);
        }
      }
    }
  }
}

// ------------------------------------------ fused x + y passes, LDS plane ----
// Where the half spectrum of one component's xy plane fits in LDS (hx ny complex
// values), one block per (component, z plane) transforms x and y in one pass,
// and y then x with the update on the way back, so the spectrum makes one
// round trip through HBM per direction less.  Lines pack two rows of the same
// component, Z_m = b[2m] + i b[2m + 1]; line m occupies the plane rows 2m and
// 2m + 1 (2 hx >= nx slots) and the Hermitian split turns it into those two
// half-spectrum rows in place.  The line and column transforms are the
// two-factor transforms of the other compile-time passes.  Any block size works:
// lines and columns go round by round.  (The rounding differs from the
// separate passes, which pack rows across components, within FP32 error.)
#define LDDMM_FUSED_PLANS(X) \
  X(140, 14, 10, 80, 10, 8) X(70, 10, 7, 40, 8, 5) X(32, 8, 4, 32, 8, 4) X(64, 8, 8, 64, 8, 8)

constexpr int kFusedBlock = 512;   // threads of a single-problem or time-batched launch
                                    // (batches of several problems: kBlock)
constexpr int kFusedBatch = 8;     // global loads in flight per thread in the row loops

// LDS of the fused passes: the plane, then the x and y twiddles.
static size_t fused_lds_bytes(int nx, int ny) {
  return sizeof(float2) * ((size_t)ny * (nx / 2 + 1) + nx + ny);
}

// Two-factor transforms of lines in LDS, in place, natural order in and out:
// line l at P + l * LSTR, element x at stride ES.  `nl` lines go round by round,
// blockDim / G per round.
template <int N1, int N2>
__device__ __forceinline__ void lds_lines(float2* P, int nl, int lstr, int es, const float2* tw) {
  constexpr int G = N1 > N2 ? N1 : N2;
  const int per = blockDim.x / G;
  for (int l0 = 0; l0 < nl; l0 += per) {
    const int l = l0 + (int)threadIdx.x / G, t = (int)threadIdx.x % G;
    const bool on = l < nl && (int)threadIdx.x < per * G;
    float2* line = P + (long long)l * lstr;
    if (on && t < N1) {
      float2 v[N2];
#pragma unroll
      for (int q = 0; q < N2; ++q) v[q] = line[(t + N1 * q) * es];
      dft::dft<N2>(v);
#pragma unroll
      for (int q = 1; q < N2; ++q) v[q] = dft::mul(v[q], tw[t * q]);
#pragma unroll
      for (int q = 0; q < N2; ++q) line[(t + N1 * q) * es] = v[q];
    }
    __syncthreads();
    float2 w[N1];
    if (on && t < N2) {
#pragma unroll
      for (int p = 0; p < N1; ++p) w[p] = line[(p + N1 * t) * es];
      dft::dft<N1>(w);
    }
    __syncthreads();
    if (on && t < N2) {
#pragma unroll
      for (int k = 0; k < N1; ++k) line[(t + N2 * k) * es] = w[k];
    }
    __syncthreads();
  }
}

// Forward: real b of component c, plane z -> S[c][z][ky][kx].
template <int NX1, int NX2, int NY1, int NY2>
__device__ __forceinline__ void fused_fwd_body(const FftPair& f, int c, int z) {
  constexpr int NX = NX1 * NX2, HX = NX / 2 + 1, NY = NY1 * NY2;
  constexpr int GY = NY1 > NY2 ? NY1 : NY2;
  static_assert(NY % 2 == 0 && GY <= 16, "rows pair up; 16 threads per column");
  extern __shared__ float2 sm[];
  float2* P = sm;                       // NY rows of HX
  float2* twx = P + NY * HX;
  float2* twy = twx + NX;
  const Geom& g = f.g;
  for (int e = threadIdx.x; e < NX; e += blockDim.x) twx[e] = f.tw[0][e];
  for (int e = threadIdx.x; e < NY; e += blockDim.x) twy[e] = f.tw[1][e];
  // rows of the plane into the lines: row y -> line y / 2, real (even y) or imaginary part
  // (kFusedBatch loads in flight per thread before their LDS writes)
  const float* __restrict__ src = f.b + (long long)c * g.n + (long long)z * NY * NX;
  float* Pf = reinterpret_cast<float*>(P);
  for (int e0 = 0; e0 < NY * NX; e0 += kFusedBatch * (int)blockDim.x) {
    float val[kFusedBatch];
#pragma unroll
    for (int r = 0; r < kFusedBatch; ++r) {
      const int e = e0 + r * (int)blockDim.x + (int)threadIdx.x;
      val[r] = e < NY * NX ? src[e] : 0.f;
    }
#pragma unroll
    for (int r = 0; r < kFusedBatch; ++r) {
      const int e = e0 + r * (int)blockDim.x + (int)threadIdx.x;
      if (e < NY * NX) {
        const int y = e / NX, x = e - y * NX;
        Pf[2 * ((y & ~1) * HX + x) + (y & 1)] = val[r];
      }
    }
  }
  __syncthreads();
  lds_lines<NX1, NX2>(P, NY / 2, 2 * HX, 1, twx);
  // Hermitian split of line m into rows 2m (A) and 2m + 1 (B), through registers,
  // in rounds of whole lines (all of a line's values are read before any of its
  // slots is written)
  const int lr = (4 * (int)blockDim.x) / HX;            // lines per round
  for (int m0 = 0; m0 < NY / 2; m0 += lr) {
    const int items = (NY / 2 - m0 < lr ? NY / 2 - m0 : lr) * HX;
    float2 A[4], B[4];
    int at[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = r * (int)blockDim.x + (int)threadIdx.x;
      at[r] = -1;
      if (e < items) {
        const int m = m0 + e / HX, k = e % HX;
        const float2* line = P + 2 * m * HX;
        const float2 zk = line[k];
        const float2 zm = dft::conj(line[k == 0 ? 0 : NX - k]);
        A[r] = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
        B[r] = make_float2(0.5f * (zk.y - zm.y), -0.5f * (zk.x - zm.x));
        at[r] = 2 * m * HX + k;
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (at[r] >= 0) {
        P[at[r]] = A[r];
        P[at[r] + HX] = B[r];
      }
    }
    __syncthreads();
  }
  // columns: blockDim / 16 kx per round, GY <= 16 threads per column
  const int ncol = (int)blockDim.x / 16;
  const int cl = (int)threadIdx.x % ncol, t = (int)threadIdx.x / ncol;
  float2* __restrict__ dst = f.S + (long long)c * g.nspec + (long long)z * NY * g.hs;
  for (int kx0 = 0; kx0 < HX; kx0 += ncol) {
    const int kx = kx0 + cl;
    const bool on = kx < HX && t < GY;
    if (on && t < NY1) {
      float2 v[NY2];
#pragma unroll
      for (int q = 0; q < NY2; ++q) v[q] = P[(t + NY1 * q) * HX + kx];
      dft::dft<NY2>(v);
#pragma unroll
      for (int q = 1; q < NY2; ++q) v[q] = dft::mul(v[q], twy[t * q]);
#pragma unroll
      for (int q = 0; q < NY2; ++q) P[(t + NY1 * q) * HX + kx] = v[q];
    }
    __syncthreads();
    if (on && t < NY2) {
      float2 w[NY1];
#pragma unroll
      for (int p = 0; p < NY1; ++p) w[p] = P[(p + NY1 * t) * HX + kx];
      dft::dft<NY1>(w);
#pragma unroll
      for (int k = 0; k < NY1; ++k) dst[(long long)(t + NY2 * k) * g.hs + kx] = w[k];
    }
  }
}

// Inverse: S[c][z] -> y inverse -> x inverse (Hermitian extension) -> epilogue
// (the update of v, or g, or Kb) for the rows of component c in plane z.
template <int NX1, int NX2, int NY1, int NY2>
__device__ __forceinline__ void fused_inv_body(const FftPair& f, const UpdArgs& u, int c, int z) {
  constexpr int NX = NX1 * NX2, HX = NX / 2 + 1, NY = NY1 * NY2;
  constexpr int GY = NY1 > NY2 ? NY1 : NY2;
  extern __shared__ float2 sm[];
  float2* P = sm;
  float2* twx = P + NY * HX;
  float2* twy = twx + NX;
  const Geom& g = f.g;
  const long long n = g.n;
  for (int e = threadIdx.x; e < NX; e += blockDim.x) twx[e] = f.tw[0][e];
  for (int e = threadIdx.x; e < NY; e += blockDim.x) twy[e] = f.tw[1][e];
  __syncthreads();
  // y inverse of each column, conj(DFT(conj X)), straight from the spectrum
  const int ncol = (int)blockDim.x / 16;
  const int cl = (int)threadIdx.x % ncol, t = (int)threadIdx.x / ncol;
  const float2* __restrict__ src = f.S + (long long)c * g.nspec + (long long)z * NY * g.hs;
  for (int kx0 = 0; kx0 < HX; kx0 += ncol) {
    const int kx = kx0 + cl;
    const bool on = kx < HX && t < GY;
    if (on && t < NY1) {
      float2 v[NY2];
#pragma unroll
      for (int q = 0; q < NY2; ++q) v[q] = dft::conj(src[(long long)(t + NY1 * q) * g.hs + kx]);
      dft::dft<NY2>(v);
#pragma unroll
      for (int q = 1; q < NY2; ++q) v[q] = dft::mul(v[q], twy[t * q]);
#pragma unroll
      for (int q = 0; q < NY2; ++q) P[(t + NY1 * q) * HX + kx] = v[q];
    }
    __syncthreads();
    float2 w[NY1];
    if (on && t < NY2) {
#pragma unroll
      for (int p = 0; p < NY1; ++p) w[p] = P[(p + NY1 * t) * HX + kx];
      dft::dft<NY1>(w);
    }
    __syncthreads();
    if (on && t < NY2) {
#pragma unroll
      for (int k = 0; k < NY1; ++k) P[(t + NY2 * k) * HX + kx] = dft::conj(w[k]);
    }
  }
  __syncthreads();
  // rows 2m (A) and 2m + 1 (B) -> line m holding conj(Z), Z = A + i B on the
  // lower half and its Hermitian extension on the upper (through registers, in
  // rounds of whole lines)
  const int lr = (4 * (int)blockDim.x) / HX;            // lines per round
  for (int m0 = 0; m0 < NY / 2; m0 += lr) {
    const int items = (NY / 2 - m0 < lr ? NY / 2 - m0 : lr) * HX;
    float2 lo[4], hi[4];
    int at[4], k_[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = r * (int)blockDim.x + (int)threadIdx.x;
      at[r] = -1;
      if (e < items) {
        const int m = m0 + e / HX, k = e % HX;
        const float2 A = P[2 * m * HX + k], B = P[(2 * m + 1) * HX + k];
        lo[r] = make_float2(A.x - B.y, -(A.y + B.x));
        hi[r] = make_float2(A.x + B.y, A.y - B.x);
        at[r] = 2 * m * HX;
        k_[r] = k;
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (at[r] >= 0) {
        const int k = k_[r];
        if (k < NX) P[at[r] + k] = lo[r];
        if (k >= 1 && NX - k >= HX) P[at[r] + NX - k] = hi[r];
      }
    }
    __syncthreads();
  }
  lds_lines<NX1, NX2>(P, NY / 2, 2 * HX, 1, twx);
  // result z = conj(DFT(conj Z)): row 2m = Re, row 2m + 1 = Im = -Im of the line
  const State* st = u.st;
  float* vA = u.vA;
  float* vB = u.vB;
  const int base = st->base;
  const float eps = (float)st->eps;
  const long long co = (long long)c * n + (long long)z * NY * NX;   // this plane of component c
  const long long jo = (long long)u.j * 3 * n;
  const float* vin = (u.kind == UPD_WRITE_G && u.vfix ? u.vfix : (base ? vB : vA)) + jo + co;
  float* dst = u.kind == UPD_WRITE_KB ? u.out + co
               : u.kind == UPD_WRITE_G ? u.out + jo + co : (base ? vA : vB) + jo + co;
  for (int e0 = 0; e0 < NY * NX; e0 += kFusedBatch * (int)blockDim.x) {
    float a[kFusedBatch];
#pragma unroll
    for (int r = 0; r < kFusedBatch; ++r) {
      const int e = e0 + r * (int)blockDim.x + (int)threadIdx.x;
      a[r] = (u.kind != UPD_WRITE_KB && e < NY * NX) ? vin[e] : 0.f;
    }
#pragma unroll
    for (int r = 0; r < kFusedBatch; ++r) {
      const int e = e0 + r * (int)blockDim.x + (int)threadIdx.x;
      if (e < NY * NX) {
        const int y = e / NX, x = e - y * NX;
        const float2 zz = P[(y & ~1) * HX + x];
        const float kb = (y & 1) ? -zz.y : zz.x;
        if (u.kind == UPD_WRITE_KB)
          dst[e] = kb;
        else if (u.kind == UPD_WRITE_G)
          dst[e] = 2.f * a[r] - kb;
        else
          dst[e] = a[r] - eps * (2.f * a[r] - kb);
      }
    }
  }
}

template <int NX1, int NX2, int NY1, int NY2>
__global__ __launch_bounds__(kFusedBlock) void k_fftf_xy(FftPair f) {
  if (!gate(f.st, f.need_mode)) return;
  fused_fwd_body<NX1, NX2, NY1, NY2>(f, (int)blockIdx.x / f.g.nz, (int)blockIdx.x % f.g.nz);
}

template <int NX1, int NX2, int NY1, int NY2>
__global__ __launch_bounds__(kFusedBlock) void k_fftf_yx(FftPair f, UpdArgs u) {
  if (!gate(u.st, u.need_mode)) return;
  fused_inv_body<NX1, NX2, NY1, NY2>(f, u, (int)blockIdx.x / f.g.nz, (int)blockIdx.x % f.g.nz);
}

// The fused passes of a batch whose problems share one fused plan (the time steps
// of one level), with the single-problem launch's kFusedBlock threads per block.
template <int NX1, int NX2, int NY1, int NY2>
__global__ __launch_bounds__(kFusedBlock) void k_fftf_xy_batched(BatchRef br) {
  const int p = batch_pair(br, blockIdx.x);
  const FftPair& f = ((const PairTab*)br.tab[p])->fft;
  if (!gate(f.st, f.need_mode)) return;
  const int b = (int)blockIdx.x - br.off[p];
  fused_fwd_body<NX1, NX2, NY1, NY2>(f, b / f.g.nz, b % f.g.nz);
}

template <int NX1, int NX2, int NY1, int NY2>
__global__ __launch_bounds__(kFusedBlock) void k_fftf_yx_batched(BatchRef br, int j) {
  const int p = batch_pair(br, blockIdx.x);
  const PairTab* t = (const PairTab*)br.tab[p];
  if (!gate(t->upd[j].st, t->upd[j].need_mode)) return;
  const int b = (int)blockIdx.x - br.off[p];
  fused_inv_body<NX1, NX2, NY1, NY2>(t->fft, t->upd[j], b / t->fft.g.nz, b % t->fft.g.nz);
}

static bool fused_plan(int nx, int ny) {
#define LDDMM_FUSED_CASE(NX, A, B, NY, C, D) \
  if (nx == NX && ny == NY) return true;
  LDDMM_FUSED_PLANS(LDDMM_FUSED_CASE)
#undef LDDMM_FUSED_CASE
  return false;
}

__device__ __forceinline__ bool fused_fwd_dispatch(const FftPair& f, int block) {
#define LDDMM_FUSED_CASE(NX, A, B, NY, C, D)                                  \
  if (f.g.nx == NX && f.g.ny == NY) {                                        \
    fused_fwd_body<A, B, C, D>(f, block / f.g.nz, block % f.g.nz);           \
    return true;                                                             \
  }
  LDDMM_FUSED_PLANS(LDDMM_FUSED_CASE)
#undef LDDMM_FUSED_CASE
  return false;
}

__device__ __forceinline__ bool fused_inv_dispatch(const FftPair& f, const UpdArgs& u, int block) {
#define LDDMM_FUSED_CASE(NX, A, B, NY, C, D)                                  \
  if (f.g.nx == NX && f.g.ny == NY) {                                        \
    fused_inv_body<A, B, C, D>(f, u, block / f.g.nz, block % f.g.nz);        \
    return true;                                                             \
  }
  LDDMM_FUSED_PLANS(LDDMM_FUSED_CASE)
#undef LDDMM_FUSED_CASE
  return false;
}

template <int N1, int N2>
__global__ __launch_bounds__(3 * kXP(N1 > N2 ? N1 : N2) * (N1 > N2 ? N1 : N2)) void k_fftc_x_fwd(
    FftPair f) {
  if (!gate(f.st, f.need_mode)) return;
  ctx_fwd_body<N1, N2>(f, blockIdx.x);
}

template <int N1, int N2>
__global__ __launch_bounds__(3 * kXP(N1 > N2 ? N1 : N2) * (N1 > N2 ? N1 : N2)) void k_fftc_x_inv(
    FftPair f, UpdArgs u) {
  if (!gate(u.st, u.need_mode)) return;
  ctx_inv_body<N1, N2>(f, u, blockIdx.x);
}

__device__ __forceinline__ bool ctx_fwd_dispatch(const FftPair& f, int block) {
  switch (f.g.nx) {
#define LDDMM_CT_CASE(N, A, B)     \
  case N:                          \
    ctx_fwd_body<A, B>(f, block);  \
    return true;
    LDDMM_CTX_PLANS(LDDMM_CT_CASE)
#undef LDDMM_CT_CASE
    default:
      return false;
  }
}

__device__ __forceinline__ bool ctx_inv_dispatch(const FftPair& f, const UpdArgs& u, int block) {
  switch (f.g.nx) {
#define LDDMM_CT_CASE(N, A, B)        \
  case N:                             \
    ctx_inv_body<A, B>(f, u, block);  \
    return true;
    LDDMM_CTX_PLANS(LDDMM_CT_CASE)
#undef LDDMM_CT_CASE
    default:
      return false;
  }
}

// ----------------------------------------------------------- x forward ----
// Row rho = z*ny + y.  Rows are processed in pairs (2m, 2m+1): complex lines
//   Z0 = bx[2m] + i by[2m],  Z1 = bx[2m+1] + i by[2m+1],  Z2 = bz[2m] + i bz[2m+1].
// After the DFT, for k < hx:  A[k] = (Z[k] + conj Z[-k]) / 2,  B[k] = (Z[k] - conj Z[-k]) / 2i.

template <int EMAX>
__device__ __forceinline__ void x_fwd_body(const FftPair& f, int block) {
  if (!gate(f.st, f.need_mode)) return;
  extern __shared__ float2 sm[];
  const float* __restrict__ b = f.b;
  float2* __restrict__ S = f.S;
  const Geom& g = f.g;
  const FFTPlan& p = f.px;
  const int ppb = f.ppb;
  const int N = g.nx;
  const long long n = g.n;
  const int nrows = g.ny * g.nz;
  const int pair0 = block * ppb;
  const int nl = 3 * ppb;
  const int tot = nl * N;
  const float2* tw = stage_twiddles(sm, tot, f.tw[0], N);
  float2 tmp[EMAX];
#pragma unroll
  for (int r = 0; r < EMAX; ++r) {
    const int e = threadIdx.x + r * kBlock;
    float2 z = make_float2(0.f, 0.f);
    if (e < tot) {
      const int l = (int)fdiv((uint32_t)e, g.fx), x = e - l * N;
      const int pp = l / 3, which = l - 3 * pp;
      const int r0 = 2 * (pair0 + pp), r1 = r0 + 1;
      if (which == 0) {
        if (r0 < nrows) z = make_float2(b[(long long)r0 * N + x], b[n + (long long)r0 * N + x]);
      } else if (which == 1) {
        if (r1 < nrows) z = make_float2(b[(long long)r1 * N + x], b[n + (long long)r1 * N + x]);
      } else {
        const float re = r0 < nrows ? b[2 * n + (long long)r0 * N + x] : 0.f;
        const float im = r1 < nrows ? b[2 * n + (long long)r1 * N + x] : 0.f;
        z = make_float2(re, im);
      }
    }
    tmp[r] = z;
  }
#pragma unroll
  for (int r = 0; r < EMAX; ++r) {
    const int e = threadIdx.x + r * kBlock;
    if (e < tot) sm[e] = tmp[r];
  }
  __syncthreads();
  lds_fft<EMAX>(sm, N, nl, p, tw);
  const int hx = g.hx, hs = g.hs;
  for (int e = threadIdx.x; e < nl * hx; e += kBlock) {
    const int l = (int)fdiv((uint32_t)e, g.fhx), k = e - l * hx;
    const int pp = l / 3, which = l - 3 * pp;
    const int r0 = 2 * (pair0 + pp), r1 = r0 + 1;
    const float2 zk = sm[l * N + k];
    const float2 zm = cconj(sm[l * N + (k == 0 ? 0 : N - k)]);
    const float2 A = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
    // (zk - zm) / 2i = -i/2 (zk - zm)
    const float2 B = make_float2(0.5f * (zk.y - zm.y), -0.5f * (zk.x - zm.x));
    if (which == 0) {
      if (r0 < nrows) {
        S[(long long)r0 * hs + k] = A;
        S[g.nspec + (long long)r0 * hs + k] = B;
      }
    } else if (which == 1) {
      if (r1 < nrows) {
        S[(long long)r1 * hs + k] = A;
        S[g.nspec + (long long)r1 * hs + k] = B;
      }
    } else {
      if (r0 < nrows) S[2 * g.nspec + (long long)r0 * hs + k] = A;
      if (r1 < nrows) S[2 * g.nspec + (long long)r1 * hs + k] = B;
    }
  }
}

template <int EMAX>
__global__ __launch_bounds__(kBlock) void k_fft_x_fwd(FftPair f) {
  x_fwd_body<EMAX>(f, blockIdx.x);
}

template <int EMAX>
__global__ __launch_bounds__(kBlock) void k_fft_x_fwd_batched(BatchRef br) {
  const int p = batch_pair(br, blockIdx.x);
  const FftPair& f = ((const PairTab*)br.tab[p])->fft;
  if (!gate(f.st, f.need_mode)) return;
  if (f.fused && fused_fwd_dispatch(f, blockIdx.x - br.off[p])) return;
  if (ctx_fwd_dispatch(f, blockIdx.x - br.off[p])) return;
  x_fwd_body<EMAX>(f, blockIdx.x - br.off[p]);
}

// Launch-shape tunables of the FFT passes (results do not depend on them: every
// line is transformed the same way whatever the tile it shares a block with).
static int g_x_elems = kFFTElems;     // complex values per x-pass block
static int g_col_cap[2] = {16, 8};    // kx columns per y tile, per z tile

void set_fft_x_elems(int e) { g_x_elems = e < 256 ? 256 : (e > 8192 ? 8192 : e); }

static int pow2_cap(int c) {
  int t = 2;
  while (t * 2 <= c && t < 32) t *= 2;
  return t;
}
void set_fft_cols(int axis, int c) { g_col_cap[axis] = pow2_cap(c); }

// Row pairs per block of the x passes and the register budget they need.
static int pairs_per_block(int N, int* emax) {
  int ppb = g_x_elems / (3 * N);
  if (ppb < 1) ppb = 1;
  if (ppb > 8) ppb = 8;
  const int tot = 3 * ppb * N;
  *emax = tot <= kBlock * 8 ? 8 : (tot <= kBlock * 16 ? 16 : 32);
  return ppb;
}

// ------------------------------------------------------ y and z passes ----
// Tile: TX consecutive kx of one (component, slab), all N points along the
// transform axis; line c of the tile is the column kx0 + c (LDS stride N + 1,
// so the transposing writes spread over the banks).

static int ilog2(int v) {
  int k = 0;
  while ((1 << (k + 1)) <= v) ++k;
  return k;
}

static int tile_cols(int N, int axis, int* emax) {
  int tx = g_col_cap[axis];
  while (tx > 2 && tx * N > 2 * kFFTElems) tx >>= 1;
  const int tot = tx * N;
  *emax = tot <= kBlock * 8 ? 8 : (tot <= kBlock * 16 ? 16 : 32);
  return tx;
}

template <int EMAX, bool INV>
__device__ __forceinline__ void tile_load(float2* sm, const float2* __restrict__ base, int lgTX,
                                          int N, int ls, int hx, int kx0, int stride) {
  float2 tmp[EMAX];
  const int TX = 1 << lgTX;
  const int tot = TX * N;
#pragma unroll
  for (int r = 0; r < EMAX; ++r) {
    const int e = threadIdx.x + r * kBlock;
    float2 v = make_float2(0.f, 0.f);
    if (e < tot) {
      const int c = e & (TX - 1), y = e >> lgTX;
      if (kx0 + c < hx) v = base[y * stride + kx0 + c];
    }
    tmp[r] = INV ? cconj(v) : v;
  }
#pragma unroll
  for (int r = 0; r < EMAX; ++r) {
    const int e = threadIdx.x + r * kBlock;
    if (e < tot) {
      const int c = e & (TX - 1), y = e >> lgTX;
      sm[c * ls + y] = tmp[r];
    }
  }
  __syncthreads();
}

template <bool INV>
__device__ __forceinline__ void tile_store(const float2* sm, float2* __restrict__ base, int lgTX,
                                           int N, int ls, int hx, int kx0, int stride) {
  const int TX = 1 << lgTX;
  for (int e = threadIdx.x; e < TX * N; e += kBlock) {
    const int c = e & (TX - 1), y = e >> lgTX;
    if (kx0 + c < hx) {
      const float2 v = sm[c * ls + y];
      base[y * stride + kx0 + c] = INV ? cconj(v) : v;
    }
  }
}

template <int EMAX, bool INV>
__device__ __forceinline__ void y_body(const FftPair& f, int bx, int bz_slab, int comp) {
  if (!gate(f.st, f.need_mode)) return;
  extern __shared__ float2 sm[];
  const Geom& g = f.g;
  const int lgTX = f.lgTXy;
  const int N = g.ny, hx = g.hx, hs = g.hs, ls = N + 1;
  const int TX = 1 << lgTX;
  const int kx0 = bx * TX;
  float2* base = f.S + (long long)comp * g.nspec + (long long)bz_slab * g.ny * hs;
  const float2* tw = stage_twiddles(sm, TX * ls, f.tw[1], N);
  tile_load<EMAX, INV>(sm, base, lgTX, N, ls, hx, kx0, hs);
  lds_fft<EMAX>(sm, ls, TX, f.py, tw);
  tile_store<INV>(sm, base, lgTX, N, ls, hx, kx0, hs);
}

template <int EMAX, bool INV>
__global__ __launch_bounds__(kBlock) void k_fft_y(FftPair f) {
  y_body<EMAX, INV>(f, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <int EMAX, bool INV>
__global__ __launch_bounds__(kBlock) void k_fft_y_batched(BatchRef br) {
  const int p = batch_pair(br, blockIdx.x);
  const FftPair& f = ((const PairTab*)br.tab[p])->fft;
  const int t = blockIdx.x - br.off[p];
  const int bx = t % f.nbx_y, r = t / f.nbx_y;
  if (!gate(f.st, f.need_mode)) return;
  if (ct_y_dispatch<INV>(f, bx, r % f.g.nz, r / f.g.nz)) return;
  y_body<EMAX, INV>(f, bx, r % f.g.nz, r / f.g.nz);
}

template <int EMAX>
__device__ __forceinline__ void zK_body(const FftPair& f, int bx, int ky, int comp) {
  if (!gate(f.st, f.need_mode)) return;
  extern __shared__ float2 sm[];
  const Geom& g = f.g;
  const int lgTX = f.lgTXz;
  const int N = g.nz, hx = g.hx, ls = N + 1;
  const int TX = 1 << lgTX;
  const int kx0 = bx * TX;
  const int zs = g.ny * g.hs;
  float2* base = f.S + (long long)comp * g.nspec + (long long)ky * g.hs;
  const float2* tw = stage_twiddles(sm, TX * ls, f.tw[2], N);
  tile_load<EMAX, false>(sm, base, lgTX, N, ls, hx, kx0, zs);
  lds_fft<EMAX>(sm, ls, TX, f.pz, tw);
  const double inv_n = 1.0 / ((double)g.nx * (double)g.ny * (double)g.nz);
  const double* __restrict__ lamx = f.lam[0];
  const double* __restrict__ lamz = f.lam[2];
  const double lyy = f.lam[1][ky];
  for (int e = threadIdx.x; e < TX * N; e += kBlock) {
    const int c = (int)fdiv((uint32_t)e, g.fz), kz = e - c * N;
    const int kx = kx0 + c < hx ? kx0 + c : 0;
    const double lam = f.alpha * (lamx[kx] + lyy + lamz[kz]) + f.gamma;
    const float kh = (float)(inv_n / (lam * lam));
    const float2 v = sm[c * ls + kz];
    sm[c * ls + kz] = make_float2(v.x * kh, -v.y * kh);     // conj(K_hat X / |P|)
  }
  __syncthreads();
  lds_fft<EMAX>(sm, ls, TX, f.pz, tw);
  tile_store<true>(sm, base, lgTX, N, ls, hx, kx0, zs);
}

// One block per tile, in an XCD-aware order: consecutive block indices go to
// the accelerator dies in turn, so block L takes tile (L mod 8) * (tiles / 8) +
// L / 8 and every die works through a contiguous run of tiles.  Neighbouring kx
// tiles (two 8-column tiles share each 128-byte line of a z row) then run at
// the same time behind the same L2 instead of fetching each line twice.
template <int EMAX>
__global__ __launch_bounds__(kBlock) void k_fft_z_K(FftPair f) {
  const uint32_t total = gridDim.x;
  uint32_t t = blockIdx.x;
  if ((total % kXCD) == 0) t = (t % kXCD) * (total / kXCD) + t / kXCD;
  const int bx = (int)(t % (uint32_t)f.nbx_z), r = (int)(t / (uint32_t)f.nbx_z);
  zK_body<EMAX>(f, bx, r % f.g.ny, r / f.g.ny);
}

template <int EMAX>
__global__ __launch_bounds__(kBlock) void k_fft_z_K_batched(BatchRef br) {
  const int p = batch_pair(br, blockIdx.x);
  const FftPair& f = ((const PairTab*)br.tab[p])->fft;
  const int t = blockIdx.x - br.off[p];
  const int bx = t % f.nbx_z, r = t / f.nbx_z;
  if (!gate(f.st, f.need_mode)) return;
  if (ct_zK_dispatch(f, bx, r % f.g.ny, r / f.g.ny)) return;
  zK_body<EMAX>(f, bx, r % f.g.ny, r / f.g.ny);
}

// ----------------------------------------------------- x inverse + update ----
// Rebuild the full spectrum of each packed line from the half spectra
// (Z'[k] = A[k] + i B[k] for k < hx, conj A[N-k] + i conj B[N-k] above),
// invert, and split real / imaginary parts back into the two real lines.

template <int EMAX>
__device__ __forceinline__ void x_inv_body(const FftPair& f, const UpdArgs& u, int block) {
  const State* st = u.st;
  if (!gate(st, u.need_mode)) return;
  extern __shared__ float2 sm[];
  const float2* __restrict__ S = f.S;
  const Geom& g = f.g;
  const FFTPlan& p = f.px;
  const int ppb = f.ppb;
  const int N = g.nx, hx = g.hx, hs = g.hs;
  const long long n = g.n;
  const int nrows = g.ny * g.nz;
  const int pair0 = block * ppb;
  const int nl = 3 * ppb;
  const int tot = nl * N;
  const float2* tw = stage_twiddles(sm, tot, f.tw[0], N);
  // each half-spectrum value is read once and written to k and to its mirror N - k
  const int toth = nl * hx;
  float2 tA[EMAX], tB[EMAX];
#pragma unroll
  for (int r = 0; r < EMAX; ++r) {
    const int e = threadIdx.x + r * kBlock;
    float2 A = make_float2(0.f, 0.f), B = make_float2(0.f, 0.f);
    if (e < toth) {
      const int l = (int)fdiv((uint32_t)e, g.fhx), k = e - l * hx;
      const int pp = l / 3, which = l - 3 * pp;
      const int r0 = 2 * (pair0 + pp), r1 = r0 + 1;
      if (which == 0) {
        if (r0 < nrows) {
          A = S[(long long)r0 * hs + k];
          B = S[g.nspec + (long long)r0 * hs + k];
        }
      } else if (which == 1) {
        if (r1 < nrows) {
          A = S[(long long)r1 * hs + k];
          B = S[g.nspec + (long long)r1 * hs + k];
        }
      } else {
        if (r0 < nrows) A = S[2 * g.nspec + (long long)r0 * hs + k];
        if (r1 < nrows) B = S[2 * g.nspec + (long long)r1 * hs + k];
      }
    }
    tA[r] = A;
    tB[r] = B;
  }
#pragma unroll
  for (int r = 0; r < EMAX; ++r) {
    const int e = threadIdx.x + r * kBlock;
    if (e < toth) {
      const int l = (int)fdiv((uint32_t)e, g.fhx), k = e - l * hx;
      const float2 A = tA[r], B = tB[r];
      // Z = A + i B, stored as conj(Z) for the forward transform of the inverse;
      // the upper half holds Z[N - k] = conj A[k] + i conj B[k]
      sm[l * N + k] = make_float2(A.x - B.y, -(A.y + B.x));
      if (k >= 1 && N - k >= hx) sm[l * N + N - k] = make_float2(A.x + B.y, A.y - B.x);
    }
  }
  __syncthreads();
  lds_fft<EMAX>(sm, N, nl, p, tw);
  // result z = conj(DFT(conj Z)): real line a = Re z = Re y, b = Im z = -Im y
  float* vA = u.vA;
  float* vB = u.vB;
  const int base = st->base;
  const float eps = (float)st->eps;
  for (int e = threadIdx.x; e < 2 * ppb * N; e += kBlock) {
    const int q = (int)fdiv((uint32_t)e, g.fx), x = e - q * N;
    const int pp = q >> 1, half = q & 1;
    const int row = 2 * (pair0 + pp) + half;
    if (row >= nrows) continue;
    const float2 y01 = sm[(3 * pp + half) * N + x];
    const float2 y2 = sm[(3 * pp + 2) * N + x];
    const float kb0 = y01.x, kb1 = -y01.y, kb2 = half ? -y2.y : y2.x;
    const long long i = (long long)row * N + x;
    if (u.kind == UPD_WRITE_KB) {
      u.out[i] = kb0;
      u.out[i + n] = kb1;
      u.out[i + 2 * n] = kb2;
    } else if (u.kind == UPD_WRITE_G) {
      const float* v = (u.vfix ? u.vfix : (base ? vB : vA)) + (long long)u.j * 3 * n;
      float* o = u.out + (long long)u.j * 3 * n;
      o[i] = 2.f * v[i] - kb0;
      o[i + n] = 2.f * v[i + n] - kb1;
      o[i + 2 * n] = 2.f * v[i + 2 * n] - kb2;
    } else {
      const float* v = (base ? vB : vA) + (long long)u.j * 3 * n;
      float* vt = (base ? vA : vB) + (long long)u.j * 3 * n;
      const float a0 = v[i], a1 = v[i + n], a2 = v[i + 2 * n];
      vt[i] = a0 - eps * (2.f * a0 - kb0);
      vt[i + n] = a1 - eps * (2.f * a1 - kb1);
      vt[i + 2 * n] = a2 - eps * (2.f * a2 - kb2);
    }
  }
}

template <int EMAX>
__global__ __launch_bounds__(kBlock) void k_fft_x_inv(FftPair f, UpdArgs u) {
  x_inv_body<EMAX>(f, u, blockIdx.x);
}

template <int EMAX>
__global__ __launch_bounds__(kBlock) void k_fft_x_inv_batched(BatchRef br, int j) {
  const int p = batch_pair(br, blockIdx.x);
  const PairTab* t = (const PairTab*)br.tab[p];
  if (!gate(t->upd[j].st, t->upd[j].need_mode)) return;
  if (t->fft.fused && fused_inv_dispatch(t->fft, t->upd[j], blockIdx.x - br.off[p])) return;
  if (ctx_inv_dispatch(t->fft, t->upd[j], blockIdx.x - br.off[p])) return;
  x_inv_body<EMAX>(t->fft, t->upd[j], blockIdx.x - br.off[p]);
}

// ------------------------------------------------------------- launchers ----

// Largest LDS of the fused x + y passes (0: never fuse).  Above 80 KB a CU
// holds one block; the finest atlas level would need 180 KB.
static int g_fused_lds = 80 * 1024;

void set_fft_fused_lds(int bytes) { g_fused_lds = bytes < 0 ? 0 : bytes; }

// Fill the per-problem tile geometry of the five passes (three when fused).
void fft_tiles(FftPair& f, FftLaunch* L) {
  int ex, ey, ez, n1, n2;
  const bool cx = ctx_plan(f.g.nx, &n1, &n2);
  f.ppb = cx ? kXP(n1 > n2 ? n1 : n2) : pairs_per_block(f.g.nx, &ex);
  if (cx) ex = 8;
  const bool cy = ct_plan(f.g.ny, &n1, &n2), cz = ct_plan(f.g.nz, &n1, &n2);
  const int ty = cy ? kCT : tile_cols(f.g.ny, 0, &ey);
  const int tz = cz ? kCT : tile_cols(f.g.nz, 1, &ez);
  if (cy) ey = 8;
  if (cz) ez = 8;
  f.lgTXy = ilog2(ty);
  f.lgTXz = ilog2(tz);
  f.nbx_y = (f.g.hx + ty - 1) / ty;
  f.nbx_z = (f.g.hx + tz - 1) / tz;
  f.fused = g_fused_lds > 0 && fused_plan(f.g.nx, f.g.ny) &&
            fused_lds_bytes(f.g.nx, f.g.ny) <= (size_t)g_fused_lds;
  L->x_tiles = f.fused ? 3 * f.g.nz : ((f.g.ny * f.g.nz + 1) / 2 + f.ppb - 1) / f.ppb;
  L->y_tiles = f.fused ? 0 : f.nbx_y * f.g.nz * 3;
  L->z_tiles = f.nbx_z * f.g.ny * 3;
  L->ex = ex;
  L->ey = ey;
  L->ez = ez;
  // tile, rounded up to 16 elements, then the axis twiddles (see stage_twiddles)
  auto lds = [](size_t tile, int n) { return ((tile + 15) / 16 * 16 + (size_t)n) * sizeof(float2); };
  L->x_lds = cx ? sizeof(float2) * ((size_t)3 * f.ppb * (f.g.nx + 1) + f.g.nx)
               : lds((size_t)3 * f.ppb * f.g.nx, f.g.nx);
  if (f.fused) L->x_lds = fused_lds_bytes(f.g.nx, f.g.ny);
  L->y_lds = cy ? ct_lds_bytes(f.g.ny) : lds((size_t)ty * (f.g.ny + 1), f.g.ny);
  L->z_lds = cz ? ct_lds_bytes(f.g.nz) : lds((size_t)tz * (f.g.nz + 1), f.g.nz);
}

#define EMAX_SWITCH(E, CALL8, CALL16, CALL32) \
  do {                                        \
    if ((E) <= 8) CALL8;                      \
    else if ((E) <= 16) CALL16;               \
    else CALL32;                              \
  } while (0)

void launch_fft_x_fwd(const FftPair& f, const FftLaunch& L, hipStream_t s) {
  if (f.fused) {
#define LDDMM_FUSED_CASE(NX, A, B, NY, C, D)                                                   \
    if (f.g.nx == NX && f.g.ny == NY) {                                                       \
      hipLaunchKernelGGL((k_fftf_xy<A, B, C, D>), dim3(L.x_tiles), dim3(kFusedBlock), L.x_lds, \
                         s, f);                                                               \
      return;                                                                                 \
    }
    LDDMM_FUSED_PLANS(LDDMM_FUSED_CASE)
#undef LDDMM_FUSED_CASE
  }
  switch (f.g.nx) {
#define LDDMM_CT_CASE(N, A, B)                                                              \
  case N:                                                                                   \
    hipLaunchKernelGGL((k_fftc_x_fwd<A, B>), dim3(L.x_tiles),                               \
                       dim3(3 * kXP(A > B ? A : B) * (A > B ? A : B)), L.x_lds, s, f);      \
    return;
    LDDMM_CTX_PLANS(LDDMM_CT_CASE)
#undef LDDMM_CT_CASE
    default:
      break;
  }
  EMAX_SWITCH(L.ex,
    hipLaunchKernelGGL(k_fft_x_fwd<8>, dim3(L.x_tiles), dim3(kBlock), L.x_lds, s, f),
    hipLaunchKernelGGL(k_fft_x_fwd<16>, dim3(L.x_tiles), dim3(kBlock), L.x_lds, s, f),
    hipLaunchKernelGGL(k_fft_x_fwd<32>, dim3(L.x_tiles), dim3(kBlock), L.x_lds, s, f));
}

void launch_fft_y(const FftPair& f, const FftLaunch& L, int inverse, hipStream_t s) {
  if (f.fused) return;                    // done by the fused x passes
  const dim3 grid(f.nbx_y, f.g.nz, 3);
  switch (f.g.ny) {
#define LDDMM_CT_CASE(N, A, B)                                                                   \
  case N:                                                                                        \
    if (inverse)                                                                                 \
      hipLaunchKernelGGL((k_fftc_y<A, B, true>), grid, dim3(kCT * (A > B ? A : B)), L.y_lds, s, f); \
    else                                                                                         \
      hipLaunchKernelGGL((k_fftc_y<A, B, false>), grid, dim3(kCT * (A > B ? A : B)), L.y_lds, s, f); \
    return;
    LDDMM_CT_PLANS(LDDMM_CT_CASE)
#undef LDDMM_CT_CASE
    default:
      break;
  }
  if (inverse)
    EMAX_SWITCH(L.ey,
      hipLaunchKernelGGL((k_fft_y<8, true>), grid, dim3(kBlock), L.y_lds, s, f),
      hipLaunchKernelGGL((k_fft_y<16, true>), grid, dim3(kBlock), L.y_lds, s, f),
      hipLaunchKernelGGL((k_fft_y<32, true>), grid, dim3(kBlock), L.y_lds, s, f));
  else
    EMAX_SWITCH(L.ey,
      hipLaunchKernelGGL((k_fft_y<8, false>), grid, dim3(kBlock), L.y_lds, s, f),
      hipLaunchKernelGGL((k_fft_y<16, false>), grid, dim3(kBlock), L.y_lds, s, f),
      hipLaunchKernelGGL((k_fft_y<32, false>), grid, dim3(kBlock), L.y_lds, s, f));
}

void launch_fft_z_K(const FftPair& f, const FftLaunch& L, hipStream_t s) {
  const dim3 grid(f.nbx_z * f.g.ny * 3);
  switch (f.g.nz) {
#define LDDMM_CT_CASE(N, A, B)                                                               \
  case N:                                                                                    \
    hipLaunchKernelGGL((k_fftc_zK<A, B>), grid, dim3(kCT * (A > B ? A : B)), L.z_lds, s, f); \
    return;
    LDDMM_CT_PLANS(LDDMM_CT_CASE)
#undef LDDMM_CT_CASE
    default:
      break;
  }
  EMAX_SWITCH(L.ez,
    hipLaunchKernelGGL(k_fft_z_K<8>, grid, dim3(kBlock), L.z_lds, s, f),
    hipLaunchKernelGGL(k_fft_z_K<16>, grid, dim3(kBlock), L.z_lds, s, f),
    hipLaunchKernelGGL(k_fft_z_K<32>, grid, dim3(kBlock), L.z_lds, s, f));
}

void launch_fft_x_inv(const FftPair& f, const FftLaunch& L, const UpdArgs& u, hipStream_t s) {
  if (f.fused) {
#define LDDMM_FUSED_CASE(NX, A, B, NY, C, D)                                                   \
    if (f.g.nx == NX && f.g.ny == NY) {                                                       \
      hipLaunchKernelGGL((k_fftf_yx<A, B, C, D>), dim3(L.x_tiles), dim3(kFusedBlock), L.x_lds, \
                         s, f, u);                                                            \
      return;                                                                                 \
    }
    LDDMM_FUSED_PLANS(LDDMM_FUSED_CASE)
#undef LDDMM_FUSED_CASE
  }
  switch (f.g.nx) {
#define LDDMM_CT_CASE(N, A, B)                                                              \
  case N:                                                                                   \
    hipLaunchKernelGGL((k_fftc_x_inv<A, B>), dim3(L.x_tiles),                               \
                       dim3(3 * kXP(A > B ? A : B) * (A > B ? A : B)), L.x_lds, s, f, u);   \
    return;
    LDDMM_CTX_PLANS(LDDMM_CT_CASE)
#undef LDDMM_CT_CASE
    default:
      break;
  }
  EMAX_SWITCH(L.ex,
    hipLaunchKernelGGL(k_fft_x_inv<8>, dim3(L.x_tiles), dim3(kBlock), L.x_lds, s, f, u),
    hipLaunchKernelGGL(k_fft_x_inv<16>, dim3(L.x_tiles), dim3(kBlock), L.x_lds, s, f, u),
    hipLaunchKernelGGL(k_fft_x_inv<32>, dim3(L.x_tiles), dim3(kBlock), L.x_lds, s, f, u));
}

// Fused x + y passes of a batch whose problems all have grid g's fused plan
// (inverse: the y-inverse and x-inverse pass with epilogue upd[j]).  Returns false,
// launching nothing, when g has no fused plan.
bool launch_fft_fused_batched(int inverse, const BatchRef& br, const Geom& g, size_t lds, int j,
                              hipStream_t s) {
  if (br.off[br.np] == 0) return true;
  const dim3 grid(br.off[br.np]);
#define LDDMM_FUSED_CASE(NX, A, B, NY, C, D)                                                  \
  if (g.nx == NX && g.ny == NY) {                                                           \
    if (inverse)                                                                            \
      hipLaunchKernelGGL((k_fftf_yx_batched<A, B, C, D>), grid, dim3(kFusedBlock), lds, s,  \
                         br, j);                                                            \
    else                                                                                    \
      hipLaunchKernelGGL((k_fftf_xy_batched<A, B, C, D>), grid, dim3(kFusedBlock), lds, s,  \
                         br);                                                               \
    return true;                                                                            \
  }
  LDDMM_FUSED_PLANS(LDDMM_FUSED_CASE)
#undef LDDMM_FUSED_CASE
  return false;
}

// Batched passes: every problem of the batch in one launch (register budget and
// LDS of the most demanding problem).
void launch_fft_batched(int pass, const BatchRef& br, int emax, size_t lds, int j, hipStream_t s) {
  if (br.off[br.np] == 0) return;         // every problem's y passes are fused into x
  const dim3 grid(br.off[br.np]);
  switch (pass) {
    case 0:
      EMAX_SWITCH(emax,
        hipLaunchKernelGGL(k_fft_x_fwd_batched<8>, grid, dim3(kBlock), lds, s, br),
        hipLaunchKernelGGL(k_fft_x_fwd_batched<16>, grid, dim3(kBlock), lds, s, br),
        hipLaunchKernelGGL(k_fft_x_fwd_batched<32>, grid, dim3(kBlock), lds, s, br));
      break;
    case 1:
      EMAX_SWITCH(emax,
        hipLaunchKernelGGL((k_fft_y_batched<8, false>), grid, dim3(kBlock), lds, s, br),
        hipLaunchKernelGGL((k_fft_y_batched<16, false>), grid, dim3(kBlock), lds, s, br),
        hipLaunchKernelGGL((k_fft_y_batched<32, false>), grid, dim3(kBlock), lds, s, br));
      break;
    case 2:
      EMAX_SWITCH(emax,
        hipLaunchKernelGGL(k_fft_z_K_batched<8>, grid, dim3(kBlock), lds, s, br),
        hipLaunchKernelGGL(k_fft_z_K_batched<16>, grid, dim3(kBlock), lds, s, br),
        hipLaunchKernelGGL(k_fft_z_K_batched<32>, grid, dim3(kBlock), lds, s, br));
      break;
    case 3:
      EMAX_SWITCH(emax,
        hipLaunchKernelGGL((k_fft_y_batched<8, true>), grid, dim3(kBlock), lds, s, br),
        hipLaunchKernelGGL((k_fft_y_batched<16, true>), grid, dim3(kBlock), lds, s, br),
        hipLaunchKernelGGL((k_fft_y_batched<32, true>), grid, dim3(kBlock), lds, s, br));
      break;
    default:
      EMAX_SWITCH(emax,
        hipLaunchKernelGGL(k_fft_x_inv_batched<8>, grid, dim3(kBlock), lds, s, br, j),
        hipLaunchKernelGGL(k_fft_x_inv_batched<16>, grid, dim3(kBlock), lds, s, br, j),
        hipLaunchKernelGGL(k_fft_x_inv_batched<32>, grid, dim3(kBlock), lds, s, br, j));
      break;
  }
}

}  // namespace lddmm
