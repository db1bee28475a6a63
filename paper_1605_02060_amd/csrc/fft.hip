// Smoothing by K = (L^dagger L)^-1, L = gamma - alpha Lap (Methods, Registration),
// as a 3D DFT on the computational grid: mixed-radix (2,3,4,5,7,8) Stockham
// transforms staged in LDS, one axis per pass.
//
//   pass x-fwd : real body force b [3][P] -> half spectrum S [3][nz][ny][hx]
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
  while (p2 >= 3) {
    if (!push(8)) return false;
    p2 -= 3;
  }
  if (p2 == 2 && !push(4)) return false;
  if (p2 == 1 && !push(2)) return false;
  for (int r : {3, 5, 7}) {
    while (m % r == 0) {
      if (!push(r)) return false;
      m /= r;
    }
  }
  p->nst = st;
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

// One Stockham stage on nl lines of length N held in LDS (line l at sm + l*N).
// Ns = product of the radices already applied.  All reads of the stage happen
// before the barrier and all writes after it, so the stage runs in place.
template <int R>
__device__ __forceinline__ void fft_stage(float2* sm, int N, int nl, int Ns,
                                          const float2* __restrict__ tw) {
  constexpr int NB = (kEMax + R - 1) / R;
  const int nb = N / R;
  const int total = nl * nb;
  float2 val[NB][R];
  int line[NB], jj[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int bi = threadIdx.x + t * kBlock;
    line[t] = -1;
    jj[t] = 0;
    if (bi < total) {
      const int l = bi / nb;
      const int j = bi - l * nb;
      line[t] = l;
      jj[t] = j;
      const float2* src = sm + l * N + j;
#pragma unroll
      for (int q = 0; q < R; ++q) val[t][q] = src[q * nb];
    }
  }
  __syncthreads();
  const int step = N / (Ns * R);
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    if (line[t] >= 0) {
      const int j = jj[t];
      const int k = j % Ns;
#pragma unroll
      for (int q = 1; q < R; ++q) val[t][q] = cmul(val[t][q], tw[q * k * step]);
      radix_dft<R>(val[t]);
      float2* dst = sm + line[t] * N + (j / Ns) * Ns * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) dst[q * Ns] = val[t][q];
    }
  }
  __syncthreads();
}

// Forward DFT of nl lines of length p.n in LDS (natural order in and out).
__device__ __forceinline__ void lds_fft(float2* sm, int nl, const FFTPlan& p, const float2* __restrict__ tw) {
  int Ns = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int R = p.radix[s];
    switch (R) {
      case 2: fft_stage<2>(sm, p.n, nl, Ns, tw); break;
      case 3: fft_stage<3>(sm, p.n, nl, Ns, tw); break;
      case 4: fft_stage<4>(sm, p.n, nl, Ns, tw); break;
      case 5: fft_stage<5>(sm, p.n, nl, Ns, tw); break;
      case 7: fft_stage<7>(sm, p.n, nl, Ns, tw); break;
      default: fft_stage<8>(sm, p.n, nl, Ns, tw); break;
    }
    Ns *= R;
  }
}

__device__ __forceinline__ bool gate(const State* st, int need_mode) {
  return need_mode < 0 || st->mode == need_mode;
}

// ----------------------------------------------------------- x forward ----
// Row rho = z*ny + y.  Rows are processed in pairs (2m, 2m+1): complex lines
//   Z0 = bx[2m] + i by[2m],  Z1 = bx[2m+1] + i by[2m+1],  Z2 = bz[2m] + i bz[2m+1].
// After the DFT, for k < hx:  A[k] = (Z[k] + conj Z[-k]) / 2,  B[k] = (Z[k] - conj Z[-k]) / 2i.

__global__ __launch_bounds__(kBlock) void k_fft_x_fwd(const float* __restrict__ b,
                                                      float2* __restrict__ S, Geom g, FFTPlan p,
                                                      const float2* __restrict__ tw, int ppb,
                                                      const State* st, int need_mode) {
  if (!gate(st, need_mode)) return;
  extern __shared__ float2 sm[];
  const int N = g.nx;
  const long long n = g.n;
  const int nrows = g.ny * g.nz;
  const int pair0 = blockIdx.x * ppb;
  const int nl = 3 * ppb;
  for (int e = threadIdx.x; e < nl * N; e += kBlock) {
    const int l = e / N, x = e - l * N;
    const int pp = l / 3, which = l - 3 * pp;
    const int r0 = 2 * (pair0 + pp), r1 = r0 + 1;
    float2 z = make_float2(0.f, 0.f);
    if (which == 0) {
      if (r0 < nrows) z = make_float2(b[(long long)r0 * N + x], b[n + (long long)r0 * N + x]);
    } else if (which == 1) {
      if (r1 < nrows) z = make_float2(b[(long long)r1 * N + x], b[n + (long long)r1 * N + x]);
    } else {
      const float re = r0 < nrows ? b[2 * n + (long long)r0 * N + x] : 0.f;
      const float im = r1 < nrows ? b[2 * n + (long long)r1 * N + x] : 0.f;
      z = make_float2(re, im);
    }
    sm[e] = z;
  }
  __syncthreads();
  lds_fft(sm, nl, p, tw);
  const int hx = g.hx;
  for (int e = threadIdx.x; e < nl * hx; e += kBlock) {
    const int l = e / hx, k = e - l * hx;
    const int pp = l / 3, which = l - 3 * pp;
    const int r0 = 2 * (pair0 + pp), r1 = r0 + 1;
    const float2 zk = sm[l * N + k];
    const float2 zm = cconj(sm[l * N + (k == 0 ? 0 : N - k)]);
    const float2 A = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
    // (zk - zm) / 2i = -i/2 (zk - zm)
    const float2 B = make_float2(0.5f * (zk.y - zm.y), -0.5f * (zk.x - zm.x));
    if (which == 0) {
      if (r0 < nrows) {
        S[(long long)r0 * hx + k] = A;
        S[g.nspec + (long long)r0 * hx + k] = B;
      }
    } else if (which == 1) {
      if (r1 < nrows) {
        S[(long long)r1 * hx + k] = A;
        S[g.nspec + (long long)r1 * hx + k] = B;
      }
    } else {
      if (r0 < nrows) S[2 * g.nspec + (long long)r0 * hx + k] = A;
      if (r1 < nrows) S[2 * g.nspec + (long long)r1 * hx + k] = B;
    }
  }
}

static int pairs_per_block(int N) {
  int ppb = kFFTElems / (3 * N);
  if (ppb < 1) ppb = 1;
  if (ppb > 8) ppb = 8;
  return ppb;
}

void launch_fft_x_fwd(const float* b, float2* S, const Geom& g, const FFTPlan& p, const float2* tw,
                      const State* st, int need_mode, hipStream_t s) {
  const int ppb = pairs_per_block(g.nx);
  const int npairs = (g.ny * g.nz + 1) / 2;
  const int grid = (npairs + ppb - 1) / ppb;
  const size_t lds = (size_t)3 * ppb * g.nx * sizeof(float2);
  hipLaunchKernelGGL(k_fft_x_fwd, dim3(grid), dim3(kBlock), lds, s, b, S, g, p, tw, ppb, st,
                     need_mode);
}

// -------------------------------------------------------------- y pass ----
// Tile: TX consecutive kx of one (component, z) slab, all ny rows.

static int tile_cols(int N) {
  int tx = 32;
  while (tx > 1 && tx * N > kFFTElems) tx >>= 1;
  return tx;
}

__global__ __launch_bounds__(kBlock) void k_fft_y(float2* __restrict__ S, Geom g, FFTPlan p,
                                                  const float2* __restrict__ tw, int TX,
                                                  int inverse, const State* st, int need_mode) {
  if (!gate(st, need_mode)) return;
  extern __shared__ float2 sm[];
  const int N = g.ny, hx = g.hx;
  const int kx0 = blockIdx.x * TX;
  float2* base = S + (long long)blockIdx.z * g.nspec + (long long)blockIdx.y * g.ny * hx;
  for (int e = threadIdx.x; e < TX * N; e += kBlock) {
    const int c = e % TX, y = e / TX;
    float2 v = make_float2(0.f, 0.f);
    if (kx0 + c < hx) v = base[(long long)y * hx + kx0 + c];
    if (inverse) v = cconj(v);
    sm[c * N + y] = v;
  }
  __syncthreads();
  lds_fft(sm, TX, p, tw);
  for (int e = threadIdx.x; e < TX * N; e += kBlock) {
    const int c = e % TX, y = e / TX;
    if (kx0 + c < hx) {
      float2 v = sm[c * N + y];
      if (inverse) v = cconj(v);
      base[(long long)y * hx + kx0 + c] = v;
    }
  }
}

void launch_fft_y(float2* S, const Geom& g, const FFTPlan& p, const float2* tw, int inverse,
                  const State* st, int need_mode, hipStream_t s) {
  const int TX = tile_cols(g.ny);
  dim3 grid((g.hx + TX - 1) / TX, g.nz, 3);
  const size_t lds = (size_t)TX * g.ny * sizeof(float2);
  hipLaunchKernelGGL(k_fft_y, grid, dim3(kBlock), lds, s, S, g, p, tw, TX, inverse, st,
                     need_mode);
}

// ----------------------------------------------------------- z pass + K ----

__global__ __launch_bounds__(kBlock) void k_fft_z_K(float2* __restrict__ S, Geom g, FFTPlan p,
                                                    const float2* __restrict__ tw, int TX,
                                                    const double* __restrict__ lamx,
                                                    const double* __restrict__ lamy,
                                                    const double* __restrict__ lamz, double alpha,
                                                    double gamma, const State* st, int need_mode) {
  if (!gate(st, need_mode)) return;
  extern __shared__ float2 sm[];
  const int N = g.nz, hx = g.hx;
  const int kx0 = blockIdx.x * TX;
  const int ky = blockIdx.y;
  const long long zs = (long long)g.ny * hx;
  float2* base = S + (long long)blockIdx.z * g.nspec + (long long)ky * hx;
  for (int e = threadIdx.x; e < TX * N; e += kBlock) {
    const int c = e % TX, z = e / TX;
    float2 v = make_float2(0.f, 0.f);
    if (kx0 + c < hx) v = base[(long long)z * zs + kx0 + c];
    sm[c * N + z] = v;
  }
  __syncthreads();
  lds_fft(sm, TX, p, tw);
  const double inv_n = 1.0 / ((double)g.nx * (double)g.ny * (double)g.nz);
  for (int e = threadIdx.x; e < TX * N; e += kBlock) {
    const int c = e / N, kz = e - c * N;
    const int kx = kx0 + c < hx ? kx0 + c : 0;
    const double lam = alpha * (lamx[kx] + lamy[ky] + lamz[kz]) + gamma;
    const float kh = (float)(inv_n / (lam * lam));
    const float2 v = sm[e];
    sm[e] = make_float2(v.x * kh, -v.y * kh);     // conj(K_hat X / |P|)
  }
  __syncthreads();
  lds_fft(sm, TX, p, tw);
  for (int e = threadIdx.x; e < TX * N; e += kBlock) {
    const int c = e % TX, z = e / TX;
    if (kx0 + c < hx) base[(long long)z * zs + kx0 + c] = cconj(sm[c * N + z]);
  }
}

void launch_fft_z_K(float2* S, const Geom& g, const FFTPlan& p, const float2* tw,
                    const double* lamx, const double* lamy, const double* lamz, double alpha,
                    double gamma, const State* st, int need_mode, hipStream_t s) {
  const int TX = tile_cols(g.nz);
  dim3 grid((g.hx + TX - 1) / TX, g.ny, 3);
  const size_t lds = (size_t)TX * g.nz * sizeof(float2);
  hipLaunchKernelGGL(k_fft_z_K, grid, dim3(kBlock), lds, s, S, g, p, tw, TX, lamx, lamy, lamz,
                     alpha, gamma, st, need_mode);
}

// ----------------------------------------------------- x inverse + update ----
// Rebuild the full spectrum of each packed line from the half spectra
// (Z'[k] = A[k] + i B[k] for k < hx, conj A[N-k] + i conj B[N-k] above),
// invert, and split real / imaginary parts back into the two real lines.

__global__ __launch_bounds__(kBlock) void k_fft_x_inv(const float2* __restrict__ S, Geom g,
                                                      FFTPlan p, const float2* __restrict__ tw,
                                                      int ppb, UpdArgs u) {
  const State* st = u.st;
  if (!gate(st, u.need_mode)) return;
  extern __shared__ float2 sm[];
  const int N = g.nx, hx = g.hx;
  const long long n = g.n;
  const int nrows = g.ny * g.nz;
  const int pair0 = blockIdx.x * ppb;
  const int nl = 3 * ppb;
  for (int e = threadIdx.x; e < nl * N; e += kBlock) {
    const int l = e / N, k = e - l * N;
    const int pp = l / 3, which = l - 3 * pp;
    const int r0 = 2 * (pair0 + pp), r1 = r0 + 1;
    const bool lo = k < hx;
    const int kk = lo ? k : N - k;
    float2 A = make_float2(0.f, 0.f), B = make_float2(0.f, 0.f);
    if (which == 0) {
      if (r0 < nrows) {
        A = S[(long long)r0 * hx + kk];
        B = S[g.nspec + (long long)r0 * hx + kk];
      }
    } else if (which == 1) {
      if (r1 < nrows) {
        A = S[(long long)r1 * hx + kk];
        B = S[g.nspec + (long long)r1 * hx + kk];
      }
    } else {
      if (r0 < nrows) A = S[2 * g.nspec + (long long)r0 * hx + kk];
      if (r1 < nrows) B = S[2 * g.nspec + (long long)r1 * hx + kk];
    }
    if (!lo) {
      A = cconj(A);
      B = cconj(B);
    }
    // Z = A + i B ; store conj(Z) for the forward transform of the inverse
    sm[e] = make_float2(A.x - B.y, -(A.y + B.x));
  }
  __syncthreads();
  lds_fft(sm, nl, p, tw);
  // result z = conj(DFT(conj Z)): real line a = Re z = Re y, b = Im z = -Im y
  float* vA = u.vA;
  float* vB = u.vB;
  const int base = st->base;
  const float eps = (float)st->eps;
  for (int e = threadIdx.x; e < 2 * ppb * N; e += kBlock) {
    const int q = e / N, x = e - q * N;
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

void launch_fft_x_inv(const float2* S, const Geom& g, const FFTPlan& p, const float2* tw,
                      const UpdArgs& u, hipStream_t s) {
  const int ppb = pairs_per_block(g.nx);
  const int npairs = (g.ny * g.nz + 1) / 2;
  const int grid = (npairs + ppb - 1) / ppb;
  const size_t lds = (size_t)3 * ppb * g.nx * sizeof(float2);
  hipLaunchKernelGGL(k_fft_x_inv, dim3(grid), dim3(kBlock), lds, s, S, g, p, tw, ppb, u);
}

}  // namespace lddmm
