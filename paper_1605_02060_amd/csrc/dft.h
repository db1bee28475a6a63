// Small DFTs of compile-time length, held in registers, and the two-factor
// line transform built from them.
//
// dft<R>(v): in-place forward DFT of R complex values in natural order,
//   v[m] <- sum_p v[p] exp(-2 pi i p m / R).
// Lengths 2, 3, 4, 5, 7, 8, 9 and 16 are written out (9 and 16 as 3 x 3 and
// 4 x 4 with twiddles); 6, 10, 12, 14, 15 and 20 are Good-Thomas (prime-factor)
// products of two coprime lengths, which need no twiddle factors: with N = A B, the input index n = (B a + A b) mod N and
// the output index k (k = ka mod A, k = kb mod B) give
//   X[k] = sum_a W_A^(a ka) sum_b W_B^(b kb) x[(B a + A b) mod N].
// Every index is a compile-time constant after unrolling, so the values stay
// in registers and the reordering costs no instructions.
//
// Usable on the host as well (the CPU tests check every length against a
// direct DFT in double precision).
#pragma once

#include <hip/hip_runtime.h>

namespace lddmm {
namespace dft {

#define LDDMM_HD __host__ __device__ __forceinline__

LDDMM_HD float2 add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
LDDMM_HD float2 sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
LDDMM_HD float2 mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
LDDMM_HD float2 conj(float2 a) { return make_float2(a.x, -a.y); }
// a * (-i)
LDDMM_HD float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }
// a * (c - i s): multiplication by a forward root of unity with cosine c, sine s
LDDMM_HD float2 rot(float2 a, float c, float s) {
  return make_float2(a.x * c + a.y * s, a.y * c - a.x * s);
}

// cos and sin of 2 pi k / R for the written-out odd lengths and 16
template <int R>
struct Roots;
template <>
struct Roots<3> {
  static constexpr float c[3] = {1.f, -0.5f, -0.5f};
  static constexpr float s[3] = {0.f, 0.86602540378443865f, -0.86602540378443865f};
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
  static constexpr float c[7] = {1.f, 0.62348980185873353f, -0.22252093395631440f,
                                 -0.90096886790241913f, -0.90096886790241913f,
                                 -0.22252093395631440f, 0.62348980185873353f};
  static constexpr float s[7] = {0.f, 0.78183148246802981f, 0.97492791218182361f,
                                 0.43388373911755812f, -0.43388373911755812f,
                                 -0.97492791218182361f, -0.78183148246802981f};
};
template <>
struct Roots<9> {
  static constexpr float c[9] = {1.f, 0.76604444311897801f, 0.17364817766693041f, -0.5f,
                                 -0.93969262078590838f, -0.93969262078590838f, -0.5f,
                                 0.17364817766693041f, 0.76604444311897801f};
  static constexpr float s[9] = {0.f, 0.64278760968653925f, 0.98480775301220802f,
                                 0.86602540378443865f, 0.34202014332566873f,
                                 -0.34202014332566873f, -0.86602540378443865f,
                                 -0.98480775301220802f, -0.64278760968653925f};
};
template <>
struct Roots<16> {
  static constexpr float c[16] = {1.f, 0.92387953251128674f, 0.70710678118654752f,
                                  0.38268343236508977f, 0.f, -0.38268343236508977f,
                                  -0.70710678118654752f, -0.92387953251128674f, -1.f,
                                  -0.92387953251128674f, -0.70710678118654752f,
                                  -0.38268343236508977f, 0.f, 0.38268343236508977f,
                                  0.70710678118654752f, 0.92387953251128674f};
  static constexpr float s[16] = {0.f, 0.38268343236508977f, 0.70710678118654752f,
                                  0.92387953251128674f, 1.f, 0.92387953251128674f,
                                  0.70710678118654752f, 0.38268343236508977f, 0.f,
                                  -0.38268343236508977f, -0.70710678118654752f,
                                  -0.92387953251128674f, -1.f, -0.92387953251128674f,
                                  -0.70710678118654752f, -0.38268343236508977f};
};

template <int R>
struct Dft;

template <int R>
LDDMM_HD void dft(float2 (&v)[R]) {
  Dft<R>::run(v);
}

template <>
struct Dft<1> {
  static LDDMM_HD void run(float2 (&)[1]) {}
};

template <>
struct Dft<2> {
  static LDDMM_HD void run(float2 (&v)[2]) {
    const float2 a = v[0], b = v[1];
    v[0] = add(a, b);
    v[1] = sub(a, b);
  }
};

LDDMM_HD void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  const float2 t0 = add(x0, x2), t1 = sub(x0, x2);
  const float2 t2 = add(x1, x3), t3 = mul_mi(sub(x1, x3));
  x0 = add(t0, t2);
  x2 = sub(t0, t2);
  x1 = add(t1, t3);
  x3 = sub(t1, t3);
}

template <>
struct Dft<4> {
  static LDDMM_HD void run(float2 (&v)[4]) { dft4(v[0], v[1], v[2], v[3]); }
};

// 8 = 2 x 4: 4-point DFTs of the even and odd samples, then W8^k and a 2-point step.
template <>
struct Dft<8> {
  static LDDMM_HD void run(float2 (&v)[8]) {
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    const float r = 0.70710678118654752f;
    const float2 w1 = make_float2(r * (o1.x + o1.y), r * (o1.y - o1.x));     // W8^1
    const float2 w2 = mul_mi(o2);                                            // W8^2 = -i
    const float2 w3 = make_float2(r * (o3.y - o3.x), -r * (o3.x + o3.y));    // W8^3
    v[0] = add(e0, o0);
    v[4] = sub(e0, o0);
    v[1] = add(e1, w1);
    v[5] = sub(e1, w1);
    v[2] = add(e2, w2);
    v[6] = sub(e2, w2);
    v[3] = add(e3, w3);
    v[7] = sub(e3, w3);
  }
};

// 16 = 4 x 4 (Cooley-Tukey): 4-point DFTs over b of x[a + 4 b], twiddles
// W16^(a kb), 4-point DFTs over a; output X[kb + 4 ka].
template <>
struct Dft<16> {
  static LDDMM_HD void run(float2 (&v)[16]) {
    float2 y[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      y[a][0] = v[a];
      y[a][1] = v[a + 4];
      y[a][2] = v[a + 8];
      y[a][3] = v[a + 12];
      dft4(y[a][0], y[a][1], y[a][2], y[a][3]);
    }
#pragma unroll
    for (int a = 1; a < 4; ++a)
#pragma unroll
      for (int kb = 1; kb < 4; ++kb) {
        const int m = a * kb;
        if (m == 4)
          y[a][kb] = mul_mi(y[a][kb]);
        else
          y[a][kb] = rot(y[a][kb], Roots<16>::c[m], Roots<16>::s[m]);
      }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      dft4(y[0][kb], y[1][kb], y[2][kb], y[3][kb]);
      v[kb] = y[0][kb];
      v[kb + 4] = y[1][kb];
      v[kb + 8] = y[2][kb];
      v[kb + 12] = y[3][kb];
    }
  }
};

// Odd prime R: pair x[p] with x[R-p].  With a_p = x_p + x_(R-p), b_p = x_p - x_(R-p):
//   y_m     = x_0 + sum_p a_p cos(2 pi p m/R) - i sum_p b_p sin(2 pi p m/R)
//   y_(R-m) = x_0 + sum_p a_p cos(2 pi p m/R) + i sum_p b_p sin(2 pi p m/R)
template <int R>
struct DftOdd {
  static LDDMM_HD void run(float2 (&v)[R]) {
    constexpr int H = (R - 1) / 2;
    float2 a[H], b[H];
#pragma unroll
    for (int p = 1; p <= H; ++p) {
      a[p - 1] = add(v[p], v[R - p]);
      b[p - 1] = sub(v[p], v[R - p]);
    }
    const float2 x0 = v[0];
    float2 y0 = x0;
#pragma unroll
    for (int p = 0; p < H; ++p) y0 = add(y0, a[p]);
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
      // -i (sr + i si) = si - i sr
      v[m] = make_float2(cr + si, ci - sr);
      v[R - m] = make_float2(cr - si, ci + sr);
    }
    v[0] = y0;
  }
};

template <>
struct Dft<3> : DftOdd<3> {};

// 9 = 3 x 3 (Cooley-Tukey): 3-point DFTs over b of x[a + 3 b], twiddles
// W9^(a kb), 3-point DFTs over a; output X[kb + 3 ka].
template <>
struct Dft<9> {
  static LDDMM_HD void run(float2 (&v)[9]);
};

LDDMM_HD void Dft<9>::run(float2 (&v)[9]) {
  float2 y[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float2 t[3] = {v[a], v[a + 3], v[a + 6]};
    Dft<3>::run(t);
    y[a][0] = t[0];
    y[a][1] = t[1];
    y[a][2] = t[2];
  }
#pragma unroll
  for (int a = 1; a < 3; ++a)
#pragma unroll
    for (int kb = 1; kb < 3; ++kb) {
      const int m = a * kb;
      y[a][kb] = rot(y[a][kb], Roots<9>::c[m], Roots<9>::s[m]);
    }
#pragma unroll
  for (int kb = 0; kb < 3; ++kb) {
    float2 t[3] = {y[0][kb], y[1][kb], y[2][kb]};
    Dft<3>::run(t);
    v[kb] = t[0];
    v[kb + 3] = t[1];
    v[kb + 6] = t[2];
  }
}
template <>
struct Dft<5> : DftOdd<5> {};
template <>
struct Dft<7> : DftOdd<7> {};

// Good-Thomas product of coprime A and B (no twiddles).
constexpr int inv_mod(int a, int m) {
  int r = 1;
  while ((a * r) % m != 1) ++r;
  return r;
}

template <int A, int B>
struct DftPfa {
  static constexpr int N = A * B;
  static LDDMM_HD void run(float2 (&v)[N]) {
    float2 y[B][A];      // y[b][ka] after the A-point DFTs
#pragma unroll
    for (int b = 0; b < B; ++b) {
      float2 t[A];
#pragma unroll
      for (int a = 0; a < A; ++a) t[a] = v[(B * a + A * b) % N];
      Dft<A>::run(t);
#pragma unroll
      for (int ka = 0; ka < A; ++ka) y[b][ka] = t[ka];
    }
    constexpr int eA = B * inv_mod(B % A, A);   // = 1 mod A, 0 mod B
    constexpr int eB = A * inv_mod(A % B, B);   // = 0 mod A, 1 mod B
#pragma unroll
    for (int ka = 0; ka < A; ++ka) {
      float2 t[B];
#pragma unroll
      for (int b = 0; b < B; ++b) t[b] = y[b][ka];
      Dft<B>::run(t);
#pragma unroll
      for (int kb = 0; kb < B; ++kb) v[(ka * eA + kb * eB) % N] = t[kb];
    }
  }
};

template <>
struct Dft<6> : DftPfa<2, 3> {};
template <>
struct Dft<10> : DftPfa<2, 5> {};
template <>
struct Dft<12> : DftPfa<4, 3> {};
template <>
struct Dft<14> : DftPfa<2, 7> {};
template <>
struct Dft<15> : DftPfa<3, 5> {};
template <>
struct Dft<20> : DftPfa<4, 5> {};
template <>
struct Dft<28> : DftPfa<4, 7> {};
template <>
struct Dft<35> : DftPfa<5, 7> {};

#undef LDDMM_HD

}  // namespace dft
}  // namespace lddmm
