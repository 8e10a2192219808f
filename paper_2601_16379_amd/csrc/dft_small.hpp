// Small DFTs with compile-time lengths, kept in registers (unit-cell grid
// FFT and k-mesh transforms).  Forward transforms: y[k] = sum_j x[j] exp(-2 pi i jk/R).
#pragma once
#include "common.hpp"

namespace {

template <int R> struct Rot;
// cos and sin of 2 pi t / R (closed forms where they exist), t = 0..R-1
template <> struct Rot<2> {
  static constexpr double c[2] = {1.0, -1.0};
  static constexpr double s[2] = {0.0, 0.0};
};
template <> struct Rot<3> {
  static constexpr double c[3] = {1.0, -0.5, -0.5};
  static constexpr double s[3] = {0.0, 0.8660254037844386, -0.8660254037844386};
};
template <> struct Rot<4> {
  static constexpr double c[4] = {1.0, 0.0, -1.0, 0.0};
  static constexpr double s[4] = {0.0, 1.0, 0.0, -1.0};
};
template <> struct Rot<5> {
  static constexpr double c[5] = {1.0, 0.30901699437494745, -0.8090169943749475, -0.8090169943749475, 0.30901699437494745};
  static constexpr double s[5] = {0.0, 0.9510565162951535, 0.5877852522924731, -0.5877852522924731, -0.9510565162951535};
};
template <> struct Rot<6> {
  static constexpr double c[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
  static constexpr double s[6] = {0.0, 0.8660254037844386, 0.8660254037844386, 0.0, -0.8660254037844386, -0.8660254037844386};
};
template <> struct Rot<7> {
  static constexpr double c[7] = {1.0, 0.6234898018587336, -0.22252093395631434, -0.900968867902419, -0.900968867902419, -0.22252093395631434, 0.6234898018587336};
  static constexpr double s[7] = {0.0, 0.7818314824680298, 0.9749279121818236, 0.43388373911755823, -0.43388373911755823, -0.9749279121818236, -0.7818314824680298};
};
template <> struct Rot<8> {
  static constexpr double c[8] = {1.0, 0.7071067811865476, 0.0, -0.7071067811865476, -1.0, -0.7071067811865476, 0.0, 0.7071067811865476};
  static constexpr double s[8] = {0.0, 0.7071067811865476, 1.0, 0.7071067811865476, 0.0, -0.7071067811865476, -1.0, -0.7071067811865476};
};


constexpr double kPiD = 3.141592653589793;
constexpr double series_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 24; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
constexpr double series_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 24; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi t / N, t = 0..N-1 (Taylor series at |x| <= pi)
template <int N> struct TwF {
  float c[N], s[N];
  constexpr TwF() : c(), s() {
    for (int t = 0; t < N; ++t) {
      double x = 2.0 * kPiD * t / N;
      if (x > kPiD) x -= 2.0 * kPiD;
      c[t] = (float)series_cos(x);
      s[t] = (float)series_sin(x);
      if ((4 * t) % N == 0) {                  // quarter turns exactly
        const int q = 4 * t / N;
        c[t] = q == 0 ? 1.f : (q == 2 ? -1.f : 0.f);
        s[t] = q == 1 ? 1.f : (q == 3 ? -1.f : 0.f);
      }
    }
  }
};

// cos and sin of 2 pi t / N in double, t = 0..N-1 (Taylor series at |x| <= pi)
template <int N> struct TwD {
  double c[N], s[N];
  constexpr TwD() : c(), s() {
    for (int t = 0; t < N; ++t) {
      double x = 2.0 * kPiD * t / N;
      if (x > kPiD) x -= 2.0 * kPiD;
      c[t] = series_cos(x);
      s[t] = series_sin(x);
      if ((4 * t) % N == 0) {                  // quarter turns exactly
        const int q = 4 * t / N;
        c[t] = q == 0 ? 1.0 : (q == 2 ? -1.0 : 0.0);
        s[t] = q == 1 ? 1.0 : (q == 3 ? -1.0 : 0.0);
      }
    }
  }
};

// Lengths 3 and 5 in place, x[k] <- sum_j x[j] w^{jk} with w = exp(S 2 pi i
// / M), from the symmetric pairs a = x_j + x_{M-j}, b = x_j - x_{M-j}: the
// outputs k and M - k share t = x0 + sum_j cos(2 pi jk / M) a_j and differ
// in the sign of i u, u = S sum_j sin(2 pi jk / M) b_j (i u = (-u.y, u.x)).
template <int S>
__host__ __device__ inline void dft3_d(cplx (&x)[3]) {
  constexpr TwD<3> tw{};
  constexpr double sn = S * tw.s[1];
  const cplx a = cadd(x[1], x[2]), b = csub(x[1], x[2]);
  const cplx t = cmk(fma(-0.5, a.x, x[0].x), fma(-0.5, a.y, x[0].y));
  const cplx u = cmk(sn * b.x, sn * b.y);
  x[0] = cadd(x[0], a);
  x[1] = cmk(t.x - u.y, t.y + u.x);
  x[2] = cmk(t.x + u.y, t.y - u.x);
}
template <int S>
__host__ __device__ inline void dft5_d(cplx (&x)[5]) {
  constexpr TwD<5> tw{};
  constexpr double c1 = tw.c[1], c2 = tw.c[2], s1 = S * tw.s[1], s2 = S * tw.s[2];
  const cplx a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
  const cplx a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
  const cplx t1 = cmk(fma(c2, a2.x, fma(c1, a1.x, x[0].x)), fma(c2, a2.y, fma(c1, a1.y, x[0].y)));
  const cplx t2 = cmk(fma(c1, a2.x, fma(c2, a1.x, x[0].x)), fma(c1, a2.y, fma(c2, a1.y, x[0].y)));
  const cplx u1 = cmk(fma(s2, b2.x, s1 * b1.x), fma(s2, b2.y, s1 * b1.y));
  const cplx u2 = cmk(fma(-s1, b2.x, s2 * b1.x), fma(-s1, b2.y, s2 * b1.y));
  x[0] = cadd(x[0], cadd(a1, a2));
  x[1] = cmk(t1.x - u1.y, t1.y + u1.x);
  x[4] = cmk(t1.x + u1.y, t1.y - u1.x);
  x[2] = cmk(t2.x - u2.y, t2.y + u2.x);
  x[3] = cmk(t2.x + u2.y, t2.y - u2.x);
}

// In-place DFT of a length-M line in registers with compile-time M and sign S:
// x[k] <- sum_j x[j] exp(S 2 pi i j k / M).  Lengths 2 and 4 by butterflies,
// 3 and 5 from symmetric pairs (dft3_d, dft5_d); even M > 4 split into even
// and odd halves (radix 2, recursively); other M summed directly; the
// twiddles are compile-time constants.
template <int M, int S>
__host__ __device__ inline void dft_line(cplx (&x)[M]) {
  constexpr TwD<M> tw{};
  if constexpr (M == 1) {
    return;
  } else if constexpr (M == 2) {
    const cplx a = x[0];
    x[0] = cadd(a, x[1]);
    x[1] = csub(a, x[1]);
  } else if constexpr (M == 3) {
    dft3_d<S>(x);
  } else if constexpr (M == 4) {
    // a = x0 + x2, b = x0 - x2, c = x1 + x3, d = S (x1 - x3):
    // y0 = a + c, y2 = a - c, y1 = b + i d, y3 = b - i d
    const cplx a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
    const cplx c = cadd(x[1], x[3]), d0 = csub(x[1], x[3]);
    const cplx d = cmk(S * d0.x, S * d0.y);
    x[0] = cadd(a, c);
    x[2] = csub(a, c);
    x[1] = cmk(b.x - d.y, b.y + d.x);
    x[3] = cmk(b.x + d.y, b.y - d.x);
  } else if constexpr (M == 5) {
    dft5_d<S>(x);
  } else if constexpr (M % 2 == 0) {
    constexpr int H = M / 2;
    cplx e[H], o[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
      e[j] = x[2 * j];
      o[j] = x[2 * j + 1];
    }
    dft_line<H, S>(e);
    dft_line<H, S>(o);
#pragma unroll
    for (int k = 0; k < H; ++k) {
      cplx t;
      if (k == 0) {
        t = o[k];
      } else if (4 * k == M) {               // times i S
        t = cmk(-S * o[k].y, S * o[k].x);
      } else {
        const double c = tw.c[k], sn = S * tw.s[k];
        t = cmk(o[k].x * c - o[k].y * sn, o[k].x * sn + o[k].y * c);
      }
      x[k] = cadd(e[k], t);
      x[k + H] = csub(e[k], t);
    }
  } else {
    cplx y[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      double re = x[0].x, im = x[0].y;
#pragma unroll
      for (int j = 1; j < M; ++j) {
        const double c = tw.c[(j * k) % M], sn = S * tw.s[(j * k) % M];
        re = fma(x[j].x, c, fma(-x[j].y, sn, re));
        im = fma(x[j].y, c, fma(x[j].x, sn, im));
      }
      y[k] = cmk(re, im);
    }
#pragma unroll
    for (int k = 0; k < M; ++k) x[k] = y[k];
  }
}

// y[k] = sum_j x[j] exp(-2 pi i j k / R), compile-time R <= 8 (the line
// transform with S = -1)
template <int R>
__device__ inline void small_dft(const cplx (&x)[R], cplx (&y)[R]) {
#pragma unroll
  for (int k = 0; k < R; ++k) y[k] = x[k];
  dft_line<R, -1>(y);
}

// a * (c - i s) with compile-time c, s (the trivial factors fold away)
__host__ __device__ inline float2 rot_f(float2 a, float c, float s) {
  if (c == 1.0f && s == 0.0f) return a;
  if (c == 0.0f && s == 1.0f) return make_float2(a.y, -a.x);
  if (c == -1.0f && s == 0.0f) return make_float2(-a.x, -a.y);
  if (c == 0.0f && s == -1.0f) return make_float2(-a.y, a.x);
  return make_float2(fmaf(a.x, c, a.y * s), fmaf(a.y, c, -a.x * s));
}

// Lengths 3 and 5 in FP32, y[k] = sum_j x[j] exp(-2 pi i jk / M), from the
// symmetric pairs as dft3_d / dft5_d (here S = -1)
__host__ __device__ inline void dft3_f(const float2 (&x)[3], float2 (&y)[3]) {
  constexpr TwF<3> tw{};
  constexpr float sn = -tw.s[1];
  const float2 a = make_float2(x[1].x + x[2].x, x[1].y + x[2].y);
  const float2 b = make_float2(x[1].x - x[2].x, x[1].y - x[2].y);
  const float2 t = make_float2(fmaf(-0.5f, a.x, x[0].x), fmaf(-0.5f, a.y, x[0].y));
  const float2 u = make_float2(sn * b.x, sn * b.y);
  y[0] = make_float2(x[0].x + a.x, x[0].y + a.y);
  y[1] = make_float2(t.x - u.y, t.y + u.x);
  y[2] = make_float2(t.x + u.y, t.y - u.x);
}
__host__ __device__ inline void dft5_f(const float2 (&x)[5], float2 (&y)[5]) {
  constexpr TwF<5> tw{};
  constexpr float c1 = tw.c[1], c2 = tw.c[2], s1 = -tw.s[1], s2 = -tw.s[2];
  const float2 a1 = make_float2(x[1].x + x[4].x, x[1].y + x[4].y);
  const float2 b1 = make_float2(x[1].x - x[4].x, x[1].y - x[4].y);
  const float2 a2 = make_float2(x[2].x + x[3].x, x[2].y + x[3].y);
  const float2 b2 = make_float2(x[2].x - x[3].x, x[2].y - x[3].y);
  const float2 t1 = make_float2(fmaf(c2, a2.x, fmaf(c1, a1.x, x[0].x)), fmaf(c2, a2.y, fmaf(c1, a1.y, x[0].y)));
  const float2 t2 = make_float2(fmaf(c1, a2.x, fmaf(c2, a1.x, x[0].x)), fmaf(c1, a2.y, fmaf(c2, a1.y, x[0].y)));
  const float2 u1 = make_float2(fmaf(s2, b2.x, s1 * b1.x), fmaf(s2, b2.y, s1 * b1.y));
  const float2 u2 = make_float2(fmaf(-s1, b2.x, s2 * b1.x), fmaf(-s1, b2.y, s2 * b1.y));
  y[0] = make_float2(x[0].x + (a1.x + a2.x), x[0].y + (a1.y + a2.y));
  y[1] = make_float2(t1.x - u1.y, t1.y + u1.x);
  y[4] = make_float2(t1.x + u1.y, t1.y - u1.x);
  y[2] = make_float2(t2.x - u2.y, t2.y + u2.x);
  y[3] = make_float2(t2.x + u2.y, t2.y - u2.x);
}

template <int R>
__host__ __device__ inline void small_dft_f(const float2 (&x)[R], float2 (&y)[R]) {
  if constexpr (R == 3) {
    dft3_f(x, y);
    return;
  } else if constexpr (R == 2) {
    y[0] = make_float2(x[0].x + x[1].x, x[0].y + x[1].y);
    y[1] = make_float2(x[0].x - x[1].x, x[0].y - x[1].y);
    return;
  } else if constexpr (R == 4) {
    // a = x0 + x2, b = x0 - x2, c = x1 + x3, d = x1 - x3:
    // y0 = a + c, y2 = a - c, y1 = b - i d, y3 = b + i d
    const float2 a = make_float2(x[0].x + x[2].x, x[0].y + x[2].y);
    const float2 b = make_float2(x[0].x - x[2].x, x[0].y - x[2].y);
    const float2 c = make_float2(x[1].x + x[3].x, x[1].y + x[3].y);
    const float2 d = make_float2(x[1].x - x[3].x, x[1].y - x[3].y);
    y[0] = make_float2(a.x + c.x, a.y + c.y);
    y[2] = make_float2(a.x - c.x, a.y - c.y);
    y[1] = make_float2(b.x + d.y, b.y - d.x);
    y[3] = make_float2(b.x - d.y, b.y + d.x);
    return;
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    float2 acc = x[0];
#pragma unroll
    for (int j = 1; j < R; ++j) {
      const float2 t = rot_f(x[j], (float)Rot<R>::c[(j * k) % R], (float)Rot<R>::s[(j * k) % R]);
      acc.x += t.x;
      acc.y += t.y;
    }
    y[k] = acc;
  }
}

// y[k] = sum_j x[j] exp(-2 pi i j k / R) for any compile-time R <= 16: the
// butterflies of small_dft_f for R = 2, 4, the symmetric pairs for R = 3, 5;
// even R split into even and odd halves (radix 2, recursively); other R by
// the direct sum with the twiddles as compile-time constants (TwF).
template <int R>
__host__ __device__ inline void dft_any_f(const float2 (&x)[R], float2 (&y)[R]) {
  if constexpr (R == 1) {
    y[0] = x[0];
  } else if constexpr (R == 2 || R == 4) {
    small_dft_f<R>(x, y);
  } else if constexpr (R == 3) {
    dft3_f(x, y);
  } else if constexpr (R == 5) {
    dft5_f(x, y);
  } else if constexpr (R % 2 == 0) {
    constexpr int H = R / 2;
    constexpr TwF<R> tw{};
    float2 e[H], o[H], fe[H], fo[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
      e[j] = x[2 * j];
      o[j] = x[2 * j + 1];
    }
    dft_any_f<H>(e, fe);
    dft_any_f<H>(o, fo);
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const float2 t = rot_f(fo[k], tw.c[k], tw.s[k]);
      y[k] = make_float2(fe[k].x + t.x, fe[k].y + t.y);
      y[k + H] = make_float2(fe[k].x - t.x, fe[k].y - t.y);
    }
  } else {
    constexpr TwF<R> tw{};
#pragma unroll
    for (int k = 0; k < R; ++k) {
      float2 acc = x[0];
#pragma unroll
      for (int j = 1; j < R; ++j) {
        const float2 t = rot_f(x[j], tw.c[(j * k) % R], tw.s[(j * k) % R]);
        acc.x += t.x;
        acc.y += t.y;
      }
      y[k] = acc;
    }
  }
}

}  // namespace
