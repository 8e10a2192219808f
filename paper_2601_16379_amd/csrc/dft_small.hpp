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


// y[k] = sum_j x[j] exp(-2 pi i j k / R), compile-time R <= 8
template <int R>
__device__ inline void small_dft(const cplx (&x)[R], cplx (&y)[R]) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    double re = x[0].x, im = x[0].y;
#pragma unroll
    for (int j = 1; j < R; ++j) {
      const double c = Rot<R>::c[(j * k) % R], sn = Rot<R>::s[(j * k) % R];
      re = fma(x[j].x, c, fma(x[j].y, sn, re));
      im = fma(x[j].y, c, fma(-x[j].x, sn, im));
    }
    y[k] = cmk(re, im);
  }
}

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
    }
  }
};

// In-place DFT of a length-M line in registers with compile-time M and sign S:
// x[k] <- sum_j x[j] exp(S 2 pi i j k / M).  Even M > 4 split into even and
// odd halves (radix 2, recursively); other M summed directly; the twiddles
// are compile-time constants.
template <int M, int S>
__host__ __device__ inline void dft_line(cplx (&x)[M]) {
  constexpr TwD<M> tw{};
  if constexpr (M == 1) {
    return;
  } else if constexpr (M % 2 == 0 && M > 4) {
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
      const double c = tw.c[k], sn = S * tw.s[k];
      const cplx t = cmk(o[k].x * c - o[k].y * sn, o[k].x * sn + o[k].y * c);
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

// a * (c - i s) with compile-time c, s (the trivial factors fold away)
__host__ __device__ inline float2 rot_f(float2 a, float c, float s) {
  if (c == 1.0f && s == 0.0f) return a;
  if (c == 0.0f && s == 1.0f) return make_float2(a.y, -a.x);
  if (c == -1.0f && s == 0.0f) return make_float2(-a.x, -a.y);
  if (c == 0.0f && s == -1.0f) return make_float2(-a.y, a.x);
  return make_float2(fmaf(a.x, c, a.y * s), fmaf(a.y, c, -a.x * s));
}

template <int R>
__host__ __device__ inline void small_dft_f(const float2 (&x)[R], float2 (&y)[R]) {
  if constexpr (R == 2) {
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
// butterflies of small_dft_f for R = 2, 4; even R split into even and odd
// halves (radix 2, recursively); other R by the direct sum with the twiddles
// as compile-time constants (TwF).
template <int R>
__host__ __device__ inline void dft_any_f(const float2 (&x)[R], float2 (&y)[R]) {
  if constexpr (R == 1) {
    y[0] = x[0];
  } else if constexpr (R == 2 || R == 4) {
    small_dft_f<R>(x, y);
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
