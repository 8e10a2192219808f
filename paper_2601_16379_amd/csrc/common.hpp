// Shared device helpers of the gfx950 ISDF library: complex arithmetic on
// interleaved float64 pairs and small launch utilities.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double2 cplx;   // (re, im)

__host__ __device__ inline cplx cmk(double r, double i) { cplx z; z.x = r; z.y = i; return z; }
__host__ __device__ inline cplx cadd(cplx a, cplx b) { return cmk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cplx csub(cplx a, cplx b) { return cmk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cplx cmul(cplx a, cplx b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__host__ __device__ inline cplx cmulc(cplx a, cplx b) {
  return cmk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__host__ __device__ inline cplx cconj(cplx a) { return cmk(a.x, -a.y); }
__host__ __device__ inline cplx cscale(cplx a, double s) { return cmk(a.x * s, a.y * s); }
// acc += a * b
__host__ __device__ inline void cfma(cplx& acc, cplx a, cplx b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}

// exp(i * pi * x) in FP64
__device__ inline cplx cexpipi(double x) {
  double s, c;
  sincospi(x, &s, &c);
  return cmk(c, s);
}

static inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// Store one complex value in one of the operand formats of the NT GEMMs:
//   0  complex128 at element off;
//   1  float planes re | im, element off of each plane (plane stride `plane`);
//   2  bf16 hi + lo (x = hi + lo per real component), interleaved by groups
//      of 8 elements: element off at u16 index bf16x3_index(off, p) with
//      p = 0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo, so that the 16 k of one
//      matrix-core step of a row are 128 contiguous bytes (rows start at
//      multiples of 8 elements; `plane` is not used);
//   3  single bf16 (re, im), interleaved by groups of 8 elements: element off
//      at u16 index (off >> 3) * 16 + p * 8 + (off & 7), p = 0 re, 1 im, so
//      that the 32 k of one stage of a row are 128 contiguous bytes.
__device__ inline unsigned short bf16_bits_of(float x) {
  __bf16 h = (__bf16)x;
  return __builtin_bit_cast(unsigned short, h);
}
__device__ inline float bf16_value(unsigned short b) { return (float)__builtin_bit_cast(__bf16, b); }
__host__ __device__ inline long long bf16x3_index(long long off, int p) { return (off >> 3) * 32 + p * 8 + (off & 7); }

__device__ inline void store_bf16x3(unsigned short* o, long long off, float re, float im) {
  const unsigned short rh = bf16_bits_of(re), ih = bf16_bits_of(im);
  const long long b = (off >> 3) * 32 + (off & 7);
  o[b] = rh;
  o[b + 8] = bf16_bits_of(re - bf16_value(rh));
  o[b + 16] = ih;
  o[b + 24] = bf16_bits_of(im - bf16_value(ih));
}

__device__ inline void store_fmt(void* out, long long off, long long plane, int fmt, cplx v) {
  if (fmt == 0) {
    ((cplx*)out)[off] = v;
  } else if (fmt == 1) {
    float* o = (float*)out;
    o[off] = (float)v.x;
    o[plane + off] = (float)v.y;
  } else if (fmt == 2) {
    store_bf16x3((unsigned short*)out, off, (float)v.x, (float)v.y);
  } else {
    unsigned short* o = (unsigned short*)out;
    const long long b = (off >> 3) * 16 + (off & 7);
    o[b] = bf16_bits_of((float)v.x);
    o[b + 8] = bf16_bits_of((float)v.y);
  }
}
