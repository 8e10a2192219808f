// Host driver for the register DFT building blocks of the k-mesh and pair
// transforms (dft_small.hpp, compiled for the host): reads cases from stdin,
// one a line -- "M S P" (length, sign, 64 or 32 bits) then M complex values
// as 2M numbers -- and prints the transformed values, one case a line.
#include <hip/hip_runtime.h>
#include <cstdio>
#include "dft_small.hpp"

template <int M>
void run(int sgn, int bits, const double* in, double* out) {
  if (bits == 64) {
    cplx x[M];
    for (int j = 0; j < M; ++j) x[j] = cmk(in[2 * j], in[2 * j + 1]);
    if (sgn > 0) dft_line<M, 1>(x); else dft_line<M, -1>(x);
    for (int j = 0; j < M; ++j) { out[2 * j] = x[j].x; out[2 * j + 1] = x[j].y; }
  } else {
    float2 x[M], y[M];
    for (int j = 0; j < M; ++j) x[j] = make_float2((float)in[2 * j], (float)in[2 * j + 1]);
    dft_any_f<M>(x, y);          // exp(-2 pi i jk / M)
    for (int j = 0; j < M; ++j) { out[2 * j] = y[j].x; out[2 * j + 1] = y[j].y; }
  }
}

int main() {
  int m, sgn, bits;
  double in[32], out[32];
  while (scanf("%d %d %d", &m, &sgn, &bits) == 3) {
    if (m < 1 || m > 16) return 1;
    for (int j = 0; j < 2 * m; ++j)
      if (scanf("%lf", &in[j]) != 1) return 1;
    switch (m) {
#define CASE(M) case M: run<M>(sgn, bits, in, out); break;
      CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
      CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
    }
    for (int j = 0; j < 2 * m; ++j) printf("%.17g%c", out[j], j + 1 < 2 * m ? ' ' : '\n');
  }
  return 0;
}
