// Kernels of the direct RPA correlation energy (eq. (16)): the frequency
// polarisabilities accumulated from the time ones, 1 - P, the traces of P and
// of P^2, and ln det of a Hermitian positive-definite matrix from the
// diagonal of its Cholesky factor.
#include "kernels.hpp"

namespace {

// out[m][e] -= ph[m] chi[e] + conj(ph[m]) chit[e]  for m < nw, ph[m] = w_n exp(i w_m tau_n)
__global__ __launch_bounds__(256) void drpa_accum_kernel(const cplx* __restrict__ chi, const cplx* __restrict__ chit,
                                                       long long n_elem, const cplx* __restrict__ ph, int nw,
                                                       cplx* __restrict__ out) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= n_elem) return;
  const cplx a = chi[e], b = chit[e];
  for (int m = 0; m < nw; ++m) {
    const cplx p = ph[m];
    const cplx t = cadd(cmul(p, a), cmulc(b, p));   // p a + conj(p) b
    cplx* o = out + (long long)m * n_elem + e;
    *o = csub(*o, t);
  }
}

// a[h][i][j] <- delta_ij - a[h][i][j]
__global__ __launch_bounds__(256) void drpa_one_minus_kernel(cplx* __restrict__ a, int n, long long total) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const long long r = i % ((long long)n * n);
  const cplx v = a[i];
  a[i] = cmk(((r / n) == (r % n) ? 1.0 : 0.0) - v.x, -v.y);
}

// tr[h] = sum_i a[h][i][i] (complex), one workgroup per matrix
__global__ __launch_bounds__(256) void drpa_trace_kernel(const cplx* __restrict__ a, int n, cplx* __restrict__ tr) {
  const int h = blockIdx.x;
  const cplx* A = a + (long long)h * n * n;
  double re = 0.0, im = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const cplx v = A[(long long)i * n + i];
    re += v.x;
    im += v.y;
  }
  __shared__ double sr[256], si[256];
  sr[threadIdx.x] = re;
  si[threadIdx.x] = im;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) tr[h] = cmk(sr[0], si[0]);
}

// part[h][t] = sum over the 32 x 32 tile t = (ti, tj) of a[h][i][j] a[h][j][i]
// (both tiles read coalesced, the second transposed through LDS)
__global__ __launch_bounds__(256) void drpa_trace2_kernel(const cplx* __restrict__ a, int n, int nt,
                                                        cplx* __restrict__ part) {
  __shared__ cplx tb[32][33];
  const int h = blockIdx.y;
  const int ti = blockIdx.x / nt, tj = blockIdx.x % nt;
  const cplx* A = a + (long long)h * n * n;
  const int i0 = ti * 32, j0 = tj * 32;
  // tb[c][r] = a[j0 + r][i0 + c]
  for (int idx = threadIdx.x; idx < 1024; idx += 256) {
    const int r = idx >> 5, c = idx & 31;
    const int gj = j0 + r, gi = i0 + c;
    tb[c][r] = (gj < n && gi < n) ? A[(long long)gj * n + gi] : cmk(0.0, 0.0);
  }
  __syncthreads();
  double re = 0.0, im = 0.0;
  for (int idx = threadIdx.x; idx < 1024; idx += 256) {
    const int r = idx >> 5, c = idx & 31;     // element (i0 + r, j0 + c)
    const int gi = i0 + r, gj = j0 + c;
    if (gi < n && gj < n) {
      const cplx x = A[(long long)gi * n + gj], y = tb[r][c];   // y = a[j][i]
      re = fma(x.x, y.x, fma(-x.y, y.y, re));
      im = fma(x.x, y.y, fma(x.y, y.x, im));
    }
  }
  __shared__ double sr[256], si[256];
  sr[threadIdx.x] = re;
  si[threadIdx.x] = im;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)h * gridDim.x + blockIdx.x] = cmk(sr[0], si[0]);
}

// ld[h] = 2 sum_j ln L[h][j][j] (the factor's real diagonal in the lower
// triangle of a), NaN where the factorisation broke down (flag[h])
__global__ __launch_bounds__(256) void drpa_logdet_kernel(const cplx* __restrict__ a, const int* __restrict__ flag,
                                                        int n, double* __restrict__ ld) {
  const int h = blockIdx.x;
  const cplx* A = a + (long long)h * n * n;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) s += log(A[(long long)j * n + j].x);
  __shared__ double sr[256];
  sr[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sr[threadIdx.x] += sr[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) ld[h] = flag[h] ? __builtin_nan("") : 2.0 * sr[0];
}

}  // namespace

hipError_t drpa_accum_launch(const cplx* chi, const cplx* chit, long long n_elem, const cplx* ph, int nw, cplx* out,
                             hipStream_t s) {
  if (n_elem <= 0 || nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(drpa_accum_kernel, dim3((unsigned)((n_elem + 255) / 256)), dim3(256), 0, s, chi, chit, n_elem,
                     ph, nw, out);
  return hipGetLastError();
}

hipError_t drpa_one_minus_launch(cplx* a, int n, int nmat, hipStream_t s) {
  const long long total = (long long)nmat * n * n;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(drpa_one_minus_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a, n, total);
  return hipGetLastError();
}

hipError_t drpa_trace_launch(const cplx* a, int n, int nmat, cplx* tr, hipStream_t s) {
  if (nmat <= 0) return hipSuccess;
  hipLaunchKernelGGL(drpa_trace_kernel, dim3(nmat), dim3(256), 0, s, a, n, tr);
  return hipGetLastError();
}

int drpa_trace2_tiles(int n) {
  const int nt = (n + 31) / 32;
  return nt * nt;
}

hipError_t drpa_trace2_launch(const cplx* a, int n, int nmat, cplx* part, hipStream_t s) {
  if (nmat <= 0) return hipSuccess;
  if (nmat > 65535) return hipErrorInvalidValue;
  const int nt = (n + 31) / 32;
  hipLaunchKernelGGL(drpa_trace2_kernel, dim3(nt * nt, nmat), dim3(256), 0, s, a, n, nt, part);
  return hipGetLastError();
}

hipError_t drpa_logdet_launch(const cplx* a, const int* flag, int n, int nmat, double* ld, hipStream_t s) {
  if (nmat <= 0) return hipSuccess;
  hipLaunchKernelGGL(drpa_logdet_kernel, dim3(nmat), dim3(256), 0, s, a, flag, n, ld);
  return hipGetLastError();
}
