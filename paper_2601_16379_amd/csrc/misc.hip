// Small data-movement kernels of the path.
#include "kernels.hpp"

namespace {

// Interpolating vectors X^k_{I mu} = phi^k_mu(r_I) (below eq. (2)), stored
// k-major as Xt[k][mu][I] so that they are the K-major operand of the GEMMs.
__global__ void gather_kernel(const cplx* __restrict__ phi, const int* __restrict__ ip, cplx* xt,
                              int nk, int norb, long long ng, int nip) {
  const long long total = (long long)nk * norb * nip;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long km = idx / nip;
    const int I = (int)(idx - km * nip);
    xt[idx] = phi[km * ng + ip[I]];
  }
}

__global__ void copy_cols_kernel(const cplx* __restrict__ in, cplx* out, int nk, int norb, int nf,
                                 int ncol, int col0) {
  const long long total = (long long)nk * norb * nf;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long km = idx / nf;
    const int p = (int)(idx - km * nf);
    out[km * ncol + col0 + p] = in[idx];
  }
}

__global__ void copy_cols_batch_kernel(const cplx* const* __restrict__ in, cplx* out, int nk, int norb,
                                       const int* __restrict__ nfa, const int* __restrict__ cola, int ncol) {
  const int f = blockIdx.y;
  const int nf = nfa[f], col0 = cola[f];
  const cplx* src = in[f];
  const long long total = (long long)nk * norb * nf;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long km = idx / nf;
    const int p = (int)(idx - km * nf);
    out[km * ncol + col0 + p] = src[idx];
  }
}

__global__ void nonfinite_kernel(const cplx* __restrict__ x, long long n, int* flag) {
  int bad = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const cplx v = x[i];
    if (!isfinite(v.x) || !isfinite(v.y)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

// Wt[h][J][I] = w_h W[h][I][J] in the four operand formats (row pitch ld,
// zero padding for I >= n), w_h = 1/2 where q = -q (hself[h]).
__global__ void wt_convert_kernel(const cplx* __restrict__ w, cplx* wt64, float* wt32, unsigned short* wt16,
                                  unsigned short* wt16s, int n, int ld, int nh, const int* __restrict__ hself) {
  const long long total = (long long)nh * n * ld;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long hJ = idx / ld;
    const int I = (int)(idx - hJ * ld);
    const int J = (int)(hJ % n);
    const int h = (int)(hJ / n);
    const long long q = h;
    const double wgt = hself[h] ? 0.5 : 1.0;
    const cplx v = (I < n) ? cscale(w[(q * n + I) * n + J], wgt) : cmk(0.0, 0.0);
    if (wt64) wt64[idx] = v;
    if (wt32) store_fmt(wt32, idx, total, 1, v);
    if (wt16) store_fmt(wt16, idx, total, 2, v);
    if (wt16s) store_fmt(wt16s, idx, total, 3, v);
  }
}

// Bt[h][j][a] = sqrt(w_h) L^h[a][j] for a >= j, zero above it and for
// a >= n (row pitch ld), from lt[h][j][a] = L^h[a][j] (the transposed
// Cholesky factor; its entries below the diagonal are not read), in the
// three mixed operand formats.
__global__ void lt_convert_kernel(const cplx* __restrict__ lt, float* wt32, unsigned short* wt16,
                                  unsigned short* wt16s, int n, int ld, int nh, const int* __restrict__ hself) {
  const long long total = (long long)nh * n * ld;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long hj = idx / ld;
    const int a = (int)(idx - hj * ld);
    const int j = (int)(hj % n);
    const int h = (int)(hj / n);
    const double wgt = hself[h] ? 0.7071067811865476 : 1.0;   // sqrt(1/2) where q = -q
    const cplx v = (a < n && a >= j) ? cscale(lt[((long long)h * n + j) * n + a], wgt) : cmk(0.0, 0.0);
    store_fmt(wt32, idx, total, 1, v);
    store_fmt(wt16, idx, total, 2, v);
    store_fmt(wt16s, idx, total, 3, v);
  }
}

__global__ void zero_c_kernel(cplx* x, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = cmk(0.0, 0.0);
}

inline int grid_for(long long n) {
  long long b = (n + 255) / 256;
  return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

}  // namespace

hipError_t gather_launch(const cplx* phi, const int* ip, cplx* xt, int nk, int norb, long long ng,
                         int nip, hipStream_t s) {
  hipLaunchKernelGGL(gather_kernel, dim3(grid_for((long long)nk * norb * nip)), dim3(256), 0, s,
                     phi, ip, xt, nk, norb, ng, nip);
  return hipGetLastError();
}

hipError_t copy_cols_batch_launch(const cplx* const* in, cplx* out, int nk, int norb, const int* nf,
                                  const int* col, int n, int maxnf, int ncol, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long per = (long long)nk * norb * maxnf;
  long long bx = (per + 255) / 256;
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(copy_cols_batch_kernel, dim3((unsigned)bx, n), dim3(256), 0, s, in, out, nk, norb, nf, col,
                     ncol);
  return hipGetLastError();
}

hipError_t copy_cols_launch(const cplx* in, cplx* out, int nk, int norb, int nf, int ncol, int col0,
                            hipStream_t s) {
  hipLaunchKernelGGL(copy_cols_kernel, dim3(grid_for((long long)nk * norb * nf)), dim3(256), 0, s,
                     in, out, nk, norb, nf, ncol, col0);
  return hipGetLastError();
}

hipError_t nonfinite_launch(const cplx* x, long long n, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(nonfinite_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, flag);
  return hipGetLastError();
}

hipError_t wt_convert_launch(const cplx* w, cplx* wt64, float* wt32, unsigned short* wt16, unsigned short* wt16s,
                             int n, int ld, int nh, const int* hself, hipStream_t s) {
  hipLaunchKernelGGL(wt_convert_kernel, dim3(grid_for((long long)nh * n * ld)), dim3(256), 0, s, w,
                     wt64, wt32, wt16, wt16s, n, ld, nh, hself);
  return hipGetLastError();
}

hipError_t lt_convert_launch(const cplx* lt, float* wt32, unsigned short* wt16, unsigned short* wt16s, int n, int ld,
                             int nh, const int* hself, hipStream_t s) {
  hipLaunchKernelGGL(lt_convert_kernel, dim3(grid_for((long long)nh * n * ld)), dim3(256), 0, s, lt, wt32, wt16,
                     wt16s, n, ld, nh, hself);
  return hipGetLastError();
}

hipError_t zero_launch(cplx* x, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_c_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n);
  return hipGetLastError();
}
