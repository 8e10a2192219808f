// Small kernels of the k-point Hartree-Fock Coulomb matrix (the q = 0 term
// of the factorised integrals, eq. (9), contracted with the density matrix):
// the density at the interpolation points summed over k, its product with
// W^0, and the row scaling of X that turns J into one NT product per k.
#include "kernels.hpp"

namespace {

// n[J] = sum_k rho[k][J][J]
__global__ __launch_bounds__(256) void hf_diag_sum_kernel(const cplx* __restrict__ rho, int nk, int nip,
                                                        cplx* __restrict__ n) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= nip) return;
  const long long nn = (long long)nip * nip;
  double re = 0.0, im = 0.0;
  for (int k = 0; k < nk; ++k) {
    const cplx v = rho[(long long)k * nn + (long long)j * nip + j];
    re += v.x;
    im += v.y;
  }
  n[j] = cmk(re, im);
}

// v[I] = scale * sum_J W[I][J] n[J] (W conjugated when conj): one wavefront
// per row, the row read coalesced.
__global__ __launch_bounds__(256) void hf_matvec_kernel(const cplx* __restrict__ w, int conj, const cplx* __restrict__ n,
                                                      int nip, double scale, cplx* __restrict__ v) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= nip) return;
  const cplx* wr = w + (long long)row * nip;
  double re = 0.0, im = 0.0;
  for (int j = lane; j < nip; j += 64) {
    cplx a = wr[j];
    if (conj) a.y = -a.y;
    const cplx b = n[j];
    re = fma(a.x, b.x, fma(-a.y, b.y, re));
    im = fma(a.x, b.y, fma(a.y, b.x, im));
  }
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_down(re, off);
    im += __shfl_down(im, off);
  }
  if (lane == 0) v[row] = cmk(re * scale, im * scale);
}

// out[k][nu][I] = v[I] xt[k][nu][I]
__global__ __launch_bounds__(256) void hf_scale_kernel(const cplx* __restrict__ xt, const cplx* __restrict__ v,
                                                     long long rows, int nip, cplx* __restrict__ out) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= rows * nip) return;
  out[i] = cmul(v[i % nip], xt[i]);
}

}  // namespace

hipError_t hf_diag_sum_launch(const cplx* rho, int nk, int nip, cplx* n, hipStream_t s) {
  hipLaunchKernelGGL(hf_diag_sum_kernel, dim3((nip + 255) / 256), dim3(256), 0, s, rho, nk, nip, n);
  return hipGetLastError();
}

hipError_t hf_matvec_launch(const cplx* w, int conj, const cplx* n, int nip, double scale, cplx* v, hipStream_t s) {
  hipLaunchKernelGGL(hf_matvec_kernel, dim3((nip + 3) / 4), dim3(256), 0, s, w, conj, n, nip, scale, v);
  return hipGetLastError();
}

hipError_t hf_scale_launch(const cplx* xt, const cplx* v, long long rows, int nip, cplx* out, hipStream_t s) {
  const long long n = rows * nip;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(hf_scale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xt, v, rows, nip, out);
  return hipGetLastError();
}
