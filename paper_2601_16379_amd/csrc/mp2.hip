// Small kernels of the opposite-spin MP2 energy in the imaginary-time form
// (eqs. (11)-(15)): the canonical orbitals at the interpolation points
// scaled by the square roots of their Laplace factors (so that each Green's
// function is one Hermitian product), and the per-class trace
// tr[(W chi)(W chit)] as the element-wise dot sum_IJ (W chi)_IJ conj((chit W)_IJ)
// (chit and W are Hermitian).
#include "kernels.hpp"

namespace {

// yo[k][I][i] = Y[k][I][i] exp(tau (e_i - mu) / 2),          i < n_occ
// yv[k][I][a] = Y[k][I][n_occ + a] exp(-tau (e_a - mu) / 2),  a < n_mo - n_occ
__global__ __launch_bounds__(256) void mp2_scale_kernel(const cplx* __restrict__ y, const double* __restrict__ e,
                                                      int nk, int nip, int nmo, int nocc, double tau, double mu,
                                                      cplx* __restrict__ yo, cplx* __restrict__ yv) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long total = (long long)nk * nip * nmo;
  if (i >= total) return;
  const int p = (int)(i % nmo);
  const long long row = i / nmo;              // k * nip + I
  const int k = (int)(row / nip);
  const double de = e[(long long)k * nmo + p] - mu;
  const cplx v = y[i];
  if (p < nocc) {
    yo[row * nocc + p] = cscale(v, exp(0.5 * tau * de));
  } else {
    const int nvir = nmo - nocc;
    yv[row * nvir + (p - nocc)] = cscale(v, exp(-0.5 * tau * de));
  }
}

// part[h][b] = sum over the b-th chunk of the n_elem elements of class h of
// t1 conj(t2)
__global__ __launch_bounds__(256) void mp2_dot_kernel(const cplx* __restrict__ t1, const cplx* __restrict__ t2,
                                                    long long n_elem, int nblk, cplx* __restrict__ part) {
  const int h = blockIdx.y;
  const long long per = (n_elem + nblk - 1) / nblk;
  const long long b0 = (long long)blockIdx.x * per;
  const long long b1 = b0 + per < n_elem ? b0 + per : n_elem;
  const cplx* a = t1 + (long long)h * n_elem;
  const cplx* b = t2 + (long long)h * n_elem;
  double re = 0.0, im = 0.0;
  for (long long i = b0 + threadIdx.x; i < b1; i += 256) {
    const cplx x = a[i], z = b[i];
    re = fma(x.x, z.x, fma(x.y, z.y, re));
    im = fma(x.y, z.x, fma(-x.x, z.y, im));
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
  if (threadIdx.x == 0) part[(long long)h * nblk + blockIdx.x] = cmk(sr[0], si[0]);
}

}  // namespace

hipError_t mp2_scale_launch(const cplx* y, const double* e, int nk, int nip, int nmo, int nocc, double tau, double mu,
                            cplx* yo, cplx* yv, hipStream_t s) {
  const long long total = (long long)nk * nip * nmo;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(mp2_scale_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, y, e, nk, nip, nmo,
                     nocc, tau, mu, yo, yv);
  return hipGetLastError();
}

hipError_t mp2_dot_launch(const cplx* t1, const cplx* t2, long long n_elem, int nclass, int nblk, cplx* part,
                          hipStream_t s) {
  if (nclass <= 0 || nblk <= 0) return hipSuccess;
  if (nclass > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mp2_dot_kernel, dim3(nblk, nclass), dim3(256), 0, s, t1, t2, n_elem, nblk, part);
  return hipGetLastError();
}
