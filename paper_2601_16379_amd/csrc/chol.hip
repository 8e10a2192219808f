// FP64 solve of the ISDF normal equations (eq. (3)) and of Pi W Pi = V
// (eq. (8)) through a pivoted Cholesky factor.
//
// Pi^q is Hermitian positive semidefinite and can be exactly singular (the
// interpolation points may span the pair space with fewer independent
// columns than points).  chol_kernel factors P^T Pi P = L L^H with diagonal
// pivoting, stopping when the largest remaining diagonal falls below
// rtol * (largest initial diagonal); the leading `rank` columns define a
// basic least-squares solution, which gives the same fitted densities, hence
// the same ERIs, as any other least-squares solution.  L is stored
// transposed (row j of `lt` = column j of L) so that both triangular solves
// read contiguous rows.
#include "kernels.hpp"

namespace {

constexpr int CT = 1024;   // threads of the factorisation workgroup

__global__ __launch_bounds__(CT) void chol_kernel(const cplx* __restrict__ pi, cplx* work, cplx* lt,
                                                  int* perm, int* rank, int n, double rtol,
                                                  int pivot) {
  const int q = blockIdx.x;
  const long long nn = (long long)n * n;
  const cplx* P = pi + q * nn;
  cplx* A = work + q * nn;
  cplx* L = lt + q * nn;
  int* pm = perm + (long long)q * n;
  __shared__ double red_v[CT / 64];
  __shared__ int red_i[CT / 64];
  __shared__ int s_p;
  __shared__ double s_d, s_dmax0;
  __shared__ int s_stop;

  for (long long idx = threadIdx.x; idx < nn; idx += CT) {
    A[idx] = P[idx];
    L[idx] = cmk(0.0, 0.0);
  }
  for (int i = threadIdx.x; i < n; i += CT) pm[i] = i;
  __syncthreads();

  int r = n;
  for (int j = 0; j < n; ++j) {
    // ---- pivot: largest remaining diagonal (or j itself without pivoting) ----
    double best = -1.0;
    int bi = j;
    for (int i = j + threadIdx.x; i < n; i += CT) {
      double d = A[(long long)i * n + i].x;
      if (d > best || (d == best && i < bi)) { best = d; bi = i; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      double ov = __shfl_xor(best, off);
      int oi = __shfl_xor(bi, off);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if ((threadIdx.x & 63) == 0) { red_v[threadIdx.x >> 6] = best; red_i[threadIdx.x >> 6] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double bv = red_v[0];
      int bj = red_i[0];
      for (int w = 1; w < CT / 64; ++w)
        if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < bj)) { bv = red_v[w]; bj = red_i[w]; }
      if (j == 0) s_dmax0 = bv;
      if (!pivot) { bj = j; bv = A[(long long)j * n + j].x; }
      s_p = bj;
      s_d = bv;
      s_stop = !(bv > rtol * s_dmax0) || !(bv > 0.0);
    }
    __syncthreads();
    if (s_stop) { r = j; break; }
    const int p = s_p;
    // ---- symmetric swap of j and p in the trailing matrix and in L ----
    if (p != j) {
      for (int c = j + threadIdx.x; c < n; c += CT) {
        cplx t = A[(long long)j * n + c];
        A[(long long)j * n + c] = A[(long long)p * n + c];
        A[(long long)p * n + c] = t;
      }
      __syncthreads();
      for (int rr = j + threadIdx.x; rr < n; rr += CT) {
        cplx t = A[(long long)rr * n + j];
        A[(long long)rr * n + j] = A[(long long)rr * n + p];
        A[(long long)rr * n + p] = t;
      }
      for (int c = threadIdx.x; c < j; c += CT) {
        cplx t = L[(long long)c * n + j];
        L[(long long)c * n + j] = L[(long long)c * n + p];
        L[(long long)c * n + p] = t;
      }
      if (threadIdx.x == 0) { int t = pm[j]; pm[j] = pm[p]; pm[p] = t; }
      __syncthreads();
    }
    // ---- column j of L ----
    const double djj = sqrt(A[(long long)j * n + j].x);
    const double inv = 1.0 / djj;
    for (int i = j + threadIdx.x; i < n; i += CT) {
      L[(long long)j * n + i] = (i == j) ? cmk(djj, 0.0) : cscale(A[(long long)i * n + j], inv);
    }
    __syncthreads();
    // ---- trailing update A[i][c] -= L_ij conj(L_cj) ----
    const int w = n - j - 1;
    const long long tot = (long long)w * w;
    const cplx* Lj = L + (long long)j * n + j + 1;
    for (long long idx = threadIdx.x; idx < tot; idx += CT) {
      const int i = (int)(idx / w), c = (int)(idx - (idx / w) * w);
      cplx* a = &A[(long long)(j + 1 + i) * n + (j + 1 + c)];
      const cplx li = Lj[i], lc = Lj[c];
      // a -= li * conj(lc)
      a->x -= li.x * lc.x + li.y * lc.y;
      a->y -= li.y * lc.x - li.x * lc.y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) rank[q] = r;
}

// Triangular solves with the factor for a block of `cb` right-hand-side
// columns held in LDS.  stage 1: B = (P^T V P)[:, cols], Z = L^-H L^-1 B.
// stage 2: B = Z^H[:, cols], W[perm][perm] = L^-H L^-1 B.
__global__ __launch_bounds__(256) void wsolve_kernel(const cplx* __restrict__ v, cplx* z, cplx* w,
                                                     const cplx* __restrict__ lt,
                                                     const int* __restrict__ perm,
                                                     const int* __restrict__ rank, int n, int cb,
                                                     int stage) {
  extern __shared__ cplx B[];   // [r][cb]
  const int nblk = (n + cb - 1) / cb;
  const int q = blockIdx.x / nblk;
  const int c0 = (blockIdx.x % nblk) * cb;
  const int r = rank[q];
  if (c0 >= r) return;
  const int nc = (r - c0) < cb ? (r - c0) : cb;
  const long long nn = (long long)n * n;
  const cplx* L = lt + q * nn;
  const int* pm = perm + (long long)q * n;
  const cplx* V = v + q * nn;
  cplx* Z = z + q * nn;
  cplx* W = w + q * nn;

  for (int idx = threadIdx.x; idx < r * cb; idx += blockDim.x) {
    const int i = idx / cb, c = idx - (idx / cb) * cb;
    cplx x = cmk(0.0, 0.0);
    if (c < nc) {
      if (stage == 1) x = V[(long long)pm[i] * n + pm[c0 + c]];
      else x = cconj(Z[(long long)(c0 + c) * n + i]);
    }
    B[idx] = x;
  }
  __syncthreads();
  // forward: L y = b, column oriented (L_ij = lt[j][i])
  for (int j = 0; j < r; ++j) {
    const double djj = L[(long long)j * n + j].x;
    if (threadIdx.x < cb) B[j * cb + threadIdx.x] = cscale(B[j * cb + threadIdx.x], 1.0 / djj);
    __syncthreads();
    const int rows = r - j - 1;
    for (int idx = threadIdx.x; idx < rows * cb; idx += blockDim.x) {
      const int i = j + 1 + idx / cb, c = idx - (idx / cb) * cb;
      const cplx lij = L[(long long)j * n + i];
      const cplx yj = B[j * cb + c];
      cplx b = B[i * cb + c];
      b.x -= lij.x * yj.x - lij.y * yj.y;
      b.y -= lij.x * yj.y + lij.y * yj.x;
      B[i * cb + c] = b;
    }
    __syncthreads();
  }
  // backward: L^H z = y, row oriented: z_i = (y_i - sum_{j>i} conj(L_ji) z_j) / L_ii
  const int tpc = blockDim.x / cb;           // threads per column (power of two, <= 64)
  const int c = threadIdx.x / tpc, sub = threadIdx.x % tpc;
  for (int i = r - 1; i >= 0; --i) {
    cplx acc = cmk(0.0, 0.0);
    if (c < cb) {
      for (int j = i + 1 + sub; j < r; j += tpc) {
        const cplx lji = L[(long long)i * n + j];   // L_ji
        const cplx zj = B[j * cb + c];
        acc.x += lji.x * zj.x + lji.y * zj.y;       // conj(L_ji) * z_j
        acc.y += lji.x * zj.y - lji.y * zj.x;
      }
    }
    for (int off = tpc >> 1; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off);
      acc.y += __shfl_xor(acc.y, off);
    }
    if (c < cb && sub == 0) {
      const double dii = L[(long long)i * n + i].x;
      B[i * cb + c] = cscale(csub(B[i * cb + c], acc), 1.0 / dii);
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < r * cb; idx += blockDim.x) {
    const int i = idx / cb, cc = idx - (idx / cb) * cb;
    if (cc >= nc) continue;
    if (stage == 1) Z[(long long)i * n + c0 + cc] = B[idx];
    else W[(long long)pm[i] * n + pm[c0 + cc]] = B[idx];
  }
}

__global__ void zero_kernel(cplx* x, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = cmk(0.0, 0.0);
}

}  // namespace

hipError_t chol_launch(const cplx* pi, cplx* work, cplx* lt, int* perm, int* rank, int n, int nq,
                       double rtol, int pivot, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(chol_kernel, dim3(nq), dim3(CT), 0, s, pi, work, lt, perm, rank, n, rtol, pivot);
  return hipGetLastError();
}

hipError_t wsolve_launch(const cplx* v, cplx* z, cplx* w, const cplx* lt, const int* perm,
                         const int* rank, int n, int nq, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  int cb = 16;
  while (cb > 4 && (size_t)n * cb * sizeof(cplx) > 128 * 1024) cb >>= 1;
  const size_t lds = (size_t)n * cb * sizeof(cplx);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const int nblk = (n + cb - 1) / cb;
  hipLaunchKernelGGL(wsolve_kernel, dim3(nq * nblk), dim3(256), lds, s, v, z, w, lt, perm, rank, n, cb, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long tot = (long long)nq * n * n;
  hipLaunchKernelGGL(zero_kernel, dim3(1024), dim3(256), 0, s, w, tot);
  hipLaunchKernelGGL(wsolve_kernel, dim3(nq * nblk), dim3(256), lds, s, v, z, w, lt, perm, rank, n, cb, 2);
  return hipGetLastError();
}
