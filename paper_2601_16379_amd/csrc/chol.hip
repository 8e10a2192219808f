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
                                                  int pivot, const int* qlist) {
  const int q = qlist ? qlist[blockIdx.x] : blockIdx.x;
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

// out[q][i][j] = in[q][pm[i]][pm[j]] for i, j < rank (dir 0, gather), or
// out[q][pm[i]][pm[j]] = in[q][i][j] with zeros outside the rank (dir 1).
__global__ void permute_kernel(const cplx* __restrict__ in, cplx* out, const int* __restrict__ perm,
                               const int* __restrict__ rank, int n, int nq, int dir) {
  const long long nn = (long long)n * n;
  const long long total = nq * nn;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int q = (int)(idx / nn);
    const long long e = idx - q * nn;
    const int i = (int)(e / n), j = (int)(e - (e / n) * n);
    const int r = rank[q];
    const int* pm = perm + (long long)q * n;
    if (dir == 0) {
      if (i < r && j < r) out[idx] = in[q * nn + (long long)pm[i] * n + pm[j]];
    } else {
      // idx enumerates destination rows/cols in permuted order
      const cplx v = (i < r && j < r) ? in[idx] : cmk(0.0, 0.0);
      out[q * nn + (long long)pm[i] * n + pm[j]] = v;
    }
  }
}

// ---- blocked, unpivoted factorisation (batched over q) ----
__global__ void bchol_setup_kernel(const cplx* __restrict__ pi, cplx* a, int* perm, int* rank,
                                   double* dmax, int* flag, int n, int nq) {
  const long long nn = (long long)n * n;
  const int q = blockIdx.y;
  const cplx* P = pi + q * nn;
  cplx* A = a + q * nn;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < nn;
       idx += (long long)gridDim.x * blockDim.x)
    A[idx] = P[idx];
  if (blockIdx.x == 0) {
    __shared__ double red[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      m = fmax(m, P[(long long)i * n + i].x);
      perm[(long long)q * n + i] = i;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      dmax[q] = red[0];
      rank[q] = n;
      flag[q] = 0;
    }
  }
}

// Unblocked Cholesky of the diagonal block A[jb:jb+nb, jb:jb+nb] in LDS.
__global__ __launch_bounds__(256) void bchol_diag_kernel(cplx* a, cplx* lt, const double* dmax, int* flag,
                                                         int n, int jb, double rtol) {
  constexpr int NB = CHOL_NB;
  __shared__ cplx D[NB][NB + 1];
  __shared__ int s_bad;
  const int q = blockIdx.x;
  if (flag[q]) return;
  const long long nn = (long long)n * n;
  cplx* A = a + q * nn;
  cplx* L = lt + q * nn;
  const int nb = (n - jb) < NB ? (n - jb) : NB;
  for (int idx = threadIdx.x; idx < nb * nb; idx += blockDim.x) {
    const int i = idx / nb, j = idx - (idx / nb) * nb;
    D[i][j] = A[(long long)(jb + i) * n + jb + j];
  }
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  const double tol = rtol * dmax[q];
  for (int j = 0; j < nb; ++j) {
    const double djj = D[j][j].x;
    if (!(djj > tol) || !(djj > 0.0)) {   // uniform: every thread reads the same value
      if (threadIdx.x == 0) s_bad = 1;
      break;
    }
    const double d = sqrt(djj);
    __syncthreads();
    for (int i = j + threadIdx.x; i < nb; i += blockDim.x) D[i][j] = (i == j) ? cmk(d, 0.0) : cscale(D[i][j], 1.0 / d);
    __syncthreads();
    const int w = nb - j - 1;
    for (int idx = threadIdx.x; idx < w * w; idx += blockDim.x) {
      const int i = j + 1 + idx / w, c = j + 1 + idx - (idx / w) * w;
      if (c > i) continue;
      const cplx li = D[i][j], lc = D[c][j];
      D[i][c].x -= li.x * lc.x + li.y * lc.y;
      D[i][c].y -= li.y * lc.x - li.x * lc.y;
    }
    __syncthreads();
  }
  __syncthreads();
  if (s_bad) {
    if (threadIdx.x == 0) flag[q] = 1;
    return;
  }
  for (int idx = threadIdx.x; idx < nb * nb; idx += blockDim.x) {
    const int i = idx / nb, j = idx - (idx / nb) * nb;
    if (j > i) continue;
    A[(long long)(jb + i) * n + jb + j] = D[i][j];
    L[(long long)(jb + j) * n + jb + i] = D[i][j];
  }
}

// L21 = A21 L11^{-H}: row i solves x L11^H = a, x_c = (a_c - sum_{d<c} x_d conj(L11[c][d])) / L11[c][c].
__global__ __launch_bounds__(64) void bchol_panel_kernel(cplx* a, cplx* lt, const int* flag, int n, int jb) {
  constexpr int NB = CHOL_NB;
  __shared__ cplx L11[NB][NB + 1];
  __shared__ cplx X[64][NB + 1];
  const int q = blockIdx.y;
  if (flag[q]) return;
  const long long nn = (long long)n * n;
  cplx* A = a + q * nn;
  cplx* L = lt + q * nn;
  const int nb = (n - jb) < NB ? (n - jb) : NB;
  const int r0 = jb + nb + blockIdx.x * 64;
  if (r0 >= n) return;
  const int nr = (n - r0) < 64 ? (n - r0) : 64;
  for (int idx = threadIdx.x; idx < nb * nb; idx += blockDim.x) {
    const int i = idx / nb, j = idx - (idx / nb) * nb;
    L11[i][j] = A[(long long)(jb + i) * n + jb + j];
  }
  for (int idx = threadIdx.x; idx < nr * nb; idx += blockDim.x) {
    const int i = idx / nb, j = idx - (idx / nb) * nb;
    X[i][j] = A[(long long)(r0 + i) * n + jb + j];
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < nr) {
    for (int c = 0; c < nb; ++c) {
      cplx acc = X[t][c];
      for (int d = 0; d < c; ++d) {
        const cplx x = X[t][d], l = L11[c][d];
        // acc -= x * conj(l)
        acc.x -= x.x * l.x + x.y * l.y;
        acc.y -= x.y * l.x - x.x * l.y;
      }
      X[t][c] = cscale(acc, 1.0 / L11[c][c].x);
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nr * nb; idx += blockDim.x) {
    const int i = idx / nb, j = idx - (idx / nb) * nb;
    A[(long long)(r0 + i) * n + jb + j] = X[i][j];
  }
  for (int idx = threadIdx.x; idx < nr * nb; idx += blockDim.x) {
    const int j = idx / nr, i = idx - (idx / nr) * nr;   // coalesced along i for lt rows
    L[(long long)(jb + j) * n + r0 + i] = X[i][j];
  }
}

__global__ void zero_kernel(cplx* x, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = cmk(0.0, 0.0);
}

}  // namespace

hipError_t chol_launch(const cplx* pi, cplx* work, cplx* lt, int* perm, int* rank, int n, int nq,
                       double rtol, int pivot, hipStream_t s, const int* qlist) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(chol_kernel, dim3(nq), dim3(CT), 0, s, pi, work, lt, perm, rank, n, rtol, pivot,
                     qlist);
  return hipGetLastError();
}

hipError_t permute_launch(const cplx* in, cplx* out, const int* perm, const int* rank, int n, int nq,
                          int dir, hipStream_t s) {
  const long long total = (long long)nq * n * n;
  long long b = (total + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(permute_kernel, dim3((unsigned)b), dim3(256), 0, s, in, out, perm, rank, n, nq, dir);
  return hipGetLastError();
}

hipError_t bchol_setup_launch(const cplx* pi, cplx* a, int* perm, int* rank, double* dmax, int* flag,
                              int n, int nq, hipStream_t s) {
  const long long nn = (long long)n * n;
  long long bx = (nn + 255) / 256;
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(bchol_setup_kernel, dim3((unsigned)bx, nq), dim3(256), 0, s, pi, a, perm, rank, dmax,
                     flag, n, nq);
  return hipGetLastError();
}

hipError_t bchol_diag_launch(cplx* a, cplx* lt, const double* dmax, int* flag, int n, int nq, int jb,
                             double rtol, hipStream_t s) {
  hipLaunchKernelGGL(bchol_diag_kernel, dim3(nq), dim3(256), 0, s, a, lt, dmax, flag, n, jb, rtol);
  return hipGetLastError();
}

hipError_t bchol_panel_launch(cplx* a, cplx* lt, const int* flag, int n, int nq, int jb, hipStream_t s) {
  const int nb = (n - jb) < CHOL_NB ? (n - jb) : CHOL_NB;
  const int rows = n - jb - nb;
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(bchol_panel_kernel, dim3((rows + 63) / 64, nq), dim3(64), 0, s, a, lt, flag, n, jb);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Blocked inverse of the Cholesky factor, Y = L^{-1}, for all q at once:
// 64-row diagonal blocks inverted in LDS, the off-diagonal block rows by two
// FP64 MFMA products each (Y_ij = -Y_ii sum_{j<=k<i} L_ik Y_kj).  Rows and
// columns at or beyond the rank are zero throughout.
// ---------------------------------------------------------------------------
namespace {

// lrow[q][i][j] = L[i][j] (j <= i < rank, else 0) from lt[q][j][i] = L[i][j],
// 32 x 32 tiles transposed through LDS; yt[q] cleared.
__global__ __launch_bounds__(256) void tri_setup_kernel(const cplx* __restrict__ lt, const int* __restrict__ rank,
                                                        cplx* lrow, cplx* yt, int n) {
  __shared__ cplx t[32][33];
  const int q = blockIdx.z;
  const int r = rank[q];
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  const long long nn = (long long)n * n;
  const cplx* L = lt + q * nn;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int j = j0 + k, i = i0 + tx;
    t[k][tx] = (j < n && i < n) ? L[(long long)j * n + i] : cmk(0.0, 0.0);   // L[i][j]
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int i = i0 + k, j = j0 + tx;
    if (i < n && j < n) {
      const long long o = q * nn + (long long)i * n + j;
      lrow[o] = (i < r && j <= i) ? t[tx][k] : cmk(0.0, 0.0);
      yt[o] = cmk(0.0, 0.0);
    }
  }
}

// Diagonal block at jb: Y_bb = L_bb^{-1} by forward substitution, one thread
// per column, the block in LDS.  Written transposed into yt
// (yt[jb+c][jb+i] = Y_bb[i][c]) and row-major into yd[q] (64 x 64).
__global__ __launch_bounds__(64) void tri_inv_diag_kernel(const cplx* __restrict__ lrow,
                                                          const int* __restrict__ rank, cplx* yt,
                                                          cplx* yd, int n, int jb) {
  __shared__ cplx Ls[64][65];
  __shared__ cplx Ys[64][65];
  const int q = blockIdx.x;
  const long long nn = (long long)n * n;
  const int nb = (n - jb) < 64 ? (n - jb) : 64;
  int rb = rank[q] - jb;
  rb = rb < 0 ? 0 : (rb > nb ? nb : rb);
  const int c = threadIdx.x;
  for (int i = 0; i < 64; ++i)
    Ls[i][c] = (i < nb && c < nb) ? lrow[q * nn + (long long)(jb + i) * n + jb + c] : cmk(0.0, 0.0);
  __syncthreads();
  for (int i = 0; i < 64; ++i) {
    cplx s = cmk(i == c ? 1.0 : 0.0, 0.0);
    for (int k = c; k < i; ++k) {
      const cplx l = Ls[i][k], y = Ys[k][c];
      s.x -= l.x * y.x - l.y * y.y;
      s.y -= l.x * y.y + l.y * y.x;
    }
    Ys[i][c] = (i < rb && c < rb && i >= c) ? cscale(s, 1.0 / Ls[i][i].x) : cmk(0.0, 0.0);
  }
  __syncthreads();
  for (int i = 0; i < 64; ++i) {
    yd[(long long)q * 4096 + i * 64 + c] = Ys[i][c];
    if (i < nb && c < nb) yt[q * nn + (long long)(jb + c) * n + jb + i] = Ys[i][c];
  }
}

}  // namespace

hipError_t tri_setup_launch(const cplx* lt, const int* rank, cplx* lrow, cplx* yt, int n, int nq,
                            hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  const int nt = (n + 31) / 32;
  hipLaunchKernelGGL(tri_setup_kernel, dim3(nt, nt, nq), dim3(256), 0, s, lt, rank, lrow, yt, n);
  return hipGetLastError();
}

hipError_t tri_inv_diag_launch(const cplx* lrow, const int* rank, cplx* yt, cplx* yd, int n, int nq, int jb,
                               hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(tri_inv_diag_kernel, dim3(nq), dim3(64), 0, s, lrow, rank, yt, yd, n, jb);
  return hipGetLastError();
}
