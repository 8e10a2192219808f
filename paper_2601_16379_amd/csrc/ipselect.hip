// Interpolation-point selection by pivoted Cholesky of the pair products
// (the IP-selection paragraph of the paper's section "Periodic k-point
// FFTISDF representation of integrals").  The products
// phi^{k_mu}_mu(r) conj(phi^{k_nu}_nu(r)) over all orbital pairs have the
// Gram matrix M(x, y) = |G(x, y)|^2 with G(x, y) = sum_k sum_mu
// phi^k_mu(x) conj(phi^k_mu(y)), whose diagonal is rho(x)^2.  The greedy
// (diagonally pivoted) Cholesky keeps a residual diagonal d and, at step i,
// takes the point p of largest residual (lowest index among equals), forms
//   L_i(x) = (|G(x, p)|^2 - sum_{j<i} L_j(x) L_j(p)) / sqrt(d(p))
// and lowers d(x) by L_i(x)^2; the chosen point leaves the candidate set
// (its residual is zero in exact arithmetic and is set to zero).  M is never
// formed.  Everything is FP64.
//
// Orbitals are rows phi_r(x), r = (k, mu), of length N_g (the context's
// [N_k][N_orb][N_g] layout).  A step is three launches and keeps the pivot
// in device memory:
//   sel_part   -- partial sums over a slice of rows, one thread per grid
//                 point (rows read coalesced along x, the slice's values at
//                 p staged in LDS): G(x, p) for a step, rho(x) for the start;
//   sel_update -- sums the slices, forms the column and the residual, writes
//                 L_i and d, and reduces its block's d to (max, argmax);
//   sel_pick   -- one workgroup reduces the block maxima to the next pivot
//                 and its residual.
// A step reads the orbitals once (N_k N_orb N_g 16 bytes, the bound), the
// previous columns once (i N_g 8 bytes) and writes one column.
#include "kernels.hpp"

namespace {

constexpr int SEL_T = 256;       // threads per workgroup (4 wavefronts)
constexpr int SEL_CHUNK = 256;   // values at p staged per LDS pass

// larger value wins; among equal values the lower index
__device__ inline void argmax_merge(double& v, long long& i, double v2, long long i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

// (max, argmax) over the workgroup; every thread returns the result
__device__ inline void block_argmax(double& v, long long& i) {
  __shared__ double sv[SEL_T];
  __shared__ long long si[SEL_T];
  sv[threadIdx.x] = v;
  si[threadIdx.x] = i;
  __syncthreads();
  for (int s = SEL_T / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      double a = sv[threadIdx.x];
      long long ia = si[threadIdx.x];
      argmax_merge(a, ia, sv[threadIdx.x + s], si[threadIdx.x + s]);
      sv[threadIdx.x] = a;
      si[threadIdx.x] = ia;
    }
    __syncthreads();
  }
  v = sv[0];
  i = si[0];
}

// The pivot of `step` as an index that is safe to read (0 when the pivot
// is invalid; sel_update then discards the column).
__device__ inline long long safe_pivot(const int* piv, const double* dmax, int step, long long ng) {
  const long long p = piv[step];
  return (p >= 0 && p < ng && dmax[step] > 0.0) ? p : 0;
}

// Slice s = blockIdx.y of the rows [s*rows_per, ...): part[s][x] =
//   RHO:  (sum_r |phi_r(x)|^2, 0)
//   else: sum_r phi_r(x) conj(phi_r(p)),  p = pivot of `step`
template <bool RHO>
__global__ __launch_bounds__(SEL_T) void sel_part_kernel(const cplx* __restrict__ phi, long long nrows, long long ng,
                                                       long long rows_per, const int* __restrict__ piv,
                                                       const double* __restrict__ dmax, int step,
                                                       cplx* __restrict__ part) {
  __shared__ cplx sp[SEL_CHUNK];
  const long long x = (long long)blockIdx.x * SEL_T + threadIdx.x;
  const long long r0 = (long long)blockIdx.y * rows_per;
  const long long r1 = r0 + rows_per < nrows ? r0 + rows_per : nrows;
  const bool in = x < ng;
  double gr = 0.0, gi = 0.0;
  if (RHO) {
    if (in)
      for (long long r = r0; r < r1; ++r) {
        const cplx a = phi[r * ng + x];
        gr = fma(a.x, a.x, fma(a.y, a.y, gr));
      }
  } else {
    const long long p = safe_pivot(piv, dmax, step, ng);
    for (long long c0 = r0; c0 < r1; c0 += SEL_CHUNK) {
      const int n = (int)(r1 - c0 < SEL_CHUNK ? r1 - c0 : SEL_CHUNK);
      __syncthreads();
      for (int j = threadIdx.x; j < n; j += SEL_T) sp[j] = phi[(c0 + j) * ng + p];
      __syncthreads();
      if (in)
        for (int j = 0; j < n; ++j) {
          const cplx a = phi[(c0 + j) * ng + x], b = sp[j];
          gr = fma(a.x, b.x, fma(a.y, b.y, gr));
          gi = fma(a.y, b.x, fma(-a.x, b.y, gi));
        }
    }
  }
  if (in) part[(long long)blockIdx.y * ng + x] = cmk(gr, gi);
}

// INIT: d(x) = rho(x)^2.  Else column `step`:
//   l = (|G(x, p)|^2 - sum_{j<step} L_j(x) L_j(p)) / sqrt(d(p)),  L_step(x) = l,
//   d(x) -= l^2, and d(p) = 0.
// Both end with the workgroup's (max d, argmax) in bv[b], bi[b].
template <bool INIT>
__global__ __launch_bounds__(SEL_T) void sel_update_kernel(const cplx* __restrict__ part, int nslice, long long ng,
                                                         double* __restrict__ lf, double* __restrict__ d,
                                                         const int* __restrict__ piv, const double* __restrict__ dmax,
                                                         int step, double* __restrict__ bv, long long* __restrict__ bi) {
  __shared__ double sl[SEL_CHUNK];
  const long long x = (long long)blockIdx.x * SEL_T + threadIdx.x;
  const bool in = x < ng;
  double gr = 0.0, gi = 0.0;
  if (in)
    for (int s = 0; s < nslice; ++s) {
      const cplx g = part[(long long)s * ng + x];
      gr += g.x;
      gi += g.y;
    }
  double dn = 0.0;
  if (INIT) {
    dn = gr * gr;
    if (in) d[x] = dn;
  } else {
    const long long p = safe_pivot(piv, dmax, step, ng);
    const double dm = dmax[step];
    const bool ok = dm > 0.0 && piv[step] == p;
    double corr = 0.0;
    for (int j0 = 0; j0 < step; j0 += SEL_CHUNK) {
      const int n = step - j0 < SEL_CHUNK ? step - j0 : SEL_CHUNK;
      __syncthreads();
      for (int j = threadIdx.x; j < n; j += SEL_T) sl[j] = lf[(long long)(j0 + j) * ng + p];
      __syncthreads();
      if (in)
        for (int j = 0; j < n; ++j) corr = fma(lf[(long long)(j0 + j) * ng + x], sl[j], corr);
    }
    if (in) {
      const double l = ok ? (gr * gr + gi * gi - corr) / sqrt(dm) : 0.0;
      lf[(long long)step * ng + x] = l;
      dn = (ok && x == p) ? 0.0 : d[x] - l * l;
      d[x] = dn;
    }
  }
  double v = in ? dn : -1.0;
  long long i = in ? x : ng;
  block_argmax(v, i);
  if (threadIdx.x == 0) {
    bv[blockIdx.x] = v;
    bi[blockIdx.x] = i;
  }
}

// next pivot: (max, argmax) over the nb workgroup results
__global__ __launch_bounds__(SEL_T) void sel_pick_kernel(const double* __restrict__ bv, const long long* __restrict__ bi,
                                                       int nb, long long ng, int step, int* __restrict__ piv,
                                                       double* __restrict__ dmax) {
  double v = -1.0;
  long long i = ng;
  for (int b = threadIdx.x; b < nb; b += SEL_T) argmax_merge(v, i, bv[b], bi[b]);
  block_argmax(v, i);
  if (threadIdx.x == 0) {
    piv[step] = (int)(i < ng ? i : -1);
    dmax[step] = i < ng ? v : -1.0;
  }
}

}  // namespace

SelPlan sel_plan(long long nrows, long long ng) {
  SelPlan p;
  p.xblocks = (int)((ng + SEL_T - 1) / SEL_T);
  // enough row slices that a step has about 2048 workgroups, each slice at
  // least 16 rows long
  long long ns = (2048 + p.xblocks - 1) / p.xblocks;
  const long long most = (nrows + 15) / 16;
  if (ns > most) ns = most;
  if (ns < 1) ns = 1;
  p.rows_per = (nrows + ns - 1) / ns;
  p.nslice = (int)((nrows + p.rows_per - 1) / p.rows_per);
  return p;
}

hipError_t sel_start_launch(const SelPlan& pl, const cplx* phi, long long nrows, long long ng, cplx* part, double* d,
                            double* bv, long long* bi, int* piv, double* dmax, hipStream_t s) {
  hipLaunchKernelGGL(sel_part_kernel<true>, dim3(pl.xblocks, pl.nslice), dim3(SEL_T), 0, s, phi, nrows, ng,
                     pl.rows_per, piv, dmax, 0, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sel_update_kernel<true>, dim3(pl.xblocks), dim3(SEL_T), 0, s, part, pl.nslice, ng, nullptr, d,
                     piv, dmax, 0, bv, bi);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sel_pick_kernel, dim3(1), dim3(SEL_T), 0, s, bv, bi, pl.xblocks, ng, 0, piv, dmax);
  return hipGetLastError();
}

hipError_t sel_step_launch(const SelPlan& pl, const cplx* phi, long long nrows, long long ng, cplx* part, double* lf,
                           double* d, double* bv, long long* bi, int* piv, double* dmax, int step, bool pick_next,
                           hipStream_t s) {
  hipLaunchKernelGGL(sel_part_kernel<false>, dim3(pl.xblocks, pl.nslice), dim3(SEL_T), 0, s, phi, nrows, ng,
                     pl.rows_per, piv, dmax, step, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sel_update_kernel<false>, dim3(pl.xblocks), dim3(SEL_T), 0, s, part, pl.nslice, ng, lf, d, piv,
                     dmax, step, bv, bi);
  e = hipGetLastError();
  if (e != hipSuccess || !pick_next) return e;
  hipLaunchKernelGGL(sel_pick_kernel, dim3(1), dim3(SEL_T), 0, s, bv, bi, pl.xblocks, ng, step + 1, piv, dmax);
  return hipGetLastError();
}
