// Transforms over the k mesh (the convolution theorem of Algorithm 1 and the
// k <-> R transforms of Algorithm 2), staged through LDS.
//
// A workgroup loads a tile of `etile` independent elements for every k of
// the m1 x m2 x m3 mesh (k-major rows of contiguous elements, so every HBM
// row access is coalesced), applies the 3-D DFT over the mesh one axis at a
// time inside LDS (each thread owns one length-m line in registers), applies
// the pointwise step, transforms back and stores: one HBM read and one HBM
// write per element, however many mesh axes there are.
#include "kernels.hpp"

namespace {

constexpr int MAXM = 16;

// In-place 3-D DFT over the mesh for every element column of buf[k][etile]:
// buf[k][e] <- sum_j exp(sign * 2 pi i sum_d j_d k_d / m_d) buf[j][e].
// tw[ax][t] = exp(2 pi i t / m_ax), filled by init_twiddles.
__device__ void init_twiddles(cplx (*tw)[MAXM], int m1, int m2, int m3) {
  const int ms[3] = {m1, m2, m3};
  if (threadIdx.x < 3 * MAXM) {
    const int ax = threadIdx.x / MAXM, t = threadIdx.x % MAXM;
    if (t < ms[ax]) tw[ax][t] = cexpipi(2.0 * (double)t / (double)ms[ax]);
  }
}

__device__ void mesh_dft(cplx* buf, const cplx (*tw)[MAXM], int etile, int m1, int m2, int m3,
                         int sign) {
  const int nk = m1 * m2 * m3;
  const int ms[3] = {m1, m2, m3};
  for (int ax = 0; ax < 3; ++ax) {
    const int m = ms[ax];
    if (m == 1) continue;
    const int nlines = (nk / m) * etile;
    for (int line = threadIdx.x; line < nlines; line += blockDim.x) {
      const int e = line % etile;
      const int rest = line / etile;
      int base, stride;
      if (ax == 0) { base = rest; stride = m2 * m3; }
      else if (ax == 1) { base = (rest / m3) * m2 * m3 + (rest % m3); stride = m3; }
      else { base = rest * m3; stride = 1; }
      cplx x[MAXM];
#pragma unroll
      for (int j = 0; j < MAXM; ++j)
        if (j < m) x[j] = buf[(long long)(base + j * stride) * etile + e];
      for (int t = 0; t < m; ++t) {
        cplx acc = cmk(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < MAXM; ++j) {
          if (j < m) {
            const int jt = (j * t) % m;
            cplx w = tw[ax][jt];
            if (sign < 0) w.y = -w.y;
            cfma(acc, x[j], w);
          }
        }
        buf[(long long)(base + t * stride) * etile + e] = acc;
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void kconv_kernel(KconvArgs a, int etile) {
  extern __shared__ cplx buf[];
  __shared__ cplx tw[3][MAXM];
  init_twiddles(tw, a.m1, a.m2, a.m3);
  const int nk = a.m1 * a.m2 * a.m3;
  const long long e0 = (long long)blockIdx.x * etile;
  const long long rem = a.n_elem - e0;
  const int ne = rem < etile ? (int)rem : etile;
  for (int idx = threadIdx.x; idx < nk * etile; idx += blockDim.x) {
    const int k = idx / etile, e = idx - (idx / etile) * etile;
    cplx v = cmk(0.0, 0.0);
    if (e < ne) {
      const long long ee = e0 + e;
      v = a.in[(long long)k * a.in_kstride + (ee / a.in_inner) * a.in_outer + ee % a.in_inner];
    }
    buf[idx] = v;
  }
  __syncthreads();
  if (a.mode == 0) {
    // T^R = sum_k exp(+i k.R) T^k ;  Z^R = |T^R|^2 ;  out^q = scale * sum_R exp(+i q.R) Z^R
    mesh_dft(buf, tw, etile, a.m1, a.m2, a.m3, +1);
    for (int idx = threadIdx.x; idx < nk * etile; idx += blockDim.x) {
      cplx v = buf[idx];
      buf[idx] = cmk(v.x * v.x + v.y * v.y, 0.0);
    }
    __syncthreads();
    mesh_dft(buf, tw, etile, a.m1, a.m2, a.m3, +1);
  } else {
    mesh_dft(buf, tw, etile, a.m1, a.m2, a.m3, a.sign);
  }
  for (int idx = threadIdx.x; idx < nk * etile; idx += blockDim.x) {
    const int q = idx / etile, e = idx - (idx / etile) * etile;
    if (e < ne) {
      const long long ee = e0 + e;
      a.out[(long long)q * a.out_qstride + (ee / a.out_inner) * a.out_outer + ee % a.out_inner] =
          cscale(buf[idx], a.scale);
    }
  }
}

// One workgroup: a tile of `tp` pairs of one fragment times `ti` consecutive
// interpolation points; LDS holds [R][tp*ti] so that the output rows (pair,
// I-range) are written as contiguous runs of I.
__global__ __launch_bounds__(256) void pair_kernel(PairArgs a) {
  extern __shared__ cplx buf[];
  __shared__ cplx tw[3][MAXM];
  init_twiddles(tw, a.m1, a.m2, a.m3);
  const int nk = a.m1 * a.m2 * a.m3;
  const int it = blockIdx.x % a.n_itiles;
  const int blk = blockIdx.x / a.n_itiles;
  const PairBlock pb = a.blocks[blk];
  const int nf = a.frag_nf[pb.frag];
  const int col = a.frag_col[pb.frag];
  const long long poff = a.frag_pair[pb.frag];
  const int w = a.tp * a.ti;
  const int I0 = it * a.ti;
  for (int idx = threadIdx.x; idx < nk * w; idx += blockDim.x) {
    const int R = idx / w, e = idx - (idx / w) * w;
    const int j = e / a.ti, i = e - (e / a.ti) * a.ti;
    cplx v = cmk(0.0, 0.0);
    const int I = I0 + i;
    if (j < pb.npair && I < a.n_ip) {
      const int P = pb.pair0 + j;
      const int p = P / nf, q = P - (P / nf) * nf;
      const cplx* base = a.psi + ((long long)R * a.ncol + col) * a.n_ip + I;
      v = cmulc(base[(long long)q * a.n_ip], base[(long long)p * a.n_ip]);   // conj(psi_p) psi_q
    }
    buf[idx] = v;
  }
  __syncthreads();
  mesh_dft(buf, tw, w, a.m1, a.m2, a.m3, -1);
  for (int idx = threadIdx.x; idx < nk * w; idx += blockDim.x) {
    const int Q = idx / w, e = idx - (idx / w) * w;
    const int j = e / a.ti, i = e - (e / a.ti) * a.ti;
    const int I = I0 + i;
    if (j < pb.npair && I < a.ld) {
      const long long off = ((long long)Q * a.ptot + poff + pb.pair0 + j) * a.ld + I;
      store_fmt(a.out, off, a.plane, a.fmt, cscale(buf[idx], a.scale));
    }
  }
}

}  // namespace

hipError_t kconv_launch(const KconvArgs& a, hipStream_t s) {
  const int nk = a.m1 * a.m2 * a.m3;
  if (a.m1 > MAXM || a.m2 > MAXM || a.m3 > MAXM) return hipErrorInvalidValue;
  int etile = 4096 / nk;                // 64 KB of complex128 per block
  if (etile > 256) etile = 256;
  if (etile < 1) etile = 1;
  const long long blocks = (a.n_elem + etile - 1) / etile;
  if (blocks <= 0) return hipSuccess;
  const size_t lds = (size_t)nk * etile * sizeof(cplx);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kconv_kernel, dim3((unsigned)blocks), dim3(256), lds, s, a, etile);
  return hipGetLastError();
}

hipError_t pair_launch(const PairArgs& a, hipStream_t s) {
  const int nk = a.m1 * a.m2 * a.m3;
  if (a.m1 > MAXM || a.m2 > MAXM || a.m3 > MAXM) return hipErrorInvalidValue;
  const size_t lds = (size_t)nk * a.tp * a.ti * sizeof(cplx);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const long long blocks = (long long)a.nblocks * a.n_itiles;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(pair_kernel, dim3((unsigned)blocks), dim3(256), lds, s, a);
  return hipGetLastError();
}
